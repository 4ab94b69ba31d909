"""Host emulation of the fused small-front launches: the two kernels of
csrc/smallfront.hip, compiled for the host through a stand-in HIP header
(tests/emu), run the upward and downward launches (one per depth and
direction) of lattices whose fronts are all small, and the selected G they
leave on the pattern must equal the oracle's dense inverse of X = alpha S - H
(Sec. II C 2, Eqs. (18)-(21), (38)-(39))."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import dense
from synth import lattice

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1005_0088_amd", "csrc")


@pytest.fixture(scope="module")
def emulator(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path_factory.mktemp("emu") / "small_schedule_emu")
    cmd = [gxx, "-std=c++20", "-O1", "-pthread", "-I", os.path.join(ROOT, "tests", "emu"), "-I", CSRC,
           "-I", os.path.join(ROOT, "include"), "-x", "c++", os.path.join(ROOT, "tests", "emu", "small_schedule_emu.cpp"),
           os.path.join(CSRC, "smallfront.hip"), "-x", "none", os.path.join(CSRC, "plan.cpp"),
           os.path.join(CSRC, "poles.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    return exe


def _run(exe, sysd, alpha, hcoef, tmp_path):
    inp, out = str(tmp_path / "in.bin"), str(tmp_path / "out.bin")
    cell = sysd["cell"]
    with open(inp, "wb") as f:
        np.array([sysd["n"], len(sysd["col"]), 0 if cell is None else 1], np.int64).tofile(f)
        sysd["row_ptr"].astype(np.int64).tofile(f)
        sysd["col"].astype(np.int32).tofile(f)
        np.ascontiguousarray(sysd["coords"], np.float64).tofile(f)
        if cell is not None:
            np.asarray(cell, np.float64).tofile(f)
        sysd["h"].astype(np.float64).tofile(f)
        sysd["s"].astype(np.float64).tofile(f)
        np.array([alpha.real, alpha.imag, hcoef], np.float64).tofile(f)
    r = subprocess.run([exe, inp, out], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, "emulator exit %d %s" % (r.returncode, r.stderr[-2000:])
    raw = np.fromfile(out, np.uint8)
    nnz = len(sysd["col"])
    g = raw[:16 * nnz].view(np.float64).reshape(nnz, 2)
    status = raw[16 * nnz:].view(np.int32)
    return g[:, 0] + 1j * g[:, 1], status


@pytest.mark.parametrize("dims,nb,seed,periodic,alpha,hcoef", [
    ((256,), "nn", 0, False, 0.3 + 0.7j, 1.0),      # the 256-site chain of the 1D workload
    ((256,), "nn", 0, False, 1.0 + 0.0j, 0.0),      # its S^{-1}: the evaluation at registration
    ((10, 10), "nn", 5, False, -0.2 + 0.314j, 1.0),
    ((4, 4, 4), "nn", 6, False, 1.0 + 0.0j, 0.0),   # S^{-1} (the M0 evaluation)
    ((6, 6), "nn", 7, True, 0.1 + 2.0j, 1.0),
])
def test_small_front_kernels_give_selected_inverse(emulator, dims, nb, seed, periodic, alpha, hcoef, tmp_path):
    sysd = lattice(dims, nb, seed, periodic=periodic)
    n = sysd["n"]
    rows = np.repeat(np.arange(n), np.diff(sysd["row_ptr"]))
    h = np.zeros((n, n))
    s = np.zeros((n, n))
    h[rows, sysd["col"]] = sysd["h"]
    s[rows, sysd["col"]] = sysd["s"]
    got, status = _run(emulator, sysd, alpha, hcoef, tmp_path)
    assert list(status) == [0, 0]               # no bad pivot
    ref = dense.green_dense(hcoef * h, s, alpha)[rows, sysd["col"]]
    assert np.max(np.abs(got - ref)) < 1e-12 * max(1.0, np.abs(ref).max())
