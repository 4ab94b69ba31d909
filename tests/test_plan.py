"""Host-side checks of the library that need no GPU: the exported C symbols,
the continued-fraction poles, the nested-dissection ordering and the symbolic
front tree with its index tables.

The last tests drive a small numpy model of the front-by-front factorization
and selected inversion (test code, independent of the oracle and the
kernels) through the library's exported plan, and compare the selected
entries with a dense inverse: this validates the plan's maps on the CPU.
"""
import os
import re

import numpy as np
import pytest

import paper_1005_0088_amd as nd
from oracle import poles as opoles
from synth import lattice

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_every_declared_symbol_is_exported():
    lib = nd.load_library()
    with open(os.path.join(ROOT, "include", "ndrho.h")) as f:
        hdr = f.read()
    names = set(re.findall(r"\b(ndrho_[a-z_0-9]+)\s*\(", hdr))
    assert len(names) >= 15
    for name in sorted(names):
        assert hasattr(lib, name), name
    declared = {s[0] for s in nd._binding.SIGNATURES}
    assert names == declared


def test_default_options_and_struct_layouts():
    # the ctypes mirrors of ndrho_options and ndrho_stats_t follow the
    # header field by field; the library's defaults are the documented ones
    import ctypes
    with open(os.path.join(ROOT, "include", "ndrho.h")) as f:
        hdr = f.read()
    for cname, mirror in (("ndrho_options", nd._binding.Options), ("ndrho_stats_t", nd._binding.Stats)):
        body = re.search(r"typedef struct \{((?:(?!typedef).)*?)\} %s;" % cname, hdr, re.S).group(1)
        body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
        fields = []
        for decl in body.split(";"):
            m = re.match(r"\s*(int32_t|int64_t|double)\s+(.*)", decl.strip())
            if m:
                fields += [(v.strip(), m.group(1)) for v in m.group(2).split(",")]
        ctype = {"int32_t": ctypes.c_int32, "int64_t": ctypes.c_int64, "double": ctypes.c_double}
        assert [(n, ctype[t]) for n, t in fields] == list(mirror._fields_), cname
    lib = nd.load_library()
    opt = nd._binding.Options()
    assert lib.ndrho_default_options(ctypes.byref(opt)) == 0
    want = {"leaf_rows": 32, "precision": 0, "pole_batch": 0, "mem_fraction": 0.8, "verbose": 0, "fp64_poles": 12,
            "fp64_pole_im": 0.05, "fp64_far_poles": 12, "use_graph": 1, "gemm_variant": -1, "fp64_small_tiles": -1,
            "split_streams": 0, "long_tail": 0.0, "small_fronts": 0,
            "pivot_variant": 0}
    assert {k: getattr(opt, k) for k, _ in opt._fields_} == want


@pytest.mark.parametrize("n_poles", [1, 2, 5, 60, 80, 100])
def test_library_poles_match_oracle(n_poles):
    z, r = nd.cf_poles(n_poles)
    zo, ro = opoles.cf_poles(n_poles)
    assert np.allclose(z, zo, rtol=1e-12, atol=0)
    assert np.allclose(r, ro, rtol=1e-11, atol=1e-13)
    assert r.sum() == pytest.approx(-n_poles * (2 * n_poles + 1) / 2.0, rel=1e-12)


def test_library_poles_reject_bad_count():
    with pytest.raises(nd.NdrhoError) as e:
        nd.cf_poles(0)
    assert e.value.name == "EINVAL"


def _pattern(sysd):
    n = sysd["n"]
    rows = np.repeat(np.arange(n), np.diff(sysd["row_ptr"]))
    return rows, sysd["col"].astype(np.int64)


def _check_plan(sysd, leaf, coords=True, long_tail=0.0, cell=None):
    n = sysd["n"]
    P = nd.Plan(n, sysd["row_ptr"], sysd["col"], sysd["coords"] if coords else None, leaf, long_tail=long_tail,
                cell=cell)
    ex = P.export()
    perm = ex["perm"]
    assert np.array_equal(np.sort(perm), np.arange(n))
    nf = P.n_fronts
    j0, nj, nu, parent = ex["j0"], ex["nj"], ex["nu"], ex["parent"]
    # postorder, contiguous J ranges covering all rows
    assert j0[0] == 0 and np.all(j0[1:] == j0[:-1] + nj[:-1]) and j0[-1] + nj[-1] == n
    for f in range(nf):
        if parent[f] >= 0:
            assert parent[f] > f
            assert ex["depth"][f] == ex["depth"][parent[f]] + 1
        else:
            assert nu[f] == 0 and ex["depth"][f] == 0
        u = ex["u_rows"][ex["u_off"][f]:ex["u_off"][f] + nu[f]]
        assert np.all(np.diff(u) > 0) and (nu[f] == 0 or u[0] >= j0[f] + nj[f])
        if parent[f] >= 0:
            p = parent[f]
            rel = ex["rel"][ex["u_off"][f]:ex["u_off"][f] + nu[f]]
            pu = ex["u_rows"][ex["u_off"][p]:ex["u_off"][p] + nu[p]]
            ploc = np.concatenate([np.arange(j0[p], j0[p] + nj[p]), pu])
            assert np.all((rel >= 0) & (rel < nj[p] + nu[p]))
            assert np.array_equal(ploc[rel], u)          # closure: U_f inside J_p + U_p
    # leaves are small; every separator separates (checked through closure)
    leaves = [f for f in range(nf) if not np.any(parent == f)]
    assert all(nj[f] <= leaf for f in leaves)
    # table function: assembly slots are unique, output slots inside the panel of the owner
    out, asm, poff = P.slots()
    a = asm[asm >= 0]
    assert len(np.unique(a)) == len(a)
    assert np.all((out >= 0) & (out < P.panel_total))
    return P, ex


@pytest.mark.parametrize("dims,nb,leaf", [((40,), "nn", 8), ((9, 7), "nn2", 12), ((5, 4, 6), "nn", 16),
                                           ((6, 6, 5), "nn2", 32), ((256,), "nn", 32)])
def test_plan_invariants(dims, nb, leaf):
    sysd = lattice(dims, nb, 3)
    _check_plan(sysd, leaf)


def test_plan_without_coordinates():
    sysd = lattice((7, 6), "nn", 1)
    _check_plan(sysd, 10, coords=False)


def test_plan_sizes_of_the_workloads():
    # 1D 256 sites x 4: 63 fronts over 6 levels, root separator = one site
    P, ex = _check_plan(lattice((256,), "nn", 0), 32)
    assert P.n_fronts == 63 and P.n_levels == 6
    assert ex["nj"][ex["parent"] < 0].tolist() == [4]
    # 3D 24^3 x 4: the top separator is one 24 x 24 plane of sites (2304 rows)
    sysd = lattice((24, 24, 24), "nn", 2)
    P = nd.Plan(sysd["n"], sysd["row_ptr"], sysd["col"], sysd["coords"], 32)
    ex = P.export()
    assert ex["nj"][ex["parent"] < 0].tolist() == [2304]
    assert P.max_u <= 2304 + 4 * 24
    flops, _ = P.model()
    assert 7.5e11 < flops < 9.5e11


def test_chain_dissection_has_one_atom_separators():
    # Fig. 1: a ten-atom s-valent chain; every separator is a single atom and
    # the top separator splits the chain into two domains of 5 and 4 atoms.
    n = 10
    rows, cols = [], []
    for i in range(n):
        for j in (i - 1, i, i + 1):
            if 0 <= j < n:
                rows.append(i)
                cols.append(j)
    row_ptr = np.searchsorted(rows, np.arange(n + 1))
    coords = np.stack([np.arange(n, dtype=float), np.zeros(n), np.zeros(n)], 1)
    P = nd.Plan(n, row_ptr, np.array(cols), coords, 2)
    ex = P.export()
    seps = [f for f in range(P.n_fronts) if np.any(ex["parent"] == f)]
    assert all(ex["nj"][f] == 1 for f in seps)
    root = int(np.nonzero(ex["parent"] < 0)[0][0])
    top_atom = ex["perm"][ex["j0"][root]]
    assert sorted([top_atom, n - 1 - top_atom]) == [4, 5]


def test_plan_empty_and_disconnected():
    # an empty structure is rejected; a pattern with no off-diagonal entries
    # (n disconnected rows) is one front holding every row, with no update
    with pytest.raises(nd.NdrhoError) as e:
        nd.Plan(0, np.array([0], dtype=np.int64), np.array([], dtype=np.int32), None, 8)
    assert e.value.name == "EINVAL"
    p = nd.Plan(3, np.array([0, 1, 2, 3], dtype=np.int64), np.array([0, 1, 2], dtype=np.int32), None, 8)
    ex = p.export()
    assert p.n_fronts == 1 and p.n_levels == 1
    assert int(ex["nj"][0]) == 3 and int(ex["nu"][0]) == 0
    assert sorted(int(x) for x in ex["perm"]) == [0, 1, 2]


def test_plan_rejects_front_beyond_32_bit_element_indexing():
    # a chain of 65536 rows kept as one leaf front: its 65536 x 65536 panel has
    # 2^32 elements, beyond the 32-bit element numbering of the extend-add
    # and gather kernels, so the plan is refused before anything is sized
    n = 1 << 16
    i = np.arange(n)
    rows = np.concatenate([i, i[:-1], i[1:]])
    cols = np.concatenate([i, i[1:], i[:-1]])
    order = np.lexsort((cols, rows))
    rows, cols = rows[order], cols[order]
    row_ptr = np.searchsorted(rows, np.arange(n + 1))
    with pytest.raises(nd.NdrhoError) as e:
        nd.Plan(n, row_ptr, cols, None, 1 << 30)
    assert e.value.name == "EINVAL" and "2^32" in str(e.value)


def test_plan_rejects_bad_csr():
    sysd = lattice((4, 3), "nn", 0)
    col = sysd["col"].copy()
    col[5], col[6] = col[6], col[5]                 # unsorted row
    with pytest.raises(nd.NdrhoError) as e:
        nd.Plan(sysd["n"], sysd["row_ptr"], col, None, 8)
    assert e.value.name == "EINVAL"
    rp = sysd["row_ptr"].copy()
    rp[0] = 1
    with pytest.raises(nd.NdrhoError):
        nd.Plan(sysd["n"], rp, sysd["col"], None, 8)


# --------------------------------------------------------- numpy model of the fronts

def _model_selected_inverse(P, ex, x_perm):
    """Front-by-front block LDL^T and selected inversion in numpy, laid out in
    the library's panel format; returns the flat panel array."""
    nf = P.n_fronts
    j0, nj, nu, parent = ex["j0"], ex["nj"], ex["nu"], ex["parent"]
    children = [[] for _ in range(nf)]
    for f in range(nf):
        if parent[f] >= 0:
            children[parent[f]].append(f)
    U = [ex["u_rows"][ex["u_off"][f]:ex["u_off"][f] + nu[f]] for f in range(nf)]
    rel = [ex["rel"][ex["u_off"][f]:ex["u_off"][f] + nu[f]] for f in range(nf)]
    ainv, lmat, upd = {}, {}, {}
    for f in range(nf):
        J = np.arange(j0[f], j0[f] + nj[f])
        idx = np.concatenate([J, U[f]])
        F = np.zeros((len(idx), len(idx)), dtype=complex)
        F[:, :nj[f]] = x_perm[np.ix_(idx, J)]
        F[:nj[f], nj[f]:] = x_perm[np.ix_(J, U[f])]
        for c in children[f]:
            F[np.ix_(rel[c], rel[c])] += upd[c]
        a = F[:nj[f], :nj[f]]
        b = F[nj[f]:, :nj[f]]
        ainv[f] = np.linalg.inv(a)
        lmat[f] = b @ ainv[f]
        upd[f] = F[nj[f]:, nj[f]:] - lmat[f] @ b.T
    gjj, guj, guu = {}, {}, {}
    for f in range(nf - 1, -1, -1):
        if parent[f] < 0:
            gjj[f] = ainv[f]
            guj[f] = np.zeros((0, nj[f]), dtype=complex)
            guu[f] = np.zeros((0, 0), dtype=complex)
            continue
        p = parent[f]
        gfull = np.block([[gjj[p], guj[p].T], [guj[p], guu[p]]])
        guu[f] = gfull[np.ix_(rel[f], rel[f])]
        guj[f] = -guu[f] @ lmat[f]
        gjj[f] = ainv[f] - lmat[f].T @ guj[f]
    _, _, poff = P.slots()
    flat = np.zeros(P.panel_total, dtype=complex)
    for f in range(nf):
        pan = np.vstack([gjj[f], guj[f]])
        flat[poff[f]:poff[f] + pan.size] = pan.ravel(order="F")
    return flat


@pytest.mark.parametrize("dims,nb,leaf,alpha", [((30,), "nn", 8, 0.2 + 0.5j), ((7, 6), "nn2", 12, -0.3 + 0.314j),
                                                 ((4, 4, 5), "nn", 16, 1.0 + 2.0j)])
def test_front_model_through_plan_matches_dense_inverse(dims, nb, leaf, alpha):
    sysd = lattice(dims, nb, 7)
    n = sysd["n"]
    rows, cols = _pattern(sysd)
    h = np.zeros((n, n))
    s = np.zeros((n, n))
    h[rows, cols] = sysd["h"]
    s[rows, cols] = sysd["s"]
    x = alpha * s - h
    P, ex = _check_plan(sysd, leaf)
    perm = ex["perm"]
    flat = _model_selected_inverse(P, ex, x[np.ix_(perm, perm)])
    out, asm, _ = P.slots()
    g = np.linalg.inv(x)
    got = flat[out]
    ref = g[rows, cols]
    assert np.max(np.abs(got - ref)) < 1e-11 * np.abs(g).max()
    # the assembly table places X_ij where the model's fronts read it
    asm_flat = np.zeros(P.panel_total, dtype=complex)
    asm_flat[asm[asm >= 0]] = x[rows[asm >= 0], cols[asm >= 0]]
    _, _, poff = P.slots()
    for f in range(P.n_fronts):
        J = np.arange(ex["j0"][f], ex["j0"][f] + ex["nj"][f])
        U = ex["u_rows"][ex["u_off"][f]:ex["u_off"][f] + ex["nu"][f]]
        idx = np.concatenate([J, U])
        want = x[np.ix_(perm[idx], perm[J])]
        have = asm_flat[poff[f]:poff[f] + want.size].reshape(want.shape, order="F")
        assert np.array_equal(have, want)


def _long_tail_system(dims, nb, seed):
    # a lattice plus three rows overlapping 30 % of all rows, centred at a
    # corner of the lattice (where they spoil the geometric cuts most)
    from synth import with_long_tail
    base = lattice(dims, nb, seed)
    sysd = with_long_tail(base, m=3, frac=0.3, seed=seed + 1)
    sysd["coords"][base["n"]:] = base["coords"][0]
    return base, sysd


@pytest.mark.parametrize("dims,nb,leaf", [((5, 4, 4), "nn", 16), ((9, 8), "nn2", 16)])
def test_long_tail_screening(dims, nb, leaf):
    # step (ii) of the dissection: the long-tail rows join the top separator
    # before the cut; the plan stays a valid front tree (closure, tables),
    # the front model through it reproduces the dense inverse, the work
    # drops, and a plain lattice is planned as without screening
    base, sysd = _long_tail_system(dims, nb, 21)
    n = sysd["n"]
    P, ex = _check_plan(sysd, leaf, long_tail=2.0)
    roots = [f for f in range(P.n_fronts) if ex["parent"][f] < 0]
    root_rows = {int(ex["perm"][j]) for f in roots for j in range(ex["j0"][f], ex["j0"][f] + ex["nj"][f])}
    assert set(range(base["n"], n)) <= root_rows
    P0 = nd.Plan(n, sysd["row_ptr"], sysd["col"], sysd["coords"], leaf)
    assert P.model()[0] < 0.9 * P0.model()[0]
    rows, cols = _pattern(sysd)
    h = np.zeros((n, n))
    s = np.zeros((n, n))
    h[rows, cols] = sysd["h"]
    s[rows, cols] = sysd["s"]
    x = (0.3 + 0.4j) * s - h
    perm = ex["perm"]
    flat = _model_selected_inverse(P, ex, x[np.ix_(perm, perm)])
    out, _, _ = P.slots()
    g = np.linalg.inv(x)
    assert np.max(np.abs(flat[out] - g[rows, cols])) < 1e-11 * np.abs(g).max()
    Pb = nd.Plan(base["n"], base["row_ptr"], base["col"], base["coords"], leaf, long_tail=2.0)
    Pb0 = nd.Plan(base["n"], base["row_ptr"], base["col"], base["coords"], leaf)
    assert np.array_equal(Pb.export()["perm"], Pb0.export()["perm"])


def test_long_tail_option_validated():
    sysd = lattice((4, 4), "nn", 3)
    with pytest.raises(nd.NdrhoError):
        nd.Plan(sysd["n"], sysd["row_ptr"], sysd["col"], sysd["coords"], 16, long_tail=0.5)


def test_pivot_variant_option_validated():
    # checked before any device call: FP32 mode accepts variants 0-2, split-BF16 mode 0-7, and -1
    for precision, pv in (("mixed_fp32", 6), ("mixed_bf16x3", 8), ("mixed_bf16x3", -2)):
        with pytest.raises(nd.NdrhoError) as e:
            nd.Context(0, precision=precision, pivot_variant=pv)
        assert e.value.name == "EINVAL" and "pivot_variant" in str(e.value)


def test_small_front_option_validated():
    # the option is checked before any device call, so this runs on the host
    with pytest.raises(nd.NdrhoError) as e:
        nd.Context(0, small_fronts=2)
    assert e.value.name == "EINVAL" and "small_fronts" in str(e.value)


def test_long_tail_generator_keeps_s_positive_definite_and_symmetric():
    base, sysd = _long_tail_system((5, 4, 4), "nn", 31)
    n = sysd["n"]
    rows, cols = _pattern(sysd)
    s = np.zeros((n, n))
    h = np.zeros((n, n))
    s[rows, cols] = sysd["s"]
    h[rows, cols] = sysd["h"]
    assert np.array_equal(s, s.T) and np.array_equal(h, h.T)
    assert np.linalg.eigvalsh(s).min() > 0.0
    deg = np.diff(sysd["row_ptr"])
    assert np.all(deg[base["n"]:] >= int(0.3 * base["n"]))


# --------------------------------------------------------- periodic cells

def test_periodic_square_lattice_of_fig2():
    # Sec. II C 1, Fig. 2: the s-valent nearest-neighbour square lattice of
    # 1024 atoms in a periodic cell.  The first separator consists of two
    # lines of atoms, there are six separator levels (0 ... 5), and every
    # innermost domain holds 9 atoms.
    sysd = lattice((32, 32), "nn", 0, norb=1, periodic=True)
    assert sysd["n"] == 1024 and sysd["cell"] == [32.0, 32.0, 0.0]
    P, ex = _check_plan(sysd, 16, cell=sysd["cell"])
    nf, parent, nj, depth = P.n_fronts, ex["parent"], ex["nj"], ex["depth"]
    leaves = [f for f in range(nf) if not np.any(parent == f)]
    seps = [f for f in range(nf) if np.any(parent == f)]
    roots = np.nonzero(parent < 0)[0]
    assert len(roots) == 1
    root = int(roots[0])
    top = ex["perm"][ex["j0"][root]:ex["j0"][root] + nj[root]]
    xy = sysd["coords"][top][:, :2]
    # two full lines along one axis: 2 x 32 atoms with two distinct coordinates on the other
    axis = [a for a in (0, 1) if len(np.unique(xy[:, a])) == 2]
    assert nj[root] == 64 and len(axis) == 1
    vals = np.unique(xy[:, axis[0]])
    assert all(np.sum(xy[:, axis[0]] == v) == 32 for v in vals)
    assert sorted({int(depth[f]) for f in seps}) == [0, 1, 2, 3, 4, 5]
    assert {int(nj[f]) for f in leaves} == {9}
    # without the cell the wrapping bonds defeat the cuts: one huge front
    P0 = nd.Plan(sysd["n"], sysd["row_ptr"], sysd["col"], sysd["coords"], 16)
    assert P0.max_j > 900
    assert P.model()[0] < 0.05 * P0.model()[0]


@pytest.mark.parametrize("dims,nb,leaf,alpha", [((24,), "nn", 8, 0.2 + 0.5j), ((8, 7), "nn2", 16, -0.3 + 0.314j),
                                                 ((4, 5, 3), "nn", 16, 1.0 + 2.0j), ((6, 2), "nn", 8, 0.5j)])
def test_periodic_front_model_matches_dense_inverse(dims, nb, leaf, alpha):
    # periodic lattices with 4 random orbitals per site (an axis shorter
    # than 3 stays open): the plan is a valid front tree and the numpy front
    # model through it gives the dense inverse on the pattern
    sysd = lattice(dims, nb, 11, periodic=True)
    n = sysd["n"]
    rows, cols = _pattern(sysd)
    h = np.zeros((n, n))
    s = np.zeros((n, n))
    h[rows, cols] = sysd["h"]
    s[rows, cols] = sysd["s"]
    assert np.array_equal(h, h.T) and np.linalg.eigvalsh(s).min() > 0.0
    x = alpha * s - h
    P, ex = _check_plan(sysd, leaf, cell=sysd["cell"])
    flat = _model_selected_inverse(P, ex, x[np.ix_(ex["perm"], ex["perm"])])
    out, _, _ = P.slots()
    g = np.linalg.inv(x)
    assert np.max(np.abs(flat[out] - g[rows, cols])) < 1e-11 * np.abs(g).max()
    # the wrapping bonds are present (degree of a corner site equals the bulk's along periodic axes)
    assert np.diff(sysd["row_ptr"]).min() == np.diff(sysd["row_ptr"]).max() or min(dims + (3,)) < 3


def test_periodic_cell_rejected_without_coordinates_or_with_bad_lengths():
    sysd = lattice((6, 6), "nn", 0, norb=1, periodic=True)
    with pytest.raises(nd.NdrhoError) as e:
        nd.Plan(sysd["n"], sysd["row_ptr"], sysd["col"], None, 8, cell=sysd["cell"])
    assert e.value.name == "EINVAL"
    with pytest.raises(nd.NdrhoError) as e:
        nd.Plan(sysd["n"], sysd["row_ptr"], sysd["col"], sysd["coords"], 8, cell=[6.0, -1.0, 0.0])
    assert e.value.name == "EINVAL"
    # open lattices are planned as before when a zero cell is given
    op = lattice((6, 5, 4), "nn", 2)
    a = nd.Plan(op["n"], op["row_ptr"], op["col"], op["coords"], 16).export()["perm"]
    b = nd.Plan(op["n"], op["row_ptr"], op["col"], op["coords"], 16, cell=[0.0, 0.0, 0.0]).export()["perm"]
    assert np.array_equal(a, b)


def test_bench_refuses_several_gpus():
    # the benchmark measures one GPU; --gpus N > 1 exits with a message
    # before touching a device
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
