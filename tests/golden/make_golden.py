"""Write the stored expected values used by the full-size parity tests.

Calls only the oracle (and the seeded input generator).  Usage:

    python tests/golden/make_golden.py cubic3d_24x4 [--procs 6]
    python tests/golden/make_golden.py square2d_64x4
    python tests/golden/make_golden.py square2d_64x4 --edm   # rho and e (Eq. (10))

    python tests/golden/make_golden.py multi2d_8x4         # the eight lattices, one file
    python tests/golden/make_golden.py cubic3d_24x4 --periodic   # the lattice closed into a periodic cell

For each workload: rows j at chosen lattice sites, and rho_ij on every pattern
entry of those rows (by symmetry also column j), from Eq. (8) with one sparse
LU per pole (oracle.sampled).  The sites are picked by geometry so that the
sample meets the dissection's levels: a pair of neighbouring sites across the
middle of the first axis (one of the two lies in the top separator, which
cuts the lattice there), a pair across the middle of the second axis in one
half (a first-level separator), and the two far corners (innermost
domains).  mu is fixed (stated in the file), since the half-filling mu of
these sizes is not available from dense algebra.  With --periodic the lattice
is closed into a periodic cell along every axis (couplings across the cell
boundary folded onto the pattern) and the same sites are sampled; the 3D cell
takes the GMRES route (its separators are two planes, so sparse LU fills in
far more).
"""
import argparse
import json
import multiprocessing as mp
import os
import sys
import time

# one BLAS thread per worker process: threaded BLAS state inherited through
# fork makes the pooled workers spin
for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS"):
    os.environ.setdefault(_v, "1")

import numpy as np  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import sampled  # noqa: E402
from synth import CONFIGS, BETA, config_system  # noqa: E402

MU = {"cubic3d_24x4": 0.0, "square2d_64x4": 0.0, "cubic3d_40x4": 0.0, "multi2d_8x4": 0.0}
N_ROWS = {"cubic3d_24x4": 8, "square2d_64x4": 8, "cubic3d_40x4": 4, "multi2d_8x4": 8}
GMRES = {"cubic3d_40x4"}   # sparse LU of every shifted matrix is out of host reach


def sample_sites(dims, count):
    """Lattice sites of the sample: the middle pair of the first axis, the
    middle pair of the second axis in one half, other mid-level sites, and
    the far corners (the first `count` of them, corners always kept)."""
    d = [x for x in dims if x > 1]
    if len(d) == 3:
        L = d[0]
        c, q = L // 2, L // 4
        mid = [(c - 1, q, q), (c, q, q), (q, q, c), (c - 1, L - 1 - q, c), (c, L - 1 - q, c), (q, c, L - 1 - q)]
        corners = [(0, 0, 0), (L - 1, L - 1, L - 1)]
    else:
        l0, l1 = d[0], d[1]
        c0, c1 = l0 // 2, l1 // 2
        mid = [(c0 - 1, l1 // 4), (c0, l1 // 4), (l0 // 4, c1 - 1), (l0 // 4, c1), (l0 - 1 - l0 // 4, c1 - 1),
               (l0 - 1 - l0 // 4, c1)]
        corners = [(0, 0), (l0 - 1, l1 - 1)]
    if count <= 4:
        return mid[:2] + [mid[2]] + corners[:1]
    return mid[:count - 2] + corners


def sample_rows(dims, count):
    """Basis rows (4 orbitals per site, x fastest) of the sample sites, the
    orbital cycling through 0..3."""
    full = tuple(dims) + (1,) * (3 - len(dims))
    rows = []
    for k, site in enumerate(sample_sites(dims, count)):
        x, y, z = tuple(site) + (0,) * (3 - len(site))
        rows.append(4 * (x + full[0] * (y + full[1] * z)) + k % 4)
    return sorted(rows)


def one_system(name, sysd, n_poles, count, edm, pool, gmres=False):
    rows = np.asarray(sample_rows(sysd["dims"], count))
    n = sysd["n"]
    h, s = sampled.csr_matrices(n, sysd["row_ptr"], sysd["col"], sysd["h"], sysd["s"])
    e_cols = None
    if edm:
        cols, e_cols = sampled.rho_edm_columns(h, s, MU[name], BETA, n_poles, rows, pool=pool)
    elif name in GMRES or gmres:
        cols = sampled.rho_columns_gmres(h, s, MU[name], BETA, n_poles, rows, pool=pool)
    else:
        cols = sampled.rho_columns(h, s, MU[name], BETA, n_poles, rows, pool=pool)
    entries, values, e_values = [], [], []
    for k, j in enumerate(rows):
        for e in range(sysd["row_ptr"][j], sysd["row_ptr"][j + 1]):
            i = int(sysd["col"][e])
            entries.append(int(e))
            values.append(float(cols[i, k]))     # rho_ji = rho_ij
            if e_cols is not None:
                e_values.append(float(e_cols[i, k]))
    return rows, entries, values, e_values


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workload")
    ap.add_argument("--procs", type=int, default=6)
    ap.add_argument("--edm", action="store_true",
                    help="also the energy density matrix e of Eq. (10) on the same entries (sparse LU route)")
    ap.add_argument("--periodic", action="store_true", help="the workload's lattice in a periodic cell")
    a = ap.parse_args()
    name = a.workload
    n_poles = CONFIGS[name]["n_poles"]
    t0 = time.time()
    gmres = a.periodic and len([d for d in CONFIGS[name]["dims"] if d > 1]) == 3
    src = ("oracle.sampled.rho_columns_gmres (GMRES per pole and column, rtol 1e-13, Eq. (8))" if name in GMRES or gmres
           else "oracle.sampled.rho_columns (sparse LU per pole, Eq. (8))")
    if a.edm:
        src = "oracle.sampled.rho_edm_columns (sparse LU per pole, Eqs. (8) and (10))"
    with mp.get_context("fork").Pool(a.procs) as pool:
        if name == "multi2d_8x4":
            members = []
            for i in range(len(CONFIGS[name]["dims"])):
                sysd = config_system(name, i)
                rows, entries, values, _ = one_system(name, sysd, n_poles, N_ROWS[name], False, pool)
                members.append({"dims": list(sysd["dims"][:2]), "seed": int(sysd["seed"]),
                                "rows": [int(r) for r in rows], "entries": entries, "values": values})
                print("member %d: %d entries, %.0f s" % (i, len(entries), time.time() - t0), flush=True)
            out = {"workload": name, "source": src, "mu": MU[name], "beta": BETA, "n_poles": n_poles,
                   "members": members, "seconds": time.time() - t0}
        else:
            sysd = config_system(name, periodic=a.periodic)
            rows, entries, values, e_values = one_system(name, sysd, n_poles, N_ROWS[name], a.edm, pool, gmres)
            out = {"workload": name + ("_periodic" if a.periodic else ""), "source": src, "cell": sysd["cell"],
                   "mu": MU[name], "beta": BETA, "n_poles": n_poles, "rows": [int(r) for r in rows],
                   "entries": entries, "values": values, "seconds": time.time() - t0}
            if a.edm:
                out["e_values"] = e_values
    tag = name + ("_periodic" if a.periodic else "")
    path = os.path.join(HERE, ("edm_sampled_%s.json" if a.edm else "rho_sampled_%s.json") % tag)
    with open(path, "w") as f:
        json.dump(out, f)
    print("wrote", path, "in %.0f s" % out["seconds"])


if __name__ == "__main__":
    main()
