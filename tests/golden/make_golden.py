"""Write the stored expected values used by the full-size parity tests.

Calls only the oracle (and the seeded input generator).  Usage:

    python tests/golden/make_golden.py cubic3d_24x4 [--procs 6]
    python tests/golden/make_golden.py square2d_64x4
    python tests/golden/make_golden.py square2d_64x4 --edm   # rho and e (Eq. (10))

For each workload: a seeded sample of rows j, and rho_ij on every pattern
entry of those rows (by symmetry also column j), from Eq. (8) with one sparse
LU per pole (oracle.sampled).  mu is fixed (stated in the file), since the
half-filling mu of these sizes is not available from dense algebra.
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

MU = {"cubic3d_24x4": 0.0, "square2d_64x4": 0.0, "cubic3d_40x4": 0.0}
N_ROWS = {"cubic3d_24x4": 8, "square2d_64x4": 8, "cubic3d_40x4": 2}
GMRES = {"cubic3d_40x4"}   # sparse LU of every shifted matrix is out of host reach


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workload")
    ap.add_argument("--procs", type=int, default=6)
    ap.add_argument("--edm", action="store_true",
                    help="also the energy density matrix e of Eq. (10) on the same entries (sparse LU route)")
    a = ap.parse_args()
    name = a.workload
    sysd = config_system(name)
    n = sysd["n"]
    n_poles = CONFIGS[name]["n_poles"]
    rng = np.random.default_rng(12345)
    rows = np.sort(rng.choice(n, size=N_ROWS[name], replace=False))
    h, s = sampled.csr_matrices(n, sysd["row_ptr"], sysd["col"], sysd["h"], sysd["s"])
    t0 = time.time()
    e_cols = None
    with mp.get_context("fork").Pool(a.procs) as pool:
        if a.edm:
            cols, e_cols = sampled.rho_edm_columns(h, s, MU[name], BETA, n_poles, rows, pool=pool)
        elif name in GMRES:
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
    src = ("oracle.sampled.rho_columns_gmres (GMRES per pole and column, rtol 1e-13, Eq. (8))" if name in GMRES
           else "oracle.sampled.rho_columns (sparse LU per pole, Eq. (8))")
    out = {"workload": name, "source": src,
           "mu": MU[name], "beta": BETA, "n_poles": n_poles, "rows": [int(r) for r in rows],
           "entries": entries, "values": values, "seconds": time.time() - t0}
    if a.edm:
        out["source"] = "oracle.sampled.rho_edm_columns (sparse LU per pole, Eqs. (8) and (10))"
        out["e_values"] = e_values
    path = os.path.join(HERE, ("edm_sampled_%s.json" if a.edm else "rho_sampled_%s.json") % name)
    with open(path, "w") as f:
        json.dump(out, f)
    print("wrote", path, len(entries), "entries in %.0f s" % out["seconds"])


if __name__ == "__main__":
    main()
