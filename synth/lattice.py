"""Random-block tight-binding lattices shaped like the paper's test systems.

The paper times its inverse on s-valent nearest-neighbour tight-binding
chains, square and cubic lattices (Sec. III, Fig. 4).  These inputs keep that
geometry with 4 orbitals per site and random blocks:

* site index s = x + Lx (y + Ly z) (x fastest); basis index 4 s + orbital;
  the coordinates of every orbital are its site's lattice coordinates;
* open boundaries, or periodic ones (``periodic=True``: bonds also join
  the last and the first site along every axis of length >= 3, the
  couplings of the cell with its images folded onto one matrix);
* H onsite block: 4x4 symmetric, upper triangle (with diagonal) iid N(0, 1) eV;
* H bond block: an independent 4x4 block per bond, iid N(0, 0.5) eV (0.5 is
  the standard deviation), H_ts = H_st^T;
* S onsite block: identity; S bond block: 0.05 * iid N(0, 1), S_ts = S_st^T;
* neighbours: "nn" = the 2 d axis neighbours, "nn2" = nn plus the face
  diagonals (4 in 2D, 12 in 3D).

Random numbers are drawn in a fixed order from numpy's default_rng(seed):
onsite blocks (all sites), then H bond blocks, then S bond blocks, bonds
enumerated offset by offset and, within an offset, by increasing site index.
"""
import numpy as np

_NN = [(1, 0, 0), (0, 1, 0), (0, 0, 1)]
_NN2 = [(1, 1, 0), (1, -1, 0), (1, 0, 1), (1, 0, -1), (0, 1, 1), (0, 1, -1)]


def _bonds(dims, offsets, periodic=False):
    lx, ly, lz = dims
    xs, ys, zs = np.meshgrid(np.arange(lx), np.arange(ly), np.arange(lz), indexing="ij")
    # lexicographic site order with x fastest
    x = xs.transpose(2, 1, 0).ravel()
    y = ys.transpose(2, 1, 0).ravel()
    z = zs.transpose(2, 1, 0).ravel()
    src, dst = [], []
    for dx, dy, dz in offsets:
        tx, ty, tz = x + dx, y + dy, z + dz
        if periodic:   # axes of length >= 3 wrap round
            tx = np.where(lx >= 3, tx % lx, tx)
            ty = np.where(ly >= 3, ty % ly, ty)
            tz = np.where(lz >= 3, tz % lz, tz)
        ok = (tx >= 0) & (tx < lx) & (ty >= 0) & (ty < ly) & (tz >= 0) & (tz < lz)
        s = np.nonzero(ok)[0]
        t = tx[ok] + lx * (ty[ok] + ly * tz[ok])
        src.append(s)
        dst.append(t)
    if src:
        return np.concatenate(src), np.concatenate(dst), np.stack([x, y, z], axis=1)
    return np.zeros(0, np.int64), np.zeros(0, np.int64), np.stack([x, y, z], axis=1)


def lattice(dims, neighbours="nn", seed=0, norb=4, onsite_std=1.0, hop_std=0.5, s_scale=0.05, periodic=False):
    """Build one system.  Returns a dict with n, row_ptr (int64), col (int32),
    h, s (float64, CSR order, both triangles), coords (n x 3 float64), dims,
    and cell: None (open), or with periodic=True the cell lengths along x,
    y, z (0 for an axis shorter than 3, which stays open)."""
    dims = tuple(int(d) for d in dims) + (1,) * (3 - len(dims))
    offsets = list(_NN)
    if neighbours == "nn2":
        offsets += _NN2
    elif neighbours != "nn":
        raise ValueError("neighbours must be 'nn' or 'nn2'")
    offsets = [o for o in offsets if all(dims[a] > 1 or o[a] == 0 for a in range(3))]
    src, dst, site_xyz = _bonds(dims, offsets, periodic)
    nsites = site_xyz.shape[0]
    nb = src.shape[0]
    rng = np.random.default_rng(seed)
    raw = rng.normal(0.0, onsite_std, (nsites, norb, norb))
    onsite = np.triu(raw) + np.transpose(np.triu(raw, 1), (0, 2, 1))
    hop = rng.normal(0.0, hop_std, (nb, norb, norb))
    sov = s_scale * rng.normal(0.0, 1.0, (nb, norb, norb))

    # COO of all 4x4 blocks: onsite, (s,t) and the transposed (t,s) block
    bi = np.arange(norb)
    rr = np.repeat(bi, norb)      # row orbital within block
    cc = np.tile(bi, norb)        # col orbital within block
    rows = [(norb * np.arange(nsites))[:, None] + rr[None, :],
            (norb * src)[:, None] + rr[None, :],
            (norb * dst)[:, None] + rr[None, :]]
    cols = [(norb * np.arange(nsites))[:, None] + cc[None, :],
            (norb * dst)[:, None] + cc[None, :],
            (norb * src)[:, None] + cc[None, :]]
    hv = [onsite.reshape(nsites, -1), hop.reshape(nb, -1),
          np.transpose(hop, (0, 2, 1)).reshape(nb, -1)]
    eye = np.broadcast_to(np.eye(norb).ravel(), (nsites, norb * norb))
    sv = [eye, sov.reshape(nb, -1), np.transpose(sov, (0, 2, 1)).reshape(nb, -1)]
    r = np.concatenate([a.ravel() for a in rows]).astype(np.int64)
    c = np.concatenate([a.ravel() for a in cols]).astype(np.int64)
    h = np.concatenate([a.ravel() for a in hv])
    s = np.concatenate([a.ravel() for a in sv])
    n = nsites * norb
    order = np.lexsort((c, r))
    r, c, h, s = r[order], c[order], h[order], s[order]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, r + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    coords = np.repeat(site_xyz.astype(np.float64), norb, axis=0)
    cell = [float(d) if d >= 3 else 0.0 for d in dims] if periodic else None
    return {"n": n, "row_ptr": row_ptr, "col": c.astype(np.int32), "h": h, "s": s,
            "coords": coords, "dims": dims, "neighbours": neighbours, "seed": seed, "cell": cell}


def with_long_tail(sysd, m=3, frac=0.3, seed=0, onsite_std=1.0, hop_std=0.1, s_offdiag=0.2):
    """Append m rows standing for basis functions with a long tail: each
    overlaps a random fraction `frac` of the existing rows.  Their H couplings
    are N(0, hop_std); their S couplings share the magnitude s_offdiag / (frac
    n) with random signs, so each new row's off-diagonal S sum is s_offdiag
    and S stays positive definite (unit diagonal).  Coordinates: the centre
    of the existing rows.  Returns a new system dict in the same format."""
    rng = np.random.default_rng(seed)
    n0 = sysd["n"]
    rp0, c0 = sysd["row_ptr"], sysd["col"].astype(np.int64)
    r0 = np.repeat(np.arange(n0, dtype=np.int64), np.diff(rp0))
    rows, cols, hv, sv = [r0], [c0], [sysd["h"]], [sysd["s"]]
    k = max(1, int(frac * n0))
    smag = s_offdiag / k
    for t in range(m):
        i = n0 + t
        nbr = np.sort(rng.choice(n0, size=k, replace=False)).astype(np.int64)
        hval = rng.normal(0.0, hop_std, k)
        sval = smag * rng.choice([-1.0, 1.0], k)
        rows += [np.full(k, i), nbr, np.array([i])]
        cols += [nbr, np.full(k, i), np.array([i])]
        hv += [hval, hval, rng.normal(0.0, onsite_std, 1)]
        sv += [sval, sval, np.ones(1)]
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    h = np.concatenate(hv)
    s = np.concatenate(sv)
    n = n0 + m
    order = np.lexsort((c, r))
    r, c, h, s = r[order], c[order], h[order], s[order]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, r + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    coords = np.vstack([sysd["coords"], np.repeat(sysd["coords"].mean(axis=0)[None, :], m, axis=0)])
    out = dict(sysd)
    out.update({"n": n, "row_ptr": row_ptr, "col": c.astype(np.int32), "h": h, "s": s, "coords": coords})
    return out


# The five workloads: 1D chain, 2D lattice, 3D lattice, eight uneven 2D
# lattices, large 3D lattice.  kT = 0.1 eV everywhere (beta = 10 / eV).
CONFIGS = {
    "chain1d_256x4": {"dims": (256,), "neighbours": "nn", "seed": 0, "n_poles": 60},
    "square2d_64x4": {"dims": (64, 64), "neighbours": "nn2", "seed": 1, "n_poles": 80},
    "cubic3d_24x4": {"dims": (24, 24, 24), "neighbours": "nn", "seed": 2, "n_poles": 80},
    "multi2d_8x4": {"dims": [(k, k) for k in (32, 40, 48, 56, 64, 72, 80, 96)],
                    "neighbours": "nn", "seed": 30, "n_poles": 100},
    "cubic3d_40x4": {"dims": (40, 40, 40), "neighbours": "nn2", "seed": 4, "n_poles": 100},
}
KT_EV = 0.1
BETA = 1.0 / KT_EV


def config_system(name, index=0, periodic=False):
    """The system of a named workload (``index`` picks a lattice of multi2d;
    ``periodic`` closes the lattice into a periodic cell along every axis of
    length 3 or more)."""
    cfg = CONFIGS[name]
    if name == "multi2d_8x4":
        return lattice(cfg["dims"][index], cfg["neighbours"], cfg["seed"] + index, periodic=periodic)
    return lattice(cfg["dims"], cfg["neighbours"], cfg["seed"], periodic=periodic)
