"""Sampled-column reference for systems too large for dense algebra.

For a few columns j, G(alpha_p) e_j = (alpha_p S - H)^{-1} e_j (Eq. (6)) is
obtained by a sparse solve, M0 e_j = S^{-1} e_j likewise, and column j of rho
follows from Eq. (8): rho e_j = S^{-1} e_j + sum_p w_p Re G(alpha_p) e_j with
w_p = -(4/beta) R_p.  Restricted to the pattern rows of column j this is the
exact density matrix up to the solver's rounding (sparse LU), or up to its
tolerance (GMRES).  The energy density matrix of Eq. (10) follows from the
same G columns (``rho_edm_columns``).
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spl

from .poles import cf_poles


def csr_matrices(n, row_ptr, col, hv, sv):
    h = sp.csr_matrix((hv, col, row_ptr), shape=(n, n))
    s = sp.csr_matrix((sv, col, row_ptr), shape=(n, n))
    return h, s


def unit_columns(n, cols, dtype):
    e = np.zeros((n, len(cols)), dtype=dtype)
    e[np.asarray(cols), np.arange(len(cols))] = 1.0
    return e


def green_columns_lu(h, s, alpha, cols):
    """(alpha S - H)^{-1}[:, cols] by a sparse LU factorization (SuperLU)."""
    x = (alpha * s.astype(np.complex128) - h).tocsc()
    lu = spl.splu(x)
    return lu.solve(unit_columns(h.shape[0], cols, np.complex128))


def s_inverse_columns(s, cols):
    """S^{-1}[:, cols] by a sparse LU factorization (the exact M0 of Eq. (8))."""
    lu = spl.splu(s.tocsc())
    return lu.solve(unit_columns(s.shape[0], cols, np.float64))


def green_column_gmres(h, s, alpha, j, rtol=1e-13):
    """(alpha S - H)^{-1} e_j by unpreconditioned GMRES(200)."""
    x = (alpha * s.astype(np.complex128) - h).tocsr()
    b = np.zeros(h.shape[0], dtype=np.complex128)
    b[j] = 1.0
    sol, info = spl.gmres(x, b, rtol=rtol, atol=0.0, restart=200, maxiter=50)
    if info != 0:
        raise RuntimeError("GMRES did not converge (info=%d)" % info)
    return sol


def rho_columns(h, s, mu, beta, n_poles, cols, pool=None):
    """Columns `cols` of rho (Eq. (8)) from one sparse LU per pole.

    pool: optional multiprocessing pool mapping over poles."""
    z, r = cf_poles(n_poles)
    alphas = mu + 1j * z / beta
    w = -(4.0 / beta) * r
    out = s_inverse_columns(s, cols).copy()
    args = [(h, s, a, cols) for a in alphas]
    cols_g = pool.starmap(green_columns_lu, args) if pool is not None else [green_columns_lu(*a) for a in args]
    for wp, g in zip(w, cols_g):
        out += wp * g.real
    return out


def rho_edm_columns(h, s, mu, beta, n_poles, cols, pool=None):
    """Columns `cols` of rho (Eq. (8)) and of the energy density matrix e
    (Eq. (10)) from the same sparse LU per pole.

    e e_j = M1 e_j + kappa M0 e_j + sum_p w_p Re(alpha_p G(alpha_p) e_j), with
    M0 = S^{-1}, M1 = S^{-1} H S^{-1} (two solves with S around a product with
    H) and kappa = (4/beta) sum_p R_p (Eq. (11)).
    """
    z, r = cf_poles(n_poles)
    alphas = mu + 1j * z / beta
    w = -(4.0 / beta) * r
    kappa = (4.0 / beta) * float(np.sum(r))
    lu_s = spl.splu(s.tocsc())
    m0 = lu_s.solve(unit_columns(s.shape[0], cols, np.float64))
    m1 = lu_s.solve(np.asarray(h @ m0))
    rho = m0.copy()
    e = m1 + kappa * m0
    args = [(h, s, a, cols) for a in alphas]
    cols_g = pool.starmap(green_columns_lu, args) if pool is not None else [green_columns_lu(*a) for a in args]
    for wp, a, g in zip(w, alphas, cols_g):
        rho += wp * g.real
        e += wp * (a * g).real
    return rho, e


def _gmres_block(h, s, alpha, cols, rtol):
    return np.stack([green_column_gmres(h, s, alpha, j, rtol) for j in cols], axis=1)


def s_inverse_columns_cg(s, cols, rtol=1e-14):
    """S^{-1}[:, cols] by conjugate gradients (S is symmetric positive definite)."""
    out = np.empty((s.shape[0], len(cols)))
    for k, j in enumerate(cols):
        b = np.zeros(s.shape[0])
        b[j] = 1.0
        x, info = spl.cg(s, b, rtol=rtol, atol=0.0, maxiter=2000)
        if info != 0:
            raise RuntimeError("CG did not converge (info=%d)" % info)
        out[:, k] = x
    return out


def rho_columns_gmres(h, s, mu, beta, n_poles, cols, pool=None, rtol=1e-13):
    """Columns `cols` of rho (Eq. (8)) with GMRES solves per pole and column
    (for systems whose sparse LU is too large); M0 columns by CG on S.
    Accurate to about rtol times the condition number of each shifted matrix."""
    z, r = cf_poles(n_poles)
    alphas = mu + 1j * z / beta
    w = -(4.0 / beta) * r
    out = s_inverse_columns_cg(s, cols).copy()
    args = [(h, s, a, cols, rtol) for a in alphas]
    cols_g = pool.starmap(_gmres_block, args) if pool is not None else [_gmres_block(*a) for a in args]
    for wp, g in zip(w, cols_g):
        out += wp * g.real
    return out
