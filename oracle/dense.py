"""Dense FP64 reference for the density matrix on the sparsity pattern.

Definitions followed (paper Sec. II):
  Eq. (2)   H c = eps S c, with the eigenvectors S-orthonormal (C^T S C = I).
  Eq. (5)   rho = -(2/pi) Im int G(E+i0) f((E-mu)/kT) dE; with the Lehmann form
            of G (Eq. (9)) this is rho = 2 C f(beta(eps-mu)) C^T, where the 2
            is the spin degeneracy.
  Eq. (6)   G(Z) = (Z S - H)^{-1}.
  Eq. (8)   rho = M0 + Im(-(4i/beta) sum_p G(alpha_p) R_p),
            alpha_p = mu + i z_p/beta.  M0 is the zeroth moment of G, whose
            exact value is S^{-1} (the constant 1/2 of Eq. (7) times spin 2).
  Eq. (10)  e = -(2/pi) Im int E G(E+i0) f((E-mu)/kT) dE, the energy density
            matrix: with Eq. (9) e = 2 C diag(eps f(beta(eps-mu))) C^T; its pole
            form is e = M1 + kappa M0 + Im(-(4i/beta) sum_p G(alpha_p) R_p alpha_p)
            with kappa = (4/beta) sum_p R_p (Eq. (11)) and M1 the first moment of
            G, exactly S^{-1} H S^{-1} = C diag(eps) C^T (G(Z) = sum_k M_k Z^-(k+1)).

All routines are dense, O(N^3), and meant for N up to a few thousand in
tests (larger N only in one-off golden-value scripts).
"""
import numpy as np
import scipy.linalg

from .poles import cf_poles, fermi, fermi_pole_form


def to_dense(m):
    """Dense float64 copy of a scipy sparse matrix or array."""
    if hasattr(m, "toarray"):
        return np.asarray(m.toarray(), dtype=np.float64)
    return np.asarray(m, dtype=np.float64)


def eigen(h, s):
    """Generalized eigenpairs of Eq. (2): returns (eps ascending, C), C^T S C = I."""
    eps, c = scipy.linalg.eigh(to_dense(h), to_dense(s), driver="gvd")
    return eps, c


def electron_count(eps, mu, beta):
    """Number of electrons 2 sum_nu f(beta(eps_nu - mu)) (spin factor 2)."""
    return 2.0 * float(np.sum(fermi(beta * (eps - mu))))


def mu_for_count(eps, beta, n_electrons, tol=1e-13):
    """Chemical potential with 2 sum f = n_electrons, by bisection.

    The count is monotone increasing in mu, so bisection on a bracket that
    spans the spectrum by many kT converges unconditionally.
    """
    lo = float(eps[0]) - 50.0 / beta
    hi = float(eps[-1]) + 50.0 / beta
    for _ in range(400):
        mid = 0.5 * (lo + hi)
        if electron_count(eps, mid, beta) < n_electrons:
            lo = mid
        else:
            hi = mid
        if hi - lo < tol:
            break
    return 0.5 * (lo + hi)


def spectral_on_pattern(c, weights, rows, cols, chunk=1 << 15):
    """sum_nu C[i,nu] weights[nu] C[j,nu] for each pattern entry (i, j)."""
    rows = np.asarray(rows)
    cols = np.asarray(cols)
    out = np.empty(rows.shape[0], dtype=np.float64)
    cw = c * weights[None, :]
    for s0 in range(0, rows.shape[0], chunk):
        s1 = min(rows.shape[0], s0 + chunk)
        out[s0:s1] = np.einsum("ij,ij->i", cw[rows[s0:s1]], c[cols[s0:s1]])
    return out


def rho_exact_pattern(eps, c, mu, beta, rows, cols):
    """rho_ij = 2 sum_nu f(beta(eps_nu - mu)) C_i,nu C_j,nu (Eqs. (5), (9))."""
    return spectral_on_pattern(c, 2.0 * fermi(beta * (eps - mu)), rows, cols)


def rho_cf_pattern(eps, c, mu, beta, n_poles, rows, cols):
    """Same as ``rho_exact_pattern`` with f replaced by its N_p-pole truncation.

    This is what the pole sum of Eq. (8) reaches exactly (up to rounding):
    the truncated fraction f_M applied to the spectrum, Eq. (9).
    """
    z, r = cf_poles(n_poles)
    occ = fermi_pole_form(beta * (eps - mu), z, r)
    return spectral_on_pattern(c, 2.0 * occ, rows, cols)


def edm_exact_pattern(eps, c, mu, beta, rows, cols):
    """e_ij = 2 sum_nu eps_nu f(beta(eps_nu - mu)) C_i,nu C_j,nu (Eq. (10), first line, with Eq. (9))."""
    return spectral_on_pattern(c, 2.0 * eps * fermi(beta * (eps - mu)), rows, cols)


def edm_cf_pattern(eps, c, mu, beta, n_poles, rows, cols):
    """``edm_exact_pattern`` with f replaced by its N_p-pole truncation f_M.

    This is what the finite pole sum of Eq. (10) reaches exactly (up to
    rounding): each eigenvalue weighted by eps f_M(beta(eps - mu)).
    """
    z, r = cf_poles(n_poles)
    occ = fermi_pole_form(beta * (eps - mu), z, r)
    return spectral_on_pattern(c, 2.0 * eps * occ, rows, cols)


def first_moment_pattern(eps, c, rows, cols):
    """M1 = S^{-1} H S^{-1} = C diag(eps) C^T on the pattern (first moment of G, Eq. (12))."""
    return spectral_on_pattern(c, np.asarray(eps, dtype=np.float64), rows, cols)


def s_inverse_pattern(c, rows, cols):
    """M0 = S^{-1} = C C^T on the pattern (the Z -> infinity limit of Z G(Z))."""
    return spectral_on_pattern(c, np.ones(c.shape[1]), rows, cols)


def green_dense(h, s, alpha):
    """G(alpha) = (alpha S - H)^{-1}, Eq. (6), by a dense complex inverse."""
    x = alpha * to_dense(s).astype(np.complex128) - to_dense(h)
    return np.linalg.inv(x)


def rho_poles_dense(h, s, mu, beta, n_poles, rows, cols):
    """rho on the pattern from Eq. (8) with one dense inverse per pole.

    M0 is taken as the dense inverse of S; each pole adds
    w_p Re G(alpha_p)_ij with w_p = -(4/beta) R_p.  Independent of ``eigen``.
    """
    z, r = cf_poles(n_poles)
    sd = to_dense(s)
    rows = np.asarray(rows)
    cols = np.asarray(cols)
    rho = np.linalg.inv(sd)[rows, cols].copy()
    for zp, rp in zip(z, r):
        g = green_dense(h, s, mu + 1j * zp / beta)
        rho += (-(4.0 / beta) * rp) * g[rows, cols].real
    return rho


def edm_poles_dense(h, s, mu, beta, n_poles, rows, cols):
    """e on the pattern from the pole form of Eq. (10) with dense matrices.

    M0 = S^{-1} and M1 = S^{-1} H S^{-1} by dense products, kappa =
    (4/beta) sum_p R_p (Eq. (11)), and per pole the term
    Im(-(4i/beta) G R_p alpha_p) = w_p Re(alpha_p G(alpha_p)) with
    w_p = -(4/beta) R_p, G from a dense complex inverse.  Independent of
    ``eigen``.
    """
    z, r = cf_poles(n_poles)
    sd = to_dense(s)
    hd = to_dense(h)
    rows = np.asarray(rows)
    cols = np.asarray(cols)
    sinv = np.linalg.inv(sd)
    kappa = (4.0 / beta) * float(np.sum(r))
    e = (sinv @ hd @ sinv)[rows, cols] + kappa * sinv[rows, cols]
    for zp, rp in zip(z, r):
        alpha = mu + 1j * zp / beta
        g = green_dense(h, s, alpha)
        e += (-(4.0 / beta) * rp) * (alpha * g[rows, cols]).real
    return e


def eigenstates_near(h, s, xi, k):
    """The k eigenpairs of Eq. (2) whose eigenvalues lie nearest the energy xi
    (Appendix B, Eq. (B1): the states a block shift-invert iteration around
    xi converges to).  Returns (eps ascending, C with C^T S C = I)."""
    eps, c = eigen(h, s)
    idx = np.sort(np.argsort(np.abs(eps - xi), kind="stable")[:k])
    return eps[idx], c[:, idx]


def green_trace_s(h, s, alpha):
    """Tr(G(alpha) S) by a dense complex inverse (Eqs. (6), (42))."""
    return complex(np.trace(green_dense(h, s, alpha) @ to_dense(s)))


def trace_rho_s(rho_vals, s_vals):
    """Tr(rho S) = sum_ij rho_ij S_ji from pattern values (both symmetric, Eq. (40))."""
    return float(np.dot(rho_vals, s_vals))
