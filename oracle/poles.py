"""Continued-fraction (CF) poles and residues of the Fermi-Dirac function.

Paper Sec. II B, Eq. (7): the Fermi function 1/(1+e^x) is written as 1/2 minus
a continued fraction in (x/2)^2 with partial denominators 1, 3, 5, ...,
(2M-1), and equivalently as 1/2 + sum_p R_p [1/(x - i z_p) + 1/(x + i z_p)].
The paper states that z_p, R_p follow from an eigenvalue problem (its ref. on
the CF method) but does not print it.  The reading used here:

  With y = x/2 the fraction is 1/2 - (1/2) tanh_M(y), where
  tanh_M(y) = y / (1 + y^2/(3 + y^2/(5 + ... /(2M-1)))).  A continued fraction
  1/(d_1 - e_1^2/(d_2 - e_2^2/...)) is the (1,1) element of the inverse of the
  tridiagonal matrix with diagonal d and off-diagonal e; here d_k = 2k-1 and
  e_k^2 = -y^2, so tanh_M(y) = y [(B + i y A)^{-1}]_{11}, with
  B = diag(1, 3, ..., 2M-1) and A the M x M matrix with zero diagonal and unit
  off-diagonals.  Expanding in the B-orthonormal eigenpairs A v = lam B v gives
  f_M(x) = 1/2 + sum_{lam>0} R [1/(x - i z) + 1/(x + i z)] with
  z = 2/lam and R = -(v_0)^2 / lam^2.

``n_poles`` (N_p) counts the poles in the upper half plane; the CF depth is
M = 2 N_p, which has exactly N_p positive eigenvalues.
"""
import numpy as np
import scipy.linalg


def cf_poles(n_poles):
    """Return (z, R), each of length n_poles, sorted by increasing z.

    Eq. (7) through the generalized symmetric eigenproblem A v = lam B v of
    size M = 2 n_poles (reading stated in the module docstring).
    """
    if n_poles < 1:
        raise ValueError("n_poles must be >= 1")
    m = 2 * n_poles
    a = np.zeros((m, m))
    idx = np.arange(m - 1)
    a[idx, idx + 1] = 1.0
    a[idx + 1, idx] = 1.0
    b = np.diag(2.0 * np.arange(1, m + 1) - 1.0)
    lam, v = scipy.linalg.eigh(a, b)          # v^T B v = I
    pos = lam > 0
    lam = lam[pos]
    v0 = v[0, pos]
    z = 2.0 / lam
    r = -(v0 ** 2) / lam ** 2
    order = np.argsort(z)
    return z[order], r[order]


def fermi(x):
    """Exact Fermi-Dirac function 1/(1+e^x), evaluated without overflow."""
    x = np.asarray(x, dtype=np.float64)
    return 0.5 * (1.0 - np.tanh(0.5 * x))


def fermi_cf_backward(x, depth):
    """Truncated CF of Eq. (7), evaluated by backward recurrence.

    Depth ``depth`` = M means the innermost partial denominator is 2M-1.  This
    evaluation never forms poles, so it checks ``cf_poles`` independently.
    """
    x = np.asarray(x, dtype=np.float64)
    y2 = (0.5 * x) ** 2
    t = np.full_like(x, 2.0 * depth - 1.0)
    for k in range(depth - 1, 0, -1):
        t = (2.0 * k - 1.0) + y2 / t
    return 0.5 - 0.25 * x / t


def fermi_pole_form(x, z, r):
    """Pole form of Eq. (7): 1/2 + sum_p R_p [1/(x-iz_p) + 1/(x+iz_p)]."""
    x = np.asarray(x, dtype=np.float64)
    acc = np.full_like(x, 0.5)
    for zp, rp in zip(z, r):
        acc = acc + rp * (2.0 * x / (x * x + zp * zp))
    return acc


def pole_shifts_and_weights(mu, beta, n_poles):
    """alpha_p = mu + i z_p / beta and w_p = -(4/beta) R_p (Eq. (8)).

    With these, rho = M0 + sum_p w_p Re G(alpha_p), because
    Im(-i c) = -Re(c) for the term -(4i/beta) G(alpha_p) R_p of Eq. (8).
    """
    z, r = cf_poles(n_poles)
    alpha = mu + 1j * z / beta
    w = -(4.0 / beta) * r
    return alpha, w
