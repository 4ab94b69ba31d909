"""Closed forms for open tight-binding chains (no eigensolver involved).

One orbital per site, n sites, H = a I + b T, S = I + s T, where T is the
adjacency matrix of the open path (|s| < 1/2 keeps S positive definite).  T,
H and S share the eigenvectors phi_k(j) = sqrt(2/(n+1)) sin(j k pi/(n+1)),
j, k = 1..n, with T phi_k = 2 c_k phi_k, c_k = cos(k pi/(n+1)).  Hence the
generalized eigenvalues of Eq. (2) are eps_k = (a + 2 b c_k)/(1 + 2 s c_k), the
S-normalised eigenvectors are phi_k / sqrt(1 + 2 s c_k), and

  rho_ij  = 2 sum_k f(beta(eps_k - mu)) phi_k(i) phi_k(j) / (1 + 2 s c_k)   (Eq. (5))
  e_ij    = 2 sum_k eps_k f(beta(eps_k - mu)) phi_k(i) phi_k(j) / (1 + 2 s c_k)   (Eq. (10))
  G(z)_ij = sum_k phi_k(i) phi_k(j) / ((1 + 2 s c_k)(z - eps_k))           (Eq. (6))

The block form takes 4x4 symmetric matrices E, V, W that commute (built from
one orthogonal Q): H = I (x) E + T (x) V, S = I (x) I + T (x) W.  Its
eigenvectors are phi_k (x) q_m with eps = (e_m + 2 c_k v_m)/(1 + 2 c_k w_m).
Sec. II C 1's s-valent chain (Fig. 1, Appendix A) is the scalar case.
"""
import numpy as np

from .poles import fermi


def chain_modes(n):
    """(c_k, phi) with phi[j-1, k-1] = sqrt(2/(n+1)) sin(j k pi/(n+1))."""
    k = np.arange(1, n + 1)
    j = np.arange(1, n + 1)
    phi = np.sqrt(2.0 / (n + 1)) * np.sin(np.outer(j, k) * np.pi / (n + 1))
    ck = np.cos(k * np.pi / (n + 1))
    return ck, phi


def chain_matrices(n, a, b, s):
    """Dense H, S of the scalar open chain."""
    t = np.zeros((n, n))
    i = np.arange(n - 1)
    t[i, i + 1] = 1.0
    t[i + 1, i] = 1.0
    return a * np.eye(n) + b * t, np.eye(n) + s * t


def chain_eigenvalues(n, a, b, s):
    ck, _ = chain_modes(n)
    return (a + 2.0 * b * ck) / (1.0 + 2.0 * s * ck)


def chain_rho(n, a, b, s, mu, beta):
    """Full n x n density matrix of the scalar chain from the closed form."""
    ck, phi = chain_modes(n)
    eps = (a + 2.0 * b * ck) / (1.0 + 2.0 * s * ck)
    occ = 2.0 * fermi(beta * (eps - mu)) / (1.0 + 2.0 * s * ck)
    return (phi * occ[None, :]) @ phi.T


def chain_edm(n, a, b, s, mu, beta):
    """Full n x n energy density matrix of the scalar chain (Eq. (10), first line):
    e_ij = 2 sum_k eps_k f(beta(eps_k - mu)) phi_k(i) phi_k(j) / (1 + 2 s c_k)."""
    ck, phi = chain_modes(n)
    eps = (a + 2.0 * b * ck) / (1.0 + 2.0 * s * ck)
    occ = 2.0 * eps * fermi(beta * (eps - mu)) / (1.0 + 2.0 * s * ck)
    return (phi * occ[None, :]) @ phi.T


def chain_green(n, a, b, s, z):
    """Full n x n Green function G(z) of the scalar chain from the closed form."""
    ck, phi = chain_modes(n)
    eps = (a + 2.0 * b * ck) / (1.0 + 2.0 * s * ck)
    d = 1.0 / ((1.0 + 2.0 * s * ck) * (z - eps))
    return (phi * d[None, :]) @ phi.T


def block_chain_matrices(n, q, e, v, w):
    """Dense H, S of the 4-orbital chain with E = Q diag(e) Q^T, V, W likewise."""
    t = np.zeros((n, n))
    i = np.arange(n - 1)
    t[i, i + 1] = 1.0
    t[i + 1, i] = 1.0
    em = q @ np.diag(e) @ q.T
    vm = q @ np.diag(v) @ q.T
    wm = q @ np.diag(w) @ q.T
    h = np.kron(np.eye(n), em) + np.kron(t, vm)
    s = np.kron(np.eye(n), np.eye(q.shape[0])) + np.kron(t, wm)
    return h, s


def block_chain_rho(n, q, e, v, w, mu, beta):
    """Density matrix of the block chain from phi_k (x) q_m eigenvectors."""
    ck, phi = chain_modes(n)
    norb = q.shape[0]
    rho = np.zeros((n * norb, n * norb))
    for m in range(norb):
        den = 1.0 + 2.0 * ck * w[m]
        eps = (e[m] + 2.0 * ck * v[m]) / den
        occ = 2.0 * fermi(beta * (eps - mu)) / den
        vec = np.kron(phi, q[:, m:m + 1])          # (n*norb, n) eigenvectors
        rho += (vec * occ[None, :]) @ vec.T
    return rho
