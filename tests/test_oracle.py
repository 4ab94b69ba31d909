"""Pins of the oracle against facts fixed by the paper and by mathematics.

Nothing here re-types an oracle formula: each check uses a value the paper
prints, a closed form derived independently (open chains), an invariant, or a
different algorithm (backward-recurrence continued fraction, dense inverse
versus eigen decomposition).
"""
import json
import os

import numpy as np
import pytest

from oracle import chain, dense, poles

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- poles (Eq. (7))

@pytest.mark.parametrize("n_poles", [1, 2, 7, 60, 80, 100])
def test_residue_sum_closed_form(n_poles):
    # tanh_M(y) -> M(M+1)/(2y) as y -> infinity for even depth M = 2 N_p, so
    # x f_M(x) -> ... gives sum_p R_p = -N_p(2N_p+1)/2 exactly.
    z, r = poles.cf_poles(n_poles)
    assert len(z) == n_poles and np.all(np.diff(z) > 0)
    assert r.sum() == pytest.approx(-n_poles * (2 * n_poles + 1) / 2.0, rel=1e-12)


@pytest.mark.parametrize("n_poles", [60, 80, 100])
def test_lowest_poles_are_matsubara(n_poles):
    # Near the real axis the CF poles coincide with the Matsubara poles
    # (2k+1) pi with residue -1 (Sec. II B: poles on the imaginary axis,
    # denser near the real axis).
    z, r = poles.cf_poles(n_poles)
    k = np.arange(8)
    assert np.allclose(z[:8], (2 * k + 1) * np.pi, rtol=1e-12, atol=0)
    assert np.allclose(r[:8], -1.0, rtol=0, atol=1e-12)
    assert np.all(np.diff(np.diff(z)) > -1e-9)       # spacing grows away from the axis


@pytest.mark.parametrize("n_poles", [3, 20, 60, 100])
def test_pole_form_equals_backward_recurrence(n_poles):
    z, r = poles.cf_poles(n_poles)
    x = np.linspace(-5.0 * n_poles ** 2, 5.0 * n_poles ** 2, 4001)
    a = poles.fermi_pole_form(x, z, r)
    b = poles.fermi_cf_backward(x, 2 * n_poles)
    assert np.max(np.abs(a - b)) < 2e-14


@pytest.mark.parametrize("n_poles", [60, 80, 100])
def test_cf_reproduces_fermi_in_double_precision(n_poles):
    # The paper states that 100 poles at 600 K reach double precision (Sec. II B).
    # With N_p poles the truncated fraction matches 1/(1+e^x) to a few ulp for
    # |x| up to about N_p^2/4.
    z, r = poles.cf_poles(n_poles)
    x = np.linspace(-n_poles ** 2 / 4.0, n_poles ** 2 / 4.0, 20001)
    err = np.abs(poles.fermi_pole_form(x, z, r) - poles.fermi(x))
    assert err.max() < 3e-14
    # far outside that window the truncation must show (the check is not vacuous)
    xf = np.array([50.0 * n_poles ** 2])
    assert abs(poles.fermi_pole_form(xf, z, r) - poles.fermi(xf))[0] > 1e-10


def test_pole_weights_sign_convention():
    # rho = M0 + sum_p w_p Re G(alpha_p) must give 2 f for one level at eps:
    # 1 + sum_p w_p Re 1/(alpha_p - eps) = 2 f(beta(eps - mu)).
    mu, beta = 0.3, 10.0
    alpha, w = poles.pole_shifts_and_weights(mu, beta, 60)
    for eps in (-3.0, -0.2, 0.3, 0.31, 0.5, 4.0):
        val = 1.0 + np.sum(w * (1.0 / (alpha - eps)).real)
        assert val == pytest.approx(2.0 * poles.fermi(beta * (eps - mu)), abs=1e-13)


# ------------------------------------------------------- closed-form chains (Eqs. (5), (6))

@pytest.mark.parametrize("n,a,b,s,mu", [(9, 0.2, -1.0, 0.1, 0.05), (40, -0.3, 0.7, -0.2, 0.4),
                                        (64, 1.0, 1.0, 0.0, 0.9)])
def test_dense_eigen_rho_matches_closed_form_chain(n, a, b, s, mu):
    beta = 10.0
    h, sm = chain.chain_matrices(n, a, b, s)
    eps, c = dense.eigen(h, sm)
    assert np.allclose(np.sort(chain.chain_eigenvalues(n, a, b, s)), eps, atol=1e-13)
    rows, cols = np.nonzero(np.ones((n, n)))
    got = dense.rho_exact_pattern(eps, c, mu, beta, rows, cols)
    ref = chain.chain_rho(n, a, b, s, mu, beta)[rows, cols]
    assert np.max(np.abs(got - ref)) < 1e-13


@pytest.mark.parametrize("n,a,b,s,mu,n_poles", [(12, 0.2, -1.0, 0.1, 0.05, 60), (30, -0.3, 0.7, -0.2, 0.4, 40)])
def test_pole_sum_by_dense_inverse_matches_closed_form_chain(n, a, b, s, mu, n_poles):
    # Eq. (8) with a dense inverse per pole reproduces the exact rho (the
    # spectrum is far inside the window where the CF is exact).
    beta = 10.0
    h, sm = chain.chain_matrices(n, a, b, s)
    rows, cols = np.nonzero(np.abs(h) + np.abs(sm) > 0)
    got = dense.rho_poles_dense(h, sm, mu, beta, n_poles, rows, cols)
    ref = chain.chain_rho(n, a, b, s, mu, beta)[rows, cols]
    assert np.max(np.abs(got - ref)) < 2e-13


@pytest.mark.parametrize("route", ["lu", "gmres"])
def test_sampled_columns_match_closed_form_chain(route):
    # the sampled-column routes of Eq. (8) (sparse LU per pole, or GMRES per
    # pole with CG for S^-1) reproduce the closed-form rho on the columns
    import scipy.sparse as sp
    from oracle import sampled
    n, a, b, s, mu, beta, n_poles = 50, 0.2, -1.0, 0.1, 0.05, 10.0, 60
    h, sm = chain.chain_matrices(n, a, b, s)
    hs, ss = sp.csr_matrix(h), sp.csr_matrix(sm)
    cols = np.array([0, 7, 31, 49])
    if route == "lu":
        got = sampled.rho_columns(hs, ss, mu, beta, n_poles, cols)
    else:
        got = sampled.rho_columns_gmres(hs, ss, mu, beta, n_poles, cols)
    ref = chain.chain_rho(n, a, b, s, mu, beta)[:, cols]
    assert np.max(np.abs(got - ref)) < 1e-12


def test_green_dense_matches_closed_form_chain():
    n, a, b, s = 17, 0.1, -0.8, 0.15
    h, sm = chain.chain_matrices(n, a, b, s)
    for zc in (0.3 + 0.314j, -1.0 + 2.0j, 0.0 + 500.0j):
        g = dense.green_dense(h, sm, zc)
        assert np.max(np.abs(g - chain.chain_green(n, a, b, s, zc))) < 1e-13 * max(1.0, np.abs(g).max())
        assert np.allclose(g, g.T, atol=1e-14)          # complex symmetric, not Hermitian


def test_block_chain_four_orbitals():
    rng = np.random.default_rng(5)
    q, _ = np.linalg.qr(rng.normal(size=(4, 4)))
    e = rng.normal(size=4)
    v = 0.5 * rng.normal(size=4)
    w = 0.1 * rng.uniform(-1, 1, size=4)
    n, mu, beta = 15, 0.1, 10.0
    h, sm = chain.block_chain_matrices(n, q, e, v, w)
    eps, c = dense.eigen(h, sm)
    rows, cols = np.nonzero(np.abs(h) + np.abs(sm) > 1e-15)
    got = dense.rho_exact_pattern(eps, c, mu, beta, rows, cols)
    ref = chain.block_chain_rho(n, q, e, v, w, mu, beta)[rows, cols]
    assert np.max(np.abs(got - ref)) < 1e-12
    got2 = dense.rho_poles_dense(h, sm, mu, beta, 60, rows, cols)
    assert np.max(np.abs(got2 - ref)) < 1e-12


# ------------------------------------------------------------- invariants

def _small_lattice(dims, nb, seed):
    import scipy.sparse as sp
    from synth import lattice
    sysd = lattice(dims, nb, seed)
    n = sysd["n"]
    h = sp.csr_matrix((sysd["h"], sysd["col"], sysd["row_ptr"]), shape=(n, n))
    s = sp.csr_matrix((sysd["s"], sysd["col"], sysd["row_ptr"]), shape=(n, n))
    rows = np.repeat(np.arange(n), np.diff(sysd["row_ptr"]))
    return sysd, h, s, rows, sysd["col"].astype(np.int64)


def test_trace_rho_s_equals_electron_count():
    # Eq. (40): Tr(rho S) = N_ideal at the half-filling mu; Tr needs rho only
    # on the pattern of S.
    sysd, h, s, rows, cols = _small_lattice((6, 5), "nn2", 11)
    beta = 10.0
    eps, c = dense.eigen(h, s)
    n = sysd["n"]
    mu = dense.mu_for_count(eps, beta, float(n))
    assert dense.electron_count(eps, mu, beta) == pytest.approx(n, abs=1e-9)
    rho = dense.rho_exact_pattern(eps, c, mu, beta, rows, cols)
    assert dense.trace_rho_s(rho, sysd["s"]) == pytest.approx(n, abs=1e-9)
    rho_p = dense.rho_poles_dense(h, s, mu, beta, 60, rows, cols)
    assert dense.trace_rho_s(rho_p, sysd["s"]) == pytest.approx(n, abs=1e-9)
    assert np.max(np.abs(rho_p - rho)) < 1e-12
    rho_cf = dense.rho_cf_pattern(eps, c, mu, beta, 60, rows, cols)
    assert np.max(np.abs(rho_cf - rho)) < 1e-12


# ------------------------------------------- energy density matrix (Eqs. (10)-(12))

@pytest.mark.parametrize("n,a,b,s,mu", [(9, 0.2, -1.0, 0.1, 0.05), (40, -0.3, 0.7, -0.2, 0.4)])
def test_edm_dense_eigen_matches_closed_form_chain(n, a, b, s, mu):
    beta = 10.0
    h, sm = chain.chain_matrices(n, a, b, s)
    eps, c = dense.eigen(h, sm)
    rows, cols = np.nonzero(np.ones((n, n)))
    got = dense.edm_exact_pattern(eps, c, mu, beta, rows, cols)
    ref = chain.chain_edm(n, a, b, s, mu, beta)[rows, cols]
    assert np.max(np.abs(got - ref)) < 1e-13
    # the first moment of G is S^-1 H S^-1 (the Z^-2 term of its expansion)
    m1 = dense.first_moment_pattern(eps, c, rows, cols)
    si = np.linalg.inv(sm)
    assert np.max(np.abs(m1 - (si @ h @ si)[rows, cols])) < 1e-13


@pytest.mark.parametrize("n,a,b,s,mu,n_poles", [(12, 0.2, -1.0, 0.1, 0.05, 60), (30, -0.3, 0.7, -0.2, 0.4, 80)])
def test_edm_pole_sum_by_dense_inverse_matches_closed_form_chain(n, a, b, s, mu, n_poles):
    # the pole form of Eq. (10) (first moment, kappa of Eq. (11) times M0,
    # and w_p Re(alpha_p G(alpha_p))) with dense inverses reproduces the
    # closed-form e; the kappa M0 term cancels most of the far poles' terms
    # (sum_p |w_p| reaches 2.6e3 at 80 poles), which sets the tolerance
    beta = 10.0
    h, sm = chain.chain_matrices(n, a, b, s)
    rows, cols = np.nonzero(np.abs(h) + np.abs(sm) > 0)
    got = dense.edm_poles_dense(h, sm, mu, beta, n_poles, rows, cols)
    ref = chain.chain_edm(n, a, b, s, mu, beta)[rows, cols]
    assert np.max(np.abs(got - ref)) < 1e-11
    # and so does the spectral form with the truncated fraction
    eps, c = dense.eigen(h, sm)
    cf = dense.edm_cf_pattern(eps, c, mu, beta, n_poles, rows, cols)
    assert np.max(np.abs(cf - ref)) < 1e-12


def test_edm_is_s_inverse_h_rho_and_traces_to_band_energy():
    # H C = S C eps with C^T S C = I gives e = S^-1 H rho for the full
    # matrices, and Tr(e S) = 2 sum_nu eps_nu f_nu (needs e only on the
    # pattern of S)
    sysd, h, s, rows, cols = _small_lattice((4, 3, 2), "nn2", 12)
    beta, n = 10.0, sysd["n"]
    eps, c = dense.eigen(h, s)
    mu = dense.mu_for_count(eps, beta, float(n))
    ii, jj = np.nonzero(np.ones((n, n)))
    rho_full = dense.rho_exact_pattern(eps, c, mu, beta, ii, jj).reshape(n, n)
    e_full = dense.edm_exact_pattern(eps, c, mu, beta, ii, jj).reshape(n, n)
    ref = np.linalg.solve(s.toarray(), h.toarray() @ rho_full)
    assert np.max(np.abs(e_full - ref)) < 1e-11
    e = dense.edm_exact_pattern(eps, c, mu, beta, rows, cols)
    band = 2.0 * float(np.sum(eps * poles.fermi(beta * (eps - mu))))
    assert dense.trace_rho_s(e, sysd["s"]) == pytest.approx(band, abs=1e-10)
    e_poles = dense.edm_poles_dense(h, s, mu, beta, 80, rows, cols)
    assert np.max(np.abs(e_poles - e)) < 1e-10


def test_edm_sampled_columns_match_closed_form_chain():
    # the sampled-column route of Eq. (10) (sparse LU per pole, M1 from two
    # solves with S) reproduces the closed-form e and rho on the columns
    import scipy.sparse as sp
    from oracle import sampled
    n, a, b, s, mu, beta, n_poles = 50, 0.2, -1.0, 0.1, 0.05, 10.0, 60
    h, sm = chain.chain_matrices(n, a, b, s)
    cols = np.array([0, 7, 31, 49])
    rho, e = sampled.rho_edm_columns(sp.csr_matrix(h), sp.csr_matrix(sm), mu, beta, n_poles, cols)
    assert np.max(np.abs(rho - chain.chain_rho(n, a, b, s, mu, beta)[:, cols])) < 1e-12
    assert np.max(np.abs(e - chain.chain_edm(n, a, b, s, mu, beta)[:, cols])) < 1e-11


def test_edm_with_h_proportional_to_s():
    # H = c S: every eigenvalue is c, so e = c rho = 2 c f(beta(c - mu)) S^-1
    sysd, _, s, rows, cols = _small_lattice((3, 3, 2), "nn", 13)
    beta, mu, cval, n_poles = 10.0, 0.05, 0.37, 60
    h = cval * s
    e = dense.edm_poles_dense(h, s, mu, beta, n_poles, rows, cols)
    rho = dense.rho_poles_dense(h, s, mu, beta, n_poles, rows, cols)
    assert np.max(np.abs(e - cval * rho)) < 1e-11
    want = 2.0 * cval * poles.fermi(beta * (cval - mu)) * np.linalg.inv(s.toarray())[rows, cols]
    assert np.max(np.abs(e - want)) < 1e-11


def test_green_trace_is_spectral_sum():
    # C^T S C = I gives Tr(G(alpha) S) = sum_nu 1/(alpha - eps_nu); its
    # -(2/pi) Im part near the real axis is a sum of Lorentzians (Eq. (42))
    sysd, h, s, rows, cols = _small_lattice((4, 3, 2), "nn", 14)
    eps, _ = dense.eigen(h, s)
    for alpha in (0.1 + 0.01j, -1.0 + 0.01j, 0.3 + 2.0j, 5.0 + 40.0j):
        got = dense.green_trace_s(h, s, alpha)
        ref = complex(np.sum(1.0 / (alpha - eps)))
        assert abs(got - ref) < 1e-10 * max(1.0, abs(ref))
        assert -(2.0 / np.pi) * got.imag > 0.0


def test_s_inverse_from_eigenvectors():
    sysd, h, s, rows, cols = _small_lattice((3, 3, 2), "nn", 2)
    eps, c = dense.eigen(h, s)
    got = dense.s_inverse_pattern(c, rows, cols)
    ref = np.linalg.inv(s.toarray())[rows, cols]
    assert np.max(np.abs(got - ref)) < 1e-13


def test_mu_bisection_brackets_gap_for_insulator():
    # Two flat levels at -1 and +1 (two-site molecule): half filling puts mu at 0.
    eps = np.array([-1.0, -1.0, 1.0, 1.0])
    mu = dense.mu_for_count(eps, 10.0, 4.0)
    assert mu == pytest.approx(0.0, abs=1e-10)


# ------------------------------------------------------------- Appendix A

def _appendix_a():
    with open(os.path.join(GOLDEN, "appendix_a.json")) as f:
        fx = json.load(f)
    x = np.zeros((7, 7))
    for i, j in fx["matrix_nonzeros"]:
        x[i - 1, j - 1] = fx["matrix_value"]
    return fx, x


def test_appendix_a_selected_inverse_dense():
    fx, x = _appendix_a()
    assert np.allclose(x, x.T)
    # G(0) = (0 S - H)^{-1} with H = -X gives X^{-1} through the oracle's routine
    g = dense.green_dense(-x, np.eye(7), 0.0)
    for i, j, v in fx["selected_inverse"]:
        assert g[i - 1, j - 1].real == pytest.approx(v, abs=1e-14)
    # every printed entry sits on the pattern, and every pattern entry is printed
    printed = {(i, j) for i, j, _ in fx["selected_inverse"]}
    assert printed == {tuple(p) for p in fx["matrix_nonzeros"]}


def test_appendix_a_is_the_chain_closed_form():
    fx, x = _appendix_a()
    order = [k - 1 for k in fx["chain_order"]]
    # chain with a = b = 1, s = 0 at z = 0: G(0) = -H^{-1} = -X^{-1}
    gc = chain.chain_green(7, 1.0, 1.0, 0.0, 0.0)
    inv_structured = np.empty((7, 7))
    for p, i in enumerate(order):
        for q, j in enumerate(order):
            inv_structured[i, j] = -gc[p, q]
    for i, j, v in fx["selected_inverse"]:
        assert inv_structured[i - 1, j - 1] == pytest.approx(v, abs=1e-13)


def test_appendix_a_intermediates():
    fx, x = _appendix_a()
    it = fx["intermediates"]
    # leaf domains {1},{2} with separator {3}; {4},{5} with {6}; top separator {7}
    a00, a01, c00 = x[0, 0], x[1, 1], x[2, 2]
    b00, b01 = x[2, 0], x[2, 1]
    s00 = c00 - b00 * (b00 / a00) - b01 * (b01 / a01)       # Eq. (20) with L = B A^{-1}
    assert [s00] == [it["S0"][0]]
    blk = x[np.ix_([0, 1, 2], [0, 1, 2])]
    pre = np.linalg.inv(blk)
    for i, j, v in it["precursor_X10_inv_selected"]:
        assert pre[i - 1, j - 1] == pytest.approx(v, abs=1e-14)
    # L_{1,0}^T = X_{left}^{-1} B_{1,0}^T and L_{1,1}^T likewise (Eq. (24))
    b10 = x[6, [0, 1, 2]]
    b11 = x[6, [3, 4, 5]]
    l10 = np.linalg.inv(x[np.ix_([0, 1, 2], [0, 1, 2])]) @ b10
    l11 = np.linalg.inv(x[np.ix_([3, 4, 5], [3, 4, 5])]) @ b11
    assert np.allclose(l10, it["L10T"]) and np.allclose(l11, it["L11T"])
    s10 = x[6, 6] - b10 @ l10 - b11 @ l11
    assert s10 == pytest.approx(it["S10"])


# ------------------------------------------------------------- selected eigenstates (Appendix B)

@pytest.mark.parametrize("n,a,b,s,xi,k", [(60, 0.1, -1.0, 0.12, 0.3, 5), (41, -0.2, 0.8, -0.2, -0.5, 8)])
def test_eigenstates_near_match_closed_form_chain(n, a, b, s, xi, k):
    # the k eigenvalues nearest xi of the open chain, from the closed form
    # eps_j = (a + 2 b c_j)/(1 + 2 s c_j) with eigenvectors phi_j / sqrt(1 + 2 s c_j)
    hm, sm = chain.chain_matrices(n, a, b, s)
    eps, c = dense.eigenstates_near(hm, sm, xi, k)
    ck, phi = chain.chain_modes(n)
    ref = (a + 2.0 * b * ck) / (1.0 + 2.0 * s * ck)
    pick = np.sort(np.argsort(np.abs(ref - xi))[:k])
    order = np.argsort(ref[pick])
    assert np.allclose(eps, ref[pick][order], rtol=0, atol=1e-12)
    for col, j in zip(c.T, pick[order]):
        v = phi[:, j] / np.sqrt(1.0 + 2.0 * s * ck[j])     # S-normalised closed-form vector
        assert abs(abs(v @ sm @ col) - 1.0) < 1e-10
    assert np.allclose(c.T @ sm @ c, np.eye(k), atol=1e-12)


def test_eigenstates_near_satisfy_shift_invert_relation():
    # Eq. (B1): (H - xi S)^{-1} S c = c / (eps - xi) for each returned pair
    from synth import lattice
    sysd = lattice((5, 4), "nn2", 3)
    n = sysd["n"]
    rows = np.repeat(np.arange(n), np.diff(sysd["row_ptr"]))
    h = np.zeros((n, n))
    s = np.zeros((n, n))
    h[rows, sysd["col"]] = sysd["h"]
    s[rows, sysd["col"]] = sysd["s"]
    xi = 0.17
    eps, c = dense.eigenstates_near(h, s, xi, 6)
    lhs = np.linalg.solve(h - xi * s, s @ c)
    assert np.allclose(lhs, c / (eps - xi)[None, :], rtol=1e-9, atol=1e-9)
    allev = np.linalg.eigvalsh(np.linalg.solve(np.linalg.cholesky(s), np.linalg.solve(np.linalg.cholesky(s), h).T))
    assert np.max(np.abs(eps - xi)) <= np.sort(np.abs(allev - xi))[5] + 1e-12
