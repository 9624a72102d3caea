"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test ties a part of the oracle to something other than itself: a closed
form, an invariant, a textbook special case or brute force on a tiny lattice.
None needs a GPU.
"""
import itertools

import numpy as np
import pytest

from oracle import dirac, estimator, lattice as lt
from oracle.schwarz import Schwarz
from paper_1211_1214_amd import inputs


# --------------------------------------------------------------------------- gamma algebra
def test_gamma_algebra():
    g = dirac.GAMMA
    for a in range(4):
        assert np.allclose(g[a], g[a].conj().T)
        for b in range(4):
            assert np.allclose(g[a] @ g[b] + g[b] @ g[a], 2 * (a == b) * np.eye(4))
    assert np.allclose(dirac.GAMMA5, np.diag([1, 1, -1, -1]))
    for a, b in itertools.product(range(4), repeat=2):
        s = dirac.SIGMA[a, b]
        assert np.allclose(s, s.conj().T)
        assert np.allclose(s @ dirac.GAMMA5, dirac.GAMMA5 @ s)


# --------------------------------------------------------------------------- links
def test_links_are_su3():
    U = inputs.make_links((4, 2, 2, 2), 0.3, 9)
    eye = np.eye(3)
    assert np.abs(U @ U.conj().swapaxes(-1, -2) - eye).max() < 1e-14
    assert np.abs(np.linalg.det(U) - 1).max() < 1e-14
    # eps -> small: U ~ 1 + i eps H with E tr H^2 = 4 (lambda/2 normalisation)
    e = 1e-4
    U = inputs.make_links((8, 8, 8, 8), e, 3)
    H = (U - eye) / (1j * e)
    trh2 = np.einsum("...ij,...ji->...", H, H).real
    assert abs(trh2.mean() - 4.0) < 0.05


# --------------------------------------------------------------------------- free field
def _free_eigs(lat, m, time_bc):
    T = lat[0]
    ps = []
    for mu, L in enumerate(lat):
        n = np.arange(L)
        if mu == 0 and time_bc == -1:
            ps.append((2 * n + 1) * np.pi / T)
        else:
            ps.append(2 * np.pi * n / L)
    out = []
    for p in itertools.product(*ps):
        p = np.array(p)
        a = m + np.sum(1 - np.cos(p))
        s = np.sqrt(np.sum(np.sin(p) ** 2))
        out += [a + 1j * s] * 6 + [a - 1j * s] * 6
    return np.array(out)


def _same_multiset(a, b, tol=1e-9):
    a = np.sort_complex(np.round(a, 9))
    b = np.sort_complex(np.round(b, 9))
    return np.abs(a - b).max() < tol


@pytest.mark.parametrize("time_bc", [-1, 1])
@pytest.mark.parametrize("csw", [0.0, 1.0])
def test_free_field_spectrum(time_bc, csw):
    lat = (4, 4, 2, 2)
    m = dirac.mass(0.1234)
    D = dirac.dirac(inputs.unit_links(lat), lat, m, csw, time_bc).toarray()
    assert _same_multiset(np.linalg.eigvals(D), _free_eigs(lat, m, time_bc))


def test_free_field_plane_wave():
    """D e^{ipx} u = [m + sum(1 - cos p) + i sum gamma_mu sin p_mu] e^{ipx} u."""
    lat = (6, 4, 4, 8)
    m = -0.07
    D = dirac.dirac(inputs.unit_links(lat), lat, m, 1.0, -1)
    x = lt.coords(lat)
    rng = np.random.default_rng(5)
    for n in [(0, 0, 0, 0), (2, 1, 3, 5), (5, 3, 2, 1)]:
        p = np.array([(2 * n[0] + 1) * np.pi / lat[0]] + [2 * np.pi * n[k] / lat[k] for k in (1, 2, 3)])
        u = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
        psi = np.exp(1j * (x @ p))[:, None, None] * u[None]
        Dp = (m + np.sum(1 - np.cos(p))) * np.eye(4) + 1j * np.einsum("m,mst->st", np.sin(p), dirac.GAMMA)
        assert np.abs(dirac.apply(D, psi) - np.exp(1j * (x @ p))[:, None, None] * (Dp @ u)[None]).max() < 1e-13


# --------------------------------------------------------------------------- invariants
def test_gamma5_hermiticity():
    lat = (4, 4, 4, 4)
    U = inputs.make_links(lat, 0.3, 1)
    D = dirac.dirac(U, lat, dirac.mass(0.12), 1.0, -1)
    psi = inputs.make_spinor(lat, 1)
    phi = inputs.make_spinor(lat, 2)
    lhs = np.vdot(phi, dirac.gamma5_vector(dirac.apply(D, dirac.gamma5_vector(psi))))
    rhs = np.conj(np.vdot(psi, dirac.apply(D, phi)))
    assert abs(lhs - rhs) < 1e-13 * abs(rhs)


def test_gauge_covariance():
    lat = (4, 4, 2, 6)
    U = inputs.make_links(lat, 0.3, 2)
    Om = inputs.make_gauge_transform(lat, 1)
    Ug = dirac.gauge_transform_links(U, lat, Om)
    m = dirac.mass(0.12)
    psi = inputs.make_spinor(lat, 3)
    lhs = dirac.apply(dirac.dirac(Ug, lat, m, 1.0), dirac.gauge_transform_spinor(psi, Om))
    rhs = dirac.gauge_transform_spinor(dirac.apply(dirac.dirac(U, lat, m, 1.0), psi), Om)
    assert np.abs(lhs - rhs).max() < 1e-13


def test_clover_properties():
    lat = (4, 4, 4, 4)
    U = inputs.make_links(lat, 0.3, 1)
    C = dirac.clover_term(U, lat, 1.0)
    assert np.abs(C - C.conj().swapaxes(1, 2)).max() < 1e-14
    g5 = np.kron(dirac.GAMMA5, np.eye(3))
    assert np.abs(C @ g5 - g5 @ C).max() < 1e-14
    tr_spin = np.einsum("xsasb->xab", C.reshape(-1, 4, 3, 4, 3))
    assert np.abs(tr_spin).max() < 1e-14
    assert np.abs(C).max() > 0.01


def test_clover_single_link():
    """One non-trivial link U_mu(x0) = diag(e^{it}, e^{-it}, 1): Fhat_{mu nu} is (i/4) sin t diag(1,-1,0)
    at x0+nu and x0+mu+nu, minus that at x0-nu and x0+mu-nu, zero elsewhere (incl. x0, x0+mu)."""
    lat = (5, 4, 3, 6)
    th = 0.7
    x0 = np.array([2, 1, 1, 3])
    G = np.diag([np.exp(1j * th), np.exp(-1j * th), 1])
    want = 0.25j * np.sin(th) * np.diag([1, -1, 0])
    for mu in range(4):
        U = inputs.unit_links(lat)
        U[mu, lt.index(lat, x0)] = G
        for nu in range(4):
            if nu == mu:
                continue
            F = dirac.field_strength(U, lat, mu, nu)
            e_m, e_n = np.eye(4, dtype=int)[mu], np.eye(4, dtype=int)[nu]
            exp = np.zeros_like(F)
            for shift, sgn in ((e_n, 1), (e_m + e_n, 1), (-e_n, -1), (e_m - e_n, -1)):
                exp[lt.index(lat, x0 + shift)] += sgn * want
            assert np.abs(F - exp).max() < 1e-15
            assert np.abs(F + dirac.field_strength(U, lat, nu, mu)).max() < 1e-15


# --------------------------------------------------------------------------- geometry
@pytest.mark.parametrize("lat,blk", [((4, 4, 4, 4), (2, 2, 2, 2)), ((8, 8, 8, 8), (4, 4, 4, 4)),
                                     ((12, 12, 12, 12), (6, 6, 6, 6)), ((16, 16, 16, 16), (8, 8, 8, 8))])
def test_face_counts(lat, blk):
    l = blk[0]
    nblk = lt.volume(lat) // l ** 4
    face = lt.face_black(lat, blk)
    col = lt.colour(lat, blk)
    assert face.sum() == (nblk // 2) * (l ** 4 - max(l - 2, 0) ** 4)
    assert (col == 0).sum() == (col == 1).sum()


def test_projector_support_and_block_structure():
    lat, blk = (6, 6, 6, 12), (3, 3, 3, 3)
    S = Schwarz(inputs.make_links(lat, 0.3, 1), lat, blk, 1.0)
    Dbb, Dbw, Dwb, Dww = S.parts(dirac.mass(0.12))
    # D_wb P = D_wb: no column of D_wb outside range(P) is non-zero
    notP = np.setdiff1d(np.arange(len(S.B)), S.P_in_B)
    assert abs(Dwb[:, notP]).max() == 0
    assert abs(Dwb[:, S.P_in_B]).max() > 0
    # D_bb couples only sites of the same block
    bid = lt.block_id(lat, blk)[S.black_sites]
    r, c = Dbb.nonzero()
    assert np.all(bid[r // 12] == bid[c // 12])


def test_invalid_geometry():
    with pytest.raises(ValueError):
        lt.check_geometry((4, 4, 4, 4), (4, 2, 2, 2))
    with pytest.raises(ValueError):
        lt.check_geometry((6, 4, 4, 4), (2, 2, 2, 2))


# --------------------------------------------------------------------------- Schur identities
def _slogdet(a):
    s, l = np.linalg.slogdet(a)
    return l + np.log(s)  # complex log det (mod 2 pi i)


def _same_logdet(a, b, tol):
    d = a - b
    d = d.real + 1j * (((d.imag + np.pi) % (2 * np.pi)) - np.pi)
    return abs(d) < tol * max(1, abs(a))


@pytest.mark.parametrize("lat,blk", [((4, 4, 4, 4), (2, 2, 2, 2)), ((4, 4, 2, 2), (1, 1, 1, 1))])
def test_schur_determinant_identity(lat, blk):
    """det D = det Dhat_P * det D_ww * det D_bb (Sec. 1)."""
    S = Schwarz(inputs.make_links(lat, 0.3, 1), lat, blk, 1.0)
    m = dirac.mass(0.121)
    Dbb, Dbw, Dwb, Dww = (a.toarray() for a in S.parts(m))
    lhs = _slogdet(S.D(m).toarray())
    rhs = _slogdet(S.hat_dense(m)) + _slogdet(Dbb) + _slogdet(Dww)
    assert _same_logdet(lhs, rhs, 1e-12)


def test_schur_inverse_formula():
    """P Dhat^-1 P = (P Dhat P)^-1 = P - P Dc_bw D_wb P (Sec. 1)."""
    lat, blk = (4, 4, 4, 4), (2, 2, 2, 2)
    S = Schwarz(inputs.make_links(lat, 0.3, 1), lat, blk, 1.0)
    m = dirac.mass(0.121)
    Dinv = np.linalg.inv(S.D(m).toarray())
    Dwb = S.parts(m)[2].toarray()
    P = S.P_in_B
    via_formula = np.eye(len(P)) - (Dinv[np.ix_(S.B, S.W)] @ Dwb)[np.ix_(P, P)]
    via_inverse = np.linalg.inv(S.hat_dense(m))
    assert np.abs(via_formula - via_inverse).max() < 1e-12
    phi = S.restrict_P(inputs.make_spinor(lat, 4))
    got = S.hat_inverse(m, phi).reshape(-1)[S.P]
    assert np.abs(got - via_inverse @ phi.reshape(-1)[S.P]).max() < 1e-12
    got = S.hat_apply(m, phi).reshape(-1)[S.P]
    assert np.abs(got - S.hat_dense(m) @ phi.reshape(-1)[S.P]).max() < 1e-12


def test_even_odd_special_case():
    """Blocks of one site: Dhat is textbook even-odd, Dhat = 1 - A_ee^-1 D_eo A_oo^-1 D_oe,
    det D = det Dhat * prod_x det A(x) with A(x) = 4 + m + C(x)."""
    lat, blk = (4, 2, 2, 4), (1, 1, 1, 1)
    U = inputs.make_links(lat, 0.3, 3)
    S = Schwarz(U, lat, blk, 1.0)
    m = dirac.mass(0.12)
    D = S.D(m).toarray()
    par = lt.coords(lat).sum(axis=1) % 2
    ev = (12 * np.nonzero(par == 0)[0][:, None] + np.arange(12)).ravel()
    od = (12 * np.nonzero(par == 1)[0][:, None] + np.arange(12)).ravel()
    Aee, Deo, Doe, Aoo = D[np.ix_(ev, ev)], D[np.ix_(ev, od)], D[np.ix_(od, ev)], D[np.ix_(od, od)]
    hat = np.eye(len(ev)) - np.linalg.solve(Aee, Deo @ np.linalg.solve(Aoo, Doe))
    assert np.abs(hat - S.hat_dense(m)).max() < 1e-12
    A = (4 + m) * np.eye(12) + dirac.clover_term(U, lat, 1.0)
    rhs = _slogdet(hat) + sum(_slogdet(a) for a in A)
    assert _same_logdet(_slogdet(D), rhs, 1e-12)


# --------------------------------------------------------------------------- Eq. (5), (6)
def test_ratio_matrix_spectrum():
    """lambda(M) = 1 + dm / lambda(D(m2)) (Eq. 6) and det M^-1 = prod lambda/(lambda + dm) (Eq. 5)."""
    lat = (4, 4, 2, 2)
    U = inputs.make_links(lat, 0.3, 4)
    m1, m2 = dirac.mass(0.12), dirac.mass(0.125)
    D1 = dirac.dirac(U, lat, m1, 1.0).toarray()
    D2 = dirac.dirac(U, lat, m2, 1.0).toarray()
    M = np.linalg.solve(D2, D1)
    lam = np.linalg.eigvals(D2)
    assert _same_multiset(np.linalg.eigvals(M), 1 + (m1 - m2) / lam, 1e-8)
    assert _same_logdet(-_slogdet(M), np.sum(np.log(lam / (lam + (m1 - m2)))), 1e-11)


def test_free_field_reweighting_factor():
    """U = 1: W = 1/|det M|^2 = prod_p [(a_p^2 + s_p^2)/((a_p + dm)^2 + s_p^2)]^6 (closed form)."""
    lat, blk = (4, 4, 4, 4), (2, 2, 2, 2)
    m1, m2 = dirac.mass(0.12), dirac.mass(0.121)
    S = Schwarz(inputs.unit_links(lat), lat, blk, 1.0)
    lw = 2 * (np.linalg.slogdet(S.D(m2).toarray())[1] - np.linalg.slogdet(S.D(m1).toarray())[1])
    ps = [(2 * np.arange(4) + 1) * np.pi / 4] + [2 * np.pi * np.arange(4) / 4] * 3
    closed = 0.0
    for p in itertools.product(*ps):
        a = m2 + np.sum(1 - np.cos(p))
        s2 = np.sum(np.sin(np.array(p)) ** 2)
        closed -= 12 * np.log(((a + m1 - m2) ** 2 + s2) / (a * a + s2))
    assert abs(lw - closed) < 1e-10 * abs(closed)
    assert abs(closed + 48.93) < 0.01


# --------------------------------------------------------------------------- estimator
def test_noise_normalisation_scalar_case():
    """E exp(-(mu - 1)|eta|^2) = 1/mu for one complex Gaussian component (Eq. 3 at dimension 1)."""
    eta = inputs.make_noise((50000, 1, 1, 1), 1, 0, 0).reshape(-1)
    for mu in (0.8, 1.3, 2.0):
        est = np.exp(-(mu - 1) * np.abs(eta) ** 2).mean()
        assert abs(est - 1 / mu) < 0.02


@pytest.mark.parametrize("op", ["full", "schur"])
def test_estimator_brute_force(op):
    """Sampling >= 1e5 noise vectors with the dense ratio matrix on a 2^4 lattice: the mean of
    e^-x is 1/det(M^dag M) (Eq. 3) and its variance is Eq. (4), within the sampling error."""
    lat, blk = (2, 2, 2, 2), (1, 1, 1, 1)
    S = Schwarz(inputs.make_links(lat, 0.3, 5), lat, blk, 1.0)
    m1, m2 = dirac.mass(0.1200), dirac.mass(0.1215)
    if op == "full":
        M = np.linalg.solve(S.D(m2).toarray(), S.D(m1).toarray())
    else:
        M = np.linalg.solve(S.hat_dense(m2), S.hat_dense(m1))
    n = M.shape[0]
    MM = M.conj().T @ M
    target = 1 / np.linalg.det(MM).real
    var = 1 / np.linalg.det(2 * MM - np.eye(n)).real - target ** 2
    rng = np.random.default_rng(7)
    N = 200000
    w = np.empty(N)
    for s in range(0, N, 20000):
        eta = (rng.standard_normal((n, 20000)) + 1j * rng.standard_normal((n, 20000))) * np.sqrt(0.5)
        x = np.sum(np.abs(M @ eta) ** 2, axis=0) - np.sum(np.abs(eta) ** 2, axis=0)
        w[s:s + 20000] = np.exp(-x)
    se = np.sqrt(var / N)
    assert abs(w.mean() - target) < 5 * se
    assert abs(w.var() - var) < 0.1 * var


def test_oracle_exponents_match_dense():
    """The oracle's solve-based x (both forms) equals eta^dag (M^dag M - 1) eta with dense M."""
    lat, blk = (4, 4, 4, 4), (2, 2, 2, 2)
    S = Schwarz(inputs.make_links(lat, 0.3, 1), lat, blk, 1.0)
    m1, m2 = dirac.mass(0.12), dirac.mass(0.121)
    eta = inputs.make_noise_batch(lat, 1, 1, 2)
    Mf = np.linalg.solve(S.D(m2).toarray(), S.D(m1).toarray())
    Ms = np.linalg.solve(S.hat_dense(m2), S.hat_dense(m1))
    for j in range(2):
        e = eta[0, j].reshape(-1)
        xf = np.linalg.norm(Mf @ e) ** 2 - np.linalg.norm(e) ** 2
        eP = e[S.P]
        xs = np.linalg.norm(Ms @ eP) ** 2 - np.linalg.norm(eP) ** 2
        for form in ("plain", "diff"):
            assert abs(estimator.x_full_plain(S, m1, m2, eta[0, j]) - xf) < 1e-9 * abs(xf)
            got = estimator.exponents(S, m1, m2, eta[:, j:j + 1], "schur", form)[0, 0]
            assert abs(got - xs) < 1e-9 * abs(xs)
        assert abs(estimator.x_full_diff(S, m1, m2, eta[0, j]) - xf) < 1e-9 * abs(xf)


def test_interpolation_telescopes():
    """prod_i det Mh_i = det Dhat_P(m1) / det Dhat_P(m2), m_i linear in m (Eq. 8)."""
    lat, blk = (4, 4, 4, 4), (2, 2, 2, 2)
    S = Schwarz(inputs.make_links(lat, 0.3, 1), lat, blk, 1.0)
    m1, m2 = dirac.mass(0.12), dirac.mass(0.1205)
    ms = estimator.interpolation_masses(m1, m2, 4)
    assert ms[0] == m1 and abs(ms[-1] - m2) < 1e-15
    assert np.allclose(np.diff(ms), (m2 - m1) / 4)
    tot = sum(_slogdet(np.linalg.solve(S.hat_dense(ms[i + 1]), S.hat_dense(ms[i]))) for i in range(4))
    assert _same_logdet(tot, _slogdet(S.hat_dense(m1)) - _slogdet(S.hat_dense(m2)), 1e-11)


def test_exponents_gauge_invariant():
    """x(U^Om, Om eta) = x(U, eta) per sample: Om is site-local, so blocks and P are preserved."""
    lat, blk = (4, 4, 4, 4), (2, 2, 2, 2)
    U = inputs.make_links(lat, 0.3, 1)
    Om = inputs.make_gauge_transform(lat, 2)
    m1, m2 = dirac.mass(0.12), dirac.mass(0.121)
    eta = inputs.make_noise_batch(lat, 1, 1, 1)
    etag = dirac.gauge_transform_spinor(eta[0, 0], Om)[None, None]
    for op in ("full", "schur"):
        for n_f in (2, 1):
            a = estimator.exponents(Schwarz(U, lat, blk, 1.0), m1, m2, eta, op, n_f=n_f)
            b = estimator.exponents(Schwarz(dirac.gauge_transform_links(U, lat, Om), lat, blk, 1.0), m1, m2, etag,
                                    op, n_f=n_f)
            assert abs(a - b).max() < 1e-10 * abs(a).max()


def test_log_domain_combination():
    x = np.array([[1000.0, 1001.0, 1003.0], [5.0, 5.0, 5.0]])
    want = np.log(np.mean(np.exp(-(x[0] - 1000)))) - 1000 + np.log(np.mean(np.exp(-x[1])))
    assert abs(estimator.log_w_gl(x) - want) < 1e-12
    assert estimator.step_variance(x)[1] == 0
    w = np.exp(-(x[0] - 1000))
    assert abs(estimator.step_variance(x)[0] - w.var(ddof=1) / w.mean() ** 2) < 1e-14


# Pins of the per-step variance (Sec. 2.1 asks for the variance of each factor, with Eq. (4)
# its expectation; Sec. 3 gives Eq. (12) for one flavour).  Each check takes the variance
# function as an argument, so that the tests below can also show that plausible mistakes
# planted in it (population instead of sample variance, the wrong power of the mean) fail.
def _check_variance_by_hand(fn):
    """Values worked out by hand: x = (0, ln 2) gives weights (1, 1/2), sample variance 1/8
    about the mean 3/4, relative 2/9; x = (0, ln 2, ln 4) gives (1, 1/2, 1/4), variance 7/48
    about 7/12, relative 3/7; a constant shift of x changes nothing; one step per row."""
    x = np.array([[0.0, np.log(2.0)], [50.0, 50.0 + np.log(2.0)]])
    ok = np.allclose(fn(x), [2 / 9, 2 / 9], rtol=1e-13, atol=0)
    x3 = np.array([[0.0, np.log(2.0), np.log(4.0)]]) + 1234.5
    return ok and abs(fn(x3)[0] - 3 / 7) < 1e-12


def _dense_ratio_2x4(kappa2):
    lat, blk = (2, 2, 2, 2), (1, 1, 1, 1)
    S = Schwarz(inputs.make_links(lat, 0.3, 5), lat, blk, 1.0)
    m1, m2 = dirac.mass(0.1200), dirac.mass(kappa2)
    return np.linalg.solve(S.hat_dense(m2), S.hat_dense(m1))


def _check_variance_sampled(fn, M, n_hit=8, batches=60000, seed=21):
    """The mean over batches of N_hit noise vectors of fn(x) * mean_j(w)^2, the sample variance
    of the weights w = exp(-x), equals Eq. (4), 1/det(2 M^+M - 1) - 1/det(M^+M)^2, within five
    standard errors (an unbiased sample variance has that expectation for any N_hit)."""
    n = M.shape[0]
    MM = M.conj().T @ M
    target = 1 / np.linalg.det(MM).real
    var = 1 / np.linalg.det(2 * MM - np.eye(n)).real - target ** 2
    rng = np.random.default_rng(seed)
    s2 = np.empty(batches)
    chunk = 5000
    for b in range(0, batches, chunk):
        eta = (rng.standard_normal((n, chunk * n_hit)) + 1j * rng.standard_normal((n, chunk * n_hit))) * np.sqrt(0.5)
        x = (np.sum(np.abs(M @ eta) ** 2, axis=0) - np.sum(np.abs(eta) ** 2, axis=0)).reshape(chunk, n_hit)
        s2[b:b + chunk] = fn(x) * np.exp(-x).mean(axis=1) ** 2
    se = s2.std(ddof=1) / np.sqrt(batches)
    return abs(s2.mean() - var) < 5 * se and se < 0.02 * var


def test_step_variance_by_hand():
    assert _check_variance_by_hand(estimator.step_variance)


def test_step_variance_expectation_is_eq4():
    """Sec. 2.1 / Eq. (4) by sampling 4.8e5 noise vectors (6e4 batches of 8) with the dense Schur
    ratio matrix on a 2^4 lattice."""
    assert _check_variance_sampled(estimator.step_variance, _dense_ratio_2x4(0.1206))


def test_step_variance_pins_catch_planted_mistakes():
    """The two pins above reject a population variance (ddof = 0, biased by (N_hit - 1)/N_hit) and
    a variance divided by the mean instead of its square."""
    def ddof0(x):
        a = -np.asarray(x, dtype=float)
        w = np.exp(a - a.max(axis=1, keepdims=True))
        return w.var(axis=1) / w.mean(axis=1) ** 2

    def over_mean(x):
        a = -np.asarray(x, dtype=float)
        w = np.exp(a - a.max(axis=1, keepdims=True))
        return w.var(axis=1, ddof=1) / w.mean(axis=1)

    M = _dense_ratio_2x4(0.1206)
    assert not (_check_variance_by_hand(ddof0) and _check_variance_sampled(ddof0, M))
    assert not (_check_variance_by_hand(over_mean) and _check_variance_sampled(over_mean, M))
    # the sampling pin alone also sees the ddof mistake
    assert not _check_variance_sampled(ddof0, M)


def _check_one_flavour_variance_by_hand(fn):
    """x = (0, ln 2 + i pi): real weights (1, -1/2), mean 1/4, sample variance 9/8, relative 18;
    x = (i pi/3, 0): weights (1/2, 1), relative 2/9."""
    x = np.array([[0.0, np.log(2.0) + 1j * np.pi], [1j * np.pi / 3, 0.0]])
    return np.allclose(fn(x), [18.0, 2 / 9], rtol=1e-12, atol=0)


def _check_one_flavour_variance_sampled(fn, M, n_hit=8, batches=60000, seed=23):
    """With w = exp(-eta^+ (M - 1) eta), Eq. (12) gives E|w|^2 = 1/det(M^+ + M - 1), and the same
    Gaussian integral gives E w^2 = 1/det(2M - 1), so the real weights Re w have the variance
    (1/2)[1/det(M^+ + M - 1) + Re 1/det(2M - 1)] - (1/det M)^2.  The mean over batches of
    fn(x) * mean_j(Re w)^2 must equal it within five standard errors."""
    n = M.shape[0]
    I = np.eye(n)
    e_abs2 = 1 / np.linalg.det(M.conj().T + M - I).real
    e_sq = 1 / np.linalg.det(2 * M - I)
    mean = 1 / np.linalg.det(M).real
    var = 0.5 * (e_abs2 + e_sq.real) - mean ** 2
    A = M - I
    rng = np.random.default_rng(seed)
    s2 = np.empty(batches)
    chunk = 5000
    for b in range(0, batches, chunk):
        eta = (rng.standard_normal((n, chunk * n_hit)) + 1j * rng.standard_normal((n, chunk * n_hit))) * np.sqrt(0.5)
        x = np.sum(eta.conj() * (A @ eta), axis=0).reshape(chunk, n_hit)
        s2[b:b + chunk] = fn(x) * np.exp(-x).real.mean(axis=1) ** 2
    se = s2.std(ddof=1) / np.sqrt(batches)
    return abs(s2.mean() - var) < 5 * se and se < 0.02 * var


def test_step_variance_one_flavour_by_hand():
    assert _check_one_flavour_variance_by_hand(estimator.step_variance_one_flavour)


def test_step_variance_one_flavour_expectation():
    """Sec. 3 / Eq. (12) by sampling 4.8e5 noise vectors with the dense Schur ratio matrix."""
    M = _dense_ratio_2x4(0.1206)
    assert np.linalg.eigvalsh(M.conj().T + M).min() > 1  # Eq. (12) exists
    assert _check_one_flavour_variance_sampled(estimator.step_variance_one_flavour, M)


def test_step_variance_one_flavour_pins_catch_planted_mistakes():
    def ddof0(x):
        _, w = estimator._one_flavour_weights(x)
        return w.var(axis=1) / w.mean(axis=1) ** 2

    def abs_weights(x):  # |w| instead of Re w
        x = np.asarray(x, dtype=complex)
        w = np.exp(-x.real + x.real.min(axis=1, keepdims=True))
        return w.var(axis=1, ddof=1) / w.mean(axis=1) ** 2

    M = _dense_ratio_2x4(0.1206)
    assert not _check_one_flavour_variance_sampled(ddof0, M)
    assert not _check_one_flavour_variance_by_hand(abs_weights)


# --------------------------------------------------------------------------- one flavour (Eq. 11, 12)
def test_one_flavour_plane_wave_closed_form():
    """U = 1: a plane wave e^{ipx} u c with u an eigenvector of sum gamma_mu sin p_mu (eigenvalue
    sigma = +-s_p) is an eigenvector of D(m) with eigenvalue a_p + i sigma, so
    x = eta^dag (M - 1) eta = dm ||eta||^2 / (a_p(m2) + i sigma) in both forms."""
    lat, blk = (4, 4, 4, 4), (2, 2, 2, 2)
    S = Schwarz(inputs.unit_links(lat), lat, blk, 1.0)
    m1, m2 = dirac.mass(0.12), dirac.mass(0.121)
    x = lt.coords(lat)
    rng = np.random.default_rng(3)
    for n in [(0, 0, 0, 0), (1, 1, 0, 3), (3, 2, 1, 1)]:
        p = np.array([(2 * n[0] + 1) * np.pi / lat[0]] + [2 * np.pi * n[k] / lat[k] for k in (1, 2, 3)])
        G = np.einsum("m,mst->st", np.sin(p), dirac.GAMMA)
        sig, vecs = np.linalg.eigh(G)
        a = m2 + np.sum(1 - np.cos(p))
        for k in (0, 3):
            c = rng.standard_normal(3) + 1j * rng.standard_normal(3)
            eta = np.exp(1j * (x @ p))[:, None, None] * np.outer(vecs[:, k], c)[None]
            want = (m1 - m2) * np.sum(np.abs(eta) ** 2) / (a + 1j * sig[k])
            for form in ("plain", "diff"):
                got = estimator.exponents(S, m1, m2, eta[None, None], "full", form, n_f=1)[0, 0]
                assert abs(got - want) < 1e-10 * abs(want), (n, k, form)


@pytest.mark.parametrize("op", ["full", "schur"])
def test_one_flavour_brute_force(op):
    """Sampling 2e5 noise vectors with the dense ratio matrix on a 2^4 lattice: the mean of
    exp(-eta^dag (M - 1) eta) is 1/det M (Eq. 11, real by gamma_5-hermiticity) and the
    variance E|w|^2 - |E w|^2 is 1/det(M^dag + M - 1) - 1/|det M|^2 (Eq. 12)."""
    lat, blk = (2, 2, 2, 2), (1, 1, 1, 1)
    S = Schwarz(inputs.make_links(lat, 0.3, 5), lat, blk, 1.0)
    m1, m2 = dirac.mass(0.1200), dirac.mass(0.1215)
    if op == "full":
        M = np.linalg.solve(S.D(m2).toarray(), S.D(m1).toarray())
    else:
        M = np.linalg.solve(S.hat_dense(m2), S.hat_dense(m1))
    n = M.shape[0]
    A = M - np.eye(n)
    H = M.conj().T + M
    assert np.linalg.eigvalsh(H).min() > 1  # the variance exists
    detM = np.linalg.det(M)
    assert abs(detM.imag) < 1e-10 * abs(detM)
    target = 1 / detM.real
    var = 1 / np.linalg.det(H - np.eye(n)).real - target ** 2
    rng = np.random.default_rng(11)
    N, chunk = 200000, 20000
    w = np.empty(N, dtype=complex)
    for s in range(0, N, chunk):
        eta = (rng.standard_normal((n, chunk)) + 1j * rng.standard_normal((n, chunk))) * np.sqrt(0.5)
        w[s:s + chunk] = np.exp(-np.sum(eta.conj() * (A @ eta), axis=0))
    se = np.sqrt(var / N)
    assert abs(w.mean().real - target) < 5 * se
    assert abs(w.mean().imag) < 5 * se
    assert abs(np.mean(np.abs(w - w.mean()) ** 2) - var) < 0.1 * var


def test_one_flavour_exponents_match_dense():
    """The oracle's solve-based one-flavour x (both forms) equals eta^dag (M - 1) eta with dense M."""
    lat, blk = (4, 4, 4, 4), (2, 2, 2, 2)
    S = Schwarz(inputs.make_links(lat, 0.3, 1), lat, blk, 1.0)
    m1, m2 = dirac.mass(0.12), dirac.mass(0.121)
    eta = inputs.make_noise_batch(lat, 1, 1, 2)
    Mf = np.linalg.solve(S.D(m2).toarray(), S.D(m1).toarray())
    Ms = np.linalg.solve(S.hat_dense(m2), S.hat_dense(m1))
    for j in range(2):
        e = eta[0, j].reshape(-1)
        xf = np.vdot(e, Mf @ e) - np.vdot(e, e)
        eP = e[S.P]
        xs = np.vdot(eP, Ms @ eP) - np.vdot(eP, eP)
        for form in ("plain", "diff"):
            got = estimator.exponents(S, m1, m2, eta[:, j:j + 1], "full", form, n_f=1)[0, 0]
            assert abs(got - xf) < 1e-9 * abs(xf)
            got = estimator.exponents(S, m1, m2, eta[:, j:j + 1], "schur", form, n_f=1)[0, 0]
            assert abs(got - xs) < 1e-9 * abs(xs)


def test_one_flavour_log_domain_combination():
    """ln Re mean_j exp(-x_j) per step, summed; nan when a step's real mean is not positive."""
    x = np.array([[700.0 + 0.3j, 701.0 - 1.2j, 702.5 + 2.0j], [3.0 + 0.1j, 2.0 - 0.4j, 4.0 + 0.0j]])
    want = (np.log(np.mean(np.exp(-(x[0] - 700))).real) - 700
            + np.log(np.mean(np.exp(-x[1])).real))
    assert abs(estimator.log_w_one_flavour(x) - want) < 1e-12 * abs(want)
    w0 = np.exp(-(x[0] - 700)).real
    assert abs(estimator.step_variance_one_flavour(x)[0] - w0.var(ddof=1) / w0.mean() ** 2) < 1e-13
    neg = np.array([[1.0 + np.pi * 1j, 1.5 + 0.9 * np.pi * 1j]])
    assert np.isnan(estimator.log_w_one_flavour(neg))


# --------------------------------------------------------------------------- block determinants (Eq. 7)
def test_block_logdets_compose_the_colour_blocks():
    """D_bb and D_ww are the direct sums of the Dirichlet blocks: their log-determinants add up."""
    lat, blk = (4, 4, 4, 4), (2, 2, 2, 2)
    S = Schwarz(inputs.make_links(lat, 0.3, 2), lat, blk, 1.0)
    m = dirac.mass(0.121)
    Dbb, _, _, Dww = (a.toarray() for a in S.parts(m))
    for c, Dc in ((0, Dbb), (1, Dww)):
        ld = S.block_logdets(c, m)
        assert len(ld) == 8
        total = sum(l for _, l in ld) + np.log(np.prod([s for s, _ in ld]) + 0j)
        assert _same_logdet(total, _slogdet(Dc), 1e-12)


def test_block_logdets_single_site_blocks():
    """1^4 blocks: D_k = (4 + m) + C(x), Hermitian positive definite; ln det = sum ln eigenvalues."""
    lat, blk = (4, 4, 2, 2), (1, 1, 1, 1)
    U = inputs.make_links(lat, 0.3, 3)
    S = Schwarz(U, lat, blk, 1.0)
    m = dirac.mass(0.121)
    C = dirac.clover_term(U, lat, 1.0)
    col = lt.colour(lat, blk)
    for c in (0, 1):
        ld = S.block_logdets(c, m)
        want = [np.sum(np.log(np.linalg.eigvalsh((4 + m) * np.eye(12) + C[x]))) for x in np.nonzero(col == c)[0]]
        assert all(s == 1.0 for s, _ in ld)
        assert np.allclose([l for _, l in ld], want, rtol=0, atol=1e-12)


def test_full_reweighting_factor_factorises():
    """2 [ln|det D(m2)| - ln|det D(m1)|] = 2 [ln|det Dhat_P(m2)| - ln|det Dhat_P(m1)|] + block part."""
    lat, blk = (4, 4, 4, 4), (2, 2, 2, 2)
    S = Schwarz(inputs.make_links(lat, 0.3, 2), lat, blk, 1.0)
    m1, m2 = dirac.mass(0.12), dirac.mass(0.121)
    lhs = 2 * (_slogdet(S.D(m2).toarray()).real - _slogdet(S.D(m1).toarray()).real)
    rhs = 2 * (_slogdet(S.hat_dense(m2)).real - _slogdet(S.hat_dense(m1)).real) + S.log_w_blocks(m1, m2)
    assert abs(lhs - rhs) < 1e-10 * abs(lhs)
