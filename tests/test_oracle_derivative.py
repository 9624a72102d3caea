"""Pins of the derivative oracle (central differences of the oracle's exponents).

The derivatives are checked against closed forms that do not use the lattice code:
the free field, where a plane wave with an eigen-spinor of sum gamma_mu sin p_mu is an
eigenvector of D, and a constant abelian background U_mu(x) = exp(i theta_mu), on which
D acts on a plane wave e^{ipx} u c as the 4x4 spin matrix D(p + theta) on u (the clover
term vanishes: every plaquette is 1).
"""
import numpy as np

from oracle import derivative, dirac, lattice as lt
from paper_1211_1214_amd import inputs

LAT, BLK = (4, 4, 2, 2), (2, 2, 1, 1)


def _dspin(q, m):
    """4x4 spin matrix of D on a plane wave of momentum q (mass normalisation)."""
    return (m + np.sum(1 - np.cos(q))) * np.eye(4) + 1j * np.einsum("m,mst->st", np.sin(q), dirac.GAMMA)


def test_richardson_is_fourth_order():
    f = lambda h: np.array([np.exp(0.3 + 2 * h), np.sin(1 + h) ** 3])
    want = np.array([2 * np.exp(0.3), 3 * np.sin(1) ** 2 * np.cos(1)])
    assert np.abs(derivative.richardson(f, 1e-3) - want).max() < 1e-11


def test_dkappa2_free_field_closed_form():
    """U = 1, eta = e^{ipx} u c with u an eigenvector of sum gamma sin p (eigenvalue sigma):
    x = (|l1|^2 / |l2|^2 - 1) ||eta||^2, l_k = a_p(m_k) + i sigma, a_p(m) = m + sum(1 - cos p), so
    dx/dkappa2 = -2 a_p(m2) |l1|^2 / |l2|^4 ||eta||^2 * dm2/dkappa2, dm2/dkappa2 = -1/(2 kappa2^2)."""
    k1, k2 = 0.12, 0.121
    m1, m2 = dirac.mass(k1), dirac.mass(k2)
    U = inputs.unit_links(LAT)
    x = lt.coords(LAT)
    rng = np.random.default_rng(4)
    etas, want = [], []
    for n in [(0, 0, 0, 0), (1, 2, 0, 1)]:
        p = np.array([(2 * n[0] + 1) * np.pi / LAT[0]] + [2 * np.pi * n[k] / LAT[k] for k in (1, 2, 3)])
        sig, vec = np.linalg.eigh(np.einsum("m,mst->st", np.sin(p), dirac.GAMMA))
        c = rng.standard_normal(3) + 1j * rng.standard_normal(3)
        eta = np.exp(1j * (x @ p))[:, None, None] * np.outer(vec[:, 0], c)[None]
        a = lambda m: m + np.sum(1 - np.cos(p))
        l1, l2 = abs(a(m1) + 1j * sig[0]) ** 2, abs(a(m2) + 1j * sig[0]) ** 2
        nrm = np.sum(np.abs(eta) ** 2)
        want.append(-2 * a(m2) * l1 / l2 ** 2 * nrm * (-1 / (2 * k2 ** 2)))
        etas.append(eta)
    got = derivative.dx_dkappa2(U, LAT, BLK, 1.0, k1, k2, np.array(etas)[None], op="full")[0]
    assert np.abs(got - np.array(want)).max() < 1e-7 * np.abs(want).max()


def test_dlinks_abelian_background_closed_form():
    """U_mu(x) = e^{i theta_mu}: x(theta) = V ||c||^2 (||D2(q)^-1 D1(q) u||^2 - ||u||^2), q = p + theta.
    The derivative along dU_mu(x) = i U_mu(x) (all x, one mu) is d x / d theta_mu."""
    k1, k2 = 0.12, 0.1212
    m1, m2 = dirac.mass(k1), dirac.mass(k2)
    theta = np.array([0.11, -0.23, 0.31, 0.07])
    V = lt.volume(LAT)
    U = np.zeros((4, V, 3, 3), dtype=complex)
    for mu in range(4):
        U[mu] = np.exp(1j * theta[mu]) * np.eye(3)
    x = lt.coords(LAT)
    n = (1, 0, 1, 1)
    p = np.array([(2 * n[0] + 1) * np.pi / LAT[0]] + [2 * np.pi * n[k] / LAT[k] for k in (1, 2, 3)])
    rng = np.random.default_rng(9)
    u = rng.standard_normal(4) + 1j * rng.standard_normal(4)
    c = rng.standard_normal(3) + 1j * rng.standard_normal(3)
    eta = (np.exp(1j * (x @ p))[:, None, None] * np.outer(u, c)[None])[None, None]

    def closed(th):
        q = p + th
        y = np.linalg.solve(_dspin(q, m2), _dspin(q, m1) @ u)
        return V * np.sum(np.abs(c) ** 2) * (np.sum(np.abs(y) ** 2) - np.sum(np.abs(u) ** 2))

    x0 = derivative.exponents_at(U, LAT, BLK, 1.0, k1, k2, eta, op="full")[0, 0]
    assert abs(x0 - closed(theta)) < 1e-10 * abs(x0)
    for mu in range(4):
        dU = np.zeros_like(U)
        dU[mu] = 1j * U[mu]
        got = derivative.dx_dlinks(U, dU, LAT, BLK, 1.0, k1, k2, eta, op="full")[0, 0]
        e = np.eye(4)[mu]
        want = derivative.richardson(lambda h: closed(theta + h * e), 1e-3)
        assert abs(got - want) < 1e-7 * abs(want), (mu, got, want)


def test_log_w_weights():
    x = np.array([[3.0, 1.0, 2.0], [0.5, 0.5, 0.7]])
    g = derivative.log_w_weights(x)
    from oracle import estimator
    for i in range(2):
        for j in range(3):
            e = np.zeros_like(x)
            e[i, j] = 1
            fd = derivative.richardson(lambda h: estimator.log_w_gl(x + h * e), 1e-4)
            assert abs(g[i, j] - fd) < 1e-10
