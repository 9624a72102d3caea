"""Pins of the matrix-free C oracle: against the assembled oracle and against closed forms."""
import numpy as np
import pytest

from oracle import cref, dirac, estimator, lattice as lt
from oracle.schwarz import Schwarz
from paper_1211_1214_amd import inputs


@pytest.fixture(scope="module")
def c1():
    lat, blk = (4, 4, 4, 4), (2, 2, 2, 2)
    U = inputs.make_links(lat, 0.3, 1)
    return lat, blk, U, cref.CRef(U, lat, blk, 1.0), Schwarz(U, lat, blk, 1.0)


def test_c_operator_matches_assembled(c1):
    lat, blk, U, R, S = c1
    m = dirac.mass(0.12)
    psi = inputs.make_spinor(lat, 1)
    assert np.abs(R.clover() - dirac.clover_term(U, lat, 1.0)).max() < 1e-15
    assert np.abs(R.dslash(m, psi) - dirac.apply(S.D(m), psi)).max() < 1e-13
    for c in (0, 1):
        assert np.abs(R.block_apply(c, m, psi) - S.block_apply(c, m, psi)).max() < 1e-13
    assert np.abs(R.hop(1, psi) - S.hop_wb(m, psi)).max() < 1e-14
    assert np.abs(R.hop(0, psi) - S.hop_bw(m, psi)).max() < 1e-14


def test_c_solves_match_assembled(c1):
    lat, blk, U, R, S = c1
    m = dirac.mass(0.121)
    b = inputs.make_spinor(lat, 2)
    assert np.abs(R.solve(m, b) - S.inv_full(m)(b.reshape(-1)).reshape(b.shape)).max() < 1e-11
    for c in (0, 1):
        assert np.abs(R.block_solve(c, m, b) - S.block_inverse(c, m, b)).max() < 1e-11
    phi = S.restrict_P(b)
    assert np.abs(R.schur_apply(m, phi) - S.hat_apply(m, phi)).max() < 1e-11
    assert np.abs(R.schur_inverse(m, phi) - S.hat_inverse(m, phi)).max() < 1e-11


@pytest.mark.parametrize("op", ["full", "schur"])
def test_c_exponents_match_assembled(c1, op):
    lat, blk, U, R, S = c1
    m1, m2 = dirac.mass(0.12), dirac.mass(0.121)
    eta = inputs.make_noise_batch(lat, 1, 1, 2)
    want = estimator.exponents(S, m1, m2, eta, op, "diff")[0]
    for j in range(2):
        for form in ("plain", "diff"):
            got = R.exponent(op, form, m1, m2, eta[0, j], 1e-13)
            assert abs(got - want[j]) < 1e-9 * max(1.0, abs(want[j]))


def test_c_free_field_plane_wave_large():
    """Closed-form free-field action at a lattice the assembled oracle does not reach."""
    lat = (16, 8, 8, 12)
    R = cref.CRef(inputs.unit_links(lat), lat, (4, 4, 4, 6), 1.0, -1)
    m = 0.05
    x = lt.coords(lat)
    n = (3, 5, 1, 7)
    p = np.array([(2 * n[0] + 1) * np.pi / lat[0]] + [2 * np.pi * n[k] / lat[k] for k in (1, 2, 3)])
    u = np.arange(12).reshape(4, 3) + 1j
    ph = np.exp(1j * (x @ p))[:, None, None]
    Dp = (m + np.sum(1 - np.cos(p))) * np.eye(4) + 1j * np.einsum("m,mst->st", np.sin(p), dirac.GAMMA)
    assert np.abs(R.dslash(m, ph * u[None]) - ph * (Dp @ u)[None]).max() < 1e-12


def test_c_gamma5_hermiticity_and_covariance():
    lat, blk = (8, 4, 4, 6), (2, 2, 2, 3)
    U = inputs.make_links(lat, 0.3, 7)
    m = dirac.mass(0.121)
    R = cref.CRef(U, lat, blk, 1.0)
    psi, phi = inputs.make_spinor(lat, 3), inputs.make_spinor(lat, 4)
    g5 = dirac.gamma5_vector
    lhs = np.vdot(phi, g5(R.dslash(m, g5(psi))))
    rhs = np.conj(np.vdot(psi, R.dslash(m, phi)))
    assert abs(lhs - rhs) < 1e-13 * abs(rhs)
    Om = inputs.make_gauge_transform(lat, 3)
    Rg = cref.CRef(dirac.gauge_transform_links(U, lat, Om), lat, blk, 1.0)
    a = Rg.dslash(m, dirac.gauge_transform_spinor(psi, Om))
    b = dirac.gauge_transform_spinor(R.dslash(m, psi), Om)
    assert np.abs(a - b).max() < 1e-13


def test_oracle_iterative_route_matches_direct(c1, monkeypatch):
    """The refined BiCGStab route the oracle takes on larger lattices agrees with sparse LU."""
    from oracle import krylov
    lat, blk, U, R, S = c1
    m = dirac.mass(0.121)
    b = inputs.make_spinor(lat, 5).reshape(-1)
    direct = S.inv_full(m)(b)
    monkeypatch.setattr(krylov, "DIRECT_MAX_DIM", 0)
    it = krylov.Inverse(S.D(m), 1e-14)
    assert it.lu is None
    assert np.abs(it(b) - direct).max() < 1e-12
