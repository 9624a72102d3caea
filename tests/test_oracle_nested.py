"""Pins of the nested-DD oracle (oracle/nested.py) against dense linear algebra.

  * determinant identity per outer colour and mass:
        ln|det A_c| = ln|det Ahat_c (on range P_c)| + sum_s ln|det D_s|,
    with A_c, the inner blocks D_s and their site sets built here from coordinates;
  * the exponents of the operator route (one inversion of A_c, difference form) against
    e^+(Mh^+ Mh - 1)e and e^+(Mh - 1)e with Mh = Ahat(m_next)^-1 Ahat(m_prev) from dense
    matrices;
  * the whole factorisation: ln|det D(m2)/det D(m1)|^2 of the full operator equals the
    outer Schur factor, the two nested Schur factors and the inner block factors, all
    from dense determinants.
"""
import numpy as np
import pytest

from oracle import dirac, estimator, lattice as lt
from oracle.nested import Nested
from oracle.schwarz import Schwarz
from paper_1211_1214_amd import inputs

CASES = {
    "4^4 / 2^4 / 1^4": ((4, 4, 4, 4), (2, 2, 2, 2), (1, 1, 1, 1)),
    "4^4 / 2^4 / 2x1^3": ((4, 4, 4, 4), (2, 2, 2, 2), (2, 1, 1, 1)),
    "8x4^3 / 4x2^3 / 2x1^3": ((8, 4, 4, 4), (4, 2, 2, 2), (2, 1, 1, 1)),
}
K1, K2 = 0.1200, 0.1210


def _sites_of_blocks(lat, blk):
    """{block coordinate tuple: site indices} from coordinates."""
    n = lt.coords(lat) // np.asarray(blk)
    out = {}
    for s, key in enumerate(map(tuple, n)):
        out.setdefault(key, []).append(s)
    return {k: np.array(v) for k, v in out.items()}


def _comp(sites):
    return (12 * np.asarray(sites)[:, None] + np.arange(12)[None, :]).ravel()


def _logabsdet(M):
    return float(np.linalg.slogdet(M)[1])


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("colour", [0, 1])
def test_determinant_identity(name, colour):
    lat, outer, inner = CASES[name]
    U = inputs.make_links(lat, 0.3, 21)
    N = Nested(U, lat, outer, inner, 1.0, colour)
    for kappa in (K1, K2):
        m = dirac.mass(kappa)
        D = dirac.dirac(U, lat, m, 1.0, -1).tocsr()
        # region: sites whose outer block coordinates sum to the colour (mod 2)
        nout = lt.coords(lat) // np.asarray(outer)
        region = np.nonzero(nout.sum(axis=1) % 2 == colour)[0]
        lhs = _logabsdet(D[_comp(region)][:, _comp(region)].toarray())
        inner_sum = 0.0
        for key, sites in _sites_of_blocks(lat, inner).items():
            if np.isin(sites, region).all():
                idx = _comp(sites)
                inner_sum += _logabsdet(D[idx][:, idx].toarray())
        rhs = _logabsdet(N.hat_dense(m)) + inner_sum
        assert abs(lhs - rhs) <= 1e-10 * abs(lhs), (lhs, rhs)


@pytest.mark.parametrize("name", list(CASES))
def test_exponents_against_dense(name):
    lat, outer, inner = CASES[name]
    U = inputs.make_links(lat, 0.3, 22)
    eta = inputs.make_noise_batch(lat, 22, 2, 2)
    m1, m2 = dirac.mass(K1), dirac.mass(K2)
    ms = estimator.interpolation_masses(m1, m2, 2)
    for colour in (0, 1):
        N = Nested(U, lat, outer, inner, 1.0, colour)
        x2 = estimator.exponents(N, m1, m2, eta, "schur", "diff")
        x1 = estimator.exponents(N, m1, m2, eta, "schur", "diff", n_f=1)
        for i in range(2):
            Mh = np.linalg.solve(N.hat_dense(ms[i + 1]), N.hat_dense(ms[i]))
            for j in range(2):
                e = eta[i, j].reshape(-1)[N.P]
                y = Mh @ e
                want2 = float(np.vdot(y, y).real - np.vdot(e, e).real)
                want1 = complex(np.vdot(e, y) - np.vdot(e, e))
                assert abs(x2[i, j] - want2) <= 1e-9 * abs(want2), (colour, i, j)
                assert abs(x1[i, j] - want1) <= 1e-9 * abs(want1), (colour, i, j)


def test_whole_factorisation():
    lat, outer, inner = CASES["4^4 / 2^4 / 2x1^3"]
    U = inputs.make_links(lat, 0.3, 23)
    m1, m2 = dirac.mass(K1), dirac.mass(K2)

    def parts(m):
        full = _logabsdet(dirac.dirac(U, lat, m, 1.0, -1).toarray())
        S = Schwarz(U, lat, outer, 1.0)
        tot = _logabsdet(S.hat_dense(m))
        for c in (0, 1):
            N = Nested(U, lat, outer, inner, 1.0, c)
            tot += _logabsdet(N.hat_dense(m)) + sum(la for _, la in N.inner_block_logdets(m))
        return full, tot

    f1, t1 = parts(m1)
    f2, t2 = parts(m2)
    assert abs(f1 - t1) <= 1e-10 * abs(f1)
    assert abs(2 * (f2 - f1) - 2 * (t2 - t1)) <= 1e-9 * abs(f2 - f1)


def test_matrix_free_route():
    """The matrix-free C route (oracle/c) against the assembled matrices, both colours."""
    from oracle.nested import NestedMatrixFree
    lat, outer, inner = (8, 4, 4, 4), (4, 2, 2, 2), (2, 2, 2, 2)
    U = inputs.make_links(lat, 0.3, 24)
    eta = inputs.make_noise_batch(lat, 24, 1, 2)
    m1, m2 = dirac.mass(K1), dirac.mass(K2)
    for colour in (0, 1):
        want = estimator.exponents(Nested(U, lat, outer, inner, 1.0, colour), m1, m2, eta, "schur", "diff")
        R = NestedMatrixFree(U, lat, outer, inner, 1.0, colour)
        got = estimator.exponents(R, m1, m2, eta, "schur", "diff")
        R.close()
        assert np.abs(got - want).max() <= 1e-10 * np.abs(want).max(), (colour, got, want)
