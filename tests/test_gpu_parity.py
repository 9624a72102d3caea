"""Parity of the HIP path (through the C ABI) with the FP64 oracle on small lattices.

Tolerances: FP64 operator <= 1e-12 relative (max-norm); FP32 operator <= 2e-6;
solves at tol 1e-12 agree with the oracle's exact solves to <= 1e-9 relative;
exponents |dx| <= 1e-8 max(|x|, 1) and log W_gl <= 1e-8 max(|log W|, 1).
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1211_1214_amd as dd  # noqa: E402
from oracle import cref, dirac, estimator  # noqa: E402
from oracle.schwarz import Schwarz  # noqa: E402
from paper_1211_1214_amd import inputs  # noqa: E402

pytestmark = pytest.mark.gpu

GEOMS = {
    "4x4^3/2^4": ((4, 4, 4, 4), (2, 2, 2, 2)),          # one tile
    "4x6^3/2x3^3 ragged": ((4, 6, 6, 6), (2, 3, 3, 3)),  # 864 sites: ragged last tile
    "8x4x4x12/2x2x2x3": ((8, 4, 4, 12), (2, 2, 2, 3)),  # 6 tiles, 32 blocks per colour
}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


_cache = {}


def setup(name, dev, seed=1):
    key = (name, seed)
    if key not in _cache:
        lat, blk = GEOMS[name]
        U = inputs.make_links(lat, 0.3, seed)
        ctx = dd.Context(torch.from_numpy(U).to(dev), lat, blk, -1, 1.0)
        _cache[key] = (lat, blk, U, ctx, Schwarz(U, lat, blk, 1.0))
    return _cache[key]


def T(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


@pytest.mark.parametrize("name", list(GEOMS))
def test_dslash_fp64(dev, name):
    lat, blk, U, ctx, S = setup(name, dev)
    say("dslash fp64", name)
    psi = inputs.make_spinor(lat, 11, nrhs=3)
    for kappa in (0.12, 0.1372):
        got = ctx.dslash_apply(kappa, T(psi, dev)).cpu().numpy()
        D = S.D(dirac.mass(kappa))
        want = np.stack([dirac.apply(D, p) for p in psi])
        assert rel(got, want) < 1e-12


@pytest.mark.parametrize("name", list(GEOMS))
def test_dslash_fp32(dev, name):
    lat, blk, U, ctx, S = setup(name, dev)
    say("dslash fp32", name)
    D = S.D(dirac.mass(0.121))
    for nrhs in (1, 2, 5):  # one RHS: RHS-major fields; several: RHS-innermost fields
        psi = inputs.make_spinor(lat, 12, nrhs=nrhs)
        got = ctx.dslash_apply(0.121, T(psi, dev), prec=dd.MIXED32).cpu().numpy()
        want = np.stack([dirac.apply(D, p) for p in psi])
        assert rel(got, want) < 2e-6, nrhs


def test_dslash_periodic_and_wilson(dev):
    lat, blk = (4, 4, 2, 6), (2, 2, 1, 3)
    U = inputs.make_links(lat, 0.3, 4)
    say("dslash periodic / c_sw = 0")
    for tbc, csw in ((1, 1.0), (-1, 0.0), (1, 1.7)):
        ctx = dd.Context(T(U, dev), lat, blk, tbc, csw)
        psi = inputs.make_spinor(lat, 3)
        got = ctx.dslash_apply(0.125, T(psi, dev)).cpu().numpy()
        want = dirac.apply(dirac.dirac(U, lat, dirac.mass(0.125), csw, tbc), psi)
        assert rel(got, want) < 1e-12
        ctx.close()


@pytest.mark.parametrize("tbc,csw", [(1, 1.0), (-1, 0.0), (1, 1.7)])
def test_staged_kernels_boundary_and_clover(dev, tbc, csw):
    """The kernels that stage per-site data in LDS (several-RHS FP32 Dslash, the global solver's
    RHS-innermost operator kernels in the interleaved order, the LDS-resident block solver) with
    periodic time and other clover coefficients, against the oracle."""
    lat, blk = (4, 4, 4, 12), (2, 2, 2, 2)
    U = inputs.make_links(lat, 0.3, 14)
    say("staged kernels tbc", tbc, "csw", csw)
    ctx = dd.Context(T(U, dev), lat, blk, tbc, csw)
    try:
        S = Schwarz(U, lat, blk, csw, tbc)
        psi = inputs.make_spinor(lat, 15, nrhs=9)
        got = ctx.dslash_apply(0.125, T(psi, dev), prec=dd.MIXED32).cpu().numpy()
        D = dirac.dirac(U, lat, dirac.mass(0.125), csw, tbc)
        want = np.stack([dirac.apply(D, p) for p in psi])
        assert rel(got, want) < 2e-6
        m = dirac.mass(0.121)
        inv = S.inv_full(m)
        want = np.stack([inv(p.reshape(-1)).reshape(p.shape) for p in psi])
        for prec in (dd.MIXED32, dd.MIXED16):
            x, st = ctx.solve(0.121, T(psi, dev), tol=1e-12, prec=prec)
            assert rel(x.cpu().numpy(), want) < 1e-9, prec
        b = psi[:2]
        for colour in (0, 1):
            xb, _ = ctx.block_solve(colour, 0.121, T(b, dev), tol=1e-12, prec=dd.MIXED32)
            want = np.stack([S.block_inverse(colour, m, bb) for bb in b])
            assert rel(xb.cpu().numpy(), want) < 1e-9
    finally:
        ctx.close()


@pytest.mark.parametrize("prec", [dd.FP64, dd.MIXED32, dd.MIXED16])
@pytest.mark.parametrize("colour", [0, 1])
@pytest.mark.parametrize("name", list(GEOMS))
def test_block_solve(dev, name, colour, prec):
    lat, blk, U, ctx, S = setup(name, dev)
    say("block solve", name, colour, prec)
    b = inputs.make_spinor(lat, 21, nrhs=2)
    m = dirac.mass(0.121)
    x, st = ctx.block_solve(colour, 0.121, T(b, dev), tol=1e-12, prec=prec)
    x = x.cpu().numpy()
    want = np.stack([S.block_inverse(colour, m, bb) for bb in b])
    assert rel(x, want) < 1e-9
    assert st["rel_residual"] <= 1e-12
    other = lt_colour_mask(lat, blk, 1 - colour)
    assert np.all(x[:, other] == 0)


def lt_colour_mask(lat, blk, c):
    from oracle import lattice as lt
    return lt.colour(lat, blk) == c


@pytest.mark.parametrize("prec", [dd.FP64, dd.MIXED32, dd.MIXED16])
@pytest.mark.parametrize("name", list(GEOMS))
def test_schur_apply_and_inverse(dev, name, prec):
    lat, blk, U, ctx, S = setup(name, dev)
    say("schur", name, prec)
    phi = inputs.make_spinor(lat, 31, nrhs=2)
    m = dirac.mass(0.1205)
    got, _ = ctx.schur_apply(0.1205, T(phi, dev), inverse=False, tol=1e-12, prec=prec)
    want = np.stack([S.hat_apply(m, p) for p in phi])
    assert rel(got.cpu().numpy(), want) < 1e-9
    got, st = ctx.schur_apply(0.1205, T(phi, dev), inverse=True, tol=1e-12, prec=prec)
    want = np.stack([S.hat_inverse(m, p) for p in phi])
    assert rel(got.cpu().numpy(), want) < 1e-9


@pytest.mark.parametrize("prec", [dd.FP64, dd.MIXED32, dd.MIXED16])
@pytest.mark.parametrize("name", list(GEOMS))
def test_solve(dev, name, prec):
    lat, blk, U, ctx, S = setup(name, dev)
    say("solve", name, prec)
    b = inputs.make_spinor(lat, 41, nrhs=3)
    m = dirac.mass(0.121)
    x, st = ctx.solve(0.121, T(b, dev), tol=1e-12, prec=prec)
    want = np.stack([S.inv_full(m)(bb.reshape(-1)).reshape(bb.shape) for bb in b])
    assert rel(x.cpu().numpy(), want) < 1e-9
    assert st["rel_residual"] <= 1e-12
    if prec != dd.FP64:
        assert st["outer_iters"] >= 2


@pytest.mark.parametrize("prec", [dd.FP64, dd.MIXED32, dd.MIXED16])
@pytest.mark.parametrize("op", ["full", "schur"])
def test_det_ratio_c1(dev, op, prec):
    cfg = inputs.WORKLOADS["4x4^3"]
    lat, blk, U, ctx, S = setup("4x4^3/2^4", dev)
    say("det ratio C1", op, prec)
    eta = inputs.make_noise_batch(lat, cfg["seed"], 1, cfg["n_hit"])
    k1, k2 = cfg["kappa1"], cfg["kappa2"]
    res = ctx.det_ratio_estimate(k1, k2, T(eta, dev), op=dd.OP_FULL if op == "full" else dd.OP_SCHUR,
                                 tol=1e-12, prec=prec)
    xo = estimator.exponents(S, dirac.mass(k1), dirac.mass(k2), eta, op, "diff")
    assert np.all(np.abs(res["x"] - xo) <= 1e-8 * np.maximum(np.abs(xo), 1))
    lw = estimator.log_w_gl(xo)
    assert abs(res["log_w_gl"] - lw) <= 1e-8 * max(abs(lw), 1)
    assert np.allclose(res["step_var"], estimator.step_variance(xo), rtol=1e-6)


@pytest.mark.parametrize("prec", [dd.FP64, dd.MIXED32])
@pytest.mark.parametrize("op", ["full", "schur"])
def test_det_ratio_one_flavour(dev, op, prec):
    """n_f = 1 (Eq. 11): complex exponents eta^+ (M - 1) eta and ln Re mean exp(-x)."""
    cfg = inputs.WORKLOADS["4x4^3"]
    lat, blk, U, ctx, S = setup("4x4^3/2^4", dev)
    say("det ratio one flavour C1", op, prec)
    eta = inputs.make_noise_batch(lat, cfg["seed"], 1, cfg["n_hit"])
    k1, k2 = cfg["kappa1"], cfg["kappa2"]
    res = ctx.det_ratio_estimate(k1, k2, T(eta, dev), op=dd.OP_FULL if op == "full" else dd.OP_SCHUR,
                                 tol=1e-12, prec=prec, n_f=1)
    xo = estimator.exponents(S, dirac.mass(k1), dirac.mass(k2), eta, op, "diff", n_f=1)
    assert res["x"].dtype == np.complex128
    assert np.all(np.abs(res["x"] - xo) <= 1e-8 * np.maximum(np.abs(xo), 1))
    lw = estimator.log_w_one_flavour(xo)
    assert np.isfinite(lw)
    assert abs(res["log_w_gl"] - lw) <= 1e-8 * max(abs(lw), 1)
    assert np.allclose(res["step_var"], estimator.step_variance_one_flavour(xo), rtol=1e-6)


def test_det_ratio_one_flavour_interpolation(dev):
    lat, blk, U, ctx, S = setup("8x4x4x12/2x2x2x3", dev)
    say("det ratio one flavour N=4")
    eta = inputs.make_noise_batch(lat, 7, 4, 3)
    res = ctx.det_ratio_estimate(0.1200, 0.1205, T(eta, dev), op=dd.OP_SCHUR, tol=1e-12, prec=dd.MIXED32, n_f=1)
    xo = estimator.exponents(S, dirac.mass(0.12), dirac.mass(0.1205), eta, "schur", "diff", n_f=1)
    assert np.all(np.abs(res["x"] - xo) <= 1e-8 * np.maximum(np.abs(xo), 1))
    lw = estimator.log_w_one_flavour(xo)
    assert abs(res["log_w_gl"] - lw) <= 1e-8 * max(abs(lw), 1)


def test_det_ratio_interpolation(dev):
    lat, blk, U, ctx, S = setup("8x4x4x12/2x2x2x3", dev)
    say("det ratio interpolation N=4")
    eta = inputs.make_noise_batch(lat, 7, 4, 3)
    res = ctx.det_ratio_estimate(0.1200, 0.1205, T(eta, dev), op=dd.OP_SCHUR, tol=1e-12, prec=dd.MIXED32)
    xo = estimator.exponents(S, dirac.mass(0.12), dirac.mass(0.1205), eta, "schur", "diff")
    assert np.all(np.abs(res["x"] - xo) <= 1e-8 * np.maximum(np.abs(xo), 1))
    lw = estimator.log_w_gl(xo)
    assert abs(res["log_w_gl"] - lw) <= 1e-8 * max(abs(lw), 1)


def test_det_ratio_c2(dev):
    """8^4 lattice, 4^4 blocks, N_hit = 16: Schur estimator vs the C oracle on every noise vector,
    full-M estimator on four of them."""
    cfg = inputs.WORKLOADS["8x8^3"]
    lat, blk = cfg["lat"], cfg["blk"]
    say("det ratio C2")
    U = inputs.make_links(lat, cfg["eps"], cfg["seed"])
    ctx = dd.Context(T(U, dev), lat, blk, -1, 1.0)
    R = cref.CRef(U, lat, blk, 1.0)
    k1, k2 = cfg["kappa1"], cfg["kappa2"]
    m1, m2 = dirac.mass(k1), dirac.mass(k2)
    eta = inputs.make_noise_batch(lat, cfg["seed"], 1, cfg["n_hit"])
    for op, nchk in (("schur", 16), ("full", 4)):
        for prec in (dd.FP64, dd.MIXED32):
            res = ctx.det_ratio_estimate(k1, k2, T(eta, dev), op=dd.OP_SCHUR if op == "schur" else dd.OP_FULL,
                                         tol=1e-12, prec=prec)
            for j in range(nchk):
                xo = R.exponent(op, "diff", m1, m2, eta[0, j], 1e-13)
                assert abs(res["x"][0, j] - xo) <= 1e-8 * max(abs(xo), 1), (op, prec, j)
            if nchk == cfg["n_hit"]:
                lw = estimator.log_w_gl(np.array([[R.exponent(op, "diff", m1, m2, eta[0, j], 1e-13)
                                                   for j in range(nchk)]]))
                assert abs(res["log_w_gl"] - lw) <= 1e-8 * max(abs(lw), 1)
    ctx.close()


def test_error_paths(dev):
    lat, blk, U, ctx, S = setup("4x4^3/2^4", dev)
    say("error paths")
    b = inputs.make_spinor(lat, 51)
    with pytest.raises(dd.DDWCError) as e:
        ctx.solve(0.121, T(b, dev), tol=1e-12, maxit=1)
    assert e.value.code == -2
    with pytest.raises(dd.DDWCError) as e:
        ctx.block_solve(0, 0.121, T(b, dev), tol=1e-12, maxit=1)
    assert e.value.code == -2
    bad = b.copy()
    bad[3, 1, 2] = np.nan
    with pytest.raises(dd.DDWCError) as e:
        ctx.solve(0.121, T(bad, dev), tol=1e-12)
    assert e.value.code == -4
    with pytest.raises(ValueError):
        ctx.dslash_apply(0.12, T(b[:-1], dev))
    eta = inputs.make_noise_batch(lat, 1, 1, 2)
    for n_f in (0, 3):
        with pytest.raises(dd.DDWCError) as e:
            ctx.det_ratio_estimate(0.12, 0.121, T(eta, dev), n_f=n_f)
        assert e.value.code == -1
