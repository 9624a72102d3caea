"""Schedule options through the C ABI: HIP-graph replay of the global solver's iteration
chunks (bit-identical to eager launches, replayed many times with other work in between),
block-solver workgroup sizes, LDS residency caps and poll intervals (each against the oracle or
bit-identical to the default), the SAP-preconditioned
GCR global solver (against the oracle's solve and exponents), the operator workgroup size
(against the oracle), option validation and the autotuner."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1211_1214_amd as dd  # noqa: E402
from oracle import dirac  # noqa: E402
from oracle.schwarz import Schwarz  # noqa: E402
from paper_1211_1214_amd import binding, inputs  # noqa: E402

pytestmark = pytest.mark.gpu
LAT, BLK = (8, 4, 4, 8), (2, 2, 2, 2)   # even-odd everywhere: the graph path


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dev = torch.device("cuda:0")
    U = inputs.make_links(LAT, 0.3, 10)
    ctx = dd.Context(torch.from_numpy(U).to(dev), LAT, BLK, -1, 1.0)
    yield dev, U, ctx, Schwarz(U, LAT, BLK, 1.0)
    ctx.close()


def T(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


@pytest.mark.parametrize("prec", [dd.MIXED32, dd.MIXED16, dd.FP64])
def test_graph_replay_matches_eager(env, prec):
    dev, U, ctx, S = env
    say("graph replay", prec)
    b = T(inputs.make_spinor(LAT, 81, nrhs=3), dev)
    ctx.set_option(binding.OPT_GRAPHS, 0)
    x0, s0 = ctx.solve(0.121, b, tol=1e-12, prec=prec)
    x0 = x0.cpu().numpy()
    ctx.set_option(binding.OPT_GRAPHS, 1)
    psi = T(inputs.make_spinor(LAT, 82), dev)
    for rep in range(4):
        x1, s1 = ctx.solve(0.121, b, tol=1e-12, prec=prec)
        assert np.array_equal(x1.cpu().numpy(), x0), rep
        assert (s1["outer_iters"], s1["inner_iters"]) == (s0["outer_iters"], s0["inner_iters"])
        ctx.dslash_apply(0.125, psi)          # other work between replays
        torch.cuda.synchronize()
    # another mass: a second graph, then the first again
    ctx.solve(0.1205, b, tol=1e-12, prec=prec)
    x2, _ = ctx.solve(0.121, b, tol=1e-12, prec=prec)
    assert np.array_equal(x2.cpu().numpy(), x0)


@pytest.mark.parametrize("threads", [64, 128, 192, 256, 512, 768])
def test_block_threads_option(env, threads):
    dev, U, ctx, S = env
    say("block threads", threads)
    ctx.set_option(binding.OPT_BLOCK_THREADS, threads)
    b = inputs.make_spinor(LAT, 83, nrhs=2)
    for colour in (0, 1):
        for prec in (dd.MIXED32, dd.MIXED16):
            x, st = ctx.block_solve(colour, 0.121, T(b, dev), tol=1e-12, prec=prec)
            want = np.stack([S.block_inverse(colour, dirac.mass(0.121), bb) for bb in b])
            got = x.cpu().numpy()
            assert np.abs(got - want).max() <= 1e-9 * np.abs(want).max()
    ctx.set_option(binding.OPT_BLOCK_THREADS, 0)


@pytest.mark.parametrize("lds", [30, 78])
def test_block_lds_option(env, lds):
    """An LDS reservation only caps residency: the block solution is bit-identical."""
    dev, U, ctx, S = env
    say("block lds", lds)
    b = T(inputs.make_spinor(LAT, 87, nrhs=2), dev)
    for prec in (dd.MIXED32, dd.MIXED16, dd.FP64):
        x0, _ = ctx.block_solve(1, 0.121, b, tol=1e-12, prec=prec)
        ctx.set_option(binding.OPT_BLOCK_LDS, lds)
        assert ctx.get_option(binding.OPT_BLOCK_LDS) == lds
        x1, _ = ctx.block_solve(1, 0.121, b, tol=1e-12, prec=prec)
        ctx.set_option(binding.OPT_BLOCK_LDS, 0)
        assert np.array_equal(x0.cpu().numpy(), x1.cpu().numpy())


@pytest.mark.parametrize("poll", [1, 8])
def test_poll_option(env, poll):
    dev, U, ctx, S = env
    say("poll", poll)
    ctx.set_option(binding.OPT_POLL, poll)
    b = inputs.make_spinor(LAT, 84, nrhs=2)
    x, st = ctx.solve(0.121, T(b, dev), tol=1e-12, prec=dd.MIXED32)
    m = dirac.mass(0.121)
    want = np.stack([S.inv_full(m)(bb.reshape(-1)).reshape(bb.shape) for bb in b])
    assert np.abs(x.cpu().numpy() - want).max() <= 1e-9 * np.abs(want).max()
    ctx.set_option(binding.OPT_POLL, 2)


def test_option_validation(env):
    dev, U, ctx, S = env
    for opt, bad in ((binding.OPT_GRAPHS, 2), (binding.OPT_POLL, 0), (binding.OPT_POLL, 65),
                     (binding.OPT_BLOCK_THREADS, 96), (binding.OPT_BLOCK_THREADS, 832), (binding.OPT_SOLVER, 2),
                     (binding.OPT_BLOCK_LDS, -1), (binding.OPT_BLOCK_LDS, 4096),
                     (binding.OPT_OP_THREADS, 64), (binding.OPT_OP_THREADS, 384), (binding.OPT_TILE_ORDER, 2),
                     (9, 1)):
        with pytest.raises(dd.DDWCError) as e:
            ctx.set_option(opt, bad)
        assert e.value.code == -1
    ctx.set_option(binding.OPT_POLL, 4)
    assert ctx.get_option(binding.OPT_POLL) == 4
    ctx.set_option(binding.OPT_POLL, 2)


OPT_LAT = (4, 4, 4, 12)  # 384 even sites: 9 RHS leave a ragged last tile at 256 and 512 threads


@pytest.mark.parametrize("threads,order", [(128, 0), (512, 0), (256, 1), (512, 1)])
@pytest.mark.parametrize("prec", [dd.MIXED32, dd.MIXED16])
def test_op_threads_option(threads, order, prec):
    """Global solves with the RHS-innermost operator kernels at another workgroup size or in the
    block-interleaved dispatch order, with (9 RHS) and without (3 RHS) the per-site staging,
    against the oracle."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    dev = torch.device("cuda:0")
    U = inputs.make_links(OPT_LAT, 0.3, 12)
    S = Schwarz(U, OPT_LAT, BLK, 1.0)
    ctx = dd.Context(torch.from_numpy(U).to(dev), OPT_LAT, BLK, -1, 1.0)
    try:
        ctx.set_option(binding.OPT_OP_THREADS, threads)
        ctx.set_option(binding.OPT_TILE_ORDER, order)
        assert ctx.get_option(binding.OPT_OP_THREADS) == threads
        assert ctx.get_option(binding.OPT_TILE_ORDER) == order
        m = dirac.mass(0.121)
        inv = S.inv_full(m)
        for nrhs in (3, 9):
            say("op threads", threads, "order", order, "prec", prec, "nrhs", nrhs)
            b = inputs.make_spinor(OPT_LAT, 90 + nrhs, nrhs=nrhs)
            x, st = ctx.solve(0.121, T(b, dev), tol=1e-12, prec=prec)
            want = np.stack([inv(bb.reshape(-1)).reshape(bb.shape) for bb in b])
            assert np.abs(x.cpu().numpy() - want).max() <= 1e-9 * np.abs(want).max()
    finally:
        ctx.close()


def test_autotune(env):
    dev, U, ctx, S = env
    say("autotune")
    r = ctx.autotune(0.121, 4, dd.MIXED32)
    assert r["graphs"] in (0, 1) and r["poll"] in (2, 4, 8) and r["block_threads"] in (0, 128, 256, 512)
    assert r["block_kernel"] in (0, 1) and r["op_threads"] in (128, 256, 512) and r["tile_order"] in (0, 1)
    assert 0 <= r["block_lds"] < 160
    assert r["seconds"] > 0
    b = inputs.make_spinor(LAT, 85, nrhs=4)
    x, st = ctx.solve(0.121, T(b, dev), tol=1e-12, prec=dd.MIXED32)
    m = dirac.mass(0.121)
    want = np.stack([S.inv_full(m)(bb.reshape(-1)).reshape(bb.shape) for bb in b])
    assert np.abs(x.cpu().numpy() - want).max() <= 1e-9 * np.abs(want).max()


LEX_LAT, LEX_BLK = (4, 4, 2, 2), (2, 2, 1, 1)  # odd block extents: the lexicographic block solver


@pytest.mark.parametrize("prec", [dd.FP64, dd.MIXED32, dd.MIXED16])
@pytest.mark.parametrize("geom", ["eo", "lex"])
def test_sap_gcr_solve(env, geom, prec):
    """OPT_SOLVER = 1 (GCR preconditioned by the Schwarz alternating procedure) against the oracle's
    dense solve, several RHS, both block-solver kinds."""
    dev, U, ctx, S = env
    say("sap-gcr solve", geom, prec)
    if geom == "lex":
        Ul = inputs.make_links(LEX_LAT, 0.3, 11)
        c = dd.Context(T(Ul, dev), LEX_LAT, LEX_BLK, -1, 1.0)
        Sx, lat = Schwarz(Ul, LEX_LAT, LEX_BLK, 1.0), LEX_LAT
    else:
        c, Sx, lat = ctx, S, LAT
    c.set_option(binding.OPT_SOLVER, 1)
    assert c.get_option(binding.OPT_SOLVER) == 1
    b = inputs.make_spinor(lat, 86, nrhs=3)
    x, st = c.solve(0.121, T(b, dev), tol=1e-12, prec=prec)
    if geom == "lex" and prec == dd.MIXED16:
        # odd block extents: FP16 storage is documented to run as MIXED32, bit for bit
        x32, st32 = c.solve(0.121, T(b, dev), tol=1e-12, prec=dd.MIXED32)
        assert torch.equal(x, x32) and st["inner_iters"] == st32["inner_iters"]
    c.set_option(binding.OPT_SOLVER, 0)
    m = dirac.mass(0.121)
    want = np.stack([Sx.inv_full(m)(bb.reshape(-1)).reshape(bb.shape) for bb in b])
    assert np.abs(x.cpu().numpy() - want).max() <= 1e-9 * np.abs(want).max()
    assert st["rel_residual"] <= 1e-12 and st["outer_iters"] >= 1
    if c is not ctx:
        c.close()


def test_sap_gcr_estimate(env):
    """The Schur estimator with the SAP-GCR global solver against the oracle's exponents."""
    from oracle import estimator
    dev, U, ctx, S = env
    say("sap-gcr estimate")
    eta = inputs.make_noise_batch(LAT, 12, 2, 3)
    ctx.set_option(binding.OPT_SOLVER, 1)
    r = ctx.det_ratio_estimate(0.1200, 0.1210, T(eta, dev), op=dd.OP_SCHUR, tol=1e-12, prec=dd.MIXED32)
    ctx.set_option(binding.OPT_SOLVER, 0)
    want = estimator.exponents(S, dirac.mass(0.1200), dirac.mass(0.1210), eta, "schur", "diff")
    assert np.abs(r["x"] - want).max() <= 1e-8 * max(np.abs(want).max(), 1.0)
    lw = estimator.log_w_gl(want)
    assert abs(r["log_w_gl"] - lw) <= 1e-8 * max(abs(lw), 1.0)
