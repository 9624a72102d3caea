"""Schedule options through the C ABI: HIP-graph replay of the global solver's iteration
chunks (bit-identical to eager launches, replayed many times with other work in between),
block-solver workgroup sizes and poll intervals (each against the oracle), option
validation and the autotuner."""
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


@pytest.mark.parametrize("threads", [64, 128, 192, 256])
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
                     (binding.OPT_BLOCK_THREADS, 96), (binding.OPT_BLOCK_THREADS, 512), (7, 1)):
        with pytest.raises(dd.DDWCError) as e:
            ctx.set_option(opt, bad)
        assert e.value.code == -1
    ctx.set_option(binding.OPT_POLL, 4)
    assert ctx.get_option(binding.OPT_POLL) == 4
    ctx.set_option(binding.OPT_POLL, 2)


def test_autotune(env):
    dev, U, ctx, S = env
    say("autotune")
    r = ctx.autotune(0.121, 4, dd.MIXED32)
    assert r["graphs"] in (0, 1) and r["poll"] in (2, 4, 8) and r["block_threads"] in (0, 128, 192, 256)
    assert r["seconds"] > 0
    b = inputs.make_spinor(LAT, 85, nrhs=4)
    x, st = ctx.solve(0.121, T(b, dev), tol=1e-12, prec=dd.MIXED32)
    m = dirac.mass(0.121)
    want = np.stack([S.inv_full(m)(bb.reshape(-1)).reshape(bb.shape) for bb in b])
    assert np.abs(x.cpu().numpy() - want).max() <= 1e-9 * np.abs(want).max()
