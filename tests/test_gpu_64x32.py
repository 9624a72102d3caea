"""The 64x32^3 workload: 8^4 Schwarz blocks (4096 sites, more than one workgroup sweep per
block), N = 4 mass-interpolation steps and 24 RHS in one multi-RHS batch, mixed precision.

The oracle cannot redo the batch in seconds, so the checks are
  * sampled exponents x_ij against the oracle values stored by tests/golden/make_golden_64x32.py,
  * the FP64 single-RHS path on noise vector 0 (all four steps) against the mixed batch,
  * the FP16-storage inner solver (DDWC_MIXED16) against the oracle values and the FP32 batch,
  * the final residuals of the solver statistics;
  * nested DD (8^4 outer, 4^4 inner blocks) against the stored oracle exponents.
"""
import json
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1211_1214_amd as dd  # noqa: E402
from paper_1211_1214_amd import inputs  # noqa: E402

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_64x32.json")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_64x32_estimate():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cfg = inputs.WORKLOADS["64x32^3"]
    lat, blk = cfg["lat"], cfg["blk"]
    say("64x32: generating inputs")
    U = inputs.make_links(lat, cfg["eps"], cfg["seed"])
    eta = inputs.make_noise_batch(lat, cfg["seed"], cfg["n_interp"], cfg["n_hit"])
    dev = torch.device("cuda:0")
    ctx = dd.Context(torch.from_numpy(U).to(dev), lat, blk, -1, cfg["csw"])
    etad = torch.from_numpy(eta).to(dev)
    del eta
    say("64x32: mixed estimate, 4 steps x 24 RHS")
    res = ctx.det_ratio_estimate(cfg["kappa1"], cfg["kappa2"], etad, op=dd.OP_SCHUR, tol=1e-10, prec=dd.MIXED32)
    x = res["x"]
    assert x.shape == (4, 24) and np.all(np.isfinite(x))
    assert res["stats"]["rel_residual"] <= 1e-10
    assert np.isfinite(res["log_w_gl"])
    gold = json.load(open(GOLDEN))
    for key, xo in gold["x_schur"].items():
        i, j = map(int, key.split(","))
        say(f"64x32: x[{i},{j}] = {x[i, j]!r}, oracle {xo!r}")
        assert abs(x[i, j] - xo) <= 1e-8 * max(abs(xo), 1.0)
    say("64x32: FP16 inner solves, 4 steps x 24 RHS")
    r16 = ctx.det_ratio_estimate(cfg["kappa1"], cfg["kappa2"], etad, op=dd.OP_SCHUR, tol=1e-10, prec=dd.MIXED16)
    assert r16["stats"]["rel_residual"] <= 1e-10
    for key, xo in gold["x_schur"].items():
        i, j = map(int, key.split(","))
        assert abs(r16["x"][i, j] - xo) <= 1e-8 * max(abs(xo), 1.0)
    assert np.all(np.abs(r16["x"] - x) <= 1e-8 * np.maximum(np.abs(x), 1.0))
    say("64x32: FP64 single-RHS path on noise vector 0")
    r64 = ctx.det_ratio_estimate(cfg["kappa1"], cfg["kappa2"], etad[:, :1].contiguous(), op=dd.OP_SCHUR, tol=1e-10,
                                 prec=dd.FP64)
    assert np.all(np.abs(r64["x"][:, 0] - x[:, 0]) <= 1e-8 * np.maximum(np.abs(x[:, 0]), 1.0))
    ctx.close()


GOLDEN_NESTED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_nested_64x32.json")


@pytest.mark.timeout(400)
def test_64x32_nested():
    """Nested DD on the 64x32^3 workload (Sec. 2.2): the 8^4 blocks split into 4^4 blocks.  The
    first of the N = 4 interpolation steps (m_0 -> m_1) with 24 RHS per outer colour, FP16
    storage and FP32 inner solves, against the oracle values stored by
    tests/golden/make_golden_nested_64x32.py, and the two precisions against each other."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cfg = inputs.WORKLOADS["64x32^3"]
    lat, blk = cfg["lat"], cfg["blk"]
    m1 = 1 / (2 * cfg["kappa1"]) - 4
    m2 = 1 / (2 * cfg["kappa2"]) - 4
    k_step = 1 / (2 * (m1 + (m2 - m1) / cfg["n_interp"] + 4))   # kappa of m_1
    gold = json.load(open(GOLDEN_NESTED))
    say("64x32 nested: inputs and contexts (8^4 outer, 4^4 inner)")
    U = inputs.make_links(lat, cfg["eps"], cfg["seed"])
    dev = torch.device("cuda:0")
    Ud = torch.from_numpy(U).to(dev)
    del U
    O = dd.Context(Ud, lat, blk, -1, cfg["csw"])
    I = dd.Context(Ud, lat, tuple(gold["inner_blocks"]), -1, cfg["csw"])
    del Ud
    for c in (0, 1):
        eta = torch.from_numpy(inputs.make_noise_batch(lat, 40 + c, 1, cfg["n_hit"])).to(dev)
        say(f"64x32 nested: colour {c}, FP16 storage")
        r16 = O.det_ratio_nested(I, c, cfg["kappa1"], k_step, eta, tol=1e-10, prec=dd.MIXED16)
        say(f"64x32 nested: colour {c}, FP32")
        r32 = O.det_ratio_nested(I, c, cfg["kappa1"], k_step, eta, tol=1e-10, prec=dd.MIXED32)
        del eta
        for r in (r16, r32):
            assert r["x"].shape == (1, cfg["n_hit"]) and np.isfinite(r["log_w"])
            assert r["stats"]["rel_residual"] <= 1e-10
        for key, xo in gold["x_nested"].items():
            cc, i, j = map(int, key.split(","))
            if cc != c:
                continue
            say(f"64x32 nested: x[{c}][{i},{j}] = {r16['x'][i, j]!r} (FP16), {r32['x'][i, j]!r} (FP32), oracle {xo!r}")
            assert abs(r16["x"][i, j] - xo) <= 1e-8 * max(abs(xo), 1.0)
            assert abs(r32["x"][i, j] - xo) <= 1e-8 * max(abs(xo), 1.0)
        assert np.all(np.abs(r16["x"] - r32["x"]) <= 1e-8 * np.maximum(np.abs(r32["x"]), 1.0))
    O.close()
    I.close()


@pytest.mark.timeout(600)
def test_64x32_dslash_largest_rhs_batches():
    """FP32 Dslash at 64x32^3 (V = 2^21) with 128 RHS (the largest RHS-innermost batch whose
    component planes stay within 32-bit byte offsets) and 129 RHS (RHS-major fields).  RHS r is
    (1 + r) times base spinor r mod 3, so a wrong plane or RHS offset changes the scale; RHS 0, 1,
    2, 64, the last two and the last are checked on every site against the C oracle's operator."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle import cref, dirac
    cfg = inputs.WORKLOADS["64x32^3"]
    lat, blk = cfg["lat"], cfg["blk"]
    say("64x32 dslash: inputs")
    U = inputs.make_links(lat, cfg["eps"], cfg["seed"])
    dev = torch.device("cuda:0")
    ctx = dd.Context(torch.from_numpy(U).to(dev), lat, blk, -1, cfg["csw"])
    R = cref.CRef(U, lat, blk, cfg["csw"], -1)
    del U
    m = dirac.mass(cfg["kappa2"])
    base = [inputs.make_spinor(lat, 140 + k) for k in range(3)]
    want = [R.dslash(m, b) for b in base]
    R.close()
    based = [torch.from_numpy(b).to(dev) for b in base]
    V = based[0].shape[0]
    for nrhs in (128, 129):
        say(f"64x32 dslash: {nrhs} RHS")
        inp = torch.empty((nrhs, V, 4, 3), dtype=torch.complex128, device=dev)
        for r in range(nrhs):
            inp[r] = based[r % 3] * (1.0 + r)
        out = ctx.dslash_apply(cfg["kappa2"], inp, prec=dd.MIXED32)
        del inp
        for r in (0, 1, 2, 64, nrhs - 2, nrhs - 1):
            got = out[r].cpu().numpy() / (1.0 + r)
            w = want[r % 3]
            err = float(np.abs(got - w).max() / np.abs(w).max())
            say(f"64x32 dslash: {nrhs} RHS, rhs {r}: rel err {err:.2e}")
            assert err <= 2e-6
        del out
        torch.cuda.empty_cache()
    ctx.close()
