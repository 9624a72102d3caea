"""Parity at the benchmark's full size: 48x24^3 lattice, 6^4 Schwarz blocks, 12 noise vectors
in one multi-RHS batch, the launch configuration bench.py times.

The oracle cannot redo the whole batch in seconds, so the checks are
  * the operator on every site against the C oracle (FP64 one RHS; FP32 on sampled RHS),
  * solve and block-solve residuals measured with the oracle's operator (a property that
    holds at any size),
  * every exponent x_0j of the 12-RHS batch, log W_gl (Eq. 8) and the step variance against
    the oracle values stored by tests/golden/make_golden_48x24.py (all solves to 1e-13),
    |dx| <= 1e-8 max(|x|, 1) and |d log W| <= 1e-8 max(|log W|, 1).
"""
import json
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1211_1214_amd as dd  # noqa: E402
from oracle import cref, dirac  # noqa: E402
from paper_1211_1214_amd import inputs  # noqa: E402

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_48x24.json")
TOL = 1e-10  # the benchmark's solver tolerance


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lat48():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cfg = inputs.WORKLOADS["48x24^3"]
    say("48x24: generating inputs")
    U = inputs.make_links(cfg["lat"], cfg["eps"], cfg["seed"])
    dev = torch.device("cuda:0")
    ctx = dd.Context(torch.from_numpy(U).to(dev), cfg["lat"], cfg["blk"], -1, cfg["csw"])
    say("48x24: building the C oracle field")
    R = cref.CRef(U, cfg["lat"], cfg["blk"], cfg["csw"], -1)
    yield cfg, U, dev, ctx, R
    ctx.close()
    R.close()


def rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def test_48x24_dslash(lat48):
    cfg, U, dev, ctx, R = lat48
    lat = cfg["lat"]
    say("48x24 dslash fp64")
    psi = inputs.make_spinor(lat, 101)
    m = dirac.mass(cfg["kappa2"])
    got = ctx.dslash_apply(cfg["kappa2"], torch.from_numpy(psi).to(dev)).cpu().numpy()
    assert rel(got, R.dslash(m, psi)) < 1e-12
    say("48x24 dslash fp32, 12 RHS")
    psi = inputs.make_spinor(lat, 102, nrhs=cfg["n_hit"])
    got = ctx.dslash_apply(cfg["kappa2"], torch.from_numpy(psi).to(dev), prec=dd.MIXED32).cpu().numpy()
    for j in (0, 5, 11):
        assert rel(got[j], R.dslash(m, psi[j])) < 2e-6


def test_48x24_solve_residuals(lat48):
    cfg, U, dev, ctx, R = lat48
    lat = cfg["lat"]
    m = dirac.mass(cfg["kappa2"])
    b = inputs.make_noise_batch(lat, cfg["seed"], 1, 2)[0]
    say("48x24 global solve, mixed")
    x, st = ctx.solve(cfg["kappa2"], torch.from_numpy(b).to(dev), tol=TOL, prec=dd.MIXED32)
    x = x.cpu().numpy()
    for j in range(2):
        r = b[j] - R.dslash(m, x[j])
        assert np.linalg.norm(r) <= 1.05 * TOL * np.linalg.norm(b[j])
    say("48x24 block solves, mixed, both colours")
    for colour in (0, 1):
        xb, st = ctx.block_solve(colour, cfg["kappa1"], torch.from_numpy(b).to(dev), tol=TOL, prec=dd.MIXED32)
        xb = xb.cpu().numpy()
        mask = (np.arange(R.V) >= 0)
        bc = R.block_apply(colour, dirac.mass(cfg["kappa1"]), xb[0])
        from oracle import lattice as lt
        sel = lt.colour(lat, cfg["blk"]) == colour
        r = (b[0] - bc)[sel]
        assert np.linalg.norm(r) <= 1.05 * TOL * np.linalg.norm(b[0][sel])
        assert np.all(xb[0][~sel] == 0)
        del mask


@pytest.mark.skipif(not os.path.exists(GOLDEN), reason="golden exponents not generated")
def test_48x24_exponents_against_oracle(lat48):
    cfg, U, dev, ctx, R = lat48
    gold = json.load(open(GOLDEN))
    lat, nhit = cfg["lat"], cfg["n_hit"]
    eta = inputs.make_noise_batch(lat, cfg["seed"], 1, nhit)
    etad = torch.from_numpy(eta).to(dev)
    say("48x24 estimate, mixed, 12 RHS")
    res = ctx.det_ratio_estimate(cfg["kappa1"], cfg["kappa2"], etad, op=dd.OP_SCHUR, tol=TOL, prec=dd.MIXED32)
    assert sorted(map(int, gold["x_schur"])) == list(range(nhit)), "oracle values must cover every noise vector"
    for j, xo in gold["x_schur"].items():
        say(f"48x24: x[0,{j}] = {res['x'][0, int(j)]!r}, oracle {xo!r}")
        assert abs(res["x"][0, int(j)] - xo) <= 1e-8 * max(abs(xo), 1), (j, res["x"][0, int(j)], xo)
    lw = gold["log_w_gl"]
    say(f"48x24: log W_gl = {res['log_w_gl']!r}, oracle {lw!r}")
    assert abs(res["log_w_gl"] - lw) <= 1e-8 * max(abs(lw), 1)
    # the relative variance of the weights e^-x moves by at most ~4 max|dx| relative to first order
    v = gold["step_var"]
    assert abs(res["step_var"][0] - v) <= 4e-8 * max(abs(res["x"]).max(), 1) * v
    say("48x24 estimate, FP64 single RHS")
    r64 = ctx.det_ratio_estimate(cfg["kappa1"], cfg["kappa2"], etad[:, :1].contiguous(), op=dd.OP_SCHUR, tol=TOL,
                                 prec=dd.FP64)
    xo = gold["x_schur"]["0"]
    assert abs(r64["x"][0, 0] - xo) <= 1e-8 * max(abs(xo), 1)
    say("48x24 estimate, full operator, mixed")
    rf = ctx.det_ratio_estimate(cfg["kappa1"], cfg["kappa2"], etad[:, :2].contiguous(), op=dd.OP_FULL, tol=TOL,
                                prec=dd.MIXED32)
    xo = gold["x_full"]["0"]
    assert abs(rf["x"][0, 0] - xo) <= 1e-8 * max(abs(xo), 1)
