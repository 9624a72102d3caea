"""Seeded synthetic inputs: gauge links, complex Gaussian noise, random spinors.

These stand in for the paper's CLS ensembles (Sec. 2), which are not available.
The module holds none of the Dirac-operator, Schwarz or estimator arithmetic;
it only draws random numbers and shapes them.  Tests, the benchmark and the
smoke check all take their inputs from here and hand the same arrays to the
HIP path and to the CPU oracle.

Conventions (canonical layout, FP64 complex, interleaved re/im):
  site index   x = ((x0*L1 + x1)*L2 + x2)*L3 + x3, x0 = time (extent T)
  links        [4 mu][V][3][3]   U_mu(x), the link x -> x + mu
  spinors      [V][4 spin][3 colour]
"""
from __future__ import annotations

import numpy as np

# The eight Gell-Mann matrices; H = sum_a h_a lambda_a / 2 is traceless Hermitian.
_GM = np.zeros((8, 3, 3), dtype=np.complex128)
_GM[0][0, 1] = _GM[0][1, 0] = 1
_GM[1][0, 1], _GM[1][1, 0] = -1j, 1j
_GM[2][0, 0], _GM[2][1, 1] = 1, -1
_GM[3][0, 2] = _GM[3][2, 0] = 1
_GM[4][0, 2], _GM[4][2, 0] = -1j, 1j
_GM[5][1, 2] = _GM[5][2, 1] = 1
_GM[6][1, 2], _GM[6][2, 1] = -1j, 1j
_GM[7][0, 0] = _GM[7][1, 1] = 1 / np.sqrt(3)
_GM[7][2, 2] = -2 / np.sqrt(3)

# Seed namespaces: links use [LINK_SEED, cfg], noise [NOISE_SEED, cfg, i, j].
LINK_SEED = 1211
NOISE_SEED = 1214
SPINOR_SEED = 1212


def volume(lat) -> int:
    return int(np.prod([int(v) for v in lat]))


def make_links(lat, eps: float = 0.3, cfg: int = 0, chunk: int = 1 << 18) -> np.ndarray:
    """SU(3) links U = exp(i*eps*H), H = sum_a h_a lambda_a/2, h_a ~ N(0,1) i.i.d.

    Draw order: standard_normal((4, V, 8)) from default_rng(SeedSequence([1211, cfg])).
    The exponential is taken through the eigen-decomposition of H, so U is
    unitary with det U = exp(i*eps*tr H) = 1 to rounding.
    """
    V = volume(lat)
    rng = np.random.default_rng(np.random.SeedSequence([LINK_SEED, int(cfg)]))
    h = rng.standard_normal((4, V, 8))
    out = np.empty((4, V, 3, 3), dtype=np.complex128)
    hf = h.reshape(4 * V, 8)
    of = out.reshape(4 * V, 3, 3)
    for s in range(0, 4 * V, chunk):
        H = np.einsum("na,aij->nij", hf[s:s + chunk], _GM / 2)
        w, Q = np.linalg.eigh(H)
        ph = np.exp(1j * eps * w)
        of[s:s + chunk] = (Q * ph[:, None, :]) @ Q.conj().swapaxes(-1, -2)
    return out


def unit_links(lat) -> np.ndarray:
    """Free field: every link is the identity."""
    V = volume(lat)
    out = np.zeros((4, V, 3, 3), dtype=np.complex128)
    out[..., 0, 0] = out[..., 1, 1] = out[..., 2, 2] = 1
    return out


def make_noise(lat, cfg: int, i: int, j: int) -> np.ndarray:
    """Complex Gaussian noise with density pi^-n exp(-eta^dag eta): Re, Im ~ N(0, 1/2).

    Drawn on the full lattice, shape [V][4][3], from
    default_rng(SeedSequence([1214, cfg, i, j])).standard_normal((V, 4, 3, 2)) * sqrt(1/2).
    """
    V = volume(lat)
    rng = np.random.default_rng(np.random.SeedSequence([NOISE_SEED, int(cfg), int(i), int(j)]))
    r = rng.standard_normal((V, 4, 3, 2)) * np.sqrt(0.5)
    return r[..., 0] + 1j * r[..., 1]


def make_noise_batch(lat, cfg: int, n_interp: int, n_hit: int) -> np.ndarray:
    """All noise vectors of one estimate, shape [n_interp][n_hit][V][4][3]."""
    V = volume(lat)
    out = np.empty((n_interp, n_hit, V, 4, 3), dtype=np.complex128)
    for i in range(n_interp):
        for j in range(n_hit):
            out[i, j] = make_noise(lat, cfg, i, j)
    return out


def make_spinor(lat, seed: int, nrhs: int | None = None) -> np.ndarray:
    """Random Gaussian spinor(s) for operator tests; shape [V][4][3] or [nrhs][V][4][3]."""
    V = volume(lat)
    rng = np.random.default_rng(np.random.SeedSequence([SPINOR_SEED, int(seed)]))
    shape = (V, 4, 3, 2) if nrhs is None else (nrhs, V, 4, 3, 2)
    r = rng.standard_normal(shape)
    return r[..., 0] + 1j * r[..., 1]


def make_gauge_transform(lat, seed: int) -> np.ndarray:
    """Random site-local SU(3) matrices Omega(x), shape [V][3][3] (same recipe, eps = 1)."""
    V = volume(lat)
    rng = np.random.default_rng(np.random.SeedSequence([SPINOR_SEED + 7, int(seed)]))
    h = rng.standard_normal((V, 8))
    H = np.einsum("na,aij->nij", h, _GM / 2)
    w, Q = np.linalg.eigh(H)
    return (Q * np.exp(1j * w)[:, None, :]) @ Q.conj().swapaxes(-1, -2)


# The benchmark and test workloads, by lattice size: lattice (T, L1, L2, L3), Schwarz block,
# kappa_1 -> kappa_2, interpolation steps N, noise vectors N_hit, and the seed that selects
# their link and noise streams (make_links(lat, eps, seed), make_noise(lat, seed, i, j)).
WORKLOADS = {
    "4x4^3": dict(seed=1, name="4x4^3 blocks 2^4", lat=(4, 4, 4, 4), blk=(2, 2, 2, 2), kappa1=0.1200,
                  kappa2=0.1210, n_interp=1, n_hit=8, csw=1.0, eps=0.3),
    "8x8^3": dict(seed=2, name="8x8^3 blocks 4^4", lat=(8, 8, 8, 8), blk=(4, 4, 4, 4), kappa1=0.1200,
                  kappa2=0.1210, n_interp=1, n_hit=16, csw=1.0, eps=0.3),
    "48x24^3": dict(seed=3, name="48x24^3 blocks 6^4", lat=(48, 24, 24, 24), blk=(6, 6, 6, 6), kappa1=0.1200,
                    kappa2=0.1205, n_interp=1, n_hit=12, csw=1.0, eps=0.3),
    "64x32^3": dict(seed=4, name="64x32^3 blocks 8^4", lat=(64, 32, 32, 32), blk=(8, 8, 8, 8), kappa1=0.1200,
                    kappa2=0.1205, n_interp=4, n_hit=24, csw=1.0, eps=0.3),
    "32x16^3": dict(seed=5, name="32x16^3 blocks 4^4", lat=(32, 16, 16, 16), blk=(4, 4, 4, 4), kappa1=0.1200,
                    kappa2=0.1205, n_interp=1, n_hit=8, csw=1.0, eps=0.3),
}
