"""Derivatives of the determinant-ratio exponents and of log W_gl (test infrastructure only).

The quantity differentiated is the log of the estimator of Eq. (8),
    L = log W_gl = sum_i [logsumexp_j(-x_ij) - ln N_hit],
as a function of kappa2 (through m2 = 1/(2 kappa2) - 4 and the interpolation masses
m_i, linear in m) and of the link matrices U (through the hops and the clover term),
with the noise vectors held fixed.

Derivatives are taken by their plain definition: central differences of the oracle's
exponents (exact solves), extrapolated (Richardson) to remove the h^2 term,
    D(h) = (f(h) - f(-h)) / 2h,    f'(0) = (4 D(h/2) - D(h)) / 3 + O(h^4).
Link derivatives are directional: along a field dU of 3x3 complex matrices (no
unitarity constraint), so that the derivative equals Re sum conj(G) . dU for the
gradient G = dL/dRe U + i dL/dIm U.
"""
from __future__ import annotations

import numpy as np

from . import dirac, estimator
from .schwarz import Schwarz


def richardson(f, h: float) -> np.ndarray:
    """f'(0) for f: float -> array, by extrapolated central differences."""
    def d(hh):
        return (np.asarray(f(hh)) - np.asarray(f(-hh))) / (2 * hh)
    return (4 * d(h / 2) - d(h)) / 3


def exponents_at(U, lat, blk, csw, kappa1, kappa2, eta, op="schur", time_bc=-1):
    """x_ij of Eq. (8) (difference form, exact solves) for links U and noise eta [N, N_hit, V, 4, 3]."""
    S = Schwarz(U, lat, blk, csw, time_bc)
    return estimator.exponents(S, dirac.mass(kappa1), dirac.mass(kappa2), eta, op, "diff")


def dx_dkappa2(U, lat, blk, csw, kappa1, kappa2, eta, op="schur", h=None):
    """d x_ij / d kappa2 for every sample."""
    h = h if h is not None else 1e-5 * kappa2
    return richardson(lambda d: exponents_at(U, lat, blk, csw, kappa1, kappa2 + d, eta, op), h)


def dx_dlinks(U, dU, lat, blk, csw, kappa1, kappa2, eta, op="schur", h=1e-5):
    """Directional derivative of every x_ij along the link field dU."""
    U = np.asarray(U)
    return richardson(lambda d: exponents_at(U + d * dU, lat, blk, csw, kappa1, kappa2, eta, op), h)


def log_w_weights(x) -> np.ndarray:
    """dL/dx_ij = -softmax_j(-x_ij) per step (L = log W_gl)."""
    a = -np.asarray(x, dtype=float)
    w = np.exp(a - a.max(axis=1, keepdims=True))
    return -w / w.sum(axis=1, keepdims=True)
