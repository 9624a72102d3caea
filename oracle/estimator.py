"""Two-flavour stochastic determinant-ratio estimator (test infrastructure only).

Eq. (2)-(3): W = det D(m2)^2 / det D(m1)^2 = 1/det(M^dag M) with
M = D(m2)^-1 D(m1), estimated as (1/N_hit) sum_j exp(-eta_j^dag (M^dag M - 1) eta_j)
for complex Gaussian eta.  Eq. (8): with N mass-interpolation steps and the
Schur complement,

   W_gl = prod_i (1/N_hit) sum_j exp(-x_ij),  x_ij = eta_ij^dag (Mh_i^dag Mh_i - 1) eta_ij,
   Mh_i = Dhat_P(m_i)^-1 Dhat_P(m_{i-1}),  m_i = (i/N) m2 + ((N - i)/N) m1.

The plain definition x = ||M eta||^2 - ||eta||^2 is computed, and beside it a
cancellation-free difference form (a second route; both must agree):

  full:   M eta - eta = dm D(m2)^-1 eta          => x = 2 dm Re<eta, psi> + dm^2 ||psi||^2
  Schur:  Mh eta - eta = Dhat_P(m2)^-1 g,
          g = dm P [D_bb1^-1 D_bb2^-1 D_bw D_ww1^-1 D_wb + D_bb2^-1 D_bw D_ww1^-1 D_ww2^-1 D_wb] eta,
  from A(m1)^-1 - A(m2)^-1 = -dm A(m1)^-1 A(m2)^-1 for A = D_bb, D_ww, which holds
  because the mass is a pure shift (Eq. 6), dm = m1 - m2.

The estimate is combined in the log domain (the exponentials under- or
overflow FP64 on large lattices): log W_gl = sum_i [logsumexp_j(-x_ij) - ln N_hit].
The per-step relative sample variance var_j(e^-x)/mean_j(e^-x)^2 (N_hit - 1 in
the denominator) is the quantity Sec. 2.1 asks to monitor with N_hit >= 6.

One flavour (Sec. 3, Eq. 11): 1/det M = E exp(-eta^dag (M - 1) eta), defined while every
eigenvalue of M has a positive real part.  The exponent x = eta^dag (M - 1) eta is complex;
by gamma_5-hermiticity the expectation is real, so only the real part of the sample mean is
kept.  Plain form x = <eta, M eta> - ||eta||^2; difference forms x = dm <eta, psi> (full)
and x = <e, zeta> (Schur), with psi and zeta as above.  Per step,
log W_i = ln Re[(1/N_hit) sum_j exp(-x_ij)], undefined (nan) when that real part is <= 0.
"""
from __future__ import annotations

import numpy as np

from .schwarz import Schwarz


def interpolation_masses(m1: float, m2: float, n: int) -> np.ndarray:
    """m_i = (i/N) m2 + ((N - i)/N) m1, i = 0..N (linear in m, Sec. 2.1)."""
    i = np.arange(n + 1)
    return (i / n) * m2 + ((n - i) / n) * m1


def _nrm2(v):
    v = np.asarray(v).reshape(-1)
    return float(np.sum(v.real ** 2 + v.imag ** 2))


def _redot(a, b):
    return float(np.vdot(np.asarray(a).reshape(-1), np.asarray(b).reshape(-1)).real)


def _dot(a, b) -> complex:
    """<a, b> = sum conj(a) b."""
    return complex(np.vdot(np.asarray(a).reshape(-1), np.asarray(b).reshape(-1)))


def x_full_plain(S: Schwarz, m_prev: float, m_next: float, eta) -> float:
    y = S.inv_full(m_next)(S.D(m_prev) @ S.flat(eta))
    return _nrm2(y) - _nrm2(eta)


def x_full_diff(S: Schwarz, m_prev: float, m_next: float, eta) -> float:
    dm = m_prev - m_next
    psi = S.inv_full(m_next)(S.flat(eta))
    return 2 * dm * _redot(eta, psi) + dm * dm * _nrm2(psi)


def x_schur_plain(S: Schwarz, m_prev: float, m_next: float, eta) -> float:
    e = S.restrict_P(eta)
    y = S.hat_inverse(m_next, S.hat_apply(m_prev, e))
    return _nrm2(y) - _nrm2(e)


def schur_difference_source(S: Schwarz, m1: float, m2: float, eta):
    """g = (Dhat_P(m1) - Dhat_P(m2)) eta in the resolvent form above."""
    dm = m1 - m2
    e = S.restrict_P(eta)
    v = S.hop_wb(m1, e)
    w1 = S.block_inverse(1, m1, v)
    w12 = S.block_inverse(1, m2, w1)
    a1 = S.block_inverse(0, m1, S.hop_bw(m1, w1))
    b = S.hop_bw(m1, w12)
    g = S.block_inverse(0, m2, S.flat(a1) + S.flat(b))
    return S.restrict_P(dm * S.flat(g))


def x_schur_diff(S: Schwarz, m_prev: float, m_next: float, eta) -> float:
    e = S.restrict_P(eta)
    zeta = S.hat_inverse(m_next, schur_difference_source(S, m_prev, m_next, e))
    return 2 * _redot(e, zeta) + _nrm2(zeta)


# ---------------------------------------------------------------- one flavour (Eq. 11)
def x1_full_plain(S: Schwarz, m_prev: float, m_next: float, eta) -> complex:
    """eta^dag (M - 1) eta with M = D(m_next)^-1 D(m_prev)."""
    y = S.inv_full(m_next)(S.D(m_prev) @ S.flat(eta))
    return _dot(eta, y) - _nrm2(eta)


def x1_full_diff(S: Schwarz, m_prev: float, m_next: float, eta) -> complex:
    dm = m_prev - m_next
    psi = S.inv_full(m_next)(S.flat(eta))
    return dm * _dot(eta, psi)


def x1_schur_plain(S: Schwarz, m_prev: float, m_next: float, eta) -> complex:
    e = S.restrict_P(eta)
    y = S.hat_inverse(m_next, S.hat_apply(m_prev, e))
    return _dot(e, y) - _nrm2(e)


def x1_schur_diff(S: Schwarz, m_prev: float, m_next: float, eta) -> complex:
    e = S.restrict_P(eta)
    zeta = S.hat_inverse(m_next, schur_difference_source(S, m_prev, m_next, e))
    return _dot(e, zeta)


def exponents(S: Schwarz, m1: float, m2: float, eta, op: str = "schur", form: str = "diff", n_f: int = 2):
    """x[i][j] for noise eta of shape (N, N_hit, V, 4, 3); complex for n_f = 1."""
    eta = np.asarray(eta)
    n, nhit = eta.shape[:2]
    ms = interpolation_masses(m1, m2, n)
    if n_f == 2:
        f = {("full", "plain"): x_full_plain, ("full", "diff"): x_full_diff,
             ("schur", "plain"): x_schur_plain, ("schur", "diff"): x_schur_diff}[(op, form)]
    elif n_f == 1:
        f = {("full", "plain"): x1_full_plain, ("full", "diff"): x1_full_diff,
             ("schur", "plain"): x1_schur_plain, ("schur", "diff"): x1_schur_diff}[(op, form)]
    else:
        raise ValueError("n_f must be 1 or 2")
    x = np.empty((n, nhit), dtype=float if n_f == 2 else complex)
    for i in range(n):
        for j in range(nhit):
            x[i, j] = f(S, ms[i], ms[i + 1], eta[i, j])
    return x


def log_w_gl(x) -> float:
    """log W_gl = sum_i [max_j a_ij + ln sum_j exp(a_ij - max_j a_ij) - ln N_hit], a = -x."""
    a = -np.asarray(x, dtype=float)
    amax = a.max(axis=1)
    return float(np.sum(amax + np.log(np.sum(np.exp(a - amax[:, None]), axis=1)) - np.log(a.shape[1])))


def step_variance(x) -> np.ndarray:
    """Relative sample variance of exp(-x_ij) over j, per step i (scale-free, log domain)."""
    a = -np.asarray(x, dtype=float)
    w = np.exp(a - a.max(axis=1, keepdims=True))
    mean = w.mean(axis=1)
    var = w.var(axis=1, ddof=1) if a.shape[1] > 1 else np.zeros(a.shape[0])
    return var / mean ** 2


def _one_flavour_weights(x):
    """Re exp(-x_ij + a_i) = exp(-Re x_ij + a_i) cos(Im x_ij), a_i = max_j(-Re x_ij)."""
    x = np.asarray(x, dtype=complex)
    a = -x.real
    amax = a.max(axis=1)
    return amax, np.exp(a - amax[:, None]) * np.cos(x.imag)


def log_w_one_flavour(x) -> float:
    """sum_i ln Re[(1/N_hit) sum_j exp(-x_ij)] (Eq. 11 per step); nan if a step's mean is <= 0."""
    amax, w = _one_flavour_weights(x)
    s = w.sum(axis=1)
    if np.any(s <= 0):
        return float("nan")
    return float(np.sum(amax + np.log(s) - np.log(w.shape[1])))


def step_variance_one_flavour(x) -> np.ndarray:
    """Relative sample variance of Re exp(-x_ij) over j, per step i."""
    _, w = _one_flavour_weights(x)
    mean = w.mean(axis=1)
    var = w.var(axis=1, ddof=1) if w.shape[1] > 1 else np.zeros(w.shape[0])
    return var / mean ** 2
