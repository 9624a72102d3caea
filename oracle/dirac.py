"""Assembled Wilson-clover Dirac operator in FP64 (test infrastructure only).

The paper uses the O(a)-improved Wilson-Dirac operator D(U, m) (Sec. 1, Sec. 2)
without printing it, and relies on the mass entering as a pure shift,
D(m1) = D(m2) + (m1 - m2), so that M = 1 + dm * D(m2)^-1 (Eq. 6).  That fixes
the mass normalisation.  The textbook Sheikholeslami-Wohlert operator in that
normalisation is written out here as a sparse 12V x 12V matrix:

  (D psi)(x) = (4 + m) psi(x) + C(x) psi(x)
               - 1/2 sum_mu [ (1 - g_mu) U_mu(x) psi(x+mu)
                            + (1 + g_mu) U_mu(x-mu)^dag psi(x-mu) ]

  C(x) = c_sw * (i/4) * sum_{mu,nu} sigma_{mu nu} (x) Fhat_{mu nu}(x),
  sigma_{mu nu} = (i/2) [g_mu, g_nu],  Fhat = (Q - Q^dag)/8,
  Q_{mu nu}(x) = sum of the four plaquette leaves at x,

  m = 1/(2 kappa) - 4, hops across the time boundary carry time_bc.

Readings: chiral gamma basis, no trace subtraction in Fhat, no boundary sign in
the clover links, component index 12*site + 3*spin + colour.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import lattice as lt

# Chiral basis: g0 = [[0,-1],[-1,0]], gk = [[0,-i s_k],[i s_k,0]] in 2x2 spin blocks.
_S = [np.array([[0, 1], [1, 0]], dtype=complex),
      np.array([[0, -1j], [1j, 0]], dtype=complex),
      np.array([[1, 0], [0, -1]], dtype=complex)]
_I2 = np.eye(2, dtype=complex)
_Z2 = np.zeros((2, 2), dtype=complex)

GAMMA = np.zeros((4, 4, 4), dtype=complex)
GAMMA[0] = np.block([[_Z2, -_I2], [-_I2, _Z2]])
for _k in range(3):
    GAMMA[_k + 1] = np.block([[_Z2, -1j * _S[_k]], [1j * _S[_k], _Z2]])
GAMMA5 = GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]
SIGMA = np.zeros((4, 4, 4, 4), dtype=complex)
for _m in range(4):
    for _n in range(4):
        SIGMA[_m, _n] = 0.5j * (GAMMA[_m] @ GAMMA[_n] - GAMMA[_n] @ GAMMA[_m])


def mass(kappa: float) -> float:
    """Bare mass of the hopping parameter: m = 1/(2 kappa) - 4."""
    return 1.0 / (2.0 * kappa) - 4.0


def _dag(a):
    return a.conj().swapaxes(-1, -2)


def plaquette_sum(U, lat, mu: int, nu: int) -> np.ndarray:
    """Q_{mu nu}(x): the four plaquette leaves in the mu-nu plane that touch x."""
    xpm, _ = lt.neighbour(lat, mu, +1)
    xpn, _ = lt.neighbour(lat, nu, +1)
    xmm, _ = lt.neighbour(lat, mu, -1)
    xmn, _ = lt.neighbour(lat, nu, -1)
    # x - mu + nu, x - mu - nu, x + mu - nu
    xmm_pn = xpn[xmm]
    xmm_mn = xmn[xmm]
    xpm_mn = xmn[xpm]
    Um, Un = U[mu], U[nu]
    q = Um @ Un[xpm] @ _dag(Um[xpn]) @ _dag(Un)
    q = q + Un @ _dag(Um[xmm_pn]) @ _dag(Un[xmm]) @ Um[xmm]
    q = q + _dag(Um[xmm]) @ _dag(Un[xmm_mn]) @ Um[xmm_mn] @ Un[xmn]
    q = q + _dag(Un[xmn]) @ Um[xmn] @ Un[xpm_mn] @ _dag(Um)
    return q


def field_strength(U, lat, mu: int, nu: int) -> np.ndarray:
    """Fhat_{mu nu}(x) = (Q - Q^dag)/8, shape (V, 3, 3)."""
    q = plaquette_sum(U, lat, mu, nu)
    return (q - _dag(q)) / 8.0


def clover_term(U, lat, csw: float) -> np.ndarray:
    """C(x) as (V, 12, 12) with index 3*spin + colour; sum over all ordered pairs mu != nu."""
    V = lt.volume(lat)
    C = np.zeros((V, 12, 12), dtype=complex)
    if csw == 0.0:
        return C
    for mu in range(4):
        for nu in range(4):
            if mu == nu:
                continue
            F = field_strength(U, lat, mu, nu)
            C += np.einsum("st,xab->xsatb", SIGMA[mu, nu], F).reshape(V, 12, 12)
    return csw * 0.25j * C


def _block_coo(rows_site, cols_site, blocks):
    """COO triplets of V 12x12 blocks placed at (12*r, 12*c)."""
    V = len(rows_site)
    ii = (12 * rows_site)[:, None, None] + np.arange(12)[None, :, None]
    jj = (12 * cols_site)[:, None, None] + np.arange(12)[None, None, :]
    ii = np.broadcast_to(ii, (V, 12, 12))
    jj = np.broadcast_to(jj, (V, 12, 12))
    return ii.ravel(), jj.ravel(), blocks.ravel()


def dirac_massless(U, lat, csw: float, time_bc: int = -1) -> sp.csr_matrix:
    """D(m = 0) = 4 + C - H/2 as a sparse matrix; D(m) = D(0) + m * 1."""
    V = lt.volume(lat)
    sites = np.arange(V)
    I4 = np.eye(4, dtype=complex)
    I3 = np.eye(3, dtype=complex)
    diag = 4.0 * np.broadcast_to(np.kron(I4, I3), (V, 12, 12)) + clover_term(U, lat, csw)
    R, Cc, Vv = [], [], []
    r, c, v = _block_coo(sites, sites, diag)
    R.append(r), Cc.append(c), Vv.append(v)
    for mu in range(4):
        fwd, ffac = lt.neighbour(lat, mu, +1, time_bc)
        bwd, bfac = lt.neighbour(lat, mu, -1, time_bc)
        pm = I4 - GAMMA[mu]
        pp = I4 + GAMMA[mu]
        bf = -0.5 * ffac[:, None, None] * np.einsum("st,xab->xsatb", pm, U[mu]).reshape(V, 12, 12)
        Ub = _dag(U[mu][bwd])
        bb = -0.5 * bfac[:, None, None] * np.einsum("st,xab->xsatb", pp, Ub).reshape(V, 12, 12)
        for cols, blk in ((fwd, bf), (bwd, bb)):
            r, c, v = _block_coo(sites, cols, blk)
            R.append(r), Cc.append(c), Vv.append(v)
    A = sp.coo_matrix((np.concatenate(Vv), (np.concatenate(R), np.concatenate(Cc))),
                      shape=(12 * V, 12 * V))
    return A.tocsr()


def dirac(U, lat, m: float, csw: float, time_bc: int = -1) -> sp.csr_matrix:
    D0 = dirac_massless(U, lat, csw, time_bc)
    return (D0 + m * sp.identity(D0.shape[0], dtype=complex, format="csr")).tocsr()


def apply(D: sp.csr_matrix, psi: np.ndarray) -> np.ndarray:
    """D psi for a canonical spinor psi of shape (V, 4, 3)."""
    return (D @ psi.reshape(-1)).reshape(psi.shape)


def gamma5_vector(psi: np.ndarray) -> np.ndarray:
    """gamma_5 acting on spin of a (..., V, 4, 3) spinor."""
    return np.einsum("st,...xtc->...xsc", GAMMA5, psi)


def gauge_transform_links(U, lat, Om):
    """U^Om_mu(x) = Om(x) U_mu(x) Om(x+mu)^dag."""
    out = np.empty_like(U)
    for mu in range(4):
        fwd, _ = lt.neighbour(lat, mu, +1)
        out[mu] = Om @ U[mu] @ _dag(Om[fwd])
    return out


def gauge_transform_spinor(psi, Om):
    return np.einsum("xab,xsb->xsa", Om, psi)
