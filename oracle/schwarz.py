"""Schwarz block decomposition and Schur complement (test infrastructure only).

Sec. 1 of the paper: with the lattice split into black and white blocks,

      D = [[D_bb, D_bw], [D_wb, D_ww]],     D^-1 = [[Dc_bb, Dc_bw], [Dc_wb, Dc_ww]],

  det D = det Dhat * det D_ww * det D_bb,   Dhat = 1 - D_bb^-1 D_bw D_ww^-1 D_wb,

D_bb (D_ww) block-diagonal with the Dirichlet block operators D_k of one colour
on the diagonal.  With the projector P defined by D_wb P = D_wb, Dhat may be
restricted to range(P) without changing its determinant, and there
Dhat^-1 = 1 - P Dc_bw D_wb: one global inversion of D (Sec. 1, Sec. 2.1).

Here the sub-matrices are taken literally as the black/white rows and columns
of the assembled D.  Black blocks never touch each other, so D_bb is
automatically the direct sum of the Dirichlet block operators.  Vectors at
this interface are canonical full-lattice spinors (V, 4, 3); Schur-space
vectors are zero off range(P).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import lattice as lt
from .dirac import dirac_massless
from .krylov import Inverse


def _components(sites: np.ndarray) -> np.ndarray:
    return (12 * sites[:, None] + np.arange(12)[None, :]).ravel()


class Schwarz:
    def __init__(self, U, lat, blk, csw: float, time_bc: int = -1, tol: float = 1e-14):
        lt.check_geometry(lat, blk)
        self.lat, self.blk = tuple(lat), tuple(blk)
        self.V = lt.volume(lat)
        self.tol = tol
        self.D0 = dirac_massless(U, lat, csw, time_bc)
        col = lt.colour(lat, blk)
        self.black_sites = np.nonzero(col == 0)[0]
        self.white_sites = np.nonzero(col == 1)[0]
        self.B = _components(self.black_sites)
        self.W = _components(self.white_sites)
        face = lt.face_black(lat, blk)
        self.p_sites = np.nonzero(face)[0]
        self.P = _components(self.p_sites)                       # in full-lattice numbering
        self.P_in_B = _components(np.nonzero(face[self.black_sites])[0])  # in black numbering
        self._cache = {}

    # -- matrices ---------------------------------------------------------
    def D(self, m: float) -> sp.csr_matrix:
        return (self.D0 + m * sp.identity(12 * self.V, dtype=complex, format="csr")).tocsr()

    def parts(self, m: float):
        key = ("parts", m)
        if key not in self._cache:
            D = self.D(m)
            Dbb = D[self.B][:, self.B]
            Dbw = D[self.B][:, self.W]
            Dwb = D[self.W][:, self.B]
            Dww = D[self.W][:, self.W]
            self._cache[key] = (Dbb, Dbw, Dwb, Dww)
        return self._cache[key]

    def inv_bb(self, m):
        key = ("ibb", m)
        if key not in self._cache:
            self._cache[key] = Inverse(self.parts(m)[0], self.tol)
        return self._cache[key]

    def inv_ww(self, m):
        key = ("iww", m)
        if key not in self._cache:
            self._cache[key] = Inverse(self.parts(m)[3], self.tol)
        return self._cache[key]

    def inv_full(self, m):
        key = ("ifull", m)
        if key not in self._cache:
            self._cache[key] = Inverse(self.D(m), self.tol)
        return self._cache[key]

    # -- vector views -----------------------------------------------------
    def flat(self, psi):
        return np.asarray(psi).reshape(-1)

    def to_full(self, vec, idx):
        out = np.zeros(12 * self.V, dtype=complex)
        out[idx] = vec
        return out.reshape(self.V, 4, 3)

    def restrict_P(self, psi):
        """P psi as a full-lattice spinor (zero off range(P))."""
        return self.to_full(self.flat(psi)[self.P], self.P)

    # -- block operators (Dirichlet blocks of one colour) -------------------
    def block_apply(self, colour: int, m: float, psi):
        """D_bb psi (colour 0) or D_ww psi (colour 1); psi is full-lattice, other colour ignored."""
        Dbb, _, _, Dww = self.parts(m)
        idx = self.B if colour == 0 else self.W
        A = Dbb if colour == 0 else Dww
        return self.to_full(A @ self.flat(psi)[idx], idx)

    def block_inverse(self, colour: int, m: float, psi):
        idx = self.B if colour == 0 else self.W
        inv = self.inv_bb(m) if colour == 0 else self.inv_ww(m)
        return self.to_full(inv(self.flat(psi)[idx]), idx)

    def hop_wb(self, m, psi):
        """D_wb psi: black -> white (white-site output)."""
        return self.to_full(self.parts(m)[2] @ self.flat(psi)[self.B], self.W)

    def hop_bw(self, m, psi):
        """D_bw psi: white -> black (black-site output)."""
        return self.to_full(self.parts(m)[1] @ self.flat(psi)[self.W], self.B)

    # -- Schur complement -------------------------------------------------
    def hat_apply(self, m: float, eta):
        """Dhat_P eta = P (1 - D_bb^-1 D_bw D_ww^-1 D_wb) P eta."""
        e = self.restrict_P(eta)
        w = self.block_inverse(1, m, self.hop_wb(m, e))
        b = self.block_inverse(0, m, self.hop_bw(m, w))
        return self.restrict_P(self.flat(e) - self.flat(b))

    def hat_inverse(self, m: float, phi):
        """Dhat_P^-1 phi = phi - P [D^-1 (0_b, D_wb phi)]_b  (Sec. 1, last formula)."""
        f = self.restrict_P(phi)
        src = self.hop_wb(m, f)
        chi = self.inv_full(m)(self.flat(src))
        return self.restrict_P(self.flat(f) - self.restrict_P(chi.reshape(self.V, 4, 3)).reshape(-1))

    def block_logdets(self, colour: int, m: float):
        """(sign, ln|det D_k(m)|) of every Dirichlet block k of one colour (Sec. 1: D_bb and D_ww
        are the direct sums of the D_k), by dense LU of each block, ordered by block coordinates
        (n_0, n_1, n_2, n_3) lexicographically.  det D_k is real (gamma_5-hermiticity), so the
        sign is the real part of the unit phase."""
        bid = lt.block_id(self.lat, self.blk)
        col = lt.colour(self.lat, self.blk)
        D = self.D(m)
        out = []
        for k in np.unique(bid[col == colour]):
            idx = _components(np.nonzero(bid == k)[0])
            sgn, la = np.linalg.slogdet(D[idx][:, idx].toarray())
            out.append((float(sgn.real), float(la)))
        return out

    def log_w_blocks(self, m1: float, m2: float) -> float:
        """Block part of log W for two flavours (Eq. 7): 2 sum_k [ln|det D_k(m2)| - ln|det D_k(m1)|]."""
        tot = 0.0
        for c in (0, 1):
            tot += sum(la for _, la in self.block_logdets(c, m2)) - sum(la for _, la in self.block_logdets(c, m1))
        return 2 * tot

    def hat_dense(self, m: float) -> np.ndarray:
        """P Dhat P as a dense matrix on range(P) (small lattices only)."""
        Dbb, Dbw, Dwb, Dww = (a.toarray() for a in self.parts(m))
        hat = np.eye(len(self.B)) - np.linalg.solve(Dbb, Dbw @ np.linalg.solve(Dww, Dwb))
        return hat[np.ix_(self.P_in_B, self.P_in_B)]
