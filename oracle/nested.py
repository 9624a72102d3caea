"""Nested domain decomposition (test infrastructure only).

Sec. 2.2 (the larger ensemble): the 8^4 Schwarz blocks are decomposed once more, into an
8^4 Schur complement with Dirichlet boundaries and 4^4 blocks.  Written out with the
identity of Sec. 1 one level down:  for the outer blocks of one colour c, the operator
A_c = D_cc is the direct sum of their Dirichlet block operators D_k (Sec. 1).  Splitting
every outer block into inner blocks and colouring those black and white gives

    prod_{k of colour c} det D_k = det A_c = det Ahat_c * det A_bb * det A_ww,
    Ahat_c = 1 - A_bb^-1 A_bw A_ww^-1 A_wb,

with A_bb, A_ww the direct sums of the inner Dirichlet blocks D_s inside colour-c outer
blocks.  The inner block determinants are small enough to compute exactly (the paper does
so for blocks up to 6^4); the ratio of det Ahat_c between two masses is estimated like
W_gl (Eq. 8), with the global inversion of D replaced by the inversion of A_c (a block
solve of colour c), so the same estimator code applies to this class unchanged.

Readings (the paper gives only the sentence above):
  * the inner blocks keep the colouring of the inner decomposition of the whole lattice
    ((sum of inner block coordinates) mod 2), so neighbouring inner blocks inside one
    outer block always have opposite colours;
  * P_c projects onto the face sites of black inner blocks inside colour-c outer blocks,
    faces on the outer boundary included: A_wb has no entries there, those columns of
    Ahat_c are the identity's and its determinant is unchanged;
  * the Schur-complement factor is estimated with the same mass interpolation and noise
    as W_gl, one estimate per outer colour.
"""
from __future__ import annotations

import numpy as np

from . import lattice as lt
from .krylov import Inverse
from .schwarz import Schwarz, _components


class Nested(Schwarz):
    """The Schwarz interface (parts, block solves, hops, P, Schur complement and its inverse)
    for A_c: the Dirichlet operator of the colour-c outer blocks, split by the inner blocks."""

    def __init__(self, U, lat, outer, inner, csw: float, colour: int, time_bc: int = -1, tol: float = 1e-14):
        super().__init__(U, lat, inner, csw, time_bc, tol)
        lt.check_geometry(lat, outer)
        for B, b in zip(outer, inner):
            if B % b != 0:
                raise ValueError(f"inner block extent {b} does not divide outer extent {B}")
        if colour not in (0, 1):
            raise ValueError("colour must be 0 or 1")
        self.outer, self.colour = tuple(outer), colour
        region = lt.colour(lat, outer) == colour
        self.region = region
        self.R = _components(np.nonzero(region)[0])
        col = lt.colour(lat, inner)
        self.black_sites = np.nonzero((col == 0) & region)[0]
        self.white_sites = np.nonzero((col == 1) & region)[0]
        self.B = _components(self.black_sites)
        self.W = _components(self.white_sites)
        face = lt.face_black(lat, inner) & region
        self.p_sites = np.nonzero(face)[0]
        self.P = _components(self.p_sites)
        self.P_in_B = _components(np.nonzero(face[self.black_sites])[0])

    def A(self, m: float):
        """A_c(m) = D(m) restricted to the sites of the colour-c outer blocks."""
        return self.D(m)[self.R][:, self.R]

    def inv_full(self, m: float):
        """A_c(m)^-1 on full-lattice vectors (input read, output written on colour-c outer blocks only)."""
        key = ("iA", m)
        if key not in self._cache:
            inv = Inverse(self.A(m), self.tol)
            R, n = self.R, 12 * self.V

            def solve(v):
                out = np.zeros(n, dtype=complex)
                out[R] = inv(np.asarray(v).reshape(-1)[R])
                return out

            self._cache[key] = solve
        return self._cache[key]

    def inner_block_logdets(self, m: float):
        """(sign, ln|det D_s(m)|) of every inner block inside the colour-c outer blocks, both inner
        colours, by dense LU of each block."""
        bid = lt.block_id(self.lat, self.blk)
        D = self.D(m)
        out = []
        for k in np.unique(bid[self.region]):
            idx = _components(np.nonzero(bid == k)[0])
            sgn, la = np.linalg.slogdet(D[idx][:, idx].toarray())
            out.append((float(sgn.real), float(la)))
        return out


def log_w_total(U, lat, outer, inner, csw, m1, m2, eta_gl, eta_nested, time_bc=-1, tol=1e-14):
    """Two-flavour log W with nested DD (Eq. 7 with the outer block factors split again):

        log W = log W_gl[outer] + sum_c log W_c[nested] + 2 sum_s [ln|det D_s(m2)| - ln|det D_s(m1)|],

    s over all inner blocks, W_gl and W_c the stochastic estimates (Eq. 8) from the noise
    eta_gl and eta_nested[c] (each [N, N_hit, V, 4, 3])."""
    from . import estimator
    S = Schwarz(U, lat, outer, csw, time_bc, tol)
    lw = estimator.log_w_gl(estimator.exponents(S, m1, m2, eta_gl, "schur", "diff"))
    for c in (0, 1):
        Nc = Nested(U, lat, outer, inner, csw, c, time_bc, tol)
        lw += estimator.log_w_gl(estimator.exponents(Nc, m1, m2, eta_nested[c], "schur", "diff"))
        lw += 2 * (sum(la for _, la in Nc.inner_block_logdets(m2)) - sum(la for _, la in Nc.inner_block_logdets(m1)))
    return lw


class NestedMatrixFree:
    """The same interface for lattices too large for assembled matrices: the matrix-free C
    version of the oracle with the inner blocks (inner block solves and hops) and with the
    outer blocks (the inversion of A_c is a block solve of colour c); every hop cut to the
    colour-c outer blocks."""

    def __init__(self, U, lat, outer, inner, csw: float, colour: int, time_bc: int = -1, tol: float = 1e-13):
        from .cref import CRef
        for B, b in zip(outer, inner):
            if B % b != 0:
                raise ValueError(f"inner block extent {b} does not divide outer extent {B}")
        self.lat, self.colour, self.tol = tuple(lat), colour, tol
        self.V = lt.volume(lat)
        self.inner = CRef(U, lat, inner, csw, time_bc)
        self.outer = CRef(U, lat, outer, csw, time_bc)
        self.region = (lt.colour(lat, outer) == colour)[:, None, None]
        self.pmask = (lt.face_black(lat, inner) & (lt.colour(lat, outer) == colour))[:, None, None]

    def close(self):
        self.inner.close()
        self.outer.close()

    def flat(self, psi):
        return np.asarray(psi).reshape(-1)

    def _spinor(self, psi):
        return np.asarray(psi).reshape(self.V, 4, 3)

    def restrict_P(self, psi):
        return self._spinor(psi) * self.pmask

    def hop_wb(self, m, psi):
        return self.inner.hop(1, self._spinor(psi)) * self.region

    def hop_bw(self, m, psi):
        return self.inner.hop(0, self._spinor(psi)) * self.region

    def block_inverse(self, colour: int, m: float, psi):
        return self.inner.block_solve(colour, m, self._spinor(psi), self.tol)

    def hat_inverse(self, m: float, phi):
        """Ahat_c^-1 phi = phi - P_c [A_c^-1 (0_b, A_wb phi)]_b."""
        f = self.restrict_P(phi)
        chi = self.outer.block_solve(self.colour, m, self.hop_wb(m, f), self.tol)
        return self.restrict_P(f - self.restrict_P(chi))
