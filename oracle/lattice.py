"""Lattice geometry for the oracle (test infrastructure only).

Sec. 1 of the paper splits the lattice into blocks coloured black and white in
a checkerboard; D_bb, D_ww are block-diagonal over the blocks of one colour and
the projector P is defined by D_wb P = D_wb.

Readings (the paper is silent on these):
  * site index x = ((x0*L1 + x1)*L2 + x2)*L3 + x3, x0 = time;
  * time boundary antiperiodic (bc = -1) unless asked otherwise, space periodic;
  * block coordinate n_mu = x_mu // b_mu, colour (sum_mu n_mu) mod 2, black = 0;
  * P projects onto the black sites that have a nearest neighbour in another
    block (x_mu mod b_mu in {0, b_mu - 1} for some mu), all 12 components.
"""
from __future__ import annotations

import numpy as np


def volume(lat) -> int:
    return int(np.prod(lat))


def coords(lat) -> np.ndarray:
    """(V, 4) integer coordinates, x3 fastest."""
    T, L1, L2, L3 = lat
    g = np.meshgrid(np.arange(T), np.arange(L1), np.arange(L2), np.arange(L3), indexing="ij")
    return np.stack([a.ravel() for a in g], axis=1)


def index(lat, c: np.ndarray) -> np.ndarray:
    """Site index of coordinates c (..., 4), wrapped periodically."""
    T, L1, L2, L3 = lat
    c0 = np.mod(c[..., 0], T)
    c1 = np.mod(c[..., 1], L1)
    c2 = np.mod(c[..., 2], L2)
    c3 = np.mod(c[..., 3], L3)
    return ((c0 * L1 + c1) * L2 + c2) * L3 + c3


def neighbour(lat, mu: int, step: int, time_bc: int = -1):
    """Index of x + step*mu_hat for every site, and the boundary factor of that hop.

    The factor is time_bc for a hop that crosses the time boundary, else 1.
    """
    c = coords(lat)
    d = c.copy()
    d[:, mu] += step
    fac = np.ones(len(c))
    if mu == 0:
        crossed = (d[:, 0] < 0) | (d[:, 0] >= lat[0])
        fac[crossed] = time_bc
    return index(lat, d), fac


def block_coords(lat, blk) -> np.ndarray:
    return coords(lat) // np.asarray(blk)


def colour(lat, blk) -> np.ndarray:
    """0 = black, 1 = white."""
    return block_coords(lat, blk).sum(axis=1) % 2


def block_id(lat, blk) -> np.ndarray:
    """Lexicographic block number of every site."""
    nb = np.asarray(lat) // np.asarray(blk)
    n = block_coords(lat, blk)
    return ((n[:, 0] * nb[1] + n[:, 1]) * nb[2] + n[:, 2]) * nb[3] + n[:, 3]


def face_black(lat, blk) -> np.ndarray:
    """Boolean per site: black and on the face of its block (the support of P)."""
    c = coords(lat)
    b = np.asarray(blk)
    r = c % b
    face = ((r == 0) | (r == b - 1)).any(axis=1)
    return face & (colour(lat, blk) == 0)


def check_geometry(lat, blk) -> None:
    for L, b in zip(lat, blk):
        if b < 1 or L % b != 0:
            raise ValueError(f"block extent {b} does not divide lattice extent {L}")
        nb = L // b
        if nb < 2 or nb % 2 != 0:
            raise ValueError(f"{nb} blocks in a direction: need an even number >= 2")
