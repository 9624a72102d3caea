"""Plain linear solves for the oracle (test infrastructure only).

The paper leaves the inversion method open ("one estimation costs one
inversion", Sec. 2 and Sec. 2.1); any solve that is exact to rounding or to a
tight tolerance gives the same estimator.  Two routes:

  * a direct sparse LU (SuperLU through scipy) for small operators;
  * textbook BiCGStab (van der Vorst 1992), run column by column on a block of
    right-hand sides, restarted from the true residual until
    ||b - A x|| <= tol * ||b|| in FP64.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as sla

DIRECT_MAX_DIM = 4096


def _bicgstab(A, b, x, maxit):
    """BiCGStab on every column of b at once (scalars are per column)."""
    r = b - A @ x
    rhat = r.copy()
    p = r.copy()
    rho = np.einsum("ij,ij->j", rhat.conj(), r)
    for _ in range(maxit):
        v = A @ p
        den = np.einsum("ij,ij->j", rhat.conj(), v)
        alpha = np.where(den != 0, rho / np.where(den != 0, den, 1), 0)
        s = r - alpha * v
        t = A @ s
        tt = np.einsum("ij,ij->j", t.conj(), t).real
        omega = np.where(tt > 0, np.einsum("ij,ij->j", t.conj(), s) / np.where(tt > 0, tt, 1), 0)
        x = x + alpha * p + omega * s
        r = s - omega * t
        rho_new = np.einsum("ij,ij->j", rhat.conj(), r)
        rn = np.sqrt(np.einsum("ij,ij->j", r.conj(), r).real)
        if np.all(rn <= 1e-9 * np.linalg.norm(b, axis=0)):
            break
        beta = np.where((rho != 0) & (omega != 0),
                        rho_new / np.where(rho != 0, rho, 1) * alpha / np.where(omega != 0, omega, 1), 0)
        p = r + beta * (p - omega * v)
        rho = rho_new
    return x


class Inverse:
    """x = A^-1 b for a sparse square A, to tolerance tol in the true FP64 residual."""

    def __init__(self, A: sp.spmatrix, tol: float = 1e-14, maxit: int = 5000):
        self.A = sp.csr_matrix(A)
        self.tol = tol
        self.maxit = maxit
        self.lu = None
        if self.A.shape[0] <= DIRECT_MAX_DIM:
            self.lu = sla.splu(sp.csc_matrix(self.A))

    def __call__(self, b: np.ndarray) -> np.ndarray:
        vec = b.ndim == 1
        B = b.reshape(-1, 1) if vec else b
        if self.lu is not None:
            X = self.lu.solve(B)
            X = X + self.lu.solve(B - self.A @ X)
        else:
            X = np.zeros_like(B)
            bn = np.linalg.norm(B, axis=0)
            for _ in range(20):
                R = B - self.A @ X
                if np.all(np.linalg.norm(R, axis=0) <= self.tol * bn):
                    break
                X = X + _bicgstab(self.A, R, np.zeros_like(R), self.maxit)
            else:
                raise RuntimeError("oracle solve did not reach its tolerance")
        return X.ravel() if vec else X
