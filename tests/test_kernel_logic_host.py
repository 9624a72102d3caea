"""The library's per-site device code (geometry, spin projection, clover build and
application) executed on the host through tests/host/kernel_logic.cpp, against the
FP64 oracle.  Needs hipcc but no GPU."""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import dirac
from oracle.schwarz import Schwarz
from paper_1211_1214_amd import inputs

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "host", "kernel_logic.cpp")
LIB = os.path.join(HERE, "host", "libkernel_logic.so")


@pytest.fixture(scope="module")
def L():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    deps = [SRC] + [os.path.join(HERE, "..", "paper_1211_1214_amd", "csrc", f)
                    for f in ("ddwc_device.h", "clover_build.h", "eo.h", "force.h")]
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < max(os.path.getmtime(d) for d in deps):
        subprocess.check_call([hipcc, "--offload-arch=gfx950", "-O2", "-std=c++17", "-fPIC", "-shared", SRC,
                               "-o", LIB + ".tmp"], stderr=subprocess.DEVNULL)
        os.replace(LIB + ".tmp", LIB)
    lib = ctypes.CDLL(LIB)
    P = ctypes.c_void_p
    lib.host_apply.argtypes = [P, P, ctypes.c_int, ctypes.c_double, P, P, ctypes.c_double, ctypes.c_int,
                               ctypes.c_int, P, P]
    lib.host_force.argtypes = [P, P, ctypes.c_int, ctypes.c_double, P, P, P, P]
    lib.host_h16_roundtrip.argtypes = [P, P, P]
    return lib


def run(L, lat, blk, tbc, csw, U, psi, kappa, mode, colour):
    out = np.zeros_like(psi)
    clov = np.zeros((int(np.prod(lat)), 72))
    L.host_apply((ctypes.c_int * 4)(*lat), (ctypes.c_int * 4)(*blk), tbc, csw, U.ctypes.data, psi.ctypes.data,
                 kappa, mode, colour, out.ctypes.data, clov.ctypes.data)
    return out, clov


@pytest.mark.parametrize("lat,blk,tbc", [((4, 4, 4, 4), (2, 2, 2, 2), -1), ((4, 6, 6, 6), (2, 3, 3, 3), -1),
                                         ((8, 4, 2, 6), (2, 2, 1, 3), 1)])
def test_host_operator_matches_oracle(L, lat, blk, tbc):
    U = inputs.make_links(lat, 0.3, 3)
    psi = inputs.make_spinor(lat, 4)
    S = Schwarz(U, lat, blk, 1.0, tbc)
    m = dirac.mass(0.121)
    out, clov = run(L, lat, blk, tbc, 1.0, U, psi, 0.121, 0, 0)
    want = dirac.apply(S.D(m), psi)
    assert np.abs(out - want).max() < 1e-13 * np.abs(want).max()
    for c in (0, 1):
        out, _ = run(L, lat, blk, tbc, 1.0, U, psi, 0.121, 1, c)
        assert np.abs(out - S.block_apply(c, m, psi)).max() < 1e-13 * np.abs(want).max()
        out, _ = run(L, lat, blk, tbc, 1.0, U, psi, 0.121, 2, c)
        hop = S.hop_wb(m, psi) if c == 1 else S.hop_bw(m, psi)
        assert np.abs(out - hop).max() < 1e-13 * np.abs(want).max()


def test_host_clover_packing(L):
    """The 72 packed reals reproduce the oracle's 12x12 clover term in its two chiral blocks."""
    lat, blk = (4, 4, 4, 4), (2, 2, 2, 2)
    U = inputs.make_links(lat, 0.3, 5)
    _, clov = run(L, lat, blk, -1, 1.3, U, inputs.make_spinor(lat, 1), 0.12, 0, 0)
    C = dirac.clover_term(U, lat, 1.3)
    for x in (0, 17, 255):
        for b in range(2):
            A = np.zeros((6, 6), complex)
            A[np.diag_indices(6)] = clov[x, 6 * b:6 * b + 6]
            off = clov[x, 12 + 30 * b:42 + 30 * b].reshape(15, 2)
            iu = np.triu_indices(6, 1)
            A[iu] = off[:, 0] + 1j * off[:, 1]
            A[(iu[1], iu[0])] = np.conj(A[iu])
            assert np.abs(A - C[x][6 * b:6 * b + 6, 6 * b:6 * b + 6]).max() < 1e-15
        assert np.abs(C[x][:6, 6:]).max() == 0


@pytest.mark.parametrize("lat,blk,tbc", [((4, 4, 4, 4), (2, 2, 2, 2), -1), ((8, 4, 4, 8), (2, 2, 2, 4), 1)])
def test_host_even_odd_operator(L, lat, blk, tbc):
    """Mee = A_ee - D_eo A_oo^-1 D_oe on sites of even parity (x0+x1+x2+x3 even), from the
    library's half-field helpers, against the oracle's assembled operator."""
    import scipy.sparse.linalg as sla
    from oracle import lattice as lt
    P = ctypes.c_void_p
    L.host_eo_apply.argtypes = [P, P, ctypes.c_int, ctypes.c_double, P, P, ctypes.c_double, P]
    U = inputs.make_links(lat, 0.3, 6)
    psi = inputs.make_spinor(lat, 9)
    out = np.zeros_like(psi)
    rc = L.host_eo_apply((ctypes.c_int * 4)(*lat), (ctypes.c_int * 4)(*blk), tbc, 1.0, U.ctypes.data,
                         psi.ctypes.data, 0.1213, out.ctypes.data)
    assert rc == 0
    D = dirac.dirac(U, lat, dirac.mass(0.1213), 1.0, tbc).tocsc()
    par = lt.coords(lat).sum(axis=1) % 2
    ev = (12 * np.nonzero(par == 0)[0][:, None] + np.arange(12)).ravel()
    od = (12 * np.nonzero(par == 1)[0][:, None] + np.arange(12)).ravel()
    x = psi.reshape(-1)
    want = D[ev][:, ev] @ x[ev] - D[ev][:, od] @ sla.spsolve(D[od][:, od], D[od][:, ev] @ x[ev])
    got = out.reshape(-1)
    assert np.abs(got[ev] - want).max() < 1e-12 * np.abs(want).max()
    assert np.all(got[od] == 0)


@pytest.mark.parametrize("csw", [0.0, 1.0])
def test_host_force_matches_finite_differences(L, csw):
    """The force code's gradient G of Re <a, D(U) b> (hop and clover terms) against extrapolated
    central differences of the oracle's operator along a random link direction dU:
    Re sum conj(G) dU = d/dh Re <a, D(U + h dU) b>."""
    lat, blk = (4, 4, 2, 6), (2, 2, 1, 3)
    V = int(np.prod(lat))
    U = np.ascontiguousarray(inputs.make_links(lat, 0.3, 8))
    rng = np.random.default_rng(3)
    a = np.ascontiguousarray(rng.standard_normal((V, 4, 3)) + 1j * rng.standard_normal((V, 4, 3)))
    b = np.ascontiguousarray(rng.standard_normal((V, 4, 3)) + 1j * rng.standard_normal((V, 4, 3)))
    dU = rng.standard_normal(U.shape) + 1j * rng.standard_normal(U.shape)
    G = np.zeros_like(U)
    L.host_force((ctypes.c_int * 4)(*lat), (ctypes.c_int * 4)(*blk), -1, csw, U.ctypes.data, a.ctypes.data,
                 b.ctypes.data, G.ctypes.data)

    def f(h):
        D = dirac.dirac(U + h * dU, lat, 0.1, csw, -1)
        return float(np.vdot(a.reshape(-1), D @ b.reshape(-1)).real)

    def d(h):
        return (f(h) - f(-h)) / (2 * h)

    fd = (4 * d(5e-5) - d(1e-4)) / 3
    got = float(np.sum(np.conj(G) * dU).real)
    assert abs(got - fd) < 1e-8 * abs(fd), (got, fd)


def test_host_fp16_spinor_storage(L):
    """FP16 storage with a per-site scale: the scale is the largest component modulus and every
    component comes back within half a unit in the last place of FP16 relative to it (2^-11)."""
    rng = np.random.default_rng(5)
    for mag in (1e-30, 1e-3, 1.0, 7e4, 3e30):
        v = np.ascontiguousarray(rng.standard_normal(24) * mag)
        out = np.zeros(24)
        sc = np.zeros(1, dtype=np.float32)
        L.host_h16_roundtrip(v.ctypes.data, out.ctypes.data, sc.ctypes.data)
        m = np.abs(v.astype(np.float32)).max()
        assert abs(sc[0] - m) <= 1e-7 * m
        assert np.abs(out - v).max() <= (2.0 ** -11 + 2e-7) * m
    z = np.zeros(24)
    out = np.ones(24)
    sc = np.ones(1, dtype=np.float32)
    L.host_h16_roundtrip(z.ctypes.data, out.ctypes.data, sc.ctypes.data)
    assert sc[0] == 0 and np.all(out == 0)
