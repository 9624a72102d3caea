"""Thin ctypes binding of libddwc.so (include/ddwc.h).

Argument marshalling only: every step of the computation runs in the library's HIP
kernels.  Tensors are torch tensors on the GPU (PyTorch provides device memory and
the stream); they are passed as raw device pointers.  If the library has not been
built this module raises on first use: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libddwc.so")

OK, EINVAL, ENOCONV, EHIP, ENONFINITE, EUNDEF = 0, -1, -2, -3, -4, -5
FP64, MIXED32, MIXED16 = 0, 1, 2
BLACK, WHITE = 0, 1
OP_FULL, OP_SCHUR = 0, 1
K_DSLASH64, K_DSLASH32, K_BLOCK, K_BLAS, K_OTHER, K_EOHOP = range(6)
(OPT_GRAPHS, OPT_POLL, OPT_BLOCK_THREADS, OPT_SOLVER, OPT_BLOCK_LDS, OPT_BLOCK_KERNEL, OPT_INNER_FLOOR,
 OPT_OP_THREADS, OPT_TILE_ORDER) = range(9)
_STATUS = {EINVAL: "EINVAL", ENOCONV: "ENOCONV", EHIP: "EHIP", ENONFINITE: "ENONFINITE", EUNDEF: "EUNDEF"}

# Every function the header declares, with its ctypes signature.
_P, _I, _D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
_PD, _PI, _PLL = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_longlong)


class Stats(ctypes.Structure):
    _fields_ = [("outer_iters", ctypes.c_int), ("inner_iters", ctypes.c_int),
                ("rel_residual", ctypes.c_double), ("seconds", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_PS = ctypes.POINTER(Stats)
SIGNATURES = {
    "ddwc_create": (_I, [ctypes.POINTER(_P), _P, _P, _I, _D, _P, _P]),
    "ddwc_destroy": (_I, [_P]),
    "ddwc_dslash_apply": (_I, [_P, _D, _P, _P, _I, _I, _P]),
    "ddwc_dslash_apply_noalloc": (_I, [_P, _D, _P, _P, _I, _I, _P]),
    "ddwc_block_solve": (_I, [_P, _I, _D, _P, _P, _I, _D, _I, _I, _PS, _P]),
    "ddwc_schur_apply": (_I, [_P, _D, _I, _P, _P, _I, _D, _I, _PS, _P]),
    "ddwc_solve": (_I, [_P, _D, _P, _P, _I, _D, _I, _I, _PS, _P]),
    "ddwc_det_ratio_estimate": (_I, [_P, _D, _D, _I, _I, _I, _P, _I, _D, _I, _PD, _PD, _PD, _PS, _P]),
    "ddwc_det_ratio_nested": (_I, [_P, _P, _I, _D, _D, _I, _I, _P, _I, _D, _I, _PD, _PD, _PD, _PS, _P]),
    "ddwc_det_ratio_grad": (_I, [_P, _D, _D, _I, _I, _P, _I, _D, _I, _PD, _PD, _P, _PS, _P]),
    "ddwc_link_force": (_I, [_P, _P, _P, _I, _PD, _P, _P]),
    "ddwc_block_logdet": (_I, [_P, _D, _I, _PD, _PI, _P]),
    "ddwc_log_w_blocks": (_I, [_P, _D, _D, _PD, _P]),
    "ddwc_log_w_combine": (_I, [_PD, _I, _I, _I, _PD, _PD, _PD]),
    "ddwc_log_w_nested_total": (_I, [_P, _P, _D, _D, _I, _P, _I, _P, _P, _I, _D, _I, _PD, _PS, _P]),
    "ddwc_set_option": (_I, [_P, _I, _I]),
    "ddwc_get_option": (_I, [_P, _I, _PI]),
    "ddwc_autotune": (_I, [_P, _D, _I, _I, _PD, _P]),
    "ddwc_profile_enable": (_I, [_P, _I]),
    "ddwc_profile_read": (_I, [_P, _I, _PLL, _PD, _PD]),
    "ddwc_dslash_bytes": (_D, [_P, _I, _I]),
    "ddwc_stream_copy": (_I, [_P, _P, ctypes.c_size_t, _P]),
    "ddwc_last_error": (ctypes.c_char_p, []),
    "ddwc_version": (ctypes.c_char_p, []),
}

_lib = None


def lib():
    """Load libddwc.so; raise loudly if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1211_1214_amd.build.build() "
                               "(there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class DDWCError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        msg = lib().ddwc_last_error().decode(errors="replace")
        super().__init__(f"{where}: {_STATUS.get(code, code)}: {msg}")


def _check(code, where, allow=()):
    if code != OK and code not in allow:
        raise DDWCError(code, where)
    return code


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t, V=None, what="tensor"):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{what} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{what} must be on the GPU")
    if t.dtype != torch.complex128:
        raise TypeError(f"{what} must be complex128")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _spinors(t, V, what):
    """Shape check: [V,4,3] or [n,V,4,3] -> number of RHS."""
    sh = tuple(t.shape)
    if sh[-3:] != (V, 4, 3):
        raise ValueError(f"{what} must end in ({V}, 4, 3), got {sh}")
    return int(np.prod(sh[:-3])) if len(sh) > 3 else 1


def log_w_combine(x, n_f=2, grad=False, allow=()):
    """ddwc_log_w_combine on given exponents x [n_interp, n_hit] (complex for n_f = 1), on the host:
    {"log_w", "step_var", "gx" (d log_w / dx for n_f = 2 when grad), "status"}."""
    x = np.asarray(x)
    if x.ndim != 2:
        raise ValueError("x must have shape (n_interp, n_hit)")
    n_interp, n_hit = x.shape
    xa = np.ascontiguousarray(np.stack([x.real, x.imag], axis=-1) if n_f == 1 else x, dtype=np.float64)
    lw = ctypes.c_double()
    var = np.zeros(n_interp)
    gx = np.zeros((n_interp, n_hit)) if grad else None
    code = _check(lib().ddwc_log_w_combine(xa.ctypes.data_as(_PD), int(n_interp), int(n_hit), int(n_f),
                                           ctypes.byref(lw), var.ctypes.data_as(_PD),
                                           gx.ctypes.data_as(_PD) if grad else None), "ddwc_log_w_combine",
                  allow=allow)
    return {"log_w": lw.value, "step_var": var, "gx": gx, "status": code}


def stream_copy(src, dst):
    """dst = src by the library's streaming reference kernel (same-size contiguous device tensors)."""
    if src.numel() * src.element_size() != dst.numel() * dst.element_size():
        raise ValueError("src and dst must have the same size in bytes")
    if not (src.is_cuda and dst.is_cuda and src.is_contiguous() and dst.is_contiguous()):
        raise ValueError("src and dst must be contiguous device tensors")
    _check(lib().ddwc_stream_copy(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                                  src.numel() * src.element_size(), _stream()), "ddwc_stream_copy")


def mass(kappa: float) -> float:
    return 1.0 / (2.0 * kappa) - 4.0


class Context:
    """One gauge field on one GPU: links (complex128 [4, V, 3, 3] on the device)."""

    def __init__(self, links, lat, blk, time_bc: int = -1, csw: float = 1.0):
        import torch
        self.lat = tuple(int(v) for v in lat)
        self.blk = tuple(int(v) for v in blk)
        self.V = int(np.prod(self.lat))
        if tuple(links.shape) != (4, self.V, 3, 3):
            raise ValueError(f"links must have shape (4, {self.V}, 3, 3)")
        self.device = links.device
        L = lib()
        h = ctypes.c_void_p()
        la = (ctypes.c_int * 4)(*self.lat)
        ba = (ctypes.c_int * 4)(*self.blk)
        with torch.cuda.device(self.device):
            _check(L.ddwc_create(ctypes.byref(h), la, ba, int(time_bc), float(csw), _ptr(links, what="links"),
                                 _stream()), "ddwc_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().ddwc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _empty_like(self, t):
        import torch
        return torch.empty_like(t)

    def dslash_apply(self, kappa, inp, out=None, prec=FP64):
        n = _spinors(inp, self.V, "input")
        out = self._empty_like(inp) if out is None else out
        _check(lib().ddwc_dslash_apply(self._h, float(kappa), _ptr(inp), _ptr(out), n, int(prec), _stream()),
               "ddwc_dslash_apply")
        return out

    def block_solve(self, colour, kappa, rhs, tol=1e-12, maxit=10000, prec=FP64, out=None):
        n = _spinors(rhs, self.V, "rhs")
        out = self._empty_like(rhs) if out is None else out
        st = Stats()
        _check(lib().ddwc_block_solve(self._h, int(colour), float(kappa), _ptr(rhs), _ptr(out), n, float(tol),
                                      int(maxit), int(prec), ctypes.byref(st), _stream()), "ddwc_block_solve")
        return out, st.as_dict()

    def schur_apply(self, kappa, inp, inverse=False, tol=1e-12, prec=FP64, out=None):
        n = _spinors(inp, self.V, "input")
        out = self._empty_like(inp) if out is None else out
        st = Stats()
        _check(lib().ddwc_schur_apply(self._h, float(kappa), int(bool(inverse)), _ptr(inp), _ptr(out), n,
                                      float(tol), int(prec), ctypes.byref(st), _stream()), "ddwc_schur_apply")
        return out, st.as_dict()

    def solve(self, kappa, b, tol=1e-12, maxit=10000, prec=FP64, out=None):
        n = _spinors(b, self.V, "b")
        out = self._empty_like(b) if out is None else out
        st = Stats()
        _check(lib().ddwc_solve(self._h, float(kappa), _ptr(b), _ptr(out), n, float(tol), int(maxit), int(prec),
                                ctypes.byref(st), _stream()), "ddwc_solve")
        return out, st.as_dict()

    def det_ratio_estimate(self, kappa1, kappa2, eta, op=OP_SCHUR, tol=1e-12, prec=FP64, n_f=2, allow=()):
        """eta: complex128 [n_interp, n_hit, V, 4, 3] on the device.  x is complex for n_f = 1.
        Status codes in `allow` (e.g. (EUNDEF,)) are returned in "status" instead of raised."""
        sh = tuple(eta.shape)
        if len(sh) != 5 or sh[2:] != (self.V, 4, 3):
            raise ValueError(f"eta must have shape (n_interp, n_hit, {self.V}, 4, 3)")
        n_interp, n_hit = sh[:2]
        x = np.zeros((n_interp, n_hit) if n_f == 2 else (n_interp, n_hit, 2))
        var = np.zeros(n_interp)
        lw = ctypes.c_double()
        st = Stats()
        code = _check(lib().ddwc_det_ratio_estimate(
            self._h, float(kappa1), float(kappa2), int(n_interp), int(op), int(n_f), _ptr(eta), int(n_hit),
            float(tol), int(prec), x.ctypes.data_as(_PD), ctypes.byref(lw), var.ctypes.data_as(_PD),
            ctypes.byref(st), _stream()), "ddwc_det_ratio_estimate", allow=allow)
        if n_f == 1:
            x = x[..., 0] + 1j * x[..., 1]
        return {"x": x, "log_w_gl": lw.value, "step_var": var, "stats": st.as_dict(), "status": code}

    def det_ratio_nested(self, inner, colour, kappa1, kappa2, eta, tol=1e-12, prec=FP64, n_f=2, allow=()):
        """Nested-DD factor of the outer blocks of one colour (this context: outer blocks; inner: a
        Context of the same links with smaller blocks): x and log |det Ahat(m2)/det Ahat(m1)|^2."""
        sh = tuple(eta.shape)
        if len(sh) != 5 or sh[2:] != (self.V, 4, 3):
            raise ValueError(f"eta must have shape (n_interp, n_hit, {self.V}, 4, 3)")
        n_interp, n_hit = sh[:2]
        x = np.zeros((n_interp, n_hit) if n_f == 2 else (n_interp, n_hit, 2))
        var = np.zeros(n_interp)
        lw = ctypes.c_double()
        st = Stats()
        code = _check(lib().ddwc_det_ratio_nested(
            self._h, inner._h, int(colour), float(kappa1), float(kappa2), int(n_interp), int(n_f), _ptr(eta),
            int(n_hit), float(tol), int(prec), x.ctypes.data_as(_PD), ctypes.byref(lw), var.ctypes.data_as(_PD),
            ctypes.byref(st), _stream()), "ddwc_det_ratio_nested", allow=allow)
        if n_f == 1:
            x = x[..., 0] + 1j * x[..., 1]
        return {"x": x, "log_w": lw.value, "step_var": var, "stats": st.as_dict(), "status": code}

    def log_w_nested(self, inner, kappa1, kappa2, eta_gl, eta_nested, tol=1e-12, prec=FP64):
        """Two-flavour log W with nested DD (ddwc_log_w_nested_total): log W_gl of this context (outer
        blocks, Schur), the nested factors of both colours, the exact inner block factor, and the total.
        eta_gl [n_interp, n_hit, V, 4, 3]; eta_nested = (black, white), each [n_interp, n_hit2, V, 4, 3]."""
        sh, sb, sw = tuple(eta_gl.shape), tuple(eta_nested[0].shape), tuple(eta_nested[1].shape)
        for s_ in (sh, sb, sw):
            if len(s_) != 5 or s_[2:] != (self.V, 4, 3):
                raise ValueError(f"noise must have shape (n_interp, n_hit, {self.V}, 4, 3)")
        if sb != sw or sb[0] != sh[0]:
            raise ValueError("the nested noise of both colours must have one shape and the same n_interp")
        parts = np.zeros(5)
        st = Stats()
        _check(lib().ddwc_log_w_nested_total(
            self._h, inner._h, float(kappa1), float(kappa2), int(sh[0]), _ptr(eta_gl, what="eta_gl"), int(sh[1]),
            _ptr(eta_nested[0], what="eta_black"), _ptr(eta_nested[1], what="eta_white"), int(sb[1]), float(tol),
            int(prec), parts.ctypes.data_as(_PD), ctypes.byref(st), _stream()), "ddwc_log_w_nested_total")
        names = ("log_w_gl", "log_w_nested0", "log_w_nested1", "log_w_inner_blocks", "log_w")
        return {k: float(v) for k, v in zip(names, parts)}

    def det_ratio_grad(self, kappa1, kappa2, eta, gx, op=OP_SCHUR, tol=1e-12, prec=FP64, want_kappa2=True,
                       want_links=True):
        """dL/dkappa2 and dL/dU (torch convention dL/dRe U + i dL/dIm U, complex128 [4, V, 3, 3] on the
        device) for L = sum_ij gx[i, j] x_ij, with x_ij the two-flavour exponents of det_ratio_estimate."""
        import torch
        sh = tuple(eta.shape)
        if len(sh) != 5 or sh[2:] != (self.V, 4, 3):
            raise ValueError(f"eta must have shape (n_interp, n_hit, {self.V}, 4, 3)")
        n_interp, n_hit = sh[:2]
        gx = np.ascontiguousarray(np.asarray(gx, dtype=np.float64))
        if gx.shape != (n_interp, n_hit):
            raise ValueError(f"gx must have shape ({n_interp}, {n_hit})")
        dk = ctypes.c_double()
        dU = torch.empty((4, self.V, 3, 3), dtype=torch.complex128, device=eta.device) if want_links else None
        st = Stats()
        _check(lib().ddwc_det_ratio_grad(
            self._h, float(kappa1), float(kappa2), int(n_interp), int(op), _ptr(eta), int(n_hit), float(tol),
            int(prec), gx.ctypes.data_as(_PD), ctypes.byref(dk) if want_kappa2 else None,
            _ptr(dU, what="dU") if want_links else None, ctypes.byref(st), _stream()), "ddwc_det_ratio_grad")
        return {"dkappa2": dk.value if want_kappa2 else None, "dU": dU, "stats": st.as_dict()}

    def link_force(self, a, b, w=None):
        """dF/dRe U + i dF/dIm U for F = sum_r w_r Re <a_r, D b_r> (complex128 [4, V, 3, 3], device)."""
        import torch
        n = _spinors(a, self.V, "a")
        if _spinors(b, self.V, "b") != n or tuple(a.shape) != tuple(b.shape):
            raise ValueError("a and b must have the same shape")
        w = np.ascontiguousarray(np.ones(n) if w is None else np.asarray(w, dtype=np.float64).reshape(n))
        dU = torch.empty((4, self.V, 3, 3), dtype=torch.complex128, device=a.device)
        _check(lib().ddwc_link_force(self._h, _ptr(a, what="a"), _ptr(b, what="b"), int(n), w.ctypes.data_as(_PD),
                                     _ptr(dU, what="dU"), _stream()), "ddwc_link_force")
        return dU

    def block_logdet(self, kappa, colour):
        """(ln|det D_k|, sign) of every Dirichlet block of one colour, blocks sorted by coordinates."""
        nbc = int(np.prod([l // b for l, b in zip(self.lat, self.blk)])) // 2
        la = np.zeros(nbc)
        sg = np.zeros(nbc, dtype=np.int32)
        _check(lib().ddwc_block_logdet(self._h, float(kappa), int(colour), la.ctypes.data_as(_PD),
                                       sg.ctypes.data_as(_PI), _stream()), "ddwc_block_logdet")
        return la, sg

    def log_w_blocks(self, kappa1, kappa2):
        """Block factor of log W for two flavours (Eq. 7): 2 sum_k [ln|det D_k(m2)| - ln|det D_k(m1)|]."""
        out = ctypes.c_double()
        _check(lib().ddwc_log_w_blocks(self._h, float(kappa1), float(kappa2), ctypes.byref(out), _stream()),
               "ddwc_log_w_blocks")
        return out.value

    def set_option(self, option, value):
        _check(lib().ddwc_set_option(self._h, int(option), int(value)), "ddwc_set_option")

    def get_option(self, option):
        v = ctypes.c_int()
        _check(lib().ddwc_get_option(self._h, int(option), ctypes.byref(v)), "ddwc_get_option")
        return v.value

    def autotune(self, kappa, nrhs, prec=MIXED32):
        """Times the schedule options and keeps the fastest; returns the options and the tuning time."""
        t = ctypes.c_double()
        _check(lib().ddwc_autotune(self._h, float(kappa), int(nrhs), int(prec), ctypes.byref(t), _stream()),
               "ddwc_autotune")
        return {"graphs": self.get_option(OPT_GRAPHS), "poll": self.get_option(OPT_POLL),
                "block_threads": self.get_option(OPT_BLOCK_THREADS), "block_lds": self.get_option(OPT_BLOCK_LDS),
                "block_kernel": self.get_option(OPT_BLOCK_KERNEL), "op_threads": self.get_option(OPT_OP_THREADS),
                "tile_order": self.get_option(OPT_TILE_ORDER), "seconds": t.value}

    def profile_enable(self, on=True):
        _check(lib().ddwc_profile_enable(self._h, int(bool(on))), "ddwc_profile_enable")

    def profile_read(self, kclass):
        n = ctypes.c_longlong()
        ms = ctypes.c_double()
        by = ctypes.c_double()
        _check(lib().ddwc_profile_read(self._h, int(kclass), ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by)),
               "ddwc_profile_read")
        return {"launches": n.value, "ms": ms.value, "bytes": by.value}

    def dslash_bytes(self, nrhs, prec):
        return lib().ddwc_dslash_bytes(self._h, int(nrhs), int(prec))
