"""Python binding of the HIP library ``libmodalproj.so`` (C ABI in
``include/modalproj.h``).

Argument marshalling only: every step of the projection runs in the
library's HIP kernels.  PyTorch supplies device memory and the stream the
library enqueues on.  There is no fallback: if the shared library is missing
or no device is usable, the calls raise.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmodalproj.so")

MODAL_FP64, MODAL_MIXED = 0, 1
ORDERED, SYMMETRIC = 0, 1
STAGES = ("gl", "legendre", "bessel", "beta", "S", "triple", "gather",
          "adj_triple", "adj_S", "adj_beta", "prep", "adj_prep")
_PREC = {"fp64": MODAL_FP64, "mixed": MODAL_MIXED}
_KIND = {"ordered": ORDERED, "symmetric": SYMMETRIC}

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)


class ModalGrid(ctypes.Structure):
    _fields_ = [("lmin", ctypes.c_int32), ("lmax", ctypes.c_int32),
                ("nk", ctypes.c_int32), ("k", ctypes.c_void_p), ("wk", ctypes.c_void_p),
                ("nr", ctypes.c_int32), ("r", ctypes.c_void_p), ("wr", ctypes.c_void_p),
                ("nmu", ctypes.c_int32), ("mu", ctypes.c_void_p), ("wmu", ctypes.c_void_p),
                ("allow_inexact_gl", ctypes.c_int32)]


class ModalProblem(ctypes.Structure):
    _fields_ = [("delta", ctypes.c_void_p), ("cl", ctypes.c_void_p),
                ("np", ctypes.c_int32), ("qk", ctypes.c_void_p),
                ("na", ctypes.c_int32), ("ql", ctypes.c_void_p),
                ("v_power", ctypes.c_double), ("kind", ctypes.c_int32),
                ("ta", ctypes.c_int32), ("tri_a", ctypes.c_void_p),
                ("tp", ctypes.c_int32), ("tri_p", ctypes.c_void_p)]


class ModalError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"modalproj status {status}: {message}")
        self.status = status


_lib = None


def lib() -> ctypes.CDLL:
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1503_08809_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
        G, P = ctypes.POINTER(ModalGrid), ctypes.POINTER(ModalProblem)
        sig = {
            "modal_create": [ctypes.POINTER(vp), ctypes.c_int, vp],
            "modal_destroy": [vp],
            "modal_set_stream": [vp, vp],
            "modal_set_workspace_limit": [vp, sz],
            "modal_workspace_bytes": [vp, G, P, ctypes.c_int, ctypes.POINTER(sz)],
            "modal_enable_timing": [vp, ctypes.c_int],
            "modal_set_forward_reuse": [vp, ctypes.c_int],
            "modal_stage_times": [vp, _dp, ctypes.c_int],
            "modal_stage_counts": [vp, ctypes.POINTER(i32), ctypes.c_int],
            "modal_gauss_legendre": [vp, i32, vp, vp],
            "modal_legendre_table": [vp, i32, i32, vp, vp],
            "modal_sph_bessel_table": [vp, i32, i64, vp, vp],
            "modal_beta": [vp, G, P, ctypes.c_int, vp],
            "modal_S": [vp, G, P, ctypes.c_int, vp, vp],
            "modal_gamma_from_S": [vp, G, P, ctypes.c_int, vp, vp],
            "modal_gamma": [vp, G, P, ctypes.c_int, vp],
            "modal_gamma_noalloc": [vp, G, P, ctypes.c_int, vp],
            "modal_gram": [vp, G, P, ctypes.c_int, vp],
            "modal_gamma_modal": [vp, G, P, ctypes.c_int, vp],
            "modal_gamma_backward": [vp, G, P, ctypes.c_int, vp, vp, vp],
            "modal_r_weights": [i32, i32, vp, vp],
            "modal_gamma_3d": [vp, G, P, i32, vp],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.modal_status_str.argtypes = [ctypes.c_int]
        L.modal_status_str.restype = ctypes.c_char_p
        L.modal_last_error.argtypes = [vp]
        L.modal_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def exported_symbols():
    """Names of the C entry points the binding declares."""
    return ["modal_create", "modal_destroy", "modal_set_stream", "modal_status_str",
            "modal_last_error", "modal_set_workspace_limit", "modal_workspace_bytes",
            "modal_enable_timing", "modal_stage_times", "modal_stage_counts", "modal_set_forward_reuse",
            "modal_gauss_legendre",
            "modal_legendre_table", "modal_sph_bessel_table", "modal_beta", "modal_S",
            "modal_gamma_from_S", "modal_gamma", "modal_gram", "modal_gamma_modal",
            "modal_gamma_backward", "modal_r_weights", "modal_gamma_3d", "modal_gamma_noalloc"]


def _ptr(x) -> Optional[int]:
    if x is None:
        return None
    if isinstance(x, torch.Tensor):
        return x.data_ptr()
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    raise TypeError(f"unsupported array type {type(x)}")


class Context:
    """A library context on one device.  Without a stream, every call runs on
    torch's current stream of that device at the time of the call (the
    library is switched to it, ordered after its earlier work, whenever it
    changes); with a stream, always on that one."""

    def __init__(self, device: int = 0, stream: Optional[torch.cuda.Stream] = None):
        L = lib()
        if not torch.cuda.is_available():
            raise ModalError(4, "no HIP device visible to torch")
        self.device = device
        self.forward_reuse = False
        self.torch_device = torch.device("cuda", device)
        self._follow = stream is None
        if stream is None:
            stream = torch.cuda.current_stream(self.torch_device)
        self.stream = stream
        h = ctypes.c_void_p()
        self._check(L.modal_create(ctypes.byref(h), device, ctypes.c_void_p(stream.cuda_stream)), None)
        self._h = h

    @property
    def handle(self):
        """The library handle; every call reaches it through here, so a
        context that follows torch's current stream is switched to it first
        (modal_set_stream orders the new stream after the old one)."""
        h = self._h
        if h is not None and self._follow:
            s = torch.cuda.current_stream(self.torch_device)
            if s.cuda_stream != self.stream.cuda_stream:
                self._check(lib().modal_set_stream(h, ctypes.c_void_p(s.cuda_stream)), h)
                self.stream = s
        return h

    def _check(self, st: int, handle):
        if st != 0:
            L = lib()
            msg = L.modal_last_error(handle).decode() if handle is not None else \
                L.modal_last_error(None).decode()
            raise ModalError(st, msg or L.modal_status_str(st).decode())

    def check(self, st: int):
        self._check(st, self._h)

    def close(self):
        if getattr(self, "_h", None):
            lib().modal_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_workspace_limit(self, nbytes: int):
        self.check(lib().modal_set_workspace_limit(self.handle, nbytes))

    def enable_timing(self, on: bool = True):
        self.check(lib().modal_enable_timing(self.handle, int(on)))

    def set_forward_reuse(self, on: bool = True):
        """Let gamma_backward take the forward tables of the context's previous
        gamma / gamma_backward call on the same projection instead of
        recomputing them; the caller guarantees the inputs are unchanged."""
        self.check(lib().modal_set_forward_reuse(self.handle, int(on)))
        self.forward_reuse = bool(on)

    def stage_times(self) -> dict:
        ms = (ctypes.c_double * len(STAGES))()
        self.check(lib().modal_stage_times(self.handle, ms, len(STAGES)))
        return {name: float(ms[i]) for i, name in enumerate(STAGES)}

    def stage_counts(self) -> dict:
        """Timed intervals per stage of the last call (one per chunk or batch)."""
        n = (ctypes.c_int32 * len(STAGES))()
        self.check(lib().modal_stage_counts(self._h, n, len(STAGES)))
        return {name: int(n[i]) for i, name in enumerate(STAGES)}

    def empty(self, *shape, dtype=torch.float64):
        return torch.empty(*shape, dtype=dtype, device=self.torch_device)

    def to_dev(self, a, dtype=torch.float64):
        if isinstance(a, torch.Tensor):
            return a.to(device=self.torch_device, dtype=dtype).contiguous()
        return torch.as_tensor(np.ascontiguousarray(a)).to(device=self.torch_device, dtype=dtype)


# ---------------------------------------------------------------- stage calls
R_RULES = {"trapezoid": 0, "hermite": 1}


def r_weights(rule, r) -> np.ndarray:
    """Weights of an r rule ("trapezoid" or "hermite", or the enum value) on
    the nodes r, for Grid's wr (host arrays; modal_r_weights)."""
    r = np.ascontiguousarray(r, dtype=np.float64)
    w = np.empty_like(r)
    L = lib()
    code = R_RULES[rule] if isinstance(rule, str) else int(rule)
    st = L.modal_r_weights(code, r.size, r.ctypes.data if r.size else None,
                           w.ctypes.data if w.size else None)
    if st != 0:
        raise ModalError(st, L.modal_last_error(None).decode() or L.modal_status_str(st).decode())
    return w


def gauss_legendre(ctx: Context, n: int):
    x, w = ctx.empty(n), ctx.empty(n)
    ctx.check(lib().modal_gauss_legendre(ctx.handle, n, x.data_ptr(), w.data_ptr()))
    return x, w


def legendre_table(ctx: Context, lmax: int, mu) -> torch.Tensor:
    """P[l][j] = P_l(mu_j), l = 0..lmax."""
    mu = ctx.to_dev(mu)
    P = ctx.empty(lmax + 1, mu.numel())
    ctx.check(lib().modal_legendre_table(ctx.handle, lmax, mu.numel(), mu.data_ptr(), P.data_ptr()))
    return P


def sph_bessel_table(ctx: Context, lmax: int, x) -> torch.Tensor:
    """J[l][i] = j_l(x_i), l = 0..lmax."""
    x = ctx.to_dev(x)
    J = ctx.empty(lmax + 1, x.numel())
    ctx.check(lib().modal_sph_bessel_table(ctx.handle, lmax, x.numel(), x.data_ptr(), J.data_ptr()))
    return J


@dataclass
class Projection:
    """The inputs of one projection, resident on the context's device."""
    ctx: Context
    lmin: int
    lmax: int
    k: torch.Tensor
    wk: torch.Tensor
    r: torch.Tensor
    wr: torch.Tensor
    nmu: int
    delta: torch.Tensor
    cl: torch.Tensor
    qk: torch.Tensor
    ql: torch.Tensor
    tri_a: torch.Tensor
    tri_p: torch.Tensor
    kind: str = "ordered"
    v_power: float = 1.0 / 6.0
    mu: Optional[torch.Tensor] = None
    wmu: Optional[torch.Tensor] = None
    allow_inexact_gl: bool = False

    @classmethod
    def create(cls, ctx: Context, *, lmin, lmax, k, wk, r, wr, nmu, delta, cl, qk, ql, tri_a,
               tri_p, kind="ordered", v_power=1.0 / 6.0, mu=None, wmu=None,
               allow_inexact_gl=False) -> "Projection":
        d = ctx.to_dev
        return cls(ctx, int(lmin), int(lmax), d(k), d(wk), d(r), d(wr), int(nmu), d(delta), d(cl),
                   d(qk), d(ql), d(tri_a, torch.int32), d(tri_p, torch.int32), kind, float(v_power),
                   None if mu is None else d(mu), None if wmu is None else d(wmu),
                   bool(allow_inexact_gl))

    @property
    def L(self) -> int:
        return self.lmax - self.lmin + 1

    @property
    def np_(self) -> int:
        return self.qk.shape[0]

    @property
    def na(self) -> int:
        return self.ql.shape[0]

    @property
    def nr(self) -> int:
        return self.r.numel()

    def versions(self):
        """In-place modification counters of every tensor the projection holds."""
        return tuple(None if t is None else t._version
                     for t in (self.k, self.wk, self.r, self.wr, self.delta, self.cl, self.qk, self.ql,
                               self.tri_a, self.tri_p, self.mu, self.wmu))

    def structs(self):
        g = ModalGrid(self.lmin, self.lmax, self.k.numel(), _ptr(self.k), _ptr(self.wk),
                      self.r.numel(), _ptr(self.r), _ptr(self.wr), self.nmu, _ptr(self.mu),
                      _ptr(self.wmu), int(self.allow_inexact_gl))
        p = ModalProblem(_ptr(self.delta), _ptr(self.cl), self.np_, _ptr(self.qk), self.na,
                         _ptr(self.ql), self.v_power, _KIND[self.kind], self.tri_a.shape[0],
                         _ptr(self.tri_a), self.tri_p.shape[0], _ptr(self.tri_p))
        return g, p

    def workspace_bytes(self, precision: str = "fp64") -> int:
        g, p = self.structs()
        n = ctypes.c_size_t()
        self.ctx.check(lib().modal_workspace_bytes(self.ctx.handle, ctypes.byref(g), ctypes.byref(p),
                                                   _PREC[precision], ctypes.byref(n)))
        return int(n.value)

    def beta(self, precision: str = "fp64") -> torch.Tensor:
        """beta[p][l - lmin][r]."""
        g, p = self.structs()
        out = self.ctx.empty(self.np_, self.L, self.nr)
        self.ctx.check(lib().modal_beta(self.ctx.handle, ctypes.byref(g), ctypes.byref(p),
                                        _PREC[precision], out.data_ptr()))
        return out

    def S(self, beta: torch.Tensor, precision: str = "fp64") -> torch.Tensor:
        """S[a][p][r][mu]."""
        g, p = self.structs()
        beta = self.ctx.to_dev(beta)
        out = self.ctx.empty(self.na, self.np_, self.nr, self.nmu)
        self.ctx.check(lib().modal_S(self.ctx.handle, ctypes.byref(g), ctypes.byref(p),
                                     _PREC[precision], beta.data_ptr(), out.data_ptr()))
        return out

    def gamma_from_S(self, S: torch.Tensor, precision: str = "fp64") -> torch.Tensor:
        g, p = self.structs()
        S = self.ctx.to_dev(S)
        out = self.ctx.empty(self.tri_a.shape[0], self.tri_p.shape[0])
        self.ctx.check(lib().modal_gamma_from_S(self.ctx.handle, ctypes.byref(g), ctypes.byref(p),
                                                _PREC[precision], S.data_ptr(), out.data_ptr()))
        return out

    def gamma(self, precision: str = "fp64", out: Optional[torch.Tensor] = None) -> torch.Tensor:
        g, p = self.structs()
        if out is None:
            out = self.ctx.empty(self.tri_a.shape[0], self.tri_p.shape[0])
        self.ctx.check(lib().modal_gamma(self.ctx.handle, ctypes.byref(g), ctypes.byref(p),
                                         _PREC[precision], out.data_ptr()))
        return out

    def gamma_noalloc(self, precision: str = "fp64", out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """Gamma through modal_gamma_noalloc: no device allocation in the
        library (its buffers come from a fixed per-device scratch array)."""
        g, p = self.structs()
        if out is None:
            out = self.ctx.empty(self.tri_a.shape[0], self.tri_p.shape[0])
        self.ctx.check(lib().modal_gamma_noalloc(self.ctx.handle, ctypes.byref(g), ctypes.byref(p),
                                                 _PREC[precision], out.data_ptr()))
        return out

    def gram(self, precision: str = "fp64") -> torch.Tensor:
        """The late-time Gram matrix <Q_n, Q_m> over tri_a x tri_a."""
        g, p = self.structs()
        out = self.ctx.empty(self.tri_a.shape[0], self.tri_a.shape[0])
        self.ctx.check(lib().modal_gram(self.ctx.handle, ctypes.byref(g), ctypes.byref(p),
                                        _PREC[precision], out.data_ptr()))
        return out

    def gamma_modal(self, precision: str = "fp64") -> torch.Tensor:
        """The full Gamma = <Q, Q>^-1 Gamma' [ta][tp]."""
        g, p = self.structs()
        out = self.ctx.empty(self.tri_a.shape[0], self.tri_p.shape[0])
        self.ctx.check(lib().modal_gamma_modal(self.ctx.handle, ctypes.byref(g), ctypes.byref(p),
                                               _PREC[precision], out.data_ptr()))
        return out

    def gamma_3d(self, threej: str = "exact") -> torch.Tensor:
        """Gamma' of Eq. (3D) [ta][tp]: the direct sum over l-triples with the
        exact ("exact") or Gosper ("gosper") Wigner symbol, FP64."""
        g, p = self.structs()
        out = self.ctx.empty(self.tri_a.shape[0], self.tri_p.shape[0])
        self.ctx.check(lib().modal_gamma_3d(self.ctx.handle, ctypes.byref(g), ctypes.byref(p),
                                            {"exact": 0, "gosper": 1}[threej], out.data_ptr()))
        return out

    def gamma_backward(self, dgamma: torch.Tensor, precision: str = "fp64", want_q: bool = True,
                       want_delta: bool = True):
        """(dL/dq [np][nk], dL/ddelta [L][nk]) for dL/dGamma = dgamma."""
        g, p = self.structs()
        dgamma = self.ctx.to_dev(dgamma)
        dq = self.ctx.empty(self.np_, self.k.numel()) if want_q else None
        dd = self.ctx.empty(self.L, self.k.numel()) if want_delta else None
        self.ctx.check(lib().modal_gamma_backward(self.ctx.handle, ctypes.byref(g), ctypes.byref(p),
                                                  _PREC[precision], dgamma.data_ptr(),
                                                  _ptr(dq), _ptr(dd)))
        return dq, dd


class ModalProjectionFunction(torch.autograd.Function):
    """Gamma as a differentiable function of (q_p(k), Delta_l(k)); the
    backward runs the library's adjoint (modal_gamma_backward)."""

    @staticmethod
    def forward(ctx, qk, delta, proj, precision):
        p2 = dataclasses.replace(proj, qk=qk.detach().contiguous(), delta=delta.detach().contiguous())
        ctx.proj = p2
        ctx.precision = precision
        out = p2.gamma(precision)
        ctx.versions = p2.versions()
        return out

    @staticmethod
    def backward(ctx, dgamma):
        # the library may reuse this forward's tables only if no input has
        # been modified in place since (it checks that no other call came
        # between, and recomputes otherwise)
        lc = ctx.proj.ctx
        before = getattr(lc, "forward_reuse", False)
        lc.set_forward_reuse(ctx.proj.versions() == ctx.versions)
        try:
            dq, dd = ctx.proj.gamma_backward(dgamma.contiguous(), ctx.precision,
                                             want_q=ctx.needs_input_grad[0],
                                             want_delta=ctx.needs_input_grad[1])
        finally:
            lc.set_forward_reuse(before)
        return dq, dd, None, None


def projection_from_inputs(ctx: Context, inp, **over) -> Projection:
    """A Projection from a seeded-input bundle (fields k, wk, r, wr, cl,
    delta, qk, ql, tri_a, tri_p and a cfg with lmin, lmax, nmu, kind,
    v_power)."""
    c = inp.cfg
    kw = dict(lmin=c.lmin, lmax=c.lmax, k=inp.k, wk=inp.wk, r=inp.r, wr=inp.wr, nmu=c.nmu,
              delta=inp.delta, cl=inp.cl, qk=inp.qk, ql=inp.ql, tri_a=inp.tri_a, tri_p=inp.tri_p,
              kind=c.kind, v_power=c.v_power)
    kw.update(over)
    return Projection.create(ctx, **kw)
