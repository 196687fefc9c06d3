"""Python binding of libcrk.so: argument marshalling only.

Every step of the CRKSPH path runs inside libcrk.so (HIP kernels for
gfx950). PyTorch supplies device memory and the current stream. There is no
fallback: if the library or a HIP device is missing, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass, replace

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcrk.so")

CUBIC_SPLINE, WENDLAND_C4 = 0, 1
FP32, FP64 = 0, 1

STATUS = {0: "CRK_OK", -1: "CRK_EINVAL", -2: "CRK_ENOMEM", -3: "CRK_EHIP", -4: "CRK_EDOMAIN",
          -5: "CRK_ENOTCONV", -6: "CRK_ENONFINITE"}


class CrkError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


class crk_params(C.Structure):
    _fields_ = [("box", C.c_double), ("gamma", C.c_double), ("alpha", C.c_double),
                ("beta", C.c_double), ("eps2", C.c_double), ("n_h", C.c_double),
                ("kernel", C.c_int), ("precision", C.c_int), ("h_mode", C.c_int),
                ("h_max_iter", C.c_int), ("h_rtol", C.c_double), ("dt_relax", C.c_double),
                ("store_corrections", C.c_int), ("check_finite", C.c_int), ("timing", C.c_int),
                ("search", C.c_int)]


class crk_stats(C.Structure):
    _fields_ = [("n_pairs_gather", C.c_longlong), ("n_pairs_force", C.c_longlong),
                ("h_iter_max", C.c_int), ("h_unconverged", C.c_int), ("m2_singular", C.c_int),
                ("relaxed", C.c_int), ("nonfinite", C.c_int), ("grid", C.c_int),
                ("speculative", C.c_int),
                ("n_candidates", C.c_longlong), ("n_searched", C.c_longlong)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


EXPORTS = ["crk_default_params", "crk_create", "crk_set_params", "crk_reserve", "crk_destroy",
           "crk_last_error", "crk_forward", "crk_backward", "crk_backward_noalloc",
           "crk_pass_count", "crk_pass_name",
           "crk_pass_times", "crk_kdk_step", "crk_hkdk_step", "crk_cooling_table", "crk_cool",
           "crk_deposit"]

_lib = None


def lib():
    """Loads libcrk.so (built by paper_2511_21921_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libcrk.so is not built: run __graft_entry__.build() "
                               "or python paper_2511_21921_amd/build.py")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.crk_default_params.argtypes = [C.POINTER(crk_params), C.c_int]
        L.crk_default_params.restype = None
        L.crk_create.argtypes = [C.POINTER(P), C.POINTER(crk_params)]
        L.crk_create.restype = C.c_int
        L.crk_set_params.argtypes = [P, C.POINTER(crk_params)]
        L.crk_set_params.restype = C.c_int
        L.crk_reserve.argtypes = [P, C.c_longlong]
        L.crk_reserve.restype = C.c_int
        L.crk_destroy.argtypes = [P]
        L.crk_destroy.restype = C.c_int
        L.crk_last_error.argtypes = [P]
        L.crk_last_error.restype = C.c_char_p
        L.crk_forward.argtypes = [P, P, C.c_longlong] + [P] * 14 + [C.POINTER(crk_stats)]
        L.crk_forward.restype = C.c_int
        L.crk_backward.argtypes = [P, P, C.c_longlong] + [P] * 6
        L.crk_backward.restype = C.c_int
        L.crk_backward_noalloc.argtypes = [P, P, C.c_longlong] + [P] * 6
        L.crk_backward_noalloc.restype = C.c_int
        L.crk_kdk_step.argtypes = ([P, P, C.c_longlong, C.c_double, C.c_double] + [P] * 14 +
                                   [C.POINTER(crk_stats)])
        L.crk_kdk_step.restype = C.c_int
        L.crk_hkdk_step.argtypes = ([P, P, C.c_longlong, C.c_double, C.c_double] + [P] * 17 +
                                    [C.POINTER(crk_stats)])
        L.crk_hkdk_step.restype = C.c_int
        L.crk_cooling_table.argtypes = [P, P, C.c_int, C.c_double, C.c_double,
                                        C.POINTER(C.c_double)]
        L.crk_cooling_table.restype = C.c_int
        L.crk_cool.argtypes = [P, P, C.c_longlong, C.c_double, P, P]
        L.crk_cool.restype = C.c_int
        L.crk_deposit.argtypes = ([P, P, C.c_longlong] + [P] * 7 + [C.c_longlong] + [P] * 5
                                  + [C.c_double] * 3 + [P] * 3)
        L.crk_deposit.restype = C.c_int
        L.crk_pass_count.argtypes = []
        L.crk_pass_count.restype = C.c_int
        L.crk_pass_name.argtypes = [C.c_int]
        L.crk_pass_name.restype = C.c_char_p
        L.crk_pass_times.argtypes = [P, C.POINTER(C.c_double), C.POINTER(C.c_longlong), C.c_int]
        L.crk_pass_times.restype = C.c_int
        _lib = L
    return _lib


@dataclass
class Params:
    box: float = 1.0
    gamma: float = 5.0 / 3.0
    alpha: float = 1.0
    beta: float = 2.0
    eps2: float = 0.01
    n_h: float = 2.4814
    kernel: int = CUBIC_SPLINE
    precision: int = FP32
    h_mode: int = 1
    h_max_iter: int = 60
    h_rtol: float | None = None      # default: 1e-6 (FP32) / 1e-13 (FP64)
    dt_relax: float = 0.0
    store_corrections: int = 0
    check_finite: int = 0
    timing: int = 0
    search: int = 0                  # 0 automatic, 1 cell list, 2 tree

    def to_c(self) -> crk_params:
        p = crk_params()
        lib().crk_default_params(C.byref(p), int(self.precision))
        for k, _ in crk_params._fields_:
            val = getattr(self, k)
            if val is not None:
                setattr(p, k, val)
        return p

    @property
    def real(self) -> torch.dtype:
        return torch.float64 if self.precision == FP64 else torch.float32


def _ptr(t: torch.Tensor | None):
    return None if t is None else C.c_void_p(t.data_ptr())


def _check(t: torch.Tensor, dtype, shape, name):
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)


class Context:
    """Owns one crk_ctx (device workspace, cell list and the last forward's state)."""

    def __init__(self, params: Params):
        self.params = params
        self._cp = params.to_c()
        h = C.c_void_p()
        st = lib().crk_create(C.byref(h), C.byref(self._cp))
        if st != 0:
            raise CrkError(st, "crk_create rejected the parameters")
        self._h = h
        self.generation = 0

    def close(self):
        if getattr(self, "_h", None):
            lib().crk_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params: Params):
        cp = params.to_c()
        self._raise(lib().crk_set_params(self._h, C.byref(cp)))
        self.params, self._cp = params, cp
        self.generation += 1  # the library drops the kept state when a parameter changed

    def reserve(self, n: int):
        self._raise(lib().crk_reserve(self._h, int(n)))

    def last_error(self) -> str:
        return lib().crk_last_error(self._h).decode()

    def _raise(self, st: int, allow=()):
        if st != 0 and st not in allow:
            raise CrkError(st, self.last_error())
        return st

    def forward(self, x: torch.Tensor, v: torch.Tensor, m: torch.Tensor, u: torch.Tensor,
                h: torch.Tensor, stats: bool = False, out: dict | None = None) -> dict:
        """Runs the forward passes. x is float64 [3, n]; v [3, n], m, u, h [n] are Real.

        Returns a dict with h, V, rho, A, B, gradA, gradB, gradv (Real), accel,
        dudt (float64) and, if stats is set, the crk_stats fields.
        """
        n = int(m.shape[0])
        R = self.params.real
        dev = x.device
        _check(x, torch.float64, (3, n), "x")
        _check(v, R, (3, n), "v")
        for t, name in [(m, "m"), (u, "u"), (h, "h")]:
            _check(t, R, (n,), name)
        if out is None:
            out = {
                "h": h.clone(), "V": torch.empty(n, dtype=R, device=dev),
                "rho": torch.empty(n, dtype=R, device=dev), "A": torch.empty(n, dtype=R, device=dev),
                "B": torch.empty(3, n, dtype=R, device=dev),
                "gradA": torch.empty(3, n, dtype=R, device=dev),
                "gradB": torch.empty(9, n, dtype=R, device=dev),
                "gradv": torch.empty(9, n, dtype=R, device=dev),
                "accel": torch.empty(3, n, dtype=torch.float64, device=dev),
                "dudt": torch.empty(n, dtype=torch.float64, device=dev)}
        else:
            out["h"].copy_(h)
        st = crk_stats()
        stream = C.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
        self.generation += 1
        rc = lib().crk_forward(self._h, stream, n, _ptr(x), _ptr(v), _ptr(m), _ptr(u),
                               _ptr(out["h"]), _ptr(out["V"]), _ptr(out["rho"]), _ptr(out["A"]),
                               _ptr(out["B"]), _ptr(out["gradA"]), _ptr(out["gradB"]),
                               _ptr(out["gradv"]), _ptr(out["accel"]), _ptr(out["dudt"]),
                               C.byref(st) if stats else None)
        self._raise(rc)
        if stats:
            out["stats"] = st.as_dict()
        return out

    def kdk_step(self, x: torch.Tensor, v: torch.Tensor, m: torch.Tensor, u: torch.Tensor,
                 out: dict, dt: float, lam: float = 0.5, stats: bool = False) -> dict:
        """One kick-drift-kick step (crk_kdk_step): advances x, v, u and out["h"]
        in place by dt and replaces out (the dict of the forward at the current
        state, as returned by forward or kdk_step) by the forward at the new
        state. The context must have h_mode 0."""
        n = int(m.shape[0])
        R = self.params.real
        _check(x, torch.float64, (3, n), "x")
        _check(v, R, (3, n), "v")
        for t, name in [(m, "m"), (u, "u"), (out["h"], "h"), (out["V"], "V")]:
            _check(t, R, (n,), name)
        _check(out["gradv"], R, (9, n), "gradv")
        _check(out["accel"], torch.float64, (3, n), "accel")
        _check(out["dudt"], torch.float64, (n,), "dudt")
        st = crk_stats()
        stream = C.c_void_p(torch.cuda.current_stream(x.device).cuda_stream)
        self.generation += 1
        rc = lib().crk_kdk_step(self._h, stream, n, float(dt), float(lam), _ptr(x), _ptr(v),
                                _ptr(m), _ptr(u), _ptr(out["h"]), _ptr(out["V"]),
                                _ptr(out["rho"]), _ptr(out["A"]), _ptr(out["B"]),
                                _ptr(out["gradA"]), _ptr(out["gradB"]), _ptr(out["gradv"]),
                                _ptr(out["accel"]), _ptr(out["dudt"]),
                                C.byref(st) if stats else None)
        self._raise(rc)
        if stats:
            out["stats"] = st.as_dict()
        return out

    def hkdk_step(self, x: torch.Tensor, v: torch.Tensor, m: torch.Tensor, u: torch.Tensor,
                  out: dict, levels: torch.Tensor, dt: float, lam: float = 0.5,
                  stats: bool = False, refine=None) -> dict:
        """One big step of the power-of-two timestep hierarchy (crk_hkdk_step):
        levels is an int32 device tensor [n]; x, v, u and out are advanced in
        place as in kdk_step, out holding each particle's latest evaluation.
        refine: None, or (refine_at, refine_level) int32 device tensors [n]
        (refine_at -1: no refinement), the timestep refinement of the step."""
        n = int(m.shape[0])
        R = self.params.real
        _check(x, torch.float64, (3, n), "x")
        _check(v, R, (3, n), "v")
        _check(levels, torch.int32, (n,), "levels")
        r_at = r_lev = None
        if refine is not None:
            r_at, r_lev = refine
            _check(r_at, torch.int32, (n,), "refine_at")
            _check(r_lev, torch.int32, (n,), "refine_level")
        for t, name in [(m, "m"), (u, "u"), (out["h"], "h"), (out["V"], "V"),
                        (out["rho"], "rho"), (out["A"], "A")]:
            _check(t, R, (n,), name)
        for k, rows in [("B", 3), ("gradA", 3), ("gradB", 9), ("gradv", 9)]:
            _check(out[k], R, (rows, n), k)
        _check(out["accel"], torch.float64, (3, n), "accel")
        _check(out["dudt"], torch.float64, (n,), "dudt")
        st = crk_stats()
        stream = C.c_void_p(torch.cuda.current_stream(x.device).cuda_stream)
        self.generation += 1
        rc = lib().crk_hkdk_step(self._h, stream, n, float(dt), float(lam), _ptr(levels),
                                 _ptr(r_at), _ptr(r_lev), _ptr(x),
                                 _ptr(v), _ptr(m), _ptr(u), _ptr(out["h"]), _ptr(out["V"]),
                                 _ptr(out["rho"]), _ptr(out["A"]), _ptr(out["B"]),
                                 _ptr(out["gradA"]), _ptr(out["gradB"]), _ptr(out["gradv"]),
                                 _ptr(out["accel"]), _ptr(out["dudt"]),
                                 C.byref(st) if stats else None)
        self._raise(rc)
        if stats:
            out["stats"] = st.as_dict()
        return out

    def cooling_table(self, log10_u0: float, dex: float, lam) -> None:
        """Sets the tabulated source function lam(u_k), u_k = 10^(log10_u0 + k dex)
        of the exact-integration cooling (crk_cooling_table); lam is host data."""
        import numpy as np
        a = np.ascontiguousarray(np.asarray(lam, dtype=np.float64))
        stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
        self._raise(lib().crk_cooling_table(self._h, stream, int(a.size), float(log10_u0),
                                            float(dex),
                                            a.ctypes.data_as(C.POINTER(C.c_double))))

    def cool(self, rho: torch.Tensor, u: torch.Tensor, dt: float) -> torch.Tensor:
        """Integrates du/dt = -rho lam(u) exactly over dt, u in place (crk_cool)."""
        n = int(u.shape[0])
        R = self.params.real
        _check(rho, R, (n,), "rho")
        _check(u, R, (n,), "u")
        stream = C.c_void_p(torch.cuda.current_stream(u.device).cuda_stream)
        self._raise(lib().crk_cool(self._h, stream, n, float(dt), _ptr(rho), _ptr(u)))
        return u

    def deposit(self, gas: dict, src: dict, n_h_src: float, z_max: float = float("inf"),
                m_max: float = float("inf")) -> dict:
        """Subgrid deposition (crk_deposit). gas: x [3][n] float64, h, V [n] and
        m, mZ, u [n], v [3][n] (updated in place); src: x [3][s] float64, dM,
        dMZ, dE [s], v [3][s]. Returns the sources' V, h and A."""
        R = self.params.real
        ng = int(gas["m"].shape[0])
        ns = int(src["dM"].shape[0])
        dev = gas["m"].device
        _check(gas["x"], torch.float64, (3, ng), "gas x")
        for k in ("h", "V", "m", "mZ", "u"):
            _check(gas[k], R, (ng,), "gas " + k)
        _check(gas["v"], R, (3, ng), "gas v")
        _check(src["x"], torch.float64, (3, ns), "source x")
        for k in ("dM", "dMZ", "dE"):
            _check(src[k], R, (ns,), "source " + k)
        _check(src["v"], R, (3, ns), "source v")
        out = {k: torch.empty(ns, dtype=R, device=dev) for k in ("V", "h", "A")}
        stream = C.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
        self._raise(lib().crk_deposit(
            self._h, stream, ng, _ptr(gas["x"]), _ptr(gas["h"]), _ptr(gas["V"]), _ptr(gas["m"]),
            _ptr(gas["v"]), _ptr(gas["mZ"]), _ptr(gas["u"]), ns, _ptr(src["x"]), _ptr(src["dM"]),
            _ptr(src["dMZ"]), _ptr(src["dE"]), _ptr(src["v"]), float(n_h_src), float(z_max),
            float(m_max), _ptr(out["V"]), _ptr(out["h"]), _ptr(out["A"])))
        return out

    def pass_times(self, reset: bool = False) -> dict:
        """Accumulated device time per pass: {name: (total_ms, launches)}."""
        L = lib()
        k = L.crk_pass_count()
        ms = (C.c_double * k)()
        calls = (C.c_longlong * k)()
        self._raise(L.crk_pass_times(self._h, ms, calls, int(reset)))
        return {L.crk_pass_name(i).decode(): (ms[i], calls[i]) for i in range(k)}

    def backward(self, g_accel: torch.Tensor, g_dudt: torch.Tensor,
                 noalloc: bool = False) -> dict:
        """Adjoint of the last forward for L = sum g_accel.accel + sum g_dudt dudt.
        noalloc: crk_backward_noalloc (workspace in the library's static array,
        at most 65,536 particles)."""
        n = int(g_dudt.shape[0])
        dev = g_dudt.device
        _check(g_accel, torch.float64, (3, n), "g_accel")
        _check(g_dudt, torch.float64, (n,), "g_dudt")
        o = {"g_x": torch.empty(3, n, dtype=torch.float64, device=dev),
             "g_v": torch.empty(3, n, dtype=torch.float64, device=dev),
             "g_u": torch.empty(n, dtype=torch.float64, device=dev),
             "g_alpha_beta": torch.empty(2, dtype=torch.float64, device=dev)}
        stream = C.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
        fn = lib().crk_backward_noalloc if noalloc else lib().crk_backward
        rc = fn(self._h, stream, n, _ptr(g_accel), _ptr(g_dudt), _ptr(o["g_x"]), _ptr(o["g_v"]),
                _ptr(o["g_u"]), _ptr(o["g_alpha_beta"]))
        self._raise(rc)
        return o


class CRKSPHFunction(torch.autograd.Function):
    """Differentiable CRKSPH evaluation through libcrk.so.

    apply(x, v, u, alpha_beta, m, h0, context) returns
    (accel, dudt, h, rho, V, A, B, gradA, gradB, gradv). Only accel and dudt
    carry gradients; the backward returns the adjoints of x (float64
    [3, n]), v, u (Real) and alpha_beta (a float64 tensor [2] holding the
    viscosity coefficients). Masses and the first h guess are constants.
    The backward runs on the state the forward left on ``context``; if
    another forward has run on that context since, the forward is first
    repeated from the saved inputs.
    """

    @staticmethod
    def _run(context, x, v, u, ab, m, h0):
        ab = ab.detach().to("cpu", torch.float64)
        context.set_params(replace(context.params, alpha=float(ab[0]), beta=float(ab[1])))
        return context.forward(x.detach().contiguous(), v.detach().contiguous(), m.contiguous(),
                               u.detach().contiguous(), h0.contiguous())

    @staticmethod
    def forward(ctx, x, v, u, alpha_beta, m, h0, context):
        out = CRKSPHFunction._run(context, x, v, u, alpha_beta, m, h0)
        ctx.context = context
        ctx.generation = context.generation
        ctx.save_for_backward(x, v, u, alpha_beta, m, h0)
        nd = [out[k] for k in ("h", "rho", "V", "A", "B", "gradA", "gradB", "gradv")]
        ctx.mark_non_differentiable(*nd)
        return (out["accel"], out["dudt"], *nd)

    @staticmethod
    def backward(ctx, g_accel, g_dudt, *unused):
        context = ctx.context
        x, v, u, ab, m, h0 = ctx.saved_tensors
        if context.generation != ctx.generation:
            CRKSPHFunction._run(context, x, v, u, ab, m, h0)
        n = int(m.shape[0])
        if g_accel is None:
            g_accel = torch.zeros(3, n, dtype=torch.float64, device=x.device)
        if g_dudt is None:
            g_dudt = torch.zeros(n, dtype=torch.float64, device=x.device)
        o = context.backward(g_accel.to(torch.float64).contiguous(),
                             g_dudt.to(torch.float64).contiguous())
        return (o["g_x"], o["g_v"].to(v.dtype), o["g_u"].to(u.dtype),
                o["g_alpha_beta"].to(ab.device, ab.dtype), None, None, None)
