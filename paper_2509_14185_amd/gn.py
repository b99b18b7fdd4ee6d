"""Python binding of the gfx950 Gauss-Newton library (include/gn.h).

Argument marshalling only: device buffers are torch tensors (PyTorch
provides memory and streams); every arithmetic step runs in the HIP kernels
of libgn.so.  There is no CPU fallback: if the library is not built, or no
GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libgn.so")
HEADER = os.path.join(os.path.dirname(_PKG), "include", "gn.h")

GN_OK, GN_ENOTPD, GN_EINVAL, GN_ENOMEM, GN_EDEVICE, GN_ENONFINITE, GN_ESTATE = 0, 1, -1, -2, -3, -4, -5
GN_EREJECTED = 2
EQUATIONS = {"ccf1d": 0, "burgers1d": 1, "ipm2d": 3, "bouss2d": 4}
PRECISIONS = {"fp64": 0, "split32": 1, "int8crt": 2}


class GNError(RuntimeError):
    def __init__(self, status: int, message: str, info: int = 0):
        super().__init__(message)
        self.status = status
        self.info = info


class _Problem(ctypes.Structure):
    _fields_ = [("equation", ctypes.c_int32), ("precision", ctypes.c_int32), ("n_layers", ctypes.c_int32),
                ("widths", ctypes.POINTER(ctypes.c_int32)), ("lam", ctypes.c_double),
                ("c_norm", ctypes.c_double), ("c_target", ctypes.c_double), ("row_chunk", ctypes.c_int64),
                ("n_fourier", ctypes.c_int32), ("fourier_b", ctypes.POINTER(ctypes.c_double))]


class _Stats(ctypes.Structure):
    _fields_ = [("half_sq_norm", ctypes.c_double), ("max_abs_R", ctypes.c_double),
                ("max_abs_R_val", ctypes.c_double), ("grad_dot_delta", ctypes.c_double),
                ("model_sq_norm", ctypes.c_double), ("chol_info", ctypes.c_int64),
                ("status", ctypes.c_int32), ("updated", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class _LM(ctypes.Structure):
    _fields_ = [("mu", ctypes.c_double), ("mu_min", ctypes.c_double), ("mu_max", ctypes.c_double),
                ("up", ctypes.c_double), ("down", ctypes.c_double), ("rho_lo", ctypes.c_double),
                ("rho_hi", ctypes.c_double), ("max_tries", ctypes.c_int32), ("tries", ctypes.c_int32),
                ("rho", ctypes.c_double), ("half_sq_norm_new", ctypes.c_double)]


class _R1Args(ctypes.Structure):
    _fields_ = [("beta", ctypes.c_double), ("gamma", ctypes.c_double), ("refactor", ctypes.c_int32),
                ("momentum", ctypes.c_int32)]


class _R1Stats(ctypes.Structure):
    _fields_ = [("half_sq_norm", ctypes.c_double), ("max_abs_R", ctypes.c_double),
                ("max_abs_R_val", ctypes.c_double), ("alpha", ctypes.c_double), ("mu", ctypes.c_double),
                ("model", ctypes.c_double), ("chol_info", ctypes.c_int64), ("used_momentum", ctypes.c_int32),
                ("status", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# Levenberg-Marquardt constants used when the caller gives none
LM_DEFAULTS = dict(mu_min=1e-12, mu_max=1e12, up=2.0, down=3.0, rho_lo=0.25, rho_hi=0.75, max_tries=20)

_lib = None
_VP = ctypes.c_void_p
_I64 = ctypes.c_int64
_D = ctypes.c_double


def exported_names():
    """Function names declared in include/gn.h."""
    return re.findall(r"^\w[\w\s\*]*?\b(gn_\w+)\s*\(", open(HEADER).read(), flags=re.M)


def load():
    """Load libgn.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2509_14185_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    sig = {
        "gn_status_string": (ctypes.c_char_p, [ctypes.c_int32]),
        "gn_last_error": (ctypes.c_char_p, [_VP]),
        "gn_create": (ctypes.c_int, [ctypes.POINTER(_Problem), ctypes.POINTER(_VP)]),
        "gn_destroy": (ctypes.c_int, [_VP]),
        "gn_set_stream": (ctypes.c_int, [_VP, _VP]),
        "gn_set_points": (ctypes.c_int, [_VP, _I64, _VP, _VP, _VP, _I64, _VP, _VP, _I64, _VP]),
        "gn_set_points_2d": (ctypes.c_int, [_VP, _I64, _VP, _I64, _VP, _I64, _VP, _I64, _VP]),
        "gn_set_points_ex": (ctypes.c_int, [_VP, _I64, _VP, _VP, _VP, _I64, _VP, _VP, _I64, _VP, _I64, _VP, _I64, _VP,
                                            _D, _D]),
        "gn_num_params": (_I64, [_VP]),
        "gn_num_rows": (_I64, [_VP]),
        "gn_residual": (ctypes.c_int, [_VP, _VP, _VP]),
        "gn_jacobian": (ctypes.c_int, [_VP, _VP, _VP, _I64, _VP]),
        "gn_gram": (ctypes.c_int, [_VP, _VP, _I64, _I64, _I64, _VP, _VP, _I64, _VP]),
        "gn_solve": (ctypes.c_int, [_VP, _VP, _I64, _I64, _D, _VP, _VP, ctypes.POINTER(_I64)]),
        "gn_solve_noalloc": (ctypes.c_int, [_VP, _VP, _I64, _I64, _D, _VP, _VP, ctypes.POINTER(_I64)]),
        "gn_step": (ctypes.c_int, [_VP, _VP, _D, ctypes.POINTER(_Stats)]),
        "gn_step_lm": (ctypes.c_int, [_VP, _VP, ctypes.POINTER(_LM), ctypes.POINTER(_Stats)]),
        "gn_step_rank1": (ctypes.c_int, [_VP, _VP, _VP, _I64, _VP, _VP, ctypes.POINTER(_R1Args),
                                         ctypes.POINTER(_R1Stats)]),
        "gn_eval": (ctypes.c_int, [_VP, _VP, ctypes.POINTER(_Stats)]),
        "gn_lambda_estimate": (ctypes.c_int, [_VP, _VP, ctypes.POINTER(_D), ctypes.POINTER(_D)]),
        "gn_funnel_residual": (ctypes.c_int, [_VP, _VP, _D, ctypes.POINTER(_D), ctypes.POINTER(_D)]),
        "gn_eval_derivs": (ctypes.c_int, [_VP, _VP, ctypes.POINTER(_D), ctypes.POINTER(_D)]),
        "gn_fields": (ctypes.c_int, [_VP, _VP, ctypes.c_int32, _VP, _VP, _VP]),
        "gn_set_stage1": (ctypes.c_int, [_VP, _D, _VP, _VP, _VP, _VP, _VP, _VP]),
        "gn_vjp": (ctypes.c_int, [_VP, _VP, _VP, _VP]),
        "gn_batch_create": (ctypes.c_int, [ctypes.POINTER(_VP), ctypes.c_int32, _VP, ctypes.POINTER(_VP)]),
        "gn_batch_destroy": (ctypes.c_int, [_VP]),
        "gn_step_batched": (ctypes.c_int, [_VP, ctypes.POINTER(_VP), _D, ctypes.POINTER(_Stats)]),
        "gn_int8_crt_params": (ctypes.c_int, [_I64, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                              ctypes.POINTER(ctypes.c_int32)]),
        "gn_probe_fp64_mfma": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_double)]),
        "gn_profile_enable": (ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int32]),
        "gn_profile_read": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_double), ctypes.c_int32,
                                           ctypes.POINTER(ctypes.c_int32)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def int8_crt_params(m: int):
    """Bits kept per column and the moduli of the GN_INT8_CRT Gram for m rows
    (host-only; see gn_int8_crt_params)."""
    lib = load()
    bits, n = ctypes.c_int32(), ctypes.c_int32()
    mods = (ctypes.c_int32 * 32)()
    st = lib.gn_int8_crt_params(int(m), ctypes.byref(bits), ctypes.byref(n), mods)
    if st != 0:
        raise GNError(st, lib.gn_status_string(st).decode())
    return bits.value, [mods[i] for i in range(n.value)]


def probe_fp64_mfma(stream=None):
    """Measured FP64 matrix-instruction throughput (TFLOP/s) of the current
    device (gn_probe_fp64_mfma)."""
    lib = load()
    out = ctypes.c_double(0.0)
    st = torch.cuda.current_stream().cuda_stream if stream is None else stream
    rc = lib.gn_probe_fp64_mfma(ctypes.c_void_p(st), ctypes.byref(out))
    if rc != 0:
        raise GNError(rc, "gn_probe_fp64_mfma failed")
    return out.value


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def solve_noalloc(G, mu, g, delta=None, stream=None):
    """gn_solve_noalloc: (G + mu I) delta = -g without a handle or any
    allocation in the library (G's lower triangle is overwritten by L).
    delta may be given (then nothing is allocated here either).  Returns
    (delta, info); raises GNError on a non-OK status."""
    lib = load()
    p = G.shape[0]
    assert G.stride(1) == 1 and G.dtype == torch.float64
    if delta is None:
        delta = torch.empty(p, dtype=torch.float64, device=G.device)
    st = torch.cuda.current_stream(G.device).cuda_stream if stream is None else stream
    info = _I64(0)
    rc = lib.gn_solve_noalloc(ctypes.c_void_p(st), _ptr(G), p, G.stride(0), float(mu), _ptr(g), _ptr(delta),
                              ctypes.byref(info))
    if rc != 0:
        raise GNError(rc, "gn_solve_noalloc: " + lib.gn_last_error(None).decode(), int(info.value))
    return delta, int(info.value)


def _dev(x, device):
    """FP64 contiguous device tensor (copies numpy / host tensors)."""
    if x is None:
        return None
    if isinstance(x, np.ndarray):
        x = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64))
    return x.to(device=device, dtype=torch.float64).contiguous()


class Problem:
    """One profile problem bound to a gn handle on the current CUDA (HIP) device."""

    def __init__(self, equation: str, widths, lam: float, c_norm: float = 1.0, c_target: float = 1.0,
                 precision: str = "fp64", device: str = "cuda", row_chunk: int = 0, fourier_b=None):
        """fourier_b: frequencies of Fourier input features (1D second stage;
        widths[0] must be 2 len(fourier_b))."""
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the gn library runs only on the GPU")
        self.lib = load()
        self.device = torch.device(device)
        self.widths = [int(w) for w in widths]
        self._w = (ctypes.c_int32 * len(self.widths))(*self.widths)
        nf = 0 if fourier_b is None else len(fourier_b)
        self._fb = (ctypes.c_double * max(nf, 1))(*([float(x) for x in fourier_b] if nf else [0.0]))
        prob = _Problem(EQUATIONS[equation], PRECISIONS[precision], len(self.widths) - 1, self._w,
                        float(lam), float(c_norm), float(c_target), int(row_chunk), nf,
                        ctypes.cast(self._fb, ctypes.POINTER(ctypes.c_double)) if nf else None)
        h = _VP()
        with torch.cuda.device(self.device):
            st = self.lib.gn_create(ctypes.byref(prob), ctypes.byref(h))
        if st != GN_OK:
            raise GNError(st, f"gn_create failed: {self.lib.gn_status_string(st).decode()}")
        self.h = h
        self.P = int(self.lib.gn_num_params(h))
        self._keep = []

    def close(self):
        if getattr(self, "h", None):
            self.lib.gn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ helpers
    def _bind(self):
        self.lib.gn_set_stream(self.h, ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream))

    def _check(self, st, what, info=0):
        if st != GN_OK:
            msg = self.lib.gn_last_error(self.h).decode()
            raise GNError(st, f"{what}: {self.lib.gn_status_string(st).decode()} ({msg})", info)

    @property
    def m(self) -> int:
        return int(self.lib.gn_num_rows(self.h))

    # ------------------------------------------------------------ ABI calls
    def set_points(self, s, rho=None, f=None, sq=None, wq=None, sval=None, s1=None, s2=None, c_d1=1.0, c_d2=1.0):
        """1D point sets; s1 / s2 (optional) add d1 / d2 derivative rows
        (gn_set_points_ex) with loss weights c_d1 / c_d2."""
        self._bind()
        s, rho, f, sq, wq, sval, s1, s2 = (_dev(x, self.device) for x in (s, rho, f, sq, wq, sval, s1, s2))
        n = s.numel()
        mq = 0 if sq is None else sq.numel()
        nv = 0 if sval is None else sval.numel()
        n1 = 0 if s1 is None else s1.numel()
        n2 = 0 if s2 is None else s2.numel()
        if n1 or n2:
            st = self.lib.gn_set_points_ex(self.h, n, _ptr(s), _ptr(rho), _ptr(f), mq, _ptr(sq), _ptr(wq), nv,
                                           _ptr(sval), n1, _ptr(s1), n2, _ptr(s2), float(c_d1), float(c_d2))
            self._check(st, "gn_set_points_ex")
        else:
            st = self.lib.gn_set_points(self.h, n, _ptr(s), _ptr(rho), _ptr(f), mq, _ptr(sq), _ptr(wq), nv,
                                        _ptr(sval))
            self._check(st, "gn_set_points")
        self.n = n
        self.nv = nv

    def set_points_2d(self, s, s1=None, se=None, sval=None):
        """2D point sets: s (n,2), s1 (n1,2) d1 points, se (ne,) y2 = 0 points, sval (nv,2)."""
        self._bind()
        s, s1, se, sval = (_dev(x, self.device) for x in (s, s1, se, sval))
        n = s.numel() // 2
        n1 = 0 if s1 is None else s1.numel() // 2
        ne = 0 if se is None else se.numel()
        nv = 0 if sval is None else sval.numel() // 2
        st = self.lib.gn_set_points_2d(self.h, n, _ptr(s), n1, _ptr(s1) if n1 else None, ne,
                                       _ptr(se) if ne else None, nv, _ptr(sval) if nv else None)
        self._check(st, "gn_set_points_2d")
        self.n = n

    def residual(self, theta, out=None):
        self._bind()
        r = out if out is not None else torch.empty(self.m, dtype=torch.float64, device=self.device)
        self._check(self.lib.gn_residual(self.h, _ptr(theta), _ptr(r)), "gn_residual")
        return r

    def jacobian(self, theta, ld=None, with_r=True):
        self._bind()
        ld = self.P if ld is None else ld
        J = torch.empty((self.m, ld), dtype=torch.float64, device=self.device)
        r = torch.empty(self.m, dtype=torch.float64, device=self.device) if with_r else None
        self._check(self.lib.gn_jacobian(self.h, _ptr(theta), _ptr(J), ld, _ptr(r)), "gn_jacobian")
        return J[:, :self.P], r

    def gram(self, J, r=None, ldG=None):
        """Lower triangle of J^T J (upper triangle left zero) and J^T r."""
        self._bind()
        m, p = J.shape
        ldJ = J.stride(0)
        assert J.stride(1) == 1 and J.dtype == torch.float64
        ldG = p if ldG is None else ldG
        G = torch.zeros((p, ldG), dtype=torch.float64, device=self.device)
        g = torch.empty(p, dtype=torch.float64, device=self.device) if r is not None else None
        st = self.lib.gn_gram(self.h, _ptr(J), m, p, ldJ, _ptr(r), _ptr(G), ldG, _ptr(g))
        self._check(st, "gn_gram")
        return G[:, :p], g

    def solve(self, G, mu, g):
        """(G + mu I) delta = -g; G (lower triangle used) is overwritten by L."""
        self._bind()
        p = G.shape[0]
        assert G.stride(1) == 1
        delta = torch.empty(p, dtype=torch.float64, device=self.device)
        info = _I64(0)
        st = self.lib.gn_solve(self.h, _ptr(G), p, G.stride(0), float(mu), _ptr(g), _ptr(delta), ctypes.byref(info))
        self._check(st, "gn_solve", info.value)
        return delta, int(info.value)

    def step(self, theta, mu, stats=True):
        self._bind()
        s = _Stats()
        st = self.lib.gn_step(self.h, _ptr(theta), float(mu), ctypes.byref(s) if stats else None)
        if stats:
            d = s.as_dict()
            d["rc"] = st
            return d
        self._check(st, "gn_step")
        return None

    def step_lm(self, theta, mu, **kw):
        """One step with Levenberg-Marquardt damping (gn_step_lm); theta updated
        in place on acceptance.  Keyword constants default to LM_DEFAULTS.
        Returns the stats dict plus rc, mu (damping for the next step), tries,
        rho and half_sq_norm_new."""
        self._bind()
        o = dict(LM_DEFAULTS)
        o.update(kw)
        lm = _LM(mu=float(mu), mu_min=float(o["mu_min"]), mu_max=float(o["mu_max"]), up=float(o["up"]),
                 down=float(o["down"]), rho_lo=float(o["rho_lo"]), rho_hi=float(o["rho_hi"]),
                 max_tries=int(o["max_tries"]))
        s = _Stats()
        st = self.lib.gn_step_lm(self.h, _ptr(theta), ctypes.byref(lm), ctypes.byref(s))
        if st not in (GN_OK, GN_EREJECTED, GN_ENONFINITE):
            self._check(st, "gn_step_lm")
        d = s.as_dict()
        d.update(rc=st, mu=lm.mu, tries=lm.tries, rho=lm.rho, half_sq_norm_new=lm.half_sq_norm_new)
        return d

    def step_rank1(self, theta, G_ema, prev, v, beta, gamma, refactor=True, momentum=True):
        """One stochastic full-matrix GN step (gn_step_rank1).  theta, G_ema
        (P x P, lower triangle, ldG = G_ema.stride(0)) and prev are updated in
        place; v holds the m probe values.  Returns the stats dict plus rc;
        raises on argument and runtime errors."""
        self._bind()
        assert G_ema.dtype == torch.float64 and G_ema.stride(1) == 1
        a = _R1Args(beta=float(beta), gamma=float(gamma), refactor=int(bool(refactor)), momentum=int(bool(momentum)))
        s = _R1Stats()
        st = self.lib.gn_step_rank1(self.h, _ptr(theta), _ptr(G_ema), int(G_ema.stride(0)), _ptr(prev),
                                    _ptr(v.contiguous()), ctypes.byref(a), ctypes.byref(s))
        if st not in (GN_OK, GN_ENOTPD, GN_ENONFINITE):
            self._check(st, "gn_step_rank1")
        d = s.as_dict()
        d["rc"] = st
        return d

    def fields(self, theta, which=0):
        """(R, V, Theta') of this first stage at the collocation points (which = 0)
        or the validation grid (which = 1), gn_fields."""
        self._bind()
        n = self.n if which == 0 else self.nv
        R, V, T = (torch.empty(n, dtype=torch.float64, device=self.device) for _ in range(3))
        self._check(self.lib.gn_fields(self.h, _ptr(theta), int(which), _ptr(R), _ptr(V), _ptr(T)), "gn_fields")
        return R, V, T

    def set_stage1(self, eps, R, V, Ty, Rv=None, Vv=None, Tyv=None):
        """Second stage around a fixed first stage (gn_set_stage1)."""
        self._bind()
        R, V, Ty, Rv, Vv, Tyv = (_dev(x, self.device) for x in (R, V, Ty, Rv, Vv, Tyv))
        self._keep_stage1 = (R, V, Ty, Rv, Vv, Tyv)
        self._check(self.lib.gn_set_stage1(self.h, float(eps), _ptr(R), _ptr(V), _ptr(Ty), _ptr(Rv), _ptr(Vv),
                                           _ptr(Tyv)), "gn_set_stage1")

    def eval_derivs(self, theta):
        """(max |R'|, max |R''|) on the validation grid (gn_eval_derivs, 1D)."""
        self._bind()
        a, b = _D(), _D()
        self._check(self.lib.gn_eval_derivs(self.h, _ptr(theta), ctypes.byref(a), ctypes.byref(b)), "gn_eval_derivs")
        return a.value, b.value

    def lambda_estimate(self, theta):
        """(lambda_hat, U'(0)) implied at the origin (gn_lambda_estimate, 1D CCF)."""
        self._bind()
        lam, du = _D(), _D()
        self._check(self.lib.gn_lambda_estimate(self.h, _ptr(theta), ctypes.byref(lam), ctypes.byref(du)),
                    "gn_lambda_estimate")
        return lam.value, du.value

    def funnel_residual(self, theta, y_max=1.0):
        """(r_hat, y_at): the validation residual of largest magnitude, with its
        sign, over the points with y <= y_max (gn_funnel_residual)."""
        self._bind()
        r, y = _D(), _D()
        self._check(self.lib.gn_funnel_residual(self.h, _ptr(theta), float(y_max), ctypes.byref(r), ctypes.byref(y)),
                    "gn_funnel_residual")
        return r.value, y.value

    def eval(self, theta):
        self._bind()
        s = _Stats()
        self._check(self.lib.gn_eval(self.h, _ptr(theta), ctypes.byref(s)), "gn_eval")
        return s.as_dict()

    def vjp(self, theta, v):
        self._bind()
        out = torch.empty(self.P, dtype=torch.float64, device=self.device)
        self._check(self.lib.gn_vjp(self.h, _ptr(theta), _ptr(v.contiguous()), _ptr(out)), "gn_vjp")
        return out


PHASES = ["forward", "jacobian_local", "coupling", "gram", "cholesky", "solve"]


def _profile_methods():
    def profile_enable(self, enable=True, max_steps=1024):
        self._bind()
        self._check(self.lib.gn_profile_enable(self.h, int(bool(enable)), int(max_steps)), "gn_profile_enable")

    def profile_read(self):
        ms = (ctypes.c_double * len(PHASES))()
        n = ctypes.c_int32(0)
        self._check(self.lib.gn_profile_read(self.h, ms, len(PHASES), ctypes.byref(n)), "gn_profile_read")
        return {k: ms[i] for i, k in enumerate(PHASES)}, int(n.value)

    return profile_enable, profile_read


Problem.profile_enable, Problem.profile_read = _profile_methods()


class Batch:
    """Independent problems with equal widths stepped together (gn_step_batched).

    The problems must have their points set; calling set_points on one of
    them afterwards makes the batch stale (GN_ESTATE)."""

    def __init__(self, problems):
        self.problems = list(problems)
        if not self.problems:
            raise ValueError("empty batch")
        self.lib = self.problems[0].lib
        self.device = self.problems[0].device
        hs = (_VP * len(self.problems))(*[p.h.value for p in self.problems])
        b = _VP()
        st = self.lib.gn_batch_create(hs, len(self.problems),
                                      ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream),
                                      ctypes.byref(b))
        if st != GN_OK:
            raise GNError(st, f"gn_batch_create: {self.lib.gn_status_string(st).decode()}")
        self.b = b

    def __len__(self):
        return len(self.problems)

    def step(self, thetas, mu, stats=True):
        """One damped GN step of every instance; thetas updated in place.
        Returns a list of per-instance stats dicts (rc = per-instance status)."""
        if len(thetas) != len(self.problems):
            raise ValueError("one parameter vector per instance")
        for t, p in zip(thetas, self.problems):
            assert t.dtype == torch.float64 and t.is_contiguous() and t.numel() == p.P
        ptrs = (_VP * len(thetas))(*[t.data_ptr() for t in thetas])
        out = (_Stats * len(thetas))() if stats else None
        st = self.lib.gn_step_batched(self.b, ptrs, float(mu), out)
        if st != GN_OK:
            raise GNError(st, f"gn_step_batched: {self.lib.gn_status_string(st).decode()}")
        if not stats:
            return None
        res = []
        for s in out:
            d = s.as_dict()
            d["rc"] = d["status"]
            res.append(d)
        return res

    def close(self):
        if getattr(self, "b", None):
            self.lib.gn_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class ResidualFunction(torch.autograd.Function):
    """r(theta) with backward J^T grad_r; activations are recomputed in backward."""

    @staticmethod
    def forward(ctx, theta, problem):
        ctx.problem = problem
        ctx.save_for_backward(theta)
        return problem.residual(theta.detach().contiguous())

    @staticmethod
    def backward(ctx, grad_r):
        (theta,) = ctx.saved_tensors
        return ctx.problem.vjp(theta.detach().contiguous(), grad_r.to(torch.float64)), None


def residual(theta, problem):
    return ResidualFunction.apply(theta, problem)
