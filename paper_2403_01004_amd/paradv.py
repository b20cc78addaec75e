"""ctypes binding of the C ABI in include/paradv.h (argument marshalling only).

Every function of the ABI is exposed under its C name (pa_init, pa_apply,
pa_advance_rkl2, ...); `Operator` wraps one context around torch device
tensors (PyTorch provides device memory and the stream; all arithmetic runs
in the library's HIP kernels).  Loading fails loudly when the library is
missing or no GPU is present -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libparadv.so")
PA_MAX_LOG = 4096
PA_PCG_XGROUP = 8

PA_OK, PA_ERR_ARG, PA_ERR_ALLOC, PA_ERR_HIP, PA_ERR_NOCONV, PA_ERR_BREAKDOWN, \
    PA_ERR_NONFINITE, PA_ERR_STATE, PA_ERR_MAXCYCLES = range(9)
STATUS_NAMES = {0: "PA_OK", 1: "PA_ERR_ARG", 2: "PA_ERR_ALLOC", 3: "PA_ERR_HIP",
                4: "PA_ERR_NOCONV", 5: "PA_ERR_BREAKDOWN", 6: "PA_ERR_NONFINITE",
                7: "PA_ERR_STATE", 8: "PA_ERR_MAXCYCLES"}
OPS = {"iso7": 0, "aligned": 1, "viscv": 2}
BCS = {"dirichlet": 0, "noflux": 1}
PRECS = {"fp64": 0, "fp32": 1}

EXPORTS = ["pa_init", "pa_destroy", "pa_last_error", "pa_default_options", "pa_set_options",
           "pa_bind_field", "pa_set_profile", "pa_set_coefficients", "pa_set_bc", "pa_dt_explicit",
           "pa_apply",
           "pa_diag", "pa_compute_ptl", "pa_compute_ptl_full", "pa_advance_rkl2", "pa_advance_rkg2",
           "pa_advance_be_pcg", "pa_lpc_default_train_opts", "pa_lpc_set_weights",
           "pa_lpc_get_weights", "pa_lpc_features", "pa_lpc_apply", "pa_lpc_loss_grad",
           "pa_lpc_train", "pa_bilu0_apply", "pa_compute_ptl_noalloc"]
PA_LPC_NPARAM = 10832
PCS = {"jacobi": 0, "learned": 1, "bilu0": 2}
PA_BILU0_BOX = (8, 4, 16)   # block ILU(0) boxes in cells along r, theta, phi

_ALLOC = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class pa_desc(ctypes.Structure):
    _fields_ = [("nr", ctypes.c_int32), ("nt", ctypes.c_int32), ("np", ctypes.c_int32),
                ("ncomp", ctypes.c_int32),
                ("r_faces", ctypes.POINTER(ctypes.c_double)),
                ("t_faces", ctypes.POINTER(ctypes.c_double)),
                ("p_faces", ctypes.POINTER(ctypes.c_double)),
                ("op", ctypes.c_int32), ("bc_in", ctypes.c_int32), ("bc_out", ctypes.c_int32),
                ("prec", ctypes.c_int32),
                ("alloc", _ALLOC), ("free", _FREE), ("alloc_user", ctypes.c_void_p)]


class pa_opts(ctypes.Structure):
    _fields_ = [("force_odd", ctypes.c_int32), ("s_override", ctypes.c_int32),
                ("pc", ctypes.c_int32), ("max_iter", ctypes.c_int32),
                ("max_cycles", ctypes.c_int32), ("force_iters", ctypes.c_int32),
                ("pcg_batch", ctypes.c_int32), ("replay_n", ctypes.c_int32),
                ("replay_dt", ctypes.POINTER(ctypes.c_double)), ("ptl_floor", ctypes.c_double),
                ("timing", ctypes.c_int32)]


PA_NKCLASS = 9
KERNEL_CLASSES = ["first", "stage", "matvec", "update", "dir", "init", "reduce", "other", "nn"]


class pa_stats(ctypes.Structure):
    _fields_ = [("cycles", ctypes.c_int32), ("s_total", ctypes.c_int32),
                ("s_max", ctypes.c_int32), ("iters_total", ctypes.c_int32),
                ("iters_max", ctypes.c_int32), ("fallbacks", ctypes.c_int32),
                ("floored", ctypes.c_int32), ("status", ctypes.c_int32),
                ("k_first", ctypes.c_int64), ("dt_explicit", ctypes.c_double),
                ("dt_ptl_first", ctypes.c_double), ("dt_ptl_min", ctypes.c_double),
                ("rel_residual", ctypes.c_double), ("ms_total", ctypes.c_double),
                ("kernel_ms", ctypes.c_double * PA_NKCLASS),
                ("kernel_calls", ctypes.c_int32 * PA_NKCLASS),
                ("dt_cycle", ctypes.c_double * PA_MAX_LOG),
                ("per_cycle", ctypes.c_int32 * PA_MAX_LOG),
                ("jacobi_rows", ctypes.c_int32)]


class pa_lpc_train_opts(ctypes.Structure):
    _fields_ = [("nsnap", ctypes.c_int32), ("batch", ctypes.c_int32),
                ("epochs", ctypes.c_int32), ("seed", ctypes.c_int32),
                ("lr", ctypes.c_double), ("tol_star", ctypes.c_double)]


class pa_lpc_report(ctypes.Structure):
    _fields_ = [("pairs", ctypes.c_int32), ("snapshots", ctypes.c_int32),
                ("steps", ctypes.c_int32), ("ref_iters", ctypes.c_int32),
                ("loss_first", ctypes.c_double), ("loss_last", ctypes.c_double),
                ("ms_pairs", ctypes.c_double), ("ms_train", ctypes.c_double)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libparadv.so and declare the ABI; raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run paper_2403_01004_amd/build.py "
                          "(there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    P, D, I32, I64, V = (ctypes.POINTER, ctypes.c_double, ctypes.c_int32, ctypes.c_int64,
                         ctypes.c_void_p)
    sig = {
        "pa_init": (I32, [P(pa_desc), V, P(V)]),
        "pa_destroy": (None, [V]),
        "pa_last_error": (ctypes.c_char_p, [V]),
        "pa_default_options": (None, [P(pa_opts)]),
        "pa_set_options": (I32, [V, P(pa_opts)]),
        "pa_bind_field": (I32, [V, V]),
        "pa_set_coefficients": (I32, [V, V, D, D, V]),
        "pa_set_profile": (I32, [V, V, V, D]),
        "pa_set_bc": (I32, [V, V, V]),
        "pa_dt_explicit": (I32, [V, P(D)]),
        "pa_apply": (I32, [V, V, V, I32]),
        "pa_diag": (I32, [V, V]),
        "pa_compute_ptl": (I32, [V, P(D), P(I64)]),
        "pa_compute_ptl_full": (I32, [V, P(D), P(I64)]),
        "pa_compute_ptl_noalloc": (I32, [V, P(D), P(I64)]),
        "pa_bilu0_apply": (I32, [V, D, V, V]),
        "pa_advance_rkl2": (I32, [V, D, I32, P(pa_stats)]),
        "pa_advance_rkg2": (I32, [V, D, I32, P(pa_stats)]),
        "pa_advance_be_pcg": (I32, [V, D, D, I32, P(pa_stats)]),
        "pa_lpc_default_train_opts": (None, [P(pa_lpc_train_opts)]),
        "pa_lpc_set_weights": (I32, [V, V]),
        "pa_lpc_get_weights": (I32, [V, V]),
        "pa_lpc_features": (I32, [V, D, V, V]),
        "pa_lpc_apply": (I32, [V, D, V, V]),
        "pa_lpc_loss_grad": (I32, [V, D, I32, V, V, P(D), V]),
        "pa_lpc_train": (I32, [V, D, P(pa_lpc_train_opts), P(pa_lpc_report)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


# ---- the ABI under its own names -------------------------------------------

def pa_init(desc, stream=None):
    ctx = ctypes.c_void_p()
    st = load().pa_init(ctypes.byref(desc), stream, ctypes.byref(ctx))
    return st, ctx


def pa_destroy(ctx):
    load().pa_destroy(ctx)


def pa_last_error(ctx):
    return load().pa_last_error(ctx).decode()


def pa_default_options():
    o = pa_opts()
    load().pa_default_options(ctypes.byref(o))
    return o


def pa_set_options(ctx, opts):
    return load().pa_set_options(ctx, ctypes.byref(opts))


def pa_bind_field(ctx, u_ptr):
    return load().pa_bind_field(ctx, u_ptr)


def pa_set_profile(ctx, w_ptr, fc_host_ptr, Tc):
    return load().pa_set_profile(ctx, w_ptr, fc_host_ptr, Tc)


def pa_set_coefficients(ctx, T0_ptr, scale, expo, B_ptr):
    return load().pa_set_coefficients(ctx, T0_ptr, scale, expo, B_ptr)


def pa_set_bc(ctx, ub_in_ptr, ub_out_ptr):
    return load().pa_set_bc(ctx, ub_in_ptr, ub_out_ptr)


def pa_dt_explicit(ctx):
    v = ctypes.c_double()
    return load().pa_dt_explicit(ctx, ctypes.byref(v)), v.value


def pa_apply(ctx, u_ptr, F_ptr, affine):
    return load().pa_apply(ctx, u_ptr, F_ptr, int(affine))


def pa_diag(ctx, d_ptr):
    return load().pa_diag(ctx, d_ptr)


def pa_compute_ptl(ctx):
    dt, k = ctypes.c_double(), ctypes.c_int64()
    st = load().pa_compute_ptl(ctx, ctypes.byref(dt), ctypes.byref(k))
    return st, dt.value, k.value


def pa_compute_ptl_full(ctx):
    dt, k = ctypes.c_double(), ctypes.c_int64()
    st = load().pa_compute_ptl_full(ctx, ctypes.byref(dt), ctypes.byref(k))
    return st, dt.value, k.value


def pa_compute_ptl_noalloc(ctx):
    dt, k = ctypes.c_double(), ctypes.c_int64()
    st = load().pa_compute_ptl_noalloc(ctx, ctypes.byref(dt), ctypes.byref(k))
    return st, dt.value, k.value


def pa_bilu0_apply(ctx, dt, r_ptr, z_ptr):
    return load().pa_bilu0_apply(ctx, float(dt), r_ptr, z_ptr)


def pa_advance_rkl2(ctx, dt, cycles, stats=None):
    return load().pa_advance_rkl2(ctx, dt, cycles, ctypes.byref(stats) if stats else None)


def pa_advance_rkg2(ctx, dt, cycles, stats=None):
    return load().pa_advance_rkg2(ctx, dt, cycles, ctypes.byref(stats) if stats else None)


def pa_advance_be_pcg(ctx, dt, tol, cycles, stats=None):
    return load().pa_advance_be_pcg(ctx, dt, tol, cycles, ctypes.byref(stats) if stats else None)


def pa_lpc_default_train_opts():
    o = pa_lpc_train_opts()
    load().pa_lpc_default_train_opts(ctypes.byref(o))
    return o


def pa_lpc_set_weights(ctx, theta_host_ptr):
    return load().pa_lpc_set_weights(ctx, theta_host_ptr)


def pa_lpc_get_weights(ctx, theta_host_ptr):
    return load().pa_lpc_get_weights(ctx, theta_host_ptr)


def pa_lpc_features(ctx, dt, r_ptr, feat_ptr):
    return load().pa_lpc_features(ctx, dt, r_ptr, feat_ptr)


def pa_lpc_apply(ctx, dt, r_ptr, z_ptr):
    return load().pa_lpc_apply(ctx, dt, r_ptr, z_ptr)


def pa_lpc_loss_grad(ctx, dt, npairs, r_ptr, e_ptr, grad_host_ptr):
    loss = ctypes.c_double()
    st = load().pa_lpc_loss_grad(ctx, dt, npairs, r_ptr, e_ptr, ctypes.byref(loss),
                                 grad_host_ptr)
    return st, loss.value


def pa_lpc_train(ctx, dt, opts=None, report=None):
    return load().pa_lpc_train(ctx, dt, ctypes.byref(opts) if opts else None,
                               ctypes.byref(report) if report else None)


def he_init(seed):
    """He-normal initial parameters (std sqrt(2 / fan_in), zero biases) as a
    flat float32 vector in the ABI's parameter order."""
    rng = np.random.default_rng(seed)
    parts = []
    for layer, (ci, co) in enumerate(((8, 16), (16, 16), (16, 1))):
        parts.append(rng.standard_normal(co * ci * 27) * math.sqrt(2.0 / (ci * 27)))
        if layer < 2:
            parts.append(np.zeros(co))
    theta = np.concatenate(parts).astype(np.float32)
    assert theta.size == PA_LPC_NPARAM
    return theta


# ---- convenience wrapper ---------------------------------------------------

class PaError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _callbacks(allocator, torch, device, stream, errors):
    """ctypes allocator callbacks for pa_desc: torch's caching allocator, or
    a user pair (alloc(nbytes) -> address or 0, free(address)).  A callback
    never raises into C: a failed allocation returns NULL, and the exception
    is appended to `errors`."""
    if allocator == "torch":
        index = device.index if device.index is not None else torch.cuda.current_device()

        def alloc(n):
            return torch.cuda.caching_allocator_alloc(n, index, stream)

        def free(p):
            torch.cuda.caching_allocator_delete(p)
    else:
        alloc, free = allocator

    def c_alloc(n, _user):
        try:
            return int(alloc(int(n)) or 0) or None
        except Exception as e:  # noqa: BLE001 -- reported through pa_init's status
            errors.append(repr(e))
            return None

    def c_free(p, _user):
        try:
            free(int(p))
        except Exception as e:  # noqa: BLE001
            errors.append(repr(e))

    return _ALLOC(c_alloc), _FREE(c_free)


def _stats_dict(s: pa_stats):
    n = min(s.cycles, PA_MAX_LOG)
    return dict(status=s.status, cycles=s.cycles, s_total=s.s_total, s_max=s.s_max,
                iters_total=s.iters_total, iters_max=s.iters_max, fallbacks=s.fallbacks,
                floored=s.floored, k_first=s.k_first, dt_explicit=s.dt_explicit,
                dt_ptl_first=s.dt_ptl_first, dt_ptl_min=s.dt_ptl_min,
                rel_residual=s.rel_residual, ms_total=s.ms_total,
                kernel_ms={k: s.kernel_ms[i] for i, k in enumerate(KERNEL_CLASSES)},
                kernel_calls={k: s.kernel_calls[i] for i, k in enumerate(KERNEL_CLASSES)},
                dt_cycle=np.array(s.dt_cycle[:n]), per_cycle=np.array(s.per_cycle[:n]),
                jacobi_rows=bool(s.jacobi_rows))


class Operator:
    """One split parabolic operator on one mesh, on the current HIP device.

    Arrays are torch tensors on the GPU (float64, contiguous); the bound
    field is advanced in place."""

    def __init__(self, mesh, op="iso7", ncomp=1, bc_in="dirichlet", bc_out="dirichlet",
                 prec="fp64", device="cuda", allocator=None):
        """allocator: None (the library calls hipMalloc / hipFree), "torch"
        (torch's caching allocator on the operator's stream), or a pair of
        Python callables (alloc(nbytes) -> device address or 0, free(address))
        passed to pa_init as the descriptor's allocator callbacks."""
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the parabolic-advance library has no CPU fallback")
        lib = load()
        self.torch = torch
        self.device = torch.device(device)
        self.mesh = mesh
        self.nr, self.nt, self.np = mesh.shape
        self.nc = ncomp
        self.op = op
        self._faces = [np.ascontiguousarray(a, dtype=np.float64)
                       for a in (mesh.r_faces, mesh.t_faces, mesh.p_faces)]
        d = pa_desc()
        d.nr, d.nt, d.np, d.ncomp = self.nr, self.nt, self.np, ncomp
        dp = ctypes.POINTER(ctypes.c_double)
        d.r_faces, d.t_faces, d.p_faces = (a.ctypes.data_as(dp) for a in self._faces)
        d.op, d.bc_in, d.bc_out, d.prec = OPS[op], BCS[bc_in], BCS[bc_out], PRECS[prec]
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
            self._cb = None
            self.alloc_errors = []
            if allocator is not None:
                self._cb = _callbacks(allocator, torch, self.device, self.stream,
                                      self.alloc_errors)
                d.alloc, d.free = self._cb
            st, ctx = pa_init(d, ctypes.c_void_p(self.stream.cuda_stream))
        if st != PA_OK:
            raise PaError(st, "pa_init failed" + (f" (allocator: {self.alloc_errors[-1]})"
                                                  if self.alloc_errors else ""))
        self.ctx = ctx
        self._lib = lib
        self._keep = {}
        self.field = None

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx is not None and ctx.value and _lib is not None:
            try:
                _lib.pa_destroy(ctx)
            except Exception:  # interpreter shutdown
                pass
            self.ctx = None

    def _check(self, st):
        if st != PA_OK:
            raise PaError(st, pa_last_error(self.ctx))

    def _dev(self, a, shape=None):
        t = self.torch
        if a is None:
            return None
        if not isinstance(a, t.Tensor):
            a = t.as_tensor(np.ascontiguousarray(a), dtype=t.float64)
        a = a.to(device=self.device, dtype=t.float64).contiguous()
        if shape is not None:
            a = a.reshape(shape)
        return a

    @staticmethod
    def _p(a):
        return None if a is None else ctypes.c_void_p(a.data_ptr())

    @property
    def field_shape(self):
        return (self.nc, self.nr, self.nt, self.np)

    def set_options(self, **kw):
        o = pa_default_options()
        replay = kw.pop("replay", None)
        for k, v in kw.items():
            if not hasattr(o, k):
                raise TypeError(f"unknown option {k}")
            setattr(o, k, v)
        if replay is not None:
            arr = np.ascontiguousarray(replay, dtype=np.float64)
            self._keep["replay"] = arr
            o.replay_n = len(arr)
            o.replay_dt = arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        self._check(pa_set_options(self.ctx, o))

    def set_coefficients(self, T0=None, scale=1.0, expo=0.0, B=None):
        T0 = self._dev(T0, (self.nr, self.nt, self.np))
        B = self._dev(B, (3, self.nr + 1, self.nt + 1, self.np))
        self._check(pa_set_coefficients(self.ctx, self._p(T0), float(scale), float(expo),
                                        self._p(B)))

    def set_profile(self, w=None, fc=None, Tc=0.0):
        """Weight w (cells), radial profile fc [nr] and f_m threshold Tc of
        the full operator forms; set_coefficients must follow."""
        w = self._dev(w, (self.nr, self.nt, self.np))
        fch = None if fc is None else np.ascontiguousarray(fc, dtype=np.float64)
        self._keep["fc"] = fch
        self._keep["w"] = w
        self._check(pa_set_profile(self.ctx, self._p(w),
                                   None if fch is None else fch.ctypes.data_as(ctypes.c_void_p),
                                   float(Tc)))

    def set_bc(self, ub_in=None, ub_out=None):
        shp = (self.nc, self.nt, self.np)
        a, b = self._dev(ub_in, shp), self._dev(ub_out, shp)
        self._check(pa_set_bc(self.ctx, self._p(a), self._p(b)))
        self.torch.cuda.current_stream(self.device).synchronize()

    @classmethod
    def from_problem(cls, prob, prec="fp64", device="cuda", allocator=None):
        o = cls(prob.mesh, prob.op, prob.ncomp, prob.bc_in, prob.bc_out, prec, device, allocator)
        if prob.w is not None or prob.fc is not None or prob.Tc > 0:
            o.set_profile(prob.w, prob.fc, prob.Tc)
        o.set_coefficients(prob.T0, prob.scale, prob.expo, prob.B)
        o.set_bc(prob.ub_in, prob.ub_out)
        return o

    def bind(self, u):
        u = self._dev(u, self.field_shape)
        self.field = u
        self._check(pa_bind_field(self.ctx, self._p(u)))
        return u

    def apply(self, u, affine=True):
        u = self._dev(u, self.field_shape)
        F = self.torch.empty_like(u)
        self._check(pa_apply(self.ctx, self._p(u), self._p(F), affine))
        return F

    def diag(self):
        d = self.torch.empty((self.nr, self.nt, self.np), dtype=self.torch.float64,
                             device=self.device)
        self._check(pa_diag(self.ctx, self._p(d)))
        return d

    def dt_explicit(self):
        st, v = pa_dt_explicit(self.ctx)
        self._check(st)
        return v

    def ptl(self):
        st, dt, k = pa_compute_ptl(self.ctx)
        self._check(st)
        return dt, k

    def ptl_noalloc(self):
        """pa_compute_ptl without allocating: scratch in the library's
        static device array (FP64 contexts)."""
        st, dt, k = pa_compute_ptl_noalloc(self.ctx)
        self._check(st)
        return dt, k

    def ptl_full(self):
        st, dt, k = pa_compute_ptl_full(self.ctx)
        self._check(st)
        return dt, k

    def bilu0_apply(self, r, dt):
        """z = P^{-1} r with the block ILU(0) preconditioner of M = wV + dt L."""
        r = self._dev(r, self.field_shape)
        z = self.torch.empty_like(r)
        self._check(pa_bilu0_apply(self.ctx, dt, self._p(r), self._p(z)))
        return z

    def _adv(self, fn, *args, check=True):
        s = pa_stats()
        st = fn(self.ctx, *args, s)
        out = _stats_dict(s)
        out["status"] = st
        if check:
            self._check(st)
        return out

    def advance_rkl2(self, dt, cycles=0, check=True):
        return self._adv(pa_advance_rkl2, float(dt), int(cycles), check=check)

    def advance_rkg2(self, dt, cycles=0, check=True):
        return self._adv(pa_advance_rkg2, float(dt), int(cycles), check=check)

    def advance_sts(self, dt, cycles=0, sts="rkl2", check=True):
        fn = pa_advance_rkl2 if sts == "rkl2" else pa_advance_rkg2
        return self._adv(fn, float(dt), int(cycles), check=check)

    def advance_be(self, dt, tol=1e-10, cycles=0, check=True):
        return self._adv(pa_advance_be_pcg, float(dt), float(tol), int(cycles), check=check)

    # ---- learned preconditioner
    def lpc_set_weights(self, theta):
        th = np.ascontiguousarray(theta, dtype=np.float32)
        if th.size != PA_LPC_NPARAM:
            raise ValueError(f"expected {PA_LPC_NPARAM} parameters")
        self._check(pa_lpc_set_weights(self.ctx, th.ctypes.data_as(ctypes.c_void_p)))

    def lpc_get_weights(self):
        th = np.empty(PA_LPC_NPARAM, dtype=np.float32)
        self._check(pa_lpc_get_weights(self.ctx, th.ctypes.data_as(ctypes.c_void_p)))
        return th

    def lpc_features(self, dt, r):
        r = self._dev(r, (self.nr, self.nt, self.np))
        f = self.torch.empty((8, self.nr, self.nt, self.np), dtype=self.torch.float32,
                             device=self.device)
        self._check(pa_lpc_features(self.ctx, float(dt), self._p(r), self._p(f)))
        return f

    def lpc_apply(self, dt, r):
        r = self._dev(r, (self.nr, self.nt, self.np))
        z = self.torch.empty_like(r)
        self._check(pa_lpc_apply(self.ctx, float(dt), self._p(r), self._p(z)))
        return z

    def lpc_loss_grad(self, dt, r, e):
        r = self._dev(r).reshape(-1, self.nr, self.nt, self.np).contiguous()
        e = self._dev(e).reshape(r.shape).contiguous()
        g = np.empty(PA_LPC_NPARAM, dtype=np.float32)
        st, loss = pa_lpc_loss_grad(self.ctx, float(dt), r.shape[0], self._p(r), self._p(e),
                                    g.ctypes.data_as(ctypes.c_void_p))
        self._check(st)
        return loss, g

    def lpc_train(self, dt, **kw):
        o = pa_lpc_default_train_opts()
        for k, v in kw.items():
            if not hasattr(o, k):
                raise TypeError(f"unknown training option {k}")
            setattr(o, k, v)
        rep = pa_lpc_report()
        self._check(pa_lpc_train(self.ctx, float(dt), o, rep))
        return {f: getattr(rep, f) for f, _ in rep._fields_}


def exported_symbols(path: str = LIB_PATH):
    """Names the shared library exports (for the ABI completeness check)."""
    lib = ctypes.CDLL(path)
    return [n for n in EXPORTS if hasattr(lib, n)]


_ = math  # noqa: kept for callers that reuse the module namespace
