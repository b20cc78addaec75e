"""CPU oracle for the parabolic-operator advance (TEST INFRASTRUCTURE ONLY).

Plain FP64 C (oracle.c) behind a ctypes wrapper.  Only the tests, the smoke
check and the benchmark's CPU-baseline leg use it; the library's GPU path
never imports it, and it imports nothing from the library.

Functions whose result is not pinned by an independent check say so in
their docstring ("parity unpinned").
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
MAX_LOG = 4096

OPS = {"iso7": 0, "aligned": 1, "viscv": 2}
BCS = {"dirichlet": 0, "noflux": 1}
STS = {"rkl2": 0, "rkg2": 1}
PCS = {"jacobi": 0, "bilu0": 2}


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (-O2, OpenMP) into liboracle.so."""
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-o", tmp, src, "-lm"], cwd=_HERE)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Stats(ctypes.Structure):
    _fields_ = [("cycles", ctypes.c_int32), ("s_total", ctypes.c_int32),
                ("s_max", ctypes.c_int32), ("iters_total", ctypes.c_int32),
                ("iters_max", ctypes.c_int32), ("floored", ctypes.c_int32),
                ("k_first", ctypes.c_int64),
                ("dt_explicit", ctypes.c_double), ("dt_ptl_first", ctypes.c_double),
                ("dt_ptl_min", ctypes.c_double), ("rel_residual", ctypes.c_double),
                ("dt_cycle", ctypes.c_double * MAX_LOG),
                ("s_cycle", ctypes.c_int32 * MAX_LOG)]


_lib = None
_D = ctypes.POINTER(ctypes.c_double)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    i, d, vp = ctypes.c_int, ctypes.c_double, ctypes.c_void_p
    lib.or_create.restype = vp
    lib.or_create.argtypes = [i, i, i, i, _D, _D, _D, i, i, i]
    lib.or_destroy.argtypes = [vp]
    lib.or_set_coefficients.restype = i
    lib.or_set_coefficients.argtypes = [vp, _D, d, d, _D]
    lib.or_set_profile.restype = i
    lib.or_set_profile.argtypes = [vp, _D, _D, d]
    lib.or_volumes.argtypes = [vp, i, _D]
    lib.or_set_bc.argtypes = [vp, _D, _D]
    lib.or_volume.restype = d
    lib.or_volume.argtypes = [vp, i, i, i]
    lib.or_apply.argtypes = [vp, _D, _D, i]
    lib.or_diag.argtypes = [vp, _D]
    lib.or_dt_explicit.restype = d
    lib.or_dt_explicit.argtypes = [vp]
    lib.or_ptl_from.restype = d
    lib.or_ptl_from.argtypes = [i, i, i, i, _D, _D, ctypes.POINTER(ctypes.c_int64)]
    lib.or_ptl_fullgrid.restype = d
    lib.or_ptl_fullgrid.argtypes = [i, i, i, i, _D, _D]
    lib.or_ptl.restype = d
    lib.or_ptl.argtypes = [vp, _D, ctypes.POINTER(ctypes.c_int64)]
    lib.or_sts_coeffs.restype = i
    lib.or_sts_coeffs.argtypes = [i, i, _D, _D, _D, _D]
    lib.or_sts_stages.restype = i
    lib.or_sts_stages.argtypes = [i, d, i]
    lib.or_num_threads.restype = i
    lib.or_num_threads.argtypes = []
    lib.or_set_num_threads.restype = None
    lib.or_set_num_threads.argtypes = [i]
    lib.or_stream_triad.restype = d
    lib.or_stream_triad.argtypes = [ctypes.c_long, i]
    lib.or_set_pc.restype = i
    lib.or_set_pc.argtypes = [vp, i, i, i, i]
    ip = ctypes.POINTER(ctypes.c_int)
    lib.or_bilu0_export.restype = i
    lib.or_bilu0_export.argtypes = [vp, d, ip, ip, _D, _D, i]
    lib.or_precondition.restype = i
    lib.or_precondition.argtypes = [vp, d, _D, _D]
    lib.or_advance.restype = i
    lib.or_advance.argtypes = [vp, _D, d, i, i, i, i, i, d, i, i, i, d, _D, i,
                               ctypes.POINTER(_Stats)]
    _lib = lib
    return lib


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _c(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def sts_coeffs(kind: str, s: int):
    """(mu, nu, mu_tilde, gamma) arrays indexed k = 0..s (entry 0 unused;
    at k = 1 only mu_tilde is used).  RKG2: App. A; RKL2: Meyer et al. 2014."""
    lib = _load()
    arr = [np.zeros(s + 1) for _ in range(4)]
    if lib.or_sts_coeffs(STS[kind], s, *[_ptr(a) for a in arr]) != 0:
        raise ValueError("s must be >= 2")
    return tuple(arr)


def num_threads() -> int:
    """OpenMP threads used by the oracle's parallel loops."""
    return int(_load().or_num_threads())


def set_num_threads(n: int) -> None:
    """Threads for the oracle's following parallel loops (n < 1: one per
    processor)."""
    _load().or_set_num_threads(int(n))


def stream_triad(n: int = 1 << 26, reps: int = 5) -> float:
    """Host memory bandwidth in GB/s (STREAM triad over n doubles per array,
    best of reps) at the current thread count; a reference for the CPU
    timings, not part of the method."""
    return float(_load().or_stream_triad(int(n), int(reps)))


def sts_stages(kind: str, ratio: float, force_odd: bool = True) -> int:
    """Stage count for dt/dt_E = ratio (App. A formula for RKG2; RKL2 analogue)."""
    return int(_load().or_sts_stages(STS[kind], float(ratio), int(force_odd)))


def ptl_from(u, F):
    """Eq. (ptl3) at the |F| maximum; u, F of shape (nc, nr, nt, np)."""
    u, F = _c(u), _c(F)
    nc, nr, nt, np_ = u.shape
    k = ctypes.c_int64(-1)
    dt = _load().or_ptl_from(nc, nr, nt, np_, _ptr(u), _ptr(F), ctypes.byref(k))
    return dt, int(k.value)


def ptl_fullgrid(u, F):
    """Eq. (ptl2) minimised over all cells and face directions."""
    u, F = _c(u), _c(F)
    nc, nr, nt, np_ = u.shape
    return _load().or_ptl_fullgrid(nc, nr, nt, np_, _ptr(u), _ptr(F))


class Stats(dict):
    pass


class Oracle:
    """One split operator on one mesh (CPU, FP64)."""

    def __init__(self, mesh, op="iso7", ncomp=1, bc_in="dirichlet", bc_out="dirichlet"):
        lib = _load()
        self.mesh = mesh
        self.nr, self.nt, self.np = mesh.shape
        self.nc = ncomp
        self._faces = [_c(mesh.r_faces), _c(mesh.t_faces), _c(mesh.p_faces)]
        h = lib.or_create(self.nr, self.nt, self.np, ncomp, *[_ptr(a) for a in self._faces],
                          OPS[op], BCS[bc_in], BCS[bc_out])
        if not h:
            raise ValueError("bad oracle grid")
        self._h = ctypes.c_void_p(h)
        self.op = op

    @classmethod
    def from_problem(cls, prob, bc_in=None, bc_out=None):
        o = cls(prob.mesh, prob.op, prob.ncomp, bc_in or prob.bc_in, bc_out or prob.bc_out)
        if prob.w is not None or prob.fc is not None or prob.Tc > 0:
            o.set_profile(prob.w, prob.fc, prob.Tc)
        o.set_coefficients(prob.T0, prob.scale, prob.expo, prob.B)
        o.set_bc(prob.ub_in, prob.ub_out)
        return o

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.or_destroy(h)
            self._h = None

    @property
    def field_shape(self):
        return (self.nc, self.nr, self.nt, self.np)

    def set_coefficients(self, T0=None, scale=1.0, expo=0.0, B=None):
        T0, B = _c(T0), _c(B)
        if _load().or_set_coefficients(self._h, _ptr(T0), float(scale), float(expo), _ptr(B)):
            raise ValueError("non-finite or negative coefficient, or missing B")

    def set_bc(self, ub_in=None, ub_out=None):
        _load().or_set_bc(self._h, _ptr(_c(ub_in)), _ptr(_c(ub_out)))

    def set_profile(self, w=None, fc=None, Tc=0.0):
        """Weight w (cells) of F = (1/w) div(...), radial profile fc [nr] and
        f_m threshold Tc; effective from the next set_coefficients."""
        if _load().or_set_profile(self._h, _ptr(_c(w)), _ptr(_c(fc)), float(Tc)):
            raise ValueError("non-positive weight or negative profile")

    def volumes(self, weighted=False):
        """Cell volumes V, or the weighted w V of the time derivative."""
        V = np.empty((self.nr, self.nt, self.np))
        _load().or_volumes(self._h, int(weighted), _ptr(V))
        return V

    def apply(self, u, affine=True):
        """F(u) (affine: with boundary data) or the linear part F_lin(u)."""
        u = _c(u).reshape(self.field_shape)
        F = np.empty_like(u)
        _load().or_apply(self._h, _ptr(u), _ptr(F), int(affine))
        return F

    def diag(self):
        """diag(L) on one component, L = -V F_lin."""
        d = np.empty((self.nr, self.nt, self.np))
        _load().or_diag(self._h, _ptr(d))
        return d

    def dt_explicit(self):
        return _load().or_dt_explicit(self._h)

    def ptl(self, u):
        k = ctypes.c_int64(-1)
        u = _c(u).reshape(self.field_shape)
        dt = _load().or_ptl(self._h, _ptr(u), ctypes.byref(k))
        return dt, int(k.value)

    def _advance(self, u, dt, cycles, scheme, sts="rkl2", force_odd=True, s_override=0,
                 tol=1e-10, max_iter=10000, force_iters=0, max_cycles=100000, ptl_floor=1.0,
                 replay=None):
        u = _c(u).reshape(self.field_shape).copy()
        st = _Stats()
        rp = _c(replay) if replay is not None else None
        rc = _load().or_advance(self._h, _ptr(u), float(dt), int(cycles), scheme, STS[sts],
                                int(force_odd), int(s_override), float(tol), int(max_iter),
                                int(force_iters), int(max_cycles), float(ptl_floor), _ptr(rp),
                                0 if rp is None else len(rp), ctypes.byref(st))
        n = min(st.cycles, MAX_LOG)
        out = Stats(status=rc, cycles=st.cycles, s_total=st.s_total, s_max=st.s_max,
                    iters_total=st.iters_total, iters_max=st.iters_max, floored=st.floored,
                    k_first=st.k_first,
                    dt_explicit=st.dt_explicit, dt_ptl_first=st.dt_ptl_first,
                    dt_ptl_min=st.dt_ptl_min, rel_residual=st.rel_residual,
                    dt_cycle=np.array(st.dt_cycle[:n]), per_cycle=np.array(st.s_cycle[:n]))
        return u, out

    def advance_sts(self, u, dt, cycles=0, sts="rkl2", force_odd=True, s_override=0,
                    max_cycles=100000, ptl_floor=1.0, replay=None):
        """STS advance (App. A recurrence), PTL-cycled when cycles == 0."""
        return self._advance(u, dt, cycles, 0, sts=sts, force_odd=force_odd,
                             s_override=s_override, max_cycles=max_cycles,
                             ptl_floor=ptl_floor, replay=replay)

    def set_pc(self, pc="jacobi", block=(8, 4, 16)):
        """Preconditioner of the BE solves: point Jacobi (PC1) or block ILU(0)
        (PC2) on boxes of block = (r, theta, phi) cells (7-point and
        field-aligned operators)."""
        if _load().or_set_pc(self._h, PCS[pc], *[int(b) for b in block]):
            raise ValueError("block ILU(0) needs a scalar operator and a positive box")

    def bilu0_csr(self, dt):
        """(rowp, col, m0, lu): the block-diagonal part of M = wV + dt L in CSR
        (columns ascending) and its ILU(0) factors in the same pattern (strict
        lower part: L with unit diagonal implied; diagonal and upper: U)."""
        n = self.nr * self.nt * self.np
        w = 27 * n  # the field-aligned operator couples 3 x 3 x 3 neighbourhoods
        rowp = np.zeros(n + 1, dtype=np.intc)
        col = np.zeros(w, dtype=np.intc)
        m0, lu = np.zeros(w), np.zeros(w)
        ip = ctypes.POINTER(ctypes.c_int)
        nnz = _load().or_bilu0_export(self._h, float(dt), rowp.ctypes.data_as(ip),
                                      col.ctypes.data_as(ip), _ptr(m0), _ptr(lu), w)
        if nnz < 0:
            raise ValueError("block ILU(0) export failed (%d)" % nnz)
        return rowp, col[:nnz], m0[:nnz], lu[:nnz]

    def precondition(self, r, dt):
        """z = P^{-1} r (all components) with the preconditioner of set_pc."""
        r = _c(r).reshape(self.field_shape)
        z = np.empty_like(r)
        if _load().or_precondition(self._h, float(dt), _ptr(r), _ptr(z)):
            raise ValueError("preconditioner set-up failed")
        return z

    def advance_be(self, u, dt, tol=1e-10, cycles=0, max_iter=10000, force_iters=0,
                   max_cycles=100000, ptl_floor=1.0, replay=None):
        """Backward Euler + PCG advance (preconditioner of set_pc, Jacobi by
        default), PTL-cycled when cycles == 0."""
        return self._advance(u, dt, cycles, 1, tol=tol, max_iter=max_iter,
                             force_iters=force_iters, max_cycles=max_cycles,
                             ptl_floor=ptl_floor, replay=replay)
