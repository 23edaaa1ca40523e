"""TEST INFRASTRUCTURE ONLY: ctypes front end of the FP64 CPU oracle.

The oracle (``wacm_oracle.c``) is a plain, slow, FP64 implementation of the
wavelet-adaptive artificial-compressibility block method of arXiv:1912.05371
(Sec. 2.2-2.3 equations and discretisation, Sec. 3.1-3.5 multiresolution and
adaptation, Sec. 4.2 ghost-node synchronisation).  Only ``tests/``, the smoke
check and the CPU-baseline leg of the benchmark may import this module; the
product library never calls it.  It shares no code with the HIP library.

Arrays: a state ``U`` is a float64 numpy array of shape (nb, 4, P, P, P),
fields (u, v, w, p), P = bs + 2 ng, x fastest (last axis).  Blocks follow the
order of the leaves given to :class:`Grid`.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "wacm_oracle.c")
SRC2D = os.path.join(HERE, "wacm_oracle2d.c")
LIB = os.path.join(HERE, "liboracle.so")
# a sanitizer build of the same source may be loaded instead (CPU tests only)
LIB = os.environ.get("WACM_ORACLE_LIB", LIB)

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fast-math, no FMA contraction)."""
    if force or not os.path.exists(LIB):
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
               "-shared", "-std=c11", "-o", LIB + ".tmp", SRC, SRC2D, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(LIB + ".tmp", LIB)
    return LIB


class OrcParams(C.Structure):
    _fields_ = [
        ("nu", C.c_double), ("c0", C.c_double), ("c_gamma", C.c_double), ("c_eta", C.c_double),
        ("c_sp", C.c_double), ("l_sp", C.c_double), ("u_inf", C.c_double * 3),
        ("p_inf", C.c_double), ("mask", C.c_int32), ("sponge", C.c_int32), ("clip", C.c_int32),
        ("pad0", C.c_int32), ("w", C.c_double), ("sph_c", C.c_double * 3), ("sph_r", C.c_double),
        ("x_le", C.c_double * 3), ("lo", C.c_double * 3), ("hi", C.c_double * 3),
        ("amp", C.c_double), ("freq", C.c_double), ("phase", C.c_double),
        ("cfl", C.c_double), ("cfl_eta", C.c_double), ("cfl_nu", C.c_double),
    ]


def make_params(d: dict) -> OrcParams:
    p = OrcParams()
    for name, ctype in OrcParams._fields_:
        if name == "pad0" or name not in d:
            continue
        v = d[name]
        if isinstance(getattr(p, name), C.Array):
            arr = getattr(p, name)
            for i, x in enumerate(v):
                arr[i] = float(x)
        elif ctype is C.c_int32:
            setattr(p, name, int(v))
        else:
            setattr(p, name, float(v))
    return p


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        dp = C.POINTER(C.c_double)
        vp = C.c_void_p
        L.orc_tam_webb.argtypes = [dp]
        L.orc_treecode_encode.restype = C.c_uint64
        L.orc_treecode_encode.argtypes = [C.c_int, C.c_int64, C.c_int64, C.c_int64]
        L.orc_treecode_decode.argtypes = [C.c_uint64, C.c_int] + [C.POINTER(C.c_int64)] * 3
        L.orc_grid_create.restype = vp
        L.orc_grid_create.argtypes = [C.c_int, C.c_int, C.c_double, C.c_int, C.c_int, C.c_int64,
                                      vp, vp, vp, vp, C.POINTER(C.c_int)]
        L.orc_grid_free.argtypes = [vp]
        L.orc_grid_nb.restype = C.c_int64
        L.orc_grid_nb.argtypes = [vp]
        L.orc_grid_leaves.argtypes = [vp, vp, vp, vp, vp]
        L.orc_is_balanced.restype = C.c_int
        L.orc_is_balanced.argtypes = [vp]
        L.orc_owner.restype = C.c_int64
        L.orc_owner.argtypes = [vp, C.c_int, C.c_int64, C.c_int64, C.c_int64] + \
            [C.POINTER(C.c_int64)] * 3
        L.orc_sync.argtypes = [vp, vp]
        L.orc_mask.argtypes = [vp, C.POINTER(OrcParams), C.c_double, vp, vp]
        L.orc_rhs.argtypes = [vp, C.POINTER(OrcParams), C.c_double, vp, vp, vp]
        L.orc_dt.restype = C.c_double
        L.orc_dt.argtypes = [vp, C.POINTER(OrcParams), vp]
        L.orc_rk4_step.argtypes = [vp, C.POINTER(OrcParams), C.c_double, C.c_double, vp, vp]
        L.orc_diagnostics.argtypes = [vp, C.POINTER(OrcParams), C.c_double, vp, vp, vp]
        L.orc_details.argtypes = [vp, C.POINTER(OrcParams), C.c_double, vp, vp, vp]
        L.orc_flags.argtypes = [vp, vp, vp, C.c_double, C.c_int, vp]
        L.orc_filter.argtypes = [vp, C.c_int, vp]
        L.orc_set_wavelet.restype = C.c_int
        L.orc_set_wavelet.argtypes = [vp, C.c_int]
        L.orc_lift_lowpass.argtypes = [C.c_int, vp]
        L.orc_mr_forward.argtypes = [C.c_int64, C.c_int, C.c_int, C.c_int, vp]
        L.orc_mr_inverse.argtypes = [C.c_int64, C.c_int, C.c_int, C.c_int, vp]
        L.orc_refine_count.restype = C.c_int64
        L.orc_refine_count.argtypes = [vp]
        L.orc_refine_all.restype = vp
        L.orc_refine_all.argtypes = [vp, vp, vp]
        L.orc_coarsen_count.restype = C.c_int64
        L.orc_coarsen_count.argtypes = [vp, vp]
        L.orc_coarsen.restype = vp
        L.orc_coarsen.argtypes = [vp, vp, vp, vp]
        L.orc_rhs_adj.argtypes = [vp, C.POINTER(OrcParams), C.c_double, vp, vp, vp, dp, vp, vp]
        L.orc_sync_adj.argtypes = [vp, vp]
        L.orc_force_x.restype = C.c_double
        L.orc_force_x.argtypes = [vp, C.POINTER(OrcParams), C.c_double, vp, vp]
        L.orc_force_x_adj.argtypes = [vp, C.POINTER(OrcParams), C.c_double, C.c_double, vp, vp,
                                      dp, vp, vp]
        L.orc_rk4_step_adj.argtypes = [vp, C.POINTER(OrcParams), C.c_double, C.c_double, vp,
                                       vp, dp, vp, vp]
        # two-dimensional form
        L.orc2_grid_create.restype = vp
        L.orc2_grid_create.argtypes = [C.c_int, C.c_int, C.c_double, C.c_int, C.c_int,
                                       C.c_int64, vp, vp, vp, C.POINTER(C.c_int)]
        L.orc2_grid_free.argtypes = [vp]
        L.orc2_grid_nb.restype = C.c_int64
        L.orc2_grid_nb.argtypes = [vp]
        L.orc2_grid_leaves.argtypes = [vp, vp, vp, vp]
        L.orc2_sync.argtypes = [vp, vp]
        L.orc2_rhs.argtypes = [vp, C.POINTER(OrcParams), vp, vp]
        L.orc2_dt.restype = C.c_double
        L.orc2_dt.argtypes = [vp, C.POINTER(OrcParams), vp]
        L.orc2_rk4_step.argtypes = [vp, C.POINTER(OrcParams), C.c_double, vp]
        L.orc2_diagnostics.argtypes = [vp, vp, vp]
        L.orc2_details.argtypes = [vp, vp, vp]
        L.orc2_flags.argtypes = [vp, vp, C.c_double, C.c_int, vp]
        L.orc2_refine_count.restype = C.c_int64
        L.orc2_refine_count.argtypes = [vp]
        L.orc2_refine_all.restype = vp
        L.orc2_refine_all.argtypes = [vp, vp, vp]
        L.orc2_coarsen_count.restype = C.c_int64
        L.orc2_coarsen_count.argtypes = [vp, vp]
        L.orc2_coarsen.restype = vp
        L.orc2_coarsen.argtypes = [vp, vp, vp, vp]
        _lib = L
    return _lib


def _ptr(a: np.ndarray | None):
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.c_void_p)


def tam_webb() -> np.ndarray:
    a = (C.c_double * 3)()
    lib().orc_tam_webb(a)
    return np.array(list(a))


def lift_lowpass(order: int) -> np.ndarray:
    """Taps at offsets -6..6 of the lifted low-pass (order 4: CDF 4/4, 2: CDF 2/2)."""
    t = np.zeros(13)
    lib().orc_lift_lowpass(int(order), _ptr(t))
    return t


def _mr(fn, u: np.ndarray, nlev: int, wavelet: int) -> np.ndarray:
    a = np.ascontiguousarray(u, dtype=np.float64).copy()
    squeeze = a.ndim == 3
    if squeeze:
        a = a[None]
    if a.ndim != 4 or not (a.shape[1] == a.shape[2] == a.shape[3]):
        raise ValueError("mr transform: expected [nf, n, n, n] or [n, n, n]")
    if fn(a.shape[1], a.shape[0], nlev, wavelet, _ptr(a)) != 0:
        raise ValueError("mr transform: invalid size, level count or wavelet")
    return a[0] if squeeze else a


def mr_forward(u: np.ndarray, nlev: int, wavelet: int = 0) -> np.ndarray:
    """Multiresolution transform (Sec. 3.1, 3.2) of periodic fields, a new
    array ([nf, n, n, n] or [n, n, n]); wavelet 0 CDF 4/0, 1 CDF 4/4."""
    return _mr(lib().orc_mr_forward, u, nlev, wavelet)


def mr_inverse(w: np.ndarray, nlev: int, wavelet: int = 0) -> np.ndarray:
    """Inverse of :func:`mr_forward`."""
    return _mr(lib().orc_mr_inverse, w, nlev, wavelet)


def treecode_encode(level: int, ix: int, iy: int, iz: int) -> int:
    return int(lib().orc_treecode_encode(level, ix, iy, iz))


def treecode_decode(code: int, level: int) -> tuple[int, int, int]:
    x, y, z = C.c_int64(), C.c_int64(), C.c_int64()
    lib().orc_treecode_decode(code, level, C.byref(x), C.byref(y), C.byref(z))
    return x.value, y.value, z.value


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__({-1: "invalid sizes", -2: "leaves overlap or do not tile",
                          -3: "grid not 2:1 balanced"}.get(code, str(code)))
        self.code = code


class Grid:
    """A leaf set (levels and block indices) with the oracle's operations."""

    def __init__(self, bs, ng, L, jmin, jmax, lev, ix, iy, iz, _handle=None):
        self.bs, self.ng, self.L, self.jmin, self.jmax = int(bs), int(ng), float(L), jmin, jmax
        self.P = self.bs + 2 * self.ng
        if _handle is None:
            lev = np.ascontiguousarray(lev, dtype=np.int32)
            ix = np.ascontiguousarray(ix, dtype=np.int64)
            iy = np.ascontiguousarray(iy, dtype=np.int64)
            iz = np.ascontiguousarray(iz, dtype=np.int64)
            err = C.c_int(0)
            h = lib().orc_grid_create(self.bs, self.ng, self.L, jmin, jmax, len(lev), _ptr(lev),
                                      _ptr(ix), _ptr(iy), _ptr(iz), C.byref(err))
            if not h:
                raise OracleError(err.value)
            _handle = h
        self._h = C.c_void_p(_handle)
        self.nb = int(lib().orc_grid_nb(self._h))
        self.lev = np.zeros(self.nb, np.int32)
        self.ix = np.zeros(self.nb, np.int64)
        self.iy = np.zeros(self.nb, np.int64)
        self.iz = np.zeros(self.nb, np.int64)
        lib().orc_grid_leaves(self._h, _ptr(self.lev), _ptr(self.ix), _ptr(self.iy), _ptr(self.iz))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.orc_grid_free(h)
            self._h = None

    def _child(self, handle) -> "Grid":
        return Grid(self.bs, self.ng, self.L, self.jmin, self.jmax, None, None, None, None,
                    _handle=handle)

    def zeros(self) -> np.ndarray:
        return np.zeros((self.nb, 4, self.P, self.P, self.P), np.float64)

    def is_balanced(self) -> bool:
        return bool(lib().orc_is_balanced(self._h))

    def owner(self, J, gx, gy, gz):
        li, lj, lk = C.c_int64(), C.c_int64(), C.c_int64()
        b = lib().orc_owner(self._h, J, gx, gy, gz, C.byref(li), C.byref(lj), C.byref(lk))
        return int(b), (li.value, lj.value, lk.value)

    def sync(self, U: np.ndarray) -> None:
        lib().orc_sync(self._h, _ptr(U))

    def mask(self, params: dict, t: float):
        n3 = self.bs ** 3
        chi = np.zeros((self.nb, n3))
        us = np.zeros((self.nb, 3, n3))
        p = make_params(params)
        lib().orc_mask(self._h, C.byref(p), t, _ptr(chi), _ptr(us))
        return chi, us

    def rhs(self, params: dict, t: float, U: np.ndarray, dus=None) -> np.ndarray:
        dU = self.zeros()
        p = make_params(params)
        lib().orc_rhs(self._h, C.byref(p), t, _ptr(U), _ptr(dus), _ptr(dU))
        return dU

    def dt(self, params: dict, U: np.ndarray) -> float:
        p = make_params(params)
        return float(lib().orc_dt(self._h, C.byref(p), _ptr(U)))

    def rk4_step(self, params: dict, t: float, dt: float, U: np.ndarray, dus=None) -> None:
        p = make_params(params)
        lib().orc_rk4_step(self._h, C.byref(p), t, dt, _ptr(U), _ptr(dus))

    def diagnostics(self, params: dict, t: float, U: np.ndarray, dus=None) -> np.ndarray:
        out = np.zeros(9)
        p = make_params(params)
        lib().orc_diagnostics(self._h, C.byref(p), t, _ptr(U), _ptr(dus), _ptr(out))
        return out

    def details(self, params: dict | None, t: float, U: np.ndarray):
        dmax = np.zeros(self.nb)
        mr = np.zeros(self.nb)
        if params is None:
            lib().orc_details(self._h, None, t, _ptr(U), _ptr(dmax), _ptr(mr))
        else:
            p = make_params(params)
            lib().orc_details(self._h, C.byref(p), t, _ptr(U), _ptr(dmax), _ptr(mr))
        return dmax, mr

    def set_wavelet(self, wavelet: int) -> None:
        """0: CDF 4/0 (decimation), 1: CDF 4/4 (lifted restriction, ng >= 6)."""
        if lib().orc_set_wavelet(self._h, int(wavelet)) != 0:
            raise ValueError("invalid wavelet for this grid")

    def filter(self, level: int, U: np.ndarray) -> None:
        """Remove the details of the blocks of `level` (all if < 0) in place;
        U ghost-synced."""
        lib().orc_filter(self._h, int(level), _ptr(U))

    def flags(self, dmax, mrange, eps: float, dealias: bool) -> np.ndarray:
        f = np.zeros(self.nb, np.int8)
        lib().orc_flags(self._h, _ptr(np.ascontiguousarray(dmax, np.float64)),
                        _ptr(np.ascontiguousarray(mrange, np.float64)), eps, int(dealias), _ptr(f))
        return f

    def refine_all(self, U: np.ndarray):
        n = int(lib().orc_refine_count(self._h))
        Un = np.zeros((n, 4, self.P, self.P, self.P))
        h = lib().orc_refine_all(self._h, _ptr(U), _ptr(Un))
        return self._child(h), Un

    def coarsen_count(self, flags: np.ndarray) -> int:
        flags = np.ascontiguousarray(flags, np.int8)
        return int(lib().orc_coarsen_count(self._h, _ptr(flags)))

    def coarsen(self, flags: np.ndarray, U: np.ndarray):
        flags = np.ascontiguousarray(flags, np.int8)
        n = int(lib().orc_coarsen_count(self._h, _ptr(flags)))
        Un = np.zeros((n, 4, self.P, self.P, self.P))
        h = lib().orc_coarsen(self._h, _ptr(flags), _ptr(U), _ptr(Un))
        return self._child(h), Un

    # ---- adjoint ----------------------------------------------------------
    def rhs_adj(self, params, t, U, V, Ubar, dtheta, dusbar=None, dus=None):
        p = make_params(params)
        th = (C.c_double * 3)(*dtheta)
        lib().orc_rhs_adj(self._h, C.byref(p), t, _ptr(U), _ptr(V), _ptr(Ubar), th,
                          _ptr(dusbar), _ptr(dus))
        dtheta[:] = list(th)

    def sync_adj(self, Ubar):
        lib().orc_sync_adj(self._h, _ptr(Ubar))

    def force_x(self, params, t, U, dus=None) -> float:
        p = make_params(params)
        return float(lib().orc_force_x(self._h, C.byref(p), t, _ptr(U), _ptr(dus)))

    def force_x_adj(self, params, t, weight, U, Ubar, dtheta, dusbar=None, dus=None):
        p = make_params(params)
        th = (C.c_double * 3)(*dtheta)
        lib().orc_force_x_adj(self._h, C.byref(p), t, weight, _ptr(U), _ptr(Ubar), th,
                              _ptr(dusbar), _ptr(dus))
        dtheta[:] = list(th)

    def rk4_step_adj(self, params, t, dt, Un, Lam, dtheta, dusbar=None, dus=None):
        p = make_params(params)
        th = (C.c_double * 3)(*dtheta)
        lib().orc_rk4_step_adj(self._h, C.byref(p), t, dt, _ptr(Un), _ptr(Lam), th,
                               _ptr(dusbar), _ptr(dus))
        dtheta[:] = list(th)

    def objective(self, params, U0, dt, nsteps, dus=None):
        """J = sum_{n=1..N} dt F_x(U^n, t^n) with a fixed dt; returns J and the
        checkpoints U^0..U^{N-1}."""
        U = U0.copy()
        ck = []
        J = 0.0
        for n in range(nsteps):
            ck.append(U.copy())
            self.rk4_step(params, n * dt, dt, U, dus)
            J += dt * self.force_x(params, (n + 1) * dt, U, dus)
        return J, ck, U

    def objective_grad(self, params, U0, dt, nsteps, dus=None):
        """Gradient of objective() by the discrete adjoint: (dJ/dtheta, dJ/ddus, dJ/dU0)."""
        J, ck, UN = self.objective(params, U0, dt, nsteps, dus)
        n3 = self.bs ** 3
        dth = [0.0, 0.0, 0.0]
        dusbar = np.zeros((self.nb, 3, n3)) if dus is not None else None
        lam = np.zeros_like(U0)
        self.force_x_adj(params, nsteps * dt, dt, UN, lam, dth, dusbar, dus)
        for n in range(nsteps - 1, -1, -1):
            self.rk4_step_adj(params, n * dt, dt, ck[n], lam, dth, dusbar, dus)
            if n >= 1:
                self.force_x_adj(params, n * dt, dt, ck[n], lam, dth, dusbar, dus)
        return J, np.array(dth), dusbar, lam

    def treecodes(self) -> np.ndarray:
        return np.array([treecode_encode(int(l), int(x), int(y), int(z))
                         for l, x, y, z in zip(self.lev, self.ix, self.iy, self.iz)], np.uint64)


class Grid2D:
    """A quadtree leaf set (levels and block indices (ix, iy)) with the 2D
    oracle's operations.  A state U is a float64 array (nb, 3, P, P), fields
    (u, v, p), x fastest."""

    def __init__(self, bs, ng, L, jmin, jmax, lev, ix, iy, _handle=None):
        self.bs, self.ng, self.L, self.jmin, self.jmax = int(bs), int(ng), float(L), jmin, jmax
        self.P = self.bs + 2 * self.ng
        if _handle is None:
            lev = np.ascontiguousarray(lev, dtype=np.int32)
            ix = np.ascontiguousarray(ix, dtype=np.int64)
            iy = np.ascontiguousarray(iy, dtype=np.int64)
            err = C.c_int(0)
            h = lib().orc2_grid_create(self.bs, self.ng, self.L, jmin, jmax, len(lev), _ptr(lev),
                                       _ptr(ix), _ptr(iy), C.byref(err))
            if not h:
                raise OracleError(err.value)
            _handle = h
        self._h = C.c_void_p(_handle)
        self.nb = int(lib().orc2_grid_nb(self._h))
        self.lev = np.zeros(self.nb, np.int32)
        self.ix = np.zeros(self.nb, np.int64)
        self.iy = np.zeros(self.nb, np.int64)
        lib().orc2_grid_leaves(self._h, _ptr(self.lev), _ptr(self.ix), _ptr(self.iy))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.orc2_grid_free(h)
            self._h = None

    def _child(self, handle) -> "Grid2D":
        return Grid2D(self.bs, self.ng, self.L, self.jmin, self.jmax, None, None, None,
                      _handle=handle)

    def zeros(self) -> np.ndarray:
        return np.zeros((self.nb, 3, self.P, self.P), np.float64)

    def sync(self, U: np.ndarray) -> None:
        lib().orc2_sync(self._h, _ptr(U))

    def rhs(self, params: dict, U: np.ndarray) -> np.ndarray:
        dU = self.zeros()
        p = make_params(params)
        lib().orc2_rhs(self._h, C.byref(p), _ptr(U), _ptr(dU))
        return dU

    def dt(self, params: dict, U: np.ndarray) -> float:
        p = make_params(params)
        return float(lib().orc2_dt(self._h, C.byref(p), _ptr(U)))

    def rk4_step(self, params: dict, dt: float, U: np.ndarray) -> None:
        p = make_params(params)
        lib().orc2_rk4_step(self._h, C.byref(p), dt, _ptr(U))

    def diagnostics(self, U: np.ndarray) -> np.ndarray:
        out = np.zeros(9)
        lib().orc2_diagnostics(self._h, _ptr(U), _ptr(out))
        return out

    def details(self, U: np.ndarray) -> np.ndarray:
        d = np.zeros(self.nb)
        lib().orc2_details(self._h, _ptr(U), _ptr(d))
        return d

    def flags(self, dmax, eps: float, dealias: bool) -> np.ndarray:
        f = np.zeros(self.nb, np.int8)
        lib().orc2_flags(self._h, _ptr(np.ascontiguousarray(dmax, np.float64)), eps,
                         int(dealias), _ptr(f))
        return f

    def refine_all(self, U: np.ndarray):
        n = int(lib().orc2_refine_count(self._h))
        Un = np.zeros((n, 3, self.P, self.P))
        h = lib().orc2_refine_all(self._h, _ptr(U), _ptr(Un))
        return self._child(h), Un

    def coarsen(self, flags: np.ndarray, U: np.ndarray):
        flags = np.ascontiguousarray(flags, np.int8)
        n = int(lib().orc2_coarsen_count(self._h, _ptr(flags)))
        Un = np.zeros((n, 3, self.P, self.P))
        h = lib().orc2_coarsen(self._h, _ptr(flags), _ptr(U), _ptr(Un))
        return self._child(h), Un
