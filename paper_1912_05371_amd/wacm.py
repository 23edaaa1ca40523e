"""Python binding of libwacm (the C ABI in include/wacm.h).

Argument marshalling only: every step of the method runs in the HIP library.
Device memory and streams come from PyTorch.  The binding refuses to run if
the library is missing (build it with ``python -m paper_1912_05371_amd.build``)
-- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwacm.so")

OK = 0
E_INVAL, E_NOMEM, E_CAPACITY, E_UNBALANCED, E_HIP, E_NONFINITE, E_TILING = -1, -2, -3, -4, -5, \
    -6, -7
F32, F64 = 1, 2
DT_FIXED, DT_CFL = 0, 1
REFINE_ALL, COARSEN = 1, 2
CDF40, CDF44 = 0, 1
MASK_NONE, MASK_SPHERE, MASK_PLATE = 0, 1, 2

EXPORTS = ["wacm_last_error", "wacm_treecode_encode", "wacm_treecode_decode", "wacm_grid_create",
           "wacm_grid_destroy", "wacm_grid_nb", "wacm_grid_info", "wacm_work_bytes",
           "wacm_sync_ghosts", "wacm_rhs_acm", "wacm_compute_dt", "wacm_rk4_step", "wacm_rk4_steps",
           "wacm_diagnostics", "wacm_threshold_blocks", "wacm_filter_blocks", "wacm_adapt",
           "wacm_profile_enable", "wacm_profile_read", "wacm_adj_work_bytes", "wacm_sync_ghosts_adj",
           "wacm_rhs_acm_adj", "wacm_force_adj", "wacm_rk4_step_adj", "wacm_set_schedule",
           "wacm_get_schedule", "wacm_set_wavelet", "wacm_get_wavelet", "wacm_mr_work_bytes",
           "wacm_mr_forward", "wacm_mr_inverse", "wacm_workspace_bytes",
           "wacm_wavelet_workspace_bytes", "wacm_adj_plan_bytes", "wacm_adj_plan_set",
           "wacm_mr_forward_noalloc", "wacm_adapt_timing", "wacm_sync_ghosts_lattice"]
MR_SCRATCH_BYTES = 64 << 20  # WACM_MR_SCRATCH_BYTES


class GridDesc(C.Structure):
    _fields_ = [("bs", C.c_int32), ("ng", C.c_int32), ("jmin", C.c_int32), ("jmax", C.c_int32),
                ("dtype", C.c_int32), ("dim", C.c_int32), ("capacity", C.c_int64),
                ("L", C.c_double)]


class Schedule(C.Structure):
    _fields_ = [("wg_per_cu", C.c_int32), ("xcd_map", C.c_int32), ("prefetch", C.c_int32),
                ("nontemporal", C.c_int32), ("tile_rows", C.c_int32), ("pen_split", C.c_int32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class Params(C.Structure):
    _fields_ = [
        ("nu", C.c_double), ("c0", C.c_double), ("c_gamma", C.c_double), ("c_eta", C.c_double),
        ("c_sp", C.c_double), ("l_sp", C.c_double), ("u_inf", C.c_double * 3),
        ("p_inf", C.c_double), ("mask", C.c_int32), ("sponge", C.c_int32), ("clip", C.c_int32),
        ("reserved", C.c_int32), ("w", C.c_double), ("sph_c", C.c_double * 3),
        ("sph_r", C.c_double), ("x_le", C.c_double * 3), ("lo", C.c_double * 3),
        ("hi", C.c_double * 3), ("amp", C.c_double), ("freq", C.c_double), ("phase", C.c_double),
        ("cfl", C.c_double), ("cfl_eta", C.c_double), ("cfl_nu", C.c_double),
    ]


def make_params(d: dict) -> Params:
    p = Params()
    for name, ctype in Params._fields_:
        if name == "reserved" or name not in d:
            continue
        v = d[name]
        cur = getattr(p, name)
        if isinstance(cur, C.Array):
            for i, x in enumerate(v):
                cur[i] = float(x)
        elif ctype is C.c_int32:
            setattr(p, name, int(v))
        else:
            setattr(p, name, float(v))
    return p


class WacmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"wacm error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load libwacm.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1912_05371_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, i64, i32, dbl = C.c_void_p, C.c_int64, C.c_int32, C.c_double
        L.wacm_last_error.restype = C.c_char_p
        L.wacm_last_error.argtypes = [vp]
        L.wacm_treecode_encode.restype = C.c_uint64
        L.wacm_treecode_encode.argtypes = [i32, i64, i64, i64]
        L.wacm_treecode_decode.restype = None
        L.wacm_treecode_decode.argtypes = [C.c_uint64, i32, vp, vp, vp]
        L.wacm_workspace_bytes.restype = C.c_size_t
        L.wacm_workspace_bytes.argtypes = [C.POINTER(GridDesc)]
        L.wacm_grid_create.argtypes = [C.POINTER(GridDesc), i64, vp, vp, vp, C.c_size_t,
                                       C.POINTER(vp)]
        L.wacm_grid_destroy.argtypes = [vp]
        L.wacm_grid_nb.restype = i64
        L.wacm_grid_nb.argtypes = [vp]
        L.wacm_grid_info.argtypes = [vp, vp, vp, vp]
        L.wacm_work_bytes.restype = C.c_size_t
        L.wacm_work_bytes.argtypes = [vp]
        L.wacm_sync_ghosts.argtypes = [vp, vp, vp]
        L.wacm_sync_ghosts_lattice.argtypes = [vp, vp, vp]
        L.wacm_rhs_acm.argtypes = [vp, C.POINTER(Params), dbl, vp, vp, vp, vp]
        L.wacm_compute_dt.argtypes = [vp, C.POINTER(Params), vp, vp, vp]
        L.wacm_rk4_step.argtypes = [vp, C.POINTER(Params), vp, vp, vp, vp, vp, i32, vp]
        L.wacm_rk4_steps.argtypes = [vp, C.POINTER(Params), vp, vp, vp, vp, vp, i32, i64, vp]
        L.wacm_diagnostics.argtypes = [vp, C.POINTER(Params), dbl, vp, vp, vp, vp]
        L.wacm_threshold_blocks.argtypes = [vp, C.POINTER(Params), dbl, vp, dbl, i32, vp, vp, vp,
                                            vp]
        L.wacm_filter_blocks.argtypes = [vp, vp, i32, vp]
        L.wacm_wavelet_workspace_bytes.restype = C.c_size_t
        L.wacm_wavelet_workspace_bytes.argtypes = [vp, i32]
        L.wacm_set_wavelet.argtypes = [vp, i32, vp, C.c_size_t]
        L.wacm_mr_work_bytes.restype = C.c_size_t
        L.wacm_mr_work_bytes.argtypes = [i64, i32, i32]
        L.wacm_mr_forward.argtypes = [i64, i32, i32, i32, i32, vp, vp, C.c_size_t, vp]
        L.wacm_mr_inverse.argtypes = [i64, i32, i32, i32, i32, vp, vp, C.c_size_t, vp]
        L.wacm_mr_forward_noalloc.argtypes = [i64, i32, i32, i32, i32, vp, vp]
        L.wacm_get_wavelet.argtypes = [vp]
        L.wacm_adapt.argtypes = [vp, i32, vp, vp, vp, vp]
        L.wacm_adj_work_bytes.restype = C.c_size_t
        L.wacm_adj_work_bytes.argtypes = [vp]
        L.wacm_adj_plan_bytes.restype = C.c_size_t
        L.wacm_adj_plan_bytes.argtypes = [vp, i32]
        L.wacm_adj_plan_set.argtypes = [vp, i32, vp, C.c_size_t]
        L.wacm_sync_ghosts_adj.argtypes = [vp, vp, vp]
        L.wacm_rhs_acm_adj.argtypes = [vp, C.POINTER(Params), dbl, vp, vp, vp, vp, vp, vp, vp]
        L.wacm_force_adj.argtypes = [vp, C.POINTER(Params), dbl, dbl, vp, vp, vp, vp, vp, vp]
        L.wacm_rk4_step_adj.argtypes = [vp, C.POINTER(Params), dbl, dbl, vp, vp, vp, vp, vp, vp,
                                        vp]
        L.wacm_set_schedule.argtypes = [vp, C.POINTER(Schedule)]
        L.wacm_get_schedule.argtypes = [vp, C.POINTER(Schedule)]
        L.wacm_profile_enable.argtypes = [vp, i32]
        L.wacm_profile_read.argtypes = [vp, vp, vp]
        L.wacm_adapt_timing.argtypes = [vp, vp]
        _lib = L
    return _lib


def _check(rc: int, handle=None):
    """Raise WacmError for a failed call; the text is the grid's last error
    (handle given) or the calling thread's."""
    if rc != OK:
        raise WacmError(rc, lib().wacm_last_error(handle).decode())


def _device_buffer(nbytes: int, device="cuda"):
    """A caller-owned device buffer (uint8 torch tensor, 256-byte aligned by
    torch's allocator) for one of the library's workspaces."""
    import torch
    t = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)
    if t.data_ptr() % 256:
        raise RuntimeError("device buffer is not 256-byte aligned")
    return t


def treecode_encode(level, ix, iy, iz) -> int:
    return int(lib().wacm_treecode_encode(int(level), int(ix), int(iy), int(iz)))


def treecode_decode(code, level):
    x, y, z = C.c_int64(), C.c_int64(), C.c_int64()
    lib().wacm_treecode_decode(int(code), int(level), C.byref(x), C.byref(y), C.byref(z))
    return x.value, y.value, z.value


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _ptr(t):
    if t is None:
        return None
    return C.c_void_p(t.data_ptr())


def _mr_args(u):
    import torch
    if u.dim() == 3:
        u = u.unsqueeze(0)
    if (u.dim() != 4 or not u.is_cuda or not u.is_contiguous()
            or not (u.shape[1] == u.shape[2] == u.shape[3])):
        raise ValueError("mr transform: expected a contiguous cuda tensor [nf, n, n, n]")
    dt = {torch.float64: F64, torch.float32: F32}.get(u.dtype)
    if dt is None:
        raise ValueError("mr transform: float32 or float64 only")
    return u.shape[1], u.shape[0], dt


def mr_work(u):
    """Work buffer (uint8 cuda tensor) for mr_forward / mr_inverse on u."""
    import torch
    n, nf, dt = _mr_args(u)
    nbytes = int(lib().wacm_mr_work_bytes(n, nf, dt))
    return torch.empty(max(nbytes, 1), dtype=torch.uint8, device=u.device)


def _mr_work_arg(u, work):
    """(pointer, size) of the work buffer; a buffer that is given must be a
    contiguous CUDA tensor on u's device, 256-byte aligned, with at least
    wacm_mr_work_bytes() bytes (the C call checks the size and alignment
    again)."""
    if work is None:
        return None, 0
    n, nf, dt = _mr_args(u)
    need = int(lib().wacm_mr_work_bytes(n, nf, dt))
    size = work.numel() * work.element_size()
    if not work.is_cuda or work.device != u.device or not work.is_contiguous():
        raise ValueError("mr transform: work must be a contiguous CUDA tensor on u's device")
    if work.data_ptr() % 256 != 0:
        raise ValueError("mr transform: work must be 256-byte aligned")
    if size < need:
        raise ValueError(f"mr transform: work has {size} bytes, {need} needed")
    return _ptr(work), size


def mr_forward(u, nlev: int, wavelet: int = CDF40, work=None, stream=None):
    """Multiresolution transform of the periodic fields u ([nf, n, n, n] or
    [n, n, n], contiguous, cuda), in place."""
    n, nf, dt = _mr_args(u)
    wp, ws = _mr_work_arg(u, work)
    _check(lib().wacm_mr_forward(n, nf, dt, int(wavelet), int(nlev), _ptr(u), wp, ws,
                                 _stream(stream)))


def mr_forward_noalloc(u, nlev: int, wavelet: int = CDF40, stream=None):
    """:func:`mr_forward` without a work buffer: the library's static device
    scratch array (MR_SCRATCH_BYTES per GPU) serves as the CDF 4/4 work; no
    allocation.  u must be on the current device."""
    n, nf, dt = _mr_args(u)
    _check(lib().wacm_mr_forward_noalloc(n, nf, dt, int(wavelet), int(nlev), _ptr(u),
                                         _stream(stream)))


def mr_inverse(u, nlev: int, wavelet: int = CDF40, work=None, stream=None):
    """Inverse of :func:`mr_forward`, in place."""
    n, nf, dt = _mr_args(u)
    wp, ws = _mr_work_arg(u, work)
    _check(lib().wacm_mr_inverse(n, nf, dt, int(wavelet), int(nlev), _ptr(u), wp, ws,
                                 _stream(stream)))


class Grid:
    """Opaque grid handle plus the geometry needed to shape tensors."""

    def __init__(self, bs, ng, L, jmin, jmax, treecodes, levels, dtype=F64, capacity=None,
                 dim=3):
        """dim 3: octree; dim 2: quadtree (treecodes of (bx, by, 0), pool of 3
        fields (u, v, p) per slot, P^2 values each)."""
        treecodes = np.ascontiguousarray(treecodes, np.uint64)
        levels = np.ascontiguousarray(levels, np.int8)
        n = len(treecodes)
        self.dim = int(dim)
        self.desc = GridDesc(int(bs), int(ng), int(jmin), int(jmax), int(dtype), self.dim,
                             int(capacity if capacity is not None else n), float(L))
        self._h = None
        nbytes = int(lib().wacm_workspace_bytes(C.byref(self.desc)))
        if nbytes == 0:
            _check(E_INVAL)
        # the grid's tables live in this caller-owned buffer until close()
        self._ws = _device_buffer(nbytes)
        self._wav_ws = None
        self._plan_ws = {0: None, 1: None}
        h = C.c_void_p()
        self._call(lib().wacm_grid_create(C.byref(self.desc), n,
                                      treecodes.ctypes.data_as(C.c_void_p),
                                      levels.ctypes.data_as(C.c_void_p), _ptr(self._ws), nbytes,
                                      C.byref(h)))
        self._h = h
        self.bs, self.ng, self.L, self.jmin, self.jmax = int(bs), int(ng), float(L), jmin, jmax
        self.P = self.bs + 2 * self.ng
        self.dtype = dtype
        self.capacity = self.desc.capacity

    @classmethod
    def from_case(cls, case, dtype=F64, capacity=None):
        if not hasattr(case, "iz"):  # a two-dimensional case
            codes = [treecode_encode(l, x, y, 0) for l, x, y in zip(case.lev, case.ix, case.iy)]
            return cls(case.bs, case.ng, case.L, case.jmin, case.jmax, codes, case.lev, dtype,
                       capacity, dim=2)
        codes = [treecode_encode(l, x, y, z) for l, x, y, z in
                 zip(case.lev, case.ix, case.iy, case.iz)]
        return cls(case.bs, case.ng, case.L, case.jmin, case.jmax, codes, case.lev, dtype,
                   capacity)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().wacm_grid_destroy(self._h)
            self._h = None
        # the workspaces may go only after the handle that points into them
        self._ws = self._wav_ws = None
        self._plan_ws = {0: None, 1: None}

    def last_error(self) -> str:
        return lib().wacm_last_error(self._h).decode()

    def _call(self, rc: int):
        _check(rc, self._h)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def nb(self) -> int:
        return int(lib().wacm_grid_nb(self._h))

    def info(self):
        nb = self.nb
        slots = np.zeros(nb, np.int64)
        codes = np.zeros(nb, np.uint64)
        levels = np.zeros(nb, np.int8)
        self._call(lib().wacm_grid_info(self._h, slots.ctypes.data_as(C.c_void_p),
                                    codes.ctypes.data_as(C.c_void_p),
                                    levels.ctypes.data_as(C.c_void_p)))
        return slots, codes, levels

    def work_bytes(self) -> int:
        return int(lib().wacm_work_bytes(self._h))

    # ---- tensors ------------------------------------------------------------
    def torch_dtype(self):
        import torch
        return torch.float64 if self.dtype == F64 else torch.float32

    def pool_shape(self):
        if self.dim == 2:
            return (self.capacity, 3, self.P, self.P)
        return (self.capacity, 4, self.P, self.P, self.P)

    def pool(self, device="cuda"):
        import torch
        return torch.zeros(self.pool_shape(), dtype=self.torch_dtype(), device=device)

    def work(self, device="cuda"):
        import torch
        return torch.empty(self.work_bytes(), dtype=torch.uint8, device=device)

    def _chk_pool(self, U):
        if tuple(U.shape) != self.pool_shape() or \
                U.dtype != self.torch_dtype() or not U.is_contiguous() or not U.is_cuda:
            raise ValueError("pool tensor must be a contiguous CUDA tensor of shape "
                             f"{self.pool_shape()} / {self.torch_dtype()}")

    @staticmethod
    def _chk_vec(t, n, dtype_name, what):
        import torch
        dt = {"f64": torch.float64, "i8": torch.int8}[dtype_name]
        if t is None or not t.is_cuda or t.dtype != dt or not t.is_contiguous() or t.numel() < n:
            raise ValueError(f"{what} must be a contiguous CUDA {dt} tensor with >= {n} entries")

    def _chk_dus(self, dus):
        if dus is None:
            return
        if tuple(dus.shape) != (self.capacity, 3, self.bs ** 3) or \
                dus.dtype != self.torch_dtype() or not dus.is_contiguous() or not dus.is_cuda:
            raise ValueError("dus must be (capacity, 3, bs^3) contiguous on the GPU")

    # ---- entry points (same names as the C ABI) ----------------------------------
    def sync_ghosts(self, U, stream=None):
        self._chk_pool(U)
        self._call(lib().wacm_sync_ghosts(self._h, _ptr(U), _stream(stream)))

    def sync_ghosts_lattice(self, U, stream=None):
        """The ghost points the thresholding reads (the even lattice within 3
        of each block), as sync_ghosts fills them."""
        self._chk_pool(U)
        self._call(lib().wacm_sync_ghosts_lattice(self._h, _ptr(U), _stream(stream)))

    def rhs_acm(self, params: dict, t: float, U, dU, dus=None, stream=None):
        self._chk_pool(U)
        self._chk_pool(dU)
        self._chk_dus(dus)
        p = make_params(params)
        self._call(lib().wacm_rhs_acm(self._h, C.byref(p), float(t), _ptr(U), _ptr(dU), _ptr(dus),
                                  _stream(stream)))

    def compute_dt(self, params: dict, U, dt_dev, stream=None):
        self._chk_pool(U)
        self._chk_vec(dt_dev, 1, "f64", "dt_dev")
        p = make_params(params)
        self._call(lib().wacm_compute_dt(self._h, C.byref(p), _ptr(U), _ptr(dt_dev), _stream(stream)))

    def rk4_step(self, params: dict, t_dev, dt_dev, U, work, dus=None, dt_mode=DT_CFL,
                 stream=None, _p=None):
        self._chk_pool(U)
        self._chk_dus(dus)
        self._chk_vec(t_dev, 1, "f64", "t_dev")
        self._chk_vec(dt_dev, 1, "f64", "dt_dev")
        if not work.is_cuda or work.numel() * work.element_size() < self.work_bytes():
            raise ValueError("work buffer too small")
        p = _p if _p is not None else make_params(params)
        self._call(lib().wacm_rk4_step(self._h, C.byref(p), _ptr(t_dev), _ptr(dt_dev), _ptr(U),
                                   _ptr(work), _ptr(dus), int(dt_mode), _stream(stream)))

    def rk4_steps(self, params: dict, t_dev, dt_dev, U, work, nsteps: int, dus=None,
                  dt_mode=DT_CFL, stream=None, _p=None):
        self._chk_pool(U)
        self._chk_dus(dus)
        self._chk_vec(t_dev, 1, "f64", "t_dev")
        self._chk_vec(dt_dev, 1, "f64", "dt_dev")
        if not work.is_cuda or work.numel() * work.element_size() < self.work_bytes():
            raise ValueError("work buffer too small")
        p = _p if _p is not None else make_params(params)
        self._call(lib().wacm_rk4_steps(self._h, C.byref(p), _ptr(t_dev), _ptr(dt_dev), _ptr(U),
                                    _ptr(work), _ptr(dus), int(dt_mode), int(nsteps),
                                    _stream(stream)))

    def diagnostics(self, params: dict, t: float, U, out, dus=None, stream=None):
        self._chk_pool(U)
        self._chk_dus(dus)
        self._chk_vec(out, 10, "f64", "out")
        p = make_params(params)
        self._call(lib().wacm_diagnostics(self._h, C.byref(p), float(t), _ptr(U), _ptr(dus),
                                          _ptr(out), _stream(stream)))

    def threshold_blocks(self, params: dict, t: float, U, eps: float, dealias: bool, dmax,
                         mrange, flags, stream=None):
        self._chk_pool(U)
        nb = self.nb
        self._chk_vec(dmax, nb, "f64", "dmax")
        self._chk_vec(mrange, nb, "f64", "mrange")
        self._chk_vec(flags, nb, "i8", "flags")
        p = make_params(params)
        self._call(lib().wacm_threshold_blocks(self._h, C.byref(p), float(t), _ptr(U), float(eps),
                                           int(bool(dealias)), _ptr(dmax), _ptr(mrange),
                                           _ptr(flags), _stream(stream)))

    def set_wavelet(self, wavelet: int):
        """CDF40 (restriction = decimation) or CDF44 (lifted, needs ng >= 6;
        its ghost-phase buffers are allocated here, sized for the capacity)."""
        nbytes = int(lib().wacm_wavelet_workspace_bytes(self._h, int(wavelet)))
        ws = _device_buffer(nbytes) if nbytes else None
        self._call(lib().wacm_set_wavelet(self._h, int(wavelet), _ptr(ws), nbytes))
        self._wav_ws = ws

    def get_wavelet(self) -> int:
        return int(lib().wacm_get_wavelet(self._h))

    def filter_blocks(self, U, level: int = -1, stream=None):
        """Remove the details of the blocks of `level` (all if < 0) in place;
        U ghost-synced."""
        self._chk_pool(U)
        self._call(lib().wacm_filter_blocks(self._h, _ptr(U), int(level), _stream(stream)))

    def adapt(self, op: int, U, flags=None, stream=None) -> int:
        self._chk_pool(U)
        nb = C.c_int64()
        fptr = None
        if flags is not None:
            flags = np.ascontiguousarray(flags, np.int8)
            if len(flags) != self.nb:
                raise ValueError("flags must have nb entries")
            fptr = flags.ctypes.data_as(C.c_void_p)
        self._call(lib().wacm_adapt(self._h, int(op), fptr, _ptr(U), C.byref(nb),
                                    _stream(stream)))
        self._plan_ws = {0: None, 1: None}  # the library dropped its plans
        return nb.value

    def set_schedule(self, **kw):
        s = Schedule()
        self._call(lib().wacm_get_schedule(self._h, C.byref(s)))
        for k, v in kw.items():
            setattr(s, k, int(v))
        self._call(lib().wacm_set_schedule(self._h, C.byref(s)))

    def get_schedule(self) -> dict:
        s = Schedule()
        self._call(lib().wacm_get_schedule(self._h, C.byref(s)))
        return s.as_dict()

    def profile_enable(self, on: bool = True):
        self._call(lib().wacm_profile_enable(self._h, int(bool(on))))

    def adapt_timing(self):
        """(host ms, device ms) of the last adapt call."""
        ms = np.zeros(2)
        self._call(lib().wacm_adapt_timing(self._h, ms.ctypes.data_as(C.c_void_p)))
        return float(ms[0]), float(ms[1])

    def profile_read(self):
        """(ms[4], launches[4]) per kernel class: dt, sync, stage, time update."""
        ms = np.zeros(4)
        n = np.zeros(4, np.int64)
        self._call(lib().wacm_profile_read(self._h, ms.ctypes.data_as(C.c_void_p),
                                       n.ctypes.data_as(C.c_void_p)))
        return ms, n

    # ---- adjoint ------------------------------------------------------------
    def adj_work_bytes(self) -> int:
        return int(lib().wacm_adj_work_bytes(self._h))

    def adj_work(self, device="cuda"):
        import torch
        return torch.empty(self.adj_work_bytes(), dtype=torch.uint8, device=device)

    def _chk_dusbar(self, dusbar):
        import torch
        if dusbar is None:
            return
        if tuple(dusbar.shape) != (self.capacity, 3, self.bs ** 3) or \
                dusbar.dtype != torch.float64 or not dusbar.is_contiguous() or not dusbar.is_cuda:
            raise ValueError("dusbar must be (capacity, 3, bs^3) float64 contiguous on the GPU")

    def adj_plan(self, face_only: int):
        """Build the transpose plan of the ghost fill (0: all layers, for
        sync_ghosts_adj; 1: the depth-3 face star, for rk4_step_adj) and copy
        it into a buffer owned here; a no-op if it is already set."""
        f = int(face_only)
        if self._plan_ws[f] is not None:
            return
        nbytes = int(lib().wacm_adj_plan_bytes(self._h, f))
        if nbytes == 0:
            self._call(E_INVAL)
        ws = _device_buffer(nbytes)
        self._call(lib().wacm_adj_plan_set(self._h, f, _ptr(ws), nbytes))
        self._plan_ws[f] = ws

    def sync_ghosts_adj(self, Ub, stream=None):
        self._chk_pool(Ub)
        self.adj_plan(0)
        self._call(lib().wacm_sync_ghosts_adj(self._h, _ptr(Ub), _stream(stream)))

    def rhs_acm_adj(self, params: dict, t: float, U, V, Ub, dtheta, dusbar=None, dus=None,
                    stream=None):
        for a in (U, V, Ub):
            self._chk_pool(a)
        self._chk_vec(dtheta, 3, "f64", "dtheta")
        self._chk_dusbar(dusbar)
        self._chk_dus(dus)
        p = make_params(params)
        self._call(lib().wacm_rhs_acm_adj(self._h, C.byref(p), float(t), _ptr(U), _ptr(V), _ptr(Ub),
                                      _ptr(dtheta), _ptr(dusbar), _ptr(dus), _stream(stream)))

    def force_adj(self, params: dict, t: float, weight: float, U, Ub, dtheta, dusbar=None,
                  dus=None, stream=None):
        self._chk_pool(U)
        self._chk_pool(Ub)
        self._chk_vec(dtheta, 3, "f64", "dtheta")
        self._chk_dusbar(dusbar)
        self._chk_dus(dus)
        p = make_params(params)
        self._call(lib().wacm_force_adj(self._h, C.byref(p), float(t), float(weight), _ptr(U),
                                    _ptr(Ub), _ptr(dtheta), _ptr(dusbar), _ptr(dus),
                                    _stream(stream)))

    def rk4_step_adj(self, params: dict, t: float, dt: float, Un, lam, dtheta, dusbar=None,
                     dus=None, work=None, stream=None):
        self._chk_pool(Un)
        self._chk_pool(lam)
        self._chk_vec(dtheta, 3, "f64", "dtheta")
        self._chk_dusbar(dusbar)
        self._chk_dus(dus)
        if work is None or not work.is_cuda or \
                work.numel() * work.element_size() < self.adj_work_bytes():
            raise ValueError("adjoint work buffer too small")
        self.adj_plan(1)
        p = make_params(params)
        self._call(lib().wacm_rk4_step_adj(self._h, C.byref(p), float(t), float(dt), _ptr(Un),
                                       _ptr(lam), _ptr(dtheta), _ptr(dusbar), _ptr(dus),
                                       _ptr(work), _stream(stream)))
