"""Thin ctypes binding of ``libwt.so`` (argument marshalling only; every step runs in the HIP
library).  Names follow the C ABI in ``include/wt.h``.

The library is loaded from this package directory.  If it has not been built, or cannot be
loaded, ``load()`` raises: there is no fallback implementation.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libwt.so")

WT_OK, WT_EINVAL, WT_ENOMEM, WT_EDEVICE, WT_ESTATE, WT_ENUMERIC = 0, -1, -2, -3, -4, -5
WT_RK4, WT_SSPRK43 = 0, 1
WT_FP64, WT_FP32_TENDENCY = 0, 1
WT_SWE, WT_ADVECTION = 0, 1
WT_THR_RELATIVE, WT_THR_QG, WT_THR_IG = 0, 1, 2


class WtError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


class wt_params(C.Structure):
    _fields_ = [("radius", C.c_double), ("omega", C.c_double), ("gravity", C.c_double),
                ("mean_depth", C.c_double), ("rk", C.c_int), ("precision", C.c_int),
                ("viscosity", C.c_double), ("equations", C.c_int), ("threshold", C.c_int),
                ("scale_u", C.c_double), ("scale_l", C.c_double), ("scale_f", C.c_double)]


class wt_diag(C.Structure):
    _fields_ = [("mass", C.c_double), ("mass_reconstructed", C.c_double), ("energy", C.c_double), ("max_abs_dh", C.c_double),
                ("max_abs_u", C.c_double), ("active_nodes", C.c_int64 * 16),
                ("active_edges", C.c_int64 * 16), ("finest_level", C.c_int32), ("pad_", C.c_int32)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


_P = C.c_void_p
_D = C.POINTER(C.c_double)
_I64 = C.POINTER(C.c_int64)
_I32 = C.POINTER(C.c_int32)
_U8 = C.POINTER(C.c_uint8)
_F = C.POINTER(C.c_float)

# (name, restype, argtypes) for every function declared in include/wt.h
SIGNATURES = [
    ("wt_grid_create", _P, [C.c_int, C.c_int, C.c_int]),
    ("wt_grid_destroy", None, [_P]),
    ("wt_set_params", C.c_int, [_P, C.POINTER(wt_params)]),
    ("wt_get_params", C.c_int, [_P, C.POINTER(wt_params)]),
    ("wt_grid_info", C.c_int, [_P, C.c_int, _I64, _I64, _I64]),
    ("wt_grid_coords", C.c_int, [_P, C.c_int, _D, _D, _D]),
    ("wt_set_state", C.c_int, [_P, C.c_int, _D, _D]),
    ("wt_set_state_device", C.c_int, [_P, C.c_int, _P, _P]),
    ("wt_get_state", C.c_int, [_P, C.c_int, _D, _D, _U8, _U8]),
    ("wt_step", C.c_int, [_P, C.c_double]),
    ("wt_tendency", C.c_int, [_P, C.c_int, _D, _D]),
    ("wt_adapt", C.c_int, [_P, C.c_double]),
    ("wt_forward", C.c_int, [_P]),
    ("wt_inverse", C.c_int, [_P]),
    ("wt_get_details", C.c_int, [_P, C.c_int, _D, _D, _D]),
    ("wt_set_mask", C.c_int, [_P, C.c_int, _U8, _U8]),
    ("wt_diagnostics", C.c_int, [_P, C.POINTER(wt_diag)]),
    ("wt_suggest_dt", C.c_double, [_P, C.c_double]),
    ("wt_set_stream", C.c_int, [_P, _P]),
    ("wt_set_allocator", C.c_int, [_P, ALLOC_FN, FREE_FN, _P]),
    ("wt_alloc_stats", C.c_int, [_P, _I64, _I64, _I64, _I64]),
    ("wt_timing_enable", C.c_int, [_P, C.c_int]),
    ("wt_timing_reset", C.c_int, [_P]),
    ("wt_kernel_time", C.c_int, [_P, C.c_char_p, _D, _I64, _D]),
    ("wt_kernel_names", C.c_char_p, []),
    ("wt_kernel_units", C.c_int, [_P, C.c_char_p, _I64]),
    ("wt_table_cache_clear", None, []),
    ("wt_save", C.c_int, [_P, C.c_char_p]),
    ("wt_load", C.c_int, [_P, C.c_char_p]),
    ("wt_host_level_tables", C.c_int, [C.c_int, C.c_double, C.c_double, _D, _D, _D, _D, _I32, _I32, _D]),
    ("wt_host_pair_tables", C.c_int, [C.c_int, C.c_int, C.c_double, C.c_double, _I32, _D, _D, _D, _I32, _D,
                                      _D, _D, _I32, _D, _I32, _D]),
    ("wt_host_lattice_check", C.c_int, [C.c_int, _I64, _I64, _D]),
    ("wt_mlp_create", _P, [_F]),
    ("wt_mlp_destroy", None, [_P]),
    ("wt_mlp_set_stream", C.c_int, [_P, _P]),
    ("wt_mlp_get_params", C.c_int, [_P, _F]),
    ("wt_mlp_forward", C.c_int, [_P, _P, C.c_int64, _P]),
    ("wt_mlp_gradient", C.c_int, [_P, _P, _P, C.c_int64, _F, _D]),
    ("wt_mlp_train_step", C.c_int, [_P, _P, _P, C.c_int64, C.c_double, _D]),
    ("wt_mlp_gradient_noalloc", C.c_int, [_P, _P, _P, C.c_int64, _P]),
    ("wt_patch_count", C.c_int64, [_P, C.c_int]),
    ("wt_patch_features", C.c_int, [_P, C.c_int, _P]),
    ("wt_patch_labels", C.c_int, [_P, C.c_int, _P]),
    ("wt_set_predictor", C.c_int, [_P, _P, C.c_double]),
    ("wt_redo_count", C.c_int, [_P, _I64]),
    ("wt_debug_force_drop", C.c_int, [_P, C.c_int, C.c_int64]),
    ("wt_set_work_lists", C.c_int, [_P, C.c_int]),
    ("wt_set_step_phases", C.c_int, [_P, C.c_int]),
    ("wt_set_dense_levels", C.c_int, [_P, C.c_double]),
    ("wt_set_dense_min_tiles", C.c_int, [_P, C.c_int]),
    ("wt_ensemble_create", _P, [C.POINTER(_P), C.c_int]),
    ("wt_ensemble_destroy", None, [_P]),
    ("wt_ensemble_adapt", C.c_int, [_P, _D]),
    ("wt_ensemble_step", C.c_int, [_P, _D]),
    ("wt_ensemble_stats", C.c_int, [_P, _I64, _I64]),
    ("wt_ensemble_set_batched", C.c_int, [_P, C.c_int]),
    ("wt_ensemble_tuning", C.c_int, [_P, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int),
                                     C.POINTER(C.c_int), C.POINTER(C.c_float)]),
    ("wt_last_error", C.c_char_p, []),
]

MLP_INPUTS, MLP_OUTPUTS, MLP_PARAMS = 64, 4, 25348

_lib = None


def load():
    """Load libwt.so (raises OSError / FileNotFoundError if it is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise FileNotFoundError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        # torch ships its own HIP runtime under the same soname; loading torch first makes
        # libwt bind to that one, so the process has a single runtime and torch streams are
        # valid handles for wt_set_stream.
        import torch  # noqa: F401
        lib = C.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


# Objects that own library handles, closed in reverse creation order when the interpreter exits:
# grids, ensembles and networks release their device memory and streams while the HIP runtime is
# still fully alive, instead of in whatever order garbage collection reaches them at shutdown.
_LIVE = weakref.WeakValueDictionary()
_LIVE_SEQ = [0]


def _register(obj):
    _LIVE_SEQ[0] += 1
    _LIVE[_LIVE_SEQ[0]] = obj


@atexit.register
def _close_all():
    for k in sorted(list(_LIVE.keys()), reverse=True):
        obj = _LIVE.get(k)
        if obj is not None:
            try:
                obj.close()
            except Exception:
                pass
    if _lib is not None:
        try:
            _lib.wt_table_cache_clear()
        except Exception:
            pass


# ---------------------------------------------------------------- device allocator hook
_ALLOC_HOOK = None   # (alloc, free) ctypes callbacks kept alive while the library may call them


def use_torch_allocator(grid=None):
    """Route the device buffers of `grid` (None: of every grid created afterwards) through
    PyTorch's caching allocator (wt_set_allocator)."""
    global _ALLOC_HOOK
    import torch

    if _ALLOC_HOOK is None:
        dev = torch.cuda.current_device()

        def _alloc(nbytes, ctx):
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes), device=dev)
            except Exception:
                return None

        def _free(ptr, ctx):
            torch.cuda.caching_allocator_delete(ptr)

        _ALLOC_HOOK = (ALLOC_FN(_alloc), FREE_FN(_free))
    a, f = _ALLOC_HOOK
    _check(load().wt_set_allocator(grid._h if grid is not None else None, a, f, None))


def use_hip_allocator(grid=None):
    """Back to hipMalloc for later allocations of `grid` (None: of grids created afterwards)."""
    _check(load().wt_set_allocator(grid._h if grid is not None else None, ALLOC_FN(), FREE_FN(), None))


def _ptr(a, ct):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(ct))


def _check(code, what=""):
    if code != WT_OK:
        raise WtError(code, load().wt_last_error().decode() or what)


def table_cache_clear():
    """Free the host geometry tables that grid creation caches per level and level pair."""
    load().wt_table_cache_clear()


def host_level_tables(level, radius=6.371e6, omega=7.292e-5):
    """Host-only geometry of the library's grid builder (no GPU)."""
    lib = load()
    n = 2 ** level
    N, E, T = 10 * n * n + 2, 30 * n * n, 20 * n * n
    out = dict(A_i=np.empty(N), A_v=np.empty(T), d_e=np.empty(E), l_e=np.empty(E),
               e_nodes=np.empty((E, 2), np.int32), ecp=np.empty((E, 10), np.int32), w=np.empty((E, 10)))
    _check(lib.wt_host_level_tables(level, radius, omega, _ptr(out["A_i"], C.c_double),
                                    _ptr(out["A_v"], C.c_double), _ptr(out["d_e"], C.c_double),
                                    _ptr(out["l_e"], C.c_double), _ptr(out["e_nodes"], C.c_int32),
                                    _ptr(out["ecp"], C.c_int32), _ptr(out["w"], C.c_double)))
    return out


def host_lattice_check(level):
    """Host-only check of the lattice form (no GPU): (tiles per lozenge, rim elements, max
    relative difference between the shared reference geometry and every lozenge)."""
    nt, nr, err = C.c_int64(), C.c_int64(), C.c_double()
    _check(load().wt_host_lattice_check(level, C.byref(nt), C.byref(nr), C.byref(err)))
    return nt.value, nr.value, err.value


def host_pair_tables(jc, jmax, radius=6.371e6, omega=7.292e-5):
    """Host-only inter-scale tables of the library between levels jc and jc+1 (no GPU)."""
    lib = load()
    n = 2 ** jc
    Nc, Ec, Tc = 10 * n * n + 2, 30 * n * n, 20 * n * n
    o = dict(cells=np.empty((Ec, 4), np.int32), st=np.empty((Ec, 4)), s_upd=np.empty((Ec, 4)),
             A_c=np.empty(Nc), v_sten=np.empty((Tc, 9), np.int32), w_int=np.empty((Tc, 3, 9)),
             w_pl=np.empty((Ec, 9)), w_pr=np.empty((Ec, 9)), rf_f=np.empty((Ec, 3), np.int32),
             rf_fw=np.empty((Ec, 3)), rf_c=np.empty((Ec, 8), np.int32), rf_cw=np.empty((Ec, 8)))
    d, i = C.c_double, C.c_int32
    _check(lib.wt_host_pair_tables(jc, jmax, radius, omega, _ptr(o["cells"], i), _ptr(o["st"], d),
                                   _ptr(o["s_upd"], d), _ptr(o["A_c"], d), _ptr(o["v_sten"], i),
                                   _ptr(o["w_int"], d), _ptr(o["w_pl"], d), _ptr(o["w_pr"], d),
                                   _ptr(o["rf_f"], i), _ptr(o["rf_fw"], d), _ptr(o["rf_c"], i),
                                   _ptr(o["rf_cw"], d)))
    return o


class Grid:
    """A multilevel grid owned by the HIP library (wt_grid)."""

    def __init__(self, jmin, jmax, patch=8):
        lib = load()
        h = lib.wt_grid_create(jmin, jmax, patch)
        if not h:
            raise WtError(WT_EDEVICE, lib.wt_last_error().decode())
        self._h = h
        self.jmin, self.jmax, self.patch = jmin, jmax, patch
        _register(self)

    def close(self):
        if getattr(self, "_h", None):
            load().wt_grid_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # parameters
    def get_params(self):
        p = wt_params()
        _check(load().wt_get_params(self._h, C.byref(p)))
        return p

    def set_params(self, **kw):
        p = self.get_params()
        for k, v in kw.items():
            setattr(p, k, v)
        _check(load().wt_set_params(self._h, C.byref(p)))

    def info(self, level):
        n, e, t = C.c_int64(), C.c_int64(), C.c_int64()
        _check(load().wt_grid_info(self._h, level, C.byref(n), C.byref(e), C.byref(t)))
        return n.value, e.value, t.value

    def coords(self, level):
        N, E, _ = self.info(level)
        x, m, t = np.empty((N, 3)), np.empty((E, 3)), np.empty((E, 3))
        _check(load().wt_grid_coords(self._h, level, _ptr(x, C.c_double), _ptr(m, C.c_double),
                                     _ptr(t, C.c_double)))
        return x, m, t

    def set_state(self, level, dh, u):
        dh = np.ascontiguousarray(dh, np.float64)
        u = np.ascontiguousarray(u, np.float64)
        N, E, _ = self.info(level)
        if dh.shape != (N,) or u.shape != (E,):
            raise ValueError(f"state shapes {dh.shape}, {u.shape} != ({N},), ({E},)")
        _check(load().wt_set_state(self._h, level, _ptr(dh, C.c_double), _ptr(u, C.c_double)))

    def set_state_device(self, level, dh_ptr, u_ptr):
        _check(load().wt_set_state_device(self._h, level, C.c_void_p(dh_ptr), C.c_void_p(u_ptr)))

    def get_state(self, level):
        N, E, _ = self.info(level)
        dh, u = np.empty(N), np.empty(E)
        na, ea = np.empty(N, np.uint8), np.empty(E, np.uint8)
        _check(load().wt_get_state(self._h, level, _ptr(dh, C.c_double), _ptr(u, C.c_double),
                                   _ptr(na, C.c_uint8), _ptr(ea, C.c_uint8)))
        return dh, u, na, ea

    def step(self, dt):
        _check(load().wt_step(self._h, float(dt)))

    def tendency(self, level):
        N, E, _ = self.info(level)
        a, b = np.empty(N), np.empty(E)
        _check(load().wt_tendency(self._h, level, _ptr(a, C.c_double), _ptr(b, C.c_double)))
        return a, b

    def adapt(self, eps):
        _check(load().wt_adapt(self._h, float(eps)))

    def forward(self):
        _check(load().wt_forward(self._h))

    def inverse(self):
        _check(load().wt_inverse(self._h))

    def get_details(self, level):
        Nc, Ec, Tc = self.info(level - 1)
        a, b, c = np.empty(Ec), np.empty(Ec), np.empty(3 * Tc)
        _check(load().wt_get_details(self._h, level, _ptr(a, C.c_double), _ptr(b, C.c_double),
                                     _ptr(c, C.c_double)))
        return a, b, c.reshape(Tc, 3)

    def set_mask(self, level, node_active, edge_active):
        na = np.ascontiguousarray(node_active, np.uint8)
        ea = np.ascontiguousarray(edge_active, np.uint8)
        _check(load().wt_set_mask(self._h, level, _ptr(na, C.c_uint8), _ptr(ea, C.c_uint8)))

    def diagnostics(self):
        d = wt_diag()
        code = load().wt_diagnostics(self._h, C.byref(d))
        if code not in (WT_OK, WT_ENUMERIC):
            _check(code)
        return d, code

    def suggest_dt(self, cfl):
        v = load().wt_suggest_dt(self._h, float(cfl))
        if v < 0:
            _check(WT_EINVAL)
        return v

    def set_stream(self, stream_handle):
        _check(load().wt_set_stream(self._h, C.c_void_p(stream_handle) if stream_handle else None))

    def alloc_stats(self):
        """Live device buffers of the grid: (count, bytes) from the allocator hook and from hipMalloc."""
        a, b, c, d = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64()
        _check(load().wt_alloc_stats(self._h, C.byref(a), C.byref(b), C.byref(c), C.byref(d)))
        return {"hook": (a.value, b.value), "direct": (c.value, d.value)}

    def timing(self, enable=True):
        _check(load().wt_timing_enable(self._h, 1 if enable else 0))

    def timing_reset(self):
        _check(load().wt_timing_reset(self._h))

    def patch_count(self, level):
        n = load().wt_patch_count(self._h, level)
        if n < 0:
            _check(int(n))
        return int(n)

    def patch_features(self, level, x):
        _check(load().wt_patch_features(self._h, level, _dev_ptr(x, "float32", (MLP_INPUTS,))))

    def patch_labels(self, level, y):
        _check(load().wt_patch_labels(self._h, level, _dev_ptr(y, "float32", (MLP_OUTPUTS,))))

    def set_predictor(self, mlp, threshold=0.5):
        self._predictor = mlp   # keeps the network alive while the grid uses it
        _check(load().wt_set_predictor(self._h, mlp._h if mlp is not None else None, float(threshold)))

    def save(self, path):
        """Write the grid's state (every level, masks, parameters) to a checkpoint file."""
        _check(load().wt_save(self._h, os.fsencode(path)))

    def load(self, path):
        """Read a checkpoint written by save() of a grid with the same levels and patch size."""
        _check(load().wt_load(self._h, os.fsencode(path)))

    def set_work_lists(self, enable):
        _check(load().wt_set_work_lists(self._h, 1 if enable else 0))

    def set_step_phases(self, enable):
        """Merge the independent launches of the listed step (default) or launch per kernel."""
        _check(load().wt_set_step_phases(self._h, 1 if enable else 0))

    def set_dense_levels(self, min_fraction):
        """Run the finest level through the masked lattice kernel when its listed support holds
        at least `min_fraction` of its elements (above 1: off, the default)."""
        _check(load().wt_set_dense_levels(self._h, float(min_fraction)))

    def set_dense_min_tiles(self, min_tiles):
        """Tile positions the level below the finest needs to run dense (-1: the device's CU count)."""
        _check(load().wt_set_dense_min_tiles(self._h, int(min_tiles)))

    def debug_force_drop(self, level, patch):
        """Withhold the children rule of a patch at the next gated adapt (test hook)."""
        _check(load().wt_debug_force_drop(self._h, level, int(patch)))

    def redo_count(self):
        r = C.c_int64()
        _check(load().wt_redo_count(self._h, C.byref(r)))
        return r.value

    def kernel_time(self, name):
        """(total ms, launches, total algorithmic bytes) since the last timing reset."""
        ms, cnt, by = C.c_double(), C.c_int64(), C.c_double()
        _check(load().wt_kernel_time(self._h, name.encode(), C.byref(ms), C.byref(cnt), C.byref(by)))
        return ms.value, cnt.value, by.value


def kernel_units(grid, name):
    """Units (elements or triangles) the last timed launch of kernel `name` processed."""
    u = C.c_int64()
    _check(load().wt_kernel_units(grid._h, name.encode(), C.byref(u)))
    return u.value


def kernel_names():
    return load().wt_kernel_names().decode().split(",")


def _dev_ptr(t, dtype_name, shape_tail):
    """Device pointer of a contiguous torch CUDA tensor of the given dtype and trailing shape."""
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.is_contiguous()):
        raise ValueError("expected a contiguous CUDA tensor")
    if str(t.dtype) != "torch." + dtype_name or tuple(t.shape[1:]) != tuple(shape_tail):
        raise ValueError(f"expected {dtype_name} [n, {shape_tail}], got {t.dtype} {tuple(t.shape)}")
    return C.c_void_p(t.data_ptr())


class Mlp:
    """Child-patch predictor network (64 -> 128 -> 128 -> 4) on the matrix cores; thin wrapper
    of the wt_mlp_* calls.  Feature/label/probability arrays are float32 CUDA tensors."""

    def __init__(self, params):
        import numpy as np
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != MLP_PARAMS:
            raise ValueError(f"need {MLP_PARAMS} parameters")
        lib = load()
        h = lib.wt_mlp_create(_ptr(p, C.c_float))
        if not h:
            raise WtError(WT_EDEVICE, lib.wt_last_error().decode())
        self._h = h
        _register(self)

    def close(self):
        if getattr(self, "_h", None):
            load().wt_mlp_destroy(self._h)
            self._h = None

    __del__ = close

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def set_stream(self, stream):
        _check(load().wt_mlp_set_stream(self._h, C.c_void_p(stream) if stream else None))

    def params(self):
        import numpy as np
        out = np.empty(MLP_PARAMS, dtype=np.float32)
        _check(load().wt_mlp_get_params(self._h, _ptr(out, C.c_float)))
        return out

    def forward(self, x, p):
        n = x.shape[0]
        _check(load().wt_mlp_forward(self._h, _dev_ptr(x, "float32", (MLP_INPUTS,)), n,
                                     _dev_ptr(p, "float32", (MLP_OUTPUTS,))))

    def gradient(self, x, y):
        import numpy as np
        g = np.empty(MLP_PARAMS, dtype=np.float32)
        loss = C.c_double()
        _check(load().wt_mlp_gradient(self._h, _dev_ptr(x, "float32", (MLP_INPUTS,)),
                                      _dev_ptr(y, "float32", (MLP_OUTPUTS,)), x.shape[0], _ptr(g, C.c_float),
                                      C.byref(loss)))
        return g, loss.value

    def gradient_noalloc(self, x, y, out):
        """Gradient and loss sum into the float32 CUDA tensor out[MLP_PARAMS + 1] without any
        device allocation (at most 1024 samples); asynchronous on the network's stream."""
        import torch
        if not (isinstance(out, torch.Tensor) and out.is_cuda and out.is_contiguous()
                and out.dtype == torch.float32 and out.numel() == MLP_PARAMS + 1):
            raise ValueError("out must be a contiguous float32 CUDA tensor of MLP_PARAMS + 1 entries")
        _check(load().wt_mlp_gradient_noalloc(self._h, _dev_ptr(x, "float32", (MLP_INPUTS,)),
                                              _dev_ptr(y, "float32", (MLP_OUTPUTS,)), x.shape[0],
                                              C.c_void_p(out.data_ptr())))

    def train_step(self, x, y, lr, want_loss=True):
        loss = C.c_double()
        _check(load().wt_mlp_train_step(self._h, _dev_ptr(x, "float32", (MLP_INPUTS,)),
                                        _dev_ptr(y, "float32", (MLP_OUTPUTS,)), x.shape[0], float(lr),
                                        C.byref(loss) if want_loss else None))
        return loss.value if want_loss else None


class Ensemble:
    """Members advanced together: one HIP graph launch, or one persistent batched launch, per
    ensemble step (wt_ensemble_*)."""

    def __init__(self, grids):
        self._grids = list(grids)   # keeps the members alive
        arr = (_P * len(self._grids))(*[g._h for g in self._grids])
        lib = load()
        h = lib.wt_ensemble_create(arr, len(self._grids))
        if not h:
            raise WtError(WT_EINVAL, lib.wt_last_error().decode())
        self._h = h
        _register(self)

    def close(self):
        if getattr(self, "_h", None):
            load().wt_ensemble_destroy(self._h)
            self._h = None

    __del__ = close

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def adapt(self, eps):
        e = np.ascontiguousarray(np.broadcast_to(np.asarray(eps, dtype=np.float64), (len(self._grids),)))
        _check(load().wt_ensemble_adapt(self._h, _ptr(e, C.c_double)))

    def step(self, dt):
        d = np.ascontiguousarray(np.broadcast_to(np.asarray(dt, dtype=np.float64), (len(self._grids),)))
        _check(load().wt_ensemble_step(self._h, _ptr(d, C.c_double)))

    def stats(self):
        c, l = C.c_int64(), C.c_int64()
        _check(load().wt_ensemble_stats(self._h, C.byref(c), C.byref(l)))
        return c.value, l.value

    def set_batched(self, on=True):
        """Later steps as one persistent launch over a work queue (True) or one graph (False)."""
        _check(load().wt_ensemble_set_batched(self._h, 1 if on else 0))

    def tuning(self):
        """Launch shape of the batched step: dict of workgroups per CU, entries per chunk, work
        queue (else round-robin), tuning finished, device ms of the last launch."""
        b, c, q, t, ms = C.c_int(), C.c_int(), C.c_int(), C.c_int(), C.c_float()
        _check(load().wt_ensemble_tuning(self._h, C.byref(b), C.byref(c), C.byref(q), C.byref(t), C.byref(ms)))
        return {"workgroups_per_cu": b.value, "chunk_entries": c.value, "work_queue": bool(q.value),
                "tuned": bool(t.value), "last_launch_ms": ms.value}
