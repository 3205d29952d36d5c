"""ctypes binding of libcavmg.so: argument marshalling only.

Every computation happens in the HIP library; this module converts Python /
numpy / torch arguments into the C structures of include/cavmg.h, passes
device pointers of contiguous float64 torch tensors, and turns status codes
into exceptions (warnings are returned in the solve summary).
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref
from typing import Dict, List, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def library_path() -> str:
    return os.path.join(HERE, "libcavmg.so")


class CAVError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"cavmg status {status}: {msg}")
        self.status = status


CAV_LAW = {"target": 0, "membrane": 1, "beam_closed": 2, "beam_open": 3, "csr": 4, "fibre": 5}
FAMILY = {"cav": 0, "vanka": 1, "box": 2}
SMOOTHER = {"additive": 0, "multiplicative": 1}
PRECISION = {"fp64": 0, "mixed": 1}
WARN_NOT_CONVERGED, WARN_FLOOR_LIMITED = 100, 101


class GridDesc(C.Structure):
    _fields_ = [("N", C.c_int32), ("n_levels", C.c_int32), ("rho", C.c_double), ("mu", C.c_double),
                ("dt", C.c_double)]


class StructureDesc(C.Structure):
    _fields_ = [("M", C.c_int32), ("X", C.POINTER(C.c_double)), ("omega", C.POINTER(C.c_double)),
                ("law", C.c_int32), ("kappa_t", C.c_double), ("kappa_s", C.c_double), ("kappa_b", C.c_double),
                ("n_segments", C.c_int32), ("seg_start", C.POINTER(C.c_int32)),
                ("seg_closed", C.POINTER(C.c_int32)), ("seg_ds", C.POINTER(C.c_double)),
                ("E_nnz", C.c_int32), ("E_rowptr", C.POINTER(C.c_int32)), ("E_col", C.POINTER(C.c_int32)),
                ("E_val", C.POINTER(C.c_double)), ("K_p", C.c_double), ("K_t", C.c_double),
                ("clamp_marker", C.c_int32), ("clamp_x", C.c_double), ("clamp_y", C.c_double),
                ("X_force", C.POINTER(C.c_double)), ("X_disp", C.POINTER(C.c_double)),
                ("links", C.POINTER(C.c_double))]


class NewtonOpts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("atol", C.c_double), ("max_newton", C.c_int32), ("lin_rtol", C.c_double),
                ("lin_max_it", C.c_int32), ("family", C.c_int32), ("precision", C.c_int32),
                ("cond_threshold", C.c_double), ("smoother", C.c_int32), ("alpha", C.c_double)]


class NewtonInfo(C.Structure):
    _fields_ = [("newton_its", C.c_int32), ("converged", C.c_int32), ("fgmres_its_total", C.c_int32),
                ("fgmres_its_max", C.c_int32), ("res0", C.c_double), ("res", C.c_double),
                ("lin_unconverged", C.c_int32), ("failed_stage", C.c_int32)]


class LevelStats(C.Structure):
    _fields_ = [("N", C.c_int32), ("n_patches", C.c_int32), ("n_explicit", C.c_int32), ("max_np", C.c_int32),
                ("avg_np", C.c_double), ("sum_np2", C.c_int64), ("n_touched", C.c_int64), ("ee_nnz", C.c_int64)]


class FactorStats(C.Structure):
    _fields_ = [("n_fp64", C.c_int32), ("n_fp32", C.c_int32), ("max_cond", C.c_double),
                ("factor_bytes", C.c_int64), ("coarse_cond_est", C.c_double)]


class FgmresOpts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("max_it", C.c_int32), ("use_learned", C.c_int32),
                ("history", C.POINTER(C.c_double))]


class SolveInfo(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("converged", C.c_int32), ("est_rel_residual", C.c_double),
                ("true_rel_residual", C.c_double), ("pressure_mean_removed", C.c_double),
                ("learned_accepted", C.c_int32), ("learned_rejected", C.c_int32)]


class BatchStats(C.Structure):
    _fields_ = [("rounds", C.c_int32), ("graph_launches", C.c_int32), ("captures", C.c_int32),
                ("iterations", C.c_int64)]


class KernelTiming(C.Structure):
    _fields_ = [("launches", C.c_int64), ("ms", C.c_double), ("bytes", C.c_double), ("vcycles", C.c_int64),
                ("vcycle_ms", C.c_double), ("coop_launches", C.c_int64), ("coop_ms", C.c_double),
                ("coop_bytes", C.c_double), ("shared_launches", C.c_int64), ("shared_ms", C.c_double),
                ("shared_bytes", C.c_double), ("flow_launches", C.c_int64), ("flow_ms", C.c_double),
                ("flow_bytes", C.c_double)]


_P = C.c_void_p
_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class Allocator(C.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("user", C.c_void_p)]


class MemoryInfo(C.Structure):
    _fields_ = [("live_bytes", C.c_int64), ("live_blocks", C.c_int64), ("cached_bytes", C.c_int64),
                ("hip_malloc_calls", C.c_int64), ("allocator_allocs", C.c_int64), ("allocator_frees", C.c_int64)]


class TorchAllocator:
    """cav_allocator backed by PyTorch's caching allocator on one device: the
    library's device memory is torch memory, allocated and released on the
    stream the library passes (stream-ordered reuse). Counts its calls."""

    def __init__(self, device: int):
        import torch
        self._torch = torch
        self.device = int(device)
        self.allocs = 0
        self.frees = 0
        self.live_bytes = 0
        self._sizes = {}

        def _alloc(nbytes, stream, user):
            try:
                p = int(torch.cuda.caching_allocator_alloc(int(nbytes), self.device, int(stream or 0)))
            except Exception:
                return None
            self.allocs += 1
            self.live_bytes += int(nbytes)
            self._sizes[p] = int(nbytes)
            return p

        def _free(ptr, stream, user):
            try:
                torch.cuda.caching_allocator_delete(int(ptr))
            except Exception:
                return
            self.frees += 1
            self.live_bytes -= self._sizes.pop(int(ptr), 0)

        # keep the callbacks alive as long as this object
        self._cfn = (_ALLOC_FN(_alloc), _FREE_FN(_free))
        self.struct = Allocator(self._cfn[0], self._cfn[1], None)


_SIGS = {
    "cav_kernel_timing": ([_P, C.c_int, C.POINTER(KernelTiming)], C.c_int),
    "cav_analyze": ([C.POINTER(GridDesc), C.POINTER(StructureDesc), C.c_int, C.POINTER(_P)], C.c_int),
    "cav_analysis_destroy": ([_P], C.c_int),
    "cav_analysis_export_ee": ([_P, C.c_int, C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.POINTER(C.c_double),
                                C.POINTER(C.c_int64)], C.c_int),
    "cav_analysis_export_patches": ([_P, C.c_int, C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                                     C.POINTER(C.c_int64)], C.c_int),
    "cav_analysis_export_phases": ([_P, C.c_int, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                    C.POINTER(C.c_int32)], C.c_int),
    "cav_analysis_export_weights": ([_P, C.c_int, C.POINTER(C.c_int32), C.POINTER(C.c_double),
                                     C.POINTER(C.c_int32)], C.c_int),
    "cav_export_phases": ([_P, C.c_int, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                           C.POINTER(C.c_int32)], C.c_int),
    "cav_create": ([C.POINTER(_P), C.c_int, _P, C.POINTER(Allocator)], C.c_int),
    "cav_memory_stats": ([_P, C.POINTER(MemoryInfo)], C.c_int),
    "cav_destroy": ([_P], C.c_int),
    "cav_set_stream": ([_P, _P], C.c_int),
    "cav_status_string": ([C.c_int], C.c_char_p),
    "cav_last_error": ([_P], C.c_char_p),
    "cav_build_operator": ([_P, C.POINTER(GridDesc), C.POINTER(StructureDesc)], C.c_int),
    "cav_build_cav_patches": ([_P, C.c_int, C.POINTER(LevelStats)], C.c_int),
    "cav_factor_patches": ([_P, C.c_int, C.c_double, C.POINTER(FactorStats)], C.c_int),
    "cav_set_smoother": ([_P, C.c_int, C.c_double, C.c_int, C.c_int], C.c_int),
    "cav_apply_operator": ([_P, _P, _P], C.c_int),
    "cav_vcycle": ([_P, _P, _P], C.c_int),
    "cav_vcycle_multi": ([_P, C.c_int32, _P, _P], C.c_int),
    "cav_fgmres_solve": ([_P, _P, _P, C.POINTER(FgmresOpts), C.POINTER(SolveInfo)], C.c_int),
    "cav_fgmres_solve_noalloc": ([_P, _P, _P, C.POINTER(FgmresOpts), C.POINTER(SolveInfo)], C.c_int),
    "cav_level_apply": ([_P, C.c_int, C.c_int, _P, _P], C.c_int),
    "cav_level_N": ([_P, C.c_int], C.c_int32),
    "cav_export_patches": ([_P, C.c_int, C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.POINTER(C.c_int64)], C.c_int),
    "cav_export_ee": ([_P, C.c_int, C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.POINTER(C.c_double),
                       C.POINTER(C.c_int64)], C.c_int),
    "cav_net_create": ([C.POINTER(_P), C.c_int, _P, C.POINTER(Allocator)], C.c_int),
    "cav_net_destroy": ([_P], C.c_int),
    "cav_net_set_stream": ([_P, _P], C.c_int),
    "cav_net_last_error": ([_P], C.c_char_p),
    "cav_net_set_weights": ([_P, C.POINTER(C.c_float)], C.c_int),
    "cav_net_get_weights": ([_P, C.POINTER(C.c_float), C.POINTER(C.c_float)], C.c_int),
    "cav_net_forward": ([_P, C.c_int32, C.c_int32, _P, _P], C.c_int),
    "cav_net_correct": ([_P, C.c_int32, _P, _P], C.c_int),
    "cav_net_train_step": ([_P, C.c_int32, C.c_int32, _P, _P, C.POINTER(C.c_int32), C.c_int64, C.c_double,
                            C.POINTER(C.c_double)], C.c_int),
    "cav_net_train_step_residual": ([_P, _P, C.c_int32, C.c_int32, _P, C.POINTER(C.c_int32), C.c_int64, C.c_double,
                                     C.POINTER(C.c_double)], C.c_int),
    "cav_learned_pairs": ([_P, C.c_int32, _P, C.c_int32, _P, _P], C.c_int),
    "cav_autotune": ([_P, C.c_int32, C.POINTER(C.c_int32)], C.c_int),
    "cav_set_level_smoother": ([_P, C.c_int, C.c_int, C.c_double], C.c_int),
    "cav_error_propagation": ([_P, C.c_int32, _P, _P], C.c_int),
    "cav_set_phase_order": ([_P, C.c_int], C.c_int),
    "cav_set_factor_layout": ([_P, C.c_int], C.c_int),
    "cav_set_wait_limit": ([_P, C.c_uint32], C.c_int),
    "cav_build_box_patches": ([_P, C.c_int, C.c_int, C.POINTER(LevelStats)], C.c_int),
    "cav_analyze_box": ([C.POINTER(GridDesc), C.POINTER(StructureDesc), C.c_int, C.c_int, C.POINTER(_P)], C.c_int),
    "cav_set_tuning": ([_P, C.POINTER(C.c_int32)], C.c_int),
    "cav_fgmres_solve_graph": ([_P, _P, _P, C.POINTER(FgmresOpts), C.POINTER(SolveInfo)], C.c_int),
    "cav_batch_solve": ([C.POINTER(_P), C.c_int32, C.POINTER(_P), C.POINTER(_P), C.POINTER(FgmresOpts),
                         C.POINTER(SolveInfo), C.c_int32, C.POINTER(BatchStats)], C.c_int),
    "cav_attach_net": ([_P, _P, C.c_double], C.c_int),
    "cav_ib_interpolate": ([_P, _P, _P], C.c_int),
    "cav_ib_spread_add": ([_P, _P, _P], C.c_int),
    "cav_structure_force": ([C.POINTER(StructureDesc), C.POINTER(C.c_double)], C.c_int),
    "cav_newton_solve": ([_P, C.POINTER(GridDesc), C.POINTER(StructureDesc), _P, _P, C.POINTER(C.c_double),
                          C.POINTER(NewtonOpts), C.POINTER(NewtonInfo)], C.c_int),
}
NET_WEIGHTS = 10944
EXPORTED_SYMBOLS = tuple(_SIGS)

_lib = None


def lib():
    """Load libcavmg.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        path = library_path()
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: build the HIP library first (__graft_entry__.build())")
        L = C.CDLL(path)
        for name, (args, res) in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _arr(a, ctype):
    return a.ctypes.data_as(C.POINTER(ctype)) if a is not None and a.size else None


def _fibre_config(d, X_force=None, X_disp=None, links=None):
    """Set the fibre law's evaluation configuration on a StructureDesc; returns
    the arrays the descriptor points into (keep them alive)."""
    keep = []
    for name, a in (("X_force", X_force), ("X_disp", X_disp), ("links", links)):
        if a is not None:
            a = np.ascontiguousarray(np.asarray(a, dtype=np.float64).ravel())
            setattr(d, name, _arr(a, C.c_double))
            keep.append(a)
    return tuple(keep)


def structure_force(system, X_force=None, X_disp=None, links=None) -> np.ndarray:
    """Host force density of the fibre law, interleaved 2M (cav_structure_force):
    at X_force, or at the markers displaced by X_disp with incrementally updated
    links (from `links`, else the markers' differences), else at the markers."""
    d, keep = describe_structure(system)
    keep = keep + _fibre_config(d, X_force, X_disp, links)
    F = np.zeros(2 * d.M, dtype=np.float64)
    st = lib().cav_structure_force(C.byref(d), _arr(F, C.c_double))
    del keep
    if st != 0:
        raise CAVError(st, "cav_structure_force failed")
    return F


def describe_structure(system):
    """Marshal a workloads.System's structure into StructureDesc (keeps arrays alive)."""
    X = np.ascontiguousarray(system.markers().ravel(), dtype=np.float64)
    om = np.ascontiguousarray(system.weights(), dtype=np.float64)
    segs = system.segments
    start = np.zeros(len(segs) + 1, dtype=np.int32)
    start[1:] = np.cumsum([len(s.X) for s in segs])
    closed = np.array([1 if s.closed else 0 for s in segs], dtype=np.int32)
    ds = np.array([s.ds for s in segs], dtype=np.float64)
    k = system.kappa
    d = StructureDesc()
    d.M = int(len(om))
    d.X = _arr(X, C.c_double)
    d.omega = _arr(om, C.c_double)
    d.law = CAV_LAW[system.law]
    d.kappa_t = float(k.get("kappa_t", 0.0))
    d.kappa_s = float(k.get("kappa_s", k.get("K_s", 0.0)))
    d.kappa_b = float(k.get("kappa_b", k.get("EI", 0.0)))
    d.K_p = float(k.get("K_p", 0.0))
    d.K_t = float(k.get("K_t", 0.0))
    d.clamp_marker = int(k.get("m", 0))
    d.clamp_x = float(k.get("clamp_x", 0.0))
    d.clamp_y = float(k.get("clamp_y", 0.0))
    d.n_segments = len(segs)
    d.seg_start = _arr(start, C.c_int32)
    d.seg_closed = _arr(closed, C.c_int32)
    d.seg_ds = _arr(ds, C.c_double)
    return d, (X, om, start, closed, ds)


class Analysis:
    """Host-only setup of one system (no device): E_E per level, patch sets,
    multiplicative phases and partition-of-unity weights, from libcavmg."""

    def __init__(self, system, family: str = "cav", box=(4, 2), X_force=None):
        self._L = lib()
        g = GridDesc(system.N, system.n_levels, system.rho, system.mu, system.dt)
        d, keep = describe_structure(system)
        keep = keep + _fibre_config(d, X_force)
        h = C.c_void_p()
        if family == "box":
            st = self._L.cav_analyze_box(C.byref(g), C.byref(d), int(box[0]), int(box[1]), C.byref(h))
        else:
            st = self._L.cav_analyze(C.byref(g), C.byref(d), FAMILY[family], C.byref(h))
        del keep
        if st != 0:
            raise CAVError(st, "cav_analyze failed")
        self._h = h
        self.N, self.n_levels = system.N, system.n_levels

    def close(self):
        if getattr(self, "_h", None):
            self._L.cav_analysis_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def level_N(self, level):
        return self.N >> (self.n_levels - 1 - level)

    def ee(self, level):
        nnz = C.c_int64()
        self._L.cav_analysis_export_ee(self._h, level, None, None, None, C.byref(nnz))
        N = self.level_N(level)
        rp = np.zeros(2 * N * N + 1, dtype=np.int64)
        col = np.zeros(nnz.value, dtype=np.int32)
        val = np.zeros(nnz.value, dtype=np.float64)
        self._L.cav_analysis_export_ee(self._h, level, _arr(rp, C.c_int64), _arr(col, C.c_int32),
                                       _arr(val, C.c_double), C.byref(nnz))
        return rp, col, val

    def patches(self, level):
        tot = C.c_int64()
        self._L.cav_analysis_export_patches(self._h, level, None, None, C.byref(tot))
        N = self.level_N(level)
        off = np.zeros(N * N + 1, dtype=np.int64)
        dofs = np.zeros(tot.value, dtype=np.int32)
        self._L.cav_analysis_export_patches(self._h, level, _arr(off, C.c_int64), _arr(dofs, C.c_int32), C.byref(tot))
        return [dofs[off[c]:off[c + 1]] for c in range(N * N)]

    def phases(self, level):
        nph, ncell = C.c_int32(), C.c_int32()
        self._L.cav_analysis_export_phases(self._h, level, None, None, C.byref(nph), C.byref(ncell))
        ptr = np.zeros(nph.value + 1, dtype=np.int32)
        cells = np.zeros(ncell.value, dtype=np.int32)
        self._L.cav_analysis_export_phases(self._h, level, _arr(ptr, C.c_int32), _arr(cells, C.c_int32),
                                           C.byref(nph), C.byref(ncell))
        return [cells[ptr[k]:ptr[k + 1]].tolist() for k in range(nph.value)]

    def weights(self, level):
        nt = C.c_int32()
        self._L.cav_analysis_export_weights(self._h, level, None, None, C.byref(nt))
        dofs = np.zeros(nt.value, dtype=np.int32)
        inv = np.zeros(nt.value, dtype=np.float64)
        self._L.cav_analysis_export_weights(self._h, level, _arr(dofs, C.c_int32), _arr(inv, C.c_double), C.byref(nt))
        return dofs, inv


# Contexts and nets still open at interpreter exit are closed by an atexit
# hook, while torch (their allocator) is still intact.
_LIVE = weakref.WeakSet()


@atexit.register
def _close_all():
    for o in list(_LIVE):
        try:
            o.close()
        except Exception:
            pass


def _dev_ptr(t, dtype=None):
    import torch
    dtype = torch.float64 if dtype is None else dtype
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise TypeError(f"expected a contiguous {dtype} tensor on a ROCm device")
    return C.c_void_p(t.data_ptr())


class Net:
    """Learned correction net (3x3 periodic convs 3 -> 32 -> 32 -> 3) on one device:
    forward, FP64 correction, Adam training steps; weights live on the device."""

    def __init__(self, device: int = 0, weights: Optional[np.ndarray] = None, allocator="torch"):
        import torch
        self._torch = torch
        self.device = torch.device("cuda", device)
        self._L = lib()
        self.allocator = TorchAllocator(device) if allocator == "torch" else allocator
        h = C.c_void_p()
        st = self._L.cav_net_create(C.byref(h), int(device), self._stream(),
                                    C.byref(self.allocator.struct) if self.allocator is not None else None)
        if st != 0:
            raise CAVError(st, "cav_net_create failed")
        self._h = h
        _LIVE.add(self)
        if weights is not None:
            self.set_weights(weights)

    def _stream(self):
        return C.c_void_p(self._torch.cuda.current_stream(self.device).cuda_stream)

    def _check(self, st):
        if st != 0:
            raise CAVError(st, self._L.cav_net_last_error(self._h).decode())

    def _sync_stream(self):
        self._L.cav_net_set_stream(self._h, self._stream())

    def close(self):
        if getattr(self, "_h", None):
            self._L.cav_net_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_weights(self, w) -> None:
        self._sync_stream()
        w = np.ascontiguousarray(w, dtype=np.float32)
        if w.shape != (NET_WEIGHTS,):
            raise ValueError(f"expected {NET_WEIGHTS} weights")
        self._check(self._L.cav_net_set_weights(self._h, _arr(w, C.c_float)))

    def weights(self):
        """(master weights, gradient of the last training step) as float32 numpy arrays."""
        self._sync_stream()
        w = np.zeros(NET_WEIGHTS, dtype=np.float32)
        g = np.zeros(NET_WEIGHTS, dtype=np.float32)
        self._check(self._L.cav_net_get_weights(self._h, _arr(w, C.c_float), _arr(g, C.c_float)))
        return w, g

    def forward(self, x, N: int):
        """x: float32 device tensor (batch, 3, N, N) -> N(x) of the same shape."""
        self._sync_stream()
        out = self._torch.empty_like(x)
        self._check(self._L.cav_net_forward(self._h, int(N), int(x.shape[0]),
                                            _dev_ptr(x, self._torch.float32), _dev_ptr(out, self._torch.float32)))
        return out

    def correct(self, r, N: int):
        """c = ||r|| N(r/||r||) with the pressure mean removed (float64 device vectors)."""
        self._sync_stream()
        c = self._torch.empty_like(r)
        self._check(self._L.cav_net_correct(self._h, int(N), _dev_ptr(r), _dev_ptr(c)))
        return c

    def train_step(self, rhat, ehat, N: int, index=None, lr: float = 1e-3) -> float:
        """One Adam step on samples `index` (host ints) of rhat/ehat (float32 device,
        n_samples x 3N^2); returns the loss before the update."""
        self._sync_stream()
        f32 = self._torch.float32
        ns = int(rhat.shape[0])
        if index is None:
            idx, batch = None, ns
        else:
            idx = np.ascontiguousarray(index, dtype=np.int32)
            batch = int(idx.size)
        loss = C.c_double(0.0)
        self._check(self._L.cav_net_train_step(self._h, int(N), batch, _dev_ptr(rhat, f32), _dev_ptr(ehat, f32),
                                               _arr(idx, C.c_int32) if idx is not None else None, ns, float(lr),
                                               C.byref(loss)))
        return loss.value


class Solver:
    """One solver context on one device; all work runs on the current torch stream."""

    def __init__(self, device: int = 0, allocator="torch"):
        """allocator: "torch" (default: the context's device memory comes from
        PyTorch's caching allocator), None (the library calls hipMalloc), or an
        object with a `struct` field holding a filled Allocator."""
        import torch
        self._torch = torch
        self.device = torch.device("cuda", device)
        self._L = lib()
        self.allocator = TorchAllocator(device) if allocator == "torch" else allocator
        h = C.c_void_p()
        st = self._L.cav_create(C.byref(h), int(device), self._stream(),
                                C.byref(self.allocator.struct) if self.allocator is not None else None)
        if st != 0:
            raise CAVError(st, "cav_create failed (no ROCm device?)")
        self._h = h
        _LIVE.add(self)
        self.N = None
        self.n_levels = None

    def _stream(self):
        return C.c_void_p(self._torch.cuda.current_stream(self.device).cuda_stream)

    def _check(self, st):
        if st not in (0, WARN_NOT_CONVERGED, WARN_FLOOR_LIMITED):
            raise CAVError(st, self._L.cav_last_error(self._h).decode())
        return st

    def _sync_stream(self):
        self._L.cav_set_stream(self._h, self._stream())

    def memory_stats(self) -> Dict:
        m = MemoryInfo()
        self._check(self._L.cav_memory_stats(self._h, C.byref(m)))
        return {f: getattr(m, f) for f, _ in MemoryInfo._fields_}

    def close(self):
        if getattr(self, "_h", None):
            self._L.cav_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- setup ----
    def build_operator(self, system, X_force=None, X_disp=None, links=None) -> None:
        """Operator and hierarchy of `system`; for the fibre law the energies'
        tangent is evaluated at X_force, or at the markers displaced by X_disp
        (links updated incrementally), J and S staying at the markers."""
        self._sync_stream()
        g = GridDesc(system.N, system.n_levels, system.rho, system.mu, system.dt)
        d, keep = describe_structure(system)
        keep = keep + _fibre_config(d, X_force, X_disp, links)
        self._check(self._L.cav_build_operator(self._h, C.byref(g), C.byref(d)))
        del keep
        self.N, self.n_levels = system.N, system.n_levels
        self._ib_rows = 2 * d.M

    def build_cav_patches(self, family: str = "cav", box=(4, 2)) -> List[Dict]:
        """Patch family per smoothed level: 'cav', 'vanka', or 'box' (B(b,o), box = (b, o))."""
        self._sync_stream()
        out = (LevelStats * self.n_levels)()
        if family == "box":
            self._check(self._L.cav_build_box_patches(self._h, int(box[0]), int(box[1]), out))
        else:
            self._check(self._L.cav_build_cav_patches(self._h, FAMILY[family], out))
        return [{f: getattr(o, f) for f, _ in LevelStats._fields_} for o in out]

    def factor_patches(self, precision: str = "fp64", cond_threshold: float = 1e6) -> Dict:
        self._sync_stream()
        st = FactorStats()
        self._check(self._L.cav_factor_patches(self._h, PRECISION[precision], float(cond_threshold), C.byref(st)))
        return {f: getattr(st, f) for f, _ in FactorStats._fields_}

    def set_smoother(self, kind: str = "additive", alpha: float = 0.7, pre: int = 1, post: int = 1) -> None:
        self._check(self._L.cav_set_smoother(self._h, SMOOTHER[kind], float(alpha), int(pre), int(post)))

    def error_propagation(self, X):
        """T = X - V(K X) for every row of X (float64 device (k, n)), 16 at a time."""
        self._sync_stream()
        T = self._torch.empty_like(X)
        self._check(self._L.cav_error_propagation(self._h, int(X.shape[0]), _dev_ptr(X), _dev_ptr(T)))
        return T

    def set_wait_limit(self, polls: int = 1 << 21) -> None:
        """Bound (in polls) of the cooperative kernels' barrier waits; a wait that
        reaches it makes the next solve raise instead of hanging."""
        self._check(self._L.cav_set_wait_limit(self._h, int(polls)))

    def set_phase_order(self, order: str = "standard_first") -> None:
        """Multiplicative sweep order: 'standard_first' (default) or 'explicit_first'."""
        self._check(self._L.cav_set_phase_order(self._h, {"explicit_first": 0, "standard_first": 1}[order]))

    def set_factor_layout(self, layout: str = "full") -> None:
        """Storage of the patch inverses from the next factorisation on: 'full'
        (default) or 'symmetric' (lower panels only; additive smoother only)."""
        self._check(self._L.cav_set_factor_layout(self._h, {"full": 0, "symmetric": 1}[layout]))

    def set_level_smoother(self, level: int, kind: Optional[str], alpha: float = 0.7) -> None:
        """Override the smoother of one smoothed level (None restores the context's)."""
        self._check(self._L.cav_set_level_smoother(self._h, int(level), -1 if kind is None else SMOOTHER[kind],
                                                   float(alpha)))

    def setup(self, system, family="cav", precision="fp64", cond_threshold=1e6, alpha=0.7, smoother="additive",
              box=(4, 2), layout="full"):
        self.set_factor_layout(layout)
        self.build_operator(system)
        stats = self.build_cav_patches(family, box)
        fstats = self.factor_patches(precision, cond_threshold)
        self.set_smoother(smoother, alpha)
        return stats, fstats

    # ---- application ----
    def n(self, level: Optional[int] = None) -> int:
        N = self.N if level is None else int(self._L.cav_level_N(self._h, level))
        return 3 * N * N

    def empty(self, level: Optional[int] = None):
        return self._torch.empty(self.n(level), dtype=self._torch.float64, device=self.device)

    def apply_operator(self, x, out=None):
        self._sync_stream()
        y = self.empty() if out is None else out
        self._check(self._L.cav_apply_operator(self._h, _dev_ptr(x), _dev_ptr(y)))
        return y

    def vcycle(self, r, out=None):
        self._sync_stream()
        z = self.empty() if out is None else out
        self._check(self._L.cav_vcycle(self._h, _dev_ptr(r), _dev_ptr(z)))
        return z

    def vcycle_multi(self, R):
        """Z = V(R) for every row of R (float64 device (k, n)), 16 at a time."""
        self._sync_stream()
        Z = self._torch.empty_like(R)
        self._check(self._L.cav_vcycle_multi(self._h, int(R.shape[0]), _dev_ptr(R), _dev_ptr(Z)))
        return Z

    def level_apply(self, level: int, op: int, x, out_level: Optional[int] = None):
        self._sync_stream()
        y = self.empty(level if out_level is None else out_level)
        self._check(self._L.cav_level_apply(self._h, int(level), int(op), _dev_ptr(x), _dev_ptr(y)))
        return y

    def fgmres_solve(self, b, rtol: float = 1e-10, max_it: int = 150, out=None, history: bool = True,
                     learned: bool = False, graph: bool = False, noalloc: bool = False):
        """FGMRES to rtol; graph=True replays the captured iteration body (same
        results); noalloc=True calls cav_fgmres_solve_noalloc (workspace in the
        library's fixed scratch; pass `out` so the call allocates nothing)."""
        self._sync_stream()
        x = self.empty() if out is None else out
        hist = np.zeros(max_it, dtype=np.float64)
        o = FgmresOpts(float(rtol), int(max_it), 1 if learned else 0, _arr(hist, C.c_double) if history else None)
        info = SolveInfo()
        if graph and noalloc:
            raise ValueError("graph and noalloc are separate entry points")
        fn = (self._L.cav_fgmres_solve_graph if graph else
              self._L.cav_fgmres_solve_noalloc if noalloc else self._L.cav_fgmres_solve)
        st = self._check(fn(self._h, _dev_ptr(b), _dev_ptr(x), C.byref(o), C.byref(info)))
        d = {f: getattr(info, f) for f, _ in SolveInfo._fields_}
        d["status"] = st
        d["history"] = hist[:info.iterations].copy()
        return x, d

    def ib_interpolate(self, x):
        """U = J u at the markers of the last operator build (device, 2M)."""
        self._sync_stream()
        M2 = int(self._ib_rows)
        U = self._torch.empty(M2, dtype=self._torch.float64, device=self.device)
        self._check(self._L.cav_ib_interpolate(self._h, _dev_ptr(x), _dev_ptr(U) if M2 else None))
        return U

    def ib_spread_add(self, F, y):
        """y_u += S F in place (device)."""
        self._sync_stream()
        self._check(self._L.cav_ib_spread_add(self._h, _dev_ptr(F) if F.numel() else None, _dev_ptr(y)))
        return y

    def newton_solve(self, system, rhs, x0=None, rtol: float = 1e-8, atol: float = 1e-8, max_newton: int = 20,
                     lin_rtol: float = 1e-9, lin_max_it: int = 150, family: str = "cav", precision: str = "fp64",
                     cond_threshold: float = 1e6, smoother: str = "multiplicative", alpha: float = 1.0):
        """One backward-Euler IB step with the fibre law by Newton's method
        (cav_newton_solve): returns (x, X_new, info)."""
        self._sync_stream()
        g = GridDesc(system.N, system.n_levels, system.rho, system.mu, system.dt)
        d, keep = describe_structure(system)
        x = self._torch.zeros(3 * system.N * system.N, dtype=self._torch.float64, device=self.device)
        if x0 is not None:
            x.copy_(x0)
        Xn = np.zeros(2 * d.M, dtype=np.float64)
        o = NewtonOpts(float(rtol), float(atol), int(max_newton), float(lin_rtol), int(lin_max_it), FAMILY[family],
                       PRECISION[precision], float(cond_threshold), SMOOTHER[smoother], float(alpha))
        info = NewtonInfo()
        st = self._check(self._L.cav_newton_solve(self._h, C.byref(g), C.byref(d), _dev_ptr(rhs), _dev_ptr(x),
                                                  _arr(Xn, C.c_double), C.byref(o), C.byref(info)))
        del keep
        self.N, self.n_levels = system.N, system.n_levels
        self._ib_rows = 2 * d.M
        out = {f: getattr(info, f) for f, _ in NewtonInfo._fields_}
        out["status"] = st
        return x, Xn, out

    def train_net_residual(self, net: Net, rhat, index=None, lr: float = 1e-3, kind: str = "residual") -> float:
        """One Adam step of `net` on the residual-norm loss through this context's
        finest K_E; rhat float32 device (n_samples, 3N^2); returns the loss."""
        self._sync_stream()
        f32 = self._torch.float32
        ns = int(rhat.shape[0])
        if index is None:
            idx, batch = None, ns
        else:
            idx = np.ascontiguousarray(index, dtype=np.int32)
            batch = int(idx.size)
        loss = C.c_double(0.0)
        self._check(self._L.cav_net_train_step_residual(net._h, self._h, {"residual": 0, "minres": 1}[kind], batch,
                                                        _dev_ptr(rhat, f32),
                                                        _arr(idx, C.c_int32) if idx is not None else None, ns,
                                                        float(lr), C.byref(loss)))
        return loss.value

    def autotune(self, reps: int = 3, cache: Optional[str] = None) -> np.ndarray:
        """Time the phase kernel's thread counts per level and size bucket and keep
        the fastest (cav_autotune); with `cache`, the table is stored as JSON
        under a key for this hierarchy (grid, levels, patch histogram) and reused."""
        import json
        key = None
        if cache is not None:
            key = self._tuning_key()
            try:
                with open(cache) as f:
                    stored = json.load(f).get(key)
            except (OSError, ValueError):
                stored = None
            if stored is not None:
                t = np.ascontiguousarray(stored, dtype=np.int32)
                self.set_tuning(t)
                return t.reshape(self.n_levels, 5)
        self._sync_stream()
        t = np.zeros(5 * self.n_levels, dtype=np.int32)
        self._check(self._L.cav_autotune(self._h, int(reps), _arr(t, C.c_int32)))
        if cache is not None:
            try:
                with open(cache) as f:
                    data = json.load(f)
            except (OSError, ValueError):
                data = {}
            data[key] = t.tolist()
            with open(cache, "w") as f:
                json.dump(data, f, indent=1)
        return t.reshape(self.n_levels, 5)

    def set_tuning(self, table) -> None:
        """Apply a phase-kernel table (n_levels x 5: four bucket entries of 256, 512
        or 1024 threads, 0 for the split form or 1/2 for the cooperative form
        with 64/128 rows per workgroup, then 1 for the one-launch sweep)."""
        t = np.ascontiguousarray(table, dtype=np.int32).ravel()
        self._check(self._L.cav_set_tuning(self._h, _arr(t, C.c_int32)))

    def _tuning_key(self) -> str:
        """gfx950 / grid / levels / patch-count signature of the built hierarchy."""
        parts = [f"gfx950:N{self.N}:L{self.n_levels}"]
        for l in range(1, self.n_levels):
            nph, ncell = C.c_int32(), C.c_int32()
            self._L.cav_export_phases(self._h, l, None, None, C.byref(nph), C.byref(ncell))
            parts.append(f"{nph.value}/{ncell.value}")
        return ":".join(parts)

    def attach_net(self, net: Optional[Net], margin: float = 1e-3) -> None:
        self._check(self._L.cav_attach_net(self._h, net._h if net is not None else None, float(margin)))
        self._net = net  # keep the handle alive while attached

    def learned_pairs(self, xstar, iters: int = 3):
        """(rhat, ehat) float32 device tensors (count*iters, 3N^2) from V-cycle iterations on b = K x*."""
        self._sync_stream()
        count = int(xstar.shape[0])
        t = self._torch
        rh = t.empty((count * iters, self.n()), dtype=t.float32, device=self.device)
        eh = t.empty_like(rh)
        self._check(self._L.cav_learned_pairs(self._h, count, _dev_ptr(xstar), int(iters),
                                              _dev_ptr(rh, t.float32), _dev_ptr(eh, t.float32)))
        return rh, eh

    def kernel_timing(self, enable: bool) -> Dict:
        """Start (True) or stop (False) live HIP-event timing of the explicit-patch
        GEMV and of top-level V-cycles; returns the totals recorded so far."""
        self._sync_stream()
        t = KernelTiming()
        self._check(self._L.cav_kernel_timing(self._h, 1 if enable else 0, C.byref(t)))
        d = {f: getattr(t, f) for f, _ in KernelTiming._fields_}
        d["vcycle_ms"] = d["vcycle_ms"] / d["vcycles"] if d["vcycles"] else 0.0
        return d

    # ---- host exports for parity checks ----
    def export_patches(self, level: int):
        tot = C.c_int64()
        self._check(self._L.cav_export_patches(self._h, level, None, None, C.byref(tot)))
        N = int(self._L.cav_level_N(self._h, level))
        off = np.zeros(N * N + 1, dtype=np.int64)
        dofs = np.zeros(tot.value, dtype=np.int32)
        self._check(self._L.cav_export_patches(self._h, level, _arr(off, C.c_int64), _arr(dofs, C.c_int32),
                                               C.byref(tot)))
        return off, dofs

    def export_phases(self, level: int):
        """Explicit-patch phases of the multiplicative sweep as lists of seed cells."""
        nph, ncell = C.c_int32(), C.c_int32()
        self._check(self._L.cav_export_phases(self._h, level, None, None, C.byref(nph), C.byref(ncell)))
        ptr = np.zeros(nph.value + 1, dtype=np.int32)
        cells = np.zeros(ncell.value, dtype=np.int32)
        self._check(self._L.cav_export_phases(self._h, level, _arr(ptr, C.c_int32), _arr(cells, C.c_int32),
                                              C.byref(nph), C.byref(ncell)))
        return [cells[ptr[k]:ptr[k + 1]].tolist() for k in range(nph.value)]

    def export_ee(self, level: int):
        nnz = C.c_int64()
        self._check(self._L.cav_export_ee(self._h, level, None, None, None, C.byref(nnz)))
        N = int(self._L.cav_level_N(self._h, level))
        rp = np.zeros(2 * N * N + 1, dtype=np.int64)
        col = np.zeros(nnz.value, dtype=np.int32)
        val = np.zeros(nnz.value, dtype=np.float64)
        self._check(self._L.cav_export_ee(self._h, level, _arr(rp, C.c_int64), _arr(col, C.c_int32),
                                          _arr(val, C.c_double), C.byref(nnz)))
        return rp, col, val


def batch_solve(solvers, bs, rtol: float = 1e-10, max_it: int = 150, mode: int = 0):
    """Solve independent systems together (cav_batch_solve): solvers[i] with
    right-hand side bs[i] (float64 device tensors). Returns (xs, infos, stats)."""
    n = len(solvers)
    L = lib()
    for s in solvers:
        s._sync_stream()
    xs = [s.empty() for s in solvers]
    hs = (_P * n)(*[s._h for s in solvers])
    bp = (_P * n)(*[_dev_ptr(b) for b in bs])
    xp = (_P * n)(*[_dev_ptr(x) for x in xs])
    o = FgmresOpts(float(rtol), int(max_it), 0, None)
    infos = (SolveInfo * n)()
    st = BatchStats()
    code = L.cav_batch_solve(hs, n, bp, xp, C.byref(o), infos, int(mode), C.byref(st))
    if code not in (0, WARN_NOT_CONVERGED, WARN_FLOOR_LIMITED):
        raise CAVError(code, L.cav_last_error(solvers[0]._h).decode())
    out = [{f: getattr(i, f) for f, _ in SolveInfo._fields_} for i in infos]
    return xs, out, {f: getattr(st, f) for f, _ in BatchStats._fields_}
