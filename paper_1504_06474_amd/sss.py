"""Python binding of libsss (speculative segmented sum CSR SpMV on gfx950).

Argument marshalling only: every step of the SpMV runs in the HIP kernels of
libsss.so.  PyTorch supplies device memory and streams.  If the library is
not built, importing works but every call raises ``SSSLibraryMissing`` --
there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
# SSS_LIBRARY selects another build of the same C ABI (for A/B timing)
LIB_PATH = os.environ.get("SSS_LIBRARY", os.path.join(HERE, "libsss.so"))

F64, F32, BF16 = 0, 1, 2
MODE_SELECTOR, MODE_GRID, MODE_FIXED = 0, 1, 2
_DTYPES = {torch.float64: F64, torch.float32: F32, torch.bfloat16: BF16}
_XTYPE = {F64: torch.float64, F32: torch.float32, BF16: torch.float32}
_VALTYPE = {F64: torch.float64, F32: torch.float32, BF16: torch.bfloat16}

STATUS = {0: "ok", -1: "invalid value", -2: "unsupported", -3: "plan mismatch", -4: "HIP error",
          -5: "invalid CSR", -6: "too large for the static scratch"}


class SSSLibraryMissing(RuntimeError):
    pass


class SSSError(RuntimeError):
    def __init__(self, status: int, what: str):
        msg = f"{what}: {STATUS.get(status, status)}"
        if status == -4 and _lib is not None:
            msg += f" ({_lib.sss_last_hip_error().decode()})"
        super().__init__(msg)
        self.status = status


class CsrDesc(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p), ("val", ctypes.c_void_p),
                ("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("S", ctypes.c_int), ("reserved", ctypes.c_int)]


class PlanOpts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int), ("W", ctypes.c_int), ("S", ctypes.c_int), ("B", ctypes.c_int),
                ("debug", ctypes.c_int), ("bind_rows", ctypes.c_int), ("batch_persistent", ctypes.c_int),
                ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t)]


_lib = None


def lib():
    """Load libsss.so (once).  Raises SSSLibraryMissing if it is not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise SSSLibraryMissing(f"{LIB_PATH} is not built; run paper_1504_06474_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        P, I64, I = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
        FP_ = ctypes.POINTER(ctypes.c_float)
        L.sss_csr_spmv_plan_create.argtypes = [I64, I64, I64, P, I, ctypes.POINTER(PlanOpts), P,
                                               ctypes.POINTER(P)]
        L.sss_csr_spmv_plan_workspace_size.argtypes = [I64, I64, I64, I, ctypes.POINTER(PlanOpts),
                                                       ctypes.POINTER(ctypes.c_size_t)]
        L.sss_csr_spmv_execute.argtypes = [P, P, P, P, P, P, P]
        L.sss_csr_spmv.argtypes = [I64, I64, I64, P, P, P, P, P, P]
        L.sss_csr_spmv_noalloc.argtypes = [I64, I64, I64, P, P, P, P, P, P]
        L.sss_csr_spmv_stage1.argtypes = [P, P, P, P, P, P, P]
        L.sss_csr_spmv_stage2.argtypes = [P, P, P, P]
        L.sss_plan_destroy.argtypes = [P]
        L.sss_batch_plan_create.argtypes = [I, ctypes.POINTER(CsrDesc), I, ctypes.POINTER(PlanOpts), P,
                                            ctypes.POINTER(P)]
        L.sss_batch_execute.argtypes = [P, P]
        L.sss_batch_plan_schedule.argtypes = [P, I, ctypes.POINTER(I), ctypes.POINTER(I)]
        L.sss_selector_scores.argtypes = [FP_, FP_]
        L.sss_batch_floor_probe.argtypes = [P, P, I, P]
        FP = ctypes.POINTER(ctypes.c_float)
        L.sss_class_params.argtypes = [I, ctypes.POINTER(I), ctypes.POINTER(I)]
        L.sss_csr_features.argtypes = [I64, I64, I64, P, I, P, FP]
        L.sss_csr_spmv_autotune.argtypes = [I64, I64, I64, P, P, P, P, P, I, I, P, FP, ctypes.POINTER(I)]
        L.sss_floor_probe.argtypes = [P, P, P, P, P, I, P]
        L.sss_gather_probe.argtypes = [P, P, P, I64, I64, I, I, I, I, I, P, I64, ctypes.POINTER(I64),
                                       ctypes.POINTER(I), P]
        L.sss_gather_probe_rows.argtypes = [P, P, P, I64, I64, I, I, I, I, I, P, I64, ctypes.POINTER(I64),
                                            ctypes.POINTER(I), P, I64, P, P]
        L.sss_probe_last_hip_error.restype = ctypes.c_char_p
        L.sss_csr_spmv_stage2_host.argtypes = [P, P, P]
        L.sss_csr_rowwise.argtypes = [I64, I64, I64, P, P, P, P, P, I, I, P]
        L.sss_rowwise_last_hip_error.restype = ctypes.c_char_p
        L.sss_batch_plan_create_grid.argtypes = [I, ctypes.POINTER(CsrDesc), I, I, P, FP, ctypes.POINTER(I),
                                                 ctypes.POINTER(P)]
        L.sss_csr_spmv_plan_create_grid.argtypes = [I64, I64, I64, P, P, P, P, P, I, I, P, ctypes.POINTER(P)]
        L.sss_mlp_forward.argtypes = [P, P, I, P, P, P, P]
        L.sss_mlp_backward.argtypes = [P, P, P, P, P, P, I, P, P, P, P]
        L.sss_mlp_adam.argtypes = [P, P, P, P, I, I, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                   ctypes.c_float, P]
        L.sss_selector_set.argtypes = [FP, FP, FP]
        L.sss_selector_predict.argtypes = [FP, ctypes.POINTER(I)]
        L.sss_batch_graph_launch.argtypes = [P, P]
        L.sss_plan_info.argtypes = [P, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(I),
                                    ctypes.POINTER(I64), ctypes.POINTER(I64)]
        L.sss_plan_shape.argtypes = [P, ctypes.POINTER(I64), ctypes.POINTER(I64), ctypes.POINTER(I64),
                                     ctypes.POINTER(I)]
        L.sss_cg_workspace_size.argtypes = [ctypes.POINTER(ctypes.c_size_t)]
        L.sss_cg_start.argtypes = [P, P, P, P, P, P, P, P, P, P, P]
        L.sss_cg_iterate.argtypes = [P, P, P, P, P, P, P, P, P, I, P]
        L.sss_cg_last_hip_error.restype = ctypes.c_char_p
        L.sss_validate_csr.argtypes = [I64, I64, I64, P, P, P]
        L.sss_plan_debug_size.argtypes = [P, ctypes.POINTER(ctypes.c_size_t)]
        L.sss_plan_debug_dump.argtypes = [P, P, ctypes.c_size_t]
        L.sss_plan_dirty_list.argtypes = [P, P, I64, ctypes.POINTER(I64)]
        L.sss_status_string.argtypes = [I]
        L.sss_status_string.restype = ctypes.c_char_p
        L.sss_last_hip_error.restype = ctypes.c_char_p
        L.sss_version.restype = ctypes.c_char_p
        for f in ("sss_csr_spmv_plan_create", "sss_csr_spmv_plan_workspace_size", "sss_csr_spmv_execute", "sss_csr_spmv",
                  "sss_csr_spmv_noalloc", "sss_csr_spmv_cache_clear",
                  "sss_plan_destroy",
                  "sss_csr_spmv_stage1", "sss_csr_spmv_stage2",
                  "sss_plan_info", "sss_validate_csr", "sss_plan_debug_size", "sss_plan_debug_dump",
                  "sss_plan_dirty_list", "sss_batch_plan_create", "sss_batch_execute", "sss_batch_graph_launch", "sss_batch_floor_probe",
                  "sss_class_params", "sss_csr_features", "sss_csr_spmv_autotune", "sss_csr_spmv_plan_create_grid", "sss_floor_probe", "sss_batch_plan_create_grid", "sss_csr_rowwise", "sss_csr_spmv_stage2_host", "sss_mlp_forward",
                  "sss_mlp_backward", "sss_mlp_adam", "sss_selector_set", "sss_selector_predict",
                  "sss_selector_loaded", "sss_gather_probe", "sss_gather_probe_rows", "sss_batch_plan_schedule", "sss_selector_scores",
                  "sss_plan_shape", "sss_cg_workspace_size", "sss_cg_start", "sss_cg_iterate"):
            getattr(L, f).restype = I
        _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc != 0:
        raise SSSError(rc, what)


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    if t is None:
        return None
    if t.device.type != "cuda":
        raise ValueError("tensors must be on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensors must be contiguous")
    return t.data_ptr() if t.numel() else None


def _check_csr(row_ptr: torch.Tensor, col: torch.Tensor, val: torch.Tensor, x: Optional[torch.Tensor],
               y: Optional[torch.Tensor], n: int):
    """The sizes a CSR call implies (m = row_ptr entries - 1, nnz = val
    entries), checked before any pointer reaches the library."""
    if row_ptr.dtype != torch.int32 or row_ptr.numel() < 1:
        raise ValueError("row_ptr must be int32 with m + 1 entries")
    if col.dtype != torch.int32 or col.numel() < val.numel():
        raise ValueError("col must be int32 with at least nnz (= val's length) entries")
    if x is not None and x.numel() < n:
        raise ValueError("x must hold n entries")
    if y is not None and y.numel() < row_ptr.numel() - 1:
        raise ValueError("y must hold m entries")


def _stream(stream) -> Optional[int]:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def workspace_size(m: int, n: int, nnz: int, dtype=torch.float64, W: int = 0, S: int = 0,
                   debug: bool = False, mode: int = MODE_FIXED, bind_rows: bool = False) -> int:
    """Bytes of device workspace a plan with these options needs
    (sss_csr_spmv_plan_workspace_size)."""
    dt = _DTYPES[dtype] if isinstance(dtype, torch.dtype) else int(dtype)
    opts = PlanOpts(mode, W, S, 0, 1 if debug else 0, 1 if bind_rows else 0)
    b = ctypes.c_size_t()
    _check(lib().sss_csr_spmv_plan_workspace_size(int(m), int(n), int(nnz), dt, ctypes.byref(opts),
                                                   ctypes.byref(b)), "sss_csr_spmv_plan_workspace_size")
    return b.value


class Plan:
    """A plan for y = A x on an m x n matrix with nnz nonzeros (sss_csr_spmv_plan_create).
    Its auxiliary arrays live in a uint8 tensor from PyTorch's allocator on
    `device` (the plan's workspace), held by this object."""

    def __init__(self, m: int, n: int, nnz: int, dtype=torch.float64, W: int = 0, S: int = 0, B: int = 0,
                 debug: bool = False, mode: int = MODE_FIXED, row_ptr: Optional[torch.Tensor] = None,
                 bind_rows: bool = False, stream=None, device=None):
        L = lib()
        self.m, self.n, self.nnz = int(m), int(n), int(nnz)
        self.dt = _DTYPES[dtype] if isinstance(dtype, torch.dtype) else int(dtype)
        if mode == MODE_SELECTOR and not L.sss_selector_loaded():
            load_selector()  # the network shipped with the package, once per device
        if device is None:
            device = row_ptr.device if row_ptr is not None else torch.device("cuda", torch.cuda.current_device())
        nbytes = workspace_size(m, n, nnz, self.dt, W, S, debug, mode, bind_rows)
        # 256-byte alignment: PyTorch's caching allocator hands out blocks aligned to 512 bytes
        self._ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=device)
        opts = PlanOpts(mode, W, S, B, 1 if debug else 0, 1 if bind_rows else 0, 0, self._ws.data_ptr(), nbytes)
        h = ctypes.c_void_p()
        rc = L.sss_csr_spmv_plan_create(self.m, self.n, self.nnz, _ptr(row_ptr), self.dt, ctypes.byref(opts),
                                        _stream(stream), ctypes.byref(h))
        _check(rc, "sss_csr_spmv_plan_create")
        self._h = h

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        W, S, B = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        nt, nb = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().sss_plan_info(self._h, ctypes.byref(W), ctypes.byref(S), ctypes.byref(B), ctypes.byref(nt),
                                   ctypes.byref(nb)), "sss_plan_info")
        return {"W": W.value, "S": S.value, "B": B.value, "n_tiles": nt.value, "n_bunches": nb.value}

    def _check_rows(self, row_ptr: torch.Tensor, y: torch.Tensor):
        if row_ptr.dtype != torch.int32 or row_ptr.numel() != self.m + 1:
            raise ValueError("row_ptr must be int32 with m + 1 entries")
        if y.dtype != _XTYPE[self.dt] or y.numel() < self.m:
            raise ValueError("y must be of the plan's y type with at least m entries")

    def _check_arrays(self, row_ptr, col, val, x, y):
        """The sizes and types the plan was made for (the C entry points
        receive bare pointers and cannot check them)."""
        self._check_rows(row_ptr, y)
        if val.dtype != _VALTYPE[self.dt] or x.dtype != _XTYPE[self.dt]:
            raise TypeError("val/x dtypes do not match the plan")
        if col.dtype != torch.int32 or col.numel() < self.nnz or val.numel() < self.nnz:
            raise ValueError("col (int32) and val must hold nnz entries")
        if x.numel() < self.n:
            raise ValueError("x too short")

    def execute(self, row_ptr: torch.Tensor, col: torch.Tensor, val: torch.Tensor, x: torch.Tensor,
                y: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        if y is None:
            y = torch.empty(self.m, dtype=_XTYPE[self.dt], device=x.device)
        self._check_arrays(row_ptr, col, val, x, y)
        rc = lib().sss_csr_spmv_execute(self._h, _ptr(row_ptr), _ptr(col), _ptr(val), _ptr(x), _ptr(y),
                                        _stream(stream))
        _check(rc, "sss_csr_spmv_execute")
        return y

    def stage1(self, row_ptr, col, val, x, y, stream=None):
        """Speculative execution only (sss_csr_spmv_stage1)."""
        self._check_arrays(row_ptr, col, val, x, y)
        _check(lib().sss_csr_spmv_stage1(self._h, _ptr(row_ptr), _ptr(col), _ptr(val), _ptr(x), _ptr(y),
                                         _stream(stream)), "sss_csr_spmv_stage1")

    def stage2(self, row_ptr, y, stream=None):
        """Checking prediction only (sss_csr_spmv_stage2)."""
        self._check_rows(row_ptr, y)
        _check(lib().sss_csr_spmv_stage2(self._h, _ptr(row_ptr), _ptr(y), _stream(stream)), "sss_csr_spmv_stage2")

    def dirty_list(self) -> np.ndarray:
        """The thread-bunches a bind_rows plan listed at plan time as holding
        a dirty tile (sss_plan_dirty_list)."""
        n = ctypes.c_int64()
        _check(lib().sss_plan_dirty_list(self._h, None, 0, ctypes.byref(n)), "sss_plan_dirty_list")
        out = np.zeros(max(n.value, 1), dtype=np.int32)
        _check(lib().sss_plan_dirty_list(self._h, out.ctypes.data, n.value, ctypes.byref(n)), "sss_plan_dirty_list")
        return out[:n.value].copy()

    def debug_dump(self) -> dict:
        L = lib()
        size = ctypes.c_size_t()
        _check(L.sss_plan_debug_size(self._h, ctypes.byref(size)), "sss_plan_debug_size")
        buf = np.zeros(size.value, dtype=np.uint8)
        _check(L.sss_plan_debug_dump(self._h, buf.ctypes.data, size.value), "sss_plan_debug_dump")
        hdr = buf[:32].view(np.int64)
        nt, nb, nd, wpt = (int(v) for v in hdr)
        o = 32
        tile_start = buf[o:o + 4 * nt].view(np.int32); o += 4 * nt
        tile_dirty = buf[o:o + 4 * nt].view(np.int32); o += 4 * nt
        heads = buf[o:o + 4 * nt * wpt].view(np.uint32).reshape(nt, wpt); o += 4 * nt * wpt
        spec = buf[o:o + 16 * nt].view(np.int32).reshape(nt, 4)[:nd]; o += 16 * nt
        sync_idx = buf[o:o + 4 * nb].view(np.int32); o += 4 * nb
        sync_val = buf[o:o + 8 * nb].view(np.float64); o += 8 * nb
        tail_val = buf[o:o + 8 * nb].view(np.float64)
        return {"n_tiles": nt, "n_bunches": nb, "dirty_count": nd, "tile_start": tile_start.copy(),
                "tile_dirty": tile_dirty.copy(), "heads": heads.copy(), "speculator": spec.copy(),
                "sync_idx": sync_idx.copy(), "sync_val": sync_val.copy(), "tail_val": tail_val.copy()}

    def stage2_host(self, row_ptr: np.ndarray, y) -> None:
        """Stage 2 on a host core (sss_csr_spmv_stage2_host), for comparison
        with the device stage 2: row_ptr a host int32 array, y a host array
        (numpy or CPU tensor) of the plan's y type holding stage 1's output."""
        row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
        if row_ptr.shape[0] != self.m + 1:
            raise ValueError("row_ptr must hold m + 1 entries")
        if isinstance(y, torch.Tensor):
            if y.device.type != "cpu" or not y.is_contiguous() or y.dtype != _XTYPE[self.dt] or y.numel() < self.m:
                raise ValueError("y must be a contiguous host tensor of the plan's y type")
            yp = y.data_ptr()
        else:
            if y.dtype != np.dtype(str(_XTYPE[self.dt]).replace("torch.", "")) or not y.flags.c_contiguous or \
                    y.shape[0] < self.m:
                raise ValueError("y must be a contiguous host array of the plan's y type")
            yp = y.ctypes.data
        _check(lib().sss_csr_spmv_stage2_host(self._h, row_ptr.ctypes.data, yp), "sss_csr_spmv_stage2_host")

    def floor_probe(self, col: torch.Tensor, val: torch.Tensor, x: Optional[torch.Tensor], out: torch.Tensor,
                    gather: bool = True, stream=None) -> torch.Tensor:
        """Memory floor of stage 1's access pattern (sss_floor_probe): streams
        col/val with this plan's tiling, gathering x when `gather`; writes one
        sum per lane to `out` (n_bunches * 64 elements of the y type)."""
        if out.numel() < self.info()["n_bunches"] * 64 or out.dtype != _XTYPE[self.dt]:
            raise ValueError("out must hold n_bunches * 64 elements of the plan's y type")
        if val.dtype != _VALTYPE[self.dt] or col.numel() < self.nnz or val.numel() < self.nnz:
            raise ValueError("col/val do not match the plan")
        if gather and (x is None or x.dtype != _XTYPE[self.dt] or x.numel() < self.n):
            raise ValueError("x does not match the plan")
        _check(lib().sss_floor_probe(self._h, _ptr(col), _ptr(val), _ptr(x) if gather else None, _ptr(out),
                                     1 if gather else 0, _stream(stream)), "sss_floor_probe")
        return out

    def close(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _check(_lib.sss_plan_destroy(self._h), "sss_plan_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchPlan:
    """y_i = A_i x_i for many matrices in one launch per stage
    (sss_batch_plan_create).  `mats` is a list of (row_ptr, col, val, x, y, n)
    device tensors (n = number of columns) or dicts with those keys and an
    optional per-matrix "S".  The tensors must stay alive and in place for the
    plan's lifetime.  persistent=True makes stage 1 a persistent grid instead
    of one wavefront per thread-bunch."""

    def __init__(self, mats, dtype=torch.float64, W: int = 0, S: int = 0, B: int = 0, stream=None,
                 persistent: bool = False, mode: int = MODE_FIXED):
        L = lib()
        descs = self._describe(mats, dtype)
        if mode == MODE_SELECTOR and not L.sss_selector_loaded():
            load_selector()
        opts = PlanOpts(mode, W, S, B, 0, 0, 1 if persistent else 0)
        h = ctypes.c_void_p()
        _check(L.sss_batch_plan_create(len(mats), descs, self.dt, ctypes.byref(opts), _stream(stream),
                                       ctypes.byref(h)), "sss_batch_plan_create")
        self._h = h

    @classmethod
    def grid(cls, mats, dtype=torch.float64, reps: int = 3, stream=None):
        """The batch plan with the grid autotuner's tile schedule
        (sss_batch_plan_create_grid); every y is overwritten while timing.
        Returns (plan, per-class microseconds per batch launch, chosen class)."""
        L = lib()
        self = cls.__new__(cls)
        descs = self._describe(mats, dtype)
        us = (ctypes.c_float * N_CLASSES)()
        best = ctypes.c_int()
        h = ctypes.c_void_p()
        _check(L.sss_batch_plan_create_grid(len(mats), descs, self.dt, int(reps), _stream(stream), us,
                                            ctypes.byref(best), ctypes.byref(h)), "sss_batch_plan_create_grid")
        self._h = h
        return self, np.array(us[:], dtype=np.float64), best.value

    def _describe(self, mats, dtype):
        self.dt = _DTYPES[dtype] if isinstance(dtype, torch.dtype) else int(dtype)
        descs = (CsrDesc * max(1, len(mats)))()
        self._keep = []
        for i, mt in enumerate(mats):
            if not isinstance(mt, dict):
                rp, col, val, x, y, n = mt
                mt = {"row_ptr": rp, "col": col, "val": val, "x": x, "y": y, "n": n}
            rp, col, val, x, y = mt["row_ptr"], mt["col"], mt["val"], mt["x"], mt["y"]
            if val.dtype != _VALTYPE[self.dt] or x.dtype != _XTYPE[self.dt] or y.dtype != _XTYPE[self.dt]:
                raise TypeError("val/x/y dtypes do not match the batch dtype")
            _check_csr(rp, col, val, x, y, int(mt["n"]))
            m = rp.numel() - 1
            d = descs[i]
            d.m, d.n, d.nnz = m, int(mt["n"]), int(val.numel())
            d.row_ptr, d.col, d.val, d.x, d.y = _ptr(rp), _ptr(col), _ptr(val), _ptr(x), _ptr(y)
            d.S = int(mt.get("S", 0))
            self._keep.append((rp, col, val, x, y))
        return descs

    def info(self) -> dict:
        return Plan.info(self)

    def schedule(self):
        """(W, per-matrix S) of this plan (sss_batch_plan_schedule)."""
        n = len(self._keep)
        W = ctypes.c_int()
        S = (ctypes.c_int * max(1, n))()
        _check(lib().sss_batch_plan_schedule(self._h, n, ctypes.byref(W), S), "sss_batch_plan_schedule")
        return W.value, list(S[:n])

    def execute(self, stream=None):
        _check(lib().sss_batch_execute(self._h, _stream(stream)), "sss_batch_execute")

    def floor_probe(self, out: torch.Tensor, gather: bool = True, stream=None) -> torch.Tensor:
        """Memory floor of the batched stage 1's access pattern
        (sss_batch_floor_probe): one sum per lane per global bunch in `out`
        (n_bunches * 64 elements of the y type)."""
        if out.numel() < self.info()["n_bunches"] * 64 or out.dtype != _XTYPE[self.dt]:
            raise ValueError("out must hold n_bunches * 64 elements of the plan's y type")
        _check(lib().sss_batch_floor_probe(self._h, _ptr(out), 1 if gather else 0, _stream(stream)),
               "sss_batch_floor_probe")
        return out

    def graph_launch(self, stream=None):
        _check(lib().sss_batch_graph_launch(self._h, _stream(stream)), "sss_batch_graph_launch")

    close = Plan.close
    __del__ = Plan.__del__


# ---------------------------------------------------------------- selection

N_CLASSES, N_FEATURES, MLP_PARAMS = 12, 8, 5516


def class_params(cls: int):
    W, S = ctypes.c_int(), ctypes.c_int()
    _check(lib().sss_class_params(int(cls), ctypes.byref(W), ctypes.byref(S)), "sss_class_params")
    return W.value, S.value


def features(row_ptr: torch.Tensor, n: int, nnz: int, dtype=torch.float64, stream=None) -> np.ndarray:
    """The 8 selector features of a CSR matrix (sss_csr_features)."""
    f = (ctypes.c_float * N_FEATURES)()
    dt = _DTYPES[dtype] if isinstance(dtype, torch.dtype) else int(dtype)
    if row_ptr.dtype != torch.int32 or row_ptr.numel() < 1:
        raise ValueError("row_ptr must be int32 with m + 1 entries")
    _check(lib().sss_csr_features(row_ptr.numel() - 1, int(n), int(nnz), _ptr(row_ptr), dt, _stream(stream), f),
           "sss_csr_features")
    return np.array(f[:], dtype=np.float32)


def autotune(row_ptr, col, val, x, y, n: int, reps: int = 5, stream=None):
    """Median microseconds of every grid class and the fastest class
    (sss_csr_spmv_autotune)."""
    t = (ctypes.c_float * N_CLASSES)()
    best = ctypes.c_int()
    dt = _DTYPES[val.dtype]
    _check_csr(row_ptr, col, val, x, y, int(n))
    _check(lib().sss_csr_spmv_autotune(row_ptr.numel() - 1, int(n), val.numel(), _ptr(row_ptr), _ptr(col),
                                       _ptr(val), _ptr(x), _ptr(y), dt, int(reps), _stream(stream), t,
                                       ctypes.byref(best)), "sss_csr_spmv_autotune")
    return np.array(t[:], dtype=np.float64), best.value


GATHER_MODES = {0: "vector", 1: "nontemporal", 2: "lds_direct", 3: "buffer_sc1"}


def gather_probe(col: torch.Tensor, x: torch.Tensor, out: torch.Tensor, val: Optional[torch.Tensor] = None,
                 mode: int = 0, unroll: int = 8, waves_per_simd: int = 8, stream=None,
                 row_ptr: Optional[torch.Tensor] = None, y: Optional[torch.Tensor] = None):
    """The device's random-gather rate (sss_gather_probe): one nonzero per
    lane per grid-stride iteration, `unroll` gathers in flight; with row_ptr
    and y also the row part (sss_gather_probe_rows: row_ptr read, y written).
    Returns (threads, resident workgroups per CU); out needs >= threads
    entries."""
    dt = _DTYPES[x.dtype]
    if val is not None and val.dtype != x.dtype:
        raise TypeError("val and x must share a type")
    if col.dtype != torch.int32 or (val is not None and val.numel() < col.numel()):
        raise ValueError("col must be int32, and val at least as long")
    th, res = ctypes.c_int64(), ctypes.c_int()
    args = (_ptr(col), _ptr(val), _ptr(x), col.numel(), x.numel(), dt, int(mode), int(unroll), int(waves_per_simd),
            1 if val is not None else 0, _ptr(out), out.numel(), ctypes.byref(th), ctypes.byref(res))
    if row_ptr is None:
        _check(lib().sss_gather_probe(*args, _stream(stream)), "sss_gather_probe")
    else:
        if y is None or y.dtype != x.dtype or y.numel() < row_ptr.numel() - 1:
            raise TypeError("y must be x's type with one entry per row")
        _check(lib().sss_gather_probe_rows(*args, _ptr(row_ptr), row_ptr.numel() - 1, _ptr(y), _stream(stream)),
               "sss_gather_probe_rows")
    return th.value, res.value


def csr_rowwise(row_ptr, col, val, x, y, n: int, lanes_per_row: int, stream=None):
    """Row-wise comparator, not the method (sss_csr_rowwise): 1 lane per row
    is CSR-scalar, 64 is CSR-vector."""
    _check_csr(row_ptr, col, val, x, y, int(n))
    _check(lib().sss_csr_rowwise(row_ptr.numel() - 1, int(n), val.numel(), _ptr(row_ptr), _ptr(col), _ptr(val),
                                 _ptr(x), _ptr(y), _DTYPES[val.dtype], int(lanes_per_row), _stream(stream)),
           "sss_csr_rowwise")
    return y


def cg_workspace_size() -> int:
    """Bytes of the device work array the CG calls need (sss_cg_workspace_size)."""
    b = ctypes.c_size_t()
    _check(lib().sss_cg_workspace_size(ctypes.byref(b)), "sss_cg_workspace_size")
    return b.value


def _check_cg(plan: "Plan", row_ptr, col, val, vectors, work):
    if plan.dt != F64 or plan.m != plan.n:
        raise ValueError("CG needs a square FP64 plan")
    for v in vectors:
        if v.dtype != torch.float64 or v.numel() < plan.m:
            raise ValueError("CG vectors must be float64 with at least m entries")
    plan._check_arrays(row_ptr, col, val, vectors[0], vectors[0])
    if work.numel() * work.element_size() < cg_workspace_size():
        raise ValueError("work must hold cg_workspace_size() bytes")


def cg_start(plan: "Plan", row_ptr, col, val, b, x, r, p, q, work, stream=None):
    """q = A x, r = b - q, p = r, and (r.r, r.r, b.b) in work's first three
    doubles, enqueued on the device (sss_cg_start)."""
    _check_cg(plan, row_ptr, col, val, (b, x, r, p, q), work)
    _check(lib().sss_cg_start(plan.handle, _ptr(row_ptr), _ptr(col), _ptr(val), _ptr(b), _ptr(x), _ptr(r),
                              _ptr(p), _ptr(q), _ptr(work), _stream(stream)), "sss_cg_start")


def cg_iterate(plan: "Plan", row_ptr, col, val, x, r, p, q, work, iterations: int, stream=None):
    """`iterations` CG steps from the state in x, r, p and work, enqueued on
    the device (sss_cg_iterate); q is scratch."""
    _check_cg(plan, row_ptr, col, val, (x, r, p, q), work)
    _check(lib().sss_cg_iterate(plan.handle, _ptr(row_ptr), _ptr(col), _ptr(val), _ptr(x), _ptr(r), _ptr(p),
                                _ptr(q), _ptr(work), int(iterations), _stream(stream)), "sss_cg_iterate")


def plan_grid(row_ptr, col, val, x, y, n: int, reps: int = 5, stream=None) -> "Plan":
    """A plan with the grid's fastest class for this matrix
    (sss_csr_spmv_plan_create_grid; y is overwritten while timing)."""
    h = ctypes.c_void_p()
    dt = _DTYPES[val.dtype]
    _check_csr(row_ptr, col, val, x, y, int(n))
    _check(lib().sss_csr_spmv_plan_create_grid(row_ptr.numel() - 1, int(n), val.numel(), _ptr(row_ptr), _ptr(col),
                                               _ptr(val), _ptr(x), _ptr(y), dt, int(reps), _stream(stream),
                                               ctypes.byref(h)), "sss_csr_spmv_plan_create_grid")
    p = Plan.__new__(Plan)
    p.m, p.n, p.nnz, p.dt, p._h = row_ptr.numel() - 1, int(n), val.numel(), dt, h
    return p


def mlp_forward(params, X, H1, H2, Z, stream=None):
    _check(lib().sss_mlp_forward(_ptr(params), _ptr(X), X.shape[0], _ptr(H1), _ptr(H2), _ptr(Z), _stream(stream)),
           "sss_mlp_forward")


def mlp_backward(params, X, H1, H2, Z, Q, grad, loss, work, stream=None):
    _check(lib().sss_mlp_backward(_ptr(params), _ptr(X), _ptr(H1), _ptr(H2), _ptr(Z), _ptr(Q), X.shape[0],
                                  _ptr(grad), _ptr(loss), _ptr(work), _stream(stream)), "sss_mlp_backward")


def mlp_adam(params, grad, m1, m2, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
    _check(lib().sss_mlp_adam(_ptr(params), _ptr(grad), _ptr(m1), _ptr(m2), params.numel(), int(step), lr, beta1,
                              beta2, eps, _stream(stream)), "sss_mlp_adam")


def selector_set(params: np.ndarray, mean: np.ndarray, std: np.ndarray):
    p = np.ascontiguousarray(params, dtype=np.float32)
    mu = np.ascontiguousarray(mean, dtype=np.float32)
    sd = np.ascontiguousarray(std, dtype=np.float32)
    FP = ctypes.POINTER(ctypes.c_float)
    _check(lib().sss_selector_set(p.ctypes.data_as(FP), mu.ctypes.data_as(FP), sd.ctypes.data_as(FP)),
           "sss_selector_set")


def selector_scores(feats: np.ndarray) -> np.ndarray:
    """The loaded selector's 12 class scores for one feature vector."""
    f = np.ascontiguousarray(feats, dtype=np.float32)
    z = np.zeros(N_CLASSES, dtype=np.float32)
    FP = ctypes.POINTER(ctypes.c_float)
    _check(lib().sss_selector_scores(f.ctypes.data_as(FP), z.ctypes.data_as(FP)), "sss_selector_scores")
    return z


def selector_predict(feats: np.ndarray) -> int:
    f = np.ascontiguousarray(feats, dtype=np.float32)
    c = ctypes.c_int()
    _check(lib().sss_selector_predict(f.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), ctypes.byref(c)),
           "sss_selector_predict")
    return c.value


SELECTOR_FILE = os.path.join(HERE, "selector_params.json")


def load_selector(path: Optional[str] = None) -> bool:
    """Load the trained selector shipped with the package (or `path`) onto the
    current device.  Returns False if there is no such file."""
    import json
    path = path or SELECTOR_FILE
    if not os.path.exists(path):
        return False
    d = json.load(open(path))
    selector_set(np.array(d["params"]), np.array(d["feature_mean"]), np.array(d["feature_std"]))
    return True


def csr_spmv(row_ptr: torch.Tensor, col: torch.Tensor, val: torch.Tensor, x: torch.Tensor,
             y: Optional[torch.Tensor] = None, n: Optional[int] = None, stream=None) -> torch.Tensor:
    """The one-call double-precision form, sss_csr_spmv (internal plan cache)."""
    m = row_ptr.numel() - 1
    n = x.numel() if n is None else int(n)
    nnz = val.numel()
    if y is None:
        y = torch.empty(m, dtype=torch.float64, device=x.device)
    for t in (val, x, y):
        if t.dtype != torch.float64:
            raise TypeError("sss_csr_spmv is the double-precision form")
    _check_csr(row_ptr, col, val, x, y, n)
    rc = lib().sss_csr_spmv(m, n, nnz, _ptr(row_ptr), _ptr(col), _ptr(val), _ptr(x), _ptr(y), _stream(stream))
    _check(rc, "sss_csr_spmv")
    return y


def csr_spmv_noalloc(row_ptr: torch.Tensor, col: torch.Tensor, val: torch.Tensor, x: torch.Tensor,
                     y: torch.Tensor, n: Optional[int] = None, stream=None) -> torch.Tensor:
    """The allocation-free one-call form, sss_csr_spmv_noalloc: y must be given
    (the library allocates nothing; its static scratch serves one call at a
    time per device)."""
    m = row_ptr.numel() - 1
    n = x.numel() if n is None else int(n)
    for t in (val, x, y):
        if t.dtype != torch.float64:
            raise TypeError("sss_csr_spmv_noalloc is the double-precision form")
    _check_csr(row_ptr, col, val, x, y, n)
    rc = lib().sss_csr_spmv_noalloc(m, n, val.numel(), _ptr(row_ptr), _ptr(col), _ptr(val), _ptr(x), _ptr(y),
                                    _stream(stream))
    _check(rc, "sss_csr_spmv_noalloc")
    return y


def csr_spmv_cache_clear():
    """Free the plans csr_spmv (sss_csr_spmv) has cached."""
    _check(lib().sss_csr_spmv_cache_clear(), "sss_csr_spmv_cache_clear")


def validate_csr(row_ptr: torch.Tensor, col: torch.Tensor, n: int, stream=None) -> bool:
    m = row_ptr.numel() - 1
    rc = lib().sss_validate_csr(m, n, col.numel(), _ptr(row_ptr), _ptr(col), _stream(stream))
    if rc == -5:
        return False
    _check(rc, "sss_validate_csr")
    return True


def version() -> str:
    return lib().sss_version().decode()
