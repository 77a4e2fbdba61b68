"""Python binding of libhm (include/hm.h): argument marshalling only.

Every step of the evaluation runs in the HIP kernels of libhm.so; PyTorch is
used only to hold device memory and to name the stream.  If libhm.so is
missing the import fails: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhm.so")

HM_OK, HM_ERR_INVALID, HM_ERR_FORMAT, HM_ERR_NOMEM = 0, -1, -2, -3
HM_ERR_DEVICE, HM_ERR_BUSY, HM_ERR_PENDING, HM_ERR_INTERNAL = -4, -5, -6, -7
HM_F64, HM_F32 = 0, 1
HM_PREC_FP64, HM_PREC_FP32, HM_PREC_BF16X3 = 0, 1, 2
HM_TREE_ORDER, HM_PROFILE, HM_NEAR_FROM_POINTS, HM_FAR_FROM_POINTS, HM_LEVEL_LAUNCHES = 1, 2, 4, 8, 16
HM_LOAD_NO_NEAR_BLOCKS, HM_LOAD_NO_FAR_BLOCKS, HM_LOAD_SYMMETRIC = 1 << 8, 1 << 9, 1 << 10
HM_BATCH_AUTOTUNE, HM_BATCH_NO_GRAPH = 1, 2


def HM_BATCH_TILE(bn: int) -> int:
    """hm_batch_create flag: fix the column tile (16, 32, 64, 128 or 256)."""
    return int(bn) << 8
HM_NOALLOC_SCRATCH_BYTES = 64 << 20
STATUS_NAMES = {0: "HM_OK", -1: "HM_ERR_INVALID", -2: "HM_ERR_FORMAT", -3: "HM_ERR_NOMEM",
                -4: "HM_ERR_DEVICE", -5: "HM_ERR_BUSY", -6: "HM_ERR_PENDING", -7: "HM_ERR_INTERNAL"}


def precbit(p: int) -> int:
    return 1 << p


class HMError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_P = ctypes.c_void_p


class hm_host_repr(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int64), ("d", ctypes.c_int64), ("n_nodes", ctypes.c_int32),
                ("depth", ctypes.c_int32), ("flags", ctypes.c_uint32), ("kernel", ctypes.c_int32),
                ("h", ctypes.c_double), ("tol", ctypes.c_double), ("tau", ctypes.c_double),
                ("rmax", ctypes.c_int32), ("m", ctypes.c_int32), ("n_far", ctypes.c_int64),
                ("n_near", ctypes.c_int64), ("basis_len", ctypes.c_int64), ("B_len", ctypes.c_int64),
                ("D_len", ctypes.c_int64), ("skel_len", ctypes.c_int64),
                ("perm", _P), ("start", _P), ("size", _P), ("parent", _P), ("left", _P),
                ("right", _P), ("level", _P), ("rank", _P), ("basis_off", _P), ("basis", _P),
                ("far_ptr", _P), ("far_col", _P), ("far_off", _P), ("B", _P), ("near_ptr", _P),
                ("near_col", _P), ("near_off", _P), ("D", _P), ("skel_ptr", _P), ("skel", _P)]


class hm_compress_opts(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int32), ("h", ctypes.c_double), ("leaf_size", ctypes.c_int32),
                ("tol", ctypes.c_double), ("max_rank", ctypes.c_int32),
                ("admissibility", ctypes.c_int32), ("tau", ctypes.c_double),
                ("sample_rows", ctypes.c_int64), ("seed", ctypes.c_uint64),
                ("threads", ctypes.c_int32), ("partitioner", ctypes.c_int32), ("budget", ctypes.c_double)]


class hm_structure_info_t(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int64), ("d", ctypes.c_int64), ("n_nodes", ctypes.c_int32),
                ("depth", ctypes.c_int32), ("n_far", ctypes.c_int64), ("n_near", ctypes.c_int64),
                ("rows_total", ctypes.c_int64)]


class hm_batch_info_t(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("column_tile", ctypes.c_int32), ("n_tasks", ctypes.c_int32),
                ("workgroups", ctypes.c_int32), ("flops", ctypes.c_double),
                ("tuned_ms", ctypes.c_double * 5), ("workspace_bytes", ctypes.c_double)]


class hm_server_stats_t(ctypes.Structure):
    _fields_ = [("completed", ctypes.c_int64), ("failed", ctypes.c_int64), ("sweeps", ctypes.c_int64),
                ("columns", ctypes.c_int64), ("pending", ctypes.c_int64), ("inflight", ctypes.c_int32),
                ("peak_inflight", ctypes.c_int32), ("peak_bytes", ctypes.c_double)]


class hm_info_t(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int64), ("n_nodes", ctypes.c_int32), ("depth", ctypes.c_int32),
                ("max_rank", ctypes.c_int32), ("device", ctypes.c_int32), ("n_far", ctypes.c_int64),
                ("n_near", ctypes.c_int64), ("E_V", ctypes.c_int64), ("E_T", ctypes.c_int64),
                ("E_B", ctypes.c_int64), ("E_D", ctypes.c_int64), ("flops_per_col", ctypes.c_double),
                ("bytes_fp64", ctypes.c_double), ("bytes_fp32", ctypes.c_double),
                ("bytes_bf16x3", ctypes.c_double), ("n_phases", ctypes.c_int32)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libhm.so is not built ({LIB_PATH}); run paper_1812_07152_amd/build.py")
    L = ctypes.CDLL(LIB_PATH)
    st = ctypes.c_int
    L.hm_last_error.restype = ctypes.c_char_p
    L.hm_last_error.argtypes = []
    L.hm_load_compressed.restype = st
    L.hm_load_compressed.argtypes = [ctypes.c_char_p, ctypes.c_int, ctypes.c_uint, ctypes.POINTER(_P)]
    L.hm_load_compressed_mem.restype = st
    L.hm_load_compressed_mem.argtypes = [ctypes.POINTER(hm_host_repr), ctypes.c_int, ctypes.c_uint,
                                         ctypes.POINTER(_P)]
    L.hm_info.restype = st
    L.hm_info.argtypes = [_P, ctypes.POINTER(hm_info_t)]
    L.hm_free.restype = st
    L.hm_free.argtypes = [_P]
    L.hm_eval.restype = st
    L.hm_eval.argtypes = [_P, _P, ctypes.c_int64, _P, ctypes.c_int64, ctypes.c_int64, ctypes.c_int,
                          ctypes.c_int, ctypes.c_uint, _P]
    L.hm_eval_noalloc.restype = st
    L.hm_eval_noalloc.argtypes = L.hm_eval.argtypes
    L.hm_profile_read.restype = st
    L.hm_profile_read.argtypes = [_P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    L.hm_profile_reset.restype = st
    L.hm_profile_reset.argtypes = [_P]
    L.hm_check.restype = st
    L.hm_set_points.argtypes = [_P, _P, ctypes.c_int64, ctypes.c_int64, ctypes.c_int, ctypes.c_double]
    L.hm_set_points.restype = ctypes.c_int
    L.hm_check.argtypes = [_P]
    _PP = ctypes.POINTER(_P)
    _I64P = ctypes.POINTER(ctypes.c_int64)
    L.hm_batch_create.restype = st
    L.hm_batch_create.argtypes = [ctypes.c_int, _PP, _I64P, ctypes.c_int, ctypes.c_int, ctypes.c_uint,
                                  ctypes.POINTER(_P)]
    L.hm_batch_eval.restype = st
    L.hm_batch_eval.argtypes = [_P, _PP, _I64P, _PP, _I64P, _P]
    L.hm_batch_info.restype = st
    L.hm_batch_info.argtypes = [_P, ctypes.POINTER(hm_batch_info_t)]
    L.hm_batch_check.restype = st
    L.hm_batch_check.argtypes = [_P]
    L.hm_batch_free.restype = st
    L.hm_batch_free.argtypes = [_P]
    L.hm_server_create.restype = st
    L.hm_server_create.argtypes = [ctypes.c_int, ctypes.c_size_t, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                   ctypes.POINTER(_P)]
    L.hm_server_add.restype = st
    L.hm_server_add.argtypes = [_P, _P, ctypes.POINTER(ctypes.c_int)]
    L.hm_submit.restype = st
    L.hm_submit.argtypes = [_P, ctypes.c_int, _P, ctypes.c_int64, _P, ctypes.c_int64, ctypes.c_int64,
                            _P, ctypes.POINTER(ctypes.c_uint64)]
    L.hm_poll.restype = st
    L.hm_poll.argtypes = [_P, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)]
    L.hm_server_stats.restype = st
    L.hm_server_stats.argtypes = [_P, ctypes.POINTER(hm_server_stats_t)]
    L.hm_server_destroy.restype = st
    L.hm_server_destroy.argtypes = [_P]
    L.hm_eval_batched.restype = st
    L.hm_eval_batched.argtypes = [ctypes.c_int, _PP, _PP, _I64P, _PP, _I64P, _I64P, ctypes.c_int,
                                  ctypes.c_int, _P]
    L.hm_compress.restype = st
    L.hm_compress.argtypes = [_P, ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(hm_compress_opts),
                              ctypes.POINTER(_P)]
    L.hm_repr_view.restype = st
    L.hm_repr_view.argtypes = [_P, ctypes.POINTER(hm_host_repr)]
    L.hm_repr_write.restype = st
    L.hm_repr_write.argtypes = [_P, ctypes.c_char_p]
    L.hm_repr_free.restype = st
    L.hm_repr_free.argtypes = [_P]
    L.hm_inspect_p1.restype = st
    L.hm_inspect_p1.argtypes = [_P, ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(hm_compress_opts),
                                ctypes.POINTER(_P)]
    L.hm_structure_info.restype = st
    L.hm_structure_info.argtypes = [_P, ctypes.POINTER(hm_structure_info_t)]
    L.hm_structure_rows.restype = st
    L.hm_structure_rows.argtypes = [_P, ctypes.c_int32, _P, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
    L.hm_structure_free.restype = st
    L.hm_structure_free.argtypes = [_P]
    L.hm_inspect_p2_load.restype = st
    L.hm_inspect_p2_load.argtypes = [_P, ctypes.c_int, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_int32, ctypes.c_uint, ctypes.POINTER(_P)]
    L.hm_inspect_p2.restype = st
    L.hm_inspect_p2.argtypes = [_P, ctypes.c_int, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                ctypes.c_int32, ctypes.POINTER(_P)]
    return L


lib = _load()


def hm_last_error() -> str:
    return lib.hm_last_error().decode(errors="replace")


def _check(status: int) -> None:
    if status != HM_OK:
        raise HMError(status, hm_last_error())


class Matrix:
    """Owning wrapper of an hm_matrix handle."""

    def __init__(self, handle: int):
        self.handle = handle

    def __del__(self):
        # (lib is None only during interpreter shutdown; the process frees all then)
        if getattr(self, "handle", None) and lib is not None:
            lib.hm_free(self.handle)
            self.handle = None

    @property
    def _as_parameter_(self):
        return self.handle


def hm_load_compressed(path: str, device: int = 0,
                       prec_mask: int = precbit(HM_PREC_FP64)) -> Matrix:
    out = _P()
    _check(lib.hm_load_compressed(os.fsencode(path), device, prec_mask, ctypes.byref(out)))
    return Matrix(out.value)


_I64 = ("perm", "start", "size", "basis_off", "far_ptr", "far_off", "near_ptr", "near_off")
_I32 = ("parent", "left", "right", "level", "rank", "far_col", "near_col")
_F64 = ("basis", "B", "D")


def host_repr(src, skeletons: bool = True) -> tuple[hm_host_repr, list]:
    """Build an hm_host_repr view of an object carrying the representation's
    arrays as attributes (numpy).  Returns the struct and the arrays it points
    to (keep them alive until the call returns).  The skeletons (skel_ptr,
    skel) are passed when the object has them and skeletons is true."""
    keep = []
    r = hm_host_repr()

    def arr(name, dt):
        a = np.ascontiguousarray(getattr(src, name), dtype=dt)
        keep.append(a)
        return a.ctypes.data if a.size else None

    for nme in _I64:
        setattr(r, nme, arr(nme, np.int64))
    for nme in _I32:
        setattr(r, nme, arr(nme, np.int32))
    for nme in _F64:
        setattr(r, nme, arr(nme, np.float64))
    r.N = int(src.N)
    r.d = int(getattr(src, "d", 0))
    # metadata: what the representation was compressed with (checked by hm_set_points)
    params = getattr(src, "params", None) or {}
    for k in ("kernel", "h", "tol", "tau", "rmax", "m"):
        if k in params:
            setattr(r, k, params[k])
    if params.get("adm") == 1:
        r.flags = 1
    r.n_nodes = int(src.n_nodes)
    r.depth = int(np.max(src.level))
    r.n_far, r.n_near = len(src.far_col), len(src.near_col)
    r.basis_len, r.B_len, r.D_len = len(src.basis), len(src.B), len(src.D)
    if skeletons and getattr(src, "skel", None) is not None and len(src.skel) > 0:
        r.skel_ptr, r.skel = arr("skel_ptr", np.int64), arr("skel", np.int64)
        r.skel_len = len(src.skel)
    else:
        r.skel_len = 0
        r.skel_ptr = r.skel = None
    return r, keep


class Repr:
    """Host representation owned by libhm (output of hm_compress).  Its arrays
    are exposed as zero-copy numpy views, valid while the object lives."""

    def __init__(self, handle: int):
        self.handle = handle
        v = hm_host_repr()
        _check(lib.hm_repr_view(handle, ctypes.byref(v)))
        self._view = v
        for k in ("N", "d", "n_nodes", "depth", "n_far", "n_near"):
            setattr(self, k, getattr(v, k))
        n = v.n_nodes

        def arr(ptr, ctype, count):
            if count == 0 or not ptr:
                return np.zeros(0, np.ctypeslib.as_ctypes_type(ctype))
            return np.ctypeslib.as_array((np.ctypeslib.as_ctypes_type(ctype) * count).from_address(ptr))

        sizes = dict(perm=v.N, start=n, size=n, basis_off=n, far_ptr=n + 1, far_off=v.n_far,
                     near_ptr=n + 1, near_off=v.n_near, parent=n, left=n, right=n, level=n, rank=n,
                     far_col=v.n_far, near_col=v.n_near, basis=v.basis_len, B=v.B_len, D=v.D_len,
                     skel_ptr=n + 1, skel=v.skel_len)
        for k, cnt in sizes.items():
            dt = np.int64 if k in _I64 or k in ("skel_ptr", "skel") else np.int32 if k in _I32 else np.float64
            setattr(self, k, arr(getattr(v, k), dt, cnt))

    def __del__(self):
        # (lib is None only during interpreter shutdown; the process frees all then)
        if getattr(self, "handle", None) and lib is not None:
            lib.hm_repr_free(self.handle)
            self.handle = None

    def write(self, path: str) -> None:
        _check(lib.hm_repr_write(self.handle, os.fsencode(path)))


def hm_compress(X: np.ndarray, *, kernel: int, h: float, leaf_size: int, tol: float, max_rank: int,
                admissibility: int, tau: float, sample_rows: int = 4096, seed: int = 7,
                threads: int = 0, partitioner: int = 0, budget: float = 0.0) -> Repr:
    X = np.ascontiguousarray(X, dtype=np.float64)
    o = hm_compress_opts(kernel, h, leaf_size, tol, max_rank, admissibility, tau, sample_rows, seed,
                         threads, partitioner, budget)
    out = _P()
    _check(lib.hm_compress(X.ctypes.data, X.shape[0], X.shape[1], ctypes.byref(o), ctypes.byref(out)))
    return Repr(out.value)


class Structure:
    """inspector-p1 output owned by libhm: tree, interaction lists and row
    samples of a point set, reused by every inspector-p2 run."""

    def __init__(self, handle: int):
        self.handle = handle
        info = hm_structure_info_t()
        _check(lib.hm_structure_info(handle, ctypes.byref(info)))
        for k, _ in hm_structure_info_t._fields_:
            setattr(self, k, getattr(info, k))

    def rows(self, node: int) -> np.ndarray:
        """Row sample of a node: original point indices in tree order."""
        cnt = ctypes.c_int64()
        _check(lib.hm_structure_rows(self.handle, int(node), None, 0, ctypes.byref(cnt)))
        out = np.zeros(max(cnt.value, 1), np.int64)
        _check(lib.hm_structure_rows(self.handle, int(node), out.ctypes.data, len(out), ctypes.byref(cnt)))
        return out[:cnt.value]

    def __del__(self):
        if getattr(self, "handle", None) and lib is not None:
            lib.hm_structure_free(self.handle)
            self.handle = None


def hm_inspect_p1(X: np.ndarray, *, leaf_size: int, admissibility: int, tau: float, sample_rows: int = 4096,
                  seed: int = 7, threads: int = 0, partitioner: int = 0, budget: float = 0.0) -> Structure:
    """inspector-p1 (host): tree, far/near lists and row samples."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    o = hm_compress_opts(0, 1.0, leaf_size, 0.0, 1, admissibility, tau, sample_rows, seed, threads,
                         partitioner, budget)
    out = _P()
    _check(lib.hm_inspect_p1(X.ctypes.data, X.shape[0], X.shape[1], ctypes.byref(o), ctypes.byref(out)))
    return Structure(out.value)


def hm_inspect_p2(s: Structure, device: int = 0, *, kernel: int, h: float, tol: float, max_rank: int) -> Repr:
    """inspector-p2 on the GPU: IDs of every node and the blocks, for one
    kernel function and accuracy, on a kept inspector-p1 structure."""
    out = _P()
    _check(lib.hm_inspect_p2(s.handle, int(device), int(kernel), float(h), float(tol), int(max_rank),
                             ctypes.byref(out)))
    return Repr(out.value)


def hm_inspect_p2_load(s: Structure, device: int = 0, *, kernel: int, h: float, tol: float, max_rank: int,
                       prec_mask: int = precbit(HM_PREC_FP64)) -> "Matrix":
    """inspector-p2 on the GPU straight into a device matrix (blocks generated
    in the device store)."""
    out = _P()
    _check(lib.hm_inspect_p2_load(s.handle, int(device), int(kernel), float(h), float(tol), int(max_rank),
                                  int(prec_mask), ctypes.byref(out)))
    return Matrix(out.value)


def hm_repr_write(r: Repr, path: str) -> None:
    r.write(path)


def hm_repr_free(r: Repr) -> None:
    if r.handle:
        _check(lib.hm_repr_free(r.handle))
        r.handle = None


def hm_load_compressed_mem(src, device: int = 0, prec_mask: int = precbit(HM_PREC_FP64),
                           skeletons: bool = True) -> Matrix:
    """Load a representation (an hm_compress result, or an object with its
    arrays); skeletons=False leaves an object's skeletons out of the view."""
    if isinstance(src, Repr):
        out = _P()
        _check(lib.hm_load_compressed_mem(ctypes.byref(src._view), device, prec_mask, ctypes.byref(out)))
        return Matrix(out.value)
    r, keep = host_repr(src, skeletons)
    out = _P()
    _check(lib.hm_load_compressed_mem(ctypes.byref(r), device, prec_mask, ctypes.byref(out)))
    del keep
    return Matrix(out.value)


def hm_info(h: Matrix) -> dict:
    info = hm_info_t()
    _check(lib.hm_info(h, ctypes.byref(info)))
    return {name: getattr(info, name) for name, _ in hm_info_t._fields_}


def hm_free(h: Matrix) -> None:
    if h.handle:
        _check(lib.hm_free(h.handle))
        h.handle = None


def _stream_ptr(stream) -> int | None:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


def _eval_args(name: str, h: Matrix, W, Y, Q, prec, flags, stream):
    """Argument checks and marshalling shared by hm_eval and hm_eval_noalloc."""
    import torch
    if not (W.is_cuda and Y.is_cuda):
        raise ValueError(f"{name}: W and Y must be device tensors")
    if W.dtype != Y.dtype or W.dtype not in (torch.float64, torch.float32):
        raise ValueError(f"{name}: W and Y must both be float64 or both float32")
    if W.dim() != 2 or Y.dim() != 2 or W.stride(1) != 1 or Y.stride(1) != 1:
        raise ValueError(f"{name}: W and Y must be 2-D with unit column stride")
    info = hm_info(h)
    if W.shape[0] < info["N"] or Y.shape[0] < info["N"]:
        raise ValueError(f"{name}: W and Y need N={info['N']} rows")
    if W.device.index != info["device"] or Y.device.index != info["device"]:
        raise ValueError(f"{name}: tensors are not on the matrix's device")
    dtype = HM_F64 if W.dtype == torch.float64 else HM_F32
    if prec is None:
        prec = HM_PREC_FP64 if dtype == HM_F64 else HM_PREC_FP32
    if Q is None:
        Q = W.shape[1]
    if Q == 0:
        return None
    if W.shape[1] < Q or Y.shape[1] < Q:
        raise ValueError(f"{name}: tensors narrower than Q")
    return (h, W.data_ptr(), W.stride(0), Y.data_ptr(), Y.stride(0), Q, dtype, prec, flags, _stream_ptr(stream))


def hm_eval(h: Matrix, W, Y, Q: int | None = None, prec: int | None = None, flags: int = 0,
            stream=None) -> None:
    """Y = K~ W on the device.  W and Y are CUDA (HIP) tensors, row-major with
    unit column stride, N x Q (leading dimensions from their row strides)."""
    args = _eval_args("hm_eval", h, W, Y, Q, prec, flags, stream)
    if args is not None:
        _check(lib.hm_eval(*args))


def hm_eval_noalloc(h: Matrix, W, Y, Q: int | None = None, prec: int | None = None, flags: int = 0,
                    stream=None) -> None:
    """hm_eval with its per-call device memory in the library's fixed device
    array (HM_NOALLOC_SCRATCH_BYTES): allocates nothing.  The evaluation's
    task graph must exist already (an hm_eval of the same width class, dtype
    and precision builds it)."""
    args = _eval_args("hm_eval_noalloc", h, W, Y, Q, prec, flags, stream)
    if args is not None:
        _check(lib.hm_eval_noalloc(*args))


def hm_set_points(h: Matrix, X: np.ndarray, kernel: int, h_param: float) -> None:
    """Points (N x d, FP64, original order) and kernel (0 Gaussian, 1
    Laplace-type) for evaluations with HM_NEAR_FROM_POINTS or
    HM_FAR_FROM_POINTS, which compute the near or far blocks from the points
    instead of reading them."""
    X = np.ascontiguousarray(X, dtype=np.float64)
    if X.ndim != 2 or X.shape[0] != hm_info(h)["N"]:
        raise ValueError("hm_set_points: X must be N x d")
    _check(lib.hm_set_points(h, X.ctypes.data, X.shape[1], X.shape[1], int(kernel), float(h_param)))


def hm_check(h: Matrix) -> None:
    """Synchronize and raise if a persistent launch's bounded wait expired."""
    _check(lib.hm_check(h))


class Batch:
    """Owning wrapper of an hm_batch handle (keeps its matrices alive)."""

    def __init__(self, handle: int, mats, Q):
        self.handle, self.mats, self.Q = handle, list(mats), list(Q)

    def __del__(self):
        # (lib is None only during interpreter shutdown; the process frees all then)
        if getattr(self, "handle", None) and lib is not None:
            lib.hm_batch_free(self.handle)
            self.handle = None


def _ptrs(xs):
    return (_P * len(xs))(*xs)


def _i64s(xs):
    return (ctypes.c_int64 * len(xs))(*[int(x) for x in xs])


def hm_batch_create(mats, Q, dtype: int = HM_F64, prec: int | None = None, flags: int = 0) -> Batch:
    if prec is None:
        prec = HM_PREC_FP64 if dtype == HM_F64 else HM_PREC_FP32
    out = _P()
    _check(lib.hm_batch_create(len(mats), _ptrs([m.handle for m in mats]), _i64s(Q), dtype, prec, flags,
                               ctypes.byref(out)))
    return Batch(out.value, mats, Q)


def _check_tensors(mats, Ws, Ys, Qs):
    import torch
    if not (len(mats) == len(Ws) == len(Ys) == len(Qs)):
        raise ValueError("one W, Y and Q per matrix")
    for m, W, Y, q in zip(mats, Ws, Ys, Qs):
        info = hm_info(m)
        if not (W.is_cuda and Y.is_cuda) or W.dtype != Y.dtype or W.dtype not in (torch.float64, torch.float32):
            raise ValueError("W and Y must be device tensors of one float dtype")
        if W.dim() != 2 or Y.dim() != 2 or W.stride(1) != 1 or Y.stride(1) != 1:
            raise ValueError("W and Y must be 2-D with unit column stride")
        if W.shape[0] < info["N"] or Y.shape[0] < info["N"] or W.shape[1] < q or Y.shape[1] < q:
            raise ValueError("W and Y too small for the matrix and width")


def hm_batch_eval(b: Batch, Ws, Ys, stream=None) -> None:
    _check_tensors(b.mats, Ws, Ys, b.Q)
    _check(lib.hm_batch_eval(b.handle, _ptrs([w.data_ptr() for w in Ws]), _i64s([w.stride(0) for w in Ws]),
                             _ptrs([y.data_ptr() for y in Ys]), _i64s([y.stride(0) for y in Ys]),
                             _stream_ptr(stream)))


def hm_batch_info(b: Batch) -> dict:
    info = hm_batch_info_t()
    _check(lib.hm_batch_info(b.handle, ctypes.byref(info)))
    d = {name: getattr(info, name) for name, _ in hm_batch_info_t._fields_}
    d["tuned_ms"] = dict(zip((16, 32, 64, 128, 256), list(info.tuned_ms)))
    return d


def hm_batch_check(b: Batch) -> None:
    _check(lib.hm_batch_check(b.handle))


def hm_batch_free(b: Batch) -> None:
    if b.handle:
        _check(lib.hm_batch_free(b.handle))
        b.handle = None


def hm_eval_batched(mats, Ws, Ys, Q=None, prec: int | None = None, stream=None) -> None:
    import torch
    Q = [w.shape[1] for w in Ws] if Q is None else list(Q)
    _check_tensors(mats, Ws, Ys, Q)
    dtype = HM_F64 if Ws[0].dtype == torch.float64 else HM_F32
    if prec is None:
        prec = HM_PREC_FP64 if dtype == HM_F64 else HM_PREC_FP32
    _check(lib.hm_eval_batched(len(mats), _ptrs([m.handle for m in mats]), _ptrs([w.data_ptr() for w in Ws]),
                               _i64s([w.stride(0) for w in Ws]), _ptrs([y.data_ptr() for y in Ys]),
                               _i64s([y.stride(0) for y in Ys]), _i64s(Q), dtype, prec, _stream_ptr(stream)))


class Server:
    """Owning wrapper of an hm_server (keeps resident matrices alive)."""

    def __init__(self, handle: int, dtype: int):
        self.handle, self.dtype, self.mats = handle, dtype, []

    def __del__(self):
        # (lib is None only during interpreter shutdown; the process frees all then)
        if getattr(self, "handle", None) and lib is not None:
            lib.hm_server_destroy(self.handle)
            self.handle = None


def hm_server_create(device: int = 0, hbm_budget: int = 8 << 30, max_slots: int = 4,
                     dtype: int = HM_F32, prec: int | None = None) -> Server:
    if prec is None:
        prec = HM_PREC_FP64 if dtype == HM_F64 else HM_PREC_FP32
    out = _P()
    _check(lib.hm_server_create(device, hbm_budget, max_slots, dtype, prec, ctypes.byref(out)))
    return Server(out.value, dtype)


def hm_server_add(s: Server, h: Matrix) -> int:
    mid = ctypes.c_int()
    _check(lib.hm_server_add(s.handle, h.handle, ctypes.byref(mid)))
    s.mats.append(h)
    return mid.value


def hm_submit(s: Server, mat_id: int, W, Y, Q: int | None = None, stream=None) -> int:
    """Queue Y = K~ W (device tensors; keep them alive until hm_poll says done).
    The request runs after the work enqueued on `stream` (default: torch's
    current stream) before the call, e.g. the kernels that wrote W."""
    import torch
    want = torch.float64 if s.dtype == HM_F64 else torch.float32
    if not (W.is_cuda and Y.is_cuda) or W.dtype != want or Y.dtype != want:
        raise ValueError("hm_submit: W and Y must be device tensors of the server's dtype")
    if W.dim() != 2 or Y.dim() != 2 or W.stride(1) != 1 or Y.stride(1) != 1:
        raise ValueError("hm_submit: W and Y must be 2-D with unit column stride")
    Q = W.shape[1] if Q is None else Q
    if 0 <= mat_id < len(s.mats):  # unknown ids are rejected by the library itself
        N = hm_info(s.mats[mat_id])["N"]
        if W.shape[0] < N or Y.shape[0] < N or W.shape[1] < Q or Y.shape[1] < Q:
            raise ValueError("hm_submit: tensors too small")
    t = ctypes.c_uint64()
    _check(lib.hm_submit(s.handle, mat_id, W.data_ptr(), W.stride(0), Y.data_ptr(), Y.stride(0), Q,
                         _stream_ptr(stream), ctypes.byref(t)))
    return t.value


def hm_poll(s: Server, ticket: int):
    """(done, latency_us): latency is None while pending."""
    done = ctypes.c_int()
    lat = ctypes.c_double()
    _check(lib.hm_poll(s.handle, ticket, ctypes.byref(done), ctypes.byref(lat)))
    return bool(done.value), (lat.value if done.value else None)


def hm_server_stats(s: Server) -> dict:
    st = hm_server_stats_t()
    _check(lib.hm_server_stats(s.handle, ctypes.byref(st)))
    return {name: getattr(st, name) for name, _ in hm_server_stats_t._fields_}


def hm_server_destroy(s: Server) -> None:
    if s.handle:
        _check(lib.hm_server_destroy(s.handle))
        s.handle = None


def hm_profile_read(h: Matrix):
    ms = (ctypes.c_double * 5)()
    n = (ctypes.c_int64 * 5)()
    _check(lib.hm_profile_read(h, ms, n))
    return list(ms), list(n)


def hm_profile_reset(h: Matrix) -> None:
    _check(lib.hm_profile_reset(h))
