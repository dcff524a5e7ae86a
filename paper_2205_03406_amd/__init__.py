"""Thin Python binding of libhm (include/hm.h): argument marshalling only.

Every step of colored peeling runs in the native library; this module only
converts arguments.  Device buffers are torch CUDA (HIP) tensors holding
column-major N x ncols blocks: a tensor of shape (N, ncols) with strides
(1, ld), e.g. ``torch.empty(ncols, N, device="cuda").t()``.  Streams default
to torch's current stream.

Importing this module loads ``libhm.so`` from the package directory and
raises if it is missing: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libhm.so")

HM_OK = 0
HM_E_ARG, HM_E_NOMEM, HM_E_DEVICE, HM_E_CALLBACK = -1, -2, -3, -4
HM_E_NUMERIC, HM_E_STATE, HM_E_SATURATED = -5, -6, -7
HM_TREE_GEOMETRIC, HM_TREE_INDEX_BINARY = 0, 1
HM_ADM_STRONG, HM_ADM_WEAK = 0, 1
HM_F64, HM_F32 = 0, 1
HM_PREC_F64, HM_PREC_MIXED = 0, 1
HM_FORMAT_H1, HM_FORMAT_UNIFORM_H1, HM_FORMAT_H2 = 0, 1, 2


def _format(uniform, h2):
    if uniform and h2:
        raise ValueError("choose one of uniform and h2")
    return HM_FORMAT_H2 if h2 else (HM_FORMAT_UNIFORM_H1 if uniform else HM_FORMAT_H1)
HM_KERNEL_LOG, HM_KERNEL_INV_R = 0, 1
HM_ORDER_ORIGINAL, HM_ORDER_TREE = 0, 1
HM_LIST_NEIGHBOR, HM_LIST_INTERACTION = 0, 1

EXPORTED = [
    "hm_last_error", "hm_build_tree", "hm_tree_free", "hm_tree_info", "hm_tree_perm",
    "hm_tree_level", "hm_tree_list", "hm_incompat_graph", "hm_color", "hm_tree_color",
    "hm_tree_set_colors", "hm_tree_colors", "hm_kernel_blackbox", "hm_kernel_apply",
    "hm_dense_blackbox", "hm_dense_blackbox_free", "hm_compress", "hm_hmatrix_free",
    "hm_matvec", "hm_test_matrix", "hm_philox4x32_10", "hm_hmatrix_stats",
    "hm_hmatrix_export_level", "hm_hmatrix_export_near", "hm_build_forest",
    "hm_tree_instances", "hm_autotune_table", "hm_server_create", "hm_server_free",
    "hm_server_submit_compress", "hm_server_submit_matvec", "hm_server_poll", "hm_server_hmatrix",
    "hm_server_release", "hm_server_info", "hm_compress_plan", "hm_plan_execute",
    "hm_plan_hmatrix", "hm_plan_free", "hm_uniform_graph", "hm_matvec_op",
    "hm_hmatrix_blackbox", "hm_product_blackbox", "hm_blackbox_free", "hm_mfma_rate",
    "hm_matvec_static", "hm_compress_footprint", "hm_matvec_footprint",
]


class HMError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("hm error %d: %s" % (code, msg))
        self.code = code


APPLY_FN = C.CFUNCTYPE(C.c_int, C.c_void_p, C.c_int, C.c_int64, C.c_int64, C.c_int,
                       C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_void_p)


class BlackBox(C.Structure):
    _fields_ = [("apply", APPLY_FN), ("ctx", C.c_void_p), ("order", C.c_int32),
                ("symmetric", C.c_int32), ("dtypes", C.c_int32)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class Allocator(C.Structure):
    """hm_allocator: the caller's device allocator."""
    _fields_ = [("ctx", C.c_void_p), ("alloc", ALLOC_FN), ("free", FREE_FN)]


class TorchAllocator:
    """An hm_allocator over PyTorch's caching allocator
    (torch.cuda.caching_allocator_alloc / caching_allocator_delete), so that
    the library's device blocks belong to torch (they show in
    torch.cuda.memory_allocated()).  `allocs`, `frees` and `live` (pointer ->
    bytes) count the blocks taken and returned; `peak_bytes` is the most
    bytes live at once since the last reset_peak().  The object must outlive
    every H-matrix, plan, tree and server that uses it."""

    def __init__(self):
        import threading
        import torch
        self.allocs = 0
        self.frees = 0
        self.live = {}
        self._bytes = 0
        self.peak_bytes = 0
        self._lock = threading.Lock()

        def _alloc(ctx, nbytes, stream):
            try:
                p = torch.cuda.caching_allocator_alloc(int(nbytes), stream=int(stream or 0))
            except Exception:
                return None
            with self._lock:
                self.allocs += 1
                self.live[p] = int(nbytes)
                self._bytes += int(nbytes)
                self.peak_bytes = max(self.peak_bytes, self._bytes)
            return p

        def _free(ctx, p, stream):
            with self._lock:
                self.frees += 1
                self._bytes -= self.live.pop(p, 0)
            try:
                torch.cuda.caching_allocator_delete(p)
            except Exception:
                pass  # interpreter shutdown: the process is ending

        self._fa = ALLOC_FN(_alloc)
        self._ff = FREE_FN(_free)
        self.struct = Allocator(None, self._fa, self._ff)

    def live_bytes(self):
        with self._lock:
            return self._bytes

    def reset_peak(self):
        """Restart peak_bytes from the bytes live now."""
        with self._lock:
            self.peak_bytes = self._bytes


_TORCH_ALLOC = None


def torch_allocator():
    """The process-wide TorchAllocator (made on first use)."""
    global _TORCH_ALLOC
    if _TORCH_ALLOC is None:
        _TORCH_ALLOC = TorchAllocator()
    return _TORCH_ALLOC


def _allocator(a):
    """allocator argument -> (TorchAllocator or None, pointer for the opts)."""
    if a is None:
        return None, None
    if isinstance(a, str):
        if a != "torch":
            raise ValueError("allocator must be None, 'torch' or a TorchAllocator")
        a = torch_allocator()
    return a, C.pointer(a.struct)


class Opts(C.Structure):
    _fields_ = [("rank", C.c_int32), ("tol", C.c_double), ("oversample", C.c_int32),
                ("r", C.c_int32), ("prec", C.c_int32), ("flags", C.c_int32),
                ("seed", C.c_uint64), ("max_retries", C.c_int32), ("format", C.c_int32),
                ("allocator", C.POINTER(Allocator))]


class Stats(C.Structure):
    _fields_ = [("nlevels", C.c_int32), ("r", C.c_int32), ("n", C.c_int64),
                ("cols_A", C.c_int64), ("cols_At", C.c_int64), ("colors", C.c_int32 * 32),
                ("leaf_colors", C.c_int32), ("leaf_width", C.c_int32), ("max_rank", C.c_int32),
                ("npairs", C.c_int64), ("nnear", C.c_int64), ("saturated", C.c_int64),
                ("nfloats", C.c_int64), ("retries", C.c_int32), ("format", C.c_int32),
                ("ucolors", C.c_int32 * 32),
                ("flops_blackbox", C.c_double),
                ("flops_peel", C.c_double), ("flops_qr", C.c_double),
                ("flops_solve", C.c_double), ("ms_total", C.c_double),
                ("ms_blackbox", C.c_double), ("ms_peel", C.c_double), ("ms_qr", C.c_double),
                ("ms_solve", C.c_double), ("ms_other", C.c_double),
                ("device_bytes", C.c_int64), ("bytes_peel", C.c_double)]

    def as_dict(self):
        d = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            d[name] = list(v) if name in ("colors", "ucolors") else v
        return d


class ServerOpts(C.Structure):
    _fields_ = [("hbm_budget", C.c_int64), ("nslots", C.c_int32),
                ("compress_slots", C.c_int32), ("allocator", C.POINTER(Allocator))]


class Completion(C.Structure):
    _fields_ = [("id", C.c_int64), ("kind", C.c_int32), ("status", C.c_int32),
                ("hmatrix", C.c_int64), ("t_submit", C.c_double), ("t_admit", C.c_double),
                ("t_start", C.c_double), ("t_end", C.c_double), ("bytes", C.c_int64),
                ("device_ms", C.c_double), ("enqueue_ms", C.c_double)]


def _load():
    # One HIP runtime per process: torch ships its own libamdhip64 (needed
    # by file name), libhm needs it by soname.  Loaded first, libhm would
    # pull in /opt/rocm's runtime and torch a second one, each with its own
    # HSA runtime on the same device; with torch loaded first the loader
    # reuses torch's runtime for libhm.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(_SO):
        raise ImportError("libhm.so is not built (run __graft_entry__.build() or "
                          "python -m paper_2205_03406_amd.build)")
    lib = C.CDLL(_SO)
    P, I, I64, D = C.c_void_p, C.c_int, C.c_int64, C.c_double
    pp = C.POINTER(C.c_void_p)
    lib.hm_last_error.restype = C.c_char_p
    lib.hm_autotune_table.restype = C.c_char_p
    lib.hm_autotune_table.argtypes = []
    sigs = {
        "hm_build_tree": [P, I64, I, I, I, I, pp],
        "hm_build_forest": [P, P, C.c_int32, I, I, I, I, pp],
        "hm_tree_instances": [P, P, P],
        "hm_tree_free": [P],
        "hm_tree_info": [P, P, P, P],
        "hm_tree_perm": [P, P],
        "hm_tree_level": [P, I, P, P, P, P, P],
        "hm_tree_list": [P, I, I, P, P, P],
        "hm_incompat_graph": [P, I, P, P, pp, pp, pp, P, pp, pp, pp],
        "hm_color": [I64, P, P, P, P],
        "hm_tree_color": [P],
        "hm_tree_set_colors": [P, I, P],
        "hm_tree_colors": [P, I, P, pp],
        "hm_kernel_blackbox": [P, I, C.POINTER(BlackBox)],
        "hm_kernel_apply": [P, I, I64, I, P, I64, P, I64, I, P],
        "hm_dense_blackbox": [P, I64, I64, I, C.POINTER(BlackBox)],
        "hm_dense_blackbox_free": [C.POINTER(BlackBox)],
        "hm_compress": [P, C.POINTER(BlackBox), C.POINTER(Opts), P, pp],
        "hm_compress_footprint": [P, C.POINTER(Opts), P],
        "hm_matvec_footprint": [P, I64, I, P],
        "hm_hmatrix_free": [P],
        "hm_matvec": [P, I64, I, P, I64, P, I64, I, P],
        "hm_matvec_op": [P, I, I64, I, P, I64, P, I64, I, P],
        "hm_matvec_static": [P, I, I64, I, P, I64, P, I64, I, P],
        "hm_hmatrix_blackbox": [P, I, C.POINTER(BlackBox)],
        "hm_product_blackbox": [C.POINTER(BlackBox), C.POINTER(BlackBox), C.POINTER(BlackBox)],
        "hm_blackbox_free": [C.POINTER(BlackBox)],
        "hm_test_matrix": [P, I, I, C.c_int32, C.c_uint64, I, P, I64, P],
        "hm_philox4x32_10": [P, I64, C.c_uint32, C.c_uint32, P, P],
        "hm_hmatrix_stats": [P, C.POINTER(Stats)],
        "hm_hmatrix_export_level": [P, I, P, P, P, P, P, P, P, P, P, P, P],
        "hm_hmatrix_export_near": [P, P, P, P, P, P],
        "hm_uniform_graph": [P, I, P, P, pp, pp, pp, P, pp],
        "hm_compress_plan": [P, C.POINTER(BlackBox), C.POINTER(Opts), P, pp],
        "hm_plan_execute": [P, P],
        "hm_plan_hmatrix": [P, pp, P],
        "hm_plan_free": [P],
        "hm_server_create": [C.POINTER(ServerOpts), pp],
        "hm_server_free": [P],
        "hm_server_submit_compress": [P, P, I64, I, I, I, I, I, C.POINTER(Opts), P],
        "hm_server_submit_matvec": [P, I64, I64, I, P, P, P],
        "hm_server_poll": [P, C.c_int32, C.c_int32, P, P],
        "hm_server_hmatrix": [P, I64, pp],
        "hm_server_release": [P, I64],
        "hm_server_info": [P, P, P, P, P, P, P],
    }
    for name, args in sigs.items():
        f = getattr(lib, name)
        f.argtypes = args
        if name in ("hm_tree_free", "hm_hmatrix_free", "hm_dense_blackbox_free", "hm_server_free",
                    "hm_plan_free", "hm_blackbox_free"):
            f.restype = None
        else:
            f.restype = C.c_int
    return lib


_lib = _load()


def lib():
    return _lib


def _check(rc):
    if rc != HM_OK:
        raise HMError(rc, _lib.hm_last_error().decode())


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def _colmajor(t, name):
    """(pointer, ld, ncols, dtype code) of an (N, ncols) column-major tensor."""
    import torch
    if t.dim() == 1:
        return C.c_void_p(t.data_ptr()), t.shape[0], 1, _dtype(t)
    if t.stride(0) != 1 and t.shape[1] > 1:
        raise ValueError("%s must be column-major: shape (N, ncols), stride (1, ld)" % name)
    ld = t.stride(1) if t.shape[1] > 1 else t.shape[0]
    return C.c_void_p(t.data_ptr()), ld, t.shape[1], _dtype(t)


def _dtype(t):
    import torch
    if t.dtype == torch.float64:
        return HM_F64
    if t.dtype == torch.float32:
        return HM_F32
    raise TypeError("dtype must be float64 or float32")


def colmajor(n, ncols, dtype=None, device="cuda", fill=None):
    """An (n, ncols) column-major device tensor (ld = n)."""
    import torch
    dtype = dtype or torch.float64
    t = torch.empty(ncols, n, dtype=dtype, device=device).t()
    if fill is not None:
        t.fill_(fill)
    return t


class Graph:
    def __init__(self, nv, xadj, adj, vbox, pa, pb, pv, color=None, ncolors=0):
        self.nv, self.xadj, self.adj, self.vbox = nv, xadj, adj, vbox
        self.pair_a, self.pair_b, self.pair_v = pa, pb, pv
        self.color, self.ncolors = color, ncolors

    @property
    def nedges(self):
        return int(self.xadj[-1]) // 2


class Tree:
    """hm_build_tree handle (box tree, lists, constraint graphs)."""

    def __init__(self, points, leaf, kind="geometric", adm="strong"):
        """points: one (n, dim) array, or a list of them for a forest
        (hm_build_forest: independent instances compressed together)."""
        kd = HM_TREE_INDEX_BINARY if kind == "index_binary" else HM_TREE_GEOMETRIC
        ad = HM_ADM_WEAK if adm == "weak" else HM_ADM_STRONG
        h = C.c_void_p()
        if isinstance(points, (list, tuple)):
            parts = [np.asarray(p, np.float64) for p in points]
            parts = [p.reshape(-1, 1) if p.ndim == 1 else p for p in parts]
            pts = np.ascontiguousarray(np.concatenate(parts, axis=0))
            counts = np.array([p.shape[0] for p in parts], np.int64)
            n, dim = pts.shape
            _check(_lib.hm_build_forest(_ptr(pts), _ptr(counts), len(parts), dim, leaf, kd, ad,
                                        C.byref(h)))
        else:
            pts = np.ascontiguousarray(points, np.float64)
            if pts.ndim == 1:
                pts = pts.reshape(-1, 1)
            n, dim = pts.shape
            _check(_lib.hm_build_tree(_ptr(pts), n, dim, leaf, kd, ad, C.byref(h)))
        self.h = h
        self.n, self.dim, self.leaf = n, dim, leaf
        nl = C.c_int32()
        _check(_lib.hm_tree_info(h, C.byref(nl), None, None))
        self.nlev = nl.value
        self.L = self.nlev - 1
        self._bbs = []
        self._allocs = []  # allocators whose blocks the tree's device copy may hold

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.hm_tree_free(self.h)
            self.h = None

    def instances(self):
        """Row offsets of the instances (ninst + 1 entries)."""
        ni = C.c_int32()
        _check(_lib.hm_tree_instances(self.h, C.byref(ni), None))
        off = np.zeros(ni.value + 1, np.int64)
        _check(_lib.hm_tree_instances(self.h, C.byref(ni), _ptr(off)))
        return off

    def perm(self):
        out = np.zeros(self.n, np.int64)
        _check(_lib.hm_tree_perm(self.h, _ptr(out)))
        return out

    def level(self, l):
        nb = C.c_int32()
        _check(_lib.hm_tree_level(self.h, l, C.byref(nb), None, None, None, None))
        nb = nb.value
        start = np.zeros(nb + 1, np.int64)
        parent = np.zeros(nb, np.int32)
        os_ = max(3, self.dim)
        org = np.zeros(os_ * nb, np.int64)
        blev = np.zeros(nb, np.int32)
        _check(_lib.hm_tree_level(self.h, l, None, _ptr(start), _ptr(parent), _ptr(org), _ptr(blev)))
        return start, parent, org.reshape(nb, os_), blev

    def list(self, l, which):
        nnz = C.c_int64()
        _check(_lib.hm_tree_list(self.h, l, which, C.byref(nnz), None, None))
        nb = len(self.level(l)[1])
        ptr = np.zeros(nb + 1, np.int32)
        idx = np.zeros(max(nnz.value, 1), np.int32)
        _check(_lib.hm_tree_list(self.h, l, which, None, _ptr(ptr), _ptr(idx)))
        return ptr, idx[:nnz.value]

    def graph(self, level):
        """level = -1: leaf graph."""
        nv, nadj, npairs = C.c_int64(), C.c_int64(), C.c_int64()
        xadj, adj, vbox, pa, pb, pv = (C.c_void_p() for _ in range(6))
        _check(_lib.hm_incompat_graph(self.h, level, C.byref(nv), C.byref(nadj), C.byref(xadj),
                                      C.byref(adj), C.byref(vbox), C.byref(npairs), C.byref(pa),
                                      C.byref(pb), C.byref(pv)))

        def arr(p, n, t):
            if n == 0 or not p.value:
                return np.zeros(0, t)
            return np.ctypeslib.as_array(C.cast(p, C.POINTER(np.ctypeslib.as_ctypes_type(t))),
                                         shape=(n,)).copy()
        g = Graph(nv.value, arr(xadj, nv.value + 1, np.int64), arr(adj, nadj.value, np.int32),
                  arr(vbox, nv.value, np.int32), arr(pa, npairs.value, np.int32),
                  arr(pb, npairs.value, np.int32), arr(pv, npairs.value, np.int32))
        if nv.value == 0:
            g.xadj = np.zeros(1, np.int64)
        nc, col = C.c_int32(), C.c_void_p()
        if _lib.hm_tree_colors(self.h, level, C.byref(nc), C.byref(col)) == HM_OK:
            g.ncolors = nc.value
            g.color = arr(col, nv.value, np.int32)
        return g

    def color(self):
        _check(_lib.hm_tree_color(self.h))
        return self

    def uniform_graph(self, level):
        """Stage-1 graph of uniform H^1 compression at `level` (hm_uniform_graph):
        (vbox, xadj, adj, color, ncolors)."""
        nv, nadj, nc = C.c_int64(), C.c_int64(), C.c_int32()
        xadj, adj, vbox, col = (C.c_void_p() for _ in range(4))
        _check(_lib.hm_uniform_graph(self.h, level, C.byref(nv), C.byref(nadj), C.byref(xadj),
                                     C.byref(adj), C.byref(vbox), C.byref(nc), C.byref(col)))

        def arr(p, n, t):
            if n == 0 or not p.value:
                return np.zeros(0, t)
            return np.ctypeslib.as_array(C.cast(p, C.POINTER(np.ctypeslib.as_ctypes_type(t))),
                                         shape=(n,)).copy()
        x = arr(xadj, nv.value + 1, np.int64) if nv.value else np.zeros(1, np.int64)
        return (arr(vbox, nv.value, np.int32), x, arr(adj, nadj.value, np.int32),
                arr(col, nv.value, np.int32), nc.value)

    def set_colors(self, level, colors):
        c = np.ascontiguousarray(colors, np.int32)
        _check(_lib.hm_tree_set_colors(self.h, level, _ptr(c)))

    def kernel_blackbox(self, kernel="log"):
        bb = BlackBox()
        _check(_lib.hm_kernel_blackbox(self.h, HM_KERNEL_INV_R if kernel == "inv_r" else HM_KERNEL_LOG,
                                       C.byref(bb)))
        self._bbs.append(bb)
        return bb

    def kernel_apply(self, kernel, X, Y, order=HM_ORDER_TREE, stream=None):
        px, ldx, nc, dt = _colmajor(X, "X")
        py, ldy, nc2, dt2 = _colmajor(Y, "Y")
        if nc != nc2 or dt != dt2:
            raise ValueError("X and Y shapes/dtypes differ")
        _check(_lib.hm_kernel_apply(self.h, HM_KERNEL_INV_R if kernel == "inv_r" else HM_KERNEL_LOG,
                                    nc, dt, px, ldx, py, ldy, order, _stream(stream)))

    def test_matrix(self, level, pas, r, seed, out, stream=None):
        po, ld, nc, dt = _colmajor(out, "out")
        _check(_lib.hm_test_matrix(self.h, level, pas, r, seed, dt, po, ld, _stream(stream)))


class Plan:
    """hm_compress_plan: a compression captured into a HIP graph and replayed
    by execute(); hmatrix() borrows the latest result."""

    def __init__(self, tree, bb, rank=0, tol=0.0, r=0, p=10, prec=HM_PREC_F64, seed=0,
                 stream=None, uniform=False, h2=False, allocator="torch"):
        al, ap = _allocator(allocator)
        o = Opts(rank=rank, tol=tol, oversample=p, r=r, prec=prec, flags=0, seed=seed,
                 max_retries=0, format=_format(uniform, h2), allocator=ap)
        h = C.c_void_p()
        _check(_lib.hm_compress_plan(tree.h, C.byref(bb), C.byref(o), _stream(stream),
                                     C.byref(h)))
        self.h = h
        self.tree = tree
        self._bb = bb
        self._alloc = al
        tree._allocs.append(al)

    def execute(self, stream=None):
        _check(_lib.hm_plan_execute(self.h, _stream(stream)))

    def hmatrix(self):
        hh = C.c_void_p()
        _check(_lib.hm_plan_hmatrix(self.h, C.byref(hh), None))
        return _Borrowed(hh, self.tree)

    @property
    def graph_nodes(self):
        k = C.c_int64()
        _check(_lib.hm_plan_hmatrix(self.h, None, C.byref(k)))
        return k.value

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.hm_plan_free(self.h)
            self.h = None


def autotune_table():
    """The kernel-apply autotuner's decisions so far (one line per shape)."""
    return _lib.hm_autotune_table().decode()


def mfma_rate(dtype=HM_F64, stream=None):
    """hm_mfma_rate: sustained TFLOP/s of the kernel apply's matrix-core
    instruction on the current device (independent chains, no memory)."""
    v = C.c_double(0.0)
    _check(_lib.hm_mfma_rate(dtype, _stream(stream), C.byref(v)))
    return v.value


def color(xadj, adj):
    """DSatur (hm_color) of a CSR graph; returns (colors, ncolors)."""
    xadj = np.ascontiguousarray(xadj, np.int64)
    adj = np.ascontiguousarray(adj if len(adj) else np.zeros(1, np.int32), np.int32)
    nv = len(xadj) - 1
    col = np.zeros(max(nv, 1), np.int32)
    nc = C.c_int32()
    _check(_lib.hm_color(nv, _ptr(xadj), _ptr(adj), _ptr(col), C.byref(nc)))
    return col[:nv], nc.value


def dense_blackbox(A, order=HM_ORDER_ORIGINAL):
    """Dense FP64 black box over a device (n, n) column-major tensor A (kept
    alive by the returned object)."""
    pa, lda, n2, dt = _colmajor(A, "A")
    if dt != HM_F64:
        raise TypeError("dense black box is FP64")
    bb = BlackBox()
    _check(_lib.hm_dense_blackbox(pa, A.shape[0], lda, order, C.byref(bb)))
    bb._keep = A
    return bb


def _own_ctx(bb):
    """Release the black box's ctx (hm_blackbox_free) when bb is collected."""
    import weakref
    copy = BlackBox(bb.apply, bb.ctx, bb.order, bb.symmetric, bb.dtypes)
    weakref.finalize(bb, lambda c=copy: _lib.hm_blackbox_free(C.byref(c)))


def product_blackbox(A, B):
    """The black box Y = A (B X) (hm_product_blackbox); keeps A and B alive."""
    bb = BlackBox()
    _check(_lib.hm_product_blackbox(C.byref(A), C.byref(B), C.byref(bb)))
    bb._keep = (A, B)
    _own_ctx(bb)
    return bb


def philox(ctr, key0, key1, out, stream=None):
    _check(_lib.hm_philox4x32_10(C.c_void_p(ctr.data_ptr()), ctr.numel() // 4, key0, key1,
                                 C.c_void_p(out.data_ptr()), _stream(stream)))


class HMatrix:
    def __init__(self, h, tree):
        self.h = h
        self.tree = tree

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.hm_hmatrix_free(self.h)
            self.h = None

    def stats(self):
        s = Stats()
        _check(_lib.hm_hmatrix_stats(self.h, C.byref(s)))
        return s.as_dict()

    def matvec_footprint(self, nrhs, dtype=np.float64):
        """Device bytes of scratch one matvec of nrhs columns takes (hm_matvec_footprint)."""
        b = C.c_int64()
        _check(_lib.hm_matvec_footprint(self.h, nrhs, HM_F32 if np.dtype(dtype) == np.float32
                                        else HM_F64, C.byref(b)))
        return b.value

    def matvec(self, X, Y, order=HM_ORDER_ORIGINAL, stream=None, trans=False):
        """Y = H X, or H* X with trans=True (hm_matvec_op)."""
        px, ldx, nc, dt = _colmajor(X, "X")
        py, ldy, nc2, dt2 = _colmajor(Y, "Y")
        if nc != nc2 or dt != dt2:
            raise ValueError("X and Y shapes/dtypes differ")
        _check(_lib.hm_matvec_op(self.h, 1 if trans else 0, nc, dt, px, ldx, py, ldy, order,
                                 _stream(stream)))

    def matvec_static(self, X, Y, order=HM_ORDER_ORIGINAL, stream=None, trans=False):
        """hm_matvec_static: matvec with the library's static device scratch
        (no allocation; calls on one device must not overlap)."""
        px, ldx, nc, dt = _colmajor(X, "X")
        py, ldy, nc2, dt2 = _colmajor(Y, "Y")
        if nc != nc2 or dt != dt2:
            raise ValueError("X and Y shapes/dtypes differ")
        _check(_lib.hm_matvec_static(self.h, 1 if trans else 0, nc, dt, px, ldx, py, ldy, order,
                                     _stream(stream)))

    def blackbox(self, order=HM_ORDER_ORIGINAL):
        """This operator as a black box (hm_hmatrix_blackbox); keeps self alive."""
        bb = BlackBox()
        _check(_lib.hm_hmatrix_blackbox(self.h, order, C.byref(bb)))
        bb._keep = self
        _own_ctx(bb)
        return bb

    def export_level(self, level):
        """List of (a, b, U, B, V) in pair order (host float64 arrays)."""
        npairs, su, sb, sv = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64()
        _check(_lib.hm_hmatrix_export_level(self.h, level, C.byref(npairs), None, None, None, None,
                                            C.byref(su), C.byref(sb), C.byref(sv), None, None, None))
        np_ = npairs.value
        if np_ == 0:
            return []
        pa, pb = np.zeros(np_, np.int32), np.zeros(np_, np.int32)
        ru, rv = np.zeros(np_, np.int32), np.zeros(np_, np.int32)
        U, B, V = np.zeros(max(su.value, 1)), np.zeros(max(sb.value, 1)), np.zeros(max(sv.value, 1))
        _check(_lib.hm_hmatrix_export_level(self.h, level, None, _ptr(pa), _ptr(pb), _ptr(ru),
                                            _ptr(rv), None, None, None, _ptr(U), _ptr(B), _ptr(V)))
        start = self.tree.level(level)[0]
        out = []
        ou = ob = ov = 0
        for q in range(np_):
            ma = int(start[pa[q] + 1] - start[pa[q]])
            mb = int(start[pb[q] + 1] - start[pb[q]])
            ku, kv = int(ru[q]), int(rv[q])
            Uq = U[ou:ou + ma * ku].reshape(ku, ma).T
            Bq = B[ob:ob + ku * kv].reshape(kv, ku).T
            Vq = V[ov:ov + mb * kv].reshape(kv, mb).T
            out.append((int(pa[q]), int(pb[q]), Uq, Bq, Vq))
            ou += ma * ku
            ob += ku * kv
            ov += mb * kv
        return out

    def export_near(self):
        npairs, size = C.c_int64(), C.c_int64()
        _check(_lib.hm_hmatrix_export_near(self.h, C.byref(npairs), None, None, C.byref(size), None))
        np_ = npairs.value
        pa, pb = np.zeros(max(np_, 1), np.int32), np.zeros(max(np_, 1), np.int32)
        D = np.zeros(max(size.value, 1))
        _check(_lib.hm_hmatrix_export_near(self.h, None, _ptr(pa), _ptr(pb), None, _ptr(D)))
        start = self.tree.level(self.tree.L)[0]
        out, o = [], 0
        for q in range(np_):
            ma = int(start[pa[q] + 1] - start[pa[q]])
            mb = int(start[pb[q] + 1] - start[pb[q]])
            out.append((int(pa[q]), int(pb[q]), D[o:o + ma * mb].reshape(mb, ma).T))
            o += ma * mb
        return out


class _Borrowed(HMatrix):
    """An H-matrix owned by a server (not freed here)."""

    def __del__(self):
        self.h = None


class Server:
    """hm_server: a request loop on one GPU with resident H-matrices.

    submit_* return request ids; a compression's H-matrix id is its request
    id.  Apply inputs and outputs are host arrays (n, nrhs); the output array
    of each apply is kept here until its completion is polled."""

    def __init__(self, nslots=4, hbm_budget=0, compress_slots=1, allocator=None):
        al, ap = _allocator(allocator)
        o = ServerOpts(hbm_budget=hbm_budget, nslots=nslots, compress_slots=compress_slots,
                       allocator=ap)
        h = C.c_void_p()
        _check(_lib.hm_server_create(C.byref(o), C.byref(h)))
        self.h = h
        self._alloc = al
        self._out = {}
        self._n = {}

    def close(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.hm_server_free(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def submit_compress(self, points, leaf, kind="geometric", adm="strong", kernel="log", rank=0,
                        tol=0.0, r=0, p=10, prec=HM_PREC_F64, seed=0, uniform=False,
                        h2=False):
        pts = np.ascontiguousarray(points, np.float64)
        if pts.ndim == 1:
            pts = pts.reshape(-1, 1)
        o = Opts(rank=rank, tol=tol, oversample=p, r=r, prec=prec, flags=0, seed=seed,
                 format=_format(uniform, h2))
        rid = C.c_int64()
        _check(_lib.hm_server_submit_compress(
            self.h, _ptr(pts), pts.shape[0], pts.shape[1], leaf,
            HM_TREE_INDEX_BINARY if kind == "index_binary" else HM_TREE_GEOMETRIC,
            HM_ADM_WEAK if adm == "weak" else HM_ADM_STRONG,
            HM_KERNEL_INV_R if kernel == "inv_r" else HM_KERNEL_LOG, C.byref(o), C.byref(rid)))
        self._n[rid.value] = pts.shape[0]
        return rid.value

    def submit_matvec(self, hmatrix, X):
        X = np.asarray(X)
        if X.ndim == 1:
            X = X.reshape(-1, 1)
        if X.dtype not in (np.float32, np.float64):
            raise ValueError("X must be float32 or float64")
        n, nrhs = X.shape
        if self._n.get(hmatrix) not in (None, n):
            raise ValueError("X has %d rows, the H-matrix %d" % (n, self._n[hmatrix]))
        Xc = np.ascontiguousarray(X.T)            # column-major n x nrhs
        Y = np.empty((nrhs, n), X.dtype)          # column-major n x nrhs
        rid = C.c_int64()
        _check(_lib.hm_server_submit_matvec(self.h, hmatrix, nrhs,
                                            HM_F32 if X.dtype == np.float32 else HM_F64,
                                            _ptr(Xc), _ptr(Y), C.byref(rid)))
        self._out[rid.value] = Y
        return rid.value

    def poll(self, max_count=256, wait_ms=0):
        buf = (Completion * max_count)()
        k = C.c_int32()
        _check(_lib.hm_server_poll(self.h, max_count, wait_ms, buf, C.byref(k)))
        out = []
        for c in buf[:k.value]:
            d = {name: getattr(c, name) for name, _ in Completion._fields_}
            Y = self._out.pop(c.id, None)
            if Y is not None:
                d["Y"] = Y.T                          # (n, nrhs) view
            out.append(d)
        return out

    def hmatrix(self, hmatrix):
        h = C.c_void_p()
        _check(_lib.hm_server_hmatrix(self.h, hmatrix, C.byref(h)))
        return _Borrowed(h, None)

    def release(self, hmatrix):
        _check(_lib.hm_server_release(self.h, hmatrix))

    def info(self):
        now, use, bud = C.c_double(), C.c_int64(), C.c_int64()
        pend, run, res = C.c_int32(), C.c_int32(), C.c_int32()
        _check(_lib.hm_server_info(self.h, C.byref(now), C.byref(use), C.byref(bud),
                                   C.byref(pend), C.byref(run), C.byref(res)))
        return dict(now=now.value, in_use=use.value, budget=bud.value, pending=pend.value,
                    running=run.value, residents=res.value)


HM_FLAG_TIMING, HM_FLAG_STRICT, HM_FLAG_MIX_GAMMA = 1, 2, 4


def _flags(timing, strict, combine):
    if combine not in ("sum", "gaussian"):
        raise ValueError("combine must be 'sum' or 'gaussian'")
    return ((HM_FLAG_TIMING if timing else 0) | (HM_FLAG_STRICT if strict else 0)
            | (HM_FLAG_MIX_GAMMA if combine == "gaussian" else 0))


def compress_footprint(tree: Tree, rank=0, tol=0.0, r=0, p=10, prec=HM_PREC_F64,
                       uniform=False, h2=False) -> int:
    """hm_compress_footprint: the most device bytes a compression of tree
    with these options holds at once (host computation, no device work)."""
    o = Opts(rank=rank, tol=tol, oversample=p, r=r, prec=prec, flags=0, seed=0,
             max_retries=0, format=_format(uniform, h2), allocator=None)
    b = C.c_int64()
    _check(_lib.hm_compress_footprint(tree.h, C.byref(o), C.byref(b)))
    return b.value


def compress(tree: Tree, bb: BlackBox, rank=0, tol=0.0, r=0, p=10, prec=HM_PREC_F64, seed=0,
             timing=False, stream=None, max_retries=0, strict=False, uniform=False,
             h2=False, combine="sum", allocator="torch") -> HMatrix:
    """hm_compress; uniform=True selects the uniform H^1 format, h2=True the
    H^2 format; combine="gaussian" sets HM_FLAG_MIX_GAMMA (their row bases
    from the Gaussian-weighted combination instead of the plain sum).
    allocator: "torch" (the default: every device block from PyTorch's
    caching allocator), a TorchAllocator, or None (the library's own)."""
    al, ap = _allocator(allocator)
    o = Opts(rank=rank, tol=tol, oversample=p, r=r, prec=prec,
             flags=_flags(timing, strict, combine),
             seed=seed, max_retries=max_retries, format=_format(uniform, h2), allocator=ap)
    h = C.c_void_p()
    _check(_lib.hm_compress(tree.h, C.byref(bb), C.byref(o), _stream(stream), C.byref(h)))
    tree._allocs.append(al)
    H = HMatrix(h, tree)
    H._alloc = al
    return H
