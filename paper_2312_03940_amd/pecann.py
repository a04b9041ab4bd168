"""Thin ctypes binding of libpecann.so (include/pecann.h).

Argument marshalling only: tensors are passed as raw device pointers together
with torch's current HIP stream; every step of the computation runs in the
library's kernels.  There is no fallback: if the library is missing, or no
GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes
import os
import re

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
# PECANN_LIB: another build of the library to load (the sanitizer tests use it)
LIB_PATH = os.environ.get("PECANN_LIB") or os.path.join(_HERE, "libpecann.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "pecann.h")

F32, U8, BF16, FP8E4M3, MXFP6 = 0, 1, 2, 3, 4
L2, COSINE = 0, 1
CENTER_PRODUCT, CENTER_THRESHOLD, CENTER_GIVEN = 0, 1, 2
DENSITY_FNS = {"kth": 0, "normalized": 1, "exp-sum": 2, "sum-exp": 3, "sum": 4}
DTYPES = {"f32": F32, "u8": U8, "bf16": BF16, "fp8": FP8E4M3, "mxfp6": MXFP6}
METRICS = {"l2": L2, "cosine": COSINE}


class PecannError(RuntimeError):
    pass


class _Dataset(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("d", ctypes.c_int32), ("metric", ctypes.c_int32),
                ("search_dtype", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("prep", ctypes.c_void_p)]


class _ProfileEntry(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double)]


class _BuildParams(ctypes.Structure):
    _fields_ = [("R", ctypes.c_int32), ("L", ctypes.c_int32), ("alpha", ctypes.c_float),
                ("num_starts", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("visited_cap", ctypes.c_int32), ("passes", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class _NndParams(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int32), ("R", ctypes.c_int32), ("alpha", ctypes.c_float),
                ("max_iters", ctypes.c_int32), ("delta", ctypes.c_float),
                ("num_repeats", ctypes.c_int32), ("chunk", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class _Tuning(ctypes.Structure):
    _fields_ = [("hash_bits_build", ctypes.c_int32), ("hash_bits_search", ctypes.c_int32),
                ("grid_per_cu", ctypes.c_int32), ("scorer", ctypes.c_int32),
                ("prune_steps", ctypes.c_int32)]


class _Instances(ctypes.Structure):
    _fields_ = [("num_instances", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("offsets", ctypes.POINTER(ctypes.c_int64)), ("k", ctypes.POINTER(ctypes.c_int32)),
                ("n_c", ctypes.POINTER(ctypes.c_int32))]


class Instances:
    """Independent instances over one point set: instance t owns rows
    [offsets[t], offsets[t+1]); optional per-instance k and n_c (host arrays)."""

    def __init__(self, offsets, k=None, n_c=None):
        import numpy as np
        self.offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        self.count = len(self.offsets) - 1
        self.k = None if k is None else np.ascontiguousarray(k, dtype=np.int32)
        self.n_c = None if n_c is None else np.ascontiguousarray(n_c, dtype=np.int32)
        if self.count < 1 or (self.k is not None and len(self.k) != self.count) or \
                (self.n_c is not None and len(self.n_c) != self.count):
            raise PecannError("instance tables have inconsistent lengths")

    @property
    def k_max(self) -> int:
        return int(self.k.max()) if self.k is not None else 0

    @property
    def struct(self):
        def p(a, t):
            return None if a is None else a.ctypes.data_as(ctypes.POINTER(t))
        return _Instances(self.count, 0, p(self.offsets, ctypes.c_int64), p(self.k, ctypes.c_int32),
                          p(self.n_c, ctypes.c_int32))


_lib = None


def header_functions():
    """Names of the functions declared in include/pecann.h."""
    with open(HEADER) as f:
        txt = f.read()
    return sorted(set(re.findall(r"\b(pecann_[a-z_0-9]+)\s*\(", txt)))


def load():
    """Load libpecann.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise PecannError(f"{LIB_PATH} is missing: build it with `python -m paper_2312_03940_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, f32, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float, ctypes.c_size_t
    D = ctypes.POINTER(_Dataset)
    B = ctypes.POINTER(_BuildParams)
    N = ctypes.POINTER(_Instances)
    sig = {
        "pecann_prepared_bytes": (sz, [i64, i32, i32, i32]),
        "pecann_prepare_vectors": (ctypes.c_int, [vp, i32, i64, i64, i32, i32, i32, vp, sz, vp]),
        "pecann_build_graph_workspace_size": (sz, [D, B]),
        "pecann_build_graph": (ctypes.c_int, [D, B, vp, ctypes.c_uint64, vp, vp, vp, vp, sz, vp]),
        "pecann_knn_density_workspace_size": (sz, [D, i32, i32, i32]),
        "pecann_knn_density": (ctypes.c_int, [D, vp, vp, i32, i32, i32, i32, vp, vp, vp, vp, vp, vp,
                                              sz, vp]),
        "pecann_dependent_search_workspace_size": (sz, [D, i32, i32]),
        "pecann_dependent_search": (ctypes.c_int, [D, vp, vp, i32, vp, vp, vp, i32, i32, i32, i32,
                                                   i32, vp, vp, vp, vp, sz, vp]),
        "pecann_cluster_workspace_size": (sz, [i64]),
        "pecann_cluster": (ctypes.c_int, [i64, vp, vp, vp, i32, i32, f32, f32, vp, vp, vp, sz, vp]),
        "pecann_profile_enable": (ctypes.c_int, [i32]),
        "pecann_profile_report": (i32, [ctypes.POINTER(_ProfileEntry), i32]),
        "pecann_build_graph_batched_workspace_size": (sz, [D, B, N]),
        "pecann_build_graph_batched": (ctypes.c_int, [D, B, N, vp, ctypes.c_uint64, vp, vp, vp, vp, sz,
                                                      vp]),
        "pecann_knn_density_batched_workspace_size": (sz, [D, N, i32, i32, i32]),
        "pecann_knn_density_batched": (ctypes.c_int, [D, N, vp, vp, i32, i32, i32, i32, vp, vp, vp, vp,
                                                      vp, vp, sz, vp]),
        "pecann_dependent_search_batched_workspace_size": (sz, [D, N, i32, i32]),
        "pecann_dependent_search_batched": (ctypes.c_int, [D, N, vp, vp, i32, vp, vp, vp, i32, i32, i32,
                                                           i32, i32, vp, vp, vp, vp, sz, vp]),
        "pecann_cluster_batched_workspace_size": (sz, [i64, N]),
        "pecann_cluster_batched": (ctypes.c_int, [i64, N, vp, vp, vp, i32, i32, f32, f32, vp, vp, vp, sz,
                                                  vp]),
        "pecann_density_workspace_size": (sz, [i64, N]),
        "pecann_density": (ctypes.c_int, [i64, N, i32, i32, vp, vp, vp, vp, vp, sz, vp]),
        "pecann_local_centers_workspace_size": (sz, [i64, N]),
        "pecann_local_centers": (ctypes.c_int, [i64, N, i32, vp, vp, vp, f32, vp, vp, sz, vp]),
        "pecann_build_graph_nndescent_workspace_size": (sz, [D, ctypes.POINTER(_NndParams)]),
        "pecann_build_graph_nndescent": (ctypes.c_int, [D, ctypes.POINTER(_NndParams), vp, vp, vp, vp,
                                                        vp, vp, vp, vp, sz, vp]),
        "pecann_set_tuning": (ctypes.c_int, [ctypes.POINTER(_Tuning)]),
        "pecann_get_tuning": (ctypes.c_int, [ctypes.POINTER(_Tuning)]),
        "pecann_read_probe": (ctypes.c_int, [vp, sz, i32, ctypes.c_uint32, vp, vp]),
        "pecann_cluster_noalloc": (ctypes.c_int, [i64, vp, vp, vp, i32, i32, f32, f32, vp, vp, vp]),
        "pecann_status_string": (ctypes.c_char_p, [ctypes.c_int]),
        "pecann_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(rc: int):
    if rc != 0:
        lib = load()
        raise PecannError(f"{lib.pecann_status_string(rc).decode()}: {lib.pecann_last_error().decode()}")


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _need_cuda(*ts):
    for t in ts:
        if t is not None and not t.is_cuda:
            raise PecannError("tensors must live on the GPU")


def _ws(nbytes: int, device):
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


class Dataset:
    """A prepared point set (pecann_prepare_vectors output) kept on the GPU."""

    def __init__(self, x: torch.Tensor, metric="l2", search_dtype="f32"):
        _need_cuda(x)
        lib = load()
        if x.dim() != 2:
            raise PecannError("x must be 2-D (n, d)")
        if x.dtype == torch.float32:
            xdt = F32
        elif x.dtype == torch.uint8:
            xdt = U8
        else:
            raise PecannError("x must be float32 or uint8")
        if x.stride(1) != 1:
            x = x.contiguous()
        self.n, self.d = x.shape
        self.metric = METRICS[metric] if isinstance(metric, str) else int(metric)
        self.search_dtype = DTYPES[search_dtype] if isinstance(search_dtype, str) else int(search_dtype)
        nb = lib.pecann_prepared_bytes(self.n, self.d, self.metric, self.search_dtype)
        if nb == 0:
            raise PecannError("invalid (n, d, metric, search dtype)")
        self.prep = torch.empty(nb, dtype=torch.uint8, device=x.device)
        self.device = x.device
        self.prepare(x)

    def prepare(self, x: torch.Tensor):
        """(Re)write the prepared buffer from rows x of the same shape (no allocation)."""
        _need_cuda(x)
        if tuple(x.shape) != (self.n, self.d) or x.stride(1) != 1:
            raise PecannError("x must match the dataset's (n, d) with unit column stride")
        xdt = F32 if x.dtype == torch.float32 else U8 if x.dtype == torch.uint8 else None
        if xdt is None:
            raise PecannError("x must be float32 or uint8")
        _check(load().pecann_prepare_vectors(_ptr(x), xdt, x.stride(0), self.n, self.d, self.metric,
                                             self.search_dtype, _ptr(self.prep), self.prep.numel(),
                                             _stream()))

    @property
    def struct(self):
        return _Dataset(self.n, self.d, self.metric, self.search_dtype, 0, self.prep.data_ptr())


def build_graph(ds: Dataset, R: int, L: int, alpha: float, num_starts: int = 8,
                max_batch: int = 0, visited_cap: int = 0, perm: torch.Tensor | None = None,
                seed: int = 0, passes: int = 2, ws: torch.Tensor | None = None, out=None,
                counters: torch.Tensor | None = None):
    """Batched Vamana construction.  -> (adj int32 [n, R], deg int32 [n]).

    counters: optional int64 device tensor of 8 entries, accumulated (see pecann.h)."""
    lib = load()
    s = ds.struct
    bp = _BuildParams(R, L, alpha, num_starts, max_batch, visited_cap, passes, 0)
    need = lib.pecann_build_graph_workspace_size(ctypes.byref(s), ctypes.byref(bp))
    if need == 0:
        raise PecannError("invalid build parameters")
    if ws is None or ws.numel() < need:
        ws = _ws(need, ds.device)
    if perm is not None:
        _need_cuda(perm)
        if perm.dtype != torch.int32 or perm.numel() != ds.n:
            raise PecannError("perm must be int32 with n entries")
    if out is None:
        out = (torch.empty((ds.n, R), dtype=torch.int32, device=ds.device),
               torch.empty(ds.n, dtype=torch.int32, device=ds.device))
    adj, deg = out
    _check(lib.pecann_build_graph(ctypes.byref(s), ctypes.byref(bp), _ptr(perm), seed, _ptr(adj),
                                  _ptr(deg), _ptr(counters), _ptr(ws), ws.numel(), _stream()))
    return adj, deg


def set_tuning(hash_bits_build: int = 0, hash_bits_search: int = 0, grid_per_cu: int = 0,
               scorer: int = 0, prune_steps: int = 0):
    """Launch settings of this host thread (0 = the library's rule).  The hash
    sizes, the grid and prune_steps (the prune tiles' row steps per memory
    round trip, 2 or 4) change speed only; scorer (1 = vector units, 2 = matrix
    cores) picks where BF16 / FP8 candidates are scored, which changes the
    rounding of their search measures."""
    t = _Tuning(hash_bits_build, hash_bits_search, grid_per_cu, scorer, prune_steps)
    _check(load().pecann_set_tuning(ctypes.byref(t)))


def reset_tuning():
    _check(load().pecann_set_tuning(None))


def get_tuning() -> dict:
    t = _Tuning()
    _check(load().pecann_get_tuning(ctypes.byref(t)))
    return {"hash_bits_build": t.hash_bits_build, "hash_bits_search": t.hash_bits_search,
            "grid_per_cu": t.grid_per_cu, "scorer": t.scorer, "prune_steps": t.prune_steps}


def build_graph_nndescent(ds: Dataset, K: int, R: int, alpha: float, init: torch.Tensor,
                          max_iters: int = 20, delta: float = 0.001, chunk: int = 0,
                          ws: torch.Tensor | None = None, out=None, counters: torch.Tensor | None = None):
    """NN-descent graph (second index).  init: int32 device tensor [num_repeats, n, K]
    (or [n, K]) of starting neighbour ids.
    -> (adj int32 [n, R], deg int32 [n], knn_idx int32 [n, K], knn_dist f32 [n, K],
        rounds int32 [num_repeats])."""
    lib = load()
    s = ds.struct
    _need_cuda(init)
    if init.dim() == 2:
        init = init.unsqueeze(0)
    if init.dtype != torch.int32 or tuple(init.shape[1:]) != (ds.n, K) or not init.is_contiguous():
        raise PecannError("init must be a contiguous int32 tensor [num_repeats, n, K]")
    reps = init.shape[0]
    npar = _NndParams(K, R, alpha, max_iters, delta, reps, chunk, 0)
    need = lib.pecann_build_graph_nndescent_workspace_size(ctypes.byref(s), ctypes.byref(npar))
    if need == 0:
        raise PecannError("invalid NN-descent parameters")
    if ws is None or ws.numel() < need:
        ws = _ws(need, ds.device)
    if out is None:
        out = (torch.empty((ds.n, R), dtype=torch.int32, device=ds.device),
               torch.empty(ds.n, dtype=torch.int32, device=ds.device),
               torch.empty((ds.n, K), dtype=torch.int32, device=ds.device),
               torch.empty((ds.n, K), dtype=torch.float32, device=ds.device),
               torch.empty(reps, dtype=torch.int32, device=ds.device))
    adj, deg, idx, dist, rounds = out
    _check(lib.pecann_build_graph_nndescent(ctypes.byref(s), ctypes.byref(npar), _ptr(init), _ptr(adj),
                                            _ptr(deg), _ptr(idx), _ptr(dist), _ptr(rounds),
                                            _ptr(counters), _ptr(ws), ws.numel(), _stream()))
    return adj, deg, idx, dist, rounds


def workspace_bytes_nndescent(ds: Dataset, K: int, R: int, alpha: float = 1.2, max_iters: int = 20,
                              delta: float = 0.001, num_repeats: int = 1, chunk: int = 0) -> int:
    npar = _NndParams(K, R, alpha, max_iters, delta, num_repeats, chunk, 0)
    return int(load().pecann_build_graph_nndescent_workspace_size(ctypes.byref(ds.struct),
                                                                   ctypes.byref(npar)))


def knn_density(ds: Dataset, k: int, adj=None, deg=None, L_search: int = 64, rerank: int | None = None,
                ws: torch.Tensor | None = None, out=None, counters: torch.Tensor | None = None):
    """kNN + kth density.  -> (knn_idx int32 [n,k], knn_dist f32 [n,k], rho f32 [n], rank_key int64 [n])."""
    lib = load()
    s = ds.struct
    R = 0 if adj is None else adj.shape[1]
    if rerank is None:
        rerank = min(L_search, max(k, 2 * k))
    need = lib.pecann_knn_density_workspace_size(ctypes.byref(s), k, L_search, 1 if adj is None else 0)
    if ws is None or ws.numel() < need:
        ws = _ws(need, ds.device)
    if out is None:
        out = (torch.empty((ds.n, k), dtype=torch.int32, device=ds.device),
               torch.empty((ds.n, k), dtype=torch.float32, device=ds.device),
               torch.empty(ds.n, dtype=torch.float32, device=ds.device),
               torch.empty(ds.n, dtype=torch.int64, device=ds.device))
    idx, dist, rho, key = out
    _check(lib.pecann_knn_density(ctypes.byref(s), _ptr(adj), _ptr(deg), R, k, L_search, rerank,
                                  _ptr(idx), _ptr(dist), _ptr(rho), _ptr(key), _ptr(counters),
                                  _ptr(ws), ws.numel(), _stream()))
    return idx, dist, rho, key


def dependent_search(ds: Dataset, rank_key, knn_idx, knn_dist, adj=None, deg=None, L_d: int = 32,
                     L_search: int = 64, threshold: int = 300, kdep_cap: int = 1024,
                     ws: torch.Tensor | None = None, out=None):
    """Alg. 3.  -> (dep int32 [n], delta f32 [n], stats int32 [32])."""
    lib = load()
    s = ds.struct
    k = knn_idx.shape[1]
    R = 0 if adj is None else adj.shape[1]
    need = lib.pecann_dependent_search_workspace_size(ctypes.byref(s), kdep_cap, L_search)
    if ws is None or ws.numel() < need:
        ws = _ws(need, ds.device)
    if out is None:
        out = (torch.empty(ds.n, dtype=torch.int32, device=ds.device),
               torch.empty(ds.n, dtype=torch.float32, device=ds.device),
               torch.zeros(32, dtype=torch.int32, device=ds.device))
    dep, delta, stats = out
    _check(lib.pecann_dependent_search(ctypes.byref(s), _ptr(adj), _ptr(deg), R, _ptr(rank_key),
                                       _ptr(knn_idx), _ptr(knn_dist), k, L_d, L_search, threshold,
                                       kdep_cap, _ptr(dep), _ptr(delta), _ptr(stats), _ptr(ws),
                                       ws.numel(), _stream()))
    return dep, delta, stats


def profile_enable(on: bool = True):
    """Start (clearing earlier records) or stop HIP-event timing of every library launch."""
    _check(load().pecann_profile_enable(1 if on else 0))


def profile_report() -> dict:
    """Synchronise recorded events; -> {family: (launches, total_ms)}."""
    buf = (_ProfileEntry * 16)()
    m = load().pecann_profile_report(buf, 16)
    if m < 0:
        raise PecannError("pecann_profile_report failed")
    return {buf[i].name.decode(): (int(buf[i].launches), float(buf[i].total_ms)) for i in range(m)}


def workspace_bytes(ds: Dataset, k: int, L_search: int, kdep_cap: int, R: int, L: int,
                    alpha: float = 1.2, num_starts: int = 8, max_batch: int = 0,
                    visited_cap: int = 0, passes: int = 2) -> int:
    """One workspace size that serves every call of a DPC run on ds."""
    lib = load()
    s = ds.struct
    bp = _BuildParams(R, L, alpha, num_starts, max_batch, visited_cap, passes, 0)
    return max(lib.pecann_build_graph_workspace_size(ctypes.byref(s), ctypes.byref(bp)),
               lib.pecann_knn_density_workspace_size(ctypes.byref(s), k, L_search, 0),
               lib.pecann_dependent_search_workspace_size(ctypes.byref(s), kdep_cap, L_search),
               lib.pecann_cluster_workspace_size(ds.n))


def cluster(rho, dep, delta, n_c: int = 1, center_mode: int = CENTER_PRODUCT,
            delta_min: float = 0.0, rho_min: float = 0.0, ws: torch.Tensor | None = None, out=None):
    """Noise, centers, labels.  -> (labels int32 [n], is_center uint8 [n])."""
    lib = load()
    n = rho.numel()
    need = lib.pecann_cluster_workspace_size(n)
    if ws is None or ws.numel() < need:
        ws = _ws(need, rho.device)
    if out is None:
        out = (torch.empty(n, dtype=torch.int32, device=rho.device),
               torch.empty(n, dtype=torch.uint8, device=rho.device))
    labels, isc = out
    _check(lib.pecann_cluster(n, _ptr(rho), _ptr(dep), _ptr(delta), center_mode, n_c, delta_min,
                              rho_min, _ptr(labels), _ptr(isc), _ptr(ws), ws.numel(), _stream()))
    return labels, isc


# ---------------------------------------------------------------------------
# Batches of independent instances (pecann_*_batched)
# ---------------------------------------------------------------------------
def build_graph_batched(ds: Dataset, inst: Instances, R: int, L: int, alpha: float,
                        num_starts: int = 8, max_batch: int = 0, visited_cap: int = 0,
                        perm: torch.Tensor | None = None, seed: int = 0, passes: int = 2,
                        ws: torch.Tensor | None = None, out=None,
                        counters: torch.Tensor | None = None):
    """Vamana construction of every instance.  -> (adj int32 [n, R], deg int32 [n])."""
    lib = load()
    s, ni = ds.struct, inst.struct
    bp = _BuildParams(R, L, alpha, num_starts, max_batch, visited_cap, passes, 0)
    need = lib.pecann_build_graph_batched_workspace_size(ctypes.byref(s), ctypes.byref(bp),
                                                         ctypes.byref(ni))
    if need == 0:
        raise PecannError(f"invalid build parameters or instances: {lib.pecann_last_error().decode()}")
    if ws is None or ws.numel() < need:
        ws = _ws(need, ds.device)
    if perm is not None:
        _need_cuda(perm)
        if perm.dtype != torch.int32 or perm.numel() != ds.n:
            raise PecannError("perm must be int32 with n entries")
    if out is None:
        out = (torch.empty((ds.n, R), dtype=torch.int32, device=ds.device),
               torch.empty(ds.n, dtype=torch.int32, device=ds.device))
    adj, deg = out
    _check(lib.pecann_build_graph_batched(ctypes.byref(s), ctypes.byref(bp), ctypes.byref(ni),
                                          _ptr(perm), seed, _ptr(adj), _ptr(deg), _ptr(counters),
                                          _ptr(ws), ws.numel(), _stream()))
    return adj, deg


def knn_density_batched(ds: Dataset, inst: Instances, k_max: int, adj=None, deg=None,
                        L_search: int = 64, rerank: int | None = None,
                        ws: torch.Tensor | None = None, out=None,
                        counters: torch.Tensor | None = None):
    """kNN + kth density of every instance; rows of stride k_max.
    -> (knn_idx int32 [n,k_max], knn_dist f32 [n,k_max], rho f32 [n], rank_key int64 [n])."""
    lib = load()
    s, ni = ds.struct, inst.struct
    R = 0 if adj is None else adj.shape[1]
    if rerank is None:
        rerank = min(L_search, 2 * k_max)
    need = lib.pecann_knn_density_batched_workspace_size(ctypes.byref(s), ctypes.byref(ni), k_max,
                                                         L_search, 1 if adj is None else 0)
    if need == 0:
        raise PecannError(f"invalid instances: {lib.pecann_last_error().decode()}")
    if ws is None or ws.numel() < need:
        ws = _ws(need, ds.device)
    if out is None:
        out = (torch.empty((ds.n, k_max), dtype=torch.int32, device=ds.device),
               torch.empty((ds.n, k_max), dtype=torch.float32, device=ds.device),
               torch.empty(ds.n, dtype=torch.float32, device=ds.device),
               torch.empty(ds.n, dtype=torch.int64, device=ds.device))
    idx, dist, rho, key = out
    _check(lib.pecann_knn_density_batched(ctypes.byref(s), ctypes.byref(ni), _ptr(adj), _ptr(deg), R,
                                          k_max, L_search, rerank, _ptr(idx), _ptr(dist), _ptr(rho),
                                          _ptr(key), _ptr(counters), _ptr(ws), ws.numel(), _stream()))
    return idx, dist, rho, key


def dependent_search_batched(ds: Dataset, inst: Instances, rank_key, knn_idx, knn_dist, adj=None,
                             deg=None, L_d: int = 32, L_search: int = 64, threshold: int = 300,
                             kdep_cap: int = 1024, ws: torch.Tensor | None = None, out=None):
    """Alg. 3 on every instance.  -> (dep int32 [n], delta f32 [n], stats int32 [32])."""
    lib = load()
    s, ni = ds.struct, inst.struct
    k_max = knn_idx.shape[1]
    R = 0 if adj is None else adj.shape[1]
    need = lib.pecann_dependent_search_batched_workspace_size(ctypes.byref(s), ctypes.byref(ni),
                                                              kdep_cap, L_search)
    if need == 0:
        raise PecannError(f"invalid instances: {lib.pecann_last_error().decode()}")
    if ws is None or ws.numel() < need:
        ws = _ws(need, ds.device)
    if out is None:
        out = (torch.empty(ds.n, dtype=torch.int32, device=ds.device),
               torch.empty(ds.n, dtype=torch.float32, device=ds.device),
               torch.zeros(32, dtype=torch.int32, device=ds.device))
    dep, delta, stats = out
    _check(lib.pecann_dependent_search_batched(ctypes.byref(s), ctypes.byref(ni), _ptr(adj), _ptr(deg),
                                               R, _ptr(rank_key), _ptr(knn_idx), _ptr(knn_dist), k_max,
                                               L_d, L_search, threshold, kdep_cap, _ptr(dep),
                                               _ptr(delta), _ptr(stats), _ptr(ws), ws.numel(),
                                               _stream()))
    return dep, delta, stats


def cluster_batched(inst: Instances, rho, dep, delta, n_c: int = 1,
                    center_mode: int = CENTER_PRODUCT, delta_min: float = 0.0,
                    rho_min: float = 0.0, ws: torch.Tensor | None = None, out=None):
    """Noise, centers, labels of every instance.  -> (labels int32 [n], is_center uint8 [n])."""
    lib = load()
    n = rho.numel()
    ni = inst.struct
    need = lib.pecann_cluster_batched_workspace_size(n, ctypes.byref(ni))
    if need == 0:
        raise PecannError(f"invalid instances: {lib.pecann_last_error().decode()}")
    if ws is None or ws.numel() < need:
        ws = _ws(need, rho.device)
    if out is None:
        out = (torch.empty(n, dtype=torch.int32, device=rho.device),
               torch.empty(n, dtype=torch.uint8, device=rho.device))
    labels, isc = out
    _check(lib.pecann_cluster_batched(n, ctypes.byref(ni), _ptr(rho), _ptr(dep), _ptr(delta),
                                      center_mode, n_c, delta_min, rho_min, _ptr(labels), _ptr(isc),
                                      _ptr(ws), ws.numel(), _stream()))
    return labels, isc


def workspace_bytes_batched(ds: Dataset, inst: Instances, k_max: int, L_search: int, kdep_cap: int,
                            R: int, L: int, alpha: float = 1.2, num_starts: int = 8,
                            max_batch: int = 0, visited_cap: int = 0, passes: int = 2,
                            exact: bool = False) -> int:
    """One workspace size that serves every batched call of a DPC run on ds."""
    lib = load()
    s, ni = ds.struct, inst.struct
    bp = _BuildParams(R, L, alpha, num_starts, max_batch, visited_cap, passes, 0)
    return max(lib.pecann_build_graph_batched_workspace_size(ctypes.byref(s), ctypes.byref(bp),
                                                             ctypes.byref(ni)),
               lib.pecann_knn_density_batched_workspace_size(ctypes.byref(s), ctypes.byref(ni), k_max,
                                                             L_search, 1 if exact else 0),
               lib.pecann_dependent_search_batched_workspace_size(ctypes.byref(s), ctypes.byref(ni),
                                                                  kdep_cap, L_search),
               lib.pecann_cluster_batched_workspace_size(ds.n, ctypes.byref(ni)))


# ---------------------------------------------------------------------------
# Other density functions and local centers
# ---------------------------------------------------------------------------
def density(knn_idx, knn_dist, fn: str = "normalized", inst: Instances | None = None,
            out=None, ws: torch.Tensor | None = None):
    """Density of another function from the kNN lists (rows of stride knn_idx.shape[1]).
    -> (rho f32 [n], rank_key int64 [n]); out may be knn_density's (rho, rank_key).
    fn="kth" leaves rank_key as it is (the keys knn_density wrote for these
    lists), so it needs out=(rho, rank_key) holding them."""
    lib = load()
    n, k = knn_idx.shape
    if fn == "kth" and out is None:
        raise ValueError("density(fn='kth') keeps knn_density's rank keys: pass out=(rho, rank_key)")
    ni = None if inst is None else ctypes.byref(inst.struct)
    need = lib.pecann_density_workspace_size(n, ni)
    if need == 0:
        raise PecannError(f"invalid arguments: {lib.pecann_last_error().decode()}")
    if ws is None or ws.numel() < need:
        ws = _ws(need, knn_idx.device)
    if out is None:
        out = (torch.empty(n, dtype=torch.float32, device=knn_idx.device),
               torch.empty(n, dtype=torch.int64, device=knn_idx.device))
    rho, key = out
    _check(lib.pecann_density(n, ni, k, DENSITY_FNS[fn], _ptr(knn_idx), _ptr(knn_dist), _ptr(rho),
                              _ptr(key), _ptr(ws), ws.numel(), _stream()))
    return rho, key


def local_centers(knn_idx, rank_key, rho, rho_min: float = 0.0, inst: Instances | None = None,
                  out: torch.Tensor | None = None, ws: torch.Tensor | None = None):
    """Non-noise points ranked above all their k nearest neighbours. -> is_center uint8 [n]."""
    lib = load()
    n, k = knn_idx.shape
    ni = None if inst is None else ctypes.byref(inst.struct)
    need = lib.pecann_local_centers_workspace_size(n, ni)
    if need == 0:
        raise PecannError(f"invalid arguments: {lib.pecann_last_error().decode()}")
    if ws is None or ws.numel() < need:
        ws = _ws(need, knn_idx.device)
    isc = torch.empty(n, dtype=torch.uint8, device=knn_idx.device) if out is None else out
    _check(lib.pecann_local_centers(n, ni, k, _ptr(knn_idx), _ptr(rank_key), _ptr(rho), rho_min,
                                    _ptr(isc), _ptr(ws), ws.numel(), _stream()))
    return isc


def read_probe(buf: torch.Tensor, passes: int = 1, sink: torch.Tensor | None = None):
    """Read the whole of `buf` `passes` times on the current stream (a bandwidth
    measurement aid).  -> the sink tensor the kernel may write."""
    lib = load()
    _need_cuda(buf)
    if sink is None:
        sink = torch.zeros(1, dtype=torch.int32, device=buf.device)
    nbytes = buf.numel() * buf.element_size()
    _check(lib.pecann_read_probe(_ptr(buf), nbytes - nbytes % 16, passes, 0x5bd1e995, _ptr(sink),
                                 _stream()))
    return sink


def cluster_noalloc(rho, dep, delta, n_c: int = 1, center_mode: int | None = None,
                    delta_min: float = 0.0, rho_min: float = 0.0, out=None):
    """pecann_cluster through the entry point that allocates nothing (its scratch
    is the library's fixed device array; n <= 2^21).  out: (labels, is_center),
    preallocated by a caller that cannot allocate.  -> (labels, is_center)."""
    lib = load()
    _need_cuda(rho, dep, delta)
    n = rho.numel()
    mode = CENTER_PRODUCT if center_mode is None else center_mode
    if out is None:
        out = (torch.empty(n, dtype=torch.int32, device=rho.device),
               torch.empty(n, dtype=torch.uint8, device=rho.device))
    labels, isc = out
    _check(lib.pecann_cluster_noalloc(n, _ptr(rho), _ptr(dep), _ptr(delta), mode, n_c, delta_min, rho_min,
                                      _ptr(labels), _ptr(isc), _stream()))
    return labels, isc
