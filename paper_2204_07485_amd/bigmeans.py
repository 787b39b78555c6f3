"""Thin ctypes binding over libbigmeans.so (the C ABI in include/bigmeans.h).

Argument marshalling only: torch tensors supply device memory and the HIP
stream; every step of the computation runs in the library's HIP kernels.  The
library must have been built (``python -m paper_2204_07485_amd.build``); a
missing library is an error, there is no fallback.
"""
import ctypes as ct
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbigmeans.so")

BM_OK, BM_EINVAL, BM_ENOMEM, BM_EDEVICE, BM_ENOTSUP, BM_ECANCELLED = 0, -1, -2, -3, -4, -5
BM_ETIMEDOUT = -6
BM_JOB_QUEUED, BM_JOB_RUNNING, BM_JOB_DONE, BM_JOB_FAILED, BM_JOB_CANCELLED = 0, 1, 2, 3, 4
BM_SERVE_FITS, BM_SERVE_ROUNDS = 0, 1
BM_F32, BM_BF16 = 0, 1
BM_STOP_SHIFT, BM_STOP_REL_OBJ = 0, 1
BM_CMP_FOPT, BM_CMP_RESAMPLE = 0, 1
BM_PREC_FP32, BM_PREC_BF16_MFMA = 0, 1
BM_INIT_KMEANSPP, BM_INIT_FORGY = 0, 1
BM_FINAL_ASSIGN, BM_FINAL_POLISH = 0, 1

FUNCTIONS = ["bm_default_options", "bm_last_error", "bm_release_scratch", "bm_abi_version",
             "bigmeans_fit", "kmeans_assign", "kmeanspp_seed", "kmeans_lloyd",
             "bm_sample_indices", "bm_gather_rows", "kmeans_lloyd_batched",
             "bm_serve_default_config", "bm_ctx_create", "bm_ctx_submit", "bm_ctx_poll",
             "bm_ctx_wait", "bm_ctx_cancel", "bm_ctx_release", "bm_ctx_info", "bm_ctx_destroy",
             "kmeans_assign_noalloc", "bigmeans_fit_collective", "bigmeans_sample_size_sweep"]


class BigmeansError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"bigmeans error {code}: {msg}")
        self.code = code


class Options(ct.Structure):
    _fields_ = [("struct_size", ct.c_uint32), ("x_dtype", ct.c_int32),
                ("max_iter", ct.c_int32), ("tol", ct.c_double),
                ("stop_rule", ct.c_int32), ("n_local_trials", ct.c_int32),
                ("compare_rule", ct.c_int32), ("precision", ct.c_int32),
                ("stream", ct.c_void_p), ("grid", ct.c_int32), ("t_start", ct.c_int32),
                ("resume", ct.c_int32), ("f_opt_in", ct.c_double),
                ("spin_limit", ct.c_uint32), ("sample_idx", ct.c_void_p),
                ("sample_f", ct.c_void_p), ("init_method", ct.c_int32),
                ("final_mode", ct.c_int32), ("time_budget_ms", ct.c_double)]


class Stats(ct.Structure):
    _fields_ = [("struct_size", ct.c_uint32), ("samples", ct.c_int32),
                ("replacements", ct.c_int32), ("grid", ct.c_int32),
                ("lloyd_iters", ct.c_int64), ("reseeded", ct.c_int64), ("n_d", ct.c_int64),
                ("boundary_draws", ct.c_int64), ("f_opt", ct.c_double),
                ("ms_solver", ct.c_double), ("ms_final", ct.c_double),
                ("ms_sampling", ct.c_double), ("ms_seeding", ct.c_double),
                ("ms_lloyd", ct.c_double), ("ms_lloyd_pass", ct.c_double),
                ("ms_lloyd_post", ct.c_double), ("ms_lloyd_wait", ct.c_double),
                ("rechecked", ct.c_int64), ("final_passes", ct.c_int32), ("pad_", ct.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f not in ("struct_size", "pad_")}


class ServeConfig(ct.Structure):
    _fields_ = [("struct_size", ct.c_uint32), ("slots", ct.c_int32), ("hbm_budget", ct.c_int64),
                ("device", ct.c_int32), ("grid_per_job", ct.c_int32), ("mode", ct.c_int32),
                ("round_max_k", ct.c_int32), ("round_max_s", ct.c_int64)]


class Job(ct.Structure):
    _fields_ = [("struct_size", ct.c_uint32), ("X", ct.c_void_p), ("n", ct.c_int64),
                ("d", ct.c_int32), ("k", ct.c_int32), ("s", ct.c_int64), ("n_samples", ct.c_int32),
                ("seed", ct.c_uint64), ("opt", Options), ("centroids", ct.c_void_p),
                ("labels", ct.c_void_p), ("degenerate", ct.c_void_p), ("sse", ct.c_void_p),
                ("stats", ct.c_void_p)]


class JobInfo(ct.Structure):
    _fields_ = [("struct_size", ct.c_uint32), ("state", ct.c_int32), ("result", ct.c_int32),
                ("slot", ct.c_int32), ("footprint", ct.c_int64), ("t_submit_ms", ct.c_double),
                ("t_start_ms", ct.c_double), ("t_end_ms", ct.c_double), ("error", ct.c_char * 160)]


class ServeInfo(ct.Structure):
    _fields_ = [("struct_size", ct.c_uint32), ("slots", ct.c_int32), ("grid_per_job", ct.c_int32),
                ("submitted", ct.c_int64), ("completed", ct.c_int64), ("failed", ct.c_int64),
                ("cancelled", ct.c_int64), ("queued", ct.c_int64), ("running", ct.c_int64),
                ("reserved_bytes", ct.c_int64), ("peak_reserved_bytes", ct.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "struct_size"}


_LIB = None


def load(path=LIB_PATH):
    """Load libbigmeans.so (raises if it has not been built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with "
                           "`python -m paper_2204_07485_amd.build` (no CPU fallback exists)")
    L = ct.CDLL(path)
    P, I32, I64, U64 = ct.c_void_p, ct.c_int32, ct.c_int64, ct.c_uint64
    L.bm_default_options.argtypes = [P]
    L.bm_default_options.restype = I32
    L.bm_last_error.argtypes = []
    L.bm_last_error.restype = ct.c_char_p
    L.bm_release_scratch.argtypes = []
    L.bm_release_scratch.restype = I32
    L.bm_abi_version.argtypes = []
    L.bm_abi_version.restype = I32
    L.bigmeans_fit.argtypes = [P, I64, I32, I32, I64, I32, U64, P, P, P, P, P, P]
    L.bigmeans_fit.restype = I32
    L.kmeans_assign.argtypes = [P, I64, I32, P, P, I32, P, P, P, P]
    L.kmeans_assign.restype = I32
    L.kmeans_assign_noalloc.argtypes = [P, I64, I32, P, P, I32, P, P, P, P]
    L.kmeans_assign_noalloc.restype = I32
    L.bigmeans_fit_collective.argtypes = [P, I64, I32, I32, I64, I32, I32, U64, P, P, P, P, P, P, P]
    L.bigmeans_fit_collective.restype = I32
    L.bigmeans_sample_size_sweep.argtypes = [P, I64, I32, I32, I64, I64, I32, U64, P, P, P, P, P, P,
                                             P, P, I32, P]
    L.bigmeans_sample_size_sweep.restype = I32
    L.kmeanspp_seed.argtypes = [P, I64, I32, I32, P, P, U64, U64, P]
    L.kmeanspp_seed.restype = I32
    L.kmeans_lloyd.argtypes = [P, I64, I32, I32, P, P, P, P, P, P]
    L.kmeans_lloyd.restype = I32
    L.bm_sample_indices.argtypes = [I64, I64, U64, I32, P, P]
    L.bm_sample_indices.restype = I32
    L.bm_serve_default_config.argtypes = [P]
    L.bm_serve_default_config.restype = I32
    L.bm_ctx_create.argtypes = [P, P]
    L.bm_ctx_create.restype = I32
    L.bm_ctx_submit.argtypes = [P, P, P]
    L.bm_ctx_submit.restype = I32
    L.bm_ctx_poll.argtypes = [P, I64, P]
    L.bm_ctx_poll.restype = I32
    L.bm_ctx_wait.argtypes = [P, I64, I32, P]
    L.bm_ctx_wait.restype = I32
    L.bm_ctx_cancel.argtypes = [P, I64]
    L.bm_ctx_cancel.restype = I32
    L.bm_ctx_release.argtypes = [P, I64]
    L.bm_ctx_release.restype = I32
    L.bm_ctx_info.argtypes = [P, P]
    L.bm_ctx_info.restype = I32
    L.bm_ctx_destroy.argtypes = [P]
    L.bm_ctx_destroy.restype = I32
    L.bm_gather_rows.argtypes = [P, I64, I32, P, I64, P, P]
    L.bm_gather_rows.restype = I32
    L.kmeans_lloyd_batched.argtypes = [I32, P, I32, P, P, P, P, P, P, P, P]
    L.kmeans_lloyd_batched.restype = I32
    L.bm_debug_batch_info.argtypes = [P, P]
    L.bm_debug_batch_info.restype = I32
    L.bm_debug_batch_round_ms.argtypes = [I32]
    L.bm_debug_batch_round_ms.restype = ct.c_double
    L.bm_debug_rechecked.argtypes = []
    L.bm_debug_rechecked.restype = I64
    L.bm_debug_assign_ms.argtypes = []
    L.bm_debug_assign_ms.restype = ct.c_double
    _LIB = L
    return L


def _check(rc):
    if rc != BM_OK:
        msg = _LIB.bm_last_error().decode(errors="replace")
        raise BigmeansError(rc, msg)


def options(stream=None, **kw):
    """bm_options with defaults, overridden by keyword fields."""
    L = load()
    o = Options()
    _check(L.bm_default_options(ct.byref(o)))
    if stream is None and torch.cuda.is_available():
        stream = torch.cuda.current_stream().cuda_stream
    o.stream = stream
    for key, val in kw.items():
        if not hasattr(o, key):
            raise TypeError(f"unknown option {key}")
        setattr(o, key, val)
    return o


def _dev_ptr(t, dtype, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA/HIP tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ct.c_void_p(t.data_ptr())


def _x_ptr(X):
    if X.dtype == torch.float32:
        return _dev_ptr(X, torch.float32, "X"), BM_F32
    if X.dtype in (torch.uint16, torch.int16, torch.bfloat16):
        return ct.c_void_p(X.data_ptr()), BM_BF16
    raise TypeError("X must be float32, or bfloat16 / 16-bit BF16 bit patterns")


def bigmeans_fit(X, k, s, n_samples, seed, want_labels=True, want_sse=True, state=None,
                 sample_idx=False, sample_f=True, **opts):
    """Big-means on X (device tensor n x d).

    state: optional (centroids tensor, degenerate uint8 array, f_opt) to resume from.
    Returns a dict: centroids (k x d float32 tensor, NaN rows degenerate),
    degenerate (numpy uint8), sse, labels (int32 tensor or None), f_opt,
    sample_f (numpy), sample_idx (int32 tensor or None), stats.
    """
    L = load()
    n, d = X.shape
    xp, xdt = _x_ptr(X)
    o = options(x_dtype=xdt, **opts)
    cent = torch.empty((k, d), dtype=torch.float32, device=X.device)
    deg = np.ones(k, dtype=np.uint8)
    if state is not None:
        cent.copy_(state[0])
        deg[:] = np.asarray(state[1], dtype=np.uint8)
        o.resume = 1
        o.f_opt_in = float(state[2])
    labels = torch.empty(n, dtype=torch.int32, device=X.device) if want_labels else None
    sidx = torch.empty((n_samples, s), dtype=torch.int32, device=X.device) if sample_idx else None
    sf = np.zeros(n_samples, dtype=np.float64)
    if sidx is not None:
        o.sample_idx = sidx.data_ptr()
    if sample_f:
        o.sample_f = sf.ctypes.data
    sse = ct.c_double(0.0)
    st = Stats()
    st.struct_size = ct.sizeof(Stats)
    rc = L.bigmeans_fit(xp, n, d, k, s, n_samples, ct.c_uint64(seed), ct.byref(o),
                        ct.c_void_p(cent.data_ptr()),
                        ct.byref(sse) if want_sse else None,
                        ct.c_void_p(labels.data_ptr()) if labels is not None else None,
                        deg.ctypes.data_as(ct.c_void_p), ct.byref(st))
    _check(rc)
    return {"centroids": cent, "degenerate": deg, "sse": sse.value if want_sse else None,
            "labels": labels, "f_opt": st.f_opt, "sample_f": sf, "sample_idx": sidx,
            "stats": st.as_dict()}


def bigmeans_fit_collective(X, k, s, n_workers, n_rounds, seed, want_labels=True, **opts):
    """Collective parallel Big-means (bigmeans_fit_collective).  Returns a dict:
    centroids, degenerate, sse, labels, f_opt, worker_f (rounds x workers), stats."""
    L = load()
    n, d = X.shape
    xp, xdt = _x_ptr(X)
    o = options(x_dtype=xdt, **opts)
    cent = torch.empty((k, d), dtype=torch.float32, device=X.device)
    deg = np.ones(k, dtype=np.uint8)
    labels = torch.empty(n, dtype=torch.int32, device=X.device) if want_labels else None
    wf = np.zeros((n_rounds, n_workers), dtype=np.float64)
    sse = ct.c_double(0.0)
    st = Stats()
    st.struct_size = ct.sizeof(Stats)
    rc = L.bigmeans_fit_collective(xp, n, d, k, s, n_workers, n_rounds, ct.c_uint64(seed),
                                   ct.byref(o), ct.c_void_p(cent.data_ptr()), ct.byref(sse),
                                   ct.c_void_p(labels.data_ptr()) if labels is not None else None,
                                   deg.ctypes.data_as(ct.c_void_p), ct.byref(st),
                                   wf.ctypes.data_as(ct.c_void_p))
    _check(rc)
    return {"centroids": cent, "degenerate": deg, "sse": sse.value, "labels": labels,
            "f_opt": st.f_opt, "worker_f": wf, "stats": st.as_dict()}


def sample_size_sweep(X, k, s_min, s_max, n_samples, seed, want_labels=False, **opts):
    """The sample-size rule of thumb (bigmeans_sample_size_sweep).  Returns a
    dict: s_best, sse, centroids, degenerate, labels, tried [(s, sse), ...]."""
    L = load()
    n, d = X.shape
    xp, xdt = _x_ptr(X)
    o = options(x_dtype=xdt, **opts)
    cent = torch.empty((k, d), dtype=torch.float32, device=X.device)
    deg = np.ones(k, dtype=np.uint8)
    labels = torch.empty(n, dtype=torch.int32, device=X.device) if want_labels else None
    sse = ct.c_double(0.0)
    s_best = ct.c_int64(0)
    s_tried = np.zeros(64, dtype=np.int64)
    sse_tried = np.zeros(64, dtype=np.float64)
    m = ct.c_int32(0)
    rc = L.bigmeans_sample_size_sweep(xp, n, d, k, s_min, s_max, n_samples, ct.c_uint64(seed),
                                      ct.byref(o), ct.c_void_p(cent.data_ptr()), ct.byref(sse),
                                      ct.c_void_p(labels.data_ptr()) if labels is not None else None,
                                      deg.ctypes.data_as(ct.c_void_p), ct.byref(s_best),
                                      s_tried.ctypes.data_as(ct.c_void_p),
                                      sse_tried.ctypes.data_as(ct.c_void_p), 64, ct.byref(m))
    _check(rc)
    return {"s_best": s_best.value, "sse": sse.value, "centroids": cent, "degenerate": deg,
            "labels": labels,
            "tried": [(int(s_tried[i]), float(sse_tried[i])) for i in range(m.value)]}


def kmeans_assign(X, C, deg=None, want_labels=True, want_min_d2=False, **opts):
    return _assign("kmeans_assign", X, C, deg, want_labels, want_min_d2, opts)


def kmeans_assign_noalloc(X, C, deg=None, want_labels=True, want_min_d2=False, **opts):
    """kmeans_assign through the entry point whose scratch is a fixed device
    array (no device allocation by the library)."""
    return _assign("kmeans_assign_noalloc", X, C, deg, want_labels, want_min_d2, opts)


def _assign(entry, X, C, deg, want_labels, want_min_d2, opts):
    L = load()
    n, d = X.shape
    k = C.shape[0]
    xp, xdt = _x_ptr(X)
    o = options(x_dtype=xdt, **opts)
    cp = _dev_ptr(C, torch.float32, "C")
    dg = None if deg is None else np.ascontiguousarray(deg, dtype=np.uint8)
    labels = torch.empty(n, dtype=torch.int32, device=X.device) if want_labels else None
    mind = torch.empty(n, dtype=torch.float32, device=X.device) if want_min_d2 else None
    sse = ct.c_double(0.0)
    rc = getattr(L, entry)(xp, n, d, cp, None if dg is None else dg.ctypes.data_as(ct.c_void_p), k,
                           ct.byref(o), None if labels is None else ct.c_void_p(labels.data_ptr()),
                           None if mind is None else ct.c_void_p(mind.data_ptr()), ct.byref(sse))
    _check(rc)
    return labels, mind, sse.value


def kmeanspp_seed(P, C, deg, seed, stream_id, n_local_trials=3, **opts):
    """Reseed the slots of C (in place) with deg[j] = 1; returns the new flags."""
    L = load()
    s, d = P.shape
    k = C.shape[0]
    o = options(n_local_trials=n_local_trials, **opts)
    dg = np.array(deg, dtype=np.uint8, copy=True)
    rc = L.kmeanspp_seed(_dev_ptr(P, torch.float32, "P"), s, d, k, _dev_ptr(C, torch.float32, "C"),
                         dg.ctypes.data_as(ct.c_void_p), ct.c_uint64(seed),
                         ct.c_uint64(stream_id), ct.byref(o))
    _check(rc)
    return dg


def kmeans_lloyd(P, C, deg, **opts):
    """Lloyd on P from C (updated in place); returns (deg, labels, f, passes)."""
    L = load()
    s, d = P.shape
    k = C.shape[0]
    o = options(**opts)
    dg = np.array(deg, dtype=np.uint8, copy=True)
    labels = torch.empty(s, dtype=torch.int32, device=P.device)
    f = ct.c_double(0.0)
    passes = ct.c_int32(0)
    rc = L.kmeans_lloyd(_dev_ptr(P, torch.float32, "P"), s, d, k, _dev_ptr(C, torch.float32, "C"),
                        dg.ctypes.data_as(ct.c_void_p), ct.byref(o),
                        ct.c_void_p(labels.data_ptr()), ct.byref(f), ct.byref(passes))
    _check(rc)
    return dg, labels, f.value, passes.value


def sample_indices(n, s, seed, t, device="cuda", **opts):
    L = load()
    idx = torch.empty(s, dtype=torch.int32, device=device)
    o = options(**opts)
    rc = L.bm_sample_indices(n, s, ct.c_uint64(seed), t, ct.c_void_p(idx.data_ptr()), ct.byref(o))
    _check(rc)
    return idx


def gather_rows(X, idx, out=None, **opts):
    """P[r] = X[idx[r]] as FP32 (device tensors)."""
    L = load()
    n, d = X.shape
    xp, xdt = _x_ptr(X)
    o = options(x_dtype=xdt, **opts)
    s = idx.shape[0]
    P = out if out is not None else torch.empty((s, d), dtype=torch.float32, device=X.device)
    _check(L.bm_gather_rows(xp, n, d, _dev_ptr(idx, torch.int32, "idx"), s,
                            _dev_ptr(P, torch.float32, "P"), ct.byref(o)))
    return P


def kmeans_lloyd_batched(P, s, k, C, deg, want_labels=True, **opts):
    """Lloyd on many problems at once.  P: device (sum(s), d) FP32 rows of the
    problems in order; s, k: per-problem rows and centroids; C: device
    (sum(k), d) FP32 start centroids, updated in place; deg: sum(k) flags.
    Returns (deg, labels or None, f per problem, passes per problem, info)."""
    L = load()
    n_solves = len(s)
    d = P.shape[1]
    s_arr = np.ascontiguousarray(s, dtype=np.int64)
    k_arr = np.ascontiguousarray(k, dtype=np.int32)
    dg = np.array(deg, dtype=np.uint8, copy=True)
    o = options(**opts)
    labels = torch.empty(int(s_arr.sum()), dtype=torch.int32, device=P.device) if want_labels else None
    f = np.zeros(n_solves, dtype=np.float64)
    passes = np.zeros(n_solves, dtype=np.int32)
    _check(L.kmeans_lloyd_batched(n_solves, _dev_ptr(P, torch.float32, "P"), d,
                                  s_arr.ctypes.data_as(ct.c_void_p), k_arr.ctypes.data_as(ct.c_void_p),
                                  _dev_ptr(C, torch.float32, "C"), dg.ctypes.data_as(ct.c_void_p),
                                  ct.byref(o), None if labels is None else ct.c_void_p(labels.data_ptr()),
                                  f.ctypes.data_as(ct.c_void_p), passes.ctypes.data_as(ct.c_void_p)))
    rounds, tile = ct.c_int32(0), ct.c_int32(0)
    L.bm_debug_batch_info(ct.byref(rounds), ct.byref(tile))
    round_ms = [L.bm_debug_batch_round_ms(i) for i in range(rounds.value)]
    return dg, labels, f, passes, {"rounds": rounds.value, "tile_rows": tile.value,
                                   "round_ms": round_ms}


def prepare_batch(X, solves, n_local_trials=3, **opts):
    """Start problems for kmeans_lloyd_batched: for solve j = (s_j, k_j, seed_j),
    the sample of sample index 0 under seed_j (bm_sample_indices), its rows
    (bm_gather_rows) and k_j K-means++ centres on it (kmeanspp_seed), as the
    first sample of a Big-means run with that seed.  Returns (P, s, k, C, deg)."""
    s = np.array([sj for sj, _, _ in solves], dtype=np.int64)
    k = np.array([kj for _, kj, _ in solves], dtype=np.int32)
    d = X.shape[1]
    P = torch.empty((int(s.sum()), d), dtype=torch.float32, device=X.device)
    C = torch.empty((int(k.sum()), d), dtype=torch.float32, device=X.device)
    deg = np.ones(int(k.sum()), dtype=np.uint8)
    r = c = 0
    for sj, kj, seed in solves:
        idx = sample_indices(X.shape[0], sj, seed, 0, device=X.device)
        Pj = P[r:r + sj]
        gather_rows(X, idx, out=Pj, **opts)
        Cj = C[c:c + kj]
        deg[c:c + kj] = kmeanspp_seed(Pj, Cj, np.ones(kj, np.uint8), seed, 0,
                                      n_local_trials=n_local_trials, **opts)
        r += sj
        c += kj
    return P, s, k, C, deg


class Server:
    """A serving context (bm_ctx).  mode BM_SERVE_FITS: jobs run whole fits
    concurrently on `slots` workers, admitted in order by device-scratch
    footprint within hbm_budget.  mode BM_SERVE_ROUNDS: one engine keeps up to
    `slots` jobs in flight and runs their Lloyd rounds together in the batched
    kernels (jobs with s <= round_max_s and k <= round_max_k)."""

    def __init__(self, slots=4, hbm_budget=8 << 30, grid_per_job=0, mode=0, round_max_k=64,
                 round_max_s=50_000):
        L = load()
        cfg = ServeConfig()
        _check(L.bm_serve_default_config(ct.byref(cfg)))
        cfg.slots = slots
        cfg.hbm_budget = hbm_budget
        cfg.grid_per_job = grid_per_job
        cfg.mode = mode
        cfg.round_max_k = round_max_k
        cfg.round_max_s = round_max_s
        h = ct.c_void_p()
        _check(L.bm_ctx_create(ct.byref(cfg), ct.byref(h)))
        self._h = h
        self._jobs = {}

    def submit(self, X, k, s, n_samples, seed, want_labels=False, want_sse=True, **opts):
        """Queue bigmeans_fit(X, ...); returns a job id.  The outputs live in
        the record until result() is called."""
        L = load()
        n, d = X.shape
        xp, xdt = _x_ptr(X)
        o = options(x_dtype=xdt, stream=None, **opts)
        rec = {"X": X, "centroids": torch.empty((k, d), dtype=torch.float32, device=X.device),
               "labels": torch.empty(n, dtype=torch.int32, device=X.device) if want_labels else None,
               "deg": np.ones(k, dtype=np.uint8), "sse": ct.c_double(0.0), "stats": Stats(),
               "sample_f": np.zeros(n_samples, dtype=np.float64)}
        rec["stats"].struct_size = ct.sizeof(Stats)
        o.sample_f = rec["sample_f"].ctypes.data
        j = Job()
        j.struct_size = ct.sizeof(Job)
        j.X = xp
        j.n, j.d, j.k, j.s, j.n_samples, j.seed = n, d, k, s, n_samples, seed
        j.opt = o
        j.centroids = rec["centroids"].data_ptr()
        j.labels = rec["labels"].data_ptr() if want_labels else None
        j.degenerate = rec["deg"].ctypes.data
        j.sse = ct.addressof(rec["sse"]) if want_sse or want_labels else None
        j.stats = ct.addressof(rec["stats"])
        jid = ct.c_int64(0)
        _check(L.bm_ctx_submit(self._h, ct.byref(j), ct.byref(jid)))
        self._jobs[jid.value] = rec
        return jid.value

    def poll(self, jid):
        info = JobInfo()
        info.struct_size = ct.sizeof(JobInfo)
        _check(load().bm_ctx_poll(self._h, jid, ct.byref(info)))
        return info

    def wait(self, jid, timeout_ms=-1):
        info = JobInfo()
        info.struct_size = ct.sizeof(JobInfo)
        _check(load().bm_ctx_wait(self._h, jid, timeout_ms, ct.byref(info)))
        return info

    def cancel(self, jid):
        _check(load().bm_ctx_cancel(self._h, jid))

    def result(self, jid):
        """Wait for the job, then return its outputs (dict as bigmeans_fit) and
        its timing record; the record is released."""
        info = self.wait(jid)
        rec = self._jobs.pop(jid)
        _check(load().bm_ctx_release(self._h, jid))
        if info.state != BM_JOB_DONE:
            raise BigmeansError(info.result, info.error.decode(errors="replace"))
        return {"centroids": rec["centroids"], "degenerate": rec["deg"], "sse": rec["sse"].value,
                "labels": rec["labels"], "sample_f": rec["sample_f"],
                "stats": rec["stats"].as_dict(),
                "t_submit_ms": info.t_submit_ms, "t_start_ms": info.t_start_ms,
                "t_end_ms": info.t_end_ms, "slot": info.slot, "footprint": info.footprint}

    def info(self):
        inf = ServeInfo()
        inf.struct_size = ct.sizeof(ServeInfo)
        _check(load().bm_ctx_info(self._h, ct.byref(inf)))
        return inf.as_dict()

    def close(self):
        if self._h is not None:
            _check(load().bm_ctx_destroy(self._h))
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def debug_presample(mode):
    """Test hook: drawing all samples before the solver (0 automatic, 1 never,
    2 report a window miss so the solver draws them itself); returns the
    previous mode."""
    L = load()
    L.bm_debug_presample.argtypes = [ct.c_int32]
    L.bm_debug_presample.restype = ct.c_int32
    return L.bm_debug_presample(mode)


def last_rechecked():
    """Points the last BF16-MFMA kmeans_assign on this thread recomputed on the
    FP32 path (near ties)."""
    return int(load().bm_debug_rechecked())


def last_assign_ms():
    """Device time of the last kmeans_assign's kernel on this thread (ms)."""
    return float(load().bm_debug_assign_ms())


def release_scratch():
    _check(load().bm_release_scratch())


def debug_counters():
    """Raw device counters of this thread's last bigmeans_fit (bm_debug_counters):
    a dict of the per-phase clock ticks and event counts."""
    L = load()
    out = (ct.c_int64 * 28)()
    L.bm_debug_counters.argtypes = [ct.c_void_p, ct.c_int32]
    L.bm_debug_counters.restype = ct.c_int32
    _check(L.bm_debug_counters(out, 28))
    names = {0: "passes", 1: "reseeded", 2: "replaced", 3: "n_d", 4: "boundary", 5: "samples",
             6: "select_passes", 8: "ticks_sample", 9: "ticks_seed", 10: "ticks_lloyd",
             11: "ticks_pass", 12: "ticks_post", 13: "ticks_barrier", 14: "ticks_collect",
             15: "ticks_collect_wait", 16: "ticks_select", 17: "ticks_emit", 18: "ticks_assign",
             19: "ticks_flush", 20: "ticks_seed_init", 21: "ticks_seed_locate",
             22: "ticks_seed_pot", 23: "ticks_seed_update", 24: "ticks_assign_init",
             25: "ticks_assign_rows", 26: "ticks_assign_sum"}
    return {v: int(out[k]) for k, v in names.items()}


def debug_fp32_mfma(on):
    """FP32 full-data assignment: 1 = on the matrix cores when d >= 8,
    k >= 8 and k d >= 256 (default), 0 = on the VALU kernel; returns the
    previous value."""
    L = load()
    L.bm_debug_fp32_mfma.argtypes = [ct.c_int32]
    L.bm_debug_fp32_mfma.restype = ct.c_int32
    return L.bm_debug_fp32_mfma(on)


def debug_exact_draws(on):
    """K-means++ draws: 1 = every draw with row-order sums, 0 = only the draws
    near a running-sum boundary (default); returns the previous value."""
    L = load()
    L.bm_debug_exact_draws.argtypes = [ct.c_int32]
    L.bm_debug_exact_draws.restype = ct.c_int32
    return L.bm_debug_exact_draws(on)


def debug_mfma_lloyd(on):
    """BF16 matrix-core fits: 1 = sample-level K-means on the matrix cores
    (default), 0 = on the FP32 persistent solver; returns the previous value."""
    L = load()
    L.bm_debug_mfma_lloyd.argtypes = [ct.c_int32]
    L.bm_debug_mfma_lloyd.restype = ct.c_int32
    return L.bm_debug_mfma_lloyd(on)
