"""ctypes view of the FP64 CPU oracle (oracle/bm_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU
baseline leg of the benchmark, never by the GPU library or its binding.
Arrays are numpy; X is float32 (or uint16 holding BF16 bits), centroids are
float64, degenerate centroids are NaN rows with deg[j] = 1.

Every function runs the single-threaded build unless called inside
``with oracle.threaded():``, which switches to the OpenMP build (same source,
bit-identical results; for timing on all host cores and for large workloads).
"""
import contextlib
import ctypes as ct
import os

import numpy as np

from . import build_oracle

_LIBS = {}
_THREADED = False

ORC_F32, ORC_BF16 = 0, 1
ORC_STOP_SHIFT, ORC_STOP_REL_OBJ = 0, 1
ORC_CMP_FOPT, ORC_CMP_RESAMPLE = 0, 1
ORC_INIT_KMEANSPP, ORC_INIT_FORGY = 0, 1


class Opts(ct.Structure):
    _fields_ = [("max_iter", ct.c_int32), ("tol", ct.c_double),
                ("stop_rule", ct.c_int32), ("n_local_trials", ct.c_int32),
                ("compare_rule", ct.c_int32), ("init_method", ct.c_int32)]


class Stats(ct.Structure):
    _fields_ = [("samples", ct.c_int32), ("replacements", ct.c_int32),
                ("lloyd_iters", ct.c_int64), ("reseeded", ct.c_int64),
                ("n_d", ct.c_int64), ("f_opt", ct.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


def lib():
    """The oracle library in use (single-threaded, or OpenMP inside threaded())."""
    key = "omp" if _THREADED else "serial"
    if key not in _LIBS:
        path = build_oracle.LIB_OMP if _THREADED else build_oracle.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(build_oracle.SRC):
            build_oracle.build()
        L = ct.CDLL(path)
        P = ct.c_void_p
        L.orc_threads.restype = ct.c_int
        L.orc_philox4x32_10.argtypes = [P, P, P]
        L.orc_seed_word.argtypes = [ct.c_uint64, ct.c_uint32, ct.c_uint64]
        L.orc_seed_word.restype = ct.c_uint64
        L.orc_sample_key.argtypes = [ct.c_uint64, ct.c_uint32, ct.c_int64]
        L.orc_sample_key.restype = ct.c_uint64
        L.orc_sample.argtypes = [ct.c_int64, ct.c_int64, ct.c_uint64, ct.c_uint32, P]
        L.orc_dist2.argtypes = [P, P, ct.c_int32]
        L.orc_dist2.restype = ct.c_double
        L.orc_assign.argtypes = [P, ct.c_int64, ct.c_int32, P, P, ct.c_int32, P, P]
        L.orc_assign.restype = ct.c_double
        L.orc_d2_pick.argtypes = [P, ct.c_int64, ct.c_double]
        L.orc_d2_pick.restype = ct.c_int64
        L.orc_kmeanspp.argtypes = [P, ct.c_int64, ct.c_int32, ct.c_int32, P, P,
                                   ct.c_uint64, ct.c_uint32, ct.c_int32, P]
        L.orc_lloyd.argtypes = [P, ct.c_int64, ct.c_int32, ct.c_int32, P, P, P, P, P, P]
        L.orc_lloyd.restype = ct.c_double
        L.orc_bigmeans_fit.argtypes = [P, ct.c_int32, ct.c_int64, ct.c_int32, ct.c_int32,
                                       ct.c_int64, ct.c_int32, ct.c_uint64, P,
                                       ct.c_int32, ct.c_int32, P, P, P, P, P, P, P, P]
        L.orc_forgy.argtypes = [P, ct.c_int64, ct.c_int32, ct.c_int32, P, P, ct.c_uint64,
                                ct.c_uint32, P]
        L.orc_bigmeans_collective.argtypes = [P, ct.c_int32, ct.c_int64, ct.c_int32, ct.c_int32,
                                              ct.c_int64, ct.c_int32, ct.c_int32, ct.c_uint64, P,
                                              P, P, P, P, P, P, P]
        L.orc_sample_size_sweep.argtypes = [P, ct.c_int32, ct.c_int64, ct.c_int32, ct.c_int32,
                                            ct.c_int64, ct.c_int64, ct.c_int32, ct.c_uint64, P,
                                            P, P, P]
        L.orc_sample_size_sweep.restype = ct.c_int64
        _LIBS[key] = L
    return _LIBS[key]


@contextlib.contextmanager
def threaded():
    """Run the oracle calls inside this block on the OpenMP build."""
    global _THREADED
    prev = _THREADED
    _THREADED = True
    try:
        yield
    finally:
        _THREADED = prev


def threads():
    """Threads the library in use runs its per-point loops on."""
    return int(lib().orc_threads())


def _p(a):
    return None if a is None else a.ctypes.data_as(ct.c_void_p)


def make_opts(max_iter=100, tol=1e-4, stop_rule=ORC_STOP_SHIFT, n_local_trials=3,
              compare_rule=ORC_CMP_FOPT, init_method=ORC_INIT_KMEANSPP):
    return Opts(max_iter, tol, stop_rule, n_local_trials, compare_rule, init_method)


def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def seed_word(seed, t, q):
    return int(lib().orc_seed_word(seed, t, q))


def sample_key(seed, t, i):
    return int(lib().orc_sample_key(seed, t, i))


def sample(n, s, seed, t):
    idx = np.zeros(s, dtype=np.int32)
    rc = lib().orc_sample(n, s, seed, t, _p(idx))
    if rc != 0:
        raise ValueError(f"orc_sample failed ({rc})")
    return idx


def dist2(x, c):
    x = np.ascontiguousarray(x, dtype=np.float64)
    c = np.ascontiguousarray(c, dtype=np.float64)
    return float(lib().orc_dist2(_p(x), _p(c), x.shape[0]))


def assign(P, C, deg=None):
    P = np.ascontiguousarray(P, dtype=np.float64)
    C = np.ascontiguousarray(C, dtype=np.float64)
    s, d = P.shape
    k = C.shape[0]
    dg = None if deg is None else np.ascontiguousarray(deg, dtype=np.uint8)
    labels = np.zeros(s, dtype=np.int32)
    mind = np.zeros(s, dtype=np.float64)
    f = lib().orc_assign(_p(P), s, d, _p(C), _p(dg), k, _p(labels), _p(mind))
    return labels, mind, f


def d2_pick(w, target):
    """One D^2 draw by inverting the running sum of w at target."""
    w = np.ascontiguousarray(w, dtype=np.float64)
    return int(lib().orc_d2_pick(_p(w), w.shape[0], float(target)))


def kmeanspp(P, C, deg, seed, t, trials=3):
    """Reseed the slots with deg[j] = 1; returns (C, deg, stats) as new arrays."""
    P = np.ascontiguousarray(P, dtype=np.float64)
    C = np.array(C, dtype=np.float64, copy=True)
    deg = np.array(deg, dtype=np.uint8, copy=True)
    s, d = P.shape
    st = Stats()
    rc = lib().orc_kmeanspp(_p(P), s, d, C.shape[0], _p(C), _p(deg), seed, t, trials,
                            ct.byref(st))
    if rc != 0:
        raise ValueError(f"orc_kmeanspp failed ({rc})")
    return C, deg, st.as_dict()


def forgy(P, C, deg, seed, t):
    """Forgy-style reinitialisation of the slots with deg[j] = 1; returns (C, deg, stats)."""
    P = np.ascontiguousarray(P, dtype=np.float64)
    C = np.array(C, dtype=np.float64, copy=True)
    deg = np.array(deg, dtype=np.uint8, copy=True)
    s, d = P.shape
    st = Stats()
    rc = lib().orc_forgy(_p(P), s, d, C.shape[0], _p(C), _p(deg), seed, t, ct.byref(st))
    if rc != 0:
        raise ValueError(f"orc_forgy failed ({rc})")
    return C, deg, st.as_dict()


def lloyd(P, C, deg, max_iter=100, tol=1e-4, stop_rule=ORC_STOP_SHIFT):
    """Lloyd from C on P; returns (C, deg, labels, f, passes, stats)."""
    P = np.ascontiguousarray(P, dtype=np.float64)
    C = np.array(C, dtype=np.float64, copy=True)
    deg = np.array(deg, dtype=np.uint8, copy=True)
    s, d = P.shape
    o = make_opts(max_iter, tol, stop_rule)
    labels = np.zeros(s, dtype=np.int32)
    iters = ct.c_int32(0)
    st = Stats()
    f = lib().orc_lloyd(_p(P), s, d, C.shape[0], _p(C), _p(deg), ct.byref(o), _p(labels),
                        ct.byref(iters), ct.byref(st))
    return C, deg, labels, f, iters.value, st.as_dict()


def bigmeans_fit(X, k, s, n_samples, seed, max_iter=100, tol=1e-4,
                 stop_rule=ORC_STOP_SHIFT, n_local_trials=3, compare_rule=ORC_CMP_FOPT,
                 t_start=0, state=None, want_labels=True, want_sse=True,
                 want_sample_idx=False, x_dtype=None, init_method=ORC_INIT_KMEANSPP):
    """Big-means (Alg. 1).  X: float32 (n, d), or uint16 BF16 bits with x_dtype=ORC_BF16.

    state: optional (C, deg, f_opt) incumbent to resume from.
    Returns a dict with C, deg, f_opt, labels, sse, sample_f, sample_idx, stats.
    """
    if x_dtype is None:
        x_dtype = ORC_BF16 if X.dtype == np.uint16 else ORC_F32
    X = np.ascontiguousarray(X)
    n, d = X.shape
    o = make_opts(max_iter, tol, stop_rule, n_local_trials, compare_rule, init_method)
    if state is not None:
        C = np.array(state[0], dtype=np.float64, copy=True)
        deg = np.array(state[1], dtype=np.uint8, copy=True)
        f_opt = ct.c_double(state[2])
        resume = 1
    else:
        C = np.zeros((k, d), dtype=np.float64)
        deg = np.ones(k, dtype=np.uint8)
        f_opt = ct.c_double(0.0)
        resume = 0
    labels = np.zeros(n, dtype=np.int32) if want_labels else None
    sse = ct.c_double(0.0)
    sample_f = np.zeros(max(n_samples, 1), dtype=np.float64)
    sample_idx = np.zeros((max(n_samples, 1), s), dtype=np.int32) if want_sample_idx else None
    st = Stats()
    rc = lib().orc_bigmeans_fit(_p(X), x_dtype, n, d, k, s, n_samples, seed, ct.byref(o),
                                t_start, resume, _p(C), _p(deg), ct.byref(f_opt),
                                _p(labels), ct.byref(sse) if want_sse else None,
                                _p(sample_f), _p(sample_idx), ct.byref(st))
    if rc != 0:
        raise ValueError(f"orc_bigmeans_fit failed ({rc})")
    return {"C": C, "deg": deg, "f_opt": f_opt.value, "labels": labels,
            "sse": sse.value if want_sse else None, "sample_f": sample_f[:n_samples],
            "sample_idx": None if sample_idx is None else sample_idx[:n_samples],
            "stats": st.as_dict()}


def _x_dtype(X, x_dtype):
    if x_dtype is None:
        x_dtype = ORC_BF16 if X.dtype == np.uint16 else ORC_F32
    return np.ascontiguousarray(X), x_dtype


def bigmeans_collective(X, k, s, n_workers, n_rounds, seed, max_iter=100, tol=1e-4,
                        stop_rule=ORC_STOP_SHIFT, n_local_trials=3, init_method=ORC_INIT_KMEANSPP,
                        want_labels=True, x_dtype=None):
    """Collective parallel Big-means (Sec. 3.6, third scheme).  Returns a dict
    with C, deg, f_opt, labels, sse, worker_f (rounds x workers), stats."""
    X, x_dtype = _x_dtype(X, x_dtype)
    n, d = X.shape
    o = make_opts(max_iter, tol, stop_rule, n_local_trials, ORC_CMP_FOPT, init_method)
    C = np.zeros((k, d), dtype=np.float64)
    deg = np.ones(k, dtype=np.uint8)
    f_opt = ct.c_double(0.0)
    labels = np.zeros(n, dtype=np.int32) if want_labels else None
    sse = ct.c_double(0.0)
    wf = np.zeros((n_rounds, n_workers), dtype=np.float64)
    st = Stats()
    rc = lib().orc_bigmeans_collective(_p(X), x_dtype, n, d, k, s, n_workers, n_rounds, seed,
                                       ct.byref(o), _p(C), _p(deg), ct.byref(f_opt), _p(labels),
                                       ct.byref(sse), _p(wf), ct.byref(st))
    if rc != 0:
        raise ValueError(f"orc_bigmeans_collective failed ({rc})")
    return {"C": C, "deg": deg, "f_opt": f_opt.value, "labels": labels, "sse": sse.value,
            "worker_f": wf, "stats": st.as_dict()}


def sample_size_sweep(X, k, s_min, s_max, n_samples, seed, max_iter=100, tol=1e-4,
                      stop_rule=ORC_STOP_SHIFT, n_local_trials=3, x_dtype=None):
    """The sample-size rule of thumb (Sec. 5).  Returns (best s, [(s, sse), ...])."""
    X, x_dtype = _x_dtype(X, x_dtype)
    n, d = X.shape
    o = make_opts(max_iter, tol, stop_rule, n_local_trials)
    s_tried = np.zeros(64, dtype=np.int64)
    sse_tried = np.zeros(64, dtype=np.float64)
    m = ct.c_int32(0)
    best = lib().orc_sample_size_sweep(_p(X), x_dtype, n, d, k, s_min, s_max, n_samples, seed,
                                       ct.byref(o), _p(s_tried), _p(sse_tried), ct.byref(m))
    if best < 0:
        raise ValueError(f"orc_sample_size_sweep failed ({best})")
    return int(best), [(int(s_tried[i]), float(sse_tried[i])) for i in range(m.value)]
