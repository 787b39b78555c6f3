"""Host-side checks of the C ABI (no GPU): the library loads, exports every
function include/bigmeans.h and include/bigmeans_debug.h declare and nothing
else of C linkage, and rejects invalid arguments with BM_EINVAL before
touching the device."""
import ctypes as ct
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bigmeans.h")
DEBUG_HEADER = os.path.join(ROOT, "include", "bigmeans_debug.h")


def _declared_functions(path=HEADER):
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:bm_status|const char\*|int32_t|int64_t|double)\s+(\w+)\s*\(",
                                 text, re.M)))


def _exported_c_symbols(path):
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", path], check=True, capture_output=True,
                         text=True).stdout
    names = {line.split()[-1] for line in out.splitlines() if line.strip()}
    # C++ symbols are mangled (_Z...); __hip_cuid_* identify the code objects
    return sorted(n for n in names if not n.startswith("_Z") and not n.startswith("__hip_cuid_"))


@pytest.fixture(scope="module")
def bm():
    from paper_2204_07485_amd import bigmeans
    return bigmeans


def test_library_exports_every_declared_function(bm):
    lib = bm.load()
    names = _declared_functions()
    assert {"bigmeans_fit", "kmeans_assign", "kmeanspp_seed"} <= set(names)
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(bm.FUNCTIONS)


def test_every_exported_symbol_is_declared(bm):
    bm.load()
    declared = set(_declared_functions(HEADER)) | set(_declared_functions(DEBUG_HEADER))
    exported = set(_exported_c_symbols(bm.LIB_PATH))
    assert exported == declared, (sorted(exported - declared), sorted(declared - exported))
    for name in _declared_functions(DEBUG_HEADER):
        assert name.startswith("bm_debug_"), name


def test_abi_version_and_struct_sizes(bm):
    lib = bm.load()
    assert lib.bm_abi_version() == 2
    o = bm.Options()
    assert lib.bm_default_options(ct.byref(o)) == 0
    assert o.struct_size == ct.sizeof(bm.Options)
    assert o.max_iter == 100 and o.n_local_trials == 3 and abs(o.tol - 1e-4) < 1e-18


def _fit(bm, n=10, d=2, k=2, s=5, T=1, X=1, C=1, opt=None, deg=None):
    lib = bm.load()
    sse = ct.c_double()
    return lib.bigmeans_fit(ct.c_void_p(X), n, d, k, s, T, ct.c_uint64(1),
                            None if opt is None else ct.byref(opt), ct.c_void_p(C),
                            ct.byref(sse), None, deg, None)


@pytest.mark.parametrize("kw", [dict(k=6, s=5), dict(s=11), dict(d=0), dict(n=0, s=0, k=0),
                                dict(T=0), dict(X=0), dict(C=0), dict(n=2**31, s=5)])
def test_fit_rejects_invalid_sizes(bm, kw):
    assert _fit(bm, **kw) == bm.BM_EINVAL
    assert bm.load().bm_last_error()


@pytest.mark.parametrize("field,value", [("max_iter", 0), ("n_local_trials", 0),
                                         ("n_local_trials", 9), ("stop_rule", 7),
                                         ("compare_rule", 5), ("x_dtype", 3), ("tol", -1.0),
                                         ("grid", 5000), ("struct_size", 3)])
def test_fit_rejects_invalid_options(bm, field, value):
    o = bm.Options()
    bm.load().bm_default_options(ct.byref(o))
    setattr(o, field, value)
    assert _fit(bm, opt=o) == bm.BM_EINVAL


def test_resume_requires_flags(bm):
    o = bm.Options()
    bm.load().bm_default_options(ct.byref(o))
    o.resume = 1
    assert _fit(bm, opt=o) == bm.BM_EINVAL


def test_other_entry_points_reject_invalid_arguments(bm):
    lib = bm.load()
    deg = np.ones(3, np.uint8)
    p = deg.ctypes.data_as(ct.c_void_p)
    assert lib.kmeans_assign(ct.c_void_p(1), 0, 2, ct.c_void_p(1), None, 2, None, None, None, None) == bm.BM_EINVAL
    assert lib.kmeans_assign(ct.c_void_p(1), 5, 2, ct.c_void_p(1), p, 3, None, None, None, None) == bm.BM_EINVAL
    assert lib.kmeanspp_seed(None, 5, 2, 3, ct.c_void_p(1), p, ct.c_uint64(1), ct.c_uint64(0), None) == bm.BM_EINVAL
    assert lib.kmeanspp_seed(ct.c_void_p(1), 5, 2, 3, ct.c_void_p(1), p, ct.c_uint64(1), ct.c_uint64(2**32), None) == bm.BM_EINVAL
    assert lib.kmeans_lloyd(ct.c_void_p(1), 5, 2, 3, ct.c_void_p(1), p, None, None, None, None) == bm.BM_EINVAL
    assert lib.bm_sample_indices(5, 6, ct.c_uint64(1), 0, ct.c_void_p(1), None) == bm.BM_EINVAL
    assert lib.bm_sample_indices(5, 3, ct.c_uint64(1), -1, ct.c_void_p(1), None) == bm.BM_EINVAL
    assert lib.bm_default_options(None) == bm.BM_EINVAL


def test_product_philox_matches_oracle_on_host():
    # the GPU library's generator header compiled for the host, against the
    # oracle's independent implementation, on 10^6 counters
    import subprocess
    import oracle
    src = os.path.join(ROOT, "tests", "philox_host_check.cpp")
    exe = os.path.join(ROOT, "tests", "_build", "philox_host_check")
    os.makedirs(os.path.dirname(exe), exist_ok=True)
    if not os.path.exists(exe) or os.path.getmtime(exe) < max(
            os.path.getmtime(src),
            os.path.getmtime(os.path.join(ROOT, "paper_2204_07485_amd", "csrc", "bm_rng.h"))):
        subprocess.run(["hipcc", "--offload-arch=gfx950", "-O2", "-std=c++17", src, "-o", exe], check=True)
    out = subprocess.run([exe, "1000000", "12345"], capture_output=True, text=True, check=True).stdout
    got = [int(v) for v in out.split()]
    # the program prints an xor-fold of all sample keys and draws, plus spot values
    seed, t = 12345, 7
    spots = [0, 1, 999_999, 500_001]
    want = [oracle.sample_key(seed, t, i) for i in spots] + [oracle.seed_word(seed, t, q) for q in spots]
    assert got[:8] == want
    fold = 0
    for i in range(0, 1_000_000, 997):
        fold ^= oracle.sample_key(seed, t, i) ^ oracle.seed_word(seed, t, i)
    assert got[8] == fold


def test_batched_and_gather_reject_invalid_arguments(bm):
    lib = bm.load()
    P = ct.c_void_p(16)
    C = ct.c_void_p(16)

    def batched(n_solves, s, k, deg, P=P, C=C):
        s = np.ascontiguousarray(s, np.int64)
        k = np.ascontiguousarray(k, np.int32)
        return lib.kmeans_lloyd_batched(n_solves, P, 2, s.ctypes.data_as(ct.c_void_p),
                                        k.ctypes.data_as(ct.c_void_p), C,
                                        deg.ctypes.data_as(ct.c_void_p), None, None, None, None)

    deg = np.zeros(9, np.uint8)
    assert batched(2, [10, 5], [3, 6], deg) == bm.BM_EINVAL          # k > s
    assert batched(0, [10], [3], deg) == bm.BM_EINVAL                # no solves
    assert batched(2, [10, 0], [3, 1], deg) == bm.BM_EINVAL          # empty solve
    assert batched(1, [10], [3], deg, P=None) == bm.BM_EINVAL        # no P
    assert batched(1, [10], [3], np.ones(3, np.uint8)) == bm.BM_EINVAL  # all degenerate
    idx = ct.c_void_p(16)
    assert lib.bm_gather_rows(ct.c_void_p(16), 0, 2, idx, 5, P, None) == bm.BM_EINVAL
    assert lib.bm_gather_rows(ct.c_void_p(16), 10, 2, None, 5, P, None) == bm.BM_EINVAL
    assert lib.bm_gather_rows(ct.c_void_p(16), 10, 0, idx, 5, P, None) == bm.BM_EINVAL
    assert lib.bm_last_error()


def test_serving_rejects_invalid_arguments(bm):
    lib = bm.load()
    cfg = bm.ServeConfig()
    assert lib.bm_serve_default_config(ct.byref(cfg)) == 0
    assert cfg.slots == 4 and cfg.struct_size == ct.sizeof(bm.ServeConfig)
    assert cfg.mode == bm.BM_SERVE_FITS and cfg.round_max_k == 64 and cfg.round_max_s == 50_000
    h = ct.c_void_p()
    for field, value in (("slots", 0), ("slots", 65), ("hbm_budget", 1000), ("grid_per_job", -1),
                         ("struct_size", 2), ("mode", 2), ("mode", -1)):
        c2 = bm.ServeConfig()
        lib.bm_serve_default_config(ct.byref(c2))
        setattr(c2, field, value)
        assert lib.bm_ctx_create(ct.byref(c2), ct.byref(h)) == bm.BM_EINVAL, field
    for field, value in (("round_max_k", 0), ("round_max_s", 0), ("round_max_s", 1 << 31)):
        c2 = bm.ServeConfig()
        lib.bm_serve_default_config(ct.byref(c2))
        c2.mode = bm.BM_SERVE_ROUNDS
        setattr(c2, field, value)
        assert lib.bm_ctx_create(ct.byref(c2), ct.byref(h)) == bm.BM_EINVAL, field
    assert lib.bm_ctx_create(ct.byref(cfg), None) == bm.BM_EINVAL
    jid = ct.c_int64()
    assert lib.bm_ctx_submit(None, None, ct.byref(jid)) == bm.BM_EINVAL
    info = bm.JobInfo()
    info.struct_size = ct.sizeof(bm.JobInfo)
    assert lib.bm_ctx_poll(None, 1, ct.byref(info)) == bm.BM_EINVAL
    assert lib.bm_ctx_wait(None, 1, 0, None) == bm.BM_EINVAL
    assert lib.bm_ctx_cancel(None, 1) == bm.BM_EINVAL
    assert lib.bm_ctx_destroy(None) == bm.BM_OK
