"""GPU parity of the batched Lloyd (kmeans_lloyd_batched): every problem of a
batch must come out as kmeans_lloyd run on it alone, and as the oracle's
K-means (Sec. 2, stop rules of Sec. 5, empty clusters degenerate, Sec. 3.3).

As for the single-problem tests, a near-tie label flip changes a whole
trajectory, so a problem is compared strictly (labels, flags, passes,
objective, centroids) when the oracle's own trajectory never comes within
the near-tie band, and otherwise checked for self-consistency."""
import numpy as np
import pytest
import torch

import oracle
from paper_2204_07485_amd import synth
from tests.parity import LABEL_TIE_REL, assert_centroids, assert_labels, assert_sse, top2_gap

pytestmark = pytest.mark.gpu


def _oracle_min_gap(P, C0, deg0, steps, **kw):
    """Smallest relative top-2 gap along the oracle's trajectory."""
    C = np.asarray(C0, np.float64)
    deg = np.array(deg0, np.uint8)
    g = np.inf
    for _ in range(steps):
        C32 = C.astype(np.float32)
        if (~deg.astype(bool)).sum() > 1:
            g = min(g, float(top2_gap(P, C32, deg).min()))
        rC, rdeg, _, _, _, _ = oracle.lloyd(P, C32, deg, max_iter=1, tol=0.0)
        if np.allclose(rC, C, equal_nan=True, rtol=0, atol=0):
            break
        C, deg = rC, rdeg
    return g


def _problems(specs, d, seed):
    """specs: list of (s, k); returns per-problem (P, C0, deg0)."""
    out = []
    for q, (s, k) in enumerate(specs):
        P = synth.gaussian_mixture(s, d, max(k, 2), seed + q, sigma_range=(0.5, 2.0),
                                   weights="dirichlet")[0]
        rng = np.random.default_rng(seed + 100 + q)
        C0 = P[rng.choice(s, k, replace=False)].copy()
        out.append((P, C0, np.zeros(k, np.uint8)))
    return out


def _run_batched(probs, **kw):
    from paper_2204_07485_amd import bigmeans
    P = torch.from_numpy(np.concatenate([p for p, _, _ in probs])).cuda()
    C = torch.from_numpy(np.concatenate([c for _, c, _ in probs]).astype(np.float32)).cuda()
    deg = np.concatenate([g for _, _, g in probs])
    s = [len(p) for p, _, _ in probs]
    k = [len(c) for _, c, _ in probs]
    dg, lab, f, passes, info = bigmeans.kmeans_lloyd_batched(P, s, k, C, deg, **kw)
    C = C.cpu().numpy()
    lab = lab.cpu().numpy()
    res = []
    r = c = 0
    for j in range(len(probs)):
        res.append((C[c:c + k[j]], dg[c:c + k[j]], lab[r:r + s[j]], f[j], passes[j]))
        r += s[j]
        c += k[j]
    return res, info


def _single(P, C0, deg, **kw):
    from paper_2204_07485_amd import bigmeans
    Cd = torch.from_numpy(np.ascontiguousarray(C0, np.float32)).cuda()
    dg, lab, f, passes = bigmeans.kmeans_lloyd(torch.from_numpy(P).cuda(), Cd, deg, **kw)
    return Cd.cpu().numpy(), dg, lab.cpu().numpy(), f, passes


def _compare(P, C0, deg0, got, ref, strict):
    gC, gdeg, glab, gf, gp = got
    rC, rdeg, rlab, rf, rp = ref
    if strict:
        assert_labels(glab, rlab, P, rC, rdeg)
        assert gp == rp, f"passes {gp} vs {rp}"
        assert np.array_equal(gdeg, rdeg)
        assert_sse(gf, rf)
        assert_centroids(gC, rC, rdeg, P, rlab)
    else:
        P64 = P.astype(np.float64)
        own = ((P64 - gC.astype(np.float64)[glab]) ** 2).sum()
        assert_sse(gf, own)
        assert_labels(glab, oracle.assign(P, gC, gdeg)[0], P, gC, gdeg)
        assert abs(gf - rf) <= 0.05 * rf


# Problems (by index in `specs`) whose oracle trajectory comes within the
# near-tie band, per parametrisation; computed from the oracle alone.  Only
# these take the relaxed whole-run check (after a lock-step check of the
# batched kernels along the oracle's path), and only when the strict one fails.
NEAR_TIE_PROBLEMS = {(2, 1, 300): {5, 8}, (16, 0, 100): {4, 5, 8}, (68, 1, 300): {2, 4, 5, 6, 8},
                     (5, 0, 1): {5}, (128, 1, 50): {4, 5, 8}}


def _lockstep_batched(P, C0, deg0, steps):
    """The batched kernels started from every oracle iterate (one round each):
    the update must equal the oracle's, unless the oracle's assignment at that
    iterate has a near tie (then a flipped point may move a centroid); the
    labels returned for the updated centroids are their nearest ones."""
    C = np.asarray(C0, np.float64)
    deg = np.array(deg0, np.uint8)
    for _ in range(steps):
        C32 = C.astype(np.float32)
        got, _ = _run_batched([(P, C32, deg)], max_iter=1, tol=0.0)
        gC, gdeg, glab, gf, gp = got[0]
        assert gp == 2
        rC, rdeg, rlab, _, _, _ = oracle.lloyd(P, C32, deg, max_iter=1, tol=0.0)
        near = (~deg.astype(bool)).sum() > 1 and float(top2_gap(P, C32, deg).min()) < LABEL_TIE_REL
        try:
            assert np.array_equal(gdeg, rdeg)
            assert_centroids(gC, rC, rdeg, P, rlab)
        except AssertionError:
            if not near:
                raise
        assert_labels(glab, oracle.assign(P, gC, gdeg)[0], P, gC, gdeg)
        if np.allclose(rC, C, equal_nan=True, rtol=0, atol=0):
            break
        C, deg = rC, rdeg


@pytest.mark.parametrize("d,rule,max_iter", [(2, 1, 300), (16, 0, 100), (68, 1, 300), (5, 0, 1),
                                             (128, 1, 50)])
def test_batched_matches_single_and_oracle(d, rule, max_iter):
    specs = [(1, 1), (7, 3), (257, 5), (1_000, 10), (5_003, 25), (20_000, 50), (2_048, 2),
             (777, 7), (30_000, 12), (64, 64)]
    print(f"batched d={d} rule={rule} max_iter={max_iter}", flush=True)
    probs = _problems(specs, d, seed=d * 10 + rule)
    kw = dict(max_iter=max_iter, tol=1e-4, stop_rule=rule)
    got, info = _run_batched(probs, **kw)
    assert info["rounds"] >= 1
    for j, (P, C0, deg0) in enumerate(probs):
        single = _single(P, C0, deg0, **kw)
        rC, rdeg, rlab, rf, rp, _ = oracle.lloyd(P, C0, deg0, **kw)
        gap = _oracle_min_gap(P, C0, deg0, steps=min(rp, 60))
        strict = gap >= LABEL_TIE_REL
        assert strict == (j not in NEAR_TIE_PROBLEMS[(d, rule, max_iter)]), f"near-tie status of {j}"
        if not strict:
            _lockstep_batched(P, C0, deg0, steps=min(rp, 20))
            try:
                _compare(P, C0, deg0, got[j], (rC, rdeg, rlab, rf, rp), True)
                print(f"  problem {j}: near tie on the oracle path; whole run still equal",
                      flush=True)
                continue
            except AssertionError:
                print(f"  problem {j}: near tie on the oracle path; trajectories diverged",
                      flush=True)
        _compare(P, C0, deg0, got[j], (rC, rdeg, rlab, rf, rp), strict)
        if strict:
            # and against the single-problem GPU path, integer results exactly
            assert np.array_equal(got[j][2], single[2])
            assert got[j][4] == single[4]
            assert np.array_equal(got[j][1], single[1])


def test_batched_empty_cluster_and_tiny_problems():
    P1 = np.array([[0.0], [0.1], [0.2], [5.0], [5.1]], np.float32)
    C1 = np.array([[0.0], [5.0], [100.0]], np.float32)
    P2 = np.array([[3.0]], np.float32)
    C2 = np.array([[1.0]], np.float32)
    probs = [(P1, C1, np.zeros(3, np.uint8)), (P2, C2, np.zeros(1, np.uint8))]
    got, _ = _run_batched(probs, max_iter=20)
    gC, gdeg, glab, gf, gp = got[0]
    assert gdeg.tolist() == [0, 0, 1]
    assert np.isnan(gC[2]).all()
    assert set(glab.tolist()) == {0, 1}
    gC, gdeg, glab, gf, gp = got[1]
    assert gC[0, 0] == 3.0 and gf == 0.0 and glab.tolist() == [0]


def test_batched_degenerate_input_flags_are_kept():
    probs = _problems([(3_000, 8), (2_000, 4)], 16, seed=5)
    probs[0][2][[1, 6]] = 1
    probs[0][1][[1, 6]] = np.nan
    got, _ = _run_batched(probs, max_iter=50, stop_rule=1)
    gdeg = got[0][1]
    assert gdeg[1] == 1 and gdeg[6] == 1
    assert not np.isin(got[0][2], [1, 6]).any()
    for j, (P, C0, deg0) in enumerate(probs):
        single = _single(P, C0, deg0, max_iter=50, stop_rule=1)
        assert_sse(got[j][3], single[3])


def test_batched_wide_workload_sampled():
    # a quarter of the batched workload's solves (64 of 256) on its full-size
    # data (10,000,000 x 68), set up as the benchmark does; 6 solves are
    # checked against the single-problem path and against the oracle's
    # assignment at their returned centroids
    from paper_2204_07485_amd import bigmeans
    X = torch.from_numpy(synth.make_wide()).cuda()
    solves = synth.wide_solves()[:64]
    P, s, k, C, deg = bigmeans.prepare_batch(X, solves)
    C0 = C.clone()
    kw = dict(max_iter=300, tol=1e-4, stop_rule=bigmeans.BM_STOP_REL_OBJ)
    dg, lab, f, passes, info = bigmeans.kmeans_lloyd_batched(P, s, k, C, deg, **kw)
    print(f"rounds {info['rounds']} tile {info['tile_rows']}", flush=True)
    assert info["rounds"] == int(passes.max())
    r0 = np.concatenate([[0], np.cumsum(s)])
    c0 = np.concatenate([[0], np.cumsum(k)])
    for j in (0, 1, 2, 3, 5, 6):
        Pj = P[r0[j]:r0[j + 1]]
        Cj = C0[c0[j]:c0[j + 1]].clone()
        sdg, slab, sf, sp = bigmeans.kmeans_lloyd(Pj, Cj, deg[c0[j]:c0[j + 1]], **kw)
        assert_sse(f[j], sf)
        assert passes[j] == sp
        Pn = Pj.cpu().numpy()
        Cb = C[c0[j]:c0[j + 1]].cpu().numpy()
        dgj = dg[c0[j]:c0[j + 1]]
        Cs = Cj.cpu().numpy()
        assert_centroids(Cb, Cs, sdg)
        # the same labels as the single-problem path, up to near ties
        assert_labels(lab[r0[j]:r0[j + 1]].cpu().numpy(), slab.cpu().numpy(), Pn, Cs, sdg)
        # at any size: the objective and labels are those the oracle gives
        # the batched path's own centroids
        with oracle.threaded():
            olab, _, of = oracle.assign(Pn, Cb, dgj)
        assert_sse(f[j], of)
        assert_labels(lab[r0[j]:r0[j + 1]].cpu().numpy(), olab, Pn, Cb, dgj)


@pytest.mark.parametrize("d,k", [(4, 6), (24, 16)])
def test_batched_nonfinite_rows_stay_in_their_problem(d, k):
    # a NaN row and an infinite row in problem 0 go to its first active slot
    # (as in the persistent solver) and touch nothing outside problem 0: the
    # other problems come out bit for bit as in a batch without those rows
    # (k d = 24 runs the VALU kernel, k d = 384 the matrix-core one)
    clean = _problems([(3_000, k), (2_500, k), (1_800, k)], d, seed=41)
    bad = [(p.copy(), c.copy(), g.copy()) for p, c, g in clean]
    bad[0][0][7, 1] = np.nan
    bad[0][0][11, 0] = np.inf
    print(f"batched nonfinite rows d={d} k={k}", flush=True)
    got, _ = _run_batched(bad, max_iter=30, stop_rule=1)
    ref, _ = _run_batched(clean, max_iter=30, stop_rule=1)
    for j in (1, 2):
        gC, gdeg, glab, gf, gp = got[j]
        rC, rdeg, rlab, rf, rp = ref[j]
        np.testing.assert_array_equal(gC, rC)
        np.testing.assert_array_equal(gdeg, rdeg)
        np.testing.assert_array_equal(glab, rlab)
        assert gf == rf and gp == rp
    glab0 = got[0][2]
    first_active = int(np.flatnonzero(bad[0][2] == 0)[0])
    assert glab0[7] == first_active and glab0[11] == first_active
