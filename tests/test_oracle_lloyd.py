"""Pins for the oracle's assignment and Lloyd local search (Eq. 1; Sec. 2: the
assignment step takes the nearest centre, the update step the mean of each
cell; Sec. 3.3: an emptied cluster is degenerate; Sec. 5: stop rule)."""
import numpy as np
import pytest

import oracle


def _np_assign(P, C, deg):
    D = ((P[:, None, :] - C[None, :, :]) ** 2).sum(axis=2)
    D[:, np.asarray(deg, bool)] = np.inf
    lab = D.argmin(axis=1)          # first minimum: ties go to the lowest index
    return lab, D[np.arange(len(P)), lab]


def test_assign_hand_example():
    P = np.array([[0.0], [1.0], [2.5], [10.0], [5.5]])
    C = np.array([[0.0], [3.0], [np.nan], [10.0]])
    lab, mind, f = oracle.assign(P, C, [0, 0, 1, 0])
    assert list(lab) == [0, 0, 1, 3, 1]
    assert np.allclose(mind, [0, 1, 0.25, 0, 6.25])
    assert f == pytest.approx(7.5)


def test_assign_exact_tie_goes_to_lowest_index():
    P = np.array([[1.0, 0.0]])
    C = np.array([[3.0, 0.0], [-1.0, 0.0], [1.0, 2.0]])
    assert oracle.assign(P, C, [0, 0, 0])[0][0] == 0
    assert oracle.assign(P, C[::-1].copy(), [0, 0, 0])[0][0] == 0


def test_assign_matches_brute_force():
    rng = np.random.default_rng(1)
    P = rng.normal(size=(500, 7))
    C = rng.normal(size=(9, 7))
    deg = np.zeros(9, np.uint8)
    deg[[2, 5]] = 1
    lab, mind, f = oracle.assign(P, C, deg)
    lab2, mind2 = _np_assign(P, C, deg)
    assert np.array_equal(lab, lab2)
    assert np.allclose(mind, mind2, rtol=1e-13)
    assert f == pytest.approx(mind2.sum(), rel=1e-13)


def test_dist2_definition():
    x = np.array([1.0, -2.0, 3.5])
    c = np.array([0.5, 0.5, 0.5])
    assert oracle.dist2(x, c) == 0.25 + 6.25 + 9.0


def _mixture(n=600, d=3, k=4, seed=0, spread=6.0):
    rng = np.random.default_rng(seed)
    mu = rng.uniform(-spread, spread, size=(k, d))
    return (mu[rng.integers(0, k, n)] + rng.normal(size=(n, d))), mu


def test_one_update_gives_cluster_means():
    P, mu = _mixture()
    C0 = mu + 0.5
    C1, deg, lab, f, passes, _ = oracle.lloyd(P, C0, [0] * 4, max_iter=1)
    lab0, _ = _np_assign(P, C0, [0] * 4)
    for j in range(4):
        assert np.allclose(C1[j], P[lab0 == j].mean(axis=0), rtol=0, atol=1e-12)
    assert passes == 2
    # the returned objective is that of the returned centroids
    assert f == pytest.approx(_np_assign(P, C1, deg)[1].sum(), rel=1e-12)


def test_sse_non_increasing():
    P, mu = _mixture(seed=3)
    C0 = P[:4].copy()
    prev = np.inf
    for it in range(1, 12):
        _, _, _, f, _, _ = oracle.lloyd(P, C0, [0] * 4, max_iter=it, tol=0.0)
        assert f <= prev * (1 + 1e-12)
        prev = f


def test_fixed_point_is_voronoi_and_means():
    P, mu = _mixture(seed=4)
    C, deg, lab, f, passes, _ = oracle.lloyd(P, P[:4], [0] * 4, max_iter=500, tol=1e-12)
    assert passes < 501
    lab2, mind = _np_assign(P, C, deg)
    assert np.array_equal(lab, lab2)
    for j in range(4):
        assert np.allclose(C[j], P[lab == j].mean(axis=0), atol=1e-12)
    # Koenig-Huygens at cluster means: f = sum |x|^2 - sum_j cnt_j |c_j|^2
    cnt = np.bincount(lab, minlength=4)
    kh = (P ** 2).sum() - (cnt * (C ** 2).sum(axis=1)).sum()
    assert f == pytest.approx(kh, rel=1e-10)


def test_single_cluster_is_the_mean():
    rng = np.random.default_rng(5)
    P = rng.normal(3.0, 2.0, size=(300, 5))
    C, deg, lab, f, passes, _ = oracle.lloyd(P, P[:1], [0], max_iter=10)
    assert np.allclose(C[0], P.mean(axis=0), atol=1e-12)
    assert f == pytest.approx(((P - P.mean(axis=0)) ** 2).sum(), rel=1e-12)


def test_emptied_cluster_becomes_degenerate():
    P = np.array([[0.0], [0.1], [0.2], [5.0], [5.1]])
    C0 = np.array([[0.0], [5.0], [100.0]])
    C, deg, lab, f, passes, _ = oracle.lloyd(P, C0, [0, 0, 0], max_iter=20)
    assert list(deg) == [0, 0, 1]
    assert np.isnan(C[2]).all()
    assert set(lab.tolist()) == {0, 1}


def test_relative_objective_rule_stops_early():
    P, mu = _mixture(n=2000, seed=6)
    C0 = P[:4].copy()
    _, _, _, f_rel, it_rel, _ = oracle.lloyd(P, C0, [0] * 4, max_iter=300, tol=1e-4,
                                             stop_rule=oracle.ORC_STOP_REL_OBJ)
    _, _, _, f_full, it_full, _ = oracle.lloyd(P, C0, [0] * 4, max_iter=300, tol=0.0)
    assert it_rel <= it_full
    assert f_rel >= f_full * (1 - 1e-12)
    # The rule returns after pass m the centroids of m-1 updates, because the
    # objective fell by at most tol (relative) from m-2 to m-1 updates, and
    # not earlier.  Runs capped at j updates give the objective after j.
    m = it_rel
    f_at = [oracle.lloyd(P, C0, [0] * 4, max_iter=j, tol=0.0)[3] for j in range(1, m)]
    f_at = [oracle.assign(P, C0, [0] * 4)[2]] + f_at          # f_at[j] = after j updates
    assert f_at[m - 1] == f_rel
    assert (f_at[m - 2] - f_at[m - 1]) <= 1e-4 * f_at[m - 2]
    for j in range(1, m - 1):
        assert (f_at[j - 1] - f_at[j]) > 1e-4 * f_at[j - 1]


def test_shift_rule_iterations_capped():
    P, mu = _mixture(n=3000, seed=7)
    _, _, _, _, passes, st = oracle.lloyd(P, P[:4], [0] * 4, max_iter=3, tol=0.0)
    assert passes == 4
    assert st["lloyd_iters"] == 4
    assert st["n_d"] == 4 * 3000 * 4
