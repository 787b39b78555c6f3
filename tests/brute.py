"""Exact MSSC optima for tiny inputs, by definition (Eq. 1), independent of the
oracle: exhaustive search over labelings, and the 1-D dynamic programme over
contiguous clusters (in one dimension an optimal partition is contiguous in
sorted order)."""
import numpy as np


def brute_force_opt(P, k, chunk=1 << 16):
    """min over all k^n labelings of sum_j sum_{i in cluster j} |p_i - mean_j|^2."""
    P = np.asarray(P, dtype=np.float64)
    n, d = P.shape
    total = k ** n
    sq = float((P ** 2).sum())
    best = np.inf
    pows = k ** np.arange(n)
    for lo in range(0, total, chunk):
        codes = np.arange(lo, min(total, lo + chunk))
        lab = (codes[:, None] // pows[None, :]) % k            # (L, n)
        onehot = (lab[:, :, None] == np.arange(k)[None, None, :]).astype(np.float64)
        cnt = onehot.sum(axis=1)                               # (L, k)
        sums = np.einsum("lnk,nd->lkd", onehot, P)             # (L, k, d)
        with np.errstate(invalid="ignore", divide="ignore"):
            between = np.where(cnt > 0, (sums ** 2).sum(axis=2) / cnt, 0.0).sum(axis=1)
        best = min(best, float((sq - between).min()))
    return best


def dp_opt_1d(x, k):
    """Optimal k-clustering cost of 1-D points (O(k n^2) DP over sorted order)."""
    x = np.sort(np.asarray(x, dtype=np.float64))
    n = len(x)
    c1 = np.concatenate([[0.0], np.cumsum(x)])
    c2 = np.concatenate([[0.0], np.cumsum(x * x)])

    def cost(a, b):  # points a..b-1
        m = b - a
        s = c1[b] - c1[a]
        return (c2[b] - c2[a]) - s * s / m

    dp = np.full((k + 1, n + 1), np.inf)
    dp[0, 0] = 0.0
    for j in range(1, k + 1):
        for b in range(1, n + 1):
            best = np.inf
            for a in range(j - 1, b):
                v = dp[j - 1, a] + cost(a, b)
                if v < best:
                    best = v
            dp[j, b] = best
    return float(dp[1:, n].min())
