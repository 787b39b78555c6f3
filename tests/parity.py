"""Comparison helpers for GPU-vs-oracle parity.

Bar (FP32 path vs the FP64 oracle):
  - integer work (sample indices, K-means++ picks, counts): bit-exact;
  - labels: equal, except at points whose two smallest oracle distances
    d1 <= d2 satisfy d2 - d1 < 1e-5 * d2 (near ties);
  - objectives (SSE): within 1e-6 relative;
  - centroids: |c_gpu - c_oracle|_2 <= 1e-6 * max(|c_oracle|_2, RMS cluster radius).
"""
import numpy as np

LABEL_TIE_REL = 1e-5
SSE_REL = 1e-6
CENTROID_REL = 1e-6


def top2_gap(P, C, deg=None, chunk=1 << 16):
    """Relative gap (d2 - d1) / d2 of the two nearest active centroids (FP64)."""
    P = np.asarray(P, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)
    act = np.ones(len(C), bool) if deg is None else ~np.asarray(deg, bool)
    Ca = C[act]
    out = np.empty(len(P))
    for lo in range(0, len(P), chunk):
        x = P[lo:lo + chunk]
        D = ((x[:, None, :] - Ca[None, :, :]) ** 2).sum(axis=2)
        if D.shape[1] == 1:
            out[lo:lo + chunk] = np.inf
            continue
        part = np.partition(D, 1, axis=1)
        d1, d2 = part[:, 0], part[:, 1]
        with np.errstate(invalid="ignore", divide="ignore"):
            out[lo:lo + chunk] = np.where(d2 > 0, (d2 - d1) / d2, 0.0)
    return out


def near_tie_count(P, C, deg=None, chunk=1 << 15):
    """Number of rows whose two nearest active centroids are within the
    near-tie band, from FP64 distances by the norm expansion (fast; only used
    to bound how far cluster sizes may move between two correct runs)."""
    P = np.asarray(P)
    C = np.asarray(C, dtype=np.float64)
    act = np.ones(len(C), bool) if deg is None else ~np.asarray(deg, bool)
    Ca = C[act]
    if len(Ca) < 2:
        return 0
    cn = (Ca * Ca).sum(axis=1)
    total = 0
    for lo in range(0, len(P), chunk):
        x = np.asarray(P[lo:lo + chunk], dtype=np.float64)
        D = (x * x).sum(axis=1)[:, None] - 2.0 * (x @ Ca.T) + cn[None, :]
        part = np.partition(D, 1, axis=1)
        d1, d2 = part[:, 0], part[:, 1]
        total += int(((d2 - d1) < 2 * LABEL_TIE_REL * np.maximum(d2, 1e-300)).sum())
    return total


def assert_labels(got, ref, P, C, deg=None):
    """Labels equal except at near ties of the oracle's distances; returns
    the number of (allowed) mismatches."""
    got = np.asarray(got)
    ref = np.asarray(ref)
    mism = np.nonzero(got != ref)[0]
    if len(mism):
        gap = top2_gap(np.asarray(P)[mism], C, deg)
        bad = mism[gap >= LABEL_TIE_REL]
        assert len(bad) == 0, (f"{len(bad)} label mismatches away from ties, e.g. rows "
                               f"{bad[:5].tolist()} gap {gap[gap >= LABEL_TIE_REL][:5]}")
    return len(mism)


def assert_sse(got, ref, rel=SSE_REL):
    err = abs(got - ref) / max(abs(ref), 1e-300)
    assert err <= rel, f"SSE {got!r} vs oracle {ref!r}: rel err {err:.3e} > {rel:.0e}"


def assert_centroids(got, ref, deg, P=None, labels=None, rel=CENTROID_REL):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    act = ~np.asarray(deg, bool)
    assert np.isnan(got[~act]).all(), "degenerate centroids must be NaN"
    for j in np.nonzero(act)[0]:
        scale = np.linalg.norm(ref[j])
        if P is not None and labels is not None:
            pts = np.asarray(P, dtype=np.float64)[np.asarray(labels) == j]
            if len(pts):
                scale = max(scale, np.sqrt(((pts - ref[j]) ** 2).sum(axis=1).mean()))
        err = np.linalg.norm(got[j] - ref[j])
        assert err <= rel * max(scale, 1e-30), (f"centroid {j}: |diff| {err:.3e} > "
                                                f"{rel:.0e} * {scale:.3e}")
