"""Failure handling on the GPU, forced from the host: a grid-barrier wait bound
of one poll makes the solver abort cleanly with BM_EDEVICE (every workgroup
exits; nothing hangs), and the next call runs normally.  Requests beyond the
library's limits return BM_ENOTSUP."""
import numpy as np
import pytest
import torch

import oracle
from paper_2204_07485_amd import synth

pytestmark = pytest.mark.gpu


def test_barrier_wait_bound_aborts_cleanly_then_recovers():
    from paper_2204_07485_amd import bigmeans
    X, _ = synth.gaussian_mixture(20_000, 4, 5, seed=3, sigma=1.0)
    Xd = torch.from_numpy(X).cuda()
    print("forced barrier abort (spin_limit=1, grid=8)", flush=True)
    with pytest.raises(bigmeans.BigmeansError) as exc:
        bigmeans.bigmeans_fit(Xd, 5, 4000, 3, 1, grid=8, spin_limit=1)
    assert exc.value.code == bigmeans.BM_EDEVICE
    assert "barrier" in str(exc.value)
    got = bigmeans.bigmeans_fit(Xd, 5, 4000, 3, 1, grid=8)
    ref = oracle.bigmeans_fit(X, 5, 4000, 3, 1)
    assert abs(got["sse"] - ref["sse"]) <= 1e-6 * ref["sse"]


def test_dimension_beyond_limit_is_not_supported():
    from paper_2204_07485_amd import bigmeans
    X = torch.zeros((100, 300), dtype=torch.float32, device="cuda")
    with pytest.raises(bigmeans.BigmeansError) as exc:
        bigmeans.bigmeans_fit(X, 2, 50, 1, 1)
    assert exc.value.code == bigmeans.BM_ENOTSUP
