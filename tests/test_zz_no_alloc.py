"""The allocation-free inner product (qtt_dot_noalloc, workspace in a file-scope
device array) against qtt_dot through the C ABI: two calls in a row, the second
on smaller trains, and the refusal of a problem whose workspace exceeds the array."""
import numpy as np
import pytest

from qtt_inputs import random_mps_cores

pytestmark = pytest.mark.gpu


def test_dot_noalloc_matches_dot():
    import torch
    from paper_2507_05222_amd import qtt as Q
    ctx = Q.Context(0)
    for L, chi, n in ((14, 64, 5), (8, 8, 2)):          # the second call is smaller
        xs = [Q.MPS.from_cores(random_mps_cores(L, chi, seed=500 + i), chi) for i in range(n)]
        ys = [Q.MPS.from_cores(random_mps_cores(L, chi, seed=600 + i), chi) for i in range(n)]
        ref = Q.dot(ctx, xs, ys)
        out = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
        Q.dot_noalloc(ctx, xs, ys, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        # the same kernels in the same order: identical values
        assert np.array_equal(got, ref), (got, ref)
    big = Q.MPS(8, 512)
    with pytest.raises(Q.QttError, match="ECAPACITY"):
        Q.dot_noalloc(ctx, [big], [big], torch.zeros(1, dtype=torch.float64, device="cuda"))
