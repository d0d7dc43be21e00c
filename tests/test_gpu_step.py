"""GPU parity of one fractional step (2^5 x 2^5 O-grid) against the FD oracle."""
import pytest

pytestmark = pytest.mark.gpu


def test_step_c1_full_rank_matches_oracle():
    from tests.smoke_check import run_c1
    res, info = run_c1(cap=32)
    for k in ("u", "v", "p"):
        assert res[k] < 1e-7, res
    # largest projected (local-system) residual of the last sweep, FP64
    assert info.helm_u.residual < 1e-8 and info.helm_v.residual < 1e-8


def test_step_c1_bf16_contractions_within_budget():
    """Mixed precision (FP32 MFMA derivative applies and Poisson products, BF16 MFMA
    Hadamard and Helmholtz products, FP32 accumulation, FP64 truncation and residual
    restarts): the step stays within the 3e-3 relative L2 budget of the FP64 oracle."""
    from tests.smoke_check import run_c1
    res, _ = run_c1(cap=32, dtype="f32", product_dtype="bf16", helm_dtype="bf16", pois_dtype="f32")
    for k in ("u", "v", "p"):
        assert res[k] < 3e-3, res
