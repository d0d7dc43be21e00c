"""Full-size parity: the FP64 HIP fractional step on the 2^10 x 2^10 O-grid
(20 interleaved cores, chi = 64) against the FD oracle, step by step."""
import pytest

pytestmark = pytest.mark.gpu


def test_c3_fp64_steps_match_oracle():
    from tests.c3_case import run
    for s, (errs, info) in enumerate(run(2)):
        # chi = 64 represents these early fields almost exactly: the TT step is the
        # FD step up to the solver tolerances (1e-9) and FP64 rounding
        assert errs["u"] < 1e-6 and errs["v"] < 1e-6 and errs["p"] < 1e-5, (s, errs)
        assert info.poisson.residual < 1e-7, (s, info.poisson.residual)
