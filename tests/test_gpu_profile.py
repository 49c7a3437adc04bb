"""Phase timing through the C-ABI: svlcov_profile times every phase of an
update, svlcov_profile_phases only the phases of its mask (the benchmark's
timed steps bracket the single-kernel phases alone), mask 0 none; a mask bit
beyond the last phase is refused.  The numbers are not checked, only which
phases were timed and that the update's result does not depend on it."""
import numpy as np
import pytest

from synth import synthetic_factors
from synth.sparse import CSR

pytestmark = pytest.mark.gpu


def _update(rng, s, width):
    E = np.where(rng.random((s, width)) < 0.05, rng.uniform(-1.0, 1.0, (s, width)), 0.0)
    return CSR.from_dense(E)


def test_phase_mask_times_only_its_phases():
    import paper_2401_09703_amd as L
    rng = np.random.default_rng(77)
    m, n, k = 600, 400, 32
    U, s, V = synthetic_factors(m, n, k, rng)
    ups = [("rows", _update(rng, 120, n)), ("rows", _update(rng, 80, n)),
           ("rows", _update(rng, 100, n))]
    plain = L.TruncatedSVD(U, s, V, precision="fp32")
    timed = L.TruncatedSVD(U, s, V, precision="fp32")
    try:
        timed.profile(True, phases=["cholesky"])
        plain.apply(ups[0])
        timed.apply(ups[0])
        ph = timed.phase_times()
        assert ph["cholesky"][1] == 1, ph
        assert all(c == 0 for name, (_, c) in ph.items() if name != "cholesky"), ph
        timed.profile(True)
        plain.apply(ups[1])
        timed.apply(ups[1])
        ph = timed.phase_times()
        assert ph["cholesky"][1] == 1 and ph["spmm_w"][1] == 1, ph
        assert sum(1 for _, c in ph.values() if c) >= 5, ph
        timed.profile(False)
        plain.apply(ups[2])
        timed.apply(ups[2])
        ph = timed.phase_times()
        assert all(c == 0 for _, c in ph.values()), ph
        with pytest.raises(Exception):
            L._check(L._lib.svlcov_profile_phases(timed._h, 1 << L.NUM_PHASES),
                     "svlcov_profile_phases")
        for x, y in zip(plain.factors(), timed.factors()):
            assert np.array_equal(x, y)
    finally:
        plain.close()
        timed.close()
