import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test")


def check_extremes(r, so, E0, K, xhat_o=None, index_o=None):
    """The extremes of a GPU run (dict of tkdv_stats fields) against the oracle's
    statistics `so` of the same accepted samples.  Counts agree up to grid
    values within FP32 rounding of 4 sigma; the peak value to FP32 accuracy;
    the peak's index is the oracle's, or (a near tie) a sample whose oracle
    maximum is within that accuracy of the oracle's peak (needs the oracle's
    rows x^ and their proposal indices)."""
    import math

    import numpy as np

    import oracle

    tol = 1e-5 * math.sqrt(2 * K * E0 / math.pi)
    assert abs(int(r["n_exceed_4sigma"]) - int(so.n_exceed4)) <= 2 + so.n_exceed4 // 100000
    assert abs(int(r["n_samples_4sigma"]) - int(so.n_max4)) <= 1 + so.n_max4 // 100000
    if so.n_accepted == 0:
        assert r["peak_u"] == -math.inf and r["peak_index"] == 2**64 - 1
        return
    assert abs(r["peak_u"] - so.peak_u) < tol
    if int(r["peak_index"]) != int(so.peak_index):
        assert xhat_o is not None, "peak index differs and no oracle rows to check the tie"
        rows = np.nonzero(np.asarray(index_o, dtype=np.uint64) == np.uint64(r["peak_index"]))[0]
        assert rows.size == 1
        um = oracle.extremes(np.asarray(xhat_o)[rows], E0, 4 * K, 1, 0.0)["umax"][0]
        assert abs(um - so.peak_u) < tol
