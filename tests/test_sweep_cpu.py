"""Host logic of the sweep driver (no GPU)."""
from paper_1402_2773_amd import sweep


def test_range_parsing():
    assert sweep._range("2:5:0.5") == [2.0, 2.5, 3.0, 3.5, 4.0, 4.5, 5.0]
    assert sweep._range("-1.2:-0.2:0.1")[0] == -1.2 and len(sweep._range("-1.2:-0.2:0.1")) == 11
    assert sweep._range("3.5") == [3.5]
    assert sweep._range("1,2.5") == [1.0, 2.5]


def test_heuristic_lambda_schedule():
    """Sec. IV-A: lambda 0.99 below 3.5 dB, 0.97 at 3.5, 0.94 at 4.0, 0.90 at
    4.25 and 4.5 dB (kept above)."""
    assert [sweep.heuristic_params(e)["lam"] for e in (2.0, 3.0, 3.5, 4.0, 4.25, 4.5, 5.0)] == \
        [0.99, 0.99, 0.97, 0.94, 0.90, 0.90, 0.90]
    assert sweep.heuristic_params(3.0)["smooth_window"] == 64


def test_wilson_interval():
    lo, hi = sweep.wilson(0, 100)
    assert lo == 0.0 and 0.03 < hi < 0.04       # rule of three, roughly
    lo, hi = sweep.wilson(50, 100)
    assert abs((lo + hi) / 2 - 0.5) < 1e-12 and 0.40 < lo < 0.41
