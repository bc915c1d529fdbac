"""GPU: the sweep driver's batched grid equals one-at-a-time decoding, and
the successive-approximation search stays in its domain and does not get
worse than its start."""
import sys

import pytest

import paper_1402_2773_amd as ng
from paper_1402_2773_amd import sweep
from synth import codes

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def c96():
    import torch

    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    c = codes.named_code("C96")
    return c, ng.Code.from_ldpc(c)


def test_grid_equals_single_points(c96):
    c, dc = c96
    grid = [{**sweep.plain_params(3.0), "theta": th, "t_max": 60} for th in (-0.9, -0.6, -0.3)]
    say("grid")
    pts = sweep.run_grid(c, dc, 3.0, grid, 4096, seed=5)
    for pr, pt in zip(grid, pts):
        one = sweep.run_point(c, dc, 3.0, pr, 4096, seed=5)
        assert (pt.ber, pt.fer, pt.avg_iterations) == (one.ber, one.fer, one.avg_iterations)


def test_successive_approximation(c96):
    c, dc = c96
    start = {**sweep.plain_params(3.0), "t_max": 60, "theta": -1.3}
    ranges = {"theta": (-1.5, -0.1), "eta": (0.3, 1.3)}
    say("search")
    best = sweep.successive_approximation(c, dc, 3.0, start, ranges, 4096, seed=6, points=5, steps=2)
    assert -1.5 <= best["theta"] <= -0.1 and 0.3 <= best["eta"] <= 1.3
    b = sweep.run_point(c, dc, 3.0, best, 4096, seed=6)
    s = sweep.run_point(c, dc, 3.0, start, 4096, seed=6)
    assert (b.ber, b.avg_iterations) <= (s.ber, s.avg_iterations)


def test_chunked_point_resumes_bit_identically(c96, tmp_path):
    """A Monte Carlo point stopped after two chunks and resumed from its
    checkpoint gives the same totals as an uninterrupted run."""
    c, dc = c96
    pr = {**sweep.heuristic_params(3.0), "t_max": 80}
    a = sweep.run_point_chunked(c, dc, 3.0, pr, 5000, 9, 1024, str(tmp_path / "a.json"))
    assert sweep.run_point_chunked(c, dc, 3.0, pr, 5000, 9, 1024, str(tmp_path / "b.json"),
                                   max_chunks=2) is None
    b = sweep.run_point_chunked(c, dc, 3.0, pr, 5000, 9, 1024, str(tmp_path / "b.json"))
    assert a == b
    assert sum(a["iteration_histogram"]) == 5000
