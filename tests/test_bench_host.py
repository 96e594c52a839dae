"""Host logic of the benchmark: the timed segments of a case that leaves the
finite range (every segment restarts from the state after the warmup)."""
import pytest

import bench


@pytest.mark.parametrize("steps,warmup,horizon", [(20000, 100, 600), (2000, 20, 100), (37, 5, 600),
                                                  (500, 50, 100), (1, 0, 1)])
def test_segments_cover_the_steps_within_the_horizon(steps, warmup, horizon):
    sizes = bench.segment_sizes(steps, warmup, horizon)
    assert sum(sizes) == steps
    assert all(0 < n <= horizon - warmup for n in sizes)
    assert sizes == sorted(sizes, reverse=True) and len(set(sizes[:-1])) <= 1


def test_a_warmup_past_the_horizon_is_refused():
    with pytest.raises(SystemExit):
        bench.segment_sizes(1000, 600, 600)


def test_the_diverging_cases_have_a_horizon_above_the_default_warmup():
    assert bench.HORIZON["c2"] > 100 and bench.HORIZON["c3"] > 20
