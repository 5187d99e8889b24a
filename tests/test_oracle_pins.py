"""The FP64 oracle against closed forms, exact rationals, hand-worked
fixtures and invariants (no GPU)."""
import pytest

import oracle_pins


@pytest.mark.parametrize("pin", oracle_pins.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(oracle, pin):
    pin(oracle)


def test_thread_count_does_not_change_results(oracle):
    import numpy as np
    import workloads as W
    V, Q = W.single_polygon_fp64(m=50_000)
    t = oracle.num_threads()
    a = oracle.voronoi(V, Q)
    oracle.set_num_threads(1)
    try:
        b = oracle.voronoi(V, Q)
    finally:
        oracle.set_num_threads(t)
    assert np.array_equal(a, b)
