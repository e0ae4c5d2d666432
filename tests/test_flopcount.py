"""The FP64 operation counts behind the push's roofline fraction: measured
on the oracle compiled with a counting scalar type (oracle/flopcount.cpp),
and the constants bench.py uses are those counts."""
import pytest

import bench
from oracle import flopcount


@pytest.fixture(scope="module")
def counts():
    return flopcount.counts(1024)


def test_bench_constants_are_the_measured_counts(counts):
    assert bench.FLOP_RK4_GRID == round(counts["rk4_step"]["flop"])
    assert bench.FLOP_RK4_NOGRID == round(counts["rk4_step_no_fields"]["flop"])
    assert bench.FLOP_ENERGY == round(counts["energy"]["flop"])
    assert bench.FLOP_WEIGHTS == round(counts["deposit_weights"]["flop"])
    assert bench.FLOP_IMR_ITER == round(counts["imr_iteration"]["flop"])
    assert bench.FLOP_NEWTON_ITER == round(counts["newton_iteration"]["flop"])
    assert bench.FLOP_GATHER == round(counts["gather"]["flop"])
    # the discrete-gradient iteration's count varies with the small-step
    # branch of App. D (analytic derivative below |dx| = 1e-10)
    assert abs(bench.FLOP_HAM_ITER - counts["ham_iteration"]["flop"]) < 0.01 * bench.FLOP_HAM_ITER


def test_counts_are_consistent_with_their_parts(counts):
    """An RK4 step evaluates the gather and the equations of motion four
    times; a Picard iteration once (plus its midpoint, update and test);
    Newton's method seven times per iteration."""
    eval_ = counts["gather"]["flop"] + counts["equations_of_motion"]["flop"]
    assert 4 * eval_ < counts["rk4_step"]["flop"] < 4 * eval_ + 500
    assert eval_ < counts["imr_iteration"]["flop"] < eval_ + 150
    assert 7 * eval_ < counts["newton_iteration"]["flop"] < 7 * eval_ + 1200
    # the equations of motion evaluate the metric and its derivatives
    assert counts["equations_of_motion"]["flop"] > (counts["metric"]["flop"] +
                                                    counts["metric_derivatives"]["flop"])
    # the deposit weights sample sqrt(gamma) on 4 x 16 trapezoid points, each
    # with one square root and one sin / cos pair
    assert counts["deposit_weights"]["sqrt"] == 64
    assert counts["deposit_weights"]["transcendental"] == 128
