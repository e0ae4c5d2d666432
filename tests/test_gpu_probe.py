"""The measured ceilings (grpic_probe_peaks) through the C ABI: positive,
and not above MI355X's published FP64 vector and HBM peaks."""
import pytest

import paper_2602_07452_amd as G

pytestmark = pytest.mark.gpu


def test_probe_peaks_are_plausible():
    cfg = G.config_default(a=0.9, max_particles=16)
    with G.Context(cfg) as ctx:
        p = ctx.probe_peaks()
    print(p)
    assert 5.0 < p["fp64_fma_tflops"] <= 78.6 * 1.02
    assert 0.5 < p["copy_tbs"] <= 8.0 * 1.02
