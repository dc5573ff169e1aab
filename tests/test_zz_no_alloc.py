"""lbcg_measure_noalloc, the diagnostics with their scratch in the library's static device array,
against lbcg_measure on the same states, through the C ABI: two calls in a row, the second on a
smaller grid with fewer directions (the array then still holds the first call's values)."""
import numpy as np
import pytest

from paper_2206_02145_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2206_02145_amd import lbcg
    lbcg.lib()
    return lbcg


def same(a, b):
    La, ma = a
    Lb, mb = b
    assert La.shape == Lb.shape and np.array_equal(La, Lb), (La, Lb)
    for k in mb:
        assert ma[k] == mb[k] or (np.isnan(ma[k]) and np.isnan(mb[k])), (k, ma[k], mb[k])


def test_measure_noalloc_equals_measure(lb):
    big = W.scaled(W.config3(), 96, 64, 64, seed_R=8.0)  # 3-D flow, 1024 reduction blocks
    small = W.sweep_instance(48, 0.25, 6.0, 0.02)          # 2-D flow, 9 reduction blocks
    cases = ((big, "fp32", W.directions(16)), (small, "fp64", W.directions(6, offset=0.3)))
    for p, prec, dirs in cases:
        s = lb.Solver(p, prec)
        s.step(30)
        first = s.measure_noalloc(dirs)
        ref = s.measure(dirs)
        same(first, ref)
        assert ref[1]["Vs"] > 0 and ref[0].min() > 0
        s.step(7)
        ref = s.measure(dirs)
        same(s.measure_noalloc(dirs), ref)
        # no directions: sums only
        L, m = s.measure_noalloc(None)
        assert L.shape == (0,)
        assert m == s.measure(None)[1]
        s.close()


def test_measure_noalloc_rejects_too_many_directions(lb):
    s = lb.Solver(W.sweep_instance(48, 0.25, 6.0, 0.02), "fp32")
    dirs = W.directions(257)
    with pytest.raises(lb.LbcgError) as e:
        s.measure_noalloc(dirs)
    assert e.value.status == "EINVAL"
    s.close()
