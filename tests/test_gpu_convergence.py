"""Self-convergence of the coupled solver on the GPU at the paper's grids (2-D, rhombic seed,
0.04 / 0.025 / 0.02 mm against 0.0125 mm), over 2 hours of physical time instead of 16 (the full
study is `python -m paper_2206_02145_amd.convergence`): the relative l2 error of phi along the
centre line falls at second order."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_second_order_self_convergence():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2206_02145_amd import convergence as C
    res = [C.run(dr, "fp64", hours=2.0, log=None) for dr in C.LEVELS_MM]
    o = C.orders(res)
    print("[convergence] 2 h:", [(d, f"{e:.3e}") for d, e in o["errors"]], f"order {o['order']:.2f}", flush=True)
    errs = [e for _, e in o["errors"]]
    assert errs[0] > errs[1] > errs[2] > 0
    assert 1.6 < o["order"] < 2.5  # 1.77 over 2 h; the 16-hour study gives 2.10
