"""Parity at full size and full length: the HIP path against the oracle's state of the 3-D
configurations after their own step counts (128^3 without flow, 5000 steps; 192x128x128 with flow,
20000 steps), on the sampled outputs that tests/golden/make_fulllength.py stored (two planes through
the seed centre and 8192 random nodes). The bar is the binary32 one: max |error| over the samples
divided by max |value| over the whole grid, 1e-4 per field."""
import json
import os

import numpy as np
import pytest

from paper_2206_02145_amd import workloads as W

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
CASES = {"c2": W.config2, "c3": W.config3}


@pytest.fixture(scope="module")
def lb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2206_02145_amd import lbcg
    lbcg.lib()
    return lbcg


def load(case):
    path = os.path.join(GOLDEN, f"fulllength_{case}.npz")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated (python tests/golden/make_fulllength.py {case})")
    z = np.load(path, allow_pickle=False)
    meta = json.loads(str(z["meta"]))
    p = CASES[case]()
    for k, v in meta["params"].items():  # the stored run is of exactly this configuration
        assert np.allclose(np.asarray(p[k], dtype=float), np.asarray(v, dtype=float)), k
    return z, meta, p


def run(lb, p, prec, steps):
    s = lb.Solver(p, prec)
    done = 0
    while done < steps:
        n = min(5000, steps - done)
        s.step(n)
        done += n
        print(f"[fulllength] {prec} {done}/{steps}", flush=True)
    return s


@pytest.mark.parametrize("case", ["c2", "c3"])
def test_full_length_fp32(lb, case):
    z, meta, p = load(case)
    steps = meta["steps"]
    print(f"[fulllength] {case} fp32 {p['nx']}x{p['ny']}x{p['nz']} flow={p['flow']} steps={steps}", flush=True)
    s = run(lb, p, "fp32", steps)
    nz_, ny_, nx_ = z["nodes"][:, 0], z["nodes"][:, 1], z["nodes"][:, 2]
    names = ["phi", "U"] + (["rho", "ux", "uy", "uz"] if p["flow"] else [])
    errs = {}
    for k in names:
        got = s.read(k)[nz_, ny_, nx_]
        errs[k] = float(np.abs(got - z[k]).max() / z["absmax_" + k])
    if p["flow"]:  # the velocity as a vector, over the largest component
        um = max(float(z["absmax_" + c]) for c in ("ux", "uy", "uz"))
        errs["u"] = max(float(np.abs(s.read(c)[nz_, ny_, nx_] - z[c]).max()) for c in ("ux", "uy", "uz")) / um
        for c in ("ux", "uy", "uz"):
            errs.pop(c)
    L, mass = s.measure(W.directions(16))
    dL = float(np.abs(L - z["L16"]).max())
    dM = abs(mass["Mprime"] - float(z["mass_Mprime"])) / abs(float(z["mass_Mprime"]))
    print(f"[fulllength] {case} fp32 errors: " + ", ".join(f"{k}={v:.2e}" for k, v in errs.items()) +
          f"; max |dL| {dL:.2e} cells; M' rel diff {dM:.2e}", flush=True)
    for k, v in errs.items():
        assert v <= 1e-4, (case, k, v)
    assert dL <= 0.05
    assert dM <= (1e-6 if not p["flow"] else 1e-4)
    s.close()
