"""Parity at full size and full length: the HIP path against the oracle's state of the 3-D
configurations (128^3 without flow after its 5000 steps; 192x128x128 with flow after 4000 and after
its 20000 steps), on the sampled outputs that tests/golden/make_fulllength.py stored (two planes
through the seed centre and 8192 random nodes).

Pointwise bar (binary32): max |error| over the samples divided by max |value| over the whole grid,
1e-4 per field. The 192x128x128 case is checked pointwise at 4000 steps only: with eps = 0.05
the interface stiffness of Eq. (a), a^2 + (a^2)'' = 1 - 72 eps cos 6 theta to first order, is
strongly negative near the axes (-2.6), and the interface shape amplifies any perturbation,
rounding included, by about 20x per 2000 steps
from step 4000 on, so two correct runs that round differently part pointwise (binary32 against
binary64 on the GPU: phi 1.4e-5 at 4000 steps, 1e-2 at 8000, 0.24 at 20000). After 20000 steps
the test checks what that amplification leaves alone: the solid volume, the crystal extents and
the binary64 diagnostics; the pointwise errors are printed. The binary16 flow-storage mode is
reported per field with a loose bound."""
import json
import os

import numpy as np
import pytest

from paper_2206_02145_amd import workloads as W

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
CASES = {"c2": W.config2, "c3": W.config3, "c3r": W.config3_reduced}


@pytest.fixture(scope="module")
def lb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2206_02145_amd import lbcg
    lbcg.lib()
    return lbcg


def load(case, step=None):
    name = f"fulllength_{case}.npz" if step is None else f"fulllength_{case}_{step}.npz"
    path = os.path.join(GOLDEN, name)
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


def errors(s, z, p):
    nz_, ny_, nx_ = z["nodes"][:, 0], z["nodes"][:, 1], z["nodes"][:, 2]
    errs = {}
    for k in ("phi", "U") + (("rho",) if p["flow"] else ()):
        errs[k] = float(np.abs(s.read(k)[nz_, ny_, nx_] - z[k]).max() / z["absmax_" + k])
    if p["flow"]:  # the velocity as a vector, over the largest component
        um = max(float(z["absmax_" + c]) for c in ("ux", "uy", "uz"))
        errs["u"] = max(float(np.abs(s.read(c)[nz_, ny_, nx_] - z[c]).max()) for c in ("ux", "uy", "uz")) / um
    return errs


def aggregates(s, z):
    L, mass = s.measure(W.directions(16))
    dL = float(np.abs(L - z["L16"]).max())
    dVs = abs(mass["Vs"] - float(z["mass_Vs"])) / abs(float(z["mass_Vs"]))
    dM = abs(mass["Mprime"] - float(z["mass_Mprime"])) / abs(float(z["mass_Mprime"]))
    return dL, dVs, dM


@pytest.mark.parametrize("case,step", [("c2", None), ("c3", 4000)])
def test_full_size_pointwise_fp32(lb, case, step):
    z, meta, p = load(case, step)
    steps = meta["steps"]
    print(f"[fulllength] {case} fp32 {p['nx']}x{p['ny']}x{p['nz']} flow={p['flow']} steps={steps}", flush=True)
    s = run(lb, p, "fp32", steps)
    errs = errors(s, z, p)
    dL, dVs, dM = aggregates(s, z)
    print(f"[fulllength] {case} fp32 @{steps}: " + ", ".join(f"{k}={v:.2e}" for k, v in errs.items()) +
          f"; max |dL| {dL:.2e} cells; Vs {dVs:.2e}; M' {dM:.2e}", flush=True)
    for k, v in errs.items():
        assert v <= 1e-4, (case, k, v)
    assert dL <= 0.05 and dVs <= 1e-5
    assert dM <= (1e-6 if not p["flow"] else 1e-5)
    s.close()
    if p["flow"]:
        s = run(lb, p, "fp16shift", steps)
        e16 = errors(s, z, p)
        print(f"[fulllength] {case} fp16shift @{steps}: " + ", ".join(f"{k}={v:.2e}" for k, v in e16.items()),
              flush=True)
        for k, v in e16.items():
            assert v <= 5e-2, (case, "fp16shift", k, v)
        s.close()


@pytest.mark.parametrize("case,step,prec", [("c2", None, "fp32"), ("c3", 4000, "fp32"), ("c3", 4000, "fp16shift")])
def test_full_size_in_the_timed_configuration(lb, case, step, prec):
    """The launch configuration bench.py times: the solver autotuned as the bench does (every tiling,
    two rounds of 20 real steps, so the run itself passes through all of them), then on the chosen
    tiling to the stored oracle state, compared pointwise as above."""
    z, meta, p = load(case, step)
    steps = meta["steps"]
    s = lb.Solver(p, prec)
    best, us = s.autotune(20)
    done = s.nstep
    print(f"[fulllength] {case} {prec} autotuned: {s.variants()[best]} ({us:.1f} us/step) after {done} steps",
          flush=True)
    assert 0 < done < steps
    s.step(steps - done)
    errs = errors(s, z, p)
    dL, dVs, dM = aggregates(s, z)
    print(f"[fulllength] {case} {prec} tuned @{steps}: " + ", ".join(f"{k}={v:.2e}" for k, v in errs.items()) +
          f"; max |dL| {dL:.2e} cells; Vs {dVs:.2e}; M' {dM:.2e}", flush=True)
    bar = 1e-4 if prec == "fp32" else 5e-2
    for k, v in errs.items():
        assert v <= bar, (case, prec, k, v)
    if prec == "fp32":
        assert dL <= 0.05 and dVs <= 1e-5
    s.close()


@pytest.mark.parametrize("prec", ["fp32", "fp16shift"])
def test_full_length_flow_aggregates(lb, prec):
    """After the configuration's 20000 steps, what the amplification leaves alone: the crystal
    extents, the solid volume and M' (measured: binary32 0.11 cells, 1.3e-4, 1.5e-4; binary16 flow
    storage 0.12 cells, 4.4e-5, 1.3e-5)."""
    z, meta, p = load("c3")
    steps = meta["steps"]
    s = run(lb, p, prec, steps)
    errs = errors(s, z, p)
    dL, dVs, dM = aggregates(s, z)
    print(f"[fulllength] c3 {prec} @{steps} pointwise (amplified, not asserted): " +
          ", ".join(f"{k}={v:.2e}" for k, v in errs.items()) +
          f"; aggregates: max |dL| {dL:.3f} cells, Vs {dVs:.2e}, M' {dM:.2e}", flush=True)
    assert dL <= 1.0 and dVs <= 2e-3 and dM <= 1e-3
    s.close()


def test_full_length_flow_fp64(lb):
    """The binary64 GPU path over the full 20000 steps: the same algorithm as the oracle, apart from
    rounding order and contraction, whose differences the interface dynamics amplifies after about
    4000 steps; the aggregates stay tight."""
    z, meta, p = load("c3")
    steps = meta["steps"]
    s = run(lb, p, "fp64", steps)
    errs = errors(s, z, p)
    dL, dVs, dM = aggregates(s, z)
    print(f"[fulllength] c3 fp64 @{steps}: " + ", ".join(f"{k}={v:.2e}" for k, v in errs.items()) +
          f"; aggregates: max |dL| {dL:.2e} cells, Vs {dVs:.2e}, M' {dM:.2e}", flush=True)
    assert dL <= 1e-4 and dVs <= 1e-8 and dM <= 1e-8
    for k, v in errs.items():  # measured 1.5e-3 (phi): rounding-order differences amplified ~20x per 2000 steps
        assert v <= 1e-2, (k, v)
    s.close()


# Binary32 against the oracle on the 96x64x64 flow grid at eps = 0.02 (stiffness 1 - 72 eps cos 6 theta
# only mildly negative near the axes, -0.44: no amplification of rounding seen within 20000 steps),
# per snapshot. phi, rho and u stay within 1e-4 through the 20000 steps, and so does U on every
# sampled node outside the crystal (oracle phi < 0.9: the liquid and the interface, where U enters
# the phase field through lambda U (1 - phi^2)^2 and sets the growth). Inside the crystal
# q = 1 - phi = 0 makes tau_U exactly 1/2: the solute lattice there has no diffusion and its
# non-equilibrium modes are not damped, so the rounding of the stored solute populations stays in
# the field (binary32 against binary64 on the GPU after 20000 steps: U off by 6e-5 at crystal nodes
# where phi is off by 1e-7, 1e-6 in the liquid and at the interface; resolving phi in the crystal
# as binary64 does leaves U there no better). U over all samples, crystal included, against the oracle:
# 1.7e-5, 4.9e-5, 1.2e-4, 2.0e-4 and 2.5e-4 at 4000 .. 20000 steps (2.3e-4 at 8000 and 9.3e-4 at
# 20000 without the compensated closure of the phase-field collision).
C3R_U_BAR = {4000: 1e-4, 8000: 1e-4, 12000: 1.6e-4, 16000: 2.6e-4, 20000: 3.2e-4}


@pytest.mark.parametrize("prec", ["fp32", "fp64", "fp16shift"])
def test_reduced_flow_grid_every_4000_steps(lb, prec):
    """The 96x64x64 flow grid at eps = 0.02 against the oracle's state every 4000 steps through
    20000: binary64 to 1e-10; binary32 as the comment above says; binary16 flow storage within the
    mode's 5e-2 per field (measured at 20000 steps: rho 1.9e-2, phi 1.6e-2, u 1.6e-2, U 3.3e-3) and
    0.1 cells in the extents (3.6e-2)."""
    snaps = {}
    for step in (4000, 8000, 12000, 16000, None):
        z, meta, p = load("c3r", step)
        snaps[meta["steps"]] = z
    p = W.config3_reduced()
    s = lb.Solver(p, prec)
    done = 0
    for step in sorted(snaps):
        s.step(step - done)
        done = step
        z = snaps[step]
        errs = errors(s, z, p)
        nz_, ny_, nx_ = z["nodes"][:, 0], z["nodes"][:, 1], z["nodes"][:, 2]
        outside = z["phi"] < 0.9  # liquid and interface nodes, by the oracle's phi
        assert outside.sum() > 1000 and (~outside).sum() > 100
        dU = np.abs(s.read("U")[nz_, ny_, nx_] - z["U"]) / z["absmax_U"]
        errs["U_outside_crystal"] = float(dU[outside].max())
        dL, dVs, dM = aggregates(s, z)
        print(f"[fulllength] c3r {prec} @{step}: " + ", ".join(f"{k}={v:.2e}" for k, v in errs.items()) +
              f"; U in the crystal {float(dU[~outside].max()):.2e}"
              f"; max |dL| {dL:.2e} cells; Vs {dVs:.2e}; M' {dM:.2e}", flush=True)
        if prec == "fp64":
            for k, v in errs.items():
                assert v <= 1e-10, (step, k, v)
            assert dL <= 1e-8 and dVs <= 1e-11 and dM <= 1e-11
        elif prec == "fp16shift":
            for k, v in errs.items():
                assert v <= 5e-2, (step, k, v)
            assert dL <= 0.1
        else:
            for k, v in errs.items():
                assert v <= (C3R_U_BAR[step] if k == "U" else 1e-4), (step, k, v)
            assert dL <= 0.01 and dVs <= 1e-4
    s.close()

