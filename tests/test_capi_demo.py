"""A plain C caller of include/lbcg.h (tests/capi_demo.c, built by build()): it owns its device
workspace and stream, and its diagnostics match the oracle's. The CPU tests check that it was
built and rejects bad parameters before touching a device."""
import os
import subprocess

import numpy as np
import pytest

from paper_2206_02145_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "tests", "capi_demo")
PREC = {"fp64": 0, "fp32": 1, "fp16shift": 2}


def argv(p, prec, steps):
    keys = ("dim", "nx", "ny", "nz", "flow", "xbc")
    vals = [str(int(p[k])) for k in keys] + [str(PREC[prec])]
    vals += [repr(float(p[k])) for k in ("W0", "tau0", "lam", "D", "eps", "nu", "h_drag", "u_in", "U0", "U_in")]
    vals += [repr(float(v)) for v in p["seed_c"]] + [repr(float(p["seed_R"]))]
    vals += [str(int(p.get("collision", 0))), repr(float(p.get("omega_bulk", 1.0))), str(steps)]
    return [EXE] + vals


def test_demo_is_built_and_validates_before_the_device():
    if not os.path.exists(EXE):  # build() compiles it; a fresh checkout may not have run build()
        from paper_2206_02145_amd import build
        build.build_capi_demo()
    assert os.path.exists(EXE)
    r = subprocess.run([EXE], capture_output=True, text=True)
    assert r.returncode == 2 and "usage" in r.stderr
    r = subprocess.run(argv(W.params(dim=4), "fp64", 1), capture_output=True, text=True)
    assert r.returncode == 1 and "invalid parameters" in r.stderr


CASES = {
    "2d_flow_fp64": (W.params(dim=2, nx=96, ny=64, flow=1, xbc=1, u_in=0.02, U0=0.25, U_in=0.25,
                              seed_c=(40.0, 32.0, 0.0), seed_R=8.0), "fp64", 300),
    "3d_mrt_fp32": (W.params(dim=3, nx=40, ny=32, nz=32, flow=1, xbc=2, u_in=0.02, U0=0.3, U_in=0.3,
                             seed_c=(16.0, 16.0, 16.0), seed_R=6.0, collision=1, omega_bulk=1.0), "fp32", 150),
}


@pytest.mark.gpu
@pytest.mark.parametrize("case", sorted(CASES))
def test_demo_matches_oracle(case):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from oracle import oracle as o
    o.build(force=False)
    p, prec, steps = CASES[case]
    print(f"[capi demo] {case}", flush=True)
    r = subprocess.run(argv(p, prec, steps), capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    out = {ln.split()[0]: [float(v) for v in ln.split()[1:]] for ln in r.stdout.splitlines()}
    assert int(out["steps"][0]) == steps
    ref = o.Sim(p)
    ref.step(steps)
    dirs = np.array([[1.0, 0, 0], [-1.0, 0, 0], [0, 1.0, 0], [0, -1.0, 0]])
    L, mass = ref.measure(dirs)
    dL = float(np.abs(np.array(out["L"]) - L).max())
    m = out["mass"]
    dVs = abs(m[2] - mass["Vs"]) / abs(mass["Vs"])
    dM = abs(m[3] - mass["Mprime"]) / abs(mass["Mprime"])
    print(f"[capi demo] {case}: L {out['L']}, |dL| {dL:.2e} cells, Vs {dVs:.2e}, M' {dM:.2e}", flush=True)
    tol = 1e-9 if prec == "fp64" else 1e-3
    assert dL <= tol * 10 and dVs <= tol and dM <= tol
    assert m[5] == 0  # no non-finite values
