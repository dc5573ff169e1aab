"""The largest grids the library takes. 2^29 - 1 nodes (2089 x 1103 x 233: ragged in x, y and z),
where the byte offsets of a binary64 population plane reach 2^32 - 8 and the stored rows fall back
to the dense layout; and 2000 x 1100 x 233, the largest kind that keeps the padded row pitch (2048)
and plane stride, with binary64 planes of 4.2 GB. Binary32 with flow and the inlet / outlet faces
(up to 148 GB of device workspace) and binary64 without flow (up to 129 GB): a seed near the far
corner of the grid, at the highest addresses, must evolve as the same seed in a small grid holding
the same neighbourhood. After a few steps the seed's influence is still far from the window's faces,
where both grids are uniform, so the window and the small grid agree to the bar of two kernel
tilings (the largest and the small grid may pick different ones)."""
import gc

import numpy as np
import pytest

from paper_2206_02145_amd import workloads as W

pytestmark = pytest.mark.gpu

NX, NY, NZ = 2089, 1103, 233          # 2089 * 1103 * 233 = 2^29 - 1
GRIDS = {"dense": (NX, NY, NZ), "padded": (2000, 1100, 233)}
WX, WY, WZ = 96, 80, 80               # the window / the small grid
STEPS = 5


@pytest.fixture(scope="module")
def lb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2206_02145_amd import lbcg
    lbcg.lib()
    return lbcg


def pair(flow: int, grid):
    """The large grid with the seed 40 nodes inside its far corner, and the small grid with the
    seed at the same place relative to the window of the last WX x WY x WZ nodes."""
    NX, NY, NZ = grid
    kw = dict(dim=3, flow=flow, xbc=1 if flow else 0, u_in=0.02 if flow else 0.0, U0=0.3, U_in=0.3, seed_R=6.0)
    big = W.params(nx=NX, ny=NY, nz=NZ, seed_c=(NX - 40.0, NY - 40.0, NZ - 40.0), **kw)
    small = W.params(nx=WX, ny=WY, nz=WZ, seed_c=(WX - 40.0, WY - 40.0, WZ - 40.0), **kw)
    return big, small


def window_errors(lb, prec, flow, fields, grid):
    import torch
    NX, NY, NZ = grid
    big, small = pair(flow, grid)
    dt = torch.float64 if prec == "fp64" else torch.float32
    print(f"[maxsize] {prec} flow={flow}: {NX}x{NY}x{NZ}, workspace "
          f"{lb.lbcg_workspace_bytes(lb.make_params(big, prec)) / 1e9:.1f} GB", flush=True)
    s = lb.Solver(small, prec)
    s.step(STEPS)
    ref = {f: s.read(f) for f in fields}
    s.close()
    assert ref["phi"].max() > 0.9                                    # the seed is in the window
    if flow:
        assert np.abs(ref["ux"]).max() > 0.01                        # and so is the flow
    b = lb.Solver(big, prec)
    b.step(STEPS)
    # the small grid's own inlet face (x = 0) differs from the big grid's interior: skip 8 columns
    m = 8
    errs = {}
    for f in fields:
        d = b.read_device(f, dt)
        win = d[NZ - WZ:, NY - WY:, NX - WX:].double().cpu().numpy()
        del d
        torch.cuda.empty_cache()
        r = ref[f]
        den = max(float(np.abs(r).max()), 1e-30)
        errs[f] = float(np.abs(win[:, :, m:] - r[:, :, m:]).max()) / den
    mass = b.measure()[1]
    b.close()
    del b
    gc.collect()
    torch.cuda.empty_cache()
    print(f"[maxsize] {prec} flow={flow} after {STEPS} steps: " + ", ".join(f"{k}={v:.2e}" for k, v in errs.items()) +
          f"; nonfinite {mass['nonfinite']:.0f}", flush=True)
    assert mass["nonfinite"] == 0
    return errs


def test_largest_grid_has_2_29_minus_1_nodes():
    assert NX * NY * NZ == 2 ** 29 - 1


@pytest.mark.parametrize("grid", list(GRIDS))
def test_largest_grid_binary32_flow(lb, grid):
    errs = window_errors(lb, "fp32", 1, ("phi", "U", "rho", "ux", "uy", "uz"), GRIDS[grid])
    for k, v in errs.items():
        assert v <= 1e-5, (k, v)


@pytest.mark.parametrize("grid", list(GRIDS))
def test_largest_grid_binary64(lb, grid):
    errs = window_errors(lb, "fp64", 0, ("phi", "U"), GRIDS[grid])
    for k, v in errs.items():
        assert v <= 1e-12, (k, v)


def test_one_node_more_is_rejected(lb):
    p = W.params(dim=3, nx=NX + 1, ny=NY, nz=NZ)
    assert lb.lbcg_workspace_bytes(lb.make_params(p, "fp32")) == 0
    with pytest.raises(lb.LbcgError):
        lb.Solver(p, "fp32")
