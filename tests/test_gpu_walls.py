"""Solid walls (reactor walls and baffles: zero-flux phase field and solute, no-slip flow) and the
pressure outlet (rho = 1 anti-bounce-back) on the GPU against the oracle, through the C ABI
(lbcg_set_walls)."""
import numpy as np
import pytest

from paper_2206_02145_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-4, "fp16shift": 5e-3}


@pytest.fixture(scope="module")
def lb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2206_02145_amd import lbcg
    lbcg.lib()
    return lbcg


@pytest.fixture(scope="module")
def orc():
    from oracle import oracle as o
    o.build(force=False)
    return o


def channel_2d():
    """96 x 48 channel: wall rows at y = 0 and y = 47, a baffle plate at x = 20 (y 16 .. 31) in
    front of a seed at (44, 24); inflow from x-."""
    p = W.params(dim=2, nx=96, ny=48, flow=1, xbc=1, u_in=0.02, U0=0.25, U_in=0.25,
                 seed_c=(44.0, 24.0, 0.0), seed_R=6.0)
    m = np.zeros((1, 48, 96), np.uint8)
    m[0, 0, :] = m[0, 47, :] = 1
    m[0, 16:32, 20] = 1
    return p, m


def box_3d():
    """48 x 24 x 20 with flow from x-: a floor (z = 0), a side wall (y = 0) and a baffle plate at
    x = 12 (y 6 .. 17, z 4 .. 15) in front of a seed at (26, 12, 10)."""
    p = W.params(dim=3, nx=48, ny=24, nz=20, flow=1, xbc=1, u_in=0.02, U0=0.3, U_in=0.3,
                 seed_c=(26.0, 12.0, 10.0), seed_R=5.0)
    m = np.zeros((20, 24, 48), np.uint8)
    m[0, :, :] = 1
    m[:, 0, :] = 1
    m[4:16, 6:18, 12] = 1
    return p, m


def relerr(a, b):
    d = np.abs(b).max()
    return float(np.abs(a - b).max() / d) if d > 0 else float(np.abs(a).max())


def compare(lb, orc, p, m, prec, steps, variant=None):
    q = dict(p, walls=1)
    s = lb.Solver(q, prec)
    if variant is not None:
        s.select_variant(variant)
    s.set_walls(m)
    s.step(steps)
    ref = orc.Sim(p)
    ref.set_walls(m)
    ref.step(steps)
    rf = ref.fields()
    errs = {k: relerr(s.read(k), rf[k]) for k in ("phi", "U", "rho")}
    um = max([np.abs(rf[c]).max() for c in ("ux", "uy", "uz")] + [p["u_in"]])
    du = max(float(np.abs(s.read(c) - rf[c]).max()) for c in ("ux", "uy", "uz"))
    errs["u"] = du / um if um > 0 else du  # no flow at all: u* = 0 on both sides
    _, mg = s.measure()
    _, mo = ref.measure()
    errs["Vs"] = abs(mg["Vs"] - mo["Vs"]) / abs(mo["Vs"])
    errs["M'"] = abs(mg["Mprime"] - mo["Mprime"]) / abs(mo["Mprime"])
    print(f"[walls] {p['dim']}-D {prec} {steps} steps" + (f" variant {variant}" if variant is not None else "") +
          ": " + ", ".join(f"{k}={v:.2e}" for k, v in errs.items()), flush=True)
    state = {k: s.read(k) for k in ("raw_h", "raw_g", "raw_f", "phi_prev")}
    s.close()
    return errs, state


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16shift"])
def test_walls_2d_channel_with_baffle(lb, orc, prec):
    p, m = channel_2d()
    errs, _ = compare(lb, orc, p, m, prec, 400)
    for k, v in errs.items():
        assert v <= TOL[prec], (prec, k, v)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_walls_3d_box_with_baffle_every_variant(lb, orc, prec):
    p, m = box_3d()
    s = lb.Solver(dict(p, walls=1), prec)
    names = s.variants()
    s.close()
    assert all("walls" in n for n in names)
    ref = None
    for k in range(len(names)):
        errs, state = compare(lb, orc, p, m, prec, 120, variant=k)
        for key, v in errs.items():
            assert v <= TOL[prec], (prec, names[k], key, v)
        if ref is None:
            ref = state
        else:
            for key in state:
                assert relerr(state[key], ref[key]) < (1e-12 if prec == "fp64" else 1e-5), (names[k], key)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16shift"])
def test_pressure_outlet_2d_channel_with_baffle(lb, orc, prec):
    p, m = channel_2d()
    errs, _ = compare(lb, orc, dict(p, xbc=2), m, prec, 400)
    for k, v in errs.items():
        assert v <= TOL[prec], (prec, k, v)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_pressure_outlet_3d_box_every_variant(lb, orc, prec):
    p, m = box_3d()
    p = dict(p, xbc=2)
    s = lb.Solver(dict(p, walls=1), prec)
    names = s.variants()
    s.close()
    assert not any(n.startswith("march") for n in names)
    for k in range(len(names)):
        errs, _ = compare(lb, orc, p, m, prec, 120, variant=k)
        for key, v in errs.items():
            assert v <= TOL[prec], (prec, names[k], key, v)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_pressure_outlet_without_walls_single_and_batched(lb, orc, prec):
    """A seed in the free stream with the pressure outlet, as one grid and inside a batch."""
    p = W.params(dim=3, nx=40, ny=24, nz=24, flow=1, xbc=2, u_in=0.03, U0=0.3, U_in=0.3,
                 seed_c=(16.0, 12.0, 12.0), seed_R=5.0)
    steps = 150
    ref = orc.Sim(p)
    ref.step(steps)
    rf = ref.fields()
    s = lb.Solver(p, prec)
    s.step(steps)
    b = lb.Batch([dict(p, U0=0.2, U_in=0.2), p], prec)
    b.run(steps)
    for k in ("phi", "U", "rho", "ux", "uy", "uz"):
        scale = max(np.abs(rf[k]).max(), 1e-3)
        e1 = float(np.abs(s.read(k) - rf[k]).max()) / scale
        e2 = float(np.abs(b.read(1, k) - rf[k]).max()) / scale
        print(f"[pressure outlet] 3-D {prec} {k}: single {e1:.2e}, batched {e2:.2e}", flush=True)
        assert e1 <= TOL[prec] and e2 <= TOL[prec], (k, e1, e2)
    s.close()
    b.close()


@pytest.mark.parametrize("case", ["2d_5x3", "3d_6x3x2", "2d_37x23_outlet"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_walls_on_tiny_and_ragged_grids(lb, orc, case, prec):
    """Grids smaller than a tile (their halo box reaches past the last row) and a ragged channel."""
    if case == "2d_5x3":
        p = W.params(dim=2, nx=5, ny=3, flow=1, xbc=0, U0=0.3, U_in=0.3, seed_c=(2.0, 1.5, 0.0), seed_R=1.5)
        m = np.zeros((1, 3, 5), np.uint8)
        m[0, 0, :] = 1
        steps = 40
    elif case == "3d_6x3x2":
        p = W.params(dim=3, nx=6, ny=3, nz=2, flow=1, xbc=0, U0=0.3, U_in=0.3, seed_c=(3.0, 1.5, 1.0), seed_R=1.5)
        m = np.zeros((2, 3, 6), np.uint8)
        m[0] = 1
        steps = 40
    else:
        p = W.params(dim=2, nx=37, ny=23, flow=1, xbc=2, u_in=0.02, U0=0.3, U_in=0.3, seed_c=(22.0, 11.5, 0.0),
                     seed_R=4.0)
        m = np.zeros((1, 23, 37), np.uint8)
        m[0, 0, :] = m[0, 22, :] = 1
        m[0, 6:17, 9] = 1
        steps = 120
    errs, _ = compare(lb, orc, p, m, prec, steps)
    for k, v in errs.items():
        assert v <= TOL[prec], (case, prec, k, v)


def test_walls_keep_solute_plus_solid_in_binary32(lb):
    n = 64
    p = W.params(dim=2, nx=n, ny=n, flow=0, xbc=0, U0=0.2, U_in=0.2, seed_c=(32, 32, 0), seed_R=8.0, walls=1)
    m = np.zeros((1, n, n), np.uint8)
    m[0, 0, :] = 1
    m[0, :, 0] = 1
    m[0, 20:44, 12] = 1
    s = lb.Solver(p, "fp32")
    s.set_walls(m)
    M0 = s.measure()[1]["Mprime"]
    s.step(1000)
    M1 = s.measure()[1]["Mprime"]
    print(f"[walls] M' drift fp32 1000 steps: {abs(M1 - M0) / M0:.2e}", flush=True)
    assert abs(M1 - M0) / M0 < 1e-6
    s.close()


def test_set_walls_errors(lb):
    p, m = channel_2d()
    s = lb.Solver(p, "fp32")  # created without walls
    with pytest.raises(lb.LbcgError) as e:
        s.set_walls(m)
    assert e.value.status == "EINVAL"
    s.close()
    s = lb.Solver(dict(p, walls=1), "fp32")
    bad = m.copy()
    bad[0, 10, 95] = 1  # one of the two outlet columns of a row
    with pytest.raises(lb.LbcgError) as e:
        s.set_walls(bad)
    assert e.value.status == "EINVAL"
    s.close()
    with pytest.raises(lb.LbcgError) as e:
        lb.Batch([dict(p, walls=1)], "fp32")
    assert e.value.status == "EINVAL"


@pytest.mark.parametrize("dims", [(2, 96, 40, 1), (3, 70, 9, 6)])
def test_wall_mask_starts_empty_on_ragged_rows(lb, dims):
    """A solver created with walls = 1 and no lbcg_set_walls call has no wall anywhere, also in the
    pad columns of rows whose length is not a multiple of 64 nodes, whatever the workspace held
    before: it evolves bit for bit as the same solver without walls."""
    dim, nx, ny, nz = dims
    p = W.params(dim=dim, nx=nx, ny=ny, nz=nz, flow=1, xbc=1, u_in=0.02, U0=0.25, U_in=0.25,
                 seed_c=(nx / 2, ny / 2, nz / 2 if dim == 3 else 0.0), seed_R=4.0)
    a = lb.Solver(dict(p, walls=1), "fp32", ws_fill=0xFF)
    b = lb.Solver(p, "fp32")
    a.step(40)
    b.step(40)
    for name in ("phi", "U", "rho", "ux", "uy", "raw_h", "raw_g", "raw_f"):
        assert np.array_equal(a.read(name), b.read(name)), name
    La, ma = a.measure(W.directions(8))
    Lb, mb = b.measure(W.directions(8))
    assert np.array_equal(La, Lb)
    assert all(ma[k] == mb[k] for k in mb), (ma, mb)
    a.close()
    b.close()

