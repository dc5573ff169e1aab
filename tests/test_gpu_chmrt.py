"""Central-Hermite MRT flow collision (lbcg_params.collision = 1) on the GPU against the oracle,
through the C ABI: coupled growth in an inflow (2-D and 3-D, every tiling), with walls, in a
batch, and a low-viscosity shear layer that BGK cannot hold."""
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


def errors(read, rf):
    """Relative max errors of phi, U, rho and u* (as a vector) against the oracle's fields."""
    out = {}
    for k in ("phi", "U", "rho"):
        out[k] = float(np.abs(read(k) - rf[k]).max() / np.abs(rf[k]).max())
    um = max(np.abs(rf[c]).max() for c in ("ux", "uy", "uz"))
    out["u"] = max(float(np.abs(read(c) - rf[c]).max()) for c in ("ux", "uy", "uz")) / um
    return out


def report(tag, errs):
    print(f"[chmrt] {tag}: " + ", ".join(f"{k}={v:.2e}" for k, v in errs.items()), flush=True)


def growth_2d():
    return W.params(dim=2, nx=96, ny=64, flow=1, xbc=1, u_in=0.03, U0=0.25, U_in=0.25, seed_c=(40.0, 32.0, 0.0),
                    seed_R=8.0, collision=1, omega_bulk=1.2, nu=0.02)


def growth_3d(xbc=1):
    return W.params(dim=3, nx=40, ny=24, nz=24, flow=1, xbc=xbc, u_in=0.03, U0=0.3, U_in=0.3,
                    seed_c=(16.0, 12.0, 12.0), seed_R=5.0, collision=1, omega_bulk=1.0)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16shift"])
def test_chmrt_growth_in_inflow_2d(lb, orc, prec):
    p = growth_2d()
    ref = orc.Sim(p)
    ref.step(400)
    s = lb.Solver(p, prec)
    assert all("chmrt" in n for n in s.variants())
    s.step(400)
    errs = errors(s.read, ref.fields())
    report(f"2-D {prec} 400 steps", errs)
    for k, v in errs.items():
        assert v <= TOL[prec], (prec, k, v)
    s.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16shift"])
def test_chmrt_growth_in_inflow_3d_every_variant(lb, orc, prec):
    p = growth_3d()
    ref = orc.Sim(p)
    ref.step(150)
    rf = ref.fields()
    s = lb.Solver(p, prec)
    names = s.variants()
    s.close()
    for k, name in enumerate(names):
        s = lb.Solver(p, prec)
        s.select_variant(k)
        s.step(150)
        errs = errors(s.read, rf)
        report(f"3-D {prec} 150 steps, {name}", errs)
        for key, v in errs.items():
            assert v <= TOL[prec], (prec, name, key, v)
        s.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_chmrt_with_walls_and_pressure_outlet(lb, orc, prec):
    """A walled 2-D channel with a baffle (pressure outlet), and a 3-D box with a floor."""
    p = W.params(dim=2, nx=96, ny=48, flow=1, xbc=2, u_in=0.02, U0=0.25, U_in=0.25, seed_c=(44.0, 24.0, 0.0),
                 seed_R=6.0, collision=1, omega_bulk=1.0)
    m = np.zeros((1, 48, 96), np.uint8)
    m[0, 0, :] = m[0, 47, :] = 1
    m[0, 16:32, 20] = 1
    q = growth_3d(xbc=2)
    m3 = np.zeros((24, 24, 40), np.uint8)
    m3[0] = 1
    for pp, mm, steps in ((p, m, 300), (q, m3, 120)):
        ref = orc.Sim(pp)
        ref.set_walls(mm)
        ref.step(steps)
        s = lb.Solver(dict(pp, walls=1), prec)
        s.set_walls(mm)
        s.step(steps)
        errs = errors(s.read, ref.fields())
        report(f"walls {pp['dim']}-D {prec} {steps} steps", errs)
        for k, v in errs.items():
            assert v <= TOL[prec], (pp["dim"], prec, k, v)
        s.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_chmrt_batched_equals_single(lb, prec):
    p = growth_2d()
    q = dict(p, u_in=0.02, omega_bulk=0.8)
    b = lb.Batch([p, q], prec)
    b.run(200)
    for i, pp in enumerate((p, q)):
        s = lb.Solver(pp, prec)
        s.step(200)
        for k in ("phi", "U", "rho", "ux", "uy"):
            d = float(np.abs(b.read(i, k) - s.read(k)).max())
            assert d <= (1e-13 if prec == "fp64" else 1e-6), (i, k, d)
        s.close()
    b.close()


def test_chmrt_low_viscosity_shear_layer(lb, orc):
    """Doubly periodic shear layer at nu = 1e-5: the GPU follows the oracle, stays bounded over
    20000 steps, and the BGK kernel on the same state does not."""
    n, u0 = 64, 0.05
    x = (np.arange(n) + 0.5) / n
    X, Y = np.meshgrid(x, x)
    ux = np.where(Y <= 0.5, u0 * np.tanh(80 * (Y - 0.25)), u0 * np.tanh(80 * (0.75 - Y)))
    uy = 0.05 * u0 * np.sin(2 * np.pi * (X + 0.25))
    umax = {}
    for coll in (1, 0):
        p = W.params(dim=2, nx=n, ny=n, flow=1, seed_R=-1e9, nu=1e-5, collision=coll)
        ref = orc.Sim(p, init=False)
        w = np.array([1 / 3, 1 / 6, 1 / 6, 1 / 6, 1 / 6])
        ref.h[:] = -w[:, None, None, None]
        ref.g[:] = (0.1 * w)[:, None, None, None]
        ref.phi_prev[:] = -1.0
        ref.set_flow_equilibrium(1.0, ux[None], uy[None], 0.0)
        s = lb.Solver(p, "fp64")
        s.write("raw_h", ref.h)
        s.write("raw_g", ref.g)
        s.write("raw_f", ref.f)
        s.write("phi_prev", ref.phi_prev)
        if coll == 1:
            ref.step(1000)
            s.step(1000)
            rf = ref.fields()
            e = max(float(np.abs(s.read(c) - rf[c]).max()) for c in ("ux", "uy")) / np.abs(rf["ux"]).max()
            print(f"[chmrt] shear layer nu 1e-5, 1000 steps: u error {e:.2e}", flush=True)
            assert e < 1e-9
            s.step(19000)
        else:
            s.step(1000)
        with np.errstate(invalid="ignore"):
            umax[coll] = float(np.abs(s.read("ux")).max())
        s.close()
    print(f"[chmrt] shear layer max |u_x|: MRT after 20000 steps {umax[1]:.4f}, BGK after 1000 steps {umax[0]:.3g}",
          flush=True)
    assert np.isfinite(umax[1]) and umax[1] < 2 * u0
    assert not np.isfinite(umax[0]) or umax[0] > 1.0


def test_chmrt_extends_the_stable_viscosity_range_in_3d(lb):
    """The coupled 3-D forced-convection problem (96 x 64 x 64, inflow 0.05, a growing seed) at
    nu = 5e-4: BGK turns non-finite within 5000 steps, the central-Hermite MRT does not."""
    status = {}
    for coll in (0, 1):
        p = W.params(dim=3, nx=96, ny=64, nz=64, flow=1, xbc=1, u_in=0.05, U0=0.3, U_in=0.3,
                     seed_c=(32.0, 32.0, 32.0), seed_R=8.0, nu=5e-4, collision=coll, omega_bulk=1.0)
        s = lb.Solver(p, "fp32")
        _, mass = s.run(5000, 500, raise_nonfinite=False)
        status[coll] = max(m["nonfinite"] for m in mass)
        s.close()
    print(f"[chmrt] 3-D nu 5e-4, 5000 steps: non-finite nodes BGK {status[0]:.0f}, MRT {status[1]:.0f}", flush=True)
    assert status[0] > 0 and status[1] == 0


def test_chmrt_parameter_errors(lb):
    p = growth_2d()
    for bad in (dict(p, collision=2), dict(p, omega_bulk=0.0), dict(p, omega_bulk=2.0), dict(p, flow=0)):
        with pytest.raises(lb.LbcgError):
            lb.Solver(bad, "fp32")
