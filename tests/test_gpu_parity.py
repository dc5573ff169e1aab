"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Error metric per field: ||x - x_ref||_inf / ||x_ref||_inf. Bars: binary64 path <= 1e-10 (the
same algorithm, rounding differences only); binary32 path <= 1e-4; the binary16-shift storage of
the flow populations is reported per field against a looser bar.
"""
import math

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


def relerr(a, b):
    den = np.abs(b).max()
    return np.abs(a - b).max() / (den if den > 0 else 1.0)


def field_errors(read, rf, fields, u_scale=0.0):
    """Per-field error; the velocity u* is compared as a vector (max component error over the
    largest reference component), since a near-zero component has no scale of its own. u_scale,
    the case's velocity scale (its inlet velocity), bounds the denominator from below: where the
    flow has died out (a single solidified node), u* is rounding noise on both sides."""
    errs = {}
    for name in fields:
        if name in ("ux", "uy", "uz"):
            continue
        errs[name] = relerr(read(name), rf[name])
    comps = [c for c in ("ux", "uy", "uz") if c in fields]
    umax = max([np.abs(rf[c]).max() for c in comps] + [u_scale])
    if comps and umax > 0:
        errs["u"] = max(np.abs(read(c) - rf[c]).max() for c in comps) / umax
    return errs


def compare(lb, orc, p, prec, steps, fields=("phi", "U", "rho", "ux", "uy", "uz"), tol=None, label=""):
    print(f"[parity] {label} {prec} grid={p['nx']}x{p['ny']}x{p['nz']} flow={p['flow']} "
          f"xbc={p['xbc']} steps={steps}", flush=True)
    ref = orc.Sim(p)
    ref.step(steps)
    rf = ref.fields()
    s = lb.Solver(p, prec)
    s.step(steps)
    errs = field_errors(s.read, rf, fields, p["u_in"] if p["flow"] else 0.0)
    errs["phi_prev"] = relerr(s.read("phi_prev"), ref.phi_prev)
    print(f"[parity]   errors: " + ", ".join(f"{k}={v:.2e}" for k, v in errs.items()), flush=True)
    bar = tol if tol is not None else TOL[prec]
    for k, v in errs.items():
        assert v <= bar, (label, prec, k, v)
    s.close()
    return errs


# ---- the small configurations at full length ---------------------------------------------------

@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_config1_2d_full_length(lb, orc, prec):
    compare(lb, orc, W.config1(), prec, 2000, fields=("phi", "U"), label="2-D 128^2 no flow")


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16shift"])
def test_2d_flow_inlet_outlet(lb, orc, prec):
    p = W.sweep_instance(96, 0.3, 8.0, 0.025)
    p["ny"] = 64
    p["seed_c"] = (48.0, 32.0, 0.0)
    compare(lb, orc, p, prec, 600, label="2-D flow open x")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_2d_flow_periodic(lb, orc, prec):
    p = W.params(dim=2, nx=64, ny=48, flow=1, xbc=0, u_in=0.03, U0=0.3, seed_c=(32, 24, 0), seed_R=7.0)
    compare(lb, orc, p, prec, 400, label="2-D flow periodic")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_3d_no_flow(lb, orc, prec):
    p = W.scaled(W.config2(), 32, 32, 32, seed_R=6.0)
    compare(lb, orc, p, prec, 300, fields=("phi", "U"), label="3-D no flow")


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp16shift"])
def test_3d_flow_inlet_outlet(lb, orc, prec):
    p = W.scaled(W.config3(), 48, 32, 32, seed_R=6.0)
    compare(lb, orc, p, prec, 200, label="3-D flow open x")


# ---- ragged tiles, tiny and degenerate grids -----------------------------------------------------

@pytest.mark.parametrize("dim,dims,flow,xbc", [
    (2, (37, 23, 1), 1, 1), (2, (37, 23, 1), 1, 0), (2, (3, 5, 1), 1, 1), (2, (1, 1, 1), 1, 0),
    (2, (2, 1, 1), 0, 0), (3, (21, 13, 9), 1, 1), (3, (21, 13, 9), 0, 0), (3, (1, 1, 1), 1, 0),
    (3, (3, 2, 5), 1, 1), (3, (70, 9, 6), 1, 0),
])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_ragged_and_tiny_grids(lb, orc, dim, dims, flow, xbc, prec):
    nx, ny, nz = dims
    c = (nx / 2, ny / 2, nz / 2 if dim == 3 else 0.0)
    p = W.params(dim=dim, nx=nx, ny=ny, nz=nz, flow=flow, xbc=xbc, u_in=0.02, U0=0.3, seed_c=c,
                 seed_R=max(1.5, min(nx, ny) / 3))
    compare(lb, orc, p, prec, 50, label=f"ragged {dims}")


@pytest.mark.parametrize("dim,dims,xbc,collision", [
    (2, (37, 23, 1), 2, 0), (2, (3, 5, 1), 2, 0), (3, (21, 13, 9), 2, 0), (3, (3, 2, 5), 2, 1),
    (2, (37, 23, 1), 1, 1), (2, (1, 1, 1), 0, 1), (3, (21, 13, 9), 1, 1), (3, (1, 1, 1), 0, 1),
    (3, (70, 9, 6), 2, 1),
])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_ragged_and_tiny_grids_pressure_outlet_and_mrt(lb, orc, dim, dims, xbc, collision, prec):
    """The same ragged and degenerate grids with the pressure outlet (xbc = 2) and the
    central-Hermite MRT flow collision."""
    nx, ny, nz = dims
    c = (nx / 2, ny / 2, nz / 2 if dim == 3 else 0.0)
    p = W.params(dim=dim, nx=nx, ny=ny, nz=nz, flow=1, xbc=xbc, u_in=0.02, U0=0.3, seed_c=c,
                 seed_R=max(1.5, min(nx, ny) / 3), collision=collision, omega_bulk=1.1)
    compare(lb, orc, p, prec, 50, label=f"ragged {dims} xbc {xbc} collision {collision}")


# ---- full-size one-step checks in the benchmark's launch configuration ------------------------

FULL_SIZE = {"config2": W.config2, "config3": W.config3,
             "config3_chmrt": lambda: dict(W.config3(), collision=1, omega_bulk=1.0),
             "config3_half_source": lambda: dict(W.config3(), solute_source=1)}


@pytest.mark.parametrize("cfg", sorted(FULL_SIZE))
def test_full_size_one_step_from_gpu_state(lb, orc, cfg):
    """Run the full-size grid a while on the GPU (binary32), hand its state to the oracle, and
    check one more step of every node against the oracle's step from the same state (also with the
    central-Hermite MRT flow collision and with the half solute source)."""
    p = FULL_SIZE[cfg]()
    print(f"[parity] full-size {cfg} one step", flush=True)
    s = lb.Solver(p, "fp32")
    s.step(30)
    ref = orc.Sim(p, init=False)
    ref.h[:] = s.read("raw_h")
    ref.g[:] = s.read("raw_g")
    if p["flow"]:
        ref.f[:] = s.read("raw_f")
    ref.phi_prev[:] = s.read("phi_prev")
    s.step(1)
    ref.step(1)
    for name, a, b in (("h", s.read("raw_h"), ref.h), ("g", s.read("raw_g"), ref.g),
                       ("phi_prev", s.read("phi_prev"), ref.phi_prev)) + (
            (("f", s.read("raw_f"), ref.f),) if p["flow"] else ()):
        # one binary32 step from the same state: rounding of a few ulp of the largest value
        err = np.abs(a - b).max() / np.abs(b).max()
        print(f"[parity]   {cfg} {name}: {err:.2e}", flush=True)
        assert err < 2e-6, (cfg, name, err)
    s.close()


# ---- diagnostics -------------------------------------------------------------------------------

@pytest.mark.parametrize("dim,flow", [(2, 0), (2, 1), (3, 1)])
def test_measure_matches_oracle_on_same_state(lb, orc, dim, flow):
    n = 64 if dim == 2 else 32
    p = W.params(dim=dim, nx=n, ny=n, nz=1 if dim == 2 else n, flow=flow, xbc=flow, u_in=0.02, U0=0.3,
                 seed_c=(n / 2, n / 2, n / 2 if dim == 3 else 0), seed_R=8.0 if dim == 2 else 6.0)
    print(f"[parity] measure dim={dim} flow={flow}", flush=True)
    ref = orc.Sim(p)
    ref.step(300 if dim == 2 else 100)
    s = lb.Solver(p, "fp64")
    s.write("raw_h", ref.h)
    s.write("raw_g", ref.g)
    if flow:
        s.write("raw_f", ref.f)
    s.write("phi_prev", ref.phi_prev)
    dirs = W.directions(16)
    if dim == 3:
        dirs = np.concatenate([dirs, [[0, 0, 1.0], [0, 0, -1.0], [0.6, 0, 0.8]]])
    L, m = s.measure(dirs)
    Lr, mr = ref.measure(dirs)
    assert np.abs(L - Lr).max() < 1e-11, (L, Lr)
    for k in ("sumU", "sumPhiPrev", "Vs", "Mprime"):
        assert abs(m[k] - mr[k]) <= 1e-12 * max(1, abs(mr[k])), k
    assert abs(m["umax"] - mr["umax"]) < 1e-14 and m["nonfinite"] == 0
    s.close()


def test_growth_rates_match_oracle_fit(lb, orc):
    from oracle import growth
    p = W.params(dim=2, nx=64, ny=64, U0=0.3, seed_c=(32, 32, 0), seed_R=6.0)
    s = lb.Solver(p, "fp64")
    dirs = W.directions(16)
    t, Ls = [], []
    for k in range(6):
        L, _ = s.measure(dirs)
        t.append(s.nstep)
        Ls.append(L)
        s.step(100)
    G, R2, Ga = s.growth_rates(16)
    Gr, R2r, Gar = growth.growth_rates(np.array(t, float), np.array(Ls))
    assert np.abs(G - Gr).max() < 1e-12 and np.abs(R2 - R2r).max() < 1e-10 and abs(Ga - Gar) < 1e-12
    assert (G > 0).all()  # a supersaturated seed grows in every direction
    s.close()


@pytest.mark.parametrize("nsteps,every,ndirs", [(1050, 100, 16), (200, 5, 256)])
def test_run_with_diagnostics_equals_step_and_measure(lb, nsteps, every, ndirs):
    """lbcg_run (diagnostics kept on the device, one copy back per block of samples; 256 directions
    make blocks of 15 samples) gives bit for bit what lbcg_step + lbcg_measure give, including the
    growth-rate history and the steps after the last sample."""
    p = W.params(dim=3, nx=40, ny=32, nz=32, flow=1, xbc=1, u_in=0.02, U0=0.3, U_in=0.3,
                 seed_c=(16.0, 16.0, 16.0), seed_R=6.0)
    dirs = W.directions(ndirs, 3)
    a = lb.Solver(p, "fp32")
    L_run, m_run = a.run(nsteps, every, dirs)
    b = lb.Solver(p, "fp32")
    L_seq, m_seq = [], []
    for _ in range(nsteps // every):
        b.step(every)
        L, m = b.measure(dirs)
        L_seq.append(L)
        m_seq.append(m)
    b.step(nsteps % every)
    assert L_run.shape == (nsteps // every, ndirs) and a.nstep == b.nstep == nsteps
    assert np.array_equal(L_run, np.array(L_seq))
    for x, y in zip(m_run, m_seq):
        assert all(x[k] == y[k] for k in ("sumU", "sumPhiPrev", "Vs", "Mprime", "umax", "nonfinite"))
    if ndirs == 16:
        assert all(np.array_equal(u, v) for u, v in zip(a.growth_rates(ndirs), b.growth_rates(ndirs)))
    for k in ("raw_h", "raw_g", "raw_f", "phi_prev"):
        assert np.array_equal(a.read(k), b.read(k)), k
    a.close()
    b.close()


def test_run_edge_cases(lb):
    """No directions (sums only), fewer steps than one interval (no sample, the steps still run),
    and the argument errors."""
    p = W.params(dim=2, nx=40, ny=40, U0=0.3, seed_c=(20, 20, 0), seed_R=5.0)
    s = lb.Solver(p, "fp64")
    L, m = s.run(30, 10)
    assert L.shape == (3, 0) and len(m) == 3 and s.nstep == 30
    L, m = s.run(7, 10, W.directions(4))
    assert L.shape == (0, 4) and m == [] and s.nstep == 37
    r = lb.Solver(p, "fp64")
    r.step(37)
    assert np.array_equal(r.read("raw_h"), s.read("raw_h"))
    for bad in ((10, 0), (-1, 5)):
        with pytest.raises(lb.LbcgError) as e:
            s.run(*bad)
        assert e.value.status == "EINVAL"
    with pytest.raises(lb.LbcgError) as e:
        s.run(10, 5, np.array([[1.0, 1.0, 0.0]]))  # not a unit vector
    assert e.value.status == "EINVAL"
    s.close()
    r.close()


def test_run_reports_nonfinite(lb):
    p = W.params(dim=2, nx=32, ny=32, seed_c=(16, 16, 0))
    s = lb.Solver(p, "fp32")
    h = s.read("raw_h")
    h[0, 0, 3, 3] = np.nan
    s.write("raw_h", h)
    with pytest.raises(lb.LbcgError) as e:
        s.run(50, 10, W.directions(4))
    assert e.value.status == "ENONFINITE"
    with pytest.raises(lb.LbcgError) as e:
        s.step(1)
    assert e.value.status == "ENONFINITE"
    s.close()


def test_solute_plus_solid_invariant_fp32(lb):
    p = W.scaled(W.config2(), 64, 64, 64, seed_R=8.0)
    s = lb.Solver(p, "fp32")
    M0 = s.measure()[1]["Mprime"]
    s.step(1000)
    M1 = s.measure()[1]["Mprime"]
    print(f"[parity] M' drift fp32 64^3 1000 steps: {abs(M1 - M0) / M0:.2e}", flush=True)
    assert abs(M1 - M0) / M0 < 1e-6
    s.close()


# ---- state handling --------------------------------------------------------------------------------

@pytest.mark.parametrize("prec,device", [("fp32", False), ("fp16shift", True), ("fp64", False)])
def test_checkpoint_restart_and_determinism_bitwise(lb, prec, device):
    p = W.scaled(W.config3(), 48, 32, 32, seed_R=6.0)
    a = lb.Solver(p, prec)
    a.step(40)
    ck = a.save_state(device=device)
    a.step(30)
    b = lb.Solver(p, prec)
    b.step(3)
    b.load_state(ck)
    assert b.nstep == 40
    b.step(30)
    c = lb.Solver(p, prec)
    c.step(70)
    for k in ("raw_h", "raw_g", "raw_f", "phi_prev"):
        ra = a.read(k, np.float64)
        assert np.array_equal(ra, b.read(k, np.float64)), k   # restart from a checkpoint
        assert np.array_equal(ra, c.read(k, np.float64)), k   # a second run
    for s in (a, b, c):
        s.close()


def test_checkpoint_rejects_another_grid(lb):
    p = W.scaled(W.config3(), 48, 32, 32, seed_R=6.0)
    a = lb.Solver(p, "fp32")
    ck = a.save_state()
    for q, prec in ((W.scaled(W.config3(), 48, 32, 30, seed_R=6.0), "fp32"), (p, "fp16shift")):
        b = lb.Solver(q, prec)
        with pytest.raises(lb.LbcgError) as e:
            b.load_state(ck)
        assert e.value.status == "EINVAL"
        b.close()
    with pytest.raises(lb.LbcgError) as e:
        a.load_state(ck[:-1])
    assert e.value.status == "ENOMEM"
    a.close()


def test_raw_population_round_trip(lb):
    """Writing back what lbcg_read_field returns reproduces the populations to the storage
    precision (binary32 here: a few units in the last place of each plane)."""
    p = W.scaled(W.config3(), 40, 24, 20, seed_R=5.0)
    a = lb.Solver(p, "fp32")
    a.step(20)
    b = lb.Solver(p, "fp32")
    for k in ("raw_h", "raw_g", "raw_f", "phi_prev"):
        v = a.read(k, np.float64)
        b.write(k, v)
        d = np.abs(b.read(k, np.float64) - v).max()
        assert d <= 2.0 ** -22 * np.abs(v).max(), (k, d)  # stored values are at most twice the decoded scale
    a.close()
    b.close()


def test_nonfinite_is_reported(lb):
    p = W.params(dim=2, nx=32, ny=32, seed_c=(16, 16, 0))
    s = lb.Solver(p, "fp32")
    h = s.read("raw_h")
    h[0, 0, 3, 3] = np.nan
    s.write("raw_h", h)
    with pytest.raises(lb.LbcgError) as e:
        s.measure()
    assert e.value.status == "ENONFINITE"
    with pytest.raises(lb.LbcgError) as e:
        s.step(1)
    assert e.value.status == "ENONFINITE"
    s.close()


# ---- kernel variants ---------------------------------------------------------------------------

@pytest.mark.parametrize("cfg,prec", [("c3small", "fp32"), ("c3small", "fp64"), ("c2small", "fp32"),
                                      ("c1small", "fp32"), ("c4inst", "fp16shift")])
def test_every_variant_computes_the_same_step(lb, cfg, prec):
    """All tilings of the step kernel give the same state (the autotuner may pick any of them)."""
    p = {"c3small": W.scaled(W.config3(), 70, 20, 18, seed_R=6.0),
         "c2small": W.scaled(W.config2(), 40, 24, 20, seed_R=6.0),
         "c1small": W.scaled(W.config1(), 100, 36, 1, seed_R=8.0),
         "c4inst": W.sweep_instance(96, 0.3, 8.0, 0.02)}[cfg]
    ref = None
    s0 = lb.Solver(p, prec)
    names = s0.variants()
    s0.close()
    print(f"[parity] variants {cfg} {prec}: {names}", flush=True)
    for k, name in enumerate(names):
        s = lb.Solver(p, prec)
        s.select_variant(k)
        s.step(25)
        state = [s.read(f) for f in ("raw_h", "raw_g", "phi_prev") + (("raw_f",) if p["flow"] else ())]
        s.close()
        if ref is None:
            ref = state
            continue
        for a, b in zip(state, ref):
            err = np.abs(a - b).max() / np.abs(b).max()
            assert err < (1e-12 if prec == "fp64" else 1e-5), (name, err)


def test_variant_timer_runs_real_steps(lb):
    """Timing a variant advances the state by launches + 1 steps of that variant and leaves the
    selected variant alone."""
    p = W.scaled(W.config3(), 70, 20, 18, seed_R=6.0)
    a, b = lb.Solver(p, "fp32"), lb.Solver(p, "fp32")
    k = len(a.variants()) - 1
    a.step(3)
    us = a.time_variant(k, 4)
    assert us > 0 and a.nstep == 8 and a.variant == 0
    b.step(3)
    b.select_variant(k)
    b.step(5)
    for f in ("raw_h", "raw_g", "raw_f", "phi_prev"):
        assert np.array_equal(a.read(f), b.read(f)), f
    best, best_us = a.autotune(2)
    assert a.variant == best and best_us > 0 and a.nstep == 8 + 2 * 3 * len(a.variants())  # two rounds
    a.close()
    b.close()


# ---- batched sweep ------------------------------------------------------------------------------

@pytest.mark.parametrize("use_graph", [True, False])
def test_batch_matches_single_instances_bitwise(lb, use_graph):
    """Each instance of a batch evolves exactly as a single solver with its parameters."""
    draws = W.sweep_draws(6, seed=7)
    draws[0] = (64,) + draws[0][1:]
    plist = [W.sweep_instance(*d) for d in draws]
    dirs = W.directions(16)
    b = lb.Batch(plist, "fp32")
    hist = b.run(300, 100, dirs, use_graph=use_graph)
    b.run(7)  # an odd remainder without measurements
    assert hist.shape == (3, len(plist), 16) and b.nstep == 307
    for i, p in enumerate(plist):
        s = lb.Solver(p, "fp32")
        s.select_variant(s.variants().index(b.variants()[b.variant]))  # the batch's tiling
        Ls = []
        for _ in range(3):
            s.step(100)
            Ls.append(s.measure(dirs)[0])
        s.step(7)
        assert np.array_equal(np.array(Ls), hist[:, i, :]), i
        for f in ("raw_h", "raw_g", "raw_f", "phi_prev"):
            assert np.array_equal(s.read(f, np.float32), b.read(i, f, np.float32)), (i, f)
        s.close()
    b.close()


def test_batch_against_oracle(lb, orc):
    draws = W.sweep_draws(3, seed=11)
    plist = [W.sweep_instance(min(d[0], 96), *d[1:]) for d in draws]
    b = lb.Batch(plist, "fp64")
    b.run(200)
    for i, p in enumerate(plist):
        ref = orc.Sim(p)
        ref.step(200)
        rf = ref.fields()
        errs = field_errors(lambda f: b.read(i, f), rf, ("phi", "U", "rho", "ux", "uy"))
        print(f"[parity] batch instance {i} side {p['nx']}: " + ", ".join(f"{k}={v:.1e}" for k, v in errs.items()))
        assert max(errs.values()) < 1e-10
    b.close()
