"""Crystal habit under forced convection at the paper's scale (Section 4.2): the Reynolds-number
effect, the seed orientation and baffles in front of the crystal, measured with the habit numbers
(quality Q = max/min of the six face-normal sizes, aspect ratio along / across the flow, and the
upstream / downstream size ratio).

Setting (the paper's 2-D convection studies, with the synthetic geometry of reading R28 in place
of the reactor, which the paper shows only in figures):
* a 31 x 26 mm domain at 0.025 mm (1240 x 1040 nodes), inflow at x = 0, outflow at x = nx - 1;
* a hexagonal seed of perimeter 3.7 mm (circumradius 0.617 mm) at (12.4, 13) mm, U = 0.045;
* the lattice time step by the diffusive scaling of the self-convergence study (W0 = 0.05 mm,
  tau0 = 11 s, D = 4.273e-4 mm^2/s), 10 hours;
* Re = u_in P / nu with P the seed perimeter and nu the lattice viscosity of the other workloads
  (reading R16), so Re 8.6 and 17.2 set u_in;
* with baffles: wall rows at y = 0 and y = ny - 1, a pressure outlet (reading R30), and plates
  across the flow upstream of the seed.

    python -m paper_2206_02145_amd.habit_study --sets re tilt baffle --out habit.json
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import habit
from . import workloads as W

PHYS = dict(Lx=31.0, Ly=26.0, perimeter=3.7, U=0.045, W0=0.05, tau0=11.0, D=4.273e-4, hours=10.0,
            seed_x=12.4, seed_y=13.0)


def lattice(dr: float = 0.025, phys: dict = PHYS) -> dict:
    """Lattice units of spacing dr (mm): cells per W0, steps per tau0, seconds per step, D."""
    k = W.BASE["W0"] ** 2 / W.BASE["tau0"]
    W0c = phys["W0"] / dr
    tau0 = W0c ** 2 / k
    dt = phys["tau0"] / tau0
    return dict(dr=dr, W0=W0c, tau0=tau0, dt=dt, D=phys["D"] * dt / dr ** 2)


def wall_mask(nx: int, ny: int, kind: str, sx: float, sy: float, R: float) -> np.ndarray | None:
    """Synthetic geometry: 'none' (no walls, periodic in y), 'channel' (wall rows at y = 0 and
    ny - 1), 'plate' (the channel plus a plate across the flow 4 R upstream of the seed, covering
    y within 1.5 R of the seed), 'wide' (the same plate covering y within 3 R), 'split' (the channel
    plus two plates 4 R upstream that leave a gap of R in front of the seed and block 3 R on either
    side of it)."""
    if kind == "none":
        return None
    m = np.zeros((1, ny, nx), np.uint8)
    m[0, 0, :] = m[0, ny - 1, :] = 1
    xb = int(round(sx - 4 * R))
    if kind in ("plate", "wide"):
        half = 1.5 * R if kind == "plate" else 3.0 * R
        m[0, int(round(sy - half)):int(round(sy + half)) + 1, xb:xb + 2] = 1
    elif kind == "split":
        m[0, int(round(sy - 3.5 * R)):int(round(sy - 0.5 * R)) + 1, xb:xb + 2] = 1
        m[0, int(round(sy + 0.5 * R)):int(round(sy + 3.5 * R)) + 1, xb:xb + 2] = 1
    elif kind != "channel":
        raise ValueError(kind)
    return m


def case(Re: float, tilt: float = 0.0, baffle: str = "none", dr: float = 0.025, hours: float | None = None,
         phys: dict = PHYS, source: int = 0) -> dict:
    """Parameters, wall mask and step count of one study case; source selects the solute source
    (0: -dphi/dt as Eq. (b) prints it, 1: -(1/2) dphi/dt, reading R33)."""
    lt = lattice(dr, phys)
    nx, ny = round(phys["Lx"] / dr), round(phys["Ly"] / dr)
    P = phys["perimeter"] / dr             # seed perimeter in cells
    R = P / 6                              # hexagon: circumradius = side
    sx, sy = phys["seed_x"] / dr, phys["seed_y"] / dr
    u_in = Re * W.BASE["nu"] / P
    m = wall_mask(nx, ny, baffle, sx, sy, R)
    p = W.params(dim=2, nx=nx, ny=ny, flow=1, xbc=2 if m is not None else 1, u_in=u_in, U0=phys["U"],
                 U_in=phys["U"], seed_c=(sx, sy, 0.0), seed_R=R, seed_shape=1, seed_tilt=tilt,
                 walls=1 if m is not None else 0, solute_source=int(source))
    p.update(W0=lt["W0"], tau0=lt["tau0"], D=lt["D"])
    h = phys["hours"] if hours is None else hours
    per_hour = round(3600 / lt["dt"])
    return dict(params=p, mask=m, steps=round(h * per_hour), per_hour=per_hour,
                dt=lt["dt"], dr=dr, Re=Re, tilt=tilt, baffle=baffle, u_in=u_in, R=R, source=int(source))


def run(c: dict, precision: str = "fp64", log=None) -> dict:
    """One case on the GPU; the habit numbers every simulated hour (one lbcg_run)."""
    from . import lbcg
    s = lbcg.Solver(c["params"], precision)
    if c["mask"] is not None:
        s.set_walls(c["mask"])
    dirs = habit.habit_directions(c["tilt"])
    t0 = time.perf_counter()
    L, mass = s.run(c["steps"], c["per_hour"], dirs)
    secs = time.perf_counter() - t0
    s.close()
    rows = [habit.from_extents(l) for l in L]
    out = dict(Re=c["Re"], tilt=c["tilt"], baffle=c["baffle"], source=c["source"], u_in=c["u_in"], steps=c["steps"], seconds=secs,
               hours=[(k + 1) * c["per_hour"] * c["dt"] / 3600 for k in range(len(rows))],
               Q=[r["Q"] for r in rows], aspect=[r["aspect"] for r in rows],
               upstream=[r["upstream"] for r in rows],
               L_mm=[(np.asarray(r["L"]) * c["dr"]).tolist() for r in rows],
               L_axes_mm=[(np.asarray(l[6:10]) * c["dr"]).tolist() for l in L],
               Vs=[m["Vs"] for m in mass], L_avg_mm=[r["L_avg"] * c["dr"] for r in rows])
    if log:
        log(f"source {c['source']} Re {c['Re']:5.1f} tilt {math.degrees(c['tilt']):4.1f} {c['baffle']:8s}: Q {out['Q'][-1]:.3f}, "
            f"aspect {out['aspect'][-1]:.3f}, upstream/downstream {out['upstream'][-1]:.3f} after "
            f"{out['hours'][-1]:.1f} h, L_avg {out['L_avg_mm'][-1]:.3f} mm ({secs:.1f} s)")
    return out


SETS = {
    # Reynolds-number effect: no flow, 8.6, 17.2 (tilt 0, no walls)
    "re": [dict(Re=0.0), dict(Re=8.6), dict(Re=17.2)],
    # seed orientation at Re 17.2
    "tilt": [dict(Re=17.2, tilt=math.radians(a)) for a in (0.0, 15.0, 30.0, 45.0)],
    # baffles: the channel without and with three kinds of plates, 2 Re x 2 tilts (16 cases)
    "baffle": [dict(Re=re, tilt=math.radians(t), baffle=b) for re in (8.6, 17.2) for t in (0.0, 30.0)
               for b in ("channel", "plate", "wide", "split")],
}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--sets", nargs="+", default=list(SETS))
    ap.add_argument("--dr", type=float, default=0.025)
    ap.add_argument("--hours", type=float, default=None)
    ap.add_argument("--precision", default="fp64")
    ap.add_argument("--source", type=int, default=0, help="0: full solute source (Eq. (b)), 1: half (R33)")
    ap.add_argument("--out", required=True)
    args = ap.parse_args(argv)
    log = lambda m: print(m, flush=True)
    res = {}
    for name in args.sets:
        res[name] = [run(case(dr=args.dr, hours=args.hours, source=args.source, **kw), args.precision, log)
                     for kw in SETS[name]]
        with open(args.out, "w") as fh:
            json.dump(res, fh)
    return 0


if __name__ == "__main__":
    sys.exit(main())
