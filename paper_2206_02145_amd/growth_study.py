"""Growth rates of rhombic seeds without flow at the paper's scale (Sections 4.1.3 and 4.1.4): the
average growth rate G_th against the supersaturation U (0.06 ... 0.2, seed perimeter 6.9 mm) and
against the seed perimeter P (6.9 ... 8.8 mm at U = 0.06), next to the values the paper's own
simulations print (Tables `ljs` and `lax`).

Setting: a periodic 31 x 26 mm box at 0.025 mm (1240 x 1040 nodes) in place of the reactor (shown
only in figures), the seed in its centre, the lattice time step by the diffusive scaling of the
self-convergence study (W0 = 0.05 mm, tau0 = 11 s, D = 4.273e-4 mm^2/s), 12 hours. As in the paper,
L_avg is the mean of the six normal lengths measured every hour and G_th the slope of its linear
fit (lbcg_growth_rates); the per-normal slopes are reported too (the rhombus's four sides and the
two facets forming at its acute vertices).

    python -m paper_2206_02145_amd.growth_study --source 1 --out growth.json
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

PHYS = dict(Lx=31.0, Ly=26.0, W0=0.05, tau0=11.0, D=4.273e-4, hours=12.0)
# average growth rates (mm/h) printed by the paper's simulations
PAPER_G_VS_U = {0.06: 0.057, 0.085: 0.0871, 0.11: 0.1136, 0.15: 0.1553, 0.2: 0.2093}   # Table ljs, P = 6.9 mm
PAPER_G_VS_P = {6.9: 0.0567, 6.96: 0.0575, 8.4: 0.0592, 8.8: 0.0598}                    # Table lax, U = 0.06


def case(U: float, P: float, dr: float = 0.025, hours: float | None = None, phys: dict = PHYS,
         source: int = 0) -> dict:
    """Parameters and step counts of one case: supersaturation U, rhombus perimeter P (mm), solute
    source (0: -dphi/dt as Eq. (b) prints it, 1: -(1/2) dphi/dt, reading R33)."""
    k = W.BASE["W0"] ** 2 / W.BASE["tau0"]
    W0c = phys["W0"] / dr
    tau0 = W0c ** 2 / k
    dt = phys["tau0"] / tau0
    nx, ny = round(phys["Lx"] / dr), round(phys["Ly"] / dr)
    R = (P / 4) * math.cos(math.pi / 6) / dr  # circumradius (half the long diagonal) in cells
    p = W.params(dim=2, nx=nx, ny=ny, U0=U, U_in=U, seed_c=(nx / 2, ny / 2, 0.0), seed_R=R, seed_shape=2)
    p.update(W0=W0c, tau0=tau0, D=phys["D"] * dt / dr ** 2, solute_source=int(source))
    per_hour = round(3600 / dt)
    h = phys["hours"] if hours is None else hours
    return dict(params=p, steps=round(h * per_hour), per_hour=per_hour, dt=dt, dr=dr, U=U, P=P, source=int(source))


def run(c: dict, precision: str = "fp64", log=None) -> dict:
    """One case on the GPU: L along the six normals at t = 0 and every hour, the least-squares
    slopes per normal and of L_avg, in mm/h."""
    from . import lbcg
    s = lbcg.Solver(c["params"], precision)
    dirs = habit.face_normals(0.0)
    t0 = time.perf_counter()
    L0, _ = s.measure(dirs)
    L, _ = s.run(c["steps"], c["per_hour"], dirs)
    G, R2, G_avg = s.growth_rates(6)
    secs = time.perf_counter() - t0
    s.close()
    to_mm_h = c["dr"] / c["dt"] * 3600.0  # cells per step -> mm per hour
    out = dict(U=c["U"], P=c["P"], source=c["source"], steps=c["steps"], seconds=secs, G_th=float(G_avg) * to_mm_h,
               G_normals=(np.asarray(G) * to_mm_h).tolist(), R2=np.asarray(R2).tolist(),
               L_mm=(np.vstack([L0[None], L]) * c["dr"]).tolist())
    if log:
        log(f"source {c['source']} U {c['U']:.3f} P {c['P']:.2f} mm: G_th {out['G_th']:.4f} mm/h, normals "
            + " ".join(f"{g:.4f}" for g in out["G_normals"]) + f" ({secs:.1f} s)")
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--dr", type=float, default=0.025)
    ap.add_argument("--hours", type=float, default=None)
    ap.add_argument("--precision", default="fp64")
    ap.add_argument("--source", type=int, default=0, help="0: full solute source (Eq. (b)), 1: half (R33)")
    ap.add_argument("--out", required=True)
    args = ap.parse_args(argv)
    log = lambda m: print(m, flush=True)
    res = dict(source=args.source, vs_U=[], vs_P=[])
    for U, g in PAPER_G_VS_U.items():
        r = run(case(U, 6.9, args.dr, args.hours, source=args.source), args.precision, log)
        r["paper_G_th"] = g
        res["vs_U"].append(r)
    for P, g in PAPER_G_VS_P.items():
        r = run(case(0.06, P, args.dr, args.hours, source=args.source), args.precision, log)
        r["paper_G_th"] = g
        res["vs_P"].append(r)
    Us = np.array([r["U"] for r in res["vs_U"]])
    Gs = np.array([r["G_th"] for r in res["vs_U"]])
    res["slope_vs_U"] = float(np.polyfit(Us, Gs, 1)[0])
    res["paper_slope_vs_U"] = float(np.polyfit(Us, [r["paper_G_th"] for r in res["vs_U"]], 1)[0])
    log(f"slope of G_th against U: {res['slope_vs_U']:.3f} mm/h (paper's table: {res['paper_slope_vs_U']:.3f})")
    with open(args.out, "w") as fh:
        json.dump(res, fh)
    return 0


if __name__ == "__main__":
    sys.exit(main())
