"""Self-convergence study of the coupled phase-field / solute solver at the paper's scale
(Section 4.1.1): a rhombic seed (perimeter 6.9 mm) in the centre of a fully periodic 31 x 26 mm
domain, U = 0.06, hexagonal anisotropy, 16 hours, at the spatial resolutions 0.04, 0.025, 0.02
and 0.0125 mm (775 x 650 ... 2480 x 2080 nodes). The finest run is the reference of the relative
l2 norm of phi along the centre line from the domain centre 4 mm in +x (the paper's Eq. eew).

The lattice time step follows the diffusive scaling that keeps W0^2 / tau0 and D fixed in lattice
units (the values of the other workloads: W0 = 1.5 cells <-> tau0 = 32 steps), so the physical
step shrinks with the square of the spacing. The profiles are compared at the physical points
15.6, 15.8, ..., 19.4 mm, which are nodes of all four grids.

    python -m paper_2206_02145_amd.convergence --levels 0.04 0.025 0.02 --out conv.json
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import workloads as W

PHYS = dict(Lx=31.0, Ly=26.0, perimeter=6.9, U=0.06, W0=0.05, tau0=11.0, D=4.273e-4, lam=3.0, eps=0.05,
            hours=16.0)
LEVELS_MM = (0.04, 0.025, 0.02, 0.0125)
SAMPLE_MM = 15.6 + 0.2 * np.arange(20)  # x positions (mm) on the centre row, nodes of every level


def level(dr: float, phys: dict = PHYS, hours: float = None) -> dict:
    """Lattice parameters and step count of one resolution dr (mm)."""
    k = W.BASE["W0"] ** 2 / W.BASE["tau0"]      # W0^2 / tau0 in lattice units
    W0c = phys["W0"] / dr                        # interface width in cells
    tau0 = W0c ** 2 / k                          # steps
    dt = phys["tau0"] / tau0                     # seconds per step
    D = phys["D"] * dt / dr ** 2                 # lattice diffusivity
    nx, ny = round(phys["Lx"] / dr), round(phys["Ly"] / dr)
    side = phys["perimeter"] / 4                 # rhombus side (mm); circumradius = side cos 30
    R = side * math.cos(math.pi / 6) / dr
    h = phys["hours"] if hours is None else hours
    steps = round(h * 3600 / dt)
    p = W.params(dim=2, nx=nx, ny=ny, U0=phys["U"], U_in=phys["U"], seed_c=(nx / 2, ny / 2, 0.0), seed_R=R,
                 seed_shape=2, eps=phys["eps"], lam=phys["lam"])
    p.update(W0=W0c, tau0=tau0, D=D)
    return dict(dr=dr, params=p, steps=steps, dt=dt, nodes=nx * ny)


def centre_profile(phi: np.ndarray, dr: float, phys: dict = PHYS) -> np.ndarray:
    """phi at SAMPLE_MM on the row through the domain centre."""
    row = round(phys["Ly"] / 2 / dr)
    cols = np.rint(SAMPLE_MM / dr).astype(int)
    assert np.allclose(cols * dr, SAMPLE_MM) and abs(row * dr - phys["Ly"] / 2) < 1e-9
    return np.asarray(phi)[0, row, cols]


def l2_error(phi: np.ndarray, ref: np.ndarray) -> float:
    """The paper's relative l2 norm, sqrt(sum (phi - phi_ref)^2 / sum phi_ref^2)."""
    return float(np.sqrt(((phi - ref) ** 2).sum() / (ref ** 2).sum()))


def run(dr: float, precision: str = "fp64", hours: float = None, log=None) -> dict:
    """One resolution on the GPU: the centre-line profile, the habit and the timing."""
    import torch

    from . import habit, lbcg
    lv = level(dr, hours=hours)
    s = lbcg.Solver(lv["params"], precision)
    chunk = max(1, lv["steps"] // 20)
    done = 0
    t0 = time.perf_counter()
    while done < lv["steps"]:
        n = min(chunk, lv["steps"] - done)
        s.step(n)
        torch.cuda.synchronize()
        done += n
        if log:
            log(f"dr {dr} mm: {done}/{lv['steps']} steps, {time.perf_counter() - t0:.0f} s")
    secs = time.perf_counter() - t0
    prof = centre_profile(s.read("phi"), dr)
    hb = habit.measure(s)
    s.close()
    return dict(dr=dr, nx=lv["params"]["nx"], ny=lv["params"]["ny"], steps=lv["steps"], dt_s=lv["dt"],
                seconds=secs, glups=lv["nodes"] * lv["steps"] / secs / 1e9, profile=prof.tolist(),
                L_mm=(np.asarray(hb["L"]) * dr).tolist(), Q=hb["Q"], aspect=hb["aspect"])


def orders(results: list) -> dict:
    """Errors of the coarser levels against the finest, and the fitted order of convergence."""
    res = sorted(results, key=lambda r: -r["dr"])
    ref = np.asarray(res[-1]["profile"])
    errs = [(r["dr"], l2_error(np.asarray(r["profile"]), ref)) for r in res[:-1]]
    dr, e = np.log([d for d, _ in errs]), np.log([v for _, v in errs])
    slope = float(np.polyfit(dr, e, 1)[0]) if len(errs) > 1 else float("nan")
    return dict(errors=errs, order=slope)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--levels", type=float, nargs="+", default=list(LEVELS_MM))
    ap.add_argument("--hours", type=float, default=None)
    ap.add_argument("--precision", default="fp64")
    ap.add_argument("--out", required=True)
    args = ap.parse_args(argv)
    log = lambda m: print(m, flush=True)
    out = [run(dr, args.precision, args.hours, log) for dr in args.levels]
    with open(args.out, "w") as fh:
        json.dump(out, fh)
    for r in out:
        log(f"dr {r['dr']}: {r['nx']}x{r['ny']}, {r['steps']} steps, {r['seconds']:.0f} s ({r['glups']:.1f} GLUPS), "
            f"L_avg {np.mean(r['L_mm']):.3f} mm, Q {r['Q']:.3f}")


if __name__ == "__main__":
    sys.exit(main())
