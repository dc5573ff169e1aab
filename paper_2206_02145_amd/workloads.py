"""Seeded synthetic workloads: parameter sets and random draws, shared by the GPU path and the
oracle. Holds none of the method's arithmetic; every number here is an input.

Physical parameters follow the paper's Section 4.1.2 (lambda = 3, eps = 0.05,
D = 4.273e-4 mm^2/s, tau0 = 11 s, W0 = 0.05 mm) mapped to lattice units by keeping the
dimensionless diffusivity D tau0 / W0^2 = 1.880 with W0 = 1.5 cells and tau0 = 32 steps.
The viscosity gives Re = u_in P / nu = 17.2 (Section 4.2) for the 3-D flow case with P = 2 pi R.
"""
from __future__ import annotations

import math

import numpy as np

W0 = 1.5
TAU0 = 32.0
D_TILDE = 4.273e-4 * 11.0 / 0.05 ** 2          # D tau0 / W0^2 of the paper's parameters
D_LATTICE = D_TILDE * W0 ** 2 / TAU0            # = 0.1322
NU = 0.02 * 2 * math.pi * 12 / 17.2             # Re 17.2 for u_in 0.02, R 12  -> 0.0877

BASE = dict(W0=W0, tau0=TAU0, lam=3.0, D=D_LATTICE, eps=0.05, nu=NU, h_drag=2.757,
            grad_eps2=1e-12)

SIDES = (64, 96, 128, 192, 256)


def params(**kw) -> dict:
    """A complete parameter dict (keys as in the C structs) with the base physics."""
    p = dict(BASE)
    p.update(dim=2, nx=64, ny=64, nz=1, flow=0, xbc=0, u_in=0.0, U0=0.2, U_in=0.2,
             seed_c=(32.0, 32.0, 0.0), seed_R=8.0)
    p.update(kw)
    p["seed_c"] = tuple(float(v) for v in p["seed_c"])
    return p


def config1() -> dict:
    """2-D 128^2, phase field + solute, no flow, periodic, seed R 8, U0 0.2 (2000 steps)."""
    return params(dim=2, nx=128, ny=128, nz=1, U0=0.2, U_in=0.2, seed_c=(64, 64, 0), seed_R=8.0)


def config2() -> dict:
    """3-D 128^3, D3Q7 phase field + D3Q7 solute, no flow, periodic, seed R 10, U0 0.2 (5000 steps)."""
    return params(dim=3, nx=128, ny=128, nz=128, U0=0.2, U_in=0.2, seed_c=(64, 64, 64),
                  seed_R=10.0)


def config3() -> dict:
    """3-D 192x128x128 with D3Q19 flow, inlet u 0.02 at x-, outlet x+, periodic y/z, seed R 12
    at (64, 64, 64), U0 = U_in = 0.3 (20000 steps)."""
    return params(dim=3, nx=192, ny=128, nz=128, flow=1, xbc=1, u_in=0.02, U0=0.3, U_in=0.3,
                  seed_c=(64, 64, 64), seed_R=12.0)


def config3_reduced() -> dict:
    """The 192x128x128 flow configuration at half size and with a moderate anisotropy: 96x64x64,
    inlet u 0.02 at x-, outlet x+, periodic y/z, seed R 6 at (32, 32, 32), U0 = U_in = 0.3,
    eps 0.02 (where the interface stiffness 1 - 72 eps cos 6 theta is only mildly negative near the
    crystal axes and does not amplify rounding within the run), 20000 steps."""
    return params(dim=3, nx=96, ny=64, nz=64, flow=1, xbc=1, u_in=0.02, U0=0.3, U_in=0.3,
                  seed_c=(32, 32, 32), seed_R=6.0, eps=0.02)


def scaled(p: dict, nx: int, ny: int, nz: int = 1, seed_R: float | None = None) -> dict:
    """The same physics on a smaller grid, the seed kept at the same relative position."""
    q = dict(p)
    q.update(nx=nx, ny=ny, nz=nz)
    c = p["seed_c"]
    q["seed_c"] = (c[0] * nx / p["nx"], c[1] * ny / p["ny"], c[2] * nz / p["nz"] if p["dim"] == 3 else 0.0)
    if seed_R is not None:
        q["seed_R"] = float(seed_R)
    return q


def sweep_draws(n: int = 256, seed: int = 2206):
    """Parameter draws of the batched sweep, in the order (side, U0, R, u_in) per instance:
    side uniform over SIDES, U0 ~ U[0.05, 0.4], R ~ U[4, 16], u_in ~ U[0, 0.03]."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        side = int(rng.choice(SIDES))
        U0 = float(rng.uniform(0.05, 0.4))
        R = float(rng.uniform(4.0, 16.0))
        u_in = float(rng.uniform(0.0, 0.03))
        out.append((side, U0, R, u_in))
    return out


SURROGATE_SIDE = 256  # domain side of the surrogate's training and held-out runs


def surrogate_draws(n: int, seed: int, side: int = SURROGATE_SIDE):
    """Draws of the surrogate's runs: (U0, R, u_in) from the sweep's distributions (sweep_draws with
    the same seed), on a domain of one fixed side length, since the surrogate's four inputs do not
    include it. Tuples (side, U0, R, u_in) as sweep_draws."""
    return [(int(side),) + d[1:] for d in sweep_draws(n, seed)]


def sweep_instance(side: int, U0: float, R: float, u_in: float) -> dict:
    """One 2-D sweep instance: D2Q9 flow with inlet/outlet in x, periodic y, centred seed."""
    return params(dim=2, nx=side, ny=side, nz=1, flow=1, xbc=1, u_in=u_in, U0=U0, U_in=U0,
                  seed_c=(side / 2, side / 2, 0.0), seed_R=R)


def directions(K: int, dim: int = 2, offset: float = 0.0) -> np.ndarray:
    """K unit vectors in the x-y plane at angles offset + 2 pi k / K."""
    a = offset + 2 * math.pi * np.arange(K) / K
    return np.stack([np.cos(a), np.sin(a), np.zeros(K)], axis=1)


def paper_face_normals() -> np.ndarray:
    """Six directions at 30 + 60 k degrees (face normals of a hexagon with vertices on the axes)."""
    return directions(6, offset=math.pi / 6)


def config3_walls():
    """The 192x128x128 flow configuration in a walled cell: a floor (z = 0), a side wall (y = 0)
    and a square baffle plate in front of the seed, normal to the inflow (x = 32, y and z 40 .. 87).
    Returns (params with walls = 1, wall mask [z][y][x] as uint8). A synthetic stand-in for the
    reactor geometry, which the paper shows only in figures."""
    import numpy as np
    p = dict(config3(), walls=1)
    m = np.zeros((p["nz"], p["ny"], p["nx"]), np.uint8)
    m[0, :, :] = 1
    m[:, 0, :] = 1
    m[40:88, 40:88, 32] = 1
    return p, m

