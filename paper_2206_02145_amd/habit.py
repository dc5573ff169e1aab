"""Crystal-habit diagnostics of the paper's Section 4 from crystal extents along directions.

* L_i, i = 1..6: the normal distances from the crystal centre to its six sides (Section 4.1.2),
  measured as crystal extents along the six face normals of the (tilted) hexagonal habit;
* the quality Q = max L_i / min L_i (the baffle study, Section 4.2), 1 for isotropic growth;
* the aspect ratio: extent along the flow (x) over the extent across it (y),
  (L(+x) + L(-x)) / (L(+y) + L(-y)) (reading of the forced-convection study, whose figure is
  missing);
* the upstream ratio L(-x) / L(+x) with the flow along +x: how much faster the inflow-facing side
  grows than the downstream one.
"""
from __future__ import annotations

import math

import numpy as np


def face_normals(tilt: float = 0.0) -> np.ndarray:
    """The six face normals of a hexagonal habit turned by tilt: tilt + 30 + 60 k degrees."""
    a = tilt + math.pi / 6 + np.arange(6) * math.pi / 3
    return np.stack([np.cos(a), np.sin(a), np.zeros(6)], axis=1)


def habit_directions(tilt: float = 0.0) -> np.ndarray:
    """The directions measure() uses: the six face normals, then +x, -x, +y, -y."""
    axes = np.array([[1.0, 0, 0], [-1.0, 0, 0], [0, 1.0, 0], [0, -1.0, 0]])
    return np.concatenate([face_normals(tilt), axes])


def quality(L6) -> float:
    L6 = np.asarray(L6, dtype=float)
    return float(L6.max() / L6.min())


def aspect_ratio(Lxp: float, Lxm: float, Lyp: float, Lym: float) -> float:
    return float((Lxp + Lxm) / (Lyp + Lym))


def from_extents(L10) -> dict:
    """Habit numbers from the ten extents along habit_directions()."""
    L = np.asarray(L10, dtype=float)
    return dict(L=L[:6], L_avg=float(L[:6].mean()), Q=quality(L[:6]), aspect=aspect_ratio(*L[6:10]),
                upstream=float(L[7] / L[6]))


def measure(solver, tilt: float = 0.0) -> dict:
    """Ray-march the solver's current state along habit_directions(tilt) (one lbcg_measure call)."""
    L, _ = solver.measure(habit_directions(tilt))
    return from_extents(L)
