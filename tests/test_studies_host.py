"""Host logic of the studies at the paper's scale (no GPU): the mapping of the paper's physical
parameters to lattice units, the seed sizes, and the synthetic geometry of the baffle study."""
import math

import numpy as np
import pytest

from paper_2206_02145_amd import convergence, growth_study, habit_study
from paper_2206_02145_amd import workloads as W


@pytest.mark.parametrize("dr", [0.04, 0.025, 0.0125])
def test_diffusive_scaling_keeps_the_dimensionless_numbers(dr):
    """At every spacing: W0 = 0.05 mm in cells, D tau0 / W0^2 = 1.880 (the paper's), W0^2 / tau0 the
    same in lattice units, and the physical time step tau0_phys / tau0_lattice."""
    lt = habit_study.lattice(dr)
    assert abs(lt["W0"] - 0.05 / dr) < 1e-12
    assert abs(lt["D"] * lt["tau0"] / lt["W0"] ** 2 - 4.273e-4 * 11.0 / 0.05 ** 2) < 1e-12
    assert abs(lt["W0"] ** 2 / lt["tau0"] - W.BASE["W0"] ** 2 / W.BASE["tau0"]) < 1e-12
    assert abs(lt["dt"] * lt["tau0"] - 11.0) < 1e-9
    lv = convergence.level(dr)
    assert abs(lv["params"]["D"] - lt["D"]) < 1e-12 and abs(lv["dt"] - lt["dt"]) < 1e-12


def test_seed_sizes_from_perimeters():
    """Rhombus of perimeter P: side P/4, circumradius (half the long diagonal) side cos 30;
    hexagon of perimeter P: circumradius = side = P/6."""
    c = growth_study.case(0.06, 6.9)
    assert abs(c["params"]["seed_R"] * 0.025 - 6.9 / 4 * math.cos(math.pi / 6)) < 1e-12
    assert c["params"]["seed_shape"] == 2 and c["params"]["nx"] == 1240 and c["params"]["ny"] == 1040
    h = habit_study.case(17.2)
    assert abs(h["params"]["seed_R"] * 0.025 - 3.7 / 6) < 1e-12 and h["params"]["seed_shape"] == 1
    assert c["steps"] == 12 * c["per_hour"] and h["steps"] == 10 * h["per_hour"]


def test_reynolds_number_sets_the_inflow():
    for Re in (8.6, 17.2):
        c = habit_study.case(Re)
        P = 3.7 / 0.025
        assert abs(c["u_in"] * P / W.BASE["nu"] - Re) < 1e-9
    assert habit_study.case(0.0)["u_in"] == 0.0


@pytest.mark.parametrize("kind", ["none", "channel", "plate", "wide", "split"])
def test_baffle_geometry(kind):
    c = habit_study.case(17.2, baffle=kind, dr=0.04)
    p, m = c["params"], c["mask"]
    if kind == "none":
        assert m is None and p["xbc"] == 1 and p["walls"] == 0
        return
    assert p["xbc"] == 2 and p["walls"] == 1 and m.shape == (1, p["ny"], p["nx"])
    assert m[0, 0].all() and m[0, -1].all()                         # the channel walls
    assert (m[0, :, -2] == m[0, :, -1]).all()                      # the outlet pairing rule
    sx, sy, R = p["seed_c"][0], p["seed_c"][1], c["R"]
    inner = m[0, 1:-1]
    cols = np.nonzero(inner.any(axis=0))[0]
    if kind == "channel":
        assert cols.size == 0
        return
    assert cols.max() < sx - 3 * R                                  # plates upstream of the seed
    rows = np.nonzero(inner.any(axis=1))[0] + 1
    if kind == "split":
        assert not m[0, int(round(sy)), cols].any()                 # the gap in front of the seed
    else:
        assert m[0, int(round(sy)), cols].all()                     # a plate in front of the seed
        half = (rows.max() - rows.min()) / 2
        assert abs(half - (1.5 if kind == "plate" else 3.0) * R) <= 1.0


def test_studies_pass_the_solute_source():
    """Both studies default to the source of Eq. (b) as printed and take the half source (R33)."""
    assert growth_study.case(0.06, 6.9)["params"].get("solute_source", 0) == 0
    assert growth_study.case(0.06, 6.9, source=1)["params"]["solute_source"] == 1
    assert habit_study.case(17.2)["params"].get("solute_source", 0) == 0
    assert habit_study.case(17.2, source=1)["params"]["solute_source"] == 1
    from paper_2206_02145_amd import lbcg
    assert lbcg.make_params(growth_study.case(0.06, 6.9, source=1)["params"], "fp64").solute_source == 1
