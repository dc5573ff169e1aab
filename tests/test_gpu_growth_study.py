"""The no-flow growth-rate study (paper_2206_02145_amd.growth_study) at a reduced scale: 0.04 mm
spacing, 6 simulated hours, binary64 on the GPU. As in the paper's Tables `ss`, `lax` and `ljs`:
at low supersaturation the rhombus's four sides grow well ahead of the two facets forming at its
acute vertices, and the average growth rate rises linearly with the supersaturation."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def runs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2206_02145_amd import growth_study as G
    return {U: G.run(G.case(U, 6.9, dr=0.04, hours=6.0), "fp64", log=lambda m: print(f"[growth] {m}", flush=True))
            for U in (0.06, 0.11, 0.2)}


def test_rhombus_sides_outgrow_the_vertex_facets(runs):
    """At the lowest supersaturation the acute vertices first round off and then grow slowly, well
    behind the four sides (at higher U they catch up in this model)."""
    g = np.array(runs[0.06]["G_normals"])
    sides, vertices = g[[0, 2, 3, 5]], g[[1, 4]]
    assert sides.min() > vertices.max() + 0.5 * sides.mean(), g
    for U, r in runs.items():  # the four sides alike (the rhombus's symmetry)
        s = np.array(r["G_normals"])[[0, 2, 3, 5]]
        assert np.ptp(s) < 0.05 * s.mean(), (U, s)


def test_growth_rate_is_linear_in_supersaturation(runs):
    U = np.array(sorted(runs))
    G = np.array([runs[u]["G_th"] for u in U])
    assert (np.diff(G) > 0).all()
    fit = np.polyfit(U, G, 1)
    resid = G - np.polyval(fit, U)
    assert np.abs(resid).max() < 0.05 * G.max(), (G, fit)
