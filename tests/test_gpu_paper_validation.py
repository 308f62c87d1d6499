"""The paper's own code validation (Section 5): the effective diffusivity of a
cube holding an impermeable sphere whose diameter equals the side, 0.3317 on the
paper's D3Q19 lattice at 200^3 (tests/golden/paper_sphere_validation.json).

The D3Q7 solver resolves the same voxel sphere with axis links only, so its
discrete value differs at the curved surface: measured 0.3340 at 64^3, 0.3385 at
128^3 and 0.3408 at 200^3, i.e. within 2.8% of the printed value.  The bound
below is 4%."""
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _sphere(hip, n):
    c = (n - 1) / 2.0
    i = np.arange(n, dtype=np.float64) - c
    d2 = i[:, None, None] ** 2 + i[None, :, None] ** 2 + i[None, None, :] ** 2
    return np.where(d2 <= (n / 2.0) ** 2, hip.CARBON, hip.PORE).astype(np.uint8)


def test_sphere_in_cube_matches_the_papers_validation(hip):
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_sphere_validation.json")) as fh:
        want = json.load(fh)["deff_over_d0"]
    ph = _sphere(hip, 128)
    assert abs((ph == hip.PORE).mean() - (1 - np.pi / 6)) < 2e-3
    s = hip.Solver(ph, hip.lbm_params_default(mode=hip.MODE_DEFF, check_every=1000), voxel_m=1e-9)
    st, info = s.run_to_steady()
    got = s.deff()[1]
    print(f"[sphere] 128^3 D_eff/D0 {got:.5f} against the paper's {want} ({got / want - 1:+.2%}), "
          f"{info.steps} steps", flush=True)
    assert st == 0
    assert abs(got / want - 1) < 0.04


def test_sphere_in_cube_on_d3q19(hip):
    """The same cube on the paper's own lattice: the edge links see the curved
    surface as the paper's code did."""
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_sphere_validation.json")) as fh:
        want = json.load(fh)["deff_over_d0"]
    ph = _sphere(hip, 128)
    s = hip.Solver19(ph, hip.lbm_params_default(mode=hip.MODE_DEFF, check_every=1000), voxel_m=1e-9)
    st, info = s.run_to_steady()
    got = s.deff()[1]
    print(f"[sphere d3q19] 128^3 D_eff/D0 {got:.5f} against the paper's {want} ({got / want - 1:+.2%}), "
          f"{info.steps} steps", flush=True)
    assert st == 0
    assert abs(got / want - 1) < 0.03
