"""Parity of the coupled oxygen / proton-potential solve on the device
(lbm19_coupled_* through the C ABI) with the coupled oracle (Eqs. 15-18b).

The oracle iterates exact FP64 fixed points to a potential change of 1e-10 V;
the device iterates FP32 solvers stopped at a relative output change of 1e-7 to
a potential change of 1e-6 V.  Outputs must agree to 1e-4 relative and the
potential to 1e-4 of the largest drop.  The potential's inner solve runs both
ways: conjugate gradients on the link Laplacian that the tau_phi = 1 lattice's
steady state equals (the default), and stepping the potential lattice."""
import json
import os

import numpy as np
import pytest

import structgen as sg
from oracle import coupled as CO
from oracle import lbm as L

pytestmark = pytest.mark.gpu


def _structure(seed, shape):
    ph = sg.pt_cl(seed, shape=shape)
    skin = ph[:, :, -1]
    skin[skin == L.PORE] = L.IONOMER      # ionomer meets the membrane face
    return ph


CASES = [(4, (6, 8, 12), 2e-3, 0), (4, (6, 8, 12), 2e-3, 1), (4, (6, 8, 12), 2e-2, 0), (3, (8, 10, 16), 5e-3, 0),
         (3, (8, 10, 16), 5e-3, 1)]


@pytest.mark.parametrize("seed,shape,gamma,solver", CASES)
def test_coupled_solve_matches_oracle(hip, seed, shape, gamma, solver):
    ph = _structure(seed, shape)
    print(f"[coupled] seed {seed} {shape} gamma {gamma} potential solver {solver}", flush=True)
    ref = CO.solve(ph, L.Params(), CO.Coupling(gamma=gamma))
    p = hip.lbm_params_default(mode=hip.MODE_REACT, check_every=100, tol_flux=1e-7, max_steps=4_000_000)
    c = hip.Coupled19(ph, p, hip.lbm_coupling_default(gamma=gamma, potential_solver=solver))
    st, info = c.run()
    if solver == 0:
        assert info.phi_cg_iterations > 0 and info.phi_steps <= 1
    else:
        assert info.phi_cg_iterations == 0 and info.phi_steps > 1000
    _, phi = c.fields()
    phi = phi.cpu().numpy().astype(np.float64)
    drop = 0.6 - ref.phi.min()
    print(f"  {info.iterations} iterations (oracle {ref.iterations}); rate {info.rate:.8g} vs {ref.rate:.8g}; "
          f"membrane current {info.proton_in:.8g} vs {ref.proton_in:.8g}; max |dphi| "
          f"{np.abs(phi - ref.phi).max():.2e} V of a {drop:.3f} V drop", flush=True)
    assert st == 0, info.as_dict()
    assert info.rate == pytest.approx(ref.rate, rel=1e-4)
    assert info.proton_in == pytest.approx(ref.proton_in, rel=1e-4)
    assert info.source == pytest.approx(gamma / 1e-2 * info.rate, rel=1e-4)
    assert np.abs(phi - ref.phi).max() < 1e-4 * max(drop, 1e-3)
    assert info.phi_min == pytest.approx(ref.phi.min(), abs=1e-4 * max(drop, 1e-3))


def test_coupled_solve_at_16_matches_the_stored_oracle_fixed_point(hip):
    """A 16^3 layer (tests/golden/oracle_coupled_16.json: the coupled oracle, 45
    Picard iterations of exact D3Q19 fixed points, minutes of CPU) with the
    default conjugate-gradient potential solve."""
    with open(os.path.join(os.path.dirname(__file__), "golden", "oracle_coupled_16.json")) as fh:
        g = json.load(fh)["cases"][0]
    ph = _structure(g["seed"], tuple(g["shape"]))
    p = hip.lbm_params_default(mode=hip.MODE_REACT, check_every=100, tol_flux=1e-7, max_steps=4_000_000)
    c = hip.Coupled19(ph, p, hip.lbm_coupling_default(gamma=g["gamma"]))
    st, info = c.run()
    _, phi = c.fields()
    phi = phi.cpu().numpy().astype(np.float64).ravel()
    ref_phi = np.asarray(g["phi"])
    drop = 0.6 - g["phi_min"]
    print(f"[coupled] 16^3: {info.iterations} iterations, {info.phi_cg_iterations} CG iterations; rate "
          f"{info.rate:.8g} vs {g['rate']:.8g}; current {info.proton_in:.8g} vs {g['proton_in']:.8g}; "
          f"max |dphi| {np.abs(phi - ref_phi).max():.2e} V of {drop:.3f} V", flush=True)
    assert st == 0, info.as_dict()
    assert info.rate == pytest.approx(g["rate"], rel=1e-4)
    assert info.proton_in == pytest.approx(g["proton_in"], rel=1e-4)
    assert np.abs(phi - ref_phi).max() < 1e-4 * drop
