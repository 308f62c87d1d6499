"""The D3Q19 and coupled pins are discriminating: each test plants one plausible
mistake in the oracle (on the CPU, through monkeypatch, undone afterwards) and
checks that the pin aimed at it fails."""
import importlib.util
import os

import numpy as np
import pytest

from oracle import coupled as CO
from oracle import lbm as L
from oracle import lbm19 as O

HERE = os.path.dirname(os.path.abspath(__file__))


def _pins(name):
    spec = importlib.util.spec_from_file_location(name, os.path.join(HERE, name + ".py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


P19 = _pins("test_oracle_d3q19")
PC = _pins("test_oracle_coupled")


def test_face_always_open_breaks_the_walled_channel(monkeypatch):
    """Mistake: ignore the face-corner reading (R16), so every entering link at
    x = 0 takes the Dirichlet value."""
    real = O.pull_map

    def faces_always_open(prob):
        kind, src = real(prob)
        for i in range(O.Q):
            if O.C19[i][0] == 1:
                kind[i][..., 0] = np.where(prob.active[..., 0], O.ANTI, kind[i][..., 0])
        return kind, src

    monkeypatch.setattr(O, "pull_map", faces_always_open)
    with pytest.raises(AssertionError):
        P19.test_walled_channels_at_tau_one()


def test_wrong_bounce_direction_breaks_the_mirror_symmetry(monkeypatch):
    """Mistake: one edge pair bounces into the wrong edge population.  At tau = 1
    every post-collision population is a_i C, so the link-Laplacian pin cannot see
    it; away from tau = 1 the y mirror can."""
    bad = O.OPP.copy()
    bad[7], bad[8] = O.OPP[8], O.OPP[7]
    monkeypatch.setattr(O, "OPP", bad)
    P19.test_tau1_equals_link_laplacian_random_solids()
    with pytest.raises(AssertionError):
        P19.test_mirror_and_transpose_symmetry()


def test_unweighted_sink_breaks_mass_balance(monkeypatch):
    """Mistake: the sink spread as S/3 on every population instead of a_i S (the
    weak-reaction limit reads R = sum k n C and cannot see how the sink acts; the
    step's mass balance can)."""
    def collide_unweighted(prob, f):
        C = f.sum(axis=0)
        w = O.W19[:, None, None, None]
        fs = f + prob.omega[None] * (w * C[None] - f) + (-prob.kn * C)[None] / 3.0
        return np.where(prob.active[None], fs, 0.0)

    monkeypatch.setattr(O, "collide", collide_unweighted)
    with pytest.raises(AssertionError):
        P19.test_mass_balance_every_step(L.MODE_REACT)


def test_inlet_flux_without_factor_two_breaks_mass_balance(monkeypatch):
    """Mistake: the net inflow of an open face link counted once, not twice."""
    real = O.fluxes

    def half_inflow(prob, f):
        fl = real(prob, f)
        fl.j_in *= 0.5
        return fl

    monkeypatch.setattr(O, "fluxes", half_inflow)
    with pytest.raises(AssertionError):
        P19.test_mass_balance_every_step(L.MODE_REACT)


def test_proton_source_sign_breaks_the_coupled_pins(monkeypatch):
    """Mistake: the proton source enters the potential with the wrong sign, so
    the potential rises away from the membrane."""
    real = O.solve_fixed_point

    def flipped(prob, method="direct"):
        if getattr(prob, "src", None) is not None:
            saved = prob.src
            prob.src = -saved
            try:
                return real(prob, method)
            finally:
                prob.src = saved
        return real(prob, method)

    monkeypatch.setattr(O, "solve_fixed_point", flipped)
    with pytest.raises(AssertionError):
        PC.test_potential_problem_at_tau_one_equals_link_laplacian()
    with pytest.raises(AssertionError):
        ph = PC._structure(4)
        r = CO.solve(ph, L.Params(), CO.Coupling(gamma=2e-3), max_iter=40)
        assert r.phi.max() <= 0.6 + 1e-12
