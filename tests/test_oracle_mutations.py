"""The oracle's pins are discriminating: each test plants one plausible mistake
in the oracle (on the CPU, through monkeypatch, undone afterwards) and checks that
the pin aimed at it fails.  Mistakes in the D3Q7 oracle's plain C are planted in a
copy of its source, compiled to a temporary library that replaces the real one for
the duration of the test."""
import importlib.util
import math
import os
import subprocess

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
P7 = _pins("test_oracle_pins")


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


# ---------------------------------------------------------------- the D3Q7 oracle


def _mutated_c(monkeypatch, tmp_path, old, new, count=1):
    """Compile lbm_ref.c with `old` replaced by `new` (exactly `count` times) and make
    the oracle load that library until the test ends."""
    src = open(os.path.join(os.path.dirname(L.__file__), "lbm_ref.c")).read()
    assert src.count(old) == count, (old, src.count(old))
    path = tmp_path / "lbm_ref_mut.c"
    path.write_text(src.replace(old, new))
    so = tmp_path / "liblbm_ref_mut.so"
    subprocess.run(["gcc", "-O1", "-std=c99", "-fopenmp", "-fPIC", "-shared", str(path), "-o", str(so), "-lm"],
                   check=True)
    monkeypatch.setattr(L, "_LIB_PATH", str(so))
    monkeypatch.setattr(L, "_lib", None)


def test_knudsen_without_voxel_size_breaks_the_channel_pin(monkeypatch):
    """Mistake: the pore size passed to Eq. 8 in voxel edges instead of metres (the
    voxel edge dropped), so D_Kn is ~1e9 times too large and D_pore ~ D_b."""
    real = L.knudsen_diffusivity
    monkeypatch.setattr(L, "knudsen_diffusivity", lambda d, T, M=0.032: real(np.asarray(d) / 2e-9, T, M))
    with pytest.raises(AssertionError):
        P7.test_knudsen_mapping_of_straight_channels(2e-9)


def test_chords_without_direction_lengths_break_the_channel_pin(monkeypatch, tmp_path):
    """Mistake: chords counted in voxels along every direction (|d| = 1 for the face
    and body diagonals too)."""
    _mutated_c(monkeypatch, tmp_path, "sum += (double)count * sqrt((double)(dx * dx + dy * dy + dz * dz));",
               "sum += (double)count;")
    with pytest.raises(AssertionError):
        P7.test_knudsen_mapping_of_straight_channels(2e-9)


def test_periodic_x_neighbours_break_the_neighbour_count(monkeypatch):
    """Mistake: catalyst neighbours counted with a periodic wrap along x as well."""
    def wrapped(phase, catalyst_mask):
        cat = ((catalyst_mask >> phase.astype(np.int64)) & 1).astype(np.int64)
        n = np.zeros(phase.shape, dtype=np.int64)
        for ax in (0, 1, 2):
            n += np.roll(cat, 1, axis=ax) + np.roll(cat, -1, axis=ax)
        return n

    monkeypatch.setattr(L, "catalyst_neighbours", wrapped)
    with pytest.raises(AssertionError):
        P7.test_catalyst_neighbour_count_hand_built()


def _mutated_c2(monkeypatch, tmp_path, pairs):
    src = open(os.path.join(os.path.dirname(L.__file__), "lbm_ref.c")).read()
    for old, new in pairs:
        assert src.count(old) == 1, old
        src = src.replace(old, new)
    path = tmp_path / "lbm_ref_mut.c"
    path.write_text(src)
    so = tmp_path / "liblbm_ref_mut.so"
    subprocess.run(["gcc", "-O1", "-std=c99", "-fopenmp", "-fPIC", "-shared", str(path), "-o", str(so), "-lm"],
                   check=True)
    monkeypatch.setattr(L, "_LIB_PATH", str(so))
    monkeypatch.setattr(L, "_lib", None)


def test_unweighted_d3q7_sink_breaks_the_cosh_channel(monkeypatch, tmp_path):
    """Mistake: the sink added as S/7 to every population instead of w_i S, in the
    step and in the assembled fixed-point system alike.  The total sink is the same
    (mass balance cannot see it); the discrete cosh profile can."""
    _mutated_c2(monkeypatch, tmp_path, [("+ w * S;", "+ S / 7.0;"),
                                        ("(om - kn) * w;", "om * w - kn / 7.0;")])
    P7.test_mass_balance_every_step(L.MODE_REACT)
    with pytest.raises(AssertionError):
        P7.test_reactive_channel_cosh(32, 0.002)


def test_single_weight_dirichlet_breaks_the_empty_box(monkeypatch, tmp_path):
    """Mistake: anti-bounce-back with w C_in instead of 2 w C_in at the inlet face
    (in the step and in the assembled fixed-point system alike)."""
    _mutated_c(monkeypatch, tmp_path, "2.0 * w * g->c_in", "w * g->c_in", count=2)
    with pytest.raises(AssertionError):
        P7.test_empty_box_deff_is_one(1.0)


def test_wrong_bounce_back_direction_breaks_the_finite_volume_pin(monkeypatch, tmp_path):
    """Mistake: populations moving in y bounce back into themselves instead of into
    the opposite direction."""
    _mutated_c(monkeypatch, tmp_path, "static const int OPP[7] = {0, 2, 1, 4, 3, 6, 5};",
               "static const int OPP[7] = {0, 2, 1, 3, 4, 6, 5};")
    P7.test_tau1_equals_finite_volume_random_solids()  # at tau = 1 only C matters
    with pytest.raises(AssertionError):
        P7.test_mirror_and_transpose_symmetry()
