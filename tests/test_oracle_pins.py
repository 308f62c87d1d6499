"""Pins of the FP64 oracle against things other than itself.

Each test fixes a part of the oracle by a value the paper prints, a closed form,
an exact equivalence with an independent discretisation, an invariant, or a brute
force solve on a tiny grid.  All run on the CPU."""
import json
import math
import os

import numpy as np
import pytest

from oracle import lbm as O
import structgen as sg

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return json.load(fh)


# ------------------------------------------------------------------ printed values

def test_knudsen_bosanquet_worked_example():
    """Section 5.1 worked example: T = 333 K, d_p = 60 nm, D_b as printed."""
    g = _golden("paper_knudsen_example.json")
    D_kn = float(O.knudsen_diffusivity(g["d_p_m"], g["T_K"]))
    assert D_kn == pytest.approx(g["D_kn"], rel=2e-3)
    D = float(O.bosanquet(g["D_b_printed"], D_kn))
    assert D == pytest.approx(g["D_total"], rel=2e-3)


def test_knudsen_constant_identity():
    """Eq. (8): (1/3) sqrt(8 R T / (pi M)) equals 48.5 sqrt(T / 32) (M = 0.032 kg/mol)."""
    for T in (293.2, 333.0, 353.0):
        lhs = float(O.knudsen_diffusivity(1.0, T, 0.032))
        assert lhs == pytest.approx(48.5 * math.sqrt(T / 32.0), rel=1e-4)


def test_bulk_diffusivity_eq7():
    """Eq. (7) as printed.  At 293.2 K, 1 atm it is exactly 0.22e-4.  At 333 K it is
    2.663e-5; the 1.33e-5 printed beside the worked example is a factor 2 off (a
    known inconsistency of the text, kept as a documented reading)."""
    assert O.bulk_diffusivity(293.2, 1.0) == pytest.approx(0.22e-4, rel=1e-15)
    assert O.bulk_diffusivity(333.0, 1.0) == pytest.approx(2.663e-5, rel=1e-3)
    assert O.bulk_diffusivity(333.0, 2.0) == pytest.approx(2.663e-5 / 2, rel=1e-3)
    # Bosanquet limits
    assert float(O.bosanquet(1.0, 1e30)) == pytest.approx(1.0)
    assert float(O.bosanquet(1.0, 1.0)) == pytest.approx(0.5)


def test_volume_fractions_worked_example():
    """Section 2.1.3: eps = 0.4, beta_N = 0.3, theta_Pt = 0.4 -> 38.12 / 1.28 / 20.59 %,
    Pt load 0.11 mg/cm^2 at 4 um (Eqs. 4, 5)."""
    g = _golden("paper_volume_fractions.json")
    eN, eC, ePt = sg.volume_fractions(g["eps"], g["beta_N"], g["theta_Pt"], g["rho_N"], g["rho_C"], g["rho_Pt"])
    assert eC == pytest.approx(g["eps_C"], abs=2e-4)
    assert ePt == pytest.approx(g["eps_Pt"], abs=2e-4)
    assert eN == pytest.approx(g["eps_N"], abs=2e-4)
    assert eN + eC + ePt == pytest.approx(1 - g["eps"], rel=1e-14)
    assert sg.pt_loading(ePt, g["rho_Pt"], g["thickness_cm"]) == pytest.approx(g["gamma_Pt"], abs=5e-3)


# ------------------------------------------------------------------ pore size

def test_chords_slit():
    """A slit of width w normal to x: the x chord is w; in-plane chords are capped at
    one period of the wrapped line; the diagonal chords through the slit are w*sqrt2
    and w*sqrt3 (each diagonal step advances one plane)."""
    nx, ny, nz, w = 9, 5, 5, 3
    pore = np.zeros((nz, ny, nx), bool)
    pore[:, :, 3:3 + w] = True
    dp = O.pore_chords(pore)
    # 13 directions: x (w), y (ny), z (nz), 4 xy/xz diagonals (w sqrt2),
    # 2 yz diagonals (period ny, sqrt2), 4 body diagonals (w sqrt3)
    expect = (w + ny + nz + 4 * w * math.sqrt(2) + 2 * ny * math.sqrt(2) + 4 * w * math.sqrt(3)) / 13
    assert np.allclose(dp[pore], expect, rtol=0, atol=1e-12)
    assert np.all(dp[~pore] == 0)


def test_chords_single_voxel_and_line():
    pore = np.zeros((4, 4, 6), bool)
    pore[1, 2, 3] = True
    dp = O.pore_chords(pore)
    s = (3 + 6 * math.sqrt(2) + 4 * math.sqrt(3)) / 13
    assert dp[1, 2, 3] == pytest.approx(s, abs=1e-14)
    # a straight channel along x, closed in y and z: x chord = nx, others = 1 step
    pore = np.zeros((4, 4, 6), bool)
    pore[1, 2, :] = True
    dp = O.pore_chords(pore)
    assert np.allclose(dp[1, 2, :], (6 + 2 + 6 * math.sqrt(2) + 4 * math.sqrt(3)) / 13)


def test_chords_diagonal_run():
    """A body-diagonal line of pore voxels gives a chord of 4*sqrt3 along (1,1,1)."""
    pore = np.zeros((8, 8, 8), bool)
    for t in range(4):
        pore[2 + t, 2 + t, 2 + t] = True
    dp = O.pore_chords(pore)
    base = 3 + 6 * math.sqrt(2) + 3 * math.sqrt(3)
    assert dp[3, 3, 3] == pytest.approx((base + 4 * math.sqrt(3)) / 13, abs=1e-14)


# ------------------------------------------------------------------ closed forms of the LBM

def _params(**kw):
    p = O.Params()
    for k, v in kw.items():
        setattr(p, k, v)
    return p


@pytest.mark.parametrize("tau_ref", [0.6, 1.0, 1.7])
def test_empty_box_deff_is_one(tau_ref):
    """Empty box, Dirichlet faces, any tau: D_eff/D0 = 1 (L = nx)."""
    ph = np.zeros((3, 4, 11), np.uint8)
    s = O.solve(ph, _params(tau_ref=tau_ref))
    assert s.deff == pytest.approx(1.0, abs=1e-11)
    assert s.fluxes.j_in == pytest.approx(s.fluxes.j_out, rel=1e-11)
    # the profile is linear with the Dirichlet values on the faces
    C = O.concentration(O.prepare(ph, _params(tau_ref=tau_ref)), s.f)[0, 0]
    assert np.allclose(C, 1.0 - (np.arange(11) + 0.5) / 11, atol=1e-11)


@pytest.mark.parametrize("tau_ref", [0.7, 1.0, 1.4])
def test_series_slabs_harmonic(tau_ref):
    """Layers normal to x with different D: D_eff = nx / sum(1/D_x) exactly."""
    nx = 12
    ph = np.zeros((2, 3, nx), np.uint8)
    ph[:, :, 4:8] = O.IONOMER
    r = 0.25
    s = O.solve(ph, _params(tau_ref=tau_ref, d_ionomer_rel=r))
    D = np.where(np.arange(nx) >= 4, 1.0, 1.0)
    D[4:8] = r
    assert s.deff == pytest.approx(nx / np.sum(1.0 / D), rel=1e-11)


@pytest.mark.parametrize("tau_ref", [0.7, 1.0, 1.4])
def test_parallel_slabs_arithmetic(tau_ref):
    """Layers parallel to x (alternating in y): D_eff = mean D exactly."""
    ph = np.zeros((2, 4, 9), np.uint8)
    ph[:, 1, :] = O.IONOMER
    ph[:, 3, :] = O.IONOMER
    r = 0.1
    s = O.solve(ph, _params(tau_ref=tau_ref, d_ionomer_rel=r))
    assert s.deff == pytest.approx((1 + r) / 2, rel=1e-11)


def _fv_solve(active, kn, c_in, c_out, react):
    """Cell-centred 7-point finite volumes for D lap(u) = r u with unit face
    conductance between active cells, conductance 2 to a Dirichlet face (half a
    cell away), zero flux at impermeable faces, periodic y and z; D = 1/8 and
    r = kn / (1 - kn).  Independent of the LBM."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla

    nz, ny, nx = active.shape
    idx = -np.ones(active.shape, np.int64)
    idx[active] = np.arange(active.sum())
    n = int(active.sum())
    rows, cols, vals = [], [], []
    rhs = np.zeros(n)
    D = 0.125
    for z, y, x in zip(*np.nonzero(active)):
        i = idx[z, y, x]
        diag = (kn[z, y, x] / (1 - kn[z, y, x])) / D
        for dz, dy, dx in ((0, 0, 1), (0, 0, -1), (0, 1, 0), (0, -1, 0), (1, 0, 0), (-1, 0, 0)):
            tx = x + dx
            ty, tz = (y + dy) % ny, (z + dz) % nz
            if tx < 0:
                diag += 2
                rhs[i] += 2 * c_in
            elif tx >= nx:
                if not react:
                    diag += 2
                    rhs[i] += 2 * c_out
            elif active[tz, ty, tx]:
                diag += 1
                rows.append(i)
                cols.append(idx[tz, ty, tx])
                vals.append(-1.0)
        rows.append(i)
        cols.append(i)
        vals.append(diag)
    A = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    u = spla.spsolve(A.tocsc(), rhs)
    U = np.zeros(active.shape)
    U[active] = u
    return U


def test_tau1_equals_finite_volume_random_solids():
    """At tau = 1 the D3Q7 steady state equals the 7-point finite-volume solution
    (faces half-way, Dirichlet on the face), for arbitrary bounce-back solids."""
    rng = np.random.default_rng(5)
    ph = np.where(rng.random((6, 6, 10)) < 0.3, O.CARBON, O.PORE).astype(np.uint8)
    prob = O.prepare(ph, _params())
    assert prob.percolates
    s = O.solve_fixed_point(prob)
    C = O.concentration(prob, s.f)
    U = _fv_solve(prob.active, np.zeros(prob.active.shape), 1.0, 0.0, False)
    assert np.allclose(C, U, atol=1e-12)
    # flux through the outlet face of the FV solution
    J = 2 * 0.125 * np.sum((U[:, :, -1] - 0.0) * prob.active[:, :, -1]) / (6 * 6)
    assert s.fluxes.j_out == pytest.approx(J, rel=1e-11)
    assert s.deff == pytest.approx(J * 10 / 0.125, rel=1e-10)


def test_tau1_with_sink_equals_finite_volume():
    """At tau = 1 with a first-order sink, u = (1 - k n) C obeys the 7-point finite
    volumes with rate k n / (1 - k n); the reaction rate equals the inlet flux."""
    rng = np.random.default_rng(9)
    ph = np.where(rng.random((5, 6, 9)) < 0.25, O.PT, O.PORE).astype(np.uint8)
    ph[rng.random(ph.shape) < 0.15] = O.IONOMER
    p = _params(mode=O.MODE_REACT, k_lat=0.03, d_ionomer_rel=1.0)
    prob = O.prepare(ph, p)
    s = O.solve_fixed_point(prob)
    C = O.concentration(prob, s.f)
    U = _fv_solve(prob.active, prob.kn, 1.0, 0.0, True)
    assert np.allclose(C * (1 - prob.kn), U, atol=1e-12)
    assert s.fluxes.j_in == pytest.approx(s.fluxes.rate, rel=1e-11)
    assert s.fluxes.j_out == 0.0


@pytest.mark.parametrize("N,k", [(16, 0.002), (32, 0.002), (40, 0.01)])
def test_reactive_channel_cosh(N, k):
    """1-D channel: a fluid row between catalyst rows (n = 2), tau = 1, Dirichlet
    inlet face, zero-gradient outlet.  Discrete closed form
    u_x = A cosh(theta (N - 1/2 - x)), cosh(theta) = 1 + kappa/(2D), kappa = 2k/(1-2k),
    D = 1/8, A = 2 C_in / (cosh theta(N+1/2) + cosh theta(N-1/2)), C = u / (1 - 2k).
    The continuum profile cosh(m (L - x)) / cosh(m L) agrees to O(h^2) + O(k)."""
    ph = np.full((1, 2, N), O.PT, np.uint8)
    ph[0, 0, :] = O.PORE
    p = _params(mode=O.MODE_REACT, k_lat=k, reservoir_plane=False)
    prob = O.prepare(ph, p)
    s = O.solve_fixed_point(prob)
    C = O.concentration(prob, s.f)[0, 0]
    kappa = 2 * k / (1 - 2 * k)
    th = math.acosh(1 + kappa / (2 * 0.125))
    A = 2.0 / (math.cosh(th * (N + 0.5)) + math.cosh(th * (N - 0.5)))
    x = np.arange(N)
    u = A * np.cosh(th * (N - 0.5 - x))
    assert np.allclose(C * (1 - 2 * k), u, rtol=1e-12, atol=1e-14)
    m = math.sqrt(kappa / 0.125)
    cont = np.cosh(m * (N - (x + 0.5))) / np.cosh(m * N)
    assert np.max(np.abs(C - cont)) < 5 * (m * m + k)


@pytest.mark.parametrize("mode", [O.MODE_DEFF, O.MODE_REACT, O.MODE_PROTON])
def test_mass_balance_every_step(mode):
    """Per step, total mass changes by J_in - J_out - R exactly (FP64)."""
    ph = sg.pt_cl(3, shape=(6, 7, 12))
    p = _params(mode=mode, k_lat=0.05, knudsen=True, voxel_m=2e-9, catalyst_phases=(1 << O.PT) | (1 << O.CARBON))
    prob = O.prepare(ph, p)
    rng = np.random.default_rng(1)
    f = rng.random((7, prob.N)) * prob.active.ravel()[None, :]
    f = np.ascontiguousarray(f)
    for _ in range(3):
        fl = O.fluxes(prob, f)
        f2 = O.step(prob, f)
        A = prob.ny * prob.nz
        dM = O.fluxes(prob, f2).mass - fl.mass
        assert dM == pytest.approx((fl.j_in - fl.j_out - fl.rate) * A, rel=1e-11, abs=1e-11)
        f = f2


def test_uniform_state_is_fixed_point():
    """With C_in = C_out = c and no sink, f_i = w_i c is a fixed point for any
    structure and any tau field (equilibrium is preserved by bounce-back)."""
    ph = sg.pt_cl(4, shape=(6, 6, 10))
    p = _params(c_in=0.7, c_out=0.7, knudsen=True)
    prob = O.prepare(ph, p)
    f = O.equilibrium(prob, 0.7)
    assert np.allclose(O.step(prob, f), f, atol=1e-15)


def test_timestepping_and_direct_solve_agree():
    """Two routes to the steady state on a heterogeneous-tau structure."""
    ph = sg.pt_cl(8, shape=(5, 6, 10))
    p = _params(knudsen=True, voxel_m=2e-9, d_ionomer_rel=0.05)
    prob = O.prepare(ph, p)
    assert prob.percolates
    a = O.solve_fixed_point(prob)
    b = O.solve_timestep(prob, tol=1e-14, check_every=50)
    assert b.deff == pytest.approx(a.deff, rel=1e-9)
    c = O.solve_fixed_point(prob, method="bicgstab", tol=1e-13)
    assert c.deff == pytest.approx(a.deff, rel=1e-9)


def test_dense_brute_force_tiny():
    """A dense LU solve of the whole 7N system on a tiny grid agrees with the sparse route."""
    ph = sg.pt_cl(11, shape=(3, 3, 4))
    for mode in (O.MODE_DEFF, O.MODE_REACT):
        p = _params(mode=mode, knudsen=True, k_lat=0.05)
        prob = O.prepare(ph, p)
        a = O.solve_fixed_point(prob, "direct")
        b = O.solve_fixed_point(prob, "dense")
        assert np.allclose(a.f, b.f, atol=1e-12)


def test_dead_pockets_do_not_matter():
    """A sealed pore cavity is excluded and leaves the result unchanged."""
    ph = np.zeros((6, 6, 10), np.uint8)
    ph[1:5, 1:5, 3:8] = O.CARBON
    base = O.solve(ph, _params(tau_ref=0.8))
    ph2 = ph.copy()
    ph2[2:4, 2:4, 4:6] = O.PORE  # sealed inside the carbon block
    prob = O.prepare(ph2, _params(tau_ref=0.8))
    assert not prob.active[2:4, 2:4, 4:6].any()
    s = O.solve(ph2, _params(tau_ref=0.8))
    assert s.deff == pytest.approx(base.deff, rel=1e-12)


def test_mirror_and_transpose_symmetry():
    """Mirroring y or swapping y and z leaves D_eff unchanged (catches index slips)."""
    ph = sg.pt_cl(13, shape=(6, 6, 9))
    p = _params(knudsen=True)
    d = O.solve(ph, p).deff
    assert O.solve(ph[:, ::-1, :].copy(), p).deff == pytest.approx(d, rel=1e-10)
    assert O.solve(np.ascontiguousarray(ph.transpose(1, 0, 2)), p).deff == pytest.approx(d, rel=1e-10)
    # reversing x and swapping inlet/outlet values gives the same flux magnitude
    q = _params(knudsen=True, c_in=0.0, c_out=1.0)
    s = O.solve(ph[:, :, ::-1].copy(), q)
    assert s.deff == pytest.approx(d, rel=1e-10)


def test_proton_mode_parallel_ionomer():
    """Proton conduction on ionomer only: sigma_eff/sigma = ionomer area fraction for
    straight ionomer sheets along x."""
    ph = np.zeros((3, 5, 8), np.uint8)
    ph[:, 1, :] = O.IONOMER
    ph[:, 3, :] = O.IONOMER
    ph[:, 2, :] = O.CARBON
    s = O.solve(ph, _params(mode=O.MODE_PROTON))
    assert s.deff == pytest.approx(2 / 5, rel=1e-11)


def test_no_percolation_gives_zero():
    ph = np.zeros((3, 3, 8), np.uint8)
    ph[:, :, 4] = O.CARBON
    prob = O.prepare(ph, _params())
    assert not prob.percolates
    assert O.solve(ph, _params()).deff == 0.0


def test_step_is_linear_in_boundary_data():
    """Doubling C_in and C_out doubles the steady state (no sink): D_eff unchanged."""
    ph = sg.pt_cl(17, shape=(4, 5, 8))
    a = O.solve(ph, _params(knudsen=True))
    b = O.solve(ph, _params(knudsen=True, c_in=2.0, c_out=0.0))
    assert b.deff == pytest.approx(a.deff, rel=1e-12)
    assert np.allclose(b.f, 2 * a.f, atol=1e-13)


# ------------------------------------------------------------------ per-voxel Knudsen mapping

def _slit_and_line(nx=16, ny=8, nz=6):
    """Carbon with two straight pore channels along x, neither touching the other:
    a slit one voxel thick in y spanning every z (y = 1), and a 1 x 1 line
    (y = 4, z = 2).  Every diagonal run with a y or z step leaves a channel after
    one voxel, so the pore size is uniform along each channel, x faces included."""
    ph = np.full((nz, ny, nx), O.CARBON, np.uint8)
    ph[:, 1, :] = O.PORE
    ph[2, 4, :] = O.PORE
    return ph


def _hand_dp(nx, ny, nz):
    """Section 2.1.3 by hand, in voxel edges: the mean over the 13 directions of the
    pore run through a voxel times |d|.
    Slit (thickness 1 in y, all of z): x -> nx, y -> 1, z -> nz (one period),
    (1,+-1,0) -> 1 x sqrt2, (1,0,+-1) -> nx x sqrt2 (z wraps, x stops at the faces),
    (0,1,+-1) -> 1 x sqrt2, the four body diagonals -> 1 x sqrt3.
    Line (1 x 1): x -> nx, every other direction -> one voxel."""
    r2, r3 = math.sqrt(2.0), math.sqrt(3.0)
    slit = (nx + 1 + nz + r2 * (1 + 1 + nx + nx + 1 + 1) + 4 * r3) / 13.0
    line = (nx + 1 + 1 + 6 * r2 + 4 * r3) / 13.0
    return slit, line


@pytest.mark.parametrize("voxel_m", [2e-9, 1e-9])
def test_knudsen_mapping_of_straight_channels(voxel_m):
    """Knudsen diffusivity per voxel, end to end: d_p by hand (Section 2.1.3), D_Kn of
    d_p * voxel edge (Eq. 8, T = 353 K, M = 0.032), Bosanquet with D_b (Eqs. 7, 9),
    tau from D / D_ref with D_ref the larger channel's D (Eq. 24), and the exact
    steady state of straight channels: D_eff/D0 = sum over channels of (area / A) D/D_b
    (anti-bounce-back faces make the linear profile exact at any tau)."""
    nx, ny, nz = 16, 8, 6
    ph = _slit_and_line(nx, ny, nz)
    T = 353.0
    prob = O.prepare(ph, _params(knudsen=True, voxel_m=voxel_m, T_K=T))
    dp_slit, dp_line = _hand_dp(nx, ny, nz)
    assert np.allclose(prob.d_p[:, 1, :], dp_slit, rtol=0, atol=1e-12)
    assert np.allclose(prob.d_p[2, 4, :], dp_line, rtol=0, atol=1e-12)
    # Eqs. 7-9 written out: D_b, D_Kn = (d / 3) sqrt(8 R T / (pi M)), 1/D = 1/D_b + 1/D_Kn
    D_b = 0.22e-4 * (T / 293.2) ** 1.5
    vbar = math.sqrt(8 * 8.314 * T / (math.pi * 0.032))
    D = [1.0 / (1.0 / D_b + 3.0 / (d * voxel_m * vbar)) for d in (dp_slit, dp_line)]
    assert D[0] > D[1]
    assert np.allclose(prob.D[:, 1, :], D[0], rtol=1e-13)
    assert np.allclose(prob.D[2, 4, :], D[1], rtol=1e-13)
    # tau_ref = 1 goes to the largest diffusivity (the slit); the line scales with it
    assert np.allclose(prob.tau[:, 1, :], 1.0, rtol=0, atol=1e-14)
    assert np.allclose(prob.tau[2, 4, :], 0.5 + 0.5 * D[1] / D[0], rtol=0, atol=1e-14)
    s = O.solve_fixed_point(prob)
    want = (nz * D[0] + 1 * D[1]) / (ny * nz) / D_b
    assert s.deff == pytest.approx(want, rel=1e-11)
    # Knudsen matters here: without it the same structure gives the open-area fraction
    s0 = O.solve(ph, _params(knudsen=False))
    assert s0.deff == pytest.approx((nz + 1) / (ny * nz), rel=1e-11)
    assert want < 0.5 * s0.deff


# ------------------------------------------------------------------ catalyst face neighbours

def test_catalyst_neighbour_count_hand_built():
    """n(x) of Eq. 18a: catalyst face neighbours, periodic in y and z, nothing
    beyond the x faces.  Counted by hand on a built map."""
    nz, ny, nx = 4, 5, 6
    ph = np.zeros((nz, ny, nx), np.uint8)
    # corner voxel (z, y, x) = (0, 0, 0): Pt at x + 1 (counts), across the y wrap
    # (y = 4) and across the z wrap (z = 3) (both count), and at x = 5 of its own
    # row (does not count: x is not periodic)
    ph[0, 0, 1] = O.PT
    ph[0, 4, 0] = O.PT
    ph[3, 0, 0] = O.PT
    ph[0, 0, 5] = O.PT
    # voxel (2, 2, 3): catalyst on all six faces, carbon on three of them
    for dz, dy, dx, phase in ((1, 0, 0, O.PT), (-1, 0, 0, O.CARBON), (0, 1, 0, O.PT), (0, -1, 0, O.CARBON),
                              (0, 0, 1, O.PT), (0, 0, -1, O.CARBON)):
        ph[2 + dz, 2 + dy, 3 + dx] = phase
    # voxel (1, 3, 5) on the outlet face: Pt at x = 0 of its row must not count,
    # Pt at x = 4 counts
    ph[1, 3, 0] = O.PT
    ph[1, 3, 4] = O.PT
    pt_only = O.catalyst_neighbours(ph, 1 << O.PT)
    pt_carbon = O.catalyst_neighbours(ph, (1 << O.PT) | (1 << O.CARBON))
    assert pt_only[0, 0, 0] == 3
    assert pt_only[2, 2, 3] == 3 and pt_carbon[2, 2, 3] == 6
    assert pt_only[1, 3, 5] == 1
    # the row-end Pt at x = 5 of row (0, 0) sees the voxel at x = 4 only
    assert pt_only[0, 0, 4] == 1
    # brute force over every voxel: count the six face neighbours one by one
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                n = 0
                for dz, dy, dx in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
                    xx = x + dx
                    if xx < 0 or xx >= nx:
                        continue
                    n += ph[(z + dz) % nz, (y + dy) % ny, xx] == O.PT
                assert pt_only[z, y, x] == n, (z, y, x)
    # the sink of the reactive problem is k n on reactive fluid voxels only
    prob = O.prepare(ph, _params(mode=O.MODE_REACT, k_lat=0.01, reservoir_plane=False))
    assert prob.kn[0, 0, 0] == pytest.approx(0.03, rel=1e-15)
    assert prob.kn[0, 0, 1] == 0.0  # a Pt voxel does not react itself


@pytest.mark.parametrize("N,k", [(24, 0.004)])
def test_reactive_channel_cosh_along_z_neighbours(N, k):
    """The cosh channel with its catalyst neighbours across the z wrap instead of y:
    a pore row at z = 0 of a (2, 1, N) map whose other plane is Pt has n = 2 (z = 1
    and, through the wrap, z = -1), and ny = 1 makes its y neighbours itself."""
    ph = np.full((2, 1, N), O.PT, np.uint8)
    ph[0, 0, :] = O.PORE
    prob = O.prepare(ph, _params(mode=O.MODE_REACT, k_lat=k, reservoir_plane=False))
    assert (prob.n_cat[0, 0] == 2).all()
    s = O.solve_fixed_point(prob)
    C = O.concentration(prob, s.f)[0, 0]
    kappa = 2 * k / (1 - 2 * k)
    th = math.acosh(1 + kappa / (2 * 0.125))
    A = 2.0 / (math.cosh(th * (N + 0.5)) + math.cosh(th * (N - 0.5)))
    u = A * np.cosh(th * (N - 0.5 - np.arange(N)))
    assert np.allclose(C * (1 - 2 * k), u, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("mode,k", [(O.MODE_DEFF, 0.0), (O.MODE_REACT, 1e-2)])
def test_preconditioned_gmres_route_agrees_with_sparse_lu(mode, k):
    """The Krylov route used for the stored fixed points of large catalyst layers
    (GMRES with an incomplete-LU preconditioner, certified by one plain step) gives
    the sparse direct solve's answer on a four-phase Knudsen layer."""
    ph = sg.pt_cl(8, shape=(8, 10, 20))
    prob = O.prepare(ph, _params(mode=mode, knudsen=True, voxel_m=2e-9, k_lat=k))
    a = O.solve_fixed_point(prob, "direct")
    b = O.solve_fixed_point(prob, "gmres")
    assert np.abs(b.f - a.f).max() < 1e-12
    if mode == O.MODE_DEFF:
        assert b.deff == pytest.approx(a.deff, rel=1e-11)
    else:
        assert b.rate == pytest.approx(a.rate, rel=1e-11)
