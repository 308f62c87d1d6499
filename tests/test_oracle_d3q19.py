"""Pins of the D3Q19 oracle (Section 4, Eqs. 21-24) against the lattice's
moment conditions, closed forms, an independent steady-state solve at tau = 1,
conservation and symmetry.  CPU only."""
import itertools

import numpy as np
import pytest

import structgen as sg
from oracle import lbm as L
from oracle import lbm19 as O


def _params(**kw):
    p = L.Params()
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def test_velocity_set_and_weights():
    """Eqs. 22-23: 1 rest, 6 face and 12 edge velocities with weights 1/3, 1/18,
    1/36; the moments of an isotropic lattice with c_s^2 = 1/3."""
    c, w = O.C19.astype(float), O.W19
    norms = (c * c).sum(axis=1)
    assert sorted(norms.tolist()) == [0] + [1] * 6 + [2] * 12
    assert len({tuple(v) for v in O.C19}) == 19
    assert np.allclose(w[norms == 0], 1 / 3) and np.allclose(w[norms == 1], 1 / 18)
    assert np.allclose(w[norms == 2], 1 / 36)
    assert w.sum() == pytest.approx(1.0, abs=1e-15)
    for a in range(3):
        assert np.dot(w, c[:, a]) == pytest.approx(0.0, abs=1e-15)
        assert np.dot(w, c[:, a] ** 3) == pytest.approx(0.0, abs=1e-15)
        assert np.dot(w, c[:, a] ** 4) == pytest.approx(1 / 3, abs=1e-15)
        for b in range(3):
            assert np.dot(w, c[:, a] * c[:, b]) == pytest.approx(O.CS2 if a == b else 0.0, abs=1e-15)
            if a != b:
                assert np.dot(w, c[:, a] ** 2 * c[:, b] ** 2) == pytest.approx(1 / 9, abs=1e-15)
    assert (O.C19[O.OPP] == -O.C19).all()


@pytest.mark.parametrize("tau_ref", [0.6, 1.0, 1.7])
def test_empty_box_deff_is_one(tau_ref):
    """Empty box, Dirichlet faces, any tau: D_eff/D0 = 1 and a linear profile."""
    ph = np.zeros((3, 4, 11), np.uint8)
    s = O.solve(ph, _params(tau_ref=tau_ref))
    assert s.deff == pytest.approx(1.0, abs=1e-11)
    assert s.fluxes.j_in == pytest.approx(s.fluxes.j_out, rel=1e-11)
    C = O.concentration(s.f)[0, 0]
    assert np.allclose(C, 1.0 - (np.arange(11) + 0.5) / 11, atol=1e-11)


@pytest.mark.parametrize("tau_ref", [0.7, 1.0, 1.4])
def test_series_slabs_harmonic(tau_ref):
    """Layers normal to x with different D: D_eff = nx / sum(1/D_x) exactly."""
    nx = 12
    ph = np.zeros((2, 3, nx), np.uint8)
    ph[:, :, 4:8] = L.IONOMER
    r = 0.25
    s = O.solve(ph, _params(tau_ref=tau_ref, d_ionomer_rel=r))
    D = np.ones(nx)
    D[4:8] = r
    assert s.deff == pytest.approx(nx / np.sum(1.0 / D), rel=1e-11)


def test_walled_channels_at_tau_one():
    """At tau = 1 the linear profile is exact in a straight channel; each wall-side
    column loses the x flux of the one edge pair that points into the wall (1/36
    of 1/6 per unit gradient): slit (W - 1/3)/N_y, square (W^2 - 2W/3)/(N_y N_z)."""
    slit = np.zeros((3, 8, 9), np.uint8)
    slit[:, [0, 7], :] = L.CARBON
    s = O.solve(slit, _params())
    assert s.deff == pytest.approx((6 - 1 / 3) / 8, rel=1e-11)
    sq = np.full((8, 8, 10), L.CARBON, np.uint8)
    sq[1:7, 1:7, :] = L.PORE
    s = O.solve(sq, _params())
    assert s.deff == pytest.approx((36 - 4) / 64, rel=1e-11)
    C = O.concentration(s.f)
    assert np.allclose(C[3, 1], 1.0 - (np.arange(10) + 0.5) / 10, atol=1e-11)


def _link_laplacian(prob, c_in, c_out, react):
    """Independent steady state at tau = 1: sum over D3Q19 links of a_i (u_n - u)
    between simulated voxels, plus 2 a_i (C_b - u) on each open face link, equals
    u k n / (1 - k n).  A face link entering through x = 0 (or leaving through
    x = nx - 1) is open when the voxel of that plane shifted by the link's y, z
    components is simulated."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla

    act = prob.active
    nz, ny, nx = act.shape
    kn = prob.kn
    idx = -np.ones(act.shape, np.int64)
    idx[act] = np.arange(act.sum())
    n = int(act.sum())
    rows, cols, vals = [], [], []
    rhs = np.zeros(n)
    links = [(cx, cy, cz) for cx, cy, cz in itertools.product((-1, 0, 1), repeat=3)
             if 0 < abs(cx) + abs(cy) + abs(cz) <= 2]
    for z, y, x in zip(*np.nonzero(act)):
        i = idx[z, y, x]
        diag = kn[z, y, x] / (1 - kn[z, y, x])
        for cx, cy, cz in links:
            a = 1 / 18 if abs(cx) + abs(cy) + abs(cz) == 1 else 1 / 36
            tx, ty, tz = x + cx, (y + cy) % ny, (z + cz) % nz
            if tx < 0 or tx >= nx:
                if not act[tz, ty, x] or (tx >= nx and react):
                    continue
                cb = c_in if tx < 0 else c_out
                diag += 2 * a
                rhs[i] += 2 * a * cb
            elif act[tz, ty, tx]:
                diag += a
                rows.append(i)
                cols.append(idx[tz, ty, tx])
                vals.append(-a)
        rows.append(i)
        cols.append(i)
        vals.append(diag)
    u = spla.spsolve(sp.csr_matrix((vals, (rows, cols)), shape=(n, n)).tocsc(), rhs)
    U = np.zeros(act.shape)
    U[act] = u
    return U


def test_tau1_equals_link_laplacian_random_solids():
    rng = np.random.default_rng(5)
    ph = np.where(rng.random((6, 6, 9)) < 0.3, L.CARBON, L.PORE).astype(np.uint8)
    prob = O.prepare(ph, _params())
    assert prob.percolates
    s = O.solve_fixed_point(prob)
    U = _link_laplacian(prob, 1.0, 0.0, False)
    assert np.allclose(O.concentration(s.f), U, atol=1e-12)
    assert s.fluxes.j_in == pytest.approx(s.fluxes.j_out, rel=1e-10)


def test_tau1_with_sink_equals_link_laplacian():
    rng = np.random.default_rng(9)
    ph = np.where(rng.random((5, 6, 8)) < 0.25, L.PT, L.PORE).astype(np.uint8)
    ph[rng.random(ph.shape) < 0.15] = L.IONOMER
    prob = O.prepare(ph, _params(mode=L.MODE_REACT, k_lat=0.03, d_ionomer_rel=1.0))
    s = O.solve_fixed_point(prob)
    U = _link_laplacian(prob, 1.0, 0.0, True)
    assert np.allclose(O.concentration(s.f) * (1 - prob.kn), U, atol=1e-12)
    assert s.fluxes.j_in == pytest.approx(s.fluxes.rate, rel=1e-10)
    assert s.fluxes.j_out == 0.0


@pytest.mark.parametrize("mode", [L.MODE_DEFF, L.MODE_REACT, L.MODE_PROTON])
def test_mass_balance_every_step(mode):
    """Per step, the total of C changes by (J_in - J_out - R) times the area."""
    ph = sg.pt_cl(3, shape=(5, 6, 9))
    p = _params(mode=mode, k_lat=0.05, knudsen=True, voxel_m=2e-9,
                catalyst_phases=(1 << L.PT) | (1 << L.CARBON))
    prob = O.prepare(ph, p)
    rng = np.random.default_rng(1)
    f = rng.random((19,) + prob.active.shape) * prob.active[None]
    A = prob.ny * prob.nz
    for _ in range(3):
        fl = O.fluxes(prob, f)
        g = O.step(prob, f)
        dm = O.concentration(g).sum() - O.concentration(f).sum()
        assert dm == pytest.approx((fl.j_in - fl.j_out - fl.rate) * A, rel=1e-10, abs=1e-12)
        f = g


def test_timestepping_and_direct_solve_agree():
    ph = sg.pt_cl(4, shape=(4, 5, 7))
    prob = O.prepare(ph, _params(tau_ref=0.9))
    d = O.solve_fixed_point(prob)
    t = O.solve_timestep(prob, tol=1e-13)
    assert t.deff == pytest.approx(d.deff, rel=1e-8)


def test_dense_brute_force_tiny():
    rng = np.random.default_rng(2)
    ph = np.where(rng.random((3, 3, 4)) < 0.25, L.CARBON, L.PORE).astype(np.uint8)
    ph[rng.random(ph.shape) < 0.2] = L.IONOMER
    prob = O.prepare(ph, _params(mode=L.MODE_REACT, k_lat=0.04, catalyst_phases=1 << L.CARBON, d_ionomer_rel=0.3))
    a = O.solve_fixed_point(prob, "direct")
    b = O.solve_fixed_point(prob, "dense")
    assert np.allclose(a.f, b.f, atol=1e-13)
    # and the fixed point is one: one more step leaves it in place
    assert np.allclose(O.step(prob, a.f), a.f, atol=1e-13)


def test_mirror_and_transpose_symmetry():
    """The lattice is symmetric under y <-> z and y -> -y: D_eff must be too."""
    rng = np.random.default_rng(11)
    ph = np.where(rng.random((5, 6, 8)) < 0.3, L.CARBON, L.PORE).astype(np.uint8)
    p = _params(tau_ref=0.8)
    base = O.solve(ph, p).deff
    assert O.solve(np.ascontiguousarray(ph.transpose(1, 0, 2)), p).deff == pytest.approx(base, rel=1e-11)
    assert O.solve(np.ascontiguousarray(ph[:, ::-1, :]), p).deff == pytest.approx(base, rel=1e-11)
    # reversing x and swapping the Dirichlet values reverses the flux only
    rev = O.solve(np.ascontiguousarray(ph[:, :, ::-1]), _params(tau_ref=0.8, c_in=0.0, c_out=1.0))
    assert -rev.fluxes.j_vol == pytest.approx(O.solve(ph, p).fluxes.j_vol, rel=1e-11)


def test_weak_reaction_limit():
    """As k -> 0 the layer stays at C_in: R -> k sum(n) C_in / A to first order."""
    ph = sg.pt_cl(6, shape=(5, 6, 8))
    k = 1e-7
    prob = O.prepare(ph, _params(mode=L.MODE_REACT, k_lat=k))
    s = O.solve_fixed_point(prob)
    react = prob.kn > 0
    lim = k * prob.n_cat[react].sum() / (prob.ny * prob.nz)
    assert lim > 0
    assert s.rate == pytest.approx(lim, rel=1e-4)
    assert s.rate < lim


def test_d3q19_differs_from_d3q7_only_off_axis():
    """Where the problem is one-dimensional both lattices agree exactly; on a
    random structure they differ (the edge links see other neighbours)."""
    ph = np.zeros((2, 3, 10), np.uint8)
    ph[:, :, 3:6] = L.IONOMER
    p = _params(tau_ref=0.8, d_ionomer_rel=0.2)
    assert O.solve(ph, p).deff == pytest.approx(L.solve(ph, p).deff, rel=1e-11)
    rng = np.random.default_rng(4)
    ph = np.where(rng.random((5, 5, 8)) < 0.35, L.CARBON, L.PORE).astype(np.uint8)
    a, b = O.solve(ph, p).deff, L.solve(ph, p).deff
    assert a > 0 and b > 0 and abs(a - b) / b > 1e-3
