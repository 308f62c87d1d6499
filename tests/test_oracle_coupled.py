"""Pins of the coupled oxygen / proton-potential oracle (Eqs. 15-18b on D3Q19):
conservation and stoichiometry, an independent steady-state solve of the
potential problem at tau = 1, the limit of no proton source, and invariants of
the iteration.  CPU only."""
import itertools

import numpy as np
import pytest

import structgen as sg
from oracle import coupled as CO
from oracle import lbm as L
from oracle import lbm19 as O


def _structure(seed, shape=(6, 8, 12)):
    ph = sg.pt_cl(seed, shape=shape)
    skin = ph[:, :, -1]
    skin[skin == L.PORE] = L.IONOMER      # ionomer meets the membrane face
    return ph


def _link_laplacian_with_source(prob, q, phi_m):
    """Independent steady state of the potential problem at tau = 1: sum over
    D3Q19 links of a_i (u_n - u) between simulated voxels, plus 2 a_i (phi_m - u)
    on each open link of the membrane face, equals q; zero flux elsewhere."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla

    act = prob.active
    nz, ny, nx = act.shape
    idx = -np.ones(act.shape, np.int64)
    idx[act] = np.arange(act.sum())
    n = int(act.sum())
    rows, cols, vals = [], [], []
    rhs = np.zeros(n)
    links = [c for c in itertools.product((-1, 0, 1), repeat=3) if 0 < sum(map(abs, c)) <= 2]
    for z, y, x in zip(*np.nonzero(act)):
        i = idx[z, y, x]
        diag = 0.0
        rhs[i] -= q[z, y, x]
        for cx, cy, cz in links:
            a = 1 / 18 if abs(cx) + abs(cy) + abs(cz) == 1 else 1 / 36
            tx, ty, tz = x + cx, (y + cy) % ny, (z + cz) % nz
            if tx >= nx:
                if act[tz, ty, x]:
                    diag += 2 * a
                    rhs[i] += 2 * a * phi_m
            elif tx >= 0 and act[tz, ty, tx]:
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


def test_potential_problem_at_tau_one_equals_link_laplacian():
    """With a given source q, the post-collision value u = phi + S (S = -q) obeys
    the link Laplacian with zero flux at x = 0 and phi_m at the membrane face."""
    ph = _structure(3)
    cp = CO.Coupling()
    pp = CO.phi_problem(ph, cp)
    assert pp.active.sum() > 80
    rng = np.random.default_rng(0)
    q = np.where(pp.active, rng.random(ph.shape) * 1e-3, 0.0)
    pp.src = -q
    s = O.solve_fixed_point(pp)
    phi = O.concentration(s.f)
    U = _link_laplacian_with_source(pp, q, cp.phi_m)
    assert np.allclose(np.where(pp.active, phi + pp.src, 0.0), U, atol=1e-12)
    # the current entering through the membrane face is the total source
    assert -s.fluxes.j_out == pytest.approx(q.sum() / (pp.ny * pp.nz), rel=1e-10)


@pytest.mark.parametrize("gamma", [2e-3, 2e-2])
def test_coupled_fixed_point_conserves_charge_and_oxygen(gamma):
    """At the coupled fixed point: membrane current = proton source, and the
    proton source = (gamma / (k_ref C_in)) x the O2 consumption (both follow one
    Tafel rate on the same sites); the potential falls away from the membrane."""
    ph = _structure(4)
    cp = CO.Coupling(gamma=gamma)
    r = CO.solve(ph, L.Params(), cp)
    assert r.dphi < 1e-10
    assert r.proton_in == pytest.approx(r.source, rel=1e-9)
    assert r.source == pytest.approx(gamma / (cp.k_ref * 1.0) * r.rate, rel=1e-9)
    assert r.phi.max() <= cp.phi_m + 1e-12
    assert r.phi.min() < cp.phi_m - 1e-3


def test_no_proton_source_leaves_the_potential_uniform():
    """gamma = 0: phi = phi_m everywhere and the O2 problem is the reactive problem
    with k_ref exp(beta (phi_m - phi_ref)) on the sites, solved once."""
    ph = _structure(4)
    cp = CO.Coupling(gamma=0.0, phi_m=0.62)
    r = CO.solve(ph, L.Params(), cp)
    assert r.iterations == 1 and np.abs(r.phi - cp.phi_m).max() < 1e-12
    po, pp = CO.o2_problem(ph, L.Params(), cp), CO.phi_problem(ph, cp)
    n = CO.sites(po, pp)
    po.kn = np.zeros(po.active.shape)
    po.kn[:, :, po.nx - pp.nx:] = cp.k_ref * n * np.exp(cp.beta * (cp.phi_m - cp.phi_ref))
    ref = O.solve_fixed_point(po)
    assert r.rate == pytest.approx(ref.rate, rel=1e-12)
    assert ref.fluxes.j_in == pytest.approx(ref.rate, rel=1e-9)


def test_fixed_point_does_not_depend_on_the_relaxation():
    ph = _structure(4)
    a = CO.solve(ph, L.Params(), CO.Coupling(gamma=5e-3, theta=0.5))
    b = CO.solve(ph, L.Params(), CO.Coupling(gamma=5e-3, theta=0.35))
    assert a.rate == pytest.approx(b.rate, rel=1e-9)
    assert np.abs(a.phi - b.phi).max() < 1e-9


def test_stronger_proton_resistance_lowers_the_rate():
    """A larger gamma (weaker conduction) deepens the potential drop and, since
    the Tafel rate grows with phi (Eq. 17b), lowers the O2 consumption."""
    ph = _structure(4)
    rates = [CO.solve(ph, L.Params(), CO.Coupling(gamma=g)).rate for g in (0.0, 2e-3, 2e-2)]
    assert rates[0] > rates[1] > rates[2] > 0


def _lap(act, rate, face_in, face_out, c_in, c_out):
    """A u = b for the D3Q19 link Laplacian at tau = 1 on the simulated voxels:
    sum a_i (u_n - u) + sum 2 a_i (C_b - u) over open face links = rate u."""
    import scipy.sparse as sp

    nz, ny, nx = act.shape
    idx = -np.ones(act.shape, np.int64)
    idx[act] = np.arange(act.sum())
    n = int(act.sum())
    rows, cols, vals = [], [], []
    b = np.zeros(n)
    links = [c for c in itertools.product((-1, 0, 1), repeat=3) if 0 < sum(map(abs, c)) <= 2]
    for z, y, x in zip(*np.nonzero(act)):
        i = idx[z, y, x]
        diag = rate[z, y, x]
        for cx, cy, cz in links:
            a = 1 / 18 if abs(cx) + abs(cy) + abs(cz) == 1 else 1 / 36
            tx, ty, tz = x + cx, (y + cy) % ny, (z + cz) % nz
            if tx < 0 or tx >= nx:
                if act[tz, ty, x] and (face_in if tx < 0 else face_out):
                    diag += 2 * a
                    b[i] += 2 * a * (c_in if tx < 0 else c_out)
            elif act[tz, ty, tx]:
                diag += a
                rows.append(i)
                cols.append(idx[tz, ty, tx])
                vals.append(-a)
        rows.append(i)
        cols.append(i)
        vals.append(diag)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n)), b


def test_coupled_fixed_point_at_tau_one_equals_a_direct_nonlinear_solve():
    """With every tau = 1, the coupled fixed point solves, independently of the
    LBM and of the Picard iteration: u = (1 - k n) C obeys the link Laplacian with
    rate k n / (1 - k n) (k from phi), and w = phi - q obeys it with phi_m on the
    membrane face and source q(C, phi).  Solved here as one nonlinear system by a
    library root finder."""
    from scipy.optimize import root

    ph = _structure(4)
    params = L.Params(d_ionomer_rel=1.0)          # every diffusivity equal: tau = 1
    cp = CO.Coupling(gamma=2e-2)
    r = CO.solve(ph, params, cp)
    po, pp = CO.o2_problem(ph, params, cp), CO.phi_problem(ph, cp)
    assert np.allclose(po.tau[po.active], 1.0) and np.allclose(pp.tau[pp.active], 1.0)
    off = po.nx - pp.nx
    n = CO.sites(po, pp)
    n_o = np.zeros(po.active.shape)
    n_o[:, :, off:] = n
    ao, ap = po.active, pp.active
    zero_o, zero_p = np.zeros(ao.shape), np.zeros(ap.shape)
    A_phi, b_phi = _lap(ap, zero_p, False, True, 0.0, cp.phi_m)
    no, npp = int(ao.sum()), int(ap.sum())

    def unpack(xv):
        C = np.zeros(ao.shape)
        C[ao] = xv[:no]
        phi = np.full(ap.shape, cp.phi_m)
        phi[ap] = xv[no:]
        return C, phi

    def residual(xv):
        C, phi = unpack(xv)
        e = np.ones(ao.shape)
        e[:, :, off:] = np.exp(cp.beta * (phi - cp.phi_ref))
        kn = cp.k_ref * n_o * e
        A_o, b_o = _lap(ao, kn / (1 - kn), True, False, params.c_in, 0.0)
        u = ((1 - kn) * C)[ao]
        q = cp.gamma * n * (C[:, :, off:] / params.c_in) * np.exp(cp.beta * (phi - cp.phi_ref))
        w = (phi - q)[ap]
        return np.concatenate([A_o @ u - b_o, A_phi @ w - b_phi + q[ap]])

    # the Picard fixed point satisfies the independent equations ...
    assert np.abs(residual(np.concatenate([r.C[ao], r.phi[ap]]))).max() < 1e-10
    # ... and a library root finder from a generic start lands on it
    x0 = np.concatenate([np.ones(no), np.full(npp, cp.phi_m)])
    sol = root(residual, x0, method="hybr", tol=1e-14)
    assert np.abs(residual(sol.x)).max() < 1e-11
    C, phi = unpack(sol.x)
    assert np.abs(phi - r.phi).max() < 1e-9
    assert np.abs(np.where(ao, C, 0) - np.where(ao, r.C, 0)).max() < 1e-9
