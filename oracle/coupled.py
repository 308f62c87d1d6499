"""Plain FP64 oracle for the coupled oxygen / proton-potential problem on the
D3Q19 lattice (Chen et al., arXiv 1410.1914, Sections 3.2-3.4, Eqs. 15-18b).

TEST INFRASTRUCTURE ONLY.  Only the test-suite may import it; it shares nothing
with the product library.

The paper writes the model and then presets a uniform ionomer potential for its
runs (Section 3.5.2).  Solving the coupling needs readings of its own, each also
listed in the design notes:

* Reaction sites are ionomer voxels with n > 0 Pt face neighbours (the active
  ionomer cells of Eqs. 18a-b) that both problems reach: joined to the oxygen
  inlet through pore and ionomer, and to the membrane face through ionomer.
* Tafel (Eq. 17b) in lattice units: the O2 sink of a site is
  k(x) n C with k(x) = k_ref exp(beta (phi(x) - phi_ref)), k_ref the rate per Pt
  face at phi_ref; beta = alpha F / (R T).
* The proton source of a site (Eq. 18b) is q(x) = gamma n (C / C_in)
  exp(beta (phi - phi_ref)), with gamma in volts per lattice step: the current of
  one Pt face at C_in and phi_ref, times the voxel edge, over the conductivity.
* The potential solves D_phi lap(phi) = q on the ionomer joined to the membrane
  face x = L, with phi = phi_m there (anti-bounce-back) and zero proton flux at
  the GDL face x = 0 and at every other boundary; D_phi follows tau_ref.
* The oxygen problem is the reactive problem of Eq. 20 (reservoir plane at
  C_in, zero-gradient outlet) with the per-voxel k(x).
* Coupling by Picard iteration from phi = phi_m: solve O2 with k(phi), then the
  potential with q(C, phi), and move phi by the fraction theta of the change,
  until phi changes by less than a tolerance.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import lbm as L
from . import lbm19 as O


@dataclass
class Coupling:
    k_ref: float = 1e-2       # O2 rate per Pt face at phi_ref, lattice units
    beta: float = 21.3        # alpha F / (R T), 1/V (alpha = 0.61, T = 333 K)
    gamma: float = 1e-3       # proton source per Pt face at C_in and phi_ref, V
    phi_m: float = 0.6        # ionomer potential at the membrane face, V
    phi_ref: float = 0.6      # potential at which k_ref holds, V
    tau_phi: float = 1.0      # relaxation time of the potential lattice
    theta: float = 0.5        # Picard under-relaxation


def o2_problem(ph: np.ndarray, params: L.Params, cp: Coupling) -> L.Problem:
    """The reactive O2 problem with sites on Pt-adjacent ionomer (k set per voxel)."""
    p = L.Params(**{**params.__dict__, "mode": L.MODE_REACT, "k_lat": cp.k_ref,
                    "catalyst_phases": 1 << L.PT, "reactive_fluids": 1 << L.IONOMER})
    return O.prepare(ph, p)


def phi_problem(ph: np.ndarray, cp: Coupling) -> L.Problem:
    """The potential problem on ionomer joined to the membrane face x = L."""
    p = L.Params(mode=L.MODE_PROTON, c_in=cp.phi_m, c_out=cp.phi_m, tau_ref=cp.tau_phi)
    prob = O.prepare(ph, p)
    seed = np.zeros(ph.shape, bool)
    seed[:, :, -1] = True
    act = L.flood(prob.transport, seed)
    prob.active = act
    prob.tau = np.where(act, cp.tau_phi, 1.0)
    prob.omega = np.where(act, 1.0 / cp.tau_phi, 0.0)
    prob.kn = np.zeros(ph.shape)
    prob.percolates = bool(act.any())
    prob.faces = (False, True)
    prob.src = np.zeros(ph.shape)
    return prob


def sites(po: L.Problem, pp: L.Problem) -> np.ndarray:
    """n (Pt face neighbours) on the reaction sites of the structure grid, 0 elsewhere."""
    off = po.nx - pp.nx
    n_pt = L.catalyst_neighbours(pp.phase, 1 << L.PT)
    ok = (pp.phase == L.IONOMER) & pp.active & po.active[:, :, off:] & (n_pt > 0)
    return np.where(ok, n_pt, 0).astype(np.float64)


def tafel(cp: Coupling, phi):
    return np.exp(cp.beta * (phi - cp.phi_ref))


@dataclass
class CoupledResult:
    C: np.ndarray            # O2 concentration, simulated grid of the O2 problem
    phi: np.ndarray          # potential on the structure grid (phi_m off the ionomer)
    rate: float              # O2 consumption per unit area (sum k n C / A)
    proton_in: float         # proton current in through the membrane face, per area
    source: float            # sum of q per area
    iterations: int
    dphi: float              # last change of phi


def solve(ph: np.ndarray, params: L.Params, cp: Coupling, tol: float = 1e-10, max_iter: int = 200) -> CoupledResult:
    po = o2_problem(ph, params, cp)
    pp = phi_problem(ph, cp)
    off = po.nx - pp.nx                 # the O2 grid's reservoir plane
    n = sites(po, pp)
    n_o = np.zeros(po.active.shape)
    n_o[:, :, off:] = n
    phi = np.full(ph.shape, cp.phi_m)
    dphi = np.inf
    it = 0
    for it in range(1, max_iter + 1):
        e = np.ones(po.active.shape)
        e[:, :, off:] = tafel(cp, phi)
        po.kn = cp.k_ref * n_o * e
        so = O.solve_fixed_point(po)
        C = O.concentration(so.f)[:, :, off:]
        pp.src = -cp.gamma * n * (C / params.c_in) * tafel(cp, phi)
        sp = O.solve_fixed_point(pp)
        new = np.where(pp.active, O.concentration(sp.f), cp.phi_m)
        dphi = float(np.abs(new - phi).max())
        phi = phi + cp.theta * (new - phi)
        if dphi < tol:
            break
    A = pp.ny * pp.nz
    return CoupledResult(C=O.concentration(so.f), phi=phi, rate=so.fluxes.rate, proton_in=-sp.fluxes.j_out,
                         source=float(-pp.src.sum()) / A, iterations=it, dphi=dphi)
