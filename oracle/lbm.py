"""Plain FP64 oracle for the D3Q7 reactive-diffusion lattice Boltzmann solver.

TEST INFRASTRUCTURE ONLY.  This module is the correctness reference for the HIP
solver; only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import it.  It shares no code with the product library and imports
nothing from it.  The heavy loops live in ``lbm_ref.c`` (plain C, FP64), built by
``oracle/build.py`` into ``oracle/liblbm_ref.so``.

What it computes, following Chen et al., arXiv 1410.1914:

* Physics (Section 3.1): bulk O2 diffusivity (Eq. 7), Knudsen diffusivity (Eq. 8),
  Bosanquet combination (Eq. 9).
* Pore size by 13-direction averaging (Section 2.1.3).
* Transport phases and a continuous concentration field over pore + ionomer
  (Eqs. 14-15); proton conduction on ionomer only (Eq. 16, Section 3.5.1).
* Local relaxation time from the local diffusivity (Eq. 24, on the D3Q7 lattice:
  c_s^2 = (1 - w0)/3).
* First-order sink S = -k n C on fluid voxels with n catalyst face-neighbours
  (Eqs. 17b, 18a with uniform ionomer potential, Section 3.5.2).
* Boundary conditions of Section 3.5: Dirichlet x faces for effective properties
  (Eq. 19); one prepended pore plane, Dirichlet inlet and zero-gradient outlet for
  the reactive problem (Eqs. 20a, 20b); periodic y, z.
* The LBM step of Eq. (21), and its steady state by two routes: plain time-stepping
  (the definition) and a direct or Krylov solve of the affine fixed point.
* D_eff/D0 from the x flux (Eq. 19), total reaction rate.

Readings where the paper is silent or garbled (each one is also listed in the
design notes): D3Q7 with rest weight w0 = 1/4 instead of D3Q19; Eq. 23 read as
g_eq = w_i C; Eq. 24 with c_s^2 = (1-w0)/3; sink sign = consumption; Dirichlet by
anti-bounce-back on the voxel faces, L = nx; tau = 1/2 + (tau_ref - 1/2) D/D_ref
with D_ref the largest diffusivity among simulated voxels; transport voxels not
6-connected to a Dirichlet face are excluded.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field

import numpy as np

PORE, CARBON, PT, IONOMER = 0, 1, 2, 3
MODE_DEFF, MODE_REACT, MODE_PROTON = 0, 1, 2

R_GAS = 8.314  # J mol^-1 K^-1, as used with Eq. (8)

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liblbm_ref.so")
_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b

        _b.build()
    lib = ctypes.CDLL(_LIB_PATH)
    dp = ctypes.POINTER(ctypes.c_double)
    u8 = ctypes.POINTER(ctypes.c_uint8)
    i64 = ctypes.POINTER(ctypes.c_int64)
    g = ctypes.POINTER(_Grid)
    lib.orc_collide.argtypes = [g, dp, dp]
    lib.orc_stream.argtypes = [g, dp, dp]
    lib.orc_step.argtypes = [g, dp, dp, dp]
    lib.orc_concentration.argtypes = [g, dp, dp]
    lib.orc_fluxes.argtypes = [g, dp, dp, dp, dp]
    lib.orc_assemble.argtypes = [g, i64, i64, dp, dp]
    lib.orc_assemble.restype = ctypes.c_int64
    lib.orc_chords.argtypes = [ctypes.c_int] * 3 + [u8, dp]
    lib.orc_flood.argtypes = [ctypes.c_int] * 3 + [u8, u8, u8]
    lib.orc_num_threads.argtypes = []
    lib.orc_num_threads.restype = ctypes.c_int
    for fn in (lib.orc_collide, lib.orc_stream, lib.orc_step, lib.orc_concentration,
               lib.orc_fluxes, lib.orc_chords, lib.orc_flood):
        fn.restype = None
    _lib = lib
    return lib


class _Grid(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("react", ctypes.c_int32),
        ("c_in", ctypes.c_double), ("c_out", ctypes.c_double), ("w0", ctypes.c_double),
        ("active", ctypes.POINTER(ctypes.c_uint8)),
        ("omega", ctypes.POINTER(ctypes.c_double)),
        ("kn", ctypes.POINTER(ctypes.c_double)),
    ]


def num_threads() -> int:
    """Threads the oracle's parallel loops use."""
    return int(_load().orc_num_threads())


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


# --------------------------------------------------------------------------- physics

def bulk_diffusivity(T_K: float, p_atm: float) -> float:
    """Binary O2-N2 bulk diffusivity, Eq. (7): 0.22e-4 (T/293.2)^1.5 / (p/1 atm), m^2/s."""
    return 0.22e-4 * (T_K / 293.2) ** 1.5 / p_atm


def knudsen_diffusivity(d_p_m, T_K: float, M_kg_mol: float = 0.032):
    """Knudsen diffusivity, Eq. (8): (d_p / 3) sqrt(8 R T / (pi M)), SI units."""
    return np.asarray(d_p_m, dtype=np.float64) / 3.0 * math.sqrt(8.0 * R_GAS * T_K / (math.pi * M_kg_mol))


def bosanquet(D_b, D_kn):
    """Bosanquet combination, Eq. (9): 1/D = 1/D_Kn + 1/D_b."""
    return 1.0 / (1.0 / np.asarray(D_kn, dtype=np.float64) + 1.0 / D_b)


def pore_chords(pore: np.ndarray) -> np.ndarray:
    """13-direction averaged pore size (Section 2.1.3), in voxel edges.

    ``pore`` is a boolean (nz, ny, nx) array; returns FP64 (nz, ny, nx), 0 off-pore."""
    pore = np.ascontiguousarray(pore, dtype=np.uint8)
    nz, ny, nx = pore.shape
    out = np.zeros(pore.shape, dtype=np.float64)
    _load().orc_chords(nx, ny, nz, _p(pore, ctypes.c_uint8), _p(out, ctypes.c_double))
    return out


def flood(transport: np.ndarray, seed: np.ndarray) -> np.ndarray:
    """6-connected reachability over ``transport`` from ``seed`` voxels (periodic y, z)."""
    t = np.ascontiguousarray(transport, dtype=np.uint8)
    s = np.ascontiguousarray(seed, dtype=np.uint8)
    nz, ny, nx = t.shape
    out = np.zeros(t.shape, dtype=np.uint8)
    _load().orc_flood(nx, ny, nz, _p(t, ctypes.c_uint8), _p(s, ctypes.c_uint8), _p(out, ctypes.c_uint8))
    return out.astype(bool)


# --------------------------------------------------------------------------- problem setup

@dataclass
class Params:
    """Problem definition (mirrors the quantities the paper's model needs)."""

    mode: int = MODE_DEFF
    c_in: float = 1.0
    c_out: float = 0.0
    tau_ref: float = 1.0
    w0: float = 0.25
    knudsen: bool = False
    T_K: float = 353.0
    p_atm: float = 1.0
    M_kg_mol: float = 0.032
    voxel_m: float = 2e-9
    d_ionomer_rel: float = 1e-3
    d_ref_rel: float = 0.0          # 0: D_ref = largest simulated diffusivity
    k_lat: float = 0.0
    catalyst_phases: int = 1 << PT  # bit mask over phase ids
    reactive_fluids: int = (1 << PORE) | (1 << IONOMER)
    reservoir_plane: bool = True    # reactive problem: prepend one pore plane


@dataclass
class Problem:
    """Per-voxel fields of the simulated grid (FP64), ready for the LBM."""

    params: Params
    nx: int
    ny: int
    nz: int
    phase: np.ndarray               # simulated grid (reservoir plane included)
    transport: np.ndarray           # bool: phase is a transport phase
    active: np.ndarray              # bool: transport and connected to a Dirichlet face
    D: np.ndarray                   # m^2/s (or relative units in proton mode), 0 off transport
    d_p: np.ndarray                 # pore size in voxel edges (structure voxels only)
    D0: float
    D_ref: float
    tau: np.ndarray
    omega: np.ndarray
    n_cat: np.ndarray               # int: catalyst face-neighbours
    kn: np.ndarray                  # k * n on reactive fluid voxels
    nx_struct: int
    percolates: bool = field(default=True)

    @property
    def N(self):
        return self.nx * self.ny * self.nz

    def grid(self):
        """ctypes view; keeps references alive on the instance."""
        self._act8 = np.ascontiguousarray(self.active, dtype=np.uint8)
        self._om = np.ascontiguousarray(self.omega, dtype=np.float64)
        self._kn = np.ascontiguousarray(self.kn, dtype=np.float64)
        p = self.params
        return _Grid(self.nx, self.ny, self.nz, 1 if p.mode == MODE_REACT else 0,
                     p.c_in, p.c_out, p.w0,
                     _p(self._act8, ctypes.c_uint8), _p(self._om, ctypes.c_double), _p(self._kn, ctypes.c_double))


def weights(w0: float) -> np.ndarray:
    w = np.full(7, (1.0 - w0) / 6.0)
    w[0] = w0
    return w


def cs2(w0: float) -> float:
    """Lattice sound speed squared of D3Q7 with rest weight w0: sum_i w_i c_ix^2."""
    return (1.0 - w0) / 3.0


def catalyst_neighbours(phase: np.ndarray, catalyst_mask: int) -> np.ndarray:
    """n(x): number of face neighbours whose phase is a catalyst phase (Eq. 18a).

    Periodic in y and z; nothing beyond the x faces."""
    cat = ((catalyst_mask >> phase.astype(np.int64)) & 1).astype(np.int64)
    n = np.zeros(phase.shape, dtype=np.int64)
    n[:, :, 1:] += cat[:, :, :-1]
    n[:, :, :-1] += cat[:, :, 1:]
    for ax in (0, 1):
        n += np.roll(cat, 1, axis=ax) + np.roll(cat, -1, axis=ax)
    return n


def prepare(phase_struct: np.ndarray, params: Params) -> Problem:
    """Map a (nz, ny, nx) phase map to the per-voxel LBM fields (Sections 3 and 4)."""
    ph = np.asarray(phase_struct, dtype=np.uint8)
    if ph.ndim != 3 or min(ph.shape) < 1:
        raise ValueError("phase map must be a non-empty 3-D array")
    if ph.max(initial=0) > IONOMER:
        raise ValueError("unknown phase id")
    p = params
    nz, ny, nxs = ph.shape

    # pore size from the structure itself (the reservoir plane is not part of it)
    d_p = pore_chords(ph == PORE)

    if p.mode == MODE_PROTON:
        transport_s = ph == IONOMER
        D0 = 1.0
        D_s = np.where(transport_s, 1.0, 0.0)
    else:
        transport_s = (ph == PORE) | (ph == IONOMER)
        D_b = bulk_diffusivity(p.T_K, p.p_atm)
        D0 = D_b
        if p.knudsen:
            D_pore = np.full(ph.shape, D_b)
            sel = ph == PORE
            D_pore[sel] = bosanquet(D_b, knudsen_diffusivity(d_p[sel] * p.voxel_m, p.T_K, p.M_kg_mol))
        else:
            D_pore = np.full(ph.shape, D_b)
        D_s = np.where(ph == PORE, D_pore, 0.0)
        D_s = np.where(ph == IONOMER, p.d_ionomer_rel * D0, D_s)

    if p.mode == MODE_REACT and p.reservoir_plane:
        # one plane of pore cells before the structure, bulk diffusivity (Section 3.5.2)
        phase = np.concatenate([np.full((nz, ny, 1), PORE, np.uint8), ph], axis=2)
        transport = np.concatenate([np.ones((nz, ny, 1), bool), transport_s], axis=2)
        D = np.concatenate([np.full((nz, ny, 1), D0), D_s], axis=2)
    else:
        phase, transport, D = ph, transport_s, D_s
    nx = phase.shape[2]

    # Dirichlet faces: inlet and outlet for effective properties, inlet only when reacting
    seed = np.zeros(phase.shape, dtype=bool)
    seed[:, :, 0] = True
    if p.mode != MODE_REACT:
        seed[:, :, -1] = True
    active = flood(transport, seed)
    if p.mode != MODE_REACT:
        left = np.zeros(phase.shape, bool)
        left[:, :, 0] = True
        percolates = bool(flood(transport, left)[:, :, -1].any())
    else:
        percolates = bool(active.any())

    D = np.where(active, D, 0.0)
    if p.d_ref_rel > 0:
        D_ref = p.d_ref_rel * D0
    else:
        D_ref = float(D.max()) if active.any() else D0
    tau = np.where(active, 0.5 + (p.tau_ref - 0.5) * D / D_ref, 1.0)
    omega = np.where(active, 1.0 / tau, 0.0)

    n_cat = catalyst_neighbours(phase, p.catalyst_phases)
    reactive = ((p.reactive_fluids >> phase.astype(np.int64)) & 1).astype(bool) & active
    if p.mode != MODE_REACT:
        reactive[:] = False
    kn = np.where(reactive, p.k_lat * n_cat, 0.0)

    return Problem(params=p, nx=nx, ny=ny, nz=nz, phase=phase, transport=transport, active=active,
                   D=D, d_p=d_p, D0=D0, D_ref=D_ref, tau=tau, omega=omega, n_cat=n_cat, kn=kn,
                   nx_struct=nxs, percolates=percolates)


# --------------------------------------------------------------------------- the LBM

def equilibrium(prob: Problem, C) -> np.ndarray:
    """f_i = w_i C on active voxels (Eq. 23 as read); C scalar or (nz, ny, nx)."""
    w = weights(prob.params.w0)
    C = np.broadcast_to(np.asarray(C, dtype=np.float64), (prob.nz, prob.ny, prob.nx)).ravel()
    f = w[:, None] * C[None, :]
    f[:, ~prob.active.ravel()] = 0.0
    return np.ascontiguousarray(f)


def collide(prob: Problem, f: np.ndarray) -> np.ndarray:
    out = np.empty_like(f)
    g = prob.grid()
    _load().orc_collide(ctypes.byref(g), _p(f, ctypes.c_double), _p(out, ctypes.c_double))
    return out


def stream(prob: Problem, fs: np.ndarray) -> np.ndarray:
    out = np.empty_like(fs)
    g = prob.grid()
    _load().orc_stream(ctypes.byref(g), _p(fs, ctypes.c_double), _p(out, ctypes.c_double))
    return out


class Stepper:
    """Repeated Eq. (21) steps without re-marshalling the fields each time."""

    def __init__(self, prob: Problem):
        self.prob = prob
        self.g = prob.grid()
        self.tmp = np.empty((7, prob.N))
        self.lib = _load()

    def step(self, f: np.ndarray, out: np.ndarray | None = None) -> np.ndarray:
        if out is None:
            out = np.empty_like(f)
        self.lib.orc_step(ctypes.byref(self.g), _p(f, ctypes.c_double), _p(out, ctypes.c_double),
                          _p(self.tmp, ctypes.c_double))
        return out


def step(prob: Problem, f: np.ndarray) -> np.ndarray:
    return Stepper(prob).step(f)


def concentration(prob: Problem, f: np.ndarray) -> np.ndarray:
    C = np.empty(prob.N)
    g = prob.grid()
    _load().orc_concentration(ctypes.byref(g), _p(f, ctypes.c_double), _p(C, ctypes.c_double))
    return C.reshape(prob.nz, prob.ny, prob.nx)


@dataclass
class Fluxes:
    j_in: float      # per unit cross-section area (lattice units)
    j_out: float
    j_vol: float     # mean over the interior x faces
    rate: float      # sum k n C per unit cross-section area
    mass: float      # total sum of C
    face: np.ndarray  # per interior face, per unit area


def fluxes(prob: Problem, f: np.ndarray) -> Fluxes:
    out = np.zeros(5)
    face = np.zeros(max(prob.nx - 1, 1))
    tmp = np.empty_like(f)
    g = prob.grid()
    _load().orc_fluxes(ctypes.byref(g), _p(f, ctypes.c_double), _p(tmp, ctypes.c_double),
                       _p(out, ctypes.c_double), _p(face, ctypes.c_double))
    A = prob.ny * prob.nz
    nfaces = prob.nx - 1
    return Fluxes(j_in=out[0] / A, j_out=out[1] / A, j_vol=(out[2] / nfaces / A) if nfaces > 0 else out[0] / A,
                  rate=out[3] / A, mass=out[4], face=face[:nfaces] / A)


def d0_lattice(prob: Problem) -> float:
    """D0 in lattice units: c_s^2 (tau_ref - 1/2) D0 / D_ref (Eq. 24 on D3Q7)."""
    p = prob.params
    return cs2(p.w0) * (p.tau_ref - 0.5) * prob.D0 / prob.D_ref


def deff_from_flux(prob: Problem, J: float) -> float:
    """Eq. (19): D_eff = J / ((C_in - C_out) / L_x), normalised by D0; L_x = nx."""
    p = prob.params
    return J * prob.nx / ((p.c_in - p.c_out) * d0_lattice(prob))


# --------------------------------------------------------------------------- steady state

@dataclass
class Steady:
    f: np.ndarray
    fluxes: Fluxes
    deff: float | None
    rate: float | None
    steps: int = 0
    residual: float = 0.0


def _finish(prob: Problem, f: np.ndarray, steps=0, residual=0.0) -> Steady:
    fl = fluxes(prob, f)
    p = prob.params
    if p.mode == MODE_REACT:
        return Steady(f, fl, None, fl.rate, steps, residual)
    deff = deff_from_flux(prob, fl.j_vol) if prob.percolates else 0.0
    return Steady(f, fl, deff, None, steps, residual)


def solve_timestep(prob: Problem, tol: float = 1e-12, max_steps: int = 10_000_000, f0=None,
                   check_every: int = 1) -> Steady:
    """Time-stepping from f = w_i C0 (C0 = 0) until max|C(t) - C(t-1)| / max|C| < tol."""
    f = equilibrium(prob, 0.0) if f0 is None else np.ascontiguousarray(f0, dtype=np.float64).copy()
    st = Stepper(prob)
    buf = np.empty_like(f)
    Cprev = f.sum(axis=0)
    res = np.inf
    for n in range(1, max_steps + 1):
        st.step(f, buf)
        f, buf = buf, f
        if n % check_every == 0:
            C = f.sum(axis=0)
            scale = np.abs(C).max()
            res = np.abs(C - Cprev).max() / scale if scale > 0 else 0.0
            Cprev = C
            if res < tol:
                return _finish(prob, f, n, res)
    return _finish(prob, f, max_steps, res)


def assemble(prob: Problem):
    """Sparse A (7N x 7N, CSR) and b with f(t+1) = A f(t) + b."""
    import scipy.sparse as sp

    n_act = int(prob.active.sum())
    cap = 49 * n_act
    rows = np.empty(cap, np.int64)
    cols = np.empty(cap, np.int64)
    vals = np.empty(cap, np.float64)
    b = np.empty(7 * prob.N)
    g = prob.grid()
    k = _load().orc_assemble(ctypes.byref(g), _p(rows, ctypes.c_int64), _p(cols, ctypes.c_int64),
                             _p(vals, ctypes.c_double), _p(b, ctypes.c_double))
    A = sp.csr_matrix((vals[:k], (rows[:k], cols[:k])), shape=(7 * prob.N, 7 * prob.N))
    return A, b


def solve_fixed_point(prob: Problem, method: str = "direct", tol: float = 1e-13, maxiter: int = 200_000) -> Steady:
    """Steady state f* = A f* + b of the affine step, by a library linear solve:
    "direct" (sparse LU), "dense" (tiny grids), "bicgstab", or "gmres" (restarted
    GMRES with an incomplete-LU preconditioner, for grids too large to factorise;
    its result is also checked to be a fixed point of one plain time step).

    Only the unknowns of active voxels enter the system (the rest are zero)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla

    A, b = assemble(prob)
    act = np.flatnonzero(np.tile(prob.active.ravel(), 7))
    As = A[act][:, act]
    bs = b[act]
    M = sp.identity(len(act), format="csr") - As
    if len(act) == 0:
        x = np.zeros(0)
    elif method == "direct":
        x = spla.spsolve(M.tocsc(), bs)
    elif method == "dense":
        x = np.linalg.solve(M.toarray(), bs)
    elif method == "bicgstab":
        x, info = spla.bicgstab(M, bs, rtol=tol, atol=0.0, maxiter=maxiter)
        if info != 0:
            raise RuntimeError(f"bicgstab did not converge (info={info})")
    elif method == "gmres":
        x = _gmres_ilu(M, bs, tol, maxiter)
    else:
        raise ValueError(method)
    f = np.zeros(7 * prob.N)
    f[act] = x
    f = f.reshape(7, prob.N)
    if method == "gmres":
        _certify(prob, f)
    return _finish(prob, f)


def _gmres_ilu(M, b, tol: float, maxiter: int) -> np.ndarray:
    """Restarted GMRES on (I - A) f = b, preconditioned by an incomplete LU factor
    of the same matrix (drop tolerance 1e-2).  For systems too large for the direct
    factorisation (the catalyst layers at 64^3 and above); the preconditioner only
    changes how fast the iteration gets there.  Raises unless the true residual
    ||(I - A) f - b|| falls below tol ||b||."""
    import scipy.sparse.linalg as spla

    Mc = M.tocsc()
    ilu = spla.spilu(Mc, drop_tol=1e-2, fill_factor=20, permc_spec="MMD_AT_PLUS_A", diag_pivot_thresh=0.0,
                     options=dict(ILU_MILU="SILU"))
    P = spla.LinearOperator(M.shape, ilu.solve)
    x = None
    bn = float(np.linalg.norm(b))
    for _ in range(8):  # outer restarts from the last iterate until the true residual is met
        x, info = spla.gmres(M, b, x0=x, M=P, rtol=tol, atol=0.0, restart=100, maxiter=max(1, maxiter // 100))
        res = float(np.linalg.norm(M @ x - b)) / bn if bn > 0 else 0.0
        if res < tol:
            return x
    raise RuntimeError(f"gmres did not reach the residual {tol:g} (last {res:.3g}, info {info})")


def _certify(prob: Problem, f: np.ndarray, tol: float = 1e-12) -> None:
    """The definition of the fixed point, checked with one plain time step: the
    largest change of C it makes, relative to max C, must be below tol (the
    time-stepping route's own stop criterion)."""
    g = Stepper(prob).step(np.ascontiguousarray(f))
    C0, C1 = f.sum(axis=0), g.sum(axis=0)
    scale = float(np.abs(C0).max())
    change = float(np.abs(C1 - C0).max()) / scale if scale > 0 else 0.0
    if not change < tol:
        raise RuntimeError(f"not a fixed point of the step: relative change {change:.3g}")


def solve(phase_struct: np.ndarray, params: Params, method: str = "direct") -> Steady:
    prob = prepare(phase_struct, params)
    if params.mode != MODE_REACT and not prob.percolates:
        f = np.zeros((7, prob.N))
        return Steady(f, fluxes(prob, f), 0.0, None)
    return solve_fixed_point(prob, method)
