"""Plain FP64 oracle for the D3Q19 variant of the reactive-diffusion LBM.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline of the benchmark may import it.  It shares no code with the product
library and imports nothing from it; within the oracle it reuses the property
mapping of ``oracle.lbm`` (phases, diffusivities, relaxation times, catalyst
neighbours, connectivity), which does not depend on the lattice.

What it computes, following Chen et al., arXiv 1410.1914, Section 4:

* The lattice of Eq. (22): the rest velocity, the six face neighbours and the
  twelve edge neighbours; the weights of Eq. (23), 1/3, 1/18 and 1/36, with the
  equilibrium read as g_eq = a_i C; c_s^2 = 1/3, so D = (tau - 1/2)/3 (Eq. 24).
* The SRT step of Eq. (21) with the sink a_i S, S = -k n C (Eqs. 17b, 18a).
* Streaming with half-way bounce-back at impermeable neighbours, periodic y and z,
  and the Dirichlet faces of Section 3.5 by anti-bounce-back (Eq. 19), or a
  zero-gradient outlet for the reactive problem (Eq. 20b).
* The steady state, by time-stepping or by a direct solve of the affine fixed
  point, and D_eff/D0 (Eq. 19) and the total reaction rate from it.

Readings where the paper is silent (each is also listed in the design notes):
a population that would enter through an x face from the reservoir takes the
anti-bounce-back value only when the voxel of the boundary plane it passes
(the face plane, shifted by its y and z components) is a simulated voxel, and
bounces back otherwise, as if the structure's boundary plane extended into the
reservoir; the relaxation time follows the local diffusivity exactly as on the
D3Q7 lattice (tau_ref at D_ref).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import lbm as L

Q = 19


def velocities() -> np.ndarray:
    """(19, 3) integer velocities (c_x, c_y, c_z), Eq. (22): rest; +x, -x, +y, -y,
    +z, -z; then the edges of the xy, xz and yz planes, each as (+,+), (+,-),
    (-,+), (-,-) of its two non-zero components."""
    c = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]
    for a, b in ((0, 1), (0, 2), (1, 2)):
        for sa in (1, -1):
            for sb in (1, -1):
                v = [0, 0, 0]
                v[a], v[b] = sa, sb
                c.append(tuple(v))
    return np.array(c, dtype=np.int64)


C19 = velocities()
W19 = np.array([1.0 / 3.0] + [1.0 / 18.0] * 6 + [1.0 / 36.0] * 12)   # Eq. (23)
OPP = np.array([int(np.flatnonzero((C19 == -C19[i]).all(axis=1))[0]) for i in range(Q)])
CS2 = 1.0 / 3.0                                                      # Eq. (24)


def prepare(phase_struct: np.ndarray, params: L.Params) -> L.Problem:
    """Per-voxel fields (phases, activity, relaxation rates, k n), Sections 3-4."""
    return L.prepare(phase_struct, params)


def d0_lattice(prob: L.Problem) -> float:
    """D0 in lattice units on D3Q19: (tau_ref - 1/2) D0 / (3 D_ref)  (Eq. 24)."""
    p = prob.params
    return CS2 * (p.tau_ref - 0.5) * prob.D0 / prob.D_ref


def equilibrium(prob: L.Problem, C) -> np.ndarray:
    """f_i = a_i C on active voxels, shape (19, nz, ny, nx)."""
    C = np.broadcast_to(np.asarray(C, dtype=np.float64), prob.active.shape)
    f = W19[:, None, None, None] * C[None]
    return np.where(prob.active[None], f, 0.0)


def dirichlet_faces(prob: L.Problem):
    """(inlet, outlet): which x faces hold a Dirichlet value.  Effective
    properties: both (Eq. 19); reactive problem: the inlet only (Eq. 20b); the
    coupled potential problem: the membrane face x = L only."""
    faces = getattr(prob, "faces", None)
    if faces is not None:
        return faces
    return (True, prob.params.mode != L.MODE_REACT)


def collide(prob: L.Problem, f: np.ndarray) -> np.ndarray:
    """Post-collision f* = f - (f - a C)/tau + a S with S = -k n C (Eq. 21), plus
    a given per-voxel source where the problem carries one."""
    C = f.sum(axis=0)
    S = -prob.kn * C
    if getattr(prob, "src", None) is not None:
        S = S + prob.src
    w = W19[:, None, None, None]
    fs = f + prob.omega[None] * (w * C[None] - f) + w * S[None]
    return np.where(prob.active[None], fs, 0.0)


PULL, BOUNCE, ANTI = 0, 1, 2


def pull_map(prob: L.Problem):
    """For every direction i and voxel x, where the post-stream f_i(x) comes from.

    Returns (kind, src) of shape (19, nz, ny, nx): kind PULL takes f*_i at the
    flat voxel index src (= x - c_i, periodic in y and z); BOUNCE takes the voxel's
    own f*_opp(i); ANTI takes -f*_opp(i) + 2 a_i C_b at an open Dirichlet face."""
    p = prob.params
    act = prob.active
    nz, ny, nx = act.shape
    idx = np.arange(nz * ny * nx).reshape(act.shape)
    kind = np.empty((Q,) + act.shape, np.int8)
    src = np.zeros((Q,) + act.shape, np.int64)
    d_in, d_out = dirichlet_faces(prob)
    del p
    for i in range(Q):
        cx, cy, cz = C19[i]
        # voxel (z - cz, y - cy) of the same x plane, and whether it is simulated
        s_idx = np.roll(np.roll(idx, cz, axis=0), cy, axis=1)
        s_act = np.roll(np.roll(act, cz, axis=0), cy, axis=1)
        a = np.zeros(act.shape, bool)
        if cx == 0:
            src[i], a = s_idx, s_act
        elif cx == 1:
            src[i][..., 1:], a[..., 1:] = s_idx[..., :-1], s_act[..., :-1]
        else:
            src[i][..., :-1], a[..., :-1] = s_idx[..., 1:], s_act[..., 1:]
        k = np.where(a, PULL, BOUNCE).astype(np.int8)
        if cx == 1 and d_in:
            k[..., 0] = np.where(s_act[..., 0], ANTI, BOUNCE)
        if cx == -1 and d_out:
            k[..., -1] = np.where(s_act[..., -1], ANTI, BOUNCE)
        kind[i] = k
    return kind, src


def boundary_value(prob: L.Problem, i: int) -> float:
    """C_b of the face direction i enters through: inlet for c_x = +1, outlet for -1."""
    return prob.params.c_in if C19[i][0] == 1 else prob.params.c_out


def stream(prob: L.Problem, fs: np.ndarray, pmap=None) -> np.ndarray:
    kind, src = pull_map(prob) if pmap is None else pmap
    out = np.zeros_like(fs)
    for i in range(Q):
        j = OPP[i]
        pulled = fs[i].ravel()[src[i].ravel()].reshape(fs[i].shape)
        anti = -fs[j] + 2.0 * W19[i] * boundary_value(prob, i)
        v = np.where(kind[i] == PULL, pulled, np.where(kind[i] == BOUNCE, fs[j], anti))
        out[i] = np.where(prob.active, v, 0.0)
    return out


def step(prob: L.Problem, f: np.ndarray, pmap=None) -> np.ndarray:
    """One step of Eq. (21): collide, then stream."""
    return stream(prob, collide(prob, f), pmap)


def concentration(f: np.ndarray) -> np.ndarray:
    return f.sum(axis=0)


@dataclass
class Fluxes:
    j_in: float      # net flux in through the inlet face, per unit cross-section
    j_out: float     # net flux out through the outlet face
    j_vol: float     # net x flux, mean over the interior faces
    rate: float      # sum k n C per unit cross-section
    mass: float      # sum C
    face: np.ndarray  # per interior face


def fluxes(prob: L.Problem, f: np.ndarray) -> Fluxes:
    """Fluxes carried by the links of f* = collide(f) during the next streaming.

    An interior face x + 1/2 is crossed by f*_i(x) with c_x = +1 and by f*_i(x+1)
    with c_x = -1 whenever the voxel the population moves to is simulated.  At an
    open Dirichlet face the outgoing f*_opp is replaced by the anti-bounce-back
    value, so the net inflow of that link is 2 a C_b - 2 f*_opp."""
    p = prob.params
    act = prob.active
    nz, ny, nx = act.shape
    A = ny * nz
    d_in, d_out = dirichlet_faces(prob)
    fs = collide(prob, f)
    face = np.zeros(max(nx - 1, 0))
    j_in = j_out = 0.0
    for i in range(Q):
        cx, cy, cz = C19[i]
        # is the voxel (z + cz, y + cy) of a plane simulated?
        dest = np.roll(np.roll(act, -cz, axis=0), -cy, axis=1)
        if cx == 1:
            face += (fs[i][..., :-1] * dest[..., 1:]).sum(axis=(0, 1))
            # leaving through the outlet face (x = nx - 1), where the link is open
            if d_out:
                open_ = dest[..., -1] & act[..., -1]
                j_out += np.sum((2.0 * fs[i][..., -1] - 2.0 * W19[i] * p.c_out) * open_)
        elif cx == -1:
            face -= (fs[i][..., 1:] * dest[..., :-1]).sum(axis=(0, 1))
            if d_in:
                open_ = dest[..., 0] & act[..., 0]
                j_in += np.sum((2.0 * W19[i] * p.c_in - 2.0 * fs[i][..., 0]) * open_)
    C = concentration(f)
    # the net sink: k n C, less any given source
    rate = float(np.sum(prob.kn * C))
    if getattr(prob, "src", None) is not None:
        rate -= float(np.sum(prob.src * act))
    nf = nx - 1
    return Fluxes(j_in=j_in / A, j_out=j_out / A,
                  j_vol=(face.sum() / nf / A) if nf > 0 else j_in / A,
                  rate=rate / A, mass=float(C.sum()), face=face / A)


def deff_from_flux(prob: L.Problem, J: float) -> float:
    """Eq. (19): D_eff = J / ((C_in - C_out) / L), L = nx, normalised by D0."""
    p = prob.params
    return J * prob.nx / ((p.c_in - p.c_out) * d0_lattice(prob))


@dataclass
class Steady:
    f: np.ndarray
    fluxes: Fluxes
    deff: float | None
    rate: float | None
    steps: int = 0


def _finish(prob, f, steps=0) -> Steady:
    fl = fluxes(prob, f)
    if prob.params.mode == L.MODE_REACT or getattr(prob, "faces", None) is not None:
        return Steady(f, fl, None, fl.rate, steps)
    return Steady(f, fl, deff_from_flux(prob, fl.j_vol) if prob.percolates else 0.0, None, steps)


def solve_timestep(prob: L.Problem, tol: float = 1e-12, max_steps: int = 2_000_000, f0=None) -> Steady:
    """Steps from f = a_i C0 (C0 = 0) until max|C(t) - C(t-1)| / max|C| < tol."""
    pmap = pull_map(prob)
    f = equilibrium(prob, 0.0) if f0 is None else np.array(f0, dtype=np.float64)
    Cprev = concentration(f)
    for n in range(1, max_steps + 1):
        f = step(prob, f, pmap)
        C = concentration(f)
        scale = np.abs(C).max()
        if scale > 0 and np.abs(C - Cprev).max() / scale < tol:
            return _finish(prob, f, n)
        Cprev = C
    return _finish(prob, f, max_steps)


def assemble(prob: L.Problem):
    """Sparse A (19N x 19N) and b with f(t+1) = A f(t) + b.

    Post-stream f_i(x) = s f*_k(v) + b, and f*_k(v) = (1 - w_v) f_k(v) +
    (w_v - kn_v) a_k sum_j f_j(v), so each row holds 20 entries before merging."""
    import scipy.sparse as sp

    act = prob.active
    N = act.size
    kind, src = pull_map(prob)
    om = prob.omega.ravel()
    kn = prob.kn.ravel()
    vox = np.arange(N)
    rows, cols, vals = [], [], []
    b = np.zeros((Q, N))
    a_vox = act.ravel()
    for i in range(Q):
        j = OPP[i]
        kd = kind[i].ravel()
        v = np.where(kd == PULL, src[i].ravel(), vox)
        k = np.where(kd == PULL, i, j)
        s = np.where(kd == ANTI, -1.0, 1.0)
        sel = a_vox & a_vox[v]
        r = i * N + vox[sel]
        vv, kk, ss = v[sel], k[sel], s[sel]
        rows.append(r)
        cols.append(kk * N + vv)
        vals.append(ss * (1.0 - om[vv]))
        for jj in range(Q):
            rows.append(r)
            cols.append(jj * N + vv)
            vals.append(ss * (om[vv] - kn[vv]) * W19[kk])
        b[i] = np.where(a_vox & (kd == ANTI), 2.0 * W19[i] * boundary_value(prob, i), 0.0)
        if getattr(prob, "src", None) is not None:
            # the source enters f*_k(v) as a_k S(v), carried with the link's sign
            sv = prob.src.ravel()
            b[i][vox[sel]] += ss * W19[kk] * sv[vv]
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(Q * N, Q * N))
    return A, b.ravel()


def solve_fixed_point(prob: L.Problem, method: str = "direct") -> Steady:
    """f* = A f* + b over the unknowns of simulated voxels, by a library solve."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla

    A, b = assemble(prob)
    act = np.flatnonzero(np.tile(prob.active.ravel(), Q))
    M = sp.identity(len(act), format="csr") - A[act][:, act]
    if len(act) == 0:
        x = np.zeros(0)
    elif method == "direct":
        x = spla.spsolve(M.tocsc(), b[act])
    elif method == "dense":
        x = np.linalg.solve(M.toarray(), b[act])
    else:
        raise ValueError(method)
    f = np.zeros(Q * prob.active.size)
    f[act] = x
    return _finish(prob, f.reshape((Q,) + prob.active.shape))


def solve(phase_struct: np.ndarray, params: L.Params, method: str = "direct") -> Steady:
    prob = prepare(phase_struct, params)
    if params.mode != L.MODE_REACT and not prob.percolates:
        f = np.zeros((Q,) + prob.active.shape)
        return Steady(f, fluxes(prob, f), 0.0, None)
    return solve_fixed_point(prob, method)
