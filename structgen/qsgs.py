"""QSGS reconstruction and the synthetic workloads (see the package docstring)."""
from __future__ import annotations

import math

import numpy as np

PORE, CARBON, PT, IONOMER = 0, 1, 2, 3


# ----------------------------------------------------------------- Eqs. (1)-(5)

def volume_fractions(eps: float, beta_N: float, theta_Pt: float,
                     rho_N: float, rho_C: float, rho_Pt: float):
    """Volume fractions of Nafion, carbon and Pt from the design loads, Eqs. (4a)-(4c)."""
    a = (1.0 + theta_Pt) * beta_N / (rho_N * (1.0 - beta_N))
    den = theta_Pt / rho_Pt + 1.0 / rho_C + a
    eps_N = (1.0 - eps) * a / den
    eps_C = (1.0 - eps) * (1.0 / rho_C) / den
    eps_Pt = (1.0 - eps) * (theta_Pt / rho_Pt) / den
    return eps_N, eps_C, eps_Pt


def pt_loading(eps_Pt: float, rho_Pt_mg_cm3: float, thickness_cm: float) -> float:
    """Pt load in mg/cm^2, Eq. (5)."""
    return eps_Pt * rho_Pt_mg_cm3 * thickness_cm


# ----------------------------------------------------------------- helpers

def _count6(mask: np.ndarray) -> np.ndarray:
    """Number of face neighbours in ``mask`` (periodic y, z; bounded x)."""
    m = mask.astype(np.int8)
    n = np.zeros(mask.shape, np.int8)
    n[:, :, 1:] += m[:, :, :-1]
    n[:, :, :-1] += m[:, :, 1:]
    for ax in (0, 1):
        n += np.roll(m, 1, axis=ax)
        n += np.roll(m, -1, axis=ax)
    return n


def _take_exact(rng, accept: np.ndarray, remaining: int) -> np.ndarray:
    """Keep a uniformly random subset of size ``remaining`` of the True cells."""
    idx = np.flatnonzero(accept)
    if len(idx) <= remaining:
        return accept
    keep = rng.choice(idx, size=remaining, replace=False)
    out = np.zeros(accept.size, bool)
    out[keep] = True
    return out.reshape(accept.shape)


def _grow(rng, grown: np.ndarray, source: np.ndarray, bond: np.ndarray, free: np.ndarray,
          p_grow: float, target: int, max_sweeps: int = 100000) -> np.ndarray:
    """QSGS growth sweeps until ``grown`` has ``target`` cells.

    Each source cell A tries to grow into each free face neighbour B.  The attempt
    succeeds outright if another of B's neighbours (other than A) is a bond cell
    (rule 2a), otherwise with probability p_grow (rule 2b).  B is accepted if any
    attempt succeeds.  With n_src source and n_bond bond neighbours of B this is:
    n_bond >= 2, or n_bond == 1 with another source neighbour -> certain; else
    1 - (1 - p)^n_src."""
    grown = grown.copy()
    for _ in range(max_sweeps):
        have = int(grown.sum())
        if have >= target:
            break
        src = source | grown
        bnd = bond | grown
        n_src = _count6(src)
        n_bond = _count6(bnd)
        cand = free & ~grown & (n_src > 0)
        if not cand.any():
            break
        certain = (n_bond >= 2) | ((n_bond == 1) & (n_src >= 2))
        p_acc = np.where(certain, 1.0, 1.0 - (1.0 - p_grow) ** n_src.astype(np.float64))
        u = rng.random(grown.shape)
        acc = cand & (u < p_acc)
        acc = _take_exact(rng, acc, target - have)
        grown |= acc
    return grown


# ----------------------------------------------------------------- reconstruction steps

def qsgs_carbon(rng, shape, c_d: float, p_grow: float, frac: float) -> np.ndarray:
    """Carbon by QSGS (Section 2.1.2.1): seeds with probability c_d, grown to ``frac``."""
    N = int(np.prod(shape))
    target = int(round(frac * N))
    u = rng.random(shape)
    seeds = u <= c_d
    if seeds.sum() > target:
        seeds = _take_exact(rng, seeds, target)
    if seeds.sum() == 0 and target > 0:
        seeds.flat[rng.integers(N)] = True
    free = np.ones(shape, bool)
    return _grow(rng, seeds, seeds, seeds, free, p_grow, target)


def disperse_pt(rng, phase: np.ndarray, p_face: float) -> np.ndarray:
    """Pt on the carbon surface (Section 2.1.2.2): every carbon-pore face is selected
    with probability p_face; a carbon voxel with a selected face becomes Pt."""
    carbon = phase == CARBON
    pore = phase == PORE
    m = _count6(pore).astype(np.float64)
    p = 1.0 - (1.0 - p_face) ** m
    u = rng.random(phase.shape)
    out = phase.copy()
    out[carbon & (m > 0) & (u < p)] = PT
    return out


def qsgs_ionomer(rng, phase: np.ndarray, p_grow: float, frac: float) -> np.ndarray:
    """Ionomer by QSGS from the solid (Section 2.1.2.3): C/Pt cells act as seeds,
    growth into pore cells, rule 2a counting ionomer neighbours only."""
    N = phase.size
    target = int(round(frac * N))
    solid = (phase == CARBON) | (phase == PT)
    ion0 = phase == IONOMER
    ion = _grow(rng, ion0, solid, np.zeros_like(ion0), phase == PORE, p_grow, target)
    out = phase.copy()
    out[ion & ~ion0] = IONOMER
    return out


_BALLS: dict = {}


def _ball(d: int) -> np.ndarray:
    """Offsets of voxels whose centres lie within d/2 of the centre voxel."""
    if d not in _BALLS:
        r = d / 2.0
        R = int(math.ceil(r))
        g = np.arange(-R, R + 1)
        z, y, x = np.meshgrid(g, g, g, indexing="ij")
        sel = (x * x + y * y + z * z) <= r * r + 1e-9
        _BALLS[d] = np.stack([z[sel], y[sel], x[sel]], axis=1)
    return _BALLS[d]


def carve_internal_pores(rng, phase: np.ndarray, frac: float, d_min: int, d_max: int) -> np.ndarray:
    """Carve spherical pores of diameter U{d_min..d_max} voxels inside carbon until
    ``frac`` of the volume has been turned to pore (Section 5.3).  Only carbon voxels
    with no ionomer face neighbour are carved, so the solid-ionomer contact is kept."""
    out = phase.copy()
    nz, ny, nx = phase.shape
    target = int(round(frac * phase.size))
    done = 0
    ion_adj = _count6(phase == IONOMER) > 0
    eligible = (out == CARBON) & ~ion_adj
    while done < target:
        cand = np.flatnonzero(eligible)
        if len(cand) == 0:
            break
        batch = min(len(cand), max(1, (target - done) // max(1, len(_ball(d_min)))))
        centres = rng.choice(cand, size=min(batch, 4096), replace=False)
        diam = rng.integers(d_min, d_max + 1, size=len(centres))
        for c, d in zip(centres, diam):
            if done >= target:
                break
            cz, rem = divmod(int(c), ny * nx)
            cy, cx = divmod(rem, nx)
            off = _ball(int(d))
            zz = (cz + off[:, 0]) % nz
            yy = (cy + off[:, 1]) % ny
            xx = cx + off[:, 2]
            ok = (xx >= 0) & (xx < nx)
            zz, yy, xx = zz[ok], yy[ok], xx[ok]
            sel = eligible[zz, yy, xx]
            zz, yy, xx = zz[sel], yy[sel], xx[sel]
            take = min(len(zz), target - done)
            zz, yy, xx = zz[:take], yy[:take], xx[:take]
            out[zz, yy, xx] = PORE
            eligible[zz, yy, xx] = False
            done += take
    return out


def percolates(phase: np.ndarray, transport_phases=(PORE, IONOMER)) -> bool:
    """True if a face-connected path of transport voxels joins x = 0 to x = nx-1
    (used only to resample unusable random structures)."""
    from scipy import ndimage

    t = np.isin(phase, transport_phases)
    lab, _ = ndimage.label(t)
    a = set(np.unique(lab[:, :, 0])) - {0}
    b = set(np.unique(lab[:, :, -1])) - {0}
    return bool(a & b)


# ----------------------------------------------------------------- workloads

def two_phase(seed: int, n: int = 32, c_d: float = 0.01, p_grow: float = 0.02, porosity: float = 0.5,
              shape=None) -> np.ndarray:
    """Two-phase QSGS structure (pore / impermeable carbon), grown to ``porosity``."""
    rng = np.random.default_rng([seed, 1])
    shape = shape or (n, n, n)
    carbon = qsgs_carbon(rng, shape, c_d, p_grow, 1.0 - porosity)
    return np.where(carbon, CARBON, PORE).astype(np.uint8)


def pt_cl(seed: int, n: int = 128, carbon: float = 0.35, ionomer: float = 0.20, pt_faces: float = 0.10,
          c_d: float = 0.01, p_carbon: float = 0.02, p_ionomer: float = 0.5, shape=None) -> np.ndarray:
    """Four-phase Pt catalyst layer: QSGS carbon (C + Pt = ``carbon``), Pt on
    ``pt_faces`` of the carbon-pore faces, QSGS ionomer to ``ionomer``, rest pore."""
    rng = np.random.default_rng([seed, 2])
    shape = shape or (n, n, n)
    c = qsgs_carbon(rng, shape, c_d, p_carbon, carbon)
    ph = np.where(c, CARBON, PORE).astype(np.uint8)
    ph = disperse_pt(rng, ph, pt_faces)
    ph = qsgs_ionomer(rng, ph, p_ionomer, ionomer)
    return ph


def npmc_cl(seed: int, n: int = 256, carbon_final: float = 0.45, ionomer: float = 0.15,
            micro: float = 0.10, meso: float = 0.05, micro_d=(1, 3), meso_d=(20, 40),
            c_d: float = 0.01, p_carbon: float = 0.02, p_ionomer: float = 0.5, shape=None) -> np.ndarray:
    """Non-precious-metal catalyst layer: carbon grown to carbon_final + micro + meso,
    ionomer grown from it, then meso- and micropores carved inside the carbon."""
    rng = np.random.default_rng([seed, 3])
    shape = shape or (n, n, n)
    c = qsgs_carbon(rng, shape, c_d, p_carbon, carbon_final + micro + meso)
    ph = np.where(c, CARBON, PORE).astype(np.uint8)
    ph = qsgs_ionomer(rng, ph, p_ionomer, ionomer)
    ph = carve_internal_pores(rng, ph, meso, *meso_d)
    ph = carve_internal_pores(rng, ph, micro, *micro_d)
    return ph


def batch_instances(master_seed: int = 2024, count: int = 64, edges=(48, 64, 96, 128, 160),
                    porosity=(0.3, 0.7), k_range=(1e-4, 1e-1), max_edge=None, first: int = 0):
    """Uneven batch of Pt-CL-like structures: edge uniform over ``edges``, porosity
    uniform, carbon:ionomer = 0.35:0.20 of the non-pore volume, Pt on 10% of the
    carbon-pore faces, first-order rate k log-uniform over ``k_range`` (lattice
    units).  Instance i uses seed master_seed*1000 + i; unusable draws (no x-spanning
    transport path) are resampled with the next attempt number.  Instances first ..
    first + count - 1 are made (each depends on its index only)."""
    out = []
    for i in range(first, first + count):
        rng = np.random.default_rng([master_seed, i])
        attempt = 0
        while True:
            e = int(rng.choice([x for x in edges if max_edge is None or x <= max_edge]))
            eps = float(rng.uniform(*porosity))
            k = float(math.exp(rng.uniform(math.log(k_range[0]), math.log(k_range[1]))))
            solid = 1.0 - eps
            ph = pt_cl(master_seed * 1000 + i + 100000 * attempt, n=e,
                       carbon=solid * 0.35 / 0.55, ionomer=solid * 0.20 / 0.55)
            if percolates(ph):
                break
            attempt += 1
        out.append({"index": i, "edge": e, "porosity": eps, "k": k, "phase": ph})
    return out


def random_state(seed: int, shape, scale: float = 1.0, offset: float = 0.0, dtype=np.float32) -> np.ndarray:
    """Seeded random populations (7, nz, ny, nx) for one-step parity checks."""
    rng = np.random.default_rng([seed, 7])
    return (offset + scale * rng.random((7,) + tuple(shape))).astype(dtype)
