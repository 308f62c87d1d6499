"""Seeded synthetic catalyst-layer structures: the shared input generator.

This package only produces inputs (voxel phase maps and per-instance parameters);
it holds none of the solver's arithmetic.  The tests, the benchmark and the oracle
callers all draw their structures from here, so the oracle and the HIP path see
identical inputs.

Phase ids: 0 pore, 1 carbon, 2 Pt, 3 ionomer.  Arrays are (nz, ny, nx), x fastest.

Reconstruction follows Chen et al., arXiv 1410.1914, Section 2.1.2:

* quartet structure generation set (QSGS) for carbon: seeds with probability c_d,
  then growth into face neighbours; a neighbour is accepted outright when another
  of its own neighbours already belongs to the growing phase (rule 2a), otherwise
  with probability P_alpha (rule 2b), repeated until the target fraction;
* Pt dispersed on the carbon surface (Section 2.1.2.2);
* QSGS for the ionomer, grown from the solid (Section 2.1.2.3);
* internal micro- and mesopores carved inside the solid, never touching the
  ionomer (Section 5.3).

Readings of unstated details: a seeded PCG64 generator; snapshot sweeps (every
decision in a sweep sees the state at the start of the sweep); the sweep that
would overshoot the target accepts a random subset so the count is exact; y and z
are periodic and x is bounded; the Pt fraction is carved out of the carbon (one Pt
voxel for every carbon voxel with at least one selected pore face).
"""
from .qsgs import (  # noqa: F401
    PORE, CARBON, PT, IONOMER,
    volume_fractions, pt_loading,
    qsgs_carbon, disperse_pt, qsgs_ionomer, carve_internal_pores,
    percolates, two_phase, pt_cl, npmc_cl, batch_instances, random_state,
)
