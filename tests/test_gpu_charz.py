"""Structure characterisation on the device (Section 2.1.3) against the oracle.

* lbm_pore_size_device: the 13-direction pore size, bit-identical to the oracle's
  FP64 chords (same directions, same order, round-to-nearest arithmetic).
* lbm_reach_device: the voxels of a phase connected to the x faces, identical to
  the oracle's breadth-first flood fill, and equal to the solver's own mask of
  simulated voxels.
Small structures cover wrapped rows and planes, ragged x ranges, closed all-pore
loops and empty phases; the 256^3 NPMC structure is the full benchmark size.
"""
import numpy as np
import pytest

import structgen as sg
from oracle import lbm as O

pytestmark = pytest.mark.gpu

SHAPES = [
    ("pt", 1, (9, 10, 70)),
    ("npmc", 2, (12, 12, 65)),
    ("two", 3, (16, 16, 32)),
    ("pt", 9, (1, 1, 150)),    # one row: y and z neighbours are the row itself
    ("pt", 10, (2, 1, 66)),
    ("two", 5, (7, 5, 9)),     # y and z loops of different lengths (lcm 35)
]


def _phase(kind, seed, shape):
    if kind == "pt":
        return sg.pt_cl(seed, shape=shape)
    if kind == "npmc":
        return sg.npmc_cl(seed, shape=shape, meso_d=(3, 6))
    return sg.two_phase(seed, shape=shape)


def _faces_seed(shape, faces):
    seed = np.zeros(shape, bool)
    if faces & 1:
        seed[:, :, 0] = True
    if faces & 2:
        seed[:, :, -1] = True
    return seed


@pytest.mark.parametrize("kind,seed,shape", SHAPES)
def test_pore_size_matches_the_oracle_bit_for_bit(hip, kind, seed, shape):
    pore = _phase(kind, seed, shape) == O.PORE
    got = hip.pore_size_device(pore).cpu().numpy()
    want = O.pore_chords(pore)
    assert np.array_equal(got, want)
    assert (got[~pore] == 0).all() and (got[pore] >= 1.0).all()


def test_pore_size_of_closed_loops_and_empty_maps(hip):
    full = np.ones((5, 7, 9), bool)  # every y/z line closes on itself
    got = hip.pore_size_device(full).cpu().numpy()
    assert np.array_equal(got, O.pore_chords(full))
    none = np.zeros((3, 4, 70), bool)
    assert not hip.pore_size_device(none).cpu().numpy().any()


@pytest.mark.parametrize("kind,seed,shape", SHAPES)
@pytest.mark.parametrize("faces", [1, 2, 3])
def test_reach_matches_the_oracle_flood(hip, kind, seed, shape, faces):
    ph = _phase(kind, seed, shape)
    transport = (ph == O.PORE) | (ph == O.IONOMER)
    got, cycles = hip.reach_device(transport, faces)
    want = O.flood(transport, _faces_seed(shape, faces))
    assert np.array_equal(got.cpu().numpy().astype(bool), want)
    assert cycles >= 1


def test_reach_of_full_and_empty_phases(hip):
    full = np.ones((4, 5, 70), bool)
    got, cycles = hip.reach_device(full, 1)
    assert got.cpu().numpy().all() and cycles >= 1
    got, _ = hip.reach_device(np.zeros((4, 5, 70), bool), 3)
    assert not got.cpu().numpy().any()


def test_reach_equals_the_solvers_simulated_mask(hip):
    """The D_eff problem simulates exactly the transport voxels reached from either
    Dirichlet face."""
    ph = sg.pt_cl(12, shape=(10, 11, 75))
    h = hip.lbm_create(ph, hip.lbm_params_default(mode=hip.MODE_DEFF))
    act, _, _ = hip.lbm_get_host_fields(h)
    hip.lbm_destroy(h)
    got, _ = hip.reach_device((ph == O.PORE) | (ph == O.IONOMER), 3)
    assert np.array_equal(got.cpu().numpy().astype(bool), act.astype(bool))


def test_full_size_npmc_256(hip):
    """The 256^3 NPMC catalyst layer of the benchmark: pore size and reach."""
    ph = sg.npmc_cl(1, n=256)
    pore = ph == O.PORE
    assert np.array_equal(hip.pore_size_device(pore).cpu().numpy(), O.pore_chords(pore))
    transport = pore | (ph == O.IONOMER)
    got, cycles = hip.reach_device(transport, 3)
    print(f"[charz] 256^3 reach: {cycles} sweep cycles", flush=True)
    assert np.array_equal(got.cpu().numpy().astype(bool), O.flood(transport, _faces_seed(ph.shape, 3)))


PREP_CASES = [
    ("pt", 1, (9, 10, 70), dict(mode=0, knudsen=1)),
    ("pt", 4, (8, 7, 130), dict(mode=1, knudsen=1, k_lat=0.02)),
    ("pt", 6, (6, 5, 64), dict(mode=2)),
    ("npmc", 2, (12, 12, 65), dict(mode=1, knudsen=1, k_lat=0.01, catalyst_phases=(1 << 1) | (1 << 2))),
    ("two", 3, (16, 16, 32), dict(mode=0, knudsen=0, tau_ref=0.8)),
    ("pt", 9, (1, 1, 150), dict(mode=0, knudsen=1)),
]


def _host_state(hip, h):
    info = hip.lbm_get_info(h)
    act, ncat, om = hip.lbm_get_host_fields(h)
    return info, act, ncat, om


@pytest.mark.parametrize("kind,seed,shape,kw", PREP_CASES)
def test_create_with_device_preparation_is_bit_identical(hip, kind, seed, shape, kw):
    """lbm_create_device (pore size and reach on the GPU) gives the handle
    lbm_create gives: the same sizes and reference values, bit-identical host
    fields, and bit-identical steps from the cold start."""
    import torch

    ph = _phase(kind, seed, shape)
    p = hip.lbm_params_default(**kw)
    a = hip.lbm_create(ph, p, 2e-9)
    b = hip.lbm_create(ph, p, 2e-9, device_prep=True)
    ia, *fa = _host_state(hip, a)
    ib, *fb = _host_state(hip, b)
    hip.lbm_destroy(a)
    hip.lbm_destroy(b)
    for f in ("nx", "ny", "nz", "n_active", "n_segments", "percolates", "d0", "d_ref", "d0_lat"):
        assert getattr(ia, f) == getattr(ib, f), f
    for x, y in zip(fa, fb):
        assert np.array_equal(x, y)
    s1, s2 = hip.Solver(ph, p), hip.Solver(ph, p, device_prep=True)
    s1.step(7)
    s2.step(7)
    assert torch.equal(s1.populations(), s2.populations())


def test_batch_create_with_device_preparation_is_bit_identical(hip):
    phases = [sg.pt_cl(2024000 + i, shape=(e, e, e)) for i, e in enumerate((24, 40, 16, 32))]
    params = [hip.lbm_params_default(mode=1, knudsen=1, k_lat=10 ** -(i + 1)) for i in range(4)]
    a = hip.Batch(phases, params)
    b = hip.Batch(phases, params, device_prep=True)
    for i in range(4):
        for x, y in zip(a.host_fields(i), b.host_fields(i)):
            assert np.array_equal(x, y), i


def test_device_preparation_of_the_256_cube():
    """The benchmark structure: identical fields, and the time of both routes."""
    import time

    from paper_1410_1914_amd import lbm as hip

    hip.require_gpu()
    ph = sg.npmc_cl(1, n=256)
    p = hip.lbm_params_default(mode=1, knudsen=1, k_lat=1e-4, catalyst_phases=(1 << O.CARBON) | (1 << O.PT))
    hip.lbm_destroy(hip.lbm_create(ph[:8], p, 1e-9, device_prep=True))  # first device use
    t0 = time.perf_counter()
    a = hip.lbm_create(ph, p, 1e-9)
    t1 = time.perf_counter()
    b = hip.lbm_create(ph, p, 1e-9, device_prep=True)
    t2 = time.perf_counter()
    print(f"[prep] 256^3 NPMC: host lbm_create {t1 - t0:.2f}s, lbm_create_device {t2 - t1:.2f}s", flush=True)
    ia, *fa = _host_state(hip, a)
    ib, *fb = _host_state(hip, b)
    hip.lbm_destroy(a)
    hip.lbm_destroy(b)
    assert ia.n_active == ib.n_active
    for x, y in zip(fa, fb):
        assert np.array_equal(x, y)


_FIRST_USE = r"""
import sys
sys.path.insert(0, sys.argv[1])
import numpy as np
import structgen as sg
from oracle import lbm as O
from paper_1410_1914_amd import lbm as hip

hip.require_gpu()
ph = sg.npmc_cl(1, n=256)
p = hip.lbm_params_default(mode=1, knudsen=1, k_lat=1e-4, catalyst_phases=(1 << O.CARBON) | (1 << O.PT))
b = hip.lbm_create(ph, p, 1e-9, device_prep=True)  # the process's first device call
a = hip.lbm_create(ph, p, 1e-9)
fa, fb = hip.lbm_get_host_fields(a), hip.lbm_get_host_fields(b)
assert all(np.array_equal(x, y) for x, y in zip(fa, fb))
print("first-use device preparation: OK,", hip.lbm_get_info(b).n_active, "simulated voxels", flush=True)
"""


def test_device_preparation_as_the_first_device_call_of_a_process():
    """The 256^3 benchmark structure prepared with device assistance as the very
    first device work of a fresh process (no earlier copy or kernel has set up the
    runtime), bit-identical to the host route."""
    import os
    import subprocess
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", _FIRST_USE, root], capture_output=True, text=True, timeout=600)
    print(r.stdout[-2000:], r.stderr[-2000:], flush=True)
    assert r.returncode == 0
    assert "first-use device preparation: OK" in r.stdout
