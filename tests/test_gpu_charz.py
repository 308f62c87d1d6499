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
