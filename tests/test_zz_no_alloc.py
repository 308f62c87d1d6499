"""The allocation-free reach (lbm_reach_device_static) against lbm_reach_device.

Both entry points run the same sweeps; the static variant keeps the sweeps' change
flag in the library's fixed device array instead of freshly allocated pinned host
memory.  Two calls in a row, the second on a smaller map, must each give the same
reach mask (bit for bit) and the same cycle count as lbm_reach_device, and the
second call must not see anything the first left in the shared array.  Run last
and alone in a fresh process alike."""
import numpy as np
import pytest

import structgen as sg
from oracle import lbm as O

pytestmark = pytest.mark.gpu

CASES = [  # (structure, faces): a large map first, then a smaller one
    (("npmc", 11, (48, 40, 130)), 3),
    (("pt", 12, (9, 10, 70)), 1),
]


def _map(kind, seed, shape):
    if kind == "npmc":
        ph = sg.npmc_cl(seed, shape=shape, meso_d=(3, 6))
    else:
        ph = sg.pt_cl(seed, shape=shape)
    return (ph == O.PORE) | (ph == O.IONOMER)


def _seed(shape, faces):
    s = np.zeros(shape, bool)
    if faces & 1:
        s[:, :, 0] = True
    if faces & 2:
        s[:, :, -1] = True
    return s


def test_static_reach_matches_the_allocating_entry_point_twice(hip):
    import torch

    for (kind, seed, shape), faces in CASES:
        print(f"reach static: {kind} seed {seed} shape {shape} faces {faces}", flush=True)
        passm = _map(kind, seed, shape)
        want, want_cycles = hip.reach_device(passm, faces)
        # the output buffer starts with stale ones everywhere: every voxel must be written
        out = torch.ones(shape, dtype=torch.uint8, device="cuda")
        got, got_cycles = hip.reach_device(passm, faces, out=out, static_scratch=True)
        torch.cuda.synchronize()
        assert got.data_ptr() == out.data_ptr()
        assert torch.equal(got, want)
        assert got_cycles == want_cycles
        # and both equal the oracle's flood fill
        assert np.array_equal(got.cpu().numpy().astype(bool), O.flood(passm, _seed(shape, faces) & passm))


def test_static_reach_rejects_bad_arguments(hip):
    import ctypes

    lib = hip.load()
    cyc = ctypes.c_int32()
    assert lib.lbm_reach_device_static(None, 4, 4, 4, 3, None, ctypes.byref(cyc), None) == hip.ERR_INVALID_ARG
