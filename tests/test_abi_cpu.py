"""C ABI on the CPU: the library loads, exports every declared symbol, and its host
preprocessing matches the oracle bit for bit (no device call is made here)."""
import os
import re

import numpy as np
import pytest

import structgen as sg
from oracle import lbm as O
from paper_1410_1914_amd import lbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared(header):
    text = open(os.path.join(ROOT, "include", header)).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm(?:19)?_\w+|unet_\w+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = lbm.load()
    names = _declared("lbm.h")
    assert len(names) >= 25
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(lbm.SIGNATURES)


def test_params_default_and_status_strings():
    p = lbm.lbm_params_default()
    assert p.struct_size == 200 or p.struct_size == __import__("ctypes").sizeof(lbm.lbm_params)
    assert p.w0 == 0.25 and p.tau_ref == 1.0 and p.check_every % 2 == 0
    for st in (0, 1, -1, -2, -3, -4, -5, -6, -7, -8, -9):
        assert lbm.lbm_status_string(st)
    assert lbm.lbm_status_string(12345) == "unknown status"


CASES = [
    ("pt", 1, (9, 10, 70), dict(knudsen=1)),
    ("pt", 4, (8, 6, 130), dict(knudsen=1, d_ionomer_rel=0.05)),
    ("pt", 8, (5, 6, 10), dict(knudsen=0)),
    ("npmc", 2, (12, 12, 65), dict(knudsen=1, voxel_m=1e-9)),
    ("two", 3, (16, 16, 32), dict(knudsen=0, tau_ref=0.8)),
]


def _phase(kind, seed, shape):
    if kind == "pt":
        return sg.pt_cl(seed, shape=shape)
    if kind == "npmc":
        return sg.npmc_cl(seed, shape=shape, meso_d=(3, 6))
    return sg.two_phase(seed, shape=shape)


@pytest.mark.parametrize("kind,seed,shape,kw", CASES)
@pytest.mark.parametrize("mode", [lbm.MODE_DEFF, lbm.MODE_REACT, lbm.MODE_PROTON])
def test_host_preprocessing_matches_oracle(kind, seed, shape, kw, mode):
    ph = _phase(kind, seed, shape)
    voxel = kw.get("voxel_m", 2e-9)
    cat = (1 << lbm.PT) | (1 << lbm.CARBON) if kind == "npmc" else (1 << lbm.PT)
    p = lbm.lbm_params_default(mode=mode, k_lat=0.05, catalyst_phases=cat,
                               **{k: v for k, v in kw.items() if k != "voxel_m"})
    h = lbm.lbm_create(ph, p, voxel)
    try:
        info = lbm.lbm_get_info(h)
        act, ncat, om = lbm.lbm_get_host_fields(h)
    finally:
        lbm.lbm_destroy(h)
    op = O.Params(mode=mode, knudsen=bool(kw.get("knudsen")), voxel_m=voxel, k_lat=0.05, catalyst_phases=cat,
                  tau_ref=kw.get("tau_ref", 1.0), d_ionomer_rel=kw.get("d_ionomer_rel", 1e-3))
    prob = O.prepare(ph, op)
    assert (info.nz, info.ny, info.nx) == prob.active.shape
    assert np.array_equal(act.astype(bool), prob.active)          # index work: bit exact
    assert np.array_equal(ncat.astype(np.int64), prob.n_cat)
    assert info.n_active == int(prob.active.sum())
    assert bool(info.percolates) == prob.percolates
    assert info.d_ref == pytest.approx(prob.D_ref, rel=1e-15)
    assert info.d0 == pytest.approx(prob.D0, rel=1e-15)
    assert info.d0_lat == pytest.approx(O.d0_lattice(prob), rel=1e-14)
    # relaxation rates: FP32 rounding of the FP64 value
    assert np.array_equal(om, prob.omega.astype(np.float32))


def test_pore_size_matches_oracle_on_knudsen_structure():
    """The library's run-length chord scan and the oracle's per-voxel walk agree
    (checked through 1/tau, which is a strictly monotone function of d_p here)."""
    ph = sg.npmc_cl(5, shape=(20, 18, 40), meso_d=(4, 8))
    p = lbm.lbm_params_default(knudsen=1, d_ionomer_rel=1e-3)
    h = lbm.lbm_create(ph, p, 1e-9)
    _, _, om = lbm.lbm_get_host_fields(h)
    lbm.lbm_destroy(h)
    prob = O.prepare(ph, O.Params(knudsen=True, voxel_m=1e-9))
    assert np.array_equal(om, prob.omega.astype(np.float32))


def test_error_codes():
    ph = np.zeros((4, 4, 8), np.uint8)
    bad = ph.copy()
    bad[0, 0, 0] = 7
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_create(bad, lbm.lbm_params_default())
    assert e.value.status == lbm.ERR_BAD_PHASE
    for kw in (dict(tau_ref=0.5), dict(w0=0.0), dict(check_every=3), dict(k_lat=-1.0), dict(struct_size=4),
               dict(mode=7)):
        with pytest.raises(lbm.LbmError) as e:
            lbm.lbm_create(ph, lbm.lbm_params_default(**kw))
        assert e.value.status == lbm.ERR_INVALID_ARG, kw
    cat = np.zeros((4, 2, 8), np.uint8)
    cat[:, 0, :] = lbm.PT  # the fluid row has Pt on both y sides: n = 2
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_create(cat, lbm.lbm_params_default(mode=lbm.MODE_REACT, k_lat=0.6))  # k n = 1.2 >= 1
    assert e.value.status == lbm.ERR_UNSTABLE
    h = lbm.lbm_create(ph, lbm.lbm_params_default())
    try:
        with pytest.raises(lbm.LbmError) as e:
            lbm.lbm_step(h, 1)
        assert e.value.status == lbm.ERR_UNBOUND
        st, _ = lbm.lbm_deff(h)
        assert st == lbm.ERR_UNBOUND or st == lbm.ERR_NO_PERCOLATION
    except lbm.LbmError as err:
        assert err.status == lbm.ERR_UNBOUND
    finally:
        lbm.lbm_destroy(h)
    lbm.lbm_destroy(None)


def test_no_percolation_flag():
    ph = np.zeros((3, 3, 8), np.uint8)
    ph[:, :, 4] = lbm.CARBON
    h = lbm.lbm_create(ph, lbm.lbm_params_default())
    assert lbm.lbm_get_info(h).percolates == 0
    lbm.lbm_destroy(h)


def test_segment_count_and_reservoir_plane():
    ph = sg.pt_cl(2, shape=(4, 5, 130))
    h = lbm.lbm_create(ph, lbm.lbm_params_default(mode=lbm.MODE_REACT, k_lat=0.01))
    i = lbm.lbm_get_info(h)
    assert (i.nx, i.nx_struct) == (131, 130)
    assert i.n_segments == 3 * 5 * 4
    lbm.lbm_destroy(h)


def _flat_windows(nx, ny, nz):
    """Windows of the flat layout by brute force: consecutive grid indices, cut
    at every plane start and at the starts of rows 1 and ny - 1, 64 at most."""
    starts = set()
    for z in range(nz):
        for y in {0, min(1, ny - 1), max(min(1, ny - 1), ny - 1)}:
            starts.add((z * ny + y) * nx)
    wins, cur = [], None
    for v in range(nx * ny * nz):
        if v in starts or cur is None or v - cur[0] == 64:
            cur = [v, 0]
            wins.append(cur)
        cur[1] += 1
    return wins


@pytest.mark.parametrize("shape,mode", [((5, 7, 64), 1), ((3, 1, 128), 1), ((4, 2, 64), 1), ((3, 3, 193), 0),
                                        ((5, 7, 64), 0), ((2, 3, 130), 1)])
def test_segment_windows_of_both_layouts(shape, mode):
    """Rows of 64 k + 1 voxels give flat windows (counted by brute force), others
    one window per 64 voxels of each row; n_listed counts those holding simulated
    voxels."""
    ph = sg.pt_cl(3, shape=shape)
    h = lbm.lbm_create(ph, lbm.lbm_params_default(mode=mode, k_lat=0.01))
    i = lbm.lbm_get_info(h)
    act, _, _ = lbm.lbm_get_host_fields(h)
    lbm.lbm_destroy(h)
    nx, ny, nz = i.nx, i.ny, i.nz
    if nx > 64 and nx % 64 == 1:
        wins = _flat_windows(nx, ny, nz)
    else:
        wins = [[(r * nx) + s0, min(64, nx - s0)] for r in range(ny * nz) for s0 in range(0, nx, 64)]
    assert i.n_segments == len(wins)
    flat = act.ravel()
    assert i.n_listed == sum(bool(flat[v0:v0 + n].any()) for v0, n in wins)


def _depth_reference(phase_sim, active, react):
    """Breadth-first distances, written out plainly: seeds are pore voxels joined to
    a Dirichlet face through pore voxels (6-neighbours, periodic y and z)."""
    from collections import deque

    nz, ny, nx = active.shape
    pore = active & (phase_sim == sg.PORE)

    def nbrs(z, y, x):
        if x > 0:
            yield z, y, x - 1
        if x + 1 < nx:
            yield z, y, x + 1
        yield z, (y - 1) % ny, x
        yield z, (y + 1) % ny, x
        yield (z - 1) % nz, y, x
        yield (z + 1) % nz, y, x

    joined = np.zeros_like(pore)
    q = deque()
    faces = [0] if react else [0, nx - 1]
    for z in range(nz):
        for y in range(ny):
            for x in faces:
                if pore[z, y, x] and not joined[z, y, x]:
                    joined[z, y, x] = True
                    q.append((z, y, x))
    while q:
        v = q.popleft()
        for t in nbrs(*v):
            if pore[t] and not joined[t]:
                joined[t] = True
                q.append(t)
    depth = np.full(active.shape, 255, np.int64)
    depth[joined] = 0
    q = deque(zip(*np.nonzero(joined)))
    while q:
        v = q.popleft()
        for t in nbrs(*v):
            if active[t] and depth[t] == 255 and depth[v] + 1 <= 254:
                depth[t] = depth[v] + 1
                q.append(t)
    return depth


@pytest.mark.parametrize("mode,seed", [(lbm.MODE_REACT, 3), (lbm.MODE_DEFF, 4), (lbm.MODE_REACT, 11)])
def test_pore_depth_matches_breadth_first_search(mode, seed):
    ph = sg.pt_cl(seed, shape=(6, 7, 24))
    h = lbm.lbm_create(ph, lbm.lbm_params_default(mode=mode, k_lat=0.01 if mode == lbm.MODE_REACT else 0.0))
    act, _, _ = lbm.lbm_get_host_fields(h)
    depth = lbm.lbm_get_pore_depth(h)
    lbm.lbm_destroy(h)
    react = mode == lbm.MODE_REACT
    phs = np.concatenate([np.zeros(ph.shape[:2] + (1,), np.uint8), ph], axis=2) if react else ph
    want = _depth_reference(phs, act.astype(bool), react)
    assert np.array_equal(depth.astype(np.int64), want)
    assert (depth[act.astype(bool)] < 255).any() and (depth[~act.astype(bool)] == 255).all()
    assert set(np.unique(depth[act.astype(bool)])) > {0, 1}


def test_batch_entry_points_reject_bad_arguments():
    """Host-side checks of the batched entry points (no device call is made)."""
    phases = [sg.pt_cl(60 + i, shape=(4, 5, 20)) for i in range(2)]
    params = [lbm.lbm_params_default(mode=lbm.MODE_REACT, k_lat=0.01) for _ in phases]
    h = lbm.lbm_batch_create(phases, params)
    lib = lbm.load()
    assert lib.lbm_batch_set_group_bytes(h, -1) == lbm.ERR_INVALID_ARG
    assert lib.lbm_batch_set_group_bytes(h, 0) == lbm.OK
    assert lib.lbm_batch_set_group_bytes(h, 1 << 20) == lbm.OK
    assert lib.lbm_batch_set_group_bytes(None, 1) == lbm.ERR_INVALID_ARG
    assert lib.lbm_batch_advance(h, -5, None) == lbm.ERR_INVALID_ARG
    assert lib.lbm_batch_advance(None, 5, None) == lbm.ERR_INVALID_ARG
    # stepping before a workspace is bound is refused, not attempted
    assert lib.lbm_batch_advance(h, 5, None) == lbm.ERR_UNBOUND
    assert lib.lbm_batch_get_pore_depth(h, 2, np.zeros(1, np.uint8).ctypes.data_as(
        __import__("ctypes").POINTER(__import__("ctypes").c_uint8))) == lbm.ERR_INVALID_ARG
    lbm.lbm_batch_destroy(h)


def test_temporal_blocking_arguments():
    """Two-step launch settings are checked on the host: 4, 6 or 8 rows per tile (0
    is one step per launch), 1 .. 64 planes per chunk."""
    import ctypes

    h = lbm.lbm_create(sg.pt_cl(61, shape=(4, 5, 20)), lbm.lbm_params_default(mode=lbm.MODE_DEFF))
    lib = lbm.load()
    for by, zc in ((3, 8), (5, 8), (16, 8), (-1, 8), (4, 0), (8, 65)):
        assert lib.lbm_set_temporal(h, by, zc) == lbm.ERR_INVALID_ARG, (by, zc)
    assert lib.lbm_set_temporal(None, 4, 8) == lbm.ERR_INVALID_ARG
    a, b = ctypes.c_int32(), ctypes.c_int32()
    assert lib.lbm_get_temporal(h, ctypes.byref(a), ctypes.byref(b)) == lbm.OK and a.value == 0
    assert lib.lbm_set_temporal(h, 8, 64) == lbm.OK
    assert lbm.lbm_get_temporal(h) == (8, 64)
    assert lib.lbm_set_temporal(h, 0, 0) == lbm.OK  # off; the chunk size is kept
    assert lbm.lbm_get_temporal(h) == (0, 64)
    lbm.lbm_destroy(h)


def test_device_characterisation_rejects_bad_arguments():
    """Host-side checks of the device characterisation calls (no device call is made)."""
    lib = lbm.load()
    fake = 1  # never dereferenced: the checks come first
    assert lib.lbm_pore_size_device(None, 4, 4, 4, fake, None) == lbm.ERR_INVALID_ARG
    assert lib.lbm_pore_size_device(fake, 0, 4, 4, fake, None) == lbm.ERR_INVALID_ARG
    assert lib.lbm_pore_size_device(fake, 4, 4, 4, None, None) == lbm.ERR_INVALID_ARG
    for faces in (0, 4, -1):
        assert lib.lbm_reach_device(fake, 4, 4, 4, faces, fake, None, None) == lbm.ERR_INVALID_ARG
    assert lib.lbm_reach_device(None, 4, 4, 4, 1, fake, None, None) == lbm.ERR_INVALID_ARG
    assert lib.lbm_reach_device(fake, 4, -2, 4, 1, fake, None, None) == lbm.ERR_INVALID_ARG


def test_d3q19_entry_points_on_the_host():
    """lbm19_*: creation, info (D0 in lattice units with c_s^2 = 1/3), workspace
    size and the errors that need no device."""
    L = lbm.load()
    import ctypes

    ph = np.zeros((4, 5, 8), np.uint8)
    ph[:, 0, :] = lbm.CARBON

    def create(phase, **kw):
        p = lbm.lbm_params_default(**kw)
        g = lbm.lbm_grid(phase.shape[2], phase.shape[1], phase.shape[0], 2e-9)
        h = ctypes.c_void_p()
        st = L.lbm19_create(ctypes.byref(g), np.ascontiguousarray(phase).ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                            ctypes.byref(p), ctypes.byref(h))
        return st, h

    st, h = create(ph, tau_ref=0.8)
    assert st == 0
    try:
        info = lbm.lbm_info()
        assert L.lbm19_get_info(h, ctypes.byref(info)) == 0
        assert (info.nx, info.ny, info.nz, info.n_active) == (8, 5, 4, 4 * 4 * 8)
        assert info.d0_lat == pytest.approx((0.8 - 0.5) / 3 * info.d0 / info.d_ref, rel=1e-15)
        n = ctypes.c_size_t()
        assert L.lbm19_workspace_bytes(h, ctypes.byref(n)) == 0
        N, nf = 8 * 5 * 4, 4 * 4 * 8
        # two compact lattices of the simulated voxels (rounded up to 64), the dense
        # bits and voxel-to-compact map, and compact 1/tau and C snapshot
        assert n.value >= 2 * 19 * 4 * 128 + 2 * 4 * N + 2 * 4 * nf
        assert n.value < 2 * 19 * 4 * N + 64 * 1024
        assert L.lbm19_step(h, 1) == lbm.ERR_UNBOUND
        assert L.lbm19_step(h, -1) == lbm.ERR_INVALID_ARG
        d = ctypes.c_double()
        assert L.lbm19_deff(h, ctypes.byref(d)) == lbm.ERR_UNBOUND
        r, j = ctypes.c_double(), ctypes.c_double()
        assert L.lbm19_reaction_rate(h, ctypes.byref(r), ctypes.byref(j)) == lbm.ERR_WRONG_MODE
        assert L.lbm19_bind(h, None, n.value, None) == -8  # LBM_ERR_WORKSPACE
    finally:
        L.lbm19_destroy(h)
    # the same parameter checks as lbm_create
    for kw in (dict(tau_ref=0.5), dict(k_lat=-1.0), dict(struct_size=4), dict(mode=7)):
        assert create(ph, **kw)[0] == lbm.ERR_INVALID_ARG, kw
    bad = ph.copy()
    bad[0, 1, 1] = 9
    assert create(bad)[0] == lbm.ERR_BAD_PHASE
    # no transport path between the faces
    blocked = ph.copy()
    blocked[:, :, 3] = lbm.CARBON
    st, h = create(blocked)
    assert st == 0
    d = ctypes.c_double()
    assert L.lbm19_deff(h, ctypes.byref(d)) == lbm.ERR_NO_PERCOLATION and d.value == 0.0
    L.lbm19_destroy(h)
    L.lbm19_destroy(None)


def test_coupled_entry_points_on_the_host():
    """lbm19_coupled_*: defaults, argument checks and the stability bound, with
    no device call."""
    import ctypes

    L = lbm.load()
    c = lbm.lbm_coupling_default()
    assert (c.k_ref, c.beta, c.gamma, c.phi_m, c.theta, c.max_iter) == (1e-2, 21.3, 1e-3, 0.6, 0.5, 200)
    ph = sg.pt_cl(4, shape=(6, 8, 12))
    ph[:, :, -1][ph[:, :, -1] == lbm.PORE] = lbm.IONOMER
    g = lbm.lbm_grid(12, 8, 6, 2e-9)
    u8 = ph.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))

    def create(p, cp):
        h = ctypes.c_void_p()
        return L.lbm19_coupled_create(ctypes.byref(g), u8, ctypes.byref(p), ctypes.byref(cp), ctypes.byref(h)), h

    st, h = create(lbm.lbm_params_default(mode=lbm.MODE_REACT), c)
    assert st == 0
    n = ctypes.c_size_t()
    assert L.lbm19_coupled_workspace_bytes(h, ctypes.byref(n)) == 0 and n.value > 2 * 19 * 4 * 12 * 8 * 6
    assert L.lbm19_coupled_run(h, None) == lbm.ERR_UNBOUND
    L.lbm19_coupled_destroy(h)
    for kw in (dict(theta=0.0), dict(theta=1.5), dict(tau_phi=0.5), dict(k_ref=0.0), dict(tol_phi=0.0),
               dict(max_iter=0), dict(struct_size=8), dict(gamma=-1.0)):
        assert create(lbm.lbm_params_default(mode=lbm.MODE_REACT), lbm.lbm_coupling_default(**kw))[0] \
            == lbm.ERR_INVALID_ARG, kw
    assert create(lbm.lbm_params_default(mode=lbm.MODE_DEFF), c)[0] == lbm.ERR_INVALID_ARG
    # k n must stay below 1 on a site with six Pt faces at the membrane potential
    assert create(lbm.lbm_params_default(mode=lbm.MODE_REACT),
                  lbm.lbm_coupling_default(k_ref=0.1, phi_m=0.7))[0] == lbm.ERR_UNSTABLE
    # no ionomer at the membrane face: no site is reached by the potential
    dry = ph.copy()
    dry[:, :, -1][dry[:, :, -1] == lbm.IONOMER] = lbm.PORE
    u8 = dry.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    assert create(lbm.lbm_params_default(mode=lbm.MODE_REACT), c)[0] == lbm.ERR_NO_PERCOLATION
    L.lbm19_coupled_destroy(None)


def test_unet_library_exports_every_declared_symbol():
    from paper_1410_1914_amd import unet

    lib = unet.load()
    names = _declared("unet.h")
    assert len(names) >= 30
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(unet.SIGNATURES)


def test_unet_handle_layout_on_the_host():
    """unet_create and the parameter layout need no device: sizes that are not
    multiples of 8 are refused, the flat parameter array holds every tensor in
    forward order without overlap, and a training handle needs more workspace."""
    import ctypes

    from paper_1410_1914_amd import unet

    lib = unet.load()
    h = ctypes.c_void_p()
    for bad in ((12, 16, 16), (0, 8, 8), (8, 8, -8)):
        assert lib.unet_create(*bad, 0, ctypes.byref(h)) == -1
    assert lib.unet_create(8, 8, 8, 0, None) == -1
    total = unet.param_count()
    end = 0
    for t, (name, cin, cout) in enumerate(unet.layer_specs() + [("head", unet.LEVELS[0], 1)]):
        ci, co, wo, wc, bo = unet.param_tensor(t)
        assert (ci, co) == (cin, cout), name
        assert wo >= end and bo >= wo + wc and wo % 64 == 0
        assert wc == (co * unet.unet_kpad(ci) if name != "head" else unet.LEVELS[0])
        end = bo + co
    assert end <= total
    assert lib.unet_param_tensor(15, None, None, None, None, None) == -1
    sizes = []
    for train in (0, 1):
        assert lib.unet_create(16, 16, 24, train, ctypes.byref(h)) == 0
        nb = ctypes.c_size_t()
        assert lib.unet_workspace_bytes(h, ctypes.byref(nb)) == 0
        sizes.append(nb.value)
        # an unbound handle refuses work
        assert lib.unet_forward(h, None, None, None) == -1
        lib.unet_destroy(h)
    assert sizes[1] > sizes[0] > 16 * 16 * 24 * 16 * 2
    lib.unet_destroy(None)


def test_convolution_refuses_bad_operands_without_touching_the_device():
    """unet_conv3d_fwd and unet_conv3d_fwd_cat check their operands before any device
    call: channel counts and strides off their multiples, pointers that are not
    16-byte aligned, an input or weight array of 2 GiB or more (the loads use 32-bit
    offsets), and for the concatenation an odd grid or a missing part are -1.  The
    pointers are never dereferenced."""
    from paper_1410_1914_amd import unet

    lib = unet.load()
    base = 1 << 20  # 16-byte aligned, never read

    def conv(x=base, w=base, y=base, y32=None, ldx=16, offx=0, ldy=16, offy=0, shape=(4, 4, 4), cin=16, cout=16):
        return lib.unet_conv3d_fwd(x, ldx, offx, w, None, y, ldy, offy, y32, *shape, cin, cout, 1, None)

    assert conv(cin=24) == -1 and conv(cout=8) == -1
    assert conv(ldx=20) == -1 and conv(offy=4, ldy=24) == -1 and conv(ldx=16, offx=8) == -1
    for bad in (dict(x=base + 8), dict(w=base + 2), dict(y=base + 4), dict(y32=base + 8)):
        assert conv(**bad) == -1, bad
    # 2 GiB of input: 1024 x 1024 x 64 voxels of 16 BF16 channels; and of weights
    assert conv(shape=(64, 1024, 1024)) == -1
    cout = 16 * 150000  # cout x unet_kpad(16) BF16 weights: 2.15 GB
    assert 2 * cout * unet.unet_kpad(16) >= 1 << 31
    assert conv(cout=cout, ldy=cout) == -1

    # the concatenation form: an even grid, both parts present, x2 aligned
    def cat(shape=(4, 4, 4), cin1=16, cin=48, x2=base, ldx2=32):
        return lib.unet_conv3d_fwd_cat(base, 16, 0, cin1, x2, ldx2, 0, base, None, base, 16, 0, None, *shape, cin,
                                       16, 1, None)

    assert cat(shape=(4, 5, 4)) == -1 and cat(cin1=48) == -1 and cat(cin1=0) == -1
    assert cat(x2=base + 8) == -1 and cat(ldx2=24) == -1 and cat(cin=40) == -1
    # the head form: weights, bias and output required, pointers aligned
    head = lambda x=base, hw=base, out=base: lib.unet_conv3d_fwd_head(x, 16, 0, base, None, hw, base, None, out, 4, 4,
                                                                       4, None)
    assert head(hw=None) == -1 and head(out=None) == -1 and head(x=base + 8) == -1


def test_device_preparation_refuses_a_bad_scratch_without_touching_the_device():
    """lbm_create_device checks the caller's scratch before any device call: a
    misaligned or too small scratch is LBM_ERR_WORKSPACE."""
    import ctypes

    lib = lbm.load()
    ph = np.ascontiguousarray(sg.pt_cl(1, shape=(6, 6, 20)))
    g = lbm.lbm_grid(20, 6, 6, 2e-9)
    p = lbm.lbm_params_default(knudsen=1)
    nb = ctypes.c_size_t()
    assert lib.lbm_prep_scratch_bytes(1, ctypes.byref(g), ctypes.byref(p), ctypes.byref(nb)) == lbm.OK
    assert nb.value >= 10 * 6 * 6 * 20
    h = ctypes.c_void_p()
    u8 = ph.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    assert lib.lbm_create_device(ctypes.byref(g), u8, ctypes.byref(p), 256 + 8, nb.value, None,
                                 ctypes.byref(h)) == lbm.ERR_WORKSPACE
    assert lib.lbm_create_device(ctypes.byref(g), u8, ctypes.byref(p), 256, 16, None,
                                 ctypes.byref(h)) == lbm.ERR_WORKSPACE
    assert not h.value
