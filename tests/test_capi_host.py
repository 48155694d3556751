"""Host-only checks of the C ABI (no GPU calls): the library loads and
exports every declared symbol; plan tables, geometry and argument errors."""
import ctypes as C

import numpy as np
import pytest

import oracle
import synth
import paper_2605_03531_amd as sdd
from paper_2605_03531_amd import _capi as A


def test_library_exports_every_header_symbol():
    names = sdd.header_functions()
    assert len(names) >= 15
    L = sdd.lib()
    missing = [n for n in names if not hasattr(L, n)]
    assert missing == []
    assert L.sdd_abi_version() == 1


def test_struct_sizes_match_c_layout():
    assert C.sizeof(A.PlanDesc) == 72
    assert C.sizeof(A.Candidate) == 24
    assert C.sizeof(A.DmBest) == 16
    assert C.sizeof(A.DmStats) == 40
    assert C.sizeof(A.DmRange) == 32


def test_tiny_plan_delays_and_geometry():
    w = synth.tiny(oracle.delay_table, with_data=False)
    p = sdd.Plan(w.freqs_mhz, w.t_samp, dm_list=w.dm_list, widths=w.widths)
    np.testing.assert_array_equal(p.delays(0), oracle.delay_table(w.freqs_mhz, w.dm_list, w.t_samp))
    np.testing.assert_array_equal(p.dms(0), w.dm_list)
    spec = oracle.make_plan(w.freqs_mhz, w.t_samp, dm_list=w.dm_list, widths=w.widths)
    assert p.overlap == spec.overlap == 4517
    g = p.geometry(w.nsamp)
    assert g["n_owned"] == 3675 and g["plane_cols"] == [3690] and g["ncells"] == [4]


def test_full_band_delays_bit_exact():
    """All 2048 x 4096 delays of the full-band workload equal the oracle's."""
    f = np.linspace(750.0, 550.0, 4096)
    dms = np.linspace(0.0, 1000.0, 2048)
    p = sdd.Plan(f, 81.92e-6, dm_list=dms)
    d = p.delays(0)
    o = oracle.delay_table(f, dms, 81.92e-6)
    assert (d == o).all()
    assert p.max_delay == [77385] and p.overlap == 77385


def test_multi_range_tables_bit_exact():
    f = np.linspace(750.0, 550.0, 512)
    p = sdd.Plan(f, 81.92e-6, ranges=synth.MULTI_RANGES, widths=[1 << k for k in range(9)])
    spec = oracle.make_plan(f, 81.92e-6, ranges=synth.MULTI_RANGES,
                            widths=[1 << k for k in range(9)])
    assert p.ndm == [1000, 1000, 800, 800, 750]
    assert p.decimation == [1, 2, 4, 8, 16]
    assert p.dm_offset == [0, 1000, 2000, 2800, 3600]
    for r, rs in enumerate(spec.ranges):
        np.testing.assert_array_equal(p.dms(r), rs.dms)
        np.testing.assert_array_equal(p.delays(r), rs.delays)
        assert p.max_delay[r] == rs.max_delay
    assert p.overlap == spec.overlap
    T = spec.overlap + (1 << 19)
    g = p.geometry(T)
    assert g["n_owned_r"] == spec.owned(T) == [1 << 19 >> k for k in range(5)]


def test_unsorted_frequencies_reference_the_max():
    f = np.array([400.0, 500.0, 300.0, 450.0])
    p = sdd.Plan(f, 1e-3, dm_list=[0.0, 50.0, 100.0])
    np.testing.assert_array_equal(p.delays(0), oracle.delay_table(f, [0.0, 50.0, 100.0], 1e-3))


@pytest.mark.parametrize("kw,status", [
    (dict(widths=[2, 1]), A.SDD_EINVAL),
    (dict(widths=[0, 1]), A.SDD_EINVAL),
    (dict(widths=[8193]), A.SDD_EINVAL),
    (dict(t_samp=0.0), A.SDD_EINVAL),
    (dict(dm_list=[-1.0]), A.SDD_EINVAL),
    (dict(freqs=[500.0, -3.0]), A.SDD_EINVAL),
    (dict(both=True), A.SDD_EINVAL),
    (dict(neither=True), A.SDD_EINVAL),
    (dict(ranges=[(0.0, 10.0, 1.0, 0)]), A.SDD_EINVAL),
    (dict(ranges=[(0.0, 10.0, 0.0, 1)]), A.SDD_EINVAL),
    (dict(cand_block=-5), A.SDD_EINVAL),
    # 65536 channels * 255 * 512 >= 2^32: boxcar sums could overflow
    (dict(freqs=list(np.linspace(500, 300, 65536)), widths=[512]), A.SDD_ERANGE),
])
def test_plan_argument_errors(kw, status):
    freqs = kw.get("freqs", [500.0, 400.0, 300.0])
    t = kw.get("t_samp", 1e-3)
    dm_list = kw.get("dm_list", [0.0, 10.0])
    ranges = kw.get("ranges")
    if ranges is not None:
        dm_list = None
    if kw.get("both"):
        ranges = [(0.0, 10.0, 1.0, 1)]
    if kw.get("neither"):
        dm_list = None
    with pytest.raises(sdd.SddError) as ei:
        sdd.Plan(freqs, t, dm_list=dm_list, ranges=ranges, widths=kw.get("widths", ()),
                 cand_block=kw.get("cand_block", 1024))
    assert ei.value.status == status
    assert len(A.lib().sdd_last_error()) > 0


def test_geometry_rejects_short_input():
    p = sdd.Plan([500.0, 300.0], 1e-3, ranges=[(0.0, 10.0, 1.0, 1), (10.0, 20.0, 1.0, 4)],
                 widths=[1, 2])
    O = p.overlap
    with pytest.raises(sdd.SddError) as ei:
        p.geometry(O + 3)
    assert ei.value.status == A.SDD_EINVAL
    g = p.geometry(O + 4)
    assert g["n_owned_r"] == [4, 1]


def test_compute_calls_validate_before_touching_the_device():
    p = sdd.Plan([500.0, 300.0], 1e-3, dm_list=[0.0, 5.0], widths=[1])
    T = p.overlap + 100
    L = A.lib()
    planes = (C.c_void_p * 1)(1)
    pitch = (C.c_int64 * 1)(4)
    # null input
    assert L.sdd_dedisperse(p.handle, None, T, T, planes, pitch, 1, 1 << 20, None) == A.SDD_EINVAL
    # pitch smaller than the plane's columns
    assert L.sdd_dedisperse(p.handle, 1, T, T, planes, pitch, 1, 1 << 20, None) == A.SDD_EINVAL
    # input pitch smaller than the row
    g = p.geometry(T)
    pitch2 = (C.c_int64 * 1)(g["plane_cols"][0])
    assert L.sdd_dedisperse(p.handle, 1, T, T - 1, planes, pitch2, 1, 1 << 20, None) == A.SDD_EINVAL
    # too short an input
    assert L.sdd_dedisperse(p.handle, 1, p.overlap, T, planes, pitch2, 1, 1 << 20, None) == A.SDD_EINVAL
    # workspace too small
    assert L.sdd_dedisperse(p.handle, 1, T, T, planes, pitch2, 1, 0, None) == A.SDD_ENOMEM
    # search on a plane-only plan
    q = sdd.Plan([500.0, 300.0], 1e-3, dm_list=[0.0])
    assert L.sdd_search_boxcar(q.handle, planes, pitch2, T, 1, 1, 1, 1, 1, 1, 1 << 20,
                               None) == A.SDD_EINVAL
    # null candidate buffer with a positive capacity
    assert L.sdd_search_boxcar(p.handle, planes, pitch2, T, 1, 1, None, 4, 1, 1, 1 << 20,
                               None) == A.SDD_EINVAL


def test_tile_menu_and_set_tile():
    menu = sdd.tile_menu()
    assert (0, 0, 0, 0, 0, 0) in menu
    # a delay span of 15 samples fits every shape's staging; the matrix-core
    # form (flag 4: kinds 5, 21) takes uint8 rows only, the aligned-word
    # vector form (flag 8: kind 9) uint16 rows (a decimated range) only
    p = sdd.Plan([500.0, 300.0], 1e-3, dm_list=[0.0, 0.5])
    q = sdd.Plan([500.0, 300.0], 1e-3, ranges=[(0.0, 1.0, 0.5, 2)])
    for t in menu:
        flags = t[0] - 1 if t[0] else 0  # kind 0: the direct kernel
        u8_ok = not flags & 8
        u16_ok = not flags & 4
        for plan, ok in ((p, u8_ok), (q, u16_ok)):
            if ok:
                plan.set_tile(t, 0)
                assert plan.get_tile(0) == t
            else:
                with pytest.raises(sdd.SddError):
                    plan.set_tile(t, 0)
    assert any(t[0] == 9 for t in menu)
    with pytest.raises(sdd.SddError):
        p.set_tile((9, 9, 9, 9, 9, 9))


def test_single_hip_runtime_in_process():
    """The library must share torch's HIP runtime: two copies of libamdhip64
    in one process make device selection fail."""
    sdd.lib()
    import torch  # noqa: F401
    maps = {l.split()[-1] for l in open("/proc/self/maps") if "libamdhip64" in l}
    assert len(maps) == 1, maps


def test_unsorted_dm_list_uses_the_direct_kernel():
    p = sdd.Plan([500.0, 400.0, 300.0], 1e-3, dm_list=[5.0, 0.0, 3.0])
    assert p.get_tile(0)[0] == 0
    lds_tiles = [t for t in sdd.tile_menu() if t[0] >= 1]
    for t in lds_tiles:
        with pytest.raises(sdd.SddError):
            p.set_tile(t)
    q = sdd.Plan([500.0, 400.0, 300.0], 1e-3, dm_list=[0.0, 3.0, 5.0])
    assert q.get_tile(0)[0] >= 1


def test_sift_validates_before_touching_the_device():
    L = A.lib()
    nb = C.c_int64()
    assert L.sdd_sift_workspace_size(0, C.byref(nb)) == A.SDD_EINVAL
    assert L.sdd_sift_workspace_size(1000, C.byref(nb)) == A.SDD_OK and nb.value > 1000 * 40
    p = sdd.Plan([500.0, 300.0], 1e-3, dm_list=[0.0, 5.0], widths=[1])
    d = A.SiftDesc()
    args = lambda desc, cap=16, ws=1 << 20: (p.handle, 1, 1, cap, C.byref(desc), 1, 1, None, 1,
                                           ws, None)
    assert L.sdd_sift_candidates(None, 1, 1, 16, C.byref(d), 1, 1, None, 1, 1 << 20,
                                 None) == A.SDD_EINVAL
    assert L.sdd_sift_candidates(*args(d, cap=0)) == A.SDD_EINVAL
    d.nstencils = A.SDD_MAX_STENCILS + 1
    assert L.sdd_sift_candidates(*args(d)) == A.SDD_EINVAL
    d.nstencils = 1
    d.stencil_dm[0] = -1.0
    assert L.sdd_sift_candidates(*args(d)) == A.SDD_EINVAL
    d.stencil_dm[0] = 1.0
    d.min_pts = -2
    assert L.sdd_sift_candidates(*args(d)) == A.SDD_EINVAL
    d.min_pts = 2
    d.eps_t = -1
    assert L.sdd_sift_candidates(*args(d)) == A.SDD_EINVAL
    d.eps_t = 10
    assert L.sdd_sift_candidates(*args(d, ws=16)) == A.SDD_ENOMEM


def test_rfi_entry_points_validate_before_touching_the_device():
    L = A.lib()
    p = sdd.Plan([500.0, 400.0, 300.0], 1e-3, dm_list=[0.0, 5.0], widths=[1], layout="time")
    nb = C.c_int64()
    assert L.sdd_rfi_workspace_size(p.handle, 0, C.byref(nb)) == A.SDD_EINVAL
    assert L.sdd_rfi_workspace_size(p.handle, 1000, C.byref(nb)) == A.SDD_OK
    ws = nb.value
    good = A.RfiDesc(21, 2, 4.0, 3.0)
    call = lambda d, pitch=3, wsb=ws: L.sdd_rfi_estimate(p.handle, 1, 1000, pitch, C.byref(d), 1,
                                                          1, None, 1, wsb, None)
    for bad in (A.RfiDesc(20, 2, 4.0, 3.0), A.RfiDesc(65, 2, 4.0, 3.0),
                A.RfiDesc(21, 0, 4.0, 3.0), A.RfiDesc(21, 2, 0.0, 3.0),
                A.RfiDesc(21, 2, 4.0, -1.0)):
        assert call(bad) == A.SDD_EINVAL
    assert call(good, pitch=2) == A.SDD_EINVAL          # time-major pitch < nchan
    assert call(good, wsb=ws - 1) == A.SDD_ENOMEM
    # the pre-conditioned search checks its workspace like the plain one
    T = p.overlap + 100
    assert L.sdd_pre_workspace_size(p.handle, T, 1, C.byref(nb)) == A.SDD_OK
    best = (C.c_byte * 64)()
    assert L.sdd_dedisperse_search_pre(p.handle, 1, T, 3, None, None, None, None, best, None,
                                       None, 0, best, 1, nb.value - 1, None) == A.SDD_ENOMEM


def test_set_stats_validates():
    L = A.lib()
    p = sdd.Plan([500.0, 300.0], 1e-3, dm_list=[0.0, 5.0], widths=[1])
    assert L.sdd_plan_set_stats(p.handle, 7, 3.0, 3) == A.SDD_EINVAL
    assert L.sdd_plan_set_stats(p.handle, A.SDD_STATS_CLIPPED, 0.0, 3) == A.SDD_EINVAL
    assert L.sdd_plan_set_stats(p.handle, A.SDD_STATS_CLIPPED, 3.0, 0) == A.SDD_EINVAL
    assert L.sdd_plan_set_stats(p.handle, A.SDD_STATS_CLIPPED, 3.0, 65) == A.SDD_EINVAL
    assert L.sdd_plan_set_stats(None, 0, 0.0, 0) == A.SDD_EINVAL
    p.set_stats("clip", 2.5, 4)
    p.set_stats("mad")
    p.set_stats()


def test_set_dereddening_validates_and_grows_the_workspace():
    L = A.lib()
    p = sdd.Plan([500.0, 300.0], 1e-3, dm_list=[0.0, 5.0], widths=[1, 2, 64])
    w0 = p.geometry(20000)["workspace_bytes"]
    # blocks outside the powers of two in 64..4096, half < 1, a window above
    # 4096 samples; (64, 1) is a 192-sample window, above twice the widest
    # boxcar (128)
    for block, half in [(32, 2), (100, 1), (8192, 1), (64, 0), (1024, 2), (64, 1)]:
        rc = L.sdd_plan_set_dereddening(p.handle, block, half)
        if (block, half) == (64, 1):
            assert rc == A.SDD_OK
        else:
            assert rc == A.SDD_EINVAL, (block, half)
    assert L.sdd_plan_set_dereddening(p.handle, 64, 1) == A.SDD_OK
    q = sdd.Plan([500.0, 300.0], 1e-3, dm_list=[0.0], widths=[1, 128])
    assert L.sdd_plan_set_dereddening(q.handle, 64, 1) == A.SDD_EINVAL  # 192 <= 2 * 128
    assert L.sdd_plan_set_dereddening(q.handle, 64, 2) == A.SDD_OK      # 320 > 2 * 128
    q.set_dereddening(128, 1)
    assert L.sdd_plan_set_dereddening(None, 64, 1) == A.SDD_EINVAL
    nw = sdd.Plan([500.0, 300.0], 1e-3, dm_list=[0.0])
    assert L.sdd_plan_set_dereddening(nw.handle, 64, 1) == A.SDD_EINVAL
    p.set_dereddening(256, 2)
    g = p.geometry(20000)
    cols = max(g["plane_cols"])
    assert g["workspace_bytes"] >= w0 + 2 * ((cols + 255) // 256) * 4
    p.set_dereddening(0)
    assert p.geometry(20000)["workspace_bytes"] == w0


def test_ffa_search_validates_before_touching_the_device():
    """Every argument check of sdd_ffa_search runs on the host, before any
    device call (fake non-null device addresses are never dereferenced)."""
    L = A.lib()
    nb = C.c_int64()
    assert L.sdd_ffa_workspace_size(4, 100000, 1000, C.byref(nb)) == A.SDD_OK
    m = 100
    assert nb.value >= 4 * m * 1000 * 4 * 2 + 4 * 16
    assert L.sdd_ffa_workspace_size(0, 100000, 1000, C.byref(nb)) == A.SDD_EINVAL
    assert L.sdd_ffa_workspace_size(4, 999, 1000, C.byref(nb)) == A.SDD_EINVAL
    fake = 0x10000
    w = (C.c_int32 * 3)(1, 2, 4)

    def call(nsamp=100000, period=1000, maxv=4096, widths=w, nw=3, ws=nb.value, pitch=None,
             best=fake, series=fake):
        return L.sdd_ffa_search(0, series, pitch or nsamp, 4, nsamp, period, maxv, widths, nw,
                                None, best, None, fake, ws, None)

    assert call(series=None) == A.SDD_EINVAL
    assert call(best=None) == A.SDD_EINVAL
    assert call(period=1) == A.SDD_EINVAL
    assert call(period=4097, nsamp=100000) == A.SDD_EINVAL
    assert call(nsamp=500) == A.SDD_EINVAL
    assert call(pitch=99999) == A.SDD_EINVAL
    assert call(nw=0) == A.SDD_EINVAL
    assert call(widths=(C.c_int32 * 3)(1, 4, 2)) == A.SDD_EINVAL     # not increasing
    assert call(widths=(C.c_int32 * 3)(1, 2, 1000)) == A.SDD_EINVAL  # not below the period
    # m * max_value = 100 * 2^26 >= 2^32: a profile bin could overflow 32 bits
    assert call(maxv=1 << 26) == A.SDD_ERANGE
    assert call(ws=nb.value - 1) == A.SDD_ENOMEM


def test_misaligned_workspaces_are_refused():
    """Every entry point that takes a device workspace refuses one that is
    not 256-byte aligned, before touching the device (fake addresses)."""
    L = A.lib()
    fake = 0x10000
    w = (C.c_int32 * 1)(1)
    nb = C.c_int64()
    assert L.sdd_ffa_workspace_size(1, 1000, 100, C.byref(nb)) == A.SDD_OK
    assert L.sdd_ffa_search(0, fake, 1000, 1, 1000, 100, 255, w, 1, None, fake, None, fake + 8,
                            nb.value, None) == A.SDD_EINVAL
    assert "aligned" in A.lib().sdd_last_error().decode()
    assert L.sdd_sift_workspace_size(16, C.byref(nb)) == A.SDD_OK
    p = sdd.Plan([500.0, 300.0], 1e-3, dm_list=[0.0, 5.0], widths=[1])
    d = A.SiftDesc()
    assert L.sdd_sift_candidates(p.handle, fake, fake, 16, C.byref(d), fake, fake, None,
                                 fake + 64, nb.value, None) == A.SDD_EINVAL


def _share_fraction(d, dt=16):
    """Groups (channel pair, trial pair 2w, 2w+1 of a DM tile) whose two
    trials start in the same 16-byte words of the windows, from the delay
    table (numpy, independent of the library)."""
    d = np.asarray(d, dtype=np.int64)
    ndm, nchan = d.shape
    shared = total = 0
    for i in range(0, ndm - 1, 2):
        i0 = i // dt * dt
        if i + 1 >= i0 + dt:
            continue
        base = d[i0] & ~15
        pa = (d[i] - base) & ~15
        pb = (d[i + 1] - base) & ~15
        same = pa == pb
        pairs = same[0:nchan - 1:2] & same[1::2]
        shared += int(pairs.sum())
        total += pairs.size
    return shared / total


def test_default_tiles_by_range():
    """The plan's default tile per range: the matrix-core form for uint8
    ranges, its read-sharing variant where at least half of the groups of
    neighbouring trials start in the same data words (fine DM steps), the
    four-copy vector form for decimated (uint16) ranges, and the two-copy
    vector form for a decimated range whose delay span is too wide for the
    four-copy staging."""
    f = np.linspace(750.0, 550.0, 4096)
    coarse = sdd.Plan(f, 81.92e-6, dm_list=np.linspace(0.0, 1000.0, 2048))
    assert _share_fraction(coarse.delays(0)) < 0.5
    assert coarse.get_tile(0) == (5, 1, 16, 1, 16, 16)
    multi = sdd.Plan(f, 81.92e-6, ranges=synth.MULTI_RANGES)
    assert _share_fraction(multi.delays(0)) >= 0.5
    assert multi.get_tile(0) == (21, 2, 8, 1, 8, 8)
    for r in range(1, len(synth.MULTI_RANGES)):
        assert multi.get_tile(r) == (9, 4, 8, 1, 8, 4)
    # DM 0-300 in 300 trials at decimation 2: about 2500 samples of delay
    # span per 64 trials, past every four-copy shape's staging
    wide = sdd.Plan(np.linspace(750.0, 550.0, 999), 81.92e-6, ranges=[(0.0, 300.0, 1.0, 2)])
    assert wide.get_tile(0)[0] == 1
