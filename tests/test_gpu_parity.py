"""GPU parity: the HIP path through the C ABI against the oracle, on the same
seeded synthetic inputs. Planes bit-exact; S/N within 1e-4 relative;
candidate lists identical away from the threshold."""
import numpy as np
import pytest

import oracle
import synth
from _parity import compare_rows, compare_search, gpu_run, oracle_plan, say

pytestmark = pytest.mark.gpu


def _sdd():
    import paper_2605_03531_amd as sdd
    return sdd


def _make(kw, layout="chan"):
    sdd = _sdd()
    return sdd.Plan(kw["freqs_mhz"], kw["t_samp"], dm_list=kw.get("dm_list"),
                    ranges=kw.get("ranges"), widths=kw.get("widths", ()),
                    cand_block=kw.get("cand_block", 1024), threshold=kw.get("threshold", 7.0),
                    layout=layout)


@pytest.fixture(scope="module")
def tiny():
    return synth.tiny(oracle.delay_table)


@pytest.mark.parametrize("layout", ["chan", "time"])
def test_tiny_full_plane_and_search(tiny, layout):
    say(f"tiny workload, layout {layout}")
    kw = dict(freqs_mhz=tiny.freqs_mhz, t_samp=tiny.t_samp, dm_list=tiny.dm_list,
              widths=tiny.widths, cand_block=tiny.cand_block, threshold=tiny.threshold)
    plan = _make(kw, layout)
    spec = oracle_plan(kw)
    ph, res, g = gpu_run(plan, tiny.x, time_major=(layout == "time"))
    assert g["plane_cols"] == [3690]
    orc = oracle.run(spec, tiny.x)
    compare_rows(spec, ph, orc)
    rel = compare_search(spec, res, orc, full_rows=True)
    say(f"max S/N rel err {rel:.2e}, candidates {res[3]}")
    best = res[0]
    k = int(np.argmax(best["snr"]))
    assert k == 100 and int(best[k]["sample"]) == 3000 and int(best[k]["width"]) == 4


@pytest.mark.parametrize("case", ["narrow_1024", "narrow_2048", "wide_halo"])
def test_segment_search_layouts(case):
    """The search with cells of whole 1024-start segments: odd and even
    widths (32-, 64- and 128-bit shifted reads of the prefix sums), a partial
    last segment, cells of two segments (combined by atomic max), and a halo
    of 1008 samples with boxcar bounds past 2^28 (the compare-and-select
    path instead of packed keys)."""
    if case == "wide_halo":
        f = np.linspace(500.0, 300.0, 200)
        ranges = [(0.0, 10.0, 1.0, 1), (10.0, 30.0, 2.0, 8)]
        kw = dict(freqs_mhz=f, t_samp=1e-3, ranges=ranges, widths=[1, 7, 100, 1000],
                  cand_block=1024, threshold=4.0)
        nown, dm_pulse = 9000, 4.0
    else:
        f = np.linspace(500.0, 300.0, 64)
        kw = dict(freqs_mhz=f, t_samp=1e-3, dm_list=np.arange(0.0, 51.0),
                  widths=[1, 2, 3, 5, 8, 12, 16, 64],
                  cand_block=1024 if case == "narrow_1024" else 2048, threshold=4.0)
        nown, dm_pulse = 5000, 30.0
    say(f"segment search case {case}")
    spec = oracle_plan(kw)
    T = spec.overlap + nown
    x = synth.filterbank(41, len(f), T, 100.0, 20.0)
    synth.inject_pulse(x, oracle.delay_table(f, [dm_pulse], 1e-3)[0], 2100, 5, 15.0)
    orc = oracle.run(spec, x)
    plan = _make(kw, "chan")
    ph, res, g = gpu_run(plan, x)
    compare_rows(spec, ph, orc)
    rel = compare_search(spec, res, orc, full_rows=True)
    say(f"max S/N rel err {rel:.2e}, candidates {res[3]}")


def test_tiny_plane_only_and_determinism(tiny):
    kw = dict(freqs_mhz=tiny.freqs_mhz, t_samp=tiny.t_samp, dm_list=tiny.dm_list)
    plan = _make(kw)
    a, _, g = gpu_run(plan, tiny.x, search=False)
    b, _, _ = gpu_run(plan, tiny.x, search=False)
    assert g["plane_cols"] == [8192 - 4502]
    assert (a[0] == b[0]).all()
    y = oracle.dedisperse(tiny.x, oracle.delay_table(tiny.freqs_mhz, tiny.dm_list, tiny.t_samp),
                          8192 - 4502)
    assert (a[0].astype(np.int64) == y).all()


def test_multi_range_small_full_plane():
    """Several decimated ranges, every row, ragged owned length."""
    f = np.linspace(500.0, 300.0, 96)
    ranges = [(0.0, 20.0, 1.0, 1), (20.0, 60.0, 2.0, 2), (60.0, 100.0, 4.0, 4),
              (100.0, 160.0, 5.0, 8)]
    kw = dict(freqs_mhz=f, t_samp=2e-3, ranges=ranges, widths=[1, 2, 3, 8, 16],
              cand_block=100, threshold=3.0)
    spec = oracle_plan(kw)
    T = spec.overlap + 5000 + 13
    x = synth.filterbank(21, 96, T, 100.0, 20.0)
    d = oracle.delay_table(f, [37.0, 123.0], 2e-3)
    synth.inject_pulse(x, d[0], 1200, 6, 30.0)
    synth.inject_pulse(x, d[1], 3001, 24, 12.0)
    orc = oracle.run(spec, x)
    for layout in ("chan", "time"):
        say(f"multi-range small, layout {layout}")
        plan = _make(kw, layout)
        assert plan.get_tile(1)[0] >= 1  # decimated ranges take the LDS kernel too
        ph, res, g = gpu_run(plan, x, time_major=(layout == "time"))
        compare_rows(spec, ph, orc)
        compare_search(spec, res, orc, full_rows=True)
    # every tile shape, on each range that takes it (uint8 and uint16 inputs)
    plan = _make(kw, "time")
    n = 0
    for tile in _menu_tiles():
        if not _set_where_it_fits(plan, tile):
            continue
        ph, res, g = gpu_run(plan, x, time_major=True)
        compare_rows(spec, ph, orc)
        n += 1
    assert n >= 3


def _pulse_rows(dms, pulses, ndm, reach=8):
    """Rows within `reach` trials of each pulse's nearest trial (pulses whose
    DM falls in this grid)."""
    rows = set()
    for p in pulses:
        if dms[0] - 1 <= p.dm <= dms[-1] + 1:
            k = int(np.argmin(np.abs(dms - p.dm)))
            rows.update(range(max(0, k - reach), min(ndm, k + reach + 1)))
    return rows


def _run_full(plan, x, cap=1 << 20):
    """Time-major upload, one call, planes kept on the device."""
    import torch
    xt = torch.from_numpy(synth.to_time_major(x)).to("cuda:0")
    T = x.shape[1]
    planes = plan.alloc_planes(T)
    _, out = plan.dedisperse_search(xt, planes=planes, cap=cap)
    torch.cuda.synchronize()
    del xt
    return planes, out.host(), plan.geometry(T)


def _check_rows_and_checksums(spec, planes, res, g, x, rows, label):
    """Bit-exact plane rows and search results on `rows` (per range), and the
    row-sum / index-weighted row-sum checksums of every row of every plane
    against the oracle's prefix-sum checksums."""
    from _parity import device_checksums, oracle_checksums_parallel, oracle_rows_parallel
    ph = []
    for r in range(len(spec.ranges)):
        idx = list(rows[r])
        full = np.zeros((planes[r].shape[0], g["plane_cols"][r]), dtype=np.uint32)
        if idx:
            full[idx] = planes[r][idx, :g["plane_cols"][r]].cpu().numpy().view(np.uint32)
        ph.append(full)
    say(f"{label}: oracle on {sum(len(r) for r in rows)} rows")
    orc = oracle_rows_parallel(spec, x, rows)
    compare_rows(spec, ph, orc)
    rel = compare_search(spec, res, orc, full_rows=False)
    say(f"{label}: rows bit-exact, S/N rel err {rel:.2e}; checksums of every row")
    for r, rs in enumerate(spec.ranges):
        xr = x if rs.dec == 1 else oracle.decimate(x, rs.dec)
        cols = g["plane_cols"][r]
        ea, eb = oracle_checksums_parallel(xr, rs.delays, cols)
        ga, gb = device_checksums(planes[r], cols)
        bad = np.flatnonzero((ga != ea) | (gb != eb))
        assert bad.size == 0, f"{label} range {r}: {bad.size} rows differ, first {bad[:8]}"
    return orc


@pytest.mark.timeout(900)
def test_full_band_bench_config_rows_checksums_and_injections():
    """The benchmark's launch configuration at full size (4096 channels,
    2048 trials 0-1000, 2^18 owned samples, spectra input, widths 1..64):
    bit-exact rows and search results on every trial within 8 of each
    injected pulse's nearest trial, the edge trials and 32 seeded random
    trials; exact row-sum and weighted row-sum checksums of all 2048 rows;
    the DM-0 row equal to the channel sum; and injection recovery."""
    widths = [1, 2, 4, 8, 16, 32, 64]
    say("generating full-band input")
    w = synth.full_band(oracle.delay_table, widths=widths)
    kw = dict(freqs_mhz=w.freqs_mhz, t_samp=w.t_samp, dm_list=w.dm_list, widths=widths,
              cand_block=1024, threshold=7.0)
    plan = _make(kw, "time")
    spec = oracle_plan(kw)
    say("running the library")
    planes, res, g = _run_full(plan, w.x)
    assert g["n_owned"] == 1 << 18
    rng = np.random.Generator(np.random.PCG64(99))
    rows = {0, 1, 1023, 2046, 2047} | _pulse_rows(w.dm_list, w.pulses, 2048)
    rows.update(int(v) for v in rng.choice(2048, 32, replace=False))
    rows = sorted(rows)
    _check_rows_and_checksums(spec, planes, res, g, w.x, [rows], "full band")
    col = w.x.sum(axis=0, dtype=np.int64)[: g["plane_cols"][0]]
    assert (planes[0][0, :g["plane_cols"][0]].cpu().numpy().astype(np.int64) == col).all()
    _injection_recovery(w, res)


def _injection_recovery(w, res):
    """Every injected pulse that should stand out is found: a candidate with
    S/N above the threshold within 2 trials of the pulse's nearest trial,
    whose window start lies where the pulse lands in that trial. The pulses
    sit at off-grid DMs, so in trial k channel c puts the pulse at
    t0 + d(c, DM) - d(c, DM_k): the pulse is smeared over the spread s of
    those offsets and keeps about A * sqrt(w / (w + s)) of its matched S/N
    A; pulses with A >= 10 whose smeared S/N stays >= 10 are required (the
    boxcar widths are powers of two, so a little is lost to the mismatch)."""
    cands = res[2]
    found, need = 0, 0
    for p in w.pulses:
        k = int(np.argmin(np.abs(w.dm_list - p.dm)))
        a = p.amp * np.sqrt(len(w.freqs_mhz) * p.width) / 16.0
        dt = oracle.delay_table(w.freqs_mhz, [p.dm], w.t_samp)[0]
        dk = oracle.delay_table(w.freqs_mhz, [w.dm_list[k]], w.t_samp)[0]
        off = dt - dk
        smeared = a * np.sqrt(p.width / (p.width + int(off.max() - off.min())))
        if a < 10 or smeared < 10:
            continue
        need += 1
        lo = p.t0 + int(off.min()) - 64
        hi = p.t0 + int(off.max()) + p.width
        hit = [c for c in cands if abs(int(c["dm_index"]) - k) <= 2
               and lo <= int(c["sample"]) <= hi and float(c["snr"]) > 7.0]
        say(f"pulse DM {p.dm:.2f} (trial {k}) width {p.width} A {a:.1f} smeared {smeared:.1f}: "
            f"{len(hit)} candidates, best S/N {max([float(c['snr']) for c in hit] or [0]):.1f}")
        assert hit, (p, k, lo, hi)
        found += 1
    assert need >= 5 and found == need


@pytest.mark.timeout(900)
def test_multi_range_config_full_size_rows_and_checksums():
    """The multi-range workload at full size: 4096 channels 750-550 MHz,
    81.92 us, 2^19 owned samples, DM ranges 0-100/0.1, 100-300/0.2 (dec 2),
    300-700/0.5 (dec 4), 700-1500/1 (dec 8), 1500-3000/2 (dec 16), widths
    1..256: bit-exact rows and search results on every trial within 8 of an
    injected pulse's nearest trial in its range, the first, middle and last
    trial and 32 seeded random trials of every range; exact checksums of all
    4350 rows."""
    widths = [1 << k for k in range(9)]
    kw = dict(freqs_mhz=np.linspace(750.0, 550.0, 4096), t_samp=81.92e-6,
              ranges=synth.MULTI_RANGES, widths=widths, cand_block=1024, threshold=7.0)
    spec = oracle_plan(kw)
    say("generating the multi-range input")
    w = synth.multi_range(spec.overlap, delay_fn=oracle.delay_table)
    plan = _make(kw, "time")
    say("running the library")
    planes, res, g = _run_full(plan, w.x)
    assert g["n_owned"] == 1 << 19
    rng = np.random.Generator(np.random.PCG64(98))
    rows = []
    for rs in spec.ranges:
        n = len(rs.dms)
        sel = {0, n // 2, n - 1} | _pulse_rows(rs.dms, w.pulses, n)
        sel.update(int(v) for v in rng.choice(n, 32, replace=False))
        rows.append(sorted(sel))
    _check_rows_and_checksums(spec, planes, res, g, w.x, rows, "multi-range")
    say(f"multi-range full size: {res[3]} candidates")


def test_edge_single_channel_single_trial_minimum_length():
    kw = dict(freqs_mhz=[400.0], t_samp=1e-3, dm_list=[0.0], widths=[1], cand_block=1,
              threshold=0.5)
    spec = oracle_plan(kw)
    x = synth.filterbank(3, 1, spec.overlap + 1, 50.0, 10.0)
    plan = _make(kw)
    ph, res, g = gpu_run(plan, x)
    orc = oracle.run(spec, x)
    compare_rows(spec, ph, orc)
    compare_search(spec, res, orc, full_rows=True)


def test_edge_unsorted_freqs_odd_channels_padded_spectra():
    import torch
    sdd = _sdd()
    f = np.array([410.0, 500.0, 305.0, 333.0, 480.0, 470.0, 301.0])
    kw = dict(freqs_mhz=f, t_samp=1e-3, dm_list=[0.0, 3.0, 7.5, 20.0, 20.5], widths=[1, 2, 4],
              cand_block=37, threshold=2.0)
    spec = oracle_plan(kw)
    T = spec.overlap + 999
    x = synth.filterbank(4, 7, T, 120.0, 30.0)
    plan = _make(kw, "time")
    # spectra with a padded row pitch of 13 bytes
    buf = np.zeros((T, 13), dtype=np.uint8)
    buf[:, :7] = x.T
    xt = torch.from_numpy(buf).to("cuda:0")[:, :7]
    planes = plan.alloc_planes(T)
    _, out = plan.dedisperse_search(xt, planes=planes)
    torch.cuda.synchronize()
    g = plan.geometry(T)
    ph = [sdd.plane_host(planes[0], g["plane_cols"][0])]
    orc = oracle.run(spec, x)
    compare_rows(spec, ph, orc)
    compare_search(spec, out.host(), orc, full_rows=True)


def test_edge_constant_input_and_candidate_cap():
    import torch
    kw = dict(freqs_mhz=np.linspace(500, 300, 32), t_samp=1e-3, dm_list=np.arange(0.0, 20.0),
              widths=[1, 2, 4], cand_block=8, threshold=-5.0)
    spec = oracle_plan(kw)
    T = spec.overlap + 500
    plan = _make(kw)
    xc = np.full((32, T), 77, dtype=np.uint8)
    ph, res, g = gpu_run(plan, xc)
    assert (ph[0] == 32 * 77).all()
    best, stats, cands, n = res
    assert n == 0 and (best["snr"] == 0).all() and (best["sample"] == 0).all()
    assert (stats["std"] == 0).all()
    # many candidates, small cap: the total is reported, the first cap written
    kw2 = dict(kw, threshold=0.5)
    spec2 = oracle_plan(kw2)
    plan2 = _make(kw2)
    x = synth.filterbank(5, 32, T, 128.0, 16.0)
    _, full, _ = gpu_run(plan2, x, cap=100000)
    _, capped, _ = gpu_run(plan2, x, cap=10)
    assert full[3] == capped[3] > 10
    assert capped[2].tobytes() == full[2][:10].tobytes()
    orc = oracle.run(spec2, x)
    compare_search(spec2, full, orc, full_rows=True)


def _menu_tiles():
    import paper_2605_03531_amd as sdd
    return sdd.tile_menu()


def _set_where_it_fits(plan, tile):
    """Sets `tile` on every range that takes it (the matrix-core shapes take
    uint8 rows only, the four-copy shapes uint16 rows only); the other ranges
    keep their tile. Returns the ranges set."""
    done = []
    for r in range(plan.nranges):
        try:
            plan.set_tile(tile, r)
        except Exception:
            continue
        done.append(r)
    return done


def test_every_tile_shape_is_exact():
    """Each kernel shape of the built menu gives the oracle's plane on a
    ragged case: 999 channels (odd, and not a multiple of any stage, so the
    last channels are added past the staged loop), 300 trials (a partial DM
    tile), a partial time tile and a padded spectra pitch. A wide DM range
    exercises large delay spans; a narrow one fits the shapes whose staging
    holds only small spans, so every shape runs on at least one of them.
    Each case runs on uint8 rows (a plain trial list) and on the uint16 rows
    of a range decimated by 2, which the four-copy shapes take."""
    f = np.linspace(750.0, 550.0, 999)
    ran = set()
    for dm_hi, dec in ((300.0, 1), (12.0, 1), (300.0, 2), (12.0, 2)):
        if dec == 1:
            kw = dict(freqs_mhz=f, t_samp=81.92e-6, dm_list=np.linspace(0.0, dm_hi, 300))
        else:
            kw = dict(freqs_mhz=f, t_samp=81.92e-6, ranges=[(0.0, dm_hi, dm_hi / 300, dec)])
        spec = oracle_plan(kw)
        assert spec.ranges[0].dms.size == 300
        T = spec.overlap + 3 * 1024 + 77
        x = synth.filterbank(31, 999, T, 128.0, 16.0)
        rows = [0, 1, 63, 64, 150, 255, 256, 298, 299]
        (_, yo, _), = oracle.run(spec, x, rows=[rows], search=False)
        plan = _make(kw, "time")
        seen = []
        for tile in _menu_tiles():
            try:
                plan.set_tile(tile)
            except Exception:
                say(f"DM 0-{dm_hi}, decimation {dec}: tile {tile} does not fit this plan")
                continue
            say(f"DM 0-{dm_hi}, decimation {dec}: tile {tile}")
            ph, _, g = gpu_run(plan, x, search=False, time_major=True)
            assert (ph[0][rows].astype(np.int64) == yo).all(), tile
            seen.append(ph[0])
            ran.add(tuple(tile))
        assert len(seen) >= 3
        for p in seen[1:]:
            assert (p == seen[0]).all()
    assert ran == {tuple(t) for t in _menu_tiles()}


def test_lds_tiles_on_channel_major_unaligned_input():
    """Channel-major input whose row pitch is not a multiple of 16 bytes (the
    staging falls back to byte loads) is still exact for every LDS shape."""
    f = np.linspace(500.0, 300.0, 130)
    dms = np.arange(0.0, 70.0)
    kw = dict(freqs_mhz=f, t_samp=1.31072e-3, dm_list=dms)
    spec = oracle_plan(kw)
    T = spec.overlap + 2000 + 3
    x = synth.filterbank(32, 130, T, 90.0, 25.0)
    (_, yo, _), = oracle.run(spec, x, search=False)
    plan = _make(kw, "chan")
    for tile in _menu_tiles():
        try:
            plan.set_tile(tile)
        except Exception:
            continue
        ph, _, _ = gpu_run(plan, x, search=False)
        assert (ph[0].astype(np.int64) == yo).all(), tile


def test_saturated_input_every_tile_grid_and_persistent():
    """Inputs at the top of the sample range keep the packed 16-bit partial
    sums at their bound: all-255 bytes (every plane value is the closed form
    nchan * 255 * dec) and a seeded 0/255 mix (checked against the oracle),
    523 channels (odd, not a multiple of any stage), a uint8 range and
    decimated ranges whose uint16 samples reach 255 * dec (dec 2 and 16). Every
    tile shape of the menu, as a grid launch and as the persistent multi-beam
    launch, gives these exact planes."""
    import paper_2605_03531_amd as sdd
    f = np.linspace(750.0, 550.0, 523)
    ranges = [(0.0, 20.0, 1.0, 1), (20.0, 40.0, 2.0, 2), (40.0, 80.0, 4.0, 16)]
    kw = dict(freqs_mhz=f, t_samp=81.92e-6, ranges=ranges)
    spec = oracle_plan(kw)
    T = spec.overlap + 4 * 1024 + 16 * 7
    rng = np.random.Generator(np.random.PCG64(255))
    inputs = {"all255": np.full((523, T), 255, dtype=np.uint8),
              "mix0_255": (rng.integers(0, 2, (523, T)) * 255).astype(np.uint8)}
    expect = {"all255": None, "mix0_255": oracle.run(spec, inputs["mix0_255"], search=False)}
    plan = _make(kw, "time")
    ran = 0
    for tile in _menu_tiles():
        if not _set_where_it_fits(plan, tile):
            continue
        ran += 1
        for name, x in inputs.items():
            say(f"saturated input {name}, tile {tile}")
            import torch
            xt = torch.from_numpy(synth.to_time_major(x)).to("cuda:0")
            g = plan.geometry(T)
            grid = plan.dedisperse(xt)
            batch_planes = plan.alloc_planes(T)
            for pl in batch_planes:
                pl.fill_(-1)
            sdd.Batch([(plan, xt, batch_planes, None)]).run()
            torch.cuda.synchronize()
            for form, planes in (("grid", grid), ("persistent", batch_planes)):
                ph = [sdd.plane_host(planes[r], g["plane_cols"][r]) for r in range(3)]
                if expect[name] is None:
                    for r, rs in enumerate(spec.ranges):
                        assert (ph[r] == 523 * 255 * rs.dec).all(), (form, tile, r)
                else:
                    compare_rows(spec, ph, expect[name])
    assert ran >= 3


@pytest.mark.parametrize("case", ["pow2_levels_skipped", "pow2_unaligned_rows", "not_pow2"])
def test_decimation_paths_exact(case):
    """Decimated ranges through both decimation paths: the one-pass kernel
    for decimations among 2, 4, 8, 16 (with levels the plan does not use
    skipped, and channel rows whose pitch is not a multiple of 16 bytes, so
    its loads fall back to bytes), and the level-by-level kernel for other
    factors (3 and 6, 6 built from 3). A ragged owned length leaves a partial
    group of samples at the row end. Full planes against the oracle."""
    import torch
    import paper_2605_03531_amd as sdd
    f = np.linspace(500.0, 300.0, 72)
    if case == "not_pow2":
        ranges = [(0.0, 10.0, 1.0, 1), (10.0, 30.0, 2.0, 3), (30.0, 60.0, 3.0, 6)]
    else:
        ranges = [(0.0, 10.0, 1.0, 1), (10.0, 30.0, 2.0, 2), (30.0, 90.0, 4.0, 16)]
    kw = dict(freqs_mhz=f, t_samp=1e-3, ranges=ranges, widths=[1, 3, 8], cand_block=300,
              threshold=4.0)
    spec = oracle_plan(kw)
    T = spec.overlap + 4000 + 48 + 5
    x = synth.filterbank(77, 72, T, 110.0, 20.0)
    synth.inject_pulse(x, oracle.delay_table(f, [40.0], 1e-3)[0], 1500, 12, 20.0)
    orc = oracle.run(spec, x)
    if case == "pow2_unaligned_rows":
        plan = _make(kw, "chan")
        buf = np.zeros((72, T + 3), dtype=np.uint8)
        buf[:, :T] = x
        xt = torch.from_numpy(buf).to("cuda:0")[:, :T]
        planes = plan.alloc_planes(T)
        _, out = plan.dedisperse_search(xt, planes=planes)
        torch.cuda.synchronize()
        g = plan.geometry(T)
        ph = [sdd.plane_host(planes[r], g["plane_cols"][r]) for r in range(3)]
        res = out.host()
    else:
        plan = _make(kw, "time")
        ph, res, g = gpu_run(plan, x, time_major=True)
    compare_rows(spec, ph, orc)
    compare_search(spec, res, orc, full_rows=True)


@pytest.mark.parametrize("pitch", [256, 272, 264])
def test_corner_turn_channel_tiles_ragged(pitch):
    """Spectra-ordered input of 256 channels through both corner turns: row
    pitches of 256 and 272 bytes take the 128-channel x 128-sample tiles
    (16-byte loads, register transposes), 264 bytes the byte-granular
    kernel. The number of spectra is not a multiple of 16, so the last tile
    of every channel row ends part-way. Full planes against the oracle."""
    import torch
    sdd = _sdd()
    f = np.linspace(500.0, 300.0, 256)
    kw = dict(freqs_mhz=f, t_samp=1e-3, dm_list=np.linspace(0.0, 30.0, 24), widths=[1, 4],
              cand_block=256, threshold=5.0)
    spec = oracle_plan(kw)
    T = spec.overlap + 2000 + 13
    say(f"corner turn, 256 channels, {T} spectra, pitch {pitch}")
    x = synth.filterbank(91, 256, T, 100.0, 25.0)
    buf = np.zeros((T, pitch), dtype=np.uint8)
    buf[:, :256] = x.T
    xt = torch.from_numpy(buf).to("cuda:0")[:, :256]
    plan = _make(kw, "time")
    planes = plan.alloc_planes(T)
    _, out = plan.dedisperse_search(xt, planes=planes)
    torch.cuda.synchronize()
    g = plan.geometry(T)
    ph = [sdd.plane_host(planes[0], g["plane_cols"][0])]
    orc = oracle.run(spec, x)
    compare_rows(spec, ph, orc)
    compare_search(spec, out.host(), orc, full_rows=True)
