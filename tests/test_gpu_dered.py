"""GPU parity of the search on running-median de-reddened series (block
baselines, half-scale re-centring, full-scale clip) against the oracle, with
every noise estimate, both search kernels, decimated ranges, a red-noise
drift and the full-band launch configuration on sampled trials."""
import numpy as np
import pytest

import oracle
import synth
from _parity import compare_rows, compare_search, gpu_run, oracle_plan, say

pytestmark = pytest.mark.gpu


def _tiny_plan(sdd, w, dered, stats=None, cand_block=None):
    cb = w.cand_block if cand_block is None else cand_block
    kw = dict(freqs_mhz=w.freqs_mhz, t_samp=w.t_samp, dm_list=w.dm_list, widths=w.widths,
              cand_block=cb, threshold=w.threshold)
    spec = oracle_plan(kw)
    spec.stats = stats
    spec.dered = dered
    plan = sdd.Plan(w.freqs_mhz, w.t_samp, dm_list=w.dm_list, widths=w.widths, cand_block=cb,
                    threshold=w.threshold)
    if stats is not None:
        plan.set_stats(stats[0], *stats[1:])
    plan.set_dereddening(*dered)
    return spec, plan


@pytest.mark.parametrize("stats", [None, ("clip", 3.0, 3), ("mad",)],
                         ids=["moments", "clip", "mad"])
def test_tiny_dereddened(stats):
    import paper_2605_03531_amd as sdd
    w = synth.tiny(oracle.delay_table)
    spec, plan = _tiny_plan(sdd, w, (64, 2), stats)
    ph, res, g = gpu_run(plan, w.x)
    orc = oracle.run(spec, w.x)
    compare_rows(spec, ph, orc)
    rel = compare_search(spec, res, orc, full_rows=True)
    best = res[0]
    k = int(np.argmax(best["snr"]))
    say(f"de-reddened {stats}: rel err {rel:.2e}, candidates {res[3]}, best DM {k} "
        f"S/N {float(best[k]['snr']):.1f}")
    assert k == 100 and int(best[k]["sample"]) == 3000


def test_red_noise_drift_removed_and_cell_kernel():
    """A slow common-mode drift on every channel: parity on both search
    kernels (segment kernel with 1024-start cells; per-cell kernel with
    700-start cells), and de-reddening raises the pulse's S/N several times
    (the drift inflates the plain sigma)."""
    import paper_2605_03531_amd as sdd
    w = synth.tiny(oracle.delay_table)
    x = w.x.astype(np.int64)
    t = np.arange(x.shape[1])
    drift = np.round(40.0 * np.sin(2 * np.pi * t / 2500.0)).astype(np.int64)
    x = np.clip(x + drift[None, :], 0, 255).astype(np.uint8)
    for cb in (w.cand_block, 700):
        spec, plan = _tiny_plan(sdd, w, (128, 3), ("mad",), cand_block=cb)
        ph, res, g = gpu_run(plan, x)
        orc = oracle.run(spec, x)
        compare_rows(spec, ph, orc)
        rel = compare_search(spec, res, orc, full_rows=True)
        best = res[0]
        k = int(np.argmax(best["snr"]))
        say(f"drift, cells of {cb}: rel err {rel:.2e}, best DM {k} sample "
            f"{int(best[k]['sample'])} S/N {float(best[k]['snr']):.1f}")
        assert k == 100 and int(best[k]["sample"]) == 3000
    plain = sdd.Plan(w.freqs_mhz, w.t_samp, dm_list=w.dm_list, widths=w.widths,
                     cand_block=w.cand_block, threshold=w.threshold)
    _, rp, _ = gpu_run(plain, x, planes=False)
    s0, s1 = float(rp[0][100]["snr"]), float(best[100]["snr"])
    say(f"pulse S/N with the drift: plain {s0:.1f}, de-reddened {s1:.1f}")
    assert s1 > 3.0 * s0


def test_multi_range_wide_boxcars_dereddened():
    """Decimated ranges (each with its own full scale) and boxcars to 256
    (a 16-sample-aligned halo of 256 samples) under a 768-sample window."""
    import paper_2605_03531_amd as sdd
    f = np.linspace(500.0, 300.0, 96)
    ranges = [(0.0, 20.0, 1.0, 1), (20.0, 60.0, 2.0, 2), (60.0, 100.0, 4.0, 4)]
    widths = [1, 2, 4, 16, 64, 256]
    kw = dict(freqs_mhz=f, t_samp=2e-3, ranges=ranges, widths=widths, cand_block=1024,
              threshold=4.0)
    spec = oracle_plan(kw)
    spec.dered = (256, 1)
    T = spec.overlap + 9000
    x = synth.filterbank(41, 96, T, 100.0, 20.0)
    synth.inject_pulse(x, oracle.delay_table(f, [37.0], 2e-3)[0], 2000, 8, 40.0)
    plan = sdd.Plan(f, 2e-3, ranges=ranges, widths=widths, cand_block=1024, threshold=4.0,
                    layout="time")
    plan.set_dereddening(256, 1)
    ph, res, g = gpu_run(plan, x, time_major=True)
    orc = oracle.run(spec, x)
    compare_rows(spec, ph, orc)
    rel = compare_search(spec, res, orc, full_rows=True)
    say(f"multi-range de-reddened: rel err {rel:.2e}, candidates {res[3]}")


def test_switching_off_restores_the_plain_search():
    import paper_2605_03531_amd as sdd
    w = synth.tiny(oracle.delay_table)
    plan = sdd.Plan(w.freqs_mhz, w.t_samp, dm_list=w.dm_list, widths=w.widths,
                    cand_block=w.cand_block, threshold=w.threshold)
    _, r0, _ = gpu_run(plan, w.x, planes=False)
    plan.set_dereddening(64, 2)
    _, r1, _ = gpu_run(plan, w.x, planes=False)
    plan.set_dereddening(0)
    _, r2, _ = gpu_run(plan, w.x, planes=False)
    assert r0[0].tobytes() == r2[0].tobytes() and r0[1].tobytes() == r2[1].tobytes()
    assert r0[0].tobytes() != r1[0].tobytes()


def test_full_band_bench_config_dereddened_sampled_rows():
    """The benchmark's launch configuration (4096 channels, 2048 trials
    0-1000, 2^18 owned samples, widths 1..64) with a 256-sample block and a
    1280-sample window: search results on sampled trials equal the oracle's."""
    import paper_2605_03531_amd as sdd
    widths = [1, 2, 4, 8, 16, 32, 64]
    say("generating full-band input")
    w = synth.full_band(oracle.delay_table, widths=widths)
    kw = dict(freqs_mhz=w.freqs_mhz, t_samp=w.t_samp, dm_list=w.dm_list, widths=widths,
              cand_block=1024, threshold=7.0)
    spec = oracle_plan(kw)
    spec.dered = (256, 2)
    plan = sdd.Plan(w.freqs_mhz, w.t_samp, dm_list=w.dm_list, widths=widths, cand_block=1024,
                    threshold=7.0, layout="time")
    plan.set_dereddening(256, 2)
    say("running the library")
    ph, res, g = gpu_run(plan, w.x, time_major=True)
    rows = {0, 2047}
    for p in w.pulses[:3]:
        rows.add(int(np.argmin(np.abs(w.dm_list - p.dm))))
    rows.update(int(v) for v in np.random.Generator(np.random.PCG64(5)).integers(0, 2048, 2))
    rows = sorted(rows)
    say(f"oracle on rows {rows}")
    orc = oracle.run(spec, w.x, rows=[rows])
    compare_rows(spec, ph, orc)
    rel = compare_search(spec, res, orc, full_rows=False)
    say(f"full band de-reddened: rel err {rel:.2e}")
