"""GPU parity of the search with robust noise statistics (sigma-clipped
moments; median and MAD) against the oracle."""
import numpy as np
import pytest

import oracle
import synth
from _parity import compare_rows, compare_search, gpu_run, oracle_plan, say

pytestmark = pytest.mark.gpu

MODES = [("clip", 3.0, 3), ("clip", 2.0, 6), ("mad",)]


@pytest.mark.parametrize("mode", MODES, ids=lambda m: "-".join(map(str, m)))
def test_tiny_with_robust_statistics(mode):
    import paper_2605_03531_amd as sdd
    w = synth.tiny(oracle.delay_table)
    kw = dict(freqs_mhz=w.freqs_mhz, t_samp=w.t_samp, dm_list=w.dm_list, widths=w.widths,
              cand_block=w.cand_block, threshold=w.threshold)
    spec = oracle_plan(kw)
    spec.stats = mode
    plan = sdd.Plan(w.freqs_mhz, w.t_samp, dm_list=w.dm_list, widths=w.widths,
                    cand_block=w.cand_block, threshold=w.threshold)
    plan.set_stats(mode[0], *mode[1:])
    ph, res, g = gpu_run(plan, w.x)
    orc = oracle.run(spec, w.x)
    compare_rows(spec, ph, orc)
    rel = compare_search(spec, res, orc, full_rows=True)
    best = res[0]
    k = int(np.argmax(best["snr"]))
    say(f"{mode}: max S/N rel err {rel:.2e}, candidates {res[3]}, best DM {k} S/N "
        f"{float(best[k]['snr']):.1f}")
    assert k == 100 and int(best[k]["sample"]) == 3000


@pytest.mark.parametrize("mode", MODES[::2], ids=lambda m: "-".join(map(str, m)))
def test_multi_range_with_robust_statistics(mode):
    import paper_2605_03531_amd as sdd
    f = np.linspace(500.0, 300.0, 96)
    ranges = [(0.0, 20.0, 1.0, 1), (20.0, 60.0, 2.0, 2), (60.0, 100.0, 4.0, 4)]
    kw = dict(freqs_mhz=f, t_samp=2e-3, ranges=ranges, widths=[1, 2, 4, 16],
              cand_block=1024, threshold=4.0)
    spec = oracle_plan(kw)
    spec.stats = mode
    T = spec.overlap + 6000
    x = synth.filterbank(31, 96, T, 100.0, 20.0)
    synth.inject_pulse(x, oracle.delay_table(f, [37.0], 2e-3)[0], 2000, 8, 40.0)
    plan = sdd.Plan(f, 2e-3, ranges=ranges, widths=[1, 2, 4, 16], cand_block=1024,
                    threshold=4.0, layout="time")
    plan.set_stats(mode[0], *mode[1:])
    ph, res, g = gpu_run(plan, x, time_major=True)
    orc = oracle.run(spec, x)
    compare_rows(spec, ph, orc)
    rel = compare_search(spec, res, orc, full_rows=True)
    say(f"multi-range {mode}: rel err {rel:.2e}, candidates {res[3]}")
