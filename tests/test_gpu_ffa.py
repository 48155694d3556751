"""GPU parity of the FFA folding transform and the boxcar search of folded
profiles against the oracle: exact uint32 profiles and moments, identical
best bins and widths, S/N within the stated tolerance, over stack heights
that exercise the LDS sub-stacks, the HBM passes, short periods (several rows
per workgroup), a single row and a two-row stack, on seeded series, on the
rows of a dedispersed plane and on the full-band plane's sampled trials."""
import numpy as np
import pytest

import oracle
import synth
from _parity import SNR_RTOL, gpu_run, oracle_plan, say

pytestmark = pytest.mark.gpu


def _series(seed, nseries, nsamp, mean=1000.0, sd=40.0, period=None, amp=0.0):
    g = np.random.Generator(np.random.PCG64(seed))
    y = np.round(g.normal(mean, sd, (nseries, nsamp))).clip(0, None).astype(np.int64)
    if period:
        for k in range(nseries):
            ph = 0.37 * period
            t = ph
            while t + 3 < nsamp:
                i = int(round(t))
                y[k, i:i + 3] += int(amp)
                t += period
    return y.astype(np.uint32)


def _check(y, p, widths, res, tag):
    """y: host uint32 [nseries][nsamp]; res = FfaOut.host()."""
    best, prof, st = res
    worst = 0.0
    for k in range(y.shape[0]):
        T, mom, ob = oracle.ffa_search(y[k].astype(np.int64), p, widths)
        if prof is not None:
            bad = np.argwhere(prof[k].astype(np.int64) != T)
            assert bad.size == 0, f"{tag} series {k}: {len(bad)} profile mismatches {bad[:4]}"
        if st is not None:
            assert (int(st[k]["n"]), int(st[k]["s1"]), int(st[k]["s2"])) == mom[:3]
            assert abs(st[k]["std"] - mom[4]) <= 1e-12 * max(mom[4], 1e-300)
        for s, o in enumerate(ob):
            b = best[k][s]
            assert (int(b["bin"]), int(b["width"])) == (o[1], o[2]), (tag, k, s, b, o)
            if o[0] != 0.0:
                rel = abs(float(b["snr"]) / o[0] - 1.0)
                worst = max(worst, rel)
                assert rel < SNR_RTOL, (tag, k, s, float(b["snr"]), o[0])
            else:
                assert float(b["snr"]) == 0.0
    return worst


@pytest.mark.parametrize("nsamp,p", [(20000, 100), (65536, 256), (70000, 1000), (9000, 4096),
                                     (12000, 3), (5000, 64), (4097, 4096), (33333, 300)],
                         ids=lambda v: str(v))
def test_seeded_series_shapes(nsamp, p):
    import torch
    import paper_2605_03531_amd as sdd
    widths = [w for w in (1, 2, 3, 4, 8, 16, 32) if w < p]
    y = _series(nsamp + p, 3, nsamp, period=p + 0.4, amp=60)
    x = torch.from_numpy(y.view(np.int32)).to("cuda:0")
    out = sdd.ffa_search(x, p, widths, int(y.max()), profiles=True)
    torch.cuda.synchronize()
    rel = _check(y, p, widths, out.host(), f"{nsamp}/{p}")
    say(f"FFA {nsamp} samples at period {p} (m {nsamp // p}): S/N rel err {rel:.2e}")


def test_strided_rows_without_profiles_and_constant_series():
    """Rows of a wider buffer (pitch > nsamp), no profile output, and a
    constant series (sigma 0: S/N 0 at bin 0, first width)."""
    import torch
    import paper_2605_03531_amd as sdd
    y = _series(5, 4, 30000, period=250.3, amp=50)
    y[2] = 77
    buf = np.zeros((4, 30016), dtype=np.uint32)
    buf[:, :30000] = y
    xb = torch.from_numpy(buf.view(np.int32)).to("cuda:0")
    out = sdd.ffa_search(xb[:, :30000], 250, [1, 2, 4, 8], 4096, profiles=False)
    torch.cuda.synchronize()
    best, prof, st = out.host()
    assert prof is None
    _check(y, 250, [1, 2, 4, 8], (best, None, st), "strided")
    assert all(float(b["snr"]) == 0.0 and int(b["bin"]) == 0 and int(b["width"]) == 1
               for b in best[2])


def test_pulse_train_found_at_its_trial_on_the_gpu():
    import torch
    import paper_2605_03531_amd as sdd
    p, m, s0 = 512, 128, 77
    y = _series(77, 1, p * m, mean=500.0, sd=20.0, period=p + s0 / (m - 1), amp=25)
    x = torch.from_numpy(y.view(np.int32)).to("cuda:0")
    out = sdd.ffa_search(x, p, [1, 2, 4, 8], int(y.max()))
    torch.cuda.synchronize()
    best, _, _ = out.host()
    k = int(np.argmax(best[0]["snr"]))
    say(f"pulse train drifting {s0} bins: best trial {k}, S/N {float(best[0][k]['snr']):.1f}")
    # the FFA folds row i of trial s with a shift within ceil(log2 m) / 2 bins
    # of i s / (m - 1), so neighbouring trials fold a narrow train almost as well
    assert abs(k - s0) <= 3 and float(best[0][k]["snr"]) > 10.0
    _check(y, p, [1, 2, 4, 8], out.host(), "train")


def test_plane_rows_of_a_dedispersed_periodic_source():
    """Dedisperse a filterbank holding a periodic dispersed pulse train, then
    fold the plane's rows (a strided view of the library's plane): profiles
    and bests equal the oracle's fold of the oracle's own plane rows, and the
    true DM's row has the strongest fold."""
    import torch
    import paper_2605_03531_amd as sdd
    f = np.linspace(500.0, 300.0, 64)
    t_samp = 1e-3
    dms = np.arange(0.0, 40.0, 2.0)
    kw = dict(freqs_mhz=f, t_samp=t_samp, dm_list=dms)
    spec = oracle_plan(kw)
    T = spec.overlap + 40000
    x = synth.filterbank(12, 64, T, 128.0, 16.0)
    d = oracle.delay_table(f, [20.0], t_samp)[0]
    P = 400.25
    t = 50.0
    while t + 3 + d.max() < T:
        synth.inject_pulse(x, d, int(round(t)), 3, 6.0)
        t += P
    plan = sdd.Plan(f, t_samp, dm_list=dms)
    ph, _, g = gpu_run(plan, x, search=False)
    n = g["n_owned"]
    pl = plan.alloc_planes(T)
    plan.dedisperse(torch.from_numpy(x).to("cuda:0"), planes=pl)
    out = sdd.ffa_search(pl[0][:, :n], 400, [1, 2, 4, 8], 64 * 255, profiles=True)
    torch.cuda.synchronize()
    best, prof, st = out.host()
    rows = [0, 5, 10, 19]
    orc = oracle.run(spec, x, rows=[rows], search=False)
    for k, i in enumerate(rows):
        yk = orc[0][1][k][:n]
        assert np.array_equal(ph[0][i][:n].astype(np.int64), yk)
        _check(yk[None, :].astype(np.uint32), 400, [1, 2, 4, 8],
               (best[i:i + 1], prof[i:i + 1], st[i:i + 1]), f"row {i}")
    peak = best["snr"].max(axis=1)
    say(f"fold S/N by DM row: {np.round(peak, 1).tolist()}")
    assert int(np.argmax(peak)) == 10


def test_full_band_plane_sampled_trials():
    """The benchmark's plane (4096 channels, 2048 trials 0-1000, 2^18 owned
    samples) folded at a 1024-sample base period (m = 256): sampled trials
    equal the oracle's fold of the oracle's own plane rows."""
    import torch
    import paper_2605_03531_amd as sdd
    widths = [1, 2, 4, 8, 16, 32, 64]
    say("generating full-band input")
    w = synth.full_band(oracle.delay_table, widths=widths)
    kw = dict(freqs_mhz=w.freqs_mhz, t_samp=w.t_samp, dm_list=w.dm_list)
    spec = oracle_plan(kw)
    plan = sdd.Plan(w.freqs_mhz, w.t_samp, dm_list=w.dm_list, layout="time")
    xt = torch.from_numpy(np.ascontiguousarray(w.x.T)).to("cuda:0")
    T = w.x.shape[1]
    g = plan.geometry(T)
    n = g["n_owned"]
    pl = plan.alloc_planes(T)
    plan.dedisperse(xt, planes=pl)
    out = sdd.ffa_search(pl[0][:, :n], 1024, widths, 4096 * 255, profiles=False)
    torch.cuda.synchronize()
    best, _, st = out.host()
    rows = [0, 777, 2047]
    say(f"oracle on rows {rows}")
    orc = oracle.run(spec, w.x, rows=[rows], search=False)
    for k, i in enumerate(rows):
        yk = orc[0][1][k][:n]
        rel = _check(yk[None, :].astype(np.uint32), 1024, widths,
                     (best[i:i + 1], None, st[i:i + 1]), f"full band row {i}")
        say(f"row {i}: S/N rel err {rel:.2e}")


def test_wide_profiles_take_the_64_bit_boxcar_path():
    """Samples up to 2^25 at a 4096-bin period: a profile's bins minus its
    smallest bin total far above 2^32, so the boxcar search runs on 64-bit
    prefix sums; one series of small values in the same call stays on the
    32-bit path."""
    import torch
    import paper_2605_03531_amd as sdd
    g = np.random.Generator(np.random.PCG64(31))
    y = g.integers(0, 1 << 25, (3, 8192 + 17)).astype(np.uint32)
    y[1] = g.integers(0, 1000, 8192 + 17).astype(np.uint32)
    x = torch.from_numpy(y.view(np.int32)).to("cuda:0")
    widths = [1, 3, 64, 1000, 4095]
    out = sdd.ffa_search(x, 4096, widths, (1 << 25) - 1, profiles=True)
    torch.cuda.synchronize()
    rel = _check(y, 4096, widths, out.host(), "wide")
    say(f"wide profiles: S/N rel err {rel:.2e}")
