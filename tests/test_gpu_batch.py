"""GPU: batches of beams with mixed channel counts and uneven lengths give,
in every execution mode, the same bits as single calls and the oracle's
results on sampled rows; graph replays stay exact across eager work."""
import numpy as np
import pytest

import oracle
import synth
from _parity import compare_rows, compare_search, oracle_plan, say

pytestmark = pytest.mark.gpu


def _beams():
    """Six beams: 512/256/384 channels, lengths spanning several time tiles."""
    out = []
    rng = np.random.Generator(np.random.PCG64(77))
    for b, C in enumerate([512, 256, 384, 512, 256, 384]):
        f = np.linspace(750.0, 550.0, C)
        kw = dict(freqs_mhz=f, t_samp=81.92e-6, dm_list=np.linspace(0.0, 200.0, 96 + 16 * b),
                  widths=[1, 2, 4, 8, 16, 32], cand_block=512, threshold=6.0)
        spec = oracle_plan(kw)
        n_owned = int(rng.integers(3000, 9000))
        mean, std = float(rng.uniform(100, 150)), float(rng.uniform(8, 24))
        x = synth.filterbank(300 + b, C, spec.overlap + n_owned, mean, std)
        d = oracle.delay_table(f, [60.0 + 20 * b], 81.92e-6)
        synth.inject_pulse(x, d[0], n_owned // 3, 4, 3.0 * std)
        out.append((kw, spec, x))
    return out


def test_batch_modes_match_single_calls_and_oracle():
    import torch
    import paper_2605_03531_amd as sdd
    beams = _beams()
    plans, xs, single = [], [], []
    for kw, spec, x in beams:
        plan = sdd.Plan(kw["freqs_mhz"], kw["t_samp"], dm_list=kw["dm_list"], widths=kw["widths"],
                        cand_block=kw["cand_block"], threshold=kw["threshold"], layout="time")
        xt = torch.from_numpy(synth.to_time_major(x)).to("cuda:0")
        planes = plan.alloc_planes(x.shape[1])
        _, out = plan.dedisperse_search(xt, planes=planes)
        torch.cuda.synchronize()
        plans.append(plan)
        xs.append(xt)
        single.append(([p.clone() for p in planes], out.host()))
    for mode in ("persistent", "per_item", "graph"):
        say(f"batch mode {mode}")
        outs = [p.alloc_search_out() for p in plans]
        planes = [p.alloc_planes(x.shape[0]) for p, x in zip(plans, xs)]
        batch = sdd.Batch([(p, x, pl, o) for p, x, pl, o in zip(plans, xs, planes, outs)])
        ws = batch.workspace()
        reps = 3 if mode == "graph" else 1
        side = torch.cuda.Stream()
        for r in range(reps):
            for o in outs:
                o.ncand.zero_()
                o.best.zero_()
            torch.cuda.synchronize()
            batch.run(workspace=ws, per_item=(mode == "per_item"), graph=(mode == "graph"),
                      stream=side)
            torch.cuda.synchronize()
            for k in range(len(plans)):
                cols = plans[k].geometry(xs[k].shape[0])["plane_cols"][0]
                assert torch.equal(planes[k][0][:, :cols], single[k][0][0][:, :cols]), (mode, r, k)
                h = outs[k].host()
                assert h[0].tobytes() == single[k][1][0].tobytes(), (mode, r, k)
                assert h[2].tobytes() == single[k][1][2].tobytes(), (mode, r, k)
            # eager work between graph replays
            _ = torch.ones(1 << 20, device="cuda:0").sum().item()
    # graph capture of the null stream is refused
    with pytest.raises(sdd.SddError):
        batch.run(workspace=ws, graph=True, stream=0)
    # oracle on sampled rows of every beam (the single calls equal the batch)
    for k, (kw, spec, x) in enumerate(beams):
        n = len(kw["dm_list"])
        rows = sorted({0, n // 2, n - 1, int(np.argmax(single[k][1][0]["snr"]))})
        orc = oracle.run(spec, x, rows=[rows])
        g = plans[k].geometry(x.shape[1])
        ph = [single[k][0][0][:, :g["plane_cols"][0]].cpu().numpy().view(np.uint32)]
        compare_rows(spec, ph, orc)
        compare_search(spec, single[k][1], orc, full_rows=False)


def test_batch_with_search_options_matches_single_calls():
    """Robust statistics and de-reddening inside batches (persistent,
    per-item and graph replays, replayed three times with eager work in
    between) give the same bits as single calls; changing a plan's option
    afterwards takes effect in the next replay."""
    import torch
    import paper_2605_03531_amd as sdd
    beams = _beams()[:3]
    opts = [("mad", (64, 2)), ("clip", None), ("moments", (128, 1))]
    plans, xs, single = [], [], []
    for (kw, spec, x), (st, dr) in zip(beams, opts):
        plan = sdd.Plan(kw["freqs_mhz"], kw["t_samp"], dm_list=kw["dm_list"], widths=kw["widths"],
                        cand_block=kw["cand_block"], threshold=kw["threshold"], layout="time")
        plan.set_stats(st)
        if dr is not None:
            plan.set_dereddening(*dr)
        xt = torch.from_numpy(synth.to_time_major(x)).to("cuda:0")
        _, out = plan.dedisperse_search(xt)
        torch.cuda.synchronize()
        plans.append(plan)
        xs.append(xt)
        single.append(out.host())
    for mode in ("persistent", "per_item", "graph"):
        say(f"batch with search options, mode {mode}")
        outs = [p.alloc_search_out() for p in plans]
        batch = sdd.Batch([(p, x, None, o) for p, x, o in zip(plans, xs, outs)])
        ws = batch.workspace()
        side = torch.cuda.Stream()
        for r in range(3 if mode == "graph" else 1):
            for o in outs:
                o.best.zero_()
            torch.cuda.synchronize()
            batch.run(workspace=ws, per_item=(mode == "per_item"), graph=(mode == "graph"),
                      stream=side)
            torch.cuda.synchronize()
            for k in range(len(plans)):
                h = outs[k].host()
                assert h[0].tobytes() == single[k][0].tobytes(), (mode, r, k)
                assert h[2].tobytes() == single[k][2].tobytes(), (mode, r, k)
            _ = torch.ones(1 << 20, device="cuda:0").sum().item()
    # an option changed after capture: the next replay uses it
    plans[1].set_dereddening(64, 1)
    _, ref = plans[1].dedisperse_search(xs[1])
    outs = [p.alloc_search_out() for p in plans]
    batch = sdd.Batch([(p, x, None, o) for p, x, o in zip(plans, xs, outs)])
    batch.run(workspace=batch.workspace(), graph=True, stream=torch.cuda.Stream())
    torch.cuda.synchronize()
    assert outs[1].host()[0].tobytes() == ref.host()[0].tobytes()


def test_autotune_choices_cache_and_exact_planes(tmp_path):
    """sdd_autotune on a plan with uint8 and decimated (uint16) ranges: every
    range gets a tile of the built menu that fits it; the cache file gets one
    line per range; a second plan tuned from that cache takes the same tiles
    without timing anything (no line is added); the planes after tuning equal
    the oracle's."""
    import torch
    import paper_2605_03531_amd as sdd
    f = np.linspace(750.0, 550.0, 640)
    ranges = [(0.0, 60.0, 0.5, 1), (60.0, 140.0, 1.0, 2), (140.0, 300.0, 2.0, 4)]
    kw = dict(freqs_mhz=f, t_samp=81.92e-6, ranges=ranges, widths=[1, 2, 4, 8],
              cand_block=1024, threshold=6.0)
    spec = oracle_plan(kw)
    T = spec.overlap + 6 * 1024 + 40
    x = synth.filterbank(61, 640, T, 128.0, 16.0)
    synth.inject_pulse(x, oracle.delay_table(f, [90.0], 81.92e-6)[0], 2500, 4, 6.0)
    cache = str(tmp_path / "tiles.txt")

    def plan():
        return sdd.Plan(f, 81.92e-6, ranges=ranges, widths=kw["widths"], cand_block=1024,
                        threshold=6.0, layout="time")

    menu = {tuple(t) for t in sdd.tile_menu()}
    p1 = plan()
    p1.autotune(T, cache_path=cache)
    tiles = [tuple(p1.get_tile(r)) for r in range(len(ranges))]
    say(f"autotuned tiles {tiles}")
    assert all(t in menu for t in tiles)
    for r, t in enumerate(tiles):
        p1.set_tile(t, r)   # refused if the shape did not fit the range
    lines = open(cache).read().splitlines()
    assert len(lines) == len(ranges)
    assert {int(ln.split()[2]) for ln in lines} == {1, 2, 4}
    p2 = plan()
    p2.autotune(T, cache_path=cache)
    assert open(cache).read().splitlines() == lines
    assert [tuple(p2.get_tile(r)) for r in range(len(ranges))] == tiles
    xt = torch.from_numpy(synth.to_time_major(x)).to("cuda:0")
    planes = p2.alloc_planes(T)
    _, out = p2.dedisperse_search(xt, planes=planes)
    torch.cuda.synchronize()
    g = p2.geometry(T)
    ph = [sdd.plane_host(planes[r], g["plane_cols"][r]) for r in range(len(ranges))]
    orc = oracle.run(spec, x)
    compare_rows(spec, ph, orc)
    compare_search(spec, out.host(), orc, full_rows=True)


@pytest.mark.timeout(900)
def test_batched_config_shape_all_modes_equal_single_calls():
    """The batched workload at its real shape: 32 beams of 4096 channels
    (750-550 MHz, 81.92 us), owned lengths U[2^16, 2^18], per-beam noise mean
    U[100,150] and sigma U[8,24], 2048 trials 0-1000, widths 1..64, spectra
    input, tiles chosen by the autotuner. The persistent multi-beam launch,
    per-(beam, range) launches and the graph replay (three replays) give the
    planes, per-trial best values and candidates of single calls byte for
    byte; the oracle matches two rows of four beams."""
    import torch
    from concurrent.futures import ThreadPoolExecutor
    import paper_2605_03531_amd as sdd
    from _parity import host_workers
    widths = [1, 2, 4, 8, 16, 32, 64]
    f = np.linspace(750.0, 550.0, 4096)
    dms = np.linspace(0.0, 1000.0, 2048)
    kw = dict(freqs_mhz=f, t_samp=81.92e-6, dm_list=dms, widths=widths, cand_block=1024,
              threshold=7.0)
    spec = oracle_plan(kw)
    plan = sdd.Plan(f, 81.92e-6, dm_list=dms, widths=widths, cand_block=1024, threshold=7.0,
                    layout="time")
    params = synth.batched_beams()
    assert len(params) == 32
    checked = {0: None, 9: None, 20: None, 31: None}

    def make(b):
        n, mean, std = params[b]
        x = synth.filterbank(900 + b, 4096, n + spec.overlap, mean, std)
        return b, x, synth.to_time_major(x)

    say("generating 32 beams")
    xs = [None] * 32
    with ThreadPoolExecutor(min(8, host_workers())) as ex:
        for b, x, xtm in ex.map(make, range(32)):
            xs[b] = torch.from_numpy(xtm).to("cuda:0")
            if b in checked:
                checked[b] = x
    say("autotuning")
    plan.autotune(xs[0].shape[0])
    say(f"tile {plan.get_tile(0)}")
    single = []
    for b in range(32):
        pl = plan.alloc_planes(xs[b].shape[0])
        _, out = plan.dedisperse_search(xs[b], planes=pl, cap=1 << 16)
        single.append((pl[0], out.host()))
    torch.cuda.synchronize()
    outs = [plan.alloc_search_out(1 << 16) for _ in range(32)]
    planes = [plan.alloc_planes(x.shape[0]) for x in xs]
    batch = sdd.Batch([(plan, x, pl, o) for x, pl, o in zip(xs, planes, outs)])
    ws = batch.workspace()
    side = torch.cuda.Stream()
    for mode in ("persistent", "per_item", "graph"):
        for rep in range(3 if mode == "graph" else 1):
            say(f"batch mode {mode}, run {rep}")
            for pl, o in zip(planes, outs):
                pl[0].fill_(-1)
                o.ncand.zero_()
                o.best.zero_()
            torch.cuda.synchronize()
            batch.run(workspace=ws, per_item=(mode == "per_item"), graph=(mode == "graph"),
                      stream=side)
            torch.cuda.synchronize()
            for b in range(32):
                cols = plan.geometry(xs[b].shape[0])["plane_cols"][0]
                assert torch.equal(planes[b][0][:, :cols], single[b][0][:, :cols]), (mode, b)
                h = outs[b].host()
                assert h[0].tobytes() == single[b][1][0].tobytes(), (mode, rep, b)
                assert h[2].tobytes() == single[b][1][2].tobytes(), (mode, rep, b)
            _ = torch.ones(1 << 20, device="cuda:0").sum().item()
    for b, x in checked.items():
        rows = [int(b * 61 % 2048), int(np.argmax(single[b][1][0]["snr"]))]
        say(f"oracle: beam {b}, rows {rows}")
        orc = oracle.run(spec, x, rows=[rows])
        cols = plan.geometry(x.shape[1])["plane_cols"][0]
        ph = np.zeros((2048, cols), dtype=np.uint32)
        ph[rows] = single[b][0][rows, :cols].cpu().numpy().view(np.uint32)
        compare_rows(spec, [ph], orc)
        compare_search(spec, single[b][1], orc, full_rows=False)
