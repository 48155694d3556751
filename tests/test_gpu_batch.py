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
