"""GPU parity of RFI pre-conditioning: the estimator's maps (per-channel byte
table, time mask, channel flags) equal the oracle's exactly, and the
pre-conditioned dedispersion + search equals the oracle's path on the
pre-conditioned chunk."""
import numpy as np
import pytest

import oracle
import synth
from _parity import compare_rows, compare_search, gpu_run, oracle_plan, say

pytestmark = pytest.mark.gpu


def _chunk(seed, C, T):
    x = synth.filterbank(seed, C, T, 100.0, 10.0).astype(np.int64)
    x += (20.0 * np.sin(np.linspace(0, 3, C))).round().astype(np.int64)[:, None]
    x[[5, C // 3, C // 3 + 1, C - 7]] += 60
    x[:, [40, 41, T // 2, T - 9]] += 40
    return np.clip(x, 0, 255).astype(np.uint8)


def _plan(C, layout, **kw):
    import paper_2605_03531_amd as sdd
    f = np.linspace(500.0, 300.0, C)
    if "ranges" not in kw:
        kw["dm_list"] = np.arange(0.0, 40.0)
    args = dict(freqs_mhz=f, t_samp=1.31072e-3, widths=[1, 2, 4, 8], cand_block=1024,
                threshold=5.0, **kw)
    plan = sdd.Plan(f, 1.31072e-3, dm_list=args.get("dm_list"), ranges=args.get("ranges"),
                    widths=args["widths"], cand_block=1024, threshold=5.0, layout=layout)
    return plan, args


@pytest.mark.parametrize("layout", ["chan", "time"])
@pytest.mark.parametrize("T", [6000, 6003])
def test_rfi_estimate_equals_oracle(layout, T):
    """T = 6000: vector loads of channel rows; T = 6003: unaligned
    channel-major rows (byte loads) and a 3-sample tail after the corner turn."""
    import torch
    C = 256
    x = _chunk(12, C, T)
    plan, _ = _plan(C, layout)
    xin = torch.from_numpy(x if layout == "chan" else synth.to_time_major(x)).to("cuda:0")
    lut, mask, flags = plan.rfi_estimate(xin)
    torch.cuda.synchronize()
    cflag, tflag, b, olut, omask = oracle.rfi_estimate(x)
    say(f"rfi {layout}: {int(cflag.sum())} channels, {int(tflag.sum())} samples flagged")
    assert np.array_equal(flags.cpu().numpy().astype(bool), cflag)
    assert np.array_equal(mask.cpu().numpy(), omask)
    assert np.array_equal(lut.cpu().numpy(), olut)


@pytest.mark.parametrize("layout", ["chan", "time"])
@pytest.mark.parametrize("ranges", [False, True])
def test_preconditioned_search_equals_oracle(layout, ranges):
    import torch
    C = 96
    kw = {"ranges": [(0.0, 20.0, 1.0, 1), (20.0, 60.0, 2.0, 2)]} if ranges else {}
    plan, args = _plan(C, layout, **kw)
    spec = oracle_plan(args)
    T = spec.overlap + 3000 + 5
    x = synth.filterbank(13, C, T, 90.0, 15.0)
    g = np.random.Generator(np.random.PCG64(14))
    olut = g.integers(0, 256, (C, 256)).astype(np.uint8)
    olut[[3, 50]] = 0
    omask = (g.random(T) > 0.1).astype(np.uint8)
    y = oracle.precondition(x, olut, omask)
    orc = oracle.run(spec, y)
    lut = torch.from_numpy(olut).to("cuda:0")
    mask = torch.from_numpy(omask).to("cuda:0")
    xin = torch.from_numpy(x if layout == "chan" else synth.to_time_major(x)).to("cuda:0")
    planes = plan.alloc_planes(T)
    _, out = plan.dedisperse_search(xin, planes=planes, lut=lut, time_mask=mask)
    torch.cuda.synchronize()
    import paper_2605_03531_amd as sdd
    g2 = plan.geometry(T)
    ph = [sdd.plane_host(planes[r], g2["plane_cols"][r]) for r in range(plan.nranges)]
    compare_rows(spec, ph, orc)
    rel = compare_search(spec, out.host(), orc, full_rows=True)
    say(f"pre-conditioned {layout} ranges={ranges}: S/N rel err {rel:.2e}")
    # identity maps through the pre-conditioned entry point equal the plain path
    ident = torch.from_numpy(np.tile(np.arange(256, dtype=np.uint8), (C, 1))).to("cuda:0")
    ones = torch.ones(T, dtype=torch.uint8, device="cuda:0")
    p1, o1 = plan.dedisperse_search(xin, planes=plan.alloc_planes(T), lut=ident, time_mask=ones)
    p2, o2 = plan.dedisperse_search(xin, planes=plan.alloc_planes(T))
    torch.cuda.synchronize()
    for r in range(plan.nranges):
        cols = g2["plane_cols"][r]
        assert torch.equal(p1[r][:, :cols], p2[r][:, :cols])
    assert (o1.host()[0] == o2.host()[0]).all()


def test_estimate_then_search_finds_the_pulse():
    """The tiny workload with planted RFI: after estimation the pulse at
    (DM 100, sample 3000, width 4) is still the best candidate."""
    import torch
    w = synth.tiny(oracle.delay_table)
    x = w.x.astype(np.int64)
    x[[30, 31, 200]] += 80
    x[:, [500, 501, 7000]] += 60
    x = np.clip(x, 0, 255).astype(np.uint8)
    import paper_2605_03531_amd as sdd
    plan = sdd.Plan(w.freqs_mhz, w.t_samp, dm_list=w.dm_list, widths=w.widths,
                    cand_block=w.cand_block, threshold=w.threshold)
    xin = torch.from_numpy(x).to("cuda:0")
    lut, mask, flags = plan.rfi_estimate(xin)
    _, out = plan.dedisperse_search(xin, lut=lut, time_mask=mask)
    best = out.host()[0]
    k = int(np.argmax(best["snr"]))
    say(f"tiny+RFI: flags {int(flags.sum().cpu())} ch, best DM {k}, sample {int(best[k]['sample'])}")
    assert k == 100 and int(best[k]["sample"]) == 3000 and int(best[k]["width"]) == 4
    fl = flags.cpu().numpy()
    assert fl[30] and fl[31] and fl[200]


@pytest.mark.parametrize("rounds", [1, 2])
def test_rfi_hand_worked_case_on_the_device(rounds):
    """The hand-worked 7 x 10 case of the oracle's pins (3-channel median
    window): round 1 flags channels {2, 5} and sample {4}; round 2 flags
    channel {5} and sample {4} (means over the kept samples, zero-DM series
    over the round's own channels)."""
    import torch
    import sys
    import os
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    from test_oracle_rfi import hand_case
    x = hand_case()
    plan, _ = _plan(7, "chan")
    lut, mask, flags = plan.rfi_estimate(torch.from_numpy(x).to("cuda:0"), median_window=3,
                                         rounds=rounds)
    torch.cuda.synchronize()
    want_c = [2, 5] if rounds == 1 else [5]
    assert np.nonzero(flags.cpu().numpy())[0].tolist() == want_c
    assert np.nonzero(mask.cpu().numpy() == 0)[0].tolist() == [4]
    _, _, _, olut, _ = oracle.rfi_estimate(x, window=3, rounds=rounds)
    assert np.array_equal(lut.cpu().numpy(), olut)
