"""GPU parity of candidate sifting (square-stencil peak filter + DBSCAN-style
clustering in the DM-time plane) against the oracle, on seeded candidate
lists uploaded as a search's output."""
import numpy as np
import pytest

import oracle
import synth
from _parity import say

pytestmark = pytest.mark.gpu


def _upload(rng, dmi, smp, wid, snr, cap=None):
    import torch
    import paper_2605_03531_amd as sdd
    n = len(rng)
    cap = cap or max(n, 1)
    arr = np.zeros(cap, dtype=sdd.CAND_DTYPE)
    m = min(n, cap)
    arr["range"][:m] = rng[:m]
    arr["dm_index"][:m] = dmi[:m]
    arr["sample"][:m] = smp[:m]
    arr["width"][:m] = wid[:m]
    arr["snr"][:m] = snr[:m]
    out = sdd.SearchOut(None, None,
                        torch.from_numpy(arr.view(np.uint8).copy()).to("cuda:0"),
                        torch.tensor([n], dtype=torch.int32, device="cuda:0"))
    return out


def _spec_and_plan(kind):
    import paper_2605_03531_amd as sdd
    f = np.linspace(750.0, 550.0, 64)
    if kind == "ranges":
        ranges = [(0.0, 50.0, 0.5, 1), (50.0, 150.0, 1.0, 2), (150.0, 350.0, 2.0, 4)]
        plan = sdd.Plan(f, 81.92e-6, ranges=ranges, widths=[1, 2, 4])
        spec = oracle.make_plan(f, 81.92e-6, ranges=ranges, widths=[1, 2, 4])
    else:  # an explicit DM list out of order: the unsorted path
        g = np.random.Generator(np.random.PCG64(3))
        dms = g.permutation(np.arange(0.0, 150.0, 0.75))
        plan = sdd.Plan(f, 81.92e-6, dm_list=dms, widths=[1, 2, 4])
        spec = oracle.make_plan(f, 81.92e-6, dm_list=dms, widths=[1, 2, 4])
    return spec, plan


CASES = [
    ("stencils", dict(stencils=[(1.0, 20)], min_pts=0)),
    ("two_stencils", dict(stencils=[(0.6, 8), (3.0, 120)], min_pts=0)),
    ("fof", dict(stencils=[], eps=(2.0, 150), min_pts=1)),
    ("dbscan", dict(stencils=[(1.0, 20)], eps=(3.0, 200), min_pts=3)),
]


@pytest.mark.parametrize("kind", ["ranges", "unsorted"])
@pytest.mark.parametrize("name,kw", CASES)
def test_sift_matches_oracle(kind, name, kw):
    spec, plan = _spec_and_plan(kind)
    ndm = [len(r.dms) for r in spec.ranges]
    owned = [20000 // r.dec for r in spec.ranges]
    rng, dmi, smp, wid, snr = synth.candidate_list(7, ndm, owned)
    say(f"sift {kind} {name}: {len(rng)} candidates")
    out = _upload(rng, dmi, smp, wid, snr)
    eps = kw.get("eps", (0.0, 0))
    res = plan.sift(out, stencils=kw["stencils"], eps=eps, min_pts=kw["min_pts"])
    got, sizes = res.host()
    keep, osizes = oracle.sift_candidates(spec, rng, dmi, smp, snr, stencils=kw["stencils"],
                                          eps_dm=eps[0], eps_t=eps[1], min_pts=kw["min_pts"])
    say(f"  kept {len(got)} (oracle {len(keep)})")
    assert len(got) == len(keep)
    assert (got["range"] == rng[keep]).all() and (got["dm_index"] == dmi[keep]).all()
    assert (got["sample"] == smp[keep]).all() and (got["snr"] == snr[keep]).all()
    assert (got["width"] == wid[keep]).all()
    assert sizes.tolist() == osizes


def test_sift_cap_empty_and_repeat():
    spec, plan = _spec_and_plan("ranges")
    ndm = [len(r.dms) for r in spec.ranges]
    owned = [20000 // r.dec for r in spec.ranges]
    rng, dmi, smp, wid, snr = synth.candidate_list(9, ndm, owned)
    kw = dict(stencils=[(1.0, 20)], eps=(3.0, 200), min_pts=2)
    # a count past cap: only the first cap entries are sifted
    cap = len(rng) // 2
    out = _upload(rng, dmi, smp, wid, snr, cap=cap)
    out.ncand.fill_(len(rng))
    got, sizes = plan.sift(out, **kw).host()
    keep, osz = oracle.sift_candidates(spec, rng[:cap], dmi[:cap], smp[:cap], snr[:cap],
                                       stencils=kw["stencils"], eps_dm=3.0, eps_t=200, min_pts=2)
    assert (got["sample"] == smp[:cap][keep]).all() and sizes.tolist() == osz
    # the same call twice on one workspace gives the same result
    import torch
    import paper_2605_03531_amd as sdd
    from paper_2605_03531_amd import _capi as A
    import ctypes as C
    nb = C.c_int64()
    A.check(A.lib().sdd_sift_workspace_size(cap, C.byref(nb)), "ws")
    ws = torch.empty(nb.value, dtype=torch.uint8, device="cuda:0")
    a1 = plan.sift(out, workspace=ws, **kw).host()
    a2 = plan.sift(out, workspace=ws, **kw).host()
    assert (a1[0] == a2[0]).all() and (a1[1] == a2[1]).all()
    # an empty list
    out.ncand.zero_()
    got, sizes = plan.sift(out, **kw).host()
    assert len(got) == 0 and len(sizes) == 0


def test_sift_after_a_real_search(tiny=None):
    """End to end on the tiny workload: the injected pulse's candidate
    (DM 100, sample 3000, width 4) survives sifting."""
    import paper_2605_03531_amd as sdd
    from _parity import gpu_run, oracle_plan
    w = synth.tiny(oracle.delay_table)
    kw = dict(freqs_mhz=w.freqs_mhz, t_samp=w.t_samp, dm_list=w.dm_list, widths=w.widths,
              cand_block=w.cand_block, threshold=5.0)
    plan = sdd.Plan(w.freqs_mhz, w.t_samp, dm_list=w.dm_list, widths=w.widths,
                    cand_block=w.cand_block, threshold=5.0)
    import torch
    x = torch.from_numpy(w.x).to("cuda:0")
    _, out = plan.dedisperse_search(x)
    res = plan.sift(out, stencils=[(2.0, 16)], eps=(10.0, 2000), min_pts=1)
    got, sizes = res.host()
    spec = oracle_plan(kw)
    orc = oracle.run(spec, w.x)
    cands = [(0, i, c[1], c[2], c[0]) for i, rr in enumerate(orc[0][2]) for c in rr.cands]
    rng = np.array([c[0] for c in cands]); dmi = np.array([c[1] for c in cands])
    smp = np.array([c[2] for c in cands]); snr = np.array([c[4] for c in cands], np.float32)
    keep, _ = oracle.sift_candidates(spec, rng, dmi, smp, snr, stencils=[(2.0, 16)],
                                     eps_dm=10.0, eps_t=2000, min_pts=1)
    say(f"tiny: {int(out.ncand.cpu()[0])} candidates -> {len(got)} kept (oracle {len(keep)})")
    hit = [(int(c["dm_index"]), int(c["sample"])) for c in got]
    assert (100, 3000) in hit
