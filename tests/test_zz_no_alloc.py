"""GPU: the allocation-free entry point (sdd_dedisperse_search_static, static
device scratch) called through the C ABI gives the bits of
sdd_dedisperse_search on the same inputs, on two calls in a row with the
second input smaller than the first (the scratch keeps the first call's
contents), for time-major input with a decimated range and for library-held
planes; sizes past the static maximum and plans whose device tables do not
exist yet are refused before anything runs."""
import ctypes as C

import numpy as np
import pytest

import oracle
import synth
from _parity import compare_rows, oracle_plan, say

pytestmark = pytest.mark.gpu


def _plan(kw):
    import paper_2605_03531_amd as sdd
    return sdd.Plan(kw["freqs_mhz"], kw["t_samp"], ranges=kw["ranges"], widths=kw["widths"],
                    cand_block=kw["cand_block"], threshold=kw["threshold"], layout="time")


def _static(plan, xt, planes, out):
    """One call through the C ABI (ctypes prototypes only)."""
    import torch
    from paper_2605_03531_amd import _capi as A
    n = len(planes)
    ptrs = (C.c_void_p * n)(*[p.data_ptr() for p in planes])
    pitch = (C.c_int64 * n)(*[p.shape[1] for p in planes])
    cap = out.cands.numel() // 24
    st = A.lib().sdd_dedisperse_search_static(
        plan.handle, xt.data_ptr(), xt.shape[0], xt.shape[1], ptrs, pitch, out.best.data_ptr(),
        out.stats.data_ptr(), out.cands.data_ptr(), cap, out.ncand.data_ptr(),
        torch.cuda.current_stream().cuda_stream)
    return st


def test_static_scratch_matches_workspace_entry_point():
    import torch
    import paper_2605_03531_amd as sdd
    from paper_2605_03531_amd import _capi as A
    f = np.linspace(750.0, 550.0, 384)
    kw = dict(freqs_mhz=f, t_samp=81.92e-6, ranges=[(0.0, 120.0, 1.0, 1), (120.0, 240.0, 2.0, 2)],
              widths=[1, 2, 4, 8, 16], cand_block=512, threshold=6.0)
    spec = oracle_plan(kw)
    plan = _plan(kw)
    sizes = [spec.overlap + 6 * 1024 + 37, spec.overlap + 2 * 1024 + 9]
    xs = []
    for k, T in enumerate(sizes):
        x = synth.filterbank(610 + k, 384, T, 128.0, 16.0)
        synth.inject_pulse(x, oracle.delay_table(f, [60.0 + 90 * k], 81.92e-6)[0], 1000 + 300 * k,
                           4, 12.0)
        xs.append(x)
    # the reference results (and the plan's device tables) from the workspace entry point
    ref = []
    for x in xs:
        xt = torch.from_numpy(synth.to_time_major(x)).to("cuda:0")
        planes = plan.alloc_planes(x.shape[1])
        _, out = plan.dedisperse_search(xt, planes=planes, cap=8192)
        torch.cuda.synchronize()
        ref.append((xt, [p.clone() for p in planes], out.host()))
    for k, (xt, rplanes, rres) in enumerate(ref):
        say(f"static scratch call {k}: {xt.shape[0]} samples")
        planes = plan.alloc_planes(xt.shape[0])
        for p in planes:
            p.fill_(-1)
        out = plan.alloc_search_out(8192)
        assert _static(plan, xt, planes, out) == 0
        torch.cuda.synchronize()
        g = plan.geometry(xt.shape[0])
        for r in range(2):
            cols = g["plane_cols"][r]
            assert torch.equal(planes[r][:, :cols], rplanes[r][:, :cols]), (k, r)
        h = out.host()
        assert h[3] == rres[3]
        for a, b in zip(h[:3], rres[:3]):
            assert a.tobytes() == b.tobytes(), k
        if k == 1:
            rows = [[0, 60, 119], [0, 30, 59]]
            orc = oracle.run(spec, xs[1], rows=rows, search=False)
            ph = [sdd.plane_host(planes[r], g["plane_cols"][r]) for r in range(2)]
            compare_rows(spec, ph, orc)
    # library-held planes (NULL) through the binding
    out = plan.alloc_search_out(8192)
    plan.dedisperse_search_static(ref[0][0], None, out)
    torch.cuda.synchronize()
    assert out.host()[0].tobytes() == ref[0][2][0].tobytes()
    # refusals: a plan never used on the device, and sizes past the static maximum
    fresh = _plan(kw)
    xt = ref[1][0]
    st = _static(fresh, xt, fresh.alloc_planes(xt.shape[0]), fresh.alloc_search_out(16))
    assert st == A.SDD_ESTATE
    big = sdd.Plan(np.linspace(750.0, 550.0, 4096), 81.92e-6, dm_list=np.linspace(0, 1000, 64),
                   widths=[1, 2], layout="time")
    xb = torch.zeros((big.overlap + (1 << 16), 4096), dtype=torch.uint8, device="cuda:0")
    big.dedisperse_search(xb[: big.overlap + 1024], cap=16)    # creates the device tables
    torch.cuda.synchronize()
    st = _static(big, xb, big.alloc_planes(xb.shape[0]), big.alloc_search_out(16))
    assert st == A.SDD_ENOMEM
    # the scratch still serves a regular-size call afterwards
    out = plan.alloc_search_out(8192)
    planes = plan.alloc_planes(ref[1][0].shape[0])
    assert _static(plan, ref[1][0], planes, out) == 0
    torch.cuda.synchronize()
    assert out.host()[0].tobytes() == ref[1][2][0].tobytes()
