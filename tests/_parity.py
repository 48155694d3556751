"""Helpers shared by the GPU parity tests: run the library on a seeded input
and compare with the oracle (bit-exact planes; S/N within the stated
relative tolerance; identical candidate lists away from the threshold)."""
from __future__ import annotations

import sys

import numpy as np

import oracle

SNR_RTOL = 1e-4        # relative S/N tolerance vs the FP64 oracle
THR_BAND = 1e-4        # candidates with |S/N/threshold - 1| below this are optional


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_run(plan, x_cm, search=True, time_major=False, planes=True, tile=None, cap=65536,
            stream=None):
    """Upload x (channel-major numpy uint8) in the plan's layout and run the
    path. Returns (planes_host list or None, search tuple or None, geometry)."""
    import torch
    import paper_2605_03531_amd as sdd
    if tile is not None:
        plan.set_tile(tile)
    xh = np.ascontiguousarray(x_cm.T) if time_major else x_cm
    x = torch.from_numpy(xh).to("cuda:0")
    T = x_cm.shape[1]
    g = plan.geometry(T)
    pl = plan.alloc_planes(T) if planes else None
    if search and plan.nwidths:
        pl, out = plan.dedisperse_search(x, planes=pl, cap=cap, stream=stream)
    else:
        plan.dedisperse(x, planes=pl, stream=stream)
        out = None
    torch.cuda.synchronize()
    ph = None
    if pl is not None:
        ph = [sdd.plane_host(pl[r], g["plane_cols"][r]) for r in range(plan.nranges)]
    res = out.host() if out is not None else None
    del x
    return ph, res, g


def oracle_plan(plan_kwargs):
    kw = dict(plan_kwargs)
    kw["threshold"] = float(np.float32(kw.get("threshold", 7.0)))
    return oracle.make_plan(**kw)


def compare_rows(spec, gpu_planes, orc):
    """orc = oracle.run(...) output. Planes bit-exact on the oracle's rows."""
    for r, (rows, y, _) in enumerate(orc):
        got = gpu_planes[r][rows].astype(np.int64)
        assert got.shape == y.shape, (r, got.shape, y.shape)
        bad = np.argwhere(got != y)
        assert bad.size == 0, f"range {r}: {len(bad)} plane mismatches, first {bad[:5].tolist()}"


def compare_search(spec, res, orc, full_rows: bool):
    """Per-trial best and stats on the oracle's rows, and the candidates of
    those rows (the whole ordered list if full_rows)."""
    best, stats, cands, ncand = res
    thr = spec.threshold
    max_rel = 0.0
    expect = []
    for r, (rows, y, rr) in enumerate(orc):
        off = sum(len(s.dms) for s in spec.ranges[:r])
        for k, i in enumerate(rows):
            o = rr[k]
            g = off + i
            st = stats[g]
            assert int(st["n"]) == o.n and int(st["s1"]) == o.s1 and int(st["s2"]) == o.s2, (r, i)
            assert st["mean"] == o.mean or abs(st["mean"] / o.mean - 1) < 1e-12
            assert abs(st["std"] - o.std) <= 1e-12 * max(o.std, 1e-300)
            b = best[g]
            assert (int(b["sample"]), int(b["width"])) == (o.best[1], o.best[2]), (r, i, b, o.best)
            if o.best[0] != 0.0:
                rel = abs(float(b["snr"]) / o.best[0] - 1.0)
                max_rel = max(max_rel, rel)
                assert rel < SNR_RTOL, (r, i, float(b["snr"]), o.best[0])
            else:
                assert float(b["snr"]) == 0.0
            for (s, j, w) in o.cands:
                expect.append((r, i, j, w, s))
    got = [(int(c["range"]), int(c["dm_index"]), int(c["sample"]), int(c["width"]),
            float(c["snr"])) for c in cands]
    assert ncand >= len(got)
    if not full_rows:
        keep = {(r, i) for r, (rows, _, _) in enumerate(orc) for i in rows}
        got = [c for c in got if (c[0], c[1]) in keep]
    if True:

        def firm(s):
            return abs(s / thr - 1.0) >= THR_BAND if thr != 0 else abs(s) >= THR_BAND

        ge = [c for c in got if firm(c[4])]
        ee = [c for c in expect if firm(c[4])]
        assert [c[:4] for c in ge] == [c[:4] for c in ee], (len(ge), len(ee))
        for a, b in zip(ge, ee):
            assert abs(a[4] / b[4] - 1.0) < SNR_RTOL
        # order: (range, dm, sample)
        keys = [c[:3] for c in got]
        assert keys == sorted(keys)
    return max_rel


def host_workers() -> int:
    """Host threads for oracle work in the full-size tests (at most 16)."""
    import os
    return max(1, min(16, os.cpu_count() or 1))


def oracle_rows_parallel(spec, x, rows, search=True):
    """oracle.run(spec, x, rows) with the rows of each range shared among host
    threads (numpy releases the GIL in the row additions). Same output
    format: per range (rows, plane rows, RowResult list or None)."""
    from concurrent.futures import ThreadPoolExecutor
    assert spec.dered is None
    owned = spec.owned(x.shape[1])
    out = []
    with ThreadPoolExecutor(host_workers()) as ex:
        for r, rs in enumerate(spec.ranges):
            rr = list(rows[r])
            length = owned[r] + spec.w_max - 1
            if not rr:
                out.append((rr, np.zeros((0, length), dtype=np.int64), [] if search else None))
                continue
            xr = x if rs.dec == 1 else oracle.decimate(x, rs.dec)

            def one(i, xr=xr, rs=rs, r=r, length=length):
                y = oracle.dedisperse_rows(xr, rs.delays, [i], length)[0]
                res = None
                if search and spec.widths:
                    res = oracle.search_row(y, spec.widths, owned[r], spec.cand_block,
                                            spec.threshold, spec.stats)
                return y, res

            parts = list(ex.map(one, rr))
            out.append((rr, np.stack([p[0] for p in parts]),
                        [p[1] for p in parts] if search and spec.widths else None))
    return out


def oracle_checksums_parallel(xr, delays, length):
    """oracle.plane_checksums over channel blocks in host threads, summed."""
    from concurrent.futures import ThreadPoolExecutor
    nchan = xr.shape[0]
    step = max(1, -(-nchan // (4 * host_workers())))
    blocks = [(c, min(nchan, c + step)) for c in range(0, nchan, step)]
    with ThreadPoolExecutor(host_workers()) as ex:
        parts = list(ex.map(lambda b: oracle.plane_checksums(xr[b[0]:b[1]],
                                                             delays[:, b[0]:b[1]], length),
                            blocks))
    return sum(p[0] for p in parts), sum(p[1] for p in parts)


def device_checksums(plane, cols):
    """Row sums and index-weighted row sums of a device plane ([rows][pitch]
    int32 view of uint32 sums below 2^31), int64 numpy."""
    import torch
    rows = plane.shape[0]
    j = torch.arange(cols, device=plane.device, dtype=torch.int64)
    a = torch.empty(rows, dtype=torch.int64, device=plane.device)
    b = torch.empty(rows, dtype=torch.int64, device=plane.device)
    for r0 in range(0, rows, 128):
        blk = plane[r0:r0 + 128, :cols].to(torch.int64)
        a[r0:r0 + 128] = blk.sum(dim=1)
        b[r0:r0 + 128] = (blk * j).sum(dim=1)
    torch.cuda.synchronize()
    return a.cpu().numpy(), b.cpu().numpy()
