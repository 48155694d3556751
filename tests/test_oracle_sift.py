"""Pins of the sifting oracle (square-stencil peak filter + DBSCAN-style
clustering in the DM-time plane) against hand-worked cases, an independent
DBSCAN (scikit-learn) and an image maximum filter (scipy)."""
import numpy as np
import pytest

import oracle
from oracle.sift import dbscan, sift_candidates, stencil_pass


class _R:
    def __init__(self, dms, dec=1):
        self.dms = np.asarray(dms, dtype=np.float64)
        self.dec = dec


class _P:
    def __init__(self, *ranges):
        self.ranges = list(ranges)


def test_hand_worked_two_events_and_noise():
    # DMs 0, 1, ..., 9; one event around (DM 5, t 1000), one at (DM 2, t 5000),
    # one isolated weak candidate at (DM 9, t 9000)
    plan = _P(_R(np.arange(10.0)))
    rng = [0] * 7
    dmi = [4, 5, 6, 5, 2, 2, 9]
    smp = [1001, 1000, 999, 1010, 5000, 5003, 9000]
    snr = [9.0, 12.0, 8.0, 10.0, 7.5, 7.6, 7.1]
    # stencil (1.0, 5): index 1 (12.0) suppresses 0 and 2; 3 (t 1010) is 10 samples away
    kept = stencil_pass(*oracle.sift_coords(plan, rng, dmi, smp, snr), list(range(7)), 1.0, 5)
    assert kept == [1, 3, 5, 6]
    # clustering: eps (1.0, 20), min_pts 2 -> {1, 3} cluster keeps 1; 5 alone is noise
    k, sz = sift_candidates(plan, rng, dmi, smp, snr, stencils=[(1.0, 5)], eps_dm=1.0,
                            eps_t=20, min_pts=2)
    assert (k, sz) == ([1], [2])
    # min_pts 1: every survivor is a core point; clusters {1, 3}, {5}, {6}
    k, sz = sift_candidates(plan, rng, dmi, smp, snr, stencils=[(1.0, 5)], eps_dm=1.0,
                            eps_t=20, min_pts=1)
    assert (k, sz) == ([1, 5, 6], [2, 1, 1])


def test_ties_prefer_the_earlier_candidate():
    plan = _P(_R([0.0, 1.0]))
    k = stencil_pass(*oracle.sift_coords(plan, [0, 0], [0, 1], [100, 101], [8.0, 8.0]),
                     [0, 1], 1.0, 1)
    assert k == [0]


def test_decimated_range_uses_native_samples():
    plan = _P(_R([0.0]), _R([0.5], dec=4))
    # range-1 sample 250 is native sample 1000, next to range-0 sample 1002
    dm, t, _ = oracle.sift_coords(plan, [0, 1], [0, 0], [1002, 250], [7.0, 9.0])
    assert t.tolist() == [1002, 1000]
    k = stencil_pass(dm, t, np.float32([7.0, 9.0]), [0, 1], 0.5, 2)
    assert k == [1]


def test_identities_and_limits():
    rng_ = np.random.Generator(np.random.PCG64(5))
    plan = _P(_R(np.sort(rng_.uniform(0, 100, 40))))
    n = 60
    dmi = rng_.integers(0, 40, n)
    smp = rng_.integers(0, 10000, n)
    order = np.lexsort((smp, dmi))
    dmi, smp = dmi[order].tolist(), smp[order].tolist()
    snr = rng_.uniform(6, 20, n).astype(np.float32).tolist()
    rng = [0] * n
    # no stencil, no clustering: identity
    assert sift_candidates(plan, rng, dmi, smp, snr)[0] == list(range(n))
    # a zero stencil suppresses only candidates at identical (DM, t)
    k, _ = sift_candidates(plan, rng, dmi, smp, snr, stencils=[(0.0, 0)])
    assert k == list(range(n))
    # a huge neighbourhood with min_pts 1: one cluster, the global best
    k, sz = sift_candidates(plan, rng, dmi, smp, snr, eps_dm=1e9, eps_t=10 ** 9, min_pts=1)
    assert k == [int(np.argmax(snr))] and sz == [n]
    # min_pts above n: everything is noise
    assert sift_candidates(plan, rng, dmi, smp, snr, eps_dm=1.0, eps_t=10, min_pts=n + 1)[0] == []


def test_stencil_equals_image_maximum_filter():
    """On a lattice (uniform DM step, integer times) with distinct S/N, one
    stencil pass keeps exactly the candidates whose S/N is the maximum of
    their (2k+1) x (2m+1) window of the S/N image (-inf where empty)."""
    from scipy.ndimage import maximum_filter
    g = np.random.Generator(np.random.PCG64(11))
    ndm, nt, k, m = 30, 80, 2, 3
    occ = g.random((ndm, nt)) < 0.25
    img = np.full((ndm, nt), -np.inf)
    img[occ] = g.permutation(int(occ.sum())).astype(np.float64) + 7.0  # distinct, exact in f32
    plan = _P(_R(np.arange(ndm) * 0.5))
    ii, jj = np.nonzero(occ)          # row-major: sorted by (DM index, sample)
    snr = img[ii, jj].astype(np.float32)
    kept = stencil_pass(*oracle.sift_coords(plan, [0] * len(ii), ii, jj, snr),
                        list(range(len(ii))), k * 0.5, m)
    mf = maximum_filter(img, size=(2 * k + 1, 2 * m + 1), mode="constant", cval=-np.inf)
    expect = [p for p in range(len(ii)) if img[ii[p], jj[p]] == mf[ii[p], jj[p]]]
    assert kept == expect


@pytest.mark.parametrize("min_pts", [1, 3, 5])
def test_dbscan_matches_scikit_learn(min_pts):
    """Core points and the partition of core points into clusters equal
    scikit-learn's DBSCAN (Chebyshev metric on coordinates scaled by the
    neighbourhood half-sizes, eps 1); each border point joins a cluster of
    one of its core neighbours; noise is the same set."""
    from sklearn.cluster import DBSCAN
    g = np.random.Generator(np.random.PCG64(100 + min_pts))
    n = 300
    dm = np.sort(g.uniform(0, 50, n))
    t = g.integers(0, 20000, n).astype(np.int64)
    eps_dm, eps_t = 1.3, 400
    pts = list(range(n))
    label, core = dbscan(dm, t, pts, eps_dm, eps_t, min_pts)
    X = np.stack([dm / eps_dm, t / eps_t], axis=1)
    sk = DBSCAN(eps=1.0, min_samples=min_pts, metric="chebyshev").fit(X)
    assert core == set(sk.core_sample_indices_.tolist())
    # the same partition of core points
    part_o = {}
    part_s = {}
    for p in sorted(core):
        part_o.setdefault(label[p], set()).add(p)
        part_s.setdefault(int(sk.labels_[p]), set()).add(p)
    assert sorted(map(sorted, part_o.values())) == sorted(map(sorted, part_s.values()))
    # border points: in the cluster of a core neighbour; noise identical
    for p in pts:
        if p in core:
            continue
        nb = [q for q in pts if q in core and abs(dm[q] - dm[p]) <= eps_dm
              and abs(int(t[q]) - int(t[p])) <= eps_t]
        if nb:
            assert label[p] == label[min(nb)]
            assert sk.labels_[p] in {sk.labels_[q] for q in nb}
        else:
            assert label[p] == -1 and sk.labels_[p] == -1
