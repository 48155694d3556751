"""Candidate sifting after the single-pulse search: redundant candidates of
one event are removed with square stencils in the DM-time plane, then the
survivors are grouped by density-based clustering in the DM-time plane and
each group keeps its highest-S/N member (Section 2.1 names both steps; the
clustering is DBSCAN, Ester et al. 1996).

TEST INFRASTRUCTURE ONLY (see the package docstring). Plain loops over the
candidate list, O(n^2); every comparison is the FP64 / integer / float32
comparison stated below.

Readings (the paper gives neither stencil sizes nor clustering parameters):
  S1  Coordinates of a candidate: the FP64 trial DM of its range and DM
      index (pc cm^-3, the plan's value), its window start in native samples
      t = sample * dec_r (int64), and its reported float32 S/N.
  S2  p is better than q iff snr_p > snr_q, or snr_p == snr_q and p comes
      earlier in the candidate list (ordered by range, DM index, sample).
  S3  Square stencil of half-sizes (a, b): q lies in p's stencil iff
      |DM_q - DM_p| <= a (FP64 subtraction, absolute value, comparison) and
      |t_q - t_p| <= b. A pass keeps p iff no better candidate of the pass's
      input lies in p's stencil. Passes ("stencils of different sizes") run
      in the order given, each on the survivors of the previous one.
  S4  Clustering: DBSCAN with the rectangular neighbourhood
      |DM_q - DM_p| <= eps_dm, |t_q - t_p| <= eps_t and core threshold
      min_pts (a point counts itself). Clusters are the connected components
      of the core points under the neighbourhood relation. A non-core point
      with a core neighbour joins the cluster of its earliest (list order)
      core neighbour; a point with none is noise and is dropped.
  S5  Each cluster keeps its best member (S2); the output is in list order
      with each kept candidate's cluster size (its members, core and border).
  S6  min_pts = 0 turns clustering off: every stencil survivor is kept with
      cluster size 1.
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np

__all__ = ["sift_coords", "stencil_pass", "dbscan", "sift_candidates"]


def sift_coords(plan, rng: Sequence[int], dmi: Sequence[int], sample: Sequence[int],
                snr: Sequence[float]):
    """(DM fp64, t int64 native samples, snr float32) per candidate (S1)."""
    dm = np.array([plan.ranges[r].dms[i] for r, i in zip(rng, dmi)], dtype=np.float64)
    t = np.array([int(s) * plan.ranges[r].dec for r, s in zip(rng, sample)], dtype=np.int64)
    return dm, t, np.asarray(snr, dtype=np.float32)


def _better(snr, q: int, p: int) -> bool:
    """S2: candidate q is better than candidate p."""
    return bool(snr[q] > snr[p]) or (bool(snr[q] == snr[p]) and q < p)


def _near(dm, t, p: int, q: int, a: float, b: int) -> bool:
    return abs(float(dm[q]) - float(dm[p])) <= a and abs(int(t[q]) - int(t[p])) <= b


def stencil_pass(dm, t, snr, alive: List[int], a: float, b: int) -> List[int]:
    """One square-stencil pass over the candidates in `alive` (S3)."""
    keep = []
    for p in alive:
        if not any(q != p and _near(dm, t, p, q, a, b) and _better(snr, q, p) for q in alive):
            keep.append(p)
    return keep


def dbscan(dm, t, pts: List[int], eps_dm: float, eps_t: int, min_pts: int):
    """Cluster label (the smallest core index of its component) per point of
    `pts`, or -1 for noise (S4). Returns (labels dict, core set)."""
    nbr = {p: [q for q in pts if _near(dm, t, p, q, eps_dm, eps_t)] for p in pts}
    core = {p for p in pts if len(nbr[p]) >= min_pts}
    label = {}
    for p in sorted(core):
        if p in label:
            continue
        # breadth-first walk of p's component over core points
        comp, todo = {p}, [p]
        while todo:
            u = todo.pop()
            for v in nbr[u]:
                if v in core and v not in comp:
                    comp.add(v)
                    todo.append(v)
        root = min(comp)
        for v in comp:
            label[v] = root
    for p in pts:
        if p in core:
            continue
        cn = [q for q in nbr[p] if q in core]
        label[p] = label[min(cn)] if cn else -1
    return label, core


def sift_candidates(plan, rng, dmi, sample, snr, stencils: Sequence[Tuple[float, int]] = (),
                    eps_dm: float = 0.0, eps_t: int = 0, min_pts: int = 0):
    """Indices (into the input list) of the kept candidates, in list order,
    and their cluster sizes (S1-S6)."""
    dm, t, sn = sift_coords(plan, rng, dmi, sample, snr)
    alive = list(range(len(dm)))
    for a, b in stencils:
        alive = stencil_pass(dm, t, sn, alive, float(a), int(b))
    if min_pts <= 0:
        return alive, [1] * len(alive)
    label, _ = dbscan(dm, t, alive, float(eps_dm), int(eps_t), int(min_pts))
    members = {}
    for p in alive:
        if label[p] >= 0:
            members.setdefault(label[p], []).append(p)
    kept, sizes = [], []
    for root, mem in members.items():
        best = mem[0]
        for q in mem[1:]:
            if _better(sn, q, best):
                best = q
        kept.append(best)
        sizes.append(len(mem))
    order = np.argsort(kept, kind="stable")
    return [kept[k] for k in order], [sizes[k] for k in order]
