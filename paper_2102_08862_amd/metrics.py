"""Track-finding quality against the generator's truth labels.

Definitions (the paper prints no efficiency figures; these are the readings
used to judge the tracker and the learned pruning):
  - a (particle, sector) pair is findable if the particle left at least
    FINDABLE_MIN signal clusters in that sector;
  - a track matches particle p if at least MATCH_FRAC of its clusters carry
    label p, otherwise it is fake;
  - efficiency = findable pairs with >= 1 matched track in that sector /
    findable pairs;
  - clone rate = matched tracks beyond the first per pair / matched pairs;
  - fake rate = fake tracks / all tracks;
  - hit efficiency = signal clusters of findable pairs that sit on a track
    matched to their own particle / signal clusters of findable pairs.
"""
from __future__ import annotations

import numpy as np

FINDABLE_MIN = 30
MATCH_FRAC = 0.9


def sector_counts(labels, clusters, lengths):
    """Counts of one sector: labels int32[n] (-1 noise), clusters = the
    sector's concatenated track cluster lists (input indices), lengths =
    clusters per track. Returns a dict of raw counts (summable)."""
    labels = np.asarray(labels)
    lengths = np.asarray(lengths, np.int64)
    T = len(lengths)
    sig = labels[labels >= 0]
    pids, pcnt = np.unique(sig, return_counts=True)
    findable = pids[pcnt >= FINDABLE_MIN]
    n_find = len(findable)
    find_hits = int(pcnt[pcnt >= FINDABLE_MIN].sum())
    if T == 0:
        return dict(findable=n_find, found=0, tracks=0, fakes=0, clones=0, matched_pairs=0,
                    find_hits=find_hits, good_hits=0)
    tid = np.repeat(np.arange(T), lengths)
    lab = labels[np.asarray(clusters)]
    # majority label per track
    key = tid.astype(np.int64) * (1 << 32) + (lab.astype(np.int64) + 1)
    uk, uc = np.unique(key, return_counts=True)
    ut = (uk >> 32).astype(np.int64)
    ul = (uk & 0xffffffff).astype(np.int64) - 1
    order = np.lexsort((-uc, ut))
    first = np.ones(len(order), bool)
    first[1:] = ut[order][1:] != ut[order][:-1]
    best = order[first]
    maj_t, maj_l, maj_c = ut[best], ul[best], uc[best]
    frac = maj_c / lengths[maj_t]
    matched = (frac >= MATCH_FRAC) & (maj_l >= 0)
    n_fake = int(T - matched.sum())
    mlab = maj_l[matched]
    is_find = np.isin(mlab, findable)
    found_p, found_c = np.unique(mlab[is_find], return_counts=True)
    clones = int((found_c - 1).sum())
    # hits on a matched track that carry the track's own (findable) label
    good_tracks = maj_t[matched][is_find]
    good_lab = mlab[is_find]
    tl = np.full(T, -2, np.int64)
    tl[good_tracks] = good_lab
    good_hits = int((lab == tl[tid]).sum())
    return dict(findable=n_find, found=len(found_p), tracks=T, fakes=n_fake, clones=clones,
                matched_pairs=len(found_p), find_hits=find_hits, good_hits=good_hits)


def summarize(counts):
    """Rates from summed sector counts."""
    c = {k: sum(d[k] for d in counts) for k in counts[0]} if counts else {}
    if not c:
        return {}
    return dict(
        efficiency=c["found"] / max(1, c["findable"]),
        fake_rate=c["fakes"] / max(1, c["tracks"]),
        clone_rate=c["clones"] / max(1, c["matched_pairs"]),
        hit_efficiency=c["good_hits"] / max(1, c["find_hits"]),
        tracks=c["tracks"], findable=c["findable"],
    )


def frame_quality(frame, get_clusters, get_lengths, sectors=None):
    """Quality of a whole frame; get_clusters(s) / get_lengths(s) return the
    tracker's outputs for sector s."""
    ss = range(len(frame.labels)) if sectors is None else sectors
    return summarize([sector_counts(frame.labels[s], get_clusters(s), get_lengths(s)) for s in ss])
