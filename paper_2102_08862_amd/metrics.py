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

Collision candidates (collision_quality) are judged by each track's
majority collision (the collision of its majority particle):
  - purity = anchors in groups of >= 10 anchors whose collision is their
    group's majority collision / those anchors;
  - a collision with >= 5 anchors is found if the group holding most of its
    anchors holds at least half of them and has it as majority collision;
  - attached = other tracks with a time that joined a group / those tracks;
    correct = attached tracks whose collision is their group's majority.
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


def track_majority(labels, clusters, lengths):
    """Majority label of each track (ties: the smaller label; -1 if noise
    wins); labels int32[n], clusters = concatenated cluster lists."""
    lengths = np.asarray(lengths, np.int64)
    T = len(lengths)
    if T == 0:
        return np.zeros(0, np.int64)
    tid = np.repeat(np.arange(T), lengths)
    lab = np.asarray(labels)[np.asarray(clusters)].astype(np.int64)
    key = tid * (1 << 32) + (lab + 1)
    uk, uc = np.unique(key, return_counts=True)
    ut = uk >> 32
    ul = (uk & 0xffffffff) - 1
    order = np.lexsort((-uc, ut))
    first = np.ones(len(order), bool)
    first[1:] = ut[order][1:] != ut[order][:-1]
    out = np.full(T, -1, np.int64)
    out[ut[order][first]] = ul[order][first]
    return out


def collision_quality(coll, group, lengths, has_time, min_len):
    """Collision-candidate quality of one frame side: coll = collision id of
    each track's majority particle (negative for fakes), group = the track's
    group (-1 none), lengths = clusters per track, has_time = finite t0."""
    coll, group = np.asarray(coll, np.float64), np.asarray(group)
    lengths, has_time = np.asarray(lengths), np.asarray(has_time, bool)
    anc = has_time & (lengths >= min_len)
    ng = int(group.max()) + 1 if len(group) else 0
    ga, ca = group[anc], coll[anc]
    size = np.bincount(ga, minlength=ng)
    maj = np.full(ng + 1, -2.0)
    if len(ga):
        o = np.lexsort((ca, ga))
        g_s, c_s = ga[o], ca[o]
        start = np.r_[True, (g_s[1:] != g_s[:-1]) | (c_s[1:] != c_s[:-1])]
        idx = np.nonzero(start)[0]
        run = np.diff(np.r_[idx, len(g_s)])
        o2 = np.lexsort((-run, g_s[idx]))
        first = np.r_[True, g_s[idx][o2][1:] != g_s[idx][o2][:-1]]
        maj[g_s[idx][o2][first]] = c_s[idx][o2][first]
    big = size[ga] >= 10 if len(ga) else np.zeros(0, bool)
    ok_a = (ca == maj[ga]) & (ca >= 0)
    purity = float(ok_a[big].mean()) if big.any() else 1.0
    found = considered = 0
    v, c = np.unique(ca[ca >= 0], return_counts=True)
    for vv, cc in zip(v[c >= 5], c[c >= 5]):
        considered += 1
        ug, uc = np.unique(ga[ca == vv], return_counts=True)
        k = int(np.argmax(uc))
        found += bool(uc[k] >= 0.5 * cc and maj[ug[k]] == vv)
    short = has_time & ~anc
    att = short & (group >= 0)
    correct = (coll == maj[np.where(group >= 0, group, ng)]) & (coll >= 0)
    return dict(groups=ng, anchors=int(anc.sum()), purity=purity, collisions=considered, found=found,
                short=int(short.sum()), attached=float(att.sum() / max(short.sum(), 1)),
                correct=float(correct[att].mean()) if att.any() else 1.0)
