"""Oracle of the greedy ambiguity resolution of found tracks.

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle/``): plain Python, one
removal at a time, written from the definition below and sharing nothing
with the GPU library.

The paper (section 4) names ambiguity resolution as the stage after the CKF
that removes duplicate tracks (several tracks with the same or nearly the
same measurements) and fake ones.  It gives no algorithm; the reading here
is the greedy resolution by shared measurements:

* a measurement is *shared* when more than one surviving track holds it;
  s(t) is the number of track t's measurements that are shared, n(t) the
  number of its measurements;
* a surviving track is *bad* when s(t) > max_shared;
* while a bad track exists, the bad track with the largest s(t) / n(t) is
  removed; ties go to the larger chi2 / ndf (taken in FP32, the precision
  both implementations decide it in), then to the larger track index; the
  shared counts are then recounted.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def _key(s, n, chi2, ndf, t):
    q = np.float32(np.float32(chi2) / np.float32(max(ndf, 1)))
    return (Fraction(int(s), int(n)), float(q), int(t))


def resolve(offsets, meas, chi2, ndf, max_shared=1):
    """Keep mask [n_tracks] (True = kept) and the removal order.  The shared
    counts are kept up to date as tracks go (a measurement whose use drops
    to one stops being shared for the track still holding it)."""
    offsets = np.asarray(offsets)
    nt = len(offsets) - 1
    tracks = [[int(m) for m in meas[offsets[t]:offsets[t + 1]]] for t in range(nt)]
    holders = {}
    for t, ms in enumerate(tracks):
        for m in ms:
            holders.setdefault(m, set()).add(t)
    shared = [sum(1 for m in ms if len(holders[m]) > 1) for ms in tracks]
    alive = np.ones(nt, bool)
    order = []
    while True:
        bad = [t for t in range(nt) if alive[t] and tracks[t] and shared[t] > max_shared]
        if not bad:
            return alive, order
        best = max(bad, key=lambda t: _key(shared[t], len(tracks[t]), chi2[t], ndf[t], t))
        alive[best] = False
        order.append(best)
        for m in tracks[best]:
            h = holders[m]
            was_shared = len(h) > 1
            h.discard(best)
            if was_shared and len(h) == 1:
                shared[next(iter(h))] -= 1


def rates(ev, offsets, meas, keep=None):
    """(efficiency-style counts of section 3.1 and section 4 rates) for the
    kept tracks: fake = no particle is double-matched, duplicate = a
    double-matched particle already matched by an earlier kept track.
    Returns dict(tracks, fakes, duplicates, fake_rate, duplicate_rate)."""
    nt = len(offsets) - 1
    mp = ev.meas_particle
    seen, fakes, dups, n = set(), 0, 0, 0
    for t in range(nt):
        if keep is not None and not keep[t]:
            continue
        n += 1
        ids = meas[offsets[t]:offsets[t + 1]]
        parts, cnt = np.unique(mp[ids], return_counts=True)
        k = int(np.argmax(cnt))
        p, N = int(parts[k]), int(cnt[k])
        if p < 0 or not (N > len(ids) / 2 and N > ev.particle_nhits[p] / 2):
            fakes += 1
        elif p in seen:
            dups += 1
        else:
            seen.add(p)
    return dict(tracks=n, fakes=fakes, duplicates=dups, fake_rate=fakes / max(1, n),
                duplicate_rate=dups / max(1, n))
