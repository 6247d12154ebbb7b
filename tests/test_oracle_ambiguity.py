"""Pins of the oracle's greedy ambiguity resolution (paper section 4: the
stage after the CKF that removes duplicate and fake tracks) on hand-worked
cases, and its invariants on the oracle's own tracks."""
import numpy as np

from synth import make_event


def _csr(tracks):
    off = np.zeros(len(tracks) + 1, np.int32)
    off[1:] = np.cumsum([len(t) for t in tracks])
    return off, np.concatenate([np.asarray(t, np.int32) for t in tracks])


def test_disjoint_tracks_are_all_kept():
    from oracle import ambiguity as OA
    off, meas = _csr([[0, 1, 2], [3, 4, 5], [6, 7, 8, 9]])
    keep, order = OA.resolve(off, meas, [1.0, 2.0, 3.0], [1, 1, 1])
    assert keep.all() and order == []


def test_identical_tracks_keep_the_better_one():
    """Two tracks with the same six measurements share all six: the one with
    the larger chi2/ndf goes; at equal chi2/ndf the larger index goes."""
    from oracle import ambiguity as OA
    off, meas = _csr([[0, 1, 2, 3, 4, 5], [0, 1, 2, 3, 4, 5]])
    keep, _ = OA.resolve(off, meas, [3.0, 5.0], [7, 7])
    assert list(keep) == [True, False]
    keep, _ = OA.resolve(off, meas, [5.0, 3.0], [7, 7])
    assert list(keep) == [False, True]
    keep, _ = OA.resolve(off, meas, [4.0, 4.0], [7, 7])
    assert list(keep) == [True, False]


def test_relative_share_decides():
    """A (6 measurements) and B (9) share 3: s/n is 1/2 for A and 1/3 for B,
    so A goes although B's chi2/ndf is worse; B then shares nothing."""
    from oracle import ambiguity as OA
    off, meas = _csr([[1, 2, 3, 4, 5, 6], [1, 2, 3, 7, 8, 9, 10, 11, 12]])
    keep, order = OA.resolve(off, meas, [1.0, 50.0], [7, 13])
    assert list(keep) == [False, True] and order == [0]


def test_chain_removes_the_middle_track():
    """A-B share 2, B-C share 2 (other measurements), A and C disjoint; all
    have 8 measurements: s/n is 1/4, 1/2, 1/4, so B goes and A, C stay."""
    from oracle import ambiguity as OA
    A = [0, 1, 2, 3, 4, 5, 6, 7]
    B = [0, 1, 10, 11, 12, 13, 20, 21]
    C = [20, 21, 30, 31, 32, 33, 34, 35]
    off, meas = _csr([A, B, C])
    keep, order = OA.resolve(off, meas, [1.0, 1.0, 1.0], [11, 11, 11])
    assert list(keep) == [True, False, True] and order == [1]


def test_one_shared_measurement_is_allowed():
    """With max_shared = 1 a single shared measurement is tolerated; with 0
    it is not and the worse track goes."""
    from oracle import ambiguity as OA
    off, meas = _csr([[0, 1, 2, 3, 4, 5], [5, 6, 7, 8, 9, 10]])
    keep, _ = OA.resolve(off, meas, [1.0, 2.0], [7, 7], max_shared=1)
    assert keep.all()
    keep, _ = OA.resolve(off, meas, [1.0, 2.0], [7, 7], max_shared=0)
    assert list(keep) == [True, False]


def test_rates_hand_built():
    """Four tracks over two particles: one clean match, one duplicate of it,
    one fake (no particle holds a majority), one match of the second
    particle."""
    from oracle import ambiguity as OA

    class Ev:
        pass
    ev = Ev()
    ev.meas_particle = np.array([0] * 6 + [1] * 6 + [-1] * 4)
    ev.particle_nhits = np.array([6, 6])
    off, meas = _csr([[0, 1, 2, 3, 4], [0, 1, 2, 3, 5], [4, 5, 12, 13, 14, 15], [6, 7, 8, 9]])
    r = OA.rates(ev, off, meas)
    assert (r["tracks"], r["fakes"], r["duplicates"]) == (4, 1, 1)
    r = OA.rates(ev, off, meas, keep=np.array([True, False, False, True]))
    assert (r["tracks"], r["fakes"], r["duplicates"]) == (2, 0, 0)


def test_invariants_on_oracle_tracks(oracle_lib, det_dense):
    """On the oracle's tracks of a mu = 100 event: no kept track shares more
    than one measurement with the other kept tracks; replaying the removal
    order, every removed track was bad and had the largest key among the bad
    tracks at its turn; the removal lowers the duplicate and fake counts."""
    from oracle import ambiguity as OA
    ev = make_event(det_dense, 41, mu=100)
    r = oracle_lib.ckf_find(oracle_lib.Inputs(det_dense.as_arrays(), (0, 0, 2.0), ev), n_threads=0)
    off, meas, chi2, ndf = r["offsets"], r["meas"], r["chi2"], r["ndf"]
    keep, order = OA.resolve(off, meas, chi2, ndf)
    assert 0 < len(order) < 0.02 * r["n_tracks"]
    use = np.bincount(meas[np.repeat(keep, np.diff(off))], minlength=ev.n_meas)
    for t in np.nonzero(keep)[0]:
        assert np.sum(use[meas[off[t]:off[t + 1]]] > 1) <= 1
    alive = np.ones(r["n_tracks"], bool)
    for t in order:
        use = np.bincount(meas[np.repeat(alive, np.diff(off))], minlength=ev.n_meas)
        s = np.array([np.sum(use[meas[off[u]:off[u + 1]]] > 1) for u in range(r["n_tracks"])])
        bad = np.nonzero(alive & (s > 1))[0]
        keys = [OA._key(s[u], off[u + 1] - off[u], chi2[u], ndf[u], u) for u in bad]
        assert bad[max(range(len(bad)), key=lambda i: keys[i])] == t
        alive[t] = False
    before, after = OA.rates(ev, off, meas), OA.rates(ev, off, meas, keep)
    assert after["duplicates"] <= before["duplicates"] and after["fakes"] <= before["fakes"]
    assert after["duplicates"] + after["fakes"] < before["duplicates"] + before["fakes"]
