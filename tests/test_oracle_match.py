"""Pins of the oracle's label-overlap table (coalescence tracking between two
bubble labellings): hand-worked cases and brute-force counting (CPU)."""
import numpy as np

from oracle import match_labels


def test_two_bubbles_merge_and_one_splits():
    # worked by hand on a 4 x 6 grid: old bubbles 1 and 2 merge into new
    # bubble 1; old bubble 3 splits into new bubbles 2 and 3; a liquid cell
    # and a cell that was liquid before do not count
    old = np.array([[1, 1, 0, 2, 2, 0],
                    [1, 1, 0, 2, 2, 0],
                    [0, 0, 0, 0, 0, 0],
                    [3, 3, 3, 3, 0, 0]])
    new = np.array([[1, 1, 1, 1, 1, 0],
                    [1, 0, 0, 1, 1, 1],
                    [0, 0, 0, 0, 0, 0],
                    [2, 2, 0, 3, 0, 0]])
    got = match_labels(old, new)
    want = np.array([[1, 1, 3], [2, 1, 4], [3, 2, 2], [3, 3, 1]])
    assert np.array_equal(got, want)
    merges = {b for b in np.unique(got[:, 1]) if (got[:, 1] == b).sum() >= 2}
    splits = {a for a in np.unique(got[:, 0]) if (got[:, 0] == a).sum() >= 2}
    assert merges == {1} and splits == {3}


def test_no_overlap_and_identity():
    old = np.zeros((5, 7), np.int32)
    assert match_labels(old, old).shape == (0, 3)
    lab = np.array([[0, 1, 1], [2, 0, 3], [2, 2, 3]])
    got = match_labels(lab, lab)
    assert np.array_equal(got, np.array([[1, 1, 2], [2, 2, 3], [3, 3, 2]]))


def test_brute_force_random():
    rng = np.random.default_rng(7)
    for _ in range(20):
        shape = tuple(rng.integers(1, 9, size=3))
        old = rng.integers(0, 5, size=shape)
        new = rng.integers(0, 4, size=shape)
        got = match_labels(old, new)
        want = []
        for a in range(1, 5):
            for b in range(1, 4):
                n = 0
                for idx in np.ndindex(*shape):
                    if old[idx] == a and new[idx] == b:
                        n += 1
                if n:
                    want.append((a, b, n))
        assert [tuple(r) for r in got.tolist()] == want
        assert got[:, 2].sum() == np.sum((old > 0) & (new > 0)) if len(got) else True
