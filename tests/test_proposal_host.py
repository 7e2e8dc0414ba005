"""Host-side example drawing of the proposal network's training (no GPU)."""
import numpy as np

from paper_2606_15476_amd import FARM_NO_ID, proposal


def test_sample_pairs_labels_and_indices():
    rng = np.random.default_rng(0)
    n, R = 50, 4
    ids = rng.permutation(np.arange(1000, 1000 + n)).astype(np.uint32)   # ids unrelated to storage order
    bind_idx = rng.integers(0, n, (R, n))
    bind = ids[bind_idx]
    bind[2, :10] = FARM_NO_ID                                             # no binding: skipped
    preds = np.array([0, 3, 1, 4], np.int32)
    o, a, p, y = proposal.sample_pairs(bind, ids, preds, np.random.default_rng(1), per_relation=40, negatives=3)
    assert o.dtype == np.int32 and a.dtype == np.int32 and p.dtype == np.int32 and y.dtype == np.float32
    assert np.all((o >= 0) & (o < n)) and np.all((a >= 0) & (a < n))
    assert set(np.unique(p)) <= set(preds.tolist())
    # every positive is the exhaustive binding of its target, mapped from id to index
    r_of = {int(pp): r for r, pp in enumerate(preds)}
    for oo, aa, pp, yy in zip(o, a, p, y):
        r = r_of[int(pp)]
        if yy == 1.0:
            assert ids[aa] == bind[r, oo]
        else:
            assert aa != oo and ids[aa] != bind[r, oo]
    # three negatives per positive, none equal to its target
    assert (y == 0).sum() + (y == 1).sum() == y.size
    neg = y == 0
    assert np.all(a[neg] != o[neg])


def test_sample_pairs_uniform_negatives_cover_the_scene():
    n = 8
    ids = np.arange(n, dtype=np.uint32)
    bind = np.zeros((1, n), np.uint32)
    o, a, p, y = proposal.sample_pairs(bind, ids, np.array([2], np.int32), np.random.default_rng(2),
                                       per_relation=2000, negatives=3)
    neg = (y == 0) & (o == 3)
    # negatives of target 3 avoid 3 and its binding 0, and reach every other anchor
    assert set(np.unique(a[neg]).tolist()) == {1, 2, 4, 5, 6, 7}
