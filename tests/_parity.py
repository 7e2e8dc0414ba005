"""Parity criteria between the GPU path and the FP64 oracle.

Tolerances (derived from the FP32 arithmetic of the GPU path):
  * returned TopK scores and rescored scores: |s_gpu - s_64| <= REL *
    max(s_64, TOPK_FLOOR), REL = 1e-5 the stated FP32 bar: pure relative for
    every score >= TOPK_FLOOR = 0.01 (every returned score of the workloads).
    Below it -- only degenerate tests with random query vectors return such
    scores -- the bound is 1e-7 absolute: a cosine near zero is a cancelling
    FP32 sum whose rounding (a few 2^-24 of the unit vectors' magnitudes) is
    not small relative to the value itself.
  * intermediate values (full score matrices, relation terms, similarities):
    |x_gpu - x_64| <= REL * |x_64| + ABS.  ABS covers values near zero: an FP32
    dot product of two unit vectors of width d carries a rounding error of
    order sqrt(d) * 2^-24 in practice (the worst-case bound d * 2^-24 is far
    looser); 4e-6 is about twice the typical error at d = 1152 and dominates
    only below 0.4.
  * TopK ids: exact wherever the oracle's score at that rank is separated
    from both neighbours by more than GAP = 1e-5; inside a near-tie group any
    order is correct, and the oracle score of each returned id must lie within
    GAP (plus value tolerance) of the oracle score at that rank.
  * Closest/Farthest: the rank is an integer decided by comparing squared
    distances.  The GPU sums them in FP32 from FP32 center differences; each
    difference, square and sum rounds once, so its squared distance is within
    5 * 2^-24 (3e-7) relative of the exact one.  Where two candidates' squared
    distances lie within RANK_EPS = 1e-6 relative of each other either order
    is correct; the oracle's rank_tolerance mode gives the lowest and highest
    values over those orders, and the GPU value must lie between them.
  * Between: its anchors range over the 64 anchors of largest similarity per
    description; an anchor whose similarity lies within BETWEEN_EPS = ABS of
    the 64th largest may be in or out of an FP32 implementation's set, so the
    oracle's between_tolerance mode gives the lowest term (surely included
    anchors only) and the highest (every possibly included one).
"""
import numpy as np

REL = 1e-5
ABS = 4e-6
GAP = 1e-5
TOPK_FLOOR = 1e-2
RANK_EPS = 1e-6
RANK_PREDS = (9, 10)
BETWEEN = 12
BETWEEN_EPS = ABS  # FP32 similarities within ABS of the oracle's may select another boundary anchor


def value_tol(x64):
    return REL * np.abs(x64) + ABS


def assert_values_close(got, want, what="values", rel=REL, abs_=ABS):
    got = np.asarray(got, np.float64)
    want = np.asarray(want, np.float64)
    err = np.abs(got - want)
    tol = rel * np.abs(want) + abs_
    bad = err > tol
    if bad.any():
        i = np.unravel_index(np.argmax(err - tol), err.shape)
        raise AssertionError(f"{what}: {int(bad.sum())} of {bad.size} outside tolerance; worst at {i}: "
                             f"got {got[i]!r} want {want[i]!r} (tol {tol[i]:.3g})")
    return float(np.max(err / np.maximum(np.abs(want), 1e-30))) if err.size else 0.0


def assert_returned_scores(got, want, what="returned scores"):
    """Returned TopK / rescored scores: |got - want| <= REL * max(want, TOPK_FLOOR)."""
    got = np.asarray(got, np.float64)
    want = np.asarray(want, np.float64)
    tol = REL * np.maximum(np.abs(want), TOPK_FLOOR)
    bad = np.abs(got - want) > tol
    if bad.any():
        i = np.unravel_index(np.argmax(np.abs(got - want) - tol), got.shape)
        raise AssertionError(f"{what}: {int(bad.sum())} of {bad.size} outside tolerance; worst at {i}: "
                             f"got {got[i]!r} want {want[i]!r}")


def assert_values_within(got, lo, hi, what="values", rel=REL, abs_=ABS):
    """lo - tol(lo) <= got <= hi + tol(hi) element-wise (lo == hi: assert_values_close)."""
    got = np.asarray(got, np.float64)
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    below = (lo - rel * np.abs(lo) - abs_) - got
    above = got - (hi + rel * np.abs(hi) + abs_)
    worst = np.maximum(below, above)
    bad = worst > 0
    if bad.any():
        i = np.unravel_index(np.argmax(worst), worst.shape)
        raise AssertionError(f"{what}: {int(bad.sum())} of {bad.size} outside [lo, hi]; worst at {i}: "
                             f"got {got[i]!r} in [{lo[i]!r}, {hi[i]!r}]")


def has_rank_preds(qb):
    return bool(np.isin(np.asarray(qb.rel_pred), RANK_PREDS).any())


def has_between(qb):
    return bool(np.isin(np.asarray(qb.rel_pred), (BETWEEN,)).any())


def oracle_bounds(scene, qb):
    """(s64, sem, t64, b64, s_lo, s_hi, t_lo, t_hi): the oracle's exact scores and
    terms, and their lowest / highest values over the rank orders that FP32
    distance comparisons may take and over Between's candidate sets that FP32
    similarities may select (equal to the exact ones without such predicates)."""
    import contextlib
    import oracle
    s64, sem, t64, b64 = oracle.score(scene, qb, terms=True)
    rank, btw = has_rank_preds(qb), has_between(qb)
    if not rank and not btw:
        return s64, sem, t64, b64, s64, s64, t64, t64
    out = []
    for mode in (-1, +1):
        with contextlib.ExitStack() as st:
            if rank:
                st.enter_context(oracle.rank_tolerance(mode, RANK_EPS))
            if btw:
                st.enter_context(oracle.between_tolerance(mode, BETWEEN_EPS))
            s_, _, t_, _ = oracle.score(scene, qb, terms=True)
        out.append((s_, t_))
    (s_lo, t_lo), (s_hi, t_hi) = out
    return s64, sem, t64, b64, s_lo, s_hi, t_lo, t_hi


def assert_topk_valid(gpu_ids, gpu_scores, oracle_ids, oracle_scores, lookup_score, k):
    """gpu_ids/gpu_scores: [k]; oracle_ids/oracle_scores: the oracle's exact ranking for at
    least k + 1 ranks (ids, FP64 scores); lookup_score(id) -> oracle FP64 score of any id."""
    oracle_ids = list(oracle_ids)
    oracle_scores = np.asarray(oracle_scores, np.float64)
    m = min(k, len([x for x in oracle_ids if x != 0xFFFFFFFF]))
    assert len(set(int(x) for x in gpu_ids[:m])) == m, "duplicate ids in the GPU TopK"
    for r in range(m):
        gid = int(gpu_ids[r])
        s64 = lookup_score(gid)
        # the returned score is the object's score (relative bound)
        if abs(float(gpu_scores[r]) - s64) > REL * max(abs(s64), TOPK_FLOOR):
            raise AssertionError(f"rank {r}: GPU score {gpu_scores[r]!r} vs oracle {s64!r} for id {gid}")
        # the object belongs at this rank up to near-ties
        want = oracle_scores[r]
        if abs(s64 - want) > GAP + REL * abs(want):
            raise AssertionError(f"rank {r}: GPU id {gid} has oracle score {s64!r}, rank score is {want!r}")
        above = oracle_scores[r - 1] - want if r > 0 else np.inf
        below = want - oracle_scores[r + 1] if r + 1 < len(oracle_scores) else np.inf
        if above > GAP and below > GAP:
            assert gid == int(oracle_ids[r]), f"rank {r}: id {gid} != oracle id {oracle_ids[r]} (isolated rank)"
    for r in range(m, k):
        assert int(gpu_ids[r]) == 0xFFFFFFFF and gpu_scores[r] == -np.inf, "padding expected beyond n"


def assert_topk_valid_bounds(gpu_ids, gpu_scores, ids, lo, hi, k):
    """TopK check where some scores are only known to lie in [lo, hi] (the rank
    predicates' open orders): every returned score lies in its object's
    interval, the list is ordered, and no object left out is certainly above
    the last returned score.  ids/lo/hi: every object of the memory."""
    n = len(ids)
    m = min(k, n)
    idx_of = {int(v): i for i, v in enumerate(ids)}
    got = [int(x) for x in gpu_ids[:m]]
    assert len(set(got)) == m, "duplicate ids in the GPU TopK"
    for r, gid in enumerate(got):
        i = idx_of[gid]
        s = float(gpu_scores[r])
        assert (lo[i] - REL * max(lo[i], TOPK_FLOOR) <= s <= hi[i] + REL * max(hi[i], TOPK_FLOOR)), \
            f"rank {r}: id {gid} score {s!r} not in [{lo[i]}, {hi[i]}]"
        if r:
            assert s <= float(gpu_scores[r - 1]), f"rank {r}: scores not descending"
    if m:
        last = float(gpu_scores[m - 1])
        chosen = np.zeros(n, bool)
        chosen[[idx_of[g] for g in got]] = True
        missed = np.flatnonzero(~chosen & (np.asarray(lo) > last * (1 + REL) + GAP))
        assert missed.size == 0, f"object {ids[missed[0]]} (lo {lo[missed[0]]}) left out above {last}"
    for r in range(m, k):
        assert int(gpu_ids[r]) == 0xFFFFFFFF and gpu_scores[r] == -np.inf, "padding expected beyond n"
