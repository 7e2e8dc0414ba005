"""Parity criteria between the GPU path and the FP64 oracle.

Tolerances (derived from the FP32 arithmetic of the GPU path):
  * score / relation-term values: |x_gpu - x_64| <= REL * |x_64| + ABS.
    REL = 1e-5 is the stated FP32 bar.  ABS covers the similarity GEMM: an
    FP32 dot product of two unit vectors of width d carries a rounding error of
    order sqrt(d) * 2^-24 in practice (the worst-case bound d * 2^-24 is far
    looser); 4e-6 is about twice the typical error at d = 1152 and dominates
    only for scores below 0.4.
  * TopK ids: exact wherever the oracle's score at that rank is separated
    from both neighbours by more than GAP = 1e-5; inside a near-tie group any
    order is correct, and the oracle score of each returned id must lie within
    GAP (plus value tolerance) of the oracle score at that rank.
"""
import numpy as np

REL = 1e-5
ABS = 4e-6
GAP = 1e-5


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
        # the returned score is the object's score
        if abs(float(gpu_scores[r]) - s64) > REL * abs(s64) + ABS:
            raise AssertionError(f"rank {r}: GPU score {gpu_scores[r]!r} vs oracle {s64!r} for id {gid}")
        # the object belongs at this rank up to near-ties
        want = oracle_scores[r]
        if abs(s64 - want) > GAP + REL * abs(want) + ABS:
            raise AssertionError(f"rank {r}: GPU id {gid} has oracle score {s64!r}, rank score is {want!r}")
        above = oracle_scores[r - 1] - want if r > 0 else np.inf
        below = want - oracle_scores[r + 1] if r + 1 < len(oracle_scores) else np.inf
        if above > GAP and below > GAP:
            assert gid == int(oracle_ids[r]), f"rank {r}: id {gid} != oracle id {oracle_ids[r]} (isolated rank)"
    for r in range(m, k):
        assert int(gpu_ids[r]) == 0xFFFFFFFF and gpu_scores[r] == -np.inf, "padding expected beyond n"
