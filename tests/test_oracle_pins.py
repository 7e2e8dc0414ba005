"""Pins for the FP64 oracle against facts the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed-form
predicate values, hand-built scenes with known winners and closed-form scores,
a brute-force joint-binding enumeration (pre-decomposition definition),
library routines for the special case R = 0, and invariants of the method
(bounds of the soft blend, duality/antisymmetry of predicates, permutation and
relation-order invariance).
"""
import math

import numpy as np
import pytest

import oracle
from oracle.brute import brute_scores
from synth import (ABOVE, ALL_PREDS, BEHIND, BELOW, CLOSEST, EVERY_PRED, FARTHEST, IN_FRONT_OF, INSIDE, LEFT_OF,
                   NEAR, NEXT_TO, ON, RIGHT_OF, CONFIGS,
                   QueryBatch, Scene, make_queries, make_scene)
from tests import _golden

LN3_TENTH = 0.1 * math.log(3.0)


# ---------------------------------------------------------------- predicates
def test_near_closed_form():
    r = [1.0, 0.0]
    assert oracle.predicate(NEAR, [0, 0, 0], [0, 0, 0], r) == 1.0
    # |D| = 0.5 m = sigma  ->  exp(-1/2)
    assert oracle.predicate(NEAR, [0, 0, 0], [0.5, 0, 0], r) == pytest.approx(math.exp(-0.5), rel=1e-15)
    assert oracle.predicate(NEAR, [1, 2, 3], [1, 2, 4], r) == pytest.approx(math.exp(-2.0), rel=1e-15)
    # symmetric
    a, b = [0.3, -1.2, 2.0], [1.1, 0.4, 1.5]
    assert oracle.predicate(NEAR, a, b, r) == oracle.predicate(NEAR, b, a, r)


def test_above_below_closed_form_and_duality():
    r = [1.0, 0.0]
    assert oracle.predicate(ABOVE, [0, 0, 0], [0, 0, 0], r) == 0.5
    # target 0.1 ln 3 above the anchor: sig(ln 3) = 3/4
    assert oracle.predicate(ABOVE, [0, 0, 0], [0, 0, -LN3_TENTH], r) == pytest.approx(0.75, abs=2e-8)
    assert oracle.predicate(BELOW, [0, 0, 0], [0, 0, -LN3_TENTH], r) == pytest.approx(0.25, abs=2e-8)
    rng = np.random.default_rng(3)
    for _ in range(50):
        a, b = rng.uniform(-3, 3, 3), rng.uniform(-3, 3, 3)
        up = oracle.predicate(ABOVE, a, b, r)
        dn = oracle.predicate(BELOW, a, b, r)
        assert up + dn == pytest.approx(1.0, abs=1e-15)
        assert dn == pytest.approx(oracle.predicate(ABOVE, b, a, r), abs=1e-15)
        # no horizontal gate: moving the anchor sideways changes nothing
        b2 = np.array(b, dtype=np.float32).copy()
        b2[:2] += np.float32(7.0)
        assert oracle.predicate(ABOVE, a, b2, r) == pytest.approx(up, abs=1e-6)


def test_left_right_antisymmetry_and_viewer():
    rng = np.random.default_rng(4)
    for _ in range(50):
        yaw = rng.uniform(0, 2 * math.pi)
        r = np.array([math.sin(yaw), -math.cos(yaw)], np.float32)
        a, b = rng.uniform(-5, 5, 3).astype(np.float32), rng.uniform(-5, 5, 3).astype(np.float32)
        lt = oracle.predicate(LEFT_OF, a, b, r)
        rt = oracle.predicate(RIGHT_OF, a, b, r)
        assert lt + rt == pytest.approx(1.0, abs=1e-15)
        assert lt == pytest.approx(oracle.predicate(RIGHT_OF, b, a, r), abs=1e-15)
        # turning the viewer around swaps left and right
        assert oracle.predicate(LEFT_OF, a, b, -r) == pytest.approx(rt, abs=1e-15)
        # height plays no part
        a2 = a.copy()
        a2[2] += 3.0
        assert oracle.predicate(RIGHT_OF, a2, b, r) == pytest.approx(rt, abs=1e-15)
    # closed form: target 0.1 ln 3 along the right vector
    r = np.array([0.0, -1.0], np.float32)
    assert oracle.predicate(RIGHT_OF, [0, -LN3_TENTH, 0], [0, 0, 0], r) == pytest.approx(0.75, abs=2e-8)


def test_left_right_translation_invariant():
    rng = np.random.default_rng(5)
    r = np.array([0.6, 0.8], np.float32)
    for _ in range(20):
        a, b = rng.uniform(-2, 2, 3), rng.uniform(-2, 2, 3)
        sh = rng.uniform(-2, 2, 3)
        v0 = oracle.predicate(RIGHT_OF, a, b, r)
        v1 = oracle.predicate(RIGHT_OF, np.float64(a) + sh, np.float64(b) + sh, r)
        assert v1 == pytest.approx(v0, abs=1e-6)


def test_next_to_closed_form_and_scale():
    r = [1.0, 0.0]
    assert oracle.predicate(NEXT_TO, [0, 0, 0], [0, 0, 0], r) == 1.0
    # |D| = 1 m = sigma  ->  exp(-1/2); |D| = 2 m -> exp(-2)
    assert oracle.predicate(NEXT_TO, [0, 0, 0], [1.0, 0, 0], r) == pytest.approx(math.exp(-0.5), rel=1e-15)
    assert oracle.predicate(NEXT_TO, [1, 2, 3], [1, 4, 3], r) == pytest.approx(math.exp(-2.0), rel=1e-15)
    # a Gaussian twice as wide as Near: NextTo(a, b) = Near(a/2, b/2) (halving is exact in FP32)
    rng = np.random.default_rng(6)
    for _ in range(30):
        a, b = rng.uniform(-3, 3, 3).astype(np.float32), rng.uniform(-3, 3, 3).astype(np.float32)
        assert oracle.predicate(NEXT_TO, a, b, r) == pytest.approx(oracle.predicate(NEAR, a / 2, b / 2, r),
                                                                    rel=1e-14)
        assert oracle.predicate(NEXT_TO, a, b, r) >= oracle.predicate(NEAR, a, b, r)


def test_front_behind_duality_and_viewer():
    rng = np.random.default_rng(7)
    for _ in range(50):
        yaw = rng.uniform(0, 2 * math.pi)
        r = np.array([math.sin(yaw), -math.cos(yaw)], np.float32)
        a, b = rng.uniform(-5, 5, 3).astype(np.float32), rng.uniform(-5, 5, 3).astype(np.float32)
        fr = oracle.predicate(IN_FRONT_OF, a, b, r)
        bh = oracle.predicate(BEHIND, a, b, r)
        assert fr + bh == pytest.approx(1.0, abs=1e-15)
        assert fr == pytest.approx(oracle.predicate(BEHIND, b, a, r), abs=1e-15)
        # the viewing direction is the right axis turned a quarter turn counter-clockwise:
        # depth relations are side relations of a viewer turned to face the old right
        r_turned = np.array([-r[1], r[0]], np.float32)
        assert fr == pytest.approx(oracle.predicate(LEFT_OF, a, b, r_turned), abs=1e-15)
        assert bh == pytest.approx(oracle.predicate(RIGHT_OF, a, b, r_turned), abs=1e-15)
        # height plays no part
        a2 = a.copy()
        a2[2] += 3.0
        assert oracle.predicate(BEHIND, a2, b, r) == pytest.approx(bh, abs=1e-15)
    # closed form: viewer right (0, -1) looks along +x; a target 0.1 ln 3 nearer than the anchor
    r = np.array([0.0, -1.0], np.float32)
    assert oracle.predicate(IN_FRONT_OF, [-LN3_TENTH, 0, 0], [0, 0, 0], r) == pytest.approx(0.75, abs=2e-8)
    assert oracle.predicate(BEHIND, [-LN3_TENTH, 0, 0], [0, 0, 0], r) == pytest.approx(0.25, abs=2e-8)



def test_on_closed_form_gate_and_band():
    """On: a gate on the horizontal center distance (sigma 0.5 m) times a band
    on the gap between the target's bottom face and the anchor's top face
    (sigma 0.125 m).  Inputs are exact in FP32, so the values are exact."""
    r = [1.0, 0.0]
    cup, table = [0.3, 0.3, 0.5], [2.0, 2.0, 1.0]   # full extents
    # a cup resting centred on a table: bottom 1.25 - 0.25 = 1.0 = top 0.5 + 0.5
    assert oracle.predicate(ON, [0, 0, 1.25], [0, 0, 0.5], r, cup, table) == 1.0
    # 0.5 m off centre: exp(-0.25 / (2 * 0.25))
    assert oracle.predicate(ON, [0.5, 0, 1.25], [0, 0, 0.5], r, cup, table) == pytest.approx(
        math.exp(-0.5), rel=1e-15)
    # hovering 0.25 m above or sunk 0.25 m into the table: exp(-0.0625 / (2 * 0.015625))
    for zc in (1.5, 1.0):
        assert oracle.predicate(ON, [0, 0, zc], [0, 0, 0.5], r, cup, table) == pytest.approx(
            math.exp(-2.0), rel=1e-14)
    # both at once multiply
    assert oracle.predicate(ON, [0, 0.5, 1.5], [0, 0, 0.5], r, cup, table) == pytest.approx(
        math.exp(-2.5), rel=1e-14)
    # roles swapped (the table "on" the cup): the table's bottom 0 is 1.5 m below the cup's top
    assert oracle.predicate(ON, [0, 0, 0.5], [0, 0, 1.25], r, table, cup) == pytest.approx(
        math.exp(-72.0), rel=1e-12)
    # a taller cup raises its own center, not the contact: same value when the center moves with it
    assert oracle.predicate(ON, [0, 0, 1.5], [0, 0, 0.5], r, [0.3, 0.3, 1.0], table) == 1.0
    rng = np.random.default_rng(8)
    for _ in range(40):
        a, b = rng.uniform(-3, 3, 3).astype(np.float32), rng.uniform(-3, 3, 3).astype(np.float32)
        ea, eb = rng.uniform(0.1, 2, 3).astype(np.float32), rng.uniform(0.1, 2, 3).astype(np.float32)
        v = oracle.predicate(ON, a, b, r, ea, eb)
        assert 0.0 <= v <= 1.0
        # neither the viewer nor the horizontal extents play a part
        yaw = rng.uniform(0, 2 * math.pi)
        r2 = np.array([math.sin(yaw), -math.cos(yaw)], np.float32)
        ea2, eb2 = ea.copy(), eb.copy()
        ea2[:2] *= 3
        eb2[:2] /= 2
        assert oracle.predicate(ON, a, b, r2, ea2, eb2) == v
        # gate: the horizontal part is Near's Gaussian (same width) on the pair flattened to the ground
        fa, fb = np.array([a[0], a[1], 0], np.float32), np.array([b[0], b[1], 0], np.float32)
        gate = oracle.predicate(NEAR, fa, fb, r)
        # band: with the horizontal offset removed only the band remains
        band = oracle.predicate(ON, np.array([b[0], b[1], a[2]], np.float32), b, r, ea, eb)
        assert v == pytest.approx(gate * band, rel=1e-14, abs=1e-300)



def test_inside_closed_form():
    """Inside: along each axis a logistic (0.1 m) of the margin between the
    anchor's half extent and the target's center offset; the product of the
    three.  Values on exact inputs."""
    r = [1.0, 0.0]
    box = [2.0, 4.0, 1.0]  # half extents 1, 2, 0.5
    sig = lambda u: 1.0 / (1.0 + math.exp(-u))
    # centred: margins 1, 2, 0.5 m -> sig(10) sig(20) sig(5)
    assert oracle.predicate(INSIDE, [0, 0, 0], [0, 0, 0], r, [0.1, 0.1, 0.1], box) == pytest.approx(
        sig(10) * sig(20) * sig(5), rel=1e-15)
    # on the x face: sig(0) = 1/2 for that axis
    assert oracle.predicate(INSIDE, [1, 0, 0], [0, 0, 0], r, [0.1, 0.1, 0.1], box) == pytest.approx(
        0.5 * sig(20) * sig(5), rel=1e-15)
    # 0.25 m outside in z (offset 0.75 against half extent 0.5), either side
    for dz in (0.75, -0.75):
        assert oracle.predicate(INSIDE, [0, 0, dz], [0, 0, 0], r, [0.1, 0.1, 0.1], box) == pytest.approx(
            sig(10) * sig(20) * sig(-2.5), rel=1e-14)
    rng = np.random.default_rng(9)
    for _ in range(30):
        a, b = rng.uniform(-3, 3, 3).astype(np.float32), rng.uniform(-3, 3, 3).astype(np.float32)
        ea, eb = rng.uniform(0.1, 4, 3).astype(np.float32), rng.uniform(0.1, 4, 3).astype(np.float32)
        v = oracle.predicate(INSIDE, a, b, r, ea, eb)
        assert 0.0 < v < 1.0
        # the target's own extent and the viewer play no part
        yaw = rng.uniform(0, 2 * math.pi)
        r2 = np.array([math.sin(yaw), -math.cos(yaw)], np.float32)
        assert oracle.predicate(INSIDE, a, b, r2, ea * 2, eb) == v
        # mirrored offsets give the same value
        assert oracle.predicate(INSIDE, 2 * b - a, b, r, ea, eb) == pytest.approx(v, rel=1e-5)
        # a larger anchor box contains more
        assert oracle.predicate(INSIDE, a, b, r, ea, eb * 2) > v


def _rank_scene():
    """Three chairs (class 1) on the x axis at 1, 2 and 3 m from a package
    (class 2) at the origin, a lamp (class 3) at 1.5 m, a fourth chair at
    -2 m (as far from the package as the second chair, with a larger id)."""
    d = 4
    e = np.eye(d, dtype=np.float32)
    desc = np.stack([e[0], e[0], e[0], e[1], e[2], e[0]])
    center = np.array([[1, 0, 0], [2, 0, 0], [3, 0, 0], [0, 0, 0], [1.5, 0, 0], [-2, 0, 0]], np.float32)
    scene = Scene(desc=desc, center=center, extent=np.full((6, 3), 0.5, np.float32),
                  ids=np.array([10, 20, 30, 40, 50, 60], np.uint32), cls=np.array([1, 1, 1, 2, 3, 1], np.int32),
                  view_right=np.array([1, 0], np.float32), centroids=np.zeros((1, d), np.float32))
    return scene, e


def _one_query(e, pred, tcls):
    return QueryBatch(target=e[0][None], target_cls=np.array([tcls], np.int32), rel_off=np.array([0, 1], np.int32),
                      rel_pred=np.array([pred], np.int32), rel_anchor=e[1][None], planted=np.zeros(1, np.int64))


def test_closest_farthest_hand_scene():
    """Closest / Farthest: 1 / (|rank - r*| + 1), the rank of the target among
    the query's candidates (its class) by distance to the anchor; only the
    package matches the anchor description, so t = P(chair, package)."""
    scene, e = _rank_scene()
    _, _, t, b = oracle.score(scene, _one_query(e, CLOSEST, 1), terms=True)
    # chairs at 1, 2, 3 m and -2 m (same distance as 2 m, larger id: after it)
    np.testing.assert_allclose(t[0, [0, 1, 2, 5]], [1.0, 1 / 2, 1 / 4, 1 / 3], rtol=0, atol=0)
    assert set(b[0, [0, 1, 2, 5]]) == {40}
    # Farthest: r* is the last rank among the other chairs (3 of them): 4
    _, _, t, b = oracle.score(scene, _one_query(e, FARTHEST, 1), terms=True)
    np.testing.assert_allclose(t[0, [0, 1, 2, 5]], [1 / 4, 1 / 3, 1.0, 1 / 2], rtol=0, atol=0)
    # without a class every object is a candidate: the lamp (1.5 m) now precedes the 2 m chair
    _, _, t, _ = oracle.score(scene, _one_query(e, CLOSEST, -1), terms=True)
    np.testing.assert_allclose(t[0, [0, 1, 2, 5]], [1.0, 1 / 3, 1 / 5, 1 / 4], rtol=0, atol=0)
    # the composite: s = s_sem (1/2 + t/2) with s_sem = 1 for every chair
    s = oracle.score(scene, _one_query(e, CLOSEST, 1))
    np.testing.assert_allclose(s[0, [0, 1, 2, 5]], [1.0, 0.75, 0.625, 2 / 3], rtol=1e-15)


def test_rank_values_are_a_permutation():
    """For one anchor, the Closest values over the candidates are 1, 1/2, ...,
    1/|C| each once, and Farthest takes them in reverse order of distance."""
    cfg = CONFIGS["mid"]
    scene = make_scene(cfg, n=150, seed=41)
    rng = np.random.default_rng(42)
    for _ in range(6):
        tc = int(scene.cls[rng.integers(0, scene.n)])
        cand = np.flatnonzero(scene.cls == tc)
        j = int(rng.integers(0, scene.n))
        members = [int(c) for c in cand if c != j]
        anchor = scene.desc[j]
        vals_c, vals_f, dist = [], [], []
        u = anchor.astype(np.float64) / np.linalg.norm(anchor.astype(np.float64))
        a = float(u @ u)  # the anchor's own similarity (1 up to rounding)
        for i in members:
            vals_c.append(oracle.binding_value(scene, CLOSEST, anchor, i, j, tc) / a)
            vals_f.append(oracle.binding_value(scene, FARTHEST, anchor, i, j, tc) / a)
            dist.append(float(np.sum((scene.center[i].astype(np.float64) - scene.center[j]) ** 2)))
        m = len(members)
        np.testing.assert_allclose(sorted(vals_c, reverse=True), [1 / (k + 1) for k in range(m)], rtol=1e-12)
        order = np.argsort(dist, kind="stable")
        np.testing.assert_allclose(np.asarray(vals_c)[order], [1 / (k + 1) for k in range(m)], rtol=1e-12)
        np.testing.assert_allclose(np.asarray(vals_f)[order], [1 / (m - k) for k in range(m)], rtol=1e-12)


def _exact_rank_value(scene, pred, tcls, i, j):
    """1 / (|rank - r*| + 1) with squared distances in exact rational arithmetic
    from the float32 centers (a check independent of floating point)."""
    from fractions import Fraction
    c = [[Fraction(float(v)) for v in row] for row in scene.center]
    d2 = lambda a, b: sum((c[a][k] - c[b][k]) ** 2 for k in range(3))
    dij = d2(i, j)
    nearer = m = 0
    for k in range(scene.n):
        if k in (i, j) or (tcls >= 0 and int(scene.cls[k]) != tcls):
            continue
        m += 1
        dk = d2(k, j)
        nearer += dk < dij or (dk == dij and int(scene.ids[k]) < int(scene.ids[i]))
    rstar = 1 if pred == CLOSEST else m + 1
    return 1.0 / (abs(nearer + 1 - rstar) + 1)


def _near_tie_scene():
    """An anchor at the origin; chair A at x = 1 m and chair B at
    (1 - 2^-24, y) with y the float just above sqrt(2^-23 - 2^-48): exactly,
    |B|^2 = 1 + a few 2^-49 > 1 = |A|^2, but the float32 sum of squares of B
    rounds to exactly 1 (a tie that the smaller id of B would win)."""
    y = np.nextafter(np.float32(math.sqrt(2.0 ** -23 - 2.0 ** -48)), np.float32(1))
    center = np.array([[0, 0, 0], [1, 0, 0], [1 - 2.0 ** -24, y, 0], [3, 0, 0]], np.float32)
    d = 4
    e = np.eye(d, dtype=np.float32)
    scene = Scene(desc=np.stack([e[1], e[0], e[0], e[0]]), center=center, extent=np.full((4, 3), 0.5, np.float32),
                  ids=np.array([7, 20, 10, 30], np.uint32), cls=np.array([2, 1, 1, 1], np.int32),
                  view_right=np.array([1, 0], np.float32), centroids=np.zeros((1, d), np.float32))
    return scene, e


def test_rank_near_tie_is_exact():
    """The rank follows the exact distances even where float32 sums of squares
    tie; the tolerance mode opens exactly that pair."""
    from fractions import Fraction
    scene, e = _near_tie_scene()
    xa, xb, yb = (Fraction(float(v)) for v in (scene.center[1, 0], scene.center[2, 0], scene.center[2, 1]))
    assert xb * xb + yb * yb > xa * xa  # B is farther, exactly
    c32 = scene.center.astype(np.float32)
    f32 = lambda v: np.float32(v[0]) * np.float32(v[0]) + np.float32(v[1]) * np.float32(v[1])
    assert f32(c32[2]) == f32(c32[1]) == np.float32(1)  # ... but float32 sums tie
    anchor = e[1]
    # Closest among the chairs by distance to the anchor (index 0): A first, B second
    assert oracle.binding_value(scene, CLOSEST, anchor, 1, 0, 1) == 1.0
    assert oracle.binding_value(scene, CLOSEST, anchor, 2, 0, 1) == 0.5
    assert oracle.binding_value(scene, FARTHEST, anchor, 2, 0, 1) == 0.5
    # tolerance mode: A and B may take either order, the far chair may not
    for i, hi, lo in ((1, 1.0, 0.5), (2, 1.0, 0.5)):
        with oracle.rank_tolerance(+1, 1e-6):
            assert oracle.binding_value(scene, CLOSEST, anchor, i, 0, 1) == hi
        with oracle.rank_tolerance(-1, 1e-6):
            assert oracle.binding_value(scene, CLOSEST, anchor, i, 0, 1) == lo
    with oracle.rank_tolerance(-1, 1e-6):
        assert oracle.binding_value(scene, CLOSEST, anchor, 3, 0, 1) == 1 / 3
    # outside the context manager the exact rank is back
    assert oracle.binding_value(scene, CLOSEST, anchor, 2, 0, 1) == 0.5


def test_rank_matches_rational_arithmetic():
    """Closest/Farthest values of random bindings (objects on a coarse grid, so
    that exact distance ties occur and are ordered by id) equal the rank taken
    with exact rational squared distances."""
    rng = np.random.default_rng(51)
    n, d = 40, 6
    scene = Scene(desc=rng.standard_normal((n, d)).astype(np.float32),
                  center=(rng.integers(0, 5, (n, 3)) * 0.5).astype(np.float32),
                  extent=np.full((n, 3), 0.3, np.float32), ids=(rng.permutation(3 * n)[:n] + 1).astype(np.uint32),
                  cls=rng.integers(0, 3, n).astype(np.int32), view_right=np.array([0, -1], np.float32),
                  centroids=np.zeros((1, d), np.float32))
    ties = 0
    for _ in range(60):
        i, j = (int(x) for x in rng.choice(n, 2, replace=False))
        tcls = int(rng.integers(-1, 3))
        anchor = scene.desc[j]
        for pred in (CLOSEST, FARTHEST):  # the anchor's own descriptor: sim(j, q_r) = 1
            got = oracle.binding_value(scene, pred, anchor, i, j, tcls)
            assert got == pytest.approx(_exact_rank_value(scene, pred, tcls, i, j), rel=1e-12)
        dij = np.sum((scene.center[i] - scene.center[j]).astype(np.float64) ** 2)
        ties += int(np.sum(np.sum((scene.center - scene.center[j]).astype(np.float64) ** 2, axis=1) == dij) > 2)
    assert ties > 0  # the grid produced exact distance ties


# ---------------------------------------------------------------- hand scenes
@pytest.mark.parametrize("path", _golden.all_paths(), ids=lambda p: p.rsplit("/", 1)[-1])
def test_golden_scenes(path):
    g, scene, queries = _golden.load(path)
    for qb, spec in queries:
        s, sem, t, b = oracle.score(scene, qb, terms=True)
        order = oracle.topk(s[0], scene.ids, scene.n)
        assert [int(scene.ids[i]) for i in order] == spec["expect_order"]
        for sid, expr in spec["expect_score"].items():
            i = int(np.flatnonzero(scene.ids == int(sid))[0])
            assert s[0, i] == pytest.approx(_golden.evaluate(expr), abs=1e-6), sid
        for sid, anchors in spec.get("expect_anchor", {}).items():
            i = int(np.flatnonzero(scene.ids == int(sid))[0])
            assert [int(x) for x in b[:, i]] == anchors, sid


@pytest.mark.parametrize("path", _golden.all_paths(), ids=lambda p: p.rsplit("/", 1)[-1])
def test_golden_scenes_brute_force(path):
    """The independent joint-binding enumeration reaches the same closed forms."""
    g, scene, queries = _golden.load(path)
    for qb, spec in queries:
        bs = brute_scores(scene, qb)[0]
        for sid, expr in spec["expect_score"].items():
            i = int(np.flatnonzero(scene.ids == int(sid))[0])
            assert bs[i] == pytest.approx(_golden.evaluate(expr), abs=1e-6), sid


# ---------------------------------------------------------------- brute force
def _tiny(seed, n, r, q=3, d=6, n_cat=3, npred=5):
    cfg = CONFIGS["tiny"]
    rng = np.random.default_rng(seed)
    cent = rng.standard_normal((n_cat, d))
    cent /= np.linalg.norm(cent, axis=1, keepdims=True)
    cls = rng.integers(0, n_cat, n).astype(np.int32)
    desc = cent[cls] + 0.4 * rng.standard_normal((n, d))
    # extents from a stream of their own (the other draws keep their values); they
    # matter to On only
    ext = np.random.default_rng(seed + 1000).uniform(0.2, 1.5, (n, 3)).astype(np.float32)
    scene = Scene(desc=desc.astype(np.float32), center=rng.uniform(0, 2, (n, 3)).astype(np.float32),
                  extent=ext, ids=rng.permutation(100)[:n].astype(np.uint32) + 1,
                  cls=cls, view_right=np.array([math.cos(seed), math.sin(seed)], np.float32),
                  centroids=cent.astype(np.float32))
    offs = [0]
    preds = []
    for _ in range(q):
        for _ in range(r):
            preds.append(int(rng.integers(0, npred)))
        offs.append(len(preds))
    qb = QueryBatch(target=rng.standard_normal((q, d)).astype(np.float32),
                    target_cls=rng.integers(-1, n_cat, q).astype(np.int32),
                    rel_off=np.asarray(offs, np.int32), rel_pred=np.asarray(preds, np.int32),
                    rel_anchor=rng.standard_normal((len(preds), d)).astype(np.float32),
                    planted=np.zeros(q, np.int64))
    return scene, qb


@pytest.mark.parametrize("n,r", [(1, 1), (2, 1), (2, 2), (5, 0), (5, 1), (6, 2), (7, 3), (9, 2)])
def test_star_decomposition_equals_joint_enumeration(n, r):
    for seed in range(3):
        scene, qb = _tiny(seed * 31 + n * 7 + r, n, r)
        s = oracle.score(scene, qb)
        bs = np.asarray(brute_scores(scene, qb))
        np.testing.assert_allclose(s, bs, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("n,r", [(2, 1), (5, 2), (7, 3)])
def test_star_decomposition_all_predicates(n, r):
    for seed in range(3):
        scene, qb = _tiny(seed * 17 + n * 5 + r, n, r, npred=len(EVERY_PRED))
        s = oracle.score(scene, qb)
        bs = np.asarray(brute_scores(scene, qb))
        np.testing.assert_allclose(s, bs, rtol=1e-12, atol=1e-14)


# ---------------------------------------------------------------- invariants
@pytest.fixture(scope="module")
def small_world():
    cfg = CONFIGS["mid"]
    scene = make_scene(cfg, n=120, seed=11)
    qb = make_queries(cfg, scene, seed=12, q=12, r_min=0, r_max=4)
    s, sem, t, b = oracle.score(scene, qb, terms=True)
    return scene, qb, s, sem, t, b


def test_r0_equals_class_weighted_clamped_cosine(small_world):
    scene, qb, s, sem, t, b = small_world
    u = scene.desc.astype(np.float64)
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    for k in range(qb.q):
        v = qb.target[k].astype(np.float64)
        v /= np.linalg.norm(v)
        cos = np.maximum(u @ v, 0.0)
        kappa = np.where((qb.target_cls[k] >= 0) & (scene.cls != qb.target_cls[k]), 0.3, 1.0)
        np.testing.assert_allclose(sem[k], kappa * cos, rtol=1e-12, atol=1e-15)
        if qb.rel_off[k + 1] == qb.rel_off[k]:
            np.testing.assert_allclose(s[k], sem[k], rtol=0, atol=0)


def test_soft_blend_bounds(small_world):
    """The spatial factor stays in [1 - w, 1] ('Why soft, not hard?')."""
    scene, qb, s, sem, t, b = small_world
    assert np.all(s <= sem * (1 + 1e-15))
    assert np.all(s >= 0.5 * sem * (1 - 1e-15))
    assert np.all((t >= 0) & (t <= 1))


def test_relation_terms_compose(small_world):
    scene, qb, s, sem, t, b = small_world
    for k in range(qb.q):
        a0, a1 = qb.rel_off[k], qb.rel_off[k + 1]
        if a1 == a0:
            continue
        g = np.exp(np.mean(np.log(np.maximum(t[a0:a1], 1e-300)), axis=0))
        g = np.where(np.any(t[a0:a1] == 0, axis=0), 0.0, g)
        np.testing.assert_allclose(s[k], sem[k] * (0.5 + 0.5 * g), rtol=1e-12, atol=1e-300)


def test_bound_anchor_attains_term(small_world):
    scene, qb, s, sem, t, b = small_world
    u = scene.desc.astype(np.float64)
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    id2idx = {int(x): i for i, x in enumerate(scene.ids)}
    for rr in range(qb.r_tot):
        v = qb.rel_anchor[rr].astype(np.float64)
        v /= np.linalg.norm(v)
        a = np.maximum(u @ v, 0.0)
        for i in range(0, scene.n, 17):
            j = id2idx[int(b[rr, i])]
            assert j != i
            val = a[j] * oracle.predicate(int(qb.rel_pred[rr]), scene.center[i], scene.center[j], scene.view_right)
            assert val == pytest.approx(t[rr, i], rel=1e-12, abs=1e-300)


def test_object_permutation_invariance(small_world):
    scene, qb, s, sem, t, b = small_world
    perm = np.random.default_rng(0).permutation(scene.n)
    sp = Scene(desc=scene.desc[perm], center=scene.center[perm], extent=scene.extent[perm],
               ids=scene.ids[perm], cls=scene.cls[perm], view_right=scene.view_right, centroids=scene.centroids)
    s2 = oracle.score(sp, qb)
    np.testing.assert_allclose(s2, s[:, perm], rtol=1e-12, atol=1e-300)
    for k in range(qb.q):
        o1 = scene.ids[oracle.topk(s[k], scene.ids, 10)]
        o2 = sp.ids[oracle.topk(s2[k], sp.ids, 10)]
        assert list(o1) == list(o2)


def test_relation_order_invariance(small_world):
    scene, qb, s, sem, t, b = small_world
    rng = np.random.default_rng(1)
    preds, anchors = [], []
    for k in range(qb.q):
        a0, a1 = qb.rel_off[k], qb.rel_off[k + 1]
        p = rng.permutation(a1 - a0) + a0
        preds.append(qb.rel_pred[p])
        anchors.append(qb.rel_anchor[p])
    qb2 = QueryBatch(target=qb.target, target_cls=qb.target_cls, rel_off=qb.rel_off,
                     rel_pred=np.concatenate(preds).astype(np.int32),
                     rel_anchor=np.concatenate(anchors).astype(np.float32), planted=qb.planted)
    np.testing.assert_allclose(oracle.score(scene, qb2), s, rtol=1e-12, atol=1e-300)


def test_no_class_gives_pure_cosine(small_world):
    scene, qb, s, sem, t, b = small_world
    qb2 = QueryBatch(target=qb.target, target_cls=np.full(qb.q, -1, np.int32), rel_off=qb.rel_off,
                     rel_pred=qb.rel_pred, rel_anchor=qb.rel_anchor, planted=qb.planted)
    _, sem2, _, _ = oracle.score(scene, qb2, terms=True)
    assert np.all(sem2 >= sem - 1e-15)
    mism = (qb.target_cls[:, None] != scene.cls[None, :])
    np.testing.assert_allclose(sem[mism], 0.3 * sem2[mism], rtol=1e-12, atol=1e-300)


# ---------------------------------------------------------------- TopK
def test_topk_matches_lexsort():
    rng = np.random.default_rng(9)
    for n in (1, 5, 37, 300):
        ids = (rng.permutation(10 * n)[:n] + 1).astype(np.uint32)
        sc = np.round(rng.uniform(0, 1, n), 2)  # many exact ties
        for k in (1, 3, 10, n + 4):
            got = oracle.topk(sc, ids, k)
            want = np.lexsort((ids, -sc))[:k]
            assert list(got[: min(k, n)]) == list(want)
            assert np.all(got[min(k, n):] == -1)


def test_bounded_topk_equals_full_topk(small_world):
    scene, qb, s, sem, t, b = small_world
    idx, sc, tt, bb, ns = oracle.topk_bounded(scene, qb, 10)
    for k in range(qb.q):
        want = oracle.topk(s[k], scene.ids, 10)
        assert list(idx[k]) == list(want)
        np.testing.assert_allclose(sc[k], s[k, want], rtol=1e-15)
        assert ns[k] <= scene.n
    # pairs entry point agrees with the full scores
    qsel = np.repeat(np.arange(qb.q), 5).astype(np.int32)
    osel = np.tile(np.arange(0, scene.n, scene.n // 5)[:5], qb.q).astype(np.int64)
    ps, psem, pt, pb = oracle.score_pairs(scene, qb, qsel, osel)
    np.testing.assert_allclose(ps, s[qsel, osel], rtol=1e-15)


# ---------------------------------------------------------------- Between (ternary)
BETWEEN, AND = 12, 13


def test_between_closed_forms():
    """Between(i; j1, j2) = sig(s/0.1) sig((L-s)/0.1) exp(-h^2/(2*0.5^2)): the
    midpoint, an endpoint, a perpendicular offset, beyond an anchor,
    coincident anchors; symmetric in the anchors, invariant to rigid motions."""
    sig = lambda u: 1 / (1 + math.exp(-u))
    a1, a2 = np.array([0, 0, 0], np.float32), np.array([2, 0, 0], np.float32)
    assert oracle.between([1, 0, 0], a1, a2) == pytest.approx(sig(10) ** 2, rel=1e-14)
    assert oracle.between([0, 0, 0], a1, a2) == pytest.approx(0.5 * sig(20), rel=1e-14)
    assert oracle.between([1, 0.5, 0], a1, a2) == pytest.approx(sig(10) ** 2 * math.exp(-0.5), rel=1e-14)
    assert oracle.between([2.5, 0, 0], a1, a2) == pytest.approx(sig(25) * sig(-5), rel=1e-14)
    assert oracle.between([1, 0, 0], a1, a1) == 0.0
    rng = np.random.default_rng(3)
    for _ in range(20):
        ci, c1, c2 = (rng.uniform(-3, 3, 3).astype(np.float32) for _ in range(3))
        v = oracle.between(ci, c1, c2)
        assert 0.0 <= v <= 1.0
        assert oracle.between(ci, c2, c1) == pytest.approx(v, rel=1e-12, abs=1e-300)
        # a rotation about z by 90 degrees and a translation
        rot = lambda c: np.array([-c[1], c[0], c[2]], np.float64) + np.array([5.0, -2.0, 1.0])
        assert oracle.between(rot(ci), rot(c1), rot(c2)) == pytest.approx(v, rel=1e-5, abs=1e-12)


def _between_scene():
    """A target at the origin, chairs A (id 5) at x = -1 m and B (id 3) at
    x = +1 m, a third chair C (id 9) off the axis; the anchor descriptions both
    match every chair equally."""
    d = 4
    e = np.eye(d, dtype=np.float32)
    center = np.array([[0, 0, 0], [-1, 0, 0], [1, 0, 0], [0, 3, 0]], np.float32)
    scene = Scene(desc=np.stack([e[0], e[1], e[1], e[1]]), center=center, extent=np.full((4, 3), 0.5, np.float32),
                  ids=np.array([1, 5, 3, 9], np.uint32), cls=np.array([0, 1, 1, 1], np.int32),
                  view_right=np.array([1, 0], np.float32), centroids=np.zeros((1, d), np.float32))
    qb = QueryBatch(target=e[0][None], target_cls=np.array([-1], np.int32), rel_off=np.array([0, 2], np.int32),
                    rel_pred=np.array([BETWEEN, AND], np.int32), rel_anchor=np.stack([e[1], e[1]]),
                    planted=np.zeros(1, np.int64))
    return scene, qb


def test_between_term_binding_and_ties():
    """The target between A and B: t = Between(o; A, B) with sim = 1 for both;
    (A, B) and (B, A) tie, so the binding is the smaller id pair (3, 5); both
    slots report the term, and it counts once in the geometric mean."""
    scene, qb = _between_scene()
    s, sem, t, b = oracle.score(scene, qb, terms=True)
    sig = lambda u: 1 / (1 + math.exp(-u))
    want = sig(10) ** 2
    assert t[0, 0] == pytest.approx(want, rel=1e-14) and t[1, 0] == t[0, 0]
    assert (int(b[0, 0]), int(b[1, 0])) == (3, 5)
    assert s[0, 0] == pytest.approx(1.0 * (0.5 + 0.5 * want), rel=1e-14)  # one invocation, not two
    # no pair of distinct anchors other than the target in a two-object memory
    two = Scene(desc=scene.desc[:2], center=scene.center[:2], extent=scene.extent[:2], ids=scene.ids[:2],
                cls=scene.cls[:2], view_right=scene.view_right, centroids=scene.centroids)
    s2, _, t2, b2 = oracle.score(two, qb, terms=True)
    assert np.all(t2 == 0) and np.all(b2 == 0xFFFFFFFF)


def test_between_must_pair_with_its_second_anchor():
    scene, qb = _between_scene()
    for preds in ([BETWEEN, 0], [AND, BETWEEN], [0, AND]):
        bad = QueryBatch(target=qb.target, target_cls=qb.target_cls, rel_off=qb.rel_off,
                         rel_pred=np.array(preds, np.int32), rel_anchor=qb.rel_anchor, planted=qb.planted)
        with pytest.raises(ValueError):
            oracle.score(scene, bad)


def _with_between(scene, qb, rng):
    """Each query gets one Between invocation (two slots) after its relations."""
    offs, preds, anchors = [0], [], []
    d = scene.desc.shape[1]
    for k in range(qb.target.shape[0]):
        a, b = int(qb.rel_off[k]), int(qb.rel_off[k + 1])
        preds += list(qb.rel_pred[a:b]) + [BETWEEN, AND]
        anchors += list(qb.rel_anchor[a:b]) + [rng.standard_normal(d).astype(np.float32) for _ in range(2)]
        offs.append(len(preds))
    return QueryBatch(target=qb.target, target_cls=qb.target_cls, rel_off=np.asarray(offs, np.int32),
                      rel_pred=np.asarray(preds, np.int32), rel_anchor=np.asarray(anchors, np.float32),
                      planted=qb.planted)


@pytest.mark.parametrize("n,r", [(2, 0), (3, 0), (4, 1), (6, 1), (7, 0)])
def test_between_star_decomposition_equals_joint_enumeration(n, r):
    """Bucket elimination of the Between factor (its two anchor variables
    maximised together, per target) equals the joint enumeration of every
    anchor variable."""
    for seed in range(3):
        scene, qb = _tiny(seed * 13 + n * 3 + r, n, r, npred=len(EVERY_PRED))
        qb = _with_between(scene, qb, np.random.default_rng(seed))
        s = oracle.score(scene, qb)
        bs = np.asarray(brute_scores(scene, qb))
        np.testing.assert_allclose(s, bs, rtol=1e-12, atol=1e-14)


def test_between_candidate_sets_of_64():
    """With more than 64 objects, Between's anchors range over the 64 of
    largest similarity per description: the oracle equals the joint
    enumeration over those sets (oracle/brute.py), and on this scene the
    restriction changes some terms (a better pair uses an anchor ranked below
    64).  The tie-aware modes bracket the exact term."""
    rng = np.random.default_rng(77)
    n, d = 150, 3
    desc = rng.standard_normal((n, d)).astype(np.float32)
    anchors = rng.standard_normal((4, d)).astype(np.float32)
    center = rng.uniform(0, 4, (n, 3)).astype(np.float32)
    # a target of query 0 sits between two anchors ranked just below 64 in similarity,
    # far from every other object: only the unrestricted maximum finds that pair
    un = desc.astype(np.float64) / np.linalg.norm(desc.astype(np.float64), axis=1, keepdims=True)
    ranked = [np.argsort(-(un @ (v / np.linalg.norm(v)))) for v in anchors[:2].astype(np.float64)]
    j1 = int(ranked[0][66])
    j2 = next(int(j) for j in ranked[1][66:] if int(j) != j1)
    o = next(i for i in range(n) if i not in (j1, j2))
    center[o] = (50, 50, 50)
    center[j1] = (49, 50, 50)
    center[j2] = (51, 50, 50)
    scene = Scene(desc=desc, center=center,
                  extent=np.full((n, 3), 0.3, np.float32), ids=(rng.permutation(400)[:n] + 1).astype(np.uint32),
                  cls=np.zeros(n, np.int32), view_right=np.array([1, 0], np.float32),
                  centroids=np.zeros((1, d), np.float32))
    qb = QueryBatch(target=rng.standard_normal((2, d)).astype(np.float32), target_cls=np.array([-1, -1], np.int32),
                    rel_off=np.array([0, 2, 4], np.int32), rel_pred=np.array([BETWEEN, AND] * 2, np.int32),
                    rel_anchor=anchors, planted=np.zeros(2, np.int64))
    sub = QueryBatch(target=qb.target[:1], target_cls=qb.target_cls[:1], rel_off=qb.rel_off[:2],
                     rel_pred=qb.rel_pred[:2], rel_anchor=qb.rel_anchor[:2], planted=qb.planted[:1])
    small = Scene(desc=desc[:70], center=scene.center[:70], extent=scene.extent[:70], ids=scene.ids[:70],
                  cls=scene.cls[:70], view_right=scene.view_right, centroids=scene.centroids)
    np.testing.assert_allclose(oracle.score(small, sub), np.asarray(brute_scores(small, sub)), rtol=1e-12, atol=1e-14)
    # unrestricted maximum over every pair (numpy, vectorised), for comparison
    c = scene.center.astype(np.float64)
    u = desc.astype(np.float64) / np.linalg.norm(desc.astype(np.float64), axis=1, keepdims=True)
    _, _, t, _ = oracle.score(scene, qb, terms=True)
    sig = lambda v: 1 / (1 + np.exp(-v))
    differs = 0
    for k in range(2):
        a = [np.maximum(0, u @ (v / np.linalg.norm(v))) for v in qb.rel_anchor[2 * k:2 * k + 2].astype(np.float64)]
        ax = c[:, None, :] - c[None, :, :]           # c_j2 - c_j1 as [j2, j1]
        L = np.linalg.norm(ax, axis=2)
        for i in sorted(set(range(0, n, 3)) | {o}):
            w = c[i][None, :] - c                    # c_i - c_j1 as [j1]
            with np.errstate(divide="ignore", invalid="ignore"):
                s_ = np.einsum("bak,ak->ba", ax, w) / L   # along the axis from j1, [j2, j1]
                h2 = np.sum(w * w, axis=1)[None, :] - s_ * s_
                B = sig(s_ / 0.1) * sig((L - s_) / 0.1) * np.exp(-np.maximum(h2, 0) / 0.5)
            B[L == 0] = 0
            val = a[1][:, None] * a[0][None, :] * B
            val[i, :] = 0
            val[:, i] = 0
            full = float(np.nanmax(val))
            assert full >= t[2 * k, i] * (1 - 1e-9) - 1e-300
            differs += full > t[2 * k, i] * (1 + 1e-9)
    assert differs > 0
    with oracle.between_tolerance(-1, 0.05):
        _, _, t_lo, _ = oracle.score(scene, qb, terms=True)
    with oracle.between_tolerance(+1, 0.05):
        _, _, t_hi, _ = oracle.score(scene, qb, terms=True)
    assert np.all(t_lo <= t + 1e-15) and np.all(t <= t_hi + 1e-15) and np.any(t_hi > t)


# ------------------------------------------------- entity Gaussians, stored views
def _rot(yaw, pitch, roll):
    cz, sz, cy, sy, cx, sx = (math.cos(yaw), math.sin(yaw), math.cos(pitch), math.sin(pitch), math.cos(roll),
                              math.sin(roll))
    Rz = np.array([[cz, -sz, 0], [sz, cz, 0], [0, 0, 1]])
    Ry = np.array([[cy, 0, sy], [0, 1, 0], [-sy, 0, cy]])
    Rx = np.array([[1, 0, 0], [0, cx, -sx], [0, sx, cx]])
    return Rz @ Ry @ Rx


def _pack(S):
    return np.array([S[0, 0], S[0, 1], S[0, 2], S[1, 1], S[1, 2], S[2, 2]])


def test_hellinger_near_closed_forms():
    """Identical Gaussians give 1; equal isotropic Gaussians at distance d give
    1 - sqrt(1 - exp(-d^2 / (8 s^2))); concentric isotropic ones with sigmas a, b
    have Bhattacharyya coefficient (2ab / (a^2 + b^2))^(3/2)."""
    c = [1.0, -2.0, 0.5]
    cov = _pack(np.diag([0.04, 0.09, 0.01]))
    assert oracle.hellinger_near(c, cov, c, cov) == pytest.approx(1.0, abs=1e-15)
    s = 0.25
    for d in (0.0, 0.1, 0.4, 1.0):
        cj = [c[0] + d * 0.6, c[1] - d * 0.8, c[2]]
        want = 1 - math.sqrt(max(0.0, 1 - math.exp(-d * d / (8 * s * s))))
        got = oracle.hellinger_near(c, _pack(np.eye(3) * s * s), cj, _pack(np.eye(3) * s * s))
        assert got == pytest.approx(want, rel=1e-6, abs=1e-12), d
    for a, b in ((0.1, 0.1), (0.1, 0.3), (0.5, 0.125)):
        bc = (2 * a * b / (a * a + b * b)) ** 1.5
        got = oracle.hellinger_near(c, _pack(np.eye(3) * a * a), c, _pack(np.eye(3) * b * b))
        assert got == pytest.approx(1 - math.sqrt(1 - bc), rel=1e-6, abs=1e-12), (a, b)


def test_hellinger_near_matches_the_integral():
    """The Bhattacharyya coefficient is the integral of sqrt(p q) over space: a
    Riemann sum on a fine grid (spacing far below the smallest sigma, range 7
    sigma) for rotated, anisotropic, offset Gaussians."""
    rng = np.random.default_rng(7)
    for case in range(3):
        Ra = _rot(*rng.uniform(0, math.pi, 3))
        Rb = _rot(*rng.uniform(0, math.pi, 3))
        A = Ra @ np.diag(rng.uniform(0.18, 0.4, 3) ** 2) @ Ra.T
        B = Rb @ np.diag(rng.uniform(0.18, 0.4, 3) ** 2) @ Rb.T
        A, B = (np.asarray(_sym_from(_pack(M).astype(np.float32))) for M in (A, B))
        mu_a = np.zeros(3)
        mu_b = rng.uniform(-0.3, 0.3, 3).astype(np.float32).astype(np.float64)
        h = 0.025
        ax = np.arange(-2.9, 2.9 + h / 2, h)
        X, Y, Z = np.meshgrid(ax, ax, ax, indexing="ij")
        P = np.stack([X, Y, Z], axis=-1)

        def logpdf(mu, S):
            Si = np.linalg.inv(S)
            D = P - mu
            return -0.5 * np.einsum("...i,ij,...j->...", D, Si, D) - 0.5 * math.log((2 * math.pi) ** 3 * np.linalg.det(S))

        bc = float(np.exp(0.5 * (logpdf(mu_a, A) + logpdf(mu_b, B))).sum() * h ** 3)
        want = 1 - math.sqrt(max(0.0, 1 - bc))
        got = oracle.hellinger_near(mu_a, _pack(A), mu_b, _pack(B))
        assert got == pytest.approx(want, abs=1e-7), case


def _sym_from(p6):
    a, b, c, d, e, f = (float(v) for v in p6)
    return [[a, b, c], [b, d, e], [c, e, f]]


def test_hellinger_near_symmetric_and_rigid_invariant():
    rng = np.random.default_rng(3)
    for _ in range(5):
        Ra, Rb = _rot(*rng.uniform(0, 3, 3)), _rot(*rng.uniform(0, 3, 3))
        A = Ra @ np.diag(rng.uniform(0.1, 0.5, 3) ** 2) @ Ra.T
        B = Rb @ np.diag(rng.uniform(0.1, 0.5, 3) ** 2) @ Rb.T
        ca, cb = rng.uniform(-1, 1, 3), rng.uniform(-1, 1, 3)
        v = oracle.hellinger_near(ca, _pack(A), cb, _pack(B))
        assert 0.0 <= v <= 1.0
        assert oracle.hellinger_near(cb, _pack(B), ca, _pack(A)) == pytest.approx(v, rel=1e-12)
        Q, t = _rot(*rng.uniform(0, 3, 3)), rng.uniform(-5, 5, 3)
        w = oracle.hellinger_near(Q @ ca + t, _pack(Q @ A @ Q.T), Q @ cb + t, _pack(Q @ B @ Q.T))
        assert w == pytest.approx(v, rel=2e-5, abs=1e-6)


def _camera(pos, yaw, pitch):
    """A level pinhole camera at pos looking along (yaw, pitch): [pos, right, down, forward]."""
    f = np.array([math.cos(pitch) * math.cos(yaw), math.cos(pitch) * math.sin(yaw), math.sin(pitch)])
    r = np.array([math.sin(yaw), -math.cos(yaw), 0.0])
    dn = np.cross(f, r)
    return np.concatenate([pos, r, dn, f]), (r, dn, f)


def test_view_predicates_recover_camera_coordinates():
    """Points placed at known camera-frame coordinates (x, y, z) of a tilted,
    turned camera: left/right follow the image-plane coordinates x / z, front /
    behind the depths z, whatever the camera's pose."""
    sig = lambda v: 1.0 / (1.0 + math.exp(-v))
    for yaw, pitch in ((0.3, -0.4), (2.5, 0.2), (-1.2, -0.9)):
        pos = np.array([1.0, -3.0, 1.5])
        view, (r, dn, f) = _camera(pos, yaw, pitch)
        world = lambda x, y, z: pos + x * r + y * dn + z * f
        for (xo, yo, zo), (xa, ya, za) in (((-0.2, 0.1, 2.0), (0.3, -0.2, 3.0)), ((0.5, 0.0, 1.0), (0.1, 0.3, 2.5)),
                                           ((0.0, 0.0, 1.5), (0.0, 0.0, 1.2))):
            ci, cj = world(xo, yo, zo).astype(np.float32), world(xa, ya, za).astype(np.float32)
            vw = view.astype(np.float32)
            uo, ua = xo / zo, xa / za
            tol = dict(rel=1e-4, abs=1e-6)  # the float32 rounding of the world coordinates
            assert oracle.view_predicate(15, vw, ci, cj) == pytest.approx(sig((ua - uo) / 0.05), **tol)
            assert oracle.view_predicate(16, vw, ci, cj) == pytest.approx(sig((uo - ua) / 0.05), **tol)
            assert oracle.view_predicate(17, vw, ci, cj) == pytest.approx(sig((za - zo) / 0.1), **tol)
            assert oracle.view_predicate(18, vw, ci, cj) == pytest.approx(sig((zo - za) / 0.1), **tol)


def test_view_predicates_need_both_objects_in_view():
    view, (r, dn, f) = _camera(np.zeros(3), 0.7, -0.3)
    world = lambda x, y, z: (x * r + y * dn + z * f).astype(np.float32)
    vw = view.astype(np.float32)
    o = world(0.0, 0.0, 2.0)
    inside = [(0.0, 0.0, 0.15), (1.9, 0.0, 2.0), (0.0, -1.4, 2.0)]
    outside = [(0.0, 0.0, 0.05), (0.0, 0.0, -2.0), (2.1, 0.0, 2.0), (0.0, 1.6, 2.0)]
    for p in (15, 16, 17, 18):
        for c in inside:
            assert oracle.view_predicate(p, vw, o, world(*c)) > 0.0, (p, c)
            assert oracle.view_predicate(p, vw, world(*c), o) > 0.0, (p, c)
        for c in outside:
            assert oracle.view_predicate(p, vw, o, world(*c)) == 0.0, (p, c)
            assert oracle.view_predicate(p, vw, world(*c), o) == 0.0, (p, c)
    # complements for a visible pair
    a = world(0.4, 0.2, 3.0)
    assert oracle.view_predicate(15, vw, o, a) + oracle.view_predicate(16, vw, o, a) == pytest.approx(1.0, abs=1e-12)
    assert oracle.view_predicate(17, vw, o, a) + oracle.view_predicate(18, vw, o, a) == pytest.approx(1.0, abs=1e-12)


def _tiny_geometry(seed, n, r, q=3):
    from synth import GEOMETRY_PREDS, add_entity_geometry
    scene, qb = _tiny(seed, n, r, q=q)
    scene = add_entity_geometry(scene, seed)
    rng = np.random.default_rng(seed + 77)
    preds = rng.choice(list(GEOMETRY_PREDS) + [NEAR, LEFT_OF], size=qb.rel_pred.shape[0]).astype(np.int32)
    return scene, QueryBatch(qb.target, qb.target_cls, qb.rel_off, preds, qb.rel_anchor, qb.planted)


@pytest.mark.parametrize("n,r", [(2, 1), (5, 2), (7, 3)])
def test_geometry_predicates_star_decomposition(n, r):
    """Hellinger Near and the stored-view predicates: the star decomposition
    equals joint enumeration, whose evaluators (elimination-based Hellinger,
    basis-vector projection) are written independently."""
    for seed in range(3):
        scene, qb = _tiny_geometry(seed * 13 + n + r, n, r)
        s = oracle.score(scene, qb)
        bs = np.asarray(brute_scores(scene, qb))
        np.testing.assert_allclose(s, bs, rtol=1e-12, atol=1e-14)


def test_geometry_predicates_need_the_scene_geometry():
    scene, qb = _tiny_geometry(5, 6, 2)
    bare = Scene(scene.desc, scene.center, scene.extent, scene.ids, scene.cls, scene.view_right, scene.centroids)
    for drop in ("cov", "view"):
        s2 = Scene(scene.desc, scene.center, scene.extent, scene.ids, scene.cls, scene.view_right, scene.centroids,
                   cov=None if drop == "cov" else scene.cov, view=None if drop == "view" else scene.view)
        needs = {"cov": [14], "view": [15, 16, 17, 18]}[drop]
        if np.isin(qb.rel_pred, needs).any():
            with pytest.raises(ValueError):
                oracle.score(s2, qb)
    with pytest.raises(ValueError):
        oracle.score(bare, qb)
    # the scene's geometry does not leak into a later call on another scene
    plain = QueryBatch(qb.target, qb.target_cls, qb.rel_off, np.zeros_like(qb.rel_pred), qb.rel_anchor, qb.planted)
    np.testing.assert_array_equal(oracle.score(bare, plain), oracle.score(scene, plain))
