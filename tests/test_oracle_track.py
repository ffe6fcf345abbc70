"""Pins of the tracking oracle against hand-worked cases, closed forms and an independent
matcher.  No GPU."""
import numpy as np
import pytest

from oracle import track as T

f32 = np.float32


def _run(frames, gate=5.0, memory=1):
    tr = T.Tracker(gate, memory)
    return [list(ids) for ids in tr.link([np.array(f, dtype=f32).reshape(-1, 3) for f in frames])], tr


def test_constant_velocity_is_followed_exactly():
    """Two particles on straight lines at 4 px per frame that pass each other 1 px apart
    (gate 5 px).  The first step links by proximity (no velocity yet); from then on the
    prediction p + v g is exact in float32 for these integers and the true continuation
    costs 0.  At the crossing a zero velocity, or a sign error (p - v g), makes the other
    particle the nearer one and swaps the ids."""
    frames = []
    for t in range(8):
        frames.append([(10.0 + 4 * t, 50.0, 12.0), (38.0 - 4 * t, 51.0, 12.0)])
    ids, tr = _run(frames, gate=5.0, memory=0)
    assert all(i == [0, 1] for i in ids), ids
    assert len(tr.p) == 2
    np.testing.assert_array_equal(tr.v, np.array([[4, 0, 0], [-4, 0, 0]], dtype=f32))


def test_velocity_starts_at_the_second_detection():
    """With a gate wide enough for the first step, the velocity learnt from it predicts the
    third position exactly (cost 0 beats a distractor at cost 1)."""
    frames = [[(0, 0, 10)], [(3, 0, 10)], [(6, 0, 10), (4, 0, 10)]]
    ids, _ = _run(frames, gate=3.5, memory=0)
    assert ids == [[0], [0], [0, 1]]


def test_radius_is_part_of_the_cost():
    """Two detections at the same (x, y) distance, one with the track's radius and one 2 px
    off: the radius term decides; without it the lower detection index would win."""
    frames = [[(10, 10, 20)], [(11, 10, 22), (9, 10, 20)]]
    ids, _ = _run(frames, gate=5.0, memory=0)
    assert ids == [[0], [1, 0]]


@pytest.mark.parametrize("memory,gap,same", [(0, 1, False), (1, 1, True), (1, 2, False), (2, 2, True), (3, 3, True),
                                             (3, 4, False)])
def test_memory_keeps_a_track_for_exactly_that_many_missed_frames(memory, gap, same):
    frames = [[(5, 5, 9)]] + [[]] * gap + [[(5, 5, 9)]]
    ids, _ = _run(frames, gate=1.0, memory=memory)
    assert (ids[-1] == [0]) == same, ids


def test_ties_go_to_the_lower_track_id_then_the_lower_detection():
    """A detection equidistant from two tracks goes to the older track; a track equidistant
    from two detections takes the lower detection index."""
    ids, _ = _run([[(0, 0, 10), (4, 0, 10)], [(2, 0, 10)]], gate=3.0, memory=0)
    assert ids[1] == [0]
    ids, _ = _run([[(0, 0, 10)], [(0, 2, 10), (0, -2, 10)]], gate=3.0, memory=0)
    assert ids[1] == [0, 1]


def test_greedy_is_not_the_optimal_assignment():
    """Greedy takes the globally closest pair first even when that strands the other
    track: tracks at 0 and 3, detections at 2 and 5 (gate 2.5).  Pair (3, 2) costs 1, so it
    goes first; track 0 then has no detection within the gate, and detection 5 opens a new
    track, although 0->2, 3->5 would link both."""
    ids, _ = _run([[(0, 0, 10), (3, 0, 10)], [(2, 0, 10), (5, 0, 10)]], gate=2.5, memory=0)
    assert ids[1] == [1, 2]


def test_new_ids_follow_detection_order():
    ids, _ = _run([[(0, 0, 10)], [(50, 0, 10), (0, 1, 10), (90, 0, 10), (30, 0, 10)]], gate=2.0, memory=0)
    assert ids[1] == [1, 0, 2, 3]


def _mutual_best(frames, gate, memory):
    """An independent tracker: the matching as rounds of pairs that are the smallest at both
    ends among the free pairs (with the order (c, i, j) this is the greedy matching)."""
    p, v, tl, ids_all, act = [], [], [], [], []
    g2 = f32(gate) * f32(gate)
    for t, det in enumerate(frames):
        det = np.array(det, dtype=f32).reshape(-1, 3)
        act = [i for i in act if t - tl[i] <= memory + 1]
        edges = []
        for i in act:
            g = f32(t - tl[i])
            q = [p[i][k] + v[i][k] * g for k in range(3)]
            for j in range(len(det)):
                d = [q[k] - det[j][k] for k in range(3)]
                c = d[0] * d[0] + d[1] * d[1] + d[2] * d[2]
                if c <= g2:
                    edges.append((c, i, j))
        ti, dj = {}, {}
        while True:
            free = [e for e in edges if e[1] not in ti and e[2] not in dj]
            if not free:
                break
            best_t, best_d = {}, {}
            for c, i, j in free:
                best_t[i] = min(best_t.get(i, (np.inf, 0)), (c, j))
                best_d[j] = min(best_d.get(j, (np.inf, 0)), (c, i))
            for c, i, j in free:
                if best_t[i] == (c, j) and best_d[j] == (c, i):
                    ti[i], dj[j] = j, i
        out = []
        for j in range(len(det)):
            if j in dj:
                i = dj[j]
                g = f32(t - tl[i])
                v[i] = [(det[j][k] - p[i][k]) / g for k in range(3)]
                p[i], tl[i] = list(det[j]), t
                out.append(i)
            else:
                out.append(-1)
        for j in range(len(det)):
            if out[j] < 0:
                out[j] = len(p)
                p.append(list(det[j]))
                v.append([f32(0)] * 3)
                tl.append(t)
                act.append(out[j])
        ids_all.append(out)
    return ids_all


@pytest.mark.parametrize("seed", range(12))
def test_sorted_greedy_equals_rounds_of_mutual_best_pairs(seed):
    """Crowded random scenes with integer coordinates (many equal costs): the oracle's
    sort-based greedy and the round-based matcher agree on every id."""
    rng = np.random.default_rng(seed)
    frames = []
    n = 14
    pos = rng.integers(0, 12, size=(n, 2)).astype(np.float64)
    for t in range(10):
        pos += rng.integers(-2, 3, size=pos.shape)
        keep = rng.random(n) > 0.15
        det = [(x, y, 10.0 + (k % 3)) for k, (x, y) in enumerate(pos) if keep[k]]
        det += [tuple(rng.integers(0, 12, 2).astype(float)) + (11.0,) for _ in range(rng.integers(0, 3))]
        rng.shuffle(det)
        frames.append(det)
    got, _ = _run(frames, gate=3.0, memory=2)
    assert got == _mutual_best(frames, 3.0, 2)


@pytest.mark.parametrize("c", [(8.0, 0.0, 72.0), (5.0, -3.0, 2.5), (20.0, 4.0, 0.5)])
def test_depth_inverts_the_quadratic(c):
    """z(r(z)) = z on the branch right of the vertex, for the stream's r = 8 + 72 z^2 and two
    general quadratics."""
    c0, c1, c2 = c
    zv = -c1 / (2 * c2)
    z = zv + np.linspace(0.0, 3.0, 301)
    r = c0 + c1 * z + c2 * z * z
    np.testing.assert_allclose(T.depth(r, c0, c1, c2), z, rtol=0, atol=1e-9 * max(1.0, abs(z).max()))
    # below the vertex the discriminant is clamped: the vertex itself
    assert T.depth(np.array([c0 + c1 * zv + c2 * zv * zv - 1.0]), c0, c1, c2)[0] == pytest.approx(zv)


def test_random_walks_are_recovered():
    """Well-separated particles on random walks (the stream's 1.5 px per frame in x and y),
    observed without noise: every id is kept for the whole sequence."""
    rng = np.random.default_rng(7)
    g = np.stack(np.meshgrid(np.arange(6), np.arange(6)), -1).reshape(-1, 2) * 60.0 + 30.0
    z = rng.uniform(0, 1, len(g))
    frames = []
    for t in range(30):
        g = g + rng.normal(0, 1.5, g.shape)
        z = np.clip(z + rng.normal(0, 0.01, z.shape), 0, 1)
        frames.append([(x, y, 8 + 72 * zz * zz) for (x, y), zz in zip(g, z)])
    ids, tr = _run(frames, gate=12.0, memory=1)
    assert all(i == list(range(len(g))) for i in ids)
    assert len(tr.p) == len(g)


# ------------------------------------------------------------------ acceleration model

def _run_model(frames, gate, memory, model):
    tr = T.Tracker(gate, memory, model=model)
    return [list(ids) for ids in tr.link([np.array(f, dtype=f32).reshape(-1, 3) for f in frames])], tr


def test_constant_acceleration_is_followed_exactly():
    """x_t = t^2 + t (0, 2, 6, 12, 20): from the third detection on, the quadratic through
    the last three is exact (weights 1, -3, 3 on integers).  At t = 4 a decoy sits where a
    constant velocity would put the particle (x_3 + (x_3 - x_2) = 18): the acceleration
    model takes the true position (cost 0 against 4), the velocity model the decoy."""
    frames = [[(t * t + t, 40.0, 15.0)] for t in range(4)] + [[(18.0, 40.0, 15.0), (20.0, 40.0, 15.0)]]
    ids, tr = _run_model(frames, gate=5.0, memory=0, model="acceleration")
    assert ids == [[0], [0], [0], [0], [1, 0]], ids
    ids, _ = _run_model(frames, gate=5.0, memory=0, model="velocity")
    assert ids == [[0], [0], [0], [0], [0, 1]], ids
    np.testing.assert_array_equal(tr.predict(0, 5), np.array([30, 40, 15], dtype=f32))


def test_acceleration_prediction_is_the_polynomial_through_the_history():
    """Irregular detection times (misses within the memory): the prediction equals the
    polynomial through the last three detections, and through the only two while the track
    has two, evaluated by numpy's polynomial fit in float64, to float32 rounding."""
    rng = np.random.default_rng(7)
    times = [0, 2, 3, 6, 7, 9]
    pts = rng.uniform(10, 500, size=(len(times), 3)).astype(f32)
    frames = [[] for _ in range(max(times) + 1)]
    for t, p in zip(times, pts):
        frames[t] = [tuple(p)]
    tr = T.Tracker(gate=1e6, memory=3, model="acceleration")
    for t, f in enumerate(frames):
        if t > 0 and f:
            hist_t = [tk for tk, _ in tr.hist[0]]
            hist_q = np.array([q for _, q in tr.hist[0]], dtype=np.float64)
            for tq in (t, t + 1):
                want = np.array([np.polyval(np.polyfit(hist_t, hist_q[:, c], len(hist_t) - 1), tq)
                                 for c in range(3)]) if len(hist_t) > 1 else hist_q[-1]
                got = tr.predict(0, tq).astype(np.float64)
                scale = np.abs(hist_q).max() * 24
                assert np.all(np.abs(got - want) <= 4e-7 * scale), (t, tq, hist_t, got, want)
        ids = tr.link_frame(np.array(f, dtype=f32).reshape(-1, 3))
        assert list(ids) == ([0] if f else [])
    assert [tk for tk, _ in tr.hist[0]] == [6, 7, 9]


def test_acceleration_history_starts_with_each_track():
    """A new track predicts its own position, then the line through two detections (a
    velocity learnt over a gap of 2 frames): x = 10, then 14 two frames later, then 16 is
    the line's value one frame on (cost 0, against a decoy at 15, cost 1)."""
    frames = [[(10.0, 0.0, 9.0)], [], [(14.0, 0.0, 9.0)], [(15.0, 0.0, 9.0), (16.0, 0.0, 9.0)]]
    ids, tr = _run_model(frames, gate=5.0, memory=1, model="acceleration")
    assert ids == [[0], [], [0], [1, 0]], ids
    assert [tk for tk, _ in tr.hist[0]] == [0, 2, 3]


def test_models_share_gate_memory_and_matching():
    """Gate, memory and the greedy tie rules do not depend on the model: a track with one
    detection predicts its position under both, so these cases give the same ids."""
    cases = [([[(0, 0, 10), (4, 0, 10)], [(2, 0, 10)]], 3.0, 0),
             ([[(0, 0, 10)], [(0, 2, 10), (0, -2, 10)]], 3.0, 0),
             ([[(5, 5, 9)], [], [], [(5, 5, 9)]], 1.0, 2),
             ([[(5, 5, 9)], [], [], [(5, 5, 9)]], 1.0, 1)]
    for frames, gate, mem in cases:
        a, _ = _run_model(frames, gate, mem, "velocity")
        b, _ = _run_model(frames, gate, mem, "acceleration")
        assert a == b, (frames, a, b)


def test_unknown_model_is_refused():
    with pytest.raises(ValueError):
        T.Tracker(1.0, 0, model="jerk")
