"""Oracle of frame-to-frame linking of detected rings into trajectories, and of the depth
read from a ring's radius.

TEST INFRASTRUCTURE ONLY, like ridge_hough.py: only the tests, the smoke check and the
benchmark's CPU-baseline leg may use it, and it shares no code with the HIP path.

The paper links its ring lists with a predictive nearest-neighbour tracker (Methods,
*Experimental details*: a kinematic prediction and a memory for occasional misses) and turns
a ring's radius into depth by inverting a quadratic fit of radius against defocus (SI,
calibration curve figure: the larger root).  It prints neither the tracker nor the gate, so
what follows fixes one (readings):

  state        every track keeps its last position p = (x, y, r), a velocity v (zero until
               its second detection) and the frame t_l it was last seen in; track ids are
               0, 1, 2, ... in order of creation.
  active       a track takes part in frame t while t - t_l <= memory + 1 (it has missed at
               most `memory` frames); after that it is retired for good.
  prediction   p^ = p + v * g with g = t - t_l.
  cost         c = (x^ - x)^2 + (y^ - y)^2 + (r^ - r)^2 against each detection (x, y, r) of
               frame t; a pair is a candidate when c <= gate^2.
  matching     greedy: candidates in increasing order of (c, track id, detection index),
               each accepted when neither its track nor its detection is taken yet.
  update       a matched track gets v = (d - p) / g, p = d, t_l = t; every unmatched
               detection starts a new track (v = 0), ids handed out in increasing order of
               detection index.
  precision    float32 throughout, in the order written above (each product and sum rounded
               on its own): the matching is a decision taken in float, so both this oracle
               and the kernel take it in the same precision.
  depth        z(r) = the larger root of c2 z^2 + c1 z + (c0 - r) = 0, the discriminant
               clamped at 0; float64 here.

The paper's linker accounts for accelerations in its kinematic model (Methods, *Precision
assessment*).  With model="acceleration" (reading) the state and prediction above change:

  state        a track keeps its last three detections (t_k, q_k), k = 0, 1, 2 with
               t_0 < t_1 < t_2 = t_l, fewer while it is young.
  prediction   the polynomial through them evaluated at t, in Lagrange form: with one
               detection p^ = q_2; with two, p^ = w_2 q_2 + w_1 q_1, w_2 = (t - t_1) /
               (t_2 - t_1), w_1 = (t - t_2) / (t_1 - t_2); with three (constant
               acceleration), p^ = (w_2 q_2 + w_1 q_1) + w_0 q_0 with
               w_k = prod_{m != k} (t - t_m) / prod_{m != k} (t_k - t_m).  Each weight is a
               float32 division of its numerator and denominator, integers formed exactly
               and converted to float32; the products and sums are float32, rounded one at
               a time in the order written.
  update       a matched track appends (t, d) and drops its oldest detection beyond three.

Detections come in as float32 (x, y, r) per frame, e.g. the fitted rings of a detection.
"""
from __future__ import annotations

import numpy as np

f32 = np.float32


MODELS = ("velocity", "acceleration")


def lagrange_weights(ts, t):
    """float32 weights of the polynomial through the detections at frames ts (ascending,
    one to three of them) evaluated at frame t, in the order of ts."""
    ts = [int(v) for v in ts]
    w = []
    for k, tk in enumerate(ts):
        num, den = 1, 1
        for m, tm in enumerate(ts):
            if m != k:
                num *= t - tm
                den *= tk - tm
        w.append(f32(num) / f32(den))
    return w


class Tracker:
    """Tracks across calls of `link`; frame numbers continue from call to call."""

    def __init__(self, gate: float, memory: int, model: str = "velocity"):
        if model not in MODELS:
            raise ValueError(f"model must be one of {MODELS}")
        self.gate = f32(gate)
        self.memory = int(memory)
        self.model = model
        self.p = np.zeros((0, 3), dtype=f32)
        self.v = np.zeros((0, 3), dtype=f32)
        self.t_last = np.zeros(0, dtype=np.int64)
        self.hist = []                                   # acceleration model: [(t, q)] per track, oldest first
        self.active = np.zeros(0, dtype=np.int64)      # ids of the tracks still taking part
        self.t = 0

    def predict(self, i: int, t: int) -> np.ndarray:
        """Predicted (x, y, r) of track i at frame t (float32)."""
        if self.model == "velocity":
            return self.p[i] + self.v[i] * f32(t - self.t_last[i])
        h = self.hist[i]
        w = lagrange_weights([tk for tk, _ in h], t)
        pred = w[-1] * h[-1][1]
        for k in range(len(h) - 2, -1, -1):           # w_2 q_2 + w_1 q_1, then + w_0 q_0
            pred = pred + w[k] * h[k][1]
        return pred

    def link_frame(self, det: np.ndarray) -> np.ndarray:
        """Link one frame's detections (n x 3 float32: x, y, r); returns their track ids."""
        det = np.asarray(det, dtype=f32).reshape(-1, 3)
        t = self.t
        act = self.active[t - self.t_last[self.active] <= self.memory + 1]
        g2 = self.gate * self.gate
        cand = []
        for i in act:
            pred = self.predict(int(i), t)
            d = pred[None, :] - det
            c = d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1] + d[:, 2] * d[:, 2]
            for j in np.nonzero(c <= g2)[0]:
                cand.append((c[j], int(i), int(j)))
        cand.sort()
        ids = np.full(len(det), -1, dtype=np.int64)
        taken = set()
        for c, i, j in cand:
            if i in taken or ids[j] >= 0:
                continue
            taken.add(i)
            ids[j] = i
        for j in np.nonzero(ids >= 0)[0]:
            i = ids[j]
            g = f32(t - self.t_last[i])
            self.v[i] = (det[j] - self.p[i]) / g
            self.p[i] = det[j]
            self.t_last[i] = t
            self.hist[i] = (self.hist[i] + [(t, det[j].copy())])[-3:]
        new = np.nonzero(ids < 0)[0]
        first = len(self.p)
        ids[new] = first + np.arange(len(new))
        self.p = np.concatenate([self.p, det[new]])
        self.v = np.concatenate([self.v, np.zeros((len(new), 3), dtype=f32)])
        self.t_last = np.concatenate([self.t_last, np.full(len(new), t, dtype=np.int64)])
        self.hist += [[(t, det[j].copy())] for j in new]
        self.active = np.concatenate([act, ids[new]])
        self.t += 1
        return ids

    def link(self, frames) -> list[np.ndarray]:
        return [self.link_frame(d) for d in frames]


def depth(r, c0: float, c1: float, c2: float) -> np.ndarray:
    """Larger root of c2 z^2 + c1 z + c0 - r = 0 (c2 != 0), discriminant clamped at 0."""
    r = np.asarray(r, dtype=np.float64)
    disc = np.maximum(c1 * c1 - 4.0 * c2 * (c0 - r), 0.0)
    return (-c1 + np.sqrt(disc)) / (2.0 * c2)
