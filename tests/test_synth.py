"""The input generator's fast paths against its reference forms (CPU only): the stream's
trajectories drawn at once equal state(t) frame by frame, and the torch renderer equals the
numpy renderer to float32 rounding, boxes and frame clipping included."""
import numpy as np
import torch

from paper_1310_1371_amd import synth


def test_trajectories_equal_state():
    st = synth.Stream(seed=4, W=512, H=384, n_rings=50)
    xs, ys, zs = st.trajectories(6)
    for t in range(6):
        x, y, z = st.state(t)
        np.testing.assert_array_equal(xs[t], x)
        np.testing.assert_array_equal(ys[t], y)
        np.testing.assert_array_equal(zs[t], z)


def test_render_torch_equals_render():
    rng = np.random.default_rng(7)
    W, H, n = 300, 200, 40
    cx = rng.uniform(-20, W + 20, n)          # some rings cut by the frame edges, some outside
    cy = rng.uniform(-20, H + 20, n)
    R = rng.uniform(3, 70, n)
    s = rng.uniform(1.0, 2.5, n)
    A = rng.uniform(100, 1000, n)
    ref = synth.render(W, H, np.full((H, W), 200.0), cx, cy, R, s, A)
    got = synth.render_torch(W, H, 200.0, cx, cy, R, s, A, "cpu").double().numpy()
    assert np.abs(got - ref).max() <= 1e-5 * np.abs(ref).max()     # float32 rounding


def test_render_device_is_the_stream_model():
    st = synth.Stream(seed=4, W=256, H=256, n_rings=20)
    x, y, z = st.state(3)
    out = torch.empty((256, 256), dtype=torch.int16)
    g = torch.Generator().manual_seed(0)
    st.render_device(x, y, z, out, g)
    clean = synth.render(256, 256, np.full((256, 256), 200.0), x, y, st.radius(z), np.full(20, 1.5),
                         np.full(20, 1000.0))
    d = out.numpy().astype(np.float64) - np.clip(clean, 0, 4095)
    assert out.min() >= 0 and out.max() <= 4095
    assert abs(d.mean()) < 1.0 and 45.0 < d.std() < 55.0     # N(0, 50^2) noise, rounded
