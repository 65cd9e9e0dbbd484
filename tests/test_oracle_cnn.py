"""Pins of the FP64 reference of the surrogate network."""

import numpy as np

from oracle import cnn


def test_identity_kernel_is_identity():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(3, 7, 5))
    w = np.zeros((3, 3, 3, 3))
    for c in range(3):
        w[c, c, 1, 1] = 1.0
    assert np.array_equal(cnn.conv3x3(x, w, np.zeros(3)), x)


def test_shift_kernel_is_periodic_shift():
    """A single 1 at offset (dy, dx) reads the periodic neighbour x[i+dy, j+dx]."""
    rng = np.random.default_rng(1)
    x = rng.normal(size=(1, 6, 9))
    for dy, dx in cnn.OFFSETS:
        w = np.zeros((1, 1, 3, 3))
        w[0, 0, dy + 1, dx + 1] = 1.0
        y = cnn.conv3x3(x, w, np.zeros(1))
        i, j = 2, 8
        assert y[0, i, j] == x[0, (i + dy) % 6, (j + dx) % 9]


def test_conv_brute_force():
    rng = np.random.default_rng(2)
    x = rng.normal(size=(2, 4, 5))
    w = rng.normal(size=(3, 2, 3, 3))
    b = rng.normal(size=3)
    y = cnn.conv3x3(x, w, b)
    for o in range(3):
        for i in range(4):
            for j in range(5):
                s = b[o]
                for c in range(2):
                    for dy in (-1, 0, 1):
                        for dx in (-1, 0, 1):
                            s += w[o, c, dy + 1, dx + 1] * x[c, (i + dy) % 4, (j + dx) % 5]
                assert abs(y[o, i, j] - s) < 1e-12


def test_translation_equivariance():
    rng = np.random.default_rng(3)
    p = cnn.init_params(3)
    x = rng.normal(size=(6, 8, 8))
    y, _ = cnn.forward(p, x)
    ys, _ = cnn.forward(p, np.roll(x, (2, -3), axis=(1, 2)))
    assert np.allclose(ys, np.roll(y, (2, -3), axis=(1, 2)), atol=1e-12)


def test_output_bounds():
    rng = np.random.default_rng(4)
    p = cnn.init_params(4)
    y, _ = cnn.forward(p, 10 * rng.normal(size=(6, 5, 5)))
    assert np.all(y >= 0) and np.all(y <= 4)


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(5)
    p = cnn.init_params(5)
    for k in p:
        if k.startswith("b"):
            p[k] = 0.1 * rng.normal(size=p[k].shape)
    x = rng.normal(size=(6, 5, 6))
    t = 4 * rng.uniform(size=(10, 5, 6))
    pred, acts = cnn.forward(p, x)
    g = cnn.backward(p, acts, t)
    eps = 1e-6
    for k in p:
        flat = p[k].reshape(-1)
        idxs = rng.choice(flat.size, size=min(6, flat.size), replace=False)
        for i in idxs:
            old = flat[i]
            flat[i] = old + eps
            lp = cnn.loss(cnn.forward(p, x)[0], t)
            flat[i] = old - eps
            lm = cnn.loss(cnn.forward(p, x)[0], t)
            flat[i] = old
            fd = (lp - lm) / (2 * eps)
            an = g[k].reshape(-1)[i]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (k, i, fd, an)


def test_input_gradient_matches_finite_differences():
    """The conv backward-data path (transposed offsets) on its own."""
    rng = np.random.default_rng(6)
    x = rng.normal(size=(3, 4, 5))
    w = rng.normal(size=(2, 3, 3, 3))
    dy_ = rng.normal(size=(2, 4, 5))
    dx_, _, _ = cnn.conv3x3_grads(x, w, dy_)
    f = lambda xx: float(np.sum(dy_ * cnn.conv3x3(xx, w, np.zeros(2))))  # noqa: E731
    for idx in [(0, 0, 0), (1, 3, 4), (2, 1, 2)]:
        e = np.zeros_like(x)
        e[idx] = 1e-6
        fd = (f(x + e) - f(x - e)) / 2e-6
        assert abs(fd - dx_[idx]) < 1e-7


def test_adam_first_step_moves_by_lr():
    """With bias correction the first Adam step moves each weight by lr * sign(g)."""
    p = {"w": np.array([1.0, -2.0, 3.0])}
    g = {"w": np.array([0.5, -4.0, 1e-3])}
    m = {"w": np.zeros(3)}
    v = {"w": np.zeros(3)}
    cnn.adam_step(p, g, m, v, 1, lr=0.01, eps=0.0)
    assert np.allclose(p["w"], [0.99, -1.99, 2.99], atol=1e-15)


def test_adam_bias_correction_with_constant_gradient():
    """A constant gradient g gives m_t = (1 - b1^t) g and v_t = (1 - b2^t) g^2,
    so with bias correction (and eps = 0) every step, not only the first,
    moves the weight by exactly lr * sign(g).  A wrong power of b1 or b2 in
    the correction fails from t = 2 on."""
    p = {"w": np.array([1.0, -2.0])}
    g = {"w": np.array([0.3, -5.0])}
    m = {"w": np.zeros(2)}
    v = {"w": np.zeros(2)}
    for t in range(1, 6):
        before = p["w"].copy()
        cnn.adam_step(p, g, m, v, t, lr=0.125, b1=0.75, b2=0.5, eps=0.0)
        assert np.allclose(p["w"] - before, [-0.125, 0.125], rtol=0, atol=1e-15), t


def test_adam_steps_two_and_three_hand_computed():
    """Gradients 1, -1, 2 with b1 = b2 = 1/2, lr = 1/10, eps = 0, from w = 0:
    t = 1: m = 1/2, v = 1/2, corrected 1 and 1: w = -1/10;
    t = 2: m = 1/4 - 1/2 = -1/4, v = 1/4 + 1/2 = 3/4, corrected by 3/4:
           m^ = -1/3, v^ = 1: w = -1/10 + 1/30;
    t = 3: m = -1/8 + 1 = 7/8, v = 3/8 + 2 = 19/8, corrected by 7/8:
           m^ = 1, v^ = 19/7: w = -1/10 + 1/30 - (1/10) sqrt(7/19)."""
    p = {"w": np.zeros(1)}
    m = {"w": np.zeros(1)}
    v = {"w": np.zeros(1)}
    want = [-0.1, -0.1 + 1.0 / 30.0, -0.1 + 1.0 / 30.0 - 0.1 * np.sqrt(7.0 / 19.0)]
    for t, gv in enumerate((1.0, -1.0, 2.0), start=1):
        cnn.adam_step(p, {"w": np.array([gv])}, m, v, t, lr=0.1, b1=0.5, b2=0.5, eps=0.0)
        assert abs(p["w"][0] - want[t - 1]) <= 1e-15, (t, p["w"][0], want[t - 1])


def test_training_reduces_loss():
    rng = np.random.default_rng(7)
    p = cnn.init_params(7)
    x = rng.normal(size=(6, 6, 6))
    t = 4 / (1 + np.exp(-x[:1].repeat(10, axis=0)))
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(val) for k, val in p.items()}
    l0 = cnn.loss(cnn.forward(p, x)[0], t)
    for it in range(1, 31):
        pred, acts = cnn.forward(p, x)
        cnn.adam_step(p, cnn.backward(p, acts, t), m, v, it, lr=3e-3)
    assert cnn.loss(cnn.forward(p, x)[0], t) < 0.5 * l0


def test_bf16_round_known_values():
    """Round to nearest even on the 8-bit significand."""
    one = 1.0
    ulp = 2.0 ** -7                     # BF16 spacing just above 1
    vals = np.array([one, one + ulp / 2, one + 3 * ulp / 2, one + ulp / 4, one + 3 * ulp / 4,
                     -2.5, 3.0e38, 1e-40])
    got = cnn.bf16_round(vals)
    assert got[0] == 1.0
    assert got[1] == 1.0                # tie -> even (1.0)
    assert got[2] == one + 2 * ulp      # tie -> even (1 + 2 ulp)
    assert got[3] == 1.0
    assert got[4] == one + ulp
    assert got[5] == -2.5
    assert np.isfinite(got[6])
    # every result is a BF16 value: low 16 bits of the float32 pattern are 0
    assert np.all((got.astype(np.float32).view(np.uint32) & 0xFFFF) == 0)


def test_bf16_mode_close_to_exact_mode():
    rng = np.random.default_rng(8)
    p = cnn.init_params(8)
    for k in p:
        if k.startswith("b"):
            p[k] = 0.05 * rng.normal(size=p[k].shape)
    x = rng.normal(size=(6, 9, 7))
    t = 4 * rng.uniform(size=(10, 9, 7))
    y64, a64 = cnn.forward(p, x)
    y16, a16 = cnn.forward(p, x, bf16=True)
    assert np.max(np.abs(y16 - y64)) < 0.05 and not np.array_equal(y16, y64)
    g64 = cnn.backward(p, a64, t)
    g16 = cnn.backward(p, a16, t, bf16=True)
    for k in g64:
        rel = np.linalg.norm(g16[k] - g64[k]) / np.linalg.norm(g64[k])
        assert rel < 0.15, (k, rel)


def test_batch_grads_are_sum_over_images():
    rng = np.random.default_rng(9)
    p = cnn.init_params(9)
    xs = [rng.normal(size=(6, 5, 5)) for _ in range(3)]
    ts = [4 * rng.uniform(size=(10, 5, 5)) for _ in range(3)]
    loss, g = cnn.batch_loss_and_grads(p, xs, ts)
    big_x = np.concatenate(xs, axis=2)      # not periodic-equivalent, so compare per image
    del big_x
    manual = 0.0
    for x, t in zip(xs, ts):
        manual += cnn.loss(cnn.forward(p, x)[0], t) / 3
    assert abs(loss - manual) < 1e-12
    eps = 1e-6
    flat = p["w1"].reshape(-1)
    i = 17
    old = flat[i]
    flat[i] = old + eps
    lp = cnn.batch_loss_and_grads(p, xs, ts)[0]
    flat[i] = old - eps
    lm = cnn.batch_loss_and_grads(p, xs, ts)[0]
    flat[i] = old
    assert abs((lp - lm) / (2 * eps) - g["w1"].reshape(-1)[i]) < 1e-7


def test_flatten_roundtrip():
    p = cnn.init_params(1)
    th = cnn.flatten(p)
    assert th.size == cnn.NPARAM == 23146
    q = cnn.unflatten(th)
    for k in p:
        assert np.array_equal(p[k], q[k])
