"""Pins of the FP64 network oracle: shift identities of the convolution, a
brute-force convolution, finite-difference gradients of the whole network and
of the loss, closed forms of Adam and of the packing."""
import numpy as np
import pytest

from oracle import nn_oracle as N


def _rng(seed):
    return np.random.default_rng(seed)


def test_center_tap_identity_is_identity():
    x = _rng(1).standard_normal((4, 5, 6, 3))
    W = np.zeros((27, 3, 3))
    W[13] = np.eye(3)                       # tap (0, 0, 0)
    b = np.array([0.5, -1.0, 2.0])
    np.testing.assert_array_equal(N.conv_forward(x, W, b), x + b)


@pytest.mark.parametrize("d", [(0, 0, 1), (0, -1, 0), (1, 0, 0), (-1, 1, -1)])
def test_single_tap_is_a_zero_padded_shift(d):
    x = _rng(2).standard_normal((4, 5, 6, 2))
    t = N.TAPS.index(d)
    W = np.zeros((27, 2, 2))
    W[t] = np.eye(2)
    y = N.conv_forward(x, W, np.zeros(2))
    D, H, Wd, _ = x.shape
    for z in range(D):
        for yy in range(H):
            for xx in range(Wd):
                zs, ys, xs = z + d[0], yy + d[1], xx + d[2]
                inside = 0 <= zs < D and 0 <= ys < H and 0 <= xs < Wd
                want = x[zs, ys, xs] if inside else np.zeros(2)
                np.testing.assert_array_equal(y[z, yy, xx], want)


def test_conv_matches_brute_force_loops():
    r = _rng(3)
    x = r.standard_normal((3, 4, 5, 2))
    W = r.standard_normal((27, 3, 2))
    b = r.standard_normal(3)
    y = N.conv_forward(x, W, b)
    D, H, Wd, Ci = x.shape
    ref = np.zeros((D, H, Wd, 3))
    for z in range(D):
        for yy in range(H):
            for xx in range(Wd):
                for o in range(3):
                    s = b[o]
                    for kz in range(3):
                        for ky in range(3):
                            for kx in range(3):
                                zs, ys, xs = z + kz - 1, yy + ky - 1, xx + kx - 1
                                if 0 <= zs < D and 0 <= ys < H and 0 <= xs < Wd:
                                    for i in range(Ci):
                                        s += W[kz * 9 + ky * 3 + kx, o, i] * x[zs, ys, xs, i]
                    ref[z, yy, xx, o] = s
    np.testing.assert_allclose(y, ref, rtol=1e-13, atol=1e-13)


def _small_net(seed, cin=6, width=4, cout=3, layers=4):
    r = _rng(seed)
    chans = [cin] + [width] * (layers - 1) + [cout]
    return [(r.standard_normal((27, chans[l + 1], chans[l])) / np.sqrt(27 * chans[l]),
             0.1 * r.standard_normal(chans[l + 1])) for l in range(layers)]


def test_network_gradients_match_central_differences():
    params = _small_net(4)
    r = _rng(5)
    x = r.standard_normal((5, 4, 6, 6))
    target = r.standard_normal((5, 4, 6, 3))
    out, cache = N.net_forward(params, x)
    # no pre-activation near a ReLU kink, so central differences are smooth
    assert min(np.min(np.abs(z)) for _, z in cache[:-1]) > 1e-5
    loss, dout = N.relmse(out, target)
    grads, dx = N.net_backward(params, cache, dout)
    eps = 1e-6

    def L(ps, xx):
        return N.relmse(N.net_forward(ps, xx)[0], target)[0]

    picks = r.integers(0, 10 ** 6, size=(12, 4))
    for l in range(4):
        W, b = params[l]
        for q in picks[:6]:
            idx = (q[0] % 27, q[1] % W.shape[1], q[2] % W.shape[2])
            Wp, Wm = W.copy(), W.copy()
            Wp[idx] += eps
            Wm[idx] -= eps
            pp = [(Wp if k == l else p[0], p[1]) for k, p in enumerate(params)]
            pm = [(Wm if k == l else p[0], p[1]) for k, p in enumerate(params)]
            fd = (L(pp, x) - L(pm, x)) / (2 * eps)
            assert abs(fd - grads[l][0][idx]) <= 1e-6 * max(1.0, abs(fd)), (l, idx, fd, grads[l][0][idx])
        o = picks[6][0] % b.size
        bp, bm = b.copy(), b.copy()
        bp[o] += eps
        bm[o] -= eps
        fd = (L([(p[0], bp if k == l else p[1]) for k, p in enumerate(params)], x)
              - L([(p[0], bm if k == l else p[1]) for k, p in enumerate(params)], x)) / (2 * eps)
        assert abs(fd - grads[l][1][o]) <= 1e-6 * max(1.0, abs(fd))
    for q in picks[6:]:
        idx = tuple(int(q[k] % x.shape[k]) for k in range(4))
        xp, xm = x.copy(), x.copy()
        xp[idx] += eps
        xm[idx] -= eps
        fd = (L(params, xp) - L(params, xm)) / (2 * eps)
        assert abs(fd - dx[idx]) <= 1e-6 * max(1.0, abs(fd))


def test_relmse_closed_forms_and_gradient():
    r = _rng(6)
    q = r.standard_normal((3, 3, 3, 2))
    assert N.relmse(q, q)[0] == 0.0
    assert N.relmse(np.zeros_like(q), q)[0] == pytest.approx(1.0, rel=1e-15)
    assert N.relmse(2 * q, q)[0] == pytest.approx(1.0, rel=1e-15)
    p = r.standard_normal(q.shape)
    _, g = N.relmse(p, q)
    eps = 1e-7
    for k in range(5):
        idx = tuple(int(v) for v in r.integers(0, 3, size=3)) + (k % 2,)
        pp, pm = p.copy(), p.copy()
        pp[idx] += eps
        pm[idx] -= eps
        fd = (N.relmse(pp, q)[0] - N.relmse(pm, q)[0]) / (2 * eps)
        assert fd == pytest.approx(g[idx], rel=1e-6, abs=1e-9)


def test_adam_constant_gradient_moves_by_the_learning_rate():
    # with a constant gradient the bias-corrected moments are g and g^2,
    # so every step moves each parameter by lr against the sign of g
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([3.0, -0.25, 1e-2])
    m = np.zeros(3)
    v = np.zeros(3)
    for t in range(1, 6):
        p2, m, v = N.adam_step(p, g, m, v, t, lr=1e-3, eps=0.0)
        np.testing.assert_allclose(p2 - p, -1e-3 * np.sign(g), rtol=1e-12)
        p = p2


def test_adam_minimises_a_quadratic():
    p = np.array([10.0])
    m = np.zeros(1)
    v = np.zeros(1)
    for t in range(1, 3001):
        p, m, v = N.adam_step(p, p - 3.0, m, v, t, lr=0.05)
    assert abs(p[0] - 3.0) < 1e-3


def test_pack_closed_forms():
    shape = (3, 4, 5)
    r = _rng(7)
    phi = r.uniform(0, 1, shape)
    assert np.all(N.eigenstrain(np.zeros(shape), 0.4) == 0.0)
    np.testing.assert_allclose(N.eigenstrain(np.ones(shape), 0.4), 0.6 ** (1 / 3) - 1, rtol=1e-15)
    assert np.all(N.eigenstrain(phi, 0.0) == 0.0)
    c = -2.5e-12
    du = [np.full(shape, c), np.full(shape, c), np.full(shape, -c)]
    eT = N.eigenstrain(phi, 0.4)
    x, s = N.pack_inputs(phi, 1 - phi, eT, du, 0.4, 7.8e-8)
    assert s == pytest.approx(abs(c), rel=1e-14)
    np.testing.assert_allclose(x[..., 3], -1.0)
    np.testing.assert_allclose(x[..., 5], 1.0)
    np.testing.assert_array_equal(x[..., 2], 0.0)          # no eigenstrain change
    np.testing.assert_array_equal(x[..., 0], phi)
    y = np.ones(shape + (3,))
    out = N.unpack_increment(y, 2.0)
    assert np.all(out[0][:, :, 0] == 0) and np.all(out[0][:, :, 1:] == 2.0)
    assert np.all(out[1][:, 0, :] == 0) and np.all(out[1][:, 1:, :] == 2.0)
    assert np.all(out[2][0] == 0) and np.all(out[2][1:] == 2.0)


def test_bf16_rounding_ties_to_even():
    one = 1.0
    assert N.bf16_round(one) == 1.0
    assert N.bf16_round(one + 2.0 ** -8) == 1.0                      # tie, even below
    assert N.bf16_round(one + 3 * 2.0 ** -8) == one + 2.0 ** -6       # tie, even above
    assert N.bf16_round(one + 2.0 ** -8 + 2.0 ** -20) == one + 2.0 ** -7
    assert N.bf16_round(-3.0) == -3.0
