"""Parity of the learned warm start's HIP kernels (through the C ABI) with the
FP64 network oracle.

Inputs of the single-kernel tests are dyadic: activations k/32 and weights
k/1024 with |k| <= 64, so every bf16 operand is exact and every FP32 partial
sum of the forward and backward-data convolutions (at most 27 * 32 products
of size <= 1/8, all multiples of 2^-15) is exact as well.  Those kernels must
therefore match the oracle bit for bit after the same bf16 rounding of the
output.  The weight gradient sums thousands of products per partial; it is
held to the FP32 accumulation bound n * 2^-24 * sum |terms|.  The whole
network stores its hidden activations and gradients in bf16: against an
oracle that rounds at the same points its outputs and gradients agree to a
relative L2 error of 5e-3, against the unrounded FP64 oracle to 1e-1 (deep
weight gradients are sums with heavy cancellation).
"""
import sys

import numpy as np
import pytest

from oracle import nn_oracle as N

pytestmark = pytest.mark.gpu

CIN = [6, 32, 32, 32]
COUT = [32, 32, 32, 3]
CINP = [8, 32, 32, 32]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _torch():
    import torch
    return torch


def dyadic(rng, shape, denom, kmax=64):
    return rng.integers(-kmax, kmax + 1, size=shape).astype(np.float64) / denom


def to_bf16(a):
    torch = _torch()
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to("cuda").to(torch.bfloat16)


def from_dev(t):
    return t.float().cpu().numpy().astype(np.float64)


def param_vector(layers):
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in layers]).astype(np.float32)


def split_params(v):
    out, o = [], 0
    for l in range(4):
        nw = 27 * COUT[l] * CIN[l]
        W = v[o:o + nw].reshape(27, COUT[l], CIN[l]).astype(np.float64)
        o += nw
        b = v[o:o + COUT[l]].astype(np.float64)
        o += COUT[l]
        out.append((W, b))
    return out


def random_layers(rng):
    return [(dyadic(rng, (27, COUT[l], CIN[l]), 1024.0), dyadic(rng, COUT[l], 1024.0)) for l in range(4)]


@pytest.fixture(scope="module")
def net():
    from paper_2111_11538_amd import pf
    n = pf.Net(max_voxels=40000, training=True, seed=7)
    yield n
    n.close()


VOL = (2, 5, 6, 70)      # two volumes; 6 rows = one full and one ragged row tile; 70 = 64 + ragged x segment


@pytest.mark.parametrize("layer", [0, 1, 2, 3])
def test_conv_forward_is_exact(net, layer):
    torch = _torch()
    from paper_2111_11538_amd import pf
    say(f"conv forward layer {layer} on {VOL}")
    rng = np.random.default_rng(100 + layer)
    layers = random_layers(rng)
    net.set_params(param_vector(layers))
    W, b = layers[layer]
    x = dyadic(rng, VOL + (CINP[layer],), 32.0)
    if layer == 0:
        x[..., 6:] = 0.0
    xd = to_bf16(x)
    n, D, H, Wd = VOL
    if layer < 3:
        out = torch.zeros(VOL + (32,), dtype=torch.bfloat16, device="cuda")
    else:
        out = torch.zeros(VOL + (4,), dtype=torch.float32, device="cuda")
    net.layer(pf.PF_NN_OP_FORWARD, layer, xd, None, out, n, D, H, Wd)
    torch.cuda.synchronize()
    got = from_dev(out)
    for s in range(n):
        z = N.conv_forward(x[s, ..., :CIN[layer]], W, b)
        if layer < 3:
            want = N.bf16_round(N.relu(z))
            np.testing.assert_array_equal(got[s], want)
        else:
            np.testing.assert_array_equal(got[s, ..., :3], z.astype(np.float32).astype(np.float64))
            assert np.all(got[s, ..., 3] == 0.0)


@pytest.mark.parametrize("layer", [1, 2, 3])
def test_conv_backward_data_is_exact(net, layer):
    torch = _torch()
    from paper_2111_11538_amd import pf
    say(f"conv backward-data layer {layer} on {VOL}")
    rng = np.random.default_rng(200 + layer)
    layers = random_layers(rng)
    net.set_params(param_vector(layers))
    W, _ = layers[layer]
    cg = 8 if layer == 3 else 32
    dy = dyadic(rng, VOL + (cg,), 32.0)
    xin = dyadic(rng, VOL + (32,), 32.0)          # the layer's input; its sign is the mask
    n, D, H, Wd = VOL
    out = torch.zeros(VOL + (32,), dtype=torch.bfloat16, device="cuda")
    net.layer(pf.PF_NN_OP_BACKWARD_DATA, layer, to_bf16(dy), to_bf16(xin), out, n, D, H, Wd)
    torch.cuda.synchronize()
    got = from_dev(out)
    for s in range(n):
        _, _, dx = N.conv_backward(xin[s], W, dy[s, ..., :COUT[layer]])
        want = N.bf16_round(dx * (xin[s] > 0))
        np.testing.assert_array_equal(got[s], want)


@pytest.mark.parametrize("layer", [0, 1, 2, 3])
def test_conv_backward_weight_within_fp32_bound(net, layer):
    torch = _torch()
    from paper_2111_11538_amd import pf
    say(f"conv backward-weight layer {layer} on {VOL}")
    rng = np.random.default_rng(300 + layer)
    cg = 8 if layer == 3 else 32
    x = dyadic(rng, VOL + (CINP[layer],), 32.0)
    dy = dyadic(rng, VOL + (cg,), 32.0)
    n, D, H, Wd = VOL
    nw = 27 * COUT[layer] * CIN[layer]
    out = torch.zeros(nw + COUT[layer], dtype=torch.float32, device="cuda")
    net.layer(pf.PF_NN_OP_BACKWARD_WEIGHT, layer, to_bf16(x), to_bf16(dy), out, n, D, H, Wd)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64)
    dW = np.zeros((27, COUT[layer], CIN[layer]))
    dWabs = np.zeros_like(dW)
    db = np.zeros(COUT[layer])
    Wz = np.zeros((27, COUT[layer], CIN[layer]))
    for s in range(n):
        a, bb, _ = N.conv_backward(x[s, ..., :CIN[layer]], Wz, dy[s, ..., :COUT[layer]], need_dx=False)
        aa, _, _ = N.conv_backward(np.abs(x[s, ..., :CIN[layer]]), Wz, np.abs(dy[s, ..., :COUT[layer]]), need_dx=False)
        dW += a
        dWabs += aa
        db += bb
    nvox = n * D * H * Wd
    bound = nvox * 2.0 ** -24 * dWabs + 1e-30
    err = np.abs(got[:nw].reshape(dW.shape) - dW)
    assert np.all(err <= bound), float(np.max(err / bound))
    np.testing.assert_allclose(got[nw:], db, rtol=1e-6, atol=1e-6)


def _oracle_net(layers, x, tgt, nsamp, round_bf16):
    """Forward, loss and gradients of one sample in FP64; with round_bf16 the
    hidden activations, the loss gradient and the masked input gradients are
    rounded to bf16 where the kernels store them in bf16."""
    R = N.bf16_round if round_bf16 else (lambda a: a)
    acts = [x]
    h = x
    for l in range(3):
        h = R(N.relu(N.conv_forward(h, *layers[l])))
        acts.append(h)
    out = N.conv_forward(h, *layers[3])
    L, dout = N.relmse(out, tgt)
    g = R(dout / nsamp)
    grads = [None] * 4
    for l in range(3, -1, -1):
        dW, db, dx = N.conv_backward(acts[l], layers[l][0], g, need_dx=l > 0)
        grads[l] = (dW, db)
        if l > 0:
            g = R(dx * (acts[l] > 0))
    return out, L, grads


def test_network_forward_and_gradients_vs_oracle(net):
    torch = _torch()
    say("network forward + loss + backward on (2, 8, 8, 40)")
    rng = np.random.default_rng(400)
    layers = []
    for l in range(4):
        a = np.sqrt(6.0 / (27 * CIN[l])) * (0.3 if l == 3 else 1.0)
        layers.append((rng.uniform(-a, a, (27, COUT[l], CIN[l])), 0.05 * rng.standard_normal(COUT[l])))
    pv = param_vector(layers)
    net.set_params(pv)
    # the kernels multiply by the bf16 images of the weights; biases stay FP32
    oracle_layers = [(N.bf16_round(W), b) for W, b in split_params(pv)]
    vol = (2, 8, 8, 40)
    x = np.zeros(vol + (8,))
    x[..., :6] = N.bf16_round(rng.standard_normal(vol + (6,)))
    tgt = np.zeros(vol + (4,))
    tgt[..., :3] = rng.standard_normal(vol + (3,))
    yd = torch.zeros(vol + (4,), dtype=torch.float32, device="cuda")
    net.forward(to_bf16(x), yd, *vol)
    loss = net.loss(torch.from_numpy(tgt.astype(np.float32)).cuda())
    net.backward()
    g = split_params(net.grads())
    y = yd.cpu().numpy().astype(np.float64)
    for round_bf16, tol in ((True, 5e-3), (False, 1e-1)):
        tot, gw, gb = 0.0, [0.0] * 4, [0.0] * 4
        for s in range(vol[0]):
            out, L, grads = _oracle_net(oracle_layers, x[s, ..., :6], tgt[s, ..., :3], vol[0], round_bf16)
            e = np.linalg.norm(y[s, ..., :3] - out) / np.linalg.norm(out)
            say(f"  bf16 rounding emulated={round_bf16} sample {s}: output rel err {e:.2e}")
            assert e < tol
            tot += L / vol[0]
            for l in range(4):
                gw[l] = gw[l] + grads[l][0]
                gb[l] = gb[l] + grads[l][1]
        assert loss == pytest.approx(tot, rel=tol)
        for l in range(4):
            ew = np.linalg.norm(g[l][0] - gw[l]) / np.linalg.norm(gw[l])
            eb = np.linalg.norm(g[l][1] - gb[l]) / np.linalg.norm(gb[l])
            say(f"  bf16 rounding emulated={round_bf16} layer {l}: dW rel err {ew:.2e}, db rel err {eb:.2e}")
        for l in range(4):
            assert np.linalg.norm(g[l][0] - gw[l]) <= tol * np.linalg.norm(gw[l])
            assert np.linalg.norm(g[l][1] - gb[l]) <= tol * np.linalg.norm(gb[l])


def test_adam_matches_oracle():
    torch = _torch()
    from paper_2111_11538_amd import pf
    say("Adam steps")
    rng = np.random.default_rng(500)
    net = pf.Net(max_voxels=4096, training=True, seed=3)
    try:
        pv = param_vector(random_layers(rng))
        net.set_params(pv)
        vol = (1, 4, 4, 16)
        x = np.zeros(vol + (8,))
        x[..., :6] = dyadic(rng, vol + (6,), 32.0)
        m = np.zeros(pv.size)
        v = np.zeros(pv.size)
        p = pv.astype(np.float64)
        for t in (1, 2, 3):
            net.forward(to_bf16(x), torch.zeros(vol + (4,), dtype=torch.float32, device="cuda"), *vol)
            net.loss(torch.from_numpy(rng.standard_normal(vol + (4,)).astype(np.float32)).cuda())
            net.backward()
            g = net.grads().astype(np.float64)
            net.adam(1e-3)
            p, m, v = N.adam_step(p, g, m, v, t, 1e-3)
            got = net.params().astype(np.float64)
            np.testing.assert_allclose(got, p, rtol=0, atol=1e-6)
            p = got                      # continue from the device's FP32 parameters
    finally:
        net.close()


def test_context_pack_matches_oracle():
    """The FP32 packing inside a mixed-precision context's learned start
    (phi_f, phi_w, the eigenstrain change since the previous solve and the
    previous increment, scaled) against the oracle's packing of the same
    state: bit for bit after the bf16 rounding in > 99.9 % of the entries of
    every channel but the eigenstrain change, which the kernel forms without
    the cancellation of two cube roots (the oracle's plain difference of cube
    roots in FP64 loses every digit where the phase barely moves near 1): that
    channel is held to one bf16 ulp of the exact difference, evaluated
    at 40 digits from the same FP32 phases."""
    torch = _torch()
    from paper_2111_11538_amd import inputs as I, pf
    n = 16
    wl = I.workload("core_shell_3d", n=n)
    say(f"context packing, core_shell_3d {n}^3 mixed")
    c = pf.Context(3, wl.shape, wl.h, wl.dt, wl.params, warm="learned", precision="mixed", plasticity=True,
                   cg_rtol=1e-6)
    c.set_fields(wl.fields)
    net = pf.Net(max_voxels=n ** 3, seed=3)
    try:
        net.attach(c)
        f0 = c.fields(["phi_f", "ux", "uy", "uz"])
        c.step()                       # no previous increment yet: records it
        f1 = c.fields(["phi_f", "phi_w", "ux", "uy", "uz"])
        c.step()                       # packs the state after the first step
        xb = torch.zeros(n ** 3 * 8, dtype=torch.bfloat16, device="cuda")
        net.copy(pf.PF_NN_BUF_INPUT, xb)
        torch.cuda.synchronize()
        got = from_dev(xb).reshape((n, n, n, 8))
    finally:
        c.close()
        net.close()
    low = [(f1[k] - f0[k])[:n, :n, :n] for k in ("ux", "uy", "uz")]
    Om = wl.params.Omega_f
    x, _ = N.pack_inputs(f1["phi_f"], f1["phi_w"], N.eigenstrain(f0["phi_f"], Om), low, Om, wl.h)
    want = np.zeros((n, n, n, 8))
    want[..., :6] = x
    want = N.bf16_round(want)
    assert np.max(np.abs(want[..., 2])) > 0 and np.max(np.abs(want[..., 3:6])) > 0
    plain = [0, 1, 3, 4, 5, 6, 7]
    exact = np.mean(got[..., plain] == want[..., plain])
    assert exact > 0.999, exact
    np.testing.assert_allclose(got[..., plain], want[..., plain], rtol=2.0 ** -7, atol=0)
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 40
    s_o = N.increment_scale(low)

    def eps_t(p):
        p = mpmath.mpf(float(p))
        return mpmath.cbrt(1 - mpmath.mpf(Om) * p ** 3 * (p * (6 * p - 15) + 10)) - 1

    gain = mpmath.mpf(N.EPS_GAIN) * mpmath.mpf(wl.h) / mpmath.mpf(s_o)
    w2 = np.array([float((eps_t(a) - eps_t(b)) * gain) for a, b in zip(f1["phi_f"].ravel(), f0["phi_f"].ravel())])
    g2 = got[..., 2].ravel()
    assert np.max(np.abs(w2)) > 0
    np.testing.assert_allclose(g2, w2, rtol=2.0 ** -7, atol=0)


def test_pack_matches_oracle(net):
    torch = _torch()
    say("pack inputs and targets, ragged crop past the grid")
    rng = np.random.default_rng(600)
    nz, ny, nx = 6, 7, 9
    cell = (nz, ny, nx)
    phi = rng.uniform(0, 1, cell)
    phiw = rng.uniform(0, 1, cell) * (1 - phi)
    phip = np.clip(phi + 1e-3 * rng.standard_normal(cell), 0, 1)
    fshape = [(nz, ny, nx + 1), (nz, ny + 1, nx), (nz + 1, ny, nx)]
    u0 = [rng.standard_normal(s) * 1e-9 for s in fshape]
    u1 = [a + rng.standard_normal(a.shape) * 1e-12 for a in u0]
    u2 = [a + rng.standard_normal(a.shape) * 1e-12 for a in u1]
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    U0, U1, U2 = [list(map(dev, u)) for u in (u0, u1, u2)]
    s = net.increment_scale(U1, U0)
    low = [u1[c][:nz, :ny, :nx] - u0[c][:nz, :ny, :nx] for c in range(3)]
    assert s == pytest.approx(N.increment_scale(low), rel=1e-13)
    origin, size = (2, 3, 4), (5, 5, 8)       # reaches past the grid in every direction
    net.pack(dev(phi), dev(phiw), dev(phip), U1, U0, U2, origin=origin, size=size, slot=1, Omega=0.4, h=7.8125e-8)
    nv = int(np.prod(size))
    xb = torch.zeros(2 * nv * 8, dtype=torch.bfloat16, device="cuda")
    tb = torch.zeros(2 * nv * 4, dtype=torch.float32, device="cuda")
    from paper_2111_11538_amd import pf
    net.copy(pf.PF_NN_BUF_INPUT, xb)
    net.copy(pf.PF_NN_BUF_TARGET, tb)
    torch.cuda.synchronize()
    got = from_dev(xb)[nv * 8:].reshape(size + (8,))
    gt = tb.cpu().numpy().astype(np.float64)[nv * 4:].reshape(size + (4,))
    x, s_o = N.pack_inputs(phi, phiw, N.eigenstrain(phip, 0.4), low, 0.4, 7.8125e-8)
    want = np.zeros(size + (8,))
    wt = np.zeros(size + (4,))
    z0, y0, x0 = origin
    sub = x[z0:z0 + size[0], y0:y0 + size[1], x0:x0 + size[2]]
    want[:sub.shape[0], :sub.shape[1], :sub.shape[2], :6] = sub
    for c in range(3):
        d = (u2[c][:nz, :ny, :nx] - u1[c][:nz, :ny, :nx]) / s_o
        d = d[z0:z0 + size[0], y0:y0 + size[1], x0:x0 + size[2]]
        wt[:d.shape[0], :d.shape[1], :d.shape[2], c] = d
    want = N.bf16_round(want)
    exact = np.mean(got == want)
    assert exact > 0.999, exact
    np.testing.assert_allclose(got, want, rtol=2.0 ** -7, atol=0)
    np.testing.assert_allclose(gt, wt.astype(np.float32).astype(np.float64), rtol=1e-6, atol=1e-7)


def test_network_lives_in_the_callers_workspace():
    """pf_nn_init carves the network out of the caller's workspace: a workspace
    one byte short or misaligned is refused, an exact one works."""
    import ctypes
    torch = _torch()
    from paper_2111_11538_amd import pf
    L = pf.lib()
    cfg = pf.pf_nn_config()
    cfg.max_voxels, cfg.training, cfg.seed = 4096, 1, 3
    nb = L.pf_nn_workspace_bytes(ctypes.byref(cfg))
    ws = torch.empty(nb + 512, dtype=torch.uint8, device="cuda")
    h = ctypes.c_void_p()
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    base = ws.data_ptr()
    assert L.pf_nn_init(ctypes.byref(cfg), ctypes.c_void_p(base), nb - 1, st, ctypes.byref(h)) == pf.PF_ERR_OOM
    assert L.pf_nn_init(ctypes.byref(cfg), ctypes.c_void_p(base + 16), nb, st, ctypes.byref(h)) == pf.PF_ERR_INVALID_ARG
    assert L.pf_nn_init(ctypes.byref(cfg), ctypes.c_void_p(base), nb, st, ctypes.byref(h)) == pf.PF_OK
    w = np.zeros(L.pf_nn_param_count(), dtype=np.float32)
    assert L.pf_nn_weights(h, 0, w.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), w.size) == pf.PF_OK
    assert np.any(w != 0)
    L.pf_nn_destroy(h)
