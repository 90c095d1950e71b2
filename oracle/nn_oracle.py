"""FP64 reference of the learned warm start: a stack of 3x3x3 convolutions,
its backward pass, the relative mean-square loss, Adam, and the packing of the
simulation state into network inputs and of network outputs into a
displacement increment on the staggered faces.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark.  The product path never imports it.

The network is an extension of the method (the paper solves mechanics without
any learned component); its definition here is the specification the GPU
kernels are checked against.

Conventions
-----------
* Tensors are channel-last: ``x[z, y, x, c]``.
* A layer is a 'same' 3x3x3 cross-correlation with zero padding,
  ``y[v, o] = b[o] + sum_t sum_i W[t, o, i] * x[v + d(t), i]`` with tap
  ``t = 9 (dz + 1) + 3 (dy + 1) + (dx + 1)`` and ``d(t) = (dz, dy, dx)``.
* ReLU follows every layer but the last, which is linear.
* Loss of one sample: ``sum (p - q)^2 / sum q^2`` (relative mean-square error;
  the denominator is replaced by 1 when the target is identically zero).
* Adam with bias correction (Kingma and Ba, 2015), applied elementwise.

Every routine is written for clarity; numpy's tensordot is the only library
step (a plain contraction over the listed axes).
"""
from __future__ import annotations

import numpy as np

TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def shifted(x, d):
    """``out[z, y, x] = x[z + dz, y + dy, x + dx]``, zero where that is outside."""
    out = np.zeros_like(x)
    src, dst = [], []
    for ax, o in enumerate(d):
        n = x.shape[ax]
        lo, hi = max(0, -o), n - max(0, o)          # destination range
        dst.append(slice(lo, hi))
        src.append(slice(lo + o, hi + o))
    out[tuple(dst)] = x[tuple(src)]
    return out


def conv_forward(x, W, b):
    """Pre-activation of one layer.  x: (D, H, W, Cin), W: (27, Cout, Cin), b: (Cout,)."""
    y = np.zeros(x.shape[:3] + (W.shape[1],), dtype=np.float64) + b
    for t, d in enumerate(TAPS):
        y += np.tensordot(shifted(x, d), W[t], axes=([3], [1]))
    return y


def conv_backward(x, W, dy, need_dx=True):
    """Gradients of ``sum(dy * conv_forward(x, W, b))`` with respect to W, b and x."""
    dW = np.zeros_like(W, dtype=np.float64)
    dx = np.zeros_like(x, dtype=np.float64) if need_dx else None
    for t, d in enumerate(TAPS):
        dW[t] = np.tensordot(dy, shifted(x, d), axes=([0, 1, 2], [0, 1, 2]))
        if need_dx:
            # x[v + d] fed y[v], so its gradient is dy[v] W_t placed at v + d
            dx += shifted(np.tensordot(dy, W[t], axes=([3], [0])), tuple(-o for o in d))
    db = dy.sum(axis=(0, 1, 2))
    return dW, db, dx


def relu(z):
    return np.maximum(z, 0.0)


def net_forward(params, x):
    """params: list of (W, b).  Returns the output and, per layer, (input, pre-activation)."""
    cache = []
    h = x
    for l, (W, b) in enumerate(params):
        z = conv_forward(h, W, b)
        cache.append((h, z))
        h = relu(z) if l < len(params) - 1 else z
    return h, cache


def net_backward(params, cache, dout):
    """Gradients of ``sum(dout * output)``: list of (dW, db) and the input gradient."""
    grads = [None] * len(params)
    g = dout
    for l in range(len(params) - 1, -1, -1):
        h, z = cache[l]
        if l < len(params) - 1:
            g = g * (z > 0.0)
        dW, db, dx = conv_backward(h, params[l][0], g, need_dx=True)
        grads[l] = (dW, db)
        g = dx
    return grads, g


def relmse(pred, target):
    """Loss of one sample and its gradient with respect to pred."""
    den = float(np.sum(target * target))
    den = den if den > 0.0 else 1.0
    diff = pred - target
    return float(np.sum(diff * diff)) / den, 2.0 * diff / den


def adam_step(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update at step t (1-based); returns new (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


# ---------------------------------------------------------------------------
# Packing between the simulation state and the network (3D).
# ---------------------------------------------------------------------------
C_IN = 6          # phi_f, phi_w, scaled eigenstrain change, scaled previous increment (3 faces)
C_OUT = 3         # increment on the x, y, z low faces of each cell
EPS_GAIN = 32.0   # the eigenstrain change enters as d(eps_T) * EPS_GAIN * h / s


def eigenstrain(phi_f, Omega):
    """Small-strain volumetric eigenstrain cbrt(1 - Omega h(phi_f)) - 1, h the quintic interpolation."""
    hf = phi_f ** 3 * (6.0 * phi_f ** 2 - 15.0 * phi_f + 10.0)
    return np.cbrt(1.0 - Omega * hf) - 1.0


def increment_scale(du_prev):
    """s = root mean square of the previous increment over all stored faces."""
    tot = sum(float(np.sum(d.astype(np.float64) ** 2)) for d in du_prev)
    n = sum(d.size for d in du_prev)
    return (tot / n) ** 0.5


def pack_inputs(phi_f, phi_w, eT_prev, du_prev, Omega, h):
    """Network input (nz, ny, nx, 6) and the scale s.  Arrays are (nz, ny, nx);
    du_prev holds the x, y, z face increments indexed by the cell on their high side."""
    s = increment_scale(du_prev)
    inv = 1.0 / s if s > 0.0 else 0.0
    x = np.zeros(phi_f.shape + (C_IN,), dtype=np.float64)
    x[..., 0] = phi_f
    x[..., 1] = phi_w
    x[..., 2] = (eigenstrain(phi_f, Omega) - eT_prev) * (EPS_GAIN * h * inv)
    for c in range(3):
        x[..., 3 + c] = du_prev[c] * inv
    return x, s


def unpack_increment(y, s):
    """Face increments from the network output: s * y, with the low boundary
    faces (fixed by the rollers) set to zero."""
    out = []
    for c in range(3):
        d = s * y[..., c]
        d = d.copy()
        if c == 0:
            d[:, :, 0] = 0.0
        elif c == 1:
            d[:, 0, :] = 0.0
        else:
            d[0, :, :] = 0.0
        out.append(d)
    return out


def bf16_round(a):
    """Round float64 values to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = ((u + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    return u.view(np.float32).astype(np.float64)
