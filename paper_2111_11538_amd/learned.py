"""Training of the learned warm start (argument marshalling and the training
schedule; every arithmetic step runs in ``libpf.so``).

A trajectory of the plain method supplies one sample per solve t >= 2: the
phase fields before step t, the ferrite phase before step t - 1, the
displacements u[t-2], u[t-1] (previous increment) and u[t] (the target
increment u[t] - u[t-1]).  Training draws random crops of random solves into
a minibatch, runs the network forward, takes the relative mean-square loss,
back-propagates and applies Adam, all through ``pf.Net``.
"""
from __future__ import annotations

import numpy as np

from . import pf

CIN = (6, 32, 32, 32)
COUT = (32, 32, 32, 3)


def record_trajectory(ctx, steps, log=None):
    """Advance ``ctx`` (3D) by ``steps`` steps and keep, per solve, the phase
    fields it used and the displacement it produced (FP64 device tensors)."""
    recs = []
    for t in range(steps):
        phi_f = ctx.get_device("phi_f")
        phi_w = ctx.get_device("phi_w")
        st = ctx.step()
        u = tuple(ctx.get_device(n) for n in ("ux", "uy", "uz"))
        recs.append({"phi_f": phi_f, "phi_w": phi_w, "u": u, "cg_iters": st["cg_iters"]})
        if log:
            log(f"[record] step {t}: {st['cg_iters']} CG iterations")
    return recs


def _split(v):
    out, o = [], 0
    for l in range(4):
        nw = 27 * COUT[l] * CIN[l]
        out.append([v[o:o + nw].reshape(27, COUT[l], CIN[l]), v[o + nw:o + nw + COUT[l]]])
        o += nw + COUT[l]
    return out


def _join(layers):
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in layers]).astype(np.float32)


def init_extrapolation(net, keep_scale=0.1):
    """Start from weights whose output equals the previous increment (input
    channels 3..5): channels 0..5 of the hidden layers carry its positive and
    negative parts through the ReLUs at the centre tap; the remaining weights
    keep the library's random initialisation (scaled by ``keep_scale`` where
    they feed the carried channels or the output).  The untrained network
    thus proposes the linear extrapolation u[t-1] + (u[t-1] - u[t-2])."""
    L = _split(net.params().astype(np.float64))
    c = 13                                   # centre tap
    W0, b0 = L[0]
    W0[:, :6, :] = 0.0
    b0[:6] = 0.0
    for k in range(3):
        W0[c, 2 * k, 3 + k] = 1.0
        W0[c, 2 * k + 1, 3 + k] = -1.0
    for l in (1, 2):
        W, b = L[l]
        W[:, :6, :] = 0.0
        b[:6] = 0.0
        for k in range(6):
            W[c, k, k] = 1.0
    W3, b3 = L[3]
    W3 *= keep_scale
    b3[:] = 0.0
    for k in range(3):
        W3[:, k, :6] = 0.0
        W3[c, k, 2 * k] = 1.0
        W3[c, k, 2 * k + 1] = -1.0
    net.set_params(_join(L))


def train(net, recs, iters, Omega, h, crop=(32, 32, 32), batch=8, lr=1e-4, seed=0, log=None, log_every=25,
          t_min=2, val_recs=None, eval_every=25):
    """Adam on random crops of the recorded solves t >= t_min; returns the
    loss history.  With ``val_recs`` the whole-grid loss on those solves is
    evaluated every ``eval_every`` iterations (and before the first) and the
    network keeps the best parameters seen (early stopping)."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = recs[0]["phi_f"].shape
    cz, cy, cx = (min(crop[0], nz), min(crop[1], ny), min(crop[2], nx))
    losses = []
    best, best_params = None, None
    if val_recs is not None:
        best = float(np.mean(evaluate(net, val_recs, Omega, h)))
        best_params = net.params()
        if log:
            log(f"[train] held-out loss at start: {best:.4e}")
    for it in range(iters):
        for b in range(batch):
            t = int(rng.integers(max(2, t_min), len(recs)))
            r2, r1, r0 = recs[t], recs[t - 1], recs[t - 2]
            net.increment_scale(r1["u"], r0["u"])
            origin = (int(rng.integers(0, nz - cz + 1)), int(rng.integers(0, ny - cy + 1)),
                      int(rng.integers(0, nx - cx + 1)))
            net.pack(r2["phi_f"], r2["phi_w"], r1["phi_f"], r1["u"], r0["u"], r2["u"], origin=origin,
                     size=(cz, cy, cx), slot=b, Omega=Omega, h=h)
        net.forward(None, None, batch, cz, cy, cx)
        loss = net.loss()
        net.backward()
        net.adam(lr)
        losses.append(loss)
        if log and (it % log_every == 0 or it == iters - 1):
            log(f"[train] iter {it}: loss {loss:.4e}")
        if val_recs is not None and ((it + 1) % eval_every == 0 or it == iters - 1):
            v = float(np.mean(evaluate(net, val_recs, Omega, h)))
            if v < best:
                best, best_params = v, net.params()
            if log:
                log(f"[train] iter {it + 1}: held-out loss {v:.4e} (best {best:.4e})")
    if best_params is not None:
        net.set_params(best_params)
    return losses


def evaluate(net, recs, Omega, h):
    """Relative mean-square error of the whole-grid prediction for every
    recorded solve t >= 2 (the loss of the network on full grids)."""
    nz, ny, nx = recs[0]["phi_f"].shape
    out = []
    for t in range(2, len(recs)):
        r2, r1, r0 = recs[t], recs[t - 1], recs[t - 2]
        net.increment_scale(r1["u"], r0["u"])
        net.pack(r2["phi_f"], r2["phi_w"], r1["phi_f"], r1["u"], r0["u"], r2["u"], Omega=Omega, h=h)
        net.forward(None, None, 1, nz, ny, nx)
        out.append(net.loss())
    return out


def evaluate_crops(net, recs, Omega, h, crop=(32, 32, 32)):
    """Loss of the network on the centre crop of every solve t >= 2 of ``recs``."""
    nz, ny, nx = recs[0]["phi_f"].shape
    cz, cy, cx = (min(crop[0], nz), min(crop[1], ny), min(crop[2], nx))
    origin = ((nz - cz) // 2, (ny - cy) // 2, (nx - cx) // 2)
    out = []
    for t in range(2, len(recs)):
        r2, r1, r0 = recs[t], recs[t - 1], recs[t - 2]
        net.increment_scale(r1["u"], r0["u"])
        net.pack(r2["phi_f"], r2["phi_w"], r1["phi_f"], r1["u"], r0["u"], r2["u"], origin=origin, size=(cz, cy, cx),
                 Omega=Omega, h=h)
        net.forward(None, None, 1, cz, cy, cx)
        out.append(net.loss())
    return out
