"""FP64 oracle of the finite-strain mechanics on a voxel grid (Bai et al.,
arXiv:2111.11538, Sec. 2.2 and Sec. 2.4): trilinear (bilinear in 2D, plane
strain) finite elements on the cells, nodal displacements, 2^d Gauss points
per cell, the energy and stresses of `fs_oracle` at every Gauss point
(F = F_E F_T F_P, Eq. 9-14; the first Piola-Kirchhoff stress as the energy's
derivative, Eq. 31 with reading R34), equilibrium Div P = 0 (Eq. 29, momentum
line) under rollers solved by Newton's method with the exact sparse tangent
and a direct sparse solve, then the J2 return in the Mandel stress (Eq. 25,
34) at every Gauss point, the elastic driving forces d psi / d phi (Eq. 33)
averaged over each cell and the largest von Mises stress of the Cauchy
stress.

The whole-array functions below are the batched forms of the pointwise ones
in `fs_oracle` (a test checks them against each other entry by entry); the
tangent comes from complex-step derivatives of the batched stress, so it
affects only how fast Newton converges, never the solution, which the
residual alone defines.

TEST INFRASTRUCTURE ONLY: imported by the tests; nothing in the product path
loads it.  It shares no code with the HIP library.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

G1, G2 = 0.5 - 0.5 / math.sqrt(3.0), 0.5 + 0.5 / math.sqrt(3.0)     # Gauss points on [0, 1]


# ---------------------------------------------------------------------------
# batched constitutive law (leading axes broadcast; complex input allowed)
# ---------------------------------------------------------------------------
def h(x):
    return x ** 3 * (6 * x ** 2 - 15 * x + 10)


def _moduli(phi_f, phi_w, p):
    """Phase-weighted K and G (Eq. 14 with the weights h of ferrite, gas, wuestite)."""
    w = (h(phi_f), h(1.0 - phi_f - phi_w), h(phi_w))
    Kb = sum(w[a] * p.K[a] for a in range(3))
    Gb = sum(w[a] * p.G[a] for a in range(3))
    return Kb, Gb


def _elastic_part(F, phi_f, Fp, p):
    dT = 1.0 - h(phi_f) * p.Omega_f
    c = dT ** (-1.0 / 3.0)
    FE = c[..., None, None] * (F @ np.linalg.inv(Fp))
    return dT, c, FE


def energy_b(F, phi_f, phi_w, Fp, p):
    """psi_ela per point: d_T sum_a h_a [K_a/4 (J^2 - 1 - 2 ln J) + G_a/2 (J^(-2/3) tr C - 3)]."""
    dT, _, FE = _elastic_part(F, phi_f, Fp, p)
    Kb, Gb = _moduli(phi_f, phi_w, p)
    J = np.linalg.det(FE)
    trC = np.sum(FE * FE, axis=(-2, -1))
    return dT * (0.25 * Kb * (J * J - 1.0 - 2.0 * np.log(J)) + 0.5 * Gb * (J ** (-2.0 / 3.0) * trC - 3.0))


def piola_b(F, phi_f, phi_w, Fp, p):
    """d psi / d F per point."""
    dT, c, FE = _elastic_part(F, phi_f, Fp, p)
    Kb, Gb = _moduli(phi_f, phi_w, p)
    J = np.linalg.det(FE)
    trC = np.sum(FE * FE, axis=(-2, -1))
    FEiT = np.swapaxes(np.linalg.inv(FE), -1, -2)
    S = ((0.5 * Kb * (J * J - 1.0))[..., None, None] * FEiT
         + (Gb * J ** (-2.0 / 3.0))[..., None, None] * (FE - (trC / 3.0)[..., None, None] * FEiT))
    return (dT * c)[..., None, None] * (S @ np.swapaxes(np.linalg.inv(Fp), -1, -2))


def mandel_b(F, phi_f, phi_w, Fp, p):
    """M = d_T sum_a h_a [K_a/2 (J^2 - 1) I + G_a J^(-2/3) (C_E - tr C_E / 3 I)]."""
    dT, _, FE = _elastic_part(F, phi_f, Fp, p)
    Kb, Gb = _moduli(phi_f, phi_w, p)
    J = np.linalg.det(FE)
    C = np.swapaxes(FE, -1, -2) @ FE
    trC = np.trace(C, axis1=-2, axis2=-1)
    I3 = np.eye(3)
    return dT[..., None, None] * ((0.5 * Kb * (J * J - 1.0))[..., None, None] * I3
                                  + (Gb * J ** (-2.0 / 3.0))[..., None, None] * (C - (trC / 3.0)[..., None, None] * I3))


def dev_b(A):
    return A - (np.trace(A, axis1=-2, axis2=-1) / 3.0)[..., None, None] * np.eye(3)


def expm_sym_b(A):
    """exp of symmetric matrices by their eigen-decomposition."""
    lam, Q = np.linalg.eigh(0.5 * (A + np.swapaxes(A, -1, -2)))
    return (Q * np.exp(lam)[..., None, :]) @ np.swapaxes(Q, -1, -2)


def return_map_b(F, phi_f, phi_w, Fp_n, epsP_n, p, tol=1e-13):
    """The pointwise return map of `fs_oracle.return_map` on every point at
    once, each point taking the same steps: the principal frame of the trial
    elastic state, the deviatoric log stretches, the yield test, then for each
    trial dl the Newton solve of e + dl s(e) / Y(dl) = e_tr (to 1e-15) and the
    bracket-and-bisection on |s(e(dl))| - Y(dl).  Returns F_P, eps_P, dl."""
    r23 = math.sqrt(2.0 / 3.0)
    dT, _, FE = _elastic_part(F, phi_f, Fp_n, p)
    c, Q = np.linalg.eigh(np.swapaxes(FE, -1, -2) @ FE)
    lnJ = 0.5 * np.sum(np.log(c), axis=-1)
    etr = 0.5 * np.log(c) - (lnJ / 3.0)[..., None]
    _, Gb = _moduli(phi_f, phi_w, p)
    k = dT * Gb

    def s_of(e, kk):
        x = np.exp(2.0 * e)
        return kk[..., None] * (x - x.mean(axis=-1, keepdims=True))

    def Y(dl, e0):
        return r23 * (p.sigY + p.Hhard * (e0 + dl))

    ytr = np.sqrt(np.sum(s_of(etr, k) ** 2, axis=-1)) - Y(0.0, epsP_n)
    Fp = Fp_n.copy()
    epsP = epsP_n.copy()
    dl = np.zeros_like(epsP_n)
    idx = np.nonzero(ytr > 0.0)
    if len(idx[0]) == 0:
        return Fp, epsP, dl
    et, ky, ey, Qy, Fpy = etr[idx], k[idx], epsP_n[idx], Q[idx], Fp_n[idx]

    def e_of(d):
        a = d / Y(d, ey)
        e = et.copy()
        todo = np.ones(len(d), bool)
        for _ in range(60):
            x = np.exp(2.0 * e)
            G = e + (a * ky)[:, None] * (x - x.mean(axis=-1, keepdims=True)) - et
            todo = np.max(np.abs(G), axis=-1) > 1e-15
            if not np.any(todo):
                break
            Jm = np.eye(3) + (a * ky)[:, None, None] * (2.0 * x[:, :, None] * np.eye(3) - (2.0 / 3.0) * x[:, None, :])
            step = np.linalg.solve(Jm, G[..., None])[..., 0]
            e = np.where(todo[:, None], e - step, e)
        return e

    def phi(d):
        return np.sqrt(np.sum(s_of(e_of(d), ky) ** 2, axis=-1)) - Y(d, ey)

    n = len(idx[0])
    lo, hi = np.zeros(n), np.full(n, 1e-3)
    grow = phi(hi) > 0.0
    while np.any(grow):
        lo = np.where(grow, hi, lo)
        hi = np.where(grow, 2.0 * hi, hi)
        grow = grow & (phi(hi) > 0.0)
    active = np.ones(n, bool)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        pos = phi(mid) > 0.0
        lo = np.where(active & pos, mid, lo)
        hi = np.where(active & ~pos, mid, hi)
        active &= ~(hi - lo <= tol * np.maximum(hi, 1e-300))
        if not np.any(active):
            break
    d = 0.5 * (lo + hi)
    sv = s_of(e_of(d), ky)
    nv = sv / np.sqrt(np.sum(sv * sv, axis=-1, keepdims=True))
    Fp[idx] = ((Qy * np.exp(d[:, None] * nv)[:, None, :]) @ np.swapaxes(Qy, -1, -2)) @ Fpy
    epsP[idx] = ey + d
    dl[idx] = d
    return Fp, epsP, dl


# ---------------------------------------------------------------------------
# finite elements on the voxel grid
# ---------------------------------------------------------------------------
class FEGrid:
    """Cells `shape` ((ny, nx) or (nz, ny, nx)), nodes at the cell corners,
    displacement u[c] on the nodes (c = 0 .. d-1 for x, y, z), bilinear or
    trilinear shape functions N_a on each cell (local node a: bit 0 the x
    offset, bit 1 y, bit 2 z), Gauss points with the same bit order at
    1/2 -+ 1/(2 sqrt 3) of the cell, weight h^d / 2^d.  Rollers: u_x = 0 on
    the nodes of the x = 0 and x = L faces, likewise y and z."""

    def __init__(self, dim, shape, h_cell, params, phi_f, phi_w):
        self.dim, self.shape, self.h, self.p = dim, tuple(shape), h_cell, params
        self.nodes = tuple(n + 1 for n in self.shape)
        self.na = 1 << dim
        self.ngp = 1 << dim
        self.w = h_cell ** dim / self.ngp
        self.phi_f = np.asarray(phi_f, float)
        self.phi_w = np.asarray(phi_w, float)
        # dN_a / dX at Gauss point g: dN[g, a, c]
        dN = np.zeros((self.ngp, self.na, 3))
        for gq in range(self.ngp):
            xi = [G2 if (gq >> c) & 1 else G1 for c in range(dim)]
            for a in range(self.na):
                for c in range(dim):
                    v = 1.0 / h_cell if (a >> c) & 1 else -1.0 / h_cell
                    for c2 in range(dim):
                        if c2 != c:
                            v *= xi[c2] if (a >> c2) & 1 else 1.0 - xi[c2]
                    dN[gq, a, c] = v
        self.dN = dN
        fixed = np.zeros((dim,) + self.nodes, bool)
        for c in range(dim):
            ax = dim - 1 - c                       # array axis of coordinate c
            sl = [slice(None)] * dim
            sl[ax] = 0
            fixed[(c,) + tuple(sl)] = True
            sl[ax] = -1
            fixed[(c,) + tuple(sl)] = True
        self.fixed = fixed
        self.free = ~fixed

    # element-local views -----------------------------------------------------
    def _node_slice(self, a):
        """Array slice of the nodes that are local node a of every cell."""
        off = [(a >> c) & 1 for c in range(self.dim)]            # x, y, z offsets
        return tuple(slice(off[self.dim - 1 - ax], off[self.dim - 1 - ax] + self.shape[ax])
                     for ax in range(self.dim))

    def deformation_gradient(self, u):
        """F at every Gauss point: F[..cells.., g, 3, 3] = I + sum_a u_a (x) grad N_a."""
        F = np.zeros(self.shape + (self.ngp, 3, 3), dtype=u.dtype)
        F[...] = np.eye(3)
        for a in range(self.na):
            ua = np.stack([u[c][self._node_slice(a)] for c in range(self.dim)], axis=-1)      # cells x d
            for gq in range(self.ngp):
                F[..., gq, :self.dim, :self.dim] += ua[..., :, None] * self.dN[gq, a, :self.dim][None, :]
        return F

    def _cellwise(self, v):
        return np.broadcast_to(v[..., None], self.shape + (self.ngp,))

    def energy(self, u, Fp):
        F = self.deformation_gradient(u)
        psi = energy_b(F, self._cellwise(self.phi_f), self._cellwise(self.phi_w), Fp, self.p)
        return self.w * np.sum(psi)

    def forces(self, P):
        """Nodal forces sum over cells and Gauss points of w P grad N_a."""
        R = np.zeros((self.dim,) + self.nodes, dtype=P.dtype)
        for a in range(self.na):
            sl = self._node_slice(a)
            for gq in range(self.ngp):
                f = self.w * np.einsum("...ij,j->...i", P[..., gq, :self.dim, :self.dim], self.dN[gq, a, :self.dim])
                for c in range(self.dim):
                    R[c][sl] += f[..., c]
        return R

    def residual(self, u, Fp):
        """d Pi / d u on the free degrees of freedom (zero on the fixed ones)."""
        F = self.deformation_gradient(u)
        P = piola_b(F, self._cellwise(self.phi_f), self._cellwise(self.phi_w), Fp, self.p)
        R = self.forces(P)
        R[self.fixed] = 0.0
        return R

    def tangent(self, u, Fp):
        """Sparse d R / d u over all degrees of freedom, by complex-step
        derivatives of the stress per cell, Gauss point and in-plane F entry."""
        d = self.dim
        F = self.deformation_gradient(u)
        pf, pw = self._cellwise(self.phi_f), self._cellwise(self.phi_w)
        step = 1e-30
        A = np.zeros(F.shape[:-2] + (d, d, d, d))        # dP_iJ / dF_kL
        for k in range(d):
            for L in range(d):
                Fc = F.astype(complex)
                Fc[..., k, L] += 1j * step
                A[..., :, :, k, L] = (piola_b(Fc, pf, pw, Fp, self.p).imag / step)[..., :d, :d]
        nn = int(np.prod(self.nodes))
        nid = np.arange(nn).reshape(self.nodes)
        rows, cols, vals = [], [], []
        for a in range(self.na):
            ia = nid[self._node_slice(a)].ravel()
            for b in range(self.na):
                ib = nid[self._node_slice(b)].ravel()
                Kab = np.zeros(self.shape + (d, d))
                for gq in range(self.ngp):
                    Kab += self.w * np.einsum("j,...ijkl,l->...ik", self.dN[gq, a, :d], A[..., gq, :, :, :, :],
                                              self.dN[gq, b, :d])
                for i in range(d):
                    for k in range(d):
                        rows.append(i * nn + ia)
                        cols.append(k * nn + ib)
                        vals.append(Kab[..., i, k].ravel())
        rows, cols, vals = np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)
        return sp.csr_matrix((vals, (rows, cols)), shape=(d * nn, d * nn))

    def solve(self, u0, Fp, rtol=1e-13, max_iter=50):
        """Newton on R(u) = 0 (free dofs) from u0, with a halving line search
        on ||R||; stop at ||R|| <= rtol ||R(0)||; u = 0 when there is no load.
        Returns u, iterations, ||R|| / ||R(0)||."""
        u = np.array(u0, float)
        u[self.fixed] = 0.0
        r0 = np.linalg.norm(self.residual(np.zeros_like(u), Fp))
        # without transformation misfit P(I) vanishes only up to rounding: a
        # load below 1e-12 of (K + G)_max h^(d-1) sqrt(dofs) is no load
        zero_load = 1e-12 * max(self.p.K[a] + self.p.G[a] for a in range(3)) * self.h ** (self.dim - 1) \
            * math.sqrt(u.size)
        if r0 <= zero_load:
            return np.zeros_like(u), 0, 0.0
        free = self.free.ravel()
        R = self.residual(u, Fp)
        nr = np.linalg.norm(R)
        it = 0
        while nr > rtol * r0 and it < max_iter:
            K = self.tangent(u, Fp)
            Kf = K[free][:, free]
            du = np.zeros(u.size)
            du[free] = spla.spsolve(Kf.tocsc(), -R.ravel()[free])
            du = du.reshape(u.shape)
            s = 1.0
            for _ in range(30):
                un = u + s * du
                Rn = self.residual(un, Fp)
                nrn = np.linalg.norm(Rn)
                if np.isfinite(nrn) and nrn < nr:
                    break
                s *= 0.5
            u, R, nr = un, Rn, nrn
            it += 1
        return u, it, nr / r0

    def return_map(self, u, Fp, epsP):
        F = self.deformation_gradient(u)
        return return_map_b(F, self._cellwise(self.phi_f), self._cellwise(self.phi_w), Fp, epsP, self.p)

    def driving_forces(self, u, Fp):
        """Per cell, the Gauss-point mean of d psi / d phi_f and d psi / d phi_w
        at fixed F and F_P (phi_g = 1 - phi_f - phi_w), by complex steps."""
        F = self.deformation_gradient(u)
        pf, pw = self._cellwise(self.phi_f), self._cellwise(self.phi_w)
        step = 1e-30
        gf = energy_b(F, pf + 1j * step, pw.astype(complex), Fp, self.p).imag / step
        gw = energy_b(F, pf.astype(complex), pw + 1j * step, Fp, self.p).imag / step
        return gf.mean(axis=-1), gw.mean(axis=-1)

    def max_von_mises(self, u, Fp):
        """Largest sqrt(3/2) |dev sigma| over the Gauss points, sigma = P F^T / det F."""
        F = self.deformation_gradient(u)
        P = piola_b(F, self._cellwise(self.phi_f), self._cellwise(self.phi_w), Fp, self.p)
        sig = (P @ np.swapaxes(F, -1, -2)) / np.linalg.det(F)[..., None, None]
        s = dev_b(sig)
        return float(np.sqrt(1.5 * np.sum(s * s, axis=(-2, -1))).max())


def identity_plastic(shape, dim):
    """F_P = I and eps_P = 0 at every Gauss point of `shape`."""
    ngp = 1 << dim
    Fp = np.zeros(tuple(shape) + (ngp, 3, 3))
    Fp[...] = np.eye(3)
    return Fp, np.zeros(tuple(shape) + (ngp,))
