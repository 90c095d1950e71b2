"""FP64 oracle of the finite-strain kinematics and elasticity of the model
(Bai et al., arXiv:2111.11538, Sec. 2.2 and Sec. 2.4): the multiplicative
split F = F_E F_T F_P (Eq. 9-12), the neo-Hooke phase energies (Eq. 13, 14),
the first Piola-Kirchhoff and Mandel stresses (Eq. 31, 19) and the J2 flow of
F_P in the Mandel stress with linear hardening (Eq. 25, 34), integrated by
backward Euler with the exponential map; and a uniaxial-strain (laminate)
equilibrium under rollers on a 1D grid.

TEST INFRASTRUCTURE ONLY: imported by the tests; nothing in the product path
loads it.  It shares no code with the HIP library.

Reading: the stresses are the derivatives of the stated energy.  The printed
forms K (det B_E - 1) F^-T and 2 G dev uni B_E F^-T are each twice the
derivative of Eq. 13 (its small-strain limits would be 2 K tr eps and
4 G dev eps); here
  P = d_T sum_a h_a [ K_a/2 (J_E^2 - 1) F_E^-T
                      + G_a J_E^(-2/3) (F_E - tr(C_E)/3 F_E^-T) ] d_T^(-1/3) F_P^-T
  M = d_T sum_a h_a [ K_a/2 (J_E^2 - 1) I + G_a dev(uni C_E) ]
(M = -(d psi / d F_P) F_P^T, Eq. 19), which reduce to K tr eps I + 2 G dev eps.
"""
from __future__ import annotations

import math

import numpy as np

I3 = np.eye(3)


def h(x):
    return x ** 3 * (6 * x ** 2 - 15 * x + 10)


def phase_weights(phi_f, phi_w):
    """h of ferrite, gas, wuestite (phi_g = 1 - phi_f - phi_w)."""
    return np.array([h(phi_f), h(1.0 - phi_f - phi_w), h(phi_w)])


def d_T(phi_f, Omega):
    """Eq. 9: det F_R = d_T = 1 - h(phi_f) Omega_f."""
    return 1.0 - h(phi_f) * Omega


def elastic_deformation(F, phi_f, Fp, Omega):
    """Eq. 12: F_E = F F_R^-1 with F_R = F_T F_P, F_T = d_T^(1/3) I."""
    return d_T(phi_f, Omega) ** (-1.0 / 3.0) * F @ np.linalg.inv(Fp)


def phase_energy(FE, K, G):
    """Eq. 13: K/4 (J^2 - 1 - 2 ln J) + G/2 (|uni F_E|^2 - 3), uni A = A / det(A)^(1/3)."""
    J = np.linalg.det(FE)
    U = FE / np.cbrt(J)
    return 0.25 * K * (J * J - 1.0 - 2.0 * math.log(J)) + 0.5 * G * (np.sum(U * U) - 3.0)


def dphase_dFE(FE, K, G):
    """Derivative of phase_energy with respect to F_E."""
    J = np.linalg.det(FE)
    FEiT = np.linalg.inv(FE).T
    trC = np.sum(FE * FE)
    return 0.5 * K * (J * J - 1.0) * FEiT + G * J ** (-2.0 / 3.0) * (FE - trC / 3.0 * FEiT)


def energy(F, phi_f, phi_w, Fp, p):
    """Eq. 14: psi_ela = d_T sum_a h(phi_a) phi_a^ela(F_E)."""
    FE = elastic_deformation(F, phi_f, Fp, p.Omega_f)
    w = phase_weights(phi_f, phi_w)
    return d_T(phi_f, p.Omega_f) * sum(w[a] * phase_energy(FE, p.K[a], p.G[a]) for a in range(3))


def piola(F, phi_f, phi_w, Fp, p):
    """First Piola-Kirchhoff stress d psi_ela / d F."""
    dT = d_T(phi_f, p.Omega_f)
    FE = elastic_deformation(F, phi_f, Fp, p.Omega_f)
    w = phase_weights(phi_f, phi_w)
    S = sum(w[a] * dphase_dFE(FE, p.K[a], p.G[a]) for a in range(3))
    return dT * dT ** (-1.0 / 3.0) * S @ np.linalg.inv(Fp).T


def mandel(F, phi_f, phi_w, Fp, p):
    """Mandel stress M = -(d psi / d F_P) F_P^T = d_T sum_a h_a F_E^T d phi_a / d F_E."""
    FE = elastic_deformation(F, phi_f, Fp, p.Omega_f)
    w = phase_weights(phi_f, phi_w)
    return d_T(phi_f, p.Omega_f) * sum(w[a] * FE.T @ dphase_dFE(FE, p.K[a], p.G[a]) for a in range(3))


def dev(A):
    return A - np.trace(A) / 3.0 * I3


def expm_sym_traceless(A):
    """exp of a symmetric traceless matrix by its eigen-decomposition."""
    lam, Q = np.linalg.eigh(0.5 * (A + A.T))
    return (Q * np.exp(lam)) @ Q.T


def return_map(F, phi_f, phi_w, Fp_n, epsP_n, p, tol=1e-13):
    """Eq. 25, 34 by backward Euler with the exponential map: F_P = exp(dl N)
    F_P^n with N = dev M / |dev M| of the END state and
    |dev M| = sqrt(2/3)(sigma_Y + H (eps_P^n + dl)).

    For an isotropic energy the end state is coaxial with the trial elastic
    state C_tr = F_E,tr^T F_E,tr (F_P = F_P^n): with C_tr = Q diag(c) Q^T,
    J = sqrt(prod c) (plastic flow keeps it) and the deviatoric log stretches
    e_tr = ln(c) / 2 - ln(J) / 3, the neo-Hooke energy gives
    dev M = k dev(exp(2 e)) in that frame, k = d_T sum_a h_a G_a, and the flow
    moves e to e = e_tr - dl n, n = s(e) / |s(e)|.  With |s| = Y(dl) at the end
    this is e + dl s(e) / Y(dl) = e_tr, solved by Newton for each dl; dl is the
    root of |s(e(dl))| - Y(dl), which falls with dl (bracket doubled from
    1e-3, then bisection to hi - lo <= tol hi).  Returns F_P, eps_P, dl."""
    r23 = math.sqrt(2.0 / 3.0)
    dT = d_T(phi_f, p.Omega_f)
    FE = elastic_deformation(F, phi_f, Fp_n, p.Omega_f)
    c, Q = np.linalg.eigh(FE.T @ FE)
    lnJ = 0.5 * float(np.sum(np.log(c)))
    etr = 0.5 * np.log(c) - lnJ / 3.0
    w = phase_weights(phi_f, phi_w)
    k = dT * sum(w[a] * p.G[a] for a in range(3))

    def s_of(e):
        x = np.exp(2.0 * e)
        return k * (x - x.mean())

    def Y(dl):
        return r23 * (p.sigY + p.Hhard * (epsP_n + dl))

    ytr = math.sqrt(float(np.sum(s_of(etr) ** 2))) - Y(0.0)
    if ytr <= 0.0:
        return Fp_n.copy(), epsP_n, 0.0

    def e_of(dl):
        a = dl / Y(dl)
        e = etr.copy()
        for _ in range(60):
            x = np.exp(2.0 * e)
            G = e + a * k * (x - x.mean()) - etr
            if np.max(np.abs(G)) <= 1e-15:
                break
            Jm = np.eye(3) + a * k * (2.0 * np.diag(x) - (2.0 / 3.0) * np.outer(np.ones(3), x))
            e = e - np.linalg.solve(Jm, G)
        return e

    def phi(dl):
        return math.sqrt(float(np.sum(s_of(e_of(dl)) ** 2))) - Y(dl)

    lo, hi = 0.0, 1e-3
    while phi(hi) > 0.0:
        lo, hi = hi, 2.0 * hi
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if phi(mid) > 0.0:
            lo = mid
        else:
            hi = mid
        if hi - lo <= tol * max(hi, 1e-300):
            break
    dl = 0.5 * (lo + hi)
    sv = s_of(e_of(dl))
    n = sv / math.sqrt(float(np.sum(sv * sv)))
    return (Q * np.exp(dl * n)) @ Q.T @ Fp_n, epsP_n + dl, dl


def laminate(phi_f, phi_w, p, h_cell=1.0, tol=1e-13):
    """Uniaxial strain along x of a stack of cells (layers) between rollers:
    F = diag(lam_i, 1, 1) per cell, with the total length fixed (sum lam_i
    = n) and P_xx equal in every cell (equilibrium).  Returns lam and P_xx,
    found by bisection on the common P_xx (lam_i(P) is increasing in P)."""
    n = len(phi_f)

    def pxx(lam, i):
        return piola(np.diag([lam, 1.0, 1.0]), phi_f[i], phi_w[i], I3, p)[0, 0]

    def lam_of(P, i):
        lo, hi = 1e-3, 10.0
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if pxx(mid, i) < P:
                lo = mid
            else:
                hi = mid
        return 0.5 * (lo + hi)

    lo, hi = -1e12, 1e12
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        tot = sum(lam_of(mid, i) for i in range(n))
        if tot < n:
            lo = mid
        else:
            hi = mid
        if hi - lo <= tol * max(abs(mid), 1.0):
            break
    P = 0.5 * (lo + hi)
    return np.array([lam_of(P, i) for i in range(n)]), P
