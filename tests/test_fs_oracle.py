"""Pins of the finite-strain oracle (F = F_E F_T F_P, neo-Hooke, J2 flow in
the Mandel stress): derivatives of the stated energy, closed forms of
homogeneous deformations, the small-strain limit (against the small-strain
C oracle), the return map's consistency, and the laminate equilibrium."""
import math

import numpy as np
import pytest

from paper_2111_11538_amd import inputs as I
from oracle import fs_oracle as FS


def _unimodular(rng, amp):
    A = rng.normal(0, amp, (3, 3))
    A = 0.5 * (A + A.T)
    A -= np.trace(A) / 3 * np.eye(3)
    return FS.expm_sym_traceless(A)


def test_piola_is_the_energy_derivative():
    rng = np.random.default_rng(1)
    p = I.Params()
    for _ in range(10):
        F = np.eye(3) + rng.normal(0, 0.15, (3, 3))
        Fp = _unimodular(rng, 0.05)
        pf, pw = rng.uniform(0, 0.6), rng.uniform(0, 0.3)
        P = FS.piola(F, pf, pw, Fp, p)
        d = 1e-7
        G = np.zeros((3, 3))
        for i in range(3):
            for j in range(3):
                E = np.zeros((3, 3))
                E[i, j] = d
                G[i, j] = (FS.energy(F + E, pf, pw, Fp, p) - FS.energy(F - E, pf, pw, Fp, p)) / (2 * d)
        assert np.max(np.abs(G - P)) < 1e-6 * np.max(np.abs(P)), (G, P)


def test_mandel_is_minus_the_plastic_derivative():
    """M = -(d psi / d F_P) F_P^T (Eq. 19), by central differences in F_P."""
    rng = np.random.default_rng(2)
    p = I.Params()
    for _ in range(6):
        F = np.eye(3) + rng.normal(0, 0.1, (3, 3))
        Fp = _unimodular(rng, 0.05)
        pf, pw = rng.uniform(0, 0.6), rng.uniform(0, 0.3)
        d = 1e-7
        D = np.zeros((3, 3))
        for i in range(3):
            for j in range(3):
                E = np.zeros((3, 3))
                E[i, j] = d
                D[i, j] = (FS.energy(F, pf, pw, Fp + E, p) - FS.energy(F, pf, pw, Fp - E, p)) / (2 * d)
        M = FS.mandel(F, pf, pw, Fp, p)
        assert np.max(np.abs(-D @ Fp.T - M)) < 1e-6 * np.max(np.abs(M))
        assert np.max(np.abs(M - M.T)) < 1e-9 * np.max(np.abs(M))       # isotropic: symmetric


def test_transformation_shrinkage_is_stress_free_and_hydrostatic_closed_form():
    """F = d_T^(1/3) I is the stress-free state of a transformed cell; under
    F = s I the stress is d_T^(2/3) K/2 (lam^6 - 1)/lam I with lam = s d_T^(-1/3)
    (no shear part, K the phase-weighted modulus without d_T)."""
    p = I.Params()
    for pf in (1.0, 0.7, 0.3):
        dT = FS.d_T(pf, p.Omega_f)
        w = FS.phase_weights(pf, 1 - pf)
        Kb = sum(w[a] * p.K[a] for a in range(3))
        F0 = dT ** (1 / 3) * np.eye(3)
        assert np.max(np.abs(FS.piola(F0, pf, 1 - pf, np.eye(3), p))) < 1e-3      # Pa, against GPa scales
        assert abs(FS.energy(F0, pf, 1 - pf, np.eye(3), p)) < 1e-12 * Kb
        for s in (0.8, 0.95, 1.1):
            lam = s * dT ** (-1 / 3)
            want = dT ** (2 / 3) * 0.5 * Kb * (lam ** 6 - 1) / lam
            P = FS.piola(s * np.eye(3), pf, 1 - pf, np.eye(3), p)
            assert np.max(np.abs(P - want * np.eye(3))) < 1e-10 * abs(want)


def test_simple_shear_closed_form():
    """Neo-Hooke in simple shear F = I + g e1 e2 (J = 1, pure wuestite): shear
    stress G g exactly and the normal-stress difference s11 - s22 = G g^2."""
    p = I.Params()
    Gw = p.G[2]
    for g in (0.01, 0.3, 1.0):
        F = np.eye(3)
        F[0, 1] = g
        P = FS.piola(F, 0.0, 1.0, np.eye(3), p)
        sig = P @ F.T
        assert abs(sig[0, 1] - Gw * g) < 1e-9 * Gw * g
        assert abs((sig[0, 0] - sig[1, 1]) - Gw * g * g) < 1e-9 * Gw * max(g * g, 1e-3)


def test_small_strain_limit_matches_the_small_strain_oracle(oracle):
    """As the transformation strain and the total strain shrink together
    (scale s), the finite-strain energy approaches the small-strain oracle's
    (eps_e = sym(F - I) - (d_T^(1/3) - 1) I) with an error of third order."""
    rng = np.random.default_rng(4)
    H0 = rng.normal(0, 1, (3, 3))
    base = I.Params()
    errs = []
    for s in (4e-3, 2e-3, 1e-3):
        p = base.replace(Omega_f=10 * s)
        pf, pw = 0.6, 0.3
        F = np.eye(3) + s * H0
        e_fs = FS.energy(F, pf, pw, np.eye(3), p)
        eb = np.array([F[0, 0] - 1, F[1, 1] - 1, F[2, 2] - 1, 0.5 * (F[0, 1] + F[1, 0]), 0.5 * (F[0, 2] + F[2, 0]),
                       0.5 * (F[1, 2] + F[2, 1])])
        e_ss = oracle.point_energy(p, pf, pw, 0.3, eb, np.zeros(6))[1]
        errs.append(abs(e_fs - e_ss) / abs(e_ss))
    assert errs[0] < 0.05
    assert 1.7 < errs[0] / errs[1] < 2.3 and 1.7 < errs[1] / errs[2] < 2.3, errs     # relative error O(s)


def test_return_map_consistency_and_small_strain_limit():
    """Monotone simple shear g with plastic flow: after each return the state
    is on the yield surface (|dev M| = sqrt(2/3)(sigma_Y + H eps_P)), det F_P
    = 1, and for small g eps_P follows the small-strain closed form
    (sqrt(2) G g - sqrt(2/3) sigma_Y) / (2 G + sqrt(2/3) H) to O(g^2)."""
    p = I.Params()
    G = p.G[2]
    Fp, eP = np.eye(3), 0.0
    gy = p.sigY / (math.sqrt(3) * G)
    r23 = math.sqrt(2 / 3)
    for g in np.linspace(0, 6 * gy, 25)[1:]:
        F = np.eye(3)
        F[0, 1] = g
        Fp, eP, dl = FS.return_map(F, 0.0, 1.0, Fp, eP, p)
        assert abs(np.linalg.det(Fp) - 1) < 1e-12
        s = FS.dev(FS.mandel(F, 0.0, 1.0, Fp, p))
        y = math.sqrt(np.sum(s * s)) - r23 * (p.sigY + p.Hhard * eP)
        assert y < 1e-6 * p.sigY
        if dl > 0:
            assert abs(y) < 1e-6 * p.sigY
        want = max(0.0, (math.sqrt(2) * G * g - r23 * p.sigY) / (2 * G + r23 * p.Hhard))
        assert abs(eP - want) < 0.01 * want + 1e-6      # the yield point itself moves by O(g^2)
    assert eP > 0


def test_laminate_equilibrium_and_small_strain_limit():
    """Layers stacked along x between rollers: every layer carries the same
    P_xx (checked with derivatives of each layer's energy, not with the
    stress routine) and the total length is kept; at small Omega_f the stress
    is the small-strain laminate's closed form."""
    layer = np.array([0, 0, 1, 2, 2, 0, 1, 2])
    pf = (layer == 0).astype(float)
    pw = (layer == 2).astype(float)
    for Om in (0.4, 0.004):
        p = I.Params(Omega_f=Om)
        lam, P = FS.laminate(pf, pw, p)
        assert abs(lam.sum() - len(lam)) < 1e-10
        # the shear term of the energy cancels to O(strain^2) from O(1) terms,
        # so the difference step is 1e-5 (rounding ~G 1e-16/d, truncation ~K d^2)
        d = 1e-5
        for i in range(len(lam)):
            E = lambda l: FS.energy(np.diag([l, 1.0, 1.0]), pf[i], pw[i], np.eye(3), p)
            dpsi = (E(lam[i] + d) - E(lam[i] - d)) / (2 * d)
            assert abs(dpsi - P) < 1e-5 * abs(P) + 30.0, (i, dpsi, P)
        if Om < 0.01:
            dT = np.where(layer == 0, 1 - Om, 1.0)
            Kl = dT * np.array([p.K[a] for a in layer])
            Gl = dT * np.array([p.G[a] for a in layer])
            el = np.where(layer == 0, (1 - Om) ** (1 / 3) - 1, 0.0)
            Ml = Kl + 4 * Gl / 3
            sig = -np.sum(3 * Kl * el / Ml) / np.sum(1 / Ml)
            assert abs(P - sig) < 0.02 * abs(sig), (P, sig)


def test_return_map_is_backward_euler_in_the_end_state():
    """One large step (no yield in between): the returned state satisfies the
    backward-Euler equations checked with the stress routine itself: F_P =
    exp(dl N) F_P^n with N = dev M / |dev M| of the END state, and |dev M| =
    sqrt(2/3)(sigma_Y + H (eps_P^n + dl))."""
    rng = np.random.default_rng(11)
    p = I.Params()
    r23 = math.sqrt(2 / 3)
    cases = []
    F = np.eye(3)
    F[0, 1] = 0.12
    cases.append((F, 0.1, 0.8, np.eye(3), 0.02))
    for _ in range(4):
        F = np.eye(3) + rng.normal(0, 0.1, (3, 3))
        cases.append((F, rng.uniform(0, 0.6), rng.uniform(0, 0.4), _unimodular(rng, 0.05), rng.uniform(0, 0.05)))
    moved = 0
    for F, pf, pw, Fp0, e0 in cases:
        Fp, eP, dl = FS.return_map(F, pf, pw, Fp0, e0, p)
        if dl == 0.0:
            continue
        moved += 1
        s = FS.dev(FS.mandel(F, pf, pw, Fp, p))
        ns = math.sqrt(np.sum(s * s))
        assert abs(ns - r23 * (p.sigY + p.Hhard * eP)) < 1e-9 * ns
        assert np.max(np.abs(FS.expm_sym_traceless(dl * s / ns) @ Fp0 - Fp)) < 1e-10
        assert abs(np.linalg.det(Fp) - np.linalg.det(Fp0)) < 1e-12
    assert moved >= 4
