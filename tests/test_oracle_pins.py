"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a value or
statement printed in the paper, a closed-form solution, an exact discrete
identity, an invariant of the model, or a brute-force construction.
"""
import math

import numpy as np
import pytest

from paper_2111_11538_amd import inputs as I


def _sim(O, dim, shape, h, dt, params, fields, **kw):
    return O.OracleSim(dim, shape, h, dt, params, fields, **kw)


def _uniform_fields(shape, **vals):
    f = {k: np.zeros(shape) for k in ("phi_f", "phi_w", "xO", "xH", "xW")}
    for k, v in vals.items():
        f[k][...] = v
    return f


# ---------------------------------------------------------------------------
# P1: calibrated free energy (Eq. 35, 36) and its common tangent (Eq. 37)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("phase", [0, 1, 2])
def test_free_energy_derivatives_match_finite_differences(oracle, phase):
    for x in np.linspace(0.0, 0.8, 17):
        d = 1e-5
        f0, fp, fpp = oracle.fe(phase, x)
        fm = oracle.fe(phase, x - d)[0]
        fP = oracle.fe(phase, x + d)[0]
        assert abs((fP - fm) / (2 * d) - fp) < 1e-6 * (1 + abs(fp))
        assert abs((fP - 2 * f0 + fm) / (d * d) - fpp) < 1e-3 * (1 + abs(fpp))


def test_common_tangent_is_the_lower_convex_hull(oracle):
    xf, xw, res = oracle.common_tangent()
    assert res < 1e-12
    # The caption of Fig. 1 prints x_f = 0.01 for ferrite.
    assert abs(xf - I.X_F_PRINTED) < 1e-3
    # The caption prints 0.571 for wuestite; the printed polynomials put the
    # tangent point at 0.517 (same digits, transposed) -- the reading used.
    assert abs(xw - 0.517) < 1e-3 and abs(xw - I.X_W_PRINTED) > 0.05
    # brute force: the tangent line touches both curves and lies below them
    ff = lambda x: oracle.fe(0, x)[0]
    fw = lambda x: oracle.fe(2, x)[0]
    slope = (fw(xw) - ff(xf)) / (xw - xf)
    line = lambda x: ff(xf) + slope * (x - xf)
    xs = np.linspace(-0.05, 0.8, 2001)
    gap = np.array([min(ff(x), fw(x)) - line(x) for x in xs])
    assert gap.min() > -1e-9
    # the inputs module carries the same digits for the initial conditions
    assert abs(xf - I.X_F_EQ) < 1e-14 and abs(xw - I.X_W_EQ) < 1e-14


def test_printed_x_w_is_not_a_tangent_point(oracle):
    # f_w'(0.571) differs from the tangent slope by more than 50 % (the reading
    # that the caption's 0.571 is a transposition of 0.517).
    xf, xw, _ = oracle.common_tangent()
    slope = oracle.fe(0, xf)[1]
    assert abs(oracle.fe(2, I.X_W_PRINTED)[1] - slope) > 0.5 * abs(slope)


# ---------------------------------------------------------------------------
# P2: equilibrium tanh interface (Allen-Cahn with the barrier m)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("m_form", [0, 1])
def test_tanh_interface_profile_and_width(oracle, m_form):
    p = I.Params(m_form=m_form, DO=(0, 0, 0), DH=(0, 0, 0), DW=(0, 0, 0), kfor=0.0)
    # stationary profile of eps phi'' = w m'(phi): phi = (1 + tanh(x / ell)) / 2
    ell = math.sqrt(p.eps[0] / (8 * p.w[0])) if m_form == 0 else math.sqrt(2 * p.eps[0] / p.w[0])
    errs = []
    for ncell_per_ell in (8, 16):
        h = ell / ncell_per_ell
        n = 24 * ncell_per_ell
        x = (np.arange(n) + 0.5) * h - n * h / 2
        f = _uniform_fields((1, n))
        f["phi_f"][0] = 0.5 * (1 + np.tanh(x / (2.0 * ell)))    # start twice too wide
        f["phi_w"][0] = 1.0 - f["phi_f"][0]
        dt = 0.2 * h * h / (4 * p.L[0] * (p.eps[0] + p.eps[1]))
        s = _sim(oracle, 2, (1, n), h, dt, p, f, mechanics=False, dirichlet=False, chem_phase=False)
        tau = 1.0 / (p.L[0] * p.w[0] * (32.0 if m_form == 0 else 2.0))
        nsteps = int(12 * tau / dt)
        s.step(nsteps)
        exact = 0.5 * (1 + np.tanh(x / ell))
        errs.append(np.max(np.abs(s.f["phi_f"][0] - exact)))
        # phi_g stays zero: phi_f + phi_w = 1 to rounding
        assert np.max(np.abs(s.f["phi_f"] + s.f["phi_w"] - 1.0)) < 1e-12
    assert errs[0] < 5e-3
    assert errs[1] < errs[0] / 3.0      # second-order convergence in h / ell


# ---------------------------------------------------------------------------
# P3: Gaussian diffusion of hydrogen in pure gas: exact second-moment identity
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dim", [2, 3])
def test_gaussian_second_moment_grows_exactly(oracle, dim):
    p = I.Params()
    n = 48 if dim == 2 else 32
    shape = (n,) * dim
    h = I.H_DEFAULT
    dt = I.stable_dt(p, h, dim)
    f = _uniform_fields(shape)
    coords = np.meshgrid(*[(np.arange(n) + 0.5) * h for _ in range(dim)], indexing="ij")
    c0 = n * h / 2
    r2 = sum((c - c0) ** 2 for c in coords)
    f["xH"] = 0.01 * np.exp(-r2 / (2 * (2.0 * h) ** 2))
    s = _sim(oracle, dim, shape, h, dt, p, f, mechanics=True, dirichlet=False)
    for _ in range(20):
        m0, M2 = s.f["xH"].sum(), (r2 * s.f["xH"]).sum()
        s.step()
        m1, M2n = s.f["xH"].sum(), (r2 * s.f["xH"]).sum()
        assert abs(m1 - m0) < 1e-14 * m0                      # mass exact
        expect = 2 * dim * p.DH[1] * dt * m0
        assert abs((M2n - M2) - expect) < 1e-8 * expect        # Laplacian of |x|^2 is 2d
    assert np.all(s.f["xO"] == 0.0) and np.all(s.f["xW"] == 0.0)


# ---------------------------------------------------------------------------
# P4: Fourier mode of x_O in pure wuestite decays with the exact factor
# ---------------------------------------------------------------------------
def test_oxygen_fourier_mode_decay_factor(oracle):
    p = I.Params()
    nx, ny, kx, ky = 32, 24, 3, 2
    h = I.H_DEFAULT
    dt = 2e-6
    f = _uniform_fields((ny, nx), phi_w=1.0)
    xb, a = 0.45, 0.02
    mode = np.outer(np.cos(np.pi * ky * (np.arange(ny) + 0.5) / ny), np.cos(np.pi * kx * (np.arange(nx) + 0.5) / nx))
    f["xO"] = xb + a * mode
    s = _sim(oracle, 2, (ny, nx), h, dt, p, f, mechanics=False, dirichlet=False)
    lam = 4 / h ** 2 * (math.sin(math.pi * kx / (2 * nx)) ** 2 + math.sin(math.pi * ky / (2 * ny)) ** 2)
    scale = p.R * p.theta / p.Vmol
    M = p.DO[2] / (scale * 2 * 173.263)
    factor = 1 - dt * (p.DO[2] * lam + M * p.kappaO * lam ** 2)
    for _ in range(5):
        prev = s.f["xO"] - xb
        s.step()
        assert np.max(np.abs((s.f["xO"] - xb) - factor * prev)) < 1e-13
    assert np.all(s.f["phi_w"] == 1.0)


# ---------------------------------------------------------------------------
# P5: reaction kinetics in a uniform cell (Eq. 27, 28)
# ---------------------------------------------------------------------------
def test_reaction_ode_and_invariants(oracle):
    p = I.Params(L=(0.0, 0.0, 0.0))
    a0, b0 = 0.3, 0.2
    m_g = 1.0     # m(1/2) = 16/16 with the reading m = 16 x^2 (1-x)^2
    T = 4e-4

    def run(dt):
        f = _uniform_fields((2, 2), phi_f=0.0, phi_w=0.5, xO=a0, xH=b0)
        s = _sim(oracle, 2, (2, 2), I.H_DEFAULT, dt, p, f, mechanics=False, dirichlet=False)
        n = int(round(T / dt))
        for _ in range(n):
            s.step()
            assert abs(s.f["xO"][0, 0] + s.f["xW"][0, 0] - a0) < 1e-15
            assert abs(s.f["xH"][0, 0] + 2 * s.f["xW"][0, 0] - b0) < 1e-15
        return s.f["xO"][0, 0]

    c = b0 - 2 * a0
    exact = c * a0 / ((2 * a0 + c) * math.exp(c * p.kfor * m_g * T) - 2 * a0)
    e1 = abs(run(2e-6) - exact)
    e2 = abs(run(1e-6) - exact)
    assert e1 < 2e-3 * a0
    assert 1.8 < e1 / e2 < 2.2      # explicit Euler: first order


def test_reaction_stops_when_pore_is_full_of_water(oracle):
    p = I.Params()
    f = _uniform_fields((2, 2), phi_f=0.0, phi_w=0.5, xO=0.3, xH=0.2, xW=1.0)
    s = _sim(oracle, 2, (2, 2), I.H_DEFAULT, 1e-6, p, f, mechanics=False, dirichlet=False)
    s.step()
    assert np.all(s.f["xO"] == 0.3) and np.all(s.f["xW"] == 1.0)


# ---------------------------------------------------------------------------
# P6: oxygen and hydrogen ledgers
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dirichlet", [False, True])
def test_oxygen_is_conserved(oracle, dirichlet):
    wl = I.workload("core_shell_2d", n=24)
    s = _sim(oracle, 2, wl.shape, wl.h, wl.dt, wl.params, wl.fields, mechanics=True, plasticity=True,
             dirichlet=dirichlet, cg_rtol=1e-10)
    O0 = (s.f["xO"] + s.f["xW"]).sum()
    H0 = (s.f["xH"] + 2 * s.f["xW"]).sum()
    for _ in range(10):
        st = s.step()
        assert abs(st["O_drift"]) < 1e-13
        assert abs(st["H_drift"]) < 1e-13
    if not dirichlet:
        assert abs((s.f["xO"] + s.f["xW"]).sum() - O0) < 1e-13 * O0
        assert abs((s.f["xH"] + 2 * s.f["xW"]).sum() - H0) < 1e-13 * H0
    else:
        assert st["H_out"] < 0          # hydrogen enters through the gas faces


# ---------------------------------------------------------------------------
# P7: the elasticity operator is symmetric positive definite; laminate exact
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dim", [2, 3])
def test_operator_symmetric_positive_definite_and_diagonal(oracle, dim):
    rng = np.random.default_rng(7)
    shape = (5, 6) if dim == 2 else (4, 5, 6)
    f = _uniform_fields(shape)
    f["phi_f"] = rng.uniform(0, 0.6, shape)
    f["phi_w"] = rng.uniform(0, 0.4, shape)
    s = _sim(oracle, dim, shape, 1e-7, 1e-9, I.Params(), f)
    K, G = s.moduli()
    fs = oracle.face_shapes(dim, shape)[:dim]

    def rand():
        u = [rng.standard_normal(fsh) for fsh in fs]
        # boundary faces are fixed
        u[0][..., 0] = 0; u[0][..., -1] = 0
        u[1][..., 0, :] = 0; u[1][..., -1, :] = 0
        if dim == 3:
            u[2][0] = 0; u[2][-1] = 0
        return u

    dot = lambda a, b: sum((x * y).sum() for x, y in zip(a, b))
    for _ in range(3):
        x, y = rand(), rand()
        Ax, Ay = s.apply(K, G, x), s.apply(K, G, y)
        assert abs(dot(y, Ax) - dot(x, Ay)) < 1e-12 * abs(dot(x, Ax))
        assert dot(x, Ax) > 0
    # diagonal entries by probing with unit vectors
    D = s.diag(K, G)
    for comp in range(dim):
        for idx in [(1,) * dim, tuple(max(1, d - 2) for d in fs[comp])]:
            e = [np.zeros(fsh) for fsh in fs]
            e[comp][idx] = 1.0
            q = s.apply(K, G, e)
            assert abs(q[comp][idx] - D[comp][idx]) < 1e-12 * abs(D[comp][idx])


@pytest.mark.parametrize("dim", [2, 3])
def test_laminate_stress_is_exact(oracle, dim):
    p = I.Params()
    n = 12
    shape = (4, n) if dim == 2 else (3, 4, n)
    f = _uniform_fields(shape)
    layer = np.array([0, 0, 1, 1, 1, 2, 2, 0, 0, 1, 2, 2])    # 0 ferrite, 1 gas, 2 wuestite, along x
    f["phi_f"][...] = (layer == 0)
    f["phi_w"][...] = (layer == 2)
    h = I.H_DEFAULT
    s = _sim(oracle, dim, shape, h, 1e-9, p, f, cg_rtol=1e-13)
    s.mech_solve()
    # closed form: sigma_xx uniform = -sum(3 K_i e*_i / M_i) / sum(1 / M_i)
    dT = np.where(layer == 0, 1 - p.Omega_f, 1.0)
    Kl = dT * np.array([p.K[a] for a in layer])
    Gl = dT * np.array([p.G[a] for a in layer])
    el = np.where(layer == 0, (1 - p.Omega_f) ** (1 / 3) - 1, 0.0)
    Ml = Kl + 4 * Gl / 3
    sig = -np.sum(3 * Kl * el / Ml) / np.sum(1 / Ml)
    exx = np.diff(s.ux, axis=-1) / h
    sig_num = Ml * exx - 3 * Kl * el
    assert np.max(np.abs(sig_num - sig)) < 1e-9 * abs(sig)
    assert np.max(np.abs(s.uy)) < 1e-12 * np.max(np.abs(s.ux))


# ---------------------------------------------------------------------------
# P8: Lame solution of a misfitting core-shell disk (plane strain)
# ---------------------------------------------------------------------------
def _lame_2d(layers, R, outer="fixed"):
    """u_r = A_k r + B_k / r per layer (plane strain), eigenstrain e_k:
    sigma_rr = 2 (K + G/3) A - 3 K e - 2 G B / r^2."""
    nl = len(layers)
    M = np.zeros((2 * nl, 2 * nl))
    rhs = np.zeros(2 * nl)
    row = 0
    M[row, 1] = 1.0; row += 1                                  # B_core = 0
    for k in range(nl - 1):
        r = layers[k][0]
        Kk, Gk, ek = layers[k][1:]
        Kn, Gn, en = layers[k + 1][1:]
        M[row, 2 * k] = r; M[row, 2 * k + 1] = 1 / r
        M[row, 2 * k + 2] = -r; M[row, 2 * k + 3] = -1 / r; row += 1
        M[row, 2 * k] = 2 * (Kk + Gk / 3); M[row, 2 * k + 1] = -2 * Gk / r ** 2
        M[row, 2 * k + 2] = -2 * (Kn + Gn / 3); M[row, 2 * k + 3] = 2 * Gn / r ** 2
        rhs[row] = 3 * Kk * ek - 3 * Kn * en; row += 1
    Kl, Gl, el = layers[-1][1:]
    if outer == "fixed":
        M[row, 2 * nl - 2] = R; M[row, 2 * nl - 1] = 1 / R
    else:
        M[row, 2 * nl - 2] = 2 * (Kl + Gl / 3); M[row, 2 * nl - 1] = -2 * Gl / R ** 2
        rhs[row] = 3 * Kl * el
    return np.linalg.solve(M, rhs)


def test_lame_core_shell_disk_converges(oracle):
    p = I.Params()
    errs = []
    for n in (32, 64, 128):
        a, b = 0.25 * n, 0.375 * n                 # core and shell radii in cells
        f = I.ic_core_shell((n, n), r_core=a, r_shell=b)
        h = 1e-7
        s = _sim(oracle, 2, (n, n), h, 1e-9, p, f, cg_rtol=1e-11)
        s.mech_solve()
        dT = 1 - p.Omega_f
        layers = [(a * h, p.K[2], p.G[2], 0.0),
                  (b * h, dT * p.K[0], dT * p.G[0], dT ** (1 / 3) - 1),
                  (n / 2 * h, p.K[1], p.G[1], 0.0)]
        A_core = _lame_2d(layers, n / 2 * h)[0]
        exx = np.diff(s.ux, axis=1) / h
        yy, xx = np.meshgrid(np.arange(n) + 0.5 - n / 2, np.arange(n) + 0.5 - n / 2, indexing="ij")
        inner = xx ** 2 + yy ** 2 < (0.5 * a) ** 2
        errs.append(abs(exx[inner].mean() - A_core) / abs(A_core))
    assert errs[-1] < 0.03
    assert errs[2] < errs[0]


# ---------------------------------------------------------------------------
# P9: radial return under monotone pure shear (Eq. 25, 34)
# ---------------------------------------------------------------------------
def test_return_map_pure_shear_closed_form(oracle):
    p = I.Params()
    G = 30e9
    epsp = np.zeros(6)
    epsP = 0.0
    gy = p.sigY / (math.sqrt(3) * G)
    for gamma in np.linspace(0, 12 * gy, 37)[1:]:
        etr = np.zeros(6)
        etr[3] = gamma / 2
        etr -= epsp
        dl, nn = oracle.return_map(p, G, etr, epsP)
        epsp = epsp + dl * nn
        epsP += dl
        expect = max(0.0, (math.sqrt(2) * G * gamma - math.sqrt(2 / 3) * p.sigY) / (2 * G + math.sqrt(2 / 3) * p.Hhard))
        assert abs(epsP - expect) < 1e-15 + 1e-12 * expect
        assert abs(epsp[0] + epsp[1] + epsp[2]) < 1e-18       # isochoric flow
        # consistency: f <= 0 after the return
        e = np.zeros(6); e[3] = gamma / 2
        s = 2 * G * (e - epsp)
        ns = math.sqrt(s[0] ** 2 + s[1] ** 2 + s[2] ** 2 + 2 * (s[3] ** 2 + s[4] ** 2 + s[5] ** 2))
        assert ns - math.sqrt(2 / 3) * (p.sigY + p.Hhard * epsP) < 1e-6 * p.sigY
        if gamma <= gy:
            assert dl == 0.0


# ---------------------------------------------------------------------------
# P11: without reaction and Dirichlet faces the free energy never increases
# ---------------------------------------------------------------------------
def test_energy_decreases(oracle):
    p = I.Params(kfor=0.0)
    n = 24
    f = I.ic_core_shell((n, n), r_core=7.0, frame=0, noise_seed=5)
    f["xO"] = np.where(f["phi_w"] > 0.5, 0.45, 0.05)
    s = _sim(oracle, 2, (n, n), I.H_DEFAULT, 5e-6, p, f, mechanics=False, dirichlet=False)
    E = [s.energy()]
    for _ in range(30):
        s.step()
        E.append(s.energy())
    dE = np.diff(E)
    assert np.all(dE <= 1e-12 * abs(E[0]))
    assert E[-1] < E[0]


# ---------------------------------------------------------------------------
# P12: driving force equals the derivative of the local energy density
# ---------------------------------------------------------------------------
def test_driving_force_is_energy_derivative(oracle):
    rng = np.random.default_rng(3)
    for _ in range(25):
        pf, pw = rng.uniform(0.05, 0.6), rng.uniform(0.05, 0.35)
        xO = rng.uniform(0.0, 0.6)
        ebar = rng.normal(0, 0.02, 6)
        epsp = rng.normal(0, 0.005, 6)
        epsp[:3] -= epsp[:3].mean()
        p = I.Params(Omega_f=rng.uniform(0.1, 0.5))
        g = oracle.driving_force(p, pf, pw, xO, ebar, epsp)
        d = 1e-6
        E = lambda a, b: oracle.point_energy(p, a, b, xO, ebar, epsp).sum()
        gf = (E(pf + d, pw) - E(pf - d, pw)) / (2 * d)
        gw = (E(pf, pw + d) - E(pf, pw - d)) / (2 * d)
        assert abs(gf - g[0]) < 1e-6 * (abs(g[0]) + 1e4 * p.w[0] * 1e-4)
        assert abs(gw - g[1]) < 1e-6 * (abs(g[1]) + 1e4 * p.w[0] * 1e-4)


# ---------------------------------------------------------------------------
# Order parameters bounded to [0, 1] (Sec. 2.2): projection onto the simplex
# ---------------------------------------------------------------------------
def test_phase_bound_is_nearest_simplex_point(oracle):
    rng = np.random.default_rng(11)
    # a dense sample of the simplex {phi >= 0, sum = 1} for a brute-force nearest point
    t = np.linspace(0.0, 1.0, 801)
    A, B = np.meshgrid(t, t, indexing="ij")
    ok = A + B <= 1.0 + 1e-15
    cand = np.stack([A[ok], 1.0 - A[ok] - B[ok], B[ok]], axis=1)
    for _ in range(200):
        pf, pw = rng.uniform(-0.6, 1.6, 2)
        qf, qw = oracle.simplex_project(pf, pw)
        q = np.array([qf, 1.0 - qf - qw, qw])
        assert np.all(q >= -1e-15) and abs(q.sum() - 1.0) < 1e-15
        u = np.array([pf, 1.0 - pf - pw, pw])
        d_best = np.min(np.sum((cand - u) ** 2, axis=1))
        # no sampled point of the simplex is nearer (grid spacing 1/800)
        assert np.sum((q - u) ** 2) <= d_best + 1e-12
        assert oracle.simplex_project(qf, qw) == (qf, qw)          # idempotent
        if np.all(u >= 0):
            assert (qf, qw) == (pf, pw)                             # inside: unchanged
    # the projection moves along the simplex's normal when one entry is slightly negative
    qf, qw = oracle.simplex_project(0.6, 0.5)                     # phi_g = -0.1
    assert abs(qf - 0.55) < 1e-15 and abs(qw - 0.45) < 1e-15


# ---------------------------------------------------------------------------
# Largest von Mises stress: closed form of the laminate
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dim", [2, 3])
def test_max_von_mises_of_the_laminate(oracle, dim):
    """Layers stacked along x under rollers: u_y = u_z = 0, uniform sigma_xx,
    strain eps_xx_i = (sigma_xx + 3 K_i e_i) / M_i in layer i, and the cell von
    Mises stress sqrt(3/2) |dev sigma| reduces to 2 G_i |eps_xx_i|."""
    p = I.Params()
    n = 12
    shape = (4, n) if dim == 2 else (3, 4, n)
    f = _uniform_fields(shape)
    layer = np.array([0, 0, 1, 1, 1, 2, 2, 0, 0, 1, 2, 2])
    f["phi_f"][...] = (layer == 0)
    f["phi_w"][...] = (layer == 2)
    h = I.H_DEFAULT
    s = _sim(oracle, dim, shape, h, 1e-12, p, f, mechanics=True, plasticity=False, dirichlet=False, cg_rtol=1e-13)
    st = s.step()
    dT = np.where(layer == 0, 1 - p.Omega_f, 1.0)
    Kl = dT * np.array([p.K[a] for a in layer])
    Gl = dT * np.array([p.G[a] for a in layer])
    el = np.where(layer == 0, (1 - p.Omega_f) ** (1 / 3) - 1, 0.0)
    Ml = Kl + 4 * Gl / 3
    sig = -np.sum(3 * Kl * el / Ml) / np.sum(1 / Ml)
    exx = (sig + 3 * Kl * el) / Ml
    vm = np.max(2 * Gl * np.abs(exx))
    assert abs(st["max_vm"] - vm) < 1e-8 * vm, (st["max_vm"], vm)


# ---------------------------------------------------------------------------
# Reduction degree f = 1 - sum x_O / sum x_O(0) (Eq. 39), closed form
# ---------------------------------------------------------------------------
def test_reduction_degree_closed_form(oracle):
    """Half of a closed box reacts (phi_g = 1/2 there, so m(phi_g) = 1), the
    other half is pure wuestite (m = 0); no transport (every diffusivity 0) and
    frozen phases (L = 0).  In the reacting half a = x_O follows
    a' = -k a (2 a + c), c = x_H - 2 x_O (constant), whose solution is
    a(t) = c a0 / ((2 a0 + c) exp(c k t) - 2 a0); Eq. 39 then gives f(t) in
    closed form.  Explicit Euler converges to it at first order in dt."""
    shape = (6, 8)
    a0, xH0, xb = 0.02, 0.08, 0.5
    k = 4.5e4
    T = 2.0e-4
    errs = []
    for nsteps in (200, 400, 800):
        p = I.Params(L=(0.0, 0.0, 0.0), DO=(0.0, 0.0, 0.0), DH=(0.0, 0.0, 0.0), DW=(0.0, 0.0, 0.0), kappaO=0.0,
                     kfor=k)
        f = _uniform_fields(shape)
        f["phi_w"][:, :4] = 1.0
        f["xO"][:, :4] = xb
        f["phi_f"][:, 4:] = 0.25
        f["phi_w"][:, 4:] = 0.25
        f["xO"][:, 4:] = a0
        f["xH"][:, 4:] = xH0
        s = _sim(oracle, 2, shape, I.H_DEFAULT, T / nsteps, p, f, mechanics=False, dirichlet=False)
        st = s.step(nsteps)
        c = xH0 - 2 * a0
        a = c * a0 / ((2 * a0 + c) * math.exp(c * k * T) - 2 * a0)
        f_exact = 1.0 - (a + xb) / (a0 + xb)
        errs.append(abs(st["red_degree"] - f_exact))
        assert f_exact > 0.01
    assert errs[-1] < 2e-3 * f_exact
    assert 1.7 < errs[0] / errs[1] < 2.3 and 1.7 < errs[1] / errs[2] < 2.3     # first order


# ---------------------------------------------------------------------------
# The discrete elastic energy's gradient is the residual A u - b
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dim", [2, 3])
def test_elastic_energy_gradient_is_the_residual(oracle, dim):
    """Pi(u) is quadratic, so central differences of the discrete elastic
    energy give its gradient exactly (up to rounding); it must equal
    h^(d-1) (A u - b) of the operator and right-hand side the solve uses (the
    net force on a face divided by the face's area), with a plastic strain
    present so that every term of b enters."""
    rng = np.random.default_rng(5 + dim)
    shape = (5, 6) if dim == 2 else (4, 5, 6)
    f = _uniform_fields(shape)
    f["phi_f"] = rng.uniform(0.0, 0.7, shape)
    f["phi_w"] = rng.uniform(0.0, 0.3, shape)
    nc = 4 if dim == 2 else 6
    epsp = rng.normal(0, 2e-3, (nc,) + shape)
    h = I.H_DEFAULT
    p = I.Params()
    s = _sim(oracle, dim, shape, h, 1e-9, p, f, epsp=epsp)
    fs = oracle.face_shapes(dim, shape)[:dim]
    u = [rng.normal(0, 1e-9, fsh) for fsh in fs]
    u[0][..., 0] = 0; u[0][..., -1] = 0
    u[1][..., 0, :] = 0; u[1][..., -1, :] = 0
    if dim == 3:
        u[2][0] = 0; u[2][-1] = 0
    s.ux[...] = u[0]
    s.uy[...] = u[1]
    if dim == 3:
        s.uz[...] = u[2]
    K, G = s.moduli()
    Au = s.apply(K, G, u)
    b = s.rhs()
    arrs = [s.ux, s.uy] + ([s.uz] if dim == 3 else [])
    d = 1e-12
    checked = [0, 0, 0]
    for comp in range(dim):
        a = arrs[comp]
        for idx in list(np.ndindex(a.shape))[::3]:
            # interior faces only (the roller faces are fixed at zero)
            ax = {0: -1, 1: -2, 2: -3}[comp]
            if idx[ax] == 0 or idx[ax] == a.shape[ax] - 1:
                continue
            v = a[idx]
            a[idx] = v + d
            Ep = s.elastic_energy()
            a[idx] = v - d
            Em = s.elastic_energy()
            a[idx] = v
            g = (Ep - Em) / (2 * d)
            want = h ** (dim - 1) * (Au[comp][idx] - b[comp][idx])
            scale = h ** (dim - 1) * (np.max(np.abs(Au[comp])) + np.max(np.abs(b[comp])))
            assert abs(g - want) < 1e-6 * scale, (comp, idx, g, want)
            checked[comp] += 1
    assert min(checked[:dim]) > 5, checked


# ---------------------------------------------------------------------------
# P11 with mechanics: the elastic energy at equilibrium joins the descent
# ---------------------------------------------------------------------------
def test_energy_decreases_with_mechanics(oracle):
    """Without reaction and Dirichlet faces the total free energy -- barrier,
    gradient and the elastic energy at mechanical equilibrium (Eq. 26) --
    never increases.  The chemical energy is switched off and the species are
    frozen (no diffusion), so that the phases move under the elastic driving
    force and the elastic energy is about half of the drop."""
    p = I.Params(kfor=0.0, DO=(0.0, 0.0, 0.0), DH=(0.0, 0.0, 0.0), DW=(0.0, 0.0, 0.0))
    n = 24
    f = I.ic_core_shell((n, n), r_core=7.0, frame=0, noise_seed=5)
    f["xO"] = np.where(f["phi_w"] > 0.5, 0.45, 0.05)
    s = _sim(oracle, 2, (n, n), I.H_DEFAULT, 1e-2, p, f, mechanics=True, plasticity=False, dirichlet=False,
             chem_phase=False, cg_rtol=1e-12)
    s.mech_solve()
    E, Eel = [s.energy()], [s.elastic_energy()]
    for _ in range(30):
        s.step()
        s.mech_solve()                 # the elastic energy at equilibrium with the new phases
        E.append(s.energy())
        Eel.append(s.elastic_energy())
    dE = np.diff(E)
    assert np.all(dE <= 1e-12 * abs(E[0]))
    assert E[-1] < E[0]
    assert Eel[-1] - Eel[0] < 0.25 * (E[-1] - E[0]) < 0


# ---------------------------------------------------------------------------
# P8 in 3D: Lame solution of a misfitting core-shell sphere
# ---------------------------------------------------------------------------
def _lame_3d(layers, R):
    """u_r = A_k r + B_k / r^2 per layer, eigenstrain e_k:
    sigma_rr = 3 K (A - e) - 4 G B / r^3; B_core = 0, u_r and sigma_rr
    continuous, u_r(R) = 0."""
    nl = len(layers)
    M = np.zeros((2 * nl, 2 * nl))
    rhs = np.zeros(2 * nl)
    row = 0
    M[row, 1] = 1.0; row += 1
    for k in range(nl - 1):
        r = layers[k][0]
        Kk, Gk, ek = layers[k][1:]
        Kn, Gn, en = layers[k + 1][1:]
        M[row, 2 * k] = r; M[row, 2 * k + 1] = 1 / r ** 2
        M[row, 2 * k + 2] = -r; M[row, 2 * k + 3] = -1 / r ** 2; row += 1
        M[row, 2 * k] = 3 * Kk; M[row, 2 * k + 1] = -4 * Gk / r ** 3
        M[row, 2 * k + 2] = -3 * Kn; M[row, 2 * k + 3] = 4 * Gn / r ** 3
        rhs[row] = 3 * Kk * ek - 3 * Kn * en; row += 1
    M[row, 2 * nl - 2] = R; M[row, 2 * nl - 1] = 1 / R ** 2
    return np.linalg.solve(M, rhs)


def test_lame_core_shell_sphere_converges(oracle):
    p = I.Params()
    errs = []
    for n in (16, 32, 48):
        a, b = 0.25 * n, 0.375 * n
        f = I.ic_core_shell((n, n, n), r_core=a, r_shell=b)
        h = 1e-7
        s = _sim(oracle, 3, (n, n, n), h, 1e-9, p, f, cg_rtol=1e-10)
        s.mech_solve()
        dT = 1 - p.Omega_f
        layers = [(a * h, p.K[2], p.G[2], 0.0),
                  (b * h, dT * p.K[0], dT * p.G[0], dT ** (1 / 3) - 1),
                  (n / 2 * h, p.K[1], p.G[1], 0.0)]
        A_core = _lame_3d(layers, n / 2 * h)[0]
        c = np.arange(n) + 0.5 - n / 2
        zz, yy, xx = np.meshgrid(c, c, c, indexing="ij")
        inner = xx ** 2 + yy ** 2 + zz ** 2 < (0.5 * a) ** 2
        e = [np.diff(s.ux, axis=2)[inner].mean() / h, np.diff(s.uy, axis=1)[inner].mean() / h,
             np.diff(s.uz, axis=0)[inner].mean() / h]
        assert max(e) - min(e) < 1e-8 * abs(A_core)          # the core's strain is isotropic
        errs.append(abs(e[0] - A_core) / abs(A_core))
    assert errs[-1] < 0.015, errs
    assert errs[-1] < errs[0]


# ---------------------------------------------------------------------------
# P10: lever rule of the ferrite / wuestite benchmark (Sec. 4.1, Eq. 38)
# ---------------------------------------------------------------------------
@pytest.mark.slow
def test_lever_rule(oracle):
    """Sec. 4.1: a box half ferrite, half wuestite with a uniform initial x_O
    (no reaction, no mechanics, closed) equilibrates to a wuestite fraction
    (Eq. 38) given by the lever rule (x_O - x_f) / (x_w - x_f).  Equilibrium
    depends on the energy only, so the mobilities L_a are raised tenfold and
    the gradient coefficients eps_a thirtyfold (a flat interface has no
    curvature, so eps moves no bulk composition) so that the interface is
    resolved on the 78 nm grid and moves within seconds of model time.  The
    diffuse interface holds an oxygen excess, so phi_bar = lever + c / length:
    two box lengths (5 and 10 um) extrapolate it away.  The bulk compositions
    reach the common tangent of Eq. 35, and the fraction discriminates the
    tangent value x_w = 0.517 from the 0.571 printed in the caption of Fig. 1."""
    base = I.Params()
    p = I.Params(kfor=0.0, eps=tuple(30 * e for e in base.eps), L=tuple(10 * l for l in base.L))
    h = 5e-6 / 64
    dt, T = 3.5e-5, 4.0
    xf, xw = oracle.common_tangent()[:2]
    for xbar in (0.3, 0.45):
        res = {}
        for nx in (64, 128):
            f = _uniform_fields((1, nx))
            f["phi_f"][:, :nx // 2] = 1.0
            f["phi_w"][:, nx // 2:] = 1.0
            f["xO"][...] = xbar
            s = _sim(oracle, 2, (1, nx), h, dt, p, f, mechanics=False, plasticity=False, dirichlet=False)
            n = int(T / dt)
            s.step(int(0.9 * n))
            a = s.f["phi_w"].mean()
            s.step(n - int(0.9 * n))
            res[nx] = s.f["phi_w"].mean()
            assert abs(res[nx] - a) < 2e-4                          # equilibrated
            assert abs(s.f["xO"][0, 0] - xf) < 0.005 and abs(s.f["xO"][0, -1] - xw) < 0.005
        ext = 2 * res[128] - res[64]
        lever = (xbar - xf) / (xw - xf)
        printed = (xbar - I.X_F_PRINTED) / (I.X_W_PRINTED - I.X_F_PRINTED)
        assert abs(ext - lever) < 0.01, (xbar, ext, lever)
        assert abs(ext - printed) > 0.05, (xbar, ext, printed)


# ---------------------------------------------------------------------------
# Linearly implicit species update (backward Euler for the diffusion)
# ---------------------------------------------------------------------------
def _mode_fields(shape, k, key, base, amp, **vals):
    f = _uniform_fields(shape, **vals)
    nx = shape[-1]
    i = np.arange(nx) + 0.5
    f[key] = base + amp * np.cos(np.pi * k * i / nx) * np.ones(shape)
    return f


def test_implicit_hydrogen_mode_decays_by_the_backward_euler_factor(oracle):
    """Pure gas, closed box, no reaction: a cosine mode of x_H (an exact
    eigenvector of the no-flux Laplacian, eigenvalue lambda = (4/h^2)
    sin^2(pi k / 2N)) is multiplied per step by exactly 1 / (1 + dt D lambda),
    at a time step 200 times the explicit limit."""
    p = I.Params(kfor=0.0)
    h = I.H_DEFAULT
    shape = (4, 32)
    D = p.DH[1]
    dt = 200 * h * h / (4 * D)
    for k in (1, 5):
        f = _mode_fields(shape, k, "xH", 0.01, 0.002, phi_f=0.0, phi_w=0.0)
        s = _sim(oracle, 2, shape, h, dt, p, f, mechanics=False, dirichlet=False, implicit=True)
        lam = 4 / h ** 2 * math.sin(math.pi * k / (2 * shape[-1])) ** 2
        for _ in range(3):
            a0 = s.f["xH"] - 0.01
            s.step()
            a1 = s.f["xH"] - 0.01
            fac = np.sum(a1 * a0) / np.sum(a0 * a0)
            assert abs(fac - 1 / (1 + dt * D * lam)) < 1e-10, (k, fac)
            assert np.max(np.abs(a1 - fac * a0)) < 1e-12 * np.max(np.abs(a0))


def test_implicit_oxygen_mode_factor(oracle):
    """Pure wuestite (quadratic free energy, constant M_O = D_O / psi_xx): a
    cosine mode of x_O has explicit tendency -(D lambda + M kappa lambda^2) a;
    with the diffusion implicit the factor per step is exactly
    1 - dt (D lambda + M kappa lambda^2) / (1 + dt D lambda)."""
    p = I.Params(kfor=0.0)
    h = I.H_DEFAULT
    shape = (3, 40)
    k = 3
    D = p.DO[2]
    psi_xx = p.R * p.theta / p.Vmol * 2 * 173.263
    M = D / psi_xx
    lam = 4 / h ** 2 * math.sin(math.pi * k / (2 * shape[-1])) ** 2
    dt = 50 * h * h / (4 * D)
    f = _mode_fields(shape, k, "xO", 0.5, 0.01, phi_w=1.0)
    s = _sim(oracle, 2, shape, h, dt, p, f, mechanics=False, dirichlet=False, implicit=True)
    want = 1 - dt * (D * lam + M * p.kappaO * lam ** 2) / (1 + dt * D * lam)
    for _ in range(3):
        a0 = s.f["xO"] - 0.5
        s.step()
        a1 = s.f["xO"] - 0.5
        fac = np.sum(a1 * a0) / np.sum(a0 * a0)
        assert abs(fac - want) < 1e-10 * abs(want), (fac, want)


@pytest.mark.parametrize("dirichlet", [False, True])
def test_implicit_species_conserve_oxygen_and_hydrogen(oracle, dirichlet):
    """The implicit solve only redistributes (no-flux faces) or exchanges
    through the boundary faces the ledger accounts for, at 100 times the
    explicit time step."""
    wl = I.workload("core_shell_2d", n=24)
    s = _sim(oracle, 2, wl.shape, wl.h, 100 * wl.dt, wl.params, wl.fields, mechanics=True, plasticity=True,
             dirichlet=dirichlet, cg_rtol=1e-10, implicit=True)
    O0 = (s.f["xO"] + s.f["xW"]).sum()
    for _ in range(10):
        st = s.step()
        assert abs(st["O_drift"]) < 1e-12
        assert abs(st["H_drift"]) < 1e-12
    if not dirichlet:
        assert abs((s.f["xO"] + s.f["xW"]).sum() - O0) < 1e-12 * O0
    else:
        assert st["H_out"] < 0


def test_implicit_matches_explicit_to_first_order(oracle):
    """Over a fixed time the implicit and explicit updates differ by O(dt):
    halving the step halves the difference."""
    wl = I.workload("core_shell_2d", n=24)
    T = 32 * wl.dt
    diffs = []
    for m in (8, 4, 2):
        dt = wl.dt * m / 8                      # at most the explicit step
        runs = []
        for implicit in (False, True):
            s = _sim(oracle, 2, wl.shape, wl.h, dt, wl.params, wl.fields, mechanics=False, dirichlet=True,
                     implicit=implicit)
            s.step(int(round(T / dt)))
            runs.append(s.f["xH"] - wl.fields["xH"])
        diffs.append(np.linalg.norm(runs[1] - runs[0]) / np.linalg.norm(runs[0]))
    assert diffs[0] < 0.2
    assert 1.7 < diffs[0] / diffs[1] < 2.3 and 1.7 < diffs[1] / diffs[2] < 2.3, diffs


def test_implicit_is_stable_far_beyond_the_explicit_limit(oracle):
    """At 1000 times the explicit gas-diffusion limit the implicit update of a
    Gaussian of x_H in gas stays bounded and positive and conserves it; the
    explicit update at the same step diverges."""
    p = I.Params(kfor=0.0)
    h = I.H_DEFAULT
    n = 32
    shape = (n, n)
    yy, xx = np.meshgrid(np.arange(n) - n / 2 + 0.5, np.arange(n) - n / 2 + 0.5, indexing="ij")
    f = _uniform_fields(shape, phi_f=0.0, phi_w=0.0)
    f["xH"] = 0.01 * np.exp(-(xx ** 2 + yy ** 2) / 8)
    dt = 1000 * h * h / (4 * p.DH[1])
    s = _sim(oracle, 2, shape, h, dt, p, f, mechanics=False, dirichlet=False, implicit=True)
    m0 = s.f["xH"].sum()
    s.step(5)
    assert np.all(np.isfinite(s.f["xH"])) and s.f["xH"].min() > 0 and s.f["xH"].max() <= 0.01
    assert abs(s.f["xH"].sum() - m0) < 1e-12 * m0
    e = _sim(oracle, 2, shape, h, dt, p, f, mechanics=False, dirichlet=False, implicit=False)
    e.step(5)
    assert not np.all(np.abs(e.f["xH"]) < 1.0)


def test_reaction_is_forward_only(oracle):
    """The rate of Eq. 27 is a forward rate: a cell whose x_O or x_H is below
    zero (the variational O flux leaves gas slightly below x_O = 0) does not
    react, in either direction."""
    p = I.Params(L=(0.0, 0.0, 0.0), DO=(0.0, 0.0, 0.0), DH=(0.0, 0.0, 0.0), DW=(0.0, 0.0, 0.0), kappaO=0.0)
    for xO, xH in ((-0.01, 0.01), (0.3, -0.002), (-0.01, -0.01)):
        f = _uniform_fields((4, 4), phi_f=0.25, phi_w=0.25, xO=xO, xH=xH, xW=0.1)
        s = _sim(oracle, 2, (4, 4), I.H_DEFAULT, 1e-6, p, f, mechanics=False, dirichlet=False)
        s.step(5)
        for k in ("xO", "xH", "xW"):
            assert np.array_equal(s.f[k], f[k]), (xO, xH, k)
    f = _uniform_fields((4, 4), phi_f=0.25, phi_w=0.25, xO=0.3, xH=0.01, xW=0.1)
    s = _sim(oracle, 2, (4, 4), I.H_DEFAULT, 1e-6, p, f, mechanics=False, dirichlet=False)
    s.step()
    assert np.all(s.f["xW"] > 0.1)                     # positive fractions do react


# ---------------------------------------------------------------------------
# Reaction solved exactly over a step (species_implicit = 2)
# ---------------------------------------------------------------------------
def test_exact_reaction_matches_the_closed_form(oracle):
    """Against a 40-digit evaluation of a(t) = c a0 / ((2 a0 + c) e^(c k m t)
    - 2 a0) (and a0 / (1 + 2 a0 k m t) at c = 0), for hydrogen-rich (c > 0),
    oxygen-rich (c < 0) and balanced cells, short and long times."""
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 40
    p = I.Params()
    for a0, b0 in ((0.02, 0.08), (0.5, 0.01), (0.01, 0.02), (0.01, 0.02 + 1e-14), (0.3, 0.3)):
        for m in (1.0, 0.3):
            for t in (1e-7, 1e-4, 1e-2, 10.0):
                R = oracle.reaction_exact(p, m, a0, b0, 0.1, t)
                A, B, K = mpmath.mpf(a0), mpmath.mpf(b0), mpmath.mpf(p.kfor) * m * mpmath.mpf(t)
                cc = B - 2 * A
                a = A / (1 + 2 * A * K) if cc == 0 else cc * A / ((2 * A + cc) * mpmath.exp(cc * K) - 2 * A)
                want = float(A - a)
                assert abs(R - want) <= 1e-12 * max(want, 1e-300) + 1e-300, (a0, b0, m, t, R, want)
                assert 0.0 <= R <= min(a0, b0 / 2) * (1 + 1e-14)


def test_exact_reaction_composes_and_halts(oracle):
    p = I.Params()
    a0, b0 = 0.2, 0.05
    R1 = oracle.reaction_exact(p, 1.0, a0, b0, 0.0, 2e-4)
    R2 = oracle.reaction_exact(p, 1.0, a0 - R1, b0 - 2 * R1, R1, 3e-4)
    R = oracle.reaction_exact(p, 1.0, a0, b0, 0.0, 5e-4)
    assert abs((R1 + R2) - R) < 1e-14 * R                    # reacting t1 then t2 is reacting t1 + t2
    assert oracle.reaction_exact(p, 1.0, a0, b0, 1.0, 1.0) == 0.0     # full of water
    assert oracle.reaction_exact(p, 1.0, -1e-3, b0, 0.0, 1.0) == 0.0  # forward only
    assert oracle.reaction_exact(p, 0.0, a0, b0, 0.0, 1.0) == 0.0     # no gas, no reaction


@pytest.mark.parametrize("dt", [1e-6, 1e-3, 1.0])
def test_exact_reaction_step_follows_the_ode_at_any_step(oracle, dt):
    """Uniform closed box (no transport, frozen phases, m(phi_g) = 1): with the
    reaction solved exactly the state after n steps is the ODE's at n dt, for
    any dt (the explicit update diverges or overshoots at the larger ones),
    and O + H2O, H + 2 H2O are unchanged."""
    shape = (4, 5)
    a0, b0, n = 0.02, 0.08, 7
    p = I.Params(L=(0.0, 0.0, 0.0), DO=(0.0, 0.0, 0.0), DH=(0.0, 0.0, 0.0), DW=(0.0, 0.0, 0.0), kappaO=0.0)
    f = _uniform_fields(shape, phi_f=0.25, phi_w=0.25, xO=a0, xH=b0)
    s = _sim(oracle, 2, shape, I.H_DEFAULT, dt, p, f, mechanics=False, dirichlet=False, implicit=2)
    s.step(n)
    c = b0 - 2 * a0
    e = math.exp(-c * p.kfor * n * dt)                  # c > 0: the decaying form
    a = c * a0 * e / ((2 * a0 + c) - 2 * a0 * e)
    assert np.max(np.abs(s.f["xO"] - a)) <= 1e-12 * a0 + 1e-300
    assert np.max(np.abs(s.f["xO"] + s.f["xW"] - a0)) <= 1e-15
    assert np.max(np.abs(s.f["xH"] + 2 * s.f["xW"] - b0)) <= 1e-15
