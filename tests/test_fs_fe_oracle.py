"""Pins of the finite-element finite-strain oracle (`oracle/fs_fe_oracle.py`):
the batched constitutive law equals the pointwise one, the nodal residual is
the derivative of the discrete energy, a homogeneous deformation leaves the
interior nodes in balance, a laminate under rollers reproduces the 1D
finite-strain solution exactly, and a misfitting core-shell disk converges
under refinement to the radially symmetric finite-strain solution, found
independently by shooting on its equilibrium ODE."""
import numpy as np
import pytest
from scipy.integrate import solve_ivp
from scipy.optimize import brentq

from paper_2111_11538_amd import inputs as I
from oracle import fs_fe_oracle as FE
from oracle import fs_oracle as FS


def _unimodular(rng, amp, n=()):
    A = rng.normal(0, amp, n + (3, 3))
    A = 0.5 * (A + np.swapaxes(A, -1, -2))
    A -= (np.trace(A, axis1=-2, axis2=-1) / 3)[..., None, None] * np.eye(3)
    return FE.expm_sym_b(A)


def test_batched_law_equals_pointwise():
    rng = np.random.default_rng(3)
    p = I.Params()
    n = 12
    F = np.eye(3) + rng.normal(0, 0.1, (n, 3, 3))
    Fp = _unimodular(rng, 0.05, (n,))
    pf, pw = rng.uniform(0, 0.6, n), rng.uniform(0, 0.35, n)
    Pb, Eb, Mb = FE.piola_b(F, pf, pw, Fp, p), FE.energy_b(F, pf, pw, Fp, p), FE.mandel_b(F, pf, pw, Fp, p)
    for i in range(n):
        P = FS.piola(F[i], pf[i], pw[i], Fp[i], p)
        assert np.max(np.abs(Pb[i] - P)) < 1e-12 * np.max(np.abs(P))
        e = FS.energy(F[i], pf[i], pw[i], Fp[i], p)
        assert abs(Eb[i] - e) < 1e-12 * abs(e)
        M = FS.mandel(F[i], pf[i], pw[i], Fp[i], p)
        assert np.max(np.abs(Mb[i] - M)) < 1e-12 * np.max(np.abs(M))


def test_batched_return_map_equals_pointwise():
    p = I.Params()
    gs = np.array([0.0, 0.004, 0.02, 0.05, 0.12])
    F = np.zeros((len(gs), 3, 3))
    F[...] = np.eye(3)
    F[:, 0, 1] = gs
    pf, pw = np.array([0.0, 0.2, 0.0, 1.0, 0.1]), np.array([1.0, 0.7, 1.0, 0.0, 0.8])
    Fp0, e0 = FE.identity_plastic((len(gs),), 0)
    Fp0, e0 = Fp0[:, 0], np.array([0.0, 0.0, 0.01, 0.0, 0.02])
    Fb, eb, db = FE.return_map_b(F, pf, pw, Fp0, e0, p)
    for i in range(len(gs)):
        Fq, eq, dq = FS.return_map(F[i], pf[i], pw[i], Fp0[i], e0[i], p)
        assert abs(dq - db[i]) <= 1e-12 * max(dq, 1e-30)
        assert np.max(np.abs(Fq - Fb[i])) < 1e-12
    assert np.count_nonzero(db) >= 2


def _grid(dim, shape, rng, plastic_amp=0.0):
    p = I.Params()
    pf = rng.uniform(0, 0.7, shape)
    pw = rng.uniform(0, 1, shape) * (1 - pf)
    g = FE.FEGrid(dim, shape, 1e-7, p, pf, pw)
    Fp, eP = FE.identity_plastic(shape, dim)
    if plastic_amp:
        Fp = _unimodular(rng, plastic_amp, tuple(shape) + (1 << dim,))
    return g, Fp


@pytest.mark.parametrize("dim,shape", [(2, (3, 4)), (3, (2, 2, 3))])
def test_residual_is_the_energy_gradient(dim, shape):
    rng = np.random.default_rng(7 + dim)
    g, Fp = _grid(dim, shape, rng, plastic_amp=0.03)
    u = rng.normal(0, 4e-9, (dim,) + g.nodes)
    u[g.fixed] = 0.0
    R = g.residual(u, Fp)
    d = 1e-12
    idx = np.argwhere(g.free)
    for q in idx[:: max(1, len(idx) // 25)]:
        q = tuple(q)
        up, um = u.copy(), u.copy()
        up[q] += d
        um[q] -= d
        fd = (g.energy(up, Fp) - g.energy(um, Fp)) / (2 * d)
        assert abs(fd - R[q]) < 1e-6 * np.max(np.abs(R)), (q, fd, R[q])
    assert np.all(R[g.fixed] == 0)


@pytest.mark.parametrize("dim,shape", [(2, (5, 6)), (3, (3, 3, 4))])
def test_homogeneous_deformation_balances_interior_nodes(dim, shape):
    """Uniform phases and a homogeneous F0: every interior node gets no net
    force (the gradients of its shape functions sum to zero over its cells)."""
    p = I.Params()
    pf = np.full(shape, 0.3)
    pw = np.full(shape, 0.5)
    g = FE.FEGrid(dim, shape, 1e-7, p, pf, pw)
    F0 = np.eye(3)
    F0[:dim, :dim] += np.array([[0.05, 0.02, 0.01], [-0.03, -0.04, 0.02], [0.01, 0.0, 0.03]])[:dim, :dim]
    coords = np.meshgrid(*[np.arange(n + 1) * 1e-7 for n in reversed(shape)], indexing="ij")
    coords = [c.transpose(tuple(reversed(range(dim)))) for c in coords]     # coordinate c on the node array
    u = np.zeros((dim,) + g.nodes)
    for i in range(dim):
        for j in range(dim):
            u[i] += (F0[i, j] - (i == j)) * coords[j]
    Fp, _ = FE.identity_plastic(shape, dim)
    F = g.deformation_gradient(u)
    assert np.max(np.abs(F - F0)) < 1e-12
    R = g.forces(FE.piola_b(F, np.full(F.shape[:-2], 0.3), np.full(F.shape[:-2], 0.5), Fp, p))
    inner = tuple(slice(1, -1) for _ in range(dim))
    scale = np.max(np.abs(R))
    assert scale > 0
    assert np.max(np.abs(R[(slice(None),) + inner])) < 1e-10 * scale


def test_laminate_under_rollers_is_the_1d_solution():
    """Layers stacked along x (2D, plane strain, rollers): the Newton solution
    has F = diag(lam_i, 1, 1) per layer with lam_i and P_xx of the 1D
    laminate of `fs_oracle`, to the solver's tolerance."""
    layer = np.array([0, 0, 1, 2, 2, 0, 1, 2])
    p = I.Params(Omega_f=0.4)
    n = len(layer)
    pf = np.tile((layer == 0).astype(float), (3, 1))
    pw = np.tile((layer == 2).astype(float), (3, 1))
    g = FE.FEGrid(2, (3, n), 1e-7, p, pf, pw)
    Fp, _ = FE.identity_plastic((3, n), 2)
    u, it, rr = g.solve(np.zeros((2,) + g.nodes), Fp, rtol=1e-13)
    assert rr < 1e-13 and it < 20
    lam, P = FS.laminate((layer == 0).astype(float), (layer == 2).astype(float), p)
    F = g.deformation_gradient(u)
    got = F[..., 0, 0].mean(axis=(0, 2))
    assert np.max(np.abs(got - lam)) < 1e-10, (got, lam)
    assert np.max(np.abs(F[..., 1, 1] - 1)) < 1e-12 and np.max(np.abs(F[..., 0, 1])) < 1e-12
    Pxx = FE.piola_b(F, np.broadcast_to(pf[..., None], F.shape[:-2]), np.broadcast_to(pw[..., None], F.shape[:-2]),
                     Fp, p)[..., 0, 0]
    assert np.max(np.abs(Pxx - P)) < 1e-8 * abs(P) + 1.0


def _radial_core_stretch(p, a, b, R_out):
    """Plane-strain radial deformation r(R) of a wuestite core (R < a), a
    transformed ferrite shell (a < R < b) and gas (b < R < R_out) with r(R_out)
    = R_out: F = diag(r', r/R, 1); Div P = 0 reads dP_RR/dR + (P_RR - P_TT)/R
    = 0; the core deforms homogeneously (r = lam R).  Shooting on lam."""
    mats = [(0.0, 1.0), (1.0, 0.0), (0.0, 0.0)]        # (phi_f, phi_w) of core, shell, gas
    I3 = np.eye(3)

    def P(fr, ft, m):
        return FS.piola(np.diag([fr, ft, 1.0]), m[0], m[1], I3, p)

    def dPrr(fr, ft, m):
        e = 1e-6
        d1 = (P(fr + e, ft, m)[0, 0] - P(fr - e, ft, m)[0, 0]) / (2 * e)
        d2 = (P(fr, ft + e, m)[0, 0] - P(fr, ft - e, m)[0, 0]) / (2 * e)
        return d1, d2

    def rhs(R, y, m):
        r, rp = y
        Pm = P(rp, r / R, m)
        d1, d2 = dPrr(rp, r / R, m)
        return [rp, (-(Pm[0, 0] - Pm[1, 1]) / R - d2 * (rp - r / R) / R) / d1]

    def match(Prr, ft, m):
        return brentq(lambda fr: P(fr, ft, m)[0, 0] - Prr, 1e-3, 1e3, xtol=1e-15)

    def end(lam):
        r, Prr = lam * a, P(lam, lam, mats[0])[0, 0]
        for (R0, R1), m in (((a, b), mats[1]), ((b, R_out), mats[2])):
            rp = match(Prr, r / R0, m)
            sol = solve_ivp(rhs, (R0, R1), [r, rp], args=(m,), rtol=1e-11, atol=1e-14 * R_out)
            r, rp = sol.y[0, -1], sol.y[1, -1]
            Prr = P(rp, r / R1, m)[0, 0]
        return r - R_out

    return brentq(end, 0.9, 1.1, xtol=1e-14)


def _small_strain_core_stretch(p, a, b, R_out):
    """The small-strain (Lame) plane-strain answer for the same disk: u_r = A r
    + B / r per layer, eigenstrain e in the shell, u_r and sigma_rr
    continuous, u_r(R_out) = 0; returns 1 + A_core."""
    dT = 1 - p.Omega_f
    layers = [(a, p.K[2], p.G[2], 0.0), (b, dT * p.K[0], dT * p.G[0], dT ** (1 / 3) - 1), (R_out, p.K[1], p.G[1], 0.0)]
    M = np.zeros((6, 6))
    rhs = np.zeros(6)
    M[0, 1] = 1.0
    row = 1
    for k in range(2):
        r, (Kk, Gk, ek), (Kn, Gn, en) = layers[k][0], layers[k][1:], layers[k + 1][1:]
        M[row, 2 * k:2 * k + 4] = [r, 1 / r, -r, -1 / r]
        row += 1
        M[row, 2 * k:2 * k + 4] = [2 * (Kk + Gk / 3), -2 * Gk / r ** 2, -2 * (Kn + Gn / 3), 2 * Gn / r ** 2]
        rhs[row] = 3 * Kk * ek - 3 * Kn * en
        row += 1
    M[row, 4:6] = [R_out, 1 / R_out]
    return 1 + np.linalg.solve(M, rhs)[0]


@pytest.mark.slow
def test_core_shell_disk_converges_to_the_radial_solution():
    """Finite-strain Lame: the core's stretch F_xx from the FE solution
    approaches the radial ODE solution under refinement (staircase
    boundaries: first order), and the finite-strain stretch differs from the
    small-strain one by several times the remaining discretisation error."""
    p = I.Params(Omega_f=0.4)
    errs = []
    for n in (16, 32, 48):
        a, b = 0.25 * n, 0.375 * n
        f = I.ic_core_shell((n, n), r_core=a, r_shell=b)
        h = 1e-7
        g = FE.FEGrid(2, (n, n), h, p, f["phi_f"], f["phi_w"])
        Fp, _ = FE.identity_plastic((n, n), 2)
        u, it, rr = g.solve(np.zeros((2,) + g.nodes), Fp, rtol=1e-12)
        assert rr < 1e-12
        lam = _radial_core_stretch(p, a * h, b * h, n / 2 * h)
        F = g.deformation_gradient(u)
        c = np.arange(n) + 0.5 - n / 2
        yy, xx = np.meshgrid(c, c, indexing="ij")
        inner = xx ** 2 + yy ** 2 < (0.5 * a) ** 2
        fxx = F[..., 0, 0].mean(axis=-1)[inner].mean()
        errs.append(abs(fxx - lam) / abs(lam - 1))
    assert errs[-1] < 0.03, errs
    assert errs[-1] < errs[1] < errs[0], errs
    small = _small_strain_core_stretch(p, a * h, b * h, n / 2 * h)
    assert abs(small - lam) > 5 * errs[-1] * abs(lam - 1), (small, lam)


# ---------------------------------------------------------------------------
# the phase-field step driven by the finite-strain mechanics
# ---------------------------------------------------------------------------
def test_external_driving_force_enters_allen_cahn(oracle):
    """A uniform box without chemistry, gradients or mechanics: the step moves
    phi_f and phi_w by exactly -dt L (barrier terms + the external driving
    force), so adding g moves them by -dt L g (Eq. 29, phase lines)."""
    p = I.Params()
    shape = (3, 4)
    f = {"phi_f": np.full(shape, 0.3), "phi_w": np.full(shape, 0.5), "xO": np.full(shape, 0.2),
         "xH": np.zeros(shape), "xW": np.zeros(shape)}
    dt = 1e-6
    a = oracle.OracleSim(2, shape, 1e-7, dt, p, f, mechanics=False, chem_phase=False, dirichlet=False)
    a.step()
    b = oracle.OracleSim(2, shape, 1e-7, dt, p, f, mechanics=False, chem_phase=False, dirichlet=False)
    g = np.concatenate([np.full(12, 3.0e6), np.full(12, -2.0e6)])
    keep = g.copy()
    b.cfg.gext = keep.ctypes.data_as(oracle.C.POINTER(oracle.C.c_double))
    b.step()
    df = b.f["phi_f"] - a.f["phi_f"]
    dw = b.f["phi_w"] - a.f["phi_w"]
    # the difference of two fields near 0.3 carries their rounding: 1e-6 of the 4.5e-10 shift
    assert np.allclose(df, -dt * p.L[0] * 3.0e6, rtol=1e-6, atol=0)
    assert np.allclose(dw, -dt * p.L[2] * -2.0e6, rtol=1e-6, atol=0)


def test_energy_decreases_with_finite_strain_mechanics(oracle):
    """Eq. 26 with the finite-strain mechanics: without reaction, Dirichlet
    faces and chemical energy (species frozen), the barrier and gradient
    energy plus the finite-strain elastic energy at equilibrium never
    increases, and the elastic part takes a share of the drop."""
    p = I.Params(kfor=0.0, DO=(0.0, 0.0, 0.0), DH=(0.0, 0.0, 0.0), DW=(0.0, 0.0, 0.0))
    n = 16
    f = I.ic_core_shell((n, n), r_core=4.5, frame=0, noise_seed=5)
    f["xO"] = np.where(f["phi_w"] > 0.5, 0.45, 0.05)
    s = oracle.OracleSim(2, (n, n), I.H_DEFAULT, 1e-2, p, f, plasticity=False, dirichlet=False, chem_phase=False,
                         finite_strain=True, fs_rtol=1e-12)
    s.fs_solve()
    E, Eel = [s.energy() + s.fs_energy()], [s.fs_energy()]
    for _ in range(15):
        s.step()
        s.fs_solve()                  # the elastic energy at equilibrium with the new phases
        E.append(s.energy() + s.fs_energy())
        Eel.append(s.fs_energy())
    dE = np.diff(E)
    assert np.all(dE <= 1e-10 * abs(E[0])), dE
    assert E[-1] < E[0]
    assert Eel[-1] < Eel[0]
