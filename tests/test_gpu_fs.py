"""Finite-strain mechanics on the GPU (pf_fs_*) against the finite-element
oracle (`oracle/fs_fe_oracle.py`), through the C ABI.

Tolerances: both sides solve R(u) = 0 of the same discretisation; the GPU's
Newton stops at ||R|| <= 1e-11 ||R(0)|| (the oracle at 1e-13), so the
displacements agree to the conditioning times that: 1e-8 relative; the GPU
displacement is also checked in the oracle's own residual (1e-10 of ||R(0)||).
Stresses, driving forces and plastic updates follow from u at the same
relative level (1e-7); the return map's bisection stops at 1e-13 of dl.
"""
import sys

import numpy as np
import pytest

from paper_2111_11538_amd import inputs as I
from oracle import fs_fe_oracle as FE
from oracle import fs_oracle as FS

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _gpu(dim, shape, h, p, pf, pw, **kw):
    from paper_2111_11538_amd import pf as P
    g = P.FiniteStrain(dim, shape, h, p, **kw)
    g.set("phi_f", pf)
    g.set("phi_w", pw)
    return g


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _core_shell(dim, n, rng_seed=None):
    if dim == 2:
        f = I.ic_core_shell((n, n), r_core=0.25 * n, r_shell=0.375 * n, noise_seed=rng_seed)
    else:
        f = I.ic_core_shell((n, n, n), r_core=0.25 * n, r_shell=0.375 * n, noise_seed=rng_seed)
    return f["phi_f"], f["phi_w"]


@pytest.mark.parametrize("dim,n", [(2, 24), (3, 8)])
def test_elastic_core_shell_matches_oracle(dim, n):
    p = I.Params(Omega_f=0.4)
    h = 1e-7
    pf, pw = _core_shell(dim, n, rng_seed=I.SEED_BASE + 7)
    shape = (n,) * dim
    say(f"finite strain elastic dim={dim} n={n}")
    g = _gpu(dim, shape, h, p, pf, pw, newton_rtol=1e-11)
    st = g.solve()
    u = g.get("u")
    drive = g.get("drive")
    g.close()
    o = FE.FEGrid(dim, shape, h, p, pf, pw)
    Fp, _ = FE.identity_plastic(shape, dim)
    uo, it, rr = o.solve(np.zeros((dim,) + o.nodes), Fp, rtol=1e-13)
    say(f"gpu newton {st['newton_iters']} cg {st['cg_iters']} rel {st['rel_resid']:.2e}; oracle newton {it}")
    assert st["rel_resid"] <= 1e-11 and st["newton_iters"] <= 12
    assert rel(u, uo) < 1e-8, rel(u, uo)
    r0 = np.linalg.norm(o.residual(np.zeros_like(uo), Fp))
    assert np.linalg.norm(o.residual(u, Fp)) < 1e-10 * r0
    gf, gw = o.driving_forces(uo, Fp)
    assert rel(drive[0], gf) < 1e-7 and rel(drive[1], gw) < 1e-7
    vm = o.max_von_mises(uo, Fp)
    assert abs(st["max_vm"] - vm) < 1e-7 * vm, (st["max_vm"], vm)
    assert st["yielded"] == 0 and st["max_epsP"] == 0.0


@pytest.mark.parametrize("dim,n,omega", [(2, 20, 0.2), (3, 6, 0.2), (3, 8, 0.4)])
def test_plastic_core_shell_matches_oracle_over_two_solves(dim, n, omega):
    """Two solves with the return map in between (the second starts from the
    first's F_P and displacement and from phases moved by hand), against the
    oracle taking the same steps; at Omega_f = 0.4 the first return is a
    large one-step flow (tens of percent of plastic strain)."""
    p = I.Params(Omega_f=omega)
    h = 1e-7
    pf, pw = _core_shell(dim, n, rng_seed=I.SEED_BASE + 8)
    shape = (n,) * dim
    say(f"finite strain plastic dim={dim} n={n}")
    g = _gpu(dim, shape, h, p, pf, pw, plasticity=True, newton_rtol=1e-11)
    o = FE.FEGrid(dim, shape, h, p, pf, pw)
    Fp, eP = FE.identity_plastic(shape, dim)
    uo = np.zeros((dim,) + o.nodes)
    for k in range(2):
        if k == 1:                         # the shell grows inwards by a little
            pf2 = np.clip(pf + 0.15 * pw, 0, 1)
            pw2 = np.clip(pw - 0.15 * pw, 0, 1)
            g.set("phi_f", pf2)
            g.set("phi_w", pw2)
            o = FE.FEGrid(dim, shape, h, p, pf2, pw2)
        st = g.solve()
        uo, it, rr = o.solve(uo, Fp, rtol=1e-13)
        Fp, eP, dl = o.return_map(uo, Fp, eP)
        say(f"solve {k}: gpu newton {st['newton_iters']} yielded {st['yielded']} max epsP {st['max_epsP']:.4e}; "
            f"oracle yielded {np.count_nonzero(dl)}")
        u = g.get("u")
        assert rel(u, uo) < 1e-7, rel(u, uo)
        cnt = np.count_nonzero(dl)
        assert abs(st["yielded"] - cnt) <= max(2, 0.01 * cnt), (st["yielded"], cnt)   # points at the threshold
        eg = g.get("epsP")
        assert np.max(np.abs(eg - eP)) < 1e-7 * max(np.max(eP), 1e-12), np.max(np.abs(eg - eP))
        assert np.max(np.abs(g.get("Fp") - Fp)) < 1e-7 * max(np.max(eP), 1e-12) + 1e-14
        assert abs(st["max_epsP"] - eP.max()) < 1e-7 * eP.max()
    assert st["yielded"] > 0
    dr = g.get("drive")
    gf, gw = o.driving_forces(uo, Fp)
    assert rel(dr[0], gf) < 1e-6 and rel(dr[1], gw) < 1e-6
    g.close()


def test_laminate_is_the_1d_solution():
    layer = np.array([0, 0, 1, 2, 2, 0, 1, 2, 0, 2])
    p = I.Params(Omega_f=0.4)
    n = len(layer)
    pf = np.tile((layer == 0).astype(float), (4, 1))
    pw = np.tile((layer == 2).astype(float), (4, 1))
    g = _gpu(2, (4, n), 1e-7, p, pf, pw, newton_rtol=1e-12)
    g.solve()
    u = g.get("u")
    g.close()
    lam, P = FS.laminate((layer == 0).astype(float), (layer == 2).astype(float), p)
    got = np.diff(u[0][0]) / 1e-7 + 1.0
    assert np.max(np.abs(got - lam)) < 1e-10, (got, lam)
    assert np.max(np.abs(u[1])) < 1e-12 * 1e-7


def test_zero_load_and_errors():
    """Uniform phases without transformation misfit: R(0) = 0 and u = 0;
    invalid field requests are rejected on the host."""
    from paper_2111_11538_amd import pf as P
    p = I.Params(Omega_f=0.4)
    shape = (5, 6)
    g = _gpu(2, shape, 1e-7, p, np.zeros(shape), np.ones(shape))
    g.set("u", np.full((2, 6, 7), 1e-9))
    st = g.solve()
    assert st["newton_iters"] == 0 and np.all(g.get("u") == 0)
    with pytest.raises(P.PFError):
        g._check(P.lib().pf_fs_fields(g.ctx, 5, 1, P.C.c_void_p(g.workspace.data_ptr()), 2 * 30 * 8, 1))
    with pytest.raises(P.PFError):
        g._check(P.lib().pf_fs_fields(g.ctx, 0, 0, P.C.c_void_p(g.workspace.data_ptr()), 8, 1))
    g.close()


def _coupled_pair(oracle, dim, n, precision, plastic, implicit, dt, steps, p, coupled=True):
    from paper_2111_11538_amd import pf as P
    h = I.H_DEFAULT
    shape = (n,) * dim
    f = I.ic_core_shell(shape, r_core=0.3 * n, r_shell=0.4 * n, frame=2 if dim == 2 else 0,
                        noise_seed=I.SEED_BASE + 9)
    say(f"finite strain coupled={coupled} dim={dim} n={n} {precision} plastic={plastic} implicit={implicit} "
        f"steps={steps}")
    kw = dict(species_implicit=implicit, species_rtol=1e-12 if precision == "fp64" else 1e-6) if implicit else {}
    g = P.Context(dim, shape, h, dt, p, precision=precision, mechanics=False, plasticity=plastic,
                  cg_rtol=1e-12 if precision == "fp64" else 1e-6, **kw)
    fs = P.FiniteStrain(dim, shape, h, p, plasticity=plastic, newton_rtol=1e-12)
    if coupled:
        g.attach_fs(fs)
    g.set_fields(f)
    gst = g.step(steps)
    out = g.fields(["phi_f", "phi_w", "xO", "xH", "xW"])
    g.close()
    fs.close()
    o = oracle.OracleSim(dim, shape, h, dt, p, f, mechanics=False, plasticity=plastic, finite_strain=coupled,
                         fs_rtol=1e-13, implicit=implicit)
    ost = o.step(steps)
    return f, out, gst, o, ost


# 3D case: gas diffusivities set to the solids' so that the explicit step
# (the LDS-tiled 3D field update) can take dt large enough for the
# finite-strain driving forces to move the phases well above rounding
_P_SLOW_GAS = dict(DO=(2.16e-11,) * 3, DH=(2.5e-11,) * 3, DW=(2.5e-20, 2.5e-11, 2.5e-20))


@pytest.mark.parametrize("dim,n,precision,plastic,implicit,steps",
                         [(2, 20, "fp64", False, 2, 3), (2, 20, "fp64", True, 2, 3),
                          (3, 8, "fp64", True, 0, 2), (2, 20, "mixed", True, 2, 3)])
def test_coupled_step_matches_oracle(oracle, dim, n, precision, plastic, implicit, steps):
    """Steps whose mechanics is the finite-strain solve (pf_fs_attach) against
    the oracle's coupled mode, field increments to 1e-6 relative in FP64 (the
    driving forces carry the Newton tolerance) and to the mixed gates in
    mixed precision; in FP64 also the part of the phase increments that the
    driving forces make (coupled minus uncoupled run, on both sides), to 1e-6."""
    if dim == 3:
        p = I.Params(Omega_f=0.4, **_P_SLOW_GAS)
        dt = I.stable_dt(p, I.H_DEFAULT, dim)
    else:
        p = I.Params(Omega_f=0.4)
        dt = 3e4 * I.stable_dt(p, I.H_DEFAULT, dim)
    f0, out, gst, o, ost = _coupled_pair(oracle, dim, n, precision, plastic, implicit, dt, steps, p)
    tol_i = {"phi_f": 1e-6, "phi_w": 1e-6, "xO": 1e-6, "xH": 1e-6, "xW": 1e-6} if precision == "fp64" else \
        {"phi_f": 1e-3, "phi_w": 1e-3, "xO": 1e-4, "xH": 1e-4, "xW": 1e-3}
    for k in ("phi_f", "phi_w", "xO", "xH", "xW"):
        db, da = o.f[k] - f0[k], out[k] - f0[k]
        if np.sqrt(np.mean(db * db)) < 1e-12:
            assert np.sqrt(np.mean((da - db) ** 2)) < 1e-14, k
            continue
        err = rel(da, db)
        say(k, f"increment error {err:.2e}")
        assert err < tol_i[k], (k, err)
    assert abs(gst["max_vm"] - ost["max_vm"]) < 1e-6 * ost["max_vm"], (gst["max_vm"], ost["max_vm"])
    if plastic:
        assert abs(gst["max_epsP"] - ost["max_epsP"]) < 1e-6 * ost["max_epsP"]
        assert gst["max_epsP"] > 0
    if precision == "fp64":
        _, out0, _, o0, _ = _coupled_pair(oracle, dim, n, precision, plastic, implicit, dt, steps, p, coupled=False)
        for k in ("phi_f", "phi_w"):
            eo, eg = o.f[k] - o0.f[k], out[k] - out0[k]
            say(k, f"driving-force effect {np.linalg.norm(eo):.3e}, error {rel(eg, eo):.2e}")
            assert np.linalg.norm(eo) > 1e-9 * np.sqrt(eo.size)
            assert rel(eg, eo) < 1e-6, (k, rel(eg, eo))


def test_attach_checks_the_grid_and_the_mechanics():
    from paper_2111_11538_amd import pf as P
    p = I.Params()
    fs = P.FiniteStrain(2, (8, 9), I.H_DEFAULT, p)
    g = P.Context(2, (8, 9), I.H_DEFAULT, 1e-9, p, mechanics=True)
    with pytest.raises(P.PFError):
        g.attach_fs(fs)
    g.close()
    g = P.Context(2, (8, 10), I.H_DEFAULT, 1e-9, p, mechanics=False)
    with pytest.raises(P.PFError):
        g.attach_fs(fs)
    g.close()
    fs.close()
