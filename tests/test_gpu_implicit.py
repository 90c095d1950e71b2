"""The linearly implicit species update on the GPU (through the C ABI)
against the oracle's.  Time steps are tens to a thousand times the explicit
gas-diffusion limit.

Tolerances: FP64 (both species solves to 1e-12 / 1e-13, the equilibrium solve
to 1e-12) as the explicit FP64 parity: fields 1e-12 relative, increments 1e-6
(they inherit the equilibrium solve's tolerance through the elastic driving
force); mixed (species and equilibrium solves to 1e-6, oracle to 1e-10 / 1e-13):
fields 1e-4, increments 1e-3 for phi_f, phi_w and x_H2O and 1e-4 for x_O, x_H
(the gates of the explicit mixed path); element by element 1e-4.
"""
import sys

import numpy as np
import pytest

from paper_2111_11538_amd import inputs as I

pytestmark = pytest.mark.gpu
NAMES = ("phi_f", "phi_w", "xO", "xH", "xW")
INCR_TOL = {"phi_f": 1e-3, "phi_w": 1e-3, "xO": 1e-4, "xH": 1e-4, "xW": 1e-3}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / nb if nb > 0 else np.linalg.norm(a - b)


def _pair(oracle, dim, shape, f, p, dt, steps, precision, g_rtol, o_rtol, sp_rtol, mechanics=True, dirichlet=True):
    from paper_2111_11538_amd import pf
    say(f"implicit species: dim={dim} shape={shape} {precision} dt={dt:.3e} steps={steps}")
    h = I.H_DEFAULT
    o = oracle.OracleSim(dim, shape, h, dt, p, f, mechanics=mechanics, plasticity=True, dirichlet=dirichlet,
                         cg_rtol=o_rtol, implicit=True)
    g = pf.Context(dim, shape, h, dt, p, precision=precision, mechanics=mechanics, plasticity=True,
                   dirichlet=dirichlet, cg_rtol=g_rtol, species_implicit=True, species_rtol=sp_rtol)
    g.set_fields(f)
    f0 = {k: np.array(f[k], dtype=np.float64) for k in NAMES}
    for _ in range(steps):
        ost = o.step()
        gst = g.step()
    out = g.fields()
    g.close()
    return o, ost, out, gst, f0


@pytest.mark.parametrize("dim,n", [(2, 64), (3, 20)])
def test_fp64_implicit_core_shell(oracle, dim, n):
    wl = I.workload("core_shell_2d" if dim == 2 else "core_shell_3d", n=n)
    o, ost, out, gst, f0 = _pair(oracle, dim, wl.shape, wl.fields, wl.params, 50 * wl.dt, 6, "fp64", 1e-12, 1e-12,
                                 1e-12)
    for k in NAMES:
        assert rel(out[k], o.f[k]) < 1e-12, k
        d = o.f[k] - f0[k]
        if np.linalg.norm(d) > 0:
            assert rel(out[k] - f0[k], d) < 1e-6, (k, rel(out[k] - f0[k], d))
    assert rel(out["ux"], o.ux) < 1e-7
    assert abs(gst["O_drift"]) < 1e-12 and abs(gst["H_drift"]) < 1e-12
    assert abs(gst["red_degree"] - ost["red_degree"]) < 1e-12
    assert gst["species_iters"] > 0


@pytest.mark.parametrize("dim,n", [(2, 40), (3, 12)])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_implicit_random_fields_elementwise(oracle, dim, n, precision):
    """All-phase random fields with 5 % of the cells at x_H2O >= 1, three
    steps at 20 times the explicit limit, element by element."""
    rng = np.random.default_rng(50 + dim)
    shape = (n,) * dim
    f = {"phi_f": rng.uniform(0.05, 0.5, shape), "phi_w": rng.uniform(0.05, 0.45, shape),
         "xO": rng.uniform(0.0, 0.5, shape), "xH": rng.uniform(0.0, 0.02, shape),
         "xW": rng.uniform(0.0, 0.05, shape)}
    wet = rng.random(shape) < 0.05
    f["xW"][wet] = rng.uniform(1.0, 1.2, int(wet.sum()))
    p = I.Params()
    dt = 20 * I.stable_dt(p, I.H_DEFAULT, dim)
    if precision == "fp64":
        o, ost, out, gst, f0 = _pair(oracle, dim, shape, f, p, dt, 3, "fp64", 1e-12, 1e-12, 1e-12)
        tol = 1e-8
    else:
        o, ost, out, gst, f0 = _pair(oracle, dim, shape, f, p, dt, 3, "mixed", 1e-6, 1e-10, 1e-6)
        tol = 1e-4
    for k in NAMES:
        db = o.f[k] - f0[k]
        err = np.max(np.abs((out[k] - f0[k]) - db)) / np.max(np.abs(db))
        say(precision, k, f"elementwise increment error {err:.2e}")
        assert err < tol, (k, err)
    assert gst["nonfinite"] == 0


@pytest.mark.parametrize("name,n", [("core_shell_2d", 64), ("core_shell_3d", 24), ("porous_3d", 32)])
def test_mixed_implicit_increments(oracle, name, n):
    wl = I.workload(name, n=n)
    o, ost, out, gst, f0 = _pair(oracle, wl.dim, wl.shape, wl.fields, wl.params, 50 * wl.dt, 6, "mixed", 1e-6, 1e-10,
                                 1e-6)
    for k in NAMES:
        b = o.f[k]
        rms = np.sqrt(np.mean(b * b))
        fe = rel(out[k], b) if rms >= 1e-6 else np.sqrt(np.mean((out[k] - b) ** 2))
        assert fe < 1e-4, (k, fe)
        db, da = b - f0[k], out[k] - f0[k]
        if np.sqrt(np.mean(db * db)) < 1e-12:
            assert np.sqrt(np.mean((da - db) ** 2)) < 1e-15, k
        else:
            say(k, f"increment error {rel(da, db):.2e}")
            assert rel(da, db) < INCR_TOL[k], (k, rel(da, db))
    # the species CG stops at rtol 1e-6: the increment's sum is conserved up to
    # the residual's sum, below rtol of the solve's right-hand side per step
    assert abs(gst["O_drift"]) < 6 * 1e-6


def test_implicit_is_stable_far_beyond_the_explicit_limit():
    """A Gaussian of x_H in gas at 1000 times the explicit limit: bounded,
    positive and conserved (closed box), on the GPU."""
    from paper_2111_11538_amd import pf
    p = I.Params(kfor=0.0)
    h = I.H_DEFAULT
    n = 48
    yy, xx = np.meshgrid(np.arange(n) - n / 2 + 0.5, np.arange(n) - n / 2 + 0.5, indexing="ij")
    f = {k: np.zeros((n, n)) for k in NAMES}
    f["xH"] = 0.01 * np.exp(-(xx ** 2 + yy ** 2) / 8)
    dt = 1000 * h * h / (4 * p.DH[1])
    g = pf.Context(2, (n, n), h, dt, p, precision="fp64", mechanics=False, dirichlet=False, species_implicit=True)
    g.set_fields(f)
    st = g.step(5)
    x = g.get("xH")
    g.close()
    assert np.all(np.isfinite(x)) and x.min() > 0 and x.max() <= 0.01
    assert abs(x.sum() - f["xH"].sum()) < 1e-12 * f["xH"].sum()
    assert abs(st["H_drift"]) < 1e-12


def test_implicit_error_paths():
    from paper_2111_11538_amd import pf
    wl = I.workload("core_shell_2d", n=24)
    g = pf.Context(2, wl.shape, wl.h, 50 * wl.dt, wl.params, species_implicit=True, species_max_iter=1,
                   species_rtol=1e-14)
    g.set_fields(wl.fields)
    with pytest.raises(pf.PFError) as e:
        g.step()
    assert e.value.status == pf.PF_ERR_CG_NOT_CONVERGED
    g.close()
    with pytest.raises(pf.PFError) as e:
        pf.Context(2, wl.shape, wl.h, wl.dt, wl.params, species_implicit=True, species_rtol=0.0)
    assert e.value.status == pf.PF_ERR_INVALID_ARG
    with pytest.raises(pf.PFError) as e:
        pf.Batch([(24, 24)], wl.h, wl.dt, wl.params, species_implicit=True)
    assert e.value.status in (pf.PF_ERR_UNSUPPORTED, pf.PF_ERR_INVALID_ARG)


@pytest.mark.parametrize("dim,n,dt", [(2, 64, 1e-3), (3, 20, 1e-3), (2, 48, 1e-2)])
def test_fp64_split_reaction_core_shell(oracle, dim, n, dt):
    """species_implicit = 2 (implicit transport, then the reaction solved
    exactly per cell) at time steps up to 1e-2 s, 500 000 times the explicit
    limit, against the oracle's."""
    from paper_2111_11538_amd import pf
    wl = I.workload("core_shell_2d" if dim == 2 else "core_shell_3d", n=n)
    h = I.H_DEFAULT
    o = oracle.OracleSim(dim, wl.shape, h, dt, wl.params, wl.fields, plasticity=True, cg_rtol=1e-12, implicit=2)
    g = pf.Context(dim, wl.shape, h, dt, wl.params, precision="fp64", plasticity=True, cg_rtol=1e-12,
                   species_implicit=2, species_rtol=1e-12)
    g.set_fields(wl.fields)
    for _ in range(8):
        ost = o.step()
        gst = g.step()
    out = g.fields()
    g.close()
    # at these steps the increments are large and the solves' tolerance (1e-12
    # on both sides) sets the agreement: fields to 1e-10; the ledgers close to
    # the species solve's residual, 1e-12 of a right-hand side dt T(x^n) that
    # holds the stiff explicit tendency (up to ~1e5 times the increment at
    # 1e-2 s): 1e-8
    for k in NAMES:
        assert rel(out[k], o.f[k]) < 1e-10, k
        d = o.f[k] - wl.fields[k]
        if np.linalg.norm(d) > 0:
            assert rel(out[k] - wl.fields[k], d) < 1e-6, (k, rel(out[k] - wl.fields[k], d))
    assert abs(gst["O_drift"]) < 1e-8 and abs(gst["H_drift"]) < 1e-8
    assert abs(gst["red_degree"] - ost["red_degree"]) < 1e-10 * max(1.0, abs(ost["red_degree"]))
    assert gst["red_degree"] > 0


def test_mixed_split_reaction_increments(oracle):
    wl = I.workload("core_shell_2d", n=64)
    o, ost, out, gst, f0 = _pair_mode(oracle, wl, 1e-3, 10, "mixed", 2)
    for k in NAMES:
        db, da = o.f[k] - f0[k], out[k] - f0[k]
        if np.sqrt(np.mean(db * db)) < 1e-12:
            assert np.sqrt(np.mean((da - db) ** 2)) < 1e-15, k
        else:
            say(k, f"increment error {rel(da, db):.2e}")
            assert rel(da, db) < INCR_TOL[k], (k, rel(da, db))


def _pair_mode(oracle, wl, dt, steps, precision, mode):
    from paper_2111_11538_amd import pf
    h = I.H_DEFAULT
    o = oracle.OracleSim(wl.dim, wl.shape, h, dt, wl.params, wl.fields, plasticity=True, cg_rtol=1e-10, implicit=mode)
    g = pf.Context(wl.dim, wl.shape, h, dt, wl.params, precision=precision, plasticity=True, cg_rtol=1e-6,
                   species_implicit=mode, species_rtol=1e-6)
    g.set_fields(wl.fields)
    f0 = {k: np.array(wl.fields[k], dtype=np.float64) for k in NAMES}
    for _ in range(steps):
        ost = o.step()
        gst = g.step()
    out = g.fields()
    g.close()
    return o, ost, out, gst, f0
