"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Tolerances (derived from the arithmetic of each path):
  * FP64 path: both sides stop CG at ||b - A u|| <= rtol ||b||; with rtol =
    1e-12 the displacements may differ by the conditioning times rtol, so u is
    compared at 1e-7 relative; the per-step increments of the five fields
    inherit that through the elastic driving force (1e-6 relative); the fields
    themselves agree to 1e-12 relative.
  * Mixed path (FP32 arithmetic, fields held as FP32 pairs, FP64
    reductions): 1e-4 relative field error, the accuracy gate of the target
    metric, and the error of the increment over the run, which exposes lost
    phase-field dynamics: 1e-3 relative for phi_f, phi_w and x_H2O, 1e-4 for
    x_O and x_H.  An increment whose RMS is below 1e-12 (x_H2O where no
    reaction has happened: rounding noise) is held to 1e-15 absolute RMS.
"""
import sys

import numpy as np
import pytest

from paper_2111_11538_amd import inputs as I

pytestmark = pytest.mark.gpu

NAMES = ("phi_f", "phi_w", "xO", "xH", "xW")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / nb if nb > 0 else np.linalg.norm(a - b)


def field_err(a, b):
    """Relative L2 error; for a field whose RMS is below 1e-6 (x_H2O before
    any reaction has happened: rounding noise only) the RMS absolute error."""
    rms = np.sqrt(np.mean(b * b))
    if rms < 1e-6:
        return np.sqrt(np.mean((a - b) ** 2))
    return rel(a, b)


INCR_TOL = {"phi_f": 1e-3, "phi_w": 1e-3, "xO": 1e-4, "xH": 1e-4, "xW": 1e-3}


def incr_err(a, b, a0):
    """Error of the increment a - a0 against b - a0: relative L2, or the RMS
    absolute error where the increment's RMS is below 1e-12."""
    da, db = a - a0, b - a0
    if np.sqrt(np.mean(db * db)) < 1e-12:
        return np.sqrt(np.mean((da - db) ** 2)), True
    return rel(da, db), False


def check_mixed_increments(out, ref, f0, tag=""):
    errs = {}
    for k in NAMES:
        e, absolute = incr_err(out[k], ref[k], f0[k])
        errs[k] = e
        assert e < (1e-15 if absolute else INCR_TOL[k]), (tag, k, e, absolute)
    return errs


def _ctx(dim, shape, h, dt, p, **kw):
    from paper_2111_11538_amd import pf
    return pf.Context(dim, shape, h, dt, p, **kw)


def _run_pair(oracle, dim, shape, fields, p, dt, steps, precision="fp64", plasticity=True, dirichlet=True,
              mechanics=True, rtol=1e-12, h=I.H_DEFAULT):
    say(f"case dim={dim} shape={shape} precision={precision} plasticity={plasticity} steps={steps}")
    o = oracle.OracleSim(dim, shape, h, dt, p, fields, mechanics=mechanics, plasticity=plasticity,
                         dirichlet=dirichlet, cg_rtol=rtol)
    g = _ctx(dim, shape, h, dt, p, precision=precision, mechanics=mechanics, plasticity=plasticity,
             dirichlet=dirichlet, cg_rtol=rtol)
    g.set_fields(fields)
    f0 = {k: np.array(fields[k], dtype=np.float64) for k in NAMES}
    ost = gst = None
    for _ in range(steps):
        ost = o.step()
        gst = g.step()
    out = g.fields()
    g.close()
    return o, ost, out, gst, f0


def _check_fp64(o, ost, out, gst, f0, u_tol=1e-7, inc_tol=1e-6):
    for k in NAMES:
        assert rel(out[k], o.f[k]) < 1e-12, k
        d_or = o.f[k] - f0[k]
        if np.linalg.norm(d_or) > 0:
            assert rel(out[k] - f0[k], d_or) < inc_tol, (k, rel(out[k] - f0[k], d_or))
    assert rel(out["ux"], o.ux) < u_tol
    assert rel(out["uy"], o.uy) < u_tol
    if o.uz is not None:
        assert rel(out["uz"], o.uz) < u_tol
    if np.max(o.epsP) > 0:
        assert rel(out["epsP"], o.epsP) < 1e-6
        assert rel(out["epsp"], o.epsp) < 1e-6
    assert abs(gst["cg_iters"] - ost["cg_iters"]) <= 2, (gst["cg_iters"], ost["cg_iters"])
    assert abs(gst["O_drift"]) < 1e-13 and abs(ost["O_drift"]) < 1e-13
    assert abs(gst["red_degree"] - ost["red_degree"]) < 1e-12
    assert abs(gst["max_vm"] - ost["max_vm"]) <= 1e-6 * ost["max_vm"] + 1.0
    assert gst["nonfinite"] == 0


@pytest.mark.parametrize("shape,plastic", [((24, 24), False), ((64, 64), False), ((43, 67), True)])
def test_fp64_2d_core_shell(oracle, shape, plastic):
    wl = I.workload("core_shell_2d", n=shape[0])
    f = I.ic_core_shell(shape, r_core=0.3 * min(shape), frame=2, noise_seed=I.SEED_BASE + 1)
    res = _run_pair(oracle, 2, shape, f, wl.params, wl.dt, 6, plasticity=plastic)
    _check_fp64(*res)


@pytest.mark.parametrize("shape", [(16, 16, 16), (13, 17, 20)])
def test_fp64_3d_core_shell(oracle, shape):
    n = min(shape)
    f = I.ic_core_shell(shape, r_core=0.35 * n, r_shell=0.43 * n, noise_seed=I.SEED_BASE + 2)
    p = I.Params()
    res = _run_pair(oracle, 3, shape, f, p, I.stable_dt(p, I.H_DEFAULT, 3), 3, plasticity=True)
    _check_fp64(*res)


def test_fp64_2d_porous_ragged(oracle):
    wl = I.workload("porous_2d", n=96)
    res = _run_pair(oracle, 2, wl.shape, wl.fields, wl.params, wl.dt, 4, plasticity=True)
    _check_fp64(*res)


@pytest.mark.parametrize("name,n", [("core_shell_2d", 64), ("core_shell_3d", 24), ("porous_2d", 128),
                                    ("porous_3d", 32)])
def test_mixed_precision_field_error(oracle, name, n):
    """Mixed GPU path (CG to 1e-6) against the oracle solved to 1e-10, ten
    steps of reduced instances of each recipe."""
    wl = I.workload(name, n=n)
    o, ost, out, gst, f0 = _run_pair_rtol(oracle, wl.dim, wl.shape, wl.fields, wl.params, wl.dt, 10, "mixed",
                                          True, g_rtol=1e-6, o_rtol=1e-10)
    errs = {k: field_err(out[k], o.f[k]) for k in NAMES}
    say("mixed field errors", errs)
    incr = check_mixed_increments(out, o.f, f0, name)
    say("mixed increment errors", incr)
    for k in NAMES:
        assert errs[k] < 1e-4, k
    assert rel(out["ux"], o.ux) < 1e-3
    assert gst["nonfinite"] == 0
    assert gst["cg_iters"] > 0


def _run_pair_rtol(oracle, dim, shape, fields, p, dt, steps, precision, plasticity, g_rtol, o_rtol,
                   h=I.H_DEFAULT):
    say(f"case dim={dim} shape={shape} precision={precision} steps={steps} rtol gpu {g_rtol} oracle {o_rtol}")
    o = oracle.OracleSim(dim, shape, h, dt, p, fields, plasticity=plasticity, cg_rtol=o_rtol)
    g = _ctx(dim, shape, h, dt, p, precision=precision, plasticity=plasticity, cg_rtol=g_rtol)
    g.set_fields(fields)
    f0 = {k: np.array(fields[k], dtype=np.float64) for k in NAMES}
    ost = gst = None
    for _ in range(steps):
        ost = o.step()
        gst = g.step()
    out = g.fields()
    g.close()
    return o, ost, out, gst, f0


def test_fp64_core_shell_2d_full_length(oracle):
    """The 64^2 plain-method recipe at its full length: 200 steps, FP64, CG
    to 1e-10, element by element against the oracle."""
    wl = I.workload("core_shell_2d")
    o, ost, out, gst, f0 = _run_pair_rtol(oracle, 2, wl.shape, wl.fields, wl.params, wl.dt, wl.steps, "fp64",
                                          False, g_rtol=1e-10, o_rtol=1e-10)
    for k in NAMES:
        b = o.f[k]
        assert np.max(np.abs(out[k] - b)) <= 1e-11 * np.max(np.abs(b)), k
        db = b - f0[k]
        if np.max(np.abs(db)) > 0:
            assert np.max(np.abs((out[k] - f0[k]) - db)) <= 1e-5 * np.max(np.abs(db)), k
    assert np.max(np.abs(out["ux"] - o.ux)) <= 1e-7 * np.max(np.abs(o.ux))
    assert abs(gst["O_drift"]) < 1e-12
    assert abs(gst["red_degree"] - ost["red_degree"]) < 1e-10
    assert abs(gst["max_vm"] - ost["max_vm"]) <= 1e-6 * ost["max_vm"]


def random_fields(shape, seed, wet=0.05):
    """Every phase present in every cell (each term of the driving forces and
    fluxes exercised), and a fraction `wet` of the cells at x_H2O >= 1, where
    the reaction has stopped (Eq. 27, 28)."""
    rng = np.random.default_rng(seed)
    f = {"phi_f": rng.uniform(0.05, 0.5, shape), "phi_w": rng.uniform(0.05, 0.45, shape),
         "xO": rng.uniform(0.0, 0.5, shape), "xH": rng.uniform(0.0, 0.02, shape),
         "xW": rng.uniform(0.0, 0.05, shape)}
    m = rng.random(shape) < wet
    f["xW"][m] = rng.uniform(1.0, 1.2, int(m.sum()))
    return f


@pytest.mark.parametrize("dim,n", [(2, 40), (3, 12), (2, 67)])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_random_fields_elementwise(oracle, dim, n, precision):
    """All-phase random fields with wet cells, three steps, element by
    element: FP64 to 1e-9 of the largest increment (both sides solve to
    1e-12), mixed to 1e-4 (the oracle solved to 1e-10)."""
    shape = (n,) * dim if dim == 3 else (n, n + 5)
    f = random_fields(shape, 7 + dim + n)
    assert np.mean(f["xW"] >= 1.0) > 0.02
    p = I.Params()
    dt = I.stable_dt(p, I.H_DEFAULT, dim)
    g_rtol, o_rtol = (1e-12, 1e-12) if precision == "fp64" else (1e-6, 1e-10)
    o, ost, out, gst, f0 = _run_pair_rtol(oracle, dim, shape, f, p, dt, 3, precision, True, g_rtol, o_rtol)
    tol = 1e-9 if precision == "fp64" else 1e-4
    for k in NAMES:
        db = o.f[k] - f0[k]
        err = np.max(np.abs((out[k] - f0[k]) - db)) / np.max(np.abs(db))
        say(precision, k, f"elementwise increment error {err:.2e}")
        assert err < tol, (k, err)
    if precision == "mixed":
        check_mixed_increments(out, o.f, f0, "random")
    assert np.max(o.epsP) > 0 and rel(out["epsP"], o.epsP) < (1e-6 if precision == "fp64" else 1e-3)
    assert gst["nonfinite"] == 0


def test_laminate_solve_is_exact(oracle):
    p = I.Params()
    n = 12
    shape = (4, n)
    layer = np.array([0, 0, 1, 1, 1, 2, 2, 0, 0, 1, 2, 2])
    f = {k: np.zeros(shape) for k in NAMES}
    f["phi_f"][...] = (layer == 0)
    f["phi_w"][...] = (layer == 2)
    h = I.H_DEFAULT
    g = _ctx(2, shape, h, 1e-9, p, cg_rtol=1e-14)
    g.set_fields(f)
    st = g.mech_solve("zero")
    ux = g.get("ux")
    g.close()
    dT = np.where(layer == 0, 1 - p.Omega_f, 1.0)
    Kl = dT * np.array([p.K[a] for a in layer])
    Gl = dT * np.array([p.G[a] for a in layer])
    el = np.where(layer == 0, (1 - p.Omega_f) ** (1 / 3) - 1, 0.0)
    Ml = Kl + 4 * Gl / 3
    sig = -np.sum(3 * Kl * el / Ml) / np.sum(1 / Ml)
    sig_num = Ml * np.diff(ux, axis=-1) / h - 3 * Kl * el
    assert np.max(np.abs(sig_num - sig)) < 1e-9 * abs(sig)
    assert st["cg_rel_resid"] < 1e-13


def test_closed_box_conserves_oxygen():
    wl = I.workload("core_shell_2d", n=32)
    g = _ctx(2, wl.shape, wl.h, wl.dt, wl.params, dirichlet=False, plasticity=True)
    g.set_fields(wl.fields)
    st = g.step(20)
    g.close()
    assert abs(st["O_drift"]) < 1e-13 and abs(st["H_drift"]) < 1e-13


def test_determinism_bitwise():
    wl = I.workload("core_shell_3d", n=20)
    outs = []
    for _ in range(2):
        g = _ctx(3, wl.shape, wl.h, wl.dt, wl.params, precision="mixed", plasticity=True, cg_rtol=1e-6)
        g.set_fields(wl.fields)
        st = g.step(3)
        outs.append((g.fields(), st))
        g.close()
    for k in outs[0][0]:
        assert np.array_equal(outs[0][0][k], outs[1][0][k]), k
    assert outs[0][1]["O_tot"] == outs[1][1]["O_tot"]


@pytest.mark.parametrize("precision,implicit", [("fp64", 0), ("mixed", 0), ("mixed", 2)])
def test_checkpoint_restart_is_bitwise(precision, implicit):
    """N steps, every field copied out, a new context set from the copies, N
    more steps: bitwise the state of 2N steps in one context.  The exchange is
    FP64, which holds an FP32 pair exactly; the displacement is part of the
    state, so the restarted solve starts where the other one would."""
    wl = I.workload("core_shell_3d", n=20)
    kw = dict(precision=precision, plasticity=True, cg_rtol=1e-6 if precision == "mixed" else 1e-10,
              species_implicit=implicit)
    dt = wl.dt * (50 if implicit else 1)
    say("checkpoint", precision, implicit)
    g = _ctx(3, wl.shape, wl.h, dt, wl.params, **kw)
    g.set_fields(wl.fields)
    g.step(3)
    g.step(3)
    want = g.fields()
    g.close()
    a = _ctx(3, wl.shape, wl.h, dt, wl.params, **kw)
    a.set_fields(wl.fields)
    a.step(3)
    saved = a.fields()
    a.close()
    b = _ctx(3, wl.shape, wl.h, dt, wl.params, **kw)
    b.set_fields(saved)
    b.step(3)
    got = b.fields()
    b.close()
    for k in want:
        assert np.array_equal(got[k], want[k]), k


def test_field_roundtrip_and_roller_faces():
    shape = (9, 7)
    rng = np.random.default_rng(1)
    g = _ctx(2, shape, I.H_DEFAULT, 1e-9, I.Params())
    for name in ("phi_f", "xO", "epsP"):
        v = rng.standard_normal(shape)
        g.set(name, v)
        assert np.array_equal(g.get(name), v)
    ux = rng.standard_normal((9, 8))
    g.set("ux", ux)
    back = g.get("ux")
    assert np.all(back[:, 0] == 0) and np.all(back[:, -1] == 0)
    assert np.array_equal(back[:, 1:-1], ux[:, 1:-1])
    ep = rng.standard_normal((4,) + shape)
    g.set("epsp", ep)
    assert np.array_equal(g.get("epsp"), ep)
    g.close()


def test_error_paths():
    from paper_2111_11538_amd import pf
    wl = I.workload("core_shell_2d", n=24)
    g = _ctx(2, wl.shape, wl.h, wl.dt, wl.params, cg_max_iter=1, cg_rtol=1e-12)
    g.set_fields(wl.fields)
    with pytest.raises(pf.PFError) as e:
        g.step()
    assert e.value.status == pf.PF_ERR_CG_NOT_CONVERGED
    with pytest.raises(pf.PFError) as e:
        g.step()
    assert e.value.status == pf.PF_ERR_BAD_STATE
    g.close()
    g = _ctx(2, wl.shape, wl.h, wl.dt, wl.params)
    f = dict(wl.fields)
    f["xH"] = f["xH"].copy()
    f["xH"][3, 4] = np.nan
    g.set_fields(f)
    with pytest.raises(pf.PFError) as e:
        g.step()
    assert e.value.status == pf.PF_ERR_NONFINITE
    g.close()
    g = _ctx(2, wl.shape, wl.h, wl.dt, wl.params, precision="mixed", cg_rtol=1e-6, ledger_tol=1e-300)
    g.set_fields(wl.fields)
    with pytest.raises(pf.PFError) as e:
        g.step(5)
    assert e.value.status == pf.PF_ERR_LEDGER
    g.close()
