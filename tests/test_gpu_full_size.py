"""Parity at the benchmark's sizes and launch configurations.

The small parity cases run the 3D apply kernels with one-plane slabs (small
grids halve the slab depth until the grid has enough blocks).  Here the
kernels run as the benchmark runs them: 128^3 (slabs of 8 planes, two tiles
across x) and 256^3 (slabs of 32 planes); the solution of the GPU's solve is
checked against the oracle's own operator and right-hand side (the residual
b - A u evaluated by the oracle), and a ragged grid with two-plane slabs and
an odd last slab is compared with the oracle field by field."""
import sys

import numpy as np
import pytest

from paper_2111_11538_amd import inputs as I

pytestmark = pytest.mark.gpu

U = ("ux", "uy", "uz")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _oracle_residual(oracle, wl, fields, u):
    o = oracle.OracleSim(3, wl.shape, wl.h, wl.dt, wl.params, fields, plasticity=True)
    K, G = o.moduli()
    b = o.rhs()
    q = o.apply(K, G, u)
    rr = sum(float(np.sum((bb - qq) ** 2)) for bb, qq in zip(b, q))
    bb = sum(float(np.sum(x ** 2)) for x in b)
    return np.sqrt(rr / bb)


# FP32 state: CG stops on its recursive residual (rtol), while the true
# residual of the stored FP32 solution levels off near 1e-5 at these sizes;
# the bound is on the true residual.  The oracle's evaluation of that
# residual (FP64, its own operator and right-hand side) must agree with the
# GPU's own to within the FP32 rounding of A u (a few per cent).
# The multigrid-preconditioned cases run the benchmark's preconditioner on
# its full hierarchy (256^3: six levels down to 8^3).
@pytest.mark.parametrize("name,n,precision,rtol,bound,agree,precond", [
    ("core_shell_3d", 128, "mixed", 1e-6, 3e-5, 0.05, "jacobi"),
    ("core_shell_3d", 128, "fp64", 1e-10, 1e-9, 1e-3, "jacobi"),
    ("porous_3d", 256, "mixed", 1e-6, 3e-5, 0.05, "jacobi"),
    ("core_shell_3d", 128, "fp64", 1e-10, 1e-9, 1e-3, "mg"),
    ("porous_3d", 256, "mixed", 1e-6, 3e-5, 0.05, "mg"),
])
def test_full_size_solve_satisfies_the_oracle_equations(oracle, name, n, precision, rtol, bound, agree, precond):
    from paper_2111_11538_amd import pf
    wl = I.workload(name, n=n)
    say(f"case {name} {n}^3 {precision} {precond}: solve from zero, residual by the oracle")
    g = pf.Context(3, wl.shape, wl.h, wl.dt, wl.params, precision=precision, plasticity=True, cg_rtol=rtol,
                   cg_precond=precond)
    g.set_fields(wl.fields)
    st = g.mech_solve("zero")
    u = [g.get(k) for k in U]
    g.close()
    rel = _oracle_residual(oracle, wl, wl.fields, u)
    say(f"  {st['cg_iters']} iterations, GPU true residual {st['cg_rel_resid']:.3e}, oracle residual {rel:.3e}")
    assert st["cg_iters"] > 10
    assert rel <= bound, rel
    assert abs(rel - st["cg_rel_resid"]) <= agree * st["cg_rel_resid"], (rel, st["cg_rel_resid"])


@pytest.mark.parametrize("shape,precond", [((53, 72, 130), "jacobi"), ((52, 72, 132), "mg")])
def test_ragged_grid_with_multi_plane_slabs_matches_oracle(oracle, shape, precond):
    """53 x 72 x 130 cells: three tiles across x (the last 2 columns wide),
    nine tile rows, and slabs of two planes with a last slab of one.  With
    the multigrid preconditioner, 132 x 72 x 52: levels 66 x 36 x 26,
    33 x 18 x 13 and 17 x 9 x 7 (ragged tiles on every level; odd sides from
    the third level on)."""
    from paper_2111_11538_amd import pf
    n = shape[0]
    f = I.ic_core_shell(shape, r_core=0.35 * n, r_shell=0.43 * n, noise_seed=I.SEED_BASE + 7)
    p = I.Params()
    dt = I.stable_dt(p, I.H_DEFAULT, 3)
    say(f"case ragged {shape} fp64 {precond}, one step")
    o = oracle.OracleSim(3, shape, I.H_DEFAULT, dt, p, f, plasticity=True, cg_rtol=1e-10)
    ost = o.step()
    g = pf.Context(3, shape, I.H_DEFAULT, dt, p, precision="fp64", plasticity=True, cg_rtol=1e-10,
                   cg_precond=precond)
    g.set_fields(f)
    gst = g.step()
    out = g.fields()
    g.close()
    of = o.fields()
    for k in U:
        err = np.max(np.abs(out[k] - of[k])) / np.max(np.abs(of[k]))
        assert err <= 1e-6, (k, err)
    for k in ("phi_f", "phi_w", "xO", "xH", "xW"):
        d = out[k] - f[k]
        od = of[k] - f[k]
        scale = max(np.max(np.abs(od)), 1e-300)
        err = np.max(np.abs(d - od)) / scale
        assert err <= 1e-5, (k, err)
    if precond == "jacobi":
        assert abs(gst["cg_iters"] - ost["cg_iters"]) <= 3, (gst["cg_iters"], ost["cg_iters"])
    else:
        say(f"  iterations: mg {gst['cg_iters']}, oracle Jacobi {ost['cg_iters']}")
        assert 3 * gst["cg_iters"] < ost["cg_iters"], (gst["cg_iters"], ost["cg_iters"])
