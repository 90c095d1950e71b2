"""The CG launch loop: results do not depend on where the convergence checks
fall (between chunks of queued launches, or inside a chunk where a launch
finds the recurrence converged), and in 3D, where the solution update of an
iteration is made by the next apply launch, a solve stopped at the iteration
limit holds the same iterate as the oracle's CG after that many iterations."""
import sys

import numpy as np
import pytest

from paper_2111_11538_amd import inputs as I

pytestmark = pytest.mark.gpu

FIELDS = ("phi_f", "phi_w", "xO", "xH", "xW", "ux", "uy", "uz", "epsp", "epsP")


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _ctx(dim, wl, **kw):
    from paper_2111_11538_amd import pf
    c = pf.Context(dim, wl.shape, wl.h, wl.dt, wl.params, **kw)
    c.set_fields(wl.fields)
    return c


@pytest.mark.parametrize("dim,precision", [(3, "mixed"), (3, "fp64"), (2, "mixed")])
def test_results_do_not_depend_on_chunking(dim, precision):
    wl = I.workload("core_shell_3d", n=24) if dim == 3 else I.workload("core_shell_2d", n=48)
    rtol = 1e-6 if precision == "mixed" else 1e-10
    ref = None
    for chunk in (0, 1, 3, 500):
        say(f"case dim={dim} precision={precision} chunk={chunk}")
        c = _ctx(dim, wl, precision=precision, plasticity=True, cg_rtol=rtol)
        c.cg_chunk(chunk)
        iters = []
        for _ in range(3):
            iters.append(c.step(1)["cg_iters"])
        f = c.fields([k for k in FIELDS if not (k == "uz" and dim == 2)])
        c.close()
        assert min(iters) > 1, iters
        if ref is None:
            ref = (f, iters)
            continue
        assert iters == ref[1], (chunk, iters, ref[1])
        for k in f:
            np.testing.assert_array_equal(f[k], ref[0][k], err_msg=f"{k} chunk={chunk}")


def test_chunk_rejects_negative():
    from paper_2111_11538_amd import pf
    wl = I.workload("core_shell_3d", n=12)
    c = _ctx(3, wl, precision="mixed")
    with pytest.raises(pf.PFError) as e:
        c.cg_chunk(-1)
    assert e.value.status == pf.PF_ERR_INVALID_ARG
    c.close()


@pytest.mark.parametrize("iters", [1, 2, 7])
@pytest.mark.parametrize("chunk", [0, 1])
def test_iteration_limit_iterate_matches_oracle(oracle, iters, chunk):
    """Stopped at the limit, u is the CG iterate u_iters: the last update's
    alpha p is still added (3D: by the apply launch the host queues after
    the limit)."""
    from paper_2111_11538_amd import pf
    wl = I.workload("core_shell_3d", n=12)
    say(f"case iters={iters} chunk={chunk}")
    o = oracle.OracleSim(3, wl.shape, wl.h, wl.dt, wl.params, wl.fields, plasticity=True, cg_rtol=1e-14,
                         cg_max_iter=iters)
    with pytest.raises(RuntimeError):
        o.mech_solve()
    g = _ctx(3, wl, precision="fp64", plasticity=True, cg_rtol=1e-14, cg_max_iter=iters)
    g.cg_chunk(chunk)
    with pytest.raises(pf.PFError) as e:
        g.mech_solve("zero")
    assert e.value.status == pf.PF_ERR_CG_NOT_CONVERGED
    of = o.fields()
    for k in ("ux", "uy", "uz"):
        a, b = g.get(k), of[k]
        err = np.max(np.abs(a - b)) / np.max(np.abs(b))
        assert np.max(np.abs(b)) > 0 and err <= 1e-10, (k, err)
    g.close()


def test_preconditioner_after_few_iterations_matches_oracle(oracle):
    """The iterate after three Jacobi-preconditioned iterations depends on
    every entry of D^-1: on a grid of many tiles and slabs, repeated solves
    from zero must all match the oracle's (the set-up pass once read the
    moduli of its neighbours after other waves had started to overwrite
    them with the next plane's)."""
    from paper_2111_11538_amd import pf
    wl = I.workload("core_shell_3d", n=48)
    o = oracle.OracleSim(3, wl.shape, wl.h, wl.dt, wl.params, wl.fields, plasticity=True, cg_rtol=1e-14,
                         cg_max_iter=3)
    with pytest.raises(RuntimeError):
        o.mech_solve()
    of = o.fields()
    g = _ctx(3, wl, precision="fp64", plasticity=True, cg_rtol=1e-14, cg_max_iter=3)
    for rep in range(4):
        say(f"case 48^3 fp64, 3 iterations, repeat {rep}")
        with pytest.raises(pf.PFError):
            g.mech_solve("zero")
        for k in ("ux", "uy", "uz"):
            a, b = g.get(k), of[k]
            err = np.max(np.abs(a - b)) / np.max(np.abs(b))
            assert err <= 1e-10, (rep, k, err)
    g.close()


def test_learned_steps_are_bitwise_repeatable():
    """Identical runs with the learned start (network weights that
    reproduce linear extrapolation) give bitwise-equal states."""
    from paper_2111_11538_amd import pf, learned as LR
    n = 64
    wl = I.workload("core_shell_3d", n=n)
    net = pf.Net(max_voxels=n ** 3, seed=5)
    LR.init_extrapolation(net)
    outs = []
    try:
        for rep in range(3):
            say(f"case learned 64^3 mixed, run {rep}")
            c = _ctx(3, wl, precision="mixed", plasticity=True, cg_rtol=1e-6, warm="learned")
            net.attach(c)
            st = c.step(10)
            outs.append((c.fields(["phi_f", "phi_w", "xO", "ux", "uy", "uz", "epsp"]), st["cg_iters_total"]))
            c.close()
    finally:
        net.close()
    for f, it in outs[1:]:
        assert it == outs[0][1]
        for k in f:
            np.testing.assert_array_equal(f[k], outs[0][0][k], err_msg=k)
