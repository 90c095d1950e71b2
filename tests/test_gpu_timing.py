"""The kernel timing interface: kind masks and the sampling of the CG
kernels (HIP events attached to the dispatches), and that timing leaves the
results untouched."""
import numpy as np
import pytest

from paper_2111_11538_amd import inputs as I

pytestmark = pytest.mark.gpu


def _ctx():
    from paper_2111_11538_amd import pf
    wl = I.workload("core_shell_3d", n=32)
    c = pf.Context(3, wl.shape, wl.h, wl.dt, wl.params, precision="mixed", plasticity=True, cg_rtol=1e-6)
    c.set_fields(wl.fields)
    return c


def test_kind_mask_and_cg_sampling():
    c = _ctx()
    c.step(1)
    c.timing(True, kinds=("update",), every=4)
    it0 = c.step(0)["cg_iters_total"]
    st = c.step(3)
    rep = c.timing_report()
    c.timing(False)
    iters = st["cg_iters_total"] - it0
    for k, (ms, n) in rep.items():
        # sampled update launches queued past convergence (they exit at entry)
        # are reported as "other"
        if k not in ("update", "other"):
            assert n == 0 and ms == 0.0, (k, n, ms)
    n_upd = rep["update"][1]
    assert n_upd > 0 and rep["update"][0] > 0.0
    # three solves; of each, the working iterations i with (i + s) % 4 == 0
    assert iters // 4 - 3 <= n_upd <= iters // 4 + 3, (n_upd, iters)
    assert rep["other"][1] <= 3 * 64 // 4 + 3
    c.timing(True)
    c.step(2)
    rep = c.timing_report()
    for k in ("apply", "update", "solve_setup", "step", "mu", "other"):
        assert rep[k][1] > 0, k
    c.close()


def test_timing_does_not_change_results():
    a, b = _ctx(), _ctx()
    b.timing(True, every=3)
    a.step(3)
    b.step(3)
    fa, fb = a.fields(), b.fields()
    for k in ("phi_f", "phi_w", "xO", "ux", "uy", "uz"):
        np.testing.assert_array_equal(fa[k], fb[k])
    a.close()
    b.close()


def test_timing_mask_rejects_unknown_bits():
    from paper_2111_11538_amd import pf
    c = _ctx()
    with pytest.raises(pf.PFError):
        c._check(pf.lib().pf_timing(c.ctx, 1 << 12))
    with pytest.raises(pf.PFError):
        c._check(pf.lib().pf_timing_every(c.ctx, 0))
    c.close()
