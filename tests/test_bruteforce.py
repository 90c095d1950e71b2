"""P13: the C oracle against the brute-force reference (dense energy assembly
plus whole-array numpy) on tiny grids, over several full coupled steps."""
import numpy as np
import pytest

from paper_2111_11538_amd import inputs as I
import bruteforce as BF


def _fields_2d(n, seed):
    f = I.ic_core_shell((n, n), r_core=n * 0.3, frame=1, noise_seed=seed)
    return f


def _random_fields(shape, seed):
    """Every phase present in every cell, so that each term of the driving
    forces and fluxes is exercised."""
    rng = np.random.default_rng(seed)
    return {"phi_f": rng.uniform(0.05, 0.5, shape), "phi_w": rng.uniform(0.05, 0.45, shape),
            "xO": rng.uniform(0.0, 0.5, shape), "xH": rng.uniform(0.0, 0.02, shape),
            "xW": rng.uniform(0.0, 0.05, shape)}


@pytest.mark.parametrize("dim,n,nsteps,kind,implicit", [(2, 8, 4, "core_shell", False), (2, 8, 3, "random", False),
                                                        (3, 4, 2, "core_shell", False), (3, 4, 2, "random", False),
                                                        (2, 8, 3, "core_shell", True), (2, 8, 3, "random", True),
                                                        (3, 4, 2, "random", True), (2, 8, 3, "core_shell", 2),
                                                        (2, 8, 3, "random", 2), (3, 4, 2, "random", 2)])
def test_oracle_matches_bruteforce(oracle, dim, n, nsteps, kind, implicit):
    p = I.Params()
    h = I.H_DEFAULT
    # a larger time step than the explicit bound of the gas is fine for a
    # handful of steps and makes every term visible above rounding; the
    # implicit species update takes 50 times that
    dt = (100 if implicit == 1 else 1000 if implicit == 2 else 2) * I.stable_dt(p, h, dim)
    shape = (n,) * dim
    if kind == "random":
        f = _random_fields(shape, 100 + dim)
    elif dim == 2:
        f = _fields_2d(n, 11)
        f["xW"] = 0.05 * f["xH"]
    else:
        f = I.ic_core_shell(shape, r_core=1.2, r_shell=1.8, noise_seed=12)
        f["xW"] = 0.05 * f["xH"]
    sim = oracle.OracleSim(dim, shape, h, dt, p, f, mechanics=True, plasticity=True, dirichlet=True, cg_rtol=1e-14,
                           implicit=implicit)
    # brute-force state with a leading z axis in 2D
    bshape = (1, n, n) if dim == 2 else shape
    bf = {k: f[k].reshape(bshape).copy() for k in ("phi_f", "phi_w", "xO", "xH", "xW")}
    epsp = np.zeros((6,) + bshape)
    epsP = np.zeros(bshape)
    nc = 4 if dim == 2 else 6
    for it in range(nsteps):
        before = {k: sim.f[k].reshape(bshape).copy() for k in bf}
        st = sim.step()
        assert st["cg_rel_resid"] < 1e-12
        bf, (ux, uy, uz), epsp, epsP = BF.step(dim, shape, h, dt, p, bf, None, epsp, epsP, implicit=implicit)
        scale_u = np.max(np.abs(ux))
        assert np.max(np.abs(sim.ux.reshape(ux.shape) - ux)) < 1e-10 * scale_u
        assert np.max(np.abs(sim.uy.reshape(uy.shape) - uy)) < 1e-10 * scale_u
        if dim == 3:
            assert np.max(np.abs(sim.uz - uz)) < 1e-10 * scale_u
        for k in ("phi_f", "phi_w", "xO", "xH", "xW"):
            # compare the per-step increments: they are many orders of magnitude
            # below the field values at this time step
            a, b = sim.f[k].reshape(bshape) - before[k], bf[k] - before[k]
            assert np.max(np.abs(a - b)) < 1e-8 * np.max(np.abs(b)), (it, k)
            bf[k] = sim.f[k].reshape(bshape).copy()
        ep = sim.epsp.reshape((nc,) + bshape)
        assert np.max(np.abs(ep - epsp[:nc])) < 1e-9 * (np.max(np.abs(epsp)) + 1e-30)
        assert np.max(np.abs(sim.epsP.reshape(bshape) - epsP)) < 1e-9 * (np.max(epsP) + 1e-30)
    assert np.max(epsP) > 0          # the step did exercise the return map
