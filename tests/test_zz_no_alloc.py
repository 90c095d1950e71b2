"""The entry point that allocates nothing (pf_increment_scale_static) against
the one it is a variant of (pf_nn_increment_scale), through the C ABI: two
calls in a row, the second on a smaller grid, both bitwise equal to the
network-held variant (same kernels, same fixed reduction order)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _faces(rng, shape, torch):
    nz, ny, nx = shape
    shp = ((nz, ny, nx + 1), (nz, ny + 1, nx), (nz + 1, ny, nx))
    return [torch.from_numpy(rng.standard_normal(s) * 1e-9).cuda() for s in shp]


def test_static_scale_matches_network_variant():
    import torch
    from paper_2111_11538_amd import pf
    rng = np.random.default_rng(31)
    net = pf.Net(max_voxels=4096, seed=2)
    s_dev = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
    try:
        for shape, with_u0 in (((40, 37, 53), True), ((9, 12, 7), False)):   # the second call is smaller
            say(f"static increment scale, grid {shape}, u0 given: {with_u0}")
            u1 = _faces(rng, shape, torch)
            u0 = _faces(rng, shape, torch) if with_u0 else None
            want = net.increment_scale(u1, u0)
            pf.increment_scale_static(u1, u0, s_dev)
            torch.cuda.synchronize()
            got = float(s_dev.cpu()[0])
            # an independent FP64 check of the definition
            diffs = [(a - (b if b is not None else 0)).cpu().numpy() for a, b in zip(u1, u0 or [None] * 3)]
            nz, ny, nx = shape
            low = [diffs[0][:, :, :nx], diffs[1][:, :ny, :], diffs[2][:nz]]
            ref = np.sqrt(sum(float(np.sum(d * d)) for d in low) / (3 * nx * ny * nz))
            say(f"  static {got!r}  network variant {want!r}  numpy {ref!r}")
            assert got == want
            assert abs(got - ref) <= 1e-13 * ref
    finally:
        net.close()


def test_static_scale_rejects_bad_arguments():
    import torch
    from paper_2111_11538_amd import pf
    s_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
    u = [torch.zeros(8, dtype=torch.float64, device="cuda") for _ in range(3)]
    for args in ((pf._ptr3(u), None, 0, 1, 1, pf.C.c_void_p(s_dev.data_ptr()), None),
                 (pf._ptr3(u), None, 50000, 50000, 2, pf.C.c_void_p(s_dev.data_ptr()), None),
                 (None, None, 2, 2, 2, pf.C.c_void_p(s_dev.data_ptr()), None),
                 (pf._ptr3(u), None, 2, 2, 2, None, None)):
        rc = pf.lib().pf_increment_scale_static(*args)
        assert rc == pf.PF_ERR_INVALID_ARG, rc
        assert pf.lib().pf_nn_last_error(None).decode()
