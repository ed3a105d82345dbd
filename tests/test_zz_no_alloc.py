"""The allocation-free vmult (pff_vmult_noalloc, for callers that cannot
allocate device memory) against pff_vmult on the same state: two calls in a
row, the second on a smaller mesh, and the size limit of the static array."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _case(n_base, n_local, p, coarse, band, seed):
    from tests.gpu_common import Case
    c = Case(n_base, n_local, p, coarse=coarse, band=band, seed=seed, u_std=1e-2, phit="shifted",
             build_oracle=False)
    c.load_state(setup_mg=False)
    return c


def _check(c, src_seed):
    import inputs
    import torch
    src = c.dev(inputs.random_vector(c.X, c.Y, src_seed))
    ref = c.g.vmult(src)
    out = torch.full_like(src, float("nan"))
    print(f"no-alloc vmult: n = {c.n}", flush=True)
    c.g.vmult_noalloc(src, out)
    torch.cuda.synchronize()
    a, b = out.cpu().numpy(), ref.cpu().numpy()
    assert np.all(np.isfinite(a))
    # same kernels, same summation order: bitwise equal (the bar is 1e-12)
    assert np.array_equal(a, b), float(np.abs(a - b).max() / np.abs(b).max())


def test_noalloc_vmult_matches_vmult_twice_then_smaller():
    big = _case(32, 2, 2, 4, (3.0, 1.0), 0)
    _check(big, 1)
    small = _case(16, 2, 1, 4, (3.0, 1.0), 3)
    _check(small, 2)
    # the first context again after the smaller call overwrote the array
    _check(big, 5)
    big.g.close()
    small.g.close()


def test_noalloc_vmult_refuses_meshes_above_the_limit():
    from paper_2404_03265_amd import PhaseFieldSolver, _lib
    import torch
    # 1024^2 + 3 local levels, Q2: about 41 MB of partial sums (> 16 MiB);
    # the size check comes before any state or device work
    g = PhaseFieldSolver(1024, 3, 2, torch_workspace=False)
    x = torch.zeros(3 * g.n, dtype=torch.float64, device="cuda")
    y = torch.zeros_like(x)
    rc = g.lib.pff_vmult_noalloc(g.h, C.c_void_p(y.data_ptr()), C.c_void_p(x.data_ptr()), None)
    assert rc == -1
    msg = g.lib.pff_last_error(g.h).decode()
    assert "static scratch" in msg and str(16 * 1024 * 1024) in msg
    g.close()
