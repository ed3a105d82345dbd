"""GPU parity at the degenerate ends of the method and at the largest size.

* a uniform mesh (no local refinement: no hanging nodes, no refinement edge,
  global levels only), and the paper's 40 x 40 mesh family;
* every phase-field unknown in the active set (the phi block of J~ is the
  identity, the phi block of every level is fixed: its eigenvalue estimate
  has no free unknown);
* the largest workload (2048 x 2048 base cells + 4 local levels, Q2, 178.5 M
  unknowns), where the oracle cannot run: properties that hold at any size.
"""
import numpy as np
import pytest

import inputs
from oracle.mg import Hierarchy, MGParams, VCycle
from tests.gpu_common import Case, rel_err

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _vcycle_oracle(c):
    lam_max, lam_min0 = c.g.get_eigen()
    return VCycle(Hierarchy(c.om), c.prm, MGParams(), c.U_o, c.phit_o, c.active_o,
                  eigen=([lam_max[l] for l in range(c.g.n_levels)], lam_min0))


def _check_operators(c):
    J = c.lp.masked_operator(c.U_o, c.phit_o, c.active_o)
    src = inputs.random_vector(c.X, c.Y, 71)
    got = c.g.vmult(c.dev(src)).cpu().numpy()
    assert rel_err(got, c.to_g(J @ c.to_o(src))) <= TOL
    gotT = c.g.vmult_T(c.dev(src)).cpu().numpy()
    assert rel_err(gotT, c.to_g(J.T @ c.to_o(src))) <= TOL
    vc = _vcycle_oracle(c)
    got = c.g.vcycle(c.dev(src)).cpu().numpy()
    ref = c.to_g(vc.apply(c.to_o(src)))
    assert rel_err(got, ref) <= TOL
    got32 = c.g.vcycle(c.dev(src), fp32=True).cpu().numpy()
    assert rel_err(got32, ref) <= 1e-5
    return src, got


@pytest.mark.parametrize("p", (1, 2))
def test_uniform_mesh(p):
    """No local refinement: vmult, vmult_T and both V-cycles against the oracle."""
    print(f"[case] uniform 32 x 32 p={p}", flush=True)
    c = Case(32, 0, p, coarse=8, mask="bernoulli", u_std=1e-2, phit="shifted")
    assert not np.any(c.om.hanging)
    c.load_state(setup_mg=True)
    assert c.g.n_levels == 3
    _check_operators(c)


@pytest.mark.parametrize("p", (1, 2))
def test_paper_mesh_family(p):
    """The paper's mesh family (Sec. 4, Table 2): a 40 x 40 base mesh from a
    10 x 10 coarse grid (tiles cut raggedly), two local levels: vmult, vmult_T
    and both V-cycles against the oracle."""
    print(f"[case] 40 x 40 + 2 p={p}", flush=True)
    c = Case(40, 2, p, coarse=10, band=(3.0, 1.0), mask="bernoulli", u_std=1e-2, phit="shifted")
    c.load_state(setup_mg=True)
    assert c.g.n_levels == 5
    _check_operators(c)


@pytest.mark.parametrize("p", (1, 2))
def test_every_phase_field_unknown_active(p):
    """All non-hanging phase-field unknowns active: the phi rows of J~ and of
    the preconditioner are the identity, the u block is unchanged."""
    print(f"[case] all phi active p={p}", flush=True)
    c = Case(16, 2, p, coarse=4, band=(3.0, 1.0), mask="bernoulli", u_std=1e-2, phit="shifted",
             build_oracle=False)
    flags = c.g.flags()
    c.active = (flags & 2) == 0
    c.build_oracle(16, 2, p, 4, (3.0, 1.0))
    c.load_state(setup_mg=True)
    assert np.array_equal(c.g.active().cpu().numpy().astype(bool), c.active)
    src, pc = _check_operators(c)
    n = c.n
    dst = c.g.vmult(c.dev(src)).cpu().numpy()
    assert np.array_equal(dst[2 * n:], src[2 * n:])
    assert np.array_equal(pc[2 * n:], src[2 * n:])
    lam_max, _ = c.g.get_eigen()
    assert np.all(lam_max[:, 1] == 1.0)       # no free phase-field unknown on any level


def test_largest_workload_properties():
    """2048^2 + 4 local levels, Q2 (178.5 M unknowns): the vmult is bitwise
    reproducible, w.(J~ v) = (J~^T w).v, the FP64 V-cycle is symmetric and the
    FP32 V-cycle stays within 1e-5 of it."""
    import time
    import torch
    t0 = time.time()
    c = Case(2048, 4, 2, mask="bernoulli", u_std=1e-4, build_oracle=False, phit="shifted")
    print(f"[largest] {3 * c.n} unknowns, mesh built {time.time() - t0:.1f}s", flush=True)
    c.load_state(setup_mg=True)
    print(f"[largest] state and multigrid set up {time.time() - t0:.1f}s", flush=True)
    v = c.dev(inputs.random_vector(c.X, c.Y, 81))
    w = c.dev(inputs.random_vector(c.X, c.Y, 82))
    Jv = c.g.vmult(v)
    assert torch.equal(Jv, c.g.vmult(v))
    a, b = torch.dot(w, Jv).item(), torch.dot(c.g.vmult_T(w), v).item()
    assert abs(a - b) <= 1e-12 * (torch.linalg.norm(w) * torch.linalg.norm(Jv)).item()
    Pv = c.g.vcycle(v)
    Pw = c.g.vcycle(w)
    a, b = torch.dot(w, Pv).item(), torch.dot(v, Pw).item()
    assert abs(a - b) <= 1e-12 * (torch.linalg.norm(w) * torch.linalg.norm(Pv)).item()
    assert rel_err(c.g.vcycle(v, fp32=True).cpu().numpy(), Pv.cpu().numpy()) <= 1e-5
    print(f"[largest] done {time.time() - t0:.1f}s", flush=True)
