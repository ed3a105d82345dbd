"""GPU parity of the leaf operators against the FP64 oracle (element by
element on the same seeded inputs): vmult, vmult_T, inverse diagonal,
residual, crack volume and parameter derivatives.

Tolerance: the operators are sums of O(10-100) products per entry in FP64;
different summation orders give relative deviations of a few 1e-16 times the
condition of the sums, so 1e-12 of the largest entry is the bar."""
import numpy as np
import pytest

import inputs
from tests.gpu_common import Case, rel_err

pytestmark = pytest.mark.gpu

TOL = 1e-12

MESHES = {
    # 4x4 coarse grid, 16x16 base, two local levels in |x|<3, |y|<1: hanging nodes on both sides
    "tiny": dict(n_base=16, n_local=2, coarse=4, band=(3.0, 1.0)),
    # 32x32 base from the 16x16 coarse grid, two local levels in the Sneddon band
    "small": dict(n_base=32, n_local=2, coarse=16, band=(2.0, 0.5)),
}

_cases = {}


def case(name, p, mask="bernoulli"):
    key = (name, p, mask)
    if key not in _cases:
        m = MESHES[name]
        print(f"[case] {key}", flush=True)
        c = Case(m["n_base"], m["n_local"], p, coarse=m["coarse"], band=m["band"], mask=mask,
                 u_std=1e-2, phit="shifted")
        c.load_state()
        _cases[key] = c
    return _cases[key]


PARAMS = [(n, p, mk) for n in MESHES for p in (1, 2) for mk in ("bernoulli", "rule")]


@pytest.mark.parametrize("name,p,mask", PARAMS)
def test_active_set_matches_rule(name, p, mask):
    c = case(name, p, mask)
    act = c.g.active().cpu().numpy().astype(bool)
    if mask == "bernoulli":
        assert np.array_equal(act, c.active)
    else:
        # the rule is a sign decision on lambda = R/B; both sides decide in FP64
        # from residuals that differ by rounding only
        ref = c.active_o[c.g2o]
        diff = np.flatnonzero(act != ref)
        R = c.lp.residual(c.U_o, c.phit_o)[2 * c.n:]
        scale = np.abs(R).max()
        assert np.all(np.abs(R[c.g2o][diff]) <= 1e-12 * scale), diff


@pytest.mark.parametrize("p", (1, 2))
@pytest.mark.parametrize("c_fixed", (0.0, 0.5, 50.0))
def test_active_set_rule_with_phase_field_change(p, c_fixed):
    """Active-set rule of Sec. 2 where phi - phi_old takes both signs (phi_old
    = phi + 0.02 N(0, 1), seeded): the per-unknown c (pdas_c = 0) and constant
    values of c. Both sides decide in FP64; they may differ only where
    lambda + c (phi - phi_old) is within rounding of zero."""
    from oracle.newton import active_set
    from paper_2404_03265_amd import SolverParams
    m = MESHES["tiny"]
    print(f"[case] tiny p={p} pdas_c={c_fixed}", flush=True)
    c = Case(m["n_base"], m["n_local"], p, coarse=m["coarse"], band=m["band"], mask="rule", u_std=1e-2,
             solver_params=SolverParams(pdas_c=c_fixed), build_oracle=False)
    c.phi_old_raw = c.phi_old_raw + 0.02 * inputs.normal(5, 40, c.X, c.Y)
    c.build_oracle(m["n_base"], m["n_local"], p, m["coarse"], m["band"])
    c.load_state()
    act = c.g.active().cpu().numpy().astype(bool)
    R = c.lp.residual(c.U_o, c.phit_o)
    ref = active_set(c.lp, R, c.U_o[2 * c.n:], c.phio_o, c_fixed)[c.g2o]
    d = (c.U_o[2 * c.n:] - c.phio_o)[c.g2o]
    assert np.count_nonzero(d > 0) > 0.2 * c.n and np.count_nonzero(d < 0) > 0.2 * c.n
    assert 0 < np.count_nonzero(ref) < c.n
    lam = (R[2 * c.n:] / np.where(c.om.hanging, 1.0, c.lp.lumped_phi_mass()))[c.g2o]
    diff = np.flatnonzero(act != ref)
    scale = np.abs(lam).max()
    cc = c_fixed if c_fixed > 0 else 2.0 * np.abs(lam[diff] / np.where(d[diff] != 0, d[diff], 1.0))
    assert np.all(np.abs(lam[diff] + cc * d[diff]) <= 1e-11 * scale), diff


@pytest.mark.parametrize("theta", (0.0, 1.0, 0.75))
def test_extrapolate_phi_matches_oracle(theta):
    """phi~ extrapolated from two load steps and clipped to [0, 1] (Sec. 2):
    bitwise equal to the oracle (each product and sum rounded separately),
    also when the output overwrites an input."""
    from oracle.newton import extrapolate_phase_field
    c = case("tiny", 2)
    x = -0.5 + 2.0 * inputs.uniform01(7, 50, c.X, c.Y)
    y = -0.5 + 2.0 * inputs.uniform01(7, 51, c.X, c.Y)
    ref = extrapolate_phase_field(x, y, theta)
    got = c.g.extrapolate_phi(c.dev(x), c.dev(y), theta).cpu().numpy()
    assert np.array_equal(got, ref)
    xd = c.dev(x)
    c.g.extrapolate_phi(xd, c.dev(y), theta, out=xd)
    assert np.array_equal(xd.cpu().numpy(), ref)
    assert 0 < np.count_nonzero(ref == 0.0) and 0 < np.count_nonzero(ref == 1.0)


@pytest.mark.parametrize("name,p,mask", PARAMS)
def test_vmult_matches_oracle(name, p, mask):
    c = case(name, p, mask)
    act_o = c.g.active().cpu().numpy().astype(bool)[c.o2g]
    J = c.lp.masked_operator(c.U_o, c.phit_o, act_o)
    src = inputs.random_vector(c.X, c.Y, 1)
    dst = c.g.vmult(c.dev(src)).cpu().numpy()
    ref = c.to_g(J @ c.to_o(src))
    for b in range(3):
        sl = slice(b * c.n, (b + 1) * c.n)
        assert rel_err(dst[sl], ref[sl]) <= TOL, (b, rel_err(dst[sl], ref[sl]))
    # deterministic: a second application is bitwise identical
    dst2 = c.g.vmult(c.dev(src)).cpu().numpy()
    assert np.array_equal(dst, dst2)


@pytest.mark.parametrize("name,p", [(n, p) for n in MESHES for p in (1, 2)])
def test_vmult_transpose_matches_oracle(name, p):
    """J~^T against the oracle's assembled transpose: one vector, and a
    batch of 11 (a full chunk of 8 right-hand sides with the state read once
    per tile, then a ragged chunk of 3), each equal bit for bit to the
    one-vector kernel."""
    c = case(name, p)
    J = c.lp.masked_operator(c.U_o, c.phit_o, c.active_o)
    batch = 11
    srcs = [inputs.random_vector(c.X, c.Y, 100 + i) for i in range(batch)]
    out = c.g.vmult_T(c.dev(np.concatenate(srcs)), batch=batch).cpu().numpy()
    for i in range(batch):
        ref = c.to_g(J.T @ c.to_o(srcs[i]))
        got = out[i * 3 * c.n:(i + 1) * 3 * c.n]
        assert rel_err(got, ref) <= TOL, i
        one = c.g.vmult_T(c.dev(srcs[i])).cpu().numpy()
        assert rel_err(one, ref) <= TOL, i
        assert np.array_equal(got, one), (i, np.abs(got - one).max())


@pytest.mark.parametrize("name,p", [(n, p) for n in MESHES for p in (1, 2)])
def test_inverse_diagonal_matches_oracle(name, p):
    c = case(name, p)
    J = c.lp.masked_operator(c.U_o, c.phit_o, c.active_o)
    ref = c.to_g(1.0 / J.diagonal())
    got = c.g.inverse_diagonal(-1).cpu().numpy()
    assert rel_err(got, ref) <= TOL


@pytest.mark.parametrize("name,p", [(n, p) for n in MESHES for p in (1, 2)])
def test_residual_matches_oracle(name, p):
    c = case(name, p)
    U = c.dev(c.to_g(c.U_o))
    R = c.g.residual(U).cpu().numpy()
    Ro = c.lp.residual(c.U_o, c.phit_o)
    hang = c.om.hanging
    Ro = Ro * np.concatenate([~hang] * 3)
    ref = c.to_g(Ro)
    assert rel_err(R, ref) <= TOL
    Rm = c.g.residual(U, masked=True).cpu().numpy()
    refm = c.to_g(Ro * c.lp.free_mask(c.active_o))
    assert rel_err(Rm, refm) <= TOL


@pytest.mark.parametrize("name,p", [(n, p) for n in MESHES for p in (1, 2)])
def test_tcv_and_parameter_derivatives(name, p):
    c = case(name, p)
    U = c.dev(c.to_g(c.U_o))
    tcv, g = c.g.tcv(U, grad=True)
    ref = c.lp.tcv(c.U_o)
    assert abs(tcv - ref) <= TOL * max(abs(ref), 1e-300) * 10
    gref = c.to_g(c.lp.tcv_gradient(c.U_o) * np.concatenate([~c.om.hanging] * 3))
    assert rel_err(g.cpu().numpy(), gref) <= TOL
    z = inputs.random_vector(c.X, c.Y, 55)
    out = c.g.param_grad(c.dev(z))
    free = c.lp.free_mask(c.active_o)
    d = c.lp.param_derivatives(c.U_o, c.phit_o)
    zo = c.to_o(z) * free
    for i, k in enumerate(("Gc", "E", "p")):
        r = zo @ (d[k] * free)
        scale = np.abs(zo).sum() * np.abs(d[k]).max()
        assert abs(out[i] - r) <= 1e-13 * scale, (k, out[i], r)


@pytest.mark.parametrize("p", (1, 2))
def test_vector_utilities_match_oracle(p):
    """The small entry points around the operators: hanging entries set from
    their masters (pff_distribute) and constrained rows zeroed
    (pff_mask_constrained) as the oracle's constraint matrix and free mask
    give them, and the deterministic dot product (pff_dot): bitwise
    repeatable and equal to a plain FP64 sum to rounding."""
    c = case("tiny", p)
    n = c.n
    v = inputs.random_vector(c.X, c.Y, 64)
    got = c.g.distribute(c.dev(v), 3).cpu().numpy()
    assert rel_err(got, c.to_g(c.lp.distribute(c.to_o(v)))) <= 1e-15
    got = c.g.mask_constrained(c.dev(v)).cpu().numpy()
    assert np.array_equal(got, v * c.to_g(c.lp.free_mask(c.active_o)).astype(float))
    w = inputs.random_vector(c.X, c.Y, 65)
    d1 = c.g.dot(c.dev(v), c.dev(w))
    d2 = c.g.dot(c.dev(v), c.dev(w))
    assert d1 == d2
    assert abs(d1 - float(np.dot(v, w))) <= 1e-13 * float(np.dot(np.abs(v), np.abs(w)))
    nt, nrec, mx = c.g.tile_stats()
    assert nt > 0 and nrec >= 1 and 0 < mx <= 256
    assert 3 * n == v.size
