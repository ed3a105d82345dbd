"""GPU parity of the tile kernels for tile shapes other than the defaults
(16 x 16 Q1 cells on four waves, 8 x 8 Q2 cells on one wave).

These shapes take the kernels' other code paths: Q1 tiles of 8 x 8 and 3 x 5
cells need several staging rounds, so their Jacobian identity rows are written
while staging and the level epilogues load their inputs themselves; Q2 tiles
of 16 x 16 cells span four waves and accumulate in colour phases. The leaf
vmult, its transpose (one vector and a batch) and the residual must match the FP64 oracle at 1e-12,
and the FP64 V-cycle must match the one of the default tiles at 1e-12 (same
operators, different summation order)."""
import numpy as np
import pytest

import inputs
from tests.gpu_common import Case, rel_err

pytestmark = pytest.mark.gpu

TOL = 1e-12
MESH = dict(n_base=16, n_local=2, coarse=4, band=(3.0, 1.0))
SHAPES = [(1, (8, 8)), (1, (3, 5)), (2, (16, 16)), (2, (3, 5))]
_cases = {}


def case(p, tile):
    key = (p, tile)
    if key not in _cases:
        print(f"[case] tiles {key}", flush=True)
        c = Case(MESH["n_base"], MESH["n_local"], p, coarse=MESH["coarse"], band=MESH["band"], u_std=1e-2,
                 tile=tile, phit="shifted")
        c.load_state(setup_mg=True)
        _cases[key] = c
    return _cases[key]


@pytest.mark.parametrize("p,tile", SHAPES, ids=lambda v: str(v))
def test_leaf_operators_other_tiles(p, tile):
    c = case(p, tile)
    J = c.lp.masked_operator(c.U_o, c.phit_o, c.active_o)
    src = inputs.random_vector(c.X, c.Y, 21)
    got = c.g.vmult(c.dev(src)).cpu().numpy()
    assert rel_err(got, c.to_g(J @ c.to_o(src))) <= TOL
    gotT = c.g.vmult_T(c.dev(src), batch=1).cpu().numpy()
    assert rel_err(gotT, c.to_g(J.T @ c.to_o(src))) <= TOL
    # the batched transpose (state staged once per tile, one pass per
    # right-hand side): bit for bit the one-vector result
    src2 = inputs.random_vector(c.X, c.Y, 22)
    gotB = c.g.vmult_T(c.dev(np.concatenate([src, src2])), batch=2).cpu().numpy()
    assert np.array_equal(gotB[:3 * c.n], gotT)
    assert rel_err(gotB[3 * c.n:], c.to_g(J.T @ c.to_o(src2))) <= TOL
    U = c.dev(c.to_g(c.U_o))
    R = c.g.residual(U).cpu().numpy()
    ref = c.to_g(c.lp.residual(c.U_o, c.phit_o) * np.concatenate([~c.om.hanging] * 3))
    assert rel_err(R, ref) <= TOL


@pytest.mark.parametrize("p,tile", SHAPES, ids=lambda v: str(v))
def test_vcycle_other_tiles(p, tile):
    c = case(p, tile)
    d = case(p, (0, 0))
    # the node numbering depends on the tiles: compare in the oracle's order
    # (inputs are functions of the lattice position, so both sides get the
    # same values); same smoothing intervals on both sides (the estimates
    # differ by rounding)
    lam_max, lam_min0 = d.g.get_eigen()
    c.g.set_eigen(lam_max, lam_min0)
    got = c.to_o(c.g.vcycle(c.dev(inputs.random_vector(c.X, c.Y, 22))).cpu().numpy())
    ref = d.to_o(d.g.vcycle(d.dev(inputs.random_vector(d.X, d.Y, 22))).cpu().numpy())
    c.g.set_eigen(None)
    assert rel_err(got, ref) <= TOL
