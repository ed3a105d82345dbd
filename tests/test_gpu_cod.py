"""GPU parity of the crack opening displacement COD(x) (Sec. 4) against the
oracle's line integrals: random states on meshes with hanging nodes, Q1 and
Q2, lines inside cells, on cell edges and at the domain ends, and more lines
than one launch takes."""
import numpy as np
import pytest

from tests.gpu_common import Case

pytestmark = pytest.mark.gpu

MESHES = {
    "tiny": dict(n_base=16, n_local=2, coarse=4, band=(3.0, 1.0)),
    "small": dict(n_base=32, n_local=2, coarse=16, band=(2.0, 0.5)),
}
XS = [-10.0, -9.99, -1.5, -0.99, -0.3, 0.0, 0.17, 0.74, 1.0, 3.3, 9.99, 10.0]


@pytest.mark.parametrize("name,p", [(n, p) for n in MESHES for p in (1, 2)])
def test_cod_matches_oracle(name, p):
    m = MESHES[name]
    print(f"[cod] {name} Q{p}", flush=True)
    c = Case(m["n_base"], m["n_local"], p, coarse=m["coarse"], band=m["band"], u_std=1e-2)
    U = c.dev(c.U_raw)
    got = c.g.cod(U, XS)
    ref = c.lp.cod(c.U_o, XS)
    scale = max(np.abs(ref).max(), 1e-300)
    assert np.abs(got - ref).max() <= 1e-12 * scale, (got, ref)
    assert got[-1] == 0.0   # x = 10 lies in no cell
    # more lines than one launch (64): two launches
    xs = np.linspace(-2.0, 2.0, 101)
    got = c.g.cod(U, xs)
    ref = c.lp.cod(c.U_o, xs)
    assert np.abs(got - ref).max() <= 1e-12 * max(np.abs(ref).max(), 1e-300)
    # an empty list and a bad position
    assert c.g.cod(U, []).size == 0
    with pytest.raises(RuntimeError):
        c.g.cod(U, [np.nan])
