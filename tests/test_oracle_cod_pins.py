"""Pins of the oracle's crack opening displacement COD(x) (Sec. 4: the line
integral of u . grad phi over y at fixed x): exact values for polynomial
fields that the Q_p space holds, and the integral of COD over x equal to the
oracle's volume integral TCV for a general finite-element field (the COD is
piecewise polynomial in x between cell edges, so Gauss points per interval
integrate it exactly)."""
import numpy as np
import pytest
import sympy as sym

import inputs
from oracle.assemble import LeafProblem, Params
from oracle.fe import gauss_01
from oracle.mesh import Mesh


def _mesh(p):
    return Mesh(16, 2, p, coarse=4, band=(3.0, 1.0))


@pytest.mark.parametrize("p", [1, 2])
def test_cod_of_polynomial_fields_is_exact(p):
    x, y = sym.symbols("x y")
    if p == 1:
        ux = sym.Rational(3, 10) + sym.Rational(1, 5) * x * y
        uy = -sym.Rational(1, 10) + sym.Rational(1, 20) * y + sym.Rational(1, 50) * x
        ph = sym.Rational(1, 2) + sym.Rational(1, 10) * x + sym.Rational(7, 100) * y + sym.Rational(1, 100) * x * y
    else:
        ux = sym.Rational(3, 10) + sym.Rational(1, 5) * x * y ** 2 - sym.Rational(1, 40) * x ** 2
        uy = -sym.Rational(1, 10) + sym.Rational(1, 20) * y ** 2 + sym.Rational(1, 50) * x * y
        ph = sym.Rational(1, 2) + sym.Rational(1, 10) * x ** 2 * y + sym.Rational(7, 100) * y ** 2 - sym.Rational(1, 30) * x
    m = _mesh(p)
    X = -10 + 20 * m.NX / m.M
    Y = -10 + 20 * m.NY / m.M
    f = [sym.lambdify((x, y), e, "numpy") for e in (ux, uy, ph)]
    U = np.concatenate([np.broadcast_to(fi(X, Y), X.shape).astype(float) for fi in f])
    lp = LeafProblem(m, Params())
    xs = [-9.3, -1.0, -0.37, 0.0, 0.5, 1.23, 7.5]    # 0.0 and 0.5 lie on cell edges
    got = lp.cod(U, xs)
    integrand = ux * sym.diff(ph, x) + uy * sym.diff(ph, y)
    for j, x0 in enumerate(xs):
        ref = float(sym.integrate(integrand.subs(x, sym.nsimplify(x0)), (y, -10, 10)))
        assert abs(got[j] - ref) <= 1e-12 * max(1.0, abs(ref)), (x0, got[j], ref)


@pytest.mark.parametrize("p", [1, 2])
def test_cod_integrates_to_tcv(p):
    """The integral of COD(x) over x equals TCV for a general field: COD is a
    polynomial of degree <= 2p in x between consecutive cell x-edges."""
    m = _mesh(p)
    lp = LeafProblem(m, Params())
    X, Y = m.NX, m.NY
    U = lp.distribute(np.concatenate([inputs.random_vector(X, Y, 5)[:2 * m.n_nodes],
                                      inputs.random_vector(X, Y, 6)[:m.n_nodes]]))
    H = m.H(m.cell_level)
    edges = np.unique(np.concatenate([-10.0 + m.cell_i * H, -10.0 + (m.cell_i + 1) * H]))
    g, w = gauss_01(p + 1)
    xs, ws = [], []
    for a, b in zip(edges[:-1], edges[1:]):
        xs.extend(a + (b - a) * g)
        ws.extend((b - a) * w)
    total = float(np.dot(ws, lp.cod(U, xs)))
    ref = lp.tcv(U)
    assert abs(total - ref) <= 1e-11 * max(1.0, abs(ref)), (total, ref)
