"""Pins of the locally refined tensor velocity grid (reading R35): per axis
the node density 1 + A (exp(-(x/w)^2) + exp(-((x - c)/w)^2)), nodes and dual
cells the images of uniform cells of u in [-1, 1] under the inverse of the
normalised cumulative density.

The checks use numerical quadrature of the density (scipy), not the
oracle's closed-form cumulative, plus quadrature convergence and the
cut-cell half-box identity.
"""
from math import exp, pi, sqrt

import numpy as np
import pytest
from scipy.integrate import quad

from paper_2512_20252_amd import cases


def _box(N, V=6.0, A=3.0, w=1.0, c=(0.0, 0.0, 0.0), dim=2):
    if dim == 2:
        return cases.case(dim=2, n=(8, 8), lo=(0.0, 0.0), hi=(1.0, 1.0), vn=(N, N), vlo=(-V, -V), vhi=(V, V),
                          rule="refined", vref_amp=A, vref_width=w, vref_centre=c, Kn=0.1, Ma=0.0)
    return cases.case(dim=3, n=(4, 4, 4), lo=(0, 0, 0), hi=(1, 1, 1), vn=(N, N, N), vlo=(-V,) * 3, vhi=(V,) * 3,
                      rule="refined", vref_amp=A, vref_width=w, vref_centre=c, Kn=0.1, Ma=0.0)


def _axis(o, a, N):
    xi, w = o.velocity()
    stride = N ** a
    idx = np.arange(N) * stride
    return xi[idx, a], None


@pytest.mark.parametrize("c", [0.0, 2.3, -1.7])
def test_refined_cells_carry_equal_density_mass(oracle_mod, c):
    """Every dual cell of an axis carries the same mass of the node density
    (the defining property of the map), measured by adaptive quadrature of
    the density over the cell, independent of the closed-form cumulative;
    cells tile [-V, V]; nodes increase; weights are the cell widths.  Fails
    on a wrong erf scaling, a bump at the wrong centre or a wrong
    inversion."""
    N, V, A, w = 18, 6.0, 3.0, 0.8
    o = oracle_mod.Oracle(_box(N, V, A, w, (c, 0.0, 0.0)))
    xi, wt = o.velocity()
    x = xi[:N, 0]
    widths = wt.reshape(N, N)[0] / wt.reshape(N, N)[0].sum() * (2 * V)  # weight of node (i, 0) over the y weight
    centres = (0.0,) if c == 0.0 else (0.0, c)

    def rho(t):
        return 1.0 + A * sum(exp(-((t - cc) / w) ** 2) for cc in centres)

    total = quad(rho, -V, V, points=list(centres), limit=200)[0]
    assert np.all(np.diff(x) > 0)
    # reconstruct the cell faces from the weights: they tile the box
    faces = -V + np.concatenate([[0.0], np.cumsum(widths)])
    assert abs(faces[-1] - V) < 1e-12
    assert np.all((faces[:-1] < x) & (x < faces[1:]))
    for i in range(N):
        m = quad(rho, faces[i], faces[i + 1], limit=200)[0]
        assert abs(m - total / N) < 1e-9 * total, (i, m, total / N)
    # the node sits at the density-mass midpoint of its cell
    for i in range(N):
        m = quad(rho, faces[i], x[i], limit=200)[0]
        assert abs(m - 0.5 * total / N) < 1e-9 * total
    # refinement: cells at the centres are narrower than far cells by about the density ratio
    near = np.argmin(np.abs(x - c))
    far = 0 if abs(x[0] - c) > abs(x[-1] - c) else N - 1
    assert widths[near] < widths[far] / 2


def test_refined_symmetric_axis_is_exactly_antisymmetric(oracle_mod):
    """With the one bump at 0 the density is even, and nodes and weights
    are exactly antisymmetric / symmetric (the rest-state and mirror pins
    rely on it)."""
    N = 17
    o = oracle_mod.Oracle(_box(N, A=4.0, w=0.7))
    xi, w = o.velocity()
    x = xi[:N, 0]
    assert np.array_equal(x, -x[::-1])
    row = w.reshape(N, N)[0]
    assert np.array_equal(row, row[::-1])


def test_refined_grid_second_order_moments(oracle_mod):
    """The midpoint rule in u under a smooth map integrates smooth functions
    at second order: Maxwellian moments on the refined grid converge to
    (rho, U, T) with error ratios near 4 per doubling of N."""
    errs = []
    for N in (12, 24, 48):
        o = oracle_mod.Oracle(_box(N, V=6.0, A=2.0, w=1.2, c=(1.5, 0.0, 0.0)))
        g = o.maxwellian(1.3, (1.4, -0.3), 0.8)
        m = o.cell_moments(*g)
        errs.append(max(abs(m[0] - 1.3) / 1.3, abs(m[1] - 1.4), abs(m[2] + 0.3), abs(m[4] - 0.8)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.0 < r1 < 6.0 and 3.0 < r2 < 6.0, errs


@pytest.mark.parametrize("dim", [2, 3])
def test_refined_cut_measures_half_box(oracle_mod, dim):
    """A plane through the origin halves the symmetric velocity box: the
    incident measures sum to half the box (Section 3.2.3), which holds only
    if the refined dual cells tile the box and each weight is its cell's
    measure, with the second centre making the grid asymmetric."""
    o = oracle_mod.Oracle(_box(9 if dim == 3 else 15, V=4.0, A=2.5, w=0.9, c=(1.2, -0.8, 0.5), dim=dim))
    _, w = o.velocity()
    rng = np.random.default_rng(8)
    for _ in range(6):
        n = rng.normal(size=dim)
        n /= np.linalg.norm(n)
        cls, wg = o.cut_sets(n)
        assert abs(wg.sum() - 0.5 * w.sum()) < 1e-12 * w.sum()
        assert np.all(wg >= 0) and np.all(wg <= w * (1 + 1e-14))


# ---------------------------------------------------------------- Jacobian weights (reading R36)


def _mapped(N, rule, V=6.0, A=2.0, w=1.2, c=(1.5, 0.0, 0.0), beta=1.2, weights="jacobian"):
    return cases.case(dim=2, n=(8, 8), lo=(0.0, 0.0), hi=(1.0, 1.0), vn=(N, N), vlo=(-V, -V), vhi=(V, V),
                      rule=rule, vref_amp=A, vref_width=w, vref_centre=c, vstretch=beta, Kn=0.1, Ma=0.0,
                      vweights=weights)


@pytest.mark.parametrize("rule", ["refined", "stretched"])
def test_jacobian_weights_are_the_map_derivative(oracle_mod, rule):
    """Each weight is the derivative of the map x(u) at the node times the
    u-cell width 2/N: checked against a central difference of the map,
    which the test builds itself (the sinh map, or the refined density's
    cumulative by adaptive quadrature, inverted by root finding).  Fails
    on a density at the wrong centre, a wrong normalisation or the dual
    cell width in place of the derivative."""
    from scipy.optimize import brentq

    N, V, A, w, c, beta = 16, 6.0, 2.0, 1.2, 1.5, 1.2
    o = oracle_mod.Oracle(_mapped(N, rule, V, A, w, (c, 0.0, 0.0), beta))
    xi, wt = o.velocity()
    W = wt.reshape(N, N)  # W[j, i] = w_x(i) w_y(j)
    # the y axis (one bump at 0) has the product structure too: w_x(i) = W[j, i] / w_y(j) for every j
    def make_map(centres):
        if rule == "stretched":
            return lambda u: V * np.sinh(beta * u) / np.sinh(beta)

        def rho(t):
            return 1.0 + A * sum(exp(-((t - cc) / w) ** 2) for cc in centres)

        total = quad(rho, -V, V, points=list(centres), limit=200)[0]

        def xmap(u):
            target = 0.5 * (u + 1.0) * total
            return brentq(lambda x: quad(rho, -V, x, limit=200)[0] - target, -V, V, xtol=1e-14, rtol=1e-15)

        return xmap

    def fd_weight(xmap, i, d=1e-4):
        u = (2 * i + 1 - N) / N
        return (xmap(u + d) - xmap(u - d)) / (2 * d) * (2.0 / N)

    xmap = make_map((0.0, c))
    ref = np.array([fd_weight(xmap, i) for i in range(N)])
    nodes = np.array([xmap((2 * i + 1 - N) / N) for i in range(N)])
    assert np.max(np.abs(xi[:N, 0] - nodes)) < 1e-10
    # row 0 of the tensor grid: w_x(i) times the y weight of node 0, whose
    # map has the one bump at 0 (the second centre lies on x only)
    wy0 = fd_weight(make_map((0.0,)), 0)
    assert np.max(np.abs(W[0] - ref * wy0)) < 1e-6 * np.max(ref * wy0)


@pytest.mark.parametrize("rule", ["refined", "stretched"])
def test_jacobian_weights_integrate_maxwellians_spectrally(oracle_mod, rule):
    """Moments of a drifting Maxwellian (rho 1.3, U (1.4, -0.3), T 0.8)
    against their closed forms: with dual-cell weights the error falls at
    second order (about 4x per doubling of N); with the map's derivative
    the rule is the midpoint rule in u of a smooth, decaying integrand and
    the error falls by orders of magnitude per doubling, below 1e-7 at 48
    nodes (refined) and 1e-10 at 24 (stretched)."""
    def err(N, weights):
        o = oracle_mod.Oracle(_mapped(N, rule, weights=weights))
        m = o.cell_moments(*o.maxwellian(1.3, (1.4, -0.3), 0.8))
        return max(abs(m[0] - 1.3) / 1.3, abs(m[1] - 1.4), abs(m[2] + 0.3), abs(m[4] - 0.8))

    if rule == "refined":
        cell = [err(N, "cell") for N in (24, 48)]
        jac = [err(N, "jacobian") for N in (24, 48)]
        assert 3.0 < cell[0] / cell[1] < 6.0, cell
        assert jac[1] < 1e-7 and jac[0] / jac[1] > 100.0, jac
        assert jac[0] < cell[0] / 20
    else:
        assert err(24, "jacobian") < 1e-10
        assert err(24, "cell") > 1e-4


def test_jacobian_cut_cells_keep_the_incident_fraction(oracle_mod):
    """With the map's derivative as weight, a cut velocity cell keeps the
    incident fraction of its dual cell (Section 3.2.3): wg / w is the same
    as with dual-cell weights, where the half-box identity pins it; uncut
    cells carry their whole weight or none."""
    N = 15
    cj = dict(_box(N, V=4.0, A=2.5, w=0.9, c=(1.2, -0.8, 0.0)), vweights="jacobian")
    oc = oracle_mod.Oracle(_box(N, V=4.0, A=2.5, w=0.9, c=(1.2, -0.8, 0.0)))
    oj = oracle_mod.Oracle(cj)
    _, wc = oc.velocity()
    _, wj = oj.velocity()
    assert np.max(np.abs(wc - wj)) > 1e-3 * wc.max()  # the two weightings differ
    rng = np.random.default_rng(3)
    for _ in range(5):
        n = rng.normal(size=2)
        n /= np.linalg.norm(n)
        clc, gc = oc.cut_sets(n)
        clj, gj = oj.cut_sets(n)
        assert np.array_equal(clc, clj)
        assert np.max(np.abs(gc / wc - gj / wj)) < 1e-13
