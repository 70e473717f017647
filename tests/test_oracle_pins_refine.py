"""Pins of the oracle's iterative intersection points (Sec. V-B; Sec. VI
says the point is computed by an iteration that stops at a desired
accuracy; here false position with the Illinois modification, a fixed
number of steps).

Each pin names the mistake it would catch:
* zero steps reproduce the interpolated point bit for bit (a different first
  step, or a different final formula);
* for an affine f the first interpolation is already a root, so any number
  of steps keeps |f(p)| at rounding level (a step that moved the wrong end,
  which would leave the bracket);
* on the sphere the radius error falls from O(lambda^2) to rounding within a
  few steps and never grows (plain false position without the halving stalls
  on one side of a convex f and stays far above rounding);
* after enough steps the point equals the root scipy's brentq finds on the
  same segment (a sign slip in the bracket update converges elsewhere or
  not at all).
"""
import math

import numpy as np
import pytest
from scipy.optimize import brentq

import oracle as O
from paper_2406_04795_amd import inputs as I


@pytest.fixture(scope="module", autouse=True)
def _built():
    O.build(force=False)


def test_zero_steps_equal_interpolated_points():
    wl = I.config_c1()
    v, m = O.trace_direct(wl)
    p0, _ = O.points(wl, v, m)
    assert np.array_equal(O.points_refined(wl, v, m, 0).view(np.uint64), p0.view(np.uint64))


def test_affine_f_stays_a_root():
    rng = np.random.default_rng(5)
    d = 3
    dom = I.box(d)
    fm = I.random_manifold(d, 10, 1, rng, dom)
    fm.bias = -fm.coef0 * fm.alpha.sum() + 0.1
    lat = I.make_lattice(d, 0.2, rng)
    wl = I.Workload("affine", fm, lat, dom, I.bisection_seeds(fm, dom, rng, 2))
    v, m = O.trace_direct(wl)
    xa = O.coords(lat, v)
    xb = O.coords(lat, v + ((m[:, None] >> np.arange(d)) & 1).astype(np.int32))
    scale = np.abs(fm.alpha).sum() * 10
    for k in (1, 3, 6):
        p = O.points_refined(wl, v[:400], m[:400], k)
        vals = np.array([O.f_at(fm, x) for x in p])
        assert np.abs(vals).max() < 1e-12 * scale
        # still on the edge
        lo, hi = np.minimum(xa[:400], xb[:400]), np.maximum(xa[:400], xb[:400])
        assert ((p >= lo - 1e-12) & (p <= hi + 1e-12)).all()


def test_sphere_radius_error_falls_to_rounding():
    wl = I.sphere_case(3, 1.0, 0.1)
    v, m = O.trace_direct(wl)
    errs, meds = [], []
    for k in range(0, 10):
        p = O.points_refined(wl, v, m, k)
        e = np.abs(np.linalg.norm(p, axis=1) - 1.0)
        errs.append(e.max())
        meds.append(np.median(e))
    lam_edge = 0.1 * math.sqrt(3 / 4) * math.sqrt(2)
    assert errs[0] < lam_edge ** 2 and errs[0] > 1e-4
    for a, b in zip(errs, errs[1:]):
        assert b <= a * 1.000001 + 1e-15
    # the typical edge converges in 4 steps, the slowest in 8
    assert meds[4] < 1e-13 and errs[8] < 1e-13


def test_converged_points_equal_a_library_root_finder():
    wl = I.cubic_case(4, 200, 0.3, 0.01, seed=3, n_seeds=2)
    v, m = O.trace_direct(wl)
    rng = np.random.default_rng(1)
    idx = rng.choice(len(v), size=min(300, len(v)), replace=False)
    v, m = v[idx], m[idx]
    d = wl.f.d
    xa = O.coords(wl.lat, v)
    xb = O.coords(wl.lat, v + ((m[:, None] >> np.arange(d)) & 1).astype(np.int32))
    p = O.points_refined(wl, v, m, 12)
    checked = 0
    for i in range(len(v)):
        g = lambda t: O.f_at(wl.f, xa[i] + t * (xb[i] - xa[i]))  # noqa: E731
        ga, gb = g(0.0), g(1.0)
        if ga == 0.0 or gb == 0.0:
            continue
        t = brentq(g, 0.0, 1.0, xtol=1e-15, rtol=8.9e-16, maxiter=200)
        root = xa[i] + t * (xb[i] - xa[i])
        assert np.abs(p[i] - root).max() <= 1e-12 * max(1.0, np.abs(root).max())
        checked += 1
    assert checked > 250
