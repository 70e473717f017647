"""Pins of the oracle's RBF-kernel decision function (the experiments train
an RBF-kernel SVM; Sec. VI) and of its own exponential.

* exp: Cody-Waite reduction by ln 2 and a degree-13 Taylor polynomial; within
  2 ulp of the C library's exp everywhere it is used (t <= 0), exactly 1 at
  0, 0 below the normal range.  Catches a wrong reduction constant, a
  dropped or mis-scaled Taylor term, a wrong power of two.
* f: equals the plain numpy sum of alpha_i exp(-gamma |x - s_i|^2) + b to
  1e-13 relative (a transposed support vector, a wrong sign of gamma, a
  missing bias).
* One support vector makes f the sphere |x - s| = R: the trace equals the
  brute force over the box (a closed component), its crossing count follows
  the sphere's area law like the polynomial sphere's, and its intersection
  points lie within O(lambda^2) of the sphere.
* Batch triangulation with k = 1 equals the direct trace for an RBF f with
  many support vectors, and every traced edge is in the brute force.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2406_04795_amd import inputs as I


@pytest.fixture(scope="module", autouse=True)
def _built():
    O.build(force=False)


def _ulps(a, b):
    a, b = np.float64(a), np.float64(b)
    if a == b:
        return 0
    ia = np.array([a]).view(np.int64)[0]
    ib = np.array([b]).view(np.int64)[0]
    return abs(int(ia) - int(ib))


def test_exp_against_library():
    rng = np.random.default_rng(0)
    ts = np.concatenate([-rng.uniform(0, 708, 20000), -rng.uniform(0, 1, 5000),
                         -np.arange(0, 700) * math.log(2.0), [-1e-300, -5e-324]])
    worst = max(_ulps(O.exp(t), math.exp(t)) for t in ts)
    assert worst <= 2
    assert O.exp(0.0) == 1.0 and O.exp(-0.0) == 1.0
    assert O.exp(-709.0) == 0.0 and O.exp(-1e6) == 0.0


def test_rbf_f_matches_numpy():
    rng = np.random.default_rng(4)
    d = 5
    dom = I.box(d)
    fm = I.rbf_manifold(d, 400, rng, dom)
    fm.bias = -0.3
    X = rng.uniform(-3, 3, size=(300, d))
    want = np.exp(-fm.gamma * ((X[:, None, :] - fm.sv[None]) ** 2).sum(-1)) @ fm.alpha + fm.bias
    got = np.array([O.f_at(fm, x) for x in X])
    scale = np.exp(-fm.gamma * ((X[:, None, :] - fm.sv[None]) ** 2).sum(-1)) @ np.abs(fm.alpha) + abs(fm.bias)
    assert (np.abs(got - want) <= 1e-13 * scale).all()


def _as_set(v, m):
    return {(tuple(int(t) for t in v[i]), int(m[i])) for i in range(len(v))}


@pytest.mark.parametrize("d,R,lam,gamma", [(2, 1.0, 0.05, 1.0), (3, 1.0, 0.1, 0.7), (4, 1.0, 0.3, 1.3)])
def test_rbf_sphere_trace_equals_brute_force(d, R, lam, gamma):
    # a box that holds the sphere and a margin of a few cells
    wl = I.rbf_sphere_case(d, R, lam, gamma, half=R + 3 * lam + 0.2)
    v, m = O.trace_direct(wl)
    assert _as_set(v, m) == _as_set(*O.brute(wl))
    pts, _ = O.points(wl, v, m)
    r = np.linalg.norm(pts, axis=1)
    assert np.abs(r - R).max() < 2 * lam ** 2


def test_rbf_sphere_crossings_follow_the_area_law():
    # the same lattice as the polynomial sphere of radius 1: the zero sets are
    # the same sphere, so the sets of crossing edges coincide
    a = O.trace_direct(I.rbf_sphere_case(3, 1.0, 0.1, 0.8, seed=0))
    b = O.trace_direct(I.sphere_case(3, 1.0, 0.1, seed=0))
    assert _as_set(*a) == _as_set(*b)


def test_rbf_batch_k1_equals_direct_and_is_in_brute_force():
    wl = I.rbf_case(3, 60, 0.2, 0.3, seed=2, n_seeds=4)
    v, m = O.trace_direct(wl)
    bv, bm, _ = O.trace_batch(wl, k=1)
    assert len(v) > 500
    assert _as_set(v, m) == _as_set(bv, bm)
    assert _as_set(v, m) <= _as_set(*O.brute(wl))
    k2 = _as_set(*O.trace_batch(wl, k=2)[:2])
    assert k2 <= _as_set(*O.brute(wl)) and len(k2) > 0.5 * len(v)
