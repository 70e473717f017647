"""Pins of the oracle's gradient and seed search (Sec. V-A: seeds are points
on the manifold found by minimising |f| from given configurations).

* The canonical gradient equals central differences of the canonical f
  (a dropped factor p or -2 gamma, a wrong support vector, a sign slip).
* On the sphere |x|^2 = R^2 (and the RBF sphere around its centre) every
  Newton step stays on the ray through the start, so the search ends at the
  radial projection R q0 / |q0| (a step along anything but the gradient, or
  a step of the wrong length, misses it).
* For an affine f one step is the orthogonal projection onto the hyperplane,
  q0 - (f(q0) / |a|^2) a, a closed form.
* Starts outside the domain end inside it (the clamp).
* A random cubic: nearly every start ends with |f| at rounding level.
"""
import numpy as np
import pytest

import oracle as O
from paper_2406_04795_amd import inputs as I


@pytest.fixture(scope="module", autouse=True)
def _built():
    O.build(force=False)


@pytest.mark.parametrize("kind", ["poly", "rbf"])
def test_gradient_matches_central_differences(kind):
    rng = np.random.default_rng(7)
    d = 5
    dom = I.box(d)
    fm = I.random_manifold(d, 300, 3, rng, dom) if kind == "poly" else I.rbf_manifold(d, 300, rng, dom)
    fm.bias = 0.1
    for x in rng.uniform(-2.5, 2.5, size=(40, d)):
        v, g = O.f_grad(fm, x)
        assert v == O.f_at(fm, x)
        h = 1e-6
        num = np.array([(O.f_at(fm, x + h * e) - O.f_at(fm, x - h * e)) / (2 * h) for e in np.eye(d)])
        scale = np.abs(num).max() + 1e-3
        assert np.abs(g - num).max() <= 1e-6 * scale


@pytest.mark.parametrize("make,center,rmin,rmax", [
    (lambda: I.sphere_case(4, 1.3, 0.2), np.zeros(4), 0.3, 3.4),
    # exp(-gamma r^2) is convex beyond r = 1 / sqrt(2 gamma) = 1: starts in
    # the shell [1.05, 1.6] stay in that region and on their ray (from far
    # out, where the gradient vanishes, a Newton step jumps past the centre)
    (lambda: I.rbf_sphere_case(4, 1.3, 0.2, gamma=0.5), np.zeros(4), 1.05, 1.6),
])
def test_sphere_search_ends_at_the_radial_projection(make, center, rmin, rmax):
    wl = make()
    rng = np.random.default_rng(3)
    u = rng.standard_normal((200, 4))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    q0 = center + u * rng.uniform(rmin, rmax, size=(200, 1))
    q, fq = O.seed_search(wl, q0, 30)
    want = center + 1.3 * (q0 - center) / np.linalg.norm(q0 - center, axis=1, keepdims=True)
    assert np.abs(q - want).max() < 1e-12
    assert np.abs(fq).max() < 1e-12


def test_affine_f_one_step_is_the_orthogonal_projection():
    rng = np.random.default_rng(5)
    d = 4
    dom = I.box(d, 50.0)
    fm = I.random_manifold(d, 12, 1, rng, dom)
    fm.bias = 0.3
    a = fm.gamma * (fm.sv.T @ fm.alpha)          # f(x) = a.x + const
    wl = I.Workload("affine", fm, I.make_lattice(d, 0.2, rng), dom, np.zeros((1, d)))
    q0 = rng.uniform(-3, 3, size=(100, d))
    q, fq = O.seed_search(wl, q0, 1)
    f0 = np.array([O.f_at(fm, x) for x in q0])
    want = q0 - (f0 / (a @ a))[:, None] * a[None, :]
    assert np.abs(q - want).max() < 1e-12 * max(1.0, np.abs(q0).max())
    assert np.abs(fq).max() < 1e-12 * np.abs(fm.alpha).sum() * 10


def test_starts_outside_the_box_end_inside():
    wl = I.sphere_case(3, 1.0, 0.2, half=1.5)
    q0 = np.array([[9.0, 0.1, 0.0], [-4.0, -4.0, 4.0]])
    q, _ = O.seed_search(wl, q0, 0)
    assert np.array_equal(q, q0)   # zero steps: unchanged
    q, _ = O.seed_search(wl, q0, 1)
    assert (q >= wl.dom.lo).all() and (q <= wl.dom.hi).all()


def test_cubic_search_reaches_the_zero_set():
    wl = I.cubic_case(5, 500, 0.1, 0.02, seed=1, n_seeds=2)
    rng = np.random.default_rng(9)
    q0 = rng.uniform(wl.dom.lo, wl.dom.hi, size=(300, 5))
    q, fq = O.seed_search(wl, q0, 40)
    scale = np.abs(wl.f.alpha).sum() * (1 + wl.f.gamma * 30) ** 3
    assert (np.abs(fq) < 1e-12 * scale).mean() > 0.9
