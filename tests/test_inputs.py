"""Input generators of the serving workload: the planted minimum is a strict
local minimum, and a planted blob is a bounded component (its trace stays
small), so serving requests have the sizes they were drawn for."""
import numpy as np
import pytest

import oracle as O
from paper_2406_04795_amd import inputs as I


@pytest.fixture(scope="module", autouse=True)
def _built():
    O.build(force=False)


@pytest.mark.parametrize("d,S,coef0", [(4, 120, 1.0), (5, 700, 3.0), (6, 2000, 3.0)])
def test_planted_minimum_is_a_strict_minimum(d, S, coef0):
    rng = np.random.default_rng(d)
    dom = I.box(d)
    fm = I.random_manifold(d, S, 3, rng, dom, alpha="normal", coef0=coef0)
    x0, H = I.planted_minimum(fm, dom, rng)
    g, H2 = I._poly_grad_hess(fm, x0)
    assert np.linalg.norm(g) <= 1e-9 * np.abs(H2).max()
    assert np.linalg.eigvalsh(H2)[0] > 0
    # f0 rises in every direction close to x0
    u = rng.standard_normal((200, d))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    f00 = I._f0(fm, x0[None])[0]
    assert (I._f0(fm, x0 + 1e-3 * u) > f00).all()


def test_serving_requests_trace_to_bounded_blobs():
    """Seeds lie on f = 0 and the traced component is the planted blob: its
    cell count stays within a few times the area model's (a leak into the
    rest of {f < 0} gives orders of magnitude more)."""
    n = 0
    for i in range(40):
        wl = I.serving_request(i)
        if wl.f.d != 4:
            continue
        fs = I.feval_np(wl.f, wl.seeds)
        assert np.abs(fs).max() <= 1e-9 * np.abs(wl.f.alpha).sum() * 100
        v, m = O.trace_direct(wl)
        assert 1000 < len(v) < 2e6
        # every vertex of every cell is within a ball around the blob centre
        x = O.coords(wl.lat, v[:: max(1, len(v) // 500)])
        c = wl.seeds.mean(0)
        r = np.linalg.norm(wl.seeds - c, axis=1).max()
        edge = np.linalg.norm(wl.lat.M, axis=0).max()
        assert np.linalg.norm(x - c, axis=1).max() < 3 * r + 4 * edge
        n += 1
        if n == 3:
            break
    assert n == 3
