"""GPU parity of the FP32-certified precision mode.

The traced set must equal the FP64 oracle's exactly (every sign decision the
FP32 bound cannot settle is taken by the canonical FP64 evaluation).  Points
must lie within 1e-5 relative of the oracle's (1e-12 where both ends were
re-evaluated in FP64, which the bound check requests whenever the FP32
values could move the point by more than half the tolerance).
"""
import numpy as np
import pytest

import oracle as O
from paper_2406_04795_amd import inputs as I
from test_gpu_trace import BATCH_CASES, CASES, oracle_batch, trace

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ip():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a device"
    from paper_2406_04795_amd import ip as _ip
    return _ip


@pytest.fixture(scope="module")
def ctx(ip):
    c = ip.Context(0)
    yield c
    c.close()


def _check_points(gpts, opts):
    scale = np.maximum(np.abs(opts).max(1, keepdims=True), 1.0)
    err = np.abs(gpts - opts) / scale
    assert err.max() <= 1e-5, err.max()


STRESS = {
    "stress_d5": lambda: I.config_c5(lam=0.35, eps=3e-3),
    "dyadic_sphere_d3": I.dyadic_sphere_case,
}


@pytest.mark.parametrize("name", list(CASES) + list(STRESS))
def test_fp32_trace_equals_fp64_oracle(ip, ctx, name):
    wl = (CASES.get(name) or STRESS[name])()
    print(f"fp32 case {name}", flush=True)
    ov, om = O.trace_direct(wl)
    gv, gm, gpts, st = trace(ip, ctx, wl, precision=ip.IP_FP32_CERTIFY)
    assert len(gv) == len(ov) and np.array_equal(gv, ov) and np.array_equal(gm, om)
    opts, _ = O.points(wl, ov, om)
    _check_points(gpts, opts)
    print(f"  cells {st['n_cells']} vertices {st['n_vertices']} fp64-basis {st['n_settled64']} "
          f"canonical fallbacks {st['n_fallback']}")
    if name == "dyadic_sphere_d3":
        # f is exactly 0.0 at some vertices: no bound can settle those signs,
        # the canonical FP64 evaluation must (s = !(f < 0) gives +)
        assert st["n_fallback"] > 0


@pytest.mark.parametrize("name", list(BATCH_CASES))
def test_fp32_batch_equals_fp64_oracle(ip, ctx, name):
    # the fused subdivision: signs of every template point from the certified
    # tiers, no vertex table
    print(f"fp32 batch case {name}", flush=True)
    wl, ov, om, ns, opts = oracle_batch(name)
    gv, gm, gpts, st = trace(ip, ctx, wl, precision=ip.IP_FP32_CERTIFY)
    assert st["n_sigma"] == ns
    assert len(gv) == len(ov) and np.array_equal(gv, ov) and np.array_equal(gm, om)
    _check_points(gpts, opts)


def test_fp32_batch_exact_zeros_take_canonical_tier(ip, ctx):
    # f is exactly 0.0 at fine vertices on the sphere: those template points
    # defer their coarse simplices to the canonical FP64 pass, and edges with
    # such an end get their points from canonical values
    wl = I.dyadic_sphere_case()
    wl.k = 2
    ov, om, ns = O.trace_batch(wl, k=2)
    gv, gm, gpts, st = trace(ip, ctx, wl, precision=ip.IP_FP32_CERTIFY)
    assert st["n_fallback"] > 0
    assert np.array_equal(gv, ov) and np.array_equal(gm, om)
    opts, _ = O.points(wl, ov, om)
    _check_points(gpts, opts)


def test_fp32_batch_budget_invariance(ip, ctx):
    make, k = BATCH_CASES["cubic_d4_k4"]
    wl = make()
    wl.k = k
    big = trace(ip, ctx, wl, precision=ip.IP_FP32_CERTIFY)
    # 12 + 16 bytes of workspace per coarse simplex at d = 4 (deferred-list
    # entry, tier-1 bound, two one-word face masks): 1024 simplices per batch
    small = trace(ip, ctx, wl, precision=ip.IP_FP32_CERTIFY, budget=28 * 1024)
    ns = big[3]["n_sigma"]
    assert small[3]["n_batches"] == (ns + 1023) // 1024 > 1
    assert np.array_equal(big[0], small[0]) and np.array_equal(big[1], small[1])
    assert np.array_equal(big[2].view(np.uint64), small[2].view(np.uint64))


@pytest.mark.parametrize("which", ["random_d6", "stress_d5"])
def test_fp32_values_within_bound(ip, ctx, which):
    import torch
    rng = np.random.default_rng(21)
    if which == "random_d6":
        d = 6
        dom = I.box(d)
        fm = I.random_manifold(d, 2000, 3, rng, dom)
        fm.bias = -2.5
        lat = I.make_lattice(d, 0.06, rng)
    else:
        w = I.config_c5(lam=0.35, eps=3e-3)
        fm, lat, dom, d = w.f, w.lat, w.dom, 5
    wl = I.Workload("fe", fm, lat, dom, np.zeros((1, d)))
    n = 4 * 4096 + 13
    # vertices inside the box (the bound is valid there)
    Y = rng.uniform(dom.lo * 0.95, dom.hi * 0.95, size=(n, d))
    V = np.floor((Y - lat.o) @ lat.Minv.T).astype(np.int32)
    want = O.feval(fm, lat, V)
    prob = ip.Problem(ctx, wl)
    try:
        vd = torch.from_numpy(V).cuda()
        fd = torch.empty(n, dtype=torch.float64, device="cuda")
        bd = torch.empty(n, dtype=torch.float64, device="cuda")
        ip.ip_feval(ctx.h, prob.h, vd.data_ptr(), n, ip.IP_FP32_CERTIFY, fd.data_ptr(), bd.data_ptr())
        torch.cuda.synchronize()
        got, bnd = fd.cpu().numpy(), bd.cpu().numpy()
    finally:
        prob.close()
    exact = bnd == 0
    assert np.array_equal(got[exact].view(np.uint64), want[exact].view(np.uint64))
    assert (np.abs(got - want) <= bnd).all()
    assert np.array_equal(got < 0, want < 0)
    assert exact.mean() < 0.5
