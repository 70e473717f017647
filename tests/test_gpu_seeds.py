"""GPU parity of the seed search (Sec. V-A: seeds minimise |f| from given
configurations) and of the loop around the traced path (Fig. 1, Sec. IV-A:
seeds -> trace -> check -> C_free points back to the host).

The seed search runs in FP64 in the canonical order on both sides, so the
found points and their f values must equal the oracle's bit for bit; the
trace from the seeds found on the GPU must equal the oracle's trace from the
same seeds, and the C_free points returned must be exactly the oracle's free
points of that set."""
import numpy as np
import pytest

import oracle as O
from paper_2406_04795_amd import inputs as I
from test_gpu_trace import _order

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


def _search(ip, ctx, prob, q0, iters):
    import torch
    n, d = q0.shape
    q0d = torch.from_numpy(np.ascontiguousarray(q0)).cuda()
    qd = torch.empty((n, d), dtype=torch.float64, device="cuda")
    fd = torch.empty(n, dtype=torch.float64, device="cuda")
    ip.ip_seed_search(ctx.h, prob.h, q0d.data_ptr(), n, iters, qd.data_ptr(), fd.data_ptr())
    torch.cuda.synchronize()
    return qd.cpu().numpy(), fd.cpu().numpy()


CASES = {
    "cubic_d5": lambda: I.cubic_case(5, 500, 0.1, 0.02, seed=1, n_seeds=2),
    "bench_f_d6": lambda: I.config_c3(eps=2e-5, k=4),
    "rbf_d4": lambda: I.rbf_case(4, 100, 0.3, 0.3, seed=1, n_seeds=2),
    "sphere_d3": lambda: I.sphere_case(3, 1.0, 0.1),
}


@pytest.mark.parametrize("name", list(CASES))
def test_seed_search_matches_oracle(ip, ctx, name):
    wl = CASES[name]()
    print(f"seed search {name}", flush=True)
    rng = np.random.default_rng(31)
    d = wl.f.d
    # several launch tiles and a ragged tail; some starts outside the box
    q0 = rng.uniform(wl.dom.lo * 1.1, wl.dom.hi * 1.1, size=(3 * 256 + 19, d))
    want_q, want_f = O.seed_search(wl, q0, 25)
    p = ip.Problem(ctx, wl)
    try:
        q, f = _search(ip, ctx, p, q0, 25)
    finally:
        p.close()
    assert np.array_equal(q.view(np.uint64), want_q.view(np.uint64))
    assert np.array_equal(f.view(np.uint64), want_f.view(np.uint64))


def test_seeds_trace_check_and_free_points_loop(ip, ctx):
    """Seeds found on the GPU from random starts feed the trace; the set
    traced from them, its verdicts and its C_free points equal the oracle's
    for the same seeds."""
    wl = I.config_c1()
    rng = np.random.default_rng(5)
    q0 = rng.uniform(wl.dom.lo, wl.dom.hi, size=(64, 3))
    p = ip.Problem(ctx, wl)
    try:
        q, f = _search(ip, ctx, p, q0, 30)
        scale = np.abs(wl.f.alpha).sum() * 100
        keep = np.abs(f) < 1e-9 * scale
        assert keep.sum() >= 8
        seeds = q[keep]
        ip.ip_problem_set_seeds(ctx.h, p.h, seeds)
        c = ip.Cells(ctx, p)
        try:
            v, m, pts = c.download()
            nf = c.check(wl.scene)
            ver, free = c.download_check()
        finally:
            c.close()
    finally:
        p.close()
    wl.seeds = seeds
    ov, om = O.trace_direct(wl)
    o = _order(v, m)
    assert np.array_equal(v[o], ov) and np.array_equal(m[o], om)
    opts, _ = O.points(wl, ov, om)
    over = O.check(wl.scene, opts)
    assert np.array_equal(ver[o], over)
    want_free = opts[over == 0]
    assert nf == len(want_free)

    def rows(a):
        return a[np.lexsort(a.T[::-1])] if len(a) else a

    assert np.array_equal(rows(free).view(np.uint64), rows(want_free).view(np.uint64))
