"""Serving loop: results are the same alone and in a concurrent mix, and
admission respects the memory pool."""
import numpy as np
import pytest

import oracle as O
from paper_2406_04795_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ip():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a device"
    from paper_2406_04795_amd import ip as _ip
    return _ip


def _mix():
    c1 = I.config_c1()
    reqs = [
        (c1, c1.scene, 0),
        (I.sphere_case(3, 1.0, 0.05), None, 1),
        (I.cubic_case(4, 200, 0.1, 0.01, seed=3, n_seeds=4), None, 0),
        (I.cubic_case(5, 500, 0.35, 0.02, seed=1, n_seeds=4),
         I.spatial_arm_scene(np.random.default_rng(1), 5, capsule_r=0.05), 1),
        (I.cubic_case(6, 2000, 0.6, 0.002, seed=2, n_seeds=4),
         I.spatial_arm_scene(np.random.default_rng(2), 6, spheres_per_link=3, n_obox=4), 0),
        (I.sphere_case(7, 1.0, 0.9), None, 1),
    ]
    wl = I.cubic_case(4, 200, 0.08, 0.01, seed=3, n_seeds=4)
    wl.k = 4
    reqs.append((wl, None, 0))
    return reqs


def _run(ip, reqs, slots, pool=0, mem=0):
    srv = ip.ip_server_create(0, pool, slots)
    try:
        ids = [ip.ip_server_submit(srv, wl, precision=prec, scene=sc, mem_bytes=mem)
               for wl, sc, prec in reqs]
        return [ip.ip_server_wait(srv, i) for i in ids]
    finally:
        ip.ip_server_destroy(srv)


def _rows(a):
    return a[np.lexsort(a.T[::-1])] if a is not None and len(a) else a


def test_results_same_alone_and_in_mix(ip):
    reqs = _mix()
    alone = [_run(ip, [r], 1)[0] for r in reqs]
    mixed = _run(ip, reqs + reqs, 4)
    for i, a in enumerate(alone):
        for m in (mixed[i], mixed[i + len(reqs)]):
            assert a["status"] == 0 and m["status"] == 0, (a["error"], m["error"])
            assert a["n_cells"] > 0
            assert a["n_cells"] == m["n_cells"] and a["digest"] == m["digest"]
            assert a["n_free"] == m["n_free"]
            if "free_pts" in a:
                assert np.array_equal(_rows(a["free_pts"]), _rows(m["free_pts"]))
    # overlap: with 4 slots some requests started before others finished
    starts = sorted(r["t_start"] for r in mixed)
    dones = sorted(r["t_done"] for r in mixed)
    assert starts[3] < dones[0]


def _no_overlap(res):
    spans = sorted((r["t_admit"], r["t_done"]) for r in res)
    for (s0, d0), (s1, d1) in zip(spans, spans[1:]):
        assert s1 >= d0


def test_admission_by_memory(ip):
    reqs = _mix()[:4]
    # every request is given the whole pool: their traces run one at a time
    res = _run(ip, reqs, 4, pool=1 << 30, mem=1 << 30)
    assert all(r["admitted_bytes"] == 1 << 30 and r["n_probe_edges"] == 0 for r in res)
    _no_overlap(res)


def test_admission_by_projection(ip):
    """The library projects each request's bytes from a coarse trace and
    admits by that: with a pool below any two projections the traces run one
    at a time, with a pool above all of them they overlap; the projections
    are the same in both runs."""
    reqs = _mix()
    big = _run(ip, reqs, 4, pool=1 << 40)
    proj = [r["admitted_bytes"] for r in big]
    assert all(r["status"] == 0 for r in big)
    assert sum(r["n_probe_edges"] > 0 for r in big) >= 3
    # the projection is the documented one: 1.25 nc kc^(d-1) cells at
    # 8 + 16 d + 57 bytes each, plus 64 MiB
    for (wl, _, _), r in zip(reqs, big):
        d = wl.f.d
        kc = wl.k if wl.k >= 2 else 4
        want = int(1.25 * r["n_probe_edges"] * kc ** (d - 1) * (8 + 16 * d + 57)) + (64 << 20)
        assert abs(r["admitted_bytes"] - want) <= 1 + want * 1e-12
    starts = sorted(r["t_admit"] for r in big)
    dones = sorted(r["t_done"] for r in big)
    assert starts[1] < dones[0]
    small = _run(ip, reqs, 4, pool=2 * min(proj) - 1)
    assert [r["admitted_bytes"] for r in small] == proj
    _no_overlap(small)
    for a, b in zip(big, small):
        assert a["digest"] == b["digest"] and a["n_cells"] == b["n_cells"]


def test_kept_cells_match_oracle(ip):
    wl = I.config_c1()
    srv = ip.ip_server_create(0, 0, 2)
    try:
        rid = ip.ip_server_submit(srv, wl, scene=wl.scene, flags=ip.IP_KEEP_CELLS)
        r = ip.ip_server_wait(srv, rid)
    finally:
        ip.ip_server_destroy(srv)
    v, m, pts = r["cells"]
    o = np.lexsort([m] + [v[:, j] for j in reversed(range(3))])
    ov, om = O.trace_direct(wl)
    assert np.array_equal(v[o], ov) and np.array_equal(m[o], om)
    opts, _ = O.points(wl, ov, om)
    ver = O.check(wl.scene, opts)
    assert r["n_free"] == int((ver == 0).sum())
    assert np.array_equal(_rows(r["free_pts"]), _rows(opts[ver == 0]))
