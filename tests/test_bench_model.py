"""The operation counts behind bench.py's roofline figures, against counts
made independently here from the polynomial's monomials and the benchmark
workload's scene (CPU only)."""
from math import comb

import pytest

import bench
from paper_2406_04795_amd import inputs as I


def _monomials(d, p):
    """Exponent vectors of every monomial of degree <= p in d variables."""
    out = [()]
    for _ in range(d):
        out = [m + (e,) for m in out for e in range(p + 1)]
    return [m for m in out if sum(m) <= p]


@pytest.mark.parametrize("d,p", [(2, 2), (3, 2), (4, 3), (5, 3), (6, 3), (7, 3), (6, 4)])
def test_nested_form_counts_its_monomials(d, p):
    mons = _monomials(d, p)
    assert len(mons) == comb(d + p, p)
    nonconst = [m for m in mons if sum(m) > 0]
    below = [m for m in nonconst if sum(m) < p]
    assert bench.nest_flops(d, p) == 2 * len(nonconst) + len(below) + 1


def test_benchmark_workload_counts():
    wl = I.config_c3(eps=2e-5, k=4)
    d, M = wl.f.d, comb(wl.f.d + wl.f.p, wl.f.p)
    assert bench.nest_flops(d, wl.f.p) == 194
    sc = wl.scene
    n_obs = len(sc.osph_r) + len(sc.obox_l) + len(getattr(sc, "ocyl_rh", []))
    assert n_obs == 16
    # per link: sincos 42, transform 36, ball centre 18, half its squared
    # norm 6; per link and obstacle: three fma
    assert bench.check_flops_per_cell(wl) == d * (42 + 36 + 18 + 6) + d * 6 * n_obs == 1188
    # d + 1 vertex coordinates (d^2 fma) and the region bound ((p + 1) per
    # non-constant monomial)
    assert bench.prep_flops_per_simplex(wl) == (d + 1) * 2 * d * d + (wl.f.p + 1) * (M - 1) == 836
    # both ends: coordinates, monomial value with bound sums, bound test;
    # then t and the point
    assert bench.points_flops_per_cell(wl) == 2 * (2 * d * d + 5 * (M - 1) + 2) + 3 * d + 2 == 998
    # a fused-subdivision point: FP64 coordinates and the nested FP32 value
    st = {"n_vertices": 1}
    assert bench.subdivide_flops(st, wl) == 2 * d * d + 194 == 266
