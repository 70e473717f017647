"""Pins of the oracle against facts fixed outside it.

Each test checks the oracle against something it does not itself compute:
the paper's worked examples (Figs. 2 and 5, stored under tests/golden/),
closed-form counts (Sec. V-A, V-B), brute force over the Kuhn/Freudenthal
description of the triangulation, geometric invariants of the traced complex,
closed forms of simple level sets, and textbook distance routines.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

import oracle as O
from paper_2406_04795_amd import inputs as I

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module", autouse=True)
def _built():
    O.build(force=False)


def _bits(parts):
    return [sum(1 << j for j in p) for p in parts]


def _cum_vertices(d, v, parts):
    """Independent restatement: walk the cycle of root sums from v."""
    out = [list(v)]
    cur = list(v)
    for p in parts[:-1]:
        for j in p:
            if j < d:
                cur[j] += 1
            else:
                cur = [c - 1 for c in cur]
        out.append(list(cur))
    return out


# --------------------------------------------------------------------------
# Worked examples
# --------------------------------------------------------------------------
def test_fig2_worked_example():
    g = json.load(open(os.path.join(GOLD, "fig2_permutahedral.json")))
    d = g["d"]
    for case in g["cases"]:
        vc, pc = O.canonical(d, case["v"], _bits(case["partition"]))
        # already canonical (d in the last part): unchanged
        assert list(vc) == case["v"]
        assert list(pc) == _bits(case["partition"])
        verts = _cum_vertices(d, vc, case["partition"])
        assert verts == case["vertices"]


def test_fig2_canonical_rotation_is_lexicographic_min():
    # every rotation of the cycle describes the same triangle; the canonical
    # form must pick the componentwise-minimum vertex (Sec. IV-B)
    d = 2
    parts = [[0], [1], [2]]
    v = [0, 0]
    verts = _cum_vertices(d, v, parts)
    for r in range(3):
        rot = parts[r:] + parts[:r]
        start = verts[r]
        vc, pc = O.canonical(d, start, _bits(rot))
        assert list(vc) == [0, 0]
        assert list(pc) == _bits(parts)


def test_fig5_template_matches_figure():
    g = json.load(open(os.path.join(GOLD, "fig5_subdivision.json")))
    for case in g["cases"]:
        d, k = case["d"], case["k"]
        pts, eu, er = O.template(d, k)
        assert len(pts) == case["n_points"] == math.comb(d + k, d)
        edges = set()
        for u, r in zip(eu, er):
            a = tuple(int(x) for x in u)
            b = tuple(int(u[j]) + ((int(r) >> j) & 1) for j in range(d))
            edges.add(frozenset([a, b]))
        P = {n: tuple(c) for n, c in case["points"].items()}
        # the first local edge (red in the figure)
        fe = case["first_local_edge"]
        a = tuple(fe["u"])
        b = tuple(a[j] + (1 if j in fe["R"] else 0) for j in range(d))
        assert frozenset([a, b]) in edges
        # halves of the coarse edges and the dashed edges are all template edges
        names = [n for n in P if len(n) == 2]
        drawn = set()
        for n in names:
            i = n[1]
            for m in names:
                j = m[1]
                if i < j:
                    mid = "v" + i + j
                    drawn.add(frozenset([P[n], P[mid]]))
                    drawn.add(frozenset([P[mid], P[m]]))
        for x, y in case["dashed"]:
            drawn.add(frozenset([P[x], P[y]]))
        assert len(drawn) == case["n_edges_drawn"]
        assert drawn <= edges
        assert len(edges) == case["n_edges_drawn"] + case.get("n_interior_diagonals", 0)


@pytest.mark.parametrize("d,k", [(2, 2), (2, 3), (3, 2), (3, 3), (4, 2)])
def test_template_subdivides_into_k_pow_d_simplices_and_is_a_ball(d, k):
    pts, eu, er = O.template(d, k)
    inside = {tuple(int(x) for x in p) for p in pts}

    # fine Kuhn simplices (y, pi) with every vertex inside the coarse simplex
    lo = -1
    simp = set()
    for y in itertools.product(range(lo, k + 1), repeat=d):
        for pi in itertools.permutations(range(d)):
            vs = [tuple(y)]
            cur = list(y)
            for j in pi:
                cur[j] += 1
                vs.append(tuple(cur))
            if all(v in inside for v in vs):
                simp.add(frozenset(vs))
    assert len(simp) == k ** d
    # Euler characteristic of the subdivided simplex (a d-ball) is 1
    faces = set()
    for s in simp:
        s = sorted(s)
        for r in range(1, d + 2):
            for c in itertools.combinations(s, r):
                faces.add(c)
    chi = sum((-1) ** (len(f) - 1) for f in faces)
    assert chi == 1
    n_edges = sum(1 for f in faces if len(f) == 2)
    assert n_edges == len(eu)


@pytest.mark.parametrize("d,k", [(2, 2), (3, 2), (3, 3)])
def test_template_reached_from_first_local_edge(d, k):
    """Sec. V-B: the subdivision's edges are found from the first local edge
    by coface-then-edge queries; that search equals direct enumeration."""
    pts, eu, er = O.template(d, k)
    want = {(tuple(int(x) for x in u), int(r)) for u, r in zip(eu, er)}

    def inside(u):
        return u[0] <= k and all(u[i] >= u[i + 1] for i in range(d - 1)) and u[-1] >= 0

    start = (tuple([0] * d), 1)
    seen = {start}
    todo = [start]
    while todo:
        v, r = todo.pop()
        for tri in O.cofaces2(d, np.array(v, np.int32), r):
            vs = [tuple(int(x) for x in t) for t in tri]
            if not all(inside(t) for t in vs):
                continue
            for a, b in ((0, 1), (0, 2), (1, 2)):
                A, B = np.array(vs[a]), np.array(vs[b])
                df = B - A
                if (df >= 0).all():
                    e = (tuple(int(x) for x in A), int(sum(1 << j for j in range(d) if df[j])))
                else:
                    e = (tuple(int(x) for x in B), int(sum(1 << j for j in range(d) if df[j])))
                if e not in seen:
                    seen.add(e)
                    todo.append(e)
    assert seen == want


# --------------------------------------------------------------------------
# Coface queries vs the Freudenthal/Kuhn description
# --------------------------------------------------------------------------
def _kuhn_simplices_around_origin(d):
    out = []
    for y in itertools.product(range(-2, 2), repeat=d):
        for pi in itertools.permutations(range(d)):
            vs = [tuple(y)]
            cur = list(y)
            for j in pi:
                cur[j] += 1
                vs.append(tuple(cur))
            out.append(frozenset(vs))
    return out


@pytest.mark.parametrize("d", [2, 3, 4])
def test_cofaces_match_kuhn_brute_force_and_count_formulas(d):
    K = _kuhn_simplices_around_origin(d)
    zero = tuple([0] * d)
    for R in range(1, 1 << d):
        b = tuple((R >> j) & 1 for j in range(d))
        containing = [s for s in K if zero in s and b in s]
        # n-cofaces (Sec. V-B): |P|! |Q|!
        nP = bin(R).count("1")
        nQ = d + 1 - nP
        nc = O.ncofaces(d, np.zeros(d, np.int32), R)
        assert len(nc) == math.factorial(nP) * math.factorial(nQ)
        got = set()
        for row in nc:
            v, w = row[:d], row[d:]
            vs = [tuple(int(x) for x in v)]
            cur = [int(x) for x in v]
            for j in w:
                cur[int(j)] += 1
                vs.append(tuple(cur))
            # canonical vertex is the componentwise minimum
            assert all(min(t[j] for t in vs) == v[j] for j in range(d))
            got.add(frozenset(vs))
        assert got == set(containing)
        # 2-cofaces (Sec. V-A): (2^|P| - 2) + (2^|Q| - 2)
        tris = O.cofaces2(d, np.zeros(d, np.int32), R)
        assert len(tris) == (2 ** nP - 2) + (2 ** nQ - 2)
        got2 = {frozenset(tuple(int(x) for x in t) for t in tri) for tri in tris}
        assert len(got2) == len(tris)
        want2 = set()
        for s in containing:
            for c in s:
                if c != zero and c != b:
                    want2.add(frozenset([zero, b, c]))
        assert got2 == want2


def test_edges_per_n_simplex_is_d_plus_1_choose_2():
    # Sec. V-A prints n(n-1)/2; an n-simplex has C(n+1, 2) edges
    for d in range(2, 8):
        assert len(list(itertools.combinations(range(d + 1), 2))) == math.comb(d + 1, 2)
        assert math.comb(d + 1, 2) != d * (d - 1) // 2


# --------------------------------------------------------------------------
# Lattice, location, f
# --------------------------------------------------------------------------
@pytest.mark.parametrize("d", [2, 3, 4, 5, 6, 7])
def test_coxeter_frame_roots_are_equal_length_equal_angle(d):
    lam = 0.37
    M = I.coxeter_frame(d, lam)
    roots = [M[:, j] for j in range(d)] + [-M.sum(1)]
    L = [np.linalg.norm(r) for r in roots]
    assert np.allclose(L, L[0])
    cos = [np.dot(a, b) / (L[0] ** 2) for a, b in itertools.combinations(roots, 2)]
    assert np.allclose(cos, -1.0 / d)


@pytest.mark.parametrize("d", [2, 3, 5, 6])
def test_locate_contains_point(d):
    rng = np.random.default_rng(d)
    lat = I.make_lattice(d, 0.3, rng)
    for _ in range(200):
        y = rng.uniform(-3, 3, d)
        v, w = O.locate(lat, y)
        vs = [v.copy()]
        cur = v.copy()
        for j in w:
            cur[j] += 1
            vs.append(cur.copy())
        X = O.coords(lat, np.array(vs))
        # barycentric coordinates: y = sum_m b_m X_m, sum b = 1
        A = np.vstack([X.T, np.ones(d + 1)])
        b = np.linalg.solve(A, np.r_[y, 1.0])
        assert (b >= -1e-9).all()


def test_f_sphere_closed_form():
    for d in (2, 3, 6):
        wl = I.sphere_case(d, 1.3, 0.2)
        rng = np.random.default_rng(1)
        V = rng.integers(-20, 20, size=(50, d)).astype(np.int32)
        X = O.coords(wl.lat, V)
        f = O.feval(wl.f, wl.lat, V)
        want = (X ** 2).sum(1) - 1.3 ** 2
        assert np.allclose(f, want, rtol=1e-13, atol=1e-13)


def test_f_degree_one_is_affine():
    # p = 1: f(x) = gamma <sum_i alpha_i s_i, x> + coef0 sum alpha + b
    rng = np.random.default_rng(2)
    d = 4
    dom = I.box(d)
    fm = I.random_manifold(d, 37, 1, rng, dom)
    fm.bias = 0.25
    w = fm.sv.T @ fm.alpha
    for _ in range(20):
        x = rng.uniform(-3, 3, d)
        want = fm.gamma * np.dot(w, x) + fm.coef0 * fm.alpha.sum() + fm.bias
        assert abs(O.f_at(fm, x) - want) < 1e-12 * (1 + np.abs(fm.alpha).sum() * 10)


# --------------------------------------------------------------------------
# Traces vs brute force and invariants
# --------------------------------------------------------------------------
def _as_set(v, m):
    return set(map(tuple, np.c_[v, m].tolist()))


@pytest.mark.parametrize("d,R,lam", [(2, 1.0, 0.05), (3, 1.0, 0.1), (4, 1.0, 0.3)])
def test_sphere_trace_equals_brute_force(d, R, lam):
    wl = I.sphere_case(d, R, lam)
    v, m = O.trace_direct(wl)
    bv, bm = O.brute(wl)
    assert len(v) > 0
    assert np.array_equal(v, bv) and np.array_equal(m, bm)


def test_closed_quadric_trace_equals_brute_force():
    wl = I.config_c1()
    v, m = O.trace_direct(wl)
    bv, bm = O.brute(wl)
    assert np.array_equal(v, bv) and np.array_equal(m, bm)


def test_open_cubic_trace_is_subset_of_brute_force():
    wl = I.cubic_case(3, 40, 0.25, 0.05, seed=3, n_seeds=2)
    s = _as_set(*O.trace_direct(wl))
    b = _as_set(*O.brute(wl))
    assert s and s <= b


def _sign_table(wl, verts):
    verts = np.array(sorted(verts), np.int32)
    f = O.feval(wl.f, wl.lat, verts)
    return {tuple(int(x) for x in v): (not (fv < 0)) for v, fv in zip(verts, f)}


def test_triangle_rule_every_coface_has_two_traced_edges():
    """Sec. V-A: in a 2-simplex exactly two edges cross the manifold, and the
    search keeps both (one is the edge it came from)."""
    wl = I.config_c1()
    v, m = O.trace_direct(wl)
    traced = _as_set(v, m)
    d = wl.f.d
    verts = set()
    tri_all = []
    for vi, mi in zip(v, m):
        for tri in O.cofaces2(d, vi, int(mi)):
            ts = [tuple(int(x) for x in t) for t in tri]
            tri_all.append(ts)
            verts.update(ts)
    X = O.coords(wl.lat, np.array(sorted(verts), np.int32))
    inb = {t: bool(((x >= wl.dom.lo) & (x <= wl.dom.hi)).all())
           for t, x in zip(sorted(verts), X)}
    sg = _sign_table(wl, verts)
    for ts in tri_all:
        if not all(inb[t] for t in ts):
            continue
        cross = []
        for a, b in ((0, 1), (0, 2), (1, 2)):
            if sg[ts[a]] != sg[ts[b]]:
                A, B = np.array(ts[a]), np.array(ts[b])
                lo = A if (B - A >= 0).all() else B
                mask = int(sum(1 << j for j in range(d) if A[j] != B[j]))
                cross.append(tuple(int(x) for x in lo) + (mask,))
        assert len(cross) == 2
        assert all(c in traced for c in cross)


def _traced_simplices(wl, v, m):
    d = wl.f.d
    simp = set()
    for vi, mi in zip(v, m):
        for row in O.ncofaces(d, vi, int(mi)):
            vs = [tuple(int(x) for x in row[:d])]
            cur = [int(x) for x in row[:d]]
            for j in row[d:]:
                cur[int(j)] += 1
                vs.append(tuple(cur))
            simp.add(frozenset(vs))
    return simp


@pytest.mark.parametrize("d,lam", [(2, 0.1), (3, 0.2), (4, 0.45)])
def test_closed_manifold_and_euler_characteristic_of_sphere(d, lam):
    """Every mixed-sign facet of a traced n-simplex is shared by exactly two
    traced n-simplices (a closed PL manifold), and the Euler characteristic of
    the traced (d-1)-sphere is 1 + (-1)^(d-1)."""
    wl = I.sphere_case(d, 1.0, lam)
    v, m = O.trace_direct(wl)
    simp = _traced_simplices(wl, v, m)
    verts = set().union(*simp)
    sg = _sign_table(wl, verts)
    count = {}
    faces = set()
    for s in simp:
        s = sorted(s)
        for f in itertools.combinations(s, d):
            if len({sg[x] for x in f}) == 2:
                count[f] = count.get(f, 0) + 1
        for r in range(2, d + 2):
            for f in itertools.combinations(s, r):
                if len({sg[x] for x in f}) == 2:
                    faces.add(f)
    assert set(count.values()) == {2}
    chi = sum((-1) ** (len(f) - 2) for f in faces)
    assert chi == 1 + (-1) ** (d - 1)


# Asymptotic density of crossing edges for a hypersurface of area A:
# N lam^(d-1) / A -> C_d = kappa_d sqrt(d+1) sum_R ||Lambda 1_R||,
# kappa_d = Gamma(d/2) / (sqrt(pi) Gamma((d+1)/2)) = E|cos| of a random
# direction against a fixed normal; ||Lambda 1_R||^2 = |R|(d+1-|R|)/(d+1).
def _C(d):
    kappa = math.gamma(d / 2) / (math.sqrt(math.pi) * math.gamma((d + 1) / 2))
    s = sum(math.comb(d, r) * math.sqrt(r * (d + 1 - r) / (d + 1)) for r in range(1, d + 1))
    return kappa * math.sqrt(d + 1) * s


def _sphere_area(d, R):
    # area of the (d-1)-sphere of radius R in R^d
    return 2 * math.pi ** (d / 2) / math.gamma(d / 2) * R ** (d - 1)


@pytest.mark.parametrize("d,lam,tol", [(2, 0.01, 0.02), (3, 0.1, 0.01), (4, 0.25, 0.03)])
def test_sphere_crossing_count_scales_with_area(d, lam, tol):
    assert abs(_C(3) - 6.464) < 1e-3
    wl = I.sphere_case(d, 1.0, lam)
    v, m = O.trace_direct(wl)
    pred = _C(d) * _sphere_area(d, 1.0) / lam ** (d - 1)
    assert abs(len(v) / pred - 1) < tol


# --------------------------------------------------------------------------
# Batch triangulation
# --------------------------------------------------------------------------
def test_batch_with_k1_equals_direct():
    wl = I.config_c1()
    v, m = O.trace_direct(wl)
    bv, bm, ns = O.trace_batch(wl, k=1)
    assert np.array_equal(v, bv) and np.array_equal(m, bm)


@pytest.mark.parametrize("k", [2, 3])
def test_batch_edges_are_intersecting_and_inside_sigma(k):
    wl = I.sphere_case(3, 1.0, 0.08)
    bv, bm, ns = O.trace_batch(wl, k=k)
    b = _as_set(*O.brute(wl))
    got = _as_set(bv, bm)
    assert got <= b
    # near-complete coverage of the direct trace for a smooth sphere
    direct = _as_set(*O.trace_direct(wl))
    assert got <= direct and len(got) > 0.99 * len(direct)
    # every fine edge lies inside one of the coarse simplices (Eq. 2 with >=):
    # local coordinates u_i = y_{w_i} - k v_{w_i} satisfy k >= u_0 >= ... >= 0
    sig = O.batch_sigma(wl, k=k)
    d = 3
    V0, W = sig[:, :d].astype(np.int64), sig[:, d:].astype(np.int64)
    rng = np.random.default_rng(0)

    def inside(y):
        u = np.take_along_axis(y[None, :] - k * V0, W, axis=1)
        return (u[:, 0] <= k) & (np.diff(u, axis=1) <= 0).all(1) & (u[:, -1] >= 0)

    for i in rng.choice(len(bv), 50, replace=False):
        a = bv[i].astype(np.int64)
        b = a + np.array([(int(bm[i]) >> j) & 1 for j in range(d)])
        assert (inside(a) & inside(b)).any()


# --------------------------------------------------------------------------
# Intersection points
# --------------------------------------------------------------------------
def test_points_of_affine_f_are_roots():
    rng = np.random.default_rng(5)
    d = 3
    dom = I.box(d)
    fm = I.random_manifold(d, 10, 1, rng, dom)
    fm.bias = -fm.coef0 * fm.alpha.sum() + 0.1
    lat = I.make_lattice(d, 0.2, rng)
    seeds = I.bisection_seeds(fm, dom, rng, 2)
    wl = I.Workload("affine", fm, lat, dom, seeds)
    v, m = O.trace_direct(wl)
    pts, t = O.points(wl, v, m)
    assert ((t >= 0) & (t <= 1)).all()
    vals = np.array([O.f_at(fm, p) for p in pts[:500]])
    scale = np.abs(fm.alpha).sum() * 10
    assert np.abs(vals).max() < 1e-12 * scale


def test_points_of_sphere_lie_near_sphere():
    wl = I.sphere_case(3, 1.0, 0.1)
    v, m = O.trace_direct(wl)
    pts, t = O.points(wl, v, m)
    r = np.linalg.norm(pts, axis=1)
    lam_edge = 0.1 * math.sqrt(3 / 4) * math.sqrt(2)  # longest edge ~ lam sqrt(|R|(d+1-|R|)/(d+1))
    assert np.abs(r - 1.0).max() < lam_edge ** 2


# --------------------------------------------------------------------------
# Collision check
# --------------------------------------------------------------------------
def test_sincos_against_library():
    for q in np.linspace(-math.pi, math.pi, 2001):
        s, c = O.sincos(q)
        assert abs(s - math.sin(q)) <= 2.5e-16
        assert abs(c - math.cos(q)) <= 2.5e-16
    assert O.sincos(0.0) == (0.0, 1.0)


def test_fk_planar_arm_hand_poses():
    sc = I.planar_arm_scene(np.random.default_rng(0))
    T = O.fk(sc, [0.0, 0.0, 0.0])
    assert np.allclose(T[:, [3, 7, 11]], [[0, 0, 0], [1, 0, 0], [2, 0, 0]])
    T = O.fk(sc, [math.pi / 2, 0.0, 0.0])
    assert np.allclose(T[:, [3, 7, 11]], [[0, 0, 0], [0, 1, 0], [0, 2, 0]], atol=1e-15)
    T = O.fk(sc, [0.0, math.pi / 2, -math.pi / 2])
    assert np.allclose(T[:, [3, 7, 11]], [[0, 0, 0], [1, 0, 0], [1, 1, 0]], atol=1e-15)
    # end effector of the last link frame: x axis after the turns
    assert np.allclose(T[2, [0, 4, 8]], [1, 0, 0], atol=1e-15)


def test_planar_arm_hand_cases():
    sc = I.planar_arm_scene(np.random.default_rng(0))
    sc.osph_c = np.array([[1.5, 0.2, 0.0]])
    sc.osph_r = np.array([0.3])
    assert O.check(sc, [[0.0, 0.0, 0.0]])[0] == 1
    sc.osph_c = np.array([[1.5, 0.4, 0.0]])
    assert O.check(sc, [[0.0, 0.0, 0.0]])[0] == 0
    # touching counts as collision (Appendix A: no collision only if > r)
    sc.osph_c = np.array([[1.5, 0.25, 0.0]])
    sc.osph_r = np.array([0.25])
    assert O.check(sc, [[0.0, 0.0, 0.0]])[0] == 1


def _clamp_dist2_box(c, T, l):
    R = np.array(T).reshape(3, 4)[:, :3]
    t = np.array(T).reshape(3, 4)[:, 3]
    p = np.abs(R.T @ (np.asarray(c) - t))
    g = np.maximum(p - np.asarray(l) / 2, 0)
    return float((g ** 2).sum())


def test_sphere_box_matches_clamp_distance():
    rng = np.random.default_rng(7)
    for _ in range(4000):
        Rm = I._random_rotation(rng)
        T = I._T(Rm, rng.uniform(-1, 1, 3))
        l = rng.uniform(0.1, 1.0, 3)
        c = rng.uniform(-2, 2, 3)
        r = rng.uniform(0.01, 0.6)
        want = _clamp_dist2_box(c, T, l) <= r * r
        assert O.sphere_box(c, r, T, l) == want


def test_sphere_box_exact_boundaries():
    T = I._T()
    l = np.array([2.0, 2.0, 2.0])     # half extents 1
    # face region, exactly touching
    assert O.sphere_box([1.5, 0.0, 0.0], 0.5, T, l) == 1
    assert O.sphere_box([1.5, 0.0, 0.0], 0.25, T, l) == 0
    # edge region: distance to the edge (1,1,z) is sqrt(0.5^2+0.5^2)
    assert O.sphere_box([1.5, 1.5, 0.0], 0.75, T, l) == 1
    assert O.sphere_box([1.5, 1.5, 0.0], 0.70, T, l) == 0
    # vertex region: distance sqrt(3)*0.5
    assert O.sphere_box([1.5, 1.5, 1.5], 0.87, T, l) == 1
    assert O.sphere_box([1.5, 1.5, 1.5], 0.86, T, l) == 0
    # inside
    assert O.sphere_box([0.1, 0.2, 0.3], 0.01, T, l) == 1


def _seg_dist2(p0, p1, c):
    p0, p1, c = map(np.asarray, (p0, p1, c))
    u = p1 - p0
    t = 0.0 if u @ u == 0 else np.clip((c - p0) @ u / (u @ u), 0, 1)
    e = c - (p0 + t * u)
    return float(e @ e)


def test_capsule_and_sphere_predicates_match_textbook():
    rng = np.random.default_rng(8)
    for _ in range(4000):
        p0, p1, c = rng.uniform(-1, 1, (3, 3))
        rc, rs = rng.uniform(0, 0.5, 2)
        assert O.capsule_sphere(p0, p1, rc, c, rs) == (_seg_dist2(p0, p1, c) <= (rc + rs) ** 2)
        a, b = rng.uniform(-1, 1, (2, 3))
        assert O.sphere_sphere(a, rc, b, rs) == (float(((a - b) ** 2).sum()) <= (rc + rs) ** 2)


def test_check_mixes_verdicts_on_c1():
    wl = I.config_c1()
    v, m = O.trace_direct(wl)
    pts, _ = O.points(wl, v, m)
    ver = O.check(wl.scene, pts)
    assert 0 < ver.mean() < 1
