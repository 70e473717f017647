"""Seeded synthetic inputs for the tracing and checking workloads.

Everything here builds *inputs*: the manifold function's parameters (a
polynomial-kernel decision function, the form a kernel SVM yields), the
lattice frame, the domain box, seed points on the manifold and the robot /
obstacle scene.  Nothing here traces, evaluates signs on the lattice or checks
collisions; both the GPU library and the reference implementation read the
arrays produced here.

The paper learns f with an SVM from planner samples and finds seeds with
SLSQP (Sec. IV-A, V-A); neither samples nor trained models exist here, so f
is drawn at random with the shapes the paper's workloads have and seeds come
from bisection along segments that cross the zero set.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

PI = math.pi


@dataclass
class Manifold:
    """f(x) = sum_i alpha_i K(s_i, x) + bias with the polynomial kernel
    K = (gamma <s_i, x> + coef0)^p or the RBF kernel K = exp(-gamma |x - s_i|^2)."""

    d: int
    p: int
    gamma: float
    coef0: float
    bias: float
    sv: np.ndarray      # (S, d) float64
    alpha: np.ndarray   # (S,) float64
    kernel: str = "poly"  # "poly" or "rbf"

    @property
    def S(self) -> int:
        return int(self.sv.shape[0])


@dataclass
class Lattice:
    """x(v) = o + M v; M is a scaled Coxeter A~_d frame, Minv its inverse."""

    M: np.ndarray       # (d, d) float64 row-major
    Minv: np.ndarray    # (d, d)
    o: np.ndarray       # (d,)
    lam: float


@dataclass
class Domain:
    lo: np.ndarray
    hi: np.ndarray


@dataclass
class Scene:
    """Serial revolute robot (link spheres / capsules) and obstacles."""

    joint_T: np.ndarray          # (n, 12) parent->joint transforms, row-major [R|t]
    joint_axis: np.ndarray       # (n,) int32 in {0,1,2}
    lsph_link: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))
    lsph_c: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    lsph_r: np.ndarray = field(default_factory=lambda: np.zeros(0))
    lcap_link: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))
    lcap_p0: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    lcap_p1: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    lcap_r: np.ndarray = field(default_factory=lambda: np.zeros(0))
    osph_c: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    osph_r: np.ndarray = field(default_factory=lambda: np.zeros(0))
    obox_T: np.ndarray = field(default_factory=lambda: np.zeros((0, 12)))
    obox_l: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    ocyl_T: np.ndarray = field(default_factory=lambda: np.zeros((0, 12)))   # axis = local z
    ocyl_rh: np.ndarray = field(default_factory=lambda: np.zeros((0, 2)))   # radius, height


@dataclass
class Workload:
    name: str
    f: Manifold
    lat: Lattice
    dom: Domain
    seeds: np.ndarray            # (n_seeds, d) float64
    k: int = 1                   # 1 = direct trace, >= 2 = batch triangulation
    scene: Scene | None = None
    note: str = ""


# --------------------------------------------------------------------------
# Lattice frame
# --------------------------------------------------------------------------
def coxeter_frame(d: int, lam: float) -> np.ndarray:
    """Upper-triangular M with M^T M = lam^2 (I - 11^T/(d+1)).

    With that Gram matrix the images of e_0..e_{d-1} and of -(1,...,1) have
    equal length and equal pairwise angles, which turns the integer lattice's
    Kuhn triangulation into the Coxeter triangulation of type A~_d.
    """
    G = np.eye(d) - np.ones((d, d)) / (d + 1)
    U = np.linalg.cholesky(G).T
    return np.ascontiguousarray(lam * U)


def make_lattice(d: int, lam: float, rng: np.random.Generator) -> Lattice:
    M = coxeter_frame(d, lam)
    Minv = np.ascontiguousarray(np.linalg.inv(M))
    o = M @ rng.uniform(0.0, 1.0, d)      # random offset within one cell
    return Lattice(M=M, Minv=Minv, o=np.ascontiguousarray(o), lam=lam)


def box(d: int, half: float = PI) -> Domain:
    return Domain(lo=np.full(d, -half), hi=np.full(d, half))


# --------------------------------------------------------------------------
# Manifold parameters (numpy evaluation used only to size inputs and seeds)
# --------------------------------------------------------------------------
def _f0(fm: Manifold, X: np.ndarray, chunk: int = 8192) -> np.ndarray:
    out = np.empty(X.shape[0])
    if fm.kernel == "rbf":
        s2 = (fm.sv ** 2).sum(1)
        for a in range(0, X.shape[0], chunk):
            Xa = X[a:a + chunk]
            d2 = np.maximum((Xa ** 2).sum(1)[:, None] + s2[None, :] - 2.0 * (Xa @ fm.sv.T), 0.0)
            out[a:a + chunk] = np.exp(-fm.gamma * d2) @ fm.alpha
        return out
    for a in range(0, X.shape[0], chunk):
        t = fm.gamma * (X[a:a + chunk] @ fm.sv.T) + fm.coef0
        tp = t.copy()
        for _ in range(fm.p - 1):
            tp *= t
        out[a:a + chunk] = tp @ fm.alpha
    return out


def feval_np(fm: Manifold, X: np.ndarray) -> np.ndarray:
    """f at points X (n, d) in plain numpy; for input generation only."""
    return _f0(fm, X) + fm.bias


def random_manifold(d, S, p, rng, dom: Domain, alpha="normal", gamma=None, coef0=1.0):
    sv = rng.uniform(dom.lo, dom.hi, size=(S, d))
    a = rng.standard_normal(S)
    if alpha == "halfnormal":
        a = np.abs(a)
    g = 1.0 / d if gamma is None else gamma
    return Manifold(d=d, p=p, gamma=float(g), coef0=float(coef0), bias=0.0,
                    sv=np.ascontiguousarray(sv), alpha=np.ascontiguousarray(a))


def sphere_manifold(d: int, R: float, center=None) -> Manifold:
    """||x - c||^2 - R^2 written as a degree-2 kernel expansion.

    (<e_j, x> - c_j)^2 summed over j: S = d support vectors e_j with
    gamma = 1, per-SV offset folded into the bias is not possible with a
    common coef0, so the centre is 0 unless all c_j are equal.
    """
    c = 0.0 if center is None else float(center)
    sv = np.eye(d)
    return Manifold(d=d, p=2, gamma=1.0, coef0=-c, bias=-R * R,
                    sv=np.ascontiguousarray(sv), alpha=np.ones(d))


def rbf_manifold(d, S, rng, dom: Domain, gamma=None, width=0.6) -> Manifold:
    """RBF-kernel decision function: S support vectors uniform in the box,
    alpha ~ N(0, 1); gamma = 1 / (2 (width * box half-width)^2) unless given,
    so one kernel reaches about `width` of the half-width."""
    sv = rng.uniform(dom.lo, dom.hi, size=(S, d))
    a = rng.standard_normal(S)
    half = float(np.max(dom.hi - dom.lo)) / 2.0
    g = 1.0 / (2.0 * (width * half) ** 2) if gamma is None else gamma
    return Manifold(d=d, p=1, gamma=float(g), coef0=0.0, bias=0.0, sv=np.ascontiguousarray(sv),
                    alpha=np.ascontiguousarray(a), kernel="rbf")


def rbf_sphere_manifold(d: int, R: float, gamma: float = 1.0, center=None) -> Manifold:
    """exp(-gamma |x - c|^2) - exp(-gamma R^2): one support vector, zero set
    the sphere of radius R around c, positive inside."""
    c = np.zeros(d) if center is None else np.asarray(center, float)
    return Manifold(d=d, p=1, gamma=float(gamma), coef0=0.0, bias=-math.exp(-gamma * R * R),
                    sv=np.ascontiguousarray(c[None, :]), alpha=np.ones(1), kernel="rbf")


def closed_quadratic_bias(fm: Manifold, dom: Domain, rng, n_probe=20000) -> float:
    """Bias for a convex quadratic f0 so that {f = 0} is closed inside the box.

    b = -(m_in + m_bd)/2 with m_in the minimum of f0 over the box and m_bd an
    estimate of its minimum over the box boundary; then f > 0 on the boundary
    and f < 0 at the interior minimiser.
    """
    d = fm.d
    # interior minimum of the convex quadratic (clipped to the box)
    Q = (fm.gamma ** 2) * (fm.sv.T * fm.alpha) @ fm.sv
    g = 2 * fm.gamma * fm.coef0 * (fm.sv.T @ fm.alpha)
    xstar = np.clip(np.linalg.solve(2 * Q, -g), dom.lo, dom.hi)
    m_in = float(_f0(fm, xstar[None])[0])
    # boundary minimum: dense random probes on the faces
    X = rng.uniform(dom.lo, dom.hi, size=(n_probe, d))
    face = rng.integers(0, d, n_probe)
    side = rng.integers(0, 2, n_probe)
    X[np.arange(n_probe), face] = np.where(side == 1, dom.hi[face], dom.lo[face])
    m_bd = float(_f0(fm, X).min())
    return -(m_in + m_bd) / 2.0


def quantile_bias(fm: Manifold, dom: Domain, rng, eps: float, n_probe=200000) -> float:
    """Bias so that a fraction eps of the box lies in {f < 0}."""
    X = rng.uniform(dom.lo, dom.hi, size=(n_probe, fm.d))
    return -float(np.quantile(_f0(fm, X), eps))


def bisection_seeds(fm: Manifold, dom: Domain, rng, n_seeds: int,
                    n_probe=20000, iters=60) -> np.ndarray:
    """Points near {f = 0}: bisect segments joining an f<0 and an f>0 probe."""
    negs = []
    pos = None
    drawn = 0
    while drawn < 4_000_000:
        X = rng.uniform(dom.lo, dom.hi, size=(n_probe, fm.d))
        drawn += n_probe
        F = feval_np(fm, X)
        negs.append(X[F < 0])
        if pos is None:
            pos = X[F >= 0]
        if sum(len(a) for a in negs) >= n_seeds:
            break
    neg = np.concatenate(negs)
    if len(neg) == 0 or len(pos) == 0:
        raise ValueError("f has no sign change over the probes")
    seeds = []
    for i in range(n_seeds):
        a = neg[i % len(neg)].copy()
        # the positive probe nearest to a keeps the crossing local
        j = np.argmin(((pos - a) ** 2).sum(1) + 1e-9 * i)
        b = pos[j].copy()
        for _ in range(iters):
            m = 0.5 * (a + b)
            if feval_np(fm, m[None])[0] < 0:
                a = m
            else:
                b = m
        seeds.append(0.5 * (a + b))
    return np.ascontiguousarray(np.array(seeds))


# --------------------------------------------------------------------------
# Scenes (Sec. V-C: robot as spheres; obstacles as spheres / boxes)
# --------------------------------------------------------------------------
def _T(R=None, t=(0.0, 0.0, 0.0)):
    R = np.eye(3) if R is None else np.asarray(R, float)
    out = np.zeros(12)
    out[[0, 1, 2, 4, 5, 6, 8, 9, 10]] = R.reshape(-1)
    out[[3, 7, 11]] = t
    return out


def _random_rotation(rng):
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def planar_arm_scene(rng, n_links=3, link=1.0, n_obst=3, r_obst=0.3) -> Scene:
    """Planar nR arm, unit links along x, z axes; circles as spheres at z=0."""
    joint_T = np.stack([_T() if i == 0 else _T(t=(link, 0, 0)) for i in range(n_links)])
    c = np.zeros((n_obst, 3))
    c[:, :2] = rng.uniform(-3.0, 3.0, size=(n_obst, 2))
    return Scene(
        joint_T=joint_T, joint_axis=np.full(n_links, 2, np.int32),
        lcap_link=np.arange(n_links, dtype=np.int32),
        lcap_p0=np.zeros((n_links, 3)),
        lcap_p1=np.tile([link, 0.0, 0.0], (n_links, 1)),
        lcap_r=np.zeros(n_links),
        osph_c=c, osph_r=np.full(n_obst, r_obst))


_SPATIAL_AXES = [2, 1, 1, 2, 1, 2, 1]


def spatial_arm_scene(rng, n_links, link=0.3, capsule_r=None, spheres_per_link=0,
                      sphere_r=0.05, n_osph=8, osph_r=(0.1, 0.3), n_obox=0,
                      obox_l=(0.1, 0.4), obst_ball=None, n_ocyl=0, ocyl_r=(0.05, 0.2),
                      ocyl_h=(0.2, 0.8)) -> Scene:
    """Spatial nR arm: axes z,y,y,z,y,z,...; links of length `link` along z.

    Obstacle centres are drawn in the reach ball (radii between 0.58 and 1
    times the reach), or, with obst_ball = (centre, radius), uniformly in that
    ball (a cluttered workspace around the arm)."""
    joint_T = np.stack([_T() if i == 0 else _T(t=(0, 0, link)) for i in range(n_links)])
    reach = link * n_links
    sc = Scene(joint_T=joint_T, joint_axis=np.array(_SPATIAL_AXES[:n_links], np.int32))
    if capsule_r is not None:
        sc.lcap_link = np.arange(n_links, dtype=np.int32)
        sc.lcap_p0 = np.zeros((n_links, 3))
        sc.lcap_p1 = np.tile([0.0, 0.0, link], (n_links, 1))
        sc.lcap_r = np.full(n_links, capsule_r)
    if spheres_per_link:
        m = spheres_per_link
        sc.lsph_link = np.repeat(np.arange(n_links, dtype=np.int32), m)
        zs = (np.arange(m) + 0.5) / m * link
        sc.lsph_c = np.tile(np.stack([np.zeros(m), np.zeros(m), zs], 1), (n_links, 1))
        sc.lsph_r = np.full(n_links * m, sphere_r)

    def in_ball(n):
        v = rng.standard_normal((n, 3))
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        if obst_ball is not None:
            return np.asarray(obst_ball[0], float) + v * (obst_ball[1] * rng.uniform(0.0, 1.0, size=(n, 1)) ** (1 / 3))
        return v * (reach * rng.uniform(0.2, 1.0, size=(n, 1)) ** (1 / 3))

    sc.osph_c = in_ball(n_osph)
    sc.osph_r = rng.uniform(osph_r[0], osph_r[1], n_osph)
    if n_obox:
        sc.obox_T = np.stack([_T(_random_rotation(rng), t) for t in in_ball(n_obox)])
        sc.obox_l = rng.uniform(obox_l[0], obox_l[1], size=(n_obox, 3))
    if n_ocyl:
        sc.ocyl_T = np.stack([_T(_random_rotation(rng), t) for t in in_ball(n_ocyl)])
        sc.ocyl_rh = np.stack([rng.uniform(ocyl_r[0], ocyl_r[1], n_ocyl),
                               rng.uniform(ocyl_h[0], ocyl_h[1], n_ocyl)], 1)
    return sc


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------
def sphere_case(d: int, R: float, lam: float, seed: int = 0, half=None, n_seeds=1) -> Workload:
    """f = ||x||^2 - R^2: a single closed component; used by the pins."""
    rng = np.random.default_rng(seed)
    dom = box(d, half if half is not None else R + 4 * lam * d + 0.5)
    fm = sphere_manifold(d, R)
    lat = make_lattice(d, lam, rng)
    u = rng.standard_normal((n_seeds, d))
    seeds = R * u / np.linalg.norm(u, axis=1, keepdims=True)
    return Workload(f"sphere_d{d}", fm, lat, dom, np.ascontiguousarray(seeds))


def quadric_case(d=3, S=50, lam=0.15, seed=0, n_seeds=4, scene=True) -> Workload:
    """Degree-2 kernel, half-normal coefficients: a closed ellipsoid-like set."""
    rng = np.random.default_rng(seed)
    dom = box(d)
    fm = random_manifold(d, S, 2, rng, dom, alpha="halfnormal")
    fm.bias = closed_quadratic_bias(fm, dom, rng)
    lat = make_lattice(d, lam, rng)
    seeds = bisection_seeds(fm, dom, rng, n_seeds)
    sc = planar_arm_scene(rng) if (scene and d == 3) else None
    return Workload(f"quadric_d{d}_S{S}", fm, lat, dom, seeds, 1, sc)


def cubic_case(d, S, lam, eps, seed=0, n_seeds=8, k=1, scene=None) -> Workload:
    """Degree-3 kernel, N(0,1) coefficients, bias at the eps-quantile of f0."""
    rng = np.random.default_rng(seed)
    dom = box(d)
    fm = random_manifold(d, S, 3, rng, dom, alpha="normal")
    fm.bias = quantile_bias(fm, dom, rng, eps)
    lat = make_lattice(d, lam, rng)
    seeds = bisection_seeds(fm, dom, rng, n_seeds)
    return Workload(f"cubic_d{d}_S{S}", fm, lat, dom, seeds, k, scene)


def rbf_sphere_case(d: int, R: float, lam: float, gamma: float = 1.0, seed: int = 0,
                    half=None) -> Workload:
    """The one-support-vector RBF sphere; a closed component for the pins."""
    rng = np.random.default_rng(seed)
    dom = box(d, half if half is not None else R + 4 * lam * d + 0.5)
    fm = rbf_sphere_manifold(d, R, gamma)
    lat = make_lattice(d, lam, rng)
    u = rng.standard_normal((1, d))
    seeds = R * u / np.linalg.norm(u, axis=1, keepdims=True)
    return Workload(f"rbf_sphere_d{d}", fm, lat, dom, np.ascontiguousarray(seeds))


def rbf_case(d, S, lam, eps, seed=0, n_seeds=8, k=1, width=0.6, scene=None) -> Workload:
    """RBF-kernel decision function (the kernel the paper's SVM is trained
    with), S support vectors, bias at the eps-quantile of the kernel sum."""
    rng = np.random.default_rng(seed)
    dom = box(d)
    fm = rbf_manifold(d, S, rng, dom, width=width)
    fm.bias = quantile_bias(fm, dom, rng, eps, n_probe=100000)
    lat = make_lattice(d, lam, rng)
    seeds = bisection_seeds(fm, dom, rng, n_seeds)
    return Workload(f"rbf_d{d}_S{S}", fm, lat, dom, seeds, k, scene)


def config_c1(seed=0) -> Workload:
    """d=3, 50 SVs, degree 2, scale 0.15, planar 3R arm with 3 circles."""
    w = quadric_case(d=3, S=50, lam=0.15, seed=seed, n_seeds=4)
    w.name = "d3_S50_p2_lam0.15_fp64"
    return w


def config_c2(seed=0, eps=0.02) -> Workload:
    """d=5, 500 SVs, degree 3, scale 0.08, 5R arm with capsules vs 8 spheres."""
    rng = np.random.default_rng(seed + 100)
    sc = spatial_arm_scene(rng, 5, capsule_r=0.05, n_osph=8)
    w = cubic_case(5, 500, 0.08, eps, seed=seed, scene=sc)
    w.name = "d5_S500_p3_lam0.08"
    return w


# Scene stream of the d=6 workload: obstacles in a ball of radius 0.9 around
# the shoulder (0, 0, 0.3), where the arm sits folded at the workload's cells.
# The stream number was picked so that the cells' verdicts are mixed (about
# 60 % in collision, estimated with the oracle on cells around each seed by
# tests/golden/make_c3_scene.py, recorded in tests/golden/c3_scene.json).
C3_SCENE_STREAM = 204
C3_OBST_BALL = ((0.0, 0.0, 0.3), 0.9)


def config_c3(seed=0, eps=0.002, k=4) -> Workload:
    """d=6, 2000 SVs, degree 3, scale 0.06, batch k; 6R arm, 8 boxes + 8 spheres."""
    rng = np.random.default_rng(seed + C3_SCENE_STREAM)
    sc = spatial_arm_scene(rng, 6, spheres_per_link=3, sphere_r=0.05,
                           n_osph=8, n_obox=8, obst_ball=C3_OBST_BALL)
    w = cubic_case(6, 2000, 0.06, eps, seed=seed, k=k, scene=sc)
    w.name = f"d6_S2000_p3_lam0.06_k{k}"
    return w


# Kernel offset of the precision stress, bisected so that 5 % of the traced
# cells' vertices have |f| below 1e-6 of the sum of the absolute terms
# (tests/golden/make_c5_calibration.py, recorded in
# tests/golden/c5_calibration.json).
C5_COEF0 = 300.5


def config_c5(seed=0, coef0=C5_COEF0, lam=0.08, eps=3e-4):
    """Precision stress: d=5, 1000 SVs, degree 3, a large kernel offset coef0
    whose constant part coef0^3 sum(alpha) is cancelled by the bias, so that
    sum_i |alpha_i t_i^3| exceeds |f| by about 1e6 near the zero set."""
    rng = np.random.default_rng(seed + 500)
    d = 5
    dom = box(d)
    fm = random_manifold(d, 1000, 3, rng, dom, alpha="normal", coef0=coef0)
    fm.bias = quantile_bias(fm, dom, rng, eps)
    lat = make_lattice(d, lam, rng)
    seeds = bisection_seeds(fm, dom, rng, 8)
    return Workload(f"d5_S1000_p3_lam{lam}_stress", fm, lat, dom, seeds, 1)


def dyadic_sphere_case(d=3, R2=1.0, step=0.125, half=1.6):
    """||x||^2 - R2 on the lattice x = step * v (identity frame): with a
    dyadic step, f is exactly 0.0 at every vertex on the sphere, which
    exercises the sign rule s = !(f < 0) and the FP64 fallback."""
    dom = box(d, half)
    fm = sphere_manifold(d, math.sqrt(R2))
    fm.bias = -R2
    M = np.eye(d) * step
    lat = Lattice(M=M, Minv=np.eye(d) / step, o=np.zeros(d), lam=step)
    u = np.ones(d) / np.sqrt(d)
    seeds = np.ascontiguousarray((math.sqrt(R2) * u)[None, :])
    return Workload(f"dyadic_sphere_d{d}", fm, lat, dom, seeds)


# --------------------------------------------------------------------------
# Serving requests: the same manifold family, each request restricted to a
# sub-box of C-space sized for a target number of cells
# --------------------------------------------------------------------------
def _edge_density(d):
    """Asymptotic crossing-edge density of the Coxeter frame, edges per unit
    area at unit scale (used only to size inputs)."""
    kappa = math.gamma(d / 2) / (math.sqrt(math.pi) * math.gamma((d + 1) / 2))
    s = sum(math.comb(d, r) * math.sqrt(r * (d + 1 - r) / (d + 1)) for r in range(1, d + 1))
    return kappa * math.sqrt(d + 1) * s


def subbox_case(d, S, lam, target_cells, seed=0, p=3, eps=3e-3, k=1, scene=None):
    """Degree-p kernel, N(0,1) coefficients, bias at the eps-quantile of f0;
    the domain is the sub-box around the first seed whose half-width w makes
    a locally flat zero set cross about target_cells edges:
    N ~ C_d (2w)^(d-1) / lam^(d-1)."""
    rng = np.random.default_rng(seed)
    full = box(d)
    fm = random_manifold(d, S, p, rng, full, alpha="normal")
    fm.bias = quantile_bias(fm, full, rng, eps, n_probe=4000)
    seeds = bisection_seeds(fm, full, rng, 1, n_probe=4000, iters=40)
    w = 0.5 * (target_cells * lam ** (d - 1) / _edge_density(d)) ** (1.0 / (d - 1))
    c = seeds[0]
    dom = Domain(lo=np.maximum(full.lo, c - w), hi=np.minimum(full.hi, c + w))
    lat = make_lattice(d, lam, rng)
    return Workload(f"subbox_d{d}_S{S}_lam{lam:.3f}", fm, lat, dom, seeds, k, scene)


def _poly_grad_hess(fm: Manifold, x):
    t = fm.gamma * (fm.sv @ x) + fm.coef0
    g = (fm.alpha * fm.p * fm.gamma * t ** (fm.p - 1)) @ fm.sv
    w = fm.alpha * fm.p * (fm.p - 1) * fm.gamma ** 2 * t ** (fm.p - 2)
    H = (fm.sv.T * w) @ fm.sv
    return g, H


def planted_minimum(fm: Manifold, dom: Domain, rng, tries=50):
    """Rewrites the coefficients of a polynomial-kernel f0 so that it has a
    strict local minimum at a random point x0 of the inner half of the box (a
    random cubic kernel sum usually has none inside the box).  Each
    coefficient keeps its magnitude and takes the sign of t^(p-2), t the
    kernel argument at x0, so every term's Hessian is positive semidefinite
    there; then the smallest correction weighted by alpha_i^2 makes
    grad f0(x0) = 0 (a d x d solve).  Draws x0 again until the Hessian is
    clearly positive definite.  Returns x0 and the Hessian there (input
    generation only)."""
    p, g = fm.p, fm.gamma
    mag = np.abs(fm.alpha).copy()
    for _ in range(tries):
        x0 = rng.uniform(dom.lo * 0.5, dom.hi * 0.5)
        t = g * (fm.sv @ x0) + fm.coef0
        a = mag * np.sign(t) ** (p - 2)
        B = (fm.sv * (p * g * t ** (p - 1))[:, None]).T     # grad f0(x0) = B a
        W = a * a
        try:
            lam = np.linalg.solve((B * W) @ B.T, B @ a)
        except np.linalg.LinAlgError:
            continue
        a = a - W * (B.T @ lam)
        fm.alpha = np.ascontiguousarray(a)
        gr, H = _poly_grad_hess(fm, x0)
        ev = np.linalg.eigvalsh(H)
        if ev[0] > 1e-3 * ev[-1] and np.linalg.norm(gr) <= 1e-9 * np.abs(H).max():
            return x0, H
    raise RuntimeError("no interior minimum could be planted")


def planted_blob(fm: Manifold, dom: Domain, rng, area, n_dirs=20000, n_rays=2000, tries=4):
    """Bias and centre that make {f < 0} a small blob of about the given
    boundary area around a planted minimum x0 of the kernel sum f0.  Near x0
    the blob {f0 < f0(x0) + delta} is the ellipsoid with semi-axes
    a_i = sqrt(2 delta / lambda_i) (lambda_i the Hessian's eigenvalues); its
    area is prod(a) times the mean over unit vectors u of sqrt(sum u_i^2 /
    a_i^2) times the unit sphere's area, which fixes delta.  delta is then
    halved until, along random rays u, h(s) = f0(x0 + s rho(u) u) - f0(x0) -
    delta (rho(u) the ellipsoid's radius along u) stays below
    -delta (1 - s^2) / 4 out to s = 0.8 and above delta (s^2 - 1) / 4 from
    s = 1.2 to 3, inside the box: the boundary then lies within 0.8 and 1.2
    of the ellipsoid on every ray and the blob is the whole traced component.
    If delta falls below 2^-30 of its first value x0 is planted anew (input
    sizing only)."""
    d = fm.d
    sphere_area = 2 * math.pi ** (d / 2) / math.gamma(d / 2)
    s = np.concatenate([np.linspace(0.2, 0.8, 7), np.linspace(1.2, 3.0, 19)])
    env = 0.25 * (s * s - 1.0)
    for _ in range(tries):
        x0, H = planted_minimum(fm, dom, rng)
        lam_i = np.linalg.eigvalsh(H)
        a1 = lam_i ** -0.5                       # semi-axes at 2 delta = 1
        u = rng.standard_normal((n_dirs, d))
        u /= np.linalg.norm(u, axis=1, keepdims=True)
        area1 = float(np.prod(a1) * np.mean(np.sqrt((u ** 2 / a1 ** 2).sum(1))) * sphere_area)
        two_delta0 = two_delta = (area / area1) ** (2.0 / (d - 1))
        f00 = float(_f0(fm, x0[None])[0])
        ur = u[:n_rays]
        uHu = np.einsum("ri,ij,rj->r", ur, H, ur)
        while two_delta > two_delta0 * 2.0 ** -30:
            rho = np.sqrt(two_delta / uHu)
            P = x0[None, None, :] + (s[None, :, None] * rho[:, None, None]) * ur[:, None, :]
            if ((P >= dom.lo) & (P <= dom.hi)).all():
                delta = 0.5 * two_delta
                h = _f0(fm, P.reshape(-1, d)).reshape(len(ur), len(s)) - f00 - delta
                inner = s < 1.0
                if (h[:, inner] <= delta * env[inner]).all() and (h[:, ~inner] >= delta * env[~inner]).all():
                    return -(f00 + delta), x0
            two_delta *= 0.5
    raise RuntimeError("planted blob does not separate from the rest of {f < 0}")


def fullbox_case(d, S, lam, target_cells, seed=0, p=3, k=1, scene=None, n_seeds=4, coef0=1.0) -> Workload:
    """Degree-p kernel over the whole box [-pi, pi]^d, coefficient
    magnitudes |N(0,1)| with the signs (and a small correction) that plant an
    interior minimum (planted_minimum), and {f < 0} a blob around it whose
    boundary crosses about target_cells edges at scale lam: area
    A = target lam^(d-1) / C_d (planted_blob).
    Seeds: bisection from the blob's centre outwards along random
    directions."""
    rng = np.random.default_rng(seed)
    dom = box(d)
    fm = random_manifold(d, S, p, rng, dom, alpha="normal", coef0=coef0)
    A = target_cells * lam ** (d - 1) / _edge_density(d)
    fm.bias, xc = planted_blob(fm, dom, rng, A)
    # a length on the blob's scale for the seed rays
    r = (A / (2 * math.pi ** (d / 2) / math.gamma(d / 2))) ** (1.0 / (d - 1))
    seeds = []
    for _ in range(n_seeds):
        u = rng.standard_normal(d)
        u /= np.linalg.norm(u)
        a, step = xc.copy(), 2 * r
        b = np.clip(xc + step * u, dom.lo, dom.hi)
        while feval_np(fm, b[None])[0] < 0 and step < 20.0:
            step *= 2
            b = np.clip(xc + step * u, dom.lo, dom.hi)
        for _ in range(60):
            m = 0.5 * (a + b)
            if feval_np(fm, m[None])[0] < 0:
                a = m
            else:
                b = m
        seeds.append(0.5 * (a + b))
    lat = make_lattice(d, lam, rng)
    return Workload(f"fullbox_d{d}_S{S}_lam{lam:.3f}", fm, lat, dom, np.ascontiguousarray(seeds), k, scene)


def serving_request(i, seed=0, cells=(1e5, 2e6)):
    """Proof request i of the serving workload: d in {4,5,6}, S log-uniform
    in [100, 2000], scale uniform in [0.06, 0.12], degree 3 with coef0 3 (the
    cubic terms then bend a planted basin less, so it holds larger blobs),
    over the whole box, the bias sized for a target cell count log-uniform in
    `cells` (smaller where the basin cannot hold that blob), its own scene
    and seed 1000 + i; coarse factor k = 2 for d = 6 below scale 0.09, else
    direct."""
    rng = np.random.default_rng((seed, i))
    d = int(rng.integers(4, 7))
    S = int(round(math.exp(rng.uniform(math.log(100), math.log(2000)))))
    lam = float(rng.uniform(0.06, 0.12))
    target = float(math.exp(rng.uniform(math.log(cells[0]), math.log(cells[1]))))
    k = 2 if (d == 6 and lam < 0.09) else 1
    srng = np.random.default_rng(1000 + i)
    sc = spatial_arm_scene(srng, d, spheres_per_link=2, sphere_r=0.05, n_osph=6, n_obox=4,
                           obst_ball=((0.0, 0.0, 0.3), 0.9))
    return fullbox_case(d, S, lam, target, seed=1000 + i, k=k, scene=sc, coef0=3.0)


def serving_requests(n=256, seed=0, cells=(1e5, 2e6)):
    return [serving_request(i, seed, cells) for i in range(n)]
