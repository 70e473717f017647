"""Pins of the oracle's joint rotations, link-sphere collision path and
closed-box clipping against facts that do not come from the oracle's own
formulas.

* Joint rotations (Sec. V-C: the robot's forward kinematics) are checked
  against Rodrigues' rotation formula built from numpy cross products, so a
  matrix typed with a wrong sign or a transposed entry fails; the hand poses
  of the spatial arm come from the geometry of a quarter turn.
* The link-sphere loop of the check (robot spheres against obstacle spheres
  and boxes, Appendix A) gets hand cases whose verdict follows from distances
  read off the pose.
* The domain box is closed (both ends of a traced edge lie in [lo, hi]); a
  lattice with vertices exactly on lo and hi shows which reading the oracle
  takes, with the box test done here in numpy.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2406_04795_amd import inputs as I


@pytest.fixture(scope="module", autouse=True)
def _built():
    O.build(force=False)


def _rodrigues(axis, q):
    """Rotation by angle q about the unit vector `axis`, right-handed, from
    v cos q + (a x v) sin q + a (a.v)(1 - cos q) applied to the basis."""
    a = np.asarray(axis, float)
    cols = []
    for v in np.eye(3):
        cols.append(v * math.cos(q) + np.cross(a, v) * math.sin(q) + a * (a @ v) * (1 - math.cos(q)))
    return np.stack(cols, 1)


def _chain(scene, q):
    """World pose of every link frame: the parent-to-joint transforms then a
    Rodrigues rotation about the joint's axis (Sec. V-C serial chain)."""
    R = np.eye(3)
    p = np.zeros(3)
    out = []
    for i in range(len(q)):
        J = np.asarray(scene.joint_T[i]).reshape(3, 4)
        p = p + R @ J[:, 3]
        R = R @ J[:, :3]
        R = R @ _rodrigues(np.eye(3)[scene.joint_axis[i]], q[i])
        out.append((R.copy(), p.copy()))
    return out


def _one_joint(axis):
    return I.Scene(joint_T=np.stack([I._T()]), joint_axis=np.array([axis], np.int32))


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_quarter_turn_maps_v_to_axis_cross_v(axis):
    """A right-handed quarter turn about a takes every v perpendicular to a
    to a x v, and a half turn takes it to -v.  Catches a flipped sign of sin
    (a left-handed turn) or a transposed rotation block for that axis."""
    sc = _one_joint(axis)
    a = np.eye(3)[axis]
    for q, want in ((math.pi / 2, lambda v: np.cross(a, v)), (math.pi, lambda v: -v),
                    (-math.pi / 2, lambda v: -np.cross(a, v))):
        T = O.fk(sc, [q])[0].reshape(3, 4)
        for v in np.eye(3):
            if v @ a != 0:
                continue
            assert np.allclose(T[:, :3] @ v, want(v), atol=1e-15)
        assert np.allclose(T[:, :3] @ a, a, atol=1e-15)
        assert np.allclose(T[:, 3], 0.0)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_rotation_matches_rodrigues_at_random_angles(axis):
    """Every angle, not only quarter turns: the oracle's rotation equals
    Rodrigues' formula (own sine/cosine within 1e-15).  Catches a swapped
    sin/cos pair or an entry on the wrong side of the diagonal."""
    sc = _one_joint(axis)
    for q in np.random.default_rng(axis).uniform(-math.pi, math.pi, 200):
        T = O.fk(sc, [q])[0].reshape(3, 4)
        assert np.allclose(T[:, :3], _rodrigues(np.eye(3)[axis], q), atol=2e-15)


def test_spatial_arm_hand_poses():
    """The 6R arm (axes z, y, y, z, y, z; links of 0.3 along z): straight up
    at q = 0, and turned onto +x by a quarter turn of joint 1 about y (a
    right-handed turn about y takes +z to +x).  Catches a left-handed y
    rotation, which would fold the arm onto -x."""
    sc = I.spatial_arm_scene(np.random.default_rng(0), 6, spheres_per_link=3)
    T = O.fk(sc, np.zeros(6))
    assert np.allclose(T[:, [3, 7, 11]], [[0, 0, 0.3 * i] for i in range(6)], atol=1e-15)
    T = O.fk(sc, [0, math.pi / 2, 0, 0, 0, 0])
    want = [[0, 0, 0], [0, 0, 0.3]] + [[0.3 * i, 0, 0.3] for i in range(1, 5)]
    assert np.allclose(T[:, [3, 7, 11]], want, atol=1e-15)
    # a second quarter turn about y, at joint 4 (frame origin (0.9, 0, 0.3)),
    # turns the last link from +x to -z: frame 5 sits 0.3 below frame 4
    T = O.fk(sc, [0, math.pi / 2, 0, 0, math.pi / 2, 0])
    assert np.allclose(T[5, [3, 7, 11]], [0.9, 0, 0.0], atol=1e-15)
    assert np.allclose(T[5].reshape(3, 4)[:, 2], [0, 0, -1], atol=1e-15)


def test_spatial_chains_match_rodrigues_chain():
    """Random poses of the 6R arm and of a chain that turns about x: every
    link frame equals the Rodrigues chain.  Catches a composition in the wrong
    order (rotation before the joint offset) or a wrong axis table."""
    rng = np.random.default_rng(3)
    arm = I.spatial_arm_scene(np.random.default_rng(1), 6, spheres_per_link=3)
    xarm = I.Scene(joint_T=np.stack([I._T(I._random_rotation(rng), rng.uniform(-0.5, 0.5, 3))
                                     for _ in range(5)]),
                   joint_axis=np.array([0, 1, 0, 2, 0], np.int32))
    for sc in (arm, xarm):
        n = len(sc.joint_axis)
        for q in rng.uniform(-math.pi, math.pi, (50, n)):
            T = O.fk(sc, q)
            for i, (R, p) in enumerate(_chain(sc, q)):
                Ti = T[i].reshape(3, 4)
                assert np.allclose(Ti[:, :3], R, atol=1e-13) and np.allclose(Ti[:, 3], p, atol=1e-13)


def _arm_with(osph=None, obox=None):
    sc = I.spatial_arm_scene(np.random.default_rng(0), 6, spheres_per_link=3, sphere_r=0.05, n_osph=0)
    sc.osph_c = np.zeros((0, 3))
    sc.osph_r = np.zeros(0)
    if osph is not None:
        sc.osph_c = np.array([osph[0]], float)
        sc.osph_r = np.array([osph[1]], float)
    if obox is not None:
        sc.obox_T = np.stack([obox[0]])
        sc.obox_l = np.array([obox[1]], float)
    return sc


def test_link_spheres_against_an_obstacle_sphere():
    """Link spheres (r = 0.05) of the 6R arm against one obstacle sphere at
    distance 0.2 from the nearest link-sphere centre: radius 0.16 reaches
    (0.2 <= 0.21), radius 0.14 does not.  At q = 0 the spheres sit on the z
    axis (link 3's middle sphere at z = 1.05); after the quarter turn of joint
    1 they sit on the line z = 0.3 along +x.  Catches a sphere placed in the
    wrong link frame (its frame's translation skipped) and a left-handed turn."""
    q0 = np.zeros(6)
    q1 = np.array([0, math.pi / 2, 0, 0, 0, 0])
    for r, hit in ((0.16, 1), (0.14, 0)):
        assert O.check(_arm_with(osph=([0.2, 0.0, 1.05], r)), [q0])[0] == hit
        assert O.check(_arm_with(osph=([1.05, 0.0, 0.5], r)), [q1])[0] == hit
        # mirrored to -x: free for a right-handed turn whatever the radius
        assert O.check(_arm_with(osph=([-1.05, 0.0, 0.5], r)), [q1])[0] == 0


def test_link_spheres_against_an_obstacle_box():
    """Link spheres against a box whose nearest face is 0.03 (collides) or
    0.07 (free) away from the nearest sphere centre, axis-aligned and turned
    by a quarter turn about z (the same box).  Catches a box pose applied
    without its inverse (world to box frame) and the sphere-box vertex or
    face region taken for the wrong sphere."""
    q1 = np.array([0, math.pi / 2, 0, 0, 0, 0])
    rz = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    for face_gap, hit in ((0.03, 1), (0.07, 0)):
        # box centred above the sphere at (1.05, 0, 0.3): the face is at 0.3 + gap
        hz = 0.2
        c = [1.05, 0.0, 0.3 + face_gap + hz]
        for R in (np.eye(3), rz):
            T = I._T(R, c)
            ext = [0.2, 0.2, 2 * hz]
            assert O.check(_arm_with(obox=(T, ext)), [q1])[0] == hit
        # the same box at q = 0 is far from the upright arm
        assert O.check(_arm_with(obox=(I._T(None, c), [0.2, 0.2, 2 * hz])), [np.zeros(6)])[0] == 0


def _numpy_sphere_edges(step, half, R, d=3):
    """Every intersecting edge of the dyadic lattice x = step v in the closed
    box [-half, half]^d for f = |x|^2 - R^2 (exact dyadic squares), with the
    sign rule s = !(f < 0)."""
    n = int(round(half / step))
    rng = np.arange(-n, n + 1)
    V = np.stack(np.meshgrid(*([rng] * d), indexing="ij"), -1).reshape(-1, d)
    out = set()
    for mask in range(1, 1 << d):
        b = V + np.array([(mask >> j) & 1 for j in range(d)])
        xa, xb = V * step, b * step
        ina = ((xa >= -half) & (xa <= half)).all(1)
        inb = ((xb >= -half) & (xb <= half)).all(1)
        fa = (xa ** 2).sum(1) - R * R
        fb = (xb ** 2).sum(1) - R * R
        hit = ina & inb & ((fa < 0) != (fb < 0))
        for v in V[hit]:
            out.add((tuple(int(t) for t in v), mask))
    return out


def test_closed_box_keeps_edges_ending_exactly_on_lo_and_hi():
    """A sphere of radius 1.45 in the box [-1.5, 1.5]^3 on the lattice
    x = v / 8: the crossing edges near the faces have one end exactly on
    x_j = +-1.5.  The closed box keeps them, in the brute force and in the
    trace, and the set equals the one numpy enumerates with a closed box
    test.  Catches an open box (< instead of <=) on either side, which the
    trace == brute-force pin alone cannot see since both share one test."""
    step, half, R = 0.125, 1.5, 1.45
    wl = I.dyadic_sphere_case(d=3, R2=R * R, step=step, half=half)
    want = _numpy_sphere_edges(step, half, R)
    v, m = O.brute(wl)
    got = {(tuple(int(t) for t in v[i]), int(m[i])) for i in range(len(v))}
    assert got == want
    tv, tm = O.trace_direct(wl)
    traced = {(tuple(int(t) for t in tv[i]), int(tm[i])) for i in range(len(tv))}
    assert traced == want
    n_side = int(round(half / step))
    on_boundary = [e for e in want
                   if any(abs(c) == n_side for c in e[0]) or
                   any(abs(e[0][j] + ((e[1] >> j) & 1)) == n_side for j in range(3))]
    # an open box would drop exactly these
    assert len(on_boundary) >= 24


# --------------------------------------------------------------------------
# Sphere vs cylinder (Appendix A)
# --------------------------------------------------------------------------
def _cyl_dist2(c, T, rc, h):
    """Squared distance from c to the solid cylinder: radial and axial
    clamps in the cylinder frame (the textbook closest point)."""
    Tm = np.asarray(T).reshape(3, 4)
    p = Tm[:, :3].T @ (np.asarray(c, float) - Tm[:, 3])
    rho = math.hypot(p[0], p[1])
    return max(rho - rc, 0.0) ** 2 + max(abs(p[2]) - h / 2, 0.0) ** 2


def test_sphere_cylinder_matches_clamp_distance():
    """Random poses, sizes and centres, away from exact contact.  Catches a
    missing fold into the first octant (the far half of the cylinder), the
    padded test with the wrong radius sum, and the ring region taken for the
    flat face or the side (their distances differ there)."""
    rng = np.random.default_rng(12)
    checked = 0
    for _ in range(6000):
        T = I._T(I._random_rotation(rng), rng.uniform(-1, 1, 3))
        rc, h = rng.uniform(0.05, 0.8), rng.uniform(0.1, 1.5)
        c = rng.uniform(-2, 2, 3)
        r = rng.uniform(0.01, 0.7)
        d2 = _cyl_dist2(c, T, rc, h)
        if abs(d2 - r * r) < 1e-9:
            continue
        assert O.sphere_cylinder(c, r, T, rc, h) == (d2 <= r * r)
        checked += 1
    assert checked > 5900


def test_sphere_cylinder_exact_contacts():
    """Touching collides (Appendix A: no collision only beyond the radius),
    on each region, with dyadic sizes so the contacts are exact: flat face,
    curved side, and the rim (ring region) at the 3-4-5 distance 1.25."""
    T = I._T()
    rc, h = 1.0, 2.0
    # flat face z = 1
    assert O.sphere_cylinder([0.25, 0.0, 1.5], 0.5, T, rc, h) == 1
    assert O.sphere_cylinder([0.25, 0.0, 1.5], 0.4375, T, rc, h) == 0
    # curved side rho = 1
    assert O.sphere_cylinder([1.5, 0.0, 0.25], 0.5, T, rc, h) == 1
    assert O.sphere_cylinder([0.0, -1.5, 0.25], 0.4375, T, rc, h) == 0
    # rim: rho - rc = 0.75, z - h/2 = 1, distance 1.25
    assert O.sphere_cylinder([1.75, 0.0, 2.0], 1.25, T, rc, h) == 1
    assert O.sphere_cylinder([0.0, 1.75, -2.0], 1.25, T, rc, h) == 1
    assert O.sphere_cylinder([1.75, 0.0, 2.0], 1.1875, T, rc, h) == 0
    # inside
    assert O.sphere_cylinder([0.1, 0.2, 0.3], 0.01, T, rc, h) == 1


def test_link_spheres_against_an_obstacle_cylinder():
    """The 6R arm turned onto +x (joint 1 a quarter turn about y): a vertical
    cylinder whose side is 0.03 (collides) or 0.07 (free) from the link
    sphere at (1.05, 0, 0.3) (r = 0.05); a mirrored one on -x stays free."""
    q1 = np.array([0, math.pi / 2, 0, 0, 0, 0])
    for gap, hit in ((0.03, 1), (0.07, 0)):
        rc = 0.1
        sc = _arm_with()
        # beside the sphere at (1.05, 0, 0.3), along +y
        sc.ocyl_T = np.stack([I._T(None, (1.05, gap + rc, 0.3))])
        sc.ocyl_rh = np.array([[rc, 0.4]])
        assert O.check(sc, [q1])[0] == hit
        sc.ocyl_T = np.stack([I._T(None, (-1.05, gap + rc, 0.3))])
        assert O.check(sc, [q1])[0] == 0
