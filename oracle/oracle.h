/*
 * Reference (oracle) implementation of manifold tracing through the
 * Coxeter triangulation and of the batch collision check, after Li & Dantam,
 * "Scaling Motion Planning Infeasibility Proofs" (arXiv 2406.04795).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists so that the GPU library can
 * be checked against a plain, slow, obviously correct computation.  Only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load it.  It shares no code with the GPU library.
 *
 * Conventions (all FP64, compiled with -ffp-contract=off; fma() only where
 * written):
 *   - lattice: x(v) = o + M v for integer v (Sec. IV-B; M is an input);
 *   - roots e_j = unit vector j for j < d, e_d = -(1,...,1);
 *   - simplex = (vertex, ordered partition of {0..d}); canonical form puts d
 *     in the last part, so the vertex is the lexicographic minimum (Fig. 2);
 *   - sign bit s(v) = !(f(x(v)) < 0);
 *   - an edge intersects the manifold when both endpoints lie in the closed
 *     domain box and their sign bits differ (Sec. V-A, reading of the strict
 *     product rule as a sign-bit rule).
 *
 * Error behaviour: functions return 0 on success and a negative value on bad
 * arguments or allocation failure.  Output arrays allocated by the oracle are
 * released with orc_free().
 */
#ifndef ORACLE_H
#define ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAXD 8

/* Decision function of a kernel SVM (Sec. IV-A; the experiments train an
 * RBF-kernel SVM):
 *   ORC_POLY: f(x) = sum_i alpha_i (gamma <s_i, x> + coef0)^p + bias,
 *   ORC_RBF:  f(x) = sum_i alpha_i exp(-gamma |x - s_i|^2) + bias. */
#define ORC_POLY 0
#define ORC_RBF 1
typedef struct {
  int32_t d;            /* ambient dimension, 2..7 */
  int32_t p;            /* polynomial kernel degree >= 1 (ORC_POLY) */
  int64_t S;            /* number of support vectors */
  double gamma, coef0, bias;
  const double *sv;     /* S x d, row-major */
  const double *alpha;  /* S */
  int32_t kernel;       /* ORC_POLY or ORC_RBF */
} orc_fparams;

typedef struct {
  int32_t d;
  const double *M;      /* d x d row-major: x_j = o_j + sum_k M[j][k] v_k */
  const double *Minv;   /* d x d row-major */
  const double *o;      /* d */
  const double *lo;     /* d, closed domain box */
  const double *hi;     /* d */
} orc_space;

/* A set of canonical edges (v, R): endpoints v and v + 1_R, R != 0. */
typedef struct {
  int64_t n;
  int32_t d;
  int32_t *v;           /* n x d */
  uint32_t *mask;       /* n */
} orc_edges;

/* Own exponential for the RBF kernel: Cody-Waite reduction by ln 2 with a
 * two-part constant (t = k ln2 + r, |r| <= ln2 / 2), the Taylor polynomial
 * of exp(r) to degree 13 in Horner form (coefficients 1/n!), then the exact
 * scaling by 2^k.  0 below t = -708 (under the normal range). */
double orc_exp(double t);

/* Canonical coordinates and f (Sec. III / IV-A: the learned manifold). */
void   orc_coords(const orc_space *sp, const int32_t *v, double *x);
double orc_f(const orc_fparams *f, const double *x);
void   orc_f_batch(const orc_fparams *f, const orc_space *sp, int64_t n,
                   const int32_t *v, double *out);

/* Point location (Sec. V-A query 1): y -> n-simplex (v, w), w a permutation
 * of {0..d-1}; vertices v, v+e_{w0}, v+e_{w0}+e_{w1}, ...  coarse_k >= 1
 * divides lattice coordinates (locating in the lattice refined by k). */
void   orc_locate(const orc_space *sp, int32_t coarse_k, const double *y,
                  int32_t *v, int32_t *w);

/* Combinatorial queries on the permutahedral representation, used by the
 * pins: 2-cofaces of an edge (Sec. V-A query 3) and n-cofaces of an edge
 * (Sec. V-B).  Outputs are written into caller arrays of sufficient size;
 * return value is the count.
 *   cof2: for each coface the 3 vertices (3*d ints);
 *   ncof: for each coface its canonical (v (d ints), w (d ints)). */
int64_t orc_cofaces2(int32_t d, const int32_t *v, uint32_t mask, int32_t *tri);
int64_t orc_ncofaces(int32_t d, const int32_t *v, uint32_t mask, int32_t *out);

/* Vertices of the canonical simplex given a starting vertex and a cyclic
 * ordered partition (parts as bitmasks over {0..d}).  Writes the canonical
 * vertex and the rotated parts.  Returns the number of parts. */
int32_t orc_canonical(int32_t d, const int32_t *v, int32_t nparts,
                      const uint32_t *parts, int32_t *vc, uint32_t *pc);

/* f and its gradient at x in the canonical order: per support vector in
 * index order, POLY: dot and t as in orc_f, t^(p-1) by repeated
 * multiplication (1 for p = 1), t^p = t^(p-1) t, acc = fma(alpha, t^p, acc),
 * w = (alpha t^(p-1)) (p gamma), g_j = fma(w, s_j, g_j); RBF: d_j = x_j - s_j,
 * d2 and e as in orc_f, acc = fma(alpha, e, acc), w = (alpha e) (-2 gamma),
 * g_j = fma(w, d_j, g_j).  Returns f = acc + bias. */
double orc_f_grad(const orc_fparams *f, const double *x, double *g);

/* Seeds by minimising |f| from given configurations (Sec. V-A: the seeds are
 * points on the manifold found by a nonlinear program that minimises the
 * absolute value of f from a configuration): `iters` minimum-norm Newton
 * steps q <- q - (f / |grad f|^2) grad f (n2 = fma chain of g_j^2, c = f / n2,
 * q_j = fma(-c, g_j, q_j)), each followed by clamping q into the domain box;
 * a zero gradient ends the steps.  Writes the final q (n x d) and f(q). */
int orc_seed_search(const orc_fparams *f, const orc_space *sp, int64_t n,
                    const double *q0, int32_t iters, double *q, double *fq);

/* Direct trace (Sec. V-A, Figs. 3-4): the closure of the seeds' intersecting
 * edges under "shares a 2-simplex".  Output sorted lexicographically by
 * (v, mask).  coarse_k >= 1 traces the lattice refined by k: vertex u of the
 * coarse lattice has coordinates x(k u).  Returns 0 or < 0 on error. */
int orc_trace_direct(const orc_fparams *f, const orc_space *sp,
                     int32_t coarse_k, const double *seeds, int64_t n_seeds,
                     orc_edges *out);

/* Batch trace (Sec. V-B, Figs. 5-6): coarse trace at k, n-cofaces of the
 * coarse edges, symmetric subdivision of each into k^d fine simplices, all
 * fine intersecting edges inside (Eq. 2 read as >=).  Global set output. */
int orc_trace_batch(const orc_fparams *f, const orc_space *sp, int32_t k,
                    const double *seeds, int64_t n_seeds, orc_edges *out,
                    int64_t *n_sigma);

/* The coarse n-simplices of the batch trace: sorted (v, w) rows of 2d ints. */
int orc_batch_sigma(const orc_fparams *f, const orc_space *sp, int32_t k,
                    const double *seeds, int64_t n_seeds, int64_t *n,
                    int32_t **sigma);

/* Brute force: every intersecting edge with both endpoints in the box. */
int orc_brute(const orc_fparams *f, const orc_space *sp, orc_edges *out);

/* Local subdivision template (Sec. V-B, Eq. 2): points u with
 * k >= u_0 >= ... >= u_{d-1} >= 0, and edges (u, R) with u + 1_R inside.
 * If pts/edges are NULL only the counts are returned. */
int orc_template(int32_t d, int32_t k, int64_t *n_pts, int32_t *pts,
                 int64_t *n_edges, int32_t *edge_u, uint32_t *edge_r);

/* Intersection points (Sec. V-B): t = f_a/(f_a - f_b), p = x_a + t(x_b-x_a)
 * with a the minimum endpoint.  Also writes t. */
int orc_points(const orc_fparams *f, const orc_space *sp, int64_t n,
               const int32_t *v, const uint32_t *mask, double *pts, double *t);

/* Intersection points computed iteratively (Sec. V-B; Sec. VI: the point
 * is refined until a desired accuracy).  The edge (a, b), a the smaller
 * endpoint, brackets the crossing: s(a) != s(b).  Each iteration is a false
 * position step with the Illinois modification (Dowell & Jarratt 1971):
 * t = f_a / (f_a - f_b), m_j = fma(t, x_b,j - x_a,j, x_a,j), f_m = f(m) in the
 * canonical order; the end whose sign bit equals s(m) = !(f_m < 0) moves to
 * m, and when the same end moves twice in a row the value kept at the other
 * end is halved.  After `iters` iterations the point is the false position
 * point of the final bracket; iters = 0 gives orc_points. */
int orc_points_refined(const orc_fparams *f, const orc_space *sp, int64_t n,
                       const int32_t *v, const uint32_t *mask, int32_t iters,
                       double *pts);

/* Collision scene (Sec. V-C and Appendix A).  Robot: d revolute joints,
 * T_i = T_{i-1} * J_i * Rot(axis_i, q_i), T_{-1} = I.  Geometry in link
 * frames; obstacles in the world frame.  3x4 transforms are row-major
 * [R | t]. */
typedef struct {
  int32_t n_joints;
  const double *joint_T;     /* n_joints x 12 */
  const int32_t *joint_axis; /* n_joints, 0=x 1=y 2=z */
  int32_t n_lsph;            /* robot spheres */
  const int32_t *lsph_link;
  const double *lsph_c;      /* x3 */
  const double *lsph_r;
  int32_t n_lcap;            /* robot capsules (segments with radius) */
  const int32_t *lcap_link;
  const double *lcap_p0;     /* x3 */
  const double *lcap_p1;     /* x3 */
  const double *lcap_r;
  int32_t n_osph;            /* obstacle spheres */
  const double *osph_c;
  const double *osph_r;
  int32_t n_obox;            /* obstacle boxes */
  const double *obox_T;      /* x12, world-from-box pose */
  const double *obox_l;      /* x3 full extents */
  int32_t n_ocyl;            /* obstacle cylinders */
  const double *ocyl_T;      /* x12, world-from-cylinder pose (axis = z) */
  const double *ocyl_rh;     /* x2: radius, height */
} orc_scene;

/* Own sine/cosine: Cody-Waite reduction by pi/2, Taylor polynomials. */
void orc_sincos(double q, double *s, double *c);
/* Appendix A predicates; 1 = collision (touching counts). */
int  orc_sphere_sphere(const double *a, double ra, const double *b, double rb);
int  orc_capsule_sphere(const double *p0, const double *p1, double rc,
                        const double *c, double rs);
int  orc_sphere_box(const double *c, double r, const double *T, const double *l);
/* Sphere vs solid cylinder of radius rc and height h (Appendix A, sphere vs
 * cylinder), the square roots of its distance tests squared away. */
int  orc_sphere_cylinder(const double *c, double r, const double *T, double rc, double h);
/* Forward kinematics: world transform of every link (n_joints x 12). */
void orc_fk(const orc_scene *sc, const double *q, double *T_out);
/* Verdicts for n configurations q (n x n_joints). */
int  orc_check(const orc_scene *sc, int64_t n, const double *q, uint8_t *verdict);

void orc_free(void *p);

#ifdef __cplusplus
}
#endif
#endif
