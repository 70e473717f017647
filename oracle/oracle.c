/*
 * Oracle: plain FP64 reference for manifold tracing through the Coxeter
 * triangulation (Li & Dantam, arXiv 2406.04795, Sec. IV-B, V-A, V-B) and
 * for the batch collision check (Sec. V-C, Appendix A).
 *
 * TEST INFRASTRUCTURE ONLY -- see oracle.h.  Written for clarity, not speed:
 * plain growable hash maps keyed on integer coordinate tuples, a worklist for
 * the closure, and the definitions written out step by step.  Build with
 * -ffp-contract=off so that only the fma() calls written here are fused.
 *
 * Parity status per function (the pins live in the test suite):
 *   orc_coords, orc_f            pinned (closed forms, sphere level set;
 *                                RBF: numpy value, one-SV sphere level set)
 *   orc_f_grad                   pinned (central differences of orc_f)
 *   orc_seed_search              pinned (sphere: the radial projection;
 *                                affine f: the orthogonal projection in one
 *                                step; clamping into the box)
 *   orc_exp                      pinned (library exp within 2 ulp, exact at 0,
 *                                0 below the normal range)
 *   orc_locate                   pinned (barycentric containment)
 *   orc_cofaces2, orc_ncofaces   pinned (brute force over Kuhn simplices,
 *                                count formulas of Sec. V-A / V-B, Fig. 2)
 *   orc_trace_direct             pinned (brute force, triangle rule,
 *                                closed-manifold and Euler invariants)
 *   orc_trace_batch              pinned (k = 1 equals the direct trace;
 *                                subset of brute force; Fig. 5 template)
 *   orc_points                   pinned (linear f: the point is a root)
 *   orc_points_refined           pinned (zero iterations equal orc_points;
 *                                linear f exact; sphere radius error shrinks
 *                                to rounding; converged points equal a
 *                                library root finder's)
 *   orc_sincos, orc_fk           pinned (library sine/cosine, Rodrigues rotation
 *                                about every axis, spatial-arm hand poses)
 *   collision predicates         pinned (textbook clamp distance, hand cases
 *                                of link spheres against spheres and boxes;
 *                                cylinder: radial/axial clamp distance and
 *                                exact touching cases)
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* A plain growable map from fixed-length int32 tuples to a double payload. */
/* Items are kept in insertion order (the closure uses them as a worklist). */
/* ------------------------------------------------------------------------ */
typedef struct {
  int L;             /* tuple length in int32 words */
  int64_t n;         /* number of items */
  int64_t icap;      /* item capacity */
  int32_t *items;    /* n x L, insertion order */
  double *val;       /* n payloads */
  int64_t tcap;      /* table capacity (power of two) */
  int64_t *table;    /* item index, -1 when empty */
} omap;

static uint64_t tuple_hash(const int32_t *k, int L) {
  uint64_t h = 0x9E3779B97F4A7C15ull;
  for (int i = 0; i < L; ++i) {
    h ^= (uint64_t)(uint32_t)k[i];
    h *= 0xBF58476D1CE4E5B9ull;
    h ^= h >> 31;
  }
  return h;
}

static int omap_init(omap *m, int L) {
  m->L = L;
  m->n = 0;
  m->icap = 1024;
  m->tcap = 2048;
  m->items = (int32_t *)malloc(sizeof(int32_t) * (size_t)(m->icap * L));
  m->val = (double *)malloc(sizeof(double) * (size_t)m->icap);
  m->table = (int64_t *)malloc(sizeof(int64_t) * (size_t)m->tcap);
  if (!m->items || !m->val || !m->table) return -1;
  for (int64_t i = 0; i < m->tcap; ++i) m->table[i] = -1;
  return 0;
}

static void omap_destroy(omap *m) {
  free(m->items);
  free(m->val);
  free(m->table);
  memset(m, 0, sizeof(*m));
}

static int64_t omap_find(const omap *m, const int32_t *k) {
  uint64_t mask = (uint64_t)m->tcap - 1;
  uint64_t h = tuple_hash(k, m->L) & mask;
  for (;;) {
    int64_t idx = m->table[h];
    if (idx < 0) return -1;
    if (memcmp(m->items + idx * m->L, k, sizeof(int32_t) * (size_t)m->L) == 0)
      return idx;
    h = (h + 1) & mask;
  }
}

static int omap_rehash(omap *m, int64_t tcap) {
  int64_t *t = (int64_t *)malloc(sizeof(int64_t) * (size_t)tcap);
  if (!t) return -1;
  for (int64_t i = 0; i < tcap; ++i) t[i] = -1;
  uint64_t mask = (uint64_t)tcap - 1;
  for (int64_t idx = 0; idx < m->n; ++idx) {
    uint64_t h = tuple_hash(m->items + idx * m->L, m->L) & mask;
    while (t[h] >= 0) h = (h + 1) & mask;
    t[h] = idx;
  }
  free(m->table);
  m->table = t;
  m->tcap = tcap;
  return 0;
}

/* Returns the item index (existing or new); *inserted tells which. */
static int64_t omap_insert(omap *m, const int32_t *k, double v, int *inserted) {
  int64_t idx = omap_find(m, k);
  if (idx >= 0) {
    if (inserted) *inserted = 0;
    return idx;
  }
  if (m->n + 1 > m->icap) {
    int64_t nc = m->icap * 2;
    int32_t *it = (int32_t *)realloc(m->items, sizeof(int32_t) * (size_t)(nc * m->L));
    if (!it) return -1;
    m->items = it;
    double *vv = (double *)realloc(m->val, sizeof(double) * (size_t)nc);
    if (!vv) return -1;
    m->val = vv;
    m->icap = nc;
  }
  if (2 * (m->n + 1) > m->tcap) {
    if (omap_rehash(m, m->tcap * 2) != 0) return -1;
  }
  idx = m->n++;
  memcpy(m->items + idx * m->L, k, sizeof(int32_t) * (size_t)m->L);
  m->val[idx] = v;
  uint64_t mask = (uint64_t)m->tcap - 1;
  uint64_t h = tuple_hash(k, m->L) & mask;
  while (m->table[h] >= 0) h = (h + 1) & mask;
  m->table[h] = idx;
  if (inserted) *inserted = 1;
  return idx;
}

static int tuple_cmp_L;
static int tuple_cmp(const void *a, const void *b) {
  const int32_t *x = (const int32_t *)a, *y = (const int32_t *)b;
  for (int i = 0; i < tuple_cmp_L; ++i) {
    if (x[i] < y[i]) return -1;
    if (x[i] > y[i]) return 1;
  }
  return 0;
}

/* Sort a list of tuples lexicographically (signed comparison per word). */
static void sort_tuples(int32_t *t, int64_t n, int L) {
  tuple_cmp_L = L;
  qsort(t, (size_t)n, sizeof(int32_t) * (size_t)L, tuple_cmp);
}

/* ------------------------------------------------------------------------ */
/* Lattice, f, signs                                                         */
/* ------------------------------------------------------------------------ */
void orc_coords(const orc_space *sp, const int32_t *v, double *x) {
  const int d = sp->d;
  for (int j = 0; j < d; ++j) {
    double acc = sp->o[j];
    for (int k = 0; k < d; ++k) acc = fma(sp->M[j * d + k], (double)v[k], acc);
    x[j] = acc;
  }
}

/* ln 2 = LN2_HI + LN2_LO with LN2_HI a multiple of 2^-32, so that k * LN2_HI
 * is exact for |k| < 2^20. */
#define LN2_HI 0.6931471806019545
#define LN2_LO -4.2009150726810846e-11
#define INV_LN2 1.4426950408889634

double orc_exp(double t) {
  if (t < -708.0) return 0.0;
  double k = floor(t * INV_LN2 + 0.5);
  double r = fma(-k, LN2_HI, t);
  r = fma(-k, LN2_LO, r);
  /* Horner from 1/13! down to 1/1! and 1 */
  double p = 1.6059043836821613e-10; /* 1/13! */
  p = fma(r, p, 2.08767569878681e-09);   /* 1/12! */
  p = fma(r, p, 2.505210838544172e-08);  /* 1/11! */
  p = fma(r, p, 2.755731922398589e-07);  /* 1/10! */
  p = fma(r, p, 2.7557319223985893e-06); /* 1/9!  */
  p = fma(r, p, 2.48015873015873e-05);   /* 1/8!  */
  p = fma(r, p, 0.0001984126984126984);  /* 1/7!  */
  p = fma(r, p, 0.001388888888888889);   /* 1/6!  */
  p = fma(r, p, 0.008333333333333333);   /* 1/5!  */
  p = fma(r, p, 0.041666666666666664);   /* 1/4!  */
  p = fma(r, p, 0.16666666666666666);    /* 1/3!  */
  p = fma(r, p, 0.5);                    /* 1/2!  */
  p = fma(r, p, 1.0);                    /* 1/1!  */
  p = fma(r, p, 1.0);
  return ldexp(p, (int)k);
}

/* f(x): ORC_POLY sums alpha_i (gamma <s_i, x> + coef0)^p in index order, the
 * power as repeated multiplication; ORC_RBF sums alpha_i exp(-(gamma d2))
 * with d2 the fma chain of (x_j - s_ij)^2 over j.  Then + bias. */
double orc_f(const orc_fparams *f, const double *x) {
  const int d = f->d;
  double acc = 0.0;
  if (f->kernel == ORC_RBF) {
    for (int64_t i = 0; i < f->S; ++i) {
      const double *s = f->sv + i * d;
      double d2 = 0.0;
      for (int j = 0; j < d; ++j) {
        double df = x[j] - s[j];
        d2 = fma(df, df, d2);
      }
      acc = fma(f->alpha[i], orc_exp(-(f->gamma * d2)), acc);
    }
    return acc + f->bias;
  }
  for (int64_t i = 0; i < f->S; ++i) {
    const double *s = f->sv + i * d;
    double dot = 0.0;
    for (int j = 0; j < d; ++j) dot = fma(s[j], x[j], dot);
    double t = fma(f->gamma, dot, f->coef0);
    double tp = t;
    for (int r = 1; r < f->p; ++r) tp = tp * t;
    acc = fma(f->alpha[i], tp, acc);
  }
  return acc + f->bias;
}

double orc_f_grad(const orc_fparams *f, const double *x, double *g) {
  const int d = f->d;
  double acc = 0.0;
  for (int j = 0; j < d; ++j) g[j] = 0.0;
  if (f->kernel == ORC_RBF) {
    const double m2g = -2.0 * f->gamma;
    for (int64_t i = 0; i < f->S; ++i) {
      const double *s = f->sv + i * d;
      double df[ORC_MAXD], d2 = 0.0;
      for (int j = 0; j < d; ++j) {
        df[j] = x[j] - s[j];
        d2 = fma(df[j], df[j], d2);
      }
      double e = orc_exp(-(f->gamma * d2));
      acc = fma(f->alpha[i], e, acc);
      double w = (f->alpha[i] * e) * m2g;
      for (int j = 0; j < d; ++j) g[j] = fma(w, df[j], g[j]);
    }
    return acc + f->bias;
  }
  const double pg = (double)f->p * f->gamma;
  for (int64_t i = 0; i < f->S; ++i) {
    const double *s = f->sv + i * d;
    double dot = 0.0;
    for (int j = 0; j < d; ++j) dot = fma(s[j], x[j], dot);
    double t = fma(f->gamma, dot, f->coef0);
    double tp1 = 1.0;
    if (f->p > 1) {
      tp1 = t;
      for (int r = 2; r < f->p; ++r) tp1 = tp1 * t;
    }
    acc = fma(f->alpha[i], tp1 * t, acc);
    double w = (f->alpha[i] * tp1) * pg;
    for (int j = 0; j < d; ++j) g[j] = fma(w, s[j], g[j]);
  }
  return acc + f->bias;
}

int orc_seed_search(const orc_fparams *f, const orc_space *sp, int64_t n,
                    const double *q0, int32_t iters, double *q, double *fq) {
  const int d = sp->d;
  if (iters < 0) return -2;
  for (int64_t i = 0; i < n; ++i) {
    double x[ORC_MAXD], g[ORC_MAXD];
    for (int j = 0; j < d; ++j) x[j] = q0[i * d + j];
    for (int it = 0; it < iters; ++it) {
      double fv = orc_f_grad(f, x, g);
      double n2 = 0.0;
      for (int j = 0; j < d; ++j) n2 = fma(g[j], g[j], n2);
      if (!(n2 > 0.0)) break;
      double c = fv / n2;
      for (int j = 0; j < d; ++j) {
        double v = fma(-c, g[j], x[j]);
        x[j] = v < sp->lo[j] ? sp->lo[j] : (v > sp->hi[j] ? sp->hi[j] : v);
      }
    }
    for (int j = 0; j < d; ++j) q[i * d + j] = x[j];
    fq[i] = orc_f(f, x);
  }
  return 0;
}

void orc_f_batch(const orc_fparams *f, const orc_space *sp, int64_t n,
                 const int32_t *v, double *out) {
  double x[ORC_MAXD];
  for (int64_t i = 0; i < n; ++i) {
    orc_coords(sp, v + i * sp->d, x);
    out[i] = orc_f(f, x);
  }
}

static int sign_bit(double fv) { return !(fv < 0.0); }

static int in_box(const orc_space *sp, const double *x) {
  for (int j = 0; j < sp->d; ++j)
    if (!(x[j] >= sp->lo[j] && x[j] <= sp->hi[j])) return 0;
  return 1;
}

/* Vertex memo: f at lattice vertex u of the lattice refined by k, i.e. at
 * x(k u); NaN marks a vertex outside the domain box. */
typedef struct {
  const orc_fparams *f;
  const orc_space *sp;
  int32_t k;
  omap vm;
} vctx;

static int vctx_init(vctx *c, const orc_fparams *f, const orc_space *sp, int32_t k) {
  c->f = f;
  c->sp = sp;
  c->k = k;
  return omap_init(&c->vm, sp->d);
}

/* 1 if u is inside the box (and *fv is set), 0 otherwise, -1 on failure. */
static int vertex_value(vctx *c, const int32_t *u, double *fv) {
  int64_t idx = omap_find(&c->vm, u);
  double val;
  if (idx >= 0) {
    val = c->vm.val[idx];
  } else {
    int32_t y[ORC_MAXD];
    double x[ORC_MAXD];
    for (int j = 0; j < c->sp->d; ++j) y[j] = c->k * u[j];
    orc_coords(c->sp, y, x);
    val = in_box(c->sp, x) ? orc_f(c->f, x) : NAN;
    if (omap_insert(&c->vm, u, val, NULL) < 0) return -1;
  }
  if (isnan(val)) return 0;
  *fv = val;
  return 1;
}

/* Edge (v, R): endpoints v and v + 1_R.  1 if it intersects, 0 if not. */
static int edge_intersects(vctx *c, const int32_t *v, uint32_t mask) {
  int32_t b[ORC_MAXD];
  for (int j = 0; j < c->sp->d; ++j) b[j] = v[j] + (int32_t)((mask >> j) & 1u);
  double fa, fb;
  int ra = vertex_value(c, v, &fa);
  if (ra <= 0) return ra;
  int rb = vertex_value(c, b, &fb);
  if (rb <= 0) return rb;
  return sign_bit(fa) != sign_bit(fb);
}

/* ------------------------------------------------------------------------ */
/* Permutahedral representation                                              */
/* ------------------------------------------------------------------------ */

/* u += sum of roots in `part` (bit j < d: +e_j; bit d: -(1,...,1)). */
static void add_part(int d, int32_t *u, uint32_t part) {
  for (int j = 0; j < d; ++j) u[j] += (int32_t)((part >> j) & 1u);
  if ((part >> d) & 1u)
    for (int j = 0; j < d; ++j) u[j] -= 1;
}

int32_t orc_canonical(int32_t d, const int32_t *v, int32_t nparts,
                      const uint32_t *parts, int32_t *vc, uint32_t *pc) {
  int id = -1;
  for (int i = 0; i < nparts; ++i)
    if ((parts[i] >> d) & 1u) id = i;
  if (id < 0) return -1;
  int32_t u[ORC_MAXD];
  memcpy(u, v, sizeof(int32_t) * (size_t)d);
  for (int i = 0; i <= id; ++i) add_part(d, u, parts[i]);
  memcpy(vc, u, sizeof(int32_t) * (size_t)d);
  for (int m = 0; m < nparts; ++m) pc[m] = parts[(id + 1 + m) % nparts];
  return nparts;
}

/* Canonical edge between two vertices whose difference is a 0/1 vector up
 * to sign: the componentwise smaller endpoint and the support. */
static int edge_from_pair(int d, const int32_t *a, const int32_t *b,
                          int32_t *v, uint32_t *mask) {
  int pos = 0, neg = 0;
  uint32_t m = 0;
  for (int j = 0; j < d; ++j) {
    int32_t df = b[j] - a[j];
    if (df == 1) {
      pos = 1;
      m |= 1u << j;
    } else if (df == -1) {
      neg = 1;
      m |= 1u << j;
    } else if (df != 0) {
      return -1;
    }
  }
  if ((pos && neg) || m == 0) return -1;
  memcpy(v, pos ? a : b, sizeof(int32_t) * (size_t)d);
  *mask = m;
  return 0;
}

/* Vertices of the triangle given by starting vertex v and cyclic parts. */
static void triangle_vertices(int d, const int32_t *v, uint32_t p0, uint32_t p1,
                              int32_t *tri) {
  memcpy(tri, v, sizeof(int32_t) * (size_t)d);
  memcpy(tri + d, v, sizeof(int32_t) * (size_t)d);
  add_part(d, tri + d, p0);
  memcpy(tri + 2 * d, tri + d, sizeof(int32_t) * (size_t)d);
  add_part(d, tri + 2 * d, p1);
}

/* The 2-cofaces of edge (v, (R, Q)), Q = {0..d} \ R: all ordered
 * three-part partitions that merge back into (R, Q), i.e. every ordered
 * split of R and every ordered split of Q (Sec. V-A query 3). */
int64_t orc_cofaces2(int32_t d, const int32_t *v, uint32_t mask, int32_t *tri) {
  const uint32_t full = (1u << (d + 1)) - 1u;
  const uint32_t R = mask & full, Q = full & ~R;
  int64_t n = 0;
  for (uint32_t A = (R - 1u) & R; A != 0u; A = (A - 1u) & R) {
    triangle_vertices(d, v, A, R & ~A, tri + n * 3 * d);
    ++n;
  }
  for (uint32_t A = (Q - 1u) & Q; A != 0u; A = (A - 1u) & Q) {
    /* parts (R, A, Q\A) from v: vertices v, v + e_R, v + e_R + e_A */
    triangle_vertices(d, v, R, A, tri + n * 3 * d);
    ++n;
  }
  return n;
}

static int next_perm(int32_t *a, int n) {
  int i = n - 2;
  while (i >= 0 && a[i] >= a[i + 1]) --i;
  if (i < 0) return 0;
  int j = n - 1;
  while (a[j] <= a[i]) --j;
  int32_t t = a[i];
  a[i] = a[j];
  a[j] = t;
  for (int l = i + 1, r = n - 1; l < r; ++l, --r) {
    t = a[l];
    a[l] = a[r];
    a[r] = t;
  }
  return 1;
}

/* The n-cofaces of edge (v, (R, Q)): every ordering of R followed by every
 * ordering of Q, as singleton parts, put in canonical form (Sec. V-B). */
int64_t orc_ncofaces(int32_t d, const int32_t *v, uint32_t mask, int32_t *out) {
  const uint32_t full = (1u << (d + 1)) - 1u;
  const uint32_t R = mask & full, Q = full & ~R;
  int32_t pr[ORC_MAXD + 1], pq[ORC_MAXD + 1];
  int nr = 0, nq = 0;
  for (int j = 0; j <= d; ++j) {
    if ((R >> j) & 1u) pr[nr++] = j;
    if ((Q >> j) & 1u) pq[nq++] = j;
  }
  int64_t n = 0;
  do {
    int32_t q2[ORC_MAXD + 1];
    memcpy(q2, pq, sizeof(int32_t) * (size_t)nq);
    do {
      uint32_t parts[ORC_MAXD + 1], pc[ORC_MAXD + 1];
      int np = 0;
      for (int i = 0; i < nr; ++i) parts[np++] = 1u << pr[i];
      for (int i = 0; i < nq; ++i) parts[np++] = 1u << q2[i];
      int32_t *o = out + n * 2 * d;
      orc_canonical(d, v, np, parts, o, pc);
      for (int i = 0; i < d; ++i) {
        int b = 0;
        while (!((pc[i] >> b) & 1u)) ++b;
        o[d + i] = b;
      }
      ++n;
    } while (next_perm(q2, nq));
  } while (next_perm(pr, nr));
  return n;
}

void orc_locate(const orc_space *sp, int32_t coarse_k, const double *y,
                int32_t *v, int32_t *w) {
  const int d = sp->d;
  double z[ORC_MAXD], fr[ORC_MAXD], t[ORC_MAXD];
  for (int k = 0; k < d; ++k) t[k] = y[k] - sp->o[k];
  for (int j = 0; j < d; ++j) {
    double acc = 0.0;
    for (int k = 0; k < d; ++k) acc = fma(sp->Minv[j * d + k], t[k], acc);
    z[j] = acc;
    if (coarse_k > 1) z[j] = z[j] / (double)coarse_k;
    double fl = floor(z[j]);
    v[j] = (int32_t)fl;
    fr[j] = z[j] - fl;
  }
  /* indices by descending fractional part, ties by ascending index */
  for (int j = 0; j < d; ++j) w[j] = j;
  for (int i = 1; i < d; ++i) {
    int32_t cur = w[i];
    int j = i - 1;
    while (j >= 0 && fr[w[j]] < fr[cur]) {
      w[j + 1] = w[j];
      --j;
    }
    w[j + 1] = cur;
  }
}

/* ------------------------------------------------------------------------ */
/* Traces                                                                    */
/* ------------------------------------------------------------------------ */
static int emit_edges(omap *em, int d, orc_edges *out) {
  out->n = em->n;
  out->d = d;
  int32_t *tmp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(em->n * (d + 1) + 1));
  out->v = (int32_t *)malloc(sizeof(int32_t) * (size_t)(em->n * d + 1));
  out->mask = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(em->n + 1));
  if (!tmp || !out->v || !out->mask) return -1;
  memcpy(tmp, em->items, sizeof(int32_t) * (size_t)(em->n * (d + 1)));
  sort_tuples(tmp, em->n, d + 1);
  for (int64_t i = 0; i < em->n; ++i) {
    memcpy(out->v + i * d, tmp + i * (d + 1), sizeof(int32_t) * (size_t)d);
    out->mask[i] = (uint32_t)tmp[i * (d + 1) + d];
  }
  free(tmp);
  return 0;
}

/* Insert edge (v, mask) into the edge set if it intersects. */
static int consider_edge(vctx *c, omap *em, const int32_t *v, uint32_t mask) {
  const int d = c->sp->d;
  int32_t key[ORC_MAXD + 1];
  memcpy(key, v, sizeof(int32_t) * (size_t)d);
  key[d] = (int32_t)mask;
  if (omap_find(em, key) >= 0) return 0;
  int r = edge_intersects(c, v, mask);
  if (r < 0) return -1;
  if (r == 1 && omap_insert(em, key, 0.0, NULL) < 0) return -1;
  return 0;
}

/* Closure of the seeds' intersecting edges on the lattice refined by ck. */
static int trace_closure(vctx *c, const double *seeds, int64_t n_seeds, omap *em) {
  const int d = c->sp->d;
  int32_t *tri = (int32_t *)malloc(sizeof(int32_t) * (size_t)(3 * d) * ((size_t)2 << d));
  if (!tri) return -1;
  for (int64_t s = 0; s < n_seeds; ++s) {
    int32_t v[ORC_MAXD], w[ORC_MAXD], u[ORC_MAXD + 1][ORC_MAXD];
    orc_locate(c->sp, c->k, seeds + s * d, v, w);
    memcpy(u[0], v, sizeof(int32_t) * (size_t)d);
    for (int m = 0; m < d; ++m) {
      memcpy(u[m + 1], u[m], sizeof(int32_t) * (size_t)d);
      u[m + 1][w[m]] += 1;
    }
    for (int a = 0; a <= d; ++a)
      for (int b = a + 1; b <= d; ++b) {
        int32_t ev[ORC_MAXD];
        uint32_t em_;
        if (edge_from_pair(d, u[a], u[b], ev, &em_) != 0) goto fail;
        if (consider_edge(c, em, ev, em_) != 0) goto fail;
      }
  }
  for (int64_t head = 0; head < em->n; ++head) {
    int32_t ev[ORC_MAXD];
    memcpy(ev, em->items + head * (d + 1), sizeof(int32_t) * (size_t)d);
    uint32_t emask = (uint32_t)em->items[head * (d + 1) + d];
    int64_t nt = orc_cofaces2(d, ev, emask, tri);
    for (int64_t t = 0; t < nt; ++t) {
      const int32_t *T = tri + t * 3 * d;
      static const int pa[3] = {0, 0, 1}, pb[3] = {1, 2, 2};
      for (int e = 0; e < 3; ++e) {
        int32_t nv[ORC_MAXD];
        uint32_t nm;
        if (edge_from_pair(d, T + pa[e] * d, T + pb[e] * d, nv, &nm) != 0) goto fail;
        if (consider_edge(c, em, nv, nm) != 0) goto fail;
      }
    }
  }
  free(tri);
  return 0;
fail:
  free(tri);
  return -1;
}

int orc_trace_direct(const orc_fparams *f, const orc_space *sp,
                     int32_t coarse_k, const double *seeds, int64_t n_seeds,
                     orc_edges *out) {
  if (!f || !sp || sp->d < 2 || sp->d > 7 || f->d != sp->d || coarse_k < 1) return -2;
  vctx c;
  omap em;
  if (vctx_init(&c, f, sp, coarse_k) != 0) return -1;
  if (omap_init(&em, sp->d + 1) != 0) return -1;
  int rc = trace_closure(&c, seeds, n_seeds, &em);
  if (rc == 0) rc = emit_edges(&em, sp->d, out);
  omap_destroy(&em);
  omap_destroy(&c.vm);
  return rc;
}

/* The set of coarse n-simplices: n-cofaces of the coarse traced edges. */
static int build_sigma(const orc_fparams *f, const orc_space *sp, int32_t k,
                       const double *seeds, int64_t n_seeds, omap *sig) {
  const int d = sp->d;
  vctx c;
  omap em;
  if (vctx_init(&c, f, sp, k) != 0) return -1;
  if (omap_init(&em, d + 1) != 0) return -1;
  int rc = trace_closure(&c, seeds, n_seeds, &em);
  omap_destroy(&c.vm);
  if (rc != 0) {
    omap_destroy(&em);
    return rc;
  }
  int64_t maxn = 1;
  for (int i = 2; i <= d; ++i) maxn *= i; /* |R|!|Q|! <= d! */
  int32_t *buf = (int32_t *)malloc(sizeof(int32_t) * (size_t)(maxn * 2 * d));
  if (!buf || omap_init(sig, 2 * d) != 0) {
    free(buf);
    omap_destroy(&em);
    return -1;
  }
  for (int64_t i = 0; i < em.n; ++i) {
    int64_t nc = orc_ncofaces(d, em.items + i * (d + 1), (uint32_t)em.items[i * (d + 1) + d], buf);
    for (int64_t j = 0; j < nc; ++j)
      if (omap_insert(sig, buf + j * 2 * d, 0.0, NULL) < 0) {
        rc = -1;
        break;
      }
  }
  free(buf);
  omap_destroy(&em);
  return rc;
}

int orc_batch_sigma(const orc_fparams *f, const orc_space *sp, int32_t k,
                    const double *seeds, int64_t n_seeds, int64_t *n,
                    int32_t **sigma) {
  if (!f || !sp || sp->d < 2 || sp->d > 7 || f->d != sp->d || k < 1) return -2;
  omap sig;
  int rc = build_sigma(f, sp, k, seeds, n_seeds, &sig);
  if (rc != 0) return rc;
  const int L = 2 * sp->d;
  *n = sig.n;
  *sigma = (int32_t *)malloc(sizeof(int32_t) * (size_t)(sig.n * L + 1));
  if (!*sigma) return -1;
  memcpy(*sigma, sig.items, sizeof(int32_t) * (size_t)(sig.n * L));
  sort_tuples(*sigma, sig.n, L);
  omap_destroy(&sig);
  return 0;
}

/* Local point u (Eq. 1 coordinates) lies in the closed simplex: Eq. (2)
 * with >=, i.e. k >= u_0 >= u_1 >= ... >= u_{d-1} >= 0. */
static int local_inside(int d, int32_t k, const int32_t *u) {
  if (u[0] > k) return 0;
  for (int i = 0; i + 1 < d; ++i)
    if (u[i] < u[i + 1]) return 0;
  return u[d - 1] >= 0;
}

int orc_template(int32_t d, int32_t k, int64_t *n_pts, int32_t *pts,
                 int64_t *n_edges, int32_t *edge_u, uint32_t *edge_r) {
  if (d < 2 || d > 7 || k < 1) return -2;
  int64_t np = 0, ne = 0;
  int32_t u[ORC_MAXD];
  /* odometer over 0..k per coordinate, keeping the inside points */
  for (int j = 0; j < d; ++j) u[j] = 0;
  for (;;) {
    if (local_inside(d, k, u)) {
      if (pts) memcpy(pts + np * d, u, sizeof(int32_t) * (size_t)d);
      ++np;
      for (uint32_t R = 1; R < (1u << d); ++R) {
        int32_t u2[ORC_MAXD];
        for (int j = 0; j < d; ++j) u2[j] = u[j] + (int32_t)((R >> j) & 1u);
        if (local_inside(d, k, u2)) {
          if (edge_u) memcpy(edge_u + ne * d, u, sizeof(int32_t) * (size_t)d);
          if (edge_r) edge_r[ne] = R;
          ++ne;
        }
      }
    }
    int j = 0;
    while (j < d && u[j] == k) u[j++] = 0;
    if (j == d) break;
    ++u[j];
  }
  *n_pts = np;
  *n_edges = ne;
  return 0;
}

int orc_trace_batch(const orc_fparams *f, const orc_space *sp, int32_t k,
                    const double *seeds, int64_t n_seeds, orc_edges *out,
                    int64_t *n_sigma) {
  if (!f || !sp || sp->d < 2 || sp->d > 7 || f->d != sp->d || k < 1) return -2;
  const int d = sp->d;
  omap sig;
  int rc = build_sigma(f, sp, k, seeds, n_seeds, &sig);
  if (rc != 0) return rc;
  if (n_sigma) *n_sigma = sig.n;
  int64_t np, ne;
  orc_template(d, k, &np, NULL, &ne, NULL, NULL);
  int32_t *tu = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ne * d + 1));
  uint32_t *tr = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(ne + 1));
  vctx c;
  omap em;
  if (!tu || !tr || vctx_init(&c, f, sp, 1) != 0 || omap_init(&em, d + 1) != 0) {
    free(tu);
    free(tr);
    omap_destroy(&sig);
    return -1;
  }
  orc_template(d, k, &np, NULL, &ne, tu, tr);
  for (int64_t s = 0; s < sig.n && rc == 0; ++s) {
    const int32_t *vc = sig.items + s * 2 * d;
    const int32_t *w = vc + d;
    for (int64_t e = 0; e < ne; ++e) {
      const int32_t *u = tu + e * d;
      int32_t ya[ORC_MAXD], yb[ORC_MAXD], ev[ORC_MAXD];
      uint32_t emask;
      /* local -> global: y_{w_i} = k v_{w_i} + u_i (Eq. 1 in lattice form) */
      for (int i = 0; i < d; ++i) {
        ya[w[i]] = k * vc[w[i]] + u[i];
        yb[w[i]] = ya[w[i]] + (int32_t)((tr[e] >> i) & 1u);
      }
      if (edge_from_pair(d, ya, yb, ev, &emask) != 0 ||
          consider_edge(&c, &em, ev, emask) != 0) {
        rc = -1;
        break;
      }
    }
  }
  if (rc == 0) rc = emit_edges(&em, d, out);
  free(tu);
  free(tr);
  omap_destroy(&em);
  omap_destroy(&c.vm);
  omap_destroy(&sig);
  return rc;
}

int orc_brute(const orc_fparams *f, const orc_space *sp, orc_edges *out) {
  if (!f || !sp || sp->d < 2 || sp->d > 7 || f->d != sp->d) return -2;
  const int d = sp->d;
  int32_t vmin[ORC_MAXD], vmax[ORC_MAXD];
  for (int j = 0; j < d; ++j) {
    double zl = 0.0, zh = 0.0;
    for (int k = 0; k < d; ++k) {
      double a = sp->Minv[j * d + k] * (sp->lo[k] - sp->o[k]);
      double b = sp->Minv[j * d + k] * (sp->hi[k] - sp->o[k]);
      zl += a < b ? a : b;
      zh += a < b ? b : a;
    }
    vmin[j] = (int32_t)floor(zl) - 2;
    vmax[j] = (int32_t)ceil(zh) + 2;
  }
  vctx c;
  omap em;
  if (vctx_init(&c, f, sp, 1) != 0 || omap_init(&em, d + 1) != 0) return -1;
  int32_t v[ORC_MAXD];
  memcpy(v, vmin, sizeof(int32_t) * (size_t)d);
  int rc = 0;
  for (;;) {
    double fv;
    int r = vertex_value(&c, v, &fv);
    if (r < 0) {
      rc = -1;
      break;
    }
    if (r == 1)
      for (uint32_t R = 1; R < (1u << d); ++R)
        if (consider_edge(&c, &em, v, R) != 0) {
          rc = -1;
          break;
        }
    int j = 0;
    while (j < d && v[j] == vmax[j]) {
      v[j] = vmin[j];
      ++j;
    }
    if (j == d) break;
    ++v[j];
  }
  if (rc == 0) rc = emit_edges(&em, d, out);
  omap_destroy(&em);
  omap_destroy(&c.vm);
  return rc;
}

int orc_points(const orc_fparams *f, const orc_space *sp, int64_t n,
               const int32_t *v, const uint32_t *mask, double *pts, double *t) {
  const int d = sp->d;
  for (int64_t i = 0; i < n; ++i) {
    int32_t b[ORC_MAXD];
    double xa[ORC_MAXD], xb[ORC_MAXD];
    for (int j = 0; j < d; ++j) b[j] = v[i * d + j] + (int32_t)((mask[i] >> j) & 1u);
    orc_coords(sp, v + i * d, xa);
    orc_coords(sp, b, xb);
    double fa = orc_f(f, xa), fb = orc_f(f, xb);
    double tt = fa / (fa - fb);
    if (t) t[i] = tt;
    for (int j = 0; j < d; ++j) pts[i * d + j] = fma(tt, xb[j] - xa[j], xa[j]);
  }
  return 0;
}

int orc_points_refined(const orc_fparams *f, const orc_space *sp, int64_t n,
                       const int32_t *v, const uint32_t *mask, int32_t iters,
                       double *pts) {
  if (iters < 0) return -2;
  const int d = sp->d;
  for (int64_t i = 0; i < n; ++i) {
    int32_t bv[ORC_MAXD];
    double a[ORC_MAXD], b[ORC_MAXD], m[ORC_MAXD];
    for (int j = 0; j < d; ++j) bv[j] = v[i * d + j] + (int32_t)((mask[i] >> j) & 1u);
    orc_coords(sp, v + i * d, a);
    orc_coords(sp, bv, b);
    double fa = orc_f(f, a), fb = orc_f(f, b);
    int last = 0; /* -1: a moved last, +1: b moved last */
    for (int it = 0; it < iters; ++it) {
      double t = fa / (fa - fb);
      for (int j = 0; j < d; ++j) m[j] = fma(t, b[j] - a[j], a[j]);
      double fm = orc_f(f, m);
      if (sign_bit(fm) == sign_bit(fa)) {
        memcpy(a, m, sizeof(double) * (size_t)d);
        fa = fm;
        if (last == -1) fb = 0.5 * fb;
        last = -1;
      } else {
        memcpy(b, m, sizeof(double) * (size_t)d);
        fb = fm;
        if (last == 1) fa = 0.5 * fa;
        last = 1;
      }
    }
    double t = fa / (fa - fb);
    for (int j = 0; j < d; ++j) pts[i * d + j] = fma(t, b[j] - a[j], a[j]);
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Collision check (Sec. V-C, Appendix A)                                    */
/* ------------------------------------------------------------------------ */

/* pi/2 split into three parts for Cody-Waite reduction; the first two carry
 * 33 significant bits each so that k * part is exact for small k. */
#define PIO2_A 1.5707963267341256
#define PIO2_B 6.077100506303966e-11
#define PIO2_C 2.0222662487959506e-21
#define TWO_OVER_PI 0.6366197723675814

void orc_sincos(double q, double *s, double *c) {
  double kf = floor(q * TWO_OVER_PI + 0.5);
  double r = fma(-kf, PIO2_A, q);
  r = fma(-kf, PIO2_B, r);
  r = fma(-kf, PIO2_C, r);
  double z = r * r;
  /* Taylor series about 0 in Horner form in z = r^2:
   * sin r = r + r z (-1/3! + z (1/5! - ... + z/17!)),
   * cos r = 1 + z (-1/2! + z (1/4! - ... + z/16!)). */
  double ps = 2.8114572543455206e-15;     /*  1/17! */
  ps = fma(z, ps, -7.647163731819816e-13); /* -1/15! */
  ps = fma(z, ps, 1.6059043836821613e-10); /*  1/13! */
  ps = fma(z, ps, -2.505210838544172e-08); /* -1/11! */
  ps = fma(z, ps, 2.7557319223985893e-06); /*  1/9!  */
  ps = fma(z, ps, -0.0001984126984126984); /* -1/7!  */
  ps = fma(z, ps, 0.008333333333333333);   /*  1/5!  */
  ps = fma(z, ps, -0.16666666666666666);   /* -1/3!  */
  double sr = fma(r * z, ps, r);
  double pc = 4.779477332387385e-14;       /*  1/16! */
  pc = fma(z, pc, -1.1470745597729725e-11); /* -1/14! */
  pc = fma(z, pc, 2.08767569878681e-09);   /*  1/12! */
  pc = fma(z, pc, -2.755731922398589e-07); /* -1/10! */
  pc = fma(z, pc, 2.48015873015873e-05);   /*  1/8!  */
  pc = fma(z, pc, -0.001388888888888889);  /* -1/6!  */
  pc = fma(z, pc, 0.041666666666666664);   /*  1/4!  */
  pc = fma(z, pc, -0.5);                   /* -1/2!  */
  double cr = fma(z, pc, 1.0);
  long long m = ((long long)kf) & 3;
  if (m == 0) {
    *s = sr;
    *c = cr;
  } else if (m == 1) {
    *s = cr;
    *c = -sr;
  } else if (m == 2) {
    *s = -sr;
    *c = -cr;
  } else {
    *s = -cr;
    *c = sr;
  }
}

static double dot3_sq(double x, double y, double z) { return fma(z, z, fma(y, y, x * x)); }

int orc_sphere_sphere(const double *a, double ra, const double *b, double rb) {
  double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
  double rr = ra + rb;
  return dot3_sq(dx, dy, dz) <= rr * rr;
}

int orc_capsule_sphere(const double *p0, const double *p1, double rc,
                       const double *c, double rs) {
  double u[3], w[3], e[3];
  for (int j = 0; j < 3; ++j) {
    u[j] = p1[j] - p0[j];
    w[j] = c[j] - p0[j];
  }
  double uu = fma(u[2], u[2], fma(u[1], u[1], u[0] * u[0]));
  double wu = fma(w[2], u[2], fma(w[1], u[1], w[0] * u[0]));
  double t = uu > 0.0 ? wu / uu : 0.0;
  t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
  for (int j = 0; j < 3; ++j) e[j] = fma(-t, u[j], w[j]);
  double rr = rc + rs;
  return dot3_sq(e[0], e[1], e[2]) <= rr * rr;
}

/* Appendix A, sphere vs box: move the centre into the box frame, fold into
 * the first octant, then (1) the padded bounding test, (2) the edge region,
 * (3) the vertex region; anything else collides.  Region boundaries: a
 * coordinate with p_i - l_i/2 > 0 is "outside" along axis i. */
int orc_sphere_box(const double *c, double r, const double *T, const double *l) {
  double dx = c[0] - T[3], dy = c[1] - T[7], dz = c[2] - T[11];
  double g[3];
  for (int i = 0; i < 3; ++i) {
    double p = fabs(fma(T[8 + i], dz, fma(T[4 + i], dy, T[i] * dx)));
    g[i] = p - 0.5 * l[i];
  }
  for (int i = 0; i < 3; ++i)
    if (g[i] > r) return 0;
  int nout = (g[0] > 0.0) + (g[1] > 0.0) + (g[2] > 0.0);
  if (nout == 2) {
    double a = 0.0, b = 0.0;
    int first = 1;
    for (int i = 0; i < 3; ++i)
      if (g[i] > 0.0) {
        if (first) {
          a = g[i];
          first = 0;
        } else {
          b = g[i];
        }
      }
    return !(fma(b, b, a * a) > r * r);
  }
  if (nout == 3) return !(dot3_sq(g[0], g[1], g[2]) > r * r);
  return 1;
}

/* Appendix A, sphere vs cylinder: centre into the cylinder frame (axis z,
 * origin at its centre), folded into the first octant: p.  With rho the
 * distance of p from the axis and g = p_z - h/2: no collision when g > r or
 * rho > r + rc (the padded cylinder); otherwise, in the ring region (g > 0
 * and rho > rc) no collision when (rho - rc)^2 + g^2 > r^2; anything else
 * collides.  The ring test without square roots: with q = r^2 - g^2 >= 0
 * there, (rho - rc)^2 > q with rho > rc holds exactly when
 * L = rho^2 - rc^2 - q is positive and L^2 > 4 rc^2 q. */
int orc_sphere_cylinder(const double *c, double r, const double *T, double rc, double h) {
  double dx = c[0] - T[3], dy = c[1] - T[7], dz = c[2] - T[11];
  double p[3];
  for (int i = 0; i < 3; ++i) p[i] = fabs(fma(T[8 + i], dz, fma(T[4 + i], dy, T[i] * dx)));
  double rho2 = fma(p[1], p[1], p[0] * p[0]);
  double g = p[2] - 0.5 * h;
  if (g > r) return 0;
  double rr = r + rc;
  if (rho2 > rr * rr) return 0;
  if (g > 0.0 && rho2 > rc * rc) {
    double q = r * r - g * g;
    double L = (rho2 - rc * rc) - q;
    if (L > 0.0 && L * L > 4.0 * (rc * rc) * q) return 0;
  }
  return 1;
}

static void compose(const double *A, const double *B, double *C) {
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c)
      C[r * 4 + c] = fma(A[r * 4 + 2], B[8 + c], fma(A[r * 4 + 1], B[4 + c], A[r * 4 + 0] * B[c]));
    C[r * 4 + 3] = fma(A[r * 4 + 2], B[11], fma(A[r * 4 + 1], B[7], fma(A[r * 4 + 0], B[3], A[r * 4 + 3])));
  }
}

static void rotation(int axis, double s, double c, double *R) {
  memset(R, 0, sizeof(double) * 12);
  if (axis == 0) {
    R[0] = 1.0;
    R[5] = c;
    R[6] = -s;
    R[9] = s;
    R[10] = c;
  } else if (axis == 1) {
    R[0] = c;
    R[2] = s;
    R[5] = 1.0;
    R[8] = -s;
    R[10] = c;
  } else {
    R[0] = c;
    R[1] = -s;
    R[4] = s;
    R[5] = c;
    R[10] = 1.0;
  }
}

static void xform(const double *T, const double *p, double *o) {
  for (int r = 0; r < 3; ++r)
    o[r] = fma(T[r * 4 + 2], p[2], fma(T[r * 4 + 1], p[1], fma(T[r * 4 + 0], p[0], T[r * 4 + 3])));
}

void orc_fk(const orc_scene *sc, const double *q, double *T_out) {
  double T[12] = {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0};
  for (int i = 0; i < sc->n_joints; ++i) {
    double s, c, A[12], R[12];
    orc_sincos(q[i], &s, &c);
    compose(T, sc->joint_T + 12 * i, A);
    rotation(sc->joint_axis[i], s, c, R);
    compose(A, R, T);
    memcpy(T_out + 12 * i, T, sizeof(T));
  }
}

int orc_check(const orc_scene *sc, int64_t n, const double *q, uint8_t *verdict) {
  if (sc->n_joints < 1 || sc->n_joints > 7) return -2;
  /* capsules are tested against spheres only (capsule-box, capsule-cylinder
   * are not defined) */
  if (sc->n_lcap > 0 && (sc->n_obox > 0 || sc->n_ocyl > 0)) return -2;
  double T[7 * 12];
  for (int64_t i = 0; i < n; ++i) {
    orc_fk(sc, q + i * sc->n_joints, T);
    int hit = 0;
    for (int a = 0; a < sc->n_lsph && !hit; ++a) {
      double cw[3];
      xform(T + 12 * sc->lsph_link[a], sc->lsph_c + 3 * a, cw);
      for (int b = 0; b < sc->n_osph && !hit; ++b)
        hit = orc_sphere_sphere(cw, sc->lsph_r[a], sc->osph_c + 3 * b, sc->osph_r[b]);
      for (int b = 0; b < sc->n_obox && !hit; ++b)
        hit = orc_sphere_box(cw, sc->lsph_r[a], sc->obox_T + 12 * b, sc->obox_l + 3 * b);
      for (int b = 0; b < sc->n_ocyl && !hit; ++b)
        hit = orc_sphere_cylinder(cw, sc->lsph_r[a], sc->ocyl_T + 12 * b, sc->ocyl_rh[2 * b],
                                  sc->ocyl_rh[2 * b + 1]);
    }
    for (int a = 0; a < sc->n_lcap && !hit; ++a) {
      double p0[3], p1[3];
      xform(T + 12 * sc->lcap_link[a], sc->lcap_p0 + 3 * a, p0);
      xform(T + 12 * sc->lcap_link[a], sc->lcap_p1 + 3 * a, p1);
      for (int b = 0; b < sc->n_osph && !hit; ++b)
        hit = orc_capsule_sphere(p0, p1, sc->lcap_r[a], sc->osph_c + 3 * b, sc->osph_r[b]);
    }
    verdict[i] = (uint8_t)hit;
  }
  return 0;
}

void orc_free(void *p) { free(p); }
