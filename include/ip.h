/*
 * ip.h -- C ABI of the MI355X library that traces an implicit manifold
 * f(q) = 0 through the Coxeter triangulation of configuration space and
 * collision-checks the traced cells (Li & Dantam, "Scaling Motion Planning
 * Infeasibility Proofs", arXiv 2406.04795, Sec. V).
 *
 * Conventions shared by every call:
 *   - Return value: IP_OK (0) or a negative IP_E* code.  Nothing aborts and
 *     no C++ exception crosses this boundary.  On error, output handles are
 *     set to NULL and ip_last_error(ctx) holds a message.
 *   - "host" pointers are read during the call only; the caller keeps
 *     ownership.  "device" pointers are HIP device addresses on the context's
 *     device, used on the context's stream; the caller keeps ownership.
 *   - Handles returned by the library (ip_problem, ip_cells) are owned by the
 *     caller until released with the matching *_free call, which must happen
 *     before ip_destroy of the context that made them.
 *   - All floating-point inputs are FP64.  Matrices are row-major.
 *   - A context is not thread-safe; use one per host thread.
 */
#ifndef IP_H
#define IP_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define IP_MAX_D 7

enum {
  IP_OK = 0,
  IP_EINVAL = -1,   /* bad argument (dimension, degree, NaN, NULL) */
  IP_ENOMEM = -2,   /* device memory or batch budget too small */
  IP_ERANGE = -3,   /* lattice coordinates of the domain overflow the 64-bit keys */
  IP_EDEVICE = -4,  /* HIP runtime error (message in ip_last_error) */
  IP_EAGAIN = -5,   /* result not ready (serving loop) */
  IP_ECANCELED = -6 /* a batch callback asked to stop (ip_trace_check_batches) */
};

enum {
  IP_FP64 = 0,          /* every f evaluation in FP64, canonical order */
  IP_FP32_CERTIFY = 1   /* FP32 evaluation with an error bound; vertices whose
                           sign the bound cannot settle are re-evaluated in
                           FP64, so the traced set equals the FP64 one.
                           ip_trace of an RBF manifold evaluates in FP64
                           in this mode too: the FP32 bound of a sum of
                           exponentials settles signs but not points, so
                           every traced vertex would need FP64 anyway */
};

typedef struct ip_ctx ip_ctx;
typedef struct ip_problem ip_problem;
typedef struct ip_cells ip_cells;

/* Manifold function, the decision function of a kernel SVM (Sec. IV-A: the
 * learned manifold; the experiments of Sec. VI train an RBF-kernel SVM):
 *   IP_KERNEL_POLY: f(x) = sum_{i<n_sv} alpha_i (gamma <sv_i, x> + coef0)^degree + bias
 *   IP_KERNEL_RBF:  f(x) = sum_{i<n_sv} alpha_i exp(-gamma |x - sv_i|^2) + bias
 * The FP64 value is defined by this evaluation order: x from the lattice
 * (see ip_space), then for i = 0..n_sv-1 in order:
 *   POLY: dot = fma chain over j = 0..d-1 of sv_ij * x_j starting at 0;
 *         t = fma(gamma, dot, coef0); t^degree by repeated multiplication;
 *         acc = fma(alpha_i, t^degree, acc);
 *   RBF:  d2 = fma chain over j of (x_j - sv_ij)^2 starting at 0;
 *         acc = fma(alpha_i, E(-(gamma * d2)), acc), with E the library's
 *         own exponential: 0 below -708, else k = floor(t / ln2 + 0.5),
 *         r = t - k ln2 (two fma with ln2 split in two parts), the Taylor
 *         polynomial of degree 13 in Horner form, times 2^k;
 * finally f = acc + bias.  Sign bit s = !(f < 0). */
enum { IP_KERNEL_POLY = 0, IP_KERNEL_RBF = 1 };
typedef struct {
  int32_t d;             /* ambient dimension, 2..IP_MAX_D */
  int32_t degree;        /* >= 1 (POLY; ignored for RBF) */
  int64_t n_sv;          /* >= 1 */
  double gamma, coef0, bias;   /* gamma > 0 for RBF; coef0 ignored for RBF */
  const double *sv;      /* host, n_sv x d */
  const double *alpha;   /* host, n_sv */
  int32_t kernel;        /* IP_KERNEL_POLY or IP_KERNEL_RBF */
} ip_fparams;

/* Coxeter triangulation frame and domain (Sec. IV-B, V-A).  Lattice vertex
 * v in Z^d has coordinates x_j = offset_j + sum_k M[j][k] v_k (fma chain over
 * k from offset_j).  Simplices are Kuhn simplices of Z^d (vertex + ordered
 * partition), so M fixes the scale lambda and the Coxeter shape.  Minv is
 * used for point location.  The domain is the closed box [lo, hi]; an edge is
 * traced only if both endpoints lie in it. */
typedef struct {
  int32_t d;
  const double *M;       /* host, d x d */
  const double *Minv;    /* host, d x d */
  const double *offset;  /* host, d */
  const double *lo;      /* host, d */
  const double *hi;      /* host, d */
} ip_space;

/* Robot and obstacles for the batch collision check (Sec. V-C, Appendix A).
 * Serial revolute robot: T_i = T_{i-1} * J_i * Rot(axis_i, q_i), T_{-1} = I,
 * with 3x4 row-major [R|t] transforms.  Robot geometry is given in link
 * frames (spheres, and capsules = segments with a radius); obstacles are
 * world-frame spheres, boxes (pose world-from-box, full extents) and
 * cylinders (pose world-from-cylinder with the axis on local z and the
 * origin at its centre; radius and height).  Capsules are tested against
 * obstacle spheres only: capsule-vs-box and capsule-vs-cylinder pairs are
 * not defined (IP_EINVAL).  Touching collides.  Sphere vs cylinder follows
 * Appendix A with its square roots squared away: in the cylinder frame,
 * folded into the first octant, rho2 = p_x^2 + p_y^2 and g = p_z - h/2; no
 * collision if g > r or rho2 > (r + rc)^2; in the ring region (g > 0 and
 * rho2 > rc^2) no collision if L = (rho2 - rc^2) - (r^2 - g^2) > 0 and
 * L^2 > 4 rc^2 (r^2 - g^2); else collision. */
typedef struct {
  int32_t n_joints;            /* equals d of the configurations */
  const double *joint_T;       /* host, n_joints x 12 */
  const int32_t *joint_axis;   /* host, n_joints, 0=x 1=y 2=z */
  int32_t n_lsph;
  const int32_t *lsph_link;    /* host */
  const double *lsph_c;        /* host, x3 */
  const double *lsph_r;
  int32_t n_lcap;
  const int32_t *lcap_link;
  const double *lcap_p0;       /* x3 */
  const double *lcap_p1;       /* x3 */
  const double *lcap_r;
  int32_t n_osph;
  const double *osph_c;        /* x3 */
  const double *osph_r;
  int32_t n_obox;
  const double *obox_T;        /* x12 */
  const double *obox_l;        /* x3 */
  int32_t n_ocyl;
  const double *ocyl_T;        /* x12 */
  const double *ocyl_rh;       /* x2: radius, height */
} ip_scene;

typedef struct {
  int64_t n_cells;       /* traced edges (1-simplices) = intersection points */
  int64_t n_vertices;    /* lattice vertices whose f was evaluated: unique
                            vertices, except in the FP32-certified batch
                            mode, which evaluates each template point of
                            each coarse simplex (in the box) once */
  int64_t n_fallback;    /* vertices whose sign the FP32 and FP64 monomial
                            bounds left open: canonical FP64 evaluations
                            (IP_FP32_CERTIFY), plus ends of edges whose point
                            needed them */
  int64_t n_settled64;   /* vertices the FP32 bound left open and the FP64
                            monomial evaluation settled (IP_FP32_CERTIFY) */
  int64_t n_cofaces;     /* 2-simplex cofaces expanded by the search */
  int64_t n_sigma;       /* coarse n-simplices (batch triangulation) */
  int64_t n_batches;     /* batches of coarse n-simplices */
  int64_t n_template_edges; /* fine edges tested in batch mode */
  int32_t levels;        /* breadth-first levels of the search */
  int32_t regrows;       /* hash-table growths */
  double ms_total;       /* wall time of ip_trace on the stream */
  double ms_feval;       /* time in f-evaluation kernels (HIP events) */
  double ms_expand;      /* time in frontier-expansion kernels */
  double ms_points;      /* time in the intersection-point kernel */
  double ms_check;       /* time in the collision kernel (ip_check_cells) */
  double ms_subdivide;   /* batch mode: time in the subdivision kernel
                            (sign codes of the template points of each coarse
                            simplex, template edge tests, edge-set inserts) */
  int64_t subdivide_launches; /* launches that ms_subdivide covers */
  int64_t n_edge_hits;   /* batch mode: intersecting (coarse simplex, template
                            edge) pairs, duplicates across simplices included */
  int64_t n_coarse_edges; /* batch mode: intersecting edges of the coarse trace */
  int64_t n_shared_probes; /* batch mode: intersecting template edges on a coarse
                              face with no traced coarse edge, which go through
                              the global edge set (all others are emitted once,
                              by the canonical coarse simplex of their face) */
  double ms_sigma;       /* batch mode: time in the coarse n-simplex kernel */
  int64_t n_ncofaces;    /* batch mode: n-simplex cofaces of the coarse edges
                            (with repeats), the probes of that kernel */
  int64_t n_hip_malloc;  /* device allocations of the call that missed the
                            context's cache and reached hipMalloc */
  int64_t hip_malloc_bytes; /* their bytes */
  double ms_refine;      /* time in the iterative intersection kernel */
  int32_t refine_iters;  /* its iterations per edge (flags of ip_trace) */
  int32_t pad0;
  double ms_prep;        /* batch mode: time in the per-coarse-simplex
                            preparation (traced coarse edges among its
                            vertices, tier-1 bound of its template points) */
} ip_stats;

/* Create a context on HIP device `device`; work is issued on `hip_stream`
 * (a hipStream_t; NULL = the null stream).  The context keeps device
 * workspace between calls. */
int ip_create(ip_ctx **ctx, int device, void *hip_stream);
void ip_destroy(ip_ctx *ctx);
const char *ip_last_error(const ip_ctx *ctx);

/* Upload one proof problem: manifold, frame/domain and seed points (host,
 * n_seeds x d; points on or near f = 0, Sec. V-A).  coarse_k = 1 traces
 * directly at the frame's scale; coarse_k >= 2 uses batch triangulation
 * (Sec. V-B): trace on the lattice coarsened by k, then subdivide every
 * n-simplex coface of the coarse edges by k.  IP_ERANGE if the domain's
 * lattice coordinates do not fit the keys. */
int ip_problem_create(ip_ctx *ctx, const ip_fparams *f, const ip_space *sp,
                      const double *seeds, int64_t n_seeds, int32_t coarse_k,
                      ip_problem **out);
void ip_problem_free(ip_problem *p);

/* Trace (Sec. V-A locate + breadth-first search; Sec. V-B batches).
 * batch_budget_bytes bounds the per-batch device workspace in batch mode
 * (0 = library default); the traced set does not depend on it.  In the
 * FP32-certified mode with a polynomial kernel a batch takes
 * 12 + 16 ceil(2^(d+1) / 64) bytes per coarse simplex (a deferred-list entry,
 * its tier-1 bound and two face masks); in the other modes the vertex table
 * of the batch's template points sets the size.
 * precision: IP_FP64 or IP_FP32_CERTIFY.  flags: IP_REFINE(n) or 0.
 * The result holds the traced edges and their intersection points
 * p = x_a + t (x_b - x_a), t = f_a / (f_a - f_b), a the smaller endpoint.
 * With IP_REFINE(n), n = 1..15, the points are computed iteratively instead
 * (Sec. V-B; Sec. VI: refined until a desired accuracy): n false-position
 * steps with the Illinois modification on the bracket [a, b]: m_j =
 * fma(t, x_b,j - x_a,j, x_a,j) with t as above, f at m (canonical FP64 order
 * in IP_FP64 mode, the FP64 monomial form in IP_FP32_CERTIFY mode), the end
 * whose sign bit !(f < 0) equals that of f(m) moves to m, and the value kept
 * at the other end is halved when the same end moved twice in a row; the
 * point is the false-position point of the final bracket. */
#define IP_REFINE(n) (((uint32_t)(n) & 15u) << 4)
int ip_trace(ip_ctx *ctx, const ip_problem *p, uint64_t batch_budget_bytes,
             int32_t precision, uint32_t flags, ip_cells **out);

/* The traced cells (Sec. V-A: the output of the trace is the set of
 * intersecting edges with their intersection points, one cell each; Sec.
 * V-B: the same set built batch by batch).  Count and statistics: */
int64_t ip_cells_count(const ip_cells *c);
int ip_cells_stats(const ip_cells *c, ip_stats *out);
/* Copy cells to host buffers (any may be NULL): v (n x d int32, smaller
 * endpoint), mask (n, endpoint b = v + sum_{j in mask} e_j), pts (n x d).
 * ctx may be NULL: the context that traced the cells is used. */
int ip_cells_download(ip_ctx *ctx, const ip_cells *c, int32_t *v, uint32_t *mask,
                      double *pts);
/* Device view of the intersection points: SoA, pts[j * ld + i]. */
int ip_cells_points(const ip_cells *c, const double **pts_dev, int64_t *ld);
/* Order-independent digest of the traced set: digest[0] = sum and
 * digest[1] = xor, over the cells, of the SplitMix64 finalizer of the packed
 * edge key (the set is unique, its order is not).  Device-side; two 8-byte
 * host outputs.  The packed key of cell (v, mask) is
 *   sum_j (v_j - vmin_j) << (j * bits)  |  mask << (d * bits)
 * with bits and vmin from ip_cells_key_layout; the finalizer is
 * z ^= z >> 30; z *= 0xbf58476d1ce4e5b9; z ^= z >> 27; z *= 0x94d049bb133111eb;
 * z ^= z >> 31 (mod 2^64). */
int ip_cells_digest(ip_ctx *ctx, const ip_cells *c, uint64_t digest[2]);
/* Key layout of the cells (host outputs): bits per coordinate and vmin (d
 * int32), fixed by the domain box and the lattice frame. */
int ip_cells_key_layout(const ip_cells *c, int32_t *bits, int32_t *vmin);
/* Copy rows idx[0 .. n) (host array, each in [0, count)) of the cells to the
 * host: vertex v (n x d), mask, point (n x d, row-major) and, once
 * ip_check_cells has run, the verdict.  Any output may be NULL.  An index out
 * of range, or a verdict request before the check, is IP_EINVAL. */
int ip_cells_gather(ip_ctx *ctx, const ip_cells *c, const int64_t *idx, int64_t n, int32_t *v, uint32_t *mask,
                    double *pts, uint8_t *verdict);
void ip_cells_free(ip_cells *c);

/* Collision verdicts for n configurations (Sec. V-C).  q_dev: device SoA,
 * q[j * ld + i], j < n_joints.  verdict_dev: device, n bytes, 1 = collision.
 * Evaluated in FP64 in a fixed operation order (own sine/cosine). */
int ip_check(ip_ctx *ctx, const ip_scene *scene, const double *q_dev, int64_t n,
             int64_t ld, uint8_t *verdict_dev);

/* Check the cells' points, keep the verdicts on the device and gather the
 * free (verdict 0) points (Sec. V-B: only C_free points go back to the
 * host).  *n_free receives their count. */
int ip_check_cells(ip_ctx *ctx, ip_cells *c, const ip_scene *scene, int64_t *n_free);
/* Batch by batch, the way the paper's batch stage runs (Sec. V-B, Fig. 6:
 * each batch's cells get their intersection points, are checked, and only
 * the C_free points go to the host before the batch's memory is reused).
 * Needs batch triangulation (coarse_k >= 2) and a scene; precision and
 * flags as for ip_trace.  For each batch, on the calling thread and in batch
 * order, fn(user, batch, free_pts, n_free, n_cells) receives the batch's
 * C_free points (host, row-major n_free x d, page-locked, valid until fn
 * returns) and its cell count; a nonzero return stops the trace with
 * IP_ECANCELED.  A batch's copy to the host runs on a second stream while
 * the next batch is traced, so its callback comes once that copy has landed
 * (at the latest when the call returns).  fn may be NULL (counts and digest
 * only).  The union over the batches is exactly
 * the set that ip_trace + ip_check_cells give (each cell once, in another
 * order).  batch_budget_bytes sizes a batch by its workspace plus its
 * projected output, (9 + 24 d) bytes per projected cell (key, points,
 * verdict, free-point copy and staging); the projection is 1.6 nc k^(d-1)
 * cells over |Sigma| per coarse simplex (nc: coarse crossing edges), so a
 * batch's memory is bounded by the budget up to the projection's error
 * (over-full batches grow their buffers and go on).  What stays resident
 * across batches: Sigma, the coarse trace and the global set of the edges
 * on shared coarse faces (8 bytes per such edge plus its table slots).
 * *out receives totals: cells, free points, batches, the digest of the
 * traced set (as ip_cells_digest) and the statistics. */
typedef int (*ip_batch_fn)(void *user, int64_t batch, const double *free_pts, int64_t n_free, int64_t n_cells);
typedef struct {
  int64_t n_cells;
  int64_t n_free;
  int64_t batches;
  uint64_t digest[2];
  ip_stats stats;
} ip_batch_summary;
int ip_trace_check_batches(ip_ctx *ctx, const ip_problem *p, uint64_t batch_budget_bytes, int32_t precision,
                           uint32_t flags, const ip_scene *scene, ip_batch_fn fn, void *user,
                           ip_batch_summary *out);

/* Host copies of the verdicts (n bytes) and free points (row-major
 * n_free x d, interleaved on the device and copied once).  Either pointer
 * may be NULL.  Waits for the context's stream. */
int ip_cells_download_check(ip_ctx *ctx, const ip_cells *c, uint8_t *verdict,
                            double *free_pts);
/* The free points to the host as they lie on the device, one column per
 * coordinate (free_soa[j * n_free + i]): d copies, no host-side transpose,
 * so that pinned host memory (hipHostMalloc) receives them at the link's
 * rate (Sec. V-B: only the C_free points go back to the host). */
int ip_cells_download_free(ip_ctx *ctx, const ip_cells *c, double *free_soa);

/* f at lattice vertices (Sec. V-A: the manifold's value at the vertices of
 * the triangulation decides which edges intersect; device v_dev: n x d
 * int32 -> device f_dev: n).
 * IP_FP64: canonical FP64.  IP_FP32_CERTIFY: FP32 with the bound, FP64 for
 * the vertices the bound cannot settle; bound_dev (may be NULL) receives the
 * bound used (0 for FP64 results). */
int ip_feval(ip_ctx *ctx, const ip_problem *p, const int32_t *v_dev, int64_t n,
             int32_t precision, double *f_dev, double *bound_dev);

/* Seeds (Sec. V-A: the seeds are points on the manifold found by a
 * nonlinear program that minimises |f| from a given configuration): from
 * each start q0 (device, n x d row-major), `iters` (0..1000) minimum-norm
 * Newton steps on f in FP64,
 *   g = grad f(q) and f(q) in the canonical order of ip_fparams, with
 *     POLY: w_i = (alpha_i t_i^(p-1)) (p gamma), g_j = fma chain of w_i s_ij;
 *     RBF:  w_i = (alpha_i e_i) (-2 gamma),    g_j = fma chain of w_i (q_j - s_ij);
 *   n2 = fma chain of g_j^2; a zero n2 ends the steps; c = f / n2;
 *   q_j = fma(-c, g_j, q_j), then clamped into the domain box;
 * then q_dev (n x d) receives the final points and f_dev (n) f there.  The
 * caller keeps the points with |f| small enough as seeds. */
int ip_seed_search(ip_ctx *ctx, const ip_problem *p, const double *q0_dev, int64_t n, int32_t iters,
                   double *q_dev, double *f_dev);
/* Replace the problem's seeds (host, n_seeds x d, copied). */
int ip_problem_set_seeds(ip_ctx *ctx, ip_problem *p, const double *seeds, int64_t n_seeds);

/* The first certified tier of batch subdivision (Sec. V-B, Eq. 1-2 with the
 * FP32 certification), on given coarse simplices, for inspection: the fused
 * subdivision evaluates each template point of a coarse simplex (v, w) in
 * FP32 (nested monomial form) and settles its sign when |f32| exceeds one
 * bound per simplex, B1 + B64, formed from the largest |x_j| over the
 * simplex's vertices.  simplex_dev: device, n x 2d int32 rows (coarse vertex
 * v, then the coordinate order w, a permutation of 0..d-1).  Outputs
 * (device): y_dev n x NP x d int32 (fine vertex of template point t of
 * simplex s: y_{w_i} = k v_{w_i} + u_i), f_dev n x NP (the FP32 value, NaN
 * outside the box), bound_dev n (B1 + B64).  *n_points receives NP =
 * C(d + k, d); with y_dev NULL only NP is returned.  k is the problem's
 * coarse_k.  IP_EINVAL when the degree has no FP32 form (above 4). */
int ip_region_eval(ip_ctx *ctx, const ip_problem *p, const int32_t *simplex_dev, int64_t n,
                   int32_t *y_dev, double *f_dev, double *bound_dev, int32_t *n_points);

/* The same evaluation for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  It calls no hipMalloc, hipFree or allocating library routine
 * and never waits for the device: the FP64 fallback list and its counters
 * live in a fixed device scratch array of 256 + 4 * IP_NOALLOC_MAX_VERTICES
 * bytes (4 MiB), one per device, held until the process ends.  n above
 * IP_NOALLOC_MAX_VERTICES is IP_EINVAL.  Arguments and results are those of
 * ip_feval (bound_dev may be NULL); the work is queued on the context's
 * stream.  Every call on one device shares that device's scratch, which
 * keeps the last call's contents (the call clears its counters itself):
 * calls that overlap on one device (two streams, or two host threads) race,
 * so serialise them. */
#define IP_NOALLOC_MAX_VERTICES 1048576
int ip_feval_noalloc(ip_ctx *ctx, const ip_problem *p, const int32_t *v_dev, int64_t n,
                     int32_t precision, double *f_dev, double *bound_dev);

/* ------------------------------------------------------------------------
 * Serving loop (the proof requests of the planning loop, Sec. IV-A / Fig. 1:
 * each retraining of the manifold produces a new trace + check request).
 * A server owns max_slots slots, each a context with its own HIP stream and
 * workspace, and one host thread per slot.  Requests queue in arrival order
 * and join as slots free up.  A request that takes a slot first projects its
 * own device bytes: it traces its manifold on a coarsened lattice (its own
 * coarse lattice in batch mode, the fine one coarsened by 4 otherwise); with
 * nc crossing edges there and coarsening kc, about N = 1.25 nc kc^(d-1) fine
 * cells, projected at N (8 + 16 d + 57) bytes + 64 MiB.  It starts its
 * trace once that projection plus those of the requests already tracing fits
 * pool_bytes (a request larger than the pool runs when nothing else
 * traces); a request's caller can give mem_bytes instead.  Admitted requests
 * run concurrently on their streams, so their kernels overlap on the device;
 * a request's result does not depend on what else runs.  Each slot's idle
 * device cache is limited to pool_bytes / max_slots.
 * ------------------------------------------------------------------------ */
typedef struct ip_server ip_server;

enum { IP_KEEP_CELLS = 1 };  /* request flag: keep the traced cells in the result */

typedef struct {
  const ip_fparams *f;       /* host, copied by ip_server_submit */
  const ip_space *sp;        /* host, copied */
  const double *seeds;       /* host, n_seeds x d, copied */
  int64_t n_seeds;
  int32_t coarse_k;
  int32_t precision;         /* IP_FP64 or IP_FP32_CERTIFY */
  const ip_scene *scene;     /* host, copied; NULL = trace only */
  uint64_t batch_budget;     /* as for ip_trace */
  uint64_t mem_bytes;        /* device bytes to admit the request by; 0 = the
                                library's projection (above) */
  uint32_t flags;            /* IP_KEEP_CELLS, and IP_REFINE(n) for ip_trace */
} ip_request;

typedef struct {
  int32_t status;            /* IP_OK or the error code of the request */
  int32_t d;
  ip_stats stats;
  int64_t n_cells;
  int64_t n_free;
  uint64_t digest[2];        /* order-independent digest of the traced edge keys:
                                sum and xor of SplitMix64(key), mod 2^64 */
  double t_submit, t_start, t_done;  /* seconds, server's monotonic clock */
  double *free_pts;          /* host, n_free x d (NULL without a scene):
                                page-locked memory from the server's pool,
                                which ip_result_free returns there */
  ip_cells *cells;           /* with IP_KEEP_CELLS; download with ctx = NULL */
  char error[160];
  uint64_t admitted_bytes;   /* the projection (or mem_bytes) it was admitted by */
  int64_t n_probe_edges;     /* crossing edges of the projection trace (0 with mem_bytes) */
  double t_admit;            /* when its trace was admitted (server clock) */
} ip_result;

int ip_server_create(ip_server **out, int device, uint64_t pool_bytes, int32_t max_slots);
/* Queue a request; *id identifies it.  Inputs are copied before return. */
int ip_server_submit(ip_server *s, const ip_request *req, uint64_t *id);
/* IP_EAGAIN while the request is queued or running; then the result, which
 * the caller releases with ip_result_free.  Each result is returned once. */
int ip_server_poll(ip_server *s, uint64_t id, ip_result **out);
int ip_server_wait(ip_server *s, uint64_t id, ip_result **out);
void ip_result_free(ip_result *r);
/* Waits for running requests, drops queued ones.  Results must be freed
 * before their server is destroyed. */
void ip_server_destroy(ip_server *s);
/* Seconds on the server's clock (for arrival schedules). */
double ip_server_clock(const ip_server *s);

#ifdef __cplusplus
}
#endif
#endif
