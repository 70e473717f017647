// Batch collision checking of traced cells (Sec. V-C, Appendix A).
//
// One lane per configuration: forward kinematics link by link (only the
// current 3x4 transform is live), each link's spheres / capsules tested
// against every obstacle as soon as its frame is known, early exit on the
// first hit.  The scene is small and read with wave-uniform loads.
//
// Verdicts are decided in FP64 with a fixed operation order (fma only where
// written, own sine/cosine: Cody-Waite reduction by pi/2 and Taylor
// polynomials), so they are reproducible bit for bit on any IEEE-754 FP64
// implementation that follows the same order.
#include <cstring>
#include <vector>

#include "ip_internal.h"

namespace {

struct SceneDev {
  int32_t nj;
  int32_t has_box;
  const double *joint_T;      // nj x 12
  const int32_t *joint_axis;  // nj
  const int32_t *lsph_off;    // nj + 1
  const double *lsph;         // [cx cy cz r] per sphere, grouped by link
  const int32_t *lcap_off;    // nj + 1
  const double *lcap;         // [p0 p1 r pad] (8 doubles) per capsule, by link
  int32_t n_osph, n_obox;
  const double *osph;         // [cx cy cz r]
  const double *obox;         // [T(12) l(3) pad] (16 doubles)
};

#define PIO2_A 1.5707963267341256
#define PIO2_B 6.077100506303966e-11
#define PIO2_C 2.0222662487959506e-21
#define TWO_OVER_PI 0.6366197723675814

__device__ void sincos_own(double q, double *s, double *c) {
  double kf = floor(q * TWO_OVER_PI + 0.5);
  double r = fma(-kf, PIO2_A, q);
  r = fma(-kf, PIO2_B, r);
  r = fma(-kf, PIO2_C, r);
  double z = r * r;
  double ps = 2.8114572543455206e-15;
  ps = fma(z, ps, -7.647163731819816e-13);
  ps = fma(z, ps, 1.6059043836821613e-10);
  ps = fma(z, ps, -2.505210838544172e-08);
  ps = fma(z, ps, 2.7557319223985893e-06);
  ps = fma(z, ps, -0.0001984126984126984);
  ps = fma(z, ps, 0.008333333333333333);
  ps = fma(z, ps, -0.16666666666666666);
  double sr = fma(r * z, ps, r);
  double pc = 4.779477332387385e-14;
  pc = fma(z, pc, -1.1470745597729725e-11);
  pc = fma(z, pc, 2.08767569878681e-09);
  pc = fma(z, pc, -2.755731922398589e-07);
  pc = fma(z, pc, 2.48015873015873e-05);
  pc = fma(z, pc, -0.001388888888888889);
  pc = fma(z, pc, 0.041666666666666664);
  pc = fma(z, pc, -0.5);
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

// C = A * B for 3x4 row-major affine transforms.
__device__ __forceinline__ void compose(const double *A, const double *B, double *C) {
#pragma unroll
  for (int r = 0; r < 3; ++r) {
#pragma unroll
    for (int c = 0; c < 3; ++c)
      C[r * 4 + c] = fma(A[r * 4 + 2], B[8 + c], fma(A[r * 4 + 1], B[4 + c], A[r * 4 + 0] * B[c]));
    C[r * 4 + 3] = fma(A[r * 4 + 2], B[11], fma(A[r * 4 + 1], B[7], fma(A[r * 4 + 0], B[3], A[r * 4 + 3])));
  }
}

__device__ __forceinline__ void rotation(int axis, double s, double c, double *R) {
#pragma unroll
  for (int i = 0; i < 12; ++i) R[i] = 0.0;
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

__device__ __forceinline__ void xform(const double *T, const double *p, double *o) {
#pragma unroll
  for (int r = 0; r < 3; ++r)
    o[r] = fma(T[r * 4 + 2], p[2], fma(T[r * 4 + 1], p[1], fma(T[r * 4 + 0], p[0], T[r * 4 + 3])));
}

__device__ __forceinline__ double sq3(double x, double y, double z) { return fma(z, z, fma(y, y, x * x)); }

__device__ __forceinline__ bool sphere_sphere(const double *a, double ra, const double *b, double rb) {
  double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
  double rr = ra + rb;
  return sq3(dx, dy, dz) <= rr * rr;
}

__device__ __forceinline__ bool capsule_sphere(const double *p0, const double *p1, double rc, const double *c,
                                               double rs) {
  double u[3], w[3], e[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    u[j] = p1[j] - p0[j];
    w[j] = c[j] - p0[j];
  }
  double uu = fma(u[2], u[2], fma(u[1], u[1], u[0] * u[0]));
  double wu = fma(w[2], u[2], fma(w[1], u[1], w[0] * u[0]));
  double t = uu > 0.0 ? wu / uu : 0.0;
  t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
#pragma unroll
  for (int j = 0; j < 3; ++j) e[j] = fma(-t, u[j], w[j]);
  double rr = rc + rs;
  return sq3(e[0], e[1], e[2]) <= rr * rr;
}

// Appendix A, sphere vs box: centre into the box frame, fold into the first
// octant, (1) padded bounding test (Eq. 3), (2) edge region (Eq. 4-5),
// (3) vertex region (Eq. 6-7); any other case collides.
__device__ __forceinline__ bool sphere_box(const double *c, double r, const double *B) {
  const double dx = c[0] - B[3], dy = c[1] - B[7], dz = c[2] - B[11];
  double g[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    double p = fabs(fma(B[8 + i], dz, fma(B[4 + i], dy, B[i] * dx)));
    g[i] = p - 0.5 * B[12 + i];
  }
  if (g[0] > r || g[1] > r || g[2] > r) return false;
  const int nout = (g[0] > 0.0) + (g[1] > 0.0) + (g[2] > 0.0);
  if (nout == 2) {
    double a, b;
    if (!(g[0] > 0.0)) {
      a = g[1];
      b = g[2];
    } else if (!(g[1] > 0.0)) {
      a = g[0];
      b = g[2];
    } else {
      a = g[0];
      b = g[1];
    }
    return !(fma(b, b, a * a) > r * r);
  }
  if (nout == 3) return !(sq3(g[0], g[1], g[2]) > r * r);
  return true;
}

// One lane per configuration.  GATHER: the free configurations (verdict 0)
// are also appended to free_pts (SoA, column stride ld_free) through per-wave
// LDS staging, one atomic per 128 free points, while their columns are still
// in cache.
template <bool GATHER>
__global__ __launch_bounds__(256) void check_kernel(SceneDev S, const double *__restrict__ q, int64_t n, int64_t ld,
                                                    uint8_t *__restrict__ verdict, double *free_pts,
                                                    int64_t ld_free, unsigned long long *count) {
  constexpr int kStage = 128;
  __shared__ uint32_t st[GATHER ? 4 : 1][GATHER ? kStage : 1];
  const int wib = threadIdx.x >> 6;
  int sn = 0;
  const int d = S.nj;
  auto put = [&](unsigned long long pos, uint32_t i) {
    for (int j = 0; j < d; ++j) free_pts[(int64_t)j * ld_free + (int64_t)pos] = q[(int64_t)j * ld + (int64_t)i];
  };
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t start = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t rounds = (n + stride - 1) / stride;
  for (int64_t it = 0; it < rounds; ++it) {
    const int64_t i = start + it * stride;
    bool hit = false;
    if (i < n) {
      double T[12] = {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0};
      for (int li = 0; li < S.nj && !hit; ++li) {
        double s, c, A[12], R[12];
        sincos_own(q[(int64_t)li * ld + i], &s, &c);
        compose(T, S.joint_T + 12 * li, A);
        rotation(S.joint_axis[li], s, c, R);
        compose(A, R, T);
        for (int a = S.lsph_off[li]; a < S.lsph_off[li + 1] && !hit; ++a) {
          const double *sp = S.lsph + 4 * a;
          double cw[3];
          xform(T, sp, cw);
          for (int b = 0; b < S.n_osph && !hit; ++b) hit = sphere_sphere(cw, sp[3], S.osph + 4 * b, S.osph[4 * b + 3]);
          for (int b = 0; b < S.n_obox && !hit; ++b) hit = sphere_box(cw, sp[3], S.obox + 16 * b);
        }
        for (int a = S.lcap_off[li]; a < S.lcap_off[li + 1] && !hit; ++a) {
          const double *cp = S.lcap + 8 * a;
          double p0[3], p1[3];
          xform(T, cp, p0);
          xform(T, cp + 3, p1);
          for (int b = 0; b < S.n_osph && !hit; ++b)
            hit = capsule_sphere(p0, p1, cp[6], S.osph + 4 * b, S.osph[4 * b + 3]);
        }
      }
      verdict[i] = hit ? 1 : 0;
    }
    if (GATHER) stage_put<kStage>(st[wib], sn, i < n && !hit, (uint32_t)i, put, count);
  }
  if (GATHER) stage_flush(st[wib], sn, put, count);
}

int upload_scene(ip_ctx *ctx, const ip_scene *sc, SceneDev *out) {
  const int nj = sc->n_joints;
  if (nj < 1 || nj > IP_MAX_D) return ip_fail(ctx, IP_EINVAL, "scene: joint count out of range");
  if (sc->n_lcap > 0 && sc->n_obox > 0) return ip_fail(ctx, IP_EINVAL, "scene: capsule-vs-box pairs are not defined");
  if (sc->n_lsph < 0 || sc->n_lcap < 0 || sc->n_osph < 0 || sc->n_obox < 0)
    return ip_fail(ctx, IP_EINVAL, "scene: negative counts");
  for (int i = 0; i < nj; ++i)
    if (sc->joint_axis[i] < 0 || sc->joint_axis[i] > 2) return ip_fail(ctx, IP_EINVAL, "scene: axis must be 0..2");
  // group robot geometry by link (stable)
  std::vector<int32_t> lsph_off(nj + 1, 0), lcap_off(nj + 1, 0);
  for (int a = 0; a < sc->n_lsph; ++a) {
    int l = sc->lsph_link[a];
    if (l < 0 || l >= nj) return ip_fail(ctx, IP_EINVAL, "scene: sphere link index out of range");
    ++lsph_off[l + 1];
  }
  for (int a = 0; a < sc->n_lcap; ++a) {
    int l = sc->lcap_link[a];
    if (l < 0 || l >= nj) return ip_fail(ctx, IP_EINVAL, "scene: capsule link index out of range");
    ++lcap_off[l + 1];
  }
  for (int i = 0; i < nj; ++i) {
    lsph_off[i + 1] += lsph_off[i];
    lcap_off[i + 1] += lcap_off[i];
  }
  std::vector<double> lsph(4 * (size_t)sc->n_lsph), lcap(8 * (size_t)sc->n_lcap);
  {
    std::vector<int32_t> fill = lsph_off;
    for (int a = 0; a < sc->n_lsph; ++a) {
      int pos = fill[sc->lsph_link[a]]++;
      for (int j = 0; j < 3; ++j) lsph[4 * pos + j] = sc->lsph_c[3 * a + j];
      lsph[4 * pos + 3] = sc->lsph_r[a];
    }
    fill = lcap_off;
    for (int a = 0; a < sc->n_lcap; ++a) {
      int pos = fill[sc->lcap_link[a]]++;
      for (int j = 0; j < 3; ++j) {
        lcap[8 * pos + j] = sc->lcap_p0[3 * a + j];
        lcap[8 * pos + 3 + j] = sc->lcap_p1[3 * a + j];
      }
      lcap[8 * pos + 6] = sc->lcap_r[a];
      lcap[8 * pos + 7] = 0.0;
    }
  }
  std::vector<double> osph(4 * (size_t)sc->n_osph), obox(16 * (size_t)sc->n_obox);
  for (int b = 0; b < sc->n_osph; ++b) {
    for (int j = 0; j < 3; ++j) osph[4 * b + j] = sc->osph_c[3 * b + j];
    osph[4 * b + 3] = sc->osph_r[b];
  }
  for (int b = 0; b < sc->n_obox; ++b) {
    for (int j = 0; j < 12; ++j) obox[16 * b + j] = sc->obox_T[12 * b + j];
    for (int j = 0; j < 3; ++j) obox[16 * b + 12 + j] = sc->obox_l[3 * b + j];
    obox[16 * b + 15] = 0.0;
  }
  // one contiguous blob: doubles first, then ints
  std::vector<double> blob;
  auto put = [&](const double *p, size_t n) {
    size_t off = blob.size();
    blob.insert(blob.end(), p, p + n);
    return off;
  };
  size_t o_jT = put(sc->joint_T, 12 * (size_t)nj);
  size_t o_ls = put(lsph.data(), lsph.size());
  size_t o_lc = put(lcap.data(), lcap.size());
  size_t o_os = put(osph.data(), osph.size());
  size_t o_ob = put(obox.data(), obox.size());
  size_t n_dbl = blob.size();
  std::vector<int32_t> ints;
  ints.insert(ints.end(), sc->joint_axis, sc->joint_axis + nj);
  size_t o_lso = ints.size();
  ints.insert(ints.end(), lsph_off.begin(), lsph_off.end());
  size_t o_lco = ints.size();
  ints.insert(ints.end(), lcap_off.begin(), lcap_off.end());
  size_t bytes = n_dbl * 8 + ints.size() * 4;
  IP_TRY(ip_ensure(ctx, ctx->scene, bytes));
  char *base = (char *)ctx->scene.p;
  IP_TRY_HIP(ctx, hipMemcpyAsync(base, blob.data(), n_dbl * 8, hipMemcpyHostToDevice, ctx->stream));
  IP_TRY_HIP(ctx, hipMemcpyAsync(base + n_dbl * 8, ints.data(), ints.size() * 4, hipMemcpyHostToDevice, ctx->stream));
  IP_TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));
  const double *db = (const double *)base;
  const int32_t *ib = (const int32_t *)(base + n_dbl * 8);
  out->nj = nj;
  out->has_box = sc->n_obox > 0;
  out->joint_T = db + o_jT;
  out->joint_axis = ib;
  out->lsph_off = ib + o_lso;
  out->lsph = db + o_ls;
  out->lcap_off = ib + o_lco;
  out->lcap = db + o_lc;
  out->n_osph = sc->n_osph;
  out->n_obox = sc->n_obox;
  out->osph = db + o_os;
  out->obox = db + o_ob;
  return IP_OK;
}

}  // namespace

int ip_check_impl(ip_ctx *ctx, const ip_scene *scene, const double *q_dev, int64_t n, int64_t ld,
                  uint8_t *verdict_dev) {
  SceneDev S;
  IP_TRY(upload_scene(ctx, scene, &S));
  if (n == 0) return IP_OK;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(check_kernel<false>, dim3((unsigned)blocks), dim3(256), 0, ctx->stream, S, q_dev, n, ld,
                     verdict_dev, (double *)nullptr, (int64_t)0, (unsigned long long *)nullptr);
  IP_TRY_HIP(ctx, hipGetLastError());
  return IP_OK;
}

// Verdicts of every cell plus the compaction of the free points, in one
// pass over the points.
int ip_check_gather_impl(ip_ctx *ctx, const ip_scene *scene, ip_cells *c) {
  SceneDev S;
  IP_TRY(upload_scene(ctx, scene, &S));
  if (c->free_pts) {
    ip_dfree(ctx, c->free_pts);
    c->free_pts = nullptr;
  }
  const int64_t n = c->n;
  if (n >= (1ll << 32)) return ip_fail(ctx, IP_EINVAL, "more than 2^32 cells in one check");
  IP_TRY(ip_dalloc(ctx, (void **)&c->free_pts, sizeof(double) * (size_t)(n ? n : 1) * c->d));
  IP_TRY_HIP(ctx, hipMemsetAsync(ctx->ctr_dev, 0, sizeof(Counters), ctx->stream));
  IP_TRY_HIP(ctx, hipEventRecord(ctx->ev0, ctx->stream));
  if (n) {
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(check_kernel<true>, dim3((unsigned)blocks), dim3(256), 0, ctx->stream, S, (const double *)c->pts,
                       n, c->ld, c->verdict, c->free_pts, n, &ctx->ctr_dev->n_aux);
    IP_TRY_HIP(ctx, hipGetLastError());
  }
  IP_TRY_HIP(ctx, hipEventRecord(ctx->ev1, ctx->stream));
  IP_TRY_HIP(ctx, hipMemcpyAsync(ctx->ctr_host, ctx->ctr_dev, sizeof(Counters), hipMemcpyDeviceToHost, ctx->stream));
  IP_TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));
  float ms = 0.0f;
  IP_TRY_HIP(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
  c->st.ms_check = ms;
  c->n_free = (int64_t)ctx->ctr_host->n_aux;
  return IP_OK;
}
