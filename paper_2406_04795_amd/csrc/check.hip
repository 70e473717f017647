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
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "ip_internal.h"

namespace {

struct SceneDev {
  int32_t nj;
  int32_t has_box;
  const double *joint_T;      // nj x 12
  const int32_t *joint_axis;  // nj
  const int32_t *joint_pure;  // nj: 1 when the joint's rotation part is exactly the identity
  const int32_t *lsph_off;    // nj + 1
  const double *lsph;         // [cx cy cz r] per sphere, grouped by link
  const int32_t *lcap_off;    // nj + 1
  const double *lcap;         // [p0 p1 r pad] (8 doubles) per capsule, by link
  int32_t n_osph, n_obox, n_ocyl, pad;
  const double *osph;         // [cx cy cz r]
  const double *obox;         // [T(12) l(3) rb] (16 doubles), rb: radius of a ball about the centre holding the box
  const double *ocyl;         // [T(12) rc h rb pad] (16 doubles), rb as for boxes
  const double *lbound;       // per link [cx cy cz R]: a ball in the link frame
                              // holding all of the link's geometry (R < 0: none)
  const double *cull;         // per link, per obstacle (spheres, boxes, cylinders, padded
                              // to a multiple of 4 with far ones) [ox oy oz t]: o the
                              // centre of a ball of radius rb holding the obstacle and
                              // t = (|o|^2 - (R + eps + rb)^2) / 2 with R the link's
                              // ball radius; the balls can meet only if c.o - |c|^2/2 >= t
  int32_t nobs_pad;           // obstacles per link row of cull
  double eps;                 // margin of the culling test
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

// One link of the forward kinematics, T <- T * J * R(axis, q), R the
// rotation by q about axis 0, 1 or 2 (x, y, z): the same values as the full
// 3x4 products compose(compose(T, J), R) with the products by the exact
// zeros and ones of R and of an identity rotation part of J (pure) left out
// (each left-out term adds an exact zero).
__device__ __forceinline__ void fk_step(double *T, const double *J, bool pure, int axis, double s, double c) {
  double A[12];
  if (pure) {
#pragma unroll
    for (int r = 0; r < 3; ++r) {
#pragma unroll
      for (int k = 0; k < 3; ++k) A[r * 4 + k] = T[r * 4 + k];
      A[r * 4 + 3] = fma(T[r * 4 + 2], J[11], fma(T[r * 4 + 1], J[7], fma(T[r * 4 + 0], J[3], T[r * 4 + 3])));
    }
  } else {
    compose(T, J, A);
  }
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const double a0 = A[r * 4 + 0], a1 = A[r * 4 + 1], a2 = A[r * 4 + 2];
    if (axis == 0) {
      T[r * 4 + 0] = a0;
      T[r * 4 + 1] = fma(a2, s, a1 * c);
      T[r * 4 + 2] = fma(a2, c, -(a1 * s));
    } else if (axis == 1) {
      T[r * 4 + 0] = fma(a2, -s, a0 * c);
      T[r * 4 + 1] = a1;
      T[r * 4 + 2] = fma(a2, c, a0 * s);
    } else {
      T[r * 4 + 0] = fma(a1, s, a0 * c);
      T[r * 4 + 1] = fma(a1, c, -(a0 * s));
      T[r * 4 + 2] = a2;
    }
    T[r * 4 + 3] = A[r * 4 + 3];
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

// Appendix A, sphere vs cylinder (axis z, origin at the centre): centre into
// the cylinder frame, fold into the first octant, (1) padded cylinder test,
// (2) ring region (rim) test with its square roots squared away: with
// q = r^2 - g^2, (rho - rc)^2 > q for rho > rc exactly when
// L = rho^2 - rc^2 - q > 0 and L^2 > 4 rc^2 q; anything else collides.
__device__ __forceinline__ bool sphere_cyl(const double *c, double r, const double *C) {
  const double dx = c[0] - C[3], dy = c[1] - C[7], dz = c[2] - C[11];
  double p[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) p[i] = fabs(fma(C[8 + i], dz, fma(C[4 + i], dy, C[i] * dx)));
  const double rc = C[12], h = C[13];
  const double rho2 = fma(p[1], p[1], p[0] * p[0]);
  const double g = p[2] - 0.5 * h;
  if (g > r) return false;
  const double rr = r + rc;
  if (rho2 > rr * rr) return false;
  if (g > 0.0 && rho2 > rc * rc) {
    const double q = r * r - g * g;
    const double L = (rho2 - rc * rc) - q;
    if (L > 0.0 && L * L > 4.0 * (rc * rc) * q) return false;
  }
  return true;
}

// Culling: can a ball (centre c, radius R) reach obstacle b?  A false
// answer proves that every sphere or capsule inside the ball misses the
// obstacle by more than the margin eps, far beyond the rounding of the exact
// predicates, so skipping their tests leaves every verdict unchanged.  Boxes
// and cylinders are first tested against a ball holding them (centre x,
// radius rb): farther than R + rb, the ball cannot reach them.
__device__ __forceinline__ bool ball_near_sphere(const double *c, double R, const double *o) {
  const double rr = R + o[3];
  return !(sq3(c[0] - o[0], c[1] - o[1], c[2] - o[2]) > rr * rr);
}

__device__ __forceinline__ bool ball_near_box(const double *c, double R, const double *B) {
  const double dx = c[0] - B[3], dy = c[1] - B[7], dz = c[2] - B[11];
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const double g = fabs(fma(B[8 + i], dz, fma(B[4 + i], dy, B[i] * dx))) - 0.5 * B[12 + i];
    if (g > 0.0) s = fma(g, g, s);
  }
  return !(s > R * R);
}

__device__ __forceinline__ bool ball_near_cyl(const double *c, double R, const double *C) {
  const double dx = c[0] - C[3], dy = c[1] - C[7], dz = c[2] - C[11];
  double p[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) p[i] = fabs(fma(C[8 + i], dz, fma(C[4 + i], dy, C[i] * dx)));
  const double gr = sqrt(fma(p[1], p[1], p[0] * p[0])) - C[12];
  const double gz = p[2] - 0.5 * C[13];
  double s = 0.0;
  if (gr > 0.0) s = gr * gr;
  if (gz > 0.0) s = fma(gz, gz, s);
  return !(s > R * R);
}

// OR over the wave, returned as a wave-uniform value (so that obstacle
// indices derived from it address the scene with scalar loads).
__device__ __forceinline__ uint64_t wave_or64(uint64_t x) {
#pragma unroll
  for (int off = 32; off; off >>= 1) x |= __shfl_xor(x, off, 64);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// One lane per configuration: forward kinematics link by link; per link,
// the obstacles its bounding ball can reach (a bit mask per 64 obstacles),
// and the exact predicates only for those pairs.  Loops run over the scene
// uniformly across the wave, so the scene is read with scalar loads; the
// wave stops early once every lane has a hit.
__global__ __launch_bounds__(256, 4) void check_kernel(SceneDev S, const double *__restrict__ q, int64_t n, int64_t ld,
                                                    uint8_t *__restrict__ verdict) {
  const int d = S.nj;
  const int nobs = S.n_osph + S.n_obox + S.n_ocyl;
  const int nsb_all = S.n_osph, nbx_all = S.n_osph + S.n_obox;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t start = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t rounds = (n + stride - 1) / stride;
  for (int64_t it = 0; it < rounds; ++it) {
    const int64_t i = start + it * stride;
    const bool valid = i < n;
    const int64_t ii = valid ? i : n - 1;
    bool hit = !valid;
    double T[12] = {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0};
    for (int li = 0; li < d; ++li) {
      double sn_, cs_;
      sincos_own(q[(int64_t)li * ld + ii], &sn_, &cs_);
      fk_step(T, S.joint_T + 12 * li, S.joint_pure[li] != 0, S.joint_axis[li], sn_, cs_);
      const double *lb = S.lbound + 4 * li;
      if (!(lb[3] >= 0.0)) continue;
      double cb[3];
      xform(T, lb, cb);
      const double Rb = lb[3] + S.eps;
      const double hc = -0.5 * sq3(cb[0], cb[1], cb[2]);
      // li is wave-uniform: the row is read with scalar loads
      const double *crow = S.cull + 4 * (int64_t)__builtin_amdgcn_readfirstlane(li * S.nobs_pad);
      for (int b0 = 0; b0 < nobs; b0 += 64) {
        const int nb = nobs - b0 < 64 ? nobs - b0 : 64;
        // every obstacle's ball, four at a time from the link's row (one
        // wave-uniform load of 16 doubles per group): c.o - |c|^2/2 against
        // the obstacle's threshold, a bit per obstacle in two 32-bit words;
        // then the boxes and cylinders that some lane's ball reaches against
        // their exact distance
        uint32_t nlo = 0, nhi = 0;
        const int nsb = nsb_all - b0 < 0 ? 0 : (nsb_all - b0 < nb ? nsb_all - b0 : nb);
        const int nbx = nbx_all - b0 < 0 ? 0 : (nbx_all - b0 < nb ? nbx_all - b0 : nb);
        for (int b = 0; b < nb; b += 4) {
          const double *cl = crow + 4 * (b0 + b);
          uint32_t m = 0;
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const double v = fma(cb[0], cl[4 * u], fma(cb[1], cl[4 * u + 1], fma(cb[2], cl[4 * u + 2], hc)));
            m |= !(v < cl[4 * u + 3]) ? (1u << u) : 0u;
          }
          if (b < 32)
            nlo |= m << b;
          else
            nhi |= m << (b - 32);
        }
        uint64_t near = ((uint64_t)nhi << 32) | nlo;
        near &= nb == 64 ? ~0ull : (1ull << nb) - 1ull;
        if (hit) near = 0;
        uint64_t any = wave_or64(near);
        const uint64_t sph = nsb >= 64 ? ~0ull : (1ull << nsb) - 1ull;
        for (uint64_t hard = any & ~sph; hard; hard &= hard - 1) {
          const int b = __ffsll((long long)hard) - 1;
          const bool nr = b < nbx ? ball_near_box(cb, Rb, S.obox + 16 * (b0 + b - nsb_all))
                                  : ball_near_cyl(cb, Rb, S.ocyl + 16 * (b0 + b - nbx_all));
          if (!nr) near &= ~(1ull << b);
          if (!__ballot((near >> b) & 1ull)) any &= ~(1ull << b);
        }
        if (!any) continue;
        for (int a = S.lsph_off[li]; a < S.lsph_off[li + 1]; ++a) {
          const double *sp = S.lsph + 4 * a;
          double cw[3];
          xform(T, sp, cw);
          for (uint64_t m = any; m; m &= m - 1) {
            const int b = __ffsll((long long)m) - 1;
            if (!((near >> b) & 1ull) || hit) continue;
            const int o = b0 + b;
            hit = o < nsb_all   ? sphere_sphere(cw, sp[3], S.osph + 4 * o, S.osph[4 * o + 3])
                  : o < nbx_all ? sphere_box(cw, sp[3], S.obox + 16 * (o - nsb_all))
                                : sphere_cyl(cw, sp[3], S.ocyl + 16 * (o - nbx_all));
          }
        }
        for (int a = S.lcap_off[li]; a < S.lcap_off[li + 1]; ++a) {
          const double *cp = S.lcap + 8 * a;
          double p0[3], p1[3];
          xform(T, cp, p0);
          xform(T, cp + 3, p1);
          for (uint64_t m = any; m; m &= m - 1) {
            const int b = __ffsll((long long)m) - 1;
            const int o = b0 + b;
            if (!((near >> b) & 1ull) || hit || o >= S.n_osph) continue;
            hit = capsule_sphere(p0, p1, cp[6], S.osph + 4 * o, S.osph[4 * o + 3]);
          }
        }
      }
      if (__ballot(!hit) == 0) break;
    }
    if (valid) verdict[i] = hit ? 1 : 0;
  }
}

// Sphere-parallel layout (Sec. V-C: threads over the robot's spheres, then
// over configurations), for batches too small to fill the device with one
// lane per configuration: a group of NSP consecutive lanes (NSP a power of
// two at least the robot's sphere count) takes one configuration, lane j of
// the group its j-th link sphere (grouped by link).  Each lane runs the
// forward kinematics up to its sphere's link, in the same operation order as
// the per-configuration kernel, and tests its sphere against every obstacle;
// the group's hits are ORed with a ballot and its first lane writes the
// verdict.  Robots with capsules use the per-configuration kernel.
template <int NSP>
__global__ __launch_bounds__(256) void check_sphere_kernel(SceneDev S, int n_lsph, const double *__restrict__ q,
                                                           int64_t n, int64_t ld, uint8_t *__restrict__ verdict) {
  constexpr int GPW = 64 / NSP;  // configurations per wave
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t n_waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const int g = lane / NSP, a = lane % NSP;
  for (int64_t w0 = wave * GPW; w0 < n; w0 += n_waves * GPW) {
    const int64_t c = w0 + g;
    bool hit = false;
    if (c < n && a < n_lsph) {
      int li = 0;
      while (li + 1 < S.nj && S.lsph_off[li + 1] <= a) ++li;
      double T[12] = {1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0};
      for (int j = 0; j <= li; ++j) {
        double sn_, cs_;
        sincos_own(q[(int64_t)j * ld + c], &sn_, &cs_);
        fk_step(T, S.joint_T + 12 * j, S.joint_pure[j] != 0, S.joint_axis[j], sn_, cs_);
      }
      const double *sp = S.lsph + 4 * a;
      double cw[3];
      xform(T, sp, cw);
      for (int b = 0; b < S.n_osph && !hit; ++b) hit = sphere_sphere(cw, sp[3], S.osph + 4 * b, S.osph[4 * b + 3]);
      for (int b = 0; b < S.n_obox && !hit; ++b) hit = sphere_box(cw, sp[3], S.obox + 16 * b);
      for (int b = 0; b < S.n_ocyl && !hit; ++b) hit = sphere_cyl(cw, sp[3], S.ocyl + 16 * b);
    }
    const uint64_t bal = __ballot(hit);
    const uint64_t gmask = (NSP == 64 ? ~0ull : ((1ull << NSP) - 1ull)) << (g * NSP);
    if (a == 0 && c < n) verdict[c] = (bal & gmask) ? 1 : 0;
  }
}

// Launches the verdict kernel for n configurations: the sphere-parallel
// layout when one lane per configuration would start fewer than 8192 waves
// and the robot is made of at most 64 spheres, else the per-configuration
// kernel.
int launch_check(ip_ctx *ctx, const SceneDev &S, int n_lsph, int n_lcap, const double *q, int64_t n, int64_t ld,
                 uint8_t *verdict) {
  if (n == 0) return IP_OK;
  if (n_lcap == 0 && n_lsph > 0 && n_lsph <= 64 && n < 8192 * 64) {
    int nsp = 1;
    while (nsp < n_lsph) nsp <<= 1;
    const int64_t per_block = 4 * (64 / nsp);
    const int64_t blocks = std::min<int64_t>((n + per_block - 1) / per_block, 65536);
#define IP_CS(NN)                                                                                              \
  hipLaunchKernelGGL((check_sphere_kernel<NN>), dim3((unsigned)blocks), dim3(256), 0, ctx->stream, S, n_lsph, q, \
                     n, ld, verdict)
    switch (nsp) {
      case 1: IP_CS(1); break;
      case 2: IP_CS(2); break;
      case 4: IP_CS(4); break;
      case 8: IP_CS(8); break;
      case 16: IP_CS(16); break;
      case 32: IP_CS(32); break;
      default: IP_CS(64); break;
    }
#undef IP_CS
  } else {
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(check_kernel, dim3((unsigned)blocks), dim3(256), 0, ctx->stream, S, q, n, ld, verdict);
  }
  IP_TRY_HIP(ctx, hipGetLastError());
  return IP_OK;
}

// Stable compaction of the free (verdict 0) points, by tiles of kTile cells:
// count per tile, exclusive scan of the counts, then each tile writes its
// free points in cell order at its offset.
constexpr int kTile = 4096;

__global__ __launch_bounds__(256) void free_count_kernel(const uint8_t *__restrict__ verdict, int64_t n,
                                                         uint32_t *__restrict__ cnt) {
  __shared__ uint32_t part[4];
  const int64_t base = (int64_t)blockIdx.x * kTile;
  uint32_t c = 0;
  for (int k = 0; k < kTile / 256; ++k) {
    const int64_t i = base + k * 256 + threadIdx.x;
    c += (i < n && verdict[i] == 0) ? 1u : 0u;
  }
  for (int off = 32; off; off >>= 1) c += __shfl_xor(c, off, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) cnt[blockIdx.x] = part[0] + part[1] + part[2] + part[3];
}

// Exclusive scan of cnt[0 .. m) into off, total into *total (one block).
__global__ __launch_bounds__(1024) void scan_tiles_kernel(const uint32_t *__restrict__ cnt, int64_t m,
                                                          uint64_t *__restrict__ off,
                                                          unsigned long long *__restrict__ total) {
  __shared__ unsigned long long wsum[16];
  __shared__ unsigned long long carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int64_t b = 0; b < m; b += 1024) {
    const int64_t i = b + threadIdx.x;
    const unsigned long long v = i < m ? cnt[i] : 0ull;
    unsigned long long x = v;
    for (int o = 1; o < 64; o <<= 1) {
      const unsigned long long y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    if (lane == 63) wsum[wv] = x;
    __syncthreads();
    unsigned long long before = carry;
    for (int w = 0; w < wv; ++w) before += wsum[w];
    if (i < m) off[i] = before + x - v;
    __syncthreads();
    if (threadIdx.x == 1023) carry = before + x;
    __syncthreads();
  }
  if (threadIdx.x == 0) *total = carry;
}

__global__ __launch_bounds__(256) void free_scatter_kernel(const uint8_t *__restrict__ verdict,
                                                           const double *__restrict__ pts, int64_t n, int64_t ld, int d,
                                                           const uint64_t *__restrict__ off,
                                                           double *__restrict__ free_pts, int64_t ld_free) {
  __shared__ uint32_t wcount[4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t base = (int64_t)blockIdx.x * kTile;
  uint64_t pos0 = off[blockIdx.x];
  for (int k = 0; k < kTile / 256; ++k) {
    const int64_t i = base + k * 256 + threadIdx.x;
    const bool fr = i < n && verdict[i] == 0;
    const uint64_t bal = __ballot(fr);
    if (lane == 0) wcount[wv] = (uint32_t)__popcll(bal);
    __syncthreads();
    uint64_t pos = pos0;
    for (int w = 0; w < wv; ++w) pos += wcount[w];
    pos += (uint64_t)__popcll(bal & ((1ull << lane) - 1ull));
    if (fr)
      for (int j = 0; j < d; ++j) free_pts[(int64_t)j * ld_free + (int64_t)pos] = pts[(int64_t)j * ld + i];
    pos0 += wcount[0] + wcount[1] + wcount[2] + wcount[3];
    __syncthreads();
  }
}

int upload_scene(ip_ctx *ctx, const ip_scene *sc, SceneDev *out) {
  const int nj = sc->n_joints;
  if (nj < 1 || nj > IP_MAX_D) return ip_fail(ctx, IP_EINVAL, "scene: joint count out of range");
  if (sc->n_lsph < 0 || sc->n_lcap < 0 || sc->n_osph < 0 || sc->n_obox < 0 || sc->n_ocyl < 0)
    return ip_fail(ctx, IP_EINVAL, "scene: negative counts");
  if (sc->n_lcap > 0 && (sc->n_obox > 0 || sc->n_ocyl > 0))
    return ip_fail(ctx, IP_EINVAL, "scene: capsules are tested against obstacle spheres only");
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
  std::vector<double> osph(4 * (size_t)sc->n_osph), obox(16 * (size_t)sc->n_obox),
      ocyl(16 * (size_t)sc->n_ocyl, 0.0);
  // bounding-ball radii, rounded up (the culling margin covers the rest)
  for (int b = 0; b < sc->n_ocyl; ++b) {
    for (int j = 0; j < 12; ++j) ocyl[16 * b + j] = sc->ocyl_T[12 * b + j];
    const double rc = sc->ocyl_rh[2 * b], h = sc->ocyl_rh[2 * b + 1];
    ocyl[16 * b + 12] = rc;
    ocyl[16 * b + 13] = h;
    ocyl[16 * b + 14] = std::sqrt(rc * rc + 0.25 * h * h) * (1.0 + 1e-12);
  }
  for (int b = 0; b < sc->n_osph; ++b) {
    for (int j = 0; j < 3; ++j) osph[4 * b + j] = sc->osph_c[3 * b + j];
    osph[4 * b + 3] = sc->osph_r[b];
  }
  for (int b = 0; b < sc->n_obox; ++b) {
    for (int j = 0; j < 12; ++j) obox[16 * b + j] = sc->obox_T[12 * b + j];
    for (int j = 0; j < 3; ++j) obox[16 * b + 12 + j] = sc->obox_l[3 * b + j];
    const double *l = sc->obox_l + 3 * b;
    obox[16 * b + 15] = 0.5 * std::sqrt(l[0] * l[0] + l[1] * l[1] + l[2] * l[2]) * (1.0 + 1e-12);
  }
  // the obstacles' balls (spheres, boxes, cylinders), padded to a multiple
  // of 4 with balls too far away to reach (centre 1e150, radius 0)
  const int nobs = sc->n_osph + sc->n_obox + sc->n_ocyl;
  const int nobs_pad = (nobs + 3) / 4 * 4;
  std::vector<double> oball(4 * (size_t)nobs_pad, 0.0);
  for (int b = nobs; b < nobs_pad; ++b) oball[4 * b] = oball[4 * b + 1] = oball[4 * b + 2] = 1e150;
  for (int b = 0; b < sc->n_osph; ++b)
    for (int j = 0; j < 4; ++j) oball[4 * b + j] = osph[4 * b + j];
  for (int b = 0; b < sc->n_obox; ++b) {
    double *c = &oball[4 * (sc->n_osph + b)];
    c[0] = obox[16 * b + 3];
    c[1] = obox[16 * b + 7];
    c[2] = obox[16 * b + 11];
    c[3] = obox[16 * b + 15];
  }
  for (int b = 0; b < sc->n_ocyl; ++b) {
    double *c = &oball[4 * (sc->n_osph + sc->n_obox + b)];
    c[0] = ocyl[16 * b + 3];
    c[1] = ocyl[16 * b + 7];
    c[2] = ocyl[16 * b + 11];
    c[3] = ocyl[16 * b + 14];
  }
  // per-link bounding balls (link frame): centre at the middle of the
  // geometry's extent, radius covering every sphere and capsule of the link
  std::vector<double> lbound(4 * (size_t)nj, 0.0);
  double scale = 1.0;
  for (int li = 0; li < nj; ++li) {
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    bool any = false;
    auto grow = [&](const double *pp) {
      for (int j = 0; j < 3; ++j) {
        lo[j] = std::min(lo[j], pp[j]);
        hi[j] = std::max(hi[j], pp[j]);
      }
      any = true;
    };
    for (int a = lsph_off[li]; a < lsph_off[li + 1]; ++a) grow(&lsph[4 * a]);
    for (int a = lcap_off[li]; a < lcap_off[li + 1]; ++a) {
      grow(&lcap[8 * a]);
      grow(&lcap[8 * a + 3]);
    }
    if (!any) {
      lbound[4 * li + 3] = -1.0;
      continue;
    }
    double c[3], R = 0.0;
    for (int j = 0; j < 3; ++j) c[j] = 0.5 * (lo[j] + hi[j]);
    auto dist = [&](const double *pp) {
      return std::sqrt((pp[0] - c[0]) * (pp[0] - c[0]) + (pp[1] - c[1]) * (pp[1] - c[1]) +
                       (pp[2] - c[2]) * (pp[2] - c[2]));
    };
    for (int a = lsph_off[li]; a < lsph_off[li + 1]; ++a) R = std::max(R, dist(&lsph[4 * a]) + lsph[4 * a + 3]);
    for (int a = lcap_off[li]; a < lcap_off[li + 1]; ++a)
      R = std::max(R, std::max(dist(&lcap[8 * a]), dist(&lcap[8 * a + 3])) + lcap[8 * a + 6]);
    for (int j = 0; j < 3; ++j) {
      lbound[4 * li + j] = c[j];
      scale = std::max(scale, std::fabs(c[j]) + R);
    }
    lbound[4 * li + 3] = R * (1.0 + 1e-12);
  }
  for (int i = 0; i < 12 * nj; ++i) scale = std::max(scale, std::fabs(sc->joint_T[i]));
  for (double x : osph) scale = std::max(scale, std::fabs(x));
  for (int b = 0; b < sc->n_obox; ++b)
    for (int j = 0; j < 15; ++j) scale = std::max(scale, std::fabs(obox[16 * b + j]));
  for (int b = 0; b < sc->n_ocyl; ++b)
    for (int j = 0; j < 14; ++j) scale = std::max(scale, std::fabs(ocyl[16 * b + j]));
  // the geometry is summed over at most a few dozen terms of size `scale`
  // (reach times the chain length): rounding stays below 1e-13 * scale
  const double eps = 1e-9 * scale * (double)(nj + 1);
  // per link and obstacle, the culling threshold of the expanded squared
  // distance |c - o|^2 = |c|^2 - 2 c.o + |o|^2; its rounding (a few ulp of
  // |c|^2 + |o|^2) is far below the margin 2 (R + rb) eps it is compared with
  std::vector<double> cull(4 * (size_t)nobs_pad * nj, 0.0);
  for (int li = 0; li < nj; ++li)
    for (int b = 0; b < nobs_pad; ++b) {
      const double *o = &oball[4 * b];
      double *c = &cull[4 * ((size_t)li * nobs_pad + b)];
      const double rr = (lbound[4 * li + 3] + eps) + o[3];
      c[0] = o[0];
      c[1] = o[1];
      c[2] = o[2];
      c[3] = b < nobs ? 0.5 * ((o[0] * o[0] + o[1] * o[1] + o[2] * o[2]) - rr * rr) : 1e300;
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
  size_t o_oc = put(ocyl.data(), ocyl.size());
  size_t o_lb = put(lbound.data(), lbound.size());
  size_t o_cl = put(cull.data(), cull.size());
  size_t n_dbl = blob.size();
  std::vector<int32_t> ints;
  ints.insert(ints.end(), sc->joint_axis, sc->joint_axis + nj);
  size_t o_jp = ints.size();
  for (int i = 0; i < nj; ++i) {
    const double *J = sc->joint_T + 12 * i;
    const bool pure = J[0] == 1.0 && J[1] == 0.0 && J[2] == 0.0 && J[4] == 0.0 && J[5] == 1.0 && J[6] == 0.0 &&
                      J[8] == 0.0 && J[9] == 0.0 && J[10] == 1.0;
    ints.push_back(pure ? 1 : 0);
  }
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
  out->joint_pure = ib + o_jp;
  out->lsph_off = ib + o_lso;
  out->lsph = db + o_ls;
  out->lcap_off = ib + o_lco;
  out->lcap = db + o_lc;
  out->n_osph = sc->n_osph;
  out->n_obox = sc->n_obox;
  out->n_ocyl = sc->n_ocyl;
  out->pad = 0;
  out->ocyl = db + o_oc;
  out->osph = db + o_os;
  out->obox = db + o_ob;
  out->lbound = db + o_lb;
  out->cull = db + o_cl;
  out->nobs_pad = nobs_pad;
  out->eps = eps;
  return IP_OK;
}

}  // namespace

int ip_check_impl(ip_ctx *ctx, const ip_scene *scene, const double *q_dev, int64_t n, int64_t ld,
                  uint8_t *verdict_dev) {
  SceneDev S;
  IP_TRY(upload_scene(ctx, scene, &S));
  return launch_check(ctx, S, scene->n_lsph, scene->n_lcap, q_dev, n, ld, verdict_dev);
}

// Verdicts of every cell, then the stable compaction of the free points.
int ip_check_gather_impl(ip_ctx *ctx, const ip_scene *scene, ip_cells *c) {
  SceneDev S;
  IP_TRY(upload_scene(ctx, scene, &S));
  if (c->free_pts) {
    ip_dfree(ctx, c->free_pts);
    c->free_pts = nullptr;
  }
  const int64_t n = c->n;
  IP_TRY(ip_dalloc(ctx, (void **)&c->free_pts, sizeof(double) * (size_t)(n ? n : 1) * c->d));
  IP_TRY_HIP(ctx, hipMemsetAsync(ctx->ctr_dev, 0, sizeof(Counters), ctx->stream));
  const int64_t ntiles = (n + kTile - 1) / kTile;
  void *tiles = nullptr;
  IP_TRY(ip_dalloc(ctx, &tiles, (size_t)(ntiles ? ntiles : 1) * 12));
  uint64_t *off = (uint64_t *)tiles;
  uint32_t *cnt = (uint32_t *)(off + (ntiles ? ntiles : 1));
  IP_TRY_HIP(ctx, hipEventRecord(ctx->ev0, ctx->stream));
  if (n) {
    const int rc = launch_check(ctx, S, scene->n_lsph, scene->n_lcap, (const double *)c->pts, n, c->ld, c->verdict);
    if (rc != IP_OK) {
      (void)hipStreamSynchronize(ctx->stream);
      ip_dfree(ctx, tiles);
      return rc;
    }
    hipLaunchKernelGGL(free_count_kernel, dim3((unsigned)ntiles), dim3(256), 0, ctx->stream,
                       (const uint8_t *)c->verdict, n, cnt);
    hipLaunchKernelGGL(scan_tiles_kernel, dim3(1), dim3(1024), 0, ctx->stream, (const uint32_t *)cnt, ntiles, off,
                       &ctx->ctr_dev->n_aux);
    hipLaunchKernelGGL(free_scatter_kernel, dim3((unsigned)ntiles), dim3(256), 0, ctx->stream,
                       (const uint8_t *)c->verdict, (const double *)c->pts, n, c->ld, c->d, (const uint64_t *)off,
                       c->free_pts, n);
  }
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipEventRecord(ctx->ev1, ctx->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ctx->ctr_host, ctx->ctr_dev, sizeof(Counters), hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  ip_dfree(ctx, tiles);
  if (e != hipSuccess) return ip_hip(ctx, e, "ip_check_cells");
  float ms = 0.0f;
  IP_TRY_HIP(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
  c->st.ms_check = ms;
  c->n_free = (int64_t)ctx->ctr_host->n_aux;
  return IP_OK;
}
