// f evaluation at lattice vertices (the edge sign tests of Sec. V-A and the
// subdivision vertices of Sec. V-B need f at every vertex they touch).
//
// Canonical FP64 kernel: one lane per vertex, R vertices per lane (register
// blocking), support vectors consumed in index order so the accumulation
// order is the canonical one of ip.h and the result is bit-identical on every
// device.  Every lane of a wave reads the same 64-byte support-vector record
// at the same time, so the record is a wave-uniform load served from the
// scalar cache into SGPRs and used as the scalar operand of v_fma_f64.
//
// FP32 certified kernel: the decision function of a degree-p polynomial
// kernel is a polynomial of degree p in d variables; it is evaluated in FP32
// in its monomial basis (C(d+p, p) coefficients, precomputed on the host in
// FP64 with rigorous error bounds) together with a rigorous bound B32 on
// |f32 - F|, F the exact value at the canonical FP64 coordinates.  With B64 a
// bound on |f64 - F| for the canonical FP64 value, a vertex with
// |f32| > B32 + B64 has sign(f32) = sign(F) = sign(f64); every other vertex
// is re-evaluated by the canonical FP64 kernel, so the sign bits, and the
// traced set, equal the FP64 ones.
#include <algorithm>
#include <mutex>

#include "ip_internal.h"

// Device scratch of ip_feval_noalloc, one copy per device at its own
// address: a 256-byte header holding two counters (the fallback-list length
// and the FP64-monomial settlements), then the fallback list, one 4-byte
// vertex index per vertex of the largest call.  Host code never passes this
// name to a kernel: it passes the address hipGetSymbolAddress returned for
// the current device (noalloc_scratch of the context).
static __device__ __align__(256) unsigned char scratch[256 + 4 * (size_t)IP_NOALLOC_MAX_VERTICES];

namespace {

// MODE 0: vertex-table entries listed by slot (key at keys[slot * 4], result
//         to out[slot * 4]);
// MODE 1: raw int32 vertices, result to out[i];
// MODE 2: raw int32 vertices at the indices in list, result to out[index].
// n_dev (may be NULL): the item count is *n_dev, written by an earlier
// kernel on the stream, at most n (the grid is sized for n).
template <int D, int P, int R, int MODE>
__global__ __launch_bounds__(256) void feval64_kernel(FDev F, LatDev L, const uint32_t *__restrict__ list,
                                                      uint64_t n, const unsigned long long *n_dev,
                                                      const uint64_t *__restrict__ keys,
                                                      const int32_t *__restrict__ vraw,
                                                      double *__restrict__ out) {
  constexpr uint64_t S4 = MODE == 0 ? 4 : 1;
  if (n_dev) n = (uint64_t)*n_dev < n ? (uint64_t)*n_dev : n;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x * R;
  for (uint64_t base = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * R; base < n; base += stride) {
    double x[R][D];
    uint64_t dst[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      uint64_t i = base + r < n ? base + r : n - 1;
      int32_t v[D];
      if (MODE == 0) {
        uint32_t s = list[i];
        dst[r] = s;
        vunpack<D>(L, keys[(uint64_t)s * 4], v);
      } else {
        const uint64_t src = MODE == 2 ? (uint64_t)list[i] : i;
        dst[r] = src;
#pragma unroll
        for (int j = 0; j < D; ++j) v[j] = vraw[src * D + j];
      }
      lat_coords<D>(L, v, x[r]);
    }
    double acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = 0.0;
    const double gamma = F.gamma, coef0 = F.coef0;
    for (int64_t s = 0; s < F.S; ++s) {
      const double *rec = F.rec + s * 8;
      double sv[D];
#pragma unroll
      for (int j = 0; j < D; ++j) sv[j] = rec[j];
      const double al = rec[D];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        double dot = 0.0;
#pragma unroll
        for (int j = 0; j < D; ++j) dot = fma(sv[j], x[r][j], dot);
        double t = fma(gamma, dot, coef0);
        double tp = t;
        if (P > 0) {
#pragma unroll
          for (int q = 1; q < P; ++q) tp = tp * t;
        } else {
          for (int q = 1; q < F.p; ++q) tp = tp * t;
        }
        acc[r] = fma(al, tp, acc[r]);
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (base + r < n) out[dst[r] * S4] = acc[r] + F.bias;
  }
}

// Canonical FP64 RBF evaluation (same MODEs as feval64_kernel): the support
// vectors pass through LDS in tiles of kRbfTile records, which every lane of
// the block then reads at the same address (a broadcast), in index order.
// The loop over vertex groups is uniform across the block, so the barriers
// around each tile are reached by every thread.
constexpr int kRbfTile = 256;

template <int D, int R, int MODE>
__global__ __launch_bounds__(256) void rbf64_kernel(FDev F, LatDev L, const uint32_t *__restrict__ list, uint64_t n,
                                                    const unsigned long long *n_dev,
                                                    const uint64_t *__restrict__ keys,
                                                    const int32_t *__restrict__ vraw, double *__restrict__ out) {
  __shared__ double tile[kRbfTile * 8];
  constexpr uint64_t S4 = MODE == 0 ? 4 : 1;
  if (n_dev) n = (uint64_t)*n_dev < n ? (uint64_t)*n_dev : n;
  const uint64_t per_block = (uint64_t)blockDim.x * R;
  for (uint64_t blk = (uint64_t)blockIdx.x * per_block; blk < n; blk += (uint64_t)gridDim.x * per_block) {
    const uint64_t base = blk + (uint64_t)threadIdx.x * R;
    double x[R][D];
    uint64_t dst[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint64_t i = base + r < n ? base + r : n - 1;
      int32_t v[D];
      if (MODE == 0) {
        const uint32_t s = list[i];
        dst[r] = s;
        vunpack<D>(L, keys[(uint64_t)s * 4], v);
      } else {
        const uint64_t src = MODE == 2 ? (uint64_t)list[i] : i;
        dst[r] = src;
#pragma unroll
        for (int j = 0; j < D; ++j) v[j] = vraw[src * D + j];
      }
      lat_coords<D>(L, v, x[r]);
    }
    double acc[R];
#pragma unroll
    for (int r = 0; r < R; ++r) acc[r] = 0.0;
    for (int64_t t0 = 0; t0 < F.S; t0 += kRbfTile) {
      const int nt = (int)(F.S - t0 < kRbfTile ? F.S - t0 : kRbfTile);
      __syncthreads();
      for (int q = threadIdx.x; q < nt * 8; q += blockDim.x) tile[q] = F.rec[t0 * 8 + q];
      __syncthreads();
      for (int s = 0; s < nt; ++s) {
        const double *sv = tile + s * 8;
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] = rbf_term<D>(sv, sv[D], F.gamma, x[r], acc[r]);
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (base + r < n) out[dst[r] * S4] = acc[r] + F.bias;
  }
}

template <int D, int P, int MODE>
void launch64(hipStream_t st, const FDev &F, const LatDev &L, const uint32_t *list, uint64_t n,
              const unsigned long long *n_dev, const uint64_t *keys, const int32_t *vraw, double *out) {
  constexpr int R = D <= 4 ? 4 : 2;
  const uint64_t threads = (n + R - 1) / R;
  uint64_t blocks = (threads + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks == 0) return;
  hipLaunchKernelGGL((feval64_kernel<D, P, R, MODE>), dim3((unsigned)blocks), dim3(256), 0, st, F, L, list, n, n_dev,
                     keys, vraw, out);
}

template <int D, int MODE>
void launch64_p(hipStream_t st, const FDev &F, const LatDev &L, const uint32_t *list, uint64_t n,
                const unsigned long long *n_dev, const uint64_t *keys, const int32_t *vraw, double *out) {
  if (F.kernel == IP_KERNEL_RBF) {
    constexpr int R = 2;
    const uint64_t blocks = std::min<uint64_t>((n + 256 * R - 1) / (256 * R), 65536);
    if (blocks == 0) return;
    hipLaunchKernelGGL((rbf64_kernel<D, R, MODE>), dim3((unsigned)blocks), dim3(256), 0, st, F, L, list, n, n_dev,
                       keys, vraw, out);
    return;
  }
  switch (F.p) {
    case 1: launch64<D, 1, MODE>(st, F, L, list, n, n_dev, keys, vraw, out); break;
    case 2: launch64<D, 2, MODE>(st, F, L, list, n, n_dev, keys, vraw, out); break;
    case 3: launch64<D, 3, MODE>(st, F, L, list, n, n_dev, keys, vraw, out); break;
    case 4: launch64<D, 4, MODE>(st, F, L, list, n, n_dev, keys, vraw, out); break;
    default: launch64<D, 0, MODE>(st, F, L, list, n, n_dev, keys, vraw, out); break;
  }
}

template <int MODE>
int dispatch64(ip_ctx *ctx, const FDev &F, const LatDev &L, const uint32_t *list, uint64_t n,
               const uint64_t *keys, const int32_t *vraw, double *out,
               const unsigned long long *n_dev = nullptr) {
  if (n == 0) return IP_OK;
  hipStream_t st = ctx->stream;
  switch (L.d) {
    case 2: launch64_p<2, MODE>(st, F, L, list, n, n_dev, keys, vraw, out); break;
    case 3: launch64_p<3, MODE>(st, F, L, list, n, n_dev, keys, vraw, out); break;
    case 4: launch64_p<4, MODE>(st, F, L, list, n, n_dev, keys, vraw, out); break;
    case 5: launch64_p<5, MODE>(st, F, L, list, n, n_dev, keys, vraw, out); break;
    case 6: launch64_p<6, MODE>(st, F, L, list, n, n_dev, keys, vraw, out); break;
    case 7: launch64_p<7, MODE>(st, F, L, list, n, n_dev, keys, vraw, out); break;
    default: return ip_fail(ctx, IP_EINVAL, "dimension out of range");
  }
  IP_TRY_HIP(ctx, hipGetLastError());
  return IP_OK;
}

// ---------------------------------------------------------------------------
// FP32 monomial-basis evaluation with certification
// ---------------------------------------------------------------------------
// Tiered certification.  Tier 1: f in FP32 in the monomial basis; settled
// when |f32| > B32 + B64.  Tier 2 (only for the rest): f in FP64 in the
// monomial basis; settled when |f64m| > B64m + B64.  Tier 3: the canonical
// FP64 sum over the support vectors, for what is left.
// MODE 0: vertex-table slots (f to vt[slot].f, bound to vb[slot]);
// MODE 1: raw vertices (f to out[i], bound to bout[i]).
// Tier-3 vertices get vb = -1 (resp. bout = 0) and are appended to fb (slot,
// resp. index) for the canonical FP64 kernel.
template <int D, int P, int MODE>
__global__ __launch_bounds__(256) void feval32_kernel(PolyDev Q, LatDev L, const uint32_t *__restrict__ list,
                                                      uint64_t n, VEnt *vt, float *vb,
                                                      const int32_t *__restrict__ vraw, double *out, double *bout,
                                                      uint32_t *fb, unsigned long long *fb_ctr,
                                                      unsigned long long *c64_ctr) {
  constexpr int kStage = 128;
  __shared__ uint32_t st[4][kStage];
  const int wib = threadIdx.x >> 6;
  int sn = 0;
  auto put = [&](unsigned long long pos, uint32_t s) { fb[pos] = s; };
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t start = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t rounds = (n + stride - 1) / stride;
  unsigned long long n64 = 0;
  for (uint64_t it = 0; it < rounds; ++it) {
    const uint64_t i = start + it * stride;
    bool unsure = false;
    uint32_t id = 0;
    if (i < n) {
      int32_t v[D];
      if (MODE == 0) {
        id = list[i];
        vunpack<D>(L, vt[id].key, v);
      } else {
        id = (uint32_t)i;
#pragma unroll
        for (int j = 0; j < D; ++j) v[j] = vraw[i * D + j];
      }
      double x64[D];
      lat_coords<D>(L, v, x64);
      double fv, bnd;
      const int tier = cert_eval<D, P>(Q, x64, &fv, &bnd);
      unsure = tier == 3;
      if (tier == 2) ++n64;
      if (MODE == 0) {
        if (!unsure) vt[id].f = fv;
        vb[id] = unsure ? -1.0f : (float)(bnd * (1.0 + 1e-6));
      } else {
        out[i] = fv;
        if (bout) bout[i] = unsure ? 0.0 : bnd + Q.B64;
      }
    }
    stage_put<kStage>(st[wib], sn, unsure, id, put, fb_ctr);
  }
  stage_flush(st[wib], sn, put, fb_ctr);
  if (n64) atomicAdd(c64_ctr, n64);
}

// FP32 certified RBF evaluation (same MODEs and outputs as feval32_kernel).
// With u = 2^-24, at the canonical FP64 coordinates x (rounded to FP32):
// per support vector d2 = the FP32 fma chain of (x_j - s_j)^2, e = the own
// FP32 exponential of -(gamma d2), term = alpha e; the terms are summed in
// blocks of 32 and the block sums added, A = sum |term| and W = sum |term| d2
// beside them.  The bound on |f32 - F| (F the exact value at x):
//   43 u A'  (exponential 40 u, alpha and product 2 u, sum of A 1 u)
// + gamma u ((d + 4) W' + 9 (|x|^2 + max |s|^2) A')  (the rounding of d2
//   and of gamma d2 moves the exponent: |dt| <= gamma u ((d + 3) d2 +
//   8.1 (|x|^2 + |s|^2)) per term, and |d exp| <= exp |dt| (1 + |dt|))
// + (32 + S / 32 + 3) u A'  (two-level summation)
// + u (|bias| + |f32|) + 2e-38 S max|alpha|  (final add; exponential underflow)
// with A' = A (1 + (S + 60) u), W' likewise (the FP32 sums of positive terms
// and the relative errors of their terms), all times 1.01 for the products
// of the first-order terms.  Tier 1 settles the sign when |f32| exceeds the
// bound plus B64; the rest go to the canonical FP64 kernel.
constexpr int kRbf32Tile = 512;

template <int D, int MODE>
__global__ __launch_bounds__(256) void rbf32_kernel(RbfDev Q, LatDev L,
                                                    const uint32_t *__restrict__ list, uint64_t n, VEnt *vt,
                                                    float *vb, const int32_t *__restrict__ vraw, double *out,
                                                    double *bout, uint32_t *fb, unsigned long long *fb_ctr) {
  __shared__ float tile[kRbf32Tile * 8];
  constexpr int kStage = 128;
  __shared__ uint32_t st[4][kStage];
  const int wib = threadIdx.x >> 6;
  int sn = 0;
  auto put = [&](unsigned long long pos, uint32_t s) { fb[pos] = s; };
  const double u = 5.9604644775390625e-08;
  for (uint64_t blk = (uint64_t)blockIdx.x * blockDim.x; blk < n; blk += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t i = blk + threadIdx.x;
    const bool valid = i < n;
    const uint64_t ii = valid ? i : n - 1;
    uint32_t id = 0;
    int32_t v[D];
    if (MODE == 0) {
      id = list[ii];
      vunpack<D>(L, vt[id].key, v);
    } else {
      id = (uint32_t)ii;
#pragma unroll
      for (int j = 0; j < D; ++j) v[j] = vraw[ii * D + j];
    }
    double x64[D];
    lat_coords<D>(L, v, x64);
    float x[D];
    float X2 = 0.0f;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      x[j] = (float)x64[j];
      X2 = fmaf(x[j], x[j], X2);
    }
    float acc = 0.0f, blk_acc = 0.0f, A = 0.0f, W = 0.0f;
    int in_blk = 0;
    for (int64_t t0 = 0; t0 < Q.S; t0 += kRbf32Tile) {
      const int nt = (int)(Q.S - t0 < kRbf32Tile ? Q.S - t0 : kRbf32Tile);
      __syncthreads();
      for (int q = threadIdx.x; q < nt * 8; q += blockDim.x) tile[q] = Q.rec[t0 * 8 + q];
      __syncthreads();
      for (int s = 0; s < nt; ++s) {
        const float *sv = tile + s * 8;
        float d2 = 0.0f;
#pragma unroll
        for (int j = 0; j < D; ++j) {
          const float df = x[j] - sv[j];
          d2 = fmaf(df, df, d2);
        }
        const float term = sv[D] * exp32_own(-(Q.gamma * d2));
        blk_acc += term;
        A += fabsf(term);
        W = fmaf(fabsf(term), d2, W);
        if (++in_blk == 32) {
          acc += blk_acc;
          blk_acc = 0.0f;
          in_blk = 0;
        }
      }
    }
    acc += blk_acc;
    const float f32 = acc + Q.bias;
    const double S = (double)Q.S;
    const double grow = 1.0 + (S + 60.0) * u;
    const double Ap = (double)A * grow, Wp = (double)W * grow;
    const double X2p = (double)X2 * (1.0 + (D + 2) * u) + 1e-30;
    const double bnd = 1.01 * (43.0 * u * Ap + (double)Q.gamma * u * ((D + 4) * Wp + 9.0 * (X2p + (double)Q.nrm_max) * Ap) +
                               (35.0 + S / 32.0) * u * Ap + u * (fabs((double)Q.bias) + fabs((double)f32))) +
                       2e-38 * S * Q.amax;
    const double B64 = Q.B64;
    const bool unsure = !(fabs((double)f32) > bnd + B64);
    if (valid) {
      if (MODE == 0) {
        if (!unsure) vt[id].f = (double)f32;
        vb[id] = unsure ? -1.0f : (float)(bnd * (1.0 + 1e-6));
      } else {
        out[i] = (double)f32;
        if (bout) bout[i] = unsure ? 0.0 : bnd + B64;
      }
    }
    stage_put<kStage>(st[wib], sn, valid && unsure, id, put, fb_ctr);
  }
  stage_flush(st[wib], sn, put, fb_ctr);
}

__global__ void set_vb_kernel(const uint32_t *list, uint64_t n, float *vb, float v) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    vb[list[i]] = v;
}

template <int D, int MODE>
void launch32_p(hipStream_t st, const PolyDev &Q, const LatDev &L, const uint32_t *list, uint64_t n, VEnt *vt,
                float *vb, const int32_t *vraw, double *out, double *bout, uint32_t *fb, unsigned long long *fb_ctr,
                unsigned long long *c64) {
  uint64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks == 0) return;
#define IP_L32(PP)                                                                                               \
  hipLaunchKernelGGL((feval32_kernel<D, PP, MODE>), dim3((unsigned)blocks), dim3(256), 0, st, Q, L, list, n, vt, vb, \
                     vraw, out, bout, fb, fb_ctr, c64)
  switch (Q.p) {
    case 1: IP_L32(1); break;
    case 2: IP_L32(2); break;
    case 3: IP_L32(3); break;
    case 4: IP_L32(4); break;
    default: break;
  }
#undef IP_L32
}

template <int MODE>
int dispatch32(ip_ctx *ctx, const PolyDev &Q, const LatDev &L, const uint32_t *list, uint64_t n, VEnt *vt, float *vb,
               const int32_t *vraw, double *out, double *bout, uint32_t *fb, unsigned long long *fb_ctr,
               unsigned long long *c64 = nullptr) {
  if (!c64) c64 = &ctx->ctr_dev->n_cert64;
  if (n == 0) return IP_OK;
  hipStream_t st = ctx->stream;
  switch (L.d) {
    case 2: launch32_p<2, MODE>(st, Q, L, list, n, vt, vb, vraw, out, bout, fb, fb_ctr, c64); break;
    case 3: launch32_p<3, MODE>(st, Q, L, list, n, vt, vb, vraw, out, bout, fb, fb_ctr, c64); break;
    case 4: launch32_p<4, MODE>(st, Q, L, list, n, vt, vb, vraw, out, bout, fb, fb_ctr, c64); break;
    case 5: launch32_p<5, MODE>(st, Q, L, list, n, vt, vb, vraw, out, bout, fb, fb_ctr, c64); break;
    case 6: launch32_p<6, MODE>(st, Q, L, list, n, vt, vb, vraw, out, bout, fb, fb_ctr, c64); break;
    case 7: launch32_p<7, MODE>(st, Q, L, list, n, vt, vb, vraw, out, bout, fb, fb_ctr, c64); break;
    default: return ip_fail(ctx, IP_EINVAL, "dimension out of range");
  }
  IP_TRY_HIP(ctx, hipGetLastError());
  return IP_OK;
}

__global__ void zero_u64_kernel(unsigned long long *p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0ull;
}

__global__ void fill_f64_kernel(double *p, uint64_t n, double v) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

std::mutex g_scratch_mu;
void *g_scratch_ptr[64] = {nullptr};

template <int MODE>
int dispatch32_rbf(ip_ctx *ctx, const RbfDev &Q, const LatDev &L, const uint32_t *list, uint64_t n, VEnt *vt,
                   float *vb, const int32_t *vraw, double *out, double *bout, uint32_t *fb,
                   unsigned long long *fb_ctr) {
  if (n == 0) return IP_OK;
  const uint64_t blocks = std::min<uint64_t>((n + 255) / 256, 16384);
  hipStream_t st = ctx->stream;
#define IP_R32(DD)                                                                                              \
  hipLaunchKernelGGL((rbf32_kernel<DD, MODE>), dim3((unsigned)blocks), dim3(256), 0, st, Q, L, list, n, vt, vb, \
                     vraw, out, bout, fb, fb_ctr)
  switch (L.d) {
    case 2: IP_R32(2); break;
    case 3: IP_R32(3); break;
    case 4: IP_R32(4); break;
    case 5: IP_R32(5); break;
    case 6: IP_R32(6); break;
    case 7: IP_R32(7); break;
    default: return ip_fail(ctx, IP_EINVAL, "dimension out of range");
  }
#undef IP_R32
  IP_TRY_HIP(ctx, hipGetLastError());
  return IP_OK;
}

// The certified FP32 tier of problem p (polynomial or RBF form).
template <int MODE>
int dispatch32_p(ip_ctx *ctx, const ip_problem *p, const LatDev &L, const uint32_t *list, uint64_t n, VEnt *vt,
                 float *vb, const int32_t *vraw, double *out, double *bout, uint32_t *fb,
                 unsigned long long *fb_ctr, unsigned long long *c64 = nullptr) {
  if (p->f.kernel == IP_KERNEL_RBF)
    return dispatch32_rbf<MODE>(ctx, p->rbf, L, list, n, vt, vb, vraw, out, bout, fb, fb_ctr);
  return dispatch32<MODE>(ctx, p->poly, L, list, n, vt, vb, vraw, out, bout, fb, fb_ctr, c64);
}

// Canonical f and gradient at x (the order of ip.h's ip_seed_search): per
// support vector in index order, read as a wave-uniform record.
template <int D>
__device__ __forceinline__ double f_grad(const FDev &F, const double *x, double *g) {
  double acc = 0.0;
#pragma unroll
  for (int j = 0; j < D; ++j) g[j] = 0.0;
  if (F.kernel == IP_KERNEL_RBF) {
    const double m2g = -2.0 * F.gamma;
    for (int64_t i = 0; i < F.S; ++i) {
      const double *rec = F.rec + i * 8;
      double df[D], d2 = 0.0;
#pragma unroll
      for (int j = 0; j < D; ++j) {
        df[j] = x[j] - rec[j];
        d2 = fma(df[j], df[j], d2);
      }
      const double e = exp_own(-(F.gamma * d2));
      acc = fma(rec[D], e, acc);
      const double w = (rec[D] * e) * m2g;
#pragma unroll
      for (int j = 0; j < D; ++j) g[j] = fma(w, df[j], g[j]);
    }
    return acc + F.bias;
  }
  const double pg = (double)F.p * F.gamma;
  for (int64_t i = 0; i < F.S; ++i) {
    const double *rec = F.rec + i * 8;
    double dot = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) dot = fma(rec[j], x[j], dot);
    const double t = fma(F.gamma, dot, F.coef0);
    double tp1 = 1.0;
    if (F.p > 1) {
      tp1 = t;
      for (int r = 2; r < F.p; ++r) tp1 = tp1 * t;
    }
    acc = fma(rec[D], tp1 * t, acc);
    const double w = (rec[D] * tp1) * pg;
#pragma unroll
    for (int j = 0; j < D; ++j) g[j] = fma(w, rec[j], g[j]);
  }
  return acc + F.bias;
}

// Seed search (Sec. V-A: minimise |f| from given configurations), one lane
// per start: `iters` minimum-norm Newton steps, each clamped into the box;
// a zero gradient ends a lane's steps.  Then f at the final point.
template <int D>
__global__ __launch_bounds__(256) void seed_kernel(FDev F, LatDev L, const double *__restrict__ q0, uint64_t n,
                                                   int iters, double *__restrict__ q, double *__restrict__ fq) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    double x[D], g[D];
#pragma unroll
    for (int j = 0; j < D; ++j) x[j] = q0[i * D + j];
    for (int it = 0; it < iters; ++it) {
      const double fv = f_grad<D>(F, x, g);
      double n2 = 0.0;
#pragma unroll
      for (int j = 0; j < D; ++j) n2 = fma(g[j], g[j], n2);
      if (!(n2 > 0.0)) break;
      const double c = fv / n2;
#pragma unroll
      for (int j = 0; j < D; ++j) {
        const double v = fma(-c, g[j], x[j]);
        x[j] = v < L.lo[j] ? L.lo[j] : (v > L.hi[j] ? L.hi[j] : v);
      }
    }
    const double fv = f_grad<D>(F, x, g);
#pragma unroll
    for (int j = 0; j < D; ++j) q[i * D + j] = x[j];
    fq[i] = fv;
  }
}

}  // namespace

int ip_seed_search_impl(ip_ctx *ctx, const ip_problem *p, const double *q0, int64_t n, int32_t iters, double *q,
                        double *fq) {
  const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 16384);
#define IP_SD(DD)                                                                                            \
  hipLaunchKernelGGL((seed_kernel<DD>), dim3(blocks), dim3(256), 0, ctx->stream, p->f, p->fine, q0, (uint64_t)n, \
                     (int)iters, q, fq)
  switch (p->d) {
    case 2: IP_SD(2); break;
    case 3: IP_SD(3); break;
    case 4: IP_SD(4); break;
    case 5: IP_SD(5); break;
    case 6: IP_SD(6); break;
    case 7: IP_SD(7); break;
    default: return ip_fail(ctx, IP_EINVAL, "dimension out of range");
  }
#undef IP_SD
  IP_TRY_HIP(ctx, hipGetLastError());
  return IP_OK;
}

bool ip_has_fp32_form(const ip_problem *p) {
  return p->f.kernel == IP_KERNEL_RBF ? p->rbf.ok != 0 : p->poly.ok != 0;
}

int ip_noalloc_setup(ip_ctx *ctx) {
  if (ctx->device < 0 || ctx->device >= 64) return ip_fail(ctx, IP_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[ctx->device]) {
    // the device is current (ip_create set it): its own copy of the array
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return ip_hip(ctx, e == hipSuccess ? hipErrorInvalidSymbol : e, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[ctx->device] = ptr;
  }
  ctx->noalloc_scratch = g_scratch_ptr[ctx->device];
  return IP_OK;
}

// Same kernels and launch shapes as ip_feval_impl, with the fallback list and
// its counters in the device scratch and the FP64 pass sized on the device
// (it reads the list length the FP32 pass left), so nothing is allocated and
// nothing waits for the host.
int ip_feval_noalloc_impl(ip_ctx *ctx, const ip_problem *p, const int32_t *v_dev, int64_t n, int32_t prec,
                          double *f_dev, double *bound_dev) {
  if (!ctx->noalloc_scratch) return ip_fail(ctx, IP_EDEVICE, "device scratch not set up");
  hipStream_t st = ctx->stream;
  if (prec == IP_FP64 || !ip_has_fp32_form(p)) {
    if (bound_dev) {
      const uint64_t blocks = std::min<uint64_t>(((uint64_t)n + 255) / 256, 4096);
      hipLaunchKernelGGL(fill_f64_kernel, dim3((unsigned)blocks), dim3(256), 0, st, bound_dev, (uint64_t)n, 0.0);
      IP_TRY_HIP(ctx, hipGetLastError());
    }
    return dispatch64<1>(ctx, p->f, p->fine, nullptr, (uint64_t)n, nullptr, v_dev, f_dev);
  }
  unsigned long long *hdr = (unsigned long long *)ctx->noalloc_scratch;
  uint32_t *fbl = (uint32_t *)((unsigned char *)ctx->noalloc_scratch + 256);
  hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(64), 0, st, hdr, 2);
  IP_TRY_HIP(ctx, hipGetLastError());
  IP_TRY(dispatch32_p<1>(ctx, p, p->fine, nullptr, (uint64_t)n, nullptr, nullptr, v_dev, f_dev, bound_dev, fbl,
                         hdr, hdr + 1));
  return dispatch64<2>(ctx, p->f, p->fine, fbl, (uint64_t)n, nullptr, v_dev, f_dev, hdr);
}

int launch_feval64(ip_ctx *ctx, const ip_problem *p, const LatDev &L, const uint32_t *list, uint64_t n_list,
                   VEnt *vt) {
  return dispatch64<0>(ctx, p->f, L, list, n_list, (const uint64_t *)vt, nullptr, (double *)vt + 1);
}

int launch_feval64_dev(ip_ctx *ctx, const ip_problem *p, const LatDev &L, const uint32_t *list, uint64_t n_max,
                       const unsigned long long *n_dev, VEnt *vt) {
  return dispatch64<0>(ctx, p->f, L, list, n_max, (const uint64_t *)vt, nullptr, (double *)vt + 1, n_dev);
}

int launch_feval64_raw(ip_ctx *ctx, const ip_problem *p, const LatDev &L, const int32_t *v, uint64_t n,
                       double *out) {
  return dispatch64<1>(ctx, p->f, L, nullptr, n, nullptr, v, out);
}

int launch_feval32(ip_ctx *ctx, const ip_problem *p, const LatDev &L, const uint32_t *list, uint64_t n_list,
                   VEnt *vt, float *vb, uint32_t *fb, unsigned long long *fb_ctr) {
  return dispatch32_p<0>(ctx, p, L, list, n_list, vt, vb, nullptr, nullptr, nullptr, fb, fb_ctr);
}

int launch_set_vb(ip_ctx *ctx, const uint32_t *list, uint64_t n, float *vb, float v) {
  if (n == 0) return IP_OK;
  uint64_t blocks = (n + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(set_vb_kernel, dim3((unsigned)blocks), dim3(256), 0, ctx->stream, list, n, vb, v);
  IP_TRY_HIP(ctx, hipGetLastError());
  return IP_OK;
}

int ip_feval_impl(ip_ctx *ctx, const ip_problem *p, const int32_t *v_dev, int64_t n, int32_t prec,
                  double *f_dev, double *bound_dev) {
  if (prec == IP_FP64 || !ip_has_fp32_form(p)) {
    if (bound_dev) IP_TRY_HIP(ctx, hipMemsetAsync(bound_dev, 0, sizeof(double) * (size_t)n, ctx->stream));
    return dispatch64<1>(ctx, p->f, p->fine, nullptr, (uint64_t)n, nullptr, v_dev, f_dev);
  }
  // FP32 pass, then canonical FP64 for the unsettled indices
  if (n >= (1ll << 32)) return ip_fail(ctx, IP_EINVAL, "ip_feval: at most 2^32 - 1 vertices per call");
  double *bnd = bound_dev;
  void *tmp_b = nullptr, *fbl = nullptr;
  if (!bnd) {
    IP_TRY(ip_dalloc(ctx, &tmp_b, sizeof(double) * (size_t)n));
    bnd = (double *)tmp_b;
  }
  if (ip_dalloc(ctx, &fbl, sizeof(uint32_t) * (size_t)n) != IP_OK) {
    ip_dfree(ctx, tmp_b);
    return IP_ENOMEM;
  }
  IP_TRY_HIP(ctx, hipMemsetAsync(ctx->ctr_dev, 0, sizeof(Counters), ctx->stream));
  int rc = dispatch32_p<1>(ctx, p, p->fine, nullptr, (uint64_t)n, nullptr, nullptr, v_dev, f_dev, bnd,
                           (uint32_t *)fbl, &ctx->ctr_dev->n_fb);
  unsigned long long nfb = 0;
  if (rc == IP_OK) {
    hipError_t e = hipMemcpyAsync(ctx->ctr_host, ctx->ctr_dev, sizeof(Counters), hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) rc = ip_hip(ctx, e, "ip_feval counters");
    nfb = ctx->ctr_host->n_fb;
  }
  if (rc == IP_OK) rc = dispatch64<2>(ctx, p->f, p->fine, (const uint32_t *)fbl, nfb, nullptr, v_dev, f_dev);
  (void)hipStreamSynchronize(ctx->stream);
  ip_dfree(ctx, tmp_b);
  ip_dfree(ctx, fbl);
  ctx->last_fallback = (int64_t)nfb;
  return rc;
}
