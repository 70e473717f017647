// f evaluation at lattice vertices (the edge sign tests of Sec. V-A and the
// subdivision vertices of Sec. V-B need f at every vertex they touch).
//
// FP64 kernel: one lane per vertex, R vertices per lane (register blocking),
// support vectors consumed in index order so the accumulation order is the
// canonical one of ip.h and the result is bit-identical on every device.
// Every lane of a wave reads the same 64-byte support-vector record at the
// same time, so the record is a wave-uniform load served from the scalar
// cache into SGPRs and used as the scalar operand of v_fma_f64.
#include "ip_internal.h"

namespace {

template <int D, int P, int R, bool FROM_KEYS>
__global__ __launch_bounds__(256) void feval64_kernel(FDev F, LatDev L, const uint32_t *__restrict__ list,
                                                      uint64_t n, const uint64_t *__restrict__ keys,
                                                      const int32_t *__restrict__ vraw,
                                                      double *__restrict__ out) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x * R;
  for (uint64_t base = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * R; base < n; base += stride) {
    double x[R][D];
    uint64_t dst[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      uint64_t i = base + r < n ? base + r : n - 1;
      int32_t v[D];
      if (FROM_KEYS) {
        uint32_t s = list[i];
        dst[r] = s;
        vunpack<D>(L, keys[s], v);
      } else {
        dst[r] = i;
#pragma unroll
        for (int j = 0; j < D; ++j) v[j] = vraw[i * D + j];
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
      if (base + r < n) out[dst[r]] = acc[r] + F.bias;
  }
}

template <int D, int P, bool FROM_KEYS>
void launch64(hipStream_t st, const FDev &F, const LatDev &L, const uint32_t *list, uint64_t n,
              const uint64_t *keys, const int32_t *vraw, double *out) {
  constexpr int R = D <= 4 ? 4 : 2;
  const uint64_t threads = (n + R - 1) / R;
  uint64_t blocks = (threads + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  if (blocks == 0) return;
  hipLaunchKernelGGL((feval64_kernel<D, P, R, FROM_KEYS>), dim3((unsigned)blocks), dim3(256), 0, st, F, L,
                     list, n, keys, vraw, out);
}

template <int D, bool FROM_KEYS>
void launch64_p(hipStream_t st, const FDev &F, const LatDev &L, const uint32_t *list, uint64_t n,
                const uint64_t *keys, const int32_t *vraw, double *out) {
  switch (F.p) {
    case 1: launch64<D, 1, FROM_KEYS>(st, F, L, list, n, keys, vraw, out); break;
    case 2: launch64<D, 2, FROM_KEYS>(st, F, L, list, n, keys, vraw, out); break;
    case 3: launch64<D, 3, FROM_KEYS>(st, F, L, list, n, keys, vraw, out); break;
    case 4: launch64<D, 4, FROM_KEYS>(st, F, L, list, n, keys, vraw, out); break;
    default: launch64<D, 0, FROM_KEYS>(st, F, L, list, n, keys, vraw, out); break;
  }
}

template <bool FROM_KEYS>
int dispatch64(ip_ctx *ctx, const FDev &F, const LatDev &L, const uint32_t *list, uint64_t n,
               const uint64_t *keys, const int32_t *vraw, double *out) {
  if (n == 0) return IP_OK;
  hipStream_t st = ctx->stream;
  switch (L.d) {
    case 2: launch64_p<2, FROM_KEYS>(st, F, L, list, n, keys, vraw, out); break;
    case 3: launch64_p<3, FROM_KEYS>(st, F, L, list, n, keys, vraw, out); break;
    case 4: launch64_p<4, FROM_KEYS>(st, F, L, list, n, keys, vraw, out); break;
    case 5: launch64_p<5, FROM_KEYS>(st, F, L, list, n, keys, vraw, out); break;
    case 6: launch64_p<6, FROM_KEYS>(st, F, L, list, n, keys, vraw, out); break;
    case 7: launch64_p<7, FROM_KEYS>(st, F, L, list, n, keys, vraw, out); break;
    default: return ip_fail(ctx, IP_EINVAL, "dimension out of range");
  }
  IP_TRY_HIP(ctx, hipGetLastError());
  return IP_OK;
}

}  // namespace

int launch_feval64(ip_ctx *ctx, const ip_problem *p, const LatDev &L, const uint32_t *list, uint64_t n_list,
                   const uint64_t *vt_keys, double *vt_vals) {
  return dispatch64<true>(ctx, p->f, L, list, n_list, vt_keys, nullptr, vt_vals);
}

int ip_feval_impl(ip_ctx *ctx, const ip_problem *p, const int32_t *v_dev, int64_t n, int32_t prec,
                  double *f_dev, double *bound_dev) {
  if (prec != IP_FP64) return ip_fail(ctx, IP_EINVAL, "ip_feval: precision not supported yet");
  if (bound_dev) IP_TRY_HIP(ctx, hipMemsetAsync(bound_dev, 0, sizeof(double) * (size_t)n, ctx->stream));
  return dispatch64<false>(ctx, p->f, p->fine, nullptr, (uint64_t)n, nullptr, v_dev, f_dev);
}
