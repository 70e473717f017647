// Order of the coarse n-simplices of a batch trace (Sec. V-B: the batches of
// Sigma).  The Sigma kernel appends keys in whatever order its waves finish;
// sorting them by the Morton code of the base vertex puts simplices that
// share faces and fine vertices next to each other, so that the waves working
// at the same time touch the same rows of the global edge set and of the
// batch vertex table, and those rows stay in cache.  The traced set does not
// depend on the order (the output is a set); the order of the cells does.
#include <hipcub/hipcub.hpp>

#include "ip_internal.h"

namespace {

// Sort key of a Sigma key (packed base vertex above LB Lehmer bits): the
// base vertex's D fields of B bits interleaved bit by bit (bit b of field j
// to bit b D + j), above the same Lehmer bits.  A bijection on the used
// bits, so sorting the pairs orders the keys themselves.
__global__ void morton_kernel(const uint64_t *__restrict__ key, uint64_t n, int D, int B, int LB,
                              uint64_t *__restrict__ skey) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t k = key[i];
    const uint64_t v = k >> LB;
    uint64_t m = 0;
    for (int b = 0; b < B; ++b)
      for (int j = 0; j < D; ++j) m |= ((v >> (j * B + b)) & 1ull) << (b * D + j);
    skey[i] = (m << LB) | (k & ((1ull << LB) - 1ull));
  }
}

}  // namespace

int ip_sort_sigma(ip_ctx *ctx, uint64_t *sig, uint64_t n, int D, int B, int LB) {
  if (n < 2) return IP_OK;
  const int bits = D * B + LB;
  if (bits > 64) return ip_fail(ctx, IP_ERANGE, "Sigma keys wider than 64 bits");
  // sort keys, sorted keys and sorted Sigma keys (three arrays of n), then
  // the sort's temporary storage
  size_t tmp_bytes = 0;
  hipError_t e = hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, (const uint64_t *)nullptr,
                                                    (uint64_t *)nullptr, (const uint64_t *)nullptr,
                                                    (uint64_t *)nullptr, (int)n, 0, bits, ctx->stream);
  if (e != hipSuccess) return ip_hip(ctx, e, "hipcub sort (size query)");
  if (n > 0x7fffffffull) return ip_fail(ctx, IP_EINVAL, "too many coarse n-simplices to sort");
  void *buf = nullptr;
  const size_t arr = ((size_t)n * 8 + 255) & ~(size_t)255;
  IP_TRY(ip_dalloc(ctx, &buf, 3 * arr + tmp_bytes));
  uint64_t *skey = (uint64_t *)buf;
  uint64_t *skey_out = (uint64_t *)((char *)buf + arr);
  uint64_t *val_out = (uint64_t *)((char *)buf + 2 * arr);
  void *tmp = (char *)buf + 3 * arr;
  const unsigned blocks = (unsigned)std::min<uint64_t>((n + 255) / 256, 16384);
  hipLaunchKernelGGL(morton_kernel, dim3(blocks), dim3(256), 0, ctx->stream, (const uint64_t *)sig, n, D, B, LB, skey);
  e = hipGetLastError();
  if (e == hipSuccess)
    e = hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, (const uint64_t *)skey, skey_out, (const uint64_t *)sig,
                                           val_out, (int)n, 0, bits, ctx->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(sig, val_out, (size_t)n * 8, hipMemcpyDeviceToDevice, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) {
    (void)hipStreamSynchronize(ctx->stream);
    ip_dfree(ctx, buf);
    return ip_hip(ctx, e, "sorting Sigma");
  }
  ip_dfree(ctx, buf);
  return IP_OK;
}
