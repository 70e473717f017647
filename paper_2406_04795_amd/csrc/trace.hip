// Manifold tracing on the Coxeter triangulation (Sec. V-A, Figs. 3-4).
//
// State lives in three device hash tables / lists:
//   VT  vertex table: packed vertex key -> f (FP64; NaN payload = pending).
//       Every lattice vertex the search touches is evaluated once.
//   ET  edge table: packed canonical edge keys (the visited set).
//   OUT append-only list of traced edges; the frontier of a level is a
//       contiguous range of it (the edges inserted by the previous level).
// One breadth-first level = pass 1 (enumerate the 2-cofaces of the frontier
// edges, insert their third vertices into VT, list the new ones), f
// evaluation of the new vertices, pass 2 (for each coface pick the one other
// edge that changes sign, insert it into ET, append winners to OUT).
// The host reads a small counter block after each pass to size the next
// launch and to grow tables; growth replays a pass, which is idempotent.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "ip_internal.h"

namespace {

constexpr int kBlock = 256;

__global__ void fill_u64_kernel(uint64_t *p, uint64_t n, uint64_t v) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void zero_counter_kernel(unsigned long long *p) { *p = 0ull; }

template <int D>
__device__ void locate(const LatDev &L, const double *y, int32_t *v, int32_t *w) {
  double t[D], fr[D];
#pragma unroll
  for (int k = 0; k < D; ++k) t[k] = y[k] - L.o[k];
#pragma unroll
  for (int j = 0; j < D; ++j) {
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) acc = fma(L.Minv[j * 8 + k], t[k], acc);
    if (L.mul > 1) acc = acc / (double)L.mul;
    double fl = floor(acc);
    v[j] = (int32_t)fl;
    fr[j] = acc - fl;
  }
  // indices by descending fractional part, ties by ascending index
#pragma unroll
  for (int j = 0; j < D; ++j) w[j] = j;
  for (int i = 1; i < D; ++i) {
    int32_t cur = w[i];
    int j = i - 1;
    while (j >= 0 && fr[w[j]] < fr[cur]) {
      w[j + 1] = w[j];
      --j;
    }
    w[j + 1] = cur;
  }
}

// Sec. V-A "find all n-simplices": locate each seed and register the
// vertices of its n-simplex that lie in the domain.
template <int D>
__global__ void seed_vertices_kernel(LatDev L, const double *seeds, int64_t ns, uint64_t *vt_keys,
                                     uint64_t vt_mask, uint32_t *eval_list, Counters *ctr) {
  int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= ns) return;
  int32_t v[D], w[D];
  locate<D>(L, seeds + s * D, v, w);
  for (int m = 0; m <= D; ++m) {
    if (m > 0) v[w[m - 1]] += 1;
    double x[D];
    lat_coords<D>(L, v, x);
    if (!lat_in_box<D>(L, x)) continue;
    uint64_t slot;
    int r = ht_insert(vt_keys, vt_mask, vpack<D>(L, v), &slot);
    if (r == 1) {
      unsigned long long idx = atomicAdd(&ctr->n_eval, 1ull);
      eval_list[idx] = (uint32_t)slot;
      atomicAdd(&ctr->vt_count, 1ull);
    } else if (r < 0) {
      atomicOr(&ctr->vt_fail, 1u);
    }
  }
}

// Sec. V-A "find all interesting n-simplices' edges" + "hash all edges".
template <int D>
__global__ void seed_edges_kernel(LatDev L, const double *seeds, int64_t ns, const uint64_t *vt_keys,
                                  const double *vt_vals, uint64_t vt_mask, uint64_t *et_keys,
                                  uint64_t et_mask, uint64_t *out, Counters *ctr) {
  int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= ns) return;
  int32_t v[D], w[D], u[D + 1][D];
  locate<D>(L, seeds + s * D, v, w);
#pragma unroll
  for (int j = 0; j < D; ++j) u[0][j] = v[j];
  for (int m = 0; m < D; ++m) {
#pragma unroll
    for (int j = 0; j < D; ++j) u[m + 1][j] = u[m][j];
    u[m + 1][w[m]] += 1;
  }
  double fv[D + 1];
  bool inb[D + 1];
  for (int m = 0; m <= D; ++m) {
    int64_t h = vin_range<D>(L, u[m]) ? ht_find(vt_keys, vt_mask, vpack<D>(L, u[m])) : -1;
    inb[m] = h >= 0;
    fv[m] = inb[m] ? vt_vals[h] : 0.0;
  }
  for (int a = 0; a <= D; ++a)
    for (int b = a + 1; b <= D; ++b) {
      if (!inb[a] || !inb[b]) continue;
      bool sa = !(fv[a] < 0.0), sb = !(fv[b] < 0.0);
      if (sa == sb) continue;
      int32_t vm[D];
      uint32_t mask;
      bool a_min = edge_canon<D>(u[a], u[b], vm, &mask);
      uint64_t key = ekey<D>(L, vm, mask);
      uint64_t slot;
      int r = ht_insert(et_keys, et_mask, key, &slot);
      if (r == 1) {
        unsigned long long idx = atomicAdd(&ctr->n_out, 1ull);
        out[idx] = key | ((a_min ? sa : sb) ? IP_SIGN_BIT : 0ull);
      } else if (r < 0) {
        atomicOr(&ctr->et_fail, 1u);
      }
    }
}

// Frontier expansion (Sec. V-A "find all cofaces" / "find all interesting
// cofaces' edges" / "hash all edges").  Each wave takes 64 frontier edges,
// prefix-sums their coface counts and walks the flattened (edge, coface)
// list 64 at a time, so lanes stay busy whatever the mix of edge classes.
//   EDGES = false: pass 1, register third vertices in VT.
//   EDGES = true : pass 2, sign test and insertion of the new edge.
template <int D, bool EDGES>
__global__ __launch_bounds__(kBlock) void expand_kernel(LatDev L, const uint64_t *__restrict__ front,
                                                        uint64_t lo, uint64_t hi, uint64_t *vt_keys,
                                                        const double *__restrict__ vt_vals, uint64_t vt_mask,
                                                        uint32_t *eval_list, uint64_t *et_keys,
                                                        uint64_t et_mask, uint64_t *out, Counters *ctr) {
  const int lane = threadIdx.x & 63;
  const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const uint64_t n_waves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  const uint64_t nchunks = (hi - lo + 63) >> 6;
  const uint64_t below = (1ull << lane) - 1ull;
  unsigned long long cof_acc = 0, new_acc = 0;
  for (uint64_t ch = wave; ch < nchunks; ch += n_waves) {
    const uint64_t ei = lo + ch * 64 + lane;
    uint64_t e = 0;
    int cnt = 0;
    if (ei < hi) {
      e = front[ei];
      cnt = n_cofaces2<D>((uint32_t)((e & ~IP_SIGN_BIT) >> (D * L.B)) & ((1u << D) - 1u));
    }
    int incl = cnt;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      int t = __shfl_up(incl, off, 64);
      if (lane >= off) incl += t;
    }
    const int excl = incl - cnt;
    const int total = __shfl(incl, 63, 64);
    cof_acc += (unsigned long long)total;
    for (int base = 0; base < total; base += 64) {
      const int idx = base + lane;
      const bool valid = idx < total;
      // owner edge: largest j with excl[j] <= idx
      int j = 0;
#pragma unroll
      for (int step = 32; step; step >>= 1) {
        int pc = __shfl(excl, j + step, 64);
        if (pc <= idx) j += step;
      }
      const uint64_t me = shfl64(e, j);
      const int r = idx - __shfl(excl, j, 64);
      bool is_new = false;
      uint64_t payload = 0;
      if (valid) {
        int32_t v[D], c[D];
        uint32_t R;
        eunpack<D>(L, me, v, &R);
        coface_vertex<D>(v, R, r, c);
        if (!EDGES) {
          double x[D];
          lat_coords<D>(L, c, x);
          if (lat_in_box<D>(L, x)) {
            uint64_t slot;
            int ins = ht_insert(vt_keys, vt_mask, vpack<D>(L, c), &slot);
            if (ins == 1) {
              is_new = true;
              payload = slot;
            } else if (ins < 0) {
              atomicOr(&ctr->vt_fail, 1u);
            }
          }
        } else {
          const int64_t h = vin_range<D>(L, c) ? ht_find(vt_keys, vt_mask, vpack<D>(L, c)) : -1;
          if (h >= 0) {
            const bool sc = !(vt_vals[h] < 0.0);
            const bool sa = (me & IP_SIGN_BIT) != 0;
            // exactly one of (a,c), (b,c) changes sign: the one whose other
            // end has the sign c does not have (Sec. V-A, two edges of a
            // triangle cross the manifold)
            int32_t other[D];
            bool so;
            if (sc != sa) {
#pragma unroll
              for (int q = 0; q < D; ++q) other[q] = v[q];
              so = sa;
            } else {
#pragma unroll
              for (int q = 0; q < D; ++q) other[q] = v[q] + (int32_t)((R >> q) & 1u);
              so = !sa;
            }
            int32_t vm[D];
            uint32_t mask;
            const bool other_min = edge_canon<D>(other, c, vm, &mask);
            const uint64_t key = ekey<D>(L, vm, mask);
            uint64_t slot;
            int ins = ht_insert(et_keys, et_mask, key, &slot);
            if (ins == 1) {
              is_new = true;
              payload = key | ((other_min ? so : sc) ? IP_SIGN_BIT : 0ull);
            } else if (ins < 0) {
              atomicOr(&ctr->et_fail, 1u);
            }
          }
        }
      }
      // wave-aggregated append
      const uint64_t bal = __ballot(is_new);
      if (bal) {
        const int nb = __popcll(bal);
        const int leader = __ffsll((long long)bal) - 1;
        unsigned long long b0 = 0;
        if (lane == leader) b0 = atomicAdd(EDGES ? &ctr->n_out : &ctr->n_eval, (unsigned long long)nb);
        b0 = shfl64(b0, leader);
        if (is_new) {
          const unsigned long long pos = b0 + (unsigned long long)__popcll(bal & below);
          if (EDGES)
            out[pos] = payload;
          else
            eval_list[pos] = (uint32_t)payload;
        }
        new_acc += (unsigned long long)nb;
      }
    }
  }
  if (lane == 0) {
    if (!EDGES) {
      if (cof_acc) atomicAdd(&ctr->n_cof, cof_acc);
      if (new_acc) atomicAdd(&ctr->vt_count, new_acc);
    }
  }
}

// Sec. V-B intersection points: t = f_a/(f_a - f_b), p = x_a + t (x_b - x_a).
template <int D>
__global__ void points_kernel(LatDev L, uint64_t *keys, uint64_t n, const uint64_t *vt_keys,
                              const double *vt_vals, uint64_t vt_mask, double *pts, int64_t ld) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t key = keys[i] & ~IP_SIGN_BIT;
    keys[i] = key;
    int32_t a[D], b[D];
    uint32_t R;
    eunpack<D>(L, key, a, &R);
#pragma unroll
    for (int j = 0; j < D; ++j) b[j] = a[j] + (int32_t)((R >> j) & 1u);
    int64_t ha = ht_find(vt_keys, vt_mask, vpack<D>(L, a));
    int64_t hb = ht_find(vt_keys, vt_mask, vpack<D>(L, b));
    double fa = ha >= 0 ? vt_vals[ha] : NAN;
    double fb = hb >= 0 ? vt_vals[hb] : NAN;
    double xa[D], xb[D];
    lat_coords<D>(L, a, xa);
    lat_coords<D>(L, b, xb);
    double t = fa / (fa - fb);
#pragma unroll
    for (int j = 0; j < D; ++j) pts[(int64_t)j * ld + (int64_t)i] = fma(t, xb[j] - xa[j], xa[j]);
  }
}

__global__ void vt_rehash_kernel(const uint64_t *ok, const double *ov, uint64_t ocap, uint64_t *nk, double *nv,
                                 uint64_t nmask, Counters *ctr) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ocap; i += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t k = ok[i];
    if (k == IP_EMPTY_KEY) continue;
    uint64_t slot;
    int r = ht_insert(nk, nmask, k, &slot);
    if (r >= 0)
      nv[slot] = ov[i];
    else
      atomicOr(&ctr->vt_fail, 1u);
  }
}

__global__ void vt_scan_pending_kernel(const uint64_t *keys, const double *vals, uint64_t cap, uint32_t *list,
                                       Counters *ctr) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cap; i += (uint64_t)gridDim.x * blockDim.x) {
    if (keys[i] == IP_EMPTY_KEY) continue;
    uint64_t bits = __double_as_longlong(vals[i]);
    if (bits == IP_UNEVAL_BITS) {
      unsigned long long idx = atomicAdd(&ctr->n_eval, 1ull);
      list[idx] = (uint32_t)i;
    }
  }
}

__global__ void et_rebuild_kernel(const uint64_t *out, uint64_t n, uint64_t *et, uint64_t mask, Counters *ctr) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t slot;
    if (ht_insert(et, mask, out[i] & ~IP_SIGN_BIT, &slot) < 0) atomicOr(&ctr->et_fail, 1u);
  }
}

unsigned grid_for(uint64_t n, unsigned cap = 16384) {
  uint64_t b = (n + kBlock - 1) / kBlock;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (unsigned)b;
}

uint64_t pow2_at_least(uint64_t x) {
  uint64_t c = 1024;
  while (c < x) c <<= 1;
  return c;
}

// ---------------------------------------------------------------------------
// Host driver
// ---------------------------------------------------------------------------
struct Run {
  ip_ctx *ctx;
  const ip_problem *p;
  LatDev L;
  uint64_t *vt_keys = nullptr;
  double *vt_vals = nullptr;
  uint64_t vt_cap = 0;
  uint64_t *et_keys = nullptr;
  uint64_t et_cap = 0;
  uint32_t *eval = nullptr;
  uint64_t eval_cap = 0;
  uint64_t *out = nullptr;
  uint64_t out_cap = 0;
  int regrows = 0;
};

// Accumulates the stream time between two event records (read after the
// next synchronisation of the stream).
struct Timer {
  hipEvent_t a = nullptr, b = nullptr;
  bool pending = false;
  double *acc = nullptr;
  ~Timer() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
  int start(ip_ctx *ctx, double *into) {
    if (!a) {
      IP_TRY_HIP(ctx, hipEventCreate(&a));
      IP_TRY_HIP(ctx, hipEventCreate(&b));
    }
    IP_TRY(flush(ctx));
    acc = into;
    IP_TRY_HIP(ctx, hipEventRecord(a, ctx->stream));
    return IP_OK;
  }
  int stop(ip_ctx *ctx) {
    IP_TRY_HIP(ctx, hipEventRecord(b, ctx->stream));
    pending = true;
    return IP_OK;
  }
  int flush(ip_ctx *ctx) {
    if (!pending) return IP_OK;
    IP_TRY_HIP(ctx, hipEventSynchronize(b));
    float ms = 0.0f;
    IP_TRY_HIP(ctx, hipEventElapsedTime(&ms, a, b));
    *acc += ms;
    pending = false;
    return IP_OK;
  }
};

int read_ctr(ip_ctx *ctx) {
  IP_TRY_HIP(ctx, hipMemcpyAsync(ctx->ctr_host, ctx->ctr_dev, sizeof(Counters), hipMemcpyDeviceToHost, ctx->stream));
  IP_TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return IP_OK;
}

int zero_field(ip_ctx *ctx, unsigned long long *field) {
  hipLaunchKernelGGL(zero_counter_kernel, dim3(1), dim3(1), 0, ctx->stream, field);
  IP_TRY_HIP(ctx, hipGetLastError());
  return IP_OK;
}

int fill(ip_ctx *ctx, void *p, uint64_t n, uint64_t v) {
  if (n == 0) return IP_OK;
  hipLaunchKernelGGL(fill_u64_kernel, dim3(grid_for(n)), dim3(kBlock), 0, ctx->stream, (uint64_t *)p, n, v);
  IP_TRY_HIP(ctx, hipGetLastError());
  return IP_OK;
}

int alloc(ip_ctx *ctx, void **p, size_t bytes) {
  hipError_t e = hipMalloc(p, bytes < 256 ? 256 : bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return ip_fail(ctx, IP_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
  }
  return IP_OK;
}

// Vertex table of capacity cap (power of two), reusing the context buffers.
int vt_init(Run &s, uint64_t cap) {
  ip_ctx *ctx = s.ctx;
  IP_TRY(ip_ensure(ctx, ctx->vt_keys, cap * 8));
  IP_TRY(ip_ensure(ctx, ctx->vt_vals, cap * 8));
  IP_TRY(ip_ensure(ctx, ctx->eval_list, cap * 4));
  s.vt_keys = (uint64_t *)ctx->vt_keys.p;
  s.vt_vals = (double *)ctx->vt_vals.p;
  s.eval = (uint32_t *)ctx->eval_list.p;
  s.vt_cap = cap;
  s.eval_cap = cap;
  IP_TRY(fill(ctx, s.vt_keys, cap, IP_EMPTY_KEY));
  IP_TRY(fill(ctx, s.vt_vals, cap, IP_UNEVAL_BITS));
  return IP_OK;
}

int et_init(Run &s, uint64_t cap) {
  ip_ctx *ctx = s.ctx;
  IP_TRY(ip_ensure(ctx, ctx->et_keys, cap * 8));
  s.et_keys = (uint64_t *)ctx->et_keys.p;
  s.et_cap = cap;
  IP_TRY(fill(ctx, s.et_keys, cap, IP_EMPTY_KEY));
  return IP_OK;
}

// Grow VT to new_cap: rehash into fresh buffers and rebuild the pending list.
int vt_grow(Run &s, uint64_t new_cap) {
  ip_ctx *ctx = s.ctx;
  void *nk = nullptr, *nv = nullptr, *nl = nullptr;
  IP_TRY(alloc(ctx, &nk, new_cap * 8));
  IP_TRY(alloc(ctx, &nv, new_cap * 8));
  IP_TRY(alloc(ctx, &nl, new_cap * 4));
  IP_TRY(fill(ctx, nk, new_cap, IP_EMPTY_KEY));
  IP_TRY(fill(ctx, nv, new_cap, IP_UNEVAL_BITS));
  hipLaunchKernelGGL(vt_rehash_kernel, dim3(grid_for(s.vt_cap)), dim3(kBlock), 0, ctx->stream, s.vt_keys,
                     s.vt_vals, s.vt_cap, (uint64_t *)nk, (double *)nv, new_cap - 1, ctx->ctr_dev);
  IP_TRY_HIP(ctx, hipGetLastError());
  IP_TRY(zero_field(ctx, &ctx->ctr_dev->n_eval));
  hipLaunchKernelGGL(vt_scan_pending_kernel, dim3(grid_for(new_cap)), dim3(kBlock), 0, ctx->stream,
                     (const uint64_t *)nk, (const double *)nv, new_cap, (uint32_t *)nl, ctx->ctr_dev);
  IP_TRY_HIP(ctx, hipGetLastError());
  IP_TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));
  (void)hipFree(ctx->vt_keys.p);
  (void)hipFree(ctx->vt_vals.p);
  (void)hipFree(ctx->eval_list.p);
  ctx->vt_keys = {nk, new_cap * 8};
  ctx->vt_vals = {nv, new_cap * 8};
  ctx->eval_list = {nl, new_cap * 4};
  s.vt_keys = (uint64_t *)nk;
  s.vt_vals = (double *)nv;
  s.eval = (uint32_t *)nl;
  s.vt_cap = s.eval_cap = new_cap;
  ++s.regrows;
  return IP_OK;
}

int et_grow(Run &s, uint64_t new_cap, uint64_t n_out) {
  ip_ctx *ctx = s.ctx;
  void *nk = nullptr;
  IP_TRY(alloc(ctx, &nk, new_cap * 8));
  IP_TRY(fill(ctx, nk, new_cap, IP_EMPTY_KEY));
  hipLaunchKernelGGL(et_rebuild_kernel, dim3(grid_for(n_out)), dim3(kBlock), 0, ctx->stream, s.out, n_out,
                     (uint64_t *)nk, new_cap - 1, ctx->ctr_dev);
  IP_TRY_HIP(ctx, hipGetLastError());
  IP_TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));
  (void)hipFree(ctx->et_keys.p);
  ctx->et_keys = {nk, new_cap * 8};
  s.et_keys = (uint64_t *)nk;
  s.et_cap = new_cap;
  ++s.regrows;
  return IP_OK;
}

int out_reserve(Run &s, uint64_t need, uint64_t n_used) {
  if (need <= s.out_cap) return IP_OK;
  ip_ctx *ctx = s.ctx;
  uint64_t cap = std::max<uint64_t>(need, s.out_cap * 2);
  void *nb = nullptr;
  IP_TRY(alloc(ctx, &nb, cap * 8));
  if (n_used)
    IP_TRY_HIP(ctx, hipMemcpyAsync(nb, s.out, n_used * 8, hipMemcpyDeviceToDevice, ctx->stream));
  IP_TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (s.out) (void)hipFree(s.out);
  s.out = (uint64_t *)nb;
  s.out_cap = cap;
  return IP_OK;
}

// Evaluate the pending vertices listed in s.eval[0 .. n).
int eval_pending(Run &s, uint64_t n) {
  return launch_feval64(s.ctx, s.p, s.L, s.eval, n, s.vt_keys, s.vt_vals);
}

template <int D>
int level_pass1(Run &s, uint64_t lo, uint64_t hi) {
  ip_ctx *ctx = s.ctx;
  unsigned grid = grid_for((hi - lo) * 4, 8192);
  hipLaunchKernelGGL((expand_kernel<D, false>), dim3(grid), dim3(kBlock), 0, ctx->stream, s.L, s.out, lo, hi,
                     s.vt_keys, s.vt_vals, s.vt_cap - 1, s.eval, s.et_keys, s.et_cap - 1, s.out, ctx->ctr_dev);
  IP_TRY_HIP(ctx, hipGetLastError());
  return IP_OK;
}

template <int D>
int level_pass2(Run &s, uint64_t lo, uint64_t hi) {
  ip_ctx *ctx = s.ctx;
  unsigned grid = grid_for((hi - lo) * 4, 8192);
  hipLaunchKernelGGL((expand_kernel<D, true>), dim3(grid), dim3(kBlock), 0, ctx->stream, s.L, s.out, lo, hi,
                     s.vt_keys, s.vt_vals, s.vt_cap - 1, s.eval, s.et_keys, s.et_cap - 1, s.out, ctx->ctr_dev);
  IP_TRY_HIP(ctx, hipGetLastError());
  return IP_OK;
}

// Direct trace on lattice s.L (fine, or coarse in batch mode).  On return
// s.out[0 .. *n_out) holds the traced edges and VT holds f at their ends.
template <int D>
int trace_direct(Run &s, ip_stats &st, uint64_t *n_out_ret) {
  ip_ctx *ctx = s.ctx;
  const ip_problem *p = s.p;
  Counters *c = ctx->ctr_host;
  Timer tf, tx;
  IP_TRY_HIP(ctx, hipMemsetAsync(ctx->ctr_dev, 0, sizeof(Counters), ctx->stream));
  // locate
  const unsigned sg = (unsigned)((p->n_seeds + 127) / 128);
  for (;;) {
    hipLaunchKernelGGL((seed_vertices_kernel<D>), dim3(sg), dim3(128), 0, ctx->stream, s.L, p->seeds_dev,
                       p->n_seeds, s.vt_keys, s.vt_cap - 1, s.eval, ctx->ctr_dev);
    IP_TRY_HIP(ctx, hipGetLastError());
    IP_TRY(read_ctr(ctx));
    if (!c->vt_fail) break;
    IP_TRY(zero_field(ctx, (unsigned long long *)&ctx->ctr_dev->vt_fail));
    IP_TRY(vt_grow(s, s.vt_cap * 4));
  }
  IP_TRY(tf.start(ctx, &st.ms_feval));
  IP_TRY(eval_pending(s, c->n_eval));
  IP_TRY(tf.stop(ctx));
  IP_TRY(out_reserve(s, (uint64_t)p->n_seeds * (D + 1) * D / 2 + 1024, 0));
  for (;;) {
    hipLaunchKernelGGL((seed_edges_kernel<D>), dim3(sg), dim3(128), 0, ctx->stream, s.L, p->seeds_dev,
                       p->n_seeds, s.vt_keys, s.vt_vals, s.vt_cap - 1, s.et_keys, s.et_cap - 1, s.out,
                       ctx->ctr_dev);
    IP_TRY_HIP(ctx, hipGetLastError());
    IP_TRY(read_ctr(ctx));
    if (!c->et_fail) break;
    IP_TRY(zero_field(ctx, (unsigned long long *)&ctx->ctr_dev->et_fail));
    IP_TRY(et_grow(s, s.et_cap * 4, c->n_out));
  }
  uint64_t lo = 0, hi = c->n_out;
  int levels = 0;
  uint64_t cof_total = 0;
  while (hi > lo) {
    ++levels;
    // pass 1: new vertices
    IP_TRY(zero_field(ctx, &ctx->ctr_dev->n_eval));
    IP_TRY(zero_field(ctx, &ctx->ctr_dev->n_cof));
    IP_TRY(tx.start(ctx, &st.ms_expand));
    IP_TRY(level_pass1<D>(s, lo, hi));
    IP_TRY(tx.stop(ctx));
    IP_TRY(read_ctr(ctx));
    int guard = 0;
    while (c->vt_fail || c->vt_count * 2 > s.vt_cap) {
      if (++guard > 40) return ip_fail(ctx, IP_ENOMEM, "vertex table cannot grow");
      const bool failed = c->vt_fail != 0;
      IP_TRY(zero_field(ctx, (unsigned long long *)&ctx->ctr_dev->vt_fail));
      IP_TRY(vt_grow(s, pow2_at_least(c->vt_count * 4)));
      if (failed) {
        // the replay finds the inserted vertices and lists the missing ones;
        // the rebuilt pending list already holds everything unevaluated
        IP_TRY(zero_field(ctx, &ctx->ctr_dev->n_cof));
        IP_TRY(level_pass1<D>(s, lo, hi));
      }
      IP_TRY(read_ctr(ctx));
    }
    cof_total += c->n_cof;
    IP_TRY(tf.start(ctx, &st.ms_feval));
    IP_TRY(eval_pending(s, c->n_eval));
    IP_TRY(tf.stop(ctx));
    // pass 2: new edges; OUT must hold one new edge per coface at most
    IP_TRY(out_reserve(s, hi + c->n_cof + 1, hi));
    if ((c->n_out + c->n_cof) * 2 > s.et_cap) IP_TRY(et_grow(s, pow2_at_least((c->n_out + c->n_cof) * 2), hi));
    IP_TRY(tx.start(ctx, &st.ms_expand));
    IP_TRY(level_pass2<D>(s, lo, hi));
    IP_TRY(tx.stop(ctx));
    IP_TRY(read_ctr(ctx));
    guard = 0;
    while (c->et_fail) {
      if (++guard > 40) return ip_fail(ctx, IP_ENOMEM, "edge table cannot grow");
      IP_TRY(zero_field(ctx, (unsigned long long *)&ctx->ctr_dev->et_fail));
      IP_TRY(et_grow(s, s.et_cap * 4, c->n_out));
      IP_TRY(level_pass2<D>(s, lo, hi));
      IP_TRY(read_ctr(ctx));
    }
    lo = hi;
    hi = c->n_out;
  }
  IP_TRY(tf.flush(ctx));
  IP_TRY(tx.flush(ctx));
  st.levels += levels;
  st.n_cofaces += (int64_t)cof_total;
  st.n_vertices += (int64_t)c->vt_count;
  *n_out_ret = hi;
  return IP_OK;
}

// ---------------------------------------------------------------------------
// Batch triangulation (Sec. V-B, Figs. 5-6)
// ---------------------------------------------------------------------------
__host__ __device__ inline int ifact(int n) {
  int f = 1;
  for (int i = 2; i <= n; ++i) f *= i;
  return f;
}

// Index of the n-th set bit of m (n counted from 0, ascending).
__device__ __forceinline__ int nth_bit(uint32_t m, int n) {
  for (int i = 0; i < n; ++i) m &= m - 1u;
  return __ffs((int)m) - 1;
}

// Lehmer code of a permutation w of {0..D-1} in the factorial number system.
template <int D>
__device__ __forceinline__ uint32_t lehmer_encode(const int32_t *w) {
  uint32_t code = 0;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    uint32_t c = 0;
#pragma unroll
    for (int j = i + 1; j < D; ++j) c += (uint32_t)(w[j] < w[i]);
    code = code * (uint32_t)(D - i) + c;
  }
  return code;
}

template <int D>
__device__ __forceinline__ void lehmer_decode(uint32_t code, int32_t *w) {
  uint32_t c[D];
#pragma unroll
  for (int i = D - 1; i >= 0; --i) {
    c[i] = code % (uint32_t)(D - i);
    code /= (uint32_t)(D - i);
  }
  uint32_t avail = (1u << D) - 1u;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    w[i] = nth_bit(avail, (int)c[i]);
    avail &= ~(1u << w[i]);
  }
}

// Coarse n-simplex key: coarse vertex in the high bits, Lehmer code of the
// coordinate order w in the low LB bits.
template <int D>
__device__ __forceinline__ uint64_t sig_key(const LatDev &Lc, const int32_t *v, const int32_t *w, int LB) {
  return (vpack<D>(Lc, v) << LB) | (uint64_t)lehmer_encode<D>(w);
}

template <int D>
__device__ __forceinline__ void sig_unpack(const LatDev &Lc, uint64_t key, int LB, int32_t *v, int32_t *w) {
  lehmer_decode<D>((uint32_t)(key & ((1ull << LB) - 1ull)), w);
  vunpack<D>(Lc, key >> LB, v);
}

// Number of n-simplex cofaces of edge (v, (R, Q)): |R|! |Q|! (Sec. V-B).
template <int D>
__device__ __forceinline__ int n_cofacesn(uint32_t R) {
  int nR = __popc(R);
  return ifact(nR) * ifact(D + 1 - nR);
}

__global__ void count_ncof_kernel(const uint64_t *edges, uint64_t n, int D, int B, unsigned long long *total) {
  unsigned long long acc = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t R = (uint32_t)((edges[i] & ~IP_SIGN_BIT) >> (D * B)) & ((1u << D) - 1u);
    int nR = __popc(R);
    acc += (unsigned long long)(ifact(nR) * ifact(D + 1 - nR));
  }
  if (acc) atomicAdd(total, acc);
}

// Sec. V-B: n-simplex cofaces of the coarse intersecting edges, hashed to
// remove duplicates; the winners are listed in discovery order.
template <int D>
__global__ __launch_bounds__(kBlock) void sigma_kernel(LatDev Lc, int LB, const uint64_t *__restrict__ edges,
                                                       uint64_t n, uint64_t *sig_tab, uint64_t sig_mask,
                                                       uint64_t *sig_list, Counters *ctr) {
  const int lane = threadIdx.x & 63;
  const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const uint64_t n_waves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  const uint64_t nchunks = (n + 63) >> 6;
  const uint64_t below = (1ull << lane) - 1ull;
  for (uint64_t ch = wave; ch < nchunks; ch += n_waves) {
    const uint64_t ei = ch * 64 + lane;
    uint64_t e = 0;
    int cnt = 0;
    if (ei < n) {
      e = edges[ei];
      cnt = n_cofacesn<D>((uint32_t)((e & ~IP_SIGN_BIT) >> (D * Lc.B)) & ((1u << D) - 1u));
    }
    int incl = cnt;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      int t = __shfl_up(incl, off, 64);
      if (lane >= off) incl += t;
    }
    const int excl = incl - cnt;
    const int total = __shfl(incl, 63, 64);
    for (int base = 0; base < total; base += 64) {
      const int idx = base + lane;
      const bool valid = idx < total;
      int j = 0;
#pragma unroll
      for (int step = 32; step; step >>= 1) {
        int pc = __shfl(excl, j + step, 64);
        if (pc <= idx) j += step;
      }
      const uint64_t me = shfl64(e, j);
      const int r = idx - __shfl(excl, j, 64);
      bool is_new = false;
      uint64_t key = 0;
      if (valid) {
        int32_t v[D];
        uint32_t R;
        eunpack<D>(Lc, me, v, &R);
        const uint32_t Q = ((1u << (D + 1)) - 1u) & ~R;
        const int nR = __popc(R), nQ = D + 1 - nR;
        const int fQ = ifact(nQ);
        // orderings of R and of Q from the factorial number system
        int32_t pi[D + 1], rho[D + 1];
        {
          uint32_t code = (uint32_t)(r / fQ);
          uint32_t avail = R;
          for (int i = 0; i < nR; ++i) {
            int f = ifact(nR - 1 - i);
            int c = (int)(code / (uint32_t)f);
            code %= (uint32_t)f;
            pi[i] = nth_bit(avail, c);
            avail &= ~(1u << pi[i]);
          }
          code = (uint32_t)(r % fQ);
          avail = Q;
          for (int i = 0; i < nQ; ++i) {
            int f = ifact(nQ - 1 - i);
            int c = (int)(code / (uint32_t)f);
            code %= (uint32_t)f;
            rho[i] = nth_bit(avail, c);
            avail &= ~(1u << rho[i]);
          }
        }
        // rotate the cycle (pi, rho) so that D comes last: the start vertex
        // is v - 1_{rho after D}, the order is (rho after D, pi, rho before D)
        int jd = 0;
        for (int i = 0; i < nQ; ++i)
          if (rho[i] == D) jd = i;
        int32_t vs[D], w[D];
#pragma unroll
        for (int q = 0; q < D; ++q) vs[q] = v[q];
        int m = 0;
        for (int i = jd + 1; i < nQ; ++i) {
          vs[rho[i]] -= 1;
          w[m++] = rho[i];
        }
        for (int i = 0; i < nR; ++i) w[m++] = pi[i];
        for (int i = 0; i < jd; ++i) w[m++] = rho[i];
        if (vin_range<D>(Lc, vs)) {
          key = sig_key<D>(Lc, vs, w, LB);
          uint64_t slot;
          int ins = ht_insert(sig_tab, sig_mask, key, &slot);
          if (ins == 1)
            is_new = true;
          else if (ins < 0)
            atomicOr(&ctr->et_fail, 1u);
        } else {
          atomicOr(&ctr->vt_fail, 1u);
        }
      }
      const uint64_t bal = __ballot(is_new);
      if (bal) {
        const int leader = __ffsll((long long)bal) - 1;
        unsigned long long b0 = 0;
        if (lane == leader) b0 = atomicAdd(&ctr->n_aux, (unsigned long long)__popcll(bal));
        b0 = shfl64(b0, leader);
        if (is_new) sig_list[b0 + __popcll(bal & below)] = key;
      }
    }
  }
}

// Template point p of coarse simplex (v, w) in fine lattice coordinates:
// y_{w_i} = k v_{w_i} + u_i (Eq. 1 with the coarse edge directions e_{w_i}).
template <int D>
__device__ __forceinline__ void template_point(const int32_t *v, const int32_t *w, int k, uint64_t up, int32_t *y) {
#pragma unroll
  for (int i = 0; i < D; ++i) y[w[i]] = k * v[w[i]] + (int32_t)((up >> (8 * i)) & 0xffu);
}

// Fine vertices of a batch of coarse simplices: insert into the batch vertex
// table, remember the slot of every (simplex, template point).
template <int D>
__global__ __launch_bounds__(kBlock) void batch_vertices_kernel(LatDev Lf, LatDev Lc, int LB, int k,
                                                                const uint64_t *__restrict__ sig, uint64_t nb,
                                                                const uint64_t *__restrict__ tpts, int NP,
                                                                uint64_t *vt_keys, uint64_t vt_mask,
                                                                uint32_t *eval_list, uint32_t *pslot,
                                                                Counters *ctr) {
  const int lane = threadIdx.x & 63;
  const uint64_t total = nb * (uint64_t)NP;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t start = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t rounds = (total + stride - 1) / stride;
  for (uint64_t it = 0; it < rounds; ++it) {
    const uint64_t t = start + it * stride;
    bool is_new = false;
    uint64_t slot = 0;
    if (t < total) {
      const uint64_t s = t / (uint64_t)NP;
      const int p = (int)(t - s * (uint64_t)NP);
      int32_t v[D], w[D], y[D];
      sig_unpack<D>(Lc, sig[s], LB, v, w);
      template_point<D>(v, w, k, tpts[p], y);
      double x[D];
      lat_coords<D>(Lf, y, x);
      uint32_t ps = 0xffffffffu;
      if (lat_in_box<D>(Lf, x)) {
        int ins = ht_insert(vt_keys, vt_mask, vpack<D>(Lf, y), &slot);
        if (ins >= 0) {
          ps = (uint32_t)slot;
          is_new = ins == 1;
        } else {
          atomicOr(&ctr->vt_fail, 1u);
        }
      }
      pslot[t] = ps;
    }
    const uint64_t bal = __ballot(is_new);
    if (bal) {
      const int leader = __ffsll((long long)bal) - 1;
      unsigned long long b0 = 0;
      if (lane == leader) b0 = atomicAdd(&ctr->n_eval, (unsigned long long)__popcll(bal));
      b0 = shfl64(b0, leader);
      if (is_new) eval_list[b0 + __popcll(bal & ((1ull << lane) - 1ull))] = (uint32_t)slot;
    }
  }
}

// Fine edges of the subdivision (Sec. V-B, Fig. 6): sign test on the two
// endpoint values, insertion of the intersecting ones into the global fine
// edge set; new edges are appended to the output key list.
template <int D>
__global__ __launch_bounds__(kBlock) void batch_edges_kernel(LatDev Lf, LatDev Lc, int LB, int k,
                                                             const uint64_t *__restrict__ sig, uint64_t nb,
                                                             const uint64_t *__restrict__ tpts, int NP,
                                                             const uint32_t *__restrict__ tedge, int NE,
                                                             const uint32_t *__restrict__ pslot,
                                                             const double *__restrict__ vt_vals, uint64_t *et_keys,
                                                             uint64_t et_mask, uint64_t *out, Counters *ctr) {
  const int lane = threadIdx.x & 63;
  const uint64_t total = nb * (uint64_t)NE;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t start = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t rounds = (total + stride - 1) / stride;
  unsigned long long hits = 0;
  for (uint64_t it = 0; it < rounds; ++it) {
    const uint64_t t = start + it * stride;
    bool is_new = false;
    uint64_t key = 0;
    if (t < total) {
      const uint64_t s = t / (uint64_t)NE;
      const int e = (int)(t - s * (uint64_t)NE);
      const uint32_t te = tedge[e];
      const int a = (int)(te & 0xfffu), b = (int)((te >> 12) & 0xfffu);
      const uint32_t Rl = te >> 24;
      const uint32_t sa = pslot[s * NP + a], sb = pslot[s * NP + b];
      if (sa != 0xffffffffu && sb != 0xffffffffu) {
        const bool pa = !(vt_vals[sa] < 0.0), pb = !(vt_vals[sb] < 0.0);
        if (pa != pb) {
          ++hits;
          int32_t v[D], w[D], y[D];
          sig_unpack<D>(Lc, sig[s], LB, v, w);
          template_point<D>(v, w, k, tpts[a], y);
          uint32_t Rg = 0;
#pragma unroll
          for (int i = 0; i < D; ++i) Rg |= ((Rl >> i) & 1u) << w[i];
          key = ekey<D>(Lf, y, Rg);
          uint64_t slot;
          int ins = ht_insert(et_keys, et_mask, key, &slot);
          if (ins == 1)
            is_new = true;
          else if (ins < 0)
            atomicOr(&ctr->et_fail, 1u);
        }
      }
    }
    const uint64_t bal = __ballot(is_new);
    if (bal) {
      const int leader = __ffsll((long long)bal) - 1;
      unsigned long long b0 = 0;
      if (lane == leader) b0 = atomicAdd(&ctr->n_out, (unsigned long long)__popcll(bal));
      b0 = shfl64(b0, leader);
      if (is_new) out[b0 + __popcll(bal & ((1ull << lane) - 1ull))] = key;
    }
  }
  if (hits) atomicAdd(&ctr->n_cof, hits);
}

// Intersection points of the edges out[lo .. hi), endpoints looked up in the
// batch vertex table.
template <int D>
__global__ void batch_points_kernel(LatDev L, const uint64_t *keys, uint64_t lo, uint64_t hi, const uint64_t *vt_keys,
                                    const double *vt_vals, uint64_t vt_mask, double *pts, int64_t ld) {
  for (uint64_t i = lo + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < hi; i += (uint64_t)gridDim.x * blockDim.x) {
    int32_t a[D], b[D];
    uint32_t R;
    eunpack<D>(L, keys[i], a, &R);
#pragma unroll
    for (int j = 0; j < D; ++j) b[j] = a[j] + (int32_t)((R >> j) & 1u);
    int64_t ha = ht_find(vt_keys, vt_mask, vpack<D>(L, a));
    int64_t hb = ht_find(vt_keys, vt_mask, vpack<D>(L, b));
    double fa = ha >= 0 ? vt_vals[ha] : NAN;
    double fb = hb >= 0 ? vt_vals[hb] : NAN;
    double xa[D], xb[D];
    lat_coords<D>(L, a, xa);
    lat_coords<D>(L, b, xb);
    double t = fa / (fa - fb);
#pragma unroll
    for (int j = 0; j < D; ++j) pts[(int64_t)j * ld + (int64_t)i] = fma(t, xb[j] - xa[j], xa[j]);
  }
}

__global__ void et_rebuild_keys_kernel(const uint64_t *keys, uint64_t n, uint64_t *et, uint64_t mask, Counters *ctr) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t slot;
    if (ht_insert(et, mask, keys[i], &slot) < 0) atomicOr(&ctr->et_fail, 1u);
  }
}

// Local subdivision template (Sec. V-B, Eq. 2 read with >=): points u with
// k >= u_0 >= ... >= u_{d-1} >= 0 and edges (u, R) whose other end u + 1_R
// is inside too.  Points packed 8 bits per coordinate; edges packed as
// (index a | index b << 12 | R << 24).
struct Template {
  std::vector<uint64_t> pts;
  std::vector<uint32_t> edges;
};

Template make_template(int d, int k) {
  Template T;
  std::vector<std::vector<int>> P;
  std::vector<int> u(d, 0);
  auto inside = [&](const std::vector<int> &x) {
    if (x[0] > k) return false;
    for (int i = 0; i + 1 < d; ++i)
      if (x[i] < x[i + 1]) return false;
    return x[d - 1] >= 0;
  };
  for (;;) {
    if (inside(u)) P.push_back(u);
    int j = 0;
    while (j < d && u[j] == k) u[j++] = 0;
    if (j == d) break;
    ++u[j];
  }
  auto index_of = [&](const std::vector<int> &x) -> int {
    for (size_t i = 0; i < P.size(); ++i)
      if (P[i] == x) return (int)i;
    return -1;
  };
  for (auto &x : P) {
    uint64_t pk = 0;
    for (int i = 0; i < d; ++i) pk |= (uint64_t)x[i] << (8 * i);
    T.pts.push_back(pk);
  }
  for (size_t a = 0; a < P.size(); ++a)
    for (uint32_t R = 1; R < (1u << d); ++R) {
      std::vector<int> y = P[a];
      for (int i = 0; i < d; ++i) y[i] += (int)((R >> i) & 1u);
      if (!inside(y)) continue;
      int b = index_of(y);
      T.edges.push_back((uint32_t)a | ((uint32_t)b << 12) | (R << 24));
    }
  return T;
}

int lehmer_bits(int d) {
  int f = ifact(d), b = 0;
  while ((1 << b) < f) ++b;
  return b < 1 ? 1 : b;
}

template <int D>
int trace_batch(ip_ctx *ctx, const ip_problem *p, uint64_t budget, ip_cells *res) {
  ip_stats &st = res->st;
  const int k = p->k;
  const int LB = lehmer_bits(D);
  if (D * p->coarse.B + LB > 63)
    return ip_fail(ctx, IP_ERANGE, "coarse simplex keys do not fit 63 bits for this domain and k");
  Template T = make_template(D, k);
  const int NP = (int)T.pts.size(), NE = (int)T.edges.size();
  if (NP >= 4096) return ip_fail(ctx, IP_EINVAL, "subdivision template too large (reduce k)");
  // ---- coarse trace (Sec. V-B: trace at scale k * lambda)
  Run s;
  s.ctx = ctx;
  s.p = p;
  s.L = p->coarse;
  IP_TRY(vt_init(s, 1ull << 16));
  IP_TRY(et_init(s, 1ull << 16));
  uint64_t nc = 0;
  {
    int rc = trace_direct<D>(s, st, &nc);
    if (rc != IP_OK) {
      if (s.out) (void)hipFree(s.out);
      return rc;
    }
  }
  uint64_t *coarse_edges = s.out;
  s.out = nullptr;
  s.out_cap = 0;
  auto free_coarse = [&]() {
    if (coarse_edges) (void)hipFree(coarse_edges);
    coarse_edges = nullptr;
  };
  // ---- Sigma: n-cofaces of the coarse edges, deduplicated
  void *sig_tab = nullptr, *sig_list = nullptr;
  uint64_t nsig = 0;
  {
    IP_TRY_HIP(ctx, hipMemsetAsync(ctx->ctr_dev, 0, sizeof(Counters), ctx->stream));
    if (nc) {
      hipLaunchKernelGGL(count_ncof_kernel, dim3(grid_for(nc)), dim3(kBlock), 0, ctx->stream, coarse_edges, nc, D,
                         p->coarse.B, &ctx->ctr_dev->n_aux);
      IP_TRY_HIP(ctx, hipGetLastError());
    }
    IP_TRY(read_ctr(ctx));
    const uint64_t bound = ctx->ctr_host->n_aux;
    const uint64_t cap = pow2_at_least(bound * 2 + 2);
    int rc = alloc(ctx, &sig_tab, cap * 8);
    if (rc == IP_OK) rc = alloc(ctx, &sig_list, (bound + 1) * 8);
    if (rc != IP_OK) {
      free_coarse();
      if (sig_tab) (void)hipFree(sig_tab);
      return rc;
    }
    IP_TRY(fill(ctx, sig_tab, cap, IP_EMPTY_KEY));
    IP_TRY_HIP(ctx, hipMemsetAsync(ctx->ctr_dev, 0, sizeof(Counters), ctx->stream));
    if (nc) {
      hipLaunchKernelGGL((sigma_kernel<D>), dim3(grid_for(nc * 4, 8192)), dim3(kBlock), 0, ctx->stream, p->coarse, LB,
                         coarse_edges, nc, (uint64_t *)sig_tab, cap - 1, (uint64_t *)sig_list, ctx->ctr_dev);
      IP_TRY_HIP(ctx, hipGetLastError());
    }
    IP_TRY(read_ctr(ctx));
    nsig = ctx->ctr_host->n_aux;
    free_coarse();
    (void)hipFree(sig_tab);
    sig_tab = nullptr;
  }
  st.n_sigma = (int64_t)nsig;
  // ---- template on the device
  void *tpts = nullptr, *tedge = nullptr;
  IP_TRY(alloc(ctx, &tpts, T.pts.size() * 8));
  IP_TRY(alloc(ctx, &tedge, T.edges.size() * 4));
  IP_TRY_HIP(ctx, hipMemcpyAsync(tpts, T.pts.data(), T.pts.size() * 8, hipMemcpyHostToDevice, ctx->stream));
  IP_TRY_HIP(ctx, hipMemcpyAsync(tedge, T.edges.data(), T.edges.size() * 4, hipMemcpyHostToDevice, ctx->stream));
  // ---- batches: per coarse simplex NP slots, NP vertex-table entries at
  // load <= 1/2 (16 B key+value each, twice) and NP eval-list entries
  const uint64_t per_sigma = (uint64_t)NP * (4 + 2 * 16 + 2 * 4);
  if (budget == 0) budget = 4ull << 30;
  if (budget < per_sigma) return ip_fail(ctx, IP_ENOMEM, "batch budget below one coarse simplex");
  uint64_t B = budget / per_sigma;
  if (B > nsig) B = nsig ? nsig : 1;
  if (B * (uint64_t)NP * 2 > (1ull << 31)) B = (1ull << 31) / ((uint64_t)NP * 2);
  Run f;
  f.ctx = ctx;
  f.p = p;
  f.L = p->fine;
  const uint64_t vcap = pow2_at_least(B * (uint64_t)NP * 2);
  IP_TRY(ip_ensure(ctx, ctx->vt_keys, vcap * 8));
  IP_TRY(ip_ensure(ctx, ctx->vt_vals, vcap * 8));
  IP_TRY(ip_ensure(ctx, ctx->eval_list, vcap * 4));
  IP_TRY(ip_ensure(ctx, ctx->vt_aux, B * (uint64_t)NP * 4));
  f.vt_keys = (uint64_t *)ctx->vt_keys.p;
  f.vt_vals = (double *)ctx->vt_vals.p;
  f.eval = (uint32_t *)ctx->eval_list.p;
  f.vt_cap = f.eval_cap = vcap;
  uint32_t *pslot = (uint32_t *)ctx->vt_aux.p;
  // global fine edge set + output keys (capacity tied to the set's)
  uint64_t et_cap = 1ull << 20;
  IP_TRY(et_init(f, et_cap));
  IP_TRY(out_reserve(f, et_cap, 0));
  double *pts = nullptr;
  uint64_t pts_ld = 0;
  uint64_t n_out = 0;
  Counters *c = ctx->ctr_host;
  IP_TRY_HIP(ctx, hipMemsetAsync(ctx->ctr_dev, 0, sizeof(Counters), ctx->stream));
  Timer tf, tx, tp;
  int64_t batches = 0;
  int rc = IP_OK;
  for (uint64_t b0 = 0; b0 < nsig && rc == IP_OK; b0 += B) {
    const uint64_t nb = std::min<uint64_t>(B, nsig - b0);
    const uint64_t *sig = (const uint64_t *)sig_list + b0;
    ++batches;
    IP_TRY(fill(ctx, f.vt_keys, vcap, IP_EMPTY_KEY));
    IP_TRY(fill(ctx, f.vt_vals, vcap, IP_UNEVAL_BITS));
    IP_TRY(zero_field(ctx, &ctx->ctr_dev->n_eval));
    IP_TRY(tx.start(ctx, &st.ms_expand));
    hipLaunchKernelGGL((batch_vertices_kernel<D>), dim3(grid_for(nb * NP)), dim3(kBlock), 0, ctx->stream, p->fine,
                       p->coarse, LB, k, sig, nb, (const uint64_t *)tpts, NP, f.vt_keys, vcap - 1, f.eval, pslot,
                       ctx->ctr_dev);
    IP_TRY_HIP(ctx, hipGetLastError());
    IP_TRY(tx.stop(ctx));
    IP_TRY(read_ctr(ctx));
    if (c->vt_fail) {
      rc = ip_fail(ctx, IP_ENOMEM, "batch vertex table overflow");
      break;
    }
    IP_TRY(tf.start(ctx, &st.ms_feval));
    IP_TRY(eval_pending(f, c->n_eval));
    IP_TRY(tf.stop(ctx));
    st.n_vertices += (int64_t)c->n_eval;
    // keep the fine edge set at load <= 1/2 before the batch; on overflow
    // grow it from the output keys (which include the partial appends of the
    // failed launch) and replay the launch, which skips edges already present
    const uint64_t batch_lo = n_out;
    uint64_t n_keys = n_out;
    int guard = 0;
    for (;;) {
      if (n_keys * 2 > f.et_cap || c->et_fail) {
        if (++guard > 40) return ip_fail(ctx, IP_ENOMEM, "edge table cannot grow");
        const uint64_t ncap = pow2_at_least(std::max<uint64_t>(n_keys * 4, f.et_cap * 2));
        IP_TRY(out_reserve(f, ncap, n_keys));
        void *nk = nullptr;
        IP_TRY(alloc(ctx, &nk, ncap * 8));
        IP_TRY(fill(ctx, nk, ncap, IP_EMPTY_KEY));
        IP_TRY(zero_field(ctx, (unsigned long long *)&ctx->ctr_dev->et_fail));
        if (n_keys) {
          hipLaunchKernelGGL(et_rebuild_keys_kernel, dim3(grid_for(n_keys)), dim3(kBlock), 0, ctx->stream, f.out,
                             n_keys, (uint64_t *)nk, ncap - 1, ctx->ctr_dev);
          IP_TRY_HIP(ctx, hipGetLastError());
        }
        IP_TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));
        (void)hipFree(ctx->et_keys.p);
        ctx->et_keys = {nk, ncap * 8};
        f.et_keys = (uint64_t *)nk;
        f.et_cap = ncap;
        ++f.regrows;
      }
      IP_TRY(zero_field(ctx, &ctx->ctr_dev->n_cof));
      IP_TRY(tx.start(ctx, &st.ms_expand));
      hipLaunchKernelGGL((batch_edges_kernel<D>), dim3(grid_for(nb * NE)), dim3(kBlock), 0, ctx->stream, p->fine,
                         p->coarse, LB, k, sig, nb, (const uint64_t *)tpts, NP, (const uint32_t *)tedge, NE, pslot,
                         f.vt_vals, f.et_keys, f.et_cap - 1, f.out, ctx->ctr_dev);
      IP_TRY_HIP(ctx, hipGetLastError());
      IP_TRY(tx.stop(ctx));
      IP_TRY(read_ctr(ctx));
      if (!c->et_fail) break;
      n_keys = c->n_out;
    }
    st.n_template_edges += (int64_t)(nb * (uint64_t)NE);
    const uint64_t lo = batch_lo, hi = c->n_out;
    if (hi > pts_ld) {
      // grow the SoA point buffer, copying the columns
      const uint64_t nld = std::max<uint64_t>(hi, pts_ld * 2);
      double *np_ = nullptr;
      IP_TRY(alloc(ctx, (void **)&np_, nld * D * 8));
      if (pts && lo) {
        for (int j = 0; j < D; ++j)
          IP_TRY_HIP(ctx, hipMemcpyAsync(np_ + (uint64_t)j * nld, pts + (uint64_t)j * pts_ld, lo * 8,
                                         hipMemcpyDeviceToDevice, ctx->stream));
      }
      IP_TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));
      if (pts) (void)hipFree(pts);
      pts = np_;
      pts_ld = nld;
    }
    if (hi > lo) {
      IP_TRY(tp.start(ctx, &st.ms_points));
      hipLaunchKernelGGL((batch_points_kernel<D>), dim3(grid_for(hi - lo)), dim3(kBlock), 0, ctx->stream, p->fine, f.out,
                         lo, hi, f.vt_keys, f.vt_vals, vcap - 1, pts, (int64_t)pts_ld);
      IP_TRY_HIP(ctx, hipGetLastError());
      IP_TRY(tp.stop(ctx));
    }
    n_out = hi;
  }
  IP_TRY(tf.flush(ctx));
  IP_TRY(tx.flush(ctx));
  IP_TRY(tp.flush(ctx));
  (void)hipFree(tpts);
  (void)hipFree(tedge);
  (void)hipFree(sig_list);
  if (rc != IP_OK) {
    if (f.out) (void)hipFree(f.out);
    if (pts) (void)hipFree(pts);
    return rc;
  }
  if (!pts) IP_TRY(alloc(ctx, (void **)&pts, 8 * D));
  res->d = D;
  res->B = p->fine.B;
  for (int j = 0; j < 8; ++j) res->vmin[j] = p->fine.vmin[j];
  res->n = (int64_t)n_out;
  res->keys = f.out;
  res->pts = pts;
  res->ld = (int64_t)(pts_ld ? pts_ld : 1);
  st.n_cells = (int64_t)n_out;
  st.n_batches = batches;
  st.regrows += s.regrows + f.regrows;
  return IP_OK;
}

template <int D>
int trace_T(ip_ctx *ctx, const ip_problem *p, uint64_t budget, int32_t prec, ip_cells *res) {
  (void)budget;
  (void)prec;
  Run s;
  s.ctx = ctx;
  s.p = p;
  s.L = p->fine;
  if (p->k != 1) return trace_batch<D>(ctx, p, budget, res);
  const uint64_t vt0 = std::max<uint64_t>(1ull << 20, ctx->vt_keys.bytes / 8);
  const uint64_t et0 = std::max<uint64_t>(1ull << 20, ctx->et_keys.bytes / 8);
  IP_TRY(vt_init(s, pow2_at_least(vt0) == vt0 ? vt0 : pow2_at_least(vt0) / 2));
  IP_TRY(et_init(s, pow2_at_least(et0) == et0 ? et0 : pow2_at_least(et0) / 2));
  ip_stats &st = res->st;
  uint64_t n = 0;
  int rc = trace_direct<D>(s, st, &n);
  if (rc != IP_OK) {
    if (s.out) (void)hipFree(s.out);
    return rc;
  }
  // intersection points
  double *pts = nullptr;
  rc = alloc(ctx, (void **)&pts, sizeof(double) * (size_t)(n ? n : 1) * D);
  if (rc != IP_OK) {
    if (s.out) (void)hipFree(s.out);
    return rc;
  }
  if (n) {
    Timer tp;
    IP_TRY(tp.start(ctx, &st.ms_points));
    hipLaunchKernelGGL((points_kernel<D>), dim3(grid_for(n)), dim3(kBlock), 0, ctx->stream, s.L, s.out, n,
                       s.vt_keys, s.vt_vals, s.vt_cap - 1, pts, (int64_t)n);
    IP_TRY_HIP(ctx, hipGetLastError());
    IP_TRY(tp.stop(ctx));
    IP_TRY(tp.flush(ctx));
  }
  res->d = D;
  res->B = s.L.B;
  for (int j = 0; j < 8; ++j) res->vmin[j] = s.L.vmin[j];
  res->n = (int64_t)n;
  res->keys = s.out;
  res->pts = pts;
  res->ld = (int64_t)n;
  st.n_cells = (int64_t)n;
  st.regrows += s.regrows;
  return IP_OK;
}

}  // namespace

int ip_trace_impl(ip_ctx *ctx, const ip_problem *p, uint64_t budget, int32_t prec, uint32_t flags,
                  ip_cells *out) {
  (void)flags;
  if (prec != IP_FP64) return ip_fail(ctx, IP_EINVAL, "precision mode not available");
  switch (p->d) {
    case 2: return trace_T<2>(ctx, p, budget, prec, out);
    case 3: return trace_T<3>(ctx, p, budget, prec, out);
    case 4: return trace_T<4>(ctx, p, budget, prec, out);
    case 5: return trace_T<5>(ctx, p, budget, prec, out);
    case 6: return trace_T<6>(ctx, p, budget, prec, out);
    case 7: return trace_T<7>(ctx, p, budget, prec, out);
    default: return ip_fail(ctx, IP_EINVAL, "dimension out of range");
  }
}
