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

template <int D>
int trace_T(ip_ctx *ctx, const ip_problem *p, uint64_t budget, int32_t prec, ip_cells *res) {
  (void)budget;
  (void)prec;
  Run s;
  s.ctx = ctx;
  s.p = p;
  s.L = p->fine;
  if (p->k != 1) return ip_fail(ctx, IP_EINVAL, "batch triangulation (coarse_k > 1) not available");
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
