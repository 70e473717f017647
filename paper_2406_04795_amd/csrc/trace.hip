// Manifold tracing on the Coxeter triangulation (Sec. V-A, Figs. 3-4) and
// batch triangulation (Sec. V-B, Figs. 5-6).
//
// Direct mode state:
//   VT   vertex table (open addressing, 32-byte VEnt entries): packed vertex
//        key, f at the vertex, and a bitmask of the visited edges whose
//        smaller endpoint is this vertex.  The bitmask is the search's
//        visited set: marking edge (v, R) is one atomicOr on bit R of v's
//        entry, an entry the search touches anyway.
//   OUT  append-only list of traced edges (key + the VT slots of both ends);
//        the frontier of a level is a contiguous range of it.
//   CSL  per level, the VT slot of the third vertex of every coface.
// One breadth-first level = pass 1 (third vertices of the 2-cofaces of the
// frontier edges into VT, slots into CSL, new vertices listed), f evaluation
// of the new vertices, pass 2 (per coface: the other sign-changing edge is
// marked in its smaller endpoint's entry; first markers append to OUT).
// The host reads a small counter block after each pass; table growth rehashes
// VT, re-points OUT's slots and replays pass 1, which is idempotent.
#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "ip_internal.h"

namespace {

constexpr int kBlock = 256;
constexpr int kStage = 128;  // per-wave staged append entries

struct OutRec {
  uint64_t key;
  uint64_t slots;  // slot of the smaller endpoint | slot of the other << 32
};

__global__ void fill_u64_kernel(uint64_t *p, uint64_t n, uint64_t v) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void fill_vent_kernel(VEnt *p, uint64_t n) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    VEnt e;
    e.key = IP_EMPTY_KEY;
    e.f = __longlong_as_double((long long)IP_UNEVAL_BITS);
    e.m[0] = 0ull;
    e.m[1] = 0ull;
    p[i] = e;
  }
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

// Mark edge (v, mask) in the entry of its smaller endpoint; true if this
// call was the first to mark it.  Bits only ever go from 0 to 1, so a plain
// load that already shows the bit proves the edge visited; most cofaces lead
// to visited edges, and they skip the atomic.  A stale 0 falls through to the
// atomicOr, which decides.
__device__ __forceinline__ bool mark_edge(VEnt *vt, uint64_t owner, uint32_t mask) {
  const unsigned long long bit = 1ull << (mask & 63u);
  unsigned long long *w = &vt[owner].m[mask >> 6];
  if (*(volatile unsigned long long *)w & bit) return false;
  const unsigned long long old = atomicOr(w, bit);
  return !(old & bit);
}

// Sec. V-A "find all n-simplices": locate each seed and register the
// vertices of its n-simplex that lie in the domain.
template <int D>
__global__ void seed_vertices_kernel(LatDev L, const double *seeds, int64_t ns, VEnt *vt, uint64_t vt_mask,
                                     uint32_t *eval_list, Counters *ctr) {
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
    int r = vt_insert(vt, vt_mask, vpack<D>(L, v), &slot);
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
__global__ void seed_edges_kernel(LatDev L, const double *seeds, int64_t ns, VEnt *vt, uint64_t vt_mask,
                                  OutRec *out, Counters *ctr) {
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
  int64_t sl[D + 1];
  double fv[D + 1];
  for (int m = 0; m <= D; ++m) {
    sl[m] = vin_range<D>(L, u[m]) ? vt_find(vt, vt_mask, vpack<D>(L, u[m])) : -1;
    fv[m] = sl[m] >= 0 ? vt[sl[m]].f : 0.0;
  }
  for (int a = 0; a <= D; ++a)
    for (int b = a + 1; b <= D; ++b) {
      if (sl[a] < 0 || sl[b] < 0) continue;
      const bool sa = !(fv[a] < 0.0), sb = !(fv[b] < 0.0);
      if (sa == sb) continue;
      int32_t vm[D];
      uint32_t mask;
      const bool a_min = edge_canon<D>(u[a], u[b], vm, &mask);
      const uint64_t smin = (uint64_t)(a_min ? sl[a] : sl[b]), smax = (uint64_t)(a_min ? sl[b] : sl[a]);
      if (mark_edge(vt, smin, mask)) {
        unsigned long long idx = atomicAdd(&ctr->n_out, 1ull);
        out[idx].key = ekey<D>(L, vm, mask) | ((a_min ? sa : sb) ? IP_SIGN_BIT : 0ull);
        out[idx].slots = smin | (smax << 32);
      }
    }
}

// Frontier expansion (Sec. V-A "find all cofaces" / "find all interesting
// cofaces' edges" / "hash all edges").  Each wave takes 64 frontier edges,
// prefix-sums their coface counts and walks the flattened (edge, coface)
// list 64 at a time, so lanes stay busy whatever the mix of edge classes.
//   EDGES = false: pass 1, third vertices into VT and CSL.
//   EDGES = true : pass 2, sign test and marking of the new edge.
template <int D, bool EDGES>
__global__ __launch_bounds__(kBlock) void expand_kernel(LatDev L, OutRec *out, uint64_t lo, uint64_t hi, VEnt *vt,
                                                        uint64_t vt_mask, uint32_t *cslot, uint32_t *eval_list,
                                                        Counters *ctr) {
  constexpr int MAXC = (1 << D) - 2;  // most 2-cofaces an edge can have
  __shared__ OutRec st_out[EDGES ? kBlock / 64 : 1][EDGES ? kStage : 1];
  __shared__ uint32_t st_ev[EDGES ? 1 : kBlock / 64][EDGES ? 1 : kStage];
  const int lane = threadIdx.x & 63;
  const int wib = threadIdx.x >> 6;
  const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const uint64_t n_waves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  const uint64_t nchunks = (hi - lo + 63) >> 6;
  int sn = 0;
  unsigned long long cof_acc = 0, new_acc = 0;
  auto put_out = [&](unsigned long long pos, const OutRec &r) { out[pos] = r; };
  auto put_ev = [&](unsigned long long pos, uint32_t s) { eval_list[pos] = s; };
  for (uint64_t ch = wave; ch < nchunks; ch += n_waves) {
    const uint64_t ei = lo + ch * 64 + lane;
    uint64_t e = 0, es = 0;
    int cnt = 0;
    if (ei < hi) {
      e = out[ei].key;
      if (EDGES) es = out[ei].slots;
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
      const uint64_t crow = (ch * 64 + (uint64_t)j) * MAXC + (uint64_t)r;
      if (!EDGES) {
        bool is_new = false;
        uint32_t slot32 = 0;
        if (valid) {
          int32_t v[D], c[D];
          uint32_t R;
          eunpack<D>(L, me, v, &R);
          coface_vertex<D>(v, R, r, c);
          double x[D];
          lat_coords<D>(L, c, x);
          uint32_t cs = 0xffffffffu;
          if (lat_in_box<D>(L, x)) {
            uint64_t slot;
            int ins = vt_insert(vt, vt_mask, vpack<D>(L, c), &slot);
            if (ins >= 0) {
              cs = (uint32_t)slot;
              is_new = ins == 1;
              slot32 = cs;
            } else {
              atomicOr(&ctr->vt_fail, 1u);
            }
          }
          cslot[crow] = cs;
        }
        new_acc += (unsigned long long)__popcll(__ballot(is_new));
        stage_put<kStage>(st_ev[wib], sn, is_new, slot32, put_ev, &ctr->n_eval);
      } else {
        const uint64_t mslots = shfl64(es, j);
        bool is_new = false;
        OutRec rec = {0, 0};
        if (valid) {
          const uint32_t cs = cslot[crow];
          if (cs != 0xffffffffu) {
            const bool sc = !(vt[cs].f < 0.0);
            const bool sa = (me & IP_SIGN_BIT) != 0;
            int32_t v[D], c[D];
            uint32_t R;
            eunpack<D>(L, me, v, &R);
            coface_vertex<D>(v, R, r, c);
            // exactly one of (a,c), (b,c) changes sign: the one whose other
            // end has the sign c does not have (Sec. V-A, two edges of a
            // triangle cross the manifold)
            int32_t other[D];
            bool so;
            uint64_t oslot;
            if (sc != sa) {
#pragma unroll
              for (int q = 0; q < D; ++q) other[q] = v[q];
              so = sa;
              oslot = mslots & 0xffffffffull;
            } else {
#pragma unroll
              for (int q = 0; q < D; ++q) other[q] = v[q] + (int32_t)((R >> q) & 1u);
              so = !sa;
              oslot = mslots >> 32;
            }
            int32_t vm[D];
            uint32_t mask;
            const bool other_min = edge_canon<D>(other, c, vm, &mask);
            const uint64_t smin = other_min ? oslot : (uint64_t)cs, smax = other_min ? (uint64_t)cs : oslot;
            if (mark_edge(vt, smin, mask)) {
              is_new = true;
              rec.key = ekey<D>(L, vm, mask) | ((other_min ? so : sc) ? IP_SIGN_BIT : 0ull);
              rec.slots = smin | (smax << 32);
            }
          }
        }
        stage_put<kStage>(st_out[wib], sn, is_new, rec, put_out, &ctr->n_out);
      }
    }
  }
  if (EDGES)
    stage_flush(st_out[wib], sn, put_out, &ctr->n_out);
  else
    stage_flush(st_ev[wib], sn, put_ev, &ctr->n_eval);
  if (!EDGES && lane == 0) {
    if (cof_acc) atomicAdd(&ctr->n_cof, cof_acc);
    if (new_acc) atomicAdd(&ctr->vt_count, new_acc);
  }
}

// Intersection point of edge (a, b), a the smaller endpoint (Sec. V-B):
// t = f_a / (f_a - f_b), p = x_a + t (x_b - x_a).  With certification on
// (FP32 mode) the stored f only settled the sign: an end whose stored value
// is not the canonical FP64 one (bound ba / bb >= 0) gets f from the FP64
// monomial-basis evaluation with its bound, a canonical end keeps its value
// (bound B64).  The call returns false when the a-priori bound on the
// distance to the point computed from canonical FP64 values exceeds half the
// FP32 tolerance, 1e-5 relative; since f_a and f_b have opposite signs,
// |dt| <= (da + db + 2 B64) / (|fa| + |fb| - da - db - 2 B64).
template <int D>
__device__ __forceinline__ bool edge_point(const LatDev &L, const PolyDev &Q, const int32_t *a, const int32_t *b,
                                           double fa, double fb, bool cert, float ba, float bb, double *p) {
  double xa[D], xb[D];
  lat_coords<D>(L, a, xa);
  lat_coords<D>(L, b, xb);
  double da = Q.B64, db = Q.B64;
  const bool exact = !cert || (ba < 0.0f && bb < 0.0f);
  if (!exact) {
    if (Q.ok) {
      // polynomial f: FP64 monomial values with their bounds
      if (ba >= 0.0f) fa = poly64_any<D>(Q, xa, &da);
      if (bb >= 0.0f) fb = poly64_any<D>(Q, xb, &db);
    } else {
      // no monomial form (RBF): the stored FP32-tier values with theirs
      if (ba >= 0.0f) da = (double)ba;
      if (bb >= 0.0f) db = (double)bb;
    }
  }
  const double t = fa / (fa - fb);
#pragma unroll
  for (int j = 0; j < D; ++j) p[j] = fma(t, xb[j] - xa[j], xa[j]);
  if (exact) return true;
  const double num = da + db + 2.0 * Q.B64;
  const double den = fabs(fa) + fabs(fb) - num;
  if (!(den > 0.0) || (fa < 0.0) == (fb < 0.0)) return false;
  double dx = 0.0, pn = 1.0;
#pragma unroll
  for (int j = 0; j < D; ++j) {
    dx = fmax(dx, fabs(xb[j] - xa[j]));
    pn = fmax(pn, fabs(p[j]));
  }
  return (num / den) * dx + 1e-15 * pn <= 0.5e-5 * pn;
}

// Record an edge whose point must be recomputed from FP64 values: its index
// goes to redo, the ends that hold FP32 values go to fb, each vertex once
// (the first edge to set its bit in the queued-slot bitmap qb lists it).
__device__ __forceinline__ void queue_fp64(uint64_t slot, const float *vb, uint32_t *fb, uint32_t *qb, Counters *ctr) {
  if (!(vb[slot] >= 0.0f)) return;
  const uint32_t bit = 1u << (slot & 31u);
  if (atomicOr(qb + (slot >> 5), bit) & bit) return;
  fb[atomicAdd(&ctr->n_fb, 1ull)] = (uint32_t)slot;
}
__device__ __forceinline__ void need_fp64(uint64_t i, uint64_t sa, uint64_t sb, const float *vb, uint64_t *redo,
                                          uint32_t *fb, uint32_t *qb, Counters *ctr) {
  redo[atomicAdd(&ctr->n_aux, 1ull)] = i;
  queue_fp64(sa, vb, fb, qb, ctr);
  queue_fp64(sb, vb, fb, qb, ctr);
}

// Points of the traced edges, f read from the slots carried by the edges.
// REDO = false: all edges (also clears the sign bits into keys);
// REDO = true : the edges listed in redo, after their ends went to FP64.
template <int D, bool REDO>
__global__ void points_kernel(LatDev L, const OutRec *out, uint64_t n, const VEnt *vt, uint64_t *keys, double *pts,
                              int64_t ld, bool cert, const float *vb, PolyDev Q, uint64_t *redo, uint32_t *fb,
                              uint32_t *qb, Counters *ctr) {
  for (uint64_t q = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t i = REDO ? redo[q] : q;
    const OutRec o = out[i];
    const uint64_t key = o.key & ~IP_SIGN_BIT;
    if (!REDO) keys[i] = key;
    int32_t a[D], b[D];
    uint32_t R;
    eunpack<D>(L, key, a, &R);
#pragma unroll
    for (int j = 0; j < D; ++j) b[j] = a[j] + (int32_t)((R >> j) & 1u);
    const uint64_t sa = o.slots & 0xffffffffull, sb = o.slots >> 32;
    double p[D];
    const bool ok = edge_point<D>(L, Q, a, b, vt[sa].f, vt[sb].f, cert && !REDO, cert ? vb[sa] : -1.0f,
                                  cert ? vb[sb] : -1.0f, p);
#pragma unroll
    for (int j = 0; j < D; ++j) pts[(int64_t)j * ld + (int64_t)i] = p[j];
    if (!ok) need_fp64(i, sa, sb, vb, redo, fb, qb, ctr);
  }
}

__global__ void vt_rehash_kernel(const VEnt *old, const float *ovb, uint64_t ocap, VEnt *nt, float *nvb,
                                 uint64_t nmask, Counters *ctr) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ocap; i += (uint64_t)gridDim.x * blockDim.x) {
    const VEnt e = old[i];
    if (e.key == IP_EMPTY_KEY) continue;
    uint64_t slot;
    if (vt_insert(nt, nmask, e.key, &slot) >= 0) {
      nt[slot].f = e.f;
      nt[slot].m[0] = e.m[0];
      nt[slot].m[1] = e.m[1];
      if (nvb) nvb[slot] = ovb[i];
    } else {
      atomicOr(&ctr->vt_fail, 1u);
    }
  }
}

__global__ void vt_scan_pending_kernel(const VEnt *vt, uint64_t cap, uint32_t *list, Counters *ctr) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < cap; i += (uint64_t)gridDim.x * blockDim.x) {
    if (vt[i].key == IP_EMPTY_KEY) continue;
    if ((uint64_t)__double_as_longlong(vt[i].f) == IP_UNEVAL_BITS) {
      unsigned long long idx = atomicAdd(&ctr->n_eval, 1ull);
      list[idx] = (uint32_t)i;
    }
  }
}

// After VT moved, point the traced edges at the new slots of their ends.
template <int D>
__global__ void remap_slots_kernel(LatDev L, OutRec *out, uint64_t n, const VEnt *vt, uint64_t vt_mask,
                                   Counters *ctr) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    int32_t a[D], b[D];
    uint32_t R;
    eunpack<D>(L, out[i].key, a, &R);
#pragma unroll
    for (int j = 0; j < D; ++j) b[j] = a[j] + (int32_t)((R >> j) & 1u);
    const int64_t sa = vt_find(vt, vt_mask, vpack<D>(L, a));
    const int64_t sb = vt_find(vt, vt_mask, vpack<D>(L, b));
    if (sa < 0 || sb < 0) atomicOr(&ctr->vt_fail, 2u);
    out[i].slots = (uint64_t)(sa < 0 ? 0 : sa) | ((uint64_t)(sb < 0 ? 0 : sb) << 32);
  }
}

__global__ void et_rebuild_keys_kernel(const uint64_t *keys, uint64_t n, uint64_t *et, uint64_t mask, Counters *ctr) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t slot;
    if (ht_insert(et, mask, keys[i], &slot) < 0) atomicOr(&ctr->et_fail, 1u);
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

struct Run {
  ip_ctx *ctx;
  const ip_problem *p;
  VtBufs *tb = nullptr;   // the context buffers that hold this run's vertex table
  LatDev L;
  VEnt *vt = nullptr;
  uint64_t vt_cap = 0;
  uint32_t *eval = nullptr;
  OutRec *out = nullptr;
  uint64_t out_cap = 0;
  uint32_t *cslot = nullptr;
  int64_t regrows = 0;
  bool cert = false;      // FP32 certified evaluation (else canonical FP64)
  float *vb = nullptr;    // per-slot bound of the stored f (cert only)
  uint32_t *fb = nullptr; // FP64 fallback list
  uint64_t fb_cap = 0;
  int64_t n_fallback = 0;
  int64_t n_settled64 = 0;
};

// Progress lines on stderr when the environment sets IP_LOG (diagnostics of
// long traces; off by default).
bool log_on() {
  static const bool on = getenv("IP_LOG") != nullptr;
  return on;
}

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

// Clears both failure flags, which share one aligned 8-byte word.
int zero_fail_flags(ip_ctx *ctx) {
  static_assert(offsetof(Counters, vt_fail) % 8 == 0 && offsetof(Counters, et_fail) == offsetof(Counters, vt_fail) + 4,
                "failure flags must share one 8-byte word");
  return zero_field(ctx, (unsigned long long *)&ctx->ctr_dev->vt_fail);
}

int fill(ip_ctx *ctx, void *p, uint64_t n, uint64_t v) {
  if (n == 0) return IP_OK;
  hipLaunchKernelGGL(fill_u64_kernel, dim3(grid_for(n)), dim3(kBlock), 0, ctx->stream, (uint64_t *)p, n, v);
  IP_TRY_HIP(ctx, hipGetLastError());
  return IP_OK;
}

int fill_vt(ip_ctx *ctx, VEnt *p, uint64_t n) {
  if (n == 0) return IP_OK;
  hipLaunchKernelGGL(fill_vent_kernel, dim3(grid_for(n)), dim3(kBlock), 0, ctx->stream, p, n);
  IP_TRY_HIP(ctx, hipGetLastError());
  return IP_OK;
}

int alloc(ip_ctx *ctx, void **p, size_t bytes) { return ip_dalloc(ctx, p, bytes); }

void release(ip_ctx *ctx, void *p) { ip_dfree(ctx, p); }

// Vertex table of capacity cap (power of two), reusing the buffers s.tb.
int vt_init(Run &s, uint64_t cap) {
  ip_ctx *ctx = s.ctx;
  VtBufs &tb = *s.tb;
  IP_TRY(ip_ensure(ctx, tb.keys, cap * sizeof(VEnt)));
  IP_TRY(ip_ensure(ctx, tb.eval, cap * 4));
  s.vt = (VEnt *)tb.keys.p;
  s.eval = (uint32_t *)tb.eval.p;
  s.vt_cap = cap;
  IP_TRY(fill_vt(ctx, s.vt, cap));
  if (s.cert) {
    IP_TRY(ip_ensure(ctx, tb.vals, cap * 4));
    IP_TRY(ip_ensure(ctx, tb.fb, cap * 4));
    s.vb = (float *)tb.vals.p;
    s.fb = (uint32_t *)tb.fb.p;
    s.fb_cap = tb.fb.bytes / 4;
  }
  return IP_OK;
}

template <int D>
int remap_out(Run &s, uint64_t n_out) {
  if (n_out == 0) return IP_OK;
  ip_ctx *ctx = s.ctx;
  hipLaunchKernelGGL((remap_slots_kernel<D>), dim3(grid_for(n_out)), dim3(kBlock), 0, ctx->stream, s.L, s.out, n_out,
                     s.vt, s.vt_cap - 1, ctx->ctr_dev);
  IP_TRY_HIP(ctx, hipGetLastError());
  return IP_OK;
}

// Grow VT to new_cap: rehash into a fresh table, re-point the first n_out
// traced edges, rebuild the pending-evaluation list.
template <int D>
int vt_grow(Run &s, uint64_t new_cap, uint64_t n_out) {
  ip_ctx *ctx = s.ctx;
  if (new_cap > (1ull << 32)) return ip_fail(ctx, IP_ENOMEM, "vertex table above 2^32 entries");
  void *nt = nullptr, *nl = nullptr, *nvb = nullptr;
  IP_TRY(alloc(ctx, &nt, new_cap * sizeof(VEnt)));
  IP_TRY(alloc(ctx, &nl, new_cap * 4));
  if (s.cert) IP_TRY(alloc(ctx, &nvb, new_cap * 4));
  IP_TRY(fill_vt(ctx, (VEnt *)nt, new_cap));
  hipLaunchKernelGGL(vt_rehash_kernel, dim3(grid_for(s.vt_cap)), dim3(kBlock), 0, ctx->stream, s.vt,
                     (const float *)s.vb, s.vt_cap, (VEnt *)nt, (float *)nvb, new_cap - 1, ctx->ctr_dev);
  IP_TRY_HIP(ctx, hipGetLastError());
  IP_TRY(zero_field(ctx, &ctx->ctr_dev->n_eval));
  hipLaunchKernelGGL(vt_scan_pending_kernel, dim3(grid_for(new_cap)), dim3(kBlock), 0, ctx->stream,
                     (const VEnt *)nt, new_cap, (uint32_t *)nl, ctx->ctr_dev);
  IP_TRY_HIP(ctx, hipGetLastError());
  IP_TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));
  VtBufs &tb = *s.tb;
  release(ctx, tb.keys.p);
  release(ctx, tb.eval.p);
  tb.keys = {nt, new_cap * sizeof(VEnt)};
  tb.eval = {nl, new_cap * 4};
  s.vt = (VEnt *)nt;
  s.eval = (uint32_t *)nl;
  s.vt_cap = new_cap;
  if (s.cert) {
    release(ctx, tb.vals.p);
    tb.vals = {nvb, new_cap * 4};
    s.vb = (float *)nvb;
    IP_TRY(ip_ensure(ctx, tb.fb, new_cap * 4));
    s.fb = (uint32_t *)tb.fb.p;
    s.fb_cap = tb.fb.bytes / 4;
  }
  IP_TRY(remap_out<D>(s, n_out));
  ++s.regrows;
  return IP_OK;
}

int out_reserve(Run &s, uint64_t need, uint64_t n_used) {
  if (need <= s.out_cap) return IP_OK;
  ip_ctx *ctx = s.ctx;
  uint64_t cap = std::max<uint64_t>(need, s.out_cap * 2);
  void *nb = nullptr;
  IP_TRY(alloc(ctx, &nb, cap * sizeof(OutRec)));
  if (n_used)
    IP_TRY_HIP(ctx, hipMemcpyAsync(nb, s.out, n_used * sizeof(OutRec), hipMemcpyDeviceToDevice, ctx->stream));
  IP_TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (s.out) release(ctx, s.out);
  s.out = (OutRec *)nb;
  s.out_cap = cap;
  return IP_OK;
}

int cslot_reserve(Run &s, uint64_t need) {
  ip_ctx *ctx = s.ctx;
  IP_TRY(ip_ensure(ctx, ctx->vt_aux, std::max<uint64_t>(need, 1024) * 4));
  s.cslot = (uint32_t *)ctx->vt_aux.p;
  return IP_OK;
}

// f at the listed pending vertices: canonical FP64, or FP32 certified with
// canonical FP64 for the vertices the bound cannot settle.
int eval_pending(Run &s, uint64_t n) {
  if (!s.cert) return launch_feval64(s.ctx, s.p, s.L, s.eval, n, s.vt);
  ip_ctx *ctx = s.ctx;
  if (n == 0) return IP_OK;
  IP_TRY(zero_field(ctx, &ctx->ctr_dev->n_fb));
  IP_TRY(zero_field(ctx, &ctx->ctr_dev->n_cert64));
  IP_TRY(launch_feval32(ctx, s.p, s.L, s.eval, n, s.vt, s.vb, s.fb, &ctx->ctr_dev->n_fb));
  IP_TRY(read_ctr(ctx));
  const uint64_t nfb = ctx->ctr_host->n_fb;
  s.n_fallback += (int64_t)nfb;
  s.n_settled64 += (int64_t)ctx->ctr_host->n_cert64;
  return launch_feval64(ctx, s.p, s.L, s.fb, nfb, s.vt);
}

// eval_pending without the host read of the fallback count: the canonical
// pass is sized on the device (at most n), and the caller takes the level's
// fallback counts from its next counter read.
int eval_pending_async(Run &s, uint64_t n) {
  if (!s.cert) return launch_feval64(s.ctx, s.p, s.L, s.eval, n, s.vt);
  ip_ctx *ctx = s.ctx;
  if (n == 0) return IP_OK;
  IP_TRY(zero_field(ctx, &ctx->ctr_dev->n_fb));
  IP_TRY(zero_field(ctx, &ctx->ctr_dev->n_cert64));
  IP_TRY(launch_feval32(ctx, s.p, s.L, s.eval, n, s.vt, s.vb, s.fb, &ctx->ctr_dev->n_fb));
  return launch_feval64_dev(ctx, s.p, s.L, s.fb, n, &ctx->ctr_dev->n_fb, s.vt);
}

template <int D, bool EDGES>
int level_pass(Run &s, uint64_t lo, uint64_t hi) {
  ip_ctx *ctx = s.ctx;
  unsigned grid = grid_for((hi - lo) * 4, 8192);
  hipLaunchKernelGGL((expand_kernel<D, EDGES>), dim3(grid), dim3(kBlock), 0, ctx->stream, s.L, s.out, lo, hi, s.vt,
                     s.vt_cap - 1, s.cslot, s.eval, ctx->ctr_dev);
  IP_TRY_HIP(ctx, hipGetLastError());
  return IP_OK;
}

// Direct trace on lattice s.L (fine, or coarse in batch mode).  On return
// s.out[0 .. *n_out) holds the traced edges and VT holds f at their ends.
template <int D>
int trace_direct(Run &s, ip_stats &st, uint64_t *n_out_ret) {
  constexpr uint64_t MAXC = (1u << D) - 2;
  ip_ctx *ctx = s.ctx;
  const ip_problem *p = s.p;
  Counters *c = ctx->ctr_host;
  Timer tf, tx;
  IP_TRY_HIP(ctx, hipMemsetAsync(ctx->ctr_dev, 0, sizeof(Counters), ctx->stream));
  // locate
  const unsigned sg = (unsigned)((p->n_seeds + 127) / 128);
  for (int guard = 0;; ++guard) {
    if (guard > 40) return ip_fail(ctx, IP_ENOMEM, "vertex table cannot grow");
    hipLaunchKernelGGL((seed_vertices_kernel<D>), dim3(sg), dim3(128), 0, ctx->stream, s.L, p->seeds_dev, p->n_seeds,
                       s.vt, s.vt_cap - 1, s.eval, ctx->ctr_dev);
    IP_TRY_HIP(ctx, hipGetLastError());
    IP_TRY(read_ctr(ctx));
    if (!c->vt_fail) break;
    IP_TRY(zero_fail_flags(ctx));
    IP_TRY(vt_grow<D>(s, s.vt_cap * 4, 0));
  }
  IP_TRY(tf.start(ctx, &st.ms_feval));
  IP_TRY(eval_pending(s, c->n_eval));
  IP_TRY(tf.stop(ctx));
  IP_TRY(out_reserve(s, (uint64_t)p->n_seeds * (D + 1) * D / 2 + 1024, 0));
  hipLaunchKernelGGL((seed_edges_kernel<D>), dim3(sg), dim3(128), 0, ctx->stream, s.L, p->seeds_dev, p->n_seeds, s.vt,
                     s.vt_cap - 1, s.out, ctx->ctr_dev);
  IP_TRY_HIP(ctx, hipGetLastError());
  IP_TRY(read_ctr(ctx));
  uint64_t lo = 0, hi = c->n_out;
  int levels = 0;
  uint64_t cof_total = 0;
  while (hi > lo) {
    ++levels;
    IP_TRY(cslot_reserve(s, ((hi - lo + 63) / 64) * 64 * MAXC));
    // pass 1: third vertices
    IP_TRY(zero_field(ctx, &ctx->ctr_dev->n_eval));
    IP_TRY(zero_field(ctx, &ctx->ctr_dev->n_cof));
    IP_TRY(tx.start(ctx, &st.ms_expand));
    IP_TRY((level_pass<D, false>(s, lo, hi)));
    IP_TRY(tx.stop(ctx));
    IP_TRY(read_ctr(ctx));
    int guard = 0;
    while (c->vt_fail || c->vt_count * 2 > s.vt_cap) {
      if (++guard > 40) return ip_fail(ctx, IP_ENOMEM, "vertex table cannot grow");
      IP_TRY(zero_fail_flags(ctx));
      IP_TRY(vt_grow<D>(s, pow2_at_least(c->vt_count * 4), hi));
      // slots moved: replay pass 1 so CSL points into the new table; it
      // finds the inserted vertices and lists the missing ones after the
      // rebuilt pending list
      IP_TRY(zero_field(ctx, &ctx->ctr_dev->n_cof));
      IP_TRY((level_pass<D, false>(s, lo, hi)));
      IP_TRY(read_ctr(ctx));
      if (c->vt_fail & 2u) return ip_fail(ctx, IP_EDEVICE, "internal: traced edge lost its vertex");
    }
    cof_total += c->n_cof;
    const bool evaluated = c->n_eval > 0;
    IP_TRY(tf.start(ctx, &st.ms_feval));
    IP_TRY(eval_pending_async(s, c->n_eval));
    IP_TRY(tf.stop(ctx));
    // pass 2: new edges; OUT must hold one new edge per coface at most
    IP_TRY(out_reserve(s, hi + c->n_cof + 1, hi));
    IP_TRY(tx.start(ctx, &st.ms_expand));
    IP_TRY((level_pass<D, true>(s, lo, hi)));
    IP_TRY(tx.stop(ctx));
    IP_TRY(read_ctr(ctx));
    if (s.cert && evaluated) {
      // this level's FP32 evaluation left these counts
      s.n_fallback += (int64_t)c->n_fb;
      s.n_settled64 += (int64_t)c->n_cert64;
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

__global__ void count_ncof_kernel(const OutRec *edges, uint64_t n, int D, int B, unsigned long long *total) {
  unsigned long long acc = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t R = (uint32_t)((edges[i].key & ~IP_SIGN_BIT) >> (D * B)) & ((1u << D) - 1u);
    int nR = __popc(R);
    acc += (unsigned long long)(ifact(nR) * ifact(D + 1 - nR));
  }
  if (acc) atomicAdd(total, acc);
}

// Sec. V-B: n-simplex cofaces of the coarse intersecting edges, hashed to
// remove duplicates; the winners are listed in discovery order.
template <int D>
__global__ __launch_bounds__(kBlock) void sigma_kernel(LatDev Lc, int LB, const OutRec *__restrict__ edges,
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
      e = edges[ei].key;
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

// The same point from the inverse order: coordinate c carries template
// coordinate winv[c] (w[winv[c]] = c); no register array is indexed at run
// time.
template <int D>
__device__ __forceinline__ void template_point_inv(const int32_t *v, const int32_t *winv, int k, uint64_t up,
                                                   int32_t *y) {
#pragma unroll
  for (int c = 0; c < D; ++c) y[c] = k * v[c] + (int32_t)((up >> (8 * winv[c])) & 0xffu);
}

template <int D>
__device__ __forceinline__ void perm_inverse(const int32_t *w, int32_t *winv) {
#pragma unroll
  for (int c = 0; c < D; ++c) {
    int32_t r = 0;
#pragma unroll
    for (int i = 0; i < D; ++i) r = w[i] == c ? i : r;
    winv[c] = r;
  }
}

// Fine vertices of a batch of coarse simplices: insert into the batch vertex
// table, remember the slot of every (simplex, template point).
template <int D>
__global__ __launch_bounds__(kBlock) void batch_vertices_kernel(LatDev Lf, LatDev Lc, int LB, int k,
                                                                const uint64_t *__restrict__ sig, uint64_t nb,
                                                                const uint64_t *__restrict__ tpts, int NP,
                                                                VEnt *vt, uint64_t vt_mask,
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
        int ins = vt_insert(vt, vt_mask, vpack<D>(Lf, y), &slot);
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

// Intersection points of the edges keys[lo .. hi) from the values of their
// ends in the batch vertex table: canonical FP64 values, or (CERT) the
// FP32-tier values with their bounds vb, an edge whose point the bound
// cannot place within tolerance listed in redo (by its index in keys).
template <int D, bool CERT>
__global__ void batch_points_kernel(LatDev L, const uint64_t *keys, uint64_t lo, uint64_t hi, const VEnt *vt,
                                    const float *vb, uint64_t vt_mask, double *pts, int64_t ld, PolyDev Q,
                                    uint64_t *redo, Counters *ctr) {
  for (uint64_t i = lo + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < hi; i += (uint64_t)gridDim.x * blockDim.x) {
    int32_t a[D], b[D];
    uint32_t R;
    eunpack<D>(L, keys[i], a, &R);
#pragma unroll
    for (int j = 0; j < D; ++j) b[j] = a[j] + (int32_t)((R >> j) & 1u);
    const int64_t ha = vt_find(vt, vt_mask, vpack<D>(L, a));
    const int64_t hb = vt_find(vt, vt_mask, vpack<D>(L, b));
    const double fa = ha >= 0 ? vt[ha].f : NAN;
    const double fb = hb >= 0 ? vt[hb].f : NAN;
    double p[D];
    const float ba = CERT && ha >= 0 ? vb[ha] : -1.0f, bb = CERT && hb >= 0 ? vb[hb] : -1.0f;
    const bool ok = edge_point<D>(L, Q, a, b, fa, fb, CERT, ba, bb, p);
#pragma unroll
    for (int j = 0; j < D; ++j) pts[(int64_t)j * ld + (int64_t)i] = p[j];
    if (CERT && !ok) redo[atomicAdd(&ctr->n_aux, 1ull)] = i;
  }
}

// ---------------------------------------------------------------------------
// Subdivision kernel (Sec. V-B, Fig. 6): one wave per coarse simplex.
//
// Ownership.  A fine edge lies in the relative interior of exactly one face
// tau of the coarse simplex (vertices: the union of the supports of its
// ends' barycentric coordinates, precomputed per template edge), and every
// coarse n-simplex containing tau sees it.  If tau contains a traced coarse
// edge, every n-coface of tau is in Sigma (they are n-cofaces of that edge),
// so the edge is emitted only by the canonical n-coface of tau: the one
// whose roots run in ascending order within each block of tau's partition.
// Those edges go straight to the output list (out_d) with no dedup.  The
// other intersecting edges go through the global edge set (et_keys), whose
// new keys are appended to out_s.
//
// Active faces.  Whether this simplex takes the edges of face tau depends
// only on the coarse trace (tau traced or not, this simplex canonical for
// tau or not), not on f.  Both are bit masks over the 2^(d+1) vertex subsets
// V, formed from two per-simplex facts: the traced coarse edges (i, j) among
// its vertices (V is traced when it holds one: the union over them of
// {V : i, j in V}), and the positions p where the root sequence descends (V
// is canonical when it holds all of them: the ascending-roots rule read
// position by position).  The wave takes the sign of f only at the template
// points of active faces' edges, and tests only the edges of active faces
// whose points carry both signs: the template edges are grouped by face, and
// those groups are laid end to end in a virtual index space [0, T) that the
// lanes walk 64 at a time (a bitmap of group starts maps a virtual index to
// its group).
//
// Preparation.  The masks and the tier-1 bound of a simplex (D + 1 probes of
// the coarse vertex table, the frame at its D + 1 vertices, one pass over
// the monomials) are computed beforehand by sub_prep_kernel, one lane per
// coarse simplex, rather than on D + 1 of the wave's 64 lanes.
//
// Sign codes.  The signs are kept in LDS as byte codes: 0 (f < 0), 1
// (f >= 0), 2 (outside the box), 3 (neither certified tier settles the
// sign).
//   MODE 0: FP32-certified signs of sig[0 .. n) (no vertex table: a point
//           shared by several coarse simplices is evaluated by each of them,
//           which costs fewer cycles than a probe into a table of 10^8
//           vertices); a simplex with a code-3 point goes to `defer`.
//   MODE 1: the deferred simplices: their code-3 points are inserted into
//           the fallback vertex table fvt (new slots to eval_list).
//   MODE 2: the deferred simplices again, code-3 points taking the sign of
//           the canonical FP64 value in fvt; then the edge pass.
//   MODE 3: FP64 mode: the sign of template point p of simplex s is read
//           from fvt[pslot[s * NP + p]].f (pslot ~0: outside the box).
// ---------------------------------------------------------------------------
constexpr int kSubStage = 128;
constexpr int kWaves = kBlock / 64;

constexpr int kEdgeStage = 128;

// Dynamic LDS of one block, as byte offsets (each array 16-byte aligned).
// Shared by the block: the fine frame (M row-major stride 8, then o, lo, hi),
// the monomial coefficients (FP64 and FP32), the template points with their
// face masks, the faces' point masks, the edges and face groups.  Per wave:
// two append stages, the start bitmap, the sign masks over the points and
// the list of the active groups, the edge stage, the active point list and
// the sign codes.
struct SubLayout {
  uint32_t lmat, lc, stage_s, stage_d, lpts, lpf, lpv, sbm, est, ledge, lgrp, lmask, agl, plist, code, total;
};

__host__ __device__ inline uint32_t sub_take(uint32_t &o, size_t bytes) {
  const uint32_t r = o;
  o += (uint32_t)((bytes + 15) & ~(size_t)15);
  return r;
}

// NP template points, NE template edges, M monomials (0: no coefficients),
// NV = 2^(d+1) vertex subsets.
// The frame and the FP32 coefficients come first, at fixed offsets (0 and
// kSubLc), so that the evaluation reads them with immediate offsets.
constexpr uint32_t kSubLc = 88 * 8;
__host__ __device__ inline SubLayout sub_layout(int NP, int NE, int M, int NV) {
  const int NVW = (NV + 63) / 64, NPW = (NP + 63) / 64, SBW = (NE + 63) / 64;
  SubLayout L;
  uint32_t o = 0;
  L.lmat = sub_take(o, 88 * 8);
  L.lc = sub_take(o, (size_t)M * 4);
  L.stage_s = sub_take(o, (size_t)kWaves * kSubStage * 8);
  L.stage_d = sub_take(o, (size_t)kWaves * kSubStage * 8);
  L.lpts = sub_take(o, (size_t)NP * 8);
  L.lpf = sub_take(o, (size_t)NP * NVW * 8);
  L.lpv = sub_take(o, (size_t)NV * NPW * 8);
  L.sbm = sub_take(o, (size_t)kWaves * SBW * 8);
  L.est = sub_take(o, (size_t)kWaves * kEdgeStage * 4);
  L.ledge = sub_take(o, (size_t)NE * 4);
  L.lgrp = sub_take(o, (size_t)NV * 4);
  L.lmask = sub_take(o, (size_t)kWaves * 2 * NPW * 8);
  L.agl = sub_take(o, (size_t)kWaves * NV * 4);
  L.plist = sub_take(o, (size_t)kWaves * NP * 2);
  L.code = sub_take(o, (size_t)kWaves * NP);
  L.total = o;
  return L;
}

// lat_coords / lat_in_box with the frame at M (row-major, stride 8), then
// o, lo, hi at M + 64, 72, 80: the same operations in the same order.
template <int D>
__device__ __forceinline__ void lat_coords_m(const double *M, const int32_t *v, double *x) {
#pragma unroll
  for (int j = 0; j < D; ++j) {
    double acc = M[64 + j];
#pragma unroll
    for (int k = 0; k < D; ++k) acc = fma(M[j * 8 + k], (double)v[k], acc);
    x[j] = acc;
  }
}

template <int D>
__device__ __forceinline__ bool in_box_m(const double *M, const double *x) {
  bool ok = true;
#pragma unroll
  for (int j = 0; j < D; ++j) ok = ok & (x[j] >= M[72 + j]) & (x[j] <= M[80 + j]);
  return ok;
}

struct SubOut {
  const VEnt *cvt;   // coarse vertex table (visited-edge masks of the coarse trace)
  uint64_t cvt_mask;
  uint64_t *et_keys;  // global edge set (edges without an owner)
  uint64_t et_mask;
  uint64_t *out_s;    // its keys in insertion order
  uint64_t *out_d;    // owner-emitted keys
  uint64_t dcap;      // capacity of out_d (appends past it are counted, not written)
};

// Bit b of word t set when vertex i belongs to the vertex subset 64 t + b.
__host__ __device__ constexpr uint64_t vertex_pattern(int i, int t) {
  return i == 0   ? 0xAAAAAAAAAAAAAAAAull
         : i == 1 ? 0xCCCCCCCCCCCCCCCCull
         : i == 2 ? 0xF0F0F0F0F0F0F0F0ull
         : i == 3 ? 0xFF00FF00FF00FF00ull
         : i == 4 ? 0xFFFF0000FFFF0000ull
         : i == 5 ? 0xFFFFFFFF00000000ull
                  : (((t >> (i - 6)) & 1) ? ~0ull : 0ull);
}

// What the subdivision of one coarse simplex takes from the coarse trace and
// the frame: its tier-1 bound B1 and two masks over the 2^(D+1) vertex
// subsets V of the simplex (bit V - 64 t of word t): A, the active faces,
// and TR, the traced ones.
template <int D>
struct SubPrep {
  static constexpr int NVW = ((1 << (D + 1)) + 63) / 64;
  double B1;
  uint64_t A[NVW], TR[NVW];
};

// One lane per coarse simplex sig[i], i < n (grid-stride).  Vertex i of the
// simplex is v + 1_{w_0 .. w_{i-1}}; edge (i, j) has direction
// R = {w_i .. w_{j-1}} from vertex i and is traced when bit R of that
// vertex's visited-edge mask is set.  Face V is traced when it holds a
// traced edge (i, j): the union over them of {V : i, j in V}.  It is
// canonical when it holds every position p whose root is below the root
// before it, cyclically (roots w_0 .. w_{D-1}, D; p = 0 always): the
// ascending-roots rule read position by position.  Active = not traced, or
// canonical; V = 0 never.  The bound: |x_j| is largest at a vertex (fine
// coordinates k (v + 1_{w_0 .. w_{i-1}})), so with X_j the maximum over the
// vertices, B1 = K32n sum_m |c_m| X^m + E0 covers every template point
// (BOUND false: B1 = 0, the FP64 mode).
template <int D, bool BOUND>
__global__ __launch_bounds__(kBlock) void sub_prep_kernel(LatDev Lf, LatDev Lc, int LB, int k,
                                                          const uint64_t *__restrict__ sig, uint64_t n,
                                                          const VEnt *__restrict__ cvt, uint64_t cvt_mask, PolyDev Q,
                                                          SubPrep<D> *__restrict__ out) {
  constexpr int NV = 1 << (D + 1), NVW = SubPrep<D>::NVW;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    int32_t v[D], w[D];
    sig_unpack<D>(Lc, sig[i], LB, v, w);
    uint64_t rows = 0;
    double X[D];
#pragma unroll
    for (int j = 0; j < D; ++j) X[j] = 0.0;
    int32_t cv[D];
#pragma unroll
    for (int c = 0; c < D; ++c) cv[c] = v[c];
    for (int vi = 0; vi <= D; ++vi) {
      if (vi > 0) {
#pragma unroll
        for (int c = 0; c < D; ++c) cv[c] += c == w[vi - 1] ? 1 : 0;
      }
      if (BOUND) {
#pragma unroll
        for (int j = 0; j < D; ++j) {
          double acc = Lf.o[j];
#pragma unroll
          for (int c = 0; c < D; ++c) acc = fma(Lf.M[j * 8 + c], (double)(k * cv[c]), acc);
          X[j] = fmax(X[j], fabs(acc));
        }
      }
      if (vi == D || !vin_range<D>(Lc, cv)) continue;
      const int64_t h = vt_find(cvt, cvt_mask, vpack<D>(Lc, cv));
      if (h < 0) continue;
      const uint64_t m0 = cvt[h].m[0], m1 = cvt[h].m[1];
      uint32_t R = 0;
      for (int j = vi + 1; j <= D; ++j) {
        R |= 1u << w[j - 1];
        const uint64_t word = R < 64 ? m0 : m1;
        if ((word >> (R & 63u)) & 1ull) rows |= 1ull << (8 * vi + j);
      }
    }
    SubPrep<D> r;
    uint32_t desc = 1u;
#pragma unroll
    for (int q = 1; q < D; ++q) desc |= w[q] < w[q - 1] ? 1u << q : 0u;
#pragma unroll
    for (int t = 0; t < NVW; ++t) {
      uint64_t tr = 0, cn = ~0ull;
#pragma unroll
      for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = a + 1; b <= D; ++b)
          if ((rows >> (8 * a + b)) & 1ull) tr |= vertex_pattern(a, t) & vertex_pattern(b, t);
#pragma unroll
      for (int q = 0; q < D; ++q)
        if ((desc >> q) & 1u) cn &= vertex_pattern(q, t);
      uint64_t valid = NV >= 64 ? ~0ull : (1ull << (NV & 63)) - 1ull;
      if (t == 0) valid &= ~1ull;
      r.TR[t] = tr & valid;
      r.A[t] = (~tr | cn) & valid;
    }
    r.B1 = 0.0;
    if (BOUND) {
#pragma unroll
      for (int j = 0; j < D; ++j) X[j] = X[j] * (1.0 + 1e-12) + 1e-300;
      double t = 0.0;
      for (int m = 0; m < Q.M; ++m) {
        const uint32_t pk = Q.mono[m];
        double term = fabs(Q.cd[m]);
        for (int q = 0; q < (int)(pk & 15u); ++q) {
          const uint32_t jj = (pk >> (4 + 4 * q)) & 15u;
          double xj = X[0];
#pragma unroll
          for (int j = 1; j < D; ++j) xj = jj == (uint32_t)j ? X[j] : xj;
          term *= xj;
        }
        t += term;
      }
      r.B1 = Q.K32n * (t * (1.0 + 1e-12)) + Q.E0;
    }
    out[i] = r;
  }
}

__device__ __forceinline__ uint64_t readlane64(uint64_t x, int j) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, j);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), j);
  return ((uint64_t)hi << 32) | lo;
}

// Four waves per SIMD (the LDS allows four blocks per CU): the register cap
// this sets costs a few spilled registers, fewer than a wave of occupancy.
template <int D, int P, int MODE>
__global__ __launch_bounds__(kBlock, 4) void subdivide_kernel(LatDev Lf, LatDev Lc, int LB, int k,
                                                           const uint64_t *__restrict__ sig,
                                                           const uint32_t *__restrict__ list, uint64_t n,
                                                           const uint64_t *__restrict__ tpts, int NP,
                                                           const uint32_t *__restrict__ tedge, int NE,
                                                           const uint32_t *__restrict__ tgrp,
                                                           const uint64_t *__restrict__ tpf,
                                                           const uint64_t *__restrict__ tpv, PolyDev Q,
                                                           VEnt *fvt, uint64_t fvt_mask, uint32_t *eval_list,
                                                           const uint32_t *__restrict__ pslot,
                                                           const SubPrep<D> *__restrict__ prep, SubOut so,
                                                           uint32_t *defer, Counters *ctr) {
  constexpr int NV = 1 << (D + 1);        // vertex subsets of a coarse simplex
  constexpr int NVW = (NV + 63) / 64;     // 64-bit words per face mask
  extern __shared__ __align__(16) unsigned char smem[];
  // the wave index is wave-uniform: say so, so that the simplex index, its
  // key and (v, w) live in scalar registers
  const int wib = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const uint64_t lt_mask = (1ull << lane) - 1ull;
  const int M = MODE == 3 ? 0 : Q.M;
  const int SBW = (NE + 63) / 64;
  const int NPW = (NP + 63) / 64;
  const SubLayout Ly = sub_layout(NP, NE, M, NV);
  uint64_t *stage_s = (uint64_t *)(smem + Ly.stage_s) + (size_t)wib * kSubStage;
  uint64_t *stage_d = (uint64_t *)(smem + Ly.stage_d) + (size_t)wib * kSubStage;
  // fine frame and FP32 coefficients in LDS at fixed offsets: read at
  // wave-uniform addresses, they stay out of the scalar registers
  double *lmat = (double *)smem;
  float *lc = (float *)(smem + kSubLc);
  uint64_t *lpts = (uint64_t *)(smem + Ly.lpts);
  uint64_t *lpf = (uint64_t *)(smem + Ly.lpf);
  uint64_t *lpv = (uint64_t *)(smem + Ly.lpv);
  uint64_t *sbm = (uint64_t *)(smem + Ly.sbm) + (size_t)wib * SBW;
  // per wave: the points with f < 0 and those with f >= 0
  uint64_t *mneg = (uint64_t *)(smem + Ly.lmask) + (size_t)wib * 2 * NPW;
  uint64_t *mpos = mneg + NPW;
  uint32_t *est = (uint32_t *)(smem + Ly.est) + (size_t)wib * kEdgeStage;
  uint32_t *ledge = (uint32_t *)(smem + Ly.ledge);
  uint32_t *lgrp = (uint32_t *)(smem + Ly.lgrp);
  uint32_t *agl = (uint32_t *)(smem + Ly.agl) + (size_t)wib * NV;
  uint16_t *plist = (uint16_t *)(smem + Ly.plist) + (size_t)wib * NP;
  uint8_t *code = (uint8_t *)(smem + Ly.code) + (size_t)wib * NP;
  for (int i = threadIdx.x; i < NP; i += kBlock) {
    lpts[i] = tpts[i];
#pragma unroll
    for (int t = 0; t < NVW; ++t) lpf[i * NVW + t] = tpf[i * NVW + t];
  }
  if (threadIdx.x < 64) lmat[threadIdx.x] = Lf.M[threadIdx.x];
  if (threadIdx.x < 8) {
    lmat[64 + threadIdx.x] = Lf.o[threadIdx.x];
    lmat[72 + threadIdx.x] = Lf.lo[threadIdx.x];
    lmat[80 + threadIdx.x] = Lf.hi[threadIdx.x];
  }
  // the FP32 monomial coefficients, read by every lane at the same index,
  // from LDS (kept out of the vector registers)
  for (int i = threadIdx.x; i < M; i += kBlock) lc[i] = Q.c[i];
  for (int i = threadIdx.x; i < NE; i += kBlock) ledge[i] = tedge[i];
  for (int i = threadIdx.x; i < NV; i += kBlock) lgrp[i] = tgrp[i];
  for (int i = threadIdx.x; i < NV * NPW; i += kBlock) lpv[i] = tpv[i];
  __syncthreads();
  int sn = 0, snd = 0;
  auto put_s = [&](unsigned long long pos, uint64_t key) { so.out_s[pos] = key; };
  auto put_d = [&](unsigned long long pos, uint64_t key) {
    if (pos < so.dcap) so.out_d[pos] = key;
  };
  // per-lane tallies (a lane sees far fewer than 2^32 events per launch)
  uint32_t hits = 0, shits = 0, n64 = 0, npts = 0, nuns = 0;
  const uint64_t wave = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) >> 6;
  const uint64_t n_waves = ((uint64_t)gridDim.x * kBlock) >> 6;
  // MODE 0 and 3 walk sig[0 .. n); MODE 1 and 2 walk the deferred list.
  // Each lane holds the index, key and preparation record of one of the
  // wave's next 64 simplices (loaded together, so their latency is paid once
  // per 64); the wave reads the current one out of lane jn.
  uint32_t st_s = 0;
  uint64_t st_key = 0;
  SubPrep<D> st_p = {};
  int jn = 64;
  for (uint64_t it = wave; it < n; it += n_waves) {
    if (jn == 64) {
      const uint64_t itj = it + (uint64_t)lane * n_waves;
      if (itj < n) {
        st_s = (MODE == 0 || MODE == 3) ? (uint32_t)itj : list[itj];
        st_key = sig[st_s];
        st_p = prep[st_s];
      }
      jn = 0;
    }
    const uint64_t s = (uint32_t)__builtin_amdgcn_readlane((int)st_s, jn);
    int32_t v[D], w[D], winv[D];
    sig_unpack<D>(Lc, readlane64(st_key, jn), LB, v, w);
    perm_inverse<D>(w, winv);
    const double B1 = __longlong_as_double((long long)readlane64((uint64_t)__double_as_longlong(st_p.B1), jn));
    uint64_t A[NVW], TR[NVW];
#pragma unroll
    for (int t = 0; t < NVW; ++t) {
      A[t] = readlane64(st_p.A[t], jn);
      TR[t] = readlane64(st_p.TR[t], jn);
    }
    ++jn;
    // active template points: an end of an edge of an active face; every
    // code starts at 2
    int NPA = 0;
    for (int p0 = 0; p0 < NP; p0 += 64) {
      const int pt = p0 + lane;
      bool a = false;
      if (pt < NP) {
        uint64_t hit = 0;
#pragma unroll
        for (int t = 0; t < NVW; ++t) hit |= lpf[pt * NVW + t] & A[t];
        a = hit != 0ull;
        code[pt] = 2;
      }
      const uint64_t bal = __ballot(a);
      if (a) plist[NPA + __popcll(bal & lt_mask)] = (uint16_t)pt;
      NPA += __popcll(bal);
    }
    wave_lds_sync();
    bool unsettled = false;
    for (int i0 = 0; i0 < NPA; i0 += 64) {
      const int i = i0 + lane;
      uint32_t c = 2;
      if (i < NPA) {
        const int pt = plist[i];
        if (MODE == 3) {
          const uint32_t ps = pslot[s * (uint64_t)NP + pt];
          if (ps != 0xffffffffu) c = fvt[ps].f < 0.0 ? 0u : 1u;
        } else {
          int32_t y[D];
          template_point_inv<D>(v, winv, k, lpts[pt], y);
          // an opaque zero base keeps the frame and coefficient reads in the
          // loop (hoisted, the 36 matrix entries alone would pin 72 vector
          // registers), each at an immediate offset from it
          int z = 0;
          asm volatile("" : "+v"(z));
          const double *Mz = lmat + z;
          double x[D];
          lat_coords_m<D>(Mz, y, x);
          if (in_box_m<D>(Mz, x)) {
            double fv;
            PolyDev Qz = Q;
            Qz.c = lc + z;
            const int tier = cert_eval_region<D, P>(Qz, x, B1, &fv);
            if (MODE == 0) ++npts;
            if (tier < 3) {
              c = fv < 0.0 ? 0u : 1u;
            } else if (MODE == 0) {
              c = 3;
              ++nuns;
            } else if (MODE == 1) {
              uint64_t slot;
              const int ins = vt_insert(fvt, fvt_mask, vpack<D>(Lf, y), &slot);
              if (ins == 1)
                eval_list[atomicAdd(&ctr->n_eval, 1ull)] = (uint32_t)slot;
              else if (ins < 0)
                atomicOr(&ctr->vt_fail, 1u);
            } else {
              const int64_t h = vt_find(fvt, fvt_mask, vpack<D>(Lf, y));
              if (h < 0) atomicOr(&ctr->vt_fail, 1u);
              c = (h >= 0 && !(fvt[h].f < 0.0)) ? 1u : 0u;
            }
          }
        }
        code[pt] = (uint8_t)c;
      }
      if (MODE == 0 && __ballot(c == 3)) unsettled = true;
    }
    if (MODE == 1) continue;
    if (MODE == 0 && unsettled) {
      if (lane == 0) defer[atomicAdd(&ctr->n_aux, 1ull)] = (uint32_t)s;
      wave_lds_sync();
      continue;
    }
    wave_lds_sync();
    // sign masks over the template points (f < 0, f >= 0)
    for (int q = 0; q < NPW; ++q) {
      const int pt = 64 * q + lane;
      const uint32_t c = pt < NP ? code[pt] : 2u;
      const uint64_t ng = __ballot(c == 0u), ps = __ballot(c == 1u);
      if (lane == 0) {
        mneg[q] = ng;
        mpos[q] = ps;
      }
    }
    for (int i = lane; i < SBW; i += 64) sbm[i] = 0ull;
    wave_lds_sync();
    // an active face whose edge ends carry both signs gets a slot in agl
    // (first edge | virtual start << 15 | set path << 31) and its virtual
    // start a bit in sbm; one with a single sign has no intersecting edge
    int T = 0, G = 0;
#pragma unroll
    for (int t = 0; t < NVW; ++t) {
      const uint32_t V = (uint32_t)(lane + 64 * t);
      const bool trv = (TR[t] >> lane) & 1ull;
      bool act = (A[t] >> lane) & 1ull;
      uint32_t gd = 0;
      if (act) {
        gd = lgrp[V];
        uint64_t hn = 0, hp = 0;
        for (int q = 0; q < NPW; ++q) {
          const uint64_t pv = lpv[V * NPW + q];
          hn |= pv & mneg[q];
          hp |= pv & mpos[q];
        }
        act = hn != 0ull && hp != 0ull;
      }
      const uint32_t cnt = act ? gd >> 16 : 0u;
      // exclusive prefix sum of cnt over the lanes, one bit plane at a time;
      // cnt is the upper half of a 32-bit group word, below 2^16, and the
      // explicit bound keeps the loop finite whatever the word holds
      uint32_t excl = 0, tot = 0;
      for (int b = 0; b < 16 && __ballot((cnt >> b) != 0u); ++b) {
        const uint64_t bb = __ballot((cnt >> b) & 1u);
        excl += (uint32_t)__popcll(bb & lt_mask) << b;
        tot += (uint32_t)__popcll(bb) << b;
      }
      const uint64_t ba = __ballot(cnt != 0u);
      if (cnt) {
        const uint32_t vs = (uint32_t)T + excl;
        agl[G + __popcll(ba & lt_mask)] = (gd & 0x7fffu) | (vs << 15) | (trv ? 0u : 0x80000000u);
        atomicOr((uint32_t *)sbm + (vs >> 5), 1u << (vs & 31u));
      }
      T += (int)tot;
      G += __popcll(ba);
    }
    // edge pass over the active groups: sign test from LDS; the edges to
    // emit (owner) or to dedup (no owner) are staged by index, and their keys
    // are formed and written 64 at a time, so the sparse hits do not
    // serialize the wave
    int sne = 0;
    auto flush_edges = [&]() {
      wave_lds_sync();
      for (int b = 0; b < sne; b += 64) {
        const int idx = b + lane;
        bool dir = false, nw = false;
        uint64_t key = 0;
        if (idx < sne) {
          const uint32_t item = est[idx];
          const uint32_t te = ledge[item & 0x7fffffffu];
          int32_t y[D];
          template_point_inv<D>(v, winv, k, lpts[te & 0xfffu], y);
          const uint32_t Rl = te >> 24;
          uint32_t Rg = 0;
#pragma unroll
          for (int c = 0; c < D; ++c) Rg |= ((Rl >> winv[c]) & 1u) << c;
          key = ekey<D>(Lf, y, Rg);
          if (item >> 31) {
            uint64_t slot;
            const int ins = ht_insert(so.et_keys, so.et_mask, key, &slot);
            if (ins == 1)
              nw = true;
            else if (ins < 0)
              atomicOr(&ctr->et_fail, 1u);
          } else {
            dir = true;
          }
        }
        stage_put<kSubStage>(stage_s, sn, nw, key, put_s, &ctr->n_out);
        stage_put<kSubStage>(stage_d, snd, dir, key, put_d, &ctr->n_direct);
      }
      wave_lds_sync();
      sne = 0;
    };
    wave_lds_sync();
    int carry = 0;  // group starts before t0
    for (int t0 = 0; t0 < T; t0 += 64) {
      const int t = t0 + lane;
      const uint64_t wd = sbm[t0 >> 6];
      const int gi = carry + __popcll(wd & ((2ull << lane) - 1ull)) - 1;
      carry += __popcll(wd);
      bool take = false;
      uint32_t item = 0;
      if (t < T) {
        const uint32_t ent = agl[gi];
        const uint32_t e = (ent & 0x7fffu) + (uint32_t)t - ((ent >> 15) & 0x7fffu);
        const uint32_t te = ledge[e];
        const uint32_t ca = code[te & 0xfffu], cb = code[(te >> 12) & 0xfffu];
        if ((ca ^ cb) == 1u && (ca | cb) == 1u) {
          ++hits;
          take = true;
          item = e | (ent & 0x80000000u);
          if (ent >> 31) ++shits;
        }
      }
      const uint64_t bal = __ballot(take);
      if (bal) {
        const int nb = __popcll(bal);
        if (sne + nb > kEdgeStage) flush_edges();
        if (take) est[sne + __popcll(bal & lt_mask)] = item;
        sne += nb;
      }
    }
    flush_edges();
  }
  if (MODE != 1) {
    stage_flush(stage_s, sn, put_s, &ctr->n_out);
    stage_flush(stage_d, snd, put_d, &ctr->n_direct);
  }
  if (hits) atomicAdd(&ctr->n_cof, (unsigned long long)hits);
  if (shits) atomicAdd(&ctr->n_shared, (unsigned long long)shits);
  if (n64) atomicAdd(&ctr->n_cert64, (unsigned long long)n64);
  if (npts) atomicAdd(&ctr->n_pts, (unsigned long long)npts);
  if (nuns) atomicAdd(&ctr->n_unsettled, (unsigned long long)nuns);
}

__global__ void set_counter_kernel(unsigned long long *p, unsigned long long v) { *p = v; }

// Ends of the listed edges as raw vertices: vraw[2r] = a, vraw[2r + 1] = b.
template <int D>
__global__ void redo_ends_kernel(LatDev L, const uint64_t *keys, const uint64_t *redo, uint64_t n, int32_t *vraw) {
  for (uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (uint64_t)gridDim.x * blockDim.x) {
    int32_t a[D];
    uint32_t R;
    eunpack<D>(L, keys[redo[r]], a, &R);
#pragma unroll
    for (int j = 0; j < D; ++j) {
      vraw[(2 * r) * D + j] = a[j];
      vraw[(2 * r + 1) * D + j] = a[j] + (int32_t)((R >> j) & 1u);
    }
  }
}

// Intersection points of the fused path: f at both ends from the FP64
// monomial basis with its bound (edge_point); an edge whose point the bound
// cannot place within tolerance is listed in redo for the canonical FP64
// evaluation of its ends.
template <int D>
__global__ void sub_points_kernel(LatDev L, const uint64_t *keys, uint64_t lo, uint64_t hi, double *pts, int64_t ld,
                                  PolyDev Q, uint64_t *redo, Counters *ctr) {
  // the FP64 monomial coefficients, read by every lane at the same index,
  // from LDS (from global memory each read would be a vector load)
  extern __shared__ __align__(16) unsigned char smem[];
  double *lcd = (double *)smem;
  for (int m = threadIdx.x; m < Q.M; m += blockDim.x) lcd[m] = Q.cd[m];
  __syncthreads();
  Q.cd = lcd;
  for (uint64_t i = lo + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < hi; i += (uint64_t)gridDim.x * blockDim.x) {
    int32_t a[D], b[D];
    uint32_t R;
    eunpack<D>(L, keys[i], a, &R);
#pragma unroll
    for (int j = 0; j < D; ++j) b[j] = a[j] + (int32_t)((R >> j) & 1u);
    double p[D];
    const bool ok = edge_point<D>(L, Q, a, b, 0.0, 0.0, true, 0.0f, 0.0f, p);
#pragma unroll
    for (int j = 0; j < D; ++j) pts[(int64_t)j * ld + (int64_t)i] = p[j];
    if (!ok) redo[atomicAdd(&ctr->n_aux, 1ull)] = i;
  }
}

// The listed edges' points from the canonical FP64 values f[2r], f[2r + 1].
template <int D>
__global__ void sub_redo_kernel(LatDev L, const uint64_t *keys, const uint64_t *redo, uint64_t n, const double *f,
                                double *pts, int64_t ld, PolyDev Q) {
  for (uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t i = redo[r];
    int32_t a[D], b[D];
    uint32_t R;
    eunpack<D>(L, keys[i], a, &R);
#pragma unroll
    for (int j = 0; j < D; ++j) b[j] = a[j] + (int32_t)((R >> j) & 1u);
    double p[D];
    edge_point<D>(L, Q, a, b, f[2 * r], f[2 * r + 1], false, -1.0f, -1.0f, p);
#pragma unroll
    for (int j = 0; j < D; ++j) pts[(int64_t)j * ld + (int64_t)i] = p[j];
  }
}

// Local subdivision template (Sec. V-B, Eq. 2 read with >=): points u with
// k >= u_0 >= ... >= u_{d-1} >= 0 and edges (u, R) whose other end u + 1_R
// is inside too.  Points packed 8 bits per coordinate; edges packed as
// (index a | index b << 12 | R << 24).  The face of an edge is the set of
// coarse-simplex vertices whose barycentric weight is positive at either end
// (Eq. 1: vertex 0 weighs k - u_0, vertex i in 1..d-1 weighs u_{i-1} - u_i,
// vertex d weighs u_{d-1}), i.e. the smallest face holding the edge.  Edges
// are grouped by face: grp[V] = first edge of face V | edge count << 16,
// pf[p * NVW + t] holds bit V - 64 t for every face V of an edge at point p,
// and pv[V * NPW + t] bit p - 64 t for every end p of an edge of face V.
struct Template {
  std::vector<uint64_t> pts;
  std::vector<uint32_t> edges;
  std::vector<uint32_t> grp;
  std::vector<uint64_t> pf;
  std::vector<uint64_t> pv;
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
  auto support = [&](const std::vector<int> &x) {
    uint32_t m = 0;
    if (x[0] < k) m |= 1u;
    for (int i = 1; i < d; ++i)
      if (x[i - 1] > x[i]) m |= 1u << i;
    if (x[d - 1] > 0) m |= 1u << d;
    return m;
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
  const int NV = 1 << (d + 1), NVW = (NV + 63) / 64;
  std::vector<std::vector<uint32_t>> by_face(NV);
  for (size_t a = 0; a < P.size(); ++a)
    for (uint32_t R = 1; R < (1u << d); ++R) {
      std::vector<int> y = P[a];
      for (int i = 0; i < d; ++i) y[i] += (int)((R >> i) & 1u);
      if (!inside(y)) continue;
      const int b = index_of(y);
      by_face[support(P[a]) | support(y)].push_back((uint32_t)a | ((uint32_t)b << 12) | (R << 24));
    }
  const size_t NPW = (P.size() + 63) / 64;
  T.grp.assign(NV, 0u);
  T.pf.assign(P.size() * NVW, 0ull);
  T.pv.assign((size_t)NV * NPW, 0ull);
  for (int V = 0; V < NV; ++V) {
    T.grp[V] = (uint32_t)T.edges.size() | ((uint32_t)by_face[V].size() << 16);
    for (uint32_t te : by_face[V]) {
      T.edges.push_back(te);
      for (uint32_t q : {te & 0xfffu, (te >> 12) & 0xfffu}) {
        T.pf[q * NVW + V / 64] |= 1ull << (V % 64);
        T.pv[(size_t)V * NPW + q / 64] |= 1ull << (q % 64);
      }
    }
  }
  return T;
}

int lehmer_bits(int d) {
  int f = ifact(d), b = 0;
  while ((1 << b) < f) ++b;
  return b < 1 ? 1 : b;
}

// Grows the SoA point buffer (columns of length ld) to hold hi rows, keeping
// the first lo rows: to at least twice its size while batches append, to
// exactly hi rows for the final size (exact).
template <int D>
int grow_points(ip_ctx *ctx, uint64_t lo, uint64_t hi, double *&pts, uint64_t &ld, bool exact = false) {
  if (hi <= ld) return IP_OK;
  const uint64_t nld = exact ? hi : std::max<uint64_t>(hi, ld * 2);
  double *np_ = nullptr;
  IP_TRY(alloc(ctx, (void **)&np_, nld * D * 8));
  if (pts && lo) {
    for (int j = 0; j < D; ++j)
      IP_TRY_HIP(ctx, hipMemcpyAsync(np_ + (uint64_t)j * nld, pts + (uint64_t)j * ld, lo * 8, hipMemcpyDeviceToDevice,
                                     ctx->stream));
  }
  IP_TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));
  if (pts) release(ctx, pts);
  pts = np_;
  ld = nld;
  return IP_OK;
}

// Batch-mode output.  Owner-emitted keys (dkeys, capacity dcap) and the
// global edge set for edges without an owner (et, open addressing, load
// kept <= 1/2) with its keys in insertion order (skeys, capacity et_cap:
// every key in the set was appended once).  FP64 mode keeps the points of
// both lists too (dpts, spts, SoA with column strides dld, sld).
struct BatchSink {
  ip_ctx *ctx = nullptr;
  uint64_t *et = nullptr, *skeys = nullptr, *dkeys = nullptr;
  uint64_t et_cap = 0, dcap = 0;
  double *dpts = nullptr, *spts = nullptr;
  uint64_t dld = 0, sld = 0;
  explicit BatchSink(ip_ctx *c) : ctx(c) {}
  ~BatchSink() {
    for (void *p : {(void *)et, (void *)skeys, (void *)dkeys, (void *)dpts, (void *)spts})
      if (p) ip_dfree(ctx, p);
  }
  // Grow the set to cap (power of two), rebuilt from its first n keys.
  int reserve_set(uint64_t cap, uint64_t n) {
    void *ne = nullptr, *nk = nullptr;
    IP_TRY(alloc(ctx, &ne, cap * 8));
    IP_TRY(alloc(ctx, &nk, cap * 8));
    IP_TRY(fill(ctx, ne, cap, IP_EMPTY_KEY));
    if (n) {
      IP_TRY_HIP(ctx, hipMemcpyAsync(nk, skeys, n * 8, hipMemcpyDeviceToDevice, ctx->stream));
      hipLaunchKernelGGL(et_rebuild_keys_kernel, dim3(grid_for(n)), dim3(kBlock), 0, ctx->stream, (const uint64_t *)nk,
                         n, (uint64_t *)ne, cap - 1, ctx->ctr_dev);
      IP_TRY_HIP(ctx, hipGetLastError());
    }
    IP_TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (et) ip_dfree(ctx, et);
    if (skeys) ip_dfree(ctx, skeys);
    et = (uint64_t *)ne;
    skeys = (uint64_t *)nk;
    et_cap = cap;
    return IP_OK;
  }
  // Grow the owner-emitted list to cap entries, keeping the first n.
  int reserve_direct(uint64_t cap, uint64_t n) {
    void *nk = nullptr;
    IP_TRY(alloc(ctx, &nk, cap * 8));
    if (n) IP_TRY_HIP(ctx, hipMemcpyAsync(nk, dkeys, n * 8, hipMemcpyDeviceToDevice, ctx->stream));
    IP_TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (dkeys) ip_dfree(ctx, dkeys);
    dkeys = (uint64_t *)nk;
    dcap = cap;
    return IP_OK;
  }
  SubOut sub_out(const VEnt *cvt, uint64_t cvt_mask) const {
    return SubOut{cvt, cvt_mask, et, et_cap - 1, skeys, dkeys, dcap};
  }
  // Final output: the set keys (and FP64 points) appended after the owner
  // keys; hands the key list over.
  template <int D>
  int assemble(uint64_t n_dir, uint64_t n_set, bool with_pts) {
    const uint64_t n = n_dir + n_set;
    if (n > dcap || !dkeys) IP_TRY(reserve_direct(std::max<uint64_t>(n, 1), n_dir));
    if (n_set) IP_TRY_HIP(ctx, hipMemcpyAsync(dkeys + n_dir, skeys, n_set * 8, hipMemcpyDeviceToDevice, ctx->stream));
    if (with_pts) {
      IP_TRY(grow_points<D>(ctx, n_dir, std::max<uint64_t>(n, 1), dpts, dld, true));
      if (n_set)
        for (int j = 0; j < D; ++j)
          IP_TRY_HIP(ctx, hipMemcpyAsync(dpts + (uint64_t)j * dld + n_dir, spts + (uint64_t)j * sld, n_set * 8,
                                         hipMemcpyDeviceToDevice, ctx->stream));
    }
    IP_TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return IP_OK;
  }
};

int set_counter(ip_ctx *ctx, unsigned long long *field, unsigned long long v) {
  hipLaunchKernelGGL(set_counter_kernel, dim3(1), dim3(1), 0, ctx->stream, field, v);
  IP_TRY_HIP(ctx, hipGetLastError());
  return IP_OK;
}

// Runs `launch` (one subdivision launch) until it neither found the edge set
// full nor overran the owner list.  Before the first launch the set is grown
// to keep its load at most 1/2.  After a set overflow the set is grown from
// its key list (which includes the partial appends of the failed launch) and
// the launch replayed: set edges already present are skipped.  The owner
// list is rewound to where the launch started and rewritten by the replay,
// after growing it to the count the launch reported.
template <typename F>
int run_with_replay(ip_ctx *ctx, BatchSink &g, int64_t &regrows, F launch) {
  Counters *c = ctx->ctr_host;
  IP_TRY(read_ctr(ctx));
  const uint64_t dir_lo = c->n_direct;
  uint64_t n_keys = c->n_out;
  bool set_failed = false;
  for (int guard = 0;; ++guard) {
    if (guard > 40) return ip_fail(ctx, IP_ENOMEM, "edge tables cannot grow");
    if (n_keys * 2 > g.et_cap || set_failed) {
      IP_TRY(zero_fail_flags(ctx));
      IP_TRY(g.reserve_set(pow2_at_least(std::max<uint64_t>(n_keys * 4, g.et_cap * 2)), n_keys));
      ++regrows;
    }
    IP_TRY(set_counter(ctx, &ctx->ctr_dev->n_direct, dir_lo));
    IP_TRY(launch());
    IP_TRY(read_ctr(ctx));
    const bool dir_over = c->n_direct > g.dcap;
    if (!c->et_fail && !dir_over) return IP_OK;
    set_failed = c->et_fail != 0;
    n_keys = c->n_out;
    if (dir_over) {
      IP_TRY(g.reserve_direct(c->n_direct + c->n_direct / 4 + 1024, dir_lo));
      ++regrows;
    }
  }
}

constexpr size_t kSubLdsMax = 64 * 1024;
constexpr uint64_t kSubGrid = 4096;

struct SubArgs {
  int LB;
  const uint64_t *tpts;
  int NP;
  const uint32_t *tedge;
  int NE;
  const uint32_t *tgrp;
  const uint64_t *tpf;
  const uint64_t *tpv;
  const VEnt *cvt;
  uint64_t cvt_mask;
};

// The preparation of coarse simplices sig[0 .. n) (B1 only with `bound`).
template <int D>
int launch_prep(ip_ctx *ctx, const ip_problem *p, const SubArgs &a, const uint64_t *sig, uint64_t n, bool bound,
                SubPrep<D> *prep) {
  if (n == 0) return IP_OK;
  if (bound)
    hipLaunchKernelGGL((sub_prep_kernel<D, true>), dim3(grid_for(n)), dim3(kBlock), 0, ctx->stream, p->fine, p->coarse,
                       a.LB, p->k, sig, n, a.cvt, a.cvt_mask, p->poly, prep);
  else
    hipLaunchKernelGGL((sub_prep_kernel<D, false>), dim3(grid_for(n)), dim3(kBlock), 0, ctx->stream, p->fine,
                       p->coarse, a.LB, p->k, sig, n, a.cvt, a.cvt_mask, p->poly, prep);
  IP_TRY_HIP(ctx, hipGetLastError());
  return IP_OK;
}

template <int D, int MODE>
int launch_sub(ip_ctx *ctx, const ip_problem *p, const SubArgs &a, const uint64_t *sig, const uint32_t *list,
               uint64_t n, VEnt *fvt, uint64_t fvt_mask, uint32_t *eval, const BatchSink &g, uint32_t *defer,
               const SubPrep<D> *prep, const uint32_t *pslot = nullptr) {
  if (n == 0) return IP_OK;
  const size_t lds = sub_layout(a.NP, a.NE, MODE == 3 ? 0 : p->poly.M, 1 << (D + 1)).total;
  const uint64_t blocks = std::min<uint64_t>((n + kWaves - 1) / kWaves, kSubGrid);
  const SubOut so = g.sub_out(a.cvt, a.cvt_mask);
#define IP_SUB(PP)                                                                                                  \
  hipLaunchKernelGGL((subdivide_kernel<D, PP, MODE>), dim3((unsigned)blocks), dim3(kBlock), lds, ctx->stream,     \
                     p->fine, p->coarse, a.LB, p->k, sig, list, n, a.tpts, a.NP, a.tedge, a.NE, a.tgrp, a.tpf, a.tpv,    \
                     p->poly,                                                                                      \
                     fvt, fvt_mask, eval, pslot, prep, so, defer, ctx->ctr_dev)
  if (MODE == 3) {
    IP_SUB(1);
    IP_TRY_HIP(ctx, hipGetLastError());
    return IP_OK;
  }
  switch (p->poly.p) {
    case 1: IP_SUB(1); break;
    case 2: IP_SUB(2); break;
    case 3: IP_SUB(3); break;
    case 4: IP_SUB(4); break;
    default: return ip_fail(ctx, IP_EINVAL, "fused subdivision needs a polynomial of degree <= 4");
  }
#undef IP_SUB
  IP_TRY_HIP(ctx, hipGetLastError());
  return IP_OK;
}

// Device buffer released when the holder goes out of scope.
struct DevTmp {
  ip_ctx *ctx;
  void *p = nullptr;
  explicit DevTmp(ip_ctx *c) : ctx(c) {}
  ~DevTmp() {
    if (p) ip_dfree(ctx, p);
  }
  DevTmp(const DevTmp &) = delete;
  DevTmp &operator=(const DevTmp &) = delete;
  int get(size_t bytes) { return alloc(ctx, &p, bytes); }
  template <typename T>
  T *as() const {
    return (T *)p;
  }
};

// Points of the fused path for the output keys [lo, hi): FP64 monomial
// values with the certified placement check, then the canonical FP64 values
// at both ends of every edge the check rejects.
template <int D>
int redo_points(ip_ctx *ctx, const ip_problem *p, const uint64_t *keys, const uint64_t *redo, uint64_t nredo,
                double *pts, uint64_t ld, int64_t &n_fallback);

template <int D>
int sub_points(ip_ctx *ctx, const ip_problem *p, const uint64_t *keys, uint64_t lo, uint64_t hi, double *pts,
               uint64_t ld, Timer &tp, ip_stats &st, int64_t &n_fallback) {
  if (hi <= lo) return IP_OK;
  IP_TRY(ip_ensure(ctx, ctx->scratch, (hi - lo) * 8));
  uint64_t *redo = (uint64_t *)ctx->scratch.p;
  IP_TRY(zero_field(ctx, &ctx->ctr_dev->n_aux));
  IP_TRY(tp.start(ctx, &st.ms_points));
  hipLaunchKernelGGL((sub_points_kernel<D>), dim3(grid_for(hi - lo)), dim3(kBlock), (size_t)p->poly.M * 8, ctx->stream,
                     p->fine, keys, lo,
                     hi, pts, (int64_t)ld, p->poly, redo, ctx->ctr_dev);
  IP_TRY_HIP(ctx, hipGetLastError());
  IP_TRY(tp.stop(ctx));
  IP_TRY(read_ctr(ctx));
  return redo_points<D>(ctx, p, keys, redo, ctx->ctr_host->n_aux, pts, ld, n_fallback);
}

// The points of the edges listed in redo (indices into keys), from canonical
// FP64 values at both ends.
template <int D>
int redo_points(ip_ctx *ctx, const ip_problem *p, const uint64_t *keys, const uint64_t *redo, uint64_t nredo,
                double *pts, uint64_t ld, int64_t &n_fallback) {
  if (nredo == 0) return IP_OK;
  DevTmp vraw(ctx), fr(ctx);
  IP_TRY(vraw.get(nredo * 2 * D * 4));
  IP_TRY(fr.get(nredo * 2 * 8));
  hipLaunchKernelGGL((redo_ends_kernel<D>), dim3(grid_for(nredo)), dim3(kBlock), 0, ctx->stream, p->fine, keys,
                     (const uint64_t *)redo, nredo, vraw.as<int32_t>());
  IP_TRY_HIP(ctx, hipGetLastError());
  IP_TRY(launch_feval64_raw(ctx, p, p->fine, vraw.as<int32_t>(), 2 * nredo, fr.as<double>()));
  hipLaunchKernelGGL((sub_redo_kernel<D>), dim3(grid_for(nredo)), dim3(kBlock), 0, ctx->stream, p->fine, keys,
                     (const uint64_t *)redo, nredo, (const double *)fr.as<double>(), pts, (int64_t)ld, p->poly);
  IP_TRY_HIP(ctx, hipGetLastError());
  IP_TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));
  n_fallback += (int64_t)(2 * nredo);
  return IP_OK;
}

template <int D>
int refine_T(ip_ctx *ctx, const ip_problem *p, int32_t prec, int iters, ip_cells *c);

// Per-batch hand-off of the batch stage (ip_trace_check_batches): each
// batch's cells get their points (by the caller), then are refined, checked
// and their C_free points interleaved into one of two device staging slots;
// a copy stream moves the slot to page-locked host memory while the compute
// stream goes on with the next batch, and the batch's callback runs once its
// copy has landed (when its slot is needed again, or at the end), in batch
// order.  The batch's other buffers are reused by the next batch.
struct BatchStream {
  ip_ctx *ctx = nullptr;
  const ip_scene *scene = nullptr;
  ip_batch_fn fn = nullptr;
  void *user = nullptr;
  int32_t prec = IP_FP64;
  int iters = 0;
  unsigned long long *dg = nullptr;  // device: digest sum and xor
  uint8_t *verdict = nullptr;        // device, vcap bytes
  uint64_t vcap = 0;
  double *pts = nullptr;             // device batch points, SoA d x ld
  uint64_t ld = 0;
  hipStream_t copy = nullptr;        // device-to-host copies of the slots
  struct Slot {
    hipEvent_t ready = nullptr, copied = nullptr;
    bool pending = false;            // a copy in flight or a callback due
    int64_t batch = 0, n_free = 0, n_cells = 0;
  } slot[2];
  size_t half = 0;                   // bytes per slot in ctx->host_stage
  int64_t n_cells = 0, n_free = 0, batches = 0;
  double ms_check = 0.0, ms_refine = 0.0;
  explicit BatchStream(ip_ctx *c) : ctx(c) {}
  ~BatchStream() {
    if (ctx) (void)hipStreamSynchronize(ctx->stream);
    if (copy) (void)hipStreamSynchronize(copy);
    for (Slot &q : slot) {
      if (q.ready) (void)hipEventDestroy(q.ready);
      if (q.copied) (void)hipEventDestroy(q.copied);
    }
    if (copy) (void)hipStreamDestroy(copy);
    for (void *q : {(void *)dg, (void *)verdict, (void *)pts})
      if (q) ip_dfree(ctx, q);
  }
  BatchStream(const BatchStream &) = delete;
  BatchStream &operator=(const BatchStream &) = delete;
  int init() {
    IP_TRY(alloc(ctx, (void **)&dg, 16));
    IP_TRY(fill(ctx, dg, 2, 0ull));
    IP_TRY_HIP(ctx, hipStreamCreateWithFlags(&copy, hipStreamNonBlocking));
    for (Slot &q : slot) {
      IP_TRY_HIP(ctx, hipEventCreateWithFlags(&q.ready, hipEventDisableTiming));
      IP_TRY_HIP(ctx, hipEventCreateWithFlags(&q.copied, hipEventDisableTiming));
    }
    return IP_OK;
  }
  double *host_of(int i) const { return (double *)((unsigned char *)ctx->host_stage + (size_t)i * half); }
  // Waits for slot i's copy and runs its callback.
  int drain(int i) {
    Slot &q = slot[i];
    if (!q.pending) return IP_OK;
    q.pending = false;
    IP_TRY_HIP(ctx, hipEventSynchronize(q.copied));
    if (fn && fn(user, q.batch, host_of(i), q.n_free, q.n_cells) != 0)
      return ip_fail(ctx, IP_ECANCELED, "stopped by the batch callback");
    return IP_OK;
  }
  // Both slots, older batch first.
  int drain_all() {
    const int first = (slot[0].pending && slot[1].pending && slot[1].batch < slot[0].batch) ? 1 : 0;
    IP_TRY(drain(first));
    return drain(1 - first);
  }
};

// Projected output bytes of one coarse simplex in the per-batch mode: its
// share of the fine cells (1.6 nc k^(d-1) / |Sigma|) times key, points,
// verdict, free-point copy and staging (9 + 24 d bytes per cell).
template <int D>
uint64_t stream_bytes_per_sigma(uint64_t nc, uint64_t nsig, int k) {
  double est = 1.6 * (double)nc;
  for (int q = 0; q < D - 1; ++q) est *= k;
  const double per = est / (double)(nsig ? nsig : 1);
  return (uint64_t)std::ceil(per * (9.0 + 24.0 * D)) + 1;
}

// Batch number bs.batches, checked in `view`: its free points interleaved
// into a staging slot on the compute stream, then copied to the host on the
// copy stream.  The slot's previous batch is handed over first; the host
// staging (two slots, in the context, kept across calls) grows only when
// neither slot has a copy in flight.
constexpr size_t kCopyChunk = 1ull << 30;

template <int D>
int stream_handoff(BatchStream &bs, const ip_cells &view, int64_t n_cells) {
  ip_ctx *ctx = bs.ctx;
  const int64_t b = bs.batches;
  const int i = (int)(b & 1);
  BatchStream::Slot &q = bs.slot[i];
  IP_TRY(bs.drain(i));
  const size_t need = (size_t)view.n_free * D * sizeof(double);
  if (need > bs.half || 2 * bs.half > ctx->host_stage_bytes) {
    IP_TRY(bs.drain_all());
    const size_t want = std::max<size_t>(need + need / 4 + (1u << 20), ctx->host_stage_bytes / 2);
    if (2 * want > ctx->host_stage_bytes) {
      if (ctx->host_stage) (void)hipHostFree(ctx->host_stage);
      ctx->host_stage = nullptr;
      ctx->host_stage_bytes = 0;
      IP_TRY_HIP(ctx, hipHostMalloc(&ctx->host_stage, 2 * want, hipHostMallocDefault));
      ctx->host_stage_bytes = 2 * want;
    }
    bs.half = ctx->host_stage_bytes / 2;
  }
  if (need > ctx->dev_stage_bytes[i]) {
    // the slot is drained: its previous copy has landed
    if (ctx->dev_stage[i]) IP_TRY_HIP(ctx, hipFree(ctx->dev_stage[i]));
    ctx->dev_stage[i] = nullptr;
    ctx->dev_stage_bytes[i] = 0;
    const size_t want = need + need / 4 + (2u << 20);
    IP_TRY_HIP(ctx, hipMalloc(&ctx->dev_stage[i], want));
    ctx->dev_stage_bytes[i] = want;
  }
  double *dev = (double *)ctx->dev_stage[i];
  IP_TRY(ip_interleave_free(ctx, &view, dev));
  IP_TRY_HIP(ctx, hipEventRecord(q.ready, ctx->stream));
  IP_TRY_HIP(ctx, hipStreamWaitEvent(bs.copy, q.ready, 0));
  // copies of at most 1 GiB each (single copies of several GiB ran well
  // below the link's rate)
  for (size_t off = 0; off < need; off += kCopyChunk) {
    const size_t len = std::min<size_t>(kCopyChunk, need - off);
    IP_TRY_HIP(ctx, hipMemcpyAsync((unsigned char *)bs.host_of(i) + off, (const unsigned char *)dev + off, len,
                                   hipMemcpyDeviceToHost, bs.copy));
  }
  IP_TRY_HIP(ctx, hipEventRecord(q.copied, bs.copy));
  q.pending = true;
  q.batch = b;
  q.n_free = view.n_free;
  q.n_cells = n_cells;
  bs.batches = b + 1;
  bs.n_cells += n_cells;
  bs.n_free += view.n_free;
  return IP_OK;
}

// The batch's cells are keys[0 .. n) with their points in bs.pts: refine,
// digest, check, C_free points to the host, callback.  The check kernels
// reset the whole counter block, so the trace's counters are saved around
// them.
template <int D>
int stream_consume(const ip_problem *p, BatchStream &bs, const uint64_t *keys, uint64_t n) {
  ip_ctx *ctx = bs.ctx;
  ip_cells view;
  view.ctx = ctx;
  view.d = D;
  view.B = p->fine.B;
  view.n = (int64_t)n;
  view.keys = const_cast<uint64_t *>(keys);
  view.pts = bs.pts;
  view.ld = (int64_t)bs.ld;
  if (n) {
    IP_TRY(refine_T<D>(ctx, p, bs.prec, bs.iters, &view));
    bs.ms_refine += view.st.ms_refine;
    IP_TRY(ip_digest_accumulate(ctx, keys, (int64_t)n, bs.dg));
  }
  if (n > bs.vcap) {
    if (bs.verdict) release(ctx, bs.verdict);
    bs.verdict = nullptr;
    bs.vcap = 0;
    IP_TRY(alloc(ctx, (void **)&bs.verdict, n + n / 4 + 1024));
    bs.vcap = n + n / 4 + 1024;
  }
  view.verdict = bs.verdict;
  IP_TRY(read_ctr(ctx));
  const Counters saved = *ctx->ctr_host;
  int rc = ip_check_gather_impl(ctx, bs.scene, &view);
  *ctx->ctr_host = saved;
  hipError_t e = hipMemcpyAsync(ctx->ctr_dev, ctx->ctr_host, sizeof(Counters), hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (rc == IP_OK && e != hipSuccess) rc = ip_hip(ctx, e, "counter restore");
  if (rc == IP_OK) rc = stream_handoff<D>(bs, view, (int64_t)n);
  if (view.free_pts) ip_dfree(ctx, view.free_pts);
  IP_TRY(rc);
  bs.ms_check += view.st.ms_check;
  return IP_OK;
}

// The batch's cell list in the owner list: its owner-emitted keys [0, n_dir)
// followed by the edge-set keys it added, skeys[set_lo, set_hi).
inline int stream_batch_keys(BatchSink &g, uint64_t n_dir, uint64_t set_lo, uint64_t set_hi, uint64_t *n_out) {
  const uint64_t n = n_dir + (set_hi - set_lo);
  if (n > g.dcap) IP_TRY(g.reserve_direct(n + n / 4 + 1024, n_dir));
  if (set_hi > set_lo)
    IP_TRY_HIP(g.ctx, hipMemcpyAsync(g.dkeys + n_dir, g.skeys + set_lo, (set_hi - set_lo) * 8, hipMemcpyDeviceToDevice,
                                     g.ctx->stream));
  *n_out = n;
  return IP_OK;
}

// Initial sizes of the batch outputs from the coarse edge count: fine edges
// are about coarse edges x k^(d-1) (the owner list gets 1.6 times that, the
// set for edges without an owner a quarter); both grow on demand.
// In the per-batch mode (frac = batch / |Sigma| < 1) both start at one
// batch's share.
template <int D>
int init_sink(BatchSink &g, uint64_t nc, int k, double frac = 1.0) {
  double est = (double)nc * std::min(1.0, frac);
  for (int q = 0; q < D - 1; ++q) est *= k;
  IP_TRY(g.reserve_direct((uint64_t)std::min(est * 1.6, 4.0e9) + 1024, 0));
  IP_TRY(g.reserve_set(pow2_at_least((uint64_t)std::min(est * 0.5, 4.0e9)), 0));
  return IP_OK;
}

// Subdivision of the coarse simplices sig[0 .. nsig) in the FP32-certified
// mode (subdivide_kernel MODE 0-2): no vertex table, so the per-batch
// workspace is one 4-byte deferred-list entry and one preparation record per
// coarse simplex, plus the fallback vertex table for the points no
// certified tier settles (sized from their count).
template <int D>
int subdivide_fused(ip_ctx *ctx, const ip_problem *p, const SubArgs &a, const uint64_t *sig_all, uint64_t nsig,
                    uint64_t nc, uint64_t budget, ip_stats &st, ip_cells *res, BatchStream *bs) {
  const int NP = a.NP, NE = a.NE;
  if (budget == 0) budget = 4ull << 30;
  const uint64_t per_sigma = 4 + sizeof(SubPrep<D>) + (bs ? stream_bytes_per_sigma<D>(nc, nsig, p->k) : 0);
  uint64_t B = std::min<uint64_t>(budget / per_sigma, 0xffffffffull);
  if (B == 0) return ip_fail(ctx, IP_ENOMEM, "batch budget below one coarse simplex");
  if (B > nsig) B = nsig ? nsig : 1;
  IP_TRY(ip_ensure(ctx, ctx->vt_aux, B * 4));
  uint32_t *defer = (uint32_t *)ctx->vt_aux.p;
  DevTmp prep_hold(ctx);
  IP_TRY(prep_hold.get(B * sizeof(SubPrep<D>)));
  SubPrep<D> *prep = prep_hold.as<SubPrep<D>>();
  BatchSink g(ctx);
  IP_TRY(init_sink<D>(g, nc, p->k, bs ? (double)B / (double)(nsig ? nsig : 1) : 1.0));
  Counters *c = ctx->ctr_host;
  IP_TRY_HIP(ctx, hipMemsetAsync(ctx->ctr_dev, 0, sizeof(Counters), ctx->stream));
  int64_t regrows = 0, n_fallback = 0, n_settled64 = 0, n_pts = 0, batches = 0;
  uint64_t set_done = 0;
  Timer tf, tx, tp, ts, tq;
  for (uint64_t b0 = 0; b0 < nsig; b0 += B) {
    const uint64_t nb = std::min<uint64_t>(B, nsig - b0);
    const uint64_t *sig = sig_all + b0;
    ++batches;
    IP_TRY(tq.start(ctx, &st.ms_prep));
    IP_TRY(launch_prep<D>(ctx, p, a, sig, nb, true, prep));
    IP_TRY(tq.stop(ctx));
    // per-batch mode: the owner list starts empty for every batch
    if (bs) IP_TRY(set_counter(ctx, &ctx->ctr_dev->n_direct, 0));
    IP_TRY(run_with_replay(ctx, g, regrows, [&]() -> int {
      IP_TRY(zero_field(ctx, &ctx->ctr_dev->n_aux));
      IP_TRY(zero_field(ctx, &ctx->ctr_dev->n_unsettled));
      IP_TRY(zero_field(ctx, &ctx->ctr_dev->n_pts));
      IP_TRY(zero_field(ctx, &ctx->ctr_dev->n_cert64));
      IP_TRY(zero_field(ctx, &ctx->ctr_dev->n_cof));
      IP_TRY(zero_field(ctx, &ctx->ctr_dev->n_shared));
      IP_TRY(ts.start(ctx, &st.ms_subdivide));
      IP_TRY((launch_sub<D, 0>(ctx, p, a, sig, nullptr, nb, nullptr, 0, nullptr, g, defer, prep)));
      ++st.subdivide_launches;
      return ts.stop(ctx);
    }));
    const uint64_t n_def = c->n_aux, n_uns = c->n_unsettled;
    n_pts += (int64_t)c->n_pts;
    n_settled64 += (int64_t)c->n_cert64;
    st.n_edge_hits += (int64_t)c->n_cof;
    st.n_shared_probes += (int64_t)c->n_shared;
    if (n_def) {
      // canonical FP64 for the points no certified tier settled
      const uint64_t fcap = pow2_at_least(2 * n_uns + 1024);
      DevTmp fvt_hold(ctx), eval_hold(ctx);
      IP_TRY(fvt_hold.get(fcap * sizeof(VEnt)));
      IP_TRY(eval_hold.get(fcap * 4));
      VEnt *fvt = fvt_hold.as<VEnt>();
      uint32_t *eval = eval_hold.as<uint32_t>();
      IP_TRY(fill_vt(ctx, fvt, fcap));
      IP_TRY(zero_field(ctx, &ctx->ctr_dev->n_eval));
      IP_TRY(zero_fail_flags(ctx));
      IP_TRY(tx.start(ctx, &st.ms_expand));
      IP_TRY((launch_sub<D, 1>(ctx, p, a, sig, defer, n_def, fvt, fcap - 1, eval, g, nullptr, prep)));
      IP_TRY(tx.stop(ctx));
      IP_TRY(read_ctr(ctx));
      if (c->vt_fail) return ip_fail(ctx, IP_ENOMEM, "fallback vertex table overflow");
      const uint64_t n_ev = c->n_eval;
      IP_TRY(tf.start(ctx, &st.ms_feval));
      IP_TRY(launch_feval64(ctx, p, p->fine, eval, n_ev, fvt));
      IP_TRY(tf.stop(ctx));
      n_fallback += (int64_t)n_ev;
      IP_TRY(run_with_replay(ctx, g, regrows, [&]() -> int {
        IP_TRY(zero_field(ctx, &ctx->ctr_dev->n_cof));
        IP_TRY(zero_field(ctx, &ctx->ctr_dev->n_shared));
        IP_TRY(ts.start(ctx, &st.ms_subdivide));
        IP_TRY((launch_sub<D, 2>(ctx, p, a, sig, defer, n_def, fvt, fcap - 1, nullptr, g, nullptr, prep)));
        ++st.subdivide_launches;
        return ts.stop(ctx);
      }));
      st.n_edge_hits += (int64_t)c->n_cof;
      st.n_shared_probes += (int64_t)c->n_shared;
      if (c->vt_fail) return ip_fail(ctx, IP_EDEVICE, "fallback vertex missing from its table");
    }
    st.n_template_edges += (int64_t)(nb * (uint64_t)NE);
    if (log_on())
      fprintf(stderr, "[ip] batch %lld: %llu coarse simplices, %llu deferred, %llu + %llu cells so far\n",
              (long long)batches, (unsigned long long)nb, (unsigned long long)n_def,
              (unsigned long long)c->n_direct, (unsigned long long)c->n_out);
    if (bs) {
      const uint64_t set_hi = c->n_out;
      uint64_t n_b = 0;
      IP_TRY(stream_batch_keys(g, c->n_direct, set_done, set_hi, &n_b));
      IP_TRY(grow_points<D>(ctx, 0, std::max<uint64_t>(n_b, 1), bs->pts, bs->ld));
      IP_TRY(sub_points<D>(ctx, p, g.dkeys, 0, n_b, bs->pts, bs->ld, tp, st, n_fallback));
      IP_TRY(stream_consume<D>(p, *bs, g.dkeys, n_b));
      set_done = set_hi;
    }
  }
  (void)NP;
  if (bs) {
    IP_TRY(bs->drain_all());
    IP_TRY(tf.flush(ctx));
    IP_TRY(tx.flush(ctx));
    IP_TRY(tp.flush(ctx));
    IP_TRY(ts.flush(ctx));
    IP_TRY(tq.flush(ctx));
    res->d = D;
    st.n_cells = bs->n_cells;
    st.n_batches = batches;
    st.n_vertices += n_pts;
    st.regrows += regrows;
    st.n_fallback += n_fallback;
    st.n_settled64 += n_settled64;
    return IP_OK;
  }
  const uint64_t n_dir = c->n_direct, n_set = c->n_out, n = n_dir + n_set;
  IP_TRY(g.assemble<D>(n_dir, n_set, false));
  double *pts = nullptr;
  uint64_t ld = 0;
  IP_TRY(grow_points<D>(ctx, 0, std::max<uint64_t>(n, 1), pts, ld));
  const int rc = sub_points<D>(ctx, p, g.dkeys, 0, n, pts, ld, tp, st, n_fallback);
  if (rc != IP_OK) {
    (void)hipStreamSynchronize(ctx->stream);
    release(ctx, pts);
    return rc;
  }
  IP_TRY(tf.flush(ctx));
  IP_TRY(tx.flush(ctx));
  IP_TRY(tp.flush(ctx));
  IP_TRY(ts.flush(ctx));
  IP_TRY(tq.flush(ctx));
  res->d = D;
  res->B = p->fine.B;
  for (int j = 0; j < 8; ++j) res->vmin[j] = p->fine.vmin[j];
  res->n = (int64_t)n;
  res->keys = g.dkeys;
  g.dkeys = nullptr;
  res->pts = pts;
  res->ld = (int64_t)ld;
  st.n_cells = (int64_t)n;
  st.n_batches = batches;
  st.n_vertices += n_pts;
  st.regrows += regrows;
  st.n_fallback += n_fallback;
  st.n_settled64 += n_settled64;
  return IP_OK;
}

// Subdivision of the coarse simplices sig[0 .. nsig) with canonical FP64
// values (FP64 mode): per batch the fine vertices of the template points go
// into a vertex table (each evaluated once), then subdivide_kernel (MODE 3)
// reads the signs through the per-simplex template slots.  Per-batch
// workspace: the vertex table (power-of-two capacity, load <= 1/2, so 2 NP
// slots per coarse simplex, each a 32-byte entry plus a 4-byte eval-list
// entry) and NP 4-byte template slots per coarse simplex; the largest table
// that fits the budget fixes the batch size.
template <int D>
int subdivide_table(ip_ctx *ctx, const ip_problem *p, const SubArgs &a, const uint64_t *sig_all, uint64_t nsig,
                    uint64_t nc, uint64_t budget, bool cert, ip_stats &st, ip_cells *res, BatchStream *bs) {
  const int k = p->k, NP = a.NP, NE = a.NE;
  // a slot: VEnt, eval-list entry and, certified, its bound and fallback
  // entry; per coarse simplex (one per 2 NP slots) its preparation record
  // and, in the per-batch mode, its projected output
  const uint64_t slot_bytes = sizeof(VEnt) + 4 + (cert ? 8 : 0);
  const uint64_t per_sigma = sizeof(SubPrep<D>) + (bs ? stream_bytes_per_sigma<D>(nc, nsig, k) : 0);
  if (budget == 0) budget = 4ull << 30;
  uint64_t vcap_b = 0;
  for (uint64_t cc = 1024; cc <= (1ull << 32); cc <<= 1)
    if (cc * slot_bytes + (cc / 2) * 4 + cc / (2 * (uint64_t)NP) * per_sigma <= budget && cc >= 2 * (uint64_t)NP)
      vcap_b = cc;
  if (vcap_b == 0) return ip_fail(ctx, IP_ENOMEM, "batch budget below one coarse simplex");
  uint64_t B = vcap_b / (2 * (uint64_t)NP);
  if (B > nsig) B = nsig ? nsig : 1;
  Run f;
  f.ctx = ctx;
  f.p = p;
  f.tb = &ctx->vtf;
  f.L = p->fine;
  const uint64_t vcap = std::min<uint64_t>(vcap_b, pow2_at_least(B * (uint64_t)NP * 2));
  IP_TRY(ip_ensure(ctx, ctx->vtf.keys, vcap * sizeof(VEnt)));
  IP_TRY(ip_ensure(ctx, ctx->vtf.eval, vcap * 4));
  IP_TRY(ip_ensure(ctx, ctx->vt_aux, B * (uint64_t)NP * 4));
  f.vt = (VEnt *)ctx->vtf.keys.p;
  f.eval = (uint32_t *)ctx->vtf.eval.p;
  f.vt_cap = vcap;
  f.cert = cert;
  if (cert) {
    IP_TRY(ip_ensure(ctx, ctx->vtf.vals, vcap * 4));
    IP_TRY(ip_ensure(ctx, ctx->vtf.fb, vcap * 4));
    f.vb = (float *)ctx->vtf.vals.p;
    f.fb = (uint32_t *)ctx->vtf.fb.p;
    f.fb_cap = ctx->vtf.fb.bytes / 4;
  }
  uint32_t *pslot = (uint32_t *)ctx->vt_aux.p;
  DevTmp prep_hold(ctx);
  IP_TRY(prep_hold.get(B * sizeof(SubPrep<D>)));
  SubPrep<D> *prep = prep_hold.as<SubPrep<D>>();
  BatchSink g(ctx);
  IP_TRY(init_sink<D>(g, nc, k, bs ? (double)B / (double)(nsig ? nsig : 1) : 1.0));
  Counters *c = ctx->ctr_host;
  IP_TRY_HIP(ctx, hipMemsetAsync(ctx->ctr_dev, 0, sizeof(Counters), ctx->stream));
  Timer tf, tx, tp, ts, tq;
  int64_t batches = 0;
  uint64_t dir_done = 0, set_done = 0;
  for (uint64_t b0 = 0; b0 < nsig; b0 += B) {
    const uint64_t nb = std::min<uint64_t>(B, nsig - b0);
    const uint64_t *sig = sig_all + b0;
    ++batches;
    IP_TRY(tq.start(ctx, &st.ms_prep));
    IP_TRY(launch_prep<D>(ctx, p, a, sig, nb, false, prep));
    IP_TRY(tq.stop(ctx));
    IP_TRY(fill_vt(ctx, f.vt, vcap));
    IP_TRY(zero_field(ctx, &ctx->ctr_dev->n_eval));
    IP_TRY(tx.start(ctx, &st.ms_expand));
    hipLaunchKernelGGL((batch_vertices_kernel<D>), dim3(grid_for(nb * NP)), dim3(kBlock), 0, ctx->stream, p->fine,
                       p->coarse, a.LB, k, sig, nb, a.tpts, NP, f.vt, vcap - 1, f.eval, pslot, ctx->ctr_dev);
    IP_TRY_HIP(ctx, hipGetLastError());
    IP_TRY(tx.stop(ctx));
    IP_TRY(read_ctr(ctx));
    if (c->vt_fail) return ip_fail(ctx, IP_ENOMEM, "batch vertex table overflow");
    const uint64_t n_ev = c->n_eval;
    IP_TRY(tf.start(ctx, &st.ms_feval));
    IP_TRY(eval_pending(f, n_ev));
    IP_TRY(tf.stop(ctx));
    st.n_vertices += (int64_t)n_ev;
    // per-batch mode: the owner list starts empty for every batch
    if (bs) IP_TRY(set_counter(ctx, &ctx->ctr_dev->n_direct, 0));
    IP_TRY(run_with_replay(ctx, g, f.regrows, [&]() -> int {
      IP_TRY(zero_field(ctx, &ctx->ctr_dev->n_cof));
      IP_TRY(zero_field(ctx, &ctx->ctr_dev->n_shared));
      IP_TRY(ts.start(ctx, &st.ms_subdivide));
      IP_TRY((launch_sub<D, 3>(ctx, p, a, sig, nullptr, nb, f.vt, vcap - 1, nullptr, g, nullptr, prep, pslot)));
      ++st.subdivide_launches;
      return ts.stop(ctx);
    }));
    st.n_edge_hits += (int64_t)c->n_cof;
    st.n_shared_probes += (int64_t)c->n_shared;
    st.n_template_edges += (int64_t)(nb * (uint64_t)NE);
    const uint64_t dir_hi = c->n_direct, set_hi = c->n_out;
    if (log_on())
      fprintf(stderr, "[ip] batch %lld: %llu coarse simplices, %llu new vertices, %llu + %llu cells so far\n",
              (long long)batches, (unsigned long long)nb, (unsigned long long)n_ev, (unsigned long long)dir_hi,
              (unsigned long long)set_hi);
    // points of this batch's new edges, from the batch vertex table (the
    // per-batch mode lists them in the owner list first)
    struct Part {
      const uint64_t *keys;
      uint64_t lo, hi;
      double *pts;
      uint64_t ld;
    };
    Part parts[2];
    int n_parts = 2;
    uint64_t n_b = 0;
    if (bs) {
      IP_TRY(stream_batch_keys(g, dir_hi, set_done, set_hi, &n_b));
      IP_TRY(grow_points<D>(ctx, 0, std::max<uint64_t>(n_b, 1), bs->pts, bs->ld));
      parts[0] = {g.dkeys, 0, n_b, bs->pts, bs->ld};
      n_parts = 1;
    } else {
      IP_TRY(grow_points<D>(ctx, dir_done, dir_hi, g.dpts, g.dld));
      IP_TRY(grow_points<D>(ctx, set_done, set_hi, g.spts, g.sld));
      parts[0] = {g.dkeys, dir_done, dir_hi, g.dpts, g.dld};
      parts[1] = {g.skeys, set_done, set_hi, g.spts, g.sld};
    }
    for (int pi = 0; pi < n_parts; ++pi) {
      const Part &q = parts[pi];
      if (q.hi <= q.lo) continue;
      uint64_t *redo = nullptr;
      if (cert) {
        IP_TRY(ip_ensure(ctx, ctx->scratch, (q.hi - q.lo) * 8));
        redo = (uint64_t *)ctx->scratch.p;
        IP_TRY(zero_field(ctx, &ctx->ctr_dev->n_aux));
      }
      IP_TRY(tp.start(ctx, &st.ms_points));
      if (cert)
        hipLaunchKernelGGL((batch_points_kernel<D, true>), dim3(grid_for(q.hi - q.lo)), dim3(kBlock), 0, ctx->stream,
                           p->fine, q.keys, q.lo, q.hi, (const VEnt *)f.vt, (const float *)f.vb, vcap - 1, q.pts,
                           (int64_t)q.ld, p->poly, redo, ctx->ctr_dev);
      else
        hipLaunchKernelGGL((batch_points_kernel<D, false>), dim3(grid_for(q.hi - q.lo)), dim3(kBlock), 0, ctx->stream,
                           p->fine, q.keys, q.lo, q.hi, (const VEnt *)f.vt, (const float *)nullptr, vcap - 1, q.pts,
                           (int64_t)q.ld, p->poly, (uint64_t *)nullptr, ctx->ctr_dev);
      IP_TRY_HIP(ctx, hipGetLastError());
      IP_TRY(tp.stop(ctx));
      if (cert) {
        IP_TRY(read_ctr(ctx));
        IP_TRY(redo_points<D>(ctx, p, q.keys, redo, ctx->ctr_host->n_aux, q.pts, q.ld, f.n_fallback));
      }
    }
    if (bs) {
      IP_TRY(stream_consume<D>(p, *bs, g.dkeys, n_b));
      dir_done = 0;
    } else {
      dir_done = dir_hi;
    }
    set_done = set_hi;
  }
  if (bs) {
    IP_TRY(bs->drain_all());
    IP_TRY(tf.flush(ctx));
    IP_TRY(tx.flush(ctx));
    IP_TRY(tp.flush(ctx));
    IP_TRY(ts.flush(ctx));
    IP_TRY(tq.flush(ctx));
    res->d = D;
    st.n_cells = bs->n_cells;
    st.n_batches = batches;
    st.regrows += f.regrows;
    st.n_fallback += f.n_fallback;
    st.n_settled64 += f.n_settled64;
    return IP_OK;
  }
  IP_TRY(g.assemble<D>(dir_done, set_done, true));
  IP_TRY(tf.flush(ctx));
  IP_TRY(tx.flush(ctx));
  IP_TRY(tp.flush(ctx));
  IP_TRY(ts.flush(ctx));
  IP_TRY(tq.flush(ctx));
  const uint64_t n = dir_done + set_done;
  res->d = D;
  res->B = p->fine.B;
  for (int j = 0; j < 8; ++j) res->vmin[j] = p->fine.vmin[j];
  res->n = (int64_t)n;
  res->keys = g.dkeys;
  g.dkeys = nullptr;
  res->pts = g.dpts;
  res->ld = (int64_t)g.dld;
  g.dpts = nullptr;
  st.n_cells = (int64_t)n;
  st.n_batches = batches;
  st.regrows += f.regrows;
  st.n_fallback += f.n_fallback;
  st.n_settled64 += f.n_settled64;
  return IP_OK;
}

template <int D>
int trace_batch(ip_ctx *ctx, const ip_problem *p, uint64_t budget, bool cert, ip_cells *res,
                BatchStream *bs = nullptr) {
  ip_stats &st = res->st;
  const int k = p->k;
  const int LB = lehmer_bits(D);
  if (D * p->coarse.B + LB > 63)
    return ip_fail(ctx, IP_ERANGE, "coarse simplex keys do not fit 63 bits for this domain and k");
  Template T = make_template(D, k);
  const int NP = (int)T.pts.size(), NE = (int)T.edges.size();
  if (sub_layout(NP, NE, p->poly.M, 1 << (D + 1)).total > kSubLdsMax || NE > 0x7fff)
    return ip_fail(ctx, IP_EINVAL, "subdivision template does not fit one workgroup's LDS (reduce k)");
  // ---- coarse trace (Sec. V-B: trace at scale k * lambda)
  Run s;
  s.ctx = ctx;
  s.p = p;
  s.tb = &ctx->vtc;
  s.L = p->coarse;
  s.cert = cert;
  IP_TRY(vt_init(s, 1ull << 16));
  uint64_t nc = 0;
  {
    int rc = trace_direct<D>(s, st, &nc);
    if (rc != IP_OK) {
      if (s.out) release(ctx, s.out);
      return rc;
    }
  }
  // the coarse vertex table (visited-edge masks = the coarse trace) stays in
  // ctx->vtc for the ownership test; the fine stage uses ctx->vtf
  const VEnt *cvt = s.vt;
  const uint64_t cvt_cap = s.vt_cap;
  OutRec *coarse_edges = s.out;
  s.out = nullptr;
  s.out_cap = 0;
  auto free_coarse = [&]() {
    if (coarse_edges) release(ctx, coarse_edges);
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
    st.n_ncofaces = (int64_t)bound;
    const uint64_t cap = pow2_at_least(bound * 2 + 2);
    int rc = alloc(ctx, &sig_tab, cap * 8);
    if (rc == IP_OK) rc = alloc(ctx, &sig_list, (bound + 1) * 8);
    if (rc != IP_OK) {
      free_coarse();
      if (sig_tab) release(ctx, sig_tab);
      return rc;
    }
    IP_TRY(fill(ctx, sig_tab, cap, IP_EMPTY_KEY));
    IP_TRY_HIP(ctx, hipMemsetAsync(ctx->ctr_dev, 0, sizeof(Counters), ctx->stream));
    Timer tsg;
    if (nc) {
      IP_TRY(tsg.start(ctx, &st.ms_sigma));
      hipLaunchKernelGGL((sigma_kernel<D>), dim3(grid_for(nc * 4, 8192)), dim3(kBlock), 0, ctx->stream, p->coarse, LB,
                         coarse_edges, nc, (uint64_t *)sig_tab, cap - 1, (uint64_t *)sig_list, ctx->ctr_dev);
      IP_TRY_HIP(ctx, hipGetLastError());
      IP_TRY(tsg.stop(ctx));
    }
    IP_TRY(read_ctr(ctx));
    IP_TRY(tsg.flush(ctx));
    nsig = ctx->ctr_host->n_aux;
    free_coarse();
    release(ctx, sig_tab);
    sig_tab = nullptr;
  }
  DevTmp sig_hold(ctx), tpts_hold(ctx), tedge_hold(ctx), tgrp_hold(ctx), tpf_hold(ctx), tpv_hold(ctx);
  sig_hold.p = sig_list;
  {
    // Morton order of the base vertices: neighbouring simplices run together
    Timer tso;
    IP_TRY(tso.start(ctx, &st.ms_sigma));
    IP_TRY(ip_sort_sigma(ctx, (uint64_t *)sig_list, nsig, D, p->coarse.B, LB));
    IP_TRY(tso.stop(ctx));
    IP_TRY(tso.flush(ctx));
  }
  st.n_sigma = (int64_t)nsig;
  st.n_coarse_edges = (int64_t)nc;
  if (log_on())
    fprintf(stderr, "[ip] coarse trace: %llu edges, %llu coarse n-simplices\n", (unsigned long long)nc,
            (unsigned long long)nsig);
  // ---- template on the device
  IP_TRY(tpts_hold.get(T.pts.size() * 8));
  IP_TRY(tedge_hold.get(T.edges.size() * 4));
  IP_TRY(tgrp_hold.get(T.grp.size() * 4));
  IP_TRY(tpf_hold.get(T.pf.size() * 8));
  IP_TRY(tpv_hold.get(T.pv.size() * 8));
  IP_TRY_HIP(ctx, hipMemcpyAsync(tpts_hold.p, T.pts.data(), T.pts.size() * 8, hipMemcpyHostToDevice, ctx->stream));
  IP_TRY_HIP(ctx,
             hipMemcpyAsync(tedge_hold.p, T.edges.data(), T.edges.size() * 4, hipMemcpyHostToDevice, ctx->stream));
  IP_TRY_HIP(ctx, hipMemcpyAsync(tgrp_hold.p, T.grp.data(), T.grp.size() * 4, hipMemcpyHostToDevice, ctx->stream));
  IP_TRY_HIP(ctx, hipMemcpyAsync(tpf_hold.p, T.pf.data(), T.pf.size() * 8, hipMemcpyHostToDevice, ctx->stream));
  IP_TRY_HIP(ctx, hipMemcpyAsync(tpv_hold.p, T.pv.data(), T.pv.size() * 8, hipMemcpyHostToDevice, ctx->stream));
  const SubArgs a{LB, tpts_hold.as<uint64_t>(), NP, tedge_hold.as<uint32_t>(), NE, tgrp_hold.as<uint32_t>(),
                  tpf_hold.as<uint64_t>(), tpv_hold.as<uint64_t>(), cvt, cvt_cap - 1};
  int rc;
  if (cert && p->poly.ok)
    rc = subdivide_fused<D>(ctx, p, a, (const uint64_t *)sig_list, nsig, nc, budget, st, res, bs);
  else
    rc = subdivide_table<D>(ctx, p, a, (const uint64_t *)sig_list, nsig, nc, budget, cert, st, res, bs);
  (void)hipStreamSynchronize(ctx->stream);
  st.regrows += s.regrows;
  st.n_fallback += s.n_fallback;
  st.n_settled64 += s.n_settled64;
  return rc;
}

// Points of OUT[0 .. n) into keys / pts; in FP32 mode the edges whose point
// the bound cannot certify get FP64 values at their ends and are redone.
template <int D>
int direct_points(Run &s, uint64_t n, uint64_t *keys, double *pts, ip_stats &st) {
  ip_ctx *ctx = s.ctx;
  uint64_t *redo = nullptr;
  DevTmp qb_hold(ctx);
  uint32_t *qb = nullptr;
  if (s.cert) {
    IP_TRY(ip_ensure(ctx, ctx->scratch, n * 8));
    IP_TRY(ip_ensure(ctx, s.tb->fb, (2 * n + 64) * 4));
    s.fb = (uint32_t *)s.tb->fb.p;
    redo = (uint64_t *)ctx->scratch.p;
    // queued-slot bitmap over the vertex table, cleared
    const uint64_t qwords = (s.vt_cap + 63) / 64;
    IP_TRY(qb_hold.get(qwords * 8));
    IP_TRY(fill(ctx, qb_hold.p, qwords, 0ull));
    qb = qb_hold.as<uint32_t>();
    IP_TRY(zero_field(ctx, &ctx->ctr_dev->n_aux));
    IP_TRY(zero_field(ctx, &ctx->ctr_dev->n_fb));
  }
  Timer tp;
  IP_TRY(tp.start(ctx, &st.ms_points));
  hipLaunchKernelGGL((points_kernel<D, false>), dim3(grid_for(n)), dim3(kBlock), 0, ctx->stream, s.L, s.out, n, s.vt,
                     keys, pts, (int64_t)n, s.cert, (const float *)s.vb, s.p->poly, redo, s.fb, qb, ctx->ctr_dev);
  IP_TRY_HIP(ctx, hipGetLastError());
  IP_TRY(tp.stop(ctx));
  if (s.cert) {
    IP_TRY(read_ctr(ctx));
    const uint64_t nredo = ctx->ctr_host->n_aux, nfb = ctx->ctr_host->n_fb;
    if (nredo) {
      IP_TRY(launch_feval64(ctx, s.p, s.L, s.fb, nfb, s.vt));
      IP_TRY(launch_set_vb(ctx, s.fb, nfb, s.vb, -1.0f));
      hipLaunchKernelGGL((points_kernel<D, true>), dim3(grid_for(nredo)), dim3(kBlock), 0, ctx->stream, s.L, s.out,
                         nredo, s.vt, keys, pts, (int64_t)n, true, (const float *)s.vb, s.p->poly, redo, s.fb,
                         qb, ctx->ctr_dev);
      IP_TRY_HIP(ctx, hipGetLastError());
      s.n_fallback += (int64_t)nfb;
    }
  }
  IP_TRY(tp.flush(ctx));
  return IP_OK;
}

template <int D>
int trace_T(ip_ctx *ctx, const ip_problem *p, uint64_t budget, int32_t prec, ip_cells *res) {
  // RBF manifolds trace in canonical FP64 in either mode: the FP32 tier's
  // bound, loose through the cancellation in the sum of exponentials, settles
  // signs but cannot place the intersection points, so every traced vertex
  // would need its FP64 value as well (ip_feval keeps the FP32 tier)
  const bool cert = prec == IP_FP32_CERTIFY && p->f.kernel == IP_KERNEL_POLY && ip_has_fp32_form(p);
  if (p->k != 1) return trace_batch<D>(ctx, p, budget, cert, res);
  Run s;
  s.ctx = ctx;
  s.p = p;
  s.tb = &ctx->vtf;
  s.L = p->fine;
  s.cert = cert;
  // start from the largest table the context already holds
  uint64_t vt0 = 1ull << 20;
  while (vt0 * 2 * sizeof(VEnt) <= ctx->vtf.keys.bytes) vt0 *= 2;
  IP_TRY(vt_init(s, vt0));
  ip_stats &st = res->st;
  uint64_t n = 0;
  int rc = trace_direct<D>(s, st, &n);
  uint64_t *keys = nullptr;
  double *pts = nullptr;
  if (rc == IP_OK) rc = alloc(ctx, (void **)&keys, sizeof(uint64_t) * (size_t)(n ? n : 1));
  if (rc == IP_OK) rc = alloc(ctx, (void **)&pts, sizeof(double) * (size_t)(n ? n : 1) * D);
  if (rc == IP_OK && n) rc = direct_points<D>(s, n, keys, pts, st);
  if (s.out) {
    (void)hipStreamSynchronize(ctx->stream);
    release(ctx, s.out);
  }
  if (rc != IP_OK) {
    if (keys) release(ctx, keys);
    if (pts) release(ctx, pts);
    return rc;
  }
  res->d = D;
  res->B = s.L.B;
  for (int j = 0; j < 8; ++j) res->vmin[j] = s.L.vmin[j];
  res->n = (int64_t)n;
  res->keys = keys;
  res->pts = pts;
  res->ld = (int64_t)n;
  st.n_cells = (int64_t)n;
  st.regrows += s.regrows;
  // FP32 requested but the degree has no FP32 form: every vertex was FP64
  st.n_fallback = s.cert ? s.n_fallback : (prec == IP_FP32_CERTIFY ? st.n_vertices : 0);
  st.n_settled64 = s.n_settled64;
  return IP_OK;
}

// The tier-1 evaluation of the fused subdivision on given coarse simplices
// (Sec. V-B, Eq. 1-2: the template points of each), for inspection: one wave
// per simplex forms the region bound B1 from the largest |x_j| over the
// simplex's vertices exactly as the subdivision kernel does, then every
// template point gets its fine vertex y, its nested FP32 value (NaN outside
// the box) and the simplex its bound B1 + B64.
template <int D, int P>
__global__ __launch_bounds__(256) void region_eval_kernel(LatDev Lf, int k, const int32_t *__restrict__ simp,
                                                          uint64_t n, const uint64_t *__restrict__ tpts, int NP,
                                                          PolyDev Q, int32_t *yout, double *fout, double *bout) {
  __shared__ double va[4][(D + 1) * D];
  __shared__ double Xs[4][8];
  const int wib = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint64_t wave = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const uint64_t n_waves = ((uint64_t)gridDim.x * blockDim.x) >> 6;
  for (uint64_t s = wave; s < n; s += n_waves) {
    int32_t v[D], w[D], winv[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
      v[j] = simp[s * 2 * D + j];
      w[j] = simp[s * 2 * D + D + j];
    }
    perm_inverse<D>(w, winv);
    const int vi = lane <= D ? lane : D;
    int32_t yv[D];
#pragma unroll
    for (int c = 0; c < D; ++c) yv[c] = k * v[c] + (winv[c] < vi ? k : 0);
    double xv[D];
    lat_coords<D>(Lf, yv, xv);
    if (lane <= D) {
#pragma unroll
      for (int j = 0; j < D; ++j) va[wib][lane * D + j] = fabs(xv[j]);
    }
    wave_lds_sync();
    if (lane < D) {
      double a = 0.0;
#pragma unroll
      for (int i = 0; i <= D; ++i) a = fmax(a, va[wib][i * D + lane]);
      Xs[wib][lane] = a * (1.0 + 1e-12) + 1e-300;
    }
    wave_lds_sync();
    const double B1 = Q.K32n * region_sabs_bound(Q, Xs[wib], lane) + Q.E0;
    if (lane == 0) bout[s] = B1 + Q.B64;
    for (int pt = lane; pt < NP; pt += 64) {
      int32_t y[D];
      template_point_inv<D>(v, winv, k, tpts[pt], y);
      double x[D];
      lat_coords<D>(Lf, y, x);
      double fv = __longlong_as_double(0x7ff8000000000000ll);
      if (lat_in_box<D>(Lf, x)) (void)cert_eval_region<D, P>(Q, x, B1, &fv);
      const uint64_t o = s * (uint64_t)NP + (uint64_t)pt;
      fout[o] = fv;
#pragma unroll
      for (int j = 0; j < D; ++j) yout[o * D + j] = y[j];
    }
    wave_lds_sync();
  }
}

template <int D>
int region_eval_T(ip_ctx *ctx, const ip_problem *p, const int32_t *simp, int64_t n, int32_t *y, double *f,
                  double *bound, int32_t *np_out) {
  const int k = p->k;
  Template T = make_template(D, k);
  const int NP = (int)T.pts.size();
  *np_out = NP;
  if (!y || n == 0) return IP_OK;
  DevTmp tp(ctx);
  IP_TRY(tp.get(T.pts.size() * 8));
  IP_TRY_HIP(ctx, hipMemcpyAsync(tp.p, T.pts.data(), T.pts.size() * 8, hipMemcpyHostToDevice, ctx->stream));
  const unsigned blocks = (unsigned)std::min<uint64_t>(((uint64_t)n + 3) / 4, 4096);
#define IP_RE(PP)                                                                                                 \
  hipLaunchKernelGGL((region_eval_kernel<D, PP>), dim3(blocks), dim3(256), 0, ctx->stream, p->fine, k, simp,      \
                     (uint64_t)n, tp.as<uint64_t>(), NP, p->poly, y, f, bound)
  switch (p->poly.p) {
    case 1: IP_RE(1); break;
    case 2: IP_RE(2); break;
    case 3: IP_RE(3); break;
    default: IP_RE(4); break;
  }
#undef IP_RE
  IP_TRY_HIP(ctx, hipGetLastError());
  IP_TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return IP_OK;
}

// Iterative intersection points (Sec. V-B; Sec. VI: the point is refined
// by an iteration until a desired accuracy), ITERS false-position steps with
// the Illinois modification on every traced edge, a fixed count so that the
// lanes of a wave stay in step.  The bracket starts as the edge (a the
// smaller endpoint); each step evaluates f at the false-position point m,
// moves the end whose sign bit s = !(f < 0) equals s(m), and halves the value
// kept at the other end when the same end moved twice in a row; the result
// is the false-position point of the final bracket.  CANON: f in the
// canonical FP64 order (the support vectors as wave-uniform scalar loads),
// so the points equal the oracle's bit for bit; otherwise f from the FP64
// monomial form (FP32-certified mode, points within the stated tolerance).
// R edges per lane share each support-vector load.
template <int D, int P, int R, bool CANON>
__global__ __launch_bounds__(256) void refine_kernel(LatDev L, const uint64_t *__restrict__ keys, uint64_t n,
                                                     double *pts, int64_t ld, FDev F, PolyDev Q, int iters) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x * R;
  for (uint64_t base = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) * R; base < n; base += stride) {
    double a[R][D], b[R][D], m[R][D], fa[R], fb[R], fm[R];
    int last[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint64_t i = base + r < n ? base + r : n - 1;
      int32_t va[D], vb[D];
      uint32_t Rm;
      eunpack<D>(L, keys[i], va, &Rm);
#pragma unroll
      for (int j = 0; j < D; ++j) vb[j] = va[j] + (int32_t)((Rm >> j) & 1u);
      lat_coords<D>(L, va, a[r]);
      lat_coords<D>(L, vb, b[r]);
      last[r] = 0;
    }
    // f at the R points held in x[r]: canonical order or monomial form
    auto feval = [&](double (*x)[D], double *out) {
      if (CANON && F.kernel == IP_KERNEL_RBF) {
        double acc[R];
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] = 0.0;
        for (int64_t s = 0; s < F.S; ++s) {
          const double *rec = F.rec + s * 8;
          double sv[D];
#pragma unroll
          for (int j = 0; j < D; ++j) sv[j] = rec[j];
          const double al = rec[D];
#pragma unroll
          for (int r = 0; r < R; ++r) acc[r] = rbf_term<D>(sv, al, F.gamma, x[r], acc[r]);
        }
#pragma unroll
        for (int r = 0; r < R; ++r) out[r] = acc[r] + F.bias;
      } else if (CANON) {
        double acc[R];
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r] = 0.0;
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
            const double t = fma(F.gamma, dot, F.coef0);
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
        for (int r = 0; r < R; ++r) out[r] = acc[r] + F.bias;
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          double bnd;
          out[r] = poly64<D, (P > 0 ? P : 4)>(Q, x[r], &bnd);
        }
      }
    };
    feval(a, fa);
    feval(b, fb);
    for (int it = 0; it < iters; ++it) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const double t = fa[r] / (fa[r] - fb[r]);
#pragma unroll
        for (int j = 0; j < D; ++j) m[r][j] = fma(t, b[r][j] - a[r][j], a[r][j]);
      }
      feval(m, fm);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (!(fm[r] < 0.0) == !(fa[r] < 0.0)) {
#pragma unroll
          for (int j = 0; j < D; ++j) a[r][j] = m[r][j];
          fa[r] = fm[r];
          if (last[r] == -1) fb[r] = 0.5 * fb[r];
          last[r] = -1;
        } else {
#pragma unroll
          for (int j = 0; j < D; ++j) b[r][j] = m[r][j];
          fb[r] = fm[r];
          if (last[r] == 1) fa[r] = 0.5 * fa[r];
          last[r] = 1;
        }
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (base + r >= n) continue;
      const double t = fa[r] / (fa[r] - fb[r]);
#pragma unroll
      for (int j = 0; j < D; ++j) pts[(int64_t)j * ld + (int64_t)(base + r)] = fma(t, b[r][j] - a[r][j], a[r][j]);
    }
  }
}

template <int D, bool CANON>
void launch_refine(ip_ctx *ctx, const ip_problem *p, const ip_cells *c, int iters) {
  constexpr int R = 2;
  const uint64_t n = (uint64_t)c->n;
  const uint64_t blocks = std::min<uint64_t>((n + 256 * R - 1) / (256 * R), 65536);
  const int P = CANON ? p->f.p : p->poly.p;
#define IP_RF(PP)                                                                                              \
  hipLaunchKernelGGL((refine_kernel<D, PP, R, CANON>), dim3((unsigned)blocks), dim3(256), 0, ctx->stream, p->fine, \
                     (const uint64_t *)c->keys, n, c->pts, c->ld, p->f, p->poly, iters)
  switch (P) {
    case 1: IP_RF(1); break;
    case 2: IP_RF(2); break;
    case 3: IP_RF(3); break;
    case 4: IP_RF(4); break;
    default: IP_RF(0); break;
  }
#undef IP_RF
}

// Refine the points of the traced cells in place (no effect for iters = 0).
template <int D>
int refine_T(ip_ctx *ctx, const ip_problem *p, int32_t prec, int iters, ip_cells *c) {
  c->st.refine_iters = iters;
  if (iters <= 0 || c->n == 0) return IP_OK;
  // the FP32-certified mode refines with the FP64 monomial form when f has
  // one (polynomial), else with the canonical values
  const bool canon = !(prec == IP_FP32_CERTIFY && p->poly.ok);
  Timer tr;
  IP_TRY(tr.start(ctx, &c->st.ms_refine));
  if (canon)
    launch_refine<D, true>(ctx, p, c, iters);
  else
    launch_refine<D, false>(ctx, p, c, iters);
  IP_TRY_HIP(ctx, hipGetLastError());
  IP_TRY(tr.stop(ctx));
  IP_TRY(tr.flush(ctx));
  return IP_OK;
}

}  // namespace

namespace {

// Memory projection: the crossing edges on the probe lattice (coarsened by
// kc) number about N / kc^(d-1) for N fine cells (the crossing count scales
// with the zero set's area over the scale^(d-1)); each fine cell then holds
// its key (8 B), two point copies (16 d B: points and free points), its
// verdict (1 B), a traced-edge record (16 B) and its share of the vertex
// table (40 B), with a 25 % margin and 64 MiB of fixed workspace.
template <int D>
int project_T(ip_ctx *ctx, const ip_problem *p, uint64_t *bytes, int64_t *n_coarse) {
  Run s;
  s.ctx = ctx;
  s.p = p;
  s.tb = &ctx->vtc;
  s.L = p->probe;
  s.cert = false;
  IP_TRY(vt_init(s, 1ull << 16));
  ip_stats st = {};
  uint64_t nc = 0;
  const int rc = trace_direct<D>(s, st, &nc);
  if (s.out) {
    (void)hipStreamSynchronize(ctx->stream);
    release(ctx, s.out);
  }
  IP_TRY(rc);
  double cells = (double)nc * 1.25;
  for (int q = 0; q < D - 1; ++q) cells *= p->probe_k;
  *bytes = (uint64_t)(cells * (8.0 + 16.0 * D + 1.0 + 16.0 + 40.0)) + (64ull << 20);
  *n_coarse = (int64_t)nc;
  return IP_OK;
}

}  // namespace

int ip_project_impl(ip_ctx *ctx, const ip_problem *p, uint64_t *bytes, int64_t *n_coarse) {
  switch (p->d) {
    case 2: return project_T<2>(ctx, p, bytes, n_coarse);
    case 3: return project_T<3>(ctx, p, bytes, n_coarse);
    case 4: return project_T<4>(ctx, p, bytes, n_coarse);
    case 5: return project_T<5>(ctx, p, bytes, n_coarse);
    case 6: return project_T<6>(ctx, p, bytes, n_coarse);
    case 7: return project_T<7>(ctx, p, bytes, n_coarse);
    default: return ip_fail(ctx, IP_EINVAL, "dimension out of range");
  }
}

int ip_region_eval_impl(ip_ctx *ctx, const ip_problem *p, const int32_t *simp, int64_t n, int32_t *y, double *f,
                        double *bound, int32_t *np_out) {
  switch (p->d) {
    case 2: return region_eval_T<2>(ctx, p, simp, n, y, f, bound, np_out);
    case 3: return region_eval_T<3>(ctx, p, simp, n, y, f, bound, np_out);
    case 4: return region_eval_T<4>(ctx, p, simp, n, y, f, bound, np_out);
    case 5: return region_eval_T<5>(ctx, p, simp, n, y, f, bound, np_out);
    case 6: return region_eval_T<6>(ctx, p, simp, n, y, f, bound, np_out);
    case 7: return region_eval_T<7>(ctx, p, simp, n, y, f, bound, np_out);
    default: return ip_fail(ctx, IP_EINVAL, "dimension out of range");
  }
}

namespace {

template <int D>
int trace_batches_T(ip_ctx *ctx, const ip_problem *p, uint64_t budget, int32_t prec, int iters,
                    const ip_scene *scene, ip_batch_fn fn, void *user, ip_batch_summary *out) {
  const bool cert = prec == IP_FP32_CERTIFY && p->f.kernel == IP_KERNEL_POLY && ip_has_fp32_form(p);
  BatchStream bs(ctx);
  bs.scene = scene;
  bs.fn = fn;
  bs.user = user;
  bs.prec = prec;
  bs.iters = iters;
  IP_TRY(bs.init());
  ip_cells res;
  res.ctx = ctx;
  IP_TRY(trace_batch<D>(ctx, p, budget, cert, &res, &bs));
  unsigned long long dg[2] = {0, 0};
  IP_TRY_HIP(ctx, hipMemcpyAsync(dg, bs.dg, 16, hipMemcpyDeviceToHost, ctx->stream));
  IP_TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));
  out->n_cells = bs.n_cells;
  out->n_free = bs.n_free;
  out->batches = bs.batches;
  out->digest[0] = dg[0];
  out->digest[1] = dg[1];
  out->stats = res.st;
  out->stats.ms_check = bs.ms_check;
  out->stats.ms_refine = bs.ms_refine;
  out->stats.refine_iters = iters;
  return IP_OK;
}

}  // namespace

int ip_trace_batches_impl(ip_ctx *ctx, const ip_problem *p, uint64_t budget, int32_t prec, uint32_t flags,
                          const ip_scene *scene, ip_batch_fn fn, void *user, ip_batch_summary *out) {
  const int iters = (int)((flags >> 4) & 15u);
#define IP_TB(DD) return trace_batches_T<DD>(ctx, p, budget, prec, iters, scene, fn, user, out)
  switch (p->d) {
    case 2: IP_TB(2);
    case 3: IP_TB(3);
    case 4: IP_TB(4);
    case 5: IP_TB(5);
    case 6: IP_TB(6);
    case 7: IP_TB(7);
    default: return ip_fail(ctx, IP_EINVAL, "dimension out of range");
  }
#undef IP_TB
}

int ip_trace_impl(ip_ctx *ctx, const ip_problem *p, uint64_t budget, int32_t prec, uint32_t flags,
                  ip_cells *out) {
  const int iters = (int)((flags >> 4) & 15u);
  switch (p->d) {
    case 2: IP_TRY(trace_T<2>(ctx, p, budget, prec, out)); return refine_T<2>(ctx, p, prec, iters, out);
    case 3: IP_TRY(trace_T<3>(ctx, p, budget, prec, out)); return refine_T<3>(ctx, p, prec, iters, out);
    case 4: IP_TRY(trace_T<4>(ctx, p, budget, prec, out)); return refine_T<4>(ctx, p, prec, iters, out);
    case 5: IP_TRY(trace_T<5>(ctx, p, budget, prec, out)); return refine_T<5>(ctx, p, prec, iters, out);
    case 6: IP_TRY(trace_T<6>(ctx, p, budget, prec, out)); return refine_T<6>(ctx, p, prec, iters, out);
    case 7: IP_TRY(trace_T<7>(ctx, p, budget, prec, out)); return refine_T<7>(ctx, p, prec, iters, out);
    default: return ip_fail(ctx, IP_EINVAL, "dimension out of range");
  }
}
