// Internal definitions shared by the library's HIP sources: device-side
// lattice frame, key packing, open-addressing hash tables, coface
// enumeration of the permutahedral representation, and the host-side
// context / problem / result objects behind the C ABI in ip.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/ip.h"

#define IP_EMPTY_KEY 0xFFFFFFFFFFFFFFFFull
// NaN payload marking a vertex slot whose f has not been evaluated yet.
#define IP_UNEVAL_BITS 0x7FF4DEADBEEF0001ull
#define IP_SIGN_BIT 0x8000000000000000ull

// ---------------------------------------------------------------------------
// Lattice frame on the device (passed by value as a kernel argument).
// Vertex u has coordinates x_j = o_j + sum_k M[j][k] * (mul * u_k), with an
// fma chain over k; mul = 1 on the fine lattice and k on the coarse lattice
// of batch triangulation, so coarse vertices share the fine vertices' bits.
// ---------------------------------------------------------------------------
struct LatDev {
  int32_t d;
  int32_t B;         // key bits per coordinate
  int32_t mul;       // lattice refinement factor (see above)
  int32_t pad;
  int32_t vmin[8];   // key offset per coordinate
  double M[64];      // row-major, stride 8
  double Minv[64];
  double o[8], lo[8], hi[8];
};

// Manifold parameters on the device.  rec holds one 64-byte record per
// support vector: s_0..s_{d-1}, alpha, zero padding (8 doubles).
// kernel: IP_KERNEL_POLY (alpha_i (gamma <s_i, x> + coef0)^p) or
// IP_KERNEL_RBF (alpha_i exp(-(gamma |x - s_i|^2))).
struct FDev {
  const double *rec;
  int64_t S;
  int32_t p;
  int32_t kernel;
  double gamma, coef0, bias;
};

// FP32 form of an RBF-kernel f: one 32-byte record per support vector
// (s_0..s_{d-1} in FP32, alpha in FP32, |s|^2 rounded up, zero padding to 8
// floats), with the constants of its error bound (see feval.hip).
struct RbfDev {
  const float *rec;
  int64_t S;
  int32_t ok;      // 0: no FP32 form, every vertex is evaluated in FP64
  float gamma, bias;
  float nrm_max;   // largest |s_i|^2 (rounded up)
  double B64;      // |f64 - F| <= B64 for the canonical FP64 value
  double amax;     // largest |alpha_i|
};

// ln 2 = LN2_HI + LN2_LO, LN2_HI a multiple of 2^-32 (k * LN2_HI exact for
// |k| < 2^20); the FP32 split has 16 significant bits in its high part.
#define IP_LN2_HI 0.6931471806019545
#define IP_LN2_LO -4.2009150726810846e-11
#define IP_INV_LN2 1.4426950408889634
#define IP_LN2_HI32 0.693145751953125f
#define IP_LN2_LO32 1.428606765330187e-06f
#define IP_INV_LN2_32 1.4426950216293335f

// Own exponential of the canonical RBF evaluation: Cody-Waite reduction by
// ln 2 (t = k ln2 + r, |r| <= ln2 / 2), the Taylor polynomial of exp(r) to
// degree 13 in Horner form (coefficients 1/n!), then the exact scaling by
// 2^k; 0 below t = -708.  Written out in this order so that every device
// and the host agree bit for bit.
__host__ __device__ __forceinline__ double exp_own(double t) {
  if (t < -708.0) return 0.0;
  const double k = floor(t * IP_INV_LN2 + 0.5);
  double r = fma(-k, IP_LN2_HI, t);
  r = fma(-k, IP_LN2_LO, r);
  double p = 1.6059043836821613e-10;
  p = fma(r, p, 2.08767569878681e-09);
  p = fma(r, p, 2.505210838544172e-08);
  p = fma(r, p, 2.755731922398589e-07);
  p = fma(r, p, 2.7557319223985893e-06);
  p = fma(r, p, 2.48015873015873e-05);
  p = fma(r, p, 0.0001984126984126984);
  p = fma(r, p, 0.001388888888888889);
  p = fma(r, p, 0.008333333333333333);
  p = fma(r, p, 0.041666666666666664);
  p = fma(r, p, 0.16666666666666666);
  p = fma(r, p, 0.5);
  p = fma(r, p, 1.0);
  p = fma(r, p, 1.0);
  return ldexp(p, (int)k);
}

// The FP32 exponential of the certified tier: the same reduction with the
// FP32 split of ln 2 and the Taylor polynomial to degree 7; relative error
// below 40 u32 on t in [-87, 0] (reduction below 1 u, truncation 0.1 u,
// coefficient roundings 2 u, Horner at most 16 roundings on terms whose
// absolute sum is at most twice the value), 0 below t = -87 (an absolute
// error under 2e-38).
__device__ __forceinline__ float exp32_own(float t) {
  if (t < -87.0f) return 0.0f;
  const float k = floorf(t * IP_INV_LN2_32 + 0.5f);
  float r = fmaf(-k, IP_LN2_HI32, t);
  r = fmaf(-k, IP_LN2_LO32, r);
  float p = 1.984126984126984e-04f;
  p = fmaf(r, p, 1.388888888888889e-03f);
  p = fmaf(r, p, 8.333333333333333e-03f);
  p = fmaf(r, p, 4.166666666666666e-02f);
  p = fmaf(r, p, 1.666666666666667e-01f);
  p = fmaf(r, p, 0.5f);
  p = fmaf(r, p, 1.0f);
  p = fmaf(r, p, 1.0f);
  return ldexpf(p, (int)k);
}

// One canonical RBF term: alpha exp(-(gamma d2)) with d2 the fma chain of
// (x_j - s_j)^2 over j, added to acc with an fma.
template <int D>
__device__ __forceinline__ double rbf_term(const double *sv, double al, double gamma, const double *x, double acc) {
  double d2 = 0.0;
#pragma unroll
  for (int j = 0; j < D; ++j) {
    const double df = x[j] - sv[j];
    d2 = fma(df, df, d2);
  }
  return fma(al, exp_own(-(gamma * d2)), acc);
}

// FP32 monomial-basis form of f (see feval.hip).  c[0] is the constant term
// (bias included), c[1..M-1] the monomial coefficients in depth-first order.
// For every vertex in the domain: |f32 - F| <= K32 * S_abs + E0, with S_abs
// the FP32 sum of |c_m| |x^m| computed beside f32, and |f64 - F| <= B64 for
// the canonical FP64 value, F the exact value at the canonical coordinates.
// The same coefficients in FP64 (cd) give a second, FP64 evaluation in the
// monomial basis with |f64m - F| <= K64 * S_abs64 + E0.
struct PolyDev {
  const float *c;
  const double *cd;
  const uint32_t *mono;  // per coefficient: degree | variable index << (4 + 4 i)
  int32_t M;
  int32_t p;
  int32_t ok;   // 0: degree above 4, every vertex is evaluated in FP64
  int32_t pad;
  double K32, K64, E0, B64;
  double K32n;  // nested FP32 evaluation: |f32 - F| <= K32n * sum |c_m| |x^m| + E0
};

struct Counters {
  unsigned long long n_eval;     // eval-list length (reset per pass)
  unsigned long long vt_count;   // vertices inserted (total)
  unsigned long long n_out;      // output-list length (== edges in ET)
  unsigned long long n_cof;      // cofaces expanded in the current level
  unsigned long long n_fb;       // FP64 fallback list length
  unsigned long long n_fb_total; // fallbacks over the whole call
  unsigned long long n_aux;      // general-purpose append counter
  unsigned long long n_cert64;   // vertices settled by the FP64 monomial tier
  unsigned long long n_pts;      // template points evaluated (fused subdivision)
  unsigned long long n_unsettled;// template points left to the canonical tier
  unsigned long long n_direct;   // owner-emitted fine edges (batch mode)
  unsigned long long n_shared;   // intersecting template edges sent to the edge set
  unsigned int vt_fail;          // vertex-table insert found the table full
  unsigned int et_fail;          // edge-table insert found the table full
};

// ---------------------------------------------------------------------------
// Device helpers
// ---------------------------------------------------------------------------
// SplitMix64 finalizer (Steele, Lea & Flood 2014; constants as published by
// Vigna) as the table hash.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t shfl64(uint64_t v, int src) {
  uint32_t lo = __shfl((unsigned int)(v & 0xffffffffu), src, 64);
  uint32_t hi = __shfl((unsigned int)(v >> 32), src, 64);
  return ((uint64_t)hi << 32) | lo;
}

template <int D>
__device__ __forceinline__ void lat_coords(const LatDev &L, const int32_t *v, double *x) {
#pragma unroll
  for (int j = 0; j < D; ++j) {
    double acc = L.o[j];
#pragma unroll
    for (int k = 0; k < D; ++k) acc = fma(L.M[j * 8 + k], (double)(L.mul * v[k]), acc);
    x[j] = acc;
  }
}

template <int D>
__device__ __forceinline__ bool lat_in_box(const LatDev &L, const double *x) {
  bool ok = true;
#pragma unroll
  for (int j = 0; j < D; ++j) ok = ok && (x[j] >= L.lo[j]) && (x[j] <= L.hi[j]);
  return ok;
}

template <int D>
__device__ __forceinline__ uint64_t vpack(const LatDev &L, const int32_t *v) {
  uint64_t k = 0;
#pragma unroll
  for (int j = 0; j < D; ++j) k |= (uint64_t)(uint32_t)(v[j] - L.vmin[j]) << (j * L.B);
  return k;
}

template <int D>
__device__ __forceinline__ void vunpack(const LatDev &L, uint64_t k, int32_t *v) {
  const uint64_t m = (1ull << L.B) - 1ull;
#pragma unroll
  for (int j = 0; j < D; ++j) v[j] = (int32_t)((k >> (j * L.B)) & m) + L.vmin[j];
}

// True when every coordinate fits the key field.  Vertices inside the domain
// always fit (the host sizes the fields from the box); a vertex that does not
// fit lies outside the box and must not be packed.
template <int D>
__device__ __forceinline__ bool vin_range(const LatDev &L, const int32_t *v) {
  bool ok = true;
#pragma unroll
  for (int j = 0; j < D; ++j) ok = ok && (uint32_t)(v[j] - L.vmin[j]) < (1u << L.B);
  return ok;
}

template <int D>
__device__ __forceinline__ uint64_t ekey(const LatDev &L, const int32_t *v, uint32_t mask) {
  return vpack<D>(L, v) | ((uint64_t)mask << (D * L.B));
}

template <int D>
__device__ __forceinline__ void eunpack(const LatDev &L, uint64_t key, int32_t *v, uint32_t *mask) {
  key &= ~IP_SIGN_BIT;
  vunpack<D>(L, key, v);
  *mask = (uint32_t)(key >> (D * L.B)) & ((1u << D) - 1u);
}

__device__ __forceinline__ uint64_t ld_relaxed(const uint64_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Longest probe sequence: a key is never placed further than this from its
// home slot, so lookups stop there too.  At the loads the host keeps
// (<= 1/2) sequences are a few slots long; hitting the cap means the table
// is overloaded, and the insert reports failure at once (the host grows the
// table and replays the pass) instead of walking the whole table.
#define IP_MAX_PROBE 4096ull

// Open addressing with linear probing.  Returns 1 when `key` was inserted,
// 0 when it was present, -1 when the table is full; *slot gets its position.
__device__ __forceinline__ int ht_insert(uint64_t *keys, uint64_t mask, uint64_t key, uint64_t *slot) {
  uint64_t h = mix64(key) & mask;
  for (uint64_t n = 0; n <= mask && n < IP_MAX_PROBE; ++n) {
    uint64_t cur = ld_relaxed(keys + h);
    if (cur == key) {
      *slot = h;
      return 0;
    }
    if (cur == IP_EMPTY_KEY) {
      uint64_t prev = atomicCAS((unsigned long long *)(keys + h), (unsigned long long)IP_EMPTY_KEY,
                                (unsigned long long)key);
      if (prev == IP_EMPTY_KEY) {
        *slot = h;
        return 1;
      }
      if (prev == key) {
        *slot = h;
        return 0;
      }
    }
    h = (h + 1) & mask;
  }
  return -1;
}

// Lookup in a table that no thread modifies during the kernel.
__device__ __forceinline__ int64_t ht_find(const uint64_t *keys, uint64_t mask, uint64_t key) {
  uint64_t h = mix64(key) & mask;
  for (uint64_t n = 0; n <= mask && n < IP_MAX_PROBE; ++n) {
    uint64_t cur = keys[h];
    if (cur == key) return (int64_t)h;
    if (cur == IP_EMPTY_KEY) return -1;
    h = (h + 1) & mask;
  }
  return -1;
}

// Vertex-table entry: packed vertex key, f at the vertex (NaN payload while
// pending), and a bitmask of the visited edges (v, R) whose smaller endpoint
// is this vertex, bit R of the 2^d-bit mask (the edge set of the search).
struct __attribute__((aligned(32))) VEnt {
  uint64_t key;
  double f;
  unsigned long long m[2];
};

// Strided variants: the key of slot h lives at base[h * SW].
template <int SW>
__device__ __forceinline__ int ht_insert_s(uint64_t *base, uint64_t mask, uint64_t key, uint64_t *slot) {
  uint64_t h = mix64(key) & mask;
  for (uint64_t n = 0; n <= mask && n < IP_MAX_PROBE; ++n) {
    uint64_t *p = base + h * SW;
    // keys only go from empty to final, so a plain (possibly stale) load is
    // safe: a stale empty slot is settled by the CAS below
    uint64_t cur = *(volatile uint64_t *)p;
    if (cur == key) {
      *slot = h;
      return 0;
    }
    if (cur == IP_EMPTY_KEY) {
      uint64_t prev = atomicCAS((unsigned long long *)p, (unsigned long long)IP_EMPTY_KEY, (unsigned long long)key);
      if (prev == IP_EMPTY_KEY || prev == key) {
        *slot = h;
        return prev == IP_EMPTY_KEY ? 1 : 0;
      }
    }
    h = (h + 1) & mask;
  }
  return -1;
}

template <int SW>
__device__ __forceinline__ int64_t ht_find_s(const uint64_t *base, uint64_t mask, uint64_t key) {
  uint64_t h = mix64(key) & mask;
  for (uint64_t n = 0; n <= mask && n < IP_MAX_PROBE; ++n) {
    uint64_t cur = base[h * SW];
    if (cur == key) return (int64_t)h;
    if (cur == IP_EMPTY_KEY) return -1;
    h = (h + 1) & mask;
  }
  return -1;
}

__device__ __forceinline__ int vt_insert(VEnt *vt, uint64_t mask, uint64_t key, uint64_t *slot) {
  return ht_insert_s<4>((uint64_t *)vt, mask, key, slot);
}
__device__ __forceinline__ int64_t vt_find(const VEnt *vt, uint64_t mask, uint64_t key) {
  return ht_find_s<4>((const uint64_t *)vt, mask, key);
}

// Wave-level staged append: the lanes' items go to a per-wave LDS buffer and
// are copied to the global list with one atomicAdd per STAGE items, instead
// of one atomic per wave and step on a single counter.  All lanes of the
// wave must call these together; `n` is wave-uniform.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T, typename W>
__device__ __forceinline__ void stage_flush(T *st, int &n, W writer, unsigned long long *ctr) {
  if (n == 0) return;
  wave_lds_sync();
  const int lane = __lane_id();
  unsigned long long base = 0;
  if (lane == 0) base = atomicAdd(ctr, (unsigned long long)n);
  base = shfl64(base, 0);
  for (int i = lane; i < n; i += 64) writer(base + (unsigned long long)i, st[i]);
  wave_lds_sync();
  n = 0;
}

template <int STAGE, typename T, typename W>
__device__ __forceinline__ void stage_put(T *st, int &n, bool pred, const T &item, W writer,
                                          unsigned long long *ctr) {
  const uint64_t bal = __ballot(pred);
  if (!bal) return;
  const int nb = __popcll(bal);
  if (n + nb > STAGE) stage_flush(st, n, writer, ctr);
  if (pred) st[n + __popcll(bal & ((1ull << __lane_id()) - 1ull))] = item;
  n += nb;
}

// Depth-first walk over the monomials x_{j1} x_{j2} ... x_{jk}, j1 <= ... <=
// jk, k = 1..K, in the order the host stored the coefficients: at index J the
// monomial mono * x_J, then its extensions by x_{j >= J}, then J + 1.
// Accumulates sum c_m x^m into acc and sum |c_m| |x^m| into aabs.
template <typename T, int D, int K, int J>
struct MonoWalk {
  static __device__ __forceinline__ void run(const T *x, T mono, const T *__restrict__ C, int &ci, T &acc,
                                             T &aabs) {
    if constexpr (J < D) {
      const T m = mono * x[J];
      const T c = C[ci];
      ++ci;
      acc = fma(c, m, acc);
      aabs = fma(fabs(c), fabs(m), aabs);
      if constexpr (K > 1) MonoWalk<T, D, K - 1, J>::run(x, m, C, ci, acc, aabs);
      MonoWalk<T, D, K, J + 1>::run(x, mono, C, ci, acc, aabs);
    }
  }
};

// The same walk without the |c| |x^m| sum: sum c_m x^m into acc.
template <typename T, int D, int K, int J>
struct MonoVal {
  static __device__ __forceinline__ void run(const T *x, T mono, const T *__restrict__ C, int &ci, T &acc) {
    if constexpr (J < D) {
      const T m = mono * x[J];
      acc = fma(C[ci], m, acc);
      ++ci;
      if constexpr (K > 1) MonoVal<T, D, K - 1, J>::run(x, m, C, ci, acc);
      MonoVal<T, D, K, J + 1>::run(x, mono, C, ci, acc);
    }
  }
};

// Nested (multivariate Horner) form of the same polynomial, in the same
// coefficient order: the sum over j = J .. D-1 of x_j * (c_{m x_j} + the
// extensions of m x_j).  Each coefficient passes through at most D + 1
// roundings per level and P levels, against the M - 1 of a flat sum.
template <typename T, int D, int K, int J>
struct MonoNest {
  static __device__ __forceinline__ T run(const T *x, const T *__restrict__ C, int &ci) {
    if constexpr (J < D) {
      T sub = C[ci];
      ++ci;
      if constexpr (K > 1) sub = sub + MonoNest<T, D, K - 1, J>::run(x, C, ci);
      const T rest = MonoNest<T, D, K, J + 1>::run(x, C, ci);
      return fma(x[J], sub, rest);
    } else {
      return T(0);
    }
  }
};

// f in the monomial basis, FP64, with the rigorous bound on |f - F|.
template <int D, int P>
__device__ __forceinline__ double poly64(const PolyDev &Q, const double *x, double *bound) {
  double acc = Q.cd[0], aabs = fabs(Q.cd[0]);
  int ci = 1;
  MonoWalk<double, D, P, 0>::run(x, 1.0, Q.cd, ci, acc, aabs);
  *bound = Q.K64 * aabs + Q.E0;
  return acc;
}

template <int D>
__device__ __forceinline__ double poly64_any(const PolyDev &Q, const double *x, double *bound) {
  switch (Q.p) {
    case 1: return poly64<D, 1>(Q, x, bound);
    case 2: return poly64<D, 2>(Q, x, bound);
    case 3: return poly64<D, 3>(Q, x, bound);
    default: return poly64<D, 4>(Q, x, bound);
  }
}

// Tiered certified evaluation at the canonical FP64 coordinates x64.  Tier 1:
// FP32 in the monomial basis, settled when |f32| > B32 + B64.  Tier 2: FP64
// in the monomial basis, settled when |f64m| > B64m + B64.  Returns the tier
// that settled the sign of the canonical FP64 value (f and its bound in *fv,
// *bnd), or 3 when neither did.
template <int D, int P>
__device__ __forceinline__ int cert_eval(const PolyDev &Q, const double *x64, double *fv, double *bnd) {
  float x[D];
#pragma unroll
  for (int j = 0; j < D; ++j) x[j] = (float)x64[j];
  float acc = Q.c[0], aabs = fabsf(Q.c[0]);
  int ci = 1;
  MonoWalk<float, D, P, 0>::run(x, 1.0f, Q.c, ci, acc, aabs);
  *bnd = Q.K32 * (double)aabs + Q.E0;
  *fv = (double)acc;
  if (fabs(*fv) > *bnd + Q.B64) return 1;
  *fv = poly64<D, P>(Q, x64, bnd);
  return fabs(*fv) > *bnd + Q.B64 ? 2 : 3;
}

// Upper bound, for every point x of a region with |x_j| <= X_j, of the FP32
// sum S_abs that the FP32 tier forms beside f32 (sum of |c_m| |x^m| with the
// FP32 roundings of coefficients, coordinates, products and the sum), from
// the FP64 monomial coefficients: K32 * Smax + E0 then bounds |f32 - F| at
// every such point.  The terms are spread over the wave (lane l takes
// monomials l, l + 64, ...) and summed with shuffles; every lane gets the
// result.  All lanes of the wave must call it together.
__device__ __forceinline__ double region_sabs_bound(const PolyDev &Q, const double *X, int lane) {
  double t = 0.0;
  for (int m = lane; m < Q.M; m += 64) {
    const uint32_t pk = Q.mono[m];
    double term = fabs(Q.cd[m]);
    for (int q = 0; q < (int)(pk & 15u); ++q) term *= X[(pk >> (4 + 4 * q)) & 15u];
    t += term;
  }
#pragma unroll
  for (int off = 32; off; off >>= 1) t += __shfl_xor(t, off, 64);
  return t * (1.0 + 1e-12);
}

// Tier-1 evaluation, nested FP32 form, against a bound B1 (= K32n * Smax +
// E0, Smax = region_sabs_bound) valid for the whole region of x64: 1 when
// |f32| settles the sign, else 3.
template <int D, int P>
__device__ __forceinline__ int cert_eval_region(const PolyDev &Q, const double *x64, double B1, double *fv) {
  float x[D];
#pragma unroll
  for (int j = 0; j < D; ++j) x[j] = (float)x64[j];
  int ci = 1;
  const float v = Q.c[0] + MonoNest<float, D, P, 0>::run(x, Q.c, ci);
  *fv = (double)v;
  return fabs(*fv) > B1 + Q.B64 ? 1 : 3;
}

// Deposit the low bits of src into the set positions of mask (ascending).
__device__ __forceinline__ uint32_t pdep32(uint32_t src, uint32_t mask) {
  uint32_t out = 0;
  for (uint32_t b = 1; mask; b <<= 1) {
    uint32_t low = mask & (0u - mask);
    if (src & b) out |= low;
    mask ^= low;
  }
  return out;
}

// Number of 2-simplex cofaces of edge (v, (R, Q)): ordered two-part splits
// of R plus those of Q = {0..D} \ R, i.e. (2^|R| - 2) + (2^|Q| - 2).
template <int D>
__device__ __forceinline__ int n_cofaces2(uint32_t R) {
  int nP = __popc(R);
  return (1 << nP) - 2 + (1 << (D + 1 - nP)) - 2;
}

// Third vertex c of coface r of edge (v, R).  Splitting R into (A, R\A)
// gives c = v + 1_A.  Splitting Q into (A, Q\A) gives c = v + 1_R + 1_A when
// D is not in A; when D is in A the root -(1..1) wraps the cycle and
// c = v - 1_{Q\A}.
template <int D>
__device__ __forceinline__ void coface_vertex(const int32_t *v, uint32_t R, int r, int32_t *c) {
  const uint32_t full = (1u << (D + 1)) - 1u;
  const uint32_t Q = full & ~R;
  const int splitR = (1 << __popc(R)) - 2;
  if (r < splitR) {
    uint32_t A = pdep32((uint32_t)r + 1u, R);
#pragma unroll
    for (int j = 0; j < D; ++j) c[j] = v[j] + (int32_t)((A >> j) & 1u);
  } else {
    uint32_t A = pdep32((uint32_t)(r - splitR) + 1u, Q);
    if (!((A >> D) & 1u)) {
#pragma unroll
      for (int j = 0; j < D; ++j) c[j] = v[j] + (int32_t)((R >> j) & 1u) + (int32_t)((A >> j) & 1u);
    } else {
      uint32_t Bm = Q & ~A;
#pragma unroll
      for (int j = 0; j < D; ++j) c[j] = v[j] - (int32_t)((Bm >> j) & 1u);
    }
  }
}

// Canonical edge between two vertices of one simplex (their difference is a
// 0/1 vector up to sign): the componentwise smaller endpoint and the support.
template <int D>
__device__ __forceinline__ bool edge_canon(const int32_t *a, const int32_t *b, int32_t *vmin, uint32_t *mask) {
  uint32_t m = 0;
  bool pos = false;
#pragma unroll
  for (int j = 0; j < D; ++j) {
    int32_t df = b[j] - a[j];
    if (df != 0) {
      m |= 1u << j;
      pos = df > 0;
    }
  }
#pragma unroll
  for (int j = 0; j < D; ++j) vmin[j] = pos ? a[j] : b[j];
  *mask = m;
  return pos;  // true when a is the smaller endpoint
}

// ---------------------------------------------------------------------------
// Host-side objects
// ---------------------------------------------------------------------------
struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
};

// Caching device allocator of a context: freed blocks are kept (by size)
// and handed out again to requests of at most their size and at least half
// of it, so repeated traces of similar size reuse their buffers instead of
// paying hipMalloc / hipFree (which synchronise the device) every call.
// Sizes round up to 2 MiB.  When hipMalloc fails the cache is released and
// the allocation retried.  Thread-safe: results of the serving loop can be
// freed from another thread.
struct DevCache {
  std::mutex mu;
  std::multimap<size_t, void *> idle;   // size -> block
  std::unordered_map<void *, size_t> size_of;
  size_t idle_bytes = 0;
  size_t limit = 0;                     // bytes kept idle at most
};

// Buffers of one vertex table: its VEnt entries, the pending-evaluation
// list, and in FP32 mode the per-slot bounds and the FP64 fallback list.
struct VtBufs {
  DevBuf keys, eval, vals, fb;
};

struct ip_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  Counters *ctr_dev = nullptr;
  Counters *ctr_host = nullptr;  // pinned
  // persistent workspace (grow-only): the fine-lattice vertex table (direct
  // trace, FP64 batch subdivision) and the coarse-lattice one (batch mode),
  // kept apart so that neither is handed to the other and reallocated
  VtBufs vtf, vtc;
  DevBuf vt_aux, scratch;
  DevBuf scene;
  DevCache cache;
  // this device's copy of the scratch array of ip_feval_noalloc
  void *noalloc_scratch = nullptr;
  // device allocations that reached hipMalloc (cache misses), for the stats
  int64_t n_hip_malloc = 0;
  int64_t hip_malloc_bytes = 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  int64_t last_fallback = 0;  // FP64 re-evaluations of the last ip_feval
  // page-locked staging of the per-batch C_free hand-off and its two device
  // staging slots (grow-only, kept across calls)
  void *host_stage = nullptr;
  size_t host_stage_bytes = 0;
  void *dev_stage[2] = {nullptr, nullptr};
  size_t dev_stage_bytes[2] = {0, 0};
};

struct ip_problem {
  ip_ctx *ctx = nullptr;
  int32_t d = 0;
  int32_t k = 1;
  LatDev fine;      // fine lattice (mul = 1)
  LatDev coarse;    // coarse lattice (mul = k); equal to fine when k = 1
  LatDev probe;     // lattice of the memory projection: the coarse one, or
                    // the fine one coarsened by 4 for a direct trace
  int32_t probe_k = 4;
  FDev f;
  double *rec_dev = nullptr;
  double *seeds_dev = nullptr;
  int64_t n_seeds = 0;
  PolyDev poly = {};
  void *poly_dev = nullptr;
  RbfDev rbf = {};
  void *rbf_dev = nullptr;
};

struct ip_cells {
  ip_ctx *ctx = nullptr;
  int32_t d = 0;
  int32_t B = 0;
  int32_t vmin[8] = {0};
  int64_t n = 0;
  uint64_t *keys = nullptr;    // n keys (sign bit cleared)
  double *pts = nullptr;       // SoA d x ld
  int64_t ld = 0;
  uint8_t *verdict = nullptr;  // n (after ip_check_cells)
  double *free_pts = nullptr;  // SoA d x ld_free
  int64_t n_free = 0;
  ip_stats st = {};
};

// Device memory through the context's cache (see DevCache).
int ip_dalloc(ip_ctx *ctx, void **p, size_t bytes);
void ip_dfree(ip_ctx *ctx, void *p);
void ip_cache_release(ip_ctx *ctx);

// Error helpers used by the host code.
int ip_fail(ip_ctx *ctx, int code, const std::string &msg);
int ip_hip(ip_ctx *ctx, hipError_t e, const char *what);
int ip_ensure(ip_ctx *ctx, DevBuf &b, size_t bytes);

#define IP_TRY_HIP(ctx, call)                            \
  do {                                                   \
    hipError_t e_ = (call);                              \
    if (e_ != hipSuccess) return ip_hip(ctx, e_, #call); \
  } while (0)
#define IP_TRY(call)        \
  do {                      \
    int r_ = (call);        \
    if (r_ != IP_OK) return r_; \
  } while (0)

// Entry points implemented across the sources.
int ip_trace_impl(ip_ctx *ctx, const ip_problem *p, uint64_t budget, int32_t prec, uint32_t flags,
                  ip_cells *out);
int ip_feval_impl(ip_ctx *ctx, const ip_problem *p, const int32_t *v_dev, int64_t n, int32_t prec,
                  double *f_dev, double *bound_dev);
int ip_feval_noalloc_impl(ip_ctx *ctx, const ip_problem *p, const int32_t *v_dev, int64_t n, int32_t prec,
                          double *f_dev, double *bound_dev);
int ip_region_eval_impl(ip_ctx *ctx, const ip_problem *p, const int32_t *simp, int64_t n, int32_t *y, double *f,
                        double *bound, int32_t *np_out);
// Projected device bytes of tracing and checking p (the serving loop's
// admission): a trace on the probe lattice gives the coarse crossing count.
int ip_project_impl(ip_ctx *ctx, const ip_problem *p, uint64_t *bytes, int64_t *n_coarse);
int ip_seed_search_impl(ip_ctx *ctx, const ip_problem *p, const double *q0, int64_t n, int32_t iters, double *q,
                        double *fq);
// True when f has a certified FP32 form (polynomial of degree <= 4, or RBF).
bool ip_has_fp32_form(const ip_problem *p);
// Looks up this device's address of the ip_feval_noalloc scratch (once per
// device) and stores it in ctx; the device must be current.
int ip_noalloc_setup(ip_ctx *ctx);
int ip_check_impl(ip_ctx *ctx, const ip_scene *scene, const double *q_dev, int64_t n, int64_t ld,
                  uint8_t *verdict_dev);
int ip_check_gather_impl(ip_ctx *ctx, const ip_scene *scene, ip_cells *c);
// Sorts the n coarse n-simplex keys sig (base vertex packed in D fields of B
// bits above LB Lehmer bits) by the Morton code of the base vertex, in place;
// waits for the stream.  Defined in order.hip.
int ip_sort_sigma(ip_ctx *ctx, uint64_t *sig, uint64_t n, int D, int B, int LB);
// Per-batch trace, check and C_free hand-off (ip_trace_check_batches).
int ip_trace_batches_impl(ip_ctx *ctx, const ip_problem *p, uint64_t budget, int32_t prec, uint32_t flags,
                          const ip_scene *scene, ip_batch_fn fn, void *user, ip_batch_summary *out);
// Adds the digest terms of keys[0 .. n) to acc[0] (sum) and acc[1] (xor),
// device accumulators, on the context's stream.
int ip_digest_accumulate(ip_ctx *ctx, const uint64_t *keys, int64_t n, unsigned long long *acc);
// The checked cells' C_free points, row-major n_free x d, into device
// memory out_dev (n_free d doubles), on the context's stream.
int ip_interleave_free(ip_ctx *ctx, const ip_cells *c, double *out_dev);
// The checked cells' C_free points, row-major n_free x d, into host memory
// (interleaved on the device, then one copy); waits for the stream.
int ip_free_points_to_host(ip_ctx *ctx, const ip_cells *c, double *host);

// f evaluation of the vertices listed in `list` (slots of the vertex table);
// results go into vt_vals[slot].  Defined in feval.hip.
// FP32 certified evaluation of the listed slots: vt[slot].f and vb[slot]
// (the bound, or -1 when the vertex needs FP64); unsettled slots are
// appended to fb (counter fb_ctr).  Then set vb[list[i]] = v.
int launch_feval32(ip_ctx *ctx, const ip_problem *p, const LatDev &L, const uint32_t *list, uint64_t n_list,
                   VEnt *vt, float *vb, uint32_t *fb, unsigned long long *fb_ctr);
int launch_set_vb(ip_ctx *ctx, const uint32_t *list, uint64_t n, float *vb, float v);
// vt: vertex-table entries; the result goes into vt[slot].f.
int launch_feval64(ip_ctx *ctx, const ip_problem *p, const LatDev &L, const uint32_t *list,
                   uint64_t n_list, VEnt *vt);
// The same for list[0 .. *n_dev) with *n_dev (written on the device by an
// earlier kernel) at most n_max: no host read of the count.
int launch_feval64_dev(ip_ctx *ctx, const ip_problem *p, const LatDev &L, const uint32_t *list, uint64_t n_max,
                       const unsigned long long *n_dev, VEnt *vt);
// Canonical FP64 f at n raw vertices (int32, row-major n x d) into out[i].
int launch_feval64_raw(ip_ctx *ctx, const ip_problem *p, const LatDev &L, const int32_t *v, uint64_t n,
                       double *out);
