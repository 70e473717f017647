// C ABI entry points (include/ip.h): argument validation, context and
// handle management.  All device work is done by the kernels in trace.hip,
// feval.hip and check.hip.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "ip_internal.h"

int ip_fail(ip_ctx *ctx, int code, const std::string &msg) {
  if (ctx) ctx->err = msg;
  return code;
}

int ip_hip(ip_ctx *ctx, hipError_t e, const char *what) {
  char buf[512];
  snprintf(buf, sizeof(buf), "HIP error %d (%s) in %s", (int)e, hipGetErrorString(e), what);
  (void)hipGetLastError();
  return ip_fail(ctx, e == hipErrorOutOfMemory ? IP_ENOMEM : IP_EDEVICE, buf);
}

// Allocator diagnostics on stderr when the environment sets IP_LOG.
static bool alloc_log_on() {
  static const bool on = getenv("IP_LOG") != nullptr;
  return on;
}

int ip_dalloc(ip_ctx *ctx, void **p, size_t bytes) {
  const size_t gran = 2ull << 20;
  size_t want = ((bytes < 256 ? 256 : bytes) + gran - 1) / gran * gran;
  {
    std::lock_guard<std::mutex> lk(ctx->cache.mu);
    auto it = ctx->cache.idle.lower_bound(want);
    if (it != ctx->cache.idle.end() && it->first <= 2 * want) {
      *p = it->second;
      ctx->cache.idle_bytes -= it->first;
      ctx->cache.idle.erase(it);
      return IP_OK;
    }
  }
  hipError_t e = hipMalloc(p, want);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    ip_cache_release(ctx);
    e = hipMalloc(p, want);
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return ip_fail(ctx, IP_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
  }
  std::lock_guard<std::mutex> lk(ctx->cache.mu);
  ctx->cache.size_of[*p] = want;
  ++ctx->n_hip_malloc;
  ctx->hip_malloc_bytes += (int64_t)want;
  if (alloc_log_on())
    fprintf(stderr, "[ip] hipMalloc %.3f GiB (idle cache %.3f GiB)\n", want / 1073741824.0,
            ctx->cache.idle_bytes / 1073741824.0);
  return IP_OK;
}

void ip_dfree(ip_ctx *ctx, void *p) {
  if (!p) return;
  std::lock_guard<std::mutex> lk(ctx->cache.mu);
  auto it = ctx->cache.size_of.find(p);
  if (it == ctx->cache.size_of.end()) return;  // not ours
  const size_t sz = it->second;
  if (ctx->cache.idle_bytes + sz > ctx->cache.limit) {
    // keep the newest blocks: drop the largest idle ones first
    while (!ctx->cache.idle.empty() && ctx->cache.idle_bytes + sz > ctx->cache.limit) {
      auto last = std::prev(ctx->cache.idle.end());
      if (alloc_log_on()) fprintf(stderr, "[ip] cache evicts %.3f GiB\n", last->first / 1073741824.0);
      (void)hipFree(last->second);
      ctx->cache.size_of.erase(last->second);
      ctx->cache.idle_bytes -= last->first;
      ctx->cache.idle.erase(last);
    }
    if (sz > ctx->cache.limit) {
      (void)hipFree(p);
      ctx->cache.size_of.erase(it);
      return;
    }
  }
  ctx->cache.idle.emplace(sz, p);
  ctx->cache.idle_bytes += sz;
}

void ip_cache_release(ip_ctx *ctx) {
  std::lock_guard<std::mutex> lk(ctx->cache.mu);
  // idle blocks were last used on this context's stream
  (void)hipStreamSynchronize(ctx->stream);
  for (auto &kv : ctx->cache.idle) {
    (void)hipFree(kv.second);
    ctx->cache.size_of.erase(kv.second);
  }
  ctx->cache.idle.clear();
  ctx->cache.idle_bytes = 0;
}

int ip_ensure(ip_ctx *ctx, DevBuf &b, size_t bytes) {
  if (b.bytes >= bytes && b.p) return IP_OK;
  if (b.p) {
    (void)hipStreamSynchronize(ctx->stream);
    ip_dfree(ctx, b.p);
  }
  b.p = nullptr;
  b.bytes = 0;
  IP_TRY(ip_dalloc(ctx, &b.p, bytes));
  b.bytes = bytes;
  return IP_OK;
}

namespace {

bool finite_all(const double *p, int64_t n) {
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

// Key packing range of lattice coordinates for vertices inside the box:
// z = Minv (y - o) / mul over the box corners, with a margin of 2.
int build_lattice(ip_ctx *ctx, const ip_space *sp, int32_t mul, LatDev *L) {
  const int d = sp->d;
  memset(L, 0, sizeof(*L));
  L->d = d;
  L->mul = mul;
  L->B = 0;
  for (int j = 0; j < d; ++j) {
    for (int k = 0; k < d; ++k) {
      L->M[j * 8 + k] = sp->M[j * d + k];
      L->Minv[j * 8 + k] = sp->Minv[j * d + k];
    }
    L->o[j] = sp->offset[j];
    L->lo[j] = sp->lo[j];
    L->hi[j] = sp->hi[j];
  }
  for (int j = 0; j < d; ++j) {
    double zl = 0.0, zh = 0.0;
    for (int k = 0; k < d; ++k) {
      double a = sp->Minv[j * d + k] * (sp->lo[k] - sp->offset[k]);
      double b = sp->Minv[j * d + k] * (sp->hi[k] - sp->offset[k]);
      zl += a < b ? a : b;
      zh += a < b ? b : a;
    }
    zl /= mul;
    zh /= mul;
    double vmin = std::floor(zl) - 2.0, vmax = std::ceil(zh) + 2.0;
    if (!(vmin > -2.0e9 && vmax < 2.0e9)) return ip_fail(ctx, IP_ERANGE, "lattice coordinates overflow int32");
    const double range = vmax - vmin + 1.0;
    int bits = 1;
    while (std::ldexp(1.0, bits) < range && bits < 31) ++bits;
    if (bits > L->B) L->B = bits;
    L->vmin[j] = (int32_t)vmin;
  }
  // an edge key holds d coordinates of B bits and a d-bit direction mask
  // below the frontier's sign bit
  if (d * L->B + d > 63)
    return ip_fail(ctx, IP_ERANGE,
                   "domain spans too many lattice steps: " + std::to_string(L->B) + " bits per coordinate in " +
                       std::to_string(d) + " dimensions exceed the 64-bit keys");
  return IP_OK;
}

void mono_dfs(int d, int left, int jmin, std::vector<int> &cur, std::vector<std::vector<int>> &out) {
  for (int j = jmin; j < d; ++j) {
    cur.push_back(j);
    out.push_back(cur);
    if (left > 1) mono_dfs(d, left - 1, j, cur, out);
    cur.pop_back();
  }
}

double binom(int n, int k) {
  double r = 1.0;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

// Monomial-basis coefficients of f and the error-bound constants of the FP32
// certified path.  With t_i = gamma <s_i, x> + coef0,
//   sum_i alpha_i t_i^p = sum_k C(p,k) coef0^(p-k) gamma^k sum_i alpha_i <s_i,x>^k
// and <s_i,x>^k expands into the monomials of degree k with multinomial
// weights.  Every FP64 step is covered by a forward error bound (Higham's
// gamma_n = n u / (1 - n u), here with generous integer factors).
int build_poly(ip_ctx *ctx, ip_problem *p, const ip_fparams *f, const ip_space *sp) {
  p->poly = PolyDev{};
  const int d = f->d, P = f->degree;
  const int64_t S = f->n_sv;
  if (f->kernel != IP_KERNEL_POLY || P > 4) return IP_OK;
  std::vector<std::vector<int>> monos;
  std::vector<int> cur;
  mono_dfs(d, P, 0, cur, monos);
  const int M = (int)monos.size() + 1;
  const double u64 = std::ldexp(1.0, -53), u32 = std::ldexp(1.0, -24);
  double X[8], X2 = 0.0;
  for (int j = 0; j < d; ++j) {
    X[j] = std::max(std::fabs(sp->lo[j]), std::fabs(sp->hi[j])) * (1.0 + 1e-12);
    X2 += X[j] * X[j];
  }
  X2 = std::sqrt(X2) * (1.0 + 1e-12);
  std::vector<double> c(M), e(M);
  double sum_a = 0.0, abs_a = 0.0, c0p = 1.0;
  for (int64_t i = 0; i < S; ++i) {
    sum_a += f->alpha[i];
    abs_a += std::fabs(f->alpha[i]);
  }
  for (int q = 0; q < P; ++q) c0p *= f->coef0;
  c[0] = c0p * sum_a + f->bias;
  e[0] = u64 * ((double)(S + P + 4) * std::fabs(c0p) * abs_a + std::fabs(f->bias) + 2.0 * std::fabs(c[0])) * 1.01;
  double fact[8] = {1, 1, 2, 6, 24, 120, 720, 5040};
  for (size_t mi = 0; mi < monos.size(); ++mi) {
    const std::vector<int> &m = monos[mi];
    const int k = (int)m.size();
    int cnt[8] = {0};
    for (int j : m) ++cnt[j];
    double multi = fact[k];
    for (int j = 0; j < d; ++j) multi /= fact[cnt[j]];
    double scale = binom(P, k) * multi;
    for (int q = 0; q < P - k; ++q) scale *= f->coef0;
    for (int q = 0; q < k; ++q) scale *= f->gamma;
    double sum = 0.0, ab = 0.0;
    for (int64_t i = 0; i < S; ++i) {
      double t = f->alpha[i];
      for (int j : m) t *= f->sv[i * d + j];
      sum += t;
      ab += std::fabs(t);
    }
    c[mi + 1] = scale * sum;
    e[mi + 1] = u64 * ((double)(S + 2 * P + 4) * std::fabs(scale) * ab + (double)(2 * P + 12) * std::fabs(c[mi + 1])) * 1.01;
  }
  double E0 = e[0];
  for (size_t mi = 0; mi < monos.size(); ++mi) {
    double xm = 1.0;
    for (int j : monos[mi]) xm *= X[j];
    E0 += e[mi + 1] * xm * (1.0 + 1e-12);
  }
  double sg = 0.0;
  for (int64_t i = 0; i < S; ++i) {
    double nn = 0.0;
    for (int j = 0; j < d; ++j) nn += f->sv[i * d + j] * f->sv[i * d + j];
    double g = std::fabs(f->gamma) * std::sqrt(nn) * (1.0 + 1e-12) * X2 + std::fabs(f->coef0);
    double gp = 1.0;
    for (int q = 0; q < P; ++q) gp *= g;
    sg += std::fabs(f->alpha[i]) * gp;
  }
  p->poly.B64 = u64 * (double)((P - 1) + P * (d + 2) + S + 3) * sg * 1.01 + 2.0 * u64 * std::fabs(f->bias);
  p->poly.K32 = u32 * (double)(2 * P + M + 4) * (1.0 + (double)(M + 4) * u32) * 1.001;
  // nested form: every term c_m x^m of f is perturbed by at most
  // P (d + 1) roundings of the nested sums, P of the FP32 coordinates, one
  // of its FP32 coefficient and one of the final addition
  {
    const double N = (double)(P * (d + 2) + 2);
    p->poly.K32n = N * u32 / (1.0 - N * u32) * 1.001;
  }
  p->poly.K64 = u64 * (double)(2 * P + M + 4) * (1.0 + (double)(M + 4) * u64) * 1.001;
  p->poly.E0 = E0 * (1.0 + 1e-9);
  p->poly.M = M;
  p->poly.p = P;
  std::vector<float> cf(M);
  for (int m = 0; m < M; ++m) cf[m] = (float)c[m];
  for (int m = 0; m < M; ++m)
    if (!std::isfinite(cf[m])) return IP_OK;  // out of FP32 range: FP64 only
  // one buffer: M doubles, M floats, M monomial index words
  // variable indices of each monomial, in the same depth-first order
  std::vector<uint32_t> mono(M, 0u);
  for (size_t mi = 0; mi < monos.size(); ++mi) {
    uint32_t pk = (uint32_t)monos[mi].size();
    for (size_t q = 0; q < monos[mi].size(); ++q) pk |= (uint32_t)monos[mi][q] << (4 + 4 * q);
    mono[mi + 1] = pk;
  }
  IP_TRY_HIP(ctx, hipMalloc((void **)&p->poly_dev, 16 * (size_t)M));
  IP_TRY_HIP(ctx, hipMemcpyAsync(p->poly_dev, c.data(), 8 * (size_t)M, hipMemcpyHostToDevice, ctx->stream));
  IP_TRY_HIP(ctx, hipMemcpyAsync((char *)p->poly_dev + 8 * (size_t)M, cf.data(), 4 * (size_t)M,
                                 hipMemcpyHostToDevice, ctx->stream));
  IP_TRY_HIP(ctx, hipMemcpyAsync((char *)p->poly_dev + 12 * (size_t)M, mono.data(), 4 * (size_t)M,
                                 hipMemcpyHostToDevice, ctx->stream));
  IP_TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));
  p->poly.cd = (const double *)p->poly_dev;
  p->poly.c = (const float *)((const char *)p->poly_dev + 8 * (size_t)M);
  p->poly.mono = (const uint32_t *)((const char *)p->poly_dev + 12 * (size_t)M);
  p->poly.ok = 1;
  return IP_OK;
}

// FP32 records of an RBF-kernel f and the bound of its canonical FP64 value.
// Each canonical term alpha exp(-(gamma d2)) carries a relative error of at
// most 62 u from the own exponential (reduction 2 u, Horner at most 28
// roundings on terms whose absolute sum is at most twice the value, the
// coefficients 2 u) and an absolute error of at most |alpha| u (d + 4) / e
// from the rounding of d2 and of gamma d2 (the exponent moves by at most
// gamma u (d + 4) d2, and gamma d2 exp(-gamma d2) <= 1/e); the sum over the
// support vectors adds at most S u sum |alpha|, the bias and the final add
// u (|bias| + sum |alpha|).
int build_rbf(ip_ctx *ctx, ip_problem *p, const ip_fparams *f) {
  p->rbf = RbfDev{};
  if (f->kernel != IP_KERNEL_RBF) return IP_OK;
  const int d = f->d;
  const int64_t S = f->n_sv;
  const double u64 = std::ldexp(1.0, -53);
  double sum_a = 0.0, amax = 0.0, nmax = 0.0;
  std::vector<float> rec((size_t)S * 8, 0.0f);
  bool ok = std::isfinite((float)f->gamma) && std::isfinite((float)f->bias);
  for (int64_t i = 0; i < S; ++i) {
    double nrm = 0.0;
    for (int j = 0; j < d; ++j) {
      rec[i * 8 + j] = (float)f->sv[i * d + j];
      nrm += f->sv[i * d + j] * f->sv[i * d + j];
      ok = ok && std::isfinite(rec[i * 8 + j]);
    }
    rec[i * 8 + d] = (float)f->alpha[i];
    ok = ok && std::isfinite(rec[i * 8 + d]);
    nmax = std::max(nmax, nrm);
    sum_a += std::fabs(f->alpha[i]);
    amax = std::max(amax, std::fabs(f->alpha[i]));
  }
  const double B64 = 1.01 * u64 * (sum_a * (62.0 + (d + 4) / 2.718281828459045 + (double)S + 1.0) + 2.0 * std::fabs(f->bias));
  p->rbf.B64 = B64;
  p->rbf.amax = amax;
  p->rbf.S = S;
  p->rbf.gamma = (float)f->gamma;
  p->rbf.bias = (float)f->bias;
  p->rbf.nrm_max = std::nextafter((float)(nmax * (1.0 + 1e-6)), INFINITY);
  // the points of FP32 mode check their placement against this bound too
  p->poly.B64 = B64;
  if (!ok) return IP_OK;  // out of FP32 range: FP64 only
  IP_TRY_HIP(ctx, hipMalloc(&p->rbf_dev, rec.size() * 4));
  IP_TRY_HIP(ctx, hipMemcpyAsync(p->rbf_dev, rec.data(), rec.size() * 4, hipMemcpyHostToDevice, ctx->stream));
  IP_TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));
  p->rbf.rec = (const float *)p->rbf_dev;
  p->rbf.ok = 1;
  return IP_OK;
}

}  // namespace

extern "C" {

int ip_create(ip_ctx **out, int device, void *stream) {
  if (!out) return IP_EINVAL;
  *out = nullptr;
  ip_ctx *ctx = new (std::nothrow) ip_ctx();
  if (!ctx) return IP_ENOMEM;
  ctx->device = device;
  ctx->stream = (hipStream_t)stream;
  hipError_t e = hipSetDevice(device);
  if (e == hipSuccess) e = hipMalloc((void **)&ctx->ctr_dev, sizeof(Counters));
  if (e == hipSuccess) e = hipHostMalloc((void **)&ctx->ctr_host, sizeof(Counters), hipHostMallocDefault);
  if (e == hipSuccess) e = hipEventCreate(&ctx->ev0);
  if (e == hipSuccess) e = hipEventCreate(&ctx->ev1);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    if (ctx->ctr_dev) (void)hipFree(ctx->ctr_dev);
    if (ctx->ctr_host) (void)hipHostFree(ctx->ctr_host);
    delete ctx;
    return IP_EDEVICE;
  }
  memset(ctx->ctr_host, 0, sizeof(Counters));
  if (ip_noalloc_setup(ctx) != IP_OK) {
    (void)hipFree(ctx->ctr_dev);
    (void)hipHostFree(ctx->ctr_host);
    (void)hipEventDestroy(ctx->ev0);
    (void)hipEventDestroy(ctx->ev1);
    delete ctx;
    return IP_EDEVICE;
  }
  {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
      (void)hipGetLastError();
      tot = 64ull << 30;
    }
    // idle blocks kept for reuse: up to half the device (a serving slot
    // gets its share of the server's pool instead)
    ctx->cache.limit = tot / 2;
  }
  *out = ctx;
  return IP_OK;
}

void ip_destroy(ip_ctx *ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  DevBuf *bufs[] = {&ctx->vtf.keys, &ctx->vtf.eval, &ctx->vtf.vals, &ctx->vtf.fb, &ctx->vtc.keys,
                    &ctx->vtc.eval, &ctx->vtc.vals, &ctx->vtc.fb, &ctx->vt_aux, &ctx->scratch, &ctx->scene};
  for (DevBuf *b : bufs)
    if (b->p) ip_dfree(ctx, b->p);
  ip_cache_release(ctx);
  for (auto &kv : ctx->cache.size_of) (void)hipFree(kv.first);  // blocks never returned
  if (ctx->ctr_dev) (void)hipFree(ctx->ctr_dev);
  if (ctx->ctr_host) (void)hipHostFree(ctx->ctr_host);
  if (ctx->host_stage) (void)hipHostFree(ctx->host_stage);
  for (void *q : ctx->dev_stage)
    if (q) (void)hipFree(q);
  if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
  if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
  delete ctx;
}

const char *ip_last_error(const ip_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int ip_problem_create(ip_ctx *ctx, const ip_fparams *f, const ip_space *sp, const double *seeds, int64_t n_seeds,
                      int32_t coarse_k, ip_problem **out) {
  if (!ctx) return IP_EINVAL;
  if (!out) return ip_fail(ctx, IP_EINVAL, "null output handle");
  *out = nullptr;
  if (!f || !sp || (!seeds && n_seeds > 0)) return ip_fail(ctx, IP_EINVAL, "null argument");
  const int d = f->d;
  if (d < 2 || d > IP_MAX_D || sp->d != d) return ip_fail(ctx, IP_EINVAL, "dimension must be 2..7 and match");
  if (f->kernel != IP_KERNEL_POLY && f->kernel != IP_KERNEL_RBF) return ip_fail(ctx, IP_EINVAL, "unknown kernel");
  if (f->kernel == IP_KERNEL_POLY && (f->degree < 1 || f->degree > 64))
    return ip_fail(ctx, IP_EINVAL, "degree must be 1..64");
  if (f->kernel == IP_KERNEL_RBF && !(f->gamma > 0.0)) return ip_fail(ctx, IP_EINVAL, "RBF gamma must be positive");
  if (f->n_sv < 1 || !f->sv || !f->alpha) return ip_fail(ctx, IP_EINVAL, "need at least one support vector");
  if (coarse_k < 1 || coarse_k > 64) return ip_fail(ctx, IP_EINVAL, "coarse_k must be 1..64");
  if (n_seeds < 1) return ip_fail(ctx, IP_EINVAL, "need at least one seed");
  if (!sp->M || !sp->Minv || !sp->offset || !sp->lo || !sp->hi) return ip_fail(ctx, IP_EINVAL, "null frame");
  if (!finite_all(f->sv, f->n_sv * d) || !finite_all(f->alpha, f->n_sv) || !std::isfinite(f->gamma) ||
      !std::isfinite(f->coef0) || !std::isfinite(f->bias) || !finite_all(sp->M, d * d) ||
      !finite_all(sp->Minv, d * d) || !finite_all(sp->offset, d) || !finite_all(sp->lo, d) ||
      !finite_all(sp->hi, d) || !finite_all(seeds, n_seeds * d))
    return ip_fail(ctx, IP_EINVAL, "non-finite input");
  for (int j = 0; j < d; ++j)
    if (!(sp->lo[j] <= sp->hi[j])) return ip_fail(ctx, IP_EINVAL, "empty domain box");
  IP_TRY_HIP(ctx, hipSetDevice(ctx->device));
  ip_problem *p = new (std::nothrow) ip_problem();
  if (!p) return ip_fail(ctx, IP_ENOMEM, "host allocation failed");
  p->ctx = ctx;
  p->d = d;
  p->k = coarse_k;
  int rc = build_lattice(ctx, sp, 1, &p->fine);
  if (rc == IP_OK) rc = build_lattice(ctx, sp, coarse_k, &p->coarse);
  p->probe_k = coarse_k >= 2 ? coarse_k : 4;
  if (rc == IP_OK) rc = build_lattice(ctx, sp, p->probe_k, &p->probe);
  if (rc != IP_OK) {
    delete p;
    return rc;
  }
  // support-vector records: s_0..s_{d-1}, alpha, padding (64 bytes)
  const int64_t S = f->n_sv;
  std::vector<double> rec((size_t)S * 8, 0.0);
  for (int64_t i = 0; i < S; ++i) {
    for (int j = 0; j < d; ++j) rec[i * 8 + j] = f->sv[i * d + j];
    rec[i * 8 + d] = f->alpha[i];
  }
  hipError_t e = hipMalloc((void **)&p->rec_dev, rec.size() * 8);
  if (e == hipSuccess) e = hipMalloc((void **)&p->seeds_dev, (size_t)n_seeds * d * 8);
  if (e == hipSuccess) e = hipMemcpyAsync(p->rec_dev, rec.data(), rec.size() * 8, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(p->seeds_dev, seeds, (size_t)n_seeds * d * 8, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) {
    int r = ip_hip(ctx, e, "ip_problem_create upload");
    ip_problem_free(p);
    return r;
  }
  p->n_seeds = n_seeds;
  p->f.rec = p->rec_dev;
  p->f.S = S;
  p->f.p = f->kernel == IP_KERNEL_POLY ? f->degree : 1;
  p->f.kernel = f->kernel;
  p->f.gamma = f->gamma;
  p->f.coef0 = f->coef0;
  p->f.bias = f->bias;
  rc = build_poly(ctx, p, f, sp);
  if (rc == IP_OK) rc = build_rbf(ctx, p, f);
  if (rc != IP_OK) {
    ip_problem_free(p);
    return rc;
  }
  *out = p;
  return IP_OK;
}

void ip_problem_free(ip_problem *p) {
  if (!p) return;
  if (p->ctx) (void)hipStreamSynchronize(p->ctx->stream);
  if (p->rec_dev) (void)hipFree(p->rec_dev);
  if (p->seeds_dev) (void)hipFree(p->seeds_dev);
  if (p->poly_dev) (void)hipFree(p->poly_dev);
  if (p->rbf_dev) (void)hipFree(p->rbf_dev);
  delete p;
}

int ip_trace_check_batches(ip_ctx *ctx, const ip_problem *p, uint64_t batch_budget_bytes, int32_t precision,
                           uint32_t flags, const ip_scene *scene, ip_batch_fn fn, void *user,
                           ip_batch_summary *out) {
  if (!ctx) return IP_EINVAL;
  if (!out || !p || !scene) return ip_fail(ctx, IP_EINVAL, "null argument");
  memset(out, 0, sizeof(*out));
  if (p->ctx != ctx) return ip_fail(ctx, IP_EINVAL, "problem belongs to another context");
  if (precision != IP_FP64 && precision != IP_FP32_CERTIFY) return ip_fail(ctx, IP_EINVAL, "unknown precision");
  if (p->k < 2) return ip_fail(ctx, IP_EINVAL, "per-batch tracing needs batch triangulation (coarse_k >= 2)");
  if (scene->n_joints != p->d) return ip_fail(ctx, IP_EINVAL, "scene joints must equal the dimension");
  IP_TRY_HIP(ctx, hipSetDevice(ctx->device));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  IP_TRY_HIP(ctx, hipEventCreate(&e0));
  hipError_t e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    (void)hipEventDestroy(e0);
    return ip_hip(ctx, e, "hipEventCreate");
  }
  const int64_t nm0 = ctx->n_hip_malloc, bm0 = ctx->hip_malloc_bytes;
  e = hipEventRecord(e0, ctx->stream);
  int rc = e == hipSuccess ? ip_trace_batches_impl(ctx, p, batch_budget_bytes, precision, flags, scene, fn, user, out)
                           : ip_hip(ctx, e, "hipEventRecord");
  out->stats.n_hip_malloc = ctx->n_hip_malloc - nm0;
  out->stats.hip_malloc_bytes = ctx->hip_malloc_bytes - bm0;
  if (rc == IP_OK) {
    e = hipEventRecord(e1, ctx->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) rc = ip_hip(ctx, e, "ip_trace_check_batches timing");
    out->stats.ms_total = ms;
  } else {
    (void)hipStreamSynchronize(ctx->stream);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return rc;
}

int ip_trace(ip_ctx *ctx, const ip_problem *p, uint64_t batch_budget_bytes, int32_t precision, uint32_t flags,
             ip_cells **out) {
  if (!ctx) return IP_EINVAL;
  if (!out || !p) return ip_fail(ctx, IP_EINVAL, "null argument");
  *out = nullptr;
  if (p->ctx != ctx) return ip_fail(ctx, IP_EINVAL, "problem belongs to another context");
  if (precision != IP_FP64 && precision != IP_FP32_CERTIFY) return ip_fail(ctx, IP_EINVAL, "unknown precision");
  IP_TRY_HIP(ctx, hipSetDevice(ctx->device));
  ip_cells *c = new (std::nothrow) ip_cells();
  if (!c) return ip_fail(ctx, IP_ENOMEM, "host allocation failed");
  c->ctx = ctx;
  IP_TRY_HIP(ctx, hipEventRecord(ctx->ev0, ctx->stream));
  const int64_t nm0 = ctx->n_hip_malloc, bm0 = ctx->hip_malloc_bytes;
  int rc = ip_trace_impl(ctx, p, batch_budget_bytes, precision, flags, c);
  c->st.n_hip_malloc = ctx->n_hip_malloc - nm0;
  c->st.hip_malloc_bytes = ctx->hip_malloc_bytes - bm0;
  if (rc == IP_OK) {
    hipError_t e = hipEventRecord(ctx->ev1, ctx->stream);
    if (e == hipSuccess) e = hipEventSynchronize(ctx->ev1);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1);
    if (e != hipSuccess) rc = ip_hip(ctx, e, "ip_trace timing");
    c->st.ms_total = ms;
  }
  if (rc != IP_OK) {
    ip_cells_free(c);
    return rc;
  }
  *out = c;
  return IP_OK;
}

int64_t ip_cells_count(const ip_cells *c) { return c ? c->n : -1; }

int ip_cells_stats(const ip_cells *c, ip_stats *out) {
  if (!c || !out) return IP_EINVAL;
  *out = c->st;
  return IP_OK;
}

int ip_cells_download(ip_ctx *ctx, const ip_cells *c, int32_t *v, uint32_t *mask, double *pts) {
  if (!ctx && c) ctx = c->ctx;
  if (!ctx) return IP_EINVAL;
  if (!c) return ip_fail(ctx, IP_EINVAL, "null cells");
  const int64_t n = c->n;
  const int d = c->d;
  if (n == 0) return IP_OK;
  if (v || mask) {
    std::vector<uint64_t> keys((size_t)n);
    IP_TRY_HIP(ctx, hipMemcpyAsync(keys.data(), c->keys, (size_t)n * 8, hipMemcpyDeviceToHost, ctx->stream));
    IP_TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));
    const uint64_t m = (1ull << c->B) - 1ull;
    for (int64_t i = 0; i < n; ++i) {
      uint64_t k = keys[i] & ~IP_SIGN_BIT;
      if (v)
        for (int j = 0; j < d; ++j) v[i * d + j] = (int32_t)((k >> (j * c->B)) & m) + c->vmin[j];
      if (mask) mask[i] = (uint32_t)(k >> (d * c->B)) & ((1u << d) - 1u);
    }
  }
  if (pts) {
    std::vector<double> soa((size_t)n * d);
    for (int j = 0; j < d; ++j)
      IP_TRY_HIP(ctx, hipMemcpyAsync(soa.data() + (size_t)j * n, c->pts + (size_t)j * c->ld, (size_t)n * 8,
                                     hipMemcpyDeviceToHost, ctx->stream));
    IP_TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));
    for (int64_t i = 0; i < n; ++i)
      for (int j = 0; j < d; ++j) pts[i * d + j] = soa[(size_t)j * n + i];
  }
  return IP_OK;
}

int ip_cells_points(const ip_cells *c, const double **pts_dev, int64_t *ld) {
  if (!c || !pts_dev || !ld) return IP_EINVAL;
  *pts_dev = c->pts;
  *ld = c->ld;
  return IP_OK;
}

namespace {

// Order-independent digest of the traced edge keys: (sum, xor) of the
// SplitMix64-finalized keys.
__global__ void digest_kernel(const uint64_t *keys, int64_t n, unsigned long long *sum, unsigned long long *x) {
  unsigned long long s = 0, q = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t h = mix64(keys[i]);
    s += h;
    q ^= h;
  }
  for (int off = 32; off; off >>= 1) {
    s += __shfl_xor(s, off, 64);
    q ^= __shfl_xor(q, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    atomicAdd(sum, s);
    atomicXor(x, q);
  }
}

// Rows idx[0 .. n) of the cells: keys, points (row-major n x d), verdicts.
__global__ void gather_kernel(const uint64_t *keys, const double *pts, int64_t ld, const uint8_t *verdict,
                              const int64_t *idx, int64_t n, int d, uint64_t *okeys, double *opts, uint8_t *over) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx[r];
    okeys[r] = keys[i];
    for (int j = 0; j < d; ++j) opts[r * d + j] = pts[(int64_t)j * ld + i];
    if (verdict) over[r] = verdict[i];
  }
}

// Rows [0, n) of a column-major point array (column j at soa + j ld) into
// row-major order, one output double per lane, so the stores coalesce.
__global__ void interleave_kernel(const double *soa, int64_t ld, int64_t n, int d, double *aos) {
  const int64_t total = n * d;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / d;
    const int j = (int)(i - r * d);
    aos[i] = soa[(int64_t)j * ld + r];
  }
}

}  // namespace

extern "C++" int ip_digest_accumulate(ip_ctx *ctx, const uint64_t *keys, int64_t n, unsigned long long *acc) {
  if (n <= 0) return IP_OK;
  hipLaunchKernelGGL(digest_kernel, dim3(1024), dim3(256), 0, ctx->stream, keys, n, acc, acc + 1);
  IP_TRY_HIP(ctx, hipGetLastError());
  return IP_OK;
}

extern "C++" int ip_interleave_free(ip_ctx *ctx, const ip_cells *c, double *out_dev) {
  const int64_t nf = c->n_free;
  if (nf <= 0) return IP_OK;
  const int64_t total = nf * c->d;
  hipLaunchKernelGGL(interleave_kernel, dim3((unsigned)std::min<int64_t>((total + 255) / 256, 8192)), dim3(256), 0,
                     ctx->stream, (const double *)c->free_pts, c->n, nf, c->d, out_dev);
  IP_TRY_HIP(ctx, hipGetLastError());
  return IP_OK;
}

extern "C++" int ip_free_points_to_host(ip_ctx *ctx, const ip_cells *c, double *host) {
  const int64_t nf = c->n_free;
  if (nf <= 0) return IP_OK;
  void *buf = nullptr;
  IP_TRY(ip_dalloc(ctx, &buf, (size_t)nf * c->d * 8));
  const int64_t total = nf * c->d;
  int rc = ip_interleave_free(ctx, c, (double *)buf);
  if (rc == IP_OK) {
    hipError_t e = hipMemcpyAsync(host, buf, (size_t)total * 8, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) rc = ip_hip(ctx, e, "free points to host");
  }
  if (rc != IP_OK) (void)hipStreamSynchronize(ctx->stream);
  ip_dfree(ctx, buf);
  return rc;
}

int ip_cells_digest(ip_ctx *ctx, const ip_cells *c, uint64_t digest[2]) {
  if (!ctx && c) ctx = c->ctx;
  if (!ctx) return IP_EINVAL;
  if (!c || !digest) return ip_fail(ctx, IP_EINVAL, "null argument");
  IP_TRY_HIP(ctx, hipSetDevice(ctx->device));
  IP_TRY_HIP(ctx, hipMemsetAsync(ctx->ctr_dev, 0, sizeof(Counters), ctx->stream));
  if (c->n > 0) {
    hipLaunchKernelGGL(digest_kernel, dim3(1024), dim3(256), 0, ctx->stream, (const uint64_t *)c->keys, c->n,
                       &ctx->ctr_dev->n_eval, &ctx->ctr_dev->n_aux);
    IP_TRY_HIP(ctx, hipGetLastError());
  }
  IP_TRY_HIP(ctx, hipMemcpyAsync(ctx->ctr_host, ctx->ctr_dev, sizeof(Counters), hipMemcpyDeviceToHost, ctx->stream));
  IP_TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));
  digest[0] = ctx->ctr_host->n_eval;
  digest[1] = ctx->ctr_host->n_aux;
  return IP_OK;
}

int ip_cells_gather(ip_ctx *ctx, const ip_cells *c, const int64_t *idx, int64_t n, int32_t *v, uint32_t *mask,
                    double *pts, uint8_t *verdict) {
  if (!ctx && c) ctx = c->ctx;
  if (!ctx) return IP_EINVAL;
  if (!c || n < 0 || (n > 0 && !idx)) return ip_fail(ctx, IP_EINVAL, "ip_cells_gather: bad arguments");
  if (verdict && !c->verdict) return ip_fail(ctx, IP_EINVAL, "cells have not been checked");
  for (int64_t r = 0; r < n; ++r)
    if (idx[r] < 0 || idx[r] >= c->n) return ip_fail(ctx, IP_EINVAL, "ip_cells_gather: index out of range");
  if (n == 0) return IP_OK;
  IP_TRY_HIP(ctx, hipSetDevice(ctx->device));
  const int d = c->d;
  const size_t bytes = (size_t)n * (8 + 8 + 8 * (size_t)d + 1);
  void *buf = nullptr;
  IP_TRY(ip_dalloc(ctx, &buf, bytes));
  int64_t *didx = (int64_t *)buf;
  uint64_t *dkeys = (uint64_t *)(didx + n);
  double *dpts = (double *)(dkeys + n);
  uint8_t *dver = (uint8_t *)(dpts + (size_t)n * d);
  std::vector<uint64_t> keys((size_t)n);
  std::vector<uint8_t> ver(verdict ? (size_t)n : 0);
  hipError_t e = hipMemcpyAsync(didx, idx, (size_t)n * 8, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(gather_kernel, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 4096)), dim3(256), 0,
                       ctx->stream, (const uint64_t *)c->keys, (const double *)c->pts, c->ld,
                       (const uint8_t *)(verdict ? c->verdict : nullptr), (const int64_t *)didx, n, d, dkeys, dpts,
                       dver);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(keys.data(), dkeys, (size_t)n * 8, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess && pts)
    e = hipMemcpyAsync(pts, dpts, (size_t)n * d * 8, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess && verdict) e = hipMemcpyAsync(verdict, dver, (size_t)n, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  ip_dfree(ctx, buf);
  if (e != hipSuccess) return ip_hip(ctx, e, "ip_cells_gather");
  const uint64_t m = (1ull << c->B) - 1ull;
  for (int64_t r = 0; r < n; ++r) {
    const uint64_t k = keys[(size_t)r] & ~IP_SIGN_BIT;
    if (v)
      for (int j = 0; j < d; ++j) v[r * d + j] = (int32_t)((k >> (j * c->B)) & m) + c->vmin[j];
    if (mask) mask[r] = (uint32_t)(k >> (d * c->B)) & ((1u << d) - 1u);
  }
  return IP_OK;
}

void ip_cells_free(ip_cells *c) {
  if (!c) return;
  if (c->ctx) {
    (void)hipStreamSynchronize(c->ctx->stream);
    ip_dfree(c->ctx, c->keys);
    ip_dfree(c->ctx, c->pts);
    ip_dfree(c->ctx, c->verdict);
    ip_dfree(c->ctx, c->free_pts);
  }
  delete c;
}

int ip_check(ip_ctx *ctx, const ip_scene *scene, const double *q_dev, int64_t n, int64_t ld, uint8_t *verdict_dev) {
  if (!ctx) return IP_EINVAL;
  if (!scene || (n > 0 && (!q_dev || !verdict_dev)) || n < 0 || ld < n)
    return ip_fail(ctx, IP_EINVAL, "ip_check: bad arguments");
  IP_TRY_HIP(ctx, hipSetDevice(ctx->device));
  return ip_check_impl(ctx, scene, q_dev, n, ld, verdict_dev);
}

int ip_check_cells(ip_ctx *ctx, ip_cells *c, const ip_scene *scene, int64_t *n_free) {
  if (!ctx) return IP_EINVAL;
  if (!c || !scene) return ip_fail(ctx, IP_EINVAL, "null argument");
  if (scene->n_joints != c->d) return ip_fail(ctx, IP_EINVAL, "scene joints must equal the dimension");
  IP_TRY_HIP(ctx, hipSetDevice(ctx->device));
  if (!c->verdict) IP_TRY(ip_dalloc(ctx, (void **)&c->verdict, (size_t)(c->n ? c->n : 1)));
  IP_TRY(ip_check_gather_impl(ctx, scene, c));
  if (n_free) *n_free = c->n_free;
  return IP_OK;
}

int ip_cells_download_check(ip_ctx *ctx, const ip_cells *c, uint8_t *verdict, double *free_pts) {
  if (!ctx && c) ctx = c->ctx;
  if (!ctx) return IP_EINVAL;
  if (!c || !c->verdict) return ip_fail(ctx, IP_EINVAL, "cells have not been checked");
  IP_TRY_HIP(ctx, hipSetDevice(ctx->device));
  if (verdict && c->n)
    IP_TRY_HIP(ctx, hipMemcpyAsync(verdict, c->verdict, (size_t)c->n, hipMemcpyDeviceToHost, ctx->stream));
  if (free_pts) IP_TRY(ip_free_points_to_host(ctx, c, free_pts));
  IP_TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return IP_OK;
}

int ip_cells_download_free(ip_ctx *ctx, const ip_cells *c, double *free_soa) {
  if (!ctx && c) ctx = c->ctx;
  if (!ctx) return IP_EINVAL;
  if (!c || !c->verdict || (c->n_free > 0 && !free_soa))
    return ip_fail(ctx, IP_EINVAL, "ip_cells_download_free: cells have not been checked");
  for (int j = 0; j < c->d && c->n_free > 0; ++j)
    IP_TRY_HIP(ctx, hipMemcpyAsync(free_soa + (size_t)j * c->n_free, c->free_pts + (size_t)j * c->n,
                                   (size_t)c->n_free * 8, hipMemcpyDeviceToHost, ctx->stream));
  IP_TRY_HIP(ctx, hipStreamSynchronize(ctx->stream));
  return IP_OK;
}

int ip_feval(ip_ctx *ctx, const ip_problem *p, const int32_t *v_dev, int64_t n, int32_t precision, double *f_dev,
             double *bound_dev) {
  if (!ctx) return IP_EINVAL;
  if (!p || (n > 0 && (!v_dev || !f_dev)) || n < 0) return ip_fail(ctx, IP_EINVAL, "ip_feval: bad arguments");
  IP_TRY_HIP(ctx, hipSetDevice(ctx->device));
  if (n == 0) return IP_OK;
  return ip_feval_impl(ctx, p, v_dev, n, precision, f_dev, bound_dev);
}

int ip_region_eval(ip_ctx *ctx, const ip_problem *p, const int32_t *simplex_dev, int64_t n, int32_t *y_dev,
                   double *f_dev, double *bound_dev, int32_t *n_points) {
  if (!ctx) return IP_EINVAL;
  if (!p || !n_points || n < 0 || (n > 0 && y_dev && (!simplex_dev || !f_dev || !bound_dev)))
    return ip_fail(ctx, IP_EINVAL, "ip_region_eval: bad arguments");
  if (p->ctx != ctx) return ip_fail(ctx, IP_EINVAL, "problem belongs to another context");
  if (!p->poly.ok) return ip_fail(ctx, IP_EINVAL, "ip_region_eval: no FP32 form for this degree");
  IP_TRY_HIP(ctx, hipSetDevice(ctx->device));
  return ip_region_eval_impl(ctx, p, simplex_dev, n, y_dev, f_dev, bound_dev, n_points);
}

int ip_seed_search(ip_ctx *ctx, const ip_problem *p, const double *q0_dev, int64_t n, int32_t iters, double *q_dev,
                   double *f_dev) {
  if (!ctx) return IP_EINVAL;
  if (!p || n < 0 || iters < 0 || iters > 1000 || (n > 0 && (!q0_dev || !q_dev || !f_dev)))
    return ip_fail(ctx, IP_EINVAL, "ip_seed_search: bad arguments");
  if (p->ctx != ctx) return ip_fail(ctx, IP_EINVAL, "problem belongs to another context");
  IP_TRY_HIP(ctx, hipSetDevice(ctx->device));
  if (n == 0) return IP_OK;
  return ip_seed_search_impl(ctx, p, q0_dev, n, iters, q_dev, f_dev);
}

int ip_problem_set_seeds(ip_ctx *ctx, ip_problem *p, const double *seeds, int64_t n_seeds) {
  if (!ctx) return IP_EINVAL;
  if (!p || n_seeds < 1 || !seeds) return ip_fail(ctx, IP_EINVAL, "ip_problem_set_seeds: need at least one seed");
  if (p->ctx != ctx) return ip_fail(ctx, IP_EINVAL, "problem belongs to another context");
  if (!finite_all(seeds, n_seeds * p->d)) return ip_fail(ctx, IP_EINVAL, "non-finite seed");
  IP_TRY_HIP(ctx, hipSetDevice(ctx->device));
  double *nd = nullptr;
  IP_TRY_HIP(ctx, hipMalloc((void **)&nd, (size_t)n_seeds * p->d * 8));
  hipError_t e = hipMemcpyAsync(nd, seeds, (size_t)n_seeds * p->d * 8, hipMemcpyHostToDevice, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) {
    (void)hipFree(nd);
    return ip_hip(ctx, e, "ip_problem_set_seeds");
  }
  if (p->seeds_dev) (void)hipFree(p->seeds_dev);
  p->seeds_dev = nd;
  p->n_seeds = n_seeds;
  return IP_OK;
}

int ip_cells_key_layout(const ip_cells *c, int32_t *bits, int32_t *vmin) {
  if (!c || !bits || !vmin) return IP_EINVAL;
  *bits = c->B;
  for (int j = 0; j < c->d; ++j) vmin[j] = c->vmin[j];
  return IP_OK;
}

int ip_feval_noalloc(ip_ctx *ctx, const ip_problem *p, const int32_t *v_dev, int64_t n, int32_t precision,
                     double *f_dev, double *bound_dev) {
  if (!ctx) return IP_EINVAL;
  if (!p || (n > 0 && (!v_dev || !f_dev)) || n < 0) return ip_fail(ctx, IP_EINVAL, "ip_feval_noalloc: bad arguments");
  if (p->ctx != ctx) return ip_fail(ctx, IP_EINVAL, "problem belongs to another context");
  if (precision != IP_FP64 && precision != IP_FP32_CERTIFY) return ip_fail(ctx, IP_EINVAL, "unknown precision");
  if (n > IP_NOALLOC_MAX_VERTICES)
    return ip_fail(ctx, IP_EINVAL, "ip_feval_noalloc: at most " + std::to_string(IP_NOALLOC_MAX_VERTICES) +
                                       " vertices per call (the size of its device scratch)");
  IP_TRY_HIP(ctx, hipSetDevice(ctx->device));
  if (n == 0) return IP_OK;
  return ip_feval_noalloc_impl(ctx, p, v_dev, n, precision, f_dev, bound_dev);
}

}  // extern "C"
