// Serving loop (include/ip.h, ip_server_*): a queue of proof requests, slots
// that each own a context (HIP stream + workspace) and a host thread, and
// admission in two steps: a request takes the next free slot and projects
// its device bytes there (a trace on a coarsened lattice), then starts its
// trace once the projection fits the pool beside the traces already
// running.  Requests on different slots run on different streams, so their
// kernels overlap on the device; a request joins as soon as a slot and
// memory are free, not when a whole batch of requests finishes.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstddef>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <type_traits>
#include <vector>

#include "ip_internal.h"

namespace {

// Deep copy of a request's host inputs.
struct OwnedRequest {
  ip_fparams f;
  ip_space sp;
  ip_scene sc;
  bool has_scene = false;
  std::vector<double> sv, alpha, M, Minv, off, lo, hi, seeds;
  std::vector<double> jT, lsc, lsr, lp0, lp1, lcr, osc, osr, obT, obl, ocT, ocrh;
  std::vector<int32_t> jax, lsl, lcl;
  int64_t n_seeds = 0;
  int32_t k = 1, prec = IP_FP64;
  uint64_t budget = 0, bytes = 0;
  uint32_t flags = 0;
};

template <typename T>
std::vector<T> cp(const T *p, int64_t n) {
  return (p && n > 0) ? std::vector<T>(p, p + n) : std::vector<T>();
}

void own(const ip_request *r, OwnedRequest &o) {
  const int d = r->f->d;
  o.sv = cp(r->f->sv, r->f->n_sv * d);
  o.alpha = cp(r->f->alpha, r->f->n_sv);
  o.f = *r->f;
  o.f.sv = o.sv.data();
  o.f.alpha = o.alpha.data();
  o.M = cp(r->sp->M, d * d);
  o.Minv = cp(r->sp->Minv, d * d);
  o.off = cp(r->sp->offset, d);
  o.lo = cp(r->sp->lo, d);
  o.hi = cp(r->sp->hi, d);
  o.sp = {d, o.M.data(), o.Minv.data(), o.off.data(), o.lo.data(), o.hi.data()};
  o.n_seeds = r->n_seeds;
  o.seeds = cp(r->seeds, r->n_seeds * d);
  o.k = r->coarse_k;
  o.prec = r->precision;
  o.budget = r->batch_budget;
  o.flags = r->flags;
  if (r->scene) {
    const ip_scene *s = r->scene;
    o.has_scene = true;
    o.jT = cp(s->joint_T, 12 * (int64_t)s->n_joints);
    o.jax = cp(s->joint_axis, s->n_joints);
    o.lsl = cp(s->lsph_link, s->n_lsph);
    o.lsc = cp(s->lsph_c, 3 * (int64_t)s->n_lsph);
    o.lsr = cp(s->lsph_r, s->n_lsph);
    o.lcl = cp(s->lcap_link, s->n_lcap);
    o.lp0 = cp(s->lcap_p0, 3 * (int64_t)s->n_lcap);
    o.lp1 = cp(s->lcap_p1, 3 * (int64_t)s->n_lcap);
    o.lcr = cp(s->lcap_r, s->n_lcap);
    o.osc = cp(s->osph_c, 3 * (int64_t)s->n_osph);
    o.osr = cp(s->osph_r, s->n_osph);
    o.obT = cp(s->obox_T, 12 * (int64_t)s->n_obox);
    o.obl = cp(s->obox_l, 3 * (int64_t)s->n_obox);
    o.ocT = cp(s->ocyl_T, 12 * (int64_t)s->n_ocyl);
    o.ocrh = cp(s->ocyl_rh, 2 * (int64_t)s->n_ocyl);
    o.sc = {s->n_joints, o.jT.data(), o.jax.data(), s->n_lsph, o.lsl.data(), o.lsc.data(), o.lsr.data(),
            s->n_lcap, o.lcl.data(), o.lp0.data(), o.lp1.data(), o.lcr.data(), s->n_osph, o.osc.data(),
            o.osr.data(), s->n_obox, o.obT.data(), o.obl.data(), s->n_ocyl, o.ocT.data(), o.ocrh.data()};
  }
}

struct Job {
  OwnedRequest req;
  ip_result *res = nullptr;
  bool done = false;
};

// Page-locked host blocks for the C_free points of results: the device
// copies into them at the link's rate, with no page faults on the host, and
// ip_result_free returns them here.  Idle blocks are kept up to `limit`
// bytes (the largest go first beyond it).
struct PinnedPool {
  std::mutex mu;
  std::multimap<size_t, void *> idle;
  size_t idle_bytes = 0, limit = 1ull << 30;

  void *get(size_t bytes, size_t *cap) {
    const size_t gran = 2ull << 20;
    const size_t want = (bytes + gran - 1) / gran * gran;
    {
      std::lock_guard<std::mutex> lk(mu);
      auto it = idle.lower_bound(want);
      if (it != idle.end() && it->first <= 2 * want) {
        void *p = it->second;
        *cap = it->first;
        idle_bytes -= it->first;
        idle.erase(it);
        return p;
      }
    }
    void *p = nullptr;
    if (hipHostMalloc(&p, want, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    *cap = want;
    return p;
  }
  void put(void *p, size_t cap) {
    std::vector<void *> drop;
    {
      std::lock_guard<std::mutex> lk(mu);
      idle.emplace(cap, p);
      idle_bytes += cap;
      while (idle_bytes > limit && !idle.empty()) {
        auto last = std::prev(idle.end());
        drop.push_back(last->second);
        idle_bytes -= last->first;
        idle.erase(last);
      }
    }
    for (void *q : drop) (void)hipHostFree(q);
  }
  ~PinnedPool() {
    for (auto &kv : idle) (void)hipHostFree(kv.second);
  }
};

// A result with where its free points came from; ip_result_free gets the
// public part, the first member.
struct ResultBox {
  ip_result r;
  PinnedPool *pool = nullptr;  // free_pts from this pool (else new[])
  size_t cap = 0;
};
static_assert(std::is_standard_layout<ResultBox>::value && offsetof(ResultBox, r) == 0,
              "ip_result must be the first member of its box");

}  // namespace

struct ip_server {
  int device = 0;
  uint64_t pool = 0;
  std::vector<ip_ctx *> ctxs;
  std::vector<hipStream_t> streams;
  std::vector<std::thread> workers;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<uint64_t> queue;
  std::map<uint64_t, std::unique_ptr<Job>> jobs;
  uint64_t next_id = 1;
  uint64_t in_use = 0;   // admitted bytes of the requests tracing now
  int tracing = 0;
  std::condition_variable cv_mem;
  bool stop = false;
  std::chrono::steady_clock::time_point t0;
  PinnedPool pinned;

  double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }

  // Waits until `bytes` fits the pool beside the traces running (or nothing
  // traces), then books them.
  void admit(uint64_t bytes, ip_result *r) {
    std::unique_lock<std::mutex> lk(mu);
    cv_mem.wait(lk, [&] { return stop || tracing == 0 || in_use + bytes <= pool; });
    in_use += bytes;
    ++tracing;
    r->t_admit = now();
  }
  void release_bytes(uint64_t bytes) {
    {
      std::lock_guard<std::mutex> lk(mu);
      in_use -= bytes;
      --tracing;
    }
    cv_mem.notify_all();
  }

  void run_job(ip_ctx *ctx, Job &job) {
    ip_result *r = job.res;
    OwnedRequest &q = job.req;
    r->d = q.f.d;
    ip_problem *p = nullptr;
    ip_cells *c = nullptr;
    int rc = ip_problem_create(ctx, &q.f, &q.sp, q.seeds.data(), q.n_seeds, q.k, &p);
    uint64_t bytes = q.bytes;
    if (rc == IP_OK && bytes == 0) rc = ip_project_impl(ctx, p, &bytes, &r->n_probe_edges);
    bool admitted = false;
    if (rc == IP_OK) {
      r->admitted_bytes = bytes;
      admit(bytes, r);
      admitted = true;
    }
    if (rc == IP_OK) rc = ip_trace(ctx, p, q.budget, q.prec, q.flags & ~(uint32_t)IP_KEEP_CELLS, &c);
    if (rc == IP_OK && q.has_scene) rc = ip_check_cells(ctx, c, &q.sc, &r->n_free);
    if (rc == IP_OK) {
      uint64_t dg[2] = {0, 0};
      rc = ip_cells_digest(ctx, c, dg);
      r->digest[0] = dg[0];
      r->digest[1] = dg[1];
    }
    if (rc == IP_OK) {
      r->n_cells = c->n;
      ip_cells_stats(c, &r->stats);
      if (q.has_scene && r->n_free > 0) {
        ResultBox *box = reinterpret_cast<ResultBox *>(r);
        const size_t bytes = (size_t)r->n_free * q.f.d * sizeof(double);
        r->free_pts = (double *)pinned.get(bytes, &box->cap);
        if (r->free_pts)
          box->pool = &pinned;
        else
          r->free_pts = new (std::nothrow) double[(size_t)r->n_free * q.f.d];
        if (!r->free_pts)
          rc = ip_fail(ctx, IP_ENOMEM, "host allocation failed");
        else
          rc = ip_free_points_to_host(ctx, c, r->free_pts);
      }
    }
    if (rc == IP_OK && (q.flags & IP_KEEP_CELLS)) {
      r->cells = c;
      c = nullptr;
    }
    if (rc != IP_OK) snprintf(r->error, sizeof(r->error), "%s", ip_last_error(ctx));
    r->status = rc;
    if (c) ip_cells_free(c);
    if (p) ip_problem_free(p);
    r->t_done = now();
    if (admitted) release_bytes(bytes);
  }

  void worker(int slot) {
    ip_ctx *ctx = ctxs[slot];
    (void)hipSetDevice(device);
    for (;;) {
      uint64_t id = 0;
      Job *job = nullptr;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv_work.wait(lk, [&] { return stop || !queue.empty(); });
        if (stop) return;
        id = queue.front();
        queue.pop_front();
        job = jobs[id].get();
        job->res->t_start = now();
      }
      run_job(ctx, *job);
      {
        std::lock_guard<std::mutex> lk(mu);
        job->done = true;
      }
      cv_done.notify_all();
      cv_work.notify_all();
    }
  }
};

extern "C" {

int ip_server_create(ip_server **out, int device, uint64_t pool_bytes, int32_t max_slots) {
  if (!out) return IP_EINVAL;
  *out = nullptr;
  if (max_slots < 1 || max_slots > 64) return IP_EINVAL;
  ip_server *s = new (std::nothrow) ip_server();
  if (!s) return IP_ENOMEM;
  s->device = device;
  s->pool = pool_bytes ? pool_bytes : (64ull << 30);
  s->t0 = std::chrono::steady_clock::now();
  if (hipSetDevice(device) != hipSuccess) {
    delete s;
    return IP_EDEVICE;
  }
  for (int i = 0; i < max_slots; ++i) {
    hipStream_t st = nullptr;
    ip_ctx *c = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess || ip_create(&c, device, st) != IP_OK) {
      if (st) (void)hipStreamDestroy(st);
      ip_server_destroy(s);
      return IP_EDEVICE;
    }
    s->streams.push_back(st);
    s->ctxs.push_back(c);
    // the slots' idle caches together stay within the pool
    c->cache.limit = s->pool / (uint64_t)max_slots;
  }
  for (int i = 0; i < max_slots; ++i) s->workers.emplace_back([s, i] { s->worker(i); });
  *out = s;
  return IP_OK;
}

int ip_server_submit(ip_server *s, const ip_request *req, uint64_t *id) {
  if (!s || !req || !id || !req->f || !req->sp || !req->seeds || req->n_seeds < 1) return IP_EINVAL;
  if (req->f->d < 2 || req->f->d > IP_MAX_D || req->sp->d != req->f->d) return IP_EINVAL;
  if (req->scene && req->scene->n_joints != req->f->d) return IP_EINVAL;
  auto job = std::unique_ptr<Job>(new (std::nothrow) Job());
  if (!job) return IP_ENOMEM;
  own(req, job->req);
  job->req.bytes = req->mem_bytes;  // 0: projected by the slot that takes it
  ResultBox *box = new (std::nothrow) ResultBox();
  if (!box) return IP_ENOMEM;
  memset(&box->r, 0, sizeof(ip_result));
  job->res = &box->r;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    job->res->t_submit = s->now();
    *id = s->next_id++;
    s->jobs[*id] = std::move(job);
    s->queue.push_back(*id);
  }
  s->cv_work.notify_all();
  return IP_OK;
}

int ip_server_poll(ip_server *s, uint64_t id, ip_result **out) {
  if (!s || !out) return IP_EINVAL;
  *out = nullptr;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->jobs.find(id);
  if (it == s->jobs.end()) return IP_EINVAL;
  if (!it->second->done) return IP_EAGAIN;
  *out = it->second->res;
  s->jobs.erase(it);
  return IP_OK;
}

int ip_server_wait(ip_server *s, uint64_t id, ip_result **out) {
  if (!s || !out) return IP_EINVAL;
  *out = nullptr;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->jobs.find(id);
  if (it == s->jobs.end()) return IP_EINVAL;
  Job *job = it->second.get();
  s->cv_done.wait(lk, [&] { return job->done; });
  *out = job->res;
  s->jobs.erase(id);
  return IP_OK;
}

void ip_result_free(ip_result *r) {
  if (!r) return;
  ResultBox *box = reinterpret_cast<ResultBox *>(r);
  if (r->free_pts) {
    if (box->pool)
      box->pool->put(r->free_pts, box->cap);
    else
      delete[] r->free_pts;
  }
  if (r->cells) ip_cells_free(r->cells);
  delete box;
}

void ip_server_destroy(ip_server *s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->queue.clear();
  }
  s->cv_work.notify_all();
  s->cv_mem.notify_all();
  for (auto &t : s->workers)
    if (t.joinable()) t.join();
  for (auto &kv : s->jobs) {
    if (kv.second->res) ip_result_free(kv.second->res);
  }
  s->jobs.clear();
  for (ip_ctx *c : s->ctxs) ip_destroy(c);
  for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
  delete s;
}

double ip_server_clock(const ip_server *s) { return s ? s->now() : 0.0; }

}  // extern "C"
