// Serving form: a request loop over one device with HBM-budget admission and
// continuous batching.  Workers (one context and one non-blocking stream
// each) take the queued jobs in arrival order, form a batch of the oldest job
// and the later queued jobs of its class, and run it through the batched
// driver, so each job's result is the same as when it runs alone.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdarg>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "common.h"

namespace {

thread_local std::string t_err;

knnkm_status srv_fail(knnkm_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  t_err = buf;
  return st;
}

constexpr int SRV_MAX_SLOTS = 16;

int64_t al(int64_t b) { return (b + 255) & ~(int64_t)255; }

// Device buffers of one job inside a batch: rows, graph ids and distances,
// labels, centroids, counts.
int64_t job_buffer_bytes(int64_t n, int64_t d, int64_t k, int64_t kappa) {
  return al(n * d * 4) + 2 * al(n * kappa * 4) + al(n * 4) + al(k * d * 4) + al(k * 4);
}

// Upper estimate of the context workspace of one batched call over n rows,
// k fit clusters and k0 graph-construction clusters in total.  Sums the
// named workspace buffers of the build, the two-means partition, the sort,
// the segmented sums and the fit (with their growth headroom of 1/8).
int64_t ws_estimate(int64_t n, int64_t d, int64_t k, int64_t k0, int64_t kappa, int64_t m, int64_t T) {
  const int64_t kx = std::max(k, k0);
  int64_t b = 0;
  b += 100 * n;                              // per-row int32/int64/double buffers
  b += (12 + 4 * 64) * n;                    // refinement survivors, their counts and row norms
  b += (4 * d + 4 * kappa + 16) * n;         // the fit's cluster-ordered copy of X and the graph
  b += 8 * d * (n / 64 + kx + 2);            // segmented-sum partials
  b += 4 * d * k0;                           // graph-construction centroids
  b += 8 * d * kx;                           // two-means split centroids
  b += 16 * d * (n / 1024 + kx + 2);         // two-means tile partials
  b += 16 * d * (n / (1024 * 16) + kx + 2);  // two-means chunk partials
  b += 200 * (k + k0);                       // per-cluster tables and the tree plan
  b += 24 * d * k + 4 * n;                   // fit: float64 sums and fixed-point composite vectors
  b += 4 * (kappa + 1) * n + 4 * n + 8 * n;  // fit: reverse graph lists, active list, flag arrays
  b += 4 * (kappa + 2) * n + 4 * k;          // fit: drift bounds (wide rows)
  b += 4 * kappa * n + k / 8;                // fit: graph-entry labels, changed-cluster flag bits
  b += 4 * 128 * n;                          // refinement: key rows of the 65-128-member clusters
  if (k0 > 0 && 2 * (n / k0) > 128)          // and of the 129-1024-member ones (clusters of up to 4n/k0)
    b += 4 * std::min<int64_t>(1024, (4 * (n / k0) + 63) / 64 * 64) * n;
  b += 2 * d * (k + k0) + 4 * (k + k0);      // bfloat16 centroid shadows (wide rows)
  b += 64 * m + 16 * (T + 1) * m;            // job tables and traces
  b += 1 << 20;                              // scans, partial sums, small tables
  return b + b / 8 + (32 << 20);
}

extern "C" knnkm_status knnkm_workspace_estimate(int64_t n, int32_t d, int32_t k, const knnkm_params* p,
                                                 int64_t* out) {
  if (!p || !out || n < 1 || d < 1 || k < 1 || k > n || p->xi < 2 || p->kappa < 1) return KNNKM_EINVAL;
  const int64_t k0 = p->tau > 0 ? std::max<int64_t>(1, n / p->xi) : 0;
  *out = ws_estimate(n, d, k, k0, p->kappa, 1, std::max(0, p->max_iters));
  return KNNKM_OK;
}

struct SJob {
  uint64_t ticket = 0;
  knnkm_job req{};
  int64_t buf_bytes = 0;
  knnkm_job_info info{};
  bool done = false;
};

bool same_class(const knnkm_job& a, const knnkm_job& b) {
  if (a.d != b.d) return false;
  knnkm_params x = a.params, y = b.params;
  x.seed = y.seed = 0;
  x.early_stop = y.early_stop = 0;
  return std::memcmp(&x, &y, sizeof(x)) == 0;
}

double now_s(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

struct knnkm_server {
  knnkm_server_config cfg{};
  bool dry = false;
  std::chrono::steady_clock::time_point t0;
  knnkm_ctx* vctx = nullptr;  // dry context: argument validation only

  std::mutex mu;
  std::condition_variable cv_work;  // workers: queue or budget changed
  std::condition_variable cv_done;  // waiters: a job finished
  bool stop = false;
  bool broken = false;  // a device error: later jobs fail
  std::deque<SJob*> queue;
  std::unordered_map<uint64_t, std::unique_ptr<SJob>> jobs;
  uint64_t next_ticket = 1;
  int64_t next_batch = 0;
  knnkm_server_stats st{};

  struct Slot {
    knnkm_ctx* ctx = nullptr;
    hipStream_t stream = nullptr;
    bool busy = false;
    int64_t ws_charged = 0;  // workspace the worker keeps between batches (its actual size)
    std::thread th;
  };
  std::vector<Slot> slots;

  void charge(int64_t b) {
    st.bytes_in_use += b;
    st.bytes_peak = std::max(st.bytes_peak, st.bytes_in_use);
  }

  // Pick the next batch for slot `s` (lock held).  Empty if nothing fits.
  std::vector<SJob*> form_batch(int s, int64_t* extra_ws) {
    std::vector<SJob*> B;
    if (queue.empty()) return B;
    SJob* head = queue.front();
    int64_t rows = 0, bytes = 0, k = 0, k0 = 0;
    auto k0_of = [](const knnkm_job& j) {
      return j.params.tau > 0 ? std::max<int64_t>(1, j.n / j.params.xi) : 0;
    };
    auto need = [&](int64_t r, int64_t by, int64_t kk, int64_t kk0, int64_t m) {
      const int64_t ws = ws_estimate(r, head->req.d, kk, kk0, head->req.params.kappa, m, head->req.params.max_iters);
      return by + ws;  // the kept workspace may all be replaced while the batch grows it
    };
    for (SJob* j : queue) {
      if (!same_class(j->req, head->req)) continue;
      if ((int64_t)B.size() >= cfg.max_batch_jobs) break;
      if (!B.empty() && rows + j->req.n > cfg.max_batch_rows) continue;
      const int64_t r = rows + j->req.n, by = bytes + j->buf_bytes;
      const int64_t kk = k + j->req.k, kk0 = k0 + k0_of(j->req);
      if (st.bytes_in_use + need(r, by, kk, kk0, (int64_t)B.size() + 1) > cfg.hbm_budget_bytes) {
        if (B.empty()) return B;  // the oldest job waits for memory
        continue;
      }
      B.push_back(j);
      rows = r;
      bytes = by;
      k = kk;
      k0 = kk0;
    }
    const int64_t ws = ws_estimate(rows, head->req.d, k, k0, head->req.params.kappa, (int64_t)B.size(),
                                   head->req.params.max_iters);
    *extra_ws = ws;
    return B;
  }

  // Idle workers keep workspace charged to the budget; release it when the
  // oldest job cannot be admitted (lock held; those contexts are not in use).
  bool release_idle_ws() {
    bool any = false;
    for (auto& sl : slots) {
      if (sl.busy || sl.ws_charged == 0) continue;
      if (!dry) (void)hipSetDevice(cfg.device);
      knnkm_ws_release(sl.ctx);
      st.bytes_in_use -= sl.ws_charged;
      sl.ws_charged = 0;
      any = true;
    }
    return any;
  }

  knnkm_status run_batch(Slot& sl, const std::vector<SJob*>& B);
  void worker(int s);
};

knnkm_status knnkm_server::run_batch(Slot& sl, const std::vector<SJob*>& B) {
  const knnkm_job& h = B[0]->req;
  const int m = (int)B.size();
  const int64_t d = h.d, kappa = h.params.kappa;
  std::vector<int64_t> n_off(m + 1, 0);
  std::vector<int32_t> ks(m);
  std::vector<uint64_t> seeds(m);
  std::vector<int64_t> k_off(m + 1, 0);
  for (int q = 0; q < m; ++q) {
    n_off[q + 1] = n_off[q] + B[q]->req.n;
    k_off[q + 1] = k_off[q] + B[q]->req.k;
    ks[q] = B[q]->req.k;
    seeds[q] = B[q]->req.params.seed;
  }
  const int64_t N = n_off[m], K = k_off[m];
  const int T = h.params.max_iters;
  std::vector<double> trace((size_t)m * (T + 1));
  if (dry) {
    knnkm_status r = knnkm_fit_batched(sl.ctx, (const float*)h.X_host, (int32_t)d, d, m, n_off.data(), ks.data(),
                                       seeds.data(), &h.params, (int32_t*)16, (float*)16, (int32_t*)16,
                                       (float*)16, (int32_t*)16, nullptr);
    if (r != KNNKM_OK) t_err = knnkm_last_error(sl.ctx);
    return r;
  }
  if (hipSetDevice(cfg.device) != hipSuccess) return srv_fail(KNNKM_EDEVICE, "server: hipSetDevice failed");
  // one allocation for the batch: X | G_ids | G_d2 | labels | C | counts
  const int64_t oX = 0, oG = oX + al(N * d * 4), oD = oG + al(N * kappa * 4), oL = oD + al(N * kappa * 4),
                oC = oL + al(N * 4), oN = oC + al(K * d * 4), total = oN + al(K * 4);
  char* base = nullptr;
  hipError_t e = hipMallocAsync((void**)&base, (size_t)total, sl.stream);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return srv_fail(KNNKM_ENOMEM, "server: cannot allocate %lld bytes for a batch", (long long)total);
  }
  float* X = (float*)(base + oX);
  int32_t* G = (int32_t*)(base + oG);
  float* G2 = (float*)(base + oD);
  int32_t* lab = (int32_t*)(base + oL);
  float* C = (float*)(base + oC);
  int32_t* cnt = (int32_t*)(base + oN);
  knnkm_status r = KNNKM_OK;
  for (int q = 0; q < m && e == hipSuccess; ++q) {
    const knnkm_job& j = B[q]->req;
    e = hipMemcpy2DAsync(X + n_off[q] * d, (size_t)d * 4, j.X_host, (size_t)j.ldx * 4, (size_t)d * 4,
                         (size_t)j.n, hipMemcpyHostToDevice, sl.stream);
  }
  if (e != hipSuccess) r = srv_fail(KNNKM_EDEVICE, "server: upload: %s", hipGetErrorString(e));
  if (r == KNNKM_OK) {
    r = knnkm_fit_batched(sl.ctx, X, (int32_t)d, d, m, n_off.data(), ks.data(), seeds.data(), &h.params, G, G2,
                          lab, C, cnt, trace.data());
    if (r != KNNKM_OK) t_err = knnkm_last_error(sl.ctx);
  }
  for (int q = 0; q < m && r == KNNKM_OK && e == hipSuccess; ++q) {
    const knnkm_job& j = B[q]->req;
    if (j.labels_host)
      e = hipMemcpyAsync(j.labels_host, lab + n_off[q], (size_t)j.n * 4, hipMemcpyDeviceToHost, sl.stream);
    if (e == hipSuccess && j.C_host)
      e = hipMemcpyAsync(j.C_host, C + k_off[q] * d, (size_t)j.k * d * 4, hipMemcpyDeviceToHost, sl.stream);
    if (e == hipSuccess && j.counts_host)
      e = hipMemcpyAsync(j.counts_host, cnt + k_off[q], (size_t)j.k * 4, hipMemcpyDeviceToHost, sl.stream);
    if (e == hipSuccess && j.G_ids_host)
      e = hipMemcpyAsync(j.G_ids_host, G + n_off[q] * kappa, (size_t)(j.n * kappa) * 4, hipMemcpyDeviceToHost,
                         sl.stream);
  }
  hipError_t e2 = hipStreamSynchronize(sl.stream);
  if (r == KNNKM_OK && (e != hipSuccess || e2 != hipSuccess))
    r = srv_fail(KNNKM_EDEVICE, "server: download: %s", hipGetErrorString(e != hipSuccess ? e : e2));
  (void)hipFreeAsync(base, sl.stream);
  if (r == KNNKM_OK) {
    // graph ids are global row ids of the batch; make them job-local
    for (int q = 0; q < m; ++q) {
      const knnkm_job& j = B[q]->req;
      if (j.G_ids_host && n_off[q] != 0) {
        const int32_t o = (int32_t)n_off[q];
        for (int64_t i = 0; i < j.n * kappa; ++i) j.G_ids_host[i] -= o;
      }
      if (j.trace_host)
        std::memcpy(j.trace_host, trace.data() + (size_t)q * (T + 1), sizeof(double) * (T + 1));
    }
  }
  return r;
}

void knnkm_server::worker(int s) {
  Slot& sl = slots[s];
  if (!dry) (void)hipSetDevice(cfg.device);
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    std::vector<SJob*> B;
    int64_t extra_ws = 0;
    for (;;) {
      if (!queue.empty()) {
        B = form_batch(s, &extra_ws);
        if (!B.empty()) break;
        // the oldest job does not fit: free idle workspace, then wait
        if (release_idle_ws()) continue;
      } else if (stop) {
        return;
      }
      cv_work.wait(lk);
    }
    // admit
    const double ta = now_s(t0);
    int64_t bytes = 0;
    for (SJob* j : B) {
      queue.erase(std::find(queue.begin(), queue.end(), j));
      j->info.t_admit = ta;
      j->info.slot = s;
      j->info.batch = next_batch;
      j->info.batch_jobs = (int32_t)B.size();
      bytes += j->buf_bytes;
    }
    ++next_batch;
    sl.busy = true;
    charge(bytes + extra_ws);
    st.queued = (int64_t)queue.size();
    st.running += (int64_t)B.size();
    st.max_batch_jobs_seen = std::max<int64_t>(st.max_batch_jobs_seen, (int64_t)B.size());
    const bool was_broken = broken;
    const int64_t ws_before = sl.ws_charged;
    lk.unlock();

    knnkm_status r = was_broken ? KNNKM_EDEVICE : run_batch(sl, B);
    int64_t ws_now = 0;
    if (!dry && r != KNNKM_EDEVICE) (void)knnkm_workspace_bytes(sl.ctx, &ws_now);

    lk.lock();
    const double td = now_s(t0);
    if (r == KNNKM_EDEVICE) broken = true;
    // from now on the worker's kept workspace is charged at its actual size
    if (!dry && r != KNNKM_EDEVICE) {
      if (ws_now > ws_before + extra_ws) ++st.ws_overruns;
      st.bytes_in_use += ws_now - sl.ws_charged;
      sl.ws_charged = ws_now;
    }
    st.bytes_in_use -= bytes + extra_ws;
    sl.busy = false;
    ++st.batches;
    st.running -= (int64_t)B.size();
    for (SJob* j : B) {
      j->info.status = r;
      j->info.t_done = td;
      j->done = true;
      if (r == KNNKM_OK)
        ++st.completed;
      else
        ++st.failed;
    }
    cv_done.notify_all();
    cv_work.notify_all();
  }
}

extern "C" knnkm_status knnkm_server_create(const knnkm_server_config* c, knnkm_server** out) {
  if (!c || !out) return srv_fail(KNNKM_EINVAL, "knnkm_server_create: null argument");
  *out = nullptr;
  if (c->struct_size != sizeof(knnkm_server_config))
    return srv_fail(KNNKM_EINVAL, "knnkm_server_create: config.struct_size %u != %zu", c->struct_size,
                    sizeof(knnkm_server_config));
  if (c->slots < 1 || c->slots > SRV_MAX_SLOTS)
    return srv_fail(KNNKM_EINVAL, "knnkm_server_create: slots must be 1..%d", SRV_MAX_SLOTS);
  if (c->max_batch_jobs < 1 || c->max_batch_rows < 1 || c->hbm_budget_bytes <= 0)
    return srv_fail(KNNKM_EINVAL, "knnkm_server_create: batch limits and budget must be positive");
  std::unique_ptr<knnkm_server> S(new (std::nothrow) knnkm_server());
  if (!S) return srv_fail(KNNKM_ENOMEM, "knnkm_server_create: out of host memory");
  S->cfg = *c;
  S->dry = c->device < 0;
  S->t0 = std::chrono::steady_clock::now();
  if (knnkm_create(-1, nullptr, &S->vctx) != KNNKM_OK)
    return srv_fail(KNNKM_ENOMEM, "knnkm_server_create: cannot create a context");
  S->slots.resize(c->slots);
  auto cleanup = [&](knnkm_status st, const std::string& msg) {
    for (auto& sl : S->slots) {
      if (sl.ctx) knnkm_destroy(sl.ctx);
      if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    knnkm_destroy(S->vctx);
    t_err = msg;
    return st;
  };
  if (!S->dry) {
    // keep freed batch memory in the device's pool up to the budget instead
    // of returning it to the driver at every synchronisation
    hipMemPool_t pool = nullptr;
    uint64_t thr = (uint64_t)c->hbm_budget_bytes;
    if (hipSetDevice(c->device) == hipSuccess && hipDeviceGetDefaultMemPool(&pool, c->device) == hipSuccess)
      (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
    (void)hipGetLastError();
  }
  for (auto& sl : S->slots) {
    if (!S->dry) {
      if (hipSetDevice(c->device) != hipSuccess ||
          hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        return cleanup(KNNKM_EDEVICE, "knnkm_server_create: cannot create a stream on the device");
      }
    }
    if (knnkm_create(S->dry ? -1 : c->device, sl.stream, &sl.ctx) != KNNKM_OK)
      return cleanup(KNNKM_EDEVICE, std::string("knnkm_server_create: ") + knnkm_last_error(nullptr));
  }
  knnkm_server* srv = S.release();
  for (int s = 0; s < c->slots; ++s) srv->slots[s].th = std::thread(&knnkm_server::worker, srv, s);
  *out = srv;
  return KNNKM_OK;
}

extern "C" knnkm_status knnkm_server_submit(knnkm_server* srv, const knnkm_job* job, uint64_t* ticket) {
  if (!srv || !job || !ticket) return srv_fail(KNNKM_EINVAL, "knnkm_server_submit: null argument");
  if (job->struct_size != sizeof(knnkm_job))
    return srv_fail(KNNKM_EINVAL, "knnkm_server_submit: job.struct_size %u != %zu", job->struct_size,
                    sizeof(knnkm_job));
  if (!job->X_host) return srv_fail(KNNKM_EINVAL, "knnkm_server_submit: X_host is null");
  if (job->ldx < job->d) return srv_fail(KNNKM_EINVAL, "knnkm_server_submit: ldx < d");
  // the batched driver's own checks, on a dry context
  {
    const int64_t noff[2] = {0, job->n};
    const int32_t k = job->k;
    const uint64_t seed = job->params.seed;
    std::lock_guard<std::mutex> g(srv->mu);  // the validation context is shared
    knnkm_status r = knnkm_fit_batched(srv->vctx, job->X_host, job->d, job->ldx, 1, noff, &k, &seed, &job->params,
                                       (int32_t*)16, (float*)16, (int32_t*)16, (float*)16, (int32_t*)16, nullptr);
    if (r != KNNKM_OK) {
      ++srv->st.rejected;
      return srv_fail(r, "knnkm_server_submit: %s", knnkm_last_error(srv->vctx));
    }
  }
  std::unique_ptr<SJob> J(new SJob());
  J->req = *job;
  J->buf_bytes = job_buffer_bytes(job->n, job->d, job->k, job->params.kappa);
  const int64_t k0 = job->params.tau > 0 ? std::max<int64_t>(1, job->n / job->params.xi) : 0;
  const int64_t alone = J->buf_bytes + ws_estimate(job->n, job->d, job->k, k0, job->params.kappa, 1, job->params.max_iters);
  J->info.footprint_bytes = alone;
  std::lock_guard<std::mutex> g(srv->mu);
  if (alone > srv->cfg.hbm_budget_bytes) {
    ++srv->st.rejected;
    return srv_fail(KNNKM_ENOMEM, "knnkm_server_submit: job needs %lld bytes, the budget is %lld",
                    (long long)alone, (long long)srv->cfg.hbm_budget_bytes);
  }
  if (srv->stop) return srv_fail(KNNKM_EINVAL, "knnkm_server_submit: server is stopping");
  J->ticket = srv->next_ticket++;
  J->info.t_submit = now_s(srv->t0);
  J->info.status = KNNKM_EAGAIN;
  J->info.slot = -1;
  J->info.batch = -1;
  *ticket = J->ticket;
  srv->queue.push_back(J.get());
  srv->jobs[J->ticket] = std::move(J);
  ++srv->st.submitted;
  srv->st.queued = (int64_t)srv->queue.size();
  srv->st.max_queued = std::max(srv->st.max_queued, srv->st.queued);
  srv->cv_work.notify_one();
  return KNNKM_OK;
}

extern "C" knnkm_status knnkm_server_wait(knnkm_server* srv, uint64_t ticket, int64_t timeout_ms,
                                          knnkm_job_info* info) {
  if (!srv) return srv_fail(KNNKM_EINVAL, "knnkm_server_wait: null server");
  std::unique_lock<std::mutex> lk(srv->mu);
  auto it = srv->jobs.find(ticket);
  if (it == srv->jobs.end()) return srv_fail(KNNKM_EINVAL, "knnkm_server_wait: unknown ticket %llu",
                                             (unsigned long long)ticket);
  SJob* j = it->second.get();
  auto ready = [&] { return j->done; };
  if (timeout_ms < 0)
    srv->cv_done.wait(lk, ready);
  else if (!srv->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready))
    return KNNKM_EAGAIN;
  if (info) *info = j->info;
  const knnkm_status r = (knnkm_status)j->info.status;
  srv->jobs.erase(it);
  if (r != KNNKM_OK) t_err = "knnkm_server_wait: the job's batch failed";
  return r;
}

extern "C" knnkm_status knnkm_server_stats_get(knnkm_server* srv, knnkm_server_stats* out) {
  if (!srv || !out) return srv_fail(KNNKM_EINVAL, "knnkm_server_stats_get: null argument");
  std::lock_guard<std::mutex> g(srv->mu);
  *out = srv->st;
  return KNNKM_OK;
}

extern "C" const char* knnkm_server_last_error(void) { return t_err.c_str(); }

extern "C" knnkm_status knnkm_server_destroy(knnkm_server* srv) {
  if (!srv) return srv_fail(KNNKM_EINVAL, "knnkm_server_destroy: null server");
  {
    std::lock_guard<std::mutex> g(srv->mu);
    srv->stop = true;
  }
  srv->cv_work.notify_all();
  for (auto& sl : srv->slots)
    if (sl.th.joinable()) sl.th.join();
  if (!srv->dry) (void)hipSetDevice(srv->cfg.device);
  for (auto& sl : srv->slots) {
    knnkm_destroy(sl.ctx);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
  }
  knnkm_destroy(srv->vctx);
  delete srv;
  return KNNKM_OK;
}
