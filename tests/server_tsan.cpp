// Thread-sanitizer run of the serving form's request loop on a dry server
// (device -1: admission, batching, budget bookkeeping and the batched
// driver's argument checks run on the host threads; nothing touches a GPU).
// Four client threads submit jobs of two shapes while others wait for theirs
// and a fifth reads the statistics; every job must come back OK, and the
// counters must add up.  Built by the test that runs it with the library's
// host code instrumented (-Xarch_host -fsanitize=thread).
#include <atomic>
#include <cstdio>
#include <thread>
#include <vector>

#include "../include/knnkm.h"

int main() {
  knnkm_server_config cfg{};
  cfg.struct_size = sizeof(cfg);
  cfg.device = -1;
  cfg.slots = 3;
  cfg.max_batch_jobs = 4;
  cfg.max_batch_rows = 4000;
  cfg.hbm_budget_bytes = 1ll << 30;
  knnkm_server* S = nullptr;
  if (knnkm_server_create(&cfg, &S) != KNNKM_OK) {
    std::printf("create failed: %s\n", knnkm_server_last_error());
    return 1;
  }
  const int kThreads = 4, kJobs = 40;
  std::vector<float> X(2000 * 32, 0.5f);
  std::atomic<int> bad{0}, done{0};
  std::atomic<bool> stop{false};
  std::thread watcher([&] {
    while (!stop.load()) {
      knnkm_server_stats st;
      if (knnkm_server_stats_get(S, &st) != KNNKM_OK) ++bad;
      std::this_thread::yield();
    }
  });
  std::vector<std::thread> clients;
  for (int t = 0; t < kThreads; ++t)
    clients.emplace_back([&, t] {
      std::vector<uint64_t> tickets;
      for (int j = 0; j < kJobs; ++j) {
        knnkm_job job{};
        job.struct_size = sizeof(job);
        job.d = (j % 2) ? 32 : 16;
        job.n = 200 + 37 * ((t * kJobs + j) % 40);
        job.ldx = 32;
        job.X_host = X.data();
        job.k = 5;
        knnkm_default_params(&job.params);
        job.params.kappa = 8;
        job.params.tau = 2;
        job.params.max_iters = 3;
        job.params.seed = (uint64_t)(t * 1000 + j);
        uint64_t tk = 0;
        if (knnkm_server_submit(S, &job, &tk) != KNNKM_OK) {
          ++bad;
          continue;
        }
        tickets.push_back(tk);
        if (j % 5 == 4) {  // wait for the oldest outstanding job now and then
          knnkm_job_info info;
          if (knnkm_server_wait(S, tickets.front(), -1, &info) != KNNKM_OK) ++bad;
          tickets.erase(tickets.begin());
          ++done;
        }
      }
      for (uint64_t tk : tickets) {
        knnkm_job_info info;
        if (knnkm_server_wait(S, tk, -1, &info) != KNNKM_OK) ++bad;
        ++done;
      }
    });
  for (auto& c : clients) c.join();
  stop = true;
  watcher.join();
  knnkm_server_stats st;
  knnkm_server_stats_get(S, &st);
  const bool counts_ok = st.submitted == kThreads * kJobs && st.completed == kThreads * kJobs && st.failed == 0 &&
                         st.queued == 0 && st.running == 0;
  knnkm_server_destroy(S);
  std::printf("jobs %d done, %d errors, submitted %lld completed %lld batches %lld\n", done.load(), bad.load(),
              (long long)st.submitted, (long long)st.completed, (long long)st.batches);
  return (bad.load() == 0 && done.load() == kThreads * kJobs && counts_ok) ? 0 : 1;
}
