// server.hip -- a request loop that keeps foam simulations resident on the
// device and advances them together (flb_server_* in include/foamlbm.h).
//
// Jobs queue in arrival order.  Each scheduling round admits queued jobs, in
// order, while the device bytes of the admitted (resident) jobs stay within
// the pool budget and below the job limit, then picks the jobs it advances:
//   FIFO     every resident job; admission also stops once the resident
//            cells would pass max_cells (enough to fill the GPU: beyond that,
//            running more jobs at once lengthens every job without adding
//            throughput);
//   SHORTEST resident jobs by least remaining work (cells x steps left) while
//            their cells stay within max_cells, so short jobs are not held
//            behind long ones; a job passed over kStarveRounds rounds in a row
//            goes first.
// The picked jobs advance by the same number of steps -- the chunk, shortened
// so that no job passes its last step -- with batched launches, one batch per
// lattice type and storage, so jobs that arrived at different times share
// every launch.  A job whose steps are done is retired at the end of the
// round: its final density and statistics are copied to host memory and its
// device memory is released, so the next round can admit more.  A job's
// fields are exactly those of the same job run alone.
//
// Health: every round gathers the non-finite-mass flag of each advanced job
// (one small kernel over their run-control blocks, one copy back) and
// retires a job whose mass has blown up as failed at once, instead of
// letting it hold device memory and launch slots until its last step; the
// other jobs are unaffected, since no launch mixes the fields of two jobs.
// A queued or running job may also be cancelled between rounds.
#include <algorithm>
#include <cstdio>
#include <deque>
#include <map>
#include <tuple>

#include "batch.hpp"

using namespace flb_rt;

namespace {

struct Job {
  int64_t id = 0;
  flb_params p;
  std::vector<flb_nucleus> nuc;
  int64_t steps = 0, done = 0;
  int32_t state = FLB_JOB_QUEUED;
  int idle = 0;  // consecutive rounds this resident job was not advanced
  flb_ctx* c = nullptr;
  size_t bytes = 0;
  std::vector<double> density;
  flb_stats stats;
  std::string err;
};

}  // namespace

struct flb_server {
  flb_server_config cfg;
  flb_allocator al;
  bool have_al = false;
  hipStream_t st = nullptr;
  int64_t next_id = 1;
  size_t used = 0;
  int64_t cells = 0;  // lattice cells of the running jobs
  int64_t n_done = 0;
  std::deque<Job*> queue;
  std::vector<Job*> running;
  std::map<int64_t, Job*> jobs;
  flb_batch* view[2][3] = {{nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr}};
  std::vector<flb_ctx*> vm[2][3];
  // health check: device and pinned host arrays of max_jobs run-control
  // pointers and flags, allocated on the first round
  void* d_health = nullptr;
  void* h_health = nullptr;
};

namespace {

constexpr int kStarveRounds = 8;

// out[k] = the non-finite-mass flag of run-control block ctl[k]
__global__ __launch_bounds__(256) void k_failed_flags(const Ctl* const* ctl, int n, int* out) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k < n) out[k] = ctl[k]->failed;
}

size_t health_bytes(const flb_server* s) { return (size_t)s->cfg.max_jobs * (sizeof(void*) + sizeof(int)); }

void* dev_alloc(flb_server* s, size_t n) {
  void* p = nullptr;
  if (s->have_al) return s->al.alloc(n, s->al.user);
  return hipMalloc(&p, n) == hipSuccess ? p : nullptr;
}

void dev_free(flb_server* s, void* p) {
  if (!p) return;
  if (s->have_al) s->al.free(p, s->al.user);
  else (void)hipFree(p);
}

// failed[k] = 1 if job act[k] saw a non-finite mass; synchronises the stream
int health(flb_server* s, const std::vector<Job*>& act, std::vector<int>& failed) {
  const int n = (int)act.size();
  if (!s->d_health) {
    s->d_health = dev_alloc(s, health_bytes(s));
    if (!s->d_health) return fail(FLB_ENOMEM, "device allocation of %zu bytes failed", health_bytes(s));
  }
  if (!s->h_health) HIPCHK(hipHostMalloc(&s->h_health, health_bytes(s), hipHostMallocDefault));
  const Ctl** hp = (const Ctl**)s->h_health;
  int* hf = (int*)(hp + s->cfg.max_jobs);
  const Ctl** dp = (const Ctl**)s->d_health;
  int* df = (int*)(dp + s->cfg.max_jobs);
  for (int k = 0; k < n; k++) hp[k] = act[k]->c->ctl;
  HIPCHK(hipMemcpyAsync(dp, hp, sizeof(void*) * n, hipMemcpyHostToDevice, s->st));
  k_failed_flags<<<(n + 255) / 256, 256, 0, s->st>>>(dp, n, df);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(hf, df, sizeof(int) * n, hipMemcpyDeviceToHost, s->st));
  HIPCHK(hipStreamSynchronize(s->st));
  failed.assign(hf, hf + n);
  return FLB_OK;
}

int64_t job_cells(const Job* j) { return (int64_t)j->p.nx * j->p.ny * j->p.nz; }

int admit(flb_server* s) {
  while (!s->queue.empty() && (int)s->running.size() < s->cfg.max_jobs) {
    Job* j = s->queue.front();
    const int64_t jc = job_cells(j);
    if (s->used + ctx_footprint(&j->p) > (size_t)s->cfg.pool_bytes) break;  // in order: wait for room
    if (s->cfg.policy == FLB_SERVE_FIFO && !s->running.empty() && s->cells + jc > s->cfg.max_cells) break;
    s->queue.pop_front();
    int rc = flb_create(&j->p, s->have_al ? &s->al : nullptr, s->st, &j->c);
    if (!rc) rc = flb_set_nuclei(j->c, j->nuc.data(), (int32_t)j->nuc.size());
    if (rc) {
      j->err = g_err;
      if (j->c) flb_destroy(j->c);
      j->c = nullptr;
      j->state = FLB_JOB_FAILED;
      s->n_done++;
      continue;
    }
    j->bytes = j->c->bytes;
    s->used += j->bytes;
    s->cells += jc;
    j->state = FLB_JOB_RUNNING;
    s->running.push_back(j);
  }
  return FLB_OK;
}

// the resident jobs this round advances
std::vector<Job*> pick(flb_server* s) {
  if (s->cfg.policy == FLB_SERVE_FIFO) return s->running;
  std::vector<Job*> order = s->running;
  auto key = [](const Job* j) {
    return std::make_tuple(j->idle >= kStarveRounds ? 0 : 1, (double)job_cells(j) * (double)(j->steps - j->done),
                           j->id);
  };
  std::sort(order.begin(), order.end(), [&](const Job* a, const Job* b) { return key(a) < key(b); });
  std::vector<Job*> act;
  int64_t cells = 0;
  for (Job* j : order)
    if (act.empty() || cells + job_cells(j) <= s->cfg.max_cells) {
      act.push_back(j);
      cells += job_cells(j);
    }
  std::sort(act.begin(), act.end(), [](const Job* a, const Job* b) { return a->id < b->id; });
  return act;
}

// batch views over the jobs of this round, rebuilt where membership changed
int sync_views(flb_server* s, const std::vector<Job*>& act) {
  std::vector<flb_ctx*> want[2][3];
  for (Job* j : act) want[j->c->D == 2 ? 0 : 1][j->c->p.storage].push_back(j->c);
  for (int d = 0; d < 2; d++)
    for (int t = 0; t < 3; t++) {
      if (want[d][t] == s->vm[d][t] && (s->view[d][t] || want[d][t].empty())) continue;
      batch_free(s->view[d][t]);
      s->view[d][t] = nullptr;
      s->vm[d][t] = want[d][t];
      if (want[d][t].empty()) continue;
      s->view[d][t] = batch_view(want[d][t], s->st, s->have_al ? &s->al : nullptr);
      if (!s->view[d][t]) return fail(FLB_ENOMEM, "host allocation failed");
      s->view[d][t]->graph_steps = s->cfg.graph_steps;
    }
  return FLB_OK;
}

// Releases a resident job's context.  A batch view's device tables hold its
// members' device pointers, so every view naming the context goes with it: a
// context created later at the same host address must never be taken for a
// member of the old view.
void release_ctx(flb_server* s, Job* j) {
  for (int d = 0; d < 2; d++)
    for (int t = 0; t < 3; t++)
      if (std::find(s->vm[d][t].begin(), s->vm[d][t].end(), j->c) != s->vm[d][t].end()) {
        batch_free(s->view[d][t]);
        s->view[d][t] = nullptr;
        s->vm[d][t].clear();
      }
  s->used -= j->bytes;
  s->cells -= j->c->N;
  flb_destroy(j->c);
  j->c = nullptr;
  s->n_done++;
}

void retire(flb_server* s, Job* j) {
  j->density.resize((size_t)j->c->N);
  int rc = flb_get_density(j->c, j->density.data(), j->density.size());
  if (!rc) rc = flb_get_stats(j->c, &j->stats);
  if (rc) {
    j->err = g_err;
    j->state = FLB_JOB_FAILED;
  } else {
    j->state = FLB_JOB_DONE;
  }
  release_ctx(s, j);
}

// a job whose mass became non-finite: no results, memory released now
void retire_failed(flb_server* s, Job* j) {
  char msg[96];
  snprintf(msg, sizeof msg, "non-finite mass within its first %lld steps", (long long)j->done);
  j->err = msg;
  j->density.clear();
  j->state = FLB_JOB_FAILED;
  release_ctx(s, j);
}

}  // namespace

extern "C" {

void flb_server_default_config(flb_server_config* cfg) {
  if (!cfg) return;
  cfg->pool_bytes = (int64_t)64 << 30;
  cfg->max_jobs = 256;
  cfg->chunk_steps = 100;
  cfg->graph_steps = 20;
  cfg->max_cells = (int64_t)1 << 22;
  cfg->policy = FLB_SERVE_FIFO;
}

int flb_server_create(const flb_server_config* cfg, const flb_allocator* alloc, void* hip_stream,
                      flb_server** out) {
  g_err.clear();
  if (!out || !cfg) return fail(FLB_EINVAL, "NULL argument");
  *out = nullptr;
  if (cfg->pool_bytes <= 0) return fail(FLB_EINVAL, "pool_bytes must be > 0");
  if (cfg->max_jobs < 1 || cfg->max_jobs > (1 << 16)) return fail(FLB_EINVAL, "max_jobs must be in 1..65536");
  if (cfg->chunk_steps < 1) return fail(FLB_EINVAL, "chunk_steps must be >= 1");
  if (cfg->graph_steps < 0 || cfg->graph_steps > 4096) return fail(FLB_EINVAL, "graph_steps must be in 0..4096");
  if (cfg->max_cells < 1) return fail(FLB_EINVAL, "max_cells must be >= 1");
  if (cfg->policy != FLB_SERVE_FIFO && cfg->policy != FLB_SERVE_SHORTEST)
    return fail(FLB_EINVAL, "policy must be FLB_SERVE_FIFO or FLB_SERVE_SHORTEST");
  if (alloc && (!alloc->alloc || !alloc->free)) return fail(FLB_EINVAL, "allocator needs alloc and free");
  flb_server* s = new (std::nothrow) flb_server();
  if (!s) return fail(FLB_ENOMEM, "host allocation failed");
  s->cfg = *cfg;
  if (alloc) {
    s->al = *alloc;
    s->have_al = true;
  }
  s->st = (hipStream_t)hip_stream;
  *out = s;
  return FLB_OK;
}

int flb_server_submit(flb_server* s, const flb_params* p, const flb_nucleus* nuc, int32_t n, int64_t steps,
                      int64_t* id) {
  if (!s || !p || !id) return fail(FLB_EINVAL, "NULL argument");
  if (n < 0 || (n > 0 && !nuc)) return fail(FLB_EINVAL, "bad nuclei array");
  if (steps < 0) return fail(FLB_EINVAL, "steps must be >= 0");
  int rc = validate(p);
  if (rc) return rc;
  if (p->model != 0 || p->open_z) return fail(FLB_EINVAL, "the server runs periodic single-lattice (model 0) jobs");
  const size_t fp = ctx_footprint(p);
  if (fp > (size_t)s->cfg.pool_bytes)
    return fail(FLB_EBUSY, "job needs %zu device bytes, more than the pool of %lld", fp,
                (long long)s->cfg.pool_bytes);
  Job* j = new (std::nothrow) Job();
  if (!j) return fail(FLB_ENOMEM, "host allocation failed");
  j->id = s->next_id++;
  j->p = *p;
  j->nuc.assign(nuc, nuc + n);
  j->steps = steps;
  memset(&j->stats, 0, sizeof j->stats);
  s->jobs[j->id] = j;
  s->queue.push_back(j);
  *id = j->id;
  return FLB_OK;
}

int flb_server_pump(flb_server* s, int32_t* n_running, int32_t* n_queued, int64_t* n_done) {
  if (!s) return fail(FLB_EINVAL, "server is NULL");
  int rc = admit(s);
  if (rc) return rc;
  // jobs of zero steps finish at once
  for (size_t k = 0; k < s->running.size();) {
    if (s->running[k]->steps == 0) {
      retire(s, s->running[k]);
      s->running.erase(s->running.begin() + (long)k);
    } else {
      k++;
    }
  }
  if (!s->running.empty()) {
    const std::vector<Job*> act = pick(s);
    int64_t r = s->cfg.chunk_steps;
    for (Job* j : act) r = std::min<int64_t>(r, j->steps - j->done);
    rc = sync_views(s, act);
    if (rc) return rc;
    for (int d = 0; d < 2 && !rc; d++)
      for (int t = 0; t < 3 && !rc; t++)
        if (s->view[d][t]) rc = FLB_BATCH_DISPATCH(s->view[d][t], batch_steps, s->view[d][t], r);
    if (rc) return rc;
    std::vector<int> failed;
    rc = health(s, act, failed);
    if (rc) return rc;
    std::vector<Job*> still;
    for (Job* j : s->running) {
      const auto it = std::find(act.begin(), act.end(), j);
      const bool adv = it != act.end();
      if (adv) {
        j->done += r;
        j->idle = 0;
      } else {
        j->idle++;
      }
      if (adv && failed[it - act.begin()]) retire_failed(s, j);
      else if (j->done >= j->steps) retire(s, j);
      else still.push_back(j);
    }
    s->running.swap(still);
  }
  if (n_running) *n_running = (int32_t)s->running.size();
  if (n_queued) *n_queued = (int32_t)s->queue.size();
  if (n_done) *n_done = s->n_done;
  return FLB_OK;
}

int flb_server_job(flb_server* s, int64_t id, int32_t* state, int64_t* steps_done) {
  if (!s) return fail(FLB_EINVAL, "server is NULL");
  auto it = s->jobs.find(id);
  if (it == s->jobs.end()) return fail(FLB_EINVAL, "unknown job %lld", (long long)id);
  if (state) *state = it->second->state;
  if (steps_done) *steps_done = it->second->done;
  return FLB_OK;
}

int flb_server_result(flb_server* s, int64_t id, double* density, size_t n, flb_stats* stats) {
  if (!s) return fail(FLB_EINVAL, "server is NULL");
  auto it = s->jobs.find(id);
  if (it == s->jobs.end()) return fail(FLB_EINVAL, "unknown job %lld", (long long)id);
  Job* j = it->second;
  if (j->state == FLB_JOB_FAILED) {
    const int code = j->err.rfind("non-finite", 0) == 0 ? FLB_ENUMERIC : FLB_EHIP;
    return fail(code, "job %lld failed: %s", (long long)id, j->err.c_str());
  }
  if (j->state == FLB_JOB_CANCELLED) return fail(FLB_EINVAL, "job %lld was cancelled", (long long)id);
  if (j->state != FLB_JOB_DONE) return fail(FLB_EINVAL, "job %lld is not done", (long long)id);
  if (density) {
    if (n != j->density.size()) return fail(FLB_EINVAL, "n must be %zu", j->density.size());
    memcpy(density, j->density.data(), sizeof(double) * n);
  }
  if (stats) *stats = j->stats;
  return FLB_OK;
}

int flb_server_release(flb_server* s, int64_t id) {
  if (!s) return fail(FLB_EINVAL, "server is NULL");
  auto it = s->jobs.find(id);
  if (it == s->jobs.end()) return fail(FLB_EINVAL, "unknown job %lld", (long long)id);
  Job* j = it->second;
  if (j->state == FLB_JOB_QUEUED || j->state == FLB_JOB_RUNNING)
    return fail(FLB_EBUSY, "job %lld is still queued or running", (long long)id);
  s->jobs.erase(it);
  delete j;
  return FLB_OK;
}

int flb_server_cancel(flb_server* s, int64_t id) {
  if (!s) return fail(FLB_EINVAL, "server is NULL");
  auto it = s->jobs.find(id);
  if (it == s->jobs.end()) return fail(FLB_EINVAL, "unknown job %lld", (long long)id);
  Job* j = it->second;
  if (j->state == FLB_JOB_QUEUED) {
    s->queue.erase(std::find(s->queue.begin(), s->queue.end(), j));
    s->n_done++;
  } else if (j->state == FLB_JOB_RUNNING) {
    release_ctx(s, j);
    s->running.erase(std::find(s->running.begin(), s->running.end(), j));
  } else {
    return fail(FLB_EINVAL, "job %lld has already finished", (long long)id);
  }
  j->state = FLB_JOB_CANCELLED;
  return FLB_OK;
}

int flb_server_usage(flb_server* s, int64_t* used_bytes, int64_t* pool_bytes) {
  if (!s) return fail(FLB_EINVAL, "server is NULL");
  if (used_bytes) *used_bytes = (int64_t)s->used;
  if (pool_bytes) *pool_bytes = s->cfg.pool_bytes;
  return FLB_OK;
}

void flb_server_destroy(flb_server* s) {
  if (!s) return;
  (void)hipStreamSynchronize(s->st);
  for (int d = 0; d < 2; d++)
    for (int t = 0; t < 3; t++) batch_free(s->view[d][t]);
  for (auto& kv : s->jobs) {
    if (kv.second->c) flb_destroy(kv.second->c);
    delete kv.second;
  }
  dev_free(s, s->d_health);
  if (s->h_health) (void)hipHostFree(s->h_health);
  delete s;
}

}  // extern "C"
