// batch.hpp -- many lattices advanced together: batch state and launches.
//
// Members are ordinary contexts of one lattice type and one storage format;
// their extents and parameters may differ.  One step of the batch is one
// batched step-kernel launch over every member's workgroups (member k owns the
// launch's workgroups [first[k], first[k+1])) and one batched finisher
// launch with a workgroup per member; with films, a batched rupture-test
// launch, and a batched launch that prunes the film members' masks and runs
// every member's finisher; film-map refreshes run batched over the members
// that are due.  So
// the launch count per step does not grow with the number of lattices, and the
// GPU is filled by all members at once instead of one small lattice at a time.
// Runs of steps are captured in a HIP graph and replayed.  D2Q9 batches may
// instead run each stretch of steps between refreshes as one persistent
// cooperative launch (persist.hpp).
#pragma once
#include "persist.hpp"
#include "runtime.hpp"

namespace flb_rt {

// ext: some member has a source term, the gas release or the body force (the
// members without them skip them inside that variant)
using BatchStepFn = void (*)(const StepArgs*, const int*, int, int, bool, bool, hipStream_t);

template <class L, class S, int TX, int TM, bool EXT, int FR>
void launch_step_batch_g(const StepArgs* tab, const int* first, int nmem, int nblk, bool buf, hipStream_t s) {
  if (buf)
    hipLaunchKernelGGL((k_step_batch<L, S, TX, TM, true, EXT, FR>), dim3(nblk),
                       dim3(StepBlock<L, S, TX, TM, true, EXT, FR>::NT), 0, s, tab, first, nmem);
  else
    hipLaunchKernelGGL((k_step_batch<L, S, TX, TM, false, EXT, FR>), dim3(nblk),
                       dim3(StepBlock<L, S, TX, TM, false, EXT, FR>::NT), 0, s, tab, first, nmem);
}
template <class L, class S, int TX, int TM, int FR>
void launch_step_batch(const StepArgs* tab, const int* first, int nmem, int nblk, bool buf, bool ext,
                       hipStream_t s) {
  if (ext) launch_step_batch_g<L, S, TX, TM, true, FR>(tab, first, nmem, nblk, buf, s);
  else launch_step_batch_g<L, S, TX, TM, false, FR>(tab, first, nmem, nblk, buf, s);
}

// batched launchers of the z-march and flat tile variants, in the order of
// the single-lattice tile tables (the two-pass variant has no batched form)
template <class L, int TX, int TM, int FR = 0>
struct BatchTile {
  static constexpr BatchStepFn fn[3] = {&launch_step_batch<L, SF64, TX, TM, FR>,
                                        &launch_step_batch<L, SF32, TX, TM, FR>,
                                        &launch_step_batch<L, SF16S, TX, TM, FR>};
};
inline const BatchStepFn* const kBatch2[] = {BatchTile<D2Q9K, 64, 1>::fn, BatchTile<D2Q9K, 128, 1>::fn,
                                      BatchTile<D2Q9K, 256, 1>::fn, BatchTile<D2Q9K, 64, 1, 2>::fn,
                                      BatchTile<D2Q9K, 64, 1, 4>::fn};
inline const BatchStepFn* const kBatch3[] = {BatchTile<D3Q19K, 64, 4>::fn, BatchTile<D3Q19K, 64, 8>::fn,
                                      BatchTile<D3Q19K, 32, 8>::fn, BatchTile<D3Q19K, 128, 4>::fn};
constexpr int kNBatch2 = sizeof(kBatch2) / sizeof(kBatch2[0]);
constexpr int kNBatch3 = sizeof(kBatch3) / sizeof(kBatch3[0]);

inline long long lcm_ll(long long a, long long b) {
  long long x = a, y = b;
  while (y) {
    const long long t = x % y;
    x = y;
    y = t;
  }
  return a / x * b;
}

}  // namespace flb_rt

struct flb_batch {
  std::vector<flb_ctx*> m;
  bool owns_members = true;  // false for a server's view over its jobs' contexts
  flb_allocator al;
  bool have_al = false;
  hipStream_t st = nullptr;
  int D = 0, storage = 0;
  // tuning shared by the members
  int tile = 0;
  long long target = 2048;  // workgroups of the whole batch step launch
  int xcd = 0;
  bool buf = true;  // every member's buffers take the buffer-resource path
  // device tables
  std::vector<void*> allocs;
  StepArgs* tab = nullptr;
  int* first = nullptr;
  int nblk = 0;
  std::vector<int> film;  // indices of film members
  StepArgs* ftab = nullptr;
  PruneArgs* ptab = nullptr;
  int* ffirst = nullptr;
  int* fidx = nullptr;  // film members' indices, then the other members' (the closing launch)
  std::vector<int> fidx_h;
  int fblk = 0;
  flb_rt::MapSet fms;  // film refresh of the film members, one launch per map kernel
  flb_rt::Fork fork;   // side stream of the refresh
  bool dirty = true;
  bool ext = false;  // some member has a source term (gas release, body force)
  // persistent launches (D2Q9): the batch tile of 256 x 1 cells, runs of at
  // most persist_max steps per launch, workgroups sized to occupancy
  bool persist = false;
  int persist_max = 1024;
  int pgrid = 0;
  // graphs
  int graph_steps = 16;
  hipGraphExec_t gexec = nullptr;
  long long gperiod = 0;
  std::vector<long long> gkey;

  void* dalloc(size_t bytes) {
    bytes = (bytes + 255) & ~(size_t)255;
    void* ptr = nullptr;
    if (have_al) ptr = al.alloc(bytes, al.user);
    else if (hipMalloc(&ptr, bytes) != hipSuccess) ptr = nullptr;
    if (ptr) allocs.push_back(ptr);
    return ptr;
  }
  void dfree(void* ptr) {
    if (!ptr) return;
    if (have_al) al.free(ptr, al.user);
    else (void)hipFree(ptr);
    auto it = std::find(allocs.begin(), allocs.end(), ptr);
    if (it != allocs.end()) allocs.erase(it);
  }
  void drop_graph() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    gexec = nullptr;
    gperiod = 0;
    gkey.clear();
  }
  int n_tiles() const { return D == 2 ? flb_rt::kNBatch2 : flb_rt::kNBatch3; }
  static constexpr int kPersistTile = 2;  // kBatch2's 256 x 1 tile
  // untuned batches: D2Q9 the flat 64 x 8 tile (the fastest on small
  // lattices), D3Q19 the 64 x 8 march
  static int default_tile(int D) { return D == 2 ? 3 : 1; }
  flb_rt::BatchStepFn step_fn() const { return (D == 2 ? flb_rt::kBatch2 : flb_rt::kBatch3)[tile][storage]; }
};

namespace flb_rt {

// per-member tuning from the batch tuning: each member gets a share of the
// target workgroups in proportion to its cells
inline void apply_tuning(flb_batch* b) {
  long long total = 0;
  for (flb_ctx* c : b->m) total += c->N;
  for (flb_ctx* c : b->m) {
    c->tile = b->tile;
    const long long share = std::max<long long>(1, (long long)((double)b->target * (double)c->N / (double)total));
    c->lz = lz_for_target(c, share);
    c->xcd = b->xcd;
  }
}

// device tables of the members' arguments and workgroup ranges
inline int rebuild(flb_batch* b) {
  apply_tuning(b);
  const int n = (int)b->m.size();
  std::vector<StepArgs> tab(n);
  std::vector<int> first(n + 1, 0);
  b->buf = true;
  for (int k = 0; k < n; k++) {
    tab[k] = step_args(b->m[k]);
    first[k + 1] = first[k] + b->m[k]->nblocks();
    if (b->m[k]->fbytes >= kBufPathLimit) b->buf = false;
  }
  b->film.clear();
  b->ext = false;
  for (int k = 0; k < n; k++) {
    if (b->m[k]->p.film_on) b->film.push_back(k);
    if (tab[k].srcw || tab[k].force_on) b->ext = true;
  }
  const int nf = (int)b->film.size();
  std::vector<StepArgs> ftab(nf);
  std::vector<PruneArgs> ptab(nf);
  std::vector<int> ffirst(nf + 1, 0);
  for (int j = 0; j < nf; j++) {
    flb_ctx* c = b->m[b->film[j]];
    ftab[j] = tab[b->film[j]];
    ptab[j] = prune_args(c);
    ffirst[j + 1] = ffirst[j] + list_grid(c->N);
  }
  if (!b->tab) {
    b->tab = (StepArgs*)b->dalloc(sizeof(StepArgs) * n);
    b->first = (int*)b->dalloc(sizeof(int) * (n + 1));
    if (nf) {
      b->ftab = (StepArgs*)b->dalloc(sizeof(StepArgs) * nf);
      b->ptab = (PruneArgs*)b->dalloc(sizeof(PruneArgs) * nf);
      b->ffirst = (int*)b->dalloc(sizeof(int) * (nf + 1));
      b->fidx = (int*)b->dalloc(sizeof(int) * n);
    }
    if (!b->tab || !b->first || (nf && (!b->ftab || !b->ptab || !b->ffirst || !b->fidx)))
      return fail(FLB_ENOMEM, "batch table allocation failed");
  }
  HIPCHK(hipMemcpyAsync(b->tab, tab.data(), sizeof(StepArgs) * n, hipMemcpyHostToDevice, b->st));
  HIPCHK(hipMemcpyAsync(b->first, first.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice, b->st));
  if (nf) {
    HIPCHK(hipMemcpyAsync(b->ftab, ftab.data(), sizeof(StepArgs) * nf, hipMemcpyHostToDevice, b->st));
    HIPCHK(hipMemcpyAsync(b->ptab, ptab.data(), sizeof(PruneArgs) * nf, hipMemcpyHostToDevice, b->st));
    HIPCHK(hipMemcpyAsync(b->ffirst, ffirst.data(), sizeof(int) * (nf + 1), hipMemcpyHostToDevice, b->st));
    b->fidx_h = b->film;
    for (int k = 0; k < n; k++)
      if (!b->m[k]->p.film_on) b->fidx_h.push_back(k);
    HIPCHK(hipMemcpyAsync(b->fidx, b->fidx_h.data(), sizeof(int) * n, hipMemcpyHostToDevice, b->st));
  }
  if (nf) {
    int rc = b->fork.init();  // outside any graph capture
    if (rc) return rc;
    std::vector<MapArgs> margs;
    for (int k : b->film) margs.push_back(map_args(b->m[k], false, GAS_AUTO));
    rc = mapset_build(b->fms, margs, b->D, [b](size_t bytes) { return b->dalloc(bytes); }, b->st);
    if (rc) return rc;
  }
  HIPCHK(hipStreamSynchronize(b->st));
  b->nblk = first[n];
  b->fblk = ffirst[nf];
  b->dirty = false;
  b->drop_graph();
  return FLB_OK;
}

// one step of every member (no synchronisation, capturable)
template <class L, class S>
int batch_one_step(flb_batch* b) {
  // one batched refresh when any film member is due; the map kernels skip
  // the members that are not
  bool due = false;
  for (int k : b->film) due = due || b->m[k]->launched % b->m[k]->p.k_own == 0;
  if (due) {
    int rc = b->fork.init();
    if (!rc) rc = map_pipeline<L, S>(b->fms, b->st, GAS_AUTO, true, &b->fork);
    if (rc) return rc;
  }
  const int n = (int)b->m.size();
  b->step_fn()(b->tab, b->first, n, b->nblk, b->buf, b->ext, b->st);
  const int nf = (int)b->film.size();
  if (nf) {
    hipLaunchKernelGGL((k_rupture_batch<L, typename S::ct>), dim3(b->fblk), dim3(MAP_NT), 0, b->st, b->ftab,
                       b->ffirst, nf);
    // the pruning launch also closes every member's step
    hipLaunchKernelGGL((k_prune_finish_batch<L>), dim3(b->fblk + (n - nf)), dim3(MAP_NT), 0, b->st, b->ptab,
                       b->ffirst, nf, b->tab, b->first, b->fidx);
  } else {
    hipLaunchKernelGGL(k_step_finish_batch, dim3(n), dim3(FIN_NT), 0, b->st, b->tab, b->first);
  }
  HIPCHK(hipGetLastError());
  for (flb_ctx* c : b->m) c->launched++;
  return FLB_OK;
}

// the refresh phase of every film member, and whether it has maps to carry
// aliases from; a captured run of steps replays correctly only from the same
// phases
inline std::vector<long long> phase_key(const flb_batch* b) {
  std::vector<long long> key;
  for (int k : b->film) key.push_back(b->m[k]->launched % b->m[k]->p.k_own);
  return key;
}

inline long long graph_period(const flb_batch* b) {
  long long per = b->graph_steps;
  for (int k : b->film) {
    per = lcm_ll(per, b->m[k]->p.k_own);
    if (per > 4096) return 0;
  }
  return per;
}

// ---- persistent runs (D2Q9) ----
template <class S, bool BUF, bool EXT>
inline const void* persist_fn() {
  return (const void*)&k_batch_persist<S, BUF, EXT>;
}
template <class S>
inline const void* persist_kernel(const flb_batch* b) {
  return b->buf ? (b->ext ? persist_fn<S, true, true>() : persist_fn<S, true, false>())
                : (b->ext ? persist_fn<S, false, true>() : persist_fn<S, false, false>());
}

// workgroups of the persistent launch: as many as are resident at once (a
// cooperative launch needs all of them resident), and no more than the
// largest phase has work for
template <class S>
int persist_grid(flb_batch* b) {
  int dev = 0, cus = 0, coop = 0, per = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev));
  if (!coop) return fail(FLB_EINVAL, "the device has no cooperative launches");
  HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, persist_kernel<S>(b), PERSIST_TX, 0));
  if (per < 1) return fail(FLB_EHIP, "the persistent kernel fits no workgroup on a compute unit");
  const int work = std::max(std::max(b->nblk, b->fblk), (int)b->m.size());
  b->pgrid = std::max(1, std::min(per * cus, work));
  return FLB_OK;
}

// steps until some film member is due for a refresh (each is due before the
// step whose index is a multiple of its k_own), at most `left`
inline int64_t steps_to_refresh(const flb_batch* b, int64_t left) {
  int64_t r = left;
  for (int k : b->film) {
    const flb_ctx* c = b->m[k];
    r = std::min<int64_t>(r, c->p.k_own - c->launched % c->p.k_own);
  }
  return r;
}

template <class S>
int persist_steps(flb_batch* b, int64_t nsteps) {
  if (b->tile != flb_batch::kPersistTile) return fail(FLB_EINVAL, "persistent runs take the 256 x 1 batch tile");
  int rc = persist_grid<S>(b);
  if (rc) return rc;
  const void* fn = persist_kernel<S>(b);
  const StepArgs* tab = b->tab;
  const int* first = b->first;
  int nmem = (int)b->m.size();
  const StepArgs* ftab = b->ftab;
  const PruneArgs* ptab = b->ptab;
  const int* ffirst = b->ffirst;
  int nf = (int)b->film.size();
  for (int64_t done = 0; done < nsteps;) {
    bool due = false;
    for (int k : b->film) due = due || b->m[k]->launched % b->m[k]->p.k_own == 0;
    if (due) {
      rc = b->fork.init();
      if (!rc) rc = map_pipeline<D2Q9K, S>(b->fms, b->st, GAS_AUTO, true, &b->fork);
      if (rc) return rc;
    }
    int run = (int)steps_to_refresh(b, std::min<int64_t>(nsteps - done, b->persist_max));
    void* args[] = {&tab, &first, &nmem, &ftab, &ptab, &ffirst, &nf, &run};
    HIPCHK(hipLaunchCooperativeKernel(fn, dim3(b->pgrid), dim3(PERSIST_TX), args, 0, b->st));
    for (flb_ctx* c : b->m) c->launched += run;
    done += run;
  }
  return FLB_OK;
}

template <class L, class S>
int batch_steps(flb_batch* b, int64_t nsteps) {
  if (b->dirty) {
    int rc = rebuild(b);
    if (rc) return rc;
  }
  if constexpr (std::is_same_v<L, D2Q9K>)
    if (b->persist) return persist_steps<S>(b, nsteps);
  int64_t done = 0;
  // graphs need a capturable (non-null) stream
  const long long per = (b->graph_steps > 0 && b->st) ? graph_period(b) : 0;
  while (per > 0 && nsteps - done >= per) {
    const std::vector<long long> key = phase_key(b);
    if (!b->gexec || b->gperiod != per || key != b->gkey) {
      // capture `per` steps; the host bookkeeping advances as the steps are
      // recorded, and the graph launch below performs them
      b->drop_graph();
      hipGraph_t g = nullptr;
      HIPCHK(hipStreamBeginCapture(b->st, hipStreamCaptureModeThreadLocal));
      int rc = FLB_OK;
      for (long long s = 0; s < per && !rc; s++) rc = batch_one_step<L, S>(b);
      hipError_t e = hipStreamEndCapture(b->st, &g);
      if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
      }
      if (e != hipSuccess) return fail(FLB_EHIP, "graph capture: %s", hipGetErrorString(e));
      e = hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) {
        b->gexec = nullptr;
        return fail(FLB_EHIP, "graph instantiation: %s", hipGetErrorString(e));
      }
      b->gperiod = per;
      b->gkey = key;
    } else {
      for (flb_ctx* c : b->m) c->launched += per;
    }
    HIPCHK(hipGraphLaunch(b->gexec, b->st));
    done += per;
  }
  for (; done < nsteps; done++) {
    int rc = batch_one_step<L, S>(b);
    if (rc) return rc;
  }
  return FLB_OK;
}

#define FLB_BATCH_DISPATCH(b, FN, ...)                                                     \
  ((b)->D == 2 ? ((b)->storage == FLB_F64   ? FN<D2Q9K, SF64>(__VA_ARGS__)                \
                  : (b)->storage == FLB_F32 ? FN<D2Q9K, SF32>(__VA_ARGS__)                \
                                            : FN<D2Q9K, SF16S>(__VA_ARGS__))              \
               : ((b)->storage == FLB_F64   ? FN<D3Q19K, SF64>(__VA_ARGS__)               \
                  : (b)->storage == FLB_F32 ? FN<D3Q19K, SF32>(__VA_ARGS__)               \
                                            : FN<D3Q19K, SF16S>(__VA_ARGS__)))

// Times `reps` launches of the batched step kernel with the current tuning
// without changing any member: each member's launch reads its current buffer
// and writes a scratch buffer, under a copy of its run control.
inline int time_trial(flb_batch* b, int reps, void* const* scratch, Ctl* sctl, float* ms) {
  int rc = rebuild(b);
  if (rc) return rc;
  const int n = (int)b->m.size();
  std::vector<StepArgs> tab(n);
  for (int k = 0; k < n; k++) {
    flb_ctx* c = b->m[k];
    tab[k] = step_args(c);
    Ctl h;
    rc = read_ctl(c, &h);
    if (rc) return rc;
    const int cur = (int)(h.steps & 1);  // the buffer the kernel will read
    tab[k].buf[cur] = c->f[cur];
    tab[k].buf[1 - cur] = scratch[k];
    tab[k].rho = (char*)scratch[k] + c->fbytes;
    tab[k].gas_k = 0;
    tab[k].ctl = sctl + k;
    HIPCHK(hipMemcpyAsync(sctl + k, c->ctl, sizeof(Ctl), hipMemcpyDeviceToDevice, b->st));
  }
  HIPCHK(hipMemcpyAsync(b->tab, tab.data(), sizeof(StepArgs) * n, hipMemcpyHostToDevice, b->st));
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  b->step_fn()(b->tab, b->first, n, b->nblk, b->buf, b->ext, b->st);  // warm-up launch
  hipError_t e = hipEventRecord(e0, b->st);
  for (int r = 0; r < reps && e == hipSuccess; r++) b->step_fn()(b->tab, b->first, n, b->nblk, b->buf, b->ext, b->st);
  if (e == hipSuccess) e = hipEventRecord(e1, b->st);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  b->dirty = true;  // the device table holds the trial arguments
  if (e != hipSuccess) return fail(FLB_EHIP, "autotune timing: %s", hipGetErrorString(e));
  return FLB_OK;
}

}  // namespace flb_rt

namespace flb_rt {

// A batch over existing contexts of one lattice type and storage, which it
// does not own (a server's running jobs).  Tables are built on first use.
inline flb_batch* batch_view(const std::vector<flb_ctx*>& ms, hipStream_t st, const flb_allocator* al) {
  flb_batch* b = new (std::nothrow) flb_batch();
  if (!b) return nullptr;
  b->owns_members = false;
  b->m = ms;
  if (al) {
    b->al = *al;
    b->have_al = true;
  }
  b->st = st;
  b->D = ms[0]->D;
  b->storage = ms[0]->p.storage;
  b->tile = flb_batch::default_tile(b->D);
  b->target = b->D == 2 ? 4096 : 512;
  return b;
}

inline void batch_free(flb_batch* b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->st);
  b->drop_graph();
  for (void* p : b->allocs) {
    if (b->have_al) b->al.free(p, b->al.user);
    else (void)hipFree(p);
  }
  b->allocs.clear();
  delete b;
}

}  // namespace flb_rt
