// batch.hip -- C ABI of batches (flb_batch_* in include/foamlbm.h).
#include "batch.hpp"

using namespace flb_rt;

extern "C" {

int flb_batch_create(const flb_params* params, int32_t count, const flb_allocator* alloc, void* hip_stream,
                     flb_batch** out) {
  g_err.clear();
  if (!out) return fail(FLB_EINVAL, "out is NULL");
  *out = nullptr;
  if (!params || count < 1) return fail(FLB_EINVAL, "need params and count >= 1");
  if (count > (1 << 16)) return fail(FLB_EINVAL, "count must be <= 65536");
  for (int k = 0; k < count; k++) {
    int rc = validate(&params[k]);
    if (rc) {
      const std::string msg = g_err;
      return fail(rc, "member %d: %s", k, msg.c_str());
    }
    if (params[k].lattice != params[0].lattice || params[k].storage != params[0].storage)
      return fail(FLB_EINVAL, "member %d: all members need the same lattice and storage", k);
    if (params[k].model != 0 || params[k].open_z)
      return fail(FLB_EINVAL, "member %d: batches hold periodic single-lattice (model 0) members", k);
  }
  if (alloc && (!alloc->alloc || !alloc->free)) return fail(FLB_EINVAL, "allocator needs alloc and free");
  flb_batch* b = new (std::nothrow) flb_batch();
  if (!b) return fail(FLB_ENOMEM, "host allocation failed");
  if (alloc) {
    b->al = *alloc;
    b->have_al = true;
  }
  b->st = (hipStream_t)hip_stream;
  b->D = params[0].lattice == FLB_D2Q9 ? 2 : 3;
  b->storage = params[0].storage;
  b->tile = flb_batch::default_tile(b->D);
  b->target = b->D == 2 ? 4096 : 512;
  for (int k = 0; k < count; k++) {
    flb_ctx* c = nullptr;
    int rc = flb_create(&params[k], alloc, hip_stream, &c);
    if (rc) {
      const std::string msg = g_err;
      for (flb_ctx* x : b->m) {
        x->in_batch = false;
        flb_destroy(x);
      }
      delete b;
      return fail(rc, "member %d: %s", k, msg.c_str());
    }
    c->in_batch = true;
    b->m.push_back(c);
  }
  *out = b;
  return FLB_OK;
}

void flb_batch_destroy(flb_batch* b) {
  if (!b) return;
  std::vector<flb_ctx*> ms = b->m;
  const bool owns = b->owns_members;
  batch_free(b);
  if (owns)
    for (flb_ctx* c : ms) {
      c->in_batch = false;
      flb_destroy(c);
    }
}

int flb_batch_size(flb_batch* b, int32_t* count) {
  if (!b || !count) return fail(FLB_EINVAL, "NULL argument");
  *count = (int32_t)b->m.size();
  return FLB_OK;
}

int flb_batch_member(flb_batch* b, int32_t k, flb_ctx** out) {
  if (!b || !out) return fail(FLB_EINVAL, "NULL argument");
  if (k < 0 || k >= (int)b->m.size()) return fail(FLB_EINVAL, "member index out of range");
  *out = b->m[k];
  return FLB_OK;
}

int flb_batch_step(flb_batch* b, int64_t nsteps) {
  if (!b) return fail(FLB_EINVAL, "batch is NULL");
  if (nsteps < 0) return fail(FLB_EINVAL, "nsteps must be >= 0");
  return FLB_BATCH_DISPATCH(b, batch_steps, b, nsteps);
}

int flb_batch_set_tuning(flb_batch* b, int32_t tile, int64_t target, int32_t xcd, int32_t graph_steps) {
  if (!b) return fail(FLB_EINVAL, "batch is NULL");
  if (tile < -1 || tile >= b->n_tiles()) return fail(FLB_EINVAL, "tile must be in -1..%d", b->n_tiles() - 1);
  if (target < 0) return fail(FLB_EINVAL, "target must be >= 0");
  if (xcd < -1 || xcd > 64) return fail(FLB_EINVAL, "xcd must be in -1..64");
  if (graph_steps < -1 || graph_steps > 4096) return fail(FLB_EINVAL, "graph_steps must be in -1..4096");
  if (b->persist && tile >= 0 && tile != flb_batch::kPersistTile)
    return fail(FLB_EINVAL, "persistent runs take tile %d", flb_batch::kPersistTile);
  HIPCHK(hipStreamSynchronize(b->st));
  if (tile >= 0) b->tile = tile;
  if (target > 0) b->target = target;
  if (xcd >= 0) b->xcd = xcd;
  if (graph_steps >= 0) b->graph_steps = graph_steps;
  b->dirty = true;
  b->drop_graph();
  return FLB_OK;
}

int flb_batch_set_persistent(flb_batch* b, int32_t on, int32_t max_steps) {
  if (!b) return fail(FLB_EINVAL, "batch is NULL");
  if (on != 0 && on != 1) return fail(FLB_EINVAL, "on must be 0 or 1");
  if (max_steps < 0 || max_steps > 1000000) return fail(FLB_EINVAL, "max_steps must be in 0..1000000");
  if (on && b->D != 2) return fail(FLB_EINVAL, "persistent runs are for D2Q9 batches");
  HIPCHK(hipStreamSynchronize(b->st));
  b->persist = on != 0;
  if (max_steps > 0) b->persist_max = max_steps;
  if (b->persist) b->tile = flb_batch::kPersistTile;
  b->dirty = true;
  b->drop_graph();
  return FLB_OK;
}

int flb_batch_get_tuning(flb_batch* b, int32_t* tile, int64_t* target, int32_t* xcd, int32_t* graph_steps,
                         int32_t* n_tiles) {
  if (!b) return fail(FLB_EINVAL, "batch is NULL");
  if (tile) *tile = b->tile;
  if (target) *target = b->target;
  if (xcd) *xcd = b->xcd;
  if (graph_steps) *graph_steps = b->graph_steps;
  if (n_tiles) *n_tiles = b->n_tiles();
  return FLB_OK;
}

int flb_batch_autotune(flb_batch* b, int32_t reps, double* best_ms) {
  if (!b) return fail(FLB_EINVAL, "batch is NULL");
  if (reps < 1 || reps > 1000) return fail(FLB_EINVAL, "reps must be in 1..1000");
  HIPCHK(hipStreamSynchronize(b->st));
  const int n = (int)b->m.size();
  // one allocation: per member its populations, then its densities (trials
  // keep the member's own), each part 256-byte aligned; the run-control
  // copies at the end
  std::vector<void*> scratch(n, nullptr);
  std::vector<size_t> ofs(n + 1, 0);
  for (int k = 0; k < n; k++) {
    const flb_ctx* c = b->m[k];
    const size_t tsz = c->p.storage == FLB_F64 ? 8 : 4;
    ofs[k + 1] = ofs[k] + ((c->fbytes + tsz * (size_t)c->N + 255) & ~(size_t)255);
  }
  const size_t total = ofs[n] + sizeof(Ctl) * n;
  char* base = (char*)b->dalloc(total);
  Ctl* sctl = base ? (Ctl*)(base + ofs[n]) : nullptr;
  for (int k = 0; k < n && base; k++) scratch[k] = base + ofs[k];
  int rc = base ? FLB_OK
                : fail(FLB_ENOMEM, "autotune scratch allocation of %zu bytes (%d members) failed", total, n);
  const long long targets[] = {256, 512, 1024, 2048, 4096, 8192};
  const int xcds[] = {0, 8};
  float best = 1e30f;
  int bt = b->tile, bx = b->xcd;
  long long bg = b->target;
  // persistent runs keep their tile and tune the rest
  for (int t = 0; t < b->n_tiles() && !rc; t++) {
    if (b->persist && t != flb_batch::kPersistTile) continue;
    for (long long tg : targets)
      for (int xc : xcds) {
        if (rc) break;
        b->tile = t;
        b->target = tg;
        b->xcd = xc;
        float ms = 0.f;
        rc = time_trial(b, reps, scratch.data(), sctl, &ms);
        if (!rc && ms < best) {
          best = ms;
          bt = t;
          bg = tg;
          bx = xc;
        }
      }
  }
  (void)hipStreamSynchronize(b->st);
  b->dfree(base);
  b->tile = bt;
  b->target = bg;
  b->xcd = bx;
  b->dirty = true;
  b->drop_graph();
  if (rc) return rc;
  if (best_ms) *best_ms = best / reps;
  return FLB_OK;
}

int flb_batch_time_steps(flb_batch* b, int64_t nsteps, double* ms) {
  if (!b || !ms) return fail(FLB_EINVAL, "NULL argument");
  if (nsteps < 0) return fail(FLB_EINVAL, "nsteps must be >= 0");
  if (b->dirty) {
    int rc = rebuild(b);
    if (rc) return rc;
  }
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  hipError_t e = hipEventRecord(e0, b->st);
  int rc = FLB_OK;
  if (e == hipSuccess) rc = FLB_BATCH_DISPATCH(b, batch_steps, b, nsteps);
  if (e == hipSuccess && !rc) e = hipEventRecord(e1, b->st);
  if (e == hipSuccess && !rc) e = hipEventSynchronize(e1);
  float f = 0.f;
  if (e == hipSuccess && !rc) e = hipEventElapsedTime(&f, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  if (e != hipSuccess) return fail(FLB_EHIP, "timing: %s", hipGetErrorString(e));
  *ms = f;
  return FLB_OK;
}

}  // extern "C"
