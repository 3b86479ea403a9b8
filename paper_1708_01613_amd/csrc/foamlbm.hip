// foamlbm.hip -- C ABI (include/foamlbm.h) of the gfx950 path: single lattices.
#include <mutex>

#include "runtime.hpp"

using namespace flb_rt;

// ---- the allocation-free histogram's device array ----
// A file-scope array every device holds its own copy of, for the bins of
// flb_get_histogram_noalloc.  In host code `scratch` names a host-side stand-in,
// not a device address: kernels and copies only ever see the address that
// hipGetSymbolAddress returned for the device, kept per device below.
constexpr int kNoAllocMaxBins = 65536;
static __device__ __align__(256) unsigned long long scratch[kNoAllocMaxBins];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned long long* g_scratch[kMaxDevices] = {};

// looks up this device's copy once, with the device current
int scratch_init(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return fail(FLB_EINVAL, "device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch[dev]) return FLB_OK;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) return fail(FLB_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
  g_scratch[dev] = (unsigned long long*)ptr;
  return FLB_OK;
}

unsigned long long* scratch_of(int dev) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return dev >= 0 && dev < kMaxDevices ? g_scratch[dev] : nullptr;
}

// labels of the current state without allocating: the context's query
// tables exist from creation, and every clear is a kernel
template <class L, class S>
int label_query_noalloc(flb_ctx* c) {
  const int B = 256;
  hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(B), 0, c->st, (unsigned long long*)c->qctl,
                     (long long)(sizeof(Ctl) / 8), 0ull);
  return map_pipeline<L, S>(c->qs_pop, c->st, GAS_POP, false);
}
}  // namespace


extern "C" {

void flb_default_params(flb_params* p) {
  if (!p) return;
  memset(p, 0, sizeof *p);
  p->lattice = FLB_D2Q9;
  p->storage = FLB_F32;
  p->nx = 64;
  p->ny = 64;
  p->nz = 1;
  p->tau = 1.0;
  p->G = -5.0;
  p->rho0 = 1.0;
  p->rho_liquid = 2.0;
  p->rho_gas = 0.15;
  p->noise_amp = 0.01;
  p->seed = 1;
  p->film_on = 0;
  p->k_own = 10;
  p->zone_width = 6;
  p->rho_th = log(2.0);
  p->psi_bar_mode = 0;
  p->rupture_warmup = 200;
  p->on_rupture = 0;
  p->velocity_mode = 0;
  p->rupture_filter = 1;
  p->refresh_src = 0;
  p->growth_on = 0;
  p->gas_A = 0.0;
  p->gas_dndt = 0.0;
  p->f16_rho_ref = 1.0;
  p->model = 0;
  p->G_mg = 0.5;
  p->G_gg = 0.0;
  p->tau_g = 1.0;
  p->rho_g_bubble = 0.5;
  p->rho_g_liquid = 0.05;
  p->open_z = 0;
  p->rho_res = 2.0;
}

const char* flb_last_error(void) { return g_err.c_str(); }

int flb_create(const flb_params* p, const flb_allocator* alloc, void* hip_stream, flb_ctx** out) {
  g_err.clear();
  if (!out) return fail(FLB_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = validate(p);
  if (rc) return rc;
  if (alloc && (!alloc->alloc || !alloc->free)) return fail(FLB_EINVAL, "allocator needs alloc and free");
  flb_ctx* c = new (std::nothrow) flb_ctx();
  if (!c) return fail(FLB_ENOMEM, "host allocation failed");
  c->p = *p;
  if (alloc) {
    c->al = *alloc;
    c->have_al = true;
  }
  c->st = (hipStream_t)hip_stream;
  c->D = p->lattice == FLB_D2Q9 ? 2 : 3;
  c->Q = p->lattice == FLB_D2Q9 ? 9 : 19;
  if (c->D == 2) c->md = MapDims{p->nx, 1, p->ny, 0};
  else c->md = MapDims{p->nx, p->ny, p->nz, 0};
  c->N = (long long)p->nx * p->ny * p->nz;
  c->md.N = c->N;
  c->geo.nx = c->md.nx;
  c->geo.nm = c->md.nm;
  c->geo.nz = c->md.nz;
  c->geo.nxb = (c->md.nx + kBlk - 1) / kBlk;
  c->geo.block_bytes = p->storage == FLB_F64   ? block_bytes<SF64>(c->Q)
                       : p->storage == FLB_F32 ? block_bytes<SF32>(c->Q)
                                               : block_bytes<SF16S>(c->Q);
  c->geo.href = (float)p->f16_rho_ref;
  c->fcomp = (size_t)c->geo.nxb * c->md.nm * c->md.nz * c->geo.block_bytes;
  c->ncomp = p->model == 1 ? 2 : 1;
  c->fbytes = c->fcomp * (size_t)c->ncomp;  // with model 1 the gas lattice follows the melt's
  c->nwords = (long long)c->geo.nxb * c->md.nm * c->md.nz;
  default_tuning(c);
  // the largest block count any tile variant can produce (one plane per
  // segment), which sizes the per-workgroup partials
  {
    const int save_tile = c->tile, save_lz = c->lz;
    const int nt = c->D == 2 ? kNTiles2 : kNTiles3;
    c->lz = 1;
    for (int t = 0; t < nt; t++) {
      c->tile = t;
      c->max_blk = std::max(c->max_blk, c->nblocks());
    }
    c->tile = save_tile;
    c->lz = save_lz;
  }
  // the two-lattice kernels and the open container run on the two-pass decomposition
  if (p->model == 1 || p->open_z) c->tile = two_pass_tile(c->D);
  bool ok = true;
  for (int b = 0; b < 2; b++) ok = ok && (c->f[b] = c->dalloc(c->fbytes));
  ok = ok && (c->ctl = (Ctl*)c->dalloc(sizeof(Ctl)));
  ok = ok && (c->qctl = (Ctl*)c->dalloc(sizeof(Ctl)));
  // (and room after them for the folded partials of the two-pass decompositions)
  ok = ok && (c->partials = (double*)c->dalloc(sizeof(double) * 4 * (size_t)(c->max_blk + c->max_blk / FOLD + 1)));
  {
    const size_t tsz = p->storage == FLB_F64 ? 8 : 4;
    ok = ok && (c->psi = c->dalloc(tsz * (size_t)c->N));
    ok = ok && (c->rho = c->dalloc(tsz * (size_t)c->N));
    if (p->model == 1) {
      ok = ok && (c->psi_g = c->dalloc(tsz * (size_t)c->N));
      ok = ok && (c->rho_g = c->dalloc(tsz * (size_t)c->N));
    }
  }
  ok = ok && (c->qd = (double*)c->dalloc(sizeof(double) * 4 * (size_t)c->N));
  ok = ok && (c->qtot = (double*)c->dalloc(sizeof(double) * 4 * 4096));
  ok = ok && (c->par = (int*)c->dalloc(sizeof(int) * (size_t)c->N));
  ok = ok && (c->rank = (int*)c->dalloc(sizeof(int) * (size_t)c->N));
  ok = ok && (c->counts = (int*)c->dalloc(sizeof(int) * (size_t)((c->N + RANK_BLOCK - 1) / RANK_BLOCK + 1)));
  ok = ok && (c->qlabel = (int*)c->dalloc(sizeof(int) * (size_t)c->N));
  ok = ok && (c->qsizes = (unsigned long long*)c->dalloc(sizeof(unsigned long long) * (size_t)(c->N + 1)));
  if (ok && p->film_on) {
    ok = ok && (c->flag = (uint8_t*)c->dalloc((size_t)c->N));
    ok = ok && (c->dist = (uint8_t*)c->dalloc((size_t)c->N));
    ok = ok && (c->mask = (uint32_t*)c->dalloc(sizeof(uint32_t) * (size_t)c->N));
    ok = ok && (c->flist = (int*)c->dalloc(sizeof(int) * (size_t)c->N));
    ok = ok && (c->own = (int2*)c->dalloc(sizeof(int2) * (size_t)c->N));
    ok = ok && (c->label = (int*)c->dalloc(sizeof(int) * (size_t)c->N));
    ok = ok && (c->label_old = (int*)c->dalloc(sizeof(int) * (size_t)c->N));
    ok = ok && (c->alias = (int*)c->dalloc(sizeof(int) * (size_t)(c->N + 1)));
    ok = ok && (c->alias_old = (int*)c->dalloc(sizeof(int) * (size_t)(c->N + 1)));
    ok = ok && (c->rep = (int*)c->dalloc(sizeof(int) * (size_t)(c->N + 1)));
    ok = ok && (c->events = (long long*)c->dalloc(sizeof(long long) * 4 * (size_t)c->ev_cap));
    ok = ok && (c->bits = (unsigned long long*)c->dalloc(sizeof(unsigned long long) * (size_t)c->nwords));
    ok = ok && (c->bfw = (unsigned long long*)c->dalloc(3 * sizeof(unsigned long long) * (size_t)c->nwords));
  }
  if (ok && p->growth_on)
    ok = ok && (c->srcw = (unsigned long long*)c->dalloc(sizeof(unsigned long long) * (size_t)c->nwords));
  if (!ok) {
    c->dfree_all();
    delete c;
    return fail(FLB_ENOMEM, "device allocation failed");
  }
  static_assert(sizeof(Ctl) % 8 == 0, "the run control is cleared as 64-bit words");
  if (hipGetDevice(&c->dev) != hipSuccess || scratch_init(c->dev) != FLB_OK) {
    c->dfree_all();
    delete c;
    return g_err.empty() ? fail(FLB_EHIP, "hipGetDevice failed") : FLB_EHIP;
  }
  if (hipMemsetAsync(c->ctl, 0, sizeof(Ctl), c->st) != hipSuccess ||
      hipMemsetAsync(c->qctl, 0, sizeof(Ctl), c->st) != hipSuccess ||
      (p->film_on && hipMemsetAsync(c->flag, 0, (size_t)c->N, c->st) != hipSuccess) ||
      (p->film_on && hipMemsetAsync(c->mask, 0, sizeof(uint32_t) * (size_t)c->N, c->st) != hipSuccess) ||
      (p->growth_on && hipMemsetAsync(c->srcw, 0, sizeof(unsigned long long) * (size_t)c->nwords, c->st) != hipSuccess) ||
      forget_rho(c) != FLB_OK || hipStreamSynchronize(c->st) != hipSuccess) {
    c->dfree_all();
    delete c;
    return fail(FLB_EHIP, "initialising device state failed");
  }
  // the map tables of queries and refreshes, built now so later calls need no allocation
  rc = ctx_mapsets(c);
  if (rc) {
    c->dfree_all();
    delete c;
    return rc;
  }
  *out = c;
  return FLB_OK;
}

void flb_destroy(flb_ctx* c) {
  if (!c || c->in_batch) return;
  (void)hipStreamSynchronize(c->st);
  c->dfree_all();
  delete c;
}

int flb_set_nuclei(flb_ctx* c, const flb_nucleus* nuc, int32_t n) {
  if (!c) return fail(FLB_EINVAL, "ctx is NULL");
  if (n < 0 || (n > 0 && !nuc)) return fail(FLB_EINVAL, "bad nuclei array");
  for (int k = 0; k < n; k++)
    if (!isfinite(nuc[k].x) || !isfinite(nuc[k].y) || !isfinite(nuc[k].z) || !isfinite(nuc[k].r))
      return fail(FLB_EINVAL, "non-finite nucleus %d", k);
  double4* dn = nullptr;
  if (n > 0) {
    dn = (double4*)c->dalloc(sizeof(double4) * (size_t)n);
    if (!dn) return fail(FLB_ENOMEM, "nuclei allocation failed");
    HIPCHK(hipMemcpyAsync(dn, nuc, sizeof(double4) * (size_t)n, hipMemcpyHostToDevice, c->st));
  }
  HIPCHK(hipMemsetAsync(c->ctl, 0, sizeof(Ctl), c->st));
  if (forget_rho(c)) return FLB_EHIP;
  // the nucleus cells become the domain gas points of the gas-release source;
  // their count goes to the run control
  unsigned long long* nsrc = (unsigned long long*)c->qtot;
  if (c->srcw) {
    HIPCHK(hipMemsetAsync(c->srcw, 0, sizeof(unsigned long long) * (size_t)c->nwords, c->st));
    HIPCHK(hipMemsetAsync(nsrc, 0, sizeof(unsigned long long), c->st));
  }
  const int B = 256, g = grid_for(c->N, B);
  hipLaunchKernelGGL(k_init_density, dim3(g), dim3(B), 0, c->st, c->qd, c->p.nx, c->p.ny, c->p.nz, c->N, dn, n,
                     c->p.rho_liquid, c->p.rho_gas, c->p.noise_amp, (unsigned long long)c->p.seed, c->srcw,
                     c->geo.nxb, nsrc);
  HIPCHK(hipGetLastError());
  if (c->srcw)
    HIPCHK(hipMemcpyAsync(&c->ctl->n_src, nsrc, sizeof(long long), hipMemcpyDeviceToDevice, c->st));
  int rc = FLB_DISPATCH(c, do_pack, c, c->qd, 0, 0);
  if (rc) return rc;
  if (c->p.model == 1) {  // the gas lattice: rho_g_bubble in the nuclei, rho_g_liquid elsewhere, no noise
    hipLaunchKernelGGL(k_init_density, dim3(g), dim3(B), 0, c->st, c->qd, c->p.nx, c->p.ny, c->p.nz, c->N, dn, n,
                       c->p.rho_g_liquid, c->p.rho_g_bubble, 0.0, (unsigned long long)c->p.seed, nullptr,
                       c->geo.nxb, nullptr);
    HIPCHK(hipGetLastError());
    rc = FLB_DISPATCH(c, do_pack, c, c->qd, 0, 0, 1);
    if (rc) return rc;
  }
  HIPCHK(hipStreamSynchronize(c->st));
  c->dfree(dn);
  c->launched = 0;
  if (c->p.film_on) {
    HIPCHK(hipMemsetAsync(c->flag, 0, (size_t)c->N, c->st));
    HIPCHK(hipMemsetAsync(c->mask, 0, sizeof(uint32_t) * (size_t)c->N, c->st));
  }
  return FLB_OK;
}

int flb_step(flb_ctx* c, int64_t nsteps) {
  if (!c) return fail(FLB_EINVAL, "ctx is NULL");
  if (nsteps < 0) return fail(FLB_EINVAL, "nsteps must be >= 0");
  return FLB_DISPATCH(c, do_steps, c, nsteps, true);
}

// Runs nsteps steps with optional per-phase events (kPhaseEv per step).
static int timed_steps(flb_ctx* c, int64_t nsteps, bool refresh, bool phases, double* ms, double ph[4]) {
  std::vector<hipEvent_t> kev(phases ? kPhaseEv * (size_t)nsteps : 0, nullptr);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  for (size_t k = 0; k < kev.size() && e == hipSuccess; k++) e = hipEventCreate(&kev[k]);
  int rc = FLB_OK;
  if (e == hipSuccess) e = hipEventRecord(e0, c->st);
  if (e == hipSuccess) rc = FLB_DISPATCH(c, do_steps, c, nsteps, refresh, phases ? kev.data() : nullptr);
  if (e == hipSuccess && !rc) e = hipEventRecord(e1, c->st);
  if (e == hipSuccess && !rc) e = hipEventSynchronize(e1);
  float f = 0.f;
  if (e == hipSuccess && !rc) e = hipEventElapsedTime(&f, e0, e1);
  double sum[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t s = 0; s < nsteps && phases && e == hipSuccess && !rc; s++)
    for (int q = 0; q < 4 && e == hipSuccess; q++) {
      float a = 0.f;
      e = hipEventElapsedTime(&a, kev[kPhaseEv * s + q], kev[kPhaseEv * s + q + 1]);
      sum[q] += (double)a;
    }
  for (hipEvent_t ev : kev)
    if (ev) (void)hipEventDestroy(ev);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (rc) return rc;
  if (e != hipSuccess) return fail(FLB_EHIP, "timing: %s", hipGetErrorString(e));
  *ms = f;
  if (ph)
    for (int q = 0; q < 4; q++) ph[q] = sum[q];
  return FLB_OK;
}

int flb_time_steps(flb_ctx* c, int64_t nsteps, int32_t refresh, double* ms, double* kernel_ms) {
  if (!c || !ms) return fail(FLB_EINVAL, "NULL argument");
  if (nsteps < 0) return fail(FLB_EINVAL, "nsteps must be >= 0");
  if (kernel_ms && nsteps > 100000) return fail(FLB_EINVAL, "nsteps must be <= 100000 with kernel_ms");
  double ph[4];
  int rc = timed_steps(c, nsteps, refresh != 0, kernel_ms != nullptr, ms, ph);
  if (!rc && kernel_ms) *kernel_ms = ph[1];
  return rc;
}

int flb_time_phases(flb_ctx* c, int64_t nsteps, double* ms, double* phase_ms) {
  if (!c || !ms || !phase_ms) return fail(FLB_EINVAL, "NULL argument");
  if (nsteps < 0 || nsteps > 100000) return fail(FLB_EINVAL, "nsteps must be in 0..100000");
  return timed_steps(c, nsteps, true, true, ms, phase_ms);
}

int flb_set_tuning(flb_ctx* c, int32_t tile, int32_t lz, int32_t xcd) {
  if (!c) return fail(FLB_EINVAL, "ctx is NULL");
  const int nt = c->D == 2 ? kNTiles2 : kNTiles3;
  if (tile < -1 || tile >= nt) return fail(FLB_EINVAL, "tile must be in -1..%d", nt - 1);
  if (lz < 0) return fail(FLB_EINVAL, "lz must be >= 0");
  if (xcd < -1 || xcd > 64) return fail(FLB_EINVAL, "xcd must be in -1..64");
  if ((c->p.model == 1 || c->p.open_z) && tile >= 0 && tile != two_pass_tile(c->D))
    return fail(FLB_EINVAL, "model 1 and the open container run on the two-pass path (tile %d)", two_pass_tile(c->D));
  HIPCHK(hipStreamSynchronize(c->st));
  if (tile >= 0) c->tile = tile;
  if (lz > 0) c->lz = std::min(lz, c->md.nz);
  if (xcd >= 0) c->xcd = xcd;
  if (c->nblocks() > c->max_blk) return fail(FLB_EINVAL, "tuning exceeds the partials capacity");
  return FLB_OK;
}

int flb_autotune(flb_ctx* c, int32_t reps, double* best_ms) {
  if (!c) return fail(FLB_EINVAL, "ctx is NULL");
  if (reps < 1 || reps > 1000) return fail(FLB_EINVAL, "reps must be in 1..1000");
  if (c->p.model == 1 || c->p.open_z) {  // one decomposition: nothing to choose
    if (best_ms) *best_ms = 0.0;
    return FLB_OK;
  }
  Ctl h;
  int rc = read_ctl(c, &h);
  if (rc) return rc;
  const int cur = (int)(h.steps & 1);
  // trials write their populations to a scratch buffer and their densities
  // after it, so the state and the densities kept for the next refresh stay
  const size_t tsz = c->p.storage == FLB_F64 ? 8 : 4;
  void* scratch = c->dalloc(c->fbytes + tsz * (size_t)c->N);
  Ctl* sctl = (Ctl*)c->dalloc(sizeof(Ctl));
  if (!scratch || !sctl) {
    c->dfree(scratch);
    c->dfree(sctl);
    return fail(FLB_ENOMEM, "autotune scratch allocation failed");
  }
  const int save_tile = c->tile, save_lz = c->lz, save_xcd = c->xcd;
  int bt = save_tile, bl = save_lz, bx = save_xcd;
  float best = 1e30f;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  const int nt = c->D == 2 ? kNTiles2 : kNTiles3;
  const int lzs[] = {8, 16, 32, 64, 128, 256, 512};
  for (int t = 0; t < nt && e == hipSuccess; t++) {
    c->tile = t;
    std::vector<int> cand;
    if (c->two_pass() || c->tcfg().fh) cand.push_back(c->md.nz);  // the segment length is fixed
    else
      for (int l : lzs) cand.push_back(std::min(l, c->md.nz));
    cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
    for (int lz : cand)
      for (int xc : {0, 8}) {
        if (e != hipSuccess) break;
        c->lz = lz;
        c->xcd = xc;
        const int nblk = c->nblocks();
        if (nblk > c->max_blk) continue;
        StepArgs a = step_args(c);
        a.buf[cur] = c->f[cur];
        a.buf[1 - cur] = scratch;
        a.rho = (char*)scratch + c->fbytes;
        a.gas_k = 0;
        a.ctl = sctl;
        e = hipMemcpyAsync(sctl, c->ctl, sizeof(Ctl), hipMemcpyDeviceToDevice, c->st);
        const StepFn fn = c->tcfg().fn[c->p.storage], coll = c->tcfg().coll[c->p.storage];
        auto launch = [&]() {
          fn(a, nblk, c->st);
          if (coll) coll(a, nblk, c->st);
        };
        if (e == hipSuccess) launch();  // warm-up
        if (e == hipSuccess) e = hipEventRecord(e0, c->st);
        for (int r = 0; r < reps && e == hipSuccess; r++) launch();
        if (e == hipSuccess) e = hipEventRecord(e1, c->st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e == hipSuccess && ms < best) {
          best = ms;
          bt = t;
          bl = lz;
          bx = xc;
        }
      }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(c->st);
  c->dfree(scratch);
  c->dfree(sctl);
  c->tile = bt;
  c->lz = bl;
  c->xcd = bx;
  if (e != hipSuccess) {
    c->tile = save_tile;
    c->lz = save_lz;
    c->xcd = save_xcd;
    return fail(FLB_EHIP, "autotune: %s", hipGetErrorString(e));
  }
  if (best_ms) *best_ms = best / reps;
  return FLB_OK;
}

int flb_get_tuning(flb_ctx* c, int32_t* tile, int32_t* lz, int32_t* xcd, int32_t* n_tiles, int32_t* tile_x,
                   int32_t* tile_m) {
  if (!c) return fail(FLB_EINVAL, "ctx is NULL");
  if (tile) *tile = c->tile;
  if (lz) *lz = c->lz;
  if (xcd) *xcd = c->xcd;
  if (n_tiles) *n_tiles = c->D == 2 ? kNTiles2 : kNTiles3;
  if (tile_x) *tile_x = c->tcfg().tx;
  if (tile_m) *tile_m = c->tcfg().tm;
  return FLB_OK;
}

int flb_get_labels(flb_ctx* c, int32_t* out, size_t n, int32_t* n_bubbles) {
  if (!c || !out) return fail(FLB_EINVAL, "NULL argument");
  if (n != (size_t)c->N) return fail(FLB_EINVAL, "n must be nx*ny*nz = %lld", c->N);
  int rc = FLB_DISPATCH(c, label_query, c, false);
  if (rc) return rc;
  int nb = 0;
  HIPCHK(hipMemcpyAsync(out, c->qlabel, sizeof(int) * n, hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipMemcpyAsync(&nb, &c->qctl->n_bubbles, sizeof(int), hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipStreamSynchronize(c->st));
  if (n_bubbles) *n_bubbles = nb;
  return FLB_OK;
}

int flb_label_field(flb_ctx* c, const double* rho, size_t n, int32_t* out, int32_t* n_bubbles) {
  if (!c || !rho || !out) return fail(FLB_EINVAL, "NULL argument");
  if (n != (size_t)c->N) return fail(FLB_EINVAL, "n must be nx*ny*nz = %lld", c->N);
  HIPCHK(hipMemcpyAsync(c->qd, rho, sizeof(double) * n, hipMemcpyHostToDevice, c->st));
  int rc = FLB_DISPATCH(c, label_query, c, true);
  if (rc) return rc;
  int nb = 0;
  HIPCHK(hipMemcpyAsync(out, c->qlabel, sizeof(int) * n, hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipMemcpyAsync(&nb, &c->qctl->n_bubbles, sizeof(int), hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipStreamSynchronize(c->st));
  if (n_bubbles) *n_bubbles = nb;
  return FLB_OK;
}

int flb_get_maps(flb_ctx* c, int32_t* label, int32_t* owner, int32_t* owner2, int32_t* dist, uint32_t* mask,
                 size_t n) {
  if (!c) return fail(FLB_EINVAL, "ctx is NULL");
  if (!c->p.film_on) return fail(FLB_EINVAL, "film maps exist only with film_on");
  if (n != (size_t)c->N) return fail(FLB_EINVAL, "n must be nx*ny*nz = %lld", c->N);
  if (owner || owner2 || dist) {
    const int rc = c->D == 2 ? complete_maps<D2Q9K>(c) : complete_maps<D3Q19K>(c);
    if (rc) return rc;
  }
  if (label) HIPCHK(hipMemcpyAsync(label, c->label, sizeof(int) * n, hipMemcpyDeviceToHost, c->st));
  if (mask) HIPCHK(hipMemcpyAsync(mask, c->mask, sizeof(uint32_t) * n, hipMemcpyDeviceToHost, c->st));
  std::vector<int2> own;
  std::vector<uint8_t> d8;
  if (owner || owner2) {
    own.resize(n);
    HIPCHK(hipMemcpyAsync(own.data(), c->own, sizeof(int2) * n, hipMemcpyDeviceToHost, c->st));
  }
  if (owner || owner2 || dist) {  // unreached cells (dist 255) have no owners
    d8.resize(n);
    HIPCHK(hipMemcpyAsync(d8.data(), c->dist, n, hipMemcpyDeviceToHost, c->st));
  }
  HIPCHK(hipStreamSynchronize(c->st));
  for (size_t k = 0; k < n; k++) {
    if (owner) owner[k] = d8[k] == 255 ? 0 : own[k].x;
    if (owner2) owner2[k] = d8[k] == 255 ? 0 : own[k].y;
    if (dist) dist[k] = d8[k] == 255 ? -1 : d8[k];
    if (mask) mask[k] &= kLinkBits;  // link bits only
  }
  return FLB_OK;
}

int flb_get_histogram(flb_ctx* c, int32_t nbins, double bin_width, int64_t* counts, int32_t* n_bubbles) {
  if (!c || !counts) return fail(FLB_EINVAL, "NULL argument");
  if (nbins < 1 || nbins > (1 << 20)) return fail(FLB_EINVAL, "nbins must be in 1..2^20");
  if (!(bin_width > 0) || !isfinite(bin_width)) return fail(FLB_EINVAL, "bin_width must be > 0");
  if (nbins > c->qhist_cap) {
    c->qhist = (unsigned long long*)c->dalloc(sizeof(unsigned long long) * (size_t)nbins);
    if (!c->qhist) return fail(FLB_ENOMEM, "histogram allocation failed");
    c->qhist_cap = nbins;
  }
  int rc = FLB_DISPATCH(c, label_query, c, false);
  if (rc) return rc;
  HIPCHK(hipMemsetAsync(c->qsizes, 0, sizeof(unsigned long long) * (size_t)(c->N + 1), c->st));
  HIPCHK(hipMemsetAsync(c->qhist, 0, sizeof(unsigned long long) * (size_t)nbins, c->st));
  const int B = 256;
  hipLaunchKernelGGL(k_label_sizes, dim3(grid_for(c->N, B)), dim3(B), 0, c->st, c->qlabel, c->N, c->qsizes);
  hipLaunchKernelGGL(k_histogram, dim3(grid_for(c->N, B)), dim3(B), 0, c->st, c->qsizes, &c->qctl->n_bubbles, c->D,
                     nbins, bin_width, c->qhist);
  HIPCHK(hipGetLastError());
  std::vector<unsigned long long> h(nbins);
  int nb = 0;
  HIPCHK(hipMemcpyAsync(h.data(), c->qhist, sizeof(unsigned long long) * (size_t)nbins, hipMemcpyDeviceToHost,
                        c->st));
  HIPCHK(hipMemcpyAsync(&nb, &c->qctl->n_bubbles, sizeof(int), hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipStreamSynchronize(c->st));
  for (int k = 0; k < nbins; k++) counts[k] = (int64_t)h[k];
  if (n_bubbles) *n_bubbles = nb;
  return FLB_OK;
}

int flb_get_foam_stats(flb_ctx* c, flb_foam_stats* out) {
  if (!c || !out) return fail(FLB_EINVAL, "NULL argument");
  int rc = FLB_DISPATCH(c, label_query, c, false);
  if (rc) return rc;
  const int B = 256;
  hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(c->N + 1, B)), dim3(B), 0, c->st, c->qsizes, c->N + 1, 0ull);
  hipLaunchKernelGGL(k_label_sizes, dim3(grid_for(c->N, B)), dim3(B), 0, c->st, c->qlabel, c->N, c->qsizes);
  hipLaunchKernelGGL(k_foam_stats, dim3(1), dim3(FS_NT), 0, c->st, c->qsizes, &c->qctl->n_bubbles, c->D, c->N,
                     c->qtot);
  HIPCHK(hipGetLastError());
  double v[5];
  int nb = 0;
  HIPCHK(hipMemcpyAsync(v, c->qtot, sizeof v, hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipMemcpyAsync(&nb, &c->qctl->n_bubbles, sizeof(int), hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipStreamSynchronize(c->st));
  out->n_bubbles = nb;
  out->gas_cells = (int64_t)v[4];
  out->gas_fraction = v[0];
  out->relative_density = v[1];
  out->mean_diameter = v[2];
  out->max_diameter = v[3];
  return FLB_OK;
}

int flb_get_histogram_noalloc(flb_ctx* c, int32_t nbins, double bin_width, int64_t* counts, int32_t* n_bubbles) {
  if (!c || !counts) return fail(FLB_EINVAL, "NULL argument");
  if (nbins < 1 || nbins > kNoAllocMaxBins)
    return fail(FLB_EINVAL, "nbins must be in 1..%d (the allocation-free maximum)", kNoAllocMaxBins);
  if (!(bin_width > 0) || !isfinite(bin_width)) return fail(FLB_EINVAL, "bin_width must be > 0");
  if (!c->ms_ready) return fail(FLB_EINVAL, "context has no query tables");
  unsigned long long* bins = scratch_of(c->dev);
  if (!bins) return fail(FLB_EINVAL, "device %d has no histogram array (no context created on it)", c->dev);
  int rc = FLB_DISPATCH(c, label_query_noalloc, c);
  if (rc) return rc;
  const int B = 256;
  hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(c->N + 1, B)), dim3(B), 0, c->st, c->qsizes, c->N + 1, 0ull);
  hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(nbins, B)), dim3(B), 0, c->st, bins, (long long)nbins, 0ull);
  hipLaunchKernelGGL(k_label_sizes, dim3(grid_for(c->N, B)), dim3(B), 0, c->st, c->qlabel, c->N, c->qsizes);
  hipLaunchKernelGGL(k_histogram, dim3(grid_for(c->N, B)), dim3(B), 0, c->st, c->qsizes, &c->qctl->n_bubbles, c->D,
                     nbins, bin_width, bins);
  HIPCHK(hipGetLastError());
  static_assert(sizeof(int64_t) == sizeof(unsigned long long), "bins copy straight into the caller's counts");
  int nb = 0;
  HIPCHK(hipMemcpyAsync(counts, bins, sizeof(unsigned long long) * (size_t)nbins, hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipMemcpyAsync(&nb, &c->qctl->n_bubbles, sizeof(int), hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipStreamSynchronize(c->st));
  if (n_bubbles) *n_bubbles = nb;
  return FLB_OK;
}

int flb_match_labels(flb_ctx* c, const int32_t* old_labels, size_t n, int64_t* pairs, int64_t cap, int64_t* n_pairs,
                     int32_t* n_bubbles) {
  if (!c || !old_labels || !n_pairs || (cap > 0 && !pairs)) return fail(FLB_EINVAL, "NULL argument");
  if (n != (size_t)c->N) return fail(FLB_EINVAL, "n must be nx*ny*nz = %lld", c->N);
  if (cap < 0) return fail(FLB_EINVAL, "cap must be >= 0");
  long long n_old = 0;
  for (size_t k = 0; k < n; k++) {
    if (old_labels[k] < 0) return fail(FLB_EINVAL, "old_labels[%zu] = %d is negative", k, old_labels[k]);
    n_old = std::max<long long>(n_old, old_labels[k]);
  }
  int rc = FLB_DISPATCH(c, label_query, c, false);
  if (rc) return rc;
  int nb = 0;
  HIPCHK(hipMemcpyAsync(&nb, &c->qctl->n_bubbles, sizeof(int), hipMemcpyDeviceToHost, c->st));
  int* dold = (int*)c->qd;  // the query field buffer (4 N doubles) holds the old labels
  int* dflag = (int*)(c->qd + c->N);
  HIPCHK(hipMemcpyAsync(dold, old_labels, sizeof(int) * n, hipMemcpyHostToDevice, c->st));
  HIPCHK(hipStreamSynchronize(c->st));
  // a table of at least twice the pairs two labellings of this size usually
  // overlap in; doubled until every pair finds a slot
  long long want = 1024;
  while (want < 2 * (n_old + nb) + 1024) want *= 2;
  std::vector<unsigned long long> hk, hc;
  for (;;) {
    if (want > c->qtab_cap) {
      c->qtab = (unsigned long long*)c->dalloc(sizeof(unsigned long long) * 2 * (size_t)want);
      if (!c->qtab) return fail(FLB_ENOMEM, "label-overlap table allocation failed");
      c->qtab_cap = want;
    }
    unsigned long long* keys = c->qtab;
    unsigned long long* counts = c->qtab + want;
    HIPCHK(hipMemsetAsync(keys, 0xff, sizeof(unsigned long long) * (size_t)want, c->st));
    HIPCHK(hipMemsetAsync(counts, 0, sizeof(unsigned long long) * (size_t)want, c->st));
    HIPCHK(hipMemsetAsync(dflag, 0, sizeof(int), c->st));
    hipLaunchKernelGGL(k_match_pairs, dim3(grid_for(c->N, 256)), dim3(256), 0, c->st, dold, c->qlabel, c->N, keys,
                       counts, (unsigned)(want - 1), dflag);
    HIPCHK(hipGetLastError());
    int over = 0;
    hk.resize((size_t)want);
    hc.resize((size_t)want);
    HIPCHK(hipMemcpyAsync(hk.data(), keys, sizeof(unsigned long long) * (size_t)want, hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipMemcpyAsync(hc.data(), counts, sizeof(unsigned long long) * (size_t)want, hipMemcpyDeviceToHost,
                          c->st));
    HIPCHK(hipMemcpyAsync(&over, dflag, sizeof(int), hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    if (!over) break;
    if (want >= (long long)1 << 31) return fail(FLB_ENOMEM, "label-overlap table would exceed 2^31 slots");
    want *= 2;
  }
  std::vector<std::pair<unsigned long long, unsigned long long>> found;
  for (size_t k = 0; k < hk.size(); k++)
    if (hk[k] != kMatchEmpty) found.emplace_back(hk[k], hc[k]);
  std::sort(found.begin(), found.end());
  const int64_t m = (int64_t)found.size();
  for (int64_t k = 0; k < std::min(m, cap); k++) {
    pairs[3 * k] = (int64_t)(found[k].first >> 32);
    pairs[3 * k + 1] = (int64_t)(found[k].first & 0xffffffffu);
    pairs[3 * k + 2] = (int64_t)found[k].second;
  }
  *n_pairs = m;
  if (n_bubbles) *n_bubbles = nb;
  return FLB_OK;
}

int flb_get_rupture_events(flb_ctx* c, int64_t* out, int64_t cap, int64_t* n) {
  if (!c || !n || (cap > 0 && !out)) return fail(FLB_EINVAL, "NULL argument");
  if (cap < 0) return fail(FLB_EINVAL, "cap must be >= 0");
  Ctl h;
  int rc = read_ctl(c, &h);
  if (rc) return rc;
  *n = c->p.film_on ? (int64_t)std::min<unsigned>(h.ev_count, c->ev_cap) : 0;
  const int64_t have = std::min<int64_t>(*n, c->ev_cap);
  const int64_t m = std::min<int64_t>(have, cap);
  if (m > 0) {
    std::vector<long long> ev(4 * (size_t)m);
    HIPCHK(hipMemcpyAsync(ev.data(), c->events, sizeof(long long) * 4 * (size_t)m, hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    for (int64_t k = 0; k < m; k++)
      for (int q = 0; q < 3; q++) out[3 * k + q] = ev[4 * k + q];
  }
  return FLB_OK;
}

int flb_get_density(flb_ctx* c, double* out, size_t n) {
  if (!c || !out) return fail(FLB_EINVAL, "NULL argument");
  if (n != (size_t)c->N) return fail(FLB_EINVAL, "n must be nx*ny*nz = %lld", c->N);
  int rc = FLB_DISPATCH(c, do_moments, c, false);
  if (rc) return rc;
  HIPCHK(hipMemcpyAsync(out, c->qd, sizeof(double) * n, hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipStreamSynchronize(c->st));
  return FLB_OK;
}

int flb_get_gas_density(flb_ctx* c, double* out, size_t n) {
  if (!c || !out) return fail(FLB_EINVAL, "NULL argument");
  if (c->p.model != 1) return fail(FLB_EINVAL, "the gas lattice exists only with model 1");
  if (n != (size_t)c->N) return fail(FLB_EINVAL, "n must be nx*ny*nz = %lld", c->N);
  int rc = FLB_DISPATCH(c, do_moments, c, false, 1);
  if (rc) return rc;
  HIPCHK(hipMemcpyAsync(out, c->qd, sizeof(double) * n, hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipStreamSynchronize(c->st));
  return FLB_OK;
}

// model 1: the mixture's velocity (what 1) or the two-component pressure
// (what 0) from the FP64 moments of both lattices
static int tl_query(flb_ctx* c, int what, double* out, size_t n) {
  const size_t planes = 1 + (size_t)c->D;
  double* gm = (double*)c->dalloc(sizeof(double) * (planes * (size_t)c->N + n));
  if (!gm) return fail(FLB_ENOMEM, "query scratch allocation failed");
  double* res = gm + planes * (size_t)c->N;
  int rc = FLB_DISPATCH(c, do_moments, c, true, 0);
  if (!rc) rc = FLB_DISPATCH(c, do_moments, c, true, 1, gm);
  hipError_t e = hipSuccess;
  if (!rc) {
    const int B = 256, g = grid_for(c->N, B);
    StepArgs a = step_args(c);
    TLArgs t = tl_args(c);
    if (c->D == 2)
      hipLaunchKernelGGL((k_tl_query<D2Q9K>), dim3(g), dim3(B), 0, c->st, a, t, c->md, c->qd, gm, what,
                         c->p.velocity_mode, res);
    else
      hipLaunchKernelGGL((k_tl_query<D3Q19K>), dim3(g), dim3(B), 0, c->st, a, t, c->md, c->qd, gm, what,
                         c->p.velocity_mode, res);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(out, res, sizeof(double) * n, hipMemcpyDeviceToHost, c->st);
    if (e == hipSuccess) e = hipStreamSynchronize(c->st);
  }
  c->dfree(gm);
  if (rc) return rc;
  if (e != hipSuccess) return fail(FLB_EHIP, "two-lattice query: %s", hipGetErrorString(e));
  return FLB_OK;
}

int flb_get_velocity(flb_ctx* c, double* out, size_t n) {
  if (!c || !out) return fail(FLB_EINVAL, "NULL argument");
  if (n != (size_t)c->D * c->N) return fail(FLB_EINVAL, "n must be D*nx*ny*nz = %lld", c->D * c->N);
  if (c->p.model == 1) return tl_query(c, 1, out, n);
  int rc = FLB_DISPATCH(c, do_moments, c, true);
  if (rc) return rc;
  double* vel = (double*)c->dalloc(sizeof(double) * n);
  if (!vel) return fail(FLB_ENOMEM, "velocity scratch allocation failed");
  const int B = 256, g = grid_for(c->N, B);
  StepArgs a = step_args(c);
  if (c->D == 2)
    hipLaunchKernelGGL((k_velocity<D2Q9K>), dim3(g), dim3(B), 0, c->st, a, c->md, c->qd, c->qd + c->N,
                       c->p.velocity_mode, vel);
  else
    hipLaunchKernelGGL((k_velocity<D3Q19K>), dim3(g), dim3(B), 0, c->st, a, c->md, c->qd, c->qd + c->N,
                       c->p.velocity_mode, vel);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(out, vel, sizeof(double) * n, hipMemcpyDeviceToHost, c->st);
  if (e == hipSuccess) e = hipStreamSynchronize(c->st);
  c->dfree(vel);
  if (e != hipSuccess) return fail(FLB_EHIP, "velocity query: %s", hipGetErrorString(e));
  return FLB_OK;
}

int flb_copy_bandwidth(const flb_allocator* alloc, void* hip_stream, int64_t bytes, int32_t reps, double* gbs) {
  if (!gbs) return fail(FLB_EINVAL, "NULL argument");
  if (bytes < (1 << 20) || bytes > (1ll << 36) || bytes % 16) return fail(FLB_EINVAL, "bytes must be a multiple of 16 in 2^20..2^36");
  if (reps < 1 || reps > 1000) return fail(FLB_EINVAL, "reps must be in 1..1000");
  if (alloc && (!alloc->alloc || !alloc->free)) return fail(FLB_EINVAL, "allocator needs alloc and free");
  hipStream_t st = (hipStream_t)hip_stream;
  void* buf[2] = {nullptr, nullptr};
  for (int k = 0; k < 2; k++) {
    if (alloc) buf[k] = alloc->alloc((size_t)bytes, alloc->user);
    else if (hipMalloc(&buf[k], (size_t)bytes) != hipSuccess) buf[k] = nullptr;
  }
  auto release = [&]() {
    for (int k = 0; k < 2; k++)
      if (buf[k]) {
        if (alloc) alloc->free(buf[k], alloc->user);
        else (void)hipFree(buf[k]);
      }
  };
  if (!buf[0] || !buf[1]) {
    release();
    return fail(FLB_ENOMEM, "copy buffers allocation failed");
  }
  const long long n = bytes / 16;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) e = hipMemsetAsync(buf[0], 0, (size_t)bytes, st);
  double best = 0.0;
  for (int grid : {8192, 32768}) {
    if (e != hipSuccess) break;
    auto launch = [&]() {
      hipLaunchKernelGGL(k_copy16<4>, dim3(grid), dim3(256), 0, st, (const f4v*)buf[0], (f4v*)buf[1], n);
    };
    launch();  // warm-up
    e = hipEventRecord(e0, st);
    for (int r = 0; r < reps && e == hipSuccess; r++) launch();
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess && ms > 0.f) best = std::max(best, 2.0 * (double)bytes * reps / ((double)ms * 1e6));
  }
  if (e == hipSuccess) e = hipGetLastError();
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(st);
  release();
  if (e != hipSuccess) return fail(FLB_EHIP, "copy bandwidth: %s", hipGetErrorString(e));
  *gbs = best;
  return FLB_OK;
}

int flb_get_pressure(flb_ctx* c, double* out, size_t n) {
  if (!c || !out) return fail(FLB_EINVAL, "NULL argument");
  if (n != (size_t)c->N) return fail(FLB_EINVAL, "n must be nx*ny*nz = %lld", c->N);
  if (c->p.model == 1) return tl_query(c, 0, out, n);
  int rc = FLB_DISPATCH(c, do_moments, c, false);
  if (rc) return rc;
  const int B = 256, g = grid_for(c->N, B);
  hipLaunchKernelGGL(k_pressure, dim3(g), dim3(B), 0, c->st, c->qd, c->N, c->p.G, c->p.rho0, c->qd + c->N);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(out, c->qd + c->N, sizeof(double) * n, hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipStreamSynchronize(c->st));
  return FLB_OK;
}

int flb_get_gas_points(flb_ctx* c, uint8_t* out, size_t n, int64_t* n_points) {
  if (!c || !n_points) return fail(FLB_EINVAL, "NULL argument");
  if (out && n != (size_t)c->N) return fail(FLB_EINVAL, "n must be nx*ny*nz = %lld", c->N);
  Ctl h;
  int rc = read_ctl(c, &h);
  if (rc) return rc;
  *n_points = c->srcw ? h.n_src : 0;
  if (!out) return FLB_OK;
  if (!c->srcw) {
    memset(out, 0, n);
    return FLB_OK;
  }
  std::vector<unsigned long long> w((size_t)c->nwords);
  HIPCHK(hipMemcpyAsync(w.data(), c->srcw, sizeof(unsigned long long) * w.size(), hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipStreamSynchronize(c->st));
  const int nx = c->p.nx, nxb = c->geo.nxb;
  for (size_t k = 0; k < n; k++) {
    const size_t row = k / (size_t)nx;
    const int x = (int)(k - row * nx);
    out[k] = (uint8_t)((w[(size_t)(x >> 6) + (size_t)nxb * row] >> (x & 63)) & 1ull);
  }
  return FLB_OK;
}

int flb_get_populations(flb_ctx* c, double* out, size_t n) {
  if (!c || !out) return fail(FLB_EINVAL, "NULL argument");
  const long long qn = (long long)c->ncomp * c->Q * c->N;
  if (n != (size_t)qn) return fail(FLB_EINVAL, "n must be %s*nx*ny*nz = %lld", c->ncomp == 2 ? "2*Q" : "Q", qn);
  double* tmp = (double*)c->dalloc(sizeof(double) * n);
  if (!tmp) return fail(FLB_ENOMEM, "population scratch allocation failed");
  int rc = FLB_OK;
  for (int lat = 0; lat < c->ncomp && !rc; lat++)
    rc = FLB_DISPATCH(c, do_unpack, c, tmp + (size_t)lat * c->Q * c->N, lat);
  hipError_t e = hipSuccess;
  if (!rc) e = hipMemcpyAsync(out, tmp, sizeof(double) * n, hipMemcpyDeviceToHost, c->st);
  if (e == hipSuccess) e = hipStreamSynchronize(c->st);
  c->dfree(tmp);
  if (rc) return rc;
  if (e != hipSuccess) return fail(FLB_EHIP, "population query: %s", hipGetErrorString(e));
  return FLB_OK;
}

int flb_set_populations(flb_ctx* c, const double* in, size_t n) {
  if (!c || !in) return fail(FLB_EINVAL, "NULL argument");
  const long long qn = (long long)c->ncomp * c->Q * c->N;
  if (n != (size_t)qn) return fail(FLB_EINVAL, "n must be %s*nx*ny*nz = %lld", c->ncomp == 2 ? "2*Q" : "Q", qn);
  Ctl h;
  int rc = read_ctl(c, &h);
  if (rc) return rc;
  double* tmp = (double*)c->dalloc(sizeof(double) * n);
  if (!tmp) return fail(FLB_ENOMEM, "population scratch allocation failed");
  hipError_t e = hipMemcpyAsync(tmp, in, sizeof(double) * n, hipMemcpyHostToDevice, c->st);
  for (int lat = 0; lat < c->ncomp && e == hipSuccess && !rc; lat++)
    rc = FLB_DISPATCH(c, do_pack, c, tmp + (size_t)lat * c->Q * c->N, 1, (int)(h.steps & 1), lat);
  if (e == hipSuccess && !rc) rc = forget_rho(c);
  if (e == hipSuccess) e = hipStreamSynchronize(c->st);
  c->dfree(tmp);
  if (e != hipSuccess) return fail(FLB_EHIP, "population import: %s", hipGetErrorString(e));
  return rc;
}

int flb_get_stats(flb_ctx* c, flb_stats* out) {
  if (!c || !out) return fail(FLB_EINVAL, "NULL argument");
  double tot[4] = {0.0, 0.0, 0.0, 0.0};
  for (int lat = 0; lat < c->ncomp; lat++) {  // with model 1, both lattices together
    int rc = FLB_DISPATCH(c, do_moments, c, true, lat);
    if (rc) return rc;
    const int nb = 1024;
    hipLaunchKernelGGL(k_reduce_partial, dim3(nb), dim3(RED_BLOCK), 0, c->st, c->qd, 1 + c->D, c->N, c->qtot + 4);
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(64), 0, c->st, c->qtot + 4, nb, c->qtot);
    HIPCHK(hipGetLastError());
    double part[4];
    HIPCHK(hipMemcpyAsync(part, c->qtot, sizeof part, hipMemcpyDeviceToHost, c->st));
    HIPCHK(hipStreamSynchronize(c->st));
    for (int k = 0; k < 4; k++) tot[k] += part[k];
  }
  int rc;
  Ctl h;
  rc = read_ctl(c, &h);
  if (rc) return rc;
  memset(out, 0, sizeof *out);
  out->mass = tot[0];
  out->mom[0] = tot[1];
  out->mom[1] = tot[2];
  out->mom[2] = c->D == 3 ? tot[3] : 0.0;
  out->step = h.steps;
  out->n_bubbles = c->p.film_on ? h.n_bubbles : 0;
  out->n_ruptures = (int32_t)h.n_ruptures;
  out->stopped = h.stopped;
  out->events_lost = h.ev_full;
  if (h.failed || !isfinite(tot[0])) return fail(FLB_ENUMERIC, "non-finite mass");
  return FLB_OK;
}

}  // extern "C"

// ---- checkpoints ----
namespace {

struct CkptHeader {
  char magic[8];
  uint32_t version, params_size;
  flb_params p;
  Ctl ctl;
  uint64_t fbytes, N, n_events, n_flagged;
};
constexpr char kCkptMagic[8] = {'F', 'L', 'B', 'C', 'K', 'P', 'T', '1'};

int dev_to_file(FILE* fp, const void* dev, size_t bytes, hipStream_t st) {
  std::vector<char> h(bytes);
  if (bytes) {
    HIPCHK(hipMemcpyAsync(h.data(), dev, bytes, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  if (bytes && fwrite(h.data(), 1, bytes, fp) != bytes) return fail(FLB_EINVAL, "checkpoint write failed");
  return FLB_OK;
}

int file_to_dev(FILE* fp, void* dev, size_t bytes, hipStream_t st) {
  std::vector<char> h(bytes);
  if (bytes && fread(h.data(), 1, bytes, fp) != bytes) return fail(FLB_EINVAL, "checkpoint truncated");
  if (bytes) {
    HIPCHK(hipMemcpyAsync(dev, h.data(), bytes, hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  return FLB_OK;
}

// the device arrays a checkpoint carries besides the populations
struct CkptArrays {
  std::vector<std::pair<void*, size_t>> v;
  CkptArrays(flb_ctx* c, size_t n_events, size_t n_flagged) {
    if (!c->p.film_on) {
      if (c->srcw) v.push_back({c->srcw, 8 * (size_t)c->nwords});
      return;
    }
    const size_t N = (size_t)c->N;
    const size_t tsz = c->p.storage == FLB_F64 ? 8 : 4;
    v = {{c->label, 4 * N},       {c->alias, 4 * (N + 1)}, {c->own, 8 * N},
         {c->dist, N},            {c->flag, N},            {c->mask, 4 * N},
         {c->flist, 4 * n_flagged}, {c->events, 32 * n_events}, {c->rho, tsz * N}};
    if (c->srcw) v.push_back({c->srcw, 8 * (size_t)c->nwords});
  }
};

}  // namespace

extern "C" {

int flb_save(flb_ctx* c, const char* path) {
  if (!c || !path) return fail(FLB_EINVAL, "NULL argument");
  int rc = FLB_OK;
  if (c->p.film_on) rc = c->D == 2 ? complete_maps<D2Q9K>(c) : complete_maps<D3Q19K>(c);
  if (rc) return rc;
  Ctl h;
  rc = read_ctl(c, &h);
  if (rc) return rc;
  CkptHeader hd;
  memset(&hd, 0, sizeof hd);
  memcpy(hd.magic, kCkptMagic, 8);
  hd.version = 4;
  hd.params_size = sizeof(flb_params);
  hd.p = c->p;
  hd.ctl = h;
  hd.fbytes = c->fbytes;
  hd.N = (uint64_t)c->N;
  hd.n_events = c->p.film_on ? std::min<unsigned>(h.ev_count, c->ev_cap) : 0;
  hd.n_flagged = c->p.film_on ? h.n_flagged : 0;
  FILE* fp = fopen(path, "wb");
  if (!fp) return fail(FLB_EINVAL, "cannot open %s for writing", path);
  rc = fwrite(&hd, sizeof hd, 1, fp) == 1 ? FLB_OK : fail(FLB_EINVAL, "checkpoint write failed");
  if (!rc) rc = dev_to_file(fp, c->f[h.steps & 1], c->fbytes, c->st);
  CkptArrays arr(c, hd.n_events, hd.n_flagged);
  for (auto& a : arr.v)
    if (!rc) rc = dev_to_file(fp, a.first, a.second, c->st);
  if (fclose(fp) != 0 && !rc) rc = fail(FLB_EINVAL, "checkpoint close failed");
  return rc;
}

int flb_load(flb_ctx* c, const char* path) {
  if (!c || !path) return fail(FLB_EINVAL, "NULL argument");
  FILE* fp = fopen(path, "rb");
  if (!fp) return fail(FLB_EINVAL, "cannot open %s", path);
  CkptHeader hd;
  int rc = fread(&hd, sizeof hd, 1, fp) == 1 ? FLB_OK : fail(FLB_EINVAL, "not a checkpoint");
  if (!rc && (memcmp(hd.magic, kCkptMagic, 8) != 0 || hd.version != 4 || hd.params_size != sizeof(flb_params)))
    rc = fail(FLB_EINVAL, "not a checkpoint of this library version");
  if (!rc && (memcmp(&hd.p, &c->p, sizeof(flb_params)) != 0 || hd.fbytes != c->fbytes || hd.N != (uint64_t)c->N))
    rc = fail(FLB_EINVAL, "checkpoint parameters differ from the context's");
  if (!rc && (hd.n_events > c->ev_cap || hd.n_flagged > (uint64_t)c->N))
    rc = fail(FLB_EINVAL, "corrupt checkpoint");
  if (!rc) rc = file_to_dev(fp, c->f[hd.ctl.steps & 1], c->fbytes, c->st);
  CkptArrays arr(c, hd.n_events, hd.n_flagged);
  for (auto& a : arr.v)
    if (!rc) rc = file_to_dev(fp, a.first, a.second, c->st);
  fclose(fp);
  if (rc) return rc;
  hd.ctl.done = 0;  // the arrival counter of a launch; zero between steps
  HIPCHK(hipMemcpyAsync(c->ctl, &hd.ctl, sizeof(Ctl), hipMemcpyHostToDevice, c->st));
  HIPCHK(hipStreamSynchronize(c->st));
  c->launched = hd.ctl.steps;
  return FLB_OK;
}

int flb_import_maps(flb_ctx* c, const int32_t* label, const int32_t* owner, const int32_t* owner2,
                    const int32_t* dist, size_t n, const int32_t* alias_root, int32_t n_bubbles) {
  if (!c || !label || !owner || !owner2 || !dist) return fail(FLB_EINVAL, "NULL argument");
  if (!c->p.film_on) return fail(FLB_EINVAL, "film maps exist only with film_on");
  if (n != (size_t)c->N) return fail(FLB_EINVAL, "n must be nx*ny*nz = %lld", c->N);
  if (n_bubbles < 0 || (long long)n_bubbles > c->N) return fail(FLB_EINVAL, "bad n_bubbles");
  std::vector<int2> own(n);
  std::vector<uint8_t> d8(n);
  for (size_t k = 0; k < n; k++) {
    if (label[k] < 0 || label[k] > n_bubbles || owner[k] < 0 || owner[k] > n_bubbles || owner2[k] < 0 ||
        owner2[k] > n_bubbles || dist[k] < -1 || dist[k] >= c->p.zone_width || (dist[k] < 0) != (owner[k] == 0))
      return fail(FLB_EINVAL, "inconsistent maps at cell %zu", k);
    own[k] = make_int2(owner[k], owner2[k]);
    d8[k] = dist[k] < 0 ? 255 : (uint8_t)dist[k];
  }
  std::vector<int> alias(n_bubbles + 1);
  for (int b = 0; b <= n_bubbles; b++) {
    alias[b] = alias_root ? alias_root[b] : b;
    if (alias[b] < 0 || alias[b] > n_bubbles || (alias_root && alias_root[alias[b]] != alias[b]))
      return fail(FLB_EINVAL, "alias_root[%d] is not a root label", b);
  }
  Ctl h;
  int rc = read_ctl(c, &h);
  if (rc) return rc;
  if (h.stopped) return fail(FLB_EINVAL, "context is stopped");
  rc = ctx_mapsets(c);
  if (rc) return rc;
  HIPCHK(hipMemcpyAsync(c->label, label, 4 * n, hipMemcpyHostToDevice, c->st));
  HIPCHK(hipMemcpyAsync(c->own, own.data(), 8 * n, hipMemcpyHostToDevice, c->st));
  HIPCHK(hipMemcpyAsync(c->dist, d8.data(), n, hipMemcpyHostToDevice, c->st));
  HIPCHK(hipMemcpyAsync(c->alias, alias.data(), 4 * alias.size(), hipMemcpyHostToDevice, c->st));
  HIPCHK(hipMemcpyAsync(&c->ctl->n_bubbles, &n_bubbles, sizeof(int), hipMemcpyHostToDevice, c->st));
  rc = c->D == 2 ? map_masks<D2Q9K>(c->ms_import, c->st) : map_masks<D3Q19K>(c->ms_import, c->st);
  if (rc) return rc;
  // the given maps are whole: no deferred layers to run
  rc = c->D == 2 ? map_deferred<D2Q9K>(c->ms_import, c->st, false) : map_deferred<D3Q19K>(c->ms_import, c->st, false);
  if (rc) return rc;
  HIPCHK(hipStreamSynchronize(c->st));
  return FLB_OK;
}

}  // extern "C"
