// foamlbm.hip -- host runtime and C ABI (include/foamlbm.h) of the gfx950 path.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "../../include/foamlbm.h"
#include "ops.hpp"
#include "twopass.hpp"

using namespace flb;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIPCHK(expr)                                                                  \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess) return fail(FLB_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// ---------------------------------------------------------------------------
// step-kernel variants: tile shapes per lattice
// ---------------------------------------------------------------------------
using StepFn = void (*)(const StepArgs&, int, hipStream_t);

// buffers below 2 GiB use buffer-resource loads with 32-bit offsets
template <class L, class S, int TX, int TM>
void launch_step(const StepArgs& a, int nblk, hipStream_t s) {
  if (a.buf_bytes < kBufPathLimit)
    hipLaunchKernelGGL((k_step<L, S, TX, TM, true>), dim3(nblk), dim3(StepBlock<L, S, TX, TM, true>::NT), 0, s, a);
  else
    hipLaunchKernelGGL((k_step<L, S, TX, TM, false>), dim3(nblk), dim3(StepBlock<L, S, TX, TM, false>::NT), 0, s,
                       a);
}

// two-pass path: k_psi then k_collide
template <class L, class S>
void launch_psi(const StepArgs& a, int nblk, hipStream_t s) {
  if (a.buf_bytes < kBufPathLimit)
    hipLaunchKernelGGL((k_psi<L, S, true>), dim3(nblk), dim3(TP_NT), 0, s, a);
  else
    hipLaunchKernelGGL((k_psi<L, S, false>), dim3(nblk), dim3(TP_NT), 0, s, a);
}
template <class L, class S>
void launch_collide(const StepArgs& a, int nblk, hipStream_t s) {
  if (a.buf_bytes < kBufPathLimit)
    hipLaunchKernelGGL((k_collide<L, S, true>), dim3(nblk), dim3(TP_NT), 0, s, a);
  else
    hipLaunchKernelGGL((k_collide<L, S, false>), dim3(nblk), dim3(TP_NT), 0, s, a);
}

// step variants: z-march tiles (tx, tm) or the two-pass path (tx = tm = 0)
struct TileCfg {
  int tx, tm;
  StepFn fn[3];    // z-march kernel, or k_psi, per storage F64, F32, F16S
  StepFn coll[3];  // k_collide of the two-pass path
};

template <class L, int TX, int TM>
constexpr TileCfg make_tile() {
  return TileCfg{TX, TM,
                 {&launch_step<L, SF64, TX, TM>, &launch_step<L, SF32, TX, TM>, &launch_step<L, SF16S, TX, TM>},
                 {nullptr, nullptr, nullptr}};
}
template <class L>
constexpr TileCfg make_two_pass() {
  return TileCfg{0, 0, {&launch_psi<L, SF64>, &launch_psi<L, SF32>, &launch_psi<L, SF16S>},
                 {&launch_collide<L, SF64>, &launch_collide<L, SF32>, &launch_collide<L, SF16S>}};
}

const TileCfg kTiles2[] = {make_tile<D2Q9K, 64, 1>(), make_tile<D2Q9K, 128, 1>(), make_tile<D2Q9K, 256, 1>(),
                           make_two_pass<D2Q9K>()};
const TileCfg kTiles3[] = {make_tile<D3Q19K, 64, 4>(), make_tile<D3Q19K, 64, 8>(), make_tile<D3Q19K, 32, 8>(),
                           make_tile<D3Q19K, 128, 4>(), make_two_pass<D3Q19K>()};
constexpr int kNTiles2 = sizeof(kTiles2) / sizeof(kTiles2[0]);
constexpr int kNTiles3 = sizeof(kTiles3) / sizeof(kTiles3[0]);

int grid_for(long long n, int block) {
  long long g = (n + block - 1) / block;
  return (int)std::min<long long>(std::max<long long>(g, 1), 65536);
}

}  // namespace

struct flb_ctx {
  flb_params p;
  flb_allocator al;
  bool have_al = false;
  hipStream_t st = nullptr;
  int Q = 0, D = 0;
  MapDims md;              // kernel-coordinate extents
  long long N = 0;         // cells
  Geo geo;                 // population block layout
  size_t fbytes = 0;       // bytes of one population buffer
  void* f[2] = {nullptr, nullptr};
  Ctl* ctl = nullptr;      // run control of the step kernel
  Ctl* qctl = nullptr;     // always-zero control for query pipelines
  double* partials = nullptr;
  int max_blk = 0;
  void* psi = nullptr;     // two-pass path: psi and rho arrays (compute type)
  void* rho = nullptr;
  // tuning
  int tile = -1, lz = 0, xcd = 0;
  // film maps
  uint8_t* flag = nullptr;
  uint8_t* dist = nullptr;
  uint32_t* mask = nullptr;
  int2* own = nullptr;
  int* label = nullptr;
  int* label_old = nullptr;
  int* alias = nullptr;
  int* alias_old = nullptr;
  int* rep = nullptr;
  int* par = nullptr;
  int* rank = nullptr;
  int* counts = nullptr;
  long long* events = nullptr;
  unsigned ev_cap = 1u << 16;
  bool maps_seen = false;  // a refresh has run since the last set_nuclei
  // query scratch
  double* qd = nullptr;    // (1 + 3) * N doubles
  int* qlabel = nullptr;
  unsigned long long* qsizes = nullptr;
  unsigned long long* qhist = nullptr;
  int qhist_cap = 0;
  double* qtot = nullptr;  // 4 doubles
  long long launched = 0;
  std::vector<void*> allocs;

  void* dalloc(size_t bytes) {
    bytes = (bytes + 255) & ~(size_t)255;
    void* ptr = nullptr;
    if (have_al) {
      ptr = al.alloc(bytes, al.user);
    } else if (hipMalloc(&ptr, bytes) != hipSuccess) {
      ptr = nullptr;
    }
    if (ptr) allocs.push_back(ptr);
    return ptr;
  }
  void dfree_all() {
    for (void* ptr : allocs) {
      if (have_al) al.free(ptr, al.user);
      else (void)hipFree(ptr);
    }
    allocs.clear();
  }
  const TileCfg& tcfg() const { return D == 2 ? kTiles2[tile] : kTiles3[tile]; }
  bool two_pass() const { return tcfg().tx == 0; }
  int tiles_x() const { return two_pass() ? 1 : (md.nx + tcfg().tx - 1) / tcfg().tx; }
  int tiles_m() const { return two_pass() ? 1 : (md.nm + tcfg().tm - 1) / tcfg().tm; }
  int nblocks() const {
    if (two_pass()) return geo.nxb * (int)((md.nm * (long long)md.nz + TP_ROWS - 1) / TP_ROWS);
    return tiles_x() * tiles_m() * ((md.nz + lz - 1) / lz);
  }
};

namespace {

void default_tuning(flb_ctx* c) {
  c->tile = c->D == 2 ? 1 : 1;  // D2Q9 128x1, D3Q19 64x8
  const long long cols = (long long)c->tiles_x() * c->tiles_m();
  // aim at ~2048 workgroups (8 per CU) without segments shorter than 8 planes
  long long nseg = std::max<long long>(1, 2048 / std::max<long long>(cols, 1));
  int lz = (int)std::max<long long>(8, (c->md.nz + nseg - 1) / nseg);
  c->lz = std::min(lz, c->md.nz);
  c->xcd = 0;
}

StepArgs step_args(flb_ctx* c) {
  StepArgs a;
  memset(&a, 0, sizeof a);
  a.buf[0] = c->f[0];
  a.buf[1] = c->f[1];
  a.geo = c->geo;
  a.nx = c->md.nx;
  a.nm = c->md.nm;
  a.nz = c->md.nz;
  a.tiles_x = c->tiles_x();
  a.tiles_m = c->tiles_m();
  a.lz = c->lz;
  const int nblk = c->nblocks();
  a.xcd_chunks = (c->xcd > 1 && nblk % c->xcd == 0) ? c->xcd : 1;
  a.tau = c->p.tau;
  a.G = c->p.G;
  a.rho0 = c->p.rho0;
  a.psi_bar = c->p.rho0 * (1.0 - exp(-c->p.rho_liquid / c->p.rho0));
  a.psi_bar_mode = c->p.psi_bar_mode;
  a.film_on = c->p.film_on;
  a.rupture_warmup = c->p.rupture_warmup;
  a.on_rupture = c->p.on_rupture;
  a.flag = c->flag;
  a.mask = c->mask;
  a.own = c->own;
  a.alias = c->alias;
  a.events = c->events;
  a.ev_cap = c->ev_cap;
  a.ctl = c->ctl;
  a.partials = c->partials;
  a.buf_bytes = c->fbytes;
  a.psi = c->psi;
  a.rho = c->rho;
  return a;
}

// ---- labels of the current state (or of a density field) into `label` ----
template <class L, class S>
int label_pipeline(flb_ctx* c, const Ctl* gate, int* total, int* label, const double* field,
                   bool from_rho = false) {
  const int B = 256, g = grid_for(c->N, B);
  if (field)
    hipLaunchKernelGGL(k_gas_from_field, dim3(g), dim3(B), 0, c->st, field, c->md, c->p.rho_th, c->par);
  else if (from_rho)
    hipLaunchKernelGGL((k_gas_from_rho<typename S::ct>), dim3(g), dim3(B), 0, c->st, gate,
                       (const typename S::ct*)c->rho, c->md, c->p.rho_th, c->par);
  else
    hipLaunchKernelGGL((k_gas_init<L, S>), dim3(g), dim3(B), 0, c->st, c->f[0], c->f[1], gate, c->geo, c->md,
                       c->p.rho_th, c->par);
  hipLaunchKernelGGL((k_cc_hook<L>), dim3(g), dim3(B), 0, c->st, gate, c->md, c->par);
  hipLaunchKernelGGL(k_cc_compress, dim3(g), dim3(B), 0, c->st, gate, c->md, c->par);
  const int nrb = (int)((c->N + RANK_BLOCK - 1) / RANK_BLOCK);
  hipLaunchKernelGGL(k_count_roots, dim3(nrb), dim3(RANK_BLOCK), 0, c->st, gate, c->md, c->par, c->counts);
  hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(1024), 0, c->st, gate, c->counts, nrb, total);
  hipLaunchKernelGGL(k_write_rank, dim3(nrb), dim3(RANK_BLOCK), 0, c->st, gate, c->md, c->par, c->counts,
                     c->rank);
  hipLaunchKernelGGL(k_write_labels, dim3(g), dim3(B), 0, c->st, gate, c->md, c->par, c->rank, label);
  HIPCHK(hipGetLastError());
  return FLB_OK;
}

// ---- film-map refresh before a step ----
template <class L, class S>
int refresh_maps(flb_ctx* c, bool from_rho) {
  const int B = 256, g = grid_for(c->N, B);
  const int gl = grid_for(c->N + 1, B);
  const Ctl* gate = c->ctl;
  if (c->maps_seen) {
    hipLaunchKernelGGL(k_copy_int, dim3(g), dim3(B), 0, c->st, gate, c->label, c->label_old, c->N);
    hipLaunchKernelGGL(k_copy_int, dim3(gl), dim3(B), 0, c->st, gate, c->alias, c->alias_old, c->N + 1);
  }
  int rc = label_pipeline<L, S>(c, gate, &c->ctl->n_bubbles, c->label, nullptr, from_rho);
  if (rc) return rc;
  hipLaunchKernelGGL(k_owner_init, dim3(g), dim3(B), 0, c->st, gate, c->md, c->label, c->own, c->dist);
  for (int layer = 1; layer <= c->p.zone_width - 1; layer++)
    hipLaunchKernelGGL((k_owner_layer<L>), dim3(g), dim3(B), 0, c->st, gate, c->md, layer, c->own, c->dist);
  hipLaunchKernelGGL(k_alias_reset, dim3(gl), dim3(B), 0, c->st, gate, c->alias, c->rep, (int)c->N);
  if (c->maps_seen) {
    hipLaunchKernelGGL(k_alias_carry1, dim3(g), dim3(B), 0, c->st, gate, c->md, c->label, c->label_old,
                       c->alias_old, c->rep);
    hipLaunchKernelGGL(k_alias_carry2, dim3(g), dim3(B), 0, c->st, gate, c->md, c->label, c->label_old,
                       c->alias_old, c->rep, c->alias);
    hipLaunchKernelGGL(k_alias_compress, dim3(gl), dim3(B), 0, c->st, gate, c->alias);
  }
  hipLaunchKernelGGL((k_masks<L>), dim3(g), dim3(B), 0, c->st, gate, c->md, c->p.zone_width, c->own, c->dist,
                     c->alias, c->flag, c->mask);
  hipLaunchKernelGGL(k_masks_done, dim3(1), dim3(64), 0, c->st, c->ctl);
  HIPCHK(hipGetLastError());
  c->maps_seen = true;
  return FLB_OK;
}

template <class L, class S>
int do_steps(flb_ctx* c, int64_t nsteps, bool refresh) {
  const StepArgs a = step_args(c);
  const int nblk = c->nblocks();
  const StepFn fn = c->tcfg().fn[c->p.storage];
  const StepFn coll = c->tcfg().coll[c->p.storage];
  for (int64_t s = 0; s < nsteps; s++) {
    const bool due = refresh && c->p.film_on && c->launched % c->p.k_own == 0;
    if (coll) {
      fn(a, nblk, c->st);  // rho / psi of the current state
      if (due) {
        int rc = refresh_maps<L, S>(c, true);
        if (rc) return rc;
      }
      coll(a, nblk, c->st);
    } else {
      if (due) {
        int rc = refresh_maps<L, S>(c, false);
        if (rc) return rc;
      }
      fn(a, nblk, c->st);
    }
    hipLaunchKernelGGL(k_step_finish, dim3(1), dim3(FIN_NT), 0, c->st, a, nblk);
    c->launched++;
  }
  HIPCHK(hipGetLastError());
  return FLB_OK;
}

template <class L, class S>
int do_pack(flb_ctx* c, const double* field_dev, int mode, int which) {
  const int B = 256, g = grid_for(c->N, B);
  hipLaunchKernelGGL((k_pack<L, S>), dim3(g), dim3(B), 0, c->st, c->f[which], c->geo, c->md, field_dev, mode);
  HIPCHK(hipGetLastError());
  return FLB_OK;
}

template <class L, class S>
int do_moments(flb_ctx* c, bool with_j) {
  const int B = 256, g = grid_for(c->N, B);
  hipLaunchKernelGGL((k_moments<L, S>), dim3(g), dim3(B), 0, c->st, c->f[0], c->f[1], c->ctl, c->geo, c->md, c->qd,
                     with_j ? c->qd + c->N : nullptr);
  HIPCHK(hipGetLastError());
  return FLB_OK;
}

template <class L, class S>
int do_unpack(flb_ctx* c, double* out_dev) {
  const int B = 256, g = grid_for(c->N, B);
  hipLaunchKernelGGL((k_unpack<L, S>), dim3(g), dim3(B), 0, c->st, c->f[0], c->f[1], c->ctl, c->geo, c->md,
                     out_dev);
  HIPCHK(hipGetLastError());
  return FLB_OK;
}

// dispatch a templated operation on (lattice, storage)
#define FLB_DISPATCH(c, FN, ...)                                                           \
  ((c)->D == 2 ? ((c)->p.storage == FLB_F64   ? FN<D2Q9K, SF64>(__VA_ARGS__)              \
                  : (c)->p.storage == FLB_F32 ? FN<D2Q9K, SF32>(__VA_ARGS__)              \
                                              : FN<D2Q9K, SF16S>(__VA_ARGS__))            \
               : ((c)->p.storage == FLB_F64   ? FN<D3Q19K, SF64>(__VA_ARGS__)             \
                  : (c)->p.storage == FLB_F32 ? FN<D3Q19K, SF32>(__VA_ARGS__)             \
                                              : FN<D3Q19K, SF16S>(__VA_ARGS__)))

int validate(const flb_params* p) {
  if (!p) return fail(FLB_EINVAL, "params is NULL");
  if (p->lattice != FLB_D2Q9 && p->lattice != FLB_D3Q19) return fail(FLB_EINVAL, "lattice must be 0 or 1");
  if (p->storage < FLB_F64 || p->storage > FLB_F16S) return fail(FLB_EINVAL, "storage must be 0, 1 or 2");
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) return fail(FLB_EINVAL, "extents must be >= 1");
  if (p->lattice == FLB_D2Q9 && p->nz != 1) return fail(FLB_EINVAL, "D2Q9 requires nz == 1");
  const long long N = (long long)p->nx * p->ny * p->nz;
  if (N > (1ll << 28)) return fail(FLB_EINVAL, "lattice too large (%lld cells > 2^28)", N);
  if (!(p->tau > 0.5) || !isfinite(p->tau)) return fail(FLB_EINVAL, "tau must be > 0.5");
  if (!(p->rho0 > 0) || !isfinite(p->rho0)) return fail(FLB_EINVAL, "rho0 must be > 0");
  if (!isfinite(p->G) || !isfinite(p->rho_liquid) || !isfinite(p->rho_gas) || !isfinite(p->noise_amp) ||
      !isfinite(p->rho_th))
    return fail(FLB_EINVAL, "non-finite parameter");
  if (p->film_on != 0 && p->film_on != 1) return fail(FLB_EINVAL, "film_on must be 0 or 1");
  if (p->k_own < 1) return fail(FLB_EINVAL, "k_own must be >= 1");
  if (p->zone_width < 1 || p->zone_width > 15) return fail(FLB_EINVAL, "zone_width must be in 1..15");
  if (p->psi_bar_mode != 0 && p->psi_bar_mode != 1) return fail(FLB_EINVAL, "psi_bar_mode must be 0 or 1");
  if (p->on_rupture != 0 && p->on_rupture != 1) return fail(FLB_EINVAL, "on_rupture must be 0 or 1");
  if (p->velocity_mode != 0 && p->velocity_mode != 1) return fail(FLB_EINVAL, "velocity_mode must be 0 or 1");
  return FLB_OK;
}

int read_ctl(flb_ctx* c, Ctl* out) {
  HIPCHK(hipMemcpyAsync(out, c->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipStreamSynchronize(c->st));
  return FLB_OK;
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
  c->fbytes = (size_t)c->geo.nxb * c->md.nm * c->md.nz * c->geo.block_bytes;
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
  bool ok = true;
  for (int b = 0; b < 2; b++) ok = ok && (c->f[b] = c->dalloc(c->fbytes));
  ok = ok && (c->ctl = (Ctl*)c->dalloc(sizeof(Ctl)));
  ok = ok && (c->qctl = (Ctl*)c->dalloc(sizeof(Ctl)));
  ok = ok && (c->partials = (double*)c->dalloc(sizeof(double) * 4 * (size_t)c->max_blk));
  {
    const size_t tsz = p->storage == FLB_F64 ? 8 : 4;
    ok = ok && (c->psi = c->dalloc(tsz * (size_t)c->N));
    ok = ok && (c->rho = c->dalloc(tsz * (size_t)c->N));
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
    ok = ok && (c->own = (int2*)c->dalloc(sizeof(int2) * (size_t)c->N));
    ok = ok && (c->label = (int*)c->dalloc(sizeof(int) * (size_t)c->N));
    ok = ok && (c->label_old = (int*)c->dalloc(sizeof(int) * (size_t)c->N));
    ok = ok && (c->alias = (int*)c->dalloc(sizeof(int) * (size_t)(c->N + 1)));
    ok = ok && (c->alias_old = (int*)c->dalloc(sizeof(int) * (size_t)(c->N + 1)));
    ok = ok && (c->rep = (int*)c->dalloc(sizeof(int) * (size_t)(c->N + 1)));
    ok = ok && (c->events = (long long*)c->dalloc(sizeof(long long) * 4 * (size_t)c->ev_cap));
  }
  if (!ok) {
    c->dfree_all();
    delete c;
    return fail(FLB_ENOMEM, "device allocation failed");
  }
  if (hipMemsetAsync(c->ctl, 0, sizeof(Ctl), c->st) != hipSuccess ||
      hipMemsetAsync(c->qctl, 0, sizeof(Ctl), c->st) != hipSuccess ||
      (p->film_on && hipMemsetAsync(c->flag, 0, (size_t)c->N, c->st) != hipSuccess) ||
      (p->film_on && hipMemsetAsync(c->mask, 0, sizeof(uint32_t) * (size_t)c->N, c->st) != hipSuccess) ||
      hipStreamSynchronize(c->st) != hipSuccess) {
    c->dfree_all();
    delete c;
    return fail(FLB_EHIP, "initialising device state failed");
  }
  *out = c;
  return FLB_OK;
}

void flb_destroy(flb_ctx* c) {
  if (!c) return;
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
  const int B = 256, g = grid_for(c->N, B);
  hipLaunchKernelGGL(k_init_density, dim3(g), dim3(B), 0, c->st, c->qd, c->p.nx, c->p.ny, c->p.nz, c->N, dn, n,
                     c->p.rho_liquid, c->p.rho_gas, c->p.noise_amp, (unsigned long long)c->p.seed);
  HIPCHK(hipGetLastError());
  int rc = FLB_DISPATCH(c, do_pack, c, c->qd, 0, 0);
  if (rc) return rc;
  HIPCHK(hipStreamSynchronize(c->st));
  if (dn) {
    if (c->have_al) c->al.free(dn, c->al.user);
    else (void)hipFree(dn);
    c->allocs.erase(std::find(c->allocs.begin(), c->allocs.end(), (void*)dn));
  }
  c->launched = 0;
  c->maps_seen = false;
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

int flb_time_steps(flb_ctx* c, int64_t nsteps, int32_t refresh, double* ms) {
  if (!c || !ms) return fail(FLB_EINVAL, "NULL argument");
  if (nsteps < 0) return fail(FLB_EINVAL, "nsteps must be >= 0");
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  hipError_t e = hipEventRecord(e0, c->st);
  int rc = FLB_OK;
  if (e == hipSuccess) rc = FLB_DISPATCH(c, do_steps, c, nsteps, refresh != 0);
  if (e == hipSuccess && !rc) e = hipEventRecord(e1, c->st);
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

int flb_set_tuning(flb_ctx* c, int32_t tile, int32_t lz, int32_t xcd) {
  if (!c) return fail(FLB_EINVAL, "ctx is NULL");
  const int nt = c->D == 2 ? kNTiles2 : kNTiles3;
  if (tile < -1 || tile >= nt) return fail(FLB_EINVAL, "tile must be in -1..%d", nt - 1);
  if (lz < 0) return fail(FLB_EINVAL, "lz must be >= 0");
  if (xcd < -1 || xcd > 64) return fail(FLB_EINVAL, "xcd must be in -1..64");
  HIPCHK(hipStreamSynchronize(c->st));
  if (tile >= 0) c->tile = tile;
  if (lz > 0) c->lz = std::min(lz, c->md.nz);
  if (xcd >= 0) c->xcd = xcd;
  if (c->nblocks() > c->max_blk) return fail(FLB_EINVAL, "tuning exceeds the partials capacity");
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
  HIPCHK(hipMemsetAsync(c->qctl, 0, sizeof(Ctl), c->st));
  int rc = FLB_DISPATCH(c, label_pipeline, c, c->qctl, &c->qctl->n_bubbles, c->qlabel, (const double*)nullptr);
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
  HIPCHK(hipMemsetAsync(c->qctl, 0, sizeof(Ctl), c->st));
  int rc = FLB_DISPATCH(c, label_pipeline, c, c->qctl, &c->qctl->n_bubbles, c->qlabel, (const double*)c->qd);
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
  if (label) HIPCHK(hipMemcpyAsync(label, c->label, sizeof(int) * n, hipMemcpyDeviceToHost, c->st));
  if (mask) HIPCHK(hipMemcpyAsync(mask, c->mask, sizeof(uint32_t) * n, hipMemcpyDeviceToHost, c->st));
  std::vector<int2> own;
  std::vector<uint8_t> d8;
  if (owner || owner2) {
    own.resize(n);
    HIPCHK(hipMemcpyAsync(own.data(), c->own, sizeof(int2) * n, hipMemcpyDeviceToHost, c->st));
  }
  if (dist) {
    d8.resize(n);
    HIPCHK(hipMemcpyAsync(d8.data(), c->dist, n, hipMemcpyDeviceToHost, c->st));
  }
  HIPCHK(hipStreamSynchronize(c->st));
  for (size_t k = 0; k < n; k++) {
    if (owner) owner[k] = own[k].x;
    if (owner2) owner2[k] = own[k].y;
    if (dist) dist[k] = d8[k] == 255 ? -1 : d8[k];
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
  HIPCHK(hipMemsetAsync(c->qctl, 0, sizeof(Ctl), c->st));
  int rc = FLB_DISPATCH(c, label_pipeline, c, c->qctl, &c->qctl->n_bubbles, c->qlabel, (const double*)nullptr);
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

int flb_get_rupture_events(flb_ctx* c, int64_t* out, int64_t cap, int64_t* n) {
  if (!c || !n || (cap > 0 && !out)) return fail(FLB_EINVAL, "NULL argument");
  if (cap < 0) return fail(FLB_EINVAL, "cap must be >= 0");
  Ctl h;
  int rc = read_ctl(c, &h);
  if (rc) return rc;
  *n = c->p.film_on ? (int64_t)h.ev_count : 0;
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

int flb_get_velocity(flb_ctx* c, double* out, size_t n) {
  if (!c || !out) return fail(FLB_EINVAL, "NULL argument");
  if (n != (size_t)c->D * c->N) return fail(FLB_EINVAL, "n must be D*nx*ny*nz = %lld", c->D * c->N);
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
  if (c->have_al) c->al.free(vel, c->al.user);
  else (void)hipFree(vel);
  c->allocs.erase(std::find(c->allocs.begin(), c->allocs.end(), (void*)vel));
  if (e != hipSuccess) return fail(FLB_EHIP, "velocity query: %s", hipGetErrorString(e));
  return FLB_OK;
}

int flb_get_populations(flb_ctx* c, double* out, size_t n) {
  if (!c || !out) return fail(FLB_EINVAL, "NULL argument");
  if (n != (size_t)c->Q * c->N) return fail(FLB_EINVAL, "n must be Q*nx*ny*nz = %lld", c->Q * c->N);
  double* tmp = (double*)c->dalloc(sizeof(double) * n);
  if (!tmp) return fail(FLB_ENOMEM, "population scratch allocation failed");
  int rc = FLB_DISPATCH(c, do_unpack, c, tmp);
  hipError_t e = hipSuccess;
  if (!rc) e = hipMemcpyAsync(out, tmp, sizeof(double) * n, hipMemcpyDeviceToHost, c->st);
  if (e == hipSuccess) e = hipStreamSynchronize(c->st);
  if (c->have_al) c->al.free(tmp, c->al.user);
  else (void)hipFree(tmp);
  c->allocs.erase(std::find(c->allocs.begin(), c->allocs.end(), (void*)tmp));
  if (rc) return rc;
  if (e != hipSuccess) return fail(FLB_EHIP, "population query: %s", hipGetErrorString(e));
  return FLB_OK;
}

int flb_set_populations(flb_ctx* c, const double* in, size_t n) {
  if (!c || !in) return fail(FLB_EINVAL, "NULL argument");
  if (n != (size_t)c->Q * c->N) return fail(FLB_EINVAL, "n must be Q*nx*ny*nz = %lld", c->Q * c->N);
  Ctl h;
  int rc = read_ctl(c, &h);
  if (rc) return rc;
  double* tmp = (double*)c->dalloc(sizeof(double) * n);
  if (!tmp) return fail(FLB_ENOMEM, "population scratch allocation failed");
  hipError_t e = hipMemcpyAsync(tmp, in, sizeof(double) * n, hipMemcpyHostToDevice, c->st);
  if (e == hipSuccess) rc = FLB_DISPATCH(c, do_pack, c, tmp, 1, (int)(h.steps & 1));
  if (e == hipSuccess) e = hipStreamSynchronize(c->st);
  if (c->have_al) c->al.free(tmp, c->al.user);
  else (void)hipFree(tmp);
  c->allocs.erase(std::find(c->allocs.begin(), c->allocs.end(), (void*)tmp));
  if (e != hipSuccess) return fail(FLB_EHIP, "population import: %s", hipGetErrorString(e));
  return rc;
}

int flb_get_stats(flb_ctx* c, flb_stats* out) {
  if (!c || !out) return fail(FLB_EINVAL, "NULL argument");
  int rc = FLB_DISPATCH(c, do_moments, c, true);
  if (rc) return rc;
  const int nb = 1024;
  hipLaunchKernelGGL(k_reduce_partial, dim3(nb), dim3(RED_BLOCK), 0, c->st, c->qd, 1 + c->D, c->N, c->qtot + 4);
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(64), 0, c->st, c->qtot + 4, nb, c->qtot);
  HIPCHK(hipGetLastError());
  double tot[4];
  HIPCHK(hipMemcpyAsync(tot, c->qtot, sizeof tot, hipMemcpyDeviceToHost, c->st));
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
  out->events_lost = h.ev_count > c->ev_cap ? (int32_t)(h.ev_count - c->ev_cap) : 0;
  if (h.failed || !isfinite(tot[0])) return fail(FLB_ENUMERIC, "non-finite mass");
  return FLB_OK;
}

}  // extern "C"
