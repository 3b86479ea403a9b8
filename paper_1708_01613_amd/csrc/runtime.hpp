// runtime.hpp -- internal state and helpers of the host runtime, shared by the
// translation units of the library (single-lattice API, batches, server).
#pragma once
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
#include "rupture.hpp"
#include "twopass.hpp"

using namespace flb;

namespace flb_rt {

inline thread_local std::string g_err;

inline int fail(int code, const char* fmt, ...) {
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

inline int grid_for(long long n, int block) {
  long long g = (n + block - 1) / block;
  return (int)std::min<long long>(std::max<long long>(g, 1), 65536);
}

// Device bytes a context of these parameters allocates at creation (the
// same list as flb_create, each rounded to 256 bytes), used for admission.
inline size_t ctx_footprint(const flb_params* p) {
  auto r = [](size_t n) { return (n + 255) & ~(size_t)255; };
  const int Q = p->lattice == FLB_D2Q9 ? 9 : 19;
  const size_t N = (size_t)p->nx * p->ny * p->nz;
  const int nx = p->nx, nm = p->lattice == FLB_D2Q9 ? 1 : p->ny, nz = p->lattice == FLB_D2Q9 ? p->ny : p->nz;
  const size_t nxb = (size_t)(nx + 63) / 64;
  const size_t bb = p->storage == FLB_F64 ? block_bytes<SF64>(Q) : p->storage == FLB_F32 ? block_bytes<SF32>(Q)
                                                                                           : block_bytes<SF16S>(Q);
  const size_t fbytes = nxb * nm * nz * bb;
  const size_t tsz = p->storage == FLB_F64 ? 8 : 4;
  // partials: every tile variant at one plane per segment has at most one
  // workgroup per 64-cell row segment
  const size_t max_blk = nxb * (size_t)nm * nz;
  size_t t = 2 * r(fbytes) + 2 * r(sizeof(Ctl)) + r(32 * max_blk) + 2 * r(tsz * N) + r(32 * N) + r(32 * 4096) +
             2 * r(4 * N) + r(4 * (N / 1024 + 2)) + r(4 * N) + r(8 * (N + 1));
  if (p->film_on) {
    const size_t nwords = nxb * nm * nz;
    t += 2 * r(N) + r(4 * N) + r(8 * N) + 2 * r(4 * N) + 3 * r(4 * (N + 1)) + r(32 * 65536) + r(24 * nwords);
  }
  return t;
}

}  // namespace flb_rt

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
  int* flist = nullptr;    // cells with barrier links at the last refresh
  int2* own = nullptr;
  int* label = nullptr;
  int* label_old = nullptr;
  int* alias = nullptr;
  int* alias_old = nullptr;
  int* rep = nullptr;
  int* par = nullptr;
  int* rank = nullptr;
  int* counts = nullptr;
  unsigned long long* bits = nullptr;  // BFS bitsets: 2 frontiers + visited
  long long nwords = 0;                // 64-bit words per bitset
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
  bool in_batch = false;   // owned by a batch (flb_destroy refuses it)
  std::vector<void*> allocs;

  size_t bytes = 0;  // device bytes held
  std::vector<size_t> sizes;

  void* dalloc(size_t n) {
    n = (n + 255) & ~(size_t)255;
    void* ptr = nullptr;
    if (have_al) {
      ptr = al.alloc(n, al.user);
    } else if (hipMalloc(&ptr, n) != hipSuccess) {
      ptr = nullptr;
    }
    if (ptr) {
      allocs.push_back(ptr);
      sizes.push_back(n);
      bytes += n;
    }
    return ptr;
  }
  void dfree(void* ptr) {
    if (!ptr) return;
    if (have_al) al.free(ptr, al.user);
    else (void)hipFree(ptr);
    auto it = std::find(allocs.begin(), allocs.end(), ptr);
    if (it != allocs.end()) {
      const size_t k = (size_t)(it - allocs.begin());
      bytes -= sizes[k];
      sizes.erase(sizes.begin() + (long)k);
      allocs.erase(it);
    }
  }
  void dfree_all() {
    for (void* ptr : allocs) {
      if (have_al) al.free(ptr, al.user);
      else (void)hipFree(ptr);
    }
    allocs.clear();
    sizes.clear();
    bytes = 0;
  }
  const flb_rt::TileCfg& tcfg() const { return D == 2 ? flb_rt::kTiles2[tile] : flb_rt::kTiles3[tile]; }
  bool two_pass() const { return tcfg().tx == 0; }
  int tiles_x() const { return two_pass() ? 1 : (md.nx + tcfg().tx - 1) / tcfg().tx; }
  int tiles_m() const { return two_pass() ? 1 : (md.nm + tcfg().tm - 1) / tcfg().tm; }
  int nblocks() const {
    if (two_pass()) return geo.nxb * (int)((md.nm * (long long)md.nz + TP_ROWS - 1) / TP_ROWS);
    return tiles_x() * tiles_m() * ((md.nz + lz - 1) / lz);
  }
};

namespace flb_rt {

// segment length for a z-march tile so that the launch has about `target`
// workgroups, with segments of at least 8 planes
inline int lz_for_target(const flb_ctx* c, long long target) {
  const long long cols = (long long)c->tiles_x() * c->tiles_m();
  const long long nseg = std::max<long long>(1, target / std::max<long long>(cols, 1));
  const int lz = (int)std::max<long long>(8, (c->md.nz + nseg - 1) / nseg);
  return std::min(lz, c->md.nz);
}

inline void default_tuning(flb_ctx* c) {
  // D2Q9: 64x1 tiles, ~2048 workgroups; D3Q19: 64x8 tiles, ~256 long
  // marches (one per CU), which spends the least on halo planes.
  // Workgroups are spread over the 8 XCDs.
  c->tile = c->D == 2 ? 0 : 1;
  c->lz = lz_for_target(c, c->D == 2 ? 2048 : 256);
  c->xcd = 8;
}

inline StepArgs step_args(flb_ctx* c) {
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
  a.rupture_filter = c->p.rupture_filter;
  a.flag = c->flag;
  a.mask = c->mask;
  a.flist = c->flist;
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

inline PruneArgs prune_args(flb_ctx* c) {
  PruneArgs p;
  p.ctl = c->ctl;
  p.d = c->md;
  p.own = c->own;
  p.alias = c->alias;
  p.flag = c->flag;
  p.mask = c->mask;
  p.flist = c->flist;
  return p;
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
    hipLaunchKernelGGL((k_gas_init<L, S>), dim3(map_grid(c->md)), dim3(MAP_NT), 0, c->st, c->f[0], c->f[1], gate, c->geo, c->md,
                       c->p.rho_th, c->par);
  hipLaunchKernelGGL((k_cc_local<L>), dim3(cc_tiles(c->md, CCTile<L>::TM, CCTile<L>::TZ)), dim3(CC_NT), 0, c->st,
                     gate, c->md, c->par);
  hipLaunchKernelGGL((k_cc_cross<L>), dim3(map_grid(c->md)), dim3(MAP_NT), 0, c->st, gate, c->md, c->par);
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
  unsigned long long* fr[2] = {c->bits, c->bits + c->nwords};
  unsigned long long* vis = c->bits + 2 * c->nwords;
  hipLaunchKernelGGL(k_owner_init, dim3(map_grid(c->md)), dim3(MAP_NT), 0, c->st, gate, c->md, c->label, c->own,
                     c->dist, fr[0], vis);
  for (int layer = 1; layer <= c->p.zone_width - 1; layer++)
    hipLaunchKernelGGL((k_owner_layer<L>), dim3(grid_for(c->nwords, MAP_NT)), dim3(MAP_NT), 0, c->st, gate, c->md, layer,
                       fr[(layer - 1) & 1], fr[layer & 1], vis, c->own, c->dist);
  hipLaunchKernelGGL(k_alias_reset, dim3(gl), dim3(B), 0, c->st, gate, c->alias, c->rep, (int)c->N);
  if (c->maps_seen) {
    hipLaunchKernelGGL(k_alias_carry1, dim3(g), dim3(MAP_NT), 0, c->st, gate, c->md, c->label, c->label_old,
                       c->alias_old, c->rep);
    hipLaunchKernelGGL(k_alias_carry2, dim3(g), dim3(MAP_NT), 0, c->st, gate, c->md, c->label, c->label_old,
                       c->alias_old, c->rep, c->alias);
    hipLaunchKernelGGL(k_alias_compress, dim3(gl), dim3(B), 0, c->st, gate, c->alias);
  }
  hipLaunchKernelGGL(k_flag_list_reset, dim3(1), dim3(64), 0, c->st, c->ctl);
  hipLaunchKernelGGL((k_masks<L>), dim3(map_grid(c->md)), dim3(MAP_NT), 0, c->st, c->ctl, c->md, c->p.zone_width,
                     c->own, c->dist, c->alias, c->flag, c->mask, c->flist);
  hipLaunchKernelGGL((k_rho_marks<L>), dim3(list_grid(c->N)), dim3(MAP_NT), 0, c->st, gate, c->md, c->flist,
                     c->mask);
  hipLaunchKernelGGL(k_masks_done, dim3(1), dim3(64), 0, c->st, c->ctl);
  HIPCHK(hipGetLastError());
  c->maps_seen = true;
  return FLB_OK;
}

// `ev`, if given, holds 4 events per step that bracket the step-kernel launches
template <class L, class S>
int do_steps(flb_ctx* c, int64_t nsteps, bool refresh, hipEvent_t* ev = nullptr) {
  const StepArgs a = step_args(c);
  const int nblk = c->nblocks();
  const StepFn fn = c->tcfg().fn[c->p.storage];
  const StepFn coll = c->tcfg().coll[c->p.storage];
  for (int64_t s = 0; s < nsteps; s++) {
    const bool due = refresh && c->p.film_on && c->launched % c->p.k_own == 0;
    if (coll) {
      if (ev) HIPCHK(hipEventRecord(ev[4 * s], c->st));
      fn(a, nblk, c->st);  // rho / psi of the current state
      if (ev) HIPCHK(hipEventRecord(ev[4 * s + 1], c->st));
      if (due) {
        int rc = refresh_maps<L, S>(c, true);
        if (rc) return rc;
      }
      if (ev) HIPCHK(hipEventRecord(ev[4 * s + 2], c->st));
      coll(a, nblk, c->st);
      if (ev) HIPCHK(hipEventRecord(ev[4 * s + 3], c->st));
    } else {
      if (due) {
        int rc = refresh_maps<L, S>(c, false);
        if (rc) return rc;
      }
      if (ev) HIPCHK(hipEventRecord(ev[4 * s], c->st));
      fn(a, nblk, c->st);
      if (ev) HIPCHK(hipEventRecord(ev[4 * s + 1], c->st));
    }
    // rupture test (applies its unions), pruning of united pairs' links,
    // then the finisher, which closes the step
    if (c->p.film_on && c->launched >= c->p.rupture_warmup) {
      hipLaunchKernelGGL((k_rupture<L, typename S::ct>), dim3(list_grid(c->N)), dim3(MAP_NT), 0, c->st, a);
      hipLaunchKernelGGL((k_mask_prune<L>), dim3(list_grid(c->N)), dim3(MAP_NT), 0, c->st, prune_args(c));
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

inline int validate(const flb_params* p) {
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
  if (p->rupture_filter != 0 && p->rupture_filter != 1) return fail(FLB_EINVAL, "rupture_filter must be 0 or 1");
  return FLB_OK;
}

inline int read_ctl(flb_ctx* c, Ctl* out) {
  HIPCHK(hipMemcpyAsync(out, c->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipStreamSynchronize(c->st));
  return FLB_OK;
}

}  // namespace flb_rt
