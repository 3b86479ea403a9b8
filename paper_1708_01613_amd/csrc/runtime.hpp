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
#include "twolattice.hpp"
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

// buffers below 2 GiB use buffer-resource loads with 32-bit offsets; the
// source terms (gas release, body force) have a variant of their own
template <class L, class S, int TX, int TM, bool EXT, int FR>
void launch_step_g(const StepArgs& a, int nblk, hipStream_t s) {
  if (a.buf_bytes < kBufPathLimit)
    hipLaunchKernelGGL((k_step<L, S, TX, TM, true, EXT, FR>), dim3(nblk),
                       dim3(StepBlock<L, S, TX, TM, true, EXT, FR>::NT), 0, s, a);
  else
    hipLaunchKernelGGL((k_step<L, S, TX, TM, false, EXT, FR>), dim3(nblk),
                       dim3(StepBlock<L, S, TX, TM, false, EXT, FR>::NT), 0, s, a);
}
template <class L, class S, int TX, int TM, int FR>
void launch_step(const StepArgs& a, int nblk, hipStream_t s) {
  if (a.srcw || a.force_on) launch_step_g<L, S, TX, TM, true, FR>(a, nblk, s);
  else launch_step_g<L, S, TX, TM, false, FR>(a, nblk, s);
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

// step variants: z-march tiles (tx, tm), flat 2-D tiles (tx = 64, tm = 1,
// fh rows: the segment length is fixed) or the two-pass path (tx = tm = 0)
struct TileCfg {
  int tx, tm;
  StepFn fn[3];    // z-march or flat kernel, or k_psi, per storage F64, F32, F16S
  StepFn coll[3];  // k_collide of the two-pass path
  int fh;          // rows of a flat tile (0: march or two-pass)
};

template <class L, int TX, int TM, int FR = 0>
constexpr TileCfg make_tile() {
  return TileCfg{TX, TM,
                 {&launch_step<L, SF64, TX, TM, FR>, &launch_step<L, SF32, TX, TM, FR>,
                  &launch_step<L, SF16S, TX, TM, FR>},
                 {nullptr, nullptr, nullptr},
                 StepBlock<L, SF32, TX, TM, true, false, FR>::FH * (FR > 0)};
}
template <class L>
constexpr TileCfg make_two_pass() {
  return TileCfg{0, 0, {&launch_psi<L, SF64>, &launch_psi<L, SF32>, &launch_psi<L, SF16S>},
                 {&launch_collide<L, SF64>, &launch_collide<L, SF32>, &launch_collide<L, SF16S>}, 0};
}

// the two-lattice step: k_psi_tl then k_collide_tl, on the two-pass decomposition
template <class L, class S>
void launch_tl(const StepArgs& a, const TLArgs& t, int nblk, hipStream_t s) {
  if (a.buf_bytes < kBufPathLimit) {
    hipLaunchKernelGGL((k_psi_tl<L, S, true>), dim3(nblk), dim3(TP_NT), 0, s, a, t);
    hipLaunchKernelGGL((k_collide_tl<L, S, true>), dim3(nblk), dim3(TP_NT), 0, s, a, t);
  } else {
    hipLaunchKernelGGL((k_psi_tl<L, S, false>), dim3(nblk), dim3(TP_NT), 0, s, a, t);
    hipLaunchKernelGGL((k_collide_tl<L, S, false>), dim3(nblk), dim3(TP_NT), 0, s, a, t);
  }
}

const TileCfg kTiles2[] = {make_tile<D2Q9K, 64, 1>(),    make_tile<D2Q9K, 128, 1>(),
                           make_tile<D2Q9K, 256, 1>(),   make_tile<D2Q9K, 64, 1, 2>(),
                           make_tile<D2Q9K, 64, 1, 4>(), make_two_pass<D2Q9K>()};
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
  size_t t = 2 * r(fbytes) + 2 * r(sizeof(Ctl)) + r(32 * (max_blk + max_blk / FOLD + 1)) + 2 * r(tsz * N) + r(32 * N) + r(32 * 4096) +
             2 * r(4 * N) + r(4 * (N / 1024 + 2)) + r(4 * N) + r(8 * (N + 1));
  const size_t nwords = nxb * nm * nz;
  if (p->film_on)
    t += 2 * r(N) + r(4 * N) + r(8 * N) + 2 * r(4 * N) + 3 * r(4 * (N + 1)) + r(32 * 65536) +
         r(4 * N) + r(8 * nwords) + r(3 * 8 * nwords);
  if (p->growth_on) t += r(8 * nwords);
  if (p->model == 1) t += 2 * r(fbytes) + 2 * r(tsz * N);  // the gas lattice's populations and arrays
  return t;
}

// A second stream for work of a refresh that does not depend on the work
// before it in the main stream: the alias carry runs beside the BFS layers
// (both only read the new labels).  Joined with events, so it also works
// inside a captured graph.  Default priority, like every stream here.
struct Fork {
  hipStream_t side = nullptr;
  hipEvent_t a = nullptr, b = nullptr;
  int init() {
    if (side) return FLB_OK;
    if (hipStreamCreateWithFlags(&side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&a, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b, hipEventDisableTiming) != hipSuccess) {
      release();
      return fail(FLB_EHIP, "creating the refresh side stream failed");
    }
    return FLB_OK;
  }
  void release() {
    if (side) (void)hipStreamSynchronize(side);
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (side) (void)hipStreamDestroy(side);
    side = nullptr;
    a = b = nullptr;
  }
  Fork() = default;
  Fork(const Fork&) = delete;
  Fork& operator=(const Fork&) = delete;
  ~Fork() { release(); }
};

// A MapSet is a device table of MapArgs plus, per decomposition, the
// workgroup ranges of its lattices.  Tables of one lattice serve a context;
// a batch builds one over its film members.
struct MapSet {
  MapArgs* tab = nullptr;  // device, n entries
  int* first = nullptr;    // device, SH_COUNT arrays of n + 1 offsets
  int n = 0;
  int total[SH_COUNT] = {};
  int max_zone = 0;
  const int* first_of(int sh) const { return first + sh * (n + 1); }
};

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
  size_t fbytes = 0;       // bytes of one population buffer (with model 1: the melt's lattice, then the gas's)
  size_t fcomp = 0;        // bytes of one lattice's populations in it
  int ncomp = 1;           // lattices: 1, or 2 with model 1
  void* f[2] = {nullptr, nullptr};
  Ctl* ctl = nullptr;      // run control of the step kernel
  Ctl* qctl = nullptr;     // always-zero control for query pipelines
  double* partials = nullptr;
  int max_blk = 0;
  void* psi = nullptr;     // two-pass path: psi and rho arrays (compute type)
  void* rho = nullptr;
  void* psi_g = nullptr;   // model 1: psi and rho of the gas lattice (compute type)
  void* rho_g = nullptr;
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
  unsigned long long* bits = nullptr;  // flag words: one bit per cell, set where the cell has barrier links
  unsigned long long* bfw = nullptr;   // BFS frontier words (three bitsets)
  long long nwords = 0;                // 64-bit words per bitset
  unsigned long long* srcw = nullptr;  // gas-release source: bits of the domain gas points (growth_on);
                                       // their number is ctl->n_src
  long long* events = nullptr;
  unsigned ev_cap = 1u << 16;
  // map-kernel tables: film refresh from the state or the rho array, label
  // queries from the state or a field
  flb_rt::MapSet ms_refresh, qs_pop, qs_field, ms_import;
  flb_rt::Fork fork;  // side stream of the refresh
  bool ms_ready = false;
  // query scratch
  double* qd = nullptr;    // (1 + 3) * N doubles
  int* qlabel = nullptr;
  unsigned long long* qsizes = nullptr;
  unsigned long long* qhist = nullptr;
  int qhist_cap = 0;
  double* qtot = nullptr;  // 4 doubles
  unsigned long long* qtab = nullptr;  // label-overlap table: qtab_cap keys, then qtab_cap counts
  long long qtab_cap = 0;
  long long launched = 0;
  bool in_batch = false;   // owned by a batch (flb_destroy refuses it)
  int dev = 0;             // the device current at creation (holds every buffer)
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
  // the segment length of the launch: the tuning's, or a flat tile's rows
  int seg_len() const { return tcfg().fh ? tcfg().fh : lz; }
  int nblocks() const {
    if (two_pass()) return geo.nxb * (int)((md.nm * (long long)md.nz + TP_ROWS - 1) / TP_ROWS);
    return tiles_x() * tiles_m() * ((md.nz + seg_len() - 1) / seg_len());
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
  // D2Q9: the flat 64 x 8-row tile; D3Q19: 64x8 tiles, ~256 long marches
  // (one per CU), which spends the least on halo planes.  Workgroups are
  // spread over the 8 XCDs.
  c->tile = c->D == 2 ? 3 : 1;
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
  a.lz = c->seg_len();
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
  // refresh_src 1: the step before a refresh stores every density for it
  a.gas_k = (c->p.film_on && c->p.refresh_src == 1) ? c->p.k_own : 0;
  if (c->p.growth_on) {
    a.srcw = c->srcw;  // the kernels read N from the run control
    a.src_rate = c->p.gas_A * c->p.gas_dndt;
  }
  if (c->p.gx != 0.0 || c->p.gy != 0.0 || c->p.gz != 0.0) {
    // gravity in kernel coordinates: D2Q9 (x, y) -> (x, z)
    a.force_on = 1;
    a.gk[0] = c->p.gx;
    a.gk[1] = c->D == 3 ? c->p.gy : 0.0;
    a.gk[2] = c->D == 3 ? c->p.gz : c->p.gy;
    a.g_rho_ref = c->p.g_rho_ref;
  }
  a.flag = c->flag;
  a.mask = c->mask;
  a.flist = c->flist;
  a.own = c->own;
  a.alias = c->alias;
  a.events = c->events;
  a.ev_cap = c->ev_cap;
  a.ctl = c->ctl;
  a.partials = c->partials;
  a.buf_bytes = c->fcomp;
  a.psi = c->psi;
  a.rho = c->rho;
  a.open_z = c->p.open_z;
  a.rho_res = c->p.rho_res;
  return a;
}

// model 1: the gas lattice, in the second half of each population buffer
inline TLArgs tl_args(flb_ctx* c) {
  TLArgs t;
  memset(&t, 0, sizeof t);
  for (int k = 0; k < 2; k++) t.gbuf[k] = (char*)c->f[k] + c->fcomp;
  t.gbytes = c->fcomp;
  t.rho_g = c->rho_g;
  t.psi_g = c->psi_g;
  t.G_mg = c->p.G_mg;
  t.G_gg = c->p.G_gg;
  t.tau_g = c->p.tau_g;
  t.psi_bar_g = c->p.rho0 * (1.0 - exp(-c->p.rho_g_liquid / c->p.rho0));
  t.rho_g_res = c->p.rho_g_liquid;
  return t;
}

// the two-pass tile index of a lattice (the decomposition model 1 runs on)
inline int two_pass_tile(int D) {
  const int n = D == 2 ? kNTiles2 : kNTiles3;
  for (int t = 0; t < n; t++)
    if ((D == 2 ? kTiles2[t] : kTiles3[t]).tx == 0) return t;
  return -1;
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

// ---- map pipelines over tables of lattices ----
// Builds (or rebuilds, reusing storage of the same size) a map set.  `alloc`
// allocates device memory that lives as long as the owner.
template <class Alloc>
int mapset_build(MapSet& ms, const std::vector<MapArgs>& args, int D, Alloc&& alloc, hipStream_t st) {
  const int n = (int)args.size();
  if (!ms.tab || ms.n != n) {
    ms.tab = (MapArgs*)alloc(sizeof(MapArgs) * (size_t)n);
    ms.first = (int*)alloc(sizeof(int) * (size_t)SH_COUNT * (n + 1));
    if (!ms.tab || !ms.first) return fail(FLB_ENOMEM, "map table allocation failed");
  }
  ms.n = n;
  std::vector<int> first((size_t)SH_COUNT * (n + 1), 0);
  ms.max_zone = 0;
  for (int sh = 0; sh < SH_COUNT; sh++) {
    int* f = first.data() + sh * (n + 1);
    for (int k = 0; k < n; k++)
      f[k + 1] = f[k] + (D == 2 ? map_share<D2Q9K>(sh, args[k].d) : map_share<D3Q19K>(sh, args[k].d));
    ms.total[sh] = f[n];
  }
  for (const MapArgs& a : args) ms.max_zone = std::max(ms.max_zone, a.zone_width);
  HIPCHK(hipMemcpyAsync(ms.tab, args.data(), sizeof(MapArgs) * (size_t)n, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(ms.first, first.data(), sizeof(int) * first.size(), hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  return FLB_OK;
}

// The map arguments of a context: its film refresh (gated by its own run
// control and k_own), or a labels-only query (gated by the zeroed query
// control) from the stored state, a host field or the two-pass rho array.
inline MapArgs map_args(flb_ctx* c, bool query, int src) {
  MapArgs a;
  memset(&a, 0, sizeof a);
  a.ctl = query ? c->qctl : c->ctl;
  a.sctl = c->ctl;
  a.d = c->md;
  a.geo = c->geo;
  a.b0 = c->f[0];
  a.b1 = c->f[1];
  a.src = src == GAS_FIELD ? (const void*)c->qd : (src == GAS_AUTO ? c->rho : nullptr);
  a.rho_th = c->p.rho_th;
  a.k_own = query ? 0 : c->p.k_own;
  a.zone_width = c->p.zone_width;
  a.refresh = query ? 0 : 1;
  a.nrb = (int)((c->N + RANK_BLOCK - 1) / RANK_BLOCK);
  a.par = c->par;
  a.rank = c->rank;
  a.counts = c->counts;
  a.label = query ? c->qlabel : c->label;
  a.n_out = query ? &c->qctl->n_bubbles : &c->ctl->n_bubbles;
  if (!query) {
    a.label_old = c->label_old;
    a.alias = c->alias;
    a.alias_old = c->alias_old;
    a.rep = c->rep;
    a.own = c->own;
    a.dist = c->dist;
    a.flag = c->flag;
    a.mask = c->mask;
    a.flist = c->flist;
    a.fwords = c->bits;
    a.bfw = c->bfw;
  }
  return a;
}

#define MAPL(K, SH, NT, ...) \
  hipLaunchKernelGGL(K, dim3(s.total[SH]), dim3(NT), 0, st, s.tab, s.first_of(SH), s.n, ##__VA_ARGS__)

// Barrier masks, the flagged-cell list and its density marks from the
// owners, distances and aliases in place.
template <class L>
int map_masks(const MapSet& s, hipStream_t st) {
  if constexpr (L::HAS_M) MAPL((k_masks_z<L>), SH_MASKZ, BFS_NT);
  else MAPL((k_masks<L>), SH_MASKT, BFS_NT);
  MAPL(k_flag_count, SH_FW, FW_BLOCK);
  MAPL(k_scan_counts, SH_ONE, 1024, 1);
  MAPL(k_flag_write, SH_FW, FW_BLOCK);
  MAPL((k_rho_marks<L>), SH_LIST, MAP_NT);
  MAPL(k_masks_done, SH_ONE, 64);
  HIPCHK(hipGetLastError());
  return FLB_OK;
}

// Labels (gas cells, connected components, canonical ranks), and for a film
// refresh also owners and distances, alias carry, barrier masks, the list of
// flagged cells and its density marks.  No synchronisation; capturable.
template <class L, class S>
int map_pipeline(const MapSet& s, hipStream_t st, int src, bool refresh, const Fork* fk = nullptr) {
  if (refresh) MAPL(k_keep_old, SH_CELLS, MAP_NT);
  constexpr int CNT = CCTile<L>::NT;
  if (src == GAS_POP) MAPL((k_cc_local<L, S, GAS_POP>), SH_CCT, CNT);
  else if (src == GAS_AUTO) MAPL((k_cc_local<L, S, GAS_AUTO>), SH_CCT, CNT);
  else MAPL((k_cc_local<L, S, GAS_FIELD>), SH_CCT, CNT);
  MAPL((k_cc_cross<L>), SH_CCT, MAP_NT);
  MAPL(k_cc_compress, SH_RANK, RANK_BLOCK);
  MAPL(k_scan_counts, SH_ONE, 1024, 0);
  MAPL(k_write_rank, SH_RANK, RANK_BLOCK);
  MAPL(k_write_labels, SH_CELLS, MAP_NT);
  if (refresh) {
    const bool fork = fk && fk->side;
    if (fork) {
      HIPCHK(hipEventRecord(fk->a, st));
      HIPCHK(hipStreamWaitEvent(fk->side, fk->a, 0));
    }
    {
      hipStream_t st_main = st;
      hipStream_t st = fork ? fk->side : st_main;  // the alias carry, beside the BFS
      MAPL(k_alias_reset, SH_FEW, MAP_NT);
      MAPL(k_alias_carry1, SH_CELLS, MAP_NT);
      MAPL(k_alias_carry2, SH_CELLS, MAP_NT);
      MAPL(k_alias_compress, SH_FEW, MAP_NT);
      if (fork) HIPCHK(hipEventRecord(fk->b, st));
    }
    for (int layer = 1; layer <= std::min(s.max_zone - 1, bfs_hot_layers(s.max_zone)); layer++)
      MAPL((k_bfs_blk<L>), SH_BFSB, 256, layer, 0);
    if (fork) HIPCHK(hipStreamWaitEvent(st, fk->b, 0));
  }
  if (refresh) return map_masks<L>(s, st);
  HIPCHK(hipGetLastError());
  return FLB_OK;
}
// the BFS layers a refresh defers (run), then the maps are whole; or (run
// false) the maps given are whole already
template <class L>
int map_deferred(const MapSet& s, hipStream_t st, bool run) {
  if (run)
    for (int layer = bfs_hot_layers(s.max_zone) + 1; layer <= s.max_zone - 1; layer++)
      MAPL((k_bfs_blk<L>), SH_BFSB, 256, layer, 1);
  MAPL(k_maps_whole, SH_ONE, 64);
  HIPCHK(hipGetLastError());
  return FLB_OK;
}

#undef MAPL

// the context's own map sets, built on first use
inline int ctx_mapsets(flb_ctx* c) {
  if (c->ms_ready) return FLB_OK;
  auto al = [c](size_t n) { return c->dalloc(n); };
  std::vector<MapArgs> q{map_args(c, true, GAS_POP)};
  int rc = mapset_build(c->qs_pop, q, c->D, al, c->st);
  if (!rc) {
    q[0] = map_args(c, true, GAS_FIELD);
    rc = mapset_build(c->qs_field, q, c->D, al, c->st);
  }
  if (!rc && c->p.film_on) {
    std::vector<MapArgs> r{map_args(c, false, GAS_AUTO)};
    rc = mapset_build(c->ms_refresh, r, c->D, al, c->st);
    if (!rc) {  // imported maps: masks at any step
      r[0] = map_args(c, false, GAS_POP);
      r[0].k_own = 0;
      rc = mapset_build(c->ms_import, r, c->D, al, c->st);
    }
  }
  if (!rc) c->ms_ready = true;
  return rc;
}

// the rho array no longer holds densities for the next refresh (the state was
// replaced): that refresh labels the state itself
inline int forget_rho(flb_ctx* c) {
  static const long long none = -1;
  HIPCHK(hipMemcpyAsync(&c->ctl->rho_step, &none, sizeof none, hipMemcpyHostToDevice, c->st));
  return FLB_OK;
}

// ---- film-map refresh of one context before its step ----
// (from the densities the previous step stored, else from the state)
template <class L, class S>
int refresh_maps(flb_ctx* c) {
  int rc = ctx_mapsets(c);
  if (rc) return rc;
  rc = c->fork.init();
  if (rc) return rc;
  return map_pipeline<L, S>(c->ms_refresh, c->st, GAS_AUTO, true, &c->fork);
}

// ---- the BFS layers a refresh defers, before owner / dist are read ----
// (a no-op unless the last refresh left them out; film_on only)
template <class L>
int complete_maps(flb_ctx* c) {
  int rc = ctx_mapsets(c);
  if (rc) return rc;
  return map_deferred<L>(c->ms_import, c->st, true);
}

// ---- labels of the current state, or of the field in c->qd ----
template <class L, class S>
int label_query(flb_ctx* c, bool from_field) {
  int rc = ctx_mapsets(c);
  if (rc) return rc;
  HIPCHK(hipMemsetAsync(c->qctl, 0, sizeof(Ctl), c->st));
  return map_pipeline<L, S>(from_field ? c->qs_field : c->qs_pop, c->st, from_field ? GAS_FIELD : GAS_POP, false);
}

// `ev`, if given, holds kPhaseEv events per step recorded on the context
// stream: before the refresh (if due), before the step kernel(s), after them,
// after the rupture test and pruning, and after the finisher; consecutive
// pairs bracket the four phases of the step
constexpr int kPhaseEv = 5;
template <class L, class S>
int do_steps(flb_ctx* c, int64_t nsteps, bool refresh, hipEvent_t* ev = nullptr) {
  const StepArgs a = step_args(c);
  const int nblk = c->nblocks();
  const StepFn fn = c->tcfg().fn[c->p.storage];
  const StepFn coll = c->tcfg().coll[c->p.storage];
  const bool tl = c->p.model == 1;
  const TLArgs t = tl ? tl_args(c) : TLArgs{};
  for (int64_t s = 0; s < nsteps; s++) {
    hipEvent_t* e = ev ? ev + kPhaseEv * s : nullptr;
    const bool due = refresh && c->p.film_on && c->launched % c->p.k_own == 0;
    if (e) HIPCHK(hipEventRecord(e[0], c->st));
    if (due) {
      int rc = refresh_maps<L, S>(c);
      if (rc) return rc;
    }
    if (e) HIPCHK(hipEventRecord(e[1], c->st));
    if (tl) {
      launch_tl<L, S>(a, t, nblk, c->st);  // both lattices: k_psi_tl, k_collide_tl
    } else {
      fn(a, nblk, c->st);              // fused step, or rho / psi of the two-pass variant
      if (coll) coll(a, nblk, c->st);  // the two-pass collide
    }
    if (e) HIPCHK(hipEventRecord(e[2], c->st));
    // rupture test (applies its unions), pruning of united pairs' links,
    // then the finisher, which closes the step
    const bool fold =
        c->two_pass() && nblk > 8 * FIN_NT && nblk + (nblk + FOLD - 1) / FOLD <= c->max_blk + c->max_blk / FOLD + 1;
    const bool test = c->p.film_on && c->launched >= c->p.rupture_warmup;
    if (test) {
      if (tl)
        hipLaunchKernelGGL((k_rupture_tl<L, typename S::ct>), dim3(list_grid(c->N)), dim3(MAP_NT), 0, c->st, a, t);
      else
        hipLaunchKernelGGL((k_rupture<L, typename S::ct>), dim3(list_grid(c->N)), dim3(MAP_NT), 0, c->st, a);
      // without the fold, the pruning launch also closes the step
      if (fold || e)
        hipLaunchKernelGGL((k_mask_prune<L>), dim3(list_grid(c->N)), dim3(MAP_NT), 0, c->st, prune_args(c));
      else
        hipLaunchKernelGGL((k_prune_finish<L>), dim3(list_grid(c->N)), dim3(MAP_NT), 0, c->st, prune_args(c), a, nblk);
    }
    if (e) HIPCHK(hipEventRecord(e[3], c->st));
    if (test && !fold && !e) {
      // closed by the pruning launch
    } else if (fold) {
      // fold the many partials of the two-pass decomposition first
      const int nf = (nblk + FOLD - 1) / FOLD;
      hipLaunchKernelGGL(k_fold_partials, dim3(nf), dim3(64), 0, c->st, a.partials, nblk);
      StepArgs af = a;
      af.partials = a.partials + 4ll * nblk;
      hipLaunchKernelGGL(k_step_finish, dim3(1), dim3(FIN_NT), 0, c->st, af, nf);
    } else {
      hipLaunchKernelGGL(k_step_finish, dim3(1), dim3(FIN_NT), 0, c->st, a, nblk);
    }
    if (e) HIPCHK(hipEventRecord(e[4], c->st));
    c->launched++;
  }
  HIPCHK(hipGetLastError());
  return FLB_OK;
}

// `lat` selects the lattice of a model-1 context (0 melt, 1 gas): its
// populations start lat * fcomp bytes into each buffer
inline void* lat_buf(const flb_ctx* c, int which, int lat) { return (char*)c->f[which] + (size_t)lat * c->fcomp; }

template <class L, class S>
int do_pack(flb_ctx* c, const double* field_dev, int mode, int which, int lat = 0) {
  const int B = 256, g = grid_for(c->N, B);
  hipLaunchKernelGGL((k_pack<L, S>), dim3(g), dim3(B), 0, c->st, lat_buf(c, which, lat), c->geo, c->md, field_dev,
                     mode);
  HIPCHK(hipGetLastError());
  return FLB_OK;
}

// FP64 moments into rho (N) and, with_j, the D momentum planes after it
template <class L, class S>
int do_moments(flb_ctx* c, bool with_j, int lat = 0, double* out = nullptr) {
  const int B = 256, g = grid_for(c->N, B);
  double* rho = out ? out : c->qd;
  hipLaunchKernelGGL((k_moments<L, S>), dim3(g), dim3(B), 0, c->st, lat_buf(c, 0, lat), lat_buf(c, 1, lat), c->ctl,
                     c->geo, c->md, rho, with_j ? rho + c->N : nullptr);
  HIPCHK(hipGetLastError());
  return FLB_OK;
}

template <class L, class S>
int do_unpack(flb_ctx* c, double* out_dev, int lat = 0) {
  const int B = 256, g = grid_for(c->N, B);
  hipLaunchKernelGGL((k_unpack<L, S>), dim3(g), dim3(B), 0, c->st, lat_buf(c, 0, lat), lat_buf(c, 1, lat), c->ctl,
                     c->geo, c->md, out_dev);
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
  if (p->refresh_src != 0 && p->refresh_src != 1) return fail(FLB_EINVAL, "refresh_src must be 0 or 1");
  if (p->growth_on != 0 && p->growth_on != 1) return fail(FLB_EINVAL, "growth_on must be 0 or 1");
  if (!isfinite(p->gas_A) || !isfinite(p->gas_dndt)) return fail(FLB_EINVAL, "non-finite gas-release parameter");
  if (!(p->f16_rho_ref >= 0.0) || !(p->f16_rho_ref <= 1e4)) return fail(FLB_EINVAL, "f16_rho_ref must be in 0..1e4");
  if (!isfinite(p->gx) || !isfinite(p->gy) || !isfinite(p->gz) || !isfinite(p->g_rho_ref))
    return fail(FLB_EINVAL, "non-finite body-force parameter");
  if (p->lattice == FLB_D2Q9 && p->gz != 0.0) return fail(FLB_EINVAL, "D2Q9 requires gz == 0");
  if (p->model != 0 && p->model != 1) return fail(FLB_EINVAL, "model must be 0 or 1");
  if (p->open_z != 0 && p->open_z != 1) return fail(FLB_EINVAL, "open_z must be 0 or 1");
  if (p->open_z && (!(p->rho_res > 0.0) || !isfinite(p->rho_res))) return fail(FLB_EINVAL, "rho_res must be > 0");
  if (p->model == 1) {
    if (p->storage == FLB_F16S) return fail(FLB_EINVAL, "model 1 needs FLB_F64 or FLB_F32 storage");
    if (p->gx != 0.0 || p->gy != 0.0 || p->gz != 0.0) return fail(FLB_EINVAL, "model 1 has no body force");
    if (!(p->tau_g > 0.5) || !isfinite(p->tau_g)) return fail(FLB_EINVAL, "tau_g must be > 0.5");
    if (!isfinite(p->G_mg) || !isfinite(p->G_gg)) return fail(FLB_EINVAL, "non-finite coupling");
    if (!(p->rho_g_bubble > 0.0) || !(p->rho_g_liquid > 0.0) || !isfinite(p->rho_g_bubble) ||
        !isfinite(p->rho_g_liquid))
      return fail(FLB_EINVAL, "rho_g_bubble and rho_g_liquid must be > 0");
  }
  return FLB_OK;
}

inline int read_ctl(flb_ctx* c, Ctl* out) {
  HIPCHK(hipMemcpyAsync(out, c->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipStreamSynchronize(c->st));
  return FLB_OK;
}

}  // namespace flb_rt
