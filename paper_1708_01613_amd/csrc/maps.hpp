// maps.hpp -- integer film maps on the device (Sec. 2.1.5, Fig. shanchenflowchart).
//
//  labels    : gas iff rho < rho_th; periodic connected components over the
//              lattice links (8 neighbours on D2Q9, 18 on D3Q19) by lock-free
//              union-find whose roots are always the smallest cell index, so
//              the result does not depend on scheduling; canonical label =
//              1 + rank of the component's smallest index.
//  owner/dist: layer-by-layer multi-source BFS from the gas cells, keeping the
//              smallest and largest label among the nearest bubbles, truncated
//              at zone_width - 1 hops.
//  alias     : union-find over labels; a rupture unites a pair; at a refresh,
//              new bubbles overlapping old bubbles of one alias class are united.
//  masks     : link i of cell c is a barrier iff both ends are owned, their
//              alias-root pairs differ and dist(c) + dist(c+e_i) + 1 <=
//              zone_width.
//
// Every kernel here works on a table of lattices (MapArgs): workgroups
// [first[k], first[k+1]) of a launch serve lattice k, with a share that
// depends on the kernel's decomposition (MapShape).  A single lattice is a
// table of one; a batch refreshes all its lattices with one launch per
// kernel.  A refresh kernel does nothing for a lattice that is stopped or
// whose step is not a refresh step (steps % k_own != 0), so a batch can
// launch the refresh whenever any member is due.
#pragma once
#include <algorithm>

#include "step.hpp"

namespace flb {

// Pointers of the map tables are plain (generic) pointers, and accesses
// through them compile to flat memory instructions; these casts name the
// address space, so the accesses become global (or, for data a kernel only
// reads, scalar-capable constant) memory instructions.
#define FLB_AS_GLOBAL __attribute__((address_space(1)))
#define FLB_AS_CONST __attribute__((address_space(4)))
template <class T>
__device__ __forceinline__ FLB_AS_GLOBAL T* as_global(T* p) {
  return (FLB_AS_GLOBAL T*)p;
}
template <class T>
__device__ __forceinline__ const FLB_AS_GLOBAL T* as_global(const T* p) {
  return (const FLB_AS_GLOBAL T*)p;
}
template <class T>
__device__ __forceinline__ const FLB_AS_CONST T* as_const(const T* p) {
  return (const FLB_AS_CONST T*)p;
}
// owner pairs (int2) through the global address space, as 64-bit words
__device__ __forceinline__ int2 ld_pair(const int2* p, unsigned i) {
  const long long v = as_global((const long long*)p)[i];
  return make_int2((int)v, (int)(v >> 32));
}
__device__ __forceinline__ void st_pair(int2* p, unsigned i, int2 v) {
  as_global((long long*)p)[i] = (long long)((unsigned long long)(unsigned)v.x | ((unsigned long long)(unsigned)v.y << 32));
}

struct MapDims {
  int nx, nm, nz;  // kernel coordinates
  long long N;
};

__device__ __forceinline__ long long cell_of(const MapDims& d, int x, int m, int z) {
  return x + (long long)d.nx * (m + (long long)d.nm * z);
}
__device__ __forceinline__ void coords_of(const MapDims& d, long long c, int& x, int& m, int& z) {
  x = (int)(c % d.nx);
  long long r = c / d.nx;
  m = (int)(r % d.nm);
  z = (int)(r / d.nm);
}

// ---- iteration over row segments ----
// The per-cell map kernels walk the lattice in segments of 64 consecutive
// x-cells of one row (m, z), one segment per wavefront, so a wavefront's
// accesses are contiguous and the row coordinates are wave-uniform: no
// per-lane division.  Cell indices fit 32 bits (N <= 2^28).
constexpr int MAP_NT = 256;
constexpr int MAP_WAVES = MAP_NT / 64;

struct SegCell {
  int x, m, z;
  unsigned c;
  int xw[3];  // x - 1, x, x + 1 (periodic)
  unsigned rb[3][3];  // nx * (m' + nm z') for m' = m + em, z' = z + ez (periodic)
  __device__ __forceinline__ unsigned nb(int ex, int em, int ez) const { return xw[1 + ex] + rb[1 + em][1 + ez]; }
};

// calls f(const SegCell&) for every cell; `HALO` fills the neighbour tables.
// Workgroup bid of nb workgroups (the launch's, or a batch member's share).
template <bool HALO, class F>
__device__ __forceinline__ void for_cells(const MapDims& d, F&& f, unsigned bid, unsigned nb) {
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nxs = (d.nx + 63) >> 6;
  const unsigned nseg = (unsigned)nxs * (unsigned)d.nm * (unsigned)d.nz;
  for (unsigned s = bid * MAP_WAVES + wv; s < nseg; s += nb * MAP_WAVES) {
    const unsigned row = s / (unsigned)nxs;
    const int xs = (int)(s - row * (unsigned)nxs);
    SegCell q;
    q.m = (int)(row % (unsigned)d.nm);
    q.z = (int)(row / (unsigned)d.nm);
    q.x = xs * 64 + lane;
    if (q.x >= d.nx) continue;
    q.c = (unsigned)q.x + (unsigned)d.nx * row;
    if constexpr (HALO) {
      q.xw[0] = q.x == 0 ? d.nx - 1 : q.x - 1;
      q.xw[1] = q.x;
      q.xw[2] = q.x == d.nx - 1 ? 0 : q.x + 1;
      const int mm[3] = {q.m == 0 ? d.nm - 1 : q.m - 1, q.m, q.m == d.nm - 1 ? 0 : q.m + 1};
      const int zz[3] = {q.z == 0 ? d.nz - 1 : q.z - 1, q.z, q.z == d.nz - 1 ? 0 : q.z + 1};
#pragma unroll
      for (int a = 0; a < 3; a++)
#pragma unroll
        for (int b = 0; b < 3; b++) q.rb[a][b] = (unsigned)d.nx * ((unsigned)mm[a] + (unsigned)d.nm * (unsigned)zz[b]);
    }
    f(q);
  }
}
template <bool HALO, class F>
__device__ __forceinline__ void for_cells(const MapDims& d, F&& f) {
  for_cells<HALO>(d, f, blockIdx.x, gridDim.x);
}

// ---- wavefront helpers ----
__device__ __forceinline__ int wave_min_i32(int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ __forceinline__ int first_lane(unsigned long long m) { return __builtin_ctzll(m); }


// ---- per-lattice arguments of the map kernels ----
// GAS_AUTO: the densities a step kernel stored for the refresh (the rho
// array, when it holds the step before this one), else the stored state
enum GasSrc { GAS_POP = 0, GAS_FIELD = 1, GAS_AUTO = 2 };

struct MapArgs {
  Ctl* ctl;               // gate: run control of the lattice (or a zeroed query control)
  const Ctl* sctl;        // run control whose step count selects the current population buffer
  MapDims d;
  Geo geo;                // population layout (gas from the stored state)
  const void* b0;
  const void* b1;
  const void* src;        // a cell-linear density field: FP64 (GAS_FIELD) or compute type (GAS_AUTO)
  double rho_th;
  int k_own;              // refresh steps: steps % k_own == 0 (0: every launch, queries)
  int zone_width;
  int refresh;            // 1: film refresh (owners, aliases, masks); 0: labels only
  int nrb;                // rank blocks, ceil(N / RANK_BLOCK)
  int* par;
  int* rank;
  int* counts;
  int* label;             // labels out
  int* n_out;             // label count out
  int* label_old;
  int* alias;
  int* alias_old;
  int* rep;
  int2* own;
  uint8_t* dist;
  uint8_t* flag;
  uint32_t* mask;
  int* flist;
  unsigned long long* fwords;  // flag words: bit l of word s = cell 64 xs + l of its row has links
  unsigned long long* bfw;     // BFS frontier words, 3 slots of one bit per cell (layer L in slot L % 3)
};

__device__ __forceinline__ bool map_due(const MapArgs& m) {
  const Ctl* c = m.ctl;
  return !c->stopped && (m.k_own == 0 || c->steps % m.k_own == 0);
}

// decompositions of a map launch (workgroups per lattice)
enum MapShape { SH_CELLS = 0, SH_CCT, SH_MASKT, SH_RANK, SH_ONE, SH_LIST, SH_FW, SH_BFSB, SH_FEW, SH_MASKZ, SH_COUNT };

#define MAP_KERNEL_PARAMS const MapArgs *__restrict__ tab, const int *__restrict__ first, int nmem
#define MAP_MEMBER                                                           \
  const int k_ = batch_member(first, nmem, blockIdx.x);                      \
  const MapArgs m = tab[k_];                                                 \
  const unsigned bid = blockIdx.x - (unsigned)first[k_];                     \
  const unsigned nbk = (unsigned)(first[k_ + 1] - first[k_]);                \
  (void)bid;                                                                 \
  (void)nbk;

// true unless the previous lane of the wavefront holds the same pair: keeps
// one lane per run of equal pairs (runs along x are the common case), so the
// remaining lanes can each do their own union or atomic at once
__device__ __forceinline__ bool run_head(int a, int b) {
  const int lane = threadIdx.x & 63;
  const int pa = __shfl_up(a, 1, 64), pb = __shfl_up(b, 1, 64);
  return lane == 0 || pa != a || pb != b;
}

// grid-stride over [0, n) within a lattice's share
#define FOR_SHARE(i, n) for (long long i = bid * (long long)blockDim.x + threadIdx.x; i < (n); i += (long long)nbk * blockDim.x)

// ---- gas cells and connected components in two phases ----
// Phase 1 (k_cc_local): a workgroup decides which cells of its tile of
// TX x TM x TZ cells are gas (rho < rho_th, from the source the refresh
// reads), labels the gas components of the tile with a union-find in LDS over
// the links that stay inside the tile, and writes every cell's parent: -1
// for liquid, the tile-local root for gas (the local order is the global
// order, so that root is the component's smallest cell index within the
// tile).  Phase 2 (k_cc_cross): the links that leave a tile (including the
// periodic wrap) unite the local roots in the global union-find; each tile
// first gathers its distinct root pairs, which are few, so few global atomics
// remain.  Large tiles keep the share of cells on tile faces, and so
// the global unions, small.
#ifndef FLB_CC_TM3
#define FLB_CC_TM3 8
#endif
#ifndef FLB_CC_TZ3
#define FLB_CC_TZ3 16
#endif
#ifndef FLB_CC_TZ2
#define FLB_CC_TZ2 64
#endif
template <class L>
struct CCTile {
  static constexpr int TX = 64;
  static constexpr int TM = L::HAS_M ? FLB_CC_TM3 : 1;
  static constexpr int TZ = L::HAS_M ? FLB_CC_TZ3 : FLB_CC_TZ2;
  static constexpr int CELLS = TX * TM * TZ;
  static constexpr int NT = CELLS / 16 > 1024 ? 1024 : (CELLS / 16 < 64 ? 64 : CELLS / 16);
  static constexpr int PER = CELLS / NT;
  static_assert(CELLS % NT == 0 && NT % 64 == 0 && PER <= 32, "CC tile shape");
};

__host__ inline int cc_tiles(const MapDims& d, int tm, int tz) {
  return ((d.nx + 63) / 64) * ((d.nm + tm - 1) / tm) * ((d.nz + tz - 1) / tz);
}

__device__ __forceinline__ int lds_find(int* lp, int a) {
  int p = lp[a];
  while (p != a) {
    a = p;
    p = lp[a];
  }
  return a;
}

__device__ __forceinline__ void lds_unite(int* lp, int a, int b) {
  while (true) {
    a = lds_find(lp, a);
    b = lds_find(lp, b);
    if (a == b) return;
    if (a < b) {
      const int t = a;
      a = b;
      b = t;
    }
    const int old = atomicCAS(&lp[a], a, b);
    if (old == a) return;
    a = old;
  }
}

// Gas sources of a refresh or a labels query (SRC):
//  GAS_POP   the density of the stored state, from its populations summed in
//            FP64;
//  GAS_AUTO  the densities the previous step stored for this refresh (the
//            rho array, cell-linear) when it holds the step before this one,
//            else as GAS_POP;
//  GAS_FIELD a cell-linear FP64 density field given by the caller.
template <class L, class S, int SRC>
__global__ __launch_bounds__(CCTile<L>::NT) void k_cc_local(MAP_KERNEL_PARAMS) {
  MAP_MEMBER
  if (!map_due(m)) return;
  using TT = CCTile<L>;
  constexpr int NT = TT::NT, PER = TT::PER;
  __shared__ int lp[TT::CELLS];
  const MapDims d = m.d;
  const int ntx = (d.nx + 63) / 64, ntm = (d.nm + TT::TM - 1) / TT::TM;
  const int b = (int)bid;
  const int tx = b % ntx, tm = (b / ntx) % ntm, tz = b / (ntx * ntm);
  const int x0 = tx * 64, m0 = tm * TT::TM, z0 = tz * TT::TZ;
  const int lane = threadIdx.x & 63;
  const int x = x0 + lane;
  // row of the tile (wave-uniform) handled by this thread's k-th cell
  auto rowk = [&](int k, int& mm_, int& z) -> bool {
    const int r = (int)(threadIdx.x >> 6) + k * (NT / 64);
    mm_ = m0 + r % TT::TM;
    z = z0 + r / TT::TM;
    return mm_ < d.nm && z < d.nz;
  };
  const bool xin = x < d.nx;
  const bool from_rho = SRC == GAS_AUTO && m.sctl->steps > 0 && m.sctl->rho_step == m.sctl->steps - 1;
  const void* pops = (m.sctl->steps & 1) ? m.b1 : m.b0;
  unsigned gas = 0;  // bit k: the k-th cell is gas
#pragma unroll 2
  for (int k = 0; k < PER; k++) {
    int mm_, z;
    if (!rowk(k, mm_, z) || !xin) continue;
    const unsigned c = (unsigned)x + (unsigned)d.nx * ((unsigned)mm_ + (unsigned)d.nm * (unsigned)z);
    double r;
    if constexpr (SRC == GAS_FIELD) {
      r = ((const double*)m.src)[c];
    } else {
      if (from_rho) {
        r = (double)((const typename S::ct*)m.src)[c];
      } else {
        typename S::ct f[L::Q];
        load_pulled<L, S>(pops, m.geo, x, mm_, z, f);
        r = 0.0;
#pragma unroll
        for (int i = 0; i < L::Q; i++) r += (double)f[i];
      }
    }
    if (r < m.rho_th) gas |= 1u << k;
  }
  // a wavefront's k-th row is one tile row (lanes = x): the gas runs along x
  // are components already, so every gas cell starts at its run's first cell.
  // On a film refresh the row's gas word is also the BFS frontier of layer 0.
  const int nxs = (d.nx + 63) >> 6;
#pragma unroll
  for (int k = 0; k < PER; k++) {
    const int l = threadIdx.x + k * NT;
    const bool g = (gas >> k) & 1u;
    const unsigned long long bg = __ballot(g);
    int mm_, z;
    if (m.refresh && lane == 0 && rowk(k, mm_, z))
      m.bfw[(unsigned)tx + (unsigned)nxs * ((unsigned)mm_ + (unsigned)d.nm * (unsigned)z)] = bg;
    const unsigned long long starts = bg & ~(bg << 1);
    const unsigned long long upto = starts & ((2ull << lane) - 1ull);  // lane 63: all bits
    lp[l] = g ? (l & ~63) + (63 - __clzll((long long)upto)) : -1;
  }
  __syncthreads();
  // links leaving the row: the parents across all of a cell's links are read
  // together, a lane's repeated parents count once, and one union is made per
  // run of equal (run, run) pairs, the runs' unions concurrently.  Rows of a
  // wavefront without gas are skipped.  (A parent read before this row's
  // unions may since have been hooked; a union finds the roots anyway.)
  constexpr int NQ = (L::Q - 1) / 2;
#pragma unroll
  for (int k = 0; k < PER; k++) {
    if (!__ballot((gas >> k) & 1u)) continue;
    const int l = threadIdx.x + k * NT;
    const int lx = l & 63, lm = (l >> 6) % TT::TM, lz = (l >> 6) / TT::TM;
    const bool g = (gas >> k) & 1u;
    int bn[NQ];
#pragma unroll
    for (int p = 0; p < NQ; p++) {
      const int i = 2 * p + 1;  // one direction of each opposite pair
      const int nx_ = lx + L::ex[i], nm_ = lm + L::em[i], nz_ = lz + L::ez[i];
      bn[p] = -1;
      if (L::em[i] == 0 && L::ez[i] == 0) continue;  // along x: inside the runs
      if (g && nx_ >= 0 && nx_ < 64 && nm_ >= 0 && nm_ < TT::TM && nz_ >= 0 && nz_ < TT::TZ &&
          x0 + nx_ < d.nx && m0 + nm_ < d.nm && z0 + nz_ < d.nz)
        bn[p] = lp[nx_ + 64 * (nm_ + TT::TM * nz_)];
    }
    const int a = g ? lp[l] : -1;
#pragma unroll
    for (int p = 1; p < NQ; p++) {
      bool seen = false;
#pragma unroll
      for (int q = 0; q < p; q++) seen |= bn[q] == bn[p];
      if (seen) bn[p] = -1;
    }
#pragma unroll
    for (int p = 0; p < NQ; p++) {
      const int i = 2 * p + 1;
      if (L::em[i] == 0 && L::ez[i] == 0) continue;
      const int aa = bn[p] >= 0 ? a : -1;
      const bool head = run_head(aa, bn[p]);
      if (aa >= 0 && head) lds_unite(lp, aa, bn[p]);
    }
  }
  __syncthreads();
  // every cell's parent: its tile-local root, or -1
#pragma unroll
  for (int k = 0; k < PER; k++) {
    const int l = threadIdx.x + k * NT;
    int mm_, z;
    if (!rowk(k, mm_, z) || !xin) continue;
    const unsigned c = (unsigned)x + (unsigned)d.nx * ((unsigned)mm_ + (unsigned)d.nm * (unsigned)z);
    int v = -1;
    if ((gas >> k) & 1u) {
      const int r = lds_find(lp, l);
      const int rx = x0 + (r & 63), rm = m0 + (r >> 6) % TT::TM, rz = z0 + (r >> 6) / TT::TM;
      v = (int)((unsigned)rx + (unsigned)d.nx * ((unsigned)rm + (unsigned)d.nm * (unsigned)rz));
    }
    m.par[c] = v;
  }
}

// One workgroup per tile of k_cc_local.  It visits the tile's cells that can
// have a link leaving the tile (every cell of a row on an m or z tile face or
// at the lattice's last row or plane, the two end cells of the other rows,
// listed first so that no wavefront walks rows it does not need),
// gathers the distinct pairs of tile-local parents across those links in an
// LDS set, and unites each pair once after the set is complete.  A face
// crossed by one component gives one pair, however many of its cells and
// directions cross it.
constexpr int CCX_HT = 1024;  // LDS set of parent pairs (8 KiB)
template <class L>
__global__ __launch_bounds__(MAP_NT) void k_cc_cross(MAP_KERNEL_PARAMS) {
  MAP_MEMBER
  if (!map_due(m)) return;
  using TT = CCTile<L>;
  constexpr int NP = (L::Q - 1) / 2;  // one direction of each opposite pair
  constexpr int RW = TT::TM * TT::TZ, CH = 4;  // rows of a tile; rows whose loads are in flight together
  constexpr unsigned long long EMPTY = ~0ull;
  __shared__ unsigned long long ht[CCX_HT];
  const MapDims d = m.d;
  int* par = m.par;
  FLB_AS_GLOBAL int* gpar = as_global(m.par);
  const int ntx = (d.nx + 63) / 64, ntm = (d.nm + TT::TM - 1) / TT::TM;
  const int b = (int)bid;
  const int x0 = (b % ntx) * 64, m0 = ((b / ntx) % ntm) * TT::TM, z0 = (b / (ntx * ntm)) * TT::TZ;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (int i = threadIdx.x; i < CCX_HT; i += MAP_NT) ht[i] = EMPTY;
  __syncthreads();
  const int xlast = min(x0 + 63, d.nx - 1);
  // the pair (lo, hi) into the set; a crowded set unites at once
  auto insert = [&](int p, int q) {
    const int lo = min(p, q), hi = max(p, q);
    const unsigned long long key = ((unsigned long long)(unsigned)lo << 32) | (unsigned)hi;
    unsigned h = (unsigned)lo * 0x9E3779B1u ^ (unsigned)hi * 0x85EBCA77u;
    h = (h ^ (h >> 16)) & (CCX_HT - 1);
    for (int t = 0; t < 16; t++) {
      const unsigned long long old = atomicCAS(&ht[h], EMPTY, key);
      if (old == EMPTY || old == key) return;
      h = (h + 1) & (CCX_HT - 1);
    }
    uf_unite(par, lo, hi);
  };
  // the remote parents of cell (x, mm_, z) with parent pc, in the chosen
  // directions whose neighbour lies in another tile (-1 elsewhere)
  auto remote = [&](int x, int mm_, int z, int pc, int (&py)[NP]) {
#pragma unroll
    for (int p = 0; p < NP; p++) {
      const int i = 2 * p + 1;
      const int xu = x + L::ex[i], mu = mm_ + L::em[i], zu = z + L::ez[i];
      const bool local = xu >= 0 && xu < d.nx && (xu >> 6) == (x >> 6) && mu >= 0 && mu < d.nm &&
                         mu / TT::TM == mm_ / TT::TM && zu >= 0 && zu < d.nz && zu / TT::TZ == z / TT::TZ;
      py[p] = -1;
      if (pc >= 0 && !local) {
        const unsigned y = (unsigned)wrap_any(xu, d.nx) +
                           (unsigned)d.nx * ((unsigned)wrap_any(mu, d.nm) + (unsigned)d.nm * wrap_any(zu, d.nz));
        py[p] = __atomic_load_n(&gpar[y], __ATOMIC_RELAXED);
      }
    }
    // a lane's repeated remote parents count once
#pragma unroll
    for (int p = 1; p < NP; p++) {
      bool seen = false;
#pragma unroll
      for (int q = 0; q < p; q++) seen |= py[q] == py[p];
      if (seen) py[p] = -1;
    }
  };
  // the tile's rows: those on an m or z face (or the lattice's last row or
  // plane), whose cells all may have links leaving the tile, and the others,
  // where only the two end cells may
  __shared__ unsigned short frow[RW], erow[RW];
  __shared__ int nfr, ner;
  if (threadIdx.x == 0) nfr = ner = 0;
  __syncthreads();
  for (int r = threadIdx.x; r < RW; r += MAP_NT) {
    const int lm = r % TT::TM, lz = r / TT::TM, mm_ = m0 + lm, z = z0 + lz;
    if (mm_ < d.nm && z < d.nz) {
      const bool face = (L::HAS_M && (lm == 0 || lm == TT::TM - 1 || mm_ == d.nm - 1)) || lz == 0 ||
                        lz == TT::TZ - 1 || z == d.nz - 1;
      if (face) frow[atomicAdd(&nfr, 1)] = (unsigned short)r;
      else erow[atomicAdd(&ner, 1)] = (unsigned short)r;
    }
  }
  __syncthreads();
  const int nf = nfr, ne = ner;
  // face rows, whole, CH at a time per wavefront (wave-uniform loop)
  const int x = x0 + lane;
  for (int k0 = wv * CH; k0 < nf; k0 += MAP_WAVES * CH) {
    int pc[CH], ms[CH], zs[CH];
#pragma unroll
    for (int u = 0; u < CH; u++) {
      const int r = frow[min(k0 + u, nf - 1)];
      ms[u] = m0 + r % TT::TM;
      zs[u] = z0 + r / TT::TM;
      const bool act = k0 + u < nf && x < d.nx;
      pc[u] = act ? gpar[(unsigned)x + (unsigned)d.nx * ((unsigned)ms[u] + (unsigned)d.nm * (unsigned)zs[u])] : -1;
    }
    int py[CH][NP];
#pragma unroll
    for (int u = 0; u < CH; u++) remote(x, ms[u], zs[u], pc[u], py[u]);
#pragma unroll
    for (int u = 0; u < CH; u++) {
      if (!__ballot(pc[u] >= 0)) continue;
      // the runs of equal pairs along x go into the set once
#pragma unroll
      for (int p = 0; p < NP; p++) {
        const int ra = py[u][p] >= 0 ? pc[u] : -1, rb = py[u][p];
        const bool head = run_head(ra, rb);
        if (ra >= 0 && ra != rb && head) insert(ra, rb);
      }
    }
  }
  // the end cells of the other rows, one per thread
  for (int k = threadIdx.x; k < 2 * ne; k += MAP_NT) {
    const int r = erow[k >> 1];
    const int xe = (k & 1) ? xlast : x0, mm_ = m0 + r % TT::TM, z = z0 + r / TT::TM;
    const bool act = !((k & 1) && xlast == x0);
    const int pc = act ? gpar[(unsigned)xe + (unsigned)d.nx * ((unsigned)mm_ + (unsigned)d.nm * (unsigned)z)] : -1;
    int py[NP];
    remote(xe, mm_, z, pc, py);
#pragma unroll
    for (int p = 0; p < NP; p++)
      if (py[p] >= 0 && py[p] != pc) insert(pc, py[p]);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < CCX_HT; i += MAP_NT) {
    const unsigned long long k = ht[i];
    if (k != EMPTY) uf_unite(par, (int)(k >> 32), (int)(unsigned)(k & 0xffffffffull));
  }
}

// ---- canonical ranks: count roots per block, scan, write labels ----
constexpr int RANK_BLOCK = 1024;
constexpr int FW_BLOCK = 1024;  // flag words per workgroup (flagged-list build)

// Every gas cell points at its component's root (path compression: a
// concurrent reader sees either the old parent or the root, both lead to the
// root), and each block of RANK_BLOCK cells counts the roots it holds.
static __global__ __launch_bounds__(RANK_BLOCK) void k_cc_compress(MAP_KERNEL_PARAMS) {
  MAP_MEMBER
  if (!map_due(m)) return;
  const long long c = bid * (long long)RANK_BLOCK + threadIdx.x;
  int is_root = 0;
  if (c < m.d.N && m.par[c] >= 0) {
    const int r = uf_find_live(m.par, (int)c);
    m.par[c] = r;
    is_root = r == (int)c;
  }
  __shared__ int s[RANK_BLOCK / 64];
  const unsigned long long bal = __ballot(is_root);
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = __popcll(bal);
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < RANK_BLOCK / 64; w++) t += s[w];
    m.counts[bid] = t;
  }
}

// one workgroup per lattice: exclusive scan of the per-block counts; the
// total goes to *n_out (which 0: roots per rank block, the label count) or
// to ctl->n_flagged (which 1: flagged cells per flag-word block).  A pass
// loads 16 Ki counts at once (each thread four 16-byte groups, coalesced)
// and scans them as four chunks of 4096 in order, a thread holding four
// consecutive counts of each chunk (the 256^3 lattice in one pass).
static __global__ __launch_bounds__(1024) void k_scan_counts(MAP_KERNEL_PARAMS, int which) {
  MAP_MEMBER
  if (!map_due(m)) return;
  constexpr int CHK = 4096, NCH = 4;
  __shared__ int s_carry;
  __shared__ int s_w[16];
  if (threadIdx.x == 0) s_carry = 0;
  __syncthreads();
  const long long nwords = (long long)((m.d.nx + 63) >> 6) * m.d.nm * m.d.nz;
  const int nblocks = which == 0 ? m.nrb : (int)((nwords + FW_BLOCK - 1) / FW_BLOCK);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int* counts = m.counts;  // 256-byte aligned
  for (int base = 0; base < nblocks; base += CHK * NCH) {
    int4 v[NCH];
#pragma unroll
    for (int k = 0; k < NCH; k++) {
      const int i = base + k * CHK + (int)threadIdx.x * 4;
      if (i + 3 < nblocks) {
        v[k] = *(const int4*)(counts + i);
      } else {
        v[k].x = i < nblocks ? counts[i] : 0;
        v[k].y = i + 1 < nblocks ? counts[i + 1] : 0;
        v[k].z = i + 2 < nblocks ? counts[i + 2] : 0;
        v[k].w = 0;
      }
    }
#pragma unroll
    for (int k = 0; k < NCH; k++) {
      if (base + k * CHK >= nblocks) break;  // uniform over the workgroup
      const int i = base + k * CHK + (int)threadIdx.x * 4;
      const int sum = v[k].x + v[k].y + v[k].z + v[k].w;
      int incl = sum;  // inclusive scan of the thread sums within the wave
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const int t = __shfl_up(incl, off, 64);
        if (lane >= off) incl += t;
      }
      if (lane == 63) s_w[w] = incl;
      __syncthreads();
      int wbase = 0;
      for (int q = 0; q < w; q++) wbase += s_w[q];
      const int carry = s_carry;
      const int e0 = carry + wbase + incl - sum;
      const int4 o = make_int4(e0, e0 + v[k].x, e0 + v[k].x + v[k].y, e0 + v[k].x + v[k].y + v[k].z);
      if (i + 3 < nblocks) {
        *(int4*)(counts + i) = o;
      } else {
        if (i < nblocks) counts[i] = o.x;
        if (i + 1 < nblocks) counts[i + 1] = o.y;
        if (i + 2 < nblocks) counts[i + 2] = o.z;
      }
      __syncthreads();
      if (threadIdx.x == 1023) s_carry = carry + wbase + incl;
      __syncthreads();
    }
  }
  if (threadIdx.x == 0) {
    if (which == 0) *m.n_out = s_carry;
    else m.ctl->n_flagged = (unsigned)s_carry;
  }
}

// rank[root] = 1-based label of the component rooted there
static __global__ __launch_bounds__(RANK_BLOCK) void k_write_rank(MAP_KERNEL_PARAMS) {
  MAP_MEMBER
  if (!map_due(m)) return;
  const long long c = bid * (long long)RANK_BLOCK + threadIdx.x;
  const int is_root = (c < m.d.N && m.par[c] == (int)c) ? 1 : 0;
  __shared__ int s[RANK_BLOCK / 64];
  const unsigned long long bal = __ballot(is_root);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) s[w] = __popcll(bal);
  __syncthreads();
  if (is_root) {
    int before = m.counts[bid];
    for (int k = 0; k < w; k++) before += s[k];
    before += __popcll(bal & ((1ull << lane) - 1ull));
    m.rank[c] = before + 1;
  }
}

// Labels; on a film refresh also the start of the owner BFS: gas cells are
// their own owners at distance 0, every other cell is unreached (dist 255;
// its owner pair is left as it was and is never read: every reader of the
// owners reads them at cells with a distance).
static __global__ __launch_bounds__(MAP_NT) void k_write_labels(MAP_KERNEL_PARAMS) {
  MAP_MEMBER
  if (!map_due(m)) return;
  const bool film = m.refresh;
  FOR_SHARE(c, m.d.N) {
    const int p = m.par[c];
    const int l = p < 0 ? 0 : m.rank[p];
    m.label[c] = l;
    if (film) {
      m.dist[c] = l > 0 ? 0 : 255;
      if (l > 0) m.own[c] = make_int2(l, l);
    }
  }
}

// ---- previous labels and aliases, kept for the alias carry ----
static __global__ __launch_bounds__(MAP_NT) void k_keep_old(MAP_KERNEL_PARAMS) {
  MAP_MEMBER
  if (!map_due(m)) return;
  const int nb = m.ctl->maps_seen ? m.ctl->n_bubbles : 0;  // labels of the maps in force
  if (bid == 0 && threadIdx.x == 0) m.ctl->nb_old = nb;  // read by k_alias_reset, after the scan
  if (!m.ctl->maps_seen) return;
  FOR_SHARE(c, m.d.N) {
    m.label_old[c] = m.label[c];
    if (c <= nb) m.alias_old[c] = m.alias[c];
  }
}

// Layers a barrier can depend on.  A barrier link joins two owned cells with
// dist(x) + dist(y) + 1 <= zone_width, and BFS distances of neighbours differ
// by at most one, so both ends lie within zone_width / 2 hops of a bubble.
// A refresh runs only these layers; the deeper ones (up to zone_width - 1)
// fill in the exported maps when they are read.
__host__ __device__ constexpr int bfs_hot_layers(int zone_width) { return zone_width / 2; }

__device__ __forceinline__ int wrap_mod(int a, int n) {
  if (a >= 0 && a < n) return a;
  const int r = a % n;
  return r < 0 ? r + n : r;
}

constexpr int BFS_NT = 256;

// Tiles of the masks kernel (the same halo layout)
#ifndef FLB_MK_TM
#define FLB_MK_TM 4
#endif
#ifndef FLB_MK_TZ
#define FLB_MK_TZ 4
#endif
template <class L>
struct MaskTile {
  static constexpr int TM = L::HAS_M ? FLB_MK_TM : 1;
  static constexpr int TZ = L::HAS_M ? FLB_MK_TZ : 16;
  static constexpr int HM = L::HAS_M ? 1 : 0;
  static constexpr int LX = 64 + 2, LM = TM + 2 * HM, LZ = TZ + 2;
  static constexpr int CELLS = 64 * TM * TZ;
  static constexpr int HALO = LX * LM * LZ;
};

// The halo of a tile, row by row: halo row hr (LM x LZ of them) holds the
// cells x0 - 1 .. x0 + 64 of lattice row (m0 - HM + hr % LM, z0 - 1 + hr / LM),
// wrapped periodically.  Wavefront w takes rows w, w + 4, ...: its lanes load
// the 64 cells x0 + lane (x0 + lane past the lattice end wraps to the cell
// that is the periodic neighbour of the last one), lanes 0 and 1 also the
// two end cells.  The row arithmetic is wave-uniform.
template <class T>
struct HaloRows {
  static constexpr int NR = T::LM * T::LZ;
  static constexpr int RPW = (NR + BFS_NT / 64 - 1) / (BFS_NT / 64);  // rows per wavefront
  int wv, lane, xa, xe;
  __device__ HaloRows(const MapDims& d, int x0) {
    wv = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    lane = (int)threadIdx.x & 63;
    xa = wrap_mod(x0 + lane, d.nx);
    xe = wrap_mod(lane == 0 ? x0 - 1 : x0 + 64, d.nx);
  }
  __device__ __forceinline__ int row(int j) const { return wv + j * (BFS_NT / 64); }
  // first cell index of halo row hr
  __device__ __forceinline__ unsigned base(const MapDims& d, int m0, int z0, int hr) const {
    const int gm = T::HM ? wrap_mod(m0 - 1 + hr % T::LM, d.nm) : 0;
    const int gz = wrap_mod(z0 - 1 + hr / T::LM, d.nz);
    return (unsigned)d.nx * ((unsigned)gm + (unsigned)d.nm * (unsigned)gz);
  }
};

// offsets from a cell to its neighbours along one axis, periodic
struct AxisStep {
  int dn, up;
  __device__ AxisStep(int i, int n, int stride)
      : dn((i == 0 ? n - 1 : -1) * stride), up((i == n - 1 ? 1 - n : 1) * stride) {}
  __device__ __forceinline__ int of(int e) const { return e < 0 ? dn : (e > 0 ? up : 0); }
};

// ---- owner / dist by layers over frontier bitsets ----
// The frontier of layer L (the cells at distance L) is a bitset in row
// words: bit l of word xs + nxs * row is cell 64 xs + l of that row.  Layer 0
// is the gas (written by k_cc_local).  A workgroup takes a block of CW words
// along x by TM x TZ rows and
//  1. stages the frontier words of layer L - 1 of the block and a one-word,
//     one-row halo in LDS, and forms, one thread per word, the word of cells
//     reached in layer L:
//       new = (union over directions e of F_{L-1} shifted by e) & ~F_{L-1} & ~F_{L-2}
//     (a neighbour of a cell at distance L - 1 is at distance L - 2, L - 1 or
//     L), together with, for each new cell, the directions that lead to the
//     frontier;
//  2. lists the new cells of the block in LDS (a block-wide scan of the word
//     counts gives each word its place);
//  3. spreads the list over all threads, which gather the owners of each
//     listed cell's frontier neighbours (all loads of a cell in flight
//     together) and keep the smallest owner and the largest owner2.
// The bit arithmetic touches no memory beyond the staged words, and the
// gathers cover only the new cells.
#ifndef FLB_BFS_U
#define FLB_BFS_U 1
#endif
template <class L>
struct BfsBlock {
  static constexpr int CW = 4;                    // words along x
  static constexpr int TM = L::HAS_M ? 8 : 1;     // rows along m
  static constexpr int TZ = L::HAS_M ? 8 : 64;    // rows along z
  static constexpr int HM = L::HAS_M ? 1 : 0;
  static constexpr int LW = CW + 2, LM = TM + 2 * HM, LZ = TZ + 2;
  static constexpr int NT = CW * TM * TZ;         // one thread per word
  static constexpr int LIST = 2048;               // listed cells per round
  static_assert(NT == 256, "one word per thread");
};

__host__ inline int bfs_blocks(const MapDims& d, int cw, int tm, int tz) {
  return ((d.nx + 64 * cw - 1) / (64 * cw)) * ((d.nm + tm - 1) / tm) * ((d.nz + tz - 1) / tz);
}

template <class L>
__global__ __launch_bounds__(256) void k_bfs_blk(MAP_KERNEL_PARAMS, int layer, int deferred) {
  MAP_MEMBER
  if (layer > m.zone_width - 1) return;
  if (deferred ? (!m.ctl->maps_partial || layer <= bfs_hot_layers(m.zone_width))
               : (!map_due(m) || layer > bfs_hot_layers(m.zone_width)))
    return;
  using T = BfsBlock<L>;
  __shared__ unsigned long long fw[T::LW * T::LM * T::LZ];
  __shared__ uint2 list[T::LIST];
  __shared__ int wsum[T::NT / 64];
  const MapDims d = m.d;
  const int nxs = (d.nx + 63) >> 6;
  const unsigned nrows = (unsigned)d.nm * (unsigned)d.nz;
  const size_t nw = (size_t)nxs * nrows;
  const FLB_AS_GLOBAL unsigned long long* Fp = as_global((const unsigned long long*)m.bfw + (size_t)((layer - 1) % 3) * nw);
  const FLB_AS_GLOBAL unsigned long long* Fq = as_global((const unsigned long long*)m.bfw + (size_t)((layer + 1) % 3) * nw);
  FLB_AS_GLOBAL unsigned long long* Fn = as_global(m.bfw + (size_t)(layer % 3) * nw);
  const int nbx = (nxs + T::CW - 1) / T::CW, nbm = (d.nm + T::TM - 1) / T::TM;
  const int b = (int)bid;
  const int xs0 = (b % nbx) * T::CW, m0 = ((b / nbx) % nbm) * T::TM, z0 = (b / (nbx * nbm)) * T::TZ;
  // 1. stage the frontier words of the block and its halo (wrapped)
  for (int i = threadIdx.x; i < T::LW * T::LM * T::LZ; i += T::NT) {
    const int wx = i % T::LW, r = i / T::LW;
    const int gx = wrap_mod(xs0 - 1 + wx, nxs);
    const int gm = T::HM ? wrap_mod(m0 - 1 + r % T::LM, d.nm) : 0;
    const int gz = wrap_mod(z0 - 1 + r / T::LM, d.nz);
    fw[i] = Fp[(unsigned)gx + (unsigned)nxs * ((unsigned)gm + (unsigned)d.nm * (unsigned)gz)];
  }
  const int wx = threadIdx.x % T::CW, tr = threadIdx.x / T::CW;
  const int lm = tr % T::TM, lz = tr / T::TM;
  const int xs = xs0 + wx, mm_ = m0 + lm, z = z0 + lz;
  const bool own_word = xs < nxs && mm_ < d.nm && z < d.nz;
  const unsigned wi = own_word ? (unsigned)xs + (unsigned)nxs * ((unsigned)mm_ + (unsigned)d.nm * (unsigned)z) : 0u;
  const unsigned long long prev = (own_word && layer >= 2) ? Fq[wi] : 0ull;
  __syncthreads();
  unsigned long long S[L::Q];
  unsigned long long nwd = 0;
  if (own_word) {
    const int x0 = xs * 64;
    const int nval = min(64, d.nx - x0);
    const unsigned long long valid = nval == 64 ? ~0ull : (1ull << nval) - 1ull;
    unsigned long long reach = 0;
#pragma unroll
    for (int i = 1; i < L::Q; i++) {
      const int at = (wx + 1) + T::LW * ((lm + T::HM + L::em[i]) + T::LM * (lz + 1 + L::ez[i]));
      const unsigned long long w = fw[at];
      unsigned long long sh;
      if (L::ex[i] == 0) {
        sh = w;
      } else if (L::ex[i] > 0) {  // the cell right of the word: bit 0 of the next word, or cell 0 of the row
        const unsigned long long cr = fw[at + 1] & 1ull;
        sh = (w >> 1) | (cr << (nval - 1));
      } else {  // the cell left of the word: bit 63 of the previous word, or the row's last cell
        const unsigned long long cl = (fw[at - 1] >> (xs == 0 ? ((d.nx - 1) & 63) : 63)) & 1ull;
        sh = ((w << 1) | cl) & valid;
      }
      S[i] = sh;
      reach |= sh;
    }
    const unsigned long long self = fw[(wx + 1) + T::LW * ((lm + T::HM) + T::LM * (lz + 1))];
    nwd = reach & ~self & ~prev & valid;
    Fn[wi] = nwd;
  }
  // 2. places of the new cells: block-wide exclusive scan of the word counts
  const int cnt = __popcll(nwd);
  int incl = cnt;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int t = __shfl_up(incl, off, 64);
    if (lane >= off) incl += t;
  }
  if (lane == 63) wsum[wv] = incl;
  __syncthreads();
  int base = incl - cnt, total = 0;
#pragma unroll
  for (int k = 0; k < T::NT / 64; k++) {
    if (k < wv) base += wsum[k];
    total += wsum[k];
  }
  const unsigned c_row = own_word ? (unsigned)(xs * 64) + (unsigned)d.nx * ((unsigned)mm_ + (unsigned)d.nm * (unsigned)z) : 0u;
  for (int r0 = 0; r0 < total; r0 += T::LIST) {  // block-uniform rounds
    // 2. this round's part of the list: (cell, frontier directions)
    if (cnt && base < r0 + T::LIST && base + cnt > r0) {
      unsigned long long bits = nwd;
      int rank = base;
      while (bits) {
        const int l = __builtin_ctzll(bits);
        bits &= bits - 1ull;
        if (rank >= r0 && rank < r0 + T::LIST) {
          unsigned hit = 0;
#pragma unroll
          for (int i = 1; i < L::Q; i++) hit |= (unsigned)((S[i] >> l) & 1ull) << i;
          list[rank - r0] = make_uint2(c_row + (unsigned)l, hit);
        }
        rank++;
      }
    }
    __syncthreads();
    // 3. owners of the listed cells, U cells per thread at a time
    const int n = min(T::LIST, total - r0);
    constexpr int U = FLB_BFS_U;
    for (int e = threadIdx.x; e < n; e += U * T::NT) {
      int2 o[U][L::Q];
      unsigned cc[U];
      bool act[U];
#pragma unroll
      for (int u = 0; u < U; u++) {
        const int ee = e + u * T::NT;
        act[u] = ee < n;
        const uint2 ent = act[u] ? list[ee] : make_uint2(0u, 0u);
        cc[u] = ent.x;
        const unsigned r = ent.x / (unsigned)d.nx;
        const int x = (int)(ent.x - r * (unsigned)d.nx);
        const AxisStep sx(x, d.nx, 1), sm((int)(r % (unsigned)d.nm), d.nm, d.nx),
            sz((int)(r / (unsigned)d.nm), d.nz, d.nx * d.nm);
#pragma unroll
        for (int i = 1; i < L::Q; i++) {
          o[u][i] = make_int2(0x7fffffff, 0);
          if (ent.y & (1u << i))
            o[u][i] = ld_pair(m.own, (unsigned)((int)ent.x + sx.of(L::ex[i]) + sm.of(L::em[i]) + sz.of(L::ez[i])));
        }
      }
#pragma unroll
      for (int u = 0; u < U; u++) {
        if (!act[u]) continue;
        int lo = 0x7fffffff, hi = 0;
#pragma unroll
        for (int i = 1; i < L::Q; i++) {
          lo = min(lo, o[u][i].x);
          hi = max(hi, o[u][i].y);
        }
        st_pair(m.own, cc[u], make_int2(lo, hi));
        as_global(m.dist)[cc[u]] = (uint8_t)layer;
      }
    }
    __syncthreads();
  }
}

// ---- alias carry across a refresh ----
static __global__ __launch_bounds__(MAP_NT) void k_alias_reset(MAP_KERNEL_PARAMS) {
  MAP_MEMBER
  if (!map_due(m)) return;
  const int nb = m.ctl->n_bubbles, nb_old = m.ctl->nb_old;
  FOR_SHARE(b, (long long)max(nb, nb_old) + 1) {
    if (b <= nb) m.alias[b] = (int)b;
    if (b <= nb_old) m.rep[b] = 0x7fffffff;  // indexed by classes of the previous labels
  }
}

// Both carry passes run over whole wavefronts (the loop bound is uniform per
// wavefront) and merge the many lanes that carry the same (old class, new
// label) pair before touching global memory.
static __global__ __launch_bounds__(MAP_NT) void k_alias_carry1(MAP_KERNEL_PARAMS) {
  MAP_MEMBER
  if (!map_due(m) || !m.ctl->maps_seen) return;
  const int lane = threadIdx.x & 63;
  const long long stride = (long long)nbk * MAP_NT;
  for (long long base = bid * (long long)MAP_NT + (threadIdx.x & ~63); base < m.d.N; base += stride) {
    const long long c = base + lane;
    int b = 0, a = 0;
    if (c < m.d.N) {
      b = m.label[c];
      a = m.label_old[c];
    }
    const bool pend = b > 0 && a > 0;
    const int r = pend ? uf_root(m.alias_old, a) : 0;
    // one atomic per run of equal (root, label), the runs' atomics at once
    if (run_head(r, b) && pend && __atomic_load_n(&m.rep[r], __ATOMIC_RELAXED) > b) atomicMin(&m.rep[r], b);
  }
}

static __global__ __launch_bounds__(MAP_NT) void k_alias_carry2(MAP_KERNEL_PARAMS) {
  MAP_MEMBER
  if (!map_due(m) || !m.ctl->maps_seen) return;
  const int lane = threadIdx.x & 63;
  const long long stride = (long long)nbk * MAP_NT;
  for (long long base = bid * (long long)MAP_NT + (threadIdx.x & ~63); base < m.d.N; base += stride) {
    const long long c = base + lane;
    int b = 0, a = 0;
    if (c < m.d.N) {
      b = m.label[c];
      a = m.label_old[c];
    }
    const int r = (b > 0 && a > 0) ? m.rep[uf_root(m.alias_old, a)] : 0;
    const bool pend = b > 0 && a > 0 && r != b;
    if (run_head(b, r) && pend) uf_unite(m.alias, b, r);
  }
}

static __global__ __launch_bounds__(MAP_NT) void k_alias_compress(MAP_KERNEL_PARAMS) {
  MAP_MEMBER
  if (!map_due(m) || !m.ctl->maps_seen) return;
  const int nb = m.ctl->n_bubbles;
  FOR_SHARE(b, (long long)nb + 1) m.alias[b] = uf_find_live(m.alias, (int)b);
}

// Barrier masks over tiles of 64 x 4 x 4 cells (64 x 16 on D2Q9): the
// workgroup stages, for its tile and a one-cell halo, every cell's distance
// and owner pair, loaded together (larger tiles measured slower: their LDS
// halves the workgroups a CU holds, and this kernel is bound by latency).
// A link is a barrier iff both ends are owned, the film is thin enough
// (dist + dist + 1 <= zone_width) and the alias-root pairs of the two owner
// pairs differ; equal owner pairs have equal root pairs, so the aliases are
// looked up only where the owner pairs differ (near the walls between zones;
// the aliases are compressed at every refresh, so one look-up gives a root).
// Each wavefront handles whole 64-cell row segments, whose cells with links
// form one word of the flag bitset, from which k_flag_count / k_scan_counts /
// k_flag_write build the flagged-cell list in cell order (no atomics).  A tile
// without owned cells only clears its masks.
template <class L>
__global__ __launch_bounds__(BFS_NT) void k_masks(MAP_KERNEL_PARAMS) {
  MAP_MEMBER
  if (!map_due(m)) return;
  using T = MaskTile<L>;
  using H = HaloRows<T>;
  constexpr int PER = T::CELLS / BFS_NT;
  constexpr int CH = 5;  // halo rows per wavefront with loads in flight together
  __shared__ uint8_t ld[T::HALO];
  __shared__ int2 lo[T::HALO];
  const MapDims d = m.d;
  const int zone_width = m.zone_width;
  const FLB_AS_GLOBAL uint8_t* dist = as_global((const uint8_t*)m.dist);
  const int ntx = (d.nx + 63) / 64, ntm = (d.nm + T::TM - 1) / T::TM;
  const int b = (int)bid;
  const int x0 = (b % ntx) * 64, m0 = ((b / ntx) % ntm) * T::TM, z0 = (b / (ntx * ntm)) * T::TZ;
  const int lane = threadIdx.x & 63;
  const int x = x0 + lane;
  const H hr(d, x0);
  // 1. distances and owner pairs of the tile and its halo, loaded together
  // (an unreached cell's owners are stale and never read)
  bool any = false;
  for (int j0 = 0; j0 < H::RPW; j0 += CH) {
    uint8_t da[CH], de[CH];
    int2 oa[CH], oe[CH];
#pragma unroll
    for (int u = 0; u < CH; u++) {
      const int j = j0 + u;
      da[u] = de[u] = 255;
      oa[u] = oe[u] = make_int2(0, 0);
      if (j < H::RPW && hr.row(j) < H::NR) {
        const unsigned base = hr.base(d, m0, z0, hr.row(j));
        da[u] = dist[base + (unsigned)hr.xa];
        oa[u] = ld_pair(m.own, base + (unsigned)hr.xa);
        if (hr.lane < 2) {
          de[u] = dist[base + (unsigned)hr.xe];
          oe[u] = ld_pair(m.own, base + (unsigned)hr.xe);
        }
      }
    }
#pragma unroll
    for (int u = 0; u < CH; u++) {
      const int j = j0 + u;
      if (j >= H::RPW || hr.row(j) >= H::NR) continue;  // wave-uniform
      const int at = hr.row(j) * T::LX;
      ld[at + 1 + hr.lane] = da[u];
      lo[at + 1 + hr.lane] = oa[u];
      if (hr.lane < 2) {
        ld[at + (hr.lane == 0 ? 0 : T::LX - 1)] = de[u];
        lo[at + (hr.lane == 0 ? 0 : T::LX - 1)] = oe[u];
      }
      any |= da[u] != 255 || de[u] != 255;
    }
  }
  const bool owned = __syncthreads_or(any);  // block-uniform: the staging is complete
  // 2. the links of the tile's cells
  const int nxs = (d.nx + 63) >> 6;
  const FLB_AS_GLOBAL int* alias = as_global((const int*)m.alias);
  auto root_pair = [&](int2 o) {
    const int ra = alias[o.x], rb = alias[o.y];
    return make_int2(min(ra, rb), max(ra, rb));
  };
  for (int k = 0; k < PER; k++) {
    const int r = (int)(threadIdx.x >> 6) + k * (BFS_NT / 64);
    const int lm = r % T::TM, lz = r / T::TM;
    const int mm_ = m0 + lm, z = z0 + lz;
    const bool rowin = mm_ < d.nm && z < d.nz;  // wave-uniform
    const bool in = rowin && x < d.nx;
    const unsigned cidx = in ? (unsigned)x + (unsigned)d.nx * ((unsigned)mm_ + (unsigned)d.nm * (unsigned)z) : 0u;
    unsigned mk = 0;
    if (owned && in) {
      const int lc = (lane + 1) + T::LX * ((lm + T::HM) + T::LM * (lz + 1));
      const int dc = ld[lc];
      if (dc != 255) {
        const int2 oc = lo[lc];
        unsigned cand = 0;  // thin links to cells with another owner pair
#pragma unroll
        for (int i = 1; i < L::Q; i++) {
          const int li = lc + L::ex[i] + T::LX * (L::em[i] + T::LM * L::ez[i]);
          // both ends owned (dist 255 fails the sum), thin enough, different owners
          if (dc + (int)ld[li] + 1 <= zone_width) {
            const int2 on = lo[li];
            if (on.x != oc.x || on.y != oc.y) cand |= 1u << i;
          }
        }
        if (cand) {
          const int2 rc = root_pair(oc);
#pragma unroll
          for (int i = 1; i < L::Q; i++) {
            if (!(cand & (1u << i))) continue;
            const int2 rn = root_pair(lo[lc + L::ex[i] + T::LX * (L::em[i] + T::LM * L::ez[i])]);
            if (rn.x != rc.x || rn.y != rc.y) mk |= 1u << i;
          }
        }
      }
    }
    if (in) {
      as_global(m.flag)[cidx] = mk ? 1 : 0;
      as_global(m.mask)[cidx] = mk;
    }
    const unsigned long long bal = __ballot(mk != 0);
    if (rowin && lane == 0) {
      const unsigned row = (unsigned)mm_ + (unsigned)d.nm * (unsigned)z;
      as_global(m.fwords)[(unsigned)(x0 >> 6) + (unsigned)nxs * row] = bal;
    }
  }
}

// ---- barrier masks, 3-D lattices: a z-march over planes ----
// A workgroup owns 64 x MZ_TM cells of MZ_LZ consecutive planes.  Iteration k
// issues the loads of plane z0-1+k (distances and owner pairs of the plane's
// 66 x (MZ_TM + 2) staged cells, periodic), computes the masks of plane
// z0+k-3 from the three planes staged before (LDS ring of 4 planes) while
// those loads are in flight, then stages the new plane and synchronises once.
// Each staged cell is loaded once per workgroup instead of once per 64 x 4 x 4
// tile with a halo all round (1.5x the tile's cells instead of 2.3x), and the
// loads of one plane overlap the links of the previous one.  Per cell the
// links and masks are those of k_masks.
constexpr int MZ_TM = 4, MZ_LZ = 16;
template <class L>
__global__ __launch_bounds__(BFS_NT) void k_masks_z(MAP_KERNEL_PARAMS) {
  static_assert(L::HAS_M && BFS_NT == 64 * MZ_TM, "one cell of a plane per thread");
  MAP_MEMBER
  if (!map_due(m)) return;
  constexpr int LX = 66, LM = MZ_TM + 2, PL = LX * LM;
  static_assert(PL <= 2 * BFS_NT, "two staged cells per thread");
  __shared__ uint8_t sd[4][PL];
  __shared__ int2 so[4][PL];
  const MapDims d = m.d;
  const int zone_width = m.zone_width;
  const FLB_AS_GLOBAL uint8_t* dist = as_global((const uint8_t*)m.dist);
  const FLB_AS_GLOBAL int* alias = as_global((const int*)m.alias);
  const int ntx = (d.nx + 63) / 64, ntm = (d.nm + MZ_TM - 1) / MZ_TM;
  const int b = (int)bid;
  const int x0 = (b % ntx) * 64, m0 = ((b / ntx) % ntm) * MZ_TM, z0 = (b / (ntx * ntm)) * MZ_LZ;
  const int L_ = min(MZ_LZ, d.nz - z0);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int nxs = (d.nx + 63) >> 6;
  // the two staged cells of this thread: in-plane offsets (periodic)
  unsigned soff[2];
  bool sv[2];
#pragma unroll
  for (int u = 0; u < 2; u++) {
    const int st = (int)threadIdx.x + u * BFS_NT;
    sv[u] = st < PL;
    const int r = st / LX, q = st % LX;
    soff[u] = (unsigned)wrap_mod(x0 - 1 + q, d.nx) + (unsigned)d.nx * (unsigned)wrap_mod(m0 - 1 + r, d.nm);
  }
  const unsigned plane = (unsigned)d.nx * (unsigned)d.nm;
  const int x = x0 + lane, mm_ = m0 + wv;
  const bool colin = x < d.nx && mm_ < d.nm;
  const int lc = (lane + 1) + LX * (wv + 1);
  auto root_pair = [&](int2 o) {
    const int ra = alias[o.x], rb = alias[o.y];
    return make_int2(min(ra, rb), max(ra, rb));
  };
  for (int k = 0; k <= L_ + 2; k++) {  // uniform over the workgroup
    uint8_t dv[2] = {255, 255};
    int2 ov[2] = {make_int2(0, 0), make_int2(0, 0)};
    if (k <= L_ + 1) {
      const unsigned zb = plane * (unsigned)wrap_mod(z0 - 1 + k, d.nz);
#pragma unroll
      for (int u = 0; u < 2; u++)
        if (sv[u]) {
          dv[u] = dist[zb + soff[u]];
          ov[u] = ld_pair(m.own, zb + soff[u]);
        }
    }
    if (k >= 3) {
      // the links of plane zc from the planes staged at iterations k-3 .. k-1
      const int zc = z0 + k - 3;
      const int sl[3] = {(k - 3) & 3, (k - 2) & 3, (k - 1) & 3};
      const bool in = colin;
      const unsigned cidx = in ? (unsigned)x + (unsigned)d.nx * ((unsigned)mm_ + (unsigned)d.nm * (unsigned)zc) : 0u;
      unsigned mk = 0;
      if (in) {
        const int dc = sd[sl[1]][lc];
        if (dc != 255) {
          const int2 oc = so[sl[1]][lc];
          unsigned cand = 0;  // thin links to cells with another owner pair
#pragma unroll
          for (int i = 1; i < L::Q; i++) {
            const int li = lc + L::ex[i] + LX * L::em[i];
            const int si = sl[1 + L::ez[i]];
            if (dc + (int)sd[si][li] + 1 <= zone_width) {
              const int2 on = so[si][li];
              if (on.x != oc.x || on.y != oc.y) cand |= 1u << i;
            }
          }
          if (cand) {
            const int2 rc = root_pair(oc);
#pragma unroll
            for (int i = 1; i < L::Q; i++) {
              if (!(cand & (1u << i))) continue;
              const int2 rn = root_pair(so[sl[1 + L::ez[i]]][lc + L::ex[i] + LX * L::em[i]]);
              if (rn.x != rc.x || rn.y != rc.y) mk |= 1u << i;
            }
          }
        }
        as_global(m.flag)[cidx] = mk ? 1 : 0;
        as_global(m.mask)[cidx] = mk;
      }
      const unsigned long long bal = __ballot(mk != 0);
      if (mm_ < d.nm && lane == 0) {
        const unsigned row = (unsigned)mm_ + (unsigned)d.nm * (unsigned)zc;
        as_global(m.fwords)[(unsigned)(x0 >> 6) + (unsigned)nxs * row] = bal;
      }
    }
    if (k <= L_ + 1) {
#pragma unroll
      for (int u = 0; u < 2; u++)
        if (sv[u]) {
          sd[k & 3][(int)threadIdx.x + u * BFS_NT] = dv[u];
          so[k & 3][(int)threadIdx.x + u * BFS_NT] = ov[u];
        }
    }
    __syncthreads();
  }
}

// ---- the flagged-cell list from the flag words, in cell order ----
static __global__ __launch_bounds__(FW_BLOCK) void k_flag_count(MAP_KERNEL_PARAMS) {
  MAP_MEMBER
  if (!map_due(m)) return;
  const long long nw = (long long)((m.d.nx + 63) >> 6) * m.d.nm * m.d.nz;
  const long long w = bid * (long long)FW_BLOCK + threadIdx.x;
  int v = w < nw ? __popcll(m.fwords[w]) : 0;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  __shared__ int s[FW_BLOCK / 64];
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int k = 0; k < FW_BLOCK / 64; k++) t += s[k];
    m.counts[bid] = t;
  }
}

static __global__ __launch_bounds__(FW_BLOCK) void k_flag_write(MAP_KERNEL_PARAMS) {
  MAP_MEMBER
  if (!map_due(m)) return;
  const int nxs = (m.d.nx + 63) >> 6;
  const long long nw = (long long)nxs * m.d.nm * m.d.nz;
  const long long w = bid * (long long)FW_BLOCK + threadIdx.x;
  const unsigned long long word = w < nw ? m.fwords[w] : 0ull;
  const int v = __popcll(word);
  int incl = v;  // inclusive scan within the wave
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int t = __shfl_up(incl, off, 64);
    if (lane >= off) incl += t;
  }
  __shared__ int s[FW_BLOCK / 64];
  if (lane == 63) s[wv] = incl;
  __syncthreads();
  int base = m.counts[bid] + incl - v;
  for (int k = 0; k < wv; k++) base += s[k];
  if (word) {
    const unsigned row = (unsigned)(w / nxs);
    const unsigned c0 = (unsigned)(w - (long long)row * nxs) * 64u + (unsigned)m.d.nx * row;
    unsigned long long b = word;
    while (b) {
      const int l = __builtin_ctzll(b);
      b &= b - 1ull;
      m.flist[base++] = (int)(c0 + (unsigned)l);
    }
  }
}


// Lattice coordinates of listed cell c (a division per cell; lists are sparse).
struct ListCell {
  int x, m, z;
  __device__ __forceinline__ ListCell(const MapDims& d, unsigned c) {
    const unsigned r = c / (unsigned)d.nx;
    x = (int)(c - r * (unsigned)d.nx);
    m = (int)(r % (unsigned)d.nm);
    z = (int)(r / (unsigned)d.nm);
  }
  __device__ __forceinline__ unsigned nb(const MapDims& d, int ex, int em, int ez) const {
    return (unsigned)wrap_any(x + ex, d.nx) +
           (unsigned)d.nx * ((unsigned)wrap_any(m + em, d.nm) + (unsigned)d.nm * (unsigned)wrap_any(z + ez, d.nz));
  }
};

// workgroups for a pass over a flagged-cell list of a lattice of N cells
__host__ inline int list_grid(long long N) {
  const long long g = N / 16384;
  return (int)(g < 1 ? 1 : (g > 1024 ? 1024 : g));
}

// wave-uniform loop over the entries of a list: f(index, active)
template <class F>
__device__ __forceinline__ void for_list(unsigned n, unsigned bid, unsigned nb, F&& f) {
  const unsigned lane = threadIdx.x & 63;
  for (unsigned base = bid * MAP_NT + (threadIdx.x & ~63u); base < n; base += nb * MAP_NT) f(base + lane, base + lane < n);
}

// Marks every cell whose density the rupture test reads: both ends and the
// outer neighbours of every barrier link.
template <class L>
__global__ __launch_bounds__(MAP_NT) void k_rho_marks(MAP_KERNEL_PARAMS) {
  MAP_MEMBER
  if (!map_due(m)) return;
  const MapDims d = m.d;
  for_list(m.ctl->n_flagged, bid, nbk, [&](unsigned idx, bool act) {
    if (!act) return;
    const unsigned c = (unsigned)m.flist[idx];
    const ListCell q(d, c);
    const unsigned mk = m.mask[c] & kLinkBits;
    atomicOr(&m.mask[c], kRhoBit);
    // the flag byte marks every cell whose mask word is not zero (the step
    // kernel reads the word only there); racing writers store the same 1
#pragma unroll
    for (int i = 1; i < L::Q; i++) {
      if (!(mk & (1u << i))) continue;
      const unsigned yp = q.nb(d, L::ex[i], L::em[i], L::ez[i]), ym = q.nb(d, -L::ex[i], -L::em[i], -L::ez[i]);
      atomicOr(&m.mask[yp], kRhoBit);
      atomicOr(&m.mask[ym], kRhoBit);
      m.flag[yp] = 1;
      m.flag[ym] = 1;
    }
  });
}

// the maps just built reflect the current aliases, and the next refresh can
// carry aliases from them
static __global__ void k_masks_done(MAP_KERNEL_PARAMS) {
  MAP_MEMBER
  if (map_due(m) && threadIdx.x == 0) {
    m.ctl->alias_dirty = 0;
    m.ctl->maps_seen = 1;
    m.ctl->maps_partial = m.zone_width - 1 > bfs_hot_layers(m.zone_width);
  }
}

// the deferred layers are done (or the maps came whole from the caller)
static __global__ void k_maps_whole(MAP_KERNEL_PARAMS) {
  MAP_MEMBER
  if (threadIdx.x == 0) m.ctl->maps_partial = 0;
}

// workgroups of lattice d for each decomposition
template <class L>
__host__ inline int map_share(int shape, const MapDims& d) {
  const long long N = d.N;
  const long long nseg = (long long)((d.nx + 63) / 64) * d.nm * d.nz;
  long long g = 1;
  switch (shape) {
    // grid-stride shapes stop at a few workgroups per CU: every workgroup of a
    // map kernel first looks up its lattice's arguments (dependent loads), so
    // many short workgroups spend their time starting
    case SH_CELLS: g = std::min<long long>((N + 1 + MAP_NT - 1) / MAP_NT, 4096); break;
    case SH_CCT: g = cc_tiles(d, CCTile<L>::TM, CCTile<L>::TZ); break;
    case SH_MASKT: g = cc_tiles(d, MaskTile<L>::TM, MaskTile<L>::TZ); break;
    case SH_MASKZ: g = cc_tiles(d, MZ_TM, MZ_LZ); break;
    case SH_RANK: g = (N + RANK_BLOCK - 1) / RANK_BLOCK; break;
    case SH_ONE: g = 1; break;
    // passes over per-bubble tables (as long as the bubble count, which only
    // the device knows): a few workgroups, grid-stride
    case SH_FEW: g = std::min<long long>((N + 1 + MAP_NT - 1) / MAP_NT, 32); break;
    case SH_LIST: g = list_grid(N); break;
    case SH_FW: g = (nseg + FW_BLOCK - 1) / FW_BLOCK; break;
    case SH_BFSB: g = bfs_blocks(d, BfsBlock<L>::CW, BfsBlock<L>::TM, BfsBlock<L>::TZ); break;
  }
  return (int)std::max<long long>(g, 1);
}

// After a step whose ruptures united bubbles: drop the links whose two ends
// now share an alias-root pair.  A union never creates a barrier, so only
// listed cells need checking.  Returns at once when nothing was united.
struct PruneArgs {
  const Ctl* ctl;
  MapDims d;
  const int2* own;
  const int* alias;
  uint8_t* flag;
  uint32_t* mask;
  const int* flist;
};

template <class L>
__device__ __forceinline__ void mask_prune(const PruneArgs& p, unsigned bid, unsigned nb) {
  if (p.ctl->stopped || !p.ctl->alias_dirty) return;
  for_list(p.ctl->n_flagged, bid, nb, [&](unsigned idx, bool act) {
    if (!act) return;
    const unsigned c = (unsigned)p.flist[idx];
    const unsigned word = p.mask[c];
    const unsigned mk = word & kLinkBits;
    if (!mk) return;
    const ListCell q(p.d, c);
    const int2 rp = root_pair(p.alias, p.own[c]);
    unsigned keep = 0;
#pragma unroll
    for (int i = 1; i < L::Q; i++) {
      if (!(mk & (1u << i))) continue;
      const int2 rq = root_pair(p.alias, p.own[q.nb(p.d, L::ex[i], L::em[i], L::ez[i])]);
      if (rq.x != rp.x || rq.y != rp.y) keep |= 1u << i;
    }
    if (keep != mk) {
      p.mask[c] = keep | (word & kRhoBit);  // a listed cell keeps its density mark, and its flag byte
    }
  });
}

template <class L>
__global__ __launch_bounds__(MAP_NT) void k_mask_prune(PruneArgs p) {
  mask_prune<L>(p, blockIdx.x, gridDim.x);
}

// The pruning launch that also closes the step (one lattice; the finisher
// of step.hpp with MAP_NT threads).  A step without unions (alias_dirty 0,
// the common case) prunes nothing, so workgroup 0 finishes the step at once.
// After unions every workgroup prunes its share and the last to arrive (an
// arrival counter in the run control, reset by that workgroup) finishes the
// step; the device-scope fences and atomics are paid only on those steps.
// Every workgroup reads alias_dirty before any finisher can clear it: in the
// first case it is 0 throughout, in the second the finisher runs after all
// workgroups have arrived.
template <class L>
__global__ __launch_bounds__(MAP_NT) void k_prune_finish(PruneArgs p, StepArgs a, int nblk) {
  __shared__ double red[MAP_NT / 64][4];
  __shared__ int last;
  Ctl* ctl = a.ctl;
  const bool dirty = ctl->alias_dirty && !ctl->stopped;  // workgroup-uniform
  if (!dirty) {
    if (blockIdx.x == 0) step_finish<MAP_NT>(a, nblk, red);
    return;
  }
  mask_prune<L>(p, blockIdx.x, gridDim.x);
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    last = atomicAdd(&ctl->done, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (last) {
    __threadfence();
    step_finish<MAP_NT>(a, nblk, red);
    if (threadIdx.x == 0) ctl->done = 0;
  }
}

// batched form of k_prune_finish: workgroups [ffirst[j], ffirst[j+1]) prune
// film member j (member index idx[j]) and close its step as k_prune_finish
// does; workgroup ffirst[nf] + i closes the step of member idx[nf + i], one
// without a film.  tab / first: the batched step launch's members and
// workgroup ranges (a member's partials count).
template <class L>
__global__ __launch_bounds__(MAP_NT) void k_prune_finish_batch(const PruneArgs* __restrict__ ptab,
                                                               const int* __restrict__ ffirst, int nf,
                                                               const StepArgs* __restrict__ tab,
                                                               const int* __restrict__ first,
                                                               const int* __restrict__ idx) {
  __shared__ double red[MAP_NT / 64][4];
  __shared__ int last;
  const int fblk = nf ? ffirst[nf] : 0;
  if ((int)blockIdx.x >= fblk) {
    const int k = idx[nf + (int)blockIdx.x - fblk];
    step_finish<MAP_NT>(tab[k], first[k + 1] - first[k], red);
    return;
  }
  const int j = batch_member(ffirst, nf, blockIdx.x);
  const int k = idx[j];
  const StepArgs& a = tab[k];  // read in place: a local copy would live in scratch
  const int nblk = first[k + 1] - first[k];
  const unsigned bid = blockIdx.x - (unsigned)ffirst[j], nb = (unsigned)(ffirst[j + 1] - ffirst[j]);
  Ctl* ctl = a.ctl;
  const bool dirty = ctl->alias_dirty && !ctl->stopped;  // workgroup-uniform
  if (!dirty) {
    if (bid == 0) step_finish<MAP_NT>(a, nblk, red);
    return;
  }
  const PruneArgs p = ptab[j];
  mask_prune<L>(p, bid, nb);
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    last = atomicAdd(&ctl->done, 1u) == nb - 1;
  }
  __syncthreads();
  if (last) {
    __threadfence();
    step_finish<MAP_NT>(a, nblk, red);
    if (threadIdx.x == 0) ctl->done = 0;
  }
}

}  // namespace flb
