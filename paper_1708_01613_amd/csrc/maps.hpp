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
//  masks     : link i of cell c is a candidate barrier iff both ends are owned,
//              their alias-root pairs differ and dist(c) + dist(c+e_i) + 1 <=
//              zone_width.
#pragma once
#include "step.hpp"

namespace flb {

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

__host__ inline int map_grid(const MapDims& d) {
  const long long nseg = (long long)((d.nx + 63) / 64) * d.nm * d.nz;
  const long long g = (nseg + MAP_WAVES - 1) / MAP_WAVES;
  return (int)(g < 1 ? 1 : (g > 65536 ? 65536 : g));
}

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

// parent[c] = c for gas cells (double-precision density of the stored state
// below rho_th), -1 otherwise
template <class L, class S>
__global__ __launch_bounds__(MAP_NT) void k_gas_init(const void* b0, const void* b1, const Ctl* ctl, Geo geo,
                                                     MapDims d, double rho_th, int* par) {
  if (ctl->stopped) return;
  const void* src = (ctl->steps & 1) ? b1 : b0;
  for_cells<false>(d, [&](const SegCell& q) {
    typename S::ct f[L::Q];
    load_pulled<L, S>(src, geo, q.x, q.m, q.z, f);
    double r = 0.0;
#pragma unroll
    for (int i = 0; i < L::Q; i++) r += (double)f[i];
    par[q.c] = r < rho_th ? (int)q.c : -1;
  });
}

// same from a host-provided density field
static __global__ void k_gas_from_field(const double* rho, MapDims d, double rho_th, int* par) {
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < d.N;
       c += (long long)gridDim.x * blockDim.x)
    par[c] = rho[c] < rho_th ? (int)c : -1;
}

// ---- connected components in two phases ----
// Phase 1 (k_cc_local): a workgroup labels the gas components of one tile of
// CC_TX x CC_TM x CC_TZ cells with a union-find in LDS over the links that
// stay inside the tile, then points every gas cell at its tile-local root
// (the local order is the global order, so that root is the component's
// smallest cell index within the tile).  Phase 2 (k_cc_cross): the links that
// leave a tile (including the periodic wrap) unite the local roots in the
// global union-find; a wavefront first merges duplicate root pairs, which are
// the common case, so few global atomics remain.
constexpr int CC_NT = 256;
constexpr int CC_CELLS = 2048;
template <class L>
struct CCTile {
  static constexpr int TX = 64;
  static constexpr int TM = L::HAS_M ? 8 : 1;
  static constexpr int TZ = CC_CELLS / (TX * TM);
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

template <class L>
__global__ __launch_bounds__(CC_NT) void k_cc_local(const Ctl* ctl, MapDims d, int* par) {
  if (ctl->stopped) return;
  using TT = CCTile<L>;
  __shared__ int lp[CC_CELLS];
  const int ntx = (d.nx + 63) / 64, ntm = (d.nm + TT::TM - 1) / TT::TM;
  const int b = blockIdx.x;
  const int tx = b % ntx, tm = (b / ntx) % ntm, tz = b / (ntx * ntm);
  const int x0 = tx * 64, m0 = tm * TT::TM, z0 = tz * TT::TZ;
  constexpr int PER = CC_CELLS / CC_NT;
  auto gcell = [&](int l, int& x, int& m, int& z) -> bool {
    x = x0 + (l & 63);
    m = m0 + (l >> 6) % TT::TM;
    z = z0 + (l >> 6) / TT::TM;
    return x < d.nx && m < d.nm && z < d.nz;
  };
#pragma unroll
  for (int k = 0; k < PER; k++) {
    const int l = threadIdx.x + k * CC_NT;
    int x, m, z;
    bool gas = false;
    if (gcell(l, x, m, z)) gas = par[x + (unsigned)d.nx * (m + (unsigned)d.nm * z)] >= 0;
    lp[l] = gas ? l : -1;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < PER; k++) {
    const int l = threadIdx.x + k * CC_NT;
    if (lp[l] < 0) continue;
    const int lx = l & 63, lm = (l >> 6) % TT::TM, lz = (l >> 6) / TT::TM;
#pragma unroll
    for (int i = 1; i < L::Q; i += 2) {  // one direction of each opposite pair
      const int nx_ = lx + L::ex[i], nm_ = lm + L::em[i], nz_ = lz + L::ez[i];
      if (nx_ < 0 || nx_ >= 64 || nm_ < 0 || nm_ >= TT::TM || nz_ < 0 || nz_ >= TT::TZ) continue;
      if (x0 + nx_ >= d.nx || m0 + nm_ >= d.nm || z0 + nz_ >= d.nz) continue;
      const int ln = nx_ + 64 * (nm_ + TT::TM * nz_);
      if (lp[ln] >= 0) lds_unite(lp, l, ln);
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < PER; k++) {
    const int l = threadIdx.x + k * CC_NT;
    if (lp[l] < 0) continue;
    const int r = lds_find(lp, l);
    int x, m, z, rx, rm, rz;
    gcell(l, x, m, z);
    gcell(r, rx, rm, rz);
    par[x + (unsigned)d.nx * (m + (unsigned)d.nm * z)] = (int)(rx + (unsigned)d.nx * (rm + (unsigned)d.nm * rz));
  }
}

template <class L>
__global__ __launch_bounds__(MAP_NT) void k_cc_cross(const Ctl* ctl, MapDims d, int* par) {
  if (ctl->stopped) return;
  using TT = CCTile<L>;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nxs = (d.nx + 63) >> 6;
  const unsigned nseg = (unsigned)nxs * (unsigned)d.nm * (unsigned)d.nz;
  // wave-uniform loop over segments: every lane takes part in the merging
  for (unsigned s = blockIdx.x * MAP_WAVES + wv; s < nseg; s += gridDim.x * MAP_WAVES) {
    const unsigned row = s / (unsigned)nxs;
    const int x = (int)(s - row * (unsigned)nxs) * 64 + lane;
    const int m = (int)(row % (unsigned)d.nm), z = (int)(row / (unsigned)d.nm);
    const bool in = x < d.nx;
    const unsigned c = (unsigned)min(x, d.nx - 1) + (unsigned)d.nx * row;
    const int pc = in ? par[c] : -1;
#pragma unroll
    for (int i = 1; i < L::Q; i += 2) {
      const int xu = x + L::ex[i], mu = m + L::em[i], zu = z + L::ez[i];
      const bool local = xu >= 0 && xu < d.nx && (xu >> 6) == (x >> 6) && mu >= 0 && mu < d.nm &&
                         mu / TT::TM == m / TT::TM && zu >= 0 && zu < d.nz && zu / TT::TZ == z / TT::TZ;
      int ra = -1, rb = -1;
      if (pc >= 0 && !local) {
        const unsigned y = (unsigned)wrap_any(xu, d.nx) +
                           (unsigned)d.nx * ((unsigned)wrap_any(mu, d.nm) + (unsigned)d.nm * wrap_any(zu, d.nz));
        const int py = __atomic_load_n(&par[y], __ATOMIC_RELAXED);
        if (py >= 0) {
          ra = __atomic_load_n(&par[c], __ATOMIC_RELAXED);
          rb = py;
        }
      }
      bool pend = ra >= 0 && ra != rb;
      unsigned long long mk = __ballot(pend);
      while (mk) {
        const int ld = first_lane(mk);
        const int a0 = __shfl(ra, ld, 64), b0 = __shfl(rb, ld, 64);
        if (lane == ld) uf_unite(par, a0, b0);
        if (pend && ra == a0 && rb == b0) pend = false;
        mk = __ballot(pend);
      }
    }
  }
}

static __global__ void k_cc_compress(const Ctl* ctl, MapDims d, int* par) {
  if (ctl->stopped) return;
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < d.N;
       c += (long long)gridDim.x * blockDim.x) {
    if (par[c] < 0) continue;
    par[c] = uf_find_live(par, (int)c);
  }
}

// ---- canonical ranks: count roots per block, scan, write labels ----
constexpr int RANK_BLOCK = 1024;

static __global__ __launch_bounds__(RANK_BLOCK) void k_count_roots(const Ctl* ctl, MapDims d, const int* par,
                                                           int* counts) {
  if (ctl->stopped) return;
  const long long c = blockIdx.x * (long long)RANK_BLOCK + threadIdx.x;
  const int is_root = (c < d.N && par[c] == (int)c) ? 1 : 0;
  __shared__ int s[RANK_BLOCK / 64];
  const unsigned long long bal = __ballot(is_root);
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = __popcll(bal);
  __syncthreads();
  if (threadIdx.x == 0) {
    int t = 0;
    for (int w = 0; w < RANK_BLOCK / 64; w++) t += s[w];
    counts[blockIdx.x] = t;
  }
}

// single workgroup: exclusive scan of the per-block counts, total to *total
static __global__ __launch_bounds__(1024) void k_scan_counts(const Ctl* ctl, int* counts, int nblocks, int* total) {
  if (ctl->stopped) return;
  __shared__ int s_carry;
  __shared__ int s_w[16];
  if (threadIdx.x == 0) s_carry = 0;
  __syncthreads();
  for (int base = 0; base < nblocks; base += 1024) {
    const int i = base + threadIdx.x;
    const int v = i < nblocks ? counts[i] : 0;
    // inclusive scan within the wave
    int incl = v;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int t = __shfl_up(incl, off, 64);
      if (lane >= off) incl += t;
    }
    if (lane == 63) s_w[w] = incl;
    __syncthreads();
    int wbase = 0;
    for (int k = 0; k < w; k++) wbase += s_w[k];
    const int carry = s_carry;
    if (i < nblocks) counts[i] = carry + wbase + incl - v;
    __syncthreads();
    if (threadIdx.x == 1023) s_carry = carry + wbase + incl;
    __syncthreads();
  }
  if (threadIdx.x == 0) *total = s_carry;
}

// rank[root] = 1-based label of the component rooted there
static __global__ __launch_bounds__(RANK_BLOCK) void k_write_rank(const Ctl* ctl, MapDims d, const int* par,
                                                          const int* offs, int* rank) {
  if (ctl->stopped) return;
  const long long c = blockIdx.x * (long long)RANK_BLOCK + threadIdx.x;
  const int is_root = (c < d.N && par[c] == (int)c) ? 1 : 0;
  __shared__ int s[RANK_BLOCK / 64];
  const unsigned long long bal = __ballot(is_root);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) s[w] = __popcll(bal);
  __syncthreads();
  if (is_root) {
    int before = offs[blockIdx.x];
    for (int k = 0; k < w; k++) before += s[k];
    before += __popcll(bal & ((1ull << lane) - 1ull));
    rank[c] = before + 1;
  }
}

static __global__ void k_write_labels(const Ctl* ctl, MapDims d, const int* par, const int* rank, int* label) {
  if (ctl->stopped) return;
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < d.N;
       c += (long long)gridDim.x * blockDim.x) {
    const int p = par[c];
    label[c] = p < 0 ? 0 : rank[p];
  }
}

// ---- owner / dist ----
// The layered BFS keeps two bitsets with one 64-bit word per row segment
// (word s covers x = 64 xs .. 64 xs + 63 of row (m, z), s = xs + nxs row):
// the frontier of the previous layer and the visited set.  A wavefront handles
// one segment; the neighbour words it needs are wave-uniform loads, so finding
// the cells a layer reaches takes bit operations instead of neighbour gathers.
// Only newly reached cells read the owners of their frontier neighbours.
static __global__ __launch_bounds__(MAP_NT) void k_owner_init(const Ctl* ctl, MapDims d, const int* label, int2* own,
                                                       uint8_t* dist, unsigned long long* front,
                                                       unsigned long long* vis) {
  if (ctl->stopped) return;
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int nxs = (d.nx + 63) >> 6;
  const unsigned nseg = (unsigned)nxs * (unsigned)d.nm * (unsigned)d.nz;
  for (unsigned s = blockIdx.x * MAP_WAVES + wv; s < nseg; s += gridDim.x * MAP_WAVES) {
    const unsigned row = s / (unsigned)nxs;
    const int x = (int)(s - row * (unsigned)nxs) * 64 + lane;
    const bool in = x < d.nx;
    const unsigned c = (unsigned)x + (unsigned)d.nx * row;
    const int l = in ? label[c] : 0;
    if (in) {
      own[c] = make_int2(l, l);
      dist[c] = l > 0 ? 0 : 255;
    }
    const unsigned long long g = __ballot(l > 0);
    if (lane == 0) {
      front[s] = g;
      vis[s] = g;
    }
  }
}

// One BFS layer, one 64-bit word (64 x-cells of a row) per lane: the words
// reached this layer are the unvisited bits of the frontier dilated by the
// lattice links, formed with whole-word shifts of the neighbour rows' words
// (x - 1 and x + 1 bring in one bit from the adjacent word, periodic across
// the row end).  Only the newly reached cells then read the owners of their
// frontier neighbours.  Word bits past the end of a row are always zero.
struct WordRow {
  const unsigned long long* __restrict__ b;
  int nxs, last_valid;  // words per row; valid bits of a row's last word
  // bits of the cells x + ex for every x of word xs of the row at rowbase
  __device__ __forceinline__ unsigned long long shifted(unsigned rowbase, int xs, int ex) const {
    const unsigned long long wc = b[rowbase + xs];
    if (ex == 0) return wc;
    if (ex > 0) {
      const unsigned long long wr = b[rowbase + (xs + 1 < nxs ? xs + 1 : 0)];
      const int top = xs == nxs - 1 ? last_valid - 1 : 63;
      return (wc >> 1) | ((wr & 1ull) << top);
    }
    const unsigned long long in = xs > 0 ? b[rowbase + xs - 1] >> 63
                                         : (b[rowbase + nxs - 1] >> (last_valid - 1)) & 1ull;
    return (wc << 1) | in;
  }
};

template <class L>
__global__ __launch_bounds__(MAP_NT) void k_owner_layer(const Ctl* ctl, MapDims d, int layer,
                                                        const unsigned long long* __restrict__ fin,
                                                        unsigned long long* __restrict__ fout,
                                                        unsigned long long* __restrict__ vis, int2* own,
                                                        uint8_t* dist) {
  if (ctl->stopped) return;
  const int nxs = (d.nx + 63) >> 6;
  const unsigned nw = (unsigned)nxs * (unsigned)d.nm * (unsigned)d.nz;
  const int last_valid = d.nx - 64 * (nxs - 1);
  const WordRow fr{fin, nxs, last_valid};
  for (unsigned s = blockIdx.x * MAP_NT + threadIdx.x; s < nw; s += gridDim.x * MAP_NT) {
    const unsigned row = s / (unsigned)nxs;
    const int xs = (int)(s - row * (unsigned)nxs);
    const unsigned long long valid = (xs == nxs - 1 && last_valid < 64) ? (1ull << last_valid) - 1ull : ~0ull;
    const unsigned long long v = vis[s];
    if ((v & valid) == valid) {
      fout[s] = 0ull;
      continue;
    }
    const int m = (int)(row % (unsigned)d.nm), z = (int)(row / (unsigned)d.nm);
    const int mm[3] = {m == 0 ? d.nm - 1 : m - 1, m, m == d.nm - 1 ? 0 : m + 1};
    const int zz[3] = {z == 0 ? d.nz - 1 : z - 1, z, z == d.nz - 1 ? 0 : z + 1};
    unsigned long long sh[L::Q];  // sh[i] bit l: the cell x + e_i of x = 64 xs + l is on the frontier
    unsigned long long reach = 0ull;
#pragma unroll
    for (int i = 1; i < L::Q; i++) {
      const unsigned rb = (unsigned)nxs * ((unsigned)mm[1 + L::em[i]] + (unsigned)d.nm * (unsigned)zz[1 + L::ez[i]]);
      sh[i] = fr.shifted(rb, xs, L::ex[i]);
      reach |= sh[i];
    }
    unsigned long long nwb = reach & ~v & valid;
    fout[s] = nwb;
    vis[s] = v | nwb;
    const unsigned cbase = (unsigned)xs * 64u + (unsigned)d.nx * row;
    while (nwb) {
      const int l = __builtin_ctzll(nwb);
      nwb &= nwb - 1ull;
      const int x = xs * 64 + l;
      const int xw[3] = {x == 0 ? d.nx - 1 : x - 1, x, x == d.nx - 1 ? 0 : x + 1};
      int lo = 0, hi = 0;
#pragma unroll
      for (int i = 1; i < L::Q; i++) {
        if (!((sh[i] >> l) & 1ull)) continue;
        const unsigned y = (unsigned)xw[1 + L::ex[i]] +
                           (unsigned)d.nx * ((unsigned)mm[1 + L::em[i]] + (unsigned)d.nm * (unsigned)zz[1 + L::ez[i]]);
        const int2 o = own[y];
        lo = (lo == 0 || o.x < lo) ? o.x : lo;
        hi = o.y > hi ? o.y : hi;
      }
      own[cbase + (unsigned)l] = make_int2(lo, hi);
      dist[cbase + (unsigned)l] = (uint8_t)layer;
    }
  }
}

// keep the previous labels and aliases for the carry (a device copy, so that
// a refresh queued after a stop leaves everything untouched)
static __global__ void k_copy_int(const Ctl* ctl, const int* src, int* dst, long long n) {
  if (ctl->stopped) return;
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n;
       c += (long long)gridDim.x * blockDim.x)
    dst[c] = src[c];
}

// ---- alias carry across a refresh ----
static __global__ void k_alias_reset(const Ctl* ctl, int* alias, int* rep, int nb_cap) {
  if (ctl->stopped) return;
  const int nb = ctl->n_bubbles;
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b <= nb_cap; b += gridDim.x * blockDim.x) {
    if (b <= nb) alias[b] = b;
    rep[b] = 0x7fffffff;
  }
}

// Both carry passes run over whole wavefronts (the loop bound is uniform per
// wavefront) and merge the many lanes that carry the same (old class, new
// label) pair before touching global memory.
static __global__ __launch_bounds__(MAP_NT) void k_alias_carry1(const Ctl* ctl, MapDims d, const int* label,
                                                         const int* label_old, const int* alias_old, int* rep) {
  if (ctl->stopped) return;
  const int lane = threadIdx.x & 63;
  const long long stride = (long long)gridDim.x * MAP_NT;
  for (long long base = blockIdx.x * (long long)MAP_NT + (threadIdx.x & ~63); base < d.N; base += stride) {
    const long long c = base + lane;
    int b = 0, a = 0;
    if (c < d.N) {
      b = label[c];
      a = label_old[c];
    }
    bool pend = b > 0 && a > 0;
    const int r = pend ? uf_root(alias_old, a) : 0;
    unsigned long long mk = __ballot(pend);
    while (mk) {
      const int ld = first_lane(mk);
      const int r0 = __shfl(r, ld, 64);
      const bool mine = pend && r == r0;
      const int bmin = wave_min_i32(mine ? b : 0x7fffffff);
      if (lane == ld && __atomic_load_n(&rep[r0], __ATOMIC_RELAXED) > bmin) atomicMin(&rep[r0], bmin);
      if (mine) pend = false;
      mk = __ballot(pend);
    }
  }
}

static __global__ __launch_bounds__(MAP_NT) void k_alias_carry2(const Ctl* ctl, MapDims d, const int* label,
                                                         const int* label_old, const int* alias_old,
                                                         const int* rep, int* alias) {
  if (ctl->stopped) return;
  const int lane = threadIdx.x & 63;
  const long long stride = (long long)gridDim.x * MAP_NT;
  for (long long base = blockIdx.x * (long long)MAP_NT + (threadIdx.x & ~63); base < d.N; base += stride) {
    const long long c = base + lane;
    int b = 0, a = 0;
    if (c < d.N) {
      b = label[c];
      a = label_old[c];
    }
    const int r = (b > 0 && a > 0) ? rep[uf_root(alias_old, a)] : 0;
    bool pend = b > 0 && a > 0 && r != b;
    unsigned long long mk = __ballot(pend);
    while (mk) {
      const int ld = first_lane(mk);
      const int b0 = __shfl(b, ld, 64), r0 = __shfl(r, ld, 64);
      if (lane == ld) uf_unite(alias, b0, r0);
      if (pend && b == b0 && r == r0) pend = false;
      mk = __ballot(pend);
    }
  }
}

static __global__ void k_alias_compress(const Ctl* ctl, int* alias) {
  if (ctl->stopped) return;
  const int nb = ctl->n_bubbles;
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b <= nb; b += gridDim.x * blockDim.x)
    alias[b] = uf_find_live(alias, b);
}

// ---- barrier candidate masks ----
// Barrier masks from the owner maps, and the list of cells that have barrier
// links (appended a wavefront at a time; its order is irrelevant to the
// results).  ctl->n_flagged must be zero before the launch.
template <class L>
__global__ __launch_bounds__(MAP_NT) void k_masks(Ctl* ctl, MapDims d, int zone_width, const int2* own,
                                                  const uint8_t* dist, const int* alias, uint8_t* flag,
                                                  uint32_t* mask, int* flist) {
  if (ctl->stopped) return;
  const int lane = threadIdx.x & 63;
  for_cells<true>(d, [&](const SegCell& q) {
    const int2 o = own[q.c];
    unsigned mk = 0;
    if (o.x > 0) {
      int2 rp = make_int2(0, 0);
      bool have_rp = false;
      const int dc = dist[q.c];
#pragma unroll
      for (int i = 1; i < L::Q; i++) {
        const unsigned y = q.nb(L::ex[i], L::em[i], L::ez[i]);
        if (dc + (int)dist[y] + 1 > zone_width) continue;  // also rejects unowned ends (dist 255)
        const int2 oy = own[y];
        if (oy.x == o.x && oy.y == o.y) continue;  // same owner pair, same root pair
        if (!have_rp) {
          rp = root_pair(alias, o);
          have_rp = true;
        }
        const int2 rq = root_pair(alias, oy);
        if (rq.x != rp.x || rq.y != rp.y) mk |= 1u << i;
      }
    }
    flag[q.c] = mk ? 1 : 0;
    mask[q.c] = mk;
    const unsigned long long bal = __ballot(mk != 0);
    if (bal) {
      const int ld = first_lane(bal);
      unsigned base = 0;
      if (lane == ld) base = atomicAdd(&ctl->n_flagged, (unsigned)__popcll(bal));
      base = __shfl(base, ld, 64);
      if (mk) flist[base + (unsigned)__popcll(bal & ((1ull << lane) - 1ull))] = (int)q.c;
    }
  });
}

// an empty flagged-cell list before k_masks fills it
static __global__ void k_flag_list_reset(Ctl* ctl) {
  if (!ctl->stopped && threadIdx.x == 0) ctl->n_flagged = 0;
}

// the masks just built reflect the current aliases
static __global__ void k_masks_done(Ctl* ctl) {
  if (!ctl->stopped && threadIdx.x == 0) ctl->alias_dirty = 0;
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
__global__ __launch_bounds__(MAP_NT) void k_rho_marks(const Ctl* ctl, MapDims d, const int* flist,
                                                      uint32_t* mask) {
  if (ctl->stopped) return;
  const unsigned n = ctl->n_flagged;
  for_list(n, blockIdx.x, gridDim.x, [&](unsigned idx, bool act) {
    if (!act) return;
    const unsigned c = (unsigned)flist[idx];
    const ListCell q(d, c);
    const unsigned mk = mask[c] & kLinkBits;
    atomicOr(&mask[c], kRhoBit);
#pragma unroll
    for (int i = 1; i < L::Q; i++) {
      if (!(mk & (1u << i))) continue;
      atomicOr(&mask[q.nb(d, L::ex[i], L::em[i], L::ez[i])], kRhoBit);
      atomicOr(&mask[q.nb(d, -L::ex[i], -L::em[i], -L::ez[i])], kRhoBit);
    }
  });
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
      p.mask[c] = keep | (word & kRhoBit);
      p.flag[c] = keep ? 1 : 0;
    }
  });
}

template <class L>
__global__ __launch_bounds__(MAP_NT) void k_mask_prune(PruneArgs p) {
  mask_prune<L>(p, blockIdx.x, gridDim.x);
}

// batched: workgroups [first[k], first[k+1]) prune member k
template <class L>
__global__ __launch_bounds__(MAP_NT) void k_mask_prune_batch(const PruneArgs* __restrict__ tab,
                                                             const int* __restrict__ first, int nmem) {
  const int k = batch_member(first, nmem, blockIdx.x);
  const PruneArgs p = tab[k];
  mask_prune<L>(p, blockIdx.x - first[k], first[k + 1] - first[k]);
}

}  // namespace flb
