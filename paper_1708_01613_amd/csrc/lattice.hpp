// lattice.hpp -- velocity sets, weights and storage formats of the GPU path.
//
// Kernels work in "kernel coordinates" (x, m, z): x is the contiguous axis, z
// the axis a workgroup marches along, m the second tile axis.  D3Q19 maps
// (x, y, z) -> (x, m, z).  D2Q9 maps its (x, y) -> (x, z) with an m axis of
// extent 1, so one kernel template serves both lattices.
//
// D2Q9 weights are the paper's (Sec. 2.1.1: rest 4/9, axes 1/9, diagonals
// 1/36); D3Q19 is the textbook lattice (rest 1/3, axes 1/18, face diagonals
// 1/36).  Directions come in opposite pairs (2p-1, 2p), p = 1..(Q-1)/2, so the
// neighbour-sum force can be accumulated as w_i e_i (psi(x+e_i) - psi(x-e_i)).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace flb {

struct D2Q9K {
  static constexpr int Q = 9;
  static constexpr int D = 2;
  static constexpr bool HAS_M = false;
  // kernel coordinates: lattice (ex, ey) -> (ex, 0, ey)
  static constexpr int ex[9] = {0, 1, -1, 0, 0, 1, -1, 1, -1};
  static constexpr int em[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  static constexpr int ez[9] = {0, 0, 0, 1, -1, 1, -1, -1, 1};
  static constexpr double w[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                                  1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
  // lattice-coordinate component k (0 = x, 1 = y) of direction i
  __host__ __device__ static constexpr int comp(int i, int k) { return k == 0 ? ex[i] : ez[i]; }
};

struct D3Q19K {
  static constexpr int Q = 19;
  static constexpr int D = 3;
  static constexpr bool HAS_M = true;
  static constexpr int ex[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
  static constexpr int em[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
  static constexpr int ez[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
  static constexpr double w[19] = {1.0 / 3,  1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
                                   1.0 / 18, 1.0 / 18, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                                   1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
                                   1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
  __host__ __device__ static constexpr int comp(int i, int k) {
    return k == 0 ? ex[i] : (k == 1 ? em[i] : ez[i]);
  }
};

// Population layout: blocks of 64 consecutive x-cells (one wavefront).  A
// block holds the Q populations of its cells one after the other (64 values
// each), so a wavefront's access to one population is one contiguous 64-value
// run and a block's Q runs share a few DRAM pages.  Block index
// b = x / 64 + nxb * (m + nm * z) in kernel coordinates (nxb = ceil(nx / 64));
// population i of lane xl = x % 64 sits at byte
//   b * block_bytes + pofs(i) + xl * esz(i).
constexpr int kBlk = 64;

struct Geo {
  int nx, nm, nz;  // kernel-coordinate extents
  int nxb;         // blocks per row, ceil(nx / 64)
  unsigned block_bytes;
  float href;      // FP16-shifted storage: population i is stored as FP16 of f_i - w_i href
};

// Storage formats: `ct` is the compute type; esz / pofs give the element
// size and the byte offset of population i's run inside a block; dec / enc
// convert between the stored element and the compute type.
struct SF64 {
  using ct = double;
  static constexpr bool HALF = false;
  __host__ __device__ static constexpr unsigned esz(int) { return 8; }
  __host__ __device__ static constexpr unsigned pofs(int i) { return 512u * i; }
};
struct SF32 {
  using ct = float;
  static constexpr bool HALF = false;
  __host__ __device__ static constexpr unsigned esz(int) { return 4; }
  __host__ __device__ static constexpr unsigned pofs(int i) { return 256u * i; }
};
// FP16 of the shifted population f_i - w_i href for the moving directions
// (href = 1: f_i - w_i), and the rest population (the largest, never
// streamed) in FP32; compute in FP32.
struct SF16S {
  using ct = float;
  static constexpr bool HALF = true;
  __host__ __device__ static constexpr unsigned esz(int i) { return i == 0 ? 4 : 2; }
  __host__ __device__ static constexpr unsigned pofs(int i) { return i == 0 ? 0u : 256u + 128u * (i - 1); }
};

// FP16-shifted element <-> compute value (wh = w_i href).  The sum and the
// difference round on their own (never fused with the product that formed
// wh), so every kernel decodes and encodes a population to the same bits.
__device__ __forceinline__ float h16_dec(unsigned short bits, float wh) {
#pragma clang fp contract(off)
  return (float)__builtin_bit_cast(_Float16, bits) + wh;
}
__device__ __forceinline__ unsigned short h16_enc(float v, float wh) {
#pragma clang fp contract(off)
  return __builtin_bit_cast(unsigned short, (_Float16)(v - wh));
}

template <class S>
__host__ __device__ constexpr unsigned block_bytes(int Q) {
  return S::pofs(Q - 1) + kBlk * S::esz(Q - 1);
}

// byte offset of a cell's block and of its lane inside a run
__host__ __device__ inline unsigned long long block_of(const Geo& g, int x, int m, int z) {
  return (unsigned long long)((x >> 6) + (long long)g.nxb * (m + (long long)g.nm * z)) * g.block_bytes;
}

// generic (global-pointer) access, used outside the step kernel
template <class L, class S>
__device__ inline typename S::ct pop_ld(const void* base, const Geo& g, int i, int x, int m, int z) {
  const char* p = (const char*)base + block_of(g, x, m, z) + S::pofs(i) + (unsigned)(x & 63) * S::esz(i);
  if constexpr (sizeof(typename S::ct) == 8) return *(const double*)p;
  else if (S::HALF && i > 0) return h16_dec(*(const unsigned short*)p, (float)L::w[i] * g.href);
  else return *(const float*)p;
}
template <class L, class S>
__device__ inline void pop_st(void* base, const Geo& g, int i, int x, int m, int z, typename S::ct v) {
  char* p = (char*)base + block_of(g, x, m, z) + S::pofs(i) + (unsigned)(x & 63) * S::esz(i);
  if constexpr (sizeof(typename S::ct) == 8) *(double*)p = v;
  else if (S::HALF && i > 0) *(unsigned short*)p = h16_enc(v, (float)L::w[i] * g.href);
  else *(float*)p = v;
}

// Barrier mask word of a cell: bit i (1 <= i < Q) marks an active barrier link
// in direction i; kRhoBit marks a cell whose density the rupture test reads
// (an end or an outer neighbour of a barrier link), so the step kernel stores
// its density only there.
constexpr uint32_t kRhoBit = 1u << 31;
constexpr uint32_t kLinkBits = ~kRhoBit;

// Device-side run control shared by every launch of one lattice.
struct Ctl {
  unsigned done;        // workgroups finished in the current launch
  int stopped;          // 1 after a rupture with on_rupture == 1
  long long steps;      // steps completed (selects the A/B buffer)
  unsigned ev_count;    // rupture-log records written so far (<= capacity)
  int ev_full;          // 1 once a record found the log full
  long long n_ruptures; // successful barrier removals (unions of two classes)
  int failed;           // 1 once the FP64 mass reduction saw a non-finite value
  int n_bubbles;        // labels in the current film maps
  int alias_dirty;      // 1 if ruptures of this step united bubbles (masks need pruning)
  int step_events;      // 1 if the rupture test of this step found a link
  unsigned n_flagged;   // cells with barrier links at the last refresh (list length)
  int maps_seen;        // 1 once a refresh has built maps (the next one carries aliases)
  int nb_old;           // labels of the previous refresh, during a refresh
  int maps_partial;     // 1 while owner/dist stop at the layers the masks need
  long long rho_step;   // the step whose entering densities the rho array holds for every cell (-1: none)
  long long n_src;      // domain gas points of the gas-release source (cells of the nuclei)
  double mass, mom[3];  // FP64 totals of the state entering the last step
};

}  // namespace flb
