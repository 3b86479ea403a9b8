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

__device__ __forceinline__ int uf_find_live(int* par, int a) {
  int p = __atomic_load_n(&par[a], __ATOMIC_RELAXED);
  while (p != a) {
    a = p;
    p = __atomic_load_n(&par[a], __ATOMIC_RELAXED);
  }
  return a;
}

// unite the sets of a and b, hooking the larger root under the smaller one
__device__ void uf_unite(int* par, int a, int b) {
  while (true) {
    a = uf_find_live(par, a);
    b = uf_find_live(par, b);
    if (a == b) return;
    if (a < b) {
      int t = a;
      a = b;
      b = t;
    }
    const int old = atomicCAS(&par[a], a, b);
    if (old == a) return;
    a = old;
  }
}

// parent[c] = c for gas cells (double-precision density of the stored state
// below rho_th), -1 otherwise
template <class L, class S>
__global__ void k_gas_init(const void* b0, const void* b1, const Ctl* ctl, Geo geo, MapDims d,
                           double rho_th, int* par) {
  if (ctl->stopped) return;
  const void* src = (ctl->steps & 1) ? b1 : b0;
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < d.N;
       c += (long long)gridDim.x * blockDim.x) {
    int x, m, z;
    coords_of(d, c, x, m, z);
    typename S::ct f[L::Q];
    load_pulled<L, S>(src, geo, x, m, z, f);
    double r = 0.0;
#pragma unroll
    for (int i = 0; i < L::Q; i++) r += (double)f[i];
    par[c] = r < rho_th ? (int)c : -1;
  }
}

// same from a host-provided density field
__global__ void k_gas_from_field(const double* rho, MapDims d, double rho_th, int* par) {
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < d.N;
       c += (long long)gridDim.x * blockDim.x)
    par[c] = rho[c] < rho_th ? (int)c : -1;
}

template <class L>
__global__ void k_cc_hook(const Ctl* ctl, MapDims d, int* par) {
  if (ctl->stopped) return;
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < d.N;
       c += (long long)gridDim.x * blockDim.x) {
    if (par[c] < 0) continue;
    int x, m, z;
    coords_of(d, c, x, m, z);
#pragma unroll
    for (int i = 1; i < L::Q; i += 2) {  // one direction of each opposite pair
      const long long y = cell_of(d, wrap_any(x + L::ex[i], d.nx), wrap_any(m + L::em[i], d.nm),
                                  wrap_any(z + L::ez[i], d.nz));
      if (par[y] >= 0) uf_unite(par, (int)c, (int)y);
    }
  }
}

__global__ void k_cc_compress(const Ctl* ctl, MapDims d, int* par) {
  if (ctl->stopped) return;
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < d.N;
       c += (long long)gridDim.x * blockDim.x) {
    if (par[c] < 0) continue;
    par[c] = uf_find_live(par, (int)c);
  }
}

// ---- canonical ranks: count roots per block, scan, write labels ----
constexpr int RANK_BLOCK = 1024;

__global__ __launch_bounds__(RANK_BLOCK) void k_count_roots(const Ctl* ctl, MapDims d, const int* par,
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
__global__ __launch_bounds__(1024) void k_scan_counts(const Ctl* ctl, int* counts, int nblocks, int* total) {
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
__global__ __launch_bounds__(RANK_BLOCK) void k_write_rank(const Ctl* ctl, MapDims d, const int* par,
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

__global__ void k_write_labels(const Ctl* ctl, MapDims d, const int* par, const int* rank, int* label) {
  if (ctl->stopped) return;
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < d.N;
       c += (long long)gridDim.x * blockDim.x) {
    const int p = par[c];
    label[c] = p < 0 ? 0 : rank[p];
  }
}

// ---- owner / dist ----
__global__ void k_owner_init(const Ctl* ctl, MapDims d, const int* label, int2* own, uint8_t* dist) {
  if (ctl->stopped) return;
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < d.N;
       c += (long long)gridDim.x * blockDim.x) {
    const int l = label[c];
    own[c] = make_int2(l, l);
    dist[c] = l > 0 ? 0 : 255;
  }
}

template <class L>
__global__ void k_owner_layer(const Ctl* ctl, MapDims d, int layer, int2* own, uint8_t* dist) {
  if (ctl->stopped) return;
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < d.N;
       c += (long long)gridDim.x * blockDim.x) {
    if (dist[c] != 255) continue;
    int x, m, z;
    coords_of(d, c, x, m, z);
    int lo = 0, hi = 0;
#pragma unroll
    for (int i = 1; i < L::Q; i++) {
      const long long y = cell_of(d, wrap_any(x + L::ex[i], d.nx), wrap_any(m + L::em[i], d.nm),
                                  wrap_any(z + L::ez[i], d.nz));
      if (dist[y] == layer - 1) {
        const int2 o = own[y];
        lo = (lo == 0 || o.x < lo) ? o.x : lo;
        hi = o.y > hi ? o.y : hi;
      }
    }
    if (lo > 0) {
      own[c] = make_int2(lo, hi);
      dist[c] = (uint8_t)layer;
    }
  }
}

// keep the previous labels and aliases for the carry (a device copy, so that
// a refresh queued after a stop leaves everything untouched)
__global__ void k_copy_int(const Ctl* ctl, const int* src, int* dst, long long n) {
  if (ctl->stopped) return;
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < n;
       c += (long long)gridDim.x * blockDim.x)
    dst[c] = src[c];
}

// ---- alias carry across a refresh ----
__global__ void k_alias_reset(const Ctl* ctl, int* alias, int* rep, int nb_cap) {
  if (ctl->stopped) return;
  const int nb = ctl->n_bubbles;
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b <= nb_cap; b += gridDim.x * blockDim.x) {
    if (b <= nb) alias[b] = b;
    rep[b] = 0x7fffffff;
  }
}

__global__ void k_alias_carry1(const Ctl* ctl, MapDims d, const int* label, const int* label_old,
                               const int* alias_old, int* rep) {
  if (ctl->stopped) return;
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < d.N;
       c += (long long)gridDim.x * blockDim.x) {
    const int b = label[c], a = label_old[c];
    if (b > 0 && a > 0) atomicMin(&rep[uf_root(alias_old, a)], b);
  }
}

__global__ void k_alias_carry2(const Ctl* ctl, MapDims d, const int* label, const int* label_old,
                               const int* alias_old, const int* rep, int* alias) {
  if (ctl->stopped) return;
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < d.N;
       c += (long long)gridDim.x * blockDim.x) {
    const int b = label[c], a = label_old[c];
    if (b > 0 && a > 0) {
      const int r = rep[uf_root(alias_old, a)];
      if (r != b) uf_unite(alias, b, r);
    }
  }
}

__global__ void k_alias_compress(const Ctl* ctl, int* alias) {
  if (ctl->stopped) return;
  const int nb = ctl->n_bubbles;
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b <= nb; b += gridDim.x * blockDim.x)
    alias[b] = uf_find_live(alias, b);
}

// ---- barrier candidate masks ----
template <class L>
__global__ void k_masks(const Ctl* ctl, MapDims d, int zone_width, const int2* own, const uint8_t* dist,
                        const int* alias, uint8_t* flag, uint32_t* mask) {
  if (ctl->stopped) return;
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < d.N;
       c += (long long)gridDim.x * blockDim.x) {
    const int2 o = own[c];
    unsigned mk = 0;
    if (o.x > 0) {
      int x, m, z;
      coords_of(d, c, x, m, z);
      const int2 rp = root_pair(alias, o);
      const int dc = dist[c];
#pragma unroll
      for (int i = 1; i < L::Q; i++) {
        const long long y = cell_of(d, wrap_any(x + L::ex[i], d.nx), wrap_any(m + L::em[i], d.nm),
                                    wrap_any(z + L::ez[i], d.nz));
        const int2 oy = own[y];
        if (oy.x <= 0) continue;
        if (dc + (int)dist[y] + 1 > zone_width) continue;
        const int2 rq = root_pair(alias, oy);
        if (rq.x != rp.x || rq.y != rp.y) mk |= 1u << i;
      }
    }
    flag[c] = mk ? 1 : 0;
    mask[c] = mk;
  }
}

// the masks just built reflect the current aliases
__global__ void k_masks_done(Ctl* ctl) {
  if (!ctl->stopped && threadIdx.x == 0) ctl->alias_dirty = 0;
}

}  // namespace flb
