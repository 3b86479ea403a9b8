// ops.hpp -- initialisation, state import/export, queries and FP64 totals.
#pragma once
#include "maps.hpp"

namespace flb {

// Vigna's SplitMix64 output function of one 64-bit state.
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long x) {
  unsigned long long z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Initial density (Sec. 2.1.3): rho_gas inside any nucleus (periodic minimum
// image, integer cell centres), rho_liquid elsewhere, plus a (2U - 1) noise.
// Lattice coordinates (x, y, z); FP64 without contraction so that the inside
// test rounds exactly like a plain C evaluation.  With srcw given, the cells
// inside a nucleus are also the domain gas points of the gas-release source:
// their bits are set in srcw (one word per 64-cell row block, the population
// block order: word x / 64 + nxb * (c / nx)) and counted in *nsrc; both must
// start at zero.
static __global__ void k_init_density(double* rho, int nx, int ny, int nz, long long N, const double4* nuc, int nn,
                               double rl, double rg, double amp, unsigned long long seed,
                               unsigned long long* srcw, int nxb, unsigned long long* nsrc) {
#pragma clang fp contract(off)
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < N;
       c += (long long)gridDim.x * blockDim.x) {
    const long long x = c % nx, y = (c / nx) % ny, z = c / ((long long)nx * ny);
    bool inside = false;
    for (int k = 0; k < nn && !inside; k++) {
      const double4 q = nuc[k];
      double dx = (double)x - q.x, dy = (double)y - q.y, dz = (double)z - q.z;
      dx = dx - (double)nx * floor(dx / (double)nx + 0.5);
      dy = dy - (double)ny * floor(dy / (double)ny + 0.5);
      dz = dz - (double)nz * floor(dz / (double)nz + 0.5);
      const double d2 = dx * dx + dy * dy + dz * dz;
      if (d2 <= q.w * q.w) inside = true;
    }
    const unsigned long long h = splitmix64(seed ^ ((unsigned long long)c * 0x9E3779B97F4A7C15ull));
    const double u = (double)(h >> 11) * (1.0 / 9007199254740992.0);
    rho[c] = (inside ? rg : rl) + amp * (2.0 * u - 1.0);
    if (srcw && inside) {
      atomicOr(&srcw[(x >> 6) + (long long)nxb * (c / nx)], 1ull << (x & 63));
      atomicAdd(nsrc, 1ull);
    }
  }
}

// Plain device copy dst[i] = src[i] of n 16-byte elements, U loads in flight
// per lane, grid-stride, non-temporal stores: the practical HBM ceiling of a
// kernel that reads and writes the same number of bytes, which the step
// kernel is compared with.
typedef float f4v __attribute__((ext_vector_type(4)));
template <int U>
__global__ __launch_bounds__(256) void k_copy16(const f4v* __restrict__ src, f4v* __restrict__ dst, long long n) {
  const long long stride = (long long)gridDim.x * 256 * U;
  for (long long base = (long long)blockIdx.x * 256 * U + threadIdx.x; base < n; base += stride) {
    f4v v[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      const long long i = base + (long long)u * 256;
      if (i < n) v[u] = src[i];
    }
#pragma unroll
    for (int u = 0; u < U; u++) {
      const long long i = base + (long long)u * 256;
      if (i < n) __builtin_nontemporal_store(v[u], &dst[i]);
    }
  }
}

// Bulk pressure p0 = rho/3 + (G/6) psi^2 (Eq. Pequ) of an FP64 density field.
static __global__ void k_pressure(const double* rho, long long N, double G, double rho0, double* out) {
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < N;
       c += (long long)gridDim.x * blockDim.x)
    out[c] = p0_of(rho[c], G, rho0);
}

// Write a state into the pull layout: buffer[i][c] holds f_i(c + e_i).
// mode 0: f_i = w_i * field[c] (rest equilibrium of a density field);
// mode 1: f_i = field[i * N + c] (populations in direction order).
template <class L, class S>
__global__ void k_pack(void* buf, Geo geo, MapDims d, const double* field, int mode) {
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < d.N;
       c += (long long)gridDim.x * blockDim.x) {
    int x, m, z;
    coords_of(d, c, x, m, z);
#pragma unroll
    for (int i = 0; i < L::Q; i++) {
      const long long y = cell_of(d, wrap_any(x + L::ex[i], d.nx), wrap_any(m + L::em[i], d.nm),
                                  wrap_any(z + L::ez[i], d.nz));
      using T = typename S::ct;
      const T v = mode == 0 ? (T)(L::w[i] * field[y]) : (T)field[(long long)i * d.N + y];
      pop_st<L, S>(buf, geo, i, x, m, z, v);
    }
  }
}

// Current populations f_i(c) = buffer[i][c - e_i] as FP64, direction order.
template <class L, class S>
__global__ void k_unpack(const void* b0, const void* b1, const Ctl* ctl, Geo geo, MapDims d, double* out) {
  const void* src = (ctl->steps & 1) ? b1 : b0;
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < d.N;
       c += (long long)gridDim.x * blockDim.x) {
    int x, m, z;
    coords_of(d, c, x, m, z);
    typename S::ct f[L::Q];
    load_pulled<L, S>(src, geo, x, m, z, f);
#pragma unroll
    for (int i = 0; i < L::Q; i++) out[(long long)i * d.N + c] = (double)f[i];
  }
}

// FP64 moments of the current state: rho, then D momentum planes (lattice axes)
template <class L, class S>
__global__ void k_moments(const void* b0, const void* b1, const Ctl* ctl, Geo geo, MapDims d,
                          double* rho, double* j) {
  const void* src = (ctl->steps & 1) ? b1 : b0;
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < d.N;
       c += (long long)gridDim.x * blockDim.x) {
    int x, m, z;
    coords_of(d, c, x, m, z);
    typename S::ct f[L::Q];
    load_pulled<L, S>(src, geo, x, m, z, f);
    double r = 0.0, jj[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < L::Q; i++) {
      const double v = (double)f[i];
      r += v;
#pragma unroll
      for (int k = 0; k < L::D; k++)
        if (L::comp(i, k)) jj[k] += L::comp(i, k) > 0 ? v : -v;
    }
    rho[c] = r;
    if (j)
#pragma unroll
      for (int k = 0; k < L::D; k++) j[(long long)k * d.N + c] = jj[k];
  }
}

// u = j/rho (mode 0) or (j + F/2)/rho (mode 1) with the force of the current
// state under the current film maps, in FP64 from the FP64 moments
template <class L>
__global__ void k_velocity(StepArgs a, MapDims d, const double* rho, const double* j, int mode, double* out) {
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < d.N;
       c += (long long)gridDim.x * blockDim.x) {
    double F[3] = {0.0, 0.0, 0.0};
    if (mode == 1) {
      int x, m, z;
      coords_of(d, c, x, m, z);
      const double psic = psi_of(rho[c], a.rho0);
      unsigned bar = 0;
      if (a.film_on && a.flag[c]) bar = active_links<L>(a, x, m, z, c);
      const double pb = a.psi_bar_mode == 0 ? a.psi_bar : psic;
      for (int i = 1; i < L::Q; i += 2) {
        const long long yp = cell_of(d, wrap_any(x + L::ex[i], d.nx), wrap_any(m + L::em[i], d.nm),
                                     wrap_any(z + L::ez[i], d.nz));
        const long long ym = cell_of(d, wrap_any(x - L::ex[i], d.nx), wrap_any(m - L::em[i], d.nm),
                                     wrap_any(z - L::ez[i], d.nz));
        double pp = psi_of(rho[yp], a.rho0), pm = psi_of(rho[ym], a.rho0);
        if (a.open_z && (z + L::ez[i] < 0 || z + L::ez[i] >= d.nz)) pp = psi_of(a.rho_res, a.rho0);  // the reservoir
        if (a.open_z && (z - L::ez[i] < 0 || z - L::ez[i] >= d.nz)) pm = psi_of(a.rho_res, a.rho0);
        if (bar & (1u << i)) pp = pb;
        if (bar & (1u << (i + 1))) pm = pb;
        const double dd = L::w[i] * (pp - pm);
        for (int k = 0; k < L::D; k++) F[k] += L::comp(i, k) * dd;
      }
      for (int k = 0; k < L::D; k++) F[k] *= -a.G * psic;
    }
    for (int k = 0; k < L::D; k++) out[(long long)k * d.N + c] = (j[(long long)k * d.N + c] + 0.5 * F[k]) / rho[c];
  }
}

// FP64 totals: per-block partial sums of up to 4 planes, then one block sums
// the partials in block order (deterministic)
constexpr int RED_BLOCK = 256;
static __global__ __launch_bounds__(RED_BLOCK) void k_reduce_partial(const double* planes, int nplanes, long long N,
                                                              double* partials) {
  double t[4] = {0.0, 0.0, 0.0, 0.0};
  for (long long c = blockIdx.x * (long long)RED_BLOCK + threadIdx.x; c < N; c += (long long)gridDim.x * RED_BLOCK)
    for (int q = 0; q < nplanes; q++) t[q] += planes[(long long)q * N + c];
  __shared__ double s[RED_BLOCK / 64][4];
  for (int q = 0; q < 4; q++)
    for (int off = 32; off > 0; off >>= 1) t[q] += __shfl_down(t[q], off, 64);
  if ((threadIdx.x & 63) == 0)
    for (int q = 0; q < 4; q++) s[threadIdx.x >> 6][q] = t[q];
  __syncthreads();
  if (threadIdx.x < 4) {
    double v = 0.0;
    for (int w = 0; w < RED_BLOCK / 64; w++) v += s[w][threadIdx.x];
    partials[4ll * blockIdx.x + threadIdx.x] = v;
  }
}

static __global__ __launch_bounds__(64) void k_reduce_final(const double* partials, int nblocks, double* out) {
  if (threadIdx.x < 4) {
    double v = 0.0;
    for (int b = 0; b < nblocks; b++) v += partials[4ll * b + threadIdx.x];
    out[threadIdx.x] = v;
  }
}

// bubble sizes (cells per label) and equivalent-diameter histogram
// p[0 .. n) = v (clears without hipMemset, which captured graphs mishandle)
static __global__ void k_fill_u64(unsigned long long* p, long long n, unsigned long long v) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}

static __global__ void k_label_sizes(const int* label, long long N, unsigned long long* sizes) {
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < N;
       c += (long long)gridDim.x * blockDim.x) {
    const int l = label[c];
    if (l > 0) atomicAdd(&sizes[l], 1ull);
  }
}

static __global__ void k_histogram(const unsigned long long* sizes, const int* n_bubbles, int D, int nbins, double width,
                            unsigned long long* counts) {
  const int nb = *n_bubbles;
  for (int b = 1 + blockIdx.x * blockDim.x + threadIdx.x; b <= nb; b += gridDim.x * blockDim.x) {
    const double v = (double)sizes[b];
    const double dm = D == 2 ? 2.0 * sqrt(v / 3.141592653589793) : cbrt(6.0 * v / 3.141592653589793);
    long long k = (long long)floor(dm / width);
    if (k >= nbins) k = nbins - 1;
    if (k < 0) k = 0;
    atomicAdd(&counts[k], 1ull);
  }
}

// Foam statistics of the label sizes (Sec. 5, Table 5): out[0] bubble cell
// fraction, out[1] relative foam density 1 - fraction, out[2] mean and
// out[3] largest equivalent diameter, out[4] bubble cells.  One workgroup;
// thread t sums bubbles t+1, t+1+FS_NT, ... in order, then fixed-order
// wavefront and workgroup reductions, so the result does not depend on timing.
constexpr int FS_NT = 1024;
static __global__ __launch_bounds__(FS_NT) void k_foam_stats(const unsigned long long* __restrict__ sizes,
                                                            const int* n_bubbles, int D, long long N, double* out) {
  __shared__ double s_sum[FS_NT / 64], s_max[FS_NT / 64];
  __shared__ unsigned long long s_gas[FS_NT / 64];
  const int nb = *n_bubbles;
  double sum = 0.0, dmax = 0.0;
  unsigned long long gas = 0;
  for (int b = 1 + (int)threadIdx.x; b <= nb; b += FS_NT) {
    const double v = (double)sizes[b];
    const double dm = D == 2 ? 2.0 * sqrt(v / 3.141592653589793) : cbrt(6.0 * v / 3.141592653589793);
    sum += dm;
    dmax = fmax(dmax, dm);
    gas += sizes[b];
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    sum += __shfl_down(sum, off, 64);
    dmax = fmax(dmax, __shfl_down(dmax, off, 64));
    gas += __shfl_down(gas, off, 64);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    s_sum[wave] = sum;
    s_max[wave] = dmax;
    s_gas[wave] = gas;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double S = 0.0, M = 0.0;
    unsigned long long Gc = 0;
    for (int w = 0; w < FS_NT / 64; w++) {
      S += s_sum[w];
      M = fmax(M, s_max[w]);
      Gc += s_gas[w];
    }
    out[0] = (double)Gc / (double)N;
    out[1] = 1.0 - out[0];
    out[2] = nb > 0 ? S / (double)nb : 0.0;
    out[3] = M;
    out[4] = (double)Gc;
  }
}

// ---- overlap of two labellings (coalescence tracking, Sec. 5) ----
// Every cell that is gas in both labellings adds one to the count of its
// (old label, new label) pair in an open-addressing table of `mask + 1`
// slots (keys kMatchEmpty when free).  Along a wavefront, equal pairs come in
// runs (bubbles are contiguous in x); the first lane of a run adds the run's
// length, so a bubble costs one atomic per row segment.  A key probes at most
// every slot once; one that finds no room sets *overflow (the host retries
// with a larger table).
constexpr unsigned long long kMatchEmpty = ~0ull;

static __global__ __launch_bounds__(256) void k_match_pairs(const int* __restrict__ old_label,
                                                            const int* __restrict__ new_label, long long N,
                                                            unsigned long long* keys, unsigned long long* counts,
                                                            unsigned mask, int* overflow) {
  const int lane = threadIdx.x & 63;
  const long long stride = (long long)gridDim.x * blockDim.x;
  // wave-uniform loop: the run detection below needs the whole wavefront
  for (long long base = blockIdx.x * (long long)blockDim.x + (threadIdx.x & ~63); base < N; base += stride) {
    const long long c = base + lane;
    int a = 0, b = 0;
    if (c < N) {
      a = old_label[c];
      b = new_label[c];
    }
    const bool valid = a > 0 && b > 0;
    const bool first = run_head(a, b);  // every lane takes part in the shuffle
    const bool head = valid && first;
    // lanes where a run (or a gap of cells that are not gas in both) starts
    const unsigned long long starts = __ballot(!valid || head);
    if (!head) continue;
    const unsigned long long above = lane == 63 ? 0ull : starts >> (lane + 1);
    const unsigned long long len = above ? (unsigned long long)__builtin_ctzll(above) + 1ull : (unsigned long long)(64 - lane);
    const unsigned long long key = ((unsigned long long)(unsigned)a << 32) | (unsigned)b;
    unsigned h = (unsigned)((key * 0x9E3779B97F4A7C15ull) >> 32) & mask;
    bool placed = false;
    for (unsigned probe = 0; probe <= mask; probe++) {
      const unsigned long long prev = atomicCAS(&keys[h], kMatchEmpty, key);
      if (prev == kMatchEmpty || prev == key) {
        atomicAdd(&counts[h], len);
        placed = true;
        break;
      }
      h = (h + 1) & mask;
    }
    if (!placed) atomicExch(overflow, 1);
  }
}

}  // namespace flb
