// twopass.hpp -- the step as two independent-lane kernels.
//
// k_psi pulls each cell's populations and writes rho and psi(rho) of the
// current state to two cell-linear arrays; k_collide pulls them again, reads
// psi of its neighbours from the array (through the caches), and does the
// force with the film barrier, the velocity-shifted BGK, the store, the FP64
// rupture test and the FP64 partials.  Every lane works on its own cell and
// no workgroup barrier sits between a load and its use, so many waves per CU
// hide the memory latency; the price is a second read of the populations
// (245 instead of 153 bytes per lattice update for FP32).
// A workgroup covers TP_ROWS rows of one 64-cell block column: cells
// (64 xb + lane, row) with row = m + nm z.
#pragma once
#include "step.hpp"

namespace flb {

constexpr int TP_ROWS = 4;
constexpr int TP_NT = 64 * TP_ROWS;

__device__ __forceinline__ int tp_block(const StepArgs& a) {
  int b = blockIdx.x;
  const int nblk = gridDim.x;
  if (a.xcd_chunks > 1) b = (b % a.xcd_chunks) * (nblk / a.xcd_chunks) + b / a.xcd_chunks;
  return b;
}

template <class T, bool BUF>
struct CellArray {
  const T* p;
  __amdgpu_buffer_rsrc_t r;
  __device__ __forceinline__ void init(const void* base, unsigned long long n) {
    p = (const T*)base;
    if (BUF) r = __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, (int)(unsigned)(n * sizeof(T)), 0x00020000);
  }
  __device__ __forceinline__ T operator[](unsigned c) const {
    if constexpr (BUF) {
      if constexpr (sizeof(T) == 8) {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, c * 8u, 0u, 0));
      } else {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, c * 4u, 0u, 0));
      }
    }
    return p[c];
  }
};

template <class L, class S, bool BUF>
__global__ __launch_bounds__(TP_NT) void k_psi(StepArgs a) {
  using T = typename S::ct;
  const Ctl* ctl = a.ctl;
  if (ctl->stopped) return;
  const long long step = ctl->steps;
  PopIO<L, S, BUF> io;
  io.init(a.buf[step & 1], a.buf[(step + 1) & 1], a.geo, a.buf_bytes);
  const int b = tp_block(a);
  const int xb = b % a.geo.nxb, rg = b / a.geo.nxb;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row = rg * TP_ROWS + wave;
  if (row >= a.nm * a.nz) return;  // a whole wave; this kernel has no barrier
  const int x = xb * kBlk + lane;
  const int m = row % a.nm, z = row / a.nm;
  T f[L::Q];
  io.pull(min(x, a.nx - 1), m, z, f);
  T r = T(0);
#pragma unroll
  for (int i = 0; i < L::Q; i++) r += f[i];
  if (x < a.nx) {
    const unsigned c = (unsigned)(x + a.nx * row);
    ((T*)a.psi)[c] = psi_of(r, (T)a.rho0);
    ((T*)a.rho)[c] = r;
  }
}

template <class L, class S, bool BUF>
__global__ __launch_bounds__(TP_NT) void k_collide(StepArgs a) {
  // the same uncontracted arithmetic as the fused kernel's collide
#pragma clang fp contract(off)
  using T = typename S::ct;
  constexpr int Q = L::Q;
  __shared__ double red[TP_NT / 64][4];
  Ctl* ctl = a.ctl;
  if (ctl->stopped) return;
  const long long step = ctl->steps;
  PopIO<L, S, BUF> io;
  io.init(a.buf[step & 1], a.buf[(step + 1) & 1], a.geo, a.buf_bytes);
  const unsigned long long N = (unsigned long long)a.nx * a.nm * a.nz;
  CellArray<T, BUF> psi;
  psi.init(a.psi, N);
  const int b = tp_block(a);
  const int xb = b % a.geo.nxb, rg = b / a.geo.nxb;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nrows = a.nm * a.nz;
  const int row_raw = rg * TP_ROWS + wave;
  const int x = xb * kBlk + lane;
  const bool act = row_raw < nrows && x < a.nx;
  // lanes outside the lattice run on a clamped cell and their stores are dropped
  const int row = min(row_raw, nrows - 1);
  const int xc = min(x, a.nx - 1);
  const int m = row % a.nm, z = row / a.nm;
  const int nx = a.nx, nm = a.nm, nz = a.nz;

  T f[Q];
  io.pull(xc, m, z, f);
  T rho = T(0), jx = T(0), jm = T(0), jz = T(0);
#pragma unroll
  for (int i = 0; i < Q; i++) {
    rho += f[i];
    if (L::ex[i]) jx += L::ex[i] > 0 ? f[i] : -f[i];
    if (L::em[i]) jm += L::em[i] > 0 ? f[i] : -f[i];
    if (L::ez[i]) jz += L::ez[i] > 0 ? f[i] : -f[i];
  }
  const unsigned c = (unsigned)(xc + nx * row);
  const int xs[3] = {wrap_dec(xc, nx), xc, wrap_inc(xc, nx)};  // index 1 + e
  const int ms[3] = {L::HAS_M ? wrap_dec(m, nm) : 0, m, L::HAS_M ? wrap_inc(m, nm) : 0};
  const int zs[3] = {wrap_dec(z, nz), z, wrap_inc(z, nz)};
  auto nb = [&](int ex, int em, int ez) -> unsigned {
    return (unsigned)(xs[1 + ex] + nx * (ms[1 + em] + nm * zs[1 + ez]));
  };
  const T psic = psi[c];
  const unsigned bar = (a.film_on && act) ? a.mask[c] & kLinkBits : 0u;  // exact active links
  const T pbar = a.psi_bar_mode == 0 ? (T)a.psi_bar : psic;
  // an open container: the planes beyond z = 0 and z = nz - 1 hold the reservoir
  const bool lo_open = a.open_z && z == 0, hi_open = a.open_z && z == nz - 1;
  // (reservoir values rounded once from FP64)
  const T pres = a.open_z ? (T)(a.rho0 * (1.0 - exp(-a.rho_res / a.rho0))) : T(0);
  T fx = T(0), fm = T(0), fz = T(0);
#pragma unroll
  for (int i = 1; i < Q; i += 2) {
    T pp = psi[nb(L::ex[i], L::em[i], L::ez[i])];
    T pm = psi[nb(-L::ex[i], -L::em[i], -L::ez[i])];
    if ((L::ez[i] > 0 && hi_open) || (L::ez[i] < 0 && lo_open)) pp = pres;
    if ((L::ez[i] > 0 && lo_open) || (L::ez[i] < 0 && hi_open)) pm = pres;
    if (bar) {
      if (bar & (1u << i)) pp = pbar;
      if (bar & (1u << (i + 1))) pm = pbar;
    }
    const T d = (T)L::w[i] * (pp - pm);
    if (L::ex[i]) fx += L::ex[i] > 0 ? d : -d;
    if (L::em[i]) fm += L::em[i] > 0 ? d : -d;
    if (L::ez[i]) fz += L::ez[i] > 0 ? d : -d;
  }
  const T G = (T)a.G, tau = (T)a.tau, omega = T(1) / (T)a.tau;
  const bool tau_one = a.tau == 1.0;
  const T gp = -G * psic;
  fx *= gp;
  fm *= gp;
  fz *= gp;
  const T inv = T(1) / rho;
  const T ux = (jx + tau * fx) * inv;
  const T um = (jm + tau * fm) * inv;
  const T uz = (jz + tau * fz) * inv;
  const T base = T(1) - T(1.5) * (ux * ux + um * um + uz * uz);
  const unsigned long long vo = act ? io.lane_off(x, m, z, 1) : kDrop;
  const unsigned long long vo0 = act ? io.lane_off(x, m, z, 0) : kDrop;
  // gas release at a domain gas point (Sec. 2.1.3): w_i drho on every population
  const long long nsrc = a.srcw ? a.ctl->n_src : 0;
  const bool src = nsrc > 0 && ((a.srcw[(xc >> 6) + a.geo.nxb * row] >> (xc & 63)) & 1ull);
  const T ds = src ? (T)(3.0 * (a.src_rate / (double)nsrc)) : T(0);
  // body force (Sec. 2.1.1, forcing equation), as in the fused kernel
  const bool force = a.force_on != 0;
  const T gkx = (T)a.gk[0], gkm = (T)a.gk[1], gkz = (T)a.gk[2];
  const T rbg = force ? rho - (T)a.g_rho_ref : T(0);
  const T ug = force ? ux * gkx + um * gkm + uz * gkz : T(0);
  // paired equilibria; the rest equilibrium is rho minus the moving ones
  T feq_moving = T(0);
#pragma unroll
  for (int i = 1; i < Q; i += 2) {
    T eu = T(0);
    if (L::ex[i]) eu += L::ex[i] > 0 ? ux : -ux;
    if (L::em[i]) eu += L::em[i] > 0 ? um : -um;
    if (L::ez[i]) eu += L::ez[i] > 0 ? uz : -uz;
    const T wr = (T)L::w[i] * rho;
    const T even = wr * (base + T(4.5) * eu * eu);
    const T odd = wr * (T(3) * eu);
    const T fp = even + odd, fq = even - odd;
    feq_moving += fp + fq;
    T se = (T)L::w[i] * ds, so = T(0);  // source terms (gas release, body force): even and odd parts
    if (force) {
      T eg = T(0);
      if (L::ex[i]) eg += L::ex[i] > 0 ? gkx : -gkx;
      if (L::em[i]) eg += L::em[i] > 0 ? gkm : -gkm;
      if (L::ez[i]) eg += L::ez[i] > 0 ? gkz : -gkz;
      const T wb = (T)L::w[i] * rbg;
      se += wb * (T(9) * eu * eg - T(3) * ug);
      so = wb * (T(3) * eg);
    }
    // the source terms are added on their own (zero when off: the fused
    // kernel's values exactly)
    T vp = add_rn(tau_one ? fp : f[i] - (f[i] - fp) * omega, se + so);
    T vq = add_rn(tau_one ? fq : f[i + 1] - (f[i + 1] - fq) * omega, se - so);
    // a population that leaves through an open plane is gone; the slot it
    // would take is the one the opposite plane pulls from, which receives the
    // reservoir's population at rest instead
    if ((L::ez[i] > 0 && hi_open) || (L::ez[i] < 0 && lo_open)) vp = (T)(L::w[i] * a.rho_res);
    if ((L::ez[i] > 0 && lo_open) || (L::ez[i] < 0 && hi_open)) vq = (T)(L::w[i] * a.rho_res);
    io.store_at(i, vo, vp);
    io.store_at(i + 1, vo, vq);
  }
  const T feq0 = rho - feq_moving;
  T s0 = (T)L::w[0] * ds;
  if (force) s0 += (T)L::w[0] * rbg * (T(-3) * ug);
  io.store_at(0, vo0, add_rn(tau_one ? feq0 : f[0] - (f[0] - feq0) * omega, s0));

  // the rupture test runs in its own kernel, on the rho array of k_psi
  const double keep = act ? 1.0 : 0.0;
  step_partials<TP_NT>(a, blockIdx.x, red, keep * (double)rho, keep * (double)jx, keep * (double)(L::HAS_M ? jm : jz),
                       keep * (double)(L::HAS_M ? jz : T(0)));
}

// The two-pass decompositions leave one partial per 256 cells (65536 at
// 256^3), more than the one-workgroup finisher reads quickly: groups of
// FOLD consecutive partials are summed, in order, into the slots after the
// last one, and the finisher reads those (a fixed order, so the totals stay
// deterministic).
constexpr int FOLD = 64;
static __global__ __launch_bounds__(64) void k_fold_partials(double* partials, int nblk) {
  const int g = blockIdx.x, q = threadIdx.x & 3, r = threadIdx.x >> 2;  // 16 rows x 4 quantities
  double t = 0.0;
  for (int k = r; k < FOLD; k += 16) {
    const int blk = g * FOLD + k;
    if (blk < nblk) t += partials[4ll * blk + q];
  }
  __shared__ double s[16][4];
  s[r][q] = t;
  __syncthreads();
  if (threadIdx.x < 4) {
    double u = 0.0;
    for (int k = 0; k < 16; k++) u += s[k][threadIdx.x];
    partials[4ll * (nblk + g) + threadIdx.x] = u;
  }
}

}  // namespace flb
