// twolattice.hpp -- the two-lattice step (Sec. 2.1.5: the melt and the gas on
// two separate lattices, coupled at the end of every step; Fig.
// Mainflowchart, "Domain coupling").
//
// Per step n, both lattices pulled from their A/B buffers:
//   1. moments of each lattice, rho_s and j_s; psi_s = rho0 (1 - e^{-rho_s/rho0})
//   2. forces on each lattice from both (Shan-Chen, summed over opposite pairs)
//        F_m = -psi_m(x) sum_i w_i e_i [G psi~_m(x+e_i) + G_mg psi~_g(x+e_i)]
//        F_g = -psi_g(x) sum_i w_i e_i [G_mg psi~_m(x+e_i) + G_gg psi~_g(x+e_i)]
//      where psi~ is the neighbour's value, or on an active barrier link that
//      of the bulk melt (psi_bar_mode 0) or of x itself (mode 1): only the
//      nearest bubble's gas acts at x, the per-bubble selection of the paper
//   3. the common velocity u' = (j_m / tau + j_g / tau_g) / (rho_m / tau +
//      rho_g / tau_g) (the printed (u_melt + u_gas) / sum rho, read with
//      momenta, of which this is the equal-tau case; it makes the collisions
//      of both lattices together conserve momentum)
//   4. BGK of each lattice towards the equilibrium at u' + tau_s F_s / rho_s
//   5. stores of both lattices; FP64 partials of the total mass and momentum
// As two independent-lane kernels: k_psi_tl writes rho and psi of both
// lattices to cell-linear arrays, k_collide_tl does the rest (the two-pass
// design of twopass.hpp, with two population sets).  The rupture test runs
// on the two-component pressure (k_rupture_tl); the film maps are built from
// the melt density as on one lattice.
#pragma once
#include "rupture.hpp"
#include "twopass.hpp"

namespace flb {

template <class L, class S, bool BUF>
__global__ __launch_bounds__(TP_NT) void k_psi_tl(StepArgs a, TLArgs t) {
  using T = typename S::ct;
  const Ctl* ctl = a.ctl;
  if (ctl->stopped) return;
  const long long step = ctl->steps;
  PopIO<L, S, BUF> im, ig;
  im.init(a.buf[step & 1], a.buf[(step + 1) & 1], a.geo, a.buf_bytes);
  ig.init(t.gbuf[step & 1], t.gbuf[(step + 1) & 1], a.geo, t.gbytes);
  const int b = tp_block(a);
  const int xb = b % a.geo.nxb, rg = b / a.geo.nxb;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row = rg * TP_ROWS + wave;
  if (row >= a.nm * a.nz) return;  // a whole wave; this kernel has no barrier
  const int x = xb * kBlk + lane;
  const int m = row % a.nm, z = row / a.nm;
  T f[L::Q], g[L::Q];
  im.pull(min(x, a.nx - 1), m, z, f);
  ig.pull(min(x, a.nx - 1), m, z, g);
  T rm = T(0), rgs = T(0);
#pragma unroll
  for (int i = 0; i < L::Q; i++) {
    rm += f[i];
    rgs += g[i];
  }
  if (x < a.nx) {
    const unsigned c = (unsigned)(x + a.nx * row);
    ((T*)a.psi)[c] = psi_of(rm, (T)a.rho0);
    ((T*)a.rho)[c] = rm;
    ((T*)t.psi_g)[c] = psi_of(rgs, (T)a.rho0);
    ((T*)t.rho_g)[c] = rgs;
  }
}

template <class L, class S, bool BUF>
__global__ __launch_bounds__(TP_NT) void k_collide_tl(StepArgs a, TLArgs t) {
#pragma clang fp contract(off)
  using T = typename S::ct;
  constexpr int Q = L::Q;
  __shared__ double red[TP_NT / 64][4];
  Ctl* ctl = a.ctl;
  if (ctl->stopped) return;
  const long long step = ctl->steps;
  PopIO<L, S, BUF> im, ig;
  im.init(a.buf[step & 1], a.buf[(step + 1) & 1], a.geo, a.buf_bytes);
  ig.init(t.gbuf[step & 1], t.gbuf[(step + 1) & 1], a.geo, t.gbytes);
  const unsigned long long N = (unsigned long long)a.nx * a.nm * a.nz;
  CellArray<T, BUF> psm, psg;
  psm.init(a.psi, N);
  psg.init(t.psi_g, N);
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

  // 1. moments of both lattices
  T f[Q], g[Q];
  im.pull(xc, m, z, f);
  ig.pull(xc, m, z, g);
  T rm = T(0), rgs = T(0), jm[3] = {T(0), T(0), T(0)}, jg[3] = {T(0), T(0), T(0)};
#pragma unroll
  for (int i = 0; i < Q; i++) {
    rm += f[i];
    rgs += g[i];
    const int e[3] = {L::ex[i], L::em[i], L::ez[i]};
#pragma unroll
    for (int k = 0; k < 3; k++)
      if (e[k]) {
        jm[k] += e[k] > 0 ? f[i] : -f[i];
        jg[k] += e[k] > 0 ? g[i] : -g[i];
      }
  }
  // 2. neighbour sums of both pseudopotentials, with the barrier substitution
  const unsigned c = (unsigned)(xc + nx * row);
  const int xs[3] = {wrap_dec(xc, nx), xc, wrap_inc(xc, nx)};  // index 1 + e
  const int ms[3] = {L::HAS_M ? wrap_dec(m, nm) : 0, m, L::HAS_M ? wrap_inc(m, nm) : 0};
  const int zs[3] = {wrap_dec(z, nz), z, wrap_inc(z, nz)};
  auto nb = [&](int ex, int em, int ez) -> unsigned {
    return (unsigned)(xs[1 + ex] + nx * (ms[1 + em] + nm * zs[1 + ez]));
  };
  const T pmc = psm[c], pgc = psg[c];
  const unsigned bar = (a.film_on && act) ? a.mask[c] & kLinkBits : 0u;  // exact active links
  const T bm = a.psi_bar_mode == 0 ? (T)a.psi_bar : pmc;
  const T bg = a.psi_bar_mode == 0 ? (T)t.psi_bar_g : pgc;
  // an open container: the planes beyond z = 0 and z = nz - 1 hold the reservoir
  const bool lo_open = a.open_z && z == 0, hi_open = a.open_z && z == nz - 1;
  // (reservoir values rounded once from FP64)
  const double rm_res = a.rho_res, rg_res = t.rho_g_res;
  const T pm_res = a.open_z ? (T)(a.rho0 * (1.0 - exp(-a.rho_res / a.rho0))) : T(0), pg_res = (T)t.psi_bar_g;
  T am[3] = {T(0), T(0), T(0)}, ag[3] = {T(0), T(0), T(0)};
#pragma unroll
  for (int i = 1; i < Q; i += 2) {
    const unsigned yp = nb(L::ex[i], L::em[i], L::ez[i]), ym = nb(-L::ex[i], -L::em[i], -L::ez[i]);
    T mp = psm[yp], mq = psm[ym], gp = psg[yp], gq = psg[ym];
    if ((L::ez[i] > 0 && hi_open) || (L::ez[i] < 0 && lo_open)) {
      mp = pm_res;
      gp = pg_res;
    }
    if ((L::ez[i] > 0 && lo_open) || (L::ez[i] < 0 && hi_open)) {
      mq = pm_res;
      gq = pg_res;
    }
    if (bar) {
      if (bar & (1u << i)) {
        mp = bm;
        gp = bg;
      }
      if (bar & (1u << (i + 1))) {
        mq = bm;
        gq = bg;
      }
    }
    const T dm = (T)L::w[i] * (mp - mq), dg = (T)L::w[i] * (gp - gq);
    const int e[3] = {L::ex[i], L::em[i], L::ez[i]};
#pragma unroll
    for (int k = 0; k < 3; k++)
      if (e[k]) {
        am[k] += e[k] > 0 ? dm : -dm;
        ag[k] += e[k] > 0 ? dg : -dg;
      }
  }
  const T G = (T)a.G, Gmg = (T)t.G_mg, Ggg = (T)t.G_gg;
  const T tm = (T)a.tau, tg = (T)t.tau_g;
  // 3. common velocity and the shifted equilibrium velocities
  const T den = rm / tm + rgs / tg;
  T um[3], ug[3];
#pragma unroll
  for (int k = 0; k < 3; k++) {
    const T Fm = -pmc * (G * am[k] + Gmg * ag[k]);
    const T Fg = -pgc * (Gmg * am[k] + Ggg * ag[k]);
    const T uc = (jm[k] / tm + jg[k] / tg) / den;
    um[k] = uc + tm * Fm / rm;
    ug[k] = uc + tg * Fg / rgs;
  }
  // 4, 5. BGK of each lattice, stores
  const unsigned long long vo = act ? im.lane_off(x, m, z, 1) : kDrop;
  const unsigned long long vo0 = act ? im.lane_off(x, m, z, 0) : kDrop;
  // gas release at a domain gas point (Sec. 2.1.3), into the gas lattice
  const long long nsrc = a.srcw ? a.ctl->n_src : 0;
  const bool src = nsrc > 0 && ((a.srcw[(xc >> 6) + a.geo.nxb * row] >> (xc & 63)) & 1ull);
  const T ds = src ? (T)(3.0 * (a.src_rate / (double)nsrc)) : T(0);
  // (rres: the reservoir density of this lattice, for the populations that
  // enter through an open plane; ds: the released density, gas lattice only)
  auto collide = [&](const PopIO<L, S, BUF>& io, const T (&p)[Q], T rho, const T (&u)[3], T tau, double rres, T dsrc) {
    const T omega = T(1) / tau;
    const T base = T(1) - T(1.5) * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    T moving = T(0);
#pragma unroll
    for (int i = 1; i < Q; i += 2) {
      T eu = T(0);
      if (L::ex[i]) eu += L::ex[i] > 0 ? u[0] : -u[0];
      if (L::em[i]) eu += L::em[i] > 0 ? u[1] : -u[1];
      if (L::ez[i]) eu += L::ez[i] > 0 ? u[2] : -u[2];
      const T wr = (T)L::w[i] * rho;
      const T even = wr * (base + T(4.5) * eu * eu);
      const T odd = wr * (T(3) * eu);
      const T fp = even + odd, fq = even - odd;
      moving += fp + fq;
      T vp = p[i] - (p[i] - fp) * omega + (T)L::w[i] * dsrc;
      T vq = p[i + 1] - (p[i + 1] - fq) * omega + (T)L::w[i] * dsrc;
      // through an open plane: out of the container; the slot is refilled from the reservoir
      if ((L::ez[i] > 0 && hi_open) || (L::ez[i] < 0 && lo_open)) vp = (T)(L::w[i] * rres);
      if ((L::ez[i] > 0 && lo_open) || (L::ez[i] < 0 && hi_open)) vq = (T)(L::w[i] * rres);
      io.store_at(i, vo, vp);
      io.store_at(i + 1, vo, vq);
    }
    const T feq0 = rho - moving;
    io.store_at(0, vo0, p[0] - (p[0] - feq0) * omega + (T)L::w[0] * dsrc);
  };
  collide(im, f, rm, um, tm, rm_res, T(0));
  collide(ig, g, rgs, ug, tg, rg_res, ds);
  const double keep = act ? 1.0 : 0.0;
  step_partials<TP_NT>(a, blockIdx.x, red, keep * ((double)rm + (double)rgs), keep * ((double)jm[0] + (double)jg[0]),
                       keep * ((double)jm[L::HAS_M ? 1 : 2] + (double)jg[L::HAS_M ? 1 : 2]),
                       keep * (L::HAS_M ? (double)jm[2] + (double)jg[2] : 0.0));
}

// FP64 queries of the two lattices from their FP64 moments (planes: rho, then
// the D momentum components, per lattice): the pressure of the two
// components, and the velocity of the mixture (j_m + j_g [+ (F_m + F_g)/2]) /
// (rho_m + rho_g) with the forces of the current state under the film maps
template <class L>
__global__ void k_tl_query(StepArgs a, TLArgs t, MapDims d, const double* mq, const double* gq, int what,
                           int mode, double* out) {
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < d.N;
       c += (long long)gridDim.x * blockDim.x) {
    const double rm = mq[c], rg = gq[c];
    if (what == 0) {
      out[c] = p_tl_of(rm, rg, a.G, t.G_mg, t.G_gg, a.rho0);
      continue;
    }
    double F[3] = {0.0, 0.0, 0.0};
    if (mode == 1) {
      int x, m, z;
      coords_of(d, c, x, m, z);
      const double pm = psi_of(rm, a.rho0), pg = psi_of(rg, a.rho0);
      unsigned bar = 0;
      if (a.film_on && a.flag[c]) bar = active_links<L>(a, x, m, z, c);
      const double bm = a.psi_bar_mode == 0 ? a.psi_bar : pm, bg = a.psi_bar_mode == 0 ? t.psi_bar_g : pg;
      double sm[3] = {0.0, 0.0, 0.0}, sg[3] = {0.0, 0.0, 0.0};
      for (int i = 1; i < L::Q; i += 2) {
        const long long yp = cell_of(d, wrap_any(x + L::ex[i], d.nx), wrap_any(m + L::em[i], d.nm),
                                     wrap_any(z + L::ez[i], d.nz));
        const long long ym = cell_of(d, wrap_any(x - L::ex[i], d.nx), wrap_any(m - L::em[i], d.nm),
                                     wrap_any(z - L::ez[i], d.nz));
        double mp = psi_of(mq[yp], a.rho0), mm = psi_of(mq[ym], a.rho0);
        double gp = psi_of(gq[yp], a.rho0), gm = psi_of(gq[ym], a.rho0);
        if (a.open_z && (z + L::ez[i] < 0 || z + L::ez[i] >= d.nz)) {  // the reservoir
          mp = psi_of(a.rho_res, a.rho0);
          gp = t.psi_bar_g;
        }
        if (a.open_z && (z - L::ez[i] < 0 || z - L::ez[i] >= d.nz)) {
          mm = psi_of(a.rho_res, a.rho0);
          gm = t.psi_bar_g;
        }
        if (bar & (1u << i)) {
          mp = bm;
          gp = bg;
        }
        if (bar & (1u << (i + 1))) {
          mm = bm;
          gm = bg;
        }
        for (int k = 0; k < L::D; k++) {
          sm[k] += L::comp(i, k) * L::w[i] * (mp - mm);
          sg[k] += L::comp(i, k) * L::w[i] * (gp - gm);
        }
      }
      for (int k = 0; k < L::D; k++) F[k] = -pm * (a.G * sm[k] + t.G_mg * sg[k]) - pg * (t.G_mg * sm[k] + t.G_gg * sg[k]);
    }
    for (int k = 0; k < L::D; k++)
      out[(long long)k * d.N + c] = (mq[(long long)(1 + k) * d.N + c] + gq[(long long)(1 + k) * d.N + c] + 0.5 * F[k]) / (rm + rg);
  }
}

}  // namespace flb
