// rupture.hpp -- the film-rupture test (Sec. 2.1.5, eta_m criterion; Sec. 5,
// Fig. plot), as a kernel of its own that runs after the step kernel.
//
// On every active barrier link (x, i) of a step from rupture_warmup on, the
// FP64 second difference of the bulk pressure p0 = rho/3 + (G/6) psi^2 along
// the link direction, D2 = p0(rho(x+e_i)) - 2 p0(rho(x)) + p0(rho(x-e_i)), is
// tested for D2 >= 0; each hit appends (step, smaller owner, larger owner2) of
// the link's two ends to the event log.  The densities are those of the state
// entering the step, which the step kernel (or k_psi) leaves in a cell-linear
// array (only at cells the refresh marked with kRhoBit).  The test walks the
// list of cells that had barrier links at the refresh.  Keeping it out of the
// step kernel keeps its sparse, divergent FP64 work off the streaming
// kernel's critical path.
#pragma once
#include "maps.hpp"

namespace flb {

// Arguments of the two-lattice model beyond those of the melt lattice (which
// the StepArgs describe): the gas lattice of Sec. 2.1.5, coupled to the melt
// at the end of every step.
struct TLArgs {
  void* gbuf[2];             // the gas lattice's A/B population buffers (the melt's layout)
  unsigned long long gbytes; // bytes of one of them
  void* rho_g;               // gas density and pseudopotential, cell-linear, compute type
  void* psi_g;
  double G_mg, G_gg, tau_g;  // couplings melt-gas and gas-gas; the gas relaxation time
  double psi_bar_g;          // psi of the gas density in the bulk melt
  double rho_g_res;          // gas density of the bulk melt (and of the reservoir of an open container)
};

// bulk pressure of the two lattices together: (rho_m + rho_g)/3 + (G psi_m^2
// + 2 G_mg psi_m psi_g + G_gg psi_g^2)/6, FP64
__device__ __forceinline__ double p_tl_of(double rm, double rg, double G, double G_mg, double G_gg, double rho0) {
  const double a = rho0 * (1.0 - exp(-rm / rho0)), b = rho0 * (1.0 - exp(-rg / rho0));
  return (rm + rg) / 3.0 + (G * a * a + 2.0 * G_mg * a * b + G_gg * b * b) / 6.0;
}

// A hit on link (x, i) unites the pair (k, k2) = (smaller owner, larger
// owner2 of the two ends) in the alias union-find at once.  No test of this
// step reads the aliases (the links to test are the mask, pruned before the
// step), so the barrier still goes away only from the next step on; the
// union-find keeps the smallest label as root, so the classes, their roots
// and the number of successful unions do not depend on the order in which
// the unions land.  A wavefront merges its lanes' identical pairs first, and
// the log keeps one record per distinct (step, k, k2) of a wavefront until it
// is full.
// TWO: the two-lattice model, whose pressure takes both densities (the gas
// densities from tl->rho_g); always FP64, no FP32 pre-check.
template <class L, class T, bool TWO = false>
__device__ __forceinline__ void rupture_cells(const StepArgs& a, unsigned bid, unsigned nb,
                                              const TLArgs* tl = nullptr) {
  Ctl* ctl = a.ctl;
  if (ctl->stopped) return;
  const long long step = ctl->steps;
  if (!a.film_on || step < a.rupture_warmup) return;
  const T* rho = (const T*)a.rho;
  const double G64 = a.G, r064 = a.rho0;
  const float g6 = (float)(G64 / 6.0), r0f = (float)r064;
  const MapDims d{a.nx, a.nm, a.nz, (long long)a.nx * a.nm * a.nz};
  const int lane = threadIdx.x & 63;
  for_list(ctl->n_flagged, bid, nb, [&](unsigned idx, bool act) {
        // every lane of the wavefront runs the loop below (inactive ones with
        // an empty mask), so the pair merging sees the whole wavefront
        const unsigned c = act ? (unsigned)a.flist[idx] : 0u;
        const unsigned mk = act ? a.mask[c] & kLinkBits : 0u;
        const ListCell q(d, c);
        const T rc = mk ? rho[c] : T(1);
        T psc = T(0);
        if constexpr (sizeof(T) == 4 && !TWO) psc = psi_of(rc, r0f);
        double pc = 0.0;
        bool have_pc = false;
        int2 oc = make_int2(0, 0);
#pragma unroll
        for (int i = 1; i < L::Q; i++) {
          if (!(mk & (1u << i))) continue;
          const unsigned yp = q.nb(d, L::ex[i], L::em[i], L::ez[i]);
          const unsigned ym = q.nb(d, -L::ex[i], -L::em[i], -L::ez[i]);
          // beyond an open plane the reservoir's densities
          const bool op = a.open_z && (q.z + L::ez[i] < 0 || q.z + L::ez[i] >= a.nz);
          const bool om = a.open_z && (q.z - L::ez[i] < 0 || q.z - L::ez[i] >= a.nz);
          const T rp = op ? (T)a.rho_res : rho[yp], rm = om ? (T)a.rho_res : rho[ym];
          bool hit = false;
          if constexpr (TWO) {
            const T* rg = (const T*)tl->rho_g;
            if (!have_pc) {
              pc = p_tl_of((double)rc, (double)rg[c], G64, tl->G_mg, tl->G_gg, r064);
              oc = a.own[c];
              have_pc = true;
            }
            const double gp = op ? tl->rho_g_res : (double)rg[yp], gm = om ? tl->rho_g_res : (double)rg[ym];
            hit = p_tl_of((double)rp, gp, G64, tl->G_mg, tl->G_gg, r064) - 2.0 * pc +
                      p_tl_of((double)rm, gm, G64, tl->G_mg, tl->G_gg, r064) >=
                  0.0;
          } else if (sizeof(T) != 4 || !a.rupture_filter || op || om ||
                     d2_may_be_nonneg((float)rp, (float)rc, (float)rm, psi_of((float)rp, r0f), (float)psc,
                                      psi_of((float)rm, r0f), g6, r0f)) {
            if (!have_pc) {
              pc = p0_of((double)rc, G64, r064);
              oc = a.own[c];
              have_pc = true;
            }
            hit = p0_of((double)rp, G64, r064) - 2.0 * pc + p0_of((double)rm, G64, r064) >= 0.0;
          }
          int k = 0, k2 = 0;
          if (hit) {
            const int2 oy = a.own[yp];
            k = min(oc.x, oy.x);
            k2 = max(oc.y, oy.y);
          }
          // one lane per distinct pair of the wavefront (its leader); the
          // leaders unite concurrently, and the wavefront takes its log
          // records and counts with one atomic each (a burst of ruptures
          // would otherwise queue on two counters)
          unsigned long long todo = __ballot(hit);
          bool leader = false;
          while (todo) {
            const int ld = first_lane(todo);
            const int k0 = __shfl(k, ld, 64), k20 = __shfl(k2, ld, 64);
            if (lane == ld) leader = true;
            if (hit && k == k0 && k2 == k20) hit = false;
            todo = __ballot(hit);
          }
          const unsigned long long lmask = __ballot(leader);
          if (lmask) {  // wave-uniform
            const int first = first_lane(lmask);
            const bool united = leader && uf_unite(a.alias, k, k2);
            const unsigned long long umask = __ballot(united);
            unsigned base = a.ev_cap;
            if (lane == first) {
              ctl->step_events = 1;
              if (umask) {
                atomicAdd((unsigned long long*)&ctl->n_ruptures, (unsigned long long)__popcll(umask));
                ctl->alias_dirty = 1;
              }
              if (__atomic_load_n(&ctl->ev_count, __ATOMIC_RELAXED) < a.ev_cap)
                base = atomicAdd(&ctl->ev_count, (unsigned)__popcll(lmask));
            }
            base = __shfl(base, first, 64);
            if (leader) {
              const unsigned e = base + (unsigned)__popcll(lmask & ((1ull << lane) - 1ull));
              if (base < a.ev_cap && e < a.ev_cap) {
                long long* ev = a.events + 4ll * e;
                ev[0] = step;
                ev[1] = k;
                ev[2] = k2;
                ev[3] = 0;
              } else {
                ctl->ev_full = 1;
              }
            }
          }
        }
      });
}

template <class L, class T>
__global__ __launch_bounds__(MAP_NT) void k_rupture(StepArgs a) {
  rupture_cells<L, T>(a, blockIdx.x, gridDim.x);
}

template <class L, class T>
__global__ __launch_bounds__(MAP_NT) void k_rupture_tl(StepArgs a, TLArgs t) {
  rupture_cells<L, T, true>(a, blockIdx.x, gridDim.x, &t);
}

// batched: workgroups [first[k], first[k+1]) test member k
template <class L, class T>
__global__ __launch_bounds__(MAP_NT) void k_rupture_batch(const StepArgs* __restrict__ tab,
                                                          const int* __restrict__ first, int nmem) {
  const int k = batch_member(first, nmem, blockIdx.x);
  const StepArgs& a = tab[k];  // read in place: a local copy would live in scratch
  rupture_cells<L, T>(a, blockIdx.x - first[k], first[k + 1] - first[k]);
}

}  // namespace flb
