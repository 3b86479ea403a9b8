// persist.hpp -- a batch of D2Q9 lattices advanced by one persistent launch
// per run of steps between film-map refreshes.
//
// The launch is cooperative: all of its workgroups are resident at once, and
// a grid-wide barrier separates the phases of each step, which otherwise
// are separate launches:
//   A. the step tiles of every member (tiles of 256 x 1 cells, the member's
//      workgroup range of the batched launch, taken round-robin);
//   B. the rupture test over the flagged cells of every film member;
//   C. the pruning of the links of pairs united in B;
//   D. the finisher of every member (its totals, stop flag and step count,
//      which select the buffers of the next step's tiles).
// Each phase reads only what the previous phases wrote, as in the separate
// launches, so the populations, maps and events equal those of the batched
// launches; the FP64 totals are summed in another (fixed) order.  The map
// refresh stays a pipeline of launches before the run.
#pragma once
#include <hip/hip_cooperative_groups.h>

#include "maps.hpp"
#include "rupture.hpp"
#include "step.hpp"

namespace flb {

constexpr int PERSIST_TX = 256;  // the D2Q9 batch tile whose workgroup is 256 threads

template <class S, bool BUF, bool EXT>
__global__ __launch_bounds__(256) void k_batch_persist(const StepArgs* __restrict__ tab,
                                                       const int* __restrict__ first, int nmem,
                                                       const StepArgs* __restrict__ ftab,
                                                       const PruneArgs* __restrict__ ptab,
                                                       const int* __restrict__ ffirst, int nf, int nsteps) {
  using SB = StepBlock<D2Q9K, S, PERSIST_TX, 1, BUF, EXT>;
  static_assert(SB::NT == 256, "persistent workgroups are 256 threads");
  __shared__ typename SB::Smem sm;
  namespace cg = cooperative_groups;
  cg::grid_group grid = cg::this_grid();
  const int nblk = first[nmem], fblk = nf ? ffirst[nf] : 0;
  for (int s = 0; s < nsteps; s++) {
    for (int t = blockIdx.x; t < nblk; t += gridDim.x) {  // A
      const int k = batch_member(first, nmem, t);
      const StepArgs& a = tab[k];
      if (a.ctl->stopped) continue;  // workgroup-uniform
      SB blk(a, sm);
      blk.run(t - first[k], first[k + 1] - first[k]);
      __syncthreads();  // the LDS ring is reused by the next tile
    }
    grid.sync();
    for (int t = blockIdx.x; t < fblk; t += gridDim.x) {  // B
      const int k = batch_member(ffirst, nf, t);
      rupture_cells<D2Q9K, typename S::ct>(ftab[k], t - ffirst[k], ffirst[k + 1] - ffirst[k]);
    }
    grid.sync();
    for (int t = blockIdx.x; t < fblk; t += gridDim.x) {  // C
      const int k = batch_member(ffirst, nf, t);
      mask_prune<D2Q9K>(ptab[k], t - ffirst[k], ffirst[k + 1] - ffirst[k]);
    }
    grid.sync();
    for (int k = blockIdx.x; k < nmem; k += gridDim.x) {  // D
      step_finish<256>(tab[k], first[k + 1] - first[k], sm.red);
      __syncthreads();
    }
    grid.sync();
  }
}

}  // namespace flb
