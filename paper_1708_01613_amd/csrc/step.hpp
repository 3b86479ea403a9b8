// step.hpp -- the fused Shan-Chen step kernel and the film-link helpers it shares
// with the query kernels.
//
// One launch advances one lattice by one step (Sec. 2.1.1, 2.1.2, 2.1.5):
// pull populations -> rho, j -> psi(rho) staged in LDS -> neighbour-sum force with
// the film-barrier substitution -> velocity-shifted BGK -> store.  Populations
// are structure-of-arrays planes f[i][cell]; the buffer written at step n holds
// post-collision values at their own cell, and step n+1 pulls f_i(x) from
// cell x - e_i of it (the streaming equation in pull form, periodic).
//
// Work decomposition: a workgroup owns a TX x TM tile of the (x, m) plane and
// a segment of LZ planes along z.  It marches z: for plane zz it pulls the Q
// populations of its own cells (kept in registers) and of a one-cell halo ring
// (summed to rho only), writes psi into a 4-plane LDS ring, and after
// one barrier collides plane zz-1, whose psi neighbours (planes zz-2..zz) are
// all in the ring.  Each population is read once per step plus the halo and
// segment-end planes, and written once.
#pragma once
#include "lattice.hpp"

namespace flb {

struct StepArgs {
  void* buf[2];          // population buffers; buf[steps & 1] holds the current state
  Geo geo;               // block layout of the population buffers
  int nx, nm, nz;        // kernel-coordinate extents
  int tiles_x, tiles_m;  // tile grid of the (x, m) plane
  int lz;                // planes per z segment
  int xcd_chunks;        // > 1: consecutive logical tiles share an XCD
  double tau, G, rho0;
  double psi_bar;        // psi(rho_liquid), used when psi_bar_mode == 0
  int psi_bar_mode;
  int film_on, rupture_warmup, on_rupture;
  int rupture_filter;    // 1: FP32 sign filter before the FP64 rupture test
  int gas_k;             // > 0: a step n with (n + 1) % gas_k == 0 stores every cell's density in rho,
                         // which the film-map refresh at step n + 1 labels
  const uint8_t* flag;   // per cell: 1 where the mask word is not zero (barrier links or kRhoBit)
  const uint32_t* mask;  // per cell: active barrier links (bit i = direction i) and kRhoBit
  const int* flist;      // cells with barrier links at the last refresh (ctl->n_flagged)
  const int2* own;       // per cell: (smallest, largest) nearest bubble label
  const unsigned long long* srcw;  // gas-release source: one bit per cell (the domain gas points),
                                   // one word per 64-cell row block (population block order); null: off
  double src_rate;       // A (dn/dt) of the gas-release law; a step adds the density 3 A (dn/dt) / N
                         // at each of the ctl->n_src = N domain gas points
  int force_on;          // 1: body force of gravity gk (kernel coordinates) on rho - g_rho_ref
  double gk[3];
  double g_rho_ref;
  int* alias;            // union-find parents over labels
  unsigned long long buf_bytes;  // bytes of one population buffer
  long long* events;     // rupture log, 4 x int64 per event: step, k, k2, 0
  unsigned ev_cap;
  Ctl* ctl;
  double* partials;      // 4 doubles per workgroup
  void* psi;             // two-pass path: psi and rho of the current state,
  void* rho;             // compute type, cell-linear
  int open_z;            // 1: the first and last z planes face a liquid reservoir at rest (two-pass path)
  double rho_res;        // its density
};

__device__ __forceinline__ int wrap_dec(int a, int n) { return a == 0 ? n - 1 : a - 1; }
__device__ __forceinline__ int wrap_inc(int a, int n) { return a == n - 1 ? 0 : a + 1; }
__device__ __forceinline__ int wrap_any(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

__device__ __forceinline__ int uf_root(const int* __restrict__ par, int a) {
  int p = par[a];
  while (p != a) {
    a = p;
    p = par[a];
  }
  return a;
}

// (low, high) alias roots of a cell's nearest bubbles
// ---- union-find with roots at the smallest index ----
// Parents only ever move to smaller indices (a root is hooked under a smaller
// root; path halving replaces a parent by its own parent), so every pointer
// stays an ancestor and concurrent finds remain correct.  Roots are written
// only by the hooking CAS.
__device__ __forceinline__ int uf_find_live(int* par, int a) {
  int p = __atomic_load_n(&par[a], __ATOMIC_RELAXED);
  while (p != a) {
    a = p;
    p = __atomic_load_n(&par[a], __ATOMIC_RELAXED);
  }
  return a;
}

__device__ __forceinline__ int uf_find_halve(int* par, int a) {
  int cur = __atomic_load_n(&par[a], __ATOMIC_RELAXED);
  if (cur == a) return a;
  int prev = a, next;
  while (cur > (next = __atomic_load_n(&par[cur], __ATOMIC_RELAXED))) {
    __atomic_store_n(&par[prev], next, __ATOMIC_RELAXED);
    prev = cur;
    cur = next;
  }
  return cur;
}

// unite the sets of a and b, hooking the larger root under the smaller one;
// true if this call did the hook.  The resulting partition and its roots do
// not depend on the order in which concurrent calls land.
__device__ inline bool uf_unite(int* par, int a, int b) {
  while (true) {
    a = uf_find_halve(par, a);
    b = uf_find_halve(par, b);
    if (a == b) return false;
    if (a < b) {
      int t = a;
      a = b;
      b = t;
    }
    const int old = atomicCAS(&par[a], a, b);
    if (old == a) return true;
    a = old;
  }
}

__device__ __forceinline__ int2 root_pair(const int* __restrict__ alias, int2 o) {
  int a = uf_root(alias, o.x), b = uf_root(alias, o.y);
  return a < b ? make_int2(a, b) : make_int2(b, a);
}

// Active barrier links of a flagged cell: candidate links whose two ends still
// have different alias-root pairs (the barrier between a pair of bubbles is
// removed once they are aliased by a rupture).
template <class L>
__device__ __forceinline__ unsigned active_links(const StepArgs& a, int x, int m, int z, long long c) {
  unsigned cand = a.mask[c];
  int2 rp = root_pair(a.alias, a.own[c]);
  unsigned act = 0;
#pragma unroll
  for (int i = 1; i < L::Q; i++) {
    if (cand & (1u << i)) {
      int yx = wrap_any(x + L::ex[i], a.nx);
      int ym = wrap_any(m + L::em[i], a.nm);
      int yz = wrap_any(z + L::ez[i], a.nz);
      long long yc = yx + (long long)a.nx * (ym + (long long)a.nm * yz);
      int2 rq = root_pair(a.alias, a.own[yc]);
      if (rq.x != rp.x || rq.y != rp.y) act |= 1u << i;
    }
  }
  return act;
}

// a + b rounded on its own: never fused with the arithmetic that produced a,
// so adding the source terms (zero when they are off) leaves a's rounding
// exactly as in the kernels that do not add them
__device__ __forceinline__ float add_rn(float a, float b) { return __fadd_rn(a, b); }
__device__ __forceinline__ double add_rn(double a, double b) { return __dadd_rn(a, b); }

template <class T>
__device__ __forceinline__ T psi_of(T rho, T rho0) {
  return rho0 * (T(1) - exp(-rho / rho0));
}

__device__ __forceinline__ double p0_of(double rho, double G, double rho0) {
  double psi = rho0 * (1.0 - exp(-rho / rho0));
  return rho / 3.0 + G / 6.0 * psi * psi;
}

template <class L, class S>
__device__ __forceinline__ void load_pulled(const void* __restrict__ src, const Geo& g, int x, int m, int z,
                                            typename S::ct (&out)[L::Q]) {
  const int xs[3] = {wrap_inc(x, g.nx), x, wrap_dec(x, g.nx)};  // index 1 - e
  const int ms[3] = {L::HAS_M ? wrap_inc(m, g.nm) : 0, m, L::HAS_M ? wrap_dec(m, g.nm) : 0};
  const int zs[3] = {wrap_inc(z, g.nz), z, wrap_dec(z, g.nz)};
#pragma unroll
  for (int i = 0; i < L::Q; i++)  // pull from x - e_i
    out[i] = pop_ld<L, S>(src, g, i, xs[1 + L::ex[i]], ms[1 + L::em[i]], zs[1 + L::ez[i]]);
}

// Sign filter for the FP64 rupture test, FP32 compute types only.  From the
// FP32 rho and psi already staged for the force, D2 = p0(r+) - 2 p0(rc) +
// p0(r-) with p0 = rho/3 + (G/6) psi^2 is formed in FP32 together with a bound
// on its distance from the FP64 value of the same formula at the same FP32
// densities.  The bound is 64 ulp of the sum of the magnitudes of every term,
// where each psi also carries its own evaluation error (at most
// rho0 (|rho/rho0| + 5) ulp for an exp accurate to 2 ulp); that is several
// times what the few FP32 roundings involved can reach.  A value below minus
// the bound proves the FP64 value negative, so no event is possible and the
// FP64 evaluation is skipped; anything else goes to the FP64 formula, which
// alone decides.  Densities outside (0, 64 rho0] always go to FP64.
__device__ __forceinline__ bool d2_may_be_nonneg(float rp, float rc, float rm, float pp, float pc, float pm,
                                                 float g6, float rho0) {
  const float lim = 64.0f * rho0;
  if (!(rp > 0.0f && rc > 0.0f && rm > 0.0f && rp <= lim && rc <= lim && rm <= lim)) return true;
  const float d2 = ((rp + rm) - 2.0f * rc) * (1.0f / 3.0f) + g6 * ((pp * pp + pm * pm) - 2.0f * pc * pc);
  const float ag = fabsf(g6);
  const float ep = 2.0f * pp * (rp + 5.0f * rho0), ec = 2.0f * pc * (rc + 5.0f * rho0),
              em = 2.0f * pm * (rm + 5.0f * rho0);
  const float mag = (rp + 2.0f * rc + rm) * (1.0f / 3.0f) +
                    ag * ((pp * pp + 2.0f * pc * pc + pm * pm) + (ep + 2.0f * ec + em));
  return d2 >= -64.0f * 5.9604645e-08f * mag;
}

// Population access of the step kernel: one buffer resource per population
// buffer, a 32-bit per-lane byte offset (block and lane) and the population's
// run offset inside the block as a constant (BUF, buffers below 2 GiB), or
// plain global addresses (larger buffers).
// Lanes outside the lattice store to kDropOffset, past the end of every buffer
// the buffer path takes (< 2^31 bytes), so the buffer unit discards them; the
// run offsets are small, so the offset sum cannot wrap into the buffer.
constexpr unsigned kDropOffset = 0x80000000u;
constexpr unsigned long long kBufPathLimit = 1ull << 31;
// Cache-policy bits of the population loads and stores on the buffer path
// (gfx950: bit 1 marks an access non-temporal).  A step writes far more than
// the caches hold and nothing it stores is read back before the next step,
// so the stores are non-temporal (measured 5 % faster on the 256^3 lattice);
// the loads stay cached, since neighbouring tiles re-read halo planes.
#ifndef FLB_LD_CPOL
#define FLB_LD_CPOL 0
#endif
#ifndef FLB_ST_CPOL
#define FLB_ST_CPOL 2
#endif
constexpr int kLdCpol = FLB_LD_CPOL;
constexpr int kStCpol = FLB_ST_CPOL;
constexpr unsigned long long kDrop = ~0ull;  // "discard" lane offset before lowering
// s_waitcnt encoding (gfx9): vmcnt(0), expcnt and lgkmcnt left at their maxima
constexpr int kWaitVmcnt0 = 0x0F70;

template <class L, class S, bool BUF>
struct PopIO {
  using T = typename S::ct;
  const char* gs;
  char* gd;
  __amdgpu_buffer_rsrc_t rs, rd;
  Geo g;

  __device__ __forceinline__ void init(const void* src, void* dst, const Geo& geo, unsigned long long bytes) {
    gs = (const char*)src;
    gd = (char*)dst;
    g = geo;
    if (BUF) {
      rs = __builtin_amdgcn_make_buffer_rsrc((void*)src, (short)0, (int)(unsigned)bytes, 0x00020000);
      rd = __builtin_amdgcn_make_buffer_rsrc(dst, (short)0, (int)(unsigned)bytes, 0x00020000);
    }
  }
  // lane offset of cell (x, m, z): block bytes + lane * esz (esz of the
  // moving populations; the FP16 format's FP32 rest run uses lane * 4)
  __device__ __forceinline__ unsigned long long lane_off(int x, int m, int z, int i) const {
    return block_of(g, x, m, z) + (unsigned)(x & 63) * S::esz(i);
  }
  __device__ __forceinline__ T load_at(int i, unsigned long long off) const {
    const unsigned po = S::pofs(i);
    const unsigned vo = (unsigned)off;  // buffer path: every offset is below 2^31
    if constexpr (sizeof(T) == 8) {
      if (BUF) {
        typedef unsigned u2 __attribute__((ext_vector_type(2)));
        const u2 v = __builtin_amdgcn_raw_buffer_load_b64(rs, vo, po, kLdCpol);
        return __builtin_bit_cast(double, v);
      }
      return *(const double*)(gs + off + po);
    } else if (S::HALF && i > 0) {
      return decode(i, load_raw(i, off));
    } else {
      if (BUF) return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, vo, po, kLdCpol));
      return *(const float*)(gs + off + po);
    }
  }
  // store population i of a cell whose lane offset is off (kDrop: discard)
  __device__ __forceinline__ void store_at(int i, unsigned long long off, T v) const {
    if (!BUF && off == kDrop) return;
    const unsigned po = S::pofs(i);
    const unsigned vo = off == kDrop ? kDropOffset : (unsigned)off;
    if constexpr (sizeof(T) == 8) {
      if (BUF) {
        typedef unsigned u2 __attribute__((ext_vector_type(2)));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u2, v), rd, vo, po, kStCpol);
      } else {
        *(double*)(gd + off + po) = v;
      }
    } else if (S::HALF && i > 0) {
      const unsigned short h = h16_enc(v, (float)L::w[i] * g.href);
      if (BUF) __builtin_amdgcn_raw_buffer_store_b16(h, rd, vo, po, kStCpol);
      else *(unsigned short*)(gd + off + po) = h;
    } else {
      if (BUF) __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), rd, vo, po, kStCpol);
      else *(float*)(gd + off + po) = v;
    }
  }
  // the Q populations pulled into cell (x, m, z): f_i(x) = buffer_i(x - e_i)
  __device__ __forceinline__ void pull(int x, int m, int z, T (&out)[L::Q]) const {
    const int xs[3] = {wrap_inc(x, g.nx), x, wrap_dec(x, g.nx)};
    const int ms[3] = {L::HAS_M ? wrap_inc(m, g.nm) : 0, m, L::HAS_M ? wrap_dec(m, g.nm) : 0};
    const int zs[3] = {wrap_inc(z, g.nz), z, wrap_dec(z, g.nz)};
#pragma unroll
    for (int i = 0; i < L::Q; i++)
      out[i] = load_at(i, lane_off(xs[1 + L::ex[i]], ms[1 + L::em[i]], zs[1 + L::ez[i]], i));
  }

  // ---- raw loads: FP16 elements stay undecoded (their 16 bits in the low
  // half of the register) until decode() after the loads have landed.  A
  // conversion right after the load would make the wavefront wait for every
  // load of the plane before the collide that the loads should overlap.
  __device__ __forceinline__ T load_raw(int i, unsigned long long off) const {
    if constexpr (S::HALF) {
      if (i > 0) {
        const unsigned po = S::pofs(i);
        unsigned short h;
        if (BUF) h = __builtin_amdgcn_raw_buffer_load_b16(rs, (unsigned)off, po, kLdCpol);
        else h = *(const unsigned short*)(gs + off + po);
        return __builtin_bit_cast(float, (unsigned)h);
      }
    }
    return load_at(i, off);
  }
  __device__ __forceinline__ T decode(int i, T raw) const {
    if constexpr (S::HALF) {
      if (i > 0) return h16_dec((unsigned short)__builtin_bit_cast(unsigned, raw), (float)L::w[i] * g.href);
    }
    return raw;
  }
  __device__ __forceinline__ void pull_raw(int x, int m, int z, T (&out)[L::Q]) const {
    const int xs[3] = {wrap_inc(x, g.nx), x, wrap_dec(x, g.nx)};
    const int ms[3] = {L::HAS_M ? wrap_inc(m, g.nm) : 0, m, L::HAS_M ? wrap_dec(m, g.nm) : 0};
    const int zs[3] = {wrap_inc(z, g.nz), z, wrap_dec(z, g.nz)};
#pragma unroll
    for (int i = 0; i < L::Q; i++)
      out[i] = load_raw(i, lane_off(xs[1 + L::ex[i]], ms[1 + L::em[i]], zs[1 + L::ez[i]], i));
  }
  __device__ __forceinline__ void decode_all(T (&r)[L::Q]) const {
#pragma unroll
    for (int i = 1; i < L::Q; i++) r[i] = decode(i, r[i]);
  }
};

// FP64 mass / momentum partials of the state entering a step: every
// workgroup reduces its lanes' partials and writes them to its slot.
template <int NT>
__device__ __forceinline__ void step_partials(const StepArgs& a, int slot, double (&red)[NT / 64][4], double acc_m,
                                              double acc_x, double acc_y, double acc_z) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    acc_m += __shfl_down(acc_m, off, 64);
    acc_x += __shfl_down(acc_x, off, 64);
    acc_y += __shfl_down(acc_y, off, 64);
    acc_z += __shfl_down(acc_z, off, 64);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    red[wave][0] = acc_m;
    red[wave][1] = acc_x;
    red[wave][2] = acc_y;
    red[wave][3] = acc_z;
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    double sum = 0.0;
    for (int wv = 0; wv < NT / 64; wv++) sum += red[wv][threadIdx.x];
    a.partials[4ll * slot + threadIdx.x] = sum;
  }
}

// One workgroup, the last launch of every step on the stream (after the step
// kernel, the rupture test and the mask pruning): FP64 totals in workgroup
// order (deterministic), the non-finite check, the stop flag, and the step
// counter that selects the A/B buffer.
constexpr int FIN_NT = 1024;
template <int NT = FIN_NT>
__device__ __forceinline__ void step_finish(const StepArgs& a, int nblk, double (&red)[NT / 64][4]) {
  Ctl* ctl = a.ctl;
  if (ctl->stopped) return;
  double t[4] = {0.0, 0.0, 0.0, 0.0};
  // thread t adds workgroups t, t + NT, ... in that order; four rows are
  // loaded ahead of their additions to keep loads in flight
  const double4* part = (const double4*)a.partials;
  int blk = threadIdx.x;
  for (; blk + 3 * NT < nblk; blk += 4 * NT) {
    const double4 v0 = part[blk], v1 = part[blk + NT], v2 = part[blk + 2 * NT], v3 = part[blk + 3 * NT];
    t[0] += v0.x; t[1] += v0.y; t[2] += v0.z; t[3] += v0.w;
    t[0] += v1.x; t[1] += v1.y; t[2] += v1.z; t[3] += v1.w;
    t[0] += v2.x; t[1] += v2.y; t[2] += v2.z; t[3] += v2.w;
    t[0] += v3.x; t[1] += v3.y; t[2] += v3.z; t[3] += v3.w;
  }
  for (; blk < nblk; blk += NT) {
    const double4 v = part[blk];
    t[0] += v.x; t[1] += v.y; t[2] += v.z; t[3] += v.w;
  }
#pragma unroll
  for (int q = 0; q < 4; q++)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) t[q] += __shfl_down(t[q], off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < 4; q++) red[wave][q] = t[q];
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot[4] = {0.0, 0.0, 0.0, 0.0};
    for (int wv = 0; wv < NT / 64; wv++)
      for (int q = 0; q < 4; q++) tot[q] += red[wv][q];
    ctl->mass = tot[0];
    ctl->mom[0] = tot[1];
    ctl->mom[1] = tot[2];
    ctl->mom[2] = tot[3];
    if (!isfinite(tot[0])) ctl->failed = 1;
  }
  if (threadIdx.x == 0) {
    // the rupture kernel of this step has applied its unions and the mask
    // pruning has consumed them; the flags start clear for the next step
    const bool any = ctl->step_events != 0;
    ctl->step_events = 0;
    ctl->alias_dirty = 0;
    if (a.gas_k > 0 && (ctl->steps + 1) % a.gas_k == 0) ctl->rho_step = ctl->steps;
    ctl->steps = ctl->steps + 1;
    if (any && a.on_rupture) ctl->stopped = 1;
  }
}

static __global__ __launch_bounds__(FIN_NT) void k_step_finish(StepArgs a, int nblk) {
  __shared__ double red[FIN_NT / 64][4];
  step_finish<FIN_NT>(a, nblk, red);
}

// ---- batched launches: many lattices of one lattice type and storage ----
// Workgroups [first[k], first[k+1]) of a batched step launch advance member k
// with its own arguments tab[k]; the finisher launch has one workgroup per
// member.  A member is found by binary search over `first` (nmem + 1 entries).
__device__ __forceinline__ int batch_member(const int* __restrict__ first, int nmem, int b) {
  int lo = 0, hi = nmem;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (first[mid] <= b) lo = mid;
    else hi = mid;
  }
  return lo;
}

static __global__ __launch_bounds__(FIN_NT) void k_step_finish_batch(const StepArgs* __restrict__ tab,
                                                              const int* __restrict__ first) {
  __shared__ double red[FIN_NT / 64][4];
  const int k = blockIdx.x;
  const StepArgs& a = tab[k];  // read in place: a local copy would live in scratch
  step_finish<FIN_NT>(a, first[k + 1] - first[k], red);
}

// Plane loop: iteration k loads plane z0-1+k (k <= L+1) into one register
// set, collides plane z0+k-3 (k >= 3) from the set loaded two iterations
// earlier while the new loads are in flight, then stores psi of the new
// plane into LDS slot k & 3 and synchronises once.  Slot j & 3 holds plane
// z0-1+j; a collide at iteration k reads slots k-3..k-1, and the slot written
// at iteration k was last read before the barrier of iteration k-1.  The three
// register sets rotate by unrolling the loop three times.
//
// FR > 0: the flat tile of 2-D lattices (no march), FR rows per wavefront.
// A workgroup of FW wavefronts owns 64 cells x FH = FW * FR rows (the rows
// z0 .. z0+FH-1, fewer in the last segment); wavefront w keeps rows w*FR ..
// w*FR+FR-1 in registers.  Every wavefront issues the loads of all its rows
// at once (wavefronts 0 and FW-1 also the rows z0-1 and z0+FH around the
// tile, and lanes 0 .. 2FR+1 the end cells x0-1 and x0+TXe of those rows),
// publishes psi of every loaded row into LDS row (z - z0 + 1), synchronises
// once and collides its rows.  A short D2Q9 march spends most of its time
// waiting on one plane of nine loads at a time; here a wavefront has all of
// its rows' loads in flight together.
template <class L, class S, int TX, int TM, bool BUF, bool EXT, int FR = 0>
struct StepBlock {
  using T = typename S::ct;
  static constexpr int Q = L::Q;
  static constexpr int NI = TX * TM;  // interior threads: one cell column each
  static constexpr int HM = L::HAS_M ? 1 : 0;
  static constexpr int LW = TX + 2;
  static constexpr int LH = TM + 2 * HM;
  // halo waves: one lane per ring cell of a full tile.  On 2-D lattices the
  // ring is the two end cells of each plane, which lanes 0 and 1 of the
  // first interior wave load beside their own cells (HIN) instead of a
  // wave of their own
  static constexpr bool HIN = !L::HAS_M;
  static constexpr int NH = 2 * (TM + 2 * HM) + (HM ? 2 * TX : 0);
  static constexpr bool FLAT = FR > 0;
  static constexpr int FW = 4;            // wavefronts of a flat tile
  static constexpr int FH = FR * FW;      // rows of a flat tile
  static_assert(!FLAT || (!L::HAS_M && TX == 64 && TM == 1), "flat tiles are 64-cell D2Q9 row blocks");
  static constexpr int NT = FLAT ? 64 * FW : (HIN ? NI : NI + (NH + 63) / 64 * 64);
  // LDS rows of psi: a ring of 4 planes for the march, every row of a flat tile
  static constexpr int NSLOT = FLAT ? FH + 2 : 4;
  __device__ static constexpr int slot(int j) { return FLAT ? j : (j & 3); }
  struct Smem {
    T psi[NSLOT][LH][LW];
    double red[NT / 64][4];
    int last;
  };

  const StepArgs& a;
  Smem& sm;
  PopIO<L, S, BUF> io;
  Ctl* ctl;
  long long step;
  int nx, nm, nz, x0, m0, z0, L_, TXe, TMe, lx, lm, x, m, xc, mc, gx, gm, hx, hm;
  bool act, has_halo, film, grow, force, test_rupture, tau_one, rho_all;
  T G, rho0, tau, omega, psi_bar, drho, gkx, gkm, gkz, grho;
  double acc_m = 0.0, acc_x = 0.0, acc_y = 0.0, acc_z = 0.0;

  __device__ __forceinline__ StepBlock(const StepArgs& a_, Smem& sm_) : a(a_), sm(sm_) {}

  // interior waves: load the new plane, collide the plane loaded two
  // iterations ago, publish psi of the new plane
  __device__ __forceinline__ void iter(int k, T (&ld)[Q], T (&co)[Q], unsigned& fl_ld, unsigned fl_co) {
    const bool loading = k <= L_ + 1;  // uniform over the workgroup
    T hv[Q];
    if (loading) {
      // every interior lane loads (lanes outside the lattice read clamped
      // cells and never publish), so no divergent branch separates the loads
      // from the collide that overlaps them; the film mask word is read
      // first so the wait that ends this iteration covers it too (one 4-byte
      // word per cell: measured faster than a 1-byte flag with the word read
      // one iteration later only where the flag is set, whose dependent load
      // and branch cost more than the 3 bytes they save)
      const int zl = wrap_any(z0 - 1 + k, nz);
      if (film) fl_ld = a.mask[(unsigned)(xc + nx * (mc + nm * zl))];
      io.pull_raw(xc, mc, zl, ld);
      if (HIN && has_halo) io.pull_raw(gx, gm, zl, hv);
    }
    // keep the collide between the loads and their first use
    __builtin_amdgcn_sched_barrier(0);
    if (k >= 3) collide(k, co, act ? fl_co : 0u);
    __builtin_amdgcn_sched_barrier(0);
    // every load and store of this wave retires here (the sum below needs the
    // loads anyway); starting the next iteration with nothing outstanding
    // keeps the compiler from waiting on the collide's registers there
    __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
    if (loading) {
      // the sum runs on every lane (so the wait for the loads is on every
      // path); only lanes inside the lattice publish it
      const int slot = k & 3;
      io.decode_all(ld);
      if (HIN && has_halo) io.decode_all(hv);
      T r = T(0);
#pragma unroll
      for (int i = 0; i < Q; i++) r += ld[i];
      const T ps = psi_of(r, rho0);
      if (act) sm.psi[slot][lm + HM][lx + 1] = ps;
      if (HIN && has_halo) {
        T rh = T(0);
#pragma unroll
        for (int i = 0; i < Q; i++) rh += hv[i];
        sm.psi[slot][hm + HM][hx + 1] = psi_of(rh, rho0);
      }
    }
    __syncthreads();
  }

  __device__ static __forceinline__ int wrap_row(int z, int n) {
    const int r = z % n;
    return r < 0 ? r + n : r;
  }
  __device__ __forceinline__ void flat_tile() {
    const int w = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const int lane = (int)threadIdx.x & 63;
    const bool actx = lane < TXe;
    T f[FR][Q];
    unsigned fl[FR];
#pragma unroll
    for (int j = 0; j < FR; j++) {
      const int zl = wrap_row(z0 + w * FR + j, nz);
      fl[j] = film ? a.mask[(unsigned)(xc + nx * zl)] : 0u;
      io.pull_raw(xc, 0, zl, f[j]);
    }
    // the rows around the tile (wave-uniform), then the end cells
    const bool hrow = w == 0 || w == FW - 1;
    const int hi = w == 0 ? 0 : FH + 1;
    T fh[Q] = {};
    if (hrow) io.pull_raw(xc, 0, wrap_row(z0 - 1 + hi, nz), fh);
    const bool hend = lane < 2 * FR + (hrow ? 2 : 0);
    const int er = lane < 2 * FR ? w * FR + (lane >> 1) + 1 : hi;
    const int ex_ = (lane & 1) ? TXe : -1;
    T fe[Q] = {};
    if (hend) io.pull_raw(wrap_row(x0 + ex_, nx), 0, wrap_row(z0 - 1 + er, nz), fe);
    __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
#pragma unroll
    for (int j = 0; j < FR; j++) {
      io.decode_all(f[j]);
      T r = T(0);
#pragma unroll
      for (int i = 0; i < Q; i++) r += f[j][i];
      if (actx) sm.psi[w * FR + j + 1][0][lane + 1] = psi_of(r, rho0);
    }
    if (hrow) {
      io.decode_all(fh);
      T r = T(0);
#pragma unroll
      for (int i = 0; i < Q; i++) r += fh[i];
      if (actx) sm.psi[hi][0][lane + 1] = psi_of(r, rho0);
    }
    if (hend) {
      io.decode_all(fe);
      T r = T(0);
#pragma unroll
      for (int i = 0; i < Q; i++) r += fe[i];
      sm.psi[er][0][ex_ + 1] = psi_of(r, rho0);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < FR; j++) {
      const int r = w * FR + j;  // wave-uniform
      if (r < L_) collide(r + 3, f[j], actx ? fl[j] : 0u);
    }
  }

  // halo waves: psi of the ring cells of every loaded plane
  __device__ __forceinline__ void halo_loop() {
    const int kend = L_ + 2;
    for (int k = 0; k <= kend; ++k) {
      if (k <= L_ + 1 && has_halo) {
        T hv[Q];
        io.pull(gx, gm, wrap_any(z0 - 1 + k, nz), hv);
        T r = T(0);
#pragma unroll
        for (int i = 0; i < Q; i++) r += hv[i];
        const int slot = k & 3;
        sm.psi[slot][hm + HM][hx + 1] = psi_of(r, rho0);
      }
      __syncthreads();
    }
  }

  __device__ __forceinline__ void collide(int k, const T (&f)[Q], unsigned flag) {
    // every operation rounds on its own (no contraction into fused
    // multiply-adds): the kernel variants and the two-pass path then give
    // the same values bit for bit whatever other code the compiler sees
#pragma clang fp contract(off)
    const int zc = z0 + k - 3;
    const int sl[3] = {slot(k - 3), slot(k - 2), slot(k - 1)};
    // lanes outside the lattice compute on clamped data and store to an
    // offset past the end of the buffer, which the buffer unit discards
    const unsigned c = (unsigned)(xc + nx * (mc + nm * zc));
    const unsigned long long vo = act ? io.lane_off(x, m, zc, 1) : kDrop;
    const unsigned long long vo0 = act ? io.lane_off(x, m, zc, 0) : kDrop;
    T rho = T(0), jx = T(0), jm = T(0), jz = T(0);
#pragma unroll
    for (int i = 0; i < Q; i++) {
      rho += f[i];
      if (L::ex[i]) jx += L::ex[i] > 0 ? f[i] : -f[i];
      if (L::em[i]) jm += L::em[i] > 0 ? f[i] : -f[i];
      if (L::ez[i]) jz += L::ez[i] > 0 ? f[i] : -f[i];
    }
    const int lm1 = lm + HM, lx1 = lx + 1;
    const T psic = sm.psi[sl[1]][lm1][lx1];
    // the mask holds exactly the active barrier links: it is rebuilt at every
    // refresh and pruned after every step whose ruptures united bubbles
    const unsigned bar = flag & kLinkBits;
    const T pbar = a.psi_bar_mode == 0 ? psi_bar : psic;
    T fx = T(0), fm = T(0), fz = T(0);
#pragma unroll
    for (int i = 1; i < Q; i += 2) {
      // pair (i, i+1) with e_{i+1} = -e_i
      T pp = sm.psi[sl[1 + L::ez[i]]][lm1 + L::em[i]][lx1 + L::ex[i]];
      T pm = sm.psi[sl[1 - L::ez[i]]][lm1 - L::em[i]][lx1 - L::ex[i]];
      if (bar) {
        if (bar & (1u << i)) pp = pbar;
        if (bar & (1u << (i + 1))) pm = pbar;
      }
      const T d = (T)L::w[i] * (pp - pm);
      if (L::ex[i]) fx += L::ex[i] > 0 ? d : -d;
      if (L::em[i]) fm += L::em[i] > 0 ? d : -d;
      if (L::ez[i]) fz += L::ez[i] > 0 ? d : -d;
    }
    const T gp = -G * psic;
    fx *= gp;
    fm *= gp;
    fz *= gp;
    const T inv = T(1) / rho;
    const T ux = (jx + tau * fx) * inv;
    const T um = (jm + tau * fm) * inv;
    const T uz = (jz + tau * fz) * inv;
    const T base = T(1) - T(1.5) * (ux * ux + um * um + uz * uz);
    // gas release at a domain gas point: w_i drho added to every population
    // after the collision (Sec. 2.1.3), zero elsewhere.  The bit's word is
    // one per 64-cell row block: with tiles a whole number of rows wide a
    // wavefront reads one word, through the scalar cache
    T ds = T(0);
    if (EXT && grow) {
      unsigned widx = (unsigned)(xc >> 6) + (unsigned)a.geo.nxb * (unsigned)(mc + nm * zc);
      if constexpr (TX % 64 == 0) widx = __builtin_amdgcn_readfirstlane(widx);
      if ((a.srcw[widx] >> (xc & 63)) & 1ull) ds = drho;
    }
    // body force (Sec. 2.1.1, forcing equation): F_i = w_i rho' [3 (e_i.g -
    // u.g) + 9 (e_i.u)(e_i.g)], rho' = rho - g_rho_ref, u the equilibrium's
    // velocity; per opposite pair its even part w rho' (9 (e.u)(e.g) - 3 u.g)
    // and its odd part w rho' 3 e.g
    T rbg = T(0), ug = T(0);
    if (EXT && force) {
      rbg = rho - grho;
      ug = ux * gkx + um * gkm + uz * gkz;
    }
    // equilibria in opposite pairs: common part w rho (base + 4.5 (e.u)^2),
    // odd part w rho 3 e.u; the rest equilibrium is rho minus the moving ones
    // (equal in exact arithmetic, and it keeps the common rounding of the FP32
    // weights from adding mass every step)
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
      T se = (T)L::w[i] * ds, so = T(0);  // source terms of this pair: even and odd parts
      if (EXT && force) {
        T eg = T(0);
        if (L::ex[i]) eg += L::ex[i] > 0 ? gkx : -gkx;
        if (L::em[i]) eg += L::em[i] > 0 ? gkm : -gkm;
        if (L::ez[i]) eg += L::ez[i] > 0 ? gkz : -gkz;
        const T wb = (T)L::w[i] * rbg;
        se += wb * (T(9) * eu * eg - T(3) * ug);
        so = wb * (T(3) * eg);
      }
      const T yp = tau_one ? fp : f[i] - (f[i] - fp) * omega;
      const T yq = tau_one ? fq : f[i + 1] - (f[i + 1] - fq) * omega;
      io.store_at(i, vo, EXT ? add_rn(yp, se + so) : yp);
      io.store_at(i + 1, vo, EXT ? add_rn(yq, se - so) : yq);
    }
    const T feq0 = rho - feq_moving;
    T s0 = (T)L::w[0] * ds;
    if (EXT && force) s0 += (T)L::w[0] * rbg * (T(-3) * ug);
    const T y0 = tau_one ? feq0 : f[0] - (f[0] - feq0) * omega;
    io.store_at(0, vo0, EXT ? add_rn(y0, s0) : y0);
    // the rupture test runs in its own kernel after this one, on the
    // densities of the state entering the step
    if (act && (rho_all || (test_rupture && (flag & kRhoBit)))) ((T*)a.rho)[c] = rho;
    const double keep = act ? 1.0 : 0.0;
    acc_m += keep * (double)rho;
    acc_x += keep * (double)jx;
    acc_y += keep * (double)(L::HAS_M ? jm : jz);
    acc_z += keep * (double)(L::HAS_M ? jz : T(0));
  }

  // b: workgroup index within this lattice's launch of nblk workgroups
  __device__ __forceinline__ void run(const int b_launch, const int nblk) {
    ctl = a.ctl;
    step = ctl->steps;
    io.init(a.buf[step & 1], a.buf[(step + 1) & 1], a.geo, a.buf_bytes);
    int b = b_launch;
    if (a.xcd_chunks > 1) b = (b % a.xcd_chunks) * (nblk / a.xcd_chunks) + b / a.xcd_chunks;
    const int tx = b % a.tiles_x;
    const int t2 = b / a.tiles_x;
    const int tm = t2 % a.tiles_m;
    const int seg = t2 / a.tiles_m;
    nx = a.nx;
    nm = a.nm;
    nz = a.nz;
    x0 = tx * TX;
    m0 = tm * TM;
    z0 = seg * a.lz;
    L_ = min(z0 + a.lz, nz) - z0;
    TXe = min(TX, nx - x0);
    TMe = min(TM, nm - m0);
    const bool interior = (int)threadIdx.x < NI;
    lx = threadIdx.x % TX;
    lm = threadIdx.x / TX;
    act = interior && lx < TXe && lm < TMe;
    x = x0 + lx;
    m = m0 + lm;
    xc = min(x, nx - 1);
    mc = min(m, nm - 1);
    // halo ring, one lane of the halo waves per cell: two columns (lx = -1,
    // TXe) over lm in [-HM, TMe - 1 + HM], then (3-D only) two rows (lm = -1,
    // TMe) over lx in [0, TXe)
    const int ncol = TMe + 2 * HM;
    const int nh = 2 * ncol + (HM ? 2 * TXe : 0);
    const int h = HIN ? (int)threadIdx.x : (int)threadIdx.x - NI;
    has_halo = (HIN || !interior) && h < nh;
    hx = 0;
    hm = 0;
    if (has_halo) {
      if (h < 2 * ncol) {
        hx = (h < ncol) ? -1 : TXe;
        hm = (h < ncol ? h : h - ncol) - HM;
      } else {
        const int r2 = h - 2 * ncol;
        hx = r2 < TXe ? r2 : r2 - TXe;
        hm = r2 < TXe ? -1 : TMe;
      }
    }
    gx = wrap_any(x0 + hx, nx);
    gm = wrap_any(m0 + hm, nm);
    G = (T)a.G;
    rho0 = (T)a.rho0;
    tau = (T)a.tau;
    omega = T(1) / (T)a.tau;
    tau_one = a.tau == 1.0;
    film = a.film_on != 0;
    grow = EXT && a.srcw != nullptr && ctl->n_src > 0;
    force = EXT && a.force_on;
    gkx = (T)a.gk[0];
    gkm = (T)a.gk[1];
    gkz = (T)a.gk[2];
    grho = (T)a.g_rho_ref;
    drho = grow ? (T)(3.0 * (a.src_rate / (double)ctl->n_src)) : T(0);
    test_rupture = film && step >= a.rupture_warmup;
    rho_all = a.gas_k > 0 && (step + 1) % a.gas_k == 0;
    psi_bar = (T)a.psi_bar;

    if constexpr (FLAT) {
      lx = (int)threadIdx.x & 63;
      lm = 0;
      m = 0;
      mc = 0;
      x = x0 + lx;
      xc = min(x, nx - 1);
      act = lx < TXe;
      flat_tile();
    } else if (interior) {
      T r0[Q], r1[Q], r2[Q];
      unsigned g0 = 0, g1 = 0, g2 = 0;
      const int kend = L_ + 2;
      for (int k = 0; k <= kend; k += 3) {
        iter(k, r0, r1, g0, g1);
        if (k + 1 > kend) break;
        iter(k + 1, r1, r2, g1, g2);
        if (k + 2 > kend) break;
        iter(k + 2, r2, r0, g2, g0);
      }
    } else {
      halo_loop();
    }
    // partials slot: the launch-order index, which the finisher sums in order
    step_partials<NT>(a, b_launch, sm.red, acc_m, acc_x, acc_y, acc_z);
  }
};

// EXT: the variant with the source terms after the collision, the gas release
// and the body force (their code costs registers, so lattices without them
// run the variant without it)
template <class L, class S, int TX, int TM, bool BUF, bool EXT, int FR = 0>
__global__ __launch_bounds__((StepBlock<L, S, TX, TM, BUF, EXT, FR>::NT)) void k_step(StepArgs a) {
  using SB = StepBlock<L, S, TX, TM, BUF, EXT, FR>;
  __shared__ typename SB::Smem sm;
  if (a.ctl->stopped) return;
  SB blk(a, sm);
  blk.run(blockIdx.x, gridDim.x);
}

template <class L, class S, int TX, int TM, bool BUF, bool EXT, int FR = 0>
__global__ __launch_bounds__((StepBlock<L, S, TX, TM, BUF, EXT, FR>::NT)) void k_step_batch(
    const StepArgs* __restrict__ tab, const int* __restrict__ first, int nmem) {
  using SB = StepBlock<L, S, TX, TM, BUF, EXT, FR>;
  __shared__ typename SB::Smem sm;
  const int k = batch_member(first, nmem, blockIdx.x);
  const StepArgs& a = tab[k];  // read in place: a local copy would live in scratch
  if (a.ctl->stopped) return;
  SB blk(a, sm);
  blk.run(blockIdx.x - first[k], first[k + 1] - first[k]);
}

}  // namespace flb
