/*
 * foamlbm.h -- C ABI of the MI355X (gfx950) Shan-Chen foam lattice-Boltzmann library.
 *
 * The library advances the single-component Shan-Chen lattice-Boltzmann model
 * with the inter-bubble film barrier and rupture criterion of Barzegari et al.,
 * "Multiphase Aluminum A356 Foam Formation Process Simulation Using Lattice
 * Boltzmann Method" (arXiv:1708.01613), on D2Q9 and D3Q19 lattices with
 * periodic boundaries.  One time step n -> n+1 (Sec. 2.1.1, Sec. 2.1.2,
 * Sec. 2.1.5) computes, per cell:
 *   rho = sum_i f_i, j = sum_i e_i f_i                    (Eq. vel_dens)
 *   psi = rho0 (1 - exp(-rho / rho0))                    (Eq. pseudopotential)
 *   F   = -G psi(x) sum_i w_i psi~(x + e_i) e_i          (Eq. shanchen3)
 *         psi~ = psi_bar on an active film-barrier link   (Sec. 2.1.5, Fig. shanchenflowchart)
 *   u_eq = (j + tau F) / rho                             (Sec. 2.1.5, final-velocity equations)
 *   f*_i = f_i - (f_i - f_i^eq(rho, u_eq)) / tau          (collision and f^eq equations)
 *   f_i(x + e_i, n + 1) = f*_i(x)                        (streaming equation)
 * and, on active barrier links from step rupture_warmup on, the FP64 test
 * p0(rho(x+e_i)) - 2 p0(rho(x)) + p0(rho(x-e_i)) >= 0 with
 * p0 = rho/3 + (G/6) psi^2 (Eq. Pequ; eta_m equation), which removes the
 * barrier between that pair of bubbles from step n+1 on.
 *
 * Conventions
 *  - Every function returns an int status: FLB_OK (0) or a negative FLB_E*
 *    code; flb_last_error() returns a thread-local message for the last error.
 *    Arguments are validated before any device work.  No C++ exception
 *    crosses this boundary.
 *  - Cell index c = x + nx * (y + ny * z) (x fastest).  D2Q9 requires nz == 1.
 *  - Population order (direction i, lattice vectors e_i):
 *      D2Q9 : (0,0) (1,0) (-1,0) (0,1) (0,-1) (1,1) (-1,-1) (1,-1) (-1,1)
 *      D3Q19: (0,0,0) (1,0,0) (-1,0,0) (0,1,0) (0,-1,0) (0,0,1) (0,0,-1)
 *             (1,1,0) (-1,-1,0) (1,-1,0) (-1,1,0) (1,0,1) (-1,0,-1)
 *             (1,0,-1) (-1,0,1) (0,1,1) (0,-1,-1) (0,1,-1) (0,-1,1)
 *    Weights: rest 4/9, axes 1/9, diagonals 1/36 (D2Q9, Sec. 2.1.1);
 *    rest 1/3, axes 1/18, face diagonals 1/36 (D3Q19).
 *  - Host buffers passed in or out are owned by the caller.  Device state is
 *    owned by the context and allocated through the caller's allocator (or
 *    hipMalloc when none is given); it is freed by flb_destroy.
 *  - All device work is enqueued on the stream given at creation.  Calls that
 *    return host data synchronise that stream; flb_step does not.
 *  - A context is not thread-safe; distinct contexts may be used concurrently.
 */
#ifndef FOAMLBM_H
#define FOAMLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  FLB_OK = 0,
  FLB_EINVAL = -1,   /* invalid argument or parameter */
  FLB_ENOMEM = -2,   /* device allocation failed */
  FLB_ENUMERIC = -3, /* NaN / non-finite mass detected by the FP64 reduction */
  FLB_EBUSY = -4,    /* resource exhausted (event log, label capacity) */
  FLB_EHIP = -5,     /* a HIP runtime call failed */
  FLB_STOPPED = 1    /* informational: the run stopped on a film rupture */
};

enum { FLB_D2Q9 = 0, FLB_D3Q19 = 1 };
enum { FLB_F64 = 0, FLB_F32 = 1, FLB_F16S = 2 };

typedef struct flb_ctx flb_ctx;

/* Device-memory allocator supplied by the caller (e.g. a framework's caching
 * allocator).  alloc returns a device pointer (or NULL on failure) aligned to
 * at least 256 bytes; free releases it.  Pass NULL to use hipMalloc/hipFree. */
typedef struct {
  void* (*alloc)(size_t bytes, void* user);
  void (*free)(void* ptr, void* user);
  void* user;
} flb_allocator;

/* Problem definition ("Input DATA", "Geometry define", "Lattice define" of
 * Fig. Mainflowchart).  All quantities in lattice units. */
typedef struct {
  int32_t lattice;       /* FLB_D2Q9 or FLB_D3Q19 */
  int32_t storage;       /* FLB_F64, FLB_F32, or FLB_F16S (FP16 of f_i - w_i, FP32 compute) */
  int32_t nx, ny, nz;    /* periodic extents, each >= 1; nz == 1 for D2Q9 */
  double tau;            /* BGK relaxation time, > 0.5 (viscosity (tau - 1/2)/3) */
  double G;              /* Shan-Chen coupling (G < -4 separates phases for rho0 = 1) */
  double rho0;           /* pseudopotential scale, > 0 (the paper uses 1) */
  double rho_liquid;     /* initial liquid density */
  double rho_gas;        /* initial density inside nuclei */
  double noise_amp;      /* initial uniform noise amplitude a: rho += a (2U - 1) */
  uint64_t seed;         /* seed of the counter-based noise */
  int32_t film_on;       /* 1: film barrier and rupture test on */
  int32_t k_own;         /* film maps are rebuilt before every step n with n % k_own == 0 (>= 1) */
  int32_t zone_width;    /* largest film thickness (lattice links) that carries a barrier, 1..15 */
  double rho_th;         /* gas iff rho < rho_th (default ln 2, the critical density) */
  int32_t psi_bar_mode;  /* psi on barrier links: 0 = psi(rho_liquid), 1 = psi(x) */
  int32_t rupture_warmup;/* first step at which the rupture test runs */
  int32_t on_rupture;    /* 0: remove the pair's barrier and continue; 1: stop after the step */
  int32_t velocity_mode; /* flb_get_velocity: 0 = j/rho, 1 = (j + F/2)/rho */
} flb_params;

/* Fills p with defaults: D2Q9 F32 64x64x1, tau 1, G -5, rho0 1, rho_liquid 2,
 * rho_gas 0.15, noise 0.01, seed 1, film off, k_own 10, zone_width 6,
 * rho_th ln 2, psi_bar_mode 0, rupture_warmup 200, on_rupture 0, velocity 0. */
void flb_default_params(flb_params* p);

/* A gas nucleus: centre (cell centres at integer coordinates) and radius. */
typedef struct {
  double x, y, z, r;
} flb_nucleus;

typedef struct {
  double mass;       /* sum of rho over the lattice (FP64) */
  double mom[3];     /* sum of j (FP64) */
  int64_t step;      /* steps completed */
  int32_t n_bubbles; /* bubbles in the film maps of the last refresh (0 if film off) */
  int32_t n_ruptures;/* barrier removals so far */
  int32_t stopped;   /* 1 once the run stopped on a rupture (on_rupture == 1) */
  int32_t events_lost; /* rupture events beyond the log capacity */
} flb_stats;

/* Create a context: validates p, allocates device state through alloc (or
 * hipMalloc when alloc is NULL) and records hip_stream (a hipStream_t; NULL =
 * the null stream).  On success *out receives the context. */
int flb_create(const flb_params* p, const flb_allocator* alloc, void* hip_stream, flb_ctx** out);

/* Initial state (Sec. 2.1.3, "Random nucleation" of Fig. Mainflowchart):
 * rho = rho_gas in cells whose periodic minimum-image distance to some nucleus
 * centre is <= its radius, rho_liquid elsewhere, then rho += noise_amp (2U-1)
 * with U the top 53 bits of splitmix64(seed ^ (c * 0x9E3779B97F4A7C15)) / 2^53
 * for cell c; populations f_i = w_i rho.  nuc: n host records (n may be 0).
 * Resets the step counter, film maps, aliases and the rupture log. */
int flb_set_nuclei(flb_ctx* ctx, const flb_nucleus* nuc, int32_t n);

/* Advance nsteps >= 0 steps (asynchronous on the context stream).  Film maps
 * are rebuilt before each step n with n % k_own == 0.  After a rupture with
 * on_rupture == 1 the remaining steps are no-ops. */
int flb_step(flb_ctx* ctx, int64_t nsteps);

/* Density of the current state into host_out[n], n == nx*ny*nz (FP64). */
int flb_get_density(flb_ctx* ctx, double* host_out, size_t n);

/* Velocity of the current state into host_out[n], n == D*nx*ny*nz, component
 * planes (x plane, then y, then z for D3Q19); mode per params.velocity_mode. */
int flb_get_velocity(flb_ctx* ctx, double* host_out, size_t n);

/* Populations of the current state, host_out[n], n == Q*nx*ny*nz, population
 * planes in the order listed above (FP64 values of the stored precision). */
int flb_get_populations(flb_ctx* ctx, double* host_out, size_t n);

/* Replace the current state by host populations (same layout); rounds to the
 * storage precision.  Does not touch the step counter or the film maps. */
int flb_set_populations(flb_ctx* ctx, const double* host_in, size_t n);

/* FP64 totals of the current state and the run counters. */
int flb_get_stats(flb_ctx* ctx, flb_stats* out);

/* Canonical bubble labels of the current state: gas iff rho < rho_th,
 * periodic connected components over the lattice links (8 neighbours on
 * D2Q9, 18 on D3Q19); component k (1-based) is the one with the k-th smallest
 * minimum cell index; liquid cells are 0.  out[n], n == nx*ny*nz;
 * *n_bubbles receives the number of components.  (Bubble statistics of
 * Sec. 5, computed from the field as "domain gas points" of Sec. 2.1.3.) */
int flb_get_labels(flb_ctx* ctx, int32_t* out, size_t n, int32_t* n_bubbles);

/* The same labelling applied to a caller-given FP64 density field rho[n]. */
int flb_label_field(flb_ctx* ctx, const double* rho, size_t n, int32_t* out, int32_t* n_bubbles);

/* Film maps of the last refresh (film_on only), each array of n == nx*ny*nz:
 * labels, the smallest / largest label among the nearest bubbles (0 = none),
 * hop distance to them (-1 = beyond zone_width - 1), and the candidate
 * barrier-link mask (bit i = direction i).  Any pointer may be NULL. */
int flb_get_maps(flb_ctx* ctx, int32_t* label, int32_t* owner, int32_t* owner2, int32_t* dist, uint32_t* mask,
                 size_t n);

/* Bubble-size histogram of the current labels: equivalent diameter
 * 2 sqrt(A/pi) (D2Q9) or (6V/pi)^(1/3) (D3Q19) in lattice units, bin
 * floor(d / bin_width), last bin open-ended.  counts[nbins]. */
int flb_get_histogram(flb_ctx* ctx, int32_t nbins, double bin_width, int64_t* counts, int32_t* n_bubbles);

/* Rupture log: up to cap records of 3 x int64 (step, k, k2) with k < k2 the
 * labels of the film's two bubbles, in the order the device wrote them
 * (several records per step and pair are possible); *n receives the total
 * number written (it may exceed cap, and the device keeps at most 65536). */
int flb_get_rupture_events(flb_ctx* ctx, int64_t* out, int64_t cap, int64_t* n);

/* Tuning of the fused step kernel: tile variant index (0..n_tiles-1, -1 keeps
 * the current one), planes per workgroup segment lz >= 1 (0 keeps), and
 * xcd > 1 to place spatially adjacent tiles on one XCD (0 or 1: off; -1
 * keeps).  Results do not depend on the tuning. */
int flb_set_tuning(flb_ctx* ctx, int32_t tile, int32_t lz, int32_t xcd);
int flb_get_tuning(flb_ctx* ctx, int32_t* tile, int32_t* lz, int32_t* xcd, int32_t* n_tiles,
                   int32_t* tile_x, int32_t* tile_m);

/* Runs nsteps steps like flb_step, bracketed by HIP events on the context
 * stream, and returns the elapsed milliseconds in *ms.  With refresh == 0 the
 * film maps are not rebuilt (only the fused step kernel runs), which times
 * that kernel alone. */
int flb_time_steps(flb_ctx* ctx, int64_t nsteps, int32_t refresh, double* ms);

/* Destroys the context and frees its device state.  NULL is ignored. */
void flb_destroy(flb_ctx* ctx);

/* Message describing the last error on this thread ("" if none). */
const char* flb_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FOAMLBM_H */
