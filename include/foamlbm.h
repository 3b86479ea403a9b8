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
 * optionally the gas release of Sec. 2.1.3 (dp/dt = A (dn/dt) / N at each of
 * the N domain gas points, added as the density 3 A (dn/dt) / N after the
 * collision), optionally a body force (the forcing term of Sec. 2.1.1 for
 * gravity), and, on active barrier links from step rupture_warmup on, the FP64 test
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

/* Problem definition (the input, geometry and lattice boxes of
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
  int32_t k_own;         /* film maps are rebuilt before every step n with n % k_own == 0 (>= 1),
                            from the density refresh_src names */
  int32_t zone_width;    /* largest film thickness (lattice links) that carries a barrier, 1..15 */
  double rho_th;         /* gas iff rho < rho_th (default ln 2, the critical density) */
  int32_t psi_bar_mode;  /* psi on barrier links: 0 = psi(rho_liquid), 1 = psi(x) */
  int32_t rupture_warmup;/* first step at which the rupture test runs */
  int32_t on_rupture;    /* 0: remove the pair's barrier and continue; 1: stop after the step */
  int32_t velocity_mode; /* flb_get_velocity: 0 = j/rho, 1 = (j + F/2)/rho */
  int32_t rupture_filter; /* FP32/FP16S storage: 1 (default) skips the FP64
                             evaluation of the rupture test where an FP32
                             evaluation with a rigorous error bound already
                             proves the second difference negative; 0 always
                             evaluates in FP64.  Both take identical decisions. */
  int32_t refresh_src;   /* density a map refresh before step n labels (Sec. 2.1.5 evaluates
                            the bubbles continuously): 0 (default) = rho^n, the state entering
                            step n, formed by one pass over the populations; 1 = rho^(n-1), the
                            density that entered step n - 1, which that step's kernel stores
                            (no extra pass; the maps lag the state by one step; at n = 0 and
                            after the state was replaced, the current density) */
  int32_t growth_on;     /* 1: gas release (Sec. 2.1.3, the bubble-growth box of
                            Fig. Mainflowchart) at the domain gas points, the cells inside a
                            nucleus at flb_set_nuclei; each gains the density 3 dp per step,
                            dp = gas_A * gas_dndt / N for N gas points, as w_i 3 dp on
                            population i after the collision (mass, no momentum) */
  double gas_A;          /* A of the gas-release law dp/dt = A (dn/dt) / N, lattice units */
  double gas_dndt;       /* dn/dt of the gas-release law, lattice units per step */
  double f16_rho_ref;    /* FLB_F16S: population i is stored as FP16 of f_i - w_i f16_rho_ref
                            (default 1: f_i - w_i).  One FP16 rounding then costs about
                            2^-12 |rho - f16_rho_ref| / rho of f_i at density rho, so a value
                            between the phase densities (their harmonic mean balances the
                            relative error of both phases) suits two-phase runs; >= 0 */
  double gx, gy, gz;     /* gravity, lattice units (gz == 0 on D2Q9); all zero: no body force.
                            Added after the collision as the forcing term of Sec. 2.1.1:
                            F_i = w_i (rho - g_rho_ref) [(e_i - u).g / c_s^2 +
                            (e_i.u)(e_i.g) / c_s^4], u the velocity of the equilibrium;
                            it adds (rho - g_rho_ref) g of momentum and no mass per cell */
  double g_rho_ref;      /* reference density of the body force (the mean density gives
                            the buoyancy form, no net force on a periodic lattice) */
  int32_t model;         /* 0 (default): one lattice.  1: the two lattices of Sec. 2.1.5, melt
                            and gas, coupled every step: the fields above describe the melt
                            (its populations, tau, its own coupling G, rho_liquid / rho_gas
                            outside / inside the nuclei, the labels from its density); the
                            gas lattice has tau_g, its own coupling G_gg, the coupling G_mg to
                            the melt, and rho_g_liquid / rho_g_bubble outside / inside the
                            nuclei.  Each lattice feels F_s = -psi_s(x) sum_i w_i e_i sum_s'
                            G_ss' psi~_s'(x + e_i), with the bulk melt's values (psi_bar_mode 0)
                            or x's own (mode 1) across active barrier links, and relaxes to
                            the equilibrium at u' + tau_s F_s / rho_s, u' = (j_m / tau + j_g /
                            tau_g) / (rho_m / tau + rho_g / tau_g).  The rupture test uses the
                            pressure (rho_m + rho_g)/3 + (G psi_m^2 + 2 G_mg psi_m psi_g +
                            G_gg psi_g^2)/6.  Storage FLB_F64 or FLB_F32; the gas release
                            (growth_on) goes to the gas lattice; no body force; single
                            lattices only (not in batches or the server). */
  double G_mg;           /* model 1: melt-gas coupling (> 0 repels) */
  double G_gg;           /* model 1: the gas lattice's own coupling */
  double tau_g;          /* model 1: relaxation time of the gas lattice, > 0.5 */
  double rho_g_bubble;   /* model 1: initial gas density inside the nuclei, > 0 */
  double rho_g_liquid;   /* model 1: initial gas density in the melt, > 0 */
  int32_t open_z;        /* 1: the container of Sec. 5, open for the liquid: the first and last
                            planes across the last axis (z on D3Q19, y on D2Q9) face a reservoir
                            at rest, melt density rho_res (and, with model 1, gas density
                            rho_g_liquid).  A population that streams out through such a plane
                            leaves; one that streams in is the reservoir's w_i rho; neighbours
                            beyond the planes (force, rupture test, velocity query) are the
                            reservoir's.  The other axes stay periodic, and so do the film maps
                            (labels, owners, barriers).  Runs on the two-pass kernels; single
                            lattices only.  0 (default): periodic. */
  double rho_res;        /* open_z: reservoir (melt) density, > 0 */
} flb_params;

/* Fills p with defaults: D2Q9 F32 64x64x1, tau 1, G -5, rho0 1, rho_liquid 2,
 * rho_gas 0.15, noise 0.01, seed 1, film off, k_own 10, zone_width 6,
 * rho_th ln 2, psi_bar_mode 0, rupture_warmup 200, on_rupture 0, velocity 0,
 * rupture_filter 1, refresh_src 0, growth off (A = dn/dt = 0), f16_rho_ref 1, no gravity,
 * model 0 (two-lattice fields: G_mg 0.5, G_gg 0, tau_g 1, rho_g_bubble 0.5, rho_g_liquid 0.05),
 * open_z 0 (rho_res 2). */
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
  int32_t n_ruptures;/* barrier removals so far: unions of two bubble classes */
  int32_t stopped;   /* 1 once the run stopped on a rupture (on_rupture == 1) */
  int32_t events_lost; /* 1 if the rupture log filled up and later records were dropped */
} flb_stats;

/* Create a context: validates p, allocates device state through alloc (or
 * hipMalloc when alloc is NULL) and records hip_stream (a hipStream_t; NULL =
 * the null stream).  On success *out receives the context. */
int flb_create(const flb_params* p, const flb_allocator* alloc, void* hip_stream, flb_ctx** out);

/* Initial state (Sec. 2.1.3, the random-nucleation box of Fig. Mainflowchart):
 * rho = rho_gas in cells whose periodic minimum-image distance to some nucleus
 * centre is <= its radius, rho_liquid elsewhere, then rho += noise_amp (2U-1)
 * with U the top 53 bits of splitmix64(seed ^ (c * 0x9E3779B97F4A7C15)) / 2^53
 * for cell c; populations f_i = w_i rho.  nuc: n host records (n may be 0).
 * Resets the step counter, film maps, aliases and the rupture log. */
int flb_set_nuclei(flb_ctx* ctx, const flb_nucleus* nuc, int32_t n);

/* Advance nsteps >= 0 steps (asynchronous on the context stream).  Film maps
 * are rebuilt before each step n with n % k_own == 0 (from the density that
 * refresh_src names).  After a rupture with on_rupture == 1 the remaining
 * steps are no-ops. */
int flb_step(flb_ctx* ctx, int64_t nsteps);

/* Density of the current state into host_out[n], n == nx*ny*nz (FP64). */
int flb_get_density(flb_ctx* ctx, double* host_out, size_t n);

/* Velocity of the current state into host_out[n], n == D*nx*ny*nz, component
 * planes (x plane, then y, then z for D3Q19); mode per params.velocity_mode. */
int flb_get_velocity(flb_ctx* ctx, double* host_out, size_t n);

/* Bulk pressure p0 = rho/3 + (G/6) psi^2 (Eq. Pequ) of the current state
 * into host_out[n], n == nx*ny*nz (FP64): the pressure the paper plots across
 * a film (Sec. 4, Fig. plot) and whose second difference the rupture test
 * reads. */
int flb_get_pressure(flb_ctx* ctx, double* host_out, size_t n);

/* Domain gas points of the gas-release source (growth_on; the cells inside a
 * nucleus at the last flb_set_nuclei): out[n] receives 1 at a gas point, 0
 * elsewhere (n == nx*ny*nz; out may be NULL), *n_points their number N (0
 * with growth off). */
int flb_get_gas_points(flb_ctx* ctx, uint8_t* out, size_t n, int64_t* n_points);

/* Populations of the current state, host_out[n], n == Q*nx*ny*nz, population
 * planes in the order listed above (FP64 values of the stored precision).
 * With model 1, n == 2*Q*nx*ny*nz: the melt lattice's planes, then the gas's. */
int flb_get_populations(flb_ctx* ctx, double* host_out, size_t n);

/* Replace the current state by host populations (same layout); rounds to the
 * storage precision.  Does not touch the step counter or the film maps. */
int flb_set_populations(flb_ctx* ctx, const double* host_in, size_t n);

/* Model 1 (the two lattices of Sec. 2.1.5, the "Domain coupling" box of
 * Fig. Mainflowchart): density of the gas lattice, host_out[n], n ==
 * nx*ny*nz, FP64 sums of its stored populations.  flb_get_density gives the
 * melt lattice's, flb_get_velocity the mixture's (j_m + j_g [+ (F_m + F_g)/2])
 * / (rho_m + rho_g), flb_get_pressure the two-component pressure and
 * flb_get_stats the totals of both lattices.  FLB_EINVAL with model 0. */
int flb_get_gas_density(flb_ctx* ctx, double* host_out, size_t n);

/* FP64 totals of the current state and the run counters. */
int flb_get_stats(flb_ctx* ctx, flb_stats* out);

/* Canonical bubble labels of the current state: gas iff rho < rho_th,
 * periodic connected components over the lattice links (8 neighbours on
 * D2Q9, 18 on D3Q19); component k (1-based) is the one with the k-th smallest
 * minimum cell index; liquid cells are 0.  out[n], n == nx*ny*nz;
 * *n_bubbles receives the number of components.  (Bubble statistics of
 * Sec. 5, computed from the field as the gas points of the domain, Sec. 2.1.3.) */
int flb_get_labels(flb_ctx* ctx, int32_t* out, size_t n, int32_t* n_bubbles);

/* The same labelling applied to a caller-given FP64 density field rho[n]. */
int flb_label_field(flb_ctx* ctx, const double* rho, size_t n, int32_t* out, int32_t* n_bubbles);

/* Film maps of the last refresh (film_on only), each array of n == nx*ny*nz:
 * labels, the smallest / largest label among the nearest bubbles (0 = none),
 * hop distance to them (-1 = beyond zone_width - 1), and the barrier-link
 * mask (bit i = direction i): the links built at the refresh, minus those
 * whose two bubbles a rupture has united since.  Any pointer may be NULL. */
int flb_get_maps(flb_ctx* ctx, int32_t* label, int32_t* owner, int32_t* owner2, int32_t* dist, uint32_t* mask,
                 size_t n);

/* Bubble-size histogram of the current labels: equivalent diameter
 * 2 sqrt(A/pi) (D2Q9) or (6V/pi)^(1/3) (D3Q19) in lattice units, bin
 * floor(d / bin_width), last bin open-ended.  counts[nbins]. */
int flb_get_histogram(flb_ctx* ctx, int32_t nbins, double bin_width, int64_t* counts, int32_t* n_bubbles);
/* Foam statistics of the current labels, the quantities the paper reads off
 * its virtual metallography (Sec. 5, Table 5 and Fig. 14): the bubble cell
 * fraction (bubble percentage), the relative foam density 1 - fraction
 * (Table 5's foam density is the melt density times it), and the mean and
 * largest equivalent diameter (2 sqrt(A/pi) on D2Q9, (6V/pi)^(1/3) on D3Q19,
 * lattice units; 0 without bubbles).  Sums run in a fixed order on the
 * device, so results do not depend on timing.  Synchronises the stream. */
typedef struct {
  int32_t n_bubbles;
  int64_t gas_cells;
  double gas_fraction;
  double relative_density;
  double mean_diameter;
  double max_diameter;
} flb_foam_stats;
int flb_get_foam_stats(flb_ctx* ctx, flb_foam_stats* out);

/* flb_get_histogram for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same result, computed without any hipMalloc, hipFree or
 * allocator call.  The bins live in a device array the library holds on
 * every GPU it runs on until the process ends (512 KiB), so nbins must be in
 * 1..65536 (FLB_EINVAL beyond).  All contexts on one GPU share that array and
 * each call clears it first: calls on one GPU that overlap in time (from
 * several threads or streams) race and must be serialised by the caller.
 * Synchronises the context stream. */
int flb_get_histogram_noalloc(flb_ctx* ctx, int32_t nbins, double bin_width, int64_t* counts, int32_t* n_bubbles);

/* Overlap of an earlier bubble labelling with the current one, for tracking
 * coalescence between snapshots (the bubble statistics of Sec. 5 taken over
 * time).  old_labels: n == nx*ny*nz labels (x fastest, 0 = liquid) as
 * flb_get_labels returned them earlier; the current labels are those
 * flb_get_labels would return now (*n_bubbles receives their count).  For
 * every pair (old bubble a, current bubble b) that share at least one cell,
 * pairs[3k .. 3k+2] = (a, b, shared cells), sorted by (a, b); up to cap pairs
 * are written and *n_pairs is their total (call again with cap >= *n_pairs for
 * all of them).  A current bubble paired with two or more old ones is a
 * coalescence; an old one paired with two or more current ones split.
 * FLB_EINVAL on a negative label.  Synchronises the stream. */
int flb_match_labels(flb_ctx* ctx, const int32_t* old_labels, size_t n, int64_t* pairs, int64_t cap,
                     int64_t* n_pairs, int32_t* n_bubbles);

/* Rupture log: up to cap records of 3 x int64 (step, k, k2), k < k2: a
 * barrier link between bubbles k and k2 (labels of the refresh in force) met
 * the criterion in that step.  Records come in device order; one pair may
 * appear several times in a step.  *n receives the number of records kept
 * (the device keeps the first 65536; flb_stats.events_lost says whether later
 * ones were dropped).  The unions a record asks for are applied whether or
 * not it was kept. */
int flb_get_rupture_events(flb_ctx* ctx, int64_t* out, int64_t cap, int64_t* n);

/* Tuning of the fused step kernel: tile variant index (0..n_tiles-1, -1 keeps
 * the current one), planes per workgroup segment lz >= 1 (0 keeps), and
 * xcd > 1 to place spatially adjacent tiles on one XCD (0 or 1: off; -1
 * keeps).  Results do not depend on the tuning.  Variants, in index order:
 * D2Q9 z-march tiles 64, 128 and 256 cells wide, flat tiles of 64 cells x 8
 * and x 16 rows (their segment is their height; lz is kept but unused), the
 * two-pass path; D3Q19 z-march tiles 64x4, 64x8, 32x8, 128x4, the two-pass
 * path.  tile_x / tile_m report the tile's cells along x and m (0 for the
 * two-pass path). */
int flb_set_tuning(flb_ctx* ctx, int32_t tile, int32_t lz, int32_t xcd);
int flb_get_tuning(flb_ctx* ctx, int32_t* tile, int32_t* lz, int32_t* xcd, int32_t* n_tiles,
                   int32_t* tile_x, int32_t* tile_m);

/* Autotuner: times `reps` launches of the step kernel(s) for every tile
 * variant, segment length and XCD setting, keeps the fastest and returns its
 * time per step in *best_ms (may be NULL).  The state is not changed: each
 * trial reads the current populations and writes a scratch buffer (one
 * population buffer, allocated while it runs) under a copy of the run
 * control. */
int flb_autotune(flb_ctx* ctx, int32_t reps, double* best_ms);

/* Runs nsteps steps like flb_step, bracketed by HIP events on the context
 * stream, and returns the elapsed milliseconds in *ms.  With refresh == 0 the
 * film maps are not rebuilt, so only the step kernel(s) and the small
 * per-step finisher run.  If kernel_ms is not NULL, every step-kernel launch
 * (the fused kernel, or both passes of the two-pass variant) is also
 * bracketed by its own pair of events and *kernel_ms receives the sum of
 * those durations, i.e. the time of the step kernel alone. */
int flb_time_steps(flb_ctx* ctx, int64_t nsteps, int32_t refresh, double* ms, double* kernel_ms);

/* Runs nsteps (0..100000) steps like flb_step and times every phase of each
 * step with HIP events on the context stream: *ms = elapsed milliseconds,
 * phase_ms[0] = map refreshes, [1] = step kernel(s), [2] = rupture test and
 * mask pruning, [3] = the per-step finisher (sums over the steps). */
int flb_time_phases(flb_ctx* ctx, int64_t nsteps, double* ms, double* phase_ms);

/* Device-copy bandwidth: copies `bytes` (a multiple of 16 in 2^20..2^36)
 * between two buffers from alloc (NULL: hipMalloc) with 16-byte accesses per
 * lane, four loads in flight, non-temporal stores, on hip_stream, `reps`
 * times per grid size, and returns the best read + write rate in *gbs
 * (GB/s): the practical HBM ceiling of a kernel that reads and writes equal
 * amounts.  The buffers are freed before return. */
int flb_copy_bandwidth(const flb_allocator* alloc, void* hip_stream, int64_t bytes, int32_t reps, double* gbs);

/* Checkpoint and resume: flb_save writes the current state (populations,
 * run control, film maps, aliases, rupture log) to a file; flb_load restores
 * it into a context created with identical parameters, after which stepping
 * continues exactly as it would have from the saved point. */
int flb_save(flb_ctx* ctx, const char* path);
int flb_load(flb_ctx* ctx, const char* path);

/* Replaces the film maps in force (film_on only) by given ones, as if a
 * refresh had built them: labels, owner / owner2 (0 = none), dist (-1 =
 * beyond zone_width - 1), each of n == nx*ny*nz cells, the alias root of
 * every label 0..n_bubbles (NULL: every label its own root), and n_bubbles;
 * masks and the flagged-cell list are rebuilt from them.  The next regular
 * refresh replaces them again.  Lets two implementations run step-locked on
 * identical maps (parity tests beyond the horizon where independently
 * computed maps may differ).  FLB_EINVAL on inconsistent maps. */
int flb_import_maps(flb_ctx* ctx, const int32_t* label, const int32_t* owner, const int32_t* owner2,
                    const int32_t* dist, size_t n, const int32_t* alias_root, int32_t n_bubbles);

/* Destroys the context and frees its device state.  NULL, and a context
 * owned by a batch (see flb_batch_member), are ignored. */
void flb_destroy(flb_ctx* ctx);

/* ---- Batches: many lattices advanced together ----------------------------
 * A batch holds `count` member lattices of one lattice type and one storage
 * format; every other parameter (extents, tau, G, film settings, seed, ...)
 * may differ per member (params[k]).  A batch step advances every member by
 * one time step exactly as flb_step would, with one batched step-kernel
 * launch over all members' workgroups and one batched finisher launch (when
 * members have films: one batched rupture-test launch and one batched launch
 * that prunes the masks and runs the finishers; film maps are refreshed in
 * batched launches over the members that are due).  Runs of steps are captured in
 * a HIP graph and replayed when the stream is not the null stream.  Results
 * of a member do not depend on the batch it is in.
 *
 * Members are contexts owned by the batch: flb_batch_member returns a
 * borrowed handle on which every flb_get_* query, flb_set_nuclei,
 * flb_set_populations and flb_step work; flb_destroy ignores it, and
 * flb_batch_destroy frees all members. */
typedef struct flb_batch flb_batch;

int flb_batch_create(const flb_params* params, int32_t count, const flb_allocator* alloc, void* hip_stream,
                     flb_batch** out);
int flb_batch_size(flb_batch* batch, int32_t* count);
int flb_batch_member(flb_batch* batch, int32_t k, flb_ctx** out);
/* Advances every member by nsteps steps (asynchronous, like flb_step). */
int flb_batch_step(flb_batch* batch, int64_t nsteps);
/* Batch tuning: z-march or flat tile variant shared by the members (-1 keeps; the
 * two-pass variant has no batched form), the total workgroup target of a step
 * launch that sets each member's segment length in proportion to its cells
 * (0 keeps), the XCD remap (-1 keeps) and the steps per captured graph
 * (0: no graphs, -1 keeps).  Results do not depend on the tuning. */
int flb_batch_set_tuning(flb_batch* batch, int32_t tile, int64_t target, int32_t xcd, int32_t graph_steps);
int flb_batch_get_tuning(flb_batch* batch, int32_t* tile, int64_t* target, int32_t* xcd, int32_t* graph_steps,
                         int32_t* n_tiles);
/* Persistent runs (D2Q9 batches only; EINVAL for D3Q19).  With on = 1 each
 * stretch of steps between film-map refreshes, of at most max_steps steps
 * (0 keeps; default 1024), is one cooperative launch whose workgroups, as
 * many as are resident at once, take the step tiles of all members in turn,
 * then the rupture test, the mask pruning and the finisher of every member,
 * with a grid-wide barrier between those phases of each step; the refreshes
 * stay launches of their own before the stretch.  The batch then uses the
 * 256 x 1 tile (flb_batch_set_tuning rejects another).  Populations, maps
 * and events equal those of the per-step launches bit for bit; the FP64
 * mass and momentum totals are summed in another order (equal to rounding).
 * on = 0 returns to per-step launches and graph replay.  Fails with EINVAL
 * when the device has no cooperative launches (at the next step). */
int flb_batch_set_persistent(flb_batch* batch, int32_t on, int32_t max_steps);
/* Autotuner: times `reps` launches of the batched step kernel for every tile
 * variant, workgroup target and XCD setting without changing any member
 * (each trial writes a scratch buffer under a copy of the run control),
 * keeps the fastest, and returns its time per launch in *best_ms (may be
 * NULL).  Allocates one scratch population buffer per member while it runs. */
int flb_batch_autotune(flb_batch* batch, int32_t reps, double* best_ms);
/* Runs nsteps batch steps bracketed by HIP events; *ms = elapsed time. */
int flb_batch_time_steps(flb_batch* batch, int64_t nsteps, double* ms);
void flb_batch_destroy(flb_batch* batch);

/* ---- Server: resident foam jobs advanced together -------------------------
 * Jobs (a parameter set, nuclei and a step count) queue in submission order.
 * Each flb_server_pump is one scheduling round: it admits queued jobs, in
 * order, while the device bytes of all admitted jobs stay within
 * pool_bytes and fewer than max_jobs are resident (a job that does not fit
 * waits, and so do the jobs behind it); it picks the resident jobs to
 * advance -- FLB_SERVE_FIFO: all of them, and admission also stops once the
 * resident jobs would hold more than max_cells lattice cells (a larger job
 * runs once nothing else does); FLB_SERVE_SHORTEST: those with the least
 * remaining work (cells x steps left) while their cells stay within
 * max_cells (at least one; a job passed over 8 rounds in a row goes first)
 * -- and advances them by the same number of steps, chunk_steps or fewer so
 * that no job passes its last step, with batched launches (one batch per lattice type and storage, runs
 * of graph_steps steps replayed from captured HIP graphs); and it retires the
 * jobs that are done: their final density and statistics are copied to host
 * memory and their device memory is released.  The round synchronises the
 * stream before it returns.  A job's results are exactly those of the same
 * job run alone with flb_create / flb_set_nuclei / flb_step.
 * Failure handling: after its launches each round reads, for every job it
 * advanced, the flag that the step kernel's mass reduction sets on a
 * non-finite value, and retires such a job at once as FLB_JOB_FAILED (its
 * device memory released, no results; flb_server_result then returns
 * FLB_ENUMERIC); a job that could not be created on admission fails the same
 * way with the creation error.  No launch mixes the fields of two jobs, so a
 * failed job leaves the others' results unchanged. */
typedef struct flb_server flb_server;
typedef struct {
  int64_t pool_bytes;  /* device bytes the resident jobs may hold together */
  int32_t max_jobs;    /* resident jobs at most */
  int32_t chunk_steps; /* steps per round at most */
  int32_t graph_steps; /* steps per captured graph (0: no graphs) */
  int64_t max_cells;   /* lattice cells of the running jobs at most: enough
                          to fill the GPU; more only lengthens every job */
  int32_t policy;      /* FLB_SERVE_FIFO or FLB_SERVE_SHORTEST */
} flb_server_config;
enum { FLB_SERVE_FIFO = 0, FLB_SERVE_SHORTEST = 1 };
enum { FLB_JOB_QUEUED = 0, FLB_JOB_RUNNING = 1, FLB_JOB_DONE = 2, FLB_JOB_FAILED = 3, FLB_JOB_CANCELLED = 4 };

/* pool 64 GiB, 256 jobs, chunks of 100 steps, graphs of 20 steps, 2^22 cells,
 * FLB_SERVE_FIFO */
void flb_server_default_config(flb_server_config* cfg);
int flb_server_create(const flb_server_config* cfg, const flb_allocator* alloc, void* hip_stream,
                      flb_server** out);
/* Queues a job; *id receives its handle.  FLB_EBUSY if the job alone needs
 * more device bytes than the pool (it could never be admitted). */
int flb_server_submit(flb_server* srv, const flb_params* p, const flb_nucleus* nuclei, int32_t n, int64_t steps,
                      int64_t* id);
/* One scheduling round (see above).  *n_done counts the jobs that have left
 * the server: done, failed or cancelled.  Any output pointer may be NULL. */
int flb_server_pump(flb_server* srv, int32_t* n_running, int32_t* n_queued, int64_t* n_done);
int flb_server_job(flb_server* srv, int64_t id, int32_t* state, int64_t* steps_done);
/* Final density (n == nx*ny*nz, x fastest) and statistics of a done job. */
int flb_server_result(flb_server* srv, int64_t id, double* density, size_t n, flb_stats* stats);
/* Forgets a done, failed or cancelled job. */
int flb_server_release(flb_server* srv, int64_t id);
/* Cancels a queued or running job between rounds: a queued job leaves the
 * queue, a running one has its device memory released at once (the stream is
 * synchronised first).  The job ends as FLB_JOB_CANCELLED, without results.
 * FLB_EINVAL for an unknown job or one that has already finished. */
int flb_server_cancel(flb_server* srv, int64_t id);
int flb_server_usage(flb_server* srv, int64_t* used_bytes, int64_t* pool_bytes);
void flb_server_destroy(flb_server* srv);

/* Message describing the last error on this thread ("" if none). */
const char* flb_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FOAMLBM_H */
