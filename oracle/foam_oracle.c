/*
 * foam_oracle.c -- plain FP64 CPU oracle for the single-component Shan-Chen
 * lattice-Boltzmann foam step with the inter-bubble film barrier and the
 * pressure-second-derivative rupture criterion of Barzegari, Bayani,
 * Mirbagheri and Shetabivash, "Multiphase Aluminum A356 Foam Formation
 * Process Simulation Using Lattice Boltzmann Method" (arXiv:1708.01613).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference the GPU library is checked against.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or generator with the HIP library.
 *
 * Everything is FP64, written as plain loops in the order the method states
 * it.  Per step n, with f^n the post-streaming populations:
 *   1. moments        rho = sum_i f_i, j = sum_i e_i f_i        (Sec. 2.1.1, Eq. vel_dens)
 *   2. pseudopotential psi = rho0 (1 - exp(-rho/rho0))          (Sec. 2.1.2, Eq. pseudopotential)
 *   3. film maps (every k_own steps): labels, owner/dist, barrier links,
 *      alias carry                                              (Sec. 2.1.5, Fig. shanchenflowchart)
 *   4. force          F = -G psi(x) sum_i w_i psi~(x+e_i) e_i    (Sec. 2.1.2, Eq. shanchen3)
 *   5. velocity shift u_eq = (j + tau F) / rho                  (Sec. 2.1.5, final-velocity equations, read with /rho)
 *   6. BGK collision  f* = f - (f - f^eq(rho, u_eq)) / tau       (Sec. 2.1.1, collision equation; f^eq equation)
 *   6b. bubble growth (optional) the gas-release law dp/dt = A (dn/dt) / N at
 *                     each of the N domain gas points             (Sec. 2.1.3, Fig. Mainflowchart "Bubble growth")
 *   6c. body force (optional) the forcing term F_i of gravity     (Sec. 2.1.1, forcing equation)
 *   7. streaming      f_i(x + e_i) = f*_i(x), periodic; with open_z the
 *                     last axis is open to a liquid reservoir       (Sec. 2.1.1, streaming equation; Sec. 5, the
 *                                                                    container open for the liquid)
 *   8. rupture test   d2 p0 / dn2 >= 0 on barrier links          (Sec. 2.1.5, eta_m equation; Sec. 4)
 *
 * With model = 1 the step is the paper's two-lattice form (Sec. 2.1.5, the
 * two separate lattices for melt and gas, coupled at the end of every step;
 * Fig. Mainflowchart "Domain coupling"): one population set per component,
 * a common velocity, a Shan-Chen force on each component from both
 * components, and the per-bubble selection taken as the nearest-bubble
 * substitution on barrier links.  It is one_step_tl below, step by step.
 *
 * Readings of passages the paper leaves silent or garbled are named where
 * they are used (R-numbers match the table of readings kept with the design
 * notes).  No part of this file is tuned for speed beyond an OpenMP pragma on
 * the independent per-cell loops; reductions are serial in index order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAXQ 19
/* lattices smaller than this run their per-cell loops on one thread: there
   the start-up cost of a parallel region exceeds the loop */
#define OR_OMP_MIN_CELLS 32768

/* ------------------------------------------------------------------ */
/* Lattices.                                                           */
/* D2Q9: Sec. 2.1.1 (velocity and weight equations): rest, 4 axes with  */
/* weight 1/9, 4 diagonals with weight 1/36.                            */
/* D3Q19 is not printed in the paper; it is the textbook lattice: rest  */
/* 1/3, 6 axes 1/18, 12 face diagonals 1/36 (c_s^2 = 1/3 as in D2Q9).   */
/* ------------------------------------------------------------------ */
static const int OR_E2[9][3] = {
    {0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {-1, 0, 0}, {0, -1, 0},
    {1, 1, 0}, {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
static const double OR_W2[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                                1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

static const int OR_E3[19][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
static const double OR_W3[19] = {
    1.0 / 3,
    1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18, 1.0 / 18,
    1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36,
    1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

/* Parameters.  Field meaning follows the boundary of the GPU library, but   */
/* the struct is declared here on its own (the oracle includes no product    */
/* header).                                                                  */
typedef struct {
  int32_t lattice; /* 0 = D2Q9, 1 = D3Q19 */
  int32_t nx, ny, nz;
  double tau, G, rho0;
  double rho_liquid, rho_gas, noise_amp;
  uint64_t seed;
  int32_t film_on;
  int32_t k_own;
  int32_t zone_width;
  double rho_th;
  int32_t psi_bar_mode;   /* 0: psi(rho_liquid); 1: psi(x) */
  int32_t rupture_warmup; /* first step at which the rupture test runs */
  int32_t on_rupture;     /* 0: remove pair barrier; 1: stop after the step */
  int32_t velocity_mode;  /* 0: j/rho; 1: (j + F/2)/rho */
  int32_t refresh_src;    /* film maps label 0: rho^n, the state entering step n (default);
                             1: rho^(n-1), the state entering the previous step */
  int32_t growth_on;      /* 1: gas release at the domain gas points (Sec. 2.1.3) */
  double gas_A;           /* A of the gas-release law (lattice units) */
  double gas_dndt;        /* dn/dt of the gas-release law (lattice units, per step) */
  double gx, gy, gz;      /* gravity (lattice units); all zero: no body force */
  double g_rho_ref;       /* the body force is (rho - g_rho_ref) g per cell */
  int32_t model;          /* 0: single component; 1: two lattices, melt and gas (Sec. 2.1.5) */
  double G_mg;            /* model 1: melt-gas coupling (G is the melt's own) */
  double G_gg;            /* model 1: the gas's own coupling */
  double tau_g;           /* model 1: relaxation time of the gas lattice */
  double rho_g_bubble;    /* model 1: gas density inside the nuclei */
  double rho_g_liquid;    /* model 1: gas density in the melt */
  int32_t open_z;         /* 1: the first and last planes of the last axis (z on D3Q19, y on D2Q9) */
                          /* are open to a liquid reservoir at rest at density rho_res (R35) */
  double rho_res;         /* density of that reservoir */
} or_params;

typedef struct {
  or_params p;
  int Q, D;
  const int (*e)[3];
  const double* w;
  int opp[OR_MAXQ];
  long N;
  double* f;     /* populations f[i*N + c], post-streaming state f^n */
  double* fpost; /* post-collision scratch */
  double* rho;
  double* rho_prev; /* density of the state that entered the last step */
  int32_t have_prev; /* rho_prev holds it (cleared when the state is replaced) */
  double* psi;
  double* force; /* 3*N, last computed force */
  /* film maps (as of the last refresh) */
  int32_t* label;     /* canonical labels, 0 = liquid */
  int32_t* label_old; /* labels of the previous refresh */
  int32_t* owner;     /* smallest label among the nearest bubbles, 0 = none */
  int32_t* owner2;    /* largest label among the nearest bubbles (== owner unless tied) */
  int32_t* dist;      /* hop distance to owner's gas, -1 = none */
  uint32_t* mask;     /* barrier-link bit mask (bit i = link i) */
  int32_t nb, nb_old;
  int32_t* alias;     /* union-find parents over labels 0..nb */
  int32_t* alias_old;
  int32_t maps_valid;
  /* rupture events: (step, k, k2) triples */
  int64_t* ev;
  long nev, evcap;
  int64_t n_ruptures;
  int64_t step;
  int32_t stopped;
  /* domain gas points: the cells of the nuclei (Sec. 2.1.3), set at nucleation */
  unsigned char* src;
  long n_src;
  /* model 1: the gas lattice (populations g[i*N + c]), its moments and force */
  double* g;
  double* gpost;
  double* rho_g;
  double* psi_g;
  double* force_g;
} or_sim;

/* ------------------------------------------------------------------ */
/* small helpers                                                       */
/* ------------------------------------------------------------------ */
static long wrap(long a, long n) {
  long r = a % n;
  return r < 0 ? r + n : r;
}

static long nbr(const or_sim* s, long c, int i, int sign) {
  long nx = s->p.nx, ny = s->p.ny, nz = s->p.nz;
  long x = c % nx, y = (c / nx) % ny, z = c / (nx * ny);
  x = wrap(x + sign * s->e[i][0], nx);
  y = wrap(y + sign * s->e[i][1], ny);
  z = wrap(z + sign * s->e[i][2], nz);
  return x + nx * (y + ny * z);
}

/* With open_z (R35): whether the neighbour of c along sign * e_i lies      */
/* beyond an open plane (outside the container, in the reservoir).          */
static int beyond_open(const or_sim* s, long c, int i, int sign) {
  if (!s->p.open_z) return 0;
  const int ax = s->D == 2 ? 1 : 2;
  const long n = ax == 1 ? s->p.ny : s->p.nz;
  const long k = ax == 1 ? (c / s->p.nx) % s->p.ny : c / ((long)s->p.nx * s->p.ny);
  const long t = k + sign * s->e[i][ax];
  return t < 0 || t >= n;
}

static double psi_of(const or_params* p, double rho) {
  /* Sec. 2.1.2, Eq. pseudopotential, generalised to rho0 (1 - e^{-rho/rho0}). */
  return p->rho0 * (1.0 - exp(-rho / p->rho0));
}

/* OpenMP threads the loops of this file use (1 without OpenMP). */
int or_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Sets the OpenMP threads of later loops (no-op without OpenMP). */
void or_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

double or_p0(double rho, double G, double rho0) {
  /* Bulk equation of state p = rho c_s^2 + (G/6) psi^2 (Sec. 2.1.2, Eq. Pequ;
   * the same expression is the interaction potential xi of Sec. 2.1.5). */
  double psi = rho0 * (1.0 - exp(-rho / rho0));
  return rho / 3.0 + G / 6.0 * psi * psi;
}

/* Vigna's SplitMix64 output function applied to one 64-bit state. */
uint64_t or_splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* Uniform in [0,1) for cell index idx: top 53 bits of the hash. */
double or_uniform(uint64_t seed, uint64_t idx) {
  uint64_t h = or_splitmix64(seed ^ (idx * 0x9E3779B97F4A7C15ULL));
  return (double)(h >> 11) * (1.0 / 9007199254740992.0);
}

/* union-find with the smaller index as root */
static int32_t uf_find(int32_t* par, int32_t a) {
  while (par[a] != a) a = par[a];
  return a;
}
static int uf_union(int32_t* par, int32_t a, int32_t b) {
  int32_t ra = uf_find(par, a), rb = uf_find(par, b);
  if (ra == rb) return 0;
  if (ra < rb) par[rb] = ra; else par[ra] = rb;
  return 1;
}

/* ------------------------------------------------------------------ */
/* creation                                                            */
/* ------------------------------------------------------------------ */
void or_destroy(or_sim* s);

or_sim* or_create(const or_params* p) {
  if (p->lattice != 0 && p->lattice != 1) return NULL;
  if (p->nx < 1 || p->ny < 1 || p->nz < 1) return NULL;
  if (p->lattice == 0 && p->nz != 1) return NULL;
  if (!(p->tau > 0.5)) return NULL;
  if (p->model != 0 && p->model != 1) return NULL;
  if (p->open_z != 0 && p->open_z != 1) return NULL;
  if (p->open_z && !(p->rho_res > 0.0)) return NULL;
  /* the two-lattice model carries no body force (its gas release goes to the gas lattice) */
  if (p->model == 1 && (!(p->tau_g > 0.5) || p->gx != 0.0 || p->gy != 0.0 || p->gz != 0.0 ||
                        !(p->rho_g_bubble > 0.0) || !(p->rho_g_liquid > 0.0)))
    return NULL;
  or_sim* s = (or_sim*)calloc(1, sizeof(or_sim));
  s->p = *p;
  if (s->p.k_own < 1) s->p.k_own = 1;
  if (p->lattice == 0) {
    s->Q = 9; s->D = 2; s->e = OR_E2; s->w = OR_W2;
  } else {
    s->Q = 19; s->D = 3; s->e = OR_E3; s->w = OR_W3;
  }
  for (int i = 0; i < s->Q; i++)
    for (int j = 0; j < s->Q; j++)
      if (s->e[j][0] == -s->e[i][0] && s->e[j][1] == -s->e[i][1] && s->e[j][2] == -s->e[i][2])
        s->opp[i] = j;
  s->N = (long)p->nx * p->ny * p->nz;
  long N = s->N;
  s->f = (double*)calloc((size_t)s->Q * N, sizeof(double));
  s->fpost = (double*)calloc((size_t)s->Q * N, sizeof(double));
  s->rho = (double*)calloc(N, sizeof(double));
  s->rho_prev = (double*)calloc(N, sizeof(double));
  s->psi = (double*)calloc(N, sizeof(double));
  s->force = (double*)calloc(3 * (size_t)N, sizeof(double));
  s->label = (int32_t*)calloc(N, sizeof(int32_t));
  s->label_old = (int32_t*)calloc(N, sizeof(int32_t));
  s->owner = (int32_t*)calloc(N, sizeof(int32_t));
  s->owner2 = (int32_t*)calloc(N, sizeof(int32_t));
  s->dist = (int32_t*)calloc(N, sizeof(int32_t));
  s->mask = (uint32_t*)calloc(N, sizeof(uint32_t));
  s->alias = (int32_t*)calloc(N + 2, sizeof(int32_t));
  s->alias_old = (int32_t*)calloc(N + 2, sizeof(int32_t));
  s->src = (unsigned char*)calloc(N, 1);
  s->evcap = 1024;
  s->ev = (int64_t*)calloc(3 * (size_t)s->evcap, sizeof(int64_t));
  if (!s->f || !s->fpost || !s->rho || !s->rho_prev || !s->psi || !s->force || !s->label || !s->label_old ||
      !s->owner || !s->owner2 || !s->dist || !s->mask || !s->alias || !s->alias_old || !s->src || !s->ev) {
    or_destroy(s);
    return NULL;
  }
  for (long c = 0; c < N; c++) s->dist[c] = -1;
  if (p->model == 1) {
    s->g = (double*)calloc((size_t)s->Q * N, sizeof(double));
    s->gpost = (double*)calloc((size_t)s->Q * N, sizeof(double));
    s->rho_g = (double*)calloc(N, sizeof(double));
    s->psi_g = (double*)calloc(N, sizeof(double));
    s->force_g = (double*)calloc(3 * (size_t)N, sizeof(double));
    if (!s->g || !s->gpost || !s->rho_g || !s->psi_g || !s->force_g) {
      or_destroy(s);
      return NULL;
    }
  }
  return s;
}

void or_destroy(or_sim* s) {
  if (!s) return;
  free(s->f); free(s->fpost); free(s->rho); free(s->rho_prev); free(s->psi); free(s->force);
  free(s->label); free(s->label_old); free(s->owner); free(s->owner2); free(s->dist); free(s->mask);
  free(s->alias); free(s->alias_old); free(s->src); free(s->ev);
  free(s->g); free(s->gpost); free(s->rho_g); free(s->psi_g); free(s->force_g);
  free(s);
}

int or_Q(const or_sim* s) { return s->Q; }
long or_N(const or_sim* s) { return s->N; }
int64_t or_step_count(const or_sim* s) { return s->step; }
int32_t or_stopped(const or_sim* s) { return s->stopped; }

/* lattice tables, for tests */
void or_lattice(int lattice, int32_t* e_out, double* w_out) {
  int Q = lattice == 0 ? 9 : 19;
  for (int i = 0; i < Q; i++) {
    for (int k = 0; k < 3; k++) e_out[3 * i + k] = lattice == 0 ? OR_E2[i][k] : OR_E3[i][k];
    w_out[i] = lattice == 0 ? OR_W2[i] : OR_W3[i];
  }
}

/* ------------------------------------------------------------------ */
/* initial state: random nucleation at gas points of the domain (Sec. 2.1.3) */
/* rho = rho_gas inside any nucleus (periodic minimum image, cell      */
/* centres at integer coordinates), rho_liquid elsewhere, plus seeded  */
/* uniform noise; populations at rest equilibrium f_i = w_i rho.       */
/* ------------------------------------------------------------------ */
static double min_image(double d, long n) { return d - (double)n * floor(d / (double)n + 0.5); }

static int in_nucleus(const or_params* p, long x, long y, long z, const double* nk) {
  double dx = min_image((double)x - nk[0], p->nx);
  double dy = min_image((double)y - nk[1], p->ny);
  double dz = min_image((double)z - nk[2], p->nz);
  return dx * dx + dy * dy + dz * dz <= nk[3] * nk[3];
}

/* integer coordinates k with |k - c| <= r, as a range [*k0, *k1] of at most n */
static void box_range(double c, double r, long n, long* k0, long* k1) {
  *k0 = (long)ceil(c - r);
  *k1 = (long)floor(c + r);
  if (*k1 - *k0 + 1 > n) {
    *k0 = 0;
    *k1 = n - 1;
  }
}

int or_set_nuclei(or_sim* s, const double* nuc, int32_t n) {
  const or_params* p = &s->p;
  long N = s->N;
  /* a cell inside a nucleus has minimum-image offsets of at most r on every
     axis, so it lies in the nucleus' bounding box taken modulo the lattice:
     testing the cells of each box finds every inside cell */
  unsigned char* inside = (unsigned char*)calloc((size_t)N, 1);
  if (!inside) return -1;
  for (int k = 0; k < n; k++) {
    const double* nk = nuc + 4 * k;
    long x0, x1, y0, y1, z0, z1;
    box_range(nk[0], nk[3], p->nx, &x0, &x1);
    box_range(nk[1], nk[3], p->ny, &y0, &y1);
    box_range(nk[2], nk[3], p->nz, &z0, &z1);
    for (long zz = z0; zz <= z1; zz++)
      for (long yy = y0; yy <= y1; yy++)
        for (long xx = x0; xx <= x1; xx++) {
          long x = wrap(xx, p->nx), y = wrap(yy, p->ny), z = wrap(zz, p->nz);
          if (in_nucleus(p, x, y, z, nk)) inside[(z * p->ny + y) * p->nx + x] = 1;
        }
  }
#pragma omp parallel for schedule(static) if (N >= OR_OMP_MIN_CELLS)
  for (long c = 0; c < N; c++) {
    double rho = inside[c] ? p->rho_gas : p->rho_liquid;
    rho += p->noise_amp * (2.0 * or_uniform(p->seed, (uint64_t)c) - 1.0);
    for (int i = 0; i < s->Q; i++) s->f[(long)i * N + c] = s->w[i] * rho;
    /* model 1: the gas lattice holds rho_g_bubble in the nuclei and the */
    /* dissolved rho_g_liquid in the melt, at rest, without noise        */
    if (p->model == 1) {
      double rg = inside[c] ? p->rho_g_bubble : p->rho_g_liquid;
      for (int i = 0; i < s->Q; i++) s->g[(long)i * N + c] = s->w[i] * rg;
    }
  }
  /* the nucleus cells are the domain gas points that release gas (Sec. 2.1.3) */
  s->n_src = 0;
  for (long c = 0; c < N; c++) {
    s->src[c] = inside[c];
    s->n_src += inside[c];
  }
  free(inside);
  s->have_prev = 0;
  s->step = 0;
  s->stopped = 0;
  s->nev = 0;
  s->n_ruptures = 0;
  s->maps_valid = 0;
  s->nb = 0;
  s->nb_old = 0;
  memset(s->label, 0, N * sizeof(int32_t));
  memset(s->label_old, 0, N * sizeof(int32_t));
  return 0;
}

/* populations [i*N + c]; with model 1 the melt's, then the gas's (2 Q N) */
void or_set_populations(or_sim* s, const double* f) {
  memcpy(s->f, f, (size_t)s->Q * s->N * sizeof(double));
  if (s->p.model == 1) memcpy(s->g, f + (size_t)s->Q * s->N, (size_t)s->Q * s->N * sizeof(double));
  s->have_prev = 0;
}
void or_get_populations(const or_sim* s, double* f) {
  memcpy(f, s->f, (size_t)s->Q * s->N * sizeof(double));
  if (s->p.model == 1) memcpy(f + (size_t)s->Q * s->N, s->g, (size_t)s->Q * s->N * sizeof(double));
}

/* ------------------------------------------------------------------ */
/* step 1-2: moments and pseudopotential of the current state          */
/* ------------------------------------------------------------------ */
static void compute_moments(or_sim* s, double* jx, double* jy, double* jz) {
  long N = s->N;
#pragma omp parallel for schedule(static) if (N >= OR_OMP_MIN_CELLS)
  for (long c = 0; c < N; c++) {
    double r = 0, a = 0, b = 0, d = 0;
    for (int i = 0; i < s->Q; i++) {
      double fi = s->f[(long)i * N + c];
      r += fi;
      a += s->e[i][0] * fi;
      b += s->e[i][1] * fi;
      d += s->e[i][2] * fi;
    }
    s->rho[c] = r;
    s->psi[c] = psi_of(&s->p, r);
    if (jx) { jx[c] = a; jy[c] = b; jz[c] = d; }
  }
}

/* ------------------------------------------------------------------ */
/* step 3: film maps                                                   */
/* ------------------------------------------------------------------ */

/* Canonical connected-component labels of the gas cells (rho < rho_th),  */
/* links = the lattice's velocity set, periodic.  Components are found by */
/* flood fill started from the lowest unlabelled gas index, so component  */
/* k (1-based) is exactly the k-th component ordered by its minimum linear */
/* index.  Returns the number of components.                              */
static int32_t label_field(const or_sim* s, const double* rho, double rho_th, int32_t* lab) {
  long N = s->N;
  long* queue = (long*)malloc(N * sizeof(long));
  for (long c = 0; c < N; c++) lab[c] = rho[c] < rho_th ? -1 : 0;
  int32_t nb = 0;
  for (long c0 = 0; c0 < N; c0++) {
    if (lab[c0] != -1) continue;
    nb++;
    long head = 0, tail = 0;
    queue[tail++] = c0;
    lab[c0] = nb;
    while (head < tail) {
      long c = queue[head++];
      for (int i = 1; i < s->Q; i++) {
        long d = nbr(s, c, i, +1);
        if (lab[d] == -1) {
          lab[d] = nb;
          queue[tail++] = d;
        }
      }
    }
  }
  free(queue);
  return nb;
}

/* Owner and hop distance (R6, R7): the hop distance (in lattice links) from */
/* each cell to the nearest gas cell, and the smallest and largest label     */
/* among the gas cells at that distance.  A cell equidistant from two        */
/* bubbles keeps both, so the wall between two bubbles is placed             */
/* symmetrically.  Distances are truncated at zone_width-1 hops.  Built      */
/* layer by layer: a cell first reached at layer d takes the min / max owner */
/* of its neighbours of layer d-1.                                           */
static void owner_dist(const or_sim* s, const int32_t* lab, int zone_width, int32_t* owner,
                       int32_t* owner2, int32_t* dist) {
  long N = s->N;
  for (long c = 0; c < N; c++) {
    owner[c] = lab[c];
    owner2[c] = lab[c];
    dist[c] = lab[c] > 0 ? 0 : -1;
  }
  for (int d = 1; d <= zone_width - 1; d++) {
    for (long c = 0; c < N; c++) {
      if (dist[c] != -1) continue;
      int32_t lo = 0, hi = 0;
      for (int i = 1; i < s->Q; i++) {
        long y = nbr(s, c, i, +1);
        if (dist[y] != d - 1) continue;
        if (lo == 0 || owner[y] < lo) lo = owner[y];
        if (owner2[y] > hi) hi = owner2[y];
      }
      if (lo > 0) {
        owner[c] = lo;
        owner2[c] = hi;
        dist[c] = -2 - d; /* provisional marker for this layer */
      }
    }
    for (long c = 0; c < N; c++)
      if (dist[c] == -2 - d) dist[c] = d;
  }
}

/* The pair of alias roots of a cell's nearest bubbles, as (low, high). */
static void root_pair(const or_sim* s, long c, int32_t* lo, int32_t* hi) {
  int32_t a = uf_find(s->alias, s->owner[c]), b = uf_find(s->alias, s->owner2[c]);
  *lo = a < b ? a : b;
  *hi = a < b ? b : a;
}

/* A link joins two walls of a film when both ends are owned and their     */
/* nearest-bubble root pairs differ (R5-R7).                               */
static int roots_differ(const or_sim* s, long c, long y) {
  int32_t a0, a1, b0, b1;
  root_pair(s, c, &a0, &a1);
  root_pair(s, y, &b0, &b1);
  return a0 != b0 || a1 != b1;
}

static void refresh_maps(or_sim* s, const double* rho) {
  long N = s->N;
  /* keep the previous labels and aliases for the alias carry */
  int32_t* t = s->label_old; s->label_old = s->label; s->label = t;
  t = s->alias_old; s->alias_old = s->alias; s->alias = t;
  s->nb_old = s->maps_valid ? s->nb : 0;

  s->nb = label_field(s, rho, s->p.rho_th, s->label);
  owner_dist(s, s->label, s->p.zone_width, s->owner, s->owner2, s->dist);

  /* alias carry: new bubbles whose gas cells overlap old components of one */
  /* old alias class become aliases of each other.                          */
  for (int32_t b = 0; b <= s->nb; b++) s->alias[b] = b;
  if (s->nb_old > 0) {
    int32_t* rep = (int32_t*)malloc((s->nb_old + 1) * sizeof(int32_t));
    for (int32_t a = 0; a <= s->nb_old; a++) rep[a] = 0;
    for (long c = 0; c < N; c++) {
      int32_t b = s->label[c], a = s->label_old[c];
      if (b > 0 && a > 0) {
        int32_t r = uf_find(s->alias_old, a);
        if (rep[r] == 0) rep[r] = b;
        else uf_union(s->alias, b, rep[r]);
      }
    }
    free(rep);
  }

  /* barrier links: both ends owned, their nearest-bubble root pairs differ,  */
  /* and the film between their gas regions is at most zone_width links      */
  /* thick (R5-R7).                                                          */
  for (long c = 0; c < N; c++) {
    uint32_t m = 0;
    if (s->owner[c] > 0) {
      for (int i = 1; i < s->Q; i++) {
        long y = nbr(s, c, i, +1);
        if (s->owner[y] > 0 && roots_differ(s, c, y) &&
            s->dist[c] + s->dist[y] + 1 <= s->p.zone_width)
          m |= 1u << i;
      }
    }
    s->mask[c] = m;
  }
  s->maps_valid = 1;
}

/* a barrier link stays active while the root pairs of its ends differ */
static int link_active(const or_sim* s, long c, int i) {
  if (!s->maps_valid || !(s->mask[c] & (1u << i))) return 0;
  return roots_differ(s, c, nbr(s, c, i, +1));
}

/* ------------------------------------------------------------------ */
/* step 4: Shan-Chen force with the film-barrier substitution            */
/* F(x) = -G psi(x) sum_i w_i psi~(x+e_i) e_i (Sec. 2.1.2, Eq. shanchen3), */
/* summed over opposite pairs so a uniform psi gives exactly zero.        */
/* psi~ = psi_bar on an active barrier link (R5), psi otherwise.          */
/* ------------------------------------------------------------------ */
static void compute_force(or_sim* s, int with_film) {
  long N = s->N;
  const or_params* p = &s->p;
  double psi_liq = psi_of(p, p->rho_liquid);
#pragma omp parallel for schedule(static) if (N >= OR_OMP_MIN_CELLS)
  for (long c = 0; c < N; c++) {
    double acc[3] = {0, 0, 0};
    for (int i = 1; i < s->Q; i++) {
      int o = s->opp[i];
      if (o < i) continue; /* each opposite pair once */
      long yp = nbr(s, c, i, +1), ym = nbr(s, c, i, -1);
      double sp = s->psi[yp], sm = s->psi[ym];
      if (beyond_open(s, c, i, +1)) sp = psi_of(p, p->rho_res); /* the reservoir (R35) */
      if (beyond_open(s, c, i, -1)) sm = psi_of(p, p->rho_res);
      if (with_film) {
        double bar = p->psi_bar_mode == 0 ? psi_liq : s->psi[c];
        if (link_active(s, c, i)) sp = bar;
        if (link_active(s, c, o)) sm = bar;
      }
      for (int k = 0; k < 3; k++) acc[k] += s->w[i] * s->e[i][k] * (sp - sm);
    }
    for (int k = 0; k < 3; k++) s->force[3 * c + k] = -p->G * s->psi[c] * acc[k];
  }
}

/* ------------------------------------------------------------------ */
/* one time step                                                       */
/* ------------------------------------------------------------------ */
static void one_step(or_sim* s) {
  long N = s->N;
  const or_params* p = &s->p;
  int Q = s->Q;
  double* jx = (double*)malloc(3 * N * sizeof(double));
  double* jy = jx + N;
  double* jz = jy + N;

  compute_moments(s, jx, jy, jz);                       /* 1, 2 */
  /* 3: maps refreshed at steps n = 0 (mod k_own) from rho^n, the density   */
  /* of the state entering the step (refresh_src 0), or from rho^(n-1),    */
  /* that of the previous step when it was taken from the current state    */
  /* (refresh_src 1; rho^n at n = 0 and after the state was replaced) (R12) */
  if (p->film_on && s->step % p->k_own == 0)
    refresh_maps(s, (p->refresh_src == 1 && s->have_prev) ? s->rho_prev : s->rho);
  compute_force(s, p->film_on);                         /* 4 */

#pragma omp parallel for schedule(static) if (N >= OR_OMP_MIN_CELLS)
  for (long c = 0; c < N; c++) {
    double rho = s->rho[c];
    double u[3];
    u[0] = (jx[c] + p->tau * s->force[3 * c + 0]) / rho; /* 5 */
    u[1] = (jy[c] + p->tau * s->force[3 * c + 1]) / rho;
    u[2] = (jz[c] + p->tau * s->force[3 * c + 2]) / rho;
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < Q; i++) {                       /* 6 */
      double eu = s->e[i][0] * u[0] + s->e[i][1] * u[1] + s->e[i][2] * u[2];
      double feq = s->w[i] * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * uu);
      double fi = s->f[(long)i * N + c];
      s->fpost[(long)i * N + c] = fi - (fi - feq) / p->tau;
    }
  }

  /* 6c: body force (Sec. 2.1.1, the forcing equation for gravity, read as  */
  /* He's term: F_i = w_i rho' [(e_i - u).g / c_s^2 + (e_i.u)(e_i.g) / c_s^4] */
  /* with rho' = rho - g_rho_ref and u the velocity of the equilibrium (R29)). */
  /* It adds rho' g of momentum and no mass per cell.                       */
  if (p->gx != 0.0 || p->gy != 0.0 || p->gz != 0.0) {
    const double g[3] = {p->gx, p->gy, p->gz};
#pragma omp parallel for schedule(static) if (N >= OR_OMP_MIN_CELLS)
    for (long c = 0; c < N; c++) {
      double rho = s->rho[c];
      double u[3];
      u[0] = (jx[c] + p->tau * s->force[3 * c + 0]) / rho;
      u[1] = (jy[c] + p->tau * s->force[3 * c + 1]) / rho;
      u[2] = (jz[c] + p->tau * s->force[3 * c + 2]) / rho;
      double rb = rho - p->g_rho_ref;
      double ug = u[0] * g[0] + u[1] * g[1] + u[2] * g[2];
      for (int i = 0; i < Q; i++) {
        double eg = s->e[i][0] * g[0] + s->e[i][1] * g[1] + s->e[i][2] * g[2];
        double eu = s->e[i][0] * u[0] + s->e[i][1] * u[1] + s->e[i][2] * u[2];
        s->fpost[(long)i * N + c] += s->w[i] * rb * (3.0 * (eg - ug) + 9.0 * eu * eg);
      }
    }
  }

  /* 6b: bubble growth (Sec. 2.1.3).  Each of the N domain gas points gets   */
  /* the pressure increment dp = A (dn/dt) / N in this step, taken as the  */
  /* ideal-gas density increment drho = dp / c_s^2 = 3 dp and added        */
  /* isotropically, w_i drho to population i: the cell gains exactly drho  */
  /* of mass and no momentum (R25).                                         */
  if (p->growth_on && s->n_src > 0) {
    double dp = p->gas_A * p->gas_dndt / (double)s->n_src;
    double drho = 3.0 * dp;
    for (long c = 0; c < N; c++) {
      if (!s->src[c]) continue;
      for (int i = 0; i < Q; i++) s->fpost[(long)i * N + c] += s->w[i] * drho;
    }
  }

  /* 8: rupture test on active barrier links, with the aliases of the start */
  /* of this step; unions take effect from the next step (R8-R11).          */
  int any_rupture = 0;
  if (p->film_on && s->maps_valid && s->step >= p->rupture_warmup) {
    long first_ev = s->nev;
    for (long c = 0; c < N; c++) {
      if (!s->mask[c]) continue;
      for (int i = 1; i < Q; i++) {
        if (!link_active(s, c, i)) continue;
        long yp = nbr(s, c, i, +1), ym = nbr(s, c, i, -1);
        /* beyond an open plane the reservoir's density (R35) */
        double rp = beyond_open(s, c, i, +1) ? p->rho_res : s->rho[yp];
        double rm = beyond_open(s, c, i, -1) ? p->rho_res : s->rho[ym];
        double d2 = or_p0(rp, p->G, p->rho0) - 2.0 * or_p0(s->rho[c], p->G, p->rho0) + or_p0(rm, p->G, p->rho0);
        if (d2 >= 0.0) {
          /* the film's pair: smallest and largest nearest-bubble label */
          int32_t k = s->owner[c] < s->owner[yp] ? s->owner[c] : s->owner[yp];
          int32_t k2 = s->owner2[c] > s->owner2[yp] ? s->owner2[c] : s->owner2[yp];
          if (s->nev == s->evcap) {
            s->evcap *= 2;
            s->ev = (int64_t*)realloc(s->ev, 3 * (size_t)s->evcap * sizeof(int64_t));
          }
          s->ev[3 * s->nev + 0] = s->step;
          s->ev[3 * s->nev + 1] = k;
          s->ev[3 * s->nev + 2] = k2;
          s->nev++;
        }
      }
    }
    for (long e = first_ev; e < s->nev; e++) {
      any_rupture = 1;
      s->n_ruptures += uf_union(s->alias, (int32_t)s->ev[3 * e + 1], (int32_t)s->ev[3 * e + 2]);
    }
  }

  /* 7: pull form of f_i(x + e_i) <- f*_i(x); across an open plane the    */
  /* population comes from the reservoir at rest, w_i rho_res (R35), and   */
  /* what streams out of the container leaves it                           */
#pragma omp parallel for schedule(static) if (N >= OR_OMP_MIN_CELLS)
  for (long c = 0; c < N; c++)
    for (int i = 0; i < Q; i++)
      s->f[(long)i * N + c] = beyond_open(s, c, i, -1) ? s->w[i] * p->rho_res : s->fpost[(long)i * N + nbr(s, c, i, -1)];

  free(jx);
  memcpy(s->rho_prev, s->rho, N * sizeof(double));
  s->have_prev = 1;
  s->step++;
  if (any_rupture && p->on_rupture == 1) s->stopped = 1;
}

/* ------------------------------------------------------------------ */
/* model 1: the two-lattice step (Sec. 2.1.5, two separate lattices for */
/* melt and gas, coupled at the end of each step; Fig. Mainflowchart    */
/* "Domain coupling").  Readings R30-R34 of the design notes.           */
/* ------------------------------------------------------------------ */

/* moments and pseudopotential of the gas lattice (steps 1-2 for the gas) */
static void compute_moments_gas(or_sim* s, double* jx, double* jy, double* jz) {
  long N = s->N;
#pragma omp parallel for schedule(static) if (N >= OR_OMP_MIN_CELLS)
  for (long c = 0; c < N; c++) {
    double r = 0, a = 0, b = 0, d = 0;
    for (int i = 0; i < s->Q; i++) {
      double gi = s->g[(long)i * N + c];
      r += gi;
      a += s->e[i][0] * gi;
      b += s->e[i][1] * gi;
      d += s->e[i][2] * gi;
    }
    s->rho_g[c] = r;
    s->psi_g[c] = psi_of(&s->p, r);
    if (jx) { jx[c] = a; jy[c] = b; jz[c] = d; }
  }
}

/* Bulk pressure of the two components (R33): the multicomponent Shan-Chen */
/* equation of state, p = (rho_m + rho_g)/3 + (G psi_m^2 + 2 G_mg psi_m    */
/* psi_g + G_gg psi_g^2)/6; each lattice's own part is the xi of Sec. 2.1.5. */
double or_p_tl(double rm, double rg, double G, double G_mg, double G_gg, double rho0) {
  double a = rho0 * (1.0 - exp(-rm / rho0)), b = rho0 * (1.0 - exp(-rg / rho0));
  return (rm + rg) / 3.0 + (G * a * a + 2.0 * G_mg * a * b + G_gg * b * b) / 6.0;
}

/* Forces on both lattices (R31, R32):                                      */
/*   F_m(x) = -psi_m(x) sum_i w_i e_i [G psi~_m(x+e_i) + G_mg psi~_g(x+e_i)] */
/*   F_g(x) = -psi_g(x) sum_i w_i e_i [G_mg psi~_m(x+e_i) + G_gg psi~_g(x+e_i)] */
/* summed over opposite pairs.  On an active barrier link the neighbour's   */
/* state is replaced in every sum by that of the bulk melt (psi_bar_mode 0: */
/* psi(rho_liquid), psi(rho_g_liquid); mode 1: x's own): only the nearest   */
/* bubble's gas acts at x, the per-bubble selection of Sec. 2.1.5.          */
static void compute_force_tl(or_sim* s, int with_film) {
  long N = s->N;
  const or_params* p = &s->p;
  double lm = psi_of(p, p->rho_liquid), lg = psi_of(p, p->rho_g_liquid);
#pragma omp parallel for schedule(static) if (N >= OR_OMP_MIN_CELLS)
  for (long c = 0; c < N; c++) {
    double am[3] = {0, 0, 0}, ag[3] = {0, 0, 0};
    for (int i = 1; i < s->Q; i++) {
      int o = s->opp[i];
      if (o < i) continue;
      long yp = nbr(s, c, i, +1), ym = nbr(s, c, i, -1);
      double pm = s->psi[yp], mm = s->psi[ym], pg = s->psi_g[yp], mg = s->psi_g[ym];
      if (beyond_open(s, c, i, +1)) { pm = psi_of(p, p->rho_res); pg = lg; } /* the reservoir (R35) */
      if (beyond_open(s, c, i, -1)) { mm = psi_of(p, p->rho_res); mg = lg; }
      if (with_film) {
        double bm = p->psi_bar_mode == 0 ? lm : s->psi[c];
        double bg = p->psi_bar_mode == 0 ? lg : s->psi_g[c];
        if (link_active(s, c, i)) { pm = bm; pg = bg; }
        if (link_active(s, c, o)) { mm = bm; mg = bg; }
      }
      for (int k = 0; k < 3; k++) {
        am[k] += s->w[i] * s->e[i][k] * (pm - mm);
        ag[k] += s->w[i] * s->e[i][k] * (pg - mg);
      }
    }
    for (int k = 0; k < 3; k++) {
      s->force[3 * c + k] = -s->psi[c] * (p->G * am[k] + p->G_mg * ag[k]);
      s->force_g[3 * c + k] = -s->psi_g[c] * (p->G_mg * am[k] + p->G_gg * ag[k]);
    }
  }
}

static void one_step_tl(or_sim* s) {
  long N = s->N;
  const or_params* p = &s->p;
  int Q = s->Q;
  double* jm = (double*)malloc(6 * N * sizeof(double));
  double* jg = jm + 3 * N;

  compute_moments(s, jm, jm + N, jm + 2 * N);           /* 1, 2: melt */
  compute_moments_gas(s, jg, jg + N, jg + 2 * N);       /* 1, 2: gas */
  /* 3: maps from the melt density, as in the single-lattice step (R34) */
  if (p->film_on && s->step % p->k_own == 0)
    refresh_maps(s, (p->refresh_src == 1 && s->have_prev) ? s->rho_prev : s->rho);
  compute_force_tl(s, p->film_on);                      /* 4 */

#pragma omp parallel for schedule(static) if (N >= OR_OMP_MIN_CELLS)
  for (long c = 0; c < N; c++) {
    double rm = s->rho[c], rg = s->rho_g[c];
    /* 5: the common velocity of the coupling (R30), then each lattice's */
    /* equilibrium velocity shifted by its own force                      */
    double den = rm / p->tau + rg / p->tau_g;
    double uc[3], um[3], ug[3];
    for (int k = 0; k < 3; k++) {
      uc[k] = (jm[k * N + c] / p->tau + jg[k * N + c] / p->tau_g) / den;
      um[k] = uc[k] + p->tau * s->force[3 * c + k] / rm;
      ug[k] = uc[k] + p->tau_g * s->force_g[3 * c + k] / rg;
    }
    double uum = um[0] * um[0] + um[1] * um[1] + um[2] * um[2];
    double uug = ug[0] * ug[0] + ug[1] * ug[1] + ug[2] * ug[2];
    for (int i = 0; i < Q; i++) {                       /* 6: BGK on both lattices */
      double eum = s->e[i][0] * um[0] + s->e[i][1] * um[1] + s->e[i][2] * um[2];
      double eug = s->e[i][0] * ug[0] + s->e[i][1] * ug[1] + s->e[i][2] * ug[2];
      double fem = s->w[i] * rm * (1.0 + 3.0 * eum + 4.5 * eum * eum - 1.5 * uum);
      double feg = s->w[i] * rg * (1.0 + 3.0 * eug + 4.5 * eug * eug - 1.5 * uug);
      double fi = s->f[(long)i * N + c], gi = s->g[(long)i * N + c];
      s->fpost[(long)i * N + c] = fi - (fi - fem) / p->tau;
      s->gpost[(long)i * N + c] = gi - (gi - feg) / p->tau_g;
    }
  }

  /* 6b: bubble growth (Sec. 2.1.3): the gas release of each domain gas    */
  /* point goes to the gas lattice, w_i drho with drho = 3 A (dn/dt) / N    */
  if (p->growth_on && s->n_src > 0) {
    double drho = 3.0 * p->gas_A * p->gas_dndt / (double)s->n_src;
    for (long c = 0; c < N; c++) {
      if (!s->src[c]) continue;
      for (int i = 0; i < Q; i++) s->gpost[(long)i * N + c] += s->w[i] * drho;
    }
  }

  /* 8: rupture test, on the two-component pressure (R33) */
  int any_rupture = 0;
  if (p->film_on && s->maps_valid && s->step >= p->rupture_warmup) {
    long first_ev = s->nev;
    for (long c = 0; c < N; c++) {
      if (!s->mask[c]) continue;
      for (int i = 1; i < Q; i++) {
        if (!link_active(s, c, i)) continue;
        long yp = nbr(s, c, i, +1), ym = nbr(s, c, i, -1);
        int op = beyond_open(s, c, i, +1), om = beyond_open(s, c, i, -1); /* the reservoir (R35) */
        double d2 = or_p_tl(op ? p->rho_res : s->rho[yp], op ? p->rho_g_liquid : s->rho_g[yp], p->G, p->G_mg,
                            p->G_gg, p->rho0) -
                    2.0 * or_p_tl(s->rho[c], s->rho_g[c], p->G, p->G_mg, p->G_gg, p->rho0) +
                    or_p_tl(om ? p->rho_res : s->rho[ym], om ? p->rho_g_liquid : s->rho_g[ym], p->G, p->G_mg,
                            p->G_gg, p->rho0);
        if (d2 >= 0.0) {
          int32_t k = s->owner[c] < s->owner[yp] ? s->owner[c] : s->owner[yp];
          int32_t k2 = s->owner2[c] > s->owner2[yp] ? s->owner2[c] : s->owner2[yp];
          if (s->nev == s->evcap) {
            s->evcap *= 2;
            s->ev = (int64_t*)realloc(s->ev, 3 * (size_t)s->evcap * sizeof(int64_t));
          }
          s->ev[3 * s->nev + 0] = s->step;
          s->ev[3 * s->nev + 1] = k;
          s->ev[3 * s->nev + 2] = k2;
          s->nev++;
        }
      }
    }
    for (long e = first_ev; e < s->nev; e++) {
      any_rupture = 1;
      s->n_ruptures += uf_union(s->alias, (int32_t)s->ev[3 * e + 1], (int32_t)s->ev[3 * e + 2]);
    }
  }

  /* 7: streaming of both lattices; across an open plane from the          */
  /* reservoir at rest: melt rho_res, gas rho_g_liquid (R35)               */
#pragma omp parallel for schedule(static) if (N >= OR_OMP_MIN_CELLS)
  for (long c = 0; c < N; c++)
    for (int i = 0; i < Q; i++) {
      long from = nbr(s, c, i, -1);
      int out = beyond_open(s, c, i, -1);
      s->f[(long)i * N + c] = out ? s->w[i] * p->rho_res : s->fpost[(long)i * N + from];
      s->g[(long)i * N + c] = out ? s->w[i] * p->rho_g_liquid : s->gpost[(long)i * N + from];
    }

  free(jm);
  memcpy(s->rho_prev, s->rho, N * sizeof(double));
  s->have_prev = 1;
  s->step++;
  if (any_rupture && p->on_rupture == 1) s->stopped = 1;
}

/* Runs up to nsteps steps; returns 1 if the run stopped on a rupture      */
/* (on_rupture == 1, the flowchart's termination), 0 otherwise.           */
int or_step(or_sim* s, int64_t nsteps) {
  for (int64_t k = 0; k < nsteps; k++) {
    if (s->stopped) return 1;
    if (s->p.model == 1) one_step_tl(s);
    else one_step(s);
  }
  return s->stopped;
}

/* ------------------------------------------------------------------ */
/* queries                                                             */
/* ------------------------------------------------------------------ */
void or_density(or_sim* s, double* out) {
  compute_moments(s, NULL, NULL, NULL);
  memcpy(out, s->rho, s->N * sizeof(double));
}

/* velocity, structure of arrays by component (D components).  Mode 0:     */
/* u = j/rho (Sec. 2.1.1, Eq. vel_dens); mode 1: (j + F/2)/rho with the    */
/* force of the current state under the current film maps.                 */
/* With model 1 the velocity of the mixture: (j_m + j_g [+ (F_m + F_g)/2]) */
/* / (rho_m + rho_g), the printed common velocity read with momenta.       */
void or_velocity(or_sim* s, double* out) {
  long N = s->N;
  double* j = (double*)malloc(6 * N * sizeof(double));
  compute_moments(s, j, j + N, j + 2 * N);
  if (s->p.model == 1) compute_moments_gas(s, j + 3 * N, j + 4 * N, j + 5 * N);
  if (s->p.velocity_mode == 1) {
    if (s->p.model == 1) compute_force_tl(s, s->p.film_on);
    else compute_force(s, s->p.film_on);
  }
  for (int k = 0; k < s->D; k++)
    for (long c = 0; c < N; c++) {
      double jk = j[k * N + c], r = s->rho[c];
      if (s->p.model == 1) {
        jk += j[(3 + k) * N + c];
        r += s->rho_g[c];
      }
      if (s->p.velocity_mode == 1) {
        jk += 0.5 * s->force[3 * c + k];
        if (s->p.model == 1) jk += 0.5 * s->force_g[3 * c + k];
      }
      out[k * N + c] = jk / r;
    }
  free(j);
}

/* model 1: density of the gas lattice */
void or_density_gas(or_sim* s, double* out) {
  if (s->p.model != 1) return;
  compute_moments_gas(s, NULL, NULL, NULL);
  memcpy(out, s->rho_g, s->N * sizeof(double));
}

/* force field of the current state (3*N, component-major), for tests */
/* (model 1: the force on the melt lattice) */
void or_force(or_sim* s, int with_film, double* out) {
  compute_moments(s, NULL, NULL, NULL);
  if (s->p.model == 1) {
    compute_moments_gas(s, NULL, NULL, NULL);
    compute_force_tl(s, with_film);
  } else {
    compute_force(s, with_film);
  }
  for (int k = 0; k < 3; k++)
    for (long c = 0; c < s->N; c++) out[k * s->N + c] = s->force[3 * c + k];
}

/* labels of the current state, computed on demand */
int32_t or_labels(or_sim* s, int32_t* out) {
  compute_moments(s, NULL, NULL, NULL);
  return label_field(s, s->rho, s->p.rho_th, out);
}

/* labels / owner / dist of an arbitrary density field (pins and parity) */
int32_t or_label_field(or_sim* s, const double* rho, int32_t* lab) {
  return label_field(s, rho, s->p.rho_th, lab);
}
void or_owner_dist(or_sim* s, const int32_t* lab, int32_t* owner, int32_t* owner2, int32_t* dist) {
  owner_dist(s, lab, s->p.zone_width, owner, owner2, dist);
}

/* film maps as of the last refresh */
int32_t or_maps(const or_sim* s, int32_t* label, int32_t* owner, int32_t* owner2, int32_t* dist,
                uint32_t* mask, int32_t* alias_root) {
  long N = s->N;
  if (label) memcpy(label, s->label, N * sizeof(int32_t));
  if (owner) memcpy(owner, s->owner, N * sizeof(int32_t));
  if (owner2) memcpy(owner2, s->owner2, N * sizeof(int32_t));
  if (dist) memcpy(dist, s->dist, N * sizeof(int32_t));
  if (mask) memcpy(mask, s->mask, N * sizeof(uint32_t));
  if (alias_root)
    for (int32_t b = 0; b <= s->nb; b++) alias_root[b] = uf_find(s->alias, b);
  return s->nb;
}

/* FP64 totals of the current state: mass and momentum, serial sums */
/* (model 1: of both lattices together) */
void or_stats(or_sim* s, double* mass, double* mom) {
  long N = s->N;
  double m = 0, px = 0, py = 0, pz = 0;
  for (long c = 0; c < N; c++)
    for (int i = 0; i < s->Q; i++) {
      double fi = s->f[(long)i * N + c];
      if (s->p.model == 1) fi += s->g[(long)i * N + c];
      m += fi;
      px += s->e[i][0] * fi;
      py += s->e[i][1] * fi;
      pz += s->e[i][2] * fi;
    }
  *mass = m;
  mom[0] = px; mom[1] = py; mom[2] = pz;
}

int64_t or_n_ruptures(const or_sim* s) { return s->n_ruptures; }

/* Foam statistics of a label field, the quantities of the paper's virtual  */
/* metallography (Sec. 5, Table 5 and Fig. 14): out[0] = bubble (gas) cell   */
/* fraction, out[1] = relative foam density 1 - fraction (Table 5's foam     */
/* density is the melt density times this), out[2] = mean equivalent         */
/* diameter over the bubbles (2-D: area-equivalent circle, 3-D: volume-      */
/* equivalent sphere; 0 without bubbles), out[3] = largest equivalent        */
/* diameter.  Plain loops: sizes by counting, diameters summed in label order. */
void or_foam_stats(const or_sim* s, const int32_t* lab, int32_t nb, double* out) {
  int64_t* sizes = (int64_t*)calloc((size_t)nb + 1, sizeof(int64_t));
  int64_t gas = 0;
  for (long c = 0; c < s->N; c++) {
    sizes[lab[c]]++;
    if (lab[c] > 0) gas++;
  }
  double sum = 0.0, dmax = 0.0;
  for (int32_t b = 1; b <= nb; b++) {
    double v = (double)sizes[b];
    double d = s->D == 2 ? 2.0 * sqrt(v / M_PI) : cbrt(6.0 * v / M_PI);
    sum += d;
    if (d > dmax) dmax = d;
  }
  free(sizes);
  out[0] = (double)gas / (double)s->N;
  out[1] = 1.0 - out[0];
  out[2] = nb > 0 ? sum / (double)nb : 0.0;
  out[3] = dmax;
}

/* domain gas points (the cells of the nuclei, Sec. 2.1.3): out[N] 0/1 (may */
/* be NULL); returns their number N of the gas-release law                  */
long or_gas_points(const or_sim* s, unsigned char* out) {
  if (out) memcpy(out, s->src, (size_t)s->N);
  return s->n_src;
}

/* bulk pressure p0 = rho/3 + (G/6) psi^2 of the current state (Sec. 2.1.2, */
/* Eq. Pequ), the quantity plotted across a film (Sec. 4, Fig. plot)        */
/* (model 1: the two-component pressure, R33)                                */
void or_pressure(or_sim* s, double* out) {
  compute_moments(s, NULL, NULL, NULL);
  if (s->p.model == 1) {
    compute_moments_gas(s, NULL, NULL, NULL);
    for (long c = 0; c < s->N; c++)
      out[c] = or_p_tl(s->rho[c], s->rho_g[c], s->p.G, s->p.G_mg, s->p.G_gg, s->p.rho0);
    return;
  }
  for (long c = 0; c < s->N; c++) out[c] = or_p0(s->rho[c], s->p.G, s->p.rho0);
}

/* Test hook: unite the alias classes of labels a and b of the maps in      */
/* force, as a rupture between them would.  Returns 1 if they were apart.   */
int or_alias_unite(or_sim* s, int32_t a, int32_t b) {
  if (!s->maps_valid || a < 1 || b < 1 || a > s->nb || b > s->nb) return -1;
  int r = uf_union(s->alias, a, b);
  s->n_ruptures += r;
  return r;
}

/* raw rupture events (step, k, k2) with k < k2, in the order found */
long or_events(const or_sim* s, int64_t* out, long cap) {
  long n = s->nev < cap ? s->nev : cap;
  memcpy(out, s->ev, 3 * n * sizeof(int64_t));
  return s->nev;
}

/* Bubble-size histogram of a label field: equivalent diameter of each     */
/* bubble (2-D: area-equivalent circle, 3-D: volume-equivalent sphere),    */
/* binned by floor(d / bin_width), last bin open-ended.                    */
void or_histogram(const or_sim* s, const int32_t* lab, int32_t nb, int32_t nbins, double bin_width,
                  int64_t* counts, int64_t* sizes) {
  for (int32_t b = 0; b <= nb; b++) sizes[b] = 0;
  for (long c = 0; c < s->N; c++) sizes[lab[c]]++;
  for (int32_t k = 0; k < nbins; k++) counts[k] = 0;
  for (int32_t b = 1; b <= nb; b++) {
    double v = (double)sizes[b];
    double d = s->D == 2 ? 2.0 * sqrt(v / M_PI) : cbrt(6.0 * v / M_PI);
    long k = (long)floor(d / bin_width);
    if (k >= nbins) k = nbins - 1;
    counts[k]++;
  }
}
