/*
 * selftest.c -- a driver that runs every entry point of the FP64 oracle on
 * small 2-D and 3-D lattices (film model, rupture test, refresh readings,
 * gas release, the two-lattice model, the open container, queries), so that a build with the address and
 * undefined-behaviour sanitizers checks the oracle's memory accesses and
 * arithmetic.  TEST INFRASTRUCTURE ONLY: built and run by the CPU tests.
 * It includes the oracle source so that it sees its types.
 */
#include <stdio.h>

#include "foam_oracle.c"

static int run(int lattice, int nx, int ny, int nz, int refresh_src, int growth, int model) {
  or_params p;
  memset(&p, 0, sizeof p);
  p.lattice = lattice;
  p.nx = nx;
  p.ny = ny;
  p.nz = nz;
  p.tau = 0.9;
  p.G = -5.5;
  p.rho0 = 1.0;
  p.rho_liquid = 2.3;
  p.rho_gas = 0.11;
  p.noise_amp = 0.01;
  p.seed = 7;
  p.film_on = 1;
  p.k_own = 2;
  p.zone_width = 6;
  p.rho_th = log(2.0);
  p.psi_bar_mode = 0;
  p.rupture_warmup = 4;
  p.on_rupture = 0;
  p.velocity_mode = 1;
  p.refresh_src = refresh_src;
  p.growth_on = growth;
  p.gas_A = 1.0;
  p.gas_dndt = 0.01;
  p.gy = growth ? 1e-5 : 0.0;
  p.gx = refresh_src ? -2e-5 : 0.0;
  p.g_rho_ref = 1.0;
  if (model == 1) {  /* two lattices: no sources */
    p.model = 1;
    p.G_mg = 0.5;
    p.tau_g = 0.8;
    p.rho_g_bubble = 0.5;
    p.rho_g_liquid = 0.05;
    p.gx = p.gy = 0.0;
  }
  if (refresh_src == 0 && lattice == 1) {  /* a container open across the last axis */
    p.open_z = 1;
    p.rho_res = 2.0;
  }
  or_sim* s = or_create(&p);
  if (!s) return 1;
  const long N = or_N(s);
  const int Q = or_Q(s);
  double nuc[12] = {nx * 0.3, ny * 0.5, nz * 0.5, 0.22 * nx, nx * 0.75, ny * 0.5, nz * 0.5, 0.22 * nx,
                    0.0,      0.0,      0.0,      1.5};
  if (lattice == 0) nuc[2] = nuc[6] = nuc[10] = 0.0;
  if (or_set_nuclei(s, nuc, 3)) return 2;
  double* d = (double*)malloc(sizeof(double) * 3 * (size_t)N);
  double* f = (double*)malloc(sizeof(double) * 2 * (size_t)Q * N);
  int32_t* lab = (int32_t*)malloc(sizeof(int32_t) * (size_t)N);
  int32_t* o1 = (int32_t*)malloc(sizeof(int32_t) * (size_t)N);
  int32_t* o2 = (int32_t*)malloc(sizeof(int32_t) * (size_t)N);
  int32_t* di = (int32_t*)malloc(sizeof(int32_t) * (size_t)N);
  uint32_t* mk = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)N);
  int32_t* al = (int32_t*)malloc(sizeof(int32_t) * (size_t)(N + 2));
  unsigned char* pts = (unsigned char*)malloc((size_t)N);
  int64_t counts[16], sizes[4096], ev[3 * 64], mom_dummy = 0;
  (void)mom_dummy;
  or_step(s, 7);
  or_density(s, d);
  or_velocity(s, d);
  or_force(s, 1, d);
  or_pressure(s, d);
  int32_t nb = or_labels(s, lab);
  if (nb >= 0 && nb < 4096) or_histogram(s, lab, nb, 16, 1.0, counts, sizes);
  or_owner_dist(s, lab, o1, o2, di);
  int32_t nbm = or_maps(s, lab, o1, o2, di, mk, al);
  if (nbm >= 2) or_alias_unite(s, 1, 2);
  or_get_populations(s, f);
  or_set_populations(s, f);
  or_step(s, 5);
  or_events(s, ev, 64);
  or_gas_points(s, pts);
  double m, mom[3];
  or_stats(s, &m, mom);
  or_label_field(s, d, lab);
  if (model == 1) or_density_gas(s, d);
  free(d); free(f); free(lab); free(o1); free(o2); free(di); free(mk); free(al); free(pts);
  or_destroy(s);
  return isfinite(m) ? 0 : 3;
}

int main(void) {
  int rc = 0;
  rc |= run(0, 40, 28, 1, 0, 1, 0);
  rc |= run(0, 33, 17, 1, 1, 0, 0);
  rc |= run(1, 14, 12, 10, 0, 1, 0);
  rc |= run(1, 11, 9, 13, 1, 1, 0);
  rc |= run(0, 31, 22, 1, 0, 0, 1);
  rc |= run(1, 12, 10, 9, 1, 0, 1);
  rc |= run(1, 12, 10, 9, 0, 1, 1);
  printf("oracle selftest %s\n", rc ? "FAILED" : "ok");
  return rc;
}
