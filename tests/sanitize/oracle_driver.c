/* Runs the oracle's entry points on small seeded cases, for a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer (test infrastructure: the
 * oracle is the checker, and this checks the checker's memory and integer use).
 * Exits nonzero if an entry point reports an error; the sanitizers abort on a
 * finding. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "mr_oracle.h"

static uint64_t rng = 0x9e3779b97f4a7c15ull;
static double urand(void) { /* splitmix64, in [0, 1) */
  uint64_t z = (rng += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  z ^= z >> 31;
  return (double)(z >> 11) * 0x1.0p-53;
}

#define CHECK(x)                                                   \
  do {                                                             \
    if ((x) != 0) {                                                \
      fprintf(stderr, "%s failed at line %d\n", #x, __LINE__);    \
      exit(1);                                                     \
    }                                                              \
  } while (0)

static void run(int scheme, int jmin, int jmax, double eps, int gamma, int metric, const int bc[4], int steps) {
  orc_params P;
  memset(&P, 0, sizeof P);
  const int dims[6] = {0, 1, 1, 2, 2, 3}, qs[6] = {0, 2, 3, 9, 16, 6}, ncs[6] = {0, 1, 1, 3, 4, 1};
  P.dim = dims[scheme];
  P.q = qs[scheme];
  P.scheme = scheme;
  P.jmin = jmin;
  P.jmax = jmax;
  P.lambda = scheme == 4 ? 5.0 : 1.0;
  P.eq_param = scheme == 2 ? 0.5 : scheme == 4 ? 1.4 : 1.0;
  P.eps = eps;
  P.mu_bar = 1.0;
  for (int h = 0; h < P.q; ++h) P.s[h] = 1.5;
  if (scheme == 1 || scheme == 2 || scheme == 5) P.s[0] = 0.0;
  P.vel[0] = 0.3;
  P.vel[1] = 0.2;
  P.vel[2] = 0.1;
  if (scheme == 3) P.s[0] = P.s[1] = P.s[2] = 0.0;
  if (scheme == 4)
    for (int i = 0; i < 4; ++i) P.s[4 * i] = 0.0;
  for (int k = 0; k < 4; ++k) P.bc[k] = bc[k];
  P.gamma = gamma;
  P.metric = metric;
  const int64_t total = orc_total_cells(&P), nJ = (int64_t)1 << (P.dim * jmax);
  const int nc = ncs[scheme];
  double *m0 = malloc(sizeof(double) * (size_t)(nc * nJ));
  for (int64_t c = 0; c < nJ; ++c) {
    const double x = ((double)(c % ((int64_t)1 << jmax)) + 0.5) / (double)((int64_t)1 << jmax);
    const double bump = (x > 0.3 && x < 0.6 ? 0.4 : 0.0) + 0.05 * urand();
    if (scheme <= 2 || scheme == 5) {
      m0[c] = 0.5 + bump;
    } else if (scheme == 3) {
      m0[c] = 1.0 + 0.1 * bump;
      m0[nJ + c] = 0.02 * bump;
      m0[2 * nJ + c] = -0.01 * bump;
    } else {
      const double rho = 1.0 + bump, u = 0.1, v = -0.1, p = 1.0 + 0.5 * bump;
      m0[c] = rho;
      m0[nJ + c] = rho * u;
      m0[2 * nJ + c] = rho * v;
      m0[3 * nJ + c] = p / 0.4 + 0.5 * rho * (u * u + v * v);
    }
  }
  uint8_t *tree = malloc((size_t)total), *tnew = malloc((size_t)total);
  double *v = malloc(sizeof(double) * (size_t)(P.q * total)), *D = malloc(sizeof(double) * (size_t)total);
  float *vf = malloc(sizeof(float) * (size_t)(P.q * total));
  CHECK(orc_init(&P, m0, tree, v));
  for (int s = 0; s < steps; ++s) CHECK(orc_step(&P, tree, v));
  CHECK(orc_check_tree(&P, tree));
  for (int64_t k = 0; k < P.q * total; ++k) vf[k] = (float)v[k];
  CHECK(orc_new_tree_f32(&P, tree, vf, tnew, D));
  CHECK(orc_step_frozen(&P, tree, tnew, v));
  int64_t counts[64];
  CHECK(orc_leaf_counts(&P, tree, counts));
  const double mass = orc_mass(&P, tree, v);
  if (!isfinite(mass)) exit(2);
  if (orc_check_tree(&P, tree)) exit(3);
  if (gamma == 1 && !bc[0] && !bc[2] && scheme <= 3) { /* the adjoint's primitives */
    double *g = calloc((size_t)(P.q * total), sizeof(double)), *go = calloc((size_t)(P.q * total), sizeof(double));
    for (int64_t k = 0; k < P.q * total; ++k) g[k] = urand();
    CHECK(orc_reconstruct_T(&P, tree, g));
    CHECK(orc_transport_T(&P, tree, g, go));
    free(g);
    free(go);
  }
  printf("scheme %d levels %d..%d gamma %d metric %d bc %d%d%d%d: mass %.6g\n", scheme, jmin, jmax, gamma, metric,
         bc[0], bc[1], bc[2], bc[3], mass);
  free(m0);
  free(tree);
  free(tnew);
  free(v);
  free(D);
  free(vf);
}

int main(void) {
  const int per[4] = {0, 0, 0, 0}, walls1[4] = {2, 3, 0, 0}, walls2[4] = {1, 2, 3, 2}, mixed[4] = {0, 0, 2, 2};
  run(1, 2, 9, 1e-4, 1, 0, per, 6);
  run(2, 2, 9, 1e-4, 3, 1, per, 6);
  run(2, 3, 9, 1e-4, 3, 0, walls1, 6);
  run(3, 2, 6, 1e-3, 1, 0, per, 4);
  run(3, 3, 6, 1e-3, 2, 1, walls2, 4);
  run(3, 2, 6, 1e-3, 1, 1, mixed, 4);
  run(4, 3, 6, 1e-3, 2, 0, walls2, 3);
  run(5, 2, 5, 1e-3, 1, 0, per, 3);
  run(5, 2, 4, 1e-3, 2, 1, per, 2);
  return 0;
}
