/* Host sanitizer run of the oracle (AddressSanitizer + UndefinedBehavior-
 * Sanitizer build, see tests/test_sanitizers.py): direct sums and butterflies
 * in both directions for every phase id, with ragged point counts, empty
 * leaves, points outside the boxes, N = 1 and several right-hand sides.
 * Exits 0 when every call returns 0 and every output is finite; a sanitizer
 * finding aborts the run. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "../../oracle/bfly_oracle.h"

static double urand(unsigned long long* s) {
  *s = *s * 6364136223846793005ULL + 1442695040888963407ULL;
  return (double)(*s >> 11) * (1.0 / 9007199254740992.0);
}

static int finite_all(const double* v, long n) {
  for (long i = 0; i < n; ++i)
    if (!isfinite(v[i])) return 0;
  return 1;
}

static int run_case(int d, long N, int q, int phase, long n_src, long n_tgt, int nrhs, const double* slo,
                    const double* shi, const double* tlo, const double* thi, unsigned long long seed) {
  double* y = malloc(sizeof(double) * (size_t)(n_src > 0 ? n_src : 1) * d);
  double* x = malloc(sizeof(double) * (size_t)(n_tgt > 0 ? n_tgt : 1) * d);
  double* g = malloc(sizeof(double) * 2 * (size_t)(n_src > 0 ? n_src : 1) * nrhs);
  double* f = malloc(sizeof(double) * 2 * (size_t)(n_tgt > 0 ? n_tgt : 1) * nrhs);
  double* fd = malloc(sizeof(double) * 2 * (size_t)(n_tgt > 0 ? n_tgt : 1) * nrhs);
  double* ga = malloc(sizeof(double) * 2 * (size_t)(n_src > 0 ? n_src : 1) * nrhs);
  unsigned long long s = seed;
  int bad = 0;
  for (long i = 0; i < n_src; ++i)
    for (int j = 0; j < d; ++j) {
      /* a few points outside the box: clamped into the nearest leaf */
      const double u = (i % 17 == 3) ? 1.3 * urand(&s) - 0.15 : urand(&s) * urand(&s);
      y[i * d + j] = slo[j] + u * (shi[j] - slo[j]);
    }
  for (long i = 0; i < n_tgt; ++i)
    for (int j = 0; j < d; ++j) x[i * d + j] = tlo[j] + urand(&s) * (thi[j] - tlo[j]);
  for (long i = 0; i < 2 * n_src * nrhs; ++i) g[i] = urand(&s) - 0.5;
  double counts[4];
  bad |= orc_butterfly(d, N, q, phase, slo, shi, tlo, thi, 0, -1, n_src, y, g, n_src, n_tgt, x, f, n_tgt, nrhs, 2,
                       counts);
  bad |= orc_direct(phase, d, N, 0, n_src, y, g, n_src, n_tgt, x, fd, n_tgt, nrhs, 2);
  bad |= orc_butterfly(d, N, q, phase, slo, shi, tlo, thi, 1, -1, n_tgt, x, f, n_tgt, n_src, y, ga, n_src, nrhs, 2,
                       NULL);
  bad |= !finite_all(f, 2 * n_tgt * nrhs) || !finite_all(fd, 2 * n_tgt * nrhs) || !finite_all(ga, 2 * n_src * nrhs);
  printf("d=%d N=%ld q=%d phase=%d n_src=%ld n_tgt=%ld nrhs=%d: %s\n", d, N, q, phase, n_src, n_tgt, nrhs,
         bad ? "FAILED" : "ok");
  free(y);
  free(x);
  free(g);
  free(f);
  free(fd);
  free(ga);
  return bad;
}

int main(void) {
  const double z3[3] = {0, 0, 0}, o3[3] = {1, 1, 1}, m3[3] = {-4, -4, -4}, p3[3] = {4, 4, 4};
  const double ylo[2] = {1, 0}, yhi[2] = {2, 1}, xlo[2] = {0, 0}, xhi[2] = {1, 1}, fx[2] = {16, 16};
  int bad = 0;
  bad |= run_case(1, 16, 5, ORC_FOURIER, 37, 21, 2, z3, o3, z3, fx, 1);
  bad |= run_case(2, 8, 4, ORC_FOURIER, 70, 64, 3, z3, o3, z3, fx, 2);
  bad |= run_case(2, 8, 3, ORC_HYPRADON2, 101, 33, 1, ylo, yhi, xlo, xhi, 3);
  bad |= run_case(2, 1, 5, ORC_HYPRADON2, 9, 4, 2, ylo, yhi, xlo, xhi, 4);
  bad |= run_case(2, 4, 2, ORC_SEPARABLE, 0, 12, 1, z3, o3, z3, o3, 5);
  bad |= run_case(3, 4, 3, ORC_GENRADON3, 80, 50, 1, z3, o3, z3, o3, 6);
  bad |= run_case(3, 2, 4, ORC_GENRADON3_PI, 30, 19, 2, m3, p3, z3, o3, 7);
  bad |= run_case(3, 2, 2, ORC_SEPARABLE, 11, 0, 1, z3, o3, z3, o3, 8);
  printf(bad ? "SANITIZE FAILED\n" : "SANITIZE OK\n");
  return bad ? 1 : 0;
}
