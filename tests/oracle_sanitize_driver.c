/*
 * Driver of the oracle's C entry points for the host sanitizer test
 * (tests/test_oracle_sanitizers.py): every entry point on D2Q9, D3Q19 and
 * D3Q27, including degenerate boxes and the argument checks, with buffers
 * of exactly the documented sizes, so that AddressSanitizer sees any access
 * beyond them and UndefinedBehaviorSanitizer any undefined operation.  Prints
 * checksums of every output, which the test compares between the sanitized
 * and a plain build of the same sources.  Test infrastructure only.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int orc_lattice(int q, int32_t *c, double *w);
int orc_transform(int q, int basis, const double *u, double *T);
int orc_norms(int q, int basis, double *b);
int orc_equilibrium(int q, double rho, const double *u, double *feq);
int orc_paper_lambda(int q, double omega, double *lambda);
int orc_normals(int q, uint64_t seed, uint32_t replica, uint64_t step, uint32_t site, double *eta);
int orc_collide_site(int q, int basis, int method, double kT, const double *lambda, const double *f,
                     const double *eta, double *out_macro, double *kpre, double *kstar, double *fstar);
int orc_run(int q, int basis, int method, int nx, int ny, int nz, double kT, const double *lambda,
            uint64_t seed, uint32_t replica, double *f, int64_t step0, int64_t nsteps, double *stats,
            int nthreads);
int orc_init_equilibrium(int q, int64_t N, double rho0, const double *rho, const double *u, double *f);
int orc_nstat(void);
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
double orc_hermite(const double *c, const int32_t *idx, int n);

static int failures = 0;

static void *alloc(size_t n, size_t size) {
  void *p = calloc(n, size);
  if (!p) {
    fprintf(stderr, "out of memory\n");
    exit(2);
  }
  return p;
}

static void report(const char *what, const double *a, size_t n) {
  double s = 0.0, s2 = 0.0;
  for (size_t i = 0; i < n; ++i) {
    s += a[i] * (double)(i + 1);
    s2 += a[i] * a[i];
  }
  printf("%s %.17g %.17g\n", what, s, s2);
}

static void expect(int rc, int want, const char *what) {
  if (rc != want) {
    printf("%s returned %d, expected %d\n", what, rc, want);
    ++failures;
  }
}

static void one_lattice(int q) {
  const int nstat = orc_nstat();
  const double u[3] = {0.03, -0.02, q == 9 ? 0.0 : 0.01};
  char tag[64];
  int32_t *c = alloc(3 * (size_t)q, sizeof(int32_t));
  double *w = alloc((size_t)q, sizeof(double));
  double *T = alloc((size_t)q * q, sizeof(double));
  double *b = alloc((size_t)q, sizeof(double));
  double *feq = alloc((size_t)q, sizeof(double));
  double *lam = alloc((size_t)q, sizeof(double));
  double *eta = alloc((size_t)q, sizeof(double));
  double *f = alloc((size_t)q, sizeof(double));
  double mac[4];
  double *kpre = alloc((size_t)q, sizeof(double));
  double *kstar = alloc((size_t)q, sizeof(double));
  double *fstar = alloc((size_t)q, sizeof(double));

  expect(orc_lattice(q, c, w), 0, "lattice");
  snprintf(tag, sizeof tag, "w%d", q);
  report(tag, w, (size_t)q);
  for (int basis = 0; basis <= (q == 9 ? 1 : 0); ++basis) {
    expect(orc_transform(q, basis, u, T), 0, "transform");
    snprintf(tag, sizeof tag, "T%d_%d", q, basis);
    report(tag, T, (size_t)q * q);
    expect(orc_norms(q, basis, b), 0, "norms");
    snprintf(tag, sizeof tag, "b%d_%d", q, basis);
    report(tag, b, (size_t)q);
  }
  expect(orc_equilibrium(q, 1.02, u, feq), 0, "equilibrium");
  snprintf(tag, sizeof tag, "feq%d", q);
  report(tag, feq, (size_t)q);
  expect(orc_paper_lambda(q, 1.0 / 0.7, lam), 0, "paper_lambda");
  const uint64_t steps[3] = {0, 5, ((uint64_t)1 << 40) + 3};
  for (int k = 0; k < 3; ++k) {
    expect(orc_normals(q, 7, 3, steps[k], 11, eta), 0, "normals");
    snprintf(tag, sizeof tag, "eta%d_%d", q, k);
    report(tag, eta, (size_t)q);
  }
  for (int i = 0; i < q; ++i) f[i] = feq[i] * (1.0 + 1e-3 * (double)((i * 7) % 5 - 2));
  for (int method = 0; method <= (q == 19 ? 0 : 1); ++method) {
    expect(orc_collide_site(q, 0, method, 1e-4, lam, f, eta, mac, kpre, kstar, fstar), 0,
           "collide_site");
    snprintf(tag, sizeof tag, "collide%d_%d", q, method);
    report(tag, fstar, (size_t)q);
    report(tag, kstar, (size_t)q);
    /* every output but fstar may be NULL */
    expect(orc_collide_site(q, 0, method, 1e-4, lam, f, eta, NULL, NULL, NULL, fstar), 0,
           "collide_site (NULL outputs)");
  }

  /* boxes: ragged, and degenerate edges of one and two sites */
  const int boxes[3][3] = {{5, 4, 3}, {1, 1, 1}, {2, 1, 2}};
  for (int k = 0; k < 3; ++k) {
    const int nx = boxes[k][0], ny = boxes[k][1], nz = q == 9 ? 1 : boxes[k][2];
    const int64_t N = (int64_t)nx * ny * nz, nsteps = 3;
    double *rho = alloc((size_t)N, sizeof(double));
    double *uf = alloc(3 * (size_t)N, sizeof(double));
    double *fl = alloc((size_t)q * N, sizeof(double));
    double *st = alloc((size_t)nsteps * nstat, sizeof(double));
    for (int64_t s = 0; s < N; ++s) {
      rho[s] = 1.0 + 0.01 * (double)(s % 3);
      uf[s] = 0.01 * (double)(s % 2);
      uf[N + s] = -0.005 * (double)(s % 5);
      uf[2 * N + s] = q == 9 ? 0.0 : 0.002;
    }
    expect(orc_init_equilibrium(q, N, 1.0, rho, uf, fl), 0, "init_equilibrium");
    snprintf(tag, sizeof tag, "init%d_%d", q, k);
    report(tag, fl, (size_t)q * N);
    for (int method = 0; method <= (q == 19 ? 0 : 1); ++method) {
      expect(orc_run(q, 0, method, nx, ny, nz, 1e-4, lam, 9, 1, fl, 0, nsteps, st, 2), 0, "run");
      snprintf(tag, sizeof tag, "run%d_%d_%d", q, k, method);
      report(tag, fl, (size_t)q * N);
      report(tag, st, (size_t)nsteps * nstat);
    }
    /* statistics may be NULL */
    expect(orc_run(q, 0, 0, nx, ny, nz, 0.0, lam, 9, 1, fl, 10, 1, NULL, 1), 0, "run (no stats)");
    free(rho);
    free(uf);
    free(fl);
    free(st);
  }
  /* argument checks */
  expect(orc_collide_site(q, q == 9 ? 2 : 1, 0, 1e-4, lam, f, eta, mac, kpre, kstar, fstar), -1,
         "collide_site (bad basis)");
  expect(orc_run(q, 0, 0, 0, 1, 1, 1e-4, lam, 9, 1, f, 0, 1, NULL, 1), -1, "run (empty box)");
  if (q == 19)
    expect(orc_run(q, 0, 1, 1, 1, 1, 1e-4, lam, 9, 1, f, 0, 1, NULL, 1), -1, "run (method 1)");
  if (q == 9) expect(orc_run(q, 0, 0, 2, 2, 2, 1e-4, lam, 9, 1, f, 0, 1, NULL, 1), -1, "run (nz 2)");

  free(c);
  free(w);
  free(T);
  free(b);
  free(feq);
  free(lam);
  free(eta);
  free(f);
  free(kpre);
  free(kstar);
  free(fstar);
}

int main(void) {
  const int qs[3] = {9, 19, 27};
  for (int k = 0; k < 3; ++k) one_lattice(qs[k]);
  expect(orc_lattice(10, NULL, NULL), -1, "lattice (q 10)");
  const uint32_t ctr[4] = {0xFFFFFFFFu, 1u, 2u, 3u}, key[2] = {0xDEADBEEFu, 0u};
  uint32_t out[4];
  orc_philox4x32_10(ctr, key, out);
  printf("philox %u %u %u %u\n", out[0], out[1], out[2], out[3]);
  const double cv[3] = {1.0, -1.0, 0.0};
  const int32_t idx[4] = {0, 0, 1, 1};
  printf("hermite %.17g %.17g\n", orc_hermite(cv, idx, 4), orc_hermite(cv, idx, 2));
  printf("failures %d\n", failures);
  return failures ? 1 : 0;
}
