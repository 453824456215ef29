/* Drives every entry point of the CPU oracle for the sanitizer builds made by
   test_oracle_sanitizers.py (AddressSanitizer + UndefinedBehaviorSanitizer,
   ThreadSanitizer over its OpenMP loops).  Inputs are seeded pseudo-random
   numbers; the gates need not be unitary, since only memory and thread
   safety are checked here (the numerics are pinned elsewhere).  Prints one
   line per stage and "done" at the end. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct om_mps om_mps;
om_mps *om_create(int n, int chi_max, double cutoff, int max_sweeps, double tol);
void om_destroy(om_mps *m);
void om_set_threads(int t);
void om_bond_dims(const om_mps *m, int32_t *out);
void om_stats(const om_mps *m, double *sum_eps, double *prod_keep, int64_t *n2q, int *last_k,
              double *last_eps, int *last_sweeps);
int om_get_site(const om_mps *m, int q, double *out, int *chiL, int *chiR);
int om_get_lambda(const om_mps *m, int bond, double *out, int *chi);
int om_set_state(om_mps *m, const double *const *sites, const double *const *lambdas,
                 const int32_t *dims);
int om_apply_1q(om_mps *m, int q, const double *u_ri);
int om_apply_2q(om_mps *m, int q0, int q1, const double *g_ri);
int om_apply_layer(om_mps *m, const int32_t *q0, const int32_t *q1, const double *g_ri,
                   int ngates);
int om_svd(const double *m_ri, int rows, int cols, double tol, int max_sweeps, double *u_ri,
           double *sigma, int *sweeps);
int om_truncation(const double *sigma, int count, int rows, int chi_max, double cutoff,
                  int *k_out, double *eps_out, double *norm_out);
int om_expect_pauli(const om_mps *m, const char *pauli, double *re, double *im);
int om_norm2(const om_mps *m, double *out);
int om_overlap(const om_mps *a, const om_mps *b, double *re, double *im);
int om_amplitude(const om_mps *m, const uint8_t *bits, double *re, double *im);
int om_statevector(const om_mps *m, double *out);
int om_sample(const om_mps *m, int shots, const double *u, uint8_t *bits, double *logp);

static uint64_t rs = 0x9e3779b97f4a7c15ull;
static double urand(void) { /* xorshift64*, uniform in [0, 1) */
  rs ^= rs >> 12;
  rs ^= rs << 25;
  rs ^= rs >> 27;
  return (double)((rs * 0x2545f4914f6cdd1dull) >> 11) * 0x1p-53;
}
static void fill(double *x, size_t n) {
  for (size_t i = 0; i < n; i++) x[i] = 2.0 * urand() - 1.0;
}
static void check(int st, const char *what) {
  if (st != 0) {
    fprintf(stderr, "%s: status %d\n", what, st);
    exit(1);
  }
}

static void circuit(om_mps *m, int n, int layers) {
  double g[32];
  int32_t q0[64], q1[64];
  double *gl = (double *)malloc(sizeof(double) * 32 * 64);
  for (int l = 0; l < layers; l++) {
    int ng = 0;
    for (int q = 0; q < n; q++) { /* one-qubit gates */
      fill(g, 8);
      check(om_apply_1q(m, q, g), "apply_1q");
    }
    for (int j = l % 2; j + 1 < n; j += 2) { /* a layer, alternating orientation */
      q0[ng] = (j / 2) % 2 ? j + 1 : j;
      q1[ng] = (j / 2) % 2 ? j : j + 1;
      fill(gl + 32 * ng, 32);
      ng++;
    }
    check(om_apply_layer(m, q0, q1, gl, ng), "apply_layer");
    fill(g, 32); /* a distant gate (SWAP chain there and back) */
    check(om_apply_2q(m, n - 1, l % (n - 2), g), "apply_2q distant");
  }
  free(gl);
}

int main(void) {
  om_set_threads(4);
  /* SVD: tall, wide and square, above the size that runs rounds in parallel */
  const int shapes[3][2] = {{200, 130}, {130, 200}, {192, 192}};
  for (int s = 0; s < 3; s++) {
    const int r = shapes[s][0], c = shapes[s][1], k = r < c ? r : c;
    double *M = (double *)malloc(sizeof(double) * 2 * r * c);
    double *U = (double *)malloc(sizeof(double) * 2 * r * k);
    double *sg = (double *)malloc(sizeof(double) * k);
    fill(M, 2 * (size_t)r * c);
    int sw = 0, kk = 0;
    double eps = 0.0, nrm = 0.0;
    check(om_svd(M, r, c, 1e-15, 60, U, sg, &sw), "svd");
    check(om_truncation(sg, k, r, k / 2, 1e-6, &kk, &eps, &nrm), "truncation");
    printf("svd %dx%d: %d sweeps, k %d\n", r, c, sw, kk);
    free(M);
    free(U);
    free(sg);
  }
  /* a truncating circuit and an untruncated one */
  const int n = 12;
  om_mps *a = om_create(n, 8, 1e-10, 60, 0.0), *b = om_create(n, 64, 0.0, 60, 0.0);
  circuit(a, n, 6);
  rs = 0x9e3779b97f4a7c15ull;
  circuit(b, n, 6);
  int32_t dims[16];
  om_bond_dims(a, dims);
  double se, pk, re, im, nr;
  int64_t n2;
  int lk, lsw;
  double leps;
  om_stats(a, &se, &pk, &n2, &lk, &leps, &lsw);
  printf("circuit: %lld two-qubit gates, sum eps %.3e\n", (long long)n2, se);
  char pauli[16];
  for (int q = 0; q < n; q++) pauli[q] = "IXYZ"[q % 4];
  pauli[n] = 0;
  check(om_expect_pauli(a, pauli, &re, &im), "expect");
  check(om_norm2(b, &nr), "norm2");
  check(om_overlap(a, b, &re, &im), "overlap");
  uint8_t bits[16] = {0};
  check(om_amplitude(b, bits, &re, &im), "amplitude");
  double *sv = (double *)malloc(sizeof(double) * 2 * (1u << n));
  check(om_statevector(a, sv), "statevector");
  /* export into a third handle and sample it on several threads */
  double *sites[16], *lams[16];
  int32_t chis[17];
  chis[0] = 1;
  for (int q = 0; q < n; q++) {
    int cl, cr;
    check(om_get_site(a, q, NULL, &cl, &cr), "site dims");
    sites[q] = (double *)malloc(sizeof(double) * 2 * cl * 2 * cr);
    check(om_get_site(a, q, sites[q], &cl, &cr), "site");
    chis[q + 1] = cr;
    if (q + 1 < n) {
      int c;
      lams[q] = (double *)malloc(sizeof(double) * cr);
      check(om_get_lambda(a, q, lams[q], &c), "lambda");
    }
  }
  om_mps *c = om_create(n, 8, 1e-10, 60, 0.0);
  check(om_set_state(c, (const double *const *)sites, (const double *const *)lams, chis),
        "set_state");
  const int shots = 64;
  double *u = (double *)malloc(sizeof(double) * shots * n), *lp = malloc(sizeof(double) * shots);
  uint8_t *sb = (uint8_t *)malloc((size_t)shots * n);
  for (int i = 0; i < shots * n; i++) u[i] = urand();
  check(om_sample(c, shots, u, sb, lp), "sample");
  printf("sampled %d shots, logp[0] %.3f\n", shots, lp[0]);
  for (int q = 0; q < n; q++) {
    free(sites[q]);
    if (q + 1 < n) free(lams[q]);
  }
  free(sv);
  free(u);
  free(lp);
  free(sb);
  om_destroy(a);
  om_destroy(b);
  om_destroy(c);
  printf("done\n");
  return 0;
}
