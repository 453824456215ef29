/*
 * tnsim_oracle.c -- CPU reference for MPS gate application.
 *
 * TEST INFRASTRUCTURE ONLY.  Plain, slow, complex128 C99 (+ optional OpenMP)
 * with no BLAS/LAPACK.  Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg may load it; the GPU library never does, and the two share
 * no code, headers or tables.
 *
 * What it computes (arXiv 2601.04422):
 *   - state: an MPS of n rank-3 site tensors A_q[a,s,b] (Sec. II, eq. 2),
 *     initialised to |0...0> with every bond of dimension 1 (Sec. IV.A);
 *   - one-qubit gate: A'[a,s',b] = sum_s U[s',s] A[a,s,b] (Sec. II, eq. 3);
 *   - local two-qubit gate: contract the two sites (Sec. IV.A, Fig. 2), contract
 *     with the gate, decompose by SVD, put the left singular vectors on the
 *     left (control) site and the singular values with the right singular
 *     vectors on the right (target) site (Sec. III.A), truncating the bond
 *     (Sec. II, best low-rank approximation; Sec. IV.A, truncation in the SVD);
 *   - perfect sampling of all qubits (Sec. III.A; see the sampling section).
 *
 * Readings where the paper is silent (each is listed in the design notes):
 *   - Gauge: every site is kept left-canonical and lambda_q holds the Schmidt
 *     values of bond q.  The SVD is taken of theta' * diag(lambda_{i+1}) and
 *     the right site is U_k^H theta' / N, so lambda is never divided out
 *     (Hastings, J. Math. Phys. 50, 095207 (2009)).
 *   - SVD: one-sided (Hestenes) Jacobi on the columns of M, in round-robin
 *     pair order (Brent & Luk 1985); a pair is rotated when
 *     |x^H y| > tol * ||x|| ||y||, tol = max(rows, 16) * 2^-53 by default.  The paper's
 *     GPU SVD is a Jacobi SVD (Sec. IV, cusolverDnZgesvdj).  When M has more
 *     columns than rows, M^H is first reduced by Householder QR and the Jacobi
 *     runs on R^H, which has the same left singular vectors.
 *   - Truncation: sigma sorted descending (ties by column index);
 *     sigma_j^2 <= rows * 2^-53 * sigma_1^2 counts as zero; k is the smallest
 *     k >= 1 whose discarded weight sum_{j>k} sigma_j^2 <= cutoff * W
 *     (W = sum sigma_j^2), capped by chi_max and the non-zero count; the kept
 *     values are renormalised by N = sqrt(sum_{j<=k} sigma_j^2).
 *   - Basis: a 4x4 gate acts on |s_q0 s_q1> with row 2*s_q0 + s_q1.  A gate
 *     given as (q0, q0-1) is applied as SWAP*G*SWAP on (q0-1, q0).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

enum { OM_OK = 0, OM_E_ARG = 1, OM_E_NONLOCAL = 2, OM_E_OVERLAP = 3,
       OM_E_CAPACITY = 4, OM_E_DEVICE = 5, OM_E_NOCONV = 6 };

#define OM_EPS 1.1102230246251565e-16 /* 2^-53 */

typedef struct {
  int n, chi_max, max_sweeps;
  double cutoff, tol; /* tol <= 0 selects max(rows, 16) * 2^-53 */
  int *dim;           /* n+1 entries, dim[0] = dim[n] = 1, dim[q+1] = bond q */
  cplx **A;           /* site q: dim[q] x 2 x dim[q+1], row-major */
  double **lam;       /* bond q (0..n-2): dim[q+1] values */
  double sum_eps, prod_keep;
  int64_t n2q;
  int last_k, last_sweeps;
  double last_eps;
} om_mps;

/* ------------------------------------------------------------------ helpers */

static void *xalloc(size_t bytes) {
  void *p = calloc(bytes ? bytes : 1, 1);
  if (!p) abort();
  return p;
}

static int om_threads = 0;

void om_set_threads(int t) {
  om_threads = t;
#ifdef _OPENMP
  if (t > 0) omp_set_num_threads(t);
#endif
}

int om_get_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------------------------------ state */

om_mps *om_create(int n, int chi_max, double cutoff, int max_sweeps, double tol) {
  if (n < 1 || chi_max < 1) return NULL;
  om_mps *m = (om_mps *)xalloc(sizeof(om_mps));
  m->n = n;
  m->chi_max = chi_max;
  m->cutoff = cutoff;
  m->max_sweeps = max_sweeps > 0 ? max_sweeps : 60;
  m->tol = tol;
  m->dim = (int *)xalloc(sizeof(int) * (n + 1));
  m->A = (cplx **)xalloc(sizeof(cplx *) * n);
  m->lam = (double **)xalloc(sizeof(double *) * (n > 1 ? n - 1 : 1));
  for (int q = 0; q <= n; q++) m->dim[q] = 1;
  for (int q = 0; q < n; q++) {
    m->A[q] = (cplx *)xalloc(sizeof(cplx) * 2);
    m->A[q][0] = 1.0; /* |0> */
    m->A[q][1] = 0.0;
  }
  for (int q = 0; q + 1 < n; q++) {
    m->lam[q] = (double *)xalloc(sizeof(double));
    m->lam[q][0] = 1.0;
  }
  m->prod_keep = 1.0;
  return m;
}

void om_destroy(om_mps *m) {
  if (!m) return;
  for (int q = 0; q < m->n; q++) free(m->A[q]);
  for (int q = 0; q + 1 < m->n; q++) free(m->lam[q]);
  free(m->A);
  free(m->lam);
  free(m->dim);
  free(m);
}

int om_n(const om_mps *m) { return m->n; }

void om_bond_dims(const om_mps *m, int32_t *out) {
  for (int q = 0; q + 1 < m->n; q++) out[q] = m->dim[q + 1];
}

void om_stats(const om_mps *m, double *sum_eps, double *prod_keep, int64_t *n2q,
              int *last_k, double *last_eps, int *last_sweeps) {
  if (sum_eps) *sum_eps = m->sum_eps;
  if (prod_keep) *prod_keep = m->prod_keep;
  if (n2q) *n2q = m->n2q;
  if (last_k) *last_k = m->last_k;
  if (last_eps) *last_eps = m->last_eps;
  if (last_sweeps) *last_sweeps = m->last_sweeps;
}

/* Site q as interleaved (re,im) doubles; chiL/chiR returned. out may be NULL. */
int om_get_site(const om_mps *m, int q, double *out, int *chiL, int *chiR) {
  if (q < 0 || q >= m->n) return OM_E_ARG;
  int a = m->dim[q], b = m->dim[q + 1];
  if (chiL) *chiL = a;
  if (chiR) *chiR = b;
  if (out) memcpy(out, m->A[q], sizeof(cplx) * (size_t)a * 2 * b);
  return OM_OK;
}

int om_get_lambda(const om_mps *m, int bond, double *out, int *chi) {
  if (bond < 0 || bond + 1 >= m->n) return OM_E_ARG;
  int c = m->dim[bond + 1];
  if (chi) *chi = c;
  if (out) memcpy(out, m->lam[bond], sizeof(double) * c);
  return OM_OK;
}

/* Replace the state: sites[q] interleaved complex (dims[q] x 2 x dims[q+1]),
   lambdas[q] (dims[q+1] values), dims has n+1 entries with dims[0]=dims[n]=1. */
int om_set_state(om_mps *m, const double *const *sites, const double *const *lambdas,
                 const int32_t *dims) {
  int n = m->n;
  if (dims[0] != 1 || dims[n] != 1) return OM_E_ARG;
  for (int q = 1; q < n; q++)
    if (dims[q] < 1) return OM_E_ARG;
  for (int q = 0; q <= n; q++) m->dim[q] = dims[q];
  for (int q = 0; q < n; q++) {
    size_t cnt = (size_t)dims[q] * 2 * dims[q + 1];
    free(m->A[q]);
    m->A[q] = (cplx *)xalloc(sizeof(cplx) * cnt);
    memcpy(m->A[q], sites[q], sizeof(cplx) * cnt);
  }
  for (int q = 0; q + 1 < n; q++) {
    free(m->lam[q]);
    m->lam[q] = (double *)xalloc(sizeof(double) * dims[q + 1]);
    memcpy(m->lam[q], lambdas[q], sizeof(double) * dims[q + 1]);
  }
  return OM_OK;
}

/* ------------------------------------------------------------------ 1q gate */

/* A'[a,s',b] = sum_s U[s',s] A[a,s,b]   (Sec. II, eq. 3) */
int om_apply_1q(om_mps *m, int q, const double *u_ri) {
  if (q < 0 || q >= m->n) return OM_E_ARG;
  const cplx *U = (const cplx *)u_ri;
  int a_n = m->dim[q], b_n = m->dim[q + 1];
  cplx *A = m->A[q];
  for (int a = 0; a < a_n; a++)
    for (int b = 0; b < b_n; b++) {
      cplx x0 = A[(a * 2 + 0) * b_n + b], x1 = A[(a * 2 + 1) * b_n + b];
      A[(a * 2 + 0) * b_n + b] = U[0] * x0 + U[1] * x1;
      A[(a * 2 + 1) * b_n + b] = U[2] * x0 + U[3] * x1;
    }
  return OM_OK;
}

/* ------------------------------------------------------------------ SVD */

/* Householder QR of X (rows x cols, column-major, rows >= cols): on return the
   upper triangle of the leading cols x cols block holds R (X = Q R).  Golub &
   Van Loan, Matrix Computations, Sec. 5.2 (complex reflectors). */
static void householder_r(cplx *X, int rows, int cols) {
  for (int j = 0; j < cols; j++) {
    cplx *x = X + (size_t)j * rows;
    double nrm2 = 0.0;
    for (int i = j; i < rows; i++) nrm2 += creal(x[i]) * creal(x[i]) + cimag(x[i]) * cimag(x[i]);
    double nrm = sqrt(nrm2);
    if (nrm == 0.0) continue;
    cplx x0 = x[j];
    double ax0 = cabs(x0);
    cplx ph = ax0 > 0.0 ? x0 / ax0 : 1.0;
    cplx alpha = -ph * nrm;           /* new diagonal entry R_jj */
    /* v = x - alpha e_j on rows j..rows-1, H = I - 2 v v^H / (v^H v) */
    cplx v0 = x0 - alpha;
    double vnorm2 = nrm2 - ax0 * ax0 + creal(v0) * creal(v0) + cimag(v0) * cimag(v0);
    x[j] = v0;                        /* x now stores v */
    for (int c = j + 1; c < cols; c++) {
      cplx *y = X + (size_t)c * rows;
      cplx d = 0.0;
      for (int i = j; i < rows; i++) d += conj(x[i]) * y[i];
      cplx f = 2.0 * d / vnorm2;
      for (int i = j; i < rows; i++) y[i] -= f * x[i];
    }
    x[j] = alpha;
    for (int i = j + 1; i < rows; i++) x[i] = 0.0;
  }
}

/* One-sided Jacobi on the columns of X (rows x cols, column-major).  Pairs are
   visited in round-robin order so that the pairs of one round touch disjoint
   columns.  Returns the number of sweeps, or -1 if max_sweeps was reached. */
static int jacobi_columns(cplx *X, int rows, int cols, double tol, int max_sweeps) {
  if (cols < 2) return 0;
  int P = cols + (cols & 1);
  int npairs = P / 2;
  /* A column whose squared norm is below (rows * 2^-53)^2 of the matrix's
     squared Frobenius norm is rounding noise: far under the numerical-zero
     floor of the truncation, so its direction never reaches the result.
     Pairs holding one are not rotated; this keeps rank-deficient matrices
     (whose noise columns would otherwise keep rotating among themselves) and
     denormals out of the sweeps. */
  double fro2 = 0.0;
  for (size_t i = 0; i < (size_t)rows * cols; i++)
    fro2 += creal(X[i]) * creal(X[i]) + cimag(X[i]) * cimag(X[i]);
  const double small = fro2 * (rows * OM_EPS) * (rows * OM_EPS);
  for (int sweep = 1; sweep <= max_sweeps; sweep++) {
    int rotated = 0;
    for (int r = 0; r < P - 1; r++) {
#pragma omp parallel for schedule(dynamic, 1) reduction(| : rotated) if (cols >= 96)
      for (int k = 0; k < npairs; k++) {
        int p, q;
        if (k == 0) {
          p = P - 1;
          q = r;
        } else {
          p = (r + k) % (P - 1);
          q = (r - k + (P - 1)) % (P - 1);
        }
        if (p > q) { int t = p; p = q; q = t; }
        if (q >= cols) continue;
        cplx *x = X + (size_t)p * rows, *y = X + (size_t)q * rows;
        double alpha = 0.0, beta = 0.0;
        cplx gamma = 0.0;
        for (int i = 0; i < rows; i++) {
          alpha += creal(x[i]) * creal(x[i]) + cimag(x[i]) * cimag(x[i]);
          beta += creal(y[i]) * creal(y[i]) + cimag(y[i]) * cimag(y[i]);
          gamma += conj(x[i]) * y[i];
        }
        double ag = cabs(gamma);
        if (alpha <= small || beta <= small) continue;
        if (!(ag > tol * sqrt(alpha) * sqrt(beta))) continue;
        rotated = 1;
        cplx eiphi = gamma / ag;            /* e^{i phi} */
        double zeta = (beta - alpha) / (2.0 * ag);
        double sg = zeta >= 0.0 ? 1.0 : -1.0;
        double t = sg / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        double c = 1.0 / sqrt(1.0 + t * t);
        double s = c * t;
        for (int i = 0; i < rows; i++) {
          cplx xv = x[i];
          cplx yt = conj(eiphi) * y[i];     /* y~ = e^{-i phi} y */
          x[i] = c * xv - s * yt;
          y[i] = s * xv + c * yt;
        }
      }
    }
    if (!rotated) return sweep;
  }
  return -1;
}

/* Sort indices by sigma descending, ties by index ascending. */
static __thread const double *g_sort_key;
static int cmp_desc(const void *pa, const void *pb) {
  int a = *(const int *)pa, b = *(const int *)pb;
  double sa = g_sort_key[a], sb = g_sort_key[b];
  if (sa > sb) return -1;
  if (sa < sb) return 1;
  return a < b ? -1 : (a > b);
}

/* Left singular vectors and singular values of M (rows x cols, column-major,
   copied).  U gets min(rows,cols) columns (rows x r, column-major), sorted by
   descending sigma.  Returns the sweep count or -1 (no convergence). */
static int svd_left(const cplx *M, int rows, int cols, double tol, int max_sweeps,
                    cplx *U, double *sigma) {
  int r = rows < cols ? rows : cols;
  cplx *X;
  int xcols;
  if (cols <= rows) {
    X = (cplx *)xalloc(sizeof(cplx) * (size_t)rows * cols);
    memcpy(X, M, sizeof(cplx) * (size_t)rows * cols);
    xcols = cols;
  } else {
    /* M^H = Q R  =>  M = R^H Q^H ; left singular vectors of M are those of R^H */
    cplx *Y = (cplx *)xalloc(sizeof(cplx) * (size_t)cols * rows); /* M^H, cols x rows */
    for (int i = 0; i < rows; i++)
      for (int j = 0; j < cols; j++) Y[(size_t)i * cols + j] = conj(M[(size_t)j * rows + i]);
    householder_r(Y, cols, rows);
    X = (cplx *)xalloc(sizeof(cplx) * (size_t)rows * rows); /* R^H, rows x rows */
    for (int i = 0; i < rows; i++)   /* row i of R^H */
      for (int j = 0; j < rows; j++) /* column j of R^H = conj of row j of R */
        X[(size_t)j * rows + i] = (i >= j) ? conj(Y[(size_t)i * cols + j]) : 0.0;
    free(Y);
    xcols = rows;
  }
  if (tol <= 0.0) tol = (rows > 16 ? rows : 16) * OM_EPS;
  int sweeps = jacobi_columns(X, rows, xcols, tol, max_sweeps);
  double *nrm = (double *)xalloc(sizeof(double) * xcols);
  int *idx = (int *)xalloc(sizeof(int) * xcols);
  for (int j = 0; j < xcols; j++) {
    double s = 0.0;
    for (int i = 0; i < rows; i++) {
      cplx v = X[(size_t)j * rows + i];
      s += creal(v) * creal(v) + cimag(v) * cimag(v);
    }
    nrm[j] = sqrt(s);
    idx[j] = j;
  }
  g_sort_key = nrm;
  qsort(idx, xcols, sizeof(int), cmp_desc);
  for (int j = 0; j < r; j++) {
    double s = nrm[idx[j]];
    sigma[j] = s;
    for (int i = 0; i < rows; i++)
      U[(size_t)j * rows + i] = s > 0.0 ? X[(size_t)idx[j] * rows + i] / s : (i == j ? 1.0 : 0.0);
  }
  free(nrm);
  free(idx);
  free(X);
  return sweeps;
}

/* Exported for the SVD pins: M row-major interleaved (rows x cols); U out
   column-major interleaved (rows x min), sigma out (min). */
int om_svd(const double *m_ri, int rows, int cols, double tol, int max_sweeps,
           double *u_ri, double *sigma, int *sweeps) {
  if (rows < 1 || cols < 1) return OM_E_ARG;
  cplx *M = (cplx *)xalloc(sizeof(cplx) * (size_t)rows * cols);
  const cplx *src = (const cplx *)m_ri;
  for (int i = 0; i < rows; i++)
    for (int j = 0; j < cols; j++) M[(size_t)j * rows + i] = src[(size_t)i * cols + j];
  int s = svd_left(M, rows, cols, tol, max_sweeps > 0 ? max_sweeps : 60, (cplx *)u_ri, sigma);
  free(M);
  if (sweeps) *sweeps = s;
  return s < 0 ? OM_E_NOCONV : OM_OK;
}

/* Truncation rule on a descending spectrum.  rows is the row count of the
   decomposed matrix (sets the numerical-zero floor). */
int om_truncation(const double *sigma, int count, int rows, int chi_max, double cutoff,
                  int *k_out, double *eps_out, double *norm_out) {
  if (count < 1) return OM_E_ARG;
  double W = 0.0;
  for (int j = 0; j < count; j++) W += sigma[j] * sigma[j];
  double floor2 = rows * OM_EPS * sigma[0] * sigma[0];
  int nz = 0;
  for (int j = 0; j < count; j++)
    if (sigma[j] * sigma[j] > floor2) nz++;
  if (nz < 1) nz = 1;
  /* tail[k] = sum_{j>k} sigma_j^2 (1-based k), summed from the small end */
  double *tail = (double *)xalloc(sizeof(double) * (count + 1));
  tail[count] = 0.0;
  for (int k = count - 1; k >= 0; k--) tail[k] = tail[k + 1] + sigma[k] * sigma[k];
  int kc = count;
  for (int k = 1; k <= count; k++)
    if (tail[k] <= cutoff * W) { kc = k; break; }
  int k = kc;
  if (k > nz) k = nz;
  if (k > chi_max) k = chi_max;
  if (k < 1) k = 1;
  double head = 0.0;
  for (int j = 0; j < k; j++) head += sigma[j] * sigma[j];
  if (k_out) *k_out = k;
  if (eps_out) *eps_out = W > 0.0 ? tail[k] / W : 0.0;
  if (norm_out) *norm_out = sqrt(head);
  free(tail);
  return OM_OK;
}

/* ------------------------------------------------------------------ 2q gate */

static int apply_2q_local(om_mps *m, int i, const cplx *G) {
  int chiL = m->dim[i], chiM = m->dim[i + 1], chiR = m->dim[i + 2];
  int rows = 2 * chiL, cols = 2 * chiR;
  const cplx *A0 = m->A[i], *A1 = m->A[i + 1];
  /* theta[a,s,t,c] = sum_b A_i[a,s,b] A_{i+1}[b,t,c]   (Fig. 2 merge) */
  cplx *th = (cplx *)xalloc(sizeof(cplx) * (size_t)rows * cols);
  for (int as = 0; as < rows; as++)
    for (int b = 0; b < chiM; b++) {
      cplx w = A0[(size_t)as * chiM + b];
      if (w == 0.0) continue;
      const cplx *r1 = A1 + (size_t)b * cols;
      cplx *o = th + (size_t)as * cols;
      for (int tc = 0; tc < cols; tc++) o[tc] += w * r1[tc];
    }
  /* theta'[a,s',t',c] = sum_{s,t} G[2s'+t', 2s+t] theta[a,s,t,c]   (gate contraction) */
  cplx *thp = (cplx *)xalloc(sizeof(cplx) * (size_t)rows * cols);
  for (int a = 0; a < chiL; a++)
    for (int c = 0; c < chiR; c++) {
      cplx v[4];
      for (int s = 0; s < 2; s++)
        for (int t = 0; t < 2; t++) v[2 * s + t] = th[(size_t)(2 * a + s) * cols + t * chiR + c];
      for (int sp = 0; sp < 2; sp++)
        for (int tp = 0; tp < 2; tp++) {
          cplx acc = 0.0;
          for (int j = 0; j < 4; j++) acc += G[(2 * sp + tp) * 4 + j] * v[j];
          thp[(size_t)(2 * a + sp) * cols + tp * chiR + c] = acc;
        }
    }
  free(th);
  /* M[2a+s, t*chiR+c] = theta'[a,s,t,c] * lambda_{i+1}[c], column-major */
  const double *lr = (i + 1 <= m->n - 2) ? m->lam[i + 1] : NULL;
  cplx *M = (cplx *)xalloc(sizeof(cplx) * (size_t)rows * cols);
  for (int r = 0; r < rows; r++)
    for (int t = 0; t < 2; t++)
      for (int c = 0; c < chiR; c++) {
        double w = lr ? lr[c] : 1.0;
        M[(size_t)(t * chiR + c) * rows + r] = thp[(size_t)r * cols + t * chiR + c] * w;
      }
  int rk = rows < cols ? rows : cols;
  cplx *U = (cplx *)xalloc(sizeof(cplx) * (size_t)rows * rk);
  double *sig = (double *)xalloc(sizeof(double) * rk);
  int sweeps = svd_left(M, rows, cols, m->tol, m->max_sweeps, U, sig);
  free(M);
  if (sweeps < 0) {
    free(U); free(sig); free(thp);
    return OM_E_NOCONV;
  }
  int k;
  double eps, N;
  om_truncation(sig, rk, rows, m->chi_max, m->cutoff, &k, &eps, &N);
  if (!(N > 0.0)) N = 1.0;
  /* A_i' = U_k as (chiL, 2, k); lambda_i' = sigma/N; A_{i+1}' = U_k^H theta' / N */
  cplx *nA0 = (cplx *)xalloc(sizeof(cplx) * (size_t)rows * k);
  for (int r = 0; r < rows; r++)
    for (int j = 0; j < k; j++) nA0[(size_t)r * k + j] = U[(size_t)j * rows + r];
  cplx *nA1 = (cplx *)xalloc(sizeof(cplx) * (size_t)k * cols);
  for (int j = 0; j < k; j++) {
    cplx *o = nA1 + (size_t)j * cols;
    for (int r = 0; r < rows; r++) {
      cplx w = conj(U[(size_t)j * rows + r]) / N;
      const cplx *src = thp + (size_t)r * cols;
      for (int tc = 0; tc < cols; tc++) o[tc] += w * src[tc];
    }
  }
  double *nl = (double *)xalloc(sizeof(double) * k);
  for (int j = 0; j < k; j++) nl[j] = sig[j] / N;
  free(m->A[i]);
  free(m->A[i + 1]);
  free(m->lam[i]);
  m->A[i] = nA0;
  m->A[i + 1] = nA1;
  m->lam[i] = nl;
  m->dim[i + 1] = k;
  m->sum_eps += eps;
  m->prod_keep *= (1.0 - eps);
  m->n2q += 1;
  m->last_k = k;
  m->last_eps = eps;
  m->last_sweeps = sweeps;
  free(U); free(sig); free(thp);
  return OM_OK;
}

static int apply_2q_adjacent(om_mps *m, int q0, int q1, const cplx *G) {
  if (q1 == q0 + 1) return apply_2q_local(m, q0, G);
  /* same gate with the two qubits listed in the other order: SWAP G SWAP */
  cplx Gs[16];
  for (int sp = 0; sp < 2; sp++)
    for (int tp = 0; tp < 2; tp++)
      for (int s = 0; s < 2; s++)
        for (int t = 0; t < 2; t++)
          Gs[(2 * sp + tp) * 4 + 2 * s + t] = G[(2 * tp + sp) * 4 + 2 * t + s];
  return apply_2q_local(m, q1, Gs);
}

/* A gate on distant qubits (Sec. IV.A): SWAP gates bring the qubit with the
   larger index next to the other one, the gate acts there, and the SWAPs are
   undone in reverse order.  Every SWAP is an ordinary two-qubit gate, with
   its own truncation. */
int om_apply_2q(om_mps *m, int q0, int q1, const double *g_ri) {
  if (q0 < 0 || q0 >= m->n || q1 < 0 || q1 >= m->n || q0 == q1) return OM_E_ARG;
  const cplx *G = (const cplx *)g_ri;
  if (q1 == q0 + 1 || q1 == q0 - 1) return apply_2q_adjacent(m, q0, q1, G);
  cplx S[16] = {0};
  for (int s = 0; s < 2; s++)
    for (int t = 0; t < 2; t++) S[(2 * t + s) * 4 + 2 * s + t] = 1.0;
  const int a = q0 < q1 ? q0 : q1, b = q0 < q1 ? q1 : q0;
  for (int j = b - 1; j > a; j--) {
    int r = apply_2q_local(m, j, S);
    if (r != OM_OK) return r;
  }
  /* the qubit from b now sits at a + 1 */
  int r = q0 == a ? apply_2q_adjacent(m, a, a + 1, G) : apply_2q_adjacent(m, a + 1, a, G);
  if (r != OM_OK) return r;
  for (int j = a + 1; j < b; j++) {
    r = apply_2q_local(m, j, S);
    if (r != OM_OK) return r;
  }
  return OM_OK;
}

/* ------------------------------------------------------------------ canonical form */

/* Canonicalisation (Sec. IV.A: the MPS is brought to left- and right-canonical
   form before sampling).  Restores the gauge this simulator keeps (every site
   left-canonical, lambda_q the Schmidt values of bond q) exactly, from any
   gauge:
   1. left to right, q = 0 .. n-2: SVD of site q as a (dim[q]*2) x dim[q+1]
      matrix, A_q <- U (numerically non-zero columns only), and
      A_{q+1} <- (U^H A_q) A_{q+1}; afterwards sites 0 .. n-2 are
      left-canonical and site n-1 carries the norm, which is divided out;
   2. right to left, b = n-2 .. 0: the Schmidt decomposition of bond b is the
      SVD of C[a, (t, c)] = A_{b+1}[a, t, c] * lambda_{b+1}[c] (lambda = 1 at
      the right end): sites 0 .. b form an orthonormal left basis and the part
      right of bond b+1 was put in its Schmidt basis by the previous step.
      C = U S V^H gives lambda_b = S / N, A_b <- A_b U, A_{b+1} <- U^H A_{b+1} / N.
   With truncate = 0 only numerically zero values are dropped (the floor of
   the truncation rule).  With truncate = 1, step 2 applies the truncation
   rule with chi_max and cutoff, adding each cut's discarded weight to the
   statistics; a cut changes the state, so the bonds right of it (already
   swept) no longer carry its Schmidt values, and both steps run once more
   without truncation.  The state is normalised. */
/* Step 1 on sites lo .. hi: sites lo .. hi-1 become left-canonical, the
   rest of the window's content moves into site hi. */
static int canon_left_sweep(om_mps *m, int lo, int hi) {
  for (int q = lo; q < hi; q++) {
    const int rows = 2 * m->dim[q], cols = m->dim[q + 1], r = rows < cols ? rows : cols;
    cplx *M = (cplx *)xalloc(sizeof(cplx) * (size_t)rows * cols); /* column-major */
    for (int i = 0; i < rows; i++)
      for (int j = 0; j < cols; j++) M[(size_t)j * rows + i] = m->A[q][(size_t)i * cols + j];
    cplx *U = (cplx *)xalloc(sizeof(cplx) * (size_t)rows * r);
    double *sig = (double *)xalloc(sizeof(double) * r);
    int sw = svd_left(M, rows, cols, m->tol, m->max_sweeps, U, sig);
    if (sw < 0) { free(M); free(U); free(sig); return OM_E_NOCONV; }
    int k;
    om_truncation(sig, r, rows, 1 << 30, 0.0, &k, NULL, NULL);
    /* R = U_k^H M  (k x cols) */
    cplx *R = (cplx *)xalloc(sizeof(cplx) * (size_t)k * cols);
    for (int j = 0; j < k; j++)
      for (int c = 0; c < cols; c++) {
        cplx acc = 0.0;
        for (int i = 0; i < rows; i++) acc += conj(U[(size_t)j * rows + i]) * M[(size_t)c * rows + i];
        R[(size_t)j * cols + c] = acc;
      }
    cplx *nA = (cplx *)xalloc(sizeof(cplx) * (size_t)rows * k);
    for (int i = 0; i < rows; i++)
      for (int j = 0; j < k; j++) nA[(size_t)i * k + j] = U[(size_t)j * rows + i];
    /* A_{q+1} <- R A_{q+1}: (k x cols) (cols x 2 dim[q+2]) */
    const int w = 2 * m->dim[q + 2];
    cplx *nB = (cplx *)xalloc(sizeof(cplx) * (size_t)k * w);
    for (int j = 0; j < k; j++)
      for (int c = 0; c < cols; c++) {
        cplx f = R[(size_t)j * cols + c];
        if (f == 0.0) continue;
        for (int e = 0; e < w; e++) nB[(size_t)j * w + e] += f * m->A[q + 1][(size_t)c * w + e];
      }
    free(m->A[q]);
    free(m->A[q + 1]);
    m->A[q] = nA;
    m->A[q + 1] = nB;
    m->dim[q + 1] = k;
    free(m->lam[q]);
    m->lam[q] = (double *)xalloc(sizeof(double) * k); /* rewritten by step 2 */
    free(M); free(U); free(sig); free(R);
  }
  return OM_OK;
}

/* Step 2 on bonds hi-1 .. lo (sites lo .. hi-1 left-canonical, bond hi in
   Schmidt form or the right end).  With truncate, the rule applies with
   chi_max and cutoff; each cut's discarded weight (relative to the weight
   of the state at that point) goes to eps_out (sum) and keep_out (product
   of 1 - eps); k_out gets the dimension of bond lo. */
static int canon_right_sweep(om_mps *m, int lo, int hi, int truncate, double *eps_out,
                             double *keep_out, int *k_out) {
  const int n = m->n;
  for (int b = hi - 1; b >= lo; b--) {
    const int rows = m->dim[b + 1], chiR = m->dim[b + 2], cols = 2 * chiR;
    const int r = rows < cols ? rows : cols;
    const double *lr = (b + 1 <= n - 2) ? m->lam[b + 1] : NULL;
    cplx *M = (cplx *)xalloc(sizeof(cplx) * (size_t)rows * cols); /* column-major */
    for (int a = 0; a < rows; a++)
      for (int t = 0; t < 2; t++)
        for (int c = 0; c < chiR; c++)
          M[(size_t)(t * chiR + c) * rows + a] =
              m->A[b + 1][((size_t)a * 2 + t) * chiR + c] * (lr ? lr[c] : 1.0);
    cplx *U = (cplx *)xalloc(sizeof(cplx) * (size_t)rows * r);
    double *sig = (double *)xalloc(sizeof(double) * r);
    int sw = svd_left(M, rows, cols, m->tol, m->max_sweeps, U, sig);
    free(M);
    if (sw < 0) { free(U); free(sig); return OM_E_NOCONV; }
    int k;
    double eps, N;
    om_truncation(sig, r, rows, truncate ? m->chi_max : 1 << 30, truncate ? m->cutoff : 0.0, &k,
                  &eps, &N);
    if (!(N > 0.0)) N = 1.0;
    /* A_b <- A_b U_k  (dim[b]*2 x rows) (rows x k) */
    const int lb = 2 * m->dim[b];
    cplx *nA = (cplx *)xalloc(sizeof(cplx) * (size_t)lb * k);
    for (int i = 0; i < lb; i++)
      for (int a = 0; a < rows; a++) {
        cplx f = m->A[b][(size_t)i * rows + a];
        if (f == 0.0) continue;
        for (int j = 0; j < k; j++) nA[(size_t)i * k + j] += f * U[(size_t)j * rows + a];
      }
    /* A_{b+1} <- U_k^H A_{b+1} / N */
    cplx *nB = (cplx *)xalloc(sizeof(cplx) * (size_t)k * cols);
    for (int j = 0; j < k; j++)
      for (int a = 0; a < rows; a++) {
        cplx f = conj(U[(size_t)j * rows + a]) / N;
        for (int e = 0; e < cols; e++) nB[(size_t)j * cols + e] += f * m->A[b + 1][(size_t)a * cols + e];
      }
    double *schmidt = (double *)xalloc(sizeof(double) * k);
    for (int j = 0; j < k; j++) schmidt[j] = sig[j] / N;
    free(m->A[b]);
    free(m->A[b + 1]);
    free(m->lam[b]);
    m->A[b] = nA;
    m->A[b + 1] = nB;
    m->lam[b] = schmidt;
    m->dim[b + 1] = k;
    if (eps_out) *eps_out += eps;
    if (keep_out) *keep_out *= (1.0 - eps);
    if (k_out) *k_out = k;
    free(U); free(sig);
  }
  return OM_OK;
}

static int canon_pass(om_mps *m, int truncate) {
  const int n = m->n;
  int r = canon_left_sweep(m, 0, n - 1);
  if (r != OM_OK) return r;
  {
    const size_t cnt = (size_t)m->dim[n - 1] * 2;
    double nrm2 = 0.0;
    for (size_t e = 0; e < cnt; e++) nrm2 += creal(m->A[n - 1][e]) * creal(m->A[n - 1][e]) +
                                             cimag(m->A[n - 1][e]) * cimag(m->A[n - 1][e]);
    if (!(nrm2 > 0.0)) return OM_E_ARG; /* the zero vector has no canonical form */
    const double inv = 1.0 / sqrt(nrm2);
    for (size_t e = 0; e < cnt; e++) m->A[n - 1][e] *= inv;
  }
  return canon_right_sweep(m, 0, n - 1, truncate, truncate ? &m->sum_eps : NULL,
                           truncate ? &m->prod_keep : NULL, NULL);
}

int om_canonicalize(om_mps *m, int truncate) {
  int r = canon_pass(m, truncate);
  if (r == OM_OK && truncate) r = canon_pass(m, 0);
  return r;
}

/* ------------------------------------------------------------------ bond propagation */

/* A gate on distant qubits by bond propagation (Sec. III.A, non-local gates):
   the 4x4 gate, cast as a 2x2x2x2 tensor, is split by SVD into
   G = sum_r X_r (x) Y_r (X_r on the qubit at the left site a, Y_r on the one
   at the right site b, the singular values folded into Y_r; r <= 4 terms).
   X_r is contracted into site a, whose right bond gains the propagating index
   r; the index is carried through every site between a and b (the
   intermediate sites become I_r (x) A_j); Y_r is contracted into site b.
   The chain then holds G|psi> exactly, with bonds a .. b-1 of dimension
   r * chi.  Then (readings of the paper, which does not fix the gauge or the
   truncation of this method): the sites a .. b-1 are decomposed in
   succession from left to right without truncation (Sec. III.A: each
   intermediate qubit is contracted and decomposed in turn; every step is an
   SVD whose left vectors stay on the site and whose remainder moves right),
   and then the bonds b-1 .. a get their Schmidt values from right to left,
   where the truncation rule applies (chi_max, cutoff), as in a canonical
   sweep.  The recorded discarded weight of the gate is the sum over its
   cuts. */
int om_apply_2q_propagate(om_mps *m, int q0, int q1, const double *g_ri) {
  if (q0 < 0 || q0 >= m->n || q1 < 0 || q1 >= m->n || q0 == q1) return OM_E_ARG;
  const cplx *G = (const cplx *)g_ri;
  if (q1 == q0 + 1 || q1 == q0 - 1) return apply_2q_adjacent(m, q0, q1, G);
  const int a = q0 < q1 ? q0 : q1, b = q0 < q1 ? q1 : q0;
  /* Gm[(x', x), (y', y)] with x the qubit on site a, y the one on site b;
     the gate's rows are 2 s_q0' + s_q1', its columns 2 s_q0 + s_q1 */
  cplx Gm[16]; /* column-major 4 x 4: Gm[col * 4 + row] */
  for (int xp = 0; xp < 2; xp++)
    for (int x = 0; x < 2; x++)
      for (int yp = 0; yp < 2; yp++)
        for (int y = 0; y < 2; y++) {
          const int row = q0 == a ? 2 * xp + yp : 2 * yp + xp;
          const int col = q0 == a ? 2 * x + y : 2 * y + x;
          Gm[(2 * yp + y) * 4 + (2 * xp + x)] = G[row * 4 + col];
        }
  cplx Ug[16];
  double sg[4];
  if (svd_left(Gm, 4, 4, 0.0, 60, Ug, sg) < 0) return OM_E_NOCONV;
  int rg;
  om_truncation(sg, 4, 4, 4, 0.0, &rg, NULL, NULL);
  /* X_r[x', x] = U[(x', x), r];  Y_r[y', y] = sum_i conj(U[i, r]) Gm[i, (y', y)] */
  cplx X[4][4], Y[4][4];
  for (int r = 0; r < rg; r++)
    for (int e = 0; e < 4; e++) {
      X[r][e] = Ug[r * 4 + e];
      cplx acc = 0.0;
      for (int i = 0; i < 4; i++) acc += conj(Ug[r * 4 + i]) * Gm[e * 4 + i];
      Y[r][e] = acc;
    }
  /* the chain with the propagating index merged into bonds a .. b-1
     (bond j index r * dim[j+1] + c) */
  int *od = (int *)xalloc(sizeof(int) * (m->n + 1));
  memcpy(od, m->dim, sizeof(int) * (m->n + 1));
  for (int q = a; q <= b; q++) {
    const int L = od[q], R = od[q + 1];
    const int nL = q == a ? L : rg * L, nR = q == b ? R : rg * R;
    cplx *nA = (cplx *)xalloc(sizeof(cplx) * (size_t)nL * 2 * nR);
    for (int r = 0; r < rg; r++)
      for (int l = 0; l < L; l++)
        for (int sp = 0; sp < 2; sp++)
          for (int c = 0; c < R; c++) {
            cplx v;
            if (q == a)
              v = X[r][2 * sp + 0] * m->A[q][((size_t)l * 2 + 0) * R + c] +
                  X[r][2 * sp + 1] * m->A[q][((size_t)l * 2 + 1) * R + c];
            else if (q == b)
              v = Y[r][2 * sp + 0] * m->A[q][((size_t)l * 2 + 0) * R + c] +
                  Y[r][2 * sp + 1] * m->A[q][((size_t)l * 2 + 1) * R + c];
            else
              v = m->A[q][((size_t)l * 2 + sp) * R + c];
            const int li = q == a ? l : r * L + l, ri = q == b ? c : r * R + c;
            nA[((size_t)li * 2 + sp) * nR + ri] = v;
          }
    free(m->A[q]);
    m->A[q] = nA;
  }
  for (int q = a + 1; q <= b; q++) m->dim[q] = rg * od[q];
  for (int j = a; j < b; j++) {
    free(m->lam[j]);
    m->lam[j] = (double *)xalloc(sizeof(double) * m->dim[j + 1]); /* rewritten below */
  }
  free(od);
  int st = canon_left_sweep(m, a, b);
  double eps = 0.0, keep = 1.0;
  int k = 0;
  if (st == OM_OK) st = canon_right_sweep(m, a, b, 1, &eps, &keep, &k);
  if (st != OM_OK) return st;
  m->sum_eps += eps;
  m->prod_keep *= keep;
  m->n2q += 1;
  m->last_k = k;
  m->last_eps = eps;
  return OM_OK;
}

/* Gates of one layer: q1[g] = -1 marks a one-qubit gate (matrix in the first
   4 complex entries of its 16-entry slot).  Qubits must be disjoint. */
int om_apply_layer(om_mps *m, const int32_t *q0, const int32_t *q1, const double *g_ri,
                   int ngates) {
  char *used = (char *)xalloc(m->n);
  int st = OM_OK;
  for (int g = 0; g < ngates && st == OM_OK; g++) {
    int a = q0[g], b = q1[g];
    if (a < 0 || a >= m->n || b >= m->n || b < -1 || a == b) st = OM_E_ARG;
    else if (b >= 0 && a - b != 1 && b - a != 1) st = OM_E_NONLOCAL;
    else if (used[a] || (b >= 0 && used[b])) st = OM_E_OVERLAP;
    else {
      used[a] = 1;
      if (b >= 0) used[b] = 1;
    }
  }
  free(used);
  if (st != OM_OK) return st;
  for (int g = 0; g < ngates; g++) {
    const double *G = g_ri + (size_t)g * 32;
    int r = q1[g] < 0 ? om_apply_1q(m, q0[g], G) : om_apply_2q(m, q0[g], q1[g], G);
    if (r != OM_OK) return r;
  }
  return OM_OK;
}

/* ------------------------------------------------------------------ readouts */

static const cplx PAULI_M[4][4] = {
    {1, 0, 0, 1},   /* I */
    {0, 1, 1, 0},   /* X */
    {0, -I, I, 0},  /* Y */
    {1, 0, 0, -1}}; /* Z */

static int pauli_index(char c) {
  switch (c) {
    case 'I': return 0;
    case 'X': return 1;
    case 'Y': return 2;
    case 'Z': return 3;
  }
  return -1;
}

/* <bra| P |ket> by left-to-right transfer contraction:
   E'[b,b'] = sum conj(B[a,s,b]) P[s,s'] E[a,a'] K[a',s',b'].  bra, ket may be
   the same MPS.  P == NULL means identity everywhere. */
static cplx transfer(const om_mps *bra, const om_mps *ket, const int *pidx) {
  int n = ket->n;
  cplx *E = (cplx *)xalloc(sizeof(cplx));
  E[0] = 1.0;
  for (int q = 0; q < n; q++) {
    int la = bra->dim[q], lb = ket->dim[q];
    int ra = bra->dim[q + 1], rb = ket->dim[q + 1];
    const cplx *B = bra->A[q], *K = ket->A[q];
    const cplx *P = PAULI_M[pidx ? pidx[q] : 0];
    /* F[a,s',b'] = sum_a' E[a,a'] K[a',s',b'] (rows a on separate threads; every
       entry is summed over a' in increasing order, as in a serial run) */
    cplx *F = (cplx *)xalloc(sizeof(cplx) * (size_t)la * 2 * rb);
#pragma omp parallel for schedule(static) if ((long)la * lb * rb >= 65536)
    for (int a = 0; a < la; a++)
      for (int ap = 0; ap < lb; ap++) {
        cplx e = E[(size_t)a * lb + ap];
        if (e == 0.0) continue;
        for (int sb = 0; sb < 2 * rb; sb++) F[(size_t)a * 2 * rb + sb] += e * K[(size_t)ap * 2 * rb + sb];
      }
    /* F2[a,s,b'] = sum_s' P[s,s'] F[a,s',b'] */
    cplx *F2 = (cplx *)xalloc(sizeof(cplx) * (size_t)la * 2 * rb);
    for (int a = 0; a < la; a++)
      for (int s = 0; s < 2; s++)
        for (int bp = 0; bp < rb; bp++) {
          cplx acc = 0.0;
          for (int sp = 0; sp < 2; sp++) acc += P[2 * s + sp] * F[((size_t)a * 2 + sp) * rb + bp];
          F2[((size_t)a * 2 + s) * rb + bp] = acc;
        }
    free(F);
    /* E'[b,b'] = sum_{a,s} conj(B[a,s,b]) F2[a,s,b'] (rows b on separate
       threads; every entry is summed over (a, s) in increasing order) */
    cplx *E2 = (cplx *)xalloc(sizeof(cplx) * (size_t)ra * rb);
#pragma omp parallel for schedule(static) if ((long)ra * la * rb >= 65536)
    for (int b = 0; b < ra; b++)
      for (int a = 0; a < la; a++)
        for (int s = 0; s < 2; s++) {
          cplx w = conj(B[((size_t)a * 2 + s) * ra + b]);
          if (w == 0.0) continue;
          const cplx *f = F2 + ((size_t)a * 2 + s) * rb;
          cplx *o = E2 + (size_t)b * rb;
          for (int bp = 0; bp < rb; bp++) o[bp] += w * f[bp];
        }
    free(F2);
    free(E);
    E = E2;
  }
  cplx v = E[0];
  free(E);
  return v;
}

int om_expect_pauli(const om_mps *m, const char *pauli, double *re, double *im) {
  int *pidx = (int *)xalloc(sizeof(int) * m->n);
  for (int q = 0; q < m->n; q++) {
    pidx[q] = pauli_index(pauli[q]);
    if (pidx[q] < 0) { free(pidx); return OM_E_ARG; }
  }
  cplx num = transfer(m, m, pidx);
  cplx den = transfer(m, m, NULL);
  free(pidx);
  cplx v = num / den;
  if (re) *re = creal(v);
  if (im) *im = cimag(v);
  return OM_OK;
}

int om_norm2(const om_mps *m, double *out) {
  *out = creal(transfer(m, m, NULL));
  return OM_OK;
}

/* <a|b> */
int om_overlap(const om_mps *a, const om_mps *b, double *re, double *im) {
  if (a->n != b->n) return OM_E_ARG;
  cplx v = transfer(a, b, NULL);
  *re = creal(v);
  *im = cimag(v);
  return OM_OK;
}

/* <bits|psi> = prod_q A_q[:, bits[q], :] */
int om_amplitude(const om_mps *m, const uint8_t *bits, double *re, double *im) {
  cplx *v = (cplx *)xalloc(sizeof(cplx));
  v[0] = 1.0;
  for (int q = 0; q < m->n; q++) {
    if (bits[q] > 1) { free(v); return OM_E_ARG; }
    int la = m->dim[q], rb = m->dim[q + 1];
    cplx *w = (cplx *)xalloc(sizeof(cplx) * rb);
    for (int a = 0; a < la; a++)
      for (int b = 0; b < rb; b++) w[b] += v[a] * m->A[q][((size_t)a * 2 + bits[q]) * rb + b];
    free(v);
    v = w;
  }
  *re = creal(v[0]);
  *im = cimag(v[0]);
  free(v);
  return OM_OK;
}

/* Dense state, index x = sum_q b_q 2^q; out has 2^n interleaved entries. */
int om_statevector(const om_mps *m, double *out) {
  int n = m->n;
  if (n > 24) return OM_E_ARG;
  size_t cur = 1;
  cplx *T = (cplx *)xalloc(sizeof(cplx)); /* T[x][b], bond dim 1 */
  T[0] = 1.0;
  for (int q = 0; q < n; q++) {
    int la = m->dim[q], rb = m->dim[q + 1];
    cplx *T2 = (cplx *)xalloc(sizeof(cplx) * cur * 2 * rb);
    for (size_t x = 0; x < cur; x++)
      for (int s = 0; s < 2; s++)
        for (int a = 0; a < la; a++) {
          cplx w = T[x * la + a];
          if (w == 0.0) continue;
          const cplx *row = m->A[q] + ((size_t)a * 2 + s) * rb;
          cplx *o = T2 + (x + (size_t)s * cur) * rb;
          for (int b = 0; b < rb; b++) o[b] += w * row[b];
        }
    free(T);
    T = T2;
    cur *= 2;
  }
  memcpy(out, T, sizeof(cplx) * cur);
  free(T);
  return OM_OK;
}

/* ----------------------------------------------------------------- sampling
 * Perfect sampling ("measure all", Sec. III.A; Ferris and Vidal, Phys. Rev. B
 * 85, 165146 (2012)): the qubits are drawn one at a time, each from its
 * marginal given the bits already drawn, and the drawn bit is projected out
 * and the rest renormalised before the next qubit.
 *
 * Order (a reading; the paper does not fix it): qubit n-1 first, then n-2,
 * ..., 0.  With v the contraction A_{q+1}^{s_{q+1}} ... A_{n-1}^{s_{n-1}} of the
 * drawn sites and
 *   E_q = sum over s_0..s_{q-1} of L^H L,  L = A_0^{s_0} ... A_{q-1}^{s_{q-1}}
 * (the Gram matrix of the left block; E_0 = 1), the weight of s_q = s is
 * p_s = w_s^H E_q w_s with w_s = A_q^s v.  Bit 0 is taken when
 * u < p_0 / (p_0 + p_1), else bit 1; then v = w_bit / sqrt(p_bit).  E_q keeps
 * the marginals exact in any gauge (it is the identity when the left block is
 * orthonormal).
 *
 * u: shots x n uniforms in [0, 1); u[shot * n + q] decides qubit q.
 * bits: shots x n bytes (bits[shot * n + q] = s_q).
 * logp (may be NULL): per shot, the sum over qubits of log(p_bit / (p_0 + p_1)),
 * i.e. log(|<x|psi>|^2 / <psi|psi>) for the drawn string x.
 */

/* E[q] for q = 0..n-1, each dim[q] x dim[q] row-major. */
static cplx **left_envs(const om_mps *m) {
  const int n = m->n;
  cplx **E = (cplx **)xalloc(sizeof(cplx *) * n);
  E[0] = (cplx *)xalloc(sizeof(cplx));
  E[0][0] = 1.0;
  for (int q = 0; q + 1 < n; q++) {
    const int la = m->dim[q], rb = m->dim[q + 1];
    const cplx *A = m->A[q];
    cplx *F = (cplx *)xalloc(sizeof(cplx) * (size_t)la * 2 * rb); /* F = E_q A_q */
    for (int a = 0; a < la; a++)
      for (int ap = 0; ap < la; ap++) {
        cplx e = E[q][(size_t)a * la + ap];
        for (int sb = 0; sb < 2 * rb; sb++) F[(size_t)a * 2 * rb + sb] += e * A[(size_t)ap * 2 * rb + sb];
      }
    cplx *En = (cplx *)xalloc(sizeof(cplx) * (size_t)rb * rb); /* A_q^H F */
    for (int a = 0; a < la; a++)
      for (int s = 0; s < 2; s++)
        for (int b = 0; b < rb; b++) {
          cplx w = conj(A[((size_t)a * 2 + s) * rb + b]);
          const cplx *f = F + ((size_t)a * 2 + s) * rb;
          for (int bp = 0; bp < rb; bp++) En[(size_t)b * rb + bp] += w * f[bp];
        }
    free(F);
    E[q + 1] = En;
  }
  return E;
}

/* w^H E w for an la x la matrix E */
static double env_weight(const cplx *E, const cplx *w, int la) {
  cplx acc = 0.0;
  for (int a = 0; a < la; a++) {
    cplx t = 0.0;
    for (int ap = 0; ap < la; ap++) t += E[(size_t)a * la + ap] * w[ap];
    acc += conj(w[a]) * t;
  }
  return creal(acc);
}

int om_sample(const om_mps *m, int shots, const double *u, uint8_t *bits, double *logp) {
  if (shots < 0) return OM_E_ARG;
  const int n = m->n;
  for (size_t i = 0; i < (size_t)shots * n; i++)
    if (!(u[i] >= 0.0 && u[i] < 1.0)) return OM_E_ARG;
  cplx **E = left_envs(m);
  int chi = 1;
  for (int q = 0; q <= n; q++) chi = m->dim[q] > chi ? m->dim[q] : chi;
#pragma omp parallel for schedule(dynamic) if (shots >= 8)
  for (int shot = 0; shot < shots; shot++) {
    cplx *v = (cplx *)xalloc(sizeof(cplx) * chi);
    cplx *w0 = (cplx *)xalloc(sizeof(cplx) * chi), *w1 = (cplx *)xalloc(sizeof(cplx) * chi);
    double lp = 0.0;
    v[0] = 1.0;
    for (int q = n - 1; q >= 0; q--) {
      const int la = m->dim[q], rb = m->dim[q + 1];
      const cplx *A = m->A[q];
      for (int a = 0; a < la; a++) {
        cplx t0 = 0.0, t1 = 0.0;
        for (int b = 0; b < rb; b++) {
          t0 += A[((size_t)a * 2 + 0) * rb + b] * v[b];
          t1 += A[((size_t)a * 2 + 1) * rb + b] * v[b];
        }
        w0[a] = t0;
        w1[a] = t1;
      }
      const double p0 = env_weight(E[q], w0, la), p1 = env_weight(E[q], w1, la);
      const int bit = u[(size_t)shot * n + q] < p0 / (p0 + p1) ? 0 : 1;
      const double pb = bit ? p1 : p0;
      bits[(size_t)shot * n + q] = (uint8_t)bit;
      lp += log(pb / (p0 + p1));
      const cplx *wb = bit ? w1 : w0;
      const double r = 1.0 / sqrt(pb);
      for (int a = 0; a < la; a++) v[a] = wb[a] * r;
    }
    if (logp) logp[shot] = lp;
    free(v);
    free(w0);
    free(w1);
  }
  for (int q = 0; q < n; q++) free(E[q]);
  free(E);
  return OM_OK;
}
