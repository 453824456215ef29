// QR preconditioning of the Jacobi SVD (Drmac and Veselic, "New fast and
// accurate Jacobi SVD algorithm", SIAM J. Matrix Anal. Appl. 29(4), 2008).
//
// The paper decomposes the merged two-site tensor with a Jacobi SVD on the GPU
// (Sec. IV.A, cusolverDnZgesvdj).  One-sided Jacobi applied to M directly
// needs many sweeps on these graded matrices; applied to R2^H from
//
//   M = Q1 R1      (m x n, m >= n, Householder)
//   R1^H = Q2 R2   (n x n, Householder; Q2 is not needed)
//
// it needs about half as many.  With R2^H = W S V^H (W from the Jacobi),
// M = (Q1 W) S (Q2 V)^H, so the left singular vectors are U = Q1 [W; 0] and
// no rotation has to be accumulated.
//
// Householder QR in the LAPACK convention: H = I - tau v v^H with v(0) = 1,
// H^H [alpha; x] = [beta; 0], beta real; a panel of QNB reflectors is
// I - V T V^H (compact WY, T upper triangular).  Everything is float64.
#include "tnsim_internal.h"
#include "tn_complex.h"

namespace tn {

struct QrView {
  double2 *A;
  int ld, rows, cols;
};

// stage 0: M in Qm (m x n); stage 1: R1^H in X (n x n)
__device__ __forceinline__ QrView qr_view(const GateDesc &d, int stage) {
  if (stage == 0) return QrView{d.Qm, d.ldq, d.m, d.n};
  return QrView{d.X, d.ldx, d.n, d.n};
}

__device__ __forceinline__ double2 *qr_tfac(const GateDesc &d, int stage, int panel) {
  const int np = d.colsPad / QNB;  // panels per stage
  return d.Tq + ((size_t)stage * np + panel) * (QNB * QNB);
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// ---------------------------------------------------------------- panel

constexpr int QP_THREADS = 512;
constexpr int QP_RPT = QR_MAX_ROWS / QP_THREADS;  // rows per thread
constexpr int QP_WAVES = QP_THREADS / 64;

// Factor columns j0 .. j0+w-1 (rows j0 ..) of one gate's matrix: one
// workgroup per gate, the panel in registers (thread t holds panel rows
// t, t + 512, ...).  Writes R's panel rows, the reflectors below the diagonal
// and the panel's T factor.
__global__ __launch_bounds__(QP_THREADS) void k_qr_panel(const GateDesc *descs, int stage,
                                                        int panel) {
  const GateDesc &d = descs[blockIdx.x];
  if (!d.qr) return;
  const QrView q = qr_view(d, stage);
  const int j0 = panel * QNB;
  if (j0 >= q.cols) return;
  const int w = min(QNB, q.cols - j0);
  const int nr = q.rows - j0;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  __shared__ double2 red[QP_WAVES][QNB];
  __shared__ double2 bsum[QNB];
  __shared__ double2 Ts[QNB][QNB];
  __shared__ double2 s_alpha, s_tau, s_scale;
  __shared__ double s_beta;

  double2 a[QP_RPT][QNB];
#pragma unroll
  for (int i = 0; i < QP_RPT; i++) {
    const int lr = tid + QP_THREADS * i;
#pragma unroll
    for (int c = 0; c < QNB; c++)
      a[i][c] = (lr < nr && c < w) ? q.A[(size_t)(j0 + c) * q.ld + j0 + lr]
                                   : make_double2(0.0, 0.0);
  }
  if (tid < QNB * QNB) Ts[tid / QNB][tid % QNB] = make_double2(0.0, 0.0);

#pragma unroll
  for (int c = 0; c < QNB; c++) {
    if (c >= w) break;
    // ||x||^2 below the diagonal of column c
    double xn = 0.0;
#pragma unroll
    for (int i = 0; i < QP_RPT; i++) {
      const int lr = tid + QP_THREADS * i;
      if (lr > c) xn += cabs2(a[i][c]);
    }
    xn = wave_sum(xn);
    if (tid == c) s_alpha = a[0][c];
    if (lane == 0) red[wave][0] = make_double2(xn, 0.0);
    __syncthreads();
    if (tid == 0) {
      double x2 = 0.0;
      for (int v = 0; v < QP_WAVES; v++) x2 += red[v][0].x;
      const double2 al = s_alpha;
      if (x2 == 0.0 && al.y == 0.0) {  // already triangular: H = I
        s_tau = make_double2(0.0, 0.0);
        s_beta = al.x;
        s_scale = make_double2(0.0, 0.0);
      } else {
        const double beta = -copysign(sqrt(cabs2(al) + x2), al.x);
        s_tau = make_double2((beta - al.x) / beta, -al.y / beta);
        const double2 dn = make_double2(al.x - beta, al.y);  // alpha - beta
        const double inv = 1.0 / cabs2(dn);
        s_scale = make_double2(dn.x * inv, -dn.y * inv);  // 1 / (alpha - beta)
        s_beta = beta;
      }
    }
    __syncthreads();
    const double2 tau = s_tau, scale = s_scale;
    // reflector below the diagonal, beta on it; vr = v at this thread's rows
    double2 vr[QP_RPT];
#pragma unroll
    for (int i = 0; i < QP_RPT; i++) {
      const int lr = tid + QP_THREADS * i;
      if (lr > c) {
        a[i][c] = cmul(a[i][c], scale);
        vr[i] = a[i][c];
      } else if (lr == c) {
        a[i][c] = make_double2(s_beta, 0.0);
        vr[i] = make_double2(1.0, 0.0);
      } else {
        vr[i] = make_double2(0.0, 0.0);
      }
    }
    // one reduction for both: s_p = v^H a_p (p > c, to update the panel) and
    // g_p = v_p^H v (p < c, for the T factor)
    double2 part[QNB];
#pragma unroll
    for (int p = 0; p < QNB; p++) {
      double2 acc = make_double2(0.0, 0.0);
      if (p != c && p < w) {
#pragma unroll
        for (int i = 0; i < QP_RPT; i++) {
          if (p > c)
            cfmac(acc, vr[i], a[i][p]);  // conj(v) a_p
          else
            cfmac(acc, a[i][p], vr[i]);  // conj(v_p) v (rows >= c, where v_p is stored)
        }
      }
      part[p] = make_double2(wave_sum(acc.x), wave_sum(acc.y));
    }
    if (lane == 0) {
#pragma unroll
      for (int p = 0; p < QNB; p++) red[wave][p] = part[p];
    }
    __syncthreads();
    if (tid < QNB) {
      double2 s = make_double2(0.0, 0.0);
      for (int v = 0; v < QP_WAVES; v++) s = cadd(s, red[v][tid]);
      bsum[tid] = s;
    }
    __syncthreads();
    // a_p <- a_p - conj(tau) v s_p for the later panel columns
    const double2 ctau = cconj(tau);
#pragma unroll
    for (int p = 0; p < QNB; p++) {
      if (p > c && p < w) {
        const double2 f = cmul(ctau, bsum[p]);
#pragma unroll
        for (int i = 0; i < QP_RPT; i++) a[i][p] = csub(a[i][p], cmul(vr[i], f));
      }
    }
    // T(0:c, c) = -tau T(0:c, 0:c) g(0:c), T(c, c) = tau
    if (tid < c) {
      double2 s = make_double2(0.0, 0.0);
      for (int l = tid; l < c; l++) s = cadd(s, cmul(Ts[tid][l], bsum[l]));
      Ts[tid][c] = cmul(make_double2(-tau.x, -tau.y), s);
    }
    if (tid == c) Ts[c][c] = tau;
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < QP_RPT; i++) {
    const int lr = tid + QP_THREADS * i;
    if (lr < nr) {
#pragma unroll
      for (int c = 0; c < QNB; c++)
        if (c < w) q.A[(size_t)(j0 + c) * q.ld + j0 + lr] = a[i][c];
    }
  }
  double2 *T = qr_tfac(d, stage, panel);
  if (tid < QNB * QNB) T[tid] = Ts[tid / QNB][tid % QNB];
}

void launch_qr_panel(hipStream_t st, const GateDesc *d, int ng, int stage, int panel) {
  if (ng <= 0) return;
  hipLaunchKernelGGL(k_qr_panel, dim3(ng), dim3(QP_THREADS), 0, st, d, stage, panel);
}

// ---------------------------------------------------------------- block update

constexpr int QU_COLS = 32;  // target columns per workgroup
constexpr int QU_ROWS = 64;  // rows per LDS chunk

// apply = 0: B = A(j0:, j0+w:) <- (I - V T V^H)^H B   (trailing part of a factor)
// apply = 1: B = U(j0:, 0:k)   <- (I - V T V^H) B     (U = Q1 [W; 0], panels in reverse)
// One workgroup per 32 target columns: S = V^H B over all rows, Y = op(T) S,
// then B -= V Y.
__global__ __launch_bounds__(256) void k_qr_update(const GateDesc *descs, int stage, int panel,
                                                   int apply) {
  const GateDesc &d = descs[blockIdx.y];
  if (!d.qr) return;
  const QrView q = qr_view(d, apply ? 0 : stage);
  const int j0 = panel * QNB;
  if (j0 >= q.cols) return;
  const int w = min(QNB, q.cols - j0);
  double2 *B;
  int ldb, rows, ncols;
  if (apply) {
    B = d.U;
    ldb = d.ldu;
    rows = d.m;
    ncols = d.sc->k;
  } else {
    B = q.A + (size_t)(j0 + w) * q.ld;
    ldb = q.ld;
    rows = q.rows;
    ncols = q.cols - j0 - w;
  }
  const int c0 = blockIdx.x * QU_COLS;
  if (c0 >= ncols) return;
  const int nc = min(QU_COLS, ncols - c0);
  B += (size_t)c0 * ldb;
  const double2 *V = q.A + (size_t)j0 * q.ld;  // reflector p is column p of V, from row j0 + p

  __shared__ double2 Vs[QU_ROWS][QNB + 1];
  __shared__ double2 Bs[QU_ROWS][QU_COLS + 1];
  __shared__ double2 S[QNB][QU_COLS];
  __shared__ double2 Y[QNB][QU_COLS];
  __shared__ double2 Tl[QNB][QNB];
  const int tid = threadIdx.x;
  const double2 *T = qr_tfac(d, apply ? 0 : stage, panel);
  if (tid < QNB * QNB) Tl[tid / QNB][tid % QNB] = T[tid];

  // reflector entry p at row r (absolute): 1 on the diagonal, stored below it
  auto vget = [&](int r, int p) -> double2 {
    if (p >= w) return make_double2(0.0, 0.0);
    const int dr = r - (j0 + p);
    if (dr < 0) return make_double2(0.0, 0.0);
    if (dr == 0) return make_double2(1.0, 0.0);
    return V[(size_t)p * q.ld + r];
  };

  // phase 1: S = V^H B; thread (p, cc) owns one entry
  const int sp = tid / QU_COLS, scc = tid % QU_COLS;  // 8 x 32 = 256 threads
  double2 sacc = make_double2(0.0, 0.0);
  for (int r0 = j0; r0 < rows; r0 += QU_ROWS) {
    for (int e = tid; e < QU_ROWS * QNB; e += 256) {
      const int r = e % QU_ROWS, p = e / QU_ROWS;
      Vs[r][p] = (r0 + r < rows) ? vget(r0 + r, p) : make_double2(0.0, 0.0);
    }
    for (int e = tid; e < QU_ROWS * QU_COLS; e += 256) {
      const int r = e % QU_ROWS, cc = e / QU_ROWS;
      Bs[r][cc] = (r0 + r < rows && cc < nc) ? B[(size_t)cc * ldb + r0 + r]
                                              : make_double2(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll 8
    for (int r = 0; r < QU_ROWS; r++) cfmac(sacc, Vs[r][sp], Bs[r][scc]);
    __syncthreads();
  }
  S[sp][scc] = sacc;
  __syncthreads();
  // phase 2: Y = T^H S (factor) or T S (apply)
  {
    double2 y = make_double2(0.0, 0.0);
    for (int l = 0; l < QNB; l++) {
      const double2 t = apply ? Tl[sp][l] : cconj(Tl[l][sp]);
      y = cadd(y, cmul(t, S[l][scc]));
    }
    Y[sp][scc] = y;
  }
  __syncthreads();
  // phase 3: B -= V Y; lanes along rows, each thread 8 columns
  const int rl = tid % QU_ROWS, cg = tid / QU_ROWS;  // 64 rows x 4 column groups
  for (int r0 = j0; r0 < rows; r0 += QU_ROWS) {
    const int r = r0 + rl;
    if (r < rows) {
      double2 v[QNB];
#pragma unroll
      for (int p = 0; p < QNB; p++) v[p] = vget(r, p);
      for (int cc = cg; cc < nc; cc += 4) {
        double2 s = make_double2(0.0, 0.0);
#pragma unroll
        for (int p = 0; p < QNB; p++) s = cadd(s, cmul(v[p], Y[p][cc]));
        double2 *bp = B + (size_t)cc * ldb + r;
        *bp = csub(*bp, s);
      }
    }
  }
}

void launch_qr_update(hipStream_t st, const GateDesc *d, int ng, int stage, int panel, int apply,
                      int max_cols) {
  if (ng <= 0 || max_cols <= 0) return;
  hipLaunchKernelGGL(k_qr_update, dim3((max_cols + QU_COLS - 1) / QU_COLS, ng), dim3(256), 0, st,
                     d, stage, panel, apply);
}

// ---------------------------------------------------------------- triangular transposes

constexpr int QT = 32;

// X (n x n) = R1^H: lower triangle conj(R1)^T, upper triangle zero.  R1 is
// the upper triangle of Qm.  grid: (tiles of X rows, tiles of X columns, gate)
__global__ __launch_bounds__(256) void k_qr_r1h(const GateDesc *descs) {
  const GateDesc &d = descs[blockIdx.z];
  if (!d.qr) return;
  const int n = d.n;
  const int i0 = blockIdx.x * QT, jc0 = blockIdx.y * QT;  // X rows i, X columns j
  if (i0 >= n || jc0 >= n) return;
  __shared__ double2 t[QT][QT + 1];
  const int tid = threadIdx.x;
  // X(i, j) = conj(R1(j, i)) = conj(Qm[i * ldq + j]) for i >= j
  for (int e = tid; e < QT * QT; e += 256) {
    const int jj = e % QT, ii = e / QT;  // read along j (rows of Qm column i)
    const int i = i0 + ii, j = jc0 + jj;
    t[ii][jj] = (i < n && j < n && i >= j) ? cconj(d.Qm[(size_t)i * d.ldq + j])
                                           : make_double2(0.0, 0.0);
  }
  __syncthreads();
  for (int e = tid; e < QT * QT; e += 256) {
    const int ii = e % QT, jj = e / QT;  // write along i (rows of X column j)
    const int i = i0 + ii, j = jc0 + jj;
    if (i < n && j < n) d.X[(size_t)j * d.ldx + i] = t[ii][jj];
  }
}

void launch_qr_r1h(hipStream_t st, const GateDesc *d, int ng, int max_n) {
  if (ng <= 0 || max_n <= 0) return;
  const int nt = (max_n + QT - 1) / QT;
  hipLaunchKernelGGL(k_qr_r1h, dim3(nt, nt, ng), dim3(256), 0, st, d);
}

// In place in X: R2 (upper triangle, reflectors below) -> R2^H (lower
// triangle, zero above).  The workgroup of tile pair (I, J), I <= J, reads
// the upper tile (I, J) and writes tiles (J, I) and (I, J); nothing else
// touches them.
__global__ __launch_bounds__(256) void k_qr_r2h(const GateDesc *descs) {
  const GateDesc &d = descs[blockIdx.z];
  if (!d.qr) return;
  const int n = d.n;
  const int I = blockIdx.x, J = blockIdx.y;
  if (I > J || I * QT >= n || J * QT >= n) return;
  __shared__ double2 t[QT][QT + 1];  // t[r][c] = R2(I*QT + r, J*QT + c)
  const int tid = threadIdx.x;
  for (int e = tid; e < QT * QT; e += 256) {
    const int r = e % QT, c = e / QT;
    const int gr = I * QT + r, gc = J * QT + c;
    t[r][c] = (gr < n && gc < n && gr <= gc) ? d.X[(size_t)gc * d.ldx + gr]
                                             : make_double2(0.0, 0.0);
  }
  __syncthreads();
  // X(J*QT + c, I*QT + r) = conj(R2(I*QT + r, J*QT + c)); upper entries cleared
  for (int e = tid; e < QT * QT; e += 256) {
    const int c = e % QT, r = e / QT;  // along the rows c of column I*QT + r
    const int gi = J * QT + c, gj = I * QT + r;
    if (gi < n && gj < n) d.X[(size_t)gj * d.ldx + gi] = cconj(t[r][c]);
  }
  for (int e = tid; e < QT * QT; e += 256) {
    const int r = e % QT, c = e / QT;
    const int gr = I * QT + r, gc = J * QT + c;
    if (gr < n && gc < n && gr < gc) d.X[(size_t)gc * d.ldx + gr] = make_double2(0.0, 0.0);
  }
}

void launch_qr_r2h(hipStream_t st, const GateDesc *d, int ng, int max_n) {
  if (ng <= 0 || max_n <= 0) return;
  const int nt = (max_n + QT - 1) / QT;
  hipLaunchKernelGGL(k_qr_r2h, dim3(nt, nt, ng), dim3(256), 0, st, d);
}

// ---------------------------------------------------------------- U = [W_k; 0]

// Column j of U: the kept Jacobi column perm[j] divided by its norm (rows
// 0..n-1), zero below.  grid: (row tiles of 64, kept columns, gate)
__global__ __launch_bounds__(64) void k_qr_gather(const GateDesc *descs) {
  const GateDesc &d = descs[blockIdx.z];
  if (!d.qr) return;
  const int j = blockIdx.y;
  if (j >= d.sc->k) return;
  const int r = blockIdx.x * 64 + threadIdx.x;
  if (r >= d.m) return;
  const int col = d.perm[j];
  const double inv = 1.0 / sqrt(d.sig2[col]);
  d.U[(size_t)j * d.ldu + r] =
      r < d.n ? cscale(d.X[(size_t)col * d.ldx + r], inv) : make_double2(0.0, 0.0);
}

void launch_qr_gather(hipStream_t st, const GateDesc *d, int ng, int max_m, int max_k) {
  if (ng <= 0 || max_m <= 0 || max_k <= 0) return;
  hipLaunchKernelGGL(k_qr_gather, dim3((max_m + 63) / 64, max_k, ng), dim3(64), 0, st, d);
}

}  // namespace tn
