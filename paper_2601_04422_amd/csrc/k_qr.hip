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
#include "tn_buffer.h"

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

// T factors: those of the QNB-column panels of both stages, then those of
// the QG-column groups (QG / QNB panels each) of both stages.
__device__ __forceinline__ double2 *qr_tfac(const GateDesc &d, int stage, int panel) {
  const int np = d.colsPad / QNB;  // panels per stage
  return d.Tq + ((size_t)stage * np + panel) * (QNB * QNB);
}
__device__ __forceinline__ double2 *qr_tgrp(const GateDesc &d, int stage, int group) {
  const int np = d.colsPad / QNB, ngp = d.colsPad / QG;
  return d.Tq + (size_t)2 * np * (QNB * QNB) + ((size_t)stage * ngp + group) * (QG * QG);
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

constexpr int QU_ROWS = 64;  // rows per LDS chunk

// Apply a block reflector of NB Householder vectors (a panel, NB = QNB, or a
// group of panels, NB = QG) to COLS target columns per workgroup:
//   apply = 0: B = A(j0:, first:last) <- (I - V T V^H)^H B  (factoring: the
//              columns after the block, up to col_end)
//   apply = 1: B = U(j0:, 0:k) <- (I - V T V^H) B          (U = Q1 [W; 0])
// S = V^H B over all rows, Y = op(T) S, B -= V Y; V is staged in LDS.
template <int NB, int COLS>
__device__ void qr_block_update(const GateDesc &d, const QrView q, int j0, const double2 *T,
                                int apply, int col_end) {
  static_assert((NB * COLS) % 256 == 0, "whole entries per thread");
  constexpr int EPT = NB * COLS / 256;
  if (j0 >= q.cols) return;
  const int w = min(NB, q.cols - j0);
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
    ncols = min(col_end, q.cols) - j0 - w;
  }
  const int c0 = blockIdx.x * COLS;
  if (c0 >= ncols) return;
  const int nc = min(COLS, ncols - c0);
  B += (size_t)c0 * ldb;
  const double2 *V = q.A + (size_t)j0 * q.ld;  // reflector p: column p, from row j0 + p

  __shared__ double2 Vs[QU_ROWS][NB + 1];
  __shared__ double2 Bs[QU_ROWS][COLS + 1];
  __shared__ double2 S[NB][COLS];
  __shared__ double2 Y[NB][COLS];
  __shared__ double2 Tl[NB][NB + 1];
  const int tid = threadIdx.x;
  for (int e = tid; e < NB * NB; e += 256) Tl[e / NB][e % NB] = T[e];

  auto load_v = [&](int r0) {  // rows r0 .. r0+63 of V: 1 on the diagonal, stored below
    for (int e = tid; e < QU_ROWS * NB; e += 256) {
      const int r = e % QU_ROWS, p = e / QU_ROWS, gr = r0 + r, dr = gr - (j0 + p);
      double2 v = make_double2(0.0, 0.0);
      if (p < w && gr < rows && dr >= 0)
        v = dr == 0 ? make_double2(1.0, 0.0) : V[(size_t)p * q.ld + gr];
      Vs[r][p] = v;
    }
  };

  // phase 1: S = V^H B
  double2 sacc[EPT];
#pragma unroll
  for (int e = 0; e < EPT; e++) sacc[e] = make_double2(0.0, 0.0);
  for (int r0 = j0; r0 < rows; r0 += QU_ROWS) {
    load_v(r0);
    for (int e = tid; e < QU_ROWS * COLS; e += 256) {
      const int r = e % QU_ROWS, cc = e / QU_ROWS;
      Bs[r][cc] = (r0 + r < rows && cc < nc) ? B[(size_t)cc * ldb + r0 + r]
                                              : make_double2(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < EPT; e++) {
      const int id = tid + 256 * e, p = id / COLS, cc = id % COLS;
#pragma unroll 8
      for (int r = 0; r < QU_ROWS; r++) cfmac(sacc[e], Vs[r][p], Bs[r][cc]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int e = 0; e < EPT; e++) {
    const int id = tid + 256 * e;
    S[id / COLS][id % COLS] = sacc[e];
  }
  __syncthreads();
  // phase 2: Y = T^H S (factor) or T S (apply)
#pragma unroll
  for (int e = 0; e < EPT; e++) {
    const int id = tid + 256 * e, p = id / COLS, cc = id % COLS;
    double2 y = make_double2(0.0, 0.0);
    for (int l = 0; l < NB; l++) {
      const double2 t = apply ? Tl[p][l] : cconj(Tl[l][p]);
      y = cadd(y, cmul(t, S[l][cc]));
    }
    Y[p][cc] = y;
  }
  __syncthreads();
  // phase 3: B -= V Y; lanes along rows
  const int rl = tid % QU_ROWS, cg = tid / QU_ROWS;  // 64 rows x 4 column groups
  for (int r0 = j0; r0 < rows; r0 += QU_ROWS) {
    load_v(r0);
    __syncthreads();
    const int r = r0 + rl;
    if (r < rows) {
      for (int cc = cg; cc < nc; cc += 4) {
        double2 acc = make_double2(0.0, 0.0);
#pragma unroll 8
        for (int p = 0; p < NB; p++) cfma(acc, Vs[rl][p], Y[p][cc]);
        double2 *bp = B + (size_t)cc * ldb + r;
        *bp = csub(*bp, acc);
      }
    }
    __syncthreads();
  }
}

constexpr int QU_COLS = 32;   // target columns per workgroup, panel updates

// One panel's reflectors on the columns after it up to col_end (inside its
// group while the group is being factored).
__global__ __launch_bounds__(256) void k_qr_update(const GateDesc *descs, int stage, int panel,
                                                   int col_end) {
  const GateDesc &d = descs[blockIdx.y];
  if (!d.qr) return;
  qr_block_update<QNB, QU_COLS>(d, qr_view(d, stage), panel * QNB, qr_tfac(d, stage, panel), 0,
                                col_end);
}

void launch_qr_update(hipStream_t st, const GateDesc *d, int ng, int stage, int panel,
                      int col_end, int max_cols) {
  if (ng <= 0 || max_cols <= 0) return;
  hipLaunchKernelGGL(k_qr_update, dim3((max_cols + QU_COLS - 1) / QU_COLS, ng), dim3(256), 0, st,
                     d, stage, panel, col_end);
}

// ------------------------------------------------ group update on matrix cores
//
// A group's QG reflectors on everything after the group (apply = 0), or on U
// (apply = 1, stage-0 groups in reverse order), in three launches so that the
// rows are spread over workgroups as well as the columns:
//   k_qrg_s : partial S = V^H B over a chunk of QR_RC rows      (per chunk)
//   k_qrg_y : Y = op(T) sum_chunks S                           (per column tile)
//   k_qrg_b : B -= V Y over a chunk of rows                     (per chunk)
// Partial sums and Y go to a scratch buffer that is idle at that time (U while
// factoring, the Jacobi matrix once its columns have been gathered into U).
// Fixed summation order: results do not depend on scheduling.

typedef double qd4_t __attribute__((ext_vector_type(4)));

// v_mfma_f64_16x16x4f64: lane l supplies A[l%16][l/16] and B[l/16][l%16];
// result entry v of lane l is D[l/16 + 4v][l%16].
__device__ __forceinline__ qd4_t qmfma(double a, double b, qd4_t c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int QGT = 32;     // target columns per workgroup

struct QrTarget {
  double2 *B;     // first target column
  int ldb, rows;  // rows of B (all of them; the reflectors start at row j0)
  int ncols;      // target columns
  double2 *scr;   // scratch: partial S then Y, QG rows of ldS each
  int ldS;
};

__device__ __forceinline__ QrTarget qr_target(const GateDesc &d, const QrView &q, int j0, int w,
                                              int apply) {
  QrTarget t;
  t.ldS = d.colsPad;
  if (apply) {
    t.B = d.U;
    t.ldb = d.ldu;
    t.rows = d.m;
    t.ncols = d.sc->k;
    t.scr = d.X;
  } else {
    t.B = q.A + (size_t)(j0 + w) * q.ld;
    t.ldb = q.ld;
    t.rows = q.rows;
    t.ncols = q.cols - j0 - w;
    t.scr = d.U;
  }
  return t;
}

// reflector p of the group at absolute row r: 1 on its diagonal, stored below
__device__ __forceinline__ double2 qr_vget(const QrView &q, int j0, int w, int r, int p) {
  if (p >= w || r >= q.rows) return make_double2(0.0, 0.0);
  const int dr = r - (j0 + p);
  if (dr < 0) return make_double2(0.0, 0.0);
  if (dr == 0) return make_double2(1.0, 0.0);
  return q.A[(size_t)(j0 + p) * q.ld + r];
}

__global__ __launch_bounds__(256) void k_qrg_s(const GateDesc *descs, int stage, int group,
                                               int apply) {
  const GateDesc &d = descs[blockIdx.z];
  if (!d.qr) return;
  const int stg = apply ? 0 : stage;
  const QrView q = qr_view(d, stg);
  const int j0 = group * QG;
  if (j0 >= q.cols) return;
  const int w = min(QG, q.cols - j0);
  const QrTarget t = qr_target(d, q, j0, w, apply);
  const int c0 = blockIdx.x * QGT;
  const int rbeg = j0 + blockIdx.y * QR_RC;
  if (c0 >= t.ncols || rbeg >= t.rows) return;
  const int rend = min(t.rows, rbeg + QR_RC);
  __shared__ double2 Vs[32][QG + 1];
  __shared__ double2 Bs[32][QGT + 1];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int l16 = lane & 15, lg = lane >> 4;
  const int tp = (wave >> 1) * 16, tc = (wave & 1) * 16;  // this wave's 16x16 tile of S
  qd4_t accR = {0.0, 0.0, 0.0, 0.0}, accI = {0.0, 0.0, 0.0, 0.0};
  // Rows come in chunks of 32, each thread holding 4 elements of V and 4 of
  // B per chunk.  Two chunks are in flight ahead of the one being
  // multiplied: buffer loads (counted apart from the LDS accesses), never
  // skipped, and masked only when written to LDS.
  static_assert(32 * QG == 4 * 256 && 32 * QGT == 4 * 256, "four elements per thread");
  const BufRes rA = make_res(q.A, q.ld * q.cols);
  const BufRes rB = make_res(t.B, t.ldb * t.ncols);
  auto load = [&](int r0, double2 *vv, double2 *bb) {
#pragma unroll
    for (int k = 0; k < 4; k++) {
      const int e = tid + 256 * k, r = e % 32, p = e / 32;
      vv[k] = bload(rA, (j0 + p) * q.ld + r0 + r);
      bb[k] = bload(rB, (c0 + p) * t.ldb + r0 + r);
    }
  };
  auto to_lds = [&](int r0, const double2 *vv, const double2 *bb) {
#pragma unroll
    for (int k = 0; k < 4; k++) {
      const int e = tid + 256 * k, r = e % 32, p = e / 32;
      const int rr = r0 + r, dr = rr - (j0 + p);  // reflector p: 1 on its diagonal, stored below
      const bool in = rr < rend;
      Vs[r][p] = (in && p < w && dr > 0) ? vv[k] : make_double2(in && p < w && dr == 0 ? 1.0 : 0.0, 0.0);
      Bs[r][p] = (in && c0 + p < t.ncols) ? bb[k] : make_double2(0.0, 0.0);
    }
  };
  auto chunk = [&]() {
#pragma unroll
    for (int kk = 0; kk < 32; kk += 4) {
      const double2 a = Vs[kk + lg][tp + l16];  // S = conj(V)^T B
      const double2 b = Bs[kk + lg][tc + l16];
      accR = qmfma(a.x, b.x, accR);
      accR = qmfma(a.y, b.y, accR);
      accI = qmfma(a.x, b.y, accI);
      accI = qmfma(-a.y, b.x, accI);
    }
  };
  const int nchunk = (rend - rbeg + 31) / 32;
  double2 va[4], ba[4], vb[4], bb[4];
  load(rbeg, va, ba);
  load(rbeg + 32, vb, bb);
  for (int c = 0; c < nchunk; c += 2) {  // an odd last chunk is followed by an all-zero one
    const int r0 = rbeg + 32 * c;
    to_lds(r0, va, ba);
    __syncthreads();
    load(r0 + 64, va, ba);
    chunk();
    __syncthreads();
    to_lds(r0 + 32, vb, bb);
    __syncthreads();
    load(r0 + 96, vb, bb);
    chunk();
    __syncthreads();
  }
  double2 *Sp = t.scr + (size_t)blockIdx.y * QG * t.ldS;
#pragma unroll
  for (int v = 0; v < 4; v++) {
    const int p = tp + lg + 4 * v, c = c0 + tc + l16;
    if (c < t.ncols) Sp[(size_t)p * t.ldS + c] = make_double2(accR[v], accI[v]);
  }
}

__global__ __launch_bounds__(256) void k_qrg_y(const GateDesc *descs, int stage, int group,
                                               int apply) {
  const GateDesc &d = descs[blockIdx.y];
  if (!d.qr) return;
  const int stg = apply ? 0 : stage;
  const QrView q = qr_view(d, stg);
  const int j0 = group * QG;
  if (j0 >= q.cols) return;
  const int w = min(QG, q.cols - j0);
  const QrTarget t = qr_target(d, q, j0, w, apply);
  const int c0 = blockIdx.x * QGT;
  if (c0 >= t.ncols) return;
  const int nch = (t.rows - j0 + QR_RC - 1) / QR_RC;
  __shared__ double2 S[QG][QGT + 1];
  __shared__ double2 Tl[QG][QG + 1];
  const double2 *T = qr_tgrp(d, stg, group);
  const int tid = threadIdx.x;
  for (int e = tid; e < QG * QG; e += 256) Tl[e / QG][e % QG] = T[e];
  for (int e = tid; e < QG * QGT; e += 256) {
    const int p = e / QGT, cc = e % QGT, c = c0 + cc;
    double2 sum = make_double2(0.0, 0.0);
    if (c < t.ncols)
      for (int ch = 0; ch < nch; ch++)
        sum = cadd(sum, t.scr[((size_t)ch * QG + p) * t.ldS + c]);
    S[p][cc] = sum;
  }
  __syncthreads();
  double2 *Yg = t.scr + (size_t)nch * QG * t.ldS;  // after the partials
  for (int e = tid; e < QG * QGT; e += 256) {
    const int p = e / QGT, cc = e % QGT, c = c0 + cc;
    double2 y = make_double2(0.0, 0.0);
    for (int l = 0; l < QG; l++) {
      const double2 tv = apply ? Tl[p][l] : cconj(Tl[l][p]);  // T or T^H
      y = cadd(y, cmul(tv, S[l][cc]));
    }
    if (c < t.ncols) Yg[(size_t)p * t.ldS + c] = y;
  }
}

__global__ __launch_bounds__(256) void k_qrg_b(const GateDesc *descs, int stage, int group,
                                               int apply) {
  const GateDesc &d = descs[blockIdx.z];
  if (!d.qr) return;
  const int stg = apply ? 0 : stage;
  const QrView q = qr_view(d, stg);
  const int j0 = group * QG;
  if (j0 >= q.cols) return;
  const int w = min(QG, q.cols - j0);
  const QrTarget t = qr_target(d, q, j0, w, apply);
  const int c0 = blockIdx.x * QGT;
  const int rbeg = j0 + blockIdx.y * QR_RC;
  if (c0 >= t.ncols || rbeg >= t.rows) return;
  const int rend = min(t.rows, rbeg + QR_RC);
  const int nch = (t.rows - j0 + QR_RC - 1) / QR_RC;
  __shared__ double2 Ys[QG][QGT + 1];
  const double2 *Yg = t.scr + (size_t)nch * QG * t.ldS;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int l16 = lane & 15, lg = lane >> 4;
  for (int e = tid; e < QG * QGT; e += 256) {
    const int p = e / QGT, cc = e % QGT;
    Ys[p][cc] = (c0 + cc < t.ncols) ? Yg[(size_t)p * t.ldS + c0 + cc] : make_double2(0.0, 0.0);
  }
  __syncthreads();
  // (V Y)^T = Y^T V^T: tiles of 16 target columns x 16 rows; the wave's tiles
  // are column tile (wave & 1) and every other row tile of the chunk
  // the next tile's V and B entries are loaded while the current tile is
  // multiplied (row tiles of one wave never overlap those of another)
  const int tc = (wave & 1) * 16;
  // Buffer loads and stores (counted apart from the LDS reads of Y), never
  // skipped: what lies past the chunk is masked when used, stores past it
  // are dropped by their offset.  Row tiles of one wave never overlap those
  // of another; the next tile's V and B are loaded while the current tile
  // is multiplied, into the other of two register sets.
  const BufRes rA = make_res(q.A, q.ld * q.cols);
  const BufRes rB = make_res(t.B, t.ldb * t.ncols);
  auto load = [&](int rt, double2 *vv, double2 *bb) {
    const int r = rt + l16;
#pragma unroll
    for (int k = 0; k < QG / 4; k++) vv[k] = bload(rA, (j0 + 4 * k + lg) * q.ld + r);  // V^T[k][row]
#pragma unroll
    for (int v = 0; v < 4; v++) bb[v] = bload(rB, (c0 + tc + lg + 4 * v) * t.ldb + r);
  };
  auto tile = [&](int rt, const double2 *vv, const double2 *bb) {
    const int r = rt + l16;
    qd4_t accR = {0.0, 0.0, 0.0, 0.0}, accI = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < QG / 4; k++) {
      const int p = 4 * k + lg, dr = r - (j0 + p);  // reflector p: 1 on its diagonal, stored below
      const bool ok = r < rend && p < w;
      const double2 b = (ok && dr > 0) ? vv[k] : make_double2(ok && dr == 0 ? 1.0 : 0.0, 0.0);
      const double2 a = Ys[4 * k + lg][tc + l16];  // Y^T[col][k]
      accR = qmfma(a.x, b.x, accR);
      accR = qmfma(-a.y, b.y, accR);
      accI = qmfma(a.x, b.y, accI);
      accI = qmfma(a.y, b.x, accI);
    }
#pragma unroll
    for (int v = 0; v < 4; v++) {
      const int c = c0 + tc + lg + 4 * v;
      const bool ok = r < rend && c < t.ncols;
      bstore_bytes(rB, ok ? (c * t.ldb + r) * 16 : BUF_DROP,
                   make_double2(bb[v].x - accR[v], bb[v].y - accI[v]));
    }
  };
  const int rt0 = rbeg + (wave >> 1) * 16;
  const int ntile = rt0 < rend ? (rend - rt0 + 31) / 32 : 0;
  double2 va[QG / 4], ba[4], vb[QG / 4], bb[4];
  load(rt0, va, ba);
  for (int i = 0; i < ntile; i += 2) {  // an odd last tile is followed by one past the chunk
    const int rt = rt0 + 32 * i;
    load(rt + 32, vb, bb);
    tile(rt, va, ba);
    load(rt + 64, va, ba);
    tile(rt + 32, vb, bb);
  }
}

void launch_qr_update_group(hipStream_t st, const GateDesc *d, int ng, int stage, int group,
                            int apply, int max_cols, int max_rows) {
  if (ng <= 0 || max_cols <= 0 || max_rows <= group * QG) return;
  const int ct = (max_cols + QGT - 1) / QGT;
  const int rc = (max_rows - group * QG + QR_RC - 1) / QR_RC;
  hipLaunchKernelGGL(k_qrg_s, dim3(ct, rc, ng), dim3(256), 0, st, d, stage, group, apply);
  hipLaunchKernelGGL(k_qrg_y, dim3(ct, ng), dim3(256), 0, st, d, stage, group, apply);
  hipLaunchKernelGGL(k_qrg_b, dim3(ct, rc, ng), dim3(256), 0, st, d, stage, group, apply);
}

// T factor of a group of QG reflectors (compact WY, forward, columnwise):
// T(i, i) = tau_i (from the panels' factors), T(0:i, i) = -tau_i T(0:i, 0:i)
// (V(:, 0:i)^H v_i), with the Gram V^H V summed over the group's rows.
__global__ __launch_bounds__(256) void k_qr_tgroup(const GateDesc *descs, int stage, int group) {
  const GateDesc &d = descs[blockIdx.x];
  if (!d.qr) return;
  const QrView q = qr_view(d, stage);
  const int j0 = group * QG;
  if (j0 >= q.cols) return;
  const int w = min(QG, q.cols - j0);
  const double2 *V = q.A + (size_t)j0 * q.ld;
  __shared__ double2 Vs[QU_ROWS][QG + 1];
  __shared__ double2 G[QG][QG + 1];
  __shared__ double2 Ts[QG][QG + 1];
  const int tid = threadIdx.x;
  constexpr int EPT = QG * QG / 256;
  double2 acc[EPT];
#pragma unroll
  for (int e = 0; e < EPT; e++) acc[e] = make_double2(0.0, 0.0);
  for (int r0 = j0; r0 < q.rows; r0 += QU_ROWS) {
    for (int e = tid; e < QU_ROWS * QG; e += 256) {
      const int r = e % QU_ROWS, p = e / QU_ROWS, gr = r0 + r, dr = gr - (j0 + p);
      double2 v = make_double2(0.0, 0.0);
      if (p < w && gr < q.rows && dr >= 0)
        v = dr == 0 ? make_double2(1.0, 0.0) : V[(size_t)p * q.ld + gr];
      Vs[r][p] = v;
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < EPT; e++) {
      const int id = tid + 256 * e, p = id / QG, l = id % QG;
#pragma unroll 8
      for (int r = 0; r < QU_ROWS; r++) cfmac(acc[e], Vs[r][p], Vs[r][l]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int e = 0; e < EPT; e++) {
    const int id = tid + 256 * e;
    G[id / QG][id % QG] = acc[e];
    Ts[id / QG][id % QG] = make_double2(0.0, 0.0);
  }
  __syncthreads();
  for (int i = 0; i < w; i++) {
    const double2 *Tp = qr_tfac(d, stage, (j0 + i) / QNB);
    const double2 tau = Tp[(i % QNB) * QNB + (i % QNB)];
    if (tid < i) {
      double2 sum = make_double2(0.0, 0.0);
      for (int l = tid; l < i; l++) sum = cadd(sum, cmul(Ts[tid][l], G[l][i]));
      Ts[tid][i] = cmul(make_double2(-tau.x, -tau.y), sum);
    }
    if (tid == i) Ts[i][i] = tau;
    __syncthreads();
  }
  double2 *Tg = qr_tgrp(d, stage, group);
  for (int e = tid; e < QG * QG; e += 256) Tg[e] = Ts[e / QG][e % QG];
}

void launch_qr_tgroup(hipStream_t st, const GateDesc *d, int ng, int stage, int group) {
  if (ng <= 0) return;
  hipLaunchKernelGGL(k_qr_tgroup, dim3(ng), dim3(256), 0, st, d, stage, group);
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
