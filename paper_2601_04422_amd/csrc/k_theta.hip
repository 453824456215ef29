// Two-site merge with the gate in the epilogue (float64 arithmetic).
//
//   theta[a,s,t,c]  = sum_b A_i[a,s,b] A_{i+1}[b,t,c]       (Sec. IV.A, Fig. 2)
//   theta'[a,s',t',c] = sum_{s,t} G[2s'+t', 2s+t] theta[a,s,t,c]   (Sec. III.A)
//   M[(a,s), (t,c)] = theta'[a,s,t,c] * lambda_{i+1}[c]
//
// Viewed as a matrix product, rows (a,s) of A_i (m x chiM) times A_{i+1}
// (chiM x 2chiR).  One output tile holds 64 rows (32 values of a, both s) and
// the same 32 values of c in both t halves, so the gate mixes entries of the
// same tile only.  The epilogue writes theta' (row-major, kept for the
// right-site write-back) and the Jacobi matrix X = M (column-major) or
// X = M^H when M is wide.
#include "tnsim_internal.h"
#include "tn_complex.h"
#include "tn_mfma.h"

namespace tn {

constexpr int TM = 64, TC = 32, TK = 16;

// Shared epilogue: Cs holds the merged tile theta (64 rows x 2*32 columns,
// row stride 2*TC+1); apply the gate, write theta' and the Jacobi matrix X.
__device__ void theta_epilogue(const GateDesc &d, int r0, int c0, double2 *Cs) {
  constexpr int LD = 2 * TC + 1;
  const int tid = threadIdx.x;
  const int m = d.m, chiR = d.chiR, n = d.n;
  for (int task = tid; task < (TM / 2) * TC; task += 256) {
    int al = task / TC, cl = task % TC;
    double2 v[4];
#pragma unroll
    for (int s = 0; s < 2; s++)
#pragma unroll
      for (int t = 0; t < 2; t++) v[2 * s + t] = Cs[(2 * al + s) * LD + t * TC + cl];
#pragma unroll
    for (int sp = 0; sp < 2; sp++)
#pragma unroll
      for (int tp = 0; tp < 2; tp++) {
        double2 o = make_double2(0.0, 0.0);
#pragma unroll
        for (int j = 0; j < 4; j++) cfma(o, d.g[(2 * sp + tp) * 4 + j], v[j]);
        Cs[(2 * al + sp) * LD + tp * TC + cl] = o;
      }
  }
  __syncthreads();
  // theta' row-major (m x n), coalesced along c
  for (int task = tid; task < TM * 2 * TC; task += 256) {
    int r = task / (2 * TC), jj = task % (2 * TC);
    int t = jj / TC, c = c0 + jj % TC, gr = r0 + r;
    if (gr < m && c < chiR) {
      size_t o = (size_t)gr * n + t * chiR + c;
      if (d.tfp32)
        ((float2 *)d.T)[o] = d2f(Cs[r * LD + jj]);
      else
        ((double2 *)d.T)[o] = Cs[r * LD + jj];
    }
  }
  if (!d.trans) {
    // M goes to Qm when the SVD is QR-preconditioned, else it is X itself.
    double2 *Xt = d.qr ? d.Qm : d.X;
    const int ldt = d.qr ? d.ldq : d.ldx;
    // X = M with its columns in the order (c, t) instead of M's (t, c):
    // lambda_{i+1} is sorted, so neighbouring columns then carry weights of
    // the same size, which saves the block Jacobi one or two sweeps (the SVD
    // does not depend on the column order).  Column-major, coalesced along rows.
    for (int task = tid; task < TM * 2 * TC; task += 256) {
      int r = task % TM, jj = task / TM;
      int t = jj / TC, c = c0 + jj % TC, gr = r0 + r;
      if (gr < m && c < chiR) {
        double w = d.lamR ? d.lamR[c] : 1.0;
        Xt[(size_t)(2 * c + t) * ldt + gr] = cscale(Cs[r * LD + jj], w);
      }
    }
  } else {
    // X = M^H (n x m): column gr holds conj(row gr of M)
    for (int task = tid; task < TM * 2 * TC; task += 256) {
      int r = task / (2 * TC), jj = task % (2 * TC);
      int t = jj / TC, c = c0 + jj % TC, gr = r0 + r;
      if (gr < m && c < chiR) {
        double w = d.lamR ? d.lamR[c] : 1.0;
        d.X[(size_t)gr * d.ldx + t * chiR + c] = cscale(cconj(Cs[r * LD + jj]), w);
      }
    }
  }
}

// float64 merge on the matrix cores (v_mfma_f64_16x16x4f64): a complex
// product is three real products (Gauss: ac, bd, (a + b)(c + d)).  Wavefront w owns the 32x32 quarter (rows
// 32 (w&1), columns 32 (w>>1)) as 2x2 tiles of 16x16; lane l supplies
// A[l%16][k + l/16] and B[k + l/16][l%16] and holds D[l/16 + 4v][l%16] of
// each tile.  The next 16-deep k step is loaded into registers while the
// current one is multiplied.
typedef double f64x4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f64x4_t mfma_f64(double a, double b, f64x4_t c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <class S>
__device__ void theta_tile_f64mfma(const GateDesc &d, int r0, int c0, double2 *smem) {
  const int tid = threadIdx.x;
  const S *A0 = (const S *)d.A0;
  const S *A1 = (const S *)d.A1;
  const int m = d.m, chiM = d.chiM, chiR = d.chiR, n = d.n;
  double2 *As = smem;            // [TK][TM]
  double2 *Bs = smem + TK * TM;  // [TK][2*TC]
  const int ar = tid >> 2, akq = (tid & 3) * 4;   // A: row ar, 4 consecutive k
  const int bk = tid >> 4, bjq = (tid & 15) * 4;  // B: row bk, 4 consecutive columns
  double2 ra[4], rb[4];
  auto load = [&](int k0) {
    const int gr = r0 + ar;
#pragma unroll
    for (int j = 0; j < 4; j++) {
      const int gk = k0 + akq + j;
      ra[j] = (gr < m && gk < chiM) ? cload(A0 + (size_t)gr * chiM + gk) : make_double2(0.0, 0.0);
    }
    const int gk = k0 + bk;
#pragma unroll
    for (int j = 0; j < 4; j++) {
      const int jj = bjq + j, t = jj >> 5, c = c0 + (jj & 31);
      rb[j] = (gk < chiM && c < chiR) ? cload(A1 + (size_t)gk * n + t * chiR + c)
                                      : make_double2(0.0, 0.0);
    }
  };
  const int w = tid >> 6, lane = tid & 63, l16 = lane & 15, lg = lane >> 4;
  const int wm = (w & 1) * 32, wn = (w >> 1) * 32;
  f64x4_t c1[2][2], c2[2][2], c3[2][2];  // Gauss: a c, b d, (a + b)(c + d)
#pragma unroll
  for (int x = 0; x < 2; x++)
#pragma unroll
    for (int y = 0; y < 2; y++) {
      c1[x][y] = f64x4_t{0.0, 0.0, 0.0, 0.0};
      c2[x][y] = f64x4_t{0.0, 0.0, 0.0, 0.0};
      c3[x][y] = f64x4_t{0.0, 0.0, 0.0, 0.0};
    }
  load(0);
  for (int k0 = 0; k0 < chiM; k0 += TK) {
#pragma unroll
    for (int j = 0; j < 4; j++) {
      As[(akq + j) * TM + ar] = ra[j];
      Bs[bk * (2 * TC) + bjq + j] = rb[j];
    }
    __syncthreads();
    if (k0 + TK < chiM) load(k0 + TK);
#pragma unroll
    for (int kk = 0; kk < TK; kk += 4) {
      double2 a[2], b[2];
#pragma unroll
      for (int x = 0; x < 2; x++) {
        a[x] = As[(kk + lg) * TM + wm + 16 * x + l16];
        b[x] = Bs[(kk + lg) * (2 * TC) + wn + 16 * x + l16];
      }
#pragma unroll
      for (int x = 0; x < 2; x++)
#pragma unroll
        for (int y = 0; y < 2; y++) {
          c1[x][y] = mfma_f64(a[x].x, b[y].x, c1[x][y]);
          c2[x][y] = mfma_f64(a[x].y, b[y].y, c2[x][y]);
          c3[x][y] = mfma_f64(a[x].x + a[x].y, b[y].x + b[y].y, c3[x][y]);
        }
    }
    __syncthreads();
  }
  constexpr int LD = 2 * TC + 1;
  double2 *Cs = smem;  // [TM][LD]
#pragma unroll
  for (int x = 0; x < 2; x++)
#pragma unroll
    for (int y = 0; y < 2; y++)
#pragma unroll
      for (int v = 0; v < 4; v++)
        Cs[(wm + 16 * x + lg + 4 * v) * LD + wn + 16 * y + l16] =
            make_double2((c1[x][y][v] - c2[x][y][v]), (c3[x][y][v] - c1[x][y][v] - c2[x][y][v]));
  __syncthreads();
  theta_epilogue(d, r0, c0, Cs);
}

__global__ __launch_bounds__(256) void k_theta_f64mfma(const GateDesc *descs) {
  const GateDesc &d = descs[blockIdx.z];
  int r0 = blockIdx.x * TM, c0 = blockIdx.y * TC;
  if (r0 >= d.m || c0 >= d.chiR) return;
  __shared__ double2 smem[TM * (2 * TC + 1)];
  if (d.storage == 0)
    theta_tile_f64mfma<double2>(d, r0, c0, smem);
  else
    theta_tile_f64mfma<float2>(d, r0, c0, smem);
}

// Same tile and epilogue on matrix cores: operands rounded to complex64 and
// multiplied in the selected split mode with float32 accumulation.
template <int MODE, class S>
__device__ void theta_tile_mfma(const GateDesc &d, int r0, int c0, double2 *smem) {
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const S *A0 = (const S *)d.A0;
  const S *A1 = (const S *)d.A1;
  const int m = d.m, chiM = d.chiM, chiR = d.chiR, n = d.n;
  float2 *Af = reinterpret_cast<float2 *>(smem);  // [64][TILE_LD]
  float2 *Bf = Af + 64 * TILE_LD;                 // [64][TILE_LD]
  f32x4_t accR[2][2], accI[2][2];
#pragma unroll
  for (int i = 0; i < 2; i++)
#pragma unroll
    for (int j = 0; j < 2; j++) {
      accR[i][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};
      accI[i][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};
    }
  for (int k0 = 0; k0 < chiM; k0 += TILE_K) {
    {  // A: row r, 4 consecutive k
      int r = tid >> 2, kq = (tid & 3) * 4, gr = r0 + r;
#pragma unroll
      for (int j = 0; j < 4; j++) {
        int gk = k0 + kq + j;
        double2 v = make_double2(0.0, 0.0);
        if (gr < m && gk < chiM) v = cload(A0 + (size_t)gr * chiM + gk);
        Af[r * TILE_LD + kq + j] = d2f(v);
      }
    }
    {  // B^T: column jj (t half, c), 4 consecutive columns of one k row
      int kk = tid >> 4, jq = (tid & 15) * 4, gk = k0 + kk;
#pragma unroll
      for (int j = 0; j < 4; j++) {
        int jj = jq + j, t = jj >> 5, c = c0 + (jj & 31);
        double2 v = make_double2(0.0, 0.0);
        if (gk < chiM && c < chiR) v = cload(A1 + (size_t)gk * n + t * chiR + c);
        Bf[jj * TILE_LD + kk] = d2f(v);
      }
    }
    __syncthreads();
    cmma_step<MODE>(Af, Bf, wave, lane, accR, accI);
    __syncthreads();
  }
  constexpr int LD = 2 * TC + 1;
  double2 *Cs = smem;
#pragma unroll
  for (int ti = 0; ti < 2; ti++)
#pragma unroll
    for (int tj = 0; tj < 2; tj++)
#pragma unroll
      for (int e = 0; e < 4; e++) {
        int row, col;
        cmma_coord(wave, lane, ti, tj, e, row, col);
        Cs[row * LD + col] = make_double2((double)accR[ti][tj][e], (double)accI[ti][tj][e]);
      }
  __syncthreads();
  theta_epilogue(d, r0, c0, Cs);
}

template <int MODE>
__global__ __launch_bounds__(256) void k_theta_mfma(const GateDesc *descs) {
  const GateDesc &d = descs[blockIdx.z];
  int r0 = blockIdx.x * TM, c0 = blockIdx.y * TC;
  if (r0 >= d.m || c0 >= d.chiR) return;
  __shared__ double2 smem[TM * (2 * TC + 1)];
  if (d.storage == 0)
    theta_tile_mfma<MODE, double2>(d, r0, c0, smem);
  else
    theta_tile_mfma<MODE, float2>(d, r0, c0, smem);
}

void launch_theta_mfma(hipStream_t st, const GateDesc *d, int ng, int precision, int max_m,
                       int max_chiR) {
  dim3 grid((max_m + TM - 1) / TM, (max_chiR + TC - 1) / TC, ng);
  if (precision == MODE_F32)
    hipLaunchKernelGGL(k_theta_mfma<MODE_F32>, grid, dim3(256), 0, st, d);
  else if (precision == MODE_BF16X3)
    hipLaunchKernelGGL(k_theta_mfma<MODE_BF16X3>, grid, dim3(256), 0, st, d);
  else
    hipLaunchKernelGGL(k_theta_mfma<MODE_BF16X6>, grid, dim3(256), 0, st, d);
}

void launch_theta(hipStream_t st, const GateDesc *d, int ng, int precision, int max_m,
                  int max_chiR) {
  if (ng <= 0) return;
  if (precision != 0) {
    launch_theta_mfma(st, d, ng, precision, max_m, max_chiR);
    return;
  }
  dim3 grid((max_m + TM - 1) / TM, (max_chiR + TC - 1) / TC, ng);
  hipLaunchKernelGGL(k_theta_f64mfma, grid, dim3(256), 0, st, d);
}

}  // namespace tn
