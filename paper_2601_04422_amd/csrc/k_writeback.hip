// Write-back of a two-qubit gate (Sec. III.A: left singular vectors to the
// left/control site, singular values with the right singular vectors to the
// right/target site):
//
//   A_i'[a,s,j]     = u_j[2a+s]                        j < k
//   A_{i+1}'[j,t,c] = (1/N) sum_{a,s} conj(u_j[2a+s]) theta'[a,s,t,c]
//
// u_j is column perm[j] of X divided by its norm (X = M), column perm[j] of
// J (X = M^H), or column j of U (QR-preconditioned SVD, U = Q1 [W_k; 0]).
// Using theta' rather than M keeps lambda_{i+1} from being divided out.
#include "tnsim_internal.h"
#include "tn_complex.h"
#include "tn_mfma.h"

namespace tn {

__device__ __forceinline__ double2 left_vec(const GateDesc &d, int r, int col, double inv) {
  if (d.qr) return d.U[(size_t)col * d.ldu + r];
  return d.trans ? d.J[(size_t)col * d.ldj + r] : cscale(d.X[(size_t)col * d.ldx + r], inv);
}

// Which stored column holds u_j, and the factor that normalises it.
__device__ __forceinline__ int left_col(const GateDesc &d, int j) { return d.qr ? j : d.perm[j]; }
__device__ __forceinline__ double left_inv(const GateDesc &d, int col) {
  return (d.trans || d.qr) ? 1.0 : 1.0 / sqrt(d.sig2[col]);
}

// grid: (m tiles of 64, k tiles of 64, gate)
template <class S>
__device__ void wb_left_tile(const GateDesc &d, int k, int r0, int j0, double2 *tile) {
  const int tid = threadIdx.x;
  constexpr int LD = 65;
  for (int e = tid; e < 64 * 64; e += 256) {
    int r = e % 64, j = e / 64;  // read along r (column-major source)
    int gr = r0 + r, gj = j0 + j;
    double2 v = make_double2(0.0, 0.0);
    if (gr < d.m && gj < k) {
      int col = left_col(d, gj);
      double inv = left_inv(d, col);
      v = left_vec(d, gr, col, inv);
    }
    tile[r * LD + j] = v;
  }
  __syncthreads();
  S *A0 = (S *)d.A0out;
  for (int e = tid; e < 64 * 64; e += 256) {
    int j = e % 64, r = e / 64;  // write along j (row-major destination)
    int gr = r0 + r, gj = j0 + j;
    if (gr < d.m && gj < k) cstore(A0 + (size_t)gr * k + gj, tile[r * LD + j]);
  }
}

__global__ __launch_bounds__(256) void k_wb_left(const GateDesc *descs) {
  const GateDesc &d = descs[blockIdx.z];
  const int k = d.sc->k;
  int r0 = blockIdx.x * 64, j0 = blockIdx.y * 64;
  if (r0 >= d.m || j0 >= k) return;
  __shared__ double2 tile[64 * 65];
  if (d.storage == 0)
    wb_left_tile<double2>(d, k, r0, j0, tile);
  else
    wb_left_tile<float2>(d, k, r0, j0, tile);
}

// A_{i+1}' = (1/N) U_k^H theta'   (k x n), tiles of 64 x 64, K = m in steps of 16.
// float64 product on the matrix cores (v_mfma_f64_16x16x4f64, three real
// products per complex one: ac, bd, (a + b)(c + d)).  Tile j (64 kept vectors) x c (64 columns
// of theta'), K = m rows in steps of 16 through LDS, the next step loaded
// into registers while the current one is multiplied.  Wavefront w owns the
// 32x32 quarter (rows 32 (w&1), columns 32 (w>>1)); lane l supplies
// A[l%16][k + l/16] and B[k + l/16][l%16] and holds D[l/16 + 4v][l%16].
typedef double f64x4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f64x4_t wb_mfma_f64(double a, double b, f64x4_t c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <class S>
__device__ void wb_right_tile_f64mfma(const GateDesc &d, int k, int j0, int c0, double2 *smem) {
  const int tid = threadIdx.x;
  double2 *As = smem;            // [16][64]  conj(U)[r][j]
  double2 *Bs = smem + 16 * 64;  // [16][64]  theta'[r][c]
  const double2 *T = (const double2 *)d.T;
  const int m = d.m, n = d.n;
  const int aj = tid >> 2, ar = (tid & 3) * 4;  // A: column j, 4 consecutive r
  const int gj = j0 + aj;
  int colA = 0;
  double invA = 1.0;
  if (gj < k) {
    colA = left_col(d, gj);
    invA = left_inv(d, colA);
  }
  const int br = tid >> 4, bc = (tid & 15) * 4;  // B: row r, 4 consecutive c
  double2 ra[4], rb[4];
  auto load = [&](int r0) {
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const int gr = r0 + ar + q;
      ra[q] = (gj < k && gr < m) ? cconj(left_vec(d, gr, colA, invA)) : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const int gr = r0 + br, gc = c0 + bc + q;
      rb[q] = (gr < m && gc < n) ? T[(size_t)gr * n + gc] : make_double2(0.0, 0.0);
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
  for (int r0 = 0; r0 < m; r0 += 16) {
#pragma unroll
    for (int q = 0; q < 4; q++) {
      As[(ar + q) * 64 + aj] = ra[q];
      Bs[br * 64 + bc + q] = rb[q];
    }
    __syncthreads();
    if (r0 + 16 < m) load(r0 + 16);
#pragma unroll
    for (int kk = 0; kk < 16; kk += 4) {
      double2 a[2], b[2];
#pragma unroll
      for (int x = 0; x < 2; x++) {
        a[x] = As[(kk + lg) * 64 + wm + 16 * x + l16];
        b[x] = Bs[(kk + lg) * 64 + wn + 16 * x + l16];
      }
#pragma unroll
      for (int x = 0; x < 2; x++)
#pragma unroll
        for (int y = 0; y < 2; y++) {
          c1[x][y] = wb_mfma_f64(a[x].x, b[y].x, c1[x][y]);
          c2[x][y] = wb_mfma_f64(a[x].y, b[y].y, c2[x][y]);
          c3[x][y] = wb_mfma_f64(a[x].x + a[x].y, b[y].x + b[y].y, c3[x][y]);
        }
    }
    __syncthreads();
  }
  const double invN = 1.0 / d.sc->N;
  S *A1 = (S *)d.A1out;
#pragma unroll
  for (int x = 0; x < 2; x++)
#pragma unroll
    for (int y = 0; y < 2; y++) {
      const int gc = c0 + wn + 16 * y + l16;
#pragma unroll
      for (int v = 0; v < 4; v++) {
        const int gjo = j0 + wm + 16 * x + lg + 4 * v;
        if (gjo < k && gc < n)
          cstore(A1 + (size_t)gjo * n + gc,
                 make_double2((c1[x][y][v] - c2[x][y][v]) * invN, (c3[x][y][v] - c1[x][y][v] - c2[x][y][v]) * invN));
      }
    }
}

// float64 write-back (theta' stored complex128) on the matrix cores
__global__ __launch_bounds__(256) void k_wb_right_f64mfma(const GateDesc *descs) {
  const GateDesc &d = descs[blockIdx.z];
  const int k = d.sc->k;
  int j0 = blockIdx.x * 64, c0 = blockIdx.y * 64;
  if (j0 >= k || c0 >= d.n) return;
  __shared__ double2 smem[2 * 16 * 64];
  if (d.storage == 0)
    wb_right_tile_f64mfma<double2>(d, k, j0, c0, smem);
  else
    wb_right_tile_f64mfma<float2>(d, k, j0, c0, smem);
}

void launch_wb_left(hipStream_t st, const GateDesc *d, int ng, int max_m, int max_k) {
  if (ng <= 0) return;
  hipLaunchKernelGGL(k_wb_left, dim3((max_m + 63) / 64, (max_k + 63) / 64, ng), dim3(256), 0, st,
                     d);
}

// A_{i+1}' = (1/N) U_k^H theta' on matrix cores (theta' stored complex64).
template <int MODE, class S>
__device__ void wb_right_tile_mfma(const GateDesc &d, int k, int j0, int c0, float2 *Af,
                                   float2 *Bf) {
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const float2 *T = (const float2 *)d.T;
  const int m = d.m, n = d.n;
  f32x4_t accR[2][2], accI[2][2];
#pragma unroll
  for (int i = 0; i < 2; i++)
#pragma unroll
    for (int j = 0; j < 2; j++) {
      accR[i][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};
      accI[i][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};
    }
  const int aj = tid >> 2, ar = (tid & 3) * 4, gj = j0 + aj;
  int colA = 0;
  double invA = 1.0;
  if (gj < k) {
    colA = left_col(d, gj);
    invA = left_inv(d, colA);
  }
  const int bk = tid >> 4, bc = (tid & 15) * 4;
  for (int r0 = 0; r0 < m; r0 += TILE_K) {
#pragma unroll
    for (int q = 0; q < 4; q++) {  // A[j][r] = conj(u_j[r])
      int gr = r0 + ar + q;
      double2 v = make_double2(0.0, 0.0);
      if (gj < k && gr < m) v = cconj(left_vec(d, gr, colA, invA));
      Af[aj * TILE_LD + ar + q] = d2f(v);
    }
#pragma unroll
    for (int q = 0; q < 4; q++) {  // B^T[c][r] = theta'[r][c]
      int gr = r0 + bk, gc = c0 + bc + q;
      float2 v = make_float2(0.f, 0.f);
      if (gr < m && gc < n) v = T[(size_t)gr * n + gc];
      Bf[(bc + q) * TILE_LD + bk] = v;
    }
    __syncthreads();
    cmma_step<MODE>(Af, Bf, wave, lane, accR, accI);
    __syncthreads();
  }
  const double invN = 1.0 / d.sc->N;
  S *A1 = (S *)d.A1out;
#pragma unroll
  for (int ti = 0; ti < 2; ti++)
#pragma unroll
    for (int tj = 0; tj < 2; tj++)
#pragma unroll
      for (int e = 0; e < 4; e++) {
        int row, col;
        cmma_coord(wave, lane, ti, tj, e, row, col);
        int gjo = j0 + row, gc = c0 + col;
        if (gjo < k && gc < n)
          cstore(A1 + (size_t)gjo * n + gc,
                 make_double2((double)accR[ti][tj][e] * invN, (double)accI[ti][tj][e] * invN));
      }
}

template <int MODE>
__global__ __launch_bounds__(256) void k_wb_right_mfma(const GateDesc *descs) {
  const GateDesc &d = descs[blockIdx.z];
  const int k = d.sc->k;
  int j0 = blockIdx.x * 64, c0 = blockIdx.y * 64;
  if (j0 >= k || c0 >= d.n) return;
  __shared__ float2 Af[64 * TILE_LD], Bf[64 * TILE_LD];
  if (d.storage == 0)
    wb_right_tile_mfma<MODE, double2>(d, k, j0, c0, Af, Bf);
  else
    wb_right_tile_mfma<MODE, float2>(d, k, j0, c0, Af, Bf);
}

void launch_wb_right(hipStream_t st, const GateDesc *d, int ng, int precision, int max_k,
                     int max_n) {
  if (ng <= 0) return;
  dim3 grid((max_k + 63) / 64, (max_n + 63) / 64, ng);
  if (precision == 0)
    hipLaunchKernelGGL(k_wb_right_f64mfma, grid, dim3(256), 0, st, d);
  else if (precision == MODE_F32)
    hipLaunchKernelGGL(k_wb_right_mfma<MODE_F32>, grid, dim3(256), 0, st, d);
  else if (precision == MODE_BF16X3)
    hipLaunchKernelGGL(k_wb_right_mfma<MODE_BF16X3>, grid, dim3(256), 0, st, d);
  else
    hipLaunchKernelGGL(k_wb_right_mfma<MODE_BF16X6>, grid, dim3(256), 0, st, d);
}

}  // namespace tn
