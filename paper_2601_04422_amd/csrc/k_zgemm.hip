// Complex float64 GEMM on the FP64 matrix cores: C = op(A) B.
//
// A complex product is four real products (C_re += A_re B_re - A_im B_im,
// C_im += A_re B_im + A_im B_re), each a v_mfma_f64_16x16x4f64.  A workgroup
// of four waves computes a 64 x 64 tile of C; each wave owns a 32 x 32
// quarter (2 x 2 MFMA tiles).  K advances 16 at a time through LDS, with
// the next step's global loads issued before the current step's products.
// Operands are read in their storage precision (complex64 sites are widened
// on load); C is complex128.  The summation order is fixed, so results do
// not depend on scheduling.
#include "tnsim_internal.h"
#include "tn_complex.h"

namespace tn {

typedef double zd4_t __attribute__((ext_vector_type(4)));

// lane l supplies A[l%16][l/16] and B[l/16][l%16]; entry v of the result is
// D[l/16 + 4v][l%16]
__device__ __forceinline__ zd4_t zmfma(double a, double b, zd4_t c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int ZT = 64, ZK = 16;

// AK: A(i,k) = A[i*sa + k], else A[k*sa + i]; AC: use conj(A).
// BK: B(k,j) = B[j*sb + k], else B[k*sb + j].
// CM: C(i,j) = C[j*sc + i], else C[i*sc + j].
// blockIdx.z: batch index, or K split (partial products to g.part).
// GA (gathered columns): output columns *g.clo .. *g.chi - 1 (device
// values; the grid covers at most N of them), column j reads column
// g.bmap[j] of B and is scaled by g.cscale[j]; tiles from column *g.asplit
// on read A + g.za.
template <class TA, class TB, bool AK, bool AC, bool BK, bool CM, bool GA>
__global__ __launch_bounds__(256, AK ? 4 : 3) void k_zgemm(ZgemmArgs g) {
  // XCD-aware tile order: workgroups are dealt to the 8 XCDs in turn, so
  // workgroup L runs on XCD L % 8.  Each XCD gets a contiguous run of tiles
  // in row-tile-major order, so the A rows of its tiles stay in its own L2.
  const int nx = gridDim.x, ntile = gridDim.x * gridDim.y;
  const int L = blockIdx.x + nx * blockIdx.y, xcd = L & 7, slot = L >> 3;
  const int per = ntile >> 3, extra = ntile & 7;
  const int t_lin = xcd * per + min(xcd, extra) + slot;
  const int tx = t_lin % nx, ty = t_lin / nx;
  int N = g.N, j0 = tx * ZT, A_off_tile = 0;
  if (GA) {
    const int lo = *g.clo;
    N = *g.chi;
    j0 += lo;
    if (g.asplit && j0 >= *g.asplit) A_off_tile = 1;
  } else if (g.mcount) {
    N = min(N, g.mult * *g.mcount);
  }
  const int i0 = ty * ZT;
  if (j0 >= N) return;
  const int M = g.M, z = blockIdx.z;
  const TA *A = (const TA *)g.A;
  const TB *B = (const TB *)g.B;
  double2 *C = g.C;
  int kb = 0, K = g.K;
  if (g.ksplit > 1) {
    kb = z * g.kchunk;
    K = min(g.K, kb + g.kchunk);
  } else {
    A += (z + A_off_tile) * g.za;
    B += z * g.zb;
    C += z * g.zc;
  }
  __shared__ double2 As[ZK][ZT], Bs[ZK][ZT];
  const int t = threadIdx.x;
  // this thread's share of a K step: 4 elements of A and 4 of B
  const int ar = AK ? (t >> 2) : (t >> 4), ac = AK ? (t & 3) * 4 : (t & 15) * 4;
  const int br = BK ? (t >> 2) : (t >> 4), bc = BK ? (t & 3) * 4 : (t & 15) * 4;
  double2 ra[4], rb[4];
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 4; q++) {
      int gi, gk;
      if (AK) {
        gi = i0 + ar;
        gk = k0 + ac + q;
      } else {
        gi = i0 + ac + q;
        gk = k0 + ar;
      }
      ra[q] = (gi < M && gk < K)
                  ? cload(A + (AK ? (long long)gi * g.sa + gk : (long long)gk * g.sa + gi))
                  : make_double2(0.0, 0.0);
      int gj;
      if (BK) {
        gj = j0 + br;
        gk = k0 + bc + q;
      } else {
        gj = j0 + bc + q;
        gk = k0 + br;
      }
      const long long bj = GA ? (long long)(gj < N ? g.bmap[gj] : 0) : gj;
      rb[q] = (gj < N && gk < K)
                  ? cload(B + (BK ? bj * g.sb + gk : (long long)gk * g.sb + bj))
                  : make_double2(0.0, 0.0);
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const double2 a = AC ? cconj(ra[q]) : ra[q];
      if (AK)
        As[ac + q][ar] = a;
      else
        As[ar][ac + q] = a;
      if (BK)
        Bs[bc + q][br] = rb[q];
      else
        Bs[br][bc + q] = rb[q];
    }
  };
  const int w = t >> 6, lane = t & 63, l16 = lane & 15, lg = lane >> 4;
  const int wm = (w & 1) * 32, wn = (w >> 1) * 32;
  zd4_t cr[2][2], ci[2][2];
#pragma unroll
  for (int a = 0; a < 2; a++)
#pragma unroll
    for (int b = 0; b < 2; b++) {
      cr[a][b] = zd4_t{0.0, 0.0, 0.0, 0.0};
      ci[a][b] = zd4_t{0.0, 0.0, 0.0, 0.0};
    }
  load(kb);
  for (int k0 = kb; k0 < K; k0 += ZK) {
    stash();
    __syncthreads();
    if (k0 + ZK < K) load(k0 + ZK);
#pragma unroll
    for (int kk = 0; kk < ZK; kk += 4) {
      double2 a[2], b[2];
#pragma unroll
      for (int x = 0; x < 2; x++) {
        a[x] = As[kk + lg][wm + 16 * x + l16];
        b[x] = Bs[kk + lg][wn + 16 * x + l16];
      }
#pragma unroll
      for (int x = 0; x < 2; x++)
#pragma unroll
        for (int y = 0; y < 2; y++) {
          cr[x][y] = zmfma(a[x].x, b[y].x, cr[x][y]);
          cr[x][y] = zmfma(-a[x].y, b[y].y, cr[x][y]);
          ci[x][y] = zmfma(a[x].x, b[y].y, ci[x][y]);
          ci[x][y] = zmfma(a[x].y, b[y].x, ci[x][y]);
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < 2; x++)
#pragma unroll
    for (int y = 0; y < 2; y++) {
      const int j = j0 + wn + 16 * y + l16;
      if (j >= N) continue;
      const double sc = GA ? g.cscale[j] : 1.0;
#pragma unroll
      for (int v = 0; v < 4; v++) {
        const int i = i0 + wm + 16 * x + lg + 4 * v;
        if (i >= M) continue;
        const double2 c = make_double2(sc * cr[x][y][v], sc * ci[x][y][v]);
        if (g.ksplit > 1)
          g.part[((size_t)z * M + i) * g.N + j] = c;
        else
          C[CM ? (long long)j * g.sc + i : (long long)i * g.sc + j] = c;
      }
    }
}

// C = sum over splits of the partial products, in split order.
template <bool CM>
__global__ __launch_bounds__(256) void k_zgemm_sum(ZgemmArgs g) {
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  const size_t MN = (size_t)g.M * g.N;
  if (e >= MN) return;
  const int i = (int)(e / g.N), j = (int)(e % g.N);
  double2 acc = g.part[e];
  for (int z = 1; z < g.ksplit; z++) acc = cadd(acc, g.part[z * MN + e]);
  g.C[CM ? (long long)j * g.sc + i : (long long)i * g.sc + j] = acc;
}

// The partial products of a split take at most ZGEMM_PART_ELEMS elements.
int zgemm_ksplit(int M, int N, int K) {
  const int tiles = ((M + ZT - 1) / ZT) * ((N + ZT - 1) / ZT);
  if (tiles >= 512) return 1;  // enough workgroups already; partial sums cost traffic
  int ks = 1;
  while (ks < 8 && tiles * ks * 2 <= 1024 && K / (ks * 2) >= 128) ks *= 2;
  return ks;
}

template <bool AK, bool AC, bool BK, bool CM, bool GA = false>
static void zgemm_dispatch(hipStream_t st, ZgemmArgs g, int a_storage, int b_storage) {
  // the partial sums cover the whole bound, and must fit the caller's buffer
  if (GA || g.mcount || !g.part || (size_t)g.ksplit * g.M * g.N > ZGEMM_PART_ELEMS) g.ksplit = 1;
  if (g.ksplit > 1) {
    g.batch = 1;
    g.kchunk = ((g.K + g.ksplit - 1) / g.ksplit + ZK - 1) / ZK * ZK;
    g.ksplit = (g.K + g.kchunk - 1) / g.kchunk;
  }
  dim3 grid((g.N + ZT - 1) / ZT, (g.M + ZT - 1) / ZT, g.ksplit > 1 ? g.ksplit : g.batch);
  if (a_storage == 0 && b_storage == 0)
    hipLaunchKernelGGL((k_zgemm<double2, double2, AK, AC, BK, CM, GA>), grid, dim3(256), 0, st, g);
  else if (a_storage == 0)
    hipLaunchKernelGGL((k_zgemm<double2, float2, AK, AC, BK, CM, GA>), grid, dim3(256), 0, st, g);
  else if (b_storage == 0)
    hipLaunchKernelGGL((k_zgemm<float2, double2, AK, AC, BK, CM, GA>), grid, dim3(256), 0, st, g);
  else
    hipLaunchKernelGGL((k_zgemm<float2, float2, AK, AC, BK, CM, GA>), grid, dim3(256), 0, st, g);
  if (g.ksplit > 1) {
    const size_t MN = (size_t)g.M * g.N;
    hipLaunchKernelGGL(k_zgemm_sum<CM>, dim3((unsigned)((MN + 255) / 256)), dim3(256), 0, st, g);
  }
}

void launch_zgemm(hipStream_t st, ZgemmKind kind, const ZgemmArgs &g, int a_storage,
                  int b_storage) {
  if (g.M <= 0 || g.N <= 0) return;
  switch (kind) {
    case ZGEMM_NN_ROW:  // C = A B, A k-contiguous, B and C row-major
      zgemm_dispatch<true, false, false, false>(st, g, a_storage, b_storage);
      break;
    case ZGEMM_CN_ROW:  // C = A^H B, A stored K x M row-major, B and C row-major
      zgemm_dispatch<false, true, false, false>(st, g, a_storage, b_storage);
      break;
    case ZGEMM_NN_COL:  // C = A B, A k-contiguous, B and C column-major
      zgemm_dispatch<true, false, true, true>(st, g, a_storage, b_storage);
      break;
    case ZGEMM_NN_COL_GATHER:  // the same on gathered, scaled columns
      if (g.clo && g.chi && g.bmap && g.cscale)
        zgemm_dispatch<true, false, true, true, true>(st, g, a_storage, b_storage);
      break;
  }
}

}  // namespace tn
