// Readout kernels: transfer-matrix contraction for <bra|P|ket> and amplitudes.
//
//   E_q[b,b'] = sum conj(B_q[a,s,b]) P[s,s'] E_{q-1}[a,a'] K_q[a',s',b']
//
// is done per site as F = E K (GEMM), F2 = P on the physical index, and
// E' = B^H F2 (GEMM with the bra conjugate-transposed), all in float64.
#include "tnsim_internal.h"
#include "tn_complex.h"

namespace tn {

constexpr int RT = 64, RK = 16;

// C (M x N) = A (M x K, complex128 row-major) * B (K x N, site storage, row-major)
template <class SB>
__global__ __launch_bounds__(256) void k_gemm_nn(int M, int N, int K, const double2 *A, int lda,
                                                 const SB *B, int ldb, double2 *C, int ldc) {
  __shared__ double2 As[RK * RT], Bs[RK * RT];
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const int i0 = blockIdx.x * RT, j0 = blockIdx.y * RT;
  double2 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; i++)
#pragma unroll
    for (int j = 0; j < 4; j++) acc[i][j] = make_double2(0.0, 0.0);
  for (int k0 = 0; k0 < K; k0 += RK) {
    {
      int r = tid >> 2, kq = (tid & 3) * 4;
#pragma unroll
      for (int q = 0; q < 4; q++) {
        int gi = i0 + r, gk = k0 + kq + q;
        As[(kq + q) * RT + r] = (gi < M && gk < K) ? A[(size_t)gi * lda + gk] : make_double2(0, 0);
      }
      int kk = tid >> 4, jq = (tid & 15) * 4;
#pragma unroll
      for (int q = 0; q < 4; q++) {
        int gk = k0 + kk, gj = j0 + jq + q;
        Bs[kk * RT + jq + q] = (gk < K && gj < N) ? cload(B + (size_t)gk * ldb + gj) : make_double2(0, 0);
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < RK; kk++) {
      double2 a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; i++) a[i] = As[kk * RT + ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; j++) b[j] = Bs[kk * RT + tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < 4; j++) cfma(acc[i][j], a[i], b[j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; i++)
#pragma unroll
    for (int j = 0; j < 4; j++) {
      int gi = i0 + ty + 16 * i, gj = j0 + tx + 16 * j;
      if (gi < M && gj < N) C[(size_t)gi * ldc + gj] = acc[i][j];
    }
}

// C (M x N) = A^H B, A stored K x M (site storage, row-major), B K x N complex128
template <class SA>
__global__ __launch_bounds__(256) void k_gemm_cn(int M, int N, int K, const SA *A, int lda,
                                                 const double2 *B, int ldb, double2 *C, int ldc) {
  __shared__ double2 As[RK * RT], Bs[RK * RT];
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const int i0 = blockIdx.x * RT, j0 = blockIdx.y * RT;
  double2 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; i++)
#pragma unroll
    for (int j = 0; j < 4; j++) acc[i][j] = make_double2(0.0, 0.0);
  for (int k0 = 0; k0 < K; k0 += RK) {
    {
      int kk = tid >> 4, iq = (tid & 15) * 4;
#pragma unroll
      for (int q = 0; q < 4; q++) {
        int gk = k0 + kk, gi = i0 + iq + q;
        As[kk * RT + iq + q] = (gk < K && gi < M) ? cconj(cload(A + (size_t)gk * lda + gi)) : make_double2(0, 0);
        int gj = j0 + iq + q;
        Bs[kk * RT + iq + q] = (gk < K && gj < N) ? B[(size_t)gk * ldb + gj] : make_double2(0, 0);
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < RK; kk++) {
      double2 a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; i++) a[i] = As[kk * RT + ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; j++) b[j] = Bs[kk * RT + tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < 4; j++) cfma(acc[i][j], a[i], b[j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; i++)
#pragma unroll
    for (int j = 0; j < 4; j++) {
      int gi = i0 + ty + 16 * i, gj = j0 + tx + 16 * j;
      if (gi < M && gj < N) C[(size_t)gi * ldc + gj] = acc[i][j];
    }
}

void launch_gemm_nn(hipStream_t st, int M, int N, int K, const double2 *A, int lda, const void *B,
                    int ldb, int b_storage, double2 *C, int ldc) {
  dim3 grid((M + RT - 1) / RT, (N + RT - 1) / RT);
  if (b_storage == 0)
    hipLaunchKernelGGL(k_gemm_nn<double2>, grid, dim3(256), 0, st, M, N, K, A, lda,
                       (const double2 *)B, ldb, C, ldc);
  else
    hipLaunchKernelGGL(k_gemm_nn<float2>, grid, dim3(256), 0, st, M, N, K, A, lda,
                       (const float2 *)B, ldb, C, ldc);
}

void launch_gemm_cn(hipStream_t st, int M, int N, int K, const void *A, int lda, int a_storage,
                    const double2 *B, int ldb, double2 *C, int ldc) {
  dim3 grid((M + RT - 1) / RT, (N + RT - 1) / RT);
  if (a_storage == 0)
    hipLaunchKernelGGL(k_gemm_cn<double2>, grid, dim3(256), 0, st, M, N, K, (const double2 *)A,
                       lda, B, ldb, C, ldc);
  else
    hipLaunchKernelGGL(k_gemm_cn<float2>, grid, dim3(256), 0, st, M, N, K, (const float2 *)A, lda,
                       B, ldb, C, ldc);
}

// F2[a,s,b] = sum_s' P[s,s'] F[a,s',b]; F is chiA x 2 x chiB
__global__ void k_pauli_phys(const double2 *F, double2 *F2, int chiA, int chiB, double2 p00,
                             double2 p01, double2 p10, double2 p11) {
  size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)chiA * chiB) return;
  size_t a = e / chiB, b = e % chiB;
  double2 f0 = F[(a * 2) * chiB + b], f1 = F[(a * 2 + 1) * chiB + b];
  F2[(a * 2) * chiB + b] = cadd(cmul(p00, f0), cmul(p01, f1));
  F2[(a * 2 + 1) * chiB + b] = cadd(cmul(p10, f0), cmul(p11, f1));
}

void launch_pauli_phys(hipStream_t st, const double2 *F, double2 *F2, int chiA, int chiB,
                       double2 p00, double2 p01, double2 p10, double2 p11) {
  size_t n = (size_t)chiA * chiB;
  hipLaunchKernelGGL(k_pauli_phys, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, F, F2,
                     chiA, chiB, p00, p01, p10, p11);
}

// w[b] = sum_a v[a] A[a, bit, b].  The rows a are split over blockIdx.y
// (chunks of AMP_ROWS) so that a wide bond still fills the GPU; the partial
// sums go to `part` (splits x chiR) and are added in split order.
constexpr int AMP_ROWS = 64;

template <class S>
__global__ __launch_bounds__(256) void k_amp_part(const double2 *v, double2 *part, const S *A,
                                                  int chiL, int chiR, int bit) {
  const int b = blockIdx.x * 256 + threadIdx.x;
  if (b >= chiR) return;
  const int a0 = blockIdx.y * AMP_ROWS, a1 = min(chiL, a0 + AMP_ROWS);
  double2 acc = make_double2(0.0, 0.0);
  for (int a = a0; a < a1; a++) cfma(acc, v[a], cload(A + ((size_t)a * 2 + bit) * chiR + b));
  part[(size_t)blockIdx.y * chiR + b] = acc;
}

__global__ void k_amp_sum(const double2 *part, int splits, int chiR, double2 *w) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= chiR) return;
  double2 acc = part[b];
  for (int k = 1; k < splits; k++) acc = cadd(acc, part[(size_t)k * chiR + b]);
  w[b] = acc;
}

// part needs ceil(chiL / 64) * chiR entries.
void launch_amp_step(hipStream_t st, const double2 *v, double2 *w, double2 *part, const void *A,
                     int storage, int chiL, int chiR, int bit) {
  const int splits = (chiL + AMP_ROWS - 1) / AMP_ROWS;
  dim3 grid((chiR + 255) / 256, splits);
  if (storage == 0)
    hipLaunchKernelGGL(k_amp_part<double2>, grid, dim3(256), 0, st, v, part, (const double2 *)A,
                       chiL, chiR, bit);
  else
    hipLaunchKernelGGL(k_amp_part<float2>, grid, dim3(256), 0, st, v, part, (const float2 *)A,
                       chiL, chiR, bit);
  hipLaunchKernelGGL(k_amp_sum, dim3((chiR + 255) / 256), dim3(256), 0, st, part, splits, chiR, w);
}

}  // namespace tn
