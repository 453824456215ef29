// Readout kernels: transfer-matrix contraction for <bra|P|ket> and amplitudes.
//
//   E_q[b,b'] = sum conj(B_q[a,s,b]) P[s,s'] E_{q-1}[a,a'] K_q[a',s',b']
//
// is done per site as F = E K (GEMM), F2 = P on the physical index, and
// E' = B^H F2 (GEMM with the bra conjugate-transposed), all in float64; the
// two GEMMs are k_zgemm's (k_zgemm.hip), the Pauli step is here.
#include "tnsim_internal.h"
#include "tn_complex.h"

namespace tn {

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
