// Attainable float64 rates of this device: long chains of independent
// v_mfma_f64_16x16x4f64 (matrix cores) or v_fma_f64 (vector ALUs) in every
// wavefront of a grid that fills the chip.  The contraction kernels of the
// Jacobi, the merge and the write-back are read against the first, the pair
// solve against the second.  The results are written out so that no product
// is dropped.  A third form runs both units at once, a fourth the four-block
// v_mfma_f64_4x4x4f64.

#include "tnsim_internal.h"

namespace tn {

typedef double d4_t __attribute__((ext_vector_type(4)));
constexpr int PROBE_CHAINS = 8;

__global__ __launch_bounds__(256) void k_probe_mfma(double *out, int iters) {
  d4_t c[PROBE_CHAINS];
#pragma unroll
  for (int i = 0; i < PROBE_CHAINS; i++) c[i] = d4_t{0.0, 0.0, 0.0, 0.0};
  const double a = 1.0 + threadIdx.x * 1e-9, b = 1.0 - threadIdx.x * 1e-9;
  for (int it = 0; it < iters; it++) {
#pragma unroll
    for (int i = 0; i < PROBE_CHAINS; i++)
      c[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c[i], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < PROBE_CHAINS; i++) s += c[i][0] + c[i][1] + c[i][2] + c[i][3];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_probe_valu(double *out, int iters) {
  double x[PROBE_CHAINS];
#pragma unroll
  for (int i = 0; i < PROBE_CHAINS; i++) x[i] = 1.0 + i + threadIdx.x * 1e-9;
  const double m = 0.999999, add = 1e-7;
  for (int it = 0; it < iters; it++) {
#pragma unroll
    for (int i = 0; i < PROBE_CHAINS; i++) x[i] = __builtin_fma(x[i], m, add);
  }
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < PROBE_CHAINS; i++) s += x[i];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// Chains of the four-block v_mfma_f64_4x4x4f64 (256 multiply-adds each).
__global__ __launch_bounds__(256) void k_probe_mfma4(double *out, int iters) {
  double c[PROBE_CHAINS];
#pragma unroll
  for (int i = 0; i < PROBE_CHAINS; i++) c[i] = 0.0;
  const double a = 1.0 + threadIdx.x * 1e-9, b = 1.0 - threadIdx.x * 1e-9;
  for (int it = 0; it < iters; it++) {
#pragma unroll
    for (int i = 0; i < PROBE_CHAINS; i++) c[i] = __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c[i], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < PROBE_CHAINS; i++) s += c[i];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// Wavefronts 0 and 2 of a workgroup run matrix-core chains, 1 and 3 vector
// chains (four times as many instructions, about the same time alone).
__global__ __launch_bounds__(256) void k_probe_mixed(double *out, int iters) {
  double s = 0.0;
  if ((threadIdx.x >> 6) & 1) {
    double x[PROBE_CHAINS];
#pragma unroll
    for (int i = 0; i < PROBE_CHAINS; i++) x[i] = 1.0 + i + threadIdx.x * 1e-9;
    const double m = 0.999999, add = 1e-7;
    for (int it = 0; it < 4 * iters; it++) {
#pragma unroll
      for (int i = 0; i < PROBE_CHAINS; i++) x[i] = __builtin_fma(x[i], m, add);
    }
#pragma unroll
    for (int i = 0; i < PROBE_CHAINS; i++) s += x[i];
  } else {
    d4_t c[PROBE_CHAINS];
#pragma unroll
    for (int i = 0; i < PROBE_CHAINS; i++) c[i] = d4_t{0.0, 0.0, 0.0, 0.0};
    const double a = 1.0 + threadIdx.x * 1e-9, b = 1.0 - threadIdx.x * 1e-9;
    for (int it = 0; it < iters; it++) {
#pragma unroll
      for (int i = 0; i < PROBE_CHAINS; i++)
        c[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c[i], 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < PROBE_CHAINS; i++) s += c[i][0] + c[i][1] + c[i][2] + c[i][3];
  }
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// Workgroups of 256 threads, `groups` of them; returns the real flops one
// launch performs.
double launch_probe(hipStream_t st, int unit, int groups, int iters, double *out) {
  if (unit == 0) {
    hipLaunchKernelGGL(k_probe_mfma, dim3(groups), dim3(256), 0, st, out, iters);
    // 16 x 16 x 4 multiply-adds per instruction and wavefront, 4 wavefronts
    return 2.0 * 16 * 16 * 4 * PROBE_CHAINS * (double)iters * 4.0 * groups;
  }
  if (unit == 1) {
    hipLaunchKernelGGL(k_probe_valu, dim3(groups), dim3(256), 0, st, out, iters);
    return 2.0 * PROBE_CHAINS * (double)iters * 256.0 * groups;
  }
  if (unit == 3) {
    hipLaunchKernelGGL(k_probe_mfma4, dim3(groups), dim3(256), 0, st, out, iters);
    return 2.0 * 4 * 4 * 4 * 4 * PROBE_CHAINS * (double)iters * 4.0 * groups;
  }
  hipLaunchKernelGGL(k_probe_mixed, dim3(groups), dim3(256), 0, st, out, iters);
  return (2.0 * 16 * 16 * 4 * PROBE_CHAINS * (double)iters * 2.0 +
          2.0 * PROBE_CHAINS * 4.0 * iters * 128.0) *
         groups;
}

}  // namespace tn
