// State kernels: |0...0> initialisation, one-qubit gates, storage conversion.
#include "tnsim_internal.h"
#include "tn_complex.h"

namespace tn {

// |0...0>: every site (1,2,1) = (1, 0), every bond weight (1)   (Sec. IV.A)
__global__ void k_init_state(void *const *sites, int n, int storage, double *const *lams, int nb) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) {
    if (storage == 0) {
      double2 *a = (double2 *)sites[q];
      a[0] = make_double2(1.0, 0.0);
      a[1] = make_double2(0.0, 0.0);
    } else {
      float2 *a = (float2 *)sites[q];
      a[0] = make_float2(1.0f, 0.0f);
      a[1] = make_float2(0.0f, 0.0f);
    }
  }
  if (q < nb) lams[q][0] = 1.0;
}

void launch_init_state(hipStream_t st, void *const *sites, int n, int storage,
                       double *const *lams, int nb) {
  int m = n > nb ? n : nb;
  hipLaunchKernelGGL(k_init_state, dim3((m + 255) / 256), dim3(256), 0, st, sites, n, storage,
                     lams, nb);
}

__global__ void k_fill_zero(uint4 *p, size_t n16) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n16; i += stride) p[i] = make_uint4(0, 0, 0, 0);
}

// Zero a 16-byte aligned region whose size is a multiple of 16 (a kernel, so
// that the call may sit inside a captured graph).
void launch_fill_zero(hipStream_t st, void *p, size_t bytes) {
  size_t n16 = bytes / 16;
  if (!n16) return;
  size_t blocks = (n16 + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(256), 0, st, (uint4 *)p, n16);
}

// One-qubit gates of a layer: A'[a,s',b] = sum_s U[s',s] A[a,s,b]  (eq. 3).
// grid.y = gate, grid.x covers the chiL*chiR (a,b) pairs of the largest site.
template <class S>
__device__ void apply_1q_body(const Gate1Desc &d, int e) {
  S *A = (S *)d.A;
  int a = e / d.chiR, b = e - a * d.chiR;
  size_t i0 = ((size_t)a * 2) * d.chiR + b, i1 = i0 + d.chiR;
  double2 x0 = cload(A + i0), x1 = cload(A + i1);
  double2 y0 = cadd(cmul(d.u[0], x0), cmul(d.u[1], x1));
  double2 y1 = cadd(cmul(d.u[2], x0), cmul(d.u[3], x1));
  cstore(A + i0, y0);
  cstore(A + i1, y1);
}

__global__ void k_apply_1q(const Gate1Desc *descs) {
  const Gate1Desc &d = descs[blockIdx.y];
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= d.chiL * d.chiR) return;
  if (d.storage == 0)
    apply_1q_body<double2>(d, e);
  else
    apply_1q_body<float2>(d, e);
}

void launch_apply_1q(hipStream_t st, const Gate1Desc *d, int ng, int max_elems) {
  if (ng <= 0 || max_elems <= 0) return;
  hipLaunchKernelGGL(k_apply_1q, dim3((max_elems + 255) / 256, ng), dim3(256), 0, st, d);
}

__global__ void k_convert(const void *src, int ss, void *dst, int ds, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) {
    double2 v = ss == 0 ? ((const double2 *)src)[i] : f2d(((const float2 *)src)[i]);
    if (ds == 0)
      ((double2 *)dst)[i] = v;
    else
      ((float2 *)dst)[i] = d2f(v);
  }
}

void launch_convert(hipStream_t st, const void *src, int ss, void *dst, int ds, size_t count) {
  if (!count) return;
  size_t blocks = (count + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_convert, dim3((unsigned)blocks), dim3(256), 0, st, src, ss, dst, ds, count);
}

// Bond propagation (Sec. III.A, non-local gates): one site of the window
// with the gate's operator bond r (rg terms) merged into its bonds.  `old`
// holds the site as it was (complex128, chiL x 2 x chiR); `out` receives
//   role 0 (left site):   out[l, s', r chiR + c]        = sum_x X_r[s',x] old[l,x,c]
//   role 1 (in between):  out[r chiL + l, s, r chiR + c] = old[l,s,c]
//   role 2 (right site):  out[r chiL + l, s', c]        = sum_y Y_r[s',y] old[l,y,c]
// (other entries of a role-1 site, r != r', are zero).  F holds rg 2x2
// factors, row-major.  One thread per output entry.
template <class S>
__global__ void k_prop_merge(const double2 *old, S *out, int chiL, int chiR, int rg, int role,
                             Mat4x4 F) {
  const int nL = role == 0 ? chiL : rg * chiL, nR = role == 2 ? chiR : rg * chiR;
  const size_t total = (size_t)nL * 2 * nR;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int ri = (int)(e % nR), sp = (int)((e / nR) % 2), li = (int)(e / ((size_t)2 * nR));
    double2 v = make_double2(0.0, 0.0);
    if (role == 1) {
      const int r = li / chiL, l = li % chiL, r2 = ri / chiR, c = ri % chiR;
      if (r == r2) v = old[((size_t)l * 2 + sp) * chiR + c];
    } else {
      const int r = role == 0 ? ri / chiR : li / chiL;
      const int l = role == 0 ? li : li % chiL, c = role == 0 ? ri % chiR : ri;
      const double2 *f = F.v[r];
      v = cadd(cmul(f[2 * sp], old[((size_t)l * 2) * chiR + c]),
               cmul(f[2 * sp + 1], old[((size_t)l * 2 + 1) * chiR + c]));
    }
    cstore(out + e, v);
  }
}

void launch_prop_merge(hipStream_t st, const double2 *old, void *out, int storage, int chiL,
                       int chiR, int rg, int role, const Mat4x4 &F) {
  const size_t total = (size_t)(role == 0 ? chiL : rg * chiL) * 2 * (role == 2 ? chiR : rg * chiR);
  size_t blocks = (total + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (storage == 0)
    hipLaunchKernelGGL(k_prop_merge<double2>, dim3((unsigned)blocks), dim3(256), 0, st, old,
                       (double2 *)out, chiL, chiR, rg, role, F);
  else
    hipLaunchKernelGGL(k_prop_merge<float2>, dim3((unsigned)blocks), dim3(256), 0, st, old,
                       (float2 *)out, chiL, chiR, rg, role, F);
}

}  // namespace tn
