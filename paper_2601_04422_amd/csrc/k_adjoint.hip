// Kernels of the reverse (adjoint) sweep, float64.
//
// Cotangents follow the convention X_bar = dL/d conj(X) for complex tensors
// (so dL = 2 Re sum conj(X_bar) dX) and lambda_bar = dL/d lambda for the real
// Schmidt weights.
#include "tnsim_internal.h"
#include "tn_complex.h"

namespace tn {

// ---------------------------------------------------------------- strided complex GEMM
// C[i][j] (+)= alpha * sum_k opA(i,k) opB(k,j), with element strides and an
// optional conjugation of each operand.  Used for the contractions of the
// adjoint and of the loss environments.  Float64 matrix cores
// (v_mfma_f64_16x16x4f64, three real products per complex one): a 64x64 tile
// of C per workgroup, K in steps of 16 through LDS with the next step loaded
// into registers during the products; wavefront w owns the 32x32 quarter
// (rows 32 (w&1), columns 32 (w>>1)), lane l supplies A[l%16][k + l/16] and
// B[k + l/16][l%16] and holds D[l/16 + 4v][l%16] of each 16x16 tile.
typedef double f64x4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f64x4_t adj_mfma(double a, double b, f64x4_t c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <class SA, class SB>
__global__ __launch_bounds__(256) void k_gemm_gen(GemmArgs g) {
  __shared__ double2 As[16 * 64], Bs[16 * 64];
  const int tid = threadIdx.x;
  const int i0 = blockIdx.x * 64, j0 = blockIdx.y * 64;
  const SA *A = (const SA *)g.A;
  const SB *B = (const SB *)g.B;
  double2 ra[4], rb[4];
  // element e = tid + 256 q of the 16 x 64 step: k = e / 64, row/column e % 64
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const int e = tid + 256 * q, kk = e >> 6, ii = e & 63;
      const int gi = i0 + ii, gj = j0 + ii, gk = k0 + kk;
      double2 v = make_double2(0.0, 0.0);
      if (gi < g.M && gk < g.K) {
        v = cload(A + gi * g.sa_i + gk * g.sa_k);
        if (g.a_conj) v = cconj(v);
      }
      ra[q] = v;
      double2 w = make_double2(0.0, 0.0);
      if (gj < g.N && gk < g.K) {
        w = cload(B + gk * g.sb_k + gj * g.sb_j);
        if (g.b_conj) w = cconj(w);
      }
      rb[q] = w;
    }
  };
  const int wv = tid >> 6, lane = tid & 63, l16 = lane & 15, lg = lane >> 4;
  const int wm = (wv & 1) * 32, wn = (wv >> 1) * 32;
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
  for (int k0 = 0; k0 < g.K; k0 += 16) {
#pragma unroll
    for (int q = 0; q < 4; q++) {
      As[tid + 256 * q] = ra[q];
      Bs[tid + 256 * q] = rb[q];
    }
    __syncthreads();
    if (k0 + 16 < g.K) load(k0 + 16);
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
          c1[x][y] = adj_mfma(a[x].x, b[y].x, c1[x][y]);
          c2[x][y] = adj_mfma(a[x].y, b[y].y, c2[x][y]);
          c3[x][y] = adj_mfma(a[x].x + a[x].y, b[y].x + b[y].y, c3[x][y]);
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < 2; x++)
#pragma unroll
    for (int y = 0; y < 2; y++) {
      const int gj = j0 + wn + 16 * y + l16;
#pragma unroll
      for (int v = 0; v < 4; v++) {
        const int gi = i0 + wm + 16 * x + lg + 4 * v;
        if (gi < g.M && gj < g.N) {
          double2 *c = g.C + gi * g.sc_i + gj * g.sc_j;
          const double2 val = cmul(g.alpha, make_double2((c1[x][y][v] - c2[x][y][v]), (c3[x][y][v] - c1[x][y][v] - c2[x][y][v])));
          *c = g.accumulate ? cadd(*c, val) : val;
        }
      }
    }
}

void launch_gemm_gen(hipStream_t st, const GemmArgs &g) {
  if (g.M <= 0 || g.N <= 0) return;
  dim3 grid((g.M + 63) / 64, (g.N + 63) / 64);
  if (g.a_storage == 0 && g.b_storage == 0)
    hipLaunchKernelGGL((k_gemm_gen<double2, double2>), grid, dim3(256), 0, st, g);
  else if (g.a_storage == 0)
    hipLaunchKernelGGL((k_gemm_gen<double2, float2>), grid, dim3(256), 0, st, g);
  else if (g.b_storage == 0)
    hipLaunchKernelGGL((k_gemm_gen<float2, double2>), grid, dim3(256), 0, st, g);
  else
    hipLaunchKernelGGL((k_gemm_gen<float2, float2>), grid, dim3(256), 0, st, g);
}

// ---------------------------------------------------------------- small element kernels

__global__ void k_fill_c(double2 *p, size_t n, double2 v) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

void launch_fill_c(hipStream_t st, double2 *p, size_t n, double2 v) {
  if (!n) return;
  hipLaunchKernelGGL(k_fill_c, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
}

// Truncated-SVD adjoint, middle step.  C = U_full^H U_bar (m x k, column-major
// with leading dim m); lam2[l] = sigma_l^2 of the full basis (sorted like
// U_full); sbar[j] = dL/d sigma_j for the kept j < k.  Output Abar = F o C
// with the Lorentzian-broadened F_lj = (l_j - l_l) / ((l_j - l_l)^2 + eta)
// off the diagonal, and sbar_j / (4 sigma_j) on it (the Hermitian Gram
// carries sigma^2; the factor follows from d sigma = d(sigma^2) / (2 sigma)
// and the 2 Re convention).
__global__ void k_svd_adj_mid(const double2 *C, double2 *Abar, const double *lam2,
                              const double *sbar, int m, int k, double eta) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m * k) return;
  int l = e % m, j = e / m;
  double2 v;
  if (l == j) {
    double s = sqrt(lam2[j]);
    v = make_double2(s > 0.0 ? sbar[j] / (4.0 * s) : 0.0, 0.0);
  } else {
    double dl = lam2[j] - lam2[l];
    double f = dl / (dl * dl + eta);
    v = cscale(C[e], f);
  }
  Abar[e] = v;
}

void launch_svd_adj_mid(hipStream_t st, const double2 *C, double2 *Abar, const double *lam2,
                        const double *sbar, int m, int k, double eta) {
  int n = m * k;
  if (n <= 0) return;
  hipLaunchKernelGGL(k_svd_adj_mid, dim3((n + 255) / 256), dim3(256), 0, st, C, Abar, lam2, sbar,
                     m, k, eta);
}

// S = H + H^H for an m x m column-major matrix (out of place).
__global__ void k_herm_sum(const double2 *H, double2 *S, int m) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m * m) return;
  int r = e % m, c = e / m;
  S[e] = cadd(H[e], cconj(H[(size_t)r * m + c]));
}

void launch_herm_sum(hipStream_t st, const double2 *H, double2 *S, int m) {
  int n = m * m;
  if (n <= 0) return;
  hipLaunchKernelGGL(k_herm_sum, dim3((n + 255) / 256), dim3(256), 0, st, H, S, m);
}

// Mbar (m x n row-major) -> theta'_bar += Mbar diag(lambda_{i+1})  (column c of
// the (t, c) index), and lambda_bar[c] += 2 Re sum conj(Mbar) theta' over the
// rows and both t.  One thread per c.
__global__ void k_weight_adj(const double2 *Mbar, const double2 *Tp, double2 *Tbar,
                             const double *lam, double *lambar, int m, int chiR) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= chiR) return;
  const int n = 2 * chiR;
  double w = lam ? lam[c] : 1.0;
  double acc = 0.0;
  for (int r = 0; r < m; r++)
    for (int t = 0; t < 2; t++) {
      size_t o = (size_t)r * n + t * chiR + c;
      double2 mb = Mbar[o];
      Tbar[o] = cadd(Tbar[o], cscale(mb, w));
      double2 tp = Tp[o];
      acc += mb.x * tp.x + mb.y * tp.y;
    }
  if (lam && lambar) lambar[c] += 2.0 * acc;
}

void launch_weight_adj(hipStream_t st, const double2 *Mbar, const double2 *Tp, double2 *Tbar,
                       const double *lam, double *lambar, int m, int chiR) {
  hipLaunchKernelGGL(k_weight_adj, dim3((chiR + 63) / 64), dim3(64), 0, st, Mbar, Tp, Tbar, lam,
                     lambar, m, chiR);
}

// M = theta' diag(lambda) (m x n row-major)
__global__ void k_weight_apply(const double2 *Tp, double2 *M, const double *lam, int m, int chiR) {
  size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int n = 2 * chiR;
  if (e >= (size_t)m * n) return;
  int c = (int)(e % n) % chiR;
  M[e] = cscale(Tp[e], lam ? lam[c] : 1.0);
}

void launch_weight_apply(hipStream_t st, const double2 *Tp, double2 *M, const double *lam, int m,
                         int chiR) {
  size_t n = (size_t)m * 2 * chiR;
  hipLaunchKernelGGL(k_weight_apply, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, Tp, M,
                     lam, m, chiR);
}

// theta_bar = G^H applied on the (s, t) pair of theta'_bar (m x n row-major, m = 2 chiL,
// n = 2 chiR), in place.
__global__ void k_gate_adj(double2 *T, int chiL, int chiR, Mat16 G) {
  const double2 *g = G.v;
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= chiL * chiR) return;
  int a = e / chiR, c = e % chiR;
  const int n = 2 * chiR;
  double2 v[4];
  for (int s = 0; s < 2; s++)
    for (int t = 0; t < 2; t++) v[2 * s + t] = T[(size_t)(2 * a + s) * n + t * chiR + c];
  for (int s = 0; s < 2; s++)
    for (int t = 0; t < 2; t++) {
      // (G^H)[st][s't'] = conj(G[s't'][st])
      double2 o = make_double2(0.0, 0.0);
      for (int j = 0; j < 4; j++) cfma(o, cconj(g[j * 4 + 2 * s + t]), v[j]);
      T[(size_t)(2 * a + s) * n + t * chiR + c] = o;
    }
}

void launch_gate_adj(hipStream_t st, double2 *T, int chiL, int chiR, const Mat16 &g) {
  int n = chiL * chiR;
  hipLaunchKernelGGL(k_gate_adj, dim3((n + 255) / 256), dim3(256), 0, st, T, chiL, chiR, g);
}

// One-qubit gate adjoint on site cotangent Abar (chiL x 2 x chiR, complex128):
//   Ubar[s'][s] += sum_{a,b} Abar[a,s',b] conj(Aold[a,s,b])  (4 atomics per block)
//   Abar <- U^H Abar on the physical index
template <class S>
__global__ void k_1q_adj(double2 *Abar, const S *Aold, int chiL, int chiR, Mat4 U,
                         double *ubar /* 8 doubles */) {
  const double2 *u = U.v;
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  double2 part[4] = {make_double2(0, 0), make_double2(0, 0), make_double2(0, 0),
                     make_double2(0, 0)};
  if (e < chiL * chiR) {
    int a = e / chiR, b = e % chiR;
    size_t i0 = ((size_t)a * 2) * chiR + b, i1 = i0 + chiR;
    double2 g0 = Abar[i0], g1 = Abar[i1];
    double2 x0 = cload(Aold + i0), x1 = cload(Aold + i1);
    part[0] = cmulc(x0, g0);  // Ubar[0][0] += g0 conj(x0)
    part[1] = cmulc(x1, g0);  // Ubar[0][1]
    part[2] = cmulc(x0, g1);  // Ubar[1][0]
    part[3] = cmulc(x1, g1);  // Ubar[1][1]
    // U^H: [[conj u00, conj u10], [conj u01, conj u11]]
    Abar[i0] = cadd(cmulc(u[0], g0), cmulc(u[2], g1));
    Abar[i1] = cadd(cmulc(u[1], g0), cmulc(u[3], g1));
  }
  for (int q = 0; q < 4; q++) {
    double re = part[q].x, im = part[q].y;
    for (int off = 32; off > 0; off >>= 1) {
      re += __shfl_down(re, off, 64);
      im += __shfl_down(im, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
      atomicAdd(&ubar[2 * q], re);
      atomicAdd(&ubar[2 * q + 1], im);
    }
  }
}

void launch_1q_adj(hipStream_t st, double2 *Abar, const void *Aold, int storage, int chiL,
                   int chiR, const Mat4 &u, double *ubar) {
  int n = chiL * chiR;
  dim3 grid((n + 255) / 256);
  if (storage == 0)
    hipLaunchKernelGGL(k_1q_adj<double2>, grid, dim3(256), 0, st, Abar, (const double2 *)Aold,
                       chiL, chiR, u, ubar);
  else
    hipLaunchKernelGGL(k_1q_adj<float2>, grid, dim3(256), 0, st, Abar, (const float2 *)Aold, chiL,
                       chiR, u, ubar);
}

// out += Re sum conj(x_i) y_i  (x, y complex128 or site storage), one atomic per wavefront
template <class S>
__global__ void k_dot_re(const double2 *x, const S *y, size_t n, double *out) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  double v = 0.0;
  if (i < n) {
    double2 a = x[i], b = cload(y + i);
    v = a.x * b.x + a.y * b.y;
  }
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  if ((threadIdx.x & 63) == 0) atomicAdd(out, v);
}

void launch_dot_re(hipStream_t st, const double2 *x, const void *y, int y_storage, size_t n,
                   double *out) {
  if (!n) return;
  dim3 grid((unsigned)((n + 255) / 256));
  if (y_storage == 0)
    hipLaunchKernelGGL(k_dot_re<double2>, grid, dim3(256), 0, st, x, (const double2 *)y, n, out);
  else
    hipLaunchKernelGGL(k_dot_re<float2>, grid, dim3(256), 0, st, x, (const float2 *)y, n, out);
}

// Normalisation adjoint: dots[0] = Re<Abar_{i+1}', A_{i+1}'>, lam2 = sigma^2
// (descending), lambark = cotangent of lambda' = sigma/N (k entries, may be
// null).  N = sqrt(sum_{j<k} sigma_j^2), so
//   Nbar   = -2 dots[0] / N - sum_j lambark_j sigma_j / N^2
//   sbar_j = lambark_j / N + Nbar sigma_j / N
__global__ void k_sigma_bar(const double *dots, const double *lambark, const double *lam2,
                            double N, int k, double *sbar) {
  __shared__ double s_dl;
  if (threadIdx.x == 0) {
    double dl = 0.0;
    if (lambark)
      for (int j = 0; j < k; j++) dl += lambark[j] * sqrt(lam2[j]);
    s_dl = dl;
  }
  __syncthreads();
  const double Nbar = -2.0 * dots[0] / N - s_dl / (N * N);
  for (int j = threadIdx.x; j < k; j += blockDim.x) {
    double sj = sqrt(lam2[j]);
    sbar[j] = (lambark ? lambark[j] : 0.0) / N + Nbar * sj / N;
  }
}

void launch_sigma_bar(hipStream_t st, const double *dots, const double *lambark,
                      const double *lam2, double N, int k, double *sbar) {
  hipLaunchKernelGGL(k_sigma_bar, dim3(1), dim3(256), 0, st, dots, lambark, lam2, N, k, sbar);
}

// d loss / d angle for a rotation R_P(t) = exp(-i t P/2):  dR/dt = -(i/2) P R,
// grad += 2 Re sum conj(Ubar) dR/dt.  ubar: 8 doubles (2x2 complex row-major).
__global__ void k_angle_grad(const double *ubar, Mat4 U, int axis, double *grad) {
  if (threadIdx.x != 0) return;
  const double2 *u = U.v;
  // P rows: X = [[0,1],[1,0]], Y = [[0,-i],[i,0]], Z = [[1,0],[0,-1]]
  double2 P[4];
  if (axis == 0) {
    P[0] = make_double2(0, 0); P[1] = make_double2(1, 0);
    P[2] = make_double2(1, 0); P[3] = make_double2(0, 0);
  } else if (axis == 1) {
    P[0] = make_double2(0, 0); P[1] = make_double2(0, -1);
    P[2] = make_double2(0, 1); P[3] = make_double2(0, 0);
  } else {
    P[0] = make_double2(1, 0); P[1] = make_double2(0, 0);
    P[2] = make_double2(0, 0); P[3] = make_double2(-1, 0);
  }
  double acc = 0.0;
  for (int r = 0; r < 2; r++)
    for (int c = 0; c < 2; c++) {
      double2 pu = cadd(cmul(P[2 * r], u[c]), cmul(P[2 * r + 1], u[2 + c]));  // (P U)[r][c]
      double2 du = make_double2(0.5 * pu.y, -0.5 * pu.x);                    // -(i/2) P U
      double2 ub = make_double2(ubar[2 * (2 * r + c)], ubar[2 * (2 * r + c) + 1]);
      acc += ub.x * du.x + ub.y * du.y;  // Re(conj(ub) du)
    }
  *grad += 2.0 * acc;
}

void launch_angle_grad(hipStream_t st, const double *ubar, const Mat4 &u, int axis,
                       double *grad) {
  hipLaunchKernelGGL(k_angle_grad, dim3(1), dim3(64), 0, st, ubar, u, axis, grad);
}

// Gather the full left basis in descending sigma order: U[:, j] = J[:, perm[j]],
// lam2[j] = sig2[perm[j]] (m columns, U column-major with leading dim m).
__global__ void k_gather_basis(const double2 *J, int ldj, const int *perm, const double *sig2,
                               double2 *U, double *lam2, int m) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m * m) return;
  int r = e % m, j = e / m;
  int col = perm[j];
  U[e] = J[(size_t)col * ldj + r];
  if (r == 0) lam2[j] = sig2[col];
}

void launch_gather_basis(hipStream_t st, const double2 *J, int ldj, const int *perm,
                         const double *sig2, double2 *U, double *lam2, int m) {
  int n = m * m;
  hipLaunchKernelGGL(k_gather_basis, dim3((n + 255) / 256), dim3(256), 0, st, J, ldj, perm, sig2,
                     U, lam2, m);
}

// Full-order permutation of all `cols` columns by descending norm (ties by
// index), written into perm (a one-block bitonic sort, cols <= 4096).
__global__ void k_sort_all(const double *sig2, int cols, int *perm) {
  __shared__ double key[4096];
  __shared__ int idx[4096];
  const int tid = threadIdx.x;
  int P = 1;
  while (P < cols) P <<= 1;
  for (int j = tid; j < P; j += blockDim.x) {
    key[j] = j < cols ? sig2[j] : -1.0;
    idx[j] = j;
  }
  __syncthreads();
  for (int size = 2; size <= P; size <<= 1)
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int j = tid; j < P; j += blockDim.x) {
        int l = j ^ stride;
        if (l > j) {
          bool up = ((j & size) == 0);
          double kj = key[j], kl = key[l];
          int ij = idx[j], il = idx[l];
          bool j_first = (kj > kl) || (kj == kl && ij < il);
          if (up ? !j_first : j_first) {
            key[j] = kl;
            key[l] = kj;
            idx[j] = il;
            idx[l] = ij;
          }
        }
      }
      __syncthreads();
    }
  for (int j = tid; j < cols; j += blockDim.x) perm[j] = idx[j];
}

void launch_sort_all(hipStream_t st, const double *sig2, int cols, int *perm) {
  hipLaunchKernelGGL(k_sort_all, dim3(1), dim3(256), 0, st, sig2, cols, perm);
}

}  // namespace tn
