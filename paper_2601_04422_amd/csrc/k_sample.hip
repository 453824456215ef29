// Perfect sampling of all qubits (Sec. III.A; Ferris and Vidal, Phys. Rev. B
// 85, 165146 (2012)), many shots at once.
//
// Qubits are drawn from q = n-1 down to 0.  A shot's drawn suffix
// s_{q+1..n-1} is represented by a node vector v (length chi_{q+1}, the
// contraction of the drawn sites, normalised so that v^H E_{q+1} v = 1).
// Shots that drew the same suffix share one node: this is the memo of
// partial contractions, kept as a table of at most min(2^(n-1-q), shots)
// columns per step, so each distinct prefix of the drawing is contracted
// once.  One step at site q:
//
//   W[:, 2j+s] = A_q^s v_j                      (two GEMMs, s = 0, 1)
//   Y          = E_q W                          (one GEMM; E_q = left-block Gram)
//   p[c]       = Re W[:, c]^H Y[:, c]           (weight of node j with bit s)
//   per shot:  bit = u < p[2j] / (p[2j] + p[2j+1]) ? 0 : 1, key = 2j + bit
//   the used keys are numbered in order (scan) and become the next nodes,
//   v' = W[:, key] / sqrt(p[key]).
//
// Everything is float64; the sites are read in their storage precision.
#include <algorithm>

#include "tnsim_internal.h"
#include "tn_complex.h"

namespace tn {

constexpr int ST = 64, SK = 16;

// C[:, c] = A B[:, c] for c < min(bound, mult * *mcount): A is M x K with row
// stride lda (unit stride along K), B is K x cols with column stride ldb
// (unit stride along K), C is M x cols with column stride ldc.
template <class SA>
__global__ __launch_bounds__(256) void k_smp_gemm(int M, int K, int bound, const int *mcount,
                                                  int mult, const SA *A, long long lda,
                                                  const double2 *B, int ldb, double2 *C,
                                                  int ldc) {
  const int ncols = min(bound, mult * *mcount);
  const int j0 = blockIdx.x * ST, i0 = blockIdx.y * ST;
  if (j0 >= ncols) return;
  __shared__ double2 As[SK * ST], Bs[SK * ST];
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  double2 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; i++)
#pragma unroll
    for (int j = 0; j < 4; j++) acc[i][j] = make_double2(0.0, 0.0);
  const int r = tid >> 2, kq = (tid & 3) * 4;
  for (int k0 = 0; k0 < K; k0 += SK) {
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const int gk = k0 + kq + q;
      const int gi = i0 + r, gj = j0 + r;
      As[(kq + q) * ST + r] = (gi < M && gk < K) ? cload(A + gi * lda + gk) : make_double2(0, 0);
      Bs[(kq + q) * ST + r] =
          (gj < ncols && gk < K) ? B[(size_t)gj * ldb + gk] : make_double2(0, 0);
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < SK; kk++) {
      double2 a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; i++) a[i] = As[kk * ST + tx + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; j++) b[j] = Bs[kk * ST + ty + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < 4; j++) cfma(acc[i][j], a[i], b[j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < 4; j++) {
    const int gj = j0 + ty + 16 * j;
    if (gj >= ncols) continue;
#pragma unroll
    for (int i = 0; i < 4; i++) {
      const int gi = i0 + tx + 16 * i;
      if (gi < M) C[(size_t)gj * ldc + gi] = acc[i][j];
    }
  }
}

// p[c] = Re sum_a conj(W[a, c]) Y[a, c], one wave per column.
__global__ __launch_bounds__(256) void k_smp_prob(const double2 *W, const double2 *Y, int M,
                                                  int bound, const int *mcount, double *p) {
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (c >= min(bound, 2 * *mcount)) return;
  double acc = 0.0;
  for (int a = lane; a < M; a += 64) {
    const double2 w = W[(size_t)c * M + a], y = Y[(size_t)c * M + a];
    acc = fma(w.x, y.x, fma(w.y, y.y, acc));
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0) p[c] = acc;
}

// Draw qubit q for every shot.
__global__ void k_smp_decide(int shots, int n, int q, const double *u, const double *p,
                             const int *node, int *key, int *flag, uint8_t *bits, double *logp,
                             int *err) {
  const int shot = blockIdx.x * blockDim.x + threadIdx.x;
  if (shot >= shots) return;
  const double x = u[(size_t)shot * n + q];
  if (!(x >= 0.0 && x < 1.0)) err[0] = 1;
  const int j = node[shot];
  const double p0 = p[2 * j], p1 = p[2 * j + 1], tot = p0 + p1;
  if (!(tot > 0.0)) err[1] = 1;
  const int bit = x < p0 / tot ? 0 : 1;
  const int k = 2 * j + bit;
  bits[(size_t)shot * n + q] = (uint8_t)bit;
  logp[shot] += log((bit ? p1 : p0) / tot);
  key[shot] = k;
  flag[k] = 1;
}

// Number the used keys in order: idx[c] = count of used keys below c,
// idx[ncols] = count; the count becomes the next step's node count
// (ctr[0]) and ncols is kept in ctr[3] for the gather.  Clears the flags it
// reads.  One workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void k_smp_scan(int *flag, int *idx, int *ctr) {
  __shared__ int wsum[16];
  __shared__ int carry_s;
  const int ncols = 2 * ctr[0];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  if (t == 0) carry_s = 0;
  __syncthreads();
  for (int base = 0; base < ncols; base += 1024) {
    const int c = base + t;
    int f = 0;
    if (c < ncols) {
      f = flag[c];
      flag[c] = 0;
    }
    int incl = f;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int y = __shfl_up(incl, off, 64);
      if (lane >= off) incl += y;
    }
    if (lane == 63) wsum[wv] = incl;
    __syncthreads();
    int before = carry_s;
    for (int w = 0; w < wv; w++) before += wsum[w];
    if (c < ncols) idx[c] = before + incl - f;
    __syncthreads();
    if (t == 1023) carry_s = before + incl;
    __syncthreads();
  }
  if (t == 0) {
    idx[ncols] = carry_s;
    ctr[0] = carry_s;
    ctr[3] = ncols;
  }
}

// V'[:, idx[c]] = W[:, c] / sqrt(p[c]) for every used key c < ctr[3] (the
// key count of this step; ctr[0] already holds the next node count).
__global__ __launch_bounds__(256) void k_smp_gather(const double2 *W, const double *p,
                                                    const int *idx, const int *ctr, int M,
                                                    double2 *Vn) {
  const int c = blockIdx.x;
  if (c >= ctr[3]) return;
  const int dst = idx[c];
  if (idx[c + 1] == dst) return;
  const double r = 1.0 / sqrt(p[c]);
  for (int a = blockIdx.y * 256 + threadIdx.x; a < M; a += 256 * gridDim.y)
    Vn[(size_t)dst * M + a] = cscale(W[(size_t)c * M + a], r);
}

__global__ void k_smp_relabel(int shots, const int *key, const int *idx, int *node) {
  const int shot = blockIdx.x * blockDim.x + threadIdx.x;
  if (shot < shots) node[shot] = idx[key[shot]];
}

__global__ void k_smp_init(int shots, int nflag, int *node, double *logp, int *flag,
                           double2 *V, double2 *E0, int *ctr) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < shots) {
    node[t] = 0;
    logp[t] = 0.0;
  }
  if (t < nflag) flag[t] = 0;
  if (t == 0) {
    V[0] = make_double2(1.0, 0.0);
    E0[0] = make_double2(1.0, 0.0);
    ctr[0] = 1;  // one node: the empty suffix
    ctr[1] = 0;  // a uniform outside [0, 1)
    ctr[2] = 0;  // a node of zero weight
    ctr[3] = 0;
  }
}

// ------------------------------------------------------------------ launchers

void launch_smp_init(hipStream_t st, int shots, int *node, double *logp, int *flag, double2 *V,
                     double2 *E0, int *ctr) {
  const int nflag = 2 * shots + 1;
  const int total = std::max(shots, nflag);
  hipLaunchKernelGGL(k_smp_init, dim3((total + 255) / 256), dim3(256), 0, st, shots, nflag, node,
                     logp, flag, V, E0, ctr);
}

void launch_smp_gemm(hipStream_t st, int M, int K, int bound, const int *mcount, int mult,
                     const void *A, int a_storage, long long lda, const double2 *B, int ldb,
                     double2 *C, int ldc) {
  if (bound <= 0 || M <= 0) return;
  dim3 grid((bound + ST - 1) / ST, (M + ST - 1) / ST);
  if (a_storage == 0)
    hipLaunchKernelGGL(k_smp_gemm<double2>, grid, dim3(256), 0, st, M, K, bound, mcount, mult,
                       (const double2 *)A, lda, B, ldb, C, ldc);
  else
    hipLaunchKernelGGL(k_smp_gemm<float2>, grid, dim3(256), 0, st, M, K, bound, mcount, mult,
                       (const float2 *)A, lda, B, ldb, C, ldc);
}

void launch_smp_prob(hipStream_t st, const double2 *W, const double2 *Y, int M, int bound,
                     const int *mcount, double *p) {
  hipLaunchKernelGGL(k_smp_prob, dim3((bound + 3) / 4), dim3(256), 0, st, W, Y, M, bound, mcount,
                     p);
}

void launch_smp_decide(hipStream_t st, int shots, int n, int q, const double *u, const double *p,
                       const int *node, int *key, int *flag, uint8_t *bits, double *logp,
                       int *err) {
  hipLaunchKernelGGL(k_smp_decide, dim3((shots + 255) / 256), dim3(256), 0, st, shots, n, q, u,
                     p, node, key, flag, bits, logp, err);
}

void launch_smp_scan(hipStream_t st, int *flag, int *idx, int *ctr) {
  hipLaunchKernelGGL(k_smp_scan, dim3(1), dim3(1024), 0, st, flag, idx, ctr);
}

void launch_smp_gather(hipStream_t st, const double2 *W, const double *p, const int *idx,
                       const int *ctr, int bound, int M, double2 *Vn) {
  dim3 grid(bound, (M + 255) / 256);
  hipLaunchKernelGGL(k_smp_gather, grid, dim3(256), 0, st, W, p, idx, ctr, M, Vn);
}

void launch_smp_relabel(hipStream_t st, int shots, const int *key, const int *idx, int *node) {
  hipLaunchKernelGGL(k_smp_relabel, dim3((shots + 255) / 256), dim3(256), 0, st, shots, key, idx,
                     node);
}

}  // namespace tn
