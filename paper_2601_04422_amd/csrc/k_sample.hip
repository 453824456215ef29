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
// (the GEMMs, and those that build E_q, run on the matrix cores: k_zgemm.hip)
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
