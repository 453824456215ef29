// Perfect sampling of all qubits (Sec. III.A; Ferris and Vidal, Phys. Rev. B
// 85, 165146 (2012)), many shots at once.
//
// Qubits are drawn from q = n-1 down to 0.  A shot's drawn suffix
// s_{q+1..n-1} is represented by a node vector v (length chi_{q+1}, the
// contraction of the drawn sites, normalised so that v^H E_{q+1} v = 1 with
// E_q the Gram matrix of sites 0..q-1).  Shots that drew the same suffix
// share one node: this is the memo of partial contractions, a table of at
// most min(2^(n-1-q), shots) columns per step, so each distinct prefix of the
// drawing is contracted once.
//
// Before the draws, one pass over the sites builds, per site,
//   M_q^s = A_q^{s H} E_q A_q^s        (s = 0, 1; E_{q+1} = M_q^0 + M_q^1),
// so that the weight of bit s for node v is v^H M_q^s v.  One step at site q:
//   Y       = [M_q^0; M_q^1] V                    (one GEMM over the nodes)
//   p[2j+s] = Re v_j^H Y_s[:, j]
//   per shot: bit = u < p[2j] / (p[2j] + p[2j+1]) ? 0 : 1; key (s, j)
//   the keys drawn are numbered, those with s = 0 first (scan), and become
//   the next nodes v' = A_q^s v_j / sqrt(p[2j+s])     (one gathered GEMM).
// The GEMMs run on the FP64 matrix cores (k_zgemm.hip); everything is
// float64, the sites are read in their storage precision.
#include <algorithm>

#include "tnsim_internal.h"
#include "tn_complex.h"

namespace tn {

// p[c] = Re sum_b conj(V[b, c/2]) Y[b, c] (Y holds 2M rows per node: s = 0
// then s = 1), one wave per (node, bit).
__global__ __launch_bounds__(256) void k_smp_prob(const double2 *V, const double2 *Y, int M,
                                                  int bound, const int *ctr, double *p) {
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (c >= min(bound, 2 * ctr[0])) return;
  const double2 *v = V + (size_t)(c >> 1) * M, *y = Y + (size_t)c * M;
  double acc = 0.0;
  for (int b = lane; b < M; b += 64) {
    const double2 w = v[b], z = y[b];
    acc = fma(w.x, z.x, fma(w.y, z.y, acc));
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0) p[c] = acc;
}

// Draw qubit q for every shot; key (s, j) is numbered s * m + j.
__global__ void k_smp_decide(int shots, int n, int q, const double *u, const double *p,
                             const int *node, int *key, int *flag, uint8_t *bits, double *logp,
                             int *ctr) {
  const int shot = blockIdx.x * blockDim.x + threadIdx.x;
  if (shot >= shots) return;
  const int m = ctr[0];
  const double x = u[(size_t)shot * n + q];
  if (!(x >= 0.0 && x < 1.0)) ctr[1] = 1;
  const int j = node[shot];
  const double p0 = p[2 * j], p1 = p[2 * j + 1], tot = p0 + p1;
  if (!(tot > 0.0)) ctr[2] = 1;
  const int bit = x < p0 / tot ? 0 : 1;
  const int k = bit * m + j;
  bits[(size_t)shot * n + q] = (uint8_t)bit;
  logp[shot] += log((bit ? p1 : p0) / tot);
  key[shot] = k;
  flag[k] = 1;
}

// Number the drawn keys in order, the keys with s = 1 from the first multiple
// of 64 after those with s = 0 (so that a 64-column tile of next nodes holds
// one bit only; the gap columns become zero nodes that no shot uses):
// idx[c] = number of key c.  ctr[0] <- next node count, ctr[3] <- 2m,
// ctr[4] <- first column of the s = 1 nodes, ctr[6] <- count of s = 0 keys.
// One workgroup of 1024 threads; the flags are cleared by k_smp_parent.
__global__ __launch_bounds__(1024) void k_smp_scan(const int *flag, int *idx, int *ctr) {
  __shared__ int wsum[16];
  __shared__ int carry_s;
  const int m = ctr[0], ncols = 2 * m;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  if (t == 0) carry_s = 0;
  __syncthreads();
  for (int base = 0; base < ncols; base += 1024) {
    const int c = base + t;
    int f = 0;
    if (c < ncols) f = flag[c];
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
  const int c0 = idx[m], c1 = carry_s - c0;  // keys drawn with s = 0, with s = 1
  const int first1 = c1 > 0 ? (c0 + 63) & ~63 : c0;
  __syncthreads();  // every thread has read idx[m] before it moves
  for (int c = m + t; c < ncols; c += 1024) idx[c] += first1 - c0;
  if (t == 0) {
    idx[ncols] = first1 + c1;
    ctr[0] = first1 + c1;
    ctr[3] = ncols;
    ctr[4] = first1;
    ctr[6] = c0;
  }
}

// For every drawn key c = s * m + j: next node idx[c] comes from node j with
// bit s, scaled by 1 / sqrt(p[2j+s]); the gap columns get scale 0.  Clears
// the flags.
__global__ void k_smp_parent(int *flag, const int *idx, const double *p, const int *ctr,
                             int bound, int *parent, double *scale) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int ncols = ctr[3], m = ncols / 2, c0 = ctr[6], first1 = ctr[4];
  if (c < 64 && c0 + c < first1) {
    parent[c0 + c] = 0;
    scale[c0 + c] = 0.0;
  }
  if (c >= min(bound, ncols) || !flag[c]) return;
  flag[c] = 0;
  const int s = c >= m ? 1 : 0, j = c - s * m;
  parent[idx[c]] = j;
  scale[idx[c]] = 1.0 / sqrt(p[2 * j + s]);
}

__global__ void k_smp_relabel(int shots, const int *key, const int *idx, int *node) {
  const int shot = blockIdx.x * blockDim.x + threadIdx.x;
  if (shot < shots) node[shot] = idx[key[shot]];
}

// E = M^0 + M^1 (n entries each, stacked)
__global__ void k_smp_add(const double2 *M01, size_t n, double2 *E) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) E[e] = cadd(M01[e], M01[e + n]);
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
    ctr[4] = 0;
    ctr[5] = 0;  // constant 0: first column of the next nodes
    ctr[6] = 0;
  }
}

// ------------------------------------------------------------------ launchers

void launch_smp_init(hipStream_t st, int shots, int node_cap, int *node, double *logp, int *flag,
                     double2 *V, double2 *E0, int *ctr) {
  const int nflag = 2 * node_cap + 1;
  const int total = std::max(shots, nflag);
  hipLaunchKernelGGL(k_smp_init, dim3((total + 255) / 256), dim3(256), 0, st, shots, nflag, node,
                     logp, flag, V, E0, ctr);
}

void launch_smp_prob(hipStream_t st, const double2 *V, const double2 *Y, int M, int bound,
                     const int *ctr, double *p) {
  hipLaunchKernelGGL(k_smp_prob, dim3((bound + 3) / 4), dim3(256), 0, st, V, Y, M, bound, ctr, p);
}

void launch_smp_decide(hipStream_t st, int shots, int n, int q, const double *u, const double *p,
                       const int *node, int *key, int *flag, uint8_t *bits, double *logp,
                       int *ctr) {
  hipLaunchKernelGGL(k_smp_decide, dim3((shots + 255) / 256), dim3(256), 0, st, shots, n, q, u,
                     p, node, key, flag, bits, logp, ctr);
}

void launch_smp_scan(hipStream_t st, const int *flag, int *idx, int *ctr) {
  hipLaunchKernelGGL(k_smp_scan, dim3(1), dim3(1024), 0, st, flag, idx, ctr);
}

void launch_smp_parent(hipStream_t st, int *flag, const int *idx, const double *p, const int *ctr,
                       int bound, int *parent, double *scale) {
  const int threads = std::max(bound, 64);
  hipLaunchKernelGGL(k_smp_parent, dim3((threads + 255) / 256), dim3(256), 0, st, flag, idx, p,
                     ctr, bound, parent, scale);
}

void launch_smp_relabel(hipStream_t st, int shots, const int *key, const int *idx, int *node) {
  hipLaunchKernelGGL(k_smp_relabel, dim3((shots + 255) / 256), dim3(256), 0, st, shots, key, idx,
                     node);
}

void launch_smp_add(hipStream_t st, const double2 *M01, size_t n, double2 *E) {
  hipLaunchKernelGGL(k_smp_add, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, M01, n, E);
}

}  // namespace tn
