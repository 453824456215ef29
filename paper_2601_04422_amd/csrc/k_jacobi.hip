// Truncated SVD of M by block one-sided Jacobi in float64.
//
// The paper decomposes the merged two-site tensor with a Jacobi SVD on the
// GPU (Sec. IV.A, cusolverDnZgesvdj).  Here the columns of X (X = M, or M^H
// when M is wide, with J accumulating the left vectors) are split into
// blocks of 32.  A sweep runs the round-robin tournament over the blocks; in
// one round every block is paired with one other block, and for every pair:
//
//   k_gram_mfma2 : G = X_IJ^H X_IJ (64x64 Hermitian), split over row chunks;
//   k_eig        : G = V D V^H by cyclic two-sided Jacobi in LDS; a pair whose
//                  columns are already orthogonal to tolerance is left alone;
//   k_rot_mfma3  : X_IJ <- X_IJ V (and J_IJ <- J_IJ V).
//
// All pairs of all gates of a batch run in the same launches.  The sweep
// ends the rounds; a gate converges after a sweep in which no pair rotated.
// Then k_colnorm gives sigma_j^2 = ||x_j||^2 and k_trunc sorts them and
// applies the truncation rule.

#include "tnsim_internal.h"
#include "tn_complex.h"
#include "tn_buffer.h"

namespace tn {

// A column whose squared norm is below (rows * 2^-53)^2 ||X||_F^2 is rounding
// noise (far under the truncation's numerical-zero floor); pairs holding one
// are not rotated.
__device__ __forceinline__ double small_norm2(const GateDesc &d) {
  const double r = d.rows * 0x1p-53;
  return d.sc->fro2 * r * r;
}

// Round-robin tournament: pair k of round r over P players (P even).
__device__ __forceinline__ void rr_pair(int r, int k, int P, int &p, int &q) {
  if (k == 0) {
    p = P - 1;
    q = r;
  } else {
    p = (r + k) % (P - 1);
    q = (r - k + (P - 1)) % (P - 1);
  }
  if (p > q) {
    int t = p;
    p = q;
    q = t;
  }
}

__device__ __forceinline__ int pair_col(int I, int J, int p) {
  return p < BW ? I * BW + p : J * BW + (p - BW);
}

// A block pair that tested orthogonal and whose two blocks have not been
// rotated since has the same Gram matrix as then, so it would test orthogonal
// again: its Gram and pair solve are skipped (the result is unchanged).
__device__ __forceinline__ bool pair_known_orthogonal(const GateDesc &d, int I, int J) {
  if (!d.blkVer) return false;
  const int2 s = d.pairSeen[I * d.nblk + J];
  return s.x == d.blkVer[I] && s.y == d.blkVer[J];
}

// ---------------------------------------------------------------- setup

// Zero X's padding columns; J = identity (trans gates).
__global__ void k_setup_slots(const GateDesc *descs) {
  const GateDesc &d = descs[blockIdx.y];
  int col = blockIdx.x;
  if (col < d.colsPad && col >= d.cols) {
    for (int r = threadIdx.x; r < d.ldx; r += blockDim.x)
      d.X[(size_t)col * d.ldx + r] = make_double2(0.0, 0.0);
  }
  if (d.trans && col < d.colsPad) {
    for (int r = threadIdx.x; r < d.ldj; r += blockDim.x)
      d.J[(size_t)col * d.ldj + r] = make_double2(r == col ? 1.0 : 0.0, 0.0);
  }
}

void launch_setup_slots(hipStream_t st, const GateDesc *d, int ng, int max_cols_pad, int) {
  if (ng <= 0) return;
  hipLaunchKernelGGL(k_setup_slots, dim3(max_cols_pad, ng), dim3(256), 0, st, d);
}

// sigma_j^2 = ||x_j||^2, one wavefront per column.
__global__ __launch_bounds__(256) void k_colnorm(const GateDesc *descs) {
  const GateDesc &d = descs[blockIdx.y];
  int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int col = blockIdx.x * 4 + wave;
  if (col >= d.colsPad) return;
  const double2 *x = d.X + (size_t)col * d.ldx;
  double s = 0.0;
  for (int r = lane; r < d.rows; r += 64) s += cabs2(x[r]);
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) d.sig2[col] = s;
}

void launch_colnorm(hipStream_t st, const GateDesc *d, int ng, int max_cols) {
  if (ng <= 0) return;
  hipLaunchKernelGGL(k_colnorm, dim3((max_cols + 3) / 4, ng), dim3(256), 0, st, d);
}

// ||X||_F^2 in a fixed order; all gates start active; no block pair is known
// orthogonal yet.
__global__ void k_gate_init(const GateDesc *descs) {
  const GateDesc &d = descs[blockIdx.x];
  if (d.blkVer) {
    for (int b = threadIdx.x; b < d.nblk; b += blockDim.x) d.blkVer[b] = 0;
    for (int e = threadIdx.x; e < d.nblk * d.nblk; e += blockDim.x)
      d.pairSeen[e] = make_int2(-1, -1);
  }
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int j = 0; j < d.cols; j++) s += d.sig2[j];
    d.sc->fro2 = s;
    d.sc->rot = 1;
    d.sc->active = 1;
    d.sc->k = 0;
  }
}

void launch_gate_init(hipStream_t st, const GateDesc *d, int ng) {
  if (ng <= 0) return;
  hipLaunchKernelGGL(k_gate_init, dim3(ng), dim3(64), 0, st, d);
}

// A gate keeps sweeping only if some pair rotated in the previous sweep.
__global__ void k_begin_sweep(const GateDesc *descs, int ng) {
  int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ng) return;
  SlotScalars *sc = descs[g].sc;
  sc->active = sc->rot;
  sc->rot = 0;
}

void launch_begin_sweep(hipStream_t st, const GateDesc *d, int ng) {
  if (ng <= 0) return;
  hipLaunchKernelGGL(k_begin_sweep, dim3((ng + 63) / 64), dim3(64), 0, st, d, ng);
}

// ---------------------------------------------------------------- Gram of a column pair

typedef double d4_t __attribute__((ext_vector_type(4)));
// v_mfma_f64_16x16x4f64 operand layout (lane l = 0..63): A[l%16][l/16],
// B[l/16][l%16]; result entry v of lane l is D[l/16 + 4v][l%16] (rows
// strided by 4, unlike the float32 16x16 results).

__device__ __forceinline__ d4_t mfma64(double a, double b, d4_t c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Pair Gram on float64 matrix cores (v_mfma_f64_16x16x4), without LDS
// staging.  G is Hermitian, so only its 10 upper 16x16 tiles are computed (the
// pair solve mirrors the lower triangle).  In one k-step (4 rows) lane l reads
// row 4 s + l/16 of the pair's columns 16 t + l%16 (t = 0..3): that is both
// the A operand (conjugated) and the B operand of v_mfma_f64_16x16x4 for
// every tile.  Each complex product conj(x) y takes three real products
// (Gauss): with x = a + ib, y = c + id, P1 = a c, P2 = b d,
// P3 = (a - b)(c + d), conj(x) y = (P1 + P2) + i (P3 - P1 + P2).  Waves 0
// and 1 compute tiles 0-4, which use all four column groups, waves 2 and 3
// tiles 5-9, which use groups 1-3 (15 MFMAs per k-step either way); the two
// waves of a set take alternate 16-row tiles, and their partial Grams are
// summed in LDS in a fixed order at the end.
constexpr int GT_A[10] = {0, 0, 0, 0, 1, 1, 1, 2, 2, 3};
constexpr int GT_B[10] = {0, 1, 2, 3, 1, 2, 3, 2, 3, 3};

template <int SET>
__device__ __forceinline__ void gram_tiles(BufRes rI, BufRes rJ, int ld, int rbeg, int rend,
                                           int half, int l16, int lg, d4_t (&p1)[5],
                                           d4_t (&p2)[5], d4_t (&p3)[5]) {
  constexpr int U0 = SET * 5, T0 = SET;  // tiles U0..U0+4 use column groups T0..3
  // loads of the 16-lane column groups T0..3 for one k-step (4 rows): buffer
  // loads (columns 16 t + l%16 of the pair, block I for t < 2), never
  // skipped (a row past the chunk reads what lies there, or zero past the
  // block, and is zeroed when used), so that the loads in flight are counted
  // exactly
  auto load_step = [&](double2 *x, int r) {
#pragma unroll
    for (int t = T0; t < 4; t++) x[t] = bload(t < 2 ? rI : rJ, (16 * (t & 1) + l16) * ld + r);
  };
  auto mfma_step = [&](const double2 *xin, int r) {
    // the step's own operands only: nothing of a later step is hoisted here
    // (its loads are still in flight)
    __builtin_amdgcn_sched_barrier(0);
    double2 x[4];
#pragma unroll
    for (int t = T0; t < 4; t++) x[t] = r < rend ? xin[t] : make_double2(0.0, 0.0);
    double dm[4], sp[4];  // a - b of the A operand, c + d of the B operand
#pragma unroll
    for (int t = T0; t < 4; t++) {
      dm[t] = x[t].x - x[t].y;
      sp[t] = x[t].x + x[t].y;
    }
#pragma unroll
    for (int u = 0; u < 5; u++) {
      const int ta = GT_A[U0 + u], tb = GT_B[U0 + u];
      const double2 a = x[ta], b = x[tb];  // G_pq += conj(x_rp) x_rq
      p1[u] = mfma64(a.x, b.x, p1[u]);
      p2[u] = mfma64(a.y, b.y, p2[u]);
      p3[u] = mfma64(dm[ta], sp[tb], p3[u]);
    }
    __builtin_amdgcn_sched_barrier(0);
  };
  // the wavefront's k-steps: 16-row tiles base, base + 32, ... (the other
  // wavefront of the set takes the tiles in between), 4 steps per tile;
  // loads run three steps ahead of the products
  const int base = rbeg + half * 16;
  const int nstep = base < rend ? (rend - base + 31) / 32 * 4 : 0;
  auto row_of = [&](int n) { return base + 32 * (n >> 2) + 4 * (n & 3) + lg; };
  if (nstep == 0) return;
  double2 x0[4], x1[4], x2[4], x3[4];
  load_step(x0, row_of(0));
  load_step(x1, row_of(1));
  load_step(x2, row_of(2));
  for (int n = 0; n < nstep; n += 4) {
    load_step(x3, row_of(n + 3));
    mfma_step(x0, row_of(n));
    load_step(x0, row_of(n + 4));
    mfma_step(x1, row_of(n + 1));
    load_step(x1, row_of(n + 5));
    mfma_step(x2, row_of(n + 2));
    load_step(x2, row_of(n + 6));
    mfma_step(x3, row_of(n + 3));
  }
}

__global__ __launch_bounds__(256, 2) void k_gram_mfma2(const GateDesc *descs, int round,
                                                       int ksplit) {
  const GateDesc &d = descs[blockIdx.y];
  const int pairIdx = blockIdx.x / ksplit, kc = blockIdx.x % ksplit;
  if (!d.sc->active || round >= d.nblk - 1 || pairIdx >= d.nblk / 2) return;
  int I, J;
  rr_pair(round, pairIdx, d.nblk, I, J);
  if (pair_known_orthogonal(d, I, J)) return;
  int chunk = (d.rows + ksplit - 1) / ksplit;
  chunk = (chunk + 15) / 16 * 16;
  const int rbeg = kc * chunk;
  const int rend = min(d.rows, rbeg + chunk);
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform (scalar)
  const int l16 = lane & 15, lg = lane >> 4;
  const int ld = d.ldx;
  const BufRes rI = make_res(d.X + (size_t)I * BW * ld, BW * ld);
  const BufRes rJ = make_res(d.X + (size_t)J * BW * ld, BW * ld);
  d4_t p1[5], p2[5], p3[5];
#pragma unroll
  for (int u = 0; u < 5; u++) {
    p1[u] = d4_t{0.0, 0.0, 0.0, 0.0};
    p2[u] = d4_t{0.0, 0.0, 0.0, 0.0};
    p3[u] = d4_t{0.0, 0.0, 0.0, 0.0};
  }
  const int set = wave >> 1, half = wave & 1;
  if (set == 0)
    gram_tiles<0>(rI, rJ, ld, rbeg, rend, half, l16, lg, p1, p2, p3);
  else
    gram_tiles<1>(rI, rJ, ld, rbeg, rend, half, l16, lg, p1, p2, p3);
  // sum of the two wavefronts of each set, the first one's partial first
  __shared__ double red[10][4][64][2];
  for (int h = 0; h < 2; h++) {
    if (half == h) {
#pragma unroll
      for (int u = 0; u < 5; u++)
#pragma unroll
        for (int v = 0; v < 4; v++) {
          const double gr = p1[u][v] + p2[u][v], gi = p3[u][v] - p1[u][v] + p2[u][v];
          double *o = red[set * 5 + u][v][lane];
          if (h == 0) {
            o[0] = gr;
            o[1] = gi;
          } else {
            o[0] += gr;
            o[1] += gi;
          }
        }
    }
    __syncthreads();
  }
  if (tid == 0 && d.ctr && rend > rbeg) {
    atomicAdd(&d.ctr[CTR_GRAM_FLOP], 8ull * (rend - rbeg) * (PW * (PW + 1) / 2));
    atomicAdd(&d.ctr[CTR_GRAM_BYTE], 16ull * (rend - rbeg) * PW + 16ull * PW * PW);
  }
  double2 *G = d.Gp + ((size_t)kc * d.gpStride + pairIdx) * (PW * PW);
  for (int e = tid; e < 10 * 4 * 64; e += 256) {
    const int u = e / 256, v = (e / 64) % 4, l = e % 64;
    const int p = GT_A[u] * 16 + (l >> 4) + 4 * v, q = GT_B[u] * 16 + (l & 15);
    G[p * PW + q] = make_double2(red[u][v][l][0], red[u][v][l][1]);
  }
}

// ---------------------------------------------------------------- 64x64 Hermitian Jacobi

constexpr int LDG = PW + 1;
constexpr int EIG_THREADS = 512;  // 8 wavefronts; two pair solves share a CU
constexpr int EIG_VROWS = PW / (EIG_THREADS / 64);  // rows of V held by each wavefront
constexpr int EIG_OFFD = (PW / 2) * (PW / 2 - 1) / 2;  // off-diagonal 2x2 blocks (i < j)

// Order of the 2016 column pairs of a pair solve (columns 0-31 from block I,
// 32-63 from block J).  Rounds 0-31 pair the blocks: slot k pairs column k
// with column 32 + (k + r) mod 32.  Rounds 32-62 pair columns inside each
// block by the circle method on 32 (round r' = r - 32; slots 0-15 block I,
// 16-31 block J, s = k mod 16): s = 0 pairs 31 with r', s >= 1 pairs
// (r' + s) mod 31 with (r' - s) mod 31.  After the first outer sweep a
// block's own columns enter a pair solve mutually orthogonal (its last pair
// solve made them so), so in the later sweeps the rounds inside the blocks
// often rotate nothing and cost only their rotation test.  Neighbouring
// slots hold neighbouring columns (distinct LDS banks of row * 65 + column).
__device__ __forceinline__ void eig_pair(int r, int k, int &p, int &q) {
  constexpr int H = PW / 2;
  if (r < H) {
    p = k;
    q = H + ((k + r) & (H - 1));
    return;
  }
  const int rr = r - H, off = k >= H / 2 ? H : 0, s = k & (H / 2 - 1);
  if (s == 0) {
    p = H - 1;
    q = rr;
  } else {
    p = rr + s;
    if (p >= H - 1) p -= H - 1;
    q = rr - s;
    if (q < 0) q += H - 1;
  }
  p += off;
  q += off;
}

// Off-diagonal entry (a, b), a != b, of the Hermitian pair Gram: only the
// upper triangle is stored, entry (a, b) at min(a, b) * 65 + max(a, b).
__device__ __forceinline__ int gslot(int a, int b) { return a < b ? a * LDG + b : b * LDG + a; }

// Cyclic two-sided Jacobi on the pair Gram G (64x64 Hermitian, in LDS) with
// the rotations accumulated in V.  A round applies the 32 disjoint rotations
// of the tournament at once: G <- R^H G R, V <- V R.  G keeps its upper
// triangle only (the diagonal in a separate array): the 496 off-diagonal
// 2x2 blocks (rows of pair i x columns of pair j, i < j) are updated by one
// thread each, and the 2x2 diagonal block of a rotating pair takes its
// exact values (new diagonal entries, zero coupling) when the rotation is
// computed.  V lives in registers: wavefront w holds rows 8w .. 8w + 7,
// lane j column j, and a lane takes its rotation partner's entries by a
// lane permute, so LDS holds only G and the rotation parameters (69 KB:
// two solves per CU).  The rotations of round r + 1 are computed by the
// first wavefront while the others apply round r to V (parameters double-
// buffered), so a round costs two barriers (one if it rotates nothing).  At
// most `inner_sweeps` sweeps; the outer sweeps finish what a capped inner
// solve leaves.
__global__ __launch_bounds__(EIG_THREADS, 4) void k_eig(const GateDesc *descs, int round, int ksplit) {
  const GateDesc &d = descs[blockIdx.y];
  const int pairIdx = blockIdx.x;
  if (!d.sc->active || round >= d.nblk - 1 || pairIdx >= d.nblk / 2) return;
  int I, J;
  rr_pair(round, pairIdx, d.nblk, I, J);
  if (pair_known_orthogonal(d, I, J)) {
    if (threadIdx.x == 0) d.pairFlag[pairIdx] = 0;
    return;
  }
  __shared__ double2 Gs[PW * LDG];
  __shared__ double dg[PW];           // diagonal of G
  __shared__ double rc[2][PW / 2];    // cos
  __shared__ double2 rse[2][PW / 2];  // s * e^{i phi}
  __shared__ int anyr[2];  // some rotation in the round held by that buffer
  __shared__ int sweep_rot, first_rot;
  const int tid = threadIdx.x;
  const double tol2 = d.tol * d.tol;
  const double small = small_norm2(d);
  unsigned nrot_local = 0;  // rotations applied by this thread (profiling)

  for (int e = tid; e < PW * PW; e += EIG_THREADS) {
    const int r = e / PW, c = e % PW;
    // upper entries lie in the upper 16x16 tiles that the Gram kernels store
    if (r <= c) {
      double2 sm = make_double2(0.0, 0.0);
      for (int kc = 0; kc < ksplit; kc++) {
        const double2 v = d.Gp[((size_t)kc * d.gpStride + pairIdx) * (PW * PW) + e];
        sm.x += v.x;
        sm.y += v.y;
      }
      if (r < c)
        Gs[r * LDG + c] = sm;
      else
        dg[r] = sm.x;
    }
  }
  const int lane = tid & 63, vrow0 = (tid >> 6) * EIG_VROWS;
  double2 vr[EIG_VROWS];  // V[vrow0 + h][lane]
#pragma unroll
  for (int h = 0; h < EIG_VROWS; h++) vr[h] = make_double2(vrow0 + h == lane ? 1.0 : 0.0, 0.0);
  if (tid == 0) first_rot = 0;
  __syncthreads();

  // Rotations of round r into buffer b, from the current G (first wavefront
  // only: lanes < 32 hold one pair each, the ballot gives the round's flag).
  // With delta = b - a and h = |g|^2 for the pair's 2x2 block [[a, g],
  // [conj g, b]], the rotation that zeroes g has tangent t = w |g|,
  // w = 2 sign(delta) / (|delta| + sqrt(delta^2 + 4h)), cosine
  // c = 1 / sqrt(1 + w^2 h), s e^{i phi} = c w g, and the new diagonal is
  // (a - w h, b + w h).  The pair's own block is set to those values here:
  // no other thread reads or writes it until the round is applied.
  auto params = [&](int r, int b) {
    int act = 0;
    if (tid < PW / 2) {
      int p, q;
      eig_pair(r, tid, p, q);
      const double a = dg[p], bb = dg[q];
      const int gs = gslot(p, q);
      const double2 g = p < q ? Gs[gs] : cconj(Gs[gs]);
      const double h = cabs2(g);
      double c = 1.0;
      double2 se = make_double2(0.0, 0.0);
      if (a > small && bb > small && h > tol2 * a * bb) {
        act = 1;
        const double delta = bb - a;
        const double w = (delta >= 0.0 ? 2.0 : -2.0) / (fabs(delta) + sqrt(delta * delta + 4.0 * h));
        c = 1.0 / sqrt(1.0 + w * w * h);
        const double cw = c * w;
        se = make_double2(cw * g.x, cw * g.y);
        dg[p] = a - w * h;
        dg[q] = bb + w * h;
        Gs[gs] = make_double2(0.0, 0.0);
        nrot_local++;
      }
      rc[b][tid] = c;
      rse[b][tid] = se;
    }
    const unsigned long long m = __ballot(act);
    if (tid == 0) anyr[b] = m != 0ull;
  };

  // this thread's off-diagonal block: the upper triangle of 32 x 32 pair
  // indices folded into 16 rows of 31 (row a with row 31 - a)
  int bi = 0, bj = 0;
  if (tid < EIG_OFFD) {
    const int a = tid / (PW / 2 - 1), col = tid - (PW / 2 - 1) * a;
    if (col < PW / 2 - 1 - a) {
      bi = a;
      bj = a + 1 + col;
    } else {
      bi = PW / 2 - 1 - a;
      bj = col + 1;
    }
  }

  for (int sweep = 0; sweep < d.innerSweeps; sweep++) {
    if (tid == 0) sweep_rot = 0;
    if (tid < 64) params(0, 0);
    __syncthreads();
    for (int r = 0; r < PW - 1; r++) {
      const int b = r & 1;
      const bool any = anyr[b] != 0;
      if (any && tid < EIG_OFFD) {
        // R = [[c, s e^{i phi}], [-s e^{-i phi}, c]] on columns (p, q);
        // block (row pair i, column pair j): B <- R_i^H B R_j.  A pair that
        // does not rotate has c = 1, s = 0, which leaves its entries exactly
        // as they are, so every block is updated without branches.
        int pi, qi, pj, qj;
        eig_pair(r, bi, pi, qi);
        eig_pair(r, bj, pj, qj);
        const int s00 = gslot(pi, pj), s01 = gslot(pi, qj), s10 = gslot(qi, pj), s11 = gslot(qi, qj);
        double2 b00 = Gs[s00], b01 = Gs[s01], b10 = Gs[s10], b11 = Gs[s11];
        if (pi > pj) b00 = cconj(b00);
        if (pi > qj) b01 = cconj(b01);
        if (qi > pj) b10 = cconj(b10);
        if (qi > qj) b11 = cconj(b11);
        {  // columns: [x_p x_q] R_j
          const double cj = rc[b][bj];
          const double2 sej = rse[b][bj], secj = cconj(sej);
          const double2 n00 = csub(cscale(b00, cj), cmul(secj, b01));
          const double2 n01 = cadd(cmul(sej, b00), cscale(b01, cj));
          const double2 n10 = csub(cscale(b10, cj), cmul(secj, b11));
          const double2 n11 = cadd(cmul(sej, b10), cscale(b11, cj));
          b00 = n00; b01 = n01; b10 = n10; b11 = n11;
        }
        {  // rows: R_i^H [row_p; row_q]
          const double ci = rc[b][bi];
          const double2 sei = rse[b][bi], seci = cconj(sei);
          const double2 n00 = csub(cscale(b00, ci), cmul(sei, b10));
          const double2 n01 = csub(cscale(b01, ci), cmul(sei, b11));
          const double2 n10 = cadd(cmul(seci, b00), cscale(b10, ci));
          const double2 n11 = cadd(cmul(seci, b01), cscale(b11, ci));
          b00 = n00; b01 = n01; b10 = n10; b11 = n11;
        }
        Gs[s00] = pi < pj ? b00 : cconj(b00);
        Gs[s01] = pi < qj ? b01 : cconj(b01);
        Gs[s10] = qi < pj ? b10 : cconj(b10);
        Gs[s11] = qi < qj ? b11 : cconj(b11);
      }
      // G after round r (a round without rotations leaves G as it was, and
      // the next rotations go to the other buffer)
      if (any) __syncthreads();
      if (tid < 64 && r + 1 < PW - 1) params(r + 1, b ^ 1);
      if (any) {
        // V <- V R on this lane's column j: the pair (p, q) holding j (slot
        // k of the order above), new x_p = c x_p - conj(se) x_q, new x_q =
        // se x_p + c x_q, the partner's entries by permute
        constexpr int H = PW / 2;
        int k, partner;
        bool isp;
        if (r < H) {
          isp = lane < H;
          k = isp ? lane : ((lane - H - r) & (H - 1));
          partner = isp ? H + ((lane + r) & (H - 1)) : k;
        } else {
          const int rr = r - H, off = lane & H, jj = lane & (H - 1);
          int d = jj - rr;
          d += d < 0 ? H - 1 : 0;
          int pt = 2 * rr - jj;
          pt += pt < 0 ? H - 1 : (pt >= H - 1 ? 1 - H : 0);
          const bool last = jj == H - 1, atr = jj == rr;
          isp = last ? true : (atr ? false : d <= H / 2 - 1);
          k = (last || atr) ? 0 : (d <= H / 2 - 1 ? d : H - 1 - d);
          pt = last ? rr : (atr ? H - 1 : pt);
          k += off >> 1;
          partner = pt + off;
        }
        const double c = rc[b][k];
        const double2 se = rse[b][k];
        const double2 kap = isp ? make_double2(-se.x, se.y) : se;
#pragma unroll
        for (int h = 0; h < EIG_VROWS; h++) {
          const double2 x = vr[h];
          const double2 y = make_double2(__shfl(x.x, partner, 64), __shfl(x.y, partner, 64));
          vr[h] = cadd(cscale(x, c), cmul(kap, y));
        }
        if (tid == 0) sweep_rot = 1;
      }
      __syncthreads();  // V after round r; rotations of round r + 1 ready
    }
    const int cont = sweep_rot;  // every thread reads before anyone clears it
    if (sweep == 0 && tid == 0) first_rot = cont;
    __syncthreads();
    if (!cont) break;
  }
  if (d.ctr && tid < 64) {
    // fold the per-thread counts of the first wavefront, one atomic per pair
    unsigned v = nrot_local;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (tid == 0 && v) atomicAdd(&d.ctr[CTR_EIG_ROT], (unsigned long long)v);
  }
  // An unrotated first sweep means the pair was already orthogonal.
  if (tid == 0) {
    d.pairFlag[pairIdx] = first_rot;
    if (first_rot) atomicOr(&d.sc->rot, 1);
    if (d.blkVer) {  // only this workgroup touches blocks I and J during the round
      if (first_rot) {
        d.blkVer[I] += 1;
        d.blkVer[J] += 1;
      } else {
        d.pairSeen[I * d.nblk + J] = make_int2(d.blkVer[I], d.blkVer[J]);
      }
    }
  }
  if (first_rot) {
    double2 *V = d.V + (size_t)pairIdx * (PW * PW);
#pragma unroll
    for (int h = 0; h < EIG_VROWS; h++) V[(vrow0 + h) * PW + lane] = vr[h];
  }
}

// ---------------------------------------------------------------- apply a pair rotation

// Pair rotation on float64 matrix cores, as the transposed product (X V)^T = V^T X^T, so that
// the X operand of v_mfma_f64_16x16x4 (B: 16 lanes = 16 consecutive rows of
// one column) and the result (16 lanes = 16 consecutive rows of one column)
// are both contiguous 256-byte segments.  A wavefront owns whole 16-row tiles
// (all 64 columns), so it overwrites exactly the rows it read and needs no
// barrier; two workgroups per CU hide the load latency.  Each complex product
// takes three real products (Gauss): with v = a + ib and x = c + id,
// P1 = a c, P2 = b d, P3 = (a + b)(c + d), v x = (P1 - P2) + i (P3 - P1 - P2).
__global__ __launch_bounds__(256, 2) void k_rot_mfma3(const GateDesc *descs, int round) {
  const GateDesc &d = descs[blockIdx.y];
  if (!d.sc->active || round >= d.nblk - 1) return;
  const int npairs = d.nblk / 2;
  const int RRW = d.rotRows;
  const int xchunks = (d.rows + RRW - 1) / RRW;
  const int jchunks = d.trans ? (d.m + RRW - 1) / RRW : 0;
  const int per = xchunks + jchunks;
  const int pairIdx = blockIdx.x / per, chunk = blockIdx.x % per;
  if (pairIdx >= npairs) return;
  if (!d.pairFlag[pairIdx]) return;
  int I, J;
  rr_pair(round, pairIdx, d.nblk, I, J);
  double2 *base;
  int ld, nrows, r0;
  if (chunk < xchunks) {
    base = d.X;
    ld = d.ldx;
    nrows = d.rows;
    r0 = chunk * RRW;
  } else {
    base = d.J;
    ld = d.ldj;
    nrows = d.m;
    r0 = (chunk - xchunks) * RRW;
  }
  const int r1 = min(nrows, r0 + RRW);
  __shared__ double2 Vs[PW * LDG];  // [k][col]
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform (scalar)
  const int l16 = lane & 15, lg = lane >> 4;
  const double2 *V = d.V + (size_t)pairIdx * (PW * PW);
  for (int e = tid; e < PW * PW; e += 256) Vs[(e / PW) * LDG + e % PW] = V[e];
  if (tid == 0 && d.ctr) {
    unsigned long long nr = (unsigned long long)(r1 - r0);
    atomicAdd(&d.ctr[CTR_ROT_FLOP], 8ull * nr * PW * PW);
    atomicAdd(&d.ctr[CTR_ROT_BYTE], 32ull * nr * PW + 16ull * PW * PW);
  }
  __syncthreads();
  // The lane's column for k-step s is pair column 4 s + lg (block I for
  // s < 8).  Buffer loads and stores (one resource per block of 32 padded columns, a
  // 32-bit element offset per access): one register per address, counted
  // on the vector memory counter only.  Tile q of the wavefront covers rows
  // r0 + 16 (wave + 4 q) ..; a tile past the chunk uses an empty resource
  // (loads read zero, stores are dropped), so every wavefront runs an even
  // number of tiles with no branch around loads or stores, and the loads in
  // flight are counted exactly: the products of a tile wait only for that
  // tile's data while the next tile's block I is still on its way.  Columns
  // are padded to whole 16-row tiles and chunks are whole tiles, so rows
  // past the matrix land in the column's padding (never read).
  const BufRes rI = make_res(base + (size_t)I * BW * ld, BW * ld);
  const BufRes rJ = make_res(base + (size_t)J * BW * ld, BW * ld);
  const BufRes rZ = make_res(base, 0);
  const int ntile = (r1 - r0 + 15) / 16;
  const int mytiles = wave < ntile ? (ntile - wave + 3) / 4 : 0;
  auto tile_row = [&](int q) { return r0 + 16 * (wave + 4 * q); };
  // k-steps 0..7 read block I, 8..15 block J
  auto load_half = [&](double2 *xv, int half, int q) {
    const int rt = tile_row(q);
    const BufRes r = rt < r1 ? (half ? rJ : rI) : rZ;
    const int lo = lg * ld + rt + l16;
#pragma unroll
    for (int s = 0; s < BW / 4; s++) xv[s] = bload(r, lo + 4 * s * ld);
  };
  // one 16-row tile: block I from xi, block J from xj
  auto tile = [&](const double2 *xi, const double2 *xj, int q) {
    d4_t p1[4], p2[4], p3[4];
#pragma unroll
    for (int t = 0; t < 4; t++) {
      p1[t] = d4_t{0.0, 0.0, 0.0, 0.0};
      p2[t] = d4_t{0.0, 0.0, 0.0, 0.0};
      p3[t] = d4_t{0.0, 0.0, 0.0, 0.0};
    }
#pragma unroll
    for (int s = 0; s < PW / 4; s++) {
      const double2 b = s < BW / 4 ? xi[s] : xj[s - BW / 4];  // X^T[k][row]
      const double bs = b.x + b.y;
#pragma unroll
      for (int t = 0; t < 4; t++) {
        const double2 a = Vs[(4 * s + lg) * LDG + t * 16 + l16];  // V^T[col][k]
        p1[t] = mfma64(a.x, b.x, p1[t]);
        p2[t] = mfma64(a.y, b.y, p2[t]);
        p3[t] = mfma64(a.x + a.y, bs, p3[t]);
      }
      __builtin_amdgcn_sched_barrier(0);  // keep each step's V reads in that step
    }
    // Loads and stores share the vector memory counter, and a load issued
    // before a store can only be waited for with the store: so the next
    // tile's block I (issued at this tile's start, long arrived) is waited
    // for here, before this tile's stores.
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    // output column t * 16 + lg + 4 v of the pair: block I for t < 2
    const int rt = tile_row(q);
    const bool live = rt < r1;
    const BufRes oI = live ? rI : rZ, oJ = live ? rJ : rZ;
    const int lo = lg * ld + rt + l16;
#pragma unroll
    for (int t = 0; t < 4; t++)
#pragma unroll
      for (int v = 0; v < 4; v++)
        bstore(t < 2 ? oI : oJ, lo + (16 * (t & 1) + 4 * v) * ld,
               make_double2(p1[t][v] - p2[t][v], p3[t][v] - p1[t][v] - p2[t][v]));
  };
  // Two block-I buffers take turns (no register copies between tiles).
  double2 xi0[BW / 4], xi1[BW / 4], xj[BW / 4];
  load_half(xi0, 0, 0);
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): the loop starts with block I in hand
  for (int q = 0; q < mytiles; q += 2) {
    load_half(xj, 1, q);
    load_half(xi1, 0, q + 1);
    tile(xi0, xj, q);
    load_half(xj, 1, q + 1);
    load_half(xi0, 0, q + 2);
    tile(xi1, xj, q + 1);
  }
}

void launch_gram(hipStream_t st, const GateDesc *d, int ng, int round, int max_pairs,
                 int ksplit) {
  if (ng <= 0) return;
  hipLaunchKernelGGL(k_gram_mfma2, dim3(max_pairs * ksplit, ng), dim3(256), 0, st, d, round,
                     ksplit);
}

void launch_eig(hipStream_t st, const GateDesc *d, int ng, int round, int max_pairs, int ksplit) {
  if (ng <= 0) return;
  hipLaunchKernelGGL(k_eig, dim3(max_pairs, ng), dim3(EIG_THREADS), 0, st, d, round, ksplit);
}

// Copy every gate's scalars into one array (one device-to-host copy per sweep).
__global__ void k_gather_sc(const GateDesc *descs, int ng, SlotScalars *out) {
  int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g < ng) out[g] = *descs[g].sc;
}

void launch_gather_sc(hipStream_t st, const GateDesc *d, int ng, SlotScalars *out) {
  if (ng <= 0) return;
  hipLaunchKernelGGL(k_gather_sc, dim3((ng + 63) / 64), dim3(64), 0, st, d, ng, out);
}

void launch_rot(hipStream_t st, const GateDesc *d, int ng, int round, int max_pairs,
                int max_rows, int max_m, int rot_rows) {
  if (ng <= 0) return;
  const int per = (max_rows + rot_rows - 1) / rot_rows + (max_m + rot_rows - 1) / rot_rows;
  hipLaunchKernelGGL(k_rot_mfma3, dim3(max_pairs * per, ng), dim3(256), 0, st, d, round);
}

// ---------------------------------------------------------------- sort + truncate

constexpr int SORT_MAX = 4096;

__global__ __launch_bounds__(256) void k_trunc(const GateDesc *descs) {
  const GateDesc &d = descs[blockIdx.x];
  __shared__ double key[SORT_MAX];
  __shared__ int idx[SORT_MAX];
  __shared__ double tail[SORT_MAX + 1];
  __shared__ int s_k;
  __shared__ double s_N;
  const int tid = threadIdx.x;
  int P = 1;
  while (P < d.cols) P <<= 1;
  for (int j = tid; j < P; j += 256) {
    key[j] = j < d.cols ? d.sig2[j] : -1.0;
    idx[j] = j;
  }
  __syncthreads();
  // bitonic sort: descending key, ascending index on ties
  for (int size = 2; size <= P; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int j = tid; j < P; j += 256) {
        int l = j ^ stride;
        if (l > j) {
          bool up = ((j & size) == 0);  // this block sorted "descending-first"
          double kj = key[j], kl = key[l];
          int ij = idx[j], il = idx[l];
          bool j_first = (kj > kl) || (kj == kl && ij < il);
          bool swap = up ? !j_first : j_first;
          if (swap) {
            key[j] = kl;
            key[l] = kj;
            idx[j] = il;
            idx[l] = ij;
          }
        }
      }
      __syncthreads();
    }
  }
  if (tid == 0) {
    const int cnt = d.cols;
    double W = 0.0;
    for (int j = 0; j < cnt; j++) W += key[j];
    double floor2 = (double)d.m * 0x1p-53 * key[0];
    int nz = 0;
    for (int j = 0; j < cnt; j++) nz += key[j] > floor2;
    if (nz < 1) nz = 1;
    tail[cnt] = 0.0;
    for (int k = cnt - 1; k >= 0; k--) tail[k] = tail[k + 1] + key[k];
    const double cutoff = d.cutoff;
    int kc = cnt;
    for (int k = 1; k <= cnt; k++)
      if (tail[k] <= cutoff * W) {
        kc = k;
        break;
      }
    int k = kc;
    if (k > nz) k = nz;
    if (k > d.chiMax) k = d.chiMax;
    if (k < 1) k = 1;
    double head = 0.0;
    for (int j = 0; j < k; j++) head += key[j];
    double N = sqrt(head);
    if (!(N > 0.0)) N = 1.0;
    d.sc->k = k;
    d.sc->N = N;
    d.sc->W = W;
    d.sc->eps = W > 0.0 ? tail[k] / W : 0.0;
    d.sc->nz = nz;
    d.dimsDev[d.i + 1] = k;
    s_k = k;
    s_N = N;
  }
  __syncthreads();
  for (int j = tid; j < s_k; j += 256) {
    d.lamOut[j] = sqrt(key[j]) / s_N;
    d.perm[j] = idx[j];
  }
}

void launch_trunc(hipStream_t st, const GateDesc *d, int ng) {
  if (ng <= 0) return;
  hipLaunchKernelGGL(k_trunc, dim3(ng), dim3(256), 0, st, d);
}

}  // namespace tn
