// Internal types shared by the library's HIP sources (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace tn {

// Jacobi block width: the SVD rotates pairs of 32-column blocks, so one pair
// problem is a 64x64 Hermitian Gram matrix that fits in one workgroup's LDS.
constexpr int BW = 32;
constexpr int PW = 64;
constexpr int KSPLIT_MAX = 16;
constexpr int GP_PER_SLOT = 4;  // K-split chunks of partial pair Grams held per workspace slot
// QR preconditioning: Householder panels of QNB columns; a panel of up to
// QR_MAX_ROWS rows is held in the registers of one 512-thread workgroup
// (4 rows x 8 complex128 columns per thread).
constexpr int QNB = 8;
constexpr int QG = 32;  // reflectors applied together to the rest of the matrix (4 panels)
constexpr int QR_RC = 256;  // rows per workgroup in a group update
constexpr int QR_MAX_ROWS = 2048;

// Scalars per gate slot (device memory).
struct SlotScalars {
  double fro2;  // squared Frobenius norm of the Jacobi matrix
  double N;     // sqrt of the kept weight
  double eps;   // discarded weight / total weight
  double W;     // total weight
  int k;        // kept bond dimension
  int rot;      // some pair rotated during the current sweep
  int active;   // gate still sweeping
  int nz;       // count above the numerical-zero floor
};

// Device descriptor of one two-qubit gate in a batch.  The host fills it from
// its copy of the bond dimensions; kernels never read dimensions elsewhere.
struct GateDesc {
  int i;                 // left site
  int chiL, chiM, chiR;  // bond dims around sites i, i+1
  int m, n;              // M is m x n: m = 2 chiL rows (a,s), n = 2 chiR cols (t,c)
  int rows, cols;        // Jacobi matrix X: rows x cols, cols = min(m, n)
  int trans;             // 1: X = M^H (n > m) and J accumulates U; 0: X = M
  int ldx, ldj;          // leading dims of X and J (column-major)
  int colsPad;           // cols rounded up to a multiple of 64
  int nblk;              // colsPad / 32
  int chiMax;
  int storage;           // 0 = complex128 sites, 1 = complex64 sites
  int tfp32;             // theta' stored as complex64 (mixed modes)
  int innerSweeps;       // sweep cap of the 64x64 pair solve
  int gpStride;          // pair blocks per K-split chunk in Gp
  int rotRows;           // rows of X (and J) per rotation workgroup, a multiple of 64
  int *dimsDev;          // device bond dimensions of the gate's state (n+1)
  double tol;            // relative off-diagonal tolerance
  double cutoff;         // discarded-weight cutoff
  void *A0, *A1;         // site i, site i+1 (read by the merge)
  void *A0out, *A1out;   // where the write-back puts them (the same sites, except
                         // for the window steps of bond propagation)
  const double *lamR;    // lambda_{i+1} or nullptr (= all ones)
  double *lamOut;        // lambda_i
  double2 *X, *J;        // Jacobi matrix, accumulated left vectors (trans only)
  void *T;               // theta' (m x n, row-major)
  double2 *Gp, *V;       // pair Gram partials, pair rotations
  int *pairFlag;         // pair rotated in this round
  int *blkVer;           // per column block: number of rotations applied to it so far
  int2 *pairSeen;        // per block pair (I * nblk + J): block versions when the pair
                         // last tested orthogonal, or (-1, -1)
  double *sig2;          // column norms squared
  int *perm;             // columns sorted by descending norm
  SlotScalars *sc;
  // QR preconditioning (qr = 1): theta writes M (m x n) to Qm, which then
  // holds Q1's reflectors below R1; X is R2^H (n x n); U gets U_k = Q1 [W_k; 0]
  // (m x k) for the write-back; Tq holds the compact-WY factor of every panel.
  int qr, ldq, ldu, pad2;
  double2 *Qm, *U, *Tq;
  unsigned long long *ctr;  // work counters (see CTR_*), may be nullptr
  double2 g[16];            // the 4x4 gate
};

// Device work counters, accumulated by the Jacobi kernels (one atomic per
// workgroup): algorithmic flops and bytes of what each launch really did.
enum { CTR_GRAM_FLOP = 0, CTR_GRAM_BYTE, CTR_EIG_ROT, CTR_ROT_FLOP, CTR_ROT_BYTE, CTR_COUNT };

struct Gate1Desc {
  void *A;
  int chiL, chiR;
  int storage, pad;
  double2 u[4];
};

// Launch wrappers (each enqueues on `st`; errors are collected by the caller
// through hipGetLastError / hipPeekAtLastError).
void launch_init_state(hipStream_t st, void *const *sites_dev_list, int n, int storage,
                       double *const *lam_list_dev, int nb);
void launch_fill_zero(hipStream_t st, void *p, size_t bytes);
// float64 rate probe: unit 0 = matrix cores (16x16x4), 1 = vector FMA, 2 = both at
// once, 3 = matrix cores (four-block 4x4x4); returns the flops launched
double launch_probe(hipStream_t st, int unit, int groups, int iters, double *out);
void launch_apply_1q(hipStream_t st, const Gate1Desc *d, int ng, int max_elems);
void launch_convert(hipStream_t st, const void *src, int src_storage, void *dst, int dst_storage,
                    size_t count);
// rg 2x2 factors of a gate's operator Schmidt decomposition (bond propagation)
struct Mat4x4 {
  double2 v[4][4];
};
void launch_prop_merge(hipStream_t st, const double2 *old, void *out, int storage, int chiL,
                       int chiR, int rg, int role, const Mat4x4 &F);
void launch_setup_slots(hipStream_t st, const GateDesc *d, int ng, int max_rows_pad,
                        int max_m_pad);
void launch_theta(hipStream_t st, const GateDesc *d, int ng, int precision, int max_m,
                  int max_chiR);
void launch_colnorm(hipStream_t st, const GateDesc *d, int ng, int max_cols);
void launch_gate_init(hipStream_t st, const GateDesc *d, int ng);
void launch_begin_sweep(hipStream_t st, const GateDesc *d, int ng);
void launch_gram(hipStream_t st, const GateDesc *d, int ng, int round, int max_pairs,
                 int ksplit);
void launch_eig(hipStream_t st, const GateDesc *d, int ng, int round, int max_pairs, int ksplit);
void launch_gather_sc(hipStream_t st, const GateDesc *d, int ng, SlotScalars *out);
void launch_rot(hipStream_t st, const GateDesc *d, int ng, int round, int max_pairs,
                int max_rows, int max_m, int rot_rows);
void launch_trunc(hipStream_t st, const GateDesc *d, int ng);
// QR preconditioning (k_qr.hip).  stage 0 factors M (in Qm), stage 1 factors
// R1^H (in X).  Panels of QNB columns are factored and applied inside their
// group of QG columns; a group's reflectors then update the rest at once
// (apply = 1: multiply U by Q1 instead).
void launch_qr_panel(hipStream_t st, const GateDesc *d, int ng, int stage, int panel);
void launch_qr_update(hipStream_t st, const GateDesc *d, int ng, int stage, int panel,
                      int col_end, int max_cols);
void launch_qr_tgroup(hipStream_t st, const GateDesc *d, int ng, int stage, int group);
void launch_qr_update_group(hipStream_t st, const GateDesc *d, int ng, int stage, int group,
                            int apply, int max_cols, int max_rows);
void launch_qr_r1h(hipStream_t st, const GateDesc *d, int ng, int max_n);
void launch_qr_r2h(hipStream_t st, const GateDesc *d, int ng, int max_n);
void launch_qr_gather(hipStream_t st, const GateDesc *d, int ng, int max_m, int max_k);
void launch_wb_left(hipStream_t st, const GateDesc *d, int ng, int max_m, int max_k);
void launch_wb_right(hipStream_t st, const GateDesc *d, int ng, int precision, int max_k,
                     int max_n);

// Adjoint sweep (k_adjoint.hip)
struct Mat4 {
  double2 v[4];
};
struct Mat16 {
  double2 v[16];
};
struct GemmArgs {
  int M, N, K;
  const void *A;
  long long sa_i, sa_k;
  int a_conj, a_storage;
  const void *B;
  long long sb_k, sb_j;
  int b_conj, b_storage;
  double2 *C;
  long long sc_i, sc_j;
  double2 alpha;
  int accumulate;
};
void launch_gemm_gen(hipStream_t st, const GemmArgs &g);
void launch_fill_c(hipStream_t st, double2 *p, size_t n, double2 v);
void launch_svd_adj_mid(hipStream_t st, const double2 *C, double2 *Abar, const double *lam2,
                        const double *sbar, int m, int k, double eta);
void launch_herm_sum(hipStream_t st, const double2 *H, double2 *S, int m);
void launch_weight_adj(hipStream_t st, const double2 *Mbar, const double2 *Tp, double2 *Tbar,
                       const double *lam, double *lambar, int m, int chiR);
void launch_weight_apply(hipStream_t st, const double2 *Tp, double2 *M, const double *lam, int m,
                         int chiR);
void launch_gate_adj(hipStream_t st, double2 *T, int chiL, int chiR, const Mat16 &g);
void launch_1q_adj(hipStream_t st, double2 *Abar, const void *Aold, int storage, int chiL,
                   int chiR, const Mat4 &u, double *ubar);
void launch_dot_re(hipStream_t st, const double2 *x, const void *y, int y_storage, size_t n,
                   double *out);
void launch_sigma_bar(hipStream_t st, const double *dots, const double *lambark,
                      const double *lam2, double N, int k, double *sbar);
void launch_gather_basis(hipStream_t st, const double2 *J, int ldj, const int *perm,
                         const double *sig2, double2 *U, double *lam2, int m);
void launch_sort_all(hipStream_t st, const double *sig2, int cols, int *perm);
void launch_angle_grad(hipStream_t st, const double *ubar, const Mat4 &u, int axis,
                       double *grad);

// Readouts
void launch_pauli_phys(hipStream_t st, const double2 *F, double2 *F2, int chiA, int chiB,
                       double2 p00, double2 p01, double2 p10, double2 p11);
// complex float64 GEMM on the matrix cores (k_zgemm.hip): C (M x N) = op(A) B
// with op(A) M x K.  N is capped at mult * *mcount when mcount is not null
// (a count that earlier kernels left on the device; the grid covers N).
struct ZgemmArgs {
  int M, N, K;
  const void *A;
  long long sa;
  const void *B;
  long long sb;
  double2 *C;
  long long sc;
  const int *mcount;
  int mult;
  int batch = 1;              // independent products, operands offset by z * (za, zb, zc)
  long long za = 0, zb = 0, zc = 0;
  int ksplit = 1;             // K split over workgroups (batch 1 only); the partial products
  double2 *part = nullptr;    // go to part (ksplit x M x N) and are added in order into C
  int kchunk = 0;             // K per split (set by the launcher)
  // ZGEMM_NN_COL_GATHER only: output columns [*clo, *chi) (device values, at
  // most N of them); column j reads column bmap[j] of B, scaled by cscale[j];
  // tiles of 64 columns from *asplit on (a multiple of 64) use A + za
  const int *clo = nullptr, *chi = nullptr, *bmap = nullptr, *asplit = nullptr;
  const double *cscale = nullptr;
};
// ksplit that gives a product of this shape about 1024 workgroups (1 if none
// needed); ksplit * M * N never exceeds ZGEMM_PART_ELEMS when it is above 1
int zgemm_ksplit(int M, int N, int K);
constexpr size_t ZGEMM_PART_ELEMS = (size_t)1024 * 64 * 64;
enum ZgemmKind {
  ZGEMM_NN_ROW,  // A(i,k) = A[i*sa + k]; B(k,j) = B[k*sb + j]; C(i,j) = C[i*sc + j]
  ZGEMM_CN_ROW,  // op(A)(i,k) = conj(A[k*sa + i]); B, C as above
  ZGEMM_NN_COL,  // A(i,k) = A[i*sa + k]; B(k,j) = B[j*sb + k]; C(i,j) = C[j*sc + i]
  ZGEMM_NN_COL_GATHER,  // as NN_COL on gathered, scaled columns (see ZgemmArgs)
};
void launch_zgemm(hipStream_t st, ZgemmKind kind, const ZgemmArgs &g, int a_storage,
                  int b_storage);

// perfect sampling (k_sample.hip)
void launch_smp_init(hipStream_t st, int shots, int node_cap, int *node, double *logp, int *flag,
                     double2 *V, double2 *E0, int *ctr);
void launch_smp_prob(hipStream_t st, const double2 *V, const double2 *Y, int M, int bound,
                     const int *ctr, double *p);
void launch_smp_decide(hipStream_t st, int shots, int n, int q, const double *u, const double *p,
                       const int *node, int *key, int *flag, uint8_t *bits, double *logp,
                       int *ctr);
void launch_smp_scan(hipStream_t st, const int *flag, int *idx, int *ctr);
void launch_smp_parent(hipStream_t st, int *flag, const int *idx, const double *p, const int *ctr,
                       int bound, int *parent, double *scale);
void launch_smp_relabel(hipStream_t st, int shots, const int *key, const int *idx, int *node);
void launch_smp_add(hipStream_t st, const double2 *M01, size_t n, double2 *E);
void launch_amp_step(hipStream_t st, const double2 *v, double2 *w, double2 *part, const void *A,
                     int storage, int chiL, int chiR, int bit);

}  // namespace tn
