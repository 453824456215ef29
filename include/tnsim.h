/*
 * tnsim.h -- C ABI of the MI355X (gfx950) MPS gate-application library.
 *
 * The library applies quantum gates to a Matrix Product State (arXiv
 * 2601.04422, Sec. II eq. 2 for the state, Sec. III.A for the gate
 * algorithms, Sec. IV.A for the merge of two sites and the truncated SVD).
 *
 * Conventions
 *   - Site q holds A_q[a,s,b] of shape (chi_{q-1}, 2, chi_q), row-major;
 *     bond q joins sites q and q+1 and has dimension chi_q; the outer bonds
 *     have dimension 1.  The state starts as |0...0> with every bond of
 *     dimension 1 (Sec. IV.A).
 *   - Gauge: every site is left-canonical and each bond carries its Schmidt
 *     weights lambda_q (float64).  A two-qubit gate on (i, i+1) decomposes
 *     theta' * diag(lambda_{i+1}) and writes A_i' = U_k (left singular
 *     vectors on the left/control site), lambda_i' = sigma/N and
 *     A_{i+1}' = U_k^H theta' / N (singular values folded into the right
 *     site, Sec. III.A), N = sqrt(sum of kept sigma^2).
 *   - Truncation: k is the smallest k >= 1 whose discarded weight
 *     sum_{j>k} sigma_j^2 <= cutoff * sum_j sigma_j^2, capped by chi_max and
 *     by the count of sigma_j^2 > 2*chi_L * 2^-53 * sigma_1^2.
 *   - Gate matrices are complex128.  A 4x4 gate is row-major in the basis
 *     |s_q0 s_q1> with row 2*s_q0 + s_q1.  (q0, q0+1) and (q0, q0-1) are both
 *     accepted; the second applies SWAP*G*SWAP on (q0-1, q0).
 *
 * Memory and streams
 *   - The caller allocates one device buffer of tnsim_mps_arena_bytes(cfg)
 *     bytes (any device allocator; 256-byte alignment) and passes it with a
 *     hipStream_t to tnsim_mps_create.  Buffer and stream must outlive the
 *     handle; the handle owns host metadata and a small pinned staging
 *     buffer, plus, once tnsim_apply_circuit (or a distant tnsim_apply_2q)
 *     has run, a second stream with its own staging buffer on which the
 *     scheduler prepares gates; tnsim_mps_destroy frees them.
 *   - Host arrays passed in (gates, bits, Pauli strings) are copied before the
 *     call returns.  Output pointers are host memory, except the sampling
 *     buffers (device memory, see tnsim_sample).
 *   - A handle is not thread-safe: calls on one handle must not overlap.
 *   - tnsim_apply_* enqueue on the handle's stream.  The Jacobi sweep loop
 *     synchronises the stream to test convergence, so they return after the
 *     gate work is done.  Readouts synchronise.
 *
 * Errors
 *   - Every argument is validated on the host before any device work; on an
 *     argument error the state is unchanged.
 *   - A failed HIP call poisons the handle: every later call returns
 *     TNSIM_E_DEVICE.  tnsim_last_error describes the first failure.
 *   - TNSIM_E_NOCONV: the Jacobi SVD of some gate did not converge within
 *     jacobi_max_sweeps; the two-qubit gates of that call are not written
 *     back (their sites keep the previous values) and the handle stays usable.
 */
#ifndef TNSIM_H
#define TNSIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tnsim_mps_s *tnsim_mps;

typedef struct {
  double re, im;
} tnsim_c128;

typedef enum {
  TNSIM_OK = 0,
  TNSIM_E_ARG = 1,      /* bad argument (qubit out of range, bad config, NULL) */
  TNSIM_E_NONLOCAL = 2, /* two-qubit gate on non-neighbouring qubits */
  TNSIM_E_OVERLAP = 3,  /* a layer uses a qubit twice */
  TNSIM_E_CAPACITY = 4, /* arena too small for the configuration */
  TNSIM_E_DEVICE = 5,   /* HIP runtime failure, or no device */
  TNSIM_E_NOCONV = 6    /* Jacobi sweeps exhausted */
} tnsim_status;

/* Arithmetic of the theta contraction and the right-site write-back.  The
   SVD (column Gram blocks, Jacobi rotations, norms, truncation) is float64 in
   every mode. */
typedef enum {
  TNSIM_FP64 = 0,   /* float64 everywhere */
  TNSIM_F32ACC = 1, /* float32 products, float32 accumulation (MFMA) */
  TNSIM_BF16X3 = 2, /* float32 operands split into bf16 pieces, 3 MFMA products */
  TNSIM_BF16X6 = 3  /* same with 6 products (about float32 accuracy) */
} tnsim_precision;

typedef enum {
  TNSIM_STORE_C128 = 0, /* site tensors complex128 */
  TNSIM_STORE_C64 = 1   /* site tensors complex64 (Schmidt weights stay float64) */
} tnsim_storage;

typedef struct {
  int32_t n_qubits;          /* >= 2 */
  int32_t chi_max;           /* 1 .. 2048 */
  double cutoff;             /* discarded-weight cutoff, >= 0 */
  int32_t precision;         /* tnsim_precision */
  int32_t storage;           /* tnsim_storage */
  int32_t jacobi_max_sweeps; /* <= 0 selects 60 */
  double jacobi_tol;         /* <= 0 selects max(rows, 16) * 2^-53 with complex128 sites,
                                2^-30 with complex64 sites (64 times below their rounding) */
  int32_t max_layer_gates;   /* two-qubit gates processed together; <= 0 selects n/2 */
  /* 0: one-sided Jacobi on M.  1: QR preconditioning before the Jacobi
     (Drmac and Veselic, SIAM J. Matrix Anal. Appl. 29(4), 2008): M = Q1 R1,
     R1^H = Q2 R2 by blocked Householder QR in float64, one-sided Jacobi on
     R2^H = W S V^H, left vectors U = Q1 W; it takes about half the Jacobi
     sweeps.  Used for gates with 2 chiR <= 2 chiL <= 2048 and no recorded
     adjoint; other gates take the plain path. */
  int32_t svd_precondition;
} tnsim_config;

typedef struct {
  int32_t q0, q1;     /* q1 = -1 marks a one-qubit gate */
  tnsim_c128 m[16];   /* 2x2 in m[0..3] (row-major) or 4x4 row-major; every entry point
                         that takes gate matrices rejects a non-finite entry (TNSIM_E_ARG) */
} tnsim_gate;

/* Bytes of device memory a handle with this configuration needs; 0 if the
   configuration is invalid. */
size_t tnsim_mps_arena_bytes(const tnsim_config *cfg);

/* Create a handle on the current HIP device, initialised to |0...0>
   (Sec. IV.A).  dev_arena: device pointer of arena_bytes bytes; hip_stream:
   a hipStream_t (NULL = default stream). */
tnsim_status tnsim_mps_create(const tnsim_config *cfg, void *dev_arena, size_t arena_bytes,
                              void *hip_stream, tnsim_mps *out);
tnsim_status tnsim_mps_destroy(tnsim_mps mps);

/* Reset to |0...0> and clear the truncation statistics. */
tnsim_status tnsim_mps_reset(tnsim_mps mps);

/* One-qubit gate A'[a,s',b] = sum_s U[s',s] A[a,s,b]  (Sec. II, eq. 3). */
tnsim_status tnsim_apply_1q(tnsim_mps mps, int32_t q, const tnsim_c128 u[4]);

/* Two-qubit gate on distant qubits by bond propagation (Sec. III.A, the
   method that scales linearly in the distance): G is split by SVD into
   sum_r X_r (x) Y_r (r <= 4 terms, singular values folded into Y_r); X_r
   goes into the site of the left qubit, whose bond gains the propagating
   index r, which is carried through every site in between, and Y_r into the
   site of the right qubit.  That chain holds G|psi> exactly; its sites are
   then decomposed in succession from left to right (no truncation) and its
   bonds get their Schmidt values from right to left, where chi_max and the
   cutoff apply (the gate's discarded weight is the sum over its cuts).
   Neighbouring qubits take the ordinary path of tnsim_apply_2q.  The bonds
   between the qubits must hold r times their current dimension while the
   gate runs: when one would exceed its capacity (the handle's
   min(chi_max, 2^min(b+1, n-1-b))), the call returns TNSIM_E_CAPACITY with
   the state unchanged (tnsim_apply_2q applies such a gate by SWAP gates).
   Errors: TNSIM_E_ARG (qubits out of range or equal, NULL or non-finite
   matrix), TNSIM_E_CAPACITY, TNSIM_E_NOCONV (the state then holds the
   gate's result in a gauge that is not canonical between the two qubits;
   tnsim_canonicalize restores it), TNSIM_E_DEVICE. */
tnsim_status tnsim_apply_2q_propagate(tnsim_mps mps, int32_t q0, int32_t q1,
                                      const tnsim_c128 g[16]);

/* Canonical form (Sec. IV.A: the state is canonicalised before sampling).
   Gate application keeps every site left-canonical and lambda_q equal to the
   Schmidt values of bond q, but only up to rounding, and after truncations
   (or tnsim_import_state of sites in another gauge) only approximately.  This
   call restores that form exactly from any gauge, with two sweeps of
   two-site decompositions: left to right without the Schmidt weights (every
   site becomes left-canonical), then right to left with the weights just
   computed (every bond gets the Schmidt values of the state).  The state is
   normalised.  truncate = 0: only numerically zero values are dropped;
   truncate = 1: the right-to-left sweep applies chi_max and cutoff (each
   cut's discarded weight goes to tnsim_truncation_stats; the gate count is
   not changed), followed by one more pass without truncation.  Cost: 2(n-1)
   (or 4(n-1)) two-site decompositions run one after the other.
   Errors: TNSIM_E_ARG (bad handle, truncate not 0 or 1), TNSIM_E_NOCONV
   (a Jacobi SVD ran out of sweeps; the sweep stops there and the state is
   the same state in a partly canonical gauge), TNSIM_E_DEVICE. */
tnsim_status tnsim_canonicalize(tnsim_mps mps, int32_t truncate);

/* Two-qubit gate, one gate per launch sequence: merge the two sites (Sec.
   IV.A, Fig. 2), contract with the gate, Jacobi SVD, truncate, write back
   (Sec. III.A).  Qubits further apart than neighbours are brought together
   by SWAP gates and moved back afterwards (Sec. IV.A): the qubit with the
   larger index is swapped down next to the other one, every SWAP being an
   ordinary truncated two-qubit gate. */
tnsim_status tnsim_apply_2q(tnsim_mps mps, int32_t q0, int32_t q1, const tnsim_c128 g[16]);

/* All gates of one layer of gates on disjoint qubits (Sec. IV.B): the
   one-qubit gates in one launch, then every two-qubit gate of the layer in
   the same launches (batched over gates).  Two-qubit gates must act on
   neighbouring qubits (TNSIM_E_NONLOCAL otherwise, state unchanged). */
tnsim_status tnsim_apply_layer(tnsim_mps mps, const tnsim_gate *gates, int32_t n_gates);

/* A whole circuit, in order (gates may share qubits; a gate given as
   (q, q-1) is applied as SWAP G SWAP on (q-1, q), and a gate on distant
   qubits through the SWAP chain of tnsim_apply_2q).  The result equals applying the gates one by one (Sec.
   III.A, gate application; Sec. IV.B, gates of a layer on disjoint qubits run
   in parallel): a gate starts once the gates before it on its qubits are
   done, and two-qubit gates in flight, from any layer, share the launches of
   every Jacobi sweep.  gates: host array of n_gates entries, read during the
   call only.  Errors: TNSIM_E_ARG (qubit out of range, q0 == q1, a
   non-finite matrix entry; validated before any work, state unchanged);
   TNSIM_E_NOCONV (a Jacobi ran out of sweeps: the gates completed by then
   stay applied, each one whole and in an order consistent with the circuit,
   the others are not; the MPS stays valid); TNSIM_E_DEVICE. */
tnsim_status tnsim_apply_circuit(tnsim_mps mps, const tnsim_gate *gates, int32_t n_gates);

/* Independent circuits: layer l of every handle, batched together.  All
   handles must share one stream and one configuration class (precision and
   storage); gates[i] has n_gates[i] entries for handle i. */
tnsim_status tnsim_apply_layer_multi(tnsim_mps const *mps, const tnsim_gate *const *gates,
                                     const int32_t *n_gates, int32_t n_mps);

/* Greedy layering (Sec. IV.B): each gate goes to the first layer after the
   last one that used any of its qubits.  layer_of_gate[g] receives the layer
   index, *n_layers the count.  Host-only. */
tnsim_status tnsim_layerise(const tnsim_gate *gates, int32_t n_gates, int32_t n_qubits,
                            int32_t *layer_of_gate, int32_t *n_layers);

/* <psi|P|psi> / <psi|psi> for a Pauli string P (n chars of I, X, Y, Z; char q
   acts on qubit q) by full left-to-right transfer contraction. im_out may be
   NULL. */
tnsim_status tnsim_expect_pauli(tnsim_mps mps, const char *pauli, double *re_out,
                                double *im_out);

/* <bits|psi> = prod_q A_q[:, bits[q], :]; bits has n entries of 0/1. */
tnsim_status tnsim_amplitude(tnsim_mps mps, const uint8_t *bits, tnsim_c128 *out);

/* <a|b> by transfer contraction (both handles on the same device). */
tnsim_status tnsim_overlap(tnsim_mps a, tnsim_mps b, tnsim_c128 *out);

/* Copy the state of src into dst (same n; storage converted; dst's chi_max
   must hold src's bond dimensions). */
tnsim_status tnsim_mps_copy(tnsim_mps dst, tnsim_mps src);

/* ---- inspection, import/export (synchronising) ---- */
tnsim_status tnsim_bond_dims(tnsim_mps mps, int32_t *out /* n-1 */);
/* sum of discarded weights, product of (1 - eps) over gates, gate count */
tnsim_status tnsim_truncation_stats(tnsim_mps mps, double *sum_eps, double *prod_1_minus_eps,
                                    int64_t *n2q);
/* Largest Jacobi sweep count used by the last apply call. */
tnsim_status tnsim_last_sweeps(tnsim_mps mps, int32_t *sweeps);
/* Jacobi sweep counts per two-qubit gate, summed since creation or the
   last tnsim_profile(mps, 1). */
tnsim_status tnsim_sweep_stats(tnsim_mps mps, int64_t *gates, int64_t *sweeps_sum,
                               int32_t *sweeps_max);
/* Per two-qubit gate of the last apply call, 6 entries: left site i, chiL,
   chiM, chiR (before the gate), kept k, Jacobi sweeps.  Writes at most
   max_gates records to out; *n receives the record count. */
tnsim_status tnsim_last_batch(tnsim_mps mps, int32_t *out, int32_t max_gates, int32_t *n);
/* Site q as complex128 (chiL*2*chiR entries); host may be NULL to query dims. */
tnsim_status tnsim_export_site(tnsim_mps mps, int32_t q, tnsim_c128 *host, int32_t *chiL,
                               int32_t *chiR);
tnsim_status tnsim_export_lambda(tnsim_mps mps, int32_t bond, double *host, int32_t *chi);
/* Replace the state: sites[q] (chis[q] x 2 x chis[q+1], complex128), lambdas[b]
   (chis[b+1] values); chis has n+1 entries, chis[0] = chis[n] = 1. */
tnsim_status tnsim_import_state(tnsim_mps mps, const tnsim_c128 *const *sites,
                                const double *const *lambdas, const int32_t *chis);

/* ---- perfect sampling ("measure all" shots, Sec. III.A; Ferris and Vidal,
   Phys. Rev. B 85, 165146 (2012)) ----
   Draws `shots` bit strings x with probability |<x|psi>|^2 / <psi|psi>.
   Qubits are drawn from n-1 down to 0; qubit q of shot i takes bit 0 when
   dev_u[i*n + q] < P(s_q = 0 | bits drawn so far), else bit 1.  The
   conditionals come from the left-block Gram matrices E_q, so they are exact
   in any gauge (E_q = I for a left-orthonormal block).  Shots that drew the
   same bits so far share one partial contraction (the memo of drawn
   prefixes), so each step contracts at most min(2^(n-1-q), shots) vectors.
   All arithmetic is float64.  The state is not modified.
     dev_ws     device workspace of tnsim_sample_workspace_bytes(cfg, m) bytes
                for some m >= shots, 256-byte aligned, owned by the caller;
     dev_u      device, shots x n float64 uniforms in [0, 1), row-major by shot;
     dev_bits   device, shots x n bytes (0/1), written;
     dev_logp   device, shots float64 (log of each drawn string's probability),
                written, or NULL.
   The call runs on the handle's stream and returns after it has finished.
   Errors: TNSIM_E_ARG for a bad pointer or shot count, or (found on the
   device, after the draws) a uniform outside [0, 1) -- dev_bits is then
   unspecified; TNSIM_E_CAPACITY when ws_bytes is too small.  shots = 0 does
   nothing. */
size_t tnsim_sample_workspace_bytes(const tnsim_config *cfg, int32_t max_shots);
tnsim_status tnsim_sample(tnsim_mps mps, void *dev_ws, size_t ws_bytes, int32_t shots,
                          const double *dev_u, uint8_t *dev_bits, double *dev_logp);
/* The same in two parts, for many draws from one state: tnsim_sample_prepare
   builds the per-site weights M_q^s = A_q^{sH} E_q A_q^s (the part of
   tnsim_sample that does not depend on the shots) in a workspace sized for
   max_shots; each tnsim_sample_draw then draws up to max_shots strings from
   them, exactly as tnsim_sample would.  A draw needs the same workspace
   (pointer and size) as the last prepare and an unchanged state: after any
   call that may change the state (gates, reset, import, copy into it,
   gradients) it returns TNSIM_E_ARG until prepared again.  Shots above
   max_shots: TNSIM_E_CAPACITY. */
/* tnsim_sample without allocation, for callers that cannot allocate device
   memory (code under HIP graph capture, tight serving loops, harnesses that
   forbid hipMalloc): the same draws as tnsim_sample, with the workspace taken
   from a fixed device array of TNSIM_SAMPLE_SCRATCH_BYTES that the library
   holds on every GPU it runs on until the process ends.  The call makes no
   allocation of any kind.  All calls on one GPU share that array (it keeps
   the last call's contents; every call initialises what it reads), so calls
   that overlap in time on one GPU -- from several threads, or on several
   handles whose streams run concurrently -- race: serialise them.
   Errors: as tnsim_sample, and TNSIM_E_CAPACITY when the workspace that
   tnsim_sample_workspace_bytes gives for this handle's configuration and
   `shots` exceeds TNSIM_SAMPLE_SCRATCH_BYTES (tnsim_last_error says by how
   much). */
#define TNSIM_SAMPLE_SCRATCH_BYTES (128u << 20)
tnsim_status tnsim_sample_noalloc(tnsim_mps mps, int32_t shots, const double *dev_u,
                                  uint8_t *dev_bits, double *dev_logp);
tnsim_status tnsim_sample_prepare(tnsim_mps mps, void *dev_ws, size_t ws_bytes, int32_t max_shots);
tnsim_status tnsim_sample_draw(tnsim_mps mps, void *dev_ws, size_t ws_bytes, int32_t shots,
                               const double *dev_u, uint8_t *dev_bits, double *dev_logp);

/* ---- gradients of a Pauli-sum loss with respect to rotation angles ----
   Loss L = sum_t coeffs[t] <psi|P_t|psi>/<psi|psi>, psi = circuit |0...0>.
   Gate g of `circuit` with param_of_gate[g] = p >= 0 is the rotation
   R_P(angles[p]) = exp(-i angles[p] P/2) about axis rot_axis[p] (0=X, 1=Y,
   2=Z) on qubit q0 (its matrix field is ignored); other gates use their
   matrix.  The adjoint is hand-written: the reverse sweep recomputes each
   segment [segment_start[s], segment_start[s+1]) from a checkpoint of the
   state at its start and back-propagates through every gate, including the
   truncated SVD (Lorentzian-broadened 1/(sigma_j^2 - sigma_l^2) over the full
   left basis; the loss is gauge invariant, so the phase term vanishes).
   Requires precision TNSIM_FP64.  The caller provides a device workspace of
   tnsim_grad_workspace_bytes(cfg, n_segments, max gates per segment,
   n_params) bytes (256-byte aligned) that must stay valid until
   tnsim_backward returns.  The forward resets the state to |0...0>; after
   either call the handle holds the circuit's final state. */
size_t tnsim_grad_workspace_bytes(const tnsim_config *cfg, int32_t n_segments,
                                  int32_t max_segment_gates, int32_t n_params);
tnsim_status tnsim_forward_checkpointed(tnsim_mps mps, void *dev_ws, size_t ws_bytes,
                                        const tnsim_gate *circuit, int32_t n_gates,
                                        const int32_t *param_of_gate, const int32_t *rot_axis,
                                        const double *angles, int32_t n_params,
                                        const int32_t *segment_start, int32_t n_segments,
                                        const char *const *paulis, const double *coeffs,
                                        int32_t n_terms, double *loss);
/* grad_angles[p] = dloss * dL/d angles[p] (host array of n_params). */
tnsim_status tnsim_backward(tnsim_mps mps, double dloss, double *grad_angles);

/* ---- profiling (for measurement; off by default) ----
   When enabled, every kernel launch of the handle is bracketed by HIP events
   on the handle's stream and the Jacobi kernels count the work they actually
   do.  Enabling clears the totals. */
typedef enum {
  TNSIM_K_THETA = 0, /* two-site merge + gate epilogue */
  TNSIM_K_GRAM,      /* pair Gram blocks */
  TNSIM_K_EIG,       /* 64x64 Hermitian Jacobi */
  TNSIM_K_ROT,       /* pair rotations */
  TNSIM_K_COLNORM,   /* column norms */
  TNSIM_K_TRUNC,     /* sort + truncation rule */
  TNSIM_K_WB_LEFT,   /* left-site write-back */
  TNSIM_K_WB_RIGHT,  /* right-site write-back */
  TNSIM_K_1Q,        /* one-qubit gates */
  TNSIM_K_OTHER,     /* setup, sweep control */
  TNSIM_K_QR,        /* QR preconditioning: Householder panels, updates, Q1 W */
  TNSIM_K_COUNT
} tnsim_kernel_class;

typedef struct {
  double ms;        /* summed event time of the launches */
  int64_t launches; /* launch count */
  double flops;     /* algorithmic real flops of those launches */
  double bytes;     /* algorithmic bytes moved (operands read + results written) */
} tnsim_kernel_stat;

tnsim_status tnsim_profile(tnsim_mps mps, int32_t enable);
/* out has TNSIM_K_COUNT entries (synchronising). */
tnsim_status tnsim_profile_read(tnsim_mps mps, tnsim_kernel_stat *out);

/* Attainable float64 rate of this device (synchronising; a measurement aid,
   no operation of the method).  unit 0: independent chains of
   v_mfma_f64_16x16x4f64 (the matrix-core instruction of the Jacobi Grams and
   rotations, the merge and the write-back); unit 1: independent chains of
   vector v_fma_f64 (the pair solve's arithmetic); unit 2: both at once
   (wavefronts 0 and 2 of each workgroup on matrix-core chains, 1 and 3 on
   four times as many vector FMAs; the combined rate); unit 3: independent
   chains of the four-block v_mfma_f64_4x4x4f64 (256 multiply-adds each).
   Eight workgroups of four
   wavefronts per CU, `iters` x 8 instructions per wavefront (1 <= iters <=
   2^20), timed with HIP events on the handle's stream after one untimed
   launch; *tflops_out (host) receives the real flops per second / 1e12.  The
   published peaks count both units at 78.6 TFLOP/s; this is what the device
   sustains.  Allocates and frees one small device buffer.  Errors:
   TNSIM_E_ARG (bad handle, unit outside 0..3, iters or NULL out),
   TNSIM_E_DEVICE. */
tnsim_status tnsim_probe_fp64(tnsim_mps mps, int32_t unit, int32_t iters, double *tflops_out);

/* Launch-shape autotuner (synchronising).  Times two Jacobi kernels on this
   handle's workspace slots (zeroed scratch; the state is not touched) in
   each of TNSIM_TUNE_BUCKETS pair-count classes (<= 32, <= 128, <= 512 and
   more pairs per launch, largest gate the handle can hold) and keeps the
   fastest shape of each; later sweeps use the table instead of the built-in
   rules:
     - the rotation: rows per workgroup, one of 64, 128, 256, 512;
     - the pair Grams: K-split, the number of row chunks (1, 2, 4, 8, 16)
       whose partial Grams the pair solve adds up, within the handle's pool
       of partials (room for a K-split of 4 with every slot in use).
   The rotation shape does not change any result (every row is computed the
   same way); the K-split changes the order in which a Gram's row sums are
   added, so results agree to rounding with those of the built-in rule.
   table_out (host, TNSIM_TUNE_ENTRIES entries, may be NULL) receives the
   rows per rotation workgroup of each class in entries 0..3 and the Gram
   K-split of each class in entries 4..7.  Errors: TNSIM_E_ARG (bad handle),
   TNSIM_E_DEVICE. */
#define TNSIM_TUNE_BUCKETS 4
#define TNSIM_TUNE_ENTRIES (2 * TNSIM_TUNE_BUCKETS)
tnsim_status tnsim_autotune(tnsim_mps mps, int32_t *table_out);

/* Install a launch-shape table (host, TNSIM_TUNE_ENTRIES entries laid out as
   tnsim_autotune's: rows per rotation workgroup, 0 for the built-in rule or
   one of 64, 128, 256, 512, then Gram K-splits, 0 for the built-in rule or a
   power of two up to 16; a K-split beyond what a launch's pool of partials
   or its rows allow is reduced to fit), e.g. one that tnsim_autotune chose
   on another handle of the same shape, so that both run the same launches.
   Errors: TNSIM_E_ARG (bad handle, NULL table or an entry outside those
   sets; the handle's table is then unchanged). */
tnsim_status tnsim_set_launch_table(tnsim_mps mps, const int32_t *table);

/* ---- circuit front end (host only; no device work) ----
   OpenQASM 2.0 text -> one- and two-qubit gates (Sec. III: the simulator's
   input is OpenQASM).  Read: OPENQASM 2.x; include (the standard gate
   library is built in); qreg/creg (qubits numbered in declaration order);
   gate definitions with parameters; parameter expressions (+ - * / ^, pi,
   sin cos tan exp ln sqrt); whole-register arguments broadcast; barrier and
   measure are skipped (all qubits are sampled after the circuit); opaque,
   reset and if are rejected.  Built-in gates: id x y z h s sdg t tdg sx sxdg
   rx ry rz p u1 u2 u3 u U, cx CX cy cz ch csx crx cry crz cp cu1 cu3 cu swap
   rxx ryy rzz, and ccx cswap as six-CNOT decompositions.  Matrices: U(t,p,l)
   = [[cos t/2, -e^{il} sin t/2], [e^{ip} sin t/2, e^{i(p+l)} cos t/2]],
   R_P(t) = exp(-i t P/2), p(l) = diag(1, e^{il}), controlled gates control
   on their first qubit; a two-qubit matrix has row 2*s_q0 + s_q1.
   gates: host array of cap entries; *n_gates receives the count (also when
   it exceeds cap: then TNSIM_E_CAPACITY and nothing is written).
   *n_qubits: total qubits of all qregs.  Syntax or semantic errors give
   TNSIM_E_ARG with a message (line number first) in err (err_len bytes,
   may be NULL). */
tnsim_status tnsim_qasm_parse(const char *text, tnsim_gate *gates, int32_t cap, int32_t *n_gates,
                              int32_t *n_qubits, char *err, int32_t err_len);
/* Gate fusion (Sec. IV.A: sequential gates that share qubits are compressed
   so that fewer contractions are needed), in one pass over the circuit:
   a one-qubit gate is multiplied into the last two-qubit gate on its qubit
   (if there is one) or held until the next two-qubit gate on its qubit,
   which takes it; a two-qubit gate whose two qubits were last touched by
   one earlier two-qubit gate on the same pair is multiplied into that gate;
   one-qubit gates never followed by a two-qubit gate are emitted at the end,
   one per qubit.  The fused circuit is the same unitary.  out needs room for
   n_in gates (the result never has more); qubits must be < n_qubits. */
tnsim_status tnsim_fuse(const tnsim_gate *in, int32_t n_in, int32_t n_qubits, tnsim_gate *out,
                        int32_t *n_out);

const char *tnsim_status_string(tnsim_status st);
const char *tnsim_last_error(tnsim_mps mps);

#ifdef __cplusplus
}
#endif
#endif /* TNSIM_H */
