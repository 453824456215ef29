// Host side of the tnsim C ABI: argument validation, arena carving, gate
// descriptors, the Jacobi sweep loop and the readout drivers.  All arithmetic
// on the state runs in the HIP kernels of this library.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/tnsim.h"
#include "tnsim_internal.h"

using namespace tn;

namespace {

constexpr size_t ALIGN = 256;
inline size_t align_up(size_t x, size_t a = ALIGN) { return (x + a - 1) / a * a; }
inline int pad_to(int x, int a) { return (x + a - 1) / a * a; }

struct Layout {
  int n = 0, chi_max = 0, storage = 0, nslots = 0, desc_cap = 0;
  size_t elem = 16;                 // site element bytes
  std::vector<int> bondcap;         // n-1
  std::vector<int> dimcap;          // n+1
  std::vector<size_t> site_off, site_cap, lam_off;
  size_t dims_off = 0, site_tab_off = 0, lam_tab_off = 0;
  int cmax = 0, ldx_max = 0, cols_pad_max = 0, npairs_max = 0, gp_blocks = 0;
  size_t slot_bytes = 0, slot0_off = 0;
  size_t x_off = 0, j_off = 0, t_off = 0, v_off = 0, pf_off = 0, ver_off = 0, seen_off = 0,
         sig_off = 0, perm_off = 0, sc_off = 0, u_off = 0, tq_off = 0;  // within a slot
  size_t gp_off = 0;  // pooled pair-Gram partials
  size_t desc_off = 0, desc2_off = 0, d1_off = 0, ctr_off = 0, scg_off = 0;
  size_t e0_off = 0, e1_off = 0, f_off = 0, f2_off = 0, va_off = 0, vb_off = 0;
  size_t total = 0;
};

bool valid_config(const tnsim_config *c) {
  if (!c) return false;
  if (c->n_qubits < 2 || c->n_qubits > 100000) return false;
  if (c->chi_max < 1 || c->chi_max > 2048) return false;
  if (!(c->cutoff >= 0.0)) return false;
  if (c->precision < 0 || c->precision > 3) return false;
  if (c->storage < 0 || c->storage > 1) return false;
  return true;
}

Layout make_layout(const tnsim_config &c) {
  Layout L;
  L.n = c.n_qubits;
  L.chi_max = c.chi_max;
  L.storage = c.storage;
  L.elem = c.storage == 0 ? 16 : 8;
  L.nslots = c.max_layer_gates > 0 ? std::min(c.max_layer_gates, std::max(1, L.n / 2))
                                   : std::max(1, L.n / 2);
  // descriptors: this handle's gates, or, for a handle that leads a
  // multi-circuit batch, up to max_layer_gates gates of all its handles
  L.desc_cap = std::max(L.nslots, c.max_layer_gates);
  const int n = L.n;
  L.bondcap.resize(n - 1);
  int maxbond = 1;
  for (int b = 0; b < n - 1; b++) {
    int e = std::min(b + 1, n - 1 - b);
    long long cap = e >= 30 ? (1LL << 30) : (1LL << e);
    L.bondcap[b] = (int)std::min<long long>(cap, c.chi_max);
    maxbond = std::max(maxbond, L.bondcap[b]);
  }
  L.dimcap.assign(n + 1, 1);
  for (int q = 1; q < n; q++) L.dimcap[q] = L.bondcap[q - 1];
  size_t off = 0;
  L.dims_off = off;
  off = align_up(off + sizeof(int32_t) * (n + 1));
  L.site_tab_off = off;
  off = align_up(off + sizeof(void *) * n);
  L.lam_tab_off = off;
  off = align_up(off + sizeof(void *) * (n - 1));
  L.site_off.resize(n);
  L.site_cap.resize(n);
  for (int q = 0; q < n; q++) {
    L.site_cap[q] = (size_t)L.dimcap[q] * 2 * L.dimcap[q + 1];
    L.site_off[q] = off;
    off = align_up(off + L.site_cap[q] * L.elem);
  }
  L.lam_off.resize(n - 1);
  for (int b = 0; b < n - 1; b++) {
    L.lam_off[b] = off;
    off = align_up(off + sizeof(double) * L.bondcap[b]);
  }
  // two-site workspaces
  L.cmax = 2 * maxbond;
  L.ldx_max = pad_to(L.cmax, 16);  // whole 16-row tiles of every column (rotation stores)
  L.cols_pad_max = pad_to(L.cmax, PW);
  L.npairs_max = L.cols_pad_max / PW;
  // with QR preconditioning, J and U also serve as scratch for the group
  // updates: partial sums and Y, (row chunks + 1) x QG rows of cols_pad_max
  const size_t xj_elems = (size_t)L.ldx_max * L.cols_pad_max;
  size_t scr_elems = 0;
  if (c.svd_precondition) {
    const int rchunks = (std::min(L.cmax, QR_MAX_ROWS) + QR_RC - 1) / QR_RC;
    scr_elems = (size_t)(rchunks + 1) * QG * L.cols_pad_max;
  }
  size_t s = 0;
  L.x_off = s;
  s = align_up(s + sizeof(double2) * xj_elems);
  L.j_off = s;
  s = align_up(s + sizeof(double2) * std::max(xj_elems, scr_elems));
  L.t_off = s;
  s = align_up(s + sizeof(double2) * (size_t)L.cmax * L.cmax);
  L.v_off = s;
  s = align_up(s + sizeof(double2) * (size_t)L.npairs_max * PW * PW);
  L.pf_off = s;
  s = align_up(s + sizeof(int) * L.npairs_max);
  L.ver_off = s;
  s = align_up(s + sizeof(int) * 2 * L.npairs_max);
  L.seen_off = s;
  s = align_up(s + sizeof(int2) * 4 * (size_t)L.npairs_max * L.npairs_max);
  L.sig_off = s;
  s = align_up(s + sizeof(double) * L.cols_pad_max);
  L.perm_off = s;
  s = align_up(s + sizeof(int) * L.cols_pad_max);
  L.sc_off = s;
  s = align_up(s + sizeof(SlotScalars));
  if (c.svd_precondition) {  // U_k and the panels' T factors of both QR stages
    L.u_off = s;
    s = align_up(s + sizeof(double2) * std::max(xj_elems, scr_elems));
    L.tq_off = s;
    s = align_up(s + sizeof(double2) * 2 *
                         ((size_t)(L.cols_pad_max / QNB) * QNB * QNB +
                          (size_t)(L.cols_pad_max / QG) * QG * QG));
  }
  L.slot_bytes = s;
  L.slot0_off = off;
  off = align_up(off + L.slot_bytes * L.nslots);
  // partial pair Grams: room for a K-split of GP_PER_SLOT with every slot active
  L.gp_blocks = std::max(L.nslots * GP_PER_SLOT, KSPLIT_MAX) * L.npairs_max;
  L.gp_off = off;
  off = align_up(off + sizeof(double2) * (size_t)L.gp_blocks * PW * PW);
  L.desc_off = off;
  off = align_up(off + sizeof(GateDesc) * L.desc_cap);
  L.desc2_off = off;  // descriptors of gates prepared on the second stream
  off = align_up(off + sizeof(GateDesc) * L.desc_cap);
  L.scg_off = off;
  off = align_up(off + sizeof(SlotScalars) * L.desc_cap);
  L.d1_off = off;
  off = align_up(off + sizeof(Gate1Desc) * n);
  L.ctr_off = off;
  off = align_up(off + sizeof(unsigned long long) * CTR_COUNT);
  const size_t ee = sizeof(double2) * (size_t)maxbond * maxbond;
  const size_t ff = sizeof(double2) * (size_t)maxbond * 2 * maxbond;
  L.e0_off = off;
  off = align_up(off + ee);
  L.e1_off = off;
  off = align_up(off + ee);
  L.f_off = off;
  off = align_up(off + ff);
  L.f2_off = off;
  off = align_up(off + ff);
  L.va_off = off;
  off = align_up(off + sizeof(double2) * maxbond);
  L.vb_off = off;
  off = align_up(off + sizeof(double2) * maxbond);
  L.total = off;
  return L;
}

// Gate with orientation fixed to (i, i+1).  Flags of the canonicalisation
// sweeps, which run the two-site path with the identity gate: UNWEIGHTED
// decomposes theta itself (no lambda_{i+1} weight), NO_CUT drops only
// numerically zero values (cutoff 0), NO_STATS leaves the gate statistics
// alone, EPS_ONLY adds the discarded weight to the truncation statistics
// without counting a gate.
enum { PEND_UNWEIGHTED = 1, PEND_NO_CUT = 2, PEND_NO_STATS = 4, PEND_EPS_ONLY = 8 };
struct Pending {
  int i;
  double2 g[16];
  int flags = 0;
  // bond propagation's window steps read and write some sites elsewhere than
  // the site buffers (nullptr: the site buffer)
  void *a0_in = nullptr, *a1_in = nullptr, *a0_out = nullptr, *a1_out = nullptr;
};

// One gate of the segment being differentiated, recorded during recompute.
struct GradRec {
  int kind = 0;  // 1 or 2 qubits
  int q = 0;     // site (1q) or left site (2q)
  int chiL = 0, chiM = 0, chiR = 0, k = 0;
  double N = 1.0;
  int param = -1, axis = -1;
  bool has_lam = false;
  Mat4 u{};
  Mat16 g{};
  size_t off = 0;  // record slot in the workspace
};

// Workspace layout and circuit of the last tnsim_forward_checkpointed call.
struct GradState {
  bool ready = false;
  char *ws = nullptr;
  size_t ws_bytes = 0;
  int n = 0, n_params = 0, n_seg = 0, max_seg = 0;
  std::vector<tnsim_gate> gates;
  std::vector<int> param, axis, seg_start;
  std::vector<double> angles;
  std::vector<std::string> paulis;
  std::vector<double> coeffs;
  std::vector<std::vector<int>> ckpt_dims;
  // workspace offsets
  size_t state_bytes = 0, ckpt0 = 0;
  std::vector<size_t> st_site, st_lam;  // offsets inside one checkpoint
  std::vector<size_t> cot_site, cot_lam;
  size_t envL = 0, envR = 0, env_stride = 0, envF = 0, envF2 = 0;
  size_t tmp0 = 0, tmp_stride = 0, lam2 = 0, sbar = 0, dots = 0, ubar = 0, grad = 0;
  size_t rec0 = 0, rec_stride = 0, rec_a = 0, rec_b = 0, rec_lam = 0, rec_T = 0, rec_J = 0,
         rec_sig = 0, rec_perm = 0;
  size_t total = 0;
  double loss = 0.0;
};

}  // namespace

struct tnsim_mps_s {
  tnsim_config cfg;
  Layout L;
  char *arena = nullptr;
  size_t arena_bytes = 0;
  hipStream_t stream = nullptr;
  int device = 0;
  std::vector<int> dims;  // host copy, n+1
  double sum_eps = 0.0, prod_keep = 1.0;
  int64_t n2q = 0;
  int last_sweeps = 0;
  bool poisoned = false;
  std::string err;
  char *pin = nullptr;
  size_t pin_bytes = 0;
  // second stream of the circuit scheduler: gates admitted into the sweeps
  // are prepared there (own descriptor region and pinned staging buffer)
  // while the gates in flight keep sweeping on `stream`
  hipStream_t stream2 = nullptr;
  char *pin2 = nullptr;
  hipEvent_t ev_main = nullptr, ev_prep = nullptr;
  // Jacobi sweeps in flight: each sweep's gathered scalars go to pinned
  // buffer 0 or 1 (the second at pin + pin_sc1_off), marked by ev_sw[b]
  hipEvent_t ev_sw[2] = {nullptr, nullptr};
  size_t pin_sc1_off = 0;
  bool speculate = true;  // TNSIM_SPECULATE=0: one sweep in flight, host test in between
  // profiling
  struct Rec {
    int cls;
    hipEvent_t a, b;
    double flops, bytes;
  };
  bool prof = false;
  int inner_sweeps = 1;  // one inner sweep per pair solve (outer sweeps finish the job)
  bool overlap_prepare = true;  // TNSIM_OVERLAP_PREPARE=0: scheduler prepares in line
  int admit_group = 16;         // scheduler: ready gates admitted together (TNSIM_ADMIT_GROUP)
  // sampling weights prepared for draws: valid while the state is unchanged
  uint64_t state_version = 0;   // bumped by every call that may change the state
  void *smp_ws = nullptr;
  size_t smp_bytes = 0;
  int smp_cap = 0;
  uint64_t smp_version = 0;
  std::vector<int32_t> last_batch;  // 6 ints per two-qubit gate of the last apply call
  GradState grad;
  // captured Jacobi sweep (reused while the batch shape is unchanged)
  bool graphs = true;
  bool pair_skip = true;  // skip Grams of block pairs known orthogonal (TNSIM_PAIR_SKIP=0: off)
  int gram_wg_target = 1024;  // K-split the pair Grams up to this many workgroups
  int tune_rot_rows[TNSIM_TUNE_BUCKETS] = {0, 0, 0, 0};  // autotuned, 0 = built-in rule
  int tune_gram_ks[TNSIM_TUNE_BUCKETS] = {0, 0, 0, 0};   // autotuned, 0 = built-in rule
  hipGraphExec_t sweep_exec = nullptr;
  long long sweep_key[7] = {-1, -1, -1, -1, -1, -1, -1};
  int64_t sw_gates = 0, sw_sum = 0;
  int sw_max = 0;
  std::vector<hipEvent_t> evpool;
  std::vector<Rec> pending, pending2;  // profiling events on stream, stream2
  tnsim_kernel_stat kstat[TNSIM_K_COUNT] = {};

  template <class T>
  T *at(size_t off) const {
    return reinterpret_cast<T *>(arena + off);
  }
  void *site(int q) const { return arena + L.site_off[q]; }
  double *lam(int b) const { return at<double>(L.lam_off[b]); }
  char *slot(int s) const { return arena + L.slot0_off + L.slot_bytes * (size_t)s; }
  int32_t *dims_dev() const { return at<int32_t>(L.dims_off); }
};

namespace {

thread_local std::string g_create_error;

tnsim_status fail(tnsim_mps h, hipError_t e, const char *where) {
  if (!h->poisoned) {
    h->poisoned = true;
    char buf[256];
    snprintf(buf, sizeof buf, "%s: %s", where, hipGetErrorString(e));
    h->err = buf;
  }
  return TNSIM_E_DEVICE;
}

#define HIPCHK(h, call)                                   \
  do {                                                    \
    hipError_t e_ = (call);                               \
    if (e_ != hipSuccess) return fail((h), e_, #call);   \
  } while (0)

#define LAUNCHCHK(h, what)                                \
  do {                                                    \
    hipError_t e_ = hipGetLastError();                    \
    if (e_ != hipSuccess) return fail((h), e_, what);     \
  } while (0)

inline double2 to_d2(const tnsim_c128 &c) { return make_double2(c.re, c.im); }

tnsim_status check_handle(tnsim_mps h) {
  if (!h) return TNSIM_E_ARG;
  if (h->poisoned) return TNSIM_E_DEVICE;
  return TNSIM_OK;
}

// ---- profiling helpers: events bracket each launch when enabled
hipEvent_t ev_get(tnsim_mps h) {
  if (!h->evpool.empty()) {
    hipEvent_t e = h->evpool.back();
    h->evpool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

struct ProfScope {
  tnsim_mps h;
  int cls;
  double flops, bytes;
  hipStream_t st;
  std::vector<tnsim_mps_s::Rec> *pend;
  hipEvent_t a = nullptr;
  ProfScope(tnsim_mps h_, int cls_, double fl = 0.0, double by = 0.0, bool second = false)
      : h(h_), cls(cls_), flops(fl), bytes(by), st(second ? h_->stream2 : h_->stream),
        pend(second ? &h_->pending2 : &h_->pending) {
    if (h->prof) {
      a = ev_get(h);
      if (a) hipEventRecord(a, st);
    }
  }
  ~ProfScope() {
    if (!h->prof || !a) return;
    hipEvent_t b = ev_get(h);
    if (!b) return;
    hipEventRecord(b, st);
    pend->push_back({cls, a, b, flops, bytes});
  }
};

// After a stream synchronisation: fold finished event pairs into the totals.
void prof_drain(tnsim_mps h, bool second = false) {
  auto &pend = second ? h->pending2 : h->pending;
  for (auto &r : pend) {
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) h->kstat[r.cls].ms += ms;
    h->kstat[r.cls].launches += 1;
    h->kstat[r.cls].flops += r.flops;
    h->kstat[r.cls].bytes += r.bytes;
    h->evpool.push_back(r.a);
    h->evpool.push_back(r.b);
  }
  pend.clear();
}

tnsim_status init_state(tnsim_mps h) {
  const int n = h->L.n;
  launch_init_state(h->stream, h->at<void *const>(h->L.site_tab_off), n, h->L.storage,
                    h->at<double *const>(h->L.lam_tab_off), n - 1);
  LAUNCHCHK(h, "init_state");
  std::vector<int32_t> ones(n + 1, 1);
  h->dims.assign(n + 1, 1);
  HIPCHK(h, hipMemcpyAsync(h->dims_dev(), ones.data(), sizeof(int32_t) * (n + 1),
                           hipMemcpyHostToDevice, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  h->sum_eps = 0.0;
  h->prod_keep = 1.0;
  h->n2q = 0;
  h->last_sweeps = 0;
  return TNSIM_OK;
}

// One two-qubit gate of a batch: the handle it belongs to, the workspace slot
// of that handle it uses, and the gate.
struct BatchItem {
  tnsim_mps h;
  int slot;
  const Pending *p;
};

// Pair-count class of a launch, for the autotuned rotation shape.
int tune_bucket(int pairs) { return pairs <= 32 ? 0 : pairs <= 128 ? 1 : pairs <= 512 ? 2 : 3; }

SlotScalars *pin_scalars(tnsim_mps o, int buf = 0) {
  if (buf) return reinterpret_cast<SlotScalars *>(o->pin + o->pin_sc1_off);
  return reinterpret_cast<SlotScalars *>(o->pin + align_up(sizeof(GateDesc) * o->L.desc_cap));
}

// Descriptor of one two-qubit gate from its handle's current bond dimensions.
// `o` owns the launches (profiling counters, the inner-sweep cap).
GateDesc make_desc(tnsim_mps o, const BatchItem &it, bool force_trans) {
  GateDesc d;
  memset(&d, 0, sizeof d);
  const tnsim_mps h = it.h;
  const Layout &L = h->L;
  const int i = it.p->i;
  d.i = i;
  d.chiL = h->dims[i];
  d.chiM = h->dims[i + 1];
  d.chiR = h->dims[i + 2];
  d.m = 2 * d.chiL;
  d.n = 2 * d.chiR;
  // X = M^H (with the left vectors accumulated in J) when M is wide, or
  // always when the caller needs the full left basis (the adjoint)
  d.trans = force_trans || d.n > d.m;
  // QR-preconditioned SVD for square or tall M that fits one panel workgroup
  d.qr = h->cfg.svd_precondition && !d.trans && d.m <= QR_MAX_ROWS;
  d.rows = d.qr ? d.n : (d.trans ? d.n : d.m);
  d.cols = d.trans ? d.m : d.n;
  d.ldx = pad_to(d.rows, 16);
  d.ldj = pad_to(d.m, 16);
  d.colsPad = pad_to(d.cols, PW);
  d.nblk = d.colsPad / BW;
  d.chiMax = h->cfg.chi_max;
  d.storage = h->cfg.storage;
  d.tfp32 = o->cfg.precision != TNSIM_FP64;
  d.innerSweeps = o->inner_sweeps;
  // default Jacobi tolerance: float64 level for complex128 sites; for
  // complex64 sites 2^-30, a factor 64 below the rounding of the stored
  // vectors (U_k is written in complex64, so orthogonality beyond that is lost)
  d.tol = h->cfg.jacobi_tol > 0 ? h->cfg.jacobi_tol
                                : (h->cfg.storage == TNSIM_STORE_C64
                                       ? 0x1p-30
                                       : std::max(d.rows, 16) * 0x1p-53);
  d.cutoff = (it.p->flags & PEND_NO_CUT) ? 0.0 : h->cfg.cutoff;
  d.A0 = it.p->a0_in ? it.p->a0_in : h->site(i);
  d.A1 = it.p->a1_in ? it.p->a1_in : h->site(i + 1);
  d.A0out = it.p->a0_out ? it.p->a0_out : h->site(i);
  d.A1out = it.p->a1_out ? it.p->a1_out : h->site(i + 1);
  d.lamR = (i + 1 <= L.n - 2 && !(it.p->flags & PEND_UNWEIGHTED)) ? h->lam(i + 1) : nullptr;
  d.lamOut = h->lam(i);
  char *sl = h->slot(it.slot);
  d.X = (double2 *)(sl + L.x_off);
  d.J = (double2 *)(sl + L.j_off);
  if (d.qr) {  // M and Q1's reflectors in the X buffer; the Jacobi on R2^H in J's
    d.Qm = d.X;
    d.ldq = pad_to(d.m, 4);
    d.X = d.J;
    d.J = nullptr;
    d.U = (double2 *)(sl + L.u_off);
    d.ldu = pad_to(d.m, 4);
    d.Tq = (double2 *)(sl + L.tq_off);
  }
  d.T = sl + L.t_off;
  d.V = (double2 *)(sl + L.v_off);
  d.pairFlag = (int *)(sl + L.pf_off);
  d.blkVer = o->pair_skip ? (int *)(sl + L.ver_off) : nullptr;
  d.pairSeen = o->pair_skip ? (int2 *)(sl + L.seen_off) : nullptr;
  d.sig2 = (double *)(sl + L.sig_off);
  d.perm = (int *)(sl + L.perm_off);
  d.sc = (SlotScalars *)(sl + L.sc_off);
  for (int e = 0; e < 16; e++) d.g[e] = it.p->g[e];
  d.gpStride = L.npairs_max;
  d.dimsDev = h->dims_dev();
  d.ctr = o->prof ? o->at<unsigned long long>(o->L.ctr_off) : nullptr;
  return d;
}

// Copy descriptors into the owner's descriptor array.  Waits for the stream
// first: the pinned staging buffer may still feed an earlier copy.  With
// `second`, the second stream, its staging buffer and descriptor region.
tnsim_status put_descs(tnsim_mps o, const GateDesc *D, int n, bool second = false) {
  hipStream_t st = second ? o->stream2 : o->stream;
  char *pin = second ? o->pin2 : o->pin;
  HIPCHK(o, hipStreamSynchronize(st));
  prof_drain(o, second);
  memcpy(pin, D, sizeof(GateDesc) * n);
  HIPCHK(o, hipMemcpyAsync(o->at<GateDesc>(second ? o->L.desc2_off : o->L.desc_off), pin,
                           sizeof(GateDesc) * n, hipMemcpyHostToDevice, st));
  return TNSIM_OK;
}

// Everything before the Jacobi sweeps: merge, gate and weight, QR
// preconditioning, column norms, the per-gate scalars.  With `second`, on
// the second stream (the caller orders it after the work it depends on).
tnsim_status gates_prepare(tnsim_mps o, const GateDesc *D, int ng, bool second = false) {
  tnsim_mps h = o;
  int maxM = 0, maxColsPad = 0, maxChiR = 0, qrN = 0, qrMr = 0;
  double theta_flop = 0.0, theta_byte = 0.0, colnorm_byte = 0.0, qr_flop = 0.0;
  for (int g = 0; g < ng; g++) {
    const GateDesc &d = D[g];
    maxM = std::max(maxM, d.m);
    maxColsPad = std::max(maxColsPad, d.colsPad);
    maxChiR = std::max(maxChiR, d.chiR);
    const double eb = d.storage == 0 ? 16.0 : 8.0, tb = d.tfp32 ? 8.0 : 16.0;
    theta_flop += 8.0 * d.m * d.chiM * d.n + 32.0 * d.m * d.n;
    theta_byte += eb * ((double)d.m * d.chiM + (double)d.chiM * d.n) + (tb + 16.0) * d.m * d.n;
    colnorm_byte += 16.0 * d.rows * d.cols;
    if (d.qr) {
      const double mm = d.m, nn = d.n;
      qrN = std::max(qrN, d.n);
      qrMr = std::max(qrMr, d.m);
      qr_flop += 8.0 * (mm * nn * nn - nn * nn * nn / 3.0) + 16.0 * nn * nn * nn / 3.0;
    }
  }
  tnsim_status s = put_descs(o, D, ng, second);
  if (s != TNSIM_OK) return s;
  GateDesc *ddev = o->at<GateDesc>(second ? o->L.desc2_off : o->L.desc_off);
  hipStream_t st = second ? o->stream2 : o->stream;
  {
    ProfScope p(h, TNSIM_K_OTHER, 0.0, 0.0, second);
    launch_setup_slots(st, ddev, ng, maxColsPad, 0);
  }
  {
    ProfScope p(h, TNSIM_K_THETA, theta_flop, theta_byte, second);
    launch_theta(st, ddev, ng, o->cfg.precision, maxM, maxChiR);
  }
  // QR preconditioning of the gates that take it: M = Q1 R1 (stage 0),
  // R1^H = Q2 R2 (stage 1), then the Jacobi matrix X = R2^H.  Panels are
  // factored one group of QG columns at a time (each panel's reflectors
  // applied inside the group), then the group's reflectors update the rest
  // of the matrix in one pass.
  const int qrGroups = (qrN + QG - 1) / QG;
  if (qrN > 0) {
    ProfScope p(h, TNSIM_K_QR, qr_flop, 0.0, second);
    for (int stage = 0; stage < 2; stage++) {
      for (int grp = 0; grp < qrGroups; grp++) {
        const int gend = (grp + 1) * QG;
        for (int pnl = grp * (QG / QNB); pnl < (grp + 1) * (QG / QNB) && pnl * QNB < qrN; pnl++) {
          launch_qr_panel(st, ddev, ng, stage, pnl);
          launch_qr_update(st, ddev, ng, stage, pnl, gend, gend - (pnl + 1) * QNB);
        }
        launch_qr_tgroup(st, ddev, ng, stage, grp);
        launch_qr_update_group(st, ddev, ng, stage, grp, 0, qrN - gend, stage ? qrN : qrMr);
      }
      if (stage == 0) launch_qr_r1h(st, ddev, ng, qrN);
    }
    launch_qr_r2h(st, ddev, ng, qrN);
  }
  {
    ProfScope p(h, TNSIM_K_COLNORM, 0.0, colnorm_byte, second);
    launch_colnorm(st, ddev, ng, maxColsPad);
  }
  {
    ProfScope p(h, TNSIM_K_OTHER, 0.0, 0.0, second);
    launch_gate_init(st, ddev, ng);
  }
  LAUNCHCHK(h, "theta");
  return TNSIM_OK;
}

// Jacobi sweeps over a changing set of gates.  A plan covers only the gates
// still sweeping (their descriptors packed at the front of the descriptor
// array); the row dimension of the pair Grams (K-split) and of the rotations
// is cut finer when those gates alone cannot fill the GPU.
struct SweepRunner {
  tnsim_mps o;
  struct Plan {
    int na = 0, maxPairs = 0, maxNblk = 0, maxRows = 0, maxMtrans = 0, ksplit = 1, rotRows = 256;
  } P;

  tnsim_status plan(const std::vector<const GateDesc *> &D, const std::vector<tnsim_mps> &hs) {
    P = Plan{};
    P.na = (int)D.size();
    for (const GateDesc *d : D) {
      P.maxPairs = std::max(P.maxPairs, d->nblk / 2);
      P.maxNblk = std::max(P.maxNblk, d->nblk);
      P.maxRows = std::max(P.maxRows, d->rows);
      if (d->trans) P.maxMtrans = std::max(P.maxMtrans, d->m);
    }
    const int pairs = P.na * P.maxPairs;
    const int tuned_ks = o->tune_gram_ks[tune_bucket(pairs)];
    int ks = tuned_ks > 0 ? tuned_ks : (o->gram_wg_target + pairs - 1) / pairs;
    ks = std::min(ks, KSPLIT_MAX);
    ks = std::min(ks, std::max(1, (P.maxRows + 31) / 32));
    // each gate's partials go to its handle's pool, at its position among the
    // active gates of that handle
    std::vector<int> pos(D.size());
    for (size_t a = 0; a < D.size(); a++) {
      int p = 0;
      for (size_t b = 0; b < a; b++) p += hs[b] == hs[a];
      pos[a] = p;
      const Layout &L = hs[a]->L;
      ks = std::min(ks, std::max(1, L.gp_blocks / ((p + 1) * L.npairs_max)));
    }
    P.ksplit = std::max(ks, 1);
    const int rchunks = std::max(1, P.maxRows + P.maxMtrans);
    const int tuned = o->tune_rot_rows[tune_bucket(pairs)];
    if (tuned > 0) {
      P.rotRows = tuned;
    } else {
      while (P.rotRows > 64 && (long long)pairs * ((rchunks + P.rotRows - 1) / P.rotRows) < 1024)
        P.rotRows /= 2;
    }
    std::vector<GateDesc> stage(D.size());
    for (size_t a = 0; a < D.size(); a++) {
      stage[a] = *D[a];
      stage[a].Gp = hs[a]->at<double2>(hs[a]->L.gp_off) +
                    (size_t)pos[a] * P.ksplit * hs[a]->L.npairs_max * PW * PW;
      stage[a].rotRows = P.rotRows;
    }
    return put_descs(o, stage.data(), P.na);
  }

  // Every round of the round-robin tournament, then the scalars gathered for
  // the host's convergence test.
  void enqueue() {
    tnsim_mps h = o;
    hipStream_t st = o->stream;
    GateDesc *ddev = o->at<GateDesc>(o->L.desc_off);
    {
      ProfScope p(h, TNSIM_K_OTHER);
      launch_begin_sweep(st, ddev, P.na);
    }
    for (int r = 0; r < P.maxNblk - 1; r++) {
      {
        ProfScope p(h, TNSIM_K_GRAM);
        launch_gram(st, ddev, P.na, r, P.maxPairs, P.ksplit);
      }
      {
        ProfScope p(h, TNSIM_K_EIG);
        launch_eig(st, ddev, P.na, r, P.maxPairs, P.ksplit);
      }
      {
        ProfScope p(h, TNSIM_K_ROT);
        launch_rot(st, ddev, P.na, r, P.maxPairs, P.maxRows, P.maxMtrans, P.rotRows);
      }
    }
    launch_gather_sc(st, ddev, P.na, o->at<SlotScalars>(o->L.scg_off));
  }

  // With a non-default stream and profiling off, the sweep of a plan shape
  // is captured once as a HIP graph and replayed.
  tnsim_status graph() {
    tnsim_mps h = o;
    hipStream_t st = o->stream;
    const long long key[7] = {P.na, P.maxPairs, P.ksplit, P.maxNblk, P.maxRows, P.maxMtrans,
                              P.rotRows};
    if (h->sweep_exec && memcmp(key, h->sweep_key, sizeof key) == 0) return TNSIM_OK;
    if (h->sweep_exec) {
      hipGraphExecDestroy(h->sweep_exec);
      h->sweep_exec = nullptr;
    }
    hipGraph_t g = nullptr;
    HIPCHK(h, hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed));
    enqueue();
    hipError_t e1 = hipGetLastError();
    hipError_t e2 = hipStreamEndCapture(st, &g);
    if (e1 != hipSuccess) return fail(h, e1, "sweep capture");
    if (e2 != hipSuccess) return fail(h, e2, "hipStreamEndCapture");
    hipError_t e3 = hipGraphInstantiate(&h->sweep_exec, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e3 != hipSuccess) {
      h->sweep_exec = nullptr;
      return fail(h, e3, "hipGraphInstantiate");
    }
    memcpy(h->sweep_key, key, sizeof key);
    return TNSIM_OK;
  }

  // Enqueue one sweep of the current plan and the copy of its gathered
  // scalars into pinned buffer `buf`, marked by event ev_sw[buf].  Nothing
  // waits: the host can enqueue the next sweep before reading this one.
  tnsim_status launch(int buf) {
    tnsim_mps h = o;
    hipStream_t st = o->stream;
    if (!h->ev_sw[buf]) HIPCHK(h, hipEventCreateWithFlags(&h->ev_sw[buf], hipEventDisableTiming));
    if (h->graphs && !h->prof && st != nullptr) {
      tnsim_status gs = graph();
      if (gs != TNSIM_OK) return gs;
      HIPCHK(h, hipGraphLaunch(h->sweep_exec, st));
    } else {
      enqueue();
    }
    LAUNCHCHK(h, "jacobi round");
    HIPCHK(h, hipMemcpyAsync(pin_scalars(o, buf), o->at<SlotScalars>(o->L.scg_off),
                             sizeof(SlotScalars) * P.na, hipMemcpyDeviceToHost, st));
    HIPCHK(h, hipEventRecord(h->ev_sw[buf], st));
    return TNSIM_OK;
  }

  // Wait for the sweep launched into `buf` (`na` gates planned then);
  // rot[a] = some pair of planned gate a rotated in that sweep.
  tnsim_status collect(int buf, int na, std::vector<char> &rot) {
    tnsim_mps h = o;
    HIPCHK(h, hipEventSynchronize(h->ev_sw[buf]));
    if (h->prof) {  // only one sweep is ever in flight while profiling
      HIPCHK(h, hipStreamSynchronize(o->stream));
      prof_drain(h);
    }
    const SlotScalars *sc_pin = pin_scalars(o, buf);
    rot.assign(na, 0);
    for (int a = 0; a < na; a++) rot[a] = sc_pin[a].rot != 0;
    return TNSIM_OK;
  }

  // One sweep of the current plan, waited for.
  tnsim_status run(std::vector<char> &rot) {
    tnsim_status s = launch(0);
    if (s != TNSIM_OK) return s;
    return collect(0, P.na, rot);
  }
};

// Record a finished (or failed) gate in its handle's statistics.
void record_gate(const BatchItem &it, const GateDesc &d, int k, int sweeps) {
  tnsim_mps hg = it.h;
  hg->last_sweeps = std::max(hg->last_sweeps, sweeps);
  hg->last_batch.insert(hg->last_batch.end(), {d.i, d.chiL, d.chiM, d.chiR, k, sweeps});
  hg->sw_gates += 1;
  hg->sw_sum += sweeps;
  hg->sw_max = std::max(hg->sw_max, sweeps);
}

// Everything after convergence: norms, sort and truncation, U_k, the
// write-back; updates each handle's bond dimensions and statistics.
tnsim_status gates_finish(tnsim_mps o, const BatchItem *items, const GateDesc *D,
                          const int *sweeps, int ng) {
  tnsim_mps h = o;
  hipStream_t st = o->stream;
  int maxM = 0, maxN = 0, maxColsPad = 0, qrN = 0;
  double colnorm_byte = 0.0;
  for (int g = 0; g < ng; g++) {
    maxM = std::max(maxM, D[g].m);
    maxN = std::max(maxN, D[g].n);
    maxColsPad = std::max(maxColsPad, D[g].colsPad);
    colnorm_byte += 16.0 * D[g].rows * D[g].cols;
    if (D[g].qr) qrN = std::max(qrN, D[g].n);
  }
  tnsim_status s = put_descs(o, D, ng);
  if (s != TNSIM_OK) return s;
  GateDesc *ddev = o->at<GateDesc>(o->L.desc_off);
  SlotScalars *scg = o->at<SlotScalars>(o->L.scg_off);
  {
    ProfScope p(h, TNSIM_K_COLNORM, 0.0, colnorm_byte);
    launch_colnorm(st, ddev, ng, maxColsPad);
  }
  {
    ProfScope p(h, TNSIM_K_TRUNC);
    launch_trunc(st, ddev, ng);
  }
  launch_gather_sc(st, ddev, ng, scg);
  LAUNCHCHK(h, "truncate");
  SlotScalars *sc_pin = pin_scalars(o);
  HIPCHK(h, hipMemcpyAsync(sc_pin, scg, sizeof(SlotScalars) * ng, hipMemcpyDeviceToHost, st));
  HIPCHK(h, hipStreamSynchronize(st));
  prof_drain(h);
  int maxK = 0, qrK = 0, qrM = 0;
  double wbl_byte = 0.0, wbr_flop = 0.0, wbr_byte = 0.0, qa_flop = 0.0;
  for (int g = 0; g < ng; g++) {
    const SlotScalars &sv = sc_pin[g];
    const GateDesc &d = D[g];
    tnsim_mps hg = items[g].h;
    const int fl = items[g].p->flags;
    hg->dims[d.i + 1] = sv.k;
    if (!(fl & PEND_NO_STATS)) {
      hg->sum_eps += sv.eps;
      hg->prod_keep *= (1.0 - sv.eps);
      if (!(fl & PEND_EPS_ONLY)) {
        record_gate(items[g], d, sv.k, sweeps[g]);
        hg->n2q += 1;
      }
    }
    maxK = std::max(maxK, sv.k);
    const double eb = d.storage == 0 ? 16.0 : 8.0, tb = d.tfp32 ? 8.0 : 16.0;
    wbl_byte += (16.0 + eb) * d.m * sv.k;
    wbr_flop += 8.0 * sv.k * d.m * d.n;
    wbr_byte += 16.0 * d.m * sv.k + tb * (double)d.m * d.n + eb * (double)sv.k * d.n;
    if (d.qr) {
      qrK = std::max(qrK, sv.k);
      qrM = std::max(qrM, d.m);
      qa_flop += 8.0 * (2.0 * d.m * d.n - (double)d.n * d.n) * sv.k;
    }
  }
  // U_k = Q1 [W_k; 0] for the QR-preconditioned gates: the groups'
  // reflectors in reverse order
  if (qrK > 0) {
    ProfScope p(h, TNSIM_K_QR, qa_flop, 0.0);
    launch_qr_gather(st, ddev, ng, qrM, qrK);
    for (int grp = (qrN + QG - 1) / QG - 1; grp >= 0; grp--)
      launch_qr_update_group(st, ddev, ng, 0, grp, 1, qrK, qrM);
    LAUNCHCHK(h, "qr apply");
  }
  {
    ProfScope p(h, TNSIM_K_WB_LEFT, 0.0, wbl_byte);
    launch_wb_left(st, ddev, ng, maxM, maxK);
  }
  {
    ProfScope p(h, TNSIM_K_WB_RIGHT, wbr_flop, wbr_byte);
    launch_wb_right(st, ddev, ng, o->cfg.precision, maxK, maxN);
  }
  LAUNCHCHK(h, "write-back");
  return TNSIM_OK;
}

// Run a batch of two-qubit gates (possibly of several handles) through the
// whole path in the same launches.  `o` owns the descriptors, the stream and
// the profiling; every gate works in its own handle's state and slot.
tnsim_status run_2q_items(tnsim_mps o, const BatchItem *items, int ng, bool force_trans) {
  std::vector<GateDesc> D(ng);
  for (int g = 0; g < ng; g++) D[g] = make_desc(o, items[g], force_trans);
  tnsim_status s = gates_prepare(o, D.data(), ng);
  if (s != TNSIM_OK) return s;

  const int max_sweeps = o->cfg.jacobi_max_sweeps > 0 ? o->cfg.jacobi_max_sweeps : 60;
  std::vector<int> done_at(ng, 0), act(ng);
  for (int g = 0; g < ng; g++) act[g] = g;
  SweepRunner sw{o};
  auto replan = [&]() {
    std::vector<const GateDesc *> pd;
    std::vector<tnsim_mps> hs;
    for (int g : act) {
      pd.push_back(&D[g]);
      hs.push_back(items[g].h);
    }
    return sw.plan(pd, hs);
  };
  s = replan();
  if (s != TNSIM_OK) return s;
  bool converged = false;
  int sweeps = 0;
  std::vector<char> rot;
  // Sweep s + 1 is enqueued before the host reads sweep s, so the host's
  // convergence test and the next launch overlap the GPU's work.  A gate
  // whose sweep rotated nothing is switched off on the device at the start
  // of the next sweep (k_begin_sweep), so a sweep enqueued after the last
  // one it needed leaves it unchanged and costs only early-exiting
  // workgroups.  Speculation is off while profiling (one sweep in flight).
  const bool spec = o->speculate && !o->prof;
  std::vector<int> act_at[2];
  int buf = 0;
  s = sw.launch(buf);
  if (s != TNSIM_OK) return s;
  act_at[buf] = act;
  for (int sweep = 1; sweep <= max_sweeps; sweep++) {
    if (spec && sweep < max_sweeps) {
      s = sw.launch(buf ^ 1);
      if (s != TNSIM_OK) return s;
      act_at[buf ^ 1] = act;
    }
    s = sw.collect(buf, (int)act_at[buf].size(), rot);
    if (s != TNSIM_OK) return s;
    sweeps = sweep;
    std::vector<int> still;
    for (size_t a = 0; a < act_at[buf].size(); a++) {
      const int g = act_at[buf][a];
      if (rot[a])
        still.push_back(g);
      else if (!done_at[g])
        done_at[g] = sweep;
    }
    if (still.empty()) {
      converged = true;
      break;
    }
    // re-plan once the active set has shrunk by a quarter (a converged gate
    // left in the plan only costs early-exiting workgroups); the new plan
    // takes effect from the next sweep launched
    if (4 * (int)still.size() <= 3 * (int)act.size()) {
      act.swap(still);
      s = replan();
      if (s != TNSIM_OK) return s;
    }
    if (spec) {
      buf ^= 1;
    } else if (sweep < max_sweeps) {
      s = sw.launch(buf);
      if (s != TNSIM_OK) return s;
      act_at[buf] = act;
    }
  }
  std::vector<int> swp(ng);
  for (int g = 0; g < ng; g++) swp[g] = done_at[g] ? done_at[g] : sweeps;
  if (!converged) {
    for (int g = 0; g < ng; g++) record_gate(items[g], D[g], 0, swp[g]);
    o->err = "Jacobi SVD did not converge within jacobi_max_sweeps";
    return TNSIM_E_NOCONV;
  }
  return gates_finish(o, items, D.data(), swp.data(), ng);
}


tnsim_status run_2q_batch(tnsim_mps h, const Pending *gates, int ng, bool force_trans = false) {
  std::vector<BatchItem> items(ng);
  for (int g = 0; g < ng; g++) items[g] = BatchItem{h, g, &gates[g]};
  return run_2q_items(h, items.data(), ng, force_trans);
}

tnsim_status run_2q(tnsim_mps h, const std::vector<Pending> &gs) {
  const int ns = h->L.nslots;
  for (size_t b = 0; b < gs.size(); b += ns) {
    int ng = (int)std::min<size_t>(ns, gs.size() - b);
    tnsim_status s = run_2q_batch(h, gs.data() + b, ng);
    if (s != TNSIM_OK) return s;
  }
  return TNSIM_OK;
}

// One canonicalisation pass (Sec. IV.A: the state is brought to canonical
// form before sampling), through the two-site path with the identity gate:
//  1. left to right, q = 0 .. n-2: theta = A_q A_{q+1} decomposed without the
//     Schmidt weight and without truncation: A_q <- U_k (left-canonical),
//     A_{q+1} <- U_k^H theta / N, so sites 0 .. n-2 end left-canonical and
//     the state normalised;
//  2. right to left, b = n-2 .. 0: theta = A_b A_{b+1} weighted by
//     lambda_{b+1}, which the previous step has just made the Schmidt
//     values of bond b+1 (1 at the right end), while sites 0 .. b form an
//     orthonormal left basis: the SVD is the Schmidt decomposition of bond
//     b, so lambda_b <- sigma / N, A_b <- U_k, A_{b+1} <- U_k^H theta / N.
// With `truncate`, step 2 applies the handle's chi_max and cutoff.
tnsim_status canonical_pass(tnsim_mps h, bool truncate) {
  const int n = h->L.n;
  Pending p{};
  for (int e = 0; e < 4; e++) p.g[5 * e] = make_double2(1.0, 0.0);
  for (int q = 0; q + 1 < n; q++) {
    p.i = q;
    p.flags = PEND_UNWEIGHTED | PEND_NO_CUT | PEND_NO_STATS;
    tnsim_status s = run_2q_batch(h, &p, 1);
    if (s != TNSIM_OK) return s;
  }
  for (int b = n - 2; b >= 0; b--) {
    p.i = b;
    p.flags = truncate ? PEND_EPS_ONLY : (PEND_NO_CUT | PEND_NO_STATS);
    tnsim_status s = run_2q_batch(h, &p, 1);
    if (s != TNSIM_OK) return s;
  }
  return TNSIM_OK;
}

tnsim_status run_1q(tnsim_mps h, const std::vector<std::pair<int, const tnsim_c128 *>> &gs) {
  if (gs.empty()) return TNSIM_OK;
  std::vector<Gate1Desc> D(gs.size());
  int maxe = 0;
  for (size_t k = 0; k < gs.size(); k++) {
    Gate1Desc &d = D[k];
    memset(&d, 0, sizeof d);
    int q = gs[k].first;
    d.A = h->site(q);
    d.chiL = h->dims[q];
    d.chiR = h->dims[q + 1];
    d.storage = h->L.storage;
    for (int e = 0; e < 4; e++) d.u[e] = to_d2(gs[k].second[e]);
    maxe = std::max(maxe, d.chiL * d.chiR);
  }
  Gate1Desc *ddev = h->at<Gate1Desc>(h->L.d1_off);
  HIPCHK(h, hipStreamSynchronize(h->stream));
  prof_drain(h);
  memcpy(h->pin, D.data(), sizeof(Gate1Desc) * D.size());
  HIPCHK(h, hipMemcpyAsync(ddev, h->pin, sizeof(Gate1Desc) * D.size(), hipMemcpyHostToDevice,
                           h->stream));
  double by = 0.0;
  for (auto &d : D) by += 2.0 * (h->L.storage == 0 ? 16.0 : 8.0) * 2.0 * d.chiL * d.chiR;
  {
    ProfScope p(h, TNSIM_K_1Q, 0.0, by);
    launch_apply_1q(h->stream, ddev, (int)D.size(), maxe);
  }
  LAUNCHCHK(h, "apply_1q");
  return TNSIM_OK;
}

void orient(int q0, int q1, const tnsim_c128 *g, Pending &p) {
  if (q1 == q0 + 1) {
    p.i = q0;
    for (int e = 0; e < 16; e++) p.g[e] = to_d2(g[e]);
  } else {
    // SWAP G SWAP: G'[2s'+t', 2s+t] = G[2t'+s', 2t+s]
    p.i = q1;
    for (int sp = 0; sp < 2; sp++)
      for (int tp = 0; tp < 2; tp++)
        for (int s = 0; s < 2; s++)
          for (int t = 0; t < 2; t++)
            p.g[(2 * sp + tp) * 4 + 2 * s + t] = to_d2(g[(2 * tp + sp) * 4 + 2 * t + s]);
  }
}

// A gate on distant qubits as local gates (Sec. IV.A): SWAP gates bring the
// qubit with the larger index next to the other one, the gate acts there, and
// the SWAPs are undone in reverse order.  Local and one-qubit gates pass
// through unchanged.
void expand_gate(const tnsim_gate &g, std::vector<tnsim_gate> &out) {
  if (g.q1 < 0 || std::abs(g.q0 - g.q1) == 1) {
    out.push_back(g);
    return;
  }
  tnsim_gate sw;
  memset(&sw, 0, sizeof sw);
  for (int s = 0; s < 2; s++)
    for (int t = 0; t < 2; t++) sw.m[(2 * t + s) * 4 + 2 * s + t].re = 1.0;
  const int a = std::min(g.q0, g.q1), b = std::max(g.q0, g.q1);
  for (int j = b - 1; j > a; j--) {
    sw.q0 = j;
    sw.q1 = j + 1;
    out.push_back(sw);
  }
  tnsim_gate moved = g;  // the qubit from b now sits at a + 1
  moved.q0 = g.q0 == a ? a : a + 1;
  moved.q1 = g.q0 == a ? a + 1 : a;
  out.push_back(moved);
  for (int j = a + 1; j < b; j++) {
    sw.q0 = j;
    sw.q1 = j + 1;
    out.push_back(sw);
  }
}

// Gate matrices must be finite: a NaN or infinity would reach the SVD.
bool finite_gate(const tnsim_c128 *m, int count) {
  for (int k = 0; k < count; k++)
    if (!std::isfinite(m[k].re) || !std::isfinite(m[k].im)) return false;
  return true;
}
bool finite_gate(const tnsim_gate &g) { return finite_gate(g.m, g.q1 < 0 ? 4 : 16); }

// Validate a layer; fills 1q and 2q lists.
tnsim_status validate_layer(tnsim_mps h, const tnsim_gate *gates, int ng,
                            std::vector<std::pair<int, const tnsim_c128 *>> &g1,
                            std::vector<Pending> &g2) {
  const int n = h->L.n;
  if (ng < 0 || (ng > 0 && !gates)) return TNSIM_E_ARG;
  std::vector<char> used(n, 0);
  for (int k = 0; k < ng; k++) {
    int a = gates[k].q0, b = gates[k].q1;
    if (a < 0 || a >= n || b < -1 || b >= n || a == b || !finite_gate(gates[k])) return TNSIM_E_ARG;
    if (b >= 0 && std::abs(a - b) != 1) return TNSIM_E_NONLOCAL;
    if (used[a] || (b >= 0 && used[b])) return TNSIM_E_OVERLAP;
    used[a] = 1;
    if (b >= 0) used[b] = 1;
  }
  for (int k = 0; k < ng; k++) {
    if (gates[k].q1 < 0) {
      g1.push_back({gates[k].q0, gates[k].m});
    } else {
      Pending p;
      orient(gates[k].q0, gates[k].q1, gates[k].m, p);
      g2.push_back(p);
    }
  }
  return TNSIM_OK;
}

// Dependency-driven execution of a circuit of local gates on one handle.
// A gate depends on the previous gate on each of its sites (a two-qubit gate
// on (i, i+1) also reads lambda_{i+1} and the bond dimensions around it, but
// every gate that writes those shares a site with it), so the results equal
// those of applying the gates in order.  Two-qubit gates whose predecessors
// are done are admitted into free workspace slots and prepared together; all
// gates in flight share each Jacobi sweep; a gate that converges is truncated
// and written back at once, which releases its successors.  Gates of
// consecutive layers thus overlap: the next layer's gates fill the sweeps in
// which the last gates of a layer converge.  Ready gates are admitted in
// groups (admit_group, or fewer when little is in flight), and a group
// admitted while others sweep is prepared on the second stream.

// The second stream of the scheduler, its events and staging buffer, made on
// first use (default priority, like every stream here).
tnsim_status ensure_stream2(tnsim_mps h) {
  if (h->stream2) return TNSIM_OK;
  HIPCHK(h, hipHostMalloc((void **)&h->pin2, h->pin_bytes, hipHostMallocDefault));
  HIPCHK(h, hipEventCreateWithFlags(&h->ev_main, hipEventDisableTiming));
  HIPCHK(h, hipEventCreateWithFlags(&h->ev_prep, hipEventDisableTiming));
  HIPCHK(h, hipStreamCreateWithFlags(&h->stream2, hipStreamNonBlocking));
  return TNSIM_OK;
}

tnsim_status run_circuit_impl(tnsim_mps h, const tnsim_gate *gates, int ng);

tnsim_status run_circuit(tnsim_mps h, const tnsim_gate *gates, int ng) {
  tnsim_status s = run_circuit_impl(h, gates, ng);
  // no preparation may outlive the call, whatever its outcome
  if (h->stream2 && hipStreamSynchronize(h->stream2) != hipSuccess && s == TNSIM_OK)
    s = fail(h, hipErrorUnknown, "second stream");
  prof_drain(h, true);
  return s;
}

tnsim_status run_circuit_impl(tnsim_mps h, const tnsim_gate *gates, int ng) {
  struct Op {
    int kind = 0;  // 1 or 2 qubits
    int q = 0;     // site (1q)
    Pending p{};   // oriented gate (2q)
    const tnsim_c128 *m = nullptr;
    int npred = 0;
    std::vector<int> succ;
  };
  const int n = h->L.n;
  std::vector<Op> ops(ng);
  std::vector<int> last(n, -1);
  for (int k = 0; k < ng; k++) {
    Op &op = ops[k];
    int sites[2], ns = 1;
    if (gates[k].q1 < 0) {
      op.kind = 1;
      op.q = gates[k].q0;
      op.m = gates[k].m;
      sites[0] = op.q;
    } else {
      op.kind = 2;
      orient(gates[k].q0, gates[k].q1, gates[k].m, op.p);
      sites[0] = op.p.i;
      sites[1] = op.p.i + 1;
      ns = 2;
    }
    int prev[2] = {-1, -1};
    for (int e = 0; e < ns; e++) {
      const int j = last[sites[e]];
      if (j >= 0 && j != prev[0]) {
        ops[j].succ.push_back(k);
        op.npred++;
        prev[e] = j;
      }
      last[sites[e]] = k;
    }
  }
  std::vector<int> ready1, ready2;  // kept in circuit order
  for (int k = 0; k < ng; k++)
    if (ops[k].npred == 0) (ops[k].kind == 1 ? ready1 : ready2).push_back(k);
  auto release = [&](int k) {
    for (int j : ops[k].succ)
      if (--ops[j].npred == 0) {
        auto &r = ops[j].kind == 1 ? ready1 : ready2;
        r.insert(std::upper_bound(r.begin(), r.end(), j), j);
      }
  };

  struct Flight {
    BatchItem it;
    GateDesc d;
    int op, sweeps;
  };
  std::vector<Flight> fl;
  std::vector<int> free_slots;
  for (int sl = h->L.nslots - 1; sl >= 0; sl--) free_slots.push_back(sl);
  const int max_sweeps = h->cfg.jacobi_max_sweeps > 0 ? h->cfg.jacobi_max_sweeps : 60;
  SweepRunner sw{h};
  bool dirty = true;
  std::vector<char> rot;
  // gates admitted while others sweep are prepared on the second stream and
  // join the sweeps once their preparation has finished
  if (h->overlap_prepare) {
    tnsim_status s = ensure_stream2(h);
    if (s != TNSIM_OK) return s;
  }
  std::vector<Flight> prep;
  auto join = [&]() -> tnsim_status {
    HIPCHK(h, hipStreamWaitEvent(h->stream, h->ev_prep, 0));
    for (const Flight &f : prep) fl.push_back(f);
    prep.clear();
    dirty = true;
    return TNSIM_OK;
  };
  for (;;) {
    // one-qubit gates: all ready ones at once (they are on distinct sites)
    while (!ready1.empty()) {
      std::vector<std::pair<int, const tnsim_c128 *>> g1;
      std::vector<int> done = ready1;
      ready1.clear();
      for (int k : done) g1.push_back({ops[k].q, ops[k].m});
      tnsim_status s = run_1q(h, g1);
      if (s != TNSIM_OK) return s;
      for (int k : done) release(k);
    }
    // two-qubit gates into free slots, in groups: a preparation (merge and
    // QR) costs about the same latency for one gate as for many, so ready
    // gates wait until there are enough of them or the GPU runs short of work
    std::vector<GateDesc> nd;
    std::vector<Flight> nf;
    size_t taken = 0;
    const bool admit = prep.empty() &&
                       ((int)ready2.size() >= h->admit_group || (int)fl.size() < h->admit_group);
    for (; admit && taken < ready2.size() && !free_slots.empty(); taken++) {
      const int k = ready2[taken];
      BatchItem it{h, free_slots.back(), &ops[k].p};
      free_slots.pop_back();
      nd.push_back(make_desc(h, it, false));
      nf.push_back(Flight{it, nd.back(), k, 0});
    }
    ready2.erase(ready2.begin(), ready2.begin() + taken);
    if (!nd.empty()) {
      if (h->overlap_prepare && !fl.empty()) {
        // after everything issued so far (the predecessors' write-backs)
        HIPCHK(h, hipEventRecord(h->ev_main, h->stream));
        HIPCHK(h, hipStreamWaitEvent(h->stream2, h->ev_main, 0));
        tnsim_status s = gates_prepare(h, nd.data(), (int)nd.size(), true);
        if (s != TNSIM_OK) return s;
        HIPCHK(h, hipEventRecord(h->ev_prep, h->stream2));
        prep = nf;
      } else {
        tnsim_status s = gates_prepare(h, nd.data(), (int)nd.size());
        if (s != TNSIM_OK) return s;
        for (const Flight &f : nf) fl.push_back(f);
        dirty = true;
      }
    }
    if (fl.empty()) {
      if (!prep.empty()) {  // nothing to sweep meanwhile
        tnsim_status s = join();
        if (s != TNSIM_OK) return s;
        continue;
      }
      if (ready1.empty() && ready2.empty()) break;
      continue;
    }
    // one Jacobi sweep over every gate in flight
    if (dirty) {
      std::vector<const GateDesc *> pd;
      std::vector<tnsim_mps> hs;
      for (const Flight &f : fl) {
        pd.push_back(&f.d);
        hs.push_back(h);
      }
      tnsim_status s = sw.plan(pd, hs);
      if (s != TNSIM_OK) return s;
      dirty = false;
    }
    tnsim_status s = sw.run(rot);
    if (s != TNSIM_OK) return s;
    std::vector<Flight> keep, fin;
    for (size_t a = 0; a < fl.size(); a++) {
      fl[a].sweeps++;
      if (!rot[a])
        fin.push_back(fl[a]);
      else if (fl[a].sweeps >= max_sweeps) {
        record_gate(fl[a].it, fl[a].d, 0, fl[a].sweeps);
        h->err = "Jacobi SVD did not converge within jacobi_max_sweeps";
        return TNSIM_E_NOCONV;
      } else
        keep.push_back(fl[a]);
    }
    if (!fin.empty()) {
      std::vector<BatchItem> fi;
      std::vector<GateDesc> fd;
      std::vector<int> fs;
      for (const Flight &f : fin) {
        fi.push_back(f.it);
        fd.push_back(f.d);
        fs.push_back(f.sweeps);
      }
      s = gates_finish(h, fi.data(), fd.data(), fs.data(), (int)fin.size());
      if (s != TNSIM_OK) return s;
      for (const Flight &f : fin) {
        free_slots.push_back(f.it.slot);
        release(f.op);
      }
      fl.swap(keep);
      dirty = true;
    }
    if (!prep.empty()) {
      const hipError_t q = hipEventQuery(h->ev_prep);
      if (q == hipSuccess) {
        s = join();
        if (s != TNSIM_OK) return s;
      } else if (q != hipErrorNotReady) {
        return fail(h, q, "hipEventQuery");
      }
    }
  }
  return TNSIM_OK;
}

// <bra| P |ket>; P holds a 2x2 per site (4n entries) and isI marks identity
// sites; P == nullptr means identity everywhere.
tnsim_status transfer(tnsim_mps h, tnsim_mps bra, tnsim_mps ket, const double2 *P,
                      const char *isI, double2 *out) {
  const Layout &L = h->L;
  hipStream_t st = h->stream;
  double2 *E = h->at<double2>(L.e0_off), *E2 = h->at<double2>(L.e1_off);
  double2 *F = h->at<double2>(L.f_off), *F2 = h->at<double2>(L.f2_off);
  double2 one = make_double2(1.0, 0.0);
  HIPCHK(h, hipStreamSynchronize(st));
  memcpy(h->pin, &one, sizeof one);
  HIPCHK(h, hipMemcpyAsync(E, h->pin, sizeof one, hipMemcpyHostToDevice, st));
  const int n = L.n;
  for (int q = 0; q < n; q++) {
    int lb = bra->dims[q], rb = bra->dims[q + 1];
    int lk = ket->dims[q], rk = ket->dims[q + 1];
    // F = E (lb x lk) * K (lk x 2rk), on the matrix cores
    launch_zgemm(st, ZGEMM_NN_ROW,
                 ZgemmArgs{lb, 2 * rk, lk, E, lk, ket->site(q), 2 * rk, F, 2 * rk, nullptr, 0}, 0,
                 ket->L.storage);
    const double2 *Fp = F;
    if (P && !isI[q]) {
      launch_pauli_phys(st, F, F2, lb, rk, P[4 * q], P[4 * q + 1], P[4 * q + 2], P[4 * q + 3]);
      Fp = F2;
    }
    // E' = B^H (rb x 2lb) * F (2lb x rk)
    launch_zgemm(st, ZGEMM_CN_ROW,
                 ZgemmArgs{rb, rk, 2 * lb, bra->site(q), rb, Fp, rk, E2, rk, nullptr, 0},
                 bra->L.storage, 0);
    LAUNCHCHK(h, "transfer");
    std::swap(E, E2);
  }
  HIPCHK(h, hipMemcpyAsync(h->pin, E, sizeof(double2), hipMemcpyDeviceToHost, st));
  HIPCHK(h, hipStreamSynchronize(st));
  memcpy(out, h->pin, sizeof(double2));
  return TNSIM_OK;
}

}  // namespace

// ============================================================== gradients
// Reverse-mode derivative of a Pauli-sum loss with respect to rotation angles.
// The forward pass checkpoints the state at segment starts; the backward pass
// walks the segments in reverse, recomputes each one from its checkpoint while
// recording every gate's inputs and SVD, and then runs the adjoint of each gate
// in reverse order.  All tensor arithmetic runs in the kernels of
// k_adjoint.hip and the forward kernels.

namespace {

constexpr double ADJ_ETA = 1e-24;  // Lorentzian broadening of 1/(lambda_j - lambda_l)

GradState grad_layout(const Layout &L, int n_seg, int max_seg, int n_params) {
  GradState G;
  const int n = L.n;
  const size_t elem = L.elem;
  int maxbond = 1;
  for (int b = 0; b < n - 1; b++) maxbond = std::max(maxbond, L.bondcap[b]);
  const size_t cmax = 2 * (size_t)maxbond;
  size_t off = 0;
  // one checkpoint
  size_t st = 0;
  G.st_site.resize(n);
  G.st_lam.resize(std::max(n - 1, 0));
  for (int q = 0; q < n; q++) {
    G.st_site[q] = st;
    st = align_up(st + L.site_cap[q] * elem);
  }
  for (int b = 0; b < n - 1; b++) {
    G.st_lam[b] = st;
    st = align_up(st + sizeof(double) * L.bondcap[b]);
  }
  G.state_bytes = st;
  G.ckpt0 = off;
  off = align_up(off + st * (n_seg + 1));
  G.cot_site.resize(n);
  for (int q = 0; q < n; q++) {
    G.cot_site[q] = off;
    off = align_up(off + L.site_cap[q] * sizeof(double2));
  }
  G.cot_lam.resize(std::max(n - 1, 0));
  for (int b = 0; b < n - 1; b++) {
    G.cot_lam[b] = off;
    off = align_up(off + sizeof(double) * L.bondcap[b]);
  }
  G.env_stride = align_up(sizeof(double2) * (size_t)maxbond * maxbond);
  G.envL = off;
  off += G.env_stride * (n + 1);
  G.envR = off;
  off += G.env_stride * (n + 1);
  G.envF = off;
  off = align_up(off + sizeof(double2) * (size_t)maxbond * 2 * maxbond);
  G.envF2 = off;
  off = align_up(off + sizeof(double2) * (size_t)maxbond * 2 * maxbond);
  G.tmp_stride = align_up(sizeof(double2) * cmax * cmax);
  G.tmp0 = off;
  off += G.tmp_stride * 12;
  G.lam2 = off;
  off = align_up(off + sizeof(double) * cmax);
  G.sbar = off;
  off = align_up(off + sizeof(double) * cmax);
  G.dots = off;
  off = align_up(off + 64);
  G.ubar = off;
  off = align_up(off + 64);
  G.grad = off;
  off = align_up(off + sizeof(double) * std::max(n_params, 1));
  // per-gate records
  const size_t site_max = (size_t)maxbond * 2 * maxbond;
  size_t r = 0;
  G.rec_a = r;
  r = align_up(r + site_max * elem);
  G.rec_b = r;
  r = align_up(r + site_max * elem);
  G.rec_lam = r;
  r = align_up(r + sizeof(double) * maxbond);
  G.rec_T = r;
  r = align_up(r + sizeof(double2) * cmax * cmax);
  G.rec_J = r;
  r = align_up(r + sizeof(double2) * cmax * cmax);
  G.rec_sig = r;
  r = align_up(r + sizeof(double) * cmax);
  G.rec_perm = r;
  r = align_up(r + sizeof(int) * cmax);
  G.rec_stride = r;
  G.rec0 = off;
  off = align_up(off + r * std::max(max_seg, 1));
  G.total = off;
  G.n = n;
  G.n_seg = n_seg;
  G.max_seg = max_seg;
  G.n_params = n_params;
  return G;
}

Mat4 rotation(int axis, double t) {
  const double c = cos(0.5 * t), sn = sin(0.5 * t);
  Mat4 u;
  // R_P(t) = cos(t/2) I - i sin(t/2) P
  if (axis == 0) {
    u.v[0] = make_double2(c, 0); u.v[1] = make_double2(0, -sn);
    u.v[2] = make_double2(0, -sn); u.v[3] = make_double2(c, 0);
  } else if (axis == 1) {
    u.v[0] = make_double2(c, 0); u.v[1] = make_double2(-sn, 0);
    u.v[2] = make_double2(sn, 0); u.v[3] = make_double2(c, 0);
  } else {
    u.v[0] = make_double2(c, -sn); u.v[1] = make_double2(0, 0);
    u.v[2] = make_double2(0, 0); u.v[3] = make_double2(c, sn);
  }
  return u;
}

GemmArgs gemm(int M, int N, int K, const void *A, long long sai, long long sak, int ac, int ast,
              const void *B, long long sbk, long long sbj, int bc, int bst, double2 *C,
              long long sci, long long scj, double2 alpha, int acc) {
  GemmArgs g;
  g.M = M; g.N = N; g.K = K;
  g.A = A; g.sa_i = sai; g.sa_k = sak; g.a_conj = ac; g.a_storage = ast;
  g.B = B; g.sb_k = sbk; g.sb_j = sbj; g.b_conj = bc; g.b_storage = bst;
  g.C = C; g.sc_i = sci; g.sc_j = scj; g.alpha = alpha; g.accumulate = acc;
  return g;
}

inline double2 cr(double x) { return make_double2(x, 0.0); }

tnsim_status save_ckpt(tnsim_mps h, int idx) {
  GradState &G = h->grad;
  char *base = G.ws + G.ckpt0 + G.state_bytes * idx;
  const int n = h->L.n;
  for (int q = 0; q < n; q++)
    HIPCHK(h, hipMemcpyAsync(base + G.st_site[q], h->site(q),
                             (size_t)h->dims[q] * 2 * h->dims[q + 1] * h->L.elem,
                             hipMemcpyDeviceToDevice, h->stream));
  for (int b = 0; b < n - 1; b++)
    HIPCHK(h, hipMemcpyAsync(base + G.st_lam[b], h->lam(b), sizeof(double) * h->dims[b + 1],
                             hipMemcpyDeviceToDevice, h->stream));
  G.ckpt_dims[idx] = h->dims;
  return TNSIM_OK;
}

tnsim_status restore_ckpt(tnsim_mps h, int idx) {
  GradState &G = h->grad;
  const char *base = G.ws + G.ckpt0 + G.state_bytes * idx;
  const int n = h->L.n;
  h->dims = G.ckpt_dims[idx];
  for (int q = 0; q < n; q++)
    HIPCHK(h, hipMemcpyAsync(h->site(q), base + G.st_site[q],
                             (size_t)h->dims[q] * 2 * h->dims[q + 1] * h->L.elem,
                             hipMemcpyDeviceToDevice, h->stream));
  for (int b = 0; b < n - 1; b++)
    HIPCHK(h, hipMemcpyAsync(h->lam(b), base + G.st_lam[b], sizeof(double) * h->dims[b + 1],
                             hipMemcpyDeviceToDevice, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  memcpy(h->pin, h->dims.data(), sizeof(int32_t) * (n + 1));
  HIPCHK(h, hipMemcpyAsync(h->dims_dev(), h->pin, sizeof(int32_t) * (n + 1),
                           hipMemcpyHostToDevice, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  return TNSIM_OK;
}

// Apply gate g of the stored circuit (forward).  With rec != nullptr the
// gate's inputs and SVD are recorded for the adjoint.
tnsim_status grad_apply(tnsim_mps h, int gi, GradRec *rec) {
  GradState &G = h->grad;
  const tnsim_gate &gt = G.gates[gi];
  hipStream_t st = h->stream;
  if (gt.q1 < 0) {
    const int q = gt.q0;
    Mat4 u;
    if (G.param[gi] >= 0)
      u = rotation(G.axis[gi], G.angles[G.param[gi]]);
    else
      for (int e = 0; e < 4; e++) u.v[e] = to_d2(gt.m[e]);
    if (rec) {
      rec->kind = 1;
      rec->q = q;
      rec->chiL = h->dims[q];
      rec->chiR = h->dims[q + 1];
      rec->param = G.param[gi];
      rec->axis = G.axis[gi];
      rec->u = u;
      HIPCHK(h, hipMemcpyAsync(G.ws + rec->off + G.rec_a, h->site(q),
                               (size_t)rec->chiL * 2 * rec->chiR * h->L.elem,
                               hipMemcpyDeviceToDevice, st));
    }
    tnsim_c128 um[4];
    for (int e = 0; e < 4; e++) um[e] = tnsim_c128{u.v[e].x, u.v[e].y};
    return run_1q(h, {{q, um}});
  }
  Pending p;
  orient(gt.q0, gt.q1, gt.m, p);
  const int i = p.i, n = h->L.n;
  if (rec) {
    rec->kind = 2;
    rec->q = i;
    rec->chiL = h->dims[i];
    rec->chiM = h->dims[i + 1];
    rec->chiR = h->dims[i + 2];
    rec->has_lam = (i + 1 <= n - 2);
    for (int e = 0; e < 16; e++) rec->g.v[e] = p.g[e];
    char *r = G.ws + rec->off;
    HIPCHK(h, hipMemcpyAsync(r + G.rec_a, h->site(i),
                             (size_t)rec->chiL * 2 * rec->chiM * h->L.elem,
                             hipMemcpyDeviceToDevice, st));
    HIPCHK(h, hipMemcpyAsync(r + G.rec_b, h->site(i + 1),
                             (size_t)rec->chiM * 2 * rec->chiR * h->L.elem,
                             hipMemcpyDeviceToDevice, st));
    if (rec->has_lam)
      HIPCHK(h, hipMemcpyAsync(r + G.rec_lam, h->lam(i + 1), sizeof(double) * rec->chiR,
                               hipMemcpyDeviceToDevice, st));
  }
  tnsim_status s = run_2q_batch(h, &p, 1, /*force_trans=*/true);
  if (s != TNSIM_OK) return s;
  if (rec) {
    const Layout &L = h->L;
    const SlotScalars *sc_pin = pin_scalars(h);
    rec->k = sc_pin[0].k;
    rec->N = sc_pin[0].N;
    const int m = 2 * rec->chiL, nn = 2 * rec->chiR, ldj = pad_to(m, 16);
    char *sl = h->slot(0), *r = G.ws + rec->off;
    HIPCHK(h, hipMemcpyAsync(r + G.rec_T, sl + L.t_off, sizeof(double2) * (size_t)m * nn,
                             hipMemcpyDeviceToDevice, st));
    HIPCHK(h, hipMemcpy2DAsync(r + G.rec_J, sizeof(double2) * m, sl + L.j_off,
                               sizeof(double2) * ldj, sizeof(double2) * m, m,
                               hipMemcpyDeviceToDevice, st));
    HIPCHK(h, hipMemcpyAsync(r + G.rec_sig, sl + L.sig_off, sizeof(double) * m,
                             hipMemcpyDeviceToDevice, st));
    launch_sort_all(st, (const double *)(sl + L.sig_off), m, (int *)(r + G.rec_perm));
    LAUNCHCHK(h, "record");
  }
  return TNSIM_OK;
}

// One left transfer step: E' (rb x rk) = B^H [P] (E (lb x lk) K) for site q.
void env_left(tnsim_mps h, int q, const double2 *E, double2 *Eo, const double2 *P) {
  GradState &G = h->grad;
  hipStream_t st = h->stream;
  const int lb = h->dims[q], rb = h->dims[q + 1], sto = h->L.storage;
  double2 *F = (double2 *)(G.ws + G.envF), *F2 = (double2 *)(G.ws + G.envF2);
  launch_gemm_gen(st, gemm(lb, 2 * rb, lb, E, lb, 1, 0, 0, h->site(q), 2 * rb, 1, 0, sto, F,
                           2 * rb, 1, cr(1.0), 0));
  const double2 *Fp = F;
  if (P) {
    launch_pauli_phys(st, F, F2, lb, rb, P[0], P[1], P[2], P[3]);
    Fp = F2;
  }
  launch_gemm_gen(st, gemm(rb, rb, 2 * lb, h->site(q), 1, rb, 1, sto, Fp, rb, 1, 0, 0, Eo, rb, 1,
                           cr(1.0), 0));
}

// One right transfer step: R' (lb x lb)[a, a'] = sum conj(A[a,s,b]) P[s,s'] A[a',s',b'] R[b,b'].
void env_right(tnsim_mps h, int q, const double2 *R, double2 *Ro, const double2 *P) {
  GradState &G = h->grad;
  hipStream_t st = h->stream;
  const int lb = h->dims[q], rb = h->dims[q + 1], sto = h->L.storage;
  double2 *F = (double2 *)(G.ws + G.envF), *F2 = (double2 *)(G.ws + G.envF2);
  // G1[(a',s'), b] = sum_b' A[(a',s'), b'] R[b, b']
  launch_gemm_gen(st, gemm(2 * lb, rb, rb, h->site(q), rb, 1, 0, sto, R, 1, rb, 0, 0, F, rb, 1,
                           cr(1.0), 0));
  const double2 *Fp = F;
  if (P) {
    launch_pauli_phys(st, F, F2, lb, rb, P[0], P[1], P[2], P[3]);
    Fp = F2;
  }
  // R'[a, a'] = sum_{(s,b)} conj(A[a, (s,b)]) G2[a', (s,b)]
  launch_gemm_gen(st, gemm(lb, lb, 2 * rb, h->site(q), 2 * rb, 1, 1, sto, Fp, 1, 2 * rb, 0, 0, Ro,
                           lb, 1, cr(1.0), 0));
}

// Abar_q += w * (d <psi|P|psi> / d conj(A_q)) for every site, P given per site
// (identity where isI).
tnsim_status loss_cotangent_term(tnsim_mps h, const double2 *tab, const char *isI, double w) {
  GradState &G = h->grad;
  hipStream_t st = h->stream;
  const int n = h->L.n, sto = h->L.storage;
  auto envL = [&](int q) { return (double2 *)(G.ws + G.envL + G.env_stride * q); };
  auto envR = [&](int q) { return (double2 *)(G.ws + G.envR + G.env_stride * q); };
  launch_fill_c(st, envL(0), 1, cr(1.0));
  for (int q = 0; q < n; q++) env_left(h, q, envL(q), envL(q + 1), isI[q] ? nullptr : tab + 4 * q);
  launch_fill_c(st, envR(n), 1, cr(1.0));
  for (int q = n - 1; q >= 0; q--)
    env_right(h, q, envR(q + 1), envR(q), isI[q] ? nullptr : tab + 4 * q);
  double2 *F = (double2 *)(G.ws + G.envF), *F2 = (double2 *)(G.ws + G.envF2);
  for (int q = 0; q < n; q++) {
    const int lb = h->dims[q], rb = h->dims[q + 1];
    launch_gemm_gen(st, gemm(lb, 2 * rb, lb, envL(q), lb, 1, 0, 0, h->site(q), 2 * rb, 1, 0, sto,
                             F, 2 * rb, 1, cr(1.0), 0));
    const double2 *Fp = F;
    if (!isI[q]) {
      const double2 *P = tab + 4 * q;
      launch_pauli_phys(st, F, F2, lb, rb, P[0], P[1], P[2], P[3]);
      Fp = F2;
    }
    double2 *Ab = (double2 *)(G.ws + G.cot_site[q]);
    // Abar[(a,s), b] += w sum_b' Fp[(a,s), b'] R[b, b']
    launch_gemm_gen(st, gemm(2 * lb, rb, rb, Fp, rb, 1, 0, 0, envR(q + 1), 1, rb, 0, 0, Ab, rb, 1,
                             cr(w), 1));
  }
  LAUNCHCHK(h, "loss cotangent");
  return TNSIM_OK;
}

// Adjoint of one recorded two-qubit gate: consumes the cotangents of
// (A_i', A_{i+1}', lambda_i') and produces those of (A_i, A_{i+1}) and the
// contribution to lambda_{i+1}.
tnsim_status adjoint_2q(tnsim_mps h, const GradRec &R) {
  GradState &G = h->grad;
  hipStream_t st = h->stream;
  const int i = R.q, chiL = R.chiL, chiM = R.chiM, chiR = R.chiR, k = R.k;
  const int m = 2 * chiL, n = 2 * chiR, sto = h->L.storage;
  const double N = R.N;
  const char *rb = G.ws + R.off;
  const double2 *T = (const double2 *)(rb + G.rec_T);
  const double2 *J = (const double2 *)(rb + G.rec_J);
  const double *sig = (const double *)(rb + G.rec_sig);
  const int *perm = (const int *)(rb + G.rec_perm);
  const double *lamR = R.has_lam ? (const double *)(rb + G.rec_lam) : nullptr;
  auto tmp = [&](int t) { return (double2 *)(G.ws + G.tmp0 + G.tmp_stride * t); };
  double2 *U = tmp(0), *Ub = tmp(1), *Tb = tmp(2), *Ap = tmp(3), *Cm = tmp(4), *Ab = tmp(5),
          *Y = tmp(6), *Hb = tmp(7), *Hs = tmp(8), *Mw = tmp(9), *Mb = tmp(10);
  double *lam2 = (double *)(G.ws + G.lam2), *sbar = (double *)(G.ws + G.sbar),
         *dots = (double *)(G.ws + G.dots);
  double2 *cotA = (double2 *)(G.ws + G.cot_site[i]);      // m x k  (A_i')
  double2 *cotB = (double2 *)(G.ws + G.cot_site[i + 1]);  // k x n  (A_{i+1}')
  double *lamb_i = (double *)(G.ws + G.cot_lam[i]);       // k      (lambda_i')
  double *lamb_r = R.has_lam ? (double *)(G.ws + G.cot_lam[i + 1]) : nullptr;

  // full left basis in descending order
  launch_gather_basis(st, J, m, perm, sig, U, lam2, m);
  // Ubar = Abar_i' + theta' Abar_{i+1}'^H / N        (m x k, row-major)
  HIPCHK(h, hipMemcpyAsync(Ub, cotA, sizeof(double2) * (size_t)m * k, hipMemcpyDeviceToDevice, st));
  launch_gemm_gen(st, gemm(m, k, n, T, n, 1, 0, 0, cotB, 1, n, 1, 0, Ub, k, 1, cr(1.0 / N), 1));
  // theta'_bar = U_k Abar_{i+1}' / N                   (m x n, row-major)
  launch_gemm_gen(st, gemm(m, n, k, U, 1, m, 0, 0, cotB, n, 1, 0, 0, Tb, n, 1, cr(1.0 / N), 0));
  // A_{i+1}' = U_k^H theta' / N (recomputed) and Re<Abar_{i+1}', A_{i+1}'>
  launch_gemm_gen(st, gemm(k, n, m, U, m, 1, 1, 0, T, n, 1, 0, 0, Ap, n, 1, cr(1.0 / N), 0));
  launch_fill_zero(st, dots, 64);
  launch_dot_re(st, cotB, Ap, 0, (size_t)k * n, dots);
  // sigma_bar from lambda' = sigma/N and N
  launch_sigma_bar(st, dots, lamb_i, lam2, N, k, sbar);
  // C = U^H Ubar (m x k col-major); Abar = F o C (+ diagonal sigma terms)
  launch_gemm_gen(st, gemm(m, k, m, U, m, 1, 1, 0, Ub, k, 1, 0, 0, Cm, 1, m, cr(1.0), 0));
  launch_svd_adj_mid(st, Cm, Ab, lam2, sbar, m, k, ADJ_ETA);
  // Hbar = U Abar U_k^H (m x m col-major), Hs = Hbar + Hbar^H
  launch_gemm_gen(st, gemm(m, k, m, U, 1, m, 0, 0, Ab, 1, m, 0, 0, Y, 1, m, cr(1.0), 0));
  launch_gemm_gen(st, gemm(m, m, k, Y, 1, m, 0, 0, U, m, 1, 1, 0, Hb, 1, m, cr(1.0), 0));
  launch_herm_sum(st, Hb, Hs, m);
  // Mbar = Hs M with M = theta' diag(lambda_{i+1})      (m x n row-major)
  launch_weight_apply(st, T, Mw, lamR, m, chiR);
  launch_gemm_gen(st, gemm(m, n, m, Hs, 1, m, 0, 0, Mw, n, 1, 0, 0, Mb, n, 1, cr(1.0), 0));
  // theta'_bar += Mbar diag(lambda); lambda_bar_{i+1} += 2 Re sum conj(Mbar) theta'
  launch_weight_adj(st, Mb, T, Tb, lamR, lamb_r, m, chiR);
  // theta_bar = G^H theta'_bar on (s, t)
  launch_gate_adj(st, Tb, chiL, chiR, R.g);
  // Abar_i = theta_bar A_{i+1}^H (m x chiM); Abar_{i+1} = A_i^H theta_bar (chiM x n)
  const void *A0 = rb + G.rec_a, *A1 = rb + G.rec_b;
  launch_gemm_gen(st, gemm(m, chiM, n, Tb, n, 1, 0, 0, A1, 1, n, 1, sto, cotA, chiM, 1, cr(1.0), 0));
  launch_gemm_gen(st, gemm(chiM, n, m, A0, 1, chiM, 1, sto, Tb, n, 1, 0, 0, cotB, n, 1, cr(1.0), 0));
  // the old lambda_i is overwritten by this gate: nothing later depends on it
  launch_fill_zero(st, lamb_i, align_up(sizeof(double) * h->L.bondcap[i], 16));
  LAUNCHCHK(h, "adjoint 2q");
  return TNSIM_OK;
}

tnsim_status adjoint_1q(tnsim_mps h, const GradRec &R) {
  GradState &G = h->grad;
  hipStream_t st = h->stream;
  double *ubar = (double *)(G.ws + G.ubar);
  launch_fill_zero(st, ubar, 64);
  launch_1q_adj(st, (double2 *)(G.ws + G.cot_site[R.q]), G.ws + R.off + G.rec_a, h->L.storage,
                R.chiL, R.chiR, R.u, ubar);
  if (R.param >= 0)
    launch_angle_grad(st, ubar, R.u, R.axis, (double *)(G.ws + G.grad) + R.param);
  LAUNCHCHK(h, "adjoint 1q");
  return TNSIM_OK;
}

tnsim_status pauli_table(const char *p, int n, std::vector<double2> &tab, std::vector<char> &isI) {
  static const double2 PM[4][4] = {{{1, 0}, {0, 0}, {0, 0}, {1, 0}},
                                   {{0, 0}, {1, 0}, {1, 0}, {0, 0}},
                                   {{0, 0}, {0, -1}, {0, 1}, {0, 0}},
                                   {{1, 0}, {0, 0}, {0, 0}, {-1, 0}}};
  tab.assign(4 * n, make_double2(0, 0));
  isI.assign(n, 1);
  for (int q = 0; q < n; q++) {
    int k;
    switch (p[q]) {
      case 'I': k = 0; break;
      case 'X': k = 1; break;
      case 'Y': k = 2; break;
      case 'Z': k = 3; break;
      default: return TNSIM_E_ARG;
    }
    isI[q] = k == 0;
    for (int e = 0; e < 4; e++) tab[4 * q + e] = PM[k][e];
  }
  return TNSIM_OK;
}

}  // namespace

// ============================================================== C ABI

extern "C" {

size_t tnsim_mps_arena_bytes(const tnsim_config *cfg) {
  if (!valid_config(cfg)) return 0;
  return make_layout(*cfg).total;
}

tnsim_status tnsim_mps_create(const tnsim_config *cfg, void *dev_arena, size_t arena_bytes,
                              void *hip_stream, tnsim_mps *out) {
  if (!out) return TNSIM_E_ARG;
  *out = nullptr;
  if (!valid_config(cfg) || !dev_arena) return TNSIM_E_ARG;
  Layout L = make_layout(*cfg);
  if (arena_bytes < L.total) return TNSIM_E_CAPACITY;
  if (reinterpret_cast<uintptr_t>(dev_arena) % ALIGN) return TNSIM_E_ARG;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    g_create_error = "no HIP device";
    return TNSIM_E_DEVICE;
  }
  tnsim_mps h = new tnsim_mps_s();
  h->cfg = *cfg;
  h->L = std::move(L);
  h->arena = (char *)dev_arena;
  h->arena_bytes = arena_bytes;
  h->stream = (hipStream_t)hip_stream;
  h->device = dev;
  if (const char *e = getenv("TNSIM_GRAPHS")) h->graphs = atoi(e) != 0;
  if (const char *e = getenv("TNSIM_PAIR_SKIP")) h->pair_skip = atoi(e) != 0;
  if (const char *e = getenv("TNSIM_GRAM_WG_TARGET")) {
    int v = atoi(e);
    if (v >= 1 && v <= 1 << 20) h->gram_wg_target = v;
  }
  if (const char *e = getenv("TNSIM_OVERLAP_PREPARE")) h->overlap_prepare = atoi(e) != 0;
  if (const char *e = getenv("TNSIM_SPECULATE")) h->speculate = atoi(e) != 0;
  if (const char *e = getenv("TNSIM_ADMIT_GROUP")) {
    const int v = atoi(e);
    if (v >= 1 && v <= 4096) h->admit_group = v;
  }
  if (const char *e = getenv("TNSIM_INNER_SWEEPS")) {
    int v = atoi(e);
    if (v >= 1 && v <= 60) h->inner_sweeps = v;
  }
  const Layout &LL = h->L;
  h->pin_bytes = align_up(sizeof(GateDesc) * LL.desc_cap) + align_up(sizeof(SlotScalars) * LL.desc_cap) +
                 align_up(sizeof(Gate1Desc) * LL.n) + 4096;
  h->pin_sc1_off = h->pin_bytes;  // the second buffer of sweep scalars
  h->pin_bytes += align_up(sizeof(SlotScalars) * LL.desc_cap);
  if (hipHostMalloc((void **)&h->pin, h->pin_bytes, hipHostMallocDefault) != hipSuccess) {
    delete h;
    return TNSIM_E_DEVICE;
  }
  // device tables of site / lambda pointers for the init kernel
  std::vector<void *> sp(LL.n), lp(std::max(LL.n - 1, 1));
  for (int q = 0; q < LL.n; q++) sp[q] = h->site(q);
  for (int b = 0; b < LL.n - 1; b++) lp[b] = h->lam(b);
  tnsim_status st = TNSIM_OK;
  if (hipMemcpy(h->arena + LL.site_tab_off, sp.data(), sizeof(void *) * LL.n,
                hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(h->arena + LL.lam_tab_off, lp.data(), sizeof(void *) * (LL.n - 1),
                hipMemcpyHostToDevice) != hipSuccess)
    st = TNSIM_E_DEVICE;
  if (st == TNSIM_OK) st = init_state(h);
  if (st != TNSIM_OK) {
    hipHostFree(h->pin);
    delete h;
    return st;
  }
  *out = h;
  return TNSIM_OK;
}

tnsim_status tnsim_mps_destroy(tnsim_mps h) {
  if (!h) return TNSIM_E_ARG;
  if (!h->poisoned) hipStreamSynchronize(h->stream);
  if (h->stream2) {
    hipStreamSynchronize(h->stream2);
    prof_drain(h, true);
    hipStreamDestroy(h->stream2);
  }
  if (h->ev_main) hipEventDestroy(h->ev_main);
  if (h->ev_prep) hipEventDestroy(h->ev_prep);
  for (hipEvent_t e : h->ev_sw)
    if (e) hipEventDestroy(e);
  if (h->pin2) hipHostFree(h->pin2);
  prof_drain(h);
  if (h->sweep_exec) hipGraphExecDestroy(h->sweep_exec);
  for (hipEvent_t e : h->evpool) hipEventDestroy(e);
  if (h->pin) hipHostFree(h->pin);
  delete h;
  return TNSIM_OK;
}

tnsim_status tnsim_mps_reset(tnsim_mps h) {
  tnsim_status s = check_handle(h);
  if (s != TNSIM_OK) return s;
  h->state_version++;
  return init_state(h);
}

tnsim_status tnsim_apply_1q(tnsim_mps h, int32_t q, const tnsim_c128 u[4]) {
  tnsim_status s = check_handle(h);
  if (s != TNSIM_OK) return s;
  h->state_version++;
  if (!u || q < 0 || q >= h->L.n || !finite_gate(u, 4)) return TNSIM_E_ARG;
  return run_1q(h, {{q, u}});
}

tnsim_status tnsim_apply_2q(tnsim_mps h, int32_t q0, int32_t q1, const tnsim_c128 g[16]) {
  tnsim_status s = check_handle(h);
  if (s != TNSIM_OK) return s;
  h->state_version++;
  if (!g || q0 < 0 || q1 < 0 || q0 >= h->L.n || q1 >= h->L.n || q0 == q1 || !finite_gate(g, 16))
    return TNSIM_E_ARG;
  h->last_sweeps = 0;
  h->last_batch.clear();
  if (std::abs(q0 - q1) != 1) {  // a SWAP chain, one local gate after the other
    tnsim_gate gt;
    gt.q0 = q0;
    gt.q1 = q1;
    memcpy(gt.m, g, sizeof gt.m);
    std::vector<tnsim_gate> chain;
    expand_gate(gt, chain);
    return run_circuit(h, chain.data(), (int)chain.size());
  }
  Pending p;
  orient(q0, q1, g, p);
  return run_2q_batch(h, &p, 1);
}

namespace {

// Operator Schmidt decomposition of a two-qubit gate for bond propagation:
// G = sum_r X_r (x) Y_r, X_r acting on the qubit at the left site and Y_r on
// the one at the right site (q0_left: q0 is the left one), with the singular
// values folded into Y_r.  Gm[(x',x),(y',y)] is factored by one-sided
// (Hestenes) Jacobi on its four columns; the terms whose squared singular
// value is above 4 * 2^-53 of the largest one are kept.  Returns their count.
int op_schmidt(const tnsim_c128 *g, bool q0_left, Mat4x4 &X, Mat4x4 &Y) {
  double2 Gm[4][4], W[4][4];  // [row][col]
  for (int xp = 0; xp < 2; xp++)
    for (int x = 0; x < 2; x++)
      for (int yp = 0; yp < 2; yp++)
        for (int y = 0; y < 2; y++) {
          const int row = q0_left ? 2 * xp + yp : 2 * yp + xp;
          const int col = q0_left ? 2 * x + y : 2 * y + x;
          Gm[2 * xp + x][2 * yp + y] = make_double2(g[row * 4 + col].re, g[row * 4 + col].im);
        }
  for (int i = 0; i < 4; i++)
    for (int j = 0; j < 4; j++) W[i][j] = Gm[i][j];
  auto dotc = [&](int p, int q) {  // column p ^H column q
    double re = 0.0, im = 0.0;
    for (int i = 0; i < 4; i++) {
      re += W[i][p].x * W[i][q].x + W[i][p].y * W[i][q].y;
      im += W[i][p].x * W[i][q].y - W[i][p].y * W[i][q].x;
    }
    return make_double2(re, im);
  };
  for (int sweep = 0; sweep < 60; sweep++) {
    bool rotated = false;
    for (int p = 0; p < 4; p++)
      for (int q = p + 1; q < 4; q++) {
        const double a = dotc(p, p).x, b = dotc(q, q).x;
        const double2 c = dotc(p, q);
        const double ac = std::sqrt(c.x * c.x + c.y * c.y);
        if (!(ac > 1e-15 * std::sqrt(a * b)) || a == 0.0 || b == 0.0) continue;
        rotated = true;
        const double2 e = make_double2(c.x / ac, c.y / ac);
        const double zeta = (b - a) / (2.0 * ac);
        const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        const double cs = 1.0 / std::sqrt(1.0 + t * t), sn = cs * t;
        for (int i = 0; i < 4; i++) {
          const double2 xv = W[i][p];
          // y~ = e^{-i phi} y
          const double2 yt = make_double2(e.x * W[i][q].x + e.y * W[i][q].y,
                                          e.x * W[i][q].y - e.y * W[i][q].x);
          W[i][p] = make_double2(cs * xv.x - sn * yt.x, cs * xv.y - sn * yt.y);
          W[i][q] = make_double2(sn * xv.x + cs * yt.x, sn * xv.y + cs * yt.y);
        }
      }
    if (!rotated) break;
  }
  int ord[4] = {0, 1, 2, 3};
  double nrm[4];
  for (int j = 0; j < 4; j++) nrm[j] = std::sqrt(dotc(j, j).x);
  std::stable_sort(ord, ord + 4, [&](int u, int v) { return nrm[u] > nrm[v]; });
  int rg = 0;
  for (int j = 0; j < 4; j++)
    if (nrm[ord[j]] * nrm[ord[j]] > 4 * 0x1p-53 * nrm[ord[0]] * nrm[ord[0]]) rg++;
  memset(&X, 0, sizeof X);
  memset(&Y, 0, sizeof Y);
  for (int r = 0; r < rg; r++) {
    const int j = ord[r];
    for (int e = 0; e < 4; e++)
      X.v[r][e] = make_double2(W[e][j].x / nrm[j], W[e][j].y / nrm[j]);
    for (int e = 0; e < 4; e++) {  // Y_r = U_r^H Gm
      double re = 0.0, im = 0.0;
      for (int i = 0; i < 4; i++) {
        re += X.v[r][i].x * Gm[i][e].x + X.v[r][i].y * Gm[i][e].y;
        im += X.v[r][i].x * Gm[i][e].y - X.v[r][i].y * Gm[i][e].x;
      }
      Y.v[r][e] = make_double2(re, im);
    }
  }
  return rg;
}

// Gate on distant qubits a < b by bond propagation (Sec. III.A): the
// operator bond of G = sum_r X_r (x) Y_r is merged into bonds a .. b-1
// (site a takes X_r, the sites in between I_r, site b takes Y_r), which
// holds G|psi> exactly; the window is then decomposed from left to right
// without truncation (each intermediate site in succession) and given its
// Schmidt values from right to left, where chi_max and the cutoff apply.
// Each step is the ordinary two-site path with the identity gate.  The
// merged sites, whose bonds may exceed a site buffer's capacity (near the
// ends of the chain a bond holds at most 2^min(b+1, n-1-b)), live in the X
// and J buffers of the gate slots 1, 2, ... (two sites per buffer) until a
// step leaves a site with its final dimensions.
tnsim_status apply_propagate(tnsim_mps h, int q0, int q1, const tnsim_c128 *g) {
  const int a = std::min(q0, q1), b = std::max(q0, q1), d = b - a;
  Mat4x4 X, Y;
  const int rg = op_schmidt(g, q0 == a, X, Y);
  const Layout &L = h->L;
  const int maxbond = L.cmax / 2;
  for (int j = a; j < b; j++)
    if ((long long)rg * h->dims[j + 1] > maxbond) {
      h->err = "bond propagation: bond " + std::to_string(j) + " would need dimension " +
               std::to_string(rg * h->dims[j + 1]) + " (operator rank " + std::to_string(rg) +
               " times " + std::to_string(h->dims[j + 1]) + "), above the capacity " +
               std::to_string(maxbond) + "; tnsim_apply_2q takes this gate by SWAPs";
      return TNSIM_E_CAPACITY;
    }
  // window storage: site w of the window at half of an X or J buffer of slot >= 1
  const size_t half = (size_t)L.ldx_max * L.cols_pad_max * sizeof(double2) / 2;
  if (d + 1 > 4 * (L.nslots - 1)) {
    h->err = "bond propagation: a window of " + std::to_string(d + 1) +
             " sites needs more gate slots than the handle has (max_layer_gates); "
             "tnsim_apply_2q takes this gate by SWAPs";
    return TNSIM_E_CAPACITY;
  }
  auto win = [&](int w) -> void * {
    const int sl = 1 + w / 4, part = w % 4;
    char *base = h->slot(sl) + (part < 2 ? L.x_off : L.j_off);
    return base + (part & 1) * half;
  };
  h->state_version++;
  h->last_sweeps = 0;
  h->last_batch.clear();
  hipStream_t st = h->stream;
  double2 *old = (double2 *)(h->slot(0) + L.x_off);  // one site at a time, complex128
  const std::vector<int> od = h->dims;
  for (int q = a; q <= b; q++) {
    const int role = q == a ? 0 : (q == b ? 2 : 1);
    launch_convert(st, h->site(q), L.storage, old, 0, (size_t)od[q] * 2 * od[q + 1]);
    launch_prop_merge(st, old, win(q - a), L.storage, od[q], od[q + 1], rg, role,
                      role == 0 ? X : Y);
  }
  LAUNCHCHK(h, "propagation merge");
  for (int q = a + 1; q <= b; q++) h->dims[q] = rg * od[q];
  HIPCHK(h, hipStreamSynchronize(st));
  memcpy(h->pin, h->dims.data(), sizeof(int32_t) * (L.n + 1));
  HIPCHK(h, hipMemcpyAsync(h->dims_dev(), h->pin, sizeof(int32_t) * (L.n + 1),
                           hipMemcpyHostToDevice, st));
  auto step = [&](int j, int flags, void *a0i, void *a1i, void *a0o, void *a1o) {
    Pending p{};
    for (int e = 0; e < 4; e++) p.g[5 * e] = make_double2(1.0, 0.0);
    p.i = j;
    p.flags = flags;
    p.a0_in = a0i;
    p.a1_in = a1i;
    p.a0_out = a0o;
    p.a1_out = a1o;
    return run_2q_batch(h, &p, 1);
  };
  // left to right inside the window (window site w = site a + w): the bonds
  // shrink to their ranks, which may still exceed a site buffer
  for (int j = a; j + 1 < b; j++) {
    tnsim_status s = step(j, PEND_UNWEIGHTED | PEND_NO_CUT | PEND_NO_STATS, win(j - a),
                          win(j + 1 - a), win(j - a), win(j + 1 - a));
    if (s != TNSIM_OK) return s;
  }
  // right to left, with the Schmidt weights and the truncation rule: the
  // right site of each step is final and goes to its buffer, the left one
  // stays in the window until the last step
  for (int j = b - 1; j >= a; j--) {
    tnsim_status s = step(j, PEND_EPS_ONLY, win(j - a), win(j + 1 - a),
                          j == a ? h->site(a) : win(j - a), h->site(j + 1));
    if (s != TNSIM_OK) return s;
  }
  h->n2q += 1;
  return TNSIM_OK;
}

}  // namespace

tnsim_status tnsim_apply_2q_propagate(tnsim_mps h, int32_t q0, int32_t q1,
                                      const tnsim_c128 g[16]) {
  tnsim_status s = check_handle(h);
  if (s != TNSIM_OK) return s;
  const int n = h->L.n;
  if (q0 < 0 || q0 >= n || q1 < 0 || q1 >= n || q0 == q1 || !g || !finite_gate(g, 16))
    return TNSIM_E_ARG;
  if (std::abs(q0 - q1) == 1) return tnsim_apply_2q(h, q0, q1, g);
  return apply_propagate(h, q0, q1, g);
}

tnsim_status tnsim_canonicalize(tnsim_mps h, int32_t truncate) {
  tnsim_status s = check_handle(h);
  if (s != TNSIM_OK) return s;
  if (truncate != 0 && truncate != 1) return TNSIM_E_ARG;
  h->state_version++;
  h->last_sweeps = 0;
  h->last_batch.clear();
  s = canonical_pass(h, truncate != 0);
  // a cut changes the state, so the bonds right of it (swept before it) no
  // longer carry its Schmidt values: one more pass without truncation
  if (s == TNSIM_OK && truncate) s = canonical_pass(h, false);
  return s;
}

tnsim_status tnsim_apply_layer(tnsim_mps h, const tnsim_gate *gates, int32_t n_gates) {
  tnsim_status s = check_handle(h);
  if (s != TNSIM_OK) return s;
  h->state_version++;
  std::vector<std::pair<int, const tnsim_c128 *>> g1;
  std::vector<Pending> g2;
  s = validate_layer(h, gates, n_gates, g1, g2);
  if (s != TNSIM_OK) return s;
  h->last_sweeps = 0;
  h->last_batch.clear();
  s = run_1q(h, g1);
  if (s != TNSIM_OK) return s;
  return run_2q(h, g2);
}

tnsim_status tnsim_apply_circuit(tnsim_mps h, const tnsim_gate *gates, int32_t n_gates) {
  tnsim_status s = check_handle(h);
  if (s != TNSIM_OK) return s;
  h->state_version++;
  const int n = h->L.n;
  if (n_gates < 0 || (n_gates > 0 && !gates)) return TNSIM_E_ARG;
  std::vector<tnsim_gate> local;
  for (int k = 0; k < n_gates; k++) {
    const int a = gates[k].q0, b = gates[k].q1;
    if (a < 0 || a >= n || b < -1 || b >= n || a == b || !finite_gate(gates[k])) return TNSIM_E_ARG;
    expand_gate(gates[k], local);
  }
  h->last_sweeps = 0;
  h->last_batch.clear();
  return run_circuit(h, local.data(), (int)local.size());
}

tnsim_status tnsim_apply_layer_multi(tnsim_mps const *mps, const tnsim_gate *const *gates,
                                     const int32_t *n_gates, int32_t n_mps) {
  if (!mps || !gates || !n_gates || n_mps < 0) return TNSIM_E_ARG;
  if (n_mps == 0) return TNSIM_OK;
  tnsim_mps o = mps[0];
  for (int k = 0; k < n_mps; k++) {
    tnsim_status s = check_handle(mps[k]);
    if (s != TNSIM_OK) return s;
    if (mps[k]->stream != o->stream || mps[k]->cfg.precision != o->cfg.precision)
      return TNSIM_E_ARG;
    for (int j = 0; j < k; j++)
      if (mps[j] == mps[k]) return TNSIM_E_ARG;
  }
  for (int k = 0; k < n_mps; k++) mps[k]->state_version++;
  std::vector<std::vector<std::pair<int, const tnsim_c128 *>>> g1(n_mps);
  std::vector<std::vector<Pending>> g2(n_mps);
  for (int k = 0; k < n_mps; k++) {
    tnsim_status s = validate_layer(mps[k], gates[k], n_gates[k], g1[k], g2[k]);
    if (s != TNSIM_OK) return s;
  }
  for (int k = 0; k < n_mps; k++) {
    mps[k]->last_sweeps = 0;
    mps[k]->last_batch.clear();
    tnsim_status s = run_1q(mps[k], g1[k]);
    if (s != TNSIM_OK) return s;
  }
  // every two-qubit gate of every handle in as few batches as the owner's
  // descriptor capacity and each handle's workspace slots allow
  std::vector<size_t> next(n_mps, 0);
  std::vector<int> used(n_mps);
  std::vector<BatchItem> items;
  for (;;) {
    items.clear();
    std::fill(used.begin(), used.end(), 0);
    bool more = true;
    while (more && (int)items.size() < o->L.desc_cap) {
      more = false;
      for (int k = 0; k < n_mps && (int)items.size() < o->L.desc_cap; k++) {
        if (next[k] < g2[k].size() && used[k] < mps[k]->L.nslots) {
          items.push_back(BatchItem{mps[k], used[k]++, &g2[k][next[k]]});
          next[k]++;
          more = true;
        }
      }
    }
    if (items.empty()) break;
    tnsim_status s = run_2q_items(o, items.data(), (int)items.size(), false);
    if (s != TNSIM_OK) return s;
  }
  return TNSIM_OK;
}

tnsim_status tnsim_layerise(const tnsim_gate *gates, int32_t n_gates, int32_t n_qubits,
                            int32_t *layer_of_gate, int32_t *n_layers) {
  if (n_gates < 0 || n_qubits < 1 || (n_gates > 0 && (!gates || !layer_of_gate)) || !n_layers)
    return TNSIM_E_ARG;
  std::vector<int> next(n_qubits, 0);
  int nl = 0;
  for (int k = 0; k < n_gates; k++) {
    int a = gates[k].q0, b = gates[k].q1;
    if (a < 0 || a >= n_qubits || b < -1 || b >= n_qubits || a == b) return TNSIM_E_ARG;
    int l = next[a];
    if (b >= 0) l = std::max(l, next[b]);
    layer_of_gate[k] = l;
    next[a] = l + 1;
    if (b >= 0) next[b] = l + 1;
    nl = std::max(nl, l + 1);
  }
  *n_layers = nl;
  return TNSIM_OK;
}

tnsim_status tnsim_expect_pauli(tnsim_mps h, const char *pauli, double *re_out, double *im_out) {
  tnsim_status s = check_handle(h);
  if (s != TNSIM_OK) return s;
  if (!pauli || !re_out) return TNSIM_E_ARG;
  const int n = h->L.n;
  static const double2 PM[4][4] = {
      {{1, 0}, {0, 0}, {0, 0}, {1, 0}},
      {{0, 0}, {1, 0}, {1, 0}, {0, 0}},
      {{0, 0}, {0, -1}, {0, 1}, {0, 0}},
      {{1, 0}, {0, 0}, {0, 0}, {-1, 0}}};
  std::vector<double2> tab(4 * n);
  std::vector<char> isI(n);
  for (int q = 0; q < n; q++) {
    int k;
    switch (pauli[q]) {
      case 'I': k = 0; break;
      case 'X': k = 1; break;
      case 'Y': k = 2; break;
      case 'Z': k = 3; break;
      default: return TNSIM_E_ARG;
    }
    isI[q] = k == 0;
    for (int e = 0; e < 4; e++) tab[4 * q + e] = PM[k][e];
  }
  double2 num, den;
  s = transfer(h, h, h, tab.data(), isI.data(), &num);
  if (s != TNSIM_OK) return s;
  s = transfer(h, h, h, nullptr, nullptr, &den);
  if (s != TNSIM_OK) return s;
  // num / den
  double dd = den.x * den.x + den.y * den.y;
  *re_out = (num.x * den.x + num.y * den.y) / dd;
  if (im_out) *im_out = (num.y * den.x - num.x * den.y) / dd;
  return TNSIM_OK;
}

tnsim_status tnsim_overlap(tnsim_mps a, tnsim_mps b, tnsim_c128 *out) {
  tnsim_status s = check_handle(a);
  if (s != TNSIM_OK) return s;
  s = check_handle(b);
  if (s != TNSIM_OK) return s;
  if (!out || a->L.n != b->L.n) return TNSIM_E_ARG;
  if (a->stream != b->stream) HIPCHK(b, hipStreamSynchronize(b->stream));
  double2 v;
  // buffers of a are sized by a's chi_max; both operands must fit them
  for (int q = 0; q <= a->L.n; q++)
    if (b->dims[q] > a->L.dimcap[q]) return TNSIM_E_CAPACITY;
  s = transfer(a, a, b, nullptr, nullptr, &v);
  if (s != TNSIM_OK) return s;
  out->re = v.x;
  out->im = v.y;
  return TNSIM_OK;
}

tnsim_status tnsim_amplitude(tnsim_mps h, const uint8_t *bits, tnsim_c128 *out) {
  tnsim_status s = check_handle(h);
  if (s != TNSIM_OK) return s;
  if (!bits || !out) return TNSIM_E_ARG;
  const int n = h->L.n;
  for (int q = 0; q < n; q++)
    if (bits[q] > 1) return TNSIM_E_ARG;
  hipStream_t st = h->stream;
  double2 *v = h->at<double2>(h->L.va_off), *w = h->at<double2>(h->L.vb_off);
  double2 one = make_double2(1.0, 0.0);
  HIPCHK(h, hipStreamSynchronize(st));
  memcpy(h->pin, &one, sizeof one);
  HIPCHK(h, hipMemcpyAsync(v, h->pin, sizeof one, hipMemcpyHostToDevice, st));
  for (int q = 0; q < n; q++) {
    launch_amp_step(st, v, w, h->at<double2>(h->L.f_off), h->site(q), h->L.storage, h->dims[q],
                    h->dims[q + 1], bits[q]);
    LAUNCHCHK(h, "amplitude");
    std::swap(v, w);
  }
  HIPCHK(h, hipMemcpyAsync(h->pin, v, sizeof(double2), hipMemcpyDeviceToHost, st));
  HIPCHK(h, hipStreamSynchronize(st));
  double2 r;
  memcpy(&r, h->pin, sizeof r);
  out->re = r.x;
  out->im = r.y;
  return TNSIM_OK;
}

// Workspace of tnsim_sample: per site the stacked weights [M_q^0; M_q^1]
// (M_q^s = A_q^{sH} E_q A_q^s), and the node tables of one step (see
// k_sample.hip).
struct SampleLayout {
  std::vector<size_t> msite;  // 2 x dimcap[q+1]^2 complex128 per site
  size_t E0 = 0, E1 = 0, F = 0, P = 0, V0 = 0, V1 = 0, Y = 0, p = 0, flag = 0, idx = 0,
         node = 0, key = 0, parent = 0, scale = 0, logp = 0, ctr = 0, total = 0;
};

static SampleLayout sample_layout(const Layout &L, int max_shots) {
  SampleLayout S;
  const int n = L.n;
  int dmax = 1;
  for (int q = 0; q <= n; q++) dmax = std::max(dmax, L.dimcap[q]);
  // node tables: at most one node per distinct drawn suffix (<= shots) plus
  // fewer than 64 zero nodes that align the bit-1 nodes to a column tile
  const size_t ms = (size_t)std::max(max_shots, 1) + 64, d2 = (size_t)dmax * dmax;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  S.msite.resize(n);
  for (int q = 0; q < n; q++)
    S.msite[q] = take(sizeof(double2) * 2 * (size_t)L.dimcap[q + 1] * L.dimcap[q + 1]);
  S.E0 = take(sizeof(double2) * d2);  // E_q, E_{q+1} in turn
  S.E1 = take(sizeof(double2) * d2);
  S.F = take(sizeof(double2) * 2 * d2);
  S.P = take(sizeof(double2) * ZGEMM_PART_ELEMS);  // split-K partial products
  S.V0 = take(sizeof(double2) * ms * dmax);
  S.V1 = take(sizeof(double2) * ms * dmax);
  S.Y = take(sizeof(double2) * 2 * ms * dmax);
  S.p = take(sizeof(double) * 2 * ms);
  S.flag = take(sizeof(int) * (2 * ms + 1));
  S.idx = take(sizeof(int) * (2 * ms + 1));
  S.node = take(sizeof(int) * (ms - 64));
  S.key = take(sizeof(int) * (ms - 64));
  S.parent = take(sizeof(int) * ms);
  S.scale = take(sizeof(double) * ms);
  S.logp = take(sizeof(double) * (ms - 64));
  S.ctr = take(sizeof(int) * 8);
  S.total = off;
  return S;
}

size_t tnsim_sample_workspace_bytes(const tnsim_config *cfg, int32_t max_shots) {
  if (!valid_config(cfg) || max_shots < 1 || max_shots > (1 << 28)) return 0;
  return sample_layout(make_layout(*cfg), max_shots).total;
}

// Per-site bit weights M_q^s = A_q^{sH} (E_q A_q^s) into the workspace: F =
// E_q A_q (rows (a, s)), then one product per s over the rows of that s;
// E_{q+1} = M_q^0 + M_q^1.
static tnsim_status sample_weights(tnsim_mps h, char *ws, const SampleLayout &S) {
  const Layout &L = h->L;
  const int n = L.n, sto = L.storage;
  hipStream_t st = h->stream;
  auto Ms = [&](int q) { return (double2 *)(ws + S.msite[q]); };
  double2 *E = (double2 *)(ws + S.E0), *En = (double2 *)(ws + S.E1);
  double2 *F = (double2 *)(ws + S.F), *Pb = (double2 *)(ws + S.P);
  // E_0 = 1 (and the node tables of a one-shot draw, unused here)
  launch_smp_init(st, 0, 64, (int *)(ws + S.node), (double *)(ws + S.logp), (int *)(ws + S.flag),
                  (double2 *)(ws + S.V0), E, (int *)(ws + S.ctr));
  for (int q = 0; q < n; q++) {
    const int la = h->dims[q], rb = h->dims[q + 1];
    ZgemmArgs f{la, 2 * rb, la, E, la, h->site(q), 2 * rb, F, 2 * rb, nullptr, 0};
    f.ksplit = zgemm_ksplit(la, 2 * rb, la);
    f.part = Pb;
    launch_zgemm(st, ZGEMM_NN_ROW, f, 0, sto);
    for (int sb = 0; sb < 2; sb++) {
      const char *A = (const char *)h->site(q) + (size_t)sb * rb * L.elem;
      ZgemmArgs e{rb, rb, la, A, 2LL * rb, F + (size_t)sb * rb, 2LL * rb,
                  Ms(q) + (size_t)sb * rb * rb, rb, nullptr, 0};
      e.ksplit = zgemm_ksplit(rb, rb, la);
      e.part = Pb;
      launch_zgemm(st, ZGEMM_CN_ROW, e, sto, 0);
    }
    if (q + 1 < n) {
      launch_smp_add(st, Ms(q), (size_t)rb * rb, En);
      std::swap(E, En);
    }
  }
  LAUNCHCHK(h, "sample weights");
  return TNSIM_OK;
}

// The draws, from weights already in the workspace (layout S, shots within
// its capacity).
static tnsim_status sample_draw(tnsim_mps h, char *ws, const SampleLayout &S, int shots,
                                const double *dev_u, uint8_t *dev_bits, double *dev_logp) {
  const Layout &L = h->L;
  const int n = L.n, sto = L.storage;
  hipStream_t st = h->stream;
  auto Ms = [&](int q) { return (double2 *)(ws + S.msite[q]); };
  double2 *V = (double2 *)(ws + S.V0), *Vn = (double2 *)(ws + S.V1), *Yb = (double2 *)(ws + S.Y);
  double *p = (double *)(ws + S.p), *logp = (double *)(ws + S.logp);
  double *scale = (double *)(ws + S.scale);
  int *flag = (int *)(ws + S.flag), *idx = (int *)(ws + S.idx), *node = (int *)(ws + S.node),
      *key = (int *)(ws + S.key), *parent = (int *)(ws + S.parent), *ctr = (int *)(ws + S.ctr);
  const int cap = shots + 64;  // node-table columns (see sample_layout)
  launch_smp_init(st, shots, cap, node, logp, flag, V, (double2 *)(ws + S.E0), ctr);
  long long mb = 1;  // bound on the node count before the step
  for (int q = n - 1; q >= 0; q--) {
    const int la = h->dims[q], rb = h->dims[q + 1];
    const int b1 = (int)std::min<long long>(mb, cap);
    const int b2 = (int)std::min<long long>(2LL * b1 + 64, cap);  // after the step
    // Y = [M^0; M^1] V, then the weights of both bits of every node
    launch_zgemm(st, ZGEMM_NN_COL, ZgemmArgs{2 * rb, b1, rb, Ms(q), rb, V, rb, Yb, 2LL * rb, ctr, 1},
                 0, 0);
    launch_smp_prob(st, V, Yb, rb, 2 * b1, ctr, p);
    launch_smp_decide(st, shots, n, q, dev_u, p, node, key, flag, dev_bits, logp, ctr);
    launch_smp_scan(st, flag, idx, ctr);
    launch_smp_parent(st, flag, idx, p, ctr, 2 * b1, parent, scale);
    // next nodes: columns [0, ctr[4]) from bit 0, [ctr[4], ctr[0]) from bit 1
    // (ctr[4] is a multiple of 64, so each column tile reads one row set of A)
    ZgemmArgs w{la, b2, rb, h->site(q), 2LL * rb, V, rb, Vn, la, nullptr, 0};
    w.za = rb;
    w.clo = ctr + 5;
    w.chi = ctr + 0;
    w.asplit = ctr + 4;
    w.bmap = parent;
    w.cscale = scale;
    launch_zgemm(st, ZGEMM_NN_COL_GATHER, w, sto, 0);
    launch_smp_relabel(st, shots, key, idx, node);
    LAUNCHCHK(h, "sample step");
    std::swap(V, Vn);
    mb = b2;
  }
  if (dev_logp)
    HIPCHK(h, hipMemcpyAsync(dev_logp, logp, sizeof(double) * shots, hipMemcpyDeviceToDevice, st));
  HIPCHK(h, hipMemcpyAsync(h->pin, ctr, sizeof(int) * 4, hipMemcpyDeviceToHost, st));
  HIPCHK(h, hipStreamSynchronize(st));
  int c[4];
  memcpy(c, h->pin, sizeof c);
  if (c[1] || c[2]) {
    h->err = c[1] ? "sample: a uniform outside [0, 1)" : "sample: a node of zero weight";
    return TNSIM_E_ARG;
  }
  return TNSIM_OK;
}

static tnsim_status sample_check_ws(tnsim_mps h, void *dev_ws, size_t ws_bytes, int cap,
                                    SampleLayout &S) {
  if (!dev_ws || reinterpret_cast<uintptr_t>(dev_ws) % ALIGN) return TNSIM_E_ARG;
  S = sample_layout(h->L, cap);
  return ws_bytes < S.total ? TNSIM_E_CAPACITY : TNSIM_OK;
}

tnsim_status tnsim_sample(tnsim_mps h, void *dev_ws, size_t ws_bytes, int32_t shots,
                          const double *dev_u, uint8_t *dev_bits, double *dev_logp) {
  tnsim_status s = check_handle(h);
  if (s != TNSIM_OK) return s;
  if (shots < 0 || shots > (1 << 28)) return TNSIM_E_ARG;
  if (shots == 0) return TNSIM_OK;
  if (!dev_u || !dev_bits) return TNSIM_E_ARG;
  SampleLayout S;
  s = sample_check_ws(h, dev_ws, ws_bytes, shots, S);
  if (s != TNSIM_OK) return s;
  s = sample_weights(h, (char *)dev_ws, S);
  if (s != TNSIM_OK) return s;
  return sample_draw(h, (char *)dev_ws, S, shots, dev_u, dev_bits, dev_logp);
}

tnsim_status tnsim_sample_prepare(tnsim_mps h, void *dev_ws, size_t ws_bytes, int32_t max_shots) {
  tnsim_status s = check_handle(h);
  if (s != TNSIM_OK) return s;
  if (max_shots < 1 || max_shots > (1 << 28)) return TNSIM_E_ARG;
  SampleLayout S;
  s = sample_check_ws(h, dev_ws, ws_bytes, max_shots, S);
  if (s != TNSIM_OK) return s;
  h->smp_ws = nullptr;  // invalid until the weights are in
  s = sample_weights(h, (char *)dev_ws, S);
  if (s != TNSIM_OK) return s;
  h->smp_ws = dev_ws;
  h->smp_bytes = ws_bytes;
  h->smp_cap = max_shots;
  h->smp_version = h->state_version;
  return TNSIM_OK;
}

tnsim_status tnsim_sample_draw(tnsim_mps h, void *dev_ws, size_t ws_bytes, int32_t shots,
                               const double *dev_u, uint8_t *dev_bits, double *dev_logp) {
  tnsim_status s = check_handle(h);
  if (s != TNSIM_OK) return s;
  if (shots < 0 || shots > (1 << 28)) return TNSIM_E_ARG;
  if (dev_ws == nullptr || dev_ws != h->smp_ws || ws_bytes != h->smp_bytes ||
      h->smp_version != h->state_version) {
    h->err = "sample_draw: no current weights in this workspace (call tnsim_sample_prepare)";
    return TNSIM_E_ARG;
  }
  if (shots > h->smp_cap) return TNSIM_E_CAPACITY;
  if (shots == 0) return TNSIM_OK;
  if (!dev_u || !dev_bits) return TNSIM_E_ARG;
  const SampleLayout S = sample_layout(h->L, h->smp_cap);
  return sample_draw(h, (char *)dev_ws, S, shots, dev_u, dev_bits, dev_logp);
}

// ---- sampling without allocation: the workspace is a fixed device array
// (one copy per GPU, resident from the library's load until the process
// ends).  In host code `scratch` names a host-side stand-in; kernels get the
// device address that hipGetSymbolAddress returns for the current device,
// looked up once per device and kept in smp_scratch_dev.
static __device__ __align__(256) char scratch[TNSIM_SAMPLE_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex smp_scratch_mu;
void *smp_scratch_dev[MAX_DEVICES] = {};

// Device address of `scratch` on `dev`, looked up with that device current.
tnsim_status scratch_on_device(tnsim_mps h, void **out) {
  const int dev = h->device;
  if (dev < 0 || dev >= MAX_DEVICES) {
    h->err = "sample_noalloc: device index beyond the supported range";
    return TNSIM_E_DEVICE;
  }
  std::lock_guard<std::mutex> lock(smp_scratch_mu);
  if (!smp_scratch_dev[dev]) {
    int cur = 0;
    HIPCHK(h, hipGetDevice(&cur));
    if (cur != dev) HIPCHK(h, hipSetDevice(dev));
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != dev) HIPCHK(h, hipSetDevice(cur));
    if (e != hipSuccess) return fail(h, e, "hipGetSymbolAddress(scratch)");
    smp_scratch_dev[dev] = ptr;
  }
  *out = smp_scratch_dev[dev];
  return TNSIM_OK;
}
}  // namespace

tnsim_status tnsim_sample_noalloc(tnsim_mps h, int32_t shots, const double *dev_u,
                                  uint8_t *dev_bits, double *dev_logp) {
  tnsim_status s = check_handle(h);
  if (s != TNSIM_OK) return s;
  if (shots < 0 || shots > (1 << 28)) return TNSIM_E_ARG;
  if (shots == 0) return TNSIM_OK;
  if (!dev_u || !dev_bits) return TNSIM_E_ARG;
  const SampleLayout S = sample_layout(h->L, shots);
  if (S.total > (size_t)TNSIM_SAMPLE_SCRATCH_BYTES) {
    h->err = "sample_noalloc: this handle's sampling workspace for that many shots (" +
             std::to_string(S.total) + " bytes) exceeds the fixed device array (" +
             std::to_string((size_t)TNSIM_SAMPLE_SCRATCH_BYTES) + " bytes)";
    return TNSIM_E_CAPACITY;
  }
  void *ws = nullptr;
  s = scratch_on_device(h, &ws);
  if (s != TNSIM_OK) return s;
  s = sample_weights(h, (char *)ws, S);
  if (s != TNSIM_OK) return s;
  return sample_draw(h, (char *)ws, S, shots, dev_u, dev_bits, dev_logp);
}

tnsim_status tnsim_mps_copy(tnsim_mps dst, tnsim_mps src) {
  tnsim_status s = check_handle(dst);
  if (s != TNSIM_OK) return s;
  s = check_handle(src);
  if (s != TNSIM_OK) return s;
  if (dst->L.n != src->L.n) return TNSIM_E_ARG;
  dst->state_version++;
  const int n = dst->L.n;
  for (int q = 1; q < n; q++)
    if (src->dims[q] > dst->L.dimcap[q]) return TNSIM_E_CAPACITY;
  HIPCHK(src, hipStreamSynchronize(src->stream));
  for (int q = 0; q < n; q++) {
    size_t cnt = (size_t)src->dims[q] * 2 * src->dims[q + 1];
    launch_convert(dst->stream, src->site(q), src->L.storage, dst->site(q), dst->L.storage, cnt);
  }
  LAUNCHCHK(dst, "copy");
  for (int b = 0; b < n - 1; b++)
    HIPCHK(dst, hipMemcpyAsync(dst->lam(b), src->lam(b), sizeof(double) * src->dims[b + 1],
                               hipMemcpyDeviceToDevice, dst->stream));
  dst->dims = src->dims;
  HIPCHK(dst, hipStreamSynchronize(dst->stream));
  memcpy(dst->pin, src->dims.data(), sizeof(int32_t) * (n + 1));
  HIPCHK(dst, hipMemcpyAsync(dst->dims_dev(), dst->pin, sizeof(int32_t) * (n + 1),
                             hipMemcpyHostToDevice, dst->stream));
  HIPCHK(dst, hipStreamSynchronize(dst->stream));
  dst->sum_eps = src->sum_eps;
  dst->prod_keep = src->prod_keep;
  dst->n2q = src->n2q;
  return TNSIM_OK;
}

tnsim_status tnsim_bond_dims(tnsim_mps h, int32_t *out) {
  tnsim_status s = check_handle(h);
  if (s != TNSIM_OK) return s;
  if (!out) return TNSIM_E_ARG;
  for (int b = 0; b < h->L.n - 1; b++) out[b] = h->dims[b + 1];
  return TNSIM_OK;
}

tnsim_status tnsim_truncation_stats(tnsim_mps h, double *sum_eps, double *prod, int64_t *n2q) {
  tnsim_status s = check_handle(h);
  if (s != TNSIM_OK) return s;
  if (sum_eps) *sum_eps = h->sum_eps;
  if (prod) *prod = h->prod_keep;
  if (n2q) *n2q = h->n2q;
  return TNSIM_OK;
}

tnsim_status tnsim_last_sweeps(tnsim_mps h, int32_t *sweeps) {
  tnsim_status s = check_handle(h);
  if (s != TNSIM_OK) return s;
  if (!sweeps) return TNSIM_E_ARG;
  *sweeps = h->last_sweeps;
  return TNSIM_OK;
}

tnsim_status tnsim_sweep_stats(tnsim_mps h, int64_t *gates, int64_t *sweeps_sum,
                               int32_t *sweeps_max) {
  tnsim_status s = check_handle(h);
  if (s != TNSIM_OK) return s;
  if (gates) *gates = h->sw_gates;
  if (sweeps_sum) *sweeps_sum = h->sw_sum;
  if (sweeps_max) *sweeps_max = h->sw_max;
  return TNSIM_OK;
}

tnsim_status tnsim_last_batch(tnsim_mps h, int32_t *out, int32_t max_gates, int32_t *n) {
  tnsim_status s = check_handle(h);
  if (s != TNSIM_OK) return s;
  if (!n || max_gates < 0 || (max_gates > 0 && !out)) return TNSIM_E_ARG;
  int cnt = (int)(h->last_batch.size() / 6);
  *n = cnt;
  int w = std::min(cnt, (int)max_gates);
  if (w > 0) memcpy(out, h->last_batch.data(), sizeof(int32_t) * 6 * w);
  return TNSIM_OK;
}

tnsim_status tnsim_export_site(tnsim_mps h, int32_t q, tnsim_c128 *host, int32_t *chiL,
                               int32_t *chiR) {
  tnsim_status s = check_handle(h);
  if (s != TNSIM_OK) return s;
  if (q < 0 || q >= h->L.n) return TNSIM_E_ARG;
  int a = h->dims[q], b = h->dims[q + 1];
  if (chiL) *chiL = a;
  if (chiR) *chiR = b;
  if (!host) return TNSIM_OK;
  size_t cnt = (size_t)a * 2 * b;
  HIPCHK(h, hipStreamSynchronize(h->stream));
  if (h->L.storage == 0) {
    HIPCHK(h, hipMemcpy(host, h->site(q), cnt * 16, hipMemcpyDeviceToHost));
  } else {
    std::vector<float> tmp(2 * cnt);
    HIPCHK(h, hipMemcpy(tmp.data(), h->site(q), cnt * 8, hipMemcpyDeviceToHost));
    for (size_t e = 0; e < cnt; e++) {
      host[e].re = tmp[2 * e];
      host[e].im = tmp[2 * e + 1];
    }
  }
  return TNSIM_OK;
}

tnsim_status tnsim_export_lambda(tnsim_mps h, int32_t bond, double *host, int32_t *chi) {
  tnsim_status s = check_handle(h);
  if (s != TNSIM_OK) return s;
  if (bond < 0 || bond >= h->L.n - 1) return TNSIM_E_ARG;
  int c = h->dims[bond + 1];
  if (chi) *chi = c;
  if (!host) return TNSIM_OK;
  HIPCHK(h, hipStreamSynchronize(h->stream));
  HIPCHK(h, hipMemcpy(host, h->lam(bond), sizeof(double) * c, hipMemcpyDeviceToHost));
  return TNSIM_OK;
}

tnsim_status tnsim_import_state(tnsim_mps h, const tnsim_c128 *const *sites,
                                const double *const *lambdas, const int32_t *chis) {
  tnsim_status s = check_handle(h);
  if (s != TNSIM_OK) return s;
  h->state_version++;
  const int n = h->L.n;
  if (!sites || !chis || (n > 1 && !lambdas)) return TNSIM_E_ARG;
  if (chis[0] != 1 || chis[n] != 1) return TNSIM_E_ARG;
  for (int q = 0; q < n; q++) {
    if (!sites[q] || chis[q + 1] < 1) return TNSIM_E_ARG;
    if (q + 1 < n && !lambdas[q]) return TNSIM_E_ARG;
  }
  for (int q = 1; q < n; q++)
    if (chis[q] > h->L.dimcap[q]) return TNSIM_E_CAPACITY;
  HIPCHK(h, hipStreamSynchronize(h->stream));
  for (int q = 0; q < n; q++) {
    size_t cnt = (size_t)chis[q] * 2 * chis[q + 1];
    if (h->L.storage == 0) {
      HIPCHK(h, hipMemcpy(h->site(q), sites[q], cnt * 16, hipMemcpyHostToDevice));
    } else {
      std::vector<float> tmp(2 * cnt);
      for (size_t e = 0; e < cnt; e++) {
        tmp[2 * e] = (float)sites[q][e].re;
        tmp[2 * e + 1] = (float)sites[q][e].im;
      }
      HIPCHK(h, hipMemcpy(h->site(q), tmp.data(), cnt * 8, hipMemcpyHostToDevice));
    }
  }
  for (int b = 0; b < n - 1; b++)
    HIPCHK(h, hipMemcpy(h->lam(b), lambdas[b], sizeof(double) * chis[b + 1],
                        hipMemcpyHostToDevice));
  HIPCHK(h, hipMemcpy(h->dims_dev(), chis, sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice));
  h->dims.assign(chis, chis + n + 1);
  return TNSIM_OK;
}

size_t tnsim_grad_workspace_bytes(const tnsim_config *cfg, int32_t n_segments,
                                  int32_t max_segment_gates, int32_t n_params) {
  if (!valid_config(cfg) || n_segments < 1 || max_segment_gates < 1 || n_params < 0) return 0;
  Layout L = make_layout(*cfg);
  return grad_layout(L, n_segments, max_segment_gates, n_params).total;
}

tnsim_status tnsim_forward_checkpointed(tnsim_mps h, void *dev_ws, size_t ws_bytes,
                                        const tnsim_gate *circuit, int32_t n_gates,
                                        const int32_t *param_of_gate, const int32_t *rot_axis,
                                        const double *angles, int32_t n_params,
                                        const int32_t *segment_start, int32_t n_segments,
                                        const char *const *paulis, const double *coeffs,
                                        int32_t n_terms, double *loss) {
  tnsim_status s = check_handle(h);
  if (s != TNSIM_OK) return s;
  h->state_version++;
  const int n = h->L.n;
  if (!dev_ws || !loss || n_gates < 0 || (n_gates > 0 && (!circuit || !param_of_gate)) ||
      n_params < 0 || (n_params > 0 && (!angles || !rot_axis)) || n_segments < 1 ||
      !segment_start || n_terms < 1 || !paulis || !coeffs)
    return TNSIM_E_ARG;
  if (h->cfg.precision != TNSIM_FP64) return TNSIM_E_ARG;  // the adjoint records float64
  if (reinterpret_cast<uintptr_t>(dev_ws) % ALIGN) return TNSIM_E_ARG;
  if (segment_start[0] != 0) return TNSIM_E_ARG;
  for (int p = 0; p < n_params; p++)
    if (!std::isfinite(angles[p])) return TNSIM_E_ARG;
  int max_seg = 0;
  for (int sg = 0; sg < n_segments; sg++) {
    int a = segment_start[sg], b = sg + 1 < n_segments ? segment_start[sg + 1] : n_gates;
    if (a > b || b > n_gates) return TNSIM_E_ARG;
    max_seg = std::max(max_seg, b - a);
  }
  for (int g = 0; g < n_gates; g++) {
    int a = circuit[g].q0, b = circuit[g].q1, p = param_of_gate[g];
    if (a < 0 || a >= n || b < -1 || b >= n || a == b) return TNSIM_E_ARG;
    if (b >= 0 && std::abs(a - b) != 1) return TNSIM_E_NONLOCAL;
    if (p >= n_params || (p >= 0 && (b >= 0 || rot_axis[p] < 0 || rot_axis[p] > 2)))
      return TNSIM_E_ARG;
    if (p < 0 && !finite_gate(circuit[g])) return TNSIM_E_ARG;
  }
  std::vector<std::vector<double2>> tabs(n_terms);
  std::vector<std::vector<char>> isIs(n_terms);
  for (int t = 0; t < n_terms; t++) {
    if (!paulis[t]) return TNSIM_E_ARG;
    if (pauli_table(paulis[t], n, tabs[t], isIs[t]) != TNSIM_OK) return TNSIM_E_ARG;
  }
  GradState G = grad_layout(h->L, n_segments, std::max(max_seg, 1), n_params);
  if (ws_bytes < G.total) return TNSIM_E_CAPACITY;
  G.ws = (char *)dev_ws;
  G.ws_bytes = ws_bytes;
  G.gates.assign(circuit, circuit + n_gates);
  G.param.assign(param_of_gate, param_of_gate + n_gates);
  G.axis.assign(n_gates, -1);
  for (int g = 0; g < n_gates; g++)
    if (G.param[g] >= 0) G.axis[g] = rot_axis[G.param[g]];
  G.angles.assign(angles, angles + n_params);
  G.seg_start.assign(segment_start, segment_start + n_segments);
  G.paulis.clear();
  for (int t = 0; t < n_terms; t++) G.paulis.emplace_back(paulis[t], paulis[t] + n);
  G.coeffs.assign(coeffs, coeffs + n_terms);
  G.ckpt_dims.assign(n_segments + 1, {});
  h->grad = std::move(G);
  GradState &GS = h->grad;
  s = init_state(h);
  if (s != TNSIM_OK) return s;
  for (int sg = 0; sg < n_segments; sg++) {
    s = save_ckpt(h, sg);
    if (s != TNSIM_OK) return s;
    int a = GS.seg_start[sg], b = sg + 1 < n_segments ? GS.seg_start[sg + 1] : n_gates;
    for (int g = a; g < b; g++) {
      s = grad_apply(h, g, nullptr);
      if (s != TNSIM_OK) return s;
    }
  }
  s = save_ckpt(h, n_segments);
  if (s != TNSIM_OK) return s;
  double2 den, num;
  s = transfer(h, h, h, nullptr, nullptr, &den);
  if (s != TNSIM_OK) return s;
  double L = 0.0;
  for (int t = 0; t < n_terms; t++) {
    s = transfer(h, h, h, tabs[t].data(), isIs[t].data(), &num);
    if (s != TNSIM_OK) return s;
    L += coeffs[t] * num.x / den.x;
  }
  GS.loss = L;
  GS.ready = true;
  *loss = L;
  return TNSIM_OK;
}

tnsim_status tnsim_backward(tnsim_mps h, double dloss, double *grad_angles) {
  tnsim_status s = check_handle(h);
  if (s != TNSIM_OK) return s;
  h->state_version++;
  GradState &G = h->grad;
  if (!G.ready || (G.n_params > 0 && !grad_angles)) return TNSIM_E_ARG;
  const int n = h->L.n;
  hipStream_t st = h->stream;
  // zero the cotangents and gradients
  for (int q = 0; q < n; q++)
    launch_fill_zero(st, G.ws + G.cot_site[q], align_up(h->L.site_cap[q] * sizeof(double2), 16));
  for (int b = 0; b < n - 1; b++)
    launch_fill_zero(st, G.ws + G.cot_lam[b], align_up(sizeof(double) * h->L.bondcap[b], 16));
  launch_fill_zero(st, G.ws + G.grad, align_up(sizeof(double) * std::max(G.n_params, 1), 16));
  LAUNCHCHK(h, "backward init");
  // the final state: loss = sum_t c_t N_t / D
  s = restore_ckpt(h, G.n_seg);
  if (s != TNSIM_OK) return s;
  double2 den, num;
  s = transfer(h, h, h, nullptr, nullptr, &den);
  if (s != TNSIM_OK) return s;
  const double D = den.x;
  std::vector<double2> tab;
  std::vector<char> isI;
  for (size_t t = 0; t < G.paulis.size(); t++) {
    pauli_table(G.paulis[t].c_str(), n, tab, isI);
    s = loss_cotangent_term(h, tab.data(), isI.data(), dloss * G.coeffs[t] / D);
    if (s != TNSIM_OK) return s;
  }
  {  // d(N/D): the norm term, weight -L/D
    std::vector<char> allI(n, 1);
    std::vector<double2> idt(4 * n, make_double2(0, 0));
    s = loss_cotangent_term(h, idt.data(), allI.data(), -dloss * G.loss / D);
    if (s != TNSIM_OK) return s;
  }
  const int n_gates = (int)G.gates.size();
  std::vector<GradRec> recs;
  for (int sg = G.n_seg - 1; sg >= 0; sg--) {
    s = restore_ckpt(h, sg);
    if (s != TNSIM_OK) return s;
    int a = G.seg_start[sg], b = sg + 1 < G.n_seg ? G.seg_start[sg + 1] : n_gates;
    recs.assign(b - a, GradRec{});
    for (int g = a; g < b; g++) {
      recs[g - a].off = G.rec0 + G.rec_stride * (size_t)(g - a);
      s = grad_apply(h, g, &recs[g - a]);
      if (s != TNSIM_OK) return s;
    }
    for (int g = b - 1; g >= a; g--) {
      const GradRec &R = recs[g - a];
      s = R.kind == 2 ? adjoint_2q(h, R) : adjoint_1q(h, R);
      if (s != TNSIM_OK) return s;
    }
  }
  s = restore_ckpt(h, G.n_seg);
  if (s != TNSIM_OK) return s;
  if (G.n_params > 0)
    HIPCHK(h, hipMemcpy(grad_angles, G.ws + G.grad, sizeof(double) * G.n_params,
                        hipMemcpyDeviceToHost));
  return TNSIM_OK;
}

tnsim_status tnsim_profile(tnsim_mps h, int32_t enable) {
  tnsim_status s = check_handle(h);
  if (s != TNSIM_OK) return s;
  HIPCHK(h, hipStreamSynchronize(h->stream));
  prof_drain(h);
  if (enable) {
    for (auto &k : h->kstat) k = tnsim_kernel_stat{0.0, 0, 0.0, 0.0};
    h->sw_gates = h->sw_sum = 0;
    h->sw_max = 0;
    launch_fill_zero(h->stream, h->at<void>(h->L.ctr_off),
                     align_up(sizeof(unsigned long long) * CTR_COUNT, 16));
    LAUNCHCHK(h, "profile");
    HIPCHK(h, hipStreamSynchronize(h->stream));
  }
  h->prof = enable != 0;
  return TNSIM_OK;
}

tnsim_status tnsim_probe_fp64(tnsim_mps h, int32_t unit, int32_t iters, double *tflops_out) {
  tnsim_status s = check_handle(h);
  if (s != TNSIM_OK) return s;
  if (unit < 0 || unit > 3 || iters < 1 || iters > (1 << 20) || !tflops_out) return TNSIM_E_ARG;
  int dev = 0, cus = 0;
  HIPCHK(h, hipGetDevice(&dev));
  HIPCHK(h, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const int groups = 8 * std::max(cus, 1);  // eight workgroups of four wavefronts per CU
  double *out = nullptr;
  HIPCHK(h, hipMalloc(&out, sizeof(double) * 256 * (size_t)groups));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  double flops = 0.0;
  float ms = 0.0f;
  if (e == hipSuccess) {
    launch_probe(h->stream, unit, groups, iters, out);  // warm-up
    e = hipEventRecord(e0, h->stream);
  }
  if (e == hipSuccess) {
    flops = launch_probe(h->stream, unit, groups, iters, out);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(e1, h->stream);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  hipFree(out);
  if (e != hipSuccess) return fail(h, e, "probe");
  *tflops_out = ms > 0.0f ? flops / (ms * 1e-3) / 1e12 : 0.0;
  return TNSIM_OK;
}

tnsim_status tnsim_profile_read(tnsim_mps h, tnsim_kernel_stat *out) {
  tnsim_status s = check_handle(h);
  if (s != TNSIM_OK) return s;
  if (!out) return TNSIM_E_ARG;
  HIPCHK(h, hipStreamSynchronize(h->stream));
  prof_drain(h);
  unsigned long long ctr[CTR_COUNT];
  HIPCHK(h, hipMemcpy(ctr, h->at<void>(h->L.ctr_off), sizeof ctr, hipMemcpyDeviceToHost));
  for (int k = 0; k < TNSIM_K_COUNT; k++) out[k] = h->kstat[k];
  out[TNSIM_K_GRAM].flops = (double)ctr[CTR_GRAM_FLOP];
  out[TNSIM_K_GRAM].bytes = (double)ctr[CTR_GRAM_BYTE];
  // one 2x2 rotation updates two columns and two rows of G and two columns of
  // V (64 entries each); an entry update is 2 complex multiply-adds = 16 flops
  out[TNSIM_K_EIG].flops = (double)ctr[CTR_EIG_ROT] * 6.0 * PW * 16.0;
  out[TNSIM_K_EIG].bytes = 0.0;
  out[TNSIM_K_ROT].flops = (double)ctr[CTR_ROT_FLOP];
  out[TNSIM_K_ROT].bytes = (double)ctr[CTR_ROT_BYTE];
  return TNSIM_OK;
}

tnsim_status tnsim_autotune(tnsim_mps h, int32_t *table_out) {
  tnsim_status s = check_handle(h);
  if (s != TNSIM_OK) return s;
  const Layout &L = h->L;
  HIPCHK(h, hipStreamSynchronize(h->stream));
  prof_drain(h);
  // Synthetic gates of the largest shape the handle holds: X (rows x cols)
  // zeroed, every pair flagged for rotation, V zeroed.
  const int cols = L.cols_pad_max, rows = L.cmax;
  const int npairs = cols / PW;
  const int want[TNSIM_TUNE_BUCKETS] = {32, 128, 512, 1600};
  const int cand[4] = {64, 128, 256, 512};
  std::vector<GateDesc> D(L.nslots);
  for (int g = 0; g < L.nslots; g++) {
    GateDesc &d = D[g];
    memset(&d, 0, sizeof d);
    char *sl = h->slot(g);
    d.rows = rows;
    d.cols = cols;
    d.m = rows;
    d.n = cols;
    d.ldx = L.ldx_max;
    d.colsPad = cols;
    d.nblk = cols / BW;
    d.X = (double2 *)(sl + L.x_off);
    d.V = (double2 *)(sl + L.v_off);
    d.pairFlag = (int *)(sl + L.pf_off);
    d.sc = (SlotScalars *)(sl + L.sc_off);
    d.gpStride = L.npairs_max;
    launch_fill_zero(h->stream, d.X, sizeof(double2) * (size_t)L.ldx_max * cols);
    launch_fill_zero(h->stream, d.V, sizeof(double2) * (size_t)npairs * PW * PW);
  }
  std::vector<int32_t> ones(npairs, 1);
  SlotScalars act{};
  act.active = 1;
  for (int g = 0; g < L.nslots; g++) {
    HIPCHK(h, hipMemcpyAsync(D[g].pairFlag, ones.data(), sizeof(int32_t) * npairs,
                             hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipMemcpyAsync(D[g].sc, &act, sizeof act, hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));  // the host sources are reused
  }
  GateDesc *ddev = h->at<GateDesc>(L.desc_off);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(h, hipEventCreate(&e0));
  HIPCHK(h, hipEventCreate(&e1));
  for (int bk = 0; bk < TNSIM_TUNE_BUCKETS; bk++) {
    const int ng = std::max(1, std::min(L.nslots, (want[bk] + npairs - 1) / npairs));
    int best = 0;
    float best_ms = 0.0f;
    for (int ci = 0; ci < 4; ci++) {
      const int rr = cand[ci];
      for (int g = 0; g < ng; g++) D[g].rotRows = rr;
      memcpy(h->pin, D.data(), sizeof(GateDesc) * ng);
      HIPCHK(h, hipMemcpyAsync(ddev, h->pin, sizeof(GateDesc) * ng, hipMemcpyHostToDevice,
                               h->stream));
      launch_rot(h->stream, ddev, ng, 0, npairs, rows, 0, rr);  // warm-up
      HIPCHK(h, hipEventRecord(e0, h->stream));
      for (int r = 0; r < 3; r++) launch_rot(h->stream, ddev, ng, r, npairs, rows, 0, rr);
      HIPCHK(h, hipEventRecord(e1, h->stream));
      LAUNCHCHK(h, "autotune");
      HIPCHK(h, hipEventSynchronize(e1));
      float ms = 0.0f;
      HIPCHK(h, hipEventElapsedTime(&ms, e0, e1));
      if (best == 0 || ms < best_ms) {
        best = rr;
        best_ms = ms;
      }
    }
    h->tune_rot_rows[bk] = best;
    if (table_out) table_out[bk] = best;
    // pair Grams: rows split over 1, 2, 4, ... workgroups (partials summed by
    // the pair solve), within the partial-Gram pool and 32 rows per chunk
    int best_ks = 0;
    best_ms = 0.0f;
    for (int ks = 1; ks <= KSPLIT_MAX; ks *= 2) {
      if (ks > 1 && (ks > (rows + 31) / 32 || (long long)ng * ks * L.npairs_max > L.gp_blocks))
        break;
      for (int g = 0; g < ng; g++)
        D[g].Gp = h->at<double2>(L.gp_off) + (size_t)g * ks * L.npairs_max * PW * PW;
      memcpy(h->pin, D.data(), sizeof(GateDesc) * ng);
      HIPCHK(h, hipMemcpyAsync(ddev, h->pin, sizeof(GateDesc) * ng, hipMemcpyHostToDevice,
                               h->stream));
      launch_gram(h->stream, ddev, ng, 0, npairs, ks);  // warm-up
      HIPCHK(h, hipEventRecord(e0, h->stream));
      for (int r = 0; r < 3; r++) launch_gram(h->stream, ddev, ng, r, npairs, ks);
      HIPCHK(h, hipEventRecord(e1, h->stream));
      LAUNCHCHK(h, "autotune");
      HIPCHK(h, hipEventSynchronize(e1));
      float ms = 0.0f;
      HIPCHK(h, hipEventElapsedTime(&ms, e0, e1));
      if (best_ks == 0 || ms < best_ms) {
        best_ks = ks;
        best_ms = ms;
      }
    }
    h->tune_gram_ks[bk] = best_ks;
    if (table_out) table_out[TNSIM_TUNE_BUCKETS + bk] = best_ks;
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  return TNSIM_OK;
}

tnsim_status tnsim_set_launch_table(tnsim_mps h, const int32_t *table) {
  tnsim_status s = check_handle(h);
  if (s != TNSIM_OK) return s;
  if (!table) return TNSIM_E_ARG;
  for (int bk = 0; bk < TNSIM_TUNE_BUCKETS; bk++) {
    const int v = table[bk], k = table[TNSIM_TUNE_BUCKETS + bk];
    if (v != 0 && v != 64 && v != 128 && v != 256 && v != 512) return TNSIM_E_ARG;
    if (k < 0 || k > KSPLIT_MAX || (k & (k - 1)) != 0) return TNSIM_E_ARG;
  }
  for (int bk = 0; bk < TNSIM_TUNE_BUCKETS; bk++) {
    h->tune_rot_rows[bk] = table[bk];
    h->tune_gram_ks[bk] = table[TNSIM_TUNE_BUCKETS + bk];
  }
  return TNSIM_OK;
}

const char *tnsim_status_string(tnsim_status st) {
  switch (st) {
    case TNSIM_OK: return "ok";
    case TNSIM_E_ARG: return "invalid argument";
    case TNSIM_E_NONLOCAL: return "two-qubit gate on non-neighbouring qubits";
    case TNSIM_E_OVERLAP: return "layer uses a qubit twice";
    case TNSIM_E_CAPACITY: return "arena or bond capacity too small";
    case TNSIM_E_DEVICE: return "HIP device failure";
    case TNSIM_E_NOCONV: return "Jacobi SVD did not converge";
  }
  return "unknown status";
}

const char *tnsim_last_error(tnsim_mps h) {
  if (!h) return g_create_error.c_str();
  return h->err.c_str();
}

}  // extern "C"
