// Host runtime of liblrdm: argument validation, the gate-pass scheduler, the compression
// pipeline (Gram -> FP64 eigensolve -> projection) and the output reductions, behind the C ABI
// declared in include/lrdm.h.  No device memory is allocated here: every device buffer is
// carved out of the caller's workspace.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "lrdm_internal.h"

using namespace lrdm;

namespace {

thread_local std::string g_last_error;

constexpr size_t kAlign = 256;
constexpr int kMaxTerms = 65536;
constexpr int kSampleBatch = 1 << 20;
constexpr size_t kPauliPartDoubles = 4u << 20;
constexpr int kZBlocks = 256;
constexpr int kMaxTimed = 8192;
constexpr int kMaxApplyTerms = 4096;
constexpr int kMaxSparse = 32768;   // sparse initial state entries (staged in the terms region)

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
int next_pow2(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

struct Layout {
  int r_pad, m_pad, ld, F_max, FO_max;
  size_t state_bytes;
  size_t off_info, off_part, off_S, off_P, off_Y, off_lam, off_W, off_out, off_pbuf, off_cdf, off_bsum, off_terms, off_pauli, off_unif, off_samp, total;
  bool adjoint;        // reverse sweep available (fused form, m_max * r_pad <= 64)
  size_t off_adj, rec_bytes;
  size_t off_chain;    // fused form: W of the pending projection, the next W (FP64) and scratch
  // overlapped compressions (LRDM_FLAG_OVERLAP): a second W slot in the bulk precision (the
  // chain region then holds a fourth block, FP64 W of slot 1), two G4 slots, the FP64 scratch
  // of the pair transform and the partials of the 4-way Gram
  bool overlap;
  size_t off_W2, off_S4, off_T4, off_part4;
  // fused form, channels on a qubit pair: W of the 4-way view (4 r_pad x 4 r_pad) and the FP64
  // operator blocks the eigensolver reads (E_a^H E_b and E_a); the 4-way Gram uses S4 and part4
  size_t off_W4, off_M4;
};

bool compute_layout(int n, int r_max, lrdm_dtype dt, int m_max, unsigned flags, Layout& L,
                    std::string& why) {
  if (n < 1 || n > 30) { why = "n must be in [1, 30]"; return false; }
  if (r_max < 1 || r_max > 64) { why = "r_max must be in [1, 64]"; return false; }
  const bool plain = flags & LRDM_FLAG_PLAIN;
  if (m_max < 1 || m_max > (plain ? 16 : 4)) {
    why = plain ? "m_max must be in [1, 16] (plain form)" : "m_max must be in [1, 4] (fused form)";
    return false;
  }
  if (dt != LRDM_C64 && dt != LRDM_C128) { why = "unknown dtype"; return false; }
  L.r_pad = std::max(8, next_pow2(r_max));
  L.m_pad = next_pow2(m_max);
  if (m_max * L.r_pad > kMaxEig) { why = "m_max * r_pad exceeds 128 (largest Gram order)"; return false; }
  if (dt == LRDM_C128 && L.r_pad > 32) { why = "complex128 supports r_pad <= 32"; return false; }
  L.overlap = flags & LRDM_FLAG_OVERLAP;
  if (L.overlap && plain) { why = "LRDM_FLAG_OVERLAP applies to the fused form"; return false; }
  if (L.overlap && n < 2) { why = "LRDM_FLAG_OVERLAP needs n >= 2"; return false; }
  L.ld = plain ? L.m_pad * L.r_pad : L.r_pad;
  if (plain && 2 * L.ld > (dt == LRDM_C64 ? 256 : 128)) { why = "plain form exceeds the GEMM width"; return false; }
  L.F_max = std::max(4 * L.r_pad, 2 * L.ld);
  L.FO_max = 4 * L.r_pad;
  const size_t cs = (dt == LRDM_C64) ? 8 : 16;   // bytes per complex
  const size_t rs = cs / 2;                        // bytes per real
  const size_t rows = 1ull << n;
  L.state_bytes = rows * L.ld * cs;
  const int NT = L.F_max / 16;
  const int NUP = NT * (NT + 1) / 2;
  const int nb = gram_blocks(n, 1);
  const int Fc = L.F_max / 2;
  const int N = kMaxEig;
  size_t o = 0;
  auto take = [&](size_t bytes) { const size_t at = o; o = align_up(o + bytes); return at; };
  L.off_info = take(sizeof(DevInfo));
  L.off_part = take((size_t)nb * NUP * 256 * rs);
  L.off_S = take((size_t)Fc * Fc * 16);
  L.off_P = take((size_t)N * (N + 1) / 2 * 16);
  L.off_Y = take(kEigYDoubles * 8);
  L.off_lam = take(N * 8);
  L.off_W = take((size_t)(L.F_max / 2) * (L.FO_max / 2) * cs);
  L.off_out = take(4096 * 8);
  L.off_pbuf = take(rows * 8 + (size_t)kZBlocks * 64 * 8);
  L.off_cdf = take(rows * 8);
  L.off_bsum = take(((rows + 1023) / 1024) * 8);
  L.off_terms = take((size_t)kMaxTerms * 16 + (size_t)(kMaxTerms + 1) * 4);
  L.off_pauli = take(kPauliPartDoubles * 8);
  L.off_unif = take((size_t)kSampleBatch * 8);
  L.off_samp = take((size_t)kSampleBatch * 8);
  const int N_rec = m_max * L.r_pad;
  L.adjoint = !plain && N_rec <= kRecMaxN;
  L.off_adj = L.adjoint ? take(adj_doubles(L.r_pad, N_rec) * 8) : 0;
  L.off_chain = plain ? 0 : take((size_t)(L.overlap ? 4 : 3) * (2 * L.r_pad) * (2 * L.r_pad) * 16);
  L.off_W2 = L.off_S4 = L.off_T4 = L.off_part4 = L.off_W4 = L.off_M4 = 0;
  if (!plain && n >= 2) {
    const size_t c4 = 4 * (size_t)L.r_pad;
    const size_t nt = c4 / 16;   // 16-wide real tiles across one half (4c reals)
    const size_t nup = nt * (nt + 1) / 2;
    L.off_S4 = take(2 * c4 * c4 * 16);
    L.off_part4 = take(std::max(((size_t)2 * gram4_blocks_halves(n) * nup + (size_t)gram4_blocks_cross(n) * nt * nt) *
                                    256 * rs,
                                rs == 4 ? gram4_stream_reals(n) * 4 : (size_t)0));
    L.off_W4 = take(c4 * c4 * cs);
    L.off_M4 = take((size_t)(16 * 16 + 4 * 16) * 16);
  }
  if (L.overlap) {
    const size_t c2 = 2 * (size_t)L.r_pad;
    L.off_W2 = take((size_t)(L.F_max / 2) * (L.FO_max / 2) * cs);
    L.off_T4 = take(3 * c2 * c2 * 16);
  }
  L.rec_bytes = L.adjoint ? align_up(record_doubles(N_rec) * 8) : 0;
  L.total = o;
  return true;
}

struct PendingGate {
  int type;          // GateOpType
  int q0, q1;        // qubits (q1 = -1 for 1q); OP_WEIGHT uses neither
  uint32_t qmask;    // qubits the gate touches (all qubits for OP_WEIGHT)
  std::vector<double> coef;
};

// Launches recorded instead of issued while a handle belongs to a batch being recorded
// (complex64 only).  Items keep the handle's issue order; job structs hold every argument.
enum RecKind : int { REC_RESET = 0, REC_GATE = 1, REC_GRAM = 2, REC_REDUCE = 3, REC_EIG = 4, REC_PROJ = 5 };
struct RecItem {
  int kind;
  int cls;          // F (Gram), N (eigensolve), FO (projection)
  int kmax;         // eigensolve
  uint32_t blocks;
  size_t shm;       // gate pass
  size_t idx;       // index into the per-kind vector
};
struct Recorder {
  std::vector<RecItem> items;
  std::vector<ResetJob> resets;
  std::vector<GateJob<float>> gates;
  std::vector<GramJob<float>> grams;
  std::vector<ReduceJob<float>> reds;
  std::vector<EigJob<float>> eigs;
  std::vector<ProjJob<float>> projs;
};

}  // namespace

void lrdm::set_last_error(const char* msg) { g_last_error = msg; }

struct lrdm_ctx {
  int n = 0, r_max = 0, m_max = 0;
  lrdm_dtype dt = LRDM_C64;
  unsigned flags = 0;
  bool plain = false;
  Layout lay{};
  void* state = nullptr;
  char* work = nullptr;
  hipStream_t stream = nullptr;
  int ncols = 0;      // active columns in the state layout
  int c_bound = 1;    // host bound on non-zero columns
  bool poisoned = false;
  std::string err;
  std::vector<PendingGate> gates;
  bool chan_pending = false;
  int chan_q = 0;
  Channel chan{};
  // fused form: the pending channel acts on the pair (chan_q, chan_q1) with the 4 x 4 operators
  // in pair_e; pair_stage holds E_a^H E_b and E_a for the upload
  bool chan_pair = false;
  int chan_q1 = -1;
  std::vector<double> pair_e, pair_stage;
  // timing
  int timing_class = -1;
  std::vector<hipEvent_t> ev;
  std::vector<int> ev_launches;   // launches inside each recorded event pair
  int ev_used = 0;
  // host staging
  std::vector<uint64_t> term_stage;
  // batch recording (non-null between lrdm_batch_begin and lrdm_batch_end)
  Recorder* rec = nullptr;
  // fused form: the projection of the last compression is deferred while only channels on the
  // same qubit follow (chained compressions); pend_q is that qubit
  bool proj_pending = false;
  int pend_q = -1;
  bool last_w_next = false;   // the last compression's own W is in the "next" buffer (chained)
  int pend_skip = 0;          // zero blocks of the pending projection's W (see reach_skip)
  // overlapped compressions: the passes over L of a compression (Gram, 4-way Gram, projection)
  // run on gemm, the eigensolves and their small FP64 products on aux, two streams of the handle
  // on disjoint sets of CUs (an eigensolve work-group then never waits for, nor shares a CU
  // with, the GEMMs).  ev_a2g orders gemm after the caller's stream, ev_g2b aux after gemm (S or
  // G4 ready), ev_b2g gemm (or the caller's stream) after aux (W ready, aux done with the
  // eigensolver buffers), ev_g2a the caller's stream after gemm.  wslot is the W slot of the
  // pending projection, s4slot the next G4 slot.
  bool overlap = false;
  hipStream_t aux = nullptr, gemm = nullptr;
  hipEvent_t ev_a2g = nullptr, ev_g2b = nullptr, ev_b2g = nullptr, ev_g2a = nullptr;
  int wslot = 0;
  int s4slot = 0;
  int gemm_cus = 256;   // CUs the gemm stream may use
  int ncu = 256;        // CUs of the device
  lrdm_tuning tune{};   // autotuned launch shapes (0 = default)
  int aux_cus = 0;      // CUs of the aux stream (overlap mode)
  // the caller's stream may hold work that gemm has not been ordered after (set wherever the
  // caller's stream is joined to the handle's streams, which precedes all work queued there)
  bool main_dirty = true;

  template <class P> P* ws(size_t off) { return reinterpret_cast<P*>(work + off); }
  // W of slot s in the bulk precision and in FP64 (the chain region: slot 0, the next W, scratch,
  // slot 1)
  template <class T> cx_t<T>* w_bulk(int s) { return ws<cx_t<T>>(s ? lay.off_W2 : lay.off_W); }
  double* chain_block(int i) { return ws<double>(lay.off_chain) + (size_t)i * 2 * (2 * lay.r_pad) * (2 * lay.r_pad); }
  double* wp64(int s) { return chain_block(s ? 3 : 0); }
};

namespace {

lrdm_status fail(lrdm_t h, lrdm_status st, const std::string& msg) {
  g_last_error = msg;
  if (h) h->err = msg;
  return st;
}

lrdm_status hip_check(lrdm_t h, hipError_t e, const char* where) {
  if (e == hipSuccess) return LRDM_OK;
  h->poisoned = true;
  return fail(h, LRDM_E_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIPCHK(h, expr)                                         \
  do {                                                          \
    lrdm_status _s = hip_check((h), (expr), #expr);             \
    if (_s != LRDM_OK) return _s;                               \
  } while (0)

lrdm_status check_usable(lrdm_t h) {
  if (!h) return fail(nullptr, LRDM_E_ARG, "null handle");
  if (h->poisoned) return fail(h, LRDM_E_STATE, "handle is poisoned by an earlier device error: " + h->err);
  return LRDM_OK;
}

// Sync the stream and check the device-side eigensolver status.
lrdm_status sync_and_check(lrdm_t h) {
  HIPCHK(h, hipStreamSynchronize(h->stream));
  if (h->overlap) {
    HIPCHK(h, hipStreamSynchronize(h->gemm));
    HIPCHK(h, hipStreamSynchronize(h->aux));
  }
  DevInfo info;
  HIPCHK(h, hipMemcpy(&info, h->ws<DevInfo>(h->lay.off_info), sizeof(info), hipMemcpyDeviceToHost));
  if (info.status != 0) {
    h->poisoned = true;
    return fail(h, LRDM_E_EIG, "eigensolver reported a non-finite or empty Gram matrix");
  }
  return LRDM_OK;
}

void timed_begin(lrdm_t h, int cls, hipStream_t s = nullptr) {
  if (h->timing_class != cls || h->ev_used + 2 > (int)h->ev.size()) return;
  hipEventRecord(h->ev[h->ev_used], s ? s : h->stream);
}
void timed_end(lrdm_t h, int cls, hipStream_t s = nullptr, int launches = 1) {
  if (h->timing_class != cls || h->ev_used + 2 > (int)h->ev.size()) return;
  hipEventRecord(h->ev[h->ev_used + 1], s ? s : h->stream);
  h->ev_launches[h->ev_used / 2] = launches;
  h->ev_used += 2;
}

// Overlap mode: work the caller's stream queues next runs after everything queued on the
// handle's two streams so far.
lrdm_status join_aux(lrdm_t h) {
  if (!h->overlap) return LRDM_OK;
  h->main_dirty = true;
  HIPCHK(h, hipEventRecord(h->ev_g2a, h->gemm));
  HIPCHK(h, hipStreamWaitEvent(h->stream, h->ev_g2a, 0));
  HIPCHK(h, hipStreamWaitEvent(h->stream, h->ev_b2g, 0));
  return LRDM_OK;
}
// The overlap mode's two streams (default priority): aux on the CUs of one XCD (the last 32 bits
// of the CU mask on this part: 8 XCDs of 32 CUs), gemm on the others.  Measured on the brickwork
// n = 20, r = 64 run: the eigensolver's kernels hand their data from one to the next through
// that XCD's L2, and no CU pair is shared between the two streams (a CU pair shares its
// instruction and scalar caches: aux CUs spread over the XCDs ran both the eigensolve and the
// GEMMs twice as slowly); the GEMM work-groups spread over the 7 remaining XCDs, whereas 16 aux
// CUs taken out of one XCD left that XCD a second round of every GEMM grid.  Where the runtime
// refuses a CU mask, both become ordinary streams (the results are the same; only the CU
// sharing differs).
constexpr int kAuxCUs = 32;
hipError_t create_overlap_streams(lrdm_t h) {
  int dev = 0, ncu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  h->ncu = ncu;
  const int aux = h->tune.aux_cus ? h->tune.aux_cus : kAuxCUs;
  if (ncu > aux && ncu - aux >= 32 && ncu <= 1024) {
    const int words = (ncu + 31) / 32;
    std::vector<uint32_t> mg(words, 0), mb(words, 0);
    for (int i = 0; i < ncu; ++i) (i >= ncu - aux ? mb : mg)[i / 32] |= 1u << (i % 32);
    if (hipExtStreamCreateWithCUMask(&h->gemm, (uint32_t)words, mg.data()) == hipSuccess &&
        hipExtStreamCreateWithCUMask(&h->aux, (uint32_t)words, mb.data()) == hipSuccess) {
      h->gemm_cus = ncu - aux;
      h->aux_cus = aux;
      return hipSuccess;
    }
    if (h->gemm) hipStreamDestroy(h->gemm);
    h->gemm = nullptr;
    (void)hipGetLastError();
  }
  h->gemm_cus = std::max(2, std::min(ncu, 256));
  h->aux_cus = 0;
  e = hipStreamCreateWithFlags(&h->gemm, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&h->aux, hipStreamNonBlocking);
  return e;
}
// work already queued on the handle's streams finishes before they and the events go
void release_overlap(lrdm_t h) {
  if (h->gemm) hipStreamSynchronize(h->gemm);
  if (h->aux) hipStreamSynchronize(h->aux);
  for (hipEvent_t* e : {&h->ev_a2g, &h->ev_g2b, &h->ev_b2g, &h->ev_g2a})
    if (*e) hipEventDestroy(*e);
  if (h->gemm) hipStreamDestroy(h->gemm);
  if (h->aux) hipStreamDestroy(h->aux);
  h->gemm = h->aux = nullptr;
}

// Overlap mode: work the gemm stream queues next runs after everything on the caller's stream.
// Only when the caller's stream has new work: the handle's CU-masked streams are blocking
// streams, so a marker on the legacy default stream would also wait for all their work and
// stall the pipeline between consecutive compressions.
lrdm_status enter_gemm(lrdm_t h) {
  if (!h->main_dirty) return LRDM_OK;
  HIPCHK(h, hipEventRecord(h->ev_a2g, h->stream));
  HIPCHK(h, hipStreamWaitEvent(h->gemm, h->ev_a2g, 0));
  h->main_dirty = false;
  return LRDM_OK;
}

bool is_unitary(const double* u, int d) {
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) {
      double re = 0, im = 0;
      for (int k = 0; k < d; ++k) {
        const double ar = u[2 * (k * d + i)], ai = -u[2 * (k * d + i) + 1];   // conj(U_ki)
        const double br = u[2 * (k * d + j)], bi = u[2 * (k * d + j) + 1];
        re += ar * br - ai * bi;
        im += ar * bi + ai * br;
      }
      if (std::fabs(re - (i == j ? 1.0 : 0.0)) > 1e-10 || std::fabs(im) > 1e-10) return false;
      if (!std::isfinite(re) || !std::isfinite(im)) return false;
    }
  return true;
}

template <class T> void fill_coef(GatePass<T>& p, int& nc, const std::vector<double>& c) {
  for (double v : c) p.coef[nc++] = (T)v;
}

// Local qubits per pass: the tile of 2^k rows x ncols complex values must fit 64 KB of LDS.
int local_budget(int n, int ncols, size_t csize) {
  int k = 0;
  while (k < 8 && k < n && ((size_t)ncols << (k + 1)) * csize <= 65536) ++k;
  return k;
}

// Register phases of a fused pass (see GatePass).  One-qubit gates join the current phase in
// list order; a gate opens a new phase when the phase already has 4 gates, a gate on the same
// qubit, or a diagonal operation on that qubit (which must act before it).  A diagonal
// operation then moves, within the phases its qubits' gates allow, to one where the most of its
// qubits are gate slots.  The register slots of a phase are its gates' slots, then local slots
// of qubits its diagonal operations act on, then any others; register bits without a gate get
// the identity.  The diagonal operations with real phases whose qubits are both register bits
// multiply into one table of 16 phases per phase (a CZ layer costs one multiply per element),
// the others stay listed.  Coefficients appended here (identity, tables) need room in coef; without it, or with
// other operation types, the pass keeps the per-operation sweeps.
constexpr int kPhaseRegs = 4;

template <class T>
void build_phases(GatePass<T>& p, int& nc) {
  p.n_phases = 0;
  if (p.k < kPhaseRegs || p.k > 8) return;
  for (int o = 0; o < p.n_ops; ++o)
    if (p.op_type[o] != OP_1Q && p.op_type[o] != OP_DIAG1 && p.op_type[o] != OP_DIAG2) return;
  struct Phase {
    int ng = 0, gslot[kPhaseRegs] = {}, gcoef[kPhaseRegs] = {};
    uint32_t gq = 0, dq = 0;   // qubits with a gate / touched by a diagonal operation
    std::vector<int> diag;
  };
  auto qmask = [&](int o) {
    return (1u << p.op_a[o]) | (p.op_type[o] == OP_DIAG2 ? (1u << p.op_b[o]) : 0u);
  };
  std::vector<Phase> ph(1);
  for (int o = 0; o < p.n_ops; ++o) {
    if (p.op_type[o] == OP_1Q) {
      const int slot = p.op_a[o];
      const uint32_t qb = 1u << p.local_q[slot];
      Phase* c = &ph.back();
      if (c->ng == kPhaseRegs || (c->gq & qb) || (c->dq & qb)) {
        ph.emplace_back();
        c = &ph.back();
      }
      c->gslot[c->ng] = slot;
      c->gcoef[c->ng] = p.op_coef[o];
      ++c->ng;
      c->gq |= qb;
    } else {
      ph.back().diag.push_back(o);
      ph.back().dq |= qmask(o);
    }
  }
  const int nph = (int)ph.size();
  if (nph > kGateMaxPhases) return;
  // move each diagonal operation to the phase in its window with the most of its qubits gated
  std::vector<std::vector<int>> diag(nph);
  for (int c = 0; c < nph; ++c)
    for (int o : ph[c].diag) {
      const uint32_t qm = qmask(o);
      int lo = c, hi = c;
      while (lo > 0 && !(ph[lo].gq & qm)) --lo;
      while (hi + 1 < nph && !(ph[hi + 1].gq & qm)) ++hi;
      int best = c, best_n = __builtin_popcount(ph[c].gq & qm);
      for (int t = lo; t <= hi; ++t) {
        const int n = __builtin_popcount(ph[t].gq & qm);
        if (n > best_n) best = t, best_n = n;
      }
      diag[best].push_back(o);
    }
  bool pad = false;
  for (const Phase& c : ph) pad |= c.ng < kPhaseRegs;
  int need = pad ? 8 : 0;
  const int ident = nc;
  if (nc + need > kGateMaxCoef) return;
  if (pad) {
    const T id[8] = {1, 0, 0, 0, 0, 0, 1, 0};
    for (int i = 0; i < 8; ++i) p.coef[nc++] = id[i];
  }
  int nd_total = 0;
  for (int i = 0; i < nph; ++i) {
    const Phase& c = ph[i];
    uint32_t dq = 0;
    for (int o : diag[i]) dq |= qmask(o);
    int slots[8], ns = 0;
    for (int g = 0; g < c.ng; ++g) slots[ns++] = c.gslot[g];
    auto taken = [&](int j) {
      for (int t = 0; t < ns; ++t)
        if (slots[t] == j) return true;
      return false;
    };
    for (int j = 0; j < p.k && ns < kPhaseRegs; ++j)
      if ((dq >> p.local_q[j]) & 1u && !taken(j)) slots[ns++] = j;
    for (int j = 0; j < p.k && ns < kPhaseRegs; ++j)
      if (!taken(j)) slots[ns++] = j;
    for (int j = 0; j < p.k; ++j)   // the thread-index slots, ascending
      if (!taken(j)) slots[ns++] = j;
    uint32_t w = 0;
    for (int t = 0; t < p.k; ++t) w |= (uint32_t)slots[t] << (t < kPhaseRegs ? 4 * t : 16 + 4 * (t - kPhaseRegs));
    p.ph_word[i] = w;
    int gc[kPhaseRegs];
    for (int g = 0; g < kPhaseRegs; ++g) gc[g] = g < c.ng ? c.gcoef[g] : ident;
    p.ph_gc[i][0] = (uint32_t)gc[0] | ((uint32_t)gc[1] << 16);
    p.ph_gc[i][1] = (uint32_t)gc[2] | ((uint32_t)gc[3] << 16);
    auto reg = [&](int q) {
      for (int t = 0; t < kPhaseRegs; ++t)
        if (p.local_q[slots[t]] == q) return t;
      return -1;
    };
    // listed: real phases first, then complex ones
    auto is_real = [&](int o) {
      const T* u = p.coef + p.op_coef[o];
      const int nphase = p.op_type[o] == OP_DIAG2 ? 4 : 2;
      for (int t = 0; t < nphase; ++t)
        if (u[2 * t + 1] != 0) return false;
      return true;
    };
    std::vector<int> regd, rest;
    for (int o : diag[i]) {
      const bool two = p.op_type[o] == OP_DIAG2;
      const bool inreg = reg(p.op_a[o]) >= 0 && (!two || reg(p.op_b[o]) >= 0);
      (inreg && is_real(o) ? regd : rest).push_back(o);
    }
    p.ph_u[i] = 0;
    if (!regd.empty() && nc + 16 <= kGateMaxCoef) {
      for (int e = 0; e < 16; ++e) {
        double v = 1;
        for (int o : regd) {
          const T* u = p.coef + p.op_coef[o];
          const bool two = p.op_type[o] == OP_DIAG2;
          const int ba = (e >> reg(p.op_a[o])) & 1, bb = two ? (e >> reg(p.op_b[o])) & 1 : 0;
          v *= (double)u[2 * (ba + 2 * bb)];
        }
        p.coef[nc + e] = (T)v;
      }
      p.ph_u[i] = (uint32_t)nc | (1u << 16);
      nc += 16;
    } else {
      rest.insert(rest.end(), regd.begin(), regd.end());
    }
    std::stable_partition(rest.begin(), rest.end(), is_real);
    int nreal = 0;
    for (int o : rest) nreal += is_real(o);
    p.ph_ops[i] = (uint32_t)nd_total | ((uint32_t)nreal << 8) | ((uint32_t)(rest.size() - nreal) << 16);
    for (int o : rest) {
      p.ph_diag[nd_total++] = o;
      const bool two = p.op_type[o] == OP_DIAG2;
      int ra = reg(p.op_a[o]), rb = two ? reg(p.op_b[o]) : -1;
      if (rb >= 0 && (ra < 0 || rb < ra)) {
        std::swap(p.op_a[o], p.op_b[o]);
        std::swap(ra, rb);
        T* u = p.coef + p.op_coef[o];   // phases of b_a + 2 b_b = 1 and 2 trade places
        std::swap(u[2], u[4]);
        std::swap(u[3], u[5]);
      }
      p.op_code[o] = (ra + 1) * 5 + (rb + 1);
    }
  }
  p.last_gates = ph.back().ng;
  p.n_phases = nph;
}

template <class T>
lrdm_status flush_gates_t(lrdm_t h) {
  int kloc_max = local_budget(h->n, h->ncols, sizeof(cx_t<T>));
  if (h->tune.gate_local_max) kloc_max = std::min(kloc_max, h->tune.gate_local_max);
  std::vector<char> placed(h->gates.size(), 0);
  size_t remaining = h->gates.size();
  int npass = 0;
  while (remaining > 0) {
    GatePass<T> p;
    std::memset(&p, 0, sizeof(p));
    p.n = h->n;
    p.ld = h->lay.ld;
    p.ncols = h->ncols;
    int nloc = 0, nc = 0;
    uint32_t locmask = 0, blocked = 0;
    std::vector<size_t> order;
    for (size_t gi = 0; gi < h->gates.size(); ++gi) {
      if (placed[gi]) continue;
      const PendingGate& g = h->gates[gi];
      if (g.qmask & blocked) { blocked |= g.qmask; continue; }
      const bool diag = (g.type == OP_DIAG1 || g.type == OP_DIAG2 || g.type == OP_WEIGHT);
      const bool room = p.n_ops < kGateMaxOps && nc + (int)g.coef.size() <= kGateMaxCoef;
      if (!room) { blocked = ~0u; continue; }
      if (!diag) {
        const uint32_t need = g.qmask & ~locmask;
        if (nloc + __builtin_popcount(need) > kloc_max) { blocked |= g.qmask; continue; }
        for (int q = 0; q < h->n; ++q)
          if (need & (1u << q)) { p.local_q[nloc++] = q; locmask |= 1u << q; }
      }
      // encode
      const int o = p.n_ops++;
      p.op_type[o] = g.type;
      p.op_coef[o] = nc;
      auto lidx = [&](int q) { for (int j = 0; j < nloc; ++j) if (p.local_q[j] == q) return j; return -1; };
      if (g.type == OP_1Q) { p.op_a[o] = lidx(g.q0); }
      else if (g.type == OP_2Q) { p.op_a[o] = lidx(g.q0); p.op_b[o] = lidx(g.q1); }
      else { p.op_a[o] = g.q0; p.op_b[o] = g.q1; }
      fill_coef(p, nc, g.coef);
      placed[gi] = 1;
      --remaining;
    }
    // pad the local set with unused qubits so that every pass works on full-size tiles: low
    // qubits, odd ones first (on MI355X a wide pass over qubits 14..19 took 194-197 us padded
    // with qubit 1, 3, 5 or 7 against 199-210 with qubit 0, 2, 4 or 6, at 2^20 x 64 complex64)
    for (int pass = 0; pass < 2; ++pass)
      for (int q = 1 - pass; q < h->n && nloc < kloc_max; q += 2)
        if (!(locmask & (1u << q))) { p.local_q[nloc++] = q; locmask |= 1u << q; }
    p.k = nloc;
    int sorted[8];
    for (int j = 0; j < nloc; ++j) sorted[j] = p.local_q[j];
    std::sort(sorted, sorted + nloc);
    for (int j = 0; j < nloc; ++j) p.sorted_q[j] = sorted[j];
    build_phases(p, nc);
    if (h->rec) {
      if constexpr (sizeof(T) == 4) {
        GateJob<float> j;
        j.p = p;
        j.L = static_cast<float2*>(h->state);
        j.cshift = 0;
        while ((1 << j.cshift) < p.ncols) ++j.cshift;
        j.block0 = 0;
        j.nblocks = 1u << (p.n - p.k);
        h->rec->items.push_back({REC_GATE, 0, 0, j.nblocks, gate_pass_shm(p.ncols, p.k, sizeof(float2), p.n_phases),
                                 h->rec->gates.size()});
        h->rec->gates.push_back(j);
      }
      continue;
    }
    // the passes of one flush run back to back on the stream: one event pair brackets them all
    if (npass++ == 0) timed_begin(h, 0);
    HIPCHK(h, launch_gate_pass<T>(p, static_cast<cx_t<T>*>(h->state), h->stream));
  }
  if (npass) timed_end(h, 0, nullptr, npass);
  h->gates.clear();
  return LRDM_OK;
}

lrdm_status settle(lrdm_t h);

lrdm_status flush_gates(lrdm_t h) {
  if (h->gates.empty()) return LRDM_OK;
  lrdm_status st = settle(h);   // a deferred projection precedes the queued gates
  if (st != LRDM_OK) return st;
  return h->dt == LRDM_C64 ? flush_gates_t<float>(h) : flush_gates_t<double>(h);
}

lrdm_status not_recording(lrdm_t h) {
  if (h->rec) return fail(h, LRDM_E_STATE, "the handle is being recorded into a batch (lrdm_batch_end first)");
  return LRDM_OK;
}

lrdm_status ready_for_output(lrdm_t h) {
  lrdm_status st = check_usable(h);
  if (st != LRDM_OK) return st;
  st = not_recording(h);
  if (st != LRDM_OK) return st;
  if (h->chan_pending) return fail(h, LRDM_E_STATE, "a Kraus channel is pending: call lrdm_compress first");
  st = settle(h);
  if (st != LRDM_OK) return st;
  return flush_gates(h);
}

EigBufs eig_bufs(lrdm_t h) {
  EigBufs b;
  b.S = h->ws<double>(h->lay.off_S);
  b.P = h->ws<double>(h->lay.off_P);
  b.lam = h->ws<double>(h->lay.off_lam);
  b.Y = h->ws<double>(h->lay.off_Y);
  b.info = h->ws<DevInfo>(h->lay.off_info);
  b.rec = nullptr;
  b.W64 = nullptr;
  return b;
}

AdjBufs adj_bufs(lrdm_t h) {
  const int c = h->lay.r_pad, N = h->m_max * c;
  const size_t w2 = 2 * (size_t)c, e = w2 * w2;
  double* p = h->ws<double>(h->lay.off_adj);
  AdjBufs b;
  b.part = p; p += 2 * e * kAdjChunks;
  b.C = p; p += 2 * e;
  b.H = p; p += 2 * (size_t)N * c;
  b.Zh = p; p += 2 * (size_t)N * c;
  b.T1 = p; p += 2 * (size_t)N * N;
  b.Gh = p; p += 2 * (size_t)N * N;
  b.M = p; p += 2 * (size_t)N * N;
  b.P = p; p += 2 * e;
  b.Q = p;
  return b;
}

// Which value of the channel's qubit can reach which: reach[b][c] = some E_a has a non-zero
// entry (E_a)_{cb}.  Where no operator maps b to c, the block of the projection matrix W from
// input half b to output half c is exactly zero (W_{(b,v),(c,j)} = scale sum_a (E_a)_{cb} V).
struct Reach {
  bool r[2][2];
};
Reach channel_reach(const Channel& ch) {
  Reach R{};
  for (int a = 0; a < ch.m; ++a)
    for (int c = 0; c < 2; ++c)
      for (int b = 0; b < 2; ++b)
        if (ch.e[a][c][b][0] != 0.0 || ch.e[a][c][b][1] != 0.0) R.r[b][c] = true;
  return R;
}
// reach of two channels applied in turn (the composed projection X W_1 W_2)
Reach compose_reach(const Reach& A, const Reach& B) {
  Reach R{};
  for (int b = 0; b < 2; ++b)
    for (int c = 0; c < 2; ++c)
      R.r[b][c] = (A.r[b][0] && B.r[0][c]) || (A.r[b][1] && B.r[1][c]);
  return R;
}
// projection skip bits: bit 0 = no path from 0 to 1, bit 1 = no path from 1 to 0
int reach_skip(const Reach& R) { return (R.r[0][1] ? 0 : 1) | (R.r[1][0] ? 0 : 2); }
Reach skip_reach(int skip) {
  Reach R{};
  R.r[0][0] = R.r[1][1] = true;
  R.r[0][1] = !(skip & 1);
  R.r[1][0] = !(skip & 2);
  return R;
}

// Materialise the factor: issue the deferred projection of the last (possibly chained)
// compression.
template <class T>
lrdm_status settle_t(lrdm_t h) {
  if (h->proj_pending) {
    h->proj_pending = false;
    const int c = h->lay.r_pad;
    hipStream_t gs = h->stream;
    if (h->overlap) {   // on gemm, once W is ready (the caller's stream has nothing newer for it)
      gs = h->gemm;
      HIPCHK(h, hipStreamWaitEvent(gs, h->ev_b2g, 0));
    }
    timed_begin(h, 4, gs);
    HIPCHK(h, launch_project<T>(static_cast<cx_t<T>*>(h->state), h->n, h->lay.ld, c, 2, h->pend_q, c,
                                h->w_bulk<T>(h->wslot), h->pend_skip, gs, h->overlap ? h->gemm_cus : h->ncu));
    timed_end(h, 4, gs);
  }
  return join_aux(h);   // overlap mode: the caller's stream after both of the handle's streams
}

lrdm_status settle(lrdm_t h) {
  if (!h->proj_pending && !h->overlap) return LRDM_OK;
  return h->dt == LRDM_C64 ? settle_t<float>(h) : settle_t<double>(h);
}

template <class T>
lrdm_status compress_pair_t(lrdm_t h, int r_target, double eps, int tie, int renorm);

template <class T>
lrdm_status compress_t(lrdm_t h, int r_target, double eps, int tie, int renorm, double* rec) {
  if (h->chan_pending && h->chan_pair) {
    if (rec) return fail(h, LRDM_E_UNSUPPORTED, "compression records take one-qubit channels");
    return compress_pair_t<T>(h, r_target, eps, tie, renorm);
  }
  const int nsplit = (h->chan_pending && !h->plain) ? 2 : 1;
  const int q = nsplit == 2 ? h->chan_q : 0;
  Channel ch{};
  int c, N, F;
  if (nsplit == 2) {
    ch = h->chan;
    c = h->lay.r_pad;
    // while the rank grows the factor's columns from c_bound on are zero: G is formed over the
    // first cw columns of each copy (a power of two >= 8), the zero eigenvalues of the rest left
    // out (the rank rule does not depend on them); the reverse sweep's records keep the full order
    const int cw = rec ? c : std::min(c, std::max(8, next_pow2(h->c_bound)));
    N = ch.m * cw;
    F = 4 * c;
  } else {
    ch.m = 1;
    c = h->ncols;
    N = c;
    F = 2 * c;
  }
  const int Fc = F / 2;
  const int kmax = rec ? N : std::min(r_target + 1, N);
  const int c_out = h->lay.r_pad;
  const int nb = gram_blocks(h->n, nsplit);
  EigBufs b = eig_bufs(h);
  b.rec = rec;
  auto* L = static_cast<cx_t<T>*>(h->state);
  T* part = h->ws<T>(h->lay.off_part);
  cx_t<T>* W = h->ws<cx_t<T>>(h->lay.off_W);
  if (h->rec) {
    if constexpr (sizeof(T) == 4) {
      Recorder& R = *h->rec;
      GramJob<float> g;
      g.L = L;
      g.partials = part;
      g.ld = h->lay.ld;
      g.seg_shift = gram_seg_shift(c);
      g.nsplit = nsplit;
      g.q = q;
      g.rows = 1u << (h->n - (nsplit == 2 ? 1 : 0));
      g.rows_per_block = gram_rows_per_block(h->n, nsplit, nb);
      g.block0 = 0;
      g.nblocks = (uint32_t)nb;
      if (g.seg_shift < 0) return fail(h, LRDM_E_UNSUPPORTED, "column count is not a power of two");
      R.items.push_back({REC_GRAM, F, 0, g.nblocks, 0, R.grams.size()});
      R.grams.push_back(g);
      ReduceJob<float> rj;
      rj.partials = part;
      rj.S = b.S;
      rj.nblocks = nb;
      rj.NT = F / 16;
      rj.NUP = rj.NT * (rj.NT + 1) / 2;
      rj.block0 = 0;
      R.items.push_back({REC_REDUCE, F, 0, (uint32_t)rj.NUP, 0, R.reds.size()});
      R.reds.push_back(rj);
      EigJob<float> e;
      e.S = b.S;
      e.ch = ch;
      e.Fc = Fc;
      e.nsplit = nsplit;
      e.c = c;
      e.N = N;
      e.kmax = kmax;
      e.r_target = r_target;
      e.tie = tie;
      e.renorm = renorm;
      e.c_out = c_out;
      e.eps = eps;
      e.B = b;
      e.W = W;
      R.items.push_back({REC_EIG, N, kmax, 1, 0, R.eigs.size()});
      R.eigs.push_back(e);
      ProjJob<float> pj;
      pj.L = L;
      pj.W = W;
      pj.ld = h->lay.ld;
      pj.F = 2 * nsplit * c;
      pj.seg_in_shift = gram_seg_shift(c);
      pj.nsplit = nsplit;
      pj.q = q;
      pj.seg_out_shift = gram_seg_shift(c_out);
      pj.skip = nsplit == 2 ? reach_skip(channel_reach(ch)) : 0;
      pj.rows = 1u << (h->n - (nsplit == 2 ? 1 : 0));
      pj.block0 = 0;
      pj.nblocks = (pj.rows + 127) / 128;
      R.items.push_back({REC_PROJ, 2 * nsplit * c_out, 0, pj.nblocks, 0, R.projs.size()});
      R.projs.push_back(pj);
    }
    h->ncols = c_out;
    const int grown_r = (nsplit == 2) ? h->c_bound * ch.m : h->c_bound;
    h->c_bound = std::min(std::min(grown_r, r_target), N);
    h->chan_pending = false;
    return LRDM_OK;
  }
  // chained compression: the previous one (same qubit) left its projection pending, so S of
  // the factor it would produce is W^H S W and the two projections compose
  const bool chain = !rec && nsplit == 2 && h->proj_pending && h->pend_q == q;
  // overlap mode: a channel on another qubit takes its S from the 4-way Gram of the bit pair,
  // and every fused eigensolve runs on aux
  const bool pipe = h->overlap && !rec && nsplit == 2 && h->proj_pending && h->pend_q != q;
  const bool on_aux = h->overlap && !rec && nsplit == 2;
  hipStream_t es = on_aux ? h->aux : h->stream;    // eigensolve
  hipStream_t gs = on_aux ? h->gemm : h->stream;   // passes over L
  if (!chain && !pipe) {
    lrdm_status st = settle_t<T>(h);
    if (st != LRDM_OK) return st;
  }
  if (on_aux && !chain) {
    lrdm_status st = enter_gemm(h);   // gates and other work on the caller's stream come first
    if (st != LRDM_OK) return st;
  }
  double* Wn64 = h->chain_block(1);   // W of this compression when chained
  double* tmp64 = h->chain_block(2);
  int slot = h->wslot;                // W slot this compression's (pending) projection uses
  if (rec) {
    // recorded compressions (reverse sweep) form S exactly from the bulk-precision factor
    HIPCHK(h, launch_gram_exact<T>(L, h->n, h->lay.ld, c, q, adj_bufs(h).part, b.S, h->stream));
  } else if (chain) {
    // S holds the Gram matrix of the split view before the previous compression; transform it
    // by that compression's own W (not the composed product)
    timed_begin(h, 5, es);
    HIPCHK(h, launch_chain_gram(b.S, h->last_w_next ? Wn64 : h->wp64(slot), tmp64, Fc, es));
    timed_end(h, 5, es);
  } else if (pipe) {
    const int p = h->pend_q;
    double* S4 = h->ws<double>(h->lay.off_S4) + (size_t)h->s4slot * 2 * (4 * c) * (4 * c);
    T* part_h = h->ws<T>(h->lay.off_part4);
    T* part_c = part_h + (size_t)2 * gram4_blocks_halves(h->n) * ((c / 4) * (c / 4 + 1) / 2) * 256;
    // the 4-way Gram of (p, q) on the factor before the projection on p ...
    timed_begin(h, 6, gs);
    HIPCHK(h, launch_gram4<T>(L, h->n, h->lay.ld, c, p, q, part_h, part_c, S4,
                              h->tune.gram4_blocks ? h->tune.gram4_blocks : h->gemm_cus, gs));
    timed_end(h, 6, gs);
    HIPCHK(h, hipEventRecord(h->ev_g2b, gs));
    // ... then that projection, once its W is ready
    HIPCHK(h, hipStreamWaitEvent(gs, h->ev_b2g, 0));
    timed_begin(h, 4, gs);
    HIPCHK(h, launch_project<T>(L, h->n, h->lay.ld, c, 2, p, c, h->w_bulk<T>(h->wslot), h->pend_skip, gs,
                                h->overlap ? h->gemm_cus : h->ncu));
    timed_end(h, 4, gs);
    h->proj_pending = false;
    // aux: the split Gram on q of the projected factor, from G4 and the projection's FP64 W
    HIPCHK(h, hipStreamWaitEvent(h->aux, h->ev_g2b, 0));
    timed_begin(h, 5, h->aux);
    HIPCHK(h, launch_pair_transform(S4, h->wp64(h->wslot), h->ws<double>(h->lay.off_T4), b.S, c, h->aux));
    timed_end(h, 5, h->aux);
    h->s4slot ^= 1;
    slot = h->wslot ^ 1;
  } else {
    int nbg = on_aux ? std::min(nb, h->gemm_cus) : nb;   // one round on the gemm stream's CUs
    if (h->tune.gram_blocks) nbg = std::min(nb, h->tune.gram_blocks);
    timed_begin(h, 1, gs);
    HIPCHK(h, launch_gram<T>(L, h->n, h->lay.ld, c, nsplit, q, part, nbg, gs));
    timed_end(h, 1, gs);
    timed_begin(h, 2, gs);
    HIPCHK(h, launch_gram_reduce<T>(part, nbg, F, b.S, gs));
    timed_end(h, 2, gs);
    if (on_aux) {
      HIPCHK(h, hipEventRecord(h->ev_g2b, gs));
      HIPCHK(h, hipStreamWaitEvent(h->aux, h->ev_g2b, 0));
      slot = h->wslot ^ 1;   // nothing is pending: either slot is free
    }
  }
  const bool defer = !rec && nsplit == 2;   // fused compressions defer their projection
  if (defer) b.W64 = chain ? Wn64 : h->wp64(slot);
  W = h->w_bulk<T>(slot);
  timed_begin(h, 3, es);
  HIPCHK(h, launch_eig<T>(b.S, Fc, ch, nsplit, c, N, kmax, r_target, eps, tie, renorm, c_out, b,
                          W, es));
  timed_end(h, 3, es);
  if (chain) {
    timed_begin(h, 5, es);
    HIPCHK(h, launch_chain_compose<T>(h->wp64(slot), Wn64, tmp64, W, Fc, es));
    timed_end(h, 5, es);
  }
  if (on_aux) HIPCHK(h, hipEventRecord(h->ev_b2g, h->aux));
  if (defer) {
    const Reach here = channel_reach(ch);
    h->pend_skip = reach_skip(chain ? compose_reach(skip_reach(h->pend_skip), here) : here);
    h->proj_pending = true;
    h->pend_q = q;
    h->last_w_next = chain;
    h->wslot = slot;
  } else {
    timed_begin(h, 4);
    HIPCHK(h, launch_project<T>(L, h->n, h->lay.ld, c, nsplit, q, c_out, W,
                                nsplit == 2 ? reach_skip(channel_reach(ch)) : 0, h->stream, h->ncu));
    timed_end(h, 4);
  }
  h->ncols = c_out;
  const int grown = (nsplit == 2) ? h->c_bound * ch.m : h->c_bound;
  h->c_bound = std::min(std::min(grown, r_target), N);
  h->chan_pending = false;
  return LRDM_OK;
}

// A channel on the qubit pair (q0, q1), fused form: G = sum_{u u'} (E_a^H E_b)_{u u'} S4_{u u'}
// from the 4-way Gram S4 of the pair (Sec. II.C: a channel group of two qubits, one truncation),
// then L_new = X4 W with W_{(u,v),(u',j)} = c sum_a (E_a)_{u'u} V[(a,v), j].  No chaining: the
// projection is issued at once, on the caller's stream.
template <class T>
lrdm_status compress_pair_t(lrdm_t h, int r_target, double eps, int tie, int renorm) {
  lrdm_status st = settle_t<T>(h);
  if (st != LRDM_OK) return st;
  const int c = h->lay.r_pad, m = h->chan.m;
  const int cw = std::min(c, std::max(8, next_pow2(h->c_bound)));
  const int N = m * cw, Fc = 4 * c;
  const int kmax = std::min(r_target + 1, N);
  const int q0 = h->chan_q, q1 = h->chan_q1;
  auto* L = static_cast<cx_t<T>*>(h->state);
  // the operator blocks (host FP64, staged once per channel)
  double* M4 = h->ws<double>(h->lay.off_M4);
  double* E4 = M4 + 2 * 16 * 16;
  h->pair_stage.assign(2 * (16 * 16 + 4 * 16), 0.0);
  const double* e = h->pair_e.data();
  for (int a = 0; a < m; ++a)
    for (int b = 0; b < m; ++b)
      for (int u = 0; u < 4; ++u)
        for (int u2 = 0; u2 < 4; ++u2) {
          double re = 0, im = 0;
          for (int r = 0; r < 4; ++r) {
            const double ar = e[((a * 4 + r) * 4 + u) * 2], ai = -e[((a * 4 + r) * 4 + u) * 2 + 1];
            const double br = e[((b * 4 + r) * 4 + u2) * 2], bi = e[((b * 4 + r) * 4 + u2) * 2 + 1];
            re += ar * br - ai * bi;
            im += ar * bi + ai * br;
          }
          const int t = ((a * m + b) * 4 + u) * 4 + u2;
          h->pair_stage[2 * t] = re;
          h->pair_stage[2 * t + 1] = im;
        }
  std::copy(e, e + 32 * m, h->pair_stage.begin() + 2 * 16 * 16);
  HIPCHK(h, hipMemcpyAsync(M4, h->pair_stage.data(), h->pair_stage.size() * 8, hipMemcpyHostToDevice, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));   // the staging vector is reused by the next channel
  // 4-way Gram of the pair on the caller's stream (the overlap mode's pipeline is settled)
  double* S4 = h->ws<double>(h->lay.off_S4);
  T* part_h = h->ws<T>(h->lay.off_part4);
  T* part_c = part_h + (size_t)2 * gram4_blocks_halves(h->n) * ((c / 4) * (c / 4 + 1) / 2) * 256;
  timed_begin(h, 6);
  HIPCHK(h, launch_gram4<T>(L, h->n, h->lay.ld, c, q0, q1, part_h, part_c, S4,
                            h->tune.gram4_blocks ? h->tune.gram4_blocks : 256, h->stream));
  timed_end(h, 6);
  EigBufs b = eig_bufs(h);
  b.M4 = M4;
  b.E4 = E4;
  Channel ch{};
  ch.m = m;
  cx_t<T>* W4 = h->ws<cx_t<T>>(h->lay.off_W4);
  timed_begin(h, 3);
  HIPCHK(h, launch_eig<T>(S4, Fc, ch, 4, c, N, kmax, r_target, eps, tie, renorm, c, b, W4, h->stream));
  timed_end(h, 3);
  timed_begin(h, 4);
  HIPCHK(h, launch_project4<T>(L, h->n, h->lay.ld, c, q0, q1, c, W4, h->stream));
  timed_end(h, 4);
  h->ncols = c;
  h->c_bound = std::min(std::min(h->c_bound * m, r_target), N);
  h->chan_pending = false;
  h->chan_pair = false;
  return LRDM_OK;
}

template <class T>
lrdm_status reset_t(lrdm_t h) {
  if (h->rec) {
    ResetJob j;
    j.state = h->state;
    j.info = h->ws<DevInfo>(h->lay.off_info);
    j.state_bytes = h->lay.state_bytes;
    j.block0 = 0;
    const uint64_t words = h->lay.state_bytes / 16;
    const uint64_t want = (words + 256 * 16 - 1) / (256 * 16);
    j.nblocks = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(want, 1024));
    h->rec->items.push_back({REC_RESET, 0, 0, j.nblocks, 0, h->rec->resets.size()});
    h->rec->resets.push_back(j);
    h->proj_pending = false;
    h->ncols = h->lay.r_pad;
    h->c_bound = 1;
    h->gates.clear();
    h->chan_pending = false;
    h->chan_pair = false;
    return LRDM_OK;
  }
  lrdm_status st = join_aux(h);   // a dropped pending compression may still run on aux
  if (st != LRDM_OK) return st;
  HIPCHK(h, hipMemsetAsync(h->state, 0, h->lay.state_bytes, h->stream));
  HIPCHK(h, hipMemsetAsync(h->ws<DevInfo>(h->lay.off_info), 0, sizeof(DevInfo), h->stream));
  HIPCHK(h, launch_set_e0<T>(static_cast<cx_t<T>*>(h->state), h->stream));
  h->proj_pending = false;
  h->ncols = h->lay.r_pad;
  h->c_bound = 1;
  h->gates.clear();
  h->chan_pending = false;
  h->chan_pair = false;
  return LRDM_OK;
}

// completeness sum_a E_a^H E_a = I within 1e-10 (FP64)
bool kraus_complete(int m, const double* e) {
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      double re = 0, im = 0;
      for (int a = 0; a < m; ++a)
        for (int r = 0; r < 2; ++r) {
          const double ar = e[((a * 2 + r) * 2 + i) * 2], ai = -e[((a * 2 + r) * 2 + i) * 2 + 1];
          const double br = e[((a * 2 + r) * 2 + j) * 2], bi = e[((a * 2 + r) * 2 + j) * 2 + 1];
          re += ar * br - ai * bi;
          im += ar * bi + ai * br;
        }
      if (!(std::fabs(re - (i == j)) <= 1e-10 && std::fabs(im) <= 1e-10)) return false;
    }
  return true;
}

Channel make_channel(int m, const double* e) {
  Channel ch{};
  ch.m = m;
  for (int a = 0; a < m; ++a)
    for (int r = 0; r < 2; ++r)
      for (int cidx = 0; cidx < 2; ++cidx)
        for (int z = 0; z < 2; ++z) ch.e[a][r][cidx][z] = e[((a * 2 + r) * 2 + cidx) * 2 + z];
  return ch;
}

bool same_shape(lrdm_t a, lrdm_t b) {
  return a->n == b->n && a->lay.r_pad == b->lay.r_pad && a->dt == b->dt && a->m_max == b->m_max &&
         a->plain == b->plain && a->lay.ld == b->lay.ld;
}

// Work already queued on stream `other` finishes before h's stream runs what it queues next.
lrdm_status order_streams_raw(hipStream_t mine, hipStream_t other) {
  if (other != mine && hipStreamSynchronize(other) != hipSuccess)
    return fail(nullptr, LRDM_E_HIP, "synchronising the other handle's stream failed");
  return LRDM_OK;
}

// Order work on a's stream before work that b's stream enqueues next.
lrdm_status order_streams(lrdm_t a, lrdm_t b) {
  if (a->stream != b->stream) HIPCHK(a, hipStreamSynchronize(a->stream));
  return LRDM_OK;
}

lrdm_status check_masks(lrdm_t h, int n_terms, const uint64_t* xmask, const uint64_t* zmask) {
  const uint64_t lim = (h->n >= 64) ? ~0ull : ((1ull << h->n) - 1ull);
  for (int t = 0; t < n_terms; ++t)
    if ((xmask[t] & ~lim) || (zmask[t] & ~lim)) return fail(h, LRDM_E_ARG, "Pauli mask beyond n qubits");
  return LRDM_OK;
}

// Tr(bra^H P_t ket) for every term: vals[t] (real part) or vals[2t], vals[2t + 1] (complex).
// Terms are grouped by X mask so that each distinct mask costs one pass over the rows.  Uses the
// workspace and stream of h (the ket's handle).
lrdm_status pauli_values(lrdm_t h, const void* bra, int n_terms, const uint64_t* xmask,
                         const uint64_t* zmask, int complex_out, double* vals) {
  std::vector<int> idx(n_terms);
  for (int t = 0; t < n_terms; ++t) idx[t] = t;
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return xmask[a] < xmask[b]; });
  const uint32_t rows = 1u << h->n;
  const int nchunks = (int)((rows + 1023) / 1024);
  const int batch_cap = std::max(1, (int)(kPauliPartDoubles / (2 * (size_t)nchunks)));
  const int cw = complex_out ? 2 : 1;
  uint64_t* dterms = h->ws<uint64_t>(h->lay.off_terms);
  double* dpart = h->ws<double>(h->lay.off_pauli);
  double* dout = h->ws<double>(h->lay.off_out);
  for (int b0 = 0; b0 < n_terms; b0 += std::min(batch_cap, 2048)) {
    const int nb = std::min(n_terms - b0, std::min(batch_cap, 2048));
    // staging: xm[nb], zm[nb], gstart[ngroups + 1] (int)
    std::vector<uint64_t> xm(nb), zm(nb);
    std::vector<int> gstart;
    for (int t = 0; t < nb; ++t) {
      xm[t] = xmask[idx[b0 + t]];
      zm[t] = zmask[idx[b0 + t]];
      if (t == 0 || xm[t] != xm[t - 1]) gstart.push_back(t);
    }
    const int ngroups = (int)gstart.size();
    gstart.push_back(nb);
    h->term_stage.assign(2 * nb + (gstart.size() + 1) / 2 + 1, 0);
    std::memcpy(h->term_stage.data(), xm.data(), nb * 8);
    std::memcpy(h->term_stage.data() + nb, zm.data(), nb * 8);
    std::memcpy(h->term_stage.data() + 2 * nb, gstart.data(), gstart.size() * 4);
    HIPCHK(h, hipMemcpyAsync(dterms, h->term_stage.data(), h->term_stage.size() * 8, hipMemcpyHostToDevice, h->stream));
    hipError_t e = h->dt == LRDM_C64
                       ? launch_pauli<float>(static_cast<const float2*>(bra), static_cast<float2*>(h->state), h->n, h->lay.ld, h->ncols, dterms, dterms + nb, nb, dpart, ngroups, dout, complex_out, h->stream)
                       : launch_pauli<double>(static_cast<const double2*>(bra), static_cast<double2*>(h->state), h->n, h->lay.ld, h->ncols, dterms, dterms + nb, nb, dpart, ngroups, dout, complex_out, h->stream);
    HIPCHK(h, e);
    std::vector<double> r((size_t)nb * cw);
    HIPCHK(h, hipMemcpyAsync(r.data(), dout, r.size() * 8, hipMemcpyDeviceToHost, h->stream));
    lrdm_status st = sync_and_check(h);
    if (st != LRDM_OK) return st;
    for (int t = 0; t < nb; ++t)
      for (int z = 0; z < cw; ++z) vals[(size_t)idx[b0 + t] * cw + z] = r[(size_t)t * cw + z];
  }
  return LRDM_OK;
}

lrdm_status compress_entry(lrdm_t h, int r_target, double eps, int tie_policy, int renorm,
                           double* rec, lrdm_compress_info* info) {
  if (h && h->rec && (info || rec))
    return fail(h, LRDM_E_STATE, "a recorded compression cannot report info or write a record");
  lrdm_status st = check_usable(h);
  if (st != LRDM_OK) return st;
  if (r_target < 1 || r_target > h->r_max) return fail(h, LRDM_E_ARG, "r_target must be in [1, r_max]");
  if (!(eps >= 0.0 && eps < 1.0)) return fail(h, LRDM_E_ARG, "eps must be in [0, 1)");
  if (tie_policy != 0 && tie_policy != 1) return fail(h, LRDM_E_ARG, "tie_policy must be 0 or 1");
  if (renorm != 0 && renorm != 1) return fail(h, LRDM_E_ARG, "renorm must be 0 or 1");
  st = flush_gates(h);
  if (st != LRDM_OK) return st;
  st = h->dt == LRDM_C64 ? compress_t<float>(h, r_target, eps, tie_policy, renorm, rec)
                         : compress_t<double>(h, r_target, eps, tie_policy, renorm, rec);
  if (st != LRDM_OK) return st;
  if (info) {
    st = sync_and_check(h);
    if (st != LRDM_OK) return st;
    DevInfo d;
    HIPCHK(h, hipMemcpy(&d, h->ws<DevInfo>(h->lay.off_info), sizeof(d), hipMemcpyDeviceToHost));
    info->rank = d.k;
    info->n_eig = d.n_eig;
    info->discarded = d.discarded;
    info->discarded_total = d.discarded_total;
    info->trace_before = d.trace;
    info->boundary_gap = d.gap;
    info->lambda_max = d.lambda_max;
  }
  return LRDM_OK;
}

}  // namespace

extern "C" {

const char* lrdm_version(void) { return "lrdm 0.1 (gfx950)"; }

const char* lrdm_last_error(lrdm_t h) { return h ? h->err.c_str() : g_last_error.c_str(); }

lrdm_status lrdm_workspace_size(int n, int r_max, lrdm_dtype dt, int m_max, unsigned flags,
                                size_t* state_bytes, size_t* work_bytes) {
  if (!state_bytes || !work_bytes) return fail(nullptr, LRDM_E_ARG, "null output pointer");
  Layout L;
  std::string why;
  if (!compute_layout(n, r_max, dt, m_max, flags, L, why)) {
    const bool range = (n < 1 || n > 30 || r_max < 1 || r_max > 64 || m_max < 1 ||
                        m_max > ((flags & LRDM_FLAG_PLAIN) ? 16 : 4) || (dt != LRDM_C64 && dt != LRDM_C128));
    return fail(nullptr, range ? LRDM_E_ARG : LRDM_E_UNSUPPORTED, why);
  }
  *state_bytes = L.state_bytes;
  *work_bytes = L.total;
  return LRDM_OK;
}

lrdm_status lrdm_init(lrdm_t* out, int n, int r_max, lrdm_dtype dt, int m_max, unsigned flags,
                      void* state_dev, size_t state_bytes, void* work_dev, size_t work_bytes,
                      void* hip_stream) {
  if (!out) return fail(nullptr, LRDM_E_ARG, "null output handle pointer");
  *out = nullptr;
  Layout L;
  std::string why;
  if (!compute_layout(n, r_max, dt, m_max, flags, L, why)) return fail(nullptr, LRDM_E_ARG, why);
  if (!state_dev || !work_dev) return fail(nullptr, LRDM_E_ARG, "null device buffer");
  if (state_bytes < L.state_bytes || work_bytes < L.total)
    return fail(nullptr, LRDM_E_NOMEM, "state or workspace buffer smaller than lrdm_workspace_size");
  if ((reinterpret_cast<uintptr_t>(state_dev) | reinterpret_cast<uintptr_t>(work_dev)) & 255)
    return fail(nullptr, LRDM_E_ARG, "device buffers must be 256-byte aligned");
  lrdm_ctx* h = new lrdm_ctx();
  h->n = n;
  h->r_max = r_max;
  h->m_max = m_max;
  h->dt = dt;
  h->flags = flags;
  h->plain = flags & LRDM_FLAG_PLAIN;
  h->lay = L;
  h->state = state_dev;
  h->work = static_cast<char*>(work_dev);
  h->stream = static_cast<hipStream_t>(hip_stream);
  h->overlap = L.overlap;
  if (h->overlap) {
    hipError_t e = create_overlap_streams(h);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&h->ev_a2g, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&h->ev_g2b, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&h->ev_b2g, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&h->ev_g2a, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(h->ev_b2g, h->aux);
    if (e != hipSuccess) {
      const std::string msg = std::string("creating the handle's streams: ") + hipGetErrorString(e);
      release_overlap(h);
      delete h;
      return fail(nullptr, LRDM_E_HIP, msg);
    }
  }
  lrdm_status st = dt == LRDM_C64 ? reset_t<float>(h) : reset_t<double>(h);
  if (st != LRDM_OK) {
    g_last_error = h->err;
    lrdm_destroy(h);
    return st;
  }
  *out = h;
  return LRDM_OK;
}

lrdm_status lrdm_layout(lrdm_t h, int* n, int* ld, int* r_pad, size_t* state_bytes) {
  if (!h) return fail(nullptr, LRDM_E_ARG, "null handle");
  if (n) *n = h->n;
  if (ld) *ld = h->lay.ld;
  if (r_pad) *r_pad = h->lay.r_pad;
  if (state_bytes) *state_bytes = h->lay.state_bytes;
  return LRDM_OK;
}

lrdm_status lrdm_reset(lrdm_t h) {
  lrdm_status st = check_usable(h);
  if (st != LRDM_OK) return st;
  return h->dt == LRDM_C64 ? reset_t<float>(h) : reset_t<double>(h);
}

lrdm_status lrdm_destroy(lrdm_t h) {
  if (!h) return fail(nullptr, LRDM_E_ARG, "null handle");
  for (hipEvent_t e : h->ev) hipEventDestroy(e);
  if (h->overlap) release_overlap(h);
  delete h;
  return LRDM_OK;
}

lrdm_status lrdm_apply_gate(lrdm_t h, int k, const int* qubits, const double* u) {
  lrdm_status st = check_usable(h);
  if (st != LRDM_OK) return st;
  if (k != 1 && k != 2) return fail(h, LRDM_E_ARG, "k must be 1 or 2");
  if (!qubits || !u) return fail(h, LRDM_E_ARG, "null qubits or matrix");
  for (int j = 0; j < k; ++j)
    if (qubits[j] < 0 || qubits[j] >= h->n) return fail(h, LRDM_E_ARG, "qubit out of range");
  if (k == 2 && qubits[0] == qubits[1]) return fail(h, LRDM_E_ARG, "repeated qubit");
  const int d = 1 << k;
  if (!is_unitary(u, d)) return fail(h, LRDM_E_ARG, "gate matrix is not unitary within 1e-10");
  if (h->chan_pending) return fail(h, LRDM_E_STATE, "a Kraus channel is pending: call lrdm_compress first");
  bool diag = true;
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j)
      if (i != j && (u[2 * (i * d + j)] != 0.0 || u[2 * (i * d + j) + 1] != 0.0)) diag = false;
  PendingGate g;
  g.q0 = qubits[0];
  g.q1 = (k == 2) ? qubits[1] : -1;
  g.qmask = (1u << qubits[0]) | (k == 2 ? (1u << qubits[1]) : 0u);
  if (diag) {
    g.type = (k == 1) ? OP_DIAG1 : OP_DIAG2;
    for (int i = 0; i < d; ++i) {
      g.coef.push_back(u[2 * (i * d + i)]);
      g.coef.push_back(u[2 * (i * d + i) + 1]);
    }
  } else {
    g.type = (k == 1) ? OP_1Q : OP_2Q;
    g.coef.assign(u, u + 2 * d * d);
  }
  h->gates.push_back(std::move(g));
  return LRDM_OK;
}

lrdm_status lrdm_apply_diagonal_weight(lrdm_t h, const double* phase) {
  lrdm_status st = check_usable(h);
  if (st != LRDM_OK) return st;
  if (!phase) return fail(h, LRDM_E_ARG, "null phase table");
  for (int w = 0; w <= h->n; ++w) {
    const double m = std::hypot(phase[2 * w], phase[2 * w + 1]);
    if (!(std::fabs(m - 1.0) <= 1e-10)) return fail(h, LRDM_E_ARG, "phase entries must have unit modulus");
  }
  if (h->chan_pending) return fail(h, LRDM_E_STATE, "a Kraus channel is pending: call lrdm_compress first");
  PendingGate g;
  g.type = OP_WEIGHT;
  g.q0 = g.q1 = -1;
  g.qmask = (h->n >= 32) ? ~0u : ((1u << h->n) - 1u);
  g.coef.assign(phase, phase + 2 * (h->n + 1));
  h->gates.push_back(std::move(g));
  return LRDM_OK;
}

lrdm_status lrdm_apply_kraus(lrdm_t h, int qubit, int m, const double* e) {
  lrdm_status st = check_usable(h);
  if (st != LRDM_OK) return st;
  if (qubit < 0 || qubit >= h->n) return fail(h, LRDM_E_ARG, "qubit out of range");
  if (m < 1 || m > h->m_max) return fail(h, LRDM_E_ARG, "Kraus count must be in [1, m_max]");
  if (!e) return fail(h, LRDM_E_ARG, "null Kraus matrices");
  if (!kraus_complete(m, e)) return fail(h, LRDM_E_ARG, "Kraus set is not complete within 1e-10");
  if (h->chan_pending) return fail(h, LRDM_E_STATE, "a Kraus channel is already pending: compress first");
  st = flush_gates(h);
  if (st != LRDM_OK) return st;
  const Channel ch = make_channel(m, e);
  if (h->plain) {
    const int c = h->ncols;
    hipError_t he = h->dt == LRDM_C64
                        ? launch_kraus_expand<float>(static_cast<float2*>(h->state), h->n, h->lay.ld, c,
                                                     qubit, ch, h->lay.m_pad, h->stream)
                        : launch_kraus_expand<double>(static_cast<double2*>(h->state), h->n, h->lay.ld,
                                                      c, qubit, ch, h->lay.m_pad, h->stream);
    HIPCHK(h, he);
    h->ncols = c * h->lay.m_pad;
    h->c_bound = std::min(h->c_bound * m, h->ncols);
    h->chan_pending = true;   // compress must follow (same contract as the fused form)
    h->chan_q = qubit;
    h->chan = ch;
    return LRDM_OK;
  }
  h->chan_pending = true;
  h->chan_q = qubit;
  h->chan = ch;
  return LRDM_OK;
}

lrdm_status lrdm_apply_kraus2(lrdm_t h, int q0, int q1, int m, const double* e) {
  lrdm_status st = check_usable(h);
  if (st != LRDM_OK) return st;
  if (q0 < 0 || q0 >= h->n || q1 < 0 || q1 >= h->n || q0 == q1)
    return fail(h, LRDM_E_ARG, "qubits out of range or repeated");
  if (m < 1 || m > h->m_max) return fail(h, LRDM_E_ARG, "Kraus count must be in [1, m_max]");
  if (!h->plain) {
    if (h->rec) return fail(h, LRDM_E_UNSUPPORTED, "channels on a qubit pair are not recorded into a batch");
    if (h->lay.r_pad > 32)
      return fail(h, LRDM_E_UNSUPPORTED, "fused channels on a qubit pair take r_pad <= 32 (else LRDM_FLAG_PLAIN)");
  }
  if (!e) return fail(h, LRDM_E_ARG, "null Kraus matrices");
  // completeness sum_a E_a^H E_a = I (4 x 4)
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      double re = 0, im = 0;
      for (int a = 0; a < m; ++a)
        for (int r = 0; r < 4; ++r) {
          const double ar = e[((a * 4 + r) * 4 + i) * 2], ai = -e[((a * 4 + r) * 4 + i) * 2 + 1];
          const double br = e[((a * 4 + r) * 4 + j) * 2], bi = e[((a * 4 + r) * 4 + j) * 2 + 1];
          re += ar * br - ai * bi;
          im += ar * bi + ai * br;
        }
      if (!(std::fabs(re - (i == j)) <= 1e-10 && std::fabs(im) <= 1e-10))
        return fail(h, LRDM_E_ARG, "Kraus set is not complete within 1e-10");
    }
  if (h->chan_pending) return fail(h, LRDM_E_STATE, "a Kraus channel is already pending: compress first");
  st = flush_gates(h);
  if (st != LRDM_OK) return st;
  if (!h->plain) {   // fused: kept for the compression, nothing materialised
    h->pair_e.assign(e, e + 32 * m);
    h->chan_pending = true;
    h->chan_pair = true;
    h->chan_q = q0;
    h->chan_q1 = q1;
    h->chan = Channel{};
    h->chan.m = m;
    return LRDM_OK;
  }
  const int c = h->ncols, m_pad = h->lay.m_pad;
  // launches over operator blocks, the one holding a = 0 (which overwrites the input columns) last
  std::vector<int> starts;
  for (int a0 = kKraus2PerLaunch; a0 < m_pad; a0 += kKraus2PerLaunch) starts.push_back(a0);
  starts.push_back(0);
  for (int a0 : starts) {
    Kraus2Chunk ck{};
    ck.a0 = a0;
    ck.na = std::min(kKraus2PerLaunch, m_pad - a0);
    ck.m = m;
    for (int u = 0; u < ck.na && a0 + u < m; ++u)
      for (int r = 0; r < 4; ++r)
        for (int cc = 0; cc < 4; ++cc)
          for (int z = 0; z < 2; ++z) ck.e[u][r][cc][z] = e[(((a0 + u) * 4 + r) * 4 + cc) * 2 + z];
    hipError_t he = h->dt == LRDM_C64
                        ? launch_kraus2_expand<float>(static_cast<float2*>(h->state), h->n, h->lay.ld, c, q0, q1, ck, h->stream)
                        : launch_kraus2_expand<double>(static_cast<double2*>(h->state), h->n, h->lay.ld, c, q0, q1, ck, h->stream);
    HIPCHK(h, he);
  }
  h->ncols = c * m_pad;
  h->c_bound = std::min(h->c_bound * m, h->ncols);
  h->chan_pending = true;   // compress must follow
  h->chan_q = q0;
  h->chan = Channel{};
  h->chan.m = m;
  return LRDM_OK;
}

lrdm_status lrdm_set_sparse(lrdm_t h, int count, const uint64_t* idx, const double* amp) {
  lrdm_status st = check_usable(h);
  if (st != LRDM_OK) return st;
  st = not_recording(h);
  if (st != LRDM_OK) return st;
  if (count < 1 || count > kMaxSparse) return fail(h, LRDM_E_ARG, "count must be in [1, 32768]");
  if (!idx || !amp) return fail(h, LRDM_E_ARG, "null indices or amplitudes");
  if (h->chan_pending) return fail(h, LRDM_E_STATE, "a Kraus channel is pending: call lrdm_compress first");
  const uint64_t rows = 1ull << h->n;
  std::vector<uint64_t> sorted(idx, idx + count);
  std::sort(sorted.begin(), sorted.end());
  for (int i = 0; i < count; ++i) {
    if (sorted[i] >= rows) return fail(h, LRDM_E_ARG, "basis index beyond 2^n");
    if (i > 0 && sorted[i] == sorted[i - 1]) return fail(h, LRDM_E_ARG, "repeated basis index");
  }
  double nrm = 0;
  for (int i = 0; i < count; ++i) nrm += amp[2 * i] * amp[2 * i] + amp[2 * i + 1] * amp[2 * i + 1];
  if (!(std::fabs(nrm - 1.0) <= 1e-10)) return fail(h, LRDM_E_ARG, "amplitudes must have unit norm within 1e-10");
  h->gates.clear();
  h->proj_pending = false;
  st = join_aux(h);
  if (st != LRDM_OK) return st;
  uint64_t* didx = h->ws<uint64_t>(h->lay.off_terms);
  double* damp = reinterpret_cast<double*>(didx + kMaxSparse);
  h->term_stage.assign(3 * (size_t)count, 0);
  std::memcpy(h->term_stage.data(), idx, (size_t)count * 8);
  std::memcpy(h->term_stage.data() + count, amp, (size_t)count * 16);
  HIPCHK(h, hipMemsetAsync(h->state, 0, h->lay.state_bytes, h->stream));
  HIPCHK(h, hipMemsetAsync(h->ws<DevInfo>(h->lay.off_info), 0, sizeof(DevInfo), h->stream));
  HIPCHK(h, hipMemcpyAsync(didx, h->term_stage.data(), (size_t)count * 8, hipMemcpyHostToDevice, h->stream));
  HIPCHK(h, hipMemcpyAsync(damp, h->term_stage.data() + count, (size_t)count * 16, hipMemcpyHostToDevice, h->stream));
  hipError_t he = h->dt == LRDM_C64
                      ? launch_set_sparse<float>(static_cast<float2*>(h->state), h->lay.ld, didx, damp, count, h->stream)
                      : launch_set_sparse<double>(static_cast<double2*>(h->state), h->lay.ld, didx, damp, count, h->stream);
  HIPCHK(h, he);
  HIPCHK(h, hipStreamSynchronize(h->stream));   // the staging vector is reused by later calls
  h->ncols = h->lay.r_pad;
  h->c_bound = 1;
  return LRDM_OK;
}

lrdm_status lrdm_to_full(lrdm_t h, lrdm_fdm_t f) {
  lrdm_status st = ready_for_output(h);
  if (st != LRDM_OK) return st;
  float2* rho = nullptr;
  int nf = 0;
  hipStream_t fs = nullptr;
  st = fdm_state(f, &rho, &nf, &fs);
  if (st != LRDM_OK) return st;
  if (nf != h->n) return fail(h, LRDM_E_ARG, "the full-rank handle has a different n");
  fdm_discard_queue(f);
  st = order_streams_raw(h->stream, fs);
  if (st != LRDM_OK) return st;
  hipError_t he = h->dt == LRDM_C64
                      ? launch_lr_to_full<float>(static_cast<float2*>(h->state), h->n, h->lay.ld, h->ncols, rho, h->stream)
                      : launch_lr_to_full<double>(static_cast<double2*>(h->state), h->n, h->lay.ld, h->ncols, rho, h->stream);
  HIPCHK(h, he);
  if (fs != h->stream) HIPCHK(h, hipStreamSynchronize(h->stream));
  return LRDM_OK;
}

lrdm_status lrdm_compress(lrdm_t h, int r_target, double eps, int tie_policy, int renorm,
                          lrdm_compress_info* info) {
  return compress_entry(h, r_target, eps, tie_policy, renorm, nullptr, info);
}

lrdm_status lrdm_compress_record(lrdm_t h, int r_target, double eps, int tie_policy, int renorm,
                                 void* rec_dev, lrdm_compress_info* info) {
  lrdm_status st = check_usable(h);
  if (st != LRDM_OK) return st;
  if (!h->lay.adjoint)
    return fail(h, LRDM_E_UNSUPPORTED, "compression records need the fused form and m_max * r_pad <= 64");
  if (!rec_dev) return fail(h, LRDM_E_ARG, "null record buffer");
  if (reinterpret_cast<uintptr_t>(rec_dev) & 255) return fail(h, LRDM_E_ARG, "record buffer must be 256-byte aligned");
  if (!h->chan_pending) return fail(h, LRDM_E_STATE, "a record needs a pending Kraus channel");
  return compress_entry(h, r_target, eps, tie_policy, renorm, static_cast<double*>(rec_dev), info);
}

lrdm_status lrdm_probabilities(lrdm_t h, double* p_dev) {
  lrdm_status st = ready_for_output(h);
  if (st != LRDM_OK) return st;
  if (!p_dev) return fail(h, LRDM_E_ARG, "null output buffer");
  hipError_t e = h->dt == LRDM_C64
                     ? launch_probabilities<float>(static_cast<float2*>(h->state), h->n, h->lay.ld, h->ncols, p_dev, h->stream)
                     : launch_probabilities<double>(static_cast<double2*>(h->state), h->n, h->lay.ld, h->ncols, p_dev, h->stream);
  HIPCHK(h, e);
  return LRDM_OK;
}

lrdm_status lrdm_expect_z(lrdm_t h, double* z_host, double* zz_host, double* trace_host) {
  lrdm_status st = ready_for_output(h);
  if (st != LRDM_OK) return st;
  if (!z_host) return fail(h, LRDM_E_ARG, "null z output");
  double* pbuf = h->ws<double>(h->lay.off_pbuf);
  double* out = h->ws<double>(h->lay.off_out);
  hipError_t e = h->dt == LRDM_C64
                     ? launch_zstats<float>(static_cast<float2*>(h->state), h->n, h->lay.ld, h->ncols, pbuf, kZBlocks, out, h->stream)
                     : launch_zstats<double>(static_cast<double2*>(h->state), h->n, h->lay.ld, h->ncols, pbuf, kZBlocks, out, h->stream);
  HIPCHK(h, e);
  std::vector<double> r(2 * h->n);
  HIPCHK(h, hipMemcpyAsync(r.data(), out, r.size() * 8, hipMemcpyDeviceToHost, h->stream));
  st = sync_and_check(h);
  if (st != LRDM_OK) return st;
  const double tot = r[0];
  for (int i = 0; i < h->n; ++i) z_host[i] = tot - 2.0 * r[1 + i];
  if (zz_host)
    for (int i = 0; i + 1 < h->n; ++i) zz_host[i] = tot - 2.0 * r[1 + h->n + i];
  if (trace_host) *trace_host = tot;
  return LRDM_OK;
}

lrdm_status lrdm_expect_pauli(lrdm_t h, int n_terms, const uint64_t* xmask, const uint64_t* zmask,
                              const double* coeff, int summed, double* out_host) {
  lrdm_status st = ready_for_output(h);
  if (st != LRDM_OK) return st;
  if (n_terms < 1 || n_terms > kMaxTerms) return fail(h, LRDM_E_ARG, "n_terms must be in [1, 65536]");
  if (!xmask || !zmask || !out_host || (summed && !coeff)) return fail(h, LRDM_E_ARG, "null argument");
  if (summed != 0 && summed != 1) return fail(h, LRDM_E_ARG, "summed must be 0 or 1");
  st = check_masks(h, n_terms, xmask, zmask);
  if (st != LRDM_OK) return st;
  std::vector<double> vals(n_terms);
  st = pauli_values(h, h->state, n_terms, xmask, zmask, 0, vals.data());
  if (st != LRDM_OK) return st;
  if (summed) {
    double s = 0;
    for (int t = 0; t < n_terms; ++t) s += coeff[t] * vals[t];
    out_host[0] = s;
  } else {
    for (int t = 0; t < n_terms; ++t) out_host[t] = vals[t];
  }
  return LRDM_OK;
}

lrdm_status lrdm_sample(lrdm_t h, int count, const double* uniforms, uint64_t* out_host) {
  lrdm_status st = ready_for_output(h);
  if (st != LRDM_OK) return st;
  if (count < 1 || count > (1 << 24)) return fail(h, LRDM_E_ARG, "count must be in [1, 2^24]");
  if (!uniforms || !out_host) return fail(h, LRDM_E_ARG, "null argument");
  for (int j = 0; j < count; ++j)
    if (!(uniforms[j] >= 0.0 && uniforms[j] < 1.0)) return fail(h, LRDM_E_ARG, "uniforms must lie in [0, 1)");
  double* p = h->ws<double>(h->lay.off_pbuf);
  hipError_t e = h->dt == LRDM_C64
                     ? launch_probabilities<float>(static_cast<float2*>(h->state), h->n, h->lay.ld, h->ncols, p, h->stream)
                     : launch_probabilities<double>(static_cast<double2*>(h->state), h->n, h->lay.ld, h->ncols, p, h->stream);
  HIPCHK(h, e);
  double* du = h->ws<double>(h->lay.off_unif);
  uint64_t* ds = h->ws<uint64_t>(h->lay.off_samp);
  for (int b0 = 0; b0 < count; b0 += kSampleBatch) {
    const int nb = std::min(count - b0, kSampleBatch);
    HIPCHK(h, hipMemcpyAsync(du, uniforms + b0, (size_t)nb * 8, hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, launch_sample(p, h->n, h->ws<double>(h->lay.off_cdf), h->ws<double>(h->lay.off_bsum), du, nb, ds, h->stream));
    HIPCHK(h, hipMemcpyAsync(out_host + b0, ds, (size_t)nb * 8, hipMemcpyDeviceToHost, h->stream));
    st = sync_and_check(h);
    if (st != LRDM_OK) return st;
  }
  return LRDM_OK;
}

lrdm_status lrdm_get_L(lrdm_t h, void* dst, int to_host, int* rank_out) {
  lrdm_status st = ready_for_output(h);
  if (st != LRDM_OK) return st;
  if (!dst) return fail(h, LRDM_E_ARG, "null destination");
  // only the active columns carry the factor (plain form leaves stale expansion columns
  // beyond them); the rest of every row is returned as zeros
  const size_t cs = (h->dt == LRDM_C64) ? 8 : 16;
  const size_t rows = 1ull << h->n;
  if (to_host)
    std::memset(dst, 0, h->lay.state_bytes);
  else
    HIPCHK(h, hipMemsetAsync(dst, 0, h->lay.state_bytes, h->stream));
  HIPCHK(h, hipMemcpy2DAsync(dst, h->lay.ld * cs, h->state, h->lay.ld * cs, h->ncols * cs, rows,
                             to_host ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, h->stream));
  if (to_host) {
    st = sync_and_check(h);
    if (st != LRDM_OK) return st;
  }
  if (rank_out) *rank_out = h->c_bound;
  return LRDM_OK;
}

lrdm_status lrdm_set_L(lrdm_t h, const void* src, int from_host, int rank) {
  lrdm_status st = check_usable(h);
  if (st != LRDM_OK) return st;
  st = not_recording(h);
  if (st != LRDM_OK) return st;
  if (!src) return fail(h, LRDM_E_ARG, "null source");
  if (rank < 1 || rank > h->lay.r_pad) return fail(h, LRDM_E_ARG, "rank must be in [1, r_pad]");
  if (h->chan_pending) return fail(h, LRDM_E_STATE, "a Kraus channel is pending: call lrdm_compress first");
  h->gates.clear();
  h->proj_pending = false;
  st = join_aux(h);
  if (st != LRDM_OK) return st;
  const size_t cs = (h->dt == LRDM_C64) ? 8 : 16;
  const size_t rows = 1ull << h->n;
  HIPCHK(h, hipMemsetAsync(h->state, 0, h->lay.state_bytes, h->stream));
  HIPCHK(h, hipMemsetAsync(h->ws<DevInfo>(h->lay.off_info), 0, sizeof(DevInfo), h->stream));
  HIPCHK(h, hipMemcpy2DAsync(h->state, h->lay.ld * cs, src, rank * cs, rank * cs, rows,
                             from_host ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, h->stream));
  if (from_host) HIPCHK(h, hipStreamSynchronize(h->stream));
  h->ncols = h->lay.r_pad;
  h->c_bound = rank;
  return LRDM_OK;
}

lrdm_status lrdm_synchronize(lrdm_t h) {
  lrdm_status st = check_usable(h);
  if (st != LRDM_OK) return st;
  st = not_recording(h);
  if (st != LRDM_OK) return st;
  st = settle(h);
  if (st != LRDM_OK) return st;
  st = flush_gates(h);
  if (st != LRDM_OK) return st;
  return sync_and_check(h);
}

lrdm_status lrdm_set_tuning(lrdm_t h, const lrdm_tuning* t) {
  lrdm_status st = check_usable(h);
  if (st != LRDM_OK) return st;
  st = not_recording(h);
  if (st != LRDM_OK) return st;
  if (!t) return fail(h, LRDM_E_ARG, "null tuning");
  if (t->gram_blocks < 0 || t->gram_blocks > 256) return fail(h, LRDM_E_ARG, "gram_blocks must be in [0, 256]");
  if (t->gram4_blocks < 0 || t->gram4_blocks == 1 || t->gram4_blocks > 256)
    return fail(h, LRDM_E_ARG, "gram4_blocks must be 0 or in [2, 256]");
  if (t->gate_local_max < 0 || t->gate_local_max > 8) return fail(h, LRDM_E_ARG, "gate_local_max must be in [0, 8]");
  if (t->aux_cus < 0 || t->aux_cus % 32 != 0) return fail(h, LRDM_E_ARG, "aux_cus must be 0 or a multiple of 32");
  if (t->aux_cus && (!h->overlap || t->aux_cus > h->ncu - 32))
    return fail(h, LRDM_E_ARG, "aux_cus needs LRDM_FLAG_OVERLAP and leaves at least 32 CUs to the GEMMs");
  // the launch shapes take effect from the next launch; queued gates keep their passes
  st = flush_gates(h);
  if (st != LRDM_OK) return st;
  const int aux_old = h->tune.aux_cus;
  h->tune = *t;
  if (h->overlap && t->aux_cus != aux_old) {
    // new CU split: pending work settles, then the two streams are made again
    st = settle(h);
    if (st != LRDM_OK) return st;
    HIPCHK(h, hipStreamSynchronize(h->stream));
    HIPCHK(h, hipStreamSynchronize(h->gemm));
    HIPCHK(h, hipStreamSynchronize(h->aux));
    HIPCHK(h, hipStreamDestroy(h->gemm));
    HIPCHK(h, hipStreamDestroy(h->aux));
    h->gemm = h->aux = nullptr;
    HIPCHK(h, create_overlap_streams(h));
    HIPCHK(h, hipEventRecord(h->ev_b2g, h->aux));
    h->main_dirty = true;
  }
  return LRDM_OK;
}

lrdm_status lrdm_get_tuning(lrdm_t h, lrdm_tuning* t) {
  if (!h || !t) return fail(h, LRDM_E_ARG, "null argument");
  const int nb = gram_blocks(h->n, h->plain ? 1 : 2);
  t->gram_blocks = h->tune.gram_blocks ? std::min(nb, h->tune.gram_blocks)
                                       : (h->overlap ? std::min(nb, h->gemm_cus) : nb);
  t->gram4_blocks = h->overlap ? (h->tune.gram4_blocks ? h->tune.gram4_blocks : h->gemm_cus) : 0;
  const int kl = local_budget(h->n, h->lay.r_pad, h->dt == LRDM_C64 ? 8 : 16);
  t->gate_local_max = h->tune.gate_local_max ? std::min(kl, h->tune.gate_local_max) : kl;
  t->aux_cus = h->overlap ? h->aux_cus : 0;
  return LRDM_OK;
}

lrdm_status lrdm_timing_begin(lrdm_t h, int kernel_class) {
  lrdm_status st = check_usable(h);
  if (st != LRDM_OK) return st;
  st = not_recording(h);
  if (st != LRDM_OK) return st;
  if (kernel_class < 0 || kernel_class > 6) return fail(h, LRDM_E_ARG, "kernel_class must be in [0, 6]");
  if (h->ev.empty()) {
    h->ev.resize(2 * kMaxTimed);
    h->ev_launches.assign(kMaxTimed, 1);
    for (auto& e : h->ev) HIPCHK(h, hipEventCreate(&e));
  }
  h->timing_class = kernel_class;
  h->ev_used = 0;
  return LRDM_OK;
}

lrdm_status lrdm_timing_end(lrdm_t h, int* launches, double* mean_ms, double* total_ms) {
  lrdm_status st = check_usable(h);
  if (st != LRDM_OK) return st;
  HIPCHK(h, hipStreamSynchronize(h->stream));
  if (h->overlap) {
    HIPCHK(h, hipStreamSynchronize(h->gemm));
    HIPCHK(h, hipStreamSynchronize(h->aux));
  }
  double tot = 0;
  const int npairs = h->ev_used / 2;
  int nl = 0;
  for (int i = 0; i < npairs; ++i) {
    float ms = 0;
    HIPCHK(h, hipEventElapsedTime(&ms, h->ev[2 * i], h->ev[2 * i + 1]));
    tot += ms;
    nl += h->ev_launches[i];
  }
  if (launches) *launches = nl;
  if (total_ms) *total_ms = tot;
  if (mean_ms) *mean_ms = nl ? tot / nl : 0.0;
  h->timing_class = -1;
  h->ev_used = 0;
  return LRDM_OK;
}

// ---------------------------------------------------------------- reverse sweep
lrdm_status lrdm_record_bytes(lrdm_t h, size_t* bytes) {
  lrdm_status st = check_usable(h);
  if (st != LRDM_OK) return st;
  if (!bytes) return fail(h, LRDM_E_ARG, "null output pointer");
  if (!h->lay.adjoint)
    return fail(h, LRDM_E_UNSUPPORTED, "compression records need the fused form and m_max * r_pad <= 64");
  *bytes = h->lay.rec_bytes;
  return LRDM_OK;
}

lrdm_status lrdm_checkpoint(lrdm_t h, void* dst_dev, int* rank_out) {
  lrdm_status st = ready_for_output(h);
  if (st != LRDM_OK) return st;
  if (!dst_dev) return fail(h, LRDM_E_ARG, "null destination");
  HIPCHK(h, hipMemcpyAsync(dst_dev, h->state, h->lay.state_bytes, hipMemcpyDeviceToDevice, h->stream));
  if (rank_out) *rank_out = h->c_bound;
  return LRDM_OK;
}

lrdm_status lrdm_restore(lrdm_t h, const void* src_dev, int rank) {
  lrdm_status st = check_usable(h);
  if (st != LRDM_OK) return st;
  st = not_recording(h);
  if (st != LRDM_OK) return st;
  if (!src_dev) return fail(h, LRDM_E_ARG, "null source");
  if (rank < 1 || rank > h->lay.r_pad) return fail(h, LRDM_E_ARG, "rank must be in [1, r_pad]");
  if (h->chan_pending) return fail(h, LRDM_E_STATE, "a Kraus channel is pending: call lrdm_compress first");
  h->gates.clear();
  h->proj_pending = false;
  st = join_aux(h);
  if (st != LRDM_OK) return st;
  HIPCHK(h, hipMemcpyAsync(h->state, src_dev, h->lay.state_bytes, hipMemcpyDeviceToDevice, h->stream));
  h->ncols = h->lay.r_pad;
  h->c_bound = rank;
  return LRDM_OK;
}

lrdm_status lrdm_apply_pauli_sum(lrdm_t dst, lrdm_t src, int n_terms, const uint64_t* xmask,
                                 const uint64_t* zmask, const double* coeff) {
  lrdm_status st = check_usable(dst);
  if (st != LRDM_OK) return st;
  st = not_recording(dst);
  if (st != LRDM_OK) return st;
  st = ready_for_output(src);
  if (st != LRDM_OK) return st;
  if (dst == src) return fail(dst, LRDM_E_ARG, "source and destination must be different handles");
  if (!same_shape(dst, src)) return fail(dst, LRDM_E_ARG, "handles differ in n, r, dtype, m_max or form");
  if (n_terms < 1 || n_terms > kMaxApplyTerms) return fail(dst, LRDM_E_ARG, "n_terms must be in [1, 4096]");
  if (!xmask || !zmask || !coeff) return fail(dst, LRDM_E_ARG, "null argument");
  st = check_masks(dst, n_terms, xmask, zmask);
  if (st != LRDM_OK) return st;
  if (dst->chan_pending) return fail(dst, LRDM_E_STATE, "a Kraus channel is pending on the destination");
  dst->gates.clear();
  dst->proj_pending = false;
  st = join_aux(dst);   // the destination's own streams are done with its state
  if (st != LRDM_OK) return st;
  st = order_streams(src, dst);
  if (st != LRDM_OK) return st;
  std::vector<uint64_t> stage(3 * (size_t)n_terms);
  std::memcpy(stage.data(), xmask, n_terms * 8);
  std::memcpy(stage.data() + n_terms, zmask, n_terms * 8);
  std::memcpy(stage.data() + 2 * n_terms, coeff, n_terms * 8);
  uint64_t* dterms = dst->ws<uint64_t>(dst->lay.off_terms);
  HIPCHK(dst, hipMemcpyAsync(dterms, stage.data(), stage.size() * 8, hipMemcpyHostToDevice, dst->stream));
  hipError_t e = dst->dt == LRDM_C64
                     ? launch_pauli_apply<float>(static_cast<float2*>(dst->state), static_cast<const float2*>(src->state), dst->n, dst->lay.ld, src->ncols, dterms, dterms + n_terms, reinterpret_cast<const double*>(dterms + 2 * n_terms), n_terms, dst->stream)
                     : launch_pauli_apply<double>(static_cast<double2*>(dst->state), static_cast<const double2*>(src->state), dst->n, dst->lay.ld, src->ncols, dterms, dterms + n_terms, reinterpret_cast<const double*>(dterms + 2 * n_terms), n_terms, dst->stream);
  HIPCHK(dst, e);
  // the staging vector is a local: wait for the upload before it goes out of scope
  HIPCHK(dst, hipStreamSynchronize(dst->stream));
  dst->ncols = src->ncols;
  dst->c_bound = src->c_bound;
  return LRDM_OK;
}

lrdm_status lrdm_pauli_overlap(lrdm_t bra, lrdm_t ket, int n_terms, const uint64_t* xmask,
                               const uint64_t* zmask, double* out_host) {
  lrdm_status st = ready_for_output(bra);
  if (st != LRDM_OK) return st;
  st = ready_for_output(ket);
  if (st != LRDM_OK) return st;
  if (!same_shape(bra, ket)) return fail(ket, LRDM_E_ARG, "handles differ in n, r, dtype, m_max or form");
  if (n_terms < 1 || n_terms > kMaxTerms) return fail(ket, LRDM_E_ARG, "n_terms must be in [1, 65536]");
  if (!xmask || !zmask || !out_host) return fail(ket, LRDM_E_ARG, "null argument");
  st = check_masks(ket, n_terms, xmask, zmask);
  if (st != LRDM_OK) return st;
  st = order_streams(bra, ket);
  if (st != LRDM_OK) return st;
  return pauli_values(ket, bra->state, n_terms, xmask, zmask, 1, out_host);
}

lrdm_status lrdm_compress_adjoint(lrdm_t bar, const void* x_dev, const void* rec_dev, int qubit,
                                  int m, const double* e) {
  lrdm_status st = check_usable(bar);
  if (st != LRDM_OK) return st;
  st = not_recording(bar);
  if (st != LRDM_OK) return st;
  if (!bar->lay.adjoint)
    return fail(bar, LRDM_E_UNSUPPORTED, "the reverse sweep needs the fused form and m_max * r_pad <= 64");
  if (!x_dev || !rec_dev || !e) return fail(bar, LRDM_E_ARG, "null argument");
  if (qubit < 0 || qubit >= bar->n) return fail(bar, LRDM_E_ARG, "qubit out of range");
  if (m < 1 || m > bar->m_max) return fail(bar, LRDM_E_ARG, "Kraus count must be in [1, m_max]");
  if (!kraus_complete(m, e)) return fail(bar, LRDM_E_ARG, "Kraus set is not complete within 1e-10");
  if (bar->chan_pending) return fail(bar, LRDM_E_STATE, "a Kraus channel is pending on the adjoint handle");
  st = settle(bar);
  if (st != LRDM_OK) return st;
  st = flush_gates(bar);
  if (st != LRDM_OK) return st;
  const Channel ch = make_channel(m, e);
  const AdjBufs b = adj_bufs(bar);
  hipError_t he = bar->dt == LRDM_C64
                      ? launch_compress_adjoint<float>(static_cast<float2*>(bar->state), static_cast<const float2*>(x_dev), bar->n, bar->lay.ld, bar->lay.r_pad, qubit, ch, static_cast<const double*>(rec_dev), b, bar->stream)
                      : launch_compress_adjoint<double>(static_cast<double2*>(bar->state), static_cast<const double2*>(x_dev), bar->n, bar->lay.ld, bar->lay.r_pad, qubit, ch, static_cast<const double*>(rec_dev), b, bar->stream);
  HIPCHK(bar, he);
  bar->ncols = bar->lay.r_pad;
  bar->c_bound = bar->lay.r_pad;
  return LRDM_OK;
}

// ---------------------------------------------------------------- batched serving
}  // extern "C"

struct lrdm_batch_ctx {
  struct Launch {
    int kind;          // RecKind, or -1 for a step stamp
    int cls, kmax, njobs;
    uint32_t blocks;
    size_t shm, off;   // off: job array (or stamp slot) offset in the plan buffer
  };
  std::vector<lrdm_t> hs;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::vector<hipStream_t> hstreams;   // distinct streams of the handles
  hipEvent_t ev_before = nullptr, ev_after = nullptr;
  bool recording = false;
  std::vector<Recorder> recs;
  std::vector<Launch> launches;
  std::vector<unsigned char> plan;
  size_t plan_bytes = 0;
  int nsteps = 0;
  std::vector<int> last_step;
  char* plan_dev = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  double ticks_per_ms = 0;
};

const lrdm_t* lrdm::batch_handles(lrdm_batch_t b, int* n) {
  *n = b ? (int)b->hs.size() : 0;
  return b ? b->hs.data() : nullptr;
}

namespace {

lrdm_status bfail(lrdm_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

void drop_graph(lrdm_batch_t b) {
  if (b->exec) hipGraphExecDestroy(b->exec);
  if (b->graph) hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  b->plan_dev = nullptr;
}

template <class J>
size_t put_jobs(std::vector<unsigned char>& plan, const std::vector<J>& jobs) {
  const size_t off = align_up(plan.size());
  plan.resize(off + jobs.size() * sizeof(J));
  std::memcpy(plan.data() + off, jobs.data(), jobs.size() * sizeof(J));
  return off;
}

int eig_class(int N) { return N <= 32 ? 0 : (N <= 64 ? 1 : 2); }

// Lockstep schedule: step s of every instance (the operations up to and including its s-th
// projection) is issued together, one batched launch per kernel kind and size class.
lrdm_status build_plan(lrdm_batch_t b) {
  const int ni = (int)b->hs.size();
  std::vector<std::vector<std::vector<RecItem>>> steps(ni);
  b->nsteps = 0;
  b->last_step.assign(ni, -1);
  for (int i = 0; i < ni; ++i) {
    std::vector<RecItem> cur;
    for (const RecItem& it : b->recs[i].items) {
      if (!cur.empty() && it.kind < cur.back().kind && !(it.kind == REC_GATE && cur.back().kind == REC_GATE))
        return bfail(LRDM_E_UNSUPPORTED, "batched instances must issue resets, gates and then one compression per step");
      cur.push_back(it);
      if (it.kind == REC_PROJ) {
        steps[i].push_back(cur);
        cur.clear();
      }
    }
    if (!cur.empty()) steps[i].push_back(cur);
    b->last_step[i] = (int)steps[i].size() - 1;
    b->nsteps = std::max(b->nsteps, (int)steps[i].size());
  }
  b->plan.assign(align_up((size_t)(b->nsteps + 1) * 8), 0);
  b->launches.clear();
  for (int s = 0; s < b->nsteps; ++s) {
    // resets
    {
      std::vector<ResetJob> jobs;
      uint32_t blocks = 0;
      for (int i = 0; i < ni; ++i) {
        if (s >= (int)steps[i].size()) continue;
        for (const RecItem& it : steps[i][s])
          if (it.kind == REC_RESET) {
            ResetJob j = b->recs[i].resets[it.idx];
            j.block0 = blocks;
            blocks += j.nblocks;
            jobs.push_back(j);
          }
      }
      if (!jobs.empty()) b->launches.push_back({REC_RESET, 0, 0, (int)jobs.size(), blocks, 0, put_jobs(b->plan, jobs)});
    }
    // gate passes, by their position inside the step
    for (int g = 0;; ++g) {
      std::vector<GateJob<float>> jobs;
      uint32_t blocks = 0;
      size_t shm = 0;
      for (int i = 0; i < ni; ++i) {
        if (s >= (int)steps[i].size()) continue;
        int seen = 0;
        for (const RecItem& it : steps[i][s])
          if (it.kind == REC_GATE && seen++ == g) {
            GateJob<float> j = b->recs[i].gates[it.idx];
            j.block0 = blocks;
            blocks += j.nblocks;
            shm = std::max(shm, it.shm);
            jobs.push_back(j);
          }
      }
      if (jobs.empty()) break;
      b->launches.push_back({REC_GATE, 0, 0, (int)jobs.size(), blocks, shm, put_jobs(b->plan, jobs)});
    }
    // Gram, by width
    for (int F : {16, 32, 64, 128, 256}) {
      std::vector<GramJob<float>> jobs;
      uint32_t blocks = 0;
      for (int i = 0; i < ni; ++i) {
        if (s >= (int)steps[i].size()) continue;
        for (const RecItem& it : steps[i][s])
          if (it.kind == REC_GRAM && it.cls == F) {
            GramJob<float> j = b->recs[i].grams[it.idx];
            j.block0 = blocks;
            blocks += j.nblocks;
            jobs.push_back(j);
          }
      }
      if (!jobs.empty()) b->launches.push_back({REC_GRAM, F, 0, (int)jobs.size(), blocks, 0, put_jobs(b->plan, jobs)});
    }
    // Gram reductions
    {
      std::vector<ReduceJob<float>> jobs;
      uint32_t blocks = 0;
      for (int i = 0; i < ni; ++i) {
        if (s >= (int)steps[i].size()) continue;
        for (const RecItem& it : steps[i][s])
          if (it.kind == REC_REDUCE) {
            ReduceJob<float> j = b->recs[i].reds[it.idx];
            j.block0 = blocks;
            blocks += it.blocks;
            jobs.push_back(j);
          }
      }
      if (!jobs.empty()) b->launches.push_back({REC_REDUCE, 0, 0, (int)jobs.size(), blocks, 0, put_jobs(b->plan, jobs)});
    }
    // eigensolves, one work-group each, by size class
    for (int cl = 0; cl < 3; ++cl) {
      std::vector<EigJob<float>> jobs;
      int kmax = 1, Nmax = 1;
      for (int i = 0; i < ni; ++i) {
        if (s >= (int)steps[i].size()) continue;
        for (const RecItem& it : steps[i][s])
          if (it.kind == REC_EIG && eig_class(it.cls) == cl) {
            jobs.push_back(b->recs[i].eigs[it.idx]);
            kmax = std::max(kmax, it.kmax);
            Nmax = std::max(Nmax, it.cls);
          }
      }
      if (!jobs.empty())
        b->launches.push_back({REC_EIG, Nmax, kmax, (int)jobs.size(), (uint32_t)jobs.size(), 0, put_jobs(b->plan, jobs)});
    }
    // projections, by output width
    for (int FO : {16, 32, 64, 128, 256}) {
      std::vector<ProjJob<float>> jobs;
      uint32_t blocks = 0;
      for (int i = 0; i < ni; ++i) {
        if (s >= (int)steps[i].size()) continue;
        for (const RecItem& it : steps[i][s])
          if (it.kind == REC_PROJ && it.cls == FO) {
            ProjJob<float> j = b->recs[i].projs[it.idx];
            j.block0 = blocks;
            blocks += j.nblocks;
            jobs.push_back(j);
          }
      }
      if (!jobs.empty()) b->launches.push_back({REC_PROJ, FO, 0, (int)jobs.size(), blocks, 0, put_jobs(b->plan, jobs)});
    }
    b->launches.push_back({-1, 0, 0, 0, 0, 0, (size_t)(s + 1) * 8});
  }
  b->plan_bytes = align_up(b->plan.size());
  b->plan.resize(b->plan_bytes, 0);
  return LRDM_OK;
}

hipError_t issue(lrdm_batch_t b, const lrdm_batch_ctx::Launch& L) {
  char* base = b->plan_dev;
  switch (L.kind) {
    case -1: return launch_stamp(reinterpret_cast<uint64_t*>(base + L.off), b->stream);
    case REC_RESET:
      return launch_reset_batched(reinterpret_cast<const ResetJob*>(base + L.off), L.njobs, L.blocks, 8, b->stream);
    case REC_GATE:
      return launch_gate_pass_batched<float>(reinterpret_cast<const GateJob<float>*>(base + L.off), L.njobs,
                                             L.blocks, L.shm, b->stream);
    case REC_GRAM:
      return launch_gram_batched<float>(L.cls, reinterpret_cast<const GramJob<float>*>(base + L.off), L.njobs,
                                        L.blocks, b->stream);
    case REC_REDUCE:
      return launch_gram_reduce_batched<float>(reinterpret_cast<const ReduceJob<float>*>(base + L.off), L.njobs,
                                               L.blocks, b->stream);
    case REC_EIG:
      return launch_eig_batched<float>(L.cls, reinterpret_cast<const EigJob<float>*>(base + L.off), L.njobs, L.kmax,
                                       b->stream);
    case REC_PROJ:
      return launch_project_batched<float>(L.cls, reinterpret_cast<const ProjJob<float>*>(base + L.off), L.njobs,
                                           L.blocks, b->stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

extern "C" {

lrdm_status lrdm_batch_create(lrdm_batch_t* out, int n_inst, const lrdm_t* handles, void* hip_stream) {
  if (!out) return bfail(LRDM_E_ARG, "null output handle pointer");
  *out = nullptr;
  if (n_inst < 1 || !handles) return bfail(LRDM_E_ARG, "need at least one handle");
  for (int i = 0; i < n_inst; ++i) {
    lrdm_t h = handles[i];
    lrdm_status st = check_usable(h);
    if (st != LRDM_OK) return st;
    if (h->dt != LRDM_C64) return bfail(LRDM_E_UNSUPPORTED, "batched serving runs complex64 handles");
    if (h->plain) return bfail(LRDM_E_UNSUPPORTED, "batched serving runs the fused form");
    if (h->rec) return bfail(LRDM_E_STATE, "a handle is already being recorded");
    for (int j = 0; j < i; ++j)
      if (handles[j] == h) return bfail(LRDM_E_ARG, "repeated handle");
  }
  lrdm_batch_ctx* b = new lrdm_batch_ctx();
  b->hs.assign(handles, handles + n_inst);
  b->stream = static_cast<hipStream_t>(hip_stream);
  hipError_t e = hipSuccess;
  if (!b->stream) {   // graphs are captured on a non-default stream (default priority)
    e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
    b->own_stream = (e == hipSuccess);
  }
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_before, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_after, hipEventDisableTiming);
  if (e != hipSuccess) {
    if (b->own_stream) hipStreamDestroy(b->stream);
    if (b->ev_before) hipEventDestroy(b->ev_before);
    delete b;
    return bfail(LRDM_E_HIP, std::string("batch stream/event: ") + hipGetErrorString(e));
  }
  for (lrdm_t h : b->hs)
    if (h->stream != b->stream &&
        std::find(b->hstreams.begin(), b->hstreams.end(), h->stream) == b->hstreams.end())
      b->hstreams.push_back(h->stream);
  b->recs.resize(n_inst);
  *out = b;
  return LRDM_OK;
}

lrdm_status lrdm_batch_begin(lrdm_batch_t b) {
  if (!b) return bfail(LRDM_E_ARG, "null batch");
  if (b->recording) return bfail(LRDM_E_STATE, "already recording");
  for (lrdm_t h : b->hs) {
    lrdm_status st = check_usable(h);
    if (st != LRDM_OK) return st;
    if (h->rec) return bfail(LRDM_E_STATE, "a handle is already being recorded");
    if (h->chan_pending) return bfail(LRDM_E_STATE, "a handle has a pending Kraus channel");
  }
  for (size_t i = 0; i < b->hs.size(); ++i) {
    lrdm_t h = b->hs[i];
    lrdm_status st = settle(h);
    if (st != LRDM_OK) return st;
    st = flush_gates(h);
    if (st != LRDM_OK) return st;
    HIPCHK(h, hipStreamSynchronize(h->stream));
    b->recs[i] = Recorder();
    h->rec = &b->recs[i];
  }
  drop_graph(b);
  b->recording = true;
  return LRDM_OK;
}

lrdm_status lrdm_batch_end(lrdm_batch_t b, size_t* plan_bytes) {
  if (!b || !plan_bytes) return bfail(LRDM_E_ARG, "null argument");
  if (!b->recording) return bfail(LRDM_E_STATE, "not recording");
  lrdm_status result = LRDM_OK;
  for (lrdm_t h : b->hs) {
    lrdm_status st = flush_gates(h);
    if (st != LRDM_OK && result == LRDM_OK) result = st;
    if (h->chan_pending && result == LRDM_OK)
      result = bfail(LRDM_E_STATE, "a recorded program ends with a Kraus channel that was not compressed");
    h->rec = nullptr;
  }
  b->recording = false;
  if (result != LRDM_OK) return result;
  lrdm_status st = build_plan(b);
  if (st != LRDM_OK) return st;
  *plan_bytes = b->plan_bytes;
  return LRDM_OK;
}

lrdm_status lrdm_batch_instantiate(lrdm_batch_t b, void* plan_dev, size_t plan_bytes) {
  if (!b || !plan_dev) return bfail(LRDM_E_ARG, "null argument");
  if (b->recording || b->plan_bytes == 0) return bfail(LRDM_E_STATE, "record and end the batch first");
  if (plan_bytes < b->plan_bytes) return bfail(LRDM_E_NOMEM, "plan buffer smaller than lrdm_batch_end reported");
  if (reinterpret_cast<uintptr_t>(plan_dev) & 255) return bfail(LRDM_E_ARG, "plan buffer must be 256-byte aligned");
  drop_graph(b);
  b->plan_dev = static_cast<char*>(plan_dev);
  hipError_t e = hipMemcpy(plan_dev, b->plan.data(), b->plan_bytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) return bfail(LRDM_E_HIP, std::string("hipMemcpy: ") + hipGetErrorString(e));
  int dev = 0, khz = 0;
  hipGetDevice(&dev);
  e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
  if (e != hipSuccess || khz <= 0) return bfail(LRDM_E_HIP, "cannot read the device wall-clock rate");
  b->ticks_per_ms = (double)khz;
  e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeRelaxed);
  if (e != hipSuccess) return bfail(LRDM_E_HIP, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
  hipError_t le = launch_stamp(reinterpret_cast<uint64_t*>(b->plan_dev), b->stream);
  for (size_t i = 0; i < b->launches.size() && le == hipSuccess; ++i) le = issue(b, b->launches[i]);
  e = hipStreamEndCapture(b->stream, &b->graph);
  if (le != hipSuccess) {
    drop_graph(b);
    return bfail(LRDM_E_HIP, std::string("batched launch: ") + hipGetErrorString(le));
  }
  if (e != hipSuccess) {
    drop_graph(b);
    return bfail(LRDM_E_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  }
  e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    drop_graph(b);
    return bfail(LRDM_E_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  }
  b->plan_dev = static_cast<char*>(plan_dev);
  return LRDM_OK;
}

lrdm_status lrdm_batch_launch(lrdm_batch_t b) {
  if (!b) return bfail(LRDM_E_ARG, "null batch");
  if (!b->exec) return bfail(LRDM_E_STATE, "instantiate the batch first");
  // the replay waits for work queued on the handles' streams, and later work there waits for it
  hipError_t e = hipSuccess;
  for (hipStream_t hs : b->hstreams) {
    if (e == hipSuccess) e = hipEventRecord(b->ev_before, hs);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->stream, b->ev_before, 0);
  }
  if (e == hipSuccess) e = hipGraphLaunch(b->exec, b->stream);
  if (e == hipSuccess) e = hipEventRecord(b->ev_after, b->stream);
  for (hipStream_t hs : b->hstreams)
    if (e == hipSuccess) e = hipStreamWaitEvent(hs, b->ev_after, 0);
  if (e != hipSuccess) return bfail(LRDM_E_HIP, std::string("batch launch: ") + hipGetErrorString(e));
  return LRDM_OK;
}

lrdm_status lrdm_batch_info(lrdm_batch_t b, int* n_steps, int* n_launches) {
  if (!b) return bfail(LRDM_E_ARG, "null batch");
  if (n_steps) *n_steps = b->nsteps;
  if (n_launches) *n_launches = (int)b->launches.size() + 1;
  return LRDM_OK;
}

lrdm_status lrdm_batch_times(lrdm_batch_t b, double* done_ms, double* total_ms) {
  if (!b) return bfail(LRDM_E_ARG, "null batch");
  if (!b->exec) return bfail(LRDM_E_STATE, "instantiate and launch the batch first");
  hipError_t e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return bfail(LRDM_E_HIP, std::string("hipStreamSynchronize: ") + hipGetErrorString(e));
  std::vector<uint64_t> st(b->nsteps + 1);
  e = hipMemcpy(st.data(), b->plan_dev, st.size() * 8, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return bfail(LRDM_E_HIP, std::string("hipMemcpy: ") + hipGetErrorString(e));
  if (done_ms)
    for (size_t i = 0; i < b->hs.size(); ++i)
      done_ms[i] = b->last_step[i] >= 0 ? (double)(st[b->last_step[i] + 1] - st[0]) / b->ticks_per_ms : 0.0;
  if (total_ms) *total_ms = (double)(st[b->nsteps] - st[0]) / b->ticks_per_ms;
  return LRDM_OK;
}

lrdm_status lrdm_batch_destroy(lrdm_batch_t b) {
  if (!b) return bfail(LRDM_E_ARG, "null batch");
  if (b->recording)
    for (lrdm_t h : b->hs) h->rec = nullptr;
  drop_graph(b);
  if (b->ev_before) hipEventDestroy(b->ev_before);
  if (b->ev_after) hipEventDestroy(b->ev_after);
  if (b->own_stream) hipStreamDestroy(b->stream);
  delete b;
  return LRDM_OK;
}

}  // extern "C"
