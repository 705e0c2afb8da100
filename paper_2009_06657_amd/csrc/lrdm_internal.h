// Internal declarations shared by the HIP kernels and the host runtime of liblrdm.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lrdm.h"

namespace lrdm {

constexpr int kMaxEig = 128;      // largest Gram order the single-work-group eigensolver takes
constexpr int kGateMaxOps = 40;   // operations per fused gate pass (kernel-argument budget)
constexpr int kGateMaxCoef = 288; // real coefficients per fused gate pass
constexpr int kGateMaxPhases = 16; // register phases per fused gate pass

template <class T> struct Cx;
template <> struct Cx<float> { using type = float2; };
template <> struct Cx<double> { using type = double2; };
template <class T> using cx_t = typename Cx<T>::type;

enum GateOpType : int { OP_1Q = 0, OP_2Q = 1, OP_DIAG1 = 2, OP_DIAG2 = 3, OP_WEIGHT = 4 };

// One fused sweep over L: every row tile holds the 2^k rows that differ only in the k "local"
// qubits; general 1q/2q gates act on local qubits, diagonal gates on any qubit (the full row
// index is known).  Operations are applied in list order.
// With n_phases > 0 the operations are applied in register phases: phase p holds the tile rows
// that differ in 4 local slots in registers (ph_word[p] bits 4b .. 4b + 3: the slot of register
// bit b; bits 16 + 4t ..: the other k - 4 local slots, ascending, which come from the thread
// index).  It first applies one 2x2 gate on each register bit b, coefficients at offset
// (ph_gc[p][b / 2] >> (16 * (b & 1))) & 0xffff (identity coefficients where the phase has fewer
// gates; the gates act on distinct qubits, so their order is free), then its diagonal
// operations, which commute with each other: those with real phases whose qubits are both
// register bits as one product, the 16 real phases of the register patterns at coefficient
// offset ph_u[p] & 0xffff (bit 16: present), then ph_diag[first .. first + nreal) with real phases
// and ph_diag[first + nreal .. first + nreal + ncplx) with complex ones (ph_ops[p]: first in
// bits 0 .. 7, nreal in bits 8 .. 15, ncplx in bits 16 .. 23).  A diagonal operation may act in
// any phase between the gates on its qubits that precede it in list order and those that
// follow it, so the list order's result is kept.  A listed diagonal operation carries its
// register bits in op_code ((ra + 1) * 5 + rb + 1, -1: not a register bit of the phase), with a
// register qubit first and two register qubits ascending (op_a / op_b and the middle two phases
// swapped to match).
// n_phases = 0: one LDS sweep per operation.
template <class T> struct GatePass {
  int n, k, ld, ncols, n_ops, n_phases;
  int last_gates;      // one-qubit gates of the last phase (its other register bits get the identity)
  int local_q[8];      // local bit j <-> qubit local_q[j]
  int sorted_q[8];     // the same qubits in ascending order (row-index deposit)
  int op_type[kGateMaxOps];
  int op_a[kGateMaxOps];
  int op_b[kGateMaxOps];
  int op_coef[kGateMaxOps];
  int op_code[kGateMaxOps];
  int ph_diag[kGateMaxOps];
  uint32_t ph_word[kGateMaxPhases];
  uint32_t ph_ops[kGateMaxPhases];
  uint32_t ph_gc[kGateMaxPhases][2];
  uint32_t ph_u[kGateMaxPhases];
  T coef[kGateMaxCoef];
};

// Device-side record of one compression (mirrors lrdm_compress_info).
struct DevInfo {
  int k;
  int n_eig;
  int status;          // 0 ok, else LRDM_E_EIG
  int pad;
  double discarded;
  double discarded_total;
  double trace;
  double gap;
  double lambda_max;
  double scale;
};

// Kraus set for the fused compression, FP64: e[a][row][col] interleaved.
struct Channel {
  int m;
  double e[4][2][2][2];
};

// Scratch carved from the caller's workspace for one compression.
struct EigBufs {
  double* S;        // (F/2)^2 complex, Gram of the split view, full Hermitian, row-major
  double* P;        // packed Householder reflector entries, (N-1)(N-2)/2 complex
  double* lam;      // kept-candidate eigenvalues, descending
  DevInfo* info;
  double* rec;      // nullable: compression record for the reverse sweep (every eigenpair)
  double* W64;      // nullable: W in FP64 as well (split view), for chained compressions
  double* Y;        // reflector scalars tau_j (2 (N - 1) doubles), then at kEigYOff the kept
                    // eigenvectors of T, column t at t * kMaxEig (eigensolver -> back-transform)
  // a channel on a qubit pair (nsplit = 4): (E_a^H E_b)_{u u'} at ((a m + b) 4 + u) 4 + u' and
  // (E_a)_{u' u} at (a 4 + u') 4 + u, complex FP64 (null otherwise)
  const double* M4 = nullptr;
  const double* E4 = nullptr;
};
constexpr int kEigYOff = 2 * kMaxEig;
// after the eigenvectors: the scaled T (d, e, e^2), tau, the trace and the Gershgorin norm,
// handed between the kernels of a single (unbatched) eigensolve
constexpr int kEigTOff = kEigYOff + 64 * kMaxEig;
constexpr size_t kEigYDoubles = (size_t)kEigTOff + 5 * (size_t)kMaxEig + 8;
constexpr int kEigBtCols = 4;                 // back-transform: columns (one wave each) per work-group
constexpr int kEigBtBlocks = 64 / kEigBtCols; // work-groups per eigensolve (at most 64 columns)

// Compression record (FP64), written by the eigensolver when EigBufs::rec is set:
// [0] k, [1] scale c, [2] N, [3] Tr G, [4] renorm, [5..8) unused, [8, 8 + N) eigenvalues
// (descending), then V as N x N complex row-major (column j = eigenvector j), interleaved.
constexpr int kRecHeader = 8;
inline size_t record_doubles(int N) { return (size_t)kRecHeader + N + 2 * (size_t)N * N; }
constexpr int kRecMaxN = 64;      // largest Gram order with a full record

// ---------------------------------------------------------------- batched launches
// A batched launch covers one kernel kind for many independent states: job j owns the blocks
// [block0, block0 + nblocks) of the grid (or block j for one-block jobs).
template <class J>
__device__ __forceinline__ int find_job(const J* __restrict__ jobs, int njobs, uint32_t b) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].block0 <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <class T> struct GateJob {
  GatePass<T> p;
  cx_t<T>* L;
  int cshift;
  uint32_t block0, nblocks;
};
template <class T> struct GramJob {
  const cx_t<T>* L;
  T* partials;
  int ld, seg_shift, nsplit, q;
  uint32_t rows, rows_per_block, block0, nblocks;
};
template <class T> struct ReduceJob {
  const T* partials;
  double* S;
  int nblocks, NT, NUP;
  uint32_t block0;
};
template <class T> struct EigJob {
  const double* S;
  Channel ch;
  int Fc, nsplit, c, N, kmax, r_target, tie, renorm, c_out;
  double eps;
  EigBufs B;
  cx_t<T>* W;
};
template <class T> struct ProjJob {
  cx_t<T>* L;
  const cx_t<T>* W;
  int ld, F, seg_in_shift, nsplit, q, seg_out_shift, skip;
  uint32_t rows, block0, nblocks;
};
struct ResetJob {
  void* state;
  DevInfo* info;
  uint64_t state_bytes;
  uint32_t block0, nblocks;
};

// Batched launchers (jobs in device memory; the host also keeps the launch shape)
template <class T> hipError_t launch_gate_pass_batched(const GateJob<T>* jobs, int njobs, uint32_t blocks, size_t shm, hipStream_t s);
template <class T> hipError_t launch_gram_batched(int F, const GramJob<T>* jobs, int njobs, uint32_t blocks, hipStream_t s);
template <class T> hipError_t launch_gram_reduce_batched(const ReduceJob<T>* jobs, int njobs, uint32_t blocks, hipStream_t s);
template <class T> hipError_t launch_eig_batched(int N, const EigJob<T>* jobs, int njobs, int kmax_max, hipStream_t s);
template <class T> hipError_t launch_project_batched(int FO, const ProjJob<T>* jobs, int njobs, uint32_t blocks, hipStream_t s);
hipError_t launch_reset_batched(const ResetJob* jobs, int njobs, uint32_t blocks, int complex_bytes, hipStream_t s);
hipError_t launch_stamp(uint64_t* slot, hipStream_t s);

// Launch-shape helpers shared by the single and batched paths
int gram_seg_shift(int c);                       // log2(2c), -1 if 2c is not a power of two
uint32_t gram_rows_per_block(int n, int nsplit, int nblocks);
size_t gate_pass_shm(int ncols, int k, size_t csize, int n_phases);

// ---------------------------------------------------------------- launchers (k_*.hip)
template <class T>
hipError_t launch_gate_pass(const GatePass<T>& p, cx_t<T>* L, hipStream_t s);

template <class T>
hipError_t launch_kraus_expand(cx_t<T>* L, int n, int ld, int c, int q, const Channel& ch,
                               int m_pad, hipStream_t s);

// Operators [a0, a0 + na) of a two-qubit Kraus set (4 x 4, local index b(q0) + 2 b(q1)) for one
// plain-form expansion launch; m is the set's size (slots a >= m are zero padding).
constexpr int kKraus2PerLaunch = 8;
struct Kraus2Chunk {
  int a0, na, m;
  double e[kKraus2PerLaunch][4][4][2];
};
template <class T>
hipError_t launch_kraus2_expand(cx_t<T>* L, int n, int ld, int c, int q0, int q1, const Kraus2Chunk& ck,
                                hipStream_t s);

// Sparse initial state: L = 0 except L[idx[i] * ld] = amp[i] (interleaved FP64), i < count
// (idx, amp in device memory).
template <class T>
hipError_t launch_set_sparse(cx_t<T>* L, int ld, const uint64_t* idx, const double* amp, int count, hipStream_t s);
// rho = L L^H (rho row-major 2^n x 2^n complex64, the full-rank comparator's layout), FP64 sums.
template <class T>
hipError_t launch_lr_to_full(const cx_t<T>* L, int n, int ld, int ncols, float2* rho, hipStream_t s);

template <class T>
hipError_t launch_gram(const cx_t<T>* L, int n, int ld, int c, int nsplit, int q, T* partials,
                       int nblocks, hipStream_t s);

template <class T>
hipError_t launch_gram_reduce(const T* partials, int nblocks, int F, double* S, hipStream_t s);

// Eigensolve of G (order N <= 128), rank rule and projection matrix W; one work-group.
template <class T>
hipError_t launch_eig(const double* S, int Fc, const Channel& ch, int nsplit, int c, int N,
                      int kmax, int r_target, double eps, int tie, int renorm, int c_out,
                      const EigBufs& b, cx_t<T>* W, hipStream_t s);

// skip (split view only): bit 0 = the block of W from input half 0 to output half 1 is zero,
// bit 1 = the block from input half 1 to output half 0 is zero (Kraus sets that never map that
// value of the qubit to the other); those MFMAs are left out.
template <class T>
hipError_t launch_project(cx_t<T>* L, int n, int ld, int c_in, int nsplit, int q, int c_out,
                          const cx_t<T>* W, int skip, hipStream_t s, int cus = 0);   // cus: CUs of s

// Projection of a channel on the qubit pair (q0, q1): the 4-way view X4 = [L_0 | L_1 | L_2 | L_3]
// (u = b(q0) + 2 b(q1), 2^(n-2) rows) times W (4c x 4c_out), in place.
template <class T>
hipError_t launch_project4(cx_t<T>* L, int n, int ld, int c_in, int q0, int q1, int c_out, const cx_t<T>* W,
                           hipStream_t s);

template <class T>
hipError_t launch_probabilities(const cx_t<T>* L, int n, int ld, int ncols, double* p,
                                hipStream_t s);

template <class T>
hipError_t launch_zstats(const cx_t<T>* L, int n, int ld, int ncols, double* partials,
                         int nblocks, double* out, hipStream_t s);

// Tr(bra^H P_t ket) per term; out[t] = real part (complex_out = 0) or out[2t], out[2t + 1] =
// (re, im) (complex_out = 1).  bra == ket gives expectation values.
template <class T>
hipError_t launch_pauli(const cx_t<T>* bra, const cx_t<T>* ket, int n, int ld, int ncols,
                        const uint64_t* xm, const uint64_t* zm, int n_terms, double* partials,
                        int nblocks, double* out, int complex_out, hipStream_t s);

// ---------------------------------------------------------------- chained compressions (k_chain.hip)
// Two compressions on the same qubit with nothing in between share the split view: the second
// acts on X W_1, so its Gram matrix is W_1^H S W_1 and both projections compose into X (W_1 W_2).
// S <- W^H S W (Hermitian part), n x n complex FP64, tmp: n x n scratch.
hipError_t launch_chain_gram(double* S, const double* W, double* tmp, int n, hipStream_t s);
// Wp <- Wp Wn (FP64) and Wt <- Wp in the bulk precision; tmp: n x n scratch.
template <class T>
hipError_t launch_chain_compose(double* Wp, const double* Wn, double* tmp, cx_t<T>* Wt, int n, hipStream_t s);

// ---------------------------------------------------------------- overlapped compressions
// 4-way Gram G4 (4c x 4c complex FP64, row-major, index (bit q, bit p, column)) of the factor on
// the bit pair (p, q): the halves with bit q = 0 and 1 (split Gram on p; partials part_h, 2
// gram4_blocks_halves(n) blocks of the upper tiles of width 4c) and the cross block (partials
// part_c, gram4_blocks_cross(n) blocks of every tile), reduced in a fixed order in FP64.  For
// complex64 with c = 64 and at least 16 rows one streamed pass forms every block instead (one
// partial per work-group from part_h on, summed in FP64 in a fixed order; part_c must be where
// the layout above puts it).  max_blocks: the CUs the stream may use (at most that many
// work-groups per pass).
template <class T>
hipError_t launch_gram4(const cx_t<T>* L, int n, int ld, int c, int p, int q, T* part_h, T* part_c, double* S4,
                        int max_blocks, hipStream_t s);
int gram4_blocks_halves(int n);
int gram4_blocks_cross(int n);
// Floats of the complex64 c = 64 streamed form (one partial per work-group, then FP64 range
// sums); the partial region of the 4-way Gram holds at least this much in complex64.
size_t gram4_stream_reals(int n);
// Split Gram on q (2c x 2c, written to S) of the factor after the projection W (2c x 2c, FP64)
// on p, from G4 taken before that projection; T: 3 (2c)^2 complex FP64 scratch.
hipError_t launch_pair_transform(const double* G4, const double* W, double* T, double* S, int c, hipStream_t s);

// ---------------------------------------------------------------- full-rank comparator (k_fdm.hip)
constexpr int kFdmLowBits = 5;     // index bits 0..4 are local in every pass (256-byte runs)
constexpr int kFdmMaxLocal = 13;   // 2^13 complex64 = 64 KB tile
constexpr int kFdmMaxOps = 48;
constexpr int kFdmMaxCoef = 512;

// One fused pass over the 2n-bit vector form of rho: local slot j <-> index bit local_q[j]
// (slots 0..4 are bits 0..4); ops on slots (1q, 2q) or on any index bit (diagonal).
// With n_phases > 0 (full tiles of kFdmMaxLocal bits) the operations run in register phases:
// phase p holds the tile elements differing in the tile slots ph_slots[p][0 .. 4) in registers
// and applies operations [ph_first[p], ph_first[p] + ph_count[p]); op_a / op_b of a 1- or
// 2-bit operation are then register bit indices (op_a < op_b for 2-bit operations), and an
// operand of a diagonal operation that is a register bit is 64 + register (register operands
// first, ascending).
constexpr int kFdmMaxPhases = kFdmMaxOps + 2;   // + an empty load and store phase
struct FdmPass {
  int nbits, k, n_ops, n_phases;
  int local_q[kFdmMaxLocal];
  int sorted_hi[kFdmMaxLocal];   // local bits above the low block, ascending
  int op_type[kFdmMaxOps];
  int op_a[kFdmMaxOps];
  int op_b[kFdmMaxOps];
  int op_coef[kFdmMaxOps];
  unsigned char ph_first[kFdmMaxPhases];
  unsigned char ph_count[kFdmMaxPhases];
  unsigned char ph_slots[kFdmMaxPhases][4];
  float coef[kFdmMaxCoef];
};

hipError_t launch_fdm_pass(const FdmPass& p, float2* rho, hipStream_t s);
hipError_t launch_fdm_reset(float2* rho, int n, hipStream_t s);
hipError_t launch_fdm_diag(const float2* rho, int n, double* p, hipStream_t s);
constexpr int kFdmMaxQubits = 16;
struct FdmPhase {   // Hamming-weight phase table, FP64 interleaved
  double ph[2 * (kFdmMaxQubits + 1)];
};
hipError_t launch_fdm_weight(float2* rho, int n, const FdmPhase& ph, hipStream_t s);

// ---------------------------------------------------------------- reverse sweep (k_adj.hip)
// dst = sum_t coeff[t] P_t src, column by column (terms: xm[n], zm[n], coeff[n] as doubles).
template <class T>
hipError_t launch_pauli_apply(cx_t<T>* dst, const cx_t<T>* src, int n, int ld, int ncols,
                              const uint64_t* xm, const uint64_t* zm, const double* coeff,
                              int n_terms, hipStream_t s);

// Scratch of the compression adjoint, carved from the workspace (all FP64 complex unless noted).
struct AdjBufs {
  double* part;     // cross-Gram partials, kAdjChunks x (2c)^2
  double* C;        // (2c)^2, C = X^H Ybar on the split view
  double* H;        // N x c
  double* Zh;       // N x c
  double* T1;       // N x N
  double* Gh;       // N x N
  double* M;        // N x N
  void* P;          // (2c)^2 in the bulk precision
  void* Q;          // (2c)^2 in the bulk precision
};
constexpr int kAdjChunks = 256;
inline size_t adj_doubles(int c, int N) {
  const size_t w = 2 * (size_t)c, e = w * w;
  return 2 * (e * kAdjChunks + e + 2 * (size_t)N * c + 3 * (size_t)N * N) + 2 * 2 * e;
}

// Split-view Gram S = X^H X (Fc = 2c, full Hermitian, FP64) with FP64 products and sums.
template <class T>
hipError_t launch_gram_exact(const cx_t<T>* L, int n, int ld, int c, int q, double* part, double* S,
                             hipStream_t s);

// Reverse of one fused channel + compression on qubit q: Ybar (the adjoint of the compressed
// factor, state layout, c columns) is replaced in place by the adjoint of the factor before the
// channel, given the forward factor X before the channel and the compression record.
template <class T>
hipError_t launch_compress_adjoint(cx_t<T>* Ybar, const cx_t<T>* X, int n, int ld, int c, int q,
                                   const Channel& ch, const double* rec, const AdjBufs& b,
                                   hipStream_t s);

hipError_t launch_sample(const double* p, int n, double* cdf, double* block_sums,
                         const double* u, int count, uint64_t* out, hipStream_t s);

template <class T>
hipError_t launch_set_e0(cx_t<T>* L, hipStream_t s);

int gram_blocks(int n, int nsplit);   // number of split-K partials the Gram uses

void set_last_error(const char* msg);   // the calling thread's last error (lrdm_last_error(NULL))

// the handles of a batch, in creation order
const lrdm_t* batch_handles(lrdm_batch_t b, int* n);
// the full-rank handle's state: rho, n and stream (after applying its queued operations)
lrdm_status fdm_state(lrdm_fdm_t f, float2** rho, int* n, hipStream_t* s);
// drop the full-rank handle's queued operations (its state is about to be replaced)
void fdm_discard_queue(lrdm_fdm_t f);

}  // namespace lrdm
