// Internal declarations shared by the HIP kernels and the host runtime of liblrdm.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lrdm.h"

namespace lrdm {

constexpr int kMaxEig = 128;      // largest Gram order the single-work-group eigensolver takes
constexpr int kGateMaxOps = 40;   // operations per fused gate pass (kernel-argument budget)
constexpr int kGateMaxCoef = 288; // real coefficients per fused gate pass

template <class T> struct Cx;
template <> struct Cx<float> { using type = float2; };
template <> struct Cx<double> { using type = double2; };
template <class T> using cx_t = typename Cx<T>::type;

enum GateOpType : int { OP_1Q = 0, OP_2Q = 1, OP_DIAG1 = 2, OP_DIAG2 = 3, OP_WEIGHT = 4 };

// One fused sweep over L: every row tile holds the 2^k rows that differ only in the k "local"
// qubits; general 1q/2q gates act on local qubits, diagonal gates on any qubit (the full row
// index is known).  Operations are applied in list order.
template <class T> struct GatePass {
  int n, k, ld, ncols, n_ops;
  int local_q[8];      // local bit j <-> qubit local_q[j]
  int sorted_q[8];     // the same qubits in ascending order (row-index deposit)
  int op_type[kGateMaxOps];
  int op_a[kGateMaxOps];
  int op_b[kGateMaxOps];
  int op_coef[kGateMaxOps];
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
};

// ---------------------------------------------------------------- launchers (k_*.hip)
template <class T>
hipError_t launch_gate_pass(const GatePass<T>& p, cx_t<T>* L, hipStream_t s);

template <class T>
hipError_t launch_kraus_expand(cx_t<T>* L, int n, int ld, int c, int q, const Channel& ch,
                               int m_pad, hipStream_t s);

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

template <class T>
hipError_t launch_project(cx_t<T>* L, int n, int ld, int c_in, int nsplit, int q, int c_out,
                          const cx_t<T>* W, hipStream_t s);

template <class T>
hipError_t launch_probabilities(const cx_t<T>* L, int n, int ld, int ncols, double* p,
                                hipStream_t s);

template <class T>
hipError_t launch_zstats(const cx_t<T>* L, int n, int ld, int ncols, double* partials,
                         int nblocks, double* out, hipStream_t s);

template <class T>
hipError_t launch_pauli(const cx_t<T>* L, int n, int ld, int ncols, const uint64_t* xm,
                        const uint64_t* zm, int n_terms, double* partials, int nblocks,
                        double* out, hipStream_t s);

hipError_t launch_sample(const double* p, int n, double* cdf, double* block_sums,
                         const double* u, int count, uint64_t* out, hipStream_t s);

template <class T>
hipError_t launch_set_e0(cx_t<T>* L, hipStream_t s);

int gram_blocks(int n, int nsplit);   // number of split-K partials the Gram uses

}  // namespace lrdm
