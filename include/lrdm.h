/*
 * lrdm.h -- C ABI of the low-rank density-matrix (LRET) library for AMD MI355X (gfx950).
 *
 * The state of n qubits is rho = L L^H with L a 2^n x r complex factor (Eq. "low rank
 * decomposition", Sec. II.A).  Gates act column-wise on L (Eq. "low rank evolution G"), a Kraus
 * channel concatenates [E_1 L | ... | E_m L] (Eq. "low rank evolution K"), and a compression
 * returns to rank <= r through the Gram matrix G = L'^H L', its leading eigenpairs and the
 * projection L' V_k (Sec. II.B and Theorem 1 of App. B).  Outputs are Prob(x) and Tr(L^H O L)
 * (Sec. II.D).
 *
 * General conventions
 *  - Every call returns an lrdm_status and never throws.  On failure lrdm_last_error() holds a
 *    message; argument errors are detected before anything is enqueued and leave the handle
 *    unchanged.
 *  - The library never allocates device memory.  The caller owns the state and workspace
 *    buffers (sizes from lrdm_workspace_size) and every host array; host arrays are consumed
 *    before the call returns.  lrdm_destroy frees only the host-side handle.
 *  - Work is enqueued on the stream given to lrdm_init in call order.  Calls that return host
 *    values synchronise that stream.  Device outputs are valid after a stream synchronisation.
 *  - Layout of L in the state buffer: row-major, L[x * ld + v], x in [0, 2^n) with qubit q =
 *    bit q of x, v in [0, ld); complex values interleaved (re, im) as float pairs (LRDM_C64) or
 *    double pairs (LRDM_C128).  r_pad = the smallest power of two >= max(r_max, 8); ld = r_pad
 *    (fused form) or m_pad * r_pad (plain form, m_pad = the smallest power of two >= m_max);
 *    lrdm_layout returns both for a handle.  Unused columns are zero.
 *  - Gate and Kraus matrices are FP64, row-major, interleaved (re, im).
 *  - Asynchronous device errors (LRDM_E_HIP, LRDM_E_EIG) poison the handle: every later call
 *    returns LRDM_E_STATE until lrdm_destroy.
 */
#ifndef LRDM_H
#define LRDM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lrdm_ctx* lrdm_t;

typedef enum {
  LRDM_OK = 0,
  LRDM_E_ARG = 1,          /* invalid argument (range, null pointer, non-unitary, incomplete Kraus set) */
  LRDM_E_NOMEM = 2,        /* a caller-provided buffer is smaller than required */
  LRDM_E_HIP = 3,          /* the HIP runtime reported an error */
  LRDM_E_EIG = 4,          /* non-finite Gram matrix or eigensolver failure */
  LRDM_E_STATE = 5,        /* call not valid in the current state (poisoned handle, pending channel) */
  LRDM_E_UNSUPPORTED = 6   /* valid request outside the supported sizes */
} lrdm_status;

typedef enum { LRDM_C64 = 0, LRDM_C128 = 1 } lrdm_dtype;

/* lrdm_init flags */
#define LRDM_FLAG_PLAIN 0x1u   /* plain low-rank form: apply_kraus materialises [E_1 L | ... | E_m L]
                                  (Eq. "low rank evolution K") and compress diagonalises its full
                                  (m r) x (m r) Gram matrix; the default fuses both (see lrdm_compress) */
#define LRDM_FLAG_OVERLAP 0x2u /* fused form only: eigensolves run on a second stream that the handle
                                  creates (default priority), beside the projections and Gram passes on
                                  the caller's stream.  A channel on qubit q that follows a compression
                                  on qubit p != q takes its split Gram matrix from the 4-way Gram of the
                                  bit pair (p, q), formed before the projection on p, transformed by that
                                  projection's W in FP64 (S_bb' = sum_c W_c^H G4_bb' W_c; Sec. II.B, the
                                  Gram of the projected factor), so the eigensolve of q needs no pass
                                  over the projected factor and overlaps the projection on p.  Same
                                  method, different rounding order; every call keeps its contract
                                  (outputs wait for both streams). */

/* Per-compression record (Sec. II.B). */
typedef struct {
  int rank;                /* kept eigenpairs k */
  int n_eig;               /* order N of the Gram matrix that was diagonalised */
  double discarded;        /* Tr G - sum_{i<=k} max(lambda_i, 0) */
  double discarded_total;  /* running sum of `discarded` since lrdm_init / lrdm_set_L */
  double trace_before;     /* Tr G = Tr(rho') before truncation */
  double boundary_gap;     /* lambda_k - lambda_{k+1}; +inf when k == N */
  double lambda_max;       /* largest eigenvalue of G */
} lrdm_compress_info;

/* Required buffer sizes for a handle.  n in [1, 30]; r_max in [1, 64]; m_max in [1, 4] is the
 * largest Kraus count that will be applied; (m_max * r_pad) must not exceed 128 (the order of
 * the largest Gram matrix the eigensolver accepts) and, for LRDM_C128, r_pad must not exceed 32.
 * Returns LRDM_E_UNSUPPORTED outside these limits. */
lrdm_status lrdm_workspace_size(int n, int r_max, lrdm_dtype dt, int m_max, unsigned flags,
                                size_t* state_bytes, size_t* work_bytes);

/* Create a handle over caller-owned device buffers and set L = e_0 = |0...0> (Algorithm 1).
 * hip_stream is a hipStream_t (NULL = the null stream).  The buffers must stay alive and
 * untouched by the caller until lrdm_destroy. */
lrdm_status lrdm_init(lrdm_t* out, int n, int r_max, lrdm_dtype dt, int m_max, unsigned flags,
                      void* state_dev, size_t state_bytes, void* work_dev, size_t work_bytes,
                      void* hip_stream);

/* Shape of a handle: qubit count n, leading dimension ld of the state layout (complex entries
 * per row), the padded rank r_pad and the state buffer's size in bytes (any pointer may be NULL).
 * Never fails for a valid handle. */
lrdm_status lrdm_layout(lrdm_t h, int* n, int* ld, int* r_pad, size_t* state_bytes);

/* Reset an existing handle to L = e_0 (rank 1), clearing the running discarded mass. */
lrdm_status lrdm_reset(lrdm_t h);

lrdm_status lrdm_destroy(lrdm_t h);

/* Gate L <- G L (Eq. "low rank evolution G").  k in {1, 2}; qubits[0..k) distinct and < n;
 * u is 2^k x 2^k, row-major, interleaved re/im, with local index i = sum_j b(qubits[j]) 2^j.
 * Unitarity is checked in FP64 (max |U^H U - I| <= 1e-10, else LRDM_E_ARG).  Gates are queued
 * and applied in fused passes (several qubits per HBM sweep) at the next non-gate call. */
lrdm_status lrdm_apply_gate(lrdm_t h, int k, const int* qubits, const double* u);

/* Diagonal gate depending on Hamming weight: L[x, :] *= phase[popcount(x)], phase has n + 1
 * unit-modulus complex entries (interleaved).  Used for the Grover oracle of Sec. III.C and the
 * reflection about |0...0>. */
lrdm_status lrdm_apply_diagonal_weight(lrdm_t h, const double* phase);

/* Kraus channel on one qubit (Eq. "low rank evolution K"): e holds m 2x2 matrices
 * E_a = sqrt(p_a) K_a (row-major, interleaved), m in [1, m_max], sum_a E_a^H E_a = I within
 * 1e-10.  The concatenation is lazy: the next call must be lrdm_compress (else LRDM_E_STATE),
 * which consumes it without ever forming the 2^n x (m r) matrix.  In plain mode the
 * concatenation is materialised here. */
lrdm_status lrdm_apply_kraus(lrdm_t h, int qubit, int m, const double* e);

/* Eigenvalue truncation (Sec. II.B) through G = L'^H L' (Theorem 1), L <- c L' V_k.
 *  r_target in [1, r_max]: rank cap.  eps in [0, 1): keep the smallest k whose kept mass
 *  sum_{i<=k} max(lambda_i, 0) reaches (1 - eps) Tr G (eps = 0 disables the threshold).
 *  tie_policy: 0 = keep eigensolver order; 1 = lower k while lambda_k - lambda_{k+1} <=
 *  1e-6 Tr G so the kept set is gap-separated (the spectrum continues with zeros past the Gram
 *  order, so zero-eigenvalue columns are dropped too).  renorm: 1 = scale to unit trace
 *  (c = kept^{-1/2}), 0 = c = 1.  The Gram matrix is accumulated in the bulk precision (FP32
 *  MFMA for LRDM_C64) and diagonalised in FP64.  info may be NULL; if not, the call
 *  synchronises the stream and fills it. */
lrdm_status lrdm_compress(lrdm_t h, int r_target, double eps, int tie_policy, int renorm,
                          lrdm_compress_info* info);

/* Two-qubit Kraus channel (Sec. II.C: noise as one- and two-qubit Kraus operators; a group of
 * M = 2 qubits' channels as their product set {E_a (x) F_b}) on (q0, q1): e holds m 4 x 4
 * matrices (row-major, interleaved, local index b(q0) + 2 b(q1)), m in [1, m_max], completeness
 * within 1e-10; the next call must be lrdm_compress.  Plain form (LRDM_FLAG_PLAIN, m_max up to 16
 * with m_pad * r_pad <= 128): [E_1 L | ... | E_m L] is materialised here.  Fused form (m_max <= 4,
 * r_pad <= 32, else LRDM_E_UNSUPPORTED; not while recording a batch): nothing is materialised;
 * the compression forms the 4-way Gram of the pair, G = sum_{u u'} (E_a^H E_b)_{u u'} S4_{u u'}
 * and projects the 4-way view in place, W_{(u,v),(u',j)} = c sum_a (E_a)_{u'u} V[(a,v), j]. */
lrdm_status lrdm_apply_kraus2(lrdm_t h, int q0, int q1, int m, const double* e);

/* Sparse superposition initial state (Sec. II.D: Algorithm 1 also starts from any sparse linear
 * combination of basis states): L = sum_i amp[i] |idx[i]> as one column, count in [1, 32768],
 * distinct indices below 2^n, amp interleaved complex with unit norm within 1e-10 (else
 * LRDM_E_ARG).  Replaces the state like lrdm_set_L.  Synchronises. */
lrdm_status lrdm_set_sparse(lrdm_t h, int count, const uint64_t* idx, const double* amp);

/* Prob(x) = sum_v |L[x, v]|^2 (Sec. II.D) for all 2^n basis states into p_dev (2^n doubles,
 * device memory owned by the caller).  Asynchronous. */
lrdm_status lrdm_probabilities(lrdm_t h, double* p_dev);

/* Tr(L^H P_t L) (Sec. II.D) for n_terms Pauli strings P_t = i^{|x&z|} X^xmask[t] Z^zmask[t]
 * (Y where both bits are set).  summed = 0: out_host[t] = Tr(L^H P_t L) for every t (n_terms
 * doubles); summed = 1: out_host[0] = sum_t coeff[t] Tr(L^H P_t L).  coeff may be NULL when
 * summed = 0.  n_terms in [1, 65536].  Synchronises. */
lrdm_status lrdm_expect_pauli(lrdm_t h, int n_terms, const uint64_t* xmask, const uint64_t* zmask,
                              const double* coeff, int summed, double* out_host);

/* <Z_i> = sum_x Prob(x) (1 - 2 x_i) for every qubit into z_host (n doubles) and, if zz_host is
 * not NULL, <Z_i Z_{i+1}> for i in [0, n-1) (n - 1 doubles).  trace_host (nullable) receives
 * sum_x Prob(x).  One pass over L.  Synchronises. */
lrdm_status lrdm_expect_z(lrdm_t h, double* z_host, double* zz_host, double* trace_host);

/* Measurement samples from Prob (Sec. II.D): for each of `count` uniforms u_j in [0, 1)
 * (host array), out_host[j] = the smallest x with CDF(x) > u_j * CDF(2^n - 1), CDF being the
 * FP64 running sum of Prob.  count in [1, 2^24].  Synchronises. */
lrdm_status lrdm_sample(lrdm_t h, int count, const double* uniforms, uint64_t* out_host);

/* Copy L out (2^n x ld, the state layout; to_host = 1: dst is host memory, else device).
 * rank_out (nullable) receives the host-side bound on the number of non-zero columns.
 * Synchronises when to_host = 1. */
lrdm_status lrdm_get_L(lrdm_t h, void* dst, int to_host, int* rank_out);

/* Replace L by a caller factor with `rank` columns (row-major 2^n x rank in the bulk
 * precision, interleaved; from_host = 1: host memory, else device).  Columns beyond rank are
 * zeroed.  Used for tests and for resuming a run. */
lrdm_status lrdm_set_L(lrdm_t h, const void* src, int from_host, int rank);

/* Wait for all work queued on the handle's stream; reports asynchronous device errors. */
lrdm_status lrdm_synchronize(lrdm_t h);

/* Kernel timing for performance reports.  kernel_class: 0 = gate sweep, 1 = Gram pass over L,
 * 2 = Gram reduction, 3 = eigensolver (all stages), 4 = projection, 5 = the small FP64 products
 * of chained compressions (the second Gram matrix W^H S W and the composed W) and, with
 * LRDM_FLAG_OVERLAP, of the pair transform, 6 = the 4-way Gram of a bit pair (LRDM_FLAG_OVERLAP:
 * its two passes over L and their reduction).  Between lrdm_timing_begin and
 * lrdm_timing_end every launch of that class is bracketed by HIP events on the stream it runs
 * on (the gate passes of one flush, launched back to back, by one pair around them all);
 * lrdm_timing_end synchronises and returns the number of launches and their mean duration in
 * milliseconds.  At most 65536 event pairs are recorded. */
lrdm_status lrdm_timing_begin(lrdm_t h, int kernel_class);

/* Launch shapes the autotuner (paper_2009_06657_amd/autotune.py) chooses per workload; they
 * change where work-groups split the rows, never the operations, so results move only by
 * rounding order.  0 in a field keeps the default.
 *   gram_blocks:    split-K work-groups of a Gram pass over L, 1..256 (default: one per CU of
 *                   the stream, at most 256, fewer when L has fewer 64-row chunks)
 *   gram4_blocks:   work-groups of each pass of the 4-way Gram (LRDM_FLAG_OVERLAP), 2..256
 *                   (default: one per CU of its stream)
 *   gate_local_max: local qubits of a fused gate pass, 1..8 (default: as many as a 64 KB tile
 *                   holds)
 *   aux_cus:        LRDM_FLAG_OVERLAP: CUs of the eigensolver stream, a multiple of 32 (whole XCDs)
 *                   below the device's CU count (default 32)
 * lrdm_set_tuning orders the change after the work already queued; LRDM_E_ARG on a value out of
 * range (nothing changes then). */
typedef struct {
  int gram_blocks;
  int gram4_blocks;
  int gate_local_max;
  int aux_cus;
} lrdm_tuning;
lrdm_status lrdm_set_tuning(lrdm_t h, const lrdm_tuning* t);
lrdm_status lrdm_get_tuning(lrdm_t h, lrdm_tuning* t);   /* the values in use (defaults resolved) */
lrdm_status lrdm_timing_end(lrdm_t h, int* launches, double* mean_ms, double* total_ms);

/* ---------------------------------------------------------------- reverse sweep (gradients)
 * The paper defines the forward map only.  These calls give the exact derivative of an energy
 * E = sum_t c_t Tr(L^H P_t L) of the final factor (Sec. II.D) with respect to the angles of
 * rotation gates R_P(theta) = exp(-i theta P / 2), by one reverse sweep over the same operations.
 * The adjoint factor Lbar (dE = 2 Re Tr(Lbar^H dL)) lives in a second handle of the same n,
 * r_max, dtype, m_max and form (the "bar" handle).  The sweep needs the fused form and
 * m_max * r_pad <= 64 (every eigenpair of G is recorded); otherwise LRDM_E_UNSUPPORTED. */

/* Bytes of one compression record: the FP64 eigen-decomposition of G kept for the reverse sweep
 * (8 + N + 2 N^2 doubles, N = m_max * r_pad, rounded up to 256 bytes). */
lrdm_status lrdm_record_bytes(lrdm_t h, size_t* bytes);

/* lrdm_compress that also writes its record to rec_dev (device memory, lrdm_record_bytes bytes,
 * 256-byte aligned, owned by the caller): k, the scale c, Tr G, the renorm flag, every eigenvalue
 * of G (descending) and every eigenvector (N x N complex, column j = eigenvector j).  All N
 * eigenvectors are formed, so the call costs more than lrdm_compress; the kept factor is the
 * same.  A Kraus channel must be pending.  Queued; info as in lrdm_compress. */
lrdm_status lrdm_compress_record(lrdm_t h, int r_target, double eps, int tie_policy, int renorm,
                                 void* rec_dev, lrdm_compress_info* info);

/* Copy the whole state buffer (state_bytes of device memory owned by the caller) to dst_dev;
 * rank_out (nullable) receives the column bound.  Pending gates are applied first.  Queued. */
lrdm_status lrdm_checkpoint(lrdm_t h, void* dst_dev, int* rank_out);

/* Replace the state buffer by a copy made with lrdm_checkpoint on a handle of the same shape;
 * `rank` is the column bound it returned.  Pending gates are discarded.  Queued. */
lrdm_status lrdm_restore(lrdm_t h, const void* src_dev, int rank);

/* dst's factor <- H src's factor, H = sum_t coeff[t] P_t (Pauli strings as in
 * lrdm_expect_pauli), column by column: the reverse-sweep seed Lbar = H L of
 * E = Tr(L^H H L).  dst and src must be different handles of the same shape.  n_terms in
 * [1, 4096].  Synchronises dst's stream (and src's when the streams differ). */
lrdm_status lrdm_apply_pauli_sum(lrdm_t dst, lrdm_t src, int n_terms, const uint64_t* xmask,
                                 const uint64_t* zmask, const double* coeff);

/* out_host[2t], out_host[2t + 1] = Re, Im of Tr(bra^H P_t ket) for n_terms Pauli strings (as in
 * lrdm_expect_pauli; bra and ket are handles of the same shape).  With bra = Lbar and ket = L
 * taken right after a gate R_P(theta) on one qubit, dE/dtheta = Im Tr(Lbar^H P L).  n_terms in
 * [1, 65536].  Synchronises. */
lrdm_status lrdm_pauli_overlap(lrdm_t bra, lrdm_t ket, int n_terms, const uint64_t* xmask,
                               const uint64_t* zmask, double* out_host);

/* Reverse of one Kraus channel and the compression after it (Eq. "low rank evolution K",
 * Sec. II.B, Theorem 1).  On entry bar holds Lbar_n, the adjoint of the compressed factor
 * L_n = c L' V_K; x_dev is the forward factor before the channel (a lrdm_checkpoint copy of the
 * forward handle, state layout); rec_dev the record of that compression; (qubit, m, e) the
 * channel as given to lrdm_apply_kraus.  On return bar holds Lbar = sum_a E_a^H Lbar'_a with
 *   Lbar' = c Lbar_n V_K^H + L' (Ghat + Ghat^H) - s c^2 L' V_K V_K^H,
 *   Ghat = V_K Zhat^H V_D^H, Zhat_ji = [V_D^H (c L'^H Lbar_n)]_ji / (lambda_i - lambda_j),
 *   s = Re Tr(Lbar_n^H L_n) (the last term only when the record says renorm = 1),
 * the first-order change of the kept spectral projector of G and of c.  Pairs with
 * |lambda_i - lambda_j| <= 1e-13 Tr G (null space of L') are skipped.  The channel is not
 * materialised: C = X^H Ybar on the split view, the small matrices in FP64, then
 * [Lbar_0 | Lbar_1] = Ybar P + X Q in place.  Queued. */
lrdm_status lrdm_compress_adjoint(lrdm_t bar, const void* x_dev, const void* rec_dev, int qubit,
                                  int m, const double* e);

/* ---------------------------------------------------------------- programs (Algorithm 1)
 * A program is a flat array of operations applied in order, the loop of Algorithm 1: gates and
 * Hamming-weight phases, Kraus channels each followed by its compression (Sec. II.C, one channel
 * per group), and layer marks.  Matrices live in one FP64 coefficient array (interleaved re/im,
 * layouts as in the operation-level calls); an operation names its first coefficient by `off`. */
typedef enum {
  LRDM_OP_GATE = 0,      /* k-qubit gate (k in {1, 2}) on q0 (, q1), 2^k x 2^k matrix at coef + off */
  LRDM_OP_ROTATION = 1,  /* R_P(theta) = exp(-i theta P / 2) on q0, P = X, Y, Z for axis 1, 2, 3; the
                            matrix is computed from theta = params[param] when params is given, else
                            read at coef + off; param also names the gradient entry (lrdm_energy_grad) */
  LRDM_OP_WEIGHT = 2,    /* L[x, :] *= phase[popcount(x)], n + 1 complex at coef + off */
  LRDM_OP_KRAUS = 3,     /* channel on q0 with m = k operators E_a at coef + off (as lrdm_apply_kraus);
                            the next operation must be LRDM_OP_COMPRESS */
  LRDM_OP_COMPRESS = 4,  /* lrdm_compress(r, eps, tie, renorm) */
  LRDM_OP_LAYER = 5,     /* end of a layer (checkpoint boundary); no arithmetic */
  LRDM_OP_KRAUS2 = 6     /* two-qubit channel on (q0, q1) with m = k operators (4 x 4) at coef + off
                            (as lrdm_apply_kraus2); the next operation must be LRDM_OP_COMPRESS */
} lrdm_op_kind;

typedef struct {
  int kind;              /* lrdm_op_kind */
  int k;                 /* gate: qubit count; channel: operator count */
  int q0, q1;            /* qubits (q1 only for two-qubit gates) */
  int axis;              /* rotation: 1 = X, 2 = Y, 3 = Z */
  int param;             /* rotation: index into params / the gradient */
  int r, tie, renorm;    /* compression */
  double eps;            /* compression */
  int64_t off;           /* first coefficient (doubles) of the operation's matrix */
} lrdm_op;

typedef struct {
  int n_ops;
  const lrdm_op* ops;
  const double* coef;    /* host array of n_coef doubles */
  int64_t n_coef;
} lrdm_program;

/* Host-only check of a program for n qubits: every rule lrdm_run applies before it enqueues
 * anything (operation kinds, qubit ranges, coefficient ranges, rotation axes and parameter
 * indices, a compression after every channel, unitarity, Kraus completeness, unit-modulus
 * phases).  Returns LRDM_OK or LRDM_E_ARG with the offending operation in lrdm_last_error(NULL). */
lrdm_status lrdm_program_validate(const lrdm_program* p, int n, const double* params, int n_params);

/* Algorithm 1 over a program, from the handle's current state (call lrdm_reset first for L =
 * e_0): every operation is issued in order through the operation-level calls.  The whole program
 * is validated first (ranges, unitarity, completeness, phase modulus, a compression after every
 * channel); on LRDM_E_ARG nothing is enqueued.  params (nullable, n_params doubles) gives the
 * rotation angles.  With ckpt_dev (device memory, 256-byte aligned) the state at the start of
 * every layer l goes to ckpt_dev + l * S, S = state bytes rounded up to 256 (ckpt_bytes >=
 * layers * S, else LRDM_E_NOMEM); ckpt_rank (nullable host array, one int per layer) receives
 * the column bound to pass to lrdm_restore.  A trailing run of operations without a layer mark
 * counts as a layer.  Queued (no synchronisation). */
lrdm_status lrdm_run(lrdm_t h, const lrdm_program* p, const double* params, int n_params, void* ckpt_dev,
                     size_t ckpt_bytes, int* ckpt_rank);

/* Device bytes lrdm_energy_grad needs for program p on handle h: keep_all_bytes keeps every
 * channel's input factor and compression record from the forward pass (the reverse sweep re-runs
 * nothing); min_bytes keeps the layer checkpoints and one layer's inputs and records (the reverse
 * sweep re-runs each layer once, bit for bit).  Fails like lrdm_energy_grad's validation. */
lrdm_status lrdm_energy_grad_bytes(lrdm_t h, const lrdm_program* p, size_t* keep_all_bytes, size_t* min_bytes);

/* Energy E = sum_t coeff[t] Tr(L^H P_t L) of the final factor of program p run from L = e_0
 * (Sec. II.D; Pauli strings as in lrdm_expect_pauli, n_terms in [1, 4096]) and its gradient with
 * respect to the rotation angles, by one forward pass and one reverse sweep (the adjoint of
 * gates, channels and truncations described at lrdm_compress_adjoint; a rotation R_P(theta)
 * contributes dE/dtheta = Im Tr(Lbar^H P L) right after it, rotations whose generators commute
 * with everything between them being evaluated together).  h is reset and ends in the state the
 * last layer's reverse step leaves; bar is a second handle of the same shape that receives the
 * adjoint factor.  Every compression must follow a channel (else LRDM_E_UNSUPPORTED), and the
 * reverse sweep's size limits apply (m_max * r_pad <= 64, fused form).  grad_host: n_params
 * doubles, overwritten; energy: one double.  store_dev: device memory of store_bytes >= min_bytes
 * of lrdm_energy_grad_bytes (256-byte aligned); with keep_all_bytes or more nothing is re-run,
 * and kept_all (nullable) reports which mode ran.  Synchronises. */
lrdm_status lrdm_energy_grad(lrdm_t h, lrdm_t bar, const lrdm_program* p, const double* params, int n_params,
                             int n_terms, const uint64_t* xmask, const uint64_t* zmask, const double* coeff,
                             double* energy, double* grad_host, void* store_dev, size_t store_bytes,
                             int* kept_all);

/* ---------------------------------------------------------------- full-rank comparator
 * Exact density-matrix evolution (Eq. "full rank evolution", Sec. II.A) in complex64, the
 * same-GPU baseline the low-rank path is measured against.  rho (2^n x 2^n, row-major, 8 * 4^n
 * bytes of caller-owned device memory) is treated as a vector over 2n index bits (column bit q =
 * index bit q, row bit q = index bit n + q): a gate U applies U to the row bits and conj(U) to the
 * column bits, a channel applies sum_a E_a (x) conj(E_a) to the bit pair (n + q, q).  Operations
 * are queued and applied in fused passes over LDS tiles of 2^13 amplitudes.  n in [1, 16]. */
typedef struct lrdm_fdm_ctx* lrdm_fdm_t;

/* Bytes of rho for n qubits (8 * 4^n). */
lrdm_status lrdm_fdm_state_bytes(int n, size_t* bytes);
/* rho = |0...0><0...0| in state_dev (256-byte aligned); work goes on hip_stream. */
lrdm_status lrdm_fdm_init(lrdm_fdm_t* out, int n, void* state_dev, size_t state_bytes, void* hip_stream);
lrdm_status lrdm_fdm_reset(lrdm_fdm_t h);
lrdm_status lrdm_fdm_destroy(lrdm_fdm_t h);
/* rho <- U rho U^H; arguments as lrdm_apply_gate. */
lrdm_status lrdm_fdm_apply_gate(lrdm_fdm_t h, int k, const int* qubits, const double* u);
/* rho <- sum_a E_a rho E_a^H on one qubit; arguments as lrdm_apply_kraus (m in [1, 4]). */
lrdm_status lrdm_fdm_apply_kraus(lrdm_fdm_t h, int qubit, int m, const double* e);
/* rho[x][y] <- phase[popcount(x)] conj(phase[popcount(y)]) rho[x][y]: the Hamming-weight
 * diagonal gate of lrdm_apply_diagonal_weight (Grover oracle and reflection, Sec. III.C) on the
 * full-rank state; phase has n + 1 unit-modulus complex entries (interleaved FP64, checked within
 * 1e-10, else LRDM_E_ARG).  Queued operations are applied first; this one runs at once as its
 * own pass over rho.  Queued on the stream. */
lrdm_status lrdm_fdm_apply_diagonal_weight(lrdm_fdm_t h, const double* phase);
/* rho = L L^H (Eq. "low rank decomposition") into the full-rank handle f (same n, n <= 16),
 * replacing its state and dropping its queued operations; L is h's factor after its pending
 * work.  The switch to full density matrix evolution of Sec. II.C.  Orders the two handles'
 * streams. */
lrdm_status lrdm_to_full(lrdm_t h, lrdm_fdm_t f);

/* Algorithm 1 with the switch of Sec. II.C: the program runs on h (from its current state) until
 * a channel group whose intermediate rank V_I, V_I^3 = N (A V)^3 / M (A operators on M qubits, V
 * the rank kept by the last compression, 1 before any), reaches 2^N; there the state goes to f
 * (lrdm_to_full) and the remaining gates, phases and one-qubit channels run as full density
 * matrix evolution on f (compressions no longer apply).  *switched_at = the index of that channel
 * operation, or -1 (the result is then h's factor).  f may be NULL when n > 16 (V_I cannot reach
 * 2^N there); programs with two-qubit channels after a possible switch are not supported
 * (LRDM_E_UNSUPPORTED before anything runs).  Every compression synchronises (its kept rank
 * decides the rule). */
lrdm_status lrdm_run_switching(lrdm_t h, lrdm_fdm_t f, const lrdm_program* p, const double* params, int n_params,
                               int* switched_at);

/* Prob(x) = Re rho[x][x] into p_dev (2^n doubles, device).  Applies queued operations. */
lrdm_status lrdm_fdm_probabilities(lrdm_fdm_t h, double* p_dev);
/* Apply queued operations and wait for the stream. */
lrdm_status lrdm_fdm_synchronize(lrdm_fdm_t h);
/* Last error message of h ("" for NULL; lrdm_last_error(NULL) also holds it). */
const char* lrdm_fdm_last_error(lrdm_fdm_t h);

/* ---------------------------------------------------------------- batched serving
 * Many independent handles (complex64, fused form; any mix of n, r_max and m_max) run together.
 * Between lrdm_batch_begin and lrdm_batch_end, lrdm_reset / lrdm_apply_gate /
 * lrdm_apply_diagonal_weight / lrdm_apply_kraus / lrdm_compress on those handles are validated
 * and recorded instead of executed (calls that need results return LRDM_E_STATE).  The recorded
 * programs are then scheduled in lockstep: step s of every instance (its gate passes and its s-th
 * compression) is issued as one batched launch per kernel kind and size class, so e.g. the s-th
 * eigensolves of all instances run concurrently, one work-group each.  The whole schedule is
 * captured in one hipGraph; lrdm_batch_launch replays it.  Per-step device timestamps give
 * each instance's completion time.  The caller owns the plan buffer (job tables + timestamps). */
typedef struct lrdm_batch_ctx* lrdm_batch_t;

/* handles: n_inst distinct handles.  The graph is captured and replayed on hip_stream, which must
 * not be the default (null) stream; NULL asks the library for a stream of its own (default
 * priority).  A replay waits for work queued before it on the handles' streams, and work queued
 * there afterwards waits for the replay. */
lrdm_status lrdm_batch_create(lrdm_batch_t* out, int n_inst, const lrdm_t* handles, void* hip_stream);
/* Apply pending gates, wait for each handle's stream, start recording. */
lrdm_status lrdm_batch_begin(lrdm_batch_t b);
/* Stop recording, build the lockstep schedule; *plan_bytes = device bytes it needs. */
lrdm_status lrdm_batch_end(lrdm_batch_t b, size_t* plan_bytes);
/* Upload the schedule to plan_dev (256-byte aligned, >= plan_bytes, owned by the caller and
 * kept until lrdm_batch_destroy) and capture the hipGraph.  Synchronous. */
lrdm_status lrdm_batch_instantiate(lrdm_batch_t b, void* plan_dev, size_t plan_bytes);
/* Replay the graph on the batch stream (asynchronous).  Every instance starts from its
 * recorded reset, so replays give identical results. */
lrdm_status lrdm_batch_launch(lrdm_batch_t b);
/* Number of lockstep steps and of captured launches. */
lrdm_status lrdm_batch_info(lrdm_batch_t b, int* n_steps, int* n_launches);
/* Wait for the last launch; done_ms[i] (nullable, n_inst doubles) = time from the start of the
 * replay to the end of instance i's last step; total_ms (nullable) = whole replay.  Device wall
 * clock. */
lrdm_status lrdm_batch_times(lrdm_batch_t b, double* done_ms, double* total_ms);
lrdm_status lrdm_batch_destroy(lrdm_batch_t b);

/* One call for a whole batch: handle i of b (creation order) is reset and runs program progs[i]
 * (params[i] / n_params[i] as in lrdm_run; params and n_params may be NULL), recorded as by
 * lrdm_batch_begin / lrdm_batch_end; *plan_needed receives the plan's device bytes.  If plan_dev
 * is NULL or plan_bytes is smaller, the call returns LRDM_E_NOMEM after setting *plan_needed
 * (call again with a buffer of that size); otherwise it instantiates the graph on plan_dev,
 * replays it once and waits, filling done_ms / total_ms as lrdm_batch_times (both nullable).
 * Later replays: lrdm_batch_launch. */
lrdm_status lrdm_batch_run(lrdm_batch_t b, const lrdm_program* const* progs, const double* const* params,
                           const int* n_params, void* plan_dev, size_t plan_bytes, size_t* plan_needed,
                           double* done_ms, double* total_ms);

/* ---------------------------------------------------------------- allocation-free outputs
 * For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): <Z_i>, <Z_i Z_{i+1}> and the trace of a factor the
 * caller holds, with no handle and no workspace.  L_dev: the factor in the state layout
 * (row-major 2^n x ld, complex64 or complex128 by dt; columns >= ncols are ignored), device
 * memory owned by the caller.  Outputs as lrdm_expect_z (z_host: n doubles; zz_host: n - 1
 * doubles, nullable; trace_host nullable).  The kernels' scratch (Prob(x) and the reduction's
 * partial sums) is a device array inside the library, 8.3 MiB per GPU, held until the process
 * ends; it limits n to 20 (larger n: LRDM_E_UNSUPPORTED).  No call allocates or frees device
 * memory.  Every call on a GPU uses that GPU's one array: calls that overlap on one GPU (several
 * threads or streams at once) race.  Synchronises hip_stream. */
lrdm_status lrdm_expect_z_noalloc(const void* L_dev, int n, int ld, int ncols, lrdm_dtype dt, void* hip_stream,
                                  double* z_host, double* zz_host, double* trace_host);

/* Last error message for h, or the calling thread's last error when h == NULL. */
const char* lrdm_last_error(lrdm_t h);

/* Library version string. */
const char* lrdm_version(void);

#ifdef __cplusplus
}
#endif
#endif /* LRDM_H */
