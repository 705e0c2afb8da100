// FP64 eigensolver of the small Gram matrix G (order N <= 128) and the truncation rule
// (Sec. II.B; Theorem 1, App. B) on the serial path between the Gram and projection GEMMs: one
// work-group for steps 1-2 (and the scaling of T), one work-group per wave for step 3, one
// work-group for steps 4-5, and a short multi-work-group back-transform (step 6).
//
//  1. Assemble G from S = X^H X and the Kraus set, G_{(a,v),(b,w)} = sum_{uv'} (E_a^H E_b)_{uv'}
//     S_{(u,v),(v',w)} (split view) or G = S (plain view).  G lives in registers: half-wave R
//     holds rows R + NH a (a < BR, NH half-waves) and lane Cc of it columns BC Cc .. BC Cc + BC - 1
//     (N <= 32 BC), so each row is spread over one half-wave.
//  2. Householder reduction to a real symmetric tridiagonal T = Q^H G Q with reflectors
//     H_j = I - tau_j v_j v_j^H, v_j(j+1) = 1.  Every half-wave forms the reflector from the
//     broadcast column, the matrix-vector product reduces across a half-wave with lane swaps and
//     DPP moves, and the rank-2 update is register arithmetic on the rows not yet eliminated:
//     two barriers per step.  At order 128 the last 64 steps run on the trailing block moved to
//     a layout with a quarter of the registers per thread.
//  3. The wanted (largest) eigenvalues of T by multisection on Sturm counts (a wave per
//     eigenvalue, each wave a work-group of its own; recorded solves use 8 or 16 lanes).
//  4. Eigenvectors of T by inverse iteration on the LDL^T factorisation of T - lambda I (one
//     lane per eigenvector, factors and vectors in LDS).  Eigenvalues closer than
//     max(1e-9 ||T||, 1e-3 lambda) form clusters whose vectors are re-orthonormalised (modified
//     Gram-Schmidt, descending order) after every iteration, so (near-)degenerate eigenvalues
//     yield an orthonormal basis.
//  5. The rank rule (cap r, threshold eps, tie policy), discarded mass and renormalisation
//     scale.  The reflectors, their scalars and the kept eigenvectors of T go to the workspace.
//  6. A second kernel over 16 work-groups (one wave per kept eigenvector) back-transforms
//     V = Q Y and writes the projection matrix in the bulk precision:
//     W_{(b,v),(b',j)} = c sum_a (E_a)_{b'b} V[(a,v), j] (split view) or W = c V_k (plain).
#include <math.h>

#include <utility>

#include "lrdm_internal.h"

namespace lrdm {

struct z64 {
  double x, y;
};
__device__ __forceinline__ z64 zmk(double a, double b) { return z64{a, b}; }
__device__ __forceinline__ z64 zadd(z64 a, z64 b) { return z64{a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ z64 zsub(z64 a, z64 b) { return z64{a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ z64 zmul(z64 a, z64 b) { return z64{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ __forceinline__ z64 zconj(z64 a) { return z64{a.x, -a.y}; }
__device__ __forceinline__ z64 zcmul(z64 a, z64 b) {  // conj(a) * b
  return z64{a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ z64 zscale(z64 a, double s) { return z64{a.x * s, a.y * s}; }

// Lane-group sums.  Inside a row of 16 lanes the exchanges are DPP moves (quad_perm xor 1,
// quad_perm xor 2, row_half_mirror, row_mirror: after the first two steps every lane of a quad
// holds the quad sum, so the mirrors add the other quad / half-row); the 16- and 32-lane
// exchanges use ds_bpermute.  Every lane of the group ends with the identical value.
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
// value of v in lane l (uniform)
__device__ __forceinline__ double read_lane(double v, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                          __builtin_amdgcn_readlane(__double2loint(v), l));
}

// v + v(lane ^ 16) and v + v(lane ^ 32) by the lane-swap moves (permlane16/32_swap): the two
// results of a swap of v with itself are v and its partner, in an order that depends on the lane.
__device__ __forceinline__ double xor16_sum(double v) {
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)__double2loint(v), (unsigned)__double2loint(v), false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)__double2hiint(v), (unsigned)__double2hiint(v), false, false);
  return __hiloint2double((int)hi[0], (int)lo[0]) + __hiloint2double((int)hi[1], (int)lo[1]);
}
__device__ __forceinline__ double xor32_sum(double v) {
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)__double2loint(v), (unsigned)__double2loint(v), false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)__double2hiint(v), (unsigned)__double2hiint(v), false, false);
  return __hiloint2double((int)hi[0], (int)lo[0]) + __hiloint2double((int)hi[1], (int)lo[1]);
}
template <int W>
__device__ __forceinline__ double gsum(double v) {
  if constexpr (W >= 2) v += dpp_mov<0xB1>(v);    // quad_perm [1,0,3,2]
  if constexpr (W >= 4) v += dpp_mov<0x4E>(v);    // quad_perm [2,3,0,1]
  if constexpr (W >= 8) v += dpp_mov<0x141>(v);   // row_half_mirror
  if constexpr (W >= 16) v += dpp_mov<0x140>(v);  // row_mirror
  if constexpr (W >= 32) v = xor16_sum(v);
  if constexpr (W >= 64) v = xor32_sum(v);
  return v;
}

// Sums of a and of b over the 64 lanes of a wave, returned in every lane.  Transposing: the
// 32-lane swap leaves lanes 0-31 with pair sums of a and lanes 32-63 with pair sums of b, the
// half-waves reduce those by DPP and the 16-lane swap, and the totals are read from lanes 0 and 32.
__device__ __forceinline__ void wsum64x2(double& a, double& b) {
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)__double2loint(a), (unsigned)__double2loint(b), false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)__double2hiint(a), (unsigned)__double2hiint(b), false, false);
  double v = __hiloint2double((int)hi[0], (int)lo[0]) + __hiloint2double((int)hi[1], (int)lo[1]);
  v = gsum<32>(v);
  a = read_lane(v, 0);
  b = read_lane(v, 32);
}

__device__ __forceinline__ double hash_unit(uint32_t a, uint32_t b) {
  uint32_t h = a * 0x9E3779B1u ^ (b + 0x7F4A7C15u) * 0x85EBCA77u;
  h ^= h >> 15;
  h *= 0x2C1B3C6Du;
  h ^= h >> 12;
  h *= 0x297A2D39u;
  h ^= h >> 15;
  return ((double)(h >> 8) + 0.5) * (1.0 / 16777216.0) - 0.5;  // (-0.5, 0.5)
}

// offset of reflector j's entries i >= j + 2 in packed storage
__device__ __forceinline__ int refl_off(int j, int N) { return j * (N - 2) - (j * (j - 1)) / 2; }

// 1 / q through the hardware reciprocal refined by two Newton steps
__device__ __forceinline__ double rcp_nr(double q) {
  double r = __builtin_amdgcn_rcp(q);
  r = fma(r, fma(-q, r, 1.0), r);
  return fma(r, fma(-q, r, 1.0), r);
}

// One step of the pivot recurrence q_i = (d_i - x) - e_{i-1}^2 / q_{i-1}: the reciprocal of q
// from the hardware estimate refined by one Newton step (a few ulp; the count needs only the
// sign pattern), fused into the update; pivots at or below pivmin count as negative and are
// replaced by -pivmin.
__device__ __forceinline__ void sturm_step(double& q, int& cnt, double dx, double f, double pivmin) {
  const double r0 = __builtin_amdgcn_rcp(q);
  const double r = fma(r0, fma(-q, r0, 1.0), r0);
  q = fma(-f, r, dx);
  if (q <= pivmin) {
    ++cnt;
    q = fmin(q, -pivmin);
  }
}

// number of eigenvalues of T (scaled, diagonal d, squared off-diagonal e2) below x
__device__ __forceinline__ int sturm_count(const double* d, const double* e2, int N, double x,
                                           double pivmin) {
  double q = d[0] - x;
  int cnt = 0;
  if (q <= pivmin) {
    ++cnt;
    q = fmin(q, -pivmin);
  }
  int i = 1;
  for (; i + 3 < N; i += 4) {
    double dd[4], ff[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      dd[u] = d[i + u] - x;
      ff[u] = e2[i + u - 1];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) sturm_step(q, cnt, dd[u], ff[u], pivmin);
  }
  for (; i < N; ++i) sturm_step(q, cnt, d[i] - x, e2[i - 1], pivmin);
  return cnt;
}

template <class F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// LDS operands of the tridiagonalisation steps.  The per-step vectors are double-buffered by
// step parity (buffer p at offset p * ld), so one barrier per step orders the writes of step
// j + 1's operands after every read of step j's.
struct TriSmem {
  z64* col_buf;   // column 0 of the (trailing) matrix, for the first reflector of a stage
  z64* vbuf;      // reflector v (local index)
  z64* pbuf;      // s = A v (local index)
  z64* cola;      // column jl + 1 of the matrix before update jl (local index)
  int ld;         // stride between the two parities
  double* d_s;    // diagonal of T (global index)
  double* e_s;    // off-diagonal of T (global index)
  double* tau_s;  // reflector scalars (global index, interleaved)
  z64* Rf;        // packed reflector entries i >= j + 2 (global packing)
  double tiny2;   // squared column norm below which a column counts as already reduced
};

// Transposing exchange across lane ^ 16: lanes with bit 4 clear get a + a(lane ^ 16), lanes
// with bit 4 set get b + b(lane ^ 16) (one 16-lane swap of a with b).
__device__ __forceinline__ double xor16_keep(double a, double b) {
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)__double2loint(a), (unsigned)__double2loint(b), false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)__double2hiint(a), (unsigned)__double2hiint(b), false, false);
  return __hiloint2double((int)hi[0], (int)lo[0]) + __hiloint2double((int)hi[1], (int)lo[1]);
}

// Half-wave sums of NV (8 or 16) values by a transposing reduction: each stage halves the
// values a lane keeps and adds its partner's copy of them (lane ^ 16 by the lane swap, then
// row_mirror, row_half_mirror and quad xor 2 pair lanes differing in bits 3, 2, 1); the lanes
// left with one value add the remaining partners.  Lane Cc ends with the total of value
// Cc >> (5 - log2 NV).
template <int NV>
__device__ __forceinline__ double tsum_halfwave(double (&v)[NV], int Cc) {
  static_assert(NV == 8 || NV == 16, "8 or 16 values");
  constexpr int H = NV / 2;
  double w8[H];
#pragma unroll
  for (int q = 0; q < H; ++q) w8[q] = xor16_keep(v[q], v[q + H]);
  const bool f3 = (Cc >> 3) & 1, f2 = (Cc >> 2) & 1, f1 = (Cc >> 1) & 1;
  double w4[H / 2];
#pragma unroll
  for (int q = 0; q < H / 2; ++q) {
    const double snd = f3 ? w8[q] : w8[q + H / 2];
    const double kp = f3 ? w8[q + H / 2] : w8[q];
    w4[q] = kp + dpp_mov<0x140>(snd);   // row_mirror
  }
  double w2[H / 4 > 0 ? H / 4 : 1];
  if constexpr (H / 4 >= 1) {
#pragma unroll
    for (int q = 0; q < H / 4; ++q) {
      const double snd = f2 ? w4[q] : w4[q + H / 4];
      const double kp = f2 ? w4[q + H / 4] : w4[q];
      w2[q] = kp + dpp_mov<0x141>(snd);   // row_half_mirror
    }
  }
  double r;
  if constexpr (NV == 16) {
    const double snd = f1 ? w2[0] : w2[1];
    const double kp = f1 ? w2[1] : w2[0];
    r = kp + dpp_mov<0x4E>(snd);   // quad_perm xor 2
  } else {
    r = w2[0];
    r += dpp_mov<0x4E>(r);
  }
  r += dpp_mov<0xB1>(r);   // quad_perm xor 1
  return r;
}

// Householder tridiagonalisation on the register-resident trailing matrix A: layout <BR, BC>
// (thread (R, Cc) holds rows R + NH a, NH = 32 BC / BR, and columns BC Cc + b), local order
// Nl, local step jl, global step j0 + jl.  Every half-wave forms each reflector redundantly
// (lane Cc owns entries BC Cc + b); rows in the eliminated part (rows <= jl) skip their
// arithmetic, and with the rows of a half-wave spread over the whole matrix that work shrinks
// evenly on every SIMD.

// Reflector of local step jl from the column entries cv[b] = A(BC Cc + b, jl), alpha =
// A(jl + 1, jl) and diag = Re A(jl, jl): H = I - tau v v^H with v(jl + 1) = 1 maps the column
// below the diagonal to (beta, 0, ..., 0).  Publishes v (parity par), the packed entries, d_j,
// e_j = beta and tau_j; returns this lane's entries of v and tau.
template <int BC>
__device__ __forceinline__ void tri_reflector(const z64 (&cv)[BC], const z64 alpha, const double diag, const int jl,
                                              const int Nl, const int j, const int N, const TriSmem& M,
                                              const int par, z64 (&vloc)[BC], z64& tau) {
  const int tid = threadIdx.x, Cc = tid & 31;
  double xn2 = 0;
#pragma unroll
  for (int b = 0; b < BC; ++b) {
    const int i = BC * Cc + b;
    if (i > jl + 1 && i < Nl) xn2 += cv[b].x * cv[b].x + cv[b].y * cv[b].y;
  }
  xn2 = gsum<32>(xn2);
  double beta = alpha.x;
  tau = zmk(0, 0);
  z64 sc = zmk(0, 0);
  // A column whose squared norm is at most tiny2 = max((1e-30 Tr G)^2, 1e-290) is taken as
  // reduced: its entries below the subdiagonal and the imaginary part of alpha are
  // dropped, a perturbation far below rounding.  Such columns hold only cancellation residue
  // (e.g. a qubit in an exact basis state); unscaled, their squared norm leaves the FP64 normal
  // range and the reciprocal square root below overflows.
  const double n2 = fma(alpha.x, alpha.x, fma(alpha.y, alpha.y, xn2));
  if (!(xn2 == 0.0 && alpha.y == 0.0) && n2 > M.tiny2) {
    // 1 / ||x|| from the hardware reciprocal square root refined by two Newton steps, and
    // 1 / |alpha - beta|^2 by the refined reciprocal (short dependency chains; a few ulp)
    double rn = __builtin_amdgcn_rsq(n2);
    rn = rn * fma(-0.5 * n2, rn * rn, 1.5);
    rn = rn * fma(-0.5 * n2, rn * rn, 1.5);
    const double nrm = n2 * rn;
    const bool pos = alpha.x >= 0;
    beta = pos ? -nrm : nrm;
    const double ib = pos ? -rn : rn;
    tau = zmk((beta - alpha.x) * ib, -alpha.y * ib);
    const double dr = alpha.x - beta, di = alpha.y;
    const double iden = rcp_nr(fma(dr, dr, di * di));
    sc = zmk(dr * iden, -di * iden);
  }
#pragma unroll
  for (int b = 0; b < BC; ++b) {
    const int i = BC * Cc + b;
    vloc[b] = (i == jl + 1) ? zmk(1, 0) : ((i > jl + 1 && i < Nl) ? zmul(sc, cv[b]) : zmk(0, 0));
  }
  if (tid < 32) {
#pragma unroll
    for (int b = 0; b < BC; ++b) {
      const int i = BC * Cc + b;
      M.vbuf[par * M.ld + i] = vloc[b];
      if (i >= jl + 2 && i < Nl) M.Rf[refl_off(j, N) + (i - jl - 2)] = vloc[b];
    }
    if (tid == 0) {
      M.d_s[j] = diag;
      M.e_s[j] = beta;
      M.tau_s[2 * j] = tau.x;
      M.tau_s[2 * j + 1] = tau.y;
    }
  }
}

// s = A v for this thread's rows, reduced over the half-wave, into pbuf (parity par); rows in
// the eliminated part publish zeros.
template <int BR, int BC>
__device__ __forceinline__ void tri_matvec(const z64 (&A)[BR][BC], const z64 (&vloc)[BC], const int jl, const int Nl,
                                           const TriSmem& M, const int par) {
  const int tid = threadIdx.x, R = tid >> 5, Cc = tid & 31;
  constexpr int NH = 32 * BC / BR;
  z64* pb = M.pbuf + par * M.ld;
  bool lv[BR];
#pragma unroll
  for (int a = 0; a < BR; ++a) lv[a] = R + NH * a > jl;   // uniform over the half-wave
  if (lv[BR - 1]) {
    if constexpr (BR == 8 || BR == 4) {
      constexpr int NV = 2 * BR;
      double vv[NV];
#pragma unroll
      for (int a = 0; a < BR; ++a) {
        // s_a = sum_b A[a][b] v_b as one FMA chain per component
        double sx = 0.0, sy = 0.0;
        if (lv[a]) {
          sx = A[a][0].x * vloc[0].x;
          sy = A[a][0].x * vloc[0].y;
          sx = fma(-A[a][0].y, vloc[0].y, sx);
          sy = fma(A[a][0].y, vloc[0].x, sy);
#pragma unroll
          for (int b = 1; b < BC; ++b) {
            sx = fma(A[a][b].x, vloc[b].x, sx);
            sy = fma(A[a][b].x, vloc[b].y, sy);
            sx = fma(-A[a][b].y, vloc[b].y, sx);
            sy = fma(A[a][b].y, vloc[b].x, sy);
          }
        }
        vv[2 * a] = sx;
        vv[2 * a + 1] = sy;
      }
      const double r = tsum_halfwave<NV>(vv, Cc);
      constexpr int SH = (NV == 16) ? 1 : 2;   // lane Cc holds value Cc >> SH
      if ((Cc & ((1 << SH) - 1)) == 0) {
        const int val = Cc >> SH;
        const int i = R + NH * (val >> 1);
        reinterpret_cast<double*>(pb)[2 * i + (val & 1)] = (i > jl && i < Nl) ? r : 0.0;
      }
    } else {
#pragma unroll
      for (int a = 0; a < BR; ++a) {
        z64 s = zmk(0, 0);
#pragma unroll
        for (int b = 0; b < BC; ++b) s = zadd(s, zmul(A[a][b], vloc[b]));
        s.x = gsum<32>(s.x);
        s.y = gsum<32>(s.y);
        const int i = R + NH * a;
        if (Cc == 0) pb[i] = (i > jl && i < Nl) ? s : zmk(0, 0);
      }
    }
  } else if (Cc == 0) {
#pragma unroll
    for (int a = 0; a < BR; ++a) pb[R + NH * a] = zmk(0, 0);
  }
}

// First reflector of a stage (local step 0) from the column in col_buf, its s = A v, and the
// next column before the update; one barrier.
template <int BR, int BC>
__device__ __forceinline__ void tri_prologue(const z64 (&A)[BR][BC], const int Nl, const int j0, const int N,
                                             const TriSmem& M, z64 (&vloc)[BC], z64& tau) {
  const int tid = threadIdx.x, R = tid >> 5, Cc = tid & 31;
  constexpr int NH = 32 * BC / BR;
  z64 cv[BC];
#pragma unroll
  for (int b = 0; b < BC; ++b) cv[b] = M.col_buf[BC * Cc + b];
  tri_reflector<BC>(cv, M.col_buf[1], M.col_buf[0].x, 0, Nl, j0, N, M, 0, vloc, tau);
  tri_matvec<BR, BC>(A, vloc, 0, Nl, M, 0);
  if (Cc == 1 / BC) {
#pragma unroll
    for (int a = 0; a < BR; ++a) M.cola[R + NH * a] = A[a][1 % BC];
  }
  __syncthreads();
}

// Local step jl (jl % BC == BB), after the barrier that published v_jl, s = A v_jl and column
// jl + 1: p = tau s, alpha2 = -1/2 tau (p^H v), w = p + alpha2 v, A -= v w^H + w v^H.  Then,
// with prep, the updated column jl + 1 is rebuilt from the published copy (every half-wave, no
// second barrier), reflector jl + 1 is formed (independent of the update, so the two overlap),
// column jl + 2 is published and s = A v_{jl+1} computed; with last, only the last diagonal
// entry of T is recorded.  One barrier.
template <int BR, int BC, int BB>
__device__ __forceinline__ void tri_step(z64 (&A)[BR][BC], z64 (&vloc)[BC], z64& tau, const int jl, const int Nl,
                                         const int j0, const int N, const TriSmem& M, const bool prep,
                                         const bool last) {
  const int tid = threadIdx.x, R = tid >> 5, Cc = tid & 31;
  constexpr int NH = 32 * BC / BR;
  const int par = jl & 1, nxt = par ^ 1;
  const z64* pb = M.pbuf + par * M.ld;
  const z64* vb = M.vbuf + par * M.ld;
  z64 dt = zmk(0, 0);
  z64 pcol[BC];
#pragma unroll
  for (int b = 0; b < BC; ++b) {
    pcol[b] = zmul(tau, pb[BC * Cc + b]);
    dt = zadd(dt, zcmul(pcol[b], vloc[b]));
  }
  dt.x = gsum<32>(dt.x);
  dt.y = gsum<32>(dt.y);
  const z64 alpha2 = zscale(zmul(tau, dt), -0.5);
  z64 wc[BC];
#pragma unroll
  for (int b = 0; b < BC; ++b) wc[b] = zadd(pcol[b], zmul(alpha2, vloc[b]));
#pragma unroll
  for (int a = 0; a < BR; ++a) {
    if (R + NH * a > jl) {   // uniform over the half-wave
      const z64 vr = vb[R + NH * a];
      const z64 wr = zadd(zmul(tau, pb[R + NH * a]), zmul(alpha2, vr));
      // A -= vr conj(wc) + wr conj(v): four FMAs per component
#pragma unroll
      for (int b = 0; b < BC; ++b) {
        double ax = A[a][b].x, ay = A[a][b].y;
        ax = fma(-vr.x, wc[b].x, ax);
        ay = fma(-vr.y, wc[b].x, ay);
        ax = fma(-vr.y, wc[b].y, ax);
        ay = fma(vr.x, wc[b].y, ay);
        ax = fma(-wr.x, vloc[b].x, ax);
        ay = fma(-wr.y, vloc[b].x, ay);
        ax = fma(-wr.y, vloc[b].y, ax);
        ay = fma(wr.x, vloc[b].y, ay);
        A[a][b] = zmk(ax, ay);
      }
    }
  }
  if (prep || last) {
    // column jl + 1 after this update at rows BC Cc + b (the same arithmetic as the update)
    const z64 v1 = vb[jl + 1];
    const z64 w1 = zadd(zmul(tau, pb[jl + 1]), zmul(alpha2, v1));
    const z64* ca = M.cola + par * M.ld;
    z64 c[BC];
#pragma unroll
    for (int b = 0; b < BC; ++b) {
      double cx = ca[BC * Cc + b].x, cy = ca[BC * Cc + b].y;
      cx = fma(-vloc[b].x, w1.x, cx);
      cy = fma(-vloc[b].y, w1.x, cy);
      cx = fma(-vloc[b].y, w1.y, cx);
      cy = fma(vloc[b].x, w1.y, cy);
      cx = fma(-wc[b].x, v1.x, cx);
      cy = fma(-wc[b].y, v1.x, cy);
      cx = fma(-wc[b].y, v1.y, cx);
      cy = fma(wc[b].x, v1.y, cy);
      c[b] = zmk(cx, cy);
    }
    constexpr int bd = (BB + 1) % BC, ba = (BB + 2) % BC;
    const double diag = read_lane(c[bd].x, (jl + 1) / BC);
    if (last) {
      if (tid == 0) M.d_s[j0 + jl + 1] = diag;
    } else {
      const int la = (jl + 2) / BC;
      const z64 alpha = zmk(read_lane(c[ba].x, la), read_lane(c[ba].y, la));
      z64 vn[BC], tn;
      tri_reflector<BC>(c, alpha, diag, jl + 1, Nl, j0 + jl + 1, N, M, nxt, vn, tn);
      if (Cc == la) {
#pragma unroll
        for (int a = 0; a < BR; ++a) M.cola[nxt * M.ld + R + NH * a] = A[a][ba];
      }
      tri_matvec<BR, BC>(A, vn, jl + 1, Nl, M, nxt);
#pragma unroll
      for (int b = 0; b < BC; ++b) vloc[b] = vn[b];
      tau = tn;
    }
  }
  __syncthreads();
}

// Lanes per eigenvalue of the multisection: one eigenvalue per wave, a 65-section per step.
// Recorded solves (reverse sweep, eigenvalues to 4 eps^2) keep the lane count of a work-group of
// 256 threads (order <= 32) or 512, the largest G <= 16 that covers kmax with 64 / G groups per
// wave, whose eigenvalues the reverse sweep was validated with.
constexpr int kSturmLanes = 64;
__host__ __device__ __forceinline__ int sturm_lanes(int N, int kmax, bool rec) {
  if (!rec) return kSturmLanes;
  const int nth = N <= 32 ? 256 : 512;
  int G = 16;
  while (G > 1 && (64 / G) * (nth / 64) < kmax) --G;
  return G;
}

// The leading eigenvalues of the scaled T (diagonal d, squared off-diagonal e2) handled by wave
// wv: eigenvalue t = wv (64 / G) + lane / G, its G lanes counting at the interior points of
// G + 1 equal sections of its bracket.  Each eigenvalue's bracket sequence depends only on T, G
// and its own counts, so batched and single solves give the same bits.
__device__ __forceinline__ void multisection_wave(const double* d_s, const double* e2_s, int N, int kmax, int G,
                                                  int wv, bool zero, bool rec, double* lam_out) {
  const double epsm = 2.220446049250313e-16;
  const double pivmin = 1e-290;
  const int lane = threadIdx.x & 63;
  const int gpw = 64 / G;
  const int gi = lane / G;
  const int t = wv * gpw + gi, g = lane - gi * G;
  const bool mine = gi < gpw && t < kmax;
  const bool active = mine && !zero;
  const int asc = N - 1 - t;
  // G-section: lane g counts at the interior point g + 1 of G + 1 equal sections.  Without a
  // record the bracket stops at an absolute width of 4 eps (eigenvalues to ||T|| eps, what the
  // rank rule and the inverse iteration need); a record (reverse sweep) needs eigenvalue
  // differences to relative accuracy and runs the relative rule down to 4 eps^2.
  const double floor_w = rec ? 4 * epsm * epsm : 4 * epsm;
  double lo = -1.0 - 4 * epsm, hi = 1.0 + 4 * epsm;
  // a 65-section reaches 4 eps in 9 iterations, a 9-section 4 eps^2 in at most 33; the loop
  // ends as soon as every bracket of the wave has converged
  for (int it = 0; it < 64; ++it) {
    const double w = hi - lo;
    const bool done = !(w > 2 * epsm * fmax(fabs(lo), fabs(hi)) + floor_w);
    if (__ballot(active && !done) == 0ull) break;
    const double x = lo + w * (double)(g + 1) / (double)(G + 1);
    const int cnt = (active && !done) ? sturm_count(d_s, e2_s, N, x, pivmin) : 0;
    const unsigned long long ball = __ballot(active && !done && cnt > asc);
    const int gb = gi * G;
    const unsigned long long grp = (ball >> gb) & (G >= 64 ? ~0ull : ((1ull << G) - 1ull));
    const int first = grp ? (__ffsll((long long)grp) - 1) : G;
    const double xh = __shfl(x, min(gb + (first < G ? first : 0), 63), 64);
    const double xl = __shfl(x, min(gb + (first == 0 ? 0 : first - 1), 63), 64);
    if (active && !done) {
      if (first < G) hi = xh;
      if (first > 0) lo = xl;
    }
  }
  if (g == 0 && mine) lam_out[t] = active ? 0.5 * (lo + hi) : 0.0;
}

// dynamic LDS of the eigensolver work-group: the pivots and vectors of the inverse iteration or
// the packed reflectors, whichever is larger
template <int BR, int BC>
__host__ __device__ __forceinline__ size_t eig_dyn_bytes(int kmax) {
  constexpr int NP = 32 * BC;
  const size_t ph4 = (size_t)2 * NP * kmax * sizeof(double);
  const size_t ph2 = (size_t)(NP * (NP - 1) / 2) * 16;
  return ph4 > ph2 ? ph4 : ph2;
}

template <int BR, int BC, int PART>
__device__ __forceinline__ void eig_body(const double* __restrict__ S, int Fc, const Channel& ch, int nsplit,
                                         int c, int N, int kmax, int r_target, double eps, int tie,
                                         int renorm, const EigBufs& B) {
  constexpr int NP = 32 * BC;            // padded order; the thread grid is (NP / BR) x 32
  constexpr int NTH = 32 * (NP / BR);    // threads
  extern __shared__ __attribute__((aligned(16))) double dyn[];   // phase-dependent scratch
  __shared__ z64 Mab[256];   // (E_a^H E_b) blocks: 2 x 2 (one qubit) or 4 x 4 (a qubit pair)
  __shared__ z64 col_buf[NP], vbuf[2 * NP], pbuf[2 * NP], cola[2 * NP];
  __shared__ double d_s[NP], e_s[NP], e2_s[NP], lam_s[NP + 1], tau_s[2 * NP], trp[32];
  __shared__ int cl_start[NP], cl_len[NP];
  __shared__ double sc_s[4];
  __shared__ int k_s;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int R = tid >> 5, Cc = tid & 31;   // half-wave / lane in it
  constexpr int NH = NP / BR;              // half-waves; thread rows R + NH a, columns BC Cc + b
  const int m = (nsplit >= 2) ? ch.m : 1;

  if constexpr (PART != 2) {   // phases 1 and 2 (and the scaling of T below) run in part 1
    // ---------------------------------------------------------------- 1. assemble G
    if (nsplit == 2 && tid < m * m * 4) {
      const int a = tid / (m * 4), b = (tid / 4) % m, u = (tid >> 1) & 1, v = tid & 1;
      z64 acc = zmk(0, 0);
      for (int r = 0; r < 2; ++r)
        acc = zadd(acc, zcmul(zmk(ch.e[a][r][u][0], ch.e[a][r][u][1]), zmk(ch.e[b][r][v][0], ch.e[b][r][v][1])));
      Mab[tid] = acc;   // (E_a^H E_b)_{uv} at ((a m + b) 2 + u) 2 + v
    }
    if (nsplit == 4 && tid < m * m * 16)   // (E_a^H E_b)_{u u'} at ((a m + b) 4 + u) 4 + u', formed on the host
      Mab[tid] = zmk(B.M4[2 * tid], B.M4[2 * tid + 1]);
    __syncthreads();
    // Each thread reads the S entries of its own G entries straight from memory (S is at most
    // 256 KiB): one row of the thread's layout per round, the 4 BC loads of a round in flight
    // before the first product; the terms of each G entry are added in the order
    // (u, v) = (0, 0), (0, 1), (1, 0), (1, 1).  (A chunked LDS staging of S was slower.)
    z64 A[BR][BC];
    if (nsplit == 4) {
      // a qubit pair: S is the 4-way Gram (blocks of c columns, index u = b(q0) + 2 b(q1)), G's
      // copies take its first cw = N / m columns of each block
      const double2* __restrict__ S2 = reinterpret_cast<const double2*>(S);
      const int cw = N / m;
      const int cs = __ffs(cw) - 1;
  #pragma unroll
      for (int a = 0; a < BR; ++a) {
        const int i = R + NH * a;
  #pragma unroll
        for (int b = 0; b < BC; ++b) {
          const int j = BC * Cc + b;
          z64 acc = zmk(0, 0);
          if (i < N && j < N) {
            const int ai = i >> cs, bj = j >> cs, v = i & (cw - 1), w = j & (cw - 1);
            for (int u = 0; u < 4; ++u)
              for (int u2 = 0; u2 < 4; ++u2) {
                const double2 sv = S2[(size_t)(u * c + v) * Fc + (u2 * c + w)];
                acc = zadd(acc, zmul(Mab[((ai * m + bj) * 4 + u) * 4 + u2], zmk(sv.x, sv.y)));
              }
          }
          A[a][b] = acc;
        }
      }
    } else if (nsplit == 2 && m == 2 && N == NP) {
      // two Kraus operators at the full order: rows i and i + N / 2 of G (copies 0 and 1, thread
      // slots a and a + BR / 2) take the same row of S's blocks, so every S entry loaded serves
      // both; the sums are formed in the same order as below
      const double2* __restrict__ S2 = reinterpret_cast<const double2*>(S);
      constexpr int HB = BR / 2, HN = NP / 2;
  #pragma unroll
      for (int a = 0; a < HB; ++a) {
        const int i = R + NH * a;   // < N / 2
        double2 t[BC][4];
  #pragma unroll
        for (int b = 0; b < BC; ++b) {
          const int w = (BC * Cc + b) & (HN - 1);
  #pragma unroll
          for (int uv = 0; uv < 4; ++uv) t[b][uv] = S2[(size_t)((uv >> 1) * c + i) * Fc + ((uv & 1) * c + w)];
        }
  #pragma unroll
        for (int b = 0; b < BC; ++b) {
          const int bj = (BC * Cc + b) / HN;
          z64 a0 = zmk(0, 0), a1 = zmk(0, 0);
  #pragma unroll
          for (int uv = 0; uv < 4; ++uv) {
            a0 = zadd(a0, zmul(Mab[bj * 4 + uv], zmk(t[b][uv].x, t[b][uv].y)));
            a1 = zadd(a1, zmul(Mab[(m + bj) * 4 + uv], zmk(t[b][uv].x, t[b][uv].y)));
          }
          A[a][b] = a0;
          A[a + HB][b] = a1;
        }
      }
    } else {
      // split view: S has halves of c columns; G's copies take the first cw = N / m of them, a
      // power of two (the factor's later columns are zero while its rank is still growing)
      const double2* __restrict__ S2 = reinterpret_cast<const double2*>(S);
      const int cw = (nsplit == 2) ? N / m : c;
      const int cs = __ffs(cw) - 1;
  #pragma unroll
      for (int a = 0; a < BR; ++a) {
        const int i = R + NH * a;
        double2 t[BC][4];
  #pragma unroll
        for (int b = 0; b < BC; ++b) {
          const int j = BC * Cc + b;
          const bool in = i < N && j < N;
  #pragma unroll
          for (int uv = 0; uv < 4; ++uv) {
            size_t off;
            if (nsplit == 2) {   // c and cw are powers of two in the split view
              off = (size_t)((uv >> 1) * c + (i & (cw - 1))) * Fc + ((uv & 1) * c + (j & (cw - 1)));
            } else {
              off = (size_t)i * Fc + j;
            }
            t[b][uv] = S2[in && (nsplit == 2 || uv == 0) ? off : 0];
          }
        }
  #pragma unroll
        for (int b = 0; b < BC; ++b) {
          const int j = BC * Cc + b;
          z64 acc = zmk(0, 0);
          if (i < N && j < N) {
            if (nsplit == 2) {
              const int ai = i >> cs, bj = j >> cs;
  #pragma unroll
              for (int uv = 0; uv < 4; ++uv)
                acc = zadd(acc, zmul(Mab[(ai * m + bj) * 4 + uv], zmk(t[b][uv].x, t[b][uv].y)));
            } else {
              acc = zmk(t[b][0].x, t[b][0].y);
            }
          }
          A[a][b] = acc;
        }
      }
    }
    {
      double t = 0;
  #pragma unroll
      for (int a = 0; a < BR; ++a) {
        const int i = R + NH * a;
  #pragma unroll
        for (int b = 0; b < BC; ++b)
          if (i == BC * Cc + b) t += A[a][b].x;
      }
      t = gsum<32>(t);
      if (Cc == 0) trp[R] = t;
    }
    if (Cc == 0) {
  #pragma unroll
      for (int a = 0; a < BR; ++a) col_buf[R + NH * a] = A[a][0];
    }
    __syncthreads();
    if (tid == 0) {
      double t = 0;
      for (int i = 0; i < NTH / 32; ++i) t += trp[i];
      sc_s[0] = t;   // trace
    }

    // ---------------------------------------------------------------- 2. tridiagonalisation
    // Reflector entries i >= j + 2 are kept in LDS while reducing (a global store inside the
    // loop would make every barrier wait for its completion) and spilled to the workspace
    // afterwards, because the eigenvector phase reuses this LDS.  With the 128-order layout the
    // last 64 steps run on the trailing 64 x 64 block moved to a <4, 2> layout (a quarter of the
    // arithmetic per step): the finished reflectors are spilled first and the move is staged
    // through the freed LDS.
    z64* Rf = reinterpret_cast<z64*>(dyn);
    double* refl = B.P;
    double tr_all = 0;   // every thread forms the trace from the published partials (same order)
    for (int i = 0; i < NTH / 32; ++i) tr_all += trp[i];
    const TriSmem M{col_buf, vbuf, pbuf, cola, NP, d_s, e_s, tau_s, Rf, fmax(1e-60 * tr_all * tr_all, 1e-290)};
    constexpr bool kShrink = (BR == 8 && BC == 4);
    const bool shrink = kShrink && N > 64;
    const int jsw = shrink ? N - 64 : N - 1;   // updates on the full layout
    if (N >= 2) {
      z64 vl[BC], tau;
      tri_prologue<BR, BC>(A, N, 0, N, M, vl, tau);
      for (int jb = 0; jb < jsw; jb += BC) {
        static_for<BC>([&](auto bbc) {
          const int jl = jb + decltype(bbc)::value;
          if (jl < jsw)
            tri_step<BR, BC, decltype(bbc)::value>(A, vl, tau, jl, N, 0, N, M, jl + 1 < jsw, !shrink && jl + 2 == N);
        });
      }
    } else if (tid == 0) {
      d_s[0] = col_buf[0].x;
    }
    int spilled = 0;   // reflector entries already in the workspace
    if constexpr (kShrink) {
      if (shrink) {
        spilled = refl_off(jsw, N);
        for (int e = tid; e < spilled; e += NTH) {
          refl[2 * e] = Rf[e].x;
          refl[2 * e + 1] = Rf[e].y;
        }
        __syncthreads();
        z64* Sg = Rf;   // 64 x 64 staging, row-major, local indices
  #pragma unroll
        for (int a = 0; a < BR; ++a)
  #pragma unroll
          for (int b = 0; b < BC; ++b) {
            const int i = R + NH * a, jj = BC * Cc + b;
            if (i >= jsw && jj >= jsw && i < N && jj < N) Sg[(i - jsw) * 64 + (jj - jsw)] = A[a][b];
          }
        __syncthreads();
        z64 A2[4][2];
  #pragma unroll
        for (int a = 0; a < 4; ++a)
  #pragma unroll
          for (int b = 0; b < 2; ++b) A2[a][b] = Sg[(R + 16 * a) * 64 + 2 * Cc + b];
        if (Cc == 0) {
  #pragma unroll
          for (int a = 0; a < 4; ++a) col_buf[R + 16 * a] = A2[a][0];
        }
        __syncthreads();   // the staging is read before the steps write reflectors over it
        z64 vl2[2], tau2;
        tri_prologue<4, 2>(A2, 64, jsw, N, M, vl2, tau2);
        for (int jb = 0; jb < 63; jb += 2) {
          static_for<2>([&](auto bbc) {
            const int jl = jb + decltype(bbc)::value;
            if (jl < 63) tri_step<4, 2, decltype(bbc)::value>(A2, vl2, tau2, jl, 64, jsw, N, M, jl + 1 < 63, jl == 62);
          });
        }
      }
    }
    if (tid == 0) e_s[N - 1] = 0.0;
    const int nref = (N >= 2) ? refl_off(N - 1, N) : 0;
    for (int e = spilled + tid; e < nref; e += NTH) {
      refl[2 * e] = Rf[e].x;
      refl[2 * e + 1] = Rf[e].y;
    }
    __syncthreads();
  }

  // ---------------------------------------------------------------- 3. eigenvalues
  const double pivmin = 1e-290;
  double* Tst = B.Y + kEigTOff;   // T, tau, trace and norm between the parts of a split solve
  if constexpr (PART != 2) {
    // scale T to unit Gershgorin norm
    if (wave == 0) {
      double mx = 0;
      for (int i = lane; i < N; i += 64) {
        const double el = (i > 0) ? fabs(e_s[i - 1]) : 0.0;
        const double er = (i + 1 < N) ? fabs(e_s[i]) : 0.0;
        mx = fmax(mx, fabs(d_s[i]) + el + er);
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
      if (lane == 0) sc_s[1] = mx;
    }
    __syncthreads();
    const double tn = sc_s[1];
    const double inv = (tn > 0.0) ? 1.0 / tn : 1.0;
    for (int i = tid; i < N; i += NTH) {
      d_s[i] *= inv;
      e_s[i] = (i + 1 < N) ? e_s[i] * inv : 0.0;
      e2_s[i] = e_s[i] * e_s[i];
    }
    __syncthreads();
  }
  if constexpr (PART == 1) {
    for (int i = tid; i < N; i += NTH) {
      Tst[i] = d_s[i];
      Tst[kMaxEig + i] = e_s[i];
      Tst[2 * kMaxEig + i] = e2_s[i];
    }
    for (int i = tid; i < 2 * N; i += NTH) Tst[3 * kMaxEig + i] = tau_s[i];
    if (tid < 2) Tst[5 * kMaxEig + tid] = sc_s[tid];   // trace, Gershgorin norm
    return;
  }
  if constexpr (PART == 2) {
    for (int i = tid; i < N; i += NTH) {
      d_s[i] = Tst[i];
      e_s[i] = Tst[kMaxEig + i];
      e2_s[i] = Tst[2 * kMaxEig + i];
    }
    for (int i = tid; i < 2 * N; i += NTH) tau_s[i] = Tst[3 * kMaxEig + i];
    if (tid < 2) sc_s[tid] = Tst[5 * kMaxEig + tid];
    for (int t = tid; t < kmax; t += NTH) lam_s[t] = B.lam[t];   // from the multisection kernel
    __syncthreads();
  }
  const double tnorm = sc_s[1];
  const bool zero = !(tnorm > 0.0);
  __syncthreads();
  if (wave == 0) {
    // clusters: a cluster starts at t = 0 and wherever lam_{t-1} - lam_t > max(1e-9, 1e-3
    // lam_{t-1}) (scaled T).  Inverse iteration leaves the vectors of eigenvalues a gap g apart
    // with an overlap near eps / g, which moves rho by about sqrt(lam_i lam_j) eps / g: the
    // relative window keeps that near 1e-13 without joining a graded spectrum into one cluster.
    // One ballot per 64 eigenvalues marks the starts (kmax <= 128, two words).
    unsigned long long starts[2] = {0ull, 0ull};
    for (int c = 0; c < 2; ++c) {
      const int t = 64 * c + lane;
      const bool st = t < kmax && (t == 0 || !(lam_s[t - 1] - lam_s[t] <= fmax(1e-9, 1e-3 * fabs(lam_s[t - 1]))));
      starts[c] = __ballot(st);
    }
    for (int c = 0; c < 2; ++c) {
      const int t = 64 * c + lane;
      if (t < kmax) {
        // start of t's cluster: the last start at or before t
        const unsigned long long upto = starts[c] & (lane == 63 ? ~0ull : ((2ull << lane) - 1ull));
        int s0;
        if (upto) s0 = 64 * c + 63 - __clzll((long long)upto);
        else s0 = 63 - __clzll((long long)starts[0]);   // c == 1: the last start of the first word
        cl_start[t] = s0;
        // length (read for starts only): up to the next start, or to kmax
        int len = 0;
        if (s0 == t) {
          const unsigned long long after = (lane == 63) ? 0ull : (starts[c] >> (lane + 1)) << (lane + 1);
          int nxt;
          if (after) nxt = 64 * c + __ffsll((long long)after) - 1;
          else if (c == 0 && starts[1]) nxt = 64 + __ffsll((long long)starts[1]) - 1;
          else nxt = kmax;
          len = nxt - t;
        }
        cl_len[t] = len;
      }
    }
  }
  __syncthreads();

  // ---------------------------------------------------------------- 4. eigenvectors of T
  // One lane per eigenvector.  The recurrences run over chunks of CH rows whose operands are
  // read from LDS before the dependent arithmetic (LDS latency paid once per chunk), with a
  // scalar remainder loop, so no load or store in a chunk is conditional.
  constexpr int CH = 8;
  const int KP = kmax;
  double* Dp = dyn;              // inverse LDL^T pivots, [i * KP + t]
  double* X = dyn + NP * KP;     // vectors, [i * KP + t]
  for (int i = wave; i < N; i += NTH / 64)
    for (int t = lane; t < kmax; t += 64) X[i * KP + t] = 1.0 + hash_unit((uint32_t)t, (uint32_t)i);
  if (tid < kmax) {
    const int t = tid;
    const double sigma = lam_s[t];
    // pivots D_i of T - sigma I = L D L^T, stored as 1 / D_i
    double dp0 = d_s[0] - sigma;
    if (fabs(dp0) < pivmin) dp0 = -pivmin;
    double rinv = rcp_nr(dp0);
    Dp[t] = rinv;
    int i = 1;
    for (; i + CH <= N; i += CH) {
      double dd[CH], ee[CH];
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        dd[u] = d_s[i + u] - sigma;
        ee[u] = e2_s[i + u - 1];
      }
#pragma unroll
      for (int u = 0; u < CH; ++u) {
        double dp = dd[u] - ee[u] * rinv;
        if (fabs(dp) < pivmin) dp = -pivmin;
        rinv = rcp_nr(dp);
        dd[u] = rinv;
      }
#pragma unroll
      for (int u = 0; u < CH; ++u) Dp[(i + u) * KP + t] = dd[u];
    }
    for (; i < N; ++i) {
      double dp = (d_s[i] - sigma) - e2_s[i - 1] * rinv;
      if (fabs(dp) < pivmin) dp = -pivmin;
      rinv = rcp_nr(dp);
      Dp[i * KP + t] = rinv;
    }
  }
  __syncthreads();
  for (int iter = 0; iter < 2; ++iter) {
    if (tid < kmax) {
      const int t = tid;
      // forward: y_i = x_i - l_{i-1} y_{i-1}, l_{i-1} = e_{i-1} / D_{i-1}
      double y = X[t];
      double rprev = Dp[t];
      int i = 1;
      for (; i + CH <= N; i += CH) {
        double xx[CH], rr[CH], ee[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
          xx[u] = X[(i + u) * KP + t];
          rr[u] = Dp[(i + u) * KP + t];
          ee[u] = e_s[i + u - 1];
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) {
          y = xx[u] - (ee[u] * rprev) * y;
          xx[u] = y;
          rprev = rr[u];
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) X[(i + u) * KP + t] = xx[u];
      }
      for (; i < N; ++i) {
        const double ri = Dp[i * KP + t];
        y = X[i * KP + t] - (e_s[i - 1] * rprev) * y;
        X[i * KP + t] = y;
        rprev = ri;
      }
      // backward: x_i = (y_i - e_i x_{i+1}) / D_i
      double xn = X[(N - 1) * KP + t] * Dp[(N - 1) * KP + t];
      X[(N - 1) * KP + t] = xn;
      double mx = fabs(xn);
      i = N - 2;
      for (; i - CH + 1 >= 0; i -= CH) {
        double yy[CH], rr[CH], ee[CH];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
          yy[u] = X[(i - u) * KP + t];
          rr[u] = Dp[(i - u) * KP + t];
          ee[u] = e_s[i - u];
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) {
          xn = (yy[u] - ee[u] * xn) * rr[u];
          yy[u] = xn;
          mx = fmax(mx, fabs(xn));
        }
#pragma unroll
        for (int u = 0; u < CH; ++u) X[(i - u) * KP + t] = yy[u];
      }
      for (; i >= 0; --i) {
        xn = (X[i * KP + t] - e_s[i] * xn) * Dp[i * KP + t];
        X[i * KP + t] = xn;
        mx = fmax(mx, fabs(xn));
      }
      // unit 2-norm (scaled by the largest entry first, so the squares cannot overflow)
      const double s1 = (mx > 0) ? 1.0 / mx : 1.0;
      double nn[4] = {0.0, 0.0, 0.0, 0.0};
      for (int r = 0; r < N; ++r) {
        const double v = X[r * KP + t] * s1;
        nn[r & 3] = fma(v, v, nn[r & 3]);
      }
      const double ns = (nn[0] + nn[1]) + (nn[2] + nn[3]);
      const double sc = s1 * ((ns > 0) ? 1.0 / sqrt(ns) : 0.0);
      for (int r = 0; r < N; ++r) X[r * KP + t] *= sc;
    }
    __syncthreads();
    for (int cs = wave; cs < kmax; cs += NTH / 64) {
      if (cl_start[cs] != cs || cl_len[cs] < 2) continue;
      const int len = cl_len[cs];
      for (int jj = cs; jj < cs + len; ++jj) {
        for (int ii = cs; ii < jj; ++ii) {
          double dtt = 0;
          for (int i = lane; i < N; i += 64) dtt += X[i * KP + ii] * X[i * KP + jj];
          dtt = gsum<64>(dtt);
          for (int i = lane; i < N; i += 64) X[i * KP + jj] -= dtt * X[i * KP + ii];
        }
        double nq = 0;
        for (int i = lane; i < N; i += 64) nq += X[i * KP + jj] * X[i * KP + jj];
        nq = gsum<64>(nq);
        const double s2 = (nq > 0) ? 1.0 / sqrt(nq) : 0.0;
        for (int i = lane; i < N; i += 64) X[i * KP + jj] *= s2;
      }
    }
    __syncthreads();
  }

  // ---------------------------------------------------------------- 5. rank rule
  if (tid == 0) {
    const double trace = sc_s[0];
    for (int t = 0; t < kmax; ++t) lam_s[t] = zero ? 0.0 : lam_s[t] * tnorm;
    int k = min(r_target, N);
    bool bad = !isfinite(trace) || !isfinite(tnorm);
    if (eps > 0.0) {
      double kept = 0;
      int keps = N;
      for (int i = 0; i < kmax; ++i) {
        kept += fmax(lam_s[i], 0.0);
        if (kept >= (1.0 - eps) * trace) {
          keps = i + 1;
          break;
        }
      }
      k = min(k, keps);
    }
    if (tie == 1)   // the spectrum continues with zeros beyond the Gram order
      while (k > 1 && (lam_s[k - 1] - (k < N ? lam_s[k] : 0.0)) <= 1e-6 * trace) --k;
    if (k < 1) k = 1;
    double kept = 0;
    for (int i = 0; i < k; ++i) kept += fmax(lam_s[i], 0.0);
    if (!(kept > 0.0)) bad = true;
    const double scl = (renorm && kept > 0.0) ? 1.0 / sqrt(kept) : 1.0;
    DevInfo* inf = B.info;
    const double disc = fmax(trace - kept, 0.0);
    inf->k = k;
    inf->n_eig = N;
    inf->discarded = disc;
    inf->discarded_total += disc;
    inf->trace = trace;
    inf->gap = (k < N) ? (lam_s[k - 1] - lam_s[k]) : INFINITY;
    inf->lambda_max = lam_s[0];
    inf->scale = scl;
    if (bad) inf->status = (int)LRDM_E_EIG;
    k_s = k;
    sc_s[2] = scl;
  }
  __syncthreads();
  for (int t = tid; t < kmax; t += NTH) B.lam[t] = lam_s[t];
  const int k = k_s;
  // with a record every eigenvector is formed (kmax == N <= 64), else only the kept ones
  const int nvec = B.rec ? N : k;
  double* Y = B.Y;
  for (int e = tid; e < 2 * (N - 1); e += NTH) Y[e] = tau_s[e];
  for (int col = tid / NP; col < nvec; col += NTH / NP) {   // NP is a power of two
    const int i = tid & (NP - 1);
    if (i < N) Y[kEigYOff + col * kMaxEig + i] = zero ? (i == col ? 1.0 : 0.0) : X[i * KP + col];
  }
  if (B.rec) {
    double* rec = B.rec;
    if (tid == 0) {
      rec[0] = (double)k;
      rec[1] = sc_s[2];
      rec[2] = (double)N;
      rec[3] = sc_s[0];
      rec[4] = (double)renorm;
    }
    for (int t = tid; t < N; t += NTH) rec[kRecHeader + t] = lam_s[t];
  }
}

// ---------------------------------------------------------------- back-transform and W
// V = Q Y for the kept eigenvectors (every eigenvector with a record), with Q = H_0 ... H_{N-2}
// applied from the right end, and the projection matrix
// W_{(b,v),(b',j)} = c sum_a (E_a)_{b'b} V[(a,v), j] (split view) or W = c V_k (plain view).
// Columns are independent, so this runs over kEigBtBlocks work-groups of kEigBtCols waves, one
// column per wave, a lane holding rows lane + 64 s.  The packed reflectors are staged in LDS in
// chunks of kBtChunk reflectors, in the order they are applied: the loads of the next chunk are
// in flight while the current one is applied.
constexpr int kBtChunk = 16;
constexpr int kBtPer = 8;   // staged entries per thread and chunk
static_assert(kBtChunk * (kMaxEig - 2) <= 64 * kEigBtCols * kBtPer, "a chunk must fit the staging registers");

__device__ __forceinline__ void bt_chunk_range(int jhi, int N, int& e0, int& e1, int& jlo) {
  jlo = max(0, jhi - kBtChunk + 1);
  e0 = refl_off(jlo, N);
  e1 = refl_off(jhi + 1, N);
}

template <class T, int RPL>
__device__ __forceinline__ void backtransform_body(const Channel& ch, int nsplit, int c, int N, int c_out,
                                                   const EigBufs& B, cx_t<T>* __restrict__ W, int cblk) {
  constexpr int NP = 64 * RPL;
  constexpr int NTB = 64 * kEigBtCols;
  extern __shared__ __attribute__((aligned(16))) double bt_dyn[];
  z64* rfl = reinterpret_cast<z64*>(bt_dyn);   // packed reflector entries (refl_off layout)
  __shared__ z64 tau_l[kMaxEig];
  __shared__ z64 Vs[kEigBtCols][NP];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int k = B.info->k;
  const double scl = B.info->scale;
  const int nvec = B.rec ? N : k;
  if (cblk * kEigBtCols >= max(nvec, c_out)) return;   // uniform over the work-group
  const int col = cblk * kEigBtCols + wave;
  const bool act = col < nvec;
  const double2* __restrict__ refl = reinterpret_cast<const double2*>(B.P);
  for (int j = tid; j < N - 1; j += NTB) tau_l[j] = zmk(B.Y[2 * j], B.Y[2 * j + 1]);
  z64 z[RPL];
#pragma unroll
  for (int s = 0; s < RPL; ++s) {
    const int i = lane + 64 * s;
    z[s] = zmk((act && i < N) ? B.Y[kEigYOff + col * kMaxEig + i] : 0.0, 0.0);
  }
  // z and tau are needed at once; waiting here keeps the loop below from waiting on the
  // staging loads it issues ahead of their use
  __builtin_amdgcn_s_waitcnt(0);
  double2 st[kBtPer];
  int e0, e1, jlo;
  if (N >= 2) {
    bt_chunk_range(N - 2, N, e0, e1, jlo);
#pragma unroll
    for (int p = 0; p < kBtPer; ++p) {
      const int e = e0 + tid + NTB * p;
      st[p] = refl[e < e1 ? e : e0];
    }
#pragma unroll
    for (int p = 0; p < kBtPer; ++p) {
      const int e = e0 + tid + NTB * p;
      if (e < e1) rfl[e] = zmk(st[p].x, st[p].y);
    }
  }
  __syncthreads();
  for (int jhi = N - 2; jhi >= 0; jhi -= kBtChunk) {
    bt_chunk_range(jhi, N, e0, e1, jlo);
    const bool more = jlo > 0;
    int f0 = 0, f1 = 0, flo = 0;
    if (more) {
      bt_chunk_range(jlo - 1, N, f0, f1, flo);
#pragma unroll
      for (int p = 0; p < kBtPer; ++p) {
        const int e = f0 + tid + NTB * p;
        st[p] = refl[e < f1 ? e : f0];
      }
    }
    if (act) {
      // four reflectors at a time: their LDS reads (every lane reads, from entry 0 where it
      // needs none, and selects the value it needs, so no read sits behind a branch) are
      // issued before the first is applied
      for (int jg = jhi; jg >= jlo; jg -= 4) {
        z64 v[4][RPL], tj[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int j = jg - u;
          const int ro = refl_off(j, N) - j - 2;
          tj[u] = tau_l[j >= 0 ? j : 0];
#pragma unroll
          for (int s = 0; s < RPL; ++s) {
            const int i = lane + 64 * s;
            const bool stv = j >= jlo && i >= j + 2 && i < N;
            const z64 ld = rfl[stv ? ro + i : 0];
            // a select, not a multiplication by 0: entry 0 may not be staged yet, and LDS left
            // by an earlier kernel can hold NaN or Inf
            v[u][s] = stv ? ld : zmk(i == j + 1 ? 1.0 : 0.0, 0.0);
          }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if (jg - u >= jlo) {   // uniform
            z64 sm = zcmul(v[u][0], z[0]);
#pragma unroll
            for (int s = 1; s < RPL; ++s) sm = zadd(sm, zcmul(v[u][s], z[s]));
            wsum64x2(sm.x, sm.y);
            const z64 ts = zmul(tj[u], sm);
#pragma unroll
            for (int s = 0; s < RPL; ++s) z[s] = zsub(z[s], zmul(v[u][s], ts));
          }
        }
      }
    }
    if (more) {
#pragma unroll
      for (int p = 0; p < kBtPer; ++p) {
        const int e = f0 + tid + NTB * p;
        if (e < f1) rfl[e] = zmk(st[p].x, st[p].y);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int s = 0; s < RPL; ++s) Vs[wave][lane + 64 * s] = z[s];
  __syncthreads();
  if (B.rec && col < N) {
    double* rv = B.rec + kRecHeader + N;
    for (int i = lane; i < N; i += 64) {
      rv[2 * (i * N + col)] = Vs[wave][i].x;
      rv[2 * (i * N + col) + 1] = Vs[wave][i].y;
    }
  }
  if (col >= c_out) return;
  using C = cx_t<T>;
  if (nsplit == 4) {
    // a qubit pair: W_{(u,v),(u',j)} = c sum_a (E_a)_{u'u} V[(a,v), j], u = b(q0) + 2 b(q1)
    const int rows = 4 * c, cols = 4 * c_out;
    const int cs = __ffs(c) - 1;
    const int cw = N / ch.m;
    for (int rw = lane; rw < rows; rw += 64) {
      const int u = rw >> cs, v = rw & (c - 1);
      for (int up = 0; up < 4; ++up) {
        z64 acc = zmk(0, 0);
        if (col < k && v < cw) {
          for (int a = 0; a < ch.m; ++a) {
            const int e = (a * 4 + up) * 4 + u;
            acc = zadd(acc, zmul(zmk(B.E4[2 * e], B.E4[2 * e + 1]), Vs[wave][a * cw + v]));
          }
        }
        C o;
        o.x = (T)(acc.x * scl);
        o.y = (T)(acc.y * scl);
        W[rw * cols + up * c_out + col] = o;
      }
    }
  } else if (nsplit == 2) {
    const int rows = 2 * c, cols = 2 * c_out;
    const int cs = __ffs(c) - 1;   // c is a power of two in the split view
    const int cw = N / ch.m;       // columns of each copy in G (rows v >= cw of W are zero)
    for (int rw = lane; rw < rows; rw += 64) {
      const int b = rw >> cs, v = rw & (c - 1);
#pragma unroll
      for (int bp = 0; bp < 2; ++bp) {
        z64 acc = zmk(0, 0);
        if (col < k && v < cw) {
          for (int a = 0; a < ch.m; ++a)
            acc = zadd(acc, zmul(zmk(ch.e[a][bp][b][0], ch.e[a][bp][b][1]), Vs[wave][a * cw + v]));
        }
        const int e = rw * cols + bp * c_out + col;
        C o;
        o.x = (T)(acc.x * scl);
        o.y = (T)(acc.y * scl);
        W[e] = o;
        if (B.W64) {
          B.W64[2 * e] = acc.x * scl;
          B.W64[2 * e + 1] = acc.y * scl;
        }
      }
    }
  } else {
    for (int i = lane; i < N; i += 64) {
      const z64 acc = (col < k) ? Vs[wave][i] : zmk(0, 0);
      C o;
      o.x = (T)(acc.x * scl);
      o.y = (T)(acc.y * scl);
      W[i * c_out + col] = o;
    }
  }
}

// A solve runs in three kernels before the back-transform: part 1 (assembly, tridiagonal
// reduction, scaling of T) and part 2 (eigenvectors of T, rank rule) on one work-group each, and
// between them the multisection with one work-group per wave (one eigenvalue per wave), each on
// a CU of its own, so the Sturm counts run at their latency instead of sharing SIMDs.  The batched
// twins take one job (or one job's wave) per work-group and compute the same bits.
template <int BR, int BC>
__global__ __launch_bounds__(32 * (32 * BC / BR)) void eig_reduce_kernel(const double* __restrict__ S, int Fc,
                                                                         Channel ch, int nsplit, int c, int N,
                                                                         int kmax, int r_target, double eps, int tie,
                                                                         int renorm, EigBufs B) {
  eig_body<BR, BC, 1>(S, Fc, ch, nsplit, c, N, kmax, r_target, eps, tie, renorm, B);
}

template <int BR, int BC>
__global__ __launch_bounds__(32 * (32 * BC / BR)) void eig_vectors_kernel(const double* __restrict__ S, int Fc,
                                                                          Channel ch, int nsplit, int c, int N,
                                                                          int kmax, int r_target, double eps, int tie,
                                                                          int renorm, EigBufs B) {
  eig_body<BR, BC, 2>(S, Fc, ch, nsplit, c, N, kmax, r_target, eps, tie, renorm, B);
}

__device__ __forceinline__ void sturm_body(int N, int kmax, int wv, const double* __restrict__ Tst,
                                           double* __restrict__ lam, bool rec) {
  const int G = sturm_lanes(N, kmax, rec);
  __shared__ double d_s[kMaxEig], e2_s[kMaxEig];
  for (int i = threadIdx.x; i < N; i += 64) {
    d_s[i] = Tst[i];
    e2_s[i] = Tst[2 * kMaxEig + i];
  }
  __syncthreads();
  const bool zero = !(Tst[5 * kMaxEig + 1] > 0.0);
  multisection_wave(d_s, e2_s, N, kmax, G, wv, zero, rec, lam);
}

// waves of one solve's multisection (at most kmax)
__host__ __device__ __forceinline__ int sturm_waves(int N, int kmax, bool rec) {
  const int per = 64 / sturm_lanes(N, kmax, rec);
  return (kmax + per - 1) / per;
}

__global__ __launch_bounds__(64) void eig_sturm_kernel(int N, int kmax, const double* __restrict__ Tst,
                                                       double* __restrict__ lam, int rec) {
  sturm_body(N, kmax, blockIdx.x, Tst, lam, rec != 0);
}

// One work-group per job; every job of a launch has the same size class (BR, BC).
template <class T, int BR, int BC>
__global__ __launch_bounds__(32 * (32 * BC / BR)) void eig_reduce_batched(const EigJob<T>* __restrict__ jobs) {
  const EigJob<T>& J = jobs[blockIdx.x];
  eig_body<BR, BC, 1>(J.S, J.Fc, J.ch, J.nsplit, J.c, J.N, J.kmax, J.r_target, J.eps, J.tie, J.renorm, J.B);
}

template <class T, int BR, int BC>
__global__ __launch_bounds__(32 * (32 * BC / BR)) void eig_vectors_batched(const EigJob<T>* __restrict__ jobs) {
  const EigJob<T>& J = jobs[blockIdx.x];
  eig_body<BR, BC, 2>(J.S, J.Fc, J.ch, J.nsplit, J.c, J.N, J.kmax, J.r_target, J.eps, J.tie, J.renorm, J.B);
}

// wpj work-groups (waves) per job; a job with fewer eigenvalues leaves its last ones idle
template <class T>
__global__ __launch_bounds__(64) void eig_sturm_batched(const EigJob<T>* __restrict__ jobs, int wpj) {
  const EigJob<T>& J = jobs[blockIdx.x / wpj];
  const int wv = blockIdx.x % wpj;
  if (wv >= sturm_waves(J.N, J.kmax, J.B.rec != nullptr)) return;   // uniform over the work-group
  sturm_body(J.N, J.kmax, wv, J.B.Y + kEigTOff, J.B.lam, J.B.rec != nullptr);
}

template <class T, int RPL>
__global__ __launch_bounds__(64 * kEigBtCols) void backtransform_kernel(Channel ch, int nsplit, int c, int N,
                                                                     int c_out, EigBufs B,
                                                                     cx_t<T>* __restrict__ W) {
  backtransform_body<T, RPL>(ch, nsplit, c, N, c_out, B, W, blockIdx.x);
}

// kEigBtBlocks work-groups per job
template <class T, int RPL>
__global__ __launch_bounds__(64 * kEigBtCols) void backtransform_batched(const EigJob<T>* __restrict__ jobs) {
  const EigJob<T>& J = jobs[blockIdx.x / kEigBtBlocks];
  backtransform_body<T, RPL>(J.ch, J.nsplit, J.c, J.N, J.c_out, J.B, J.W, blockIdx.x % kEigBtBlocks);
}

template <int BR, int BC>
static size_t eig_shm(int kmax) {
  return eig_dyn_bytes<BR, BC>(kmax);
}

// packed reflector entries of an order-N eigensolve (at least one entry)
static size_t bt_shm(int N) {
  const int ne = N >= 3 ? (N - 1) * (N - 2) / 2 : 1;
  return (size_t)ne * 16;
}

template <class F>
static hipError_t allow_shm(F* fn, size_t shm) {
  if (shm <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(fn), hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
}

template <class T, int BR, int BC>
static hipError_t launch_eig_batched_bs(const EigJob<T>* jobs, int njobs, int kmax_max, hipStream_t s) {
  constexpr int NP = 32 * BC;
  constexpr int NTH = 32 * (NP / BR);
  const size_t shm = eig_shm<BR, BC>(kmax_max);
  hipError_t e = allow_shm(eig_reduce_batched<T, BR, BC>, shm);
  if (e != hipSuccess) return e;
  e = allow_shm(eig_vectors_batched<T, BR, BC>, shm);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((eig_reduce_batched<T, BR, BC>), dim3(njobs), dim3(NTH), shm, s, jobs);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int wpj = kmax_max;   // the most waves any job of the launch needs
  hipLaunchKernelGGL(eig_sturm_batched<T>, dim3(njobs * wpj), dim3(64), 0, s, jobs, wpj);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((eig_vectors_batched<T, BR, BC>), dim3(njobs), dim3(NTH), shm, s, jobs);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  constexpr int RPL = NP > 64 ? 2 : 1;
  const size_t bshm = bt_shm(NP);
  e = allow_shm(backtransform_batched<T, RPL>, bshm);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((backtransform_batched<T, RPL>), dim3(njobs * kEigBtBlocks), dim3(64 * kEigBtCols), bshm, s,
                     jobs);
  return hipGetLastError();
}

template <class T>
hipError_t launch_eig_batched(int N, const EigJob<T>* jobs, int njobs, int kmax_max, hipStream_t s) {
  if (njobs < 1 || N < 1 || N > kMaxEig || kmax_max < 1) return hipErrorInvalidValue;
  if (N <= 32) return launch_eig_batched_bs<T, 4, 1>(jobs, njobs, kmax_max, s);
  if (N <= 64) return launch_eig_batched_bs<T, 4, 2>(jobs, njobs, kmax_max, s);
  return launch_eig_batched_bs<T, 8, 4>(jobs, njobs, kmax_max, s);
}

template hipError_t launch_eig_batched<float>(int, const EigJob<float>*, int, int, hipStream_t);
template hipError_t launch_eig_batched<double>(int, const EigJob<double>*, int, int, hipStream_t);

template <int BR, int BC>
static hipError_t launch_eig_bs(const double* S, int Fc, const Channel& ch, int nsplit, int c, int N, int kmax,
                                int r_target, double eps, int tie, int renorm, const EigBufs& b, hipStream_t s) {
  constexpr int NP = 32 * BC;
  constexpr int NTH = 32 * (NP / BR);
  const size_t shm = eig_shm<BR, BC>(kmax);
  hipError_t e = allow_shm(eig_reduce_kernel<BR, BC>, shm);
  if (e != hipSuccess) return e;
  e = allow_shm(eig_vectors_kernel<BR, BC>, shm);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((eig_reduce_kernel<BR, BC>), dim3(1), dim3(NTH), shm, s, S, Fc, ch, nsplit, c, N, kmax,
                     r_target, eps, tie, renorm, b);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(eig_sturm_kernel, dim3(sturm_waves(N, kmax, b.rec != nullptr)), dim3(64), 0, s, N, kmax,
                     b.Y + kEigTOff, b.lam, b.rec ? 1 : 0);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((eig_vectors_kernel<BR, BC>), dim3(1), dim3(NTH), shm, s, S, Fc, ch, nsplit, c, N, kmax,
                     r_target, eps, tie, renorm, b);
  return hipGetLastError();
}

template <class T>
hipError_t launch_eig(const double* S, int Fc, const Channel& ch, int nsplit, int c, int N,
                      int kmax, int r_target, double eps, int tie, int renorm, int c_out,
                      const EigBufs& b, cx_t<T>* W, hipStream_t s) {
  if (N < 1 || N > kMaxEig || kmax < 1 || kmax > N || r_target > 64 || c_out > 64) return hipErrorInvalidValue;
  if (nsplit >= 2 && (c < 1 || (c & (c - 1)))) return hipErrorInvalidValue;   // split view: c a power of two
  if (nsplit == 4 && (!b.M4 || !b.E4 || b.rec || N % ch.m)) return hipErrorInvalidValue;
  if (b.rec && (N > kRecMaxN || kmax != N)) return hipErrorInvalidValue;
  hipError_t e;
  // layouts: order <= 32 on 256 threads (<4, 1>), <= 64 on 512 threads (<4, 2>), <= 128 on 512
  // threads (<8, 4>, the last 64 steps on <4, 2>): fewer waves per barrier and reduction where the
  // matrix is small (a 64 x 64 reduction on 1024 threads took 1.5x as long)
  if (N <= 32) e = launch_eig_bs<4, 1>(S, Fc, ch, nsplit, c, N, kmax, r_target, eps, tie, renorm, b, s);
  else if (N <= 64) e = launch_eig_bs<4, 2>(S, Fc, ch, nsplit, c, N, kmax, r_target, eps, tie, renorm, b, s);
  else e = launch_eig_bs<8, 4>(S, Fc, ch, nsplit, c, N, kmax, r_target, eps, tie, renorm, b, s);
  if (e != hipSuccess) return e;
  const size_t bshm = bt_shm(N);
  if (N <= 64) {
    e = allow_shm(backtransform_kernel<T, 1>, bshm);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((backtransform_kernel<T, 1>), dim3(kEigBtBlocks), dim3(64 * kEigBtCols), bshm, s, ch, nsplit,
                       c, N, c_out, b, W);
  } else {
    e = allow_shm(backtransform_kernel<T, 2>, bshm);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((backtransform_kernel<T, 2>), dim3(kEigBtBlocks), dim3(64 * kEigBtCols), bshm, s, ch, nsplit,
                       c, N, c_out, b, W);
  }
  return hipGetLastError();
}

template hipError_t launch_eig<float>(const double*, int, const Channel&, int, int, int, int, int, double,
                                      int, int, int, const EigBufs&, float2*, hipStream_t);
template hipError_t launch_eig<double>(const double*, int, const Channel&, int, int, int, int, int, double,
                                       int, int, int, const EigBufs&, double2*, hipStream_t);

}  // namespace lrdm
