// Gate sweeps over the low-rank factor: L <- G L column by column (Eq. "low rank evolution G",
// Sec. II.A), fused so that one HBM read + write of L applies every gate of a pass.
//
// Layout: L is row-major [2^n][ld] complex.  A pass picks k <= 8 "local" qubits; a row tile is
// the 2^k rows that differ only in those bits (up to 64 KB).  A work-group stages one tile in
// LDS, applies every operation of the pass in order as a sweep over row pairs (1q), quads (2q)
// or rows (diagonal gates, which act on any qubit because the full row index is known), and
// writes the tile back.  Consecutive threads handle consecutive columns of one row, so every
// global load/store is a contiguous ncols-wide row segment whatever the qubit.
#include <utility>

#include "lrdm_internal.h"

namespace lrdm {

typedef float f4v __attribute__((ext_vector_type(4)));   // 16-byte register unit
constexpr int kGateThreads = 512;   // 8 waves: one register group per thread for a 64 KB tile

template <class C> __device__ __forceinline__ C cmul(C a, C b) {
  C r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}
template <class C> __device__ __forceinline__ C cadd(C a, C b) {
  C r;
  r.x = a.x + b.x;
  r.y = a.y + b.y;
  return r;
}
template <class C, class T> __device__ __forceinline__ C cmk(T re, T im) {
  C r;
  r.x = re;
  r.y = im;
  return r;
}

__device__ __forceinline__ uint32_t insert_zero(uint32_t p, int j) {
  return ((p >> j) << (j + 1)) | (p & ((1u << j) - 1u));
}

template <class F, int... I>
__device__ __forceinline__ void gate_static_for_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void gate_static_for(F&& f) {
  gate_static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// plain two-field complex for register arrays (the HIP vector types are unions, which keeps
// arrays of them out of registers)
template <class T> struct RC {
  T x, y;
};

// Non-temporal HBM access of one complex value (the factor is streamed once per pass)
template <class T> struct NtV;
template <> struct NtV<float> { typedef float type __attribute__((ext_vector_type(2))); };
template <> struct NtV<double> { typedef double type __attribute__((ext_vector_type(2))); };
template <class T>
__device__ __forceinline__ RC<T> ld_nt(const cx_t<T>* p) {
  const auto v = __builtin_nontemporal_load(reinterpret_cast<const typename NtV<T>::type*>(p));
  return RC<T>{v[0], v[1]};
}
template <class T>
__device__ __forceinline__ void st_nt(cx_t<T>* p, RC<T> x) {
  typename NtV<T>::type v;
  v[0] = x.x;
  v[1] = x.y;
  __builtin_nontemporal_store(v, reinterpret_cast<typename NtV<T>::type*>(p));
}

// 1q gate on register bit B of 2^R registers (all indices compile-time)
template <int B, int R, class T>
__device__ __forceinline__ void reg_1q(RC<T> (&x)[1 << R], const T* u) {
  using C = RC<T>;
  const C u00{u[0], u[1]}, u01{u[2], u[3]};
  const C u10{u[4], u[5]}, u11{u[6], u[7]};
#pragma unroll
  for (int i = 0; i < (1 << R); ++i) {
    if (!(i & (1 << B))) {
      const C a = x[i], b = x[i | (1 << B)];
      x[i] = C{u00.x * a.x - u00.y * a.y + u01.x * b.x - u01.y * b.y,
               u00.x * a.y + u00.y * a.x + u01.x * b.y + u01.y * b.x};
      x[i | (1 << B)] = C{u10.x * a.x - u10.y * a.y + u11.x * b.x - u11.y * b.y,
                          u10.x * a.y + u10.y * a.x + u11.x * b.y + u11.y * b.x};
    }
  }
}

// OR of the uniform values v[b] over the set bits b of i (i is a constant after unrolling)
template <int R>
__device__ __forceinline__ uint32_t pick_or(int i, const uint32_t (&v)[R]) {
  uint32_t r = 0;
#pragma unroll
  for (int b = 0; b < R; ++b)
    if (i & (1 << b)) r |= v[b];
  return r;
}

// Register layout of phase ph (GatePass::ph_word): the thread's 2^R elements differ in the
// phase's register slots (sh_pos: their tile offsets, sh_row: their row bits); the column and
// the other slots come from the thread index te (pos: its tile offset, sub: the local-qubit part
// of its row index).
template <class T, int R>
__device__ __forceinline__ void phase_layout(const GatePass<T>& P, int ph, int cshift, uint32_t te, uint32_t& pos,
                                             uint32_t& sub, uint32_t (&sh_pos)[R], uint32_t (&sh_row)[R]) {
  const uint32_t w = P.ph_word[ph];
#pragma unroll
  for (int b = 0; b < R; ++b) {
    const uint32_t slot = (w >> (4 * b)) & 15u;
    sh_pos[b] = 1u << (cshift + slot);
    sh_row[b] = 1u << P.local_q[slot];
  }
  pos = te & ((1u << cshift) - 1u);
  sub = 0;
  for (int t = 0; t < P.k - R; ++t) {
    const uint32_t slot = (w >> (16 + 4 * t)) & 15u;
    const uint32_t bit = (te >> (cshift + t)) & 1u;
    pos |= bit << (cshift + slot);
    sub |= bit << P.local_q[slot];
  }
}

// Diagonal operation on the registers of one thread.  Its phase index is sel = b_a + 2 b_b
// (b_a, b_b: the row bits of its two qubits).  RA / RB is the register bit holding qubit a / b
// in this phase, or -1 where that bit comes from the thread's row index (ta / tb, shared by all
// its registers).  The registers fall into at most four patterns s = (bit RA of i, bit RB of i)
// with one phase each (the same on every lane when both qubits are register bits).  Every
// register is multiplied in place, without branches, so the registers keep their places.
template <int RA, int RB, bool REAL, class T, int R>
__device__ __forceinline__ void reg_diag(RC<T> (&x)[1 << R], RC<T> d0, RC<T> d1, RC<T> d2, RC<T> d3, uint32_t ta,
                                         uint32_t tb) {
  constexpr int NR = 1 << R;
  T px[4], py[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    if ((RA < 0 && (s & 1)) || (RB < 0 && (s & 2))) continue;
    if (RA >= 0 && RB >= 0) {
      px[s] = (s == 3) ? d3.x : (s == 2) ? d2.x : (s == 1) ? d1.x : d0.x;
      py[s] = (s == 3) ? d3.y : (s == 2) ? d2.y : (s == 1) ? d1.y : d0.y;
    } else {
      // a per-lane choice: the phases go through registers first, so that it stays a chain of
      // lane selects (not a table in scratch memory indexed per lane)
      const uint32_t sa = (uint32_t)(s & 1) | ta, sb = (uint32_t)((s >> 1) & 1) | tb;
      T a0 = d0.x, a1 = d1.x, a2 = d2.x, a3 = d3.x, b0 = d0.y, b1 = d1.y, b2 = d2.y, b3 = d3.y;
      asm volatile("" : "+v"(a0), "+v"(a1), "+v"(a2), "+v"(a3), "+v"(b0), "+v"(b1), "+v"(b2), "+v"(b3));
      px[s] = sb ? (sa ? a3 : a2) : (sa ? a1 : a0);
      py[s] = sb ? (sa ? b3 : b2) : (sa ? b1 : b0);
    }
  }
#pragma unroll
  for (int i = 0; i < NR; ++i) {
    const int s = (RA >= 0 ? (i >> (RA >= 0 ? RA : 0)) & 1 : 0) + 2 * (RB >= 0 ? (i >> (RB >= 0 ? RB : 0)) & 1 : 0);
    if constexpr (REAL) {
      x[i].x *= px[s];
      x[i].y *= px[s];
    } else {
      const T xr = x[i].x, xi = x[i].y;
      x[i].x = px[s] * xr - py[s] * xi;
      x[i].y = px[s] * xi + py[s] * xr;
    }
  }
}

// The diagonal operations ph_diag[j0 .. j1) of a phase, all with real phases (REAL) or all with
// complex ones.
template <bool REAL, class T, int R>
__device__ __forceinline__ void phase_diagonals(const GatePass<T>& P, RC<T> (&x)[1 << R], uint32_t row_g, int j0,
                                                int j1) {
  using C = RC<T>;
  for (int j = j0; j < j1; ++j) {
    const int o = P.ph_diag[j];
    const T* u = P.coef + P.op_coef[o];
    // OP_DIAG1 / OP_DIAG2: the phases d[b_a + 2 b_b] (a one-qubit diagonal takes b_b = 0 and
    // lists its two phases twice)
    const bool two = (P.op_type[o] == OP_DIAG2);
    const C d0{u[0], u[1]}, d1{u[2], u[3]};
    const C d2 = two ? C{u[4], u[5]} : d0, d3 = two ? C{u[6], u[7]} : d1;
    const int code = P.op_code[o];
    const int ra = code / 5 - 1, rb = code % 5 - 1;
    const uint32_t ta = ra < 0 ? (row_g >> P.op_a[o]) & 1u : 0u;
    const uint32_t tb = (two && rb < 0) ? (row_g >> P.op_b[o]) & 1u : 0u;
    switch (code) {
      case 0: reg_diag<-1, -1, REAL, T, R>(x, d0, d1, d2, d3, ta, tb); break;
      case 5: reg_diag<0, -1, REAL, T, R>(x, d0, d1, d2, d3, ta, tb); break;
      case 10: reg_diag<1, -1, REAL, T, R>(x, d0, d1, d2, d3, ta, tb); break;
      case 15: reg_diag<2, -1, REAL, T, R>(x, d0, d1, d2, d3, ta, tb); break;
      case 20: reg_diag<3, -1, REAL, T, R>(x, d0, d1, d2, d3, ta, tb); break;
      case 7: reg_diag<0, 1, REAL, T, R>(x, d0, d1, d2, d3, ta, tb); break;
      case 8: reg_diag<0, 2, REAL, T, R>(x, d0, d1, d2, d3, ta, tb); break;
      case 9: reg_diag<0, 3, REAL, T, R>(x, d0, d1, d2, d3, ta, tb); break;
      case 13: reg_diag<1, 2, REAL, T, R>(x, d0, d1, d2, d3, ta, tb); break;
      case 14: reg_diag<1, 3, REAL, T, R>(x, d0, d1, d2, d3, ta, tb); break;
      default: reg_diag<2, 3, REAL, T, R>(x, d0, d1, d2, d3, ta, tb); break;
    }
  }
}

// Operations of phase ph on the registers (row_g: the row index of register 0, whose register
// bits are clear): a 2x2 gate on each register bit b < NG (the host puts the identity on the
// bits without a gate; NG < 4 leaves them out, for a last phase of NG gates), then the phase's
// diagonal operations (see GatePass).
template <class T, int R, int NG = 4>
__device__ __forceinline__ void phase_apply(const GatePass<T>& P, int ph, RC<T> (&x)[1 << R], uint32_t row_g) {
  static_assert(R == 4, "four register bits per phase");
  const uint32_t g01 = P.ph_gc[ph][0], g23 = P.ph_gc[ph][1];
  if constexpr (NG > 0) reg_1q<0, R, T>(x, P.coef + (g01 & 0xffffu));
  if constexpr (NG > 1) reg_1q<1, R, T>(x, P.coef + (g01 >> 16));
  if constexpr (NG > 2) reg_1q<2, R, T>(x, P.coef + (g23 & 0xffffu));
  if constexpr (NG > 3) reg_1q<3, R, T>(x, P.coef + (g23 >> 16));
  const uint32_t ut = P.ph_u[ph];
  if (ut & (1u << 16)) {
    // the product of the real diagonal operations on register bits only: one uniform real
    // phase per register, in place
    const T* uu = P.coef + (ut & 0xffffu);
#pragma unroll
    for (int i = 0; i < (1 << R); ++i) {
      x[i].x *= uu[i];
      x[i].y *= uu[i];
    }
  }
  const uint32_t ops = P.ph_ops[ph];
  const int j0 = (int)(ops & 255u), j1 = j0 + (int)((ops >> 8) & 255u), j2 = j1 + (int)((ops >> 16) & 255u);
  if (j1 > j0) phase_diagonals<true, T, R>(P, x, row_g, j0, j1);
  if (j2 > j1) phase_diagonals<false, T, R>(P, x, row_g, j1, j2);
}

// One phase's register <-> LDS exchange: the registers go to the tile in the current layout and
// come back in phase ph's.
template <class T, int R>
__device__ __forceinline__ void phase_exchange(const GatePass<T>& P, int ph, RC<T> (&x)[1 << R], cx_t<T>* tile,
                                               int cshift, uint32_t te, bool first, uint32_t& pos, uint32_t& sub,
                                               uint32_t (&sh_pos)[R], uint32_t (&sh_row)[R]) {
  constexpr int NR = 1 << R;
  if (!first) __syncthreads();   // the previous exchange's reads are done
#pragma unroll
  for (int i = 0; i < NR; ++i) {
    cx_t<T> v;
    v.x = x[i].x;
    v.y = x[i].y;
    tile[pos | pick_or<R>(i, sh_pos)] = v;
  }
  __syncthreads();
  phase_layout<T, R>(P, ph, cshift, te, pos, sub, sh_pos, sh_row);
#pragma unroll
  for (int i = 0; i < NR; ++i) {
    const cx_t<T> v = tile[pos | pick_or<R>(i, sh_pos)];
    x[i] = RC<T>{v.x, v.y};
  }
}

// Apply the pass's operations phase by phase in registers, one tile: phase 0 reads from HBM and
// the last phase writes to HBM (lanes run along the columns of a row); before every later phase
// the registers go through LDS into that phase's layout.  NPH > 0: the pass has exactly NPH
// phases (unrolled), the last of them applying GL gates; 0: any number.  Threads beyond the
// 2^(E - R) distinct register groups repeat a group (their LDS writes are the same values) and
// do not store, so that every thread runs the same code and reaches every barrier.
template <class T, int R, int NPH, int GL = 4>
__device__ __forceinline__ void gate_phases(const GatePass<T>& P, cx_t<T>* __restrict__ L, size_t ld,
                                            cx_t<T>* tile, int cshift, uint32_t base) {
  constexpr int NR = 1 << R;
  const int E = P.k + cshift;
  const uint32_t groups = 1u << (E - R);
  const uint32_t te = threadIdx.x & (groups - 1u);
  RC<T> x[NR];
  uint32_t pos = 0, sub = 0, sh_pos[R], sh_row[R];
  phase_layout<T, R>(P, 0, cshift, te, pos, sub, sh_pos, sh_row);
  {
    const uint32_t col = pos & ((1u << cshift) - 1u);
    const cx_t<T>* tp = L + (size_t)(base | sub) * ld + col;   // row offsets below are uniform
#pragma unroll
    for (int i = 0; i < NR; ++i) x[i] = ld_nt<T>(tp + (size_t)pick_or<R>(i, sh_row) * ld);
  }
  if constexpr (NPH > 0) {
#pragma unroll
    for (int ph = 0; ph < NPH; ++ph) {
      if (ph > 0) phase_exchange<T, R>(P, ph, x, tile, cshift, te, ph == 1, pos, sub, sh_pos, sh_row);
      if (ph + 1 < NPH)
        phase_apply<T, R>(P, ph, x, base | sub);
      else
        phase_apply<T, R, GL>(P, ph, x, base | sub);
    }
  } else {
    for (int ph = 0; ph < P.n_phases; ++ph) {
      if (ph > 0) phase_exchange<T, R>(P, ph, x, tile, cshift, te, ph == 1, pos, sub, sh_pos, sh_row);
      phase_apply<T, R>(P, ph, x, base | sub);
    }
  }
  if (threadIdx.x < groups) {
    const uint32_t col = pos & ((1u << cshift) - 1u);
    cx_t<T>* tp = L + (size_t)(base | sub) * ld + col;
#pragma unroll
    for (int i = 0; i < NR; ++i) st_nt<T>(tp + (size_t)pick_or<R>(i, sh_row) * ld, x[i]);
  }
}

// Row index of the tile's first row: the tile index deposited into the non-local bit positions
// (ascending local qubits).
template <class T>
__device__ __forceinline__ uint32_t tile_base(const GatePass<T>& P, uint32_t tile_index) {
  uint32_t base = tile_index;
  for (int j = 0; j < P.k; ++j) {
    const int p = P.sorted_q[j];
    base = ((base >> p) << (p + 1)) | (base & ((1u << p) - 1u));
  }
  return base;
}

// One LDS sweep per operation over the tile (passes without register phases).
template <class T>
__device__ __forceinline__ void gate_sweep_body(const GatePass<T>& P, cx_t<T>* __restrict__ L, int cshift,
                                                uint32_t base) {
  using C = cx_t<T>;
  extern __shared__ __attribute__((aligned(16))) unsigned char gate_smem[];
  C* tile = reinterpret_cast<C*>(gate_smem);   // [2^k][ncols]
  __shared__ uint32_t slot_off[256];           // row offset of tile slot i (local bits of i)
  const int k = P.k, nc = P.ncols, tid = threadIdx.x;
  const size_t ld = (size_t)P.ld;
  if (tid < (1 << k)) {
    uint32_t off = 0;
    for (int j = 0; j < k; ++j) off |= ((uint32_t)(tid >> j) & 1u) << P.local_q[j];
    slot_off[tid] = off;
  }
  __syncthreads();
  const int elems = nc << k;
  // HBM -> LDS with 16-byte accesses, kUnroll loads in flight per thread before the LDS writes
  constexpr int CPU = 16 / (int)sizeof(C);   // complex values per 16-byte unit
  constexpr int kUnroll = 16;
  const int units = elems / CPU;
  for (int u0 = 0; u0 < units; u0 += kGateThreads * kUnroll) {
    f4v buf[kUnroll];
#pragma unroll
    for (int j = 0; j < kUnroll; ++j) {
      const int uu = u0 + j * kGateThreads + tid;
      if (uu < units) {
        const int e = uu * CPU;
        const uint32_t i = (uint32_t)e >> cshift;
        const int v = e & (nc - 1);
        buf[j] = *reinterpret_cast<const f4v*>(L + (size_t)(base | slot_off[i]) * ld + v);
      }
    }
#pragma unroll
    for (int j = 0; j < kUnroll; ++j) {
      const int uu = u0 + j * kGateThreads + tid;
      if (uu < units) *reinterpret_cast<f4v*>(tile + uu * CPU) = buf[j];
    }
  }
  __syncthreads();

  for (int o = 0; o < P.n_ops; ++o) {
    const T* u = P.coef + P.op_coef[o];
    const int ty = P.op_type[o];
    if (ty == OP_1Q) {
      const int j = P.op_a[o];
      const C u00 = cmk<C, T>(u[0], u[1]), u01 = cmk<C, T>(u[2], u[3]);
      const C u10 = cmk<C, T>(u[4], u[5]), u11 = cmk<C, T>(u[6], u[7]);
#pragma unroll 4
      for (int e = tid; e < (elems >> 1); e += kGateThreads) {
        const int v = e & (nc - 1);
        const uint32_t i0 = insert_zero((uint32_t)e >> cshift, j), i1 = i0 | (1u << j);
        C& a0 = tile[(i0 << cshift) + v];
        C& a1 = tile[(i1 << cshift) + v];
        const C x0 = a0, x1 = a1;
        a0 = cadd(cmul(u00, x0), cmul(u01, x1));
        a1 = cadd(cmul(u10, x0), cmul(u11, x1));
      }
    } else if (ty == OP_2Q) {
      const int ja = P.op_a[o], jb = P.op_b[o];
      const int jlo = ja < jb ? ja : jb, jhi = ja < jb ? jb : ja;
#pragma unroll 2
      for (int e = tid; e < (elems >> 2); e += kGateThreads) {
        const int v = e & (nc - 1);
        const uint32_t i00 = insert_zero(insert_zero((uint32_t)e >> cshift, jlo), jhi);
        const uint32_t idx[4] = {i00, i00 | (1u << ja), i00 | (1u << jb), i00 | (1u << ja) | (1u << jb)};
        C x[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) x[m] = tile[(idx[m] << cshift) + v];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          C acc = cmul(cmk<C, T>(u[8 * r], u[8 * r + 1]), x[0]);
#pragma unroll
          for (int m = 1; m < 4; ++m) acc = cadd(acc, cmul(cmk<C, T>(u[8 * r + 2 * m], u[8 * r + 2 * m + 1]), x[m]));
          tile[(idx[r] << cshift) + v] = acc;
        }
      }
    } else {
      // diagonal in the computational basis: phase from the full row index
      const int qa = P.op_a[o], qb = P.op_b[o];
      for (int e = tid; e < elems; e += kGateThreads) {
        const uint32_t x = base | slot_off[(uint32_t)e >> cshift];
        int sel;
        if (ty == OP_DIAG1)
          sel = (int)((x >> qa) & 1u);
        else if (ty == OP_DIAG2)
          sel = (int)((x >> qa) & 1u) | ((int)((x >> qb) & 1u) << 1);
        else
          sel = __popc(x);
        tile[e] = cmul(cmk<C, T>(u[2 * sel], u[2 * sel + 1]), tile[e]);
      }
    }
    __syncthreads();
  }
  for (int u0 = 0; u0 < units; u0 += kGateThreads * kUnroll) {
    f4v buf[kUnroll];
#pragma unroll
    for (int j = 0; j < kUnroll; ++j) {
      const int uu = u0 + j * kGateThreads + tid;
      if (uu < units) buf[j] = *reinterpret_cast<const f4v*>(tile + uu * CPU);
    }
#pragma unroll
    for (int j = 0; j < kUnroll; ++j) {
      const int uu = u0 + j * kGateThreads + tid;
      if (uu < units) {
        const int e = uu * CPU;
        const uint32_t i = (uint32_t)e >> cshift;
        const int v = e & (nc - 1);
        *reinterpret_cast<f4v*>(L + (size_t)(base | slot_off[i]) * ld + v) = buf[j];
      }
    }
  }
}

template <class T>
__device__ __forceinline__ void gate_phase_body(const GatePass<T>& P, cx_t<T>* __restrict__ L, int cshift,
                                                uint32_t base, int nph) {
  extern __shared__ __attribute__((aligned(16))) unsigned char gate_smem[];
  cx_t<T>* tile = reinterpret_cast<cx_t<T>*>(gate_smem);
  const size_t ld = (size_t)P.ld;
  switch (nph) {
    case 1: gate_phases<T, 4, 1>(P, L, ld, tile, cshift, base); break;
    case 2: gate_phases<T, 4, 2>(P, L, ld, tile, cshift, base); break;
    case 3: gate_phases<T, 4, 3>(P, L, ld, tile, cshift, base); break;
    default: gate_phases<T, 4, 0>(P, L, ld, tile, cshift, base); break;
  }
}

// Passes without register phases: one LDS sweep per operation.
template <class T>
__global__ __launch_bounds__(kGateThreads) void gate_pass_kernel(const GatePass<T> P, cx_t<T>* __restrict__ L,
                                                        int cshift) {
  gate_sweep_body<T>(P, L, cshift, tile_base(P, blockIdx.x));
}

// Register-phase passes, one kernel per phase count NPH (1 .. 3; 0: any), so that each unrolls
// its phases, and (wide passes) per gate count GL of the last phase.  SPLIT: the columns of a
// wide factor are split in two, a work-group owns one half of a tile's columns (the gates act on
// rows only) with 256 threads and half the LDS, so that five work-groups share a CU.
//
// Work-group order: work-groups go round-robin over the 8 XCDs.  A wide pass whose local qubits
// include qubit 0 has tiles of consecutive row pairs; those run faster when each XCD takes one
// contiguous eighth of the work-groups (xcd_ranges: 185 against 193 us for a pass over 2^20 x 64
// complex64), while tiles spread over high row bits run faster in plain order (187 against 202).
template <class T, int NPH, bool SPLIT, int GL>
__global__ __launch_bounds__(SPLIT ? kGateThreads / 2 : kGateThreads, SPLIT ? 4 : 1) void gate_phase_kernel(
    const GatePass<T> pass, cx_t<T>* __restrict__ L, int cshift, int xcd_ranges) {
  // read the pass where the launch put it (the first kernel argument): uniform scalar loads,
  // never a private copy of the whole structure
  (void)pass;
  const GatePass<T>& P = *(const GatePass<T>*)__builtin_amdgcn_kernarg_segment_ptr();
  extern __shared__ __attribute__((aligned(16))) unsigned char gate_smem[];
  cx_t<T>* tile = reinterpret_cast<cx_t<T>*>(gate_smem);
  const uint32_t W = gridDim.x, b = blockIdx.x;
  const uint32_t g = (xcd_ranges && W % 8u == 0u) ? (b % 8u) * (W / 8u) + b / 8u : b;
  const uint32_t half = SPLIT ? (g & 1u) : 0u;
  const uint32_t t = SPLIT ? (g >> 1) : g;
  gate_phases<T, 4, NPH, GL>(P, L + (size_t)half * (1u << cshift), (size_t)P.ld, tile, cshift, tile_base(P, t));
}

template <class T>
__global__ __launch_bounds__(kGateThreads) void gate_pass_batched(const GateJob<T>* __restrict__ jobs, int njobs) {
  const int j = find_job(jobs, njobs, blockIdx.x);
  const GatePass<T>& P = jobs[j].p;
  const uint32_t base = tile_base(P, blockIdx.x - jobs[j].block0);
  if (P.n_phases > 0)
    gate_phase_body<T>(P, jobs[j].L, jobs[j].cshift, base, P.n_phases);
  else
    gate_sweep_body<T>(P, jobs[j].L, jobs[j].cshift, base);
}

size_t gate_pass_shm(int ncols, int k, size_t csize, int n_phases) {
  return (n_phases == 1) ? 0 : ((size_t)ncols << k) * csize;
}

template <class T>
hipError_t launch_gate_pass_batched(const GateJob<T>* jobs, int njobs, uint32_t blocks, size_t shm,
                                    hipStream_t s) {
  if (njobs < 1 || blocks < 1 || shm > 65536) return hipErrorInvalidValue;
  hipLaunchKernelGGL(gate_pass_batched<T>, dim3(blocks), dim3(kGateThreads), shm, s, jobs, njobs);
  return hipGetLastError();
}

template <class T>
hipError_t launch_gate_pass(const GatePass<T>& p, cx_t<T>* L, hipStream_t s) {
  if (p.ncols < 1 || (p.ncols & (p.ncols - 1)) || p.k < 0 || p.k > 8 || p.k > p.n)
    return hipErrorInvalidValue;
  int cshift = 0;
  while ((1 << cshift) < p.ncols) ++cshift;
  const size_t shm = gate_pass_shm(p.ncols, p.k, sizeof(cx_t<T>), p.n_phases);
  if (shm > 65536) return hipErrorInvalidValue;
  const uint32_t tiles = 1u << (p.n - p.k);
  if (p.n_phases > 0) {
    // passes with several operations split wide factors (a lone gate streams slightly faster
    // unsplit); the complex128 phases need more than 128 registers, so they stay unsplit
    const bool split = sizeof(T) == 4 && p.n_ops > 2 && p.ncols >= 64 && p.k + cshift - 1 >= 8;
    const int cs = split ? cshift - 1 : cshift;
    // each thread holds 16 elements: 2^(k + cs) = 16 * threads at most
    if (p.k + cs - 4 > (split ? 8 : 9)) return hipErrorInvalidValue;
    const dim3 grid(split ? 2 * tiles : tiles), block(split ? kGateThreads / 2 : kGateThreads);
    const size_t sh = split ? shm / 2 : shm;
    const int xcd_ranges = (split && p.k > 0 && p.sorted_q[0] == 0) ? 1 : 0;
    auto go = [&](auto kernel) { hipLaunchKernelGGL(kernel, grid, block, sh, s, p, L, cs, xcd_ranges); };
    if constexpr (sizeof(T) == 4) {
      if (split && p.n_phases >= 1 && p.n_phases <= 3) {
        const int gl = std::min(std::max(p.last_gates, 0), 4);
#define LRDM_SPLIT_GL(NPH)                                      \
  switch (gl) {                                                 \
    case 0: go(gate_phase_kernel<T, NPH, true, 0>); break;      \
    case 1: go(gate_phase_kernel<T, NPH, true, 1>); break;      \
    case 2: go(gate_phase_kernel<T, NPH, true, 2>); break;      \
    case 3: go(gate_phase_kernel<T, NPH, true, 3>); break;      \
    default: go(gate_phase_kernel<T, NPH, true, 4>); break;     \
  }
        switch (p.n_phases) {
          case 1: LRDM_SPLIT_GL(1); break;
          case 2: LRDM_SPLIT_GL(2); break;
          default: LRDM_SPLIT_GL(3); break;
        }
#undef LRDM_SPLIT_GL
        return hipGetLastError();
      }
      if (split) {
        go(gate_phase_kernel<T, 0, true, 4>);
        return hipGetLastError();
      }
    }
    switch (p.n_phases) {
      case 1: go(gate_phase_kernel<T, 1, false, 4>); break;
      case 2: go(gate_phase_kernel<T, 2, false, 4>); break;
      case 3: go(gate_phase_kernel<T, 3, false, 4>); break;
      default: go(gate_phase_kernel<T, 0, false, 4>); break;
    }
    return hipGetLastError();
  }
  hipLaunchKernelGGL(gate_pass_kernel<T>, dim3(tiles), dim3(kGateThreads), shm, s, p, L, cshift);
  return hipGetLastError();
}

// Plain-form Kraus concatenation (Eq. "low rank evolution K"): for every row pair
// (x0, x1) = (bit q clear, bit q set) and column v < c, column a*c + v of row x_b' becomes
// sum_b E_a[b'][b] L[x_b][v].  Each thread reads its two inputs before writing, and no other
// thread touches them, so the expansion is done in place inside the ld-wide rows.
template <class T>
__global__ __launch_bounds__(256) void kraus_expand_kernel(cx_t<T>* __restrict__ L, uint32_t half_rows,
                                                           int ld, int c, int q, Channel ch,
                                                           int m_pad) {
  using C = cx_t<T>;
  const uint64_t gid = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  const uint32_t y = (uint32_t)(gid / (uint64_t)c);
  const int v = (int)(gid % (uint64_t)c);
  if (y >= half_rows) return;
  const uint32_t lo = y & ((1u << q) - 1u);
  const uint32_t x0 = ((y >> q) << (q + 1)) | lo, x1 = x0 | (1u << q);
  const C l0 = L[(size_t)x0 * ld + v], l1 = L[(size_t)x1 * ld + v];
  for (int a = 0; a < m_pad; ++a) {
    if (a >= ch.m) {   // unused Kraus slots of the padded column blocks
      L[(size_t)x0 * ld + a * c + v] = cmk<C, T>((T)0, (T)0);
      L[(size_t)x1 * ld + a * c + v] = cmk<C, T>((T)0, (T)0);
      continue;
    }
    for (int bp = 0; bp < 2; ++bp) {
      const C e0 = cmk<C, T>((T)ch.e[a][bp][0][0], (T)ch.e[a][bp][0][1]);
      const C e1 = cmk<C, T>((T)ch.e[a][bp][1][0], (T)ch.e[a][bp][1][1]);
      const C r = cadd(cmul(e0, l0), cmul(e1, l1));
      L[(size_t)(bp ? x1 : x0) * ld + a * c + v] = r;
    }
  }
}

template <class T>
hipError_t launch_kraus_expand(cx_t<T>* L, int n, int ld, int c, int q, const Channel& ch,
                               int m_pad, hipStream_t s) {
  const uint64_t total = (uint64_t)(1u << (n - 1)) * (uint64_t)c;
  const uint32_t blocks = (uint32_t)((total + 255) / 256);
  hipLaunchKernelGGL(kraus_expand_kernel<T>, dim3(blocks), dim3(256), 0, s, L, 1u << (n - 1), ld,
                     c, q, ch, m_pad);
  return hipGetLastError();
}

// Plain-form expansion of a two-qubit channel (Sec. II.C) on (q0, q1): for the row quad x_b,
// b = b(q0) + 2 b(q1), and column v < c, column a c + v of row x_b' becomes
// sum_b E_a[b'][b] L[x_b][v] for the operators a0 <= a < a0 + na of this launch (a >= m: zero
// padding).  Every launch reads columns 0 .. c - 1 and the launch holding a = 0, which
// overwrites them, comes last; one thread owns one (quad, column) pair.
template <class T>
__global__ __launch_bounds__(256) void kraus2_expand_kernel(cx_t<T>* __restrict__ L, uint32_t quarter_rows, int ld,
                                                            int c, int q0, int q1, Kraus2Chunk ck) {
  using C = cx_t<T>;
  const uint64_t gid = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  const uint32_t y = (uint32_t)(gid / (uint64_t)c);
  const int v = (int)(gid % (uint64_t)c);
  if (y >= quarter_rows) return;
  const int lo = q0 < q1 ? q0 : q1, hi = q0 < q1 ? q1 : q0;
  const uint32_t t = ((y >> lo) << (lo + 1)) | (y & ((1u << lo) - 1u));
  const uint32_t x0 = ((t >> hi) << (hi + 1)) | (t & ((1u << hi) - 1u));
  uint32_t xb[4];
  C l[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    xb[b] = x0 | ((uint32_t)(b & 1) << q0) | ((uint32_t)(b >> 1) << q1);
    l[b] = L[(size_t)xb[b] * ld + v];
  }
  for (int u = 0; u < ck.na; ++u) {
    const int a = ck.a0 + u;
#pragma unroll
    for (int bp = 0; bp < 4; ++bp) {
      C r = cmk<C, T>((T)0, (T)0);
      if (a < ck.m) {
#pragma unroll
        for (int b = 0; b < 4; ++b)
          r = cadd(r, cmul(cmk<C, T>((T)ck.e[u][bp][b][0], (T)ck.e[u][bp][b][1]), l[b]));
      }
      L[(size_t)xb[bp] * ld + a * c + v] = r;
    }
  }
}

template <class T>
hipError_t launch_kraus2_expand(cx_t<T>* L, int n, int ld, int c, int q0, int q1, const Kraus2Chunk& ck,
                                hipStream_t s) {
  if (n < 2 || c < 1) return hipErrorInvalidValue;
  const uint64_t total = (uint64_t)(1u << (n - 2)) * (uint64_t)c;
  const uint32_t blocks = (uint32_t)((total + 255) / 256);
  hipLaunchKernelGGL(kraus2_expand_kernel<T>, dim3(blocks), dim3(256), 0, s, L, 1u << (n - 2), ld, c, q0, q1, ck);
  return hipGetLastError();
}

template <class T>
__global__ void set_e0_kernel(cx_t<T>* L) {
  L[0].x = (T)1;
  L[0].y = (T)0;
}

template <class T>
hipError_t launch_set_e0(cx_t<T>* L, hipStream_t s) {
  hipLaunchKernelGGL(set_e0_kernel<T>, dim3(1), dim3(1), 0, s, L);
  return hipGetLastError();
}

// State reset of many handles: zero the factor and the compression record, L[0][0] = 1.
__global__ __launch_bounds__(256) void reset_batched(const ResetJob* __restrict__ jobs, int njobs,
                                                     int complex_bytes) {
  const int j = find_job(jobs, njobs, blockIdx.x);
  const ResetJob& J = jobs[j];
  const uint64_t words = J.state_bytes / 16;
  uint4* st = static_cast<uint4*>(J.state);
  for (uint64_t w = (uint64_t)(blockIdx.x - J.block0) * 256 + threadIdx.x; w < words;
       w += (uint64_t)J.nblocks * 256)
    st[w] = make_uint4(0u, 0u, 0u, 0u);
  if (blockIdx.x == J.block0 && threadIdx.x == 0) {
    DevInfo zero{};
    *J.info = zero;
  }
  __syncthreads();
  if (blockIdx.x == J.block0 && threadIdx.x == 0) {
    if (complex_bytes == 8) {
      static_cast<float2*>(J.state)[0] = make_float2(1.f, 0.f);
    } else {
      static_cast<double2*>(J.state)[0] = make_double2(1.0, 0.0);
    }
  }
}

hipError_t launch_reset_batched(const ResetJob* jobs, int njobs, uint32_t blocks, int complex_bytes,
                                hipStream_t s) {
  if (njobs < 1 || blocks < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(reset_batched, dim3(blocks), dim3(256), 0, s, jobs, njobs, complex_bytes);
  return hipGetLastError();
}

// Device wall clock (constant-rate counter) into one slot: per-step completion times of a
// captured batch.
__global__ void stamp_kernel(uint64_t* slot) { *slot = wall_clock64(); }

hipError_t launch_stamp(uint64_t* slot, hipStream_t s) {
  hipLaunchKernelGGL(stamp_kernel, dim3(1), dim3(1), 0, s, slot);
  return hipGetLastError();
}

template hipError_t launch_gate_pass_batched<float>(const GateJob<float>*, int, uint32_t, size_t, hipStream_t);
template hipError_t launch_gate_pass_batched<double>(const GateJob<double>*, int, uint32_t, size_t, hipStream_t);
template hipError_t launch_kraus2_expand<float>(float2*, int, int, int, int, int, const Kraus2Chunk&, hipStream_t);
template hipError_t launch_kraus2_expand<double>(double2*, int, int, int, int, int, const Kraus2Chunk&, hipStream_t);
template hipError_t launch_gate_pass<float>(const GatePass<float>&, float2*, hipStream_t);
template hipError_t launch_gate_pass<double>(const GatePass<double>&, double2*, hipStream_t);
template hipError_t launch_kraus_expand<float>(float2*, int, int, int, int, const Channel&, int, hipStream_t);
template hipError_t launch_kraus_expand<double>(double2*, int, int, int, int, const Channel&, int, hipStream_t);
template hipError_t launch_set_e0<float>(float2*, hipStream_t);
template hipError_t launch_set_e0<double>(double2*, hipStream_t);

}  // namespace lrdm
