// Full-rank density-matrix evolution (Eq. "full rank evolution", Sec. II.A), the same-GPU
// comparator of the low-rank path.  rho (2^n x 2^n complex64, row-major) is treated as a vector
// over 2n index bits: bit q of the column index y is index bit q, bit q of the row index x is
// index bit n + q.  U rho U^H applies U to the row bits and conj(U) to the column bits; a channel
// sum_a E_a rho E_a^H applies the 4x4 superoperator S = sum_a E_a (x) conj(E_a) to the bit pair
// (n + q, q).
//
// A pass stages a tile of 2^k amplitudes (k <= 13, 64 KB) in LDS: index bits 0..4 are always
// local, so every global access is a contiguous 256-byte run, plus up to 8 further bits on which
// the pass's operations act.  Diagonal operations use the full index and act on any bit.
#include "lrdm_internal.h"

namespace lrdm {

typedef float fv4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float2 fmulc(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 faddc(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ uint32_t ins0(uint32_t p, int j) {
  return ((p >> j) << (j + 1)) | (p & ((1u << j) - 1u));
}

__global__ __launch_bounds__(256) void fdm_pass_kernel(const FdmPass P, float2* __restrict__ rho) {
  extern __shared__ __attribute__((aligned(16))) unsigned char fdm_smem[];
  float2* tile = reinterpret_cast<float2*>(fdm_smem);   // [2^k]
  __shared__ uint32_t hi_off[256];                       // offset of the non-low local bits
  const int k = P.k, tid = threadIdx.x;
  const int lo = k < kFdmLowBits ? k : kFdmLowBits;
  const int kh = k - lo;
  if (tid < (1 << kh)) {
    uint32_t off = 0;
    for (int j = 0; j < kh; ++j) off |= ((uint32_t)(tid >> j) & 1u) << P.local_q[lo + j];
    hi_off[tid] = off;
  }
  __syncthreads();
  // deposit the tile index into the non-local bit positions (local bits in ascending order)
  uint32_t base = blockIdx.x;
  for (int j = 0; j < lo; ++j) base = ins0(base, j);
  for (int j = 0; j < kh; ++j) base = ins0(base, P.sorted_hi[j]);
  const int elems = 1 << k;
  const int lomask = (1 << lo) - 1;
  constexpr int kUnroll = 8;
  if (lo >= 1) {
    // two complex64 per 16-byte unit; units never straddle the contiguous low block
    const int units = elems >> 1;
    for (int u0 = 0; u0 < units; u0 += 256 * kUnroll) {
      fv4 buf[kUnroll];
#pragma unroll
      for (int j = 0; j < kUnroll; ++j) {
        const int uu = u0 + j * 256 + tid;
        if (uu < units) {
          const int e = uu * 2;
          buf[j] = *reinterpret_cast<const fv4*>(rho + (size_t)(base | hi_off[e >> lo] | (uint32_t)(e & lomask)));
        }
      }
#pragma unroll
      for (int j = 0; j < kUnroll; ++j) {
        const int uu = u0 + j * 256 + tid;
        if (uu < units) *reinterpret_cast<fv4*>(tile + uu * 2) = buf[j];
      }
    }
  } else {
    for (int e = tid; e < elems; e += 256) tile[e] = rho[base | hi_off[e]];
  }
  __syncthreads();

  for (int o = 0; o < P.n_ops; ++o) {
    const float* u = P.coef + P.op_coef[o];
    const int ty = P.op_type[o];
    if (ty == OP_1Q) {
      const int j = P.op_a[o];
      const float2 u00 = make_float2(u[0], u[1]), u01 = make_float2(u[2], u[3]);
      const float2 u10 = make_float2(u[4], u[5]), u11 = make_float2(u[6], u[7]);
#pragma unroll 4
      for (int e = tid; e < (elems >> 1); e += 256) {
        const uint32_t i0 = ins0((uint32_t)e, j), i1 = i0 | (1u << j);
        const float2 x0 = tile[i0], x1 = tile[i1];
        tile[i0] = faddc(fmulc(u00, x0), fmulc(u01, x1));
        tile[i1] = faddc(fmulc(u10, x0), fmulc(u11, x1));
      }
    } else if (ty == OP_2Q) {
      const int ja = P.op_a[o], jb = P.op_b[o];
      const int jlo = ja < jb ? ja : jb, jhi = ja < jb ? jb : ja;
#pragma unroll 2
      for (int e = tid; e < (elems >> 2); e += 256) {
        const uint32_t i00 = ins0(ins0((uint32_t)e, jlo), jhi);
        const uint32_t idx[4] = {i00, i00 | (1u << ja), i00 | (1u << jb), i00 | (1u << ja) | (1u << jb)};
        float2 x[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) x[m] = tile[idx[m]];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          float2 acc = fmulc(make_float2(u[8 * r], u[8 * r + 1]), x[0]);
#pragma unroll
          for (int m = 1; m < 4; ++m) acc = faddc(acc, fmulc(make_float2(u[8 * r + 2 * m], u[8 * r + 2 * m + 1]), x[m]));
          tile[idx[r]] = acc;
        }
      }
    } else {
      // diagonal in the computational basis of the 2n index bits
      const int qa = P.op_a[o], qb = P.op_b[o];
      for (int e = tid; e < elems; e += 256) {
        const uint32_t x = base | hi_off[e >> lo] | (uint32_t)(e & lomask);
        int sel = (int)((x >> qa) & 1u);
        if (ty == OP_DIAG2) sel |= (int)((x >> qb) & 1u) << 1;
        tile[e] = fmulc(make_float2(u[2 * sel], u[2 * sel + 1]), tile[e]);
      }
    }
    __syncthreads();
  }

  if (lo >= 1) {
    const int units = elems >> 1;
    for (int u0 = 0; u0 < units; u0 += 256 * kUnroll) {
      fv4 buf[kUnroll];
#pragma unroll
      for (int j = 0; j < kUnroll; ++j) {
        const int uu = u0 + j * 256 + tid;
        if (uu < units) buf[j] = *reinterpret_cast<const fv4*>(tile + uu * 2);
      }
#pragma unroll
      for (int j = 0; j < kUnroll; ++j) {
        const int uu = u0 + j * 256 + tid;
        if (uu < units) {
          const int e = uu * 2;
          *reinterpret_cast<fv4*>(rho + (size_t)(base | hi_off[e >> lo] | (uint32_t)(e & lomask))) = buf[j];
        }
      }
    }
  } else {
    for (int e = tid; e < elems; e += 256) rho[base | hi_off[e]] = tile[e];
  }
}

// ---------------------------------------------------------------- register-phase passes
// Full tiles (kFdmMaxLocal = 13 bits, 64 KB): 512 threads hold 16 elements each, the elements
// that differ in the current phase's 4 register slots; 1- and 2-bit operators on those slots are
// register arithmetic, diagonal operators use the full index.  Phase 0 loads from HBM, the last
// phase stores to HBM (non-temporal accesses; lanes run along the low, contiguous bits), and
// consecutive phases exchange the tile through LDS.
constexpr int kFdmThreads = 512;

struct FC {
  float x, y;
};
typedef float f2v __attribute__((ext_vector_type(2)));

__device__ __forceinline__ FC fcmac(FC acc, float ur, float ui, FC a) {
  return FC{fmaf(ur, a.x, fmaf(-ui, a.y, acc.x)), fmaf(ur, a.y, fmaf(ui, a.x, acc.y))};
}

// The coefficients are read once per operation into registers: after full unrolling a
// pointer into the pass argument would have hundreds of users, enough that the compiler
// stops reading the argument in place and copies it to the stack.
template <int N>
__device__ __forceinline__ void fdm_coef(const float* u, float (&c)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) c[i] = u[i];
}

template <int B>
__device__ __forceinline__ void fdm_reg_1q(FC (&x)[16], const float (&u)[8]) {
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    if (!(i & (1 << B))) {
      const FC a = x[i], b = x[i | (1 << B)];
      x[i] = fcmac(fcmac(FC{0.f, 0.f}, u[0], u[1], a), u[2], u[3], b);
      x[i | (1 << B)] = fcmac(fcmac(FC{0.f, 0.f}, u[4], u[5], a), u[6], u[7], b);
    }
  }
}

// 4 x 4 operator (row-major, element t = bit RA + 2 bit RB) on register bits RA < RB
template <int RA, int RB>
__device__ __forceinline__ void fdm_reg_2q(FC (&x)[16], const float (&u)[32]) {
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    if (!(i & (1 << RA)) && !(i & (1 << RB))) {
      const int idx[4] = {i, i | (1 << RA), i | (1 << RB), i | (1 << RA) | (1 << RB)};
      FC e[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) e[m] = x[idx[m]];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        FC acc{0.f, 0.f};
#pragma unroll
        for (int m = 0; m < 4; ++m) acc = fcmac(acc, u[8 * r + 2 * m], u[8 * r + 2 * m + 1], e[m]);
        x[idx[r]] = acc;
      }
    }
  }
}

__device__ __forceinline__ uint32_t fpick(int i, const uint32_t (&v)[4]) {
  uint32_t r = 0;
#pragma unroll
  for (int b = 0; b < 4; ++b)
    if (i & (1 << b)) r |= v[b];
  return r;
}

// complex scale of one element; REAL: the imaginary part of the coefficient is zero
template <bool REAL>
__device__ __forceinline__ FC fscale(FC a, float cr, float ci) {
  if (REAL) return FC{cr * a.x, cr * a.y};
  return FC{fmaf(cr, a.x, -ci * a.y), fmaf(cr, a.y, ci * a.x)};
}

// diagonal operator whose operands are register bits RA (< RB), or no register bit (-1); the
// per-thread coefficients c0..c3 already account for the operands that are thread or tile bits
template <int RA, int RB, bool REAL>
__device__ __forceinline__ void fdm_reg_diag(FC (&x)[16], const float (&c)[8]) {
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    int s = 0;
    if (RA >= 0) s |= (i >> RA) & 1;
    if (RB >= 0) s |= ((i >> RB) & 1) << 1;
    x[i] = fscale<REAL>(x[i], c[2 * s], c[2 * s + 1]);
  }
}

// pick per lane one of two complex coefficients
__device__ __forceinline__ void fsel2(bool hi, float r0, float i0, float r1, float i1, float& r, float& i) {
  r = hi ? r1 : r0;
  i = hi ? i1 : i0;
}

template <bool REAL>
__device__ __forceinline__ void fdm_diag_dispatch(FC (&x)[16], int key, const float (&c)[8]) {
  switch (key) {
    case 0: fdm_reg_diag<-1, -1, REAL>(x, c); break;
    case 1: fdm_reg_diag<0, -1, REAL>(x, c); break;
    case 2: fdm_reg_diag<1, -1, REAL>(x, c); break;
    case 3: fdm_reg_diag<2, -1, REAL>(x, c); break;
    case 4: fdm_reg_diag<3, -1, REAL>(x, c); break;
    case 5 + 1: fdm_reg_diag<0, 1, REAL>(x, c); break;
    case 5 + 2: fdm_reg_diag<0, 2, REAL>(x, c); break;
    case 5 + 3: fdm_reg_diag<0, 3, REAL>(x, c); break;
    case 5 + 4 + 2: fdm_reg_diag<1, 2, REAL>(x, c); break;
    case 5 + 4 + 3: fdm_reg_diag<1, 3, REAL>(x, c); break;
    default: fdm_reg_diag<2, 3, REAL>(x, c); break;
  }
}

// register layout of phase ph (pos: tile offset of register 0, g: its global index)
__device__ __forceinline__ void fdm_layout(const FdmPass& P, int ph, uint32_t base, const uint32_t* hi_off,
                                           uint32_t& pos, uint32_t& g, uint32_t (&sh_pos)[4],
                                           uint32_t (&goff)[4]) {
  constexpr int lo = kFdmLowBits, K = kFdmMaxLocal;
  const int tid = threadIdx.x;
  uint32_t rmask = 0;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int slot = P.ph_slots[ph][b];
    sh_pos[b] = 1u << slot;
    goff[b] = 1u << P.local_q[slot];
    rmask |= sh_pos[b];
  }
  const uint32_t tmask = ((1u << K) - 1u) & ~rmask;
  uint32_t p = 0;
  int src = 0;
  for (int q = 0; q < K; ++q)
    if ((tmask >> q) & 1u) {
      p |= ((uint32_t)(tid >> src) & 1u) << q;
      ++src;
    }
  pos = p;
  g = base | (p & ((1u << lo) - 1u)) | hi_off[p >> lo];
}

__device__ __forceinline__ void fdm_apply(const FdmPass& P, int ph, FC (&x)[16], uint32_t g,
                                          const uint32_t (&goff)[4]) {
  const int o0 = P.ph_first[ph], o1 = o0 + P.ph_count[ph];
  for (int o = o0; o < o1; ++o) {
    const float* u = P.coef + P.op_coef[o];
    const int ty = P.op_type[o];
    if (ty == OP_1Q) {
      float c[8];
      fdm_coef(u, c);
      switch (P.op_a[o]) {
        case 0: fdm_reg_1q<0>(x, c); break;
        case 1: fdm_reg_1q<1>(x, c); break;
        case 2: fdm_reg_1q<2>(x, c); break;
        default: fdm_reg_1q<3>(x, c); break;
      }
    } else if (ty == OP_2Q) {
      float c[32];
      fdm_coef(u, c);
      switch (P.op_a[o] * 4 + P.op_b[o]) {
        case 1: fdm_reg_2q<0, 1>(x, c); break;
        case 2: fdm_reg_2q<0, 2>(x, c); break;
        case 3: fdm_reg_2q<0, 3>(x, c); break;
        case 6: fdm_reg_2q<1, 2>(x, c); break;
        case 7: fdm_reg_2q<1, 3>(x, c); break;
        default: fdm_reg_2q<2, 3>(x, c); break;
      }
    } else {
      // diagonal: an operand >= 64 is register (operand - 64), else a global index bit, which
      // is the same for all 16 registers of a lane.  Register operands come first (ra < rb).
      const int qa = P.op_a[o], qb = ty == OP_DIAG2 ? P.op_b[o] : -1;
      float u8[8];
      if (ty == OP_DIAG1) {
        float u4[4];
        fdm_coef(u, u4);
#pragma unroll
        for (int t = 0; t < 8; ++t) u8[t] = u4[t & 3];
      } else {
        fdm_coef(u, u8);
      }
      const int ra = qa >= 64 ? qa - 64 : -1, rb = qb >= 64 ? qb - 64 : -1;
      // lane bits of the non-register operands
      const bool ta = qa >= 0 && qa < 64 && ((g >> qa) & 1u);
      const bool tb = qb >= 0 && qb < 64 && ((g >> qb) & 1u);
      float c[8];
      if (ra < 0) {
        // no register operand: one coefficient per lane
        float r0, i0, r1, i1;
        fsel2(ta, u8[0], u8[1], u8[2], u8[3], r0, i0);
        fsel2(ta, u8[4], u8[5], u8[6], u8[7], r1, i1);
        fsel2(tb, r0, i0, r1, i1, c[0], c[1]);
      } else if (rb < 0) {
        // register bit a, lane bit b (or none)
        fsel2(tb, u8[0], u8[1], u8[4], u8[5], c[0], c[1]);
        fsel2(tb, u8[2], u8[3], u8[6], u8[7], c[2], c[3]);
      } else {
#pragma unroll
        for (int t = 0; t < 8; ++t) c[t] = u8[t];
      }
      const int key = ra < 0 ? 0 : (rb < 0 ? 1 + ra : 5 + ra * 4 + rb);
      const bool real = u8[1] == 0.f && u8[3] == 0.f && u8[5] == 0.f && u8[7] == 0.f;
      if (real) fdm_diag_dispatch<true>(x, key, c);
      else fdm_diag_dispatch<false>(x, key, c);
    }
  }
}

__device__ __forceinline__ void fdm_phase_body(const FdmPass& P, float2* __restrict__ rho, uint32_t tile_index) {
  extern __shared__ __attribute__((aligned(16))) unsigned char fdm_psmem[];
  float2* tile = reinterpret_cast<float2*>(fdm_psmem);   // [2^13]
  __shared__ uint32_t hi_off[256];                         // global bits of the high tile slots
  const int tid = threadIdx.x;
  constexpr int lo = kFdmLowBits, K = kFdmMaxLocal;
  if (tid < 256) {
    uint32_t off = 0;
    for (int j = 0; j < K - lo; ++j) off |= ((uint32_t)(tid >> j) & 1u) << P.local_q[lo + j];
    hi_off[tid] = off;
  }
  uint32_t base = tile_index;
  for (int j = 0; j < lo; ++j) base = ins0(base, j);
  for (int j = 0; j < K - lo; ++j) base = ins0(base, P.sorted_hi[j]);
  __syncthreads();
  FC x[16];
  uint32_t pos = 0, g = 0, sh_pos[4], goff[4];
  fdm_layout(P, 0, base, hi_off, pos, g, sh_pos, goff);
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const f2v v = __builtin_nontemporal_load(reinterpret_cast<const f2v*>(rho + (g | fpick(i, goff))));
    x[i] = FC{v[0], v[1]};
  }
  fdm_apply(P, 0, x, g, goff);
  for (int ph = 1; ph < P.n_phases; ++ph) {
#pragma unroll
    for (int i = 0; i < 16; ++i) tile[pos | fpick(i, sh_pos)] = make_float2(x[i].x, x[i].y);
    __syncthreads();
    fdm_layout(P, ph, base, hi_off, pos, g, sh_pos, goff);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const float2 v = tile[pos | fpick(i, sh_pos)];
      x[i] = FC{v.x, v.y};
    }
    fdm_apply(P, ph, x, g, goff);
    if (ph + 1 < P.n_phases) __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    f2v v;
    v[0] = x[i].x;
    v[1] = x[i].y;
    __builtin_nontemporal_store(v, reinterpret_cast<f2v*>(rho + (g | fpick(i, goff))));
  }
}

__global__ __launch_bounds__(kFdmThreads) void fdm_phase_kernel(const FdmPass P, float2* __restrict__ rho) {
  fdm_phase_body(P, rho, blockIdx.x);
}

hipError_t launch_fdm_pass(const FdmPass& p, float2* rho, hipStream_t s) {
  if (p.n_phases > 0) {
    if (p.k != kFdmMaxLocal || p.nbits > 32 || p.n_phases > kFdmMaxPhases) return hipErrorInvalidValue;
    const size_t shm = ((size_t)1 << kFdmMaxLocal) * sizeof(float2);
    static bool attr = false;
    if (!attr) {
      const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fdm_phase_kernel),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
      if (e != hipSuccess) return e;
      attr = true;
    }
    const uint64_t tiles = 1ull << (p.nbits - p.k);
    if (tiles > 0x7fffffffull) return hipErrorInvalidValue;
    hipLaunchKernelGGL(fdm_phase_kernel, dim3((uint32_t)tiles), dim3(kFdmThreads), shm, s, p, rho);
    return hipGetLastError();
  }
  if (p.k < 1 || p.k > kFdmMaxLocal || p.k > p.nbits || p.nbits > 32) return hipErrorInvalidValue;
  if (p.k < p.nbits && p.k < kFdmLowBits) return hipErrorInvalidValue;
  const size_t shm = ((size_t)1 << p.k) * sizeof(float2);
  const uint64_t tiles = 1ull << (p.nbits - p.k);
  if (tiles > 0x7fffffffull) return hipErrorInvalidValue;
  hipLaunchKernelGGL(fdm_pass_kernel, dim3((uint32_t)tiles), dim3(256), shm, s, p, rho);
  return hipGetLastError();
}

// rho = |0><0|
__global__ void fdm_zero_kernel(float2* __restrict__ rho, uint64_t count) {
  const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * 256;
  for (uint64_t e = i; e < count; e += stride) rho[e] = make_float2(e == 0 ? 1.f : 0.f, 0.f);
}

hipError_t launch_fdm_reset(float2* rho, int n, hipStream_t s) {
  const uint64_t count = 1ull << (2 * n);
  const uint64_t want = (count + 255) / 256;
  const uint32_t blocks = (uint32_t)(want < 65536 ? want : 65536);
  hipLaunchKernelGGL(fdm_zero_kernel, dim3(blocks), dim3(256), 0, s, rho, count);
  return hipGetLastError();
}

// Prob(x) = Re rho[x][x]
__global__ void fdm_diag_kernel(const float2* __restrict__ rho, int n, double* __restrict__ p) {
  const uint32_t x = blockIdx.x * 256 + threadIdx.x;
  if (x >= (1u << n)) return;
  p[x] = (double)rho[((size_t)x << n) + x].x;
}

hipError_t launch_fdm_diag(const float2* rho, int n, double* p, hipStream_t s) {
  const uint32_t rows = 1u << n;
  hipLaunchKernelGGL(fdm_diag_kernel, dim3((rows + 255) / 256), dim3(256), 0, s, rho, n, p);
  return hipGetLastError();
}

// rho[x][y] *= phase[pop(x)] conj(phase[pop(y)]): a diagonal gate that depends on the Hamming
// weight, on the row and the column side (Sec. III.C's Grover oracle and |0..0> reflection).
// The (n + 1)^2 products are formed in FP64 once per work-group and kept in LDS as complex64;
// each thread step takes two neighbouring entries of one row (a 16-byte access).
__global__ void __launch_bounds__(256) fdm_weight_kernel(float2* __restrict__ rho, int n, FdmPhase P) {
  __shared__ float2 tab[(kFdmMaxQubits + 1) * (kFdmMaxQubits + 1)];
  const int nw = n + 1;
  for (int i = threadIdx.x; i < nw * nw; i += 256) {
    const int a = i / nw, b = i - a * nw;
    const double ax = P.ph[2 * a], ay = P.ph[2 * a + 1], bx = P.ph[2 * b], by = P.ph[2 * b + 1];
    tab[i] = make_float2((float)(ax * bx + ay * by), (float)(ay * bx - ax * by));
  }
  __syncthreads();
  const uint64_t pairs = 1ull << (2 * n - 1);
  const uint32_t cmask = (1u << n) - 1u;
  const uint64_t stride = (uint64_t)gridDim.x * 256;
  float4* r4 = reinterpret_cast<float4*>(rho);
  for (uint64_t e = (uint64_t)blockIdx.x * 256 + threadIdx.x; e < pairs; e += stride) {
    const uint32_t x = (uint32_t)((2 * e) >> n), y = (uint32_t)(2 * e) & cmask;   // y even
    const int px = __popc(x) * nw, py = __popc(y);
    const float2 w0 = tab[px + py], w1 = tab[px + py + 1];   // pop(y + 1) = pop(y) + 1
    const float4 v = r4[e];
    r4[e] = make_float4(v.x * w0.x - v.y * w0.y, v.x * w0.y + v.y * w0.x,
                        v.z * w1.x - v.w * w1.y, v.z * w1.y + v.w * w1.x);
  }
}

hipError_t launch_fdm_weight(float2* rho, int n, const FdmPhase& ph, hipStream_t s) {
  const uint64_t pairs = 1ull << (2 * n - 1);
  const uint64_t want = (pairs + 255) / 256;
  const uint32_t blocks = (uint32_t)(want < 8192 ? want : 8192);
  hipLaunchKernelGGL(fdm_weight_kernel, dim3(blocks), dim3(256), 0, s, rho, n, ph);
  return hipGetLastError();
}

}  // namespace lrdm
