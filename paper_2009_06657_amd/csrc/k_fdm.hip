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

hipError_t launch_fdm_pass(const FdmPass& p, float2* rho, hipStream_t s) {
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

}  // namespace lrdm
