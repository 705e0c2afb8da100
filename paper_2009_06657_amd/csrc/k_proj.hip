// Projection onto the kept eigenvectors on MFMA: L_new = c L' V_k (Sec. II.B; by Theorem 1 the
// truncated state sum_{i<=k} lambda_i u_i u_i^H with u_i = L' v_i / sqrt(lambda_i) equals
// (L' V_k)(L' V_k)^H).
//
// In the split view X = [L_0 | L_1] (qubit q) the Kraus concatenation is folded into the small
// matrix: [L_new(bit q = 0) | L_new(bit q = 1)] = X W with W_{(b,v),(b',j)} =
// c sum_a (E_a)_{b'b} V[(a,v), j], so the projection is one tall-skinny GEMM whose output rows
// overwrite the same row pair they were read from (in place).  The plain view is X = L', W =
// c V_k.  Complex products use the real embedding: row (re, im) times the 2x2 block
// [[w_re, w_im], [-w_im, w_re]] on v_mfma_*_16x16x4.
//
// Tiling: a work-group owns 128 rows of X (32 per wave) and all output columns; K is streamed
// in chunks of 32 reals through LDS together with the matching 32 rows of the expanded W.
// Every row is read before any row is written, and no other work-group touches these rows.
#include "lrdm_internal.h"

namespace lrdm {

typedef float pv4f __attribute__((ext_vector_type(4)));
typedef double pv4d __attribute__((ext_vector_type(4)));
template <class T> struct PAcc4;
template <> struct PAcc4<float> { using type = pv4f; };
template <> struct PAcc4<double> { using type = pv4d; };

__device__ __forceinline__ pv4f pmfma16(float a, float b, pv4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ pv4d pmfma16(double a, double b, pv4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int kProjBM = 128;   // rows per work-group
constexpr int kProjKC = 32;    // reals of K per chunk
constexpr int kProjXS = kProjKC + 2;   // LDS row stride of the X chunk

template <class T, int FO>
__global__ __launch_bounds__(256, 2) void project_kernel(cx_t<T>* __restrict__ L, int ld, int c_in,
                                                         int nsplit, int q, int c_out,
                                                         const cx_t<T>* __restrict__ W,
                                                         uint32_t rows) {
  using A4 = typename PAcc4<T>::type;
  constexpr int NTO = FO / 16;
  constexpr int WS = FO + 16;   // LDS row stride of the W chunk
  __shared__ __attribute__((aligned(16))) T xs[kProjBM * kProjXS];
  __shared__ __attribute__((aligned(16))) T ws[kProjKC * WS];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m = lane & 15, kq = lane >> 4;
  const uint32_t y0 = blockIdx.x * kProjBM;
  const int F = 2 * nsplit * c_in;          // input reals per row
  const int seg_in = 2 * c_in;
  const int fco = FO / 2;                   // complex output columns of W
  T* Lr = reinterpret_cast<T*>(L);
  const T* Wr = reinterpret_cast<const T*>(W);

  A4 acc[2][NTO];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int t = 0; t < NTO; ++t) acc[r][t] = A4{0, 0, 0, 0};

  auto row_index = [&](uint32_t y, int h) -> uint32_t {
    if (nsplit == 1) return y;
    const uint32_t lo = y & ((1u << q) - 1u);
    return (((y >> q) << (q + 1)) | lo) | ((uint32_t)h << q);
  };

  for (int kc = 0; kc < F; kc += kProjKC) {
    // X chunk: 128 rows x 32 reals, two reals per thread-step
    for (int e = tid; e < kProjBM * kProjKC / 2; e += 256) {
      const int rr = e / (kProjKC / 2);
      const int f = kc + (e % (kProjKC / 2)) * 2;
      const uint32_t y = y0 + rr;
      T a = 0, b = 0;
      if (y < rows && f < F) {
        const int h = f / seg_in;
        const int w = f - h * seg_in;
        const T* src = Lr + ((size_t)row_index(y, h) * ld) * 2 + w;
        a = src[0];
        b = src[1];
      }
      xs[rr * kProjXS + (f - kc)] = a;
      xs[rr * kProjXS + (f - kc) + 1] = b;
    }
    // W chunk: complex rows kc/2 .. kc/2 + 15 expanded to 32 real rows
    for (int e = tid; e < (kProjKC / 2) * fco; e += 256) {
      const int pr = e / fco, qc = e % fco;
      const size_t gi = ((size_t)(kc / 2 + pr) * fco + qc) * 2;
      const bool in = (kc / 2 + pr) < F / 2;
      const T re = in ? Wr[gi] : (T)0, im = in ? Wr[gi + 1] : (T)0;
      T* w0 = ws + (2 * pr) * WS + 2 * qc;
      T* w1 = w0 + WS;
      w0[0] = re;
      w0[1] = im;
      w1[0] = -im;
      w1[1] = re;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < kProjKC / 4; ++ks) {
      const T a0 = xs[(32 * wave + m) * kProjXS + 4 * ks + kq];
      const T a1 = xs[(32 * wave + 16 + m) * kProjXS + 4 * ks + kq];
      const T* wrow = ws + (4 * ks + kq) * WS + m;
#pragma unroll
      for (int t = 0; t < NTO; ++t) {
        const T b = wrow[16 * t];
        acc[0][t] = pmfma16(a0, b, acc[0][t]);
        acc[1][t] = pmfma16(a1, b, acc[1][t]);
      }
    }
    __syncthreads();
  }

  // write back: output real column f -> half h, real offset w inside that half
  const int seg_out = 2 * c_out;
#pragma unroll
  for (int r = 0; r < 2; ++r) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      // 16x16x4 MFMA output row: 4 (lane / 16) + v for FP32, 4 v + lane / 16 for FP64
      const int orow = (sizeof(T) == 8) ? (4 * v + kq) : (4 * kq + v);
      const uint32_t y = y0 + 32 * wave + 16 * r + orow;
      if (y >= rows) continue;
#pragma unroll
      for (int t = 0; t < NTO; ++t) {
        const int f = 16 * t + m;
        const int h = f / seg_out;
        const int w = f - h * seg_out;
        Lr[((size_t)row_index(y, h) * ld) * 2 + w] = acc[r][t][v];
      }
    }
  }
}

template <class T, int FO>
static hipError_t launch_proj_f(cx_t<T>* L, int n, int ld, int c_in, int nsplit, int q, int c_out,
                                const cx_t<T>* W, hipStream_t s) {
  const uint32_t rows = 1u << (n - (nsplit == 2 ? 1 : 0));
  const uint32_t blocks = (rows + kProjBM - 1) / kProjBM;
  hipLaunchKernelGGL((project_kernel<T, FO>), dim3(blocks), dim3(256), 0, s, L, ld, c_in, nsplit, q,
                     c_out, W, rows);
  return hipGetLastError();
}

template <class T>
hipError_t launch_project(cx_t<T>* L, int n, int ld, int c_in, int nsplit, int q, int c_out,
                          const cx_t<T>* W, hipStream_t s) {
  const int FO = 2 * nsplit * c_out;
  switch (FO) {
    case 16: return launch_proj_f<T, 16>(L, n, ld, c_in, nsplit, q, c_out, W, s);
    case 32: return launch_proj_f<T, 32>(L, n, ld, c_in, nsplit, q, c_out, W, s);
    case 64: return launch_proj_f<T, 64>(L, n, ld, c_in, nsplit, q, c_out, W, s);
    case 128: return launch_proj_f<T, 128>(L, n, ld, c_in, nsplit, q, c_out, W, s);
    case 256:
      if constexpr (sizeof(T) == 4) return launch_proj_f<T, 256>(L, n, ld, c_in, nsplit, q, c_out, W, s);
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

template hipError_t launch_project<float>(float2*, int, int, int, int, int, int, const float2*, hipStream_t);
template hipError_t launch_project<double>(double2*, int, int, int, int, int, int, const double2*, hipStream_t);

}  // namespace lrdm
