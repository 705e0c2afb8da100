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
// in chunks of 32 reals through LDS together with the matching 32 rows of the expanded W, the
// next chunk prefetched into registers (16-byte loads) during the MFMAs.  W is the first MFMA
// operand, so the accumulator of a lane holds 4 consecutive output columns of one row, written
// back as one 16-byte store (ordinary stores: the cache joins the two 64-byte halves of each
// 128-byte line that a wave writes with consecutive stores, non-temporal ones reached HBM as
// partial lines and raised the written bytes by a third).  Every row is read before any row is
// written, and no other work-group touches these rows.
#include <algorithm>

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
constexpr int kProjXS = kProjKC + 4;   // LDS row stride of the X chunk (16-byte aligned rows)

template <class T> struct PPair;   // two reals: one complex entry
template <> struct PPair<float> { typedef float type __attribute__((ext_vector_type(2))); };
template <> struct PPair<double> { typedef double type __attribute__((ext_vector_type(2))); };

// Software pipeline over K chunks: the next chunk of X rows and of W rows is fetched into
// registers while the MFMAs consume the current chunk from LDS.
template <class T, int FO>
__device__ __forceinline__ void project_body(cx_t<T>* __restrict__ L, int ld, int F, int seg_in_shift,
                                             int nsplit, int q, int seg_out_shift,
                                             const cx_t<T>* __restrict__ W, int skip, uint32_t rows,
                                             uint32_t bid, int q1 = -1) {
  using A4 = typename PAcc4<T>::type;
  using P2 = typename PPair<T>::type;
  constexpr int NTO = FO / 16;
  constexpr int FCO = FO / 2;              // complex output columns of W
  constexpr int WS = FO + 16;              // LDS row stride of the W chunk
  __shared__ __attribute__((aligned(16))) T xs[kProjBM * kProjXS];
  __shared__ __attribute__((aligned(16))) T ws[kProjKC * WS];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m = lane & 15, kq = lane >> 4;
  const uint32_t y0 = bid * kProjBM;
  const int seg_in_mask = (1 << seg_in_shift) - 1;
  T* Lr = reinterpret_cast<T*>(L);
  const T* Wr = reinterpret_cast<const T*>(W);

  A4 acc[2][NTO];
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int t = 0; t < NTO; ++t) acc[r][t] = A4{0, 0, 0, 0};

  auto row_index = [&](uint32_t y, int h) -> uint32_t {
    if (nsplit == 1) return y;
    if (nsplit == 4) {   // qubit pair (q, q1): segment h = b(q) + 2 b(q1)
      const int lo = q < q1 ? q : q1, hi = q < q1 ? q1 : q;
      uint32_t t = ((y >> lo) << (lo + 1)) | (y & ((1u << lo) - 1u));
      t = ((t >> hi) << (hi + 1)) | (t & ((1u << hi) - 1u));
      return t | ((uint32_t)(h & 1) << q) | ((uint32_t)(h >> 1) << q1);
    }
    return ((((y >> q) << (q + 1)) | (y & ((1u << q) - 1u))) | ((uint32_t)h << q));
  };

  using Q4 = typename PAcc4<T>::type;
  constexpr int XQ = kProjBM * kProjKC / 4 / 256;             // X quads per thread
  constexpr int WP = (kProjKC / 2) * FCO / 2;                 // W complex pairs per chunk
  constexpr int WQ = (WP + 255) / 256;                         // per thread (the last guarded)
  static_assert(XQ * 256 * 4 == kProjBM * kProjKC, "shape");
  Q4 xb[XQ];
  Q4 wb[WQ > 0 ? WQ : 1];
  auto fetch = [&](int kc) {
#pragma unroll
    for (int k = 0; k < XQ; ++k) {
      const int e = tid + k * 256;
      const int rr = e >> 3, f = kc + ((e & 7) << 2);
      const uint32_t y = y0 + rr;
      Q4 v = {0, 0, 0, 0};
      if (y < rows && f < F) {
        if (seg_in_shift >= 2) {
          const int h = f >> seg_in_shift, w = f & seg_in_mask;
          v = *reinterpret_cast<const Q4*>(Lr + ((size_t)row_index(y, h) * ld) * 2 + w);
        } else {
          // one complex column per half (rank 1): the quad spans both halves
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            const int fu = f + 2 * u;
            if (fu < F) {
              const int h = fu >> seg_in_shift, w = fu & seg_in_mask;
              const P2 p = *reinterpret_cast<const P2*>(Lr + ((size_t)row_index(y, h) * ld) * 2 + w);
              v[2 * u] = p[0];
              v[2 * u + 1] = p[1];
            }
          }
        }
      }
      xb[k] = v;
    }
#pragma unroll
    for (int k = 0; k < WQ; ++k) {
      const int e = tid + k * 256;
      const int pr = e / (FCO / 2), qc = 2 * (e % (FCO / 2));
      Q4 v = {0, 0, 0, 0};
      if (e < WP && kc / 2 + pr < F / 2) v = *reinterpret_cast<const Q4*>(Wr + ((size_t)(kc / 2 + pr) * FCO + qc) * 2);
      wb[k] = v;
    }
  };
  auto stage = [&]() {
#pragma unroll
    for (int k = 0; k < XQ; ++k) {
      const int e = tid + k * 256;
      *reinterpret_cast<Q4*>(xs + (e >> 3) * kProjXS + ((e & 7) << 2)) = xb[k];
    }
#pragma unroll
    for (int k = 0; k < WQ; ++k) {
      const int e = tid + k * 256;
      if (e >= WP) break;
      const int pr = e / (FCO / 2), qc = 2 * (e % (FCO / 2));
      T* w0 = ws + (2 * pr) * WS + 2 * qc;
      const Q4 v = wb[k];
      *reinterpret_cast<Q4*>(w0) = v;                                  // ( re, im) of two entries
      *reinterpret_cast<Q4*>(w0 + WS) = Q4{-v[1], v[0], -v[3], v[2]};  // (-im, re)
    }
  };

  // Zero blocks of W (split view): a chunk lies inside one input half when the half spans
  // whole chunks, and an output tile inside one output half (16 reals per tile, seg_out >= 16),
  // so the output tiles of a zero block are skipped for that chunk (uniform branches).
  const bool halves = nsplit == 2 && seg_in_shift >= 5 && seg_out_shift >= 4 && skip != 0;
  fetch(0);
  for (int kc = 0; kc < F; kc += kProjKC) {
    stage();
    __syncthreads();
    if (kc + kProjKC < F) fetch(kc + kProjKC);
    const int hin = kc >> seg_in_shift;
    const bool do0 = !(halves && hin == 1 && (skip & 2));   // output half 0 from this chunk
    const bool do1 = !(halves && hin == 0 && (skip & 1));   // output half 1 from this chunk
#pragma unroll
    for (int ks = 0; ks < kProjKC / 4; ++ks) {
      const T a0 = xs[(32 * wave + m) * kProjXS + 4 * ks + kq];
      const T a1 = xs[(32 * wave + 16 + m) * kProjXS + 4 * ks + kq];
      const T* wrow = ws + (4 * ks + kq) * WS + m;
      if (do0) {
#pragma unroll
        for (int t = 0; t < NTO / 2; ++t) {
          const T b = wrow[16 * t];
          acc[0][t] = pmfma16(b, a0, acc[0][t]);
          acc[1][t] = pmfma16(b, a1, acc[1][t]);
        }
      }
      if (do1) {
#pragma unroll
        for (int t = NTO / 2; t < NTO; ++t) {
          const T b = wrow[16 * t];
          acc[0][t] = pmfma16(b, a0, acc[0][t]);
          acc[1][t] = pmfma16(b, a1, acc[1][t]);
        }
      }
    }
    __syncthreads();
  }

  // write back: lane (kq, m) holds row m of its 16-row tile and output real columns
  // 16 t + 4 kq .. + 3 (the MFMA output rows index W's columns)
  const int seg_out_mask = (1 << seg_out_shift) - 1;
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const uint32_t y = y0 + 32 * wave + 16 * r + m;
    if (y >= rows) continue;
#pragma unroll
    for (int t = 0; t < NTO; ++t) {
      if constexpr (sizeof(T) == 4) {
        // FP32 output: register v is column 16 t + 4 kq + v (a half holds >= 8 reals here)
        const int f = 16 * t + 4 * kq;
        const int h = f >> seg_out_shift;
        const int w = f & seg_out_mask;
        *reinterpret_cast<A4*>(Lr + ((size_t)row_index(y, h) * ld) * 2 + w) = acc[r][t];
      } else {
        // FP64 output: register v is column 16 t + 4 v + kq
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int f = 16 * t + 4 * v + kq;
          const int h = f >> seg_out_shift;
          const int w = f & seg_out_mask;
          Lr[((size_t)row_index(y, h) * ld) * 2 + w] = acc[r][t][v];
        }
      }
    }
  }
}

template <class T, int FO>
__global__ __launch_bounds__(256, 2) void project_kernel(cx_t<T>* __restrict__ L, int ld, int F,
                                                         int seg_in_shift, int nsplit, int q,
                                                         int seg_out_shift,
                                                         const cx_t<T>* __restrict__ W, int skip,
                                                         uint32_t rows) {
  project_body<T, FO>(L, ld, F, seg_in_shift, nsplit, q, seg_out_shift, W, skip, rows, blockIdx.x);
}

// the qubit-pair view (nsplit = 4)
template <class T, int FO>
__global__ __launch_bounds__(256, 2) void project4_kernel(cx_t<T>* __restrict__ L, int ld, int F, int seg_in_shift,
                                                          int q0, int q1, int seg_out_shift,
                                                          const cx_t<T>* __restrict__ W, uint32_t rows) {
  project_body<T, FO>(L, ld, F, seg_in_shift, 4, q0, seg_out_shift, W, 0, rows, blockIdx.x, q1);
}

template <class T, int FO>
__global__ __launch_bounds__(256, 2) void project_batched(const ProjJob<T>* __restrict__ jobs, int njobs) {
  const int j = find_job(jobs, njobs, blockIdx.x);
  const ProjJob<T>& J = jobs[j];
  project_body<T, FO>(J.L, J.ld, J.F, J.seg_in_shift, J.nsplit, J.q, J.seg_out_shift, J.W, J.skip,
                      J.rows, blockIdx.x - J.block0);
}

template <class T>
hipError_t launch_project_batched(int FO, const ProjJob<T>* jobs, int njobs, uint32_t blocks, hipStream_t s) {
  if (njobs < 1 || blocks < 1) return hipErrorInvalidValue;
  switch (FO) {
    case 16: hipLaunchKernelGGL((project_batched<T, 16>), dim3(blocks), dim3(256), 0, s, jobs, njobs); break;
    case 32: hipLaunchKernelGGL((project_batched<T, 32>), dim3(blocks), dim3(256), 0, s, jobs, njobs); break;
    case 64: hipLaunchKernelGGL((project_batched<T, 64>), dim3(blocks), dim3(256), 0, s, jobs, njobs); break;
    case 128: hipLaunchKernelGGL((project_batched<T, 128>), dim3(blocks), dim3(256), 0, s, jobs, njobs); break;
    case 256:
      if constexpr (sizeof(T) == 4) {
        hipLaunchKernelGGL((project_batched<T, 256>), dim3(blocks), dim3(256), 0, s, jobs, njobs);
        break;
      }
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Resident-W projection for the wide split view in complex64 (c_in = c_out = 64: X is
// 2^(n-1) x 128 complex, W 128 x 128 complex).  Every work-group copies W once into LDS as two
// real planes (rows padded to 130 floats: the four lane groups of a wave read rows 8 apart, which
// then fall on different banks) and keeps it there; each wave then streams its own 16-row blocks
// of X from HBM straight into registers (the next block's loads in flight while it works on the
// current one), so there is no barrier after the copy of W.  The complex product takes four real
// MFMAs per (k, tile): Y_re += W_re x X_re + W_im x (-X_im), Y_im += W_im x X_re + W_re x X_im.
// Lane group g = lane / 16 takes k = 32 c + 8 g + j (j < 8) of K chunk c, so a lane's operand of
// X for a whole chunk is 8 consecutive complex values of its row (64 bytes); W is read at the same
// k.  Rows are read before they are written, by the same wave only.
constexpr int kPRThreads = 256;        // 4 waves, one per SIMD (the whole register file each)
constexpr int kPRK = 128;              // complex K (both halves of X)
constexpr int kPRO = 128;              // complex outputs (both halves)
constexpr int kPRS = 130;              // LDS row stride of a W plane (floats)
constexpr size_t kPRShm = (size_t)2 * kPRK * kPRS * sizeof(float);

__device__ __forceinline__ uint32_t pr_row(uint32_t y, int h, int q) {
  return ((y >> q) << (q + 1)) | (y & ((1u << q) - 1u)) | ((uint32_t)h << q);
}

// one half of X row y (complex columns 64 h .. 64 h + 63): chunks 2 h and 2 h + 1
__device__ __forceinline__ void pr_load_half(const float2* __restrict__ L, int ld, int q, uint32_t y, int h, int kq,
                                             pv4f (&x)[2][4]) {
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const float2* src = L + (size_t)pr_row(y, h, q) * ld + 32 * c + 8 * kq;
#pragma unroll
    for (int u = 0; u < 4; ++u) x[c][u] = *reinterpret_cast<const pv4f*>(src + 2 * u);
  }
}

// the MFMAs of input half h (chunks 2 h, 2 h + 1) into the output tiles t0 .. t0 + 3
__device__ __forceinline__ void pr_half(const float* __restrict__ wre, const float* __restrict__ wim, int h, int kq,
                                        int m, int t0, const pv4f (&x)[2][4], pv4f (&ar)[8], pv4f (&ai)[8]) {
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = 32 * (2 * h + c) + 8 * kq + j;
      const float xr = x[c][j >> 1][2 * (j & 1)], xi = x[c][j >> 1][2 * (j & 1) + 1];
      const float* wr = wre + k * kPRS + m;
      const float* wi = wim + k * kPRS + m;
#pragma unroll
      for (int t = t0; t < t0 + 4; ++t) {
        const float a_r = wr[16 * t], a_i = wi[16 * t];
        ar[t] = pmfma16(a_r, xr, ar[t]);
        ar[t] = pmfma16(a_i, -xi, ar[t]);
        ai[t] = pmfma16(a_i, xr, ai[t]);
        ai[t] = pmfma16(a_r, xi, ai[t]);
      }
    }
}

__global__ __launch_bounds__(kPRThreads, 1) void project_resident_kernel(float2* __restrict__ L, int ld, int q,
                                                                         const float2* __restrict__ W, int skip,
                                                                         uint32_t rows) {
  extern __shared__ __attribute__((aligned(16))) float prs[];
  float* wre = prs;
  float* wim = prs + kPRK * kPRS;
  for (int e = threadIdx.x; e < kPRK * kPRO; e += kPRThreads) {
    const float2 w = W[e];
    const int k = e / kPRO, o = e % kPRO;
    wre[k * kPRS + o] = w.x;
    wim[k * kPRS + o] = w.y;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int m = lane & 15, kq = lane >> 4;
  const uint32_t nblk = rows / 16;
  const uint32_t step = gridDim.x * (kPRThreads / 64);
  uint32_t b = blockIdx.x * (kPRThreads / 64) + wave;
  // output half 1 from input half 0 is zero (skip & 1), output half 0 from input half 1 (skip & 2)
  const bool z10 = (skip & 1) != 0, z01 = (skip & 2) != 0;
  // x0: the input half 0 of the current block (its loads issued one half ahead), x1: half 1
  pv4f x0[2][4], x1[2][4];
  if (b < nblk) pr_load_half(L, ld, q, 16 * b + m, 0, kq, x0);
  for (; b < nblk; b += step) {
    const uint32_t y = 16 * b + m;
    pr_load_half(L, ld, q, y, 1, kq, x1);
    pv4f ar[8], ai[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      ar[t] = pv4f{0, 0, 0, 0};
      ai[t] = pv4f{0, 0, 0, 0};
    }
    pr_half(wre, wim, 0, kq, m, 0, x0, ar, ai);
    if (!z10) pr_half(wre, wim, 0, kq, m, 4, x0, ar, ai);
    if (b + step < nblk) pr_load_half(L, ld, q, 16 * (b + step) + m, 0, kq, x0);
    if (!z01) pr_half(wre, wim, 1, kq, m, 0, x1, ar, ai);
    pr_half(wre, wim, 1, kq, m, 4, x1, ar, ai);
    // lane (kq, m) holds output columns 16 t + 4 kq + v (v < 4) of row m
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      float2* dst = L + (size_t)pr_row(y, t >> 2, q) * ld + ((16 * t + 4 * kq) & 63);
      *reinterpret_cast<pv4f*>(dst) = pv4f{ar[t][0], ai[t][0], ar[t][1], ai[t][1]};
      *reinterpret_cast<pv4f*>(dst + 2) = pv4f{ar[t][2], ai[t][2], ar[t][3], ai[t][3]};
    }
  }
}

static hipError_t launch_project_resident(float2* L, int n, int ld, int q, const float2* W, int skip, int cus,
                                          hipStream_t s) {
  static bool attr_set = false;
  if (!attr_set) {
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(project_resident_kernel),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)kPRShm);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  const uint32_t rows = 1u << (n - 1);
  const uint32_t wgs = (uint32_t)std::max(1, std::min(cus > 0 ? cus : 256, 1024));
  hipLaunchKernelGGL(project_resident_kernel, dim3(wgs), dim3(kPRThreads), kPRShm, s, L, ld, q, W, skip, rows);
  return hipGetLastError();
}

template <class T, int FO>
static hipError_t launch_proj_f(cx_t<T>* L, int n, int ld, int c_in, int nsplit, int q, int c_out,
                                const cx_t<T>* W, int skip, hipStream_t s) {
  const uint32_t rows = 1u << (n - (nsplit == 2 ? 1 : 0));
  const uint32_t blocks = (rows + kProjBM - 1) / kProjBM;
  int si = 0, so = 0;
  while ((1 << si) < 2 * c_in) ++si;
  while ((1 << so) < 2 * c_out) ++so;
  if ((1 << si) != 2 * c_in || (1 << so) != 2 * c_out) return hipErrorInvalidValue;
  hipLaunchKernelGGL((project_kernel<T, FO>), dim3(blocks), dim3(256), 0, s, L, ld, 2 * nsplit * c_in,
                     si, nsplit, q, so, W, skip, rows);
  return hipGetLastError();
}

template <class T>
hipError_t launch_project(cx_t<T>* L, int n, int ld, int c_in, int nsplit, int q, int c_out,
                          const cx_t<T>* W, int skip, hipStream_t s, int cus) {
  const int FO = 2 * nsplit * c_out;
  if constexpr (sizeof(T) == 4) {
    if (nsplit == 2 && c_in == 64 && c_out == 64 && n >= 8 && ld >= 64 && q >= 0 && q < n)
      return launch_project_resident(L, n, ld, q, W, skip, cus, s);
  }
  switch (FO) {
    case 16: return launch_proj_f<T, 16>(L, n, ld, c_in, nsplit, q, c_out, W, skip, s);
    case 32: return launch_proj_f<T, 32>(L, n, ld, c_in, nsplit, q, c_out, W, skip, s);
    case 64: return launch_proj_f<T, 64>(L, n, ld, c_in, nsplit, q, c_out, W, skip, s);
    case 128: return launch_proj_f<T, 128>(L, n, ld, c_in, nsplit, q, c_out, W, skip, s);
    case 256:
      if constexpr (sizeof(T) == 4) return launch_proj_f<T, 256>(L, n, ld, c_in, nsplit, q, c_out, W, skip, s);
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

template <class T, int FO>
static hipError_t launch_proj4_f(cx_t<T>* L, int n, int ld, int c_in, int q0, int q1, int c_out, const cx_t<T>* W,
                                 hipStream_t s) {
  const uint32_t rows = 1u << (n - 2);
  const uint32_t blocks = (rows + kProjBM - 1) / kProjBM;
  int si = 0, so = 0;
  while ((1 << si) < 2 * c_in) ++si;
  while ((1 << so) < 2 * c_out) ++so;
  if ((1 << si) != 2 * c_in || (1 << so) != 2 * c_out) return hipErrorInvalidValue;
  hipLaunchKernelGGL((project4_kernel<T, FO>), dim3(blocks), dim3(256), 0, s, L, ld, 8 * c_in, si, q0, q1, so, W,
                     rows);
  return hipGetLastError();
}

template <class T>
hipError_t launch_project4(cx_t<T>* L, int n, int ld, int c_in, int q0, int q1, int c_out, const cx_t<T>* W,
                           hipStream_t s) {
  if (n < 2 || q0 == q1 || q0 < 0 || q1 < 0 || q0 >= n || q1 >= n || c_in > 32 || c_in < 1 || c_out > 32)
    return hipErrorInvalidValue;
  switch (8 * c_out) {
    case 64: return launch_proj4_f<T, 64>(L, n, ld, c_in, q0, q1, c_out, W, s);
    case 128: return launch_proj4_f<T, 128>(L, n, ld, c_in, q0, q1, c_out, W, s);
    case 256:
      if constexpr (sizeof(T) == 4) return launch_proj4_f<T, 256>(L, n, ld, c_in, q0, q1, c_out, W, s);
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

template hipError_t launch_project4<float>(float2*, int, int, int, int, int, int, const float2*, hipStream_t);
template hipError_t launch_project4<double>(double2*, int, int, int, int, int, int, const double2*, hipStream_t);
template hipError_t launch_project_batched<float>(int, const ProjJob<float>*, int, uint32_t, hipStream_t);
template hipError_t launch_project_batched<double>(int, const ProjJob<double>*, int, uint32_t, hipStream_t);
template hipError_t launch_project<float>(float2*, int, int, int, int, int, int, const float2*, int, hipStream_t, int);
template hipError_t launch_project<double>(double2*, int, int, int, int, int, int, const double2*, int, hipStream_t, int);

}  // namespace lrdm
