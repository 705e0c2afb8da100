// Gram matrix of the (split) factor on MFMA: the contraction step of the eigenvalue truncation
// (Sec. II.B): G = L'^H L' (Theorem 1, App. B) is formed from S = X^H X, where X is the
// factor viewed row by row.
//
//  * Split view (fused Kraus step): X = [L_0 | L_1], row y of X holds row x0 = y with a zero
//    inserted at bit q followed by row x1 = x0 | 2^q, so X is 2^(n-1) x 2c.  For a channel on
//    qubit q, (E_a L)_{b'} = sum_b (E_a)_{b'b} L_b, hence G_{ab} = sum_{uv} (E_a^H E_b)_{uv}
//    L_u^H L_v: G follows from S without ever forming [E_1 L | ... | E_m L].
//  * Plain view: X = L (2^n x c).
//
// Complex arithmetic runs on the real embedding X_r (interleaved re/im, F = 2 * nsplit * c real
// columns): R = X_r^T X_r, S_jk = (R[2j,2k] + R[2j+1,2k+1]) + i (R[2j,2k+1] - R[2j+1,2k]).
// R is a tall-skinny SYRK: only its upper 16x16 tiles are computed with v_mfma_*_16x16x4, each
// work-group reduces a contiguous slab of rows into a private partial (split-K), and a second
// kernel sums the partials in a fixed order in FP64 (deterministic).  Row chunks are staged
// through two LDS buffers, the next one fetched into registers during the MFMAs.
#include <algorithm>
#include <utility>

#include "lrdm_internal.h"

namespace lrdm {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));
template <class T> struct Acc4;
template <> struct Acc4<float> { using type = v4f; };
template <> struct Acc4<double> { using type = v4d; };

__device__ __forceinline__ v4f mfma16(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ v4d mfma16(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <int NT> struct UpperTiles {
  static constexpr int NUP = NT * (NT + 1) / 2;
  int ti[NUP];
  int tj[NUP];
  constexpr UpperTiles() : ti(), tj() {
    int u = 0;
    for (int i = 0; i < NT; ++i)
      for (int j = i; j < NT; ++j) {
        ti[u] = i;
        tj[u] = j;
        ++u;
      }
  }
};

template <class F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

constexpr int kGramKC = 64;   // rows per LDS chunk

template <class T, int F> struct GramCfg {
  static constexpr int NT = F / 16;
  static constexpr int NUP = NT * (NT + 1) / 2;
  static constexpr int NW = (F >= 256) ? 8 : 4;            // waves per work-group
  static constexpr int THREADS = 64 * NW;
  static constexpr int PER_WAVE = (NUP + NW - 1) / NW;
  static constexpr int STRIDE = F + 16;   // conflict-free 16-lane row reads
};

// One wave's share of the upper tiles: tile u = W + NW s.
template <class T, int F, int W>
__device__ __forceinline__ void gram_chunk_mma(const T* __restrict__ lds, typename Acc4<T>::type* acc,
                                               int lane) {
  using Cfg = GramCfg<T, F>;
  constexpr UpperTiles<Cfg::NT> tab{};
  const int m = lane & 15, k = lane >> 4;
#pragma unroll 2
  for (int kk = 0; kk < kGramKC / 4; ++kk) {
    const T* row = lds + (4 * kk + k) * Cfg::STRIDE + m;
    T f[Cfg::NT];
#pragma unroll
    for (int b = 0; b < Cfg::NT; ++b) f[b] = row[16 * b];
    static_for<Cfg::PER_WAVE>([&](auto s) {
      constexpr int u = W + Cfg::NW * decltype(s)::value;
      if constexpr (u < Cfg::NUP) {
        acc[decltype(s)::value] = mfma16(f[tab.ti[u]], f[tab.tj[u]], acc[decltype(s)::value]);
      }
    });
  }
}

template <class T, int F, int W>
__device__ __forceinline__ void gram_store(T* __restrict__ out, const typename Acc4<T>::type* acc,
                                           int lane) {
  using Cfg = GramCfg<T, F>;
  static_for<Cfg::PER_WAVE>([&](auto s) {
    constexpr int u = W + Cfg::NW * decltype(s)::value;
    if constexpr (u < Cfg::NUP) {
      typename Acc4<T>::type v = acc[decltype(s)::value];
      *reinterpret_cast<typename Acc4<T>::type*>(out + (size_t)u * 256 + lane * 4) = v;
    }
  });
}

typedef float gf4 __attribute__((ext_vector_type(4)));   // 16-byte register unit

// The chunk loop is software-pipelined: the next kGramKC rows are fetched into registers while
// the MFMAs consume the current chunk from one of two LDS buffers (one barrier per chunk).
// Row y of the view with a zero inserted at bits lo < hi (two qubits split out).
__device__ __forceinline__ uint32_t insert2(uint32_t y, int lo, int hi) {
  uint32_t t = ((y >> lo) << (lo + 1)) | (y & ((1u << lo) - 1u));
  return ((t >> hi) << (hi + 1)) | (t & ((1u << hi) - 1u));
}

// qf >= 0 (split view only): the rows are those with bit qf equal to bf, so X = [L_0 | L_1] on
// bit q over half of the rows (one half of the 4-way Gram on the bit pair (q, qf)).
template <class T, int F>
__device__ __forceinline__ void gram_body(const cx_t<T>* __restrict__ L, int ld, int seg_shift, int nsplit,
                                          int q, T* __restrict__ partials, uint32_t rows,
                                          uint32_t rows_per_block, uint32_t bid, int qf = -1,
                                          uint32_t bf = 0) {
  using Cfg = GramCfg<T, F>;
  using A4 = typename Acc4<T>::type;
  constexpr int VPR = 16 / sizeof(T);          // reals per 16-byte unit
  constexpr int UPR = F / VPR;                 // 16-byte units per row
  constexpr int UNITS = kGramKC * UPR;         // 16-byte units per chunk
  constexpr int UPT = UNITS / Cfg::THREADS;    // per thread
  static_assert(UNITS % Cfg::THREADS == 0, "chunk must split evenly");
  extern __shared__ __attribute__((aligned(16))) unsigned char gram_smem[];
  T* lds0 = reinterpret_cast<T*>(gram_smem);
  T* lds1 = lds0 + kGramKC * Cfg::STRIDE;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  A4 acc[Cfg::PER_WAVE];
#pragma unroll
  for (int s = 0; s < Cfg::PER_WAVE; ++s) acc[s] = A4{0, 0, 0, 0};

  const uint32_t r_begin = bid * rows_per_block;
  const uint32_t r_end = min(rows, r_begin + rows_per_block);
  const T* Lr = reinterpret_cast<const T*>(L);
  const int seg_mask = (1 << seg_shift) - 1;

  gf4 buf[UPT];
  auto fetch = [&](uint32_t r0) {
#pragma unroll
    for (int k = 0; k < UPT; ++k) {
      const int u = tid + k * Cfg::THREADS;
      const int rr = u / UPR, f = (u % UPR) * VPR;
      const uint32_t y = r0 + rr;
      gf4 val = {0.f, 0.f, 0.f, 0.f};
      if (y < r_end) {
        const int h = f >> seg_shift, w = f & seg_mask;
        uint32_t x = y;
        if (qf >= 0) x = insert2(y, min(q, qf), max(q, qf)) | ((uint32_t)h << q) | (bf << qf);
        else if (nsplit == 2) x = ((((y >> q) << (q + 1)) | (y & ((1u << q) - 1u))) | ((uint32_t)h << q));
        val = *reinterpret_cast<const gf4*>(Lr + ((size_t)x * ld) * 2 + w);
      }
      buf[k] = val;
    }
  };
  auto stage = [&](T* dst) {
#pragma unroll
    for (int k = 0; k < UPT; ++k) {
      const int u = tid + k * Cfg::THREADS;
      *reinterpret_cast<gf4*>(dst + (u / UPR) * Cfg::STRIDE + (u % UPR) * VPR) = buf[k];
    }
  };
  auto mma = [&](const T* src) {
    switch (wave) {
      case 0: gram_chunk_mma<T, F, 0>(src, acc, lane); break;
      case 1: gram_chunk_mma<T, F, 1>(src, acc, lane); break;
      case 2: gram_chunk_mma<T, F, 2>(src, acc, lane); break;
      case 3: gram_chunk_mma<T, F, 3>(src, acc, lane); break;
      case 4: if constexpr (Cfg::NW > 4) gram_chunk_mma<T, F, 4>(src, acc, lane); break;
      case 5: if constexpr (Cfg::NW > 5) gram_chunk_mma<T, F, 5>(src, acc, lane); break;
      case 6: if constexpr (Cfg::NW > 6) gram_chunk_mma<T, F, 6>(src, acc, lane); break;
      default: if constexpr (Cfg::NW > 7) gram_chunk_mma<T, F, 7>(src, acc, lane); break;
    }
  };

  if (r_begin < r_end) fetch(r_begin);
  bool odd = false;
  for (uint32_t r0 = r_begin; r0 < r_end; r0 += kGramKC) {
    T* cur = odd ? lds1 : lds0;
    stage(cur);
    __syncthreads();
    if (r0 + kGramKC < r_end) fetch(r0 + kGramKC);
    mma(cur);
    odd = !odd;
  }
  T* out = partials + (size_t)bid * Cfg::NUP * 256;
  switch (wave) {
    case 0: gram_store<T, F, 0>(out, acc, lane); break;
    case 1: gram_store<T, F, 1>(out, acc, lane); break;
    case 2: gram_store<T, F, 2>(out, acc, lane); break;
    case 3: gram_store<T, F, 3>(out, acc, lane); break;
    case 4: if constexpr (Cfg::NW > 4) gram_store<T, F, 4>(out, acc, lane); break;
    case 5: if constexpr (Cfg::NW > 5) gram_store<T, F, 5>(out, acc, lane); break;
    case 6: if constexpr (Cfg::NW > 6) gram_store<T, F, 6>(out, acc, lane); break;
    default: if constexpr (Cfg::NW > 7) gram_store<T, F, 7>(out, acc, lane); break;
  }
}

template <class T, int F>
__global__ __launch_bounds__((GramCfg<T, F>::THREADS)) void gram_kernel(const cx_t<T>* __restrict__ L, int ld,
                                                                       int seg_shift, int nsplit, int q,
                                                                       T* __restrict__ partials, uint32_t rows,
                                                                       uint32_t rows_per_block) {
  gram_body<T, F>(L, ld, seg_shift, nsplit, q, partials, rows, rows_per_block, blockIdx.x);
}

template <class T, int F>
__global__ __launch_bounds__((GramCfg<T, F>::THREADS)) void gram_batched(const GramJob<T>* __restrict__ jobs,
                                                                        int njobs) {
  const int j = find_job(jobs, njobs, blockIdx.x);
  const GramJob<T>& J = jobs[j];
  gram_body<T, F>(J.L, J.ld, J.seg_shift, J.nsplit, J.q, J.partials, J.rows, J.rows_per_block,
                  blockIdx.x - J.block0);
}

// ------------------------------------------------------------------ 4-way Gram on a bit pair
// For two qubits p != q, X4 = [X_0 | X_1] with X_b = [L(bit p = 0, bit q = b) | L(bit p = 1,
// bit q = b)] (2^(n-2) rows, 4c complex columns).  Its Gram matrix G4 = X4^H X4 has the blocks
// A = X_0^H X_0, B = X_1^H X_1 (the split Gram on bit p over the rows with bit q = 0 or 1: the
// kernel above with qf = q) and C = X_0^H X_1 (the kernel below, every tile of the real
// embedding X_0r^T X_1r).  One G4 taken before the projection on p gives the split Gram on q
// after it (see launch_pair_transform).

// Halves A and B in one launch: blocks [0, nbh) take the rows with bit q = 0, [nbh, 2 nbh) bit q = 1.
template <class T, int F>
__global__ __launch_bounds__((GramCfg<T, F>::THREADS)) void gram_halves_kernel(const cx_t<T>* __restrict__ L, int ld,
                                                                              int seg_shift, int p, int q,
                                                                              T* __restrict__ partials, uint32_t rows,
                                                                              uint32_t rows_per_block, uint32_t nbh) {
  const uint32_t bf = blockIdx.x / nbh, bl = blockIdx.x - bf * nbh;
  gram_body<T, F>(L, ld, seg_shift, 2, p, partials + (size_t)bf * nbh * GramCfg<T, F>::NUP * 256, rows,
                  rows_per_block, bl, q, bf);
}

template <class T, int FH> struct CrossCfg {
  static constexpr int NT = FH / 16;            // tile columns of each half
  static constexpr int NTILE = NT * NT;
  // wave w owns the tile columns tj = w + NW j of C (every ti): NT / NW columns of NT tiles
  static constexpr int NW = NT < 16 ? NT : 16;
  static constexpr int NJ = NT / NW;
  static constexpr int THREADS = 64 * NW;
  static constexpr int PER_WAVE = NT * NJ;
  // rows per LDS chunk: two buffers fit in LDS, and at 16 waves the register prefetch of the next
  // chunk stays within the 128-register budget
  static constexpr int KC = (NW == 16) ? 16 : ((FH * sizeof(T) >= 512) ? 32 : 64);
  static constexpr int STRIDE = 2 * FH + 16;
};

template <class T, int FH>
__device__ __forceinline__ void cross_chunk_mma(const T* __restrict__ lds, typename Acc4<T>::type* acc, int lane,
                                                int wave) {
  using Cfg = CrossCfg<T, FH>;
  const int m = lane & 15, k = lane >> 4;
#pragma unroll 1
  for (int kk = 0; kk < Cfg::KC / 4; ++kk) {
    const T* row = lds + (4 * kk + k) * Cfg::STRIDE + m;
    T f0[Cfg::NT], f1[Cfg::NJ];
#pragma unroll
    for (int b = 0; b < Cfg::NT; ++b) f0[b] = row[16 * b];
#pragma unroll
    for (int j = 0; j < Cfg::NJ; ++j) f1[j] = row[FH + 16 * (wave + Cfg::NW * j)];
#pragma unroll
    for (int j = 0; j < Cfg::NJ; ++j)
#pragma unroll
      for (int ti = 0; ti < Cfg::NT; ++ti)
        acc[j * Cfg::NT + ti] = mfma16(f0[ti], f1[j], acc[j * Cfg::NT + ti]);
  }
}

// C = X_0^H X_1 on the real embedding: each work-group reduces a slab of rows into a private
// partial of all (FH/16)^2 tiles; row chunks are staged through two LDS buffers as in the Gram.
template <class T, int FH>
__global__ __launch_bounds__((CrossCfg<T, FH>::THREADS)) void gram_cross_kernel(const cx_t<T>* __restrict__ L, int ld,
                                                                               int seg_shift, int p, int q,
                                                                               T* __restrict__ partials, uint32_t rows,
                                                                               uint32_t rows_per_block) {
  using Cfg = CrossCfg<T, FH>;
  using A4 = typename Acc4<T>::type;
  constexpr int VPR = 16 / sizeof(T);
  constexpr int UPR = 2 * FH / VPR;            // 16-byte units per row
  constexpr int UNITS = Cfg::KC * UPR;
  constexpr int UPT = UNITS / Cfg::THREADS;
  static_assert(UNITS % Cfg::THREADS == 0, "chunk must split evenly");
  extern __shared__ __attribute__((aligned(16))) unsigned char cross_smem[];
  T* lds0 = reinterpret_cast<T*>(cross_smem);
  T* lds1 = lds0 + Cfg::KC * Cfg::STRIDE;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  A4 acc[Cfg::PER_WAVE];
#pragma unroll
  for (int s = 0; s < Cfg::PER_WAVE; ++s) acc[s] = A4{0, 0, 0, 0};
  const uint32_t bid = blockIdx.x;
  const uint32_t r_begin = bid * rows_per_block;
  const uint32_t r_end = min(rows, r_begin + rows_per_block);
  const T* Lr = reinterpret_cast<const T*>(L);
  const int seg_mask = (1 << seg_shift) - 1;
  const int lo = min(p, q), hi = max(p, q);
  gf4 buf[UPT];
  auto fetch = [&](uint32_t r0) {
#pragma unroll
    for (int k = 0; k < UPT; ++k) {
      const int u = tid + k * Cfg::THREADS;
      const int rr = u / UPR, f = (u % UPR) * VPR;
      const uint32_t y = r0 + rr;
      gf4 val = {0.f, 0.f, 0.f, 0.f};
      if (y < r_end) {
        const int sg = f >> seg_shift, w = f & seg_mask;   // segment (bit q, bit p) = (sg >> 1, sg & 1)
        const uint32_t x = insert2(y, lo, hi) | ((uint32_t)(sg & 1) << p) | ((uint32_t)(sg >> 1) << q);
        val = *reinterpret_cast<const gf4*>(Lr + ((size_t)x * ld) * 2 + w);
      }
      buf[k] = val;
    }
  };
  auto stage = [&](T* dst) {
#pragma unroll
    for (int k = 0; k < UPT; ++k) {
      const int u = tid + k * Cfg::THREADS;
      *reinterpret_cast<gf4*>(dst + (u / UPR) * Cfg::STRIDE + (u % UPR) * VPR) = buf[k];
    }
  };
  auto mma = [&](const T* src) { cross_chunk_mma<T, FH>(src, acc, lane, wave); };
  if (r_begin < r_end) fetch(r_begin);
  bool odd = false;
  for (uint32_t r0 = r_begin; r0 < r_end; r0 += Cfg::KC) {
    T* cur = odd ? lds1 : lds0;
    stage(cur);
    __syncthreads();
    if (r0 + Cfg::KC < r_end) fetch(r0 + Cfg::KC);
    mma(cur);
    odd = !odd;
  }
  // tile (ti, tj) at index ti NT + tj of the block's partial
  T* out = partials + (size_t)bid * Cfg::NTILE * 256;
#pragma unroll
  for (int j = 0; j < Cfg::NJ; ++j)
#pragma unroll
    for (int ti = 0; ti < Cfg::NT; ++ti) {
      const int u = ti * Cfg::NT + wave + Cfg::NW * j;
      *reinterpret_cast<A4*>(out + (size_t)u * 256 + lane * 4) = acc[j * Cfg::NT + ti];
    }
}

int gram_seg_shift(int c) {
  int s = 0;
  while ((1 << s) < 2 * c) ++s;
  return ((1 << s) == 2 * c) ? s : -1;
}

uint32_t gram_rows_per_block(int n, int nsplit, int nblocks) {
  const uint32_t rows = 1u << (n - (nsplit == 2 ? 1 : 0));
  const uint32_t chunks = (rows + kGramKC - 1) / kGramKC;
  const uint32_t cpb = (chunks + nblocks - 1) / nblocks;
  return cpb * kGramKC;
}

template <class T, int F>
static hipError_t launch_gram_batched_f(const GramJob<T>* jobs, int njobs, uint32_t blocks, hipStream_t s) {
  const size_t shm = 2 * (size_t)kGramKC * GramCfg<T, F>::STRIDE * sizeof(T);
  if (shm > 65536) {
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(gram_batched<T, F>),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((gram_batched<T, F>), dim3(blocks), dim3(GramCfg<T, F>::THREADS), shm, s, jobs, njobs);
  return hipGetLastError();
}

template <class T>
hipError_t launch_gram_batched(int F, const GramJob<T>* jobs, int njobs, uint32_t blocks, hipStream_t s) {
  if (njobs < 1 || blocks < 1) return hipErrorInvalidValue;
  switch (F) {
    case 16: return launch_gram_batched_f<T, 16>(jobs, njobs, blocks, s);
    case 32: return launch_gram_batched_f<T, 32>(jobs, njobs, blocks, s);
    case 64: return launch_gram_batched_f<T, 64>(jobs, njobs, blocks, s);
    case 128: return launch_gram_batched_f<T, 128>(jobs, njobs, blocks, s);
    case 256:
      if constexpr (sizeof(T) == 4) return launch_gram_batched_f<T, 256>(jobs, njobs, blocks, s);
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

int gram_blocks(int n, int nsplit) {
  const uint64_t rows = 1ull << (n - (nsplit == 2 ? 1 : 0));
  const uint64_t chunks = (rows + kGramKC - 1) / kGramKC;
  return (int)(chunks < 256 ? chunks : 256);   // one work-group per CU at the largest size
}

template <class T, int F>
static hipError_t launch_gram_f(const cx_t<T>* L, int n, int ld, int c, int nsplit, int q,
                                T* partials, int nblocks, hipStream_t s) {
  const uint32_t rows = 1u << (n - (nsplit == 2 ? 1 : 0));
  const uint32_t chunks = (rows + kGramKC - 1) / kGramKC;
  const uint32_t cpb = (chunks + nblocks - 1) / nblocks;
  int seg_shift = 0;
  while ((1 << seg_shift) < 2 * c) ++seg_shift;
  if ((1 << seg_shift) != 2 * c) return hipErrorInvalidValue;
  const size_t shm = 2 * (size_t)kGramKC * GramCfg<T, F>::STRIDE * sizeof(T);
  if (shm > 65536) {
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(gram_kernel<T, F>),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((gram_kernel<T, F>), dim3(nblocks), dim3(GramCfg<T, F>::THREADS), shm, s, L, ld,
                     seg_shift, nsplit, q, partials, rows, cpb * kGramKC);
  return hipGetLastError();
}

template <class T>
hipError_t launch_gram(const cx_t<T>* L, int n, int ld, int c, int nsplit, int q, T* partials,
                       int nblocks, hipStream_t s) {
  const int F = 2 * nsplit * c;
  switch (F) {
    case 16: return launch_gram_f<T, 16>(L, n, ld, c, nsplit, q, partials, nblocks, s);
    case 32: return launch_gram_f<T, 32>(L, n, ld, c, nsplit, q, partials, nblocks, s);
    case 64: return launch_gram_f<T, 64>(L, n, ld, c, nsplit, q, partials, nblocks, s);
    case 128: return launch_gram_f<T, 128>(L, n, ld, c, nsplit, q, partials, nblocks, s);
    case 256:
      if constexpr (sizeof(T) == 4) return launch_gram_f<T, 256>(L, n, ld, c, nsplit, q, partials, nblocks, s);
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

// Sum the split-K partials of one upper tile (fixed order, FP64) and convert the real tile of
// R into the complex entries of S it covers.
// Tile u of the partials (tiles_per_block tiles per block) is the real tile (ti, tj); its complex
// entries go to S[row0 + j][col0 + k] (leading dimension ldS) and, with mirror, their conjugates
// to S[col0 + k][row0 + j].
template <class T>
__device__ __forceinline__ void reduce_tile(const T* __restrict__ partials, int nblocks, int tiles_per_block, int u,
                                            int ti, int tj, double* __restrict__ S, int ldS, int row0, int col0,
                                            bool mirror) {
  __shared__ double R[16][17];
  const int e = threadIdx.x;
  const T* p = partials + (size_t)u * 256 + e;
  const size_t stride = (size_t)tiles_per_block * 256;
  // 16 partials per round, all loads issued before the first add (memory-level parallelism);
  // 16 FP64 running sums, combined in a fixed order
  constexpr int RB = 16;
  double acc[RB];
#pragma unroll
  for (int k = 0; k < RB; ++k) acc[k] = 0.0;
  int b = 0;
  for (; b + RB <= nblocks; b += RB) {
    T v[RB];
#pragma unroll
    for (int k = 0; k < RB; ++k) v[k] = p[(size_t)(b + k) * stride];
#pragma unroll
    for (int k = 0; k < RB; ++k) acc[k] += (double)v[k];
  }
  for (; b < nblocks; ++b) acc[0] += (double)p[(size_t)b * stride];
#pragma unroll
  for (int w = RB / 2; w >= 1; w /= 2)
#pragma unroll
    for (int k = 0; k < w; ++k) acc[k] += acc[k + w];
  const double sum = acc[0];
  const int lane = e >> 2, v = e & 3;
  // 16x16x4 MFMA output layout: column lane % 16; row 4 (lane / 16) + v for FP32, but
  // 4 v + lane / 16 for FP64
  const int row = (sizeof(T) == 8) ? (4 * v + (lane >> 4)) : (4 * (lane >> 4) + v);
  R[row][lane & 15] = sum;
  __syncthreads();
  if (e < 64) {
    const int jl = e >> 3, kl = e & 7;   // complex entry inside the tile
    const double re = R[2 * jl][2 * kl] + R[2 * jl + 1][2 * kl + 1];
    const double im = R[2 * jl][2 * kl + 1] - R[2 * jl + 1][2 * kl];
    const int j = row0 + 8 * ti + jl, k = col0 + 8 * tj + kl;
    S[2 * ((size_t)j * ldS + k)] = re;
    S[2 * ((size_t)j * ldS + k) + 1] = im;
    if (mirror) {
      S[2 * ((size_t)k * ldS + j)] = re;
      S[2 * ((size_t)k * ldS + j) + 1] = -im;
    }
  }
}

template <class T>
__device__ __forceinline__ void gram_reduce_body(const T* __restrict__ partials, int nblocks, int NT, int NUP,
                                                 double* __restrict__ S, int u) {
  int ti = 0, rem = u;
  while (rem >= NT - ti) {
    rem -= NT - ti;
    ++ti;
  }
  const int tj = ti + rem;
  reduce_tile<T>(partials, nblocks, NUP, u, ti, tj, S, NT * 8, 0, 0, ti != tj);
}

// G4 (4c x 4c complex, row-major) from the partials of the halves (A, B: upper tiles, nbh blocks
// each) and of the cross block C (every tile, nbc blocks): blocks [0, NUP) reduce A,
// [NUP, 2 NUP) B, then C with its conjugate transpose mirrored.
template <class T>
__global__ __launch_bounds__(256) void gram4_reduce_kernel(const T* __restrict__ part_h, int nbh,
                                                           const T* __restrict__ part_c, int nbc, int NT,
                                                           double* __restrict__ S4) {
  const int NUP = NT * (NT + 1) / 2;
  const int c2 = NT * 8;   // complex columns of one half (2c)
  int u = blockIdx.x;
  if (u < 2 * NUP) {
    const int b = u >= NUP ? 1 : 0;
    u -= b * NUP;
    int ti = 0, rem = u;
    while (rem >= NT - ti) {
      rem -= NT - ti;
      ++ti;
    }
    const int tj = ti + rem;
    reduce_tile<T>(part_h + (size_t)b * nbh * NUP * 256, nbh, NUP, u, ti, tj, S4, 2 * c2, b * c2, b * c2, ti != tj);
  } else {
    u -= 2 * NUP;
    reduce_tile<T>(part_c, nbc, NT * NT, u, u / NT, u % NT, S4, 2 * c2, 0, c2, true);
  }
}

template <class T>
__global__ __launch_bounds__(256) void gram_reduce_kernel(const T* __restrict__ partials, int nblocks,
                                                          int NT, int NUP, double* __restrict__ S) {
  gram_reduce_body<T>(partials, nblocks, NT, NUP, S, blockIdx.x);
}

template <class T>
__global__ __launch_bounds__(256) void gram_reduce_batched(const ReduceJob<T>* __restrict__ jobs, int njobs) {
  const int j = find_job(jobs, njobs, blockIdx.x);
  const ReduceJob<T>& J = jobs[j];
  gram_reduce_body<T>(J.partials, J.nblocks, J.NT, J.NUP, J.S, (int)(blockIdx.x - J.block0));
}

template <class T>
hipError_t launch_gram_reduce_batched(const ReduceJob<T>* jobs, int njobs, uint32_t blocks, hipStream_t s) {
  if (njobs < 1 || blocks < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(gram_reduce_batched<T>, dim3(blocks), dim3(256), 0, s, jobs, njobs);
  return hipGetLastError();
}

template <class T>
hipError_t launch_gram_reduce(const T* partials, int nblocks, int F, double* S, hipStream_t s) {
  const int NT = F / 16;
  const int NUP = NT * (NT + 1) / 2;
  hipLaunchKernelGGL(gram_reduce_kernel<T>, dim3(NUP), dim3(256), 0, s, partials, nblocks, NT, NUP, S);
  return hipGetLastError();
}

int gram4_blocks_halves(int n) {
  const uint64_t rows = 1ull << (n - 2);
  const uint64_t chunks = (rows + kGramKC - 1) / kGramKC;
  return (int)(chunks < 128 ? chunks : 128);
}
int gram4_blocks_cross(int n) {
  const uint64_t rows = 1ull << (n - 2);
  const uint64_t chunks = (rows + 31) / 32;
  return (int)(chunks < 256 ? chunks : 256);
}

// The whole 4-way Gram G4 = Y^H Y for c = 64 in complex64, streamed through registers.  Row y of
// Y (256 complex) is the four rows of L with the bit pair (p, q) = (0,0), (1,0), (0,1), (1,1)
// inserted, so column group G (16 columns) of Y is columns 16 (G mod 4) of the L row of segment
// G / 4.  A lane (g, m) of a wave holds Y[y0 + g][16 G + m] for the groups G it needs: these are
// the MFMA operands of the 16 x 16 blocks (I, J) over a 4-row step, so the 136 upper blocks
// accumulate in registers with no LDS: S_IJ += Y_I^H Y_J as Re += Yr_I Yr_J + Yi_I Yi_J and
// Im += Yr_I Yi_J - Yi_I Yr_J.  On a diagonal block Im is A - A^T with A = Yr_I^T Yi_I, so one
// MFMA gives it and the reduction takes the antisymmetric part.  The eight waves of a work-group
// stream the same rows (the repeated reads hit L2); wave s owns 17 blocks (two diagonal,
// 66 MFMAs a step for every wave) whose groups lie in four of the eight group pairs
// {2k, 2k+1}, so it loads 8 groups a step, three steps ahead of their MFMAs.  The ownership
// table is a balanced covering of the block triangle by unions of four pairs (found by a flow
// search; the compile-time check below proves that it covers every block once).  The
// work-group's partial is [block u][re, im][lane * 4 + v] for the entry (4 g + v, m) of block u.
constexpr int kG4Blocks = 136;                 // upper 16 x 16 blocks of the 256 x 256 complex G4
constexpr int kG4Part = kG4Blocks * 2 * 256;   // floats per work-group partial
constexpr int kG4Threads = 512;                // eight waves, two per SIMD
constexpr int kG4Own = 17;                     // blocks per wave
constexpr int kG4Split = 4;                    // partial ranges summed in parallel by the reduction

constexpr int kG4Pair[8][4] = {
    {1, 3, 4, 6},
    {0, 4, 6, 7},
    {1, 2, 4, 5},
    {1, 2, 3, 7},
    {0, 2, 3, 6},
    {0, 1, 5, 7},
    {3, 4, 5, 6},
    {0, 3, 5, 7}};
constexpr int kG4Blk[8][kG4Own][2] = {
    {{2, 2}, {3, 3}, {2, 3}, {2, 6}, {2, 7}, {2, 8}, {2, 9}, {2, 12}, {2, 13}, {3, 6}, {3, 7}, {3, 8}, {3, 9}, {3, 12}, {3, 13}, {6, 8}, {12, 13}},
    {{0, 0}, {1, 1}, {0, 8}, {0, 9}, {1, 8}, {1, 9}, {1, 13}, {8, 9}, {8, 12}, {8, 14}, {8, 15}, {9, 14}, {9, 15}, {12, 14}, {12, 15}, {13, 14}, {13, 15}},
    {{4, 4}, {5, 5}, {2, 5}, {2, 11}, {3, 4}, {3, 5}, {3, 10}, {3, 11}, {4, 5}, {4, 8}, {4, 9}, {4, 10}, {4, 11}, {5, 8}, {5, 9}, {5, 10}, {5, 11}},
    {{6, 6}, {7, 7}, {2, 4}, {2, 14}, {2, 15}, {3, 14}, {3, 15}, {4, 6}, {4, 7}, {4, 14}, {4, 15}, {5, 6}, {5, 7}, {5, 14}, {5, 15}, {6, 15}, {7, 14}},
    {{12, 12}, {13, 13}, {0, 4}, {0, 5}, {0, 12}, {0, 13}, {1, 4}, {1, 5}, {1, 7}, {1, 12}, {4, 12}, {4, 13}, {5, 12}, {5, 13}, {6, 12}, {6, 13}, {7, 12}},
    {{10, 10}, {11, 11}, {0, 2}, {0, 3}, {0, 10}, {0, 11}, {1, 2}, {1, 3}, {1, 10}, {1, 11}, {2, 10}, {10, 11}, {10, 14}, {10, 15}, {11, 14}, {11, 15}, {14, 15}},
    {{8, 8}, {9, 9}, {6, 9}, {7, 8}, {7, 9}, {7, 13}, {8, 10}, {8, 11}, {8, 13}, {9, 10}, {9, 11}, {9, 12}, {9, 13}, {10, 12}, {10, 13}, {11, 12}, {11, 13}},
    {{14, 14}, {15, 15}, {0, 1}, {0, 6}, {0, 7}, {0, 14}, {0, 15}, {1, 6}, {1, 14}, {1, 15}, {6, 7}, {6, 10}, {6, 11}, {6, 14}, {7, 10}, {7, 11}, {7, 15}}};

__host__ __device__ constexpr int g4_upper(int I, int J) { return I * 16 - I * (I - 1) / 2 + (J - I); }

// Register slot of group G in wave s's buffer (-1: not loaded by that wave).
__host__ __device__ constexpr int g4_slot(int s, int G) {
  for (int t = 0; t < 4; ++t)
    if (kG4Pair[s][t] == G >> 1) return 2 * t + (G & 1);
  return -1;
}

constexpr bool g4_table_ok() {
  int seen[16][16] = {};
  for (int s = 0; s < 8; ++s)
    for (int b = 0; b < kG4Own; ++b) {
      const int I = kG4Blk[s][b][0], J = kG4Blk[s][b][1];
      if (I < 0 || J > 15 || I > J || g4_slot(s, I) < 0 || g4_slot(s, J) < 0) return false;
      if ((b < 2) != (I == J)) return false;
      ++seen[I][J];
    }
  for (int I = 0; I < 16; ++I)
    for (int J = I; J < 16; ++J)
      if (seen[I][J] != 1) return false;
  return true;
}
static_assert(g4_table_ok(), "every upper block of G4 must have exactly one owning wave");

template <int S>
__device__ __forceinline__ void g4_load(const float2* __restrict__ L, int ld, uint32_t x0, int p, int q, int m,
                                        float2 (&v)[8]) {
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int k = kG4Pair[S][t];   // groups 2k, 2k+1: segment k / 2, columns 32 (k mod 2) + {0, 16}
    const int sg = k >> 1;
    const uint32_t x = x0 | ((uint32_t)(sg & 1) << p) | ((uint32_t)(sg >> 1) << q);
    const float2* src = L + (size_t)x * ld + 32 * (k & 1) + m;
    v[2 * t] = src[0];
    v[2 * t + 1] = src[16];
  }
}

template <int S, int B>
__device__ __forceinline__ void g4_block(const float2 (&x)[8], const float (&nxi)[8], v4f& re, v4f& im) {
  constexpr int I = kG4Blk[S][B][0], J = kG4Blk[S][B][1];
  constexpr int a = g4_slot(S, I), b = g4_slot(S, J);
  re = mfma16(x[a].x, x[b].x, re);
  re = mfma16(x[a].y, x[b].y, re);
  im = mfma16(x[a].x, x[b].y, im);
  if constexpr (I != J) im = mfma16(nxi[a], x[b].x, im);
}

template <int S>
__device__ __forceinline__ void g4_wave(const float2* __restrict__ L, int ld, int p, int q, float* __restrict__ out,
                                        uint32_t r_begin, uint32_t r_end, int lane) {
  const int m = lane & 15, g = lane >> 4;
  const int lo = p < q ? p : q, hi = p < q ? q : p;
  v4f re[kG4Own], im[kG4Own];
#pragma unroll
  for (int k = 0; k < kG4Own; ++k) {
    re[k] = v4f{0, 0, 0, 0};
    im[k] = v4f{0, 0, 0, 0};
  }
  if (r_begin >= r_end) {   // an idle work-group still writes its (zero) partial
    r_begin = r_end = 0;
  }
  auto step = [&](const float2(&x)[8]) {
    float nxi[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) nxi[k] = -x[k].y;
    static_for<kG4Own>([&](auto b) {
      constexpr int B = decltype(b)::value;
      g4_block<S, B>(x, nxi, re[B], im[B]);
    });
  };
  auto row = [&](uint32_t r) { return insert2(r + g, lo, hi); };
  // look-ahead rows past the slab's end load the current 16 rows again rather than branch
  auto ahead = [&](uint32_t r) { return r < r_end ? r : r - 16; };
  // four register buffers in turn: each step's rows are requested three steps before their MFMAs
  // (the scheduling barriers keep every load ahead of the MFMAs that follow it: left alone, the
  // scheduler sinks the loads to their first use to save registers)
  float2 b0[8], b1[8], b2[8], b3[8];
  g4_load<S>(L, ld, row(r_begin), p, q, m, b0);
  g4_load<S>(L, ld, row(r_begin + 4), p, q, m, b1);
  g4_load<S>(L, ld, row(r_begin + 8), p, q, m, b2);
  for (uint32_t r0 = r_begin; r0 < r_end; r0 += 16) {
    // every 16 steps the eight waves meet (each runs the same number of iterations): left free,
    // they drift apart until lines one wave brought into L2 are evicted before the last of the
    // four waves that read them gets there (2.5 times the bytes of L fetched; with the barrier,
    // exactly the bytes of L, in the same time)
    if (((r0 - r_begin) & 63) == 0) __syncthreads();
    g4_load<S>(L, ld, row(r0 + 12), p, q, m, b3);
    __builtin_amdgcn_sched_barrier(0);
    step(b0);
    g4_load<S>(L, ld, row(ahead(r0 + 16)), p, q, m, b0);
    __builtin_amdgcn_sched_barrier(0);
    step(b1);
    g4_load<S>(L, ld, row(ahead(r0 + 20)), p, q, m, b1);
    __builtin_amdgcn_sched_barrier(0);
    step(b2);
    g4_load<S>(L, ld, row(ahead(r0 + 24)), p, q, m, b2);
    __builtin_amdgcn_sched_barrier(0);
    step(b3);
  }
  static_for<kG4Own>([&](auto b) {
    constexpr int B = decltype(b)::value;
    constexpr int u = g4_upper(kG4Blk[S][B][0], kG4Blk[S][B][1]);
    *reinterpret_cast<v4f*>(out + (2 * u) * 256 + lane * 4) = re[B];
    *reinterpret_cast<v4f*>(out + (2 * u + 1) * 256 + lane * 4) = im[B];
  });
}

// Work-group b streams rows [b rpt, (b + 1) rpt) of Y; rows and rpt are multiples of 16, so every
// group of four 4-row steps is whole.
__global__ __launch_bounds__(kG4Threads) __attribute__((amdgpu_waves_per_eu(2, 2))) void gram4_stream_kernel(
    const float2* __restrict__ L, int ld, int p, int q, float* __restrict__ part, uint32_t rows, uint32_t rpt) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t r_begin = min(rows, blockIdx.x * rpt), r_end = min(rows, r_begin + rpt);
  float* out = part + (size_t)blockIdx.x * kG4Part;
  switch (wave) {
    case 0: g4_wave<0>(L, ld, p, q, out, r_begin, r_end, lane); break;
    case 1: g4_wave<1>(L, ld, p, q, out, r_begin, r_end, lane); break;
    case 2: g4_wave<2>(L, ld, p, q, out, r_begin, r_end, lane); break;
    case 3: g4_wave<3>(L, ld, p, q, out, r_begin, r_end, lane); break;
    case 4: g4_wave<4>(L, ld, p, q, out, r_begin, r_end, lane); break;
    case 5: g4_wave<5>(L, ld, p, q, out, r_begin, r_end, lane); break;
    case 6: g4_wave<6>(L, ld, p, q, out, r_begin, r_end, lane); break;
    default: g4_wave<7>(L, ld, p, q, out, r_begin, r_end, lane); break;
  }
}

// First reduction level: work-group (u, sp) sums, in FP64 and a fixed order, the partials
// [nb sp / kG4Split, nb (sp + 1) / kG4Split) of block u; thread t takes the four consecutive
// floats 4 t of the block's 512 (the re plane, then the im plane).  Result:
// sums[(u kG4Split + sp)][512], in the same order.
constexpr int kG4SumThreads = 128;
__global__ __launch_bounds__(kG4SumThreads) void gram4_stream_sum(const float* __restrict__ part, int nb,
                                                                  double* __restrict__ sums) {
  const int u = blockIdx.x / kG4Split, sp = blockIdx.x % kG4Split;
  const int t = threadIdx.x, off = 2 * u * 256 + 4 * t;
  const int b0 = nb * sp / kG4Split, b1 = nb * (sp + 1) / kG4Split;
  double a[4] = {0, 0, 0, 0};
  int b = b0;
  constexpr int RB = 8;   // partials in flight per thread
  for (; b + RB <= b1; b += RB) {
    v4f v[RB];
#pragma unroll
    for (int k = 0; k < RB; ++k) v[k] = *reinterpret_cast<const v4f*>(part + (size_t)(b + k) * kG4Part + off);
#pragma unroll
    for (int k = 0; k < RB; ++k)
#pragma unroll
      for (int c = 0; c < 4; ++c) a[c] += (double)v[k][c];
  }
  for (; b < b1; ++b) {
    const v4f v = *reinterpret_cast<const v4f*>(part + (size_t)b * kG4Part + off);
#pragma unroll
    for (int c = 0; c < 4; ++c) a[c] += (double)v[c];
  }
  double* dst = sums + (size_t)blockIdx.x * 512 + 4 * t;
#pragma unroll
  for (int c = 0; c < 4; ++c) dst[c] = a[c];
}

// G4 (256 x 256 complex, row-major, FP64) from the range sums: work-group u, thread e = lane * 4 + v
// for the entry (4 (lane / 16) + v, lane % 16) of block u.  Off-diagonal blocks are mirrored as
// conjugates; a diagonal block's imaginary part is A - A^T.
__global__ __launch_bounds__(256) void gram4_stream_combine(const double* __restrict__ sums,
                                                            double* __restrict__ S4) {
  const int u = blockIdx.x;
  int I = 0, rem = u;
  while (rem >= 16 - I) {
    rem -= 16 - I;
    ++I;
  }
  const int J = I + rem;
  const int e = threadIdx.x, lane = e >> 2, v = e & 3;
  const int i = 4 * (lane >> 4) + v, j = lane & 15;
  const int et = (16 * (j >> 2) + i) * 4 + (j & 3);   // entry (j, i) of the block
  const double* src = sums + (size_t)u * kG4Split * 512;
  double re = 0.0, im = 0.0, imt = 0.0;
#pragma unroll
  for (int sp = 0; sp < kG4Split; ++sp) {
    re += src[sp * 512 + e];
    im += src[sp * 512 + 256 + e];
    imt += src[sp * 512 + 256 + et];
  }
  if (I == J) im -= imt;
  const int r = 16 * I + i, c = 16 * J + j;
  S4[2 * ((size_t)r * 256 + c)] = re;
  S4[2 * ((size_t)r * 256 + c) + 1] = im;
  if (I != J) {
    S4[2 * ((size_t)c * 256 + r)] = re;
    S4[2 * ((size_t)c * 256 + r) + 1] = -im;
  }
}

size_t gram4_stream_reals(int n) {
  if (n < 6) return 0;
  const uint64_t nb = std::min<uint64_t>(256, (1ull << (n - 2)) / 16);   // one work-group per CU at most
  return (size_t)nb * kG4Part + (size_t)kG4Blocks * kG4Split * 512 * 2;
}

template <class T, int FH>
static hipError_t launch_gram4_f(const cx_t<T>* L, int n, int ld, int c, int p, int q, T* part_h, T* part_c,
                                 double* S4, int max_blocks, hipStream_t s) {
  const int seg_shift = gram_seg_shift(c);
  if (seg_shift < 0) return hipErrorInvalidValue;
  const uint32_t rows = 1u << (n - 2);
  // at most one work-group per CU the stream may use (a second round would double the time)
  const int nbh = std::max(1, std::min(gram4_blocks_halves(n), max_blocks / 2));
  const int nbc = std::max(1, std::min(gram4_blocks_cross(n), max_blocks));
  if constexpr (sizeof(T) == 4 && FH == 256) {
    // streamed form (rows a multiple of 16): the partials and then the range sums go to the one
    // region that starts at part_h (at least gram4_stream_reals(n) floats in complex64); below
    // 16 rows the tiled kernels run instead
    const int NT = FH / 16;
    const size_t room = std::max(((size_t)2 * gram4_blocks_halves(n) * (NT * (NT + 1) / 2) +
                                  (size_t)gram4_blocks_cross(n) * NT * NT) * 256,
                                 gram4_stream_reals(n));
    const size_t sums = (size_t)kG4Blocks * kG4Split * 512 * 2;   // FP64, in floats
    if (part_c != part_h + (size_t)2 * gram4_blocks_halves(n) * (NT * (NT + 1) / 2) * 256)
      return hipErrorInvalidValue;
    const size_t fit = room > sums ? (room - sums) / kG4Part : 0;
    const int nb = (int)std::min<size_t>({(size_t)max_blocks, fit, rows / 16});
    if (rows >= 16 && nb >= 1) {
      const uint32_t rpt = (((rows + nb - 1) / nb) + 15) & ~15u;
      double* sum_buf = reinterpret_cast<double*>(part_h + (size_t)nb * kG4Part);
      hipLaunchKernelGGL(gram4_stream_kernel, dim3(nb), dim3(kG4Threads), 0, s, L, ld, p, q, part_h, rows, rpt);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(gram4_stream_sum, dim3(kG4Blocks * kG4Split), dim3(kG4SumThreads), 0, s, part_h, nb,
                         sum_buf);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(gram4_stream_combine, dim3(kG4Blocks), dim3(256), 0, s, sum_buf, S4);
      return hipGetLastError();
    }
  }
  {
    const uint32_t chunks = (rows + kGramKC - 1) / kGramKC;
    const uint32_t cpb = (chunks + nbh - 1) / nbh;
    const size_t shm = 2 * (size_t)kGramKC * GramCfg<T, FH>::STRIDE * sizeof(T);
    if (shm > 65536) {
      const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(gram_halves_kernel<T, FH>),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((gram_halves_kernel<T, FH>), dim3(2 * nbh), dim3(GramCfg<T, FH>::THREADS), shm, s, L, ld,
                       seg_shift, p, q, part_h, rows, cpb * kGramKC, (uint32_t)nbh);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  {
    using Cfg = CrossCfg<T, FH>;
    const uint32_t chunks = (rows + Cfg::KC - 1) / Cfg::KC;
    const uint32_t cpb = (chunks + nbc - 1) / nbc;
    const size_t shm = 2 * (size_t)Cfg::KC * Cfg::STRIDE * sizeof(T);
    if (shm > 65536) {
      const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(gram_cross_kernel<T, FH>),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((gram_cross_kernel<T, FH>), dim3(nbc), dim3(Cfg::THREADS), shm, s, L, ld, seg_shift, p, q,
                       part_c, rows, cpb * Cfg::KC);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int NT = FH / 16;
  const int NUP = NT * (NT + 1) / 2;
  hipLaunchKernelGGL(gram4_reduce_kernel<T>, dim3(2 * NUP + NT * NT), dim3(256), 0, s, part_h, nbh, part_c, nbc, NT,
                     S4);
  return hipGetLastError();
}

template <class T>
hipError_t launch_gram4(const cx_t<T>* L, int n, int ld, int c, int p, int q, T* part_h, T* part_c, double* S4,
                        int max_blocks, hipStream_t s) {
  if (n < 2 || p == q || p < 0 || q < 0 || p >= n || q >= n || max_blocks < 2) return hipErrorInvalidValue;
  switch (4 * c) {
    case 32: return launch_gram4_f<T, 32>(L, n, ld, c, p, q, part_h, part_c, S4, max_blocks, s);
    case 64: return launch_gram4_f<T, 64>(L, n, ld, c, p, q, part_h, part_c, S4, max_blocks, s);
    case 128: return launch_gram4_f<T, 128>(L, n, ld, c, p, q, part_h, part_c, S4, max_blocks, s);
    case 256:
      if constexpr (sizeof(T) == 4) return launch_gram4_f<T, 256>(L, n, ld, c, p, q, part_h, part_c, S4, max_blocks, s);
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

template hipError_t launch_gram4<float>(const float2*, int, int, int, int, int, float*, float*, double*, int,
                                        hipStream_t);
template hipError_t launch_gram4<double>(const double2*, int, int, int, int, int, double*, double*, double*, int,
                                         hipStream_t);
template hipError_t launch_gram<float>(const float2*, int, int, int, int, int, float*, int, hipStream_t);
template hipError_t launch_gram<double>(const double2*, int, int, int, int, int, double*, int, hipStream_t);
template hipError_t launch_gram_reduce<float>(const float*, int, int, double*, hipStream_t);
template hipError_t launch_gram_reduce<double>(const double*, int, int, double*, hipStream_t);
template hipError_t launch_gram_batched<float>(int, const GramJob<float>*, int, uint32_t, hipStream_t);
template hipError_t launch_gram_batched<double>(int, const GramJob<double>*, int, uint32_t, hipStream_t);
template hipError_t launch_gram_reduce_batched<float>(const ReduceJob<float>*, int, uint32_t, hipStream_t);
template hipError_t launch_gram_reduce_batched<double>(const ReduceJob<double>*, int, uint32_t, hipStream_t);

}  // namespace lrdm
