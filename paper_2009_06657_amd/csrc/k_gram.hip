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

template <class T, int FH>
static hipError_t launch_gram4_f(const cx_t<T>* L, int n, int ld, int c, int p, int q, T* part_h, T* part_c,
                                 double* S4, int max_blocks, hipStream_t s) {
  const int seg_shift = gram_seg_shift(c);
  if (seg_shift < 0) return hipErrorInvalidValue;
  const uint32_t rows = 1u << (n - 2);
  // at most one work-group per CU the stream may use (a second round would double the time)
  const int nbh = std::max(1, std::min(gram4_blocks_halves(n), max_blocks / 2));
  const int nbc = std::max(1, std::min(gram4_blocks_cross(n), max_blocks));
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
