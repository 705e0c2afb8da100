// Chained compressions on one qubit (Sec. II.B, Theorem 1).  After a compression on qubit q the
// new factor's split view on q is X W (X = [L_0 | L_1] of the factor before it, W the fused
// projection matrix).  When the next operation is another channel on the same qubit, its Gram
// matrix is therefore (X W)^H (X W) = W^H S W, computed here from the previous S without a pass
// over L, and the two projections compose: X W_1 W_2.  The factor is materialised once, when an
// operation that needs it arrives.
#include "lrdm_internal.h"

namespace lrdm {

// C = op(A) B for n x n complex FP64 matrices (row-major, interleaved; n a multiple of 16), op =
// identity or ^H.  A 16 x 16 tile of C per work-group: 16 rows of op(A) and 16 columns of B are
// staged through LDS in K chunks of 64, and each thread accumulates one entry over two
// interleaved partial sums.
constexpr int kZT = 16, kZK = 64;
__global__ __launch_bounds__(256) void small_zgemm(const double2* __restrict__ A, int opA_h,
                                                   const double2* __restrict__ B, double2* __restrict__ C, int n) {
  __shared__ double2 As[kZT][kZK + 1];
  __shared__ double2 Bs[kZK][kZT + 1];
  const int tid = threadIdx.x, ti = tid / kZT, tj = tid % kZT;
  const int I = blockIdx.y * kZT, J = blockIdx.x * kZT;
  double sr0 = 0, si0 = 0, sr1 = 0, si1 = 0;
  for (int k0 = 0; k0 < n; k0 += kZK) {
    const int kc = min(kZK, n - k0);
    for (int e = tid; e < kZT * kZK; e += 256) {
      if (opA_h) {   // (A^H)[I + r][k] = conj(A[k][I + r]): consecutive threads read consecutive r
        const int r = e % kZT, k = e / kZT;
        if (k < kc) {
          const double2 v = A[(size_t)(k0 + k) * n + I + r];
          As[r][k] = make_double2(v.x, -v.y);
        }
      } else {
        const int r = e / kZK, k = e % kZK;
        if (k < kc) As[r][k] = A[(size_t)(I + r) * n + k0 + k];
      }
      const int k = e / kZT, c = e % kZT;
      if (k < kc) Bs[k][c] = B[(size_t)(k0 + k) * n + J + c];
    }
    __syncthreads();
    for (int k = 0; k + 1 < kc; k += 2) {
      const double2 a0 = As[ti][k], b0 = Bs[k][tj], a1 = As[ti][k + 1], b1 = Bs[k + 1][tj];
      sr0 = fma(a0.x, b0.x, fma(-a0.y, b0.y, sr0));
      si0 = fma(a0.x, b0.y, fma(a0.y, b0.x, si0));
      sr1 = fma(a1.x, b1.x, fma(-a1.y, b1.y, sr1));
      si1 = fma(a1.x, b1.y, fma(a1.y, b1.x, si1));
    }
    if (kc & 1) {
      const double2 a0 = As[ti][kc - 1], b0 = Bs[kc - 1][tj];
      sr0 = fma(a0.x, b0.x, fma(-a0.y, b0.y, sr0));
      si0 = fma(a0.x, b0.y, fma(a0.y, b0.x, si0));
    }
    __syncthreads();
  }
  C[(size_t)(I + ti) * n + J + tj] = make_double2(sr0 + sr1, si0 + si1);
}

// S = (S + S^H) / 2 in place (one thread per entry pair i <= j)
__global__ __launch_bounds__(256) void hermitian_part(double2* __restrict__ S, int n) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= n * n) return;
  const int i = e / n, j = e % n;
  if (i > j) return;
  if (i == j) {
    S[(size_t)i * n + i].y = 0.0;
    return;
  }
  const double2 a = S[(size_t)i * n + j], b = S[(size_t)j * n + i];
  const double2 h = make_double2(0.5 * (a.x + b.x), 0.5 * (a.y - b.y));
  S[(size_t)i * n + j] = h;
  S[(size_t)j * n + i] = make_double2(h.x, -h.y);
}

template <class T>
__global__ __launch_bounds__(256) void copy_cast(const double* __restrict__ src, double* __restrict__ dst64,
                                                 cx_t<T>* __restrict__ dstT, int count) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= count) return;
  const double re = src[2 * e], im = src[2 * e + 1];
  dst64[2 * e] = re;
  dst64[2 * e + 1] = im;
  cx_t<T> o;
  o.x = (T)re;
  o.y = (T)im;
  dstT[e] = o;
}

hipError_t launch_chain_gram(double* S, const double* W, double* tmp, int n, hipStream_t s) {
  if (n < kZT || n > 256 || n % kZT) return hipErrorInvalidValue;
  const dim3 grid(n / kZT, n / kZT);
  auto* S2 = reinterpret_cast<double2*>(S);
  auto* T2 = reinterpret_cast<double2*>(tmp);
  const auto* W2 = reinterpret_cast<const double2*>(W);
  hipLaunchKernelGGL(small_zgemm, grid, dim3(256), 0, s, S2, 0, W2, T2, n);   // tmp = S W
  hipLaunchKernelGGL(small_zgemm, grid, dim3(256), 0, s, W2, 1, T2, S2, n);   // S = W^H tmp
  hipLaunchKernelGGL(hermitian_part, dim3((n * n + 255) / 256), dim3(256), 0, s, S2, n);
  return hipGetLastError();
}

template <class T>
hipError_t launch_chain_compose(double* Wp, const double* Wn, double* tmp, cx_t<T>* Wt, int n, hipStream_t s) {
  if (n < kZT || n > 256 || n % kZT) return hipErrorInvalidValue;
  const dim3 grid(n / kZT, n / kZT);
  hipLaunchKernelGGL(small_zgemm, grid, dim3(256), 0, s, reinterpret_cast<const double2*>(Wp), 0,
                     reinterpret_cast<const double2*>(Wn), reinterpret_cast<double2*>(tmp), n);   // tmp = Wp Wn
  hipLaunchKernelGGL(copy_cast<T>, dim3((n * n + 255) / 256), dim3(256), 0, s, tmp, Wp, Wt, n * n);
  return hipGetLastError();
}

// ------------------------------------------------------------ split Gram across a projection
// The projection on qubit p maps row y of the split view on p to [L'_0 | L'_1](y) = X_p(y) W
// (W of size 2c x 2c, column block c' = output half bit p = c').  For a second qubit q, with
// G4 the Gram matrix of X4 = [X_0 | X_1], X_b the split view on p over the rows with bit q = b
// (row-major 4c x 4c, index (b, bit p, v)), the split Gram on q of the projected factor is
//     S_bb' = sum_c' W_c'^H G4_bb' W_c'   (c x c blocks, b, b' the bit q),
// since bit q is untouched by the projection.  Computed in two FP64 steps: T_bb' = G4_bb' W
// (three 2c x 2c products: b b' = 00, 01, 11), then S_bb' from the diagonal blocks of W^H T_bb',
// S_10 = S_01^H, and the Hermitian part of the whole.

// Accumulate one entry of C = op(A) B over k in [0, K) for a 16 x 16 output tile at (I, J) with
// bounds M x N; A is row-major with leading dimension lda (op = ^H reads A[k][i]).
__device__ __forceinline__ void ztile_acc(const double2* __restrict__ A, int lda, int opA_h,
                                          const double2* __restrict__ B, int ldb, int I, int J, int M, int N, int K,
                                          double& sr, double& si) {
  __shared__ double2 As[kZT][kZK + 1];
  __shared__ double2 Bs[kZK][kZT + 1];
  const int tid = threadIdx.x, ti = tid / kZT, tj = tid % kZT;
  for (int k0 = 0; k0 < K; k0 += kZK) {
    const int kc = min(kZK, K - k0);
    for (int e = tid; e < kZT * kZK; e += 256) {
      if (opA_h) {
        const int r = e % kZT, k = e / kZT;
        if (k < kc) {
          const double2 v = (I + r < M) ? A[(size_t)(k0 + k) * lda + I + r] : make_double2(0.0, 0.0);
          As[r][k] = make_double2(v.x, -v.y);
        }
      } else {
        const int r = e / kZK, k = e % kZK;
        if (k < kc) As[r][k] = (I + r < M) ? A[(size_t)(I + r) * lda + k0 + k] : make_double2(0.0, 0.0);
      }
      const int k = e / kZT, c = e % kZT;
      if (k < kc) Bs[k][c] = (J + c < N) ? B[(size_t)(k0 + k) * ldb + J + c] : make_double2(0.0, 0.0);
    }
    __syncthreads();
    for (int k = 0; k < kc; ++k) {
      const double2 a = As[ti][k], b = Bs[k][tj];
      sr = fma(a.x, b.x, fma(-a.y, b.y, sr));
      si = fma(a.x, b.y, fma(a.y, b.x, si));
    }
    __syncthreads();
  }
}

// T_z = G4_{b b'} W for z = 0, 1, 2 <-> (b, b') = (0, 0), (0, 1), (1, 1)
__global__ __launch_bounds__(256) void pair_t_kernel(const double2* __restrict__ G4, const double2* __restrict__ W,
                                                     double2* __restrict__ T, int c2) {
  const int z = blockIdx.z, b = z >> 1, bp = (z + 1) >> 1;
  const int I = blockIdx.y * kZT, J = blockIdx.x * kZT;
  double sr = 0, si = 0;
  ztile_acc(G4 + (size_t)b * c2 * (2 * c2) + (size_t)bp * c2, 2 * c2, 0, W, c2, I, J, c2, c2, c2, sr, si);
  const int ti = threadIdx.x / kZT, tj = threadIdx.x % kZT;
  T[(size_t)z * c2 * c2 + (size_t)(I + ti) * c2 + J + tj] = make_double2(sr, si);
}

// S_{b b'}[j][j'] = sum_c' sum_k conj(W[k][c' c + j]) T_z[k][c' c + j']
__global__ __launch_bounds__(256) void pair_fold_kernel(const double2* __restrict__ W, const double2* __restrict__ T,
                                                        double2* __restrict__ S, int c) {
  const int c2 = 2 * c;
  const int z = blockIdx.z, b = z >> 1, bp = (z + 1) >> 1;
  const int I = blockIdx.y * kZT, J = blockIdx.x * kZT;
  double sr = 0, si = 0;
  const double2* Tz = T + (size_t)z * c2 * c2;
  for (int cp = 0; cp < 2; ++cp) ztile_acc(W + cp * c, c2, 1, Tz + cp * c, c2, I, J, c, c, c2, sr, si);
  const int ti = threadIdx.x / kZT, tj = threadIdx.x % kZT;
  const int j = I + ti, jp = J + tj;
  if (j < c && jp < c) {
    S[(size_t)(b * c + j) * c2 + bp * c + jp] = make_double2(sr, si);
    if (b != bp) S[(size_t)(bp * c + jp) * c2 + b * c + j] = make_double2(sr, -si);
  }
}

hipError_t launch_pair_transform(const double* G4, const double* W, double* T, double* S, int c, hipStream_t s) {
  const int c2 = 2 * c;
  if (c < 8 || c > 64 || (c & (c - 1))) return hipErrorInvalidValue;
  const auto* G2 = reinterpret_cast<const double2*>(G4);
  const auto* W2 = reinterpret_cast<const double2*>(W);
  auto* T2 = reinterpret_cast<double2*>(T);
  auto* S2 = reinterpret_cast<double2*>(S);
  hipLaunchKernelGGL(pair_t_kernel, dim3(c2 / kZT, c2 / kZT, 3), dim3(256), 0, s, G2, W2, T2, c2);
  hipLaunchKernelGGL(pair_fold_kernel, dim3((c + kZT - 1) / kZT, (c + kZT - 1) / kZT, 3), dim3(256), 0, s, W2, T2, S2,
                     c);
  hipLaunchKernelGGL(hermitian_part, dim3((c2 * c2 + 255) / 256), dim3(256), 0, s, S2, c2);
  return hipGetLastError();
}

template hipError_t launch_chain_compose<float>(double*, const double*, double*, float2*, int, hipStream_t);
template hipError_t launch_chain_compose<double>(double*, const double*, double*, double2*, int, hipStream_t);

}  // namespace lrdm
