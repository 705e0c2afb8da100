// Chained compressions on one qubit (Sec. II.B, Theorem 1).  After a compression on qubit q the
// new factor's split view on q is X W (X = [L_0 | L_1] of the factor before it, W the fused
// projection matrix).  When the next operation is another channel on the same qubit, its Gram
// matrix is therefore (X W)^H (X W) = W^H S W, computed here from the previous S without a pass
// over L, and the two projections compose: X W_1 W_2.  The factor is materialised once, when an
// operation that needs it arrives.
#include "lrdm_internal.h"

namespace lrdm {

// C = op(A) B for n x n complex FP64 matrices (row-major, interleaved), op = identity or ^H;
// with herm = 1 the Hermitian part (C + C^H) / 2 of the product is stored.
__global__ __launch_bounds__(256) void small_zgemm(const double* __restrict__ A, int opA_h,
                                                   const double* __restrict__ B, double* __restrict__ C,
                                                   int n, int herm) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= n * n) return;
  const int i = e / n, j = e % n;
  auto entry = [&](int r, int c) {
    double sr = 0, si = 0;
    for (int k = 0; k < n; ++k) {
      double ar, ai;
      if (opA_h) {   // (A^H)[r][k] = conj(A[k][r])
        ar = A[2 * (k * n + r)];
        ai = -A[2 * (k * n + r) + 1];
      } else {
        ar = A[2 * (r * n + k)];
        ai = A[2 * (r * n + k) + 1];
      }
      const double br = B[2 * (k * n + c)], bi = B[2 * (k * n + c) + 1];
      sr += ar * br - ai * bi;
      si += ar * bi + ai * br;
    }
    return make_double2(sr, si);
  };
  double2 v = entry(i, j);
  if (herm) {
    const double2 t = entry(j, i);
    v = make_double2(0.5 * (v.x + t.x), 0.5 * (v.y - t.y));
  }
  C[2 * e] = v.x;
  C[2 * e + 1] = v.y;
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
  if (n < 1 || n > 256) return hipErrorInvalidValue;
  const unsigned blocks = (unsigned)((n * n + 255) / 256);
  hipLaunchKernelGGL(small_zgemm, dim3(blocks), dim3(256), 0, s, S, 0, W, tmp, n, 0);   // tmp = S W
  hipLaunchKernelGGL(small_zgemm, dim3(blocks), dim3(256), 0, s, W, 1, tmp, S, n, 1);   // S = herm(W^H tmp)
  return hipGetLastError();
}

template <class T>
hipError_t launch_chain_compose(double* Wp, const double* Wn, double* tmp, cx_t<T>* Wt, int n, hipStream_t s) {
  if (n < 1 || n > 256) return hipErrorInvalidValue;
  const unsigned blocks = (unsigned)((n * n + 255) / 256);
  hipLaunchKernelGGL(small_zgemm, dim3(blocks), dim3(256), 0, s, Wp, 0, Wn, tmp, n, 0);  // tmp = Wp Wn
  hipLaunchKernelGGL(copy_cast<T>, dim3(blocks), dim3(256), 0, s, tmp, Wp, Wt, n * n);
  return hipGetLastError();
}

template hipError_t launch_chain_compose<float>(double*, const double*, double*, float2*, int, hipStream_t);
template hipError_t launch_chain_compose<double>(double*, const double*, double*, double2*, int, hipStream_t);

}  // namespace lrdm
