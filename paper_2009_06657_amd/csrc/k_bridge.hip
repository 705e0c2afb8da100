// Kernels between representations of the state (Sec. II.A, II.D): a sparse superposition as the
// initial factor (the other initial states Algorithm 1 admits), and rho = L L^H (Eq. "low rank
// decomposition") written in the full-rank comparator's layout, for the switch to full density
// matrix evolution once the intermediate rank reaches 2^N (Sec. II.C).
#include "lrdm_internal.h"

namespace lrdm {

template <class T>
__global__ void set_sparse_kernel(cx_t<T>* __restrict__ L, int ld, const uint64_t* __restrict__ idx,
                                  const double* __restrict__ amp, int count) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= count) return;
  cx_t<T> v;
  v.x = (T)amp[2 * i];
  v.y = (T)amp[2 * i + 1];
  L[(size_t)idx[i] * ld] = v;
}

template <class T>
hipError_t launch_set_sparse(cx_t<T>* L, int ld, const uint64_t* idx, const double* amp, int count, hipStream_t s) {
  if (count < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(set_sparse_kernel<T>, dim3((count + 255) / 256), dim3(256), 0, s, L, ld, idx, amp, count);
  return hipGetLastError();
}

// One 16 x 16 tile of rho per work-group: rows x0 .. x0 + 15, columns y0 .. y0 + 15; the two row
// blocks of L are staged through LDS 16 columns at a time and each thread sums its entry in FP64.
constexpr int kBt = 16;
template <class T>
__global__ __launch_bounds__(256) void lr_to_full_kernel(const cx_t<T>* __restrict__ L, uint32_t rows, int ld,
                                                         int ncols, float2* __restrict__ rho) {
  __shared__ double2 lx[kBt][kBt + 1], ly[kBt][kBt + 1];
  const int tx = threadIdx.x & (kBt - 1), ty = threadIdx.x / kBt;
  const uint32_t x0 = blockIdx.y * kBt, y0 = blockIdx.x * kBt;
  double re = 0.0, im = 0.0;
  for (int c0 = 0; c0 < ncols; c0 += kBt) {
    const int col = c0 + tx;
    const bool cin = col < ncols;
    double2 a = {0.0, 0.0}, b = {0.0, 0.0};
    if (cin && x0 + ty < rows) {
      const cx_t<T> v = L[(size_t)(x0 + ty) * ld + col];
      a = double2{(double)v.x, (double)v.y};
    }
    if (cin && y0 + ty < rows) {
      const cx_t<T> v = L[(size_t)(y0 + ty) * ld + col];
      b = double2{(double)v.x, (double)v.y};
    }
    lx[ty][tx] = a;
    ly[ty][tx] = b;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kBt; ++k) {
      const double2 p = lx[ty][k], q = ly[tx][k];   // L[x, k] conj(L[y, k])
      re = fma(p.x, q.x, fma(p.y, q.y, re));
      im = fma(p.y, q.x, fma(-p.x, q.y, im));
    }
    __syncthreads();
  }
  const uint32_t x = x0 + ty, y = y0 + tx;
  if (x < rows && y < rows) rho[(size_t)x * rows + y] = float2{(float)re, (float)im};
}

template <class T>
hipError_t launch_lr_to_full(const cx_t<T>* L, int n, int ld, int ncols, float2* rho, hipStream_t s) {
  if (n < 1 || n > 16 || ncols < 1 || ncols > ld) return hipErrorInvalidValue;
  const uint32_t rows = 1u << n, tiles = (rows + kBt - 1) / kBt;
  hipLaunchKernelGGL(lr_to_full_kernel<T>, dim3(tiles, tiles), dim3(256), 0, s, L, rows, ld, ncols, rho);
  return hipGetLastError();
}

template hipError_t launch_set_sparse<float>(float2*, int, const uint64_t*, const double*, int, hipStream_t);
template hipError_t launch_set_sparse<double>(double2*, int, const uint64_t*, const double*, int, hipStream_t);
template hipError_t launch_lr_to_full<float>(const float2*, int, int, int, float2*, hipStream_t);
template hipError_t launch_lr_to_full<double>(const double2*, int, int, int, float2*, hipStream_t);

}  // namespace lrdm
