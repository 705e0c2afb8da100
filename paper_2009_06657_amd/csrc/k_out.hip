// Outputs computed from the low-rank factor without forming rho (Sec. II.D):
//   Prob(x) = sum_v |L[x, v]|^2, <Z_i> and <Z_i Z_{i+1}> from Prob, Tr(L^H P L) for Pauli
//   strings, and inverse-CDF sampling of Prob.
// Row reductions use lane groups with shuffles; block and grid sums are FP64 in a fixed order.
#include "lrdm_internal.h"

namespace lrdm {

__device__ __forceinline__ double gsum(double v, int width) {
  for (int o = width >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Prob(x): a group of `lpr` lanes reads one row with 16-byte loads.
template <class T>
__global__ __launch_bounds__(256) void probabilities_kernel(const cx_t<T>* __restrict__ L, uint32_t rows,
                                                            int ld, int ncols, int lshift,
                                                            double* __restrict__ p) {
  constexpr int CPU = 16 / sizeof(cx_t<T>);   // complex values per 16-byte unit
  const int lpr = 1 << lshift;
  const int g = threadIdx.x & (lpr - 1);
  const uint32_t rows_per_block = 256 >> lshift;
  const uint32_t x = blockIdx.x * rows_per_block + (threadIdx.x >> lshift);
  double s = 0;
  if (x < rows) {
    const T* row = reinterpret_cast<const T*>(L + (size_t)x * ld);
    for (int u = g; u * CPU < ncols; u += lpr) {
      if constexpr (CPU == 2) {
        const float4 v = *reinterpret_cast<const float4*>(row + 4 * u);
        s += (double)v.x * v.x + (double)v.y * v.y + (double)v.z * v.z + (double)v.w * v.w;
      } else {
        const double2 v = *reinterpret_cast<const double2*>(row + 2 * u);
        s += v.x * v.x + v.y * v.y;
      }
    }
  }
  s = gsum(s, lpr);
  if (x < rows && g == 0) p[x] = s;
}

template <class T>
hipError_t launch_probabilities(const cx_t<T>* L, int n, int ld, int ncols, double* p,
                                hipStream_t s) {
  constexpr int CPU = 16 / sizeof(cx_t<T>);
  int units = (ncols + CPU - 1) / CPU;
  int lshift = 0;
  while ((1 << lshift) < units && lshift < 6) ++lshift;
  const uint32_t rows = 1u << n;
  const uint32_t rpb = 256u >> lshift;
  hipLaunchKernelGGL(probabilities_kernel<T>, dim3((rows + rpb - 1) / rpb), dim3(256), 0, s, L, rows,
                     ld, ncols, lshift, p);
  return hipGetLastError();
}

// ---------------------------------------------------------------- <Z_i>, <Z_i Z_{i+1}>
constexpr int kZMax = 64;   // accumulators: 1 + n + (n - 1) <= 60

__global__ __launch_bounds__(256) void zstats_partial_kernel(const double* __restrict__ p, int n,
                                                             uint32_t rows, double* __restrict__ part) {
  __shared__ double red[4][kZMax];
  // [0] total, [1..n] sums of P x_i, [n+1..2n-1] sums of P (x_i xor x_{i+1})
  const int nacc = 2 * n;
  double tot = 0, sb[30], sp[30];
#pragma unroll
  for (int i = 0; i < 30; ++i) sb[i] = sp[i] = 0;
  for (uint32_t x = blockIdx.x * 256 + threadIdx.x; x < rows; x += gridDim.x * 256) {
    const double v = p[x];
    tot += v;
#pragma unroll
    for (int i = 0; i < 30; ++i) {
      sb[i] += ((x >> i) & 1u) ? v : 0.0;
      sp[i] += (((x >> i) ^ (x >> (i + 1))) & 1u) ? v : 0.0;
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  {
    const double r = gsum(tot, 64);
    if (lane == 0) red[wave][0] = r;
  }
#pragma unroll
  for (int i = 0; i < 30; ++i) {
    if (i < n) {
      const double r = gsum(sb[i], 64);
      if (lane == 0) red[wave][1 + i] = r;
    }
    if (i + 1 < n) {
      const double r = gsum(sp[i], 64);
      if (lane == 0) red[wave][1 + n + i] = r;
    }
  }
  __syncthreads();
  if (threadIdx.x < nacc)
    part[(size_t)blockIdx.x * kZMax + threadIdx.x] =
        (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
}

__global__ void zstats_final_kernel(const double* __restrict__ part, int nblocks, int n,
                                    double* __restrict__ out) {
  const int i = threadIdx.x;
  if (i >= 2 * n) return;
  double s = 0;
  for (int b = 0; b < nblocks; ++b) s += part[(size_t)b * kZMax + i];
  out[i] = s;
}

template <class T>
hipError_t launch_zstats(const cx_t<T>* L, int n, int ld, int ncols, double* partials,
                         int nblocks, double* out, hipStream_t s) {
  // out[0] = trace, out[1..n] = sum P x_i, out[n+1..] = sum P (x_i xor x_{i+1});
  // partials must hold 2^n doubles of Prob followed by nblocks * 64 doubles.
  double* p = partials;
  double* part = partials + (1ull << n);
  hipError_t e = launch_probabilities<T>(L, n, ld, ncols, p, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(zstats_partial_kernel, dim3(nblocks), dim3(256), 0, s, p, n, 1u << n, part);
  hipLaunchKernelGGL(zstats_final_kernel, dim3(1), dim3(64), 0, s, part, nblocks, n, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------- Pauli strings
// Terms are sorted by X mask on the host; group g covers terms [gstart[g], gstart[g+1]) sharing
// xm = xm[gstart[g]].  For P = i^{|x&z|} X^xm Z^zm: Tr(L^H P L) = i^{|x&z|} sum_x
// (-1)^{|x & zm|} sum_v conj(L[x ^ xm, v]) L[x, v].
constexpr int kPauliRPT = 4;   // rows per thread

template <class T>
__global__ __launch_bounds__(256) void pauli_partial_kernel(const cx_t<T>* __restrict__ Lbra,
                                                            const cx_t<T>* __restrict__ L, uint32_t rows,
                                                            int ld, int ncols,
                                                            const uint64_t* __restrict__ xm,
                                                            const uint64_t* __restrict__ zm,
                                                            const int* __restrict__ gstart,
                                                            double* __restrict__ part, int nchunks) {
  __shared__ double red[4][2];
  const int grp = blockIdx.y;
  const int t0 = gstart[grp], t1 = gstart[grp + 1];
  const uint32_t xmask = (uint32_t)xm[t0];
  double cr[kPauliRPT], ci[kPauliRPT];
  uint32_t xs[kPauliRPT];
#pragma unroll
  for (int r = 0; r < kPauliRPT; ++r) {
    const uint32_t x = (blockIdx.x * kPauliRPT + r) * 256 + threadIdx.x;
    xs[r] = x;
    double sr = 0, si = 0;
    if (x < rows) {
      const cx_t<T>* a = Lbra + (size_t)(x ^ xmask) * ld;
      const cx_t<T>* b = L + (size_t)x * ld;
      for (int v = 0; v < ncols; ++v) {
        const cx_t<T> av = a[v], bv = b[v];
        sr += (double)av.x * bv.x + (double)av.y * bv.y;
        si += (double)av.x * bv.y - (double)av.y * bv.x;
      }
    }
    cr[r] = sr;
    ci[r] = si;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int t = t0; t < t1; ++t) {
    const uint32_t zmask = (uint32_t)zm[t];
    double ar = 0, ai = 0;
#pragma unroll
    for (int r = 0; r < kPauliRPT; ++r) {
      const double sg = (__popc(xs[r] & zmask) & 1) ? -1.0 : 1.0;
      ar += sg * cr[r];
      ai += sg * ci[r];
    }
    ar = gsum(ar, 64);
    ai = gsum(ai, 64);
    if (lane == 0) {
      red[wave][0] = ar;
      red[wave][1] = ai;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      part[((size_t)t * nchunks + blockIdx.x) * 2 + 0] = (red[0][0] + red[1][0]) + (red[2][0] + red[3][0]);
      part[((size_t)t * nchunks + blockIdx.x) * 2 + 1] = (red[0][1] + red[1][1]) + (red[2][1] + red[3][1]);
    }
    __syncthreads();
  }
}

__global__ void pauli_final_kernel(const double* __restrict__ part, int nchunks, int n_terms,
                                   const uint64_t* __restrict__ xm, const uint64_t* __restrict__ zm,
                                   double* __restrict__ out, int complex_out) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= n_terms) return;
  double sr = 0, si = 0;
  for (int b = 0; b < nchunks; ++b) {
    sr += part[((size_t)t * nchunks + b) * 2];
    si += part[((size_t)t * nchunks + b) * 2 + 1];
  }
  // multiply by i^{ny}; for bra == ket the real part is the expectation value
  const int ny = __popcll(xm[t] & zm[t]) & 3;
  double re, im;
  switch (ny) {
    case 0: re = sr; im = si; break;
    case 1: re = -si; im = sr; break;
    case 2: re = -sr; im = -si; break;
    default: re = si; im = -sr; break;
  }
  if (complex_out) {
    out[2 * t] = re;
    out[2 * t + 1] = im;
  } else {
    out[t] = re;
  }
}

template <class T>
hipError_t launch_pauli(const cx_t<T>* bra, const cx_t<T>* L, int n, int ld, int ncols,
                        const uint64_t* xm, const uint64_t* zm, int n_terms, double* partials,
                        int ngroups, double* out, int complex_out, hipStream_t s) {
  // partials layout: [n_terms * nchunks * 2] doubles; gstart (ngroups + 1 ints) follows zm.
  const uint32_t rows = 1u << n;
  const int nchunks = (int)((rows + 256 * kPauliRPT - 1) / (256 * kPauliRPT));
  const int* gstart = reinterpret_cast<const int*>(zm + n_terms);
  hipLaunchKernelGGL(pauli_partial_kernel<T>, dim3(nchunks, ngroups), dim3(256), 0, s, bra, L, rows,
                     ld, ncols, xm, zm, gstart, partials, nchunks);
  hipLaunchKernelGGL(pauli_final_kernel, dim3((n_terms + 255) / 256), dim3(256), 0, s, partials,
                     nchunks, n_terms, xm, zm, out, complex_out);
  return hipGetLastError();
}

// ---------------------------------------------------------------- sampling
constexpr int kScanB = 1024;   // elements per scan block (256 threads x 4)

__global__ __launch_bounds__(256) void scan_block_sums(const double* __restrict__ p, uint32_t rows,
                                                       double* __restrict__ bs) {
  __shared__ double red[256];
  const uint32_t base = blockIdx.x * kScanB + threadIdx.x * 4;
  double s = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i)
    if (base + i < rows) s += p[base + i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) bs[blockIdx.x] = red[0];
}

// exclusive scan of the block sums, one work-group, sequential per thread over a slab
__global__ __launch_bounds__(1024) void scan_offsets(double* __restrict__ bs, int nb) {
  __shared__ double slab[1024];
  const int per = (nb + 1023) / 1024;
  const int b0 = threadIdx.x * per;
  double s = 0;
  for (int i = 0; i < per; ++i)
    if (b0 + i < nb) s += bs[b0 + i];
  slab[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double run = 0;
    for (int i = 0; i < 1024; ++i) {
      const double v = slab[i];
      slab[i] = run;
      run += v;
    }
  }
  __syncthreads();
  double run = slab[threadIdx.x];
  for (int i = 0; i < per; ++i)
    if (b0 + i < nb) {
      const double v = bs[b0 + i];
      bs[b0 + i] = run;
      run += v;
    }
}

__global__ __launch_bounds__(256) void scan_apply(const double* __restrict__ p, uint32_t rows,
                                                  const double* __restrict__ bs, double* __restrict__ cdf) {
  __shared__ double th[256];
  const uint32_t base = blockIdx.x * kScanB + threadIdx.x * 4;
  double v[4], s = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    v[i] = (base + i < rows) ? p[base + i] : 0.0;
    s += v[i];
  }
  th[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double run = bs[blockIdx.x];
    for (int i = 0; i < 256; ++i) {
      const double t = th[i];
      th[i] = run;
      run += t;
    }
  }
  __syncthreads();
  double run = th[threadIdx.x];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    run += v[i];
    if (base + i < rows) cdf[base + i] = run;
  }
}

__global__ __launch_bounds__(256) void sample_search(const double* __restrict__ cdf, uint32_t rows,
                                                     const double* __restrict__ u, int count,
                                                     uint64_t* __restrict__ out) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= count) return;
  const double target = u[j] * cdf[rows - 1];
  uint32_t lo = 0, hi = rows - 1;   // smallest x with cdf[x] > target
  while (lo < hi) {
    const uint32_t mid = lo + ((hi - lo) >> 1);
    if (cdf[mid] > target)
      hi = mid;
    else
      lo = mid + 1;
  }
  out[j] = lo;
}

hipError_t launch_sample(const double* p, int n, double* cdf, double* block_sums, const double* u,
                         int count, uint64_t* out, hipStream_t s) {
  const uint32_t rows = 1u << n;
  const int nb = (int)((rows + kScanB - 1) / kScanB);
  hipLaunchKernelGGL(scan_block_sums, dim3(nb), dim3(256), 0, s, p, rows, block_sums);
  hipLaunchKernelGGL(scan_offsets, dim3(1), dim3(1024), 0, s, block_sums, nb);
  hipLaunchKernelGGL(scan_apply, dim3(nb), dim3(256), 0, s, p, rows, block_sums, cdf);
  hipLaunchKernelGGL(sample_search, dim3((count + 255) / 256), dim3(256), 0, s, cdf, rows, u, count, out);
  return hipGetLastError();
}

template hipError_t launch_probabilities<float>(const float2*, int, int, int, double*, hipStream_t);
template hipError_t launch_probabilities<double>(const double2*, int, int, int, double*, hipStream_t);
template hipError_t launch_zstats<float>(const float2*, int, int, int, double*, int, double*, hipStream_t);
template hipError_t launch_zstats<double>(const double2*, int, int, int, double*, int, double*, hipStream_t);
template hipError_t launch_pauli<float>(const float2*, const float2*, int, int, int, const uint64_t*,
                                        const uint64_t*, int, double*, int, double*, int, hipStream_t);
template hipError_t launch_pauli<double>(const double2*, const double2*, int, int, int, const uint64_t*,
                                         const uint64_t*, int, double*, int, double*, int, hipStream_t);

}  // namespace lrdm
