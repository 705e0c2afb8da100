// Reverse sweep for energy gradients through the low-rank evolution.
//
// The paper defines the forward map only; these kernels give its exact derivative for an energy
// E = sum_t c_t Tr(L^H P_t L) of the final factor (observable formula of Sec. II.D), with the
// adjoint Lbar defined by dE = 2 Re Tr(Lbar^H dL):
//   * seed Lbar = H L (pauli_apply_kernel);
//   * truncation L_n = c L' V_K with L' = [E_1 L | ... | E_m L] (Eq. "low rank evolution K",
//     Theorem 1): with Z = V_D^H (c L'^H Lbar_n), Zhat_ji = Z_ji / (lambda_i - lambda_j) (i kept,
//     j discarded), Ghat = V_K Zhat^H V_D^H, s = Re Tr(Lbar_n^H L_n) and
//     M = Ghat + Ghat^H - s c^2 V_K V_K^H (last term when renormalising),
//         Lbar' = c Lbar_n V_K^H + L' M,   Lbar = sum_a E_a^H Lbar'_a.
//     This is the first-order change of the kept spectral projector of G = L'^H L' and of
//     c^2 = 1 / Tr(P_K G).
//
// Like the forward compression, the channel is never materialised.  On the split view
// X = [L_0 | L_1] (rows with bit q = 0 | = 1) and Ybar = [Lbar_n0 | Lbar_n1]:
//     [Lbar_0 | Lbar_1] = Ybar P + X Q,
//     P[(b', j), (b, v)] = c sum_a conj(E_a[b'][b]) conj(V[(a, v), j])      (j < k),
//     Q[(b2, v2), (b, v)] = sum_{b', a2, a} E_a2[b'][b2] M[(a2, v2), (a, v)] conj(E_a[b'][b]),
// and L'^H Lbar_n = sum_{b, b'} conj(E_a[b'][b]) C[(b, v), (b', j)] with the cross Gram matrix
// C = X^H Ybar.  Three kernels: the cross Gram (split-K over rows, fixed-order FP64 reduction),
// one FP64 work-group for the small matrices, and the two-operand projection written in place.
#include "lrdm_internal.h"

namespace lrdm {
namespace {

struct zd {
  double x, y;
};
__device__ __forceinline__ zd zmake(double a, double b) { return zd{a, b}; }
__device__ __forceinline__ zd zplus(zd a, zd b) { return zd{a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ zd ztimes(zd a, zd b) { return zd{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ __forceinline__ zd zbar(zd a) { return zd{a.x, -a.y}; }
__device__ __forceinline__ zd zget(const double* p, size_t i) { return zd{p[2 * i], p[2 * i + 1]}; }
__device__ __forceinline__ void zput(double* p, size_t i, zd v) {
  p[2 * i] = v.x;
  p[2 * i + 1] = v.y;
}
__device__ __forceinline__ uint32_t with_bit(uint32_t y, int q, int b) {
  return (((y >> q) << (q + 1)) | (y & ((1u << q) - 1u))) | ((uint32_t)b << q);
}
__device__ __forceinline__ zd echan(const Channel& ch, int a, int r, int c) {
  return zd{ch.e[a][r][c][0], ch.e[a][r][c][1]};
}

// rows per split-K chunk of the cross Gram: at least 64, at most kAdjChunks chunks
__host__ inline uint32_t adj_rows_per_chunk(uint32_t half_rows) {
  const uint32_t by_count = (half_rows + kAdjChunks - 1) / kAdjChunks;
  return by_count > 64u ? by_count : 64u;
}

}  // namespace

// ---------------------------------------------------------------- H L
template <class T>
__global__ __launch_bounds__(256) void pauli_apply_kernel(cx_t<T>* __restrict__ dst,
                                                          const cx_t<T>* __restrict__ src, int ld,
                                                          int cshift, uint32_t rows,
                                                          const uint64_t* __restrict__ xm,
                                                          const uint64_t* __restrict__ zm,
                                                          const double* __restrict__ coeff,
                                                          int n_terms) {
  const uint64_t gid = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  const uint32_t x = (uint32_t)(gid >> cshift);
  const int v = (int)(gid & ((1u << cshift) - 1u));
  if (x >= rows) return;
  double ar = 0, ai = 0;
  for (int t = 0; t < n_terms; ++t) {
    const uint32_t xmask = (uint32_t)xm[t], zmask = (uint32_t)zm[t];
    const uint32_t y = x ^ xmask;
    // (P L)[x] = i^{|xm & zm|} (-1)^{|y & zm|} L[y] with y = x ^ xm
    const int ph = ((__popc(xmask & zmask) & 3) + 2 * (__popc(y & zmask) & 1)) & 3;
    const cx_t<T> s = src[(size_t)y * ld + v];
    const double c = coeff[t];
    double pr, pi;
    switch (ph) {
      case 0: pr = s.x; pi = s.y; break;
      case 1: pr = -(double)s.y; pi = s.x; break;
      case 2: pr = -(double)s.x; pi = -(double)s.y; break;
      default: pr = s.y; pi = -(double)s.x; break;
    }
    ar += c * pr;
    ai += c * pi;
  }
  cx_t<T> o;
  o.x = (T)ar;
  o.y = (T)ai;
  dst[(size_t)x * ld + v] = o;
}

template <class T>
hipError_t launch_pauli_apply(cx_t<T>* dst, const cx_t<T>* src, int n, int ld, int ncols,
                              const uint64_t* xm, const uint64_t* zm, const double* coeff,
                              int n_terms, hipStream_t s) {
  if (ncols < 1 || (ncols & (ncols - 1))) return hipErrorInvalidValue;
  int cshift = 0;
  while ((1 << cshift) < ncols) ++cshift;
  const uint32_t rows = 1u << n;
  const uint64_t total = (uint64_t)rows << cshift;
  hipLaunchKernelGGL(pauli_apply_kernel<T>, dim3((uint32_t)((total + 255) / 256)), dim3(256), 0, s, dst,
                     src, ld, cshift, rows, xm, zm, coeff, n_terms);
  return hipGetLastError();
}

// ---------------------------------------------------------------- C = X^H Ybar (split view)
// Thread = one entry (i, j) of C, i = (b, v), j = (b', w); block row blockIdx.x sums a slice of
// rows y.  Partials are FP64 and reduced in a fixed order.
template <class T>
__global__ __launch_bounds__(256) void cross_gram_kernel(const cx_t<T>* __restrict__ X,
                                                         const cx_t<T>* __restrict__ Y, int ld, int c,
                                                         int q, uint32_t half_rows, uint32_t rpc,
                                                         double* __restrict__ part) {
  const int w2 = 2 * c, nent = w2 * w2;
  const int e = blockIdx.y * 256 + threadIdx.x;
  if (e >= nent) return;
  const int i = e / w2, j = e % w2;
  const int b = i / c, v = i % c, bp = j / c, w = j % c;
  const uint32_t y0 = blockIdx.x * rpc;
  const uint32_t y1 = min(y0 + rpc, half_rows);
  double sr = 0, si = 0;
  for (uint32_t y = y0; y < y1; ++y) {
    const cx_t<T> a = X[(size_t)with_bit(y, q, b) * ld + v];
    const cx_t<T> g = Y[(size_t)with_bit(y, q, bp) * ld + w];
    sr += (double)a.x * g.x + (double)a.y * g.y;
    si += (double)a.x * g.y - (double)a.y * g.x;
  }
  part[((size_t)blockIdx.x * nent + e) * 2] = sr;
  part[((size_t)blockIdx.x * nent + e) * 2 + 1] = si;
}

__global__ __launch_bounds__(256) void cross_gram_reduce_kernel(const double* __restrict__ part, int nchunks,
                                                                int nent, double* __restrict__ C) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= nent) return;
  double sr = 0, si = 0;
  for (int k = 0; k < nchunks; ++k) {
    sr += part[((size_t)k * nent + e) * 2];
    si += part[((size_t)k * nent + e) * 2 + 1];
  }
  C[2 * e] = sr;
  C[2 * e + 1] = si;
}

// S = X^H X of the split view with products and sums in FP64 (exact products of complex64
// entries): the Gram matrix of a recorded compression, whose null space then stays at the FP64
// rounding level so that the reverse sweep can recognise it.
template <class T>
hipError_t launch_gram_exact(const cx_t<T>* L, int n, int ld, int c, int q, double* part, double* S,
                             hipStream_t s) {
  if (c < 1 || 2 * c > 128 || n < 1 || q < 0 || q >= n) return hipErrorInvalidValue;
  const uint32_t half_rows = 1u << (n - 1);
  const int w2 = 2 * c, nent = w2 * w2;
  const uint32_t rpc = adj_rows_per_chunk(half_rows);
  const int nchunks = (int)((half_rows + rpc - 1) / rpc);
  hipLaunchKernelGGL(cross_gram_kernel<T>, dim3(nchunks, (nent + 255) / 256), dim3(256), 0, s, L, L, ld, c,
                     q, half_rows, rpc, part);
  hipLaunchKernelGGL(cross_gram_reduce_kernel, dim3((nent + 255) / 256), dim3(256), 0, s, part, nchunks, nent, S);
  return hipGetLastError();
}

// ---------------------------------------------------------------- small FP64 matrices
// One work-group of kAdjSmallThreads.  The recorded eigenvectors V (N x N, N <= kRecMaxN), H
// (later U) and Zhat live in LDS (4.5 N^2 doubles, 144 KiB at N = 64); M goes through the
// workspace, written and read by this work-group only.  Phases are separated by barriers.
constexpr int kAdjSmallThreads = 1024;
inline size_t adj_small_shm(int N) { return (size_t)(4 * N * N + (N * N) / 2) * sizeof(double); }

template <class T>
__global__ __launch_bounds__(kAdjSmallThreads) void adj_small_kernel(const double* __restrict__ rec, Channel ch, int c,
                                                                     AdjBufs b) {
  extern __shared__ __attribute__((aligned(16))) double adj_dyn[];
  __shared__ double red[kAdjSmallThreads / 64];
  constexpr int NT = kAdjSmallThreads;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int k = (int)rec[0];
  const double cs = rec[1];
  const int N = (int)rec[2];
  const int renorm = (int)rec[4];
  const int m = ch.m;
  const int w2 = 2 * c;
  const double* lam = rec + kRecHeader;
  const double* Vg = rec + kRecHeader + N;   // complex N x N
  const int nd = N - k;
  double* Vs = adj_dyn;                      // N x N complex
  double* HU = Vs + 2 * N * N;               // N x k complex: H, then U
  double* Zs = HU + 2 * N * N;               // nd x k complex (nd k <= N^2 / 4)

  for (int e = tid; e < 2 * N * N; e += NT) Vs[e] = Vg[e];
  // 1. H[(a, v), j] = (L'^H Lbar_n)[(a, v), j] = sum_{b, b'} conj(E_a[b'][b]) C[(b, v), (b', j)]
  for (int e = tid; e < N * k; e += NT) {
    const int row = e / k, j = e % k;
    const int a = row / c, v = row % c;
    zd acc = zmake(0, 0);
    for (int bb = 0; bb < 2; ++bb)
      for (int bp = 0; bp < 2; ++bp)
        acc = zplus(acc, ztimes(zbar(echan(ch, a, bp, bb)), zget(b.C, (size_t)(bb * c + v) * w2 + (bp * c + j))));
    zput(HU, e, acc);
  }
  __syncthreads();
  // 2. Zhat[d, i] = c (V_D^H H)[d, i] / (lambda_i - lambda_{k+d});  s = c Re sum_j (H^H V_K)_jj
  const double tiny = 1e-13 * fmax(rec[3], 1e-300);
  for (int e = tid; e < nd * k; e += NT) {
    const int d = e / k, i = e % k;
    zd acc = zmake(0, 0);
    for (int row = 0; row < N; ++row)
      acc = zplus(acc, ztimes(zbar(zget(Vs, row * N + k + d)), zget(HU, row * k + i)));
    const double den = lam[i] - lam[k + d];
    const double f = (fabs(den) > tiny) ? cs / den : 0.0;
    zput(Zs, e, zmake(acc.x * f, acc.y * f));
  }
  double sp = 0;
  for (int e = tid; e < N * k; e += NT) {
    const int row = e / k, j = e % k;
    const zd h = zget(HU, e), vv = zget(Vs, row * N + j);
    sp += h.x * vv.x + h.y * vv.y;   // Re(conj(h) v)
  }
  for (int o = 32; o > 0; o >>= 1) sp += __shfl_xor(sp, o, 64);
  if (lane == 0) red[wave] = sp;
  __syncthreads();
  double sval = 0;
  for (int w = 0; w < NT / 64; ++w) sval += red[w];   // fixed order
  sval *= cs;
  // 3. U = V_D Zhat (N x k), over H:  V_K Zhat^H V_D^H = V_K U^H
  for (int e = tid; e < N * k; e += NT) {
    const int r = e / k, i = e % k;
    zd acc = zmake(0, 0);
    for (int d = 0; d < nd; ++d) acc = zplus(acc, ztimes(zget(Vs, r * N + k + d), zget(Zs, d * k + i)));
    zput(HU, e, acc);
  }
  __syncthreads();
  // 4. M = Ghat + Ghat^H - s c^2 V_K V_K^H with Ghat = V_K U^H
  const double sc2 = renorm ? sval * cs * cs : 0.0;
  for (int e = tid; e < N * N; e += NT) {
    const int r1 = e / N, r2 = e % N;
    zd acc = zmake(0, 0);
    for (int i = 0; i < k; ++i) {
      const zd v1 = zget(Vs, r1 * N + i), v2 = zget(Vs, r2 * N + i);
      const zd u1 = zget(HU, r1 * k + i), u2 = zget(HU, r2 * k + i);
      acc = zplus(acc, zplus(ztimes(v1, zbar(u2)), ztimes(u1, zbar(v2))));
      if (sc2 != 0.0) {
        const zd p = ztimes(v1, zbar(v2));
        acc = zplus(acc, zmake(-sc2 * p.x, -sc2 * p.y));
      }
    }
    zput(b.M, e, acc);
  }
  __syncthreads();
  const double* V = Vs;
  // 6. P and Q in the bulk precision
  cx_t<T>* P = static_cast<cx_t<T>*>(b.P);
  cx_t<T>* Q = static_cast<cx_t<T>*>(b.Q);
  for (int e = tid; e < w2 * w2; e += NT) {
    const int rr = e / w2, cc = e % w2;
    const int bo = cc / c, v = cc % c;   // output column (b, v)
    {
      const int bp = rr / c, j = rr % c;
      zd acc = zmake(0, 0);
      if (j < k)
        for (int a = 0; a < m; ++a)
          acc = zplus(acc, ztimes(zbar(echan(ch, a, bp, bo)), zbar(zget(V, (size_t)(a * c + v) * N + j))));
      cx_t<T> o;
      o.x = (T)(cs * acc.x);
      o.y = (T)(cs * acc.y);
      P[e] = o;
    }
    {
      const int b2 = rr / c, v2 = rr % c;
      zd acc = zmake(0, 0);
      for (int bp = 0; bp < 2; ++bp)
        for (int a2 = 0; a2 < m; ++a2) {
          const zd e2 = echan(ch, a2, bp, b2);
          if (e2.x == 0.0 && e2.y == 0.0) continue;
          for (int a = 0; a < m; ++a) {
            const zd e1 = zbar(echan(ch, a, bp, bo));
            if (e1.x == 0.0 && e1.y == 0.0) continue;
            acc = zplus(acc, ztimes(ztimes(e2, zget(b.M, (size_t)(a2 * c + v2) * N + (a * c + v))), e1));
          }
        }
      cx_t<T> o;
      o.x = (T)acc.x;
      o.y = (T)acc.y;
      Q[e] = o;
    }
  }
}

// ---------------------------------------------------------------- Ybar <- Ybar P + X Q
// A block owns kAdjRB row pairs (y with bit q = 0 and 1): it stages their Ybar and X rows in LDS,
// waits, and overwrites the Ybar rows; no other block touches them.
constexpr int kAdjRB = 16;

template <class T>
__global__ __launch_bounds__(256) void dual_project_kernel(cx_t<T>* __restrict__ Y, const cx_t<T>* __restrict__ X,
                                                           int ld, int c, int q, uint32_t half_rows,
                                                           const cx_t<T>* __restrict__ P,
                                                           const cx_t<T>* __restrict__ Q) {
  extern __shared__ __attribute__((aligned(16))) unsigned char adj_smem[];
  using Cx = cx_t<T>;
  const int w2 = 2 * c;
  Cx* ys = reinterpret_cast<Cx*>(adj_smem);   // [kAdjRB][w2]
  Cx* xs = ys + kAdjRB * w2;                  // [kAdjRB][w2]
  const uint32_t y0 = blockIdx.x * kAdjRB;
  for (int e = threadIdx.x; e < kAdjRB * w2; e += 256) {
    const int r = e / w2, col = e % w2;
    const uint32_t y = y0 + r;
    Cx a, g;
    a.x = a.y = g.x = g.y = (T)0;
    if (y < half_rows) {
      const size_t off = (size_t)with_bit(y, q, col / c) * ld + (col % c);
      g = Y[off];
      a = X[off];
    }
    ys[e] = g;
    xs[e] = a;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < kAdjRB * w2; e += 256) {
    const int r = e / w2, col = e % w2;
    const uint32_t y = y0 + r;
    if (y >= half_rows) continue;
    double ar = 0, ai = 0;
    for (int t = 0; t < w2; ++t) {
      const Cx g = ys[r * w2 + t], p = P[(size_t)t * w2 + col];
      const Cx a = xs[r * w2 + t], qq = Q[(size_t)t * w2 + col];
      ar += (double)g.x * p.x - (double)g.y * p.y + (double)a.x * qq.x - (double)a.y * qq.y;
      ai += (double)g.x * p.y + (double)g.y * p.x + (double)a.x * qq.y + (double)a.y * qq.x;
    }
    Cx o;
    o.x = (T)ar;
    o.y = (T)ai;
    Y[(size_t)with_bit(y, q, col / c) * ld + (col % c)] = o;
  }
}

template <class T>
hipError_t launch_compress_adjoint(cx_t<T>* Ybar, const cx_t<T>* X, int n, int ld, int c, int q,
                                   const Channel& ch, const double* rec, const AdjBufs& b,
                                   hipStream_t s) {
  if (c < 1 || 2 * c > 128 || ch.m < 1 || ch.m > 4 || ch.m * c > kRecMaxN || n < 1 || q < 0 || q >= n)
    return hipErrorInvalidValue;
  const uint32_t half_rows = 1u << (n - 1);
  const int w2 = 2 * c, nent = w2 * w2;
  const uint32_t rpc = adj_rows_per_chunk(half_rows);
  const int nchunks = (int)((half_rows + rpc - 1) / rpc);
  hipLaunchKernelGGL(cross_gram_kernel<T>, dim3(nchunks, (nent + 255) / 256), dim3(256), 0, s, X, Ybar, ld,
                     c, q, half_rows, rpc, b.part);
  hipLaunchKernelGGL(cross_gram_reduce_kernel, dim3((nent + 255) / 256), dim3(256), 0, s, b.part, nchunks,
                     nent, b.C);
  const int Nr = ch.m * c;
  const size_t sshm = adj_small_shm(Nr);
  static bool attr_set = false;
  if (!attr_set) {
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(adj_small_kernel<T>),
                                             hipFuncAttributeMaxDynamicSharedMemorySize,
                                             (int)adj_small_shm(kRecMaxN));
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL(adj_small_kernel<T>, dim3(1), dim3(kAdjSmallThreads), sshm, s, rec, ch, c, b);
  const size_t shm = (size_t)2 * kAdjRB * w2 * sizeof(cx_t<T>);
  hipLaunchKernelGGL(dual_project_kernel<T>, dim3((half_rows + kAdjRB - 1) / kAdjRB), dim3(256), shm, s,
                     Ybar, X, ld, c, q, half_rows, static_cast<const cx_t<T>*>(b.P),
                     static_cast<const cx_t<T>*>(b.Q));
  return hipGetLastError();
}

template hipError_t launch_pauli_apply<float>(float2*, const float2*, int, int, int, const uint64_t*,
                                              const uint64_t*, const double*, int, hipStream_t);
template hipError_t launch_pauli_apply<double>(double2*, const double2*, int, int, int, const uint64_t*,
                                               const uint64_t*, const double*, int, hipStream_t);
template hipError_t launch_gram_exact<float>(const float2*, int, int, int, int, double*, double*, hipStream_t);
template hipError_t launch_gram_exact<double>(const double2*, int, int, int, int, double*, double*, hipStream_t);
template hipError_t launch_compress_adjoint<float>(float2*, const float2*, int, int, int, int,
                                                   const Channel&, const double*, const AdjBufs&,
                                                   hipStream_t);
template hipError_t launch_compress_adjoint<double>(double2*, const double2*, int, int, int, int,
                                                    const Channel&, const double*, const AdjBufs&,
                                                    hipStream_t);

}  // namespace lrdm
