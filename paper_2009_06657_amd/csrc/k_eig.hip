// FP64 eigensolver of the small Gram matrix G (order N <= 128) and the truncation rule
// (Sec. II.B; Theorem 1, App. B).  Three single-work-group kernels on the serial path between
// the Gram and projection GEMMs:
//
//  1. eig_tridiag: assemble G from S = X^H X and the Kraus set, G_{(a,v),(b,w)} =
//     sum_{uv'} (E_a^H E_b)_{uv'} S_{(u,v),(v',w)}, in packed lower storage in LDS (132 KB at
//     N = 128), then reduce it to a real symmetric tridiagonal T = Q^H G Q with N - 2 Householder
//     reflectors H_j = I - tau_j v_j v_j^H (v_j(j+1) = 1), each a Hermitian matrix-vector product
//     and a rank-2 update over the trailing block.
//  2. eig_solve: the wanted (largest) eigenvalues of T by multisection on Sturm counts (one
//     group of 8 or 16 lanes per eigenvalue), then eigenvectors by inverse iteration on a
//     pivoted LU of T - lambda I (one lane per eigenvector).  Eigenvalues closer than 1e-9 ||T||
//     form clusters whose vectors are re-orthonormalised (modified Gram-Schmidt, descending
//     order) after every iteration, so degenerate eigenvalues yield an orthonormal basis of the
//     cluster.
//  3. eig_finish: the rank rule (cap r, threshold eps, tie policy), discarded mass,
//     renormalisation scale, back-transform V = Q Y, and the projection matrix W in the bulk
//     precision: W_{(b,v),(b',j)} = c sum_a (E_a)_{b'b} V[(a,v),j] (split view) or W = c V_k.
#include <math.h>

#include "lrdm_internal.h"

namespace lrdm {

struct z64 {
  double x, y;
};
__device__ __forceinline__ z64 zmk(double a, double b) { return z64{a, b}; }
__device__ __forceinline__ z64 zadd(z64 a, z64 b) { return z64{a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ z64 zsub(z64 a, z64 b) { return z64{a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ z64 zmul(z64 a, z64 b) { return z64{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ __forceinline__ z64 zconj(z64 a) { return z64{a.x, -a.y}; }
__device__ __forceinline__ z64 zcmul(z64 a, z64 b) {  // conj(a) * b
  return z64{a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ z64 zscale(z64 a, double s) { return z64{a.x * s, a.y * s}; }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double group_sum(double v, int width) {
  for (int o = width >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ int poff(int j, int N) { return j * N - (j * (j - 1)) / 2; }

// ------------------------------------------------------------------------------------------
// 1. assemble + Householder tridiagonalisation
// ------------------------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void eig_tridiag_kernel(const double* __restrict__ S, int Fc,
                                                           Channel ch, int nsplit, int c, int N,
                                                           EigBufs B) {
  extern __shared__ double smem[];
  z64* P = reinterpret_cast<z64*>(smem);                 // N(N+1)/2
  z64* vb = P + (N * (N + 1)) / 2;                        // N
  z64* pb = vb + N;                                       // N
  z64* Mab = pb + N;                                      // m*m*4 entries of E_a^H E_b
  double* scal = reinterpret_cast<double*>(Mab + 64);    // tau.re, tau.im, flag, trace
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m = (nsplit == 2) ? ch.m : 1;

  if (nsplit == 2 && tid < m * m * 4) {
    const int a = tid / (m * 4), b = (tid / 4) % m, u = (tid >> 1) & 1, v = tid & 1;
    z64 acc = zmk(0, 0);
    for (int r = 0; r < 2; ++r) {
      const z64 ea = zmk(ch.e[a][r][u][0], ch.e[a][r][u][1]);
      const z64 eb = zmk(ch.e[b][r][v][0], ch.e[b][r][v][1]);
      acc = zadd(acc, zcmul(ea, eb));
    }
    Mab[tid] = acc;   // (E_a^H E_b)_{uv} at index ((a*m + b)*2 + u)*2 + v
  }
  __syncthreads();
  // packed lower G
  const int npk = (N * (N + 1)) / 2;
  for (int e = tid; e < N * N; e += 1024) {
    const int i = e / N, j = e % N;
    if (i < j) continue;
    z64 g;
    if (nsplit == 2) {
      const int a = i / c, vv = i % c, b = j / c, w = j % c;
      g = zmk(0, 0);
      for (int u = 0; u < 2; ++u)
        for (int v = 0; v < 2; ++v) {
          const z64 mm = Mab[((a * m + b) * 2 + u) * 2 + v];
          const size_t si = 2 * ((size_t)(u * c + vv) * Fc + (v * c + w));
          g = zadd(g, zmul(mm, zmk(S[si], S[si + 1])));
        }
    } else {
      const size_t si = 2 * ((size_t)i * Fc + j);
      g = zmk(S[si], S[si + 1]);
    }
    P[poff(j, N) + (i - j)] = g;
  }
  __syncthreads();
  if (wave == 0) {
    double t = 0;
    for (int i = lane; i < N; i += 64) t += P[poff(i, N)].x;
    t = wave_sum(t);
    if (lane == 0) scal[3] = t;
  }
  (void)npk;

  for (int j = 0; j + 1 < N; ++j) {
    const int mlen = N - 1 - j;   // trailing order
    // ---- reflector for column j (wave 0)
    if (wave == 0) {
      const z64 alpha = P[poff(j, N) + 1];
      double xn2 = 0;
      for (int i = j + 2 + lane; i < N; i += 64) {
        const z64 x = P[poff(j, N) + (i - j)];
        xn2 += x.x * x.x + x.y * x.y;
      }
      xn2 = wave_sum(xn2);
      double taur = 0, taui = 0, beta = alpha.x;
      z64 sc = zmk(0, 0);
      const bool trivial = (xn2 == 0.0 && alpha.y == 0.0);
      if (!trivial) {
        const double nrm = sqrt(alpha.x * alpha.x + alpha.y * alpha.y + xn2);
        beta = (alpha.x >= 0) ? -nrm : nrm;
        taur = (beta - alpha.x) / beta;
        taui = -alpha.y / beta;
        // sc = 1 / (alpha - beta)
        const double dr = alpha.x - beta, di = alpha.y;
        const double den = dr * dr + di * di;
        sc = zmk(dr / den, -di / den);
      }
      for (int i = j + 2 + lane; i < N; i += 64) {
        const z64 x = P[poff(j, N) + (i - j)];
        const z64 v = trivial ? zmk(0, 0) : zmul(sc, x);
        P[poff(j, N) + (i - j)] = v;
        vb[i - j - 1] = v;
      }
      if (lane == 0) {
        vb[0] = zmk(1, 0);
        P[poff(j, N) + 1] = zmk(beta, 0);
        B.e[j] = beta;
        B.d[j] = P[poff(j, N)].x;
        B.tau[2 * j] = taur;
        B.tau[2 * j + 1] = taui;
        scal[0] = taur;
        scal[1] = taui;
      }
    }
    __syncthreads();
    const z64 tau = zmk(scal[0], scal[1]);
    if (tau.x == 0.0 && tau.y == 0.0) {
      __syncthreads();   // everyone has read scal before wave 0 rewrites it
      continue;
    }
    const int base = j + 1;
    // ---- p = tau * A_sub v  (8 lanes per row)
    {
      const int i = tid >> 3, g = tid & 7;
      z64 s = zmk(0, 0);
      if (i < mlen) {
        for (int k = g; k < mlen; k += 8) {
          z64 a;
          if (i >= k)
            a = P[poff(base + k, N) + (i - k)];
          else
            a = zconj(P[poff(base + i, N) + (k - i)]);
          s = zadd(s, zmul(a, vb[k]));
        }
      }
      s.x = group_sum(s.x, 8);
      s.y = group_sum(s.y, 8);
      if (i < mlen && g == 0) pb[i] = zmul(tau, s);
    }
    __syncthreads();
    // ---- alpha2 = -1/2 tau (p^H v) (every wave), w = p + alpha2 v, A -= v w^H + w v^H
    z64 dot = zmk(0, 0);
    for (int i = lane; i < mlen; i += 64) dot = zadd(dot, zcmul(pb[i], vb[i]));
    dot.x = wave_sum(dot.x);
    dot.y = wave_sum(dot.y);
    const z64 alpha2 = zscale(zmul(tau, dot), -0.5);
    for (int k = wave; k < mlen; k += 16) {
      const z64 vk = vb[k];
      const z64 wk = zadd(pb[k], zmul(alpha2, vk));
      for (int i = k + lane; i < mlen; i += 64) {
        const z64 vi = vb[i];
        const z64 wi = zadd(pb[i], zmul(alpha2, vi));
        z64& a = P[poff(base + k, N) + (i - k)];
        // a -= v_i conj(w_k) + w_i conj(v_k)
        a = zsub(a, zadd(zmul(vi, zconj(wk)), zmul(wi, zconj(vk))));
      }
    }
    __syncthreads();
  }
  __syncthreads();
  if (tid == 0) {
    B.d[N - 1] = P[poff(N - 1, N)].x;
    if (N == 1) B.d[0] = P[0].x;
    B.trace[0] = scal[3];
  }
  double* Pg = B.P;
  for (int e = tid; e < (N * (N + 1)) / 2; e += 1024) {
    Pg[2 * e] = P[e].x;
    Pg[2 * e + 1] = P[e].y;
  }
}

hipError_t launch_eig_tridiag(const double* S, int Fc, const Channel& ch, int nsplit, int c,
                              int N, const EigBufs& b, hipStream_t s) {
  const size_t shm = ((size_t)(N * (N + 1)) / 2 + 2 * N + 64) * sizeof(z64) + 8 * sizeof(double);
  if (shm > 65536) {
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(eig_tridiag_kernel),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(eig_tridiag_kernel, dim3(1), dim3(1024), shm, s, S, Fc, ch, nsplit, c, N, b);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// 2. eigenvalues (multisection) + eigenvectors (inverse iteration) of T
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ int sturm_count(const double* d, const double* e2, int N, double x,
                                           double pivmin) {
  double q = d[0] - x;
  int cnt = 0;
  if (q <= pivmin) {
    ++cnt;
    q = fmin(q, -pivmin);
  }
  for (int i = 1; i < N; ++i) {
    q = (d[i] - x) - e2[i - 1] / q;
    if (q <= pivmin) {
      ++cnt;
      q = fmin(q, -pivmin);
    }
  }
  return cnt;
}

__device__ __forceinline__ double hash_unit(uint32_t a, uint32_t b) {
  uint32_t h = a * 0x9E3779B1u ^ (b + 0x7F4A7C15u) * 0x85EBCA77u;
  h ^= h >> 15;
  h *= 0x2C1B3C6Du;
  h ^= h >> 12;
  h *= 0x297A2D39u;
  h ^= h >> 15;
  return ((double)(h >> 8) + 0.5) * (1.0 / 16777216.0) - 0.5;  // (-0.5, 0.5)
}

__global__ __launch_bounds__(1024) void eig_solve_kernel(int N, int kmax, EigBufs B) {
  __shared__ double d[kMaxEig], e2[kMaxEig], es[kMaxEig], lam[kMaxEig];
  __shared__ int cl_start[kMaxEig], cl_len[kMaxEig];
  __shared__ double red[2];
  extern __shared__ double X[];                 // N x kmax, X[i * kmax + t]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  // scale T to unit norm (Gershgorin)
  if (wave == 0) {
    double mx = 0;
    for (int i = lane; i < N; i += 64) {
      const double el = (i > 0) ? fabs(B.e[i - 1]) : 0.0;
      const double er = (i + 1 < N) ? fabs(B.e[i]) : 0.0;
      mx = fmax(mx, fabs(B.d[i]) + el + er);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
    if (lane == 0) red[0] = mx;
  }
  __syncthreads();
  const double tnorm = red[0];
  const bool zero = !(tnorm > 0.0);
  const double inv = zero ? 1.0 : 1.0 / tnorm;
  for (int i = tid; i < N; i += 1024) {
    d[i] = B.d[i] * inv;
    es[i] = (i + 1 < N) ? B.e[i] * inv : 0.0;
    e2[i] = es[i] * es[i];
  }
  __syncthreads();
  const double eps = 2.220446049250313e-16;
  const double pivmin = 1e-290;

  // ---- multisection: group of G lanes per wanted eigenvalue (descending index t)
  const int G = (kmax <= 64) ? 16 : 8;
  {
    const int t = tid / G, g = tid % G;
    const bool active = (t < kmax) && !zero;
    const int a = N - 1 - t;                      // ascending index
    double lo = -1.0 - 4 * eps, hi = 1.0 + 4 * eps;   // |lambda| <= ||T|| = 1
    for (int it = 0; it < 24; ++it) {
      const double w = hi - lo;
      const bool done = !(w > 2 * eps * fmax(fabs(lo), fabs(hi)) + 4 * eps * eps);
      const double x = lo + w * (double)(g + 1) / (double)(G + 1);
      const int cnt = active ? sturm_count(d, e2, N, x, pivmin) : 0;
      const unsigned long long ball = __ballot(active && cnt > a);
      const int gb = lane & ~(G - 1);
      const unsigned long long grp = (ball >> gb) & ((1ull << G) - 1ull);
      const int first = grp ? (__ffsll((long long)grp) - 1) : G;   // G: no sample above
      const double xh = __shfl(x, gb + (first < G ? first : 0), 64);
      const double xl = __shfl(x, gb + (first == 0 ? 0 : first - 1), 64);
      if (active && !done) {
        if (first < G) hi = xh;
        if (first > 0) lo = xl;
      }
    }
    if (active && g == 0) lam[t] = 0.5 * (lo + hi);
    if (zero && g == 0 && t < kmax) lam[t] = 0.0;
  }
  __syncthreads();

  // ---- clusters (descending order)
  if (tid == 0) {
    const double ctol = 1e-9;
    int s = 0;
    for (int t = 0; t < kmax; ++t) {
      if (t > 0 && !(lam[t - 1] - lam[t] <= ctol)) s = t;
      cl_start[t] = s;
    }
    for (int t = kmax - 1; t >= 0; --t) cl_len[t] = 0;
    for (int t = 0; t < kmax; ++t) cl_len[cl_start[t]] += 1;
  }
  __syncthreads();

  // ---- inverse iteration: lane t owns eigenvector t
  double* la = B.lu;                 // U diagonal (inverse stored)
  double* lb = la + N * kmax;        // U first superdiagonal
  double* lc = lb + N * kmax;        // multipliers
  double* ldd = lc + N * kmax;       // U second superdiagonal
  double* lp = ldd + N * kmax;       // pivot flags
  const int t = tid;
  const bool owner = t < kmax;
  if (owner) {
    const double sigma = lam[t];
    // factor T - sigma I = P L U (partial pivoting)
    double ak = d[0] - sigma;
    double bk = (N > 1) ? es[0] : 0.0;
    for (int k = 0; k + 1 < N; ++k) {
      const double ck = es[k];
      const double a1 = d[k + 1] - sigma;
      const double b1 = (k + 2 < N) ? es[k + 1] : 0.0;
      double piv, mult, u0, u1, u2, an, bn;
      if (fabs(ak) >= fabs(ck)) {
        piv = 0;
        mult = (ak != 0.0) ? ck / ak : 0.0;
        u0 = ak; u1 = bk; u2 = 0.0;
        an = a1 - mult * bk;
        bn = b1;
      } else {
        piv = 1;
        mult = ak / ck;
        u0 = ck; u1 = a1; u2 = b1;
        an = bk - mult * a1;
        bn = -mult * b1;
      }
      if (fabs(u0) < eps) u0 = (u0 >= 0) ? eps : -eps;
      la[k * kmax + t] = 1.0 / u0;
      lb[k * kmax + t] = u1;
      ldd[k * kmax + t] = u2;
      lc[k * kmax + t] = mult;
      lp[k * kmax + t] = piv;
      ak = an;
      bk = bn;
    }
    if (fabs(ak) < eps) ak = (ak >= 0) ? eps : -eps;
    la[(N - 1) * kmax + t] = 1.0 / ak;
    for (int i = 0; i < N; ++i) X[i * kmax + t] = 1.0 + hash_unit((uint32_t)t, (uint32_t)i);
  }
  __syncthreads();

  for (int iter = 0; iter < 3; ++iter) {
    if (owner) {
      // forward: y <- L^{-1} P y
      double yk = X[t];
      for (int k = 0; k + 1 < N; ++k) {
        double yk1 = X[(k + 1) * kmax + t];
        if (lp[k * kmax + t] != 0.0) {
          const double tmp = yk;
          yk = yk1;
          yk1 = tmp;
        }
        X[k * kmax + t] = yk;
        yk = yk1 - lc[k * kmax + t] * yk;
      }
      X[(N - 1) * kmax + t] = yk;
      // backward: U x = y
      double x1 = 0.0, x2 = 0.0, mx = 0.0;
      for (int k = N - 1; k >= 0; --k) {
        double v = X[k * kmax + t];
        if (k + 1 < N) v -= lb[k * kmax + t] * x1;
        if (k + 2 < N) v -= ldd[k * kmax + t] * x2;
        v *= la[k * kmax + t];
        X[k * kmax + t] = v;
        x2 = x1;
        x1 = v;
        mx = fmax(mx, fabs(v));
      }
      const double sc = (mx > 0) ? 1.0 / mx : 1.0;
      double nn = 0;
      for (int i = 0; i < N; ++i) {
        const double v = X[i * kmax + t] * sc;
        nn += v * v;
        X[i * kmax + t] = v;
      }
      const double s2 = 1.0 / sqrt(nn);
      for (int i = 0; i < N; ++i) X[i * kmax + t] *= s2;
    }
    __syncthreads();
    // cluster re-orthonormalisation, one wave per cluster
    for (int cs = 0; cs < kmax; ++cs) {
      if (cl_start[cs] != cs || cl_len[cs] < 2) continue;
      if ((cs % 16) != wave) continue;
      const int len = cl_len[cs];
      for (int jj = cs; jj < cs + len; ++jj) {
        for (int ii = cs; ii < jj; ++ii) {
          double dt = 0;
          for (int i = lane; i < N; i += 64) dt += X[i * kmax + ii] * X[i * kmax + jj];
          dt = wave_sum(dt);
          for (int i = lane; i < N; i += 64) X[i * kmax + jj] -= dt * X[i * kmax + ii];
        }
        double nn = 0;
        for (int i = lane; i < N; i += 64) nn += X[i * kmax + jj] * X[i * kmax + jj];
        nn = wave_sum(nn);
        const double s2 = (nn > 0) ? 1.0 / sqrt(nn) : 0.0;
        for (int i = lane; i < N; i += 64) X[i * kmax + jj] *= s2;
      }
    }
    __syncthreads();
  }
  // outputs: lam (unscaled, descending) and Y column-major by eigenvector
  for (int e = tid; e < kmax; e += 1024) B.lam[e] = lam[e] * tnorm;
  for (int e = tid; e < N * kmax; e += 1024) {
    const int tt = e / N, i = e % N;
    B.Y[e] = zero ? ((i == tt) ? 1.0 : 0.0) : X[i * kmax + tt];
  }
}

hipError_t launch_eig_solve(int N, int kmax, const EigBufs& b, hipStream_t s) {
  const size_t shm = (size_t)N * kmax * sizeof(double);
  if (shm > 65536) {
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(eig_solve_kernel),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(eig_solve_kernel, dim3(1), dim3(1024), shm, s, N, kmax, b);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// 3. rank rule, back-transform, projection matrix W
// ------------------------------------------------------------------------------------------
template <class T>
__global__ __launch_bounds__(1024) void eig_finish_kernel(int N, int kmax, int r_target, double eps,
                                                          int tie, int renorm, Channel ch,
                                                          int nsplit, int c, int c_out, EigBufs B,
                                                          cx_t<T>* __restrict__ W) {
  extern __shared__ double smem[];
  z64* P = reinterpret_cast<z64*>(smem);          // packed reflectors, later V (N x k)
  __shared__ double tau_s[2 * kMaxEig];
  __shared__ int k_s;
  __shared__ double scale_s;
  const int tid = threadIdx.x;
  const int npk = (N * (N + 1)) / 2;

  if (tid == 0) {
    const double trace = B.trace[0];
    int k = min(r_target, N);
    bool bad = !isfinite(trace);
    for (int i = 0; i < kmax; ++i) bad = bad || !isfinite(B.lam[i]);
    if (eps > 0.0) {
      double kept = 0;
      int keps = N;
      for (int i = 0; i < kmax; ++i) {
        kept += fmax(B.lam[i], 0.0);
        if (kept >= (1.0 - eps) * trace) {
          keps = i + 1;
          break;
        }
      }
      k = min(k, keps);
    }
    if (tie == 1) {
      while (k > 1 && k < N && (B.lam[k - 1] - B.lam[k]) <= 1e-6 * trace) --k;
    }
    if (k < 1) k = 1;
    double kept = 0;
    for (int i = 0; i < k; ++i) kept += fmax(B.lam[i], 0.0);
    if (!(kept > 0.0)) bad = true;
    const double sc = (renorm && kept > 0.0) ? 1.0 / sqrt(kept) : 1.0;
    DevInfo* inf = B.info;
    const double disc = fmax(trace - kept, 0.0);
    inf->k = k;
    inf->n_eig = N;
    inf->discarded = disc;
    inf->discarded_total += disc;
    inf->trace = trace;
    inf->gap = (k < N) ? (B.lam[k - 1] - B.lam[k]) : INFINITY;
    inf->lambda_max = B.lam[0];
    inf->scale = sc;
    if (bad) inf->status = (int)LRDM_E_EIG;
    k_s = k;
    scale_s = sc;
  }
  for (int e = tid; e < npk; e += 1024) P[e] = zmk(B.P[2 * e], B.P[2 * e + 1]);
  for (int e = tid; e < 2 * (N - 1); e += 1024) tau_s[e] = B.tau[e];
  __syncthreads();
  const int k = k_s;
  const double sc = scale_s;

  // back-transform: 16 lanes per kept column, lane g holds rows g, g+16, ...
  const int col = tid >> 4, g = tid & 15;
  z64 z[kMaxEig / 16];
  if (col < k) {
#pragma unroll
    for (int s = 0; s < kMaxEig / 16; ++s) {
      const int i = g + 16 * s;
      z[s] = zmk(i < N ? B.Y[(size_t)col * N + i] : 0.0, 0.0);
    }
    for (int j = N - 2; j >= 0; --j) {
      const z64 tj = zmk(tau_s[2 * j], tau_s[2 * j + 1]);
      if (tj.x == 0.0 && tj.y == 0.0) continue;
      z64 s = zmk(0, 0);
#pragma unroll
      for (int q = 0; q < kMaxEig / 16; ++q) {
        const int i = g + 16 * q;
        if (i >= j + 1 && i < N) {
          const z64 v = (i == j + 1) ? zmk(1, 0) : P[poff(j, N) + (i - j)];
          s = zadd(s, zcmul(v, z[q]));
        }
      }
      s.x = group_sum(s.x, 16);
      s.y = group_sum(s.y, 16);
      const z64 ts = zmul(tj, s);
#pragma unroll
      for (int q = 0; q < kMaxEig / 16; ++q) {
        const int i = g + 16 * q;
        if (i >= j + 1 && i < N) {
          const z64 v = (i == j + 1) ? zmk(1, 0) : P[poff(j, N) + (i - j)];
          z[q] = zsub(z[q], zmul(v, ts));
        }
      }
    }
  }
  __syncthreads();
  // V in LDS as V[i * 64 + col]
  z64* V = P;
  if (col < k) {
#pragma unroll
    for (int s = 0; s < kMaxEig / 16; ++s) {
      const int i = g + 16 * s;
      if (i < N) V[i * 64 + col] = z[s];
    }
  }
  __syncthreads();
  // W in the bulk precision
  using C = cx_t<T>;
  if (nsplit == 2) {
    const int rows = 2 * c, cols = 2 * c_out;
    for (int e = tid; e < rows * cols; e += 1024) {
      const int rw = e / cols, cl = e % cols;
      const int b = rw / c, v = rw % c, bp = cl / c_out, j = cl % c_out;
      z64 acc = zmk(0, 0);
      if (j < k) {
        for (int a = 0; a < ch.m; ++a)
          acc = zadd(acc, zmul(zmk(ch.e[a][bp][b][0], ch.e[a][bp][b][1]), V[(a * c + v) * 64 + j]));
      }
      C o;
      o.x = (T)(acc.x * sc);
      o.y = (T)(acc.y * sc);
      W[e] = o;
    }
  } else {
    const int cols = c_out;
    for (int e = tid; e < N * cols; e += 1024) {
      const int i = e / cols, j = e % cols;
      const z64 acc = (j < k) ? V[i * 64 + j] : zmk(0, 0);
      C o;
      o.x = (T)(acc.x * sc);
      o.y = (T)(acc.y * sc);
      W[e] = o;
    }
  }
}

template <class T>
hipError_t launch_eig_finish(int N, int kmax, int r_target, double eps, int tie, int renorm,
                             const Channel& ch, int nsplit, int c, int c_out, const EigBufs& b,
                             cx_t<T>* W, hipStream_t s) {
  const size_t npk = (size_t)(N * (N + 1)) / 2;
  const size_t nv = (size_t)N * 64;
  const size_t shm = (npk > nv ? npk : nv) * sizeof(z64);
  if (shm > 65536) {
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(eig_finish_kernel<T>),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(eig_finish_kernel<T>, dim3(1), dim3(1024), shm, s, N, kmax, r_target, eps, tie,
                     renorm, ch, nsplit, c, c_out, b, W);
  return hipGetLastError();
}

template hipError_t launch_eig_finish<float>(int, int, int, double, int, int, const Channel&, int,
                                             int, int, const EigBufs&, float2*, hipStream_t);
template hipError_t launch_eig_finish<double>(int, int, int, double, int, int, const Channel&, int,
                                              int, int, const EigBufs&, double2*, hipStream_t);

}  // namespace lrdm
