// FP64 eigensolver of the small Gram matrix G (order N <= 128) and the truncation rule
// (Sec. II.B; Theorem 1, App. B), as one single-work-group kernel on the serial path between
// the Gram and projection GEMMs.
//
//  1. Assemble G from S = X^H X and the Kraus set, G_{(a,v),(b,w)} = sum_{uv'} (E_a^H E_b)_{uv'}
//     S_{(u,v),(v',w)} (split view) or G = S (plain view).  G lives in registers: a grid of
//     (32 BC / BR) x 32 threads holds BR x BC blocks (N <= 32 BC), so a row of blocks is one
//     half-wave.
//  2. Householder reduction to a real symmetric tridiagonal T = Q^H G Q with reflectors
//     H_j = I - tau_j v_j v_j^H, v_j(j+1) = 1.  Every half-wave forms the reflector from the
//     broadcast column, the matrix-vector product reduces across a half-wave with shuffles, and
//     the rank-2 update is register arithmetic: two barriers per step.
//  3. The wanted (largest) eigenvalues of T by multisection on Sturm counts (a group of 8 or 16
//     lanes per eigenvalue).
//  4. Eigenvectors of T by inverse iteration on the LDL^T factorisation of T - lambda I (one
//     lane per eigenvector, factors and vectors in LDS).  Eigenvalues closer than 1e-9 ||T|| form
//     clusters whose vectors are re-orthonormalised (modified Gram-Schmidt, descending order)
//     after every iteration, so (near-)degenerate eigenvalues yield an orthonormal basis.
//  5. The rank rule (cap r, threshold eps, tie policy), discarded mass and renormalisation
//     scale; back-transform V = Q Y; the projection matrix in the bulk precision:
//     W_{(b,v),(b',j)} = c sum_a (E_a)_{b'b} V[(a,v), j] (split view) or W = c V_k (plain).
#include <math.h>

#include <utility>

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

// Lane-group sums.  Inside a row of 16 lanes the exchanges are DPP moves (quad_perm xor 1,
// quad_perm xor 2, row_half_mirror, row_mirror: after the first two steps every lane of a quad
// holds the quad sum, so the mirrors add the other quad / half-row); the 16- and 32-lane
// exchanges use ds_bpermute.  Every lane of the group ends with the identical value.
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
template <int W>
__device__ __forceinline__ double gsum(double v) {
  if constexpr (W >= 2) v += dpp_mov<0xB1>(v);    // quad_perm [1,0,3,2]
  if constexpr (W >= 4) v += dpp_mov<0x4E>(v);    // quad_perm [2,3,0,1]
  if constexpr (W >= 8) v += dpp_mov<0x141>(v);   // row_half_mirror
  if constexpr (W >= 16) v += dpp_mov<0x140>(v);  // row_mirror
  if constexpr (W >= 32) v += __shfl_xor(v, 16, 64);
  if constexpr (W >= 64) v += __shfl_xor(v, 32, 64);
  return v;
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

// offset of reflector j's entries i >= j + 2 in packed storage
__device__ __forceinline__ int refl_off(int j, int N) { return j * (N - 2) - (j * (j - 1)) / 2; }

// f / q through the hardware reciprocal refined by one Newton step (a few ulp; the Sturm
// count only needs the sign pattern of the recurrence)
__device__ __forceinline__ double fdiv(double f, double q) {
  double r = __builtin_amdgcn_rcp(q);
  r = fma(r, fma(-q, r, 1.0), r);
  return f * r;
}

// number of eigenvalues of T (scaled, diagonal d, squared off-diagonal e2) below x
__device__ __forceinline__ int sturm_count(const double* d, const double* e2, int N, double x,
                                           double pivmin) {
  double q = d[0] - x;
  int cnt = 0;
  if (q <= pivmin) {
    ++cnt;
    q = fmin(q, -pivmin);
  }
  int i = 1;
  for (; i + 3 < N; i += 4) {
    const double d0 = d[i], d1 = d[i + 1], d2 = d[i + 2], d3 = d[i + 3];
    const double f0 = e2[i - 1], f1 = e2[i], f2 = e2[i + 1], f3 = e2[i + 2];
    q = (d0 - x) - fdiv(f0, q);
    if (q <= pivmin) { ++cnt; q = fmin(q, -pivmin); }
    q = (d1 - x) - fdiv(f1, q);
    if (q <= pivmin) { ++cnt; q = fmin(q, -pivmin); }
    q = (d2 - x) - fdiv(f2, q);
    if (q <= pivmin) { ++cnt; q = fmin(q, -pivmin); }
    q = (d3 - x) - fdiv(f3, q);
    if (q <= pivmin) { ++cnt; q = fmin(q, -pivmin); }
  }
  for (; i < N; ++i) {
    q = (d[i] - x) - fdiv(e2[i - 1], q);
    if (q <= pivmin) { ++cnt; q = fmin(q, -pivmin); }
  }
  return cnt;
}

template <class F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

template <class T, int BR, int BC>
__device__ __forceinline__ void eig_body(const double* __restrict__ S, int Fc, const Channel& ch, int nsplit,
                                         int c, int N, int kmax, int r_target, double eps, int tie,
                                         int renorm, int c_out, const EigBufs& B,
                                         cx_t<T>* __restrict__ W) {
  constexpr int NP = 32 * BC;            // padded order; the thread grid is (NP / BR) x 32
  constexpr int NTH = 32 * (NP / BR);    // threads
  extern __shared__ __attribute__((aligned(16))) double dyn[];   // phase-dependent scratch
  __shared__ z64 Mab[64];
  __shared__ z64 col_buf[NP], vbuf[NP], pbuf[NP];
  __shared__ double d_s[NP], e_s[NP], e2_s[NP], lam_s[NP + 1], tau_s[2 * NP], trp[32];
  __shared__ int cl_start[NP], cl_len[NP];
  __shared__ double sc_s[4];
  __shared__ int k_s;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int R = tid >> 5, Cc = tid & 31;   // block row / block column of this thread
  const int m = (nsplit == 2) ? ch.m : 1;

  // ---------------------------------------------------------------- 1. assemble G
  if (nsplit == 2 && tid < m * m * 4) {
    const int a = tid / (m * 4), b = (tid / 4) % m, u = (tid >> 1) & 1, v = tid & 1;
    z64 acc = zmk(0, 0);
    for (int r = 0; r < 2; ++r)
      acc = zadd(acc, zcmul(zmk(ch.e[a][r][u][0], ch.e[a][r][u][1]), zmk(ch.e[b][r][v][0], ch.e[b][r][v][1])));
    Mab[tid] = acc;   // (E_a^H E_b)_{uv} at ((a m + b) 2 + u) 2 + v
  }
  __syncthreads();
  z64 A[BR][BC];
#pragma unroll
  for (int a = 0; a < BR; ++a)
#pragma unroll
    for (int b = 0; b < BC; ++b) {
      const int i = BR * R + a, j = BC * Cc + b;
      z64 g = zmk(0, 0);
      if (i < N && j < N) {
        if (nsplit == 2) {
          const int ai = i / c, vv = i % c, bj = j / c, w = j % c;
          for (int u = 0; u < 2; ++u)
            for (int v = 0; v < 2; ++v) {
              const z64 mm = Mab[((ai * m + bj) * 2 + u) * 2 + v];
              const size_t si = 2 * ((size_t)(u * c + vv) * Fc + (v * c + w));
              g = zadd(g, zmul(mm, zmk(S[si], S[si + 1])));
            }
        } else {
          const size_t si = 2 * ((size_t)i * Fc + j);
          g = zmk(S[si], S[si + 1]);
        }
      }
      A[a][b] = g;
    }
  {
    double t = 0;
#pragma unroll
    for (int a = 0; a < BR; ++a) {
      const int i = BR * R + a;
      if (i / BC == Cc) t += A[a][a % BC].x;   // BR is a multiple of BC
    }
    t = gsum<32>(t);
    if (Cc == 0) trp[R] = t;
  }
  if (Cc == 0) {
#pragma unroll
    for (int a = 0; a < BR; ++a) col_buf[BR * R + a] = A[a][0];
  }
  __syncthreads();
  if (tid == 0) {
    double t = 0;
    for (int i = 0; i < NTH / 32; ++i) t += trp[i];
    sc_s[0] = t;   // trace
  }

  // ---------------------------------------------------------------- 2. tridiagonalisation
  // Reflector entries i >= j + 2 are kept in LDS while reducing (a global store inside the
  // loop would make every barrier wait for its completion); they are spilled to the workspace
  // in one pass afterwards, because the eigenvector phase reuses this LDS.
  z64* Rf = reinterpret_cast<z64*>(dyn);
  double* refl = B.P;
  auto step = [&](const int j, auto bbc) {
    constexpr int bb = decltype(bbc)::value;   // j % BC
    // reflector from column j (every half-wave redundantly; lane Cc owns entries BC Cc + b)
    const z64 alpha = col_buf[j + 1];
    z64 cv[BC];
    double xn2 = 0;
#pragma unroll
    for (int b = 0; b < BC; ++b) {
      const int i = BC * Cc + b;
      cv[b] = col_buf[i];
      if (i > j + 1 && i < N) xn2 += cv[b].x * cv[b].x + cv[b].y * cv[b].y;
    }
    xn2 = gsum<32>(xn2);
    double beta = alpha.x;
    z64 tau = zmk(0, 0), sc = zmk(0, 0);
    const bool trivial = (xn2 == 0.0 && alpha.y == 0.0);
    if (!trivial) {
      const double nrm = sqrt(alpha.x * alpha.x + alpha.y * alpha.y + xn2);
      beta = (alpha.x >= 0) ? -nrm : nrm;
      const double ib = 1.0 / beta;
      tau = zmk((beta - alpha.x) * ib, -alpha.y * ib);
      const double dr = alpha.x - beta, di = alpha.y;
      const double iden = 1.0 / (dr * dr + di * di);
      sc = zmk(dr * iden, -di * iden);
    }
    z64 (&vloc)[BC] = cv;   // v overwrites the column entries it is built from
#pragma unroll
    for (int b = 0; b < BC; ++b) {
      const int i = BC * Cc + b;
      vloc[b] = (i == j + 1) ? zmk(1, 0) : ((i > j + 1 && i < N) ? zmul(sc, cv[b]) : zmk(0, 0));
    }
    if (tid < 32) {
#pragma unroll
      for (int b = 0; b < BC; ++b) {
        const int i = BC * Cc + b;
        vbuf[i] = vloc[b];
        if (i >= j + 2 && i < N) Rf[refl_off(j, N) + (i - j - 2)] = vloc[b];
      }
      if (tid == 0) {
        d_s[j] = col_buf[j].x;
        e_s[j] = beta;
        tau_s[2 * j] = tau.x;
        tau_s[2 * j + 1] = tau.y;
      }
    }
    // s = A v for this thread's rows, reduced over the half-wave (pbuf holds s; p = tau s);
    // row blocks that lie entirely in the eliminated part (rows <= j) only publish zeros
    const bool live = BR * R + BR - 1 > j;   // uniform over the half-wave
    if (live) {
      if constexpr (BR == 8) {
        // 16 values (8 rows x re/im) over 32 lanes by a transposing reduction: each stage
        // halves the values a lane keeps and swaps the other half with its partner (lane ^ 16,
        // then row_mirror, row_half_mirror and quad xor 2 pair lanes that differ in bits 3, 2,
        // 1), and a last exchange adds the pair differing in bit 0: lane Cc ends with the
        // half-wave total of value Cc >> 1, i.e. row Cc >> 2, component (Cc >> 1) & 1.
        double v16[16];
#pragma unroll
        for (int a = 0; a < BR; ++a) {
          z64 s = zmk(0, 0);
#pragma unroll
          for (int b = 0; b < BC; ++b) s = zadd(s, zmul(A[a][b], vloc[b]));
          v16[2 * a] = s.x;
          v16[2 * a + 1] = s.y;
        }
        const bool f4 = (Cc >> 4) & 1, f3 = (Cc >> 3) & 1, f2 = (Cc >> 2) & 1, f1 = (Cc >> 1) & 1;
        double v8[8], v4[4], v2[2];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const double snd = f4 ? v16[q] : v16[q + 8];
          const double kp = f4 ? v16[q + 8] : v16[q];
          v8[q] = kp + __shfl_xor(snd, 16, 64);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const double snd = f3 ? v8[q] : v8[q + 4];
          const double kp = f3 ? v8[q + 4] : v8[q];
          v4[q] = kp + dpp_mov<0x140>(snd);   // row_mirror
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const double snd = f2 ? v4[q] : v4[q + 2];
          const double kp = f2 ? v4[q + 2] : v4[q];
          v2[q] = kp + dpp_mov<0x141>(snd);   // row_half_mirror
        }
        double v1;
        {
          const double snd = f1 ? v2[0] : v2[1];
          const double kp = f1 ? v2[1] : v2[0];
          v1 = kp + dpp_mov<0x4E>(snd);       // quad_perm xor 2
        }
        v1 += dpp_mov<0xB1>(v1);              // quad_perm xor 1
        if (!(Cc & 1)) {
          const int i = BR * R + (Cc >> 2);
          reinterpret_cast<double*>(pbuf)[2 * i + ((Cc >> 1) & 1)] = (i > j && i < N) ? v1 : 0.0;
        }
      } else {
#pragma unroll
        for (int a = 0; a < BR; ++a) {
          z64 s = zmk(0, 0);
#pragma unroll
          for (int b = 0; b < BC; ++b) s = zadd(s, zmul(A[a][b], vloc[b]));
          s.x = gsum<32>(s.x);
          s.y = gsum<32>(s.y);
          const int i = BR * R + a;
          if (Cc == 0) pbuf[i] = (i > j && i < N) ? s : zmk(0, 0);
        }
      }
    } else if (Cc == 0) {
#pragma unroll
      for (int a = 0; a < BR; ++a) pbuf[BR * R + a] = zmk(0, 0);
    }
    __syncthreads();
    // p = tau s; alpha2 = -1/2 tau (p^H v); w = p + alpha2 v; A -= v w^H + w v^H
    z64 dt = zmk(0, 0);
    z64 pcol[BC];
#pragma unroll
    for (int b = 0; b < BC; ++b) {
      pcol[b] = zmul(tau, pbuf[BC * Cc + b]);
      dt = zadd(dt, zcmul(pcol[b], vloc[b]));
    }
    dt.x = gsum<32>(dt.x);
    dt.y = gsum<32>(dt.y);
    const z64 alpha2 = zscale(zmul(tau, dt), -0.5);
    if (live) {
#pragma unroll
    for (int a = 0; a < BR; ++a) {
      const z64 vr = vbuf[BR * R + a];
      const z64 wr = zadd(zmul(tau, pbuf[BR * R + a]), zmul(alpha2, vr));
#pragma unroll
      for (int b = 0; b < BC; ++b) {
        const z64 wc = zadd(pcol[b], zmul(alpha2, vloc[b]));
        A[a][b] = zsub(A[a][b], zadd(zmul(vr, zconj(wc)), zmul(wr, zconj(vloc[b]))));
      }
    }
    }
    // owners of column j + 1 broadcast it for the next step
    if (Cc == (j + 1) / BC) {
      constexpr int bsel = (bb + 1) % BC;
#pragma unroll
      for (int a = 0; a < BR; ++a) col_buf[BR * R + a] = A[a][bsel];
    }
    __syncthreads();
  };
  for (int jb = 0; jb + 1 < N; jb += BC) {
    static_for<BC>([&](auto bbc) {
      const int j = jb + decltype(bbc)::value;
      if (j + 1 < N) step(j, bbc);
    });
  }
  if (tid == 0) {
    d_s[N - 1] = col_buf[N - 1].x;
    e_s[N - 1] = 0.0;
  }
  const int nref = (N >= 2) ? refl_off(N - 1, N) : 0;
  for (int e = tid; e < nref; e += NTH) {
    refl[2 * e] = Rf[e].x;
    refl[2 * e + 1] = Rf[e].y;
  }
  __syncthreads();

  // ---------------------------------------------------------------- 3. eigenvalues
  // scale T to unit Gershgorin norm
  if (wave == 0) {
    double mx = 0;
    for (int i = lane; i < N; i += 64) {
      const double el = (i > 0) ? fabs(e_s[i - 1]) : 0.0;
      const double er = (i + 1 < N) ? fabs(e_s[i]) : 0.0;
      mx = fmax(mx, fabs(d_s[i]) + el + er);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
    if (lane == 0) sc_s[1] = mx;
  }
  __syncthreads();
  const double tnorm = sc_s[1];
  const bool zero = !(tnorm > 0.0);
  const double inv = zero ? 1.0 : 1.0 / tnorm;
  const double epsm = 2.220446049250313e-16;
  const double pivmin = 1e-290;
  for (int i = tid; i < N; i += NTH) {
    d_s[i] *= inv;
    e_s[i] = (i + 1 < N) ? e_s[i] * inv : 0.0;
    e2_s[i] = e_s[i] * e_s[i];
  }
  __syncthreads();
  {
    int G = 16;   // lanes per eigenvalue: the largest power of two <= 16 with G kmax <= NTH
    while (G * kmax > NTH) G >>= 1;
    const int t = tid / G, g = tid % G;
    const bool active = (t < kmax) && !zero;
    const int asc = N - 1 - t;
    double lo = -1.0 - 4 * epsm, hi = 1.0 + 4 * epsm;
    for (int it = 0; it < 24; ++it) {
      const double w = hi - lo;
      const bool done = !(w > 2 * epsm * fmax(fabs(lo), fabs(hi)) + 4 * epsm * epsm);
      if (__ballot(active && !done) == 0ull) break;
      const double x = lo + w * (double)(g + 1) / (double)(G + 1);
      const int cnt = (active && !done) ? sturm_count(d_s, e2_s, N, x, pivmin) : 0;
      const unsigned long long ball = __ballot(active && !done && cnt > asc);
      const int gb = lane & ~(G - 1);
      const unsigned long long grp = (ball >> gb) & ((1ull << G) - 1ull);
      const int first = grp ? (__ffsll((long long)grp) - 1) : G;
      const double xh = __shfl(x, gb + (first < G ? first : 0), 64);
      const double xl = __shfl(x, gb + (first == 0 ? 0 : first - 1), 64);
      if (active && !done) {
        if (first < G) hi = xh;
        if (first > 0) lo = xl;
      }
    }
    if (g == 0 && t < kmax) lam_s[t] = active ? 0.5 * (lo + hi) : 0.0;
  }
  __syncthreads();
  if (tid == 0) {
    const double ctol = 1e-9;
    int s = 0;
    for (int t = 0; t < kmax; ++t) {
      if (t > 0 && !(lam_s[t - 1] - lam_s[t] <= ctol)) s = t;
      cl_start[t] = s;
      cl_len[t] = 0;
    }
    for (int t = 0; t < kmax; ++t) cl_len[cl_start[t]] += 1;
  }
  __syncthreads();

  // ---------------------------------------------------------------- 4. eigenvectors of T
  const int KP = kmax;
  double* Dp = dyn;              // inverse LDL^T pivots, [i * KP + t]
  double* X = dyn + NP * KP;     // vectors, [i * KP + t]
  if (tid < kmax) {
    const int t = tid;
    const double sigma = lam_s[t];
    // pivots D_i of T - sigma I = L D L^T, stored as 1 / D_i
    double dp = d_s[0] - sigma;
    if (fabs(dp) < pivmin) dp = -pivmin;
    double rinv = 1.0 / dp;
    Dp[t] = rinv;
    for (int i = 1; i < N; ++i) {
      dp = (d_s[i] - sigma) - e2_s[i - 1] * rinv;
      if (fabs(dp) < pivmin) dp = -pivmin;
      rinv = 1.0 / dp;
      Dp[i * KP + t] = rinv;
    }
    for (int i = 0; i < N; ++i) X[i * KP + t] = 1.0 + hash_unit((uint32_t)t, (uint32_t)i);
  }
  __syncthreads();
  for (int iter = 0; iter < 2; ++iter) {
    if (tid < kmax) {
      const int t = tid;
      // forward: y_i -= l_{i-1} y_{i-1}, l_{i-1} = e_{i-1} / D_{i-1}
      double y = X[t];
      double rprev = Dp[t];
      for (int i = 1; i < N; ++i) {
        const double ri = Dp[i * KP + t];
        y = X[i * KP + t] - (e_s[i - 1] * rprev) * y;
        X[i * KP + t] = y;
        rprev = ri;
      }
      // backward: x_i = (y_i - e_i x_{i+1}) / D_i
      double xn = X[(N - 1) * KP + t] * Dp[(N - 1) * KP + t];
      X[(N - 1) * KP + t] = xn;
      double mx = fabs(xn);
      for (int i = N - 2; i >= 0; --i) {
        xn = (X[i * KP + t] - e_s[i] * xn) * Dp[i * KP + t];
        X[i * KP + t] = xn;
        mx = fmax(mx, fabs(xn));
      }
      const double s1 = (mx > 0) ? 1.0 / mx : 1.0;
      double nn = 0;
      for (int i = 0; i < N; ++i) {
        const double v = X[i * KP + t] * s1;
        nn += v * v;
        X[i * KP + t] = v;
      }
      const double s2 = (nn > 0) ? 1.0 / sqrt(nn) : 0.0;
      for (int i = 0; i < N; ++i) X[i * KP + t] *= s2;
    }
    __syncthreads();
    for (int cs = wave; cs < kmax; cs += NTH / 64) {
      if (cl_start[cs] != cs || cl_len[cs] < 2) continue;
      const int len = cl_len[cs];
      for (int jj = cs; jj < cs + len; ++jj) {
        for (int ii = cs; ii < jj; ++ii) {
          double dtt = 0;
          for (int i = lane; i < N; i += 64) dtt += X[i * KP + ii] * X[i * KP + jj];
          dtt = gsum<64>(dtt);
          for (int i = lane; i < N; i += 64) X[i * KP + jj] -= dtt * X[i * KP + ii];
        }
        double nn = 0;
        for (int i = lane; i < N; i += 64) nn += X[i * KP + jj] * X[i * KP + jj];
        nn = gsum<64>(nn);
        const double s2 = (nn > 0) ? 1.0 / sqrt(nn) : 0.0;
        for (int i = lane; i < N; i += 64) X[i * KP + jj] *= s2;
      }
    }
    __syncthreads();
  }

  // ---------------------------------------------------------------- 5. rank rule, V = Q Y, W
  if (tid == 0) {
    const double trace = sc_s[0];
    for (int t = 0; t < kmax; ++t) lam_s[t] = zero ? 0.0 : lam_s[t] * tnorm;
    int k = min(r_target, N);
    bool bad = !isfinite(trace) || !isfinite(tnorm);
    if (eps > 0.0) {
      double kept = 0;
      int keps = N;
      for (int i = 0; i < kmax; ++i) {
        kept += fmax(lam_s[i], 0.0);
        if (kept >= (1.0 - eps) * trace) {
          keps = i + 1;
          break;
        }
      }
      k = min(k, keps);
    }
    if (tie == 1)
      while (k > 1 && k < N && (lam_s[k - 1] - lam_s[k]) <= 1e-6 * trace) --k;
    if (k < 1) k = 1;
    double kept = 0;
    for (int i = 0; i < k; ++i) kept += fmax(lam_s[i], 0.0);
    if (!(kept > 0.0)) bad = true;
    const double scl = (renorm && kept > 0.0) ? 1.0 / sqrt(kept) : 1.0;
    DevInfo* inf = B.info;
    const double disc = fmax(trace - kept, 0.0);
    inf->k = k;
    inf->n_eig = N;
    inf->discarded = disc;
    inf->discarded_total += disc;
    inf->trace = trace;
    inf->gap = (k < N) ? (lam_s[k - 1] - lam_s[k]) : INFINITY;
    inf->lambda_max = lam_s[0];
    inf->scale = scl;
    if (bad) inf->status = (int)LRDM_E_EIG;
    k_s = k;
    sc_s[2] = scl;
  }
  __syncthreads();
  for (int t = tid; t < kmax; t += NTH) B.lam[t] = lam_s[t];
  const int k = k_s;
  const double scl = sc_s[2];
  // with a record every eigenvector is formed (kmax == N <= 64), else only the kept ones
  const int nvec = B.rec ? N : k;
  // LPC lanes per kept column (64 columns); lane g holds rows g, g + LPC, ...
  constexpr int LPC = NTH / 64;
  const int col = tid / LPC, g = tid % LPC;
  constexpr int ZR = NP / LPC;
  z64 z[ZR];
#pragma unroll
  for (int s = 0; s < ZR; ++s) {
    const int i = g + LPC * s;
    z[s] = zmk((col < nvec && i < N) ? (zero ? (i == col ? 1.0 : 0.0) : X[i * KP + col]) : 0.0, 0.0);
  }
  __syncthreads();
  // bring the reflectors back into LDS
  for (int e = tid; e < nref; e += NTH) Rf[e] = zmk(refl[2 * e], refl[2 * e + 1]);
  __syncthreads();
  if (col < nvec) {
    for (int j = N - 2; j >= 0; --j) {
      const z64 tj = zmk(tau_s[2 * j], tau_s[2 * j + 1]);
      if (tj.x == 0.0 && tj.y == 0.0) continue;
      const int ro = refl_off(j, N);
      z64 s = zmk(0, 0);
#pragma unroll
      for (int q = 0; q < ZR; ++q) {
        const int i = g + LPC * q;
        if (i >= j + 1 && i < N) {
          const z64 v = (i == j + 1) ? zmk(1, 0) : Rf[ro + (i - j - 2)];
          s = zadd(s, zcmul(v, z[q]));
        }
      }
      s.x = gsum<LPC>(s.x);
      s.y = gsum<LPC>(s.y);
      const z64 ts = zmul(tj, s);
#pragma unroll
      for (int q = 0; q < ZR; ++q) {
        const int i = g + LPC * q;
        if (i >= j + 1 && i < N) {
          const z64 v = (i == j + 1) ? zmk(1, 0) : Rf[ro + (i - j - 2)];
          z[q] = zsub(z[q], zmul(v, ts));
        }
      }
    }
  }
  __syncthreads();
  z64* V = reinterpret_cast<z64*>(dyn);   // V[i * 64 + col]
  if (col < nvec) {
#pragma unroll
    for (int s = 0; s < ZR; ++s) {
      const int i = g + LPC * s;
      if (i < N) V[i * 64 + col] = z[s];
    }
  }
  __syncthreads();
  if (B.rec) {
    double* rec = B.rec;
    if (tid == 0) {
      rec[0] = (double)k;
      rec[1] = scl;
      rec[2] = (double)N;
      rec[3] = sc_s[0];
      rec[4] = (double)renorm;
    }
    for (int t = tid; t < N; t += NTH) rec[kRecHeader + t] = lam_s[t];
    double* rv = rec + kRecHeader + N;
    for (int e = tid; e < N * N; e += NTH) {
      const z64 v = V[(e / N) * 64 + (e % N)];
      rv[2 * e] = v.x;
      rv[2 * e + 1] = v.y;
    }
  }
  using C = cx_t<T>;
  if (nsplit == 2) {
    const int rows = 2 * c, cols = 2 * c_out;
    for (int e = tid; e < rows * cols; e += NTH) {
      const int rw = e / cols, cl = e % cols;
      const int b = rw / c, v = rw % c, bp = cl / c_out, jj = cl % c_out;
      z64 acc = zmk(0, 0);
      if (jj < k) {
        for (int a = 0; a < ch.m; ++a)
          acc = zadd(acc, zmul(zmk(ch.e[a][bp][b][0], ch.e[a][bp][b][1]), V[(a * c + v) * 64 + jj]));
      }
      C o;
      o.x = (T)(acc.x * scl);
      o.y = (T)(acc.y * scl);
      W[e] = o;
      if (B.W64) {
        B.W64[2 * e] = acc.x * scl;
        B.W64[2 * e + 1] = acc.y * scl;
      }
    }
  } else {
    for (int e = tid; e < N * c_out; e += NTH) {
      const int i = e / c_out, jj = e % c_out;
      const z64 acc = (jj < k) ? V[i * 64 + jj] : zmk(0, 0);
      C o;
      o.x = (T)(acc.x * scl);
      o.y = (T)(acc.y * scl);
      W[e] = o;
    }
  }
}

template <class T, int BR, int BC>
__global__ __launch_bounds__(32 * (32 * BC / BR)) void eig_kernel(const double* __restrict__ S, int Fc, Channel ch,
                                                   int nsplit, int c, int N, int kmax, int r_target,
                                                   double eps, int tie, int renorm, int c_out,
                                                   EigBufs B, cx_t<T>* __restrict__ W) {
  eig_body<T, BR, BC>(S, Fc, ch, nsplit, c, N, kmax, r_target, eps, tie, renorm, c_out, B, W);
}

// One work-group per job; every job of a launch has the same size class (BR, BC).
template <class T, int BR, int BC>
__global__ __launch_bounds__(32 * (32 * BC / BR)) void eig_batched(const EigJob<T>* __restrict__ jobs) {
  const EigJob<T>& J = jobs[blockIdx.x];
  eig_body<T, BR, BC>(J.S, J.Fc, J.ch, J.nsplit, J.c, J.N, J.kmax, J.r_target, J.eps, J.tie, J.renorm,
                      J.c_out, J.B, J.W);
}

template <int BR, int BC>
static size_t eig_shm(int kmax) {
  constexpr int NP = 32 * BC;
  const size_t ph4 = (size_t)2 * NP * kmax * sizeof(double);
  const size_t ph5a = (size_t)(NP * (NP - 1) / 2) * 16;
  const size_t ph5b = (size_t)NP * 64 * 16;
  size_t shm = ph4;
  if (ph5a > shm) shm = ph5a;
  if (ph5b > shm) shm = ph5b;
  return shm;
}

template <class T, int BR, int BC>
static hipError_t launch_eig_batched_bs(const EigJob<T>* jobs, int njobs, int kmax_max, hipStream_t s) {
  constexpr int NP = 32 * BC;
  constexpr int NTH = 32 * (NP / BR);
  const size_t shm = eig_shm<BR, BC>(kmax_max);
  if (shm > 65536) {
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(eig_batched<T, BR, BC>),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((eig_batched<T, BR, BC>), dim3(njobs), dim3(NTH), shm, s, jobs);
  return hipGetLastError();
}

template <class T>
hipError_t launch_eig_batched(int N, const EigJob<T>* jobs, int njobs, int kmax_max, hipStream_t s) {
  if (njobs < 1 || N < 1 || N > kMaxEig || kmax_max < 1) return hipErrorInvalidValue;
  if (N <= 32) return launch_eig_batched_bs<T, 1, 1>(jobs, njobs, kmax_max, s);
  if (N <= 64) return launch_eig_batched_bs<T, 2, 2>(jobs, njobs, kmax_max, s);
  return launch_eig_batched_bs<T, 8, 4>(jobs, njobs, kmax_max, s);
}

template hipError_t launch_eig_batched<float>(int, const EigJob<float>*, int, int, hipStream_t);
template hipError_t launch_eig_batched<double>(int, const EigJob<double>*, int, int, hipStream_t);

template <class T, int BR, int BC>
static hipError_t launch_eig_bs(const double* S, int Fc, const Channel& ch, int nsplit, int c,
                                int N, int kmax, int r_target, double eps, int tie, int renorm,
                                int c_out, const EigBufs& b, cx_t<T>* W, hipStream_t s) {
  constexpr int NP = 32 * BC;
  constexpr int NTH = 32 * (NP / BR);
  const size_t ph4 = (size_t)2 * NP * kmax * sizeof(double);
  const size_t ph5a = (size_t)(NP * (NP - 1) / 2) * 16;   // packed reflectors
  const size_t ph5b = (size_t)NP * 64 * 16;               // V
  size_t shm = ph4;
  if (ph5a > shm) shm = ph5a;
  if (ph5b > shm) shm = ph5b;
  if (shm > 65536) {
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(eig_kernel<T, BR, BC>),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((eig_kernel<T, BR, BC>), dim3(1), dim3(NTH), shm, s, S, Fc, ch, nsplit, c, N, kmax,
                     r_target, eps, tie, renorm, c_out, b, W);
  return hipGetLastError();
}

template <class T>
hipError_t launch_eig(const double* S, int Fc, const Channel& ch, int nsplit, int c, int N,
                      int kmax, int r_target, double eps, int tie, int renorm, int c_out,
                      const EigBufs& b, cx_t<T>* W, hipStream_t s) {
  if (N < 1 || N > kMaxEig || kmax < 1 || kmax > N || r_target > 64) return hipErrorInvalidValue;
  if (b.rec && (N > kRecMaxN || kmax != N)) return hipErrorInvalidValue;
  if (N <= 32) return launch_eig_bs<T, 1, 1>(S, Fc, ch, nsplit, c, N, kmax, r_target, eps, tie, renorm, c_out, b, W, s);
  if (N <= 64) return launch_eig_bs<T, 2, 2>(S, Fc, ch, nsplit, c, N, kmax, r_target, eps, tie, renorm, c_out, b, W, s);
  return launch_eig_bs<T, 8, 4>(S, Fc, ch, nsplit, c, N, kmax, r_target, eps, tie, renorm, c_out, b, W, s);
}

template hipError_t launch_eig<float>(const double*, int, const Channel&, int, int, int, int, int, double,
                                      int, int, int, const EigBufs&, float2*, hipStream_t);
template hipError_t launch_eig<double>(const double*, int, const Channel&, int, int, int, int, int, double,
                                       int, int, int, const EigBufs&, double2*, hipStream_t);

}  // namespace lrdm
