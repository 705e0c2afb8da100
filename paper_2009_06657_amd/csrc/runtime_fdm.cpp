// Host runtime of the full-rank density-matrix comparator (Eq. "full rank evolution",
// Sec. II.A): validation, the pass scheduler over the 2n index bits of rho, and the C ABI
// (lrdm_fdm_*) declared in include/lrdm.h.  No device memory is allocated here.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "lrdm_internal.h"

using namespace lrdm;

struct lrdm_fdm_ctx {
  struct Op {
    int type;          // OP_1Q, OP_2Q (slots), OP_DIAG1, OP_DIAG2 (index bits)
    int a, b;          // index bits
    uint64_t mask;     // index bits touched
    std::vector<double> coef;  // interleaved complex: 2x2 / 4x4 row-major, or 2 / 4 diagonal entries
  };
  int n = 0;
  float2* rho = nullptr;
  hipStream_t stream = nullptr;
  bool poisoned = false;
  std::string err;
  std::vector<Op> ops;
};

namespace {

lrdm_status ffail(lrdm_fdm_t h, lrdm_status st, const std::string& msg) {
  set_last_error(msg.c_str());
  if (h) h->err = msg;
  return st;
}

lrdm_status fhip(lrdm_fdm_t h, hipError_t e, const char* where) {
  if (e == hipSuccess) return LRDM_OK;
  h->poisoned = true;
  return ffail(h, LRDM_E_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define FHIP(h, expr)                                      \
  do {                                                     \
    lrdm_status _s = fhip((h), (expr), #expr);             \
    if (_s != LRDM_OK) return _s;                          \
  } while (0)

lrdm_status fusable(lrdm_fdm_t h) {
  if (!h) return ffail(nullptr, LRDM_E_ARG, "null handle");
  if (h->poisoned) return ffail(h, LRDM_E_STATE, "handle is poisoned by an earlier device error: " + h->err);
  return LRDM_OK;
}

bool unitary(const double* u, int d) {
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) {
      double re = 0, im = 0;
      for (int k = 0; k < d; ++k) {
        const double ar = u[2 * (k * d + i)], ai = -u[2 * (k * d + i) + 1];
        const double br = u[2 * (k * d + j)], bi = u[2 * (k * d + j) + 1];
        re += ar * br - ai * bi;
        im += ar * bi + ai * br;
      }
      if (!(std::fabs(re - (i == j ? 1.0 : 0.0)) <= 1e-10 && std::fabs(im) <= 1e-10)) return false;
    }
  return true;
}

void push_op(lrdm_fdm_t h, int type, int a, int b, const std::vector<double>& coef) {
  lrdm_fdm_ctx::Op op;
  op.type = type;
  op.a = a;
  op.b = b;
  op.mask = (1ull << a) | (b >= 0 ? (1ull << b) : 0ull);
  op.coef = coef;
  h->ops.push_back(op);
}

// d x d complex matrix (interleaved FP64), optionally conjugated
std::vector<double> mat(const double* u, int d, bool conj) {
  std::vector<double> c(2 * d * d);
  for (int i = 0; i < d * d; ++i) {
    c[2 * i] = u[2 * i];
    c[2 * i + 1] = conj ? -u[2 * i + 1] : u[2 * i + 1];
  }
  return c;
}

// An operation as a dense d x d matrix over the ordered bit list (x) or (x, y), element
// t = bit x + 2 bit y.
void dense_on(const lrdm_fdm_ctx::Op& op, int x, int y, int d, double* m) {
  std::fill(m, m + 2 * d * d, 0.0);
  const bool diag = op.type == OP_DIAG1 || op.type == OP_DIAG2;
  const bool two = op.type == OP_2Q || op.type == OP_DIAG2;
  auto bitof = [&](int t, int bit) { return bit == x ? (t & 1) : ((t >> 1) & 1); };
  for (int to = 0; to < d; ++to)
    for (int ti = 0; ti < d; ++ti) {
      // the operation's own indices and the identity on the remaining bit
      const int so = bitof(to, op.a) + (two ? 2 * bitof(to, op.b) : 0);
      const int si = bitof(ti, op.a) + (two ? 2 * bitof(ti, op.b) : 0);
      bool same_rest = true;
      if (d == 4 && !two) {
        const int other = op.a == x ? y : x;
        same_rest = bitof(to, other) == bitof(ti, other);
      }
      if (!same_rest) continue;
      const int od = two ? 4 : 2;
      double re, im;
      if (diag) {
        if (so != si) continue;
        re = op.coef[2 * so];
        im = op.coef[2 * so + 1];
      } else {
        re = op.coef[2 * (so * od + si)];
        im = op.coef[2 * (so * od + si) + 1];
      }
      m[2 * (to * d + ti)] = re;
      m[2 * (to * d + ti) + 1] = im;
    }
}

// Operator fusion: an operation joins the latest earlier operation that touches any of its index
// bits when the two together act on at most 2 bits (everything in between acts on other bits
// and commutes with it).  The product is formed in FP64; two diagonal operations stay diagonal.
// A 1-bit operation may also join the latest operation on the other index bit of the same qubit
// (row bit n + q <-> column bit q) when nothing after that one touches its own bit: the pair
// U (x) conj(U) then becomes one 4 x 4 operator that the qubit's channels fuse into.
void fuse_ops(std::vector<lrdm_fdm_ctx::Op>& ops, int n) {
  std::vector<lrdm_fdm_ctx::Op> out;
  std::vector<int> latest(64, -1);
  for (auto& op : ops) {
    int x = -1;
    for (int b = 0; b < 64; ++b)
      if ((op.mask >> b) & 1ull) x = std::max(x, latest[b]);
    if ((x < 0 || __builtin_popcountll(out[x].mask | op.mask) > 2) && __builtin_popcountll(op.mask) == 1) {
      const int b = __builtin_ctzll(op.mask);
      const int y = latest[b >= n ? b - n : b + n];
      if (y >= 0 && y >= x && __builtin_popcountll(out[y].mask | op.mask) <= 2) x = y;
    }
    if (x >= 0 && __builtin_popcountll(out[x].mask | op.mask) <= 2) {
      auto& X = out[x];
      const uint64_t um = X.mask | op.mask;
      const int b0 = __builtin_ctzll(um);
      const int b1 = um == (1ull << b0) ? -1 : 63 - __builtin_clzll(um);
      const int d = b1 < 0 ? 2 : 4;
      double mx[32], mo[32];
      dense_on(X, b0, b1, d, mx);
      dense_on(op, b0, b1, d, mo);
      std::vector<double> prod(2 * d * d, 0.0);
      for (int i = 0; i < d; ++i)
        for (int j = 0; j < d; ++j)
          for (int k = 0; k < d; ++k) {
            const double ar = mo[2 * (i * d + k)], ai = mo[2 * (i * d + k) + 1];
            const double br = mx[2 * (k * d + j)], bi = mx[2 * (k * d + j) + 1];
            prod[2 * (i * d + j)] += ar * br - ai * bi;
            prod[2 * (i * d + j) + 1] += ar * bi + ai * br;
          }
      const bool diag = (X.type == OP_DIAG1 || X.type == OP_DIAG2) && (op.type == OP_DIAG1 || op.type == OP_DIAG2);
      X.a = b0;
      X.b = b1;
      X.mask = um;
      if (diag) {
        X.type = d == 2 ? OP_DIAG1 : OP_DIAG2;
        X.coef.assign(2 * d, 0.0);
        for (int i = 0; i < d; ++i) {
          X.coef[2 * i] = prod[2 * (i * d + i)];
          X.coef[2 * i + 1] = prod[2 * (i * d + i) + 1];
        }
      } else {
        X.type = d == 2 ? OP_1Q : OP_2Q;
        X.coef = prod;
      }
      // a bit of X may have later operations; only the joining operation's bits move to X
      for (int b = 0; b < 64; ++b)
        if ((op.mask >> b) & 1ull) latest[b] = std::max(latest[b], x);
    } else {
      out.push_back(op);
      for (int b = 0; b < 64; ++b)
        if ((op.mask >> b) & 1ull) latest[b] = (int)out.size() - 1;
    }
  }
  ops.swap(out);
}

// Register phases of a full-tile pass: consecutive operations whose non-diagonal operands fit
// in 4 tile slots share a phase (diagonal operations join the current one).  Each phase holds
// exactly 4 distinct slots, filled preferably above the low block so that lanes run along the
// contiguous low index bits; operands become register indices (0..3), and a 2-slot operator
// whose first operand maps above its second has its 4x4 matrix permuted (t = 1 <-> t = 2).
void build_phases(FdmPass& p) {
  int nph = 0, cur[4], ncur = 0;
  auto reg_of = [&](int slot) {
    for (int r = 0; r < ncur; ++r) if (cur[r] == slot) return r;
    return -1;
  };
  auto close_phase = [&](int ph) {
    bool used[kFdmMaxLocal] = {};
    for (int r = 0; r < ncur; ++r) used[cur[r]] = true;
    for (int sl = p.k - 1; sl >= 0 && ncur < 4; --sl)
      if (!used[sl]) { cur[ncur++] = sl; used[sl] = true; }
    for (int r = 0; r < 4; ++r) p.ph_slots[ph][r] = (unsigned char)cur[r];
  };
  for (int o = 0; o < p.n_ops; ++o) {
    const int ty = p.op_type[o];
    const bool diag = ty == OP_DIAG1 || ty == OP_DIAG2;
    int need[2], nn = 0;
    if (!diag) {
      need[nn++] = p.op_a[o];
      if (ty == OP_2Q) need[nn++] = p.op_b[o];
    }
    int extra = 0;
    for (int j = 0; j < nn; ++j) extra += reg_of(need[j]) < 0;
    if (nph == 0 || ncur + extra > 4) {
      if (nph > 0) close_phase(nph - 1);
      p.ph_first[nph] = (unsigned char)o;
      p.ph_count[nph] = 0;
      ++nph;
      ncur = 0;
    }
    for (int j = 0; j < nn; ++j)
      if (reg_of(need[j]) < 0) cur[ncur++] = need[j];
    ++p.ph_count[nph - 1];
  }
  if (nph > 0) close_phase(nph - 1);
  // HBM accesses happen in the first and last phase: when one of them holds a low slot (lanes
  // would then not run along the contiguous low bits), an empty phase on the top 4 slots does
  // the load or the store instead, at the cost of one more LDS exchange
  auto has_low = [&](int ph) {
    for (int r = 0; r < 4; ++r) if (p.ph_slots[ph][r] < kFdmLowBits) return true;
    return false;
  };
  auto empty_phase = [&](int at, int first) {
    for (int ph = nph; ph > at; --ph) {
      p.ph_first[ph] = p.ph_first[ph - 1];
      p.ph_count[ph] = p.ph_count[ph - 1];
      for (int r = 0; r < 4; ++r) p.ph_slots[ph][r] = p.ph_slots[ph - 1][r];
    }
    p.ph_first[at] = (unsigned char)first;
    p.ph_count[at] = 0;
    for (int r = 0; r < 4; ++r) p.ph_slots[at][r] = (unsigned char)(p.k - 4 + r);
    ++nph;
  };
  if (nph > 0 && has_low(0)) empty_phase(0, 0);
  if (nph > 0 && has_low(nph - 1)) empty_phase(nph, p.n_ops);
  p.n_phases = nph;
  // slots -> register indices
  for (int ph = 0; ph < nph; ++ph)
    for (int o = p.ph_first[ph]; o < p.ph_first[ph] + p.ph_count[ph]; ++o) {
      const int ty = p.op_type[o];
      auto reg = [&](int slot) {
        for (int r = 0; r < 4; ++r) if (p.ph_slots[ph][r] == slot) return r;
        return -1;
      };
      if (ty == OP_DIAG1 || ty == OP_DIAG2) {
        // an operand on a register bit becomes 64 + register; register operands come first, in
        // ascending order (a swap permutes the 4 diagonal entries, t = 1 <-> t = 2)
        auto reg_of_bit = [&](int bit) {
          for (int sl = 0; sl < p.k; ++sl)
            if (p.local_q[sl] == bit) return reg(sl);
          return -1;
        };
        int qa = p.op_a[o], qb = ty == OP_DIAG2 ? p.op_b[o] : -1;
        int ra = reg_of_bit(qa), rb = qb >= 0 ? reg_of_bit(qb) : -1;
        if (ty == OP_DIAG2 && ((ra < 0 && rb >= 0) || (ra >= 0 && rb >= 0 && rb < ra))) {
          float* u = p.coef + p.op_coef[o];
          std::swap(u[2], u[4]);
          std::swap(u[3], u[5]);
          std::swap(qa, qb);
          std::swap(ra, rb);
        }
        p.op_a[o] = ra >= 0 ? 64 + ra : qa;
        if (ty == OP_DIAG2) p.op_b[o] = rb >= 0 ? 64 + rb : qb;
        continue;
      }
      int ra = reg(p.op_a[o]), rb = ty == OP_2Q ? reg(p.op_b[o]) : 0;
      if (ty == OP_2Q && ra > rb) {
        float* u = p.coef + p.op_coef[o];
        float t[32];
        const int sg[4] = {0, 2, 1, 3};
        for (int r = 0; r < 4; ++r)
          for (int m = 0; m < 4; ++m) {
            t[8 * r + 2 * m] = u[8 * sg[r] + 2 * sg[m]];
            t[8 * r + 2 * m + 1] = u[8 * sg[r] + 2 * sg[m] + 1];
          }
        std::memcpy(u, t, sizeof(t));
        std::swap(ra, rb);
      }
      p.op_a[o] = ra;
      p.op_b[o] = rb;
    }
}

lrdm_status flush(lrdm_fdm_t h) {
  const int nbits = 2 * h->n;
  const int kmax = std::min(kFdmMaxLocal, nbits);
  const int lo = std::min(kmax, kFdmLowBits);
  const int free_slots = kmax - lo;
  const uint64_t lowmask = (1ull << lo) - 1ull;
  fuse_ops(h->ops, h->n);
  std::vector<char> placed(h->ops.size(), 0);
  size_t remaining = h->ops.size();
  while (remaining > 0) {
    FdmPass p;
    std::memset(&p, 0, sizeof(p));
    p.nbits = nbits;
    std::vector<int> hi;
    uint64_t locmask = lowmask, blocked = 0;
    int nc = 0;
    for (size_t i = 0; i < h->ops.size(); ++i) {
      if (placed[i]) continue;
      const auto& op = h->ops[i];
      if (op.mask & blocked) { blocked |= op.mask; continue; }
      if (p.n_ops >= kFdmMaxOps || nc + (int)op.coef.size() > kFdmMaxCoef) { blocked = ~0ull; continue; }
      const bool diag = op.type == OP_DIAG1 || op.type == OP_DIAG2;
      if (!diag) {
        const uint64_t need = op.mask & ~locmask;
        if ((int)hi.size() + __builtin_popcountll(need) > free_slots) { blocked |= op.mask; continue; }
        for (int b = 0; b < nbits; ++b)
          if (need & (1ull << b)) { hi.push_back(b); locmask |= 1ull << b; }
      }
      auto slot = [&](int bit) {
        if (bit < lo) return bit;
        for (size_t j = 0; j < hi.size(); ++j) if (hi[j] == bit) return lo + (int)j;
        return -1;
      };
      const int o = p.n_ops++;
      p.op_type[o] = op.type;
      p.op_coef[o] = nc;
      if (diag) {
        p.op_a[o] = op.a;
        p.op_b[o] = op.b;
      } else {
        p.op_a[o] = slot(op.a);
        p.op_b[o] = op.b >= 0 ? slot(op.b) : 0;
      }
      for (double v : op.coef) p.coef[nc++] = (float)v;
      placed[i] = 1;
      --remaining;
    }
    // fill the tile with unused bits so that every pass has full-size tiles
    for (int b = lo; b < nbits && (int)hi.size() < free_slots; ++b)
      if (!(locmask & (1ull << b))) { hi.push_back(b); locmask |= 1ull << b; }
    p.k = lo + (int)hi.size();
    for (int j = 0; j < lo; ++j) p.local_q[j] = j;
    for (size_t j = 0; j < hi.size(); ++j) p.local_q[lo + j] = hi[j];
    std::vector<int> sh = hi;
    std::sort(sh.begin(), sh.end());
    for (size_t j = 0; j < sh.size(); ++j) p.sorted_hi[j] = sh[j];
    if (p.k == kFdmMaxLocal) build_phases(p);
    FHIP(h, launch_fdm_pass(p, h->rho, h->stream));
  }
  h->ops.clear();
  return LRDM_OK;
}

}  // namespace

extern "C" {

lrdm_status lrdm_fdm_state_bytes(int n, size_t* bytes) {
  if (!bytes) return ffail(nullptr, LRDM_E_ARG, "null output pointer");
  if (n < 1 || n > 16) return ffail(nullptr, LRDM_E_ARG, "n must be in [1, 16]");
  *bytes = (size_t)8 << (2 * n);
  return LRDM_OK;
}

lrdm_status lrdm_fdm_init(lrdm_fdm_t* out, int n, void* state_dev, size_t state_bytes, void* hip_stream) {
  if (!out) return ffail(nullptr, LRDM_E_ARG, "null output handle pointer");
  *out = nullptr;
  if (n < 1 || n > 16) return ffail(nullptr, LRDM_E_ARG, "n must be in [1, 16]");
  if (!state_dev) return ffail(nullptr, LRDM_E_ARG, "null device buffer");
  if (state_bytes < ((size_t)8 << (2 * n))) return ffail(nullptr, LRDM_E_NOMEM, "state buffer smaller than 8 * 4^n bytes");
  if (reinterpret_cast<uintptr_t>(state_dev) & 255) return ffail(nullptr, LRDM_E_ARG, "device buffer must be 256-byte aligned");
  lrdm_fdm_ctx* h = new lrdm_fdm_ctx();
  h->n = n;
  h->rho = static_cast<float2*>(state_dev);
  h->stream = static_cast<hipStream_t>(hip_stream);
  const hipError_t e = launch_fdm_reset(h->rho, n, h->stream);
  if (e != hipSuccess) {
    ffail(nullptr, LRDM_E_HIP, std::string("launch_fdm_reset: ") + hipGetErrorString(e));
    delete h;
    return LRDM_E_HIP;
  }
  *out = h;
  return LRDM_OK;
}

lrdm_status lrdm_fdm_reset(lrdm_fdm_t h) {
  lrdm_status st = fusable(h);
  if (st != LRDM_OK) return st;
  h->ops.clear();
  FHIP(h, launch_fdm_reset(h->rho, h->n, h->stream));
  return LRDM_OK;
}

lrdm_status lrdm_fdm_destroy(lrdm_fdm_t h) {
  if (!h) return ffail(nullptr, LRDM_E_ARG, "null handle");
  delete h;
  return LRDM_OK;
}

lrdm_status lrdm_fdm_apply_gate(lrdm_fdm_t h, int k, const int* qubits, const double* u) {
  lrdm_status st = fusable(h);
  if (st != LRDM_OK) return st;
  if (k != 1 && k != 2) return ffail(h, LRDM_E_ARG, "k must be 1 or 2");
  if (!qubits || !u) return ffail(h, LRDM_E_ARG, "null qubits or matrix");
  for (int j = 0; j < k; ++j)
    if (qubits[j] < 0 || qubits[j] >= h->n) return ffail(h, LRDM_E_ARG, "qubit out of range");
  if (k == 2 && qubits[0] == qubits[1]) return ffail(h, LRDM_E_ARG, "repeated qubit");
  const int d = 1 << k;
  if (!unitary(u, d)) return ffail(h, LRDM_E_ARG, "gate matrix is not unitary within 1e-10");
  bool diag = true;
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j)
      if (i != j && (u[2 * (i * d + j)] != 0.0 || u[2 * (i * d + j) + 1] != 0.0)) diag = false;
  const int n = h->n;
  if (diag) {
    std::vector<double> ph(2 * d), phc(2 * d);
    for (int i = 0; i < d; ++i) {
      ph[2 * i] = phc[2 * i] = u[2 * (i * d + i)];
      ph[2 * i + 1] = u[2 * (i * d + i) + 1];
      phc[2 * i + 1] = -ph[2 * i + 1];
    }
    if (k == 1) {
      push_op(h, OP_DIAG1, n + qubits[0], -1, ph);
      push_op(h, OP_DIAG1, qubits[0], -1, phc);
    } else {
      push_op(h, OP_DIAG2, n + qubits[0], n + qubits[1], ph);
      push_op(h, OP_DIAG2, qubits[0], qubits[1], phc);
    }
    return LRDM_OK;
  }
  if (k == 1) {
    push_op(h, OP_1Q, n + qubits[0], -1, mat(u, 2, false));
    push_op(h, OP_1Q, qubits[0], -1, mat(u, 2, true));
  } else {
    push_op(h, OP_2Q, n + qubits[0], n + qubits[1], mat(u, 4, false));
    push_op(h, OP_2Q, qubits[0], qubits[1], mat(u, 4, true));
  }
  return LRDM_OK;
}

lrdm_status lrdm_fdm_apply_kraus(lrdm_fdm_t h, int qubit, int m, const double* e) {
  lrdm_status st = fusable(h);
  if (st != LRDM_OK) return st;
  if (qubit < 0 || qubit >= h->n) return ffail(h, LRDM_E_ARG, "qubit out of range");
  if (m < 1 || m > 4) return ffail(h, LRDM_E_ARG, "Kraus count must be in [1, 4]");
  if (!e) return ffail(h, LRDM_E_ARG, "null Kraus matrices");
  // completeness sum_a E_a^H E_a = I
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      double re = 0, im = 0;
      for (int a = 0; a < m; ++a)
        for (int r = 0; r < 2; ++r) {
          const double ar = e[((a * 2 + r) * 2 + i) * 2], ai = -e[((a * 2 + r) * 2 + i) * 2 + 1];
          const double br = e[((a * 2 + r) * 2 + j) * 2], bi = e[((a * 2 + r) * 2 + j) * 2 + 1];
          re += ar * br - ai * bi;
          im += ar * bi + ai * br;
        }
      if (!(std::fabs(re - (i == j)) <= 1e-10 && std::fabs(im) <= 1e-10))
        return ffail(h, LRDM_E_ARG, "Kraus set is not complete within 1e-10");
    }
  // S[(r + 2c), (r' + 2c')] = sum_a E_a[r][r'] conj(E_a[c][c']) on the bit pair (n + q, q)
  std::vector<double> S(32);
  for (int mo = 0; mo < 4; ++mo)
    for (int mi = 0; mi < 4; ++mi) {
      const int r = mo & 1, c = mo >> 1, rp = mi & 1, cp = mi >> 1;
      double re = 0, im = 0;
      for (int a = 0; a < m; ++a) {
        const double xr = e[((a * 2 + r) * 2 + rp) * 2], xi = e[((a * 2 + r) * 2 + rp) * 2 + 1];
        const double yr = e[((a * 2 + c) * 2 + cp) * 2], yi = -e[((a * 2 + c) * 2 + cp) * 2 + 1];
        re += xr * yr - xi * yi;
        im += xr * yi + xi * yr;
      }
      S[2 * (mo * 4 + mi)] = re;
      S[2 * (mo * 4 + mi) + 1] = im;
    }
  push_op(h, OP_2Q, h->n + qubit, qubit, S);
  return LRDM_OK;
}

lrdm_status lrdm_fdm_apply_diagonal_weight(lrdm_fdm_t h, const double* phase) {
  lrdm_status st = fusable(h);
  if (st != LRDM_OK) return st;
  if (!phase) return ffail(h, LRDM_E_ARG, "null phase table");
  FdmPhase ph{};
  for (int w = 0; w <= h->n; ++w) {
    const double m = std::hypot(phase[2 * w], phase[2 * w + 1]);
    if (!(std::fabs(m - 1.0) <= 1e-10)) return ffail(h, LRDM_E_ARG, "phase entries must have unit modulus");
    ph.ph[2 * w] = phase[2 * w];
    ph.ph[2 * w + 1] = phase[2 * w + 1];
  }
  st = flush(h);   // queued operations come first
  if (st != LRDM_OK) return st;
  FHIP(h, launch_fdm_weight(h->rho, h->n, ph, h->stream));
  return LRDM_OK;
}

lrdm_status lrdm_fdm_probabilities(lrdm_fdm_t h, double* p_dev) {
  lrdm_status st = fusable(h);
  if (st != LRDM_OK) return st;
  if (!p_dev) return ffail(h, LRDM_E_ARG, "null output buffer");
  st = flush(h);
  if (st != LRDM_OK) return st;
  FHIP(h, launch_fdm_diag(h->rho, h->n, p_dev, h->stream));
  return LRDM_OK;
}

lrdm_status lrdm_fdm_synchronize(lrdm_fdm_t h) {
  lrdm_status st = fusable(h);
  if (st != LRDM_OK) return st;
  st = flush(h);
  if (st != LRDM_OK) return st;
  FHIP(h, hipStreamSynchronize(h->stream));
  return LRDM_OK;
}

const char* lrdm_fdm_last_error(lrdm_fdm_t h) { return h ? h->err.c_str() : ""; }

}  // extern "C"

lrdm_status lrdm::fdm_state(lrdm_fdm_t f, float2** rho, int* n, hipStream_t* s) {
  lrdm_status st = fusable(f);
  if (st != LRDM_OK) return st;
  *rho = f->rho;
  *n = f->n;
  *s = f->stream;
  return LRDM_OK;
}

void lrdm::fdm_discard_queue(lrdm_fdm_t f) {
  if (f) f->ops.clear();
}
