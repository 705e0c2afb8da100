// Program-level entry points of liblrdm: Algorithm 1 over a flat operation array (lrdm_run),
// the energy and its gradient by one forward pass and one reverse sweep (lrdm_energy_grad), and
// a whole batch recorded, captured and replayed in one call (lrdm_batch_run).  Everything here
// is host control flow over the operation-level C ABI; every step of the evolution and of its
// adjoint runs in the library's kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "lrdm_internal.h"

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

lrdm_status pfail(lrdm_status st, const std::string& msg) {
  lrdm::set_last_error(msg.c_str());
  return st;
}

// Shape facts of a handle needed here, read through the public ABI.
struct Shape {
  int n = 0;
  size_t state_bytes = 0, rec_bytes = 0;
};

// R_P(theta) = exp(-i theta P / 2) = cos(theta/2) I - i sin(theta/2) P, 2 x 2 interleaved.
void rotation_matrix(int axis, double theta, double* u) {
  const double c = std::cos(0.5 * theta), s = std::sin(0.5 * theta);
  std::memset(u, 0, 8 * sizeof(double));
  u[0] = c;   // (0,0)
  u[6] = c;   // (1,1)
  if (axis == 1) {        // X: -i s on the off-diagonal
    u[3] = -s;
    u[5] = -s;
  } else if (axis == 2) { // Y: [[0, -1], [1, 0]] * s
    u[2] = -s;
    u[4] = s;
  } else {                // Z: diag(e^{-i theta/2}, e^{i theta/2})
    u[1] = -s;
    u[7] = s;
  }
}

bool op_uses_coef(const lrdm_op& o, int n, int64_t& need) {
  switch (o.kind) {
    case LRDM_OP_GATE: need = 2ll * (1 << o.k) * (1 << o.k); return true;
    case LRDM_OP_ROTATION: need = 8; return true;
    case LRDM_OP_WEIGHT: need = 2ll * (n + 1); return true;
    case LRDM_OP_KRAUS: need = 8ll * o.k; return true;
    case LRDM_OP_KRAUS2: need = 32ll * o.k; return true;
    default: need = 0; return false;
  }
}

// Structural validation of a program for a handle of n qubits (everything that does not need
// the matrices' values; those are checked by the operation-level calls, and by a dry check
// below before anything is enqueued).
lrdm_status validate(const lrdm_program* p, int n, const double* params, int n_params, bool need_channels) {
  if (!p || p->n_ops < 0 || (p->n_ops > 0 && !p->ops)) return pfail(LRDM_E_ARG, "null or empty program");
  for (int i = 0; i < p->n_ops; ++i) {
    const lrdm_op& o = p->ops[i];
    const std::string at = "op " + std::to_string(i) + ": ";
    int64_t need = 0;
    if (o.kind < LRDM_OP_GATE || o.kind > LRDM_OP_KRAUS2) return pfail(LRDM_E_ARG, at + "unknown kind");
    if (op_uses_coef(o, n, need)) {
      if (!p->coef || o.off < 0 || o.off + need > p->n_coef)
        if (!(o.kind == LRDM_OP_ROTATION && params)) return pfail(LRDM_E_ARG, at + "coefficients out of range");
    }
    if (o.kind == LRDM_OP_GATE) {
      if (o.k != 1 && o.k != 2) return pfail(LRDM_E_ARG, at + "gate k must be 1 or 2");
      if (o.q0 < 0 || o.q0 >= n || (o.k == 2 && (o.q1 < 0 || o.q1 >= n || o.q1 == o.q0)))
        return pfail(LRDM_E_ARG, at + "gate qubits out of range or repeated");
    } else if (o.kind == LRDM_OP_ROTATION) {
      if (o.q0 < 0 || o.q0 >= n) return pfail(LRDM_E_ARG, at + "rotation qubit out of range");
      if (o.axis < 1 || o.axis > 3) return pfail(LRDM_E_ARG, at + "rotation axis must be 1 (X), 2 (Y) or 3 (Z)");
      if (o.param < 0 || (params && o.param >= n_params)) return pfail(LRDM_E_ARG, at + "rotation parameter index out of range");
    } else if (o.kind == LRDM_OP_KRAUS) {
      if (o.q0 < 0 || o.q0 >= n) return pfail(LRDM_E_ARG, at + "channel qubit out of range");
      if (o.k < 1 || o.k > 4) return pfail(LRDM_E_ARG, at + "channel operator count must be in [1, 4]");
      if (i + 1 >= p->n_ops || p->ops[i + 1].kind != LRDM_OP_COMPRESS)
        return pfail(LRDM_E_ARG, at + "a channel must be followed by a compression");
    } else if (o.kind == LRDM_OP_KRAUS2) {
      if (o.q0 < 0 || o.q0 >= n || o.q1 < 0 || o.q1 >= n || o.q0 == o.q1)
        return pfail(LRDM_E_ARG, at + "channel qubits out of range or repeated");
      if (o.k < 1 || o.k > 16) return pfail(LRDM_E_ARG, at + "two-qubit channel operator count must be in [1, 16]");
      if (i + 1 >= p->n_ops || p->ops[i + 1].kind != LRDM_OP_COMPRESS)
        return pfail(LRDM_E_ARG, at + "a channel must be followed by a compression");
      if (need_channels) return pfail(LRDM_E_UNSUPPORTED, at + "the reverse sweep takes one-qubit channels only");
    } else if (o.kind == LRDM_OP_COMPRESS) {
      if (need_channels && (i == 0 || p->ops[i - 1].kind != LRDM_OP_KRAUS))
        return pfail(LRDM_E_UNSUPPORTED, at + "the reverse sweep needs a channel before every compression");
    }
  }
  return LRDM_OK;
}

const double* op_matrix(const lrdm_program* p, const lrdm_op& o, const double* params, double* tmp) {
  if (o.kind == LRDM_OP_ROTATION && params) {
    rotation_matrix(o.axis, params[o.param], tmp);
    return tmp;
  }
  return p->coef + o.off;
}

// Issue one operation on h (the operation-level calls validate their arguments).
lrdm_status issue(lrdm_t h, const lrdm_program* p, const lrdm_op& o, const double* params,
                  double* rec_dev) {
  double tmp[8];
  switch (o.kind) {
    case LRDM_OP_GATE:
    case LRDM_OP_ROTATION: {
      const int q[2] = {o.q0, o.q1};
      return lrdm_apply_gate(h, o.kind == LRDM_OP_GATE ? o.k : 1, q, op_matrix(p, o, params, tmp));
    }
    case LRDM_OP_WEIGHT: return lrdm_apply_diagonal_weight(h, p->coef + o.off);
    case LRDM_OP_KRAUS: return lrdm_apply_kraus(h, o.q0, o.k, p->coef + o.off);
    case LRDM_OP_KRAUS2: return lrdm_apply_kraus2(h, o.q0, o.q1, o.k, p->coef + o.off);
    case LRDM_OP_COMPRESS:
      return rec_dev ? lrdm_compress_record(h, o.r, o.eps, o.tie, o.renorm, rec_dev, nullptr)
                     : lrdm_compress(h, o.r, o.eps, o.tie, o.renorm, nullptr);
    default: return LRDM_OK;
  }
}

// Layers: [begin, end) ranges of operation indices separated by LRDM_OP_LAYER marks (a trailing
// range without a mark counts as a layer).
std::vector<std::pair<int, int>> split_layers(const lrdm_program* p) {
  std::vector<std::pair<int, int>> segs;
  int b = 0;
  for (int i = 0; i < p->n_ops; ++i)
    if (p->ops[i].kind == LRDM_OP_LAYER) {
      segs.push_back({b, i});
      b = i + 1;
    }
  if (b < p->n_ops) segs.push_back({b, p->n_ops});
  return segs;
}

lrdm_status shape_of(lrdm_t h, Shape& s) {
  int n = 0, ld = 0, r_pad = 0;
  size_t sb = 0;
  lrdm_status st = lrdm_layout(h, &n, &ld, &r_pad, &sb);
  if (st != LRDM_OK) return st;
  s.n = n;
  s.state_bytes = sb;
  return LRDM_OK;
}

// Dry check of the values (unitarity, completeness, phase modulus) on a scratch copy of the
// rules the operation-level calls apply, so that lrdm_run enqueues nothing for a bad program.
bool values_ok(const lrdm_program* p, int n, const double* params, std::string& why) {
  for (int i = 0; i < p->n_ops; ++i) {
    const lrdm_op& o = p->ops[i];
    double tmp[8];
    if (o.kind == LRDM_OP_GATE || o.kind == LRDM_OP_ROTATION) {
      const int d = o.kind == LRDM_OP_GATE ? (1 << o.k) : 2;
      const double* u = op_matrix(p, o, params, tmp);
      for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) {
          double re = 0, im = 0;
          for (int k = 0; k < d; ++k) {
            const double ar = u[2 * (k * d + a)], ai = -u[2 * (k * d + a) + 1];
            const double br = u[2 * (k * d + b)], bi = u[2 * (k * d + b) + 1];
            re += ar * br - ai * bi;
            im += ar * bi + ai * br;
          }
          if (!(std::fabs(re - (a == b ? 1.0 : 0.0)) <= 1e-10 && std::fabs(im) <= 1e-10)) {
            why = "op " + std::to_string(i) + ": gate matrix is not unitary within 1e-10";
            return false;
          }
        }
    } else if (o.kind == LRDM_OP_WEIGHT) {
      for (int w = 0; w <= n; ++w)
        if (!(std::fabs(std::hypot(p->coef[o.off + 2 * w], p->coef[o.off + 2 * w + 1]) - 1.0) <= 1e-10)) {
          why = "op " + std::to_string(i) + ": phase entries must have unit modulus";
          return false;
        }
    } else if (o.kind == LRDM_OP_KRAUS || o.kind == LRDM_OP_KRAUS2) {
      const double* e = p->coef + o.off;
      const int d = o.kind == LRDM_OP_KRAUS ? 2 : 4;
      for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b) {
          double re = 0, im = 0;
          for (int m = 0; m < o.k; ++m)
            for (int r = 0; r < d; ++r) {
              const double xr = e[((m * d + r) * d + a) * 2], xi = -e[((m * d + r) * d + a) * 2 + 1];
              const double yr = e[((m * d + r) * d + b) * 2], yi = e[((m * d + r) * d + b) * 2 + 1];
              re += xr * yr - xi * yi;
              im += xr * yi + xi * yr;
            }
          if (!(std::fabs(re - (a == b ? 1.0 : 0.0)) <= 1e-10 && std::fabs(im) <= 1e-10)) {
            why = "op " + std::to_string(i) + ": Kraus set is not complete within 1e-10";
            return false;
          }
        }
    }
  }
  return true;
}

// Pauli masks of a rotation generator on qubit q
void rot_masks(const lrdm_op& o, uint64_t& xm, uint64_t& zm) {
  xm = (o.axis == 1 || o.axis == 2) ? (1ull << o.q0) : 0;
  zm = (o.axis == 2 || o.axis == 3) ? (1ull << o.q0) : 0;
}

// Does the generator P of rotation `rot` commute with operation o?  (Then the derivative of
// rot can be taken after o as well.)
bool commutes(const lrdm_program* p, const lrdm_op& o, const lrdm_op& rot, const double* params) {
  const int q = rot.q0;
  if (o.kind == LRDM_OP_WEIGHT) return rot.axis == 3;   // diagonal
  if (o.kind == LRDM_OP_ROTATION) return o.q0 != q || o.axis == rot.axis;
  if (o.kind != LRDM_OP_GATE) return false;
  const bool on_q = o.q0 == q || (o.k == 2 && o.q1 == q);
  if (!on_q) return true;
  const int d = 1 << o.k;
  const double* u = p->coef + o.off;
  bool diag = true;
  for (int a = 0; a < d; ++a)
    for (int b = 0; b < d; ++b)
      if (a != b && (u[2 * (a * d + b)] != 0.0 || u[2 * (a * d + b) + 1] != 0.0)) diag = false;
  if (o.k == 2) return diag && rot.axis == 3;
  // one-qubit gate on q: U P == P U within 1e-12
  double P[8];
  std::memset(P, 0, sizeof(P));
  if (rot.axis == 1) { P[2] = 1; P[4] = 1; }
  else if (rot.axis == 2) { P[3] = -1; P[5] = 1; }
  else { P[0] = 1; P[6] = -1; }
  (void)params;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      double d_re = 0, d_im = 0;
      for (int k = 0; k < 2; ++k) {
        const double ur = u[2 * (a * 2 + k)], ui = u[2 * (a * 2 + k) + 1];
        const double pr = P[2 * (k * 2 + b)], pi = P[2 * (k * 2 + b) + 1];
        const double qr = P[2 * (a * 2 + k)], qi = P[2 * (a * 2 + k) + 1];
        const double vr = u[2 * (k * 2 + b)], vi = u[2 * (k * 2 + b) + 1];
        d_re += (ur * pr - ui * pi) - (qr * vr - qi * vi);
        d_im += (ur * pi + ui * pr) - (qr * vi + qi * vr);
      }
      if (std::fabs(d_re) > 1e-12 || std::fabs(d_im) > 1e-12) return false;
    }
  return true;
}

// Undo one gate-like operation on both handles (U^H, or the conjugate phases).
lrdm_status unapply(lrdm_t h, lrdm_t bar, const lrdm_program* p, const lrdm_op& o, const double* params) {
  double tmp[8];
  double adj[32];
  if (o.kind == LRDM_OP_WEIGHT) {
    int nq = 0, ld = 0, rp = 0;
    size_t sb = 0;
    lrdm_status st = lrdm_layout(h, &nq, &ld, &rp, &sb);
    if (st != LRDM_OK) return st;
    std::vector<double> ph(2 * (size_t)(nq + 1));
    for (int w = 0; w <= nq; ++w) {
      ph[2 * w] = p->coef[o.off + 2 * w];
      ph[2 * w + 1] = -p->coef[o.off + 2 * w + 1];
    }
    st = lrdm_apply_diagonal_weight(h, ph.data());
    if (st != LRDM_OK) return st;
    return lrdm_apply_diagonal_weight(bar, ph.data());
  }
  const int k = o.kind == LRDM_OP_GATE ? o.k : 1;
  const int d = 1 << k;
  const double* u = op_matrix(p, o, params, tmp);
  for (int a = 0; a < d; ++a)
    for (int b = 0; b < d; ++b) {
      adj[2 * (a * d + b)] = u[2 * (b * d + a)];
      adj[2 * (a * d + b) + 1] = -u[2 * (b * d + a) + 1];
    }
  const int q[2] = {o.q0, o.q1};
  lrdm_status st = lrdm_apply_gate(h, k, q, adj);
  if (st != LRDM_OK) return st;
  return lrdm_apply_gate(bar, k, q, adj);
}

// Reverse a run of gate-like operations [b, e) on both handles, accumulating the derivatives of
// the rotations among them.  A rotation's derivative is Im Tr(Lbar^H P L) taken right after it;
// rotations whose generator commutes with every operation between them and the current point
// are evaluated together in one overlap call.
lrdm_status gates_backward(lrdm_t h, lrdm_t bar, const lrdm_program* p, int b, int e, const double* params,
                           double* grad) {
  std::vector<char> done(e - b, 0);
  int pos = e;
  std::vector<uint64_t> xm, zm;
  std::vector<int> batch;
  std::vector<double> ov;
  while (pos > b) {
    batch.clear();
    xm.clear();
    zm.clear();
    for (int i = pos - 1; i >= b; --i) {
      const lrdm_op& g = p->ops[i];
      if (g.kind == LRDM_OP_ROTATION && !done[i - b]) {
        bool ok = true;
        for (int j = i + 1; j < pos && ok; ++j) ok = commutes(p, p->ops[j], g, params);
        if (ok) {
          batch.push_back(i);
          uint64_t x, z;
          rot_masks(g, x, z);
          xm.push_back(x);
          zm.push_back(z);
        }
      }
    }
    if (!batch.empty()) {
      ov.assign(2 * batch.size(), 0.0);
      lrdm_status st = lrdm_pauli_overlap(bar, h, (int)batch.size(), xm.data(), zm.data(), ov.data());
      if (st != LRDM_OK) return st;
      for (size_t t = 0; t < batch.size(); ++t) {
        grad[p->ops[batch[t]].param] += ov[2 * t + 1];
        done[batch[t] - b] = 1;
      }
    }
    int nxt = b - 1;
    for (int i = pos - 1; i >= b; --i)
      if (p->ops[i].kind == LRDM_OP_ROTATION && !done[i - b]) {
        nxt = i;
        break;
      }
    for (int i = pos - 1; i > nxt; --i) {
      lrdm_status st = unapply(h, bar, p, p->ops[i], params);
      if (st != LRDM_OK) return st;
    }
    pos = nxt + 1;
  }
  return LRDM_OK;
}

}  // namespace

extern "C" {

lrdm_status lrdm_program_validate(const lrdm_program* p, int n, const double* params, int n_params) {
  if (n < 1 || n > 30) return pfail(LRDM_E_ARG, "n must be in [1, 30]");
  lrdm_status st = validate(p, n, params, n_params, false);
  if (st != LRDM_OK) return st;
  std::string why;
  if (!values_ok(p, n, params, why)) return pfail(LRDM_E_ARG, why);
  return LRDM_OK;
}

lrdm_status lrdm_run(lrdm_t h, const lrdm_program* p, const double* params, int n_params, void* ckpt_dev,
                     size_t ckpt_bytes, int* ckpt_rank) {
  Shape s;
  lrdm_status st = shape_of(h, s);
  if (st != LRDM_OK) return st;
  st = validate(p, s.n, params, n_params, false);
  if (st != LRDM_OK) return st;
  std::string why;
  if (!values_ok(p, s.n, params, why)) return pfail(LRDM_E_ARG, why);
  const auto segs = split_layers(p);
  if (ckpt_dev) {
    if ((reinterpret_cast<uintptr_t>(ckpt_dev) & 255) != 0) return pfail(LRDM_E_ARG, "checkpoint buffer must be 256-byte aligned");
    if (ckpt_bytes < segs.size() * align_up(s.state_bytes))
      return pfail(LRDM_E_NOMEM, "checkpoint buffer smaller than (layers) x (state bytes rounded up to 256)");
  }
  for (size_t l = 0; l < segs.size(); ++l) {
    if (ckpt_dev) {
      int rk = 0;
      st = lrdm_checkpoint(h, static_cast<char*>(ckpt_dev) + l * align_up(s.state_bytes), &rk);
      if (st != LRDM_OK) return st;
      if (ckpt_rank) ckpt_rank[l] = rk;
    }
    for (int i = segs[l].first; i < segs[l].second; ++i) {
      st = issue(h, p, p->ops[i], params, nullptr);
      if (st != LRDM_OK) return st;
    }
  }
  return LRDM_OK;
}

lrdm_status lrdm_run_switching(lrdm_t h, lrdm_fdm_t f, const lrdm_program* p, const double* params, int n_params,
                               int* switched_at) {
  Shape s;
  lrdm_status st = shape_of(h, s);
  if (st != LRDM_OK) return st;
  if (!switched_at) return pfail(LRDM_E_ARG, "null switched_at");
  st = validate(p, s.n, params, n_params, false);
  if (st != LRDM_OK) return st;
  std::string why;
  if (!values_ok(p, s.n, params, why)) return pfail(LRDM_E_ARG, why);
  if (s.n <= 16 && !f) return pfail(LRDM_E_ARG, "n <= 16 needs a full-rank handle for the switch");
  if (s.n <= 16)
    for (int i = 0; i < p->n_ops; ++i)
      if (p->ops[i].kind == LRDM_OP_KRAUS2)
        return pfail(LRDM_E_UNSUPPORTED, "op " + std::to_string(i) +
                                             ": two-qubit channels cannot follow a switch to full rank");
  *switched_at = -1;
  const double two_n = std::ldexp(1.0, s.n);
  // V: the column count of the factor as Algorithm 1 keeps it, min(r, A V, the kept rank); the
  // device's reported rank alone can be larger while zero eigenvalues pad its Gram order
  int V = 1, A_pend = 1;
  bool full = false;
  double tmp[8];
  for (int i = 0; i < p->n_ops; ++i) {
    const lrdm_op& o = p->ops[i];
    if (!full && (o.kind == LRDM_OP_KRAUS || o.kind == LRDM_OP_KRAUS2)) {
      const int M = o.kind == LRDM_OP_KRAUS ? 1 : 2;
      const double VI = std::cbrt((double)s.n / M) * o.k * V;   // V_I^3 = N (A V)^3 / M
      if (VI >= two_n) {
        st = lrdm_to_full(h, f);
        if (st != LRDM_OK) return st;
        full = true;
        *switched_at = i;
      }
    }
    if (full) {
      if (o.kind == LRDM_OP_GATE || o.kind == LRDM_OP_ROTATION) {
        const int q[2] = {o.q0, o.q1};
        st = lrdm_fdm_apply_gate(f, o.kind == LRDM_OP_GATE ? o.k : 1, q, op_matrix(p, o, params, tmp));
      } else if (o.kind == LRDM_OP_WEIGHT) {
        st = lrdm_fdm_apply_diagonal_weight(f, p->coef + o.off);
      } else if (o.kind == LRDM_OP_KRAUS) {
        st = lrdm_fdm_apply_kraus(f, o.q0, o.k, p->coef + o.off);
      }
      if (st != LRDM_OK) return st;
      continue;
    }
    if (o.kind == LRDM_OP_COMPRESS) {
      lrdm_compress_info info;
      st = lrdm_compress(h, o.r, o.eps, o.tie, o.renorm, &info);
      if (st != LRDM_OK) return st;
      V = std::min(std::min(info.rank, A_pend * V), o.r);
      continue;
    }
    if (o.kind == LRDM_OP_KRAUS || o.kind == LRDM_OP_KRAUS2) A_pend = o.k;
    st = issue(h, p, o, params, nullptr);
    if (st != LRDM_OK) return st;
  }
  return full ? lrdm_fdm_synchronize(f) : LRDM_OK;
}

lrdm_status lrdm_energy_grad_bytes(lrdm_t h, const lrdm_program* p, size_t* keep_all_bytes, size_t* min_bytes) {
  Shape s;
  lrdm_status st = shape_of(h, s);
  if (st != LRDM_OK) return st;
  if (!keep_all_bytes || !min_bytes) return pfail(LRDM_E_ARG, "null output pointer");
  st = validate(p, s.n, nullptr, 0, true);
  if (st != LRDM_OK) return st;
  size_t rb = 0;
  st = lrdm_record_bytes(h, &rb);
  if (st != LRDM_OK) return st;
  const auto segs = split_layers(p);
  int total = 0, most = 0;
  for (const auto& sg : segs) {
    int c = 0;
    for (int i = sg.first; i < sg.second; ++i) c += p->ops[i].kind == LRDM_OP_KRAUS;
    total += c;
    most = std::max(most, c);
  }
  const size_t sb = align_up(s.state_bytes), per = sb + align_up(rb);
  *keep_all_bytes = segs.size() * sb + (size_t)total * per;
  *min_bytes = segs.size() * sb + (size_t)most * per;
  return LRDM_OK;
}

lrdm_status lrdm_energy_grad(lrdm_t h, lrdm_t bar, const lrdm_program* p, const double* params, int n_params,
                             int n_terms, const uint64_t* xmask, const uint64_t* zmask, const double* coeff,
                             double* energy, double* grad_host, void* store_dev, size_t store_bytes,
                             int* kept_all) {
  Shape s;
  lrdm_status st = shape_of(h, s);
  if (st != LRDM_OK) return st;
  if (!bar || bar == h) return pfail(LRDM_E_ARG, "the adjoint needs a second, distinct handle");
  if (!energy || !grad_host || !store_dev) return pfail(LRDM_E_ARG, "null argument");
  if (n_params < 0) return pfail(LRDM_E_ARG, "n_params must be >= 0");
  if ((reinterpret_cast<uintptr_t>(store_dev) & 255) != 0) return pfail(LRDM_E_ARG, "store buffer must be 256-byte aligned");
  st = validate(p, s.n, params, n_params, true);
  if (st != LRDM_OK) return st;
  for (int i = 0; i < p->n_ops; ++i)
    if (p->ops[i].kind == LRDM_OP_ROTATION && p->ops[i].param >= n_params)
      return pfail(LRDM_E_ARG, "op " + std::to_string(i) + ": rotation parameter index beyond n_params");
  std::string why;
  if (!values_ok(p, s.n, params, why)) return pfail(LRDM_E_ARG, why);
  size_t all_b = 0, min_b = 0, rb = 0;
  st = lrdm_energy_grad_bytes(h, p, &all_b, &min_b);
  if (st != LRDM_OK) return st;
  st = lrdm_record_bytes(h, &rb);
  if (st != LRDM_OK) return st;
  if (store_bytes < min_b) return pfail(LRDM_E_NOMEM, "store buffer smaller than lrdm_energy_grad_bytes' minimum");
  const bool keep = store_bytes >= all_b;
  if (kept_all) *kept_all = keep ? 1 : 0;

  const auto segs = split_layers(p);
  const size_t sb = align_up(s.state_bytes), rbb = align_up(rb);
  std::vector<int> chans(segs.size(), 0);
  for (size_t l = 0; l < segs.size(); ++l)
    for (int i = segs[l].first; i < segs[l].second; ++i) chans[l] += p->ops[i].kind == LRDM_OP_KRAUS;
  int total = 0, most = 0;
  for (int c : chans) { total += c; most = std::max(most, c); }
  const int slots = keep ? total : most;
  char* base = static_cast<char*>(store_dev);
  char* ckpt = base;
  char* xbuf = ckpt + segs.size() * sb;
  char* recs = xbuf + (size_t)slots * sb;
  std::vector<int> ckrank(segs.size(), 0), xrank(std::max(slots, 1), 0), j0(segs.size(), 0);
  if (keep)
    for (size_t l = 1; l < segs.size(); ++l) j0[l] = j0[l - 1] + chans[l - 1];

  // one layer forward; with keep, every channel's input and its compression record go to the
  // channel slots from j
  auto run_layer = [&](size_t l, bool keep_inputs) -> lrdm_status {
    int j = j0[l];
    for (int i = segs[l].first; i < segs[l].second; ++i) {
      const lrdm_op& o = p->ops[i];
      lrdm_status r = LRDM_OK;
      if (o.kind == LRDM_OP_KRAUS && keep_inputs) {
        r = lrdm_checkpoint(h, xbuf + (size_t)j * sb, &xrank[j]);
        if (r != LRDM_OK) return r;
      }
      if (o.kind == LRDM_OP_COMPRESS) {
        r = issue(h, p, o, params, reinterpret_cast<double*>(recs + (size_t)j * rbb));
        ++j;
      } else {
        r = issue(h, p, o, params, nullptr);
      }
      if (r != LRDM_OK) return r;
    }
    return LRDM_OK;
  };

  // forward
  st = lrdm_reset(h);
  if (st != LRDM_OK) return st;
  for (size_t l = 0; l < segs.size(); ++l) {
    st = lrdm_checkpoint(h, ckpt + l * sb, &ckrank[l]);
    if (st != LRDM_OK) return st;
    st = run_layer(l, keep);
    if (st != LRDM_OK) return st;
  }
  st = lrdm_expect_pauli(h, n_terms, xmask, zmask, coeff, 1, energy);
  if (st != LRDM_OK) return st;

  // reverse sweep
  std::memset(grad_host, 0, sizeof(double) * (size_t)n_params);
  st = lrdm_apply_pauli_sum(bar, h, n_terms, xmask, zmask, coeff);
  if (st != LRDM_OK) return st;
  for (int l = (int)segs.size() - 1; l >= 0; --l) {
    if (keep) {
      // the layer's inputs and records are kept; its end state is the next layer's checkpoint
      if (l + 1 < (int)segs.size()) {
        st = lrdm_restore(h, ckpt + (size_t)(l + 1) * sb, ckrank[l + 1]);
        if (st != LRDM_OK) return st;
      }
    } else {
      st = lrdm_restore(h, ckpt + (size_t)l * sb, ckrank[l]);
      if (st != LRDM_OK) return st;
      st = run_layer((size_t)l, true);
      if (st != LRDM_OK) return st;
    }
    int j = j0[l] + chans[l];
    int i = segs[l].second;
    while (i > segs[l].first) {
      const lrdm_op& o = p->ops[i - 1];
      if (o.kind == LRDM_OP_COMPRESS) {
        const lrdm_op& kr = p->ops[i - 2];
        --j;
        st = lrdm_compress_adjoint(bar, xbuf + (size_t)j * sb, recs + (size_t)j * rbb, kr.q0, kr.k, p->coef + kr.off);
        if (st != LRDM_OK) return st;
        st = lrdm_restore(h, xbuf + (size_t)j * sb, xrank[j]);
        if (st != LRDM_OK) return st;
        i -= 2;
        continue;
      }
      int k = i;
      while (k > segs[l].first && p->ops[k - 1].kind != LRDM_OP_COMPRESS && p->ops[k - 1].kind != LRDM_OP_KRAUS) --k;
      st = gates_backward(h, bar, p, k, i, params, grad_host);
      if (st != LRDM_OK) return st;
      i = k;
    }
  }
  return lrdm_synchronize(bar);
}

lrdm_status lrdm_batch_run(lrdm_batch_t b, const lrdm_program* const* progs, const double* const* params,
                           const int* n_params, void* plan_dev, size_t plan_bytes, size_t* plan_needed,
                           double* done_ms, double* total_ms) {
  if (!b || !progs || !plan_needed) return pfail(LRDM_E_ARG, "null argument");
  int n_inst = 0;
  const lrdm_t* handles = lrdm::batch_handles(b, &n_inst);
  for (int i = 0; i < n_inst; ++i) {
    Shape s;
    lrdm_status st = shape_of(handles[i], s);
    if (st != LRDM_OK) return st;
    st = validate(progs[i], s.n, params ? params[i] : nullptr, n_params ? n_params[i] : 0, false);
    if (st != LRDM_OK) return st;
    std::string why;
    if (!values_ok(progs[i], s.n, params ? params[i] : nullptr, why))
      return pfail(LRDM_E_ARG, "instance " + std::to_string(i) + ": " + why);
  }
  lrdm_status st = lrdm_batch_begin(b);
  if (st != LRDM_OK) return st;
  for (int i = 0; i < n_inst && st == LRDM_OK; ++i) {
    st = lrdm_reset(handles[i]);
    for (int o = 0; o < progs[i]->n_ops && st == LRDM_OK; ++o)
      st = issue(handles[i], progs[i], progs[i]->ops[o], params ? params[i] : nullptr, nullptr);
  }
  size_t need = 0;
  const lrdm_status st_end = lrdm_batch_end(b, &need);
  if (st != LRDM_OK) return st;
  if (st_end != LRDM_OK) return st_end;
  *plan_needed = need;
  if (!plan_dev || plan_bytes < need) return pfail(LRDM_E_NOMEM, "plan buffer smaller than *plan_needed");
  st = lrdm_batch_instantiate(b, plan_dev, plan_bytes);
  if (st != LRDM_OK) return st;
  st = lrdm_batch_launch(b);
  if (st != LRDM_OK) return st;
  return lrdm_batch_times(b, done_ms, total_ms);
}

}  // extern "C"
