// Drives the host runtime of liblrdm (built with the launcher and HIP stubs of stubs.cpp) through
// every entry point over a sweep of shapes: workspace sizing and carving, gate passes, fused and
// plain compressions (chained ones included), outputs, records, the reverse-sweep calls, the
// program-level calls, the full-rank comparator and a batch, plus the argument checks.  Exit
// status 0 when no kernel region fell outside its buffer; the sanitizers abort on any host-side
// error of their own.
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "lrdm.h"

namespace hs {
void reg(const void* p, size_t n);
void unreg(const void* p);
extern long violations, launches;
}  // namespace hs

static long failures = 0;
#define EXPECT(cond)                                                              \
  do {                                                                            \
    if (!(cond)) {                                                                \
      ++failures;                                                                 \
      std::fprintf(stderr, "%s:%d: expected %s (%s)\n", __FILE__, __LINE__, #cond, \
                   lrdm_last_error(nullptr));                                     \
    }                                                                             \
  } while (0)

struct DevBuf {
  void* p = nullptr;
  size_t n = 0;
  explicit DevBuf(size_t bytes) : n(bytes) {
    p = std::aligned_alloc(256, (bytes + 255) / 256 * 256);
    std::memset(p, 0, (bytes + 255) / 256 * 256);
    hs::reg(p, bytes);
  }
  ~DevBuf() {
    hs::unreg(p);
    std::free(p);
  }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
};

using cd = std::complex<double>;

static void mat_h(double* u) {   // Hadamard
  const double s = 1.0 / std::sqrt(2.0);
  const double m[8] = {s, 0, s, 0, s, 0, -s, 0};
  std::memcpy(u, m, sizeof(m));
}
static void kraus_ad(double g, double* e) {   // amplitude damping
  std::memset(e, 0, 16 * sizeof(double));
  e[0] = 1;
  e[6] = std::sqrt(1 - g);
  e[8 + 2] = std::sqrt(g);
}
static void kraus_deph(double p, double* e) {
  std::memset(e, 0, 16 * sizeof(double));
  e[0] = std::sqrt(1 - p);
  e[6] = std::sqrt(1 - p);
  e[8] = std::sqrt(p);
  e[14] = -std::sqrt(p);
}
static void kraus_dep(double p, double* e) {
  std::memset(e, 0, 32 * sizeof(double));
  const double a = std::sqrt(1 - p), b = std::sqrt(p / 3);
  e[0] = a; e[6] = a;                    // I
  e[8 + 2] = b; e[8 + 4] = b;            // X
  e[16 + 3] = -b; e[16 + 5] = b;         // Y = [[0, -i], [i, 0]]
  e[24 + 0] = b; e[24 + 6] = -b;         // Z
}

// a channel of at most m_max operators: amplitude damping / dephasing (two), or for m_max = 1 the
// one-operator channel Z (a unitary)
static int chan2(int m_max, bool ad, double p, double* e) {
  if (m_max >= 2) {
    if (ad) kraus_ad(p, e);
    else kraus_deph(p, e);
    return 2;
  }
  std::memset(e, 0, 8 * sizeof(double));
  e[0] = 1;
  e[6] = -1;
  return 1;
}

static void exercise(int n, int r, lrdm_dtype dt, int m_max, unsigned flags) {
  size_t sb = 0, wb = 0;
  if (lrdm_workspace_size(n, r, dt, m_max, flags, &sb, &wb) != LRDM_OK) return;
  DevBuf state(sb), work(wb);
  lrdm_t h = nullptr;
  EXPECT(lrdm_init(&h, n, r, dt, m_max, flags, state.p, sb, work.p, wb, nullptr) == LRDM_OK);
  if (!h) return;
  int nn = 0, ld = 0, rp = 0;
  size_t sbb = 0;
  EXPECT(lrdm_layout(h, &nn, &ld, &rp, &sbb) == LRDM_OK && sbb == sb && nn == n);
  // launch shapes: defaults resolved, a value out of range refused, odd shapes taken
  lrdm_tuning tu{};
  EXPECT(lrdm_get_tuning(h, &tu) == LRDM_OK && tu.gram_blocks >= 1 && tu.gate_local_max >= 1);
  lrdm_tuning bad_t{};
  bad_t.gram_blocks = 300;
  EXPECT(lrdm_set_tuning(h, &bad_t) == LRDM_E_ARG);
  bad_t = lrdm_tuning{};
  bad_t.aux_cus = 48;
  EXPECT(lrdm_set_tuning(h, &bad_t) == LRDM_E_ARG);
  lrdm_tuning odd{};
  odd.gram_blocks = 7;
  odd.gate_local_max = 3;
  if (flags & LRDM_FLAG_OVERLAP) {
    odd.gram4_blocks = 5;
    odd.aux_cus = 64;
  }
  EXPECT(lrdm_set_tuning(h, &odd) == LRDM_OK);
  double u[32], e[32], ph[2 * 31];
  mat_h(u);
  for (int q = 0; q < n; ++q) {
    const int qq[1] = {q};
    EXPECT(lrdm_apply_gate(h, 1, qq, u) == LRDM_OK);
  }
  if (n >= 2) {
    double cz[32] = {0};
    cz[0] = 1; cz[10] = 1; cz[20] = 1; cz[30] = -1;
    const int q2[2] = {0, n - 1};
    EXPECT(lrdm_apply_gate(h, 2, q2, cz) == LRDM_OK);
  }
  for (int w = 0; w <= n; ++w) { ph[2 * w] = std::cos(0.3 * w); ph[2 * w + 1] = std::sin(0.3 * w); }
  EXPECT(lrdm_apply_diagonal_weight(h, ph) == LRDM_OK);
  const int rt = r;
  for (int q = 0; q < n; ++q) {
    int m = chan2(m_max, true, 0.01, e);
    EXPECT(lrdm_apply_kraus(h, q, m, e) == LRDM_OK);
    lrdm_compress_info info;
    EXPECT(lrdm_compress(h, rt, 0.0, 0, 1, q == 0 ? &info : nullptr) == LRDM_OK);
    m = chan2(m_max, false, 0.01, e);
    EXPECT(lrdm_apply_kraus(h, q, m, e) == LRDM_OK);           // chained on the same qubit
    EXPECT(lrdm_compress(h, rt, 1e-4, 1, 1, nullptr) == LRDM_OK);
    if (m_max >= 4) {
      kraus_dep(0.01, e);
      EXPECT(lrdm_apply_kraus(h, q, 4, e) == LRDM_OK);
      EXPECT(lrdm_compress(h, rt, 0.0, 0, 0, nullptr) == LRDM_OK);
    }
  }
  DevBuf prob((size_t)8 << n);
  EXPECT(lrdm_probabilities(h, static_cast<double*>(prob.p)) == LRDM_OK);
  std::vector<double> z(n), zz(n), tr(1);
  EXPECT(lrdm_expect_z(h, z.data(), zz.data(), tr.data()) == LRDM_OK);
  std::vector<uint64_t> xm = {1, 0, n >= 2 ? 3ull : 1ull}, zm = {0, 1ull << (n - 1), 1};
  std::vector<double> co = {0.5, -0.25, 1.0}, ev(3);
  EXPECT(lrdm_expect_pauli(h, 3, xm.data(), zm.data(), co.data(), 0, ev.data()) == LRDM_OK);
  EXPECT(lrdm_expect_pauli(h, 3, xm.data(), zm.data(), co.data(), 1, ev.data()) == LRDM_OK);
  std::vector<double> un(100);
  for (int i = 0; i < 100; ++i) un[i] = i / 100.0;
  std::vector<uint64_t> smp(100);
  EXPECT(lrdm_sample(h, 100, un.data(), smp.data()) == LRDM_OK);
  std::vector<char> host(sb);
  int rk = 0;
  EXPECT(lrdm_get_L(h, host.data(), 1, &rk) == LRDM_OK);
  EXPECT(lrdm_set_L(h, host.data(), 1, rp) == LRDM_OK);
  DevBuf ck(sb);
  EXPECT(lrdm_checkpoint(h, ck.p, &rk) == LRDM_OK);
  EXPECT(lrdm_restore(h, ck.p, rk) == LRDM_OK);
  for (int cls = 0; cls <= 5; ++cls) {
    EXPECT(lrdm_timing_begin(h, cls) == LRDM_OK);
    const int m = chan2(m_max, true, 0.02, e);
    EXPECT(lrdm_apply_kraus(h, 0, m, e) == LRDM_OK);
    EXPECT(lrdm_compress(h, rt, 0.0, 0, 1, nullptr) == LRDM_OK);
    int nl = 0;
    double mean = 0, tot = 0;
    EXPECT(lrdm_timing_end(h, &nl, &mean, &tot) == LRDM_OK);
  }
  // reverse-sweep calls where the record fits
  size_t rb = 0;
  if (lrdm_record_bytes(h, &rb) == LRDM_OK) {
    lrdm_t bar = nullptr;
    DevBuf s2(sb), w2(wb), rec(rb);
    EXPECT(lrdm_init(&bar, n, r, dt, m_max, flags, s2.p, sb, w2.p, wb, nullptr) == LRDM_OK);
    EXPECT(lrdm_checkpoint(h, ck.p, &rk) == LRDM_OK);
    const int mr = chan2(m_max, true, 0.05, e);
    EXPECT(lrdm_apply_kraus(h, n - 1, mr, e) == LRDM_OK);
    EXPECT(lrdm_compress_record(h, rt, 0.0, 0, 1, rec.p, nullptr) == LRDM_OK);
    EXPECT(lrdm_apply_pauli_sum(bar, h, 3, xm.data(), zm.data(), co.data()) == LRDM_OK);
    std::vector<double> ov(6);
    EXPECT(lrdm_pauli_overlap(bar, h, 3, xm.data(), zm.data(), ov.data()) == LRDM_OK);
    EXPECT(lrdm_compress_adjoint(bar, ck.p, rec.p, n - 1, mr, e) == LRDM_OK);
    // program level: a small parametrised program, energy and gradient in both memory modes
    std::vector<lrdm_op> ops;
    std::vector<double> coef;
    auto put = [&](const double* a, int cnt) {
      const int64_t off = (int64_t)coef.size();
      coef.insert(coef.end(), a, a + cnt);
      return off;
    };
    for (int l = 0; l < 2; ++l) {
      for (int q = 0; q < n; ++q) {
        lrdm_op o{};
        o.kind = LRDM_OP_ROTATION;
        o.k = 1;
        o.q0 = q;
        o.axis = 1 + (q % 3);
        o.param = l * n + q;
        o.off = 0;
        ops.push_back(o);
      }
      for (int q = 0; q < n; ++q) {
        lrdm_op o{};
        o.kind = LRDM_OP_KRAUS;
        o.q0 = q;
        o.k = chan2(m_max, true, 0.02, e);
        o.off = put(e, 8 * o.k);
        ops.push_back(o);
        lrdm_op c{};
        c.kind = LRDM_OP_COMPRESS;
        c.r = rt;
        c.renorm = 1;
        ops.push_back(c);
      }
      lrdm_op m{};
      m.kind = LRDM_OP_LAYER;
      ops.push_back(m);
    }
    std::vector<double> theta(2 * n);
    for (int i = 0; i < 2 * n; ++i) theta[i] = 0.1 * i;
    lrdm_program p{(int)ops.size(), ops.data(), coef.data(), (int64_t)coef.size()};
    EXPECT(lrdm_program_validate(&p, n, theta.data(), 2 * n) == LRDM_OK);
    DevBuf cks(2 * ((sb + 255) / 256 * 256));
    int ranks[2];
    EXPECT(lrdm_reset(h) == LRDM_OK);
    EXPECT(lrdm_run(h, &p, theta.data(), 2 * n, cks.p, cks.n, ranks) == LRDM_OK);
    EXPECT(lrdm_run(h, &p, theta.data(), 2 * n, cks.p, cks.n - 1, ranks) == LRDM_E_NOMEM);
    size_t keep = 0, mn = 0;
    EXPECT(lrdm_energy_grad_bytes(h, &p, &keep, &mn) == LRDM_OK);
    for (size_t bytes : {keep, mn}) {
      DevBuf store(bytes);
      double E = 0;
      std::vector<double> g(2 * n);
      int kept = -1;
      EXPECT(lrdm_energy_grad(h, bar, &p, theta.data(), 2 * n, 3, xm.data(), zm.data(), co.data(), &E, g.data(),
                              store.p, bytes, &kept) == LRDM_OK);
      EXPECT(kept == (bytes == keep ? 1 : 0));
    }
    lrdm_destroy(bar);
  }
  // sparse initial state, two-qubit channel (plain form), conversion to full rank
  {
    const uint64_t sidx[2] = {0, (1ull << n) - 1};
    const double samp[4] = {std::sqrt(0.5), 0, 0, std::sqrt(0.5)};
    EXPECT(lrdm_set_sparse(h, n >= 1 && sidx[1] != 0 ? 2 : 1, sidx, samp) == (sidx[1] != 0 ? LRDM_OK : LRDM_E_ARG));
    if (n >= 2) {   // a channel on a qubit pair: plain form, or fused (r_pad <= 32)
      std::vector<double> e2(32 * m_max, 0.0);
      const double w = 1.0 / std::sqrt((double)m_max);
      for (int a = 0; a < m_max; ++a)
        for (int i = 0; i < 4; ++i) e2[32 * a + 2 * (4 * i + i)] = w;
      const lrdm_status want = ((flags & LRDM_FLAG_PLAIN) || rp <= 32) ? LRDM_OK : LRDM_E_UNSUPPORTED;
      EXPECT(lrdm_apply_kraus2(h, n - 1, 0, m_max, e2.data()) == want);
      if (want == LRDM_OK) EXPECT(lrdm_compress(h, rt, 0.0, 0, 1, nullptr) == LRDM_OK);
    }
    if (n <= 8) {
      size_t fb = 0;
      EXPECT(lrdm_fdm_state_bytes(n, &fb) == LRDM_OK);
      DevBuf rho(fb);
      lrdm_fdm_t f = nullptr;
      EXPECT(lrdm_fdm_init(&f, n, rho.p, fb, nullptr) == LRDM_OK);
      EXPECT(lrdm_to_full(h, f) == LRDM_OK);
      lrdm_fdm_destroy(f);
    }
  }
  // argument checks
  const int bad[1] = {n};
  EXPECT(lrdm_apply_gate(h, 1, bad, u) == LRDM_E_ARG);
  EXPECT(lrdm_compress(h, r + 1, 0.0, 0, 1, nullptr) == LRDM_E_ARG);
  EXPECT(lrdm_compress(h, 1, 1.0, 0, 1, nullptr) == LRDM_E_ARG);
  EXPECT(lrdm_sample(h, 0, un.data(), smp.data()) == LRDM_E_ARG);
  EXPECT(lrdm_set_L(h, host.data(), 1, rp + 1) == LRDM_E_ARG);
  EXPECT(lrdm_timing_begin(h, 7) == LRDM_E_ARG);
  lrdm_destroy(h);
}

static void exercise_fdm(int n) {
  size_t b = 0;
  EXPECT(lrdm_fdm_state_bytes(n, &b) == LRDM_OK);
  DevBuf rho(b);
  lrdm_fdm_t f = nullptr;
  EXPECT(lrdm_fdm_init(&f, n, rho.p, b, nullptr) == LRDM_OK);
  double u[8], e[32], ph[2 * 17];
  mat_h(u);
  for (int q = 0; q < n; ++q) {
    const int qq[1] = {q};
    EXPECT(lrdm_fdm_apply_gate(f, 1, qq, u) == LRDM_OK);
    kraus_dep(0.01, e);
    EXPECT(lrdm_fdm_apply_kraus(f, q, 4, e) == LRDM_OK);
  }
  for (int w = 0; w <= n; ++w) { ph[2 * w] = 1; ph[2 * w + 1] = 0; }
  EXPECT(lrdm_fdm_apply_diagonal_weight(f, ph) == LRDM_OK);
  DevBuf p((size_t)8 << n);
  EXPECT(lrdm_fdm_probabilities(f, static_cast<double*>(p.p)) == LRDM_OK);
  EXPECT(lrdm_fdm_synchronize(f) == LRDM_OK);
  lrdm_fdm_destroy(f);
}

static void exercise_batch() {
  const int shapes[3][2] = {{6, 8}, {8, 16}, {7, 32}};
  std::vector<DevBuf*> bufs;
  std::vector<lrdm_t> hs_;
  for (auto& s : shapes) {
    size_t sb = 0, wb = 0;
    EXPECT(lrdm_workspace_size(s[0], s[1], LRDM_C64, 4, 0, &sb, &wb) == LRDM_OK);
    bufs.push_back(new DevBuf(sb));
    bufs.push_back(new DevBuf(wb));
    lrdm_t h = nullptr;
    EXPECT(lrdm_init(&h, s[0], s[1], LRDM_C64, 4, 0, bufs[bufs.size() - 2]->p, sb, bufs.back()->p, wb, nullptr) ==
           LRDM_OK);
    hs_.push_back(h);
  }
  lrdm_batch_t b = nullptr;
  EXPECT(lrdm_batch_create(&b, 3, hs_.data(), nullptr) == LRDM_OK);
  std::vector<lrdm_op> ops;
  std::vector<double> coef(8 + 32);
  mat_h(coef.data());
  kraus_dep(0.01, coef.data() + 8);
  for (int l = 0; l < 2; ++l)
    for (int q = 0; q < 6; ++q) {
      lrdm_op g{};
      g.kind = LRDM_OP_GATE;
      g.k = 1;
      g.q0 = q;
      g.off = 0;
      ops.push_back(g);
      lrdm_op k{};
      k.kind = LRDM_OP_KRAUS;
      k.k = 4;
      k.q0 = q;
      k.off = 8;
      ops.push_back(k);
      lrdm_op c{};
      c.kind = LRDM_OP_COMPRESS;
      c.r = 8;
      c.renorm = 1;
      ops.push_back(c);
    }
  lrdm_program p{(int)ops.size(), ops.data(), coef.data(), (int64_t)coef.size()};
  const lrdm_program* progs[3] = {&p, &p, &p};
  size_t need = 0;
  EXPECT(lrdm_batch_run(b, progs, nullptr, nullptr, nullptr, 0, &need, nullptr, nullptr) == LRDM_E_NOMEM);
  EXPECT(need > 0);
  DevBuf plan(need);
  std::vector<double> done(3);
  double total = 0;
  EXPECT(lrdm_batch_run(b, progs, nullptr, nullptr, plan.p, need, &need, done.data(), &total) == LRDM_OK);
  EXPECT(lrdm_batch_launch(b) == LRDM_OK);
  int steps = 0, nl = 0;
  EXPECT(lrdm_batch_info(b, &steps, &nl) == LRDM_OK && steps > 0);
  lrdm_batch_destroy(b);
  for (lrdm_t h : hs_) lrdm_destroy(h);
  for (DevBuf* d : bufs) delete d;
}

int main() {
  // sizing and carving over a sweep of shapes, then the full exercise on small n
  for (int n = 1; n <= 12; n += (n < 4 ? 1 : 4))
    for (int r : {1, 3, 8, 13, 16, 24, 32, 40, 64})
      for (int m : {1, 2, 4})
        for (lrdm_dtype dt : {LRDM_C64, LRDM_C128})
          for (unsigned fl : {0u, LRDM_FLAG_PLAIN, LRDM_FLAG_OVERLAP}) exercise(n, r, dt, m, fl);
  for (int n : {1, 2, 3, 5, 7}) exercise_fdm(n);
  exercise_batch();
  // entry points with no handle
  size_t a = 0, b = 0;
  EXPECT(lrdm_workspace_size(0, 8, LRDM_C64, 2, 0, &a, &b) == LRDM_E_ARG);
  EXPECT(lrdm_workspace_size(10, 64, LRDM_C64, 4, 0, &a, &b) == LRDM_E_UNSUPPORTED);
  EXPECT(lrdm_compress(nullptr, 1, 0.0, 0, 1, nullptr) == LRDM_E_ARG);
  EXPECT(lrdm_program_validate(nullptr, 4, nullptr, 0) == LRDM_E_ARG);
  std::printf("launch checks %ld, regions outside their buffers %ld, failed expectations %ld\n", hs::launches,
              hs::violations, failures);
  return (hs::violations || failures) ? 1 : 0;
}
