// CPU check of the full-rank comparator's host scheduler (operator fusion, pass building,
// register phases).  The runtime source is compiled with its device launches replaced by an
// interpreter of the pass descriptors: every operation of a pass is applied to the whole state
// in plain loops, with its operands decoded the way the pass kernels decode them (tile slots,
// register indices of a phase, register-tagged diagonal operands).  Structural rules of the
// descriptors are counted as violations.
//
//   check <program.txt> <out.bin>
// program.txt: "n" then lines "G k q0 [q1] <2 * d * d doubles>" (gate, row-major, interleaved
// complex) or "K q m <8 * m doubles>" (Kraus set).  out.bin: the final state (complex64, 4^n).
#include "runtime_fdm.cpp"

#include <complex>
#include <cstdio>

namespace lrdm {
void set_last_error(const char* m) { std::fprintf(stderr, "error: %s\n", m); }

static std::vector<std::complex<float>> g_state;
static int g_passes = 0, g_phases = 0, g_violations = 0;

static void apply(int nbits, int ty, int a, int b, const float* u) {
  auto& v = g_state;
  const size_t N = (size_t)1 << nbits;
  auto C = [&](int i) { return std::complex<float>(u[2 * i], u[2 * i + 1]); };
  if (ty == OP_DIAG1 || ty == OP_DIAG2) {
    for (size_t i = 0; i < N; ++i) {
      int sel = (i >> a) & 1;
      if (ty == OP_DIAG2) sel |= ((i >> b) & 1) << 1;
      v[i] *= C(sel);
    }
  } else if (ty == OP_1Q) {
    for (size_t i = 0; i < N; ++i)
      if (!((i >> a) & 1)) {
        const auto x0 = v[i], x1 = v[i | (1ull << a)];
        v[i] = C(0) * x0 + C(1) * x1;
        v[i | (1ull << a)] = C(2) * x0 + C(3) * x1;
      }
  } else {
    for (size_t i = 0; i < N; ++i)
      if (!((i >> a) & 1) && !((i >> b) & 1)) {
        const size_t idx[4] = {i, i | (1ull << a), i | (1ull << b), i | (1ull << a) | (1ull << b)};
        std::complex<float> x[4], y[4];
        for (int m = 0; m < 4; ++m) x[m] = v[idx[m]];
        for (int r = 0; r < 4; ++r) {
          y[r] = 0;
          for (int m = 0; m < 4; ++m) y[r] += C(4 * r + m) * x[m];
        }
        for (int r = 0; r < 4; ++r) v[idx[r]] = y[r];
      }
  }
}

hipError_t launch_fdm_pass(const FdmPass& p, float2*, hipStream_t) {
  ++g_passes;
  if (p.n_ops > kFdmMaxOps || p.k > kFdmMaxLocal) ++g_violations;
  if (p.n_phases == 0) {
    for (int o = 0; o < p.n_ops; ++o) {
      const int ty = p.op_type[o];
      int a = p.op_a[o], b = p.op_b[o];
      if (ty == OP_1Q || ty == OP_2Q) {
        if (a >= p.k || (ty == OP_2Q && (b >= p.k || b == a))) ++g_violations;
        a = p.local_q[a];
        b = p.local_q[b];
      }
      apply(p.nbits, ty, a, b, p.coef + p.op_coef[o]);
    }
    return hipSuccess;
  }
  // register phases: full tiles, 4 distinct slots per phase, the phases cover the ops in order
  g_phases += p.n_phases;
  if (p.k != kFdmMaxLocal) ++g_violations;
  int next = 0;
  for (int ph = 0; ph < p.n_phases; ++ph) {
    if (p.ph_first[ph] != next) ++g_violations;
    next += p.ph_count[ph];
    for (int r = 0; r < 4; ++r) {
      if (p.ph_slots[ph][r] >= p.k) ++g_violations;
      for (int s = r + 1; s < 4; ++s)
        if (p.ph_slots[ph][r] == p.ph_slots[ph][s]) ++g_violations;
    }
    auto bit_of_reg = [&](int r) { return p.local_q[p.ph_slots[ph][r]]; };
    for (int o = p.ph_first[ph]; o < p.ph_first[ph] + p.ph_count[ph]; ++o) {
      const int ty = p.op_type[o];
      int a = p.op_a[o], b = p.op_b[o];
      if (ty == OP_1Q || ty == OP_2Q) {
        // register operands 0..3, ascending for a 2-bit operator
        if (a < 0 || a > 3 || (ty == OP_2Q && (b <= a || b > 3))) ++g_violations;
        a = bit_of_reg(a & 3);
        b = bit_of_reg(b & 3);
      } else {
        // 64 + r: register r; register operands first and ascending
        if (ty == OP_DIAG2 && b >= 64 && (a < 64 || b <= a)) ++g_violations;
        if (a >= 64) a = bit_of_reg((a - 64) & 3);
        if (ty == OP_DIAG2 && b >= 64) b = bit_of_reg((b - 64) & 3);
      }
      apply(p.nbits, ty, a, b, p.coef + p.op_coef[o]);
    }
  }
  if (next != p.n_ops) ++g_violations;
  return hipSuccess;
}

hipError_t launch_fdm_reset(float2*, int n, hipStream_t) {
  g_state.assign((size_t)1 << (2 * n), 0.f);
  g_state[0] = 1.f;
  return hipSuccess;
}

hipError_t launch_fdm_diag(const float2*, int, double*, hipStream_t) { return hipSuccess; }

// rho[x][y] *= phase[pop(x)] conj(phase[pop(y)]), row bits above the column bits
hipError_t launch_fdm_weight(float2*, int n, const FdmPhase& ph, hipStream_t) {
  const size_t dim = size_t(1) << n;
  for (size_t x = 0; x < dim; ++x)
    for (size_t y = 0; y < dim; ++y) {
      const int a = __builtin_popcountll(x), b = __builtin_popcountll(y);
      const std::complex<double> w = std::complex<double>(ph.ph[2 * a], ph.ph[2 * a + 1]) *
                                     std::conj(std::complex<double>(ph.ph[2 * b], ph.ph[2 * b + 1]));
      std::complex<float>& v = g_state[(x << n) | y];
      v = std::complex<float>(std::complex<double>(v) * w);
    }
  return hipSuccess;
}
}  // namespace lrdm

int main(int argc, char** argv) {
  if (argc != 3) return 2;
  FILE* f = std::fopen(argv[1], "r");
  if (!f) return 2;
  int n = 0;
  if (std::fscanf(f, "%d", &n) != 1) return 2;
  static float2 placeholder[1] __attribute__((aligned(256)));
  lrdm_fdm_t h;
  if (lrdm_fdm_init(&h, n, placeholder, (size_t)8 << (2 * n), nullptr) != LRDM_OK) return 3;
  char t[4];
  while (std::fscanf(f, "%3s", t) == 1) {
    if (t[0] == 'G') {
      int k, q[2] = {0, 0};
      if (std::fscanf(f, "%d", &k) != 1 || k < 1 || k > 2) return 4;
      for (int j = 0; j < k; ++j) if (std::fscanf(f, "%d", &q[j]) != 1) return 4;
      std::vector<double> u(2 << (2 * k));
      for (auto& x : u) if (std::fscanf(f, "%lf", &x) != 1) return 4;
      if (lrdm_fdm_apply_gate(h, k, q, u.data()) != LRDM_OK) return 5;
    } else if (t[0] == 'W') {
      std::vector<double> ph(2 * (n + 1));
      for (auto& x : ph) if (std::fscanf(f, "%lf", &x) != 1) return 4;
      if (lrdm_fdm_apply_diagonal_weight(h, ph.data()) != LRDM_OK) return 5;
    } else {
      int q, m;
      if (std::fscanf(f, "%d %d", &q, &m) != 2 || m < 1 || m > 4) return 4;
      std::vector<double> e(8 * m);
      for (auto& x : e) if (std::fscanf(f, "%lf", &x) != 1) return 4;
      if (lrdm_fdm_apply_kraus(h, q, m, e.data()) != LRDM_OK) return 5;
    }
  }
  std::fclose(f);
  if (flush(h) != LRDM_OK) return 6;
  FILE* o = std::fopen(argv[2], "wb");
  if (!o) return 2;
  std::fwrite(lrdm::g_state.data(), 8, lrdm::g_state.size(), o);
  std::fclose(o);
  std::printf("passes %d phases %d violations %d\n", lrdm::g_passes, lrdm::g_phases, lrdm::g_violations);
  lrdm_fdm_destroy(h);
  return lrdm::g_violations ? 7 : 0;
}
