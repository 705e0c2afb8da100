// Host-only build of the liblrdm runtime for sanitizer runs on the CPU: the HIP runtime calls
// the runtime makes act on host memory standing in for device memory, and every kernel launcher
// is replaced by a check that each buffer the kernel would read or write lies inside one
// registered allocation (the caller's state, workspace, record, checkpoint and plan buffers).
// No arithmetic of the method runs here; the point is the host code: argument validation,
// workspace carving, pass building and the program and batch drivers, under AddressSanitizer
// and UndefinedBehaviorSanitizer.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "lrdm_internal.h"

namespace hs {
struct Buf {
  const char* p;
  size_t n;
};
std::vector<Buf> bufs;
long violations = 0, launches = 0;

void reg(const void* p, size_t n) { bufs.push_back({static_cast<const char*>(p), n}); }
void unreg(const void* p) {
  for (size_t i = 0; i < bufs.size(); ++i)
    if (bufs[i].p == p) {
      bufs.erase(bufs.begin() + i);
      return;
    }
}
// the region [p, p + n) must lie inside one registered buffer; its first and last bytes are read
// (an out-of-bounds host access is then AddressSanitizer's to report)
void touch(const void* p, size_t n, const char* what) {
  if (n == 0) return;
  const char* c = static_cast<const char*>(p);
  for (const Buf& b : bufs)
    if (c >= b.p && c + n <= b.p + b.n) {
      volatile char x = c[0];
      volatile char y = c[n - 1];
      (void)x;
      (void)y;
      return;
    }
  ++violations;
  std::fprintf(stderr, "region outside every buffer: %s (%p, %zu bytes)\n", what, p, n);
}
}  // namespace hs

using hs::touch;

// ------------------------------------------------------------------ HIP runtime on host memory
extern "C" {
hipError_t hipMemsetAsync(void* dst, int v, size_t n, hipStream_t) {
  touch(dst, n, "memset");
  std::memset(dst, v, n);
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t n, hipMemcpyKind, hipStream_t) {
  std::memmove(dst, src, n);
  return hipSuccess;
}
hipError_t hipMemcpy(void* dst, const void* src, size_t n, hipMemcpyKind) {
  std::memmove(dst, src, n);
  return hipSuccess;
}
hipError_t hipMemcpy2DAsync(void* dst, size_t dp, const void* src, size_t sp, size_t w, size_t h, hipMemcpyKind,
                            hipStream_t) {
  for (size_t r = 0; r < h; ++r)
    std::memmove(static_cast<char*>(dst) + r * dp, static_cast<const char*>(src) + r * sp, w);
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) {
  *s = reinterpret_cast<hipStream_t>(new char[8]);
  return hipSuccess;
}
hipError_t hipExtStreamCreateWithCUMask(hipStream_t* s, uint32_t words, const uint32_t* mask) {
  if (words == 0 || !mask) return hipErrorInvalidValue;
  volatile uint32_t last = mask[words - 1];   // the mask array is read whole
  (void)last;
  return hipStreamCreateWithFlags(s, 0);
}
hipError_t hipStreamDestroy(hipStream_t s) {
  delete[] reinterpret_cast<char*>(s);
  return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }
hipError_t hipEventCreate(hipEvent_t* e) {
  *e = reinterpret_cast<hipEvent_t>(new char[8]);
  return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e) {
  delete[] reinterpret_cast<char*>(e);
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) {
  *ms = 0.f;
  return hipSuccess;
}
const char* hipGetErrorString(hipError_t) { return "host stub"; }
hipError_t hipGetLastError(void) { return hipSuccess; }
hipError_t hipGetDevice(int* d) {
  *d = 0;
  return hipSuccess;
}
hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t, int) {
  *v = 100000;
  return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) { return hipSuccess; }
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t* g) {
  *g = reinterpret_cast<hipGraph_t>(new char[8]);
  return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t, hipGraphNode_t*, char*, size_t) {
  *e = reinterpret_cast<hipGraphExec_t>(new char[8]);
  return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return hipSuccess; }
hipError_t hipGraphDestroy(hipGraph_t g) {
  delete[] reinterpret_cast<char*>(g);
  return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t e) {
  delete[] reinterpret_cast<char*>(e);
  return hipSuccess;
}
}

// ------------------------------------------------------------------ kernel launchers: extents only
namespace lrdm {

int gram_blocks(int n, int nsplit) {
  const uint64_t rows = 1ull << (n - (nsplit == 2 ? 1 : 0));
  const uint64_t chunks = (rows + 63) / 64;
  return (int)(chunks < 256 ? chunks : 256);
}
int gram_seg_shift(int c) {
  int s = 0;
  while ((1 << s) < 2 * c) ++s;
  return ((1 << s) == 2 * c) ? s : -1;
}
uint32_t gram_rows_per_block(int n, int nsplit, int nblocks) {
  const uint32_t rows = 1u << (n - (nsplit == 2 ? 1 : 0));
  const uint32_t chunks = (rows + 63) / 64;
  return (chunks + nblocks - 1) / nblocks * 64;
}
size_t gate_pass_shm(int ncols, int k, size_t csize, int) { return ((size_t)ncols << k) * csize; }

static int nup(int F) {
  const int NT = F / 16;
  return NT * (NT + 1) / 2;
}
template <class T>
static void touch_L(const cx_t<T>* L, int n, int ld, int ncols, const char* what) {
  touch(L, (((size_t)1 << n) - 1) * ld * sizeof(cx_t<T>) + (size_t)ncols * sizeof(cx_t<T>), what);
}
static void touch_eig(const double* S, int Fc, int N, int nsplit, int c, int c_out, const EigBufs& b, const void* W,
                      size_t wsz) {
  touch(S, (size_t)Fc * Fc * 16, "eig S");
  touch(b.P, (size_t)(N - 1) * (N > 1 ? N - 2 : 0) / 2 * 16 + 16, "eig reflectors");
  touch(b.lam, (size_t)N * 8, "eig lambda");
  touch(b.Y, kEigYDoubles * 8, "eig Y");
  touch(b.info, sizeof(DevInfo), "eig info");
  if (b.rec) touch(b.rec, record_doubles(N) * 8, "eig record");
  if (b.W64) touch(b.W64, (size_t)(nsplit * c) * (nsplit * c_out) * 16, "eig W64");
  if (b.M4) touch(b.M4, (size_t)16 * 16 * 16, "eig operator products");
  if (b.E4) touch(b.E4, (size_t)4 * 16 * 16, "eig operators");
  touch(W, (size_t)(nsplit * c) * (nsplit * c_out) * wsz, "eig W");
}

template <class T>
hipError_t launch_gate_pass_batched(const GateJob<T>* jobs, int njobs, uint32_t, size_t, hipStream_t) {
  ++hs::launches;
  touch(jobs, sizeof(GateJob<T>) * njobs, "gate jobs");
  for (int j = 0; j < njobs; ++j) touch_L<T>(jobs[j].L, jobs[j].p.n, jobs[j].p.ld, jobs[j].p.ncols, "gate L");
  return hipSuccess;
}
template <class T>
hipError_t launch_gram_batched(int F, const GramJob<T>* jobs, int njobs, uint32_t, hipStream_t) {
  ++hs::launches;
  touch(jobs, sizeof(GramJob<T>) * njobs, "gram jobs");
  for (int j = 0; j < njobs; ++j) {
    const GramJob<T>& J = jobs[j];
    const int n = 31 - __builtin_clz(J.rows) + (J.nsplit == 2 ? 1 : 0);
    touch_L<T>(J.L, n, J.ld, F / (2 * J.nsplit), "gram L");
    touch(J.partials, (size_t)J.nblocks * nup(F) * 256 * sizeof(T), "gram partials");
  }
  return hipSuccess;
}
template <class T>
hipError_t launch_gram_reduce_batched(const ReduceJob<T>* jobs, int njobs, uint32_t, hipStream_t) {
  ++hs::launches;
  touch(jobs, sizeof(ReduceJob<T>) * njobs, "reduce jobs");
  for (int j = 0; j < njobs; ++j) {
    touch(jobs[j].partials, (size_t)jobs[j].nblocks * jobs[j].NUP * 256 * sizeof(T), "reduce partials");
    touch(jobs[j].S, (size_t)(jobs[j].NT * 8) * (jobs[j].NT * 8) * 16, "reduce S");
  }
  return hipSuccess;
}
template <class T>
hipError_t launch_eig_batched(int, const EigJob<T>* jobs, int njobs, int, hipStream_t) {
  ++hs::launches;
  touch(jobs, sizeof(EigJob<T>) * njobs, "eig jobs");
  for (int j = 0; j < njobs; ++j) {
    const EigJob<T>& J = jobs[j];
    touch_eig(J.S, J.Fc, J.N, J.nsplit, J.c, J.c_out, J.B, J.W, sizeof(cx_t<T>));
  }
  return hipSuccess;
}
template <class T>
hipError_t launch_project_batched(int FO, const ProjJob<T>* jobs, int njobs, uint32_t, hipStream_t) {
  ++hs::launches;
  touch(jobs, sizeof(ProjJob<T>) * njobs, "proj jobs");
  for (int j = 0; j < njobs; ++j) {
    const ProjJob<T>& J = jobs[j];
    const int n = 31 - __builtin_clz(J.rows) + (J.nsplit == 2 ? 1 : 0);
    const int c_in = J.F / (2 * J.nsplit), c_out = FO / (2 * J.nsplit);
    touch_L<T>(J.L, n, J.ld, c_in > c_out ? c_in : c_out, "proj L");
    touch(J.W, (size_t)(J.nsplit * c_in) * (J.nsplit * c_out) * sizeof(cx_t<T>), "proj W");
  }
  return hipSuccess;
}
hipError_t launch_reset_batched(const ResetJob* jobs, int njobs, uint32_t, int, hipStream_t) {
  ++hs::launches;
  touch(jobs, sizeof(ResetJob) * njobs, "reset jobs");
  for (int j = 0; j < njobs; ++j) {
    touch(jobs[j].state, jobs[j].state_bytes, "reset state");
    touch(jobs[j].info, sizeof(DevInfo), "reset info");
  }
  return hipSuccess;
}
hipError_t launch_stamp(uint64_t* slot, hipStream_t) {
  touch(slot, 8, "stamp");
  return hipSuccess;
}
template <class T>
hipError_t launch_gate_pass(const GatePass<T>& p, cx_t<T>* L, hipStream_t) {
  ++hs::launches;
  if (p.k < 0 || p.k > 8 || p.n_ops > kGateMaxOps || p.n_phases > kGateMaxPhases) {
    ++hs::violations;
    std::fprintf(stderr, "gate pass descriptor out of range\n");
  }
  touch_L<T>(L, p.n, p.ld, p.ncols, "gate L");
  return hipSuccess;
}
template <class T>
hipError_t launch_kraus_expand(cx_t<T>* L, int n, int ld, int c, int, const Channel& ch, int m_pad, hipStream_t) {
  ++hs::launches;
  touch_L<T>(L, n, ld, c * m_pad, "kraus expand L");
  return ch.m <= m_pad ? hipSuccess : hipErrorInvalidValue;
}
template <class T>
hipError_t launch_gram(const cx_t<T>* L, int n, int ld, int c, int nsplit, int, T* partials, int nblocks, hipStream_t) {
  ++hs::launches;
  touch_L<T>(L, n, ld, c, "gram L");
  touch(partials, (size_t)nblocks * nup(2 * nsplit * c) * 256 * sizeof(T), "gram partials");
  return hipSuccess;
}
template <class T>
hipError_t launch_gram_reduce(const T* partials, int nblocks, int F, double* S, hipStream_t) {
  ++hs::launches;
  touch(partials, (size_t)nblocks * nup(F) * 256 * sizeof(T), "reduce partials");
  touch(S, (size_t)(F / 2) * (F / 2) * 16, "reduce S");
  return hipSuccess;
}
template <class T>
hipError_t launch_eig(const double* S, int Fc, const Channel&, int nsplit, int c, int N, int, int, double, int, int,
                      int c_out, const EigBufs& b, cx_t<T>* W, hipStream_t) {
  ++hs::launches;
  if (N > kMaxEig) {
    ++hs::violations;
    std::fprintf(stderr, "eigensolve order %d above %d\n", N, kMaxEig);
  }
  touch_eig(S, Fc, N, nsplit, c, c_out, b, W, sizeof(cx_t<T>));
  return hipSuccess;
}
template <class T>
hipError_t launch_project(cx_t<T>* L, int n, int ld, int c_in, int nsplit, int, int c_out, const cx_t<T>* W, int,
                          hipStream_t, int) {
  ++hs::launches;
  touch_L<T>(L, n, ld, c_in > c_out ? c_in : c_out, "proj L");
  touch(W, (size_t)(nsplit * c_in) * (nsplit * c_out) * sizeof(cx_t<T>), "proj W");
  return hipSuccess;
}
template <class T>
hipError_t launch_probabilities(const cx_t<T>* L, int n, int ld, int ncols, double* p, hipStream_t) {
  ++hs::launches;
  touch_L<T>(L, n, ld, ncols, "prob L");
  touch(p, ((size_t)1 << n) * 8, "prob out");
  return hipSuccess;
}
template <class T>
hipError_t launch_zstats(const cx_t<T>* L, int n, int ld, int ncols, double* partials, int nblocks, double* out,
                         hipStream_t s) {
  launch_probabilities<T>(L, n, ld, ncols, partials, s);
  touch(partials, (((size_t)1 << n) + (size_t)nblocks * 64) * 8, "zstats partials");
  touch(out, (size_t)2 * n * 8, "zstats out");
  return hipSuccess;
}
template <class T>
hipError_t launch_pauli(const cx_t<T>* bra, const cx_t<T>* ket, int n, int ld, int ncols, const uint64_t* xm,
                        const uint64_t* zm, int n_terms, double* partials, int ngroups, double* out, int complex_out,
                        hipStream_t) {
  ++hs::launches;
  touch_L<T>(bra, n, ld, ncols, "pauli bra");
  touch_L<T>(ket, n, ld, ncols, "pauli ket");
  touch(xm, (size_t)n_terms * 8, "pauli xmask");
  touch(zm, (size_t)n_terms * 8 + (size_t)(ngroups + 1) * 4, "pauli zmask + group starts");
  const size_t nchunks = ((size_t(1) << n) + 1023) / 1024;
  touch(partials, (size_t)n_terms * nchunks * 2 * 8, "pauli partials");
  touch(out, (size_t)n_terms * (complex_out ? 2 : 1) * 8, "pauli out");
  return hipSuccess;
}
int gram4_blocks_halves(int n) {
  const uint64_t chunks = ((1ull << (n - 2)) + 63) / 64;
  return (int)(chunks < 128 ? chunks : 128);
}
int gram4_blocks_cross(int n) {
  const uint64_t chunks = ((1ull << (n - 2)) + 31) / 32;
  return (int)(chunks < 256 ? chunks : 256);
}
size_t gram4_stream_reals(int n) {
  if (n < 6) return 0;
  const uint64_t nb = std::min<uint64_t>(256, (1ull << (n - 2)) / 16);
  return (size_t)nb * 136 * 2 * 256 + (size_t)136 * 4 * 512 * 2;
}
template <class T>
hipError_t launch_gram4(const cx_t<T>* L, int n, int ld, int c, int p, int q, T* part_h, T* part_c, double* S4,
                        int, hipStream_t) {
  ++hs::launches;
  if (p == q || p < 0 || q < 0 || p >= n || q >= n) {
    ++hs::violations;
    std::fprintf(stderr, "4-way Gram on bits %d, %d of %d qubits\n", p, q, n);
  }
  touch_L<T>(L, n, ld, c, "gram4 L");
  const size_t nt = (size_t)(4 * c) / 16;
  touch(part_h, (size_t)2 * gram4_blocks_halves(n) * (nt * (nt + 1) / 2) * 256 * sizeof(T), "gram4 halves partials");
  touch(part_c, (size_t)gram4_blocks_cross(n) * nt * nt * 256 * sizeof(T), "gram4 cross partials");
  if (sizeof(T) == 4 && c == 64 && n >= 6) touch(part_h, gram4_stream_reals(n) * sizeof(T), "gram4 streamed partials");
  touch(S4, (size_t)(4 * c) * (4 * c) * 16, "gram4 S4");
  return hipSuccess;
}
template <class T>
hipError_t launch_project4(cx_t<T>* L, int n, int ld, int c_in, int q0, int q1, int c_out, const cx_t<T>* W,
                           hipStream_t) {
  ++hs::launches;
  if (q0 == q1 || q0 < 0 || q1 < 0 || q0 >= n || q1 >= n) {
    ++hs::violations;
    std::fprintf(stderr, "pair projection on bits %d, %d of %d qubits\n", q0, q1, n);
  }
  touch_L<T>(L, n, ld, c_in > c_out ? c_in : c_out, "proj4 L");
  touch(W, (size_t)(4 * c_in) * (4 * c_out) * sizeof(cx_t<T>), "proj4 W");
  return hipSuccess;
}
hipError_t launch_pair_transform(const double* G4, const double* W, double* T, double* S, int c, hipStream_t) {
  ++hs::launches;
  touch(G4, (size_t)(4 * c) * (4 * c) * 16, "pair G4");
  touch(W, (size_t)(2 * c) * (2 * c) * 16, "pair W");
  touch(T, (size_t)3 * (2 * c) * (2 * c) * 16, "pair T");
  touch(S, (size_t)(2 * c) * (2 * c) * 16, "pair S");
  return hipSuccess;
}
hipError_t launch_chain_gram(double* S, const double* W, double* tmp, int n, hipStream_t) {
  ++hs::launches;
  touch(S, (size_t)n * n * 16, "chain S");
  touch(W, (size_t)n * n * 16, "chain W");
  touch(tmp, (size_t)n * n * 16, "chain tmp");
  return hipSuccess;
}
template <class T>
hipError_t launch_chain_compose(double* Wp, const double* Wn, double* tmp, cx_t<T>* Wt, int n, hipStream_t) {
  ++hs::launches;
  touch(Wp, (size_t)n * n * 16, "compose Wp");
  touch(Wn, (size_t)n * n * 16, "compose Wn");
  touch(tmp, (size_t)n * n * 16, "compose tmp");
  touch(Wt, (size_t)n * n * sizeof(cx_t<T>), "compose Wt");
  return hipSuccess;
}
hipError_t launch_fdm_pass(const FdmPass& p, float2* rho, hipStream_t) {
  ++hs::launches;
  touch(rho, ((size_t)1 << p.nbits) * 8, "fdm rho");
  return hipSuccess;
}
hipError_t launch_fdm_reset(float2* rho, int n, hipStream_t) {
  touch(rho, ((size_t)1 << (2 * n)) * 8, "fdm reset");
  return hipSuccess;
}
hipError_t launch_fdm_diag(const float2* rho, int n, double* p, hipStream_t) {
  touch(rho, ((size_t)1 << (2 * n)) * 8, "fdm diag rho");
  touch(p, ((size_t)1 << n) * 8, "fdm diag out");
  return hipSuccess;
}
hipError_t launch_fdm_weight(float2* rho, int n, const FdmPhase&, hipStream_t) {
  touch(rho, ((size_t)1 << (2 * n)) * 8, "fdm weight");
  return hipSuccess;
}
template <class T>
hipError_t launch_pauli_apply(cx_t<T>* dst, const cx_t<T>* src, int n, int ld, int ncols, const uint64_t* xm,
                              const uint64_t* zm, const double* coeff, int n_terms, hipStream_t) {
  ++hs::launches;
  touch_L<T>(dst, n, ld, ncols, "pauli apply dst");
  touch_L<T>(src, n, ld, ncols, "pauli apply src");
  touch(xm, (size_t)n_terms * 8, "apply xm");
  touch(zm, (size_t)n_terms * 8, "apply zm");
  touch(coeff, (size_t)n_terms * 8, "apply coeff");
  return hipSuccess;
}
static size_t adj_chunks(int n) {
  (void)n;
  return kAdjChunks;
}
template <class T>
hipError_t launch_gram_exact(const cx_t<T>* L, int n, int ld, int c, int, double* part, double* S, hipStream_t) {
  ++hs::launches;
  touch_L<T>(L, n, ld, c, "exact gram L");
  touch(part, adj_chunks(n) * (size_t)(2 * c) * (2 * c) * 16, "exact gram partials");
  touch(S, (size_t)(2 * c) * (2 * c) * 16, "exact gram S");
  return hipSuccess;
}
template <class T>
hipError_t launch_compress_adjoint(cx_t<T>* Ybar, const cx_t<T>* X, int n, int ld, int c, int, const Channel& ch,
                                   const double* rec, const AdjBufs& b, hipStream_t) {
  ++hs::launches;
  const int N = ch.m * c;
  const size_t e = (size_t)(2 * c) * (2 * c);
  touch_L<T>(Ybar, n, ld, c, "adjoint Ybar");
  touch_L<T>(X, n, ld, c, "adjoint X");
  touch(rec, record_doubles(N) * 8, "adjoint record");
  touch(b.part, adj_chunks(n) * e * 16, "adjoint partials");
  touch(b.C, e * 16, "adjoint C");
  touch(b.H, (size_t)N * c * 16, "adjoint H");
  touch(b.Zh, (size_t)N * c * 16, "adjoint Zh");
  touch(b.T1, (size_t)N * N * 16, "adjoint T1");
  touch(b.Gh, (size_t)N * N * 16, "adjoint Gh");
  touch(b.M, (size_t)N * N * 16, "adjoint M");
  touch(b.P, e * sizeof(cx_t<T>), "adjoint P");
  touch(b.Q, e * sizeof(cx_t<T>), "adjoint Q");
  return hipSuccess;
}
hipError_t launch_sample(const double* p, int n, double* cdf, double* block_sums, const double* u, int count,
                         uint64_t* out, hipStream_t) {
  ++hs::launches;
  const size_t rows = (size_t)1 << n;
  touch(p, rows * 8, "sample p");
  touch(cdf, rows * 8, "sample cdf");
  touch(block_sums, ((rows + 1023) / 1024) * 8, "sample block sums");
  touch(u, (size_t)count * 8, "sample uniforms");
  touch(out, (size_t)count * 8, "sample out");
  return hipSuccess;
}
template <class T>
hipError_t launch_kraus2_expand(cx_t<T>* L, int n, int ld, int c, int, int, const Kraus2Chunk& ck, hipStream_t) {
  ++hs::launches;
  if (ck.na < 1 || ck.na > kKraus2PerLaunch) {
    ++hs::violations;
    std::fprintf(stderr, "two-qubit expansion chunk out of range\n");
  }
  touch_L<T>(L, n, ld, (ck.a0 + ck.na) * c, "kraus2 expand L");
  return hipSuccess;
}
template <class T>
hipError_t launch_set_sparse(cx_t<T>* L, int ld, const uint64_t* idx, const double* amp, int count, hipStream_t) {
  ++hs::launches;
  touch(idx, (size_t)count * 8, "sparse idx");
  touch(amp, (size_t)count * 16, "sparse amp");
  for (int i = 0; i < count; ++i) touch(L + idx[i] * ld, sizeof(cx_t<T>), "sparse entry");
  return hipSuccess;
}
template <class T>
hipError_t launch_lr_to_full(const cx_t<T>* L, int n, int ld, int ncols, float2* rho, hipStream_t) {
  ++hs::launches;
  touch_L<T>(L, n, ld, ncols, "to_full L");
  touch(rho, ((size_t)1 << (2 * n)) * 8, "to_full rho");
  return hipSuccess;
}
template <class T>
hipError_t launch_set_e0(cx_t<T>* L, hipStream_t) {
  touch(L, sizeof(cx_t<T>), "set e0");
  return hipSuccess;
}

#define LRDM_STUB_INST(T)                                                                                        \
  template hipError_t launch_gate_pass_batched<T>(const GateJob<T>*, int, uint32_t, size_t, hipStream_t);       \
  template hipError_t launch_gram_batched<T>(int, const GramJob<T>*, int, uint32_t, hipStream_t);               \
  template hipError_t launch_gram_reduce_batched<T>(const ReduceJob<T>*, int, uint32_t, hipStream_t);           \
  template hipError_t launch_eig_batched<T>(int, const EigJob<T>*, int, int, hipStream_t);                      \
  template hipError_t launch_project_batched<T>(int, const ProjJob<T>*, int, uint32_t, hipStream_t);            \
  template hipError_t launch_gate_pass<T>(const GatePass<T>&, cx_t<T>*, hipStream_t);                           \
  template hipError_t launch_kraus_expand<T>(cx_t<T>*, int, int, int, int, const Channel&, int, hipStream_t);   \
  template hipError_t launch_gram<T>(const cx_t<T>*, int, int, int, int, int, T*, int, hipStream_t);           \
  template hipError_t launch_gram_reduce<T>(const T*, int, int, double*, hipStream_t);                         \
  template hipError_t launch_eig<T>(const double*, int, const Channel&, int, int, int, int, int, double, int,    \
                                    int, int, const EigBufs&, cx_t<T>*, hipStream_t);                           \
  template hipError_t launch_project<T>(cx_t<T>*, int, int, int, int, int, int, const cx_t<T>*, int,            \
                                        hipStream_t, int);                                                          \
  template hipError_t launch_probabilities<T>(const cx_t<T>*, int, int, int, double*, hipStream_t);            \
  template hipError_t launch_zstats<T>(const cx_t<T>*, int, int, int, double*, int, double*, hipStream_t);     \
  template hipError_t launch_pauli<T>(const cx_t<T>*, const cx_t<T>*, int, int, int, const uint64_t*,          \
                                      const uint64_t*, int, double*, int, double*, int, hipStream_t);           \
  template hipError_t launch_chain_compose<T>(double*, const double*, double*, cx_t<T>*, int, hipStream_t);    \
  template hipError_t launch_pauli_apply<T>(cx_t<T>*, const cx_t<T>*, int, int, int, const uint64_t*,          \
                                            const uint64_t*, const double*, int, hipStream_t);                  \
  template hipError_t launch_gram_exact<T>(const cx_t<T>*, int, int, int, int, double*, double*, hipStream_t); \
  template hipError_t launch_compress_adjoint<T>(cx_t<T>*, const cx_t<T>*, int, int, int, int, const Channel&, \
                                                 const double*, const AdjBufs&, hipStream_t);                   \
  template hipError_t launch_set_e0<T>(cx_t<T>*, hipStream_t);                                                   \
  template hipError_t launch_kraus2_expand<T>(cx_t<T>*, int, int, int, int, int, const Kraus2Chunk&, hipStream_t);  \
  template hipError_t launch_set_sparse<T>(cx_t<T>*, int, const uint64_t*, const double*, int, hipStream_t);       \
  template hipError_t launch_lr_to_full<T>(const cx_t<T>*, int, int, int, float2*, hipStream_t);                 \
  template hipError_t launch_gram4<T>(const cx_t<T>*, int, int, int, int, int, T*, T*, double*, int, hipStream_t); \
  template hipError_t launch_project4<T>(cx_t<T>*, int, int, int, int, int, int, const cx_t<T>*, hipStream_t);
LRDM_STUB_INST(float)
LRDM_STUB_INST(double)

}  // namespace lrdm
