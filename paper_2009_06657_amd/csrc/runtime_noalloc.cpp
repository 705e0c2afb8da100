// Allocation-free <Z_i> / <Z_i Z_{i+1}> of a caller-held factor, for callers that cannot allocate
// device memory.  The kernels' scratch (Prob(x) and the per-block partial sums of the reduction)
// lives in a file-scope device array of the library, one per GPU, held until the process ends.
// Its device address is looked up once per device (hipGetSymbolAddress, with that device
// current) and only that address is handed to kernels and copies.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "lrdm_internal.h"

namespace {

constexpr int kNoallocMaxQubits = 20;
constexpr int kNoallocBlocks = 256;   // reduction blocks (the same split as lrdm_expect_z)
constexpr size_t kProbDoubles = (size_t)1 << kNoallocMaxQubits;
constexpr size_t kPartDoubles = (size_t)kNoallocBlocks * 64;
constexpr size_t kOutDoubles = 64;
constexpr size_t kScratchBytes = (kProbDoubles + kPartDoubles + kOutDoubles) * sizeof(double);

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

lrdm_status nfail(lrdm_status st, const std::string& msg) {
  lrdm::set_last_error(msg.c_str());
  return st;
}

}  // namespace

// Per-GPU scratch of lrdm_expect_z_noalloc: Prob(x) (2^20 doubles), the reduction's block
// partials and its outputs.
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

extern "C" lrdm_status lrdm_expect_z_noalloc(const void* L_dev, int n, int ld, int ncols, lrdm_dtype dt,
                                             void* hip_stream, double* z_host, double* zz_host,
                                             double* trace_host) {
  if (!L_dev || !z_host) return nfail(LRDM_E_ARG, "null factor or z output");
  if (dt != LRDM_C64 && dt != LRDM_C128) return nfail(LRDM_E_ARG, "unknown dtype");
  if (n < 1) return nfail(LRDM_E_ARG, "n must be >= 1");
  if (n > kNoallocMaxQubits)
    return nfail(LRDM_E_UNSUPPORTED, "lrdm_expect_z_noalloc takes n <= 20 (its scratch holds 2^20 probabilities)");
  if (ld < 1 || ncols < 1 || ncols > ld) return nfail(LRDM_E_ARG, "need 1 <= ncols <= ld");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return nfail(LRDM_E_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return nfail(LRDM_E_UNSUPPORTED, "device index above 63");
  double* base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
      void* p = nullptr;
      e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !p)
        return nfail(LRDM_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
      g_ptr[dev] = p;
    }
    base = static_cast<double*>(g_ptr[dev]);
  }
  double* prob_and_part = base;                  // 2^n Prob, then the block partials
  double* out = base + kProbDoubles + kPartDoubles;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  // every entry the reduction reads is written earlier in the same call (Prob for every x, a
  // partial for every block and accumulator), so nothing is cleared between calls
  e = dt == LRDM_C64
          ? lrdm::launch_zstats<float>(static_cast<const float2*>(L_dev), n, ld, ncols, prob_and_part,
                                      kNoallocBlocks, out, s)
          : lrdm::launch_zstats<double>(static_cast<const double2*>(L_dev), n, ld, ncols, prob_and_part,
                                       kNoallocBlocks, out, s);
  if (e != hipSuccess) return nfail(LRDM_E_HIP, std::string("zstats launch: ") + hipGetErrorString(e));
  double r[2 * kNoallocMaxQubits];
  e = hipMemcpyAsync(r, out, sizeof(double) * 2 * n, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return nfail(LRDM_E_HIP, std::string("result copy: ") + hipGetErrorString(e));
  const double tot = r[0];
  for (int i = 0; i < n; ++i) z_host[i] = tot - 2.0 * r[1 + i];
  if (zz_host)
    for (int i = 0; i + 1 < n; ++i) zz_host[i] = tot - 2.0 * r[1 + n + i];
  if (trace_host) *trace_host = tot;
  return LRDM_OK;
}
