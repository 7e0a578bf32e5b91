// Allocation-free crystal linewidths: kaldo_linewidths with its workspace in
// a device array of the library instead of a caller buffer, for callers that
// cannot allocate (code under HIP graph capture, serving loops, harnesses
// that forbid hipMalloc).
//
// The array is a file-scope __device__ symbol: every GPU the library runs on
// holds its own copy, at its own address, until the process ends.  Host code
// never passes the symbol itself to a kernel (in host code it is only a
// stand-in for the device object); its device address is looked up once per
// device with hipGetSymbolAddress and kept here.
#include <mutex>

#include "common.h"

namespace kaldo {

int linewidths_enqueue(const kaldo_crystal* c, const int32_t* mesh, const double* omega,
                       const double* evec, const double* vel, double temperature,
                       const kaldo_broadening* b, int32_t precision,
                       const int32_t* modes_subset, int64_t n_subset, void* workspace,
                       size_t workspace_bytes, double* gamma, hipStream_t st);

constexpr size_t kScratchBytes = size_t(32) << 20;  // 32 MiB per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (looked up on first use).
static int scratch_address(void** out) {
  int dev = -1;
  KALDO_HIP(hipGetDevice(&dev));
  KALDO_REQUIRE(dev >= 0 && dev < kMaxDevices, "kaldo_linewidths_noalloc: device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    KALDO_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    KALDO_REQUIRE(p != nullptr, "kaldo_linewidths_noalloc: no device address for the scratch array");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return KALDO_OK;
}

}  // namespace kaldo

using namespace kaldo;

extern "C" size_t kaldo_linewidths_noalloc_max_bytes(void) { return kScratchBytes; }

extern "C" int kaldo_linewidths_noalloc(const kaldo_crystal* c, const int32_t* mesh,
                                        const double* omega, const double* evec,
                                        const double* vel, double temperature,
                                        const kaldo_broadening* b, int32_t precision,
                                        const int32_t* modes_subset, int64_t n_subset,
                                        double* gamma, void* stream) {
  KALDO_REQUIRE(c && mesh, "kaldo_linewidths_noalloc: NULL argument");
  KALDO_REQUIRE(mesh[0] >= 1 && mesh[1] >= 1 && mesh[2] >= 1,
                "kaldo_linewidths_noalloc: mesh must be >= 1");
  const size_t need = kaldo_linewidths_workspace(c, mesh, precision);
  if (need > kScratchBytes) {
    set_error("kaldo_linewidths_noalloc: this crystal, mesh and precision need " +
              std::to_string(need) + " bytes of workspace, more than the " +
              std::to_string(kScratchBytes) + "-byte device scratch array");
    return KALDO_EINVAL;
  }
  void* ws = nullptr;
  int rc = scratch_address(&ws);
  if (rc) return rc;
  return linewidths_enqueue(c, mesh, omega, evec, vel, temperature, b, precision, modes_subset,
                            n_subset, ws, kScratchBytes, gamma, static_cast<hipStream_t>(stream));
}
