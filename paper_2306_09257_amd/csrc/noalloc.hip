// Allocation-free variant of apf_weighted_power for callers that cannot
// allocate device memory (code under HIP graph capture, serving loops,
// harnesses that forbid hipMalloc).
//
// The block partial sums of the objective's reduction live in a file-scope
// device array instead of a library allocation.  Each device holds its own
// copy; its address is looked up once per device (with that device current)
// and kept, and only that address is ever handed to kernels or copies.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "apf_internal.h"
#include "kernels.h"

namespace apf {

// Block partials of one call: the reduction runs at most 1024 blocks of 256
// threads (grid-stride over the entries), so 8 KiB per device suffice.
constexpr int kNoAllocParts = 1024;
// Largest S the call accepts (entries): beyond it the 64-bit byte offsets of
// the interleaved complex array would leave the range the kernels index.
constexpr int64_t kNoAllocMaxEntries = int64_t(1) << 40;

namespace {

static __device__ __align__(256) double scratch[kNoAllocParts];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double *g_scratch[kMaxDevices] = {nullptr};

// Device address of this device's copy of `scratch` (looked up on the first
// call on the device).  Returns null and sets `err` on failure.
double *scratch_on(int dev, std::string &err) {
  if (dev < 0 || dev >= kMaxDevices) {
    err = "device index out of range";
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      err = std::string("hipGetSymbolAddress: ") + hipGetErrorString(e);
      return nullptr;
    }
    g_scratch[dev] = static_cast<double *>(p);
  }
  return g_scratch[dev];
}

}  // namespace

// Block count of the weighted-power reduction for n entries; the same formula
// as apf_weighted_power's, so both entry points sum in the same order.
int weighted_power_parts(int64_t n) {
  const int64_t b = (n + 255) / 256;
  return (int)(b < 1024 ? b : 1024);
}

}  // namespace apf

// thread-local message shared with the rest of the library (api.cpp)
void apf_set_error(const std::string &msg);

extern "C" apf_status apf_weighted_power_noalloc(const double *S_dev, const double *w_dev, int64_t n,
                                                 double *f_dev, double *dfdS_dev, void *stream) {
  using namespace apf;
  if (!S_dev || !w_dev || !f_dev || !dfdS_dev) {
    apf_set_error("null argument");
    return APF_EINVAL;
  }
  if (n < 1 || n > kNoAllocMaxEntries) {
    apf_set_error("n must be in [1, 2^40] entries");
    return APF_EINVAL;
  }
  const int npart = weighted_power_parts(n);
  if (npart > kNoAllocParts) {
    apf_set_error("more block partials than the static scratch holds");
    return APF_EINVAL;
  }
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    apf_set_error(std::string("hipGetDevice: ") + hipGetErrorString(e));
    return APF_EHIP;
  }
  std::string err;
  double *part = scratch_on(dev, err);
  if (!part) {
    apf_set_error(err);
    return APF_EHIP;
  }
  e = launch_weighted_power(reinterpret_cast<const cplx *>(S_dev), w_dev, f_dev, reinterpret_cast<cplx *>(dfdS_dev),
                            n, part, npart, (hipStream_t)stream);
  if (e != hipSuccess) {
    apf_set_error(std::string("kernel launch: ") + hipGetErrorString(e));
    return APF_EHIP;
  }
  apf_set_error("");
  return APF_OK;
}
