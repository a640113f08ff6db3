// hssmf_solve_noalloc: the outer solve with its work vectors in a static
// device array, for callers that cannot allocate device memory.
//
// The array below is a file-scope __device__ symbol: every GPU the library
// runs on holds its own copy, at its own address, until the process ends.
// In host code the symbol's name is only a host-side stand-in, never a
// device address, so the address each device sees is looked up once per
// device with hipGetSymbolAddress (with that device current) and kept in
// scratch_ptr[]; host code hands kernels that pointer only.
#include <mutex>

#include "solver.hpp"

namespace {

constexpr size_t kScratchDoubles = HSSMF_NOALLOC_SCRATCH_BYTES / sizeof(double);
static_assert(HSSMF_NOALLOC_SCRATCH_BYTES % 256 == 0, "scratch size");

__device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
double* scratch_ptr[kMaxDevices] = {};

// device address of this GPU's scratch (looked up on first use per device)
double* device_scratch(int dev) {
  REQUIRE(dev >= 0 && dev < kMaxDevices, HSSMF_EDEVICE, "no-allocation solve: device index out of range");
  std::lock_guard<std::mutex> lk(scratch_mu);
  if (!scratch_ptr[dev]) {
    int cur = -1;
    HIP_CHECK(hipGetDevice(&cur));
    if (cur != dev) HIP_CHECK(hipSetDevice(dev));
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    HIP_CHECK(e);
    REQUIRE(p != nullptr, HSSMF_EDEVICE, "no-allocation solve: no address for the scratch array");
    scratch_ptr[dev] = static_cast<double*>(p);
  }
  return scratch_ptr[dev];
}

}  // namespace

extern "C" int hssmf_solve_noalloc(void* hv, int32_t nrhs, const double* b, double* x, hssmf_info* info) {
  using namespace hssmf;
  Handle* h = static_cast<Handle*>(hv);
  if (!h || nrhs < 0 || (nrhs > 0 && (!b || !x))) return HSSMF_EINVAL;
  if (h->factor_status != HSSMF_OK) return h->factor_status;
  const size_t need = outer_workspace(h->o, h->P.n);
  if (need > kScratchDoubles) return HSSMF_ETOOBIG;
  int out = HSSMF_OK;
  try {
    double* ws = device_scratch(h->device);
    for (int j = 0; j < nrhs; ++j) {
      const size_t off = (size_t)j * (size_t)h->P.n;
      int st = outer_solve(*h, 0, b + off, x + off, info ? info + j : nullptr, ws, kScratchDoubles);
      if (st != HSSMF_OK && out == HSSMF_OK) out = st;
    }
  } catch (const Error& e) {
    if (std::getenv("HSSMF_VERBOSE")) std::fprintf(stderr, "hssmf: %s\n", e.what());
    return e.code;
  } catch (const std::exception& e) {
    if (std::getenv("HSSMF_VERBOSE")) std::fprintf(stderr, "hssmf: %s\n", e.what());
    return HSSMF_EDEVICE;
  }
  return out;
}
