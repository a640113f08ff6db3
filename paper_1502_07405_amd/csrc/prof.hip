// Kernel timing hooks: event pairs stamped by hipExtLaunchKernelGGL with the
// start and end of selected kernels.
#include <mutex>
#include <vector>

#include "common.hpp"

namespace hssmf {
namespace prof {

namespace {
struct Rec {
  int kclass;
  hipEvent_t a, b;
  double flops;
};
std::mutex mu;
bool on = false;
std::vector<Rec> recs;
std::vector<hipEvent_t> pool;
double extra_flops[8] = {0};

hipEvent_t get_event() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e;
  HIP_CHECK(hipEventCreate(&e));
  return e;
}
}  // namespace

bool enabled() { return on; }

int begin(int kclass, hipStream_t s) {
  if (!on) return -1;
  std::lock_guard<std::mutex> g(mu);
  Rec r{kclass, get_event(), get_event(), 0.0};
  HIP_CHECK(hipEventRecord(r.a, s));
  recs.push_back(r);
  return (int)recs.size() - 1;
}

void end(int token, hipStream_t s) {
  if (token < 0) return;
  std::lock_guard<std::mutex> g(mu);
  HIP_CHECK(hipEventRecord(recs[token].b, s));
}

int ext(int kclass, double flops, hipEvent_t* start, hipEvent_t* stop) {
  *start = *stop = nullptr;
  if (!on) return -1;
  std::lock_guard<std::mutex> g(mu);
  Rec r{kclass, get_event(), get_event(), flops};
  *start = r.a;
  *stop = r.b;
  recs.push_back(r);
  return (int)recs.size() - 1;
}

void add_flops(int kclass, double flops) {
  if (!on || kclass < 0 || kclass >= 8) return;
  std::lock_guard<std::mutex> g(mu);
  extra_flops[kclass] += flops;
}

int read(int kclass, double* ms, int64_t* launches, double* flops) {
  std::lock_guard<std::mutex> g(mu);
  double t = 0, w = 0;
  int64_t n = 0;
  std::vector<Rec> keep;
  for (auto& r : recs) {
    if (r.kclass != kclass) { keep.push_back(r); continue; }
    HIP_CHECK(hipEventSynchronize(r.b));
    float e = 0;
    HIP_CHECK(hipEventElapsedTime(&e, r.a, r.b));
    t += e;
    w += r.flops;
    ++n;
    pool.push_back(r.a);
    pool.push_back(r.b);
  }
  recs.swap(keep);
  if (kclass >= 0 && kclass < 8) { w += extra_flops[kclass]; extra_flops[kclass] = 0; }
  if (ms) *ms = t;
  if (launches) *launches = n;
  if (flops) *flops = w;
  return 0;
}

void set(bool v) {
  std::lock_guard<std::mutex> g(mu);
  on = v;
}

}  // namespace prof
}  // namespace hssmf

extern "C" int hssmf_profile_enable(int32_t v) {
  try {
    hssmf::prof::set(v != 0);
    return HSSMF_OK;
  } catch (...) {
    return HSSMF_EDEVICE;
  }
}

extern "C" int hssmf_profile_read(int32_t kclass, double* ms, int64_t* launches, double* flops) {
  if (kclass < 0 || kclass > 7) return HSSMF_EINVAL;
  try {
    return hssmf::prof::read(kclass, ms, launches, flops);
  } catch (const hssmf::Error& e) {
    return e.code;
  } catch (...) {
    return HSSMF_EDEVICE;
  }
}
