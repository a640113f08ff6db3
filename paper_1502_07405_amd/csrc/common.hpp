// Shared host/device definitions of the HIP library: status handling,
// device memory arena, launch descriptors.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/hssmf.h"

namespace hssmf {

// pointer into device global memory: descriptor fields are generic pointers,
// and a kernel that casts them to this keeps its memory operations off the
// flat path (whose completion is counted together with LDS traffic)
template <class T>
using gptr = __attribute__((address_space(1))) T*;

struct Error : std::runtime_error {
  int code;
  int front;
  Error(int c, const std::string& m, int f = -1) : std::runtime_error(m), code(c), front(f) {}
};

#define HIP_CHECK(expr)                                                                  \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      throw ::hssmf::Error(HSSMF_EDEVICE, std::string(#expr ": ") + hipGetErrorString(e_)); \
  } while (0)

#define REQUIRE(cond, code, msg)                  \
  do {                                            \
    if (!(cond)) throw ::hssmf::Error(code, msg); \
  } while (0)

// Bump allocator over large device chunks.  Everything a factorization
// holds lives here and is released at once.  Chunks go back to a process
// wide cache so repeated factorizations do not pay hipMalloc again.
class Arena {
 public:
  ~Arena() { release(); }
  void* alloc(size_t bytes, size_t align = 256);
  template <class T>
  T* get(size_t n) {
    return static_cast<T*>(alloc(sizeof(T) * (n ? n : 1)));
  }
  void release();
  size_t used() const { return used_; }
  // high-water mark of used() since the last reset_peak()
  size_t peak() const { return peak_; }
  void reset_peak() { peak_ = used_; }
  // scoped marks: everything allocated after mark() is reclaimed by reset()
  struct Mark {
    size_t chunk, off, used;
  };
  Mark mark() const { return {chunks_.empty() ? 0 : chunks_.size() - 1, off_, used_}; }
  void reset(const Mark& m);

 private:
  struct Chunk {
    char* p;
    size_t size;
  };
  std::vector<Chunk> chunks_;
  size_t off_ = 0;
  size_t used_ = 0;
  size_t peak_ = 0;
};

// returns every released chunk held for reuse to the runtime
void arena_trim_cache();

// --- batched GEMM descriptor ------------------------------------------------
// C(m x n) = alpha * op(A) op(B) + beta * C, column major.  Optional row maps:
// op(A) row i reads A row amap[i] (transA == 0 only), op(B) row kk reads B
// row bmap[kk] (transB == 0 only), C row i is C row cmap[i].
struct GemmDesc {
  const void* A;
  const void* B;
  void* C;
  const int* amap;
  const int* bmap;
  const int* cmap;
  int m, n, k;
  int lda, ldb, ldc;
  int transA, transB;
  double alpha, beta;
  int tiles_m, tiles_n;
  int64_t tile_base;
};

// input precision of A and B / storage of C
enum GemmType {
  GEMM_F64 = 0,     // double x double -> double (FP64 MFMA)
  GEMM_F32 = 1,     // float x float -> float (FP32 MFMA)
  GEMM_F32_D = 2,   // float x float -> double C
  GEMM_BF16 = 3,    // bf16 x bf16 -> float (FP32 accumulation)
  GEMM_BF16_D = 4,  // bf16 x bf16 -> double C
  GEMM_D_F32 = 5,   // double operands rounded to float on load, FP32 MFMA, double C
};

// launch a batch of GEMMs (descriptors in host memory; staged to the device)
class Stager;
// prints and clears the GEMM shape census when HSSMF_GEMM_CENSUS=1
void gemm_census_print();
// tile_pref: 64 or 128 forces the FP64 tile size, anything else lets the
// autotuner pick (per process, per shape class; results do not depend on it)
void gemm_batched(const std::vector<GemmDesc>& d, GemmType t, Stager& st, hipStream_t s, int tile_pref = 0);

// Pinned host ring + device mirror for per-launch descriptor arrays.
class Stager {
 public:
  Stager() = default;
  ~Stager();
  void init(size_t bytes);
  // copy host bytes to device memory valid until the next sync()
  void* put(const void* src, size_t bytes, hipStream_t s);
  template <class T>
  T* put_vec(const std::vector<T>& v, hipStream_t s) {
    return static_cast<T*>(put(v.data(), v.size() * sizeof(T), s));
  }
  // copy host bytes straight into device memory the caller owns (one
  // pinned H2D copy)
  void put_to(void* dst, const void* src, size_t bytes, hipStream_t s);
  // caller guarantees the stream has drained
  void sync() { off_ = 0; }
  // device workspace for split-K partial products (stream ordered)
  double* ws = nullptr;
  size_t ws_elems = 0;
  // host-to-device copies issued (diagnostics: HSSMF_UPLOAD_CENSUS=1)
  int64_t n_put = 0, n_put_to = 0;

 private:
  char* host_ = nullptr;
  char* dev_ = nullptr;
  size_t cap_ = 0, off_ = 0;
};

// kernel timing hooks (see hssmf_profile_enable)
namespace prof {
bool enabled();
void add_flops(int kclass, double flops);
// event pair recorded around a launch on stream s (for launches that cannot
// take hipExtLaunchKernelGGL events); returns a token for end(), -1 when off
int begin(int kclass, hipStream_t s);
void end(int token, hipStream_t s);
// one timed kernel: events for hipExtLaunchKernelGGL, which stamps them with
// that kernel's own start and end (nullptr events and -1 when off)
int ext(int kclass, double flops, hipEvent_t* start, hipEvent_t* stop);
// waits for a class's recorded events; summed ms, launches and work; resets
int read(int kclass, double* ms, int64_t* launches, double* flops);
}  // namespace prof

}  // namespace hssmf
