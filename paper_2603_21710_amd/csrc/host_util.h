// Host helpers shared by the library's translation units: error reporting,
// stream-ordered scratch, launch helpers and dataset validation.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <string>
#include <vector>

#include "fgim.h"

namespace fgim {

fgim_status fail(fgim_status s, const char* fmt, ...);
int device_cus();
hipError_t fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t s);
fgim_status check_dataset(const fgim_dataset* d, bool need_cross);
// a non-blocking, default-priority stream owned by the library (one per
// device), used where work has to be captured into a hipGraph
hipError_t library_stream(hipStream_t* out);
// BF16 (round to nearest even) or FP8 E4M3 (per-row scale) copy of n rows
fgim_status quantize_into(const float* base, uint64_t n, uint32_t dim, uint64_t ld, fgim_precision prec,
                          void* codes, float* scales, hipStream_t s);

// Stream-ordered scratch, released (stream-ordered) at scope exit.
struct Scratch {
  hipStream_t s;
  std::vector<void*> ptrs;
  explicit Scratch(hipStream_t st) : s(st) {}
  Scratch(const Scratch&) = delete;
  Scratch& operator=(const Scratch&) = delete;
  ~Scratch() {
    for (void* p : ptrs) (void)hipFreeAsync(p, s);
  }
  template <class T>
  fgim_status get(T** out, size_t count) {
    void* p = nullptr;
    size_t bytes = std::max<size_t>(count * sizeof(T), 16);
    hipError_t e = hipMallocAsync(&p, bytes, s);
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return fail(FGIM_ERR_OUT_OF_MEMORY, "scratch allocation of %zu bytes failed", bytes);
    }
    ptrs.push_back(p);
    *out = static_cast<T*>(p);
    return FGIM_OK;
  }
};

}  // namespace fgim

#define FGIM_TRY(x)                 \
  do {                              \
    fgim_status st_ = (x);          \
    if (st_ != FGIM_OK) return st_; \
  } while (0)

#define HIP_TRY(x)                                                                          \
  do {                                                                                      \
    hipError_t e_ = (x);                                                                    \
    if (e_ != hipSuccess)                                                                   \
      return ::fgim::fail(FGIM_ERR_DEVICE, "%s failed: %s", #x, hipGetErrorString(e_));     \
  } while (0)
