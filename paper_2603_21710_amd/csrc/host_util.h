// Host helpers shared by the library's translation units: error reporting,
// the scratch arena, launch helpers and dataset validation.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <string>
#include <vector>

#include "fgim.h"

namespace fgim {

fgim_status fail(fgim_status s, const char* fmt, ...);
// empties the calling thread's last-error detail (start of every entry point)
void clear_error();
int device_cus();
hipError_t fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t s);
fgim_status check_dataset(const fgim_dataset* d, bool need_cross);
// a non-blocking, default-priority stream owned by the library (one per
// device), used where work has to be captured into a hipGraph
hipError_t library_stream(hipStream_t* out);
// BF16 (round to nearest even) or FP8 E4M3 (per-row scale) copy of n rows
fgim_status quantize_into(const float* base, uint64_t n, uint32_t dim, uint64_t ld, fgim_precision prec,
                          void* codes, float* scales, hipStream_t s);

// Raise the release threshold of the device's current memory pool (once per
// device, and only when it is still 0, the runtime's default), so that
// memory freed by stream-ordered release stays in the pool instead of going
// back to the driver at every synchronisation.
void keep_scratch_cached();

// Scratch memory for one library call.  Buffers come from a library-owned
// arena on the current device, bump-allocated in nested scopes and reused
// by later calls: stream-ordered allocation and release cost the host tens
// to hundreds of microseconds per buffer, which the device would wait out
// between stages.  The arena grows, between calls, to the largest total a
// call has asked for; until it has, the excess comes from the device's
// memory pool (stream-ordered).  One call at a time holds a device's arena
// (other host threads wait), and a call's stream first waits for the device
// work of the previous call that used it.  fgim_release_scratch() returns
// the arena to the driver.
struct Scratch {
  hipStream_t s;
  int dev = -1;
  size_t mark_top = 0, mark_virt = 0;
  std::vector<void*> spill;  // buffers outside the arena
  explicit Scratch(hipStream_t st);
  ~Scratch();
  Scratch(const Scratch&) = delete;
  Scratch& operator=(const Scratch&) = delete;
  void* take(size_t bytes);  // from the arena, or nullptr when it is full
  template <class T>
  fgim_status get(T** out, size_t count) {
    const size_t bytes = std::max<size_t>(count * sizeof(T), 16);
    void* p = take(bytes);
    if (!p) {
      hipError_t e = hipMallocAsync(&p, bytes, s);
      if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        return fail(FGIM_ERR_OUT_OF_MEMORY, "scratch allocation of %zu bytes failed", bytes);
      }
      spill.push_back(p);
    }
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
