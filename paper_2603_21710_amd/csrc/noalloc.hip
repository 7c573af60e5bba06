// Stage 1 (cross-querying) without any device allocation, for callers that
// cannot allocate: the beam kernel's queue head, error flag, counters and
// sub-index table live in `scratch`, a fixed array in the library's own
// device memory, instead of the per-call scratch arena.
#include <mutex>

#include "fgim.h"
#include "fgim_internal.h"
#include "host_util.h"

namespace fgim {
namespace noalloc {

constexpr uint32_t kMaxSubs = 4096;   // the library's limit on h
constexpr size_t kHeadBytes = 256;    // header: 4 uint32 at 0, 4 counters at 64
constexpr size_t kBytes = kHeadBytes + sizeof(SubDev) * kMaxSubs;  // 131,328 bytes
constexpr int kMaxDevices = 64;

}  // namespace noalloc
}  // namespace fgim

// Each GPU holds its own copy of this array until the process ends.  In host
// code its name is only a stand-in for the symbol: the device address comes
// from hipGetSymbolAddress (scratch_base below), never from `scratch`.
static __device__ __align__(256) unsigned char scratch[fgim::noalloc::kBytes];

namespace fgim {
namespace noalloc {

struct Device {
  std::mutex mu;        // held for a whole call: calls on one GPU run one at a time
  void* ptr = nullptr;  // device address of this GPU's `scratch`
  SubDev host_subs[kMaxSubs];  // host staging of the sub-index table
};

Device g_dev[kMaxDevices];

// The device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
fgim_status scratch_base(Device& dv, void** out) {
  if (!dv.ptr) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return fail(FGIM_ERR_DEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    }
    dv.ptr = p;
  }
  *out = dv.ptr;
  return FGIM_OK;
}

}  // namespace noalloc
}  // namespace fgim

using namespace fgim;

extern "C" fgim_status fgim_cross_query_noalloc(const fgim_dataset* data, const fgim_params* params,
                                                uint32_t* knn_ids, float* knn_dist, void* stream) {
  clear_error();
  FGIM_TRY(cross_query_check(data, params, knn_ids, knn_dist));
  if (params->autotune)
    return fail(FGIM_ERR_INVALID_ARG, "autotune = 1 needs scratch memory for its trial launches; "
                                      "fgim_cross_query_noalloc takes autotune = 0 only");
  if (params->precision != FGIM_FP32 &&
      (!data->base_lp || (params->precision == FGIM_FP8_E4M3 && !data->base_lp_scale)))
    return fail(FGIM_ERR_INVALID_ARG, "the BF16 / FP8 forms need the low-precision copy in data->base_lp "
                                      "(and data->base_lp_scale for FP8): fgim_cross_query_noalloc does not "
                                      "quantise");
  if (data->h > noalloc::kMaxSubs)
    return fail(FGIM_ERR_INVALID_ARG, "h = %u sub-indexes exceeds the fixed scratch table (%u)", data->h,
                noalloc::kMaxSubs);
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= noalloc::kMaxDevices) return fail(FGIM_ERR_DEVICE, "device %d out of range", dev);
  noalloc::Device& dv = noalloc::g_dev[dev];
  std::lock_guard<std::mutex> lock(dv.mu);
  void* base = nullptr;
  FGIM_TRY(noalloc::scratch_base(dv, &base));
  char* p = static_cast<char*>(base);
  CrossBufs b{};
  b.hdr = reinterpret_cast<uint32_t*>(p);
  b.cnt = reinterpret_cast<unsigned long long*>(p + 64);
  b.subs = reinterpret_cast<SubDev*>(p + noalloc::kHeadBytes);
  b.host_subs = dv.host_subs;
  b.lp = data->base_lp;
  b.lps = data->base_lp_scale;
  // cross_query_run clears the header with fill kernels before the launch
  // and synchronises the stream before it returns
  return cross_query_run(data, params, knn_ids, knn_dist, nullptr, static_cast<hipStream_t>(stream), nullptr, b);
}
