// Spline prolongation for callers that cannot allocate device memory.
//
// The same operator as mg_prolong with kind MG_PROLONG_SPLINE (the tensor
// cubic spline through the coarse nodes, Section 2.2; the appendix's
// V-cycle prolongates the correction), computed by the same two kernels: the
// B-spline prefilter, whose x-filtered intermediate and coefficients are the
// scratch this operator needs, then the evaluation on the fine grid.  Here
// that scratch is a file-scope device array instead of a context's
// workspace, so a call needs no context and allocates nothing.

#include <mutex>
#include <new>
#include <string>

#include "mg.h"
#include "mg_internal.h"

namespace mg {
namespace {

// Largest coarse side the static scratch holds, and the scratch itself: the
// x-filtered intermediate and the coefficients, each nc x nc elements of the
// call's dtype at pitch nc, each starting on a 256-byte boundary.
constexpr int kNoAllocMaxCoarse = 1025;
constexpr size_t kNoAllocArrayBytes =
    ((size_t)kNoAllocMaxCoarse * kNoAllocMaxCoarse * sizeof(double) + 255) / 256 * 256;
constexpr size_t kNoAllocScratchBytes = 2 * kNoAllocArrayBytes;  // 16.8 MB

// One copy per GPU, held until the process ends.  Host code never uses this
// name as an address (on the host it is a stand-in, not device memory): it
// uses the per-device address that scratch_for() looks up.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this GPU's scratch, looked up once per device with that
// device current (the first call on it).
int32_t scratch_for(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices)
    return set_last_error(MG_ERR_UNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return set_last_error(MG_ERR_HIP, (std::string("hipGetSymbolAddress(scratch): ") +
                                         hipGetErrorString(e)).c_str());
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return MG_OK;
}

template <typename T>
int32_t prolong_noalloc(int nc, int bc, const T* coarse, T* fine, hipStream_t s,
                        unsigned char* base) {
  const int n = 2 * nc - 1;
  T* tmp = reinterpret_cast<T*>(base);
  T* c = reinterpret_cast<T*>(base + kNoAllocArrayBytes);
  PrefilterTaps taps;
  spline_taps(nc, bc, sizeof(T) == 8 ? kPrefilterHalfTapsF64 : kPrefilterHalfTapsF32, &taps);
  hipError_t e = launch_prefilter<T>(s, bc, nc, taps, coarse, nc, tmp, nc, c, nc);
  if (e == hipSuccess) e = launch_prolong<T>(s, bc, n, fine, n, c, nc, false);
  if (e != hipSuccess)
    return set_last_error(MG_ERR_HIP, (std::string("prolongation launch: ") +
                                       hipGetErrorString(e)).c_str());
  return MG_OK;
}

}  // namespace
}  // namespace mg

using namespace mg;

namespace {
int32_t prolong_noalloc_entry(int32_t nc, int32_t bc, const void* coarse, void* fine,
                              int32_t dtype, void* hip_stream) {
  if (!valid_side(nc) || !valid_side(2 * nc - 1))
    return set_last_error(MG_ERR_INVALID_ARG, "coarse side is not 4*2^k+1 with a valid fine side");
  if (nc > kNoAllocMaxCoarse)
    return set_last_error(MG_ERR_UNSUPPORTED,
                          "coarse side above 1025, the largest the static scratch holds");
  if (bc != kDirichlet && bc != kPeriodic)
    return set_last_error(MG_ERR_INVALID_ARG, "bad boundary condition");
  if (dtype != MG_DT_F64 && dtype != MG_DT_F32)
    return set_last_error(MG_ERR_INVALID_ARG, "bad dtype");
  if (!coarse || !fine) return set_last_error(MG_ERR_INVALID_ARG, "NULL array");
  if (coarse == fine) return set_last_error(MG_ERR_INVALID_ARG, "fine aliases coarse");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return set_last_error(MG_ERR_HIP, "hipGetDevice");
  void* base = nullptr;
  const int32_t st = scratch_for(dev, &base);
  if (st != MG_OK) return st;
  const hipStream_t s = static_cast<hipStream_t>(hip_stream);
  unsigned char* b = static_cast<unsigned char*>(base);
  if (dtype == MG_DT_F64)
    return prolong_noalloc<double>(nc, bc, static_cast<const double*>(coarse),
                                   static_cast<double*>(fine), s, b);
  return prolong_noalloc<float>(nc, bc, static_cast<const float*>(coarse),
                                static_cast<float*>(fine), s, b);
}
}  // namespace

extern "C" int32_t mg_prolong_noalloc(int32_t nc, int32_t bc, const void* coarse, void* fine,
                                      int32_t dtype, void* hip_stream) {
  set_last_error(MG_OK, "");
  try {
    return prolong_noalloc_entry(nc, bc, coarse, fine, dtype, hip_stream);
  } catch (const std::bad_alloc&) {
    return set_last_error(MG_ERR_OOM, "host allocation failed");
  } catch (...) {
    return set_last_error(MG_ERR_HIP, "unexpected exception");
  }
}
