// A host-only stand-in for the HIP runtime and for the library's kernel launchers, so that the
// host runtime of the library (qhvp_host.cpp: planning, workspace layout, argument checks, error
// paths, FP64 utilities, the call sequences) can be built with g++ under AddressSanitizer and
// UndefinedBehaviorSanitizer and run on a machine without a GPU.  "Device" memory is host memory;
// kernel launches do nothing and succeed.  Allocation failures can be injected.
#include <hip/hip_runtime_api.h>

#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "../../paper_2604_20384_amd/csrc/qhvp_internal.h"

namespace {
std::mutex g_mu;
std::map<const char*, size_t> g_device;   // live hipMalloc blocks: start -> bytes
int g_fail_device = 0;       // the next g_fail_device hipMalloc calls fail
int g_fail_pinned = 0;       // the next g_fail_pinned hipHostMalloc calls fail
int g_pinned_nth = 0;        // > 0: the g_pinned_nth-th next hipHostMalloc call fails (only that one)
long g_live = 0;             // device + pinned blocks not freed yet
std::vector<unsigned char> g_scratch;      // the scratch of the allocation-free entry point
}  // namespace

extern "C" void stub_fail_allocations(int device_calls, int pinned_calls) {
  std::lock_guard<std::mutex> l(g_mu);
  g_fail_device = device_calls;
  g_fail_pinned = pinned_calls;
}
extern "C" void stub_fail_pinned_nth(int nth) {
  std::lock_guard<std::mutex> l(g_mu);
  g_pinned_nth = nth;
}
extern "C" long stub_live_blocks() {
  std::lock_guard<std::mutex> l(g_mu);
  return g_live;
}

extern "C" {
hipError_t hipGetDeviceCount(int* count) { *count = 1; return hipSuccess; }
hipError_t hipSetDevice(int device) { return device == 0 ? hipSuccess : hipErrorInvalidDevice; }
hipError_t hipMalloc(void** ptr, size_t size) {
  std::lock_guard<std::mutex> l(g_mu);
  if (g_fail_device > 0) { --g_fail_device; *ptr = nullptr; return hipErrorOutOfMemory; }
  *ptr = std::calloc(1, size ? size : 1);
  if (!*ptr) return hipErrorOutOfMemory;
  g_device[(const char*)*ptr] = size;
  ++g_live;
  return hipSuccess;
}
hipError_t hipFree(void* ptr) {
  std::lock_guard<std::mutex> l(g_mu);
  if (!ptr) return hipSuccess;
  if (!g_device.erase((const char*)ptr)) return hipErrorInvalidValue;
  std::free(ptr);
  --g_live;
  return hipSuccess;
}
hipError_t hipHostMalloc(void** ptr, size_t size, unsigned int) {
  std::lock_guard<std::mutex> l(g_mu);
  if (g_fail_pinned > 0) { --g_fail_pinned; *ptr = nullptr; return hipErrorOutOfMemory; }
  if (g_pinned_nth > 0 && --g_pinned_nth == 0) { *ptr = nullptr; return hipErrorOutOfMemory; }
  *ptr = std::calloc(1, size ? size : 1);
  if (!*ptr) return hipErrorOutOfMemory;
  ++g_live;
  return hipSuccess;
}
hipError_t hipHostFree(void* ptr) {
  std::lock_guard<std::mutex> l(g_mu);
  if (ptr) { std::free(ptr); --g_live; }
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind, hipStream_t) {
  std::memmove(dst, src, bytes);
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipDeviceSynchronize(void) { return hipSuccess; }
hipError_t hipEventCreate(hipEvent_t* e) { *e = (hipEvent_t)new int(0); return hipSuccess; }
hipError_t hipEventDestroy(hipEvent_t e) { delete (int*)e; return hipSuccess; }
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) { *ms = 0.f; return hipSuccess; }
hipError_t hipGetLastError(void) { return hipSuccess; }
const char* hipGetErrorString(hipError_t e) { return e == hipSuccess ? "hipSuccess" : "stub error"; }
hipError_t hipPointerGetAttributes(hipPointerAttribute_t* at, const void* ptr) {
  std::lock_guard<std::mutex> l(g_mu);
  const char* p = (const char*)ptr;
  auto it = g_device.upper_bound(p);
  if (it != g_device.begin()) {
    --it;
    if (p >= it->first && p < it->first + it->second) {
      std::memset(at, 0, sizeof(*at));
      at->type = hipMemoryTypeDevice;
      at->device = 0;
      return hipSuccess;
    }
  }
  return hipErrorInvalidValue;   // plain host memory
}
}  // extern "C"

namespace qhvp {
int grid_size(long long items) { return (int)(items < 2048 ? items : 2048); }
int bwd_grid(Prec, int, int, long long items, int) { return grid_size(items); }
int launch_fwd(Prec, const FwdArgs&, void*) { return 0; }
int launch_bwd(Prec, const BwdArgs&, void*) { return 0; }
int launch_bwd_out(Prec, const BwdArgs&, void*) { return 0; }
int launch_zero_ints(int* p, int n, void*) { std::memset(p, 0, sizeof(int) * (size_t)n); return 0; }
int launch_reduce_overlaps(const double*, int, int, double*, void*) { return 0; }
int launch_reduce_env(const double*, int, int, const int*, const PassDesc&, double*, void*) { return 0; }
int launch_prep(const PrepArgs&, void*) { return 0; }
int launch_post(const PostArgs&, void*) { return 0; }
int launch_convert(const double*, void*, long long, int, void*) { return 0; }
int launch_ti_expand(const double*, int, int, double*, void*) { return 0; }
int launch_ti_reduce(const double*, int, int, const int*, double*, void*) { return 0; }
int noalloc_scratch_init(int) { return 0; }
void* noalloc_scratch(int) {
  std::lock_guard<std::mutex> l(g_mu);
  if (g_scratch.empty()) g_scratch.resize(kNoAllocScratchBytes);
  return g_scratch.data();
}
}  // namespace qhvp
