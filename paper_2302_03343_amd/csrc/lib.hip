// Library-wide helpers: thread-local error message, allocation wrappers,
// device properties.
#include "common.h"

#include <mutex>
#include <stdlib.h>
#include <string>

namespace vgx {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

vgx_status hip_fail(hipError_t e, const char* what, const char* file, int line) {
  set_error("%s failed: %s (%s:%d)", what, hipGetErrorString(e), file, line);
  return (e == hipErrorOutOfMemory) ? VGX_ENOMEM : VGX_EDEVICE;
}

// Failure injection for tests of the error paths: with VGX_FAIL_ALLOC=k in
// the environment, the k-th allocation (device or pinned host) counted from
// the last change of that variable fails with VGX_ENOMEM.
static bool injected_failure() {
  static std::mutex mu;
  static std::string last;
  static long count = 0;
  const char* v = getenv("VGX_FAIL_ALLOC");
  std::lock_guard<std::mutex> lock(mu);
  const std::string cur = v ? v : "";
  if (cur != last) {
    last = cur;
    count = 0;
  }
  if (cur.empty()) return false;
  const long k = strtol(cur.c_str(), nullptr, 10);
  return k > 0 && ++count == k;
}

vgx_status dev_alloc(void** p, size_t bytes) {
  *p = nullptr;
  if (injected_failure()) {
    set_error("hipMalloc(%zu): failure injected by VGX_FAIL_ALLOC", bytes);
    return VGX_ENOMEM;
  }
  if (bytes == 0) bytes = 16;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    set_error("hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    return VGX_ENOMEM;
  }
  return VGX_OK;
}

vgx_status host_alloc(void** p, size_t bytes) {
  *p = nullptr;
  if (injected_failure()) {
    set_error("hipHostMalloc(%zu): failure injected by VGX_FAIL_ALLOC", bytes);
    return VGX_ENOMEM;
  }
  hipError_t e = hipHostMalloc(p, bytes ? bytes : 16, hipHostMallocDefault);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    set_error("hipHostMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    return VGX_ENOMEM;
  }
  return VGX_OK;
}

int device_cus() {
  static thread_local int cache_dev = -1, cache_cus = 0;
  int dev = 0;
  hipGetDevice(&dev);
  if (dev != cache_dev) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
    cache_dev = dev;
    cache_cus = cus;
  }
  return cache_cus;
}

}  // namespace vgx

extern "C" const char* vgx_last_error(void) { return vgx::g_err; }

extern "C" const char* vgx_version(void) { return "vgx 0.1 (gfx950)"; }
