// Status strings, thread-local error detail and cached device facts.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <mutex>

#include "common.h"

namespace emri {

static thread_local char g_last_error[512] = "";

int fail(int status, const char *fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_last_error, sizeof g_last_error, fmt, ap);
  va_end(ap);
  return status;
}

void clear_error() { g_last_error[0] = '\0'; }

int device_cu_count(int *out) {
  static std::mutex mu;
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
    return fail(EMRI_EDEVICE, "hipGetDevice failed");
  std::lock_guard<std::mutex> lock(mu);
  if (cached[dev] == 0) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
      return fail(EMRI_EDEVICE, "cannot query the compute-unit count of device %d", dev);
    cached[dev] = cus;
  }
  *out = cached[dev];
  return EMRI_OK;
}

}  // namespace emri

extern "C" const char *emri_status_string(int status) {
  switch (status) {
    case EMRI_OK: return "EMRI_OK";
    case EMRI_EINVAL: return "EMRI_EINVAL: invalid argument";
    case EMRI_ERANGE: return "EMRI_ERANGE: size overflow";
    case EMRI_ENOMEM: return "EMRI_ENOMEM: workspace too small";
    case EMRI_EDEVICE: return "EMRI_EDEVICE: HIP error";
    case EMRI_EUNSUPPORTED: return "EMRI_EUNSUPPORTED: not supported by this library";
    default: return "unknown emri status";
  }
}

extern "C" const char *emri_last_error(void) { return emri::g_last_error; }
