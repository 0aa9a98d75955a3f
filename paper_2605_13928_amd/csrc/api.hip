// ABI metadata entry points and the per-thread HIP error record.
#include "common.hpp"

#include <atomic>
#include <cstring>

namespace tsne {
static thread_local int g_last_hip_error = 0;
void set_last_hip_error(hipError_t e) { g_last_hip_error = int(e); }

// Per device ordinal: 0 = not queried yet, else the status to return.
constexpr int MAX_CACHED_DEVICES = 64;
static std::atomic<int> g_device_status[MAX_CACHED_DEVICES];

static int query_device(int dev) {
  hipDeviceProp_t prop;
  const hipError_t e = hipGetDeviceProperties(&prop, dev);
  if (e != hipSuccess) {
    set_last_hip_error(e);
    return TSNE_ERR_HIP;
  }
  // gcnArchName is "gfx950" followed by optional target features (":sramecc+:xnack-")
  const char* a = prop.gcnArchName;
  const bool ok = std::strncmp(a, "gfx950", 6) == 0 && (a[6] == '\0' || a[6] == ':');
  return ok ? TSNE_OK : TSNE_ERR_UNSUPPORTED;
}

int require_gfx950() {
  int dev = -1;
  const hipError_t e = hipGetDevice(&dev);
  if (e == hipErrorNoDevice || e == hipErrorInsufficientDriver) return TSNE_ERR_UNSUPPORTED;
  if (e != hipSuccess) {
    set_last_hip_error(e);
    return TSNE_ERR_HIP;
  }
  if (dev < 0 || dev >= MAX_CACHED_DEVICES) return query_device(dev);
  int st = g_device_status[dev].load(std::memory_order_acquire);
  if (st == 0) {
    st = query_device(dev) + 1;  // stored shifted so that TSNE_OK is not 0
    if (st - 1 == TSNE_ERR_HIP) return TSNE_ERR_HIP;  // not cached: may succeed later
    g_device_status[dev].store(st, std::memory_order_release);
  }
  return st - 1;
}
}  // namespace tsne

extern "C" int tsne_abi_version(void) { return TSNE_ABI_VERSION; }

extern "C" const char* tsne_status_string(int status) {
  switch (status) {
    case TSNE_OK: return "ok";
    case TSNE_ERR_INVALID_ARG: return "invalid argument";
    case TSNE_ERR_UNSUPPORTED: return "unsupported size, mode or device (the library runs on gfx950 only)";
    case TSNE_ERR_WORKSPACE: return "workspace too small";
    case TSNE_ERR_HIP: return "HIP launch error";
    case TSNE_ERR_NONFINITE: return "non-finite (NaN or infinite) input coordinates";
    case TSNE_ERR_SCRATCH: return "problem too large for the static scratch of the allocation-free entry point";
    default: return "unknown status";
  }
}

extern "C" int tsne_last_hip_error(void) { return tsne::g_last_hip_error; }
