// ABI metadata entry points and the per-thread HIP error record.
#include "common.hpp"

namespace tsne {
static thread_local int g_last_hip_error = 0;
void set_last_hip_error(hipError_t e) { g_last_hip_error = int(e); }
}  // namespace tsne

extern "C" int tsne_abi_version(void) { return TSNE_ABI_VERSION; }

extern "C" const char* tsne_status_string(int status) {
  switch (status) {
    case TSNE_OK: return "ok";
    case TSNE_ERR_INVALID_ARG: return "invalid argument";
    case TSNE_ERR_UNSUPPORTED: return "unsupported size or mode";
    case TSNE_ERR_WORKSPACE: return "workspace too small";
    case TSNE_ERR_HIP: return "HIP launch error";
    default: return "unknown status";
  }
}

extern "C" int tsne_last_hip_error(void) { return tsne::g_last_hip_error; }
