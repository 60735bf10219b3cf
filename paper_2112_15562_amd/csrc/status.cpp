// Status codes and the per-thread last-error message of the C ABI.
#include <hip/hip_runtime.h>

#include <string>

#include "common.h"

namespace bttb {

static thread_local std::string g_last_error;

int fail(int status, const std::string& msg) {
  g_last_error = msg;
  return status;
}

int hip_fail(hipError_t e, const char* what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return BTTB_EHIP;
}

}  // namespace bttb

extern "C" const char* bttb_strerror(int status) {
  switch (status) {
    case BTTB_OK: return "ok";
    case BTTB_EINVAL: return "invalid argument";
    case BTTB_ENOMEM: return "out of device memory";
    case BTTB_EHIP: return "HIP runtime error";
    case BTTB_ESIZE: return "size out of range";
    case BTTB_ESTATE: return "incompatible state";
    case BTTB_ENAN: return "non-finite value";
    default: return "unknown status";
  }
}

extern "C" const char* bttb_last_error(void) { return bttb::g_last_error.c_str(); }
