// Library-level entry points: version and status strings.
#include "aps_common.h"

extern "C" {

int aps_version(void) { return 1 * 10000 + 0 * 100 + 0; }

const char* aps_status_string(int status) {
  switch (status) {
    case APS_OK: return "ok";
    case APS_ERR_NULL: return "a required pointer is NULL";
    case APS_ERR_SHAPE: return "inconsistent or unsupported sizes";
    case APS_ERR_UNSUPPORTED: return "no compiled kernel for this configuration";
    case APS_ERR_WORKSPACE: return "workspace missing or too small";
    case APS_ERR_HIP: return "HIP runtime error";
    case APS_ERR_ARG: return "scalar argument out of range";
    case APS_ERR_TOO_LARGE: return "problem larger than the static scratch of a no-allocation entry point";
    default: return "unknown status";
  }
}

}  // extern "C"
