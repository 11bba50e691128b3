// Status strings and version of libutcompass.
#include "common.hpp"

extern "C" const char* utc_status_string(int status)
{
  switch (status) {
    case UTC_OK: return "ok";
    case UTC_ERR_ARG: return "invalid argument";
    case UTC_ERR_WORKSPACE: return "workspace missing or too small";
    case UTC_ERR_HIP: return "HIP launch failed";
    default: return "unknown status";
  }
}

extern "C" const char* utc_version(void) { return "utcompass 0.1 gfx950"; }
