// Status strings and version of the C ABI.
#include "common.h"

extern "C" const char *lsrvt_status_string(int32_t status) {
  switch (status) {
    case LSRVT_OK: return "ok";
    case LSRVT_EINVAL: return "invalid argument";
    case LSRVT_ENAN: return "field contains NaN";
    case LSRVT_ECAPACITY: return "output table capacity exceeded";
    case LSRVT_EWORKSPACE: return "workspace missing, misaligned or too small";
    case LSRVT_ELIMIT: return "volume exceeds size limits";
    case LSRVT_EDEVICE: return "HIP device or launch error";
    default: return "unknown status";
  }
}

extern "C" int32_t lsrvt_version(void) { return 100; }
