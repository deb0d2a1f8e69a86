// Status strings of the C ABI (include/wsm.h).
#include "wsm_internal.h"

extern "C" const char *wsm_status_string(int status) {
    switch (status) {
        case WSM_OK: return "ok";
        case WSM_EINVAL: return "invalid argument";
        case WSM_ENOSPC: return "workspace, state or output capacity too small";
        case WSM_EHIP: return "HIP launch or device query failed";
        default: return "unknown status";
    }
}
