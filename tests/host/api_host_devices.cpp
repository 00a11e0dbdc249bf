// Number of HIP devices (0 when there is none or the runtime cannot start),
// for the host API test: it reaches the device only where there is none.
#include <hip/hip_runtime_api.h>

extern "C" int hip_device_count(void) {
    int n = 0;
    return hipGetDeviceCount(&n) == hipSuccess ? n : 0;
}
