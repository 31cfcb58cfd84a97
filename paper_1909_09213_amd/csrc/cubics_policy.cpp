// Learned branching policy objects (weights resident on the device).
#include <hip/hip_runtime.h>

#include <cstring>

#include "../../include/cubics.h"
#include "cubics_internal.h"

using namespace cubics;

struct cubics_policy {
    PolicyDev dev;
};

int policy_fill(const cubics_policy *pol, PolicyDev *out) {
    *out = pol->dev;
    return 0;
}
