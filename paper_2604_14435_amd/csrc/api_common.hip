// Status strings, error reporting and small entry points of the C ABI.
#include <mutex>
#include <unordered_map>

#include "common.h"

namespace dvq {

static thread_local char g_last_error[512] = "no error";

dvq_status fail(dvq_status s, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
    va_end(ap);
    return s;
}

hipError_t allow_lds(const void* kernel, size_t bytes) {
    // The attribute is per kernel and per device; remember the largest value
    // set so far so repeated calls cost nothing.
    static std::mutex mu;
    static std::unordered_map<const void*, size_t> done;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const void* key = reinterpret_cast<const char*>(kernel) + dev;  // per device
    std::lock_guard<std::mutex> lock(mu);
    auto it = done.find(key);
    if (it != done.end() && it->second >= bytes) return hipSuccess;
    if (bytes <= 64 * 1024) {
        done[key] = bytes;
        return hipSuccess;
    }
    e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e == hipSuccess) done[key] = bytes;
    return e;
}

}  // namespace dvq

extern "C" {

const char* dvq_status_string(dvq_status s) {
    switch (s) {
        case DVQ_OK: return "DVQ_OK";
        case DVQ_EINVAL: return "DVQ_EINVAL: invalid argument";
        case DVQ_ECAPACITY: return "DVQ_ECAPACITY: output capacity or workspace too small";
        case DVQ_ENOMEM: return "DVQ_ENOMEM: out of memory";
        case DVQ_EDEVICE: return "DVQ_EDEVICE: HIP runtime error";
        case DVQ_EUNSUPPORTED: return "DVQ_EUNSUPPORTED: not supported by this build";
        case DVQ_ENONFINITE: return "DVQ_ENONFINITE: non-finite result";
        default: return "unknown dvq_status";
    }
}

const char* dvq_last_error(void) { return dvq::g_last_error; }

const char* dvq_version(void) { return "dvq 0.1.0 gfx950"; }

int64_t dvq_circuit_count(int32_t n, int32_t L, int32_t cost_kind) {
    if (n < 1 || L < 1) return 0;
    const int64_t l2 = (int64_t)L * L;
    return cost_kind == DVQ_COST_LOCAL ? 2 * (int64_t)(n + 1) * l2 : 2 * (l2 + L);
}

}  // extern "C"
