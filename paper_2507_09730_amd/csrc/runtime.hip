// runtime.hip — error state, allocation and device selection for libmwalk.
#include <cstdlib>
#include <cstring>
#include <mutex>

#include "common.h"

namespace mw {

static thread_local std::string g_err;

void set_error(const char* fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
}

void clear_error() { g_err.clear(); }

static std::mutex g_fault_mu;
static long g_alloc_count = 0;

bool inject_alloc_failure() {
    const char* f = getenv("MWALK_FAULT");
    if (!f || strncmp(f, "alloc:", 6) != 0) return false;
    long k = atol(f + 6);
    std::lock_guard<std::mutex> g(g_fault_mu);
    ++g_alloc_count;
    return g_alloc_count == k;
}

void* dev_alloc(size_t bytes) {
    if (bytes == 0) bytes = 256;
    MW_REQUIRE(!inject_alloc_failure(), MW_ENOMEM, "injected device allocation failure (%zu bytes)", bytes);
    void* p = nullptr;
    MW_HIP(hipMalloc(&p, bytes));
    return p;
}

void dev_free(void* p) {
    if (p) (void)hipFree(p);
}

}  // namespace mw

extern "C" const char* mw_last_error(void) { return mw::g_err.c_str(); }

extern "C" mw_status mw_init(int32_t device) {
    return mw::guarded([&] {
        int count = 0;
        MW_HIP(hipGetDeviceCount(&count));
        MW_REQUIRE(device >= 0 && device < count, MW_EINVAL, "device %d out of range (%d devices)", device, count);
        MW_HIP(hipSetDevice(device));
    });
}
