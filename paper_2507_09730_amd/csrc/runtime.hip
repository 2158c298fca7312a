// runtime.hip — error state, allocation and device selection for libmwalk.
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

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

// Device blocks are cached by (device, exact size) after they are freed, so
// that repeated calls of the same shape (one extraction after another) do not
// pay hipMalloc and the synchronising hipFree each time.  A freed block keeps
// an event recorded on the null stream at release; it is handed out again
// only after that event has completed, so work still queued on it (an error
// path that unwinds before synchronising) finishes first.  At most CACHE_CAP
// bytes are kept; larger releases go back to the runtime.
namespace {
constexpr size_t CACHE_CAP = size_t(4) << 30;
struct Cached {
    void* p;
    hipEvent_t done;
};
struct BlockCache {
    std::mutex mu;
    std::map<std::pair<int, size_t>, std::vector<Cached>> free_blocks;
    std::map<void*, std::pair<int, size_t>> live;
    size_t cached = 0;
};
BlockCache& block_cache() {
    static BlockCache* c = new BlockCache();  // outlives static destruction order
    return *c;
}
}  // namespace

void* dev_alloc(size_t bytes) {
    if (bytes == 0) bytes = 256;
    MW_REQUIRE(!inject_alloc_failure(), MW_ENOMEM, "injected device allocation failure (%zu bytes)", bytes);
    int dev = 0;
    MW_HIP(hipGetDevice(&dev));
    BlockCache& C = block_cache();
    {
        std::lock_guard<std::mutex> g(C.mu);
        auto it = C.free_blocks.find({dev, bytes});
        if (it != C.free_blocks.end() && !it->second.empty()) {
            const Cached b = it->second.back();
            it->second.pop_back();
            C.cached -= bytes;
            C.live[b.p] = {dev, bytes};
            if (b.done) {
                (void)hipEventSynchronize(b.done);
                (void)hipEventDestroy(b.done);
            }
            return b.p;
        }
    }
    void* p = nullptr;
    MW_HIP(hipMalloc(&p, bytes));
    std::lock_guard<std::mutex> g(C.mu);
    C.live[p] = {dev, bytes};
    return p;
}

void dev_free(void* p) {
    if (!p) return;
    BlockCache& C = block_cache();
    {
        std::lock_guard<std::mutex> g(C.mu);
        auto it = C.live.find(p);
        if (it != C.live.end()) {
            const auto key = it->second;
            C.live.erase(it);
            if (C.cached + key.second <= CACHE_CAP) {
                hipEvent_t ev = nullptr;
                if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) ev = nullptr;
                if (ev && hipEventRecord(ev, 0) != hipSuccess) {
                    (void)hipEventDestroy(ev);
                    ev = nullptr;
                    (void)hipDeviceSynchronize();
                }
                C.free_blocks[key].push_back(Cached{p, ev});
                C.cached += key.second;
                return;
            }
        }
    }
    (void)hipFree(p);
}

}  // namespace mw

extern "C" const char* mw_last_error(void) { return mw::g_err.c_str(); }

extern "C" mw_status mw_init(int32_t device) {
    return mw::guarded([&] {
        int count = 0;
        MW_HIP(hipGetDeviceCount(&count));
        MW_REQUIRE(device >= 0 && device < count, MW_EINVAL, "device %d out of range (%d devices)", device, count);
        MW_HIP(hipSetDevice(device));
        // the device address of mw_transition_noalloc's static scratch
        (void)mw::noalloc_scratch();
    });
}
