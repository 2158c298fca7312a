// common.h — status handling, HIP checks and small device helpers shared by
// the libmwalk translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdarg>
#include <cstdio>
#include <string>

#include "../../include/libmwalk.h"

namespace mw {

// Thread-local message of the last failure (mw_last_error).
void set_error(const char* fmt, ...);
void clear_error();

struct Fail {
    mw_status code;
};

#define MW_REQUIRE(cond, code, ...)          \
    do {                                     \
        if (!(cond)) {                       \
            ::mw::set_error(__VA_ARGS__);    \
            throw ::mw::Fail{code};          \
        }                                    \
    } while (0)

#define MW_HIP(call)                                                                             \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess) {                                                                  \
            ::mw::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__,     \
                            __LINE__);                                                           \
            throw ::mw::Fail{e_ == hipErrorOutOfMemory ? MW_ENOMEM : MW_EDEVICE};                \
        }                                                                                        \
    } while (0)

// Runs body, maps failures to status codes; nothing escapes the C ABI.
template <class F>
mw_status guarded(F&& body) {
    try {
        clear_error();
        body();
        return MW_OK;
    } catch (const Fail& f) {
        return f.code;
    } catch (const std::bad_alloc&) {
        set_error("host allocation failed");
        return MW_ENOMEM;
    } catch (...) {
        set_error("unexpected internal error");
        return MW_EDEVICE;
    }
}

// Optional fault injection for allocation-failure tests:
// MWALK_FAULT=alloc:<k> makes the k-th device allocation (1-based) fail.
bool inject_alloc_failure();

// Device address of the static scratch of mw_transition_noalloc on the
// current device (looked up on the first call per device).
char* noalloc_scratch();

// Tuned FRW walker geometry (resident waves per CU) for lattice size n and
// MicroWalk-E factor m (0 = off), from this process or MWALK_TUNE_CACHE.
bool frw_tuned_waves(int n, int expand_m, int* waves);
void frw_store_waves(int n, int expand_m, int waves);

// Device allocation helpers (throw Fail on error).
void* dev_alloc(size_t bytes);
void dev_free(void* p);

// Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11).  Ten rounds; each
// round multiplies counter words 0 and 2 by the round multipliers, mixes the
// high products with the other two words and the round key, and the key
// advances by the Weyl increments.  Key words are wave-uniform, so the key
// schedule runs on the scalar unit.
struct Rand4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ Rand4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                          uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t m0 = (uint64_t)c0 * 0xD2511F53u;
        const uint64_t m2 = (uint64_t)c2 * 0xCD9E8D57u;
        const uint32_t n0 = (uint32_t)(m2 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(m0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)m2;
        c3 = (uint32_t)m0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return Rand4{c0, c1, c2, c3};
}

// Global-memory views.  Pointers loaded from device structs are generic;
// reading through them emits flat instructions, which also count against the
// LDS wait counter, so a wait for an LDS read would stall on every global
// access in flight.  Kernels that mix LDS and global accesses read and write
// global data through these address-space-1 views.  HIP's vector structs are
// class types whose copy constructors take generic references, so 16-byte
// values move through the builtin vector types below.
#define GAS __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ const GAS T* gp(const T* p) {
    return (const GAS T*)p;
}
template <class T>
__device__ __forceinline__ GAS T* gpw(T* p) {
    return (GAS T*)p;
}
typedef float gvec4 __attribute__((ext_vector_type(4)));
typedef unsigned int guvec4 __attribute__((ext_vector_type(4)));

enum : uint32_t { PURPOSE_MICROWALK = 0, PURPOSE_GAUSS = 1, PURPOSE_FIRST = 2, PURPOSE_TABLE = 3 };

__device__ __forceinline__ uint32_t ctr_hi(uint64_t walk, uint32_t purpose) {
    return (uint32_t)((walk >> 32) & 0xffffffu) | (purpose << 24);
}

// T = ceil(S * 2^32 / S5) for 0 < S < S5 < 2^32, in 64-bit integers (table
// preparation only; the walk steps compare mulhi(u, S5) with S instead).
__device__ __forceinline__ uint32_t ceil_threshold(uint64_t S, uint64_t S5) {
    return (uint32_t)(((S << 32) + S5 - 1) / S5);
}

}  // namespace mw
