// common.hpp -- internal helpers shared by the library's translation units:
// error reporting, value-type traits, launch geometry.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include <cstdio>
#include <string>

#include "../../include/spx.h"

namespace spx {

// Thread-local last error text (spx_last_error).
void set_error(const char *fmt, ...) __attribute__((format(printf, 1, 2)));
void clear_error();

#define SPX_REQUIRE(cond, status, ...)        \
    do {                                      \
        if (!(cond)) {                        \
            ::spx::set_error(__VA_ARGS__);    \
            return (status);                  \
        }                                     \
    } while (0)

#define SPX_HIP(call)                                                                  \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess) {                                                        \
            ::spx::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_),    \
                             __FILE__, __LINE__);                                      \
            return SPX_ERR_HIP;                                                        \
        }                                                                              \
    } while (0)

#define SPX_LAUNCHED()                                                                 \
    do {                                                                               \
        hipError_t e_ = hipGetLastError();                                             \
        if (e_ != hipSuccess) {                                                        \
            ::spx::set_error("kernel launch failed: %s (%s:%d)", hipGetErrorString(e_), \
                             __FILE__, __LINE__);                                      \
            return SPX_ERR_HIP;                                                        \
        }                                                                              \
    } while (0)

#define SPX_CHECK(...)                     \
    do {                                   \
        spx_status s_ = (__VA_ARGS__);     \
        if (s_ != SPX_OK) return s_;       \
    } while (0)

// Stored value type -> arithmetic type. binary16 values are widened to float.
template <typename V>
struct acc_of;
template <>
struct acc_of<double> {
    using type = double;
};
template <>
struct acc_of<float> {
    using type = float;
};
template <>
struct acc_of<_Float16> {
    using type = float;
};

template <typename V>
__device__ __forceinline__ typename acc_of<V>::type widen(V v)
{
    return static_cast<typename acc_of<V>::type>(v);
}

// Streaming (read-once) loads: non-temporal so that the matrix stream does
// not evict the gathered vector from the caches.
template <typename T>
__device__ __forceinline__ T ld_stream(const T *p)
{
    return __builtin_nontemporal_load(p);
}

// gfx950: 8 XCDs, work-groups are dealt to them round robin. Remap a linear
// block id so that each XCD receives a contiguous range of logical blocks
// (keeps the gathered vector entries of neighbouring rows in one L2).
constexpr int kXcds = 8;

__device__ __forceinline__ int64_t xcd_remap(int64_t bid, int64_t nblocks_padded)
{
    const int64_t per = nblocks_padded / kXcds;
    return (bid % kXcds) * per + bid / kXcds;
}

inline int64_t pad_to_xcds(int64_t nblocks) { return ((nblocks + kXcds - 1) / kXcds) * kXcds; }

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace spx
