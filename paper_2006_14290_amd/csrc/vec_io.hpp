// vec_io.hpp -- per-thread access to kVecItems (4) consecutive vector
// entries: one 32-byte (float64) or 16-byte (float32) load/store when the
// pointers allow it and the group lies inside [0, n), else entry by entry
// with entries past n reading as 0 and never written.
#pragma once

#include <initializer_list>

#include "solver_common.hpp"

namespace spx {

template <typename X>
using vec4_t = X __attribute__((ext_vector_type(kVecItems)));

template <typename X, bool kVec>
__device__ __forceinline__ vec4_t<X> ld4(const X *__restrict__ p, int64_t i0, int64_t n)
{
    if (kVec && i0 + kVecItems <= n) return *reinterpret_cast<const vec4_t<X> *>(p + i0);
    vec4_t<X> v = {};
#pragma unroll
    for (int u = 0; u < kVecItems; ++u)
        if (i0 + u < n) v[u] = p[i0 + u];
    return v;
}

template <typename X, bool kVec>
__device__ __forceinline__ void st4(X *__restrict__ p, int64_t i0, int64_t n, const vec4_t<X> &v)
{
    if (kVec && i0 + kVecItems <= n) {
        *reinterpret_cast<vec4_t<X> *>(p + i0) = v;
        return;
    }
#pragma unroll
    for (int u = 0; u < kVecItems; ++u)
        if (i0 + u < n) p[i0 + u] = v[u];
}

// First entry of this thread's group (groups of kVecItems, kVecThreads
// threads per work-group, vec_blocks(n) work-groups).
__device__ __forceinline__ int64_t vec_i0() { return ((int64_t)blockIdx.x * kVecThreads + threadIdx.x) * kVecItems; }

// True when every pointer is aligned for whole-group loads.
template <typename X>
inline bool vec_aligned(std::initializer_list<const void *> ptrs)
{
    for (const void *p : ptrs)
        if (p != nullptr && reinterpret_cast<uintptr_t>(p) % (kVecItems * sizeof(X)) != 0) return false;
    return true;
}

}  // namespace spx
