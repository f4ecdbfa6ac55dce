// prims.hip -- entry points exposing the wavefront primitives of wave.hpp
// (the subwarp cooperative-group operations of Section 3.3) and a streaming
// copy used as the attainable-bandwidth reference of the SpMV measurements.
#include "common.hpp"
#include "wave.hpp"

namespace spx {

constexpr int kPrimThreads = 256;

// The paper's reduction benchmark kernel: each thread loads one value and
// applies `inner_loops` subwarp reductions to its running value.
template <int Size>
__global__ __launch_bounds__(kPrimThreads) void subwarp_sum_kernel(const double *__restrict__ in,
                                                                  double *__restrict__ out, int64_t n,
                                                                  int inner_loops)
{
    const int64_t t = (int64_t)blockIdx.x * kPrimThreads + threadIdx.x;
    // n is a multiple of 64, so a wavefront is either wholly in range or wholly out.
    if (t - lane_id() >= n) return;
    double v = in[t];
    for (int i = 0; i < inner_loops; ++i) v = subwave_sum<Size>(v);
    out[t] = v;
}

template <int Size>
__global__ __launch_bounds__(kPrimThreads) void subwarp_vote_kernel(const int32_t *__restrict__ pred,
                                                                   uint64_t *__restrict__ ballot,
                                                                   int32_t *__restrict__ any,
                                                                   int32_t *__restrict__ all, int64_t n)
{
    const int64_t t = (int64_t)blockIdx.x * kPrimThreads + threadIdx.x;
    if (t - lane_id() >= n) return;
    const bool p = pred[t] != 0;
    ballot[t] = subwave<Size>::ballot(p);
    any[t] = subwave<Size>::any(p) ? 1 : 0;
    all[t] = subwave<Size>::all(p) ? 1 : 0;
}

__global__ __launch_bounds__(kPrimThreads) void segscan_kernel(const double *__restrict__ in,
                                                              const int32_t *__restrict__ head,
                                                              double *__restrict__ out, int64_t n)
{
    const int64_t t = (int64_t)blockIdx.x * kPrimThreads + threadIdx.x;
    if (t - lane_id() >= n) return;
    out[t] = wave_segscan(in[t], head[t] != 0);
}

typedef double dvec2 __attribute__((ext_vector_type(2)));

// Streaming copy and read, the attainable-bandwidth references: a work-group
// moves U * 256 consecutive 16-byte vectors, every thread issuing its U
// non-temporal loads (coalesced across the wavefront) before any store; one
// work-group per chunk; stores are plain (non-temporal stores measured no
// faster). Measured on MI355X (1 GiB copied, 2 GiB read): the
// copy is fastest with one vector per thread and many small work-groups
// (U = 1: 6.5 TB/s of reads plus writes; U = 4: 6.0; U = 8: 4.4), the read
// with four (U = 4: 7.2 TB/s; 1, 2, 8 and 16: 6.8-7.1).
constexpr int kCopyU = 1;
constexpr int kReadU = 4;
constexpr int64_t kCopyChunk = (int64_t)kCopyU * kPrimThreads;
constexpr int64_t kReadChunk = (int64_t)kReadU * kPrimThreads;

__global__ __launch_bounds__(kPrimThreads) void stream_copy_kernel(const dvec2 *__restrict__ src,
                                                                  dvec2 *__restrict__ dst, int64_t n2,
                                                                  const double *__restrict__ src1,
                                                                  double *__restrict__ dst1, int64_t n)
{
    const int64_t base = (int64_t)blockIdx.x * kCopyChunk + threadIdx.x;
    dvec2 v[kCopyU];
#pragma unroll
    for (int u = 0; u < kCopyU; ++u) {
        const int64_t i = base + (int64_t)u * kPrimThreads;
        if (i < n2) v[u] = __builtin_nontemporal_load(src + i);
    }
#pragma unroll
    for (int u = 0; u < kCopyU; ++u) {
        const int64_t i = base + (int64_t)u * kPrimThreads;
        if (i < n2) dst[i] = v[u];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && (n & 1)) dst1[n - 1] = src1[n - 1];
}

// Read-only stream: the loaded values are summed and the sum is stored only
// if it equals a value it cannot take for finite data (keeps the loads live).
__global__ __launch_bounds__(kPrimThreads) void stream_read_kernel(const dvec2 *__restrict__ src, int64_t n2,
                                                                  double *__restrict__ sink)
{
    const int64_t base = (int64_t)blockIdx.x * kReadChunk + threadIdx.x;
    dvec2 v[kReadU];
#pragma unroll
    for (int u = 0; u < kReadU; ++u) {
        const int64_t i = base + (int64_t)u * kPrimThreads;
        v[u] = (i < n2) ? __builtin_nontemporal_load(src + i) : dvec2{0.0, 0.0};
    }
    double acc = 0.0;
#pragma unroll
    for (int u = 0; u < kReadU; ++u) acc += v[u].x + v[u].y;
    if (acc == -1.2345678e300) sink[0] = acc;
}

}  // namespace spx

using namespace spx;

#define SPX_SIZE_DISPATCH(SIZE, KERNEL, ...)                                   \
    switch (SIZE) {                                                            \
    case 1: KERNEL<1><<<grid, kPrimThreads, 0, stream>>>(__VA_ARGS__); break;  \
    case 2: KERNEL<2><<<grid, kPrimThreads, 0, stream>>>(__VA_ARGS__); break;  \
    case 4: KERNEL<4><<<grid, kPrimThreads, 0, stream>>>(__VA_ARGS__); break;  \
    case 8: KERNEL<8><<<grid, kPrimThreads, 0, stream>>>(__VA_ARGS__); break;  \
    case 16: KERNEL<16><<<grid, kPrimThreads, 0, stream>>>(__VA_ARGS__); break; \
    case 32: KERNEL<32><<<grid, kPrimThreads, 0, stream>>>(__VA_ARGS__); break; \
    case 64: KERNEL<64><<<grid, kPrimThreads, 0, stream>>>(__VA_ARGS__); break; \
    default: break;                                                            \
    }

static bool pow2_le64(int32_t s) { return s >= 1 && s <= 64 && (s & (s - 1)) == 0; }

extern "C" spx_status spx_subwarp_sum(const double *in, double *out, int64_t n, int32_t size, int32_t inner_loops,
                                      hipStream_t stream)
{
    clear_error();
    SPX_REQUIRE(in && out, SPX_ERR_ARG, "spx_subwarp_sum: null pointer");
    SPX_REQUIRE(n >= 0 && n % kWave == 0, SPX_ERR_ARG, "spx_subwarp_sum: n=%lld is not a multiple of 64", (long long)n);
    SPX_REQUIRE(pow2_le64(size), SPX_ERR_ARG, "spx_subwarp_sum: size=%d is not a power of two <= 64", size);
    SPX_REQUIRE(inner_loops >= 0, SPX_ERR_ARG, "spx_subwarp_sum: inner_loops < 0");
    if (n == 0) return SPX_OK;
    const unsigned grid = (unsigned)ceil_div(n, kPrimThreads);
    SPX_SIZE_DISPATCH(size, subwarp_sum_kernel, in, out, n, inner_loops);
    SPX_LAUNCHED();
    return SPX_OK;
}

extern "C" spx_status spx_subwarp_vote(const int32_t *pred, uint64_t *ballot, int32_t *any, int32_t *all, int64_t n,
                                       int32_t size, hipStream_t stream)
{
    clear_error();
    SPX_REQUIRE(pred && ballot && any && all, SPX_ERR_ARG, "spx_subwarp_vote: null pointer");
    SPX_REQUIRE(n >= 0 && n % kWave == 0, SPX_ERR_ARG, "spx_subwarp_vote: n=%lld is not a multiple of 64", (long long)n);
    SPX_REQUIRE(pow2_le64(size), SPX_ERR_ARG, "spx_subwarp_vote: size=%d is not a power of two <= 64", size);
    if (n == 0) return SPX_OK;
    const unsigned grid = (unsigned)ceil_div(n, kPrimThreads);
    SPX_SIZE_DISPATCH(size, subwarp_vote_kernel, pred, ballot, any, all, n);
    SPX_LAUNCHED();
    return SPX_OK;
}

extern "C" spx_status spx_wave_segscan(const double *in, const int32_t *head, double *out, int64_t n,
                                       hipStream_t stream)
{
    clear_error();
    SPX_REQUIRE(in && head && out, SPX_ERR_ARG, "spx_wave_segscan: null pointer");
    SPX_REQUIRE(n >= 0 && n % kWave == 0, SPX_ERR_ARG, "spx_wave_segscan: n=%lld is not a multiple of 64", (long long)n);
    if (n == 0) return SPX_OK;
    segscan_kernel<<<(unsigned)ceil_div(n, kPrimThreads), kPrimThreads, 0, stream>>>(in, head, out, n);
    SPX_LAUNCHED();
    return SPX_OK;
}

extern "C" spx_status spx_stream_copy(const double *src, double *dst, int64_t n, hipStream_t stream)
{
    clear_error();
    SPX_REQUIRE(src && dst, SPX_ERR_ARG, "spx_stream_copy: null pointer");
    SPX_REQUIRE(n >= 0, SPX_ERR_ARG, "spx_stream_copy: n < 0");
    SPX_REQUIRE((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) % 16 == 0, SPX_ERR_ARG,
                "spx_stream_copy: pointers must be 16-byte aligned");
    if (n == 0) return SPX_OK;
    const int64_t n2 = n / 2;
    const int64_t grid = ceil_div(n2 > 0 ? n2 : 1, kCopyChunk);
    SPX_REQUIRE(grid <= INT32_MAX, SPX_ERR_ARG, "spx_stream_copy: n too large");
    stream_copy_kernel<<<(unsigned)grid, kPrimThreads, 0, stream>>>(reinterpret_cast<const dvec2 *>(src),
                                                                   reinterpret_cast<dvec2 *>(dst), n2, src, dst, n);
    SPX_LAUNCHED();
    return SPX_OK;
}

extern "C" spx_status spx_stream_read(const double *src, int64_t n, double *sink, hipStream_t stream)
{
    clear_error();
    SPX_REQUIRE(src && sink, SPX_ERR_ARG, "spx_stream_read: null pointer");
    SPX_REQUIRE(n >= 0 && n % 2 == 0, SPX_ERR_ARG, "spx_stream_read: n must be even and >= 0");
    SPX_REQUIRE(reinterpret_cast<uintptr_t>(src) % 16 == 0, SPX_ERR_ARG, "spx_stream_read: src must be 16-byte aligned");
    if (n == 0) return SPX_OK;
    const int64_t n2 = n / 2;
    const int64_t grid = ceil_div(n2, kReadChunk);
    SPX_REQUIRE(grid <= INT32_MAX, SPX_ERR_ARG, "spx_stream_read: n too large");
    stream_read_kernel<<<(unsigned)grid, kPrimThreads, 0, stream>>>(reinterpret_cast<const dvec2 *>(src), n2, sink);
    SPX_LAUNCHED();
    return SPX_OK;
}
