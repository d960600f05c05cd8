// Fill and exclusive-scan kernels (int32).  The scan is three passes over tiles of
// kScanItems * 256 elements: per-tile sums, a single-block scan of the tile sums, then the
// per-tile scan that adds the tile prefix.  out has n + 1 entries: out[n] is the total.
#include "fof_internal.h"

namespace fof {

namespace {

constexpr int kScanBlock = 256;
constexpr int64_t kTile = (int64_t)kScanBlock * kScanItems;

template <typename T>
__global__ void k_fill(T *__restrict__ p, int64_t n, T v)
{
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = gtid(); i < n; i += stride)
        p[i] = v;
}

struct LoadI32 {
    const int32_t *p;
    __device__ int32_t operator()(int64_t i) const { return p[i]; }
};

struct LoadNonNeg {
    const int32_t *p;
    __device__ int32_t operator()(int64_t i) const { return max(p[i], 0); }
};

struct LoadNonZero {
    const int32_t *p;
    __device__ int32_t operator()(int64_t i) const { return p[i] != 0 ? 1 : 0; }
};

// Roots of kept components in per-sample forests laid out [K][vcap]: entry (k, v) counts
// when v is below the device count *nv, is its tree's root and has at least min_size members.
struct LoadSampleKeep {
    const int32_t *forest, *cnt, *nv;
    int64_t vcap;
    int32_t min_size;
    __device__ int32_t operator()(int64_t i) const
    {
        const int64_t v = i % vcap;
        return (v < *nv && forest[i] == (int32_t)v && cnt[i] >= min_size) ? 1 : 0;
    }
};

struct LoadPopc {
    const uint32_t *p;
    __device__ int32_t operator()(int64_t i) const { return __popc(p[i]); }
};

// Block-wide exclusive scan of one value per thread; returns the block total in *total.
__device__ int32_t block_exclusive_scan(int32_t v, int32_t *total)
{
    __shared__ int32_t wsum[kScanBlock / kWave];
    const int lane = lane_id(), wid = threadIdx.x / kWave;
    int32_t x = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        int32_t y = __shfl_up(x, o, kWave);
        if (lane >= o)
            x += y;
    }
    if (lane == kWave - 1)
        wsum[wid] = x;
    __syncthreads();
    int32_t wpre = 0, tot = 0;
    for (int k = 0; k < kScanBlock / kWave; ++k) {
        int32_t s = wsum[k];
        if (k < wid)
            wpre += s;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return wpre + x - v;
}

template <typename Load>
__global__ __launch_bounds__(kScanBlock) void k_tile_sums(Load ld, int64_t n,
                                                          int32_t *__restrict__ tsum)
{
    const int64_t base = (int64_t)blockIdx.x * kTile;
    int32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + (int64_t)k * kScanBlock + threadIdx.x;  // coalesced
        if (i < n)
            s += ld(i);
    }
    int32_t tot;
    block_exclusive_scan(s, &tot);
    if (threadIdx.x == 0)
        tsum[blockIdx.x] = tot;
}

// Single block: exclusive scan of the tile sums in place; tsum[ntiles] = grand total.
__global__ __launch_bounds__(kScanBlock) void k_scan_tile_sums(int32_t *__restrict__ tsum,
                                                               int64_t ntiles)
{
    int32_t carry = 0;
    for (int64_t base = 0; base < ntiles; base += kScanBlock) {
        int64_t i = base + threadIdx.x;
        int32_t v = i < ntiles ? tsum[i] : 0;
        int32_t tot;
        int32_t ex = block_exclusive_scan(v, &tot);
        if (i < ntiles)
            tsum[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0)
        tsum[ntiles] = carry;
}

template <typename Load>
__global__ __launch_bounds__(kScanBlock) void k_scan_tiles(Load ld, int64_t n,
                                                           const int32_t *__restrict__ tsum,
                                                           int32_t *__restrict__ out,
                                                           int64_t ntiles)
{
    // Each thread owns kScanItems consecutive elements of the tile.
    const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kScanItems;
    int32_t v[kScanItems];
    int32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + k;
        v[k] = i < n ? ld(i) : 0;
        s += v[k];
    }
    int32_t tot;
    int32_t ex = block_exclusive_scan(s, &tot) + tsum[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + k;
        if (i < n)
            out[i] = ex;
        ex += v[k];
    }
    if (blockIdx.x == ntiles - 1 && threadIdx.x == 0)
        out[n] = tsum[ntiles];
}

template <typename Load>
hipError_t scan_impl(Load ld, int32_t *out, int64_t n, int32_t *scratch, hipStream_t s)
{
    if (n <= 0) {
        hipLaunchKernelGGL(k_fill<int32_t>, dim3(1), dim3(64), 0, s, out, (int64_t)1, 0);
        return hipGetLastError();
    }
    int64_t ntiles = (n + kTile - 1) / kTile;
    hipLaunchKernelGGL(k_tile_sums<Load>, dim3((unsigned)ntiles), dim3(kScanBlock), 0, s, ld, n,
                       scratch);
    hipLaunchKernelGGL(k_scan_tile_sums, dim3(1), dim3(kScanBlock), 0, s, scratch, ntiles);
    hipLaunchKernelGGL(k_scan_tiles<Load>, dim3((unsigned)ntiles), dim3(kScanBlock), 0, s, ld,
                       n, scratch, out, ntiles);
    return hipGetLastError();
}

unsigned fill_blocks(int64_t n)
{
    int64_t b = (n + 1023) / 1024;
    if (b > 65536)
        b = 65536;
    return (unsigned)(b > 0 ? b : 1);
}

}  // namespace

int64_t scan_scratch_elems(int64_t n) { return (n + kTile - 1) / kTile + 1; }

hipError_t launch_scan_i32(const int32_t *in, int32_t *out, int64_t n, int32_t *scratch,
                           hipStream_t s)
{
    return scan_impl(LoadI32{in}, out, n, scratch, s);
}

hipError_t launch_scan_nonneg(const int32_t *in, int32_t *out, int64_t n, int32_t *scratch,
                              hipStream_t s)
{
    return scan_impl(LoadNonNeg{in}, out, n, scratch, s);
}

hipError_t launch_scan_nonzero(const int32_t *in, int32_t *out, int64_t n, int32_t *scratch,
                               hipStream_t s)
{
    return scan_impl(LoadNonZero{in}, out, n, scratch, s);
}

hipError_t launch_scan_sample_keep(const int32_t *forest, const int32_t *cnt, const int32_t *nv,
                                   int64_t vcap, int32_t K, int32_t min_size, int32_t *out,
                                   int32_t *scratch, hipStream_t s)
{
    return scan_impl(LoadSampleKeep{forest, cnt, nv, vcap, min_size}, out, (int64_t)K * vcap,
                     scratch, s);
}

hipError_t launch_scan_popc(const uint32_t *in, int32_t *out, int64_t n, int32_t *scratch,
                            hipStream_t s)
{
    return scan_impl(LoadPopc{in}, out, n, scratch, s);
}

hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_fill<int32_t>, dim3(fill_blocks(n)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_fill<uint32_t>, dim3(fill_blocks(n)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_u64(uint64_t *p, int64_t n, uint64_t v, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_fill<uint64_t>, dim3(fill_blocks(n)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_f64(double *p, int64_t n, double v, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_fill<double>, dim3(fill_blocks(n)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

}  // namespace fof
