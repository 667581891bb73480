// Device-wide exclusive scans and fills (building blocks of every compaction
// step: kept-pair offsets, output-slot assignment, octree node lists).
#include "common.hpp"

namespace spamm {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;  // 2048 items per block
constexpr int kScanMaxBlocks = kScanTile;             // second level: one block

int grid_for(int64_t items, int per_block, int max_blocks) {
    int64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > max_blocks) g = max_blocks;
    return (int)g;
}

size_t scan_temp_bytes(int64_t n) {
    int64_t nblk = (n + kScanTile - 1) / kScanTile;
    if (nblk < 1) nblk = 1;
    return (size_t)(nblk + 1) * sizeof(int64_t);
}

// Arrays of at most kScanSingle items: the whole scan in one block.
constexpr int kScanSingleThreads = 1024;
constexpr int kScanSingle = kScanSingleThreads * kScanItems;  // 8192 items

template <typename TO>
__global__ __launch_bounds__(kScanSingleThreads) void k_scan_single(const int32_t* __restrict__ in,
                                                                   TO* __restrict__ out, int64_t n,
                                                                   const int64_t* __restrict__ n_dev,
                                                                   int64_t* __restrict__ total) {
    __shared__ int64_t sh[kScanSingleThreads / 64];
    int64_t nn = n;
    if (n_dev && *n_dev < nn) nn = *n_dev;
    const int64_t base = (int64_t)threadIdx.x * kScanItems;
    int32_t v[kScanItems];
    int64_t s = 0;
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
        v[q] = base + q < nn ? in[base + q] : 0;
        s += v[q];
    }
    int64_t tot;
    int64_t run = block_inclusive_scan<kScanSingleThreads>(s, sh, tot) - s;
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
        if (base + q < nn) out[base + q] = (TO)run;
        run += v[q];
    }
    if (threadIdx.x == 0 && total) *total = tot;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_up(const int32_t* __restrict__ in, int64_t n,
                                                         const int64_t* __restrict__ n_dev,
                                                         int64_t* __restrict__ bsum) {
    __shared__ int64_t sh[kScanThreads / 64];
    int64_t nn = n;
    if (n_dev && *n_dev < nn) nn = *n_dev;
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t s = 0;
#pragma unroll
    for (int q = 0; q < kScanItems; ++q)
        if (base + q < nn) s += in[base + q];
    int64_t tot;
    block_inclusive_scan(s, sh, tot);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_mid(int64_t* __restrict__ bsum, int nblocks,
                                                          int64_t* __restrict__ total) {
    __shared__ int64_t sh[kScanThreads / 64];
    int64_t v[kScanItems];
    int64_t s = 0;
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
        int idx = threadIdx.x * kScanItems + q;
        v[q] = idx < nblocks ? bsum[idx] : 0;
        s += v[q];
    }
    int64_t tot;
    int64_t incl = block_inclusive_scan(s, sh, tot);
    int64_t run = incl - s;
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
        int idx = threadIdx.x * kScanItems + q;
        if (idx < nblocks) bsum[idx] = run;
        run += v[q];
    }
    if (threadIdx.x == 0 && total) *total = tot;
}

template <typename TO>
__global__ __launch_bounds__(kScanThreads) void k_scan_down(const int32_t* in, TO* out, int64_t n,
                                                           const int64_t* __restrict__ n_dev,
                                                           const int64_t* __restrict__ bsum) {
    __shared__ int64_t sh[kScanThreads / 64];
    int64_t nn = n;
    if (n_dev && *n_dev < nn) nn = *n_dev;
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int32_t v[kScanItems];
    int64_t s = 0;
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
        v[q] = base + q < nn ? in[base + q] : 0;
        s += v[q];
    }
    int64_t tot;
    int64_t incl = block_inclusive_scan(s, sh, tot);
    int64_t run = incl - s + bsum[blockIdx.x];
#pragma unroll
    for (int q = 0; q < kScanItems; ++q) {
        if (base + q < nn) out[base + q] = (TO)run;
        run += v[q];
    }
}

template <typename TO>
static void scan_impl(const int32_t* in, TO* out, int64_t n, const int64_t* n_dev, int64_t* total_dev,
                      void* temp, hipStream_t s) {
    if (n <= kScanSingle) {
        hipLaunchKernelGGL(k_scan_single<TO>, dim3(1), dim3(kScanSingleThreads), 0, s, in, out, n, n_dev, total_dev);
        return;
    }
    int64_t nblk = (n + kScanTile - 1) / kScanTile;
    if (nblk < 1) nblk = 1;
    if (nblk > kScanMaxBlocks) return;  // callers keep n <= 2048 * 2048
    int64_t* bsum = (int64_t*)temp;
    hipLaunchKernelGGL(k_scan_up, dim3((unsigned)nblk), dim3(kScanThreads), 0, s, in, n, n_dev, bsum);
    hipLaunchKernelGGL(k_scan_mid, dim3(1), dim3(kScanThreads), 0, s, bsum, (int)nblk, total_dev);
    hipLaunchKernelGGL(k_scan_down<TO>, dim3((unsigned)nblk), dim3(kScanThreads), 0, s, in, out, n, n_dev,
                       (const int64_t*)bsum);
}

void scan_i32(const int32_t* in, int32_t* out, int64_t n, const int64_t* n_dev, int64_t* total_dev, void* temp,
              hipStream_t s) {
    scan_impl<int32_t>(in, out, n, n_dev, total_dev, temp, s);
}

// ---------------------------------------------------------------------------
__global__ void k_fill_u8(uint8_t* p, int64_t n, uint8_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_fill_i64(int64_t* p, int64_t n, int64_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_copy_i64(int64_t* dst, const int64_t* src) { *dst = *src; }

void fill_u8(uint8_t* p, int64_t n, uint8_t v, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill_u8, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, p, n, v);
}
void fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, p, n, v);
}
void fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s) { fill_i32((int32_t*)p, n, (int32_t)v, s); }
void fill_i64(int64_t* p, int64_t n, int64_t v, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill_i64, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, p, n, v);
}
void copy_i64(int64_t* dst, const int64_t* src, hipStream_t s) {
    hipLaunchKernelGGL(k_copy_i64, dim3(1), dim3(1), 0, s, dst, src);
}

}  // namespace spamm
