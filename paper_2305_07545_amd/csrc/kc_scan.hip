// Multi-workgroup exclusive prefix sums (block sums, then a rescan of each
// block with the sum of the blocks before it) used for the ordered outputs
// and the bin offsets.
#include <hip/hip_runtime.h>

#include "kc_kernels.hpp"

namespace kc {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanPer = 16;
constexpr int kScanBlock = kScanThreads * kScanPer;  // elements per workgroup

// Exclusive sum of one value per thread over the workgroup: wave scans by
// shuffles, then the wave totals.  s_wave: kScanThreads / 64 entries.
template <typename T>
__device__ __forceinline__ T wg_exclusive_sum(T v, T *s_wave, T &total) {
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    T incl = v;
#pragma unroll
    for (uint32_t d = 1; d < 64; d <<= 1) {
        T o = __shfl_up(incl, d, 64);
        if (lane >= d)
            incl += o;
    }
    if (lane == 63)
        s_wave[wave] = incl;
    __syncthreads();
    T before = 0;
    total = 0;
#pragma unroll
    for (uint32_t w = 0; w < kScanThreads / 64; w++) {
        const T t = s_wave[w];
        if (w < wave)
            before += t;
        total += t;
    }
    __syncthreads();
    return before + incl - v;
}

// Sum of each workgroup's kScanBlock elements (coalesced: element i*256+tid).
template <typename TIn, typename TOut>
__global__ void __launch_bounds__(kScanThreads) k_scan_reduce(const TIn *__restrict__ in, uint64_t n,
                                                             TOut *__restrict__ partial) {
    __shared__ TOut s_wave[kScanThreads / 64];
    const uint64_t base = (uint64_t)blockIdx.x * kScanBlock + threadIdx.x;
    TOut sum = 0;
#pragma unroll
    for (int i = 0; i < kScanPer; i++) {
        const uint64_t x = base + (uint64_t)i * kScanThreads;
        if (x < n)
            sum += (TOut)in[x];
    }
    TOut total;
    (void)wg_exclusive_sum<TOut>(sum, s_wave, total);
    if (threadIdx.x == 0)
        partial[blockIdx.x] = total;
}

// LDS slot of element e of a block: one pad word after every kScanPer
// elements, so that thread t's run (elements 16t .. 16t+15) and the
// coalesced rows (elements i*256 + t) are both free of bank conflicts.
__device__ __forceinline__ uint32_t pad_at(uint32_t e) { return e + e / kScanPer; }

// Exclusive scan of each workgroup's elements, offset by base and the sums
// of the workgroups before it (each workgroup adds up those block sums
// itself: a few KB from L2, one launch fewer than a separate scan of the
// sums): coalesced loads into LDS, a sequential scan of 16 consecutive
// elements per thread, the workgroup scan of the thread sums, coalesced
// stores.  The last workgroup writes the grand total (without base).
template <typename TIn, typename TOut>
__global__ void __launch_bounds__(kScanThreads) k_scan_down(const TIn *__restrict__ in, uint64_t n,
                                                           const TOut *__restrict__ partial,
                                                           const TOut *__restrict__ base,
                                                           TOut *__restrict__ out,
                                                           TOut *__restrict__ total_out) {
    __shared__ TOut s_buf[kScanBlock + kScanBlock / kScanPer];
    __shared__ TOut s_wave[kScanThreads / 64];
    TOut before = 0;
    for (uint32_t i = threadIdx.x; i < blockIdx.x; i += kScanThreads)
        before += partial[i];
    TOut pre;
    (void)wg_exclusive_sum<TOut>(before, s_wave, pre);
    const TOut offset = (base ? *base : (TOut)0) + pre;
    const uint64_t b0 = (uint64_t)blockIdx.x * kScanBlock;
#pragma unroll
    for (int i = 0; i < kScanPer; i++) {
        const uint32_t e = (uint32_t)i * kScanThreads + threadIdx.x;
        s_buf[pad_at(e)] = b0 + e < n ? (TOut)in[b0 + e] : (TOut)0;
    }
    __syncthreads();
    TOut v[kScanPer];
    TOut sum = 0;
#pragma unroll
    for (int i = 0; i < kScanPer; i++) {
        v[i] = s_buf[pad_at(threadIdx.x * kScanPer + i)];
        sum += v[i];
    }
    TOut total;
    TOut run = offset + wg_exclusive_sum<TOut>(sum, s_wave, total);
#pragma unroll
    for (int i = 0; i < kScanPer; i++) {
        s_buf[pad_at(threadIdx.x * kScanPer + i)] = run;
        run += v[i];
    }
    if (total_out && threadIdx.x == 0 && blockIdx.x + 1 == gridDim.x)
        *total_out = pre + total;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kScanPer; i++) {
        const uint32_t e = (uint32_t)i * kScanThreads + threadIdx.x;
        if (b0 + e < n)
            out[b0 + e] = s_buf[pad_at(e)];
    }
}

template <typename TIn, typename TOut>
hipError_t scan_impl(const TIn *in, TOut *out, uint64_t n, const TOut *base, TOut *total,
                     TOut *partial, hipStream_t s) {
    uint64_t nb = (n + kScanBlock - 1) / kScanBlock;
    if (nb == 0)
        nb = 1;
    hipLaunchKernelGGL((k_scan_reduce<TIn, TOut>), dim3((unsigned)nb), dim3(kScanThreads), 0, s,
                       in, n, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL((k_scan_down<TIn, TOut>), dim3((unsigned)nb), dim3(kScanThreads), 0, s, in,
                       n, (const TOut *)partial, base, out, total);
    return hipGetLastError();
}

// 64 x 64 tiles through LDS (one pad word per row: no bank conflicts on the
// column reads); reads and writes are 256-byte rows.  Batch z transposes the
// rows x cols block at in + z*rows*cols into out + z*cols*rows, its columns
// cut at total_cols - z*cols (the last block may be narrower).
__global__ void __launch_bounds__(256) k_transpose_u32(const uint32_t *__restrict__ in,
                                                       uint32_t *__restrict__ out, uint64_t rows,
                                                       uint64_t cols, uint64_t total_cols) {
    __shared__ uint32_t t[64][65];
    const uint64_t z0 = (uint64_t)blockIdx.z * cols;
    const uint64_t cz = total_cols - z0 < cols ? total_cols - z0 : cols;
    const uint32_t *__restrict__ src = in + (uint64_t)blockIdx.z * rows * cols;
    uint32_t *__restrict__ dst = out + z0 * rows;
    const uint64_t c0 = (uint64_t)blockIdx.x * 64, r0 = (uint64_t)blockIdx.y * 64;
    const uint32_t tx = threadIdx.x & 63u, ty = threadIdx.x >> 6;
    for (uint32_t j = ty; j < 64; j += 4) {
        const uint64_t r = r0 + j, c = c0 + tx;
        if (r < rows && c < cz)
            t[j][tx] = src[r * cols + c];
    }
    __syncthreads();
    for (uint32_t j = ty; j < 64; j += 4) {
        const uint64_t c = c0 + j, r = r0 + tx;
        if (c < cz && r < rows)
            dst[c * rows + r] = t[tx][j];
    }
}

}  // namespace

hipError_t transpose_u32(const uint32_t *in, uint32_t *out, uint64_t rows, uint64_t cols,
                         hipStream_t s) {
    return transpose_u32_blocks(in, out, rows, cols, cols, s);
}

hipError_t transpose_u32_blocks(const uint32_t *in, uint32_t *out, uint64_t rows, uint64_t cols,
                                uint64_t total_cols, hipStream_t s) {
    if (rows == 0 || cols == 0 || total_cols == 0)
        return hipSuccess;
    const uint64_t gx = (cols + 63) / 64, gy = (rows + 63) / 64;
    const uint64_t gz = (total_cols + cols - 1) / cols;
    if (gx > 0x7FFFFFFFull || gy > 65535 || gz > 65535)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_transpose_u32, dim3((unsigned)gx, (unsigned)gy, (unsigned)gz), dim3(256),
                       0, s, in, out, rows, cols, total_cols);
    return hipGetLastError();
}

uint64_t scan_partials(uint64_t n) { return (n + kScanBlock - 1) / kScanBlock + 1; }

hipError_t scan_u32_u64(const uint32_t *in, uint64_t *out, uint64_t n, const uint64_t *base,
                        uint64_t *total, uint64_t *partial, hipStream_t s) {
    return scan_impl<uint32_t, uint64_t>(in, out, n, base, total, partial, s);
}

hipError_t scan_u32_u32(const uint32_t *in, uint32_t *out, uint64_t n, uint32_t *total,
                        uint32_t *partial, hipStream_t s) {
    return scan_impl<uint32_t, uint32_t>(in, out, n, (const uint32_t *)nullptr, total, partial, s);
}

}  // namespace kc
