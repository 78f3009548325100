// Microbenchmarks that give the KmerCo kernels their roofline denominators on
// gfx950: uniform-random 64-bit atomics / reads and 32-bit atomicMin over a
// chosen footprint (L2-, Infinity-Cache- or HBM-sized), a streaming copy, LDS
// atomics, and the issue rate of the integer VALU instructions the hashing
// uses (add, 32-bit multiply low / high, 64-bit multiply-add).  Built as its own library
// (libkmerco_microbench.so); the KmerCo library does not use it.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

// splitmix64 finaliser: a stateless mixer from op index to a random word
__device__ __forceinline__ uint64_t mix(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

// uniform index in [0, n) (multiply-high range reduction)
__device__ __forceinline__ uint64_t pick(uint64_t r, uint64_t n) { return __umul64hi(r, n); }

enum Kind {
    kRead64 = 0,        // random 8-byte loads
    kAdd64 = 1,         // random 8-byte atomicAdd, result unused
    kCas64 = 2,         // random 8-byte load + CAS increment loop
    kMin32 = 3,         // random 4-byte atomicMin, result unused
    kAdd64Ret = 4,      // random 8-byte atomicAdd, result used
    kCopy64 = 5,        // streaming copy, 8 bytes read + 8 written per op
    kLds = 6,           // random LDS add + min within 128 KiB per workgroup
    kAluAdd = 7,        // v_add_u32 chains (ops = lane operations)
    kAluMulLo = 8,      // v_mul_lo_u32 chains
    kAluMulHi = 9,      // v_mul_hi_u32 chains
    kAluMad64 = 10,     // v_mad_u64_u32 chains
};

// Eight independent dependency chains per thread, one instruction per link,
// so that issue rate rather than latency bounds the loop.
template <int K>
__global__ void __launch_bounds__(256) k_alu(uint32_t iters, uint32_t c,
                                             uint64_t *__restrict__ sink) {
    uint32_t x[8];
    uint64_t y[8];
#pragma unroll
    for (int j = 0; j < 8; j++) {
        x[j] = threadIdx.x * 8u + (uint32_t)j + 1u;
        y[j] = x[j];
    }
    for (uint32_t i = 0; i < iters; i++) {
#pragma unroll
        for (int j = 0; j < 8; j++) {
            if (K == kAluAdd)
                asm volatile("v_add_u32 %0, %0, %1" : "+v"(x[j]) : "v"(c));
            else if (K == kAluMulLo)
                asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(x[j]) : "v"(c));
            else if (K == kAluMulHi)
                asm volatile("v_mul_hi_u32 %0, %0, %1" : "+v"(x[j]) : "v"(c));
            else {
                uint64_t carry;
                asm volatile("v_mad_u64_u32 %0, %1, %2, %3, %0"
                             : "+v"(y[j]), "=s"(carry)
                             : "v"((uint32_t)y[j]), "v"(c));
            }
        }
    }
    uint64_t acc = 0;
#pragma unroll
    for (int j = 0; j < 8; j++)
        acc += x[j] + y[j];
    if (acc == 0x123456789ull)
        *sink = acc;
}

__global__ void __launch_bounds__(256) k_random(int kind, uint64_t *__restrict__ buf, uint64_t n64,
                                                uint64_t *__restrict__ dst, uint64_t ops,
                                                uint64_t seed, uint64_t *__restrict__ sink) {
    uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint64_t acc = 0;
    if (kind == kRead64) {
        for (uint64_t i = tid; i < ops; i += stride)
            acc += buf[pick(mix(i ^ seed), n64)];
    } else if (kind == kAdd64) {
        for (uint64_t i = tid; i < ops; i += stride)
            atomicAdd((unsigned long long *)&buf[pick(mix(i ^ seed), n64)], 1ull);
    } else if (kind == kAdd64Ret) {
        for (uint64_t i = tid; i < ops; i += stride)
            acc += atomicAdd((unsigned long long *)&buf[pick(mix(i ^ seed), n64)], 1ull);
    } else if (kind == kCas64) {
        for (uint64_t i = tid; i < ops; i += stride) {
            unsigned long long *p = (unsigned long long *)&buf[pick(mix(i ^ seed), n64)];
            unsigned long long old = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            for (;;) {
                unsigned long long prev = atomicCAS(p, old, old + 1ull);
                if (prev == old)
                    break;
                old = prev;
            }
        }
    } else if (kind == kMin32) {
        uint32_t *b32 = (uint32_t *)buf;
        for (uint64_t i = tid; i < ops; i += stride) {
            uint64_t r = mix(i ^ seed);
            atomicMin(&b32[pick(r, 2 * n64)], (uint32_t)(r >> 40));
        }
    } else if (kind == kCopy64) {
        for (uint64_t i = tid; i < ops; i += stride)
            dst[i] = buf[i];
    }
    if (acc == 0x123456789ull)
        *sink = acc;  // keeps the loads alive
}

__global__ void __launch_bounds__(256) k_lds(uint64_t ops_per_block, uint64_t seed,
                                             uint64_t *__restrict__ sink) {
    __shared__ uint32_t s[2][16384];  // 2 x 64 KiB
    for (int i = threadIdx.x; i < 16384; i += 256) {
        s[0][i] = 0;
        s[1][i] = 0xFFFFFFFFu;
    }
    __syncthreads();
    for (uint64_t i = threadIdx.x; i < ops_per_block; i += 256) {
        uint64_t r = mix((blockIdx.x * ops_per_block + i) ^ seed);
        uint32_t idx = (uint32_t)(r & 16383u);
        atomicAdd(&s[0][idx], 1u);
        atomicMin(&s[1][idx], (uint32_t)(r >> 32));
    }
    __syncthreads();
    if (threadIdx.x == 0 && s[0][0] == 0x7FFFFFFFu)
        *sink = s[1][0];
}


int run_alu(int kind, uint64_t ops, double *ms) {
    uint64_t *sink = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    int rc = 0;
    const unsigned blocks = 256 * 8, threads = 256;
    const uint64_t per_iter = (uint64_t)blocks * threads * 8;  // lane operations
    const uint32_t iters = (uint32_t)((ops + per_iter - 1) / per_iter);
    if (hipMalloc((void **)&sink, 8) != hipSuccess)
        return -4;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)
        rc = -4;
    for (int rep = 0; rep < 2 && rc == 0; rep++) {  // rep 0 warms up
        (void)hipEventRecord(a, nullptr);
        const uint32_t c = 0x9E3779B9u + (uint32_t)rep;
        if (kind == kAluAdd)
            hipLaunchKernelGGL(k_alu<kAluAdd>, dim3(blocks), dim3(threads), 0, nullptr, iters, c,
                               sink);
        else if (kind == kAluMulLo)
            hipLaunchKernelGGL(k_alu<kAluMulLo>, dim3(blocks), dim3(threads), 0, nullptr, iters,
                               c, sink);
        else if (kind == kAluMulHi)
            hipLaunchKernelGGL(k_alu<kAluMulHi>, dim3(blocks), dim3(threads), 0, nullptr, iters,
                               c, sink);
        else
            hipLaunchKernelGGL(k_alu<kAluMad64>, dim3(blocks), dim3(threads), 0, nullptr, iters,
                               c, sink);
        (void)hipEventRecord(b, nullptr);
        if (hipGetLastError() != hipSuccess || hipEventSynchronize(b) != hipSuccess)
            rc = -4;
    }
    float t = 0.f;
    if (rc == 0 && hipEventElapsedTime(&t, a, b) != hipSuccess)
        rc = -4;
    // report the time of exactly `ops` lane operations
    *ms = t * (double)ops / ((double)iters * per_iter);
    if (a)
        (void)hipEventDestroy(a);
    if (b)
        (void)hipEventDestroy(b);
    (void)hipFree(sink);
    return rc;
}

}  // namespace

extern "C" {

// Run one microbenchmark and return its time in milliseconds through *ms.
// kind: see Kind; footprint_bytes: size of the random-access array (a
// multiple of 8, allocated and freed here); ops: operations to issue.
// Returns 0 on success, -1 on bad arguments, -4 on a runtime error.
int kcmb_run(int kind, uint64_t footprint_bytes, uint64_t ops, double *ms) {
    if (!ms || kind < 0 || kind > kAluMad64 || ops == 0)
        return -1;
    if (kind >= kAluAdd)
        return run_alu(kind, ops, ms);
    uint64_t n64 = footprint_bytes / 8;
    if (kind != kLds && n64 == 0)
        return -1;
    if (kind == kCopy64 && ops > n64)
        ops = n64;
    uint64_t *buf = nullptr, *dst = nullptr, *sink = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    int rc = 0;
    if (kind != kLds && hipMalloc((void **)&buf, n64 * 8) != hipSuccess)
        return -4;
    if (kind == kCopy64 && hipMalloc((void **)&dst, n64 * 8) != hipSuccess)
        rc = -4;
    if (rc == 0 && hipMalloc((void **)&sink, 8) != hipSuccess)
        rc = -4;
    if (rc == 0 && buf && hipMemset(buf, 0, n64 * 8) != hipSuccess)
        rc = -4;
    if (rc == 0 && (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess))
        rc = -4;
    if (rc == 0) {
        const unsigned blocks = 256 * 16;  // 16 workgroups per CU
        const uint64_t lds_per_block = (ops + blocks - 1) / blocks;
        for (int rep = 0; rep < 2 && rc == 0; rep++) {  // rep 0 warms up
            (void)hipEventRecord(a, nullptr);
            if (kind == kLds)
                hipLaunchKernelGGL(k_lds, dim3(blocks), dim3(256), 0, nullptr, lds_per_block,
                                   (uint64_t)rep, sink);
            else
                hipLaunchKernelGGL(k_random, dim3(blocks), dim3(256), 0, nullptr, kind, buf, n64,
                                   dst, ops, (uint64_t)rep * 0x51ED27ull, sink);
            (void)hipEventRecord(b, nullptr);
            if (hipGetLastError() != hipSuccess || hipEventSynchronize(b) != hipSuccess)
                rc = -4;
        }
        float t = 0.f;
        if (rc == 0 && hipEventElapsedTime(&t, a, b) != hipSuccess)
            rc = -4;
        *ms = t;
    }
    if (a)
        (void)hipEventDestroy(a);
    if (b)
        (void)hipEventDestroy(b);
    (void)hipFree(buf);
    (void)hipFree(dst);
    (void)hipFree(sink);
    return rc;
}
}
