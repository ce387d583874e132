// Calibration program for the roofline figures (not part of the library):
//   copy    : 16-byte vector copy of 4 GiB -> 4 GiB (attainable HBM rate, and
//             the reference kernel whose FETCH_SIZE / WRITE_SIZE counters
//             scale the sweep kernel's counters to bytes);
//   read    : 4 GiB read-only stream;
//   rrw     : read a, read b, write a (the traffic shape of a half-sweep);
//   philox  : Philox4x32-10 blocks/s alone: the library's form (one
//             v_mad_u64_u32 per product, one v_bitop3_b32 per pair of xors,
//             counter words as the sweep's accept draws use them: a per-lane
//             block index, zero high word, wave-uniform t and colour), and
//             for comparison separate high/low multiplies with plain xors;
//   alu/mad : 32-bit integer VALU issue rate (lane-instructions/s) and the
//             v_mad_u64_u32 rate (full rate on gfx950).
// Usage: mcl_calibrate [copy|philox]   (with an argument only that test runs)
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "common.h"

#define CHECK(x) do { hipError_t e = (x); if (e != hipSuccess) { printf("HIP error %s at %d\n", hipGetErrorString(e), __LINE__); exit(1);} } while (0)

__global__ void copy_kernel(const uint4* __restrict__ a, uint4* __restrict__ b, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) b[i] = a[i];
}

__global__ void read_kernel(const uint4* __restrict__ a, int64_t n, uint32_t* out)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    uint32_t acc = 0;
    for (; i < n; i += stride) { uint4 v = a[i]; acc ^= v.x ^ v.y ^ v.z ^ v.w; }
    if (acc == 0x12345678u) out[0] = acc;
}

// 3 streams: read a, read b, write a (the half-sweep's traffic shape)
__global__ void rrw_kernel(uint4* __restrict__ a, const uint4* __restrict__ b, int64_t n)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) { uint4 x = a[i], y = b[i]; x.x ^= y.x; x.y ^= y.y; x.z ^= y.z; x.w ^= y.w; a[i] = x; }
}

__device__ __forceinline__ void philox_hilo(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t h0 = __umulhi(0xD2511F53u, c0), l0 = 0xD2511F53u * c0;
        const uint32_t h1 = __umulhi(0xCD9E8D57u, c2), l1 = 0xCD9E8D57u * c2;
        const uint32_t n0 = h1 ^ c1 ^ k0;
        const uint32_t n2 = h0 ^ c3 ^ k1;
        c1 = l1; c3 = l0; c0 = n0; c2 = n2;
        k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
    }
}

// Each thread generates nblk consecutive blocks, four at a time, and folds
// their words into one output word so that nothing is optimised away.
template <int VARIANT>
__global__ __launch_bounds__(256) void philox_kernel(uint32_t* out, int nblk, uint32_t k0, uint32_t k1, uint32_t t)
{
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t acc = 0;
    for (int i = 0; i < nblk; i += 4) {
        const uint32_t b = tid * (uint32_t)nblk + (uint32_t)i;
        if (VARIANT == 0) {
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                const mcl::Philox4 p = mcl::philox4x32_10(b + d, 0u, t, 1u, k0, k1);
                acc += mcl::xor3(p.v0, p.v1, p.v2) ^ p.v3;
            }
        } else {
            uint32_t a0 = b, a1 = 0, a2 = t, a3 = 1, b0 = b + 1, b1 = 0, b2 = t, b3 = 1;
            uint32_t c0 = b + 2, c1 = 0, c2 = t, c3 = 1, d0 = b + 3, d1 = 0, d2 = t, d3 = 1;
            philox_hilo(a0, a1, a2, a3, k0, k1); philox_hilo(b0, b1, b2, b3, k0, k1);
            philox_hilo(c0, c1, c2, c3, k0, k1); philox_hilo(d0, d1, d2, d3, k0, k1);
            acc += (a0 ^ a1 ^ a2 ^ a3) + (b0 ^ b1 ^ b2 ^ b3) + (c0 ^ c1 ^ c2 ^ c3) + (d0 ^ d1 ^ d2 ^ d3);
        }
    }
    out[tid] = acc;
}

// Pure 32-bit integer ALU: 8 independent chains of xor/add.
__global__ __launch_bounds__(256) void alu_kernel(uint32_t* out, int iters, uint32_t s)
{
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t v0 = tid, v1 = tid + 1, v2 = tid + 2, v3 = tid + 3, v4 = tid + 4, v5 = tid + 5, v6 = tid + 6, v7 = tid + 7;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            v0 = (v0 ^ s) + v7; v1 = (v1 ^ s) + v0; v2 = (v2 ^ s) + v1; v3 = (v3 ^ s) + v2;
            v4 = (v4 ^ s) + v3; v5 = (v5 ^ s) + v4; v6 = (v6 ^ s) + v5; v7 = (v7 ^ s) + v6;
        }
    }
    out[tid] = v0 ^ v1 ^ v2 ^ v3 ^ v4 ^ v5 ^ v6 ^ v7;
}

// 64-bit mad throughput: 8 independent chains.
__global__ __launch_bounds__(256) void mad_kernel(uint32_t* out, int iters, uint32_t s)
{
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = tid + k;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < 16; ++k) {
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                uint64_t p = (uint64_t)0xD2511F53u * v[j];
                v[j] = (uint32_t)(p >> 32) ^ (uint32_t)p;
            }
        }
    }
    uint32_t a = 0;
    for (int k = 0; k < 8; ++k) a ^= v[k];
    out[tid] = a;
}

// Time one launch: the event pair around it, in milliseconds.
template <typename F>
static float timed(hipEvent_t e0, hipEvent_t e1, F launch)
{
    float ms = 0.f;
    CHECK(hipEventRecord(e0));
    launch();
    CHECK(hipGetLastError());
    CHECK(hipEventRecord(e1));
    CHECK(hipEventSynchronize(e1));
    CHECK(hipEventElapsedTime(&ms, e0, e1));
    return ms;
}

int main(int argc, char** argv)
{
    const bool copy_only = argc > 1 && strcmp(argv[1], "copy") == 0;
    const bool philox_only = argc > 1 && strcmp(argv[1], "philox") == 0;
    if (argc > 1 && !copy_only && !philox_only) {
        fprintf(stderr, "usage: %s [copy|philox]\n", argv[0]);
        return 2;
    }
    hipDeviceProp_t prop;
    CHECK(hipGetDeviceProperties(&prop, 0));
    printf("device %s CUs %d clock %d kHz mem clock %d kHz bus %d LDS/CU %zu L2 %d\n", prop.gcnArchName,
           prop.multiProcessorCount, prop.clockRate, prop.memoryClockRate, prop.memoryBusWidth,
           (size_t)prop.maxSharedMemoryPerMultiProcessor, prop.l2CacheSize);
    const int threads = 256 * 256 * 16;   // 1M threads
    uint32_t* out;
    CHECK(hipMalloc(&out, (size_t)threads * 4));
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    if (!philox_only) {
        const int64_t bytes = (int64_t)4 << 30;   // 4 GiB per buffer
        const int64_t n = bytes / 16;
        uint4 *a, *b;
        CHECK(hipMalloc(&a, bytes));
        CHECK(hipMalloc(&b, bytes));
        CHECK(hipMemset(a, 1, bytes));
        CHECK(hipMemset(b, 2, bytes));
        const int grid = 256 * 8 * 4;
        for (int rep = 0; rep < 3; ++rep) {
            const float ms = timed(e0, e1, [&] { hipLaunchKernelGGL(copy_kernel, dim3(grid), dim3(256), 0, 0, a, b, n); });
            printf("copy 4GiB->4GiB: %.3f ms  %.1f GB/s\n", ms, 2.0 * bytes / ms / 1e6);
        }
        if (!copy_only) {
            for (int rep = 0; rep < 3; ++rep) {
                const float ms = timed(e0, e1, [&] { hipLaunchKernelGGL(read_kernel, dim3(grid), dim3(256), 0, 0, a, n, out); });
                printf("read 4GiB: %.3f ms  %.1f GB/s\n", ms, 1.0 * bytes / ms / 1e6);
            }
            for (int rep = 0; rep < 3; ++rep) {
                const float ms = timed(e0, e1, [&] { hipLaunchKernelGGL(rrw_kernel, dim3(grid), dim3(256), 0, 0, a, b, n); });
                printf("read a + read b + write a (4GiB each): %.3f ms  %.1f GB/s\n", ms, 3.0 * bytes / ms / 1e6);
            }
        }
        CHECK(hipFree(a));
        CHECK(hipFree(b));
    }
    if (!copy_only) {
        // Philox: threads * nblk blocks per launch (2^30), the first launch a warm-up
        const int nblk = 1024;
        const double blocks = (double)threads * nblk;
        for (int variant = 0; variant < 2; ++variant) {
            double best = 0.0;
            for (int rep = 0; rep < 4; ++rep) {
                const float ms = timed(e0, e1, [&] {
                    if (variant == 0)
                        hipLaunchKernelGGL(philox_kernel<0>, dim3(threads / 256), dim3(256), 0, 0, out, nblk, 1001u, 0u, 5u);
                    else
                        hipLaunchKernelGGL(philox_kernel<1>, dim3(threads / 256), dim3(256), 0, 0, out, nblk, 1001u, 0u, 5u);
                });
                if (rep == 0) continue;
                const double g = blocks / ms / 1e6;
                if (g > best) best = g;
                printf("philox variant %d (%s): %.3f ms  %.1f Gblocks/s = %.1f draws/ns\n", variant,
                       variant == 0 ? "library: mad_u64 + bitop3" : "mul_hi + mul_lo, plain xors", ms, g, 4 * g);
            }
            if (variant == 0) printf("philox attainable: %.1f Gblocks/s\n", best);
        }
    }
    if (!copy_only && !philox_only) {
        for (int rep = 0; rep < 2; ++rep) {
            const int iters = 256;
            const float ms = timed(e0, e1, [&] { hipLaunchKernelGGL(alu_kernel, dim3(threads / 256), dim3(256), 0, 0, out, iters, 3u); });
            // each xor-then-add is one v_xad_u32: one lane-instruction per step
            const double insts = (double)threads * iters * 16 * 8;
            printf("alu v_xad: %.3f ms  %.2f T lane-instructions/s (%.3f of 39.32e12)\n", ms, insts / ms / 1e9,
                   insts / ms / 1e9 / 39.3216);
        }
        for (int rep = 0; rep < 2; ++rep) {
            const int iters = 64;
            const float ms = timed(e0, e1, [&] { hipLaunchKernelGGL(mad_kernel, dim3(threads / 256), dim3(256), 0, 0, out, iters, 3u); });
            // each step is one v_mad_u64_u32 and one xor: two lane-instructions
            const double ops = (double)threads * iters * 16 * 8;
            printf("mad_u64 (+1 xor each): %.3f ms  %.2f T mads/s (%.3f of the issue peak with the xors)\n", ms,
                   ops / ms / 1e9, 2 * ops / ms / 1e9 / 39.3216);
        }
    }
    CHECK(hipFree(out));
    printf("calibrate done\n");
    return 0;
}
