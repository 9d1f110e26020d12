// cae_ubench.hip -- issue-rate microbenchmarks that fix the engine's roofline denominators.
//
// Each kernel runs 8 independent dependency chains of one instruction per lane (enough
// independent work per wave, and 8 waves per SIMD, to reach the issue limit) and the host
// times the whole grid with HIP events.  Rates are lane-operations per second; the ratio
// against a full-rate op (v_add_u32) is the instruction's issue cost in full-rate slots.
// The LDS kernels issue ds_add_u32 without return: conflict-free (one bank per lane) and with
// addresses drawn from a narrow window, as the engine's order aggregation does.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

enum Kind : int {
    K_ADD = 0,
    K_XOR = 1,
    K_BITOP3 = 2,
    K_MUL_HI = 3,
    K_MUL_LO = 4,
    K_MAD_U64 = 5,
    K_LDS_ADD_NOCONFLICT = 6,
    K_LDS_ADD_WINDOW = 7,
    K_FMA_F32 = 8,
    K_FMA_F64 = 9,
};

// Shader-clock cycles and 100 MHz real-time ticks of the timed loop, per workgroup.
__device__ __forceinline__ void stamp(uint64_t *clk, uint64_t &c, uint64_t &r)
{
    (void)clk;
    __builtin_amdgcn_s_waitcnt(0);
    c = clock64();
    r = wall_clock64();
}

template <int KIND>
__global__ void __launch_bounds__(1024) ub_valu(uint32_t *out, uint64_t *clk, uint32_t iters, uint32_t seed)
{
    uint32_t a[8];
    float f[8];
    double g[8];
    const uint32_t b = seed * 2654435761u + 1u;
#pragma unroll
    for (int j = 0; j < 8; ++j) a[j] = threadIdx.x * 7u + (uint32_t)j * 13u + seed;
    uint64_t p[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        p[j] = a[j];
        f[j] = (float)a[j];
        g[j] = (double)a[j];
    }
    const float fb = 0.999f;
    const double gb = 0.999;
    __syncthreads();
    uint64_t c0, r0, c1, r1;
    stamp(clk, c0, r0);
    for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            if constexpr (KIND == K_ADD) {
                asm volatile("v_add_u32 %0, %0, %1" : "+v"(a[j]) : "v"(b));
            } else if constexpr (KIND == K_XOR) {
                asm volatile("v_xor_b32 %0, %0, %1" : "+v"(a[j]) : "v"(b));
            } else if constexpr (KIND == K_BITOP3) {
                asm volatile("v_bitop3_b32 %0, %0, %1, %1 bitop3:0x96" : "+v"(a[j]) : "v"(b));
            } else if constexpr (KIND == K_MUL_HI) {
                asm volatile("v_mul_hi_u32 %0, %0, %1" : "+v"(a[j]) : "v"(b));
            } else if constexpr (KIND == K_MUL_LO) {
                asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(a[j]) : "v"(b));
            } else if constexpr (KIND == K_MAD_U64) {
                uint64_t cc;
                asm volatile("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(p[j]), "=s"(cc) : "v"(a[j]), "v"(b));
            } else if constexpr (KIND == K_FMA_F32) {
                asm volatile("v_fma_f32 %0, %0, %1, %1" : "+v"(f[j]) : "v"(fb));
            } else if constexpr (KIND == K_FMA_F64) {
                asm volatile("v_fma_f64 %0, %0, %1, %1" : "+v"(g[j]) : "v"(gb));
            }
        }
    }
    __syncthreads();  // the loop ends when the workgroup's last wave ends
    stamp(clk, c1, r1);
    uint32_t r = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j)
        r ^= a[j] ^ (uint32_t)p[j] ^ (uint32_t)(p[j] >> 32) ^ (uint32_t)f[j] ^ (uint32_t)g[j];
    out[blockIdx.x * blockDim.x + threadIdx.x] = r;
    if (threadIdx.x == 0) {
        clk[2 * blockIdx.x] = c1 - c0;
        clk[2 * blockIdx.x + 1] = r1 - r0;
    }
}

template <int KIND>
__global__ void __launch_bounds__(1024) ub_lds(uint32_t *out, uint64_t *clk, uint32_t iters, uint32_t seed)
{
    __shared__ uint32_t buf[16][256];
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    for (uint32_t i = threadIdx.x; i < 16 * 256; i += blockDim.x) (&buf[0][0])[i] = 0;
    __syncthreads();
    uint32_t addr[8];
    uint32_t x = (threadIdx.x + 1u) * 2654435761u ^ seed;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        if constexpr (KIND == K_LDS_ADD_NOCONFLICT) {
            addr[j] = lane;  // 64 consecutive words: every bank hit by exactly 2 lanes
        } else {
            x = x * 1664525u + 1013904223u;  // fixed per-lane address in a 66-word window
            addr[j] = 96u + (uint32_t)(((uint64_t)(x >> 8) * 66u) >> 24);
        }
    }
    uint64_t c0, r0, c1, r1;
    stamp(clk, c0, r0);
    for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int j = 0; j < 8; ++j) atomicAdd(&buf[wave][addr[j] & 255u], 1u);
    }
    __syncthreads();
    stamp(clk, c1, r1);
    if (threadIdx.x == 0) {
        clk[2 * blockIdx.x] = c1 - c0;
        clk[2 * blockIdx.x + 1] = r1 - r0;
    }
    out[blockIdx.x * blockDim.x + threadIdx.x] = buf[wave][lane];
}

}  // namespace

extern "C" {

// Runs one microbenchmark: `blocks` workgroups of `threads` threads (64..1024), `iters` iterations of 8
// operations per lane.  Writes the elapsed milliseconds to *ms and, per workgroup, the shader
// clock cycles and 100 MHz real-time ticks of its timed loop to clk[2*b], clk[2*b+1].  out must
// hold blocks*threads words and clk 2*blocks 64-bit words of device memory.  Returns 0, or -1 for
// an unknown kind, -4 for a HIP error.
int cae_ubench_run(int kind, uint32_t blocks, uint32_t threads, uint32_t iters, uint32_t *out, uint64_t *clk, float *ms)
{
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -4;
    if (threads < 64 || threads > 1024 || threads % 64) return -1;
    const dim3 g(blocks), b(threads);
    (void)hipEventRecord(e0, nullptr);
    switch (kind) {
    case K_ADD: hipLaunchKernelGGL(ub_valu<K_ADD>, g, b, 0, nullptr, out, clk, iters, 1u); break;
    case K_XOR: hipLaunchKernelGGL(ub_valu<K_XOR>, g, b, 0, nullptr, out, clk, iters, 1u); break;
    case K_BITOP3: hipLaunchKernelGGL(ub_valu<K_BITOP3>, g, b, 0, nullptr, out, clk, iters, 1u); break;
    case K_MUL_HI: hipLaunchKernelGGL(ub_valu<K_MUL_HI>, g, b, 0, nullptr, out, clk, iters, 1u); break;
    case K_MUL_LO: hipLaunchKernelGGL(ub_valu<K_MUL_LO>, g, b, 0, nullptr, out, clk, iters, 1u); break;
    case K_MAD_U64: hipLaunchKernelGGL(ub_valu<K_MAD_U64>, g, b, 0, nullptr, out, clk, iters, 1u); break;
    case K_LDS_ADD_NOCONFLICT:
        hipLaunchKernelGGL(ub_lds<K_LDS_ADD_NOCONFLICT>, g, b, 0, nullptr, out, clk, iters, 1u);
        break;
    case K_LDS_ADD_WINDOW: hipLaunchKernelGGL(ub_lds<K_LDS_ADD_WINDOW>, g, b, 0, nullptr, out, clk, iters, 1u); break;
    case K_FMA_F32: hipLaunchKernelGGL(ub_valu<K_FMA_F32>, g, b, 0, nullptr, out, clk, iters, 1u); break;
    case K_FMA_F64: hipLaunchKernelGGL(ub_valu<K_FMA_F64>, g, b, 0, nullptr, out, clk, iters, 1u); break;
    default:
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return -1;
    }
    (void)hipEventRecord(e1, nullptr);
    const hipError_t err = hipEventSynchronize(e1);
    float t = 0.f;
    (void)hipEventElapsedTime(&t, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess || hipGetLastError() != hipSuccess) return -4;
    *ms = t;
    return 0;
}

// Frequency of the real-time counter read by wall_clock64(), in kHz (0 on error).
int cae_ubench_wallclock_khz(void)
{
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess) return 0;
    return khz;
}

}  // extern "C"
