// cae_ubench.hip -- issue-rate microbenchmarks that fix the engine's roofline denominators.
//
// Each kernel runs 8 independent dependency chains of one instruction per lane (enough
// independent work per wave, and 8 waves per SIMD, to reach the issue limit) and the host
// times the whole grid with HIP events.  Rates are lane-operations per second; the ratio
// against a full-rate op (v_add_u32) is the instruction's issue cost in full-rate slots.
// The LDS kernels issue ds_add_u32 without return: conflict-free (one bank per lane) and with
// addresses drawn from a narrow window, as the engine's order aggregation does.
//
// Three kernels time the generator in the form the engine issues it, with the multiplier and the
// keys uniform (scalar registers) as in the engine:
//   * mad_u64_const: v_mad_u64_u32 with a scalar multiplier and a zero addend, 8 chains;
//   * philox_rounds: Philox4x32-10 rounds on two independent counters per lane (2 products and
//     2 three-input xors per round and counter);
//   * gen_noise: the engine's own per-agent code (cae_philox.h: the hoisted generator for a row of
//     agents, the offset and quantity reductions, the clamp and the book word of a NOISE order),
//     two rows per pass as in the engine, with the book word and quantity folded into a register
//     instead of an LDS atomic.  Its rate is the generator-alone ceiling of the order loop.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "cae_philox.h"

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
    K_MAD_U64_CONST = 10,
    K_PHILOX_ROUNDS = 11,
    K_GEN_NOISE = 12,
    K_LDS_RW_B64 = 13,
    K_GEN_NOISE4 = 14,
    K_ADD_SMUL = 15,  // v_add_u32 and s_mul_i32 alternating, eight independent chains of each
    K_SMUL = 16,      // s_mul_i32 alone
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
    uint32_t sc[8];
    const uint32_t sb = (uint32_t)__builtin_amdgcn_readfirstlane((int)(b | 1u));
#pragma unroll
    for (int j = 0; j < 8; ++j) sc[j] = (uint32_t)__builtin_amdgcn_readfirstlane((int)(blockIdx.x + 3u * (uint32_t)j));
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
            } else if constexpr (KIND == K_ADD_SMUL) {
                // scalar products leave SCC alone, so the loop's own compare is undisturbed
                asm volatile("v_add_u32 %0, %0, %1" : "+v"(a[j]) : "v"(b));
                asm volatile("s_mul_i32 %0, %0, %1" : "+s"(sc[j]) : "s"(sb));
            } else if constexpr (KIND == K_SMUL) {
                asm volatile("s_mul_i32 %0, %0, %1" : "+s"(sc[j]) : "s"(sb));
            }
        }
    }
    __syncthreads();  // the loop ends when the workgroup's last wave ends
    stamp(clk, c1, r1);
    uint32_t r = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j)
        r ^= a[j] ^ (uint32_t)p[j] ^ (uint32_t)(p[j] >> 32) ^ (uint32_t)f[j] ^ (uint32_t)g[j] ^ sc[j];
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

// The clearing's LDS traffic: each lane reads a (bid, ask) pair with ds_read_b64, adds to both
// words and writes the pair back with ds_write_b64; four independent pairs per lane (lane l of a
// wave owns pairs l, 64 + l, 128 + l, 192 + l of the wave's own region, so a wave's accesses
// cover consecutive 8-byte slots without bank conflicts).  16 lane-words moved per iteration.
__global__ void __launch_bounds__(1024) ub_lds_rw(uint32_t *out, uint64_t *clk, uint32_t iters, uint32_t seed)
{
    __shared__ uint2 pairs[16][256];
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    for (uint32_t i = threadIdx.x; i < 16 * 256; i += blockDim.x) (&pairs[0][0])[i] = make_uint2(0u, 0u);
    __syncthreads();
    uint64_t c0, r0, c1, r1;
    stamp(clk, c0, r0);
    for (uint32_t i = 0; i < iters; ++i) {
        uint2 v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = pairs[wave][64u * j + lane];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            v[j].x += seed;
            v[j].y += i;
            pairs[wave][64u * j + lane] = v[j];
        }
    }
    __syncthreads();
    stamp(clk, c1, r1);
    if (threadIdx.x == 0) {
        clk[2 * blockIdx.x] = c1 - c0;
        clk[2 * blockIdx.x + 1] = r1 - r0;
    }
    const uint2 a = pairs[wave][lane], b = pairs[wave][192u + lane];
    out[blockIdx.x * blockDim.x + threadIdx.x] = a.x ^ a.y ^ b.x ^ b.y;
}

// 8 chains of v_mad_u64_u32 with a uniform multiplier and no addend; the high word feeds the
// next product of its chain (a sub-register, no extra instruction).  The carry-out goes to a
// scalar register pair that nothing reads, as in the compiler's code for the engine.
__global__ void __launch_bounds__(1024) ub_mad_const(uint32_t *out, uint64_t *clk, uint32_t iters, uint32_t mul)
{
    uint32_t x[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) x[j] = threadIdx.x * 7u + (uint32_t)j * 13u + 1u;
    __syncthreads();
    uint64_t c0, r0, c1, r1;
    stamp(clk, c0, r0);
    for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            // the engine's form of a Philox product (both halves of it live on in the engine, so
            // the compiler cannot narrow it to a multiply-high; here it is written out)
            uint64_t p, carry;
            asm volatile("v_mad_u64_u32 %0, %1, %2, %3, 0" : "=v"(p), "=s"(carry) : "v"(x[j]), "s"(mul));
            x[j] = (uint32_t)(p >> 32);
        }
    }
    __syncthreads();
    stamp(clk, c1, r1);
    uint32_t r = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) r ^= x[j];
    out[blockIdx.x * blockDim.x + threadIdx.x] = r;
    if (threadIdx.x == 0) {
        clk[2 * blockIdx.x] = c1 - c0;
        clk[2 * blockIdx.x + 1] = r1 - r0;
    }
}

// Philox4x32-10 on two counters per lane per iteration (10 rounds each: 40 products and 40
// three-input xors per lane per iteration), keys uniform.
__global__ void __launch_bounds__(1024) ub_philox_rounds(uint32_t *out, uint64_t *clk, uint32_t iters, uint32_t k0,
                                                         uint32_t k1)
{
    uint32_t a[4], b[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        a[j] = threadIdx.x * 7u + (uint32_t)j;
        b[j] = threadIdx.x * 11u + (uint32_t)j * 3u;
    }
    __syncthreads();
    uint64_t c0, r0, c1, r1;
    stamp(clk, c0, r0);
    for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
        for (uint32_t r = 0; r < 10; ++r) {
            const uint32_t q0 = k0 + r * kW0, q1 = k1 + r * kW1;
            uint32_t h0, l0, h1, l1, g0, m0, g1, m1;
            mulhilo(kM0, a[0], h0, l0);
            mulhilo(kM1, a[2], h1, l1);
            mulhilo(kM0, b[0], g0, m0);
            mulhilo(kM1, b[2], g1, m1);
            a[0] = xor3(h1, a[1], q0);
            a[2] = xor3(h0, a[3], q1);
            a[1] = l1;
            a[3] = l0;
            b[0] = xor3(g1, b[1], q0);
            b[2] = xor3(g0, b[3], q1);
            b[1] = m1;
            b[3] = m0;
        }
        a[1] ^= i;  // a new counter every iteration
    }
    __syncthreads();
    stamp(clk, c1, r1);
    out[blockIdx.x * blockDim.x + threadIdx.x] = a[0] ^ a[1] ^ a[2] ^ a[3] ^ b[0] ^ b[1] ^ b[2] ^ b[3];
    if (threadIdx.x == 0) {
        clk[2 * blockIdx.x] = c1 - c0;
        clk[2 * blockIdx.x + 1] = r1 - r0;
    }
}

// The engine's NOISE-order code for 2 x 64 agents per wave and iteration (two rows at uniform
// bases, as the engine's order loop issues them), one market-step per `rows` iterations.  The
// book word 2 tick + side and the quantity of every order are folded into one register.
template <int NR>
__global__ void __launch_bounds__(1024) ub_gen_noise(uint32_t *out, uint64_t *clk, uint32_t iters, uint32_t k0,
                                                     uint32_t k1)
{
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t m = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);  // one "market" per wave
    const uint32_t span = 33u, Q = 100u;                                  // K = 16, quantities 1..100
    const int top = 255, base = 128 - 16;
    uint32_t acc = 0;
    __syncthreads();
    uint64_t c0, r0, c1, r1;
    stamp(clk, c0, r0);
    constexpr uint32_t rows = 8;  // 16 rows of 64 agents per market-step (A = 1024)
    for (uint32_t i = 0; i < iters; i += rows) {
        const PhiloxStep gen(i / rows, __builtin_amdgcn_readfirstlane(m), k0, k1);
        for (uint32_t j = 0; j < rows * 2u / NR; ++j) {
            const uint32_t bb = j * 64u * NR;
#pragma unroll
            for (int r = 0; r < NR; r += 2) {
                uint32_t w0, w1, w2, w3, x0, x1, x2, x3;
                gen.words4_row(bb + 64u * r, lane, w0, w1, w2, w3);
                gen.words4_row(bb + 64u * r + 64u, lane, x0, x1, x2, x3);
                const uint32_t wa = 2u * (uint32_t)clamp_tick(base + (int)__umulhi(w1, span), top) + (w0 >> 31);
                const uint32_t wb = 2u * (uint32_t)clamp_tick(base + (int)__umulhi(x1, span), top) + (x0 >> 31);
                acc = xor3(acc, wa, qty1(w2, Q));
                acc = xor3(acc, wb, qty1(x2, Q));
            }
        }
    }
    __syncthreads();
    stamp(clk, c1, r1);
    out[blockIdx.x * blockDim.x + threadIdx.x] = acc;
    if (threadIdx.x == 0) {
        clk[2 * blockIdx.x] = c1 - c0;
        clk[2 * blockIdx.x + 1] = r1 - r0;
    }
}

}  // namespace

extern "C" {

// Runs one microbenchmark: `blocks` workgroups of `threads` threads (64..1024), `iters` iterations
// (8 operations per lane for the single-instruction kinds; 80 instructions per lane for
// philox_rounds; 16 LDS words read or written per lane for lds_rw_b64; 128 agent events per wave
// for gen_noise and gen_noise4 (two or four rows of agents per pass), whose iters must be a
// multiple of 8).  Writes the elapsed milliseconds to *ms and, per workgroup, the shader
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
    case K_ADD_SMUL: hipLaunchKernelGGL(ub_valu<K_ADD_SMUL>, g, b, 0, nullptr, out, clk, iters, 1u); break;
    case K_SMUL: hipLaunchKernelGGL(ub_valu<K_SMUL>, g, b, 0, nullptr, out, clk, iters, 1u); break;
    case K_LDS_RW_B64: hipLaunchKernelGGL(ub_lds_rw, g, b, 0, nullptr, out, clk, iters, 1u); break;
    case K_MAD_U64_CONST: hipLaunchKernelGGL(ub_mad_const, g, b, 0, nullptr, out, clk, iters, kM0); break;
    case K_PHILOX_ROUNDS: hipLaunchKernelGGL(ub_philox_rounds, g, b, 0, nullptr, out, clk, iters, 1u, 2u); break;
    case K_GEN_NOISE:
        if (iters % 8u) {
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            return -1;
        }
        hipLaunchKernelGGL(ub_gen_noise<2>, g, b, 0, nullptr, out, clk, iters, 1u, 0u);
        break;
    case K_GEN_NOISE4:
        if (iters % 8u) {
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            return -1;
        }
        hipLaunchKernelGGL(ub_gen_noise<4>, g, b, 0, nullptr, out, clk, iters, 1u, 0u);
        break;
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
