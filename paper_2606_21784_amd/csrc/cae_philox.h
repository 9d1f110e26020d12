// cae_philox.h -- the per-agent order generator shared by the engine (cae_engine.hip) and the
// issue-rate microbenchmarks (cae_ubench.hip), so that the microbenchmark times exactly the
// instruction stream the engine issues per agent event.
//
// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11), the counter-based generator that stands in
// for the paper's hashed SplitMix64 stream (section III-G), evaluated at counter (s, a, m, 0) with
// key (k0, k1); and the two range reductions of the order rules (section III-C).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

constexpr uint32_t kM0 = 0xD2511F53u;
constexpr uint32_t kM1 = 0xCD9E8D57u;
constexpr uint32_t kW0 = 0x9E3779B9u;
constexpr uint32_t kW1 = 0xBB67AE85u;

// a ^ b ^ c in one gfx950 VALU op (v_bitop3_b32 with the truth table of a three-way xor)
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ void mulhilo(uint32_t m, uint32_t x, uint32_t &hi, uint32_t &lo)
{
    const uint64_t p = (uint64_t)m * (uint64_t)x;
    hi = (uint32_t)(p >> 32);
    lo = (uint32_t)p;
}

// Philox4x32-10 for counter (s, a, m, 0) and key (k0, k1), split into the part that is the same
// for every agent of a market-step (rounds 1-3 without the agent word) and the per-agent rest.
struct PhiloxStep {
    uint32_t ua, ux3k, uz0, uz2, z3k, k0, k1;

    __device__ __forceinline__ PhiloxStep(uint32_t s, uint32_t m, uint32_t key0, uint32_t key1)
    {
        uint32_t h0, l0, h1, l1;
        // round 1 (key k): products of the step and market words
        mulhilo(kM0, s, h0, l0);
        mulhilo(kM1, m, h1, l1);
        ua = h1 ^ key0;  // x0 = ua ^ a
        const uint32_t x1 = l1, x2 = h0 ^ key1, x3 = l0;
        // round 2 (key k + W): the x2 product is agent-independent
        mulhilo(kM1, x2, h1, l1);
        const uint32_t y0 = h1 ^ x1 ^ (key0 + kW0);
        const uint32_t y1 = l1;
        ux3k = x3 ^ (key1 + kW1);  // y2 = hi(M0 x0) ^ ux3k, y3 = lo(M0 x0)
        // round 3 (key k + 2W): the y0 product is agent-independent
        mulhilo(kM0, y0, h0, l0);
        uz0 = y1 ^ (key0 + 2u * kW0);  // z0 = hi(M1 y2) ^ uz0, z1 = lo(M1 y2)
        uz2 = h0 ^ (key1 + 2u * kW1);  // z2 = uz2 ^ y3
        z3k = l0 ^ (key1 + 3u * kW1);  // z3 = lo(M0 y0) is agent-independent: round 4 adds it to its key
        k0 = key0;
        k1 = key1;
    }

    __device__ __forceinline__ void words(uint32_t a, uint32_t &w0, uint32_t &w1, uint32_t &w2) const
    {
        uint32_t w3;
        words4(a, w0, w1, w2, w3);
    }

    __device__ __forceinline__ void words4(uint32_t a, uint32_t &w0, uint32_t &w1, uint32_t &w2,
                                           uint32_t &w3) const
    {
        words4x(ua ^ a, w0, w1, w2, w3);
    }

    // Agent b | t for a row base b (uniform) and a lane offset t below b's lowest set bit: the
    // first product's input ua ^ a = (ua ^ b) ^ t, whose uniform half is scalar work.
    __device__ __forceinline__ void words4_row(uint32_t b, uint32_t t, uint32_t &w0, uint32_t &w1, uint32_t &w2,
                                               uint32_t &w3) const
    {
        words4x((ua ^ b) ^ t, w0, w1, w2, w3);
    }

    __device__ __forceinline__ void words4x(uint32_t x0, uint32_t &w0, uint32_t &w1, uint32_t &w2,
                                            uint32_t &w3) const
    {
        uint32_t h, l;
        mulhilo(kM0, x0, h, l);
        const uint32_t y2 = h ^ ux3k, y3 = l;
        mulhilo(kM1, y2, h, l);
        const uint32_t z0 = h ^ uz0, z1 = l, z2 = uz2 ^ y3;
        // round 4 (key k + 3W)
        uint32_t h0, l0, h1, l1;
        mulhilo(kM0, z0, h0, l0);
        mulhilo(kM1, z2, h1, l1);
        uint32_t c0 = xor3(h1, z1, k0 + 3u * kW0), c1 = l1, c2 = h0 ^ z3k, c3 = l0;
#pragma unroll
        for (uint32_t r = 4; r < 10; ++r) {  // rounds 5..10 use key k + r W
            uint32_t h0, l0, h1, l1;
            mulhilo(kM0, c0, h0, l0);
            mulhilo(kM1, c2, h1, l1);
            c0 = xor3(h1, c1, k0 + r * kW0);
            c2 = xor3(h0, c3, k1 + r * kW1);
            c1 = l1;
            c3 = l0;
        }
        w0 = c0;
        w1 = c1;
        w2 = c2;
        w3 = c3;
    }
};

// A tick clamped to [0, top] (top >= 0) in one v_med3_i32 (top may differ between lanes: the
// naive engine runs one market per lane).
__device__ __forceinline__ int clamp_tick(int x, int top)
{
    int r;
    asm("v_med3_i32 %0, %1, 0, %2" : "=v"(r) : "v"(x), "v"(top));
    return r;
}

// 1 + floor(w2 Q / 2^32): the high word of w2 Q + 2^32, one multiply-add
__device__ __forceinline__ uint32_t qty1(uint32_t w2, uint32_t Q)
{
    return (uint32_t)(((uint64_t)w2 * Q + (1ull << 32)) >> 32);
}

}  // namespace
