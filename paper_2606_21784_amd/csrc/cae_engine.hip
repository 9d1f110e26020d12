// cae_engine.hip -- persistent call-auction ensemble engine for gfx950 (MI355X) and its C ABI.
//
// Method: KineticSim paper, section II-A (Eq. 1, Eq. 2: cumulative demand/supply, clearing price
// of maximal executable volume), section III-B..E (books resident in on-chip memory for all S
// steps of a launch, orders aggregated with on-chip atomics, cooperative clearing, residual book
// carried across steps), Algorithm 1 (the persistent per-market step loop).
//
// gfx950 design (what differs from the paper's CUDA design, and why):
//   * A market is owned by a group of `wpm` wave64s (1..16).  All of them generate orders
//     (agents strided over the group's lanes) and add them to the book in LDS with ds_add_u32.
//     ONE wave then clears the whole book: each lane owns TPL contiguous ticks, in-lane serial
//     sums plus a wave64 DPP scan give D and S, two ballots at the crossing of D and S give the
//     maximal volume and its lowest tick (no max reduction), and the fill uses the closed form
//        fill_bid(q) = min(D(q), V*) - min(D(q+1), V*),  fill_ask(q) = min(S(q), V*) - min(S(q-1), V*)
//     (books of at most 4 ticks per lane keep the residuals as max(D(q) - V*, 0) - max(D(q+1) - V*, 0)
//     and the ask counterpart).
//     No cross-wave scan pass and only two barriers per step; the clearing wave rotates with the
//     step so the clearing work spreads over the CU's four SIMDs.  Optionally (last-tick model)
//     the other waves generate the NEXT step's orders while the clearing runs, aggregated by
//     their offset from the not-yet-known reference; the clearing wave adds them to the book
//     once the price is known: one barrier per step and no wave waits for a clearing.
//   * Books are uint32 (exact integers; a host-side guard proves no overflow), stored in LDS as
//     interleaved (bid, ask) pairs so the clearing wave reads a tick with one 64-bit access.
//   * The order generator is Philox4x32-10 with counter (step, agent, market, 0): the first round
//     multiplies only the step and market words, so the products of rounds 1-3 that do not depend
//     on the agent are computed once per step in scalar registers.
//   * Work items (one market, or several equal-size markets sharing a workgroup in lock-step) are
//     claimed from an on-device queue in longest-first order, so markets of uneven size run in a
//     single launch; the last workgroup to finish resets the queue for the next launch.
//   * HBM is read when an item starts (book + state) and written when it ends: traffic per launch
//     is independent of S.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "cae.h"
#include "cae_philox.h"

namespace {

// ------------------------------------------------------------------------------------------
// Device-side data (workspace layout is private to this file).
// ------------------------------------------------------------------------------------------
struct DevMarket {
    uint32_t L, A, K, Q;
    uint32_t n_noise, n_mom, h, tpl;  // tpl: ticks per lane of the clearing wave (power of 2)
    uint64_t book_off;                // word offset of bid[0]; ask[0] is at book_off + L
    uint32_t id;                      // market index in the generator counter
    uint32_t flags;                   // agent model (bits 0-7) and P_mkt (bits 16-31)
};
static_assert(sizeof(DevMarket) == 48, "DevMarket layout");

struct Item {
    uint32_t first;     // index into the market order list
    uint32_t count;     // markets in this item
    uint32_t wpm_log2;  // log2(waves per market) (single-wave or lock-step items)
    uint32_t stride;    // LDS words per market slice (book pairs + kScr scratch words)
    uint32_t pipe;      // 1: two markets share all the workgroup's waves in alternating phases;
                        // 2: lock-step with the next step's orders generated during the clearing
    uint32_t share;     // pipe 2: rows of 64 agents the clearing wave generates after clearing
    uint32_t hoff;      // pipe 2: word offset of the two order-bin buffers in a market slice
    uint32_t hwords;    // pipe 2: words per order-bin buffer
    uint32_t boost;     // 1: its waves issue one priority level above other items' (see base_prio)
};

constexpr uint32_t kScr = 32;  // scratch words at the end of every market slice

struct EngineArgs {
    const DevMarket *desc;
    const uint32_t *order;
    const Item *items;
    uint32_t *ctr;  // [0] next item, [1] finished claimers
    uint32_t *book;
    cae_state *state;
    const double *lnT;  // lnT[n] = ln(n), n in [0, 2048]
    uint32_t *tr_price;  // optional per-step series, row m at m * tr_ld: last tick after step i
    uint32_t *tr_vol;    // and the volume executed in step i
    uint64_t tr_ld;
    uint32_t n_items;
    uint32_t n_claimers;
    uint32_t S;
    uint32_t k0, k1;
};

// Records step i of market m in the optional series (one lane per market-step).
__device__ __forceinline__ void trace_step(const EngineArgs &args, uint32_t m, uint32_t i, uint32_t last,
                                           uint32_t v)
{
    const uint64_t at = (uint64_t)m * args.tr_ld + i;
    if (args.tr_price != nullptr) args.tr_price[at] = last;
    if (args.tr_vol != nullptr) args.tr_vol[at] = v;
}

constexpr uint32_t kNone = 0xFFFFFFFFu;

// ------------------------------------------------------------------------------------------
// wave64 primitives (GFX9 DPP: row_shr within 16-lane rows, row_bcast:15/31 across rows).
// ------------------------------------------------------------------------------------------
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint32_t dpp(uint32_t x)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, ROW_MASK, 0xf, false);
}

// Two inclusive scans interleaved, so each DPP read follows an unrelated write (no wait states).
__device__ __forceinline__ void wave_scan_add2(uint32_t &x, uint32_t &y)
{
    x += dpp<0x111, 0xf>(x);
    y += dpp<0x111, 0xf>(y);
    x += dpp<0x112, 0xf>(x);
    y += dpp<0x112, 0xf>(y);
    x += dpp<0x114, 0xf>(x);
    y += dpp<0x114, 0xf>(y);
    x += dpp<0x118, 0xf>(x);
    y += dpp<0x118, 0xf>(y);
    x += dpp<0x142, 0xa>(x);
    y += dpp<0x142, 0xa>(y);
    x += dpp<0x143, 0xc>(x);
    y += dpp<0x143, 0xc>(y);
}

__device__ __forceinline__ uint32_t readlane(uint32_t x, uint32_t l)
{
    return (uint32_t)__builtin_amdgcn_readlane((int)x, (int)l);
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// Orders LDS traffic of one wave with respect to itself (LDS executes one wave's accesses in
// issue order; this only keeps the compiler from moving accesses across the point).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Issue priority of a wave that is not clearing.  In a mixed ensemble the markets with the most
// work per step set the launch's length (every market runs the same number of steps), so their
// items may be boosted one level above the rest; `hi` selects the upper of the two levels a
// group alternates between (the clearing wave itself runs at 3).  Levels: boosted 2 / 1, others
// 1 / 0.  s_setprio takes an immediate, hence the branches.
__device__ __forceinline__ void base_prio(uint32_t boost, bool hi)
{
    if (boost) {
        if (hi) __builtin_amdgcn_s_setprio(2);
        else __builtin_amdgcn_s_setprio(1);
    } else {
        if (hi) __builtin_amdgcn_s_setprio(1);
        else __builtin_amdgcn_s_setprio(0);
    }
}

struct ClearOut {
    uint32_t p, v, bb, ba;  // clearing tick, volume, best bid / best ask after the fill (kNone: empty)
};

// max(x - v, 0) in one instruction (v_sub_u32 with clamp).  With it the price-priority fill is
// one subtract per tick and side: D(q) - min(D(q), V*) = max(D(q) - V*, 0) is the demand at or
// above q that stays unmatched, so the residual bids at q are max(D(q) - V*, 0) -
// max(D(q+1) - V*, 0), and the residual asks max(S(q) - V*, 0) - max(S(q-1) - V*, 0): the same
// numbers as b - (min(D(q), V*) - min(D(q+1), V*)) and its ask counterpart, with fewer steps.
__device__ __forceinline__ uint32_t unmatched(uint32_t x, uint32_t v) { return __builtin_elementwise_sub_sat(x, v); }

// min(x, 1) in one instruction, for counting ticks with a positive unmatched quantity.  Written
// out because the compiler's own form of the count (a compare and a carry-add per tick) puts
// every tick on the condition register, one after another with wait states between them.
__device__ __forceinline__ uint32_t nonzero(uint32_t x)
{
    uint32_t r;
    asm("v_min_u32 %0, 1, %1" : "=v"(r) : "v"(x));
    return r;
}

// Reads / writes CH consecutive (bid, ask) pairs starting at tick q of an LDS book.
template <int CH>
__device__ __forceinline__ void load_pairs(const uint32_t *bk, uint32_t q, uint32_t (&b)[CH], uint32_t (&k)[CH])
{
    if constexpr (CH == 1) {
        const uint2 v = reinterpret_cast<const uint2 *>(bk)[q];
        b[0] = v.x;
        k[0] = v.y;
    } else {
#pragma unroll
        for (int j = 0; j < CH / 2; ++j) {
            const uint4 v = reinterpret_cast<const uint4 *>(bk)[(q >> 1) + j];
            b[2 * j] = v.x;
            k[2 * j] = v.y;
            b[2 * j + 1] = v.z;
            k[2 * j + 1] = v.w;
        }
    }
}

template <int CH>
__device__ __forceinline__ void store_pairs(uint32_t *bk, uint32_t q, const uint32_t (&b)[CH], const uint32_t (&k)[CH])
{
    if constexpr (CH == 1) {
        reinterpret_cast<uint2 *>(bk)[q] = make_uint2(b[0], k[0]);
    } else {
#pragma unroll
        for (int j = 0; j < CH / 2; ++j)
            reinterpret_cast<uint4 *>(bk)[(q >> 1) + j] = make_uint4(b[2 * j], k[2 * j], b[2 * j + 1], k[2 * j + 1]);
    }
}

// Clearing price and volume without a cross-lane reduction.  D falls and S rises with the tick,
// so V = min(D, S) follows S up to the first tick qc with S(qc) >= D(qc) and follows D from there
// on: V* = max(S(qc - 1), D(qc)), or S of the top tick when no tick crosses.  A lane whose ticks
// start at q0 takes the candidate max(S(q0 - 1), max over its ticks of V), which equals V* in the
// lane holding qc (and in the top lane when nothing crosses); that lane is the first whose top
// tick has S >= D.  The lowest tick reaching V* is the lowest tick with S >= V* (before qc V is
// S, and when V* = D(qc) > S(qc - 1) the first tick with S >= V* is qc itself), so it is found
// the same way: in the first lane whose top tick has S >= V*, at that lane's count of ticks with
// S < V*.  crossing_lane returns the first lane where a predicate that holds on a suffix of the
// lanes is true, or 63 when it is true nowhere.
__device__ __forceinline__ uint32_t crossing_lane(bool pred)
{
    return (uint32_t)__builtin_ctzll(ballot(pred) | (1ull << 63));
}

// Clearing of a book of at most 4 ticks per lane, its ticks held in registers throughout: the
// demand D and supply S of every tick are formed once, the volume pass and the fill reuse them,
// and the fill leaves the residual of each tick as a difference of unmatched quantities:
// max(D(q) - V*, 0) - max(D(q+1) - V*, 0) bids, max(S(q) - V*, 0) - max(S(q-1) - V*, 0) asks.
// Every instruction here is on the step's critical path (one wave, the rest of the market
// waiting), so the pass is kept short.
template <int TPL>
__device__ __forceinline__ ClearOut clear_small(uint32_t *__restrict__ bk, uint32_t lane)
{
    const uint32_t q0 = lane * TPL;
    uint32_t b[TPL], k[TPL];
    load_pairs<TPL>(bk, q0, b, k);
    uint32_t sb = 0, sa = 0;
#pragma unroll
    for (int j = 0; j < TPL; ++j) {
        sb += b[j];
        sa += k[j];
    }
    uint32_t ib = sb, ia = sa;
    wave_scan_add2(ib, ia);
    const uint32_t Tb = readlane(ib, 63);
    uint32_t D[TPL + 1], Sq[TPL];  // D(q0 + j), S(q0 + j); D[TPL] = D(q0 + TPL)
    D[0] = Tb - (ib - sb);
    const uint32_t Sb = ia - sa;   // asks below this lane's first tick
#pragma unroll
    for (int j = 0; j < TPL; ++j) {
        D[j + 1] = D[j] - b[j];
        Sq[j] = (j ? Sq[j - 1] : Sb) + k[j];
    }
    uint32_t vc = Sb;
#pragma unroll
    for (int j = 0; j < TPL; ++j) vc = max(vc, min(D[j], Sq[j]));
    ClearOut out;
    out.v = readlane(vc, crossing_lane(Sq[TPL - 1] >= D[TPL - 1]));
    const uint32_t vs = out.v;
    {
        uint32_t pj = q0;
#pragma unroll
        for (int j = 0; j < TPL; ++j) pj += Sq[j] < vs ? 1u : 0u;
        out.p = readlane(pj, crossing_lane(Sq[TPL - 1] >= vs));
    }
    // Best quotes after the fill, from the curves: the unmatched demand max(D(q) - V*, 0) falls
    // with q and the residual bids are its drops, so the best bid is the highest tick with
    // D > V*; likewise the best ask is the lowest tick with S > V*.  The ticks with D > V* are a
    // prefix of the book (the last lane whose first tick is in it holds the best bid), those
    // with S <= V* too (the first lane whose top tick is past it holds the best ask).
    uint32_t ud = unmatched(D[0], vs), us = unmatched(Sb, vs);
    uint32_t nb = q0 - 1u, ns = 0;
#pragma unroll
    for (int j = 0; j < TPL; ++j) {
        const uint32_t ud1 = unmatched(D[j + 1], vs), us1 = unmatched(Sq[j], vs);
        nb += nonzero(ud);
        ns += nonzero(us1);
        b[j] = ud - ud1;
        k[j] = us1 - us;
        ud = ud1;
        us = us1;
    }
    store_pairs<TPL>(bk, q0, b, k);
    const uint64_t mb = ballot(D[0] > vs);
    const uint64_t ma = ballot(Sq[TPL - 1] > vs);
    out.bb = mb ? readlane(nb, 63u - (uint32_t)__builtin_clzll(mb)) : kNone;
    out.ba = ma ? readlane(q0 + TPL - ns, (uint32_t)__builtin_ctzll(ma)) : kNone;
    return out;
}

// Clears one book with one wave.  bk: LDS pairs (bid, ask) for ticks [0, 64*TPL), zero beyond L.
// Lane l owns ticks [l*TPL, l*TPL + TPL) and streams them from LDS in chunks of at most four
// ticks per pass (sums; volumes; fill), so registers do not grow with L.  Wave-uniform result.
template <int TPL>
__device__ __forceinline__ ClearOut clear_wave(uint32_t *__restrict__ bk, uint32_t lane)
{
    if constexpr (TPL <= 4) return clear_small<TPL>(bk, lane);
    constexpr int CH = TPL < 4 ? TPL : 4;
    constexpr int NCH = TPL / CH;
    const uint32_t q0 = lane * TPL;

    uint32_t sb = 0, sa = 0;  // this lane's bid and ask totals
#pragma unroll 2
    for (int c = 0; c < NCH; ++c) {
        uint32_t b[CH], k[CH];
        load_pairs<CH>(bk, q0 + c * CH, b, k);
#pragma unroll
        for (int j = 0; j < CH; ++j) {
            sb += b[j];
            sa += k[j];
        }
    }
    uint32_t ib = sb, ia = sa;
    wave_scan_add2(ib, ia);
    const uint32_t Tb = readlane(ib, 63);  // all bids
    const uint32_t eb = ib - sb;          // bids on ticks below this lane's first tick
    const uint32_t ea = ia - sa;          // asks on ticks below this lane's first tick

    // V(q) = min(D(q), S(q)); D(q) = Tb - bids below q; S(q) = asks at or below q.  The lane's
    // crossing-point candidate (see crossing_lane), and D of its top tick.
    uint32_t vc = ea, dtop = 0;
    {
        uint32_t cb = eb, ca = ea;
#pragma unroll 2
        for (int c = 0; c < NCH; ++c) {
            uint32_t b[CH], k[CH];
            load_pairs<CH>(bk, q0 + c * CH, b, k);
#pragma unroll
            for (int j = 0; j < CH; ++j) {
                dtop = Tb - cb;
                ca += k[j];
                vc = max(vc, min(dtop, ca));
                cb += b[j];
            }
        }
    }
    ClearOut out;
    out.v = readlane(vc, crossing_lane(ia >= dtop));  // ia: S of the lane's top tick

    // closed-form price-priority fill (all zero when V* = 0), then best bid / best ask; the
    // clearing tick is the lowest tick with S >= V*
    const uint32_t vs = out.v;
    // best quotes after the fill as in clear_small: the best bid is the highest tick with
    // D > V*, the best ask the lowest tick with S > V*
    uint32_t nb = q0 - 1u, na = q0 + TPL, pj = q0;
    {
        uint32_t cb = eb, ca = ea;
#pragma unroll 2
        for (int c = 0; c < NCH; ++c) {
            uint32_t b[CH], k[CH];
            const uint32_t qc = q0 + c * CH;
            load_pairs<CH>(bk, qc, b, k);
            bool changed = false;
#pragma unroll
            for (int j = 0; j < CH; ++j) {
                const uint32_t D = Tb - cb;
                const uint32_t Sq = ca + k[j];
                const uint32_t fb = min(D, vs) - min(D - b[j], vs);
                const uint32_t fs = min(Sq, vs) - min(ca, vs);
                cb += b[j];
                ca = Sq;
                b[j] -= fb;
                k[j] -= fs;
                pj += Sq < vs ? 1u : 0u;
                nb += nonzero(unmatched(D, vs));
                na -= nonzero(unmatched(Sq, vs));
                changed |= (fb | fs) != 0;
            }
            if (changed) store_pairs<CH>(bk, qc, b, k);
        }
    }
    out.p = readlane(pj, crossing_lane(ia >= vs));
    const uint64_t mb = ballot(Tb - eb > vs);  // D of the lane's first tick
    const uint64_t ma = ballot(ia > vs);       // S of the lane's top tick
    out.bb = mb ? readlane(nb, 63u - (uint32_t)__builtin_clzll(mb)) : kNone;
    out.ba = ma ? readlane(na, (uint32_t)__builtin_ctzll(ma)) : kNone;
    return out;
}

template <int TPL_MAX>
__device__ __forceinline__ ClearOut clear_dispatch(uint32_t *bk, uint32_t tpl, uint32_t lane)
{
    if constexpr (TPL_MAX >= 16) {
        if (tpl == 16) return clear_wave<16>(bk, lane);
    }
    if constexpr (TPL_MAX >= 8) {
        if (tpl == 8) return clear_wave<8>(bk, lane);
    }
    if constexpr (TPL_MAX >= 4) {
        if (tpl == 4) return clear_wave<4>(bk, lane);
    }
    if constexpr (TPL_MAX >= 2) {
        if (tpl == 2) return clear_wave<2>(bk, lane);
    }
    return clear_wave<1>(bk, lane);
}

// SplitMix64 words (the generator named in section III-G), for markets that select it: channel
// c of agent gid = m A + a at step s is the high half of mix(seed + (k + 1) g) with
// k = gid 2^34 + 4 s + c and g = 0x9e3779b97f4a7c15, i.e. mix(base_c + ((gid g mod 2^32) << 34))
// with base_c = seed + (4 s + c + 1) g uniform over the step.
constexpr uint64_t kGamma = 0x9e3779b97f4a7c15ull;

__device__ __forceinline__ uint32_t splitmix_hi(uint64_t x)
{
    uint64_t z = x;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return (uint32_t)((z ^ (z >> 31)) >> 32);
}

struct SplitMixStep {
    uint64_t base[4];
    uint32_t gid0;  // m A (mod 2^32)

    __device__ __forceinline__ SplitMixStep(uint32_t s, uint32_t m, uint32_t A, uint64_t seed)
    {
#pragma unroll
        for (uint32_t c = 0; c < 4; ++c) base[c] = seed + (4ull * s + c + 1ull) * kGamma;
        gid0 = m * A;
    }

    __device__ __forceinline__ void words4(uint32_t a, uint32_t &w0, uint32_t &w1, uint32_t &w2,
                                           uint32_t &w3) const
    {
        const uint64_t g = (uint64_t)((gid0 + a) * (uint32_t)kGamma) << 34;
        w0 = splitmix_hi(base[0] + g);
        w1 = splitmix_hi(base[1] + g);
        w2 = splitmix_hi(base[2] + g);
        w3 = splitmix_hi(base[3] + g);
    }

    __device__ __forceinline__ void words4_row(uint32_t b, uint32_t t, uint32_t &w0, uint32_t &w1, uint32_t &w2,
                                               uint32_t &w3) const
    {
        words4(b | t, w0, w1, w2, w3);
    }
};

__device__ __forceinline__ bool uses_splitmix(const DevMarket &d)
{
    return ((d.flags >> CAE_GEN_SHIFT) & 0xFFu) == CAE_GEN_SPLITMIX;
}

// The references the agents of a market read at the start of a step.
struct Refs {
    uint32_t last, prev;   // last clearing tick, and the one before the previous step
    uint32_t mid2, mid2p;  // mid-price model: 2 mid of this step and of the previous step
};

// The order rules of section III-C, shared by the persistent engine and the naive
// one-thread-per-market engine so both produce identical books.  Last-tick model: reference =
// last, momentum follows sign(last - prev).  Mid-price model: reference = mid (half-ticks,
// round(x) = floor(x + 1/2)), momentum follows sign(mid - mid of the previous step), NOISE and
// MOMENTUM orders are marketable with probability P_mkt.  Every value here is uniform.
struct OrderCtx {
    int base;           // last-tick NOISE: last - K
    uint32_t span;      // 2K + 1
    uint64_t nbase;     // mid-price NOISE: (2 mid + 1) 2^31 - K 2^32 (two's complement)
    uint32_t twoK;
    uint32_t tmkt;      // marketable iff w3 < tmkt (0 in the last-tick model)
    uint32_t Q;
    int top;            // L - 1
    uint32_t n_noise, mom_end, s;
    uint32_t mom_dir;   // 0 up (buy), 1 down (sell), 2 unchanged (coin)
    int mom_bid, mom_ask, mk_bid, mk_ask;  // unclamped ticks
    bool mid;
};

// FULL: the code may meet mid-price markets (false compiles the last-tick rules alone).
template <bool FULL>
__device__ __forceinline__ OrderCtx order_ctx(const DevMarket &d, uint32_t s, const Refs &r)
{
    OrderCtx o;
    o.mid = FULL && (d.flags & CAE_MODEL_MASK) == CAE_MODEL_MID;
    o.span = 2u * d.K + 1u;
    o.twoK = 2u * d.K;
    o.Q = d.Q;
    o.top = (int)d.L - 1;
    o.n_noise = d.n_noise;
    o.mom_end = d.n_noise + d.n_mom;
    o.s = s;
    const int h = (int)d.h;
    if (o.mid) {
        const int m2 = (int)r.mid2;
        o.base = 0;
        o.nbase = ((uint64_t)(r.mid2 + 1u) << 31) - ((uint64_t)d.K << 32);
        o.tmkt = (d.flags >> CAE_PMKT_SHIFT) << CAE_PMKT_SHIFT;
        o.mom_dir = r.mid2 > r.mid2p ? 0u : (r.mid2 < r.mid2p ? 1u : 2u);
        o.mom_bid = (m2 + 3) >> 1;           // round(mid + 1)
        o.mom_ask = (m2 - 1) >> 1;           // round(mid - 1)
        o.mk_bid = (m2 - 2 * h + 1) >> 1;    // round(mid - h)
        o.mk_ask = (m2 + 2 * h + 1) >> 1;    // round(mid + h)
    } else {
        const int l = (int)r.last;
        o.base = l - (int)d.K;
        o.nbase = 0;
        o.tmkt = 0;
        o.mom_dir = r.last > r.prev ? 0u : (r.last < r.prev ? 1u : 2u);
        o.mom_bid = l + 1;
        o.mom_ask = l - 1;
        o.mk_bid = l - h;
        o.mk_ask = l + h;
    }
    return o;
}


__device__ __forceinline__ uint32_t order_qty(const OrderCtx &o, uint32_t w2) { return qty1(w2, o.Q); }

// Last-tick NOISE agent: fair coin for the side (w0), uniform offset in {-K..K} (w1); book
// word 2*tick+side.
__device__ __forceinline__ uint32_t noise_word(const OrderCtx &o, uint32_t w0, uint32_t w1)
{
    const int tick = clamp_tick(o.base + (int)__umulhi(w1, o.span), o.top);
    return 2u * (uint32_t)tick + (w0 >> 31);
}

// Mid-price NOISE agent: tick = floor(mid + K (2 w1 / 2^32 - 1) + 1/2), the high word of a
// 64-bit fixed-point sum with 32 fraction bits; marketable when w3 < tmkt.
__device__ __forceinline__ uint32_t mid_noise_word(const OrderCtx &o, uint32_t w0, uint32_t w1, uint32_t w3)
{
    const uint32_t sell = w0 >> 31;
    int tick = (int)(uint32_t)((o.nbase + (uint64_t)o.twoK * (uint64_t)w1) >> 32);
    if (w3 < o.tmkt) tick = sell ? 0 : o.top;
    tick = clamp_tick(tick, o.top);
    return 2u * (uint32_t)tick + sell;
}

// MOMENTUM (a < mom_end) or MAKER agent a, either model.
template <bool FULL>
__device__ __forceinline__ uint32_t other_word(const OrderCtx &o, uint32_t a, uint32_t w0, uint32_t w3)
{
    // tick = bid tick + sell x (ask tick - bid tick), written as arithmetic so that the four
    // candidate ticks are not gathered into an indexed table in private memory
    const bool mom = a < o.mom_end;
    const uint32_t sell = mom ? (o.mom_dir == 2u ? (w0 >> 31) : o.mom_dir) : ((a ^ o.s) & 1u);
    const int lo = mom ? o.mom_bid : o.mk_bid;
    const int span = mom ? o.mom_ask - o.mom_bid : o.mk_ask - o.mk_bid;
    int tick = lo + (int)sell * span;
    if (FULL && mom && w3 < o.tmkt) tick = sell ? 0 : o.top;
    tick = clamp_tick(tick, o.top);
    return 2u * (uint32_t)tick + sell;
}

// Every order of one market-step, added into the LDS book (interleaved pairs: word 2*tick+side).
// Agents run in rows of nthr at uniform bases b: agent b + t for t < nthr.  POW2: nthr is a power
// of two, so b + t = b | t and the generator folds the uniform half of its input in scalar work.
template <bool POW2, typename Gen>
__device__ __forceinline__ void row_words(const Gen &gen, uint32_t b, uint32_t t, uint32_t &w0, uint32_t &w1,
                                          uint32_t &w2, uint32_t &w3)
{
    if constexpr (POW2) gen.words4_row(b, t, w0, w1, w2, w3);
    else gen.words4(b + t, w0, w1, w2, w3);
}

template <bool FULL, bool POW2, typename Gen>
__device__ __forceinline__ void gen_with(const DevMarket &d, const OrderCtx &o, const Gen &gen, uint32_t t,
                                         uint32_t nthr, uint32_t *bk)
{
    const uint32_t nn = d.n_noise;
    uint32_t b = 0;
    if (FULL && o.mid) {
        for (; b + nthr <= nn; b += nthr) {
            uint32_t w0, w1, w2, w3;
            row_words<POW2>(gen, b, t, w0, w1, w2, w3);
            atomicAdd(&bk[mid_noise_word(o, w0, w1, w3)], order_qty(o, w2));
        }
    } else {
        // two full rows per pass: two independent generator chains for the wave to issue from
        for (; b + 2u * nthr <= nn; b += 2u * nthr) {
            uint32_t w0, w1, w2, w3, x0, x1, x2, x3;
            row_words<POW2>(gen, b, t, w0, w1, w2, w3);
            row_words<POW2>(gen, b + nthr, t, x0, x1, x2, x3);
            atomicAdd(&bk[noise_word(o, w0, w1)], order_qty(o, w2));
            atomicAdd(&bk[noise_word(o, x0, x1)], order_qty(o, x2));
        }
    }
    // the rest: a NOISE row cut by the class boundary, then MOMENTUM and MAKER agents
    for (; b < d.A; b += nthr) {
        const uint32_t a = b + t;
        if (a < d.A) {
            uint32_t w0, w1, w2, w3 = 0;
            row_words<POW2>(gen, b, t, w0, w1, w2, w3);
            const uint32_t w = a >= nn ? other_word<FULL>(o, a, w0, w3)
                               : (FULL && o.mid) ? mid_noise_word(o, w0, w1, w3)
                                                 : noise_word(o, w0, w1);
            atomicAdd(&bk[w], order_qty(o, w2));
        }
    }
}

template <bool FULL, bool POW2 = true>
__device__ __forceinline__ void gen_orders(const DevMarket &d, uint32_t m, uint32_t s, const Refs &r,
                                           uint32_t key0, uint32_t key1, uint32_t t, uint32_t nthr,
                                           uint32_t *bk)
{
    const OrderCtx o = order_ctx<FULL>(d, s, r);
    if (FULL && uses_splitmix(d)) {
        gen_with<FULL, POW2>(d, o, SplitMixStep(s, m, d.A, ((uint64_t)key1 << 32) | key0), t, nthr, bk);
        return;
    }
    gen_with<FULL, POW2>(d, o, PhiloxStep(s, m, key0, key1), t, nthr, bk);
}

// Last-tick orders of step s aggregated by their position relative to the reference, before the
// reference is known (section III-C: no rule of the last-tick model looks at the price until the
// tick is formed).  Bins, as (bid, ask) pairs: pair o < 2K+1 holds the NOISE orders of offset
// o - K; pair 2K+1 the MOMENTUM quantities by their coin (the trend decides at the flush whether
// the coin or the trend picks the side); pair 2K+2 the MAKER quantities by side.  Agents
// b | lane for the row bases b = b0, b0 + stride, ... (multiples of 64), below `end`.
template <typename Gen>
__device__ __forceinline__ void gen_rel(const DevMarket &d, uint32_t s, const Gen &gen, uint32_t b0,
                                        uint32_t stride, uint32_t end, uint32_t lane, uint32_t *H)
{
    // rows of 64 agents b | lane at the uniform bases b0, b0 + stride, ... (multiples of 64)
    const uint32_t span = 2u * d.K + 1u;
    const uint32_t nend = min(d.n_noise, end);
    uint32_t b = b0;
    // two full NOISE rows per pass: two independent generator chains for the wave to issue from
    for (; b + stride + 64u <= nend; b += 2u * stride) {
        uint32_t w0, w1, w2, w3, x0, x1, x2, x3;
        gen.words4_row(b, lane, w0, w1, w2, w3);
        gen.words4_row(b + stride, lane, x0, x1, x2, x3);
        atomicAdd(&H[2u * __umulhi(w1, span) + (w0 >> 31)], qty1(w2, d.Q));
        atomicAdd(&H[2u * __umulhi(x1, span) + (x0 >> 31)], qty1(x2, d.Q));
    }
    const uint32_t mom_end = d.n_noise + d.n_mom;
    for (; b < end; b += stride) {
        const uint32_t a = b | lane;
        if (a < end) {
            uint32_t w0, w1, w2, w3;
            gen.words4_row(b, lane, w0, w1, w2, w3);
            const uint32_t bin = a < nend ? 2u * __umulhi(w1, span) + (w0 >> 31)
                                          : 2u * span + (a < mom_end ? (w0 >> 31) : 2u + ((a ^ s) & 1u));
            atomicAdd(&H[bin], qty1(w2, d.Q));
        }
    }
}

// Adds the bins of one step to the book at reference `last` (momentum direction from last vs
// prev, as order_ctx) and clears them.  Lane j < 2K+1 adds noise pair j at tick last - K + j;
// lanes 2K+1 .. 2K+4 add the momentum buys (last + 1), momentum sells (last - 1), maker bids
// (last - h) and maker asks (last + h); every tick clamped to the book.  One 64-bit LDS add per
// lane, without branches (a tick's bid count cannot carry into its ask count: the host guard
// keeps every count below 2^32).  One wave.
__device__ __forceinline__ void flush_rel(const DevMarket &d, uint32_t last, uint32_t prev, uint32_t *H,
                                          uint32_t *bk, uint32_t lane)
{
    const uint32_t span = 2u * d.K + 1u;
    const int l = (int)last, top = (int)d.L - 1, h = (int)d.h;
    const bool up = last > prev, down = last < prev, flat = last == prev;
    uint2 *P = reinterpret_cast<uint2 *>(H);
    for (uint32_t j0 = 0; j0 < span + 4u; j0 += 64u) {
        const uint32_t j = j0 + lane;
        const uint32_t e = j - span;  // 0..3 for the momentum and maker lanes
        const bool noise = j < span;
        const uint32_t pj = noise ? j : span + min(e >> 1, 1u);
        const uint2 v = P[min(pj, span + 1u)];
        // momentum: buys take everything when the trend is up, the coin's buys when it is flat
        const uint32_t mom = v.x + v.y;
        const uint32_t mbuy = up ? mom : (flat ? v.x : 0u);
        const uint32_t msell = down ? mom : (flat ? v.y : 0u);
        uint32_t lo, hi;
        int tick;
        if (noise) {
            lo = v.x;
            hi = v.y;
            tick = l - (int)d.K + (int)j;
        } else {
            lo = e == 0u ? mbuy : (e == 2u ? v.x : 0u);
            hi = e == 1u ? msell : (e == 3u ? v.y : 0u);
            const int dlt = (e & 2u) ? h : 1;
            tick = (e == 1u || e == 2u) ? l - dlt : l + dlt;
        }
        tick = clamp_tick(tick, top);
        if (j < span + 4u)
            atomicAdd(reinterpret_cast<unsigned long long *>(bk) + tick, ((unsigned long long)hi << 32) | lo);
    }
    // after every pass has read its bins (one wave's LDS accesses execute in order)
    for (uint32_t j0 = 0; j0 < span + 2u; j0 += 64u)
        if (j0 + lane < span + 2u) P[j0 + lane] = make_uint2(0u, 0u);
}

// The same flush when the bins fit one pass (2K + 5 <= 64 lanes), with each lane's role fixed
// for the market: the pair it reads, its tick relative to the reference, and masks that pick
// which bin words go to the bid and to the ask.  Only the momentum lanes' masks depend on the
// step (through the trend), so a step's flush is a few masks, one read, one 64-bit add and the
// bins' reset, without branches.
struct FlushLanes {
    uint32_t pj;        // bin pair the lane reads
    int dt;             // its tick relative to the reference
    uint32_t bx, ay;    // ~0: the pair's bid word goes to the bid / its ask word to the ask
    uint32_t mb, ms;    // ~0: the momentum-buy lane / the momentum-sell lane
};

// A per-lane value the compiler must keep as a vector word (it would otherwise turn the masks
// into lane masks held in scalar registers, which the step loop cannot spare).
__device__ __forceinline__ uint32_t vword(uint32_t x)
{
    asm volatile("" : "+v"(x));
    return x;
}

__device__ __forceinline__ FlushLanes flush_lanes(const DevMarket &d, uint32_t lane)
{
    const uint32_t span = 2u * d.K + 1u;
    const uint32_t e = lane - span;  // 0..3 for the momentum and maker lanes
    const bool noise = lane < span;
    FlushLanes f;
    f.pj = noise ? lane : span + min(e >> 1, 1u);
    // lanes past the four momentum and maker lanes add zero at distinct ticks (no collisions)
    f.dt = (noise || e > 3u) ? (int)lane - (int)d.K
                              : (e == 0u ? 1 : (e == 1u ? -1 : (e == 2u ? -(int)d.h : (int)d.h)));
    f.bx = vword((noise || e == 2u) ? ~0u : 0u);
    f.ay = vword((noise || e == 3u) ? ~0u : 0u);
    f.mb = vword((!noise && e == 0u) ? ~0u : 0u);
    f.ms = vword((!noise && e == 1u) ? ~0u : 0u);
    return f;
}

__device__ __forceinline__ void flush_rel_lanes(const FlushLanes &f, uint32_t span, int top, uint32_t last,
                                                uint32_t prev, uint32_t *H, uint32_t *bk, uint32_t lane)
{
    const uint32_t up = last > prev ? ~0u : 0u, dn = last < prev ? ~0u : 0u, flat = last == prev ? ~0u : 0u;
    uint2 *P = reinterpret_cast<uint2 *>(H);
    const uint2 v = P[f.pj];
    // momentum buys take both coins' quantities when the trend is up, the coin's buys when it is
    // flat; sells alike
    const uint32_t lo = (v.x & (f.bx | (f.mb & (up | flat)))) + (v.y & f.mb & up);
    const uint32_t hi = (v.x & f.ms & dn) + (v.y & (f.ay | (f.ms & (dn | flat))));
    const int tick = clamp_tick((int)last + f.dt, top);
    atomicAdd(reinterpret_cast<unsigned long long *>(bk) + tick, ((unsigned long long)hi << 32) | lo);
    // after the reads (one wave's LDS accesses execute in order)
    if (lane < span + 2u) P[lane] = make_uint2(0u, 0u);
}

// Mid-price orders of step s aggregated before the reference 2 mid = 2n + e is known.  A NOISE
// order's tick floor(mid + K (2 w1 / 2^32 - 1) + 1/2) is n - K + g + c for e = 0 and
// n - K + g + 1 for e = 1, with g = hi(2K w1) and c = [lo(2K w1) >= 2^31]; it is binned by
// (u = g + c, c) as pair 2u + c.  After the 2(2K+1) noise pairs: pair 0 marketable NOISE (buys
// go to the top tick, sells to tick 0), pair 1 MOMENTUM by coin, pair 2 marketable MOMENTUM by
// coin, pair 3 MAKER by side (section III-C's rules as in order_ctx).
template <typename Gen>
__device__ __forceinline__ void gen_rel_mid(const DevMarket &d, uint32_t s, const Gen &gen, uint32_t b0,
                                            uint32_t stride, uint32_t end, uint32_t lane, uint32_t *H)
{
    const uint32_t twoK = 2u * d.K, xb = 2u * (2u * twoK + 2u);  // first extra pair, in words
    const uint32_t tmkt = (d.flags >> CAE_PMKT_SHIFT) << CAE_PMKT_SHIFT;
    const uint32_t mom_end = d.n_noise + d.n_mom;
    for (uint32_t b = b0; b < end; b += stride) {
        const uint32_t a = b | lane;
        if (a < end) {
            uint32_t w0, w1, w2, w3;
            gen.words4_row(b, lane, w0, w1, w2, w3);
            const uint32_t side = w0 >> 31;
            const bool mkt = w3 < tmkt;
            uint32_t word;
            if (a < d.n_noise) {
                const uint64_t x = (uint64_t)twoK * w1;
                const uint32_t c = (uint32_t)x >> 31, u = (uint32_t)(x >> 32) + c;
                word = mkt ? xb + side : 2u * (2u * u + c) + side;
            } else if (a < mom_end) {
                word = xb + (mkt ? 4u : 2u) + side;
            } else {
                word = xb + 6u + ((a ^ s) & 1u);
            }
            atomicAdd(&H[word], qty1(w2, d.Q));
        }
    }
}

// Adds the mid-price bins of one step to the book at reference mid2 = 2n + e (momentum
// direction from mid2 vs mid2p) and clears them.  Lanes: 2(2K+1) noise pairs, then marketable
// NOISE buys / sells, MOMENTUM buys / sells, marketable MOMENTUM buys / sells, MAKER bids / asks.
__device__ __forceinline__ void flush_rel_mid(const DevMarket &d, uint32_t mid2, uint32_t mid2p, uint32_t *H,
                                              uint32_t *bk, uint32_t lane)
{
    const uint32_t np = 2u * (2u * d.K + 1u);  // noise pairs
    const int n = (int)(mid2 >> 1), e = (int)(mid2 & 1u), top = (int)d.L - 1, h = (int)d.h;
    const bool up = mid2 > mid2p, down = mid2 < mid2p, flat = mid2 == mid2p;
    uint2 *P = reinterpret_cast<uint2 *>(H);
    for (uint32_t j0 = 0; j0 < np + 8u; j0 += 64u) {
        const uint32_t j = j0 + lane;
        const uint32_t x = j - np;  // 0..7 for the extra lanes
        const bool noise = j < np;
        const uint2 v = P[noise ? j : np + min(x >> 1, 3u)];
        const uint32_t all = v.x + v.y;
        const uint32_t buys = up ? all : (flat ? v.x : 0u), sells = down ? all : (flat ? v.y : 0u);
        uint32_t lo = 0, hi = 0;
        int tick;
        if (noise) {
            const int u = (int)(j >> 1), c = (int)(j & 1u);
            tick = n - (int)d.K + u + (e ? 1 - c : 0);
            lo = v.x;
            hi = v.y;
        } else {
            switch (x) {
            case 0: tick = top; lo = v.x; break;            // marketable NOISE buys
            case 1: tick = 0; hi = v.y; break;              // marketable NOISE sells
            case 2: tick = n + 1 + e; lo = buys; break;     // MOMENTUM buys at round(mid + 1)
            case 3: tick = n - 1 + e; hi = sells; break;    // MOMENTUM sells at round(mid - 1)
            case 4: tick = top; lo = buys; break;           // marketable MOMENTUM buys
            case 5: tick = 0; hi = sells; break;            // marketable MOMENTUM sells
            case 6: tick = n - h + e; lo = v.x; break;      // MAKER bids at round(mid - h)
            default: tick = n + h + e; hi = v.y; break;     // MAKER asks at round(mid + h)
            }
        }
        tick = clamp_tick(tick, top);
        if (j < np + 8u && (lo | hi) != 0u)
            atomicAdd(reinterpret_cast<unsigned long long *>(bk) + tick, ((unsigned long long)hi << 32) | lo);
    }
    for (uint32_t j0 = 0; j0 < np + 4u; j0 += 64u)
        if (j0 + lane < np + 4u) P[j0 + lane] = make_uint2(0u, 0u);
}

// Best bid / best ask (kNone when a side is empty) of an LDS book, by one wave: the reference
// of the mid-price model at the start of a call (later steps take them from the clearing).
__device__ __forceinline__ void book_ends(const uint32_t *bk, uint32_t tpl, uint32_t lane, uint32_t &bb,
                                          uint32_t &ba)
{
    uint32_t hb = kNone, la = kNone;
    for (uint32_t j = 0; j < tpl; ++j) {
        const uint32_t q = lane * tpl + j;
        const uint2 v = reinterpret_cast<const uint2 *>(bk)[q];
        if (v.x != 0) hb = q;
        if (v.y != 0 && la == kNone) la = q;
    }
    const uint64_t mb = ballot(hb != kNone);
    const uint64_t ma = ballot(la != kNone);
    bb = mb ? readlane(hb, 63u - (uint32_t)__builtin_clzll(mb)) : kNone;
    ba = ma ? readlane(la, (uint32_t)__builtin_ctzll(ma)) : kNone;
}

// The reference of the step after one that left best bid bb and best ask ba and price last.
__device__ __forceinline__ uint32_t next_mid2(bool mid, uint32_t bb, uint32_t ba, uint32_t last)
{
    return (mid && bb != kNone && ba != kNone) ? bb + ba : 2u * last;
}

// One market (or an idle slot of a lock-step item) for all S steps.  MULTI: the market spans
// several waves and the workgroup barrier separates the phases (Algorithm 1's barriers).
// Lock-step markets keep their statistics in LDS scratch words 8..21 (n_trade, sum_vol,
// sum_px, sum_spread, n_spread, sum_r, sum_r2) and the clearing result of step i in words
// 4 (i & 1) .. 4 (i & 1) + 3.  A step's statistics are added during the next step's clearing by
// a wave that would otherwise wait for it, in step order.  last / prev: the prices after the
// step whose result `cob` holds.
__device__ __forceinline__ void stats_to_lds(uint32_t *scr, const uint32_t *cob, uint32_t last, uint32_t prev,
                                             const double *lnT, uint32_t lane)
{
    const uint4 r = *reinterpret_cast<const uint4 *>(cob);
    const uint32_t p = (uint32_t)__builtin_amdgcn_readfirstlane((int)r.x);
    const uint32_t v = (uint32_t)__builtin_amdgcn_readfirstlane((int)r.y);
    const uint32_t bb = (uint32_t)__builtin_amdgcn_readfirstlane((int)r.z);
    const uint32_t ba = (uint32_t)__builtin_amdgcn_readfirstlane((int)r.w);
    const double x = lnT[last] - lnT[prev];
    if (lane == 0) {
        uint64_t *a = reinterpret_cast<uint64_t *>(scr + 8);
        double *f = reinterpret_cast<double *>(scr + 18);
        if (v != 0) {
            a[0] += 1;
            a[1] += v;
            a[2] += p;
        }
        if (bb != kNone && ba != kNone) {
            a[3] += (uint64_t)(ba - bb);
            a[4] += 1;
        }
        f[0] = f[0] + x;
        f[1] = f[1] + x * x;
    }
}

template <int TPL_MAX, bool MULTI, bool FULL, bool TRACE>
__device__ __forceinline__ void run_market(const EngineArgs &args, const Item &item, uint32_t sub,
                                           uint32_t w_in, uint32_t lane, bool active,
                                           uint32_t *lds)
{
    const uint32_t wpm_mask = (1u << item.wpm_log2) - 1u;
    const uint32_t nthr = 64u << item.wpm_log2;
    const uint32_t t = (w_in << 6) | lane;
    uint32_t *bk = lds + sub * item.stride;
    uint32_t *scr = bk + item.stride - kScr;

    // statistics in LDS, added by an idle wave (lock-step markets; the widest books keep them
    // in registers, where the extra live values would spill)
    constexpr bool kLazy = MULTI && TPL_MAX <= 8;
    uint32_t m = 0;
    DevMarket d{};
    uint32_t last = 0, prev = 0, mid2 = 0, mid2p = 0;
    uint64_t steps0 = 0, n_trade = 0, sum_vol = 0, sum_px = 0, sum_spread = 0, n_spread = 0;
    double sum_r = 0.0, sum_r2 = 0.0;
    if (active) {
        m = args.order[item.first + sub];
        d = args.desc[m];
        const cae_state *st = args.state + m;
        last = st->last;
        prev = st->prev;
        steps0 = st->steps_done;
        n_trade = st->n_trade;
        sum_vol = st->sum_vol;
        sum_px = st->sum_px;
        sum_spread = st->sum_spread;
        n_spread = st->n_spread;
        sum_r = st->sum_r;
        sum_r2 = st->sum_r2;
        mid2p = st->ref2;
        if constexpr (kLazy) {
            if (t < 14u) scr[8u + t] = reinterpret_cast<const uint32_t *>(st)[4u + t];  // n_trade .. sum_r2
        }
        const uint32_t *gb = args.book + d.book_off;
        const uint32_t padded = 64u * d.tpl;
        for (uint32_t q = t; q < padded; q += nthr) {
            uint2 v = make_uint2(0u, 0u);
            if (q < d.L) {
                v.x = gb[q];
                v.y = gb[d.L + q];
            }
            reinterpret_cast<uint2 *>(bk)[q] = v;
        }
    }
    if constexpr (MULTI) __syncthreads();
    else wave_sync();
    const bool mid = FULL && (d.flags & CAE_MODEL_MASK) == CAE_MODEL_MID;
    mid2 = 2u * last;
    if (FULL && active && mid) {
        uint32_t bb, ba;
        book_ends(bk, d.tpl, lane, bb, ba);
        mid2 = next_mid2(true, bb, ba, last);
    }
    if constexpr (FULL && MULTI) __syncthreads();  // every wave has read the book before orders land

    const double *lnT = args.lnT + d.L;  // ln(L + tick)
    // The log return of step i is added at the end of step i + 1: the table load for the price
    // step i set is issued when step i + 1 starts and has long returned after its orders and
    // clearing (same values, same order of the floating-point sums).  ln_prev = ln(L + price)
    // before step i.
    double ln_prev = 0.0;
    if constexpr (!kLazy) {
        if (active) ln_prev = lnT[last];
    }
    for (uint32_t i = 0; i < args.S; ++i) {
        const uint32_t s = (uint32_t)steps0 + i;
        double ln_cur = 0.0;
        if constexpr (!kLazy) {
            if (active && i >= 1u) ln_cur = lnT[last];
        }
        if (active) gen_orders<FULL>(d, d.id, s, Refs{last, prev, mid2, mid2p}, args.k0, args.k1, t, nthr, bk);
        if constexpr (MULTI) __syncthreads();
        else wave_sync();
        ClearOut co;
        const uint32_t c = i & wpm_mask;
        if (active && w_in == c) {
            // the clearing is a chain of dependent scans and reductions that the market's other
            // waves wait for; top issue priority lets it run ahead of other markets' generation
            __builtin_amdgcn_s_setprio(3);
            co = clear_dispatch<TPL_MAX>(bk, d.tpl, lane);
            base_prio(item.boost, item.boost != 0u);
            if constexpr (MULTI) {
                if (lane == 0)
                    *reinterpret_cast<uint4 *>(scr + 4u * (i & 1u)) = make_uint4(co.p, co.v, co.bb, co.ba);
            }
        } else if (kLazy && active && i >= 1u && w_in == ((c + 1u) & wpm_mask)) {
            stats_to_lds(scr, scr + 4u * ((i - 1u) & 1u), last, prev, lnT, lane);  // the previous step's
        }
        if constexpr (MULTI) __syncthreads();
        else wave_sync();
        if (active) {
            if constexpr (MULTI) {
                const uint4 r = *reinterpret_cast<const uint4 *>(scr + 4u * (i & 1u));
                co.p = (uint32_t)__builtin_amdgcn_readfirstlane((int)r.x);
                co.v = (uint32_t)__builtin_amdgcn_readfirstlane((int)r.y);
                co.bb = (uint32_t)__builtin_amdgcn_readfirstlane((int)r.z);
                co.ba = (uint32_t)__builtin_amdgcn_readfirstlane((int)r.w);
            }
            prev = last;
            if (co.v != 0) last = co.p;
            if constexpr (!kLazy) {
                if (co.v != 0) {
                    n_trade += 1;
                    sum_vol += co.v;
                    sum_px += co.p;
                }
                if (co.bb != kNone && co.ba != kNone) {
                    sum_spread += (uint64_t)(co.ba - co.bb);
                    n_spread += 1;
                }
                if (i >= 1u) {  // the previous step's return
                    const double r = ln_cur - ln_prev;
                    sum_r = sum_r + r;
                    sum_r2 = sum_r2 + r * r;
                    ln_prev = ln_cur;
                }
            }
            mid2p = mid2;
            mid2 = next_mid2(mid, co.bb, co.ba, last);
            if constexpr (TRACE) {
                if (t == 0) trace_step(args, m, i, last, co.v);
            }
        }
    }
    if constexpr (!kLazy) {
        if (active && args.S >= 1u) {  // the last step's log return
            const double r = lnT[last] - ln_prev;
            sum_r = sum_r + r;
            sum_r2 = sum_r2 + r * r;
        }
    }
    if constexpr (kLazy) {
        // the last step's statistics; then wave 0 holds the totals of every step
        if (active && w_in == 0u && args.S >= 1u) {
            stats_to_lds(scr, scr + 4u * ((args.S - 1u) & 1u), last, prev, lnT, lane);
            wave_sync();
            const uint64_t *a = reinterpret_cast<const uint64_t *>(scr + 8);
            const double *f = reinterpret_cast<const double *>(scr + 18);
            n_trade = a[0];
            sum_vol = a[1];
            sum_px = a[2];
            sum_spread = a[3];
            n_spread = a[4];
            sum_r = f[0];
            sum_r2 = f[1];
        }
    }
    if (active) {
        uint32_t *gb = args.book + d.book_off;
        for (uint32_t q = t; q < d.L; q += nthr) {
            const uint2 v = reinterpret_cast<const uint2 *>(bk)[q];
            gb[q] = v.x;
            gb[d.L + q] = v.y;
        }
        if (t == 0) {
            cae_state *st = args.state + m;
            st->last = last;
            st->prev = prev;
            st->steps_done = steps0 + args.S;
            st->n_trade = n_trade;
            st->sum_vol = sum_vol;
            st->sum_px = sum_px;
            st->sum_spread = sum_spread;
            st->n_spread = n_spread;
            st->sum_r = sum_r;
            st->sum_r2 = sum_r2;
            st->ref2 = mid2p;
        }
    }
}

// Lock-step market of the last-tick model with the next step's orders generated while the
// current step clears.  One wave at a time owns the clearing for a block of kOvlBlock steps (the
// role rotates over the market's waves block by block, which spreads the clearing over the
// SIMDs): in step i the owner adds the bins of step i to the book around the price after step
// i - 1 (the reference of step i), clears it, keeps the step's price and statistics in its
// registers and then
// generates `share` rows of 64 agents of step i + 1; the other waves generate the rest of step
// i + 1 into the other bin buffer.  No other wave needs the price: one barrier per step, no LDS
// round trip for the result, and no wave waits for a clearing.  At the end of its block the
// owner hands the price and the floating-point sums (kept in step order) to the next owner
// through LDS.  Step 0 of the call is generated into the book directly.  Same books, prices
// and statistics as run_market.
//
// Scratch words: 0 last, 1 prev, 2 ref2 (hand-over), 4-5 sum_r, 6-7 sum_r2 (hand-over), 8-17
// n_trade, sum_vol, sum_px, sum_spread, n_spread (each wave's totals added at the end).
constexpr uint32_t kOvlBlockLog2 = 4;
constexpr uint32_t kOvlBlock = 1u << kOvlBlockLog2;

template <int TPL_MAX, bool TRACE>
__device__ __forceinline__ void run_market_ovl(const EngineArgs &args, const Item &item, uint32_t sub,
                                               uint32_t w_in, uint32_t lane, bool active, uint32_t *lds)
{
    const uint32_t wpm_mask = (1u << item.wpm_log2) - 1u;
    const uint32_t nthr = 64u << item.wpm_log2;
    const uint32_t t = (w_in << 6) | lane;
    uint32_t *bk = lds + sub * item.stride;
    uint32_t *scr = bk + item.stride - kScr;
    uint32_t *H0 = bk + item.hoff;
    uint32_t *H1 = H0 + item.hwords;
    double *fs = reinterpret_cast<double *>(scr + 4);

    uint32_t m = 0;
    DevMarket d{};
    uint32_t last = 0, prev = 0, ref2 = 0;
    uint64_t steps0 = 0;
    double sum_r = 0.0, sum_r2 = 0.0;
    if (active) {
        m = args.order[item.first + sub];
        d = args.desc[m];
        const cae_state *st = args.state + m;
        last = st->last;
        prev = st->prev;
        steps0 = st->steps_done;
        ref2 = st->ref2;
        sum_r = st->sum_r;
        sum_r2 = st->sum_r2;
        if (t < 10u) scr[8u + t] = reinterpret_cast<const uint32_t *>(st)[4u + t];  // n_trade .. n_spread
        const uint32_t *gb = args.book + d.book_off;
        const uint32_t padded = 64u * d.tpl;
        for (uint32_t q = t; q < padded; q += nthr) {
            uint2 v = make_uint2(0u, 0u);
            if (q < d.L) {
                v.x = gb[q];
                v.y = gb[d.L + q];
            }
            reinterpret_cast<uint2 *>(bk)[q] = v;
        }
        for (uint32_t q = t; q < 2u * item.hwords; q += nthr) H0[q] = 0u;
    }
    __syncthreads();
    if (active) gen_orders<false>(d, d.id, (uint32_t)steps0, Refs{last, prev, 2u * last, 0u}, args.k0, args.k1, t,
                                  nthr, bk);
    __syncthreads();

    const double *lnT = args.lnT + d.L;
    uint64_t n_trade = 0, sum_vol = 0, sum_px = 0, sum_spread = 0, n_spread = 0;  // this wave's steps
    // the statistics of the steps of the current block, in 32 bits: its volumes sum to at most
    // the shares ever added to the book (below 2^32 by the host guard), its ticks and spreads to
    // at most kOvlBlock (L - 1)
    uint32_t b_trade = 0, b_vol = 0, b_px = 0, b_spread = 0, b_nspread = 0;
    double ln_cur = 0.0;  // ln(L + last) on the clearing wave
    const uint32_t own = min(d.A, item.share * 64u);        // agents of the clearing wave
    const uint32_t ostride = nthr - 64u;                   // the other waves' stride
    const uint32_t span = 2u * d.K + 1u;
    const int top = (int)d.L - 1;
    const bool one_pass = span + 4u <= 64u;
    const FlushLanes fl = flush_lanes(d, lane);
    for (uint32_t i = 0; i < args.S; ++i) {
        const uint32_t s = (uint32_t)steps0 + i;
        const uint32_t c = (i >> kOvlBlockLog2) & wpm_mask;
        uint32_t *Hn = (i & 1u) ? H0 : H1;  // bins of step i + 1
        const bool more = i + 1u < args.S;
        if (active && w_in == c) {
            // top issue priority for the whole block (the wave waits at the barrier between its
            // steps, and the next block's base_prio lowers it again)
            if ((i & (kOvlBlock - 1u)) == 0u) __builtin_amdgcn_s_setprio(3);
            if (i != 0u && (i & (kOvlBlock - 1u)) == 0u) {  // first step of this wave's block
                const uint4 h = *reinterpret_cast<const uint4 *>(scr);
                last = (uint32_t)__builtin_amdgcn_readfirstlane((int)h.x);
                prev = (uint32_t)__builtin_amdgcn_readfirstlane((int)h.y);
                ref2 = (uint32_t)__builtin_amdgcn_readfirstlane((int)h.z);
                sum_r = fs[0];
                sum_r2 = fs[1];
            }
            if ((i & (kOvlBlock - 1u)) == 0u) ln_cur = lnT[last];  // used after this step's rows
            if (i >= 1u) {
                if (one_pass) flush_rel_lanes(fl, span, top, last, prev, (i & 1u) ? H1 : H0, bk, lane);
                else flush_rel(d, last, prev, (i & 1u) ? H1 : H0, bk, lane);
            }
            wave_sync();
            const ClearOut co = clear_dispatch<TPL_MAX>(bk, d.tpl, lane);
            const bool traded = co.v != 0;
            const bool quoted = co.bb != kNone && co.ba != kNone;
            b_trade += traded ? 1u : 0u;
            b_vol += co.v;
            b_px += traded ? co.p : 0u;
            b_spread += quoted ? co.ba - co.bb : 0u;
            b_nspread += quoted ? 1u : 0u;
            ref2 = 2u * last;
            prev = last;
            if (traded) last = co.p;
            if constexpr (TRACE) {
                if (lane == 0) trace_step(args, m, i, last, co.v);
            }
            // the log-table load is issued here and consumed after the wave's rows
            const double ln_new = lnT[last];
            if (more) gen_rel(d, s + 1u, PhiloxStep(s + 1u, d.id, args.k0, args.k1), 0u, 64u, own, lane, Hn);
            const double x = ln_new - ln_cur;
            sum_r = sum_r + x;
            sum_r2 = sum_r2 + x * x;
            ln_cur = ln_new;
            if (((i + 1u) & (kOvlBlock - 1u)) == 0u || !more) {  // hand over (or finish)
                if (lane == 0) {
                    *reinterpret_cast<uint4 *>(scr) = make_uint4(last, prev, ref2, 0u);
                    fs[0] = sum_r;
                    fs[1] = sum_r2;
                }
                n_trade += b_trade;
                sum_vol += b_vol;
                sum_px += b_px;
                sum_spread += b_spread;
                n_spread += b_nspread;
                b_trade = b_vol = b_px = b_spread = b_nspread = 0u;
            }
        } else if (active && more) {
            // Generating waves alternate between issue priorities 0 and 1 every block of steps,
            // out of step between workgroups of even and odd index: the SIMD arbiter otherwise
            // favours the oldest waves for the whole persistent launch, and the markets of the
            // youngest workgroups on a CU set the launch's length.  Set once per block.
            if ((i & (kOvlBlock - 1u)) == 0u)
                base_prio(item.boost, (((i >> kOvlBlockLog2) + blockIdx.x) & 1u) != 0u);
            const uint32_t r = (w_in - c - 1u) & wpm_mask;  // 0 .. wpm - 2
            gen_rel(d, s + 1u, PhiloxStep(s + 1u, d.id, args.k0, args.k1), own + (r << 6), ostride, d.A, lane,
                    Hn);
        }
        __syncthreads();
    }
    // every wave adds the integer totals of the steps it cleared
    if (active && lane == 0) {
        unsigned long long *a = reinterpret_cast<unsigned long long *>(scr + 8);
        atomicAdd(a + 0, (unsigned long long)n_trade);
        atomicAdd(a + 1, (unsigned long long)sum_vol);
        atomicAdd(a + 2, (unsigned long long)sum_px);
        atomicAdd(a + 3, (unsigned long long)sum_spread);
        atomicAdd(a + 4, (unsigned long long)n_spread);
    }
    __syncthreads();
    if (active) {
        uint32_t *gb = args.book + d.book_off;
        for (uint32_t q = t; q < d.L; q += nthr) {
            const uint2 v = reinterpret_cast<const uint2 *>(bk)[q];
            gb[q] = v.x;
            gb[d.L + q] = v.y;
        }
        if (t == 0) {
            const uint64_t *a = reinterpret_cast<const uint64_t *>(scr + 8);
            cae_state *st = args.state + m;
            st->last = scr[0];
            st->prev = scr[1];
            st->steps_done = steps0 + args.S;
            st->n_trade = a[0];
            st->sum_vol = a[1];
            st->sum_px = a[2];
            st->sum_spread = a[3];
            st->n_spread = a[4];
            st->sum_r = fs[0];
            st->sum_r2 = fs[1];
            st->ref2 = scr[2];
        }
    }
}

// The same schedule for ensembles that may hold mid-price or SplitMix64 markets (the FULL
// instantiation): the reference is 2 x mid, tracked as in run_market, and the bins are the
// model's (gen_rel / gen_rel_mid).  Scratch words 2 and 3 hand over mid2 and mid2p.
template <int TPL_MAX, bool FULL, bool TRACE>
__device__ __forceinline__ void run_market_ovl_any(const EngineArgs &args, const Item &item, uint32_t sub,
                                               uint32_t w_in, uint32_t lane, bool active, uint32_t *lds)
{
    const uint32_t wpm_mask = (1u << item.wpm_log2) - 1u;
    const uint32_t nthr = 64u << item.wpm_log2;
    const uint32_t t = (w_in << 6) | lane;
    uint32_t *bk = lds + sub * item.stride;
    uint32_t *scr = bk + item.stride - kScr;
    uint32_t *H0 = bk + item.hoff;
    uint32_t *H1 = H0 + item.hwords;
    double *fs = reinterpret_cast<double *>(scr + 4);

    uint32_t m = 0;
    DevMarket d{};
    uint32_t last = 0, prev = 0, mid2 = 0, mid2p = 0;
    uint64_t steps0 = 0;
    double sum_r = 0.0, sum_r2 = 0.0;
    if (active) {
        m = args.order[item.first + sub];
        d = args.desc[m];
        const cae_state *st = args.state + m;
        last = st->last;
        prev = st->prev;
        steps0 = st->steps_done;
        mid2p = st->ref2;
        sum_r = st->sum_r;
        sum_r2 = st->sum_r2;
        if (t < 10u) scr[8u + t] = reinterpret_cast<const uint32_t *>(st)[4u + t];  // n_trade .. n_spread
        const uint32_t *gb = args.book + d.book_off;
        const uint32_t padded = 64u * d.tpl;
        for (uint32_t q = t; q < padded; q += nthr) {
            uint2 v = make_uint2(0u, 0u);
            if (q < d.L) {
                v.x = gb[q];
                v.y = gb[d.L + q];
            }
            reinterpret_cast<uint2 *>(bk)[q] = v;
        }
        for (uint32_t q = t; q < 2u * item.hwords; q += nthr) H0[q] = 0u;
    }
    __syncthreads();
    const bool mid = FULL && (d.flags & CAE_MODEL_MASK) == CAE_MODEL_MID;
    const bool smx = FULL && uses_splitmix(d);
    mid2 = 2u * last;
    if (FULL && active && mid) {
        uint32_t bb, ba;
        book_ends(bk, d.tpl, lane, bb, ba);
        mid2 = next_mid2(true, bb, ba, last);
    }
    if constexpr (FULL) __syncthreads();  // every wave has read the book before orders land
    if (active) gen_orders<FULL>(d, d.id, (uint32_t)steps0, Refs{last, prev, mid2, mid2p}, args.k0, args.k1, t,
                                 nthr, bk);
    __syncthreads();

    const double *lnT = args.lnT + d.L;
    const uint64_t seed64 = ((uint64_t)args.k1 << 32) | args.k0;
    // the next step's orders into bin buffer Hn, agents b | lane for b = b0, b0 + stride, ...
    const auto gen_bins = [&](uint32_t sn, uint32_t b0, uint32_t stride, uint32_t end, uint32_t *Hn) {
        if constexpr (FULL) {
            if (smx) {
                const SplitMixStep g(sn, d.id, d.A, seed64);
                if (mid) gen_rel_mid(d, sn, g, b0, stride, end, lane, Hn);
                else gen_rel(d, sn, g, b0, stride, end, lane, Hn);
                return;
            }
            if (mid) {
                gen_rel_mid(d, sn, PhiloxStep(sn, d.id, args.k0, args.k1), b0, stride, end, lane, Hn);
                return;
            }
        }
        gen_rel(d, sn, PhiloxStep(sn, d.id, args.k0, args.k1), b0, stride, end, lane, Hn);
    };
    uint64_t n_trade = 0, sum_vol = 0, sum_px = 0, sum_spread = 0, n_spread = 0;  // this wave's steps
    const uint32_t own = min(d.A, item.share * 64u);        // agents of the clearing wave
    const uint32_t ostride = nthr - 64u;                   // the other waves' stride
    for (uint32_t i = 0; i < args.S; ++i) {
        const uint32_t s = (uint32_t)steps0 + i;
        const uint32_t c = (i >> kOvlBlockLog2) & wpm_mask;
        uint32_t *Hn = (i & 1u) ? H0 : H1;  // bins of step i + 1
        const bool more = i + 1u < args.S;
        if (active && w_in == c) {
            __builtin_amdgcn_s_setprio(3);
            if (i != 0u && (i & (kOvlBlock - 1u)) == 0u) {  // first step of this wave's block
                const uint4 h = *reinterpret_cast<const uint4 *>(scr);
                last = (uint32_t)__builtin_amdgcn_readfirstlane((int)h.x);
                prev = (uint32_t)__builtin_amdgcn_readfirstlane((int)h.y);
                mid2 = (uint32_t)__builtin_amdgcn_readfirstlane((int)h.z);
                mid2p = (uint32_t)__builtin_amdgcn_readfirstlane((int)h.w);
                sum_r = fs[0];
                sum_r2 = fs[1];
            }
            if (i >= 1u) {
                if (FULL && mid) flush_rel_mid(d, mid2, mid2p, (i & 1u) ? H1 : H0, bk, lane);
                else flush_rel(d, last, prev, (i & 1u) ? H1 : H0, bk, lane);
            }
            wave_sync();
            const ClearOut co = clear_dispatch<TPL_MAX>(bk, d.tpl, lane);
            if (co.v != 0) {
                n_trade += 1;
                sum_vol += co.v;
                sum_px += co.p;
            }
            if (co.bb != kNone && co.ba != kNone) {
                sum_spread += (uint64_t)(co.ba - co.bb);
                n_spread += 1;
            }
            prev = last;
            if (co.v != 0) last = co.p;
            mid2p = mid2;
            mid2 = next_mid2(mid, co.bb, co.ba, last);
            if constexpr (TRACE) {
                if (lane == 0) trace_step(args, m, i, last, co.v);
            }
            // the log-table loads are issued here and consumed after the wave's rows
            const double x = lnT[last] - lnT[prev];
            if (more) gen_bins(s + 1u, 0u, 64u, own, Hn);
            sum_r = sum_r + x;
            sum_r2 = sum_r2 + x * x;
            if (((i + 1u) & (kOvlBlock - 1u)) == 0u || !more) {  // hand over (or finish)
                if (lane == 0) {
                    *reinterpret_cast<uint4 *>(scr) = make_uint4(last, prev, mid2, mid2p);
                    fs[0] = sum_r;
                    fs[1] = sum_r2;
                }
            }
            __builtin_amdgcn_s_setprio(0);
        } else if (active && more) {
            // issue priority alternating by block and workgroup parity, as in run_market_ovl
            base_prio(item.boost, (((i >> kOvlBlockLog2) + blockIdx.x) & 1u) != 0u);
            const uint32_t r = (w_in - c - 1u) & wpm_mask;  // 0 .. wpm - 2
            gen_bins(s + 1u, own + (r << 6), ostride, d.A, Hn);
        }
        __syncthreads();
    }
    // every wave adds the integer totals of the steps it cleared
    if (active && lane == 0) {
        unsigned long long *a = reinterpret_cast<unsigned long long *>(scr + 8);
        atomicAdd(a + 0, (unsigned long long)n_trade);
        atomicAdd(a + 1, (unsigned long long)sum_vol);
        atomicAdd(a + 2, (unsigned long long)sum_px);
        atomicAdd(a + 3, (unsigned long long)sum_spread);
        atomicAdd(a + 4, (unsigned long long)n_spread);
    }
    __syncthreads();
    if (active) {
        uint32_t *gb = args.book + d.book_off;
        for (uint32_t q = t; q < d.L; q += nthr) {
            const uint2 v = reinterpret_cast<const uint2 *>(bk)[q];
            gb[q] = v.x;
            gb[d.L + q] = v.y;
        }
        if (t == 0) {
            const uint64_t *a = reinterpret_cast<const uint64_t *>(scr + 8);
            cae_state *st = args.state + m;
            st->last = scr[0];
            st->prev = scr[1];
            st->steps_done = steps0 + args.S;
            st->n_trade = a[0];
            st->sum_vol = a[1];
            st->sum_px = a[2];
            st->sum_spread = a[3];
            st->n_spread = a[4];
            st->sum_r = fs[0];
            st->sum_r2 = fs[1];
            st->ref2 = scr[3];
        }
    }
}

// Scratch layout of a pipelined market (32-bit words): 0 last, 1 prev, 2-3 steps at item start,
// 4-5 n_trade, 6-7 sum_vol, 8-9 sum_px, 10-11 sum_spread, 12-13 n_spread, 14-15 sum_r,
// 16-17 sum_r2, 18 ref2 (2 x the previous step's reference), 19 reserved (words 0-19 are the
// cae_state record), 20 mid2 (2 x the next step's reference).
constexpr uint32_t kStateWords = sizeof(cae_state) / 4u;
static_assert(kStateWords == 20 && kStateWords + 1u <= kScr, "pipelined scratch layout");
__device__ __forceinline__ uint64_t lds_u64(const uint32_t *p)
{
    const uint2 v = *reinterpret_cast<const uint2 *>(p);
    return ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)v.y) << 32) |
           (uint32_t)__builtin_amdgcn_readfirstlane((int)v.x);
}

__device__ __forceinline__ void st_u64(uint32_t *p, uint64_t v)
{
    *reinterpret_cast<uint2 *>(p) = make_uint2((uint32_t)v, (uint32_t)(v >> 32));
}

// Two markets (A, B) share all G waves of the workgroup in alternating phases: in phase p one
// wave (rotating) clears the market whose orders were aggregated in phase p-1 while the other
// G-1 waves generate and aggregate the other market's orders.  One barrier per phase; no wave
// waits for a clearing.  With one market the phases alternate between its orders and its
// clearing.  Phase count: 2S (+1 to clear B's last step).
template <int TPL_MAX, bool FULL, bool TRACE>
__device__ __forceinline__ void run_pair(const EngineArgs &args, const Item &item, uint32_t wave, uint32_t lane,
                                         uint32_t G, uint32_t *lds)
{
    const uint32_t npair = item.count;
    const uint32_t tid = (wave << 6) | lane;
    const uint32_t nthr = G << 6;
    DevMarket dA{}, dB{};  // two named descriptors: a runtime index into an array would spill
    uint32_t mA = 0, mB = 0;
#pragma unroll
    for (uint32_t x = 0; x < 2; ++x) {
        if (x < npair) {
            const uint32_t m = args.order[item.first + x];
            const DevMarket dm = args.desc[m];
            if (x == 0) {
                dA = dm;
                mA = m;
            } else {
                dB = dm;
                mB = m;
            }
            uint32_t *bk = lds + x * item.stride;
            uint32_t *scr = bk + item.stride - kScr;
            const uint32_t *gb = args.book + dm.book_off;
            const uint32_t padded = 64u * dm.tpl;
            for (uint32_t q = tid; q < padded; q += nthr) {
                uint2 v = make_uint2(0u, 0u);
                if (q < dm.L) {
                    v.x = gb[q];
                    v.y = gb[dm.L + q];
                }
                reinterpret_cast<uint2 *>(bk)[q] = v;
            }
            if (tid < kStateWords) scr[tid] = reinterpret_cast<const uint32_t *>(args.state + m)[tid];
        }
    }
    __syncthreads();
    // reference of each market's first step (wave x of the workgroup reads market x's book)
#pragma unroll
    for (uint32_t x = 0; x < 2; ++x) {
        if (x < npair && wave == x % G) {
            const DevMarket &dm = x ? dB : dA;
            uint32_t *bk = lds + x * item.stride;
            uint32_t *scr = bk + item.stride - kScr;
            const uint32_t last = (uint32_t)__builtin_amdgcn_readfirstlane((int)scr[0]);
            uint32_t mid2 = 2u * last;
            if (FULL && (dm.flags & CAE_MODEL_MASK) == CAE_MODEL_MID) {
                uint32_t bb, ba;
                book_ends(bk, dm.tpl, lane, bb, ba);
                mid2 = next_mid2(true, bb, ba, last);
            }
            if (lane == 0) scr[20] = mid2;
        }
    }
    __syncthreads();
    const uint32_t S = args.S;
    const uint32_t nph = 2u * S + (npair == 2u ? 1u : 0u);
    // generator index of this wave, (wave - c - 1) mod G for clearing wave c = p mod G; it steps
    // down by one per phase, and the clearing wave is the one at G - 1
    uint32_t gidx = (wave + G - 1u) % G;
    for (uint32_t p = 0; p < nph; ++p) {
        const uint32_t X = p & 1u, Y = X ^ 1u;
        if (gidx == G - 1u) {
            if (p >= 1u && Y < npair) {
                uint32_t *bk = lds + Y * item.stride;
                uint32_t *scr = bk + item.stride - kScr;
                const DevMarket &dy = Y ? dB : dA;
                __builtin_amdgcn_s_setprio(3);
                const ClearOut co = clear_dispatch<TPL_MAX>(bk, dy.tpl, lane);
                __builtin_amdgcn_s_setprio(0);
                const uint4 s0 = *reinterpret_cast<const uint4 *>(scr);       // last, prev, steps
                const uint4 s1 = *reinterpret_cast<const uint4 *>(scr + 4);   // n_trade, sum_vol
                const uint4 s2 = *reinterpret_cast<const uint4 *>(scr + 8);   // sum_px, sum_spread
                const uint4 s3 = *reinterpret_cast<const uint4 *>(scr + 12);  // n_spread, sum_r
                const uint2 s4 = *reinterpret_cast<const uint2 *>(scr + 16);  // sum_r2
                auto u = [](uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); };
                auto u64 = [&](uint32_t lo, uint32_t hi) { return ((uint64_t)u(hi) << 32) | u(lo); };
                const uint32_t last0 = u(s0.x);
                uint64_t n_trade = u64(s1.x, s1.y), sum_vol = u64(s1.z, s1.w);
                uint64_t sum_px = u64(s2.x, s2.y), sum_spread = u64(s2.z, s2.w);
                uint64_t n_spread = u64(s3.x, s3.y);
                const double sum_r = __longlong_as_double((long long)u64(s3.z, s3.w));
                const double sum_r2 = __longlong_as_double((long long)u64(s4.x, s4.y));
                uint32_t last = last0;
                if (co.v != 0) {
                    last = co.p;
                    n_trade += 1;
                    sum_vol += co.v;
                    sum_px += co.p;
                }
                if (co.bb != kNone && co.ba != kNone) {
                    sum_spread += (uint64_t)(co.ba - co.bb);
                    n_spread += 1;
                }
                const double *lnT = args.lnT + dy.L;
                const double r = lnT[last] - lnT[last0];
                if constexpr (TRACE) {
                    if (lane == 0) trace_step(args, Y ? mB : mA, (p - 1u) >> 1, last, co.v);
                }
                const uint32_t mid2_used = (uint32_t)__builtin_amdgcn_readfirstlane((int)scr[20]);
                const uint32_t mid2_next =
                    next_mid2(FULL && (dy.flags & CAE_MODEL_MASK) == CAE_MODEL_MID, co.bb, co.ba, last);
                if (lane == 0) {
                    scr[18] = mid2_used;
                    scr[20] = mid2_next;
                    scr[0] = last;
                    scr[1] = last0;
                    st_u64(scr + 4, n_trade);
                    st_u64(scr + 6, sum_vol);
                    st_u64(scr + 8, sum_px);
                    st_u64(scr + 10, sum_spread);
                    st_u64(scr + 12, n_spread);
                    st_u64(scr + 14, (uint64_t)__double_as_longlong(sum_r + r));
                    st_u64(scr + 16, (uint64_t)__double_as_longlong(sum_r2 + r * r));
                }
            }
        } else if (p < 2u * S && X < npair) {
            uint32_t *bk = lds + X * item.stride;
            const uint4 s0 = *reinterpret_cast<const uint4 *>(bk + item.stride - kScr);
            const uint32_t last = (uint32_t)__builtin_amdgcn_readfirstlane((int)s0.x);
            const uint32_t prev = (uint32_t)__builtin_amdgcn_readfirstlane((int)s0.y);
            const uint32_t s = (uint32_t)__builtin_amdgcn_readfirstlane((int)s0.z) + (p >> 1);
            const DevMarket &dx = X ? dB : dA;
            Refs r{last, prev, 0u, 0u};
            if (FULL && (dx.flags & CAE_MODEL_MASK) == CAE_MODEL_MID) {
                const uint32_t *scr = bk + item.stride - kScr;
                r.mid2p = (uint32_t)__builtin_amdgcn_readfirstlane((int)scr[18]);
                r.mid2 = (uint32_t)__builtin_amdgcn_readfirstlane((int)scr[20]);
            }
            gen_orders<FULL, false>(dx, dx.id, s, r, args.k0, args.k1, (gidx << 6) | lane, (G - 1u) << 6, bk);
        }
        __syncthreads();
        gidx = gidx == 0u ? G - 1u : gidx - 1u;
    }
#pragma unroll
    for (uint32_t x = 0; x < 2; ++x) {
        if (x < npair) {
            const DevMarket &dm = x ? dB : dA;
            const uint32_t m = x ? mB : mA;
            const uint32_t *bk = lds + x * item.stride;
            uint32_t *scr = lds + x * item.stride + item.stride - kScr;
            uint32_t *gb = args.book + dm.book_off;
            for (uint32_t q = tid; q < dm.L; q += nthr) {
                const uint2 v = reinterpret_cast<const uint2 *>(bk)[q];
                gb[q] = v.x;
                gb[dm.L + q] = v.y;
            }
            if (tid == 0) st_u64(scr + 2, lds_u64(scr + 2) + S);
            __syncthreads();
            if (tid < kStateWords) reinterpret_cast<uint32_t *>(args.state + m)[tid] = scr[tid];
        }
    }
}

// ------------------------------------------------------------------------------------------
// Packed small markets: P = 64 / SEG markets share one wave, market k of the wave owning the
// lane segment [k SEG, k SEG + SEG).  A segment generates its market's orders in rows of SEG
// agents and clears its book with SEG lanes of TPL ticks each, so a market of 16 agents no longer
// leaves 48 lanes of its wave idle in every step, and P books clear in one pass.  The clearing is
// clear_small's on a lane segment: the scan stops at the segment's edge, and each lane reads its
// own segment's crossing lane, totals and best quotes by a lane permute instead of a readlane.
// Last-tick model with the Philox generator (the host packs no other market); every value that
// is wave-uniform elsewhere (the market, its descriptor, state and step counter, the generator's
// per-step rounds) is per lane here, so the whole Philox evaluation runs per agent.
// ------------------------------------------------------------------------------------------

// Inclusive scans of x and y within lane segments of 2^SEGLOG lanes (SEGLOG 4 or 5).
template <int SEGLOG>
__device__ __forceinline__ void seg_scan_add2(uint32_t &x, uint32_t &y)
{
    x += dpp<0x111, 0xf>(x);
    y += dpp<0x111, 0xf>(y);
    x += dpp<0x112, 0xf>(x);
    y += dpp<0x112, 0xf>(y);
    x += dpp<0x114, 0xf>(x);
    y += dpp<0x114, 0xf>(y);
    x += dpp<0x118, 0xf>(x);
    y += dpp<0x118, 0xf>(y);
    if constexpr (SEGLOG >= 5) {
        x += dpp<0x142, 0xa>(x);
        y += dpp<0x142, 0xa>(y);
    }
}

// x of lane l (any lane of the wave; l may differ between lanes)
__device__ __forceinline__ uint32_t lane_value(uint32_t x, uint32_t l)
{
    return (uint32_t)__builtin_amdgcn_ds_bpermute((int)(l << 2), (int)x);
}

// The bits of a wave-wide mask that belong to this lane's segment (segment base `base`).
template <int SEGLOG>
__device__ __forceinline__ uint32_t seg_bits(uint64_t mask, uint32_t base)
{
    constexpr uint32_t kSeg = 1u << SEGLOG;
    return (uint32_t)(mask >> base) & (uint32_t)((1ull << kSeg) - 1ull);
}

// First lane of this lane's segment where a predicate that holds on a suffix of the segment is
// true, or the segment's last lane when it holds nowhere (as crossing_lane, per segment).
template <int SEGLOG>
__device__ __forceinline__ uint32_t seg_crossing_lane(bool pred, uint32_t base)
{
    constexpr uint32_t kSeg = 1u << SEGLOG;
    return base + (uint32_t)__builtin_ctz(seg_bits<SEGLOG>(ballot(pred), base) | (1u << (kSeg - 1u)));
}

// Packed books hold two (bid, ask) pairs of padding after every 32 ticks: a segment's lanes read
// their ticks as runs of TPL pairs, and without the padding the lanes of one 16-lane LDS pass
// whose runs start 256 bytes apart would share banks.  Pair index of tick q, and the LDS word of
// book word w = 2 q + side.
__device__ __forceinline__ uint32_t pad_pair(uint32_t q) { return q + 2u * (q >> 5); }
__device__ __forceinline__ uint32_t pad_word(uint32_t w) { return w + ((w >> 6) << 2); }

// One clearing pass over the book of each lane segment (bk: this lane's book, pairs for ticks
// [0, SEG TPL), zero beyond L, its residual written back; ll: the lane's index in its segment;
// mid: independent work issued after the book loads, which the pass's own dependency chain leaves
// room for).  Segment-uniform result.
template <int TPL, int SEGLOG, class F>
__device__ __forceinline__ ClearOut clear_seg(uint32_t *__restrict__ bk, uint32_t ll, uint32_t base, F &&mid)
{
    const uint32_t q0 = ll * TPL;
    uint32_t b[TPL], k[TPL];
    load_pairs<TPL>(bk, pad_pair(q0), b, k);
    mid();
    uint32_t sb = 0, sa = 0;
#pragma unroll
    for (int j = 0; j < TPL; ++j) {
        sb += b[j];
        sa += k[j];
    }
    uint32_t ib = sb, ia = sa;
    seg_scan_add2<SEGLOG>(ib, ia);
    constexpr uint32_t kSeg = 1u << SEGLOG;
    const uint32_t Tb = lane_value(ib, base + kSeg - 1u);
    uint32_t D[TPL + 1], Sq[TPL];
    D[0] = Tb - (ib - sb);
    const uint32_t Sb = ia - sa;
#pragma unroll
    for (int j = 0; j < TPL; ++j) {
        D[j + 1] = D[j] - b[j];
        Sq[j] = (j ? Sq[j - 1] : Sb) + k[j];
    }
    uint32_t vc = Sb;
#pragma unroll
    for (int j = 0; j < TPL; ++j) vc = max(vc, min(D[j], Sq[j]));
    ClearOut out;
    out.v = lane_value(vc, seg_crossing_lane<SEGLOG>(Sq[TPL - 1] >= D[TPL - 1], base));
    const uint32_t vs = out.v;
    {
        uint32_t pj = q0;
#pragma unroll
        for (int j = 0; j < TPL; ++j) pj += Sq[j] < vs ? 1u : 0u;
        out.p = lane_value(pj, seg_crossing_lane<SEGLOG>(Sq[TPL - 1] >= vs, base));
    }
    uint32_t ud = unmatched(D[0], vs), us = unmatched(Sb, vs);
#pragma unroll
    for (int j = 0; j < TPL; ++j) {
        const uint32_t ud1 = unmatched(D[j + 1], vs), us1 = unmatched(Sq[j], vs);
        b[j] = ud - ud1;
        k[j] = us1 - us;
        ud = ud1;
        us = us1;
    }
    store_pairs<TPL>(bk, pad_pair(q0), b, k);
    uint32_t hb = kNone, la = kNone;
#pragma unroll
    for (int j = 0; j < TPL; ++j)
        if (b[j] != 0) hb = q0 + j;
#pragma unroll
    for (int j = TPL - 1; j >= 0; --j)
        if (k[j] != 0) la = q0 + j;
    const uint32_t mb = seg_bits<SEGLOG>(ballot(hb != kNone), base);
    const uint32_t ma = seg_bits<SEGLOG>(ballot(la != kNone), base);
    const uint32_t bbv = lane_value(hb, base + (mb ? 31u - (uint32_t)__builtin_clz(mb) : 0u));
    const uint32_t bav = lane_value(la, base + (ma ? (uint32_t)__builtin_ctz(ma) : 0u));
    out.bb = mb ? bbv : kNone;
    out.ba = ma ? bav : kNone;
    return out;
}

// Segments of 16 lanes are DPP rows, so every per-segment value comes from row operations in
// registers (no lane permute through the LDS): a row reduction (row_shr by 1, 2, 4, 8, with the
// reduction's identity for lanes shifted in from outside the row) leaves the row's result in its
// last lane, and row_newbcast:15 hands that lane's value to the whole row.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_or(uint32_t identity, uint32_t x)
{
    return (uint32_t)__builtin_amdgcn_update_dpp((int)identity, (int)x, CTRL, 0xf, 0xf, false);
}

__device__ __forceinline__ uint32_t row_last(uint32_t x) { return dpp_or<0x15F>(0u, x); }

__device__ __forceinline__ uint32_t row_sum(uint32_t x)
{
    x += dpp_or<0x111>(0u, x);
    x += dpp_or<0x112>(0u, x);
    x += dpp_or<0x114>(0u, x);
    x += dpp_or<0x118>(0u, x);
    return row_last(x);
}

__device__ __forceinline__ uint32_t row_max(uint32_t x)
{
    x = max(x, dpp_or<0x111>(0u, x));
    x = max(x, dpp_or<0x112>(0u, x));
    x = max(x, dpp_or<0x114>(0u, x));
    x = max(x, dpp_or<0x118>(0u, x));
    return row_last(x);
}

// One clearing pass over the book of each 16-lane segment (four books per wave), TPL ticks per
// lane (ll: the lane's index in its segment; mid: as in clear_seg).  By the definitions:
// V* = max over ticks of min(D, S) (a row maximum of the lanes' maxima); since S rises with the
// tick, the lowest tick with V = V* is the number of ticks with S < V* (a row sum); the best
// quotes after the fill are counts of ticks too, summed with it.  D and S of each tick are re-formed by
// running sums in every pass, so only the book words stay live.  Segment-uniform result.
template <int TPL, class F>
__device__ __forceinline__ ClearOut clear_row(uint32_t *__restrict__ bk, uint32_t ll, F &&mid)
{
    const uint32_t q0 = ll * TPL;
    uint32_t b[TPL], k[TPL];
    load_pairs<TPL>(bk, pad_pair(q0), b, k);
    mid();
    uint32_t sb = 0, sa = 0;
#pragma unroll
    for (int j = 0; j < TPL; ++j) {
        sb += b[j];
        sa += k[j];
    }
    uint32_t ib = sb, ia = sa;
    seg_scan_add2<4>(ib, ia);
    const uint32_t D0 = row_last(ib) - (ib - sb);  // demand at the lane's first tick
    const uint32_t Sb = ia - sa;                    // asks below the lane's first tick
    uint32_t mv = 0, d = D0, sq = Sb;
#pragma unroll
    for (int j = 0; j < TPL; ++j) {
        sq += k[j];
        mv = max(mv, min(d, sq));
        d -= b[j];
    }
    ClearOut out;
    out.v = row_max(mv);
    const uint32_t vs = out.v;
    // the fill, counting the ticks with S < V* (the clearing tick is their number), with D > V*
    // (the best bid after the fill is the highest such tick: the unmatched demand max(D - V*, 0)
    // falls with the tick and the residual bids are its drops) and with S > V* (the best ask is
    // the lowest such tick)
    uint32_t ud = unmatched(D0, vs), us = unmatched(Sb, vs), cp = 0, cb = 0, cs = 0;
    d = D0;
    sq = Sb;
#pragma unroll
    for (int j = 0; j < TPL; ++j) {
        d -= b[j];
        sq += k[j];
        const uint32_t ud1 = unmatched(d, vs), us1 = unmatched(sq, vs);
        cp += nonzero(unmatched(vs, sq));
        cb += nonzero(ud);
        cs += nonzero(us1);
        b[j] = ud - ud1;
        k[j] = us1 - us;
        ud = ud1;
        us = us1;
    }
    store_pairs<TPL>(bk, pad_pair(q0), b, k);
    // the three counts in one row sum, in 10-bit fields (a row has at most 16 TPL = 128 ticks)
    const uint32_t tot = row_sum(cp | (cb << 10) | (cs << 20));
    out.p = tot & 1023u;
    out.bb = ((tot >> 10) & 1023u) - 1u;  // no tick: kNone
    const uint32_t nsa = tot >> 20;       // ticks with S > V*, the top of the row's ticks
    out.ba = nsa ? 16u * TPL - nsa : kNone;
    return out;
}

template <int SEGLOG, class F>
__device__ __forceinline__ ClearOut clear_seg_dispatch(uint32_t *bk, uint32_t tpl, uint32_t ll, uint32_t base,
                                                       F &&mid)
{
    if constexpr (SEGLOG == 4) {  // 16-lane segments (DPP rows) hold books of up to 128 ticks
        (void)base;
        if (tpl >= 8u) return clear_row<8>(bk, ll, mid);
        if (tpl >= 4u) return clear_row<4>(bk, ll, mid);
        if (tpl == 2u) return clear_row<2>(bk, ll, mid);
        return clear_row<1>(bk, ll, mid);
    }
    if (tpl >= 4u) return clear_seg<4, SEGLOG>(bk, ll, base, mid);
    if (tpl == 2u) return clear_seg<2, SEGLOG>(bk, ll, base, mid);
    return clear_seg<1, SEGLOG>(bk, ll, base, mid);
}

// All S steps of the packed markets of one wave (wave `wave` of the item takes markets
// wave P .. wave P + P - 1 of it).  item.share = P, item.hwords = ticks per lane of the segments.
template <int SEGLOG, bool TRACE>
__device__ __forceinline__ void run_packed_seg(const EngineArgs &args, const Item &item, uint32_t wave,
                                               uint32_t lane, uint32_t *lds)
{
    constexpr uint32_t kSeg = 1u << SEGLOG;
    constexpr uint32_t kP = 64u / kSeg;
    if (wave * kP >= item.count) return;  // a wave beyond the item's markets has no LDS slots
    const uint32_t seg = lane >> SEGLOG, ll = lane & (kSeg - 1u), base = seg << SEGLOG;
    const uint32_t slot = wave * kP + seg;
    const bool active = slot < item.count;
    const uint32_t tpl = item.hwords;
    // every slot of the item's waves has its LDS (the item's share is whole waves), so a segment
    // without a market clears an empty book of its own, and the clearing has no masked store
    uint32_t *bk = lds + slot * item.stride;
    // the integer statistics live in the slot's scratch words (64-bit LDS adds by the segment's
    // first lane), which keeps registers for the per-lane generator and clearing
    uint64_t *acc = reinterpret_cast<uint64_t *>(bk + item.stride - kScr);
    uint32_t m = 0;
    DevMarket d{};
    uint32_t last = 0, prev = 0, s0 = 0;
    double sum_r = 0.0, sum_r2 = 0.0;
    if (active) {
        m = args.order[item.first + slot];
        d = args.desc[m];
        const cae_state *st = args.state + m;
        last = st->last;
        prev = st->prev;
        s0 = (uint32_t)st->steps_done;
        sum_r = st->sum_r;
        sum_r2 = st->sum_r2;
        if (ll < 5u) acc[ll] = (&st->n_trade)[ll];  // n_trade, sum_vol, sum_px, sum_spread, n_spread
    }
    {
        const uint32_t *gb = args.book + d.book_off;  // d.L = 0 without a market
        for (uint32_t q = ll; q < kSeg * tpl; q += kSeg) {
            uint2 v = make_uint2(0u, 0u);
            if (q < d.L) {
                v.x = gb[q];
                v.y = gb[d.L + q];
            }
            reinterpret_cast<uint2 *>(bk)[pad_pair(q)] = v;
        }
    }
    wave_sync();
    const double *lnT = args.lnT + d.L;  // ln(L + tick)
    const uint32_t A = active ? d.A : 0u;
    // each step's log return is added at the end of the next step, whose start issues the table
    // load (long back by then); ln_prev = ln(L + price) before the step whose return is pending
    double ln_prev = active ? lnT[last] : 0.0;
    // the generator words of agent ll (the first row) for the coming step: they do not depend on
    // the book, so each step's clearing pass computes the next step's alongside its own chain
    // (every lane computes them, unmasked, so that they share the clearing's basic block; only
    // lanes with an agent use them)
    uint32_t pw0, pw1, pw2, pw3;
    const bool row0 = ll < A;
    PhiloxStep(s0, d.id, args.k0, args.k1).words4(ll, pw0, pw1, pw2, pw3);
    for (uint32_t i = 0; i < args.S; ++i) {
        const uint32_t s = s0 + i;
        const double ln_cur = (active && i >= 1u) ? lnT[last] : 0.0;
        {
            const OrderCtx o = order_ctx<false>(d, s, Refs{last, prev, 2u * last, 0u});
            if (row0) {
                const uint32_t w = ll >= o.n_noise ? other_word<false>(o, ll, pw0, pw3) : noise_word(o, pw0, pw1);
                atomicAdd(&bk[pad_word(w)], order_qty(o, pw2));
            }
            // further rows of SEG agents until every segment's market is done (the markets of a
            // wave may have different populations), two rows at a time where both have agents:
            // their generator chains are independent, and unmasked they share one basic block
            if (ballot(kSeg < A)) {
                const PhiloxStep gen(s, d.id, args.k0, args.k1);
                for (uint32_t b0 = kSeg;; b0 += 2u * kSeg) {
                    const uint32_t a = b0 + ll, a2 = a + kSeg;
                    const bool on = a < A, on2 = a2 < A;
                    if (!ballot(on)) break;
                    if (ballot(on2)) {
                        uint32_t w0, w1, w2, w3, v0, v1, v2, v3;
                        gen.words4(a, w0, w1, w2, w3);
                        gen.words4(a2, v0, v1, v2, v3);
                        if (on) {
                            const uint32_t w = a >= o.n_noise ? other_word<false>(o, a, w0, w3) : noise_word(o, w0, w1);
                            atomicAdd(&bk[pad_word(w)], order_qty(o, w2));
                        }
                        if (on2) {
                            const uint32_t w = a2 >= o.n_noise ? other_word<false>(o, a2, v0, v3) : noise_word(o, v0, v1);
                            atomicAdd(&bk[pad_word(w)], order_qty(o, v2));
                        }
                    } else {
                        if (on) {
                            uint32_t w0, w1, w2, w3 = 0;
                            gen.words4(a, w0, w1, w2, w3);
                            const uint32_t w = a >= o.n_noise ? other_word<false>(o, a, w0, w3) : noise_word(o, w0, w1);
                            atomicAdd(&bk[pad_word(w)], order_qty(o, w2));
                        }
                        break;
                    }
                }
            }
        }
        wave_sync();
        const ClearOut co = clear_seg_dispatch<SEGLOG>(bk, tpl, ll, base, [&] {
            PhiloxStep(s + 1u, d.id, args.k0, args.k1).words4(ll, pw0, pw1, pw2, pw3);
        });
        if (active) {
            prev = last;
            if (co.v != 0) last = co.p;
            if (ll == 0) {
                if (co.v != 0) {
                    atomicAdd(reinterpret_cast<unsigned long long *>(acc), 1ull);
                    atomicAdd(reinterpret_cast<unsigned long long *>(acc + 1), (unsigned long long)co.v);
                    atomicAdd(reinterpret_cast<unsigned long long *>(acc + 2), (unsigned long long)co.p);
                }
                if (co.bb != kNone && co.ba != kNone) {
                    atomicAdd(reinterpret_cast<unsigned long long *>(acc + 3), (unsigned long long)(co.ba - co.bb));
                    atomicAdd(reinterpret_cast<unsigned long long *>(acc + 4), 1ull);
                }
            }
            if (i >= 1u) {  // the previous step's return
                const double r = ln_cur - ln_prev;
                sum_r = sum_r + r;
                sum_r2 = sum_r2 + r * r;
                ln_prev = ln_cur;
            }
            if constexpr (TRACE) {
                if (ll == 0) trace_step(args, m, i, last, co.v);
            }
        }
        wave_sync();
    }
    if (active && args.S >= 1u) {  // the last step's log return
        const double r = lnT[last] - ln_prev;
        sum_r = sum_r + r;
        sum_r2 = sum_r2 + r * r;
    }
    if (active) {
        uint32_t *gb = args.book + d.book_off;
        for (uint32_t q = ll; q < d.L; q += kSeg) {
            const uint2 v = reinterpret_cast<const uint2 *>(bk)[pad_pair(q)];
            gb[q] = v.x;
            gb[d.L + q] = v.y;
        }
        cae_state *st = args.state + m;
        if (ll < 5u) (&st->n_trade)[ll] = acc[ll];
        if (ll == 0) {
            st->last = last;
            st->prev = prev;
            st->steps_done += args.S;
            st->sum_r = sum_r;
            st->sum_r2 = sum_r2;
            st->ref2 = 2u * prev;  // twice the reference of the call's last step
        }
    }
}

template <bool TRACE>
__device__ __forceinline__ void run_packed(const EngineArgs &args, const Item &item, uint32_t wave, uint32_t lane,
                                           uint32_t *lds)
{
    if (item.share == 4u) run_packed_seg<4, TRACE>(args, item, wave, lane, lds);
    else run_packed_seg<5, TRACE>(args, item, wave, lane, lds);
}

// FULL: some market may use the mid-price model; TRACE: record the per-step series; PACK: some
// items hold packed small markets (their per-lane generator and clearing need more vector
// registers, so only ensembles that use them run this code).  Each instantiation carries only
// the code it needs, which keeps registers for the step loop.
template <int TPL_MAX, bool FULL, bool TRACE, bool PACK>
__global__ void __launch_bounds__(1024) cae_engine_kernel(const EngineArgs args)
{
    extern __shared__ __align__(16) uint32_t lds[];
    __shared__ uint32_t s_claim;
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63u;
    // wave index made provably wave-uniform, so everything derived from it (market, descriptor,
    // state, the per-step generator rounds) lives in scalar registers
    const uint32_t wave = (uint32_t)__builtin_amdgcn_readfirstlane((int)(tid >> 6));
    for (;;) {
        if (tid == 0) s_claim = atomicAdd(args.ctr, 1u);
        __syncthreads();
        const uint32_t it = (uint32_t)__builtin_amdgcn_readfirstlane((int)s_claim);
        __syncthreads();
        if (it >= args.n_items) break;
        const Item item = args.items[it];
        base_prio(item.boost, item.boost != 0u);
        const uint32_t sub = wave >> item.wpm_log2;
        const uint32_t w_in = wave & ((1u << item.wpm_log2) - 1u);
        const bool active = sub < item.count;
        if (item.pipe == 1u) {
            run_pair<TPL_MAX, FULL, TRACE>(args, item, wave, lane, blockDim.x >> 6, lds);
        } else if (PACK && item.pipe == 3u) {
            if constexpr (PACK) run_packed<TRACE>(args, item, wave, lane, lds);
        } else if (item.wpm_log2 == 0) {
            if (active) run_market<TPL_MAX, false, FULL, TRACE>(args, item, sub, w_in, lane, true, lds);
        } else if (item.pipe == 2u) {
            if constexpr (FULL) run_market_ovl_any<TPL_MAX, true, TRACE>(args, item, sub, w_in, lane, active, lds);
            else run_market_ovl<TPL_MAX, TRACE>(args, item, sub, w_in, lane, active, lds);
        } else {
            run_market<TPL_MAX, true, FULL, TRACE>(args, item, sub, w_in, lane, active, lds);
        }
        __syncthreads();
    }
    if (tid == 0) {
        // the last claimer to finish leaves the queue at zero for the next launch
        const uint32_t done = atomicAdd(args.ctr + 1, 1u);
        if (done == args.n_claimers - 1u) {
            atomicExch(args.ctr, 0u);
            atomicExch(args.ctr + 1, 0u);
        }
    }
}

// The naive engine of the paper's ablation (section IV-I): one thread per market, the book in
// global memory, every step's orders added one by one and the market cleared by serial loops
// over the L ticks (sums, argmax, top-down / bottom-up fill).  Same orders and statistics as the
// persistent engine; for comparison only.
__global__ void __launch_bounds__(64) cae_naive_kernel(const EngineArgs args, uint32_t M)
{
    const uint32_t m = blockIdx.x * 64u + threadIdx.x;
    if (m >= M) return;
    const DevMarket d = args.desc[m];
    uint32_t *bid = args.book + d.book_off;
    uint32_t *ask = bid + d.L;
    cae_state st = args.state[m];
    const double *lnT = args.lnT + d.L;
    const bool mid = (d.flags & CAE_MODEL_MASK) == CAE_MODEL_MID;
    uint32_t mid2p = st.ref2, mid2 = 2u * st.last;
    if (mid) {
        int bb = -1, ba = -1;
        for (int p = (int)d.L - 1; p >= 0 && bb < 0; --p)
            if (bid[p]) bb = p;
        for (int p = 0; p < (int)d.L && ba < 0; ++p)
            if (ask[p]) ba = p;
        if (bb >= 0 && ba >= 0) mid2 = (uint32_t)(bb + ba);
    }
    for (uint32_t i = 0; i < args.S; ++i) {
        const uint32_t s = (uint32_t)st.steps_done + i;
        const PhiloxStep ph(s, d.id, args.k0, args.k1);
        const SplitMixStep sm(s, d.id, d.A, ((uint64_t)args.k1 << 32) | args.k0);
        const bool smx = uses_splitmix(d);
        const OrderCtx o = order_ctx<true>(d, s, Refs{st.last, st.prev, mid2, mid2p});
        for (uint32_t a = 0; a < d.A; ++a) {
            uint32_t w0, w1, w2, w3;
            if (smx) sm.words4(a, w0, w1, w2, w3);
            else ph.words4(a, w0, w1, w2, w3);
            const uint32_t w = a >= d.n_noise ? other_word<true>(o, a, w0, w3)
                               : mid          ? mid_noise_word(o, w0, w1, w3)
                                              : noise_word(o, w0, w1);
            const uint32_t q = order_qty(o, w2);
            if (w & 1u) ask[w >> 1] += q;
            else bid[w >> 1] += q;
        }
        uint32_t Tb = 0;
        for (uint32_t p = 0; p < d.L; ++p) Tb += bid[p];
        uint32_t best = 0, pbest = 0, cb = 0, ca = 0;
        for (uint32_t p = 0; p < d.L; ++p) {
            ca += ask[p];
            const uint32_t V = min(Tb - cb, ca);
            if (V > best) {
                best = V;
                pbest = p;
            }
            cb += bid[p];
        }
        if (best != 0) {
            uint32_t rem = best;
            for (int p = (int)d.L - 1; p >= 0 && rem; --p) {
                const uint32_t f = min(bid[p], rem);
                bid[p] -= f;
                rem -= f;
            }
            rem = best;
            for (uint32_t p = 0; p < d.L && rem; ++p) {
                const uint32_t f = min(ask[p], rem);
                ask[p] -= f;
                rem -= f;
            }
        }
        const uint32_t old_last = st.last;
        st.prev = old_last;
        if (best != 0) {
            st.last = pbest;
            st.n_trade += 1;
            st.sum_vol += best;
            st.sum_px += pbest;
        }
        int bb = -1, ba = -1;
        for (int p = (int)d.L - 1; p >= 0; --p)
            if (bid[p]) {
                bb = p;
                break;
            }
        for (uint32_t p = 0; p < d.L; ++p)
            if (ask[p]) {
                ba = (int)p;
                break;
            }
        if (bb >= 0 && ba >= 0) {
            st.sum_spread += (uint64_t)(ba - bb);
            st.n_spread += 1;
        }
        mid2p = mid2;
        mid2 = next_mid2(mid, bb >= 0 ? (uint32_t)bb : kNone, ba >= 0 ? (uint32_t)ba : kNone, st.last);
        const double r = lnT[st.last] - lnT[st.prev];
        st.sum_r = st.sum_r + r;
        st.sum_r2 = st.sum_r2 + r * r;
    }
    st.ref2 = mid2p;
    st.steps_done += args.S;
    args.state[m] = st;
}

// One clearing pass over n books of L ticks: one wave per book, four books per workgroup.
template <int TPL>
__global__ void __launch_bounds__(256) cae_clear_kernel(uint32_t L, uint32_t n, uint32_t *book,
                                                        uint32_t *pstar, uint32_t *vstar)
{
    extern __shared__ __align__(16) uint32_t lds[];
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = threadIdx.x >> 6;
    const uint32_t i = blockIdx.x * 4u + wave;
    if (i >= n) return;
    uint32_t *bk = lds + wave * (2u * 64u * TPL);
    uint32_t *gb = book + (uint64_t)i * 2u * L;
    for (uint32_t q = lane; q < 64u * TPL; q += 64u) {
        uint2 v = make_uint2(0u, 0u);
        if (q < L) {
            v.x = gb[q];
            v.y = gb[L + q];
        }
        reinterpret_cast<uint2 *>(bk)[q] = v;
    }
    wave_sync();
    const ClearOut co = clear_wave<TPL>(bk, lane);
    wave_sync();
    for (uint32_t q = lane; q < L; q += 64u) {
        const uint2 v = reinterpret_cast<const uint2 *>(bk)[q];
        gb[q] = v.x;
        gb[L + q] = v.y;
    }
    if (lane == 0) {
        pstar[i] = co.p;
        vstar[i] = co.v;
    }
}

__global__ void cae_fill_kernel(uint32_t *p, uint64_t n, uint32_t v)
{
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// ------------------------------------------------------------------------------------------
// Host side.
// ------------------------------------------------------------------------------------------
thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                   \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess) return fail(CAE_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

constexpr uint32_t kVersion = 1;
constexpr size_t kAlign = 256;

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

uint32_t tpl_for(uint32_t L)
{
    uint32_t t = 1;
    while (64u * t < L) t <<= 1;
    return t;
}

// Words of one order-bin buffer of an overlapped market: 2K + 3 (bid, ask) pairs, rounded up to
// a power of two of at least 64 so that markets of nearby K share items.
constexpr uint32_t kMaxOverlapK = 1022, kMaxOverlapKMid = 510;
uint32_t hwords_for(uint32_t K, bool mid)
{
    const uint32_t need = mid ? 8u * K + 12u : 4u * K + 6u;  // last-tick: 2K + 3 pairs; mid: 4K + 6
    uint32_t w = 64;
    while (w < need) w <<= 1;
    return w;
}

uint32_t lclass(uint32_t L)
{
    uint32_t c = 0;
    while (c < 4 && (64u << c) < L) ++c;
    return c;
}

uint32_t aclass(uint32_t A)
{
    uint32_t lg = 31u - (uint32_t)__builtin_clz(A);
    lg = std::min(std::max(lg, 6u), 13u);
    return lg - 6u;
}

int validate(const cae_market *desc, uint32_t M)
{
    if (!desc) return fail(CAE_EINVAL, "desc is NULL");
    if (M == 0) return fail(CAE_EINVAL, "M must be >= 1");
    for (uint32_t m = 0; m < M; ++m) {
        const cae_market &d = desc[m];
        if (d.L < 1 || d.L > 1024) return fail(CAE_EINVAL, "market %u: L=%u outside 1..1024", m, d.L);
        if (d.A < 1) return fail(CAE_EINVAL, "market %u: A must be >= 1", m);
        if (d.K > (1u << 30)) return fail(CAE_EINVAL, "market %u: K=%u too large", m, d.K);
        if (d.Q < 1) return fail(CAE_EINVAL, "market %u: Q must be >= 1", m);
        if ((uint64_t)d.A * d.Q >= (1ull << 32)) return fail(CAE_EINVAL, "market %u: A*Q >= 2^32", m);
        if ((uint64_t)d.n_noise + d.n_mom > d.A)
            return fail(CAE_EINVAL, "market %u: n_noise + n_mom > A", m);
        if (d.maker_half_spread >= d.L) return fail(CAE_EINVAL, "market %u: maker_half_spread >= L", m);
        const uint32_t model = d.flags & CAE_MODEL_MASK;
        if (model != CAE_MODEL_LAST && model != CAE_MODEL_MID)
            return fail(CAE_EINVAL, "market %u: unknown agent model %u", m, model);
        const uint32_t gen = (d.flags >> CAE_GEN_SHIFT) & 0xFFu;
        if (gen != CAE_GEN_PHILOX && gen != CAE_GEN_SPLITMIX)
            return fail(CAE_EINVAL, "market %u: unknown generator %u", m, gen);
        if (model == CAE_MODEL_LAST && (d.flags >> CAE_PMKT_SHIFT) != 0)
            return fail(CAE_EINVAL, "market %u: P_mkt needs the mid-price model", m);
        if (model == CAE_MODEL_MID && d.K >= (1u << 20))
            return fail(CAE_EINVAL, "market %u: K=%u too large for the mid-price model", m, d.K);
    }
    return CAE_OK;
}

struct Layout {
    size_t off_desc, off_order, off_items, off_ctr, off_lnt, total;
};

Layout layout_for(uint32_t M)
{
    Layout l;
    size_t o = 0;
    l.off_desc = o;
    o = align_up(o + sizeof(DevMarket) * (size_t)M, kAlign);
    l.off_order = o;
    o = align_up(o + sizeof(uint32_t) * (size_t)M, kAlign);
    l.off_items = o;
    o = align_up(o + sizeof(Item) * (size_t)M, kAlign);
    l.off_ctr = o;
    o = align_up(o + 4 * sizeof(uint32_t), kAlign);
    l.off_lnt = o;
    o = align_up(o + sizeof(double) * 2049, kAlign);
    l.total = o;
    return l;
}

int device_cus(int dev, uint32_t *num_cu)
{
    int v = 0;
    HIP_TRY(hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev));
    *num_cu = (uint32_t)v;
    return CAE_OK;
}

using EngineFn = void (*)(const EngineArgs);

// Packed items exist only in ensembles whose books all have at most kPackMaxL ticks (so the
// packed instantiations are those of small books).
constexpr uint32_t kPackMaxL = 128;

template <bool FULL, bool TRACE>
EngineFn engine_fn_t(uint32_t tpl_max, bool pack)
{
    if (pack) return tpl_max <= 1 ? cae_engine_kernel<1, FULL, TRACE, true> : cae_engine_kernel<2, FULL, TRACE, true>;
    switch (tpl_max) {
    case 1: return cae_engine_kernel<1, FULL, TRACE, false>;
    case 2: return cae_engine_kernel<2, FULL, TRACE, false>;
    case 4: return cae_engine_kernel<4, FULL, TRACE, false>;
    case 8: return cae_engine_kernel<8, FULL, TRACE, false>;
    default: return cae_engine_kernel<16, FULL, TRACE, false>;
    }
}

// The instantiation for the largest book, with mid-price code only when some market uses that
// model, trace stores only for cae_step_traced and the packed path only when items use it.
EngineFn engine_fn(uint32_t tpl_max, bool mid, bool trace, bool pack)
{
    if (mid) return trace ? engine_fn_t<true, true>(tpl_max, pack) : engine_fn_t<true, false>(tpl_max, pack);
    return trace ? engine_fn_t<false, true>(tpl_max, pack) : engine_fn_t<false, false>(tpl_max, pack);
}

uint32_t auto_wpm(uint32_t L, uint32_t A)
{
    (void)L;
    // about 8 agents per lane per step, at most 16 waves
    uint32_t w = 1;
    while (w < 16 && 64u * 8u * (2u * w) <= A) w <<= 1;
    return w;
}

}  // namespace

struct cae_ensemble {
    int device = 0;
    uint32_t M = 0;
    uint64_t seed = 0;
    hipStream_t stream = nullptr;
    cae_buffers dev{};
    std::vector<cae_market> desc;
    std::vector<uint64_t> steps_done;
    uint64_t book_words = 0;
    Layout lay{};
    uint32_t n_items = 0, tpl_max = 1, waves_per_group = 1, lds_bytes = 0, grid = 0;
    bool any_mid = false;  // some market uses the mid-price model or the SplitMix64 generator
    bool any_pack = false; // some item holds packed small markets
    cae_tuning tuning{};
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    bool have_timing = false;
};

namespace {

// Build the work list: markets of equal (waves per market, ticks per lane) are packed into
// items that fill a workgroup; items run longest first.
int build_schedule(cae_ensemble *e, const cae_tuning *tn, const uint32_t *ids,
                   std::vector<DevMarket> &dm, std::vector<uint32_t> &order, std::vector<Item> &items)
{
    const uint32_t M = e->M;
    cae_tuning t{};
    if (tn) t = *tn;
    std::vector<uint32_t> wpm(M);
    uint32_t wpm_max = 1, tpl_max = 1;
    for (uint32_t m = 0; m < M; ++m)
        e->any_mid |= (e->desc[m].flags & CAE_MODEL_MASK) == CAE_MODEL_MID ||
                      ((e->desc[m].flags >> CAE_GEN_SHIFT) & 0xFFu) == CAE_GEN_SPLITMIX;
    std::vector<uint32_t> packp(M, 0u);
    for (uint32_t c = 0; c < CAE_NUM_CLASSES; ++c)
        if (t.pack[c] != 0 && t.pack[c] != 2 && t.pack[c] != 4) return fail(CAE_EINVAL, "pack[%u] must be 0, 2 or 4", c);
    uint32_t maxL = 0;
    for (uint32_t m = 0; m < M; ++m) maxL = std::max(maxL, e->desc[m].L);
    e->any_pack = false;
    for (uint32_t m = 0; m < M; ++m) {
        const cae_market &d = e->desc[m];
        const uint32_t c = lclass(d.L) * 8u + aclass(d.A);
        // packed: last-tick Philox markets whose book fits 8 ticks per lane of a segment, in an
        // ensemble of small books
        const uint32_t P = maxL <= kPackMaxL ? t.pack[c] : 0u;
        if (P && (d.flags & 0xFFFFu) == 0u && d.L <= 512u / P) {
            packp[m] = P;
            wpm[m] = 1;
            e->any_pack = true;
            continue;
        }
        uint32_t w = t.waves_per_market[c];
        if (w == 0) w = auto_wpm(d.L, d.A);
        if (w > 16 || (w & (w - 1)) != 0) return fail(CAE_EINVAL, "waves_per_market[%u]=%u not a power of 2 <= 16", c, w);
        if (t.pipelined[c] > 1) return fail(CAE_EINVAL, "pipelined[%u] must be 0 or 1", c);
        if (t.pipelined[c]) w = 1;  // a pipelined pair uses the whole workgroup
        wpm[m] = w;
        t.waves_per_market[c] = (uint8_t)w;
        if (w < 2) t.overlap[c] = 0;
        wpm_max = std::max(wpm_max, w);
        tpl_max = std::max(tpl_max, tpl_for(d.L));
    }
    {  // report packing only for the classes it applies to
        bool used[CAE_NUM_CLASSES] = {};
        for (uint32_t m = 0; m < M; ++m)
            if (packp[m]) used[lclass(e->desc[m].L) * 8u + aclass(e->desc[m].A)] = true;
        for (uint32_t c = 0; c < CAE_NUM_CLASSES; ++c)
            if (!used[c]) t.pack[c] = 0;
    }
    uint32_t G = t.waves_per_group;
    if (G == 0) G = std::max(wpm_max, 4u);
    if (G > 16 || G < wpm_max) return fail(CAE_EINVAL, "waves_per_group=%u must be in [max waves_per_market=%u, 16]", G, wpm_max);
    bool any_pipe = false;
    for (uint32_t c = 0; c < CAE_NUM_CLASSES; ++c) any_pipe |= t.pipelined[c] != 0;
    if (any_pipe && G < 2) return fail(CAE_EINVAL, "pipelined classes need waves_per_group >= 2");
    uint32_t lds_budget = t.max_lds_bytes ? t.max_lds_bytes : 64u * 1024u;
    if (lds_budget > 160u * 1024u) lds_budget = 160u * 1024u;

    // LPT cost of one market-step: measured per class if given, else agent work plus the
    // clearing wave's pass over 64*tpl ticks
    std::vector<double> cost(M);
    for (uint32_t m = 0; m < M; ++m) {
        const cae_market &d = e->desc[m];
        const uint32_t c = lclass(d.L) * 8u + aclass(d.A);
        const float cc = tn ? tn->class_cost[c] : 0.0f;
        if (!(cc >= 0.0f)) return fail(CAE_EINVAL, "class_cost[%u] is negative or NaN", c);
        cost[m] = cc > 0.0f ? (double)cc : (double)d.A + 2.0 * 64.0 * tpl_for(d.L);
    }
    order.resize(M);
    for (uint32_t m = 0; m < M; ++m) order[m] = m;
    const bool keep = (t.flags & 1u) != 0;
    if (!keep)
        std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return cost[a] > cost[b]; });

    // open bins per (wpm, tpl, mode, clearing share, bin buffer size)
    struct Bin { std::vector<uint32_t> ms; uint32_t wpm, tpl, pipe, share, hw; };
    std::vector<Bin> open;
    std::vector<std::pair<double, Bin>> done;
    for (uint32_t idx = 0; idx < M; ++idx) {
        const uint32_t m = order[idx];
        const uint32_t w = wpm[m];
        uint32_t tp = tpl_for(e->desc[m].L);
        const uint32_t c = lclass(e->desc[m].L) * 8u + aclass(e->desc[m].A);
        // overlapped markets keep two buffers of bins in LDS; wider offset ranges run plain
        const bool mid = (e->desc[m].flags & CAE_MODEL_MASK) == CAE_MODEL_MID;
        const uint32_t ov = e->desc[m].K <= (mid ? kMaxOverlapKMid : kMaxOverlapK) ? t.overlap[c] : 0u;
        uint32_t pp = t.pipelined[c] ? 1u : (ov ? 2u : 0u);
        uint32_t share = ov ? ov - 1u : 0u;
        uint32_t hw = ov ? hwords_for(e->desc[m].K, mid) : 0u;
        uint32_t stride = 2u * 64u * tp + 2u * hw + kScr;
        uint32_t cap = pp == 1u ? 2u : G / w;
        if (packp[m]) {  // P markets per wave, books of seg * hw ticks (hw ticks per lane)
            const uint32_t seg = 64u / packp[m];
            pp = 3u;
            share = packp[m];
            hw = 1u;
            while (seg * hw < e->desc[m].L) hw <<= 1;
            tp = 0u;
            stride = 2u * seg * hw + 4u * ((seg * hw + 31u) / 32u) + kScr;  // padded (pad_pair)
            cap = G * packp[m];
        }
        cap = std::max(1u, std::min(cap, lds_budget / (stride * 4u)));
        if (packp[m] && cap > packp[m]) cap -= cap % packp[m];  // whole waves (the LDS holds them)
        Bin *b = nullptr;
        for (auto &x : open)
            if (x.wpm == w && x.tpl == tp && x.pipe == pp && x.share == share && x.hw == hw) b = &x;
        if (!b) {
            open.push_back(Bin{{}, w, tp, pp, share, hw});
            b = &open.back();
        }
        b->ms.push_back(m);
        if (b->ms.size() == cap) {
            double c = 0;
            for (uint32_t mm : b->ms) c = std::max(c, cost[mm]);
            done.push_back({c, *b});
            b->ms.clear();
        }
    }
    for (auto &b : open)
        if (!b.ms.empty()) {
            double c = 0;
            for (uint32_t mm : b.ms) c = std::max(c, cost[mm]);
            done.push_back({c, b});
        }
    if (!keep)
        std::stable_sort(done.begin(), done.end(), [](const auto &a, const auto &b) { return a.first > b.first; });

    // Priority boost (tuning flag bit 1): items of lock-step or single-wave markets whose cost
    // per step is within a quarter of the largest, when some item falls below that (a uniform
    // ensemble keeps one level for all).
    const bool boost = (t.flags & 2u) != 0;
    double cmax = 0.0, cmin = 0.0;
    for (size_t i = 0; i < done.size(); ++i) {
        cmax = i ? std::max(cmax, done[i].first) : done[i].first;
        cmin = i ? std::min(cmin, done[i].first) : done[i].first;
    }
    const bool tiers = boost && cmin < 0.75 * cmax;

    order.clear();
    items.clear();
    uint32_t lds_max = 0;
    for (auto &p : done) {
        const Bin &b = p.second;
        Item it;
        it.first = (uint32_t)order.size();
        it.count = (uint32_t)b.ms.size();
        it.wpm_log2 = (uint32_t)__builtin_ctz(b.wpm);
        // packed books: 2 words per tick plus 4 words of padding per 32 ticks (pad_pair)
        const uint32_t pticks = b.pipe == 3u ? (64u / b.share) * b.hw : 0u;
        it.stride = b.pipe == 3u ? 2u * pticks + 4u * ((pticks + 31u) / 32u) + kScr
                                 : 2u * 64u * b.tpl + 2u * b.hw + kScr;
        it.pipe = b.pipe;
        it.share = b.share;
        it.hoff = 2u * 64u * b.tpl;
        it.hwords = b.hw;
        it.boost = (tiers && (b.pipe == 0u || b.pipe == 2u) && p.first >= 0.75 * cmax) ? 1u : 0u;
        for (uint32_t mm : b.ms) order.push_back(mm);
        items.push_back(it);
        // packed items hold LDS for every slot of their waves, markets or not
        const uint32_t slots = b.pipe == 3u ? (it.count + b.share - 1u) / b.share * b.share : it.count;
        lds_max = std::max(lds_max, slots * it.stride * 4u);
    }

    // device descriptors
    dm.resize(M);
    uint64_t off = 0;
    for (uint32_t m = 0; m < M; ++m) {
        const cae_market &d = e->desc[m];
        DevMarket x{};
        x.L = d.L; x.A = d.A; x.K = d.K; x.Q = d.Q;
        x.n_noise = d.n_noise; x.n_mom = d.n_mom; x.h = d.maker_half_spread;
        x.tpl = tpl_for(d.L);
        x.book_off = off;
        x.id = ids ? ids[m] : m;
        x.flags = d.flags;
        off += 2ull * d.L;
        dm[m] = x;
    }
    t.waves_per_group = G;
    t.max_lds_bytes = lds_budget;
    e->tuning = t;
    e->n_items = (uint32_t)items.size();
    e->tpl_max = tpl_max;
    e->waves_per_group = G;
    e->lds_bytes = lds_max;

    uint32_t ncu = 0;
    int rc = device_cus(e->device, &ncu);
    if (rc) return rc;
    int per_cu = 0;
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(engine_fn(tpl_max, e->any_mid, false, e->any_pack)),
                                                         (int)(G * 64u), (size_t)lds_max));
    if (per_cu < 1) return fail(CAE_EINVAL, "schedule does not fit on a CU (lds %u B, %u waves)", lds_max, G);
    if (t.groups_per_cu) per_cu = std::min<int>(per_cu, (int)t.groups_per_cu);
    e->tuning.groups_per_cu = (uint32_t)per_cu;
    e->grid = std::min<uint32_t>(e->n_items, ncu * (uint32_t)per_cu);
    return CAE_OK;
}

}  // namespace

namespace cae_detail {
int set_error(int code, const char *msg) { return fail(code, "%s", msg); }
}  // namespace cae_detail

extern "C" {

const char *cae_strerror(int code)
{
    switch (code) {
    case CAE_OK: return "ok";
    case CAE_EINVAL: return "invalid argument";
    case CAE_EOVERFLOW: return "book could overflow 32 bits";
    case CAE_ENOSPACE: return "buffer too small";
    case CAE_EHIP: return "HIP runtime error";
    case CAE_ESTATE: return "invalid state";
    default: return "unknown error";
    }
}

const char *cae_last_error(void) { return g_err.c_str(); }

int cae_device_info(uint32_t *num_cu, uint32_t *version)
{
    if (version) *version = kVersion;
    if (num_cu) {
        int dev = 0;
        HIP_TRY(hipGetDevice(&dev));
        return device_cus(dev, num_cu);
    }
    return CAE_OK;
}

int cae_sizes(const cae_market *desc, uint32_t M, cae_sizes_t *out)
{
    if (!out) return fail(CAE_EINVAL, "out is NULL");
    int rc = validate(desc, M);
    if (rc) return rc;
    uint64_t words = 0;
    for (uint32_t m = 0; m < M; ++m) words += 2ull * desc[m].L;
    out->book_words = words;
    out->book_bytes = 4ull * words;
    out->state_bytes = (uint64_t)M * sizeof(cae_state);
    out->workspace_bytes = layout_for(M).total;
    return CAE_OK;
}

int cae_create(const cae_market *desc, uint32_t M, uint64_t seed, const uint32_t *market_ids,
               const cae_buffers *dev, void *stream, const cae_tuning *tuning, cae_ensemble **out)
{
    if (!out || !dev || !dev->book || !dev->state || !dev->workspace)
        return fail(CAE_EINVAL, "NULL handle or device buffer");
    *out = nullptr;
    int rc = validate(desc, M);
    if (rc) return rc;
    cae_ensemble *e = new cae_ensemble();
    HIP_TRY(hipGetDevice(&e->device));
    e->M = M;
    e->seed = seed;
    e->stream = (hipStream_t)stream;
    e->dev = *dev;
    e->desc.assign(desc, desc + M);
    e->steps_done.assign(M, 0);
    e->lay = layout_for(M);
    for (uint32_t m = 0; m < M; ++m) e->book_words += 2ull * desc[m].L;

    std::vector<DevMarket> dm;
    std::vector<uint32_t> order;
    std::vector<Item> items;
    rc = build_schedule(e, tuning, market_ids, dm, order, items);
    if (rc) {
        delete e;
        return rc;
    }
    std::vector<unsigned char> ws(e->lay.total, 0);
    std::memcpy(ws.data() + e->lay.off_desc, dm.data(), sizeof(DevMarket) * M);
    std::memcpy(ws.data() + e->lay.off_order, order.data(), sizeof(uint32_t) * M);
    std::memcpy(ws.data() + e->lay.off_items, items.data(), sizeof(Item) * items.size());
    std::vector<double> lnt(2049, 0.0);
    for (int n = 1; n <= 2048; ++n) lnt[n] = std::log((double)n);
    std::memcpy(ws.data() + e->lay.off_lnt, lnt.data(), sizeof(double) * 2049);
    std::vector<cae_state> st(M);
    for (uint32_t m = 0; m < M; ++m) {
        std::memset(&st[m], 0, sizeof(cae_state));
        st[m].last = desc[m].L / 2;
        st[m].prev = desc[m].L / 2;
        st[m].ref2 = 2u * (desc[m].L / 2);
    }
    auto cleanup = [&](int code) {
        delete e;
        return code;
    };
    hipError_t he;
    he = hipMemcpyAsync(dev->workspace, ws.data(), ws.size(), hipMemcpyHostToDevice, e->stream);
    if (he == hipSuccess)
        he = hipMemcpyAsync(dev->state, st.data(), sizeof(cae_state) * M, hipMemcpyHostToDevice, e->stream);
    if (he == hipSuccess) {
        const uint32_t blocks = (uint32_t)std::min<uint64_t>((e->book_words + 255) / 256, 4096);
        hipLaunchKernelGGL(cae_fill_kernel, dim3(blocks), dim3(256), 0, e->stream, dev->book, e->book_words, 0u);
        he = hipGetLastError();
    }
    if (he == hipSuccess) he = hipStreamSynchronize(e->stream);
    if (he == hipSuccess) he = hipEventCreate(&e->ev0);
    if (he == hipSuccess) he = hipEventCreate(&e->ev1);
    if (he != hipSuccess) return cleanup(fail(CAE_EHIP, "create: %s", hipGetErrorString(he)));
    *out = e;
    return CAE_OK;
}

static int step_impl(cae_ensemble *e, uint32_t S, bool naive, uint32_t *tr_price = nullptr,
                     uint32_t *tr_vol = nullptr, uint64_t tr_ld = 0)
{
    if (!e) return fail(CAE_EINVAL, "NULL ensemble");
    if ((tr_price || tr_vol) && tr_ld < S) return fail(CAE_EINVAL, "trace row length %llu < S = %u",
                                                        (unsigned long long)tr_ld, S);
    if (S == 0) return CAE_OK;
    for (uint32_t m = 0; m < e->M; ++m) {
        const unsigned __int128 tot = (unsigned __int128)(e->steps_done[m] + S) * e->desc[m].A * e->desc[m].Q;
        if (tot >= ((unsigned __int128)1 << 32))
            return fail(CAE_EOVERFLOW, "market %u: (steps_done + S) * A * Q >= 2^32", m);
    }
    HIP_TRY(hipSetDevice(e->device));
    unsigned char *ws = static_cast<unsigned char *>(e->dev.workspace);
    EngineArgs a;
    a.desc = reinterpret_cast<const DevMarket *>(ws + e->lay.off_desc);
    a.order = reinterpret_cast<const uint32_t *>(ws + e->lay.off_order);
    a.items = reinterpret_cast<const Item *>(ws + e->lay.off_items);
    a.ctr = reinterpret_cast<uint32_t *>(ws + e->lay.off_ctr);
    a.book = e->dev.book;
    a.state = e->dev.state;
    a.lnT = reinterpret_cast<const double *>(ws + e->lay.off_lnt);
    a.tr_price = tr_price;
    a.tr_vol = tr_vol;
    a.tr_ld = tr_ld;
    a.n_items = e->n_items;
    a.n_claimers = e->grid;
    a.S = S;
    a.k0 = (uint32_t)e->seed;
    a.k1 = (uint32_t)(e->seed >> 32);
    HIP_TRY(hipEventRecord(e->ev0, e->stream));
    if (naive)
        hipLaunchKernelGGL(cae_naive_kernel, dim3((e->M + 63u) / 64u), dim3(64), 0, e->stream, a, e->M);
    else
        hipLaunchKernelGGL(engine_fn(e->tpl_max, e->any_mid, tr_price != nullptr || tr_vol != nullptr, e->any_pack),
                           dim3(e->grid), dim3(e->waves_per_group * 64u), e->lds_bytes,
                           e->stream, a);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipEventRecord(e->ev1, e->stream));
    e->have_timing = true;
    for (uint32_t m = 0; m < e->M; ++m) e->steps_done[m] += S;
    return CAE_OK;
}

int cae_step(cae_ensemble *e, uint32_t S) { return step_impl(e, S, false); }

int cae_step_naive(cae_ensemble *e, uint32_t S) { return step_impl(e, S, true); }

int cae_step_traced(cae_ensemble *e, uint32_t S, uint32_t *dev_price, uint32_t *dev_volume, uint64_t ld)
{
    return step_impl(e, S, false, dev_price, dev_volume, ld);
}

int cae_last_step_ms(cae_ensemble *e, float *ms)
{
    if (!e || !ms) return fail(CAE_EINVAL, "NULL argument");
    if (!e->have_timing) return fail(CAE_ESTATE, "no step has been launched");
    HIP_TRY(hipEventSynchronize(e->ev1));
    HIP_TRY(hipEventElapsedTime(ms, e->ev0, e->ev1));
    return CAE_OK;
}

int cae_read_books(cae_ensemble *e, uint32_t *host_book, uint64_t n_words)
{
    if (!e || !host_book) return fail(CAE_EINVAL, "NULL argument");
    if (n_words < e->book_words) return fail(CAE_ENOSPACE, "need %llu words", (unsigned long long)e->book_words);
    HIP_TRY(hipSetDevice(e->device));
    HIP_TRY(hipMemcpyAsync(host_book, e->dev.book, 4ull * e->book_words, hipMemcpyDeviceToHost, e->stream));
    HIP_TRY(hipStreamSynchronize(e->stream));
    return CAE_OK;
}

int cae_read_state(cae_ensemble *e, cae_state *host_state, uint32_t M)
{
    if (!e || !host_state) return fail(CAE_EINVAL, "NULL argument");
    if (M < e->M) return fail(CAE_ENOSPACE, "need %u states", e->M);
    HIP_TRY(hipSetDevice(e->device));
    HIP_TRY(hipMemcpyAsync(host_state, e->dev.state, sizeof(cae_state) * e->M, hipMemcpyDeviceToHost, e->stream));
    HIP_TRY(hipStreamSynchronize(e->stream));
    return CAE_OK;
}

int cae_write_state(cae_ensemble *e, const cae_state *host_state, uint32_t M, const uint32_t *host_book,
                    uint64_t n_words)
{
    if (!e || !host_state || !host_book) return fail(CAE_EINVAL, "NULL argument");
    if (M != e->M) return fail(CAE_EINVAL, "M=%u does not match the ensemble (%u)", M, e->M);
    if (n_words != e->book_words)
        return fail(CAE_EINVAL, "n_words=%llu does not match the ensemble (%llu)", (unsigned long long)n_words,
                    (unsigned long long)e->book_words);
    for (uint32_t m = 0; m < M; ++m) {
        if (host_state[m].last >= e->desc[m].L || host_state[m].prev >= e->desc[m].L)
            return fail(CAE_EINVAL, "market %u: last/prev outside the grid", m);
        if (host_state[m].ref2 > 2u * (e->desc[m].L - 1u) || host_state[m].reserved != 0)
            return fail(CAE_EINVAL, "market %u: ref2 outside the grid or reserved != 0", m);
        const unsigned __int128 tot = (unsigned __int128)host_state[m].steps_done * e->desc[m].A * e->desc[m].Q;
        if (tot >= ((unsigned __int128)1 << 32)) return fail(CAE_EINVAL, "market %u: steps_done past the guard", m);
    }
    // Every step adds at most A Q shares to a market's book, so a book reached by steps_done steps
    // holds at most steps_done A Q shares on its two sides together.  cae_step's overflow guard
    // relies on that bound (it keeps every per-tick count, cumulative sum and the 64-bit packed
    // (bid, ask) additions below 2^32); a book that breaks it is rejected here.
    uint64_t off = 0;
    for (uint32_t m = 0; m < M; ++m) {
        const uint32_t L = e->desc[m].L;
        uint64_t held = 0;
        for (uint64_t i = 0; i < 2ull * L; ++i) held += host_book[off + i];
        const uint64_t bound = host_state[m].steps_done * e->desc[m].A * e->desc[m].Q;  // < 2^32 (checked above)
        if (held > bound)
            return fail(CAE_EINVAL, "market %u: the book holds %llu shares, more than steps_done * A * Q = %llu", m,
                        (unsigned long long)held, (unsigned long long)bound);
        off += 2ull * L;
    }
    HIP_TRY(hipSetDevice(e->device));
    HIP_TRY(hipMemcpyAsync(e->dev.state, host_state, sizeof(cae_state) * M, hipMemcpyHostToDevice, e->stream));
    HIP_TRY(hipMemcpyAsync(e->dev.book, host_book, 4ull * n_words, hipMemcpyHostToDevice, e->stream));
    HIP_TRY(hipStreamSynchronize(e->stream));
    for (uint32_t m = 0; m < M; ++m) e->steps_done[m] = host_state[m].steps_done;
    return CAE_OK;
}

int cae_get_tuning(const cae_ensemble *e, cae_tuning *out)
{
    if (!e || !out) return fail(CAE_EINVAL, "NULL argument");
    *out = e->tuning;
    return CAE_OK;
}

int cae_destroy(cae_ensemble *e)
{
    if (!e) return CAE_OK;
    if (e->ev0) (void)hipEventDestroy(e->ev0);
    if (e->ev1) (void)hipEventDestroy(e->ev1);
    delete e;
    return CAE_OK;
}

int cae_clear(uint32_t L, uint32_t M, uint32_t *dev_book, uint32_t *dev_pstar, uint32_t *dev_vstar, void *stream)
{
    if (L < 1 || L > 1024) return fail(CAE_EINVAL, "L=%u outside 1..1024", L);
    if (!dev_book || !dev_pstar || !dev_vstar) return fail(CAE_EINVAL, "NULL device pointer");
    if (M == 0) return CAE_OK;
    const uint32_t tpl = tpl_for(L);
    const dim3 grid((M + 3u) / 4u), block(256);
    const size_t lds = 4u * 2u * 64u * tpl * 4u;
    hipStream_t s = (hipStream_t)stream;
    switch (tpl) {
    case 1: hipLaunchKernelGGL(cae_clear_kernel<1>, grid, block, lds, s, L, M, dev_book, dev_pstar, dev_vstar); break;
    case 2: hipLaunchKernelGGL(cae_clear_kernel<2>, grid, block, lds, s, L, M, dev_book, dev_pstar, dev_vstar); break;
    case 4: hipLaunchKernelGGL(cae_clear_kernel<4>, grid, block, lds, s, L, M, dev_book, dev_pstar, dev_vstar); break;
    case 8: hipLaunchKernelGGL(cae_clear_kernel<8>, grid, block, lds, s, L, M, dev_book, dev_pstar, dev_vstar); break;
    default: hipLaunchKernelGGL(cae_clear_kernel<16>, grid, block, lds, s, L, M, dev_book, dev_pstar, dev_vstar); break;
    }
    HIP_TRY(hipGetLastError());
    return CAE_OK;
}

}  // extern "C"
