/*
 * cae_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, sequential CPU implementation of the call-auction ensemble that the GPU
 * library computes.  Only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it; the product path never does.  It shares no code, header, table or
 * constant generator with the GPU library: both sides are written independently from the
 * definitions below.
 *
 * What is computed (KineticSim paper, section II-A and section III):
 *   - per agent and step, an order (side, tick, quantity) drawn from a counter-based
 *     generator (section III-C "Order Quantity and RNG", section III-G);
 *   - aggregation of all orders into the resting book (section III-C "Aggregation");
 *   - cumulative demand D(p) = sum_{q>=p} BUY[q] and supply S(p) = sum_{q<=p} SELL[q]
 *     (Eq. 1), the clearing price p* = argmax_p min(D(p), S(p)) with ties to the lowest
 *     tick (Eq. 2; section III-D), and price-priority allocation with the unmatched
 *     interest resting for the next step (section II-A; worked example of section IV-C);
 *   - per-step market statistics kept with the final book (Algorithm 1, "ENSURE").
 *
 * Readings where the paper is silent (each one is listed in the design notes):
 *   - generator: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel Random Numbers: As
 *     Easy as 1, 2, 3", SC'11) instead of the paper's under-specified SplitMix64 hash.
 *     Counter = (absolute step, agent, market, 0), key = (seed low word, seed high word).
 *     A descriptor may select the paper's SplitMix64 instead, with the coordinate hash read as
 *     a position in the seeded stream (orc_splitmix_words);
 *   - integer ranges use the exact multiply-high floor(w * n / 2^32) of a 32-bit word w,
 *     which is the paper's 1 + floor(u * q_max) with u = w / 2^32;
 *   - the agents' reference price is the last clearing tick (integer, no rounding step);
 *   - the combined book (resting + new orders) is cleared each step;
 *   - a step whose best volume is 0 trades nothing and leaves the last price unchanged;
 *   - the opening book is empty and the opening price is floor(L/2).
 *
 * Everything here is written for clarity, not speed: no scans, no atomics, no blocking.
 * Build: gcc -O2 -std=c11 -ffp-contract=off -shared -fPIC (see build.py next to this file).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------------------------------
 * Philox4x32-10, as published (SC'11, section 3.2; the Philox-4x32 S-box and the key
 * schedule with Weyl constants).  Ten rounds; round r (1-based) uses the key
 * (k0 + (r-1)*W0, k1 + (r-1)*W1) mod 2^32.  One round maps (c0, c1, c2, c3) to
 * (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0)).
 * ------------------------------------------------------------------------------------- */
#define ORC_PHILOX_M0 0xD2511F53u
#define ORC_PHILOX_M1 0xCD9E8D57u
#define ORC_PHILOX_W0 0x9E3779B9u
#define ORC_PHILOX_W1 0xBB67AE85u

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t prod0 = (uint64_t)ORC_PHILOX_M0 * (uint64_t)c0;
        uint64_t prod1 = (uint64_t)ORC_PHILOX_M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += ORC_PHILOX_W0;
        k1 += ORC_PHILOX_W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* ---------------------------------------------------------------------------------------
 * SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number generators",
 * OOPSLA 2014), the generator the paper names in section III-G.  Its output for a 64-bit input
 * x: z = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9; z = (z ^ (z >> 27)) * 0x94d049bb133111eb;
 * z ^ (z >> 31) (the mixing steps printed in section III-G).  The k-th output of the stream
 * seeded with s mixes s + (k + 1) * 0x9e3779b97f4a7c15.
 * ------------------------------------------------------------------------------------- */
uint64_t orc_splitmix64_mix(uint64_t x)
{
    uint64_t z = x;
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

/* Reading of the paper's coordinate hash(m A + a, s, c, seed): the stream seeded with `seed`,
 * at position k = gid * 2^34 + s * 4 + c (gid = m A + a, channel c = 0..3), i.e. the mix of
 * seed + (k + 1) * 0x9e3779b97f4a7c15; each channel's word is the output's high half. */
void orc_splitmix_words(uint64_t gid, uint32_t s, uint64_t seed, uint32_t w[4])
{
    for (uint32_t c = 0; c < 4; ++c) {
        uint64_t k = (gid << 34) + ((uint64_t)s << 2) + c;
        w[c] = (uint32_t)(orc_splitmix64_mix(seed + (k + 1u) * 0x9e3779b97f4a7c15ull) >> 32);
    }
}

/* floor(w * n / 2^32): a uniform integer in [0, n) from one 32-bit word. */
uint32_t orc_range(uint32_t w, uint32_t n)
{
    return (uint32_t)(((uint64_t)w * (uint64_t)n) >> 32);
}

/* ---------------------------------------------------------------------------------------
 * Market description and state.
 * ------------------------------------------------------------------------------------- */
typedef struct {
    uint32_t L;       /* ticks on the price grid, 1..1024                                   */
    uint32_t A;       /* agents                                                             */
    uint32_t K;       /* noise offsets are uniform on {-K..K}                               */
    uint32_t Q;       /* quantities are uniform on {1..Q}                                   */
    uint32_t n_noise; /* agents [0, n_noise) are NOISE                                      */
    uint32_t n_mom;   /* agents [n_noise, n_noise + n_mom) are MOMENTUM, the rest MAKER     */
    uint32_t h;       /* maker half-spread in ticks                                         */
    uint32_t flags;   /* bits 0-7: agent model (ORC_MODEL_*); bits 8-15: generator (ORC_GEN_*);
                         bits 16-31: the probability P_mkt of a marketable order in units of
                         2^-16 (mid-price model only) */
} orc_market;

enum { ORC_MODEL_LAST = 0, ORC_MODEL_MID = 1 };
enum { ORC_GEN_PHILOX = 0, ORC_GEN_SPLITMIX = 1 };

/* The four words of agent a of market m at absolute step s, from the descriptor's generator. */
static void orc_agent_words(const orc_market *d, uint32_t m, uint64_t seed, uint32_t a, uint32_t s,
                            uint32_t w[4])
{
    if (((d->flags >> 8) & 0xFFu) == ORC_GEN_SPLITMIX) {
        orc_splitmix_words((uint64_t)m * d->A + a, s, seed, w);
    } else {
        uint32_t ctr[4] = {s, a, m, 0u};
        uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
        orc_philox4x32_10(ctr, key, w);
    }
}

typedef struct {
    uint32_t last;        /* last clearing tick (agents' reference price)                  */
    uint32_t prev;        /* reference price before the last step                          */
    uint64_t steps_done;  /* absolute step counter                                         */
    uint64_t n_trade;     /* steps with volume > 0                                         */
    uint64_t sum_vol;     /* sum of executed volume                                        */
    uint64_t sum_px;      /* sum of clearing ticks over trading steps                      */
    uint64_t sum_spread;  /* sum of (best ask - best bid) over steps where both exist      */
    uint64_t n_spread;    /* number of such steps                                          */
    double sum_r;         /* sum of log returns ln(L+last) - ln(L+prev)                    */
    double sum_r2;        /* sum of their squares                                          */
    uint32_t ref2;        /* twice the reference price the agents used in the latest step  */
    uint32_t reserved;    /* 0                                                             */
} orc_state;

enum { ORC_BUY = 0, ORC_SELL = 1 };

void orc_initial_state(const orc_market *d, orc_state *st)
{
    memset(st, 0, sizeof(*st));
    st->last = d->L / 2;
    st->prev = d->L / 2;
    st->ref2 = 2u * (d->L / 2);
}

static uint32_t clamp_tick(int64_t t, uint32_t L)
{
    if (t < 0) return 0;
    if (t > (int64_t)L - 1) return L - 1;
    return (uint32_t)t;
}

/* The order of agent a of market m at absolute step s (section III-C, agent classes;
 * quantity rule of "Order Quantity and RNG").  Counter (s, a, m, 0), key = seed words. */
void orc_agent_order(const orc_market *d, uint32_t m, uint64_t seed, uint32_t a, uint32_t s,
                     uint32_t last, uint32_t prev, uint32_t *side, uint32_t *tick, uint32_t *qty)
{
    uint32_t w[4];
    orc_agent_words(d, m, seed, a, s, w);

    uint32_t coin = (w[0] < 0x80000000u) ? ORC_BUY : ORC_SELL;
    int64_t ref = (int64_t)last;
    uint32_t sd;
    int64_t t;
    if (a < d->n_noise) {
        /* NOISE: fair coin for the side, tick = last + uniform offset in {-K..K}. */
        int64_t off = (int64_t)orc_range(w[1], 2u * d->K + 1u) - (int64_t)d->K;
        sd = coin;
        t = ref + off;
    } else if (a < d->n_noise + d->n_mom) {
        /* MOMENTUM: side = sign of the last price change, coin when unchanged;
         * tick one step beyond the reference in the direction of the side. */
        if (last > prev) sd = ORC_BUY;
        else if (last < prev) sd = ORC_SELL;
        else sd = coin;
        t = (sd == ORC_BUY) ? ref + 1 : ref - 1;
    } else {
        /* MAKER: buys when (a + s) is even, sells otherwise; posts h ticks away. */
        sd = (((uint64_t)a + (uint64_t)s) % 2u == 0u) ? ORC_BUY : ORC_SELL;
        t = (sd == ORC_BUY) ? ref - (int64_t)d->h : ref + (int64_t)d->h;
    }
    *side = sd;
    *tick = clamp_tick(t, d->L);
    *qty = 1u + orc_range(w[2], d->Q);
}

/* The paper's own agent rules (section III-C, "State Retrieval" and "Agent Strategy Classes"):
 * the reference is the mid-price of the resting book, mid = (bb + ba) / 2 when both sides are
 * quoted, else the last clearing price; round(x) is floor(x + 1/2).  mid and mid_prev are
 * half-integers, passed as doubles.
 *   NOISE: fair coin for the side; price round(mid + eta) with eta = K (2u - 1), u = w1 / 2^32,
 *          so eta is uniform on [-K, K).  With probability P_mkt (u3 = w3 / 2^32 < P_mkt) the
 *          order is marketable: price L-1 for a buy, 0 for a sell.
 *   MOMENTUM: side = sign(mid - mid_prev), the coin when the mid did not move; price
 *          round(mid + 1) for a buy, round(mid - 1) for a sell; marketable like NOISE.
 *   MAKER: buys when (a + s) is even; price round(mid - h) for a bid, round(mid + h) for an
 *          ask; never marketable.
 * Every price is then clamped to the grid.  Quantities as in the last-tick model.  All the
 * doubles involved are exact: K and h are below 2^10 and u has 32 significant bits. */
void orc_agent_order_mid(const orc_market *d, uint32_t m, uint64_t seed, uint32_t a, uint32_t s,
                         double mid, double mid_prev, uint32_t *side, uint32_t *tick, uint32_t *qty)
{
    uint32_t w[4];
    orc_agent_words(d, m, seed, a, s, w);

    const double two32 = 4294967296.0;
    uint32_t coin = (w[0] < 0x80000000u) ? ORC_BUY : ORC_SELL;
    double p_mkt = (double)(d->flags >> 16) / 65536.0;
    int marketable = ((double)w[3] / two32) < p_mkt;
    uint32_t sd;
    double price;
    if (a < d->n_noise) {
        double eta = (double)d->K * (2.0 * ((double)w[1] / two32) - 1.0);
        sd = coin;
        price = floor(mid + eta + 0.5);
    } else if (a < d->n_noise + d->n_mom) {
        if (mid > mid_prev) sd = ORC_BUY;
        else if (mid < mid_prev) sd = ORC_SELL;
        else sd = coin;
        price = floor(mid + (sd == ORC_BUY ? 1.0 : -1.0) + 0.5);
    } else {
        sd = (((uint64_t)a + (uint64_t)s) % 2u == 0u) ? ORC_BUY : ORC_SELL;
        price = floor(mid + (sd == ORC_BUY ? -(double)d->h : (double)d->h) + 0.5);
        marketable = 0;
    }
    if (marketable) price = (sd == ORC_BUY) ? (double)d->L - 1.0 : 0.0;
    *side = sd;
    *tick = clamp_tick((int64_t)price, d->L);
    *qty = 1u + orc_range(w[2], d->Q);
}

/* ---------------------------------------------------------------------------------------
 * Uniform-price clearing of one book (Eq. 1, Eq. 2, price-priority allocation).
 * Sums are formed in 64 bits so nothing here depends on the books' overflow guard.
 * On return bid/ask hold the residual book, *pstar the lowest tick of maximal volume
 * (0 when every volume is 0) and *vstar the executed volume.
 * ------------------------------------------------------------------------------------- */
void orc_clear(uint32_t L, uint32_t *bid, uint32_t *ask, uint32_t *pstar, uint64_t *vstar)
{
    uint64_t *D = (uint64_t *)malloc(sizeof(uint64_t) * L);
    uint64_t *S = (uint64_t *)malloc(sizeof(uint64_t) * L);
    uint64_t run = 0;
    for (int64_t p = (int64_t)L - 1; p >= 0; --p) { run += bid[p]; D[p] = run; }
    run = 0;
    for (uint32_t p = 0; p < L; ++p) { run += ask[p]; S[p] = run; }

    uint64_t best = 0;
    uint32_t best_p = 0;
    for (uint32_t p = 0; p < L; ++p) {
        uint64_t v = D[p] < S[p] ? D[p] : S[p];
        if (v > best) { best = v; best_p = p; } /* strict: the first maximiser is kept */
    }

    if (best > 0) {
        uint64_t rem = best; /* bids: highest limit first */
        for (int64_t p = (int64_t)L - 1; p >= 0; --p) {
            uint64_t f = bid[p] < rem ? bid[p] : rem;
            bid[p] -= (uint32_t)f;
            rem -= f;
        }
        rem = best; /* asks: lowest limit first */
        for (uint32_t p = 0; p < L; ++p) {
            uint64_t f = ask[p] < rem ? ask[p] : rem;
            ask[p] -= (uint32_t)f;
            rem -= f;
        }
    }
    free(D);
    free(S);
    *pstar = best_p;
    *vstar = best;
}

/* ln(L + t) for t in [0, L): prices are L + tick so that every log is finite. */
static void build_log_prices(uint32_t L, double *lnp)
{
    for (uint32_t t = 0; t < L; ++t) lnp[t] = log((double)L + (double)t);
}

/* Statistics of one finished step (see orc_state).  The state's last/prev are updated
 * here: prev takes the old last; last takes p* only if something traded. */
void orc_update_stats(uint32_t L, const uint32_t *bid, const uint32_t *ask, uint32_t pstar,
                      uint64_t vstar, const double *lnp, orc_state *st)
{
    uint32_t old_last = st->last;
    st->prev = old_last;
    if (vstar > 0) {
        st->last = pstar;
        st->n_trade += 1;
        st->sum_vol += vstar;
        st->sum_px += pstar;
    }
    int64_t bb = -1, ba = -1;
    for (int64_t p = (int64_t)L - 1; p >= 0; --p)
        if (bid[p] > 0) { bb = p; break; }
    for (uint32_t p = 0; p < L; ++p)
        if (ask[p] > 0) { ba = p; break; }
    if (bb >= 0 && ba >= 0) {
        st->sum_spread += (uint64_t)(ba - bb);
        st->n_spread += 1;
    }
    double r = lnp[st->last] - lnp[st->prev];
    double r2 = r * r;
    st->sum_r = st->sum_r + r;
    st->sum_r2 = st->sum_r2 + r2;
    st->steps_done += 1;
}

/* One full step of one market: every agent's order into the book, clearing, statistics.
 * agent_order (may be NULL) gives the order in which agents are visited. */
void orc_market_step(const orc_market *d, uint32_t m, uint64_t seed, orc_state *st,
                     uint32_t *bid, uint32_t *ask, const double *lnp,
                     const uint32_t *agent_order)
{
    uint32_t s = (uint32_t)st->steps_done;
    uint32_t model = d->flags & 0xFFu;
    double mid = (double)st->last, mid_prev = 0.5 * (double)st->ref2;
    if (model == ORC_MODEL_MID) {
        /* state retrieval on the resting book: best bid, best ask, mid-price */
        int64_t bb = -1, ba = -1;
        for (int64_t p = (int64_t)d->L - 1; p >= 0; --p)
            if (bid[p] > 0) { bb = p; break; }
        for (uint32_t p = 0; p < d->L; ++p)
            if (ask[p] > 0) { ba = p; break; }
        if (bb >= 0 && ba >= 0) mid = 0.5 * (double)(bb + ba);
    }
    for (uint32_t i = 0; i < d->A; ++i) {
        uint32_t a = agent_order ? agent_order[i] : i;
        uint32_t side, tick, qty;
        if (model == ORC_MODEL_MID)
            orc_agent_order_mid(d, m, seed, a, s, mid, mid_prev, &side, &tick, &qty);
        else
            orc_agent_order(d, m, seed, a, s, st->last, st->prev, &side, &tick, &qty);
        if (side == ORC_BUY) bid[tick] += qty;
        else ask[tick] += qty;
    }
    uint32_t pstar;
    uint64_t vstar;
    orc_clear(d->L, bid, ask, &pstar, &vstar);
    orc_update_stats(d->L, bid, ask, pstar, vstar, lnp, st);
    st->ref2 = (uint32_t)(2.0 * mid);  /* the reference of this step (the last price, or the mid) */
}

/* S steps of one market (book = bid[L] followed by ask[L]).  When tr_price / tr_vol are not
 * NULL they receive, for every step i of this call, the reference (last clearing) tick after the
 * step and the volume V* executed in it: the per-step price and volume series that the paper's
 * market-dynamics experiments read (section IV-J). */
int orc_market_run_traced(const orc_market *d, uint32_t m, uint64_t seed, uint32_t S, orc_state *st,
                          uint32_t *book, const uint32_t *agent_order, uint32_t *tr_price,
                          uint64_t *tr_vol)
{
    if (d->L < 1 || d->L > 1024) return -1;
    if ((d->flags & 0xFFu) > ORC_MODEL_MID) return -1;
    if ((d->flags & 0xFFu) == ORC_MODEL_LAST && (d->flags >> 16) != 0) return -1;
    if (((d->flags >> 8) & 0xFFu) > ORC_GEN_SPLITMIX) return -1;
    /* Books are 32-bit: every quantity ever added must fit. */
    if (((uint64_t)st->steps_done + S) * (uint64_t)d->A * (uint64_t)d->Q >= (1ull << 32)) return -2;
    double *lnp = (double *)malloc(sizeof(double) * d->L);
    build_log_prices(d->L, lnp);
    for (uint32_t i = 0; i < S; ++i) {
        uint64_t vol_before = st->sum_vol;
        orc_market_step(d, m, seed, st, book, book + d->L, lnp, agent_order);
        if (tr_price) tr_price[i] = st->last;
        if (tr_vol) tr_vol[i] = st->sum_vol - vol_before;
    }
    free(lnp);
    return 0;
}

int orc_market_run(const orc_market *d, uint32_t m, uint64_t seed, uint32_t S, orc_state *st,
                   uint32_t *book, const uint32_t *agent_order)
{
    return orc_market_run_traced(d, m, seed, S, st, book, agent_order, NULL, NULL);
}

/* ---------------------------------------------------------------------------------------
 * Many markets, split over host threads (markets are independent).
 * descs[i] describes market ids[i]; its book is at book + book_off[i] (words).
 * ------------------------------------------------------------------------------------- */
typedef struct {
    const orc_market *descs;
    const uint32_t *ids;
    const uint64_t *book_off;
    uint32_t *book;
    orc_state *states;
    uint64_t seed;
    uint32_t S;
    uint32_t n;
    uint32_t *tr_price; /* optional traces, row i at i * tr_ld */
    uint64_t *tr_vol;
    uint64_t tr_ld;
    uint32_t next; /* guarded by lock */
    int status;
    pthread_mutex_t lock;
} orc_job;

static void *orc_worker(void *arg)
{
    orc_job *job = (orc_job *)arg;
    for (;;) {
        pthread_mutex_lock(&job->lock);
        uint32_t i = job->next++;
        pthread_mutex_unlock(&job->lock);
        if (i >= job->n) break;
        int rc = orc_market_run_traced(&job->descs[i], job->ids[i], job->seed, job->S, &job->states[i],
                                       job->book + job->book_off[i], NULL,
                                       job->tr_price ? job->tr_price + (size_t)i * job->tr_ld : NULL,
                                       job->tr_vol ? job->tr_vol + (size_t)i * job->tr_ld : NULL);
        if (rc != 0) {
            pthread_mutex_lock(&job->lock);
            job->status = rc;
            pthread_mutex_unlock(&job->lock);
        }
    }
    return NULL;
}

int orc_run_traced(const orc_market *descs, const uint32_t *ids, const uint64_t *book_off, uint32_t n,
                   uint64_t seed, uint32_t S, orc_state *states, uint32_t *book, int nthreads,
                   uint32_t *tr_price, uint64_t *tr_vol, uint64_t tr_ld)
{
    orc_job job;
    job.descs = descs; job.ids = ids; job.book_off = book_off; job.book = book;
    job.states = states; job.seed = seed; job.S = S; job.n = n; job.next = 0; job.status = 0;
    job.tr_price = tr_price; job.tr_vol = tr_vol; job.tr_ld = tr_ld;
    pthread_mutex_init(&job.lock, NULL);
    if (nthreads < 1) nthreads = 1;
    if ((uint32_t)nthreads > n) nthreads = (int)(n ? n : 1);
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
    for (int t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, orc_worker, &job);
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    free(th);
    pthread_mutex_destroy(&job.lock);
    return job.status;
}

int orc_run(const orc_market *descs, const uint32_t *ids, const uint64_t *book_off, uint32_t n,
            uint64_t seed, uint32_t S, orc_state *states, uint32_t *book, int nthreads)
{
    return orc_run_traced(descs, ids, book_off, n, seed, S, states, book, nthreads, NULL, NULL, 0);
}

/* Clearing of many independent books of one size (used by the exhaustive pins). */
void orc_clear_batch(uint32_t L, uint32_t n, uint32_t *books, uint32_t *pstar, uint64_t *vstar)
{
    for (uint32_t i = 0; i < n; ++i)
        orc_clear(L, books + (size_t)i * 2 * L, books + (size_t)i * 2 * L + L, &pstar[i], &vstar[i]);
}

/* Raw Philox words for a batch of counters (pins and distribution checks). */
void orc_philox_batch(uint32_t n, const uint32_t *ctrs, const uint32_t key[2], uint32_t *out)
{
    for (uint32_t i = 0; i < n; ++i) orc_philox4x32_10(ctrs + 4 * (size_t)i, key, out + 4 * (size_t)i);
}

/* Orders of agents [0, A) of one market at one step (order-mapping checks). */
void orc_orders(const orc_market *d, uint32_t m, uint64_t seed, uint32_t s, uint32_t last,
                uint32_t prev, uint32_t *side, uint32_t *tick, uint32_t *qty)
{
    for (uint32_t a = 0; a < d->A; ++a)
        orc_agent_order(d, m, seed, a, s, last, prev, &side[a], &tick[a], &qty[a]);
}

/* Mid-price-model orders of agents [0, A) at one step, given mid and the previous mid as
 * half-tick integers (2 mid, 2 mid_prev). */
void orc_orders_mid(const orc_market *d, uint32_t m, uint64_t seed, uint32_t s, uint32_t mid2,
                    uint32_t mid2_prev, uint32_t *side, uint32_t *tick, uint32_t *qty)
{
    for (uint32_t a = 0; a < d->A; ++a)
        orc_agent_order_mid(d, m, seed, a, s, 0.5 * (double)mid2, 0.5 * (double)mid2_prev,
                            &side[a], &tick[a], &qty[a]);
}

/* Generator words of a batch: SplitMix64 for (gid, s) pairs (pins). */
void orc_splitmix_batch(uint32_t n, const uint64_t *gid, const uint32_t *steps, uint64_t seed, uint32_t *out)
{
    for (uint32_t i = 0; i < n; ++i) orc_splitmix_words(gid[i], steps[i], seed, out + 4 * (size_t)i);
}

uint32_t orc_state_size(void) { return (uint32_t)sizeof(orc_state); }
uint32_t orc_market_size(void) { return (uint32_t)sizeof(orc_market); }
