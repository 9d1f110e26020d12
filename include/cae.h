/*
 * cae.h -- C ABI of libcae: a call-auction ensemble engine for AMD Instinct MI355X (gfx950).
 *
 * The engine steps many independent limit-order books through repeated uniform-price call
 * auctions (KineticSim paper, section II-A, Eq. 1 and Eq. 2): every agent posts an order,
 * the orders are aggregated per tick, cumulative demand D(p) = sum_{q>=p} BUY[q] and supply
 * S(p) = sum_{q<=p} SELL[q] are formed, the market clears at the lowest tick maximising
 * min(D, S), fills go by price priority and the residual book carries to the next step.
 * All S steps of a call run in one persistent kernel launch with the books resident in LDS
 * (section III, Algorithm 1); HBM is touched only when a call starts and ends.
 *
 * Conventions for every function below:
 *   - the return value is CAE_OK (0) or a negative CAE_E* code; cae_last_error() then
 *     holds a message for the calling thread;
 *   - "device" pointers are HIP device memory owned by the caller (for example the data
 *     pointers of torch tensors); the library never allocates or frees device memory;
 *   - "host" pointers are ordinary host memory owned by the caller;
 *   - a stream is a hipStream_t passed as void* (NULL = the default stream); work is
 *     ordered on it and the calls marked "asynchronous" return before it completes;
 *   - an ensemble handle must not be used from two host threads or two streams at once.
 *
 * Orders (section III-C, readings of this library):
 *   agent a of market m at absolute step s draws w = Philox4x32-10(counter (s, a, m, 0),
 *   key (seed mod 2^32, seed / 2^32)) (Salmon et al., SC'11; the paper's counter-based
 *   generator of section III-G).  With ref = the last clearing tick:
 *     NOISE    (a < n_noise):          side BUY iff w0 < 2^31; tick = ref + floor(w1*(2K+1)/2^32) - K
 *     MOMENTUM (a < n_noise + n_mom):  side = sign(last - prev) (BUY up, SELL down, w0 rule if 0);
 *                                      tick = ref + 1 for BUY, ref - 1 for SELL
 *     MAKER    (the rest):             BUY iff (a + s) is even; tick = ref - h (BUY) or ref + h (SELL)
 *   every tick is clamped to [0, L-1]; quantity = 1 + floor(w2 * Q / 2^32).
 * That is the last-tick model (CAE_MODEL_LAST).  The mid-price model (CAE_MODEL_MID) follows
 * the paper's own rules (section III-C, "State Retrieval", "Agent Strategy Classes"): at the
 * start of each step the reference is mid = (bb + ba) / 2 of the resting book when both sides
 * are quoted, else the last clearing tick; round(x) = floor(x + 1/2); u_i = w_i / 2^32:
 *     NOISE:    side BUY iff w0 < 2^31; tick = round(mid + K (2 u1 - 1)), eta uniform on [-K, K)
 *     MOMENTUM: side = sign(mid - mid of the previous step) (w0 rule if 0); tick = round(mid +- 1)
 *     MAKER:    BUY iff (a + s) is even; tick = round(mid - h) (BUY) or round(mid + h) (SELL)
 *   and a NOISE or MOMENTUM order is marketable when u3 < P_mkt: tick L-1 for a BUY, 0 for a
 *   SELL.  Ticks are clamped and quantities drawn as above.
 * Clearing: the combined book (resting + new) clears at p*, the lowest tick of maximal
 * V(p) = min(D(p), S(p)); bids fill from the highest tick down and asks from the lowest tick
 * up until V* shares each.  If V* = 0 nothing trades and the price is unchanged.
 * Statistics per step: prev <- last; if V* > 0 then last <- p*, n_trade += 1,
 * sum_vol += V*, sum_px += p*; if the residual book has both a best bid bb and a best ask ba,
 * sum_spread += ba - bb and n_spread += 1; r = ln(L + last) - ln(L + prev), sum_r += r,
 * sum_r2 += r * r (double, no fused multiply-add).  The opening book is empty and
 * last = prev = floor(L / 2).
 */
#ifndef CAE_H
#define CAE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Return codes. */
#define CAE_OK 0
#define CAE_EINVAL (-1)    /* bad argument or descriptor; nothing was launched             */
#define CAE_EOVERFLOW (-2) /* the call could overflow a 32-bit book; nothing was launched   */
#define CAE_ENOSPACE (-3)  /* a caller buffer is smaller than required                      */
#define CAE_EHIP (-4)      /* the HIP runtime reported an error (message has its text)      */
#define CAE_ESTATE (-5)    /* the handle is not in a state that allows the call             */

/* Agent models (bits 0-7 of cae_market.flags), the generator (bits 8-15) and the
 * marketable-order probability P_mkt of the mid-price model (bits 16-31, in units of 2^-16: an
 * order is marketable iff w3 < (flags >> 16) << 16).
 * CAE_GEN_SPLITMIX selects the paper's SplitMix64 (section III-G; Steele, Lea and Flood,
 * OOPSLA 2014) instead of Philox: word c (0..3) of agent a of market m at step s is the high
 * half of mix(seed + (k + 1) 0x9e3779b97f4a7c15) with k = (m A + a) 2^34 + 4 s + c, where mix is
 * the output function printed in section III-G (the paper leaves the coordinate hash open;
 * this reads it as a position in the seeded stream). */
#define CAE_MODEL_LAST 0u
#define CAE_MODEL_MID 1u
#define CAE_MODEL_MASK 0xFFu
#define CAE_GEN_PHILOX 0u
#define CAE_GEN_SPLITMIX 1u
#define CAE_GEN_SHIFT 8
#define CAE_PMKT_SHIFT 16

/* One market (32 bytes).  Constraints checked by cae_sizes and cae_create:
 *   1 <= L <= 1024, A >= 1, K <= 2^30 (K < 2^20 in the mid-price model), Q >= 1,
 *   A * Q < 2^32, n_noise + n_mom <= A, maker_half_spread < L; flags: model LAST or MID,
 *   generator PHILOX or SPLITMIX, P_mkt zero in the last-tick model. */
typedef struct cae_market {
    uint32_t L;                 /* ticks on the price grid                                */
    uint32_t A;                 /* agents                                                 */
    uint32_t K;                 /* noise offsets are uniform on {-K..K}                   */
    uint32_t Q;                 /* quantities are uniform on {1..Q}                       */
    uint32_t n_noise;           /* agents [0, n_noise) are NOISE                          */
    uint32_t n_mom;             /* agents [n_noise, n_noise + n_mom) MOMENTUM; rest MAKER */
    uint32_t maker_half_spread; /* h, in ticks                                            */
    uint32_t flags;             /* agent model and P_mkt (CAE_MODEL_*, CAE_PMKT_SHIFT)    */
} cae_market;

/* Per-market state and statistics (80 bytes, this exact layout in device memory). */
typedef struct cae_state {
    uint32_t last;       /* last clearing tick                                 */
    uint32_t prev;       /* reference before the last step                     */
    uint64_t steps_done; /* absolute step counter (the generator's counter)     */
    uint64_t n_trade;
    uint64_t sum_vol;
    uint64_t sum_px;
    uint64_t sum_spread;
    uint64_t n_spread;
    double sum_r;
    double sum_r2;
    uint32_t ref2;       /* twice the reference price of the latest step (the last tick, or
                            the mid-price), the mid-price model's momentum memory; opening
                            value 2 floor(L / 2) */
    uint32_t reserved;   /* 0                                                  */
} cae_state;

/* Device memory an ensemble needs (from cae_sizes). */
typedef struct cae_sizes_t {
    uint64_t book_words;      /* uint32 words of the packed books: sum over markets of 2*L */
    uint64_t book_bytes;      /* 4 * book_words                                             */
    uint64_t state_bytes;     /* M * sizeof(cae_state)                                      */
    uint64_t workspace_bytes; /* library-private workspace (descriptors, schedule, tables)  */
} cae_sizes_t;

/* Caller-owned device buffers, each at least the size cae_sizes reports, 256-byte aligned.
 * book:  market m occupies words [2*o_m, 2*o_m + 2*L_m), o_m = sum_{j<m} L_j; bid[0..L)
 *        then ask[0..L), uint32 per tick (structure of arrays per market).
 * state: M cae_state records in market order.
 * workspace: opaque; must not be modified while the ensemble exists. */
typedef struct cae_buffers {
    uint32_t *book;
    cae_state *state;
    void *workspace;
} cae_buffers;

/* Schedule of the persistent launch.  Zero fields mean "choose automatically"; an
 * autotuner result can be passed back in.  waves_per_market[c] applies to size class c
 * (class = index of the smallest of 64,128,256,512,1024 that is >= L, times 8, plus the
 * A bucket floor(log2(A)) clamped to 6..13 minus 6): 40 classes. */
#define CAE_NUM_CLASSES 40
typedef struct cae_tuning {
    uint32_t waves_per_group;                   /* waves per workgroup (1..16)           */
    uint32_t groups_per_cu;                     /* resident workgroups per CU to launch   */
    uint32_t max_lds_bytes;                     /* LDS budget per workgroup               */
    uint32_t flags;                             /* bit 0: keep descriptor order (no LPT);
                                                   bit 1: in an ensemble whose work items
                                                   differ in cost per step, the waves of the
                                                   items within a quarter of the costliest
                                                   (lock-step or single-wave markets) issue
                                                   one priority level above the others'     */
    uint8_t waves_per_market[CAE_NUM_CLASSES];  /* 1,2,4,8,16 per size class; 0 = auto    */
    uint8_t pipelined[CAE_NUM_CLASSES];         /* 1: markets of this class run in pairs
                                                   that share all waves_per_group waves in
                                                   alternating phases (one wave clears one
                                                   market while the others generate the
                                                   other's orders); waves_per_market is then
                                                   ignored.  Needs waves_per_group >= 2.   */
    uint8_t overlap[CAE_NUM_CLASSES];           /* k >= 1: lock-step markets of this class
                                                   generate the next step's orders while the
                                                   current step clears, the clearing wave
                                                   taking k - 1 rows of 64 agents after its
                                                   clearing; 0 = off.  Applies to classes of
                                                   2 or more waves per market, not pipelined
                                                   (ignored and reported as 0 elsewhere);
                                                   markets with K above 1022 (510 for the
                                                   mid-price model) run plain lock-step.    */
    float class_cost[CAE_NUM_CLASSES];          /* relative cost of one market-step per
                                                   class for the longest-first order;
                                                   0 = the built-in model A + 2*64*TPL    */
    uint8_t pack[CAE_NUM_CLASSES];              /* P = 2 or 4: P small markets of this class
                                                   share one wave, 64/P lanes each, for the
                                                   orders (rows of 64/P agents) and for the
                                                   clearing (one book per lane segment);
                                                   0 = off.  Applies to last-tick Philox
                                                   markets with L <= 512/P (up to 8 ticks
                                                   per lane of a segment) in ensembles whose
                                                   books all have at most 128 ticks (others
                                                   of the class run unpacked); the class runs
                                                   one wave per P markets (waves_per_market,
                                                   pipelined and overlap are ignored).     */
} cae_tuning;

typedef struct cae_ensemble cae_ensemble;

/* Text for a return code.  Never NULL. */
const char *cae_strerror(int code);

/* Message of the last failing call on this host thread ("" if none).  Never NULL. */
const char *cae_last_error(void);

/* Library and device information: number of compute units of the current device and the
 * library version.  Either pointer may be NULL. */
int cae_device_info(uint32_t *num_cu, uint32_t *version);

/* Sizes of the device buffers for M markets described by host array desc[M] (the inputs of
 * Algorithm 1, "REQUIRE": M markets, each with its A agents and L price ticks; the books of
 * section III-B, here bid[L] and ask[L] per market).  Pure host computation; nothing is
 * allocated.  CAE_EINVAL on a bad descriptor (the message names the market). */
int cae_sizes(const cae_market *desc, uint32_t M, cae_sizes_t *out);

/* Create an ensemble of M markets (Algorithm 1, "REQUIRE": M markets with their A agents
 * and L ticks).  The paper seeds opening quotes (Algorithm 1, section III-B) without stating
 * them; this library's reading is an empty opening book with last = prev = floor(L / 2).
 * Copies the descriptors and schedule into dev->workspace, zeroes dev->book and writes the
 * opening state to dev->state, ordered on `stream`; returns after those copies completed.
 * market_ids (host, M entries, may be NULL = 0..M-1) is the market index each market uses in
 * the generator counter, so a subset of a larger ensemble (a shard, or one size group)
 * reproduces that ensemble's markets bit for bit.  tuning may be NULL (automatic schedule).
 * *out receives a host handle that owns only host memory.
 * Errors: CAE_EINVAL (descriptor, M == 0, NULL pointer, bad tuning), CAE_EHIP. */
int cae_create(const cae_market *desc, uint32_t M, uint64_t seed, const uint32_t *market_ids,
               const cae_buffers *dev, void *stream, const cae_tuning *tuning,
               cae_ensemble **out);

/* Advance every market by S steps in one persistent launch on the ensemble's stream
 * (Algorithm 1: the S-step loop runs on the device; section III-E phases 2-5 each step).
 * Asynchronous.  Fails with CAE_EOVERFLOW, launching nothing, if for some market
 * (steps_done + S) * A * Q >= 2^32 (a 32-bit book could then overflow).  S == 0 is a
 * no-op.  Errors: CAE_EINVAL, CAE_EOVERFLOW, CAE_EHIP. */
int cae_step(cae_ensemble *e, uint32_t S);

/* cae_step that also records each market's per-step price and volume series, the raw data of
 * the paper's market-dynamics experiments (section IV-J: volatility, return kurtosis, volume
 * and return autocorrelations against the agent mix).  For market m (descriptor order) and
 * step i of this call (0 <= i < S):
 *   dev_price[m * ld + i]  = the reference tick `last` after step i (unchanged when nothing
 *                            traded), in [0, L);
 *   dev_volume[m * ld + i] = the volume V* executed in step i (0: no trade).
 * Both are caller-owned device arrays of at least M * ld words; either may be NULL (then that
 * series is not written).  ld >= S, so successive calls can fill columns of one larger array.
 * Same schedule, results and errors as cae_step, plus CAE_EINVAL when ld < S. */
int cae_step_traced(cae_ensemble *e, uint32_t S, uint32_t *dev_price, uint32_t *dev_volume,
                    uint64_t ld);

/* Copy the packed books (layout of cae_buffers.book) to host_book[n_words] after the
 * stream's pending work; returns when the copy is complete.  These are the final books that
 * Algorithm 1 leaves in global memory ("ENSURE": the final limit-order books).
 * CAE_ENOSPACE if n_words is smaller than book_words; CAE_EINVAL on NULL; CAE_EHIP. */
int cae_read_books(cae_ensemble *e, uint32_t *host_book, uint64_t n_words);

/* Copy the M states (price, step counter and clearing statistics: Algorithm 1, "ENSURE": the
 * clearing statistics in global memory) to host_state[M]; synchronous like cae_read_books.
 * CAE_ENOSPACE if M is smaller than the ensemble's; CAE_EINVAL on NULL; CAE_EHIP. */
int cae_read_state(cae_ensemble *e, cae_state *host_state, uint32_t M);

/* Replace the device books and states with host copies (checkpoint resume: the books and
 * statistics one call leaves, Algorithm 1 "ENSURE", become the starting state of the next
 * call).  host_book must hold book_words words in the packed layout.  Synchronous.
 * CAE_EINVAL, writing nothing, if M or n_words do not match the ensemble, or a state is
 * inconsistent with its market: last or prev >= L, ref2 > 2 (L - 1), reserved != 0,
 * steps_done A Q >= 2^32, or a book holding more than steps_done A Q shares on its two sides
 * together (more than steps_done steps can add; cae_step's overflow guard relies on that
 * bound).  CAE_EHIP. */
int cae_write_state(cae_ensemble *e, const cae_state *host_state, uint32_t M,
                    const uint32_t *host_book, uint64_t n_words);

/* The schedule in use (as chosen at create).  */
int cae_get_tuning(const cae_ensemble *e, cae_tuning *out);

/* The same S steps as cae_step, computed by the naive engine of the paper's ablation
 * (section IV-I, "Naive Custom CUDA"): one GPU thread per market, the book read and written in
 * global memory at every step, clearing by serial loops over the L ticks.  Bit-identical results
 * to cae_step (the same order rules and statistics); for comparison only.  Asynchronous; same
 * errors as cae_step. */
int cae_step_naive(cae_ensemble *e, uint32_t S);

/* Duration in milliseconds of the last cae_step or cae_step_naive launch, from HIP events
 * recorded on the ensemble's stream around the kernel; waits for that launch to finish. */
int cae_last_step_ms(cae_ensemble *e, float *ms);

/* Release the host handle made by cae_create (host metadata only).  The device buffers, which
 * hold the ensemble's books and statistics (Algorithm 1, "ENSURE"), stay owned by the caller
 * and keep their contents.  NULL is accepted.  Always CAE_OK. */
int cae_destroy(cae_ensemble *e);

/* One clearing pass over M books of L ticks each (Eq. 1, Eq. 2 and price-priority fill;
 * the worked example of section IV-C is one such book).  dev_book holds M books in the
 * packed layout (bid[L] then ask[L] per book) and is updated in place to the residual
 * books; dev_pstar[M] receives the lowest tick of maximal volume (0 when nothing can trade)
 * and dev_vstar[M] the executed volume.  Every per-book total must be below 2^32.
 * Asynchronous on `stream`.  Errors: CAE_EINVAL (L outside 1..1024, NULL), CAE_EHIP. */
int cae_clear(uint32_t L, uint32_t M, uint32_t *dev_book, uint32_t *dev_pstar,
              uint32_t *dev_vstar, void *stream);

/* ----------------------------------------------------------------------------------------
 * Calibration surrogate: a multilayer perceptron d_in -> H -> H -> d_out with SiLU hidden
 * activations, trained and evaluated on the GPU by bfloat16 matrix-core kernels with fp32
 * accumulation.  It is not part of the paper's method: it maps agent-population parameters to
 * ensemble statistics for the parameter sweeps the paper motivates (section IV-J), with the
 * exact engine above as its fallback and the reference that measures its error.
 *
 * Parameter layout (fp32, row-major, input index first), P = cae_mlp_sizes().n_params floats:
 *   W1[d_in][H], b1[H], W2[H][H], b2[H], W3[H][d_out], b3[d_out]
 * bfloat16 weight copies (n_weights halfwords): W1, W2, W3 in the same layouts, back to back,
 * then W2 transposed (W2T[n][k] = W2[k][n], H * H halfwords) for cae_mlp_predict.
 * bfloat16 (round to nearest even) is stored for the inputs, weights, hidden activations and
 * back-propagated gradients; products are accumulated in fp32; biases, pre-activations,
 * outputs, weight gradients and Adam moments are fp32.
 * Constraints: 1 <= d_in <= 64, H a multiple of 16 in 16..1024, 1 <= d_out <= 16.
 * ------------------------------------------------------------------------------------- */
typedef struct cae_mlp {
    uint32_t d_in, d_hidden, d_out, flags; /* flags: 0                                       */
    float *params;                         /* device, caller-owned fp32 parameters           */
    uint16_t *weights;                     /* device, caller-owned bfloat16 weight copies    */
} cae_mlp;

typedef struct cae_mlp_sizes_t {
    uint64_t n_params;        /* fp32 parameters                                            */
    uint64_t n_weights;       /* bfloat16 weight copies                                     */
    uint64_t workspace_bytes; /* per cae_mlp_forward/backward call with N <= max_batch      */
} cae_mlp_sizes_t;

/* Sizes for a network of the given shape and batches of at most max_batch samples.  Host only. */
int cae_mlp_sizes(uint32_t d_in, uint32_t d_hidden, uint32_t d_out, uint32_t max_batch, cae_mlp_sizes_t *out);

/* Rewrite the bfloat16 weight copies from net->params (after initialising or loading the
 * parameters).  Asynchronous on stream. */
int cae_mlp_refresh_weights(const cae_mlp *net, void *stream);

/* y[N][d_out] (fp32, device) = network(x[N][d_in] (fp32, device)).  ws (device, workspace_bytes
 * for a batch >= N) receives the activations that cae_mlp_backward reuses.  Asynchronous. */
int cae_mlp_forward(const cae_mlp *net, const float *x, float *y, uint32_t N, void *ws, void *stream);

/* Inference only: y[N][d_out] = network(x[N][d_in]) in one fused launch (all three layers per
 * tile of 32 samples, activations kept on chip), with no workspace and no limit on N.  The
 * outputs are bit-identical to cae_mlp_forward's (same matrix-core tiles, summation order and
 * bfloat16 rounding points); nothing is kept for cae_mlp_backward.  Requires d_hidden <= 496.
 * Asynchronous.  Errors: CAE_EINVAL (shape, NULL), CAE_EHIP. */
int cae_mlp_predict(const cae_mlp *net, const float *x, float *y, uint32_t N, void *stream);

/* Gradient of sum_{n,k} dy[n][k] * y[n][k] with respect to every parameter, summed over the N
 * samples, written to grads (device, n_params fp32 in the parameter layout).  ws must hold the
 * activations of the preceding cae_mlp_forward on the same N inputs (x itself is not read).
 * N >= 1.  Asynchronous. */
int cae_mlp_backward(const cae_mlp *net, const float *x, const float *dy, float *grads, uint32_t N, void *ws,
                     void *stream);

/* One Adam step (Kingma and Ba 2015, algorithm 1; step counts from 1) on net->params with the
 * fp32 moments m, v (device, n_params each, zero before step 1); refreshes the bfloat16 weight
 * copies.  Asynchronous. */
int cae_mlp_adam(const cae_mlp *net, const float *grads, float *m, float *v, uint32_t step, float lr, float beta1,
                 float beta2, float eps, void *stream);

/* One training step fused into two launches: forward pass on the batch, the mean loss over its
 * N d_out outputs (kind and delta as in cae_mlp_loss_grad) and its gradient, back-propagation,
 * and an Adam step (as cae_mlp_adam) that also refreshes the bfloat16 weight copies.  Same
 * rounding points and fp32 accumulation as cae_mlp_forward + cae_mlp_loss_grad +
 * cae_mlp_backward + cae_mlp_adam; each weight gradient is reduced over the whole batch by one
 * wave in a fixed order (deterministic; the sums run in another order than the unfused path's).
 * x[n][d_in] and target[n][d_out] (fp32, device) hold all samples; idx (device, N entries, may be
 * NULL = rows 0..N-1) lists the rows of this batch.  m, v: Adam moments (device, n_params fp32).
 * loss (device): receives the batch's mean loss.  grads (device, n_params fp32, may be NULL):
 * receives the gradient.  ws: workspace of cae_mlp_sizes with max_batch >= N.
 * Requires d_hidden a multiple of 32 up to 256 and d_in <= 32.  Asynchronous.
 * Errors: CAE_EINVAL (shape, NULL, N == 0, step == 0, loss kind, delta), CAE_EHIP. */
int cae_mlp_train_step(const cae_mlp *net, const float *x, const float *target, const uint32_t *idx, uint32_t N,
                       float *m, float *v, uint32_t step, float lr, float beta1, float beta2, float eps, int loss_kind,
                       float delta, float *loss, float *grads, void *ws, void *stream);

/* cae_mlp_train_step without a workspace argument, for callers that cannot allocate device
 * memory (code under HIP graph capture, serving loops, harnesses that forbid allocation).  The
 * workspace is a static array of 8 MiB (8 << 20 bytes) inside the library, one copy per device,
 * held until the process ends; its address is looked up once per device on the first call made
 * with that device current.  Allocates nothing (no hipMalloc, no hipFree) and computes exactly
 * what cae_mlp_train_step computes (same kernels, same results bit for bit).  Batches whose
 * workspace (about 2 (d_in + 4 H + 16) bytes per sample, N rounded up to 32) exceeds the array
 * are refused with CAE_EINVAL before anything is launched: at d_in = 4, H = 256 that is N above
 * 4000.  Every call on one device shares that device's array, so calls that overlap on one
 * device (two streams, or two host threads) race and must be ordered by the caller; calls that
 * are ordered on one stream are safe.  Asynchronous.
 * Errors: those of cae_mlp_train_step, CAE_EINVAL for a batch beyond the array, CAE_EHIP. */
int cae_mlp_train_step_noalloc(const cae_mlp *net, const float *x, const float *target, const uint32_t *idx,
                               uint32_t N, float *m, float *v, uint32_t step, float lr, float beta1, float beta2,
                               float eps, int loss_kind, float delta, float *loss, float *grads, void *stream);

/* Mean loss over n values and its gradient with respect to y, r = y - target (device pointers;
 * one workgroup, fixed summation order).  Asynchronous.
 *   CAE_LOSS_MSE:   loss[0] = mean r^2, dy = 2 r / n
 *   CAE_LOSS_HUBER: loss[0] = mean of (r^2 / 2 if |r| <= delta else delta (|r| - delta / 2)),
 *                   dy = clamp(r, -delta, delta) / n   (delta > 0)
 * Errors: CAE_EINVAL (NULL, n == 0, unknown kind, delta <= 0 for Huber), CAE_EHIP. */
#define CAE_LOSS_MSE 0
#define CAE_LOSS_HUBER 1
int cae_mlp_loss_grad(const float *y, const float *target, float *dy, float *loss, uint32_t n, int kind, float delta,
                      void *stream);

#ifdef __cplusplus
}
#endif

#endif /* CAE_H */
