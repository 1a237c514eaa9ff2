/*
 * ppo.h -- C ABI of the MI355X (gfx950) learning hot path of massively
 * parallel PPO (Rudin, Hoeller, Reist and Hutter, "Learning to Walk in
 * Minutes Using Massively Parallel Deep Reinforcement Learning", CoRL 2021).
 *
 * The paper keeps the whole on-policy loop on one GPU (Section 2: data
 * collection and policy update both on the device; Section 2.2: a custom PPO
 * that stores every tensor on the GPU).  This library implements the learner
 * half of that loop as hand-written HIP kernels:
 *   - ppo_assemble_obs  : observations from proprioception, a height scan
 *                         around the base and uniform noise (Section 3.2,
 *                         Table 4), in front of inference;
 *   - ppo_rollout_infer : actor-critic inference for every environment plus
 *                         diagonal-Gaussian action sampling (Philox4x32-10);
 *   - ppo_gae           : GAE over a [T, N] rollout with time-out
 *                         bootstrapping (Sections 2.2.1 and 2.2.2) and the
 *                         batch advantage statistics;
 *   - ppo_update_epoch  : one PPO epoch of K mini-batch steps (clipped
 *                         surrogate, value loss, entropy bonus, global
 *                         gradient-norm clip, Adam) (Section 2.2.1,
 *                         Appendix A.4 Table 3).
 *
 * Conventions shared by every entry point
 *   - Return value: PPO_OK (0) or a negative PPO_E_* code.  On error,
 *     ppo_last_error() returns a thread-local message.  No C++ exception
 *     crosses this boundary.
 *   - All arguments are validated on the host BEFORE anything is enqueued;
 *     a call that returns an error has enqueued nothing.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Every call is asynchronous on that stream and never synchronises the
 *     host, except ppo_ctx_create/destroy, first-use autotuning (below) and
 *     ppo_update_epoch_profiled.
 *   - Ownership: the caller allocates and owns all device memory (rollout
 *     buffers, parameters, optimiser state, statistics, workspace) and keeps
 *     it alive until the enqueued work has completed.  The library never
 *     allocates device memory; a context owns host-side state only (network
 *     shape, precision, tile choices, cached HIP graphs).
 *   - Pointers to device memory must be 16-byte aligned; arrays are dense
 *     (no strides) in the layouts given below.
 *   - Sample index s = t * N + n over a rollout (time-major, environment
 *     contiguous).
 *   - Autotuning: the first call for a given row count (N for inference, M
 *     for the update) times the GEMM tile candidates of every launch site
 *     with HIP events on the caller's stream and waits for them (the only
 *     host synchronisation outside ctx create/destroy); the choice is cached
 *     in the context, and in the file named by the environment variable
 *     PPO_TUNE_CACHE if set.  PPO_AUTOTUNE=0 keeps 128 x 128 tiles.
 *     PPO_GEMM_GRID_CAP=0 launches one workgroup per GEMM tile (by default
 *     128 x 128-tile launches are persistent: as many workgroups as fit on
 *     the device at once, each taking every G-th tile).
 *   - bf16 update steps of networks whose hidden widths split evenly over
 *     the waves of a workgroup (e.g. [512, 256, 128], [64, 64] or
 *     [1024, 512, 256]; input width a multiple of 16) run everything that is
 *     independent per sample (gather, hidden layers, output layers with the
 *     loss, input-gradient chain) as one fused launch with the activations in
 *     LDS, then the split-sample weight-gradient GEMMs; other shapes, and the
 *     fp32 path, run the layer-by-layer kernels.  The results agree to
 *     float32 rounding (bf16 ulps downstream of it).  Where it fits, the
 *     fused pass runs three 64-sample workgroups per CU with the first hidden
 *     layer computed in 128-feature chunks, each added into the second
 *     layer's accumulators at once (e.g. [512, 256, 128] with 48 or 235
 *     inputs; with 235 the loss inputs load after the first two layers).
 *     PPO_FUSED=0 forces the layer-by-layer kernels; PPO_FUSED_ROWS=32 or 64
 *     (and PPO_FUSED_THREADS=256 or 512, PPO_FUSED_PER_CU=2 or 3) override
 *     the fused pass's block shape.
 *   - bf16 precision: GEMM operands are bf16 with float32 accumulation,
 *     except that the critic's hidden-layer weights enter its forward GEMMs
 *     as two bf16 terms, bf16(W) and bf16(W - bf16(W)) (about 16 significant
 *     bits): a common rounding of the weights would shift every sample's
 *     value the same way, and the value loss's gradient is a mean of
 *     (V - R) that such a shift biases directly.  Output layers, biases,
 *     log-std, log-probabilities (float32 with compensated summation) and the
 *     loss are float32; the advantage statistics and the gradient norm's sum
 *     of squares are float64.
 */
#ifndef PPO_MI355X_PPO_H
#define PPO_MI355X_PPO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define PPO_OK             0
#define PPO_E_INVAL       -1  /* NULL or misaligned pointer, bad enum value   */
#define PPO_E_SHAPE       -2  /* dimension out of range or inconsistent       */
#define PPO_E_UNSUPPORTED -3  /* device is not gfx950 / precision not built   */
#define PPO_E_HIP         -4  /* HIP runtime, launch or graph error           */
#define PPO_E_NOMEM       -5  /* caller's workspace smaller than required     */

/* ---- precision of the GEMM operands ------------------------------------ */
#define PPO_FP32 0  /* all arithmetic in float32 (the plain path)              */
#define PPO_BF16 1  /* bf16 GEMM operands, float32 accumulation; float32
                       master weights, Adam state, heads, log-prob and loss    */

/* ---- limits ------------------------------------------------------------- */
#define PPO_MAX_HIDDEN   4      /* hidden layers per network                 */
#define PPO_MAX_WIDTH    2048   /* hidden width (multiple of 16)             */
#define PPO_MAX_OBS      4096   /* observation dimension                     */
#define PPO_MAX_ACT      16     /* action dimension                          */
#define PPO_MAX_T        4096   /* rollout horizon                           */
#define PPO_STATS_WIDTH  10     /* floats per mini-batch statistics row      */
#define PPO_MAX_RUNS     64     /* runs in one batched update                */

/* Statistics row written per mini-batch step (floats):
 *   [0] total loss L = L_pi + c_v L_V - c_e H
 *   [1] policy loss L_pi      [2] value loss L_V      [3] entropy H
 *   [4] clip fraction (|rho - 1| > clip)
 *   [5] approximate KL, mean((rho - 1) - log rho)
 *   [6] global gradient norm before clipping (accumulated in float64)
 *   [7] flags: bit 0 = non-finite gradient norm (the Adam step was skipped)
 *   [8] KL(pi_old || pi_new) of the diagonal Gaussians, mean over the
 *       mini-batch at the step's parameters (0 when batch.mu_old is NULL)
 *   [9] learning rate the step used (after the KL adaptation, if enabled;
 *       0 when no learning rate is given)
 */

/* Network shape.  Actor: obs_dim -> hidden[0] -> ... -> act_dim; critic:
 * obs_dim -> hidden[0] -> ... -> 1.  ELU (alpha = 1) on hidden layers,
 * linear outputs, a state-independent log standard deviation per action.
 * The paper fixes none of this (Sections 2.2 and 3.2 name a policy and a
 * critic only); these are the project's workload definitions. */
typedef struct ppo_net_desc {
    int32_t obs_dim;                  /* D, 1..PPO_MAX_OBS                   */
    int32_t act_dim;                  /* A, 1..PPO_MAX_ACT                   */
    int32_t n_hidden;                 /* L, 1..PPO_MAX_HIDDEN                */
    int32_t hidden[PPO_MAX_HIDDEN];   /* widths, multiples of 16, <= 2048    */
} ppo_net_desc;

/* Flat parameter vector (float32, P entries): actor W1, b1, ..., W_{L+1},
 * b_{L+1}, actor log-std [A], then critic W1, b1, ..., W_{L+1}, b_{L+1}.
 * Every W is row-major [out, in]. */
typedef struct ppo_params {
    float    *theta;   /* [P] float32 master weights                          */
    float    *grad;    /* [P] raw (pre-clip) gradient of the latest step      */
    float    *adam_m;  /* [P] Adam first moment                               */
    float    *adam_v;  /* [P] Adam second moment                              */
    uint16_t *shadow;  /* [P] bf16 copy of theta (round to nearest even);
                          required for PPO_BF16, ignored for PPO_FP32         */
    int32_t  *step;    /* device scalar: Adam steps taken so far              */
    float    *lr;      /* device scalar: learning rate                        */
} ppo_params;

/* One rollout batch flattened over samples (B = T * N). */
typedef struct ppo_batch {
    const float *obs;      /* [B, D]                                          */
    const float *actions;  /* [B, A]                                          */
    const float *logp;     /* [B] log-probabilities at collection time        */
    const float *adv;      /* [B] normalised advantages                       */
    const float *returns;  /* [B] returns R = A + V (un-normalised A)         */
    const float *values;   /* [B] values at collection (value clipping only;
                              may be NULL when clip_value == 0)               */
    const float *mu_old;   /* [B, A] action means at collection (the mu output
                              of ppo_rollout_infer); NULL unless the KL is
                              wanted (required when desired_kl > 0)           */
    const float *logstd_old; /* [A] log-std at collection; with mu_old      */
    int32_t B;
} ppo_batch;

/* Update hyper-parameters (Appendix A.4 Table 3 gives clip 0.2, entropy
 * coefficient 0.01, 5 epochs; the rest are the project's settings). */
typedef struct ppo_hparams {
    float   clip;           /* surrogate (and value) clip range, > 0          */
    float   value_coef;     /* c_v >= 0                                       */
    float   entropy_coef;   /* c_e >= 0                                       */
    float   max_grad_norm;  /* > 0                                            */
    float   beta1, beta2;   /* Adam, in [0, 1)                                */
    float   adam_eps;       /* > 0, added outside the square root             */
    int32_t clip_value;     /* 0/1: clipped value loss (needs batch.values)   */
    int32_t use_graph;      /* 0/1: capture the epoch into a HIP graph and
                               replay it (cached per pointer/shape set)       */
    /* KL-adaptive learning rate (App. A.4, Algorithm 1).  With desired_kl > 0
     * each mini-batch step first measures KL(pi_old || pi_new) over its rows
     * at the current parameters, then sets, on the device,
     *   lr = max(lr_min, lr / lr_factor)  if KL > 2 desired_kl,
     *   lr = min(lr_max, lr * lr_factor)  if KL < desired_kl / 2,
     * and takes its Adam step with that rate (written back to params.lr, so a
     * replayed graph continues from it).  0 keeps params.lr unchanged. */
    float   desired_kl;     /* >= 0 (Table 3: 0.01)                           */
    float   lr_factor;      /* >= 1 (Algorithm 1: 1.5)                        */
    float   lr_min, lr_max; /* 0 < lr_min <= lr_max (Algorithm 1: 1e-5, 1e-2) */
} ppo_hparams;

typedef struct ppo_ctx ppo_ctx;

/* Thread-local message of the last error on this thread ("" if none). */
const char *ppo_last_error(void);

/* Creates a context for one network shape and precision.  Checks the shape
 * (PPO_E_SHAPE) and precision (PPO_E_INVAL).  Does not touch the GPU. */
int ppo_ctx_create(const ppo_net_desc *net, int32_t precision, ppo_ctx **out);

/* Destroys the context and its cached graphs.  Synchronises nothing; the
 * caller must have completed work that used the context's graphs. */
int ppo_ctx_destroy(ppo_ctx *ctx);

/* Number of float32 parameters P of the flat vector. */
int ppo_param_count(const ppo_net_desc *net, int64_t *count);

/* Offsets of every tensor in the flat vector, in the order given above:
 * 2 (L + 1) actor entries, 1 log-std entry, 2 (L + 1) critic entries.
 * `capacity` is the length of `offsets`; PPO_E_SHAPE if it is too small. */
int ppo_param_offsets(const ppo_net_desc *net, int64_t *offsets, int32_t capacity);

/* Context options (ppo_ctx_set_option).
 * PPO_OPT_KEEP_PACKED (0 or 1, default 0): bf16 inference keeps the forward
 *   weights it packs into a workspace and reuses them on the next
 *   ppo_rollout_infer with the same workspace and shadow, instead of packing
 *   again on every call.  They are packed again when this library has written
 *   the shadow since (ppo_pack_weights, ppo_update_epoch,
 *   ppo_update_epoch_profiled, ppo_update_batched), when another call used an
 *   overlapping workspace, and always for calls captured into a graph (a
 *   shadow written under capture is never trusted again).  With the option
 *   set, the caller promises that a workspace passed to ppo_rollout_infer
 *   stays allocated and is written only by this library's calls, and that
 *   the shadow is written only by them or followed by ppo_pack_weights. */
#define PPO_OPT_KEEP_PACKED 1
int ppo_ctx_set_option(ppo_ctx *ctx, int32_t option, int32_t value);

/* Bytes of device workspace the calls below need for N environments per
 * rollout step, T steps and mini-batch size M.  One workspace of this size
 * serves ppo_rollout_infer (N rows), ppo_gae (T x N) and
 * ppo_update_epoch / ppo_loss_grad (M rows). */
int ppo_workspace_size(const ppo_ctx *ctx, int32_t N, int32_t T, int32_t M, size_t *bytes);

/* Rounds theta to bf16 (round to nearest even) into `shadow` [P].  Needed
 * once after theta is written by anything other than ppo_update_epoch. */
int ppo_pack_weights(const ppo_ctx *ctx, void *stream, const float *theta, uint16_t *shadow);

/* Policy inference for one rollout step (Section 2: policy inference for
 * every robot on the GPU).  obs [N, D] float32.  Writes, when non-NULL:
 * actions [N, A] = mu + sigma * eps, logp [N] (log-density of the action),
 * values [N] (critic), mu [N, A].  eps is drawn from Philox4x32-10 with key
 * (seed mod 2^32, seed >> 32) and counter (n * ceil(A/4) + g, t, iteration,
 * 1) for action group g; uniforms ((x >> 9) + 1/2) 2^-23; Box-Muller pairs.
 * With actions == NULL only the critic runs (value-only mode, e.g. for the
 * bootstrap values of the observation after the last step); values must be
 * non-NULL.  `ws` must hold ppo_workspace_size(ctx, N, *, *) bytes.
 * bf16 networks run from forward weights packed into `ws` at every call,
 * unless the context has PPO_OPT_KEEP_PACKED set (see ppo_ctx_set_option). */
int ppo_rollout_infer(const ppo_ctx *ctx, void *stream, const ppo_params *p,
                      const float *obs, int32_t N, int32_t t, uint64_t seed,
                      uint32_t iteration, float *actions, float *logp,
                      float *values, float *mu, void *ws, size_t ws_bytes);

/* GAE over a [T, N] rollout (Section 2.2.1; time-out bootstrap of Section
 * 2.2.2 read as r'_t = r_t + gamma V_t timeout_t).  rewards, values [T, N]
 * float32; dones, timeouts [T, N] uint8 (timeouts may be NULL; a time-out
 * must also be a done); last_values [N].  Writes returns [T, N] = A + V,
 * adv_stats[2] = (mean, unbiased std) of A in float64, and adv [T, N]: the
 * raw advantages, or (A - mean) / (std + 1e-8) when normalize != 0.
 * T in 1..PPO_MAX_T, T * N >= 2. */
int ppo_gae(const ppo_ctx *ctx, void *stream, const float *rewards, const uint8_t *dones,
            const uint8_t *timeouts, const float *values, const float *last_values,
            int32_t T, int32_t N, float gamma, float lam, float *adv, float *returns,
            double *adv_stats, int32_t normalize, void *ws, size_t ws_bytes);

/* Allocation-free variant of ppo_gae, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops, harnesses that
 * forbid allocation): the same computation and results bit for bit, with no
 * workspace argument.  The per-block statistics partials it needs (24 bytes
 * per 256 environments) live in a fixed device array of the library, one per
 * GPU, held until the process ends; N must not exceed PPO_GAE_NOALLOC_MAX_N
 * (PPO_E_SHAPE otherwise, before anything is enqueued).  The first call on a
 * device looks up that device's copy of the array (with the device current)
 * and synchronises nothing.  No call allocates or frees anything.  Every call
 * on one GPU uses the same array and every partial is written before it is
 * read, so nothing needs clearing; calls that overlap in time on one GPU (on
 * different streams) race and must be serialised by the caller. */
#define PPO_GAE_NOALLOC_MAX_N (1 << 21)
int ppo_gae_noalloc(const ppo_ctx *ctx, void *stream, const float *rewards, const uint8_t *dones,
                    const uint8_t *timeouts, const float *values, const float *last_values,
                    int32_t T, int32_t N, float gamma, float lam, float *adv, float *returns,
                    double *adv_stats, int32_t normalize);

/* One PPO epoch: for k in 0..K-1 the mini-batch perm[k M : (k+1) M]
 * (M = B / K) goes through forward, loss, hand-written backward, global
 * norm clip and Adam (step count and lr read from p->step / p->lr; step is
 * advanced by K).  perm [B] int32 is a permutation of [0, B) chosen by the
 * caller.  stats [K, PPO_STATS_WIDTH] float32.  p->grad holds the raw
 * gradient of the last step afterwards.  B % K must be 0. */
int ppo_update_epoch(ppo_ctx *ctx, void *stream, const ppo_params *p, const ppo_batch *b,
                     const int32_t *perm, int32_t n_minibatches, const ppo_hparams *hp,
                     float *stats, void *ws, size_t ws_bytes);

/* One epoch of R independent PPO runs of uneven size in the same launches
 * (sweep-style training of several policies at once, each with its own
 * network shape, data, permutation, optimiser state and workspace).  Runs
 * must share the precision, the number of hidden layers and n_minibatches;
 * observation widths, hidden widths and batch sizes may differ.  When every
 * run takes the fused pass (bf16, widths it covers), each run's whole epoch
 * runs on one of four side streams forked from `stream` and joined back to
 * it, runs placed largest first on the least-loaded stream, so the runs
 * proceed independently and the small ones fill the workgroup slots the
 * large ones leave free.  Otherwise (or with PPO_BATCHED_GROUPED=1),
 * mini-batch step k of every run goes through one grouped launch per GEMM
 * site (all runs' actor and critic problems in one grid) with per-run
 * gather, loss, gradient-reduce and Adam kernels in between.  With
 * hp->use_graph the whole batched epoch is one cached HIP graph.  The first call for a set of run
 * shapes times the tile candidates of every grouped site (see autotuning
 * above) and gives the weight-gradient workgroups of all runs one common
 * k-length.  With PPO_AUTOTUNE=0 every site uses 128 x 128 tiles and each
 * run keeps the weight-gradient split count it would use alone, so every
 * run's result equals its own ppo_update_epoch bit for bit.  Arrays have R
 * entries; ws_bytes[i] must cover ppo_workspace_size(ctxs[i], 0, 0,
 * B_i / n_minibatches). */
int ppo_update_batched(ppo_ctx *const *ctxs, int32_t R, void *stream, const ppo_params *params,
                       const ppo_batch *batches, const int32_t *const *perms, int32_t n_minibatches,
                       const ppo_hparams *hp, float *const *stats, void *const *ws,
                       const size_t *ws_bytes);

/* Loss and gradient of one mini-batch (rows idx[0..M)) without an optimiser
 * step: writes stats[PPO_STATS_WIDTH] (entry 6 = gradient norm, entry 7 =
 * flags) and grad_out [P] (the raw gradient).  grad_out == NULL computes the
 * loss terms only (no backward pass; stats entry 6 is then 0).  Optional
 * per-row outputs for
 * checkers (NULL = not written): ratio_out [M] float32 (4-byte aligned), the
 * probability ratio rho = pi(a|s) / pi_old(a|s) this call computed, and
 * active_out [M] uint8, 1 if the sample's clipped surrogate passes gradient
 * (A >= 0 and rho <= 1 + clip, or A < 0 and rho >= 1 - clip: the PPO
 * objective of Section 2.2 on the closed band) and 0 otherwise.  A sample
 * whose ratio lies within rounding of a clip edge may legitimately take
 * either branch; a checker adopts this call's branch exactly where the
 * exported ratio and its own lie on different sides of the edge.  Used by
 * the autograd wrapper and gradient checks. */
int ppo_loss_grad(const ppo_ctx *ctx, void *stream, const ppo_params *p, const ppo_batch *b,
                  const int32_t *idx, int32_t M, const ppo_hparams *hp, float *stats,
                  float *grad_out, uint8_t *active_out, float *ratio_out, void *ws,
                  size_t ws_bytes);

/* Kernel phases of one mini-batch step, in launch order. */
#define PPO_PHASE_GATHER       0  /* mini-batch rows of obs -> GEMM operand     */
#define PPO_PHASE_FORWARD      1  /* hidden-layer GEMMs + bias + ELU (L launches) */
#define PPO_PHASE_HEAD_LOSS    2  /* output layers, PPO loss, output gradients  */
#define PPO_PHASE_INPUT_GRAD   3  /* dz W times ELU' GEMMs (L - 1 launches)     */
#define PPO_PHASE_WEIGHT_GRAD  4  /* split-sample weight-gradient GEMMs         */
#define PPO_PHASE_GRAD_REDUCE  5  /* split sums, flat gradient, float64 norm^2  */
#define PPO_PHASE_ADAM         6  /* clip coefficient + Adam + bf16 shadow      */
#define PPO_PHASE_FUSED        7  /* bf16: gather, forward, loss and input
                                     gradients of both networks in one launch
                                     (replaces phases 0-3 except the weight
                                     staging, which stays in phase 0)         */
#define PPO_N_PHASES           8

/* Same computation as ppo_update_epoch, launched eagerly with a HIP event
 * pair recorded on `stream` around every kernel launch.  Launches that only
 * read what earlier launches wrote (all but Adam, and the gradient reduction
 * when the rate adapts) are enqueued `reps` (1..1000) times back to back
 * inside their event pair, which leaves the results unchanged and spreads
 * the event overhead; phase_ms then reports one repetition.  Synchronises
 * the stream before returning, then writes phase_ms[PPO_N_PHASES] (summed
 * event-measured milliseconds per phase over the epoch) and
 * phase_launches[PPO_N_PHASES] (launch counts of one repetition).  For
 * measurement only. */
int ppo_update_epoch_profiled(ppo_ctx *ctx, void *stream, const ppo_params *p, const ppo_batch *b,
                              const int32_t *perm, int32_t n_minibatches, const ppo_hparams *hp,
                              float *stats, void *ws, size_t ws_bytes, int32_t reps, float *phase_ms,
                              int32_t *phase_launches);

/* Verification: one launch of the library's GEMM kernel on caller data.
 * C[M, N] = A[M, K] B[N, K]^T with float32 accumulation; operands are float32
 * (PPO_FP32) or bf16 bit patterns (PPO_BF16).  a_mode / b_mode: 0 = row-major
 * [rows, K], 1 = stored transposed [K, rows].  Supported combinations:
 *   (0, 0, epilogue 0): C = ELU(acc + bias[n])              (C in operand type)
 *   (0, 1, epilogue 1): C = acc * ELU'(z), with h = ELU(z) read from H[M, ldh]
 *   (1, 1, epilogue 2): C[s, M, ldc] float32 partial sums over `splits` slices
 *                       of K, rowsum[s, M] = per-slice row sums of A.
 * The number of slices actually used is ceil(K / kps), kps = ceil(K / splits)
 * rounded up to the kernel's k-slab.  tile: output tile per workgroup,
 * 0 = 128 x 128, 1 = 64 x 128, 2 = 128 x 64, 3 = 64 x 64 (rows x columns). */
int ppo_gemm_check(void *stream, int32_t precision, int32_t a_mode, int32_t b_mode, int32_t epilogue,
                   int32_t M, int32_t N, int32_t K, const void *A, int32_t lda, const void *B,
                   int32_t ldb, void *C, int32_t ldc, const float *bias, const void *H, int32_t ldh,
                   float *rowsum, int32_t splits, int32_t tile);

/* Tile choices recorded for `rows` GEMM rows (update != 0: the update's
 * sites, else inference).  choices[2 s] = tile shape (as in
 * ppo_gemm_check), choices[2 s + 1] = weight-gradient splits in half rounds
 * of resident workgroups (1, 2 or 4; 2 elsewhere), for sites
 * s = 0..3 forward layer s, 4..7 input gradient of layer s - 4, 8 weight
 * gradients.  capacity >= 18.  PPO_E_SHAPE if nothing was tuned yet. */
int ppo_ctx_tuning(const ppo_ctx *ctx, int32_t rows, int32_t update, int32_t *choices, int32_t capacity);

/* Block shape of the fused per-sample pass that bf16 update steps of this
 * network take: *rows samples per workgroup of *threads threads (both 0 when
 * the layer-by-layer kernels run: fp32, PPO_FUSED=0, or a network shape the
 * fused kernel does not cover).  Reflects PPO_FUSED, PPO_FUSED_ROWS and
 * PPO_FUSED_THREADS as set now; a step also falls back for batches of more
 * than 2^31 bytes of observations or misaligned biases.  Host only. */
int ppo_fused_shape(const ppo_ctx *ctx, int32_t *rows, int32_t *threads);

/* The same for bf16 inference (ppo_rollout_infer): without PPO_FUSED_ROWS /
 * PPO_FUSED_THREADS it prefers 32 rows x 256 threads (two workgroups per
 * CU): a policy step over a few thousand environments is latency-bound, and
 * more, shorter workgroups finish it sooner.  Host only. */
int ppo_fused_infer_shape(const ppo_ctx *ctx, int32_t *rows, int32_t *threads);

/* Terrain seen by the height scan: a height field on a uniform grid and the
 * scan pattern.  Cell (i, j) of `height` [nx, ny] (row-major, float32) is the
 * terrain height at world (i / inv_res, j / inv_res); `scan` [n_scan, 2] holds
 * the body-frame (x, y) offsets of the scan points in metres (17 x 11 points at
 * 0.1 m in the rough-terrain workloads; the paper's robot uses 108).  The
 * library only reads these. */
typedef struct ppo_terrain {
    const float *height;
    int32_t nx, ny;       /* 1..2^24 each                                     */
    float inv_res;        /* cells per metre, positive and finite             */
    const float *scan;
    int32_t n_scan;       /* S >= 0                                           */
} ppo_terrain;

/* Observation assembly in front of ppo_rollout_infer (Section 3.2: what the
 * policy observes; appendix Table 4: observation noise).  Writes obs [N, D],
 * D = n_proprio + S (must equal the network's obs_dim):
 *   obs[n, j]     = proprio[n, j]                              for j < n_proprio,
 *   obs[n, P + k] = base_z - height[cell nearest to scan point k],
 * plus noise_scale[j] * (2u - 1) on every element when noise_scale [D] is
 * non-NULL (uniform on (-scale, scale)).  base [N, 5] = (x, y, z, cos yaw,
 * sin yaw) of each robot; scan point k lands at world
 * (x + (c px - s py), y + (s px + c py)), every product and sum rounded to
 * float32 on its own, and reads cell (rint(wx inv_res), rint(wy inv_res))
 * (round half to even) clamped to the grid; a NaN position reads cell 0.
 * u comes from Philox4x32-10 with key (seed mod 2^32, seed >> 32) and counter
 * (n * ceil(D/4) + g, t, iteration, 2) for column j = 4 g + i (draw i), mapped
 * as in ppo_rollout_infer; tag 2 keeps it apart from the action noise (tag 1).
 * terrain may be NULL when S = 0; proprio may be NULL when n_proprio = 0;
 * base may be NULL when S = 0.  N <= 2^24 and N * ceil(D/4) < 2^31.  Asynchronous on
 * `stream`; the caller owns every buffer. */
int ppo_assemble_obs(const ppo_ctx *ctx, void *stream, const float *proprio, int32_t n_proprio,
                     const float *base, const ppo_terrain *terrain, const float *noise_scale,
                     int32_t N, int32_t t, uint64_t seed, uint32_t iteration, float *obs);

/* Debug/verification: raw Philox4x32-10 blocks.  out[4 i + w] = word w of
 * Philox(counter = (c0_base + i mod 2^32, c1, c2, c3), key = (seed mod 2^32,
 * seed >> 32)) for i in [0, n).  n in 1..2^28. */
int ppo_philox_blocks(void *stream, uint64_t seed, uint32_t c0_base, uint32_t c1, uint32_t c2,
                      uint32_t c3, int64_t n, uint32_t *out);

#ifdef __cplusplus
}
#endif

#endif /* PPO_MI355X_PPO_H */
