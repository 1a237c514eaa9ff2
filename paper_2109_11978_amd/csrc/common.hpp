// Internal declarations shared by the HIP kernels and the host runtime of the
// PPO learner library.  Nothing here is part of the public ABI (include/ppo.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ppo {

constexpr int kMaxHidden = 4;
constexpr int kMaxLayers = kMaxHidden + 1;
constexpr int kStatsWidth = 10;
constexpr int kHeadPad = 16;        // output-layer gradient rows padded to 16 columns
constexpr int kGemmMaxProblems = 16;

enum Precision { kFP32 = 0, kBF16 = 1 };

// ---------------------------------------------------------------- bf16 ----
__host__ __device__ inline float bf16_to_f32(uint16_t h) {
    union { uint32_t u; float f; } v;
    v.u = static_cast<uint32_t>(h) << 16;
    return v.f;
}

// Round to nearest, ties to even; NaN stays NaN (quiet bit set).
__host__ __device__ inline uint16_t f32_to_bf16(float f) {
    union { uint32_t u; float f; } v;
    v.f = f;
    if ((v.u & 0x7F800000u) == 0x7F800000u && (v.u & 0x007FFFFFu))
        return static_cast<uint16_t>((v.u >> 16) | 0x0040u);
    uint32_t lsb = (v.u >> 16) & 1u;
    return static_cast<uint16_t>((v.u + 0x7FFFu + lsb) >> 16);
}

// Log-density of a diagonal Gaussian in float32 with compensated summation.
// s carries the sum, c the rounding errors of its additions (Neumaier's
// variant of Kahan summation) plus the exact errors of the squares (from a
// fused multiply-add) and the float32 residual of ln(2 pi) / 2, so the
// result is within a few float32 ulps of the exact sum of the float32
// inputs.  Contraction is off: each product and sum is rounded on its own,
// as the error terms assume.
constexpr float kHalfLog2PiHi = 0.918938517570495605f;
constexpr float kHalfLog2PiLo = static_cast<float>(0.91893853320467274178 - static_cast<double>(kHalfLog2PiHi));
struct CompSum {
    float s = 0.0f, c = 0.0f;
    __device__ inline void add(float x) {
#pragma clang fp contract(off)
        const float t = s + x;
        c += fabsf(s) >= fabsf(x) ? (s - t) + x : (x - t) + s;
        s = t;
    }
    // one dimension of a diagonal-Gaussian log-density: -z^2 / 2 - log sigma - ln(2 pi) / 2
    __device__ inline void add_gauss(float z, float logstd) {
#pragma clang fp contract(off)
        const float p = z * z;
        const float e = __builtin_fmaf(z, z, -p);   // p + e = z^2 exactly
        add(-0.5f * p);
        add(-logstd);
        add(-kHalfLog2PiHi);
        c += -0.5f * e - kHalfLog2PiLo;
    }
    __device__ inline float value() const { return s + c; }
};

template <typename T> struct Elem;
template <> struct Elem<float> {
    __device__ static inline float load(const float *p, long long i) { return p[i]; }
    __device__ static inline float to_f(float x) { return x; }
    __device__ static inline float from_f(float x) { return x; }
};
template <> struct Elem<uint16_t> {
    __device__ static inline float load(const uint16_t *p, long long i) { return bf16_to_f32(p[i]); }
    __device__ static inline float to_f(uint16_t x) { return bf16_to_f32(x); }
    __device__ static inline uint16_t from_f(float x) { return f32_to_bf16(x); }
};

// -------------------------------------------------------------- GEMMs -----
// C[M, N] = A[M, K] * B[N, K]^T (float32 accumulation) with a fused epilogue.
// Operand modes: 0 = row-major [rows, K] (K contiguous);
//                1 = stored transposed, [K, rows] (rows contiguous).
enum GemmEpilogue {
    kEpiBiasElu = 0,   // C(T) = ELU(acc + bias[n])
    kEpiDElu = 1,      // C(T) = acc * ELU'(z), with ELU'(z) recovered from h = ELU(z) in H
    kEpiPartial = 2,   // C(float) partial sums of split s at C + s * c_split_stride;
                       // rowsum[s * M + m] = sum_k A[m, k] over the split (bias gradient)
};

struct GemmProblem {
    const void *A;
    const void *B;
    // Optional second B operand of the same layout (bf16 only): the launch
    // then computes A (B + B2)^T, running the k-range once with B and once with
    // B2 into the same accumulators.  The critic's forward layers pass the
    // bf16 residual theta - bf16(theta) here, so their weights carry about 16
    // significant bits.
    const void *B2;
    void *C;
    const float *bias;
    const void *H;
    float *rowsum;
    long long c_split_stride;
    int M, N, K;
    int lda, ldb, ldc, ldh;
    int tiles_m, tiles_n, splits, kps;
    int tile_begin;
};

// Output tile shapes (rows x columns per workgroup of 4 wave64s).
enum GemmTileShape { kTile128x128 = 0, kTile64x128 = 1, kTile128x64 = 2, kTile64x64 = 3, kNumTileShapes = 4 };
inline int tile_rows(int t) { return (t == kTile64x128 || t == kTile64x64) ? 64 : 128; }
inline int tile_cols(int t) { return (t == kTile128x64 || t == kTile64x64) ? 64 : 128; }

struct GemmArgs {
    GemmProblem p[kGemmMaxProblems];
    int count;
    int total_tiles;
    int tile;    // GemmTileShape shared by every problem of the launch
};

// k-slab depth per operand type (shared with the host planner).
template <typename T> struct GemmTile;
template <> struct GemmTile<uint16_t> { static constexpr int BK = 64; };
template <> struct GemmTile<float> { static constexpr int BK = 32; };

hipError_t launch_gemm(Precision prec, int a_mode, int b_mode, int epi, const GemmArgs &args,
                       hipStream_t stream);

// ------------------------------------------------ fused per-sample pass ---
// One launch per bf16 mini-batch step for everything independent per
// sample: the gather of the observation rows, every hidden layer, the output
// layers with the PPO loss and their gradients, and the input-gradient chain.
// Its outputs are exactly the operands of the weight-gradient GEMMs and the
// loss partials of the head kernel.
constexpr int kFusedMaxAct = 16;

// Weights of the fused pass in MFMA A-fragment order (pack_frags): for a
// matrix with `rows` output features (a multiple of 32) and K inputs, S =
// ceil(K / 16) k-steps; fragment (fb, s) is 64 lanes x 8 bf16 at element
// ((fb * S + s) * 64) * 8, lane l holding row 32 fb + l % 32 and inputs
// 16 s + 8 (l / 32) .. + 7 (zero past K).
struct FragJob {
    const uint16_t *src;   // row-major bf16 W [out][in] with row pitch ld
    // split jobs: row-major float32 W instead; feature block fb stores its S
    // fragments of bf16(W), then S of bf16(W - bf16(W)) (the split layout)
    const float *src32;
    uint16_t *dst;
    int rows, K, S, ld;
    int transpose;         // 1: pack W^T (rows = in, K = out)
    int split;             // 1: the split layout from src32 (no transpose)
    int begin;             // first lane chunk of this job
};
constexpr int kMaxFragJobs = 16;
struct FragArgs {
    FragJob job[kMaxFragJobs];
    int count;
    int total;             // lane chunks (8 elements each)
};
void add_frag_job(FragArgs &a, const FragJob &j);
hipError_t launch_pack_frags(const FragArgs &a, hipStream_t s);

struct FusedNet {
    // layer l weights, fragment order, K = kpad for l = 0; the critic's (net
    // 1) in the split layout of FragJob (all bf16 fragments of a feature
    // block, then all residual fragments)
    const uint16_t *W[kMaxHidden];
    const uint16_t *WT[kMaxHidden];   // W_l^T, fragment order ([H_{l-1}] x H_l), l >= 1
    const float *bias[kMaxHidden];    // [H_l], 16-byte aligned
    const float *Wout, *bout;         // output layer (float32) [n_out][H_{L-1}], [n_out]
    uint16_t *h[kMaxHidden];          // [M][H_l] activations
    uint16_t *dz[kMaxHidden];         // [M][H_l] gradients wrt the pre-activations
    uint16_t *dzh;                    // [M][kHeadPad] gradient wrt the output layer
};

struct FusedArgs {
    FusedNet net[2];                  // actor, critic (n_out = A, 1)
    int L, D, kpad, A;
    int H[kMaxHidden];
    const float *obs;                 // [B][D]
    const int32_t *idx;               // [M] rows of the batch (clamped to [0, B)), or null
    int B, M;
    const float *actions, *logp_old, *adv, *returns, *values_old, *mu_old, *logstd_old, *logstd;
    uint16_t *xg;                     // [M][kpad] gathered inputs (written by the actor blocks)
    float *partials;                  // [blocks][A + 8], the layout of HeadLossArgs::partials
    uint8_t *active_out;              // [M] or null: 1 where the sample's surrogate passes gradient
    float *ratio_out;                 // [M] or null: the sample's probability ratio
    float clip, value_coef, inv_m;
    int clip_value;
    int no_backward;                  // loss terms only: skip the input-gradient chain
    // rollout inference (launch_fused_infer): outputs for the M environments
    // of obs (each may be null), Philox key and counter words, networks to run
    float *act_out, *logp_out, *val_out, *mu_out;
    uint32_t key0, key1, t_step, iteration;
    int net_mask;                     // bit 0: actor, bit 1: critic
    int R, NT, per_cu;                // samples, threads and workgroups per CU (a fused_shape)
    // filled in by launch_fused_update
    int blocks;
    int lds_region[kMaxHidden], lds_x, lds_w, lds_sum, lds_in, lds_rows, lds_bias, lds_head;
    // update pass only: offsets in its shared activation region of the last
    // hidden layer's output, of each backward layer's input gradient and of
    // the staged activation it multiplies by ELU', and the feature chunk of
    // the first hidden layer's input gradient
    int lds_last, lds_g, lds_bdz[kMaxHidden], lds_bst[kMaxHidden], chunk;
    // three workgroups per CU (streamed first layer): the first hidden
    // layer's output comes in chunks of chunk0 features at lds_cb, each added
    // into the second layer's accumulators as soon as it is written
    int lds_cb, chunk0;
    int defer_in;                     // the loss inputs load during the first layer after the streamed pair
    int vec_out;                      // inference: actions and means by 16-byte stores (A % 4 == 0, 16-byte aligned)
    int bias_off[kMaxHidden];         // floats into the staged biases
};
// Samples per workgroup and threads per workgroup of the fused pass for this
// network shape ({0, 0} when it does not apply: hidden widths that do not
// split over the waves, an input width that is not a multiple of 16, or
// activations that do not fit in LDS); per_cu = workgroups sharing a CU.
// Nonzero prefer_rows / prefer_threads / prefer_per_cu restrict the candidates.
struct FusedShape {
    int rows, threads, per_cu;
};
// update = true: the shapes of the update pass (its LDS plan differs from
// inference's).
FusedShape fused_shape(int L, const int *H, int kpad, int A, int prefer_rows = 0, int prefer_threads = 0,
                       bool update = false, int prefer_per_cu = 0);
int fused_blocks(int M, int R);
hipError_t launch_fused_update(FusedArgs a, hipStream_t s);
// Forward pass and sampling head for M environments (rows of obs in order).
hipError_t launch_fused_infer(FusedArgs a, hipStream_t s);

// -------------------------------------------------------- other kernels ---
// Observation assembly: proprio [N, P], then S height-scan columns; noise_scale
// may be null (no noise).
hipError_t launch_assemble_obs(hipStream_t s, const float *proprio, int P, const float *base, const float *height,
                               int nx, int ny, float inv_res, const float *scan, int S, const float *noise_scale,
                               long long N, uint64_t seed, uint32_t t, uint32_t iteration, float *obs);
hipError_t launch_philox_blocks(hipStream_t s, uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2,
                                uint32_t c3, long long n, uint32_t *out);

// Rows of obs (gathered by idx when non-null) converted to T, zero-padded to ld.
// Indices are clamped to [0, src_rows).
hipError_t launch_gather_obs(Precision prec, hipStream_t s, const float *obs, const int32_t *idx,
                             int src_rows, int rows, int D, int ld, void *out);

struct HeadSampleArgs {
    const void *ha;      // actor last hidden [N, Hl] (T)
    const void *hc;      // critic last hidden [N, Hl] (T)
    const float *Wa;     // [A, Hl]
    const float *ba;     // [A]
    const float *logstd; // [A]
    const float *Wc;     // [1, Hl]
    const float *bc;     // [1]
    float *actions, *logp, *values, *mu;
    int N, A, Hl;
    uint32_t key0, key1, t, iteration;
    int value_only;
};
hipError_t launch_head_sample(Precision prec, const HeadSampleArgs &a, hipStream_t s);

struct HeadLossArgs {
    const void *ha, *hc;           // last hidden [M, Hl] (T)
    const float *Wa, *ba, *logstd, *Wc, *bc;
    const float *actions, *logp_old, *adv, *returns, *values_old;  // full batch, indexed by idx
    const float *mu_old;           // [B, A] collection-time means, or null (no KL)
    const float *logstd_old;       // [A] collection-time log-std (with mu_old)
    const int32_t *idx;            // [M] rows of the batch, clamped to [0, B)
    int B;
    void *dza, *dzc;               // [M, Hl] (T): gradient wrt the last hidden pre-activations
    void *dz_head_a, *dz_head_c;   // [M, kHeadPad] (T): gradient wrt the output layer
    // [blocks, A + 8]: policy, value, clipped, ratio-KL sums, log-std gradient [A],
    // entropy, mean-shift KL sum, log-std KL part (entropy and the log-std part
    // in block 0, zero in the other blocks)
    float *partials;
    uint8_t *active_out;           // [M] or null: 1 where the sample's surrogate passes gradient
    float *ratio_out;              // [M] or null: the sample's probability ratio
    int M, A, Hl;
    float clip, value_coef, inv_m;
    int clip_value;
};
int head_loss_blocks(int M);
int head_loss_partial_width(int A);
hipError_t launch_head_loss(Precision prec, const HeadLossArgs &a, hipStream_t s);

struct GaeArgs {
    const float *rewards, *values, *last_values;
    const uint8_t *dones, *timeouts;
    float *adv, *returns;
    double *partials;   // [blocks, 3]: count, mean, M2
    int T, N;
    float gamma, lam;
};
int gae_blocks(int N);
// Environments the allocation-free GAE entry point serves (its partials live
// in a fixed device array of the library).
constexpr int kGaeNoAllocMaxN = 1 << 21;
// This device's copy of that array (looked up once per device).
hipError_t gae_scratch(double **out);
hipError_t launch_gae(const GaeArgs &a, hipStream_t s);
hipError_t launch_adv_finalize(const double *partials, int nparts, float *adv, long long count,
                               double *stats_out, int normalize, hipStream_t s);

// Gradient assembly: sum split-K partials per segment into the flat gradient,
// and per-block float64 sums of squares.
struct ReduceSegment {
    const float *src;         // partial s, row r, col c at src + s * split_stride + r * ld + c
    long long split_stride;
    int splits, rows, cols, ld;
    long long dst_offset;     // into the flat gradient
    long long begin;          // first global element index of this segment
    float add;                // constant added after the split sum
};
constexpr int kMaxSegments = 24;
struct ReduceArgs {
    ReduceSegment seg[kMaxSegments];
    int count;
    long long total;
    float *grad;
    double *sumsq_partials;   // [blocks]
    // loss partials of the head/loss kernel, reduced by the last block
    const float *loss_partials;  // [n_loss, loss_width]
    int n_loss, loss_width, A;
    long long logstd_offset;
    float entropy_coef;
    float *loss_sums;            // [8]: policy, value, clipped count, ratio-KL sums; entropy; mean KL
    // KL-adaptive rate: with lr non-null and desired_kl > 0 the last block
    // rescales *lr from the mean KL (inv_m = 1 / M)
    float *lr;
    float inv_m, desired_kl, lr_factor, lr_min, lr_max;
};
int reduce_blocks(long long total);  // includes the loss-partial block
hipError_t launch_grad_reduce(const ReduceArgs &a, hipStream_t s);

// A hidden-layer weight whose fragment copies (the layouts of
// pack_frags_kernel) Adam refreshes with every updated element, so that the
// next mini-batch step of the fused pass needs no packing launch.
struct AdamFrag {
    long long begin;        // flat offset of W_l [rows][cols] in theta
    int rows, cols, S, S_t; // S: k-steps of the forward fragments, S_t: of the transposed ones
    int split;              // forward fragments in the split layout (hi and lo per k-step)
    uint16_t *dst, *dst_t;  // forward and transposed fragments (dst_t null when not kept)
};
constexpr int kMaxAdamFrags = 2 * kMaxHidden;
struct AdamArgs {
    AdamFrag frag[kMaxAdamFrags];
    int n_frag;                // 0: no fragment copies to refresh
    float *theta, *grad, *m, *v;
    uint16_t *shadow;          // may be null
    const int32_t *step;       // steps already taken before this epoch
    int step_offset;           // this launch is step (*step + step_offset + 1)
    const float *lr;
    const double *sumsq_partials;
    int n_sumsq;
    const float *loss_sums;      // [8], written by the gradient reduction
    float max_grad_norm, beta1, beta2, eps, inv_m, value_coef, entropy_coef;
    float *stats;                // [kStatsWidth]
    long long P;
    int apply;                   // 0: only statistics (loss/grad without an optimiser step)
};
int adam_blocks(long long P);
hipError_t launch_adam(const AdamArgs &a, hipStream_t s);
hipError_t launch_step_advance(int32_t *step, int k, hipStream_t s);

// Per-step copies of weight matrices in the layouts the GEMMs load fastest:
// the first layer zero-padded to a vector-multiple width, and the hidden
// layers transposed for the input-gradient chain.  Elements of the GEMM
// operand type (bf16 or float32).
struct StageJob {
    const void *src;   // rows x cols, row pitch src_ld
    // bf16 staging only: when set, the job reads float32 W from here instead
    // of src and writes its bf16 residual bf16(W - bf16(W)) (no transpose)
    const float *lo_src;
    void *dst;         // transpose ? cols x rows : rows x dst_ld (cols..dst_ld zero-filled)
    int rows, cols, src_ld, dst_ld;
    int transpose;
    int tile_begin;    // first 64 x 64 tile of this job
};
constexpr int kMaxStageJobs = 16;
struct StageArgs {
    StageJob job[kMaxStageJobs];
    int count;
    int total_tiles;
};
void add_stage_job(StageArgs &a, const StageJob &j);
hipError_t launch_stage_weights(Precision prec, const StageArgs &a, hipStream_t s);
hipError_t launch_pack_bf16(const float *theta, uint16_t *shadow, long long n, hipStream_t s);

}  // namespace ppo
