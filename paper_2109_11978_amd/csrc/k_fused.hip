// Fused per-sample pass of the bf16 PPO update for gfx950 (CDNA4).
//
// Everything in a mini-batch step that is independent per sample runs in
// one launch: one workgroup takes R samples of one network (actor or critic)
// through the gather of their observation rows, every hidden layer
// (z = h W^T + b, h = ELU(z)), the output layer with the PPO loss of Section
// 2.2 and Appendix A.4, Table 3 (clipped surrogate, value loss, entropy
// bonus through the log-std gradient, KL statistic), and the input-gradient
// chain dz_{l-1} = (dz_l W_l) * ELU'(z_{l-1}) back to the first hidden layer.
// The activations live in LDS while they are used (fused_update_kernel
// shares one region between the layers); what leaves the chip is what the
// split-sample weight gradients read (gathered inputs, hidden activations,
// pre-activation and output gradients), in the layouts of the layer-by-layer
// path, each written once with coalesced 16-byte stores.
//
// MFMA layout: every layer is computed transposed, C[feature][sample] =
// W[feature, :] . act[sample, :], with v_mfma_f32_32x32x16_bf16.  The weights
// are the A operand (lane l: feature row l % 32, k = 8 (l / 32) .. + 7, one
// 16-byte buffer load from the row-major weight matrix), the activations the
// B operand (lane l: sample l % 32, the same 8 k, one 16-byte LDS read).  A
// lane's accumulators then hold, per group of four registers, 4 consecutive
// features of one sample: one 8-byte LDS write each.  The four waves split
// the output features and each covers all R samples, so every weight element
// is read from L2 once per workgroup; PF k-steps of weight fragments are in
// flight ahead of the MFMAs.
#include <type_traits>

#include "common.hpp"
#include "philox.hpp"

namespace ppo {
namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int kOutside = 0x7FFFFFF0;   // buffer offset past any resource: loads read zero
constexpr int kMaxLdsBytes = 160 * 1024;
constexpr float kLog2Pi = 1.8378770664093453f;
// per-sample loss terms: policy, value, clipped, ratio-KL, mean-shift KL,
// log-std gradient [kFusedMaxAct]
constexpr int kSums = 5 + kFusedMaxAct;
// per-sample loss inputs in LDS: actions [kFusedMaxAct], collection-time
// means [kFusedMaxAct] (both zero past A), old log-prob, advantage, return,
// old value
constexpr int kInW = 2 * kFusedMaxAct + 4;

__device__ inline __amdgpu_buffer_rsrc_t make_rsrc(const void *base, long long bytes) {
    const int n = bytes > 0x7FFFFFFFLL ? 0x7FFFFFFF : static_cast<int>(bytes < 0 ? 0 : bytes);
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), static_cast<short>(0), n, 0x00020000);
}

__device__ inline uint32_t bf16_bits(float v) {
    return __builtin_bit_cast(uint16_t, static_cast<__bf16>(v));
}
__device__ inline uint32_t pack2(float lo, float hi) { return bf16_bits(lo) | (bf16_bits(hi) << 16); }
__device__ inline float lo_f(uint32_t w) { return __uint_as_float(w << 16); }
__device__ inline float hi_f(uint32_t w) { return __uint_as_float(w & 0xFFFF0000u); }

// ELU and its derivative recovered from the activation h = ELU(z), with the
// values of the layer-by-layer GEMM epilogues in fewer instructions:
// e^z - 1 >= z everywhere and both sides share the sign of z, so ELU(z) is the
// median of (e^z - 1, z, 0); ELU'(z) is 1 for h > 0 and h + 1 = e^z otherwise,
// i.e. min(h + 1, 1).
__device__ inline float elu(float v) { return __builtin_amdgcn_fmed3f(__expf(v) - 1.0f, v, 0.0f); }
__device__ inline float delu(float h) { return fminf(h + 1.0f, 1.0f); }

__device__ inline float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// acc[f][j] = sum_k W[f0 + 32 f + (l % 32), k] * act[32 (sb0 + j) + (l % 32), k] over
// K = 16 S in k-steps of 16.  W is stored in MFMA fragment order (see
// pack_frags_kernel): the A fragment of feature block fb at k-step s is 1 KB
// at ((fb * S + s) * 64 + lane) * 16 bytes, so each load instruction reads
// one contiguous kilobyte.  act: LDS rows of `pitch` elements.  Weight
// fragments are loaded PF k-steps ahead and activation fragments one step
// ahead; scheduling barriers keep every step's loads behind its MFMAs, so
// the loads retire in issue order and each step waits only for its own
// fragments.  The loop runs whole groups of PF steps; steps past K multiply
// zero weight fragments (loaded from outside the buffer) with a clamped,
// finite activation fragment.
struct NoHook {
    __device__ void operator()() const {}
};

// The update pass runs its layers with a copy-out hook and shares each CU
// with a second workgroup: raising the wave priority over the MFMA loop lets
// one workgroup's matrix work run ahead of the other's epilogues and copies
// (1 % off the update).  Inference (no hook, one workgroup per CU) was 1 %
// slower with it and keeps the default priority.
template <class Hook>
constexpr bool kRaisePrio = !std::is_same<Hook, NoHook>::value;

template <int FBW, int SB, int PF, int SPLIT, class Hook = NoHook>
__device__ __forceinline__ void mma_layer(floatx16 (&acc)[FBW][SB], const uint16_t *W, int rows_w, int S, int f0,
                                          int sb0, const uint16_t *act, int pitch, int lane,
                                          const Hook &hook = Hook(), int s0 = 0, int Sc = -1, bool zero = true) {
    static_assert(SPLIT == 1 || SPLIT == 2, "one or two weight passes");
    // SPLIT = 2: each feature block has S fragments of bf16(W), then S of the
    // bf16 residual W - bf16(W); both passes multiply the same activation
    // fragments into the same accumulators, in the order of the layer-by-layer
    // GEMM (all of the first pass, then all of the second).
    // A call may take the k-steps s0 .. s0 + Sc of the layer only (its
    // activation fragments then start at act's column 0) and add to the
    // accumulators instead of starting from zero.
    if (Sc < 0) Sc = S;
    const int SW = S * SPLIT;     // weight fragments per feature block
    const int SWc = Sc * SPLIT;   // fragments this call multiplies
    auto frag = [&](int q) { return SPLIT == 1 || q < Sc ? s0 + q : S + s0 + (q - Sc); };
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(W, static_cast<long long>(rows_w / 32) * SW * 1024);
    const int kh = (lane >> 5) * 8;
    // per-block lane offsets in VGPRs, one scalar step offset per load
    int vo[FBW];
#pragma unroll
    for (int f = 0; f < FBW; ++f) vo[f] = (f0 / 32 + f) * SW * 1024 + lane * 16;
    const uint16_t *bp = act + (32 * sb0 + (lane & 31)) * pitch + kh;
    if (zero)
#pragma unroll
        for (int f = 0; f < FBW; ++f)
#pragma unroll
            for (int j = 0; j < SB; ++j) acc[f][j] = floatx16{};
    u32x4 w[PF][FBW];
#pragma unroll
    for (int p = 0; p < PF; ++p) {
        const int so = __builtin_amdgcn_readfirstlane(frag(p) * 1024);
#pragma unroll
        for (int f = 0; f < FBW; ++f)
            w[p][f] = __builtin_amdgcn_raw_buffer_load_b128(rs, p < SWc ? vo[f] : kOutside, so, 0);
        __builtin_amdgcn_sched_barrier(0);
    }
    // work that needs no weights (e.g. copying the previous layer's output to
    // global memory) runs while the first fragments are in flight
    hook();
    if constexpr (kRaisePrio<Hook>) __builtin_amdgcn_s_setprio(1);
    u32x4 b[SB];
#pragma unroll
    for (int j = 0; j < SB; ++j) b[j] = *reinterpret_cast<const u32x4 *>(bp + 32 * j * pitch);
    for (int q0 = 0; q0 < SWc; q0 += PF) {
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            // activation fragment of weight fragment q + 1: k-step (q + 1) mod Sc,
            // the last one again past the end
            const int q1 = q0 + u + 1;
            const int s1 = q1 < Sc ? q1 : (q1 < SWc ? q1 - Sc : Sc - 1);
            u32x4 bn[SB];
#pragma unroll
            for (int j = 0; j < SB; ++j) bn[j] = *reinterpret_cast<const u32x4 *>(bp + 32 * j * pitch + 16 * s1);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int f = 0; f < FBW; ++f)
#pragma unroll
                for (int j = 0; j < SB; ++j)
                    acc[f][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8_t, w[u][f]),
                                                                      __builtin_bit_cast(bf16x8_t, b[j]), acc[f][j],
                                                                      0, 0, 0);
            const int qn = q0 + u + PF;
            const int so = __builtin_amdgcn_readfirstlane(frag(qn) * 1024);
#pragma unroll
            for (int f = 0; f < FBW; ++f)
                w[u][f] = __builtin_amdgcn_raw_buffer_load_b128(rs, qn < SWc ? vo[f] : kOutside, so, 0);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int j = 0; j < SB; ++j) b[j] = bn[j];
        }
    }
    if constexpr (kRaisePrio<Hook>) __builtin_amdgcn_s_setprio(0);
}

// Forward epilogue: out[sample][feature] = bf16(ELU(acc + bias)).
template <int FBW, int SB>
__device__ __forceinline__ void epi_forward(const floatx16 (&acc)[FBW][SB], const float *bias, int f0, int sb0,
                                            uint16_t *out, int pitch, int lane) {
    const int h4 = (lane >> 5) * 4;
    const int i0 = 32 * sb0 + (lane & 31);
#pragma unroll
    for (int f = 0; f < FBW; ++f)
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const int fr = f0 + 32 * f + 8 * g + h4;
            const float4 b = *reinterpret_cast<const float4 *>(bias + fr);
#pragma unroll
            for (int j = 0; j < SB; ++j) {
                const float v0 = elu(acc[f][j][4 * g + 0] + b.x);
                const float v1 = elu(acc[f][j][4 * g + 1] + b.y);
                const float v2 = elu(acc[f][j][4 * g + 2] + b.z);
                const float v3 = elu(acc[f][j][4 * g + 3] + b.w);
                *reinterpret_cast<u32x2 *>(out + (i0 + 32 * j) * pitch + fr) = u32x2{pack2(v0, v1), pack2(v2, v3)};
            }
        }
}

// Backward epilogue, in place: hz holds h_{l-1}[sample][feature] on entry and
// dz_{l-1} = bf16(acc * ELU'(h_{l-1})) on exit.  Each element is read and
// written by the same lane.
template <int FBW, int SB>
__device__ __forceinline__ void epi_backward(const floatx16 (&acc)[FBW][SB], int f0, int sb0, uint16_t *hz, int pitch,
                                             int lane) {
    const int h4 = (lane >> 5) * 4;
    const int i0 = 32 * sb0 + (lane & 31);
#pragma unroll
    for (int f = 0; f < FBW; ++f)
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const int fr = f0 + 32 * f + 8 * g + h4;
#pragma unroll
            for (int j = 0; j < SB; ++j) {
                u32x2 *p = reinterpret_cast<u32x2 *>(hz + (i0 + 32 * j) * pitch + fr);
                const u32x2 h = *p;
                const float v0 = acc[f][j][4 * g + 0] * delu(lo_f(h.x));
                const float v1 = acc[f][j][4 * g + 1] * delu(hi_f(h.x));
                const float v2 = acc[f][j][4 * g + 2] * delu(lo_f(h.y));
                const float v3 = acc[f][j][4 * g + 3] * delu(hi_f(h.y));
                *p = u32x2{pack2(v0, v1), pack2(v2, v3)};
            }
        }
}

// Between a layer's MMA loop and its epilogue.  sync_epi 1: an output that
// overwrites the layer's input waits until every wave has read its input
// fragments.  2: also until the LDS-direct loads this wave issued (the
// epilogue's ELU' inputs, staged during the loop) have landed, which the
// barrier then extends to every wave's.
__device__ __forceinline__ void epi_sync(int sync_epi) {
    if (sync_epi == 2) __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
    if (sync_epi) __syncthreads();
}

template <int FBW, int SB, int PF, bool BWD, int SPLIT, class Hook>
__device__ __forceinline__ void layer_impl(const uint16_t *W, int K, int nout, const float *bias, const uint16_t *in,
                                           int in_pitch, uint16_t *out, int out_pitch, int f0, int sb0, int lane,
                                           const Hook &hook, int sync_epi) {
    floatx16 acc[FBW][SB];
    mma_layer<FBW, SB, PF, SPLIT>(acc, W, nout, K >> 4, f0, sb0, in, in_pitch, lane, hook);
    epi_sync(sync_epi);
    if constexpr (BWD)
        epi_backward<FBW, SB>(acc, f0, sb0, out, out_pitch, lane);
    else
        epi_forward<FBW, SB>(acc, bias, f0, sb0, out, out_pitch, lane);
}

// Weight fragments in flight per lane: PF fragments x FBW blocks, up to 32,
// with PF no larger than the layer's fragment count S * SPLIT (S = K / 16, a
// power of two for hidden layers; a first layer of 3 or 15 k-steps takes
// PF = 4).
template <int FBW, int SB, bool BWD, int PFMAX, int SPLIT, class Hook>
__device__ __forceinline__ void layer_pf(int S, const uint16_t *W, int K, int nout, const float *bias,
                                         const uint16_t *in, int in_pitch, uint16_t *out, int out_pitch, int f0,
                                         int sb0, int lane, const Hook &hook, int sync_epi) {
    const int SW = S * SPLIT;
    if (PFMAX >= 32 && SW >= 32)
        layer_impl<FBW, SB, (PFMAX >= 32 ? 32 : 4), BWD, SPLIT>(W, K, nout, bias, in, in_pitch, out, out_pitch, f0,
                                                                sb0, lane, hook, sync_epi);
    else if (PFMAX >= 16 && SW >= 16)
        layer_impl<FBW, SB, (PFMAX >= 16 ? 16 : 4), BWD, SPLIT>(W, K, nout, bias, in, in_pitch, out, out_pitch, f0,
                                                                sb0, lane, hook, sync_epi);
    else if (PFMAX >= 8 && SW >= 8)
        layer_impl<FBW, SB, (PFMAX >= 8 ? 8 : 4), BWD, SPLIT>(W, K, nout, bias, in, in_pitch, out, out_pitch, f0,
                                                              sb0, lane, hook, sync_epi);
    else
        layer_impl<FBW, SB, 4, BWD, SPLIT>(W, K, nout, bias, in, in_pitch, out, out_pitch, f0, sb0, lane, hook, sync_epi);
}

// Deepest weight prefetch (k-steps) that keeps the accumulators (FBW x SBW
// blocks of 16 registers) and the fragment ring (PF x FBW x 4 registers)
// within REGS registers, at most 8 fragments in flight per wave (deeper rings
// measured slower: the waves of a CU share its memory pipe, and long bursts
// queue there), at least 4 steps.
template <int FBW, int SBW, int REGS>
constexpr int pf_max() {
    int pf = 32 / FBW;
    while (pf > 4 && (FBW * SBW * 16 + pf * FBW * 4 > REGS || pf * FBW > 8)) pf /= 2;
    return pf;
}

// Feature blocks per wave whose accumulators (16 registers per block and
// sample block) fit a register budget; the shape checks (width_splits with
// the same budget) keep other widths from being launched.
constexpr bool acc_fits(int fbw, int sbw, int regs) { return fbw * sbw * 16 <= regs; }

template <int SBW, bool BWD, bool WIDE, int REGS, int SPLIT, class Hook>
__device__ __forceinline__ void layer_fb(int fbw, int S, const uint16_t *W, int K, int nout, const float *bias,
                                         const uint16_t *in, int in_pitch, uint16_t *out, int out_pitch, int f0,
                                         int sb0, int lane, const Hook &hook, int sync_epi) {
    switch (fbw) {
    case 1:
        layer_pf<1, SBW, BWD, pf_max<1, SBW, REGS>(), SPLIT>(S, W, K, nout, bias, in, in_pitch, out, out_pitch, f0,
                                                             sb0, lane, hook, sync_epi);
        break;
    case 2:
        if constexpr (acc_fits(2, SBW, REGS)) {
            layer_pf<2, SBW, BWD, pf_max<2, SBW, REGS>(), SPLIT>(S, W, K, nout, bias, in, in_pitch, out, out_pitch,
                                                                 f0, sb0, lane, hook, sync_epi);
            break;
        }
        hook();
        epi_sync(sync_epi);
        break;
    case 4:
        if constexpr (acc_fits(4, SBW, REGS)) {
            layer_pf<4, SBW, BWD, pf_max<4, SBW, REGS>(), SPLIT>(S, W, K, nout, bias, in, in_pitch, out, out_pitch,
                                                                 f0, sb0, lane, hook, sync_epi);
            break;
        }
        hook();
        epi_sync(sync_epi);
        break;
    default:
        if constexpr (WIDE)
            layer_pf<8, SBW, BWD, pf_max<8, SBW, REGS>(), SPLIT>(S, W, K, nout, bias, in, in_pitch, out, out_pitch,
                                                                 f0, sb0, lane, hook, sync_epi);
        else {
            hook();
            epi_sync(sync_epi);
        }
        break;
    }
}

// Registers for a layer's accumulators and fragment ring per lane: 512 /
// WPE, less what the addresses, activation fragments and epilogue keep live
// (and, at three workgroups per CU, the streamed first layer's accumulators).
// At three workgroups per CU the budget is lower than that on purpose: a
// one-block layer then keeps 8 fragments in flight rather than 16, and the
// twelve waves' shorter bursts queue less at the CU's shared memory pipe
// (measured faster).  Likewise for one sample block at two per CU (rollout
// inference): 64, not 192, so a layer of four or two feature blocks per wave
// keeps 4 k-steps in flight rather than 8 or 16, and a one-block layer 8
// rather than 32 (measured faster at each step down); and for two sample
// blocks at two waves per SIMD (the [1024, 512, 256] update): 128, not 160,
// so its one-block layer keeps 16 rather than 32 (measured faster).
constexpr int layer_regs(int wpe, int sb) { return wpe == 1 ? 320 : (wpe >= 3 ? 80 : (sb >= 2 ? 128 : 64)); }

// One layer for all R samples of the block.  The layer's 32-feature blocks
// are split over the NT / 64 waves; when there are fewer blocks than waves,
// the waves sharing a block split the sample blocks instead (each weight
// fragment is then read by two waves, the second time from L1).
template <int R, int NT, int WPE, bool BWD, int SPLIT = 1, class Hook = NoHook>
__device__ __forceinline__ void run_layer(const uint16_t *W, int K, int nout, const float *bias, const uint16_t *in,
                                          int in_pitch, uint16_t *out, int out_pitch, int wave, int lane,
                                          const Hook &hook = Hook(), int sync_epi = 0) {
    constexpr int NW = NT / 64;
    constexpr int SB = R / 32;
    // registers for accumulators and fragments: 512 / WPE per lane, less
    // what the addresses, activation fragments and epilogue keep live
    constexpr int REGS = layer_regs(WPE, SB);
    // eight feature blocks per wave only with one sample block and a full
    // register file
    constexpr bool WIDE = SB == 1 && WPE == 1;
    const int S = K >> 4;
    const int fb = nout / 32;
    if (fb >= NW) {
        const int fbw = fb / NW;
        layer_fb<SB, BWD, WIDE, REGS, SPLIT>(fbw, S, W, K, nout, bias, in, in_pitch, out, out_pitch,
                                             wave * fbw * 32, 0, lane, hook, sync_epi);
    } else if constexpr (SB >= 2) {
        // two waves per feature block, each with half the sample blocks
        layer_fb<SB / 2, BWD, false, REGS, SPLIT>(1, S, W, K, nout, bias, in, in_pitch, out, out_pitch,
                                                  (wave % fb) * 32, (wave / fb) * (SB / 2), lane, hook, sync_epi);
    } else {
        hook();   // a wave without a feature block still does its share of the hook
        epi_sync(sync_epi);
    }
}

// rows x cols bf16 from LDS (row pitch `pitch`) to global rows of `ld`
// elements; cols is a multiple of 8 and at most 8 * NT.  Each
// thread keeps one 16-byte column chunk and strides over the rows; four LDS
// reads go out before their stores, and stores past the last row fall
// outside the buffer and are dropped.
template <int NT>
__device__ inline void copy_out(const uint16_t *src, int pitch, uint16_t *dst, int ld, int cols, int rows) {
    constexpr int U = 4;
    const int cpr = cols >> 3;
    const int rpp = NT / cpr;   // rows per pass
    const int r0 = threadIdx.x / cpr;
    const int c = (threadIdx.x - r0 * cpr) * 8;
    if (r0 >= rpp) return;
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(dst, static_cast<long long>(rows) * ld * 2);
    for (int i0 = r0; i0 < rows; i0 += U * rpp) {
        u32x4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = min(i0 + u * rpp, rows - 1);
            v[u] = *reinterpret_cast<const u32x4 *>(src + i * pitch + c);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u * rpp;
            __builtin_amdgcn_raw_buffer_store_b128(v[u], rs, i < rows ? (i * ld + c) * 2 : kOutside, 0, 0);
        }
    }
}

// Observation rows of the block (batch rows s_rows[0 .. R), or m0 .. m0 + R
// when s_rows is null) as bf16 into
// LDS, zero-padded to kpad columns and zero past the last valid row.  Wave w
// takes rows w, w + NW, ...; its lanes take consecutive 16-byte chunks of
// those rows (coalesced), four loads in flight per lane (out-of-range ones
// read zero).
template <int R, int NT>
__device__ inline void gather_rows(const FusedArgs &a, const int *s_rows, int rows, uint16_t *x, int pitch,
                                   int wave, int lane, int m0 = 0) {
    constexpr int NW = NT / 64;
    constexpr int PER_WAVE = R / NW;
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(a.obs, static_cast<long long>(a.B) * a.D * 4);
    if ((a.D & 3) == 0) {
        // rows start 16-byte aligned: four elements per lane and load, the
        // wave's rows one after another over its lanes (four loads in flight)
        constexpr int V = 4;
        const int n4 = a.kpad >> 2;         // 4-element chunks per row (padded)
        const int d4 = a.D >> 2;
        const int total = PER_WAVE * n4;    // chunks per wave
        for (int t0 = 0; t0 < total; t0 += V * 64) {
            float4 v[V];
#pragma unroll
            for (int u = 0; u < V; ++u) {
                const int t = min(t0 + 64 * u + lane, total - 1);
                const int il = t / n4, c4 = t - il * n4;
                const int i = wave + NW * il;
                const bool ok = t0 + 64 * u + lane < total && i < rows && c4 < d4;
                const int row = s_rows ? s_rows[i] : m0 + min(i, rows - 1);
                const u32x4 w = __builtin_amdgcn_raw_buffer_load_b128(rs, ok ? (row * a.D + 4 * c4) * 4 : kOutside, 0, 0);
                v[u] = make_float4(__uint_as_float(w[0]), __uint_as_float(w[1]), __uint_as_float(w[2]),
                                   __uint_as_float(w[3]));
            }
#pragma unroll
            for (int u = 0; u < V; ++u) {
                const int t = t0 + 64 * u + lane;
                if (t < total) {
                    const int il = t / n4, c4 = t - il * n4;
                    const int i = wave + NW * il;
                    *reinterpret_cast<u32x2 *>(x + i * pitch + 4 * c4) =
                        u32x2{pack2(v[u].x, v[u].y), pack2(v[u].z, v[u].w)};
                }
            }
        }
        return;
    }
    // rows at any alignment: each lane loads one 16-byte aligned chunk of
    // the buffer that overlaps the row and writes the row's elements in it.
    // Row element k sits in chunk (k + off) / 4, slot (k + off) % 4, where
    // off = (row D) mod 4, so chunks 0 .. kpad / 4 cover every padded column
    // once; columns past D and rows past the block's last read as zero.
    // The last row's last chunk may run up to 12 bytes past the buffer: the
    // range is rounded up to 16 bytes (the same 16-byte granule, so the same
    // page), and those elements fall in columns past D.
    constexpr int V = 4;
    const int n4 = (a.kpad >> 2) + 1;       // chunks per row
    const int total = PER_WAVE * n4;        // chunks per wave
    const __amdgpu_buffer_rsrc_t ru = make_rsrc(a.obs, (static_cast<long long>(a.B) * a.D * 4 + 15) & ~15LL);
    for (int t0 = 0; t0 < total; t0 += V * 64) {
        u32x4 w[V];
        int e0[V];
#pragma unroll
        for (int u = 0; u < V; ++u) {
            const int t = min(t0 + 64 * u + lane, total - 1);
            const int il = t / n4, c = t - il * n4;
            const int i = wave + NW * il;
            const int row = s_rows ? s_rows[i] : m0 + min(i, rows - 1);
            e0[u] = row * a.D;
            const bool ok = t0 + 64 * u + lane < total && i < rows;
            w[u] = __builtin_amdgcn_raw_buffer_load_b128(ru, ok ? ((e0[u] >> 2) + c) * 16 : kOutside, 0, 0);
        }
#pragma unroll
        for (int u = 0; u < V; ++u) {
            const int t = t0 + 64 * u + lane;
            if (t >= total) continue;
            const int il = t / n4, c = t - il * n4;
            const int i = wave + NW * il;
            const int k0 = 4 * c - (e0[u] & 3);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int k = k0 + q;
                if (k >= 0 && k < a.kpad)
                    x[i * pitch + k] = static_cast<uint16_t>(k < a.D ? bf16_bits(__uint_as_float(w[u][q])) : 0u);
            }
        }
    }
}

// Sum over the KP adjacent lanes of a sample (KP = 4, 8 or 16) with DPP lane
// swaps: xor 1 and xor 2 inside each quad, then the quads of an 8-lane half
// row exchanged by the half-row mirror, then the halves of a 16-lane row by
// the row mirror.  Every lane ends with the same value (each step adds a
// value and its partner's in commuted order).
template <int KP>
__device__ inline float kpart_sum(float v) {
    v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, true));   // quad [1,0,3,2]
    v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xF, 0xF, true));   // quad [2,3,0,1]
    if constexpr (KP >= 8)
        v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x141, 0xF, 0xF, true));  // half mirror
    if constexpr (KP >= 16)
        v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x140, 0xF, 0xF, true));  // row mirror
    return v;
}

// Output-layer values o[j] = b_j + h . W_j (j < NO) of one sample: each of
// its KP lanes loads NCK 8-element chunks of h (kept in hx for the caller)
// and multiplies them with its slice of the staged float32 weights; the
// partial sums are combined with DPP lane swaps that leave the same value in
// every lane of the sample.
template <int KP, int NCK, int NO>
__device__ __forceinline__ void head_dots(const uint16_t *hrow, const float *wl, int WP, const float *s_head,
                                          u32x4 (&hx)[NCK], float (&o)[NO]) {
#pragma unroll
    for (int c = 0; c < NCK; ++c) hx[c] = *reinterpret_cast<const u32x4 *>(hrow + 8 * c);
#pragma unroll
    for (int j = 0; j < NO; ++j) o[j] = 0.0f;
#pragma unroll
    for (int c = 0; c < NCK; ++c) {
        float xv[8];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            xv[2 * e] = lo_f(hx[c][e]);
            xv[2 * e + 1] = hi_f(hx[c][e]);
        }
#pragma unroll
        for (int j = 0; j < NO; ++j) {
            const float4 w0 = *reinterpret_cast<const float4 *>(wl + j * WP + 8 * c);
            const float4 w1 = *reinterpret_cast<const float4 *>(wl + j * WP + 8 * c + 4);
            o[j] += xv[0] * w0.x + xv[1] * w0.y + xv[2] * w0.z + xv[3] * w0.w + xv[4] * w1.x + xv[5] * w1.y +
                    xv[6] * w1.z + xv[7] * w1.w;
        }
    }
#pragma unroll
    for (int j = 0; j < NO; ++j) o[j] = kpart_sum<KP>(o[j]) + s_head[j];
}

// Network and sample block of workgroup b when both networks run in one
// grid.  Workgroups go round-robin over the 8 XCDs, so the network index
// alternates every 8 workgroups rather than every one: each XCD then runs
// both networks' blocks in equal numbers (the critic's forward makes its
// blocks the longer ones) and keeps both networks' weights in its L2.
// Returns false for the padding workgroups past the last sample block.
__device__ inline bool net_block(int b, int blocks, int &net, int &sblk) {
    net = (b >> 3) & 1;
    sblk = (b >> 4) * 8 + (b & 7);
    return sblk < blocks;
}

// rows x cols bf16 from global rows of `ld` elements into LDS (row pitch
// `pitch`; rows past `rows` up to R and the row pads zero), the inverse of
// copy_out.  The source was written earlier in the same launch by this
// workgroup's copy_out (visible after the workgroup barriers in between).
// Each LDS-direct buffer load of a wave fills one
// contiguous kilobyte of the padded tile, lane i its bytes 16 i .. 16 i + 15,
// so every lane derives its source row and column from that position.  No
// registers hold the data, so the loads can be issued ahead of an MMA loop;
// the tile is complete once every wave has waited for its loads (vmcnt) and
// the workgroup has synchronised.  pitch and cols are multiples of 8.
template <int NT>
__device__ inline void copy_in_async(const uint16_t *src, int ld, uint16_t *dst, int pitch, int cols, int rows,
                                     int R, int wave, int lane) {
    constexpr int NW = NT / 64;
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(src, static_cast<long long>(rows) * ld * 2);
    const int row_bytes = pitch * 2;
    const int total = R * row_bytes;
    typedef __attribute__((address_space(3))) void lds_void;
    for (int b = wave; b * 1024 < total; b += NW) {
        const int o = b * 1024 + lane * 16;
        const int r = o / row_bytes, cb = o - r * row_bytes;
        const int voff = r < rows && cb < cols * 2 ? r * ld * 2 + cb : kOutside;
        if (o < total)
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_void *)(reinterpret_cast<char *>(dst) + b * 1024), 16,
                                                     voff, 0, 0, 0);
    }
}

// Output layer, PPO loss terms and output gradients of the block's samples.
// KP = NT / R adjacent lanes per sample, NCK 8-element chunks of
// the last hidden layer per lane; the actor computes kFusedMaxAct outputs
// (weights, biases, log-std and loss inputs zero past A, which makes the
// extra terms vanish), the critic one.  Partial dot products are combined
// with DPP lane swaps that leave the same value in every lane of a sample,
// so all of them compute the same loss terms and output gradients; the
// sample's first lane stores its output-gradient row and loss terms.  On
// return the last hidden layer in LDS holds the gradient wrt its
// pre-activations (after a barrier: every thread's copy of h_{L-1} to global
// memory has read it).
template <int R, int NT, int NCK, bool ACTOR>
__device__ __forceinline__ void head_pass(const FusedArgs &a, const FusedNet &N, uint16_t *hl, int PL,
                                          const float *w_out, int WP, const float *s_head, const float *s_in,
                                          float *s_sum, int m0, int rows) {
    constexpr int KP = NT / R;
    constexpr int CK = NCK * 8;
    constexpr int NO = ACTOR ? kFusedMaxAct : 1;
    const int tid = threadIdx.x;
    const int si = tid / KP, kq = tid % KP;
    const bool valid = si < rows;
    const bool lead = valid && kq == 0;
    const float *in_s = s_in + si * kInW;
    uint16_t *hrow = hl + si * PL + kq * CK;
    const float *wl = w_out + kq * CK;
    u32x4 hx[NCK];
    float o[NO];
    head_dots<KP, NCK, NO>(hrow, wl, WP, s_head, hx, o);

    float g[NO];
    float sums[kSums];
#pragma unroll
    for (int q = 0; q < kSums; ++q) sums[q] = 0.0f;
    if constexpr (ACTOR) {
        const int A = a.A;
        // log-ratio log pi(a|s) - lp_old: the A log-density terms and -lp_old
        // summed with compensation in float32 (terms of order 1 that nearly
        // cancel against lp_old)
        float z[NO], inv_sig[NO];
        CompSum lr;
        float kl_mu = 0.0f;
#pragma unroll
        for (int j = 0; j < NO; ++j) {
            const float ls = s_head[kFusedMaxAct + j];
            inv_sig[j] = expf(-ls);
            z[j] = (in_s[j] - o[j]) * inv_sig[j];
            if (j < A) lr.add_gauss(z[j], ls);
            const float dm = (in_s[kFusedMaxAct + j] - o[j]) * inv_sig[j];
            kl_mu += 0.5f * dm * dm;
        }
        lr.add(-in_s[2 * kFusedMaxAct]);
        const float adv = in_s[2 * kFusedMaxAct + 1];
        const float ratio = expf(lr.value());
        const float lo = 1.0f - a.clip, hi = 1.0f + a.clip;
        const bool active = adv >= 0.0f ? (ratio <= hi) : (ratio >= lo);
        if (lead && a.active_out) a.active_out[m0 + si] = active ? 1 : 0;
        if (lead && a.ratio_out) a.ratio_out[m0 + si] = ratio;
        const float g_lp = valid && active ? -a.inv_m * adv * ratio : 0.0f;
        sums[0] = -fminf(ratio * adv, fminf(fmaxf(ratio, lo), hi) * adv);
        sums[2] = fabsf(ratio - 1.0f) > a.clip ? 1.0f : 0.0f;
        sums[3] = (ratio - 1.0f) - logf(ratio);
        sums[4] = kl_mu;
#pragma unroll
        for (int j = 0; j < NO; ++j) {
            g[j] = g_lp * z[j] * inv_sig[j];
            sums[5 + j] = g_lp * (z[j] * z[j] - 1.0f);
        }
    } else {
        const float V = o[0];
        const float ret = in_s[2 * kFusedMaxAct + 2], v_old = in_s[2 * kFusedMaxAct + 3];
        const float diff = V - ret;
        float pass = 1.0f, vl = diff * diff;
        if (a.clip_value) {
            const float vc = v_old + fminf(fmaxf(V - v_old, -a.clip), a.clip);
            const float sqc = (vc - ret) * (vc - ret);
            pass = vl >= sqc ? 1.0f : 0.0f;
            vl = fmaxf(vl, sqc);
        }
        g[0] = valid ? 2.0f * a.value_coef * a.inv_m * diff * pass : 0.0f;
        sums[1] = vl;
    }
    if (lead) {
        // output-layer gradient row, zero-padded to kHeadPad columns
        float gp[kHeadPad];
#pragma unroll
        for (int e = 0; e < kHeadPad; ++e) gp[e] = e < NO ? g[e < NO ? e : 0] : 0.0f;
        uint32_t pk[kHeadPad / 2];
#pragma unroll
        for (int e = 0; e < kHeadPad / 2; ++e) pk[e] = pack2(gp[2 * e], gp[2 * e + 1]);
        u32x4 *dst = reinterpret_cast<u32x4 *>(N.dzh + static_cast<long long>(m0 + si) * kHeadPad);
        dst[0] = u32x4{pk[0], pk[1], pk[2], pk[3]};
        dst[1] = u32x4{pk[4], pk[5], pk[6], pk[7]};
#pragma unroll
        for (int q = 0; q < kSums; ++q) s_sum[si * kSums + q] = sums[q];
    }

    // gradient into the last hidden pre-activations, in place over h_{L-1}
    __syncthreads();
#pragma unroll
    for (int c = 0; c < NCK; ++c) {
        float dh[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) dh[e] = 0.0f;
#pragma unroll
        for (int j = 0; j < NO; ++j) {
            const float4 w0 = *reinterpret_cast<const float4 *>(wl + j * WP + 8 * c);
            const float4 w1 = *reinterpret_cast<const float4 *>(wl + j * WP + 8 * c + 4);
            dh[0] += g[j] * w0.x; dh[1] += g[j] * w0.y; dh[2] += g[j] * w0.z; dh[3] += g[j] * w0.w;
            dh[4] += g[j] * w1.x; dh[5] += g[j] * w1.y; dh[6] += g[j] * w1.z; dh[7] += g[j] * w1.w;
        }
        u32x4 ov;
#pragma unroll
        for (int e = 0; e < 4; ++e)
            ov[e] = pack2(dh[2 * e] * delu(lo_f(hx[c][e])), dh[2 * e + 1] * delu(hi_f(hx[c][e])));
        *reinterpret_cast<u32x4 *>(hrow + 8 * c) = ov;
    }
}

// bf16 pieces of float32 values: hi = bf16(x), then the bf16 residuals.
__device__ inline void split3(const float (&x)[8], u32x4 &hi, u32x4 &mid, u32x4 &lo) {
    float r1[8], r2[8];
    uint32_t h[8], m[8], l[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        h[e] = bf16_bits(x[e]);
        r1[e] = x[e] - __uint_as_float(h[e] << 16);
        m[e] = bf16_bits(r1[e]);
        r2[e] = r1[e] - __uint_as_float(m[e] << 16);
        l[e] = bf16_bits(r2[e]);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        hi[e] = h[2 * e] | (h[2 * e + 1] << 16);
        mid[e] = m[2 * e] | (m[2 * e + 1] << 16);
        lo[e] = l[2 * e] | (l[2 * e + 1] << 16);
    }
}
__device__ inline void split2(const float (&x)[8], u32x4 &hi, u32x4 &lo) {
    u32x4 mid;
    split3(x, hi, lo, mid);
}
__device__ inline floatx16 mfma16(const u32x4 &a, const u32x4 &b, const floatx16 &c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8_t, a), __builtin_bit_cast(bf16x8_t, b), c,
                                                   0, 0, 0);
}

// Output layer, PPO loss terms and output gradients of the block's samples on
// MFMA (the update pass).  Wave w < R / 32 takes sample block w: the output
// layer C[output][sample] = W_out[output, :] . h[sample, :] + b with the
// float32 weights as three bf16 terms (their sum is the float32 weight
// exactly, so each product is exact and the sums are float32 sums), which
// leaves in lane l sample 32 w + l % 32 and outputs 8 g + 4 (l / 32) + e
// (g = 0, 1; e = 0 .. 3): every sample's outputs sit in two lanes, l and
// l ^ 32, which combine their partial sums with one lane swap.  Both lanes
// then compute the loss terms and the output gradients of their outputs.
// The gradient into the last hidden layer, dh[feature][sample] =
// sum_j g_j W_out[j, feature], is a second MFMA pass over all waves (the
// float32 gradients and weights as bf16 pairs, the three larger products;
// the result is rounded to bf16 anyway), whose epilogue multiplies by ELU'
// in place over h, as the hidden layers' backward epilogue does.  s_g holds
// the output gradients [R][kFusedMaxAct] between the two passes.
template <int R, int NT, bool ACTOR>
__device__ __forceinline__ void head_mfma(const FusedArgs &a, const FusedNet &N, uint16_t *hl, int PL,
                                          const float *w_out, int WP, const float *s_head, const float *s_in,
                                          float *s_sum, float *s_g, int m0, int rows, int wave, int lane) {
    constexpr int SB = R / 32;
    constexpr int NW = NT / 64;
    const int Hl = a.H[a.L - 1];
    const int S = Hl / 16;
    const int half = lane >> 5;
    if (wave < SB) {
        const int si = 32 * wave + (lane & 31);
        const bool valid = si < rows;
        // ---- output layer
        floatx16 acc = floatx16{};
        const int orow = lane & 31;   // output row of the A operand
        const uint16_t *bp = hl + si * PL + 8 * half;
        for (int s = 0; s < S; ++s) {
            float w8[8];
            const float *wr = w_out + orow * WP + 16 * s + 8 * half;
#pragma unroll
            for (int e = 0; e < 8; ++e) w8[e] = orow < kFusedMaxAct ? wr[e] : 0.0f;
            u32x4 hi, mid, lo;
            split3(w8, hi, mid, lo);
            const u32x4 b = *reinterpret_cast<const u32x4 *>(bp + 16 * s);
            acc = mfma16(lo, b, acc);
            acc = mfma16(mid, b, acc);
            acc = mfma16(hi, b, acc);
        }
        // this lane's outputs: j(g, e) = 8 g + 4 half + e, g = 0, 1
        float o[8];
#pragma unroll
        for (int g = 0; g < 2; ++g)
#pragma unroll
            for (int e = 0; e < 4; ++e) o[4 * g + e] = acc[4 * g + e] + s_head[8 * g + 4 * half + e];
        const float *in_s = s_in + si * kInW;
        float g8[8];
        float sums[kSums];
#pragma unroll
        for (int q = 0; q < kSums; ++q) sums[q] = 0.0f;
        if constexpr (ACTOR) {
            const int A = a.A;
            CompSum lr;
            float kl_mu = 0.0f, z[8], inv_sig[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const int j = 8 * (t >> 2) + 4 * half + (t & 3);
                const float ls = s_head[kFusedMaxAct + j];
                inv_sig[t] = expf(-ls);
                z[t] = (in_s[j] - o[t]) * inv_sig[t];
                if (j < A) lr.add_gauss(z[t], ls);
                // mean-shift part of KL(pi_old || pi), only with collection-time means
                const float dm = (in_s[kFusedMaxAct + j] - o[t]) * inv_sig[t];
                if (a.mu_old && j < A) kl_mu += 0.5f * dm * dm;
            }
            // the partner lane's half of the log-density and KL (the same
            // result in both lanes: every combination below is symmetric)
            {
                const float ps = __shfl_xor(lr.s, 32), pc = __shfl_xor(lr.c, 32);
                const float t = lr.s + ps;
                const float err = fabsf(lr.s) >= fabsf(ps) ? (lr.s - t) + ps : (ps - t) + lr.s;
                lr.c = (lr.c + pc) + err;
                lr.s = t;
                kl_mu += __shfl_xor(kl_mu, 32);
            }
            lr.add(-in_s[2 * kFusedMaxAct]);
            const float adv = in_s[2 * kFusedMaxAct + 1];
            const float ratio = expf(lr.value());
            const float lo = 1.0f - a.clip, hi = 1.0f + a.clip;
            const bool active = adv >= 0.0f ? (ratio <= hi) : (ratio >= lo);
            const float g_lp = valid && active ? -a.inv_m * adv * ratio : 0.0f;
            if (valid && half == 0) {
                if (a.active_out) a.active_out[m0 + si] = active ? 1 : 0;
                if (a.ratio_out) a.ratio_out[m0 + si] = ratio;
            }
            sums[0] = -fminf(ratio * adv, fminf(fmaxf(ratio, lo), hi) * adv);
            sums[2] = fabsf(ratio - 1.0f) > a.clip ? 1.0f : 0.0f;
            sums[3] = (ratio - 1.0f) - logf(ratio);
            sums[4] = kl_mu;
#pragma unroll
            for (int t = 0; t < 8; ++t) {
                const int j = 8 * (t >> 2) + 4 * half + (t & 3);
                g8[t] = g_lp * z[t] * inv_sig[t];
                sums[5 + j] = g_lp * (z[t] * z[t] - 1.0f);
            }
        } else {
            // the value is output 0: lane half 0, first accumulator
            const float V = __shfl(o[0], lane & 31);
            const float ret = in_s[2 * kFusedMaxAct + 2], v_old = in_s[2 * kFusedMaxAct + 3];
            const float diff = V - ret;
            float pass = 1.0f, vl = diff * diff;
            if (a.clip_value) {
                const float vc = v_old + fminf(fmaxf(V - v_old, -a.clip), a.clip);
                const float sqc = (vc - ret) * (vc - ret);
                pass = vl >= sqc ? 1.0f : 0.0f;
                vl = fmaxf(vl, sqc);
            }
#pragma unroll
            for (int t = 0; t < 8; ++t) g8[t] = 0.0f;
            if (half == 0) g8[0] = valid ? 2.0f * a.value_coef * a.inv_m * diff * pass : 0.0f;
            sums[1] = vl;
        }
        if (valid) {
            // output-layer gradient row [kHeadPad] in bf16: this lane's 8 of 16
            uint16_t *row = N.dzh + static_cast<long long>(m0 + si) * kHeadPad;
            *reinterpret_cast<u32x2 *>(row + 4 * half) = u32x2{pack2(g8[0], g8[1]), pack2(g8[2], g8[3])};
            *reinterpret_cast<u32x2 *>(row + 8 + 4 * half) = u32x2{pack2(g8[4], g8[5]), pack2(g8[6], g8[7])};
        }
        // per-sample loss terms (lane half 0: the scalars; both: their log-std terms)
        float *ss = s_sum + si * kSums;
        if (half == 0)
#pragma unroll
            for (int q = 0; q < 5; ++q) ss[q] = sums[q];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int j = 8 * (t >> 2) + 4 * half + (t & 3);
            ss[5 + j] = sums[5 + j];
            s_g[si * kFusedMaxAct + j] = g8[t];
        }
    }
    __syncthreads();
    // ---- gradient into the last hidden layer, in place over h
    const int FB = Hl / 32;
    for (int tile = wave; tile < FB * SB; tile += NW) {
        const int fb = tile % FB, sb = tile / FB;
        // B: the output gradients of sample 32 sb + l % 32, outputs 8 half .. + 7
        float gb[8], wa[8];
        const float *gs = s_g + (32 * sb + (lane & 31)) * kFusedMaxAct + 8 * half;
#pragma unroll
        for (int e = 0; e < 8; ++e) gb[e] = gs[e];
        // A: W_out^T rows = features 32 fb + l % 32, k = outputs 8 half .. + 7
        const float *wc = w_out + 32 * fb + (lane & 31);
#pragma unroll
        for (int e = 0; e < 8; ++e) wa[e] = wc[(8 * half + e) * WP];
        u32x4 bh, bl, ah, al;
        split2(gb, bh, bl);
        split2(wa, ah, al);
        floatx16 acc[1][1];
        acc[0][0] = floatx16{};
        acc[0][0] = mfma16(al, bh, acc[0][0]);
        acc[0][0] = mfma16(ah, bl, acc[0][0]);
        acc[0][0] = mfma16(ah, bh, acc[0][0]);
        epi_backward<1, 1>(acc, 32 * fb, sb, hl, PL, lane);
    }
}

// Loss inputs of the block's samples into s_in [R][kInW]: TPS = NT / R
// threads per sample, each loading columns part, part + TPS, ... of the
// actions and collection-time means and one of the four per-sample scalars
// (log-probability and advantage for the actor, return and old value for the
// critic).  load() only issues the loads; store() writes them to LDS.
template <int R, int NT>
struct LossInputs {
    static constexpr int TPS = NT / R;
    float v[2 * (kFusedMaxAct / TPS) + 1];
    __device__ __forceinline__ void load(const FusedArgs &a, const int *s_rows, int net, int tid) {
        const int i = tid / TPS, part = tid - (tid / TPS) * TPS;
        const int A = a.A;
        const long long row = s_rows[i];
#pragma unroll
        for (int u = 0; u < kFusedMaxAct / TPS; ++u) {
            const int j = part + TPS * u;
            v[2 * u] = net == 0 && j < A ? a.actions[row * A + j] : 0.0f;
            v[2 * u + 1] = net == 0 && j < A && a.mu_old ? a.mu_old[row * A + j] : 0.0f;
        }
        const float *sc = part == 0 ? a.logp_old : part == 1 ? a.adv : part == 2 ? a.returns : a.values_old;
        const bool want = part < 4 && (part < 2 ? net == 0 : net == 1) && (part != 3 || a.clip_value);
        v[2 * (kFusedMaxAct / TPS)] = want ? sc[row] : 0.0f;
    }
    __device__ __forceinline__ void store(float *s_in, int tid) const {
        const int i = tid / TPS, part = tid - (tid / TPS) * TPS;
#pragma unroll
        for (int u = 0; u < kFusedMaxAct / TPS; ++u) {
            const int j = part + TPS * u;
            s_in[i * kInW + j] = v[2 * u];
            s_in[i * kInW + kFusedMaxAct + j] = v[2 * u + 1];
        }
        if (part < 4) s_in[i * kInW + 2 * kFusedMaxAct + part] = v[2 * (kFusedMaxAct / TPS)];
    }
};

// The first two hidden layers with the first one's output in chunks of
// chunk0 features (one feature block per wave): each chunk goes through
// ELU into the chunk buffer, is copied to global memory (a weight-gradient
// operand) while the second layer's fragments for its k-range are in
// flight, and is added into the second layer's accumulators, which stay in
// registers across the chunks; then the second layer's epilogue writes h_1 at
// the region's start, over the inputs and the chunk buffer.  The actor's
// gathered inputs go to global memory during the first chunk.
template <int R, int NT, int WPE, int SPLIT, int FBW1>
__device__ __forceinline__ void stream_first_layers(const FusedArgs &a, const FusedNet &N, int net, const uint16_t *x,
                                                    int xp, char *reg, const float *s_bias, int m0, int rows,
                                                    int wave, int lane) {
    constexpr int SB = R / 32;
    const int H0 = a.H[0], H1 = a.H[1], C0 = a.chunk0;
    const int S0 = a.kpad >> 4, S1 = H0 >> 4;
    uint16_t *cb = reinterpret_cast<uint16_t *>(reg + a.lds_cb);
    const int cbp = C0 + 8;
    const int f1 = wave * FBW1 * 32;
    floatx16 acc1[FBW1][SB];
    for (int c0 = 0; c0 < H0; c0 += C0) {
        {
            floatx16 acc0[1][SB];
            auto hook0 = [&]() {
                if (c0 == 0 && net == 0)
                    copy_out<NT>(x, xp, a.xg + static_cast<long long>(m0) * a.kpad, a.kpad, a.kpad, rows);
            };
            mma_layer<1, SB, 4, SPLIT>(acc0, N.W[0] + static_cast<long long>(c0 / 32) * S0 * SPLIT * 512, C0, S0,
                                       32 * wave, 0, x, xp, lane, hook0);
            epi_forward<1, SB>(acc0, s_bias + a.bias_off[0] + c0, 32 * wave, 0, cb, cbp, lane);
        }
        __syncthreads();
        auto hook1 = [&]() { copy_out<NT>(cb, cbp, N.h[0] + static_cast<long long>(m0) * H0 + c0, H0, C0, rows); };
        mma_layer<FBW1, SB, 4, SPLIT>(acc1, N.W[1], H1, S1, f1, 0, cb, cbp, lane, hook1, c0 >> 4, C0 >> 4, c0 == 0);
        // every wave has read the chunk before the next one overwrites it
        __syncthreads();
    }
    epi_forward<FBW1, SB>(acc1, s_bias + a.bias_off[1], f1, 0, reinterpret_cast<uint16_t *>(reg), H1 + 8, lane);
    __syncthreads();
}

// R samples per workgroup of NT threads; WPE waves per SIMD (the NT / 256
// waves of one workgroup times the workgroups that share a CU).
//
// LDS: one activation region shared by all layers (offsets from
// fused_update_layout) plus the loss inputs, the hidden biases and the row
// indices.  A hidden layer's output stays in the accumulators until every
// wave has read the layer's input, then overwrites it; only the last hidden
// layer's output goes elsewhere (it is the input of the head).  The
// backward pass multiplies by ELU' of activations the forward pass already
// copied to global memory (they are weight-gradient operands): each is
// staged back into the region next to the incoming gradient, and the
// gradient of the first hidden layer, which nothing else consumes, is
// computed a feature chunk at a time and copied out.  The region then needs
// room for about one wide layer rather than all of them, which lets 64
// samples (or 32 of a 1024-wide network) share a CU two workgroups at a time.
template <int R, int NT, int WPE, bool STREAM = false>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WPE, WPE)))
void fused_update_kernel(const FusedArgs a) {
    extern __shared__ __attribute__((aligned(16))) char lds[];
    int net, sblk;
    if (!net_block(static_cast<int>(blockIdx.x), a.blocks, net, sblk)) return;
    const int m0 = sblk * R;
    const int rows = min(R, a.M - m0);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int L = a.L, A = a.A;
    const int Hl = a.H[L - 1];
    const int n_out = net == 0 ? A : 1;
    const int WP = Hl + 4;                 // row pitch of the staged output-layer weights
    char *reg = lds;                       // the shared activation region at offset 0
    float *s_in = reinterpret_cast<float *>(lds + a.lds_in);      // [R][kInW] per-sample loss inputs
    float *s_bias = reinterpret_cast<float *>(lds + a.lds_bias);  // hidden-layer biases
    int *s_rows = reinterpret_cast<int *>(lds + a.lds_rows);      // [R] batch rows of the block
    float *s_head = reinterpret_cast<float *>(lds + a.lds_head);  // output biases [n_out], log-std [A]
    const FusedNet &N = a.net[net];

    // ------------------------------------------------------- prologue
    // batch rows of the block (rows past the end repeat the last one; their
    // results are discarded), then the hidden biases, output bias and log-std
    // in one round of buffer loads, then the observations and loss inputs
    if (tid < R) {
        int r = m0 + min(tid, rows - 1);
        if (a.idx) r = min(max(a.idx[r], 0), a.B - 1);
        s_rows[tid] = r;
    }
    {
        // hidden biases: one 16-byte load per thread and layer (the biases
        // are 16-byte aligned and at most 4 NT wide)
        u32x4 vb[kMaxHidden];
#pragma unroll
        for (int l = 0; l < kMaxHidden; ++l) {
            const int H = l < L ? a.H[l] : 0;
            const __amdgpu_buffer_rsrc_t rb = make_rsrc(N.bias[l], static_cast<long long>(H) * 4);
            vb[l] = __builtin_amdgcn_raw_buffer_load_b128(rb, 4 * tid < H ? tid * 16 : kOutside, 0, 0);
        }
        const __amdgpu_buffer_rsrc_t ro = make_rsrc(N.bout, static_cast<long long>(n_out) * 4);
        const __amdgpu_buffer_rsrc_t rl = make_rsrc(a.logstd, static_cast<long long>(A) * 4);
        const float vo = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(ro, tid < n_out ? tid * 4 : kOutside, 0, 0));
        const float vl = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rl, tid < A ? tid * 4 : kOutside, 0, 0));
#pragma unroll
        for (int l = 0; l < kMaxHidden; ++l)
            if (l < L && 4 * tid < a.H[l]) *reinterpret_cast<u32x4 *>(s_bias + a.bias_off[l] + 4 * tid) = vb[l];
        if (tid < kFusedMaxAct) {
            s_head[tid] = tid < n_out ? vo : 0.0f;
            s_head[kFusedMaxAct + tid] = tid < A ? vl : 0.0f;
        }
    }
    __syncthreads();
    uint16_t *x = reinterpret_cast<uint16_t *>(reg);
    const int xp = a.kpad + 8;
    {
        // the loss inputs in the same round as the observation rows, unless
        // the LDS plan defers them (their place is in use until the streamed
        // pair is done: they load during the next layer's MMA loop, or before
        // the head when no layer follows the pair)
        LossInputs<R, NT> li;
        if (!a.defer_in) li.load(a, s_rows, net, tid);
        gather_rows<R, NT>(a, s_rows, rows, x, xp, wave, lane);
        if (!a.defer_in) li.store(s_in, tid);
    }
    __syncthreads();

    // --------------------------------------------------------- forward
    // hidden layers 0 .. L-2 write their output over their input (at the
    // region's start) once every wave has read it; the last goes to
    // lds_last (over its input too when that is the region's start).  Each
    // layer's input goes to global memory while its first weight fragments
    // are in flight (the gathered observations: actor only).  STREAM: the
    // first two layers as stream_first_layers computes them.
    {
        const uint16_t *in = x;
        int in_pitch = xp, K = a.kpad;
        int l0 = 0;
        if constexpr (STREAM) {
            const bool two = a.H[1] / 32 / (NT / 64) == 2;
            if (net == 1) {
                if (two) stream_first_layers<R, NT, WPE, 2, 2>(a, N, net, x, xp, reg, s_bias, m0, rows, wave, lane);
                else stream_first_layers<R, NT, WPE, 2, 1>(a, N, net, x, xp, reg, s_bias, m0, rows, wave, lane);
            } else {
                if (two) stream_first_layers<R, NT, WPE, 1, 2>(a, N, net, x, xp, reg, s_bias, m0, rows, wave, lane);
                else stream_first_layers<R, NT, WPE, 1, 1>(a, N, net, x, xp, reg, s_bias, m0, rows, wave, lane);
            }
            in = reinterpret_cast<const uint16_t *>(reg);
            in_pitch = a.H[1] + 8;
            K = a.H[1];
            l0 = 2;
        }
        for (int l = l0; l < L; ++l) {
            const int H = a.H[l];
            const bool last = l == L - 1;
            uint16_t *out = reinterpret_cast<uint16_t *>(reg + (last ? a.lds_last : 0));
            const int sync = !last || a.lds_last == 0 ? 1 : 0;
            const int Hp = l > 0 ? a.H[l - 1] : 0;
            auto hook = [&]() {
                if (l == 0) {
                    if (net == 0)
                        copy_out<NT>(x, xp, a.xg + static_cast<long long>(m0) * a.kpad, a.kpad, a.kpad, rows);
                } else {
                    copy_out<NT>(in, Hp + 8, N.h[l - 1] + static_cast<long long>(m0) * Hp, Hp, Hp, rows);
                }
                if (a.defer_in && l == l0 && l0 > 0) {
                    LossInputs<R, NT> li;
                    li.load(a, s_rows, net, tid);
                    li.store(s_in, tid);
                }
            };
            // the critic's weights come in the split layout (bf16 and residual fragments)
            if (net == 1)
                run_layer<R, NT, WPE, false, 2>(N.W[l], K, H, s_bias + a.bias_off[l], in, in_pitch, out, H + 8,
                                                wave, lane, hook, sync);
            else
                run_layer<R, NT, WPE, false, 1>(N.W[l], K, H, s_bias + a.bias_off[l], in, in_pitch, out, H + 8,
                                                wave, lane, hook, sync);
            __syncthreads();
            in = out;
            in_pitch = H + 8;
            K = H;
        }
    }
    uint16_t *hl = reinterpret_cast<uint16_t *>(reg + a.lds_last);
    const int PL = Hl + 8;
    // the last hidden layer to global memory; the output-layer weights into
    // the region's start (free once the last layer has read its input)
    float *w_out = reinterpret_cast<float *>(reg + a.lds_w);
    float *s_sum = reinterpret_cast<float *>(reg + a.lds_sum);   // [R][kSums] per-sample loss terms
    {
        if (a.defer_in && L == 2) {
            // deferred loss inputs with no layer after the streamed pair to hide them
            LossInputs<R, NT> li;
            li.load(a, s_rows, net, tid);
            li.store(s_in, tid);
        }
        constexpr int UW = 4;   // 4-element chunks (16-byte loads) of the output-layer weights per thread
        const int nw = n_out * Hl;
        const __amdgpu_buffer_rsrc_t rw = make_rsrc(N.Wout, static_cast<long long>(nw) * 4);
        u32x4 vw[UW];
#pragma unroll
        for (int u = 0; u < UW; ++u) {
            const int q4 = tid + u * NT;
            vw[u] = __builtin_amdgcn_raw_buffer_load_b128(rw, 4 * q4 < nw ? q4 * 16 : kOutside, 0, 0);
        }
        copy_out<NT>(hl, PL, N.h[L - 1] + static_cast<long long>(m0) * Hl, Hl, Hl, rows);
#pragma unroll
        for (int u = 0; u < UW; ++u) {
            const int q = 4 * (tid + u * NT);
            const int j = q / Hl;
            if (q < nw) *reinterpret_cast<u32x4 *>(w_out + j * WP + (q - j * Hl)) = vw[u];
        }
        // zero rows of the output-layer weights past n_out (read by the
        // actor's kFusedMaxAct-wide head)
        for (int q = nw + tid; q < kFusedMaxAct * Hl; q += NT) {
            const int j = q / Hl;
            w_out[j * WP + (q - j * Hl)] = 0.0f;
        }
        // output layers wider than 4 UW elements per thread (not the paper's shapes)
        for (int q = tid + 4 * UW * NT; q < nw; q += NT) {
            const int j = q / Hl;
            w_out[j * WP + (q - j * Hl)] = N.Wout[q];
        }
    }
    __syncthreads();

    // ----------------------------------------- output layer and PPO loss
    float *s_g = reinterpret_cast<float *>(reg + a.lds_g);       // [R][kFusedMaxAct] output gradients
    // the actor's 12-16 outputs on MFMA; the critic's single output on VALU
    // dot products (KP lanes per sample), which is the shorter of the two
    constexpr int KP = NT / R;
    if (net == 0) {
        head_mfma<R, NT, true>(a, N, hl, PL, w_out, WP, s_head, s_in, s_sum, s_g, m0, rows, wave, lane);
    } else {
        switch ((Hl / KP) / 8) {
        case 2: head_pass<R, NT, 2, false>(a, N, hl, PL, w_out, WP, s_head, s_in, s_sum, m0, rows); break;
        case 4: head_pass<R, NT, 4, false>(a, N, hl, PL, w_out, WP, s_head, s_in, s_sum, m0, rows); break;
        default: head_pass<R, NT, 8, false>(a, N, hl, PL, w_out, WP, s_head, s_in, s_sum, m0, rows); break;
        }
    }
    __syncthreads();
    // block sums of the loss terms: eight lanes per term, lane p adding the
    // samples p, p + 8, ... in order, then a fixed three-level lane tree;
    // each term's first lane writes its slot of the block's partials row
    // (shared by the block's actor and critic workgroups, which write
    // disjoint slots).  The order is fixed, so the result does not depend
    // on timing.
    {
        float *out = a.partials + static_cast<long long>(m0 / R) * (A + 8);
        const int q = tid >> 3, p = tid & 7;
        float v = 0.0f;
        if (q < kSums) {
            float t8[R / 8];
#pragma unroll
            for (int u = 0; u < R / 8; ++u) t8[u] = s_sum[min(p + 8 * u, R - 1) * kSums + q];
#pragma unroll
            for (int u = 0; u < R / 8; ++u)
                if (p + 8 * u < rows) v += t8[u];
        }
        // the 8 lanes of a term are adjacent lanes of one wave
        v += __shfl_xor(v, 1);
        v += __shfl_xor(v, 2);
        v += __shfl_xor(v, 4);
        if (q < kSums && p == 0) {
            if (net == 0) {
                if (q == 0 || q == 2 || q == 3) out[q] = v;
                else if (q == 4) out[5 + A] = v;
                else if (q >= 5 && q - 5 < A) out[4 + (q - 5)] = v;
            } else if (q == 1) {
                out[1] = v;
            }
        }
        if (net == 0 && tid == 0) {
            float ent = 0.0f, kl_ls = 0.0f;
            if (m0 == 0) {
                // entropy of the state-independent policy, and the
                // sample-independent part of KL(pi_old || pi):
                //   sum_j log(sigma / sigma_old) + sigma_old^2 / (2 sigma^2) - 1/2
                ent = 0.5f * A * (1.0f + kLog2Pi);
                for (int j = 0; j < A; ++j) ent += a.logstd[j];
                if (a.mu_old)
                    for (int j = 0; j < A; ++j) {
                        const float d = a.logstd_old[j] - a.logstd[j];
                        kl_ls += -d + 0.5f * expf(2.0f * d) - 0.5f;
                    }
            }
            out[4 + A] = ent;
            out[6 + A] = kl_ls;
        }
    }
    if (a.no_backward) return;
    // every lane has read its block sums before the staging below reuses
    // their place
    __syncthreads();

    // ------------------------------------------------ input-gradient chain
    // layer l multiplies dz_l (at lds_bdz[l]) by W_l and by ELU' of h_{l-1},
    // which is staged back from global memory at lds_bst[l] during the
    // layer's MMA loop (LDS-direct loads issued while its first weight
    // fragments are in flight, waited for before the epilogue) and
    // overwritten in place by dz_{l-1}; dz_l goes to global memory at the same
    // point.  The first hidden layer's gradient is computed `chunk` features
    // at a time and copied out.
    for (int l = L - 1; l >= 1; --l) {
        const int Hin = a.H[l], Hout = a.H[l - 1];
        const uint16_t *dz = reinterpret_cast<const uint16_t *>(reg + a.lds_bdz[l]);
        uint16_t *st = reinterpret_cast<uint16_t *>(reg + a.lds_bst[l]);
        const int C = l == 1 ? a.chunk : Hout;
        const int S = Hin / 16;
        for (int c0 = 0; c0 < Hout; c0 += C) {
            auto hook = [&]() {
                copy_in_async<NT>(N.h[l - 1] + static_cast<long long>(m0) * Hout + c0, Hout, st, C + 8, C, rows, R,
                                  wave, lane);
                if (c0 == 0) copy_out<NT>(dz, Hin + 8, N.dz[l] + static_cast<long long>(m0) * Hin, Hin, Hin, rows);
            };
            run_layer<R, NT, WPE, true, 1>(N.WT[l] + static_cast<long long>(c0 / 32) * S * 512, Hin, C, nullptr,
                                           dz, Hin + 8, st, C + 8, wave, lane, hook, 2);
            __syncthreads();
            if (l == 1) {
                copy_out<NT>(st, C + 8, N.dz[0] + static_cast<long long>(m0) * Hout + c0, Hout, C, rows);
                __syncthreads();
            }
        }
    }
    if (L == 1) {
        // one hidden layer: its gradient is the head's output, in place over h_0
        copy_out<NT>(hl, PL, N.dz[0] + static_cast<long long>(m0) * Hl, Hl, Hl, rows);
    }
}

// Weights in MFMA A-fragment order.  For a matrix with `rows` output
// features and K inputs (zero-padded to 16 S), fragment (fb, s) holds, for
// lane l, the 8 elements W[32 fb + l % 32][16 s + 8 (l / 32) .. + 7]; fragment
// (fb, s) starts at element ((fb * S + s) * 64) * 8.  transpose = 1 packs
// W^T from the row-major W: element (r, k) = src[k * ld + r].  split = 1
// reads float32 W and stores 2 S fragments per feature block fb: fragment
// ((2 fb + part) * S + s) holds bf16(W) for part 0 and the bf16 residual
// bf16(W - bf16(W)) for part 1 (the subtraction is exact in float32).
__global__ __launch_bounds__(256) void pack_frags_kernel(const FragArgs a) {
    const int t = blockIdx.x * 256 + threadIdx.x;   // one 8-element lane chunk per thread
    if (t >= a.total) return;
    int j = 0;
#pragma unroll 1
    for (int q = 1; q < a.count; ++q)
        if (t >= a.job[q].begin) j = q;
    // jobs cover whole multiples of 64 lane chunks, so a wave never straddles
    // two: the index is uniform and the descriptor comes through scalar loads
    j = __builtin_amdgcn_readfirstlane(j);
    const FragJob &J = a.job[j];
    const int local = t - J.begin;
    const int lane = local & 63;
    const int frag = local >> 6;
    const int fbp = frag / J.S, s = frag - (frag / J.S) * J.S;
    const int fb = J.split ? fbp >> 1 : fbp;
    const int part = J.split ? fbp & 1 : 0;
    const int r = 32 * fb + (lane & 31);
    const int k0 = 16 * s + 8 * (lane >> 5);
    uint32_t v[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        uint32_t lo = 0, hi = 0;
        const int k = k0 + 2 * e;
        if (J.split) {
            auto piece = [&](int kk) -> uint32_t {
                if (kk >= J.K) return 0u;
                const float x = J.src32[static_cast<long long>(r) * J.ld + kk];
                const uint16_t h = f32_to_bf16(x);
                return part == 0 ? h : f32_to_bf16(x - bf16_to_f32(h));
            };
            lo = piece(k);
            hi = piece(k + 1);
        } else if (J.transpose) {
            if (k < J.K) lo = J.src[static_cast<long long>(k) * J.ld + r];
            if (k + 1 < J.K) hi = J.src[static_cast<long long>(k + 1) * J.ld + r];
        } else {
            if (k < J.K) lo = J.src[static_cast<long long>(r) * J.ld + k];
            if (k + 1 < J.K) hi = J.src[static_cast<long long>(r) * J.ld + k + 1];
        }
        v[e] = lo | (hi << 16);
    }
    *reinterpret_cast<u32x4 *>(J.dst + static_cast<long long>(local) * 8) = u32x4{v[0], v[1], v[2], v[3]};
}

// Rollout inference for R environments of one network per workgroup: the
// observation rows, every hidden layer with the activations in LDS, the
// output layer, then for the actor the diagonal-Gaussian action
// a = mu + sigma eps with Philox noise (counter (n * groups + g, t,
// iteration, 1) for the g-th group of four actions of environment n, two
// Box-Muller pairs per draw) and its log-density
// sum_j (-eps_j^2 / 2 - log sigma_j) - (A / 2) log(2 pi); for the critic the
// value.  Same draws, formulas and float64 log-density as the
// layer-by-layer sampling kernel; only the output layer's summation order
// differs.
template <int R, int NT, int WPE>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WPE, WPE)))
void fused_infer_kernel(const FusedArgs a) {
    extern __shared__ __attribute__((aligned(16))) char lds[];
    constexpr int KP = NT / R;
    const bool both = a.net_mask == 3;
    int net = a.net_mask == 1 ? 0 : 1, sblk = static_cast<int>(blockIdx.x);
    if (both && !net_block(static_cast<int>(blockIdx.x), a.blocks, net, sblk)) return;
    const int m0 = sblk * R;
    const int rows = min(R, a.M - m0);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int L = a.L, A = a.A;
    const int Hl = a.H[L - 1];
    const int n_out = net == 0 ? A : 1;
    const int WP = Hl + 4;
    float *w_out = reinterpret_cast<float *>(lds + a.lds_w);
    float *s_bias = reinterpret_cast<float *>(lds + a.lds_bias);
    float *s_head = reinterpret_cast<float *>(lds + a.lds_head);
    const FusedNet &N = a.net[net];
    uint16_t *x = reinterpret_cast<uint16_t *>(lds + a.lds_x);
    const int xp = a.kpad + 8;
    {
        // output-layer weights, output biases, log-std and hidden biases in one
        // round of buffer loads, then the LDS stores (as in the update pass)
        // 16-byte loads: the output-layer weights and the hidden biases are
        // 16-byte aligned, rows of a multiple of 32 elements
        constexpr int UW = 4;   // 4-element chunks of the output-layer weights per thread
        const int nw = n_out * Hl;
        const __amdgpu_buffer_rsrc_t rw = make_rsrc(N.Wout, static_cast<long long>(nw) * 4);
        u32x4 vw[UW], vb[kMaxHidden];
#pragma unroll
        for (int u = 0; u < UW; ++u) {
            const int q4 = tid + u * NT;
            vw[u] = __builtin_amdgcn_raw_buffer_load_b128(rw, 4 * q4 < nw ? q4 * 16 : kOutside, 0, 0);
        }
#pragma unroll
        for (int l = 0; l < kMaxHidden; ++l) {
            const int H = l < L ? a.H[l] : 0;
            const __amdgpu_buffer_rsrc_t rb = make_rsrc(N.bias[l], static_cast<long long>(H) * 4);
            vb[l] = __builtin_amdgcn_raw_buffer_load_b128(rb, 4 * tid < H ? tid * 16 : kOutside, 0, 0);
        }
        const __amdgpu_buffer_rsrc_t ro = make_rsrc(N.bout, static_cast<long long>(n_out) * 4);
        const __amdgpu_buffer_rsrc_t rl = make_rsrc(a.logstd, static_cast<long long>(A) * 4);
        const float vo = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(ro, tid < n_out ? tid * 4 : kOutside, 0, 0));
        const float vl = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rl, tid < A ? tid * 4 : kOutside, 0, 0));
        // the observation rows are the block's own (no index list): their loads
        // go out behind the weight loads, so the prologue waits for memory once
        gather_rows<R, NT>(a, nullptr, rows, x, xp, wave, lane, m0);
#pragma unroll
        for (int u = 0; u < UW; ++u) {
            const int q = 4 * (tid + u * NT);
            const int j = q / Hl;
            if (q < nw) *reinterpret_cast<u32x4 *>(w_out + j * WP + (q - j * Hl)) = vw[u];
        }
#pragma unroll
        for (int l = 0; l < kMaxHidden; ++l)
            if (l < L && 4 * tid < a.H[l]) *reinterpret_cast<u32x4 *>(s_bias + a.bias_off[l] + 4 * tid) = vb[l];
        if (tid < kFusedMaxAct) {
            s_head[tid] = tid < n_out ? vo : 0.0f;
            s_head[kFusedMaxAct + tid] = tid < A ? vl : 0.0f;
        }
        for (int q = nw + tid; q < kFusedMaxAct * Hl; q += NT) {
            const int j = q / Hl;
            w_out[j * WP + (q - j * Hl)] = 0.0f;
        }
        for (int q = tid + 4 * UW * NT; q < nw; q += NT) {
            const int j = q / Hl;
            w_out[j * WP + (q - j * Hl)] = N.Wout[q];
        }
    }
    __syncthreads();

    const uint16_t *in = x;
    int in_pitch = xp, K = a.kpad;
    for (int l = 0; l < L; ++l) {
        const int H = a.H[l];
        uint16_t *out = reinterpret_cast<uint16_t *>(lds + a.lds_region[l]);
        if (net == 1)
            run_layer<R, NT, WPE, false, 2>(N.W[l], K, H, s_bias + a.bias_off[l], in, in_pitch, out, H + 8, wave,
                                            lane);
        else
            run_layer<R, NT, WPE, false, 1>(N.W[l], K, H, s_bias + a.bias_off[l], in, in_pitch, out, H + 8, wave,
                                            lane);
        __syncthreads();
        in = out;
        in_pitch = H + 8;
        K = H;
    }

    const uint16_t *hl = reinterpret_cast<const uint16_t *>(lds + a.lds_region[L - 1]);
    const int si = tid / KP, kq = tid % KP;
    const bool lead = si < rows && kq == 0;
    const int n = m0 + si;
    const int nck = (Hl / KP) / 8;
    const uint16_t *hrow = hl + si * (Hl + 8) + kq * (Hl / KP);
    const float *wl = w_out + kq * (Hl / KP);
    if (net == 1) {
        float o[1];
        if (nck == 2) { u32x4 hx[2]; head_dots<KP, 2, 1>(hrow, wl, WP, s_head, hx, o); }
        else if (nck == 4) { u32x4 hx[4]; head_dots<KP, 4, 1>(hrow, wl, WP, s_head, hx, o); }
        else { u32x4 hx[8]; head_dots<KP, 8, 1>(hrow, wl, WP, s_head, hx, o); }
        if (lead && a.val_out) a.val_out[n] = o[0];
        return;
    }
    // outputs past A are zero: 12 of them suffice when A <= 12
    float o[kFusedMaxAct];
#pragma unroll
    for (int j = 0; j < kFusedMaxAct; ++j) o[j] = 0.0f;
    if (A <= 12) {
        float o12[12];
        if (nck == 2) { u32x4 hx[2]; head_dots<KP, 2, 12>(hrow, wl, WP, s_head, hx, o12); }
        else if (nck == 4) { u32x4 hx[4]; head_dots<KP, 4, 12>(hrow, wl, WP, s_head, hx, o12); }
        else { u32x4 hx[8]; head_dots<KP, 8, 12>(hrow, wl, WP, s_head, hx, o12); }
#pragma unroll
        for (int j = 0; j < 12; ++j) o[j] = o12[j];
    } else {
        if (nck == 2) { u32x4 hx[2]; head_dots<KP, 2, kFusedMaxAct>(hrow, wl, WP, s_head, hx, o); }
        else if (nck == 4) { u32x4 hx[4]; head_dots<KP, 4, kFusedMaxAct>(hrow, wl, WP, s_head, hx, o); }
        else { u32x4 hx[8]; head_dots<KP, 8, kFusedMaxAct>(hrow, wl, WP, s_head, hx, o); }
    }
    // lane kq of a sample draws action group kq (KP >= 4 lanes per sample,
    // at most 4 groups); every lane holds all the sample's means
    const int groups = (A + 3) / 4;
    const bool draws = si < rows && kq < groups;
    float eps[4];
    {
        uint32_t c[4] = {static_cast<uint32_t>(n) * groups + kq, a.t_step, a.iteration, 1u};
        philox4x32_10(c, a.key0, a.key1);
        box_muller(c[0], c[1], eps[0], eps[1]);
        box_muller(c[2], c[3], eps[2], eps[3]);
    }
    float act4[4], mu4[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        float m = o[q];
#pragma unroll
        for (int g = 1; g < kFusedMaxAct / 4; ++g) m = kq == g ? o[4 * g + q] : m;
        const int j = 4 * kq + q;
        mu4[q] = m;
        act4[q] = m + expf(s_head[kFusedMaxAct + min(j, kFusedMaxAct - 1)]) * eps[q];
    }
    if (a.vec_out) {
        // the lane's group of four actions and means, one 16-byte store each
        if (draws) {
            const long long e = static_cast<long long>(n) * A + 4 * kq;
            if (a.act_out) *reinterpret_cast<float4 *>(a.act_out + e) = make_float4(act4[0], act4[1], act4[2], act4[3]);
            if (a.mu_out) *reinterpret_cast<float4 *>(a.mu_out + e) = make_float4(mu4[0], mu4[1], mu4[2], mu4[3]);
        }
    } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int j = 4 * kq + q;
            if (draws && j < A) {
                if (a.act_out) a.act_out[static_cast<long long>(n) * A + j] = act4[q];
                if (a.mu_out) a.mu_out[static_cast<long long>(n) * A + j] = mu4[q];
            }
        }
    }
    // the lead lane sums the log-density over the actions in order
    float e_all[kFusedMaxAct];
#pragma unroll
    for (int g = 0; g < kFusedMaxAct / 4; ++g)
#pragma unroll
        for (int q = 0; q < 4; ++q) e_all[4 * g + q] = g == 0 ? eps[q] : __shfl(eps[q], lane + g);
    if (!lead || !a.logp_out) return;
    CompSum lp;
#pragma unroll
    for (int j = 0; j < kFusedMaxAct; ++j)
        if (j < A) lp.add_gauss(e_all[j], s_head[kFusedMaxAct + j]);
    a.logp_out[n] = lp.value();
}

size_t align16(size_t v) { return (v + 15) & ~static_cast<size_t>(15); }

// Grid size for both networks over `blocks` sample blocks (see net_block).
int two_net_grid(int blocks) { return 2 * ((blocks + 7) / 8) * 8; }

// LDS layout for R rows; returns the total bytes (0 if a constraint fails).
size_t fused_layout(int L, const int *H, int kpad, int A, int R, int NT, FusedArgs *a) {
    const int KP = NT / R;
    const int Hl = H[L - 1];
    if (Hl % KP != 0 || (Hl / KP != 16 && Hl / KP != 32 && Hl / KP != 64)) return 0;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const int at = static_cast<int>(off);
        off += align16(bytes);
        return at;
    };
    const int lds_w = take(static_cast<size_t>(kFusedMaxAct) * (Hl + 4) * 4);
    const int lds_sum = take(static_cast<size_t>(R + 1) * kSums * 4);
    const int lds_in = take(static_cast<size_t>(R) * kInW * 4);
    const int lds_rows = take(static_cast<size_t>(R) * 4);
    const int lds_head = take(static_cast<size_t>(2 * kFusedMaxAct) * 4);
    int bias_off[kMaxHidden] = {0};
    size_t nb = 0;
    for (int l = 0; l < L; ++l) {
        bias_off[l] = static_cast<int>(nb);
        nb += (H[l] + 3) & ~3;
    }
    const int lds_bias = take(nb * 4);
    int region[kMaxHidden] = {0};
    for (int l = 0; l < L; ++l) region[l] = take(static_cast<size_t>(R) * (H[l] + 8) * 2);
    int lds_x;
    if (L >= 2 && kpad <= H[1])
        lds_x = region[1];   // the inputs are dead once the first layer has run
    else
        lds_x = take(static_cast<size_t>(R) * (kpad + 8) * 2);
    if (off > static_cast<size_t>(kMaxLdsBytes)) return 0;
    if (a) {
        a->lds_w = lds_w;
        a->lds_sum = lds_sum;
        a->lds_in = lds_in;
        a->lds_rows = lds_rows;
        a->lds_head = lds_head;
        a->lds_bias = lds_bias;
        a->lds_x = lds_x;
        for (int l = 0; l < L; ++l) {
            a->lds_region[l] = region[l];
            a->bias_off[l] = bias_off[l];
        }
    }
    return off;
}

// Whether R rows per workgroup of NT threads cover this network: every
// layer width splits over the waves as run_layer does, the output layer's
// per-lane slice is 16 to 64 activations, and the LDS layout fits (in half
// of it for two workgroups per CU).
bool fused_fits(int L, const int *H, int kpad, int A, int R, int NT, bool two_per_cu) {
    const int NW = NT / 64, SB = R / 32;
    const bool wide_ok = SB == 1 && NT == 256 && !two_per_cu;   // the WIDE case of run_layer
    for (int l = 0; l < L; ++l) {
        const int fb = H[l] / 32;
        if (H[l] % 32 != 0) return false;
        if (fb >= NW) {
            const int fbw = fb / NW;
            if (fb % NW != 0 || (fbw != 1 && fbw != 2 && fbw != 4 && !(fbw == 8 && wide_ok))) return false;
        } else if (!(SB >= 2 && 2 * fb == NW)) {
            return false;
        }
    }
    const size_t bytes = fused_layout(L, H, kpad, A, R, NT, nullptr);
    return bytes > 0 && bytes <= static_cast<size_t>(two_per_cu ? kMaxLdsBytes / 2 : kMaxLdsBytes);
}

// Whether `width` output features split over the waves as run_layer does.
bool width_splits(int width, int NW, int SB, bool wide_ok, int regs = 320) {
    if (width <= 0 || width % 32 != 0) return false;
    const int fb = width / 32;
    if (fb >= NW) {
        const int fbw = fb / NW;
        return fb % NW == 0 && acc_fits(fbw, SB, regs) && (fbw == 1 || fbw == 2 || fbw == 4 || (fbw == 8 && wide_ok));
    }
    return SB >= 2 && 2 * fb == NW;
}

// LDS plan of the update pass for R rows (see fused_update_kernel) within
// `budget` bytes: the shared activation region (the gathered inputs and each
// hidden layer's output at its start, the last hidden layer's output after
// its input, the output-layer weights and loss terms wherever they fit during
// the head, and per backward layer the incoming gradient next to the staged
// activation), then the loss inputs, hidden biases, row indices and head
// constants.  The first hidden layer's gradient is computed in the widest
// feature chunk that fits.  Returns the total bytes, 0 if nothing fits.
size_t fused_update_layout(int L, const int *H, int kpad, int A, int R, int NT, size_t budget, FusedArgs *a) {
    (void)A;
    const int Hl = H[L - 1];
    const int NW = NT / 64, SB = R / 32;
    // the critic's output layer: KP = NT / R lanes per sample, 16 to 64 activations each
    const int KP = NT / R;
    if (Hl % KP != 0 || (Hl / KP != 16 && Hl / KP != 32 && Hl / KP != 64)) return 0;
    const bool wide_ok = SB == 1 && NT == 256 && budget >= static_cast<size_t>(kMaxLdsBytes);
    for (int l = 0; l < L; ++l)
        if (!width_splits(H[l], NW, SB, wide_ok)) return 0;
    auto P = [&](int w) { return align16(static_cast<size_t>(R) * (w + 8) * 2); };
    size_t fixed = 0;
    auto take = [&](size_t bytes) {
        const size_t at = fixed;
        fixed += align16(bytes);
        return at;
    };
    const size_t in_off = take(static_cast<size_t>(R) * kInW * 4);
    int bias_off[kMaxHidden] = {0};
    size_t nb = 0;
    for (int l = 0; l < L; ++l) {
        bias_off[l] = static_cast<int>(nb);
        nb += (H[l] + 3) & ~3;
    }
    const size_t bias = take(nb * 4);
    const size_t rows_off = take(static_cast<size_t>(R) * 4);
    const size_t head = take(static_cast<size_t>(2 * kFusedMaxAct) * 4);
    const int H0 = H[0];
    for (int C = H0; C >= 32; C /= 2) {
        if (H0 % C != 0 || (L >= 2 && !width_splits(C, NW, SB, wide_ok))) continue;
        size_t ext = P(kpad);
        for (int l = 0; l + 1 < L; ++l) ext = std::max(ext, P(H[l]));
        const size_t last = L >= 2 ? P(H[L - 2]) : P(kpad);
        ext = std::max(ext, last + P(Hl));
        const size_t wb = align16(static_cast<size_t>(kFusedMaxAct) * (Hl + 4) * 4);
        const size_t sb = align16(static_cast<size_t>(R + 1) * kSums * 4);
        const size_t gb = align16(static_cast<size_t>(R) * kFusedMaxAct * 4);
        size_t w_off = 0, s_off = wb, g_off = wb + sb;
        if (wb + sb + gb > last) {
            w_off = last + P(Hl);
            s_off = w_off + wb;
            g_off = s_off + sb;
            ext = std::max(ext, g_off + gb);
        }
        size_t bdz[kMaxHidden] = {0}, bst[kMaxHidden] = {0};
        size_t cur = last;
        for (int l = L - 1; l >= 1; --l) {
            const int Cl = l == 1 ? C : H[l - 1];
            const size_t dz_size = P(H[l]), st_size = P(Cl);
            const size_t st = cur >= st_size ? 0 : cur + dz_size;
            ext = std::max(ext, st + st_size);
            bdz[l] = cur;
            bst[l] = st;
            cur = st;
        }
        ext = align16(ext);
        const size_t total = ext + fixed;
        if (total > budget) continue;
        if (a) {
            a->lds_in = static_cast<int>(ext + in_off);
            a->lds_bias = static_cast<int>(ext + bias);
            a->lds_rows = static_cast<int>(ext + rows_off);
            a->lds_head = static_cast<int>(ext + head);
            a->lds_last = static_cast<int>(last);
            a->lds_w = static_cast<int>(w_off);
            a->lds_sum = static_cast<int>(s_off);
            a->lds_g = static_cast<int>(g_off);
            a->chunk = C;
            for (int l = 0; l < L; ++l) {
                a->bias_off[l] = bias_off[l];
                a->lds_bdz[l] = static_cast<int>(bdz[l]);
                a->lds_bst[l] = static_cast<int>(bst[l]);
            }
        }
        return total;
    }
    return 0;
}

// LDS plan of the update pass with a streamed first layer (three workgroups
// per CU, `budget` bytes each): the first hidden layer's output is never held
// whole.  Forward: the gathered inputs at the region's start, followed by a
// chunk buffer of chunk0 = 32 NW features (one feature block per wave); the
// second layer's output at the start once every chunk has been added in,
// and each later layer's output over its input.  Head: the last hidden layer
// at the start, then the output-layer weights, the per-sample loss terms and
// the output gradients.  The loss inputs load during the first layer after
// the streamed pair (defer_in) into space that is free from then until the
// head: behind the head's areas and that layer's input and output.  The
// biases, row indices and head constants, needed from the prologue on, sit
// behind everything the forward pass uses.  The backward chain may overwrite
// all of these (none is read after the head): dz_{L-1} in place over h_{L-1}
// at the start, each staged ELU' input next to its incoming gradient, the
// first hidden layer's gradient in the widest chunk that fits.  Returns the
// total bytes, 0 if the network does not fit or does not split this way.
size_t fused_stream_layout(int L, const int *H, int kpad, int A, int R, int NT, size_t budget, FusedArgs *a) {
    (void)A;
    if (L < 2) return 0;
    const int Hl = H[L - 1];
    const int NW = NT / 64, SB = R / 32;
    const int regs = layer_regs(3, SB);
    const int KP = NT / R;
    if (Hl % KP != 0 || (Hl / KP != 16 && Hl / KP != 32 && Hl / KP != 64)) return 0;
    const int C0 = 32 * NW;
    // the first layer one feature block per wave per chunk; the second
    // layer's accumulators live across the chunks (at most two feature blocks)
    if (H[0] % C0 != 0 || H[1] % 32 != 0 || H[1] / 32 < NW || (H[1] / 32) % NW != 0 || H[1] / 32 / NW > 2)
        return 0;
    for (int l = 1; l < L; ++l)
        if (!width_splits(H[l], NW, SB, false, regs)) return 0;
    auto P = [&](int w) { return align16(static_cast<size_t>(R) * (w + 8) * 2); };
    size_t fixed = 0;
    auto take = [&](size_t bytes) {
        const size_t at = fixed;
        fixed += align16(bytes);
        return at;
    };
    int bias_off[kMaxHidden] = {0};
    size_t nb = 0;
    for (int l = 0; l < L; ++l) {
        bias_off[l] = static_cast<int>(nb);
        nb += (H[l] + 3) & ~3;
    }
    const size_t bias = take(nb * 4);
    const size_t rows_off = take(static_cast<size_t>(R) * 4);
    const size_t head = take(static_cast<size_t>(2 * kFusedMaxAct) * 4);
    size_t fwd = P(kpad) + P(C0);
    for (int l = 1; l < L; ++l) fwd = std::max(fwd, P(H[l]));
    const size_t wb = align16(static_cast<size_t>(kFusedMaxAct) * (Hl + 4) * 4);
    const size_t sbytes = align16(static_cast<size_t>(R + 1) * kSums * 4);
    const size_t gb = align16(static_cast<size_t>(R) * kFusedMaxAct * 4);
    const size_t w_off = P(Hl), s_off = w_off + wb, g_off = s_off + sbytes;
    // from the layer the loss inputs load during to the head: each layer's
    // input at the start and its output over it
    size_t late = 0;
    for (int l = 1; l < L; ++l) late = std::max(late, P(H[l]));
    const size_t in_off = align16(std::max(late, g_off + gb));
    const size_t in_end = in_off + align16(static_cast<size_t>(R) * kInW * 4);
    const size_t pers = align16(std::max(fwd, in_end));
    for (int C = H[0]; C >= 32; C /= 2) {
        if (H[0] % C != 0 || !width_splits(C, NW, SB, false, regs)) continue;
        size_t bdz[kMaxHidden] = {0}, bst[kMaxHidden] = {0};
        size_t cur = 0, ext = pers + fixed;
        for (int l = L - 1; l >= 1; --l) {
            const int Cl = l == 1 ? C : H[l - 1];
            const size_t dz_size = P(H[l]), st_size = P(Cl);
            const size_t st = cur >= st_size ? 0 : cur + dz_size;
            ext = std::max(ext, st + st_size);
            bdz[l] = cur;
            bst[l] = st;
            cur = st;
        }
        const size_t total = align16(ext);
        if (total > budget) continue;
        if (a) {
            a->lds_in = static_cast<int>(in_off);
            a->defer_in = 1;
            a->lds_bias = static_cast<int>(pers + bias);
            a->lds_rows = static_cast<int>(pers + rows_off);
            a->lds_head = static_cast<int>(pers + head);
            a->lds_last = 0;
            a->lds_w = static_cast<int>(w_off);
            a->lds_sum = static_cast<int>(s_off);
            a->lds_g = static_cast<int>(g_off);
            a->lds_cb = static_cast<int>(P(kpad));
            a->chunk0 = C0;
            a->chunk = C;
            for (int l = 0; l < L; ++l) {
                a->bias_off[l] = bias_off[l];
                a->lds_bdz[l] = static_cast<int>(bdz[l]);
                a->lds_bst[l] = static_cast<int>(bst[l]);
            }
        }
        return total;
    }
    return 0;
}

// The update pass's LDS plan for a shape: streamed first layer at three
// workgroups per CU, else the shared-region plan.
size_t update_layout(int L, const int *H, int kpad, int A, const FusedShape &sh, FusedArgs *a) {
    const size_t budget = kMaxLdsBytes / sh.per_cu;
    return sh.per_cu == 3 ? fused_stream_layout(L, H, kpad, A, sh.rows, sh.threads, budget, a)
                          : fused_update_layout(L, H, kpad, A, sh.rows, sh.threads, budget, a);
}

}  // namespace

FusedShape fused_shape(int L, const int *H, int kpad, int A, int prefer_rows, int prefer_threads, bool update,
                       int prefer_per_cu) {
    FusedShape none{0, 0, 0};
    if (L < 1 || L > kMaxHidden || A < 1 || A > kFusedMaxAct || kpad < 16 || kpad % 16 != 0) return none;
    // inference candidates (the update pass's are below) in order of
    // preference: 32 rows x 4 waves with two workgroups per CU (a policy step
    // is latency-bound: more, shorter workgroups; one hides the other's
    // prologue, head and barrier latencies); 64 rows x 8 waves (each weight
    // fragment feeds two MFMAs, two waves per SIMD, one workgroup per CU).
    // The shapes with one workgroup of 32 rows or of 4 waves per CU run only
    // when asked for by rows and threads.
    if (update) {
        // the update pass's LDS plan holds about one wide layer: 64 samples x
        // 4 waves with two workgroups per CU first (each weight fragment feeds
        // two MFMAs, and one workgroup's prologue, head and barriers overlap
        // the other's MFMA phases), then 32 samples x 4 waves two per CU, then
        // 64 samples x 8 waves alone on a CU (the [1024, 512, 256] network: its
        // update runs in 0.8x the time of the layer-by-layer GEMMs); 32 samples
        // x 8 waves alone on a CU loses to those GEMMs and runs only when asked
        const FusedShape cand[5] = {{64, 256, 3}, {64, 256, 2}, {32, 256, 2}, {64, 512, 1}, {32, 512, 1}};
        const bool asked = prefer_rows && prefer_threads;
        for (int i = 0; i < 5; ++i) {
            const FusedShape &c = cand[i];
            if (i >= 4 && !asked) break;
            if (prefer_rows && c.rows != prefer_rows) continue;
            if (prefer_threads && c.threads != prefer_threads) continue;
            if (prefer_per_cu && c.per_cu != prefer_per_cu) continue;
            if (update_layout(L, H, kpad, A, c, nullptr) > 0) return c;
        }
        return none;
    }
    const FusedShape cand[4] = {{32, 256, 2}, {64, 512, 1}, {32, 512, 1}, {64, 256, 1}};
    const bool asked = prefer_rows && prefer_threads;
    for (int i = 0; i < 4; ++i) {
        const FusedShape &c = cand[i];
        if (i >= 2 && !asked) break;
        if (prefer_rows && c.rows != prefer_rows) continue;
        if (prefer_threads && c.threads != prefer_threads) continue;
        if (fused_fits(L, H, kpad, A, c.rows, c.threads, c.per_cu == 2)) return c;
    }
    return none;
}

int fused_blocks(int M, int R) { return R > 0 ? (M + R - 1) / R : 0; }

void add_frag_job(FragArgs &a, const FragJob &j) {
    FragJob q = j;
    q.begin = a.total;
    a.job[a.count++] = q;
    a.total += (q.rows / 32) * q.S * 64 * (q.split ? 2 : 1);
}

hipError_t launch_pack_frags(const FragArgs &a, hipStream_t s) {
    if (a.total == 0) return hipSuccess;
    hipLaunchKernelGGL(pack_frags_kernel, dim3((a.total + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_fused_infer(FusedArgs a, hipStream_t s) {
    const FusedShape sh = fused_shape(a.L, a.H, a.kpad, a.A, a.R, a.NT);
    if (sh.rows == 0 || a.M < 1 || a.net_mask < 1 || a.net_mask > 3) return hipErrorInvalidValue;
    const size_t bytes = fused_layout(a.L, a.H, a.kpad, a.A, sh.rows, sh.threads, &a);
    if (bytes == 0) return hipErrorInvalidValue;
    a.blocks = fused_blocks(a.M, sh.rows);
    static bool attr_set = false;
    if (!attr_set) {
        const void *fns[4] = {reinterpret_cast<const void *>(&fused_infer_kernel<64, 512, 2>),
                              reinterpret_cast<const void *>(&fused_infer_kernel<32, 256, 2>),
                              reinterpret_cast<const void *>(&fused_infer_kernel<32, 512, 2>),
                              reinterpret_cast<const void *>(&fused_infer_kernel<64, 256, 1>)};
        for (const void *fn : fns) {
            const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLdsBytes);
            if (e != hipSuccess) return e;
        }
        attr_set = true;
    }
    const dim3 grid(a.net_mask == 3 ? two_net_grid(a.blocks) : a.blocks), block(sh.threads);
    if (sh.rows == 64 && sh.threads == 512)
        hipLaunchKernelGGL((fused_infer_kernel<64, 512, 2>), grid, block, bytes, s, a);
    else if (sh.rows == 32 && sh.threads == 256)
        hipLaunchKernelGGL((fused_infer_kernel<32, 256, 2>), grid, block, bytes, s, a);
    else if (sh.rows == 32)
        hipLaunchKernelGGL((fused_infer_kernel<32, 512, 2>), grid, block, bytes, s, a);
    else
        hipLaunchKernelGGL((fused_infer_kernel<64, 256, 1>), grid, block, bytes, s, a);
    return hipGetLastError();
}

hipError_t launch_fused_update(FusedArgs a, hipStream_t s) {
    const FusedShape sh = fused_shape(a.L, a.H, a.kpad, a.A, a.R, a.NT, true, a.per_cu);
    if (sh.per_cu != a.per_cu) return hipErrorInvalidValue;
    if (sh.rows == 0 || a.M < 1) return hipErrorInvalidValue;
    const size_t bytes = update_layout(a.L, a.H, a.kpad, a.A, sh, &a);
    if (bytes == 0) return hipErrorInvalidValue;
    a.blocks = fused_blocks(a.M, sh.rows);
    static bool attr_set = false;
    if (!attr_set) {
        const void *fns[5] = {reinterpret_cast<const void *>(&fused_update_kernel<64, 256, 2>),
                              reinterpret_cast<const void *>(&fused_update_kernel<32, 256, 2>),
                              reinterpret_cast<const void *>(&fused_update_kernel<64, 512, 2>),
                              reinterpret_cast<const void *>(&fused_update_kernel<32, 512, 2>),
                              reinterpret_cast<const void *>(&fused_update_kernel<64, 256, 3, true>)};
        for (const void *fn : fns) {
            const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, kMaxLdsBytes);
            if (e != hipSuccess) return e;
        }
        attr_set = true;
    }
    const dim3 grid(two_net_grid(a.blocks)), block(sh.threads);
    if (sh.per_cu == 3)
        hipLaunchKernelGGL((fused_update_kernel<64, 256, 3, true>), grid, block, bytes, s, a);
    else if (sh.rows == 64 && sh.threads == 256)
        hipLaunchKernelGGL((fused_update_kernel<64, 256, 2>), grid, block, bytes, s, a);
    else if (sh.rows == 32 && sh.threads == 256)
        hipLaunchKernelGGL((fused_update_kernel<32, 256, 2>), grid, block, bytes, s, a);
    else if (sh.rows == 64)
        hipLaunchKernelGGL((fused_update_kernel<64, 512, 2>), grid, block, bytes, s, a);
    else
        hipLaunchKernelGGL((fused_update_kernel<32, 512, 2>), grid, block, bytes, s, a);
    return hipGetLastError();
}

}  // namespace ppo
