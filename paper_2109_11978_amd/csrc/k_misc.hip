// Non-GEMM kernels of the PPO learner for gfx950: Philox4x32-10 action noise,
// the policy/critic output heads fused with sampling (rollout) or with the
// PPO loss and its output gradients (update), GAE with the float64 advantage
// statistics, gradient assembly with the float64 global norm, and Adam.
#include "common.hpp"

#include <mutex>
#include "philox.hpp"

namespace ppo {
namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr float kLog2Pi = 1.8378770664093453f;
constexpr int kMaxAct = 16;

// ------------------------------------------------------------------ Philox
__global__ void philox_blocks_kernel(uint32_t k0, uint32_t k1, uint32_t c0, uint32_t c1, uint32_t c2,
                                     uint32_t c3, long long n, uint32_t *out) {
    for (long long i = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<long long>(gridDim.x) * blockDim.x) {
        uint32_t c[4] = {c0 + static_cast<uint32_t>(i), c1, c2, c3};
        philox4x32_10(c, k0, k1);
        *reinterpret_cast<u32x4 *>(out + 4 * i) = u32x4{c[0], c[1], c[2], c[3]};
    }
}

// --------------------------------------------------------------- reductions
__device__ inline float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ inline double wave_sum_d(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// ------------------------------------------------------------ obs gather
template <typename T>
__global__ void gather_obs_kernel(const float *obs, const int32_t *idx, int src_rows, int rows, int D, int ld,
                                  T *out) {
    const long long total = static_cast<long long>(rows) * ld;
    for (long long e = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x; e < total;
         e += static_cast<long long>(gridDim.x) * blockDim.x) {
        const int r = static_cast<int>(e / ld);
        const int k = static_cast<int>(e - static_cast<long long>(r) * ld);
        // indices outside [0, src_rows) are clamped so a bad permutation cannot fault
        const long long src_row = idx ? min(max(idx[r], 0), src_rows - 1) : r;
        const float v = k < D ? obs[src_row * D + k] : 0.0f;
        out[e] = Elem<T>::from_f(v);
    }
}

// ------------------------------------------------- output-layer helpers
constexpr int kHeadThreads = 256;
constexpr int kLossRows = 32;     // mini-batch samples per block (loss)
constexpr int kSampleRows = 16;   // environments per block (rollout)
constexpr int kWPad = 4;          // floats of row padding for staged output-layer weights

// 8 consecutive activations of one row as float32.
template <typename T>
__device__ inline void load8(const T *src, float (&x)[8]) {
    if constexpr (sizeof(T) == 2) {
        const u32x4 r = *reinterpret_cast<const u32x4 *>(src);
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            x[2 * w] = __uint_as_float(r[w] << 16);
            x[2 * w + 1] = __uint_as_float(r[w] & 0xFFFF0000u);
        }
    } else {
        const float4 p = reinterpret_cast<const float4 *>(src)[0];
        const float4 q = reinterpret_cast<const float4 *>(src)[1];
        x[0] = p.x; x[1] = p.y; x[2] = p.z; x[3] = p.w;
        x[4] = q.x; x[5] = q.y; x[6] = q.z; x[7] = q.w;
    }
}

// Output-layer weights of both networks: rows j < A are the actor's, row A
// the critic's, each padded to Hl + kWPad floats.  Staged in LDS when they
// fit (dynamic shared memory), else read from global memory.
struct HeadWeights {
    const float *w;
    int pitch;
};

__device__ inline HeadWeights stage_head_weights(float *s_w, bool in_lds, const float *Wa, const float *Wc, int A,
                                                 int Hl) {
    if (!in_lds) return HeadWeights{nullptr, 0};
    const int pitch = Hl + kWPad;
    const int n = (A + 1) * Hl;
    // eight loads in flight per thread before any store
    constexpr int U = 8;
    for (int q0 = threadIdx.x; q0 < n; q0 += U * blockDim.x) {
        float v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int q = q0 + u * blockDim.x;
            const int j = q / Hl, k = q - (q / Hl) * Hl;
            v[u] = q < n ? (j < A ? Wa[static_cast<long long>(j) * Hl + k] : Wc[k]) : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int q = q0 + u * blockDim.x;
            const int j = q / Hl, k = q - (q / Hl) * Hl;
            if (q < n) s_w[j * pitch + k] = v[u];
        }
    }
    __syncthreads();
    return HeadWeights{s_w, pitch};
}

__device__ inline const float *head_row(const HeadWeights &hw, const float *Wa, const float *Wc, int A, int Hl,
                                        int j) {
    if (hw.w) return hw.w + j * hw.pitch;
    return j < A ? Wa + static_cast<long long>(j) * Hl : Wc;
}

// out[i][j] = b_j + h_i . W_j for the A actor outputs (j < A) and the critic
// value (j == A); one dot product per thread.  Hl is a multiple of 16.
// The block's rows of both last hidden layers, staged in LDS (pitch Hl + 8
// elements) with coalesced 16-byte loads, four in flight per thread.
template <typename T>
__device__ inline void stage_hidden_rows(T *ha_l, T *hc_l, const T *ha, const T *hc, int r0, int rows, int Hl,
                                         bool actor, bool critic) {
    constexpr int VEC = 16 / sizeof(T);
    const int pitch = Hl + 8;
    const int per_row = Hl / VEC;
    const int n = 2 * rows * per_row;
    constexpr int U = 4;
    for (int q0 = threadIdx.x; q0 < n; q0 += U * blockDim.x) {
        u32x4 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int q = q0 + u * blockDim.x;
            const int net = q / (rows * per_row);
            const int rem = q - net * rows * per_row;
            const int i = rem / per_row, c = (rem - i * per_row) * VEC;
            const bool want = q < n && (net == 0 ? actor : critic);
            if (want)
                v[u] = *reinterpret_cast<const u32x4 *>((net == 0 ? ha : hc) + static_cast<long long>(r0 + i) * Hl + c);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int q = q0 + u * blockDim.x;
            const int net = q / (rows * per_row);
            const int rem = q - net * rows * per_row;
            const int i = rem / per_row, c = (rem - i * per_row) * VEC;
            const bool want = q < n && (net == 0 ? actor : critic);
            if (want) *reinterpret_cast<u32x4 *>((net == 0 ? ha_l : hc_l) + i * pitch + c) = v[u];
        }
    }
    __syncthreads();
}

// Bytes of dynamic LDS for `rows` staged rows of both last hidden layers,
// 0 when they do not fit next to the output-layer weights.
template <typename T>
size_t head_rows_lds(int rows, int Hl, size_t weight_bytes) {
    const size_t bytes = 2 * static_cast<size_t>(rows) * (Hl + 8) * sizeof(T);
    return weight_bytes + bytes <= 48 * 1024 ? bytes : 0;
}

template <typename T, int ROWS>
__device__ inline void output_layers(const T *ha, const T *hc, const T *ha_l, const T *hc_l,
                                     const HeadWeights &hw, const float *Wa,
                                     const float *ba, const float *Wc, const float *bc, int r0, int rows, int A,
                                     int Hl, bool actor, float (*out)[kMaxAct + 1]) {
    const int n_out = A + 1;
    for (int q = threadIdx.x; q < ROWS * n_out; q += kHeadThreads) {
        const int i = q / n_out, j = q - (q / n_out) * n_out;
        if (i >= rows || (j < A && !actor)) continue;
        const T *h = ha_l ? (j < A ? ha_l : hc_l) + i * (Hl + 8)
                          : (j < A ? ha : hc) + static_cast<long long>(r0 + i) * Hl;
        const float *w = head_row(hw, Wa, Wc, A, Hl, j);
        float acc = j < A ? ba[j] : bc[0];
        // 64 activations (eight 8-wide loads) in flight per step; Hl is a multiple of 16
        for (int k0 = 0; k0 < Hl; k0 += 64) {
            float x[8][8];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (k0 + 8 * u < Hl) load8<T>(h + k0 + 8 * u, x[u]);
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (k0 + 8 * u < Hl)
#pragma unroll
                    for (int e = 0; e < 8; ++e) acc += x[u][e] * w[k0 + 8 * u + e];
        }
        out[i][j] = acc;
    }
}

// ----------------------------------------------------------- head + sample
// Rollout: mu = h_a Wa^T + ba and V = h_c Wc^T + bc for 16 environments per
// block, then one lane per environment draws the diagonal-Gaussian action
// a = mu + sigma * eps with Philox noise and its log-density
// sum_j(-eps_j^2 / 2 - log sigma_j) - (A/2) log(2 pi).
template <typename T>
__global__ __launch_bounds__(kHeadThreads) void head_sample_kernel(const HeadSampleArgs a, int w_in_lds,
                                                                    int rows_lds_offset) {
    extern __shared__ float s_w[];
    __shared__ float s_out[kSampleRows][kMaxAct + 1];
    const int r0 = blockIdx.x * kSampleRows;
    const int rows = min(kSampleRows, a.N - r0);
    const int A = a.A;
    const HeadWeights hw = stage_head_weights(s_w, w_in_lds, a.Wa, a.Wc, A, a.Hl);
    const T *ha = static_cast<const T *>(a.ha);
    const T *hc = static_cast<const T *>(a.hc);
    T *ha_l = nullptr, *hc_l = nullptr;
    if (rows_lds_offset >= 0) {
        ha_l = reinterpret_cast<T *>(reinterpret_cast<char *>(s_w) + rows_lds_offset);
        hc_l = ha_l + kSampleRows * (a.Hl + 8);
        stage_hidden_rows<T>(ha_l, hc_l, ha, hc, r0, rows, a.Hl, !a.value_only, true);
    }
    output_layers<T, kSampleRows>(ha, hc, ha_l, hc_l, hw, a.Wa, a.ba, a.Wc, a.bc, r0, rows, A, a.Hl,
                                  !a.value_only, s_out);
    __syncthreads();
    const int i = threadIdx.x;
    if (i >= rows) return;
    const int n = r0 + i;
    if (a.values) a.values[n] = s_out[i][A];
    if (a.value_only) return;
    const int groups = (A + 3) / 4;
    CompSum lp;   // log-density in float32 with compensated summation
    for (int g = 0; g < groups; ++g) {
        uint32_t c[4] = {static_cast<uint32_t>(n) * groups + g, a.t, a.iteration, 1u};
        philox4x32_10(c, a.key0, a.key1);
        float eps[4];
        box_muller(c[0], c[1], eps[0], eps[1]);
        box_muller(c[2], c[3], eps[2], eps[3]);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int j = 4 * g + q;
            if (j >= A) break;
            const float m = s_out[i][j];
            const float ls = a.logstd[j];
            lp.add_gauss(eps[q], ls);
            if (a.actions) a.actions[static_cast<long long>(n) * A + j] = m + expf(ls) * eps[q];
            if (a.mu) a.mu[static_cast<long long>(n) * A + j] = m;
        }
    }
    if (a.logp) a.logp[n] = lp.value();
}

// ------------------------------------------------------------- head + loss
// Update: for 32 mini-batch samples per block, the output layers, the
// log-probability of the stored action, the ratio, clipped surrogate and
// value loss with their gradients wrt mu and V (one lane per sample), then
// the gradient through the output layers and the last ELU into the last
// hidden pre-activations (8-wide row segments, coalesced).  Per-block sums of
// the loss terms and of the log-std gradient go to `partials` (wave-0
// shuffle reduction, fixed order).
template <typename T>
__global__ __launch_bounds__(kHeadThreads) void head_loss_kernel(const HeadLossArgs a, int w_in_lds,
                                                                  int rows_lds_offset) {
    extern __shared__ float s_w[];
    __shared__ float s_out[kLossRows][kMaxAct + 1];
    const int r0 = blockIdx.x * kLossRows;
    const int rows = min(kLossRows, a.M - r0);
    const int A = a.A, Hl = a.Hl;
    const int W = A + 8;
    const T *ha = static_cast<const T *>(a.ha);
    const T *hc = static_cast<const T *>(a.hc);
    const HeadWeights hw = stage_head_weights(s_w, w_in_lds, a.Wa, a.Wc, A, Hl);
    // the block's activation rows, read once from HBM and reused by the
    // output layers and the backward below
    T *ha_l = nullptr, *hc_l = nullptr;
    if (rows_lds_offset >= 0) {
        ha_l = reinterpret_cast<T *>(reinterpret_cast<char *>(s_w) + rows_lds_offset);
        hc_l = ha_l + kLossRows * (Hl + 8);
        stage_hidden_rows<T>(ha_l, hc_l, ha, hc, r0, rows, Hl, true, true);
    }
    output_layers<T, kLossRows>(ha, hc, ha_l, hc_l, hw, a.Wa, a.ba, a.Wc, a.bc, r0, rows, A, Hl, true, s_out);
    __syncthreads();

    const int tid = threadIdx.x;
    if (tid < 64) {
        float pl = 0.0f, vl = 0.0f, clipped = 0.0f, kl = 0.0f, kl_mu = 0.0f;
        float dls[kMaxAct];
#pragma unroll
        for (int j = 0; j < kMaxAct; ++j) dls[j] = 0.0f;
        if (tid < rows) {
            const int i = tid;
            const long long row = a.idx ? min(max(a.idx[r0 + i], 0), a.B - 1) : r0 + i;
            // Log-ratio log pi(a|s) - lp_old: the A log-density terms and -lp_old
            // summed with compensation in float32 (terms of order 1 that nearly
            // cancel against lp_old).
            float z[kMaxAct];
            CompSum lr;
#pragma unroll
            for (int j = 0; j < kMaxAct; ++j) {
                z[j] = 0.0f;
                if (j < A) {
                    const float ls = a.logstd[j];
                    const float inv_sigma = expf(-ls);
                    z[j] = (a.actions[row * A + j] - s_out[i][j]) * inv_sigma;
                    lr.add_gauss(z[j], ls);
                    if (a.mu_old) {
                        // mean-shift part of KL(pi_old || pi_new): (mu_old - mu)^2 / (2 sigma^2)
                        const float dm = (a.mu_old[row * A + j] - s_out[i][j]) * inv_sigma;
                        kl_mu += 0.5f * dm * dm;
                    }
                }
            }
            const float adv = a.adv[row];
            lr.add(-a.logp_old[row]);
            const float ratio = expf(lr.value());
            const float lo = 1.0f - a.clip, hi = 1.0f + a.clip;
            pl = -fminf(ratio * adv, fminf(fmaxf(ratio, lo), hi) * adv);
            const bool active = adv >= 0.0f ? (ratio <= hi) : (ratio >= lo);
            if (a.active_out) a.active_out[r0 + i] = active ? 1 : 0;
            if (a.ratio_out) a.ratio_out[r0 + i] = ratio;
            clipped = fabsf(ratio - 1.0f) > a.clip ? 1.0f : 0.0f;
            kl = (ratio - 1.0f) - logf(ratio);
            const float g_lp = active ? -a.inv_m * adv * ratio : 0.0f;

            const float V = s_out[i][A];
            const float ret = a.returns[row];
            const float diff = V - ret;
            float pass = 1.0f;
            vl = diff * diff;
            if (a.clip_value) {
                const float v_old = a.values_old[row];
                const float vc = v_old + fminf(fmaxf(V - v_old, -a.clip), a.clip);
                const float sqc = (vc - ret) * (vc - ret);
                pass = vl >= sqc ? 1.0f : 0.0f;
                vl = fmaxf(vl, sqc);
            }
            const float g_v = 2.0f * a.value_coef * a.inv_m * diff * pass;

            T *dha = static_cast<T *>(a.dz_head_a) + static_cast<long long>(r0 + i) * kHeadPad;
            T *dhc = static_cast<T *>(a.dz_head_c) + static_cast<long long>(r0 + i) * kHeadPad;
#pragma unroll
            for (int j = 0; j < kMaxAct; ++j) {
                float gm = 0.0f;
                if (j < A) {
                    gm = g_lp * z[j] * expf(-a.logstd[j]);
                    dls[j] = g_lp * (z[j] * z[j] - 1.0f);
                    s_out[i][j] = gm;
                }
                dha[j] = Elem<T>::from_f(gm);
                dhc[j] = Elem<T>::from_f(j == 0 ? g_v : 0.0f);
            }
            s_out[i][A] = g_v;
        }
        // wave 0 holds every sample of the block: shuffle-reduce in a fixed order
        const float w_pl = wave_sum(pl), w_vl = wave_sum(vl), w_cl = wave_sum(clipped), w_kl = wave_sum(kl);
        const float w_klmu = wave_sum(kl_mu);
        float w_dls[kMaxAct];
#pragma unroll
        for (int j = 0; j < kMaxAct; ++j) w_dls[j] = wave_sum(dls[j]);
        if (tid == 0) {
            float *out = a.partials + static_cast<long long>(blockIdx.x) * W;
            out[0] = w_pl;
            out[1] = w_vl;
            out[2] = w_cl;
            out[3] = w_kl;
#pragma unroll
            for (int j = 0; j < kMaxAct; ++j)
                if (j < A) out[4 + j] = w_dls[j];
            float ent = 0.0f, kl_ls = 0.0f;
            if (blockIdx.x == 0) {
                // entropy of the state-independent policy at this step's parameters
                ent = 0.5f * A * (1.0f + kLog2Pi);
                for (int j = 0; j < A; ++j) ent += a.logstd[j];
                // sample-independent part of the KL:
                //   sum_j log(sigma / sigma_old) + sigma_old^2 / (2 sigma^2) - 1/2
                if (a.mu_old)
                    for (int j = 0; j < A; ++j) {
                        const float d = a.logstd_old[j] - a.logstd[j];
                        kl_ls += -d + 0.5f * expf(2.0f * d) - 0.5f;
                    }
            }
            out[4 + A] = ent;
            out[5 + A] = w_klmu;
            out[6 + A] = kl_ls;
        }
    }
    __syncthreads();

    // gradient into the last hidden pre-activations, both networks
    const int chunks = Hl / 8;
    const int n_q = 2 * kLossRows * chunks;
    // four 8-wide activation loads in flight per thread before the arithmetic
    constexpr int U = 4;
    for (int q0 = tid; q0 < n_q; q0 += U * kHeadThreads) {
        float xs[U][8];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int q = q0 + u * kHeadThreads;
            const int net = q / (kLossRows * chunks);
            const int rem = q - net * kLossRows * chunks;
            const int i = rem / chunks;
            const int k = (rem - i * chunks) * 8;
            if (q < n_q && i < rows) {
                if (ha_l)
                    load8<T>((net == 0 ? ha_l : hc_l) + i * (Hl + 8) + k, xs[u]);
                else
                    load8<T>((net == 0 ? ha : hc) + static_cast<long long>(r0 + i) * Hl + k, xs[u]);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
        const int q = q0 + u * kHeadThreads;
        const int net = q / (kLossRows * chunks);
        const int rem = q - net * kLossRows * chunks;
        const int i = rem / chunks;
        const int k = (rem - i * chunks) * 8;
        if (q >= n_q || i >= rows) continue;
        const long long off = static_cast<long long>(r0 + i) * Hl + k;
        const float *x = xs[u];
        float g[8];
        if (net == 0) {
#pragma unroll
            for (int e = 0; e < 8; ++e) g[e] = 0.0f;
            for (int j = 0; j < A; ++j) {
                const float gm = s_out[i][j];
                const float *w = head_row(hw, a.Wa, a.Wc, A, Hl, j) + k;
#pragma unroll
                for (int e = 0; e < 8; ++e) g[e] += gm * w[e];
            }
        } else {
            const float gv = s_out[i][A];
            const float *w = head_row(hw, a.Wa, a.Wc, A, Hl, A) + k;
#pragma unroll
            for (int e = 0; e < 8; ++e) g[e] = gv * w[e];
        }
        T o[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) o[e] = Elem<T>::from_f(g[e] * (x[e] > 0.0f ? 1.0f : x[e] + 1.0f));
        T *dst = static_cast<T *>(net == 0 ? a.dza : a.dzc) + off;
        if constexpr (sizeof(T) == 2) {
            *reinterpret_cast<u32x4 *>(dst) = *reinterpret_cast<const u32x4 *>(o);
        } else {
            reinterpret_cast<u32x4 *>(dst)[0] = reinterpret_cast<const u32x4 *>(o)[0];
            reinterpret_cast<u32x4 *>(dst)[1] = reinterpret_cast<const u32x4 *>(o)[1];
        }
        }
    }
}

// ------------------------------------------------------------------- GAE
// One lane per environment walks t = T-1 .. 0 (coalesced across lanes):
//   r' = r + gamma V timeout;  delta = r' + gamma (1 - d) V_next - V;
//   A = delta + gamma lambda (1 - d) A_next;  R = A + V.
// Each lane keeps a float64 Welford (count, mean, M2) of its advantages; the
// block merges them (Chan et al.) in a fixed order into one partial.
constexpr int kGaeThreads = 256;
constexpr int kGaeChunk = 16;   // rollout steps whose inputs a lane loads together
constexpr int kFinalizeThreads = 256;

struct Welford { double n, mean, m2; };

__device__ inline Welford merge(const Welford &x, const Welford &y) {
    if (x.n == 0.0) return y;
    if (y.n == 0.0) return x;
    const double n = x.n + y.n;
    const double d = y.mean - x.mean;
    return {n, x.mean + d * (y.n / n), x.m2 + y.m2 + d * d * (x.n * y.n / n)};
}

__device__ inline Welford shfl_xor_w(const Welford &w, int o) {
    return {__shfl_xor(w.n, o), __shfl_xor(w.mean, o), __shfl_xor(w.m2, o)};
}

__global__ __launch_bounds__(kGaeThreads) void gae_kernel(const GaeArgs a) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    Welford w{0.0, 0.0, 0.0};
    if (n < a.N) {
        float next_v = a.last_values[n];
        float next_a = 0.0f;
        const float gl = a.gamma * a.lam;
        // the scan runs backwards in chunks of kGaeChunk steps whose inputs
        // are all loaded before the chunk's arithmetic, so a lane waits for
        // memory once per chunk rather than once per step
        for (int t0 = a.T - 1; t0 >= 0; t0 -= kGaeChunk) {
            float vv[kGaeChunk], rr[kGaeChunk];
            uint8_t dd[kGaeChunk], tt[kGaeChunk];
#pragma unroll
            for (int i = 0; i < kGaeChunk; ++i) {
                const int t = t0 - i;
                if (t >= 0) {
                    const long long s = static_cast<long long>(t) * a.N + n;
                    vv[i] = a.values[s];
                    rr[i] = a.rewards[s];
                    dd[i] = a.dones[s];
                    tt[i] = a.timeouts ? a.timeouts[s] : 0;
                }
            }
#pragma unroll
            for (int i = 0; i < kGaeChunk; ++i) {
                const int t = t0 - i;
                if (t >= 0) {
                    const long long s = static_cast<long long>(t) * a.N + n;
                    const float v = vv[i];
                    float r = rr[i];
                    if (tt[i]) r += a.gamma * v;
                    const float nd = dd[i] ? 0.0f : 1.0f;
                    const float delta = r + a.gamma * nd * next_v - v;
                    const float adv = delta + gl * nd * next_a;
                    a.adv[s] = adv;
                    a.returns[s] = adv + v;
                    next_v = v;
                    next_a = adv;
                    const double x = adv;
                    w.n += 1.0;
                    const double d = x - w.mean;
                    w.mean += d / w.n;
                    w.m2 += d * (x - w.mean);
                }
            }
        }
    }
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const Welford other = shfl_xor_w(w, o);
        // merge in lane order so every lane holds the same value
        const bool lower = (threadIdx.x & o) == 0;
        w = lower ? merge(w, other) : merge(other, w);
    }
    // then the block's waves, in wave order
    __shared__ Welford s_wave[kGaeThreads / 64];
    if ((threadIdx.x & 63) == 0) s_wave[threadIdx.x >> 6] = w;
    __syncthreads();
    if (threadIdx.x == 0) {
        w = s_wave[0];
#pragma unroll
        for (int i = 1; i < kGaeThreads / 64; ++i) w = merge(w, s_wave[i]);
        a.partials[3 * blockIdx.x + 0] = w.n;
        a.partials[3 * blockIdx.x + 1] = w.mean;
        a.partials[3 * blockIdx.x + 2] = w.m2;
    }
}

// Every block merges all partials the same way, so each holds the identical
// result: thread i merges a contiguous chunk of partials in index order, then
// a pairwise tree over the threads in index order.  Block 0 publishes (mean,
// unbiased std), and all blocks optionally normalise.
__global__ __launch_bounds__(kFinalizeThreads) void adv_finalize_kernel(const double *partials, int nparts,
                                                                        float *adv, long long count,
                                                                        double *stats_out, int normalize) {
    __shared__ Welford s_w[kFinalizeThreads];
    __shared__ double s_mean, s_std;
    const int chunk = (nparts + kFinalizeThreads - 1) / kFinalizeThreads;
    const int p0 = min(nparts, static_cast<int>(threadIdx.x) * chunk), p1 = min(nparts, p0 + chunk);
    Welford w{0.0, 0.0, 0.0};
    for (int p = p0; p < p1; ++p) w = merge(w, Welford{partials[3 * p], partials[3 * p + 1], partials[3 * p + 2]});
    s_w[threadIdx.x] = w;
    __syncthreads();
    for (int off = 1; off < kFinalizeThreads; off <<= 1) {
        if ((threadIdx.x & (2 * off - 1)) == 0) s_w[threadIdx.x] = merge(s_w[threadIdx.x], s_w[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        w = s_w[0];
        s_mean = w.mean;
        s_std = w.n > 1.0 ? sqrt(w.m2 / (w.n - 1.0)) : 0.0;
        if (blockIdx.x == 0) {
            stats_out[0] = s_mean;
            stats_out[1] = s_std;
        }
    }
    __syncthreads();
    if (!normalize) return;
    const double mean = s_mean;
    const double inv = 1.0 / (s_std + 1e-8);
    auto norm = [&](float x) { return static_cast<float>((static_cast<double>(x) - mean) * inv); };
    // 16-byte accesses (adv is 16-byte aligned), then the tail of count % 4
    const long long stride = static_cast<long long>(gridDim.x) * blockDim.x;
    const long long first = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x;
    const long long n4 = count / 4;
    float4 *adv4 = reinterpret_cast<float4 *>(adv);
    for (long long e = first; e < n4; e += stride) {
        float4 v = adv4[e];
        v.x = norm(v.x);
        v.y = norm(v.y);
        v.z = norm(v.z);
        v.w = norm(v.w);
        adv4[e] = v;
    }
    for (long long e = 4 * n4 + first; e < count; e += stride) adv[e] = norm(adv[e]);
}

// -------------------------------------------------------- gradient reduce
// Blocks 0 .. gridDim-2 sum the split partials of every segment into the
// flat gradient; the last block sums the loss partials column-wise (8 row
// stripes, then the stripes in order) into the log-std gradient and the
// loss sums.  Every block writes the float64 sum of squares of what it wrote.
constexpr int kReduceThreads = 256;

__global__ __launch_bounds__(kReduceThreads) void grad_reduce_kernel(const ReduceArgs a) {
    __shared__ double red[kReduceThreads / 64];
    double ss = 0.0;
    if (blockIdx.x + 1 < gridDim.x) {
        const long long stride = static_cast<long long>(gridDim.x - 1) * blockDim.x;
        for (long long e = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x; e < a.total; e += stride) {
            int si = 0;
            while (si + 1 < a.count && e >= a.seg[si + 1].begin) ++si;
            const ReduceSegment &S = a.seg[si];
            const long long local = e - S.begin;
            const int r = static_cast<int>(local / S.cols);
            const int c = static_cast<int>(local - static_cast<long long>(r) * S.cols);
            const float *src = S.src + static_cast<long long>(r) * S.ld + c;
            // eight partials in flight at a time, added in split order
            float sum = 0.0f;
            for (int s0 = 0; s0 < S.splits; s0 += 8) {
                float v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) v[u] = s0 + u < S.splits ? src[(s0 + u) * S.split_stride] : 0.0f;
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (s0 + u < S.splits) sum += v[u];
            }
            sum += S.add;
            a.grad[S.dst_offset + local] = sum;
            ss += static_cast<double>(sum) * sum;
        }
    } else {
        // columns: 4 loss sums, A log-std gradients, entropy, mean-shift KL, log-std KL
        __shared__ float stripe[8][kMaxAct + 8];
        __shared__ float total[kMaxAct + 8];
        const int cols = 7 + a.A;
        const int c = threadIdx.x & 31, st = threadIdx.x >> 5;
        if (c < cols) {
            // sixteen independent running sums keep sixteen loads in flight (the
            // partials come from every XCD, so each round trip is long); they
            // are combined in a fixed pairwise order, so the result does not
            // depend on timing
            constexpr int U = 16;
            float acc[U];
#pragma unroll
            for (int u = 0; u < U; ++u) acc[u] = 0.0f;
            int b = st;
            for (; b + 8 * (U - 1) < a.n_loss; b += 8 * U)
#pragma unroll
                for (int u = 0; u < U; ++u)
                    acc[u] += a.loss_partials[static_cast<long long>(b + 8 * u) * a.loss_width + c];
            for (; b < a.n_loss; b += 8) acc[0] += a.loss_partials[static_cast<long long>(b) * a.loss_width + c];
#pragma unroll
            for (int w = 1; w < U; w *= 2)
#pragma unroll
                for (int u = 0; u < U; u += 2 * w) acc[u] += acc[u + w];
            stripe[st][c] = acc[0];
        }
        __syncthreads();
        if (threadIdx.x < cols) {
            float v = 0.0f;
            for (int q = 0; q < 8; ++q) v += stripe[q][threadIdx.x];
            total[threadIdx.x] = v;
            if (threadIdx.x < 4) {
                a.loss_sums[threadIdx.x] = v;
            } else if (threadIdx.x < 4 + a.A && a.grad) {
                const float g = v - a.entropy_coef;
                a.grad[a.logstd_offset + threadIdx.x - 4] = g;
                ss = static_cast<double>(g) * g;
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            a.loss_sums[4] = total[4 + a.A];
            const float kl = total[5 + a.A] * a.inv_m + total[6 + a.A];
            a.loss_sums[5] = kl;
            if (a.lr && a.desired_kl > 0.0f) {
                // Algorithm 1: shrink the rate when the step moved the policy too
                // far, grow it when it moved too little, within [lr_min, lr_max]
                float lr = *a.lr;
                if (kl > 2.0f * a.desired_kl)
                    lr = fmaxf(a.lr_min, lr / a.lr_factor);
                else if (kl < 0.5f * a.desired_kl)
                    lr = fminf(a.lr_max, lr * a.lr_factor);
                *a.lr = lr;
            }
        }
    }
    ss = wave_sum_d(ss);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = ss;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kReduceThreads / 64; ++w) t += red[w];
        a.sumsq_partials[blockIdx.x] = t;
    }
}

// ------------------------------------------------------------------ Adam
constexpr int kAdamThreads = 256;

__global__ __launch_bounds__(kAdamThreads) void adam_kernel(const AdamArgs a) {
    __shared__ double s_sumsq;
    __shared__ double red[kAdamThreads / 64];
    __shared__ float s_bc[2];
    // this thread's first element goes out before the norm is known
    const long long first = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x;
    const bool pre = a.apply && first < a.P;
    const float g_first = pre ? a.grad[first] : 0.0f;
    const float m_first = pre ? a.m[first] : 0.0f;
    const float v_first = pre ? a.v[first] : 0.0f;
    const float th_first = pre ? a.theta[first] : 0.0f;
    // global norm: every block sums the same partials in the same order
    // (four loads in flight, added in index order)
    double ss = 0.0;
    int p = threadIdx.x;
    for (; p + 3 * kAdamThreads < a.n_sumsq; p += 4 * kAdamThreads) {
        const double s0 = a.sumsq_partials[p], s1 = a.sumsq_partials[p + kAdamThreads];
        const double s2 = a.sumsq_partials[p + 2 * kAdamThreads], s3 = a.sumsq_partials[p + 3 * kAdamThreads];
        ss += s0;
        ss += s1;
        ss += s2;
        ss += s3;
    }
    for (; p < a.n_sumsq; p += kAdamThreads) ss += a.sumsq_partials[p];
    ss = wave_sum_d(ss);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = ss;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kAdamThreads / 64; ++w) t += red[w];
        s_sumsq = t;
        if (a.apply) {
            // bias corrections of this step, once per block
            const int step = *a.step + a.step_offset + 1;
            s_bc[0] = static_cast<float>(1.0 - pow(static_cast<double>(a.beta1), step));
            s_bc[1] = static_cast<float>(1.0 - pow(static_cast<double>(a.beta2), step));
        }
    }
    __syncthreads();
    const double norm = sqrt(s_sumsq);
    const bool finite = isfinite(norm);
    const float coef = static_cast<float>(fmin(1.0, static_cast<double>(a.max_grad_norm) / (norm + 1e-6)));

    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const float pl = a.loss_sums[0] * a.inv_m, vl = a.loss_sums[1] * a.inv_m;
        const float ent = a.loss_sums[4];
        a.stats[0] = pl + a.value_coef * vl - a.entropy_coef * ent;
        a.stats[1] = pl;
        a.stats[2] = vl;
        a.stats[3] = ent;
        a.stats[4] = a.loss_sums[2] * a.inv_m;
        a.stats[5] = a.loss_sums[3] * a.inv_m;
        a.stats[6] = static_cast<float>(norm);
        a.stats[7] = finite ? 0.0f : 1.0f;
        a.stats[8] = a.loss_sums[5];
        a.stats[9] = a.lr ? *a.lr : 0.0f;
    }
    if (!a.apply || !finite) return;

    const float bc1 = s_bc[0], bc2 = s_bc[1];
    const float lr = *a.lr;
    auto update = [&](long long e, float g_raw, float m_old, float v_old, float th_old) {
        const float g = g_raw * coef;
        const float m = a.beta1 * m_old + (1.0f - a.beta1) * g;
        const float v = a.beta2 * v_old + (1.0f - a.beta2) * g * g;
        a.m[e] = m;
        a.v[e] = v;
        const float th = th_old - lr * (m / bc1) / (sqrtf(v / bc2) + a.eps);
        a.theta[e] = th;
        if (a.shadow) a.shadow[e] = f32_to_bf16(th);
        // the same bf16 value into the fragment copies of its weight matrix:
        // element (r, c) of W [rows][cols] sits in fragment (r / 32, c / 16),
        // lane r % 32 + 32 ((c % 16) / 8), element c % 8; in the transposed
        // copy the roles of r and c swap.  The matrices are disjoint, so at
        // most one matches; every lane visits all of them, which keeps the
        // matrix descriptors uniform across the wave
        for (int j = 0; j < a.n_frag; ++j) {
            const AdamFrag &F = a.frag[j];
            const long long local = e - F.begin;
            if (local < 0 || local >= static_cast<long long>(F.rows) * F.cols) continue;
            // rows * cols < 2^31 (width and observation limits): 32-bit division
            const unsigned li = static_cast<unsigned>(local), cols = static_cast<unsigned>(F.cols);
            const int r = static_cast<int>(li / cols), c = static_cast<int>(li - static_cast<unsigned>(r) * cols);
            const uint16_t bits = f32_to_bf16(th);
            const int li_in = (r & 31) + 32 * ((c & 15) >> 3);
            if (F.split) {
                // split layout: the feature block's S bf16 fragments, then its S
                // residual fragments
                const long long f0 = static_cast<long long>(2 * (r >> 5)) * F.S + (c >> 4);
                F.dst[(f0 * 64 + li_in) * 8 + (c & 7)] = bits;
                F.dst[((f0 + F.S) * 64 + li_in) * 8 + (c & 7)] = f32_to_bf16(th - bf16_to_f32(bits));
            } else {
                const long long fs = static_cast<long long>(r >> 5) * F.S + (c >> 4);
                F.dst[(fs * 64 + li_in) * 8 + (c & 7)] = bits;
            }
            if (F.dst_t)
                F.dst_t[((static_cast<long long>(c >> 5) * F.S_t + (r >> 4)) * 64 + (c & 31) + 32 * ((r & 15) >> 3)) *
                            8 +
                        (r & 7)] = bits;
        }
    };
    const long long stride = static_cast<long long>(gridDim.x) * blockDim.x;
    if (pre) update(first, g_first, m_first, v_first, th_first);
    for (long long e = first + stride; e < a.P; e += stride) update(e, a.grad[e], a.m[e], a.v[e], a.theta[e]);
}

// ------------------------------------------------------- weight staging
// One 64 x 64 tile of one job per block: coalesced reads of source rows into
// LDS, coalesced writes of destination rows (transposed or padded).
constexpr int kStageTile = 64;

template <typename T>
__global__ __launch_bounds__(256) void stage_weights_kernel(const StageArgs a) {
    __shared__ T tile[kStageTile][kStageTile + 1];
    int ji = 0;
    while (ji + 1 < a.count && static_cast<int>(blockIdx.x) >= a.job[ji + 1].tile_begin) ++ji;
    const StageJob &j = a.job[ji];
    const int local = blockIdx.x - j.tile_begin;
    // tiles cover the source (transpose) or the padded destination (copy)
    const int cols_t = j.transpose ? j.cols : j.dst_ld;
    const int tiles_c = (cols_t + kStageTile - 1) / kStageTile;
    const int r0 = (local / tiles_c) * kStageTile;
    const int c0 = (local % tiles_c) * kStageTile;
    const T *src = static_cast<const T *>(j.src);
    T *dst = static_cast<T *>(j.dst);
    for (int e = threadIdx.x; e < kStageTile * kStageTile; e += blockDim.x) {
        const int r = e / kStageTile, c = e % kStageTile;
        const int gr = r0 + r, gc = c0 + c;
        T v = T(0);
        if (gr < j.rows && gc < j.cols) {
            if constexpr (sizeof(T) == 2) {
                if (j.lo_src) {
                    // bf16 residual of the float32 weight (exact subtraction)
                    const float x = j.lo_src[static_cast<long long>(gr) * j.src_ld + gc];
                    v = f32_to_bf16(x - bf16_to_f32(f32_to_bf16(x)));
                } else {
                    v = src[static_cast<long long>(gr) * j.src_ld + gc];
                }
            } else {
                v = src[static_cast<long long>(gr) * j.src_ld + gc];
            }
        }
        tile[r][c] = v;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kStageTile * kStageTile; e += blockDim.x) {
        const int r = e / kStageTile, c = e % kStageTile;
        if (j.transpose) {
            // destination row c0 + r holds source column c0 + r
            const int dr = c0 + r, dc = r0 + c;
            if (dr < j.cols && dc < j.rows) dst[static_cast<long long>(dr) * j.dst_ld + dc] = tile[c][r];
        } else {
            const int dr = r0 + r, dc = c0 + c;
            if (dr < j.rows && dc < j.dst_ld) dst[static_cast<long long>(dr) * j.dst_ld + dc] = tile[r][c];
        }
    }
}

__global__ void step_advance_kernel(int32_t *step, int k) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *step += k;
}

__global__ void pack_bf16_kernel(const float *theta, uint16_t *shadow, long long n) {
    for (long long e = blockIdx.x * static_cast<long long>(blockDim.x) + threadIdx.x; e < n;
         e += static_cast<long long>(gridDim.x) * blockDim.x)
        shadow[e] = f32_to_bf16(theta[e]);
}

int grid_for(long long n, int threads, int cap) {
    long long b = (n + threads - 1) / threads;
    if (b < 1) b = 1;
    return static_cast<int>(b < cap ? b : cap);
}

}  // namespace

hipError_t launch_philox_blocks(hipStream_t s, uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2,
                                uint32_t c3, long long n, uint32_t *out) {
    const uint32_t k0 = static_cast<uint32_t>(seed), k1 = static_cast<uint32_t>(seed >> 32);
    hipLaunchKernelGGL(philox_blocks_kernel, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, k0, k1, c0, c1, c2, c3,
                       n, out);
    return hipGetLastError();
}

hipError_t launch_gather_obs(Precision prec, hipStream_t s, const float *obs, const int32_t *idx, int src_rows,
                             int rows, int D, int ld, void *out) {
    const long long total = static_cast<long long>(rows) * ld;
    const dim3 grid(grid_for(total, 256, 8192)), block(256);
    if (prec == kBF16)
        hipLaunchKernelGGL(gather_obs_kernel<uint16_t>, grid, block, 0, s, obs, idx, src_rows, rows, D, ld,
                           static_cast<uint16_t *>(out));
    else
        hipLaunchKernelGGL(gather_obs_kernel<float>, grid, block, 0, s, obs, idx, src_rows, rows, D, ld,
                           static_cast<float *>(out));
    return hipGetLastError();
}

// Dynamic LDS for the staged output-layer weights, 0 when they do not fit.
size_t head_weight_lds(int A, int Hl) {
    const size_t bytes = static_cast<size_t>(A + 1) * (Hl + kWPad) * sizeof(float);
    return bytes <= 48 * 1024 ? bytes : 0;
}

hipError_t launch_head_sample(Precision prec, const HeadSampleArgs &a, hipStream_t s) {
    const dim3 grid((a.N + kSampleRows - 1) / kSampleRows), block(kHeadThreads);
    const size_t wsh = head_weight_lds(a.A, a.Hl);
    if (prec == kBF16) {
        const size_t rsh = head_rows_lds<uint16_t>(kSampleRows, a.Hl, wsh);
        hipLaunchKernelGGL(head_sample_kernel<uint16_t>, grid, block, wsh + rsh, s, a, wsh > 0 ? 1 : 0,
                           rsh > 0 ? static_cast<int>(wsh) : -1);
    } else {
        const size_t rsh = head_rows_lds<float>(kSampleRows, a.Hl, wsh);
        hipLaunchKernelGGL(head_sample_kernel<float>, grid, block, wsh + rsh, s, a, wsh > 0 ? 1 : 0,
                           rsh > 0 ? static_cast<int>(wsh) : -1);
    }
    return hipGetLastError();
}

void add_stage_job(StageArgs &a, const StageJob &j) {
    StageJob q = j;
    const int cols_t = q.transpose ? q.cols : q.dst_ld;
    q.tile_begin = a.total_tiles;
    a.job[a.count++] = q;
    a.total_tiles += ((q.rows + kStageTile - 1) / kStageTile) * ((cols_t + kStageTile - 1) / kStageTile);
}

hipError_t launch_stage_weights(Precision prec, const StageArgs &a, hipStream_t s) {
    if (a.count == 0 || a.total_tiles == 0) return hipSuccess;
    const dim3 grid(a.total_tiles), block(256);
    if (prec == kBF16)
        hipLaunchKernelGGL(stage_weights_kernel<uint16_t>, grid, block, 0, s, a);
    else
        hipLaunchKernelGGL(stage_weights_kernel<float>, grid, block, 0, s, a);
    return hipGetLastError();
}

int head_loss_blocks(int M) { return (M + kLossRows - 1) / kLossRows; }
int head_loss_partial_width(int A) { return A + 8; }

hipError_t launch_head_loss(Precision prec, const HeadLossArgs &a, hipStream_t s) {
    const dim3 grid(head_loss_blocks(a.M)), block(kHeadThreads);
    const size_t wsh = head_weight_lds(a.A, a.Hl);
    if (prec == kBF16) {
        const size_t rsh = head_rows_lds<uint16_t>(kLossRows, a.Hl, wsh);
        hipLaunchKernelGGL(head_loss_kernel<uint16_t>, grid, block, wsh + rsh, s, a, wsh > 0 ? 1 : 0,
                           rsh > 0 ? static_cast<int>(wsh) : -1);
    } else {
        const size_t rsh = head_rows_lds<float>(kLossRows, a.Hl, wsh);
        hipLaunchKernelGGL(head_loss_kernel<float>, grid, block, wsh + rsh, s, a, wsh > 0 ? 1 : 0,
                           rsh > 0 ? static_cast<int>(wsh) : -1);
    }
    return hipGetLastError();
}

int gae_blocks(int N) { return (N + kGaeThreads - 1) / kGaeThreads; }

// Scratch of the allocation-free GAE entry point: the Welford partials (three
// doubles per block of kGaeThreads environments) of up to kGaeNoAllocMaxN
// environments, one copy per device for the life of the process.
static __device__ __align__(256) double scratch[3 * ((kGaeNoAllocMaxN + kGaeThreads - 1) / kGaeThreads)];

hipError_t gae_scratch(double **out) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static double *ptr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!ptr[dev]) {
        // the host-side name of the array is not a device address: ask the
        // runtime for this device's copy once, with the device current
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        ptr[dev] = static_cast<double *>(p);
    }
    *out = ptr[dev];
    return hipSuccess;
}

hipError_t launch_gae(const GaeArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(gae_kernel, dim3(gae_blocks(a.N)), dim3(kGaeThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_adv_finalize(const double *partials, int nparts, float *adv, long long count, double *stats_out,
                               int normalize, hipStream_t s) {
    const int blocks = normalize ? grid_for(count, kFinalizeThreads, 1024) : 1;
    hipLaunchKernelGGL(adv_finalize_kernel, dim3(blocks), dim3(kFinalizeThreads), 0, s, partials, nparts, adv, count,
                       stats_out,
                       normalize);
    return hipGetLastError();
}

int reduce_blocks(long long total) { return grid_for(total, kReduceThreads, 1023) + 1; }

hipError_t launch_grad_reduce(const ReduceArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(grad_reduce_kernel, dim3(reduce_blocks(a.total)), dim3(kReduceThreads), 0, s, a);
    return hipGetLastError();
}

int adam_blocks(long long P) { return grid_for(P, kAdamThreads, 1024); }

hipError_t launch_adam(const AdamArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(adam_kernel, dim3(adam_blocks(a.P)), dim3(kAdamThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_step_advance(int32_t *step, int k, hipStream_t s) {
    hipLaunchKernelGGL(step_advance_kernel, dim3(1), dim3(64), 0, s, step, k);
    return hipGetLastError();
}

hipError_t launch_pack_bf16(const float *theta, uint16_t *shadow, long long n, hipStream_t s) {
    hipLaunchKernelGGL(pack_bf16_kernel, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, theta, shadow, n);
    return hipGetLastError();
}

}  // namespace ppo
