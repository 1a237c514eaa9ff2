// Observation assembly in front of policy inference (Section 3.2, what the
// policy observes; appendix Table 4, observation noise): the proprioceptive
// columns, then terrain heights sampled around each robot's base from a height
// field on a uniform grid, each element plus uniform noise of its own scale.
//
// A block takes up to 16 robots (fewer at small N, to fill the chip): one
// thread per (robot, group of 4 columns) draws one Philox4x32-10 block for the
// group's 4 noise values, as in the action sampling, and puts the group's
// values in LDS; then the block writes its robots' rows, one contiguous range
// of the output, with 16-byte stores.  The
// height field (a few MB at most) stays in L2 across the scan points of
// neighbouring robots.
#include <algorithm>

#include "common.hpp"
#include "philox.hpp"

namespace ppo {
namespace {

constexpr uint32_t kTagObsNoise = 2;  // counter word 3: 1 is the action noise

struct ObsArgs {
    const float *proprio;      // [N, P]
    const float *base;         // [N, 5]: x, y, z, cos(yaw), sin(yaw)
    const float *height;       // [nx, ny]
    const float *scan;         // [S, 2]
    const float *noise_scale;  // [D] or null
    float *obs;                // [N, D]
    long long N;
    int P, S, D, groups, nx, ny;
    int rows_per_block;        // robots per workgroup, rows_per_block * D floats of LDS
    float inv_res;
    uint32_t k0, k1, t, iteration;
};

// Height of the cell nearest to scan point k of a robot at (x, y) with heading
// (c, s).  The index is a rounding decision, so every product and sum is
// rounded on its own (no fused multiply-add): the world point is
// x + (c px - s py), y + (s px + c py), the cell rint(w * inv_res), clamped
// (fmax/fmin return the other operand for a NaN, so a NaN point reads cell 0).
__device__ inline float cell_height(const ObsArgs &a, int k, float x, float y, float c, float s) {
#pragma clang fp contract(off)
    const float px = a.scan[2 * k], py = a.scan[2 * k + 1];
    const float wx = x + (c * px - s * py);
    const float wy = y + (s * px + c * py);
    const float fi = fminf(fmaxf(rintf(wx * a.inv_res), 0.0f), static_cast<float>(a.nx - 1));
    const float fj = fminf(fmaxf(rintf(wy * a.inv_res), 0.0f), static_cast<float>(a.ny - 1));
    return a.height[static_cast<long long>(fi) * a.ny + static_cast<int>(fj)];
}

// Value of column j of robot n (j in its Philox group with draw x).
__device__ inline float obs_value(const ObsArgs &a, long long n, int j, uint32_t x, float bx, float by, float bz,
                                  float bc, float bs) {
#pragma clang fp contract(off)
    float v = j < a.P ? a.proprio[n * a.P + j] : bz - cell_height(a, j - a.P, bx, by, bc, bs);
    if (a.noise_scale) {
        // 2u - 1 is exact in float32: u = (k + 1/2) 2^-23 with k < 2^23
        const float e = 2.0f * uniform23(x) - 1.0f;
        const float w = a.noise_scale[j] * e;
        v = v + w;
    }
    return v;
}

// One block per rows_per_block robots.  Phase 1: one thread per (robot, group
// of 4 columns) computes the group's values into LDS.  Phase 2: the block's
// rows are one contiguous range of obs, written with 16-byte stores when the
// range starts 16-byte aligned (always when rows_per_block * D is a multiple
// of 4 and obs is aligned), else with 4-byte stores.
constexpr int kObsRows = 16;                 // robots per block at most (D <= 1024)
constexpr int kObsLdsFloats = 16 * 1024;     // 64 KB of staging at most
constexpr int kObsThreads = 256;
constexpr long long kObsMinBlocks = 1024;   // workgroups to aim for at small N

__global__ __launch_bounds__(kObsThreads) void assemble_obs_kernel(ObsArgs a) {
#pragma clang fp contract(off)
    extern __shared__ float s_obs[];   // [rows * D]
    const long long n0 = static_cast<long long>(blockIdx.x) * a.rows_per_block;
    const int rows = static_cast<int>(a.N - n0 < a.rows_per_block ? a.N - n0 : a.rows_per_block);
    const int work = rows * a.groups;
    for (int q = threadIdx.x; q < work; q += kObsThreads) {
        const int r = q / a.groups;
        const int g = q - r * a.groups;
        const long long n = n0 + r;
        uint32_t x[4] = {static_cast<uint32_t>(n * a.groups + g), a.t, a.iteration, kTagObsNoise};
        if (a.noise_scale) philox4x32_10(x, a.k0, a.k1);
        float bx = 0.0f, by = 0.0f, bz = 0.0f, bc = 1.0f, bs = 0.0f;
        if (4 * g + 3 >= a.P && a.S > 0) {
            const float *b = a.base + 5 * n;
            bx = b[0];
            by = b[1];
            bz = b[2];
            bc = b[3];
            bs = b[4];
        }
        float *row = s_obs + r * a.D;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int j = 4 * g + i;
            if (j < a.D) row[j] = obs_value(a, n, j, x[i], bx, by, bz, bc, bs);
        }
    }
    __syncthreads();
    float *dst = a.obs + n0 * a.D;
    const int total = rows * a.D;
    if ((reinterpret_cast<uintptr_t>(dst) & 15) == 0) {
        const int v4 = total / 4;
        for (int i = threadIdx.x; i < v4; i += kObsThreads) {
            const float4 v = make_float4(s_obs[4 * i], s_obs[4 * i + 1], s_obs[4 * i + 2], s_obs[4 * i + 3]);
            *reinterpret_cast<float4 *>(dst + 4 * i) = v;
        }
        for (int i = 4 * v4 + threadIdx.x; i < total; i += kObsThreads) dst[i] = s_obs[i];
    } else {
        for (int i = threadIdx.x; i < total; i += kObsThreads) dst[i] = s_obs[i];
    }
}

}  // namespace

hipError_t launch_assemble_obs(hipStream_t s, const float *proprio, int P, const float *base, const float *height,
                               int nx, int ny, float inv_res, const float *scan, int S, const float *noise_scale,
                               long long N, uint64_t seed, uint32_t t, uint32_t iteration, float *obs) {
    ObsArgs a;
    a.proprio = proprio;
    a.base = base;
    a.height = height;
    a.scan = scan;
    a.noise_scale = noise_scale;
    a.obs = obs;
    a.N = N;
    a.P = P;
    a.S = S;
    a.D = P + S;
    a.groups = (a.D + 3) / 4;
    a.nx = nx;
    a.ny = ny;
    a.inv_res = inv_res;
    a.k0 = static_cast<uint32_t>(seed);
    a.k1 = static_cast<uint32_t>(seed >> 32);
    a.t = t;
    a.iteration = iteration;
    // fewer robots per workgroup when there are few robots: at least about
    // 1024 workgroups (four per compute unit), so a thread's share of a block
    // is one (robot, group) item with its chain of dependent loads rather
    // than several in a row
    const long long fill = (N + kObsMinBlocks - 1) / kObsMinBlocks;
    a.rows_per_block = static_cast<int>(std::max<long long>(
        1, std::min<long long>(std::min(kObsRows, kObsLdsFloats / a.D), fill)));
    const long long blocks = (N + a.rows_per_block - 1) / a.rows_per_block;
    const size_t lds = static_cast<size_t>(a.rows_per_block) * a.D * sizeof(float);
    hipLaunchKernelGGL(assemble_obs_kernel, dim3(static_cast<unsigned>(blocks)), dim3(kObsThreads), lds, s, a);
    return hipGetLastError();
}

}  // namespace ppo
