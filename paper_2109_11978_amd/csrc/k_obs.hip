// Observation assembly in front of policy inference (Section 3.2, what the
// policy observes; appendix Table 4, observation noise): the proprioceptive
// columns, then terrain heights sampled around each robot's base from a height
// field on a uniform grid, each element plus uniform noise of its own scale.
//
// One thread per (environment, group of 4 columns): one Philox4x32-10 block
// gives the 4 noise draws of the group, as in the action sampling.  The output
// row of an environment is written by ceil(D / 4) adjacent lanes, so a wave's
// stores cover contiguous memory.  The height field (a few MB at most) stays in
// L2 across the scan points of neighbouring robots.
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

__global__ __launch_bounds__(256) void assemble_obs_kernel(ObsArgs a) {
#pragma clang fp contract(off)
    const long long q = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (q >= a.N * a.groups) return;
    const long long n = q / a.groups;
    const int g = static_cast<int>(q - n * a.groups);
    uint32_t x[4] = {static_cast<uint32_t>(q), a.t, a.iteration, kTagObsNoise};
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
    float *row = a.obs + n * a.D;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int j = 4 * g + i;
        if (j >= a.D) break;
        float v = j < a.P ? a.proprio[n * a.P + j] : bz - cell_height(a, j - a.P, bx, by, bc, bs);
        if (a.noise_scale) {
            // 2u - 1 is exact in float32: u = (k + 1/2) 2^-23 with k < 2^23
            const float e = 2.0f * uniform23(x[i]) - 1.0f;
            const float w = a.noise_scale[j] * e;
            v = v + w;
        }
        row[j] = v;
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
    const long long threads = N * a.groups;
    hipLaunchKernelGGL(assemble_obs_kernel, dim3(static_cast<unsigned>((threads + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace ppo
