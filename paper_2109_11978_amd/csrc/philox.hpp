// Counter-based action noise shared by the sampling kernels: Philox4x32-10
// (Salmon et al., SC'11) and a Box-Muller transform of its 32-bit outputs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ppo {

// Ten rounds of two 32x32->64-bit multiplies with key bumps by the Weyl
// constants between rounds.
__device__ inline void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t a = c[0], b = c[2];
        const uint32_t hi_a = __umulhi(0xD2511F53u, a), lo_a = 0xD2511F53u * a;
        const uint32_t hi_b = __umulhi(0xCD9E8D57u, b), lo_b = 0xCD9E8D57u * b;
        c[0] = hi_b ^ c[1] ^ k0;
        c[1] = lo_b;
        c[2] = hi_a ^ c[3] ^ k1;
        c[3] = lo_a;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// Top 23 bits plus half a step: exact in float32, strictly inside (0, 1).
__device__ inline float uniform23(uint32_t x) { return (static_cast<float>(x >> 9) + 0.5f) * 1.1920928955078125e-07f; }

__device__ inline void box_muller(uint32_t xa, uint32_t xb, float &ea, float &eb) {
    const float r = sqrtf(-2.0f * logf(uniform23(xa)));
    float s, c;
    sincospif(2.0f * uniform23(xb), &s, &c);
    ea = r * c;
    eb = r * s;
}

}  // namespace ppo
