// Per-chain pieces of the evolve step: regeneration from the uniform
// distribution on the torus (Alg. 4.2), the Euler-Maruyama move with
// rotational drift (Eq. local-dynamics, Alg. 5.1) and the hold/kill draw of
// Accumulate (Alg. 4.1) with holding rate 1/dt
// (Eq. diffusion-restore-holding-rate) and killing rate k0/(p + eps)
// (Eq. modified-killing-rate).  Chain state is planar: coordinate i of chain
// c at x[i * N] relative to the chain's base pointer.
#pragma once

#include "dr_device.h"

namespace dr {

// x ~ uniform on the torus.  Coordinate i takes word i & 3 of block i >> 2;
// d need only be even (a path's d = 4(L-1) is a multiple of 4; an analytic
// target may end on a half block).
__device__ __forceinline__ void regen(uint64_t seed, int d, size_t N, float* x, int c, uint64_t s) {
    for (int b = 0; b < d / 4; ++b) {
        const uint4 r = rng_block(seed, (uint32_t)c, s, TAG_REGEN, (uint32_t)b);
        x[(size_t)(4 * b + 0) * N] = u24(r.x);
        x[(size_t)(4 * b + 1) * N] = u24(r.y);
        x[(size_t)(4 * b + 2) * N] = u24(r.z);
        x[(size_t)(4 * b + 3) * N] = u24(r.w);
    }
    if (d & 2) {
        const int b = d / 4;
        const uint4 r = rng_block(seed, (uint32_t)c, s, TAG_REGEN, (uint32_t)b);
        x[(size_t)(4 * b + 0) * N] = u24(r.x);
        x[(size_t)(4 * b + 1) * N] = u24(r.y);
    }
}

__device__ __forceinline__ float wrap01(float y) {
    y -= floorf(y);
    return y >= 1.0f ? 0.0f : y;
}

// Euler-Maruyama move with rotational drift, per 2-D block (Alg. 5.1):
// x += (sd^2/2) s + gt (s2, -s1) + sd xi, then wrap to the torus.  Pair i
// takes its normals from words 2i, 2i+1 (block i >> 1); d must be even.
__device__ __forceinline__ void move(uint64_t seed, int d, size_t N, float stddev, float gt, float* x, const float* score,
                                     const float* sigma, int c, uint64_t s) {
    for (int b = 0; b < (d + 2) / 4; ++b) {
        const uint4 r = rng_block(seed, (uint32_t)c, s, TAG_GAUSS, (uint32_t)b);
        const float uu[4] = {u24(r.x), u24(r.y), u24(r.z), u24(r.w)};
        const int npair = 4 * b + 2 < d ? 2 : 1;  // a trailing half block holds one pair
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            if (q >= npair) break;
            const int i0 = 4 * b + 2 * q, i1 = i0 + 1;
            const float rad = sqrtf(-2.0f * logf(1.0f - uu[2 * q]));
            float sn, cs;
            sincosf(2.0f * DR_PI * uu[2 * q + 1], &sn, &cs);
            const float xi0 = rad * cs, xi1 = rad * sn;
            const size_t a0 = (size_t)i0 * N, a1 = (size_t)i1 * N;
            const float s0 = score[a0], s1 = score[a1];
            const float sd0 = sigma ? sigma[a0] : stddev;
            const float sd1 = sigma ? sigma[a1] : stddev;
            const float y0 = x[a0] + 0.5f * sd0 * sd0 * s0 + gt * s1 + sd0 * xi0;
            const float y1 = x[a1] + 0.5f * sd1 * sd1 * s1 - gt * s0 + sd1 * xi1;
            x[a0] = wrap01(y0);
            x[a1] = wrap01(y1);
        }
    }
}

// Competing exponential clocks E_a (hold) and E_b (kill): the tour survives
// if k dt E_a < E_b.  wdt receives the splat weight in units of dt: the
// Rao-Blackwellised 1/(1 + k dt) = E[holding time]/dt, or the sampled
// min(E_a, E_b/(k dt)).
__device__ __forceinline__ bool hold_kill(uint64_t seed, int c, uint64_t s, float k0, float p, float eps, float dt,
                                          int rb, float& wdt) {
    const uint4 r = rng_block(seed, (uint32_t)c, s, TAG_HOLD, 0);
    const float Ea = -logf(1.0f - u24(r.x));
    const float Eb = -logf(1.0f - u24(r.y));
    const float k = k0 / (p + eps);
    wdt = rb ? 1.0f / (1.0f + k * dt) : fminf(Ea, Eb / (k * dt));
    return (k * dt) * Ea < Eb;
}

}  // namespace dr
