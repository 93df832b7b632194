// The chain step on an analytic target: a wrapped Gaussian mixture on the
// torus T^d with a constant floor,
//   p(x) = c0 + sum_j w_j prod_i N_wrap(x_i; m_ji, s_j^2),
// and f = p g with the test functions g = (1, cos 2 pi x_i, sin 2 pi x_i).
// The Restore estimator k0 accum / tourCount then converges to
// lambda(p g) = (c0 + sum_j w_j, sum_j w_j exp(-2 pi^2 s_j^2) cos / sin 2 pi m_ji),
// which pins the chain machinery (regeneration, the Euler-Maruyama move with
// rotation and per-chain Sigma, hold/kill with the estimated k0, the holding
// weights, the ratio estimator; Alg. 4.1-4.3, Alg. 5.1) on the device against
// closed forms, with the same per-chain pieces (dr_chain.h) and random streams
// as the path-space chain step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "../../include/dr.h"
#include "dr_chain.h"

// Sets the thread's dr_last_error() message (dr_lib.hip).
void dr_set_last_error(const char* msg);

using namespace dr;

namespace {

constexpr int kMaxModes = 16;
constexpr int kBlock = 256;

struct MixDev {
    const float* w;      // n_modes
    const float* s;      // n_modes
    const float* mean;   // n_modes x d
    int nm;
    float c0;
};

struct MixParams {
    uint64_t seed;
    int N;
    float stddev, dt, gt, eps;
    int rb;
};

// p(x) and its gradient.  Each factor is the wrapped normal density summed
// over the images z - 2 .. z + 2 of the nearest-image difference z (further
// images are below FP32 resolution for s <= 0.25).
template <int D>
__device__ __forceinline__ float mix_eval(const MixDev& M, const float (&x)[D], float (&grad)[D]) {
    float p = M.c0;
#pragma unroll
    for (int i = 0; i < D; ++i) grad[i] = 0.0f;
    for (int j = 0; j < M.nm; ++j) {
        const float sj = M.s[j];
        const float inv2 = 1.0f / (sj * sj);
        const float norm = 1.0f / (sj * 2.50662827463100050f);  // 1 / (s sqrt(2 pi))
        float fac[D], dfac[D];
#pragma unroll
        for (int i = 0; i < D; ++i) {
            float z0 = x[i] - M.mean[j * D + i];
            z0 -= rintf(z0);
            float acc = 0.0f, dacc = 0.0f;
#pragma unroll
            for (int k = -2; k <= 2; ++k) {
                const float z = z0 + (float)k;
                const float e = expf(-0.5f * z * z * inv2) * norm;
                acc += e;
                dacc -= z * inv2 * e;
            }
            fac[i] = acc;
            dfac[i] = dacc;
        }
        // prefix and suffix products give prod_{k != i} fac_k without division
        float pre[D + 1];
        pre[0] = M.w[j];
#pragma unroll
        for (int i = 0; i < D; ++i) pre[i + 1] = pre[i] * fac[i];
        p += pre[D];
        float suf = 1.0f;
#pragma unroll
        for (int i = D - 1; i >= 0; --i) {
            grad[i] += pre[i] * dfac[i] * suf;
            suf *= fac[i];
        }
    }
    return p;
}

template <int D>
__device__ __forceinline__ void load_x(const float* x, int N, int c, float (&xr)[D]) {
#pragma unroll
    for (int i = 0; i < D; ++i) xr[i] = x[(size_t)i * N + c];
}

// score = grad p / (p + eps); a non-finite component is set to 0.
template <int D>
__device__ __forceinline__ void store_score(float* score, int N, int c, const float (&g)[D], float p, float eps) {
#pragma unroll
    for (int i = 0; i < D; ++i) {
        const float v = g[i] / (p + eps);
        score[(size_t)i * N + c] = isfinite(v) ? v : 0.0f;
    }
}

// Initialise, phase 1: x ~ uniform, p(x) (Alg. 4.1).
template <int D>
__global__ void __launch_bounds__(kBlock) k_mix_init_eval(MixDev M, MixParams P, uint64_t s0, float* x, float* p_out) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= P.N) return;
    regen(P.seed, D, P.N, x + c, c, s0);
    float xr[D], g[D];
    load_x<D>(x, P.N, c, xr);
    p_out[c] = mix_eval<D>(M, xr, g);
}

// Sum of p in FP64: per-block partials (fixed order), then one thread.
__global__ void __launch_bounds__(kBlock) k_mix_sum(const float* p, int N, double* partial) {
    __shared__ double sh[kBlock];
    double acc = 0.0;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < N; c += gridDim.x * blockDim.x) acc += (double)p[c];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}
// k0 = p_lambda / (m dt) with p_lambda the mean of p (Eq. killing-rate-constant),
// unless given; scal[0] = k0 (FP64), scal[1] = p_lambda, and the FP32 k0 the
// chains use after them.
__global__ void k_mix_k0(const double* partial, int nparts, int N, double k0_given, double m, double dt, double eps,
                         double* scal) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int i = 0; i < nparts; ++i) s += partial[i];
    const double pl = s / (double)N;
    double k0 = k0_given;
    if (!(k0 > 0.0)) k0 = pl > 0.0 ? pl / (m * dt) : eps / (m * dt);
    scal[0] = k0;
    scal[1] = pl;
    reinterpret_cast<float*>(scal + 2)[0] = (float)k0;
}

// Test functions g = (1, cos 2 pi x_i, sin 2 pi x_i) added with weight wdt.
template <int D>
__device__ __forceinline__ void splat(double (&acc)[1 + 2 * D], const float (&xr)[D], float wdt) {
    acc[0] += (double)wdt;
#pragma unroll
    for (int i = 0; i < D; ++i) {
        float sn, cs;
        sincosf(2.0f * DR_PI * xr[i], &sn, &cs);
        acc[1 + 2 * i] += (double)(wdt * cs);
        acc[2 + 2 * i] += (double)(wdt * sn);
    }
}

// Initialise phase 2 (hold/kill/splat of the initial states with the final
// k0, scores of the survivors), then n_steps evolve steps (Alg. 4.2 with
// Alg. 5.1), one thread per chain.  Each thread sums its splats in FP64; a
// block's sums and tour count go to partial[block] (1 + 2D accumulators, in
// units of dt) and tours[block].
template <int D>
__global__ void __launch_bounds__(kBlock) k_mix_run(MixDev M, MixParams P, uint64_t s0, uint32_t n_steps,
                                                    const double* scal, float* x, float* score, uint32_t* killed,
                                                    const float* p0, const float* sigma, double* partial,
                                                    unsigned long long* tours) {
    constexpr int NF = 1 + 2 * D;
    __shared__ double sh[kBlock];
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const float k0 = reinterpret_cast<const float*>(scal + 2)[0];
    double acc[NF];
#pragma unroll
    for (int q = 0; q < NF; ++q) acc[q] = 0.0;
    uint32_t kills = 0;
    if (c < P.N) {
        float xr[D], g[D];
        load_x<D>(x, P.N, c, xr);
        float p = p0[c];
        float wdt;
        bool alive = hold_kill(P.seed, c, s0, k0, p, P.eps, P.dt, P.rb, wdt);
        if (p > 0.0f) splat<D>(acc, xr, wdt);
        if (alive) {
            mix_eval<D>(M, xr, g);
            store_score<D>(score, P.N, c, g, p, P.eps);
        }
        kills += alive ? 0u : 1u;
        for (uint32_t k = 1; k <= n_steps; ++k) {
            const uint64_t s = s0 + k;
            if (!alive) regen(P.seed, D, P.N, x + c, c, s);
            else move(P.seed, D, P.N, P.stddev, P.gt, x + c, score + c, sigma ? sigma + c : nullptr, c, s);
            load_x<D>(x, P.N, c, xr);
            p = mix_eval<D>(M, xr, g);
            alive = hold_kill(P.seed, c, s, k0, p, P.eps, P.dt, P.rb, wdt);
            if (p > 0.0f) splat<D>(acc, xr, wdt);
            if (alive) store_score<D>(score, P.N, c, g, p, P.eps);
            kills += alive ? 0u : 1u;
        }
        killed[c] = alive ? 0u : 1u;
    }
#pragma unroll
    for (int q = 0; q <= NF; ++q) {
        sh[threadIdx.x] = q < NF ? acc[q] : (double)kills;
        __syncthreads();
        for (int o = blockDim.x / 2; o > 0; o >>= 1) {
            if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            if (q < NF) partial[(size_t)blockIdx.x * NF + q] = sh[0];
            else tours[blockIdx.x] = (unsigned long long)sh[0];
        }
        __syncthreads();
    }
}

// One evolve step from a given state (x, score, killed at step s): the same
// arithmetic as k_mix_run's loop body; outputs the new state, p and the
// splat weight w (time units).
template <int D>
__global__ void __launch_bounds__(kBlock) k_mix_step(MixDev M, MixParams P, uint64_t s, float k0, float* x,
                                                     float* score, uint32_t* killed, const float* sigma, float* p_out,
                                                     float* w_out) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= P.N) return;
    if (killed[c]) regen(P.seed, D, P.N, x + c, c, s);
    else move(P.seed, D, P.N, P.stddev, P.gt, x + c, score + c, sigma ? sigma + c : nullptr, c, s);
    float xr[D], g[D];
    load_x<D>(x, P.N, c, xr);
    const float p = mix_eval<D>(M, xr, g);
    float wdt;
    const bool alive = hold_kill(P.seed, c, s, k0, p, P.eps, P.dt, P.rb, wdt);
    if (alive) store_score<D>(score, P.N, c, g, p, P.eps);
    killed[c] = alive ? 0u : 1u;
    p_out[c] = p;
    w_out[c] = wdt * P.dt;
}

dr_status mfail(dr_status s, const std::string& m) {
    dr_set_last_error(("dr_mixture: " + m).c_str());
    return s;
}

// Validate a mixture description and parameters, copy the modes to the
// device.  On success *buf holds w[nm], s[nm], mean[nm x d].
dr_status mix_prepare(const dr_mixture_desc* m, const dr_params* p, std::vector<float>& host) {
    if (!m || !p) return mfail(DR_ERR_INVALID_ARG, "null argument");
    if (m->d < 2 || m->d > 16 || (m->d & 1)) return mfail(DR_ERR_INVALID_ARG, "d must be even, 2..16");
    if (m->n_modes > (uint32_t)kMaxModes) return mfail(DR_ERR_INVALID_ARG, "at most 16 modes");
    if (m->n_modes && (!m->weights || !m->means || !m->stds)) return mfail(DR_ERR_INVALID_ARG, "null mode arrays");
    if (!(m->c0 >= 0.0f) || !std::isfinite(m->c0)) return mfail(DR_ERR_INVALID_ARG, "c0 must be finite and >= 0");
    double total = m->c0;
    for (uint32_t j = 0; j < m->n_modes; ++j) {
        if (!(m->stds[j] > 0.0f && m->stds[j] <= 0.25f)) return mfail(DR_ERR_INVALID_ARG, "stds must be in (0, 0.25]");
        if (!(m->weights[j] >= 0.0f) || !std::isfinite(m->weights[j]))
            return mfail(DR_ERR_INVALID_ARG, "weights must be finite and >= 0");
        total += m->weights[j];
    }
    if (!(total > 0.0)) return mfail(DR_ERR_INVALID_ARG, "the density is zero");
    if (p->n_chains == 0) return mfail(DR_ERR_INVALID_ARG, "n_chains must be >= 1");
    if (!(p->dt > 0.0f) || !(p->m > 0.0f) || !(p->eps > 0.0f) || !(p->stddev > 0.0f))
        return mfail(DR_ERR_INVALID_ARG, "stddev, dt, m and eps must be > 0");
    const uint32_t nm = m->n_modes, d = m->d;
    host.assign(2 * nm + (size_t)nm * d + 1, 0.0f);
    for (uint32_t j = 0; j < nm; ++j) {
        host[j] = m->weights[j];
        host[nm + j] = m->stds[j];
        for (uint32_t i = 0; i < d; ++i) host[2 * nm + (size_t)j * d + i] = m->means[(size_t)j * d + i];
    }
    return DR_OK;
}

struct DevBufs {
    std::vector<void*> ptrs;
    hipError_t get(void** p, size_t bytes) {
        const hipError_t e = hipMalloc(p, bytes ? bytes : 4);
        if (e == hipSuccess) ptrs.push_back(*p);
        return e;
    }
    ~DevBufs() {
        for (void* q : ptrs) (void)hipFree(q);
    }
};

#define MIX_DISPATCH(D, FN, ...)               \
    switch (D) {                               \
        case 2: FN<2>(__VA_ARGS__); break;     \
        case 4: FN<4>(__VA_ARGS__); break;     \
        case 6: FN<6>(__VA_ARGS__); break;     \
        case 8: FN<8>(__VA_ARGS__); break;     \
        case 10: FN<10>(__VA_ARGS__); break;   \
        case 12: FN<12>(__VA_ARGS__); break;   \
        case 14: FN<14>(__VA_ARGS__); break;   \
        case 16: FN<16>(__VA_ARGS__); break;   \
        default: break;                        \
    }

template <int D>
void launch_mix_init(int blocks, hipStream_t st, const MixDev& M, const MixParams& P, uint64_t s0, float* x, float* p) {
    hipLaunchKernelGGL(k_mix_init_eval<D>, dim3(blocks), dim3(kBlock), 0, st, M, P, s0, x, p);
}
template <int D>
void launch_mix_run(int blocks, hipStream_t st, const MixDev& M, const MixParams& P, uint64_t s0, uint32_t n,
                    const double* scal, float* x, float* score, uint32_t* killed, const float* p0, const float* sigma,
                    double* partial, unsigned long long* tours) {
    hipLaunchKernelGGL(k_mix_run<D>, dim3(blocks), dim3(kBlock), 0, st, M, P, s0, n, scal, x, score, killed, p0,
                       sigma, partial, tours);
}
template <int D>
void launch_mix_step(int blocks, hipStream_t st, const MixDev& M, const MixParams& P, uint64_t s, float k0, float* x,
                     float* score, uint32_t* killed, const float* sigma, float* p, float* w) {
    hipLaunchKernelGGL(k_mix_step<D>, dim3(blocks), dim3(kBlock), 0, st, M, P, s, k0, x, score, killed, sigma, p, w);
}

MixParams mix_params(const dr_params* p, uint64_t seed) {
    MixParams P;
    P.seed = seed;
    P.N = (int)p->n_chains;
    P.stddev = p->stddev;
    P.dt = p->dt;
    P.gt = p->dt * p->gamma / 2.0f;
    P.eps = p->eps;
    P.rb = p->rao_blackwell ? 1 : 0;
    return P;
}

}  // namespace

#define MIX_TRY(expr)                                                                                 \
    do {                                                                                              \
        const hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess) return mfail(DR_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

extern "C" {

dr_status dr_mixture_run(const dr_mixture_desc* m, const dr_params* p, uint64_t seed, uint32_t frame, uint32_t n_steps,
                         uint32_t n_batches, double* batch_accum, uint64_t* batch_tours, double* k0_out,
                         double* p_lambda_out, void* hip_stream) {
    std::vector<float> host;
    dr_status r = mix_prepare(m, p, host);
    if (r != DR_OK) return r;
    if (n_batches == 0 || !batch_accum || !batch_tours) return mfail(DR_ERR_INVALID_ARG, "need n_batches >= 1 and outputs");
    const int D = (int)m->d, NF = 1 + 2 * D, N = (int)p->n_chains;
    const int blocks = (N + kBlock - 1) / kBlock;
    hipStream_t st = (hipStream_t)hip_stream;
    DevBufs mem;
    void *modes, *x, *score, *killed, *p0, *partial, *tours, *scal;
    MIX_TRY(mem.get(&modes, sizeof(float) * host.size()));
    MIX_TRY(mem.get(&x, sizeof(float) * (size_t)D * N));
    MIX_TRY(mem.get(&score, sizeof(float) * (size_t)D * N));
    MIX_TRY(mem.get(&killed, sizeof(uint32_t) * (size_t)N));
    MIX_TRY(mem.get(&p0, sizeof(float) * (size_t)N));
    MIX_TRY(mem.get(&partial, sizeof(double) * (size_t)blocks * NF));
    MIX_TRY(mem.get(&tours, sizeof(unsigned long long) * (size_t)blocks));
    MIX_TRY(mem.get(&scal, 64));
    MIX_TRY(hipMemcpyAsync(modes, host.data(), sizeof(float) * host.size(), hipMemcpyHostToDevice, st));
    const uint32_t nm = m->n_modes;
    MixDev M{(const float*)modes, (const float*)modes + nm, (const float*)modes + 2 * nm, (int)nm, m->c0};
    const MixParams P = mix_params(p, seed);
    const uint64_t s0 = (uint64_t)frame << 32;
    (void)hipGetLastError();
    MIX_DISPATCH(D, launch_mix_init, blocks, st, M, P, s0, (float*)x, (float*)p0);
    const int parts = std::min(1024, blocks);
    hipLaunchKernelGGL(k_mix_sum, dim3(parts), dim3(kBlock), 0, st, (const float*)p0, N, (double*)partial);
    hipLaunchKernelGGL(k_mix_k0, dim3(1), dim3(64), 0, st, (const double*)partial, parts, N, (double)p->k0,
                       (double)p->m, (double)p->dt, (double)p->eps, (double*)scal);
    MIX_DISPATCH(D, launch_mix_run, blocks, st, M, P, s0, n_steps, (const double*)scal, (float*)x, (float*)score,
                 (uint32_t*)killed, (const float*)p0, p->sigma_diag, (double*)partial, (unsigned long long*)tours);
    MIX_TRY(hipGetLastError());
    std::vector<double> hp((size_t)blocks * NF), hs(2);
    std::vector<unsigned long long> ht(blocks);
    MIX_TRY(hipMemcpyAsync(hp.data(), partial, sizeof(double) * hp.size(), hipMemcpyDeviceToHost, st));
    MIX_TRY(hipMemcpyAsync(ht.data(), tours, sizeof(unsigned long long) * ht.size(), hipMemcpyDeviceToHost, st));
    MIX_TRY(hipMemcpyAsync(hs.data(), scal, sizeof(double) * 2, hipMemcpyDeviceToHost, st));
    MIX_TRY(hipStreamSynchronize(st));
    for (size_t i = 0; i < (size_t)n_batches * NF; ++i) batch_accum[i] = 0.0;
    for (uint32_t i = 0; i < n_batches; ++i) batch_tours[i] = 0;
    for (int b = 0; b < blocks; ++b) {
        const int q = b % (int)n_batches;
        for (int k = 0; k < NF; ++k) batch_accum[(size_t)q * NF + k] += hp[(size_t)b * NF + k];
        batch_tours[q] += ht[b];
    }
    if (k0_out) *k0_out = hs[0];
    if (p_lambda_out) *p_lambda_out = hs[1];
    dr_set_last_error("");
    return DR_OK;
}

dr_status dr_mixture_step(const dr_mixture_desc* m, const dr_params* p, uint64_t seed, uint64_t step, double k0,
                          float* x, float* score, uint32_t* killed, float* p_out, float* w_out, void* hip_stream) {
    std::vector<float> host;
    dr_status r = mix_prepare(m, p, host);
    if (r != DR_OK) return r;
    if (!x || !score || !killed || !p_out || !w_out) return mfail(DR_ERR_INVALID_ARG, "null state array");
    if (!(k0 > 0.0)) return mfail(DR_ERR_INVALID_ARG, "k0 must be > 0");
    const int D = (int)m->d, N = (int)p->n_chains;
    for (int c = 0; c < N; ++c)
        if (killed[c] > 1) return mfail(DR_ERR_INVALID_ARG, "killed must be 0/1");
    const int blocks = (N + kBlock - 1) / kBlock;
    hipStream_t st = (hipStream_t)hip_stream;
    DevBufs mem;
    void *modes, *dx, *ds, *dk, *dp, *dw;
    MIX_TRY(mem.get(&modes, sizeof(float) * host.size()));
    MIX_TRY(mem.get(&dx, sizeof(float) * (size_t)D * N));
    MIX_TRY(mem.get(&ds, sizeof(float) * (size_t)D * N));
    MIX_TRY(mem.get(&dk, sizeof(uint32_t) * (size_t)N));
    MIX_TRY(mem.get(&dp, sizeof(float) * (size_t)N));
    MIX_TRY(mem.get(&dw, sizeof(float) * (size_t)N));
    MIX_TRY(hipMemcpyAsync(modes, host.data(), sizeof(float) * host.size(), hipMemcpyHostToDevice, st));
    MIX_TRY(hipMemcpyAsync(dx, x, sizeof(float) * (size_t)D * N, hipMemcpyHostToDevice, st));
    MIX_TRY(hipMemcpyAsync(ds, score, sizeof(float) * (size_t)D * N, hipMemcpyHostToDevice, st));
    MIX_TRY(hipMemcpyAsync(dk, killed, sizeof(uint32_t) * (size_t)N, hipMemcpyHostToDevice, st));
    const uint32_t nm = m->n_modes;
    MixDev M{(const float*)modes, (const float*)modes + nm, (const float*)modes + 2 * nm, (int)nm, m->c0};
    const MixParams P = mix_params(p, seed);
    (void)hipGetLastError();
    MIX_DISPATCH(D, launch_mix_step, blocks, st, M, P, step, (float)k0, (float*)dx, (float*)ds, (uint32_t*)dk,
                 p->sigma_diag, (float*)dp, (float*)dw);
    MIX_TRY(hipGetLastError());
    MIX_TRY(hipMemcpyAsync(x, dx, sizeof(float) * (size_t)D * N, hipMemcpyDeviceToHost, st));
    MIX_TRY(hipMemcpyAsync(score, ds, sizeof(float) * (size_t)D * N, hipMemcpyDeviceToHost, st));
    MIX_TRY(hipMemcpyAsync(killed, dk, sizeof(uint32_t) * (size_t)N, hipMemcpyDeviceToHost, st));
    MIX_TRY(hipMemcpyAsync(p_out, dp, sizeof(float) * (size_t)N, hipMemcpyDeviceToHost, st));
    MIX_TRY(hipMemcpyAsync(w_out, dw, sizeof(float) * (size_t)N, hipMemcpyDeviceToHost, st));
    MIX_TRY(hipStreamSynchronize(st));
    dr_set_last_error("");
    return DR_OK;
}

}  // extern "C"
