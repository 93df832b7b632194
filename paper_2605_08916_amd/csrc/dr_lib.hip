// Diffusion Restore chain-step library: kernels and the C ABI (include/dr.h).
//
// Two forms of the evolve step run the same arithmetic and draw the same
// Philox streams:
//  * fused: one persistent kernel per dr_step.  Wavefronts pull chains from a
//    device work queue (one atomic per wavefront pop, ballot-compacted), and
//    each lane runs its chain's steps: regenerate or move, one forward path
//    trace, hold/kill, splat, and, for survivors, the reverse-mode adjoint that
//    yields the score used by the next move.  One traversal per chain-step.
//  * plain: the paper's pass structure as separate kernels with the state
//    round-tripping through HBM: score (a forward trace plus the adjoint at the
//    current state, which Alg. 5.1 starts from), move/regenerate, forward trace at the new
//    state (Accumulate), hold/kill/splat.  Two traversals per chain-step.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/dr.h"
#include "dr_kernels.h"

extern "C" dr_status dr_bvh_build_impl(const float* vertices, uint32_t n_vertices, const uint32_t* indices,
                                       uint32_t n_triangles, uint32_t max_leaf, dr_bvh_node* nodes_out,
                                       uint32_t* n_nodes_out, uint32_t* prim_order_out, const char** err);

// ===========================================================================
// Kernels
// ===========================================================================
__global__ void k_fill_u32(uint32_t* a, size_t n, uint32_t v) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) a[i] = v;
}
__global__ void k_fill_f32(float* a, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) a[i] = 0.f;
}
__global__ void k_fill_u64(unsigned long long* a, int n) {
    if (threadIdx.x < (unsigned)n) a[threadIdx.x] = 0ull;
}

// Start of an evolve launch of n steps: reset the work queue and advance the
// device step counter (one thread).
__global__ void k_begin_launch(KBufs B, uint32_t n) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    *B.queue = 0u;
    B.steps[1] = B.steps[0];
    B.steps[0] += n;
}
// Start of an initialise pass: frame index `frame`, or the device frame
// counter plus one when from_device (a captured frame advances it each replay);
// the pass uses step frame << 32 and the next step is that plus one.
__global__ void k_begin_init(KBufs B, uint32_t frame, int from_device) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const unsigned long long f = from_device ? B.steps[2] + 1ull : (unsigned long long)frame;
    B.steps[2] = f;
    B.steps[1] = f << 32;
    B.steps[0] = (f << 32) + 1ull;
    *B.queue = 0u;  // the init kernel's work queue
}

// Initialise, phase 1: x ~ mu and f(x) for every chain (Alg. 4.1).  DELTA:
// the scene has smooth conductors or dielectrics.  Persistent: each wavefront
// takes the next 64 consecutive chains from the work queue (one atomic) until
// the queue is drained, so a wavefront slot never idles waiting for the other
// wavefronts of its block.  Registers capped for three wavefronts per SIMD,
// as in the one-lane evolve kernel.
template <bool DELTA>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
k_init_eval(KParams P, DevScene S, KBufs B) {
    extern __shared__ uint32_t s_stack[];
    uint32_t* stk = s_stack + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const uint64_t s0 = B.steps[1];
    Counters ctr = {0, 0, 0};
    while (true) {
        uint32_t base = 0;
        if (lane == 0) base = atomicAdd(B.queue, 64u);
        base = __shfl(base, 0);
        if (base >= (uint32_t)P.N) break;
        const int c = (int)base + lane;
        if (c >= P.N) continue;
        regen(P.seed, P.d, P.N, B.x + c, c, s0);
        int nv;
        const V3 f = path_forward<false, DELTA>(S, P.L, SoaU{B.x + c, P.N}, B.rec + c, P.N, stk, blockDim.x, ctr, &nv);
        B.p_tmp[c] = lum(f);
        B.f_tmp[c] = f.x;
        B.f_tmp[(size_t)P.N + c] = f.y;
        B.f_tmp[(size_t)2 * P.N + c] = f.z;
        B.pix_tmp[c] = pixel_of(S, B.x[c], B.x[(size_t)P.N + c]);
        B.key[c] = (uint32_t)nv;
        B.ids[c] = (uint32_t)c;
    }
    if (P.count) {
        wave_add(&B.ctr[C_RAYS], ctr.rays);
        wave_add(&B.ctr[C_NODES], ctr.nodes);
        wave_add(&B.ctr[C_TRIS], ctr.tris);
    }
}

// Sum of p over chains in FP64: per-block partials, then one block in order.
__global__ void k_reduce_p(KParams P, KBufs B) {
    __shared__ double sh[256];
    double acc = 0.0;
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < P.N; c += gridDim.x * blockDim.x) acc += (double)B.p_tmp[c];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) B.partial[blockIdx.x] = sh[0];
}
// p_lambda estimate and k0 = p_lambda/(m dt) (Eq. killing-rate-constant),
// unless k0_given > 0; p_lambda = 0 falls back to eps/(m dt).
__global__ void k_finish_k0(KParams P, KBufs B, int nparts, double k0_given, double m) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int i = 0; i < nparts; ++i) s += B.partial[i];
    const double pl = s / (double)P.N;
    *B.plam = pl;
    double k0 = k0_given;
    if (!(k0 > 0.0)) k0 = pl > 0.0 ? pl / (m * (double)P.dt) : (double)P.eps / (m * (double)P.dt);
    *B.k0d = k0;
    *B.k0 = (float)k0;
}

// ---- grouping chains before a fused launch: a counting sort over nbins keys,
// block-aggregated (one global atomic per block and key).  Keys: the last
// path length (DR_NBIN keys: 0..7 vertices, killed), or the screen tile of
// the chain's film coordinates (64 x 64 tiles in Morton order, then killed
// chains: DR_TILE_BINS keys).  bins[0..nbins) counts, bins[nbins..2 nbins)
// running offsets.
#define DR_TILE_BINS 4097
__device__ __forceinline__ uint32_t order_key(const KBufs& B, int N, int c, int by_tile, int nbins) {
    if (!by_tile) return min(B.key[c], (uint32_t)(nbins - 1));
    if (B.killed[c]) return DR_TILE_BINS - 1;
    const uint32_t tx = min((uint32_t)(B.x[c] * 64.0f), 63u), ty = min((uint32_t)(B.x[(size_t)N + c] * 64.0f), 63u);
    uint32_t m = 0;
#pragma unroll
    for (int b = 0; b < 6; ++b) m |= (((tx >> b) & 1u) << (2 * b)) | (((ty >> b) & 1u) << (2 * b + 1));
    return m;
}
__global__ void __launch_bounds__(256) k_sort_hist(KBufs B, int N, int by_tile, int nbins) {
    __shared__ uint32_t h[DR_TILE_BINS];
    for (int b = threadIdx.x; b < nbins; b += blockDim.x) h[b] = 0;
    __syncthreads();
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < N) atomicAdd(&h[order_key(B, N, c, by_tile, nbins)], 1u);
    __syncthreads();
    for (int b = threadIdx.x; b < nbins; b += blockDim.x)
        if (h[b]) atomicAdd(&B.bins[b], h[b]);
}
// Exclusive prefix of the counts (one block of 256 threads: a chunk of bins
// per thread, a sequential pass over the 256 chunk sums).
__global__ void __launch_bounds__(256) k_sort_prefix(uint32_t* bins, int nbins) {
    __shared__ uint32_t part[256];
    const int per = (nbins + 255) / 256;
    const int b0 = threadIdx.x * per, b1 = min(b0 + per, nbins);
    uint32_t sum = 0;
    for (int b = b0; b < b1; ++b) sum += bins[b];
    part[threadIdx.x] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int t = 0; t < 256; ++t) {
            const uint32_t v = part[t];
            part[t] = run;
            run += v;
        }
    }
    __syncthreads();
    uint32_t run = part[threadIdx.x];
    for (int b = b0; b < b1; ++b) {
        bins[nbins + b] = run;
        run += bins[b];
    }
}
__global__ void __launch_bounds__(256) k_sort_scatter(KBufs B, int N, int by_tile, int nbins) {
    __shared__ uint32_t h[DR_TILE_BINS], base[DR_TILE_BINS];
    for (int b = threadIdx.x; b < nbins; b += blockDim.x) h[b] = 0;
    __syncthreads();
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t k = 0, r = 0;
    if (c < N) {
        k = order_key(B, N, c, by_tile, nbins);
        r = atomicAdd(&h[k], 1u);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nbins; b += blockDim.x)
        if (h[b]) base[b] = atomicAdd(&B.bins[nbins + b], h[b]);
    __syncthreads();
    if (c < N) B.order[base[k] + r] = (uint32_t)c;
}
// alt[row][q] = state[row][order[q]]: chains move to the slots the sort gave them
__global__ void __launch_bounds__(256) k_slots_gather(const uint32_t* state, uint32_t* alt, const uint32_t* order,
                                                      int N) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    const size_t row = (size_t)blockIdx.y * N;
    if (q < N) alt[row + q] = state[row + order[q]];
}
// alt[row][ids[q]] = state[row][q]: every chain back to the slot of its id
__global__ void __launch_bounds__(256) k_slots_restore(const uint32_t* state, uint32_t* alt, const uint32_t* ids,
                                                       int N) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    const size_t row = (size_t)blockIdx.y * N;
    if (q < N) alt[row + ids[q]] = state[row + q];
}
__global__ void __launch_bounds__(256) k_copy_u32(const uint32_t* src, uint32_t* dst, size_t n) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

__global__ void __launch_bounds__(256) k_plain_move(KParams P, KBufs B) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= P.N) return;
    const uint64_t s = B.steps[1];
    if (B.killed[c]) regen(P.seed, P.d, P.N, B.x + c, c, s);
    else move(P.seed, P.d, P.N, P.stddev, P.gt, B.x + c, B.score + c, B.sigma ? B.sigma + c : nullptr, c, s);
}
__global__ void __launch_bounds__(256) k_plain_forward(KParams P, DevScene S, KBufs B) {
    extern __shared__ uint32_t s_stack[];
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    Counters ctr = {0, 0, 0};
    if (c < P.N) {
        const V3 f = path_forward<false>(S, P.L, SoaU{B.x + c, P.N}, B.rec + c, P.N, s_stack + threadIdx.x, blockDim.x,
                                         ctr);
        B.p_tmp[c] = lum(f);
        B.f_tmp[c] = f.x;
        B.f_tmp[(size_t)P.N + c] = f.y;
        B.f_tmp[(size_t)2 * P.N + c] = f.z;
        B.pix_tmp[c] = pixel_of(S, B.x[c], B.x[(size_t)P.N + c]);
    }
    if (P.count) {
        wave_add(&B.ctr[C_RAYS], ctr.rays);
        wave_add(&B.ctr[C_NODES], ctr.nodes);
        wave_add(&B.ctr[C_TRIS], ctr.tris);
    }
}
__global__ void __launch_bounds__(256) k_plain_accumulate(KParams P, DevScene S, KBufs B) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t s = B.steps[1];
    uint32_t kill = 0;
    if (c < P.N) {
        const float p = B.p_tmp[c];
        const V3 f = v3(B.f_tmp[c], B.f_tmp[(size_t)P.N + c], B.f_tmp[(size_t)2 * P.N + c]);
        const bool alive = hold_kill_splat(P, B, S, c, c, s, *B.k0, f, p, B.pix_tmp[c]);
        B.killed[c] = alive ? 0u : 1u;
        kill = alive ? 0u : 1u;
    }
    wave_add(&B.ctr[C_TOURS], kill);
    if (P.count) wave_add(&B.ctr[C_STEPS], c < P.N ? 1u : 0u);
}

// Resolve (Alg. 4.3): img = W H k0 accum / tourCount; accum is in units of dt.
__global__ void k_resolve(const float* accum, float* img, size_t npx, const double* k0d, const unsigned long long* ctr,
                          double dt) {
    const unsigned long long tours = ctr[C_TOURS];
    const float scale = tours ? (float)((double)npx * (*k0d) * dt / (double)tours) : 0.0f;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < 3 * npx; i += (size_t)gridDim.x * blockDim.x)
        img[i] = scale * accum[i];
}

// Independent path tracing, one thread per pixel.
struct PtU {  // generated coordinates: always finite
    static constexpr bool kChecked = false;
    uint64_t seed;
    uint32_t pix;
    uint64_t k;
    int W, H, px, py;
    __device__ __forceinline__ float operator()(int i) const {
        const uint4 r = rng_block(seed, pix, k, TAG_PT, (uint32_t)(i >> 2));
        const uint32_t w = (i & 3) == 0 ? r.x : ((i & 3) == 1 ? r.y : ((i & 3) == 2 ? r.z : r.w));
        const float v = u24(w);
        if (i == 0) return ((float)px + v) / (float)W;
        if (i == 1) return ((float)py + v) / (float)H;
        return v;
    }
};
template <bool DELTA>
__global__ void __launch_bounds__(256) k_pt(DevScene S, int L, uint64_t seed, uint32_t spp, float* img) {
    extern __shared__ uint32_t s_stack[];
    const int pix = blockIdx.x * blockDim.x + threadIdx.x;
    const int npx = S.W * S.H;
    if (pix >= npx) return;
    Counters ctr = {0, 0, 0};
    V3 acc = v3(0.f, 0.f, 0.f);
    for (uint32_t k = 0; k < spp; ++k) {
        const PtU u{seed, (uint32_t)pix, (uint64_t)k, S.W, S.H, pix % S.W, pix / S.W};
        acc = acc + path_forward<false, DELTA>(S, L, u, nullptr, 0, s_stack + threadIdx.x, blockDim.x, ctr);
    }
    const float inv = 1.0f / (float)spp;
    img[pix] = acc.x * inv;
    img[npx + pix] = acc.y * inv;
    img[2 * npx + pix] = acc.z * inv;
}

// ===========================================================================
// Host side
// ===========================================================================
namespace {
thread_local std::string g_err;

dr_status fail(dr_status s, const std::string& msg) {
    g_err = msg;
    return s;
}

#define HIP_TRY(expr)                                                                                  \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess) return fail(DR_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// Device memory: hipMalloc, or the caller's hooks installed by
// dr_set_allocator.  Every block remembers the hooks that made it.
struct AllocHooks {
    dr_alloc_fn alloc = nullptr;
    dr_free_fn free_ = nullptr;
    void* user = nullptr;
};
static AllocHooks g_hooks;

static hipError_t dev_alloc(void** p, size_t bytes, void* stream, const AllocHooks& h) {
    if (!h.alloc) return hipMalloc(p, bytes);
    *p = h.alloc(bytes, stream, h.user);
    if (!*p) return hipErrorOutOfMemory;
    if (reinterpret_cast<uintptr_t>(*p) % 256) {  // the kernels' vector loads need aligned buffers
        h.free_(*p, bytes, stream, h.user);
        *p = nullptr;
        return hipErrorInvalidValue;
    }
    return hipSuccess;
}
static void dev_free(void* p, size_t bytes, void* stream, const AllocHooks& h) {
    if (h.free_) h.free_(p, bytes, stream, h.user);
    else (void)hipFree(p);
}

struct DevAlloc {
    struct Block {
        void* p;
        size_t bytes;
        AllocHooks hooks;
        void* stream;
    };
    std::vector<Block> blocks;
    void* stream = nullptr;  // stream handed to the allocator hooks
    hipError_t get(void** p, size_t bytes) {
        bytes = bytes ? bytes : 4;
        const AllocHooks h = g_hooks;
        const hipError_t e = dev_alloc(p, bytes, stream, h);
        if (e == hipSuccess) blocks.push_back({*p, bytes, h, stream});
        return e;
    }
    void release() {
        for (const Block& b : blocks) dev_free(b.p, b.bytes, b.stream, b.hooks);
        blocks.clear();
    }
};

void camera_basis(const dr_camera& c, float4 out[4]) {
    double eye[3] = {c.eye[0], c.eye[1], c.eye[2]}, at[3] = {c.at[0], c.at[1], c.at[2]}, up[3] = {c.up[0], c.up[1], c.up[2]};
    double w[3] = {eye[0] - at[0], eye[1] - at[1], eye[2] - at[2]};
    double wl = std::sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    for (double& v : w) v /= wl;
    double u[3] = {up[1] * w[2] - up[2] * w[1], up[2] * w[0] - up[0] * w[2], up[0] * w[1] - up[1] * w[0]};
    double ul = std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    for (double& v : u) v /= ul;
    double v[3] = {w[1] * u[2] - w[2] * u[1], w[2] * u[0] - w[0] * u[2], w[0] * u[1] - w[1] * u[0]};
    const double th = std::tan(0.5 * (double)c.vfov_deg * M_PI / 180.0);
    const double aspect = (double)c.width / (double)c.height;
    out[0] = make_float4(c.eye[0], c.eye[1], c.eye[2], 0.f);
    out[1] = make_float4((float)(u[0] * th * aspect), (float)(u[1] * th * aspect), (float)(u[2] * th * aspect), 0.f);
    out[2] = make_float4((float)(v[0] * th), (float)(v[1] * th), (float)(v[2] * th), 0.f);
    out[3] = make_float4((float)-w[0], (float)-w[1], (float)-w[2], 0.f);
}

int g_num_cu(int dev) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) {
        (void)hipGetLastError();
        return 256;
    }
    return n;
}

}  // namespace

struct dr_scene {
    int device = 0;
    DevScene ds{};
    DevAlloc mem;
    std::vector<uint32_t> slot_to_prim;
    dr_camera cam{};
    uint32_t cam_version = 0;
    uint32_t n_tris = 0;
    uint32_t n_nodes = 0;
    bool has_delta = false;  // a triangle has a smooth conductor or dielectric
};

struct dr_chains {
    dr_scene* scene = nullptr;
    uint32_t cam_version = 0;
    dr_params P{};
    KParams kp{};
    KBufs kb{};
    DevAlloc mem;
    uint64_t seed = 0;
    int n_partials = 0;
    int record = 0, count = 0;
    dr_launch_cfg launch{256, 2, 1, 2, 0, 0, 50, 50, 0, 0, 0};
    int n_cu = 256;
    int rows_move = 0, rows_all = 0;  // state rows moved per sorted launch / restored before host access
    bool permuted = false;            // chains may sit outside the slot of their id
};

// ---------------------------------------------------------------------------

// the L-templated launchers are instantiated in the dr_inst_*.hip units
#define DR_EXTERN_L(L) DR_LAUNCHERS(extern, L)
DR_EXTERN_L(2) DR_EXTERN_L(3) DR_EXTERN_L(4) DR_EXTERN_L(5) DR_EXTERN_L(6) DR_EXTERN_L(7) DR_EXTERN_L(8)
DR_EXTERN_L(9) DR_EXTERN_L(10) DR_EXTERN_L(11) DR_EXTERN_L(12) DR_EXTERN_L(13) DR_EXTERN_L(14) DR_EXTERN_L(15)
DR_EXTERN_L(16)
#undef DR_EXTERN_L

#define DR_DISPATCH_L(L, FN, ...)          \
    switch (L) {                           \
        case 2: FN<2>(__VA_ARGS__); break;   \
        case 3: FN<3>(__VA_ARGS__); break;   \
        case 4: FN<4>(__VA_ARGS__); break;   \
        case 5: FN<5>(__VA_ARGS__); break;   \
        case 6: FN<6>(__VA_ARGS__); break;   \
        case 7: FN<7>(__VA_ARGS__); break;   \
        case 8: FN<8>(__VA_ARGS__); break;   \
        case 9: FN<9>(__VA_ARGS__); break;   \
        case 10: FN<10>(__VA_ARGS__); break; \
        case 11: FN<11>(__VA_ARGS__); break; \
        case 12: FN<12>(__VA_ARGS__); break; \
        case 13: FN<13>(__VA_ARGS__); break; \
        case 14: FN<14>(__VA_ARGS__); break; \
        case 15: FN<15>(__VA_ARGS__); break; \
        case 16: FN<16>(__VA_ARGS__); break; \
        default: break;                      \
    }

// Event threshold of the ray-refill initialise kernel (percent of the busy
// lanes waiting for an event): the best of 30, 50, 75 and 90 on the 53k- and
// 2M-triangle scenes.
#define DR_INIT_EVENT_PCT 75

// Buffers of the ray-wave initialise form (path states, pending rays, their
// answers, two slot queues): allocated the first time the form is selected.
static hipError_t ensure_wf_buffers(dr_chains* c) {
    if (c->kb.wf) return hipSuccess;
    const size_t N = (size_t)c->kp.N;
    void *a = nullptr, *r = nullptr, *h = nullptr, *t = nullptr, *q = nullptr, *n = nullptr;
    hipError_t e = c->mem.get(&a, sizeof(uint32_t) * DR_WF_ROWS * N);
    if (e == hipSuccess) e = c->mem.get(&r, sizeof(float4) * 2 * N);
    if (e == hipSuccess) e = c->mem.get(&h, sizeof(int) * N);
    if (e == hipSuccess) e = c->mem.get(&t, sizeof(float) * N);
    if (e == hipSuccess) e = c->mem.get(&q, sizeof(uint32_t) * 2 * N);
    if (e == hipSuccess) e = c->mem.get(&n, 64);
    if (e != hipSuccess) return e;
    KBufs& B = c->kb;
    B.wf_ray = (float4*)r;
    B.wf_hit = (int*)h;
    B.wf_t = (float*)t;
    B.wf_q = (uint32_t*)q;
    B.wf_cnt = (uint32_t*)n;
    B.wf = (uint32_t*)a;  // last: marks the set complete
    return hipSuccess;
}

// Enqueue the initialise pass (Alg. 4.1).  from_device: take the frame index
// from the device frame counter plus one (used inside captured frames).
static void enqueue_init(dr_chains* c, uint32_t frame, int from_device, hipStream_t st) {
    (void)hipGetLastError();  // drop a stale error left by an earlier, unrelated call
    const int N = c->kp.N;
    const int blk = 256;
    const dim3 g((N + blk - 1) / blk), b(blk);
    const size_t npx = (size_t)c->scene->ds.W * c->scene->ds.H;
    KParams P = c->kp;
    P.record = c->record;
    P.count = c->count;
    hipLaunchKernelGGL(k_begin_init, dim3(1), dim3(64), 0, st, c->kb, frame, from_device);
    hipLaunchKernelGGL(k_fill_f32, dim3(1024), dim3(256), 0, st, c->kb.accum, 3 * npx);
    hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, st, c->kb.ctr, (int)C_N);
    const DevScene& S = c->scene->ds;
    if (c->launch.init_refill) {
        // ray-refill form: persistent blocks (more than fit at once; the
        // extra ones find the queue drained)
        const dim3 gp((unsigned)std::max(1L, std::min((long)g.x, (long)c->n_cu * 4)));
        DR_DISPATCH_L(c->kp.L, launch_init_sm, gp, b, st, P, S, c->kb, DR_INIT_EVENT_PCT, c->scene->has_delta);
    } else if (c->launch.wavefront && c->kb.wf) {
        // ray waves: persistent traversal blocks (more than fit at once; the
        // extra ones find the queue drained)
        DR_DISPATCH_L(c->kp.L, launch_wf_init, g, b, c->n_cu * 4, st, P, S, c->kb, c->scene->has_delta);
    } else {
        const size_t lds = stack_bytes(S, blk);
        // persistent grid: as many blocks as can be resident at once
        int per_cu = 0;
        if (c->scene->has_delta)
            (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_init_eval<true>, blk, lds);
        else
            (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_init_eval<false>, blk, lds);
        const dim3 gp((unsigned)std::max(1L, std::min((long)g.x, (long)c->n_cu * std::max(per_cu, 1))));
        if (c->scene->has_delta) hipLaunchKernelGGL(k_init_eval<true>, gp, b, lds, st, P, S, c->kb);
        else hipLaunchKernelGGL(k_init_eval<false>, gp, b, lds, st, P, S, c->kb);
    }
    hipLaunchKernelGGL(k_reduce_p, dim3(c->n_partials), dim3(256), 0, st, P, c->kb);
    hipLaunchKernelGGL(k_finish_k0, dim3(1), dim3(64), 0, st, P, c->kb, c->n_partials, (double)c->P.k0, (double)c->P.m);
    const int with_score = c->P.mode == DR_MODE_FUSED ? 1 : 0;
    DR_DISPATCH_L(c->kp.L, launch_init_acc, g, b, st, P, c->scene->ds, c->kb, with_score);
}

// Enqueue n_steps evolve steps (Alg. 4.2) in the chain set's form.  Returns
// true when the enqueued work moves chains between slots (an ordered fused
// launch); the caller records that in c->permuted once the work is sure to
// run (at once for dr_step, at each launch for a captured frame).
static bool enqueue_steps(dr_chains* c, uint32_t n_steps, hipStream_t st) {
    (void)hipGetLastError();  // drop a stale error left by an earlier, unrelated call
    KParams P = c->kp;
    P.record = c->record;
    P.count = c->count;
    const int N = P.N;
    bool permutes = false;
    if (c->P.mode == DR_MODE_FUSED) {
        const int by_tile = c->launch.sort_by_tile ? 1 : 0;
        const int sorted = c->launch.sort_by_length && !by_tile ? 1 : 0;  // the kernels record length keys
        if (by_tile || sorted) {
            const int nb = by_tile ? DR_TILE_BINS : DR_NBIN;
            const dim3 gs((N + 255) / 256), bs(256);
            hipLaunchKernelGGL(k_fill_u32, dim3(16), dim3(256), 0, st, c->kb.bins, (size_t)(2 * nb), 0u);
            hipLaunchKernelGGL(k_sort_hist, gs, bs, 0, st, c->kb, N, by_tile, nb);
            hipLaunchKernelGGL(k_sort_prefix, dim3(1), bs, 0, st, c->kb.bins, nb);
            hipLaunchKernelGGL(k_sort_scatter, gs, bs, 0, st, c->kb, N, by_tile, nb);
            hipLaunchKernelGGL(k_slots_gather, dim3(gs.x, c->rows_move), bs, 0, st, c->kb.state, c->kb.alt,
                               c->kb.order, N);
            hipLaunchKernelGGL(k_copy_u32, dim3(2048), bs, 0, st, c->kb.alt, c->kb.state,
                               (size_t)c->rows_move * N);
            permutes = true;
        }
        hipLaunchKernelGGL(k_begin_launch, dim3(1), dim3(64), 0, st, c->kb, n_steps);
        const int blk = (int)c->launch.block;
        if (c->launch.refill) {
            int blocks = (int)(c->n_cu * c->launch.blocks_per_cu);
            blocks = (int)std::max(1L, std::min((long)blocks, ((long)N + blk - 1) / blk));
            DR_DISPATCH_L(P.L, launch_sm, dim3(blocks), dim3(blk), st, P, c->scene->ds, c->kb, n_steps, sorted,
                          (int)c->launch.refill_event_pct, (int)c->launch.refill_advance_pct, c->scene->has_delta);
            return permutes;
        }
        const bool pair = c->launch.lanes_per_chain == 2;
        const long lanes = (long)N * (pair ? 2 : 1);
        int blocks = (int)(c->n_cu * c->launch.blocks_per_cu);
        blocks = (int)std::max(1L, std::min((long)blocks, (lanes + blk - 1) / blk));
        const DevScene& S = c->scene->ds;
        DR_DISPATCH_L(P.L, launch_fused, dim3(blocks), dim3(blk), st, P, S, c->kb, n_steps, c->launch.grab, pair,
                      sorted, c->scene->has_delta);
    } else {
        const int blk = 256;
        const dim3 g((N + blk - 1) / blk), b(blk);
        for (uint32_t k = 0; k < n_steps; ++k) {
            hipLaunchKernelGGL(k_begin_launch, dim3(1), dim3(64), 0, st, c->kb, 1u);
            DR_DISPATCH_L(P.L, launch_plain_score, g, b, st, P, c->scene->ds, c->kb);
            hipLaunchKernelGGL(k_plain_move, g, b, 0, st, P, c->kb);
            hipLaunchKernelGGL(k_plain_forward, g, b, stack_bytes(c->scene->ds, blk), st, P, c->scene->ds, c->kb);
            hipLaunchKernelGGL(k_plain_accumulate, g, b, 0, st, P, c->scene->ds, c->kb);
        }
    }
    return permutes;
}

static void enqueue_resolve(dr_chains* c, float* image_dev, hipStream_t st) {
    (void)hipGetLastError();  // drop a stale error left by an earlier, unrelated call
    const size_t npx = (size_t)c->scene->ds.W * c->scene->ds.H;
    hipLaunchKernelGGL(k_resolve, dim3(std::min<size_t>(4096, (3 * npx + 255) / 256)), dim3(256), 0, st, c->kb.accum,
                       image_dev, npx, c->kb.k0d, c->kb.ctr, (double)c->P.dt);
}

// Put every chain back into the slot of its id (before the host reads or
// writes per-chain state).
static dr_status restore_slots(dr_chains* c, hipStream_t st) {
    if (!c->permuted) return DR_OK;
    (void)hipGetLastError();
    const int N = c->kp.N;
    hipLaunchKernelGGL(k_slots_restore, dim3((N + 255) / 256, c->rows_all), dim3(256), 0, st, c->kb.state, c->kb.alt,
                       c->kb.ids, N);
    hipLaunchKernelGGL(k_copy_u32, dim3(2048), dim3(256), 0, st, c->kb.alt, c->kb.state, (size_t)c->rows_all * N);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(DR_ERR_DEVICE, std::string("slot restore launch: ") + hipGetErrorString(e));
    c->permuted = false;
    return DR_OK;
}

static dr_status run_init(dr_chains* c, uint32_t frame, hipStream_t st) {
    c->permuted = false;  // the initialise pass puts chain c in slot c
    enqueue_init(c, frame, 0, st);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(DR_ERR_DEVICE, std::string("initialise pass launch: ") + hipGetErrorString(e));
    c->cam_version = c->scene->cam_version;
    return DR_OK;
}

struct dr_frame {
    dr_chains* c = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int reinit = 0;
    bool permutes = false;  // the frame's steps move chains between slots
};

// For the other translation units of the library (declared where used).
void dr_set_last_error(const char* msg) { g_err = msg; }

extern "C" {

const char* dr_last_error(void) { return g_err.c_str(); }
const char* dr_version(void) { return "drestore-gfx950 0.1"; }

dr_status dr_bvh_build(const float* vertices, uint32_t n_vertices, const uint32_t* indices, uint32_t n_triangles,
                       uint32_t max_leaf, dr_bvh_node* nodes_out, uint32_t* n_nodes_out, uint32_t* prim_order_out) {
    const char* err = "";
    dr_status s = dr_bvh_build_impl(vertices, n_vertices, indices, n_triangles, max_leaf, nodes_out, n_nodes_out,
                                    prim_order_out, &err);
    if (s != DR_OK) return fail(s, err);
    g_err.clear();
    return DR_OK;
}

dr_status dr_scene_create(const dr_scene_desc* desc, int device, dr_scene** out) {
    if (!desc || !out) return fail(DR_ERR_INVALID_ARG, "dr_scene_create: null argument");
    const uint32_t T = desc->n_triangles;
    if (T == 0 || !desc->vertices || !desc->indices || !desc->tri_material || !desc->materials)
        return fail(DR_ERR_INVALID_ARG, "dr_scene_create: empty mesh or null array");
    if (T >= (1u << 24)) return fail(DR_ERR_INVALID_ARG, "dr_scene_create: at most 2^24-1 triangles");
    if (desc->n_lights == 0 || desc->n_lights > 127 || !desc->lights)
        return fail(DR_ERR_INVALID_ARG, "dr_scene_create: need 1..127 lights");
    if (desc->camera.width == 0 || desc->camera.height == 0)
        return fail(DR_ERR_INVALID_ARG, "dr_scene_create: empty image");
    for (uint64_t i = 0; i < 3ull * T; ++i)
        if (desc->indices[i] >= desc->n_vertices) return fail(DR_ERR_INVALID_ARG, "dr_scene_create: vertex index out of range");
    for (uint32_t t = 0; t < T; ++t)
        if (desc->tri_material[t] >= desc->n_materials)
            return fail(DR_ERR_INVALID_ARG, "dr_scene_create: material index out of range");
    for (uint32_t m = 0; m < desc->n_materials; ++m) {
        const dr_material& q = desc->materials[m];
        if (q.kind > DR_MAT_SMOOTH_DIELECTRIC) return fail(DR_ERR_INVALID_ARG, "dr_scene_create: unknown material kind");
        if (q.kind == DR_MAT_SMOOTH_DIELECTRIC && !(q.eta > 0.0f && std::isfinite(q.eta)))
            return fail(DR_ERR_INVALID_ARG, "dr_scene_create: dielectric eta must be finite and > 0");
    }

    // BVH: given or built here
    std::vector<dr_bvh_node> nodes;
    std::vector<uint32_t> order;
    if (desc->bvh) {
        if (!desc->bvh_prim_order || desc->n_nodes == 0)
            return fail(DR_ERR_INVALID_ARG, "dr_scene_create: bvh without prim order");
        nodes.assign(desc->bvh, desc->bvh + desc->n_nodes);
        order.assign(desc->bvh_prim_order, desc->bvh_prim_order + T);
        std::vector<uint8_t> seen(T, 0);
        for (uint32_t p : order) {
            if (p >= T || seen[p]) return fail(DR_ERR_INVALID_ARG, "dr_scene_create: prim order is not a permutation");
            seen[p] = 1;
        }
    } else {
        nodes.resize(2 * (size_t)T);
        order.resize(T);
        uint32_t nn = 0;
        dr_status s = dr_bvh_build(desc->vertices, desc->n_vertices, desc->indices, T, 4, nodes.data(), &nn, order.data());
        if (s != DR_OK) return s;
        nodes.resize(nn);
    }
    // Validate the tree and recompute exact f32 bounds bottom-up.
    const size_t NN = nodes.size();
    std::vector<int> depth(NN, -1), parent(NN, -1);
    std::vector<int> stack = {0};
    depth[0] = 0;
    std::vector<int> topo;
    uint64_t covered = 0;
    while (!stack.empty()) {
        const int i = stack.back();
        stack.pop_back();
        topo.push_back(i);
        const dr_bvh_node& n = nodes[i];
        if (n.a < 0) {
            const int64_t first = ~(int64_t)n.a, cnt = n.b;
            if (cnt < 1 || cnt > 16 || first + cnt > (int64_t)T)
                return fail(DR_ERR_INVALID_ARG, "dr_scene_create: bad BVH leaf");
            covered += (uint64_t)cnt;
        } else {
            for (int ch : {n.a, n.b}) {
                if (ch <= 0 || (size_t)ch >= NN || depth[ch] != -1)
                    return fail(DR_ERR_INVALID_ARG, "dr_scene_create: bad BVH child index");
                depth[ch] = depth[i] + 1;
                if (depth[ch] > 64) return fail(DR_ERR_INVALID_ARG, "dr_scene_create: BVH deeper than 64");
                parent[ch] = i;
                stack.push_back(ch);
            }
        }
    }
    if (covered != T) return fail(DR_ERR_INVALID_ARG, "dr_scene_create: BVH leaves do not cover every triangle once");
    std::vector<float> blo(3 * NN, INFINITY), bhi(3 * NN, -INFINITY);
    for (auto it = topo.rbegin(); it != topo.rend(); ++it) {
        const int i = *it;
        const dr_bvh_node& n = nodes[i];
        if (n.a < 0) {
            for (int64_t k = ~(int64_t)n.a; k < ~(int64_t)n.a + n.b; ++k) {
                const uint32_t t = order[k];
                for (int v = 0; v < 3; ++v) {
                    const float* p = desc->vertices + 3 * (size_t)desc->indices[3 * (size_t)t + v];
                    for (int a = 0; a < 3; ++a) {
                        blo[3 * i + a] = std::min(blo[3 * i + a], p[a]);
                        bhi[3 * i + a] = std::max(bhi[3 * i + a], p[a]);
                    }
                }
            }
        } else {
            for (int a = 0; a < 3; ++a) {
                blo[3 * i + a] = std::min(blo[3 * n.a + a], blo[3 * n.b + a]);
                bhi[3 * i + a] = std::max(bhi[3 * n.a + a], bhi[3 * n.b + a]);
            }
        }
    }
    // Collapse the binary tree into 4-wide nodes with the fewest expected node
    // visits.  Under the surface-area model a ray visits a node with
    // probability proportional to the area of its box, so the collapse
    // minimises the summed area of the 4-wide nodes (the leaves, and so the
    // triangle tests, are the binary tree's whatever the collapse).  Dynamic
    // programming over the binary tree, children before parents (after the
    // optimal wide-BVH collapse of Ylitie, Karras and Laine, HPG 2017):
    // cost[4 n + i - 1] is the least summed area of the 4-wide nodes within
    // binary subtree n when n may take at most i slots of its parent's node:
    // one slot (a leaf, or a 4-wide node whose four slots its two subtrees
    // share), or, for i >= 2, n dissolved into its subtrees' slots.  pick
    // records the choice: for i = 1 the slots of n's own node given to its
    // first child, for i >= 2 0 (keep n as one slot) or the slots given to
    // its first child.  Device nodes are created in depth-first order; leaves
    // stay embedded in their parent.
    auto area = [&](int i) {
        const double dx = (double)bhi[3 * i] - blo[3 * i], dy = (double)bhi[3 * i + 1] - blo[3 * i + 1],
                     dz = (double)bhi[3 * i + 2] - blo[3 * i + 2];
        return dx * dy + dy * dz + dz * dx;
    };
    std::vector<double> cost(4 * NN, 0.0);
    std::vector<uint8_t> pick(4 * NN, 0);
    for (auto it = topo.rbegin(); it != topo.rend(); ++it) {
        const int n = *it;
        if (nodes[n].a < 0) continue;  // a leaf takes one slot and adds no node
        const size_t ca = 4 * (size_t)nodes[n].a, cb = 4 * (size_t)nodes[n].b, cn = 4 * (size_t)n;
        double best = INFINITY;
        for (int j = 1; j <= 3; ++j) {
            const double c = cost[ca + j - 1] + cost[cb + 3 - j];
            if (c < best) { best = c; pick[cn] = (uint8_t)j; }
        }
        const double as_node = area(n) + best;
        cost[cn] = as_node;
        for (int i = 2; i <= 4; ++i) {
            cost[cn + i - 1] = as_node;
            pick[cn + i - 1] = 0;
            for (int j = 1; j < i; ++j) {
                const double c = cost[ca + j - 1] + cost[cb + i - j - 1];
                if (c < cost[cn + i - 1]) { cost[cn + i - 1] = c; pick[cn + i - 1] = (uint8_t)j; }
            }
        }
    }
    // the slots of binary subtree x given at most i of them
    struct Expand {
        const std::vector<dr_bvh_node>& nodes;
        const std::vector<uint8_t>& pick;
        void operator()(int x, int i, int out[4], int& k) const {
            const int j = i > 1 && nodes[x].a >= 0 ? pick[4 * (size_t)x + i - 1] : 0;
            if (j == 0) {
                out[k++] = x;
                return;
            }
            (*this)(nodes[x].a, j, out, k);
            (*this)(nodes[x].b, i - j, out, k);
        }
    };
    const Expand expand{nodes, pick};
    // the children of the 4-wide node made from inner binary node n
    auto gather = [&](int n, int out[4]) {
        int k = 0;
        const int j = pick[4 * (size_t)n];
        expand(nodes[n].a, j, out, k);
        expand(nodes[n].b, 4 - j, out, k);
        return k;
    };
    // the first 512 nodes laid out breadth-first, the rest depth-first
    constexpr int DR_BFS_TOP = 512;
    std::vector<DevNode> dn;
    std::vector<int> need;  // worst-case traversal stack entries below each device node
    {
        struct Item { int bin; int dev; };
        std::vector<Item> work;
        std::vector<std::vector<int>> kids;  // device children (inner) per device node
        auto fill_leafroot = [&]() {
            DevNode r{};
            const float nan = std::numeric_limits<float>::quiet_NaN();
            r.lox = make_float4(blo[0], nan, nan, nan); r.loy = make_float4(blo[1], nan, nan, nan);
            r.loz = make_float4(blo[2], nan, nan, nan); r.hix = make_float4(bhi[0], nan, nan, nan);
            r.hiy = make_float4(bhi[1], nan, nan, nan); r.hiz = make_float4(bhi[2], nan, nan, nan);
            r.child = make_int4(leaf_code(~nodes[0].a, nodes[0].b), 0, 0, 0);
            r.count = make_int4(nodes[0].b, -1, -1, -1);
            dn.push_back(r);
            kids.emplace_back();
        };
        if (nodes[0].a < 0) {
            fill_leafroot();
        } else {
            dn.emplace_back();
            kids.emplace_back();
            // breadth-first for the first nodes (indices grow level by level,
            // so the top levels, which every ray visits, share a few cache
            // lines), depth-first below them, so that each deeper subtree's
            // nodes lie together in memory and a ray descending it stays on
            // nearby lines
            std::vector<Item> deep;  // depth-first stack
            work.push_back({0, 0});
            size_t w = 0;
            while (w < work.size() || !deep.empty()) {
                Item it;
                if (w < work.size()) {
                    it = work[w++];
                } else {
                    it = deep.back();
                    deep.pop_back();
                }
                int ch[4];
                const int k = gather(it.bin, ch);
                float lo[3][4], hi[3][4];
                int cidx[4], ccnt[4];
                for (int q = 0; q < 4; ++q) {
                    if (q >= k) {  // empty slot: a NaN box, which no ray hits
                        for (int a2 = 0; a2 < 3; ++a2) lo[a2][q] = hi[a2][q] = std::numeric_limits<float>::quiet_NaN();
                        cidx[q] = 0;
                        ccnt[q] = -1;
                        continue;
                    }
                    const int c = ch[q];
                    for (int a2 = 0; a2 < 3; ++a2) { lo[a2][q] = blo[3 * c + a2]; hi[a2][q] = bhi[3 * c + a2]; }
                    if (nodes[c].a < 0) {
                        cidx[q] = leaf_code(~nodes[c].a, nodes[c].b);
                        ccnt[q] = nodes[c].b;
                    } else {
                        cidx[q] = (int)dn.size();
                        ccnt[q] = 0;
                        dn.emplace_back();
                        kids.emplace_back();
                        kids[it.dev].push_back(cidx[q]);
                        if (cidx[q] < DR_BFS_TOP) work.push_back({c, cidx[q]});
                    }
                }
                // deeper children go on the depth-first stack, first child on top
                for (int q = k - 1; q >= 0; --q)
                    if (nodes[ch[q]].a >= 0 && cidx[q] >= DR_BFS_TOP) deep.push_back({ch[q], cidx[q]});
                DevNode& r = dn[it.dev];
                r.lox = make_float4(lo[0][0], lo[0][1], lo[0][2], lo[0][3]);
                r.loy = make_float4(lo[1][0], lo[1][1], lo[1][2], lo[1][3]);
                r.loz = make_float4(lo[2][0], lo[2][1], lo[2][2], lo[2][3]);
                r.hix = make_float4(hi[0][0], hi[0][1], hi[0][2], hi[0][3]);
                r.hiy = make_float4(hi[1][0], hi[1][1], hi[1][2], hi[1][3]);
                r.hiz = make_float4(hi[2][0], hi[2][1], hi[2][2], hi[2][3]);
                r.child = make_int4(cidx[0], cidx[1], cidx[2], cidx[3]);
                r.count = make_int4(ccnt[0], ccnt[1], ccnt[2], ccnt[3]);
            }
        }
        // Stack bound.  Inner children and postponed leaves share the stack:
        // a visit that descends pushes at most (children - 1) entries (the
        // one descended into is not pushed), and a visit that does not
        // descend pushes at most all its leaves and is followed by a pop.  So
        // the height never exceeds, over root-to-node paths, the sum of
        // (children - 1) along the path plus the children of its last node.
        need.assign(dn.size(), 0);
        for (int i = (int)dn.size() - 1; i >= 0; --i) {  // children have larger indices
            const int4 cc = dn[i].count;
            const int c = (cc.x >= 0) + (cc.y >= 0) + (cc.z >= 0) + (cc.w >= 0);
            int m = 0;
            for (int k : kids[i]) m = std::max(m, need[k]);
            need[i] = kids[i].empty() ? c : std::max(c, c - 1 + m);
        }
        if (need[0] > DR_STACK) return fail(DR_ERR_UNSUPPORTED, "dr_scene_create: BVH needs a deeper traversal stack than 64");
    }
    // triangles in leaf order
    std::vector<DevTri> tris(T);
    std::vector<uint32_t> slot_to_prim(T);
    for (uint32_t k = 0; k < T; ++k) {
        const uint32_t t = order[k];
        const float* v0 = desc->vertices + 3 * (size_t)desc->indices[3 * (size_t)t];
        const float* v1 = desc->vertices + 3 * (size_t)desc->indices[3 * (size_t)t + 1];
        const float* v2 = desc->vertices + 3 * (size_t)desc->indices[3 * (size_t)t + 2];
        uint32_t mb = desc->tri_material[t], pb = t;
        float mf, pf;
        std::memcpy(&mf, &mb, 4);
        std::memcpy(&pf, &pb, 4);
        tris[k].v0 = make_float4(v0[0], v0[1], v0[2], pf);
        tris[k].e1 = make_float4((float)((double)v1[0] - v0[0]), (float)((double)v1[1] - v0[1]), (float)((double)v1[2] - v0[2]), mf);
        tris[k].e2 = make_float4((float)((double)v2[0] - v0[0]), (float)((double)v2[1] - v0[1]), (float)((double)v2[2] - v0[2]), 0.f);
        slot_to_prim[k] = t;
    }
    std::vector<float4> mats(3 * desc->n_materials);
    for (uint32_t m = 0; m < desc->n_materials; ++m) {
        const dr_material& q = desc->materials[m];
        mats[3 * m] = make_float4((float)q.kind, q.albedo[0], q.albedo[1], q.albedo[2]);
        mats[3 * m + 1] = make_float4(q.roughness, q.f0[0], q.f0[1], q.f0[2]);
        mats[3 * m + 2] = make_float4(q.Le[0], q.Le[1], q.Le[2], q.kind == DR_MAT_SMOOTH_DIELECTRIC ? q.eta : 0.f);
    }
    std::vector<float4> lights(5 * desc->n_lights);
    for (uint32_t l = 0; l < desc->n_lights; ++l) {
        const dr_quad_light& q = desc->lights[l];
        const double e1[3] = {q.e1[0], q.e1[1], q.e1[2]}, e2[3] = {q.e2[0], q.e2[1], q.e2[2]};
        const double nn[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
        const double area = std::sqrt(nn[0] * nn[0] + nn[1] * nn[1] + nn[2] * nn[2]);
        if (!(area > 0)) return fail(DR_ERR_INVALID_ARG, "dr_scene_create: degenerate light");
        lights[5 * l] = make_float4(q.p0[0], q.p0[1], q.p0[2], 0.f);
        lights[5 * l + 1] = make_float4(q.e1[0], q.e1[1], q.e1[2], 0.f);
        lights[5 * l + 2] = make_float4(q.e2[0], q.e2[1], q.e2[2], 0.f);
        lights[5 * l + 3] = make_float4((float)(nn[0] / area), (float)(nn[1] / area), (float)(nn[2] / area), (float)area);
        lights[5 * l + 4] = make_float4(q.Le[0], q.Le[1], q.Le[2], 0.f);
    }
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (uint32_t v = 0; v < desc->n_vertices; ++v)
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::min(lo[a], (double)desc->vertices[3 * (size_t)v + a]);
            hi[a] = std::max(hi[a], (double)desc->vertices[3 * (size_t)v + a]);
        }
    const double diag = std::sqrt((hi[0] - lo[0]) * (hi[0] - lo[0]) + (hi[1] - lo[1]) * (hi[1] - lo[1]) +
                                  (hi[2] - lo[2]) * (hi[2] - lo[2]));

    HIP_TRY(hipSetDevice(device));
    auto* S = new dr_scene();
    S->device = device;
    void *dnodes, *dtris, *dmats, *dlights, *dcam;
    float4 cam4[4];
    camera_basis(desc->camera, cam4);
    if (S->mem.get(&dcam, sizeof(cam4)) != hipSuccess ||
        S->mem.get(&dnodes, dn.size() * sizeof(DevNode)) != hipSuccess ||
        S->mem.get(&dtris, tris.size() * sizeof(DevTri)) != hipSuccess ||
        S->mem.get(&dmats, mats.size() * sizeof(float4)) != hipSuccess ||
        S->mem.get(&dlights, lights.size() * sizeof(float4)) != hipSuccess) {
        S->mem.release();
        delete S;
        return fail(DR_ERR_OUT_OF_MEMORY, "dr_scene_create: device allocation failed");
    }
    if (hipMemcpy(dcam, cam4, sizeof(cam4), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(dnodes, dn.data(), dn.size() * sizeof(DevNode), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(dtris, tris.data(), tris.size() * sizeof(DevTri), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(dmats, mats.data(), mats.size() * sizeof(float4), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(dlights, lights.data(), lights.size() * sizeof(float4), hipMemcpyHostToDevice) != hipSuccess) {
        S->mem.release();
        delete S;
        return fail(DR_ERR_DEVICE, "dr_scene_create: upload failed");
    }
    S->ds.nodes = (const DevNode*)dnodes;
    S->ds.tris = (const DevTri*)dtris;
    S->ds.mats = (const float4*)dmats;
    S->ds.lights = (const float4*)dlights;
    S->ds.n_lights = (int)desc->n_lights;
    S->ds.n_tris = (int)T;
    S->ds.n_nodes = (int)dn.size();
    {
        int max_count = 0;
        for (const DevNode& nd : dn)
            max_count = std::max({max_count, nd.count.x, nd.count.y, nd.count.z, nd.count.w});
        S->ds.leaf_batch = max_count <= 2 ? 2 : 4;
    }
    S->ds.tmin = (float)(1e-4 * diag);
    S->ds.cam = (const float4*)dcam;
    S->ds.W = (int)desc->camera.width;
    S->ds.H = (int)desc->camera.height;
    S->ds.stack_cap = std::max(1, need.empty() ? 1 : need[0]);
    S->n_nodes = (uint32_t)dn.size();
    S->cam = desc->camera;
    S->slot_to_prim = std::move(slot_to_prim);
    S->n_tris = T;
    for (uint32_t t = 0; t < T && !S->has_delta; ++t)
        S->has_delta = desc->materials[desc->tri_material[t]].kind >= DR_MAT_SMOOTH_CONDUCTOR;
    *out = S;
    g_err.clear();
    return DR_OK;
}

dr_status dr_scene_set_camera(dr_scene* s, const dr_camera* cam) {
    if (!s || !cam) return fail(DR_ERR_INVALID_ARG, "dr_scene_set_camera: null argument");
    if (cam->width != s->cam.width || cam->height != s->cam.height)
        return fail(DR_ERR_INVALID_ARG, "dr_scene_set_camera: image size cannot change");
    float4 cam4[4];
    camera_basis(*cam, cam4);
    HIP_TRY(hipSetDevice(s->device));
    // work in flight may still read the camera: wait for it, then update
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy((void*)s->ds.cam, cam4, sizeof(cam4), hipMemcpyHostToDevice));
    s->cam = *cam;
    s->cam_version++;
    g_err.clear();
    return DR_OK;
}

dr_status dr_set_allocator(dr_alloc_fn alloc, dr_free_fn free_, void* user) {
    if ((alloc == nullptr) != (free_ == nullptr))
        return fail(DR_ERR_INVALID_ARG, "dr_set_allocator: give both hooks or neither");
    g_hooks.alloc = alloc;
    g_hooks.free_ = free_;
    g_hooks.user = alloc ? user : nullptr;
    g_err.clear();
    return DR_OK;
}

dr_status dr_scene_get_stats(const dr_scene* s, dr_scene_stats* out) {
    if (!s || !out) return fail(DR_ERR_INVALID_ARG, "dr_scene_get_stats: null argument");
    out->n_triangles = s->n_tris;
    out->n_nodes = s->n_nodes;
    out->stack_entries = (uint32_t)s->ds.stack_cap;
    out->stack_bytes_per_lane = (uint32_t)(s->ds.stack_cap * sizeof(uint32_t));
    g_err.clear();
    return DR_OK;
}

void dr_scene_destroy(dr_scene* s) {
    if (!s) return;
    (void)hipSetDevice(s->device);
    (void)hipDeviceSynchronize();  // allocator hooks may hand the memory out again at once
    s->mem.release();
    delete s;
}

dr_status dr_chains_init(dr_scene* s, const dr_params* p, uint64_t seed, uint32_t frame, void* hip_stream,
                         dr_chains** out) {
    if (!s || !p || !out) return fail(DR_ERR_INVALID_ARG, "dr_chains_init: null argument");
    if (p->n_chains == 0) return fail(DR_ERR_INVALID_ARG, "dr_chains_init: n_chains must be >= 1");
    if (p->n_chains > (1u << 30)) return fail(DR_ERR_INVALID_ARG, "dr_chains_init: n_chains too large");
    if (p->max_path_len < 2 || p->max_path_len > 16) return fail(DR_ERR_INVALID_ARG, "dr_chains_init: max_path_len must be 2..16");
    if (!(p->stddev > 0) || !(p->dt > 0) || !(p->m > 0) || !(p->eps > 0) || !(p->gamma >= 0))
        return fail(DR_ERR_INVALID_ARG, "dr_chains_init: stddev, dt, m, eps must be > 0 and gamma >= 0");
    if (p->mode > 1) return fail(DR_ERR_INVALID_ARG, "dr_chains_init: unknown mode");
    HIP_TRY(hipSetDevice(s->device));
    auto* c = new dr_chains();
    c->mem.stream = hip_stream;
    c->scene = s;
    c->P = *p;
    c->seed = seed;
    c->n_cu = g_num_cu(s->device);
    // two lanes per chain while chains alone cannot fill two wavefronts per
    // SIMD (4 SIMDs per compute unit, 64 lanes per wavefront); one otherwise
    c->launch.lanes_per_chain = (uint64_t)p->n_chains < (uint64_t)c->n_cu * 4 * 64 * 2 ? 2u : 1u;
    c->launch.blocks_per_cu = 4;
    const int N = (int)p->n_chains, L = (int)p->max_path_len, d = 4 * (L - 1);
    c->kp.seed = seed;
    c->kp.N = N;
    c->kp.L = L;
    c->kp.d = d;
    c->kp.stddev = p->stddev;
    c->kp.dt = p->dt;
    c->kp.gt = p->dt * p->gamma / 2.0f;
    c->kp.eps = p->eps;
    c->kp.rb = p->rao_blackwell ? 1 : 0;
    const size_t npx = (size_t)s->ds.W * s->ds.H;
    c->n_partials = std::min(1024, (N + 255) / 256);
    KBufs& B = c->kb;
    void* q;
    bool ok = true;
    auto get = [&](void** ptr, size_t bytes) { if (ok && c->mem.get(ptr, bytes) != hipSuccess) ok = false; };
    c->rows_move = 2 * d + (L - 1) + 2;
    c->rows_all = c->rows_move + 6;
    get(&q, sizeof(uint32_t) * c->rows_all * (size_t)N); B.state = (uint32_t*)q;
    get(&q, sizeof(uint32_t) * c->rows_all * (size_t)N); B.alt = (uint32_t*)q;
    if (ok) {
        uint32_t* r = B.state;
        B.x = (float*)r; r += (size_t)d * N;
        B.score = (float*)r; r += (size_t)d * N;
        B.rec = r; r += (size_t)(L - 1) * N;
        B.killed = r; r += N;
        B.ids = r; r += N;
        B.p_tmp = (float*)r; r += N;
        B.r_w = (float*)r; r += N;
        B.pix_tmp = r; r += N;
        B.f_tmp = (float*)r;
    }
    get(&q, sizeof(float) * 3 * npx); B.accum = (float*)q;
    get(&q, sizeof(unsigned long long) * C_N); B.ctr = (unsigned long long*)q;
    get(&q, 64); B.k0 = (float*)q; B.k0d = (double*)((char*)q + 16); B.plam = (double*)((char*)q + 32);
    get(&q, 64); B.queue = (uint32_t*)q;
    get(&q, sizeof(double) * c->n_partials); B.partial = (double*)q;
    get(&q, sizeof(float) * 3 * npx); B.img = (float*)q;
    get(&q, 64); B.steps = (unsigned long long*)q;
    get(&q, sizeof(uint32_t) * N); B.key = (uint32_t*)q;
    get(&q, sizeof(uint32_t) * N); B.order = (uint32_t*)q;
    get(&q, sizeof(uint32_t) * 2 * DR_TILE_BINS); B.bins = (uint32_t*)q;
    B.wf = nullptr;  // the ray-wave buffers are allocated when that form is first selected
    B.sigma = p->sigma_diag;
    if (!ok) {
        c->mem.release();
        delete c;
        return fail(DR_ERR_OUT_OF_MEMORY, "dr_chains_init: device allocation failed");
    }
    hipStream_t st = (hipStream_t)hip_stream;
    if (hipMemsetAsync(B.score, 0, sizeof(float) * d * (size_t)N, st) != hipSuccess) {
        c->mem.release();
        delete c;
        return fail(DR_ERR_DEVICE, "dr_chains_init: clear failed");
    }
    dr_status r = run_init(c, frame, st);
    if (r != DR_OK) {
        c->mem.release();
        delete c;
        return r;
    }
    *out = c;
    g_err.clear();
    return DR_OK;
}

dr_status dr_chains_reinit(dr_chains* c, uint32_t frame, void* hip_stream) {
    if (!c) return fail(DR_ERR_INVALID_ARG, "dr_chains_reinit: null handle");
    HIP_TRY(hipSetDevice(c->scene->device));
    dr_status r = run_init(c, frame, (hipStream_t)hip_stream);
    if (r == DR_OK) g_err.clear();
    return r;
}

dr_status dr_step(dr_chains* c, uint32_t n_steps, void* hip_stream) {
    if (!c) return fail(DR_ERR_INVALID_ARG, "dr_step: null handle");
    if (c->cam_version != c->scene->cam_version)
        return fail(DR_ERR_BAD_STATE, "dr_step: the scene changed since init; call dr_chains_reinit");
    if (n_steps == 0) { g_err.clear(); return DR_OK; }
    HIP_TRY(hipSetDevice(c->scene->device));
    if (enqueue_steps(c, n_steps, (hipStream_t)hip_stream)) c->permuted = true;
    HIP_TRY(hipGetLastError());
    g_err.clear();
    return DR_OK;
}

dr_status dr_resolve(dr_chains* c, float* image_dev, void* hip_stream) {
    if (!c || !image_dev) return fail(DR_ERR_INVALID_ARG, "dr_resolve: null argument");
    HIP_TRY(hipSetDevice(c->scene->device));
    enqueue_resolve(c, image_dev, (hipStream_t)hip_stream);
    HIP_TRY(hipGetLastError());
    g_err.clear();
    return DR_OK;
}

dr_status dr_image_read(dr_chains* c, float* host_rgb, uint64_t* tour_count, void* hip_stream) {
    if (!c || !host_rgb) return fail(DR_ERR_INVALID_ARG, "dr_image_read: null argument");
    HIP_TRY(hipSetDevice(c->scene->device));
    hipStream_t st = (hipStream_t)hip_stream;
    const size_t npx = (size_t)c->scene->ds.W * c->scene->ds.H;
    float* img = c->kb.img;
    dr_status r = dr_resolve(c, img, hip_stream);
    if (r == DR_OK) {
        hipError_t e = hipMemcpyAsync(host_rgb, img, 3 * npx * sizeof(float), hipMemcpyDeviceToHost, st);
        unsigned long long tours = 0;
        if (e == hipSuccess) e = hipMemcpyAsync(&tours, c->kb.ctr + C_TOURS, sizeof(tours), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) r = fail(DR_ERR_DEVICE, std::string("dr_image_read: ") + hipGetErrorString(e));
        if (tour_count) *tour_count = tours;
    }
    if (r == DR_OK) g_err.clear();
    return r;
}

dr_status dr_chains_destroy(dr_chains* c) {
    if (!c) return DR_OK;
    (void)hipSetDevice(c->scene->device);
    (void)hipDeviceSynchronize();
    c->mem.release();
    delete c;
    g_err.clear();
    return DR_OK;
}

dr_status dr_chains_read_state(dr_chains* c, dr_state* o, void* hip_stream) {
    if (!c || !o) return fail(DR_ERR_INVALID_ARG, "dr_chains_read_state: null argument");
    HIP_TRY(hipSetDevice(c->scene->device));
    hipStream_t st = (hipStream_t)hip_stream;
    if (restore_slots(c, st) != DR_OK) return DR_ERR_DEVICE;
    HIP_TRY(hipStreamSynchronize(st));
    const size_t N = c->kp.N, d = c->kp.d, V = c->kp.L - 1;
    const size_t npx = (size_t)c->scene->ds.W * c->scene->ds.H;
    const KBufs& B = c->kb;
    if (o->x) HIP_TRY(hipMemcpy(o->x, B.x, sizeof(float) * d * N, hipMemcpyDeviceToHost));
    if (o->score) HIP_TRY(hipMemcpy(o->score, B.score, sizeof(float) * d * N, hipMemcpyDeviceToHost));
    if (o->killed) HIP_TRY(hipMemcpy(o->killed, B.killed, sizeof(uint32_t) * N, hipMemcpyDeviceToHost));
    if (o->accum) HIP_TRY(hipMemcpy(o->accum, B.accum, sizeof(float) * 3 * npx, hipMemcpyDeviceToHost));
    if (o->p) HIP_TRY(hipMemcpy(o->p, B.p_tmp, sizeof(float) * N, hipMemcpyDeviceToHost));
    if (o->weight) HIP_TRY(hipMemcpy(o->weight, B.r_w, sizeof(float) * N, hipMemcpyDeviceToHost));
    if (o->pixel) HIP_TRY(hipMemcpy(o->pixel, B.pix_tmp, sizeof(uint32_t) * N, hipMemcpyDeviceToHost));
    if (o->f_over_p) HIP_TRY(hipMemcpy(o->f_over_p, B.f_tmp, sizeof(float) * 3 * N, hipMemcpyDeviceToHost));
    if (o->path_rec) {
        HIP_TRY(hipMemcpy(o->path_rec, B.rec, sizeof(uint32_t) * V * N, hipMemcpyDeviceToHost));
        const auto& s2p = c->scene->slot_to_prim;
        for (size_t i = 0; i < V * N; ++i) {
            const uint32_t r = o->path_rec[i];
            if (r != DR_NO_VERTEX) o->path_rec[i] = (s2p[r >> 8] << 8) | (r & 0xFFu);
        }
    }
    unsigned long long ctr[C_N];
    HIP_TRY(hipMemcpy(ctr, B.ctr, sizeof(ctr), hipMemcpyDeviceToHost));
    double k0 = 0, pl = 0;
    HIP_TRY(hipMemcpy(&k0, B.k0d, sizeof(double), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(&pl, B.plam, sizeof(double), hipMemcpyDeviceToHost));
    unsigned long long steps[3];
    HIP_TRY(hipMemcpy(steps, B.steps, sizeof(steps), hipMemcpyDeviceToHost));
    o->step = steps[0];
    o->tour_count = ctr[C_TOURS];
    o->k0 = k0;
    o->p_lambda_hat = pl;
    g_err.clear();
    return DR_OK;
}

dr_status dr_chains_write_state(dr_chains* c, const dr_state* in, void* hip_stream) {
    if (!c || !in) return fail(DR_ERR_INVALID_ARG, "dr_chains_write_state: null argument");
    HIP_TRY(hipSetDevice(c->scene->device));
    if (restore_slots(c, (hipStream_t)hip_stream) != DR_OK) return DR_ERR_DEVICE;
    HIP_TRY(hipStreamSynchronize((hipStream_t)hip_stream));
    const size_t N = c->kp.N, d = c->kp.d;
    const size_t npx = (size_t)c->scene->ds.W * c->scene->ds.H;
    const KBufs& B = c->kb;
    if (in->killed)
        for (size_t i = 0; i < N; ++i)
            if (in->killed[i] > 1) return fail(DR_ERR_INVALID_ARG, "dr_chains_write_state: killed must be 0/1");
    if (in->x) HIP_TRY(hipMemcpy(B.x, in->x, sizeof(float) * d * N, hipMemcpyHostToDevice));
    if (in->score) HIP_TRY(hipMemcpy(B.score, in->score, sizeof(float) * d * N, hipMemcpyHostToDevice));
    if (in->killed) HIP_TRY(hipMemcpy(B.killed, in->killed, sizeof(uint32_t) * N, hipMemcpyHostToDevice));
    if (in->accum) {
        HIP_TRY(hipMemcpy(B.accum, in->accum, sizeof(float) * 3 * npx, hipMemcpyHostToDevice));
        unsigned long long ctr[C_N];
        HIP_TRY(hipMemcpy(ctr, B.ctr, sizeof(ctr), hipMemcpyDeviceToHost));
        ctr[C_TOURS] = in->tour_count;
        HIP_TRY(hipMemcpy(B.ctr, ctr, sizeof(ctr), hipMemcpyHostToDevice));
    }
    if (in->k0 > 0) {
        const double k0 = in->k0;
        const float k0f = (float)k0;
        HIP_TRY(hipMemcpy(B.k0d, &k0, sizeof(double), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(B.k0, &k0f, sizeof(float), hipMemcpyHostToDevice));
    }
    {
        unsigned long long steps[3];
        HIP_TRY(hipMemcpy(steps, B.steps, sizeof(steps), hipMemcpyDeviceToHost));
        steps[0] = in->step;
        HIP_TRY(hipMemcpy(B.steps, steps, sizeof(steps), hipMemcpyHostToDevice));
    }
    g_err.clear();
    return DR_OK;
}

dr_status dr_chains_set_record(dr_chains* c, int enable) {
    if (!c) return fail(DR_ERR_INVALID_ARG, "dr_chains_set_record: null handle");
    c->record = enable ? 1 : 0;
    g_err.clear();
    return DR_OK;
}

dr_status dr_chains_set_counters(dr_chains* c, int enable) {
    if (!c) return fail(DR_ERR_INVALID_ARG, "dr_chains_set_counters: null handle");
    c->count = enable ? 1 : 0;
    g_err.clear();
    return DR_OK;
}

dr_status dr_stats(dr_chains* c, dr_counters* out, void* hip_stream) {
    if (!c || !out) return fail(DR_ERR_INVALID_ARG, "dr_stats: null argument");
    HIP_TRY(hipSetDevice(c->scene->device));
    HIP_TRY(hipStreamSynchronize((hipStream_t)hip_stream));
    unsigned long long ctr[C_N];
    HIP_TRY(hipMemcpy(ctr, c->kb.ctr, sizeof(ctr), hipMemcpyDeviceToHost));
    out->tours = ctr[C_TOURS];
    out->kills = ctr[C_TOURS];
    out->chain_steps = ctr[C_STEPS];
    out->rays = ctr[C_RAYS];
    out->node_visits = ctr[C_NODES];
    out->tri_tests = ctr[C_TRIS];
    out->adjoints = ctr[C_ADJ];
    HIP_TRY(hipMemcpy(&out->k0, c->kb.k0d, sizeof(double), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(&out->p_lambda_hat, c->kb.plam, sizeof(double), hipMemcpyDeviceToHost));
    g_err.clear();
    return DR_OK;
}

dr_status dr_chains_set_launch(dr_chains* c, const dr_launch_cfg* cfg) {
    if (!c || !cfg) return fail(DR_ERR_INVALID_ARG, "dr_chains_set_launch: null argument");
    if (cfg->block && (cfg->block % 64 != 0 || cfg->block > 256))
        return fail(DR_ERR_INVALID_ARG, "dr_chains_set_launch: block must be 64, 128, 192 or 256");
    if (cfg->blocks_per_cu > 64) return fail(DR_ERR_INVALID_ARG, "dr_chains_set_launch: blocks_per_cu must be <= 64");
    if (cfg->grab > 64) return fail(DR_ERR_INVALID_ARG, "dr_chains_set_launch: grab must be <= 64");
    if (cfg->lanes_per_chain > 2) return fail(DR_ERR_INVALID_ARG, "dr_chains_set_launch: lanes_per_chain must be 1 or 2");
    if (cfg->sort_by_length > 2) return fail(DR_ERR_INVALID_ARG, "dr_chains_set_launch: sort_by_length must be 0, 1 or 2");
    if (cfg->refill > 2) return fail(DR_ERR_INVALID_ARG, "dr_chains_set_launch: refill must be 0, 1 or 2");
    if (cfg->sort_by_tile > 2) return fail(DR_ERR_INVALID_ARG, "dr_chains_set_launch: sort_by_tile must be 0, 1 or 2");
    if (cfg->wavefront > 2) return fail(DR_ERR_INVALID_ARG, "dr_chains_set_launch: wavefront must be 0, 1 or 2");
    if (cfg->init_refill > 2) return fail(DR_ERR_INVALID_ARG, "dr_chains_set_launch: init_refill must be 0, 1 or 2");
    if (cfg->refill_event_pct > 100 || cfg->refill_advance_pct > 100)
        return fail(DR_ERR_INVALID_ARG, "dr_chains_set_launch: refill thresholds are percentages (1..100)");
    // the one request that allocates, before any field changes (a failed call changes nothing)
    if (cfg->wavefront == 1) {
        HIP_TRY(hipSetDevice(c->scene->device));
        if (ensure_wf_buffers(c) != hipSuccess)
            return fail(DR_ERR_OUT_OF_MEMORY, "dr_chains_set_launch: ray-wave buffer allocation failed");
    }
    if (cfg->block) c->launch.block = cfg->block;
    if (cfg->blocks_per_cu) c->launch.blocks_per_cu = cfg->blocks_per_cu;
    if (cfg->grab) c->launch.grab = cfg->grab;
    if (cfg->lanes_per_chain) c->launch.lanes_per_chain = cfg->lanes_per_chain;
    if (cfg->sort_by_length) c->launch.sort_by_length = cfg->sort_by_length == 1 ? 1u : 0u;
    if (cfg->refill) c->launch.refill = cfg->refill == 1 ? 1u : 0u;
    if (cfg->sort_by_tile) c->launch.sort_by_tile = cfg->sort_by_tile == 1 ? 1u : 0u;
    if (cfg->wavefront) c->launch.wavefront = cfg->wavefront == 1 ? 1u : 0u;
    if (cfg->init_refill) c->launch.init_refill = cfg->init_refill == 1 ? 1u : 0u;
    if (cfg->refill_event_pct) c->launch.refill_event_pct = cfg->refill_event_pct;
    if (cfg->refill_advance_pct) c->launch.refill_advance_pct = cfg->refill_advance_pct;
    g_err.clear();
    return DR_OK;
}

dr_status dr_chains_get_launch(dr_chains* c, dr_launch_cfg* cfg) {
    if (!c || !cfg) return fail(DR_ERR_INVALID_ARG, "dr_chains_get_launch: null argument");
    *cfg = c->launch;
    g_err.clear();
    return DR_OK;
}

// Enqueue the evaluation kernels with the caller's scratch: 4 bytes (the
// forward-only evaluator's work counter, cleared by a fill kernel) or
// 4 (L-1) n bytes (the score pass's path records).
static void enqueue_eval(dr_scene* s, uint32_t L, const float* u_dev, uint32_t n, float eps, float* f_dev,
                         float* logp_dev, float* grad_dev, uint32_t* rec_dev, uint32_t* rs, hipStream_t st) {
    if (!grad_dev) {
        // forward only: the ray-refill evaluator, persistent, points taken
        // from a counter in the scratch buffer
        const int blk = 256;
        const int blocks = (int)std::min<long>((long)g_num_cu(s->device) * 4, ((long)n + blk - 1) / blk);
        hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, rs, (size_t)1, 0u);
        DR_DISPATCH_L((int)L, launch_eval_sm, dim3(blocks), dim3(blk), st, s->ds, u_dev, (int)n, eps, f_dev,
                      logp_dev, rec_dev, rs, 50);
    } else {
        const int blk = 128;
        DR_DISPATCH_L((int)L, launch_eval, dim3((n + blk - 1) / blk), dim3(blk), st, s->ds, u_dev, (int)n, eps, f_dev,
                      logp_dev, grad_dev, rs, rec_dev);
    }
}

static size_t eval_scratch_bytes(uint32_t L, uint32_t n, bool grad) {
    return grad ? sizeof(uint32_t) * (L - 1) * (size_t)n : sizeof(uint32_t);
}

// Scratch of dr_eval_logp_grad_noalloc: a file-scope device array (each GPU
// the library runs on holds its own copy until the process ends).  Host code
// never passes the array's name to a kernel: it takes the array's device
// address from hipGetSymbolAddress once per device (with that device
// current) and passes that address.
#define DR_NOALLOC_SCRATCH_BYTES (16u << 20)
static __device__ __align__(256) uint32_t scratch[DR_NOALLOC_SCRATCH_BYTES / sizeof(uint32_t)];
namespace {
std::mutex g_scratch_mu;
std::vector<uint32_t*> g_scratch_ptr;  // per device, nullptr until resolved
}  // namespace

static dr_status noalloc_scratch(int device, uint32_t** out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((int)g_scratch_ptr.size() <= device) g_scratch_ptr.resize((size_t)device + 1, nullptr);
    if (!g_scratch_ptr[device]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(DR_ERR_DEVICE, std::string("dr_eval_logp_grad_noalloc: scratch address: ") +
                                           hipGetErrorString(e));
        g_scratch_ptr[device] = static_cast<uint32_t*>(ptr);
    }
    *out = g_scratch_ptr[device];
    return DR_OK;
}

dr_status dr_eval_logp_grad(dr_scene* s, uint32_t L, const float* u_dev, uint32_t n, float eps, float* f_dev,
                            float* logp_dev, float* grad_dev, uint32_t* rec_dev, void* hip_stream) {
    if (!s || !u_dev) return fail(DR_ERR_INVALID_ARG, "dr_eval_logp_grad: null argument");
    if (L < 2 || L > 16) return fail(DR_ERR_INVALID_ARG, "dr_eval_logp_grad: L must be 2..16");
    if (!(eps > 0)) return fail(DR_ERR_INVALID_ARG, "dr_eval_logp_grad: eps must be > 0");
    if (n == 0) { g_err.clear(); return DR_OK; }
    HIP_TRY(hipSetDevice(s->device));
    (void)hipGetLastError();  // drop a stale error left by an earlier, unrelated call
    hipStream_t st = (hipStream_t)hip_stream;
    void* rs = nullptr;
    const AllocHooks hooks = g_hooks;
    const size_t rs_bytes = eval_scratch_bytes(L, n, grad_dev != nullptr);
    if (hooks.alloc) {
        if (dev_alloc(&rs, rs_bytes, st, hooks) != hipSuccess)
            return fail(DR_ERR_OUT_OF_MEMORY, "dr_eval_logp_grad: scratch allocation failed");
    } else {
        HIP_TRY(hipMallocAsync(&rs, rs_bytes, st));
    }
    enqueue_eval(s, L, u_dev, n, eps, f_dev, logp_dev, grad_dev, rec_dev, (uint32_t*)rs, st);
    hipError_t e = hipGetLastError();
    if (hooks.alloc) dev_free(rs, rs_bytes, st, hooks);
    else (void)hipFreeAsync(rs, st);
    if (e != hipSuccess) return fail(DR_ERR_DEVICE, std::string("dr_eval_logp_grad: ") + hipGetErrorString(e));
    g_err.clear();
    return DR_OK;
}

dr_status dr_eval_logp_grad_noalloc(dr_scene* s, uint32_t L, const float* u_dev, uint32_t n, float eps, float* f_dev,
                                    float* logp_dev, float* grad_dev, uint32_t* rec_dev, void* hip_stream) {
    if (!s || !u_dev) return fail(DR_ERR_INVALID_ARG, "dr_eval_logp_grad_noalloc: null argument");
    if (L < 2 || L > 16) return fail(DR_ERR_INVALID_ARG, "dr_eval_logp_grad_noalloc: L must be 2..16");
    if (!(eps > 0)) return fail(DR_ERR_INVALID_ARG, "dr_eval_logp_grad_noalloc: eps must be > 0");
    if (eval_scratch_bytes(L, n, grad_dev != nullptr) > DR_NOALLOC_SCRATCH_BYTES)
        return fail(DR_ERR_INVALID_ARG, "dr_eval_logp_grad_noalloc: with a score, 4 (L-1) n bytes of scratch must fit "
                                        "the library's 16 MiB");
    if (n == 0) { g_err.clear(); return DR_OK; }
    HIP_TRY(hipSetDevice(s->device));
    (void)hipGetLastError();  // drop a stale error left by an earlier, unrelated call
    uint32_t* rs = nullptr;
    if (noalloc_scratch(s->device, &rs) != DR_OK) return DR_ERR_DEVICE;
    enqueue_eval(s, L, u_dev, n, eps, f_dev, logp_dev, grad_dev, rec_dev, rs, (hipStream_t)hip_stream);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return fail(DR_ERR_DEVICE, std::string("dr_eval_logp_grad_noalloc: ") + hipGetErrorString(e));
    g_err.clear();
    return DR_OK;
}

dr_status dr_pt_render(dr_scene* s, uint32_t L, uint64_t seed, uint32_t spp, float* img_dev, void* hip_stream) {
    if (!s || !img_dev) return fail(DR_ERR_INVALID_ARG, "dr_pt_render: null argument");
    if (L < 2 || L > 16 || spp == 0) return fail(DR_ERR_INVALID_ARG, "dr_pt_render: L must be 2..16 and spp >= 1");
    HIP_TRY(hipSetDevice(s->device));
    (void)hipGetLastError();  // drop a stale error left by an earlier, unrelated call
    const int npx = s->ds.W * s->ds.H;
    const int blk = 128;
    if (s->has_delta)
        hipLaunchKernelGGL(k_pt<true>, dim3((npx + blk - 1) / blk), dim3(blk), stack_bytes(s->ds, blk),
                           (hipStream_t)hip_stream, s->ds, (int)L, seed, spp, img_dev);
    else
        hipLaunchKernelGGL(k_pt<false>, dim3((npx + blk - 1) / blk), dim3(blk), stack_bytes(s->ds, blk),
                           (hipStream_t)hip_stream, s->ds, (int)L, seed, spp, img_dev);
    HIP_TRY(hipGetLastError());
    g_err.clear();
    return DR_OK;
}

dr_status dr_frame_capture(dr_chains* c, uint32_t n_steps, int reinit, float* image_dev, void* hip_stream,
                           dr_frame** out) {
    if (!c || !image_dev || !out) return fail(DR_ERR_INVALID_ARG, "dr_frame_capture: null argument");
    if (!hip_stream) return fail(DR_ERR_INVALID_ARG, "dr_frame_capture: needs a non-default stream to capture on");
    HIP_TRY(hipSetDevice(c->scene->device));
    hipStream_t st = (hipStream_t)hip_stream;
    HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    if (reinit) enqueue_init(c, 0, 1, st);
    // capturing runs nothing: the slot bookkeeping changes only at launch
    const bool permutes = n_steps ? enqueue_steps(c, n_steps, st) : false;
    enqueue_resolve(c, image_dev, st);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(st, &g);
    if (e != hipSuccess) return fail(DR_ERR_DEVICE, std::string("dr_frame_capture: ") + hipGetErrorString(e));
    hipGraphExec_t ge = nullptr;
    e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(DR_ERR_DEVICE, std::string("dr_frame_capture: instantiate: ") + hipGetErrorString(e));
    }
    auto* f = new dr_frame();
    f->c = c;
    f->graph = g;
    f->exec = ge;
    f->reinit = reinit ? 1 : 0;
    f->permutes = permutes;
    *out = f;
    g_err.clear();
    return DR_OK;
}

dr_status dr_frame_launch(dr_frame* f, void* hip_stream) {
    if (!f) return fail(DR_ERR_INVALID_ARG, "dr_frame_launch: null handle");
    dr_chains* c = f->c;
    if (!f->reinit && c->cam_version != c->scene->cam_version)
        return fail(DR_ERR_BAD_STATE, "dr_frame_launch: the scene changed and this frame does not re-initialise");
    HIP_TRY(hipSetDevice(c->scene->device));
    HIP_TRY(hipGraphLaunch(f->exec, (hipStream_t)hip_stream));
    if (f->reinit) c->cam_version = c->scene->cam_version;
    // the initialise pass puts chain c in slot c; ordered steps then move them
    if (f->permutes) c->permuted = true;
    else if (f->reinit) c->permuted = false;
    g_err.clear();
    return DR_OK;
}

dr_status dr_frame_destroy(dr_frame* f) {
    if (!f) return DR_OK;
    (void)hipSetDevice(f->c->scene->device);
    if (f->exec) (void)hipGraphExecDestroy(f->exec);
    if (f->graph) (void)hipGraphDestroy(f->graph);
    delete f;
    g_err.clear();
    return DR_OK;
}

}  // extern "C"
