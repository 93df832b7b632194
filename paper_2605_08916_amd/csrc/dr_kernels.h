// L-templated kernels of the chain-step library and their host launchers.
//
// Each launcher is explicitly instantiated for L = 2..16 in the dr_inst_*.hip
// translation units (compiled in parallel); dr_lib.hip declares them extern
// and dispatches on L at run time.  Nothing here is built on its own.
#pragma once

#include <hip/hip_runtime.h>

#include "dr_adjoint.h"
#include "dr_chain.h"
#include "dr_device.h"
#include "dr_machine.h"

using namespace dr;

// ===========================================================================
// Kernel-side parameter blocks
// ===========================================================================
struct KParams {
    uint64_t seed;
    int N, L, d;
    float stddev, dt, gt, eps;  // gt = gamma tilde = dt gamma / 2
    int rb, record, count;
};

struct KBufs {
    float* x;            // d x N
    float* score;        // d x N
    uint32_t* killed;    // N
    uint32_t* rec;       // (L-1) x N, triangle slots
    float* accum;        // 3 x W*H, sum of (w/dt) f/p
    unsigned long long* ctr;  // [0] tours, [1] chain steps, [2] rays, [3] nodes, [4] tris, [5] adjoints
    float* k0;           // device scalar (float) ; k0d at ((double*)k0ptr)
    double* k0d;
    double* plam;        // p_lambda estimate
    const float* sigma;  // d x N or null
    uint32_t* queue;
    // per-chain scratch and record
    float* p_tmp;        // N
    float* f_tmp;        // 3 x N
    uint32_t* pix_tmp;   // N
    float* r_w;          // N (record)
    double* partial;     // reduction partials
    float* img;          // 3 x W*H resolved image (dr_image_read)
    // step counters in device memory so captured graphs replay correctly:
    // [0] next step index, [1] first step index of the current launch, [2] frame
    unsigned long long* steps;
    // Chain state sits in slots; ids[slot] is the chain occupying it (its RNG
    // streams and its row of a per-chain Sigma).  The fused form may move
    // chains between slots so chains with equal last path length share a
    // wavefront: key per slot (vertex count, or DR_NBIN-1 for a killed chain),
    // order = source slot of each destination slot, bins = counting-sort
    // counts and offsets, alt = staging rows for the move.
    uint32_t* ids;
    uint32_t* key;
    uint32_t* order;
    uint32_t* bins;
    uint32_t* state;  // rows: x[d], score[d], rec[L-1], killed, ids, then the record rows p, w, pix, f[3]
    // ray waves (the wavefront form of a path pass): per slot the path state
    // between ray queries (DR_WF_ROWS rows), the pending ray (o, tmax | d,
    // anyhit), its answer, and two queues of slots with a ray in flight
    uint32_t* wf;
    float4* wf_ray;
    int* wf_hit;
    float* wf_t;
    uint32_t* wf_q;    // 2 x N slot queues
    uint32_t* wf_cnt;  // [0], [1] queue lengths, [2] trace work counter
    uint32_t* alt;    // same shape as state
};

#define DR_NBIN 9

enum { C_TOURS = 0, C_STEPS = 1, C_RAYS = 2, C_NODES = 3, C_TRIS = 4, C_ADJ = 5, C_N = 8 };

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Add a per-lane count to a global counter with one atomic per wavefront.
// Must be called by all active lanes of the wavefront together.
__device__ __forceinline__ void wave_add(unsigned long long* dst, uint32_t v) {
    const uint32_t s = wave_sum(v);
    const uint64_t act = __ballot(1);
    if ((threadIdx.x & 63) == (uint32_t)(__ffsll((long long)act) - 1) && s) atomicAdd(dst, (unsigned long long)s);
}

// Hold/kill and splat (Accumulate).  Returns true if the tour survives.
// c: slot of the chain, id: the chain (RNG streams).
__device__ __forceinline__ bool hold_kill_splat(const KParams& P, const KBufs& B, const DevScene& S, int c, int id,
                                                uint64_t s, float k0, V3 f, float p, uint32_t pix, bool lead = true) {
    float wdt;
    const bool alive = hold_kill(P.seed, id, s, k0, p, P.eps, P.dt, P.rb, wdt);
    if (lead && p > 0.0f) {
        const float sc = wdt / p;
        const size_t npx = (size_t)S.W * S.H;
        atomicAdd(&B.accum[pix], sc * f.x);
        atomicAdd(&B.accum[npx + pix], sc * f.y);
        atomicAdd(&B.accum[2 * npx + pix], sc * f.z);
    }
    if (P.record) {
        B.p_tmp[c] = p;
        B.r_w[c] = wdt * P.dt;
        B.pix_tmp[c] = pix;
        B.f_tmp[c] = p > 0.0f ? f.x / p : 0.0f;
        B.f_tmp[(size_t)P.N + c] = p > 0.0f ? f.y / p : 0.0f;
        B.f_tmp[(size_t)2 * P.N + c] = p > 0.0f ? f.z / p : 0.0f;
    }
    return alive;
}

template <int L, bool DELTA = true>
__device__ __forceinline__ void score_at(const KParams& P, const KBufs& B, const DevScene& S, int c, float p) {
    path_score<L, DELTA>(S, SoaU{B.x + c, P.N}, B.rec + c, P.N, p, P.eps, B.score + c, P.N);
}

// Traversal stack bytes of a block (the tree's exact per-lane need).
inline size_t stack_bytes(const DevScene& S, int block) { return (size_t)S.stack_cap * block * sizeof(uint32_t); }

// Initialise, phase 2: hold/kill/splat with the final k0, then scores.
template <int L>
__global__ void __launch_bounds__(256) k_init_accumulate(KParams P, DevScene S, KBufs B, int with_score) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t s0 = B.steps[1];
    uint32_t kill = 0, adj = 0;
    if (c < P.N) {
        const float p = B.p_tmp[c];
        const V3 f = v3(B.f_tmp[c], B.f_tmp[(size_t)P.N + c], B.f_tmp[(size_t)2 * P.N + c]);
        const bool alive = hold_kill_splat(P, B, S, c, c, s0, *B.k0, f, p, B.pix_tmp[c]);
        B.killed[c] = alive ? 0u : 1u;
        if (!alive) B.key[c] = DR_NBIN - 1;
        kill = alive ? 0u : 1u;
        if (alive && with_score) {
            score_at<L>(P, B, S, c, p);
            adj = 1;
        }
    }
    wave_add(&B.ctr[C_TOURS], kill);
    if (P.count) {
        wave_add(&B.ctr[C_STEPS], c < P.N ? 1u : 0u);
        wave_add(&B.ctr[C_ADJ], adj);
    }
}

// Fused persistent evolve step: every chain advances nsteps steps.  With
// PAIR, two adjacent lanes share a chain: both run its step on the same data,
// the path's continuation and shadow rays are traced concurrently (one per
// lane), and only the even lane performs the atomics.
template <int L, bool PAIR, bool DELTA>
__device__ __forceinline__ void step_fused_body(const KParams& P, const DevScene& S, const KBufs& B, uint32_t nsteps,
                                                uint32_t grab, int sorted) {
    extern __shared__ uint32_t s_stack[];
    uint32_t* stk = s_stack + threadIdx.x;
    const int stride = blockDim.x;
    const int lane = threadIdx.x & 63;
    const bool lead = PAIR ? (lane & 1) == 0 : true;
    const float k0 = *B.k0;
    const uint64_t s0 = B.steps[1];
    int c = -1, cend = -1;
    uint32_t k = nsteps;
    Counters ctr = {0, 0, 0};
    uint32_t kills = 0, steps = 0, adj = 0;
    while (true) {
        // a lane done with its chain moves to the next of its `grab` chains;
        // units (lanes or lane pairs) out of chains refill with one queue
        // atomic per wavefront
        if (k >= nsteps && c + 1 < cend) {
            ++c;
            k = 0;
        }
        const bool need = k >= nsteps;
        const uint64_t mask = __ballot(need);
        if (mask) {
            const uint64_t umask = PAIR ? (mask & 0x5555555555555555ull) : mask;
            const int leader = __ffsll((long long)umask) - 1;
            uint32_t base = 0;
            if (lane == leader) base = atomicAdd(B.queue, (uint32_t)__popcll(umask) * grab);
            base = __shfl(base, leader);
            if (need) {
                const int me = PAIR ? (lane & ~1) : lane;
                const uint32_t first = base + (uint32_t)__popcll(umask & ((1ull << me) - 1ull)) * grab;
                c = (int)min(first, (uint32_t)P.N);
                cend = (int)min(first + grab, (uint32_t)P.N);
                k = 0;
            }
        }
        const bool active = c < cend;
        if (!__any(active)) break;
        if (active) {
            const uint64_t s = s0 + k;
            const int id = (int)B.ids[c];  // the chain in slot c
            float* xc = B.x + c;
            // both lanes of a pair store identical values
            const bool was_killed = B.killed[c] != 0;
            if (was_killed) regen(P.seed, P.d, P.N, xc, id, s);
            else move(P.seed, P.d, P.N, P.stddev, P.gt, xc, B.score + c, B.sigma ? B.sigma + id : nullptr, id, s);
            const SoaU u{xc, P.N};
            int nv;
            const V3 f = path_forward<PAIR, DELTA>(S, L, u, B.rec + c, P.N, stk, stride, ctr, &nv);
            const float p = lum(f);
            const uint32_t pix = pixel_of(S, xc[0], xc[P.N]);
            const bool alive = hold_kill_splat(P, B, S, c, id, s, k0, f, p, pix, lead);
            B.killed[c] = alive ? 0u : 1u;
            if (sorted) B.key[c] = alive ? (uint32_t)nv : (uint32_t)(DR_NBIN - 1);
            if (lead) kills += alive ? 0u : 1u;
            if (alive) {
                score_at<L, DELTA>(P, B, S, c, p);
                if (lead) ++adj;
            }
            ++k;
            if (lead) ++steps;
        } else {
            k = 0;  // drained lanes stop asking for work
            cend = c;
        }
    }
    wave_add(&B.ctr[C_TOURS], kills);
    if (P.count) {
        wave_add(&B.ctr[C_STEPS], steps);
        wave_add(&B.ctr[C_ADJ], adj);
        wave_add(&B.ctr[C_RAYS], ctr.rays);
        wave_add(&B.ctr[C_NODES], ctr.nodes);
        wave_add(&B.ctr[C_TRIS], ctr.tris);
    }
}

// Paired lanes (two per chain): at 128 of the kernel's registers or more a
// SIMD holds two wavefronts, which is all the paired form has at the chain
// counts it is used for.  DELTA: the scene has smooth conductors or
// dielectrics (false compiles their handling out).
template <int L, bool DELTA>
__global__ void __launch_bounds__(256) k_step_fused_pair(KParams P, DevScene S, KBufs B, uint32_t nsteps, uint32_t grab,
                                                         int sorted) {
    step_fused_body<L, true, DELTA>(P, S, B, nsteps, grab, sorted);
}
// One lane per chain (used when chains outnumber two wavefronts per SIMD):
// registers capped for three wavefronts per SIMD, which hides more of the
// traversal's memory latency than the spills it costs.
template <int L, bool DELTA>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3)))
k_step_fused(KParams P, DevScene S, KBufs B, uint32_t nsteps, uint32_t grab, int sorted) {
    step_fused_body<L, false, DELTA>(P, S, B, nsteps, grab, sorted);
}

// Path records of the chain in slot c, written as the state machine reaches
// each vertex.
template <int L>
struct StepRec {
    uint32_t* rec;
    int N, c;
    __device__ __forceinline__ void vertex(int j, uint32_t r) const { rec[(size_t)(j - 1) * N + c] = r; }
    __device__ __forceinline__ void finish(V3, int nv) const {
        for (int j = nv + 1; j <= L - 1; ++j) rec[(size_t)(j - 1) * N + c] = DR_NO_VERTEX;
    }
};

enum { LS_POP = 0, LS_ADVANCE = 1, LS_EVENT = 2, LS_TRACE = 3, LS_DONE = 4 };

// Fused persistent evolve step with ray-level refill: one lane per chain,
// every chain advances nsteps steps (the same arithmetic and random streams as
// k_step_fused).  A lane is in one of four states:
//   POP      out of chains: takes the next one from the work queue;
//   ADVANCE  finishes its chain's last step (hold/kill, splat, adjoint) and
//            starts the next (move or regenerate, camera ray);
//   EVENT    its ray query finished: shade, issue the next ray or end the path;
//   TRACE    a ray query in flight.
// Each iteration the wavefront runs one of ADVANCE, EVENT or one node visit
// of TRACE: ADVANCE once adv_pct percent of the busy lanes wait for it, EVENT
// once ev_pct percent of the lanes tracing or waiting for an event do, and the
// traversal otherwise.  So traversal keeps most lanes busy, and the long
// ADVANCE code runs for many chains at once.
template <int L, bool DELTA>
__global__ void __launch_bounds__(256) k_step_sm(KParams P, DevScene S, KBufs B, uint32_t nsteps, int sorted,
                                                 int ev_pct, int adv_pct) {
    extern __shared__ uint32_t s_stack[];
    uint32_t* stk = s_stack + threadIdx.x;
    const int stride = blockDim.x;
    const int lane = threadIdx.x & 63;
    const float k0 = *B.k0;
    const uint64_t s0 = B.steps[1];
    const Cam C = load_cam(S);
    Counters ctr = {0, 0, 0};
    uint32_t kills = 0, steps = 0, adj = 0;
    RayQ q;
    PathSM ps;
    int state = LS_POP;
    int c = 0, id = 0;
    uint32_t k = 0;
    bool has_path = false;  // a finished path waits for its hold/kill, splat and adjoint
    while (true) {
        const bool need = state == LS_POP;
        const uint64_t nm = __ballot(need);
        if (nm) {
            const int leader = __ffsll((long long)nm) - 1;
            uint32_t base = 0;
            if (lane == leader) base = atomicAdd(B.queue, (uint32_t)__popcll(nm));
            base = __shfl(base, leader);
            if (need) {
                const uint32_t it = base + (uint32_t)__popcll(nm & ((1ull << lane) - 1ull));
                if (it < (uint32_t)P.N) {
                    c = (int)it;
                    id = (int)B.ids[c];
                    k = 0;
                    has_path = false;
                    state = LS_ADVANCE;
                } else {
                    state = LS_DONE;
                }
            }
        }
        const uint64_t mt = __ballot(state == LS_TRACE), me = __ballot(state == LS_EVENT),
                       ma = __ballot(state == LS_ADVANCE);
        if (!(mt | me | ma)) break;
        const int nt = __popcll(mt), ne = __popcll(me), na = __popcll(ma);
        if (na && (nt + ne == 0 || 100 * na >= adv_pct * (nt + ne + na))) {
            if (state == LS_ADVANCE) {
                if (has_path) {
                    const uint64_t s = s0 + k;
                    const float p = lum(ps.f);
                    const uint32_t pix = pixel_of(S, B.x[c], B.x[(size_t)P.N + c]);
                    const bool alive = hold_kill_splat(P, B, S, c, id, s, k0, ps.f, p, pix);
                    B.killed[c] = alive ? 0u : 1u;
                    if (sorted) B.key[c] = alive ? (uint32_t)ps.nv : (uint32_t)(DR_NBIN - 1);
                    kills += alive ? 0u : 1u;
                    if (alive) {
                        score_at<L, DELTA>(P, B, S, c, p);
                        ++adj;
                    }
                    ++steps;
                    ++k;
                    has_path = false;
                }
                if (k < nsteps) {
                    const uint64_t s = s0 + k;
                    float* xc = B.x + c;
                    if (B.killed[c]) regen(P.seed, P.d, P.N, xc, id, s);
                    else
                        move(P.seed, P.d, P.N, P.stddev, P.gt, xc, B.score + c, B.sigma ? B.sigma + id : nullptr, id,
                             s);
                    ps.phase = PH_NEW;
                    sm_event<L, DELTA>(S, C, SoaU{xc, P.N}, ps, q, StepRec<L>{B.rec, P.N, c}, ctr);
                    state = LS_TRACE;
                } else {
                    state = LS_POP;
                }
            }
        } else if (ne && (nt == 0 || 100 * ne >= ev_pct * (nt + ne))) {
            if (state == LS_EVENT) {
                if (sm_event<L, DELTA>(S, C, SoaU{B.x + c, P.N}, ps, q, StepRec<L>{B.rec, P.N, c}, ctr)) {
                    state = LS_TRACE;
                } else {
                    state = LS_ADVANCE;
                    has_path = true;
                }
            }
        } else {
            uint64_t ml, mv;
            ray_masks(q, state == LS_TRACE, ml, mv);
            if (state == LS_TRACE && ray_step(S, q, stk, stride, ctr, ml, mv)) state = LS_EVENT;
        }
    }
    wave_add(&B.ctr[C_TOURS], kills);
    if (P.count) {
        wave_add(&B.ctr[C_STEPS], steps);
        wave_add(&B.ctr[C_ADJ], adj);
        wave_add(&B.ctr[C_RAYS], ctr.rays);
        wave_add(&B.ctr[C_NODES], ctr.nodes);
        wave_add(&B.ctr[C_TRIS], ctr.tris);
    }
}

// ---- plain multi-kernel form -------------------------------------------------
// score = grad ln(p + eps) at the current state of every live chain.
template <int L>
__global__ void __launch_bounds__(256) k_plain_score(KParams P, DevScene S, KBufs B) {
    extern __shared__ uint32_t s_stack[];
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    Counters ctr = {0, 0, 0};
    uint32_t adj = 0;
    if (c < P.N && !B.killed[c]) {
        const SoaU u{B.x + c, P.N};
        const V3 f = path_forward<false>(S, L, u, B.rec + c, P.N, s_stack + threadIdx.x, blockDim.x, ctr);
        score_at<L>(P, B, S, c, lum(f));
        adj = 1;
    }
    if (P.count) {
        wave_add(&B.ctr[C_ADJ], adj);
        wave_add(&B.ctr[C_RAYS], ctr.rays);
        wave_add(&B.ctr[C_NODES], ctr.nodes);
        wave_add(&B.ctr[C_TRIS], ctr.tris);
    }
}
// Path evaluation for n points (row-major n x d): f, log(p + eps), score, record.
struct RowU {
    static constexpr bool kChecked = true;
    const float* p;
    __device__ __forceinline__ float operator()(int i) const { return p[i]; }
};
template <int L>
__global__ void __launch_bounds__(256) k_eval(DevScene S, const float* u, int n, float eps, float* fo, float* logp, float* grad,
                       uint32_t* rec_scratch, uint32_t* rec_out) {
    extern __shared__ uint32_t s_stack[];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    constexpr int d = 4 * (L - 1);
    Counters ctr = {0, 0, 0};
    const RowU uu{u + (size_t)i * d};
    uint32_t* rc = rec_scratch + i;
    const V3 f = path_forward<false>(S, L, uu, rc, n, s_stack + threadIdx.x, blockDim.x, ctr);
    const float p = lum(f);
    if (fo) {
        fo[3 * (size_t)i] = f.x;
        fo[3 * (size_t)i + 1] = f.y;
        fo[3 * (size_t)i + 2] = f.z;
    }
    if (logp) logp[i] = logf(p + eps);
    if (grad) path_score<L>(S, uu, rc, n, p, eps, grad + (size_t)i * d, 1);
    if (rec_out)
        for (int j = 0; j < L - 1; ++j) {
            const uint32_t r = rc[(size_t)j * n];
            rec_out[(size_t)i * (L - 1) + j] =
                r == DR_NO_VERTEX ? r : ((__float_as_uint(S.tris[r >> 8].v0.w) << 8) | (r & 0xFFu));
        }
}

// Outputs of the state-machine evaluator for point i.
template <int L>
struct EvalRec {
    const DevTri* tris;
    uint32_t* rec_out;
    float* fo;
    float* logp;
    float eps;
    int i;
    __device__ __forceinline__ void vertex(int j, uint32_t r) const {
        if (rec_out)
            rec_out[(size_t)i * (L - 1) + (j - 1)] = (__float_as_uint(tris[r >> 8].v0.w) << 8) | (r & 0xFFu);
    }
    __device__ __forceinline__ void finish(V3 f, int nv) const {
        if (rec_out)
            for (int j = nv + 1; j <= L - 1; ++j) rec_out[(size_t)i * (L - 1) + (j - 1)] = DR_NO_VERTEX;
        if (fo) {
            fo[3 * (size_t)i] = f.x;
            fo[3 * (size_t)i + 1] = f.y;
            fo[3 * (size_t)i + 2] = f.z;
        }
        if (logp) logp[i] = logf(lum(f) + eps);
    }
};

// Forward evaluation of n points with the ray-refill state machine
// (persistent; points are taken from a device counter).  thresh: events run
// once at least thresh percent of the busy lanes wait for one.
template <int L>
__global__ void __launch_bounds__(256) k_eval_sm(DevScene S, const float* u, int n, float eps, float* fo, float* logp,
                                                 uint32_t* rec_out, uint32_t* queue, int thresh) {
    extern __shared__ uint32_t s_stack[];
    uint32_t* stk = s_stack + threadIdx.x;
    const int stride = blockDim.x;
    const int lane = threadIdx.x & 63;
    constexpr int d = 4 * (L - 1);
    const Cam C = load_cam(S);
    Counters ctr = {0, 0, 0};
    RayQ q;
    PathSM P;
    P.phase = PH_NEW;
    int item = -1;
    bool tracing = false, drained = false;
    while (true) {
        const bool need = !drained && item < 0;
        const uint64_t nm = __ballot(need);
        if (nm) {
            const int leader = __ffsll((long long)nm) - 1;
            uint32_t base = 0;
            if (lane == leader) base = atomicAdd(queue, (uint32_t)__popcll(nm));
            base = __shfl(base, leader);
            if (need) {
                const uint32_t it = base + (uint32_t)__popcll(nm & ((1ull << lane) - 1ull));
                if (it < (uint32_t)n) item = (int)it;
                else drained = true;
            }
        }
        const bool ev = !drained && !tracing;
        const uint64_t em = __ballot(ev), tm = __ballot(tracing);
        if (!em && !tm) break;
        const int nev = __popcll(em), ntr = __popcll(tm);
        if (nev && (!ntr || 100 * nev >= thresh * (nev + ntr))) {
            if (ev) {
                const RowU uu{u + (size_t)item * d};
                const EvalRec<L> R{S.tris, rec_out, fo, logp, eps, item};
                tracing = sm_event<L>(S, C, uu, P, q, R, ctr);
                if (!tracing) item = -1;
            }
        } else {
            uint64_t ml, mv;
            ray_masks(q, tracing, ml, mv);
            if (tracing && ray_step(S, q, stk, stride, ctr, ml, mv)) tracing = false;
        }
    }
}

// ---------------------------------------------------------------------------
// Ray waves: a path pass as alternating launches of a traversal kernel (all
// pending rays, persistent lanes that take the next ray as theirs finishes)
// and an event kernel (each path whose ray finished shades its vertex and
// issues its next ray, or ends).  The path arithmetic is the state machine's
// (dr_machine.h), the same operations as path_forward, so results are
// bit-identical to the straight-line kernels; the traversal kernel holds no
// shading code, so its lanes stay busy with traversal.
// ---------------------------------------------------------------------------
#define DR_WF_ROWS 33

// Path state of slot c <-> rows of B.wf (planar, coalesced per wavefront).
__device__ __forceinline__ void wf_store(const KBufs& B, size_t N, int c, const PathSM& P) {
    uint32_t* w = B.wf + c;
    int r = 0;
    auto put = [&](uint32_t v) { w[(size_t)(r++) * N] = v; };
    auto putf = [&](float v) { put(__float_as_uint(v)); };
    auto put3 = [&](V3 v) { putf(v.x); putf(v.y); putf(v.z); };
    put((uint32_t)P.phase); put((uint32_t)P.j); put((uint32_t)P.slot); put((uint32_t)P.li); put((uint32_t)P.nv);
    put((P.shadow ? 1u : 0u) | (P.cont ? 2u : 0u) | (P.delta ? 4u : 0u));
    putf(P.cx); putf(P.cy); putf(P.r2);
    put3(P.x); put3(P.d); put3(P.n); put3(P.beta); put3(P.f); put3(P.wi); put3(P.wt); put3(P.wl);
}
__device__ __forceinline__ void wf_load(const KBufs& B, size_t N, int c, PathSM& P) {
    const uint32_t* w = B.wf + c;
    int r = 0;
    auto get = [&]() { return w[(size_t)(r++) * N]; };
    auto getf = [&]() { return __uint_as_float(get()); };
    auto get3 = [&]() { const float a = getf(), b = getf(), d = getf(); return v3(a, b, d); };
    P.phase = (int)get(); P.j = (int)get(); P.slot = (int)get(); P.li = (int)get(); P.nv = (int)get();
    const uint32_t fl = get();
    P.shadow = (fl & 1u) != 0; P.cont = (fl & 2u) != 0; P.delta = (fl & 4u) != 0;
    P.cx = getf(); P.cy = getf(); P.r2 = getf();
    P.x = get3(); P.d = get3(); P.n = get3(); P.beta = get3(); P.f = get3(); P.wi = get3(); P.wt = get3(); P.wl = get3();
}

// Appends slot c to a queue with one atomic per wavefront (all lanes call it).
__device__ __forceinline__ void wf_push(uint32_t* q, uint32_t* cnt, bool push, int c) {
    const uint64_t m = __ballot(push);
    if (!m) return;
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((long long)m) - 1;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(cnt, (uint32_t)__popcll(m));
    base = __shfl(base, leader);
    if (push) q[base + (uint32_t)__popcll(m & ((1ull << lane) - 1ull))] = (uint32_t)c;
}

__device__ __forceinline__ void wf_put_ray(const KBufs& B, int c, const RayQ& q) {
    B.wf_ray[2 * (size_t)c] = make_float4(q.o.x, q.o.y, q.o.z, q.tmax);
    B.wf_ray[2 * (size_t)c + 1] = make_float4(q.d.x, q.d.y, q.d.z, q.anyhit ? 1.0f : 0.0f);
}

// Path records of the initialise pass: vertices into the record rows; at the
// end p, f, the pixel and the vertex count (as k_init_eval stores them).
template <int L>
struct InitRec {
    uint32_t *rec, *pix, *key, *ids;
    float *p, *f;
    const float* x;
    int N, c, W, H;
    __device__ __forceinline__ void vertex(int j, uint32_t r) const { rec[(size_t)(j - 1) * N + c] = r; }
    __device__ __forceinline__ void finish(V3 fv, int nv) const {
        for (int j = nv + 1; j <= L - 1; ++j) rec[(size_t)(j - 1) * N + c] = DR_NO_VERTEX;
        p[c] = lum(fv);
        f[c] = fv.x;
        f[(size_t)N + c] = fv.y;
        f[(size_t)2 * N + c] = fv.z;
        pix[c] = pixel_of_wh(W, H, x[c], x[(size_t)N + c]);
        key[c] = (uint32_t)nv;
        ids[c] = (uint32_t)c;
    }
};
template <int L>
__device__ __forceinline__ InitRec<L> init_rec(const KBufs& B, const DevScene& S, int N, int c) {
    return InitRec<L>{B.rec, B.pix_tmp, B.key, B.ids, B.p_tmp, B.f_tmp, B.x, N, c, S.W, S.H};
}

// Initialise pass, path evaluation with the ray-refill state machine
// (persistent): a lane takes the next chain from the work queue, draws x ~ mu
// and follows the chain's path one event at a time; events (shade a hit,
// issue the next ray, or end the path and store p, f, the pixel and the
// record) run once thresh percent of the busy lanes wait for one, otherwise
// the lanes with a ray in flight take one traversal step.  A lane whose ray
// or path ends takes new work while the others keep traversing.  The same
// arithmetic as k_init_eval, so the same state.
template <int L, bool DELTA>
__global__ void __launch_bounds__(256) k_init_sm(KParams P, DevScene S, KBufs B, int thresh) {
    extern __shared__ uint32_t s_stack[];
    uint32_t* stk = s_stack + threadIdx.x;
    const int stride = blockDim.x;
    const int lane = threadIdx.x & 63;
    const uint64_t s0 = B.steps[1];
    const Cam C = load_cam(S);
    Counters ctr = {0, 0, 0};
    RayQ q;
    PathSM ps;
    ps.phase = PH_NEW;
    int c = -1;
    bool tracing = false, drained = false;
    while (true) {
        const bool need = !drained && c < 0;
        const uint64_t nm = __ballot(need);
        if (nm) {
            const int leader = __ffsll((long long)nm) - 1;
            uint32_t base = 0;
            if (lane == leader) base = atomicAdd(B.queue, (uint32_t)__popcll(nm));
            base = __shfl(base, leader);
            if (need) {
                const uint32_t it = base + (uint32_t)__popcll(nm & ((1ull << lane) - 1ull));
                if (it < (uint32_t)P.N) {
                    c = (int)it;
                    regen(P.seed, P.d, P.N, B.x + c, c, s0);
                    ps.phase = PH_NEW;
                } else {
                    drained = true;
                }
            }
        }
        const bool ev = !drained && !tracing;
        const uint64_t em = __ballot(ev), tm = __ballot(tracing);
        if (!em && !tm) break;
        const int nev = __popcll(em), ntr = __popcll(tm);
        if (nev && (!ntr || 100 * nev >= thresh * (nev + ntr))) {
            if (ev) {
                tracing = sm_event<L, DELTA>(S, C, SoaU{B.x + c, P.N}, ps, q, init_rec<L>(B, S, P.N, c), ctr);
                if (!tracing) c = -1;
            }
        } else {
            uint64_t ml, mv;
            ray_masks(q, tracing, ml, mv);
            if (tracing && ray_step(S, q, stk, stride, ctr, ml, mv)) tracing = false;
        }
    }
    if (P.count) {
        wave_add(&B.ctr[C_RAYS], ctr.rays);
        wave_add(&B.ctr[C_NODES], ctr.nodes);
        wave_add(&B.ctr[C_TRIS], ctr.tris);
    }
}

// Initialise pass, first wave: x ~ mu and the camera ray of every chain.
template <int L, bool DELTA>
__global__ void __launch_bounds__(256) k_wf_init_begin(KParams P, DevScene S, KBufs B) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    Counters ctr = {0, 0, 0};
    bool ray = false;
    if (c < P.N) {
        regen(P.seed, P.d, P.N, B.x + c, c, B.steps[1]);
        const Cam C = load_cam(S);
        PathSM ps;
        ps.phase = PH_NEW;
        RayQ q;
        ray = sm_event<L, DELTA>(S, C, SoaU{B.x + c, P.N}, ps, q, init_rec<L>(B, S, P.N, c), ctr);
        if (ray) {
            wf_store(B, P.N, c, ps);
            wf_put_ray(B, c, q);
        }
    }
    wf_push(B.wf_q, &B.wf_cnt[0], ray, c);
    if (P.count) wave_add(&B.ctr[C_RAYS], ctr.rays);
}

// Traversal of the pending rays of queue `in` (length B.wf_cnt[in]):
// persistent lanes take the next slot once enough of the wavefront is idle,
// run trace()'s speculative traversal and store the answer.
static __global__ void __launch_bounds__(256) k_wf_trace(KParams P, DevScene S, KBufs B, int in) {
    extern __shared__ uint32_t s_stack[];
    uint32_t* stk = s_stack + threadIdx.x;
    const int stride = blockDim.x;
    const int lane = threadIdx.x & 63;
    const uint32_t n = B.wf_cnt[in];
    const uint32_t* queue = B.wf_q + (size_t)in * P.N;
    Counters ctr = {0, 0, 0};
    RayQ q;
    q.node = -1;
    q.pleaf = 0;
    int c = -1;
    bool drained = false;
    while (true) {
        const bool idle = q.node < 0 && q.pleaf == 0;
        if (idle && c >= 0) {
            B.wf_hit[c] = q.best;
            B.wf_t[c] = q.bt;
            c = -1;
        }
        const bool want = idle && !drained;
        const uint64_t mw = __ballot(want), mb = __ballot(!idle);
        const int nw = __popcll(mw);
        // refill once three quarters of the wavefront wait (or none is busy)
        if (nw && (mb == 0 || 4 * nw >= 3 * 64)) {
            const int leader = __ffsll((long long)mw) - 1;
            uint32_t base = 0;
            if (lane == leader) base = atomicAdd(&B.wf_cnt[2], (uint32_t)nw);
            base = __shfl(base, leader);
            if (want) {
                const uint32_t it = base + (uint32_t)__popcll(mw & ((1ull << lane) - 1ull));
                if (it < n) {
                    c = (int)queue[it];
                    const float4 a = B.wf_ray[2 * (size_t)c], b = B.wf_ray[2 * (size_t)c + 1];
                    Counters unused = {0, 0, 0};  // rays are counted where they are issued
                    ray_begin(S, q, v3(a.x, a.y, a.z), v3(b.x, b.y, b.z), a.w, b.w != 0.0f, unused);
                } else {
                    drained = true;
                }
            }
        }
        uint64_t ml, mv;
        ray_masks(q, true, ml, mv);
        if (!(ml | mv)) {
            if (__ballot(!drained || c >= 0) == 0) break;
            continue;
        }
        (void)ray_step(S, q, stk, stride, ctr, ml, mv);
    }
    if (P.count) {
        wave_add(&B.ctr[C_NODES], ctr.nodes);
        wave_add(&B.ctr[C_TRIS], ctr.tris);
    }
}

// Events of the initialise pass: every slot of queue `in` consumes its
// answer, shades and issues its next ray into queue `out`, or ends its path.
template <int L, bool DELTA>
__global__ void __launch_bounds__(256) k_wf_init_event(KParams P, DevScene S, KBufs B, int in) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int out = 1 - in;
    Counters ctr = {0, 0, 0};
    bool ray = false;
    int c = -1;
    if (i < (int)B.wf_cnt[in]) {
        c = (int)B.wf_q[(size_t)in * P.N + i];
        PathSM ps;
        wf_load(B, P.N, c, ps);
        RayQ q;
        q.best = B.wf_hit[c];
        q.bt = B.wf_t[c];
        const Cam C = load_cam(S);
        ray = sm_event<L, DELTA>(S, C, SoaU{B.x + c, P.N}, ps, q, init_rec<L>(B, S, P.N, c), ctr);
        if (ray) {
            wf_store(B, P.N, c, ps);
            wf_put_ray(B, c, q);
        }
    }
    wf_push(B.wf_q + (size_t)out * P.N, &B.wf_cnt[out], ray, c);
    if (P.count) wave_add(&B.ctr[C_RAYS], ctr.rays);
}
// Clears a queue's length and the traversal work counter before a wave.
static __global__ void k_wf_reset(KBufs B, int which) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        B.wf_cnt[which] = 0u;
        B.wf_cnt[2] = 0u;
    }
}

// ---------------------------------------------------------------------------
// Host launchers (one instantiation per path length L)
// ---------------------------------------------------------------------------
template <int L>
void launch_init_acc(dim3 g, dim3 b, hipStream_t st, const KParams& P, const DevScene& S, const KBufs& B,
                            int with_score) {
    hipLaunchKernelGGL(k_init_accumulate<L>, g, b, 0, st, P, S, B, with_score);
}
template <int L>
void launch_fused(dim3 g, dim3 b, hipStream_t st, const KParams& P, const DevScene& S, const KBufs& B,
                         uint32_t n, uint32_t grab, bool pair, int sorted, bool delta) {
    const size_t lds = stack_bytes(S, b.x);
    if (delta) {
        if (pair) hipLaunchKernelGGL((k_step_fused_pair<L, true>), g, b, lds, st, P, S, B, n, grab, sorted);
        else hipLaunchKernelGGL((k_step_fused<L, true>), g, b, lds, st, P, S, B, n, grab, sorted);
    } else {
        if (pair) hipLaunchKernelGGL((k_step_fused_pair<L, false>), g, b, lds, st, P, S, B, n, grab, sorted);
        else hipLaunchKernelGGL((k_step_fused<L, false>), g, b, lds, st, P, S, B, n, grab, sorted);
    }
}
template <int L>
void launch_sm(dim3 g, dim3 b, hipStream_t st, const KParams& P, const DevScene& S, const KBufs& B, uint32_t n,
                      int sorted, int ev_pct, int adv_pct, bool delta) {
    if (delta)
        hipLaunchKernelGGL((k_step_sm<L, true>), g, b, stack_bytes(S, b.x), st, P, S, B, n, sorted, ev_pct, adv_pct);
    else
        hipLaunchKernelGGL((k_step_sm<L, false>), g, b, stack_bytes(S, b.x), st, P, S, B, n, sorted, ev_pct, adv_pct);
}
template <int L>
void launch_plain_score(dim3 g, dim3 b, hipStream_t st, const KParams& P, const DevScene& S, const KBufs& B) {
    hipLaunchKernelGGL(k_plain_score<L>, g, b, stack_bytes(S, b.x), st, P, S, B);
}
template <int L>
void launch_eval_sm(dim3 g, dim3 b, hipStream_t st, const DevScene& S, const float* u, int n, float eps,
                           float* fo, float* logp, uint32_t* ro, uint32_t* queue, int thresh) {
    hipLaunchKernelGGL(k_eval_sm<L>, g, b, stack_bytes(S, b.x), st, S, u, n, eps, fo, logp, ro, queue, thresh);
}
template <int L>
void launch_eval(dim3 g, dim3 b, hipStream_t st, const DevScene& S, const float* u, int n, float eps, float* fo,
                        float* logp, float* grad, uint32_t* rs, uint32_t* ro) {
    hipLaunchKernelGGL(k_eval<L>, g, b, stack_bytes(S, b.x), st, S, u, n, eps, fo, logp, grad, rs, ro);
}

template <int L>
void launch_init_sm(dim3 g, dim3 b, hipStream_t st, const KParams& P, const DevScene& S, const KBufs& B, int thresh,
                    bool delta) {
    const size_t lds = stack_bytes(S, b.x);
    if (delta) hipLaunchKernelGGL((k_init_sm<L, true>), g, b, lds, st, P, S, B, thresh);
    else hipLaunchKernelGGL((k_init_sm<L, false>), g, b, lds, st, P, S, B, thresh);
}

// The initialise pass's path evaluation as ray waves: the first wave, then
// 2(L-1) rounds of traversal and events (a path issues at most that many
// rays after its camera ray).  Graph-capturable: a fixed number of launches,
// queue lengths in device memory.
template <int L>
void launch_wf_init(dim3 g, dim3 b, int trace_blocks, hipStream_t st, const KParams& P, const DevScene& S,
                    const KBufs& B, bool delta) {
    const size_t lds = stack_bytes(S, b.x);
    hipLaunchKernelGGL(k_wf_reset, dim3(1), dim3(64), 0, st, B, 0);
    hipLaunchKernelGGL(k_wf_reset, dim3(1), dim3(64), 0, st, B, 1);
    if (delta) hipLaunchKernelGGL((k_wf_init_begin<L, true>), g, b, 0, st, P, S, B);
    else hipLaunchKernelGGL((k_wf_init_begin<L, false>), g, b, 0, st, P, S, B);
    int in = 0;
    for (int r = 0; r < 2 * (L - 1); ++r) {
        hipLaunchKernelGGL(k_wf_trace, dim3(trace_blocks), b, lds, st, P, S, B, in);
        hipLaunchKernelGGL(k_wf_reset, dim3(1), dim3(64), 0, st, B, 1 - in);
        if (delta) hipLaunchKernelGGL((k_wf_init_event<L, true>), g, b, 0, st, P, S, B, in);
        else hipLaunchKernelGGL((k_wf_init_event<L, false>), g, b, 0, st, P, S, B, in);
        in = 1 - in;
    }
}

// Explicit instantiation (X empty) or extern declaration (X = extern) of every
// launcher for one L.
#define DR_LAUNCHERS(X, L)                                                                                          \
    X template void launch_init_acc<L>(dim3, dim3, hipStream_t, const KParams&, const DevScene&, const KBufs&, int); \
    X template void launch_fused<L>(dim3, dim3, hipStream_t, const KParams&, const DevScene&, const KBufs&, uint32_t, \
                                    uint32_t, bool, int, bool);                                                     \
    X template void launch_sm<L>(dim3, dim3, hipStream_t, const KParams&, const DevScene&, const KBufs&, uint32_t,    \
                                 int, int, int, bool);                                                              \
    X template void launch_plain_score<L>(dim3, dim3, hipStream_t, const KParams&, const DevScene&, const KBufs&);   \
    X template void launch_eval_sm<L>(dim3, dim3, hipStream_t, const DevScene&, const float*, int, float, float*,   \
                                      float*, uint32_t*, uint32_t*, int);                                           \
    X template void launch_eval<L>(dim3, dim3, hipStream_t, const DevScene&, const float*, int, float, float*, float*, \
                                   float*, uint32_t*, uint32_t*);                                                  \
    X template void launch_wf_init<L>(dim3, dim3, int, hipStream_t, const KParams&, const DevScene&, \
                                      const KBufs&, bool);                                                          \
    X template void launch_init_sm<L>(dim3, dim3, hipStream_t, const KParams&, const DevScene&, const KBufs&, int, bool);
