// Path evaluation as a per-lane state machine with ray-level refill.
//
// The straight-line evaluator (path_forward) makes a wavefront wait, at every
// ray query, for its longest traversal, and at the end of every path for its
// longest path.  Here each lane owns a resumable ray query (RayQ: the
// traversal state between node visits, stack in LDS) and a path state
// (PathSM).  The wavefront alternates two phases:
//   traverse: every lane with a ray in flight visits one BVH node (its leaves
//             included);
//   event:    every lane whose ray has finished consumes the result and
//             advances its path to the next ray query (shadow ray, then
//             continuation), or finishes the path and takes the next one.
// It runs events once enough lanes wait for one, so traversal keeps most lanes
// busy and the shading code runs with many lanes at once.  Every lane computes
// exactly what path_forward computes for its path, with the same operations
// in the same order, so the results are bit-identical; only the interleaving
// of lanes changes.
#pragma once

#include "dr_device.h"

namespace dr {

// Resumable ray query over (tmin, tmax): closest hit (ties in t to the lower
// input triangle index) or, with anyhit, the first hit found.  The traversal
// is trace()'s speculative one: pleaf is the lane's pending leaf, tested in
// the wavefront's leaf rounds.
struct RayQ {
    V3 o, d;
    RayOrd rs;
    float tmax, bt;
    int best;
    uint32_t best_prim;
    int node, sp, pleaf;  // sp: stack height as an element offset (entries times stride)
    bool anyhit, found;
};

// Starts a query; false when there is no ray (tmax <= tmin), which finishes
// with no hit at once (node -1, nothing pending).
__device__ __forceinline__ bool ray_begin(const DevScene& S, RayQ& q, V3 o, V3 d, float tmax, bool anyhit,
                                          Counters& ctr) {
    q.o = o;
    q.d = d;
    q.tmax = tmax;
    q.bt = tmax;
    q.best = -1;
    q.best_prim = 0xFFFFFFFFu;
    q.node = 0;
    q.sp = 0;
    q.pleaf = 0;
    q.anyhit = anyhit;
    q.found = false;
    if (!(tmax > S.tmin)) {
        q.node = -1;
        return false;
    }
    q.rs = ray_ord(o, d);
    ctr.rays++;
    return true;
}

// Wavefront masks of the lanes whose query holds a pending leaf (ml) or a
// node to visit (mv); taken by every lane of the wavefront, tracing or not.
__device__ __forceinline__ void ray_masks(const RayQ& q, bool tracing, uint64_t& ml, uint64_t& mv) {
    ml = __ballot(tracing && q.pleaf != 0);
    mv = __ballot(tracing && q.node >= 0);
}

// One iteration of trace()'s loop for a lane with a query in flight: a leaf
// round (when enough of the wavefront's busy lanes hold a pending leaf, or
// none can visit a node) or a node visit; the same tests as trace(), so the
// result is the same.  Returns true when the query has finished: then q.best
// is the hit slot (or -1) and, for a closest-hit query, q.bt its distance.
__device__ __forceinline__ bool ray_step(const DevScene& S, RayQ& q, uint32_t* stk, int stride, Counters& ctr,
                                         uint64_t ml, uint64_t mv) {
    const int cap_o = S.stack_cap * stride;
    const int nl = __popcll(ml);
    if (nl && (mv == 0 || 100 * nl >= DR_LEAF_PCT * __popcll(ml | mv))) {
        if (q.pleaf != 0) {
            const bool f = S.leaf_batch == 2
                               ? test_leaf<2>(S, q.pleaf, q.o, q.d, q.tmax, q.anyhit, q.bt, q.best, q.best_prim, ctr)
                               : test_leaf<4>(S, q.pleaf, q.o, q.d, q.tmax, q.anyhit, q.bt, q.best, q.best_prim, ctr);
            q.pleaf = 0;
            if (f) {
                q.found = true;
                q.node = -1;
                q.sp = 0;
            } else if (q.node < 0) {
                pop_entry(q.node, q.pleaf, q.sp, stk, stride);
            }
        }
    } else if (q.node >= 0) {
        ctr.nodes++;
        float tn[4];
        bool hit[4];
        const int4 child = box4_ord(node_rsrc(S), q.node, q.rs, S.tmin, q.bt, hit, tn);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int code = i4(child, k);
            if (hit[k] && code < 0) {
                if (q.pleaf == 0) q.pleaf = code;
                else push_entry(q.sp, stk, stride, cap_o, (uint32_t)code);
            }
        }
        float kt[4];
        int kc[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const bool inner = hit[k] && i4(child, k) >= 0;
            kt[k] = inner ? tn[k] : INFINITY;
            kc[k] = inner ? i4(child, k) : -1;
        }
#define DR_CSWAP(i, j)                                       \
    if (kt[j] < kt[i]) {                                     \
        const float tt_ = kt[i]; kt[i] = kt[j]; kt[j] = tt_; \
        const int cc_ = kc[i]; kc[i] = kc[j]; kc[j] = cc_;   \
    }
        DR_CSWAP(0, 1)
        DR_CSWAP(2, 3)
        DR_CSWAP(0, 2)
        DR_CSWAP(1, 3)
        DR_CSWAP(1, 2)
#undef DR_CSWAP
        if (kc[0] >= 0) {
            if (kc[3] >= 0) push_entry(q.sp, stk, stride, cap_o, (uint32_t)kc[3]);
            if (kc[2] >= 0) push_entry(q.sp, stk, stride, cap_o, (uint32_t)kc[2]);
            if (kc[1] >= 0) push_entry(q.sp, stk, stride, cap_o, (uint32_t)kc[1]);
            q.node = kc[0];
        } else {
            pop_entry(q.node, q.pleaf, q.sp, stk, stride);
        }
    }
    if (q.node >= 0 || q.pleaf != 0) return false;
    if (q.anyhit && !q.found) q.best = -1;
    return true;
}

enum { PH_NEW = 0, PH_CAM = 1, PH_SHADOW = 2, PH_CONT = 3 };

// Path state of one lane between ray queries.
struct PathSM {
    int phase, j, slot, li, nv;  // nv: vertices of the finished path; li: the lobe at a delta vertex
    bool shadow, cont, delta;
    float cx, cy, r2;
    V3 x, d, n, beta, f, wi, wt, wl;
};

// Sets up the vertex at path.slot (the NEE and BSDF candidates of vertex j)
// and issues its first ray.  Returns true when a ray is in flight; false when
// the path is finished (path.phase == PH_NEW afterwards).
template <int L, bool DELTA, class U, class Rec>
__device__ __forceinline__ bool sm_vertex(const DevScene& S, const U& u, PathSM& P, RayQ& q, const Rec& rec,
                                          Counters& ctr);

// Consumes the shadow query's answer (occluded) at vertex j, adds the NEE
// term, then issues the continuation ray or ends the path.
template <int L, class U, class Rec>
__device__ __forceinline__ bool sm_after_shadow(const DevScene& S, const U& u, PathSM& P, RayQ& q, bool occluded,
                                                const Rec& rec, Counters& ctr) {
    const int j = P.j;
    const bool contrib = P.shadow && !occluded;
    rec.vertex(j, ((uint32_t)P.slot << 8) | ((uint32_t)P.li << 1) | (contrib ? 1u : 0u));
    if (contrib) {
        const DevTri T = S.tris[P.slot];
        const Material m = load_material(S, __float_as_uint(T.e1.w));
        const V3 wo = -P.d;
        const V3 fs = bsdf_eval(m, P.n, wo, P.wl);
        const float4 l3 = S.lights[5 * P.li + 3], l4 = S.lights[5 * P.li + 4];
        const float g = P.cx * P.cy / P.r2 * ((float)S.n_lights * l3.w);
        P.f = P.f + mul(mul(P.beta, fs), xyz(l4)) * g;
    }
    if (P.cont) {
        P.phase = PH_CONT;
        ray_begin(S, q, P.x, P.wi, INFINITY, false, ctr);
        return true;
    }
    P.nv = j;
    rec.finish(P.f, j);
    P.phase = PH_NEW;
    return false;
}

template <int L, bool DELTA, class U, class Rec>
__device__ __forceinline__ bool sm_vertex(const DevScene& S, const U& u, PathSM& P, RayQ& q, const Rec& rec,
                                          Counters& ctr) {
    const int j = P.j;
    const DevTri T = S.tris[P.slot];
    const Material m = load_material(S, __float_as_uint(T.e1.w));
    bool front;
    P.n = facing_normal(T, P.d, front);
    P.delta = DELTA && is_delta(m);
    const V3 wo = -P.d;
    float ap;
    const float a = u(4 * j - 2), b = u(4 * j - 1);
    const int nl = S.n_lights;
    P.li = select_light(a, nl, ap);
    const float4 l0 = S.lights[5 * P.li], l1 = S.lights[5 * P.li + 1], l2 = S.lights[5 * P.li + 2],
                 l3 = S.lights[5 * P.li + 3];
    const V3 y = xyz(l0) + xyz(l1) * ap + xyz(l2) * b;
    const V3 w = y - P.x;
    P.r2 = dot(w, w);
    const float r = sqrtf(P.r2);
    P.wl = w * (1.0f / r);
    P.cx = dot(P.n, P.wl);
    P.cy = -dot(xyz(l3), P.wl);
    P.shadow = !P.delta && P.cx > 1e-6f && P.cy > 1e-6f;
    P.wi = v3(0.f, 0.f, 1.f);
    P.wt = v3(0.f, 0.f, 0.f);
    int lobe = -1;
    P.cont = j < L - 1 && !(P.beta.x == 0.0f && P.beta.y == 0.0f && P.beta.z == 0.0f);
    if (P.cont) {
        if (P.delta) delta_sample(m, P.n, front, wo, u(4 * j), P.wi, P.wt, lobe);
        else P.cont = bsdf_sample(m, P.n, wo, u(4 * j), u(4 * j + 1), P.wi, P.wt);
    }
    if (P.delta) P.li = max(lobe, 0);  // recorded in the light field
    if (P.shadow) {
        P.phase = PH_SHADOW;
        if (ray_begin(S, q, P.x, P.wl, (1.0f - 1e-4f) * r, true, ctr)) return true;
    }
    return sm_after_shadow<L>(S, u, P, q, false, rec, ctr);
}

// Event of one lane whose query has finished (or that holds a new path, phase
// PH_NEW with its coordinates in u): advances the path to its next ray query.
// Returns true when a ray is in flight afterwards, false when the path is
// finished (rec.finish has been called and phase is PH_NEW again).  DELTA:
// false compiles the delta-lobe handling out.
template <int L, bool DELTA = true, class U, class Rec>
__device__ __forceinline__ bool sm_event(const DevScene& S, const Cam& C, const U& u, PathSM& P, RayQ& q,
                                         const Rec& rec, Counters& ctr) {
    if (P.phase == PH_NEW) {
        P.f = v3(0.f, 0.f, 0.f);
        if (!point_finite(u, 4 * (L - 1))) {  // as path_forward: f = 0, nothing traced
            P.nv = 0;
            rec.finish(P.f, 0);
            return false;
        }
        P.d = camera_dir(C, u(0), u(1));
        P.j = 1;
        P.phase = PH_CAM;
        ray_begin(S, q, C.eye, P.d, INFINITY, false, ctr);
        return true;
    }
    if (P.phase == PH_CAM) {
        if (q.best < 0) {
            P.nv = 0;
            rec.finish(P.f, 0);
            P.phase = PH_NEW;
            return false;
        }
        P.slot = q.best;
        P.x = C.eye + P.d * q.bt;
        const DevTri T = S.tris[P.slot];
        const Material m = load_material(S, __float_as_uint(T.e1.w));
        if (faces_ray(T, P.d)) P.f = P.f + m.Le;
        P.beta = v3(1.f, 1.f, 1.f);
        return sm_vertex<L, DELTA>(S, u, P, q, rec, ctr);
    }
    if (P.phase == PH_SHADOW) return sm_after_shadow<L>(S, u, P, q, q.best >= 0, rec, ctr);
    // PH_CONT
    if (q.best < 0) {
        P.nv = P.j;
        rec.finish(P.f, P.j);
        P.phase = PH_NEW;
        return false;
    }
    P.beta = mul(P.beta, P.wt);
    P.x = P.x + P.wi * q.bt;
    P.d = P.wi;
    P.slot = q.best;
    ++P.j;
    if (DELTA && P.delta) {  // emission seen through the delta vertex
        const DevTri T = S.tris[P.slot];
        if (faces_ray(T, P.d)) P.f = P.f + mul(P.beta, load_material(S, __float_as_uint(T.e1.w)).Le);
    }
    return sm_vertex<L, DELTA>(S, u, P, q, rec, ctr);
}

}  // namespace dr
