// Device-side building blocks of the Diffusion Restore chain step (gfx950).
//
// Contents: small vector math, the Philox4x32-10 counter generator and the
// stream layout, the scene's device layout, ray/box and ray/triangle tests,
// BVH traversal with a per-lane stack in LDS, the materials, and the forward
// evaluation of the path contribution f(u) that records the discrete choices
// of the taken path.  The reverse-mode adjoint lives in dr_adjoint.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define DR_STACK 64       // traversal stack entries per lane (checked against the tree on the host)
#define DR_NO_VERTEX 0xFFFFFFFFu
#define DR_PI 3.14159265358979323846f

namespace dr {

// ---------------------------------------------------------------------------
// Vector math
// ---------------------------------------------------------------------------
struct V3 {
    float x, y, z;
};
__host__ __device__ __forceinline__ V3 v3(float x, float y, float z) { return V3{x, y, z}; }
__device__ __forceinline__ V3 operator+(V3 a, V3 b) { return v3(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ V3 operator-(V3 a, V3 b) { return v3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ V3 operator-(V3 a) { return v3(-a.x, -a.y, -a.z); }
__device__ __forceinline__ V3 operator*(V3 a, float s) { return v3(a.x * s, a.y * s, a.z * s); }
__device__ __forceinline__ V3 mul(V3 a, V3 b) { return v3(a.x * b.x, a.y * b.y, a.z * b.z); }
__device__ __forceinline__ float dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3 cross(V3 a, V3 b) {
    return v3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ V3 normalize(V3 a) { return a * (1.0f / sqrtf(dot(a, a))); }
__device__ __forceinline__ V3 xyz(float4 a) { return v3(a.x, a.y, a.z); }
__device__ __forceinline__ float lum(V3 c) { return 0.2126f * c.x + 0.7152f * c.y + 0.0722f * c.z; }

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC 2011) and the stream layout:
// counter = (chain, step lo, step hi, tag << 24 | i >> 2), key = seed,
// uniform = top 24 bits of word i & 3 times 2^-24.
// ---------------------------------------------------------------------------
enum { TAG_REGEN = 0, TAG_GAUSS = 1, TAG_HOLD = 2, TAG_PT = 4 };

__device__ __forceinline__ uint4 philox(uint4 c, uint2 k) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k.x += 0x9E3779B9u;
            k.y += 0xBB67AE85u;
        }
        const uint32_t hi0 = __umulhi(0xD2511F53u, c.x), lo0 = 0xD2511F53u * c.x;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z), lo1 = 0xCD9E8D57u * c.z;
        c = make_uint4(hi1 ^ c.y ^ k.x, lo1, hi0 ^ c.w ^ k.y, lo0);
    }
    return c;
}
__device__ __forceinline__ uint4 rng_block(uint64_t seed, uint32_t chain, uint64_t step, uint32_t tag, uint32_t blk) {
    return philox(make_uint4(chain, (uint32_t)step, (uint32_t)(step >> 32), (tag << 24) | blk),
                  make_uint2((uint32_t)seed, (uint32_t)(seed >> 32)));
}
__device__ __forceinline__ float u24(uint32_t w) { return (float)(w >> 8) * (1.0f / 16777216.0f); }

// ---------------------------------------------------------------------------
// Scene layout in HBM
// ---------------------------------------------------------------------------
// 4-wide BVH node (128 B, two cache lines fetched together per visit): the
// boxes of its four children in SOA form (lo/hi per axis for children 0..3),
// then per child the traversal-stack entry and the triangle count.  child >= 0:
// inner node index; child < 0: a leaf, already in its stack form (leaf_code
// below).  count is the leaf's triangle count (0 for an inner node, -1 for an
// empty slot) and is read only by the host; an empty slot's box is NaN, which
// the slab test never reports as hit.
struct alignas(128) DevNode {
    float4 lox, loy, loz, hix, hiy, hiz;
    int4 child, count;
};
// Triangle in leaf order (48 B): v0 | prim id bits, e1 = v1 - v0 | material
// bits, e2 = v2 - v0 | 0.
struct alignas(16) DevTri {
    float4 v0, e1, e2;
};
// Material: m0 = (kind, albedo), m1 = (roughness, f0), m2 = (Le, eta).
// Light: l0 = (p0, 0), l1 = (e1, 0), l2 = (e2, 0), l3 = (unit normal, area), l4 = (Le, 0).
struct DevScene {
    const DevNode* nodes;
    const DevTri* tris;
    const float4* mats;
    const float4* lights;
    const float4* cam;   // camera in device memory (so captured graphs see updates):
                         // eye, cu, cv, cw; ray direction = cw + (2u0-1) cu + (1-2u1) cv
    int n_lights;
    float tmin;
    int W, H;
    int stack_cap;   // traversal stack entries per lane (the tree's exact worst case, <= DR_STACK)
    int n_tris;
    int leaf_batch;  // triangles fetched together per leaf iteration: 2 if no leaf holds more, else 4
    int n_nodes;     // nodes in the array
};

struct Cam {
    V3 eye, cu, cv, cw;
};
__device__ __forceinline__ Cam load_cam(const DevScene& S) {
    Cam c;
    c.eye = v3(S.cam[0].x, S.cam[0].y, S.cam[0].z);
    c.cu = v3(S.cam[1].x, S.cam[1].y, S.cam[1].z);
    c.cv = v3(S.cam[2].x, S.cam[2].y, S.cam[2].z);
    c.cw = v3(S.cam[3].x, S.cam[3].y, S.cam[3].z);
    return c;
}

struct Counters {
    uint32_t rays, nodes, tris;
};

// ---------------------------------------------------------------------------
// Ray queries
// ---------------------------------------------------------------------------
__device__ __forceinline__ float safe_rcp(float d) {
    return 1.0f / (fabsf(d) < 1e-20f ? copysignf(1e-20f, d) : d);
}

// Per-ray constants of the slab test.  A plane at coordinate p along axis a
// is crossed at t = (p - o_a) inv_a, computed as one FMA p * inv_a + c with
// c = -(o_a inv_a).  The rounding of o_a inv_a (and of c) is at most
// |o_a inv_a| 2^-23 in t, so each axis's interval is widened by
// E_a = |o_a inv_a| 2^-22, folded into the constants: the near plane takes
// c - E_a, the far one c + E_a.  With the far distance also widened
// relatively (the final FMA's own rounding), no box a ray truly enters
// within (tmin, tmax) is ever culled.  The reciprocal itself is the
// hardware one (within a few ulp): its error scales an axis's whole
// interval by one factor, which the far distance's relative widening
// (4e-7) also covers.
//
// Which of a box's two planes on an axis the ray meets first depends only on
// the sign of its direction there: the low plane when inv_a >= 0, else the
// high one.  So per ray the near and far plane vectors of each axis sit at
// fixed byte offsets of the SoA node (lo_x at 0, lo_y 16, lo_z 32, hi_x 48,
// hi_y 64, hi_z 80): they are fetched from there, and the test needs no
// per-axis min / max.  For a box with lo <= hi the near distance is then the
// smaller of the two (the FMA is monotone in each operand and the near
// constant is below the far one), so this is the usual slab test, value for
// value.
struct RayOrd {
    V3 inv, cn, cf;       // reciprocal direction; near / far plane constants
    uint32_t noff, foff;  // byte offsets of the near / far planes, one byte per axis
};
__device__ __forceinline__ void plane_consts(float o, float inv, float& cn, float& cf) {
    const float oi = o * inv;
    const float e = fabsf(oi) * 2.384185791015625e-07f;  // 2^-22
    cn = -(oi + e);
    cf = -(oi - e);
}
__device__ __forceinline__ RayOrd ray_ord(V3 o, V3 d) {
    RayOrd r;
    r.inv = v3(safe_rcp(d.x), safe_rcp(d.y), safe_rcp(d.z));
    plane_consts(o.x, r.inv.x, r.cn.x, r.cf.x);
    plane_consts(o.y, r.inv.y, r.cn.y, r.cf.y);
    plane_consts(o.z, r.inv.z, r.cn.z, r.cf.z);
    const bool nx = r.inv.x < 0.0f, ny = r.inv.y < 0.0f, nz = r.inv.z < 0.0f;
    r.noff = (nx ? 48u : 0u) | (ny ? 64u : 16u) << 8 | (nz ? 80u : 32u) << 16;
    r.foff = (nx ? 0u : 48u) | (ny ? 16u : 64u) << 8 | (nz ? 32u : 80u) << 16;
    return r;
}

// NaN-propagating minimum / maximum: a NaN box (an empty child slot) never
// passes, and no operand needs canonicalising.  Every other operand is finite
// (|inv| <= 1e20, finite planes), where they equal fminf / fmaxf except on the
// sign of a zero, which cannot change a decision (tnear >= tmin > 0).
__device__ __forceinline__ float mn(float a, float b) { return __builtin_elementwise_minimum(a, b); }
__device__ __forceinline__ float mx(float a, float b) { return __builtin_elementwise_maximum(a, b); }
// Component q of a vector (q is a compile-time constant after unrolling).
__device__ __forceinline__ float f4(const float4& v, int q) { return q == 0 ? v.x : (q == 1 ? v.y : (q == 2 ? v.z : v.w)); }
__device__ __forceinline__ int i4(const int4& v, int q) { return q == 0 ? v.x : (q == 1 ? v.y : (q == 2 ? v.z : v.w)); }
// Buffer resources over the scene's node and triangle arrays (raw, byte
// offsets, range checked against the array's size: below 2^31 bytes for the
// at most 2^24 - 1 triangles a scene holds).  A fetch through one needs a
// 32-bit offset instead of a 64-bit address.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t node_rsrc(const DevScene& S) {
    return __builtin_amdgcn_make_buffer_rsrc((void*)S.nodes, (short)0, S.n_nodes * (int)sizeof(DevNode), 0x00020000);
}
__device__ __forceinline__ __amdgpu_buffer_rsrc_t tri_rsrc(const DevScene& S) {
    return __builtin_amdgcn_make_buffer_rsrc((void*)S.tris, (short)0, S.n_tris * (int)sizeof(DevTri), 0x00020000);
}
// 16 bytes at byte offset off of a buffer.
__device__ __forceinline__ float4 ld16(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    typedef uint32_t u4 __attribute__((ext_vector_type(4)));
    const u4 v = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
    return make_float4(__uint_as_float(v.x), __uint_as_float(v.y), __uint_as_float(v.z), __uint_as_float(v.w));
}
// The four child boxes of node `node` against one ray: hit[q] and tnear[q];
// returns the children's stack entries.  Seven 16-byte fetches through the
// buffer resource rn (32-bit offsets: the per-lane plane offsets come from the
// ray, the axis offsets fold into the instructions).  The top levels stay in
// the L1 and L2 (an LDS copy of them measured no faster with this form).
__device__ __forceinline__ int4 box4_ord(__amdgpu_buffer_rsrc_t rn, int node, const RayOrd& r, float tmin, float tmax,
                                         bool hit[4], float tn[4]) {
    const uint32_t b = (uint32_t)node << 7;
    const float4 nx = ld16(rn, b + (r.noff & 0xffu)), fx = ld16(rn, b + (r.foff & 0xffu));
    const float4 ny = ld16(rn, b + ((r.noff >> 8) & 0xffu)), fy = ld16(rn, b + ((r.foff >> 8) & 0xffu));
    const float4 nz = ld16(rn, b + (r.noff >> 16)), fz = ld16(rn, b + (r.foff >> 16));
    const float4 cf = ld16(rn, b + 96u);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const float tnx = fmaf(f4(nx, q), r.inv.x, r.cn.x), tfx = fmaf(f4(fx, q), r.inv.x, r.cf.x);
        const float tny = fmaf(f4(ny, q), r.inv.y, r.cn.y), tfy = fmaf(f4(fy, q), r.inv.y, r.cf.y);
        const float tnz = fmaf(f4(nz, q), r.inv.z, r.cn.z), tfz = fmaf(f4(fz, q), r.inv.z, r.cf.z);
        const float t0 = mx(mx(tnx, tny), mx(tnz, tmin));
        const float t1 = mn(mn(tfx, tfy), tfz) * 1.0000004f;
        tn[q] = t0;
        hit[q] = t0 <= mn(t1, tmax);
    }
    return make_int4(__float_as_int(cf.x), __float_as_int(cf.y), __float_as_int(cf.z), __float_as_int(cf.w));
}

// Moller-Trumbore, two-sided; t in (tmin, inf) before the caller's range test.
// The reciprocal of the determinant is the hardware one (1 ulp).  Evaluated
// without early exits (a wavefront's lanes diverge on them anyway); the
// conditions keep the branching form's treatment of NaN (a NaN barycentric
// does not reject), so the answers are the same.
__device__ __forceinline__ bool tri_test(const DevTri& T, V3 o, V3 d, float tmin, float& t) {
    const V3 e1 = xyz(T.e1), e2 = xyz(T.e2);
    const V3 pv = cross(d, e2);
    const float det = dot(e1, pv);
    const float inv = __builtin_amdgcn_rcpf(det);
    const V3 tv = o - xyz(T.v0);
    const float b1 = dot(tv, pv) * inv;
    const V3 qv = cross(tv, e1);
    const float b2 = dot(d, qv) * inv;
    t = dot(e2, qv) * inv;
    return (det != 0.0f) & !(b1 < 0.0f || b1 > 1.0f) & !(b2 < 0.0f || b1 + b2 > 1.0f) & (t > tmin);
}

// Leaf entries share the traversal stack with inner nodes: a leaf of cnt
// triangles from slot first is stored as -1 - (first << 5 | cnt) (cnt <= 16,
// first < 2^24), inner nodes as their index (>= 0).  The scene upload writes
// leaves in this form into the nodes' child fields.
__host__ __device__ __forceinline__ int leaf_code(int first, int cnt) { return -1 - ((first << 5) | cnt); }

// Triangle tests of one leaf; returns true when an any-hit query has found
// its hit (slot in best).
template <int BATCH>
__device__ __forceinline__ bool test_leaf(const DevScene& S, int code, V3 o, V3 d, float tmax, bool anyhit, float& bt,
                                          int& best, uint32_t& best_prim, Counters& ctr) {
    const int v = -1 - code;
    const int first = v >> 5, cnt = v & 31;
    const __amdgpu_buffer_rsrc_t rt = tri_rsrc(S);
    for (int k0 = first; k0 < first + cnt; k0 += BATCH) {
        DevTri T[BATCH];
#pragma unroll
        for (int e = 0; e < BATCH; ++e) {
            const uint32_t off = (uint32_t)min(k0 + e, S.n_tris - 1) * (uint32_t)sizeof(DevTri);
            T[e].v0 = ld16(rt, off);
            T[e].e1 = ld16(rt, off + 16u);
            T[e].e2 = ld16(rt, off + 32u);
        }
#pragma unroll
        for (int e = 0; e < BATCH; ++e) {
            if (k0 + e >= first + cnt) break;
            ctr.tris++;
            float t;
            if (tri_test(T[e], o, d, S.tmin, t) && t <= bt) {
                const uint32_t prim = __float_as_uint(T[e].v0.w);
                if (anyhit && t < tmax) {
                    best = k0 + e;
                    return true;
                }
                if (t < bt || (t == bt && prim < best_prim)) {
                    bt = t;
                    best = k0 + e;
                    best_prim = prim;
                }
            }
        }
    }
    return false;
}

// Next work from the stack: an inner node to visit, or a leaf to hold as the
// pending one (if the lane already holds one, the leaf stays on the stack
// and the lane waits for the next leaf round).
// so is the stack height as an element offset (entries times stride), so a
// push or pop is an add rather than a multiply.
__device__ __forceinline__ void pop_entry(int& node, int& pleaf, int& so, const uint32_t* stk, int stride) {
    node = -1;
    if (so == 0) return;
    so -= stride;
    const int e = (int)stk[so];
    if (e >= 0) node = e;
    else if (pleaf == 0) pleaf = e;
    else so += stride;
}
// Push v if the stack (capacity cap_o as an element offset) has room.
__device__ __forceinline__ void push_entry(int& so, uint32_t* stk, int stride, int cap_o, uint32_t v) {
    if (so < cap_o) {
        stk[so] = v;
        so += stride;
    }
}

#define DR_LEAF_PCT 40  // leaf round once this share of the wavefront's busy lanes hold a pending leaf

// One ray query over (tmin, tmax): the closest hit (ties in t go to the lower
// input triangle index) or, with anyhit, the first hit found.  The answer
// (res_a, t_a) is the triangle slot (leaf order) or -1 and the hit distance
// (tmax if none); tmax <= tmin means "no ray" and answers -1 at once (used
// by paired lanes that have nothing to trace).  stk is this lane's LDS stack,
// entries at stk[k * stride].
//
// Leaf tests are postponed (speculative traversal): a lane that reaches a leaf
// holds it as pending and keeps visiting nodes (further leaves go to the
// stack), and the wavefront tests triangles only once enough of its lanes hold
// a leaf, or none can visit a node.  Node visits and leaf tests then each run
// with many lanes active instead of a leaf round whenever any one lane meets a
// leaf.  The closest hit and the tie rule do not depend on the order of the
// tests (a postponed leaf only means fewer boxes culled meanwhile), and an
// any-hit query only reports whether a hit exists.
//
// TWO: each lane runs a second query from the same origin (closest hit along
// db over (tmin, inf), if b_on; answer in res_b, t_b) right after its first
// ends, in the same wavefront loop and on the same (then empty) stack.  The
// wavefront then iterates as long as its longest per-lane sum of the two
// traversals rather than the sum of the two longest, and the lanes done with
// their first query keep working while others finish theirs.  Each query's
// answer is the one it has alone.
template <bool TWO>
__device__ __forceinline__ void trace_core(const DevScene& S, V3 o, V3 d, float tmax, bool anyhit, bool b_on, V3 db,
                                           int& res_a, float& t_a, int& res_b, float& t_b,
                                           uint32_t* stk, int stride, Counters& ctr) {
    float bt, qmax = tmax;
    int best, so = 0, node = -1, pleaf = 0;
    uint32_t best_prim;
    bool found = false, qany = anyhit;
    V3 qd = d;
    RayOrd rs;
    const __amdgpu_buffer_rsrc_t rn = node_rsrc(S);
    // set up one query at the root (node stays -1 when there is no query)
    auto start = [&](V3 dd, float mx, bool any) {
        qd = dd;
        qmax = mx;
        qany = any;
        bt = mx;
        best = -1;
        best_prim = 0xFFFFFFFFu;
        found = false;
        so = 0;
        pleaf = 0;
        node = -1;
        if (!(mx > S.tmin)) return;
        ctr.rays++;
        rs = ray_ord(o, dd);
        node = 0;
    };
    start(d, tmax, anyhit);
    int phase = 0;
    const int cap_o = S.stack_cap * stride;
    while (true) {
        if (TWO && phase == 0 && node < 0 && pleaf == 0) {
            // first query over (its stack is empty): keep its answer, start the second
            res_a = qany ? (found ? best : -1) : best;
            t_a = bt;
            phase = 1;
            start(db, b_on ? INFINITY : -1.0f, false);
        }
        const bool has_leaf = pleaf != 0, can_visit = node >= 0;
        const uint64_t ml = __ballot(has_leaf), mv = __ballot(can_visit);
        if (!(ml | mv)) break;
        const int nl = __popcll(ml);
        if (nl && (mv == 0 || 100 * nl >= DR_LEAF_PCT * __popcll(ml | mv))) {
            if (has_leaf) {
                const bool f = S.leaf_batch == 2 ? test_leaf<2>(S, pleaf, o, qd, qmax, qany, bt, best, best_prim, ctr)
                                                 : test_leaf<4>(S, pleaf, o, qd, qmax, qany, bt, best, best_prim, ctr);
                pleaf = 0;
                if (f) {
                    found = true;
                    node = -1;
                    so = 0;
                } else if (node < 0) {
                    pop_entry(node, pleaf, so, stk, stride);
                }
            }
        } else if (can_visit) {
            ctr.nodes++;
            float tn[4];
            bool hit[4];
            const int4 child = box4_ord(rn, node, rs, S.tmin, bt, hit, tn);
            // hit leaves: the first becomes the pending leaf if the lane holds none, the others wait on the stack
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int code = i4(child, q);
                if (hit[q] && code < 0) {
                    if (pleaf == 0) pleaf = code;
                    else push_entry(so, stk, stride, cap_o, (uint32_t)code);
                }
            }
            // hit inner children: visit the nearest next, push the others
            // far-first (a fixed sorting network keeps every index static)
            float kt[4];
            int kc[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const bool inner = hit[q] && i4(child, q) >= 0;
                kt[q] = inner ? tn[q] : INFINITY;
                kc[q] = inner ? i4(child, q) : -1;
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
                if (kc[3] >= 0) push_entry(so, stk, stride, cap_o, (uint32_t)kc[3]);
                if (kc[2] >= 0) push_entry(so, stk, stride, cap_o, (uint32_t)kc[2]);
                if (kc[1] >= 0) push_entry(so, stk, stride, cap_o, (uint32_t)kc[1]);
                node = kc[0];
            } else {
                pop_entry(node, pleaf, so, stk, stride);
            }
        }
    }
    if (TWO) {
        res_b = best;
        t_b = bt;
    } else {
        res_a = qany ? (found ? best : -1) : best;
        t_a = bt;
    }
}

// One query (trace_core without a second): returns the slot or -1, t_hit the distance.
__device__ int trace(const DevScene& S, V3 o, V3 d, float tmax, bool anyhit, float& t_hit, uint32_t* stk, int stride,
                     Counters& ctr) {
    int ra, rb;
    float tb;
    trace_core<false>(S, o, d, tmax, anyhit, false, d, ra, t_hit, rb, tb, stk, stride, ctr);
    return ra;
}

// ---------------------------------------------------------------------------
// Surfaces
// ---------------------------------------------------------------------------
// Unit geometric normal of a triangle, flipped to face the incoming direction.
__device__ __forceinline__ V3 facing_normal(const DevTri& T, V3 din) {
    const V3 ng = normalize(cross(xyz(T.e1), xyz(T.e2)));
    return dot(ng, din) > 0.0f ? -ng : ng;
}
// Same; front: the incoming direction arrives on the e1 x e2 side (outside
// a dielectric).
__device__ __forceinline__ V3 facing_normal(const DevTri& T, V3 din, bool& front) {
    const V3 ng = normalize(cross(xyz(T.e1), xyz(T.e2)));
    front = !(dot(ng, din) > 0.0f);
    return front ? ng : -ng;
}
// True when a ray along d meets the triangle's emitting (e1 x e2) side.
__device__ __forceinline__ bool faces_ray(const DevTri& T, V3 d) {
    return dot(cross(xyz(T.e1), xyz(T.e2)), d) < 0.0f;
}

// Orthonormal basis around a unit normal (Duff et al., JCGT 2017).
__device__ __forceinline__ void onb(V3 n, V3& t, V3& b) {
    const float sign = copysignf(1.0f, n.z);
    const float a = -1.0f / (sign + n.z);
    const float bb = n.x * n.y * a;
    t = v3(1.0f + sign * n.x * n.x * a, sign * bb, -sign * n.x);
    b = v3(bb, sign + n.y * n.y * a, -n.y);
}

// Separable Smith masking for GGX: G1(c) = 2 / (1 + sqrt(1 + a2 (1 - c^2)/c^2)).
__device__ __forceinline__ float smith_g1(float c, float a2) {
    const float c2 = c * c;
    return 2.0f / (1.0f + sqrtf(1.0f + a2 * (1.0f - c2) / c2));
}

enum { MAT_LAMBERT = 0, MAT_GGX = 1, MAT_MIRROR = 2, MAT_GLASS = 3 };
struct Material {
    int kind;
    V3 albedo, f0, Le;
    float a2;   // GGX alpha^2
    float eta;  // dielectric: index of refraction inside (opposite e1 x e2)
};
// Smooth conductor and smooth dielectric: BSDFs with a delta lobe.
__device__ __forceinline__ bool is_delta(const Material& m) { return m.kind >= MAT_MIRROR; }
__device__ __forceinline__ Material load_material(const DevScene& S, uint32_t id) {
    const float4 m0 = S.mats[3 * id], m1 = S.mats[3 * id + 1], m2 = S.mats[3 * id + 2];
    Material m;
    m.kind = (int)m0.x;
    m.albedo = v3(m0.y, m0.z, m0.w);
    m.a2 = m1.x * m1.x;
    m.f0 = v3(m1.y, m1.z, m1.w);
    m.Le = xyz(m2);
    m.eta = m2.w;
    return m;
}

// f_s(wo, wi) for n.wo > 0, n.wi > 0.
__device__ __forceinline__ V3 bsdf_eval(const Material& m, V3 n, V3 wo, V3 wi) {
    if (m.kind == 0) return m.albedo * (1.0f / DR_PI);
    const float co = dot(n, wo), ci = dot(n, wi);
    const V3 h = normalize(wo + wi);
    const float ch = dot(n, h);
    const float den = ch * ch * (m.a2 - 1.0f) + 1.0f;
    const float D = m.a2 / (DR_PI * den * den);
    const float G = smith_g1(co, m.a2) * smith_g1(ci, m.a2);
    const float oh = dot(wi, h);
    const float om = 1.0f - oh;
    const float f5 = om * om * om * om * om;
    const float k = D * G / (4.0f * co * ci);
    return v3(k * (m.f0.x + (1.0f - m.f0.x) * f5), k * (m.f0.y + (1.0f - m.f0.y) * f5),
              k * (m.f0.z + (1.0f - m.f0.z) * f5));
}

// Sample wi from the 2-D block (u, v); weight = f_s cos / pdf.  False when the
// sample leaves the upper hemisphere (the path ends).
__device__ __forceinline__ bool bsdf_sample(const Material& m, V3 n, V3 wo, float u, float v, V3& wi, V3& weight) {
    V3 t, b;
    onb(n, t, b);
    float sp, cp;
    __sincosf(2.0f * DR_PI * v, &sp, &cp);
    if (m.kind == 0) {
        const float r = sqrtf(u), lz = sqrtf(1.0f - u);
        wi = t * (r * cp) + b * (r * sp) + n * lz;
        weight = m.albedo;
        return true;
    }
    const float den = (1.0f - u) + m.a2 * u;
    const float ch = sqrtf((1.0f - u) / den);
    const float sh = sqrtf(m.a2 * u / den);
    const V3 h = t * (sh * cp) + b * (sh * sp) + n * ch;
    const float oh = dot(wo, h);
    if (oh <= 0.0f) return false;
    wi = h * (2.0f * oh) - wo;
    const float ci = dot(n, wi);
    if (ci <= 0.0f) return false;
    const float co = dot(n, wo);
    const float g = smith_g1(co, m.a2) * smith_g1(ci, m.a2) * oh / (co * ch);
    const float om = 1.0f - oh;
    const float f5 = om * om * om * om * om;
    weight = v3(g * (m.f0.x + (1.0f - m.f0.x) * f5), g * (m.f0.y + (1.0f - m.f0.y) * f5),
                g * (m.f0.z + (1.0f - m.f0.z) * f5));
    return true;
}

// Fresnel reflectance of a smooth dielectric for unpolarised light: the mean
// of the squared s and p amplitude ratios.  ci: incident cosine (>= 0); etap:
// n_transmitted / n_incident.  1 under total internal reflection; ct: the
// transmitted cosine.
__device__ __forceinline__ float fresnel_dielectric(float ci, float etap, float& ct) {
    const float s2 = (1.0f - ci * ci) / (etap * etap);
    if (s2 >= 1.0f) {
        ct = 0.0f;
        return 1.0f;
    }
    ct = sqrtf(1.0f - s2);
    const float rs = (ci - etap * ct) / (ci + etap * ct);
    const float rp = (etap * ci - ct) / (etap * ci + ct);
    return 0.5f * (rs * rs + rp * rp);
}

// Relative index of refraction across a dielectric's surface, seen from the
// incident side.
__device__ __forceinline__ float rel_eta(const Material& m, bool front) { return front ? m.eta : 1.0f / m.eta; }

// Delta lobe of a smooth conductor (mirror direction, weight Schlick's F at
// the incidence cosine) or smooth dielectric (reflection when u < F, weight
// 1; else Snell refraction, weight 1/etap^2: radiance scales with the
// squared index).  n faces wo.  Lobe 0 reflection, 1 refraction; with
// lobe >= 0 on entry the choice is taken as given (replay of a recorded
// path) instead of drawn from u.
__device__ __forceinline__ void delta_sample(const Material& m, V3 n, bool front, V3 wo, float u, V3& wi, V3& weight,
                                             int& lobe) {
    const float ci = dot(n, wo);
    if (m.kind == MAT_MIRROR) {
        wi = n * (2.0f * ci) - wo;
        const float om = 1.0f - ci;
        const float f5 = om * om * om * om * om;
        weight = v3(m.f0.x + (1.0f - m.f0.x) * f5, m.f0.y + (1.0f - m.f0.y) * f5, m.f0.z + (1.0f - m.f0.z) * f5);
        lobe = 0;
        return;
    }
    const float etap = rel_eta(m, front);
    float ct;
    const float F = fresnel_dielectric(ci, etap, ct);
    if (lobe < 0) lobe = u < F ? 0 : 1;
    if (lobe == 0) {
        wi = n * (2.0f * ci) - wo;
        weight = v3(1.f, 1.f, 1.f);
    } else {
        const float ie = 1.0f / etap;
        wi = wo * (-ie) + n * (ci * ie - ct);
        const float w = ie * ie;
        weight = v3(w, w, w);
    }
}

// Light selection from the first coordinate of the light block, in FP32.
__device__ __forceinline__ int select_light(float a, int nl, float& ap) {
    const float sel = a * (float)nl;
    int li = (int)floorf(sel);
    li = min(max(li, 0), nl - 1);
    ap = a * (float)nl - (float)li;
    return li;
}

// Camera ray direction for the film block.
__device__ __forceinline__ V3 camera_dir(const Cam& C, float u0, float u1) {
    return normalize(C.cw + C.cu * (2.0f * u0 - 1.0f) + C.cv * (1.0f - 2.0f * u1));
}

// Pixel of the film block, in FP32: px = min(floor(u0 W), W-1), row 0 at top.
__device__ __forceinline__ uint32_t pixel_of_wh(int W, int H, float u0, float u1) {
    int px = (int)floorf(u0 * (float)W), py = (int)floorf(u1 * (float)H);
    px = min(max(px, 0), W - 1);
    py = min(max(py, 0), H - 1);
    return (uint32_t)(py * W + px);
}
__device__ __forceinline__ uint32_t pixel_of(const DevScene& S, float u0, float u1) {
    return pixel_of_wh(S.W, S.H, u0, u1);
}

// ---------------------------------------------------------------------------
// Forward path contribution with next-event estimation.
// U is an accessor: float operator()(int i) returns coordinate i of u.
// rec (nullable): per vertex j = 1..L-1, rec[(j-1) * rs] = slot << 8 |
// light << 1 | contributed (at a delta vertex: lobe << 1), or DR_NO_VERTEX.
// Emission counts at the primary hit and at a vertex reached from a delta
// vertex (next-event estimation cannot sample a light through a delta
// lobe); a delta vertex takes no next-event estimate.
//
// DELTA: false compiles the delta-lobe handling out, for scenes without
// smooth conductors or dielectrics.
//
// PAIR: two adjacent lanes evaluate the same path.  Both run the same control
// flow on the same data (so they take the same branches and hold the same
// values); at each vertex the even lane traces the continuation ray and the
// odd lane the shadow ray, concurrently, and they swap the results with a
// lane shuffle.  Without PAIR one lane traces both rays in turn.
// ---------------------------------------------------------------------------
// Value held by the adjacent lane (lane ^ 1): a DPP quad permutation
// [1,0,3,2], read straight from the partner's register.
__device__ __forceinline__ int swap_pair(int v) { return __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false); }
__device__ __forceinline__ float swap_pair(float v) { return __int_as_float(swap_pair(__float_as_int(v))); }

// The shadow ray (any hit, up to smax) and the continuation ray (closest
// hit) of a vertex.
template <bool PAIR>
__device__ __forceinline__ void trace_vertex_rays(const DevScene& S, V3 x, bool shadow, V3 wl, float smax, bool cont,
                                                  V3 wi, bool& occluded, int& nslot, float& tn, uint32_t* stk,
                                                  int stride, Counters& ctr) {
    if (PAIR) {
        const bool odd = (threadIdx.x & 1) != 0;
        float tt;
        const int r = trace(S, x, odd ? wl : wi, odd ? (shadow ? smax : -1.0f) : (cont ? INFINITY : -1.0f), odd, tt,
                            stk, stride, ctr);
        const int ro = swap_pair(r);
        const float to = swap_pair(tt);
        occluded = shadow && (odd ? r : ro) >= 0;
        nslot = cont ? (odd ? ro : r) : -1;
        tn = odd ? to : tt;
    } else {
        // the shadow query, then the continuation, back to back in one loop
        float ts;
        int ra, rb;
        trace_core<true>(S, x, wl, shadow ? smax : -1.0f, true, cont, wi, ra, ts, rb, tn, stk, stride, ctr);
        occluded = shadow && ra >= 0;
        nslot = cont ? rb : -1;
    }
}

// True when every coordinate of the point is finite (accessors over generated
// coordinates skip the check).
template <class U>
__device__ __forceinline__ bool point_finite(const U& u, int d) {
    if constexpr (U::kChecked) {
        bool ok = true;
        for (int i = 0; i < d; ++i) ok &= isfinite(u(i));
        return ok;
    } else {
        return true;
    }
}

template <bool PAIR, bool DELTA = true, class U>
__device__ V3 path_forward(const DevScene& S, int L, const U& u, uint32_t* rec, int rs, uint32_t* stk, int stride,
                           Counters& ctr, int* nverts = nullptr) {
    V3 f = v3(0.f, 0.f, 0.f);
    // a point with a non-finite coordinate (a state that left the torus) has
    // f = 0: its tour is killed and regenerates
    if (!point_finite(u, 4 * (L - 1))) {
        if (nverts) *nverts = 0;
        if (rec)
            for (int j = 1; j <= L - 1; ++j) rec[(j - 1) * rs] = DR_NO_VERTEX;
        return f;
    }
    const Cam C = load_cam(S);
    V3 d = camera_dir(C, u(0), u(1));
    float t;
    int slot;
    if (PAIR) {
        const bool odd = (threadIdx.x & 1) != 0;
        const int r = trace(S, C.eye, d, odd ? -1.0f : INFINITY, false, t, stk, stride, ctr);
        slot = swap_pair(r);
        const float to = swap_pair(t);
        if (!odd) slot = r;
        else t = to;
    } else {
        slot = trace(S, C.eye, d, INFINITY, false, t, stk, stride, ctr);
    }
    int j = 1;
    if (slot >= 0) {
        V3 x = C.eye + d * t;
        DevTri T = S.tris[slot];
        {
            const Material m = load_material(S, __float_as_uint(T.e1.w));
            if (faces_ray(T, d)) f = f + m.Le;
        }
        V3 beta = v3(1.f, 1.f, 1.f);
        const int nl = S.n_lights;
        for (; j <= L - 1; ++j) {
            const Material m = load_material(S, __float_as_uint(T.e1.w));
            bool front;
            const V3 n = facing_normal(T, d, front);
            const V3 wo = -d;
            const bool delta = DELTA && is_delta(m);
            // next-event estimation candidate
            float ap;
            const float a = u(4 * j - 2), b = u(4 * j - 1);
            const int li = select_light(a, nl, ap);
            const float4 l0 = S.lights[5 * li], l1 = S.lights[5 * li + 1], l2 = S.lights[5 * li + 2],
                         l3 = S.lights[5 * li + 3], l4 = S.lights[5 * li + 4];
            const V3 y = xyz(l0) + xyz(l1) * ap + xyz(l2) * b;
            const V3 w = y - x;
            const float r2 = dot(w, w);
            const float r = sqrtf(r2);
            const V3 wl = w * (1.0f / r);
            const float cx = dot(n, wl);
            const float cy = -dot(xyz(l3), wl);
            // both cosines must clear 1e-6 (a vertex in the light's own plane
            // has cosines that are rounding noise around zero)
            const bool shadow = !delta && cx > 1e-6f && cy > 1e-6f;
            // continuation candidate: BSDF sample at vertex j
            V3 wi = v3(0.f, 0.f, 1.f), wt = v3(0.f, 0.f, 0.f);
            int lobe = -1;
            bool cont = j < L - 1 && !(beta.x == 0.0f && beta.y == 0.0f && beta.z == 0.0f);
            if (cont) {
                if (delta) delta_sample(m, n, front, wo, u(4 * j), wi, wt, lobe);
                else cont = bsdf_sample(m, n, wo, u(4 * j), u(4 * j + 1), wi, wt);
            }
            bool occluded;
            int ns;
            float tn;
            trace_vertex_rays<PAIR>(S, x, shadow, wl, (1.0f - 1e-4f) * r, cont, wi, occluded, ns, tn, stk, stride, ctr);
            const bool contrib = shadow && !occluded;
            if (rec)
                rec[(j - 1) * rs] = ((uint32_t)slot << 8) | ((uint32_t)(delta ? max(lobe, 0) : li) << 1) |
                                    (contrib ? 1u : 0u);
            if (contrib) {
                const V3 fs = bsdf_eval(m, n, wo, wl);
                const float g = cx * cy / r2 * ((float)nl * l3.w);
                f = f + mul(mul(beta, fs), xyz(l4)) * g;
            }
            if (ns < 0) break;
            beta = mul(beta, wt);
            x = x + wi * tn;
            d = wi;
            slot = ns;
            T = S.tris[slot];
            if (delta && faces_ray(T, d)) f = f + mul(beta, load_material(S, __float_as_uint(T.e1.w)).Le);
        }
        ++j;
    }
    if (nverts) *nverts = j - 1;
    if (rec)
        for (; j <= L - 1; ++j) rec[(j - 1) * rs] = DR_NO_VERTEX;
    return f;
}

// Coordinate accessors
struct SoaU {  // chain state: coordinate i at p[i * stride]
    static constexpr bool kChecked = true;
    const float* p;
    int stride;
    __device__ __forceinline__ float operator()(int i) const { return p[(size_t)i * stride]; }
};

}  // namespace dr
