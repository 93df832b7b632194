// Reverse-mode adjoint of the path contribution: score = grad_u ln(p + eps)
// for the Langevin drift of Sec. 5 (Eq. langevin-drift; Alg. 5.1 computes
// grad ln p at the current state).
//
// The forward pass (path_forward) records the discrete choices of the taken
// path: the triangle of every vertex, the light picked for next-event
// estimation and whether it contributed.  With those held fixed, f is a
// smooth function of u, and this file re-traces the path without any ray
// query (vertex positions come from the recorded triangles' planes) and
// propagates adjoints backwards through the camera, vertex, BSDF and
// geometry terms.  Vertex states (position, incoming direction, throughput)
// are kept in registers for segments of up to DR_SEG vertices; longer paths
// keep one checkpoint per segment and recompute each segment's vertices when
// its turn in the reverse sweep comes, instead of storing all of them.
#pragma once

#include "dr_device.h"

#define DR_SEG 8

namespace dr {

struct VState {
    V3 x, din, beta;
};
struct Adj {
    V3 gx, gd, gb;
};

__device__ __forceinline__ uint32_t rec_slot(uint32_t r) { return r >> 8; }
__device__ __forceinline__ int rec_light(uint32_t r) { return (int)((r >> 1) & 0x7Fu); }
__device__ __forceinline__ bool rec_contrib(uint32_t r) { return (r & 1u) != 0; }

// Division and square root in the adjoint: the hardware reciprocal and
// square root (within 1 ulp), the quotient as a product with the reciprocal.  The adjoint divides often, and these roundings sit far below
// the score's own conditioning.  (Directions and decisions are recomputed
// with the forward path's own functions, so they stay bit-identical.)
__device__ __forceinline__ float arcp(float b) { return __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ float adiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ float asqrt(float a) { return __builtin_amdgcn_sqrtf(a); }

// d G1/dc / G1 for the separable Smith term.
__device__ __forceinline__ float smith_dlog(float c, float a2) {
    const float c2 = c * c;
    const float lam = asqrt(1.0f + adiv(a2 * (1.0f - c2), c2));
    return adiv(a2, c2 * c * lam * (1.0f + lam));
}

// Position of the hit on triangle T along (o, d): plane distance.
__device__ __forceinline__ float plane_t(const DevTri& T, V3 ng, V3 o, V3 d) {
    return adiv(dot(ng, xyz(T.v0) - o), dot(ng, d));
}

// Camera vertex (vertex 1) state.
__device__ __forceinline__ VState camera_state(const Cam& C, float u0, float u1, const DevTri& T1) {
    const V3 d = camera_dir(C, u0, u1);
    const V3 ng = normalize(cross(xyz(T1.e1), xyz(T1.e2)));
    VState s;
    s.x = C.eye + d * plane_t(T1, ng, C.eye, d);
    s.din = d;
    s.beta = v3(1.f, 1.f, 1.f);
    return s;
}

// State of vertex j+1 from vertex j (BSDF sample with block (u, v), or the
// recorded lobe of a delta vertex, then the recorded next triangle Tn).  The
// sample is known to be valid.
template <bool DELTA>
__device__ __forceinline__ VState advance(const DevScene& S, const VState& s, const DevTri& T, const DevTri& Tn, float u,
                                          float v, uint32_t recj) {
    const Material m = load_material(S, __float_as_uint(T.e1.w));
    bool front;
    const V3 n = facing_normal(T, s.din, front);
    V3 wi, wt;
    if (DELTA && is_delta(m)) {
        int lobe = rec_light(recj) & 1;
        delta_sample(m, n, front, -s.din, u, wi, wt, lobe);
    } else {
        bsdf_sample(m, n, -s.din, u, v, wi, wt);
    }
    const V3 ngn = normalize(cross(xyz(Tn.e1), xyz(Tn.e2)));
    VState r;
    r.x = s.x + wi * plane_t(Tn, ngn, s.x, wi);
    r.din = wi;
    r.beta = mul(s.beta, wt);
    return r;
}

// Reverse sweep through vertex j.  `an` holds the adjoints of vertex j+1's
// state (zero if it does not exist).  Writes the gradients of the light block
// (4j-2, 4j-1) and, for j <= L-2, of the BSDF block (4j, 4j+1), scaled by
// 1/(p + eps).  Returns the adjoints of vertex j's state.
template <bool DELTA, class U>
__device__ Adj reverse_vertex(const DevScene& S, int L, int j, const VState& s, const Adj& an, uint32_t recj,
                              uint32_t recn, const U& u, float inv_pe, float* out, int os) {
    const DevTri T = S.tris[rec_slot(recj)];
    const Material m = load_material(S, __float_as_uint(T.e1.w));
    bool front;
    const V3 n = facing_normal(T, s.din, front);
    const V3 wo = -s.din;
    V3 gx = v3(0.f, 0.f, 0.f), gwo = v3(0.f, 0.f, 0.f), gb = v3(0.f, 0.f, 0.f);
    float gu = 0.f, gv = 0.f, ga = 0.f, gbl = 0.f;

    // ---- delta step j -> j+1: the direction follows from wo alone (the
    // dielectric's lobe is the recorded one), so the BSDF block has no
    // gradient; the emission counted at j+1 adds Le_{j+1} . d p / d beta'
    const bool delta = DELTA && is_delta(m);
    if (delta && j <= L - 2 && recn != DR_NO_VERTEX) {
        int lobe = rec_light(recj) & 1;
        V3 wi, W;
        delta_sample(m, n, front, wo, 0.0f, wi, W, lobe);
        const DevTri Tn = S.tris[rec_slot(recn)];
        const V3 ngn = normalize(cross(xyz(Tn.e1), xyz(Tn.e2)));
        const float Dn = dot(ngn, wi);
        const float iDn = arcp(Dn);
        const float tp = dot(ngn, xyz(Tn.v0) - s.x) * iDn;
        const float sc = dot(an.gx, wi) * iDn;
        const V3 gproj = an.gx - ngn * sc;
        gx = gx + gproj;
        const V3 gwi = gproj * tp + an.gd;
        V3 gbn = an.gb;
        if (faces_ray(Tn, wi)) {
            const V3 Le = load_material(S, __float_as_uint(Tn.e1.w)).Le;
            gbn = gbn + v3(0.2126f * Le.x, 0.7152f * Le.y, 0.0722f * Le.z);
        }
        gb = gb + mul(gbn, W);
        const float ci = dot(n, wo);
        if (lobe == 0) {
            // wi = 2 ci n - wo (mirror and dielectric reflection)
            float g_ci = 2.0f * dot(gwi, n);
            if (m.kind == MAT_MIRROR) {  // W = f0 + (1 - f0)(1 - ci)^5
                const V3 gW = mul(gbn, s.beta);
                const float om = 1.0f - ci;
                const float om4 = om * om * om * om;
                g_ci -= 5.0f * om4 *
                        (gW.x * (1.0f - m.f0.x) + gW.y * (1.0f - m.f0.y) + gW.z * (1.0f - m.f0.z));
            }
            gwo = gwo - gwi + n * g_ci;
        } else {
            // wi = -wo / etap + (ci / etap - ct) n, ct^2 = 1 - (1 - ci^2) / etap^2; W constant
            const float ie = arcp(rel_eta(m, front));
            float ct;
            fresnel_dielectric(ci, rel_eta(m, front), ct);
            const float dct = ct > 0.0f ? adiv(ci * ie * ie, ct) : 0.0f;
            gwo = gwo - gwi * ie + n * (dot(gwi, n) * (ie - dct));
        }
    }

    // ---- BSDF step j -> j+1: x' = x + t' wi, din' = wi, beta' = beta * W
    if (!delta && j <= L - 2 && recn != DR_NO_VERTEX) {
        const float uu = u(4 * j), vv = u(4 * j + 1);
        V3 tt, bb;
        onb(n, tt, bb);
        float sp, cp;
        __sincosf(2.0f * DR_PI * vv, &sp, &cp);
        V3 wi, W;
        // intermediates of the GGX branch
        V3 h = v3(0.f, 0.f, 0.f);
        float oh = 0.f, ch = 0.f, sh = 0.f, co = 0.f, ci = 0.f, den = 1.f, r = 0.f, lz = 0.f, wg = 0.f;
        if (m.kind == 0) {
            r = asqrt(uu);
            lz = asqrt(1.0f - uu);
            wi = tt * (r * cp) + bb * (r * sp) + n * lz;
            W = m.albedo;
        } else {
            den = (1.0f - uu) + m.a2 * uu;
            const float iden = arcp(den);
            ch = asqrt((1.0f - uu) * iden);
            sh = asqrt(m.a2 * uu * iden);
            h = tt * (sh * cp) + bb * (sh * sp) + n * ch;
            oh = dot(wo, h);
            wi = h * (2.0f * oh) - wo;
            ci = dot(n, wi);
            co = dot(n, wo);
            wg = adiv(smith_g1(co, m.a2) * smith_g1(ci, m.a2) * oh, co * ch);
            const float om = 1.0f - oh;
            const float f5 = om * om * om * om * om;
            W = v3(wg * (m.f0.x + (1.0f - m.f0.x) * f5), wg * (m.f0.y + (1.0f - m.f0.y) * f5),
                   wg * (m.f0.z + (1.0f - m.f0.z) * f5));
        }
        const DevTri Tn = S.tris[rec_slot(recn)];
        const V3 ngn = normalize(cross(xyz(Tn.e1), xyz(Tn.e2)));
        const float Dn = dot(ngn, wi);
        const float iDn = arcp(Dn);
        const float tp = dot(ngn, xyz(Tn.v0) - s.x) * iDn;
        // x' = x + tp wi with tp = ngn.(v0 - x)/(ngn.wi)
        const float sc = dot(an.gx, wi) * iDn;
        const V3 gproj = an.gx - ngn * sc;
        gx = gx + gproj;
        V3 gwi = gproj * tp + an.gd;
        gb = gb + mul(an.gb, W);
        const V3 gW = mul(an.gb, s.beta);
        if (m.kind == 0) {
            const float ir = 0.5f * arcp(r);
            gu += dot(gwi, tt * (cp * ir) + bb * (sp * ir) - n * (0.5f * arcp(lz)));
            gv += dot(gwi, bb * cp - tt * sp) * (r * 2.0f * DR_PI);
        } else {
            // W_c = F_c(oh) wg, wg = G1(co) G1(ci) oh / (co ch)
            const float om = 1.0f - oh;
            const float om4 = om * om * om * om;
            const V3 F = v3(m.f0.x + (1.0f - m.f0.x) * om4 * om, m.f0.y + (1.0f - m.f0.y) * om4 * om,
                            m.f0.z + (1.0f - m.f0.z) * om4 * om);
            const V3 dF = v3(-5.0f * (1.0f - m.f0.x) * om4, -5.0f * (1.0f - m.f0.y) * om4,
                             -5.0f * (1.0f - m.f0.z) * om4);
            const float gwg = dot(gW, F);                 // d/d wg
            const float g_oh_F = dot(gW, dF) * wg;        // through F(oh)
            float g_oh = g_oh_F + adiv(gwg * wg, oh);
            const float g_co = gwg * wg * (smith_dlog(co, m.a2) - arcp(co));
            const float g_ci = gwg * wg * smith_dlog(ci, m.a2);
            const float g_ch = adiv(-gwg * wg, ch);
            gwi = gwi + n * g_ci;
            // wi = 2 oh h - wo
            g_oh += 2.0f * dot(gwi, h);
            V3 g_h = gwi * (2.0f * oh);
            gwo = gwo - gwi;
            // oh = wo . h ; co = n . wo
            gwo = gwo + h * g_oh + n * g_co;
            g_h = g_h + wo * g_oh;
            // h = tt (sh cos) + bb (sh sin) + n ch ; ch, sh functions of uu
            const float dch = adiv(-m.a2, 2.0f * ch * den * den);
            const float dsh = adiv(m.a2, 2.0f * sh * den * den);
            gu += dot(g_h, tt * cp + bb * sp) * dsh + (dot(g_h, n) + g_ch) * dch;
            gv += dot(g_h, bb * cp - tt * sp) * (sh * 2.0f * DR_PI);
        }
    }

    // ---- next-event estimation at vertex j
    if (rec_contrib(recj)) {
        const int li = rec_light(recj);
        const int nl = S.n_lights;
        const float a = u(4 * j - 2), b = u(4 * j - 1);
        const float ap = a * (float)nl - (float)li;
        const float4 l0 = S.lights[5 * li], l1 = S.lights[5 * li + 1], l2 = S.lights[5 * li + 2],
                     l3 = S.lights[5 * li + 3], l4 = S.lights[5 * li + 4];
        const V3 E1 = xyz(l1), E2 = xyz(l2), NL = xyz(l3), Le = xyz(l4);
        const V3 y = xyz(l0) + E1 * ap + E2 * b;
        const V3 w = y - s.x;
        const float r2 = dot(w, w);
        const float r = asqrt(r2);
        const V3 wl = w * arcp(r);
        const float cx = dot(n, wl);
        const float cy = -dot(NL, wl);
        const float Cc = (float)nl * l3.w;
        const float ir2 = arcp(r2);
        const float g = cx * cy * ir2 * Cc;
        const V3 K = v3(0.2126f * Le.x, 0.7152f * Le.y, 0.0722f * Le.z);  // d p / d T
        float g_g, g_cx = 0.f;
        V3 g_wl = v3(0.f, 0.f, 0.f);
        if (m.kind == 0) {
            const V3 fs = m.albedo * (1.0f / DR_PI);
            gb = gb + mul(K, fs) * g;
            g_g = dot(mul(K, s.beta), fs);
        } else {
            const float co = dot(n, wo);
            const V3 hs = wo + wl;
            const float hl = asqrt(dot(hs, hs));
            const float ihl = arcp(hl);
            const V3 h = hs * ihl;
            const float chh = dot(n, h);
            const float den = chh * chh * (m.a2 - 1.0f) + 1.0f;
            const float D = adiv(m.a2, DR_PI * den * den);
            const float G = smith_g1(co, m.a2) * smith_g1(cx, m.a2);
            const float oh = dot(wl, h);
            const float om = 1.0f - oh;
            const float om4 = om * om * om * om;
            const V3 F = v3(m.f0.x + (1.0f - m.f0.x) * om4 * om, m.f0.y + (1.0f - m.f0.y) * om4 * om,
                            m.f0.z + (1.0f - m.f0.z) * om4 * om);
            const V3 dF = v3(-5.0f * (1.0f - m.f0.x) * om4, -5.0f * (1.0f - m.f0.y) * om4,
                             -5.0f * (1.0f - m.f0.z) * om4);
            const float kk = D * G / (4.0f * co * cx);  // f_s = kk F
            const V3 Kb = mul(K, s.beta);
            gb = gb + mul(K, F) * (kk * g);
            const float fsum = kk * dot(Kb, F);
            g_g = fsum;
            const float gl = g * fsum;  // this vertex's share of p
            const float g_chh = gl * adiv(-4.0f * chh * (m.a2 - 1.0f), den);
            const float g_co = gl * (smith_dlog(co, m.a2) - arcp(co));
            g_cx = gl * (smith_dlog(cx, m.a2) - arcp(cx));
            const float g_oh = g * kk * dot(Kb, dF);
            const V3 g_h = n * g_chh + wl * g_oh;
            g_wl = h * g_oh;
            const V3 g_hs = (g_h - h * dot(h, g_h)) * ihl;
            gwo = gwo + g_hs + n * g_co;
            g_wl = g_wl + g_hs;
        }
        g_cx += g_g * cy * ir2 * Cc;
        const float g_cy = g_g * cx * ir2 * Cc;
        const float g_r2 = -g_g * g * ir2;
        g_wl = g_wl + n * g_cx - NL * g_cy;
        const V3 g_w = w * (2.0f * g_r2) + (g_wl - wl * dot(wl, g_wl)) * arcp(r);
        gx = gx - g_w;
        ga = (float)nl * dot(g_w, E1);
        gbl = dot(g_w, E2);
    }

    auto put = [&](int i, float gval) {
        float q = gval * inv_pe;
        if (!isfinite(q)) q = 0.0f;
        out[(size_t)i * os] = q;
    };
    put(4 * j - 2, ga);
    put(4 * j - 1, gbl);
    if (j <= L - 2) {
        put(4 * j, gu);
        put(4 * j + 1, gv);
    }
    Adj r;
    r.gx = gx;
    r.gd = -gwo;
    r.gb = gb;
    return r;
}

// score[i * os] = d ln(p + eps) / d u_i for the recorded path (rec[(j-1)*rs]).
template <int L, bool DELTA = true, class U>
__device__ void path_score(const DevScene& S, const U& u, const uint32_t* rec, int rs, float p, float eps, float* out,
                           int os) {
    constexpr int V = L - 1;
    constexpr int NSEG = (V + DR_SEG - 1) / DR_SEG;
    const uint32_t r1 = rec[0];
    if (!(p > 0.0f) || r1 == DR_NO_VERTEX) {
        for (int i = 0; i < 4 * V; ++i) out[(size_t)i * os] = 0.0f;
        return;
    }
    const float inv_pe = arcp(p + eps);
    const Cam Cm = load_cam(S);
    uint32_t R[V + 1];
#pragma unroll
    for (int j = 1; j <= V; ++j) R[j] = rec[(j - 1) * rs];
    R[0] = 0;

    // checkpoints at the first vertex of every segment
    VState cp[NSEG];
    {
        VState st = camera_state(Cm, u(0), u(1), S.tris[rec_slot(R[1])]);
#pragma unroll
        for (int j = 1; j <= V; ++j) {
            if ((j - 1) % DR_SEG == 0) cp[(j - 1) / DR_SEG] = st;
            if (NSEG > 1 && j < V && (j - 1) / DR_SEG < NSEG - 1 && R[j + 1] != DR_NO_VERTEX)
                st = advance<DELTA>(S, st, S.tris[rec_slot(R[j])], S.tris[rec_slot(R[j + 1])], u(4 * j), u(4 * j + 1), R[j]);
        }
    }
    Adj a;
    a.gx = a.gd = a.gb = v3(0.f, 0.f, 0.f);
#pragma unroll
    for (int sg = NSEG - 1; sg >= 0; --sg) {
        constexpr int dummy = 0;
        (void)dummy;
        const int j0 = sg * DR_SEG + 1;
        VState tape[DR_SEG];
        VState st = cp[sg];
#pragma unroll
        for (int k = 0; k < DR_SEG; ++k) {
            const int j = j0 + k;
            if (j <= V) {
                tape[k] = st;
                if (k < DR_SEG - 1 && j < V && R[j] != DR_NO_VERTEX && R[j + 1] != DR_NO_VERTEX)
                    st = advance<DELTA>(S, st, S.tris[rec_slot(R[j])], S.tris[rec_slot(R[j + 1])], u(4 * j), u(4 * j + 1), R[j]);
            }
        }
#pragma unroll
        for (int k = DR_SEG - 1; k >= 0; --k) {
            const int j = j0 + k;
            if (j <= V) {
                const uint32_t rn = (j < V) ? R[j + 1] : DR_NO_VERTEX;
                if (R[j] != DR_NO_VERTEX) {
                    a = reverse_vertex<DELTA>(S, L, j, tape[k], a, R[j], rn, u, inv_pe, out, os);
                } else {
                    out[(size_t)(4 * j - 2) * os] = 0.0f;
                    out[(size_t)(4 * j - 1) * os] = 0.0f;
                    if (j <= L - 2) {
                        out[(size_t)(4 * j) * os] = 0.0f;
                        out[(size_t)(4 * j + 1) * os] = 0.0f;
                    }
                }
            }
        }
    }
    // camera: x1 = eye + t1 d, d = D/|D|, D = cw + (2u0-1) cu + (1-2u1) cv
    {
        const float u0 = u(0), u1 = u(1);
        const V3 D = Cm.cw + Cm.cu * (2.0f * u0 - 1.0f) + Cm.cv * (1.0f - 2.0f * u1);
        const float Dl = asqrt(dot(D, D));
        const float iDl = arcp(Dl);
        const V3 d = D * iDl;
        const DevTri T1 = S.tris[rec_slot(R[1])];
        const V3 ng = normalize(cross(xyz(T1.e1), xyz(T1.e2)));
        const float Dn = dot(ng, d);
        const float iDn = arcp(Dn);
        const float t1 = dot(ng, xyz(T1.v0) - Cm.eye) * iDn;
        const float sc = dot(a.gx, d) * iDn;
        const V3 gd = a.gd + (a.gx - ng * sc) * t1;
        const V3 gD = (gd - d * dot(d, gd)) * iDl;
        float g0 = 2.0f * dot(gD, Cm.cu) * inv_pe, g1 = -2.0f * dot(gD, Cm.cv) * inv_pe;
        if (!isfinite(g0)) g0 = 0.0f;
        if (!isfinite(g1)) g1 = 0.0f;
        out[0] = g0;
        out[(size_t)os] = g1;
    }
}

}  // namespace dr
