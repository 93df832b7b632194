// Diffusion Restore CPU oracle — FP64, plain, slow, single-purpose.
//
// TEST INFRASTRUCTURE ONLY.  This file is the reference against which the HIP
// library is checked.  Only the test-suite, the smoke check and the CPU
// baseline leg of the benchmark may load it.  It shares no code, header,
// table or helper with the GPU library; both sides only consume the same
// seeded inputs (scene arrays, chain states, per-chain sigma).
//
// What it computes (paper sections in brackets):
//   * Philox4x32-10 counter-based generator [Sec. 4.3, the tour state's rng;
//     generator of Salmon et al. 2011] and the uniform / Gaussian /
//     exponential draws built on it.
//   * f(u): a primary-sample-space path sampler (camera, Lambertian, GGX
//     conductor, smooth conductor and smooth dielectric surfaces [Sec. 6, the
//     material set of the test scenes], quad area lights with next-event
//     estimation).  The paper does not specify its sampler; the definition
//     used here is the one written out in the design notes (readings A1,
//     A10, A13-A15, A24).
//   * score = grad_u ln(p(u) + eps) by forward-mode dual numbers over the
//     taken path (discrete choices held fixed) [Sec. 5, Langevin drift].
//   * The Diffusion Restore chain: initialise / evolve / resolve
//     [Alg. 4.1, 4.2, 4.3], Euler-Maruyama local dynamics with rotational
//     drift [Eq. local-dynamics, Alg. 5.1], holding rate 1/dt
//     [Eq. diffusion-restore-holding-rate], modified killing rate k0/p
//     [Eq. modified-killing-rate], k0 = p_lambda/(m dt)
//     [Eq. killing-rate-constant], Rao-Blackwellised or sampled holding
//     weights (reading A8).
//   * Independent path tracing (brute-force Monte Carlo reference image).
//   * An analytic wrapped-Gaussian-mixture target on the torus, used to pin
//     the chain's estimator against closed forms.
//
// Precision: FP64 everywhere, except the decisions that map a float to an
// integer (pixel index, light index, kill, reflect-or-refract), which are
// taken in FP32 as the GPU kernels take them.
//
// Built with: g++ -O2 -std=c++17 -ffp-contract=off -fPIC -shared -pthread

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <memory>
#include <thread>
#include <type_traits>
#include <vector>

namespace orc {

// ----------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw: "Parallel random numbers: as easy
// as 1, 2, 3", SC 2011).  Ten rounds of the 4x32 S-box with multipliers
// 0xD2511F53 / 0xCD9E8D57 and Weyl key increments 0x9E3779B9 / 0xBB67AE85.
// ----------------------------------------------------------------------------
static void philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
    uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
    uint32_t k[2] = {key_in[0], key_in[1]};
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k[0] += 0x9E3779B9u;
            k[1] += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c[0];
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c[2];
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c[1] ^ k[0];
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c[3] ^ k[1];
        uint32_t n3 = lo0;
        c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
    }
    out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

// Stream layout (reading A12): counter = (chain, step lo, step hi,
// tag<<24 | i>>2), key = seed; word i&3; uniform = top 24 bits * 2^-24.
enum { TAG_REGEN = 0, TAG_GAUSS = 1, TAG_HOLD = 2, TAG_PT = 4 };

static double uniform(uint64_t seed, uint32_t chain, uint64_t step, uint32_t tag, uint32_t i) {
    uint32_t ctr[4] = {chain, (uint32_t)step, (uint32_t)(step >> 32), (tag << 24) | (i >> 2)};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    philox4x32_10(ctr, key, out);
    return (double)(out[i & 3] >> 8) * (1.0 / 16777216.0);
}

// Box-Muller: r = sqrt(-2 ln(1-U0)), (cos 2 pi U1, sin 2 pi U1).
static void box_muller(double u0, double u1, double& z0, double& z1) {
    const double r = std::sqrt(-2.0 * std::log(1.0 - u0));
    const double a = 2.0 * M_PI * u1;
    z0 = r * std::cos(a);
    z1 = r * std::sin(a);
}

// Unit exponential by inversion.
static double expo(double u) { return -std::log(1.0 - u); }

// ----------------------------------------------------------------------------
// Forward-mode dual numbers over the d primary-sample coordinates.
// ----------------------------------------------------------------------------
constexpr int DMAX = 64;
static thread_local int g_nd = 0;  // number of live derivative slots

struct Dual {
    double v;
    double g[DMAX];
    Dual() : v(0) { for (int i = 0; i < g_nd; ++i) g[i] = 0; }
    Dual(double x) : v(x) { for (int i = 0; i < g_nd; ++i) g[i] = 0; }
    static Dual var(double x, int slot) { Dual r(x); r.g[slot] = 1.0; return r; }
};
static inline double val(double x) { return x; }
static inline double val(const Dual& x) { return x.v; }

static inline Dual operator+(const Dual& a, const Dual& b) { Dual r; r.v = a.v + b.v; for (int i = 0; i < g_nd; ++i) r.g[i] = a.g[i] + b.g[i]; return r; }
static inline Dual operator-(const Dual& a, const Dual& b) { Dual r; r.v = a.v - b.v; for (int i = 0; i < g_nd; ++i) r.g[i] = a.g[i] - b.g[i]; return r; }
static inline Dual operator*(const Dual& a, const Dual& b) { Dual r; r.v = a.v * b.v; for (int i = 0; i < g_nd; ++i) r.g[i] = a.g[i] * b.v + a.v * b.g[i]; return r; }
static inline Dual operator/(const Dual& a, const Dual& b) { Dual r; r.v = a.v / b.v; for (int i = 0; i < g_nd; ++i) r.g[i] = (a.g[i] * b.v - a.v * b.g[i]) / (b.v * b.v); return r; }
static inline Dual operator+(const Dual& a, double b) { Dual r = a; r.v += b; return r; }
static inline Dual operator+(double a, const Dual& b) { return b + a; }
static inline Dual operator-(const Dual& a, double b) { Dual r = a; r.v -= b; return r; }
static inline Dual operator-(double a, const Dual& b) { Dual r; r.v = a - b.v; for (int i = 0; i < g_nd; ++i) r.g[i] = -b.g[i]; return r; }
static inline Dual operator-(const Dual& a) { Dual r; r.v = -a.v; for (int i = 0; i < g_nd; ++i) r.g[i] = -a.g[i]; return r; }
static inline Dual operator*(const Dual& a, double b) { Dual r; r.v = a.v * b; for (int i = 0; i < g_nd; ++i) r.g[i] = a.g[i] * b; return r; }
static inline Dual operator*(double a, const Dual& b) { return b * a; }
static inline Dual operator/(const Dual& a, double b) { Dual r; r.v = a.v / b; for (int i = 0; i < g_nd; ++i) r.g[i] = a.g[i] / b; return r; }
static inline Dual operator/(double a, const Dual& b) { Dual r; r.v = a / b.v; for (int i = 0; i < g_nd; ++i) r.g[i] = -a * b.g[i] / (b.v * b.v); return r; }
static inline Dual sqrt(const Dual& a) { Dual r; r.v = std::sqrt(a.v); for (int i = 0; i < g_nd; ++i) r.g[i] = a.g[i] / (2.0 * r.v); return r; }
static inline Dual sin(const Dual& a) { Dual r; r.v = std::sin(a.v); double c = std::cos(a.v); for (int i = 0; i < g_nd; ++i) r.g[i] = c * a.g[i]; return r; }
static inline Dual cos(const Dual& a) { Dual r; r.v = std::cos(a.v); double s = -std::sin(a.v); for (int i = 0; i < g_nd; ++i) r.g[i] = s * a.g[i]; return r; }

// Forward mode with a running magnitude (a conditioning measure, not part of
// the method): besides the derivative g, a[i] accumulates, for input i, the
// sum over the computation's dependency paths of the products of the
// magnitudes of the local partial derivatives, so a >= |g|.  Evaluating the
// derivative in a lower precision, in forward or reverse mode, rounds every
// intermediate term; to first order the error is at most (roundings along a
// path) x (unit roundoff) x a, and a / |g| is the derivative's condition
// number (large where terms cancel).
struct DualA {
    double v;
    double g[DMAX], a[DMAX];
    DualA() : v(0) { for (int i = 0; i < g_nd; ++i) g[i] = a[i] = 0; }
    DualA(double x) : v(x) { for (int i = 0; i < g_nd; ++i) g[i] = a[i] = 0; }
    static DualA var(double x, int slot) { DualA r(x); r.g[slot] = 1.0; r.a[slot] = 1.0; return r; }
};
static inline double val(const DualA& x) { return x.v; }
static inline DualA operator+(const DualA& x, const DualA& y) { DualA r; r.v = x.v + y.v; for (int i = 0; i < g_nd; ++i) { r.g[i] = x.g[i] + y.g[i]; r.a[i] = x.a[i] + y.a[i]; } return r; }
static inline DualA operator-(const DualA& x, const DualA& y) { DualA r; r.v = x.v - y.v; for (int i = 0; i < g_nd; ++i) { r.g[i] = x.g[i] - y.g[i]; r.a[i] = x.a[i] + y.a[i]; } return r; }
static inline DualA operator*(const DualA& x, const DualA& y) { DualA r; r.v = x.v * y.v; for (int i = 0; i < g_nd; ++i) { r.g[i] = x.g[i] * y.v + x.v * y.g[i]; r.a[i] = x.a[i] * std::fabs(y.v) + std::fabs(x.v) * y.a[i]; } return r; }
static inline DualA operator/(const DualA& x, const DualA& y) { DualA r; r.v = x.v / y.v; const double y2 = y.v * y.v; for (int i = 0; i < g_nd; ++i) { r.g[i] = (x.g[i] * y.v - x.v * y.g[i]) / y2; r.a[i] = (x.a[i] * std::fabs(y.v) + std::fabs(x.v) * y.a[i]) / y2; } return r; }
static inline DualA operator+(const DualA& x, double y) { DualA r = x; r.v += y; return r; }
static inline DualA operator+(double x, const DualA& y) { return y + x; }
static inline DualA operator-(const DualA& x, double y) { DualA r = x; r.v -= y; return r; }
static inline DualA operator-(double x, const DualA& y) { DualA r; r.v = x - y.v; for (int i = 0; i < g_nd; ++i) { r.g[i] = -y.g[i]; r.a[i] = y.a[i]; } return r; }
static inline DualA operator-(const DualA& x) { DualA r; r.v = -x.v; for (int i = 0; i < g_nd; ++i) { r.g[i] = -x.g[i]; r.a[i] = x.a[i]; } return r; }
static inline DualA operator*(const DualA& x, double y) { DualA r; r.v = x.v * y; for (int i = 0; i < g_nd; ++i) { r.g[i] = x.g[i] * y; r.a[i] = x.a[i] * std::fabs(y); } return r; }
static inline DualA operator*(double x, const DualA& y) { return y * x; }
static inline DualA operator/(const DualA& x, double y) { DualA r; r.v = x.v / y; for (int i = 0; i < g_nd; ++i) { r.g[i] = x.g[i] / y; r.a[i] = x.a[i] / std::fabs(y); } return r; }
static inline DualA operator/(double x, const DualA& y) { DualA r; r.v = x / y.v; const double y2 = y.v * y.v; for (int i = 0; i < g_nd; ++i) { r.g[i] = -x * y.g[i] / y2; r.a[i] = std::fabs(x) * y.a[i] / y2; } return r; }
static inline DualA sqrt(const DualA& x) { DualA r; r.v = std::sqrt(x.v); for (int i = 0; i < g_nd; ++i) { r.g[i] = x.g[i] / (2.0 * r.v); r.a[i] = x.a[i] / (2.0 * r.v); } return r; }
static inline DualA sin(const DualA& x) { DualA r; r.v = std::sin(x.v); const double c = std::cos(x.v); for (int i = 0; i < g_nd; ++i) { r.g[i] = c * x.g[i]; r.a[i] = std::fabs(c) * x.a[i]; } return r; }
static inline DualA cos(const DualA& x) { DualA r; r.v = std::cos(x.v); const double sn = -std::sin(x.v); for (int i = 0; i < g_nd; ++i) { r.g[i] = sn * x.g[i]; r.a[i] = std::fabs(sn) * x.a[i]; } return r; }
using std::sqrt; using std::sin; using std::cos;

template <class T> struct V3 {
    T x, y, z;
    V3() : x(0.0), y(0.0), z(0.0) {}
    V3(T a, T b, T c) : x(a), y(b), z(c) {}
};
template <class T> static inline V3<T> operator+(const V3<T>& a, const V3<T>& b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <class T> static inline V3<T> operator-(const V3<T>& a, const V3<T>& b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <class T, class S> static inline V3<T> operator*(const V3<T>& a, const S& s) { return {a.x * s, a.y * s, a.z * s}; }
template <class T> static inline T dot(const V3<T>& a, const V3<T>& b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <class T> static inline V3<T> cross(const V3<T>& a, const V3<T>& b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <class T> static inline V3<T> normalize(const V3<T>& a) { T l = sqrt(dot(a, a)); return {a.x / l, a.y / l, a.z / l}; }
template <class T> static inline V3<T> lift(const V3<double>& a) { return {T(a.x), T(a.y), T(a.z)}; }
static inline V3<double> vald(const V3<Dual>& a) { return {a.x.v, a.y.v, a.z.v}; }
static inline V3<double> vald(const V3<DualA>& a) { return {a.x.v, a.y.v, a.z.v}; }
static inline V3<double> vald(const V3<double>& a) { return a; }

// ----------------------------------------------------------------------------
// Scene: triangles, materials, quad lights, pinhole camera.
// ----------------------------------------------------------------------------
struct Material {
    int kind;            // 0 Lambertian, 1 GGX conductor, 2 smooth conductor, 3 smooth dielectric
    double albedo[3];
    double rough;        // GGX alpha
    double f0[3];        // Schlick normal-incidence reflectance (conductors)
    double Le[3];        // emitted radiance (emitter triangles)
    double eta;          // dielectric: index of refraction of the inside (the side opposite e1 x e2)
};
static inline bool is_delta(const Material& m) { return m.kind >= 2; }
struct Light {
    V3<double> p0, e1, e2, n;  // parallelogram p0 + a e1 + b e2, unit normal e1 x e2
    double area;
    double Le[3];
};
struct BvhNode {
    double lo[3], hi[3];
    int left, right;     // children; left < 0 => leaf
    int first, count;    // leaf range in `order`
};

struct Scene {
    std::vector<V3<double>> v;
    std::vector<uint32_t> idx;
    std::vector<uint32_t> tmat;
    std::vector<Material> mats;
    std::vector<Light> lights;
    V3<double> eye, cu, cv, cw;  // camera: dir = (2u0-1) cu + (1-2u1) cv + cw
    int W = 0, H = 0;
    double tmin = 0;
    std::vector<BvhNode> nodes;
    std::vector<int> order;
    bool brute = false;

    int ntri() const { return (int)(idx.size() / 3); }
    V3<double> vert(int t, int k) const { return v[idx[3 * t + k]]; }
};

// Median-split BVH on centroids (longest axis), leaves of up to 4 triangles.
static int bvh_build(Scene& S, int first, int count) {
    BvhNode nd;
    for (int a = 0; a < 3; ++a) { nd.lo[a] = 1e300; nd.hi[a] = -1e300; }
    double clo[3] = {1e300, 1e300, 1e300}, chi[3] = {-1e300, -1e300, -1e300};
    for (int i = first; i < first + count; ++i) {
        int t = S.order[i];
        for (int k = 0; k < 3; ++k) {
            V3<double> p = S.vert(t, k);
            double c[3] = {p.x, p.y, p.z};
            for (int a = 0; a < 3; ++a) { nd.lo[a] = std::min(nd.lo[a], c[a]); nd.hi[a] = std::max(nd.hi[a], c[a]); }
        }
        V3<double> c = (S.vert(t, 0) + S.vert(t, 1) + S.vert(t, 2)) * (1.0 / 3.0);
        double cc[3] = {c.x, c.y, c.z};
        for (int a = 0; a < 3; ++a) { clo[a] = std::min(clo[a], cc[a]); chi[a] = std::max(chi[a], cc[a]); }
    }
    int me = (int)S.nodes.size();
    S.nodes.push_back(nd);
    if (count <= 4) {
        S.nodes[me].left = S.nodes[me].right = -1;
        S.nodes[me].first = first; S.nodes[me].count = count;
        return me;
    }
    int axis = 0;
    for (int a = 1; a < 3; ++a) if (chi[a] - clo[a] > chi[axis] - clo[axis]) axis = a;
    auto key = [&](int t) {
        V3<double> c = S.vert(t, 0) + S.vert(t, 1) + S.vert(t, 2);
        return axis == 0 ? c.x : (axis == 1 ? c.y : c.z);
    };
    int half = count / 2;
    std::nth_element(S.order.begin() + first, S.order.begin() + first + half, S.order.begin() + first + count,
                     [&](int a, int b) { double ka = key(a), kb = key(b); return ka < kb || (ka == kb && a < b); });
    int l = bvh_build(S, first, half);
    int r = bvh_build(S, first + half, count - half);
    S.nodes[me].left = l; S.nodes[me].right = r;
    S.nodes[me].first = 0; S.nodes[me].count = 0;
    return me;
}

// Moller-Trumbore, two-sided.  Returns true and t on a hit in (tmin, tmax).
template <class T>
static bool tri_hit(const Scene& S, int tri, const V3<T>& o, const V3<T>& d, double tmin, double tmax, T& t_out,
                    bool force) {
    V3<double> v0 = S.vert(tri, 0), v1 = S.vert(tri, 1), v2 = S.vert(tri, 2);
    V3<T> e1 = lift<T>(v1 - v0), e2 = lift<T>(v2 - v0);
    V3<T> pv = cross(d, e2);
    T det = dot(e1, pv);
    if (!force && val(det) == 0.0) return false;
    T inv = 1.0 / det;
    V3<T> tv = o - lift<T>(v0);
    T b1 = dot(tv, pv) * inv;
    if (!force && (val(b1) < 0.0 || val(b1) > 1.0)) return false;
    V3<T> qv = cross(tv, e1);
    T b2 = dot(d, qv) * inv;
    if (!force && (val(b2) < 0.0 || val(b1) + val(b2) > 1.0)) return false;
    T t = dot(e2, qv) * inv;
    if (!force && !(val(t) > tmin && val(t) < tmax)) return false;
    t_out = t;
    return true;
}

static bool box_hit(const BvhNode& n, const V3<double>& o, const V3<double>& d, double tmin, double tmax) {
    double oo[3] = {o.x, o.y, o.z}, dd[3] = {d.x, d.y, d.z};
    double t0 = tmin, t1 = tmax;
    for (int a = 0; a < 3; ++a) {
        if (dd[a] == 0.0) {
            if (oo[a] < n.lo[a] || oo[a] > n.hi[a]) return false;
            continue;
        }
        double ta = (n.lo[a] - oo[a]) / dd[a], tb = (n.hi[a] - oo[a]) / dd[a];
        if (ta > tb) std::swap(ta, tb);
        t0 = std::max(t0, ta);
        t1 = std::min(t1, tb);
    }
    // inclusive with a relative pad so that FP64 slab rounding never culls a hit
    double pad = 1e-9 * (std::fabs(t1) + 1.0);
    return t0 <= t1 + pad;
}

// Closest hit over (tmin, tmax); ties in t go to the lower triangle index.
static int closest(const Scene& S, const V3<double>& o, const V3<double>& d, double tmin, double tmax, double* t_hit) {
    int best = -1;
    double bt = tmax;
    auto test = [&](int tri) {
        double t;
        if (tri_hit<double>(S, tri, o, d, tmin, tmax, t, false)) {
            if (t < bt || (t == bt && tri < best)) { bt = t; best = tri; }
        }
    };
    if (S.brute) {
        for (int tri = 0; tri < S.ntri(); ++tri) test(tri);
    } else {
        std::vector<int> stack;
        stack.push_back(0);
        while (!stack.empty()) {
            int ni = stack.back(); stack.pop_back();
            const BvhNode& n = S.nodes[ni];
            // bt is inclusive here so that an equal-t triangle with a lower index is still found
            if (!box_hit(n, o, d, tmin, bt)) continue;
            if (n.left < 0) {
                for (int i = n.first; i < n.first + n.count; ++i) test(S.order[i]);
            } else {
                stack.push_back(n.left);
                stack.push_back(n.right);
            }
        }
    }
    if (t_hit) *t_hit = bt;
    return best;
}

static bool occluded(const Scene& S, const V3<double>& o, const V3<double>& d, double tmin, double tmax) {
    if (S.brute) {
        for (int tri = 0; tri < S.ntri(); ++tri) { double t; if (tri_hit<double>(S, tri, o, d, tmin, tmax, t, false)) return true; }
        return false;
    }
    std::vector<int> stack;
    stack.push_back(0);
    while (!stack.empty()) {
        int ni = stack.back(); stack.pop_back();
        const BvhNode& n = S.nodes[ni];
        if (!box_hit(n, o, d, tmin, tmax)) continue;
        if (n.left < 0) {
            for (int i = n.first; i < n.first + n.count; ++i) { double t; if (tri_hit<double>(S, S.order[i], o, d, tmin, tmax, t, false)) return true; }
        } else {
            stack.push_back(n.left);
            stack.push_back(n.right);
        }
    }
    return false;
}

// ----------------------------------------------------------------------------
// BSDFs.  Lambertian: albedo/pi, cosine-weighted sampling.  GGX conductor:
// Trowbridge-Reitz D, separable Smith G, Schlick F, D-proportional half-vector
// sampling, alpha = roughness.
// ----------------------------------------------------------------------------
// Orthonormal basis from a unit normal (Duff et al., "Building an Orthonormal
// Basis, Revisited", JCGT 2017).
static void onb(const V3<double>& n, V3<double>& t, V3<double>& b) {
    double sign = std::copysign(1.0, n.z);
    double a = -1.0 / (sign + n.z);
    double bb = n.x * n.y * a;
    t = {1.0 + sign * n.x * n.x * a, sign * bb, -sign * n.x};
    b = {bb, sign + n.y * n.y * a, -n.y};
}

template <class T> static T smith_g1(T c, double alpha) {
    T c2 = c * c;
    T tan2 = (1.0 - c2) / c2;
    return 2.0 / (1.0 + sqrt(1.0 + alpha * alpha * tan2));
}

// Trowbridge-Reitz (GGX) normal distribution at cos(theta_h) = ch.
template <class T> static T ggx_d(T ch, double a2) {
    T den = ch * ch * (a2 - 1.0) + 1.0;
    return a2 / (M_PI * den * den);
}

// f_s(wo, wi) * (per channel).  Caller guarantees n.wo > 0 and n.wi > 0.
template <class T>
static void bsdf_eval(const Material& m, const V3<double>& n, const V3<T>& wo, const V3<T>& wi, T fs[3]) {
    if (m.kind == 0) {
        for (int c = 0; c < 3; ++c) fs[c] = T(m.albedo[c] / M_PI);
        return;
    }
    const double a = m.rough, a2 = a * a;
    V3<T> nn = lift<T>(n);
    T co = dot(nn, wo), ci = dot(nn, wi);
    V3<T> h = normalize(wo + wi);
    T ch = dot(nn, h);
    T D = ggx_d(ch, a2);
    T G = smith_g1(co, a) * smith_g1(ci, a);
    T oh = dot(wi, h);
    T one_m = 1.0 - oh;
    T f5 = one_m * one_m * one_m * one_m * one_m;
    for (int c = 0; c < 3; ++c) {
        T F = m.f0[c] + (1.0 - m.f0[c]) * f5;
        fs[c] = D * G * F / (4.0 * co * ci);
    }
}

// Sample wi given wo and the 2-D block (u, v).  Returns false if the sample
// leaves the upper hemisphere (the path then ends).  weight = f_s cos / pdf.
template <class T>
static bool bsdf_sample(const Material& m, const V3<double>& n, const V3<T>& wo, const T& u, const T& v, V3<T>& wi,
                        T weight[3]) {
    V3<double> tt, bb;
    onb(n, tt, bb);
    V3<T> nn = lift<T>(n), tT = lift<T>(tt), bT = lift<T>(bb);
    T phi = 2.0 * M_PI * v;
    if (m.kind == 0) {
        T r = sqrt(u);
        T lz = sqrt(1.0 - u);
        wi = tT * (r * cos(phi)) + bT * (r * sin(phi)) + nn * lz;
        for (int c = 0; c < 3; ++c) weight[c] = T(m.albedo[c]);
        return true;
    }
    const double a = m.rough, a2 = a * a;
    T den = (1.0 - u) + a2 * u;
    T ch = sqrt((1.0 - u) / den);
    T sh = sqrt(a2 * u / den);
    V3<T> h = tT * (sh * cos(phi)) + bT * (sh * sin(phi)) + nn * ch;
    T oh = dot(wo, h);
    if (val(oh) <= 0.0) return false;
    wi = h * (2.0 * oh) - wo;
    T ci = dot(nn, wi);
    if (val(ci) <= 0.0) return false;
    T co = dot(nn, wo);
    T g = smith_g1(co, a) * smith_g1(ci, a);
    T one_m = 1.0 - oh;
    T f5 = one_m * one_m * one_m * one_m * one_m;
    for (int c = 0; c < 3; ++c) {
        T F = m.f0[c] + (1.0 - m.f0[c]) * f5;
        weight[c] = F * g * oh / (co * ch);
    }
    return true;
}

// Fresnel reflectance of a smooth dielectric interface for unpolarised light
// (the Fresnel equations: the mean of the squared s- and p-amplitude ratios).
// ci = cosine on the incident side, etap = n_transmitted / n_incident.  Returns
// 1 under total internal reflection; ct is the transmitted cosine.
template <class T> static T fresnel_dielectric(const T& ci, double etap, T& ct) {
    T sin2_t = (1.0 - ci * ci) / (etap * etap);
    if (val(sin2_t) >= 1.0) {
        ct = T(0.0);
        return T(1.0);
    }
    ct = sqrt(1.0 - sin2_t);
    T rs = (ci - etap * ct) / (ci + etap * ct);  // n_i cos_i vs n_t cos_t, over n_i
    T rp = (etap * ci - ct) / (etap * ci + ct);  // n_t cos_i vs n_i cos_t, over n_i
    return 0.5 * (rs * rs + rp * rp);
}

// Delta (specular) lobes.  n faces wo; `front` says wo lies on the e1 x e2
// side (outside a dielectric).  Smooth conductor: mirror direction, weight
// Schlick's F at the incidence cosine.  Smooth dielectric: the coordinate u
// picks reflection when u < F (in FP32, as the kernels decide), else
// refraction by Snell's law; the weights are F/F = 1 and, for refraction,
// (1-F)/(1-F) divided by etap^2 (radiance is compressed into the denser
// medium).  lobe = 0 reflection, 1 refraction.
template <class T>
static void delta_sample(const Material& m, const V3<double>& n, bool front, const V3<T>& wo, const T& u, V3<T>& wi,
                         T weight[3], int& lobe) {
    V3<T> nn = lift<T>(n);
    T ci = dot(nn, wo);
    lobe = 0;
    if (m.kind == 2) {
        wi = nn * (2.0 * ci) - wo;
        T one_m = 1.0 - ci;
        T f5 = one_m * one_m * one_m * one_m * one_m;
        for (int c = 0; c < 3; ++c) weight[c] = m.f0[c] + (1.0 - m.f0[c]) * f5;
        return;
    }
    const double etap = front ? m.eta : 1.0 / m.eta;
    T ct;
    T F = fresnel_dielectric(ci, etap, ct);
    if ((float)val(u) < (float)val(F)) {
        wi = nn * (2.0 * ci) - wo;
        for (int c = 0; c < 3; ++c) weight[c] = T(1.0);
        return;
    }
    lobe = 1;
    wi = wo * (-1.0 / etap) + nn * (ci / etap - ct);
    for (int c = 0; c < 3; ++c) weight[c] = T(1.0 / (etap * etap));
}

// ----------------------------------------------------------------------------
// The path sampler f(u) (reading A1).  d = 4(L-1); block 0 = film; vertex j
// (1..L-1) uses light block (u[4j-2], u[4j-1]) and, for j <= L-2, BSDF block
// (u[4j], u[4j+1]).  Emission at the primary hit and at a vertex reached from
// a delta (specular) vertex; next-event estimation at every non-delta vertex;
// no MIS, no Russian roulette (readings A1, A24).
// ----------------------------------------------------------------------------
struct PathRec {
    // per vertex j = 1..L-1: triangle index (or -1), and light code
    // (light << 1 | contributed; at a delta vertex lobe << 1) or 0xFFFFFFFF
    // when the vertex does not exist
    int prim[32];
    uint32_t nee[32];
};

static const double LUM[3] = {0.2126, 0.7152, 0.0722};

template <class T>
static void path_eval(const Scene& S, int L, const T* u, PathRec& rec, bool replay, T f[3]) {
    for (int c = 0; c < 3; ++c) f[c] = T(0.0);
    if (!replay) {
        for (int j = 0; j < L - 1; ++j) { rec.prim[j] = -1; rec.nee[j] = 0xFFFFFFFFu; }
        // a point with a non-finite coordinate (a state that left the torus)
        // has f = 0: its tour is killed and regenerates
        if constexpr (std::is_same<T, double>::value)
            for (int i = 0; i < 4 * (L - 1); ++i)
                if (!std::isfinite(u[i])) return;
    }
    const int nl = (int)S.lights.size();

    // camera ray
    V3<T> o = lift<T>(S.eye);
    V3<T> dir = lift<T>(S.cw) + lift<T>(S.cu) * (2.0 * u[0] - 1.0) + lift<T>(S.cv) * (1.0 - 2.0 * u[1]);
    V3<T> d = normalize(dir);
    int prim;
    if (!replay) {
        prim = closest(S, vald(o), vald(d), S.tmin, INFINITY, nullptr);
        rec.prim[0] = prim;
    } else {
        prim = rec.prim[0];
    }
    if (prim < 0) return;
    T t;
    tri_hit<T>(S, prim, o, d, S.tmin, INFINITY, t, true);
    V3<T> x = o + d * t;
    V3<double> nw = cross(S.vert(prim, 1) - S.vert(prim, 0), S.vert(prim, 2) - S.vert(prim, 0));
    V3<double> ng = normalize(nw);
    double side = dot(ng, vald(d));
    V3<double> n = side > 0 ? ng * -1.0 : ng;
    bool front = !(side > 0);
    {
        const Material& m = S.mats[S.tmat[prim]];
        if (dot(nw, vald(d)) < 0.0)
            for (int c = 0; c < 3; ++c) f[c] = f[c] + m.Le[c];
    }
    T beta[3] = {T(1.0), T(1.0), T(1.0)};

    for (int j = 1; j <= L - 1; ++j) {
        const Material& m = S.mats[S.tmat[prim]];
        V3<T> wo = d * -1.0;
        // ---- next-event estimation at vertex j (none at a delta vertex:
        // its BSDF is zero for every light sample)
        if (!replay && is_delta(m)) rec.nee[j - 1] = 0;
        if (!is_delta(m)) {
            const T& a = u[4 * j - 2];
            const T& b = u[4 * j - 1];
            // light selection: FP32 decision, as on the device
            float sel = (float)val(a) * (float)nl;
            int li = (int)std::floor(sel);
            if (li > nl - 1) li = nl - 1;
            const Light& lt = S.lights[li];
            T ap = a * (double)nl - (double)li;
            V3<T> y = lift<T>(lt.p0) + lift<T>(lt.e1) * ap + lift<T>(lt.e2) * b;
            V3<T> w = y - x;
            T r2 = dot(w, w);
            T r = sqrt(r2);
            V3<T> wl = w * (1.0 / r);
            T cx = dot(lift<T>(n), wl);
            T cy = -dot(lift<T>(lt.n), wl);
            bool contrib;
            if (!replay) {
                // both cosines must clear 1e-6: a vertex lying in the light's own
                // plane gives cosines that are rounding noise around zero
                contrib = val(cx) > 1e-6 && val(cy) > 1e-6 &&
                          !occluded(S, vald(x), vald(wl), S.tmin, (1.0 - 1e-4) * val(r));
                rec.nee[j - 1] = ((uint32_t)li << 1) | (contrib ? 1u : 0u);
            } else {
                contrib = (rec.nee[j - 1] & 1u) != 0;
            }
            if (contrib) {
                T fs[3];
                bsdf_eval<T>(m, n, wo, wl, fs);
                T g = cx * cy / r2 * ((double)nl * lt.area);
                for (int c = 0; c < 3; ++c) f[c] = f[c] + beta[c] * fs[c] * g * lt.Le[c];
            }
        }
        if (j == L - 1) break;
        if (val(beta[0]) == 0.0 && val(beta[1]) == 0.0 && val(beta[2]) == 0.0) break;
        // ---- BSDF sampling and the next vertex
        V3<T> wi;
        T wgt[3];
        if (is_delta(m)) {
            int lobe;
            delta_sample<T>(m, n, front, wo, u[4 * j], wi, wgt, lobe);
            if (!replay) rec.nee[j - 1] = (uint32_t)lobe << 1;
        } else if (!bsdf_sample<T>(m, n, wo, u[4 * j], u[4 * j + 1], wi, wgt)) {
            break;
        }
        for (int c = 0; c < 3; ++c) beta[c] = beta[c] * wgt[c];
        int nprim;
        if (!replay) {
            nprim = closest(S, vald(x), vald(wi), S.tmin, INFINITY, nullptr);
            rec.prim[j] = nprim;
        } else {
            nprim = rec.prim[j];
        }
        if (nprim < 0) break;
        T tn;
        tri_hit<T>(S, nprim, x, wi, S.tmin, INFINITY, tn, true);
        x = x + wi * tn;
        d = wi;
        prim = nprim;
        V3<double> nw2 = cross(S.vert(prim, 1) - S.vert(prim, 0), S.vert(prim, 2) - S.vert(prim, 0));
        V3<double> ng2 = normalize(nw2);
        front = !(dot(ng2, vald(d)) > 0);
        n = front ? ng2 : ng2 * -1.0;
        // emission seen through a delta vertex (next-event estimation cannot
        // reach it): the emitter's radiance times the throughput
        if (is_delta(m) && dot(nw2, vald(d)) < 0.0) {
            const Material& me = S.mats[S.tmat[prim]];
            for (int c = 0; c < 3; ++c) f[c] = f[c] + beta[c] * me.Le[c];
        }
    }
}

// Condition measure of the score at one point: kappa[i] = a_i / (p + eps),
// the running magnitude of d p / d u_i (DualA) over the same taken path.
static void cond_point(const Scene& S, int L, const double* u, double eps, double* kappa) {
    const int d = 4 * (L - 1);
    g_nd = d;
    double f[3];
    PathRec rec;
    path_eval<double>(S, L, u, rec, false, f);  // the taken path, replayed below
    std::vector<DualA> ud(d);
    for (int i = 0; i < d; ++i) ud[i] = DualA::var(u[i], i);
    DualA fd[3];
    path_eval<DualA>(S, L, ud.data(), rec, true, fd);
    const DualA pd = LUM[0] * fd[0] + LUM[1] * fd[1] + LUM[2] * fd[2];
    for (int i = 0; i < d; ++i) kappa[i] = pd.a[i] / (pd.v + eps);
}

// f, p and optionally the score grad ln(p + eps) at one point.
static void eval_point(const Scene& S, int L, const double* u, double eps, double f[3], double& p, double* score,
                       PathRec& rec) {
    path_eval<double>(S, L, u, rec, false, f);
    p = LUM[0] * f[0] + LUM[1] * f[1] + LUM[2] * f[2];
    if (!score) return;
    const int d = 4 * (L - 1);
    g_nd = d;
    std::vector<Dual> ud(d);
    for (int i = 0; i < d; ++i) ud[i] = Dual::var(u[i], i);
    Dual fd[3];
    path_eval<Dual>(S, L, ud.data(), rec, true, fd);
    Dual pd = LUM[0] * fd[0] + LUM[1] * fd[1] + LUM[2] * fd[2];
    // a non-finite component (a measure-zero singularity of the sampler, e.g.
    // u = 0 in the cosine map) is set to zero so the chain stays on the torus
    for (int i = 0; i < d; ++i) {
        score[i] = pd.g[i] / (p + eps);
        if (!std::isfinite(score[i])) score[i] = 0.0;
    }
}

// ----------------------------------------------------------------------------
// Analytic target on the torus: p(x) = c0 + sum_j w_j N_wrap(x; m_j, s_j^2 I),
// f = p * g with g = (1, cos 2 pi x_0, sin 2 pi x_0, ..., cos 2 pi x_{d-1},
// sin 2 pi x_{d-1}).  Used only to pin the chain against closed forms.
// ----------------------------------------------------------------------------
struct Mixture {
    int d = 0;
    double c0 = 0;
    std::vector<double> w, m, s;  // modes: weight, mean (d each), std
    int nf() const { return 1 + 2 * d; }
    void eval(const double* x, double* fvec, double& p, double* grad) const {
        p = c0;
        std::vector<double> gp(d, 0.0);
        for (size_t j = 0; j < w.size(); ++j) {
            const double sj = s[j];
            double prod = w[j];
            std::vector<double> fac(d), dfac(d);
            for (int i = 0; i < d; ++i) {
                double acc = 0, dacc = 0;
                for (int k = -2; k <= 2; ++k) {
                    double z = x[i] - m[j * d + i] + k;
                    double e = std::exp(-z * z / (2 * sj * sj)) / (std::sqrt(2 * M_PI) * sj);
                    acc += e;
                    dacc += -z / (sj * sj) * e;
                }
                fac[i] = acc; dfac[i] = dacc;
                prod *= acc;
            }
            p += prod;
            if (grad)
                for (int i = 0; i < d; ++i) {
                    double q = w[j] * dfac[i];
                    for (int k = 0; k < d; ++k) if (k != i) q *= fac[k];
                    gp[i] += q;
                }
        }
        fvec[0] = p;
        for (int i = 0; i < d; ++i) {
            fvec[1 + 2 * i] = p * std::cos(2 * M_PI * x[i]);
            fvec[2 + 2 * i] = p * std::sin(2 * M_PI * x[i]);
        }
        if (grad) for (int i = 0; i < d; ++i) grad[i] = gp[i];
    }
};

// ----------------------------------------------------------------------------
// The Diffusion Restore chain ensemble.
// ----------------------------------------------------------------------------
struct Params {
    double stddev, dt, gamma, m, eps, k0;
    int rao_blackwell;
};

struct Chains {
    const Scene* scene = nullptr;
    const Mixture* mix = nullptr;
    int L = 0, d = 0, N = 0, nf = 3, nbucket = 1;
    Params P;
    uint64_t seed = 0, step = 0;
    double k0 = 0, p_lambda_hat = 0;
    std::vector<double> x, score, sigma;     // planar: [i * N + c]
    std::vector<uint32_t> killed, pixel, rec;
    std::vector<double> p, fop, w;
    std::vector<double> accum;
    uint64_t tour_count = 0, kills_step = 0;
    std::vector<double> xtrace;  // optional per-step trace of x
    std::vector<uint32_t> ids;   // RNG chain id of each slot (identity by default)
    uint32_t id(int c) const { return ids.empty() ? (uint32_t)c : ids[c]; }

    void evaluate(int c, const double* xc, double* fvec, double& pc, double* gr, uint32_t* rc) const {
        if (scene) {
            PathRec pr;
            eval_point(*scene, L, xc, P.eps, fvec, pc, gr, pr);
            for (int j = 0; j < L - 1; ++j) { rc[2 * j] = (uint32_t)pr.prim[j]; rc[2 * j + 1] = pr.nee[j]; }
        } else {
            mix->eval(xc, fvec, pc, gr);
            if (gr)
                for (int i = 0; i < d; ++i) {
                    gr[i] /= (pc + P.eps);
                    if (!std::isfinite(gr[i])) gr[i] = 0.0;
                }
        }
        (void)c;
    }
    // pixel index from x[0], x[1], taken in FP32 (reading A10)
    uint32_t pixel_of(const double* xc) const {
        if (!scene) return 0;
        const int W = scene->W, H = scene->H;
        float fx = (float)xc[0] * (float)W, fy = (float)xc[1] * (float)H;
        int px = (int)std::floor(fx), py = (int)std::floor(fy);
        if (px > W - 1) px = W - 1;
        if (py > H - 1) py = H - 1;
        if (px < 0) px = 0;
        if (py < 0) py = 0;
        return (uint32_t)(py * W + px);
    }
};

struct Tls {
    std::vector<double> accum;
    uint64_t tours = 0;
};

// Evaluate f, p at the chain's current x (Accumulate's first half).
static void chain_eval(Chains& C, int c, std::vector<double>& xc, std::vector<double>& fvec) {
    for (int i = 0; i < C.d; ++i) xc[i] = C.x[(size_t)i * C.N + c];
    double pc;
    std::vector<uint32_t> rc(2 * std::max(C.L - 1, 1));
    C.evaluate(c, xc.data(), fvec.data(), pc, nullptr, rc.data());
    C.p[c] = pc;
    for (int j = 0; j < 2 * (C.L - 1) && C.scene; ++j) C.rec[(size_t)j * C.N + c] = rc[j];
    C.pixel[c] = C.pixel_of(xc.data());
}

// Accumulate's second half: hold / kill, splat, and the score of survivors.
static void chain_accumulate(Chains& C, int c, uint64_t s, std::vector<double>& xc, std::vector<double>& fvec,
                             Tls& tls) {
    const double pc = C.p[c];
    // killing rate k = k0/(p + eps) (Eq. modified-killing-rate with uniform
    // regeneration); holding rate h = 1/dt.  Competing exponential clocks.
    const double Ea = expo(uniform(C.seed, C.id(c), s, TAG_HOLD, 0));
    const double Eb = expo(uniform(C.seed, C.id(c), s, TAG_HOLD, 1));
    const float kf = (float)C.k0 / ((float)pc + (float)C.P.eps);
    const bool alive = (kf * (float)C.P.dt) * (float)Ea < (float)Eb;  // FP32 decision
    const double k = C.k0 / (pc + C.P.eps);
    double w;
    if (C.P.rao_blackwell) w = 1.0 / (1.0 / C.P.dt + k);             // E[holding time | x] = 1/c(x)
    else w = std::min(Ea * C.P.dt, Eb / k);                          // sampled holding time
    C.w[c] = w;
    C.killed[c] = alive ? 0u : 1u;
    if (!alive) tls.tours += 1;
    const uint32_t pix = C.pixel[c];
    for (int q = 0; q < C.nf; ++q) C.fop[(size_t)q * C.N + c] = pc > 0 ? fvec[q] / pc : 0.0;
    if (pc > 0)
        for (int q = 0; q < C.nf; ++q) tls.accum[(size_t)pix * C.nf + q] += w * fvec[q] / pc;
    if (alive) {
        std::vector<double> gr(C.d), fv(C.nf);
        double p2;
        std::vector<uint32_t> rc(2 * std::max(C.L - 1, 1));
        C.evaluate(c, xc.data(), fv.data(), p2, gr.data(), rc.data());
        for (int i = 0; i < C.d; ++i) C.score[(size_t)i * C.N + c] = gr[i];
    } else {
        for (int i = 0; i < C.d; ++i) C.score[(size_t)i * C.N + c] = 0.0;
    }
}

// Regenerate from the uniform distribution on the torus.
static void chain_regen(Chains& C, int c, uint64_t s) {
    for (int i = 0; i < C.d; ++i) C.x[(size_t)i * C.N + c] = uniform(C.seed, C.id(c), s, TAG_REGEN, i);
}

// Euler-Maruyama step with rotational drift, wrapped to the torus (Alg. 5.1).
static void chain_move(Chains& C, int c, uint64_t s) {
    const double gt = C.P.dt * C.P.gamma / 2.0;  // gamma tilde
    for (int i = 0; i < C.d / 2; ++i) {
        double xi[2];
        box_muller(uniform(C.seed, C.id(c), s, TAG_GAUSS, 2 * i), uniform(C.seed, C.id(c), s, TAG_GAUSS, 2 * i + 1),
                   xi[0], xi[1]);
        const size_t i0 = (size_t)(2 * i) * C.N + c, i1 = (size_t)(2 * i + 1) * C.N + c;
        const double s0 = C.score[i0], s1 = C.score[i1];
        const double rot[2] = {gt * s1, -gt * s0};
        const double sc[2] = {s0, s1};
        const size_t ii[2] = {i0, i1};
        for (int k = 0; k < 2; ++k) {
            const double sd = C.sigma.empty() ? C.P.stddev : C.sigma[ii[k]];
            double y = C.x[ii[k]] + 0.5 * sd * sd * sc[k] + rot[k] + sd * xi[k];
            y -= std::floor(y);
            if (y >= 1.0) y = 0.0;  // torus identification of 1 with 0
            C.x[ii[k]] = y;
        }
    }
}

template <class F>
static void parallel_chains(int N, int nthreads, F&& fn) {
    nthreads = std::max(1, std::min(nthreads, N));
    if (nthreads == 1) { fn(0, 0, N); return; }
    std::vector<std::thread> th;
    for (int t = 0; t < nthreads; ++t) {
        int b = (int)((int64_t)N * t / nthreads), e = (int)((int64_t)N * (t + 1) / nthreads);
        th.emplace_back([&, t, b, e] { fn(t, b, e); });
    }
    for (auto& x : th) x.join();
}

static void reduce_tls(Chains& C, std::vector<Tls>& tls) {
    for (auto& t : tls) {  // fixed thread order => deterministic for a given thread count
        for (size_t i = 0; i < C.accum.size(); ++i) C.accum[i] += t.accum[i];
        C.tour_count += t.tours;
    }
}

static void chains_init(Chains& C, uint32_t frame, int nthreads) {
    const uint64_t s = (uint64_t)frame << 32;
    std::fill(C.accum.begin(), C.accum.end(), 0.0);
    C.tour_count = 0;
    // phase 1: x ~ mu and f(x) for every chain
    parallel_chains(C.N, nthreads, [&](int, int b, int e) {
        std::vector<double> xc(C.d), fv(C.nf);
        for (int c = b; c < e; ++c) {
            chain_regen(C, c, s);
            chain_eval(C, c, xc, fv);
        }
    });
    // p_lambda estimate and k0 (Eq. killing-rate-constant), unless given
    if (C.P.k0 > 0) {
        C.k0 = C.P.k0;
    } else {
        double sum = 0;
        for (int c = 0; c < C.N; ++c) sum += C.p[c];
        C.p_lambda_hat = sum / C.N;
        C.k0 = C.p_lambda_hat > 0 ? C.p_lambda_hat / (C.P.m * C.P.dt) : C.P.eps / (C.P.m * C.P.dt);
    }
    // phase 2: hold / kill / splat with that k0
    std::vector<Tls> tls(std::max(1, std::min(nthreads, C.N)));
    for (auto& t : tls) t.accum.assign(C.accum.size(), 0.0);
    parallel_chains(C.N, nthreads, [&](int ti, int b, int e) {
        std::vector<double> xc(C.d), fv(C.nf);
        for (int c = b; c < e; ++c) {
            chain_eval(C, c, xc, fv);  // re-evaluate (cheap, deterministic) to recover f
            chain_accumulate(C, c, s, xc, fv, tls[ti]);
        }
    });
    reduce_tls(C, tls);
    C.step = s + 1;
}

static void chains_step(Chains& C, int nsteps, int nthreads, double* xtrace) {
    for (int k = 0; k < nsteps; ++k) {
        const uint64_t s = C.step;
        std::vector<Tls> tls(std::max(1, std::min(nthreads, C.N)));
        for (auto& t : tls) t.accum.assign(C.accum.size(), 0.0);
        parallel_chains(C.N, nthreads, [&](int ti, int b, int e) {
            std::vector<double> xc(C.d), fv(C.nf);
            for (int c = b; c < e; ++c) {
                if (C.killed[c]) chain_regen(C, c, s);     // Alg. 4.2: regenerate killed tours
                else chain_move(C, c, s);                  // Alg. 4.2: local dynamics
                chain_eval(C, c, xc, fv);
                chain_accumulate(C, c, s, xc, fv, tls[ti]);
            }
        });
        reduce_tls(C, tls);
        if (xtrace) std::memcpy(xtrace + (size_t)k * C.d * C.N, C.x.data(), sizeof(double) * C.d * C.N);
        C.step = s + 1;
    }
}

}  // namespace orc

// ============================================================================
// C interface (ctypes)
// ============================================================================
using namespace orc;

extern "C" {

void orc_philox(const uint32_t* ctr, const uint32_t* key, uint32_t* out) { philox4x32_10(ctr, key, out); }

double orc_uniform(uint64_t seed, uint32_t chain, uint64_t step, uint32_t tag, uint32_t i) {
    return uniform(seed, chain, step, tag, i);
}

void orc_box_muller(double u0, double u1, double* z) { box_muller(u0, u1, z[0], z[1]); }

// materials: nm x 12 floats (kind, albedo[3], roughness, f0[3], Le[3], eta)
// lights:    nl x 12 floats (p0[3], e1[3], e2[3], Le[3])
// camera:    10 floats (eye[3], at[3], up[3], vfov_deg)
// One material from its 12 floats (kind, albedo[3], roughness, f0[3], Le[3], eta).
static Material mat_from(const float* q) {
    Material m;
    m.kind = (int)q[0];
    for (int c = 0; c < 3; ++c) { m.albedo[c] = q[1 + c]; m.f0[c] = q[5 + c]; m.Le[c] = q[8 + c]; }
    m.rough = q[4];
    m.eta = q[11];
    return m;
}

void* orc_scene_new(const float* V, int nv, const uint32_t* I, int nt, const uint32_t* tmat, const float* mats, int nm,
                    const float* lights, int nl, const float* cam, int W, int H, int brute) {
    auto* S = new Scene();
    S->v.resize(nv);
    for (int i = 0; i < nv; ++i) S->v[i] = {(double)V[3 * i], (double)V[3 * i + 1], (double)V[3 * i + 2]};
    S->idx.assign(I, I + 3 * (size_t)nt);
    S->tmat.assign(tmat, tmat + nt);
    for (int i = 0; i < nm; ++i) {
        S->mats.push_back(mat_from(mats + 12 * i));
    }
    for (int i = 0; i < nl; ++i) {
        const float* q = lights + 12 * i;
        Light l;
        l.p0 = {q[0], q[1], q[2]};
        l.e1 = {q[3], q[4], q[5]};
        l.e2 = {q[6], q[7], q[8]};
        for (int c = 0; c < 3; ++c) l.Le[c] = q[9 + c];
        V3<double> nn = cross(l.e1, l.e2);
        l.area = std::sqrt(dot(nn, nn));
        l.n = nn * (1.0 / l.area);
        S->lights.push_back(l);
    }
    V3<double> eye = {cam[0], cam[1], cam[2]}, at = {cam[3], cam[4], cam[5]}, up = {cam[6], cam[7], cam[8]};
    const double th = std::tan(0.5 * (double)cam[9] * M_PI / 180.0);
    const double aspect = (double)W / (double)H;
    V3<double> w = normalize(eye - at);
    V3<double> uu = normalize(cross(up, w));
    V3<double> vv = cross(w, uu);
    S->eye = eye;
    S->cu = uu * (th * aspect);
    S->cv = vv * th;
    S->cw = w * -1.0;
    S->W = W; S->H = H;
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (auto& p : S->v) {
        double c[3] = {p.x, p.y, p.z};
        for (int a = 0; a < 3; ++a) { lo[a] = std::min(lo[a], c[a]); hi[a] = std::max(hi[a], c[a]); }
    }
    double diag = std::sqrt((hi[0] - lo[0]) * (hi[0] - lo[0]) + (hi[1] - lo[1]) * (hi[1] - lo[1]) + (hi[2] - lo[2]) * (hi[2] - lo[2]));
    S->tmin = 1e-4 * diag;
    S->brute = brute != 0;
    S->order.resize(nt);
    for (int i = 0; i < nt; ++i) S->order[i] = i;
    if (nt > 0) bvh_build(*S, 0, nt);
    return S;
}

void orc_scene_free(void* s) { delete (Scene*)s; }
double orc_scene_tmin(void* s) { return ((Scene*)s)->tmin; }
void orc_scene_set_brute(void* s, int brute) { ((Scene*)s)->brute = brute != 0; }

// Closest hit / occlusion queries for n rays (o, d: n x 3).
void orc_trace(void* s, int n, const double* o, const double* d, double tmax, int* prim, double* t) {
    Scene* S = (Scene*)s;
    for (int i = 0; i < n; ++i) {
        V3<double> oo = {o[3 * i], o[3 * i + 1], o[3 * i + 2]}, dd = {d[3 * i], d[3 * i + 1], d[3 * i + 2]};
        prim[i] = closest(*S, oo, dd, S->tmin, tmax, &t[i]);
    }
}
void orc_occluded(void* s, int n, const double* o, const double* d, const double* tmax, int* hit) {
    Scene* S = (Scene*)s;
    for (int i = 0; i < n; ++i) {
        V3<double> oo = {o[3 * i], o[3 * i + 1], o[3 * i + 2]}, dd = {d[3 * i], d[3 * i + 1], d[3 * i + 2]};
        hit[i] = occluded(*S, oo, dd, S->tmin, tmax[i]) ? 1 : 0;
    }
}

// f(u), p(u) and optionally score = grad ln(p + eps) and the path record for
// n points u (n x d, d = 4(L-1)).  rec: n x 2(L-1) (triangle, light code).
void orc_path_eval(void* s, int L, int n, const double* u, double eps, double* f, double* p, double* score,
                   uint32_t* rec, int nthreads) {
    Scene* S = (Scene*)s;
    const int d = 4 * (L - 1);
    parallel_chains(n, nthreads, [&](int, int b, int e) {
        for (int i = b; i < e; ++i) {
            PathRec pr;
            double pp;
            eval_point(*S, L, u + (size_t)i * d, eps, f + 3 * (size_t)i, pp, score ? score + (size_t)i * d : nullptr, pr);
            p[i] = pp;
            if (rec)
                for (int j = 0; j < L - 1; ++j) {
                    rec[(size_t)i * 2 * (L - 1) + 2 * j] = (uint32_t)pr.prim[j];
                    rec[(size_t)i * 2 * (L - 1) + 2 * j + 1] = pr.nee[j];
                }
        }
    });
}

void orc_path_cond(void* s, int L, int n, const double* u, double eps, double* kappa, int nthreads) {
    Scene* S = (Scene*)s;
    const int d = 4 * (L - 1);
    parallel_chains(n, nthreads, [&](int, int b, int e) {
        for (int i = b; i < e; ++i) cond_point(*S, L, u + (size_t)i * d, eps, kappa + (size_t)i * d);
    });
}

int orc_bsdf_sample(const float* mat, const double* n, const double* wo, double u, double v, double* wi,
                    double* weight) {
    Material m = mat_from(mat);
    V3<double> nn = {n[0], n[1], n[2]}, o = {wo[0], wo[1], wo[2]}, w;
    double wt[3];
    bool ok = bsdf_sample<double>(m, nn, o, u, v, w, wt);
    wi[0] = w.x; wi[1] = w.y; wi[2] = w.z;
    for (int c = 0; c < 3; ++c) weight[c] = ok ? wt[c] : 0.0;
    return ok ? 1 : 0;
}
// Delta lobe sample (mat: a smooth conductor or dielectric); returns the lobe.
int orc_delta_sample(const float* mat, const double* n, int front, const double* wo, double u, double* wi,
                     double* weight) {
    Material m = mat_from(mat);
    V3<double> nn = {n[0], n[1], n[2]}, o = {wo[0], wo[1], wo[2]}, w;
    int lobe;
    delta_sample<double>(m, nn, front != 0, o, u, w, weight, lobe);
    wi[0] = w.x; wi[1] = w.y; wi[2] = w.z;
    return lobe;
}
double orc_fresnel_dielectric(double ci, double etap) {
    double ct;
    return fresnel_dielectric<double>(ci, etap, ct);
}
void orc_bsdf_eval(const float* mat, const double* n, const double* wo, const double* wi, double* fs) {
    Material m = mat_from(mat);
    V3<double> nn = {n[0], n[1], n[2]}, o = {wo[0], wo[1], wo[2]}, i = {wi[0], wi[1], wi[2]};
    bsdf_eval<double>(m, nn, o, i, fs);
}
// Batched forms: count samples (u, v) or directions wi (count x 3).
void orc_bsdf_sample_n(const float* mat, const double* n, const double* wo, int count, const double* u,
                       const double* v, double* wi, double* weight, int* ok) {
    for (int i = 0; i < count; ++i) ok[i] = orc_bsdf_sample(mat, n, wo, u[i], v[i], wi + 3 * i, weight + 3 * i);
}
void orc_bsdf_eval_n(const float* mat, const double* n, const double* wo, int count, const double* wi, double* fs) {
    for (int i = 0; i < count; ++i) orc_bsdf_eval(mat, n, wo, wi + 3 * i, fs + 3 * i);
}
// GGX distribution D(cos theta_h) and Smith masking G1(cos theta) for alpha.
double orc_ggx_d(double ch, double alpha) { return ggx_d<double>(ch, alpha * alpha); }
double orc_smith_g1(double c, double alpha) { return smith_g1<double>(c, alpha); }

void orc_onb(const double* n, double* t, double* b) {
    V3<double> tt, bb;
    onb({n[0], n[1], n[2]}, tt, bb);
    t[0] = tt.x; t[1] = tt.y; t[2] = tt.z;
    b[0] = bb.x; b[1] = bb.y; b[2] = bb.z;
}

// params: stddev, dt, gamma, m, eps, k0, rao_blackwell
static Params params_from(const double* q) {
    Params P;
    P.stddev = q[0]; P.dt = q[1]; P.gamma = q[2]; P.m = q[3]; P.eps = q[4]; P.k0 = q[5];
    P.rao_blackwell = (int)q[6];
    return P;
}
static void alloc_chains(Chains* C) {
    const size_t N = C->N;
    C->x.assign((size_t)C->d * N, 0.0);
    C->score.assign((size_t)C->d * N, 0.0);
    C->killed.assign(N, 1u);
    C->pixel.assign(N, 0u);
    C->p.assign(N, 0.0);
    C->w.assign(N, 0.0);
    C->fop.assign((size_t)C->nf * N, 0.0);
    C->rec.assign((size_t)2 * std::max(C->L - 1, 1) * N, 0u);
    C->accum.assign((size_t)C->nbucket * C->nf, 0.0);
}

void* orc_chains_new_scene(void* scene, int L, int n_chains, const double* params, uint64_t seed, const float* sigma) {
    auto* C = new Chains();
    C->scene = (Scene*)scene;
    C->L = L; C->d = 4 * (L - 1); C->N = n_chains; C->nf = 3;
    C->nbucket = C->scene->W * C->scene->H;
    C->P = params_from(params);
    C->seed = seed;
    alloc_chains(C);
    if (sigma) C->sigma.assign(sigma, sigma + (size_t)C->d * n_chains);
    return C;
}

// modes: nm weights, nm*d means, nm stds
void* orc_chains_new_mixture(int d, int nm, const double* w, const double* means, const double* stds, double c0,
                             int n_chains, const double* params, uint64_t seed) {
    auto* M = new Mixture();
    M->d = d; M->c0 = c0;
    M->w.assign(w, w + nm); M->m.assign(means, means + (size_t)nm * d); M->s.assign(stds, stds + nm);
    auto* C = new Chains();
    C->mix = M;
    C->L = 0; C->d = d; C->N = n_chains; C->nf = M->nf(); C->nbucket = 1;
    C->P = params_from(params);
    C->seed = seed;
    alloc_chains(C);
    return C;
}

// Give every chain its own diagonal stddev (d x N planar), as for a scene's
// chains (reading A16).
void orc_chains_set_sigma(void* c, const float* sigma) {
    Chains* C = (Chains*)c;
    if (sigma) C->sigma.assign(sigma, sigma + (size_t)C->d * C->N);
    else C->sigma.clear();
}

void orc_chains_free(void* c) {
    Chains* C = (Chains*)c;
    delete C->mix;
    delete C;
}

void orc_chains_init(void* c, uint32_t frame, int nthreads) { chains_init(*(Chains*)c, frame, nthreads); }
void orc_chains_step(void* c, int nsteps, int nthreads, double* xtrace) { chains_step(*(Chains*)c, nsteps, nthreads, xtrace); }

// Overwrite the chain state (x, score: d x N planar, killed: N) and the step
// counter; k0 > 0 also sets the killing constant.
void orc_chains_set_state(void* c, const float* x, const float* score, const uint32_t* killed, uint64_t step, double k0) {
    Chains* C = (Chains*)c;
    for (size_t i = 0; i < C->x.size(); ++i) { C->x[i] = x[i]; C->score[i] = score[i]; }
    for (int i = 0; i < C->N; ++i) C->killed[i] = killed[i];
    C->step = step;
    if (k0 > 0) C->k0 = k0;
}

// Give slot c the generator chain id ids[c] (to evaluate a sample of a larger
// ensemble's chains).
void orc_chains_set_ids(void* c, const uint32_t* ids) {
    Chains* C = (Chains*)c;
    C->ids.assign(ids, ids + C->N);
}

// Read the chain state and the last step's per-chain record.
void orc_chains_get_state(void* c, double* x, double* score, uint32_t* killed, double* p, uint32_t* pixel, double* fop,
                          double* w, uint32_t* rec) {
    Chains* C = (Chains*)c;
    if (x) std::memcpy(x, C->x.data(), sizeof(double) * C->x.size());
    if (score) std::memcpy(score, C->score.data(), sizeof(double) * C->score.size());
    if (killed) std::memcpy(killed, C->killed.data(), sizeof(uint32_t) * C->N);
    if (p) std::memcpy(p, C->p.data(), sizeof(double) * C->N);
    if (pixel) std::memcpy(pixel, C->pixel.data(), sizeof(uint32_t) * C->N);
    if (fop) std::memcpy(fop, C->fop.data(), sizeof(double) * C->fop.size());
    if (w) std::memcpy(w, C->w.data(), sizeof(double) * C->N);
    if (rec) std::memcpy(rec, C->rec.data(), sizeof(uint32_t) * C->rec.size());
}

// accum (nbucket x nf), tour count, k0, p_lambda estimate, step
void orc_chains_accum(void* c, double* accum, uint64_t* tours, double* k0, double* plam, uint64_t* step) {
    Chains* C = (Chains*)c;
    if (accum) std::memcpy(accum, C->accum.data(), sizeof(double) * C->accum.size());
    if (tours) *tours = C->tour_count;
    if (k0) *k0 = C->k0;
    if (plam) *plam = C->p_lambda_hat;
    if (step) *step = C->step;
}

// Resolve (Alg. 4.3, reading A9): image = W H k0 accum / tourCount, planar 3 x W H.
void orc_chains_resolve(void* c, double* img) {
    Chains* C = (Chains*)c;
    const size_t npx = C->nbucket;
    const double scale = C->tour_count > 0 ? (double)npx * C->k0 / (double)C->tour_count : 0.0;
    for (size_t px = 0; px < npx; ++px)
        for (int q = 0; q < C->nf; ++q) img[(size_t)q * npx + px] = scale * C->accum[px * C->nf + q];
}

// Independent path tracing reference: spp stratified-by-pixel samples per
// pixel, u0 = (px + U)/W, u1 = (py + U)/H, other coordinates U.
void orc_pt_render(void* s, int L, uint64_t seed, int spp, int nthreads, double* img) {
    Scene* S = (Scene*)s;
    const int W = S->W, H = S->H, d = 4 * (L - 1);
    parallel_chains(W * H, nthreads, [&](int, int b, int e) {
        std::vector<double> u(d);
        for (int pix = b; pix < e; ++pix) {
            const int px = pix % W, py = pix / W;
            double acc[3] = {0, 0, 0};
            for (int k = 0; k < spp; ++k) {
                for (int i = 0; i < d; ++i) u[i] = uniform(seed, (uint32_t)pix, (uint64_t)k, TAG_PT, i);
                u[0] = (px + u[0]) / W;
                u[1] = (py + u[1]) / H;
                PathRec pr;
                double f[3];
                path_eval<double>(*S, L, u.data(), pr, false, f);
                for (int c = 0; c < 3; ++c) acc[c] += f[c];
            }
            for (int c = 0; c < 3; ++c) img[(size_t)c * W * H + pix] = acc[c] / spp;
        }
    });
}

}  // extern "C"
