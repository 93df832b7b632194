// Driver for an AddressSanitizer/UndefinedBehaviorSanitizer build of the CPU
// oracle (host code only, built with g++).  Reads a scene written by
// tests/test_sanitizers.py and exercises the oracle's entry points: scene
// construction and its BVH, path evaluation with the score, chains (init,
// steps, state, accumulators, resolve), per-chain Sigma, the mixture target
// and path tracing.  Any sanitizer report makes the process exit non-zero.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

extern "C" {
void* orc_scene_new(const float* V, int nv, const uint32_t* I, int nt, const uint32_t* tmat, const float* mats, int nm,
                    const float* lights, int nl, const float* cam, int W, int H, int brute);
void orc_scene_free(void* s);
void orc_path_eval(void* s, int L, int n, const double* u, double eps, double* f, double* p, double* score,
                   uint32_t* rec, int nthreads);
void* orc_chains_new_scene(void* scene, int L, int n_chains, const double* params, uint64_t seed, const float* sigma);
void* orc_chains_new_mixture(int d, int nm, const double* w, const double* means, const double* stds, double c0,
                             int n_chains, const double* params, uint64_t seed);
void orc_chains_free(void* c);
void orc_chains_init(void* c, uint32_t frame, int nthreads);
void orc_chains_step(void* c, int nsteps, int nthreads, double* xtrace);
void orc_chains_get_state(void* c, double* x, double* score, uint32_t* killed, double* p, uint32_t* pixel, double* fop,
                          double* w, uint32_t* rec);
void orc_chains_accum(void* c, double* accum, uint64_t* tours, double* k0, double* plam, uint64_t* step);
void orc_chains_resolve(void* c, double* img);
void orc_pt_render(void* s, int L, uint64_t seed, int spp, int nthreads, double* img);
}

template <class T>
static std::vector<T> read_file(const char* dir, const char* name, size_t count) {
    char path[4096];
    std::snprintf(path, sizeof(path), "%s/%s", dir, name);
    FILE* f = std::fopen(path, "rb");
    if (!f) { std::fprintf(stderr, "cannot open %s\n", path); std::exit(2); }
    std::vector<T> v(count);
    if (std::fread(v.data(), sizeof(T), count, f) != count) { std::fprintf(stderr, "short read %s\n", path); std::exit(2); }
    std::fclose(f);
    return v;
}

int main(int argc, char** argv) {
    if (argc != 9) { std::fprintf(stderr, "usage: dir nv nt nm nl W H L\n"); return 2; }
    const char* dir = argv[1];
    const int nv = std::atoi(argv[2]), nt = std::atoi(argv[3]), nm = std::atoi(argv[4]), nl = std::atoi(argv[5]);
    const int W = std::atoi(argv[6]), H = std::atoi(argv[7]), L = std::atoi(argv[8]);
    const auto V = read_file<float>(dir, "V.bin", 3 * (size_t)nv);
    const auto I = read_file<uint32_t>(dir, "I.bin", 3 * (size_t)nt);
    const auto TM = read_file<uint32_t>(dir, "TM.bin", nt);
    const auto M = read_file<float>(dir, "M.bin", 12 * (size_t)nm);
    const auto Lt = read_file<float>(dir, "Lt.bin", 12 * (size_t)nl);
    const auto cam = read_file<float>(dir, "cam.bin", 10);
    const int d = 4 * (L - 1), n = 257;
    void* S = orc_scene_new(V.data(), nv, I.data(), nt, TM.data(), M.data(), nm, Lt.data(), nl, cam.data(), W, H, 0);
    std::vector<double> u((size_t)n * d);
    uint64_t z = 88172645463325252ull;  // xorshift64 points on the torus
    for (double& x : u) {
        z ^= z << 13; z ^= z >> 7; z ^= z << 17;
        x = (double)(z >> 40) / 16777216.0;
    }
    std::vector<double> f(3 * (size_t)n), p(n), score((size_t)n * d);
    std::vector<uint32_t> rec((size_t)n * 2 * (L - 1));
    orc_path_eval(S, L, n, u.data(), 1e-8, f.data(), p.data(), score.data(), rec.data(), 2);
    // params: stddev, dt, gamma, m, eps, k0, rao_blackwell
    const double prm[7] = {5e-3, 1e-5, 0.5, 64.0, 1e-8, 0.0, 1.0};
    const int N = 96;
    std::vector<float> sigma((size_t)d * N, 4e-3f);
    for (int with_sigma = 0; with_sigma < 2; ++with_sigma) {
        void* Ch = orc_chains_new_scene(S, L, N, prm, 7, with_sigma ? sigma.data() : nullptr);
        orc_chains_init(Ch, 1, 2);
        std::vector<double> tr(3 * (size_t)d * N);
        orc_chains_step(Ch, 3, 2, tr.data());
        orc_chains_step(Ch, 5, 1, nullptr);
        std::vector<double> x((size_t)d * N), sc((size_t)d * N), pp(N), fop(3 * (size_t)N), w(N);
        std::vector<uint32_t> killed(N), pix(N), r((size_t)2 * (L - 1) * N);
        orc_chains_get_state(Ch, x.data(), sc.data(), killed.data(), pp.data(), pix.data(), fop.data(), w.data(), r.data());
        std::vector<double> acc(3 * (size_t)W * H), img(3 * (size_t)W * H);
        uint64_t tours = 0, step = 0;
        double k0 = 0, pl = 0;
        orc_chains_accum(Ch, acc.data(), &tours, &k0, &pl, &step);
        orc_chains_resolve(Ch, img.data());
        orc_chains_free(Ch);
    }
    {
        const double w[2] = {0.6, 0.4}, means[16] = {0.2, 0.3, 0.4, 0.5, 0.6, 0.7, 0.8, 0.9,
                                                     0.7, 0.1, 0.9, 0.3, 0.5, 0.2, 0.4, 0.6};
        const double stds[2] = {0.05, 0.03};
        void* Mx = orc_chains_new_mixture(8, 2, w, means, stds, 0.1, 64, prm, 3);
        orc_chains_init(Mx, 0, 2);
        orc_chains_step(Mx, 20, 2, nullptr);
        std::vector<double> acc(1 + 2 * 8);  // one bucket of 1 + 2d test functions
        uint64_t tours = 0, step = 0;
        double k0 = 0, pl = 0;
        orc_chains_accum(Mx, acc.data(), &tours, &k0, &pl, &step);
        orc_chains_free(Mx);
    }
    std::vector<double> pt(3 * (size_t)W * H);
    orc_pt_render(S, L, 5, 1, 2, pt.data());
    orc_scene_free(S);
    std::printf("sanitized oracle run ok\n");
    return 0;
}
