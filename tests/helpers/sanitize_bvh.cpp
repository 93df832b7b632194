// Driver for an AddressSanitizer/UndefinedBehaviorSanitizer build of the
// library's host BVH builder (bvh_build.cpp, host code only, built with g++).
// Builds trees over a triangle soup written by tests/test_sanitizers.py with
// every leaf size, plus degenerate inputs (all triangles at one point, a
// single triangle) and the rejected cases (index out of range, empty input).
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../include/dr.h"

extern "C" dr_status dr_bvh_build_impl(const float* vertices, uint32_t n_vertices, const uint32_t* indices,
                                       uint32_t n_triangles, uint32_t max_leaf, dr_bvh_node* nodes_out,
                                       uint32_t* n_nodes_out, uint32_t* prim_order_out, const char** err);

static int build(const std::vector<float>& V, const std::vector<uint32_t>& I, uint32_t max_leaf, bool expect_ok) {
    const uint32_t nt = (uint32_t)(I.size() / 3);
    std::vector<dr_bvh_node> nodes(2 * (size_t)(nt ? nt : 1));
    std::vector<uint32_t> order(nt ? nt : 1);
    uint32_t nn = 0;
    const char* err = "";
    const dr_status s = dr_bvh_build_impl(V.data(), (uint32_t)(V.size() / 3), I.data(), nt, max_leaf, nodes.data(), &nn,
                                          order.data(), &err);
    if ((s == DR_OK) != expect_ok) {
        std::fprintf(stderr, "unexpected status %d (%s)\n", (int)s, err);
        return 1;
    }
    return 0;
}

int main(int argc, char** argv) {
    if (argc != 4) { std::fprintf(stderr, "usage: dir nv nt\n"); return 2; }
    char path[4096];
    const int nv = std::atoi(argv[2]), nt = std::atoi(argv[3]);
    std::vector<float> V(3 * (size_t)nv);
    std::vector<uint32_t> I(3 * (size_t)nt);
    std::snprintf(path, sizeof(path), "%s/V.bin", argv[1]);
    FILE* f = std::fopen(path, "rb");
    if (!f || std::fread(V.data(), 4, V.size(), f) != V.size()) return 2;
    std::fclose(f);
    std::snprintf(path, sizeof(path), "%s/I.bin", argv[1]);
    f = std::fopen(path, "rb");
    if (!f || std::fread(I.data(), 4, I.size(), f) != I.size()) return 2;
    std::fclose(f);
    int bad = 0;
    for (uint32_t leaf : {1u, 2u, 4u, 16u}) bad += build(V, I, leaf, true);
    std::vector<float> point(9, 0.5f);  // three coincident vertices
    std::vector<uint32_t> same;
    for (int t = 0; t < 1000; ++t) same.insert(same.end(), {0u, 1u, 2u});
    bad += build(point, same, 2, true);
    bad += build(point, std::vector<uint32_t>{0u, 1u, 2u}, 2, true);
    bad += build(point, std::vector<uint32_t>{0u, 1u, 3u}, 2, false);  // index out of range
    bad += build(point, std::vector<uint32_t>{}, 2, false);            // empty
    if (bad) return 1;
    std::printf("sanitized bvh run ok\n");
    return 0;
}
