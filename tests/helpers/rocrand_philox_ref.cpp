// Prints rocRAND's Philox4x32-10 block for (seed, subsequence, offset) given on
// stdin, one triple per line.  rocRAND keys the generator with the 64-bit seed
// and places the subsequence in counter words 2-3 and offset/4 in words 0-1,
// so its first block is Philox4x32-10(counter, key) for that counter.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>

int main() {
    unsigned long long seed, sub, off;
    while (std::scanf("%llu %llu %llu", &seed, &sub, &off) == 3) {
        rocrand_state_philox4x32_10 st;
        rocrand_init(seed, sub, off, &st);
        uint4 r = rocrand4(&st);
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
