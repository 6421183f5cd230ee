// arena_sim.cpp -- CPU check of the server's arena (test infrastructure;
// built by tests/test_server_host.py).  Random allocations and frees against
// a brute-force map of the region: no two live blocks overlap, every block is
// aligned and inside the region, the used count is exact, freeing everything
// merges the region back into one free block, and an allocation fails only
// when no free block is large enough.
#include <stdio.h>
#include <stdlib.h>

#include <random>
#include <vector>

#include "../paper_1406_5597_amd/csrc/fft3d_arena.hpp"

int main(int argc, char** argv)
{
    const unsigned seed = argc > 1 ? (unsigned)atoi(argv[1]) : 1;
    const size_t region = (size_t)1 << 24;
    fft3d::Arena a;
    a.reset(region);
    std::mt19937_64 rng(seed);
    struct Blk {
        size_t off, n;
    };
    std::vector<Blk> live;
    std::vector<unsigned char> map(region / fft3d::Arena::kAlign, 0);
    size_t used = 0;
    for (int step = 0; step < 200000; ++step) {
        const bool do_alloc = live.empty() || (rng() % 100) < 55;
        if (do_alloc) {
            const size_t n = 1 + rng() % (rng() % 8 == 0 ? region / 8 : 65536);
            size_t off;
            if (a.alloc(n, &off)) {
                const size_t r = fft3d::Arena::round(n);
                if (off % fft3d::Arena::kAlign || off + r > region) {
                    printf("FAIL: block outside the region or misaligned\n");
                    return 1;
                }
                for (size_t g = off / fft3d::Arena::kAlign; g < (off + r) / fft3d::Arena::kAlign; ++g) {
                    if (map[g]) {
                        printf("FAIL: overlapping blocks\n");
                        return 1;
                    }
                    map[g] = 1;
                }
                live.push_back({off, n});
                used += r;
            } else if (a.largest_free() >= fft3d::Arena::round(n)) {
                printf("FAIL: allocation refused with a large enough free block\n");
                return 1;
            }
        } else {
            const size_t i = rng() % live.size();
            const Blk b = live[i];
            live[i] = live.back();
            live.pop_back();
            const size_t r = fft3d::Arena::round(b.n);
            for (size_t g = b.off / fft3d::Arena::kAlign; g < (b.off + r) / fft3d::Arena::kAlign; ++g) map[g] = 0;
            a.free(b.off, b.n);
            used -= r;
        }
        if (a.used() != used) {
            printf("FAIL: used count\n");
            return 1;
        }
    }
    for (const Blk& b : live) a.free(b.off, b.n);
    if (a.used() != 0 || a.free_blocks() != 1 || a.largest_free() != region) {
        printf("FAIL: the region did not merge back (%zu blocks)\n", a.free_blocks());
        return 1;
    }
    printf("ok\n");
    return 0;
}
