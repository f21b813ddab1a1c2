// Randomised check of the first-fit arena (csrc/arena.h) against a byte map:
// every allocation lies inside the arena, is 256-byte aligned and overlaps no
// live allocation; releases merge neighbours (an emptied arena is one range);
// a request fails only when no free range of that size exists.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "arena.h"

int main(int argc, char **argv)
{
    const unsigned seed = argc > 1 ? (unsigned)atoi(argv[1]) : 1u;
    const size_t cap = 1 << 20;
    lbm_arena::Arena a(cap + 100);  // capacity rounds down to 256 bytes
    if (a.capacity() != cap) return printf("capacity %zu\n", a.capacity()), 1;
    std::vector<int> owner(cap / 256, -1);
    struct Live { size_t off, bytes; };
    std::vector<Live> live;
    std::mt19937_64 rng(seed);
    size_t used = 0;
    for (int it = 0; it < 20000; ++it) {
        if (live.empty() || rng() % 100 < 55) {
            const size_t bytes = 1 + rng() % (rng() % 4 == 0 ? 200000 : 5000);
            size_t off;
            const size_t blocks = (bytes + 255) / 256;
            bool exists = false;  // a run of `blocks` free blocks somewhere?
            for (size_t b = 0, run = 0; b < owner.size() && !exists; ++b) {
                run = owner[b] < 0 ? run + 1 : 0;
                exists = run >= blocks;
            }
            if (!a.alloc(bytes, &off)) {
                if (exists) return printf("alloc of %zu failed with room\n", bytes), 1;
                continue;
            }
            if (!exists) return printf("alloc succeeded without room\n"), 1;
            if (off % 256 || off + blocks * 256 > cap) return printf("bad range\n"), 1;
            for (size_t b = off / 256; b < off / 256 + blocks; ++b) {
                if (owner[b] >= 0) return printf("overlap at %zu\n", b * 256), 1;
                owner[b] = it;
            }
            live.push_back({off, bytes});
            used += blocks * 256;
        } else {
            const size_t k = rng() % live.size();
            const Live l = live[k];
            live.erase(live.begin() + (long)k);
            a.release(l.off, l.bytes);
            for (size_t b = l.off / 256; b < l.off / 256 + (l.bytes + 255) / 256; ++b)
                owner[b] = -1;
            used -= (l.bytes + 255) / 256 * 256;
        }
        if (a.used() != used) return printf("used %zu vs %zu\n", a.used(), used), 1;
        if (a.peak() < used) return printf("peak below used\n"), 1;
    }
    for (const Live &l : live)
        a.release(l.off, l.bytes);
    if (a.used() != 0 || a.free_ranges() != 1 || a.largest_free() != cap)
        return printf("not merged back: %zu ranges\n", a.free_ranges()), 1;
    printf("ok\n");
    return 0;
}
