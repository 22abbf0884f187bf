// Randomised check of the first-fit arena against a unit-map model: every
// block handed out lies inside the arena, overlaps no live block, is the
// lowest-offset fit, and the free list stays sorted, coalesced and equal to
// the complement of the live blocks.  Exit status 0 on success.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "../../paper_2003_02547_amd/csrc/arena.h"

int main(int argc, char** argv)
{
    const unsigned seed = argc > 1 ? (unsigned)atoi(argv[1]) : 1u;
    const size_t unit = 256, units = 4096;
    const int max_blocks = 300;
    std::mt19937_64 rng(seed);
    std::vector<ArenaRange> store(max_blocks + 2);
    Arena a;
    arena_reset(a, store.data(), units * unit);
    std::vector<int> owner(units, -1);
    struct Blk { size_t off, len; };
    std::vector<Blk> live;
    for (int step = 0; step < 200000; ++step) {
        const bool do_alloc = live.empty() || ((int)live.size() < max_blocks && (rng() % 100) < 55);
        if (do_alloc) {
            const size_t len = unit * (1 + rng() % 96);
            // model: lowest offset with len/unit free units
            size_t want = (size_t)-1;
            for (size_t u = 0, run = 0; u < units; ++u) {
                run = owner[u] < 0 ? run + 1 : 0;
                if (run == len / unit) { want = (u + 1 - run) * unit; break; }
            }
            size_t off;
            const bool ok = arena_alloc(a, len, &off);
            if (ok != (want != (size_t)-1)) { printf("alloc success mismatch at step %d\n", step); return 1; }
            if (!ok) continue;
            if (off != want) { printf("not first fit at step %d: %zu vs %zu\n", step, off, want); return 1; }
            if (off % unit || off + len > units * unit) { printf("out of arena\n"); return 1; }
            for (size_t u = off / unit; u < (off + len) / unit; ++u) {
                if (owner[u] >= 0) { printf("overlap at step %d\n", step); return 1; }
                owner[u] = (int)live.size();
            }
            live.push_back({off, len});
        } else {
            const size_t k = rng() % live.size();
            const Blk b = live[k];
            arena_free(a, b.off, b.len);
            for (size_t u = b.off / unit; u < (b.off + b.len) / unit; ++u) owner[u] = -1;
            live[k] = live.back();
            live.pop_back();
            for (size_t j = 0; j < live.size(); ++j)
                for (size_t u = live[j].off / unit; u < (live[j].off + live[j].len) / unit; ++u) owner[u] = (int)j;
        }
        // free list == complement of live blocks, sorted and coalesced
        size_t used = 0;
        for (const Blk& b : live) used += b.len;
        if (a.used != used) { printf("used mismatch\n"); return 1; }
        if (a.nfr > (int)live.size() + 1) { printf("free list too long\n"); return 1; }
        int r = 0;
        for (size_t u = 0; u < units;) {
            if (owner[u] >= 0) { ++u; continue; }
            size_t v = u;
            while (v < units && owner[v] < 0) ++v;
            if (r >= a.nfr || a.fr[r].off != u * unit || a.fr[r].len != (v - u) * unit) {
                printf("free list mismatch at step %d\n", step);
                return 1;
            }
            ++r;
            u = v;
        }
        if (r != a.nfr) { printf("extra free ranges\n"); return 1; }
    }
    printf("ok peak=%zu\n", a.peak);
    return 0;
}
