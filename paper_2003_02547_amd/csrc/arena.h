// First-fit allocator over one device arena, with its bookkeeping in caller
// memory: a list of free ranges sorted by offset, coalesced on free.  With k
// blocks allocated there are at most k + 1 free ranges, so a list of
// max_blocks + 1 entries never overflows.  Host code only.
#pragma once

#include <stddef.h>

#include <cstring>

struct ArenaRange {
    size_t off, len;
};

struct Arena {
    ArenaRange* fr;  // free ranges, sorted by offset, none empty, none adjacent
    int nfr;
    size_t used, peak;
};

inline void arena_reset(Arena& a, ArenaRange* storage, size_t bytes)
{
    a.fr = storage;
    a.nfr = bytes > 0 ? 1 : 0;
    a.fr[0] = ArenaRange{0, bytes};
    a.used = a.peak = 0;
}

// Lowest-offset free range of at least len bytes; false when none fits.
inline bool arena_alloc(Arena& a, size_t len, size_t* off)
{
    for (int i = 0; i < a.nfr; ++i) {
        if (a.fr[i].len < len) continue;
        *off = a.fr[i].off;
        a.fr[i].off += len;
        a.fr[i].len -= len;
        if (a.fr[i].len == 0) {
            std::memmove(a.fr + i, a.fr + i + 1, sizeof(ArenaRange) * (a.nfr - i - 1));
            --a.nfr;
        }
        a.used += len;
        if (a.used > a.peak) a.peak = a.used;
        return true;
    }
    return false;
}

// Return [off, off + len), which must be a block arena_alloc handed out.
inline void arena_free(Arena& a, size_t off, size_t len)
{
    int i = 0;
    while (i < a.nfr && a.fr[i].off < off) ++i;
    const bool join_prev = i > 0 && a.fr[i - 1].off + a.fr[i - 1].len == off;
    const bool join_next = i < a.nfr && off + len == a.fr[i].off;
    if (join_prev && join_next) {
        a.fr[i - 1].len += len + a.fr[i].len;
        std::memmove(a.fr + i, a.fr + i + 1, sizeof(ArenaRange) * (a.nfr - i - 1));
        --a.nfr;
    } else if (join_prev) {
        a.fr[i - 1].len += len;
    } else if (join_next) {
        a.fr[i].off = off;
        a.fr[i].len += len;
    } else {
        std::memmove(a.fr + i + 1, a.fr + i, sizeof(ArenaRange) * (a.nfr - i));
        a.fr[i] = ArenaRange{off, len};
        ++a.nfr;
    }
    a.used -= len;
}
