// Host unit test of the server's arena bookkeeping (arena.h): random
// allocation/release sequences against a byte-level shadow map.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "arena.h"

#define CHECK(c)                                                        \
    do {                                                                \
        if (!(c)) {                                                     \
            std::fprintf(stderr, "CHECK failed line %d: %s\n", __LINE__, #c); \
            return 1;                                                   \
        }                                                               \
    } while (0)

int main() {
    using heat::ArenaBook;
    const size_t cap = 1 << 20;
    ArenaBook a;
    a.reset(cap + 100);                      // capacity is rounded down to the alignment
    CHECK(a.cap() == cap);
    std::vector<int> owner(cap / ArenaBook::ALIGN, -1);
    struct Blk { size_t off, bytes; int id; };
    std::vector<Blk> live;
    std::mt19937_64 rng(7);
    int next_id = 0;
    size_t used = 0, peak = 0;
    for (int it = 0; it < 200000; ++it) {
        const bool do_alloc = live.empty() || (rng() % 100) < 55;
        if (do_alloc) {
            const size_t bytes = 1 + rng() % (64 * 1024);
            size_t off = 0;
            const size_t before_largest = a.largest_free();
            if (!a.alloc(bytes, &off)) {
                CHECK(before_largest < ArenaBook::round(bytes));   // refusal only when nothing fits
                continue;
            }
            const size_t rb = ArenaBook::round(bytes);
            CHECK(off % ArenaBook::ALIGN == 0 && off + rb <= cap);
            for (size_t u = off / ArenaBook::ALIGN; u < (off + rb) / ArenaBook::ALIGN; ++u) {
                CHECK(owner[u] == -1);                             // no overlap
                owner[u] = next_id;
            }
            live.push_back({off, bytes, next_id++});
            used += rb;
            peak = used > peak ? used : peak;
        } else {
            const size_t k = rng() % live.size();
            Blk b = live[k];
            live[k] = live.back();
            live.pop_back();
            const size_t rb = ArenaBook::round(b.bytes);
            for (size_t u = b.off / ArenaBook::ALIGN; u < (b.off + rb) / ArenaBook::ALIGN; ++u) {
                CHECK(owner[u] == b.id);
                owner[u] = -1;
            }
            a.release(b.off, b.bytes);
            used -= rb;
        }
        CHECK(a.used() == used && a.peak() == peak);
    }
    for (const Blk &b : live) a.release(b.off, b.bytes);
    CHECK(a.used() == 0 && a.free_ranges() == 1 && a.largest_free() == cap);   // fully coalesced
    std::printf("arena ok\n");
    return 0;
}
