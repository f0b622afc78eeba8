// Host checks of the serving scheduler's memory arena and admission pass:
// first-fit placement, coalescing of freed neighbours, the skip-ahead
// admission order, and a randomized comparison with a granule bitmap model.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "arena.hpp"

#define CHECK(c)                                                          \
    do {                                                                  \
        if (!(c)) {                                                       \
            std::fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
            std::exit(1);                                                 \
        }                                                                 \
    } while (0)

using cfi::Arena;

// Reference: a bitmap of 256-byte granules, first fit by linear scan.
struct Bitmap {
    std::vector<bool> used;
    explicit Bitmap(size_t size) : used(size / 256, false) {}
    bool alloc(size_t bytes, size_t* off) {
        const size_t g = Arena::granule(bytes) / 256;
        size_t run = 0;
        for (size_t k = 0; k < used.size(); ++k) {
            run = used[k] ? 0 : run + 1;
            if (run == g) {
                const size_t first = k + 1 - g;
                for (size_t j = first; j <= k; ++j) used[j] = true;
                *off = first * 256;
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        for (size_t j = off / 256; j < (off + Arena::granule(bytes)) / 256; ++j) used[j] = false;
    }
};

int main() {
    // placement and coalescing
    Arena a;
    a.reset(10 * 256);
    size_t o1, o2, o3, o4;
    CHECK(a.alloc(256, &o1) && o1 == 0);
    CHECK(a.alloc(300, &o2) && o2 == 256);          // two granules
    CHECK(a.alloc(256, &o3) && o3 == 768);
    CHECK(a.used() == 4 * 256);
    a.release(o2, 300);                             // hole of 2 granules at 256
    CHECK(a.n_free_ranges() == 2);
    CHECK(a.alloc(3 * 256, &o4) && o4 == 1024);     // does not fit the hole
    a.release(o1, 256);                             // merges with the hole: 3 granules at 0
    CHECK(a.n_free_ranges() == 2 && a.largest_free() == 3 * 256);
    size_t o5;
    CHECK(a.alloc(3 * 256, &o5) && o5 == 0);        // first fit takes the merged range
    a.release(o3, 256);
    a.release(o4, 3 * 256);
    a.release(o5, 3 * 256);
    CHECK(a.used() == 0 && a.n_free_ranges() == 1 && a.largest_free() == 10 * 256);
    CHECK(!a.alloc(11 * 256, &o1));

    // admission pass: a big head waits, later small requests pass it
    a.reset(8 * 256);
    size_t hold;
    CHECK(a.alloc(4 * 256, &hold));
    auto picked = cfi::admit_pass(a, {6 * 256, 2 * 256, 256, 3 * 256});
    CHECK(picked.size() == 2 && picked[0].first == 1 && picked[1].first == 2);
    CHECK(picked[0].second == 4 * 256 && picked[1].second == 6 * 256);
    a.release(hold, 4 * 256);
    picked = cfi::admit_pass(a, {6 * 256, 3 * 256});
    CHECK(picked.size() == 1 && picked[0].first == 1 && picked[0].second == 0);

    // randomized: same offsets as the bitmap model, no overlap, exact accounting
    std::mt19937_64 rng(12345);
    for (int trial = 0; trial < 20; ++trial) {
        const size_t size = 256 * (64 + rng() % 512);
        Arena ar;
        ar.reset(size);
        Bitmap bm(size);
        std::vector<std::pair<size_t, size_t>> live;
        size_t used = 0;
        for (int op = 0; op < 4000; ++op) {
            if (live.empty() || rng() % 3 != 0) {
                const size_t bytes = 1 + rng() % (size / 8);
                size_t oa = 0, ob = 0;
                const bool fa = ar.alloc(bytes, &oa), fb = bm.alloc(bytes, &ob);
                CHECK(fa == fb);
                if (fa) {
                    CHECK(oa == ob && oa + Arena::granule(bytes) <= size);
                    live.emplace_back(oa, bytes);
                    used += Arena::granule(bytes);
                }
            } else {
                const size_t k = rng() % live.size();
                ar.release(live[k].first, live[k].second);
                bm.release(live[k].first, live[k].second);
                used -= Arena::granule(live[k].second);
                live.erase(live.begin() + k);
            }
            CHECK(ar.used() == used);
        }
        for (auto& l : live) ar.release(l.first, l.second);
        CHECK(ar.used() == 0 && ar.n_free_ranges() == 1);
    }
    std::printf("arena ok\n");
    return 0;
}
