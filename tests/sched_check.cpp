// CPU check of the request server's arena and admission policy (hrlb_sched.h):
//   - random alloc/release sequences keep the free and used ranges an exact, non-overlapping tiling
//     of the arena, blocks never overlap, and a fully released arena is one free range again;
//   - admission is in arrival order, never exceeds the free slots, lets later requests pass one that
//     does not fit only up to max_bypass times, and with max_bypass = 0 is strict FIFO.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <random>
#include <vector>

#include "hrlb_sched.h"

using namespace hrlb;

static int fails = 0;
#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            std::fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
            ++fails;                                                          \
        }                                                                     \
    } while (0)

static void arena_random(unsigned seed)
{
    std::mt19937 rng(seed);
    const size_t cap = (size_t(1) << 20) + 200;  // not a multiple of 256: the tail is unusable
    Arena a(cap);
    CHECK(a.capacity() == (size_t(1) << 20));
    CHECK(a.consistent());
    std::map<size_t, size_t> live;  // offset -> rounded size
    for (int it = 0; it < 4000; ++it) {
        if (live.empty() || rng() % 3 != 0) {
            const size_t want = 1 + rng() % 40000;
            const long long off = a.alloc(want);
            if (off >= 0) {
                const size_t sz = Arena::round_up(want);
                CHECK(off % 256 == 0);
                CHECK((size_t)off + sz <= a.capacity());
                for (const auto& kv : live) CHECK((size_t)off + sz <= kv.first || kv.first + kv.second <= (size_t)off);
                live[(size_t)off] = sz;
            } else {
                CHECK(a.largest_free() < Arena::round_up(want));
            }
        } else {
            auto k = live.begin();
            std::advance(k, rng() % live.size());
            CHECK(a.release(k->first));
            live.erase(k);
        }
        CHECK(!a.release(1));  // not a block start
        size_t used = 0;
        for (const auto& kv : live) used += kv.second;
        CHECK(a.used_bytes() == used);
        CHECK(a.live_blocks() == live.size());
        if (it % 97 == 0) CHECK(a.consistent());
    }
    for (const auto& kv : live) CHECK(a.release(kv.first));
    CHECK(a.consistent());
    CHECK(a.largest_free() == a.capacity());
    CHECK(a.used_bytes() == 0);
}

// a simulated admission round: requests with given sizes against a plain capacity counter
static std::vector<int> round_of(std::vector<Waiting>& q, const std::vector<size_t>& size, size_t& free_bytes,
                                 int slots, int max_bypass)
{
    return admit_in_order(q, slots, max_bypass, [&](int i) {
        if (size[i] > free_bytes) return false;
        free_bytes -= size[i];
        return true;
    });
}

static void admission()
{
    // strict FIFO: nothing passes a request that does not fit
    {
        std::vector<Waiting> q(4, Waiting{0});
        size_t free_b = 100;
        auto a = round_of(q, {50, 80, 10, 10}, free_b, 8, 0);
        CHECK(a.size() == 1 && a[0] == 0);
    }
    // backfill up to the limit, then hold the line
    {
        std::vector<Waiting> q(5, Waiting{0});
        size_t free_b = 100;
        auto a = round_of(q, {120, 10, 10, 10, 10}, free_b, 8, 2);
        CHECK(a.size() == 2 && a[0] == 1 && a[1] == 2);
        CHECK(q[0].bypassed == 2);
        // next round: the starved head still does not fit, so nothing behind it is admitted
        std::vector<Waiting> q2 = {q[0], q[3], q[4]};
        auto b = round_of(q2, {120, 10, 10}, free_b, 8, 2);
        CHECK(b.empty());
    }
    // slots bound the admissions
    {
        std::vector<Waiting> q(6, Waiting{0});
        size_t free_b = 1000;
        auto a = round_of(q, {1, 1, 1, 1, 1, 1}, free_b, 3, 4);
        CHECK(a.size() == 3 && a[0] == 0 && a[1] == 1 && a[2] == 2);
    }
    // random rounds: admitted indices increase, never exceed the slots, and a request that did not
    // fit is never passed more than max_bypass times in total
    std::mt19937 rng(7);
    for (int trial = 0; trial < 2000; ++trial) {
        const int n = 1 + rng() % 12, slots = rng() % 6, mb = rng() % 4;
        std::vector<Waiting> q(n, Waiting{0});
        std::vector<size_t> size(n);
        for (int i = 0; i < n; ++i) {
            size[i] = 1 + rng() % 60;
            q[i].bypassed = rng() % (mb + 1);
        }
        std::vector<int> before(n);
        for (int i = 0; i < n; ++i) before[i] = q[i].bypassed;
        size_t free_b = rng() % 120;
        auto a = round_of(q, size, free_b, slots, mb);
        CHECK((int)a.size() <= slots);
        for (size_t k = 1; k < a.size(); ++k) CHECK(a[k] > a[k - 1]);
        std::vector<bool> adm(n, false);
        for (int i : a) adm[i] = true;
        for (int i = 0; i < n; ++i) {
            if (adm[i]) continue;
            int passed = 0;
            for (int j : a)
                if (j > i) ++passed;
            CHECK(q[i].bypassed == before[i] + passed || i > (a.empty() ? -1 : a.back()));
            CHECK(q[i].bypassed <= std::max(mb, before[i]));
        }
    }
}

int main()
{
    for (unsigned s = 1; s <= 6; ++s) arena_random(s);
    admission();
    if (fails) {
        std::fprintf(stderr, "%d checks failed\n", fails);
        return 1;
    }
    std::printf("ok\n");
    return 0;
}
