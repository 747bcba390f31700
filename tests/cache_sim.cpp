// Host-only checks of the serving form's subtree-cache bookkeeping
// (subtree_cache.h): arena first fit and coalescing, LRU eviction order,
// pinning, unfinished and private entries, run ends, and seeded random
// workloads whose invariants are checked as they run (pinned entries stay in
// the arena and never overlap, a pinned ready entry is still the one its key
// finds, the arena's use covers the pinned entries, everything is given back
// at the end).
#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <random>
#include <set>
#include <vector>

#include "subtree_cache.h"

using namespace tgp;

static int failures = 0;
#define CHECK(c)                                                         \
    do {                                                                 \
        if (!(c)) {                                                      \
            printf("FAIL line %d: %s\n", __LINE__, #c);                  \
            ++failures;                                                  \
        }                                                                \
    } while (0)

static SubtreeKey key(uint64_t i, uint64_t dom = 7) {
    SubtreeKey k;
    k.h0 = i * 0x9e3779b97f4a7c15ull + 1;
    k.h1 = ~i;
    k.dom = dom;
    return k;
}

static void arena_basics() {
    UnitArena a(100);
    uint64_t o1, o2, o3, o4;
    CHECK(a.alloc(30, &o1) && o1 == 0);
    CHECK(a.alloc(30, &o2) && o2 == 30);
    CHECK(a.alloc(30, &o3) && o3 == 60);
    CHECK(!a.alloc(20, &o4));           // 10 left
    a.release(o2, 30);                  // hole [30, 60)
    CHECK(a.largest_free() == 30 && a.free_runs() == 2);
    CHECK(!a.alloc(40, &o4));
    a.release(o1, 30);                  // merges with the hole: [0, 60)
    CHECK(a.largest_free() == 60 && a.free_runs() == 2);
    CHECK(a.alloc(40, &o4) && o4 == 0);  // first fit
    a.release(o3, 30);                  // [60, 100) merges with [40, 60)
    CHECK(a.free_runs() == 1 && a.largest_free() == 60 && a.used() == 40);
    a.release(o4, 40);
    CHECK(a.used() == 0 && a.free_runs() == 1 && a.largest_free() == 100);
}

static void lru_order_and_pins() {
    SubtreeCache c(30);
    CacheEntry *e[3];
    for (int i = 0; i < 3; ++i) {
        SubtreeKey k = key(i);
        e[i] = c.create(&k, 10, 1);
        CHECK(e[i] != nullptr);
    }
    CHECK(c.find(key(0)) == nullptr);  // not written yet
    for (int i = 0; i < 3; ++i) c.unpin(e[i], true);  // released in order 0, 1, 2
    // touching 0 makes it the most recent
    CacheEntry *f = c.find(key(0));
    CHECK(f == e[0]);
    c.unpin(f, false);
    // a new entry needs one slot: the least recently used (1) goes
    SubtreeKey k3 = key(3);
    CacheEntry *n = c.create(&k3, 10, 1);
    CHECK(n != nullptr && c.evictions() == 1);
    CHECK(c.find(key(1)) == nullptr);
    CacheEntry *g = c.find(key(2));
    CHECK(g != nullptr);  // 2 is pinned now, 0 is the only unpinned entry
    SubtreeKey k4 = key(4);
    CacheEntry *m = c.create(&k4, 20, 1);  // needs 20: evicting 0 gives only 10
    CHECK(m == nullptr);
    CHECK(c.find(key(0)) == nullptr);  // 0 was evicted trying
    c.unpin(g, false);
    c.unpin(n, true);
    m = c.create(&k4, 20, 1);  // 2 and 3 can go now
    CHECK(m != nullptr && c.used_units() == 20);
    c.unpin(m, true);
    CHECK(c.entries() == 1 && c.keyed_entries() == 1);
}

static void private_and_unfinished() {
    SubtreeCache c(40);
    SubtreeKey k = key(9);
    CacheEntry *a = c.create(&k, 10, 1);
    CacheEntry *b = c.create(&k, 10, 2);  // same key while a is being written: private
    CHECK(a->keyed && !b->keyed);
    c.unpin(b, true);  // a private entry is freed at once
    CHECK(c.entries() == 1 && c.used_units() == 10);
    c.unpin(a, false);  // never finished: freed, not findable
    CHECK(c.entries() == 0 && c.find(k) == nullptr && c.used_units() == 0);
    // a different domain is a different key
    SubtreeKey k2 = key(9, 8);
    CacheEntry *d = c.create(&k, 10, 1);
    c.unpin(d, true);
    CHECK(c.find(k2) == nullptr);
    CacheEntry *h = c.find(k);
    CHECK(h == d);
    c.unpin(h, false);
}

static void run_end() {
    SubtreeCache c(100);
    SubtreeKey k1 = key(1), k2 = key(2), k3 = key(3);
    CacheEntry *a = c.create(&k1, 10, 5);
    CacheEntry *b = c.create(&k2, 10, 5);
    CacheEntry *o = c.create(&k3, 10, 6);
    c.unpin(a, true);
    c.unpin(o, true);
    c.end_run(5);  // a goes now, b when released
    CHECK(c.entries() == 2 && c.find(k1) == nullptr);
    c.unpin(b, true);
    CHECK(c.entries() == 1 && c.find(k2) == nullptr);
    CacheEntry *f = c.find(k3);
    CHECK(f == o);
    c.unpin(f, false);
}

// Random operations against a model of the live entries.
static void random_workload(unsigned seed) {
    std::mt19937_64 rng(seed);
    const uint64_t cap = 1000;
    SubtreeCache c(cap);
    struct Held {
        CacheEntry *e;
        bool writer;
    };
    std::vector<Held> held;  // pins we hold
    for (int step = 0; step < 20000; ++step) {
        const int op = (int)(rng() % 10);
        if (op < 4) {
            SubtreeKey k = key(rng() % 64, rng() % 2);
            CacheEntry *e = c.create(&k, 1 + rng() % 120, (int64_t)(rng() % 4));
            if (e) held.push_back({e, true});
        } else if (op < 7) {
            CacheEntry *e = c.find(key(rng() % 64, rng() % 2));
            if (e) {
                CHECK(e->ready && !e->doomed);
                held.push_back({e, false});
            }
        } else if (op < 9 && !held.empty()) {
            const size_t i = rng() % held.size();
            c.unpin(held[i].e, held[i].writer && (rng() % 8 != 0));
            held[i] = held.back();
            held.pop_back();
        } else if (op == 9) {
            c.end_run((int64_t)(rng() % 4));
        }
        // invariants: live entries do not overlap and fill the arena's use
        if (step % 50 == 0 || step > 19900) {
            uint64_t total = 0;
            // every pinned entry is live and within the arena
            for (const Held &h : held) CHECK(h.e->off + h.e->len <= cap && h.e->pins > 0);
            // a pinned entry is never evicted: its key still finds it when ready
            for (const Held &h : held)
                if (h.e->keyed && h.e->ready && !h.e->doomed) {
                    CacheEntry *f = c.find(h.e->key);
                    CHECK(f == h.e);
                    if (f) c.unpin(f, false);
                }
            // distinct pinned entries never overlap
            std::set<CacheEntry *> uniq;
            for (const Held &h : held) uniq.insert(h.e);
            std::vector<std::pair<uint64_t, uint64_t>> iv;
            for (CacheEntry *e : uniq) {
                iv.push_back({e->off, e->len});
                total += e->len;
            }
            std::sort(iv.begin(), iv.end());
            for (size_t i = 1; i < iv.size(); ++i) CHECK(iv[i - 1].first + iv[i - 1].second <= iv[i].first);
            CHECK(total <= c.used_units() && c.used_units() <= cap);
            CHECK(c.used_units() + c.largest_free_units() <= cap);
        }
    }
    for (const Held &h : held) c.unpin(h.e, false);
    c.clear_unpinned();
    CHECK(c.used_units() == 0 && c.entries() == 0 && c.largest_free_units() == cap);
}

int main() {
    arena_basics();
    lru_order_and_pins();
    private_and_unfinished();
    run_end();
    for (unsigned s = 1; s <= 5; ++s) random_workload(s);
    if (failures) {
        printf("%d failures\n", failures);
        return 1;
    }
    printf("OK\n");
    return 0;
}
