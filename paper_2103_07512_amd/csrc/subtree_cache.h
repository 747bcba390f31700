// subtree_cache.h -- bookkeeping of the resident subtree results kept by the
// serving form: a first-fit arena of fixed-size units and an LRU map from
// (structural hash of a subtree, domain) to the arena rows holding its value
// at every fitness case.
//
// TensorGP reuses the results of subtrees that were already evaluated, which
// pays off after the first generations of a run (Sec. 4.2); here those results
// stay in device memory across generations and runs until the space is
// needed.  Pure host code with no HIP dependency, so it can be tested alone.
#pragma once

#include <stdint.h>

#include <iterator>
#include <list>
#include <map>
#include <unordered_map>
#include <unordered_set>

namespace tgp {

// First-fit allocator over [0, capacity) units with coalescing frees.
class UnitArena {
public:
    explicit UnitArena(uint64_t units = 0) { reset(units); }
    void reset(uint64_t units) {
        free_.clear();
        cap_ = units;
        used_ = 0;
        if (units) free_[0] = units;
    }
    bool alloc(uint64_t len, uint64_t *off) {
        if (len == 0) len = 1;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < len) continue;
            *off = it->first;
            const uint64_t rest = it->second - len, start = it->first + len;
            free_.erase(it);
            if (rest) free_[start] = rest;
            used_ += len;
            return true;
        }
        return false;
    }
    void release(uint64_t off, uint64_t len) {
        if (len == 0) len = 1;
        used_ -= len;
        auto next = free_.lower_bound(off);
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                off = prev->first;
                len += prev->second;
                free_.erase(prev);
            }
        }
        if (next != free_.end() && off + len == next->first) {
            len += next->second;
            free_.erase(next);
        }
        free_[off] = len;
    }
    uint64_t capacity() const { return cap_; }
    uint64_t used() const { return used_; }
    uint64_t largest_free() const {
        uint64_t m = 0;
        for (auto &kv : free_) m = kv.second > m ? kv.second : m;
        return m;
    }
    size_t free_runs() const { return free_.size(); }

private:
    std::map<uint64_t, uint64_t> free_;  // offset -> length
    uint64_t cap_ = 0, used_ = 0;
};

struct SubtreeKey {
    uint64_t h0 = 0, h1 = 0;  // 128-bit structural hash of the subtree
    uint64_t dom = 0;         // hash of the domain (axes, sizes, bounds)
    bool operator==(const SubtreeKey &o) const { return h0 == o.h0 && h1 == o.h1 && dom == o.dom; }
};

struct SubtreeKeyHash {
    size_t operator()(const SubtreeKey &k) const {
        return (size_t)(k.h0 ^ (k.h1 * 0x9e3779b97f4a7c15ull) ^ (k.dom * 0xc2b2ae3d27d4eb4full));
    }
};

struct CacheEntry {
    SubtreeKey key;
    bool keyed = false;   // reachable by key (else private to the request that made it)
    uint64_t off = 0, len = 0;
    int pins = 0;
    bool ready = false;   // every case written
    bool doomed = false;  // freed when the last pin is released
    int64_t run = -1;     // the run that created it
    bool in_lru = false;
    std::list<CacheEntry *>::iterator lru_it;
};

// Entries are pinned while a request reads or writes them; unpinned ready
// entries sit in LRU order and are evicted oldest first when space is needed.
// Not thread-safe: the owner serialises calls.
class SubtreeCache {
public:
    explicit SubtreeCache(uint64_t units = 0) : arena_(units) {}
    ~SubtreeCache() {
        for (CacheEntry *e : all_) delete e;
    }
    SubtreeCache(const SubtreeCache &) = delete;
    SubtreeCache &operator=(const SubtreeCache &) = delete;

    // The ready entry for k, pinned; nullptr when there is none (absent, or
    // still being written by another request).
    CacheEntry *find(const SubtreeKey &k) {
        auto it = map_.find(k);
        if (it == map_.end() || !it->second->ready || it->second->doomed) return nullptr;
        pin(it->second);
        ++hits_;
        return it->second;
    }

    // A new pinned entry of len units, evicting unpinned entries oldest first
    // until the arena has room; nullptr if even that is not enough.  With a
    // key that no entry holds yet, the entry becomes reachable by it.
    CacheEntry *create(const SubtreeKey *key, uint64_t len, int64_t run) {
        uint64_t off = 0;
        while (!arena_.alloc(len, &off)) {
            if (lru_.empty()) return nullptr;
            evict_one();
        }
        CacheEntry *e = new CacheEntry();
        e->off = off;
        e->len = len;
        e->pins = 1;
        e->run = run;
        if (key && map_.find(*key) == map_.end()) {
            e->key = *key;
            e->keyed = true;
            map_[*key] = e;
        }
        all_.insert(e);
        ++created_;
        return e;
    }

    void pin(CacheEntry *e) {
        if (e->in_lru) {
            lru_.erase(e->lru_it);
            e->in_lru = false;
        }
        ++e->pins;
    }

    // Releases one pin; written marks the entry complete.  An entry nobody
    // can find again (private, unfinished or doomed) is freed at once.
    void unpin(CacheEntry *e, bool written) {
        if (written) e->ready = true;
        if (--e->pins > 0) return;
        if (e->doomed || !e->keyed || !e->ready) {
            destroy(e);
            return;
        }
        lru_.push_front(e);
        e->lru_it = lru_.begin();
        e->in_lru = true;
    }

    // Frees what run created: unpinned entries now, pinned ones on release.
    void end_run(int64_t run) {
        std::list<CacheEntry *> victims;
        for (CacheEntry *e : all_)
            if (e->run == run) victims.push_back(e);
        for (CacheEntry *e : victims) {
            if (e->pins == 0)
                destroy(e);
            else
                e->doomed = true;
        }
    }

    // Evicts every unpinned entry.
    void clear_unpinned() {
        while (!lru_.empty()) evict_one();
    }

    uint64_t capacity_units() const { return arena_.capacity(); }
    uint64_t used_units() const { return arena_.used(); }
    uint64_t largest_free_units() const { return arena_.largest_free(); }
    // Units that evicting every unpinned entry would give back.
    uint64_t evictable_units() const {
        uint64_t u = 0;
        for (CacheEntry *e : lru_) u += e->len;
        return u;
    }
    size_t entries() const { return all_.size(); }
    size_t keyed_entries() const { return map_.size(); }
    uint64_t hits() const { return hits_; }
    uint64_t created() const { return created_; }
    uint64_t evictions() const { return evictions_; }

private:
    void evict_one() {
        CacheEntry *e = lru_.back();
        destroy(e);
        ++evictions_;
    }
    void destroy(CacheEntry *e) {
        if (e->in_lru) {
            lru_.erase(e->lru_it);
            e->in_lru = false;
        }
        if (e->keyed) {
            auto it = map_.find(e->key);
            if (it != map_.end() && it->second == e) map_.erase(it);
        }
        arena_.release(e->off, e->len);
        all_.erase(e);
        delete e;
    }

    UnitArena arena_;
    std::unordered_map<SubtreeKey, CacheEntry *, SubtreeKeyHash> map_;
    std::list<CacheEntry *> lru_;  // front = most recently released
    std::unordered_set<CacheEntry *> all_;
    uint64_t hits_ = 0, created_ = 0, evictions_ = 0;
};

}  // namespace tgp
