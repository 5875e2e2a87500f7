// bed_lru.hpp -- bounded least-recently-used map for the process caches of
// the convenience entry points (plans with device work lists, backward work
// lists).  Entries can be pinned (a HIP graph captured their device pointers)
// and are then never evicted; evicted values are handed back to the caller,
// which frees their device memory once their last use has completed.  Host
// code only (no HIP), so the policy is testable without a GPU.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <map>
#include <utility>
#include <vector>

namespace bed {

template <class K, class V>
class Lru {
public:
    explicit Lru(size_t capacity) : cap_(capacity ? capacity : 1) {}

    // The value for k (marked most recently used), or nullptr.
    V *find(const K &k)
    {
        auto it = map_.find(k);
        if (it == map_.end()) return nullptr;
        it->second.tick = ++tick_;
        return &it->second.value;
    }

    void pin(const K &k)
    {
        auto it = map_.find(k);
        if (it != map_.end()) it->second.pinned = true;
    }

    // Inserts k -> v.  While the map is at capacity, the least recently used
    // unpinned entries are removed and returned (when every entry is pinned
    // the map grows past its capacity instead).
    std::vector<V> insert(K k, V v)
    {
        std::vector<V> out;
        while (map_.size() >= cap_) {
            auto victim = map_.end();
            for (auto it = map_.begin(); it != map_.end(); ++it)
                if (!it->second.pinned && (victim == map_.end() || it->second.tick < victim->second.tick))
                    victim = it;
            if (victim == map_.end()) break;
            out.push_back(std::move(victim->second.value));
            map_.erase(victim);
        }
        Entry e;
        e.value = std::move(v);
        e.tick = ++tick_;
        e.pinned = false;
        map_[std::move(k)] = std::move(e);
        return out;
    }

    size_t size() const { return map_.size(); }
    size_t capacity() const { return cap_; }

private:
    struct Entry {
        V value;
        uint64_t tick;
        bool pinned;
    };
    std::map<K, Entry> map_;
    uint64_t tick_ = 0;
    size_t cap_;
};

}  // namespace bed
