// Fixed-capacity hash table with least-recently-used eviction.
//
// The graph cache of Section 4.2 keeps instantiated graphs in a fixed-size
// hash table keyed by the communication configuration (buffer addresses and
// size), evicts the least recently used entry, and takes its size from the
// environment.  Here one cache per request maps a binding (rank buffers,
// outputs, scales, stream) to its device descriptor table and, in graph
// mode, the instantiated graph of the persistent launch.
//
// Host-only C++17 (no HIP): the owner supplies a disposer that releases an
// evicted value, which lets the policy be unit-tested with a fake value.
#pragma once
#include <cstddef>
#include <functional>
#include <list>
#include <unordered_map>
#include <utility>

namespace pcoll {

template <class Key, class Value, class Hash = std::hash<Key>>
class LruCache {
 public:
  using Disposer = std::function<void(const Key&, Value&)>;

  LruCache(std::size_t capacity, Disposer dispose)
      : cap_(capacity ? capacity : 1), dispose_(std::move(dispose)) {}
  LruCache(const LruCache&) = delete;
  LruCache& operator=(const LruCache&) = delete;
  ~LruCache() { clear(); }

  // Returns the cached value and marks it most recently used, or nullptr.
  Value* get(const Key& k) {
    auto it = map_.find(k);
    if (it == map_.end()) {
      ++misses_;
      return nullptr;
    }
    ++hits_;
    order_.splice(order_.begin(), order_, it->second);
    return &it->second->second;
  }

  // Inserts (or replaces) a value, evicting the least recently used entry
  // when full.  Returns the stored value.
  Value& put(const Key& k, Value v) {
    auto it = map_.find(k);
    if (it != map_.end()) {
      dispose_(it->first, it->second->second);
      it->second->second = std::move(v);
      order_.splice(order_.begin(), order_, it->second);
      return it->second->second;
    }
    if (map_.size() >= cap_) {
      auto& victim = order_.back();
      dispose_(victim.first, victim.second);
      map_.erase(victim.first);
      order_.pop_back();
      ++evictions_;
    }
    order_.emplace_front(k, std::move(v));
    map_.emplace(k, order_.begin());
    return order_.front().second;
  }

  // Applies f to every value (most recent first).
  template <class F>
  void for_each(F&& f) {
    for (auto& kv : order_) f(kv.first, kv.second);
  }

  void clear() {
    for (auto& kv : order_) dispose_(kv.first, kv.second);
    order_.clear();
    map_.clear();
  }

  std::size_t size() const { return map_.size(); }
  std::size_t capacity() const { return cap_; }
  std::size_t hits() const { return hits_; }
  std::size_t misses() const { return misses_; }
  std::size_t evictions() const { return evictions_; }

 private:
  using Entry = std::pair<Key, Value>;
  std::size_t cap_;
  Disposer dispose_;
  std::list<Entry> order_;  // most recently used first
  std::unordered_map<Key, typename std::list<Entry>::iterator, Hash> map_;
  std::size_t hits_ = 0, misses_ = 0, evictions_ = 0;
};

}  // namespace pcoll
