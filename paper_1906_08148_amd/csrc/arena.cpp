// Sub-allocator over the caller's device arena: first-fit ranges with an
// exact-size cache in front.  Short-lived blocks (a multiply's plan) are
// taken from the top of the highest range that fits and go straight back to
// the range map when released, so they do not leave holes between the
// long-lived blocks (leaf stores, pyramids) that fill the arena from the
// bottom.
#include <algorithm>
#include <cstdint>

#include "internal.h"

namespace spamm {

void Arena::init(char* base, size_t bytes) {
  base_ = base;
  size_ = bytes;
  used_ = 0;
  free_.clear();
  cache_.clear();
  free_[0] = bytes;
}

static uint64_t cache_key(size_t bytes, size_t align) {
  int la = 0;
  while ((size_t(1) << la) < align) ++la;
  return (uint64_t(bytes) << 6) | uint64_t(la);
}

size_t Arena::fit(size_t bytes, size_t align) const {
  for (auto it = free_.begin(); it != free_.end(); ++it) {
    const size_t off = it->first, len = it->second;
    const size_t start = (off + align - 1) / align * align;
    const size_t lead = start - off;
    if (len < lead + bytes) continue;
    free_.erase(it);
    if (lead) free_[off] = lead;
    const size_t tail = len - lead - bytes;
    if (tail) free_[start + bytes] = tail;
    return start;
  }
  return SIZE_MAX;
}

// Last fit: the top of the highest range that holds an aligned block.
size_t Arena::fit_high(size_t bytes, size_t align) const {
  for (auto it = free_.rbegin(); it != free_.rend(); ++it) {
    const size_t off = it->first, len = it->second;
    if (len < bytes) continue;
    const size_t start = (off + len - bytes) / align * align;
    if (start < off) continue;
    free_.erase(std::next(it).base());
    if (start > off) free_[off] = start - off;
    const size_t tail = off + len - (start + bytes);
    if (tail) free_[start + bytes] = tail;
    return start;
  }
  return SIZE_MAX;
}

size_t Arena::alloc(size_t bytes, size_t align, bool high) {
  if (bytes == 0) bytes = align;
  bytes = (bytes + align - 1) / align * align;
  if (!high) {
    auto c = cache_.find(cache_key(bytes, align));
    if (c != cache_.end() && !c->second.empty()) {
      const size_t off = c->second.back();
      c->second.pop_back();
      used_ += bytes;
      return off;
    }
  }
  size_t off = high ? fit_high(bytes, align) : fit(bytes, align);
  if (off == SIZE_MAX && !cache_.empty()) {
    trim();
    off = high ? fit_high(bytes, align) : fit(bytes, align);
  }
  if (off != SIZE_MAX) used_ += bytes;
  return off;
}

void Arena::release(size_t off, size_t bytes, size_t align, bool merge) {
  if (bytes == 0) return;
  used_ -= bytes;
  if (merge) insert_free(off, bytes);
  else cache_[cache_key(bytes, align)].push_back(off);
}

// A range back into the range map, merged with its free neighbours.
void Arena::insert_free(size_t off, size_t bytes) const {
  auto next = free_.lower_bound(off);
  size_t start = off, len = bytes;
  if (next != free_.begin()) {
    auto prev = std::prev(next);
    if (prev->first + prev->second == off) {
      start = prev->first;
      len += prev->second;
      free_.erase(prev);
    }
  }
  if (next != free_.end() && next->first == off + bytes) {
    len += next->second;
    free_.erase(next);
  }
  free_[start] = len;
}

// Return every cached range to the range map, merging neighbours.
void Arena::trim() const {
  for (auto& kv : cache_) {
    const size_t bytes = size_t(kv.first >> 6);
    for (const size_t off : kv.second) insert_free(off, bytes);
  }
  cache_.clear();
}

size_t Arena::largest_free() const {
  trim();
  size_t best = 0;
  for (auto& kv : free_) best = std::max(best, kv.second);
  return best;
}

Region::~Region() {
  if (ctx) ctx->arena.release(off, bytes, align, temp);
}

void* Region::ptr() const { return ctx->arena.base() + off; }

RegionP Ctx::alloc(size_t bytes, size_t align, bool temp) {
  align = std::max<size_t>(align, 256);
  const size_t rounded = (std::max<size_t>(bytes, 1) + align - 1) / align * align;
  const size_t off = arena.alloc(rounded, align, temp);
  if (off == SIZE_MAX) return nullptr;
  auto r = std::make_shared<Region>();
  r->ctx = this;
  r->off = off;
  r->bytes = rounded;
  r->align = align;
  r->temp = temp;
  return r;
}

}  // namespace spamm
