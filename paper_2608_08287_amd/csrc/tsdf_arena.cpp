// Host half of the region sub-allocator of include/tsdf.h (tsdf_region_*):
// first-fit over a caller-owned device region, 256-byte aligned, with
// coalescing of neighbouring free ranges.  Pure host bookkeeping: the region's
// memory is never touched, so every call works without a GPU.

#include <cstdint>
#include <iterator>
#include <map>
#include <new>

#include "../../include/tsdf.h"

struct tsdf_region {
  uint64_t base;       // device address of the region's first usable byte
  uint64_t capacity;   // usable bytes (a multiple of the alignment)
  uint64_t used;       // bytes handed out
  std::map<uint64_t, uint64_t> free_ranges;  // offset -> size, disjoint, coalesced
  std::map<uint64_t, uint64_t> live;         // offset -> size of each allocation
};

namespace {

constexpr uint64_t kRegionAlign = 256;

uint64_t round_up(uint64_t x) { return (x + kRegionAlign - 1) / kRegionAlign * kRegionAlign; }

}  // namespace

extern "C" {

tsdf_status tsdf_region_create(void* device_base, uint64_t bytes, tsdf_region** out) {
  if (!out) return TSDF_ERR_INVALID_ARGUMENT;
  *out = nullptr;
  if (!device_base) return TSDF_ERR_INVALID_ARGUMENT;
  const uint64_t b = reinterpret_cast<uint64_t>(device_base);
  const uint64_t start = round_up(b);
  if (bytes < start - b) return TSDF_ERR_INVALID_ARGUMENT;
  const uint64_t cap = (bytes - (start - b)) / kRegionAlign * kRegionAlign;
  tsdf_region* r = new (std::nothrow) tsdf_region();
  if (!r) return TSDF_ERR_INTERNAL;
  r->base = start;
  r->capacity = cap;
  r->used = 0;
  if (cap > 0) r->free_ranges.emplace(0, cap);
  *out = r;
  return TSDF_OK;
}

tsdf_status tsdf_region_destroy(tsdf_region* region) {
  if (!region) return TSDF_ERR_INVALID_ARGUMENT;
  delete region;
  return TSDF_OK;
}

tsdf_status tsdf_region_alloc(tsdf_region* region, uint64_t bytes, void** out) {
  if (!region || !out || bytes == 0) return TSDF_ERR_INVALID_ARGUMENT;
  *out = nullptr;
  const uint64_t need = round_up(bytes);
  if (need < bytes) return TSDF_ERR_INVALID_ARGUMENT;  // overflow
  for (auto it = region->free_ranges.begin(); it != region->free_ranges.end(); ++it) {
    if (it->second < need) continue;
    const uint64_t off = it->first;
    const uint64_t rest = it->second - need;
    region->free_ranges.erase(it);
    if (rest) region->free_ranges.emplace(off + need, rest);
    region->live.emplace(off, need);
    region->used += need;
    *out = reinterpret_cast<void*>(region->base + off);
    return TSDF_OK;
  }
  return TSDF_ERR_BUDGET;
}

tsdf_status tsdf_region_free(tsdf_region* region, void* ptr) {
  if (!region || !ptr) return TSDF_ERR_INVALID_ARGUMENT;
  const uint64_t a = reinterpret_cast<uint64_t>(ptr);
  if (a < region->base) return TSDF_ERR_INVALID_ARGUMENT;
  const uint64_t off = a - region->base;
  auto lit = region->live.find(off);
  if (lit == region->live.end()) return TSDF_ERR_INVALID_ARGUMENT;
  uint64_t start = off, size = lit->second;
  region->live.erase(lit);
  region->used -= size;
  // merge with the free range that ends here and the one that starts after
  auto next = region->free_ranges.lower_bound(start);
  if (next != region->free_ranges.begin()) {
    auto prev = std::prev(next);
    if (prev->first + prev->second == start) {
      start = prev->first;
      size += prev->second;
      region->free_ranges.erase(prev);
    }
  }
  next = region->free_ranges.lower_bound(start + size);
  if (next != region->free_ranges.end() && next->first == start + size) {
    size += next->second;
    region->free_ranges.erase(next);
  }
  region->free_ranges.emplace(start, size);
  return TSDF_OK;
}

tsdf_status tsdf_region_usage(const tsdf_region* region, uint64_t* capacity, uint64_t* used,
                              uint64_t* largest_free, uint32_t* n_live) {
  if (!region) return TSDF_ERR_INVALID_ARGUMENT;
  uint64_t largest = 0;
  for (const auto& fr : region->free_ranges) largest = fr.second > largest ? fr.second : largest;
  if (capacity) *capacity = region->capacity;
  if (used) *used = region->used;
  if (largest_free) *largest_free = largest;
  if (n_live) *n_live = (uint32_t)region->live.size();
  return TSDF_OK;
}

}  // extern "C"
