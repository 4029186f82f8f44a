// Host half of the multi-volume batch calls of include/tsdf.h: work-list
// staging, the persistent launches, the online autotuner and the graph cache.
//
// Per call: the items are sorted by band half-width K (counting sort, stable),
// each item's tile count is taken for the configuration's tile width, and the
// work list (K ranges, tile prefix sums, item descriptors) is written into one
// slot of a pinned host ring and copied, on the caller's stream, to the same
// slot of the device workspace, which holds one work list per ring slot.  Then
// one persistent kernel per K present runs over the list.
//
// Reuse of a slot is ordered, so calls may come from several streams:
//   - the host rewrites a ring slot only after the event behind its last copy
//     has completed (the copy engine has read it);
//   - the copy into a device slot waits (on the device) for the event behind
//     the launches that last read that slot, whatever stream they ran on.

#include <algorithm>
#include <cstdlib>
#include <limits>
#include <new>
#include <vector>

#include "tsdf_host.h"

using namespace tsdf_host;

namespace {

constexpr int kRingSlots = 8;
constexpr int kMaxGraphs = 32;
constexpr uint64_t kHeaderBytes = 256;  // k_begin[kBatchGroups], padded
static_assert(4 * (tsdf::kBatchGroups + 1) <= kHeaderBytes, "group ranges fit the header");
constexpr int kAccChoices[2] = {4, 8};
constexpr uint32_t kTileWidths[3] = {16, 32, 64};
constexpr int kMaxPixelsPerThread = 2;

struct WorkLayout {
  uint64_t tile_start, items, total;
};

WorkLayout work_layout(uint32_t max_items) {
  WorkLayout L;
  L.tile_start = kHeaderBytes;
  L.items = align_up(L.tile_start + 4ull * ((uint64_t)max_items + 1));
  L.total = align_up(L.items + sizeof(tsdf::BatchItem) * (uint64_t)max_items);
  return L;
}

int acc_index(uint32_t ab) { return ab == 4 ? 0 : ab == 8 ? 1 : -1; }

unsigned log2_u32(uint32_t x) {
  unsigned l = 0;
  while ((1u << l) < x) ++l;
  return l;
}

bool valid_config(const tsdf_batch_config* c) {
  if (!c || !(c->tile_width == 16 || c->tile_width == 32 || c->tile_width == 64)) return false;
  if (c->pixels_per_thread < 1 || c->pixels_per_thread > (uint32_t)kMaxPixelsPerThread) return false;
  if (acc_index(c->acc_blocks) < 0 || c->groups_per_cu > 64) return false;
  return tsdf::multi_kernel(1, (int)c->pixels_per_thread, (int)c->acc_blocks, false) != nullptr;
}

bool same_config(const tsdf_batch_config& a, const tsdf_batch_config& b) {
  return a.tile_width == b.tile_width && a.pixels_per_thread == b.pixels_per_thread &&
         a.acc_blocks == b.acc_blocks && a.groups_per_cu == b.groups_per_cu;
}

struct Timing {
  int cand;
  hipEvent_t start, stop;
  double pixels;
};

struct GraphEntry {
  uint32_t k_mask;
  int slot;  // the device work list its kernel nodes read
  tsdf_batch_config cfg;
  hipGraph_t graph;
  hipGraphExec_t exec;
  uint64_t last_use;
};

}  // namespace

struct tsdf_batch {
  uint32_t max_items;
  int device;  // current at tsdf_batch_create
  char* ws;
  WorkLayout L;
  int n_cu;
  // resident workgroups per CU by [K][pixels per thread - 1][acc index][colour];
  // 0 = not yet asked
  int occupancy[TSDF_MAX_BAND_HALF + 1][kMaxPixelsPerThread][2][2];
  // staging ring and the device work lists, one per slot
  char* ring;
  hipEvent_t ring_done[kRingSlots];  // behind the copy out of the ring slot
  bool ring_pending[kRingSlots];
  hipEvent_t slot_done[kRingSlots];  // behind the launches that read the device slot
  bool slot_used[kRingSlots];
  int next_slot;
  // configuration and tuner
  tsdf_batch_config cfg;
  bool tuned;
  uint32_t trials;
  std::vector<tsdf_batch_config> cands;
  std::vector<double> best;  // per candidate: least seconds per pixel seen
  uint32_t issued;           // tuning calls launched
  std::vector<Timing> pending;
  std::vector<Timing> spare;  // event pairs ready for reuse
  // graphs
  GraphEntry graphs[kMaxGraphs];
  int n_graphs;
  uint64_t calls;
  // per-call scratch
  std::vector<uint32_t> order;
};

namespace {

// A group's kernel shape: the configuration's, except for colour volumes,
// which have one (1 pixel per thread, 4 LDS blocks).
struct Shape {
  int K, ppt, ab;
  bool colour;
};

Shape shape_of(int group, const tsdf_batch_config& c) {
  const bool colour = group >= tsdf::batch_group(0, true);
  const int K = colour ? group - tsdf::batch_group(0, true) : group;
  return colour ? Shape{K, 1, 4, true} : Shape{K, (int)c.pixels_per_thread, (int)c.acc_blocks, false};
}

int occupancy(tsdf_batch* b, int K, int ppt, int ai, bool colour = false) {
  int& o = b->occupancy[K][ppt - 1][ai][colour ? 1 : 0];
  if (o == 0) {
    int n = 0;
    const void* fn = tsdf::multi_kernel(K, ppt, kAccChoices[ai], colour);
    if (!fn || hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, 256, 0) != hipSuccess || n < 1)
      n = 1;
    o = n;
  }
  return o;
}

unsigned grid_for(tsdf_batch* b, const Shape& sh, const tsdf_batch_config& c) {
  int per_cu = occupancy(b, sh.K, sh.ppt, acc_index((uint32_t)sh.ab), sh.colour);
  if (c.groups_per_cu != 0 && (int)c.groups_per_cu < per_cu) per_cu = (int)c.groups_per_cu;
  return (unsigned)per_cu * (unsigned)b->n_cu;
}

// Every tile width x pixels per thread x accumulator size at full residency,
// then the 16-pixel-wide, 8-block shapes at half residency (K = 4 sets the
// number).
void build_candidates(tsdf_batch* b) {
  b->cands.clear();
  for (int ppt = 1; ppt <= kMaxPixelsPerThread; ++ppt)
    for (uint32_t tw : kTileWidths)
      for (int ab : kAccChoices)
        if (tsdf::multi_kernel(4, ppt, ab, false))
          b->cands.push_back(tsdf_batch_config{tw, (uint32_t)ppt, (uint32_t)ab, 0u});
  for (int ppt = 1; ppt <= kMaxPixelsPerThread; ++ppt) {
    const int full = occupancy(b, 4, ppt, acc_index(8));
    if (full >= 2) b->cands.push_back(tsdf_batch_config{16u, (uint32_t)ppt, 8u, (uint32_t)(full / 2)});
  }
  b->best.assign(b->cands.size(), std::numeric_limits<double>::infinity());
}

void release_timings(tsdf_batch* b) {
  for (Timing& t : b->pending) {
    (void)hipEventSynchronize(t.stop);
    b->spare.push_back(t);
  }
  b->pending.clear();
}

// Fold in the timings of finished tuning calls; fix the configuration once
// every candidate has all its trials.
void poll_tuner(tsdf_batch* b) {
  if (b->tuned) return;
  size_t keep = 0;
  for (size_t i = 0; i < b->pending.size(); ++i) {
    Timing& t = b->pending[i];
    if (hipEventQuery(t.stop) == hipSuccess) {
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, t.start, t.stop) == hipSuccess && t.pixels > 0.0) {
        const double spp = 1e-3 * (double)ms / t.pixels;
        if (spp < b->best[t.cand]) b->best[t.cand] = spp;
      }
      b->spare.push_back(t);
    } else {
      b->pending[keep++] = t;
    }
  }
  b->pending.resize(keep);
  const uint32_t total = (uint32_t)b->cands.size() * b->trials;
  if (b->issued >= total && b->pending.empty()) {
    size_t arg = 0;
    for (size_t i = 1; i < b->best.size(); ++i)
      if (b->best[i] < b->best[arg]) arg = i;
    b->cfg = b->cands[arg];
    b->tuned = true;
  }
}

// The configuration of the next call and, while tuning, its candidate index.
tsdf_batch_config next_config(tsdf_batch* b, int* cand) {
  *cand = -1;
  if (b->tuned) return b->cfg;
  const uint32_t n = (uint32_t)b->cands.size();
  if (b->issued < n * b->trials) {
    *cand = (int)(b->issued % n);
    return b->cands[*cand];
  }
  // every trial launched, some not finished: the best measured so far
  size_t arg = 0;
  for (size_t i = 1; i < b->best.size(); ++i)
    if (b->best[i] < b->best[arg]) arg = i;
  return std::isfinite(b->best[arg]) ? b->cands[arg] : b->cands[0];
}

// The work list at `list` (a device slot of the workspace, or other device
// memory laid out the same way).
tsdf::BatchWork device_work(const tsdf_batch* b, const char* list) {
  tsdf::BatchWork w;
  w.k_begin = reinterpret_cast<const unsigned*>(list);
  w.tile_start = reinterpret_cast<const unsigned*>(list + b->L.tile_start);
  w.items = reinterpret_cast<const tsdf::BatchItem*>(list + b->L.items);
  return w;
}

const char* slot_list(const tsdf_batch* b, int slot) { return b->ws + (size_t)slot * b->L.total; }

hipError_t launch_direct(tsdf_batch* b, const char* list, uint32_t g_mask,
                         const tsdf_batch_config& c, const uint32_t* g_tiles, hipStream_t s) {
  tsdf::BatchWork w = device_work(b, list);
  unsigned tw_log2 = log2_u32(c.tile_width);
  void* args[] = {&w, &tw_log2};
  for (int g = 0; g < tsdf::kBatchGroups; ++g) {
    if (!(g_mask & (1u << g))) continue;
    const Shape sh = shape_of(g, c);
    unsigned grid = grid_for(b, sh, c);
    if (g_tiles[g] < grid) grid = g_tiles[g];
    const hipError_t e = hipLaunchKernel(tsdf::multi_kernel(sh.K, sh.ppt, sh.ab, sh.colour),
                                         dim3(grid), dim3(256), args, 0, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

void destroy_graph(GraphEntry& g) {
  (void)hipGraphExecDestroy(g.exec);
  (void)hipGraphDestroy(g.graph);
}

// The instantiated graph of one kernel node per group in k_mask (band width
// and colour) for configuration c reading the work list of device slot `slot`
// (no memory nodes: the work list arrives by the copy before the launch).
hipError_t graph_for(tsdf_batch* b, uint32_t k_mask, int slot, const tsdf_batch_config& c,
                     hipGraphExec_t* out) {
  for (int i = 0; i < b->n_graphs; ++i) {
    GraphEntry& g = b->graphs[i];
    if (g.k_mask == k_mask && g.slot == slot && same_config(g.cfg, c)) {
      g.last_use = b->calls;
      *out = g.exec;
      return hipSuccess;
    }
  }
  hipGraph_t graph = nullptr;
  hipError_t e = hipGraphCreate(&graph, 0);
  if (e != hipSuccess) return e;
  tsdf::BatchWork w = device_work(b, slot_list(b, slot));
  unsigned tw_log2 = log2_u32(c.tile_width);
  void* args[] = {&w, &tw_log2};
  for (int g = 0; g < tsdf::kBatchGroups && e == hipSuccess; ++g) {
    if (!(k_mask & (1u << g))) continue;
    const Shape sh = shape_of(g, c);
    hipKernelNodeParams p;
    std::memset(&p, 0, sizeof(p));
    p.func = const_cast<void*>(tsdf::multi_kernel(sh.K, sh.ppt, sh.ab, sh.colour));
    p.gridDim = dim3(grid_for(b, sh, c));
    p.blockDim = dim3(256);
    p.sharedMemBytes = 0;
    p.kernelParams = args;
    p.extra = nullptr;
    hipGraphNode_t node;
    e = hipGraphAddKernelNode(&node, graph, nullptr, 0, &p);
  }
  hipGraphExec_t exec = nullptr;
  if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(graph);
    return e;
  }
  int at = b->n_graphs;
  if (at == kMaxGraphs) {
    // evict the least recently used; its last replay may still be queued, on
    // any stream, and is done once the event behind its slot's last use is
    at = 0;
    for (int i = 1; i < kMaxGraphs; ++i)
      if (b->graphs[i].last_use < b->graphs[at].last_use) at = i;
    const int vs = b->graphs[at].slot;
    e = b->slot_used[vs] ? hipEventSynchronize(b->slot_done[vs]) : hipSuccess;
    if (e != hipSuccess) {
      (void)hipGraphExecDestroy(exec);
      (void)hipGraphDestroy(graph);
      return e;
    }
    destroy_graph(b->graphs[at]);
  } else {
    ++b->n_graphs;
  }
  b->graphs[at] = GraphEntry{k_mask, slot, c, graph, exec, b->calls};
  *out = exec;
  return hipSuccess;
}

void free_batch(tsdf_batch* b) {
  for (int i = 0; i < kRingSlots; ++i) {
    if (b->ring_done[i]) {
      (void)hipEventSynchronize(b->ring_done[i]);
      (void)hipEventDestroy(b->ring_done[i]);
    }
    if (b->slot_done[i]) {
      (void)hipEventSynchronize(b->slot_done[i]);
      (void)hipEventDestroy(b->slot_done[i]);
    }
  }
  release_timings(b);
  for (Timing& t : b->spare) {
    (void)hipEventDestroy(t.start);
    (void)hipEventDestroy(t.stop);
  }
  for (int i = 0; i < b->n_graphs; ++i) destroy_graph(b->graphs[i]);
  if (b->ring) (void)hipHostFree(b->ring);
  delete b;
}

bool valid_items(const tsdf_fuse_item* items, uint32_t n_items) {
  for (uint32_t i = 0; i < n_items; ++i) {
    const tsdf_fuse_item& it = items[i];
    if (!it.volume || !valid_camera(&it.camera)) return false;
    const bool pixels = (uint64_t)it.camera.width * it.camera.height > 0;
    if (pixels && !it.depth_dev) return false;
    if (pixels && it.volume->dev.colour && !it.rgba_dev) return false;
  }
  return true;
}

// One call of the batch path.  The work list goes to device slot `slot` of
// the workspace, or, if `list_dev` is not null, to that device memory (whose
// uses the caller orders); then the launches.  With `list_dev` the call is
// launched directly, never timed for the tuner nor replayed from a graph.
tsdf_status batch_fuse_impl(tsdf_batch* b, const tsdf_fuse_item* items, uint32_t n_items,
                            uint32_t flags, char* list_dev, hipStream_t s) {
  if (!valid_items(items, n_items)) return TSDF_ERR_INVALID_ARGUMENT;
  if (n_items == 0) return TSDF_OK;
  if (!list_dev) poll_tuner(b);  // (its bookkeeping may allocate host memory)
  int cand = -1;
  const tsdf_batch_config c = next_config(b, &cand);
  if (list_dev) cand = -1;  // not a tuning trial
  const uint32_t tw = c.tile_width;

  // the ring slot: wait until the copy that last read it has run
  const int slot = b->next_slot;
  b->next_slot = (slot + 1) % kRingSlots;
  if (b->ring_pending[slot] && hipEventSynchronize(b->ring_done[slot]) != hipSuccess)
    return TSDF_ERR_HIP;
  b->ring_pending[slot] = false;
  char* host = b->ring + (size_t)slot * b->L.total;
  unsigned* k_begin = reinterpret_cast<unsigned*>(host);
  unsigned* tile_start = reinterpret_cast<unsigned*>(host + b->L.tile_start);
  tsdf::BatchItem* out = reinterpret_cast<tsdf::BatchItem*>(host + b->L.items);

  // counting sort by group (band width, colour)
  auto group_of = [](const tsdf_fuse_item& it) {
    return tsdf::batch_group(band_half(it.volume->params), it.volume->dev.colour != nullptr);
  };
  uint32_t count[tsdf::kBatchGroups] = {0};
  for (uint32_t i = 0; i < n_items; ++i) ++count[group_of(items[i])];
  uint32_t k_mask = 0, acc = 0;
  for (int g = 0; g < tsdf::kBatchGroups; ++g) {
    k_begin[g] = acc;
    acc += count[g];
    if (count[g]) k_mask |= 1u << g;
  }
  k_begin[tsdf::kBatchGroups] = acc;
  uint32_t cursor[tsdf::kBatchGroups];
  for (int g = 0; g < tsdf::kBatchGroups; ++g) cursor[g] = k_begin[g];
  b->order.resize(n_items);
  for (uint32_t i = 0; i < n_items; ++i) b->order[cursor[group_of(items[i])]++] = i;

  uint64_t tiles = 0;
  double pixels = 0.0;
  uint32_t k_tiles[tsdf::kBatchGroups] = {0};
  for (uint32_t j = 0; j < n_items; ++j) {
    const tsdf_fuse_item& it = items[b->order[j]];
    const int g = group_of(it);
    const uint32_t th = (uint32_t)shape_of(g, c).ppt * (256u / tw);
    tsdf::BatchItem& bi = out[j];
    std::memset(&bi, 0, sizeof(bi));
    bi.vol = it.volume->dev;
    bi.wp = walk_params(it.volume);
    bi.fr = frame_dev(it.depth_dev, &it.camera, it.volume->dev.colour ? it.rgba_dev : nullptr);
    const uint32_t tx = (it.camera.width + tw - 1) / tw;
    const uint32_t ty = (it.camera.height + th - 1) / th;
    bi.tiles_x = tx;
    tile_start[j] = (uint32_t)tiles;
    tiles += (uint64_t)tx * ty;
    k_tiles[g] += tx * ty;
    pixels += (double)it.camera.width * it.camera.height;
    if (tiles > 0x7FFFFFFFull) return TSDF_ERR_INVALID_ARGUMENT;  // tile indices stay in 31 bits
  }
  tile_start[n_items] = (uint32_t)tiles;
  for (int g = 0; g < tsdf::kBatchGroups; ++g)
    if (k_tiles[g] == 0) k_mask &= ~(1u << g);

  // the device list: the slot's, once the launches that last read it are done
  char* list = list_dev;
  if (!list) {
    list = const_cast<char*>(slot_list(b, slot));
    if (b->slot_used[slot] && hipStreamWaitEvent(s, b->slot_done[slot], 0) != hipSuccess)
      return TSDF_ERR_HIP;
  }
  const size_t bytes = (size_t)b->L.items + (size_t)n_items * sizeof(tsdf::BatchItem);
  if (hipMemcpyAsync(list, host, bytes, hipMemcpyHostToDevice, s) != hipSuccess) return TSDF_ERR_HIP;
  if (hipEventRecord(b->ring_done[slot], s) != hipSuccess) return TSDF_ERR_HIP;
  b->ring_pending[slot] = true;
  ++b->calls;

  if (k_mask != 0) {
    hipError_t e = hipSuccess;
    if (cand >= 0) {
      Timing t;
      if (!b->spare.empty()) {
        t = b->spare.back();
        b->spare.pop_back();
      } else {
        e = hipEventCreate(&t.start);
        if (e == hipSuccess) e = hipEventCreate(&t.stop);
        if (e != hipSuccess) return TSDF_ERR_HIP;
      }
      t.cand = cand;
      t.pixels = pixels;
      e = hipEventRecord(t.start, s);
      if (e == hipSuccess) e = launch_direct(b, list, k_mask, c, k_tiles, s);
      if (e == hipSuccess) e = hipEventRecord(t.stop, s);
      if (e != hipSuccess) {
        b->spare.push_back(t);
        return TSDF_ERR_HIP;
      }
      b->pending.push_back(t);
      ++b->issued;
    } else if (!list_dev && b->tuned && !(flags & TSDF_BATCH_NO_GRAPH)) {
      hipGraphExec_t exec = nullptr;
      e = graph_for(b, k_mask, slot, c, &exec);
      if (e == hipSuccess) e = hipGraphLaunch(exec, s);
    } else {
      e = launch_direct(b, list, k_mask, c, k_tiles, s);
    }
    if (e != hipSuccess) return TSDF_ERR_HIP;
  }
  if (!list_dev) {
    if (hipEventRecord(b->slot_done[slot], s) != hipSuccess) return TSDF_ERR_HIP;
    b->slot_used[slot] = true;
  }
  for (uint32_t i = 0; i < n_items; ++i) items[i].volume->frames++;
  return TSDF_OK;
}

}  // namespace

extern "C" {

size_t tsdf_batch_workspace_bytes(uint32_t max_items) {
  if (max_items == 0 || max_items > TSDF_BATCH_MAX_ITEMS) return 0;
  return (size_t)work_layout(max_items).total * kRingSlots;
}

tsdf_status tsdf_batch_create(uint32_t max_items, void* workspace_dev, size_t workspace_bytes,
                              tsdf_batch** out) {
  if (!out) return TSDF_ERR_INVALID_ARGUMENT;
  *out = nullptr;
  if (max_items == 0 || max_items > TSDF_BATCH_MAX_ITEMS) return TSDF_ERR_INVALID_ARGUMENT;
  if (!workspace_dev || ((uintptr_t)workspace_dev % kAlign) != 0) return TSDF_ERR_INVALID_ARGUMENT;
  const WorkLayout L = work_layout(max_items);
  if (workspace_bytes < L.total * kRingSlots) return TSDF_ERR_BUFFER_TOO_SMALL;
  tsdf_batch* b = new (std::nothrow) tsdf_batch();
  if (!b) return TSDF_ERR_INTERNAL;
  b->max_items = max_items;
  b->ws = static_cast<char*>(workspace_dev);
  b->L = L;
  std::memset(b->occupancy, 0, sizeof(b->occupancy));
  b->ring = nullptr;
  for (int i = 0; i < kRingSlots; ++i) {
    b->ring_done[i] = nullptr;
    b->ring_pending[i] = false;
    b->slot_done[i] = nullptr;
    b->slot_used[i] = false;
  }
  b->next_slot = 0;
  b->n_graphs = 0;
  b->calls = 0;
  b->tuned = false;
  b->trials = 2;
  b->issued = 0;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  b->device = dev;
  if (e == hipSuccess) e = hipDeviceGetAttribute(&b->n_cu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&b->ring), kRingSlots * L.total,
                                         hipHostMallocDefault);
  for (int i = 0; i < kRingSlots && e == hipSuccess; ++i) {
    e = hipEventCreateWithFlags(&b->ring_done[i], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->slot_done[i], hipEventDisableTiming);
  }
  if (e != hipSuccess || b->n_cu < 1) {
    free_batch(b);
    return TSDF_ERR_HIP;
  }
  b->order.reserve(max_items);
  build_candidates(b);
  b->cfg = b->cands[0];
  *out = b;
  return TSDF_OK;
}

tsdf_status tsdf_batch_destroy(tsdf_batch* batch) {
  if (!batch) return TSDF_ERR_INVALID_ARGUMENT;
  free_batch(batch);
  return TSDF_OK;
}

tsdf_status tsdf_batch_set_config(tsdf_batch* batch, const tsdf_batch_config* config) {
  if (!batch || !valid_config(config)) return TSDF_ERR_INVALID_ARGUMENT;
  release_timings(batch);
  batch->cfg = *config;
  batch->tuned = true;
  return TSDF_OK;
}

tsdf_status tsdf_batch_autotune(tsdf_batch* batch, uint32_t trials) {
  if (!batch || trials < 1 || trials > 16) return TSDF_ERR_INVALID_ARGUMENT;
  release_timings(batch);
  batch->trials = trials;
  batch->issued = 0;
  batch->tuned = false;
  batch->best.assign(batch->cands.size(), std::numeric_limits<double>::infinity());
  return TSDF_OK;
}

tsdf_status tsdf_batch_get_config(tsdf_batch* batch, tsdf_batch_config* config, uint32_t* tuned) {
  if (!batch) return TSDF_ERR_INVALID_ARGUMENT;
  poll_tuner(batch);
  int cand = -1;
  const tsdf_batch_config c = next_config(batch, &cand);
  if (config) *config = c;
  if (tuned) *tuned = batch->tuned ? 1u : 0u;
  return TSDF_OK;
}

tsdf_status tsdf_batch_candidates(tsdf_batch* batch, uint32_t max, tsdf_batch_config* configs,
                                  double* ns_per_pixel, uint32_t* n_out) {
  if (!batch || !n_out) return TSDF_ERR_INVALID_ARGUMENT;
  poll_tuner(batch);
  const uint32_t n = (uint32_t)batch->cands.size();
  *n_out = n;
  for (uint32_t i = 0; i < n && i < max; ++i) {
    if (configs) configs[i] = batch->cands[i];
    if (ns_per_pixel) ns_per_pixel[i] = batch->best[i] * 1e9;
  }
  return TSDF_OK;
}

tsdf_status tsdf_batch_fuse(tsdf_batch* b, const tsdf_fuse_item* items, uint32_t n_items,
                            uint32_t flags, void* hip_stream) {
  if (!b || (n_items > 0 && !items) || n_items > b->max_items) return TSDF_ERR_INVALID_ARGUMENT;
  if ((flags & ~TSDF_BATCH_NO_GRAPH) != 0) return TSDF_ERR_INVALID_ARGUMENT;
  return batch_fuse_impl(b, items, n_items, flags, nullptr, as_stream(hip_stream));
}

tsdf_status tsdf_batch_fuse_static(tsdf_batch* b, const tsdf_fuse_item* items, uint32_t n_items,
                                   void* hip_stream) {
  if (!b || (n_items > 0 && !items) || n_items > b->max_items) return TSDF_ERR_INVALID_ARGUMENT;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return TSDF_ERR_HIP;
  if (dev != b->device) return TSDF_ERR_INVALID_ARGUMENT;
  void* list = nullptr;
  size_t cap = 0;
  if (tsdf::static_scratch(&list, &cap) != hipSuccess) return TSDF_ERR_HIP;
  if ((uint64_t)b->L.items + (uint64_t)n_items * sizeof(tsdf::BatchItem) > cap)
    return TSDF_ERR_BUFFER_TOO_SMALL;
  return batch_fuse_impl(b, items, n_items, 0, static_cast<char*>(list), as_stream(hip_stream));
}

}  // extern "C"
