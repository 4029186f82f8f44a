// Device code of libtsdf.so shared by its translation units: constants,
// hashing, atomics, the probe/insert protocol, the band walk and the fused
// kernel template.  Each tsdf_fuse_k<K>.hip instantiates the fused kernel for
// one band half-width K so that the variants compile in parallel.
//
// The fused kernel: one workgroup of 256 lanes (4 wave64) owns a 32x8 pixel
// tile of each of the F frames of its launch (F = 1 for a single frame) and
// runs three phases separated by workgroup barriers:
//
//   1. walk   -- each lane walks its pixel's truncation band (2K+1 samples) in
//                each frame and keeps, per sample, the voxel's in-block index
//                and its LDS key-set slot in one register (the truncated
//                distance is recomputed when it is added).  The block keys of the
//                tile are deduplicated into an LDS key set (open addressing,
//                64-bit LDS compare-exchange); a lane inserts a key only when it
//                differs from its previous sample's, and lanes of one wave that
//                race for a slot are serialised by the LDS itself.
//   2. resolve -- each distinct key of the tile is resolved once against the
//                global open-addressed table (Section 2.3's insert protocol):
//                probe linearly from the home slot, plain first read of the
//                entry, agent-scope compare-exchange on an empty slot, pool index
//                from a bump counter (one atomic per wave), publication of the
//                index with an agent-scope store.  The probe is unbounded up to a
//                full cyclic scan and written as a converged step loop (every busy
//                lane takes exactly one step per iteration and "waiting for a
//                publication" means "look again next iteration"), so a waiter
//                never spins while a publisher in its own wave is masked off.
//   3. integrate -- the tile's contributions (of all its frames) are first summed
//                in LDS, one slot per touched voxel: each dense block marks the
//                voxels its pairs touch in a 512-bit mask, a prefix sum over the
//                masks' counts gives each touched voxel a slot in block and
//                voxel order, and the slots (a sum and a count) are summed in
//                one pass when the LDS region holds them all, which is the
//                common case, else in passes of as many as it holds.  The slots
//                are then flushed with agent-scope float atomics, two lanes per
//                voxel (its sum and its count, which share a 64-byte pool
//                segment), so that a wave instruction touches a few segments.
//                Device-scope
//                float atomics on gfx950 are performed beyond L2, one request
//                per touched 64-byte segment per instruction whatever its lane
//                count, so the cost is the number of (tile, segment) pairs: a
//                voxel gets one update per tile (and per launch), not one per
//                contribution, and the TSDF sums and weights of a segment's 8
//                voxels share it (see the pool layout in tsdf_internal.h).
//
// A workgroup only ever accumulates into blocks whose indices it resolved itself,
// so one launch needs no grid-wide barrier.  The two-pass structure of Section
// 2.2 (allocate over all points, then integrate over all points) is the same
// code with phase 3 switched off, or with phase 2 restricted to lookups.
//
// All walk arithmetic is float32 +, -, *, floor and comparisons in a fixed order
// and every file that includes this header must be compiled with
// -ffp-contract=off so that no FMA changes a voxel choice.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/tsdf.h"
#include "tsdf_internal.h"

namespace tsdf {
namespace {

// The fused kernels' tile, 32x8 pixels.  It was chosen when a pool segment was
// an x-row of 8 voxels, where its contributions fell into about 6 % fewer
// segments than a 16x16 tile's on a room trajectory; with the 4x1x2 segments
// the two touch about as many.
constexpr int kTileW = 32;
constexpr int kTileH = 8;
constexpr int kThreads = kTileW * kTileH;  // 256 = 4 x wave64
constexpr int kWave = 64;
constexpr unsigned kSetCap = 1024;          // LDS key-set slots per workgroup
constexpr unsigned kSetNone = 0x7FFu;       // "no LDS slot" (set full)
constexpr unsigned kAccBlocks = 8;          // phase-3 LDS region, in blocks' worth of floats
constexpr int kProbeAhead = 4;              // table slots read per probe step
constexpr int kProbeAheadLong = 8;          // ... per later step, for tables that can fill
// A publication is one store after the winner's compare-exchange, so a wait is a
// handful of steps.  A wait this long means the invariant broke: report it as
// INTERNAL instead of spinning forever.
constexpr unsigned kMaxWaitSteps = 1u << 20;
constexpr int kFramePad = 3;  // spare frame descriptors after a launch's frames
// frame descriptors of a launch of up to NB frames (one-frame launches need no spares)
constexpr int frame_slots(int NB) { return NB > 1 ? NB + kFramePad : NB; }

// Two design alternatives stay buildable so that they can be measured against
// the shipped choice (both are off in the library; the build script's
// --variant turns one on in a separate library):
//   TSDF_FIRST_READ_COHERENT  the probe's first read of each entry is an
//       agent-scope atomic load, as the wait's reads are, instead of a plain
//       cacheable load;
//   TSDF_KEYSET_BALLOT  a wave elects one lane per distinct key (ballot, then
//       the leader's key broadcast) and only that lane inserts into the tile's
//       LDS key set, instead of every lane inserting its own key.
// Both give the same results as the shipped code.
#ifndef TSDF_FIRST_READ_COHERENT
#define TSDF_FIRST_READ_COHERENT 0
#endif
#ifndef TSDF_KEYSET_BALLOT
#define TSDF_KEYSET_BALLOT 0
#endif

// ---------------------------------------------------------------------------
// Keys and hashing
// ---------------------------------------------------------------------------

// Section 2.1: three 21-bit axes biased by 2^20, x in the top field.
__device__ __forceinline__ unsigned long long pack_key(int bx, int by, int bz) {
  return ((unsigned long long)(unsigned)(bx + (1 << 20)) << 42) |
         ((unsigned long long)(unsigned)(by + (1 << 20)) << 21) |
         (unsigned long long)(unsigned)(bz + (1 << 20));
}

// MurmurHash3 fmix64, then Lemire's multiply-shift range reduction of its high
// word onto [0, C).  C need not be a power of two.
__device__ __forceinline__ unsigned home_slot(unsigned long long k, unsigned C) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ull;
  k ^= k >> 33;
  return __umulhi((unsigned)(k >> 32), C);
}

// Slot of a key in the LDS set: Fibonacci hashing of the whole key.
__device__ __forceinline__ unsigned set_home(unsigned long long k) {
  return (unsigned)((k * 0x9E3779B97F4A7C15ull) >> 54) & (kSetCap - 1);
}

// ---------------------------------------------------------------------------
// Wave helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ unsigned lane_id() { return __lane_id(); }

__device__ __forceinline__ unsigned rank_in(unsigned long long mask) {
  return __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
}

__device__ __forceinline__ unsigned long long readlane64(unsigned long long v, int l) {
  const unsigned lo = __builtin_amdgcn_readlane((int)(unsigned)v, l);
  const unsigned hi = __builtin_amdgcn_readlane((int)(unsigned)(v >> 32), l);
  return ((unsigned long long)hi << 32) | lo;
}

// Sum over the wave of any per-lane count; every lane receives the total.
__device__ __forceinline__ unsigned wave_sum(unsigned v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += (unsigned)__shfl_xor((int)v, off, kWave);
  return v;
}

// Inclusive prefix sum over the lanes of the wave.
__device__ __forceinline__ unsigned wave_inclusive_scan(unsigned v) {
  const unsigned lane = lane_id();
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const unsigned o = (unsigned)__shfl_up((int)v, (unsigned)off, kWave);
    v += lane >= (unsigned)off ? o : 0u;
  }
  return v;
}

__device__ __forceinline__ unsigned wave_max(unsigned v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const unsigned o = (unsigned)__shfl_xor((int)v, off, kWave);
    v = o > v ? o : v;
  }
  return v;
}

// ---------------------------------------------------------------------------
// Atomics.  Agent scope: workgroups on every XCD see one another's claims.
// ---------------------------------------------------------------------------

__device__ __forceinline__ unsigned long long cas_key(unsigned long long* p,
                                                      unsigned long long expected,
                                                      unsigned long long desired) {
  __hip_atomic_compare_exchange_strong(p, &expected, desired, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
  return expected;  // the value seen in memory
}

__device__ __forceinline__ unsigned add_u32(unsigned* p, unsigned v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void add_u64(unsigned long long* p, unsigned long long v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void add_f32(float* p, float v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void set_flag(DevCounters* c, unsigned f) {
  __hip_atomic_fetch_or(&c->status_bits, f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// A key that found the table full (Section 7.2: probe exhaustion is accounted,
// never silent) enters the volume's overflow set once, so that the count of
// such keys is exact however many tiles, frames and launches meet the key.
// A full overflow set is itself flagged: the count is then a lower bound.
__device__ void record_table_overflow(const VolumeDev& vol, unsigned long long key) {
  unsigned h = home_slot(key, TSDF_OVERFLOW_KEY_SLOTS);
  for (unsigned i = 0; i < TSDF_OVERFLOW_KEY_SLOTS; ++i) {
    const unsigned long long prev = cas_key(&vol.overflow_keys[h], kEmptyKey, key);
    if (prev == kEmptyKey) {
      add_u32(&vol.ctr->keys_table_overflow, 1u);
      return;
    }
    if (prev == key) return;
    h = (h + 1 == TSDF_OVERFLOW_KEY_SLOTS) ? 0u : h + 1;
  }
  set_flag(vol.ctr, TSDF_FLAG_OVERFLOW_RECORD_FULL);
}

// ---------------------------------------------------------------------------
// Section 2.3: find or insert one key.  Converged step loop over the busy lanes.
// Returns the pool index, kBlockPoolFull, kBlockTableFull, or (lookup only)
// kBlockTableFull for a key that is absent.  In a slot-index volume (Section 6.4,
// the block index derived from the slot) the pool index is the slot where the
// key sits, so a lane that finds its key, or loses the exchange to it, is done
// at once; the winner still counts the block and lists it for extraction.
// ---------------------------------------------------------------------------

template <bool kInsert, bool kLong = false>
__device__ int resolve_key(const VolumeDev& vol, unsigned long long want, bool active,
                           unsigned& probes_out, bool& missing_out) {
  const unsigned C = vol.table_capacity;
  unsigned slot = active ? home_slot(want, C) : 0u;  // the slot at distance `probes`
  unsigned probes = 0, waits = 0;
  bool waiting = false, busy = active, missing = false, broken = false;
  int result = kBlockTableFull;
  while (busy) {
    bool won = false;
    TableEntry* e = vol.table + slot;
    if (waiting) {
      // only while waiting is the index read with an atomic (coherent) load
      const int b = __hip_atomic_load(&e->block, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (b != kBlockPublishing) {
        result = b;
        busy = false;
      } else if (++waits >= kMaxWaitSteps) {
        broken = true;
        busy = false;
      }
    } else {
      // Read consecutive slots with plain, cacheable loads issued together (one
      // memory latency per step instead of one per slot), then examine them in
      // probe order.  A stale key costs one more step; a stale index only
      // enters the wait.
      // The first read takes kProbeAhead slots.  In a table that can fill
      // (kLong), a chain that goes on past them takes kProbeAheadLong per read:
      // fewer dependent reads on long chains, at the cost of registers.
      constexpr int kMax = kLong ? kProbeAheadLong : kProbeAhead;
      const unsigned n_read = (!kLong || probes == 0) ? (unsigned)kProbeAhead : (unsigned)kMax;
      unsigned sl[kMax];
      TableEntry en[kMax];
#pragma unroll
      for (int i = 0; i < kMax; ++i) {
        sl[i] = (i == 0) ? slot : ((sl[i - 1] + 1 == C) ? 0u : sl[i - 1] + 1);
        if ((unsigned)i < n_read) {
#if TSDF_FIRST_READ_COHERENT
          en[i].key = __hip_atomic_load(&vol.table[sl[i]].key, __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT);
          en[i].block = __hip_atomic_load(&vol.table[sl[i]].block, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
          en[i].pad = 0u;
#else
          en[i] = vol.table[sl[i]];
#endif
        } else {
          en[i] = TableEntry{0ull, 0, 0u};  // not read: never a candidate
        }
      }
      // the first candidate in probe order (compile-time indices only, so the
      // read-ahead stays in registers)
      int at = -1;
      bool is_key = false;
      unsigned at_slot = 0;
      int at_block = 0;
#pragma unroll
      for (int i = kMax - 1; i >= 0; --i) {
        const bool cand = (unsigned)i < n_read && (probes + (unsigned)i < C) &&
                          (en[i].key == want || en[i].key == kEmptyKey);
        if (cand) {
          at = i;
          is_key = en[i].key == want;
          at_slot = sl[i];
          at_block = en[i].block;
        }
      }
      if (at < 0) {
        // none of them: move on (a full cyclic scan means the table is full)
        probes += n_read;
        const unsigned last = n_read == (unsigned)kProbeAhead ? sl[kProbeAhead - 1] : sl[kMax - 1];
        slot = (last + 1 == C) ? 0u : last + 1;
        if (probes >= C) {
          result = kBlockTableFull;
          busy = false;
        }
      } else {
        probes += (unsigned)at;
        slot = at_slot;
        e = vol.table + slot;
        if (is_key) {
          if (vol.slot_index) {  // the slot is the block: nothing to wait for
            result = (int)slot;
            busy = false;
          } else if (at_block != kBlockPublishing) {
            result = at_block;
            busy = false;
          } else {
            waiting = true;
          }
        } else if (kInsert) {
          const unsigned long long prev = cas_key(&e->key, kEmptyKey, want);
          if (prev == kEmptyKey) {
            won = true;
          } else if (prev == want) {
            if (vol.slot_index) {
              result = (int)slot;
              busy = false;
            } else {
              waiting = true;
            }
          } else {  // another key took the slot: keep probing after it
            ++probes;
            slot = (slot + 1 == C) ? 0u : slot + 1;
            if (probes >= C) {
              result = kBlockTableFull;
              busy = false;
            }
          }
        } else {
          missing = true;  // lookup only: an empty slot ends the chain
          busy = false;
        }
      }
    }
    // winners take consecutive pool indices with one atomic per wave
    const unsigned long long wmask = __ballot(won);
    if (wmask) {
      const int leader = __ffsll((long long)wmask) - 1;
      unsigned base = 0;
      if ((int)lane_id() == leader) base = add_u32(&vol.ctr->block_count, (unsigned)__popcll(wmask));
      base = (unsigned)__builtin_amdgcn_readlane((int)base, leader);
      if (won) {
        const unsigned idx = base + rank_in(wmask);
        int pub;
        if (idx < vol.pool_capacity) {
          // read only after the launch: no fence needed
          vol.block_keys[idx] = want;
          if (vol.slot_index) vol.alloc_list[idx] = slot;
          pub = vol.slot_index ? (int)slot : (int)idx;
        } else {
          pub = kBlockPoolFull;
          add_u32(&vol.ctr->keys_pool_overflow, 1u);
          set_flag(vol.ctr, TSDF_FLAG_POOL_EXHAUSTED);
        }
        __hip_atomic_store(&e->block, pub, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        result = pub;
        busy = false;
      }
    }
  }
  // a pool index is used as an address only if it lies inside the pool
  if (active && (broken || result >= (int)vol.pool_capacity || result < kBlockTableFull)) {
    set_flag(vol.ctr, TSDF_FLAG_INTERNAL);
    result = kBlockTableFull;
    missing = true;  // counted as a loss, not as a full table
  } else if (active && result == kBlockTableFull && !missing) {
    add_u32(&vol.ctr->table_full_events, 1u);
    set_flag(vol.ctr, TSDF_FLAG_TABLE_FULL);
    record_table_overflow(vol, want);
  }
  probes_out = probes;
  missing_out = missing;
  return result;
}

// Probe-histogram volumes: one resolution at `probes` slots past home.
__device__ __forceinline__ void count_probe(const VolumeDev& vol, unsigned probes) {
  const unsigned bin = probes == 0u ? 0u : 32u - (unsigned)__builtin_clz(probes);
  add_u64(&vol.ctr->probe_hist[bin < TSDF_PROBE_HIST_BINS ? bin : TSDF_PROBE_HIST_BINS - 1u], 1ull);
  if (probes) add_u64(&vol.ctr->probe_sum, probes);
}

// ---------------------------------------------------------------------------
// The band walk of one sample (shared by every phase that needs a voxel).
// ---------------------------------------------------------------------------

struct Sample {
  int vx, vy, vz;
  float val;
  bool in_range;  // the voxel can be keyed
  bool keep;      // passes the occlusion test (meaningful when in_range)
};

__device__ __forceinline__ Sample walk_sample(const FrameDev& f, const WalkParams& wp, float d,
                                              float a, float b, int k_minus_K) {
  Sample s;
  const float z = d + (float)k_minus_K * wp.v;
  const float xc = a * z, yc = b * z, zc = z;
  float w[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    float acc = f.R[3 * r + 0] * xc;
    acc = acc + f.R[3 * r + 1] * yc;
    acc = acc + f.R[3 * r + 2] * zc;
    w[r] = acc + f.t[r];
  }
  const float q0 = w[0] * wp.iv, q1 = w[1] * wp.iv, q2 = w[2] * wp.iv;
  s.in_range = (z > 0.0f) && (__builtin_fabsf(q0) < 8388608.0f) &&
               (__builtin_fabsf(q1) < 8388608.0f) && (__builtin_fabsf(q2) < 8388608.0f);
  const float f0 = __builtin_floorf(q0), f1 = __builtin_floorf(q1), f2 = __builtin_floorf(q2);
  s.vx = s.in_range ? (int)f0 : 0;
  s.vy = s.in_range ? (int)f1 : 0;
  s.vz = s.in_range ? (int)f2 : 0;
  // in range (|q| < 2^23) the floored float is the voxel index exactly, so the
  // centre (i + 1/2) v is computed from it without converting back
  const float c0 = (f0 + 0.5f) * wp.v;
  const float c1 = (f1 + 0.5f) * wp.v;
  const float c2 = (f2 + 0.5f) * wp.v;
  float zcv = f.R[2] * (c0 - f.t[0]);
  zcv = zcv + f.R[5] * (c1 - f.t[1]);
  zcv = zcv + f.R[8] * (c2 - f.t[2]);
  const float sdf = d - zcv;
  s.keep = s.in_range && (zcv > 0.0f) && !(sdf < -wp.trunc);
  s.val = sdf < wp.trunc ? sdf : wp.trunc;
  return s;
}

// Insert a block key into a tile's LDS key set (open addressing, linear
// probe): its slot, found or claimed, or kSetNone when the set is full.  A
// claimed slot is appended to the set's list of distinct keys.  The probe
// stays a loop: it is inlined once per band sample of every frame of a tile,
// and unrolled copies of it (rarely run past the first step) pushed the
// three-frame kernel's code past what the instruction cache holds.
__device__ __forceinline__ unsigned set_insert(unsigned long long* s_keys, unsigned short* s_list,
                                               unsigned* s_n, unsigned long long key) {
  unsigned h = set_home(key);
#pragma unroll 1
  for (unsigned i = 0; i < kSetCap; ++i) {
    const unsigned long long old = atomicCAS(&s_keys[h], kEmptyKey, key);
    if (old == kEmptyKey) {
      s_list[atomicAdd(s_n, 1u)] = (unsigned short)h;
      return h;
    }
    if (old == key) return h;
    h = (h + 1) & (kSetCap - 1);
  }
  return kSetNone;
}

// Per-sample state carried from phase 1 to phase 3 in one register:
// bit 31 valid pair, bits 9..19 LDS slot (kSetNone when the set overflowed;
// replaced by the dense block id in phase 3), bits 0..8 in-block voxel index.
constexpr unsigned kPairValid = 1u << 31;

__device__ __forceinline__ unsigned tile_of_group(unsigned g, unsigned n_tiles, bool remap) {
  if (!remap) return g;
  // Workgroups are dealt round-robin to the 8 XCDs.  Give XCD j the j-th
  // contiguous run of tiles so that neighbouring tiles, which share blocks and
  // table entries, meet in the same L2.
  const unsigned q = n_tiles >> 3, r = n_tiles & 7u;
  const unsigned xcd = g & 7u, local = g >> 3;
  return xcd * q + (xcd < r ? xcd : r) + local;
}

// Read-only data of a whole launch (kernel arguments, a batch's work list) read
// through the constant address space, where uniform loads become scalar loads
// that may be repeated at will instead of values held in registers.
template <typename T>
using ConstPtr = const __attribute__((address_space(4))) T*;

// The arguments of one fused launch, passed by value as the kernel's only
// argument so that they start the kernel argument segment.  A workgroup reads
// its frames from that segment with a uniform index: scalar loads of its own
// frames only, rather than selects over all NB frames held in registers.
template <int NB>
struct FuseArgs {
  VolumeDev vol;
  WalkParams wp;
  // NB frames and (NB > 1) kFramePad copies of the first past them, so that
  // the last group of F <= kFramePad + 1 frames reads inside the array
  FrameDev f[frame_slots(NB)];
  unsigned n_frames, tiles_x, n_tiles;
  int remap;
};

// One workgroup = one 32x8 tile of F consecutive frames of the launch's NB
// frames: workgroup g covers tile g % n_tiles of frames F * (g / n_tiles) + 0..F-1
// (frames past the batch are empty).  F > 1 sums the frames' contributions to a
// tile before they reach the pool; NB > F puts several frames in one grid so
// one frame's start-up overlaps another's pool updates.
// Two or three frames per workgroup ask for 4 waves per SIMD (at most 128
// VGPRs), the residency the LDS allows: three frames fit in 126 without
// spilling; capped while they still spilled 80 bytes per lane, they already
// measured faster than at 3 waves per SIMD without spills (room orbit, 32
// frames per launch: 7.87 against 7.57 G points/s).  Four frames need 158
// VGPRs and run at 3 waves per SIMD without spilling: 7.83 against 8.87 G
// points/s for three frames at 4 waves (capped at 4 waves, an earlier build
// of four frames spilled 152 bytes per lane; their 94 KB of code also
// overflows the instruction cache).  Colour workgroups take more LDS, three
// per CU: no cap.
constexpr int waves_per_eu_for(int F, bool colour) {
  return colour ? 1 : F == 4 ? 3 : (F == 2 || F == 3) ? 4 : 1;
}

// Accumulator floats per block: sums and counts in the pool's segment layout,
// then (colour volumes) the red, green and blue sums in the colour layout.
constexpr unsigned acc_block_floats(bool colour) {
  return colour ? kBlockFloats + kColourFloats : kBlockFloats;
}

// Phase 3 sums a tile's contributions per voxel in LDS before they reach the
// pool.  The dense blocks are taken in windows of kWin (one window unless the
// tile touches more blocks); per window, each block has a 512-bit mask of the
// voxels its pairs touch (eight 64-bit words) and per word the first voxel
// slot of its bits (16 bits: a window has at most 128 * 512 voxels), and the
// slots hold, as arrays: the TSDF sum; a tagged count (window block << 21 |
// voxel << 12 | count); and for colour volumes the red, green and blue sums.
constexpr unsigned slot_floats(bool colour) { return colour ? 5u : 2u; }
constexpr unsigned kWin = 128;
constexpr unsigned kMetaFloats = kWin * 8u * (8u + 2u) / 4u;  // masks, then word bases

// Floats of the shared region (below): AB pool blocks' worth and 4 KiB for a
// plain volume; 48 KiB for a colour volume, whose slots are 2.5 times as wide
// (52 KiB per workgroup with the block indices, three per CU either way).
constexpr unsigned region_floats(int AB, bool colour) {
  return colour ? 12288u : (unsigned)AB * kBlockFloats + kSetCap;
}

// LDS of one tile: the pool index of each dense block, and a region shared by
// the key set, the key list and the dense-id map (phases 1-2; the map, which
// phase 3 reads first, sits at the end) and by phase 3's masks, word bases and
// voxel slots.
template <int AB, bool kColour = false>
struct alignas(16) TileShared {
  static constexpr unsigned kRegion = region_floats(AB, kColour);
  static constexpr unsigned kCap = (kRegion - kMetaFloats) / slot_floats(kColour);
  union alignas(16) {
    struct {
      unsigned long long keys[kSetCap];
      unsigned n;  // distinct keys in the set
      unsigned pad[3];
      unsigned short list[kSetCap];
      unsigned short gap[(4u * kRegion - 12u * kSetCap - 16u) / 2u];
      unsigned short dense[kSetCap];
    } set;
    float region[kRegion];
  } u;
  int blockd[kSetCap];
  static_assert(sizeof(u.set) == 4u * kRegion, "the dense-id map ends the region");
  static_assert(2u * kMetaFloats <= kRegion, "the masks and word bases take at most half");
  static_assert(kCap >= 512, "a pass holds at least one block's voxels");
};

// A tile's frames, copied into registers (from a work list): read in place.
template <int F>
struct HeldFrames {
  const FrameDev (&f)[F];
  __device__ const FrameDev& operator[](int i) const { return f[i]; }
  __device__ HeldFrames reread() const { return *this; }
};

// A tile's frames in the launch's argument segment, frames first, first + 1,
// ...  With kReload, reread() hides the index from the optimiser, so what is
// read through its result is loaded again (scalar loads that hit the constant
// cache) where it is used, instead of being kept in scalar registers from the
// first read on: several frames' constants held through phases 1 and 2 spill
// to vector lanes.  One frame's fit, and reloading them in every pass of
// phase 3 only adds latency.
template <bool kReload>
struct ArgFrames {
  ConstPtr<FrameDev> f;
  unsigned first;
  __device__ const FrameDev& operator[](int i) const {
    return *(const FrameDev*)&f[first + (unsigned)i];
  }
  __device__ ArgFrames reread() const {
    unsigned g = first;
    if (kReload) asm volatile("" : "+s"(g));
    return {f, g};
  }
};

// One tile of F pixel slots per thread: the three phases.  Slot fi of the
// calling thread is pixel (px[fi], py[fi]) of frame frs[fi] (a HeldFrames or
// an ArgFrames; phase 3 reads its frames through frs.reread()); the slots may be
// the same pixel of F frames of one trajectory or F pixels of one frame.
// Frames with width 0 are empty.  Every thread of the workgroup must call it;
// it begins with a workgroup barrier, so a persistent workgroup may call it
// tile after tile.
template <int K, int F, int AB, FuseMode kMode, bool kColour = false, bool kRowFlush = true,
          bool kLong = false, class Frames>
__device__ __forceinline__ void fuse_tile(const VolumeDev& vol, const WalkParams& wp,
                                          const Frames& frs, const unsigned (&px)[F],
                                          const unsigned (&py)[F], unsigned shard,
                                          TileShared<AB, kColour>& sh) {
  constexpr int NS = 2 * K + 1;
  constexpr bool kInsert = kMode != FuseMode::kIntegrate;
  constexpr bool kAccumulate = kMode != FuseMode::kAllocate;

  unsigned long long* const s_keys = sh.u.set.keys;
  unsigned* const s_n = &sh.u.set.n;
  int* const s_blockd = sh.blockd;            // pool index per dense block id
  unsigned short* const s_dense = sh.u.set.dense;  // dense block id per set slot
  unsigned short* const s_list = sh.u.set.list;    // set slot per dense block id

  const unsigned tid = threadIdx.x;
  __syncthreads();  // the previous tile of a persistent workgroup is done with the LDS
  for (unsigned i = tid; i < kSetCap; i += kThreads) s_keys[i] = kEmptyKey;
  if (tid == 0) *s_n = 0;

  float d[F];
  unsigned rgb[F];  // colour volumes: the pixel's packed colour
#pragma unroll
  for (int fi = 0; fi < F; ++fi) {
    const FrameDev& fr = frs[fi];
    const bool inside = px[fi] < fr.width && py[fi] < fr.height;
    const size_t pix = (size_t)py[fi] * fr.width + px[fi];
    d[fi] = inside ? fr.depth[pix] : 0.0f;
    rgb[fi] = (kColour && inside) ? fr.rgba[pix] : 0u;
  }
  __syncthreads();

  // ---- phase 1: walk, per-point dedupe, key dedupe into LDS ----------------
  unsigned st[F][NS];
  unsigned ovf[F];  // per frame: samples whose key did not fit in the LDS set
  unsigned n_pts = 0, n_pairs = 0, n_oor = 0;
#pragma unroll
  for (int fi = 0; fi < F; ++fi) {
    const FrameDev& fr = frs[fi];
    const float df = d[fi];
    const bool point = __builtin_isfinite(df) && df > 0.0f;  // 0 outside the frame
    n_pts += point ? 1u : 0u;
    const float a = ((float)px[fi] - fr.cx) * fr.ifx;
    const float b = ((float)py[fi] - fr.cy) * fr.ify;
    unsigned long long prev_key = kEmptyKey;
    unsigned prev_slot = kSetNone;
    ovf[fi] = 0u;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const Sample smp = walk_sample(fr, wp, df, a, b, s - K);
      const bool z_ok = point && (df + (float)(s - K) * wp.v > 0.0f);
      if (z_ok && !smp.in_range) ++n_oor;
      // Whether a sample is kept is a function of its voxel (the centre's
      // depth against the pixel's), so the voxel-once-per-point rule only has
      // to compare kept samples; it does so after the key set has placed the
      // sample's block (below).
      const bool cand = point && smp.in_range && smp.keep;
      const unsigned long long key = pack_key(smp.vx >> 3, smp.vy >> 3, smp.vz >> 3);
      const unsigned loc = voxel_index((unsigned)smp.vx & 7u, (unsigned)smp.vy & 7u, (unsigned)smp.vz & 7u);
      // consecutive samples of a point mostly share a block: reuse its slot
      const bool need = cand && key != prev_key;
      unsigned slot = prev_slot;
#if TSDF_KEYSET_BALLOT
      for (unsigned long long todo = __ballot(need); todo != 0ull;) {
        const int leader = __builtin_ctzll(todo);
        const unsigned long long lk = __shfl(key, leader);
        const bool same = need && key == lk;
        unsigned ls = kSetNone;
        if (__lane_id() == (unsigned)leader) ls = set_insert(s_keys, s_list, s_n, key);
        ls = __shfl(ls, leader);
        if (same) slot = ls;
        todo &= ~__ballot(same);
      }
#else
      // every lane inserts its own key; the LDS serialises lanes of one wave
      // that aim at the same slot, so exactly one of them claims it and the
      // others find the key there
      if (need) slot = set_insert(s_keys, s_list, s_n, key);
#endif
      if (cand) {
        prev_key = key;
        prev_slot = slot;
      }
      // A voxel counts once per point.  A kept sample's voxel is (its block's
      // set slot, its in-block index): one compare with each earlier sample's
      // state.  The set never loses a key, so a block that found the set full
      // finds it full again: such samples compare coordinates, recomputed, with
      // the earlier ones that also found it full (a tile of more than kSetCap
      // blocks only).
      const unsigned word = kPairValid | (slot << 9) | loc;
      bool dup = false;
      if (cand && slot != kSetNone) {
#pragma unroll
        for (int j = 0; j < s; ++j) dup |= st[fi][j] == word;
      } else if (cand) {
#pragma unroll 1  // rare (a tile of more than kSetCap blocks): kept small
        for (unsigned m = ovf[fi]; m != 0u; m &= m - 1u) {
          const Sample o = walk_sample(fr, wp, df, a, b, __builtin_ctz(m) - K);
          dup |= o.vx == smp.vx && o.vy == smp.vy && o.vz == smp.vz;
        }
      }
      const bool pair = cand && !dup;
      n_pairs += pair ? 1u : 0u;
      // a pair whose key found the LDS set full is handled on its own in phase 3
      const bool spilled = pair && slot == kSetNone;
      ovf[fi] |= spilled ? (1u << s) : 0u;
      st[fi][s] = (pair && !spilled) ? word : 0u;
    }
  }
  // Phase 1's counts are reported only at the end of the tile; computed there,
  // they would keep every sample's inputs to them alive through phases 2 and 3
  // (with three frames per workgroup, spilled).  The empty asm fixes them here.
  asm volatile("" : "+v"(n_pts), "+v"(n_pairs), "+v"(n_oor));
  __syncthreads();

  // ---- phase 2: resolve each distinct key of the tile once ----------------
  const unsigned n_keys = *s_n;
  unsigned my_probe_max = 0;
  unsigned my_missing = 0;
  for (unsigned base = 0; base < n_keys; base += kThreads) {
    const unsigned j = base + tid;
    const bool act = j < n_keys;
    const unsigned h = act ? s_list[j] : 0u;
    const unsigned long long key = act ? s_keys[h] : kEmptyKey;
    unsigned probes = 0;
    bool missing = false;
    const int blk = resolve_key<kInsert, kLong>(vol, key, act, probes, missing);
    if (act) {
      s_blockd[j] = blk;
      s_dense[h] = (unsigned short)j;
      my_probe_max = probes > my_probe_max ? probes : my_probe_max;
      my_missing += missing ? 1u : 0u;
      if (vol.probe_hist) count_probe(vol, probes);
    }
  }
  __syncthreads();

  // ---- phase 3: integrate --------------------------------------------------
  // A pair's truncated distance is recomputed from its sample (the same
  // function on the same inputs, so the same bits) when its block's pass comes,
  // rather than held in registers for the whole kernel.
  unsigned n_drop = 0;
  if (kAccumulate) {
    // LDS slot -> dense block id
#pragma unroll
    for (int fi = 0; fi < F; ++fi) {
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const unsigned w = st[fi][s];
        if (w & kPairValid)
          st[fi][s] = kPairValid | ((unsigned)s_dense[(w >> 9) & 0x7FFu] << 9) | (w & 511u);
      }
    }
    // Pairs whose key did not fit in the LDS set (a tile touching more than
    // kSetCap distinct blocks): resolve each one directly (same protocol, same
    // result) and add it straight to the pool.  Rare; kept out of line of the
    // unrolled fast path by looping over the bits of a mask.
    const Frames fr3 = frs.reread();
#pragma unroll
    for (int fi = 0; fi < F; ++fi) {
      const FrameDev& fr = fr3[fi];
      const float a = ((float)px[fi] - fr.cx) * fr.ifx;
      const float b = ((float)py[fi] - fr.cy) * fr.ify;
#pragma unroll 1
      for (unsigned m = ovf[fi]; m != 0u; m &= m - 1u) {
        const int s = __builtin_ctz(m);
        const Sample smp = walk_sample(fr, wp, d[fi], a, b, s - K);
        unsigned probes = 0;
        bool missing = false;
        const int blk = resolve_key<kInsert, kLong>(
            vol, pack_key(smp.vx >> 3, smp.vy >> 3, smp.vz >> 3), true, probes, missing);
        my_missing += missing ? 1u : 0u;
        if (vol.probe_hist) count_probe(vol, probes);
        if (blk >= 0) {
          const unsigned loc =
              voxel_index((unsigned)smp.vx & 7u, (unsigned)smp.vy & 7u, (unsigned)smp.vz & 7u);
          float* bp = vol.voxels + (size_t)blk * kBlockFloats;
          add_f32(bp + pool_tsdf_index(loc), smp.val);
          add_f32(bp + pool_weight_index(loc), 1.0f);
          if (kColour) {
            float* cp = vol.colour + (size_t)blk * kColourFloats;
#pragma unroll
            for (unsigned c = 0; c < 3; ++c)
              add_f32(cp + colour_index(loc, c), (float)((rgb[fi] >> (8 * c)) & 255u));
          }
        } else {
          ++n_drop;
        }
      }
    }

    // Voxel slots, window by window of dense blocks.
    using Shared = TileShared<AB, kColour>;
    constexpr unsigned kCap = Shared::kCap;
    constexpr unsigned kInWin = 1u << 30;  // st: the pair's slot of this window, not its block
    unsigned long long* const s_mark = reinterpret_cast<unsigned long long*>(sh.u.region);
    unsigned short* const s_wbase = reinterpret_cast<unsigned short*>(s_mark + 8u * kWin);
    float* const s_sum = sh.u.region + kMetaFloats;
    unsigned* const s_tag = reinterpret_cast<unsigned*>(s_sum + kCap);
    float* const s_col = s_sum + 2u * kCap;  // colour: [3][kCap]
    // the scan's per-wave totals: the region's last words, which the map held
    // before and the slots hold after
    unsigned* const s_wsum = reinterpret_cast<unsigned*>(sh.u.region + Shared::kRegion) - kThreads / kWave;
    for (unsigned k0 = 0; k0 < n_keys; k0 += kWin) {
      const unsigned kn = n_keys - k0 < kWin ? n_keys - k0 : kWin;
      for (unsigned i = tid; i < kn * 8u; i += kThreads) s_mark[i] = 0ull;
      __syncthreads();
#pragma unroll
      for (int fi = 0; fi < F; ++fi)
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          const unsigned w = st[fi][s];
          const unsigned db = ((w >> 9) & 0x7FFu) - k0;
          if ((w & kPairValid) && db < kn)
            atomicOr(&s_mark[db * 8u + ((w & 511u) >> 6)], 1ull << (w & 63u));
        }
      __syncthreads();
      // word bases: one thread per block sums its words, a scan over the
      // blocks places them; every thread keeps the window's total
      unsigned total = 0;
      {
        unsigned cnt[8], key_total = 0;
        if (tid < kn) {
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            cnt[q] = (unsigned)__popcll(s_mark[tid * 8u + q]);
            key_total += cnt[q];
          }
        }
        const unsigned incl = wave_inclusive_scan(key_total);
        if (lane_id() == kWave - 1) s_wsum[tid / kWave] = incl;
        __syncthreads();
        unsigned before = 0;
#pragma unroll
        for (unsigned wv = 0; wv < kThreads / kWave; ++wv) {
          const unsigned ws = s_wsum[wv];
          before += wv < tid / kWave ? ws : 0u;
          total += ws;
        }
        if (tid < kn) {
          unsigned at = before + incl - key_total;
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            s_wbase[tid * 8u + q] = (unsigned short)at;
            at += cnt[q];
          }
        }
        __syncthreads();
      }
      // a pair of this window trades its block for its slot
#pragma unroll
      for (int fi = 0; fi < F; ++fi)
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          const unsigned w = st[fi][s];
          const unsigned db = ((w >> 9) & 0x7FFu) - k0;
          if ((w & kPairValid) && !(w & kInWin) && db < kn) {
            const unsigned item = db * 8u + ((w & 511u) >> 6);
            const unsigned slot = s_wbase[item] +
                                  (unsigned)__popcll(s_mark[item] & ((1ull << (w & 63u)) - 1ull));
            st[fi][s] = kPairValid | kInWin | (slot << 9) | (w & 511u);
          }
        }

      for (unsigned lo = 0; lo < total; lo += kCap) {
        const unsigned n_here = total - lo < kCap ? total - lo : kCap;
        // this pass's slots start from zero sums and tagged zero counts
        for (unsigned item = tid; item < kn * 8u; item += kThreads) {
          unsigned at = s_wbase[item];
          const unsigned tag = (item >> 3) << 21 | (item & 7u) << 18;  // block, voxel bits 6..8
          for (unsigned long long m = s_mark[item]; m != 0ull && at < lo + n_here;
               m &= m - 1ull, ++at) {
            if (at >= lo) {
              s_sum[at - lo] = 0.0f;
              s_tag[at - lo] = tag | (unsigned)__builtin_ctzll(m) << 12;
              if (kColour) {
#pragma unroll
                for (unsigned c = 0; c < 3; ++c) s_col[c * kCap + at - lo] = 0.0f;
              }
            }
          }
        }
        __syncthreads();
        const Frames frp = frs.reread();  // loaded again for each pass
#pragma unroll
        for (int fi = 0; fi < F; ++fi) {
          const FrameDev& fr = frp[fi];
          const float a = ((float)px[fi] - fr.cx) * fr.ifx;
          const float b = ((float)py[fi] - fr.cy) * fr.ify;
#pragma unroll
          for (int s = 0; s < NS; ++s) {
            const unsigned w = st[fi][s];
            const unsigned sl = ((w >> 9) & 0x1FFFFu) - lo;
            if ((w & kInWin) && sl < n_here) {
              // the empty asm makes the depth opaque to the optimiser so the
              // recomputation stays inside this pass instead of being hoisted
              // out of the loop (which would hold every pair's value in registers)
              float dk = d[fi];
              asm volatile("" : "+v"(dk));
              const float v = walk_sample(fr, wp, dk, a, b, s - K).val;
              __hip_atomic_fetch_add(s_sum + sl, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
              __hip_atomic_fetch_add(s_tag + sl, 1u, __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_WORKGROUP);
              if (kColour) {
#pragma unroll
                for (unsigned c = 0; c < 3; ++c)
                  __hip_atomic_fetch_add(s_col + c * kCap + sl,
                                         (float)((rgb[fi] >> (8 * c)) & 255u), __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_WORKGROUP);
              }
            }
          }
        }
        __syncthreads();
        // flush: two lanes per voxel slot, its sum and its count, which share
        // a 64-byte pool segment; slots are in block and voxel order, so a
        // segment's voxels are consecutive slots.
        if (kRowFlush) {
          // Each wave walks its quarter of the pass's slots in windows of at
          // most 32 slots that end where a segment ends, so that every touched
          // segment is one memory-side request (a segment cut by a fixed window
          // would cost two).  For kernels bound by those requests.
          const unsigned wv = tid / kWave, lane = lane_id();
          const unsigned half = lane & 1u, li = lane >> 1;
          unsigned pos = n_here * wv / (kThreads / kWave);
          const unsigned end = n_here * (wv + 1u) / (kThreads / kWave);
          while (pos < end) {  // uniform across the wave
            const unsigned j = pos + li;
            const bool in = j < end;
            const unsigned tg = in ? s_tag[j] : 0u;
            const float sm = in ? s_sum[j] : 0.0f;
            unsigned take = end - pos < 32u ? end - pos : 32u;
            if (pos + 32u < end) {
              // the window's last segment may go on past it: it opens the next one
              const unsigned last = (unsigned)__shfl((int)(tg >> 15), kWave - 1, kWave);
              const unsigned long long m = __ballot(in && half == 0u && (tg >> 15) == last);
              const unsigned first = (unsigned)__ffsll((long long)m) - 1u;
              if (first > 0u) take = first >> 1;
            }
            if (li < take) {
              const unsigned cnt = tg & 0xFFFu;
              const int blk = s_blockd[k0 + (tg >> 21)];
              const unsigned loc = (tg >> 12) & 511u;
              if (blk >= 0)
                add_f32(vol.voxels + (size_t)blk * kBlockFloats + (loc >> 3) * 16u + half * 8u +
                            (loc & 7u),
                        half ? (float)cnt : sm);
              else if (half)
                n_drop += cnt;  // the pool had no block for this key
            }
            pos += take;
          }
        } else {
          // Fixed windows of 32 slots per wave instruction, four slots per
          // lane read before any atomic is issued: one LDS wait per four,
          // for kernels bound by latency rather than by requests.
          const unsigned half = tid & 1u;
          for (unsigned j0 = tid >> 1; j0 < n_here; j0 += 4u * (kThreads / 2u)) {
            unsigned tg[4];
            float sm[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const unsigned j = j0 + (unsigned)q * (kThreads / 2u);
              const bool ok = j < n_here;
              tg[q] = ok ? s_tag[j] : 0u;
              sm[q] = ok ? s_sum[j] : 0.0f;
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const unsigned cnt = tg[q] & 0xFFFu;
              if (cnt == 0u) continue;  // past the pass's slots
              const int blk = s_blockd[k0 + (tg[q] >> 21)];
              const unsigned loc = (tg[q] >> 12) & 511u;
              if (blk >= 0)
                add_f32(vol.voxels + (size_t)blk * kBlockFloats + (loc >> 3) * 16u + half * 8u +
                            (loc & 7u),
                        half ? (float)cnt : sm[q]);
              else if (half)
                n_drop += cnt;  // the pool had no block for this key
            }
          }
        }
        if (kColour) {
          // colour sums: three lanes per slot (its red, green and blue sums), so
          // a wave instruction covers 21 slots and a touched 96-byte colour
          // segment costs about two requests; a zero sum needs no update
          constexpr unsigned kPer = kThreads / 3u;  // slots per iteration
          const unsigned c = tid % 3u;
          for (unsigned j0 = tid / 3u; j0 < n_here; j0 += 2u * kPer) {
            unsigned tg[2];
            float cv[2];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
              const unsigned j = j0 + (unsigned)q * kPer;
              const bool ok = tid < 3u * kPer && j < n_here;
              tg[q] = ok ? s_tag[j] : 0u;
              cv[q] = ok ? s_col[c * kCap + j] : 0.0f;
            }
#pragma unroll
            for (int q = 0; q < 2; ++q) {
              if (cv[q] == 0.0f) continue;
              const int blk = s_blockd[k0 + (tg[q] >> 21)];
              if (blk >= 0)
                add_f32(vol.colour + (size_t)blk * kColourFloats +
                            colour_index((tg[q] >> 12) & 511u, c),
                        cv[q]);
            }
          }
        }
        if (lo + kCap < total || k0 + kWin < n_keys) __syncthreads();
      }
      // this window's pairs are done
      if (k0 + kWin < n_keys) {
#pragma unroll
        for (int fi = 0; fi < F; ++fi)
#pragma unroll
          for (int s = 0; s < NS; ++s)
            if (st[fi][s] & kInWin) st[fi][s] = 0u;
      }
    }
  }

  // ---- counters: one atomic per wave, spread over shards -------------------
  const unsigned wave = tid / kWave;
  const bool leader = lane_id() == 0;
  if (kAccumulate) {
    const unsigned pts_w = wave_sum(n_pts);
    const unsigned pairs_w = wave_sum(n_pairs);
    const unsigned sh_i = (shard * 4u + wave) & (kCounterShards - 1);
    if (leader && pts_w) add_u64(&vol.ctr->points_valid[sh_i], pts_w);
    if (leader && pairs_w) add_u64(&vol.ctr->pairs[sh_i], pairs_w);
    if (__ballot(n_drop)) {
      const unsigned dw = wave_sum(n_drop);
      if (leader) add_u64(&vol.ctr->pairs_dropped, dw);
    }
    if (__ballot(n_oor)) {
      const unsigned ow = wave_sum(n_oor);
      if (leader) add_u64(&vol.ctr->coord_out_of_range, ow);
    }
  }
  if (__ballot(my_missing)) {
    const unsigned mw = wave_sum(my_missing);
    if (leader) add_u32(&vol.ctr->lookup_misses, mw);
  }
  if (__ballot(my_probe_max)) {
    const unsigned pm = wave_max(my_probe_max);
    // a plain read filters almost every update; the atomic keeps the maximum exact
    if (leader && pm > *(volatile unsigned*)&vol.ctr->max_probe)
      __hip_atomic_fetch_max(&vol.ctr->max_probe, pm, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// One workgroup = one 32x8 tile of F consecutive frames of the launch's NB
// frames: workgroup g covers tile g % n_tiles of frames F * (g / n_tiles) + 0..F-1
// (frames past the batch are empty).  F > 1 sums the frames' contributions to a
// tile before they reach the pool; NB > F puts several frames in one grid so
// one frame's start-up overlaps another's pool updates.
// Colour volumes accumulate 2.5x the floats per block in LDS: 4 blocks per
// pass keep the tile's LDS at 48 KiB.
constexpr int kColourAccBlocks = 4;
constexpr int acc_blocks_for(bool colour) { return colour ? kColourAccBlocks : kAccBlocks; }

template <int K, int F, int NB, FuseMode kMode, bool kColour, bool kLong = false>
__global__ __launch_bounds__(kThreads)
__attribute__((amdgpu_waves_per_eu(waves_per_eu_for(F, kColour))))
void fuse_kernel(FuseArgs<NB> args) {
  constexpr int AB = acc_blocks_for(kColour);
  __shared__ TileShared<AB, kColour> sh;
  // the argument segment seen through the constant address space (the
  // compiler keeps the address space through the cast, so reads stay scalar)
  const FuseArgs<NB>& A =
      *(const FuseArgs<NB>*)(ConstPtr<FuseArgs<NB>>)__builtin_amdgcn_kernarg_segment_ptr();
  const unsigned n_tiles = A.n_tiles, tiles_x = A.tiles_x;
  const unsigned group = blockIdx.x / n_tiles;
  const unsigned tile = tile_of_group(blockIdx.x % n_tiles, n_tiles, A.remap != 0);
  const unsigned x = (tile % tiles_x) * kTileW + (threadIdx.x % kTileW);
  const unsigned y = (tile / tiles_x) * kTileH + (threadIdx.x / kTileW);
  // the group's frames, read where they are used from the argument segment
  // rather than copied (a copy of three frames would hold 66 scalar registers
  // for the whole tile); a frame past the batch gets a pixel column past any
  // width, so it has no point and adds nothing
  const ArgFrames<(F > 1)> frs{(ConstPtr<FrameDev>)(const FrameDev*)A.f, group * F};
  unsigned px[F], py[F];
#pragma unroll
  for (int fi = 0; fi < F; ++fi) {
    px[fi] = group * F + fi < A.n_frames ? x : ~0u;
    py[fi] = y;
  }
  // several frames per workgroup: the trajectory launches that reach the
  // memory-side atomic ceiling flush in segment-aligned windows
  fuse_tile<K, F, AB, kMode, kColour, (F >= 2), kLong>(A.vol, A.wp, frs, px, py, blockIdx.x, sh);
}

// Many volumes, one frame each, in one persistent launch.  The grid is a
// fixed number of resident workgroups; workgroup g takes global tiles
// first + g, first + g + gridDim.x, ... of the items of band K (items sorted by
// K, tiles numbered by the prefix sum in the work list), finds each tile's item
// by bisection and runs the same tile steps as the one-volume kernel against
// that item's volume.  A tile is tw = 2^tw_log2 pixels wide and PPT * 256 / tw
// tall: each thread takes PPT pixels of one column, 256 / tw rows apart, so a
// wave covers 64 * PPT pixels and the workgroup sums 256 * PPT pixels'
// contributions before they reach the pool.
//
// The work list is read-only for the whole launch: it is read through the
// constant address space (ConstPtr).

// Four workgroups of a plain volume fit a CU's LDS, so registers are capped to
// match: 128 VGPRs (two pixels per thread fit without spilling).
// Colour workgroups take more LDS, three per CU: no cap.
constexpr int multi_waves_per_eu(bool colour) { return colour ? 1 : 4; }

template <int K, int PPT, int AB, bool kColour>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(multi_waves_per_eu(kColour))))
void fuse_multi_kernel(BatchWork w, unsigned tw_log2) {
  __shared__ TileShared<AB, kColour> sh;
  const ConstPtr<unsigned> k_begin = (ConstPtr<unsigned>)w.k_begin;
  const ConstPtr<unsigned> tile_start = (ConstPtr<unsigned>)w.tile_start;
  const ConstPtr<BatchItem> items = (ConstPtr<BatchItem>)w.items;
  constexpr int kGroup = batch_group(K, kColour);
  const unsigned first = k_begin[kGroup], last = k_begin[kGroup + 1];
  if (first >= last) return;
  const unsigned t_end = tile_start[last];
  const unsigned lx = threadIdx.x & ((1u << tw_log2) - 1u);
  const unsigned ly = threadIdx.x >> tw_log2;
  const unsigned rows = kThreads >> tw_log2;  // rows per pixel slot
  for (unsigned t = tile_start[first] + blockIdx.x; t < t_end; t += gridDim.x) {
    // the item i with tile_start[i] <= t < tile_start[i + 1]
    unsigned lo = first, hi = last;
    while (hi - lo > 1u) {
      const unsigned mid = (lo + hi) >> 1;
      if (tile_start[mid] <= t) lo = mid;
      else hi = mid;
    }
    const BatchItem& it = *(const BatchItem*)&items[lo];
    const unsigned local = t - tile_start[lo];
    const unsigned x = ((local % it.tiles_x) << tw_log2) + lx;
    const unsigned y0 = (local / it.tiles_x) * (rows * PPT) + ly;
    FrameDev frs[PPT];
    unsigned px[PPT], py[PPT];
#pragma unroll
    for (int p = 0; p < PPT; ++p) {
      frs[p] = it.fr;
      px[p] = x;
      py[p] = y0 + p * rows;
    }
    // latency-bound (its workloads sit below the atomic ceiling): fixed windows
    fuse_tile<K, PPT, AB, FuseMode::kFused, kColour, false>(it.vol, it.wp, HeldFrames<PPT>{frs},
                                                            px, py, blockIdx.x, sh);
  }
}

template <int K>
const void* multi_kernel_k(int pixels_per_thread, int acc_blocks, bool colour) {
  if (colour)  // one shape: one pixel per thread, the colour slot region
    return pixels_per_thread == 1 && acc_blocks == kColourAccBlocks
               ? reinterpret_cast<const void*>(&fuse_multi_kernel<K, 1, kColourAccBlocks, true>)
               : nullptr;
  if (pixels_per_thread == 1) {
    switch (acc_blocks) {
      case 4: return reinterpret_cast<const void*>(&fuse_multi_kernel<K, 1, 4, false>);
      case 8: return reinterpret_cast<const void*>(&fuse_multi_kernel<K, 1, 8, false>);
      default: return nullptr;
    }
  }
  if (pixels_per_thread == 2) {
    switch (acc_blocks) {
      case 8: return reinterpret_cast<const void*>(&fuse_multi_kernel<K, 2, 8, false>);
      default: return nullptr;
    }
  }
  return nullptr;
}

// Frames a workgroup may sum before flushing, keeping the per-pair state
// (F x (2K+1) registers) in registers: 4 for bands of up to 9 samples, 2 above.
constexpr int max_frames_for(int K) { return 2 * K + 1 <= 9 ? 4 : 2; }

// The long probe read-ahead is for tables that can fill: a pool of at least
// 80 % of the table.  Slot-index volumes keep the short read: their pool is the
// table by construction, so the ratio says nothing of the load they reach.
inline bool long_probe(const VolumeDev& vol) {
  return !vol.slot_index &&
         (unsigned long long)vol.pool_capacity * 5ull >= (unsigned long long)vol.table_capacity * 4ull;
}

template <int K, int F, int NB, bool kColour>
hipError_t launch_fuse_kf(VolumeDev vol, const WalkParams& wp, const FrameDev* frames, int n,
                          FuseMode mode, bool remap, hipStream_t s) {
  FuseArgs<NB> args;
  args.vol = vol;
  args.wp = wp;
  unsigned w = 0, h = 0;
  for (int i = 0; i < frame_slots(NB); ++i) {
    args.f[i] = frames[i < n ? i : 0];
    if (i < n) {
      w = frames[i].width > w ? frames[i].width : w;
      h = frames[i].height > h ? frames[i].height : h;
    }
  }
  const unsigned tx = (w + kTileW - 1) / kTileW;
  const unsigned ty = (h + kTileH - 1) / kTileH;
  const unsigned n_tiles = tx * ty;
  if (n_tiles == 0) return hipSuccess;
  args.n_frames = (unsigned)n;
  args.tiles_x = tx;
  args.n_tiles = n_tiles;
  args.remap = remap ? 1 : 0;
  const unsigned groups = ((unsigned)n + F - 1) / F;
  const dim3 grid(n_tiles * groups), block(kThreads);
  const bool lp = long_probe(vol);
  if constexpr (F == 1 && NB == 1) {
    switch (mode) {
      case FuseMode::kFused:
        if (lp)
          hipLaunchKernelGGL((fuse_kernel<K, 1, 1, FuseMode::kFused, kColour, true>), grid, block,
                             0, s, args);
        else
          hipLaunchKernelGGL((fuse_kernel<K, 1, 1, FuseMode::kFused, kColour, false>), grid,
                             block, 0, s, args);
        break;
      case FuseMode::kAllocate:  // allocation touches no accumulator
        if (lp)
          hipLaunchKernelGGL((fuse_kernel<K, 1, 1, FuseMode::kAllocate, false, true>), grid,
                             block, 0, s, args);
        else
          hipLaunchKernelGGL((fuse_kernel<K, 1, 1, FuseMode::kAllocate, false, false>), grid,
                             block, 0, s, args);
        break;
      case FuseMode::kIntegrate:
        if (lp)
          hipLaunchKernelGGL((fuse_kernel<K, 1, 1, FuseMode::kIntegrate, kColour, true>), grid,
                             block, 0, s, args);
        else
          hipLaunchKernelGGL((fuse_kernel<K, 1, 1, FuseMode::kIntegrate, kColour, false>), grid,
                             block, 0, s, args);
        break;
    }
  } else {
    (void)mode;
    if (lp)
      hipLaunchKernelGGL((fuse_kernel<K, F, NB, FuseMode::kFused, kColour, true>), grid, block, 0,
                         s, args);
    else
      hipLaunchKernelGGL((fuse_kernel<K, F, NB, FuseMode::kFused, kColour, false>), grid, block, 0,
                         s, args);
  }
  return hipGetLastError();
}

// n frames (1..kMaxBatchFrames) in one launch; frames_per_group frames summed
// per workgroup (1 to 4).  The two-pass stages are single-frame launches.
template <int K>
hipError_t launch_fuse_k(VolumeDev vol, const WalkParams& wp, const FrameDev* frames, int n,
                         int frames_per_group, FuseMode mode, bool remap, hipStream_t s) {
  if (n < 1 || n > kMaxBatchFrames) return hipErrorInvalidValue;
  if (mode != FuseMode::kFused && n != 1) return hipErrorInvalidValue;
  const bool colour = vol.colour != nullptr;
  if (n == 1)
    return colour ? launch_fuse_kf<K, 1, 1, true>(vol, wp, frames, 1, mode, remap, s)
                  : launch_fuse_kf<K, 1, 1, false>(vol, wp, frames, 1, mode, remap, s);
  if (colour) {
    // colour volumes: one or two frames per workgroup (the colour slot region
    // holds 1945 voxels; four frames of a tile would take several passes)
    if (frames_per_group == 1)
      return launch_fuse_kf<K, 1, kMaxBatchFrames, true>(vol, wp, frames, n, mode, remap, s);
    return launch_fuse_kf<K, 2, kMaxBatchFrames, true>(vol, wp, frames, n, mode, remap, s);
  }
  switch (frames_per_group) {
    case 1: return launch_fuse_kf<K, 1, kMaxBatchFrames, false>(vol, wp, frames, n, mode, remap, s);
    case 2: return launch_fuse_kf<K, 2, kMaxBatchFrames, false>(vol, wp, frames, n, mode, remap, s);
    case 3:
      if constexpr (max_frames_for(K) >= 3)
        return launch_fuse_kf<K, 3, kMaxBatchFrames, false>(vol, wp, frames, n, mode, remap, s);
      return hipErrorInvalidValue;
    case 4:
      if constexpr (max_frames_for(K) >= 4)
        return launch_fuse_kf<K, 4, kMaxBatchFrames, false>(vol, wp, frames, n, mode, remap, s);
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

}  // namespace
}  // namespace tsdf
