/*
 * tsdf.h -- C ABI of libtsdf.so: hash-blocked TSDF fusion on one AMD Instinct
 * MI355X (gfx950).
 *
 * The operation is the two-stage fusion kernel of "What Irregularity Costs"
 * (Section 2): an irregular *allocate* stage walks every depth point's truncation
 * band, maps each touched voxel to its 8^3 block, and makes sure the block exists
 * in an open-addressed, linear-probe hash table (16-byte entries keyed by the
 * packed 64-bit block coordinate of Section 2.1, inserted by compare-exchange
 * with the two-step publication of Section 2.3); a regular *integrate* stage
 * walks the same band and adds truncated signed distances and unit weights into a
 * flat structure-of-arrays voxel pool that stores sums, so that means are
 * recovered only at extraction (Section 2.2).
 *
 * Conventions for every call:
 *  - Every call returns a tsdf_status.  No call aborts, prints or throws.
 *  - Arguments that are invalid are detected on the host; the call then returns
 *    TSDF_ERR_INVALID_ARGUMENT and enqueues nothing.
 *  - Device memory is owned by the caller: the volume arena, batch workspace,
 *    depth frames and extraction outputs are device pointers the caller
 *    allocated (with hipMalloc, or a framework's allocator) and keeps alive
 *    while work that uses them may still run; depth frames may instead be
 *    pinned host memory passed at its device address, which the kernels then
 *    read over PCIe (tsdf_fuse_frame).  The library allocates no device
 *    memory at any time; it owns host handles, and a batch also owns a small
 *    pinned host staging ring, HIP events and HIP graphs (tsdf_batch_create).
 *  - `hip_stream` is a hipStream_t (NULL = the null stream).  All device work is
 *    enqueued on it in call order; only tsdf_query_status and
 *    tsdf_extract_blocks wait on it.  One volume must not be used from two
 *    streams at once.
 *  - Capacity problems met on the device (a full pool, a full table, voxel
 *    coordinates beyond the 21-bit key range) never lose data silently: they are
 *    counted, latched as sticky status bits in the volume, and reported by the
 *    next tsdf_query_status.
 */
#ifndef TSDF_H_
#define TSDF_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum tsdf_status {
  TSDF_OK = 0,
  TSDF_ERR_INVALID_ARGUMENT = 1,
  TSDF_ERR_BUFFER_TOO_SMALL = 2,  /* extraction output smaller than the block count */
  TSDF_ERR_POOL_EXHAUSTED = 3,    /* a new block found the pool full (sticky) */
  TSDF_ERR_TABLE_FULL = 4,        /* a key found neither itself nor a free slot (sticky) */
  TSDF_ERR_COORD_RANGE = 5,       /* a sample's voxel lies outside the key range (sticky) */
  TSDF_ERR_INTERNAL = 6,          /* an invariant broke on the device (sticky) */
  TSDF_ERR_HIP = 7,               /* a HIP runtime call failed */
  TSDF_ERR_BUDGET = 8,            /* a region, queue or session table has no room */
  /* not a status: keeps the type 32 bits wide, so that every non-negative
   * code a caller hands back (tsdf_status_str) is a value of the type */
  TSDF_STATUS_RANGE_ = 0x7FFFFFFF
} tsdf_status;

/* Sticky status bits, as returned in tsdf_stats.status_bits. */
#define TSDF_FLAG_POOL_EXHAUSTED 0x1u
#define TSDF_FLAG_TABLE_FULL 0x2u
#define TSDF_FLAG_COORD_RANGE 0x4u
#define TSDF_FLAG_INTERNAL 0x8u
/* More distinct keys found the table full than the volume's record of them
 * holds (TSDF_OVERFLOW_KEY_SLOTS): keys_table_overflow is then a lower bound. */
#define TSDF_FLAG_OVERFLOW_RECORD_FULL 0x10u

/* Block and table geometry (Section 2.1). */
#define TSDF_BLOCK_EDGE 8u
#define TSDF_BLOCK_VOXELS 512u
#define TSDF_EMPTY_KEY 0xFFFFFFFFFFFFFFFFull /* never a packed key: those use 63 bits */
#define TSDF_MAX_POOL_BLOCKS ((1u << 22) - 1u) /* keeps voxel indices below 2^31 */
#define TSDF_MAX_BAND_HALF 8 /* round(trunc / voxel_size) must lie in [1, 8] */
/* Distinct keys a volume can record as having found its table full (Sections
 * 3.4 and 7.2: probe exhaustion is accounted, never silent). */
#define TSDF_OVERFLOW_KEY_SLOTS 8192u

/* Volume variants (tsdf_volume_params.flags), from Sections 6.4 and 2.1:
 *   TSDF_VOLUME_SLOT_INDEX  a block's pool index is its hash-table slot
 *       (the location derived from the slot): no pool counter to win and
 *       no index to wait for, at the cost of a pool as large as the table.
 *       pool_capacity must equal the table capacity; table_capacity 0 means
 *       "equal to pool_capacity" here.  The pool cannot run out.
 *   TSDF_VOLUME_COLOUR  three more accumulators per voxel, the red, green and
 *       blue sums of the colour of every contribution (Section 2.1: five
 *       parallel arrays); frames then come with a colour image
 *       (tsdf_fuse_frame_rgb, tsdf_fuse_item.rgba_dev). */
#define TSDF_VOLUME_SLOT_INDEX 0x1u
#define TSDF_VOLUME_COLOUR 0x2u
/* Instrumentation, not a design variant: the volume also counts, for every
 * resolution of a tile's block key against the table (Section 2.3's probe),
 * its probe distance in a histogram read by tsdf_probe_histogram.  Costs one
 * device atomic per resolution; results are otherwise unchanged. */
#define TSDF_VOLUME_PROBE_HISTOGRAM 0x4u

typedef struct tsdf_volume_params {
  float voxel_size;        /* voxel edge in metres, finite and > 0 */
  float trunc;             /* truncation distance tau in metres, finite and
                              >= voxel_size; the band walk takes 2K+1 samples,
                              K = round(trunc/voxel_size), and K must lie in
                              [1, TSDF_MAX_BAND_HALF] */
  uint32_t table_capacity; /* hash-table slots C >= 1 (any value, not only powers
                              of two); 0 selects the paper's sizing, the next power
                              of two >= 2 * pool_capacity (Section 2.1) */
  uint32_t pool_capacity;  /* voxel blocks P, 1 .. TSDF_MAX_POOL_BLOCKS */
  uint32_t flags;          /* TSDF_VOLUME_* (0: the paper's main design) */
} tsdf_volume_params;

typedef struct tsdf_camera {
  uint32_t width, height;  /* depth image size; width * height <= 2^31 */
  float fx, fy, cx, cy;    /* pinhole intrinsics in pixels, finite, fx, fy != 0;
                              pixel (x, y) looks along ((x - cx)/fx, (y - cy)/fy, 1) */
  float pose[12];          /* camera->world [R | t], row-major 3x4, finite
                              (R = pose[0..2], pose[4..6], pose[8..10]) */
} tsdf_camera;

/* Counters of a volume (Section 3.4: pool exhaustion reported; Section 7.2:
 * probe exhaustion accounted).  Cumulative since tsdf_create_volume /
 * tsdf_reset_volume, except blocks_new. */
typedef struct tsdf_stats {
  uint64_t points_valid;       /* pixels with finite depth > 0 that were fused */
  uint64_t pairs;              /* (point, voxel) contributions that passed the walk */
  uint64_t pairs_dropped;      /* contributions lost to a full pool or table */
  uint64_t coord_out_of_range; /* band samples whose voxel cannot be keyed */
  uint32_t blocks_total;       /* allocated pool blocks, <= pool_capacity */
  uint32_t blocks_new;         /* blocks allocated since the previous
                                  tsdf_query_status of this volume (or since its
                                  creation or reset) */
  uint32_t keys_pool_overflow; /* distinct keys that found the pool full */
  uint32_t keys_table_overflow;/* distinct keys that found the table full (exact
                                  up to TSDF_OVERFLOW_KEY_SLOTS; beyond that a
                                  lower bound, flagged TSDF_FLAG_OVERFLOW_RECORD_FULL) */
  uint32_t table_full_events;  /* failed resolutions against a full table (one per
                                  workgroup tile and key, so a key can count more
                                  than once) */
  uint32_t max_probe;          /* longest probe distance met (slots past home) */
  uint32_t lookup_misses;      /* two-pass mode: integrate found no key */
  uint32_t status_bits;        /* TSDF_FLAG_* */
  uint32_t frames;             /* frames fused */
  uint32_t reserved;
} tsdf_stats;

/* Byte offsets of the regions carved from the caller's arena; all 256-aligned.
 *   counters   : 8192 bytes of device counters (internal format)
 *   table      : table_capacity entries of 16 bytes: {uint64 key; int32 block;
 *                uint32 pad}, key TSDF_EMPTY_KEY when free; block >= 0 is a pool
 *                index, -1 = being published, -2 = the pool was full
 *   overflow_keys : TSDF_OVERFLOW_KEY_SLOTS uint64, an open-addressed set of
 *                the keys that found the table full (TSDF_EMPTY_KEY when free)
 *   block_keys : pool_capacity uint64, the key of the i-th allocated block
 *   alloc_list : (TSDF_VOLUME_SLOT_INDEX only) pool_capacity uint32, the pool
 *                index (= table slot) of the i-th allocated block; without the
 *                flag the i-th allocated block is pool block i
 *   voxels     : pool_capacity * 1024 float, the voxel pool.  A block is 64
 *                segments of 64 bytes; voxel (lx, ly, lz) of block b lies in
 *                segment g = ((ly % 4) * 2 + (lz / 2) % 2) * 8 + (lz / 4) * 4 +
 *                (ly / 4) * 2 + lx / 4, at place e = (lz % 2) * 4 + lx % 4, and
 *                a segment holds its 8 TSDF sums then its 8 weights:
 *                  TSDF sum : voxels[b * 1024 + g * 16 + e]
 *                  weight   : voxels[b * 1024 + g * 16 + 8 + e]
 *                (a segment is a 4 x 1 x 2 box of voxels, so that one 64-byte
 *                memory request updates both accumulators of 8 neighbours).
 *                Weights count contributions; TSDF values are sums (the mean is
 *                sum / weight).  tsdf_extract_blocks returns plain arrays in the
 *                canonical in-block order loc = (lz * 8 + ly) * 8 + lx.
 *   colour     : (TSDF_VOLUME_COLOUR only) pool_capacity * 1536 float: per
 *                block 64 segments of 24 floats, the segment's 8 red, 8 green,
 *                8 blue sums (colour values 0..255):
 *                  red sum : colour[b * 1536 + g * 24 + e], green + 8, blue + 16
 *                Regions a volume does not use have size 0. */
typedef struct tsdf_layout {
  uint64_t counters, table, overflow_keys, block_keys, alloc_list, voxels, colour, total_bytes;
  uint32_t table_capacity, pool_capacity, flags, reserved;
} tsdf_layout;

typedef struct tsdf_volume tsdf_volume;

/* Arena bytes the volume needs; 0 if `params` is invalid. */
size_t tsdf_volume_bytes(const tsdf_volume_params* params);

/* Region offsets for `params` (see tsdf_layout). */
tsdf_status tsdf_volume_layout(const tsdf_volume_params* params, tsdf_layout* out);

/* Make a volume over the caller's device arena (>= tsdf_volume_bytes bytes,
 * 256-byte aligned) and enqueue its initialisation on `hip_stream`: empty table,
 * zero pool, zero counters.  *out receives a host handle. */
tsdf_status tsdf_create_volume(const tsdf_volume_params* params, void* dev_arena,
                               size_t arena_bytes, void* hip_stream, tsdf_volume** out);

/* Free the host handle.  The arena is the caller's and is not touched. */
tsdf_status tsdf_destroy_volume(tsdf_volume* vol);

/* Enqueue an empty table, zero counters and zeroed pool blocks (only the
 * blocks that were handed out are cleared; the rest are still zero). */
tsdf_status tsdf_reset_volume(tsdf_volume* vol, void* hip_stream);

/* Fuse one depth frame (Section 2.2: allocate then integrate).  `depth_dev` is
 * height x width float32 metres, row-major, camera-frame z; pixels that are not
 * finite or not > 0 are not points.  It may be device memory or pinned host
 * memory at its device address (hipHostGetDevicePointer); the kernels read
 * each pixel once, so a pinned frame is read over PCIe with no copy.
 * Asynchronous: returns once enqueued; the frame must stay valid until the
 * fusion completes. */
tsdf_status tsdf_fuse_frame(tsdf_volume* vol, const float* depth_dev, const tsdf_camera* cam,
                            void* hip_stream);

/* As tsdf_fuse_frame with a choice of kernel structure:
 *   TSDF_FUSE_DEFAULT   one fused launch (allocate and integrate per workgroup)
 *   TSDF_FUSE_TWO_PASS  two launches, allocate over all points then integrate
 *                       over all points, as in Section 2.2
 *   TSDF_FUSE_ALLOCATE_ONLY / TSDF_FUSE_INTEGRATE_ONLY  one stage of TWO_PASS
 *                       (for stage timing; integrate-only assumes the frame's
 *                       blocks were allocated before)
 *   | TSDF_FUSE_XCD_REMAP  give each of the 8 XCDs a contiguous band of tiles
 *                       instead of the hardware's round-robin of row-major tiles
 * Results are identical for every choice (up to float summation order). */
#define TSDF_FUSE_DEFAULT 0u
#define TSDF_FUSE_TWO_PASS 1u
#define TSDF_FUSE_ALLOCATE_ONLY 2u
#define TSDF_FUSE_INTEGRATE_ONLY 3u
#define TSDF_FUSE_MODE_MASK 3u
#define TSDF_FUSE_XCD_REMAP 0x100u
tsdf_status tsdf_fuse_frame_ex(tsdf_volume* vol, const float* depth_dev, const tsdf_camera* cam,
                               uint32_t flags, void* hip_stream);

/* As tsdf_fuse_frame_ex, for a TSDF_VOLUME_COLOUR volume: `rgba_dev` is a
 * height x width array of packed 8-bit colours (red | green << 8 |
 * blue << 16; the top byte is ignored) registered with the depth image; every
 * contribution also adds its pixel's red, green and blue values to the
 * voxel's colour sums.  Colour volumes take frames only through this call and
 * through tsdf_batch_fuse; tsdf_fuse_frame, _ex and tsdf_fuse_frames refuse
 * them (TSDF_ERR_INVALID_ARGUMENT).  rgba_dev may be NULL only for an empty
 * frame. */
tsdf_status tsdf_fuse_frame_rgb(tsdf_volume* vol, const float* depth_dev, const uint32_t* rgba_dev,
                                const tsdf_camera* cam, uint32_t flags, void* hip_stream);

/* Fuse `n_frames` depth frames into the volume, up to 32 frames per launch:
 * the tiles of all frames of a launch share one grid, so one frame's start-up
 * overlaps another's pool updates.  Each workgroup takes the same 32x8 pixel
 * tile of F consecutive frames and sums their contributions in LDS before
 * adding them to the pool, so frames of one trajectory that see the same
 * surface share pool updates.  F is set by TSDF_FUSE_BATCH(m): m = 1, 2 or 3
 * -> m, m >= 4 -> 4, and m = 0 (the default) -> 3; F is capped at 2 when
 * round(trunc/voxel_size) > 4.  The result is that of fusing the frames
 * one by one with tsdf_fuse_frame, in any order (keys and weights identical,
 * TSDF sums up to float summation order).
 *   depth_devs  host array of n_frames device-accessible pointers (height x
 *               width float32; device memory or pinned host memory, as for
 *               tsdf_fuse_frame)
 *   cams        host array of n_frames cameras (sizes may differ)
 *   flags       TSDF_FUSE_XCD_REMAP and/or TSDF_FUSE_BATCH(m), m in 0..15
 * A colour volume is TSDF_ERR_INVALID_ARGUMENT (its frames carry colour
 * images: tsdf_fuse_frames_rgb).  Asynchronous, like tsdf_fuse_frame. */
#define TSDF_FUSE_BATCH_SHIFT 16
#define TSDF_FUSE_BATCH_MASK (0xFu << TSDF_FUSE_BATCH_SHIFT)
#define TSDF_FUSE_BATCH(m) (((uint32_t)(m) & 0xFu) << TSDF_FUSE_BATCH_SHIFT)
tsdf_status tsdf_fuse_frames(tsdf_volume* vol, uint32_t n_frames, const float* const* depth_devs,
                             const tsdf_camera* cams, uint32_t flags, void* hip_stream);

/* Staged accumulation of many frames of one volume (Section 2.2: the integrate
 * stage is a sum of contributions, so it can be gathered before it reaches the
 * pool).  As tsdf_fuse_frames, 32 frames per launch, but a launch's tiles do
 * not add their contributions to the pool: each tile writes one 4-byte record
 * per contribution (the voxel and its truncated distance, carried in 23-bit
 * fixed point of trunc: to within trunc / 2^23), grouped by block, into the
 * caller's staging memory, and lists each of its (tile, block) runs in that
 * block's run table (one device atomic per tile and block).  An apply kernel
 * then sums each block's records per voxel, one work item per 1024 records of
 * a block, and adds the sums to its pool segments with one memory-side
 * request per touched 64-byte segment and item.  Runs that do not fit a block's table of 128, or a
 * launch's records beyond the staging memory, go to the pool directly with
 * device atomics, so any size is correct; the size only decides how much is
 * staged.  The staging memory holds two sets used by alternate launches, and
 * the apply kernels run on a second stream of the device (default priority,
 * made on first use and kept for the process), so that a launch's tile kernel
 * overlaps the previous launch's apply; the caller's stream waits for every
 * apply before the call's later work.  The result is that of fusing the frames
 * one by one with tsdf_fuse_frame (keys and weights identical, TSDF sums up to
 * float summation order and the fixed-point carry).  Plain volumes only
 * (colour volumes: TSDF_ERR_INVALID_ARGUMENT).  Calls from several host
 * threads are serialised while they enqueue.
 *   staging_dev    caller-owned device memory, 256-byte aligned, of at least
 *                  tsdf_staging_bytes(pool_capacity, 65536) bytes for the
 *                  volume's pool (else TSDF_ERR_BUFFER_TOO_SMALL, nothing
 *                  enqueued); what it holds beyond that sets the records per
 *                  launch (a launch of 32 frames of W x H pixels makes at most
 *                  32 * W * H * (2K + 1)).  Its contents need no initialisation
 *                  and are meaningless after the call; it may serve any volume of
 *                  at most that pool, one call at a time (calls on one stream are
 *                  ordered).
 *   flags          TSDF_FUSE_BATCH(1): one frame per workgroup; otherwise two
 *                  (one when round(trunc/voxel_size) > 4).
 *                  TSDF_FUSE_ONE_STREAM: every kernel on hip_stream (no second
 *                  stream, no overlap).
 * Asynchronous, like tsdf_fuse_frame.
 * tsdf_staging_bytes: the staging bytes for a pool of pool_capacity blocks
 * (1 .. TSDF_MAX_POOL_BLOCKS) and `records` records per launch (2^16 .. 2^32 -
 * 1); 0 for other values. */
#define TSDF_FUSE_ONE_STREAM 0x200u
size_t tsdf_staging_bytes(uint32_t pool_capacity, uint64_t records);
tsdf_status tsdf_fuse_frames_staged(tsdf_volume* vol, uint32_t n_frames,
                                    const float* const* depth_devs, const tsdf_camera* cams,
                                    uint32_t flags, void* staging_dev, size_t staging_bytes,
                                    void* hip_stream);

/* tsdf_fuse_frames for colour volumes (TSDF_VOLUME_COLOUR): frame i also adds
 * the colours of rgba_devs[i] (height x width packed red | green << 8 |
 * blue << 16, as for tsdf_fuse_frame_rgb) to the voxels its pairs touch.  F is
 * set as for tsdf_fuse_frames but at most 2: the colour slot region holds 1945
 * voxels per pass.  The result is that of fusing the frames one by one with
 * tsdf_fuse_frame_rgb (keys, weights and colour sums identical, TSDF sums up
 * to float summation order).  A plain volume, or a null rgba_devs (or entry
 * for a frame with pixels), is TSDF_ERR_INVALID_ARGUMENT.
 *   rgba_devs   host array of n_frames device-accessible pointers
 * Asynchronous, like tsdf_fuse_frame. */
tsdf_status tsdf_fuse_frames_rgb(tsdf_volume* vol, uint32_t n_frames,
                                 const float* const* depth_devs,
                                 const uint32_t* const* rgba_devs, const tsdf_camera* cams,
                                 uint32_t flags, void* hip_stream);

/* Wait for `hip_stream`, read the counters and return the most severe sticky
 * condition (INTERNAL > TABLE_FULL > POOL_EXHAUSTED > COORD_RANGE), or TSDF_OK.
 * `out` may be NULL. */
tsdf_status tsdf_query_status(tsdf_volume* vol, void* hip_stream, tsdf_stats* out);

/* Probe-distance histogram of a TSDF_VOLUME_PROBE_HISTOGRAM volume since its
 * creation or last reset.  A resolution is one (workgroup tile, distinct block
 * key) of a fused frame; its distance is the number of slots past the key's
 * home where the probe found the key or claimed a slot for it.
 *   bins            host array of TSDF_PROBE_HIST_BINS: bins[0] counts
 *                   resolutions at distance 0, bins[b] for b >= 1 those at
 *                   a distance in [2^(b-1), 2^b), the last bin open-ended
 *   total_distance  optional (NULL): the distances summed
 * Waits for `hip_stream` like tsdf_query_status.  INVALID_ARGUMENT if the
 * volume was made without the flag or `bins` is NULL; nothing is written
 * then. */
#define TSDF_PROBE_HIST_BINS 16u
tsdf_status tsdf_probe_histogram(tsdf_volume* vol, void* hip_stream, uint64_t* bins,
                                 uint64_t* total_distance);

/* Wait for `hip_stream` to learn the block count n, then, if n <= max_blocks,
 * enqueue the extraction of every allocated block in pool order:
 *   keys_dev[i]          packed key of pool block i          (n uint64)
 *   tsdf_dev[i*512 + l]  mean TSDF = sum / weight, 0 where the weight is 0
 *   weight_dev[i*512+l]  weight                              (n * 512 float)
 * Any output pointer may be NULL to skip it.  *n_blocks_out = n always.
 * Returns TSDF_ERR_BUFFER_TOO_SMALL (nothing enqueued) if n > max_blocks.  The
 * outputs are complete once `hip_stream` has drained. */
tsdf_status tsdf_extract_blocks(tsdf_volume* vol, void* hip_stream, uint32_t max_blocks,
                                uint64_t* keys_dev, float* tsdf_dev, float* weight_dev,
                                uint32_t* n_blocks_out);

/* Colour volumes: as tsdf_extract_blocks, the mean colour of every allocated
 * block in the same order: rgb_dev[(i * 512 + loc) * 3 + c] = colour sum c /
 * weight (0 where the weight is 0), c = 0, 1, 2 for red, green, blue, values
 * in 0..255.  TSDF_ERR_INVALID_ARGUMENT for a volume without colour. */
tsdf_status tsdf_extract_colour(tsdf_volume* vol, void* hip_stream, uint32_t max_blocks,
                                float* rgb_dev, uint32_t* n_blocks_out);

/* Surface extraction: the zero crossing of the mean TSDF as a triangle mesh,
 * by marching tetrahedra over the voxel centres (the extraction the paper
 * runs after fusion and leaves out of its timing, Section 2.4; Section 3.3
 * checks its output).
 *   - Samples are voxel centres ((i + 1/2) * voxel_size per axis, metres) with
 *     value sum / weight.  A cube of 8 neighbouring centres is meshed only
 *     when all 8 voxels have a weight, and is skipped when it changes sign
 *     while a corner's |value| >= (1 - 2^-10) * trunc (a jump at an occlusion
 *     edge, not a surface).
 *   - Each cube is cut into the 6 tetrahedra around its corner-0 to corner-7
 *     diagonal (corner c has offset (c & 1, (c >> 1) & 1, c >> 2)).  A corner
 *     is inside when its value is < 0.  Vertices are interpolated linearly on
 *     crossing edges; triangles are wound with the normal towards positive
 *     values (free space).
 * Waits for `hip_stream` twice (block count, triangle count).  Triangle i
 * writes vertices_dev[9i .. 9i+8] (three x, y, z vertices, float32) and, if
 * ids_dev is not NULL, ids_dev[2i] = its block's packed key and
 * ids_dev[2i+1] = cube << 4 | tetrahedron << 1 | triangle (cube = the
 * in-block index of its lowest corner, as for voxels).  Triangles come in no
 * particular order; their identities are unique.  *n_triangles_out = the
 * number of triangles found; if it exceeds max_triangles, only max_triangles
 * are written and TSDF_ERR_BUFFER_TOO_SMALL is returned.  vertices_dev may be
 * NULL only when max_triangles is 0 (a count). */
tsdf_status tsdf_extract_mesh(tsdf_volume* vol, void* hip_stream, uint32_t max_triangles,
                              float* vertices_dev, uint64_t* ids_dev, uint32_t* n_triangles_out);

/* Measurement only (no volume): the memory-side rate of the device-scope fp32
 * atomic adds with which fusion flushes its sums into the pool.  Launches
 * `waves` waves (a multiple of 4, at most 2^24); each issues `iters` (at most
 * 2^16) instructions, and each instruction adds 1.0 to `lanes_per_row`
 * consecutive floats at the start of each of `rows_per_instr` 64-byte rows of
 * `buf_dev`, picked pseudo-randomly.  That is waves * iters * rows_per_instr
 * requests.  lanes_per_row is 1..16, and rows_per_instr * lanes_per_row is at
 * most 64.  `bytes` (a multiple of 64, at least 64) bounds the rows; the
 * buffer's contents are changed.  Asynchronous on `hip_stream`: the caller
 * times it with events. */
tsdf_status tsdf_measure_atomic_rate(float* buf_dev, uint64_t bytes, uint32_t waves,
                                     uint32_t iters, uint32_t rows_per_instr,
                                     uint32_t lanes_per_row, void* hip_stream);

/* Allocate pool blocks for `n` block coordinates (device array of n rows of
 * int32 bx, by, bz, each in [-2^20, 2^20)) through the same insertion protocol
 * as fusion, as if a frame had touched them.  Used to pre-fill a table to a
 * chosen load factor.  Coordinates out of range are counted as
 * coord_out_of_range and skipped. */
tsdf_status tsdf_insert_blocks(tsdf_volume* vol, const int32_t* block_coords_dev, uint32_t n,
                               void* hip_stream);

/* ---------------------------------------------------------------------------
 * Multi-volume batches.  One call fuses one frame into each of many
 * independent volumes (one frame per item; an item may repeat a volume) with
 * one persistent launch per band half-width present: a fixed grid of resident
 * workgroups strides over the 16x16-pixel (or 32x8, 64x4) tiles of every
 * item's frame, each tile running the same allocate-then-integrate steps as
 * tsdf_fuse_frame against its own volume.  Each volume ends as if its items
 * had been fused alone with tsdf_fuse_frame (keys and weights identical, TSDF
 * sums up to float summation order); each volume's counters and sticky status
 * are its own.
 *
 * The work list lives in a caller-owned device workspace; the kernels read
 * their item ranges from it, so once the configuration is fixed the launches
 * are kept as one instantiated HIP graph and replayed every call whatever the
 * number and sizes of the items.  A batch is bound to the device current at
 * tsdf_batch_create and is not thread-safe.
 * ------------------------------------------------------------------------- */
typedef struct tsdf_batch tsdf_batch;

typedef struct tsdf_fuse_item {
  tsdf_volume* volume;      /* target volume */
  const float* depth_dev;   /* height x width float32, as for tsdf_fuse_frame
                               (device memory or pinned host memory) */
  const uint32_t* rgba_dev; /* colour volumes: height x width packed colours, as
                               for tsdf_fuse_frame_rgb; ignored otherwise */
  tsdf_camera camera;
} tsdf_fuse_item;

/* The work partition of a batch launch.  A workgroup of 256 threads takes a
 * tile tile_width pixels wide and pixels_per_thread * 256 / tile_width tall;
 * each thread takes pixels_per_thread pixels of one column, so a wave covers
 * 64 * pixels_per_thread points.  The workgroup sums the tile's contributions
 * in LDS, one slot per touched voxel, before adding them to the pool; the LDS
 * region is acc_blocks voxel blocks' worth of floats plus 4 KiB, which holds
 * 1280 voxel slots per pass with 4 and 3328 with 8 (colour volumes take a
 * fixed 48 KiB region of 1945 slots).  A tile that touches more voxels takes
 * more passes. */
typedef struct tsdf_batch_config {
  uint32_t tile_width;         /* 16, 32 or 64 */
  uint32_t pixels_per_thread;  /* 1 or 2 */
  uint32_t acc_blocks;         /* LDS region: 4 or 8 (8 with 2 pixels per thread) */
  uint32_t groups_per_cu;      /* workgroups of the persistent grid per compute
                                  unit; 0 = as many as can be resident */
} tsdf_batch_config;

/* Device workspace bytes for batches of up to `max_items` items (0 if
 * max_items is 0 or above TSDF_BATCH_MAX_ITEMS).  The workspace holds eight
 * work lists, one per slot of the batch's staging ring, so that calls from
 * several streams may overlap: a slot's list is rewritten only behind the
 * launches that last read it (a device-side wait on their event). */
#define TSDF_BATCH_MAX_ITEMS 65536u
size_t tsdf_batch_workspace_bytes(uint32_t max_items);

/* Make a batch over the caller's device workspace (>= the bytes above,
 * 256-byte aligned).  The batch starts with the autotuner on: its first calls
 * of tsdf_batch_fuse cycle through the candidate configurations (tile widths,
 * pixels per thread and LDS blocks per pass at full residency, and a few at
 * half residency), time each on the stream with HIP events, and then keep the
 * fastest per pixel.  Results do not depend on the configuration. */
tsdf_status tsdf_batch_create(uint32_t max_items, void* workspace_dev, size_t workspace_bytes,
                              tsdf_batch** out);

/* Release the host handle, its staging ring, events and graphs (waits for the
 * batch's outstanding uploads).  The workspace is the caller's. */
tsdf_status tsdf_batch_destroy(tsdf_batch* batch);

/* Fix the configuration (stops any tuning) or restart the autotuner with
 * `trials` timed calls per candidate (1..16). */
tsdf_status tsdf_batch_set_config(tsdf_batch* batch, const tsdf_batch_config* config);
tsdf_status tsdf_batch_autotune(tsdf_batch* batch, uint32_t trials);

/* The configuration the next call uses; *tuned = 1 once it is fixed.  Reads
 * the timings of finished tuning calls without waiting for pending ones. */
tsdf_status tsdf_batch_get_config(tsdf_batch* batch, tsdf_batch_config* config, uint32_t* tuned);

/* The autotuner's candidates and the least time per pixel it has measured
 * for each (nanoseconds; infinity if not yet measured).  Up to `max` entries
 * are written; *n_out receives the number of candidates.  Either output array
 * may be NULL. */
tsdf_status tsdf_batch_candidates(tsdf_batch* batch, uint32_t max, tsdf_batch_config* configs,
                                  double* ns_per_pixel, uint32_t* n_out);

/* Fuse items[i].depth_dev into items[i].volume for i < n_items (n_items <= the
 * batch's max_items): copies the work list to the workspace (a small
 * host-to-device copy from the staging ring) and launches, both on
 * `hip_stream`.  Asynchronous.  Calls may come from several streams (each
 * call uses its own work-list slot); a volume may appear in calls on several
 * streams at once, whose launches then fuse into it concurrently (the result
 * is the same, up to float summation order).
 *   flags  TSDF_BATCH_NO_GRAPH: launch directly even once the configuration is
 *          fixed (by default a fixed configuration replays a HIP graph). */
#define TSDF_BATCH_NO_GRAPH 0x1u
tsdf_status tsdf_batch_fuse(tsdf_batch* batch, const tsdf_fuse_item* items, uint32_t n_items,
                            uint32_t flags, void* hip_stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): tsdf_batch_fuse with its
 * work list in a device array of TSDF_STATIC_LIST_BYTES that the library holds
 * for the life of the process on each device it runs on, instead of in the
 * batch's workspace.  The call allocates no memory, device or host; it copies
 * the work list from the batch's pinned staging ring and launches directly
 * (never a graph, never a tuning trial) with the batch's current
 * configuration.  Results are those of tsdf_batch_fuse.
 *   - The list takes 256 + 4 * (max_items + 1) bytes, rounded up to a multiple
 *     of 256, plus 192 bytes per item (max_items of the batch); a call whose
 *     list would not fit returns TSDF_ERR_BUFFER_TOO_SMALL with nothing
 *     enqueued.
 *   - The current device must be the batch's (TSDF_ERR_INVALID_ARGUMENT).
 *   - Every call on a device shares that device's array and leaves its list
 *     there: calls on one stream are ordered, calls that overlap on one GPU
 *     (from different streams or threads) race and must not be made. */
#define TSDF_STATIC_LIST_BYTES (1u << 20)
tsdf_status tsdf_batch_fuse_static(tsdf_batch* batch, const tsdf_fuse_item* items,
                                   uint32_t n_items, void* hip_stream);

/* ---------------------------------------------------------------------------
 * Device-region sub-allocator.  Carves 256-byte-aligned ranges out of one
 * caller-owned device region (first fit, neighbouring free ranges merged).
 * Host bookkeeping only: the region's memory is never read or written, and
 * every call works without a GPU.  Not thread-safe.
 * ------------------------------------------------------------------------- */
typedef struct tsdf_region tsdf_region;

/* Manage [device_base, device_base + bytes); the usable part starts at the
 * first 256-byte boundary and is a whole number of 256-byte units. */
tsdf_status tsdf_region_create(void* device_base, uint64_t bytes, tsdf_region** out);
tsdf_status tsdf_region_destroy(tsdf_region* region);

/* A range of at least `bytes` (rounded up to 256); TSDF_ERR_BUDGET if no free
 * range is large enough. */
tsdf_status tsdf_region_alloc(tsdf_region* region, uint64_t bytes, void** out);

/* Return a range from tsdf_region_alloc; anything else is rejected with
 * TSDF_ERR_INVALID_ARGUMENT. */
tsdf_status tsdf_region_free(tsdf_region* region, void* ptr);

/* Usable bytes, bytes handed out, the largest free range and the number of
 * live ranges; any output may be NULL. */
tsdf_status tsdf_region_usage(const tsdf_region* region, uint64_t* capacity, uint64_t* used,
                              uint64_t* largest_free, uint32_t* n_live);

/* ---------------------------------------------------------------------------
 * Serving.  A server holds many reconstruction sessions, each one resident
 * volume carved from a device budget, and fuses the frames submitted to them
 * with continuous batching: each launch takes every queued frame (up to
 * max_batch, first come first served, any mix of sessions) through the batch
 * path above (a lone frame through tsdf_fuse_frame), and a new launch starts
 * whenever fewer than max_inflight are running.  A session's result is the
 * one it would have alone (the batch path's guarantee).  Behind each launch a
 * small kernel copies every session's sticky status to pinned host memory;
 * once that copy has finished, a session whose pool or table ran out is
 * marked failed, and its later frames are refused instead of probing a full
 * table, without touching the other sessions.  Frames are handed back when
 * their launch finishes, ahead of the status copy.
 *
 * The server is driven from one host thread: tsdf_server_submit queues,
 * tsdf_server_step retires finished launches and starts new ones, and
 * tsdf_server_completions hands back the tags of finished frames.  Each launch
 * in flight has a stream of its own: the stream given at creation and
 * max_inflight - 1 streams the server makes (default priority), so launches
 * overlap on the device and a frame that arrives while others are fused
 * starts at once; launches into one volume may run together (fusion is a sum
 * of atomic updates, so the result is that of fusing the frames one by one,
 * up to the order of the fp32 additions).  Volume initialisation
 * and the plain launches of tsdf_server_replay use the stream given at
 * creation; status and extraction calls on a session's volume belong on that
 * stream too, after tsdf_server_step has retired the session's launches.
 * Depth frames must stay valid until their tags come back.
 * ------------------------------------------------------------------------- */
typedef struct tsdf_server tsdf_server;

typedef struct tsdf_server_params {
  uint32_t max_sessions;  /* 1 .. 65536 */
  uint32_t max_batch;     /* frames per launch, 1 .. TSDF_BATCH_MAX_ITEMS */
  uint32_t max_inflight;  /* launches running at once, one stream each, 1 .. 4 */
  uint32_t max_queue;     /* frames waiting, max_batch .. 2^24 */
} tsdf_server_params;

/* Device workspace bytes for `params` (the batch work list); 0 if invalid. */
size_t tsdf_server_workspace_bytes(const tsdf_server_params* params);

/* Make a server.  workspace_dev: >= tsdf_server_workspace_bytes, 256-aligned.
 * Session volumes are carved from [session_region_dev, + budget_bytes).  The
 * server also owns a tsdf_batch (its autotuner starts on), pinned host status
 * words and one HIP event per in-flight launch. */
tsdf_status tsdf_server_create(const tsdf_server_params* params, void* workspace_dev,
                               size_t workspace_bytes, void* session_region_dev,
                               uint64_t budget_bytes, void* hip_stream, tsdf_server** out);

/* Wait for every launch, then free the server's host resources.  Queued
 * frames are dropped without completions. */
tsdf_status tsdf_server_destroy(tsdf_server* server);

/* Admit a session: carve tsdf_volume_bytes(params) from the budget and
 * enqueue the volume's initialisation.  TSDF_ERR_BUDGET if the budget (or
 * the session table) has no room.  Colour volumes are not served
 * (TSDF_ERR_INVALID_ARGUMENT). */
tsdf_status tsdf_server_open(tsdf_server* server, const tsdf_volume_params* params,
                             uint32_t* session_out);

/* Retire a session: its queued frames are dropped (completed with
 * TSDF_ERR_INVALID_ARGUMENT), the server waits for launches that hold its
 * frames, and its memory returns to the budget. */
tsdf_status tsdf_server_close(tsdf_server* server, uint32_t session);

/* Queue one frame (depth_dev: height x width float32 in device memory, or in
 * pinned host memory at its device address, as for tsdf_fuse_frame; it must
 * stay valid until the frame completes) for a session.  Returns
 * TSDF_ERR_BUDGET if the queue is full, and the session's failure status
 * (TSDF_ERR_POOL_EXHAUSTED, TSDF_ERR_TABLE_FULL, TSDF_ERR_INTERNAL) once it
 * has failed. */
tsdf_status tsdf_server_submit(tsdf_server* server, uint32_t session, const float* depth_dev,
                               const tsdf_camera* camera, uint64_t tag);

/* Retire finished launches (non-blocking) and, if fewer than max_inflight
 * are running and frames are queued, launch one batch.  *launched (may be
 * NULL) receives the number of frames launched. */
tsdf_status tsdf_server_step(tsdf_server* server, uint32_t* launched);

/* Pop up to `max` finished frames: their tags and statuses (TSDF_OK when
 * fused; a failed session's status when its frame was refused at launch;
 * TSDF_ERR_INVALID_ARGUMENT when its session was closed first). */
tsdf_status tsdf_server_completions(tsdf_server* server, uint64_t* tags, int32_t* statuses,
                                    uint32_t max, uint32_t* n_out);

/* A session's volume (for tsdf_query_status / tsdf_extract_blocks on the
 * server's stream) and its failure status (TSDF_OK while healthy). */
tsdf_status tsdf_server_session(tsdf_server* server, uint32_t session, tsdf_volume** volume,
                                int32_t* failure);

/* The server's batch, e.g. to fix its configuration. */
tsdf_status tsdf_server_batch(tsdf_server* server, tsdf_batch** out);

/* Frames queued and in flight, launches in flight, sessions open, and budget
 * bytes used; any output may be NULL. */
tsdf_status tsdf_server_load(tsdf_server* server, uint32_t* queued, uint32_t* inflight_frames,
                             uint32_t* inflight_launches, uint32_t* sessions,
                             uint64_t* budget_used);

/* Replay an arrival trace in real time on the host's steady clock and report
 * each request's latency: completion (when the host sees the frame's launch
 * finish) minus arrival.  Requests must be sorted by arrival_ns, offsets from
 * the start of the replay.
 *   TSDF_REPLAY_SERVED  through tsdf_server_submit / _step / _completions
 *   TSDF_REPLAY_PLAIN   one tsdf_fuse_frame per request, launched when it
 *                       arrives, on the server's stream (the comparison)
 * latency_ns[i] gets request i's latency (-1 if it was refused);
 * *elapsed_ns the time from the start to the last completion.  The server
 * must have no queued, running or uncollected frames when the replay starts
 * (TSDF_ERR_INVALID_ARGUMENT otherwise). */
typedef struct tsdf_request {
  uint64_t arrival_ns;
  uint32_t session;
  uint32_t reserved;
  const float* depth_dev;
  tsdf_camera camera;
} tsdf_request;
#define TSDF_REPLAY_SERVED 0u
#define TSDF_REPLAY_PLAIN 1u
tsdf_status tsdf_server_replay(tsdf_server* server, const tsdf_request* requests, uint32_t n,
                               uint32_t mode, double* latency_ns, double* elapsed_ns);

/* Static text for a status code. */
const char* tsdf_status_str(tsdf_status status);

#ifdef __cplusplus
}
#endif

#endif /* TSDF_H_ */
