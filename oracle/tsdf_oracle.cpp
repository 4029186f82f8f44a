// TEST INFRASTRUCTURE ONLY -- NOT PART OF THE PRODUCT PATH.
//
// A plain, slow, sequential CPU model of hash-blocked TSDF fusion, written from
// the paper's description of its workload (Section 2: "Structure", "Two passes,
// and why", "The insert protocol") and used only by the tests, by the smoke check
// and by the CPU-baseline leg of the benchmark.  It shares no code with the GPU
// path: no headers, no helpers, no constants are common to the two.
//
// What it computes, per fused depth frame (one "point" = one valid pixel):
//
//   PASS 1 (allocate): walk every point's truncation band, select the voxels it
//     touches, apply the occlusion test, and make sure a block exists for the 8^3
//     block holding each selected voxel.  Blocks come from a pool of fixed
//     capacity; a block that does not fit is recorded as overflowed, never lost
//     silently (Section 3.4: pool-exhaustion reporting).
//   PASS 2 (update): walk the same band again and add, for each selected voxel,
//     the truncated signed distance to its block's running *sum* and 1 to its
//     weight.  Means are recovered only at extraction (Section 2.2).
//
// The walk is a fixed sequence of float32 operations (+, -, *, floor and
// comparisons, no contraction into FMA), so the set of voxels a point selects is
// defined to the bit.  Where the paper leaves the walk unstated (sample
// positions, occlusion rule, voxel centre, per-point dedupe), the readings used
// are the ones listed beside each step below.  Sums are kept in float64 here; the
// GPU keeps float32 sums, so TSDF means agree only to a tolerance while block keys
// and weights agree exactly.
//
// Also here: a sequential linear-probe table model (Section 2.1: open addressing,
// linear probing, 16-byte entries keyed by the packed block coordinate) used to
// check the occupied-slot set and the total probe displacement of the GPU table.
//
// Parity pins for each function live in tests/test_oracle_*.py.

#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <set>
#include <vector>

namespace {

// ---------------------------------------------------------------------------
// Section 2.1, the key equation: each block axis is biased by 2^20 into 21 bits
// and the three axes are packed into one 64-bit word, x in the top field.
// ---------------------------------------------------------------------------
const int64_t kAxisBias = int64_t(1) << 20;

uint64_t pack_block_key(int64_t bx, int64_t by, int64_t bz) {
  return (uint64_t(bx + kAxisBias) << 42) | (uint64_t(by + kAxisBias) << 21) |
         uint64_t(bz + kAxisBias);
}

// Block coordinate of a voxel: the 8^3 block containing it, i.e. floor(v / 8),
// written as plain floor division (rounds toward minus infinity).
int64_t block_of(int64_t v) {
  int64_t q = v / 8;
  if (v % 8 != 0 && v < 0) q -= 1;
  return q;
}

// Position of a voxel inside its block, 0..7 per axis.
int64_t offset_in_block(int64_t v) { return v - 8 * block_of(v); }

struct Params {
  float v;      // voxel edge (metres)
  float trunc;  // truncation distance tau (metres)
  float iv;     // 1/v, rounded once to float32
  int K;        // samples per half band: round(tau / v); band has 2K+1 samples
};

struct Frame {
  const float* depth;  // H*W row-major, metres (camera-frame z)
  uint32_t W, H;
  float fx, fy, cx, cy;
  float ifx, ify;      // 1/fx, 1/fy rounded once to float32
  float R[3][3];       // camera->world rotation
  float t[3];          // camera->world translation
};

struct Pair {
  uint64_t key;   // packed block key
  uint32_t loc;   // voxel index inside the block: (lz*8 + ly)*8 + lx
  float val;      // truncated signed distance contributed
  int32_t vx, vy, vz;
  uint64_t pixel; // row-major index of the point's pixel
};

struct WalkCounts {
  uint64_t points_valid = 0;
  uint64_t pairs = 0;
  uint64_t coord_out_of_range = 0;  // samples whose voxel coordinate cannot be packed
};

// The truncation-band walk of one frame, calling emit(pair) for every
// (point, voxel) pair in a fixed order: points row-major (reverse row-major if
// `reverse`), samples nearest-first along the ray.
//
// Readings of the paper (its Section 2 names the steps, not their arithmetic):
//  * a point is a pixel with finite depth d > 0;
//  * the band is walked with 2K+1 samples at camera depths z_k = d + (k-K) v,
//    k = 0..2K, on the pixel's ray (x, y, z) = (a z, b z, z);
//  * a sample's voxel is floor(world / v), voxel i spanning [i v, (i+1) v);
//  * a voxel counts at most once per point;
//  * the signed distance is taken at the voxel centre (the fix to the half-voxel
//    bias of Section 4.1): sdf = d - (camera-frame z of the centre);
//  * occlusion test, identical in both passes (Section 2.2): keep the pair only
//    if the centre is in front of the camera and sdf >= -tau;
//  * the contribution is min(sdf, tau).
template <class Emit>
void walk_frame(const Params& p, const Frame& f, bool reverse, WalkCounts& cnt, Emit emit) {
  const uint64_t n = uint64_t(f.W) * f.H;
  for (uint64_t step = 0; step < n; ++step) {
    const uint64_t i = reverse ? n - 1 - step : step;
    const uint32_t x = uint32_t(i % f.W), y = uint32_t(i / f.W);
    const float d = f.depth[i];
    if (!(std::isfinite(d) && d > 0.0f)) continue;
    cnt.points_valid++;
    const float a = (float(x) - f.cx) * f.ifx;
    const float b = (float(y) - f.cy) * f.ify;
    std::vector<int32_t> chosen;  // voxels already selected by this point, 3 ints each
    for (int k = 0; k <= 2 * p.K; ++k) {
      const float z = d + float(k - p.K) * p.v;
      if (!(z > 0.0f)) continue;
      const float xc = a * z, yc = b * z, zc = z;
      float w[3];
      for (int r = 0; r < 3; ++r) {
        float s = f.R[r][0] * xc;
        s = s + f.R[r][1] * yc;
        s = s + f.R[r][2] * zc;
        w[r] = s + f.t[r];
      }
      float q[3];
      bool in_range = true;
      for (int r = 0; r < 3; ++r) {
        q[r] = w[r] * p.iv;
        if (!(std::fabs(q[r]) < 8388608.0f)) in_range = false;  // 2^23 = 2^20 blocks of 8
      }
      if (!in_range) {
        cnt.coord_out_of_range++;
        continue;
      }
      const int32_t vx = int32_t(std::floor(q[0]));
      const int32_t vy = int32_t(std::floor(q[1]));
      const int32_t vz = int32_t(std::floor(q[2]));
      bool seen = false;
      for (size_t j = 0; j < chosen.size(); j += 3)
        if (chosen[j] == vx && chosen[j + 1] == vy && chosen[j + 2] == vz) seen = true;
      if (seen) continue;
      chosen.push_back(vx);
      chosen.push_back(vy);
      chosen.push_back(vz);
      // centre of the voxel in world coordinates, then its camera-frame z
      const float c0 = (float(vx) + 0.5f) * p.v;
      const float c1 = (float(vy) + 0.5f) * p.v;
      const float c2 = (float(vz) + 0.5f) * p.v;
      float zcv = f.R[0][2] * (c0 - f.t[0]);
      zcv = zcv + f.R[1][2] * (c1 - f.t[1]);
      zcv = zcv + f.R[2][2] * (c2 - f.t[2]);
      const float sdf = d - zcv;
      if (!(zcv > 0.0f) || sdf < -p.trunc) continue;
      Pair pr;
      pr.key = pack_block_key(block_of(vx), block_of(vy), block_of(vz));
      pr.loc = uint32_t((offset_in_block(vz) * 8 + offset_in_block(vy)) * 8 + offset_in_block(vx));
      pr.val = sdf < p.trunc ? sdf : p.trunc;
      pr.vx = vx;
      pr.vy = vy;
      pr.vz = vz;
      pr.pixel = i;
      cnt.pairs++;
      emit(pr);
    }
  }
}

struct Block {
  double sum[512];
  uint32_t weight[512];
  double colour[3][512];  // red, green, blue sums (Section 2.1: five parallel arrays)
};

struct Volume {
  Params p;
  uint32_t pool_capacity;
  std::map<uint64_t, Block> blocks;       // allocated blocks, by key
  std::set<uint64_t> pool_overflow_keys;  // keys that found the pool full
  uint64_t points_valid = 0, pairs = 0, pairs_dropped = 0, coord_out_of_range = 0;
  uint64_t frames = 0;
};

bool make_params(float v, float trunc, Params& p) {
  if (!(v > 0.0f) || !(trunc >= v) || !std::isfinite(v) || !std::isfinite(trunc)) return false;
  p.v = v;
  p.trunc = trunc;
  p.iv = 1.0f / v;
  p.K = int(std::llround(double(trunc) / double(v)));
  return p.K >= 1;
}

bool make_frame(const float* depth, uint32_t W, uint32_t H, const float* intr4,
                const float* pose12, Frame& f) {
  if (!depth && uint64_t(W) * H > 0) return false;
  f.depth = depth;
  f.W = W;
  f.H = H;
  f.fx = intr4[0];
  f.fy = intr4[1];
  f.cx = intr4[2];
  f.cy = intr4[3];
  if (!(f.fx != 0.0f) || !(f.fy != 0.0f)) return false;
  f.ifx = 1.0f / f.fx;
  f.ify = 1.0f / f.fy;
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) f.R[r][c] = pose12[r * 4 + c];
    f.t[r] = pose12[r * 4 + 3];
  }
  return true;
}

// Allocation step of PASS 1 for one key.
void ensure_block(Volume& vol, uint64_t key) {
  if (vol.blocks.count(key)) return;
  if (vol.blocks.size() < vol.pool_capacity) {
    Block& b = vol.blocks[key];
    std::memset(&b, 0, sizeof(b));
  } else {
    vol.pool_overflow_keys.insert(key);
  }
}

// Section 2.1 names "the same multiply-xor hash" without giving it.  Reading:
// MurmurHash3's 64-bit finaliser (fmix64), then the home slot is the high 32
// bits of the hash scaled to [0, C) by a 32x32->64 multiply (Lemire's range
// reduction).  Written here from those published definitions.
uint64_t murmur3_fmix64(uint64_t k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdULL;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ULL;
  k ^= k >> 33;
  return k;
}

uint32_t home_slot(uint64_t key, uint32_t C) {
  const uint64_t hi = murmur3_fmix64(key) >> 32;
  return uint32_t((hi * uint64_t(C)) >> 32);
}

// ---------------------------------------------------------------------------
// Surface extraction: marching tetrahedra over the voxel centres.
//
// The paper extracts the zero crossing of the fused field with marching
// tetrahedra (Section 2.4) and checks the result on a sphere of known radius
// and by vertex distances between runs (Section 3.3).  It does not spell the method out; the readings:
//   - samples are voxel centres ((i + 1/2) v per axis), values the mean TSDF
//     sum / weight;
//   - a cube of 8 neighbouring centres is used only when all 8 voxels have a
//     weight, and it is skipped when its values change sign while some corner
//     has |value| >= (1 - 2^-10) tau: a jump across the truncation limit at an
//     occlusion edge, not a surface;
//   - the cube is cut into the 6 tetrahedra that share its diagonal from
//     corner 0 to corner 7 (corner c has offset (c & 1, c >> 1 & 1, c >> 2));
//   - a corner is inside when its value is < 0; a tetrahedron with one or three
//     inside corners gives one triangle, with two it gives two;
//   - a vertex lies on an edge with one inside and one outside corner, at
//     t = f_a / (f_a - f_b) from corner a, where a is the edge's corner that
//     comes first in (x, y, z) lexicographic grid order;
//   - each triangle is wound so that its normal points to the outside corners.
// Triangle identity: (block key, cube << 4 | tetrahedron << 1 | triangle).
// ---------------------------------------------------------------------------

struct MeshTri {
  uint64_t key;
  uint32_t code;         // cube << 4 | tet << 1 | sub
  double p[3][3];        // vertices
  int64_t edge[3][2][3]; // per vertex: the edge's two corners (global voxel index)
};

const int kTet[6][4] = {{0, 1, 3, 7}, {0, 3, 2, 7}, {0, 2, 6, 7},
                        {0, 6, 4, 7}, {0, 4, 5, 7}, {0, 5, 1, 7}};

bool lex_less(const int64_t* a, const int64_t* b) {
  if (a[0] != b[0]) return a[0] < b[0];
  if (a[1] != b[1]) return a[1] < b[1];
  return a[2] < b[2];
}

// Mean and presence of the voxel at global index g (per axis).
bool voxel_value(const Volume& vol, const int64_t* g, double* f) {
  const uint64_t key = pack_block_key(block_of(g[0]), block_of(g[1]), block_of(g[2]));
  auto it = vol.blocks.find(key);
  if (it == vol.blocks.end()) return false;
  const int loc = int((offset_in_block(g[2]) * 8 + offset_in_block(g[1])) * 8 + offset_in_block(g[0]));
  const uint32_t w = it->second.weight[loc];
  if (w == 0) return false;
  *f = it->second.sum[loc] / double(w);
  return true;
}

void mesh_cube(const Volume& vol, uint64_t key, int64_t bx, int64_t by, int64_t bz, int loc,
               std::vector<MeshTri>& out) {
  const int lx = loc & 7, ly = (loc >> 3) & 7, lz = loc >> 6;
  int64_t corner[8][3];
  double f[8];
  bool any_in = false, any_out = false, truncated = false;
  const double tau_limit = (1.0 - 1.0 / 1024.0) * double(vol.p.trunc);
  for (int c = 0; c < 8; ++c) {
    corner[c][0] = bx * 8 + lx + (c & 1);
    corner[c][1] = by * 8 + ly + ((c >> 1) & 1);
    corner[c][2] = bz * 8 + lz + ((c >> 2) & 1);
    if (!voxel_value(vol, corner[c], &f[c])) return;
    (f[c] < 0.0 ? any_in : any_out) = true;
    if (std::fabs(f[c]) >= tau_limit) truncated = true;
  }
  if (!(any_in && any_out) || truncated) return;
  const double v = double(vol.p.v);
  for (int t = 0; t < 6; ++t) {
    const int* q = kTet[t];
    int ins[4], outs[4], ni = 0, no = 0;
    for (int k = 0; k < 4; ++k) (f[q[k]] < 0.0 ? ins[ni++] : outs[no++]) = q[k];
    if (ni == 0 || no == 0) continue;
    // the crossing edges, as (inside corner, outside corner)
    int e[4][2];
    int ne = 0;
    if (ni == 1) {
      for (int k = 0; k < 3; ++k) e[ne][0] = ins[0], e[ne++][1] = outs[k];
    } else if (ni == 3) {
      for (int k = 0; k < 3; ++k) e[ne][0] = ins[k], e[ne++][1] = outs[0];
    } else {  // two and two: the quad i0-o0, i0-o1, i1-o1, i1-o0
      e[0][0] = ins[0], e[0][1] = outs[0];
      e[1][0] = ins[0], e[1][1] = outs[1];
      e[2][0] = ins[1], e[2][1] = outs[1];
      e[3][0] = ins[1], e[3][1] = outs[0];
      ne = 4;
    }
    double P[4][3];
    int64_t E[4][2][3];
    for (int k = 0; k < ne; ++k) {
      int a = e[k][0], b = e[k][1];
      if (lex_less(corner[b], corner[a])) std::swap(a, b);
      const double tt = f[a] / (f[a] - f[b]);
      for (int d = 0; d < 3; ++d) {
        const double pa = (double(corner[a][d]) + 0.5) * v, pb = (double(corner[b][d]) + 0.5) * v;
        P[k][d] = pa + tt * (pb - pa);
        E[k][0][d] = corner[a][d];
        E[k][1][d] = corner[b][d];
      }
    }
    // outward reference: from an inside corner to an outside corner
    double g[3];
    for (int d = 0; d < 3; ++d) g[d] = double(corner[outs[0]][d] - corner[ins[0]][d]);
    const int tris[2][3] = {{0, 1, 2}, {0, 2, 3}};
    const int ntri = ne == 4 ? 2 : 1;
    for (int k = 0; k < ntri; ++k) {
      int i0 = tris[k][0], i1 = tris[k][1], i2 = tris[k][2];
      double u[3], w[3], n[3];
      for (int d = 0; d < 3; ++d) u[d] = P[i1][d] - P[i0][d], w[d] = P[i2][d] - P[i0][d];
      n[0] = u[1] * w[2] - u[2] * w[1];
      n[1] = u[2] * w[0] - u[0] * w[2];
      n[2] = u[0] * w[1] - u[1] * w[0];
      if (n[0] * g[0] + n[1] * g[1] + n[2] * g[2] < 0.0) std::swap(i1, i2);
      MeshTri m;
      m.key = key;
      m.code = uint32_t(loc) << 4 | uint32_t(t) << 1 | uint32_t(k);
      const int idx[3] = {i0, i1, i2};
      for (int j = 0; j < 3; ++j)
        for (int d = 0; d < 3; ++d) {
          m.p[j][d] = P[idx[j]][d];
          m.edge[j][0][d] = E[idx[j]][0][d];
          m.edge[j][1][d] = E[idx[j]][1][d];
        }
      out.push_back(m);
    }
  }
}

std::vector<MeshTri> extract_mesh(const Volume& vol) {
  std::vector<MeshTri> out;
  for (const auto& kv : vol.blocks) {
    const uint64_t key = kv.first;
    const int64_t bx = int64_t(key >> 42) - kAxisBias;
    const int64_t by = int64_t((key >> 21) & ((1u << 21) - 1)) - kAxisBias;
    const int64_t bz = int64_t(key & ((1u << 21) - 1)) - kAxisBias;
    for (int loc = 0; loc < 512; ++loc) mesh_cube(vol, key, bx, by, bz, loc, out);
  }
  return out;
}

}  // namespace

extern "C" {

// ---- volume model ---------------------------------------------------------

void* ora_create(float voxel_size, float trunc, uint32_t pool_capacity) {
  Params p;
  if (!make_params(voxel_size, trunc, p) || pool_capacity == 0) return nullptr;
  Volume* vol = new Volume();
  vol->p = p;
  vol->pool_capacity = pool_capacity;
  return vol;
}

void ora_destroy(void* h) { delete static_cast<Volume*>(h); }

int ora_band_samples(void* h) { return 2 * static_cast<Volume*>(h)->p.K + 1; }

// Allocate blocks for given block coordinates (rows of bx, by, bz), in order,
// exactly as PASS 1 would for keys met in that order.
int ora_insert_blocks(void* h, const int32_t* coords, uint64_t n) {
  Volume& vol = *static_cast<Volume*>(h);
  for (uint64_t i = 0; i < n; ++i) {
    const int64_t bx = coords[3 * i], by = coords[3 * i + 1], bz = coords[3 * i + 2];
    if (bx < -kAxisBias || bx >= kAxisBias || by < -kAxisBias || by >= kAxisBias ||
        bz < -kAxisBias || bz >= kAxisBias)
      return -1;
    ensure_block(vol, pack_block_key(bx, by, bz));
  }
  return 0;
}

// Fuse one frame: PASS 1 over every pair, then PASS 2 over every pair.
// intr4 = (fx, fy, cx, cy); pose12 = camera->world [R|t] row-major.
// Both passes of one frame; with `rgba` (packed red | green << 8 | blue << 16
// per pixel) every contribution also adds its pixel's colour to the voxel's
// three colour sums.
static int fuse_impl(void* h, const float* depth, const uint32_t* rgba, uint32_t W, uint32_t H,
              const float* intr4, const float* pose12, int reverse) {
  Volume& vol = *static_cast<Volume*>(h);
  Frame f;
  if (!make_frame(depth, W, H, intr4, pose12, f)) return -1;
  WalkCounts c1, c2;
  walk_frame(vol.p, f, reverse != 0, c1, [&](const Pair& pr) { ensure_block(vol, pr.key); });
  walk_frame(vol.p, f, reverse != 0, c2, [&](const Pair& pr) {
    auto it = vol.blocks.find(pr.key);
    if (it == vol.blocks.end()) {
      vol.pairs_dropped++;
      return;
    }
    it->second.sum[pr.loc] += double(pr.val);
    it->second.weight[pr.loc] += 1;
    if (rgba)
      for (int c = 0; c < 3; ++c)
        it->second.colour[c][pr.loc] += double((rgba[pr.pixel] >> (8 * c)) & 255u);
  });
  vol.points_valid += c2.points_valid;
  vol.pairs += c2.pairs;
  vol.coord_out_of_range += c2.coord_out_of_range;
  vol.frames++;
  return 0;
}

int ora_fuse(void* h, const float* depth, uint32_t W, uint32_t H, const float* intr4,
             const float* pose12, int reverse) {
  return fuse_impl(h, depth, nullptr, W, H, intr4, pose12, reverse);
}

int ora_fuse_rgb(void* h, const float* depth, const uint32_t* rgba, uint32_t W, uint32_t H,
                 const float* intr4, const float* pose12, int reverse) {
  if (!rgba && uint64_t(W) * H > 0) return -1;
  return fuse_impl(h, depth, rgba, W, H, intr4, pose12, reverse);
}

// Colour sums of every block in ascending key order: sums[(i * 3 + c) * 512 + l].
uint64_t ora_export_colour(void* h, double* sums, uint64_t cap) {
  const Volume& vol = *static_cast<Volume*>(h);
  uint64_t i = 0;
  for (const auto& kv : vol.blocks) {
    if (i >= cap) break;
    for (int c = 0; c < 3; ++c)
      for (int l = 0; l < 512; ++l) sums[(i * 3 + c) * 512 + l] = kv.second.colour[c][l];
    ++i;
  }
  return vol.blocks.size();
}

// stats: [points_valid, pairs, pairs_dropped, coord_out_of_range, blocks,
//         pool_overflow_keys, frames, pool_capacity]
void ora_stats(void* h, uint64_t* out) {
  const Volume& vol = *static_cast<Volume*>(h);
  out[0] = vol.points_valid;
  out[1] = vol.pairs;
  out[2] = vol.pairs_dropped;
  out[3] = vol.coord_out_of_range;
  out[4] = vol.blocks.size();
  out[5] = vol.pool_overflow_keys.size();
  out[6] = vol.frames;
  out[7] = vol.pool_capacity;
}

// Export blocks in ascending key order.  sums/weights hold 512 entries per block;
// mean = sum / weight where weight > 0 (Section 2.2: means recovered at extraction).
uint64_t ora_export(void* h, uint64_t* keys, double* sums, double* means, uint32_t* weights,
                    uint64_t cap) {
  const Volume& vol = *static_cast<Volume*>(h);
  uint64_t i = 0;
  for (const auto& kv : vol.blocks) {
    if (i >= cap) break;
    if (keys) keys[i] = kv.first;
    for (int l = 0; l < 512; ++l) {
      const uint32_t w = kv.second.weight[l];
      if (sums) sums[i * 512 + l] = kv.second.sum[l];
      if (means) means[i * 512 + l] = w ? kv.second.sum[l] / double(w) : 0.0;
      if (weights) weights[i * 512 + l] = w;
    }
    ++i;
  }
  return vol.blocks.size();
}

// Replace (or create) the block `key` with the given sums and weights (512 of
// each): lets tests build a field directly.
void ora_set_block(void* h, uint64_t key, const double* sums, const uint32_t* weights) {
  Volume& vol = *static_cast<Volume*>(h);
  Block& b = vol.blocks[key];
  for (int l = 0; l < 512; ++l) {
    b.sum[l] = sums[l];
    b.weight[l] = weights[l];
  }
}

// Marching-tetrahedra mesh of the volume, triangles in block-key order, then
// cube, tetrahedron, triangle.  Per triangle: ids[2] = {key, code}, verts[9],
// edges[18] (per vertex the two corners of its edge, global voxel indices).
// Returns the triangle count; writes at most `cap`.  Any output may be NULL.
uint64_t ora_extract_mesh(void* h, uint64_t* ids, double* verts, int64_t* edges, uint64_t cap) {
  const std::vector<MeshTri> tris = extract_mesh(*static_cast<Volume*>(h));
  for (uint64_t i = 0; i < tris.size() && i < cap; ++i) {
    const MeshTri& m = tris[i];
    if (ids) ids[2 * i] = m.key, ids[2 * i + 1] = m.code;
    for (int j = 0; j < 3; ++j)
      for (int d = 0; d < 3; ++d) {
        if (verts) verts[9 * i + 3 * j + d] = m.p[j][d];
        if (edges) {
          edges[18 * i + 6 * j + d] = m.edge[j][0][d];
          edges[18 * i + 6 * j + 3 + d] = m.edge[j][1][d];
        }
      }
  }
  return tris.size();
}

uint64_t ora_export_overflow_keys(void* h, uint64_t* keys, uint64_t cap) {
  const Volume& vol = *static_cast<Volume*>(h);
  uint64_t i = 0;
  for (uint64_t k : vol.pool_overflow_keys) {
    if (i >= cap) break;
    keys[i++] = k;
  }
  return vol.pool_overflow_keys.size();
}

// Enumerate the pairs of one frame in walk order (for tests).  Returns the pair
// count; writes at most `cap`.  counts3 = [points_valid, pairs, coord_out_of_range].
uint64_t ora_frame_pairs(float voxel_size, float trunc, const float* depth, uint32_t W,
                         uint32_t H, const float* intr4, const float* pose12, int reverse,
                         uint64_t* keys, uint32_t* locs, float* vals, int32_t* voxels,
                         uint64_t cap, uint64_t* counts3) {
  Params p;
  Frame f;
  if (!make_params(voxel_size, trunc, p) || !make_frame(depth, W, H, intr4, pose12, f))
    return ~uint64_t(0);
  WalkCounts c;
  uint64_t n = 0;
  walk_frame(p, f, reverse != 0, c, [&](const Pair& pr) {
    if (n < cap) {
      if (keys) keys[n] = pr.key;
      if (locs) locs[n] = pr.loc;
      if (vals) vals[n] = pr.val;
      if (voxels) {
        voxels[3 * n] = pr.vx;
        voxels[3 * n + 1] = pr.vy;
        voxels[3 * n + 2] = pr.vz;
      }
    }
    ++n;
  });
  if (counts3) {
    counts3[0] = c.points_valid;
    counts3[1] = c.pairs;
    counts3[2] = c.coord_out_of_range;
  }
  return n;
}

uint64_t ora_pack_key(int32_t bx, int32_t by, int32_t bz) { return pack_block_key(bx, by, bz); }

int64_t ora_block_of(int64_t v) { return block_of(v); }

uint64_t ora_fmix64(uint64_t k) { return murmur3_fmix64(k); }

uint32_t ora_home_slot(uint64_t key, uint32_t C) { return home_slot(key, C); }

// ---- linear-probe table model ----------------------------------------------
// Insert keys in order into a table of C slots (EMPTY = all ones), probing
// home, home+1, ... cyclically until the key or an empty slot is found; a key
// that meets neither after C probes is counted as a table overflow.  Duplicate
// keys are found, not re-inserted.
//   slot_of[i]   slot holding keys[i] (-1 if it overflowed)
//   disp_of[i]   probes past home at which keys[i] was placed or found
//   table_out    (optional) final table, C keys
// Returns the number of keys (counting duplicates once) that overflowed.
uint64_t ora_probe_model(const uint64_t* keys, uint64_t n, uint32_t C, int64_t* slot_of,
                         uint64_t* disp_of, uint64_t* table_out) {
  const uint64_t kEmpty = ~uint64_t(0);
  std::vector<uint64_t> table(C, kEmpty);
  std::set<uint64_t> overflowed;
  for (uint64_t i = 0; i < n; ++i) {
    const uint32_t home = home_slot(keys[i], C);
    int64_t found = -1;
    uint64_t probes = 0;
    for (; probes < C; ++probes) {
      const uint32_t s = uint32_t((uint64_t(home) + probes) % C);
      if (table[s] == keys[i]) {
        found = s;
        break;
      }
      if (table[s] == kEmpty) {
        table[s] = keys[i];
        found = s;
        break;
      }
    }
    if (found < 0) overflowed.insert(keys[i]);
    if (slot_of) slot_of[i] = found;
    if (disp_of) disp_of[i] = found < 0 ? C : probes;
  }
  if (table_out) std::memcpy(table_out, table.data(), sizeof(uint64_t) * C);
  return overflowed.size();
}

}  // extern "C"
