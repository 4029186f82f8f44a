// Surface extraction: marching tetrahedra over the voxel centres of every
// allocated block (the extraction the paper runs after fusion and leaves out
// of its timing, Section 2.4; its checks are those of Section 3.3).
//
// One workgroup per pool block.  The block's 8^3 voxels and the one-voxel
// skirt of its +x, +y, +z neighbours (found by lookups in the hash table) are
// staged in LDS as a 9^3 grid of means (sum / weight, NaN where unobserved);
// each thread then meshes two of the block's 512 cubes (the cube whose lowest
// corner is the voxel).  A cube is used only when its 8 corners are observed,
// and is skipped when it changes sign next to a value at the truncation limit
// (a jump at an occlusion edge).  It is cut into the 6 tetrahedra around its
// corner-0 to corner-7 diagonal; each tetrahedron with a sign change gives one
// or two triangles with vertices interpolated linearly on its crossing edges,
// from the edge's lexicographically lower corner, wound with the normal
// towards the positive side.  Triangles are appended with one global atomic
// per workgroup; the output order is therefore arbitrary, and each triangle
// carries an identity (block key, cube << 4 | tetrahedron << 1 | triangle).

#include "tsdf_device.h"

namespace tsdf {
namespace {

constexpr int kSkirt = 9;  // 8 voxels of the block + 1 of the next block per axis
constexpr int kGrid = kSkirt * kSkirt * kSkirt;

__device__ __forceinline__ int grid_index(int x, int y, int z) {
  return (z * kSkirt + y) * kSkirt + x;
}

// Pool index of `key`, or -1 when it is absent or its block was never given
// one.  Run after fusion has finished: no entry is still being published.
__device__ int lookup_block(const VolumeDev& vol, unsigned long long key) {
  const unsigned C = vol.table_capacity;
  unsigned slot = home_slot(key, C);
  for (unsigned probes = 0; probes < C; ++probes) {
    const TableEntry e = vol.table[slot];
    if (e.key == key) return e.block >= 0 ? e.block : -1;
    if (e.key == kEmptyKey) return -1;
    slot = (slot + 1 == C) ? 0u : slot + 1;
  }
  return -1;
}

// The six tetrahedra around the diagonal 0-7; corner c = x + 2y + 4z.
__constant__ const unsigned char kTets[6][4] = {{0, 1, 3, 7}, {0, 3, 2, 7}, {0, 2, 6, 7},
                                                {0, 6, 4, 7}, {0, 4, 5, 7}, {0, 5, 1, 7}};

struct CubeGeom {
  int gx, gy, gz;  // global voxel index of corner 0
  float f[8];
};

// Triangles of one tetrahedron; emit(k, P0, P1, P2) for each (k = 0, 1).
template <typename Emit>
__device__ __forceinline__ int mesh_tet(const CubeGeom& c, int t, float v, bool write, Emit emit) {
  int ins[4], outs[4], ni = 0, no = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int q = kTets[t][k];
    if (c.f[q] < 0.0f) ins[ni++] = q;
    else outs[no++] = q;
  }
  if (ni == 0 || no == 0) return 0;
  const int ntri = (ni == 2) ? 2 : 1;
  if (!write) return ntri;
  // crossing edges as (inside corner, outside corner)
  int ea[4], eb[4], ne;
  if (ni == 1) {
    ea[0] = ins[0], eb[0] = outs[0];
    ea[1] = ins[0], eb[1] = outs[1];
    ea[2] = ins[0], eb[2] = outs[2];
    ne = 3;
  } else if (ni == 3) {
    ea[0] = ins[0], eb[0] = outs[0];
    ea[1] = ins[1], eb[1] = outs[0];
    ea[2] = ins[2], eb[2] = outs[0];
    ne = 3;
  } else {
    ea[0] = ins[0], eb[0] = outs[0];
    ea[1] = ins[0], eb[1] = outs[1];
    ea[2] = ins[1], eb[2] = outs[1];
    ea[3] = ins[1], eb[3] = outs[0];
    ne = 4;
  }
  float P[4][3];
  for (int k = 0; k < ne; ++k) {
    int a = ea[k], b = eb[k];
    // lexicographic (x, y, z) order of the two corners: compare x, then y, then z
    const int ax = a & 1, ay = (a >> 1) & 1, az = a >> 2;
    const int bx = b & 1, by = (b >> 1) & 1, bz = b >> 2;
    const bool b_first = (bx != ax) ? (bx < ax) : (by != ay) ? (by < ay) : (bz < az);
    if (b_first) {
      const int tmp = a;
      a = b;
      b = tmp;
    }
    const float tt = c.f[a] / (c.f[a] - c.f[b]);
    const int ga[3] = {c.gx + (a & 1), c.gy + ((a >> 1) & 1), c.gz + (a >> 2)};
    const int gb[3] = {c.gx + (b & 1), c.gy + ((b >> 1) & 1), c.gz + (b >> 2)};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const float pa = ((float)ga[d] + 0.5f) * v;
      const float pb = ((float)gb[d] + 0.5f) * v;
      P[k][d] = pa + tt * (pb - pa);
    }
  }
  // outward reference: from an inside corner to an outside corner
  const float g0 = (float)((outs[0] & 1) - (ins[0] & 1));
  const float g1 = (float)(((outs[0] >> 1) & 1) - ((ins[0] >> 1) & 1));
  const float g2 = (float)((outs[0] >> 2) - (ins[0] >> 2));
  for (int k = 0; k < ntri; ++k) {
    const int i0 = 0, i1 = k == 0 ? 1 : 2, i2 = k == 0 ? 2 : 3;
    const float u0 = P[i1][0] - P[i0][0], u1 = P[i1][1] - P[i0][1], u2 = P[i1][2] - P[i0][2];
    const float w0 = P[i2][0] - P[i0][0], w1 = P[i2][1] - P[i0][1], w2 = P[i2][2] - P[i0][2];
    const float n0 = u1 * w2 - u2 * w1, n1 = u2 * w0 - u0 * w2, n2 = u0 * w1 - u1 * w0;
    const bool flip = (n0 * g0 + n1 * g1) + n2 * g2 < 0.0f;
    emit(k, P[i0], flip ? P[i2] : P[i1], flip ? P[i1] : P[i2]);
  }
  return ntri;
}

__global__ __launch_bounds__(256) void mesh_kernel(VolumeDev vol, float v, float trunc,
                                                   unsigned* counter, unsigned max_tris,
                                                   float* verts, unsigned long long* ids) {
  __shared__ float s_f[kGrid];
  __shared__ int s_nb[8];
  __shared__ unsigned s_scan[256];
  __shared__ unsigned s_base;
  const unsigned tid = threadIdx.x;
  const unsigned blk = allocated_block(vol, blockIdx.x);
  const unsigned long long key = vol.block_keys[blockIdx.x];
  const int bx = (int)(key >> 42) - (1 << 20);
  const int by = (int)((key >> 21) & ((1u << 21) - 1)) - (1 << 20);
  const int bz = (int)(key & ((1u << 21) - 1)) - (1 << 20);
  if (tid < 8) {
    const int dx = tid & 1, dy = (tid >> 1) & 1, dz = tid >> 2;
    const int nx = bx + dx, ny = by + dy, nz = bz + dz;
    const bool in_range = nx < (1 << 20) && ny < (1 << 20) && nz < (1 << 20);
    s_nb[tid] = tid == 0 ? (int)blk
                         : (in_range ? lookup_block(vol, pack_key(nx, ny, nz)) : -1);
  }
  __syncthreads();
  for (unsigned i = tid; i < (unsigned)kGrid; i += 256) {
    const int x = (int)(i % kSkirt), y = (int)((i / kSkirt) % kSkirt), z = (int)(i / (kSkirt * kSkirt));
    const int nb = s_nb[(x >> 3) | ((y >> 3) << 1) | ((z >> 3) << 2)];
    float f = __builtin_nanf("");
    if (nb >= 0) {
      const unsigned loc = voxel_index((unsigned)x & 7u, (unsigned)y & 7u, (unsigned)z & 7u);
      const float* bp = vol.voxels + (size_t)nb * kBlockFloats;
      const float w = bp[pool_weight_index(loc)];
      if (w > 0.0f) f = bp[pool_tsdf_index(loc)] / w;
    }
    s_f[i] = f;
  }
  __syncthreads();

  const float limit = (1.0f - 1.0f / 1024.0f) * trunc;
  CubeGeom cube[2];
  bool use[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int loc = (int)tid + 256 * h;
    const int lx = loc & 7, ly = (loc >> 3) & 7, lz = loc >> 6;
    cube[h].gx = bx * 8 + lx;
    cube[h].gy = by * 8 + ly;
    cube[h].gz = bz * 8 + lz;
    bool ok = true, any_in = false, any_out = false, truncated = false;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const float f = s_f[grid_index(lx + (c & 1), ly + ((c >> 1) & 1), lz + (c >> 2))];
      cube[h].f[c] = f;
      ok = ok && !__builtin_isnan(f);
      any_in = any_in || f < 0.0f;
      any_out = any_out || f >= 0.0f;
      truncated = truncated || __builtin_fabsf(f) >= limit;
    }
    use[h] = ok && any_in && any_out && !truncated;
  }
  // count, scan, reserve
  unsigned mine = 0;
#pragma unroll
  for (int h = 0; h < 2; ++h)
    if (use[h])
      for (int t = 0; t < 6; ++t)
        mine += (unsigned)mesh_tet(cube[h], t, v, false, [](int, const float*, const float*, const float*) {});
  s_scan[tid] = mine;
  __syncthreads();
  for (unsigned off = 1; off < 256; off <<= 1) {
    const unsigned add = tid >= off ? s_scan[tid - off] : 0u;
    __syncthreads();
    s_scan[tid] += add;
    __syncthreads();
  }
  if (tid == 255) s_base = s_scan[255] ? atomicAdd(counter, s_scan[255]) : 0u;
  __syncthreads();
  unsigned at = s_base + s_scan[tid] - mine;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    if (!use[h]) continue;
    const unsigned loc = tid + 256u * (unsigned)h;
    for (int t = 0; t < 6; ++t) {
      mesh_tet(cube[h], t, v, true, [&](int k, const float* p0, const float* p1, const float* p2) {
        if (at < max_tris) {
          float* o = verts + (size_t)at * 9;
          o[0] = p0[0], o[1] = p0[1], o[2] = p0[2];
          o[3] = p1[0], o[4] = p1[1], o[5] = p1[2];
          o[6] = p2[0], o[7] = p2[1], o[8] = p2[2];
          if (ids) {
            ids[(size_t)at * 2] = key;
            ids[(size_t)at * 2 + 1] = (unsigned long long)((loc << 4) | ((unsigned)t << 1) | (unsigned)k);
          }
        }
        ++at;
      });
    }
  }
}

}  // namespace

hipError_t launch_mesh(VolumeDev vol, const WalkParams& wp, unsigned n_blocks, unsigned* counter,
                       unsigned max_tris, float* verts, unsigned long long* ids, hipStream_t s) {
  if (n_blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(mesh_kernel, dim3(n_blocks), dim3(256), 0, s, vol, wp.v, wp.trunc, counter,
                     max_tris, verts, ids);
  return hipGetLastError();
}

}  // namespace tsdf
