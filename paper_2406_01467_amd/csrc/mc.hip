// Marching Cubes over a fused TSDF grid: the zero level set of the truncated
// signed distance becomes a triangle mesh (the mesh extraction of Sec. 4.1,
// Lorensen and Cline's method) (gfx950).
//
// Grid values sit at voxel centres (x fastest).  A cell is the cube between
// 2 x 2 x 2 neighbouring centres; it is meshed only when all eight corners
// were observed (weight > 0).  Corner b of a cell is at offset (b & 1,
// b >> 1 & 1, b >> 2 & 1) and is inside when its value is below the iso
// level (bit b of the cell code).  Local edge 4 a + o1 + 2 o2 runs along axis
// a at offsets o1, o2 on the other two axes (increasing axis order).
//
// Per-cell triangulation, derived at compile time from a face rule (no typed
// table):
//  * a face with two sign changes along its boundary holds one segment
//    between its two crossed edges; a face with four (inside corners on a
//    diagonal) holds two, each cutting off one inside corner -- the choice
//    depends on the face alone, so the two cells sharing it agree;
//  * a segment is directed so that, seen from the side where the field is
//    above the iso level, the surface lies on its left (normals point up the
//    field);
//  * every crossed edge starts one segment and ends one: the segments close
//    into cycles, taken in the order of their smallest edge; a cycle is cut
//    into a fan from the smallest edge whose chords to the non-adjacent
//    edges of the cycle join edges sharing no face (chords through the cell
//    interior keep the mesh a manifold), triangles (e0, ei, ei+1) in segment
//    order.
//
// Pipeline: one byte per voxel (observed, inside) -> cell codes (2 bytes per
// cell) -> compaction of the voxels by their used edges (crossed between
// observed voxels and part of an observed cell, up to three per voxel): the
// count is evaluated on the fly in the compaction's reduce and emit
// kernels, the emit writes each vertex (linear zero along the edge, FP64)
// and its id in a per-edge table -> compaction of the cells by triangle
// count, the emit writing each cell's triangles.  No count array is stored
// or scanned: the FP32 grids are read once, the byte and code grids a few
// times, the surface written once.  Vertices are ordered by global edge id
// 3 q + a, triangles by cell index then the cell's rule order, so the mesh
// is deterministic.
#include "common.hpp"
#include "grid.hpp"
#include "scan.hpp"

namespace rade {
namespace {

// ---------------------------------------------------------------------------
// Compile-time triangulation table.
constexpr int kMcMaxTri = 5;

struct McTable {
  uint8_t ntri[256];
  uint8_t tri[256][3 * kMcMaxTri];
};

constexpr int mc_other(int a, int which) {  // the two axes other than a, increasing
  return a == 0 ? (which ? 2 : 1) : a == 1 ? (which ? 2 : 0) : (which ? 1 : 0);
}
constexpr int mc_bit(int c, int axis) { return (c >> axis) & 1; }
constexpr int mc_edge_lo(int e) {
  const int a = e / 4;
  return (mc_bit(e, 0) << mc_other(a, 0)) | (mc_bit(e, 1) << mc_other(a, 1));
}
constexpr int mc_edge_hi(int e) { return mc_edge_lo(e) | (1 << (e / 4)); }
constexpr int mc_edge_of(int c0, int c1) {  // corners differing in one axis
  const int d = c0 ^ c1;
  const int a = d == 1 ? 0 : d == 2 ? 1 : 2;
  const int c = c0 & ~d;
  return 4 * a + mc_bit(c, mc_other(a, 0)) + 2 * mc_bit(c, mc_other(a, 1));
}
// faces of an edge: (axis * 2 + side) for its two fixed coordinates
constexpr int mc_face_mask(int e) {
  const int a = e / 4, u = mc_other(a, 0), v = mc_other(a, 1);
  return (1 << (2 * u + mc_bit(e, 0))) | (1 << (2 * v + mc_bit(e, 1)));
}

constexpr McTable make_mc_table() {
  McTable t{};
  for (int code = 0; code < 256; ++code) {
    int nxt[12] = {-1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1};
    for (int a = 0; a < 3; ++a) {
      const int u = mc_other(a, 0), v = mc_other(a, 1);
      for (int side = 0; side < 2; ++side) {
        // corners in cyclic order (u, v) = (0,0) (1,0) (1,1) (0,1); coordinates
        // doubled so that edge midpoints are integers
        int ring[4] = {0, 0, 0, 0};
        const int du[4] = {0, 1, 1, 0}, dv[4] = {0, 0, 1, 1};
        for (int k = 0; k < 4; ++k) ring[k] = (side << a) | (du[k] << u) | (dv[k] << v);
        int in[4] = {0, 0, 0, 0}, ncross = 0;
        for (int k = 0; k < 4; ++k) in[k] = (code >> ring[k]) & 1;
        for (int k = 0; k < 4; ++k) ncross += in[k] != in[(k + 1) & 3];
        int segA[2] = {0, 0}, segB[2] = {0, 0}, g[2][3] = {{0, 0, 0}, {0, 0, 0}}, nseg = 0;
        if (ncross == 2) {
          int first = -1, second = -1, nin = 0, s_in[3] = {0, 0, 0}, s_out[3] = {0, 0, 0};
          for (int k = 0; k < 4; ++k) {
            if (in[k] != in[(k + 1) & 3]) {
              const int e = mc_edge_of(ring[k], ring[(k + 1) & 3]);
              if (first < 0) first = e; else second = e;
            }
            for (int x = 0; x < 3; ++x) {
              if (in[k]) s_in[x] += 2 * mc_bit(ring[k], x);
              else s_out[x] += 2 * mc_bit(ring[k], x);
            }
            nin += in[k];
          }
          // nin * nout (mean(out) - mean(in)), a positive multiple
          for (int x = 0; x < 3; ++x) g[0][x] = nin * s_out[x] - (4 - nin) * s_in[x];
          segA[0] = first;
          segB[0] = second;
          nseg = 1;
        } else if (ncross == 4) {
          int sum[3] = {0, 0, 0};
          for (int k = 0; k < 4; ++k)
            for (int x = 0; x < 3; ++x) sum[x] += 2 * mc_bit(ring[k], x);
          for (int k = 0; k < 4; ++k) {
            if (!in[k]) continue;
            segA[nseg] = mc_edge_of(ring[(k + 3) & 3], ring[k]);
            segB[nseg] = mc_edge_of(ring[k], ring[(k + 1) & 3]);
            for (int x = 0; x < 3; ++x) g[nseg][x] = sum[x] - 8 * mc_bit(ring[k], x);  // 4 (centre - corner)
            ++nseg;
          }
        }
        const int sn = side ? 1 : -1;  // outward normal sn * e_a
        for (int s = 0; s < nseg; ++s) {
          int A = segA[s], B = segB[s];
          // g x e_a, component by component
          int c[3] = {0, 0, 0};
          if (a == 0) { c[1] = g[s][2]; c[2] = -g[s][1]; }
          if (a == 1) { c[0] = -g[s][2]; c[2] = g[s][0]; }
          if (a == 2) { c[0] = g[s][1]; c[1] = -g[s][0]; }
          int dot = 0;
          for (int x = 0; x < 3; ++x) {
            const int mA = mc_bit(mc_edge_lo(A), x) + mc_bit(mc_edge_hi(A), x);
            const int mB = mc_bit(mc_edge_lo(B), x) + mc_bit(mc_edge_hi(B), x);
            dot += (mB - mA) * c[x] * sn;
          }
          if (dot < 0) { const int tmp = A; A = B; B = tmp; }
          nxt[A] = B;
        }
      }
    }
    int n = 0, seen = 0;
    for (int start = 0; start < 12; ++start) {
      if (nxt[start] < 0 || ((seen >> start) & 1)) continue;
      int cyc[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0}, k = 0, e = start;
      do {
        cyc[k++] = e;
        seen |= 1 << e;
        e = nxt[e];
      } while (e != start);
      int apex = -1;
      for (int i = 0; i < k; ++i) {
        bool clean = true;
        for (int j = 0; j < k; ++j) {
          if (j == i || j == (i + 1) % k || j == (i + k - 1) % k) continue;
          if (mc_face_mask(cyc[i]) & mc_face_mask(cyc[j])) clean = false;
        }
        if (clean && (apex < 0 || cyc[i] < cyc[apex])) apex = i;
      }
      for (int i = 1; i + 1 < k; ++i) {
        t.tri[code][3 * n + 0] = (uint8_t)cyc[apex];
        t.tri[code][3 * n + 1] = (uint8_t)cyc[(apex + i) % k];
        t.tri[code][3 * n + 2] = (uint8_t)cyc[(apex + i + 1) % k];
        ++n;
      }
    }
    t.ntri[code] = (uint8_t)n;
  }
  return t;
}

constexpr McTable kMcHost = make_mc_table();
static_assert(kMcHost.ntri[0] == 0 && kMcHost.ntri[255] == 0, "empty and full cells");
static_assert(kMcHost.ntri[1] == 1 && kMcHost.tri[1][0] == 0 && kMcHost.tri[1][1] == 4 &&
                  kMcHost.tri[1][2] == 8,
              "one inside corner: edges x, y, z of corner 0, normal away from it");
__constant__ McTable kMc = make_mc_table();

constexpr int kT = 256;
constexpr uint16_t kObserved = 0x100;

__global__ void k_mc_zero_counts(uint32_t* nv, uint64_t* nt) {
  *nv = 0u;
  *nt = 0u;
}

inline unsigned grid_for(int64_t n) {
  int64_t b = (n + kT - 1) / kT;
  if (b > ((int64_t)1 << 20)) b = (int64_t)1 << 20;  // grid-stride beyond
  return (unsigned)(b > 0 ? b : 1);
}

// One byte per voxel: bit 0 observed (weight > 0), bit 1 inside (value
// below the iso level).  Every later pass reads these bytes instead of the
// two FP32 grids.
constexpr uint8_t kSeen = 1, kIn = 2;

__global__ void __launch_bounds__(kT)
k_mc_bits(const float* __restrict__ f, const float* __restrict__ w, uint64_t nvox, float iso,
          uint8_t* __restrict__ bits) {
  for (uint64_t q = (uint64_t)blockIdx.x * kT + threadIdx.x; q < nvox;
       q += (uint64_t)gridDim.x * kT) {
    const float fv = f[q], wv = w[q];
    bits[q] = (uint8_t)((wv > 0.0f ? kSeen : 0) | (fv < iso ? kIn : 0));
  }
}

// Cell codes (bit 8: all corners observed), one per cell.
__global__ void __launch_bounds__(kT)
k_mc_cells(const uint8_t* __restrict__ bits, uint32_t nx, uint32_t ny, uint32_t ncell,
           Grid3 cells, uint16_t* __restrict__ info) {
  for (uint64_t cc = (uint64_t)blockIdx.x * kT + threadIdx.x; cc < ncell;
       cc += (uint64_t)gridDim.x * kT) {
    const uint32_t c = (uint32_t)cc;
    uint32_t i, j, k;
    cells.split(c, i, j, k);
    const uint32_t q0 = (k * ny + j) * nx + i;
    uint32_t bv[8];
#pragma unroll
    for (int b = 0; b < 8; ++b)
      bv[b] = bits[q0 + (b & 1) + ((b >> 1) & 1) * nx + ((b >> 2) & 1) * nx * ny];
    uint32_t code = 0, seen = kSeen;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      seen &= bv[b];
      code |= ((bv[b] >> 1) & 1u) << b;
    }
    info[c] = seen ? (uint16_t)(kObserved | code) : (uint16_t)0;
  }
}

// Edges of voxel q along +x, +y, +z (bit a) that change sign between two
// observed voxels and belong to an observed cell: each such edge carries a
// vertex used by that cell's triangles.
struct VoxelEdges {
  const uint8_t* bits;
  const uint16_t* info;
  Grid3 vox;
  uint32_t nz;
  __device__ uint32_t mask(uint32_t q) const {
    const uint32_t nx = vox.nx, ny = vox.ny;
    uint32_t p[3];
    vox.split(q, p[0], p[1], p[2]);
    const uint32_t n[3] = {nx, ny, nz};
    const uint32_t step[3] = {1u, nx, nx * ny};
    const uint32_t b0 = bits[q];
    uint32_t m = 0;
    if (!(b0 & kSeen)) return 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (p[a] + 1 >= n[a]) continue;
      const uint32_t b1 = bits[q + step[a]];
      if (!(b1 & kSeen) || ((b0 ^ b1) & kIn) == 0) continue;
      const int u = a == 0 ? 1 : 0, v = a == 2 ? 1 : 2;
      for (int s = 0; s < 4; ++s) {
        const uint32_t du = s & 1, dv = s >> 1;
        if (du > p[u] || dv > p[v]) continue;
        uint32_t c[3] = {p[0], p[1], p[2]};
        c[u] -= du;
        c[v] -= dv;
        if (c[u] >= n[u] - 1 || c[v] >= n[v] - 1) continue;
        if (info[(c[2] * (ny - 1) + c[1]) * (nx - 1) + c[0]] & kObserved) {
          m |= 1u << a;
          break;
        }
      }
    }
    return m;
  }
  __device__ uint32_t operator()(int64_t item) const {
    return (uint32_t)__builtin_popcount(mask((uint32_t)item));
  }
};

// The used edges of voxel q get vertex ids first, first + 1, ... in axis
// order (so ids follow the global edge id 3 q + a): position at the linear
// zero of the field along the edge (FP64), id in the per-edge table the
// triangles read.
struct EmitVertices {
  VoxelEdges edges;
  const float* f;
  double o0, o1, o2, voxel;
  float iso;
  uint32_t* vid;
  float* verts;
  int64_t max_verts;
  __device__ void operator()(int64_t item, uint32_t first, uint32_t) const {
    const uint32_t q = (uint32_t)item;
    const uint32_t m = edges.mask(q);
    const uint32_t nx = edges.vox.nx, ny = edges.vox.ny;
    uint32_t i, j, k;
    edges.vox.split(q, i, j, k);
    const double f0 = f[q];
    uint32_t id = first;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (!((m >> a) & 1u)) continue;
      vid[3u * q + (uint32_t)a] = id;
      if ((int64_t)id < max_verts) {
        const double f1 = f[q + (a == 0 ? 1u : a == 1 ? nx : nx * ny)];
        const double t = ((double)iso - f0) / (f1 - f0);
        double x = o0 + ((double)i + 0.5) * voxel;
        double y = o1 + ((double)j + 0.5) * voxel;
        double z = o2 + ((double)k + 0.5) * voxel;
        if (a == 0) x += t * voxel;
        if (a == 1) y += t * voxel;
        if (a == 2) z += t * voxel;
        verts[3 * (int64_t)id + 0] = (float)x;
        verts[3 * (int64_t)id + 1] = (float)y;
        verts[3 * (int64_t)id + 2] = (float)z;
      }
      ++id;
    }
  }
};

// Triangles of a cell (0 unless all corners were observed).
struct CellTriangles {
  const uint16_t* info;
  __device__ uint64_t operator()(int64_t c) const {
    const uint16_t inf = info[c];
    return (inf & kObserved) ? (uint64_t)kMc.ntri[inf & 0xff] : 0;
  }
};

// The cell's triangles at `base`, vertex indices looked up per edge.
struct EmitTriangles {
  const uint16_t* info;
  const uint32_t* vid;
  Grid3 cells;
  uint32_t nx, ny;
  uint32_t* tris;
  int64_t max_tris;
  __device__ void operator()(int64_t item, uint64_t base, uint64_t n) const {
    const uint32_t c = (uint32_t)item;
    const int code = info[c] & 0xff;
    uint32_t i, j, k;
    cells.split(c, i, j, k);
    for (int t = 0; t < (int)n; ++t) {
      if ((int64_t)base + t >= max_tris) break;
      for (int m = 0; m < 3; ++m) {
        const int e = kMc.tri[code][3 * t + m];
        const int a = e >> 2;
        uint32_t p[3] = {i, j, k};
        p[a == 0 ? 1 : 0] += e & 1;
        p[a == 2 ? 1 : 2] += (e >> 1) & 1;
        const uint32_t ge = 3u * ((p[2] * ny + p[1]) * nx + p[0]) + (uint32_t)a;
        tris[3 * ((int64_t)base + t) + m] = vid[ge];
      }
    }
  }
};

struct McLayout {
  size_t bits, info, vid, sums, totals, total;
};

McLayout mc_layout(int64_t nx, int64_t ny, int64_t nz) {
  const int64_t nvox = nx * ny * nz, nedge = 3 * nvox;
  const int64_t ncell = (nx - 1) * (ny - 1) * (nz - 1);
  const int64_t nmax = nvox > ncell ? nvox : ncell;
  McLayout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) & ~(size_t)255;
    return o;
  };
  L.bits = take((size_t)nvox);
  L.info = take(sizeof(uint16_t) * (size_t)ncell);
  L.vid = take(sizeof(uint32_t) * (size_t)nedge);  // written only for used edges
  L.sums = take(sizeof(uint64_t) * (size_t)(compact_blocks(nmax) + 1));
  L.totals = take(16);
  L.total = off;
  return L;
}

}  // namespace

void marching_cubes_table(uint8_t* ntri, uint8_t* tri) {
  for (int c = 0; c < 256; ++c) {
    ntri[c] = kMcHost.ntri[c];
    for (int k = 0; k < 3 * kMcMaxTri; ++k) tri[c * 3 * kMcMaxTri + k] = kMcHost.tri[c][k];
  }
}

size_t marching_cubes_workspace(int64_t nx, int64_t ny, int64_t nz) {
  return mc_layout(nx, ny, nz).total;
}

// Enqueues the whole extraction; the counts are left in the workspace
// (uint32 vertices at *nv_dev, uint64 triangles at *nt_dev).
hipError_t launch_marching_cubes(const float* tsdf, const float* weight, int64_t nx, int64_t ny,
                                 int64_t nz, const double* origin, double voxel, float iso,
                                 void* ws, float* verts, int64_t max_verts, uint32_t* tris,
                                 int64_t max_tris, const uint32_t** nv_dev,
                                 const uint64_t** nt_dev, hipStream_t st) {
  const McLayout L = mc_layout(nx, ny, nz);
  char* base = (char*)ws;
  uint8_t* bits = (uint8_t*)(base + L.bits);
  uint16_t* info = (uint16_t*)(base + L.info);
  uint32_t* vid = (uint32_t*)(base + L.vid);
  void* sums = base + L.sums;
  uint64_t* nt = (uint64_t*)(base + L.totals);
  uint32_t* nv = (uint32_t*)(base + L.totals + 8);
  *nv_dev = nv;
  *nt_dev = nt;
  const int64_t nvox = nx * ny * nz;
  const int64_t ncell = (nx - 1) * (ny - 1) * (nz - 1);
  if (ncell == 0) {  // a flat grid has no cell: empty mesh
    hipLaunchKernelGGL(k_mc_zero_counts, dim3(1), dim3(1), 0, st, nv, nt);
    return hipGetLastError();
  }
  // every index fits 32 bits: 3 nx ny nz <= 2^32 - 1 is checked by the caller
  const Grid3 vox((uint32_t)nx, (uint32_t)ny);
  const Grid3 cells((uint32_t)(nx - 1), (uint32_t)(ny - 1));
  hipLaunchKernelGGL(k_mc_bits, dim3(grid_for(nvox)), dim3(kT), 0, st, tsdf, weight,
                     (uint64_t)nvox, iso, bits);
  hipLaunchKernelGGL(k_mc_cells, dim3(grid_for(ncell)), dim3(kT), 0, st, bits, (uint32_t)nx,
                     (uint32_t)ny, (uint32_t)ncell, cells, info);
  const VoxelEdges edges{bits, info, vox, (uint32_t)nz};
  scan_emit<uint32_t>(edges, nvox, (uint32_t*)sums, nv,
                      EmitVertices{edges, tsdf, origin[0], origin[1], origin[2], voxel, iso, vid,
                                   verts, max_verts},
                      st);
  scan_emit<uint64_t>(CellTriangles{info}, ncell, (uint64_t*)sums, nt,
                      EmitTriangles{info, vid, cells, (uint32_t)nx, (uint32_t)ny, tris, max_tris},
                      st);
  return hipGetLastError();
}

}  // namespace rade
