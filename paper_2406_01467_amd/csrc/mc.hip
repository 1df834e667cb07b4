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
// Pipeline: cell codes and triangle counts -> edge flags (crossed and used by
// an observed cell) -> exclusive scans (vertex id per grid edge, triangle
// offset per cell) -> vertices at the linear zero of each used edge (FP64) ->
// triangles.  Vertices are ordered by global edge id 3 q + a, triangles by
// cell index then the cell's rule order, so the mesh is deterministic.
#include "common.hpp"
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

inline unsigned grid_for(int64_t n) {
  int64_t b = (n + kT - 1) / kT;
  if (b > ((int64_t)1 << 20)) b = (int64_t)1 << 20;  // grid-stride beyond
  return (unsigned)(b > 0 ? b : 1);
}

// Cell codes (bit 8: all corners observed) and triangle counts.
__global__ void __launch_bounds__(kT)
k_mc_cells(const float* __restrict__ f, const float* __restrict__ w, int64_t nx, int64_t ny,
           int64_t nz, float iso, uint16_t* __restrict__ info, uint64_t* __restrict__ ntri) {
  const int64_t cx = nx - 1, cy = ny - 1, ncell = cx * cy * (nz - 1);
  for (int64_t c = (int64_t)blockIdx.x * kT + threadIdx.x; c < ncell;
       c += (int64_t)gridDim.x * kT) {
    const int64_t i = c % cx, j = (c / cx) % cy, k = c / (cx * cy);
    const int64_t q0 = (k * ny + j) * nx + i;
    int code = 0;
    bool observed = true;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const int64_t q = q0 + (b & 1) + ((b >> 1) & 1) * nx + ((b >> 2) & 1) * nx * ny;
      observed = observed && w[q] > 0.0f;
      code |= (f[q] < iso ? 1 : 0) << b;
    }
    info[c] = observed ? (uint16_t)(kObserved | code) : (uint16_t)0;
    ntri[c] = observed ? (uint64_t)kMc.ntri[code] : 0;
  }
}

// 1 for a grid edge that changes sign between two observed voxels and
// belongs to an observed cell.
__global__ void __launch_bounds__(kT)
k_mc_edges(const float* __restrict__ f, const float* __restrict__ w,
           const uint16_t* __restrict__ info, int64_t nx, int64_t ny, int64_t nz, float iso,
           uint32_t* __restrict__ flag) {
  const int64_t nvox = nx * ny * nz, nedge = 3 * nvox;
  const int64_t n[3] = {nx, ny, nz};
  for (int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x; e < nedge;
       e += (int64_t)gridDim.x * kT) {
    const int64_t q = e / 3;
    const int a = (int)(e - 3 * q);
    const int64_t p[3] = {q % nx, (q / nx) % ny, q / (nx * ny)};
    uint32_t out = 0;
    if (p[a] + 1 < n[a]) {
      const int64_t q1 = q + (a == 0 ? 1 : a == 1 ? nx : nx * ny);
      const bool cross = w[q] > 0.0f && w[q1] > 0.0f && ((f[q] < iso) != (f[q1] < iso));
      if (cross) {
        const int u = a == 0 ? 1 : 0, v = a == 2 ? 1 : 2;
        for (int s = 0; s < 4 && !out; ++s) {
          int64_t c[3] = {p[0], p[1], p[2]};
          c[u] -= s & 1;
          c[v] -= s >> 1;
          if (c[u] < 0 || c[u] >= n[u] - 1 || c[v] < 0 || c[v] >= n[v] - 1) continue;
          const int64_t cell = (c[2] * (ny - 1) + c[1]) * (nx - 1) + c[0];
          if (info[cell] & kObserved) out = 1;
        }
      }
    }
    flag[e] = out;
  }
}

// Vertex of every used edge (vid holds the exclusive scan of the flags).
__global__ void __launch_bounds__(kT)
k_mc_verts(const float* __restrict__ f, int64_t nx, int64_t ny, int64_t nz, double o0, double o1,
           double o2, double voxel, float iso, const uint32_t* __restrict__ vid,
           const uint32_t* __restrict__ nv_total, float* __restrict__ verts, int64_t max_verts) {
  const int64_t nedge = 3 * nx * ny * nz;
  const uint32_t total = *nv_total;
  for (int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x; e < nedge;
       e += (int64_t)gridDim.x * kT) {
    const uint32_t id = vid[e];
    const uint32_t next = e + 1 < nedge ? vid[e + 1] : total;
    if (next == id || (int64_t)id >= max_verts) continue;
    const int64_t q = e / 3;
    const int a = (int)(e - 3 * q);
    const int64_t q1 = q + (a == 0 ? 1 : a == 1 ? nx : nx * ny);
    const double f0 = f[q], f1 = f[q1];
    const double t = ((double)iso - f0) / (f1 - f0);
    double x = o0 + ((double)(q % nx) + 0.5) * voxel;
    double y = o1 + ((double)((q / nx) % ny) + 0.5) * voxel;
    double z = o2 + ((double)(q / (nx * ny)) + 0.5) * voxel;
    if (a == 0) x += t * voxel;
    if (a == 1) y += t * voxel;
    if (a == 2) z += t * voxel;
    verts[3 * (int64_t)id + 0] = (float)x;
    verts[3 * (int64_t)id + 1] = (float)y;
    verts[3 * (int64_t)id + 2] = (float)z;
  }
}

// Triangles of every observed cell (toff holds the exclusive scan of the counts).
__global__ void __launch_bounds__(kT)
k_mc_tris(const uint16_t* __restrict__ info, const uint64_t* __restrict__ toff,
          const uint32_t* __restrict__ vid, int64_t nx, int64_t ny, int64_t nz,
          uint32_t* __restrict__ tris, int64_t max_tris) {
  const int64_t cx = nx - 1, cy = ny - 1, ncell = cx * cy * (nz - 1);
  for (int64_t c = (int64_t)blockIdx.x * kT + threadIdx.x; c < ncell;
       c += (int64_t)gridDim.x * kT) {
    const uint16_t inf = info[c];
    if (!(inf & kObserved)) continue;
    const int code = inf & 0xff;
    const int n = kMc.ntri[code];
    if (n == 0) continue;
    const int64_t i = c % cx, j = (c / cx) % cy, k = c / (cx * cy);
    const int64_t base = (int64_t)toff[c];
    for (int t = 0; t < n; ++t) {
      if (base + t >= max_tris) break;
      for (int m = 0; m < 3; ++m) {
        const int e = kMc.tri[code][3 * t + m];
        const int a = e >> 2;
        int64_t p[3] = {i, j, k};
        p[a == 0 ? 1 : 0] += e & 1;
        p[a == 2 ? 1 : 2] += (e >> 1) & 1;
        const int64_t ge = 3 * ((p[2] * ny + p[1]) * nx + p[0]) + a;
        tris[3 * (base + t) + m] = vid[ge];
      }
    }
  }
}

struct McLayout {
  size_t info, toff, vid, sums, totals, total;
};

McLayout mc_layout(int64_t nx, int64_t ny, int64_t nz) {
  const int64_t nvox = nx * ny * nz, nedge = 3 * nvox;
  const int64_t ncell = (nx - 1) * (ny - 1) * (nz - 1);
  const int64_t nmax = nedge > ncell ? nedge : ncell;
  McLayout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) & ~(size_t)255;
    return o;
  };
  L.info = take(sizeof(uint16_t) * (size_t)ncell);
  L.toff = take(sizeof(uint64_t) * (size_t)ncell);
  L.vid = take(sizeof(uint32_t) * (size_t)nedge);
  L.sums = take(sizeof(uint64_t) * (size_t)((nmax + kScanTile - 1) / kScanTile + 1));
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
  uint16_t* info = (uint16_t*)(base + L.info);
  uint64_t* toff = (uint64_t*)(base + L.toff);
  uint32_t* vid = (uint32_t*)(base + L.vid);
  void* sums = base + L.sums;
  uint64_t* nt = (uint64_t*)(base + L.totals);
  uint32_t* nv = (uint32_t*)(base + L.totals + 8);
  *nv_dev = nv;
  *nt_dev = nt;
  const int64_t nedge = 3 * nx * ny * nz;
  const int64_t ncell = (nx - 1) * (ny - 1) * (nz - 1);
  if (ncell > 0) {
    hipLaunchKernelGGL(k_mc_cells, dim3(grid_for(ncell)), dim3(kT), 0, st, tsdf, weight, nx, ny,
                       nz, iso, info, toff);
  }
  hipLaunchKernelGGL(k_mc_edges, dim3(grid_for(nedge)), dim3(kT), 0, st, tsdf, weight, info, nx,
                     ny, nz, iso, vid);
  // in place: each scan thread reads its items before writing them
  scan<uint32_t>(PlainInput{vid}, nedge, nullptr, vid, (uint32_t*)sums, nv, st);
  scan<uint64_t>(PlainInput64{toff}, ncell, nullptr, toff, (uint64_t*)sums, nt, st);
  hipLaunchKernelGGL(k_mc_verts, dim3(grid_for(nedge)), dim3(kT), 0, st, tsdf, nx, ny, nz,
                     origin[0], origin[1], origin[2], voxel, iso, vid, nv, verts, max_verts);
  if (ncell > 0) {
    hipLaunchKernelGGL(k_mc_tris, dim3(grid_for(ncell)), dim3(kT), 0, st, info, toff, vid, nx, ny,
                       nz, tris, max_tris);
  }
  return hipGetLastError();
}

}  // namespace rade
