// HIP kernels (gfx950) of the MUSTER iteration.
//
// Data layout: a volume is float32 [D][H][W] (x fastest); a vector field is
// three such planes (components z, y, x).  Fields hold displacements in
// voxels.  Every kernel walks a table of work items (see muster_internal.h),
// so one launch covers all intervals, pairs and subjects of a stage.
//
// Sampling (paper Sec. 2.2, "trilinear interpolation"): the sample position
// q = p + u is clamped to the grid; the cell index is p + floor(u) and the
// fraction u - floor(u), which keeps the fraction exact for large p; an axis
// whose coordinate was clamped contributes no derivative.  Interpolation is
// the nested linear form a + t (b - a), so a constant field is reproduced
// exactly.
//
// The gather/scatter kernels use 8x8x16-voxel tiles and an XCD-aware
// block-to-tile map: blocks are dealt round-robin over the 8 XCDs, and the
// map hands each XCD a contiguous run of tiles so the neighbouring rows that
// the gathers touch stay in that XCD's L2.
#include <map>
#include <mutex>
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <climits>
#include <cmath>

#include "muster_internal.h"

namespace muster {

namespace {

// Field pointers are used through the global address space so that loads,
// stores and atomics compile to global (not flat) memory instructions.
#define GLOBAL __attribute__((address_space(1)))
typedef GLOBAL float gfloat;
typedef GLOBAL const float cgfloat;
typedef float float2a __attribute__((ext_vector_type(2), aligned(4)));

__device__ __forceinline__ const cgfloat* gp(const float* p) { return (const cgfloat*)p; }
__device__ __forceinline__ gfloat* gp(float* p) { return (gfloat*)p; }
__device__ __forceinline__ void gadd(gfloat* p, float v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

constexpr float EPS_LNCC = 1e-10f;
constexpr float EPS_SILNCC = 1e-6f;

__device__ __forceinline__ int xcd_remap(int b, int n) {
  const int q = n >> 3, r = n & 7;
  const int x = b & 7, j = b >> 3;
  return x * q + min(x, r) + j;
}

template <class Item>
__device__ __forceinline__ int find_item(const Item* __restrict__ items, int n, int tile) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (items[mid].tile0 <= tile) lo = mid; else hi = mid - 1;
  }
  return lo;
}

struct Ax {
  int i0;
  float t;
  float live;  // 1 inside the grid, 0 where the coordinate was clamped
};

// Axis of a displaced position p + u on n grid points.
__device__ __forceinline__ Ax axis_disp(int p, float u, int n) {
  u = fminf(fmaxf(u, -1.0e6f), 1.0e6f);
  const float fl = floorf(u);
  const int i = p + (int)fl;
  const float t = u - fl;
  Ax a;
  if (i < 0) {
    a.i0 = 0; a.t = 0.f; a.live = 0.f;
  } else if (i >= n - 1) {
    a.i0 = n - 2; a.t = 1.f; a.live = (i == n - 1 && t == 0.f) ? 1.f : 0.f;
  } else {
    a.i0 = i; a.t = t; a.live = 1.f;
  }
  return a;
}

// Axis of an absolute position q on n grid points.
__device__ __forceinline__ Ax axis_pos(float q, int n) {
  q = fminf(fmaxf(q, -1.0e6f), 1.0e6f);
  const float fl = floorf(q);
  const int i = (int)fl;
  const float t = q - fl;
  Ax a;
  if (i < 0) {
    a.i0 = 0; a.t = 0.f; a.live = 0.f;
  } else if (i >= n - 1) {
    a.i0 = n - 2; a.t = 1.f; a.live = (i == n - 1 && t == 0.f) ? 1.f : 0.f;
  } else {
    a.i0 = i; a.t = t; a.live = 1.f;
  }
  return a;
}

__device__ __forceinline__ float lerp_(float a, float b, float t) { return fmaf(t, b - a, a); }

// Two consecutive floats in one 8-byte load (dword alignment suffices for
// multi-dword global loads); halves the address work of a gather.
__device__ __forceinline__ float2a ld2(const cgfloat* p) { return *(const GLOBAL float2a*)p; }

// Loads at element i of a plane whose base is uniform across the wave: the
// byte offset is formed in 32 bits (i < 2^30 for any volume the library
// accepts), so the load takes the scalar base plus a 32-bit vector offset
// instead of a 64-bit vector address.
__device__ __forceinline__ float2a ld2o(const cgfloat* plane, uint32_t i) {
  return *(const GLOBAL float2a*)((const GLOBAL char*)plane + (i << 2));
}

__device__ __forceinline__ float ldo(const cgfloat* plane, uint32_t i) {
  return *(const GLOBAL float*)((const GLOBAL char*)plane + (i << 2));
}
// One float per lane from global memory straight into LDS: lane l of the
// wave writes lds_wave[l], where lds_wave is the same for the whole wave (the
// first element of its run).  No register holds the value, and the barrier
// that follows waits for the load like for any other.  The callers walk
// element i = threadIdx.x + k * (block size), with block sizes multiples of
// 64, so a wave's run starts at i & ~63; lanes past the end stay inactive
// and write nothing.
__device__ __forceinline__ void ld_to_lds(const cgfloat* src, float* lds_wave) {
  __builtin_amdgcn_global_load_lds((const GLOBAL void*)src,
                                   (__attribute__((address_space(3))) void*)lds_wave, 4, 0, 0);
}

__device__ __forceinline__ void sto(gfloat* plane, uint32_t i, float v) {
  *(GLOBAL float*)((GLOBAL char*)plane + (i << 2)) = v;
}

// The 8 corners of a cell.  Corner order: bit 0 = x+1, bit 1 = y+1,
// bit 2 = z+1; the x pairs are adjacent in memory and come in one load.
__device__ __forceinline__ void load8(const cgfloat* __restrict__ f, int base, int sy, int sz,
                                      float (&v)[8]) {
  const uint32_t b0 = (uint32_t)base;
  const float2a a = ld2o(f, b0);
  const float2a b = ld2o(f, b0 + (uint32_t)sy);
  const float2a c = ld2o(f, b0 + (uint32_t)sz);
  const float2a d = ld2o(f, b0 + (uint32_t)(sz + sy));
  v[0] = a.x; v[1] = a.y;
  v[2] = b.x; v[3] = b.y;
  v[4] = c.x; v[5] = c.y;
  v[6] = d.x; v[7] = d.y;
}

__device__ __forceinline__ float tri_val(const float (&v)[8], float tz, float ty, float tx) {
  const float c00 = lerp_(v[0], v[1], tx);
  const float c01 = lerp_(v[2], v[3], tx);
  const float c10 = lerp_(v[4], v[5], tx);
  const float c11 = lerp_(v[6], v[7], tx);
  const float c0 = lerp_(c00, c01, ty);
  const float c1 = lerp_(c10, c11, ty);
  return lerp_(c0, c1, tz);
}

// Value and the three partial derivatives of the trilinear interpolant.
__device__ __forceinline__ float tri_grad(const float (&v)[8], float tz, float ty, float tx,
                                          float& dz, float& dy, float& dx) {
  const float c00 = lerp_(v[0], v[1], tx);
  const float c01 = lerp_(v[2], v[3], tx);
  const float c10 = lerp_(v[4], v[5], tx);
  const float c11 = lerp_(v[6], v[7], tx);
  const float c0 = lerp_(c00, c01, ty);
  const float c1 = lerp_(c10, c11, ty);
  dz = c1 - c0;
  dy = lerp_(c01 - c00, c11 - c10, tz);
  const float e0 = lerp_(v[1] - v[0], v[3] - v[2], ty);
  const float e1 = lerp_(v[5] - v[4], v[7] - v[6], ty);
  dx = lerp_(e0, e1, tz);
  return lerp_(c0, c1, tz);
}

struct PTile {
  int z0, y0, x0;
};

__device__ __forceinline__ PTile point_tile(int local, int H, int W) {
  const int ntx = (W + PT_X - 1) / PT_X;
  const int nty = (H + PT_Y - 1) / PT_Y;
  PTile t;
  t.x0 = (local % ntx) * PT_X;
  const int r = local / ntx;
  t.y0 = (r % nty) * PT_Y;
  t.z0 = (r / nty) * PT_Z;
  return t;
}

// Sum over a block of NT threads; the result is valid in thread 0.
template <int NT = BLOCK>
__device__ __forceinline__ double block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < NT / 64; ++i) s += red[i];
  return s;
}

// Minimum / maximum over a wave: four DPP steps leave each row of 16 lanes
// holding its row's result (swap neighbours, swap pairs, mirror the half
// rows, mirror the rows), and the four row results are read from lanes 15,
// 31, 47 and 63.  The result is wave-uniform.  Every lane must be active.
__device__ __forceinline__ int dpp_min(int v) {
  v = min(v, __builtin_amdgcn_update_dpp(v, v, 0xB1, 0xF, 0xF, false));
  v = min(v, __builtin_amdgcn_update_dpp(v, v, 0x4E, 0xF, 0xF, false));
  v = min(v, __builtin_amdgcn_update_dpp(v, v, 0x141, 0xF, 0xF, false));
  v = min(v, __builtin_amdgcn_update_dpp(v, v, 0x140, 0xF, 0xF, false));
  return min(min(__builtin_amdgcn_readlane(v, 15), __builtin_amdgcn_readlane(v, 31)),
             min(__builtin_amdgcn_readlane(v, 47), __builtin_amdgcn_readlane(v, 63)));
}
__device__ __forceinline__ int dpp_max(int v) {
  v = max(v, __builtin_amdgcn_update_dpp(v, v, 0xB1, 0xF, 0xF, false));
  v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x4E, 0xF, 0xF, false));
  v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x141, 0xF, 0xF, false));
  v = max(v, __builtin_amdgcn_update_dpp(v, v, 0x140, 0xF, 0xF, false));
  return max(max(__builtin_amdgcn_readlane(v, 15), __builtin_amdgcn_readlane(v, 31)),
             max(__builtin_amdgcn_readlane(v, 47), __builtin_amdgcn_readlane(v, 63)));
}

// Sum over a wave by the same four DPP steps: after them every lane of a row
// holds its row's sum, in the same order in every lane, so the result is
// wave-uniform and does not depend on the lane a value came from.
__device__ __forceinline__ float dpp_sum(float v) {
  v += __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), 0xB1, 0xF, 0xF, false));
  v += __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), 0x4E, 0xF, 0xF, false));
  v += __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), 0x141, 0xF, 0xF, false));
  v += __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(v), __float_as_int(v), 0x140, 0xF, 0xF, false));
  const float a = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 15));
  const float b = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 31));
  const float c = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 47));
  const float d = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
  return (a + b) + (c + d);
}

// Bounding box of the cells a tile touches.
struct BBox {
  int lz, ly, lx, ez, ey, ex, cells;
};

// Regulariser of Eq. reg_ss at voxel p for one component plane f: forward
// differences, mean per (component, axis) over its valid set.  Returns the
// gradient of R with respect to f(p) and adds f's own forward-difference terms
// to *val.
__device__ __forceinline__ float reg_point(const cgfloat* __restrict__ f, int z, int y, int x, int D,
                                           int H, int W, float inv_mz, float inv_my, float inv_mx,
                                           double* val) {
  const int HW = H * W;
  const int p = (z * H + y) * W + x;
  const float c = f[p];
  float g = 0.f;
  if (z + 1 < D) { const float d = f[p + HW] - c; g -= 2.f * d * inv_mz; *val += (double)d * d * inv_mz; }
  if (z > 0)     { const float d = c - f[p - HW]; g += 2.f * d * inv_mz; }
  if (y + 1 < H) { const float d = f[p + W] - c;  g -= 2.f * d * inv_my; *val += (double)d * d * inv_my; }
  if (y > 0)     { const float d = c - f[p - W];  g += 2.f * d * inv_my; }
  if (x + 1 < W) { const float d = f[p + 1] - c;  g -= 2.f * d * inv_mx; *val += (double)d * d * inv_mx; }
  if (x > 0)     { const float d = c - f[p - 1];  g += 2.f * d * inv_mx; }
  return g;
}

// The same regulariser read from a halo tile in LDS: the field over a point
// tile and one voxel around it (coordinates clamped to the grid; a clamped
// neighbour is never used), three component planes of RH_N values.
constexpr int RH_Z = PT_Z + 2, RH_Y = PT_Y + 2, RH_X = PT_X + 2, RH_N = RH_Z * RH_Y * RH_X;
static_assert(RH_N <= SCATTER_CELLS, "the halo tile must fit the scatter bins");

__device__ __forceinline__ void reg_tile_load(const cgfloat* __restrict__ f, int V, int z0, int y0,
                                              int x0, int D, int H, int W, float* __restrict__ t) {
  for (int i = threadIdx.x; i < 3 * RH_N; i += BLOCK) {
    const int c = i / RH_N, r = i - c * RH_N;
    const int hz = r / (RH_Y * RH_X), r2 = r - hz * (RH_Y * RH_X);
    const int hy = r2 / RH_X, hx = r2 - hy * RH_X;
    const int z = min(max(z0 - 1 + hz, 0), D - 1);
    const int y = min(max(y0 - 1 + hy, 0), H - 1);
    const int x = min(max(x0 - 1 + hx, 0), W - 1);
    ld_to_lds(f + c * V + (z * H + y) * W + x, t + (i & ~63));  // i = threadIdx.x + k * BLOCK
  }
}

__device__ __forceinline__ float reg_tile_point(const float* __restrict__ t, int lz, int ly, int lx,
                                                int z, int y, int x, int D, int H, int W,
                                                float inv_mz, float inv_my, float inv_mx,
                                                float* val) {
  constexpr int SZ = RH_Y * RH_X, SY = RH_X;
  const int q = ((lz + 1) * RH_Y + ly + 1) * RH_X + lx + 1;
  const float c = t[q];
  float g = 0.f, e = 0.f;
  if (z + 1 < D) { const float d = t[q + SZ] - c; g -= 2.f * d * inv_mz; e = fmaf(d * d, inv_mz, e); }
  if (z > 0)     { const float d = c - t[q - SZ]; g += 2.f * d * inv_mz; }
  if (y + 1 < H) { const float d = t[q + SY] - c; g -= 2.f * d * inv_my; e = fmaf(d * d, inv_my, e); }
  if (y > 0)     { const float d = c - t[q - SY]; g += 2.f * d * inv_my; }
  if (x + 1 < W) { const float d = t[q + 1] - c;  g -= 2.f * d * inv_mx; e = fmaf(d * d, inv_mx, e); }
  if (x > 0)     { const float d = c - t[q - 1];  g += 2.f * d * inv_mx; }
  *val += e;
  return g;
}

// ---------------------------------------------------------------------------
// Point tiles.  A thread owns VPT voxels of an 8x8x16 tile.  Their loads are
// issued together, component by component across the voxels, so each round
// trip to memory carries VPT gathers per thread: the gather kernels are bound
// by memory latency, not by bandwidth or address throughput, so memory-level
// parallelism is what sets their speed.  Voxels beyond the grid are clamped
// onto it (their loads stay in bounds) and their results are discarded.
// ---------------------------------------------------------------------------
constexpr int VPT = PT_VOX / BLOCK;

struct VoxSet {
  int p[VPT];           // linear index of the (clamped) voxel
  int z[VPT], y[VPT], x[VPT];
  bool ok[VPT];
};

__device__ __forceinline__ void vox_set(const PTile& tc, int D, int H, int W, VoxSet& vs) {
#pragma unroll
  for (int j = 0; j < VPT; ++j) {
    const int k = threadIdx.x + j * BLOCK;
    const int x = tc.x0 + (k % PT_X), y = tc.y0 + (k / PT_X) % PT_Y, z = tc.z0 + k / (PT_X * PT_Y);
    vs.ok[j] = x < W && y < H && z < D;
    vs.x[j] = min(x, W - 1);
    vs.y[j] = min(y, H - 1);
    vs.z[j] = min(z, D - 1);
    vs.p[j] = (vs.z[j] * H + vs.y[j]) * W + vs.x[j];
  }
}

struct CellSet {
  int base[VPT];
  Ax az[VPT], ay[VPT], ax[VPT];
};

// Displacements (scaled by a) of the owned voxels and the cells they sample.
__device__ __forceinline__ void load_cells(const cgfloat* __restrict__ u, float a, int D, int H,
                                           int W, const VoxSet& vs, float (&uu)[VPT][3],
                                           CellSet& cs) {
  const int V = D * H * W;
#pragma unroll
  for (int j = 0; j < VPT; ++j) {
    uu[j][0] = a * ldo(u, vs.p[j]);
    uu[j][1] = a * ldo(u + V, vs.p[j]);
    uu[j][2] = a * ldo(u + 2 * V, vs.p[j]);
  }
#pragma unroll
  for (int j = 0; j < VPT; ++j) {
    cs.az[j] = axis_disp(vs.z[j], uu[j][0], D);
    cs.ay[j] = axis_disp(vs.y[j], uu[j][1], H);
    cs.ax[j] = axis_disp(vs.x[j], uu[j][2], W);
    cs.base[j] = (cs.az[j].i0 * H + cs.ay[j].i0) * W + cs.ax[j].i0;
  }
}

// Trilinear values of the three components of f at the cells.
__device__ __forceinline__ void sample_cells(const cgfloat* __restrict__ f, int V, int H, int W,
                                             const CellSet& cs, float (&out)[VPT][3]) {
  const int HW = H * W;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    float v[VPT][8];
#pragma unroll
    for (int j = 0; j < VPT; ++j) load8(f + c * V, cs.base[j], W, HW, v[j]);
#pragma unroll
    for (int j = 0; j < VPT; ++j) out[j][c] = tri_val(v[j], cs.az[j].t, cs.ay[j].t, cs.ax[j].t);
  }
}

// (J^T g) at the cells, J the Jacobian of a * f (rows: components of f,
// columns: z, y, x; clamped axes contribute nothing).
__device__ __forceinline__ void jt_cells(const cgfloat* __restrict__ f, float a, int V, int H,
                                         int W, const CellSet& cs, const float (&g)[VPT][3],
                                         float (&acc)[VPT][3]) {
  const int HW = H * W;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    float v[VPT][8];
#pragma unroll
    for (int j = 0; j < VPT; ++j) load8(f + c * V, cs.base[j], W, HW, v[j]);
#pragma unroll
    for (int j = 0; j < VPT; ++j) {
      float dz, dy, dx;
      tri_grad(v[j], cs.az[j].t, cs.ay[j].t, cs.ax[j].t, dz, dy, dx);
      const float gc = a * g[j][c];
      acc[j][0] = fmaf(dz * cs.az[j].live, gc, acc[j][0]);
      acc[j][1] = fmaf(dy * cs.ay[j].live, gc, acc[j][1]);
      acc[j][2] = fmaf(dx * cs.ax[j].live, gc, acc[j][2]);
    }
  }
}

// Scatter of per-voxel cell contributions into a field through LDS bins.
// Each thread holds up to VPT voxels: cell origin (cz, cy, cx), fractions,
// the 3-vector to spread with the trilinear weights, and optionally an own
// term to add at its own position (oz, oy, ox).
//
// The bins are 32-bit fixed point: every contribution is scaled by
// min(2^23 / m, 2^30 / S), where m is the largest magnitude the block
// spreads and S the sum over its voxels of their largest magnitudes,
// truncated, and added with an integer LDS atomic; integer LDS atomics run
// several times faster than float ones on this hardware and make the in-block
// sum independent of the order of the adds.  A bin holds at most the weighted
// values of the block's voxels, so its magnitude stays below 2^30 however
// strongly the sampling positions crowd into one cell: no bin can overflow.
// The error per contribution is below one quantum, 2^-23 m for spread-out
// boxes and 2^-30 S where many voxels share cells.  Each non-zero bin is then
// added to the field with one hardware float atomic.
constexpr float FIX_SCALE = 8388608.0f;   // 2^23
constexpr float FIX_TOTAL = 1073741824.0f; // 2^30
static_assert(SCATTER_CELLS % 4 == 0, "bin planes are cleared as int4");

struct ScatterVox {
  int cz, cy, cx;      // cell origin; cz < 0 marks an empty slot
  int oz, oy, ox;      // own voxel (for the own term)
  float tz, ty, tx;
  float g[3];          // value spread over the 8 corners
  float own[3];        // value added at the own voxel
};

// Bounding box (lo/hi per axis), largest magnitude and sum of magnitudes over
// the block in one reduction: wave DPP steps, one LDS exchange, one barrier.
struct ScatterBox {
  BBox bb;
  float bmax;
  float bsum;
};

template <int NT>
__device__ __forceinline__ ScatterBox scatter_box(int (&lo)[3], int (&hi)[3], float mx, float sm,
                                                  int* sred) {
  // mx >= 0 (fmaxf drops NaN operands), so its bits order like its values
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    lo[d] = dpp_min(lo[d]);
    hi[d] = dpp_max(hi[d]);
  }
  const int mxb = dpp_max(__float_as_int(mx));
  const float smw = dpp_sum(sm);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      sred[w * 8 + d] = lo[d];
      sred[w * 8 + 3 + d] = hi[d];
    }
    sred[w * 8 + 6] = mxb;
    sred[w * 8 + 7] = __float_as_int(smw);
  }
  __syncthreads();
  int l[3] = {INT_MAX, INT_MAX, INT_MAX}, h[3] = {INT_MIN, INT_MIN, INT_MIN};
  int mb = 0;
  float sb_sum = 0.f;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      l[d] = min(l[d], sred[i * 8 + d]);
      h[d] = max(h[d], sred[i * 8 + 3 + d]);
    }
    mb = max(mb, sred[i * 8 + 6]);
    sb_sum += __int_as_float(sred[i * 8 + 7]);
  }
  ScatterBox sb;
  sb.bmax = __int_as_float(mb);
  sb.bsum = sb_sum;
  sb.bb.lz = l[0]; sb.bb.ly = l[1]; sb.bb.lx = l[2];
  if (h[0] < l[0]) {
    sb.bb.ez = sb.bb.ey = sb.bb.ex = 0;
    sb.bb.cells = 0;
    return sb;
  }
  sb.bb.ez = h[0] - l[0] + 1;
  sb.bb.ey = h[1] - l[1] + 1;
  sb.bb.ex = h[2] - l[2] + 1;
  const long long c = (long long)sb.bb.ez * sb.bb.ey * sb.bb.ex;
  sb.bb.cells = c > (long long)INT_MAX ? INT_MAX : (int)c;
  return sb;
}

// ---------------------------------------------------------------------------
// Gathers from a box staged in LDS.  The block reduces the bounding box of
// the cells its voxels sample (the reduction of the scatters), loads that box
// of the three component planes straight into LDS (coalesced loads that do
// not pass through registers), and reads the 8 corners of each cell there.  A few wide row loads per cell then replace
// the scattered corner loads of every voxel, which otherwise keep the L1 and
// texture path saturated.  The values and the arithmetic are those of
// sample_cells, so the result is bit-identical; a box larger than
// GATHER_CELLS falls back to sample_cells.  box: LDS of 3 * GATHER_CELLS
// floats.  Every thread of the block must call this.
//
// 2560 cells (30 KB of LDS) let five blocks share a CU, and the kernels that
// stage a box are held to five waves per SIMD (at most 102 VGPRs, no spill):
// 3-7 % faster than 3072 cells at four waves.  2048 cells at six waves per
// SIMD (80 VGPRs, a few bytes of spill) ran no faster.
// ---------------------------------------------------------------------------
constexpr int GATHER_CELLS = 2560;
// The adjoints read their corners from a box in the scatter bins' LDS.
constexpr int ADJ_BOX_CELLS = GATHER_CELLS < SCATTER_CELLS ? GATHER_CELLS : SCATTER_CELLS;
#define GATHER_WAVES __attribute__((amdgpu_waves_per_eu(5)))

__device__ __forceinline__ void sample_cells_lds(const cgfloat* __restrict__ f, int V, int H, int W,
                                                 const VoxSet& vs, const CellSet& cs,
                                                 float* __restrict__ box, int* sred,
                                                 float (&out)[VPT][3]) {
  int lo[3] = {INT_MAX, INT_MAX, INT_MAX};
  int hi[3] = {INT_MIN, INT_MIN, INT_MIN};
#pragma unroll
  for (int j = 0; j < VPT; ++j) {
    if (!vs.ok[j]) continue;
    lo[0] = min(lo[0], cs.az[j].i0); hi[0] = max(hi[0], cs.az[j].i0 + 1);
    lo[1] = min(lo[1], cs.ay[j].i0); hi[1] = max(hi[1], cs.ay[j].i0 + 1);
    lo[2] = min(lo[2], cs.ax[j].i0); hi[2] = max(hi[2], cs.ax[j].i0 + 1);
  }
  const BBox bb = scatter_box<BLOCK>(lo, hi, 0.f, 0.f, sred).bb;
  if (bb.cells == 0 || bb.cells > GATHER_CELLS) {  // block-uniform
    sample_cells(f, V, H, W, cs, out);
    return;
  }
  const int cells = bb.cells;
  // cell i -> (lz, ly, lx) by float reciprocals: exact here since i < 2^22
  const float inv_ex = 1.f / (float)bb.ex, inv_ey = 1.f / (float)bb.ey;
  for (int i = threadIdx.x; i < cells; i += BLOCK) {
    const int r = (int)(((float)i + 0.5f) * inv_ex);
    const int lx = i - r * bb.ex;
    const int lz = (int)(((float)r + 0.5f) * inv_ey);
    const int ly = r - lz * bb.ey;
    const int g = ((bb.lz + lz) * H + (bb.ly + ly)) * W + (bb.lx + lx);
    const int w0 = i & ~63;  // the wave's first cell: i = threadIdx.x + k * block
    ld_to_lds(f + g, box + w0);
    ld_to_lds(f + V + g, box + cells + w0);
    ld_to_lds(f + 2 * V + g, box + 2 * cells + w0);
  }
  __syncthreads();
  const int sy = bb.ex, sz = bb.ex * bb.ey;
  int l[VPT];
#pragma unroll
  for (int j = 0; j < VPT; ++j)
    l[j] = vs.ok[j] ? ((cs.az[j].i0 - bb.lz) * bb.ey + (cs.ay[j].i0 - bb.ly)) * bb.ex +
                          (cs.ax[j].i0 - bb.lx)
                    : 0;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float* __restrict__ b = box + c * cells;
#pragma unroll
    for (int j = 0; j < VPT; ++j) {
      const float* q = b + l[j];
      const float v[8] = {q[0], q[1], q[sy], q[sy + 1], q[sz], q[sz + 1], q[sz + sy], q[sz + sy + 1]};
      out[j][c] = tri_val(v, cs.az[j].t, cs.ay[j].t, cs.ax[j].t);
    }
  }
}

// ---------------------------------------------------------------------------
// Exp forward: one squaring u' = u + u o (Omega + u)   (Alg. 1)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) GATHER_WAVES void k_exp_fwd(const ExpFwdItem* __restrict__ items,
                                                   int n_items, int n_tiles) {
  const int tile = xcd_remap(blockIdx.x, n_tiles);
  const ExpFwdItem it = items[find_item(items, n_items, tile)];
  const int D = it.D, H = it.H, W = it.W, V = D * H * W;
  const PTile tc = point_tile(tile - it.tile0, H, W);
  const float a = it.a;
  const cgfloat* __restrict__ s = gp(it.src);
  gfloat* __restrict__ d = gp(it.dst);
  __shared__ float box[3 * GATHER_CELLS];
  __shared__ int sred[8 * (BLOCK / 64)];
  VoxSet vs;
  vox_set(tc, D, H, W, vs);
  float uu[VPT][3];
  CellSet cs;
  load_cells(s, a, D, H, W, vs, uu, cs);
  float sm[VPT][3];
  sample_cells_lds(s, V, H, W, vs, cs, box, sred, sm);
#pragma unroll
  for (int j = 0; j < VPT; ++j) {
    if (!vs.ok[j]) continue;
    sto(d, vs.p[j], uu[j][0] + a * sm[j][0]);
    sto(d + V, vs.p[j], uu[j][1] + a * sm[j][1]);
    sto(d + 2 * V, vs.p[j], uu[j][2] + a * sm[j][2]);
  }
}

// ---------------------------------------------------------------------------
// Composition forward: out = prev + C o (Omega + prev)   (Eq. cum_deformation)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) GATHER_WAVES void k_compose_fwd(const ComposeItem* __restrict__ items,
                                                       int n_items, int n_tiles) {
  const int tile = xcd_remap(blockIdx.x, n_tiles);
  const ComposeItem it = items[find_item(items, n_items, tile)];
  const int D = it.D, H = it.H, W = it.W, V = D * H * W;
  const PTile tc = point_tile(tile - it.tile0, H, W);
  const cgfloat* __restrict__ pr = gp(it.prev);
  const cgfloat* __restrict__ C = gp(it.C);
  gfloat* __restrict__ o = gp(it.out);
  __shared__ float box[3 * GATHER_CELLS];
  __shared__ int sred[8 * (BLOCK / 64)];
  VoxSet vs;
  vox_set(tc, D, H, W, vs);
  float uu[VPT][3];
  CellSet cs;
  load_cells(pr, 1.f, D, H, W, vs, uu, cs);
  float sm[VPT][3];
  sample_cells_lds(C, V, H, W, vs, cs, box, sred, sm);
#pragma unroll
  for (int j = 0; j < VPT; ++j) {
    if (!vs.ok[j]) continue;
    sto(o, vs.p[j], uu[j][0] + sm[j][0]);
    sto(o + V, vs.p[j], uu[j][1] + sm[j][1]);
    sto(o + 2 * V, vs.p[j], uu[j][2] + sm[j][2]);
  }
}

// Staged output of a scatter: this tile's slot ([3][STAGE_CAP]) and
// descriptor in the staging buffers, the overflow flag, and the tile origin.
struct StageOut {
  gfloat* slot;
  int* desc;
  int* flag;
  int z0, y0, x0;
};

// Deterministic accumulation: a block that would add into the float field
// with global atomics adds round(value * scale) into out64 instead (64-bit
// integer atomics, whose sum does not depend on their order).
struct DetOut {
  long long* out64 = nullptr;
  double scale = 0.0;
};

__device__ __forceinline__ void det_add(long long* p, float v, double scale) {
  const long long q = __double2ll_rn((double)v * scale);
  if (q != 0) atomicAdd(reinterpret_cast<unsigned long long*>(p), (unsigned long long)q);
}

// Scale of a job's deterministic slot over `blocks` blocks: 2^(61 - e) with
// 2^e >= blocks * m (m the slot's largest summed block magnitude), so that
// no cell of the 64-bit field can exceed 2^61; 0 when nothing finite was
// recorded.
__device__ __forceinline__ double det_scale(const JobState* js, int slot, int blocks) {
  const float m = __int_as_float((int)js->det_max[slot]);
  if (!(m > 0.f) || !(m < 3.0e38f)) return 0.0;
  int e;
  frexp((double)m * (double)blocks, &e);
  return ldexp(1.0, 61 - e);
}

// Bounding box, largest magnitude and summed magnitudes of a block's
// scatter (every thread must call it).
template <bool OWN, int NT>
__device__ __forceinline__ ScatterBox scatter_bound(const ScatterVox (&sv)[PT_VOX / NT], int* sred) {
  constexpr int VP = PT_VOX / NT;
  int lo[3] = {INT_MAX, INT_MAX, INT_MAX};
  int hi[3] = {INT_MIN, INT_MIN, INT_MIN};
  float mx = 0.f, sm = 0.f;
#pragma unroll
  for (int j = 0; j < VP; ++j) {
    if (sv[j].cz < 0) continue;
    lo[0] = min(lo[0], sv[j].cz); hi[0] = max(hi[0], sv[j].cz + 1);
    lo[1] = min(lo[1], sv[j].cy); hi[1] = max(hi[1], sv[j].cy + 1);
    lo[2] = min(lo[2], sv[j].cx); hi[2] = max(hi[2], sv[j].cx + 1);
    const float gm = fmaxf(fabsf(sv[j].g[0]), fmaxf(fabsf(sv[j].g[1]), fabsf(sv[j].g[2])));
    mx = fmaxf(mx, gm);
    sm += gm;
    if (OWN) {
      lo[0] = min(lo[0], sv[j].oz); hi[0] = max(hi[0], sv[j].oz);
      lo[1] = min(lo[1], sv[j].oy); hi[1] = max(hi[1], sv[j].oy);
      lo[2] = min(lo[2], sv[j].ox); hi[2] = max(hi[2], sv[j].ox);
      const float om = fmaxf(fabsf(sv[j].own[0]), fmaxf(fabsf(sv[j].own[1]), fabsf(sv[j].own[2])));
      mx = fmaxf(mx, om);
      sm += om;
    }
  }
  return scatter_box<NT>(lo, hi, mx, sm, sred);
}

// Largest magnitude and summed magnitudes of a block's scatter whose
// bounding box is already known; the same per-thread order and reductions as
// scatter_bound, so the scale is the same (every thread must call it).
template <bool OWN, int NT>
__device__ __forceinline__ ScatterBox scatter_mag(const ScatterVox (&sv)[PT_VOX / NT], int* sred,
                                                  const BBox& bb) {
  constexpr int VP = PT_VOX / NT;
  float mx = 0.f, sm = 0.f;
#pragma unroll
  for (int j = 0; j < VP; ++j) {
    if (sv[j].cz < 0) continue;
    const float gm = fmaxf(fabsf(sv[j].g[0]), fmaxf(fabsf(sv[j].g[1]), fabsf(sv[j].g[2])));
    mx = fmaxf(mx, gm);
    sm += gm;
    if (OWN) {
      const float om = fmaxf(fabsf(sv[j].own[0]), fmaxf(fabsf(sv[j].own[1]), fabsf(sv[j].own[2])));
      mx = fmaxf(mx, om);
      sm += om;
    }
  }
  const int mxb = dpp_max(__float_as_int(mx));
  const float smw = dpp_sum(sm);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sred[w * 8 + 6] = mxb;
    sred[w * 8 + 7] = __float_as_int(smw);
  }
  __syncthreads();
  int mb = 0;
  float sb_sum = 0.f;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) {
    mb = max(mb, sred[i * 8 + 6]);
    sb_sum += __int_as_float(sred[i * 8 + 7]);
  }
  ScatterBox sb;
  sb.bb = bb;
  sb.bmax = __int_as_float(mb);
  sb.bsum = sb_sum;
  return sb;
}

// Whether a block's box goes to its staging slot: it fits the slot and
// reaches no farther than the 26 neighbouring tiles (where the reading step
// looks for it).
__device__ __forceinline__ bool stage_fits(const ScatterBox& sb, const StageOut& so) {
  const BBox& bb = sb.bb;
  const bool finite = sb.bmax > 0.f && sb.bmax < 3.0e38f && sb.bsum < 3.0e38f;
  return bb.cells > 0 && bb.cells <= STAGE_CAP && finite &&
         bb.lz >= so.z0 - PT_Z && bb.lz + bb.ez <= so.z0 + 2 * PT_Z &&
         bb.ly >= so.y0 - PT_Y && bb.ly + bb.ey <= so.y0 + 2 * PT_Y &&
         bb.lx >= so.x0 - PT_X && bb.lx + bb.ex <= so.x0 + 2 * PT_X;
}

// Deterministic mode, reduce-only pass: a block that will add into the flat
// field (every block unless it stages its box) raises the job's slot to its
// summed magnitude.
template <bool OWN, bool STAGE, int NT>
__device__ __forceinline__ void det_bound(const ScatterVox (&sv)[PT_VOX / NT], int* sred,
                                          const StageOut& so, JobState* js, int slot) {
  const ScatterBox sb = scatter_bound<OWN, NT>(sv, sred);
  if (sb.bb.cells == 0 || !(sb.bmax > 0.f)) return;
  if (STAGE && stage_fits(sb, so)) return;
  if (threadIdx.x == 0) atomicMax(&js->det_max[slot], (unsigned int)__float_as_int(sb.bsum));
}

template <bool OWN, bool STAGE = false, int NT = BLOCK>
__device__ __forceinline__ void scatter_tile(const ScatterVox (&sv)[PT_VOX / NT], gfloat* __restrict__ out,
                                             int D, int H, int W, int* acc, int* sred,
                                             const StageOut& so = StageOut{},
                                             const DetOut& det = DetOut{},
                                             const BBox* known = nullptr) {
  constexpr int VP = PT_VOX / NT;
  const int HW = H * W, V = D * HW;
  const ScatterBox sb =
      known ? scatter_mag<OWN, NT>(sv, sred, *known) : scatter_bound<OWN, NT>(sv, sred);
  const BBox& bb = sb.bb;
  const float bmax = sb.bmax;
  // the bins take finite values only; bsum bounds every bin's magnitude
  const bool finite = bmax > 0.f && bmax < 3.0e38f && sb.bsum < 3.0e38f;
  bool staged = false;
  if (STAGE) {
    staged = stage_fits(sb, so);
    if (threadIdx.x == 0) {
      so.desc[0] = bb.lz; so.desc[1] = bb.ly; so.desc[2] = bb.lx;
      so.desc[3] = staged ? bb.ez : 0;
      so.desc[4] = bb.ey; so.desc[5] = bb.ex;
      // anything the flat path adds must be picked up by the reading step
      if (!staged && bb.cells > 0 && !(bmax == 0.f)) *so.flag = 1;
    }
  }
  if (bb.cells == 0) return;
  if (bb.cells <= SCATTER_CELLS && finite) {
    const float scale = fminf(FIX_SCALE / bmax, FIX_TOTAL / sb.bsum);
    const float inv = 1.f / scale;
    const int cells = bb.cells;
    // one plane of SCATTER_CELLS bins per component: the plane offsets are
    // constants, which the LDS instructions take as immediate offsets
    {
      int4* a4 = reinterpret_cast<int4*>(acc);
      const int n4 = (cells + 3) >> 2;
#pragma unroll
      for (int c = 0; c < 3; ++c)
        for (int i = threadIdx.x; i < n4; i += NT) a4[c * (SCATTER_CELLS / 4) + i] = make_int4(0, 0, 0, 0);
    }
    __syncthreads();
    const int sy = bb.ex, sz = bb.ex * bb.ey;
#pragma unroll
    for (int j = 0; j < VP; ++j) {
      if (sv[j].cz < 0) continue;
      const int l = ((sv[j].cz - bb.lz) * bb.ey + (sv[j].cy - bb.ly)) * bb.ex + (sv[j].cx - bb.lx);
      const float tz = sv[j].tz, ty = sv[j].ty, tx = sv[j].tx;
      const float w0z = 1.f - tz, w0y = 1.f - ty, w0x = 1.f - tx;
      const float w[8] = {w0z * w0y * w0x, w0z * w0y * tx, w0z * ty * w0x, w0z * ty * tx,
                          tz * w0y * w0x,  tz * w0y * tx,  tz * ty * w0x,  tz * ty * tx};
      const int off[8] = {0, 1, sy, sy + 1, sz, sz + 1, sz + sy, sz + sy + 1};
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float g = sv[j].g[c] * scale;
        int* a = acc + c * SCATTER_CELLS + l;
#pragma unroll
        for (int q = 0; q < 8; ++q) atomicAdd(a + off[q], (int)(w[q] * g));
      }
      if (OWN) {
        const int lo2 = ((sv[j].oz - bb.lz) * bb.ey + (sv[j].oy - bb.ly)) * bb.ex + (sv[j].ox - bb.lx);
#pragma unroll
        for (int c = 0; c < 3; ++c) atomicAdd(acc + c * SCATTER_CELLS + lo2, (int)(sv[j].own[c] * scale));
      }
    }
    __syncthreads();
    if (STAGE && staged) {
      // plain stores of the whole box (zeros included): the slot is this
      // tile's alone.  The descriptor also records the largest cell
      // magnitude, from which the reading step sizes its fixed point.
      int amax = 0;
      for (int i = threadIdx.x; i < cells; i += NT) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const int v = acc[c * SCATTER_CELLS + i];
          amax = max(amax, abs(v));
          sto(so.slot, c * STAGE_CAP + i, (float)v * inv);
        }
      }
      amax = dpp_max(amax);
      if ((threadIdx.x & 63) == 0) sred[threadIdx.x >> 6] = amax;
      __syncthreads();
      if (threadIdx.x == 0) {
        int m = 0;
        for (int w = 0; w < NT / 64; ++w) m = max(m, sred[w]);
        so.desc[6] = __float_as_int((float)m * inv);
      }
      return;
    }
    // i -> (lz, ly, lx) by float reciprocals: exact here since i < 2^22
    const float inv_ex = 1.f / (float)bb.ex, inv_ey = 1.f / (float)bb.ey;
    for (int i = threadIdx.x; i < cells; i += NT) {
      const int r = (int)(((float)i + 0.5f) * inv_ex);
      const int lx = i - r * bb.ex;
      const int lz = (int)(((float)r + 0.5f) * inv_ey);
      const int ly = r - lz * bb.ey;
      const int gpos = ((bb.lz + lz) * H + (bb.ly + ly)) * W + (bb.lx + lx);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int v = acc[c * SCATTER_CELLS + i];
        if (v == 0) continue;
        if (det.out64)
          det_add(det.out64 + c * V + gpos, (float)v * inv, det.scale);
        else
          gadd(out + c * V + gpos, (float)v * inv);
      }
    }
  } else {
    // The footprint does not fit the bins (or the values are not finite):
    // global float atomics.
#pragma unroll
    for (int j = 0; j < VP; ++j) {
      if (sv[j].cz < 0) continue;
      const int base = (sv[j].cz * H + sv[j].cy) * W + sv[j].cx;
      const float tz = sv[j].tz, ty = sv[j].ty, tx = sv[j].tx;
      const float w0z = 1.f - tz, w0y = 1.f - ty, w0x = 1.f - tx;
      const float w[8] = {w0z * w0y * w0x, w0z * w0y * tx, w0z * ty * w0x, w0z * ty * tx,
                          tz * w0y * w0x,  tz * w0y * tx,  tz * ty * w0x,  tz * ty * tx};
      const int off[8] = {0, 1, W, W + 1, HW, HW + 1, HW + W, HW + W + 1};
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float g = sv[j].g[c];
        if (g == 0.f) continue;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          if (det.out64)
            det_add(det.out64 + c * V + base + off[q], w[q] * g, det.scale);
          else
            gadd(out + c * V + base + off[q], w[q] * g);
        }
      }
      if (OWN) {
        const int po = (sv[j].oz * H + sv[j].oy) * W + sv[j].ox;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          if (det.out64)
            det_add(det.out64 + c * V + po, sv[j].own[c], det.scale);
          else
            gadd(out + c * V + po, sv[j].own[c]);
        }
      }
    }
  }
}

// G over a point tile from the staged boxes of a scatter step.  The tile's
// own box (which holds every owned voxel) is read straight into registers.
// The parts of the 26 neighbours' boxes that reach into the tile form one
// list of cells, which the block reads with all its loads in flight and adds
// into LDS bins (neighbouring boxes overlap) in 32-bit fixed point, scaled so
// that the sum of the boxes' largest cell magnitudes maps to 2^30: no bin can
// overflow.  Then the flat overflow gin, if any block of that step used it
// (*flag_in); gin is cleared where read.
//
// Three parts, so that a kernel can put its own loads between them: the
// descriptor loads (pull_desc), the neighbour list (pull_setup, which ends
// with a barrier) and the reads and sums (pull_finish).  pull_staged runs
// the three in a row.

// Per neighbour d: nyx, nx, the box's z and y strides, the tile-local index
// of the overlap's first cell, 1 / nyx and 1 / nx (float bits), [7] = cells,
// and [8..9] the address of that cell's first component.  pre[d]: first list
// position of d; pre[27] = total, and the padding above it never compares
// below a position.
struct PullList {
  int nbd[27][12];
  int pre[32];
  float nbmax;
};

// The descriptors a thread needs: the tile's own box (every thread) and, in
// lane d < 27 of the first wave, neighbour d's box (n[3] = 0: none).
struct PullDesc {
  int own[6];
  int n[7];
  int nb;
};

__device__ __forceinline__ PullDesc pull_desc(const int* desc_in, int local, const PTile& tc, int D,
                                              int H, int W) {
  PullDesc pd;
  {
    const int* dsc = desc_in + local * 8;
#pragma unroll
    for (int k = 0; k < 6; ++k) pd.own[k] = dsc[k];
  }
#pragma unroll
  for (int k = 0; k < 7; ++k) pd.n[k] = 0;
  pd.nb = 0;
  if (threadIdx.x < 32) {
    const int ntz = (D + PT_Z - 1) / PT_Z, nty = (H + PT_Y - 1) / PT_Y, ntx = (W + PT_X - 1) / PT_X;
    const int tz = tc.z0 / PT_Z, ty = tc.y0 / PT_Y, tx = tc.x0 / PT_X;
    const int d = threadIdx.x;
    const int nz = tz + d / 9 - 1, ny = ty + (d / 3) % 3 - 1, nx = tx + d % 3 - 1;
    if (d < 27 && d != 13 && nz >= 0 && nz < ntz && ny >= 0 && ny < nty && nx >= 0 && nx < ntx) {
      pd.nb = (nz * nty + ny) * ntx + nx;
      const int* dsc = desc_in + pd.nb * 8;
#pragma unroll
      for (int k = 0; k < 7; ++k) pd.n[k] = dsc[k];
    }
  }
  return pd;
}

// The neighbour list and the cleared bins; acc: LDS of at least 3 * PT_VOX
// ints.  Every thread of the block must call this.
__device__ __forceinline__ void pull_setup(const PullDesc& pd, const float* stage_in,
                                           const PTile& tc, int D, int H, int W, int* acc,
                                           PullList& pl) {
  if (threadIdx.x < 32) {
    // one lane per neighbour (lanes 27..31 and absent neighbours count 0)
    const int d = threadIdx.x;
    int n = 0;
    float bm = 0.f;
    int* e = pl.nbd[d < 27 ? d : 26];
    const int bz = pd.n[0], by = pd.n[1], bx = pd.n[2], ez = pd.n[3], ey = pd.n[4], ex = pd.n[5];
    // intersection with this tile, in global coordinates
    const int z0 = max(bz, tc.z0), z1 = min(bz + ez, min(tc.z0 + PT_Z, D));
    const int y0 = max(by, tc.y0), y1 = min(by + ey, min(tc.y0 + PT_Y, H));
    const int x0 = max(bx, tc.x0), x1 = min(bx + ex, min(tc.x0 + PT_X, W));
    if (ez > 0 && z1 > z0 && y1 > y0 && x1 > x0) {
      const int nyx = (y1 - y0) * (x1 - x0);
      n = (z1 - z0) * nyx;
      bm = __int_as_float(pd.n[6]);
      const cgfloat* first = gp(stage_in) + (size_t)pd.nb * 3 * STAGE_CAP +
                             (((z0 - bz) * ey + (y0 - by)) * ex + (x0 - bx));
      e[0] = nyx;
      e[1] = x1 - x0;
      e[2] = ey * ex;
      e[3] = ex;
      e[4] = ((z0 - tc.z0) * PT_Y + (y0 - tc.y0)) * PT_X + (x0 - tc.x0);
      e[5] = __float_as_int(1.f / (float)nyx);
      e[6] = __float_as_int(1.f / (float)(x1 - x0));
      *reinterpret_cast<const cgfloat**>(e + 8) = first;
    }
    if (d < 27) e[7] = n;
    // exclusive prefix of the counts and sum of the largest magnitudes over
    // the 32 lanes by shuffles (the same order in every block)
    int incl = n;
    float msum = bm;
#pragma unroll
    for (int o = 1; o < 32; o <<= 1) {
      const int t = __shfl_up(incl, o, 32);
      if (d >= o) incl += t;
      msum += __shfl_xor(msum, o, 32);
    }
    if (d < 27) pl.pre[d] = incl - n;
    if (d == 26) pl.pre[27] = incl;
    if (d >= 28) pl.pre[d] = INT_MAX;
    if (d == 0) pl.nbmax = msum;
  }
  {
    int4* g4 = reinterpret_cast<int4*>(acc);
    for (int i = threadIdx.x; i < 3 * PT_VOX / 4; i += BLOCK) g4[i] = make_int4(0, 0, 0, 0);
  }
  __syncthreads();
}

// G at the owned voxels: the own box, the neighbour list summed in the
// bins, and the flat overflow.  gv must hold zeros on entry.  Every thread
// of the block must call this.
__device__ __forceinline__ void pull_finish(const PullDesc& pd, const float* stage_in,
                                            const int* flag_in, gfloat* __restrict__ gin, int local,
                                            int D, int H, int W, const int (&vz)[VPT],
                                            const int (&vy)[VPT], const int (&vx)[VPT],
                                            const bool (&vok)[VPT], float (&gv)[VPT][3], int* acc,
                                            const PullList& pl, bool clear) {
  const int V = D * H * W;
  int* gacc = acc;  // [3][PT_VOX]
  const int* pre = pl.pre;
  // own box, straight into registers
  {
    const int bz = pd.own[0], by = pd.own[1], bx = pd.own[2], ez = pd.own[3], ey = pd.own[4],
              ex = pd.own[5];
    if (ez > 0) {
      const cgfloat* __restrict__ sl = gp(stage_in) + (size_t)local * 3 * STAGE_CAP;
#pragma unroll
      for (int j = 0; j < VPT; ++j) {
        if (!vok[j]) continue;
        const int idx = ((vz[j] - bz) * ey + (vy[j] - by)) * ex + (vx[j] - bx);
        gv[j][0] = ldo(sl, idx);
        gv[j][1] = ldo(sl + STAGE_CAP, idx);
        gv[j][2] = ldo(sl + 2 * STAGE_CAP, idx);
      }
    }
  }
  const int total = pre[27];
  const float nbmax = pl.nbmax;
  const float qscale = nbmax > 0.f ? 1073741824.0f / nbmax : 0.f;  // 2^30 / sum of maxima
  const float qinv = nbmax / 1073741824.0f;
  constexpr int U = 4;
  for (int w0 = threadIdx.x; w0 < total; w0 += BLOCK * U) {
    // positions past the end repeat the last cell (a valid load) and add
    // nothing; with no branch per position the U searches run side by side
    int w[U], d[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      w[u] = min(w0 + u * BLOCK, total - 1);
      d[u] = 0;
    }
    // the last d with pre[d] <= w: the non-empty entry holding w (the search
    // stays below 32, and pre above 27 is never <= w)
#pragma unroll
    for (int step = 16; step > 0; step >>= 1)
#pragma unroll
      for (int u = 0; u < U; ++u) d[u] = pre[d[u] + step] <= w[u] ? d[u] + step : d[u];
    float v0[U], v1[U], v2[U];
    int loc[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int* e = pl.nbd[d[u]];
      const int r = w[u] - pre[d[u]];
      // (iz, iy, ix) of cell r of the overlap; the float quotients are
      // exact here (r < 1024, the overlap lies in one tile)
      const int nyx = e[0], nx = e[1];
      const int iz = (int)(((float)r + 0.5f) * __int_as_float(e[5]));
      const int rr = r - iz * nyx;
      const int iy = (int)(((float)rr + 0.5f) * __int_as_float(e[6]));
      const int ix = rr - iy * nx;
      const cgfloat* __restrict__ sl =
          *reinterpret_cast<const cgfloat* const*>(e + 8) + (uint32_t)(iz * e[2] + iy * e[3] + ix);
      v0[u] = sl[0];
      v1[u] = sl[STAGE_CAP];
      v2[u] = sl[2 * STAGE_CAP];
      loc[u] = w0 + u * BLOCK < total ? e[4] + (iz * PT_Y + iy) * PT_X + ix : -1;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (loc[u] < 0) continue;
      atomicAdd(&gacc[loc[u]], (int)(v0[u] * qscale));
      atomicAdd(&gacc[PT_VOX + loc[u]], (int)(v1[u] * qscale));
      atomicAdd(&gacc[2 * PT_VOX + loc[u]], (int)(v2[u] * qscale));
    }
  }
  __syncthreads();
  const bool flat = *flag_in != 0;
#pragma unroll
  for (int j = 0; j < VPT; ++j) {
    if (!vok[j]) continue;
    const int k = threadIdx.x + j * BLOCK;
    gv[j][0] += (float)gacc[k] * qinv;
    gv[j][1] += (float)gacc[PT_VOX + k] * qinv;
    gv[j][2] += (float)gacc[2 * PT_VOX + k] * qinv;
    if (flat) {
      const int p = (vz[j] * H + vy[j]) * W + vx[j];
      gv[j][0] += gin[p];
      gv[j][1] += gin[V + p];
      gv[j][2] += gin[2 * V + p];
      if (clear) {
        gin[p] = 0.f;
        gin[V + p] = 0.f;
        gin[2 * V + p] = 0.f;
      }
    }
  }
}

// The three parts in a row; acc: LDS of at least 3 * PT_VOX ints.
__device__ __forceinline__ void pull_staged(const float* stage_in, const int* desc_in,
                                            const int* flag_in, gfloat* __restrict__ gin, int local,
                                            const PTile& tc, int D, int H, int W,
                                            const int (&vz)[VPT], const int (&vy)[VPT],
                                            const int (&vx)[VPT], const bool (&vok)[VPT],
                                            float (&gv)[VPT][3], int* acc, bool clear = true) {
  __shared__ PullList pl;
  const PullDesc pd = pull_desc(desc_in, local, tc, D, H, W);
  pull_setup(pd, stage_in, tc, D, H, W, acc, pl);
  pull_finish(pd, stage_in, flag_in, gin, local, D, H, W, vz, vy, vx, vok, gv, acc, pl, clear);
}

// ---------------------------------------------------------------------------
// Exp backward: one squaring, dL/du_s from dL/du_{s+1}
//   G_s(p) = G(p) + J_u(q)^T G(p) + sum_{p': corners of q(p') contain p} w G(p')
// ---------------------------------------------------------------------------
// MODE: 0 flat G_{s+1} in, flat G_s out; 1 flat in, staged out; 2 staged
// in, staged out; 3 staged in, flat out (see ExpBwdItem).  A staged G_0 is
// turned into a flat field by k_unstage.  DETMAX: the deterministic mode's
// reduce-only pass (no writes but the job's slot).
template <int MODE, bool REG, bool DETMAX = false>
__global__ __launch_bounds__(BLOCK) void k_exp_bwd(const ExpBwdItem* __restrict__ items,
                                                   int n_items, int n_tiles) {
  constexpr bool IN_ST = MODE >= 2, OUT_ST = MODE == 1 || MODE == 2;
  __shared__ __align__(16) int acc[3 * SCATTER_CELLS];
  __shared__ int sred[16 * (BLOCK / 64)];
  __shared__ double red[BLOCK / 64];
  const int tile = xcd_remap(blockIdx.x, n_tiles);
  const ExpBwdItem it = items[find_item(items, n_items, tile)];
  const int D = it.D, H = it.H, W = it.W, HW = H * W, V = D * HW;
  const int local = tile - it.tile0;
  const PTile tc = point_tile(local, H, W);
  const float a = it.a;
  const cgfloat* __restrict__ s = gp(it.src);
  gfloat* __restrict__ gin = gp(it.gin);
  const bool reg = REG && (it.reg_w != 0.f || it.ext);
  const float inv_mz = 1.f / (float)((D - 1) * H * W), inv_my = 1.f / (float)(D * (H - 1) * W),
              inv_mx = 1.f / (float)(D * H * (W - 1));
  double rval = 0.0, rext = 0.0;
  // G_{s+1} at the owned voxels
  float gv[VPT][3];
  int vz[VPT], vy[VPT], vx[VPT];
  bool vok[VPT];
#pragma unroll
  for (int j = 0; j < VPT; ++j) {
    const int k = threadIdx.x + j * BLOCK;
    vx[j] = tc.x0 + (k % PT_X);
    vy[j] = tc.y0 + (k / PT_X) % PT_Y;
    vz[j] = tc.z0 + k / (PT_X * PT_Y);
    vok[j] = vx[j] < W && vy[j] < H && vz[j] < D;
    gv[j][0] = gv[j][1] = gv[j][2] = 0.f;
  }
  // G_{s+1} over this tile from the staged boxes of the previous step: the
  // box descriptors are read first and u_s at the owned voxels next, so that
  // those loads are in flight while the neighbour list is formed
  __shared__ PullList pl;
  PullDesc pd;
  if (IN_ST) pd = pull_desc(it.desc_in, local, tc, D, H, W);
  float uo[VPT][3];
#pragma unroll
  for (int j = 0; j < VPT; ++j) {
    const int p = vok[j] ? (vz[j] * H + vy[j]) * W + vx[j] : 0;
    uo[j][0] = a * ldo(s, p);
    uo[j][1] = a * ldo(s + V, p);
    uo[j][2] = a * ldo(s + 2 * V, p);
  }
  if (IN_ST) {
    pull_setup(pd, it.stage_in, tc, D, H, W, acc, pl);
    pull_finish(pd, it.stage_in, it.flag_in, gin, local, D, H, W, vz, vy, vx, vok, gv, acc, pl,
                !DETMAX);
  } else {
#pragma unroll
    for (int j = 0; j < VPT; ++j) {
      if (!vok[j]) continue;
      const int p = (vz[j] * H + vy[j]) * W + vx[j];
      gv[j][0] = gin[p];
      gv[j][1] = gin[V + p];
      gv[j][2] = gin[2 * V + p];
      if (it.zero_in && !DETMAX) {
        gin[p] = 0.f;
        gin[V + p] = 0.f;
        gin[2 * V + p] = 0.f;
      }
    }
  }
  // the regulariser's stencil reads a halo tile of src staged in acc, which
  // the scatter below reuses once every thread has formed its own terms
  float* rt = reinterpret_cast<float*>(acc);
  float rvf = 0.f;
  if ((REG && it.reg_w != 0.f)) {
    __syncthreads();  // the staged pull above is done with acc
    reg_tile_load(s, V, tc.z0, tc.y0, tc.x0, D, H, W, rt);
    __syncthreads();
  }
  // the cells the owned voxels sample
  Ax cz[VPT], cy[VPT], cx[VPT];
#pragma unroll
  for (int j = 0; j < VPT; ++j) {
    cz[j] = axis_disp(vz[j], uo[j][0], D);
    cy[j] = axis_disp(vy[j], uo[j][1], H);
    cx[j] = axis_disp(vx[j], uo[j][2], W);
  }
  // Without the regulariser's tile (which holds acc until the scatter), the
  // corners come from a box of src staged in acc: the bounding box of the
  // cells and the owned voxels, which is also the scatter's box.  The values
  // and the arithmetic are those of the direct loads, so the result is the
  // same; a box larger than ADJ_BOX_CELLS reads the corners directly.
  BBox gb{};
  bool lds_box = false;
  if (!REG) {
    int lo[3] = {INT_MAX, INT_MAX, INT_MAX};
    int hi[3] = {INT_MIN, INT_MIN, INT_MIN};
#pragma unroll
    for (int j = 0; j < VPT; ++j) {
      if (!vok[j]) continue;
      lo[0] = min(lo[0], min(cz[j].i0, vz[j])); hi[0] = max(hi[0], max(cz[j].i0 + 1, vz[j]));
      lo[1] = min(lo[1], min(cy[j].i0, vy[j])); hi[1] = max(hi[1], max(cy[j].i0 + 1, vy[j]));
      lo[2] = min(lo[2], min(cx[j].i0, vx[j])); hi[2] = max(hi[2], max(cx[j].i0 + 1, vx[j]));
    }
    // the second half of sred: the scatter's own reduction uses the first
    gb = scatter_box<BLOCK>(lo, hi, 0.f, 0.f, sred + 8 * (BLOCK / 64)).bb;
    lds_box = gb.cells > 0 && gb.cells <= ADJ_BOX_CELLS;  // block-uniform
    if (lds_box) {
      float* box = reinterpret_cast<float*>(acc);
      const int cells = gb.cells;
      // cell i -> (lz, ly, lx) by float reciprocals: exact here since i < 2^22
      const float inv_ex = 1.f / (float)gb.ex, inv_ey = 1.f / (float)gb.ey;
      for (int i = threadIdx.x; i < cells; i += BLOCK) {
        const int r = (int)(((float)i + 0.5f) * inv_ex);
        const int lx = i - r * gb.ex;
        const int lz = (int)(((float)r + 0.5f) * inv_ey);
        const int ly = r - lz * gb.ey;
        const int g = ((gb.lz + lz) * H + (gb.ly + ly)) * W + (gb.lx + lx);
        const int w0 = i & ~63;  // the wave's first cell: i = threadIdx.x + k * block
        ld_to_lds(s + g, box + w0);
        ld_to_lds(s + V + g, box + cells + w0);
        ld_to_lds(s + 2 * V + g, box + 2 * cells + w0);
      }
      __syncthreads();
    }
  }
  ScatterVox sv[VPT];
#pragma unroll
  for (int j = 0; j < VPT; ++j) {
    sv[j].cz = -1;
    if (!vok[j]) continue;
    const int x = vx[j], y = vy[j], z = vz[j];
    const int p = (z * H + y) * W + x;
    const Ax az = cz[j], ay = cy[j], ax = cx[j];
    const float g0 = gv[j][0], g1 = gv[j][1], g2 = gv[j][2];
    // (J^T g) of the Jacobian J of src at q is the gradient of the
    // interpolant of sum_c g_c src_c: combine the corners first, then one
    // gradient; the factor a and the clamped axes apply per column
    float v0[8], v1[8], v2[8], jz, jy, jx;
    if (lds_box) {
      const float* box = reinterpret_cast<const float*>(acc);
      const int cells = gb.cells, sy = gb.ex, sz = gb.ex * gb.ey;
      const int l = ((az.i0 - gb.lz) * gb.ey + (ay.i0 - gb.ly)) * gb.ex + (ax.i0 - gb.lx);
      const int off[8] = {0, 1, sy, sy + 1, sz, sz + 1, sz + sy, sz + sy + 1};
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        v0[k] = box[l + off[k]];
        v1[k] = box[cells + l + off[k]];
        v2[k] = box[2 * cells + l + off[k]];
      }
    } else {
      const int base = (az.i0 * H + ay.i0) * W + ax.i0;
      load8(s, base, W, HW, v0);
      load8(s + V, base, W, HW, v1);
      load8(s + 2 * V, base, W, HW, v2);
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) v0[k] = fmaf(g2, v2[k], fmaf(g1, v1[k], g0 * v0[k]));
    tri_grad(v0, az.t, ay.t, ax.t, jz, jy, jx);
    float own0 = fmaf(a * az.live, jz, g0);
    float own1 = fmaf(a * ay.live, jy, g1);
    float own2 = fmaf(a * ax.live, jx, g2);
    if ((REG && it.reg_w != 0.f)) {
      const int lz = z - tc.z0, ly = y - tc.y0, lx = x - tc.x0;
      own0 = fmaf(it.reg_w, reg_tile_point(rt, lz, ly, lx, z, y, x, D, H, W, inv_mz, inv_my,
                                           inv_mx, &rvf), own0);
      own1 = fmaf(it.reg_w, reg_tile_point(rt + RH_N, lz, ly, lx, z, y, x, D, H, W, inv_mz,
                                           inv_my, inv_mx, &rvf), own1);
      own2 = fmaf(it.reg_w, reg_tile_point(rt + 2 * RH_N, lz, ly, lx, z, y, x, D, H, W, inv_mz,
                                           inv_my, inv_mx, &rvf), own2);
    }
    if (REG && it.ext) {
      // L_L2 and L_ts (Sec. 2.4): linear in the flows of this interval and its neighbours
      const float f0 = s[p], f1 = s[V + p], f2 = s[2 * V + p];
      own0 = fmaf(it.w_self, f0, own0);
      own1 = fmaf(it.w_self, f1, own1);
      own2 = fmaf(it.w_self, f2, own2);
      double e = (double)it.l2_loss_w * ((double)f0 * f0 + (double)f1 * f1 + (double)f2 * f2);
      if (it.flow_prev) {
        const cgfloat* __restrict__ fp = gp(it.flow_prev);
        const float p0 = fp[p], p1 = fp[V + p], p2 = fp[2 * V + p];
        own0 = fmaf(it.w_prev, p0, own0);
        own1 = fmaf(it.w_prev, p1, own1);
        own2 = fmaf(it.w_prev, p2, own2);
        const double a0 = (double)p0 * it.inv_dprev - (double)f0 * it.inv_dself;
        const double a1 = (double)p1 * it.inv_dprev - (double)f1 * it.inv_dself;
        const double a2 = (double)p2 * it.inv_dprev - (double)f2 * it.inv_dself;
        e += (double)it.ts_loss_w * (a0 * a0 + a1 * a1 + a2 * a2);
      }
      if (it.flow_next) {
        const cgfloat* __restrict__ fn = gp(it.flow_next);
        own0 = fmaf(it.w_next, fn[p], own0);
        own1 = fmaf(it.w_next, fn[V + p], own1);
        own2 = fmaf(it.w_next, fn[2 * V + p], own2);
      }
      rext += e;
    }
    sv[j].cz = az.i0; sv[j].cy = ay.i0; sv[j].cx = ax.i0;
    sv[j].oz = z; sv[j].oy = y; sv[j].ox = x;
    sv[j].tz = az.t; sv[j].ty = ay.t; sv[j].tx = ax.t;
    sv[j].g[0] = g0; sv[j].g[1] = g1; sv[j].g[2] = g2;
    sv[j].own[0] = own0; sv[j].own[1] = own1; sv[j].own[2] = own2;
  }
  StageOut so{};
  if (OUT_ST) {
    so.slot = gp(it.stage_out) + (size_t)local * 3 * STAGE_CAP;
    so.desc = it.desc_out + local * 8;
    so.flag = it.flag_out;
    so.z0 = tc.z0; so.y0 = tc.y0; so.x0 = tc.x0;
  }
  if (DETMAX) {
    det_bound<true, OUT_ST, BLOCK>(sv, sred, so, it.js, it.det_slot);
    return;
  }
  DetOut det;
  if (it.gout64) {
    det.out64 = it.gout64;
    det.scale = det_scale(it.js, it.det_slot, it.det_blocks);
  }
  // with the box known, the scatter reduces only the magnitudes; the gathers
  // from acc end before its barrier, after which the bins are cleared
  const BBox* known = REG ? nullptr : &gb;
  if (OUT_ST)
    scatter_tile<true, true>(sv, gp(it.gout), D, H, W, acc, sred, so, det, known);
  else
    scatter_tile<true>(sv, gp(it.gout), D, H, W, acc, sred, StageOut{}, det, known);
  rval = (double)rvf;
  if (reg) {
    const double tot = block_sum(rval * (double)it.reg_loss_w + rext, red);
    if (threadIdx.x == 0 && it.js) unsafeAtomicAdd(&it.js->loss_reg, tot);
  }
}

// ---------------------------------------------------------------------------
// Staged G_0 of the last backward squaring to the flat field gout: each
// voxel gets the boxes that hold it plus the flat overflow, which is read
// from gout itself before it is overwritten.  Plain stores, no atomics.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void k_unstage(const ExpBwdItem* __restrict__ items,
                                                   int n_items, int n_tiles) {
  __shared__ __align__(16) int acc[3 * PT_VOX];
  const int tile = xcd_remap(blockIdx.x, n_tiles);
  const ExpBwdItem it = items[find_item(items, n_items, tile)];
  const int D = it.D, H = it.H, W = it.W, V = D * H * W;
  const int local = tile - it.tile0;
  const PTile tc = point_tile(local, H, W);
  gfloat* __restrict__ g = gp(it.gout);
  float gv[VPT][3];
  int vz[VPT], vy[VPT], vx[VPT];
  bool vok[VPT];
#pragma unroll
  for (int j = 0; j < VPT; ++j) {
    const int k = threadIdx.x + j * BLOCK;
    vx[j] = tc.x0 + (k % PT_X);
    vy[j] = tc.y0 + (k / PT_X) % PT_Y;
    vz[j] = tc.z0 + k / (PT_X * PT_Y);
    vok[j] = vx[j] < W && vy[j] < H && vz[j] < D;
    gv[j][0] = gv[j][1] = gv[j][2] = 0.f;
  }
  pull_staged(it.stage_in, it.desc_in, it.flag_in, g, local, tc, D, H, W, vz, vy, vx, vok, gv, acc);
#pragma unroll
  for (int j = 0; j < VPT; ++j) {
    if (!vok[j]) continue;
    const int p = (vz[j] * H + vy[j]) * W + vx[j];
    g[p] = gv[j][0];
    g[V + p] = gv[j][1];
    g[2 * V + p] = gv[j][2];
  }
}

// The gradient of each SVF from the staged G_0 of its forward and backward
// directions (PullItem), without a flat G_0 in between.
__global__ __launch_bounds__(BLOCK) void k_pull_combine(const PullItem* __restrict__ items,
                                                        int n_items, int n_tiles) {
  // the pulls' bins, then the regulariser's halo tile of the flow
  constexpr int ACC = 3 * PT_VOX > 3 * RH_N ? 3 * PT_VOX : 3 * RH_N;
  __shared__ __align__(16) int acc[ACC];
  __shared__ double red[BLOCK / 64];
  const int tile = xcd_remap(blockIdx.x, n_tiles);
  const PullItem it = items[find_item(items, n_items, tile)];
  const int D = it.D, H = it.H, W = it.W, V = D * H * W;
  const int local = tile - it.tile0;
  const PTile tc = point_tile(local, H, W);
  float gf[VPT][3], gb[VPT][3];
  int vz[VPT], vy[VPT], vx[VPT];
  bool vok[VPT];
#pragma unroll
  for (int j = 0; j < VPT; ++j) {
    const int k = threadIdx.x + j * BLOCK;
    vx[j] = tc.x0 + (k % PT_X);
    vy[j] = tc.y0 + (k / PT_X) % PT_Y;
    vz[j] = tc.z0 + k / (PT_X * PT_Y);
    vok[j] = vx[j] < W && vy[j] < H && vz[j] < D;
    gf[j][0] = gf[j][1] = gf[j][2] = 0.f;
    gb[j][0] = gb[j][1] = gb[j][2] = 0.f;
  }
  pull_staged(it.stage[0], it.desc[0], it.flag[0], gp(it.gflat[0]), local, tc, D, H, W, vz, vy,
              vx, vok, gf, acc);
  __syncthreads();  // the first pull is done with acc
  pull_staged(it.stage[1], it.desc[1], it.flag[1], gp(it.gflat[1]), local, tc, D, H, W, vz, vy,
              vx, vok, gb, acc);
  gfloat* __restrict__ out = gp(it.out);
  if (it.reg_w != 0.f) {  // block-uniform
    const float inv_mz = 1.f / (float)((D - 1) * H * W), inv_my = 1.f / (float)(D * (H - 1) * W),
                inv_mx = 1.f / (float)(D * H * (W - 1));
    float* rt = reinterpret_cast<float*>(acc);
    __syncthreads();  // the second pull is done with acc
    reg_tile_load(gp(it.flow), V, tc.z0, tc.y0, tc.x0, D, H, W, rt);
    __syncthreads();
    float rvf = 0.f;
#pragma unroll
    for (int j = 0; j < VPT; ++j) {
      if (!vok[j]) continue;
      const int p = (vz[j] * H + vy[j]) * W + vx[j];
      const int lz = vz[j] - tc.z0, ly = vy[j] - tc.y0, lx = vx[j] - tc.x0;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float rg = reg_tile_point(rt + c * RH_N, lz, ly, lx, vz[j], vy[j], vx[j], D, H, W,
                                        inv_mz, inv_my, inv_mx, &rvf);
        out[c * V + p] = fmaf(it.reg_w, rg, it.scale * (gf[j][c] - gb[j][c]));
      }
    }
    const double tot = block_sum((double)rvf * (double)it.reg_loss_w, red);
    if (threadIdx.x == 0 && it.js) unsafeAtomicAdd(&it.js->loss_reg, tot);
    return;
  }
#pragma unroll
  for (int j = 0; j < VPT; ++j) {
    if (!vok[j]) continue;
    const int p = (vz[j] * H + vy[j]) * W + vx[j];
#pragma unroll
    for (int c = 0; c < 3; ++c) out[c * V + p] = it.scale * (gf[j][c] - gb[j][c]);
  }
}

// ---------------------------------------------------------------------------
// Composition backward
// ---------------------------------------------------------------------------
// The composition adjoint runs 512 threads per point tile (two voxels each):
// with its extra streams (G, U_prev, G_prev) it gains more from the higher
// occupancy than it loses in loads in flight per thread (measured: 11 %).
constexpr int CB_NT = 2 * BLOCK, CB_VP = PT_VOX / CB_NT;
static_assert(BLOCK % 64 == 0 && CB_NT % 64 == 0, "blocks of whole waves (ld_to_lds)");

template <bool DETMAX>
__global__ __launch_bounds__(CB_NT) void k_compose_bwd(const ComposeBwdItem* __restrict__ items,
                                                       int n_items, int n_tiles) {
  __shared__ __align__(16) int acc[3 * SCATTER_CELLS];
  __shared__ int sred[16 * (CB_NT / 64)];
  const int tile = xcd_remap(blockIdx.x, n_tiles);
  const ComposeBwdItem it = items[find_item(items, n_items, tile)];
  const int D = it.D, H = it.H, W = it.W, HW = H * W, V = D * HW;
  const PTile tc = point_tile(tile - it.tile0, H, W);
  const cgfloat* __restrict__ C = gp(it.C);
  const cgfloat* __restrict__ pr = gp(it.prev);
  const cgfloat* __restrict__ G = gp(it.g);
  gfloat* __restrict__ gpv = gp(it.gprev);
  // the owned voxels, the cells they sample and G there
  int vp[CB_VP], vz[CB_VP], vy[CB_VP], vx[CB_VP];
  bool vok[CB_VP];
  Ax cz[CB_VP], cy[CB_VP], cx[CB_VP];
  float gv[CB_VP][3];
#pragma unroll
  for (int j = 0; j < CB_VP; ++j) {
    const int k = threadIdx.x + j * CB_NT;
    vx[j] = tc.x0 + (k % PT_X);
    vy[j] = tc.y0 + (k / PT_X) % PT_Y;
    vz[j] = tc.z0 + k / (PT_X * PT_Y);
    vok[j] = vx[j] < W && vy[j] < H && vz[j] < D;
    vp[j] = vok[j] ? (vz[j] * H + vy[j]) * W + vx[j] : 0;
    const float uz = ldo(pr, vp[j]), uy = ldo(pr + V, vp[j]), ux = ldo(pr + 2 * V, vp[j]);
    cz[j] = axis_disp(vz[j], uz, D);
    cy[j] = axis_disp(vy[j], uy, H);
    cx[j] = axis_disp(vx[j], ux, W);
    gv[j][0] = ldo(G, vp[j]);
    gv[j][1] = ldo(G + V, vp[j]);
    gv[j][2] = ldo(G + 2 * V, vp[j]);
  }
  // the corners come from a box of C staged in acc (the bounding box of the
  // cells, which is also the scatter's box; the values are those of the
  // direct loads), or directly when the box is larger than ADJ_BOX_CELLS; the
  // reduce-only pass needs no corners
  BBox gb{};
  bool lds_box = false;
  if (!DETMAX) {
    int lo[3] = {INT_MAX, INT_MAX, INT_MAX};
    int hi[3] = {INT_MIN, INT_MIN, INT_MIN};
#pragma unroll
    for (int j = 0; j < CB_VP; ++j) {
      if (!vok[j]) continue;
      lo[0] = min(lo[0], cz[j].i0); hi[0] = max(hi[0], cz[j].i0 + 1);
      lo[1] = min(lo[1], cy[j].i0); hi[1] = max(hi[1], cy[j].i0 + 1);
      lo[2] = min(lo[2], cx[j].i0); hi[2] = max(hi[2], cx[j].i0 + 1);
    }
    // the second half of sred: the scatter's own reduction uses the first
    gb = scatter_box<CB_NT>(lo, hi, 0.f, 0.f, sred + 8 * (CB_NT / 64)).bb;
    lds_box = gb.cells > 0 && gb.cells <= ADJ_BOX_CELLS;  // block-uniform
    if (lds_box) {
      float* box = reinterpret_cast<float*>(acc);
      const int cells = gb.cells;
      // cell i -> (lz, ly, lx) by float reciprocals: exact here since i < 2^22
      const float inv_ex = 1.f / (float)gb.ex, inv_ey = 1.f / (float)gb.ey;
      for (int i = threadIdx.x; i < cells; i += CB_NT) {
        const int r = (int)(((float)i + 0.5f) * inv_ex);
        const int lx = i - r * gb.ex;
        const int lz = (int)(((float)r + 0.5f) * inv_ey);
        const int ly = r - lz * gb.ey;
        const int g = ((gb.lz + lz) * H + (gb.ly + ly)) * W + (gb.lx + lx);
        const int w0 = i & ~63;  // the wave's first cell: i = threadIdx.x + k * block
        ld_to_lds(C + g, box + w0);
        ld_to_lds(C + V + g, box + cells + w0);
        ld_to_lds(C + 2 * V + g, box + 2 * cells + w0);
      }
      __syncthreads();
    }
  }
  ScatterVox sv[CB_VP];
#pragma unroll
  for (int j = 0; j < CB_VP; ++j) {
    sv[j].cz = -1;
    if (!vok[j]) continue;
    const int x = vx[j], y = vy[j], z = vz[j], p = vp[j];
    const Ax az = cz[j], ay = cy[j], ax = cx[j];
    const float g0 = gv[j][0], g1 = gv[j][1], g2 = gv[j][2];
    float v0[8], v1[8], v2[8], dz, dy, dx;
    if (lds_box) {
      const float* box = reinterpret_cast<const float*>(acc);
      const int cells = gb.cells, sy = gb.ex, sz = gb.ex * gb.ey;
      const int l = ((az.i0 - gb.lz) * gb.ey + (ay.i0 - gb.ly)) * gb.ex + (ax.i0 - gb.lx);
      const int off[8] = {0, 1, sy, sy + 1, sz, sz + 1, sz + sy, sz + sy + 1};
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        v0[k] = box[l + off[k]];
        v1[k] = box[cells + l + off[k]];
        v2[k] = box[2 * cells + l + off[k]];
      }
    } else if (!DETMAX) {
      const int base = (az.i0 * H + ay.i0) * W + ax.i0;
      load8(C, base, W, HW, v0);
      load8(C + V, base, W, HW, v1);
      load8(C + 2 * V, base, W, HW, v2);
    } else {
#pragma unroll
      for (int k = 0; k < 8; ++k) v0[k] = v1[k] = v2[k] = 0.f;
    }
    tri_grad(v0, az.t, ay.t, ax.t, dz, dy, dx);
    float jz = dz * g0, jy = dy * g0, jx = dx * g0;
    tri_grad(v1, az.t, ay.t, ax.t, dz, dy, dx);
    jz = fmaf(dz, g1, jz); jy = fmaf(dy, g1, jy); jx = fmaf(dx, g1, jx);
    tri_grad(v2, az.t, ay.t, ax.t, dz, dy, dx);
    jz = fmaf(dz, g2, jz); jy = fmaf(dy, g2, jy); jx = fmaf(dx, g2, jx);
    const float o0 = fmaf(az.live, jz, g0);
    const float o1 = fmaf(ay.live, jy, g1);
    const float o2 = fmaf(ax.live, jx, g2);
    if (DETMAX) {
      // reduce-only pass: no writes
    } else if (it.prev_atomic && !it.gc64) {
      gadd(gpv + p, o0);
      gadd(gpv + V + p, o1);
      gadd(gpv + 2 * V + p, o2);
    } else {
      gpv[p] += o0;
      gpv[V + p] += o1;
      gpv[2 * V + p] += o2;
    }
    sv[j].cz = az.i0; sv[j].cy = ay.i0; sv[j].cx = ax.i0;
    sv[j].oz = z; sv[j].oy = y; sv[j].ox = x;
    sv[j].tz = az.t; sv[j].ty = ay.t; sv[j].tx = ax.t;
    sv[j].g[0] = g0; sv[j].g[1] = g1; sv[j].g[2] = g2;
  }
  if (DETMAX) {
    det_bound<false, false, CB_NT>(sv, sred, StageOut{}, it.js, it.det_slot);
    return;
  }
  DetOut det;
  if (it.gc64) {
    det.out64 = it.gc64;
    det.scale = det_scale(it.js, it.det_slot, it.det_blocks);
  }
  // with the box known, the scatter reduces only the magnitudes; the gathers
  // from acc end before its barrier, after which the bins are cleared
  scatter_tile<false, false, CB_NT>(sv, gp(it.gc), D, H, W, acc, sred, StageOut{}, det, &gb);
}

// ---------------------------------------------------------------------------
// Deterministic mode: fold of a 64-bit fixed-point field into its float
// field (one pass over the elements, in no particular order: each element
// is independent), and the clearing of the jobs' slots.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void k_det_fold(const DetFoldItem* __restrict__ items,
                                                    int n_items, int n_tiles) {
  const int tile = blockIdx.x;
  const DetFoldItem it = items[find_item(items, n_items, tile)];
  if (it.flag && *it.flag == 0) return;
  const double sc = det_scale(it.js, it.det_slot, it.det_blocks);
  const double inv = sc > 0.0 ? 1.0 / sc : 0.0;
  const int e0 = (tile - it.tile0) * ELEM_PER_BLOCK;
  for (int k = threadIdx.x; k < ELEM_PER_BLOCK; k += BLOCK) {
    const int e = e0 + k;
    if (e >= it.n) break;
    const long long q = it.q[e];
    if (q == 0) continue;
    it.f[e] += (float)((double)q * inv);
    it.q[e] = 0;
  }
}

__global__ void k_det_clear(JobState* const* __restrict__ states, int n_jobs) {
  const int j = blockIdx.x;
  if (j >= n_jobs) return;
  for (int k = threadIdx.x; k < DET_SLOTS; k += blockDim.x) states[j]->det_max[k] = 0u;
}

// ---------------------------------------------------------------------------
// Windowed statistics (Sec. 2.6): warp + LNCC/SiLNCC per window, loss and
// the per-window adjoint coefficients.
//
// The source image is first warped by the pair field once per voxel
// (k_warp).  A block of the statistics owns TY x TX window centres in (y, x)
// and marches through a chunk of z.  Every thread owns a few columns of the
// (TY + 2r) x (TX + 2r) patch around them.  For each input slice it reads the
// fixed and the warped image at its columns and keeps the last w slices of
// its per-column values in registers with their running sums over z.  For
// every centre slice the z-sums go to LDS and are summed over x, then over y
// (box_x, box_y).  Values are shifted by one per-block constant before the
// products, which keeps the variance differences well conditioned.
// ---------------------------------------------------------------------------
struct STile {
  int z0, z1, y0, x0;
};

template <int TY, int TX>
__device__ __forceinline__ STile stat_tile(int local, int D, int H, int W, int zc) {
  const int ntx = (W + TX - 1) / TX;
  const int nty = (H + TY - 1) / TY;
  STile t;
  t.x0 = (local % ntx) * TX;
  const int r = local / ntx;
  t.y0 = (r % nty) * TY;
  t.z0 = (r / nty) * zc;
  t.z1 = min(t.z0 + zc, D);
  return t;
}

// Geometry of the window sums of Q quantities.  A block of TY x TX threads;
// thread t owns the patch columns t + k * NT.  LDS holds, per quantity, the
// z-sums of the patch (rows of PXS floats), their x-sums (PY rows of TXS
// floats) and the finished sums of the centres (TY x TX).  The row strides
// are odd, so the rows a wave walks along fall in distinct banks.  The x and
// y passes give each thread a segment of 8 outputs: it reads the 8 + 2r
// inputs once and forms the 8 sums from registers as a sliding sum.
template <int R, int TY, int TX, int Q>
struct Box {
  static constexpr int NT = TY * TX, RW = R, TXO = TX;
  static constexpr int WN = 2 * R + 1;
  static constexpr int PY = TY + 2 * R, PX = TX + 2 * R, P1 = PY * PX;
  static constexpr int NS = (P1 + NT - 1) / NT;
  static constexpr int PXS = PX | 1, TXS = TX + 1;
  static constexpr int SX = 8, SY = 8, NXS = TX / SX, NYS = TY / SY;
  static constexpr int ZQ = PY * PXS, XQ = PY * TXS, YQ = TY * TX;
  static constexpr int LDS = Q * (ZQ + XQ + YQ);
  static_assert(TX % SX == 0 && TY % SY == 0, "tile not a multiple of the segments");
};

// x-sums of the window: xs[q][row][c] = sum_k zs[q][row][c + k].
template <class B>
__device__ __forceinline__ void box_x(const float* __restrict__ zs, float* __restrict__ xs, int Q) {
  constexpr int R = B::RW, WN = B::WN, SX = B::SX, PY = B::PY, NXS = B::NXS;
  const int n = Q * PY * NXS;
  for (int e = threadIdx.x; e < n; e += B::NT) {
    const int q = e / (PY * NXS), r = e - q * (PY * NXS);
    // segments fastest across lanes: with the odd row stride, the lanes of a
    // half wave read and write distinct banks
    const int row = r / NXS, seg = r - row * NXS;
    const float* s = zs + q * B::ZQ + row * B::PXS + seg * SX;
    float* d = xs + q * B::XQ + row * B::TXS + seg * SX;
    float v[SX + 2 * R];
#pragma unroll
    for (int k = 0; k < SX + 2 * R; ++k) v[k] = s[k];
    float acc = v[0];
#pragma unroll
    for (int k = 1; k < WN; ++k) acc += v[k];
    d[0] = acc;
#pragma unroll
    for (int i = 1; i < SX; ++i) {
      acc += v[i + 2 * R] - v[i - 1];
      d[i] = acc;
    }
  }
}

// y-sums of the x-sums: ys[q][y][c] = sum_k xs[q][y + k][c].
template <class B>
__device__ __forceinline__ void box_y(const float* __restrict__ xs, float* __restrict__ ys, int Q) {
  constexpr int R = B::RW, WN = B::WN, SY = B::SY, TX = B::TXO, NYS = B::NYS, TXS = B::TXS;
  const int n = Q * TX * NYS;
  for (int e = threadIdx.x; e < n; e += B::NT) {
    const int q = e / (TX * NYS), r = e - q * (TX * NYS);
    const int seg = r / TX, x = r - seg * TX;
    const float* s = xs + q * B::XQ + seg * SY * TXS + x;
    float* d = ys + q * B::YQ + seg * SY * TX + x;
    float v[SY + 2 * R];
#pragma unroll
    for (int k = 0; k < SY + 2 * R; ++k) v[k] = s[k * TXS];
    float acc = v[0];
#pragma unroll
    for (int k = 1; k < WN; ++k) acc += v[k];
    d[0] = acc;
#pragma unroll
    for (int i = 1; i < SY; ++i) {
      acc += v[i + 2 * R] - v[i - 1];
      d[i * TX] = acc;
    }
  }
}

// Warp of the source image by the pair field (Sec. 2.1): M(p) = I(p + U(p)),
// with the rigid adjustment of the source session added to U (Sec. 2.5).
__global__ __launch_bounds__(BLOCK) void k_warp(const SimItem* __restrict__ items, int n_items,
                                                int n_tiles) {
  const int tile = xcd_remap(blockIdx.x, n_tiles);
  const SimItem it = items[find_item(items, n_items, tile)];
  const int D = it.D, H = it.H, W = it.W, HW = H * W, V = D * HW;
  const PTile tc = point_tile(tile - it.tile0, H, W);
  const cgfloat* __restrict__ I = gp(it.I);
  const cgfloat* __restrict__ U = gp(it.U);
  gfloat* __restrict__ M = gp(it.M);
  VoxSet vs;
  vox_set(tc, D, H, W, vs);
  float u[VPT][3];
#pragma unroll
  for (int j = 0; j < VPT; ++j) {
    u[j][0] = ldo(U, vs.p[j]);
    u[j][1] = ldo(U + V, vs.p[j]);
    u[j][2] = ldo(U + 2 * V, vs.p[j]);
  }
  if (it.rigid) {
    float rA[9], rO[3];
#pragma unroll
    for (int k = 0; k < 9; ++k) rA[k] = it.rigid->A[k];
#pragma unroll
    for (int k = 0; k < 3; ++k) rO[k] = it.rigid->off[k];
#pragma unroll
    for (int j = 0; j < VPT; ++j) {
      const float fz = (float)vs.z[j], fy = (float)vs.y[j], fx = (float)vs.x[j];
#pragma unroll
      for (int c = 0; c < 3; ++c)
        u[j][c] += fmaf(rA[3 * c], fz, fmaf(rA[3 * c + 1], fy, fmaf(rA[3 * c + 2], fx, rO[c])));
    }
  }
  float v[VPT][8];
  Ax az[VPT], ay[VPT], ax[VPT];
#pragma unroll
  for (int j = 0; j < VPT; ++j) {
    az[j] = axis_disp(vs.z[j], u[j][0], D);
    ay[j] = axis_disp(vs.y[j], u[j][1], H);
    ax[j] = axis_disp(vs.x[j], u[j][2], W);
    load8(I, (az[j].i0 * H + ay[j].i0) * W + ax[j].i0, W, HW, v[j]);
  }
#pragma unroll
  for (int j = 0; j < VPT; ++j)
    if (vs.ok[j]) sto(M, vs.p[j], tri_val(v[j], az[j].t, ay[j].t, ax[j].t));
}

template <int R, int TY, int TX>
__global__ __launch_bounds__(TY * TX) void k_sim_stats(const SimItem* __restrict__ items, int n_items,
                                                       int n_tiles, int metric) {
  using B = Box<R, TY, TX, 5>;
  constexpr int WN = B::WN, PX = B::PX, P1 = B::P1, NS = B::NS, NT = B::NT;
  __shared__ float lds[B::LDS];
  __shared__ double red[NT / 64];
  float* zs = lds;
  float* xs = lds + 5 * B::ZQ;
  float* ys = xs + 5 * B::XQ;
  const int tile = xcd_remap(blockIdx.x, n_tiles);
  const SimItem it = items[find_item(items, n_items, tile)];
  const int D = it.D, H = it.H, W = it.W, HW = H * W, V = D * HW;
  const STile tc = stat_tile<TY, TX>(tile - it.tile0, D, H, W, it.zc);
  const cgfloat* __restrict__ F = gp(it.F);
  const cgfloat* __restrict__ M = gp(it.M);
  gfloat* __restrict__ coef = gp(it.coef);
  const int pm = (min((tc.z0 + tc.z1) / 2, D - 1) * H + min(tc.y0 + TY / 2, H - 1)) * W +
                 min(tc.x0 + TX / 2, W - 1);
  const float sF = F[pm], sM = M[pm];
  const float inv_n = 1.f / (float)(WN * WN * WN);
  const int ty = threadIdx.x / TX, tx = threadIdx.x % TX;
  const int y = tc.y0 + ty, x = tc.x0 + tx;
  const bool yx_in = (y < H) && (x < W);
  const bool yx_valid = yx_in && y >= R && y <= H - 1 - R && x >= R && x <= W - 1 - R;
  // owned patch columns: offset in a slice (-1 outside the volume) and place
  // in the z-sum rows
  int cofs[NS], zofs[NS];
  bool cval[NS];
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    const int col = threadIdx.x + k * NT;
    const int row = col / PX, cx = col % PX;
    const int yy = tc.y0 - R + row, xx = tc.x0 - R + cx;
    cval[k] = col < P1;
    cofs[k] = (cval[k] && yy >= 0 && yy < H && xx >= 0 && xx < W) ? yy * W + xx : -1;
    zofs[k] = row * B::PXS + cx;
  }
  // shifted values of slice z at the owned columns (0 outside the volume)
  auto load = [&](int z, float (&f)[NS], float (&m)[NS]) {
    const bool zin = z >= 0 && z < D;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      const bool in = zin && cofs[k] >= 0;
      const int p = in ? z * HW + cofs[k] : 0;
      f[k] = in ? ldo(F, p) - sF : 0.f;
      m[k] = in ? ldo(M, p) - sM : 0.f;
    }
  };
  // the last WN slices of each owned column (oldest first) and their sums
  // of f, m, f^2, m^2 and f m over z; the sums are formed anew from the
  // ring every WN slices, so rounding does not build up along the chunk
  float rf[NS][WN], rm[NS][WN], S[NS][5];
#pragma unroll
  for (int k = 0; k < NS; ++k) {
#pragma unroll
    for (int j = 0; j < WN; ++j) rf[k][j] = rm[k][j] = 0.f;
#pragma unroll
    for (int q = 0; q < 5; ++q) S[k][q] = 0.f;
  }
  // values of slice zi are loaded one iteration ahead
  float fn[NS], mn[NS];
  load(tc.z0 - R, fn, mn);
  int phase = 0;
  double lsum = 0.0;
  for (int zi = tc.z0 - R; zi < tc.z1 + R; ++zi) {
    const bool exact = ++phase == WN;
    if (exact) phase = 0;
    float fv[NS], mv[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      fv[k] = fn[k];
      mv[k] = mn[k];
    }
    load(zi + 1, fn, mn);
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      const float fo = rf[k][0], mo = rm[k][0];
#pragma unroll
      for (int j = 0; j + 1 < WN; ++j) {
        rf[k][j] = rf[k][j + 1];
        rm[k][j] = rm[k][j + 1];
      }
      const float f = fv[k], m = mv[k];
      rf[k][WN - 1] = f;
      rm[k][WN - 1] = m;
      if (exact) {
        float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f, s4 = 0.f;
#pragma unroll
        for (int j = 0; j < WN; ++j) {
          s0 += rf[k][j];
          s1 += rm[k][j];
          s2 = fmaf(rf[k][j], rf[k][j], s2);
          s3 = fmaf(rm[k][j], rm[k][j], s3);
          s4 = fmaf(rf[k][j], rm[k][j], s4);
        }
        S[k][0] = s0; S[k][1] = s1; S[k][2] = s2; S[k][3] = s3; S[k][4] = s4;
      } else {
        S[k][0] += f - fo;
        S[k][1] += m - mo;
        S[k][2] += fmaf(f, f, -fo * fo);
        S[k][3] += fmaf(m, m, -mo * mo);
        S[k][4] += fmaf(f, m, -fo * mo);
      }
    }
    const int zcen = zi - R;
    if (zcen >= tc.z0) {
      const bool zvalid = zcen >= R && zcen <= D - 1 - R;
      if (zvalid) {
#pragma unroll
        for (int k = 0; k < NS; ++k) {
          if (!cval[k]) continue;
#pragma unroll
          for (int q = 0; q < 5; ++q) zs[q * B::ZQ + zofs[k]] = S[k][q];
        }
        __syncthreads();
        box_x<B>(zs, xs, 5);
        __syncthreads();
        box_y<B>(xs, ys, 5);
        __syncthreads();
      }
      if (yx_in) {
        const int p = (zcen * H + y) * W + x;
        float al = 0.f, be = 0.f, ga = 0.f;
        if (zvalid && yx_valid) {
          float Sw[5];
#pragma unroll
          for (int q = 0; q < 5; ++q) Sw[q] = ys[q * B::YQ + threadIdx.x];
          const float mF = Sw[0] * inv_n, mM = Sw[1] * inv_n;
          const float vFr = Sw[2] * inv_n - mF * mF;
          const float vMr = Sw[3] * inv_n - mM * mM;
          const float c = Sw[4] * inv_n - mF * mM;
          const float vF = fmaxf(vFr, 0.f), vM = fmaxf(vMr, 0.f);
          float l, av, ac;
          if (metric == 0) {
            const float den = vF * vM;
            if (den > EPS_LNCC) {
              const float sd = sqrtf(den);
              l = 1.f - c / sd;
              ac = -1.f / sd;
              av = c / (2.f * vM * sd);
            } else {
              const float sd = sqrtf(EPS_LNCC);
              l = 1.f - c / sd;
              ac = -1.f / sd;
              av = 0.f;
            }
          } else {
            const float dd = fmaxf(vF, EPS_SILNCC);
            l = vM - c * c / dd;
            ac = -2.f * c / dd;
            av = 1.f;
          }
          if (!(vMr > 0.f)) av = 0.f;
          lsum += (double)l;
          const float mFt = mF + sF, mMt = mM + sM;
          al = -(2.f * mMt * av + mFt * ac) * inv_n;
          be = av * inv_n;
          ga = ac * inv_n;
        }
        if (coef) {
          sto(coef, p, al);
          sto(coef + V, p, be);
          sto(coef + 2 * V, p, ga);
        }
      }
    }
  }
  const double tot = block_sum<NT>(lsum, red);
  if (threadIdx.x == 0) {
    const double v = tot * it.inv_nr;
    if (it.js) unsafeAtomicAdd(&it.js->loss_sim, v);
    if (it.sim_out) unsafeAtomicAdd(it.sim_out, v);
  }
}

// Gradient of Sim with respect to the pair field:
//   dSim/dM(y) = (Box alpha + 2 M Box beta + F Box gamma)(y) / N_R,
//   dSim/dU(y) = dSim/dM(y) * grad I_j(y + U(y)).
// The window sums of the coefficients are formed like those of k_sim_stats;
// the coefficients of the next slice and the output voxel's loads are issued
// before the current slice's sums.
template <int R, int TY, int TX>
__global__ __launch_bounds__(TY * TX) void k_sim_grad(const SimItem* __restrict__ items, int n_items,
                                                      int n_tiles) {
  using B = Box<R, TY, TX, 3>;
  constexpr int WN = B::WN, PX = B::PX, P1 = B::P1, NS = B::NS, NT = B::NT;
  __shared__ float lds[B::LDS];
  float* zs = lds;
  float* xs = lds + 3 * B::ZQ;
  float* ys = xs + 3 * B::XQ;
  const int tile = xcd_remap(blockIdx.x, n_tiles);
  const SimItem it = items[find_item(items, n_items, tile)];
  const int D = it.D, H = it.H, W = it.W, HW = H * W, V = D * HW;
  const STile tc = stat_tile<TY, TX>(tile - it.tile0, D, H, W, it.zc);
  const cgfloat* __restrict__ F = gp(it.F);
  const cgfloat* __restrict__ I = gp(it.I);
  const cgfloat* __restrict__ U = gp(it.U);
  const cgfloat* __restrict__ coef = gp(it.coef);
  gfloat* __restrict__ gU = gp(it.gU);
  const float inv_nr = (float)it.inv_nr;
  const int ty = threadIdx.x / TX, tx = threadIdx.x % TX;
  const int y = tc.y0 + ty, x = tc.x0 + tx;
  const bool yx_in = y < H && x < W;
  int cyy[NS], cxx[NS], zofs[NS];
  bool cin[NS], cval[NS];
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    const int col = threadIdx.x + k * NT;
    const int row = col / PX, cx = col % PX;
    cval[k] = col < P1;
    cyy[k] = tc.y0 - R + row;
    cxx[k] = tc.x0 - R + cx;
    zofs[k] = row * B::PXS + cx;
    cin[k] = cval[k] && cyy[k] >= 0 && cyy[k] < H && cxx[k] >= 0 && cxx[k] < W;
  }
  auto load_coef = [&](int z, float (&c)[NS][3]) {
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      const bool in = cin[k] && z >= 0 && z < D;
      const int p = in ? (z * H + cyy[k]) * W + cxx[k] : 0;
      c[k][0] = in ? coef[p] : 0.f;
      c[k][1] = in ? coef[V + p] : 0.f;
      c[k][2] = in ? coef[2 * V + p] : 0.f;
    }
  };
  // output voxel (zo, y, x): U first, then F and the corners of I
  float rA[9], rO[3];
  const bool rigid = it.rigid != nullptr;
  if (rigid) {
#pragma unroll
    for (int k = 0; k < 9; ++k) rA[k] = it.rigid->A[k];
#pragma unroll
    for (int k = 0; k < 3; ++k) rO[k] = it.rigid->off[k];
  }
  auto load_uo = [&](int zo, float (&u)[3]) {
    const bool in = yx_in && zo >= 0 && zo < D;
    const int p = in ? (zo * H + y) * W + x : 0;
    u[0] = in ? U[p] : 0.f;
    u[1] = in ? U[V + p] : 0.f;
    u[2] = in ? U[2 * V + p] : 0.f;
    if (rigid && in) {
      const float fz = (float)zo, fy = (float)y, fx = (float)x;
#pragma unroll
      for (int c = 0; c < 3; ++c)
        u[c] += fmaf(rA[3 * c], fz, fmaf(rA[3 * c + 1], fy, fmaf(rA[3 * c + 2], fx, rO[c])));
    }
  };
  float c0[NS][3];
  load_coef(tc.z0 - R, c0);
  float uo[3];
  load_uo(tc.z0, uo);
  // the last WN slices of the coefficients of each owned column and their
  // sums over z (formed anew every WN slices)
  float rc[NS][3][WN], S[NS][3];
#pragma unroll
  for (int k = 0; k < NS; ++k)
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      S[k][q] = 0.f;
#pragma unroll
      for (int j = 0; j < WN; ++j) rc[k][q][j] = 0.f;
    }
  int phase = 0;
  for (int zi = tc.z0 - R; zi < tc.z1 + R; ++zi) {
    const bool exact = ++phase == WN;
    if (exact) phase = 0;
#pragma unroll
    for (int k = 0; k < NS; ++k)
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const float o = rc[k][q][0];
#pragma unroll
        for (int j = 0; j + 1 < WN; ++j) rc[k][q][j] = rc[k][q][j + 1];
        rc[k][q][WN - 1] = c0[k][q];
        if (exact) {
          float s = 0.f;
#pragma unroll
          for (int j = 0; j < WN; ++j) s += rc[k][q][j];
          S[k][q] = s;
        } else {
          S[k][q] += c0[k][q] - o;
        }
      }
    float c1[NS][3];
    load_coef(zi + 1, c1);
    const int zo = zi - R;
    const bool out_now = zo >= tc.z0;
    // loads of the output voxel of this iteration
    float vI[8], fo = 0.f;
    Ax az, ay, ax;
    {
      const bool in = yx_in && zo >= tc.z0 && zo < D;
      const int zz = in ? zo : 0, yy = in ? y : 0, xx = in ? x : 0;
      az = axis_disp(zz, uo[0], D);
      ay = axis_disp(yy, uo[1], H);
      ax = axis_disp(xx, uo[2], W);
      load8(I, (az.i0 * H + ay.i0) * W + ax.i0, W, HW, vI);
      fo = F[(zz * H + yy) * W + xx];
    }
    float un[3];
    load_uo(out_now ? zo + 1 : tc.z0, un);
    if (out_now) {
#pragma unroll
      for (int k = 0; k < NS; ++k) {
        if (!cval[k]) continue;
#pragma unroll
        for (int q = 0; q < 3; ++q) zs[q * B::ZQ + zofs[k]] = S[k][q];
      }
      __syncthreads();
      box_x<B>(zs, xs, 3);
      __syncthreads();
      box_y<B>(xs, ys, 3);
      __syncthreads();
      if (yx_in) {
        const float B0 = ys[threadIdx.x], B1 = ys[B::YQ + threadIdx.x],
                    B2 = ys[2 * B::YQ + threadIdx.x];
        const int p = (zo * H + y) * W + x;
        float dz, dy, dx;
        const float M = tri_grad(vI, az.t, ay.t, ax.t, dz, dy, dx);
        const float dM = (B0 + 2.f * M * B1 + fo * B2) * inv_nr;
        gU[p] = dM * dz * az.live;
        gU[V + p] = dM * dy * ay.live;
        gU[2 * V + p] = dM * dx * ax.live;
      }
    }
#pragma unroll
    for (int k = 0; k < NS; ++k) {
      c0[k][0] = c1[k][0];
      c0[k][1] = c1[k][1];
      c0[k][2] = c1[k][2];
    }
    if (out_now) {
      uo[0] = un[0];
      uo[1] = un[1];
      uo[2] = un[2];
    }
  }
}

// ---------------------------------------------------------------------------
// Adam (PyTorch semantics) with the warm-up + cosine schedule (Sec. 2.7),
// or the plain gradient (mode 1).  Clears g0f / g0b after reading them.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double schedule_lr(const JobState* js, int step) {
  const int T = js->T, Wu = js->W;
  if (step <= Wu) return (double)js->lr0 * step / (double)Wu;
  if (T == Wu) return (double)js->lr0;
  return (double)js->lr0 * 0.5 * (1.0 + cos(M_PI * (double)(step - Wu) / (double)(T - Wu)));
}

__global__ __launch_bounds__(BLOCK) void k_adam(const AdamItem* __restrict__ items, int n_items,
                                                int n_tiles) {
  const int tile = blockIdx.x;
  const AdamItem it = items[find_item(items, n_items, tile)];
  const int n = it.n;
  const int q0 = (tile - it.tile0) * ELEM_PER_BLOCK;
  gfloat* __restrict__ g0f = gp(it.g0f);
  gfloat* __restrict__ g0b = gp(it.g0b);
  const cgfloat* __restrict__ gs = gp(it.gsrc);
  auto grad = [&](int i) -> float {
    if (it.gsrc) return gs[i];
    const float g = it.scale * (g0f[i] - g0b[i]);
    g0f[i] = 0.f;
    g0b[i] = 0.f;
    return g;
  };
  if (it.mode != 0) {
    gfloat* __restrict__ go = gp(it.gout);
    const float sc = it.mode == 1 ? it.gscale : 1.f;
    for (int k = threadIdx.x; k < ELEM_PER_BLOCK; k += BLOCK) {
      const int q = q0 + k;
      if (q >= n) break;
#pragma unroll
      for (int c = 0; c < 3; ++c) go[c * n + q] = grad(c * n + q) * sc;
    }
    return;
  }
  const JobState* js = it.js;
  const int step = js->t + 1;
  const double lr = schedule_lr(js, step);
  const double bc1 = 1.0 - pow((double)js->b1, (double)step);
  const double bc2 = 1.0 - pow((double)js->b2, (double)step);
  const float step_size = (float)(lr / bc1);
  const float bc2s = (float)sqrt(bc2);
  const float b1 = js->b1, b2 = js->b2, eps = js->eps;
  gfloat* __restrict__ phi = gp(it.phi);
  gfloat* __restrict__ mm = gp(it.m);
  gfloat* __restrict__ vv = gp(it.v);
  for (int k = threadIdx.x; k < ELEM_PER_BLOCK; k += BLOCK) {
    const int q = q0 + k;
    if (q >= n) break;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int i = c * n + q;
      const float g = grad(i);
      float m = mm[i], v = vv[i];
      m = fmaf(1.f - b1, g - m, m);
      v = fmaf(1.f - b2, g * g, v * b2);
      const float den = sqrtf(v) / bc2s + eps;
      phi[i] -= step_size * (m / den);
      mm[i] = m;
      vv[i] = v;
    }
  }
}

// ---------------------------------------------------------------------------
// Gaussian smoothing of the flow (Sec. 2.4, Appendix A): one separable pass of
// the periodic filter along one axis, on the three components.  Appendix A
// applies the Gaussian transfer function in the Fourier domain; its spatial
// form on a periodic line is a circular convolution whose taps the host
// computes from that transfer function (out to where they vanish below float
// rounding, or over the whole line), so one pass per axis applies the whole
// 3-D filter.  The taps are symmetric, so the same pass is its own adjoint.
// ---------------------------------------------------------------------------
// SMOOTH_S consecutive outputs, from p0 on, of the circular convolution of a
// line of n samples held in LDS at line[pos * ls] with the taps w.  The line
// is read once per chunk; each sample feeds every output it reaches (taps
// outside 0..2r are zero), so output p0+o sums its taps in the order k = 0..2r.
__device__ __forceinline__ void smooth_chunk(const float* line, int ls, int n, int p0, int r,
                                             const float* __restrict__ w,
                                             float (&acc)[SMOOTH_S]) {
#pragma unroll
  for (int o = 0; o < SMOOTH_S; ++o) acc[o] = 0.f;
  int pos = (p0 - r) % n;
  if (pos < 0) pos += n;
  const int m = SMOOTH_S + 2 * r;
  for (int j = 0; j < m; ++j) {
    const float v = line[pos * ls];
#pragma unroll
    for (int o = 0; o < SMOOTH_S; ++o) acc[o] = fmaf(w[SMOOTH_WPAD + j - o], v, acc[o]);
    if (++pos == n) pos = 0;
  }
}

// One pass of the separable periodic Gaussian with the item's taps.  A block
// stages whole lines of one component in LDS, so every sample is read from
// HBM once and written once; a radius up to half the line wraps round it.
__global__ __launch_bounds__(BLOCK) void k_smooth(const SmoothItem* __restrict__ items, int n_items,
                                                  int n_tiles) {
  extern __shared__ float lds[];
  const int tile = xcd_remap(blockIdx.x, n_tiles);
  const SmoothItem& it = items[find_item(items, n_items, tile)];
  const int D = it.D, H = it.H, W = it.W;
  const int V = D * H * W;
  const int local = tile - it.tile0;
  const int comp = local / it.tiles_comp;
  const int t = local - comp * it.tiles_comp;
  const cgfloat* __restrict__ src = gp(it.src) + comp * V;
  gfloat* __restrict__ dst = gp(it.dst) + comp * V;
  const int r = it.radius, L = it.lines, ls = it.lshift;
  if (it.axis < 2) {
    // lines along z (axis 0) or y (axis 1); the tile is L adjacent x columns
    const int n = it.axis == 0 ? D : H;
    const int stride = it.axis == 0 ? H * W : W;
    const int nxc = (W + L - 1) >> ls;
    const int outer = t / nxc;
    const int x0 = (t - outer * nxc) << ls;
    const int width = min(L, W - x0);
    const int base = (it.axis == 0 ? outer * W : outer * H * W) + x0;
    // SMOOTH_U loads in flight per thread before they land in LDS
    const int total = n << ls;
    for (int e0 = threadIdx.x; e0 < total; e0 += BLOCK * SMOOTH_U) {
      float v[SMOOTH_U];
#pragma unroll
      for (int u = 0; u < SMOOTH_U; ++u) {
        const int e = e0 + u * BLOCK;
        const int p = e >> ls, c = e & (L - 1);
        v[u] = (e < total && c < width) ? src[base + p * stride + c] : 0.f;
      }
#pragma unroll
      for (int u = 0; u < SMOOTH_U; ++u) {
        const int e = e0 + u * BLOCK;
        if (e < total) lds[e] = v[u];
      }
    }
    __syncthreads();
    const int c = threadIdx.x & (L - 1);
    if (c < width) {
      const int chunks = (n + SMOOTH_S - 1) / SMOOTH_S;
      for (int q = threadIdx.x >> ls; q < chunks; q += BLOCK >> ls) {
        const int p0 = q * SMOOTH_S;
        float acc[SMOOTH_S];
        smooth_chunk(lds + c, L, n, p0, r, it.w, acc);
#pragma unroll
        for (int o = 0; o < SMOOTH_S; ++o)
          if (p0 + o < n) dst[base + (p0 + o) * stride + c] = acc[o];
      }
    }
  } else {
    // lines along x: the tile is L consecutive rows, staged with an odd row
    // pitch so lanes on different rows hit different banks
    const int Wp = W | 1;
    const int row0 = t << ls;
    const int rows = min(L, D * H - row0);
    float* in = lds;
    float* out = lds + L * Wp;
    // the tile is rows * W contiguous floats; e -> (e / W, e % W) through a
    // float reciprocal, exact here since e < 2^14 leaves a wide margin
    const int total = rows * W;
    const float invW = 1.f / (float)W;
    const cgfloat* __restrict__ tsrc = src + row0 * W;
    for (int e0 = threadIdx.x; e0 < total; e0 += BLOCK * SMOOTH_U) {
      float v[SMOOTH_U];
#pragma unroll
      for (int u = 0; u < SMOOTH_U; ++u) {
        const int e = e0 + u * BLOCK;
        v[u] = e < total ? tsrc[e] : 0.f;
      }
#pragma unroll
      for (int u = 0; u < SMOOTH_U; ++u) {
        const int e = e0 + u * BLOCK;
        const int row = (int)(((float)e + 0.5f) * invW);
        if (e < total) in[e + row * (Wp - W)] = v[u];
      }
    }
    __syncthreads();
    const int rr = threadIdx.x & (L - 1);
    if (rr < rows) {
      const int chunks = (W + SMOOTH_S - 1) / SMOOTH_S;
      for (int q = threadIdx.x >> ls; q < chunks; q += BLOCK >> ls) {
        const int p0 = q * SMOOTH_S;
        float acc[SMOOTH_S];
        smooth_chunk(in + rr * Wp, 1, W, p0, r, it.w, acc);
#pragma unroll
        for (int o = 0; o < SMOOTH_S; ++o)
          if (p0 + o < W) out[rr * Wp + p0 + o] = acc[o];
      }
    }
    __syncthreads();
    gfloat* __restrict__ tdst = dst + row0 * W;
    for (int e = threadIdx.x; e < total; e += BLOCK) {
      const int row = (int)(((float)e + 0.5f) * invW);
      tdst[e] = out[e + row * (Wp - W)];
    }
  }
}

__global__ void k_finish(JobState* const* __restrict__ states, int n_jobs) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_jobs) return;
  JobState* js = states[i];
  const double L = js->loss_sim + js->loss_reg + js->loss_ext;
  const int h = js->hist_base + js->t;
  if (js->history && h >= 0 && h < js->hist_len) js->history[h] = L;
  if (!isfinite(L)) js->nonfinite = 1;
  js->loss_sim = 0.0;
  js->loss_reg = 0.0;
  js->loss_ext = 0.0;
  for (int k = 0; k < js->n_flags; ++k) js->flags[k] = 0;
  js->t += 1;
}

// ---------------------------------------------------------------------------
// Pyramid (Sec. 2.7)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void k_pool2(const PoolItem* __restrict__ items, int n_items,
                                                 int n_tiles) {
  const int tile = blockIdx.x;
  const PoolItem it = items[find_item(items, n_items, tile)];
  const int D = it.D, H = it.H, W = it.W;
  const int D2 = D / 2, H2 = H / 2, W2 = W / 2;
  const int n = D2 * H2 * W2;
  const int q0 = (tile - it.tile0) * ELEM_PER_BLOCK;
  for (int k = threadIdx.x; k < ELEM_PER_BLOCK; k += BLOCK) {
    const int q = q0 + k;
    if (q >= n) break;
    const int X = q % W2, Y = (q / W2) % H2, Z = q / (W2 * H2);
    const float* s = it.src + ((2 * Z) * H + 2 * Y) * W + 2 * X;
    const int HW = H * W;
    const float a = (s[0] + s[1]) + (s[W] + s[W + 1]);
    const float b = (s[HW] + s[HW + 1]) + (s[HW + W] + s[HW + W + 1]);
    it.dst[q] = (a + b) * 0.125f;
  }
}

// A block stages the coarse cells behind a tile of UF_TZ x UF_TY x UF_TX fine
// voxels (t/2 + 2 per axis, three components, coordinates clamped to the
// grid) in LDS; every fine voxel then reads its 8 corners from there.
__global__ __launch_bounds__(BLOCK) void k_upsample2(const UpItem* __restrict__ items, int n_items,
                                                     int n_tiles) {
  constexpr int CZ = UF_TZ / 2 + 2, CY = UF_TY / 2 + 2, CX = UF_TX / 2 + 2, CN = CZ * CY * CX;
  constexpr int PER = UF_TZ * UF_TY * UF_TX / BLOCK;
  static_assert(UF_TY * UF_TX == BLOCK, "one fine slice of the tile per thread pass");
  __shared__ float cs[3 * CN];
  const int tile = xcd_remap(blockIdx.x, n_tiles);
  const UpItem it = items[find_item(items, n_items, tile)];
  const int D = it.D, H = it.H, W = it.W, HW = H * W, V = D * HW;
  const int D2 = 2 * D, H2 = 2 * H, W2 = 2 * W;
  const int n = D2 * H2 * W2;
  const int local = tile - it.tile0;
  const int ntx = (W2 + UF_TX - 1) / UF_TX, nty = (H2 + UF_TY - 1) / UF_TY;
  const int fx0 = (local % ntx) * UF_TX, fy0 = ((local / ntx) % nty) * UF_TY,
            fz0 = (local / ntx / nty) * UF_TZ;
  // first staged coarse cell per axis: the floor cell of the tile's first
  // fine sample, (f0 - 0.5) / 2 = f0 / 2 - 0.25
  const int cz0 = fz0 / 2 - 1, cy0 = fy0 / 2 - 1, cx0 = fx0 / 2 - 1;
  const cgfloat* __restrict__ src = gp(it.src);
  for (int i = threadIdx.x; i < 3 * CN; i += BLOCK) {
    const int c = i / CN, r = i - c * CN;
    const int lz = r / (CY * CX), r2 = r - lz * (CY * CX), ly = r2 / CX, lx = r2 - ly * CX;
    const int z = min(max(cz0 + lz, 0), D - 1), y = min(max(cy0 + ly, 0), H - 1),
              x = min(max(cx0 + lx, 0), W - 1);
    cs[i] = src[c * V + (z * H + y) * W + x];
  }
  __syncthreads();
  const int fy = fy0 + threadIdx.x / UF_TX, fx = fx0 + threadIdx.x % UF_TX;
  const Ax ay = axis_pos(((float)fy - 0.5f) * 0.5f, H), ax = axis_pos(((float)fx - 0.5f) * 0.5f, W);
  gfloat* __restrict__ dst = gp(it.dst);
#pragma unroll
  for (int j = 0; j < PER; ++j) {
    const int fz = fz0 + j;
    if (fz >= D2 || fy >= H2 || fx >= W2) continue;
    const Ax az = axis_pos(((float)fz - 0.5f) * 0.5f, D);
    const int base = ((az.i0 - cz0) * CY + (ay.i0 - cy0)) * CX + (ax.i0 - cx0);
    const int q = (fz * H2 + fy) * W2 + fx;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float* p = cs + c * CN + base;
      const float v[8] = {p[0], p[1], p[CX], p[CX + 1],
                          p[CY * CX], p[CY * CX + 1], p[CY * CX + CX], p[CY * CX + CX + 1]};
      dst[c * n + q] = 2.f * tri_val(v, az.t, ay.t, ax.t);
    }
  }
}

// Adjoint of k_upsample2 (flow grid -> image grid, values doubled): each
// coarse voxel gathers, with weight 2 w, the fine voxels whose sample cell has
// it as a corner.  Along an axis those are the fine indices 2c-1 .. 2c+2; the
// weight is evaluated with the forward's own clamp and cell rules, so borders
// match it exactly.  A gather, so no atomics and a fixed summation order.
__device__ __forceinline__ float up_weight(int f, int c, int n) {
  const Ax a = axis_pos(((float)f - 0.5f) * 0.5f, n);
  return c == a.i0 ? 1.f - a.t : (c == a.i0 + 1 ? a.t : 0.f);
}

// The weights are separable, so a block stages the fine region behind a tile
// of UA_TZ x UA_TY x UA_TX coarse voxels (2t + 2 fine samples per axis) in
// LDS, one component at a time, and sums along x, then y, then z, with the
// 4 weights per coarse index of each axis computed once per block: every fine
// sample is read from HBM once and the 64-tap gather becomes 3 x 4 taps.
__global__ __launch_bounds__(BLOCK) void k_upsample2_adj(const UpItem* __restrict__ items,
                                                         int n_items, int n_tiles) {
  constexpr int FZ = 2 * UA_TZ + 2, FY = 2 * UA_TY + 2, FX = 2 * UA_TX + 2;
  constexpr int FN = FZ * FY * FX;           // fine region; later the y sums
  constexpr int S1 = FZ * FY * UA_TX;        // x sums
  constexpr int S2 = FZ * UA_TY * UA_TX;     // y sums
  constexpr int TN = UA_TZ * UA_TY * UA_TX;  // outputs
  static_assert(S2 <= FN, "the y sums reuse the fine region");
  __shared__ float fine[FN];
  __shared__ float s1[S1];
  __shared__ float wz[UA_TZ][4], wy[UA_TY][4], wx[UA_TX][4];
  const int tile = xcd_remap(blockIdx.x, n_tiles);
  const UpItem it = items[find_item(items, n_items, tile)];
  const int D = it.D, H = it.H, W = it.W, V = D * H * W;
  const int D2 = 2 * D, H2 = 2 * H, W2 = 2 * W, n2 = 8 * V;
  const int local = tile - it.tile0;
  const int ntx = (W + UA_TX - 1) / UA_TX, nty = (H + UA_TY - 1) / UA_TY;
  const int cx0 = (local % ntx) * UA_TX, cy0 = ((local / ntx) % nty) * UA_TY,
            cz0 = (local / ntx / nty) * UA_TZ;
  // fine index of the first staged sample along each axis: 2 c0 - 1
  const int fz0 = 2 * cz0 - 1, fy0 = 2 * cy0 - 1, fx0 = 2 * cx0 - 1;
  // w[o][k]: weight of fine 2(c0 + o) - 1 + k for coarse c0 + o (0 off the grid)
  auto weight = [](int f, int c, int n) { return (f >= 0 && f < 2 * n) ? up_weight(f, c, n) : 0.f; };
  for (int i = threadIdx.x; i < (UA_TZ + UA_TY + UA_TX) * 4; i += BLOCK) {
    const int o = i / 4, k = i % 4;
    if (o < UA_TZ) {
      wz[o][k] = weight(fz0 + 2 * o + k, cz0 + o, D);
    } else if (o < UA_TZ + UA_TY) {
      const int q = o - UA_TZ;
      wy[q][k] = weight(fy0 + 2 * q + k, cy0 + q, H);
    } else {
      const int q = o - UA_TZ - UA_TY;
      wx[q][k] = weight(fx0 + 2 * q + k, cx0 + q, W);
    }
  }
  const cgfloat* __restrict__ g = gp(it.src);
  gfloat* __restrict__ out = gp(it.dst);
  for (int c = 0; c < 3; ++c) {
    // UL loads in flight per thread before they land in LDS
    constexpr int UL = 8;
    for (int i0 = threadIdx.x; i0 < FN; i0 += BLOCK * UL) {
      float v[UL];
#pragma unroll
      for (int u = 0; u < UL; ++u) {
        const int i = i0 + u * BLOCK;
        const int lz = i / (FY * FX), r = i - lz * (FY * FX), ly = r / FX, lx = r - ly * FX;
        const int fz = fz0 + lz, fy = fy0 + ly, fx = fx0 + lx;
        const bool in = i < FN && fz >= 0 && fz < D2 && fy >= 0 && fy < H2 && fx >= 0 && fx < W2;
        v[u] = in ? g[c * n2 + (fz * H2 + fy) * W2 + fx] : 0.f;
      }
#pragma unroll
      for (int u = 0; u < UL; ++u)
        if (i0 + u * BLOCK < FN) fine[i0 + u * BLOCK] = v[u];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < S1; i += BLOCK) {
      const int row = i / UA_TX, ox = i - row * UA_TX;
      const float* f = fine + row * FX + 2 * ox;
      s1[i] = fmaf(wx[ox][3], f[3], fmaf(wx[ox][2], f[2], fmaf(wx[ox][1], f[1], wx[ox][0] * f[0])));
    }
    __syncthreads();
    float* s2 = fine;
    for (int i = threadIdx.x; i < S2; i += BLOCK) {
      const int lz = i / (UA_TY * UA_TX), r = i - lz * (UA_TY * UA_TX);
      const int oy = r / UA_TX, ox = r - oy * UA_TX;
      const float* f = s1 + (lz * FY + 2 * oy) * UA_TX + ox;
      s2[i] = fmaf(wy[oy][3], f[3 * UA_TX],
                   fmaf(wy[oy][2], f[2 * UA_TX], fmaf(wy[oy][1], f[UA_TX], wy[oy][0] * f[0])));
    }
    __syncthreads();
    for (int i = threadIdx.x; i < TN; i += BLOCK) {
      const int oz = i / (UA_TY * UA_TX), r = i - oz * (UA_TY * UA_TX);
      const int oy = r / UA_TX, ox = r - oy * UA_TX;
      const int z = cz0 + oz, y = cy0 + oy, x = cx0 + ox;
      if (z >= D || y >= H || x >= W) continue;
      const float* f = s2 + (2 * oz) * (UA_TY * UA_TX) + oy * UA_TX + ox;
      constexpr int SZ = UA_TY * UA_TX;
      const float v = fmaf(wz[oz][3], f[3 * SZ],
                           fmaf(wz[oz][2], f[2 * SZ], fmaf(wz[oz][1], f[SZ], wz[oz][0] * f[0])));
      out[c * V + (z * H + y) * W + x] = 2.f * v;
    }
    __syncthreads();  // before the next component overwrites the fine region
  }
}

// ---------------------------------------------------------------------------
// Single-step helpers for the unit entry points
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void k_adam_flat(int64_t n, float* x, const float* g, float* m,
                                                     float* v, float step_size, float bc2s,
                                                     float b1, float b2, float eps) {
  const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (i >= n) return;
  const float gg = g[i];
  float mm = m[i], vv = v[i];
  mm = fmaf(1.f - b1, gg - mm, mm);
  vv = fmaf(1.f - b2, gg * gg, vv * b2);
  const float den = sqrtf(vv) / bc2s + eps;
  x[i] -= step_size * (mm / den);
  m[i] = mm;
  v[i] = vv;
}

__global__ __launch_bounds__(BLOCK) void k_reg(int D, int H, int W, const float* phi, double* out,
                                               float* grad) {
  __shared__ double red[BLOCK / 64];
  const int V = D * H * W;
  const int q = blockIdx.x * BLOCK + threadIdx.x;
  const float inv_mz = 1.f / (float)((D - 1) * H * W), inv_my = 1.f / (float)(D * (H - 1) * W),
              inv_mx = 1.f / (float)(D * H * (W - 1));
  double val = 0.0;
  if (q < V) {
    const int x = q % W, y = (q / W) % H, z = q / (W * H);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float g = reg_point(gp(phi) + c * V, z, y, x, D, H, W, inv_mz, inv_my, inv_mx, &val);
      if (grad) grad[c * V + q] = g;
    }
  }
  const double tot = block_sum(val, red);
  if (threadIdx.x == 0) unsafeAtomicAdd(out, tot);
}

__global__ void k_fill(float* p, int64_t n, float v) {
  const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
// Optional start / stop events of the next launches on this thread (the
// runtime's kernel timing): recorded by the launch packet itself, so a timed
// launch costs one API call and the events bracket the kernel alone.
static thread_local hipEvent_t t_launch_start = nullptr, t_launch_stop = nullptr;

void set_launch_events(hipEvent_t start, hipEvent_t stop) {
  t_launch_start = start;
  t_launch_stop = stop;
}

#define MUSTER_LAUNCH(kernel, grid, block, shm, stream, ...)                                  \
  do {                                                                                         \
    if (t_launch_start)                                                                        \
      hipExtLaunchKernelGGL(kernel, grid, block, shm, stream, t_launch_start, t_launch_stop, 0, \
                            __VA_ARGS__);                                                      \
    else                                                                                       \
      hipLaunchKernelGGL(kernel, grid, block, shm, stream, __VA_ARGS__);                      \
  } while (0)

hipError_t launch_exp_fwd(const ExpFwdItem* items, int n_items, int n_tiles, hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  MUSTER_LAUNCH(k_exp_fwd, dim3(n_tiles), dim3(BLOCK), 0, s, items, n_items, n_tiles);
  return hipGetLastError();
}

hipError_t launch_compose_fwd(const ComposeItem* items, int n_items, int n_tiles, hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  MUSTER_LAUNCH(k_compose_fwd, dim3(n_tiles), dim3(BLOCK), 0, s, items, n_items, n_tiles);
  return hipGetLastError();
}

template <bool REG>
static hipError_t launch_exp_bwd_(const ExpBwdItem* items, int n_items, int n_tiles, int staged,
                                  hipStream_t s) {
  switch (staged) {
    case 0: MUSTER_LAUNCH((k_exp_bwd<0, REG>), dim3(n_tiles), dim3(BLOCK), 0, s, items, n_items, n_tiles); break;
    case 1: MUSTER_LAUNCH((k_exp_bwd<1, REG>), dim3(n_tiles), dim3(BLOCK), 0, s, items, n_items, n_tiles); break;
    case 2: MUSTER_LAUNCH((k_exp_bwd<2, REG>), dim3(n_tiles), dim3(BLOCK), 0, s, items, n_items, n_tiles); break;
    case 3: MUSTER_LAUNCH((k_exp_bwd<3, REG>), dim3(n_tiles), dim3(BLOCK), 0, s, items, n_items, n_tiles); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_exp_bwd_detmax(const ExpBwdItem* items, int n_items, int n_tiles, int staged,
                                 hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  switch (staged) {
    case 0: MUSTER_LAUNCH((k_exp_bwd<0, true, true>), dim3(n_tiles), dim3(BLOCK), 0, s, items, n_items, n_tiles); break;
    case 1: MUSTER_LAUNCH((k_exp_bwd<1, true, true>), dim3(n_tiles), dim3(BLOCK), 0, s, items, n_items, n_tiles); break;
    case 2: MUSTER_LAUNCH((k_exp_bwd<2, true, true>), dim3(n_tiles), dim3(BLOCK), 0, s, items, n_items, n_tiles); break;
    case 3: MUSTER_LAUNCH((k_exp_bwd<3, true, true>), dim3(n_tiles), dim3(BLOCK), 0, s, items, n_items, n_tiles); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_det_fold(const DetFoldItem* items, int n_items, int n_tiles, hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  MUSTER_LAUNCH(k_det_fold, dim3(n_tiles), dim3(BLOCK), 0, s, items, n_items, n_tiles);
  return hipGetLastError();
}

hipError_t launch_det_clear(JobState* const* states, int n_jobs, hipStream_t s) {
  if (n_jobs <= 0) return hipSuccess;
  MUSTER_LAUNCH(k_det_clear, dim3(n_jobs), dim3(64), 0, s, states, n_jobs);
  return hipGetLastError();
}

hipError_t launch_exp_bwd(const ExpBwdItem* items, int n_items, int n_tiles, int staged, bool reg,
                          hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  return reg ? launch_exp_bwd_<true>(items, n_items, n_tiles, staged, s)
             : launch_exp_bwd_<false>(items, n_items, n_tiles, staged, s);
}

hipError_t launch_unstage(const ExpBwdItem* items, int n_items, int n_tiles, hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  MUSTER_LAUNCH(k_unstage, dim3(n_tiles), dim3(BLOCK), 0, s, items, n_items, n_tiles);
  return hipGetLastError();
}

hipError_t launch_pull_combine(const PullItem* items, int n_items, int n_tiles, hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  MUSTER_LAUNCH(k_pull_combine, dim3(n_tiles), dim3(BLOCK), 0, s, items, n_items, n_tiles);
  return hipGetLastError();
}

hipError_t launch_compose_bwd(const ComposeBwdItem* items, int n_items, int n_tiles,
                              hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  MUSTER_LAUNCH(k_compose_bwd<false>, dim3(n_tiles), dim3(CB_NT), 0, s, items, n_items, n_tiles);
  return hipGetLastError();
}

hipError_t launch_compose_bwd_detmax(const ComposeBwdItem* items, int n_items, int n_tiles,
                                     hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  MUSTER_LAUNCH(k_compose_bwd<true>, dim3(n_tiles), dim3(CB_NT), 0, s, items, n_items, n_tiles);
  return hipGetLastError();
}

template <int R, int TY, int TX>
static void sim_launch(bool grad, const SimItem* items, int n_items, int n_tiles, int metric,
                       hipStream_t s) {
  if (grad)
    MUSTER_LAUNCH((k_sim_grad<R, TY, TX>), dim3(n_tiles), dim3(TY * TX), 0, s, items, n_items,
                       n_tiles);
  else
    MUSTER_LAUNCH((k_sim_stats<R, TY, TX>), dim3(n_tiles), dim3(TY * TX), 0, s, items,
                       n_items, n_tiles, metric);
}

template <int R>
static hipError_t sim_shape(bool grad, const SimItem* items, int n_items, int n_tiles, int metric,
                            int shape, hipStream_t s) {
  switch (shape) {
    case 0: sim_launch<R, 8, 32>(grad, items, n_items, n_tiles, metric, s); break;
    case 1: sim_launch<R, 16, 32>(grad, items, n_items, n_tiles, metric, s); break;
    case 2: sim_launch<R, 8, 64>(grad, items, n_items, n_tiles, metric, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

static hipError_t sim_window(bool grad, const SimItem* items, int n_items, int n_tiles, int window,
                             int metric, int shape, hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  switch (window) {
    case 3: return sim_shape<1>(grad, items, n_items, n_tiles, metric, shape, s);
    case 5: return sim_shape<2>(grad, items, n_items, n_tiles, metric, shape, s);
    case 7: return sim_shape<3>(grad, items, n_items, n_tiles, metric, shape, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_warp(const SimItem* items, int n_items, int n_tiles, hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  MUSTER_LAUNCH(k_warp, dim3(n_tiles), dim3(BLOCK), 0, s, items, n_items, n_tiles);
  return hipGetLastError();
}

hipError_t launch_sim_stats(const SimItem* items, int n_items, int n_tiles, int window, int metric,
                            int shape, hipStream_t s) {
  return sim_window(false, items, n_items, n_tiles, window, metric, shape, s);
}

hipError_t launch_sim_grad(const SimItem* items, int n_items, int n_tiles, int window, int shape,
                           hipStream_t s) {
  return sim_window(true, items, n_items, n_tiles, window, 0, shape, s);
}

hipError_t launch_adam(const AdamItem* items, int n_items, int n_tiles, hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  MUSTER_LAUNCH(k_adam, dim3(n_tiles), dim3(BLOCK), 0, s, items, n_items, n_tiles);
  return hipGetLastError();
}

hipError_t launch_smooth(const SmoothItem* items, int n_items, int n_tiles, int lds_floats,
                         hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  if (lds_floats <= 0 || lds_floats > SMOOTH_LDS) return hipErrorInvalidValue;
  MUSTER_LAUNCH(k_smooth, dim3(n_tiles), dim3(BLOCK), lds_floats * sizeof(float), s, items,
                     n_items, n_tiles);
  return hipGetLastError();
}

__global__ void k_pattern(float* __restrict__ p, int64_t n, int D, int H, int W, float off,
                          float amp, float phase) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t V = (int64_t)D * H * W;
  const int c = (int)(i / V);
  const int q = (int)(i - c * V);
  const int x = q % W, y = (q / W) % H, z = q / (W * H);
  p[i] = off + amp * sinf(0.21f * x + 0.13f * y + 0.17f * z + phase + 1.7f * c) *
                   cosf(0.05f * x - 0.09f * z + phase);
}

hipError_t launch_pattern(float* p, int64_t n, const int dims[3], float off, float amp,
                          float phase, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  MUSTER_LAUNCH(k_pattern, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, dims[0],
                     dims[1], dims[2], off, amp, phase);
  return hipGetLastError();
}

__global__ __launch_bounds__(BLOCK) void k_reg_ext(GridDims d, const float* __restrict__ f_,
                                                   const float* __restrict__ fprev_, float l2w,
                                                   float tsw, float inv_dp, float inv_ds,
                                                   double* out) {
  __shared__ double red[BLOCK / 64];
  const int V = d.D * d.H * d.W;
  const cgfloat* __restrict__ f = gp(f_);
  const cgfloat* __restrict__ fprev = fprev_ ? gp(fprev_) : nullptr;
  double acc = 0.0;
  for (int p = blockIdx.x * BLOCK + threadIdx.x; p < V; p += gridDim.x * BLOCK) {
    const float f0 = f[p], f1 = f[V + p], f2 = f[2 * V + p];
    acc += (double)l2w * ((double)f0 * f0 + (double)f1 * f1 + (double)f2 * f2);
    if (fprev) {
      const double a0 = (double)fprev[p] * inv_dp - (double)f0 * inv_ds;
      const double a1 = (double)fprev[V + p] * inv_dp - (double)f1 * inv_ds;
      const double a2 = (double)fprev[2 * V + p] * inv_dp - (double)f2 * inv_ds;
      acc += (double)tsw * (a0 * a0 + a1 * a1 + a2 * a2);
    }
  }
  const double tot = block_sum(acc, red);
  if (threadIdx.x == 0) unsafeAtomicAdd(out, tot);
}

hipError_t launch_reg_ext(GridDims d, const float* f, const float* fprev, float l2w, float tsw,
                          float inv_dp, float inv_ds, double* out, hipStream_t s) {
  const int V = d.D * d.H * d.W;
  if (V <= 0) return hipSuccess;
  const int blocks = ceil_div(V, BLOCK) < 2048 ? ceil_div(V, BLOCK) : 2048;
  MUSTER_LAUNCH(k_reg_ext, dim3(blocks), dim3(BLOCK), 0, s, d, f, fprev, l2w, tsw, inv_dp,
                     inv_ds, out);
  return hipGetLastError();
}

hipError_t launch_finish(JobState* const* states, int n_jobs, hipStream_t s) {
  if (n_jobs <= 0) return hipSuccess;
  MUSTER_LAUNCH(k_finish, dim3(ceil_div(n_jobs, 64)), dim3(64), 0, s, states, n_jobs);
  return hipGetLastError();
}

hipError_t launch_pool2(const PoolItem* items, int n_items, int n_tiles, hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  MUSTER_LAUNCH(k_pool2, dim3(n_tiles), dim3(BLOCK), 0, s, items, n_items, n_tiles);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Outputs and evaluation (Sec. 2.8): Jacobian determinants of Omega + U, and
// the sums from which Eu, the vector PCC and the regression slope follow.
// ---------------------------------------------------------------------------
__device__ __forceinline__ float fd_axis(const cgfloat* __restrict__ f, int p, int i, int n,
                                         int stride) {
  // central difference inside, one-sided at the two faces
  if (i == 0) return f[p + stride] - f[p];
  if (i == n - 1) return f[p] - f[p - stride];
  return 0.5f * (f[p + stride] - f[p - stride]);
}

__global__ __launch_bounds__(BLOCK) void k_jacobian_det(GridDims d, const float* __restrict__ U_,
                                                        float* __restrict__ out) {
  const int D = d.D, H = d.H, W = d.W, HW = H * W, V = D * HW;
  const cgfloat* __restrict__ U = gp(U_);
  for (int p = blockIdx.x * BLOCK + threadIdx.x; p < V; p += gridDim.x * BLOCK) {
    const int x = p % W, y = (p / W) % H, z = p / HW;
    float J[3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const cgfloat* __restrict__ f = U + (size_t)c * V;
      J[c][0] = fd_axis(f, p, z, D, HW) + (c == 0 ? 1.f : 0.f);
      J[c][1] = fd_axis(f, p, y, H, W) + (c == 1 ? 1.f : 0.f);
      J[c][2] = fd_axis(f, p, x, W, 1) + (c == 2 ? 1.f : 0.f);
    }
    gp(out)[p] = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                 J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                 J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
  }
}

// Sums over the region of interest (roi may be NULL: every voxel): count,
// sum |b - a|, sum a (3), sum b (3), sum a a^T (9), sum b a^T (9), sum b.b.
constexpr int FIELD_STATS = 27;

__global__ __launch_bounds__(BLOCK) void k_field_stats(int V, const float* __restrict__ a_,
                                                       const float* __restrict__ b_,
                                                       const unsigned char* __restrict__ roi,
                                                       double* __restrict__ out) {
  __shared__ double red[BLOCK / 64];
  const cgfloat* __restrict__ a = gp(a_);
  const cgfloat* __restrict__ b = gp(b_);
  double acc[FIELD_STATS];
#pragma unroll
  for (int k = 0; k < FIELD_STATS; ++k) acc[k] = 0.0;
  for (int p = blockIdx.x * BLOCK + threadIdx.x; p < V; p += gridDim.x * BLOCK) {
    if (roi && !roi[p]) continue;
    double av[3], bv[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      av[c] = a[(size_t)c * V + p];
      bv[c] = b[(size_t)c * V + p];
    }
    acc[0] += 1.0;
    acc[1] += sqrt((bv[0] - av[0]) * (bv[0] - av[0]) + (bv[1] - av[1]) * (bv[1] - av[1]) +
                   (bv[2] - av[2]) * (bv[2] - av[2]));
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      acc[2 + c] += av[c];
      acc[5 + c] += bv[c];
#pragma unroll
      for (int e = 0; e < 3; ++e) {
        acc[8 + 3 * c + e] += av[c] * av[e];
        acc[17 + 3 * c + e] += bv[c] * av[e];
      }
    }
    acc[26] += bv[0] * bv[0] + bv[1] * bv[1] + bv[2] * bv[2];
  }
#pragma unroll
  for (int k = 0; k < FIELD_STATS; ++k) {
    const double t = block_sum(acc[k], red);
    if (threadIdx.x == 0) unsafeAtomicAdd(out + k, t);
    __syncthreads();
  }
}

hipError_t launch_jacobian_det(GridDims d, const float* U, float* out, hipStream_t s) {
  const int V = d.D * d.H * d.W;
  if (V <= 0) return hipSuccess;
  const int blocks = ceil_div(V, BLOCK) < 4096 ? ceil_div(V, BLOCK) : 4096;
  MUSTER_LAUNCH(k_jacobian_det, dim3(blocks), dim3(BLOCK), 0, s, d, U, out);
  return hipGetLastError();
}

hipError_t launch_field_stats(int V, const float* a, const float* b, const unsigned char* roi,
                              double* out, hipStream_t s) {
  if (V <= 0) return hipSuccess;
  const int blocks = ceil_div(V, BLOCK) < 1024 ? ceil_div(V, BLOCK) : 1024;
  MUSTER_LAUNCH(k_field_stats, dim3(blocks), dim3(BLOCK), 0, s, V, a, b, roi, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Rigid adjustment (Sec. 2.5)
// ---------------------------------------------------------------------------
// sum_p G(p) and sum_p G(p) (p - c)^T over one pair's gradient, into the
// source session's accumulators.
__global__ __launch_bounds__(BLOCK) void k_rigid_grad(const RigidGradItem* __restrict__ items,
                                                      int n_items, int n_tiles) {
  __shared__ double red[BLOCK / 64][12];
  const int tile = blockIdx.x;
  const RigidGradItem it = items[find_item(items, n_items, tile)];
  const int D = it.D, H = it.H, W = it.W, V = D * H * W;
  const float cz = 0.5f * (D - 1), cy = 0.5f * (H - 1), cx = 0.5f * (W - 1);
  const cgfloat* __restrict__ G = gp(it.G);
  double acc[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = 0.0;
  const int q0 = (tile - it.tile0) * ELEM_PER_BLOCK;
  for (int k = threadIdx.x; k < ELEM_PER_BLOCK; k += BLOCK) {
    const int q = q0 + k;
    if (q >= V) break;
    const int x = q % W, y = (q / W) % H, z = q / (W * H);
    const double pz = (double)z - cz, py = (double)y - cy, px = (double)x - cx;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double g = G[(size_t)c * V + q];
      acc[c] += g;
      acc[3 + 3 * c] += g * pz;
      acc[4 + 3 * c] += g * py;
      acc[5 + 3 * c] += g * px;
    }
  }
#pragma unroll
  for (int k = 0; k < 12; ++k)
    for (int o = 32; o > 0; o >>= 1) acc[k] += __shfl_xor(acc[k], o);
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int k = 0; k < 12; ++k) red[threadIdx.x >> 6][k] = acc[k];
  __syncthreads();
  if (threadIdx.x < 12) {
    double t = 0.0;
    for (int w = 0; w < BLOCK / 64; ++w) t += red[w][threadIdx.x];
    double* dst = threadIdx.x < 3 ? &it.rg->gsum[threadIdx.x] : &it.rg->gmom[threadIdx.x - 3];
    unsafeAtomicAdd(dst, t);
  }
}

// One Adam step of a session's rigid parameters (PyTorch semantics, the
// job's schedule; the angles' step scaled by rot_lr), then the displacement
// the kernels apply, and the sums cleared for the next iteration.
__global__ void k_rigid_step(const RigidStepItem* __restrict__ items, int n_items) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_items) return;
  const RigidStepItem it = items[i];
  RigidState* rg = it.rg;
  const JobState* js = it.js;
  const int step = js->t + 1;
  const double lr = schedule_lr(js, step);
  const double bc1 = 1.0 - pow((double)js->b1, (double)step);
  const double bc2 = 1.0 - pow((double)js->b2, (double)step);
  float g[6];
  for (int k = 0; k < 3; ++k) {
    float dR[9];
    rigid_rotation(rg->theta, k, dR);
    double acc = 0.0;
    for (int e = 0; e < 9; ++e) acc += (double)dR[e] * rg->gmom[e];
    g[k] = (float)acc;
    g[3 + k] = (float)rg->gsum[k];
  }
  const float b1 = js->b1, b2 = js->b2, eps = js->eps;
  float prm[6] = {rg->theta[0], rg->theta[1], rg->theta[2], rg->t[0], rg->t[1], rg->t[2]};
  for (int k = 0; k < 6; ++k) {
    const float m = fmaf(1.f - b1, g[k] - rg->m[k], rg->m[k]);
    const float v = fmaf(1.f - b2, g[k] * g[k], rg->v[k] * b2);
    rg->m[k] = m;
    rg->v[k] = v;
    const float scale = k < 3 ? it.rot_lr : 1.f;
    const float den = sqrtf(v) / (float)sqrt(bc2) + eps;
    prm[k] -= (float)(lr * scale / bc1) * (m / den);
  }
  for (int k = 0; k < 3; ++k) {
    rg->theta[k] = prm[k];
    rg->t[k] = prm[3 + k];
  }
  float R[9];
  rigid_rotation(rg->theta, -1, R);
  for (int a = 0; a < 3; ++a) {
    float rc = 0.f;
    for (int b = 0; b < 3; ++b) {
      rg->A[3 * a + b] = R[3 * a + b] - (a == b ? 1.f : 0.f);
      rc += R[3 * a + b] * it.c[b];
    }
    rg->off[a] = it.c[a] + rg->t[a] - rc;
  }
  for (int k = 0; k < 3; ++k) rg->gsum[k] = 0.0;
  for (int k = 0; k < 9; ++k) rg->gmom[k] = 0.0;
}

__global__ __launch_bounds__(BLOCK) void k_add_rigid(GridDims d, float* __restrict__ f_,
                                                     const RigidState* __restrict__ rg) {
  const int V = d.D * d.H * d.W;
  gfloat* __restrict__ f = gp(f_);
  for (int p = blockIdx.x * BLOCK + threadIdx.x; p < V; p += gridDim.x * BLOCK) {
    const float x = (float)(p % d.W), y = (float)((p / d.W) % d.H), z = (float)(p / (d.W * d.H));
#pragma unroll
    for (int c = 0; c < 3; ++c)
      f[(size_t)c * V + p] += fmaf(rg->A[3 * c], z, fmaf(rg->A[3 * c + 1], y,
                                                         fmaf(rg->A[3 * c + 2], x, rg->off[c])));
  }
}

hipError_t launch_rigid_grad(const RigidGradItem* items, int n_items, int n_tiles, hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  MUSTER_LAUNCH(k_rigid_grad, dim3(n_tiles), dim3(BLOCK), 0, s, items, n_items, n_tiles);
  return hipGetLastError();
}

hipError_t launch_rigid_step(const RigidStepItem* items, int n_items, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  MUSTER_LAUNCH(k_rigid_step, dim3(ceil_div(n_items, 64)), dim3(64), 0, s, items, n_items);
  return hipGetLastError();
}

hipError_t launch_add_rigid(GridDims d, float* field, const RigidState* rg, hipStream_t s) {
  const int V = d.D * d.H * d.W;
  if (V <= 0) return hipSuccess;
  const int blocks = ceil_div(V, BLOCK) < 2048 ? ceil_div(V, BLOCK) : 2048;
  MUSTER_LAUNCH(k_add_rigid, dim3(blocks), dim3(BLOCK), 0, s, d, field, rg);
  return hipGetLastError();
}

hipError_t launch_upsample2_adj(const UpItem* items, int n_items, int n_tiles, hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  MUSTER_LAUNCH(k_upsample2_adj, dim3(n_tiles), dim3(BLOCK), 0, s, items, n_items, n_tiles);
  return hipGetLastError();
}

hipError_t launch_upsample2(const UpItem* items, int n_items, int n_tiles, hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  MUSTER_LAUNCH(k_upsample2, dim3(n_tiles), dim3(BLOCK), 0, s, items, n_items, n_tiles);
  return hipGetLastError();
}

hipError_t launch_adam_flat(int64_t n, float* x, const float* g, float* m, float* v, int t,
                            float lr, float b1, float b2, float eps, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const double bc1 = 1.0 - std::pow((double)b1, (double)t);
  const double bc2 = 1.0 - std::pow((double)b2, (double)t);
  const float step_size = (float)(lr / bc1);
  const float bc2s = (float)std::sqrt(bc2);
  const int64_t blocks = (n + BLOCK - 1) / BLOCK;
  MUSTER_LAUNCH(k_adam_flat, dim3((unsigned)blocks), dim3(BLOCK), 0, s, n, x, g, m, v,
                     step_size, bc2s, b1, b2, eps);
  return hipGetLastError();
}

hipError_t launch_reg(GridDims d, const float* phi, double* out, float* grad, hipStream_t s) {
  const int V = d.D * d.H * d.W;
  MUSTER_LAUNCH(k_reg, dim3(ceil_div(V, BLOCK)), dim3(BLOCK), 0, s, d.D, d.H, d.W, phi, out,
                     grad);
  return hipGetLastError();
}

// Scratch of the allocation-free similarity entry point (see
// NOALLOC_SCRATCH_BYTES).  Host code never passes the array's name to a
// kernel or a copy: only the address hipGetSymbolAddress returns for the
// current device.
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

hipError_t noalloc_scratch_address(int device, void** ptr) {
  static std::mutex mu;
  static std::map<int, void*> addr;
  std::lock_guard<std::mutex> lk(mu);
  auto it = addr.find(device);
  if (it != addr.end()) {
    *ptr = it->second;
    return hipSuccess;
  }
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!p) return hipErrorInvalidSymbol;
  addr.emplace(device, p);
  *ptr = p;
  return hipSuccess;
}

hipError_t launch_fill(float* p, int64_t n, float v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + BLOCK - 1) / BLOCK;
  MUSTER_LAUNCH(k_fill, dim3((unsigned)blocks), dim3(BLOCK), 0, s, p, n, v);
  return hipGetLastError();
}

}  // namespace muster
