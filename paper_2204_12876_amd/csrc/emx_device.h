// Device-side definitions shared by the emx kernels (gfx950, wave64).
//
// Every file of this library is compiled with -ffp-contract=off and correctly
// rounded float32 division/sqrt.  Kernels that take decisions (binning, gate,
// ray samples, clearing predicate) rely on that to reproduce the operation
// order the ABI documents exactly.
//
// Every kernel body works on one `Item`: one map with one frame.  It is called
// either from a plain launch (the Item passed by value, one workgroup per unit
// of work) or from a batched persistent launch that looks its units up in a
// device-resident `Batch` table.  The arithmetic is the same code either way,
// so a map's results are identical alone and in a batch.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace emx {

// Points per fusion work unit (one workgroup of pass 1, the wall counts and
// the drift partials).
constexpr int kChunk = 1024;
// Map tiles of 32 x 16 cells: pass 2 of the fusion visits only the tiles the
// frame touched (a 400 x 400 map has 13 x 25 = 325 tiles).
constexpr int kTileLogX = 5;
constexpr int kTileLogY = 4;
constexpr int kTileW = 1 << kTileLogX;
constexpr int kTileH = 1 << kTileLogY;
constexpr int kTileCells = kTileW * kTileH;

// Clearing queue: kSubQ sub-queues, each with its own counter kCtrStride words
// apart.
constexpr int kSubQ = 64;
constexpr int kCtrStride = 32;
constexpr int kOverCtr = kSubQ * kCtrStride;          // the overflow list's counter
constexpr int kCtrWords = (kSubQ + 1) * kCtrStride;   // one set of queue counters

// One buffer set of map layers, row-major [ny][nx].
// The map's layers, [ny][nx] each in the ring layout (pcell).
struct Layers {
  float* h;
  float* v;
  int32_t* t;
  float* nx;
  float* ny;
  float* nz;
  float* trav;
  uint8_t* valid;
  uint8_t* mark;  // the fusion's per-cell flags (kMark*); all zero between calls
  float* cmax;    // per logical block: max height over cells a ray may clear (transient)
  float* ub;      // upper bound of the ground height (+inf: none), or null
  float2* clr;    // per logical cell {h, or -inf if a ray may not clear it, v} (transient)
  uint64_t* fx;   // the fusion's fixed-point sums: kFxWords planes of fxs words, one word
                  // per physical cell each; all zero between calls
  int64_t fxs;    // plane stride in words
};

// Fixed-point sums of a cell, one word in each plane.  A value x enters as the
// integer X = round(x * 2^S) (S: the item's shift for that sum), split as
// X = hi * 2^32 + lo with 0 <= lo < 2^32; the hi and lo parts are summed in
// separate words (hi as two's complement).  Integer addition is associative,
// so the sums do not depend on the order of the atomics that form them: the
// fused result is the same in every run, alone or batched.
enum FxWord { kFxWhi = 0, kFxWlo, kFxZhi, kFxZlo, kFxWords };  // sum 1/sp2; sum rz/sp2

// Clearing prunes samples by square blocks of 8 x 8 cells: one cell per lane
// of the wave that computes a block's maximum (the setup relies on it).  The maxima are read through
// the caches, so their count is not bounded by LDS.
// The setup's block role gives a wave 1 block, or 4 on maps of at least 4096
// blocks, where more work per wave beats more waves.
constexpr int kMaxBlocksPerWave = 4;
__host__ __device__ inline int blocks_of(int n, int b) { return (n + (1 << b) - 1) >> b; }
__host__ __device__ inline int block_log_of(int nx, int ny) {
  (void)nx;
  (void)ny;
  return 3;
}

// Float32 constants derived once on the host from emx_params.
struct Consts {
  float inv_r;     // float32(1/r)
  float rmin2;     // float32(min_range^2)
  float k2;        // float32(gate_k^2)
  float alpha;     // noise_alpha
  float an2;       // float32(clear_normal_alpha^2)
  float inv_step;  // float32(1/ray_step)
  float inv6r;     // float32(1/(6 r))
  float h_init;
  float v_init;
  float nxf, nyf;  // nx, ny as float (exact)
  int nx, ny;
  int32_t tau;     // clear_min_age_ms
  float var_t;     // time variance per fusion, 0 = off
  int32_t wall;    // wall/edge rule threshold, 0 = off
  int32_t excl_on;     // exclusion area on
  float excl_slope;    // float32(tan(theta_a))
  float excl_b, excl_c, excl_d;
  float var_o;     // outlier variance per fusion, 0 = off
  int ox, oy;      // ring origin: physical column and row of logical cell (0, 0)
};

// Sensor -> map-local transform, float32.
struct Pose32 {
  float R[9];
  float t[3];
};

struct FuseScratch {
  uint32_t* tcnt;       // [T] nonzero if pass 1 added to a cell of the tile; part of the
                        // map state, zero between calls (pass 2 resets it)
  uint32_t* count;      // [nx * ny] the frame's valid points per cell (wall rule), or null
};

// Where a clearing setup queues its ray segments.  A ray is named by its
// global index ray_base + i (i: its point in the item's frame); the march
// rebuilds the ray from the point, in the same float32 operations.
struct ClearQueue {
  uint2* queue;       // kSubQ sub-queues of qcap (ray, k_start << 8 | count) entries
  uint4* over;        // rays that did not fit their sub-queue: (ray, k0, k1, 0)
  uint32_t* counter;  // kSubQ sub-queue counters and the overflow counter (at
                      // kOverCtr), kCtrStride apart; zero on entry
  uint32_t* counter_next;  // the next call's counter set, zeroed by this call's
                           // setup (plain calls alternate two sets), or null
  int64_t qcap;       // entries per sub-queue
  int seg;            // samples per queued segment (1..255)
};

// Queue capacity: on average kQueueSamplesPerRay samples per point fit.
constexpr int kQueueSamplesPerRay = 128;

// Stages of one frame, in pipeline order.
constexpr uint32_t kStageMove = 1u;
constexpr uint32_t kStageFuse = 2u;
constexpr uint32_t kStageClear = 4u;
constexpr uint32_t kStageNormals = 8u;
constexpr uint32_t kStageTrav = 16u;

// One map with one frame: everything a kernel body reads.
struct Item {
  Consts c;
  Pose32 P;
  Layers L;     // the map's layers (ring layout; c holds the origin after any move)
  const float* x;
  const float* y;
  const float* z;
  int64_t n;
  int32_t t_now;
  int sx, sy;   // move shift in cells (the cells entering the map)
  uint32_t stages;
  const float* w;  // traversability weights (89)
  int32_t* out_cell;
  uint8_t* out_accept;
  uint8_t* out_cleared;
  FuseScratch fs;
  ClearQueue cq;
  int64_t ray_base;  // this item's first ray in cq
  int fxw, fxz;      // fixed-point shifts S of the sums of 1/sp2 and rz/sp2 (FxWord)
  int tiles_x, T, B;
  int bl, bx, by, nb, nprep;
  int bpw;           // clearing blocks per wave in the setup's block role
  int32_t index;     // position in its batch
};

// Batched launches: a device-resident table of items and, per stage, the
// prefix of work units over the items.
constexpr int kMaxItems = 64;
// kBZero, kBCount: the wall/edge rule's per-cell counts (zeroed, then
// counted); kBVar: the per-cell time and outlier variance after the fusion.
enum BatchStage { kBMove = 0, kBZero, kBCount, kBChunk, kBTile, kBVar, kBSetup, kBCells, kBNum };

// Only the header and the first n items are uploaded for a batch of n.
struct Batch {
  int n;
  int64_t off[kBNum][kMaxItems + 1];
  int64_t rays[kMaxItems + 1];  // prefix of the items' clearing rays (ray_base)
  Item items[kMaxItems];
};

struct PointEval {
  float xm, ym, zm, d2, sp2;
  float rz;  // the rotated point's height (zm before the translation is added)
  bool valid;
};

// Transform, range and noise of one sensor-frame point, in the ABI's order.
__device__ __forceinline__ PointEval eval_point(const Pose32& P, const Consts& c, float xs,
                                                float ys, float zs) {
  PointEval e;
  e.xm = ((P.R[0] * xs + P.R[1] * ys) + P.R[2] * zs) + P.t[0];
  e.ym = ((P.R[3] * xs + P.R[4] * ys) + P.R[5] * zs) + P.t[1];
  e.rz = (P.R[6] * xs + P.R[7] * ys) + P.R[8] * zs;
  e.zm = e.rz + P.t[2];
  e.d2 = (xs * xs + ys * ys) + zs * zs;
  e.sp2 = c.alpha * e.d2;
  e.valid = isfinite(xs) && isfinite(ys) && isfinite(zs) && isfinite(e.d2) &&
            (e.d2 >= c.rmin2) && isfinite(e.sp2);
  return e;
}

// Exclusion area: the point lies above the line around the sensor origin
// (Pose32::t), in the ABI's float32 order.
__device__ __forceinline__ bool excluded_point(const Pose32& P, const Consts& c,
                                               const PointEval& e) {
  const float dxr = e.xm - P.t[0];
  const float dyr = e.ym - P.t[1];
  const float rho = sqrtf(dxr * dxr + dyr * dyr);
  const float eup = e.zm - P.t[2];
  const float line = fminf(c.excl_b + c.excl_slope * fmaxf(rho - c.excl_c, 0.0f), c.excl_d);
  return eup > line;
}

// Mark layer bits between the fusion's passes and its per-cell pass.
constexpr uint8_t kMarkUpdated = 1;   // pass 2 updated the cell
constexpr uint8_t kMarkOutlier = 2;   // a gate-rejected point fell in the (valid) cell

// Half-open binning of map-local float32 coordinates; false outside.
__device__ __forceinline__ bool bin_xy(float xm, float ym, const Consts& c, int& ix, int& iy) {
  const float fx = xm * c.inv_r;
  const float fy = ym * c.inv_r;
  if (!(fx >= 0.0f && fx < c.nxf && fy >= 0.0f && fy < c.nyf)) return false;
  ix = (int)floorf(fx);
  iy = (int)floorf(fy);
  return true;
}

// ---------------------------------------------------------------- ring layout
// The map is stored as a ring (a circular buffer in both axes): logical cell
// (ix, iy) lives at physical cell pcell(c, ix, iy), with the origin (ox, oy)
// the physical column and row of logical (0, 0).  A move turns the ring
// instead of copying the layers; only the cells that enter the map are reset.
__host__ __device__ __forceinline__ int64_t pcell(const Consts& c, int ix, int iy) {
  int px = ix + c.ox;
  px -= (px >= c.nx) ? c.nx : 0;
  int py = iy + c.oy;
  py -= (py >= c.ny) ? c.ny : 0;
  return (int64_t)py * c.nx + px;
}

// Physical cell o back to the prior: no estimate, no normal or
// traversability, no bound; the mark is cleared.
__device__ __forceinline__ void prior_cell(const Consts& c, const Layers& L, int64_t o) {
  const float qnan = __builtin_nanf("");
  L.h[o] = c.h_init;
  L.v[o] = c.v_init;
  L.t[o] = 0;
  L.nx[o] = qnan;
  L.ny[o] = qnan;
  L.nz[o] = qnan;
  L.trav[o] = qnan;
  L.valid[o] = 0;
  L.mark[o] = 0;
  if (L.ub) L.ub[o] = INFINITY;
}

// ---------------------------------------------------------------- block scans
// Exclusive prefix sum of one int per thread over a block of NT threads.
// `sm` holds NT/64 ints.  Contains two barriers; every thread must call it.
template <int NT>
__device__ __forceinline__ int block_exclusive_sum(int v, int& total, int* sm) {
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) sm[wid] = x;
  __syncthreads();
  int pre = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) {
    const int s = sm[w];
    pre += (w < wid) ? s : 0;
    tot += s;
  }
  __syncthreads();
  total = tot;
  return pre + x - v;
}

// Minimum of one uint32 per thread over a block of NT threads.  `sm` holds
// NT/64 words.  Contains two barriers; every thread must call it.
template <int NT>
__device__ __forceinline__ uint32_t block_min_u32(uint32_t v, uint32_t* sm) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const uint32_t y = (uint32_t)__shfl_xor((int)v, o, 64);
    v = y < v ? y : v;
  }
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = v;
  __syncthreads();
  uint32_t r = sm[0];
#pragma unroll
  for (int w = 1; w < NT / 64; ++w) r = sm[w] < r ? sm[w] : r;
  __syncthreads();
  return r;
}

// ------------------------------------------------------------- batched units
// Item holding global unit w of `stage`: the last item whose prefix is <= w.
__device__ __forceinline__ int batch_item(const Batch* bt, int stage, int64_t w) {
  int lo = 0, hi = bt->n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (bt->off[stage][mid] <= w) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

}  // namespace emx
