// Per-cell passes: prior fill, robot-centric move, 3x3 normals, conv traversability.
//
// The stencils (normals, traversability) stage a 66 x 18 halo tile of heights
// and validity in LDS.  Each 256-thread workgroup then produces a 64 x 16
// output tile, four cells per thread (a 400 x 400 map: 7 x 25 = 175 tiles).
// The halo makes each height read about 1.16 times, the repeats mostly from
// the L2 that the neighbouring tile shares (see the unit order below).
// The batched launch computes normals and traversability from one staged tile.
#include "emx_kernels.h"

namespace emx {

namespace {

// ------------------------------------------------------- XCD-aware unit order
// Workgroups are dispatched to the chip's 8 XCDs (each with its own L2) in
// turn: workgroup b goes to XCD b % 8.  Stencil tiles share their halos with
// their neighbours, so each XCD is given a contiguous range of the n units
// (unit order is row-major over tiles), and neighbouring tiles meet in one L2.
constexpr int kXcds = 8;

// The unit of workgroup b in a launch of exactly n workgroups, a bijection of
// [0, n).
__device__ __forceinline__ int64_t xcd_unit(int64_t b, int64_t n) {
  const int64_t q = n / kXcds, r = n % kXcds;
  const int64_t x = b % kXcds;
  return x * q + (x < r ? x : r) + b / kXcds;
}

// The k-th unit of workgroup b in a persistent launch of g workgroups over n
// units, or -1 past its share.  With g a multiple of 8, the g/8 workgroups of
// XCD x walk that XCD's contiguous range in turn; otherwise units go round
// robin (b, b + g, ...).
__device__ __forceinline__ int64_t xcd_unit_k(int64_t b, int64_t g, int64_t n, int64_t k) {
  if (g % kXcds != 0) {
    const int64_t u = b + k * g;
    return u < n ? u : -1;
  }
  const int64_t q = n / kXcds, r = n % kXcds;
  const int64_t x = b % kXcds;
  const int64_t cnt = q + (x < r ? 1 : 0);
  const int64_t j = b / kXcds + k * (g / kXcds);
  return j < cnt ? x * q + (x < r ? x : r) + j : -1;
}

constexpr int kNTf = 256;

// ------------------------------------------------------------------ prior fill
struct FillArgs {
  Consts c;
  Layers L;
  int64_t cells;
  uint32_t* ctl;
  int nctl;
};

__global__ __launch_bounds__(kNTf) void k_fill_prior(FillArgs a) {
  const int64_t i = (int64_t)blockIdx.x * kNTf + threadIdx.x;
  if (i < a.nctl) a.ctl[i] = 0u;
  if (i >= a.cells) return;
  const float qnan = __builtin_nanf("");
  a.L.h[i] = a.c.h_init;
  a.L.v[i] = a.c.v_init;
  a.L.t[i] = 0;
  a.L.nx[i] = qnan;
  a.L.ny[i] = qnan;
  a.L.nz[i] = qnan;
  a.L.trav[i] = qnan;
  a.L.valid[i] = 0;
  a.L.mark[i] = 0;
  if (a.L.ub) a.L.ub[i] = INFINITY;
  for (int k = 0; k < kFxWords; ++k) a.L.fx[k * a.L.fxs + i] = 0u;
}

// ------------------------------------------------------------------------ move
// The ring has already turned (it.c holds the new origin); the cells that
// enter the map go back to the prior.  With a shift (sx, sy) they are the
// logical columns [nx - sx, nx) (sx > 0) or [0, -sx) (sx < 0) in every row,
// and the logical rows [ny - sy, ny) or [0, -sy) in every column; a shift of a
// whole side resets every cell.  One thread per cell: the column strip, then
// the row strip (their corner twice, with the same values).
struct Strips {
  int ncol, nrow;   // entering columns and rows
  bool all;         // every cell enters
  int64_t cells;    // threads needed
};

__host__ __device__ __forceinline__ Strips strips_of(const Item& it) {
  Strips s;
  const int ax = it.sx < 0 ? -it.sx : it.sx;
  const int ay = it.sy < 0 ? -it.sy : it.sy;
  s.ncol = ax < it.c.nx ? ax : it.c.nx;
  s.nrow = ay < it.c.ny ? ay : it.c.ny;
  s.all = s.ncol == it.c.nx || s.nrow == it.c.ny;
  s.cells = s.all ? (int64_t)it.c.nx * it.c.ny
                  : (int64_t)s.ncol * it.c.ny + (int64_t)s.nrow * it.c.nx;
  return s;
}

__device__ __forceinline__ void move_body(const Item& it, int64_t unit) {
  const Strips st = strips_of(it);
  const int64_t q = unit * kNTf + threadIdx.x;
  if (q >= st.cells) return;
  int ix, iy;
  if (st.all) {
    iy = (int)(q / it.c.nx);
    ix = (int)(q - (int64_t)iy * it.c.nx);
  } else if (q < (int64_t)st.ncol * it.c.ny) {
    iy = (int)(q / st.ncol);
    const int k = (int)(q - (int64_t)iy * st.ncol);
    ix = it.sx > 0 ? it.c.nx - st.ncol + k : k;
  } else {
    const int64_t q2 = q - (int64_t)st.ncol * it.c.ny;
    const int k = (int)(q2 / it.c.nx);
    ix = (int)(q2 - (int64_t)k * it.c.nx);
    iy = it.sy > 0 ? it.c.ny - st.nrow + k : k;
  }
  prior_cell(it.c, it.L, pcell(it.c, ix, iy));
}

// ------------------------------------------------------------ overlap clearance
// Valid cells within a horizontal radius of the robot whose height differs
// from the robot's by more than the threshold return to the prior.
__global__ __launch_bounds__(kNTf) void k_overlap(OverlapArgs a) {
  const int64_t i = (int64_t)blockIdx.x * kNTf + threadIdx.x;  // logical cell
  const int64_t C = (int64_t)a.c.nx * a.c.ny;
  if (i >= C) return;
  const int iy = (int)(i / a.c.nx);
  const int ix = (int)(i - (int64_t)iy * a.c.nx);
  const int64_t p = pcell(a.c, ix, iy);
  const float dx = ((float)ix + 0.5f) * a.r32 - a.rx;
  const float dy = ((float)iy + 0.5f) * a.r32 - a.ry;
  const bool hit = a.L.valid[p] && ((dx * dx + dy * dy) <= a.rad2) &&
                   (fabsf(a.L.h[p] - a.rz) > a.thr);
  if (hit) {
    a.L.h[p] = a.c.h_init;
    a.L.v[p] = a.c.v_init;
    a.L.valid[p] = 0;
  }
  if (a.out) a.out[i] = hit ? 1 : 0;
}

// ---------------------------------------------------------------- stencil tile
// Output tiles of 64 x 16 cells, four per thread.  Each row of the halo tile is
// read by one wave: lane l takes column x0 + l (one 256-byte load of heights
// and one 64-byte load of validity per row), two lanes take the halo columns.
constexpr int kSW = 64;            // output tile width (one wave per row)
constexpr int kSH = 16;            // output tile height
constexpr int kHW = kSW + 2;       // halo tile
constexpr int kHH = kSH + 2;
constexpr int kSWLog = 6;
constexpr int kSHLog = 4;

struct HaloTile {
  float h[kHH][kHW + 1];
  uint8_t ok[kHH][kHW + 2];
};

__device__ __forceinline__ void load_halo(HaloTile& s, const Consts& c, const Layers& L, int x0,
                                          int y0) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  for (int ly = wave; ly < kHH; ly += kNTf / 64) {
    const int gy = y0 - 1 + ly;
    const bool row = gy >= 0 && gy < c.ny;
    {  // body column lx = lane + 1
      const int gx = x0 + lane;
      float hv = 0.0f;
      uint8_t ok = 0;
      if (row && gx < c.nx) {
        const int64_t o = pcell(c, gx, gy);
        ok = L.valid[o];
        hv = L.h[o];
      }
      s.h[ly][lane + 1] = hv;
      s.ok[ly][lane + 1] = ok;
    }
    if (lane < 2) {  // halo columns lx = 0 and lx = kSW + 1
      const int lx = lane == 0 ? 0 : kSW + 1;
      const int gx = x0 - 1 + lx;
      float hv = 0.0f;
      uint8_t ok = 0;
      if (row && gx >= 0 && gx < c.nx) {
        const int64_t o = pcell(c, gx, gy);
        ok = L.valid[o];
        hv = L.h[o];
      }
      s.h[ly][lx] = hv;
      s.ok[ly][lx] = ok;
    }
  }
}

// the cell at halo position (lx, ly) is interior and its 3x3 window is valid
__device__ __forceinline__ bool window_ok(const HaloTile& s, const Consts& c, int gx, int gy,
                                          int lx, int ly) {
  if (gx < 1 || gy < 1 || gx > c.nx - 2 || gy > c.ny - 2) return false;
  bool ok = true;
#pragma unroll
  for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
    for (int dx = -1; dx <= 1; ++dx) ok = ok && (s.ok[ly + dy][lx + dx] != 0);
  return ok;
}

__device__ __forceinline__ void normal_at(const HaloTile& s, int lx, int ly, float inv6r,
                                          float& nx, float& ny, float& nz) {
  const float dxm = s.h[ly - 1][lx + 1] - s.h[ly - 1][lx - 1];
  const float dx0 = s.h[ly][lx + 1] - s.h[ly][lx - 1];
  const float dxp = s.h[ly + 1][lx + 1] - s.h[ly + 1][lx - 1];
  const float dym = s.h[ly + 1][lx - 1] - s.h[ly - 1][lx - 1];
  const float dy0 = s.h[ly + 1][lx] - s.h[ly - 1][lx];
  const float dyp = s.h[ly + 1][lx + 1] - s.h[ly - 1][lx + 1];
  const float gxv = ((dxm + dx0) + dxp) * inv6r;
  const float gyv = ((dym + dy0) + dyp) * inv6r;
  const float q = (gxv * gxv + gyv * gyv) + 1.0f;
  const float inv = 1.0f / sqrtf(q);
  nx = -gxv * inv;
  ny = -gyv * inv;
  nz = inv;
}

__device__ __forceinline__ float trav_at(const HaloTile& s, int lx, int ly, const float* sw) {
  float win[9];
#pragma unroll
  for (int dy = 0; dy < 3; ++dy)
#pragma unroll
    for (int dx = 0; dx < 3; ++dx) win[dy * 3 + dx] = s.h[ly - 1 + dy][lx - 1 + dx];
  float T = sw[88];
#pragma unroll
  for (int ch = 0; ch < 8; ++ch) {
    float acc = sw[72 + ch];
#pragma unroll
    for (int k = 0; k < 9; ++k) acc = fmaf(sw[ch * 9 + k], win[k], acc);
    T = fmaf(sw[80 + ch], fmaxf(acc, 0.0f), T);
  }
  return T;
}

// Normals and/or traversability of one output tile.
__device__ __forceinline__ void cells_body(const Item& it, int64_t unit, bool do_n, bool do_t) {
  __shared__ HaloTile s;
  __shared__ float sw[89];
  const int ux = blocks_of(it.c.nx, kSWLog);
  const int x0 = (int)(unit % ux) * kSW;
  const int y0 = (int)(unit / ux) * kSH;
  if (do_t && threadIdx.x < 89) sw[threadIdx.x] = it.w[threadIdx.x];
  load_halo(s, it.c, it.L, x0, y0);
  __syncthreads();
  const int tx = threadIdx.x & (kSW - 1);
  const int ty0 = threadIdx.x / kSW;
  const float qnan = __builtin_nanf("");
#pragma unroll
  for (int j = 0; j < kSH / (kNTf / kSW); ++j) {
    const int ty = ty0 + j * (kNTf / kSW);
    const int gx = x0 + tx;
    const int gy = y0 + ty;
    if (gx >= it.c.nx || gy >= it.c.ny) continue;
    const int lx = tx + 1;
    const int ly = ty + 1;
    const bool ok = window_ok(s, it.c, gx, gy, lx, ly);
    const int64_t o = pcell(it.c, gx, gy);
    if (do_n) {
      float nx = qnan, ny = qnan, nz = qnan;
      if (ok) normal_at(s, lx, ly, it.c.inv6r, nx, ny, nz);
      it.L.nx[o] = nx;
      it.L.ny[o] = ny;
      it.L.nz[o] = nz;
    }
    if (do_t) it.L.trav[o] = ok ? trav_at(s, lx, ly, sw) : qnan;
  }
}

// ---------------------------------------------------------------- launches
__global__ __launch_bounds__(kNTf) void k_move(Item it) { move_body(it, blockIdx.x); }
// One workgroup per output tile, each XCD taking a contiguous range of tiles.
__global__ __launch_bounds__(kNTf) void k_normals(Item it) {
  cells_body(it, xcd_unit(blockIdx.x, gridDim.x), true, false);
}
__global__ __launch_bounds__(kNTf) void k_trav(Item it) {
  cells_body(it, xcd_unit(blockIdx.x, gridDim.x), false, true);
}
// Both from one staged tile: the heights are read once.
__global__ __launch_bounds__(kNTf) void k_normals_trav(Item it) {
  cells_body(it, xcd_unit(blockIdx.x, gridDim.x), true, true);
}

// The batch's first launch: also zeroes the clearing queue counters, which
// the later setup launch increments.
__global__ __launch_bounds__(kNTf) void k_move_b(const Batch* bt) {
  if (blockIdx.x == 0 && threadIdx.x <= kSubQ)  // the sub-queues' and the overflow counter
    bt->items[0].cq.counter[threadIdx.x * kCtrStride] = 0u;
  const int64_t total = bt->off[kBMove][bt->n];
  for (int64_t w = blockIdx.x; w < total; w += gridDim.x) {
    const int i = batch_item(bt, kBMove, w);
    move_body(bt->items[i], w - bt->off[kBMove][i]);
  }
}

// Each XCD takes a contiguous range of the batch's tiles (xcd_unit_k).
__global__ __launch_bounds__(kNTf) void k_cells_b(const Batch* bt) {
  const int64_t total = bt->off[kBCells][bt->n];
  for (int64_t k = 0;; ++k) {
    const int64_t w = xcd_unit_k(blockIdx.x, gridDim.x, total, k);
    if (w < 0) break;
    const int i = batch_item(bt, kBCells, w);
    const Item& it = bt->items[i];
    cells_body(it, w - bt->off[kBCells][i], (it.stages & kStageNormals) != 0,
               (it.stages & kStageTrav) != 0);
    __syncthreads();
  }
}

}  // namespace

int64_t move_units(const Item& it) { return (strips_of(it).cells + kNTf - 1) / kNTf; }
int64_t cells_units(int nx, int ny) {
  return (int64_t)blocks_of(nx, kSWLog) * blocks_of(ny, kSHLog);
}

hipError_t launch_fill_prior(const Consts& c, const Layers& L, uint32_t* ctl, int nctl,
                             hipStream_t stream) {
  FillArgs a;
  a.c = c;
  a.L = L;
  a.cells = (int64_t)c.nx * c.ny;
  a.ctl = ctl;
  a.nctl = ctl ? nctl : 0;
  const int64_t n = a.cells > a.nctl ? a.cells : a.nctl;
  TimedLaunch tl("k_fill_prior", stream);
  hipLaunchKernelGGL(k_fill_prior, dim3((unsigned)((n + kNTf - 1) / kNTf)), dim3(kNTf), 0, stream,
                     a);
  return hipGetLastError();
}

hipError_t launch_overlap(const OverlapArgs& a, hipStream_t stream) {
  const int64_t C = (int64_t)a.c.nx * a.c.ny;
  TimedLaunch tl("k_overlap", stream);
  hipLaunchKernelGGL(k_overlap, dim3((unsigned)((C + kNTf - 1) / kNTf)), dim3(kNTf), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_move(const Item& it, hipStream_t stream) {
  const int64_t units = move_units(it);
  if (units == 0) return hipSuccess;
  TimedLaunch tl("k_move", stream);
  hipLaunchKernelGGL(k_move, dim3((unsigned)units), dim3(kNTf), 0, stream, it);
  return hipGetLastError();
}

hipError_t launch_normals(const Item& it, hipStream_t stream) {
  TimedLaunch tl("k_normals", stream);
  hipLaunchKernelGGL(k_normals, dim3((unsigned)cells_units(it.c.nx, it.c.ny)), dim3(kNTf), 0,
                     stream, it);
  return hipGetLastError();
}

hipError_t launch_trav(const Item& it, hipStream_t stream) {
  TimedLaunch tl("k_trav", stream);
  hipLaunchKernelGGL(k_trav, dim3((unsigned)cells_units(it.c.nx, it.c.ny)), dim3(kNTf), 0, stream,
                     it);
  return hipGetLastError();
}

hipError_t launch_normals_trav(const Item& it, hipStream_t stream) {
  TimedLaunch tl("k_normals_trav", stream);
  hipLaunchKernelGGL(k_normals_trav, dim3((unsigned)cells_units(it.c.nx, it.c.ny)), dim3(kNTf), 0,
                     stream, it);
  return hipGetLastError();
}

hipError_t launch_move_batch(const Batch* d_batch, int grid, hipStream_t stream) {
  {
    TimedLaunch tl("k_move_b", stream);
    hipLaunchKernelGGL(k_move_b, dim3(grid), dim3(kNTf), 0, stream, d_batch);
  }
  return hipGetLastError();
}

hipError_t launch_cells_batch(const Batch* d_batch, int grid, hipStream_t stream) {
  {
    TimedLaunch tl("k_cells_b", stream);
    hipLaunchKernelGGL(k_cells_b, dim3(grid), dim3(kNTf), 0, stream, d_batch);
  }
  return hipGetLastError();
}

}  // namespace emx
