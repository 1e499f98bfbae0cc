// Height fusion (Sec. II-C, Eq. 1 and Eq. 2) with exact integer sums and no
// float atomics.
//
// Eq. 2 fuses a cell's accepted points through two sums, of 1/sp2 and of
// zm/sp2.  Both are formed in fixed point: a term x enters as the integer
// round(x * 2^S), held as hi * 2^32 + lo (FxWord), with one shift S per sum and
// frame chosen on the host so that no sum can overflow (fuse_fixed_shifts).
// Integer addition is associative, so the sums come out the same whatever the
// order the additions land in: results are bitwise identical from run to run,
// alone or batched, whatever the grid shape.
//
// Pass 1, chunk body: one workgroup per chunk of kChunk points, kPerThread
// points per thread, consecutive points in consecutive lanes.
//   - Takes the per-point decisions: transform, range, bin, exclusion area,
//     wall/edge rule, and the Mahalanobis gate against the frame-start prior.
//   - Converts an accepted point's 1/sp2 and rz/sp2 to fixed point (rz: the
//     rotated point's height, zm = rz + tz; tz * sum 1/sp2 is added back in
//     pass 2, which keeps the terms independent of the sensor's height).
//   - Sums each run of consecutive lanes in one cell within the wave
//     (sensors emit points in scan order, so most runs span several points),
//     then each cell's runs in an LDS table for the chunk, and adds the
//     chunk's sums to the cell's words (FxWord planes) with integer atomics;
//     the cell's tile is flagged.
// Pass 2, tile body: per 32 x 16-cell tile of the physical layout, a
// workgroup with one thread per cell (plain calls) or one wave with eight
// cells per lane (batches).  An unflagged tile returns after one load;
// otherwise the flag is reset, and each cell with a nonzero sum converts its
// sums back to floating point, applies the information-form update once and
// resets its words to zero for the next call.
#include <math.h>

#include "emx_kernels.h"

namespace emx {

namespace {

constexpr int kNT1 = 256;                   // pass-1 threads
constexpr int kPerThread = kChunk / kNT1;   // points per thread
constexpr uint32_t kNoCell = 0xFFFFFFFFu;   // lanes without an accepted point

// The integer X = round(x * 2^S) of a finite float32 x (ties to even), as
// X = hi * 2^32 + lo with 0 <= lo < 2^32.  Exact for |x| * 2^S < 2^94, which
// the choice of S guarantees: x = m * 2^(e - 150) with the 24-bit significand
// m, so X is m shifted by e - 150 + S bits, in two words.
__device__ __forceinline__ void fx_split(float x, int S, int64_t& hi, uint64_t& lo) {
  const uint32_t b = __float_as_uint(x);
  const uint32_t ex = (b >> 23) & 255u;
  const uint64_t m = (uint64_t)((b & 0x7FFFFFu) | (ex ? 0x800000u : 0u));
  const int sh = (int)(ex ? ex : 1u) - 150 + S;
  uint64_t h = 0, l = 0;
  if (sh >= 32) {
    h = m << (sh - 32);  // X < 2^94: h < 2^62
  } else if (sh >= 0) {
    const uint64_t v = m << sh;  // < 2^56
    h = v >> 32;
    l = v & 0xFFFFFFFFull;
  } else if (sh >= -24) {
    const int r = -sh;
    const uint64_t q = m >> r;
    const uint64_t rem = m & ((1ull << r) - 1ull);
    const uint64_t half = 1ull << (r - 1);
    l = q + ((rem > half || (rem == half && (q & 1ull))) ? 1ull : 0ull);
  }  // else |x| * 2^S < 2^-1: rounds to zero
  if (b >> 31) {  // -(h * 2^32 + l) with the low word kept non-negative
    hi = -(int64_t)h - (l != 0 ? 1 : 0);
    lo = (0x100000000ull - l) & 0xFFFFFFFFull;
  } else {
    hi = (int64_t)h;
    lo = l;
  }
}

// (hi * 2^32 + lo) * 2^-S in float64.
__device__ __forceinline__ double fx_value(int64_t hi, uint64_t lo, int S) {
  return ldexp((double)hi * 4294967296.0 + (double)lo, -S);
}

// ------------------------------------------------------------------ pass 1
// Inclusive sums over each run of equal keys in the wave, in place: after the
// call a lane holds the sum of its run's lanes up to and including itself.
// Combining (flag, value) pairs: earlier (+) later = later.flag ? later :
// earlier + later, where a flag marks a run's first lane.
__device__ __forceinline__ void run_sums(uint32_t key, int64_t& whi, uint64_t& wlo,
                                         int64_t& zhi, uint64_t& zlo) {
  const int lane = threadIdx.x & 63;
  const uint32_t prev = (uint32_t)__shfl_up((int)key, 1, 64);
  int f = (lane == 0 || prev != key) ? 1 : 0;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int pf = __shfl_up(f, o, 64);
    const int64_t a = __shfl_up(whi, o, 64);
    const uint64_t b = __shfl_up(wlo, o, 64);
    const int64_t c = __shfl_up(zhi, o, 64);
    const uint64_t d = __shfl_up(zlo, o, 64);
    if (lane >= o) {
      if (!f) {
        whi += a;
        wlo += b;
        zhi += c;
        zlo += d;
      }
      f |= pf;
    }
  }
}

// A chunk's sums are gathered per cell in an LDS table before they go to the
// map: kAggSlots slots of (cell + 1, four words), open addressing with at most
// kAggProbes probes.  A run that finds no slot adds to the map directly.
constexpr int kAggSlots = 512;
constexpr int kAggProbes = 8;

struct AggTable {
  uint32_t key[kAggSlots];                   // physical cell + 1; 0 = free
  unsigned long long v[kFxWords][kAggSlots];  // the words, as in the map's planes
};

__device__ __forceinline__ void add_to_map(const Item& it, uint32_t cell, const uint64_t (&v)[4]) {
#pragma unroll
  for (int k = 0; k < kFxWords; ++k)
    if (v[k]) atomicAdd((unsigned long long*)(it.L.fx + k * it.L.fxs + cell), v[k]);
}

__device__ __forceinline__ uint32_t tile_of_cell(const Item& it, uint32_t cell) {
  const uint32_t py = cell / (uint32_t)it.c.nx;
  const uint32_t px = cell - py * (uint32_t)it.c.nx;
  return (py >> kTileLogY) * (uint32_t)it.tiles_x + (px >> kTileLogX);
}

// Zeroes the table (every thread of the block; the caller synchronises).
__device__ __forceinline__ void agg_clear(AggTable& t) {
  for (int s = threadIdx.x; s < kAggSlots; s += kNT1) {
    t.key[s] = 0u;
#pragma unroll
    for (int k = 0; k < kFxWords; ++k) t.v[k][s] = 0ull;
  }
}

// One chunk of kChunk points: point chunk * kChunk + j * kNT1 + thread of
// step j.  Every lane runs the wave's run sums, also past the frame's end.
// On entry the table is zero; it is zero again on return.
__device__ __forceinline__ void chunk_body(const Item& it, int64_t chunk, AggTable& tab) {
  const int lane = threadIdx.x & 63;
  // the thread's kPerThread points, every load issued before any is used:
  // first the coordinates, then the prior of each point's cell
  PointEval e[kPerThread];
  int64_t pc[kPerThread];
  int cell[kPerThread];
  bool in[kPerThread], gated[kPerThread];
  float h0[kPerThread], v0[kPerThread];
  uint32_t cnt[kPerThread];
  uint8_t vd[kPerThread];
  {
    float xs[kPerThread], ys[kPerThread], zs[kPerThread];
#pragma unroll
    for (int j = 0; j < kPerThread; ++j) {
      const int64_t i = chunk * kChunk + j * kNT1 + threadIdx.x;
      in[j] = i < it.n;
      xs[j] = in[j] ? it.x[i] : 0.0f;
      ys[j] = in[j] ? it.y[i] : 0.0f;
      zs[j] = in[j] ? it.z[i] : 0.0f;
    }
#pragma unroll
    for (int j = 0; j < kPerThread; ++j) {
      e[j] = eval_point(it.P, it.c, xs[j], ys[j], zs[j]);
      int ix = 0, iy = 0;
      const bool inmap = in[j] && e[j].valid && bin_xy(e[j].xm, e[j].ym, it.c, ix, iy);
      cell[j] = inmap ? iy * it.c.nx + ix : -1;
      pc[j] = inmap ? pcell(it.c, ix, iy) : 0;
      // points of the exclusion area are ignored
      gated[j] = inmap && (!it.c.excl_on || !excluded_point(it.P, it.c, e[j]));
      h0[j] = 0.0f;
      v0[j] = 0.0f;
      cnt[j] = 0u;
      vd[j] = 0;
      if (gated[j]) {
        h0[j] = it.L.h[pc[j]];
        v0[j] = it.L.v[pc[j]];
        if (it.fs.count) cnt[j] = it.fs.count[pc[j]];
        if (it.fs.count || it.c.var_o != 0.0f) vd[j] = it.L.valid[pc[j]];
      }
    }
  }
#pragma unroll
  for (int j = 0; j < kPerThread; ++j) {
    const int64_t i = chunk * kChunk + j * kNT1 + threadIdx.x;
    uint32_t key = kNoCell;  // the accepted point's physical cell
    float w = 0.0f, u = 0.0f;
    bool acc = false;
    if (gated[j]) {
      const float d = e[j].zm - h0[j];
      const bool inside = (d * d) <= (it.c.k2 * (v0[j] + e[j].sp2));
      // wall/edge rule: in a crowded cell that holds an estimate, points
      // below the estimate are ignored (before the gate)
      const bool walled =
          it.fs.count && e[j].zm < h0[j] && cnt[j] > (uint32_t)it.c.wall && vd[j];
      acc = inside && !walled;
      // a gate-rejected point in a cell with an estimate flags the cell for
      // the outlier variance (a plain store: every writer stores 2)
      if (it.c.var_o != 0.0f && !inside && !walled && vd[j]) it.L.mark[pc[j]] = kMarkOutlier;
      if (acc) {
        key = (uint32_t)pc[j];
        w = 1.0f / e[j].sp2;
        u = w * e[j].rz;
      }
    }
    if (in[j]) {
      if (it.out_cell) it.out_cell[i] = cell[j];
      if (it.out_accept) it.out_accept[i] = acc ? 1 : 0;
    }
    int64_t whi = 0, zhi = 0;
    uint64_t wlo = 0, zlo = 0;
    if (key != kNoCell) {
      fx_split(w, it.fxw, whi, wlo);
      if (whi == 0 && wlo == 0) wlo = 1;  // an accepted point adds at least one unit
      fx_split(u, it.fxz, zhi, zlo);
    }
    run_sums(key, whi, wlo, zhi, zlo);
    const uint32_t next = (uint32_t)__shfl_down((int)key, 1, 64);
    if (key != kNoCell && (lane == 63 || next != key)) {
      // the run's sums into the chunk's table, or straight to the map
      const uint64_t v[4] = {(uint64_t)whi, wlo, (uint64_t)zhi, zlo};
      uint32_t h = (key * 2654435761u) >> (32 - 9);
      static_assert(kAggSlots == 1 << 9, "the hash yields 9 bits");
      bool placed = false;
      for (int p = 0; p < kAggProbes; ++p) {
        const uint32_t prev = atomicCAS(&tab.key[h], 0u, key + 1u);
        if (prev == 0u || prev == key + 1u) {
#pragma unroll
          for (int k = 0; k < kFxWords; ++k)
            if (v[k]) atomicAdd(&tab.v[k][h], (unsigned long long)v[k]);
          placed = true;
          break;
        }
        h = (h + 1u) & (kAggSlots - 1);
      }
      if (!placed) {
        add_to_map(it, key, v);
        it.fs.tcnt[tile_of_cell(it, key)] = 1u;
      }
    }
  }
  __syncthreads();
  // the table's cells to the map; the table back to zero
  for (int s = threadIdx.x; s < kAggSlots; s += kNT1) {
    const uint32_t k1 = tab.key[s];
    if (k1 == 0u) continue;
    const uint32_t cell = k1 - 1u;
    const uint64_t v[4] = {tab.v[0][s], tab.v[1][s], tab.v[2][s], tab.v[3][s]};
    add_to_map(it, cell, v);
    it.fs.tcnt[tile_of_cell(it, cell)] = 1u;
    tab.key[s] = 0u;
#pragma unroll
    for (int k = 0; k < kFxWords; ++k) tab.v[k][s] = 0ull;
  }
  __syncthreads();
}

// ------------------------------------------------------------------ pass 2
constexpr int kNT2 = kTileCells;               // plain pass 2: one thread per cell of the tile
constexpr int kNT2b = 256;                     // batched pass 2: one wave per tile
constexpr int kTilesPerGroup = kNT2b / 64;
constexpr int kCellsPerLane = kTileCells / 64;  // 8: lane l owns cells l, l + 64, ...
constexpr int kHalf = kCellsPerLane / 2;

// Information-form update of physical cell `cell` from its sums (Σw's words
// whi, wlo given, not both zero); the sums are reset to zero.
__device__ __forceinline__ void update_cell(const Item& it, int64_t cell, int64_t whi,
                                            uint64_t wlo, int64_t zhi, uint64_t zlo, float h0,
                                            float v0) {
  uint64_t* f = it.L.fx + cell;
  const int64_t fs = it.L.fxs;
#pragma unroll
  for (int k = 0; k < kFxWords; ++k) f[k * fs] = 0u;
  const double sw = fx_value(whi, wlo, it.fxw);
  const double srz = fx_value(zhi, zlo, it.fxz);
  const float acc_w = (float)sw;
  const float acc_wz = (float)(srz + (double)it.P.t[2] * sw);
  const float W = (1.0f / v0) + acc_w;
  const float v1 = 1.0f / W;
  const float h1 = ((h0 / v0) + acc_wz) * v1;
  it.L.h[cell] = h1;
  it.L.v[cell] = v1;
  it.L.t[cell] = it.t_now;
  it.L.valid[cell] = 1;
  // updated: no time variance (the owning thread keeps pass 1's outlier flag)
  if (it.c.var_t != 0.0f) it.L.mark[cell] = it.L.mark[cell] | kMarkUpdated;
}

// Tile t, by a workgroup of kNT2 threads, one cell each: the plain call's
// form, where a single frame's tiles are few and each cell's loads should be
// in flight at once.
__device__ __forceinline__ void tile_body_group(const Item& it, int64_t t) {
  if (it.fs.tcnt[t] == 0u) return;  // uniform: the frame added to no cell of the tile
  __syncthreads();                  // every thread has read the flag
  if (threadIdx.x == 0) it.fs.tcnt[t] = 0u;  // zero again for the next call
  const int l = threadIdx.x;
  const int tx = (int)(t % it.tiles_x);
  const int ty = (int)(t / it.tiles_x);
  // the owned cell, physical (tiles cover the ring layout as stored)
  const int px = (tx << kTileLogX) + (l & (kTileW - 1));
  const int py = (ty << kTileLogY) + (l >> kTileLogX);
  if (px >= it.c.nx || py >= it.c.ny) return;
  const int64_t cell = (int64_t)py * it.c.nx + px;
  const int64_t fs = it.L.fxs;
  const int64_t whi = (int64_t)it.L.fx[kFxWhi * fs + cell];
  const uint64_t wlo = it.L.fx[kFxWlo * fs + cell];
  if (whi == 0 && wlo == 0) return;  // no accepted point: every term is positive
  update_cell(it, cell, whi, wlo, (int64_t)it.L.fx[kFxZhi * fs + cell],
              it.L.fx[kFxZlo * fs + cell], it.L.h[cell], it.L.v[cell]);
}

// Tile t, by one wave: lane l takes cells l + 64 i of the tile (two rows of 32
// per step), in two halves of kHalf cells, each half's loads issued together.
// The batched form: a batch holds tens of thousands of tiles, many untouched,
// so a workgroup's waves take one tile each and an untouched tile costs one
// wave one load.  The same update_cell as the plain form: the same bits.
__device__ __forceinline__ void tile_body_wave(const Item& it, int64_t t) {
  const int lane = threadIdx.x & 63;
  if (it.fs.tcnt[t] == 0u) return;  // wave-uniform: the frame added to no cell of the tile
  // the flag's load has completed for the whole wave (the branch used it)
  if (lane == 0) it.fs.tcnt[t] = 0u;  // zero again for the next call
  const int tx = (int)(t % it.tiles_x);
  const int ty = (int)(t / it.tiles_x);
  const int64_t fs = it.L.fxs;
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    int64_t cell[kHalf];
    bool in[kHalf];
    int64_t whi[kHalf];
    uint64_t wlo[kHalf];
#pragma unroll
    for (int i = 0; i < kHalf; ++i) {
      const int c = lane + 64 * (half * kHalf + i);
      // the cell, physical (tiles cover the ring layout as stored)
      const int px = (tx << kTileLogX) + (c & (kTileW - 1));
      const int py = (ty << kTileLogY) + (c >> kTileLogX);
      in[i] = px < it.c.nx && py < it.c.ny;
      cell[i] = in[i] ? (int64_t)py * it.c.nx + px : 0;
      whi[i] = 0;
      wlo[i] = 0;
      if (in[i]) {
        whi[i] = (int64_t)it.L.fx[kFxWhi * fs + cell[i]];
        wlo[i] = it.L.fx[kFxWlo * fs + cell[i]];
      }
    }
    // cells with an accepted point (every term is positive): the rest of
    // their sums and their prior, all loads issued before any is used
    bool hit[kHalf];
    int64_t zhi[kHalf];
    uint64_t zlo[kHalf];
    float h0[kHalf], v0[kHalf];
#pragma unroll
    for (int i = 0; i < kHalf; ++i) {
      hit[i] = in[i] && (whi[i] != 0 || wlo[i] != 0);
      zhi[i] = 0;
      zlo[i] = 0;
      h0[i] = 0.0f;
      v0[i] = 1.0f;
      if (hit[i]) {
        zhi[i] = (int64_t)it.L.fx[kFxZhi * fs + cell[i]];
        zlo[i] = it.L.fx[kFxZlo * fs + cell[i]];
        h0[i] = it.L.h[cell[i]];
        v0[i] = it.L.v[cell[i]];
      }
    }
#pragma unroll
    for (int i = 0; i < kHalf; ++i)
      if (hit[i]) update_cell(it, cell[i], whi[i], wlo[i], zhi[i], zlo[i], h0[i], v0[i]);
  }
}

// ------------------------------------------------------- wall rule: counts
// The frame's valid in-map points per cell.  Near the sensor thousands of
// points share a cell, and global atomics on one address serialise, so each
// workgroup first counts its chunk in an LDS hash table (open addressing,
// twice as many slots as points: a free slot always exists) and then adds one
// count per distinct cell.  Integer sums do not depend on their order.  The
// counts are zeroed by the launch before.
constexpr int kCountSlotsLog = 11;
constexpr int kCountSlots = 1 << kCountSlotsLog;
static_assert(kCountSlots >= 2 * kChunk, "the table must keep a free slot");

__device__ __forceinline__ void count_body(const Item& it, int64_t chunk) {
  __shared__ uint32_t s_key[kCountSlots];  // cell + 1, 0 = empty
  __shared__ uint32_t s_cnt[kCountSlots];
  for (int j = threadIdx.x; j < kCountSlots; j += kNT1) {
    s_key[j] = 0u;
    s_cnt[j] = 0u;
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kChunk / kNT1; ++j) {
    const int64_t i = chunk * kChunk + j * kNT1 + threadIdx.x;
    if (i >= it.n) continue;
    const PointEval e = eval_point(it.P, it.c, it.x[i], it.y[i], it.z[i]);
    int ix, iy;
    if (!e.valid || !bin_xy(e.xm, e.ym, it.c, ix, iy)) continue;
    if (it.c.excl_on && excluded_point(it.P, it.c, e)) continue;
    const uint32_t key = (uint32_t)pcell(it.c, ix, iy) + 1u;
    uint32_t h = (key * 2654435761u) >> (32 - kCountSlotsLog);
    while (true) {
      const uint32_t prev = atomicCAS(s_key + h, 0u, key);
      if (prev == 0u || prev == key) {
        atomicAdd(s_cnt + h, 1u);
        break;
      }
      h = (h + 1u) & (kCountSlots - 1);
    }
  }
  __syncthreads();
  for (int j = threadIdx.x; j < kCountSlots; j += kNT1) {
    const uint32_t key = s_key[j];
    if (key) atomicAdd(it.fs.count + (key - 1u), s_cnt[j]);
  }
}

// ------------------------------------- per-cell variances after a fusion
// Time variance: valid cells that the fusion did not update (no kMarkUpdated)
// gain sigma_t^2.  Outlier variance: cells flagged kMarkOutlier by pass 1
// then gain sigma_o^2.  The flags are cleared: marks are zero between calls.
constexpr int kNTv = 256;

__device__ __forceinline__ void timevar_body(const Item& it, int64_t unit) {
  const int64_t i = unit * kNTv + threadIdx.x;
  if (i >= (int64_t)it.c.nx * it.c.ny) return;
  const uint8_t m = it.L.mark[i];
  if (m) it.L.mark[i] = 0;
  const bool grow = it.c.var_t != 0.0f && !(m & kMarkUpdated) && it.L.valid[i];
  const bool outl = (m & kMarkOutlier) != 0;
  if (!grow && !outl) return;
  float v = it.L.v[i];
  if (grow) v = v + it.c.var_t;
  if (outl) v = v + it.c.var_o;
  it.L.v[i] = v;
}

__global__ __launch_bounds__(kNT1) void k_fuse_count(Item it) { count_body(it, blockIdx.x); }

__global__ __launch_bounds__(kNTv) void k_time_variance(Item it) { timevar_body(it, blockIdx.x); }

__global__ __launch_bounds__(256) void k_zero_u32(uint32_t* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// ---------------------------------------------------------------- launches
__global__ __launch_bounds__(kNT1) void k_fuse_chunk(Item it) {
  __shared__ AggTable tab;
  agg_clear(tab);
  __syncthreads();
  chunk_body(it, blockIdx.x, tab);
}

__global__ __launch_bounds__(kNT2) void k_fuse_tile(Item it) { tile_body_group(it, blockIdx.x); }

__global__ __launch_bounds__(kNT1) void k_fuse_chunk_b(const Batch* bt) {
  __shared__ AggTable tab;
  agg_clear(tab);
  __syncthreads();
  const int64_t total = bt->off[kBChunk][bt->n];
  for (int64_t w = blockIdx.x; w < total; w += gridDim.x) {
    const int i = batch_item(bt, kBChunk, w);
    chunk_body(bt->items[i], w - bt->off[kBChunk][i], tab);
  }
}

__global__ __launch_bounds__(256) void k_zero_b(const Batch* bt) {
  const int64_t total = bt->off[kBZero][bt->n];
  for (int64_t w = blockIdx.x; w < total; w += gridDim.x) {
    const int i = batch_item(bt, kBZero, w);
    const Item& it = bt->items[i];
    const int64_t c = (w - bt->off[kBZero][i]) * 256 + threadIdx.x;
    if (c < (int64_t)it.c.nx * it.c.ny) it.fs.count[c] = 0u;
  }
}

__global__ __launch_bounds__(kNT1) void k_fuse_count_b(const Batch* bt) {
  const int64_t total = bt->off[kBCount][bt->n];
  for (int64_t w = blockIdx.x; w < total; w += gridDim.x) {
    const int i = batch_item(bt, kBCount, w);
    count_body(bt->items[i], w - bt->off[kBCount][i]);
    __syncthreads();
  }
}

__global__ __launch_bounds__(kNTv) void k_time_variance_b(const Batch* bt) {
  const int64_t total = bt->off[kBVar][bt->n];
  for (int64_t w = blockIdx.x; w < total; w += gridDim.x) {
    const int i = batch_item(bt, kBVar, w);
    timevar_body(bt->items[i], w - bt->off[kBVar][i]);
  }
}

// Each wave takes its own tiles: units w = (workgroup * kTilesPerGroup +
// wave) + k * (grid * kTilesPerGroup).
__global__ __launch_bounds__(kNT2b) void k_fuse_tile_b(const Batch* bt) {
  const int64_t total = bt->off[kBTile][bt->n];
  const int64_t step = (int64_t)gridDim.x * kTilesPerGroup;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  for (int64_t w = (int64_t)blockIdx.x * kTilesPerGroup + wave; w < total; w += step) {
    const int i = batch_item(bt, kBTile, w);
    tile_body_wave(bt->items[i], w - bt->off[kBTile][i]);
  }
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Smallest E with x < 2^E, for finite x > 0.
int exp_above(double x) {
  int e = 0;
  const double f = frexp(x, &e);  // x = f * 2^e, 0.5 <= f < 1
  (void)f;
  return e;
}

// Largest shift S with n * bound * 2^S <= 2^93: then every term is below
// 2^94 / n (fx_split's range), and n such terms, plus the unit an accepted
// point may add, stay below 2^94 in total, so the hi words stay below 2^62
// and the lo words, each below 2^32, sum below 2^63 for n < 2^31.
int fixed_shift(double bound, int64_t n) {
  int ln = 0;
  while (((int64_t)1 << ln) < n) ++ln;
  return 93 - ln - exp_above(bound);
}

}  // namespace

int tiles_x_of(int nx) { return (nx + kTileW - 1) >> kTileLogX; }
int tiles_y_of(int ny) { return (ny + kTileH - 1) >> kTileLogY; }

void fuse_fixed_shifts(const Consts& c, const Pose32& P, int64_t n, int* fxw, int* fxz) {
  // Every accepted point has d2 >= rmin2 (float32 comparison), so its float32
  // 1/sp2 is at most 1/fl(alpha * rmin2): rounding is monotone.
  const float sp2min = c.alpha * c.rmin2;
  const double wmax = (double)(1.0f / sp2min);
  // |rz| <= |R20 xs| + |R21 ys| + |R22 zs| <= L1 * sqrt(d2) with the rounding of
  // the three products, two sums, d2 and sp2 bounded by a factor 1 + 2^-20,
  // so |fl(w * rz)| <= L1 / (alpha * sqrt(d2)) * (1 + 2^-20), largest at
  // d2 = rmin2.  The bound below adds a further margin.
  // A row with a non-finite entry makes every rz NaN or infinite: the gate
  // rejects every point, and any shift serves.
  const double l1 = fabs((double)P.R[6]) + fabs((double)P.R[7]) + fabs((double)P.R[8]);
  const double l1b = (l1 > 0.0 && isfinite(l1)) ? l1 : 1.0;
  const double zmax = l1b / ((double)c.alpha * sqrt((double)c.rmin2)) * (1.0 + 1.0 / 1024.0);
  const int64_t nn = n > 1 ? n : 1;
  *fxw = fixed_shift(wmax * (1.0 + 1.0 / 1024.0), nn);
  *fxz = fixed_shift(zmax, nn);
}

size_t fuse_scratch_layout(int64_t count_cells, char* base, FuseScratch* out) {
  if (out && base) out->count = count_cells > 0 ? (uint32_t*)base : nullptr;
  return align256((size_t)count_cells * sizeof(uint32_t));
}

hipError_t launch_fuse(const Item& it, hipStream_t stream) {
  hipError_t err = hipSuccess;
  const int64_t cells = (int64_t)it.c.nx * it.c.ny;
  if (it.n > 0) {
    if (it.fs.count) {  // wall/edge rule: the frame's points per cell first
      {
        TimedLaunch tl("k_zero_u32", stream);
        hipLaunchKernelGGL(k_zero_u32, dim3((unsigned)((cells + 255) / 256)), dim3(256), 0,
                           stream, it.fs.count, cells);
      }
      if ((err = hipGetLastError()) != hipSuccess) return err;
      {
        TimedLaunch tl("k_fuse_count", stream);
        hipLaunchKernelGGL(k_fuse_count, dim3(it.B), dim3(kNT1), 0, stream, it);
      }
      if ((err = hipGetLastError()) != hipSuccess) return err;
    }
    {
      TimedLaunch tl("k_fuse_chunk", stream);
      hipLaunchKernelGGL(k_fuse_chunk, dim3(it.B), dim3(kNT1), 0, stream, it);
    }
    if ((err = hipGetLastError()) != hipSuccess) return err;
    {
      TimedLaunch tl("k_fuse_tile", stream);
      hipLaunchKernelGGL(k_fuse_tile, dim3(it.T), dim3(kNT2), 0, stream, it);
    }
    if ((err = hipGetLastError()) != hipSuccess) return err;
  }
  if (it.c.var_t != 0.0f || (it.c.var_o != 0.0f && it.n > 0)) {
    // time variance (also after an empty frame) and outlier variance
    TimedLaunch tl("k_time_variance", stream);
    hipLaunchKernelGGL(k_time_variance, dim3((unsigned)((cells + kNTv - 1) / kNTv)), dim3(kNTv),
                       0, stream, it);
    err = hipGetLastError();
  }
  return err;
}

int64_t zero_units(int64_t cells) { return (cells + 255) / 256; }
int64_t var_units(int64_t cells) { return (cells + kNTv - 1) / kNTv; }

hipError_t launch_fuse_batch(const Batch* d_batch, const int grid[5], hipStream_t stream) {
  // grid: zero, count, chunk, tile, var; the first two and the last may be 0
  // (no item needs the stage: no launch)
  const int grid_chunk = grid[2], grid_tile = grid[3];
  if (grid[0] > 0) {
    TimedLaunch tl("k_zero_b", stream);
    hipLaunchKernelGGL(k_zero_b, dim3(grid[0]), dim3(256), 0, stream, d_batch);
  }
  if (grid[1] > 0) {
    TimedLaunch tl("k_fuse_count_b", stream);
    hipLaunchKernelGGL(k_fuse_count_b, dim3(grid[1]), dim3(kNT1), 0, stream, d_batch);
  }
  {
    TimedLaunch tl("k_fuse_chunk_b", stream);
    hipLaunchKernelGGL(k_fuse_chunk_b, dim3(grid_chunk), dim3(kNT1), 0, stream, d_batch);
  }
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  {
    TimedLaunch tl("k_fuse_tile_b", stream);
    // grid_tile counts tiles in flight; a workgroup holds kTilesPerGroup
    hipLaunchKernelGGL(k_fuse_tile_b, dim3((unsigned)((grid_tile + kTilesPerGroup - 1) / kTilesPerGroup)),
                       dim3(kNT2b), 0, stream, d_batch);
  }
  if (grid[4] > 0) {
    TimedLaunch tl("k_time_variance_b", stream);
    hipLaunchKernelGGL(k_time_variance_b, dim3(grid[4]), dim3(kNTv), 0, stream, d_batch);
  }
  return hipGetLastError();
}

}  // namespace emx
