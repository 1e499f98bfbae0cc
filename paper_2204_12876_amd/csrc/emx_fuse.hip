// Height fusion (Sec. II-C, Eq. 1 and Eq. 2) as a deterministic two-pass
// sort-and-reduce, with no float atomics.
//
// Pass 1, chunk body: one workgroup per chunk of kChunk (1024) consecutive points.
//   - Takes the per-point decisions: transform, range, bin, and the Mahalanobis
//     gate against the frame-start prior.
//   - Compacts the accepted points in point order and sums each run of
//     consecutive points in one cell (sensors emit points in scan order, so a
//     chunk of 1024 points holds a few hundred runs).
//   - Sorts the runs in LDS by (tile, cell in tile, run index), with a bitonic
//     network sized to the run count.
//   - Sums each cell's runs in run order into one partial, sum 1/sp2 and sum
//     zm/sp2.  Both sums are segmented inclusive scans (thread, wave, then a
//     carry across waves), read at a segment's last item.
//   - Writes the partials, grouped by tile, and appends one entry per touched
//     tile (chunk, first partial, partial count) to that tile's list; an
//     integer atomic on the tile's count, kept in the map state, picks the slot.
// Pass 2, tile body: one workgroup per 32x16-cell map tile, one thread per cell.
//   - A tile no chunk touched returns at once; otherwise the tile's count is
//     read and zeroed for the next call.
//   - The tile's entries are put back in chunk order through windows of chunk
//     ids in LDS (at most one entry per chunk and tile).
//   - Loads the tile's partials from every chunk that touched it, a group of
//     chunks at a time, all loads of a thread issued together.
//   - Places each partial in its cell's list in chunk order: a chunk holds at
//     most one partial per cell, so a partial's rank is the number of earlier
//     chunks holding its cell, read off a per-cell chunk bitmask in LDS.
//   - Each thread adds its cell's list in chunk order and applies the
//     information-form update once.
//
// The float32 sums therefore run in an order fixed by the frame and the map's
// placement: within a chunk (a fixed slice of the frame), the scan over its
// points in order, then the scan over its runs sorted by cell; then chunk
// partials left to right in chunk order.  Results are bitwise identical from
// run to run and alone or batched, whatever the grid shape.
#include "emx_kernels.h"

namespace emx {

namespace {

constexpr int kNT1 = kChunk / 2;          // pass-1 threads: two keys each
constexpr int kPBits = 10;                // run index within the chunk
static_assert((1 << kPBits) == kChunk, "the key's run field spans one chunk");
constexpr int kSegBits = kTileLogX + kTileLogY;  // local cell within the tile
// 32-bit keys hold (tile, local, run) while tile * kTileCells < 2^22.
constexpr int64_t kMaxCells32 = (int64_t)1 << (32 - kPBits);

// Value of v held by lane (lane ^ X) of the wave.  Lane distances below 16
// stay within a DPP row and use row moves (quad permutes for 1 and 2; for 4
// and 8, two masked row shifts, one per half of each group of 2X lanes);
// larger distances use a lane permute through the LDS crossbar.
template <int X>
__device__ __forceinline__ uint32_t lane_xor32(uint32_t v) {
  if constexpr (X == 1) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);  // [1,0,3,2]
  } else if constexpr (X == 2) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false);  // [2,3,0,1]
  } else if constexpr (X == 4) {
    const int t = __builtin_amdgcn_update_dpp((int)v, (int)v, 0x104, 0xF, 0x5, false);  // row_shl:4
    return (uint32_t)__builtin_amdgcn_update_dpp(t, (int)v, 0x114, 0xF, 0xA, false);    // row_shr:4
  } else if constexpr (X == 8) {
    const int t = __builtin_amdgcn_update_dpp((int)v, (int)v, 0x108, 0xF, 0x3, false);  // row_shl:8
    return (uint32_t)__builtin_amdgcn_update_dpp(t, (int)v, 0x118, 0xF, 0xC, false);    // row_shr:8
  } else {
    return (uint32_t)__shfl_xor((int)v, X, 64);
  }
}

template <int X>
__device__ __forceinline__ uint32_t lane_xor(uint32_t v) {
  return lane_xor32<X>(v);
}

template <int X>
__device__ __forceinline__ uint64_t lane_xor(uint64_t v) {
  const uint32_t lo = lane_xor32<X>((uint32_t)v);
  const uint32_t hi = lane_xor32<X>((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// One compare-exchange step of a bitonic merge of size Z at key stride S and
// every smaller stride down to 2, between the lanes of a wave.
template <typename KeyT, int Z, int S>
__device__ __forceinline__ void lane_steps(KeyT& a, KeyT& b, int i0) {
  if constexpr (S >= 2) {
    const KeyT pa = lane_xor<S / 2>(a);
    const KeyT pb = lane_xor<S / 2>(b);
    const bool up = (i0 & Z) == 0;
    const bool keep_min = ((i0 & S) == 0) == up;
    a = keep_min ? (a < pa ? a : pa) : (a < pa ? pa : a);
    b = keep_min ? (b < pb ? b : pb) : (b < pb ? pb : b);
    lane_steps<KeyT, Z, S / 2>(a, b, i0);
  }
}

// Ascending bitonic sort of the first NS keys of the block, two per thread:
// thread t < NS/2 holds the keys of sorted positions 2t and 2t+1 in (a, b);
// other threads take part in the barriers only.  The network is unrolled at
// compile time over merge sizes Z and key strides S:
//   - strides >= 128 cross waves and go through LDS with block barriers;
//   - strides 2..64 pair lane t with lane t ^ (S / 2) of the same wave;
//   - stride 1 stays within the thread.
template <typename KeyT, int NS, int Z>
__device__ __forceinline__ void bitonic_prefix_from(KeyT& a, KeyT& b, KeyT* s) {
  if constexpr (Z <= NS) {
    static_assert(NS >= 128 && NS <= 2 * kNT1, "whole waves sort");
    const int tid = threadIdx.x;
    const int i0 = 2 * tid;
    const bool active = tid < NS / 2;  // whole waves
    if constexpr (Z / 2 >= 128) {
      if (active) {
        s[i0] = a;
        s[i0 + 1] = b;
      }
      __syncthreads();
      for (int stride = Z / 2; stride >= 128; stride >>= 1) {
        if (active) {
          const int lo = 2 * tid - (tid & (stride - 1));
          const int hi = lo + stride;
          const bool up = (lo & Z) == 0;
          const KeyT x = s[lo];
          const KeyT y = s[hi];
          if ((x > y) == up) {
            s[lo] = y;
            s[hi] = x;
          }
        }
        __syncthreads();
      }
      if (active) {
        a = s[i0];
        b = s[i0 + 1];
      }
      __syncthreads();
    }
    if (active) {
      lane_steps<KeyT, Z, (Z / 2 < 64 ? Z / 2 : 64)>(a, b, i0);
      const bool up = (i0 & Z) == 0;
      if ((a > b) == up) {
        const KeyT t = a;
        a = b;
        b = t;
      }
    }
    bitonic_prefix_from<KeyT, NS, 2 * Z>(a, b, s);
  }
}

// ------------------------------------------------------------------ pass 1
// Segmented sums over a block-wide sequence of n items, two per thread (items
// 2t and 2t+1).  Item q belongs to segment seg(q) and carries the values
// val(q); a segment is a maximal run of equal seg values.  The additions take
// a fixed shape over the sequence: the thread's pair, the wave's lanes by
// shuffles, then a carry across waves in wave order.  A segment's sums are
// read at its last item (its tail).
struct SegTails {
  bool t0, t1;           // item 2t (2t+1) is the tail of its segment
  uint32_t s0, s1;       // the segments of items 2t and 2t+1
  float w0, wz0, w1, wz1;  // the segment sums at those tails
  int r;                 // rank of the thread's first tail among all tails
  int total;             // segments in the sequence
};

template <class Acc>
__device__ __forceinline__ SegTails segment_sums(int n, const Acc& acc, int* s_isum) {
  __shared__ int s_wf[kNT1 / 64];
  __shared__ float s_ww[kNT1 / 64];
  __shared__ float s_wwz[kNT1 / 64];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wid = tid >> 6;
  const int q0 = 2 * tid;
  const int q1 = q0 + 1;
  const bool in0 = q0 < n;
  const bool in1 = q1 < n;
  SegTails o;
  o.s0 = in0 ? acc.seg(q0) : 0xFFFFFFFFu;
  o.s1 = in1 ? acc.seg(q1) : 0xFFFFFFFFu;
  // segment heads; items past n start segments of their own and hold zero
  const bool f0 = !in0 || q0 == 0 || acc.seg(q0 - 1) != o.s0;
  const bool f1 = !in1 || o.s0 != o.s1;
  float w0 = 0.0f, wz0 = 0.0f, w1 = 0.0f, wz1 = 0.0f;
  if (in0) acc.val(q0, w0, wz0);
  if (in1) acc.val(q1, w1, wz1);
  // the thread's pair, then the wave: (flag, value) pairs combine as
  // earlier (+) later = later's flag ? later : earlier + later
  bool tf = f0 || f1;
  float tw = f1 ? w1 : w0 + w1;
  float twz = f1 ? wz1 : wz0 + wz1;
#pragma unroll
  for (int o2 = 1; o2 < 64; o2 <<= 1) {
    const bool pf = __shfl_up((int)tf, o2, 64) != 0;
    const float pw = __shfl_up(tw, o2, 64);
    const float pwz = __shfl_up(twz, o2, 64);
    if (lane >= o2) {
      if (!tf) {
        tw = pw + tw;
        twz = pwz + twz;
      }
      tf = tf || pf;
    }
  }
  if (lane == 63) {
    s_wf[wid] = tf ? 1 : 0;
    s_ww[wid] = tw;
    s_wwz[wid] = twz;
  }
  // the exclusive prefix of this thread within its wave
  bool ef = __shfl_up((int)tf, 1, 64) != 0;
  float ew = __shfl_up(tw, 1, 64);
  float ewz = __shfl_up(twz, 1, 64);
  if (lane == 0) {
    ef = false;
    ew = 0.0f;
    ewz = 0.0f;
  }
  __syncthreads();
  // carry from the preceding waves, combined in wave order
  float cw = 0.0f, cwz = 0.0f;
  for (int v = 0; v < wid; ++v) {
    if (s_wf[v]) {
      cw = s_ww[v];
      cwz = s_wwz[v];
    } else {
      cw = cw + s_ww[v];
      cwz = cwz + s_wwz[v];
    }
  }
  float pw, pwz;  // sum of the segment's items before q0
  if (lane == 0) {
    pw = cw;
    pwz = cwz;
  } else if (ef) {
    pw = ew;
    pwz = ewz;
  } else {
    pw = cw + ew;
    pwz = cwz + ewz;
  }
  o.w0 = f0 ? w0 : pw + w0;
  o.wz0 = f0 ? wz0 : pwz + wz0;
  o.w1 = f1 ? w1 : o.w0 + w1;
  o.wz1 = f1 ? wz1 : o.wz0 + wz1;
  o.t0 = in0 && f1;
  o.t1 = in1 && (q1 == n - 1 || acc.seg(q1 + 1) != o.s1);
  o.r = block_exclusive_sum<kNT1>((o.t0 ? 1 : 0) + (o.t1 ? 1 : 0), o.total, s_isum);
  return o;
}

// The frame's accepted points of the chunk, in point order.
struct PointSeq {
  const uint32_t* sg;
  const float* w;
  const float* wz;
  __device__ uint32_t seg(int q) const { return sg[q]; }
  __device__ void val(int q, float& a, float& b) const {
    a = w[q];
    b = wz[q];
  }
};

// The chunk's runs sorted by (segment, run): key = segment << kRunBits | run.
constexpr int kRunBits = kPBits;
template <typename KeyT>
struct RunSeq {
  const KeyT* key;
  const float* w;
  const float* wz;
  __device__ uint32_t seg(int q) const { return (uint32_t)(key[q] >> kRunBits); }
  __device__ void val(int q, float& a, float& b) const {
    const int r = (int)(key[q] & (KeyT)(kChunk - 1));
    a = w[r];
    b = wz[r];
  }
};

template <typename KeyT, int NS>
__device__ __forceinline__ void sort_runs(KeyT* s_key, int nrun) {
  constexpr KeyT kNoKey = (KeyT)~(KeyT)0;
  const int tid = threadIdx.x;
  KeyT a = kNoKey, b = kNoKey;
  if (tid < NS / 2) {
    a = 2 * tid < nrun ? s_key[2 * tid] : kNoKey;
    b = 2 * tid + 1 < nrun ? s_key[2 * tid + 1] : kNoKey;
  }
  __syncthreads();
  bitonic_prefix_from<KeyT, NS, 2>(a, b, s_key);
  if (tid < NS / 2) {
    s_key[2 * tid] = a;
    s_key[2 * tid + 1] = b;
  }
  __syncthreads();
}

// One chunk of kChunk points:
//   1. per-point decisions (transform, range, bin, gate), points 2t and 2t+1
//      in thread t;
//   2. the accepted points compacted in point order;
//   3. runs of consecutive accepted points in one cell summed in order
//      (segmented sums over the compacted sequence);
//   4. the runs sorted by (tile, cell in tile, run): a bitonic network sized
//      to the run count, not to the chunk;
//   5. each cell's runs summed in run order (segmented sums over the sorted
//      runs): one partial per cell, written grouped by tile, and one entry per
//      touched tile appended to that tile's list.
template <typename KeyT>
__device__ __forceinline__ void chunk_body(const Item& it, int64_t chunk) {
  __shared__ uint32_t s_cseg[kChunk];  // accepted points: (tile << kSegBits | local); later
                                       // the tile-and-cell of each partial
  __shared__ float s_cw[kChunk];
  __shared__ float s_cwz[kChunk];
  __shared__ KeyT s_key[kChunk];       // runs: (segment << kRunBits | run), sorted
  __shared__ float s_rw[kChunk];       // run sums by run index
  __shared__ float s_rwz[kChunk];
  __shared__ int s_isum[kNT1 / 64];

  const int tid = threadIdx.x;
  const int64_t base = chunk * kChunk;

  // ---- 1. per-point decisions
  uint32_t seg[2] = {0u, 0u};
  float w[2] = {0.0f, 0.0f}, wz[2] = {0.0f, 0.0f};
  bool acc[2] = {false, false};
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int64_t i = base + 2 * tid + j;
    if (i < it.n) {
      const PointEval e = eval_point(it.P, it.c, it.x[i], it.y[i], it.z[i]);
      int cell = -1;
      int ix = 0, iy = 0;
      int64_t pc = 0;
      if (e.valid && bin_xy(e.xm, e.ym, it.c, ix, iy)) {
        cell = iy * it.c.nx + ix;
        pc = pcell(it.c, ix, iy);
        // points of the exclusion area are ignored
        if (!it.c.excl_on || !excluded_point(it.P, it.c, e)) {
          const float h0 = it.L.h[pc];
          const float v0 = it.L.v[pc];
          const float d = e.zm - h0;
          const bool inside = (d * d) <= (it.c.k2 * (v0 + e.sp2));
          // wall/edge rule: in a crowded cell that holds an estimate, points
          // below the estimate are ignored (before the gate)
          const bool walled = it.fs.count && e.zm < h0 &&
                              it.fs.count[pc] > (uint32_t)it.c.wall && it.L.valid[pc];
          acc[j] = inside && !walled;
          // a gate-rejected point in a cell with an estimate flags the cell
          // for the outlier variance (a plain store: every writer stores 2)
          if (it.c.var_o != 0.0f && !inside && !walled && it.L.valid[pc])
            it.L.mark[pc] = kMarkOutlier;
        }
      }
      if (it.out_cell) it.out_cell[i] = cell;
      if (it.out_accept) it.out_accept[i] = acc[j] ? 1 : 0;
      if (acc[j]) {
        w[j] = 1.0f / e.sp2;
        wz[j] = w[j] * e.zm;
        // tiles cover the physical layout, so pass 2 writes whole rows
        const int py = (int)(pc / it.c.nx);
        const int px = (int)(pc - (int64_t)py * it.c.nx);
        const uint32_t tile = (uint32_t)((py >> kTileLogY) * it.tiles_x + (px >> kTileLogX));
        const uint32_t local =
            (uint32_t)(((py & (kTileH - 1)) << kTileLogX) | (px & (kTileW - 1)));
        seg[j] = (tile << kSegBits) | local;
      }
    }
  }

  // ---- 2. compaction in point order
  int nacc = 0;
  int pos = block_exclusive_sum<kNT1>((acc[0] ? 1 : 0) + (acc[1] ? 1 : 0), nacc, s_isum);
  if (nacc == 0) return;  // uniform: the chunk touches no tile
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    if (acc[j]) {
      s_cseg[pos] = seg[j];
      s_cw[pos] = w[j];
      s_cwz[pos] = wz[j];
      ++pos;
    }
  }
  __syncthreads();

  // ---- 3. runs of one cell in point order
  const SegTails ru = segment_sums(nacc, PointSeq{s_cseg, s_cw, s_cwz}, s_isum);
  const int nrun = ru.total;
  {
    int r = ru.r;
    if (ru.t0) {
      s_key[r] = ((KeyT)ru.s0 << kRunBits) | (KeyT)r;
      s_rw[r] = ru.w0;
      s_rwz[r] = ru.wz0;
      ++r;
    }
    if (ru.t1) {
      s_key[r] = ((KeyT)ru.s1 << kRunBits) | (KeyT)r;
      s_rw[r] = ru.w1;
      s_rwz[r] = ru.wz1;
    }
  }
  __syncthreads();

  // ---- 4. runs sorted by (tile, cell, run)
  if (nrun <= 128) sort_runs<KeyT, 128>(s_key, nrun);
  else if (nrun <= 256) sort_runs<KeyT, 256>(s_key, nrun);
  else if (nrun <= 512) sort_runs<KeyT, 512>(s_key, nrun);
  else sort_runs<KeyT, 1024>(s_key, nrun);

  // ---- 5. one partial per cell: its runs summed in run order
  const SegTails pa = segment_sums(nrun, RunSeq<KeyT>{s_key, s_rw, s_rwz}, s_isum);
  const int nrec = pa.total;
  {
    int r = pa.r;
    if (pa.t0) {
      const int64_t o = base + r;
      it.fs.rec_local[o] = (uint16_t)(pa.s0 & (kTileCells - 1));
      it.fs.rec_w[o] = pa.w0;
      it.fs.rec_wz[o] = pa.wz0;
      s_cseg[r] = pa.s0;
      ++r;
    }
    if (pa.t1) {
      const int64_t o = base + r;
      it.fs.rec_local[o] = (uint16_t)(pa.s1 & (kTileCells - 1));
      it.fs.rec_w[o] = pa.w1;
      it.fs.rec_wz[o] = pa.wz1;
      s_cseg[r] = pa.s1;
    }
  }
  __syncthreads();

  // ---- one entry per touched tile: the chunk, its first partial and partial
  // count, appended to the tile's list (an integer atomic picks the slot; pass
  // 2 restores chunk order, so the slot order never shows)
  for (int r2 = tid; r2 < nrec; r2 += kNT1) {
    const uint32_t tile = s_cseg[r2] >> kSegBits;
    if (r2 > 0 && (s_cseg[r2 - 1] >> kSegBits) == tile) continue;
    int lo = r2, hi = nrec;  // first partial of a later tile
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if ((s_cseg[mid] >> kSegBits) == tile) lo = mid + 1;
      else hi = mid;
    }
    const uint32_t slot = atomicAdd(it.fs.tcnt + tile, 1u);
    it.fs.ent[(int64_t)tile * it.B + slot] =
        make_uint2((uint32_t)chunk, ((uint32_t)r2 << 16) | (uint32_t)(lo - r2));
  }
}

// ------------------------------------------------------------------ pass 2
constexpr int kNT2 = kTileCells;           // pass-2 threads: one per cell of the tile
static_assert(kNT2 == kTileCells, "pass 2 gives each thread one cell of the tile");
constexpr int kCap = 8 * kNT2;             // partials staged per group
constexpr int kPer = kCap / kNT2;          // partials each thread loads per group
constexpr int kGroupChunks = 256;          // chunks per group
constexpr int kMaskWords = kGroupChunks / 32;
constexpr int kWin = kNT2;                 // chunk ids per directory window

__device__ __forceinline__ void tile_body(const Item& it, int t) {
  __shared__ uint32_t s_mask[kMaskWords][kTileCells];  // chunks of the group holding each cell
  __shared__ uint32_t s_start[kTileCells];             // per cell: count, then first slot
  __shared__ float s_w[kCap];                          // the group's partials by (cell, chunk)
  __shared__ float s_wz[kCap];
  __shared__ uint32_t e_win[kWin];                     // directory word per chunk of the window
  __shared__ uint32_t e_chunk[kWin];                   // touching chunks of the window
  __shared__ uint32_t e_dir[kWin];                     // their directory words
  __shared__ uint32_t e_pre[kWin + 1];                 // prefix of their partial counts
  __shared__ int s_isum[kNT2 / 64];
  __shared__ uint32_t s_umin[kNT2 / 64];
  __shared__ int s_g1;

  const int l = threadIdx.x;  // the cell of the tile this thread owns
  // the tile's entries: one per chunk that touched it, in slot order
  const uint32_t E = it.fs.tcnt[t];
  if (E == 0u) return;  // uniform: the frame did not touch the tile
  __syncthreads();      // every thread has read the count
  if (l == 0) it.fs.tcnt[t] = 0u;  // zero again for the next call
  const uint2* ent = it.fs.ent + (int64_t)t * it.B;
  float acc_w = 0.0f;
  float acc_wz = 0.0f;
  bool hit = false;
  const int tx = t % it.tiles_x;
  const int ty = t / it.tiles_x;
  // the owned cell, physical (tiles cover the ring layout as stored)
  const int ix = (tx << kTileLogX) + (l & (kTileW - 1));
  const int iy = (ty << kTileLogY) + (l >> kTileLogX);
  const int64_t cell = (int64_t)iy * it.c.nx + ix;

  // windows of kWin chunk ids, each starting at the smallest touching chunk
  // not yet taken; within a window the chunks come out in chunk order
  uint32_t next = 0u;
  while (true) {
    uint32_t mn = 0xFFFFFFFFu;
    for (uint32_t j = (uint32_t)l; j < E; j += kNT2) {
      const uint32_t c = ent[j].x;
      if (c >= next && c < mn) mn = c;
    }
    mn = block_min_u32<kNT2>(mn, s_umin);
    if (mn == 0xFFFFFFFFu) break;
    const uint32_t w0 = mn;
    e_win[l] = 0u;
    __syncthreads();
    for (uint32_t j = (uint32_t)l; j < E; j += kNT2) {
      const uint2 e = ent[j];
      if (e.x >= w0 && e.x - w0 < (uint32_t)kWin) e_win[e.x - w0] = e.y;
    }
    __syncthreads();
    next = w0 + (uint32_t)kWin;
    // compact the window's touching chunks, in chunk order
    const uint32_t d = e_win[l];
    int L = 0;
    const int pos = block_exclusive_sum<kNT2>(d != 0u ? 1 : 0, L, s_isum);
    if (d != 0u) {
      e_chunk[pos] = w0 + (uint32_t)l;
      e_dir[pos] = d;
    }
    __syncthreads();
    int totw = 0;
    const int pre = block_exclusive_sum<kNT2>(l < L ? (int)(e_dir[l] & 0xFFFFu) : 0, totw, s_isum);
    if (l < L) e_pre[l] = (uint32_t)pre;
    if (l == 0) e_pre[L] = (uint32_t)totw;
    __syncthreads();
    for (int g0 = 0; g0 < L;) {
      // the group: chunks [g0, g1), at most kGroupChunks of them and kCap partials
      if (l == 0) {
        int lo = g0 + 1, hi = min(L, g0 + kGroupChunks);
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (e_pre[mid] - e_pre[g0] <= (uint32_t)kCap) lo = mid;
          else hi = mid - 1;
        }
        s_g1 = lo;
      }
#pragma unroll
      for (int w = 0; w < kMaskWords; ++w) s_mask[w][l] = 0u;
      s_start[l] = 0u;
      __syncthreads();
      const int g1 = s_g1;
      const uint32_t pbase = e_pre[g0];
      const int tot = (int)(e_pre[g1] - pbase);

      // load this thread's partials; every load is issued before any is used
      int pg[kPer], pl[kPer];
      float pw[kPer], pwz[kPer];
#pragma unroll
      for (int j = 0; j < kPer; ++j) {
        const int p = l + j * kNT2;
        pg[j] = -1;
        pl[j] = 0;
        pw[j] = 0.0f;
        pwz[j] = 0.0f;
        if (p < tot) {
          const uint32_t gp = pbase + (uint32_t)p;
          int lo = g0, hi = g1 - 1;  // the chunk whose partials include gp
          while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (e_pre[mid] <= gp) lo = mid;
            else hi = mid - 1;
          }
          pg[j] = lo;
          const int64_t idx =
              (int64_t)e_chunk[lo] * kChunk + (e_dir[lo] >> 16) + (gp - e_pre[lo]);
          pl[j] = it.fs.rec_local[idx];
          pw[j] = it.fs.rec_w[idx];
          pwz[j] = it.fs.rec_wz[idx];
        }
      }
      // which chunks of the group hold each cell (a chunk holds a cell at most once)
#pragma unroll
      for (int j = 0; j < kPer; ++j) {
        if (pg[j] < 0) continue;
        const int gg = pg[j] - g0;
        atomicOr(&s_mask[gg >> 5][pl[j]], 1u << (gg & 31));
        atomicAdd(&s_start[pl[j]], 1u);
      }
      __syncthreads();
      const int my_cnt = (int)s_start[l];
      int all = 0;
      const int my_start = block_exclusive_sum<kNT2>(my_cnt, all, s_isum);
      s_start[l] = (uint32_t)my_start;
      __syncthreads();
      // each partial's slot: its cell's first slot plus the number of earlier
      // chunks of the group that hold the cell
#pragma unroll
      for (int j = 0; j < kPer; ++j) {
        if (pg[j] < 0) continue;
        const int gg = pg[j] - g0;
        const int c = pl[j];
        int rank = __popc(s_mask[gg >> 5][c] & ((1u << (gg & 31)) - 1u));
        for (int w = 0; w < (gg >> 5); ++w) rank += __popc(s_mask[w][c]);
        const int slot = (int)s_start[c] + rank;
        s_w[slot] = pw[j];
        s_wz[slot] = pwz[j];
      }
      __syncthreads();
      // the owned cell's partials, in chunk order
      for (int k = 0; k < my_cnt; ++k) {
        acc_w = acc_w + s_w[my_start + k];
        acc_wz = acc_wz + s_wz[my_start + k];
      }
      hit = hit || my_cnt > 0;
      __syncthreads();  // the next group reuses the arrays
      g0 = g1;
    }
  }
  if (!hit) return;

  // ---- information-form update of the owned cell
  const float h0 = it.L.h[cell];
  const float v0 = it.L.v[cell];
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
template <typename KeyT>
__global__ __launch_bounds__(kNT1) void k_fuse_chunk(Item it) {
  chunk_body<KeyT>(it, blockIdx.x);
}

__global__ __launch_bounds__(kNT2) void k_fuse_tile(Item it) { tile_body(it, blockIdx.x); }

template <typename KeyT>
__global__ __launch_bounds__(kNT1) void k_fuse_chunk_b(const Batch* bt) {
  const int64_t total = bt->off[kBChunk][bt->n];
  for (int64_t w = blockIdx.x; w < total; w += gridDim.x) {
    const int i = batch_item(bt, kBChunk, w);
    chunk_body<KeyT>(bt->items[i], w - bt->off[kBChunk][i]);
    __syncthreads();
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

__global__ __launch_bounds__(kNT2) void k_fuse_tile_b(const Batch* bt) {
  const int64_t total = bt->off[kBTile][bt->n];
  for (int64_t w = blockIdx.x; w < total; w += gridDim.x) {
    const int i = batch_item(bt, kBTile, w);
    tile_body(bt->items[i], (int)(w - bt->off[kBTile][i]));
    __syncthreads();
  }
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

int tiles_x_of(int nx) { return (nx + kTileW - 1) >> kTileLogX; }
int tiles_y_of(int ny) { return (ny + kTileH - 1) >> kTileLogY; }
bool fuse_needs_key64(int T) { return (int64_t)T * kTileCells > kMaxCells32; }

size_t fuse_scratch_layout(int64_t max_points, int T, int64_t count_cells, char* base,
                           FuseScratch* out) {
  const int64_t B = (max_points + kChunk - 1) / kChunk;
  const size_t nrec = (size_t)B * kChunk;
  size_t off = 0;
  const size_t o_local = off;
  off = align256(off + nrec * sizeof(uint16_t));
  const size_t o_w = off;
  off = align256(off + nrec * sizeof(float));
  const size_t o_wz = off;
  off = align256(off + nrec * sizeof(float));
  const size_t o_ent = off;
  off = align256(off + (size_t)B * (size_t)T * sizeof(uint2));
  const size_t o_cnt = off;
  off = align256(off + (size_t)count_cells * sizeof(uint32_t));
  if (out && base) {
    out->rec_local = (uint16_t*)(base + o_local);
    out->rec_w = (float*)(base + o_w);
    out->rec_wz = (float*)(base + o_wz);
    out->ent = (uint2*)(base + o_ent);
    out->count = count_cells > 0 ? (uint32_t*)(base + o_cnt) : nullptr;
  }
  return off;
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
      if (fuse_needs_key64(it.T))
        hipLaunchKernelGGL(k_fuse_chunk<uint64_t>, dim3(it.B), dim3(kNT1), 0, stream, it);
      else
        hipLaunchKernelGGL(k_fuse_chunk<uint32_t>, dim3(it.B), dim3(kNT1), 0, stream, it);
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

hipError_t launch_fuse_batch(const Batch* d_batch, bool key64, const int grid[5],
                             hipStream_t stream) {
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
    if (key64)
      hipLaunchKernelGGL(k_fuse_chunk_b<uint64_t>, dim3(grid_chunk), dim3(kNT1), 0, stream,
                         d_batch);
    else
      hipLaunchKernelGGL(k_fuse_chunk_b<uint32_t>, dim3(grid_chunk), dim3(kNT1), 0, stream,
                         d_batch);
  }
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  {
    TimedLaunch tl("k_fuse_tile_b", stream);
    hipLaunchKernelGGL(k_fuse_tile_b, dim3(grid_tile), dim3(kNT2), 0, stream, d_batch);
  }
  if (grid[4] > 0) {
    TimedLaunch tl("k_time_variance_b", stream);
    hipLaunchKernelGGL(k_time_variance_b, dim3(grid[4]), dim3(kNTv), 0, stream, d_batch);
  }
  return hipGetLastError();
}

}  // namespace emx
