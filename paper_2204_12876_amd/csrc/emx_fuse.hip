// Height fusion (Sec. II-C, Eq. 1 and Eq. 2) as a deterministic two-pass
// sort-and-reduce, with no float atomics.
//
// Pass 1, chunk body: one workgroup per chunk of kChunk (1024) consecutive points.
//   - Takes the per-point decisions: transform, range, bin, and the Mahalanobis
//     gate against the frame-start prior.
//   - Sorts the accepted points in LDS by (tile, cell in tile, point index).
//   - Each cell's run is reduced to one partial, sum 1/sp2 and sum zm/sp2, by
//     a segmented inclusive scan over the sorted keys (thread, wave, then a
//     carry across waves), read at the run's last key.
//   - Writes the partials, grouped by tile, and a dense tile directory row for
//     the chunk.
// Pass 2, tile body: one workgroup per 32x32-cell map tile, one thread per cell.
//   - Loads the tile's partials from every chunk that touched it, a group of
//     chunks at a time, all loads of a thread issued together.
//   - Places each partial in its cell's list in chunk order: a chunk holds at
//     most one partial per cell, so a partial's rank is the number of earlier
//     chunks holding its cell, read off a per-cell chunk bitmask in LDS.
//   - Each thread adds its cell's list in chunk order and applies the
//     information-form update once.
//
// The float32 sums therefore run in an order fixed by the frame alone: the
// scan over each chunk's sorted keys (chunks are fixed slices of the frame),
// then chunk partials left to right in chunk order.  Results are bitwise
// identical from run to run, whatever the tile size, grid shape or batching.
#include "emx_kernels.h"

namespace emx {

namespace {

constexpr int kNT1 = kChunk / 2;          // pass-1 threads: two keys each
constexpr int kPBits = 10;                // point index within the chunk
static_assert((1 << kPBits) == kChunk, "the key's point field spans one chunk");
constexpr int kSegBits = kTileLogX + kTileLogY;  // local cell within the tile
// 32-bit keys hold (tile, local, point) while tile * kTileCells < 2^21.
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

// Ascending bitonic sort of the block's 2 * kNT1 keys.  Thread t holds the
// keys of sorted positions 2t and 2t+1 in (a, b).  The network is unrolled at
// compile time over merge sizes Z and key strides S:
//   - strides >= 128 cross waves and go through LDS with block barriers;
//   - strides 2..64 pair lane t with lane t ^ (S / 2) of the same wave;
//   - stride 1 stays within the thread.
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

template <typename KeyT, int Z>
__device__ __forceinline__ void bitonic_from(KeyT& a, KeyT& b, KeyT* s) {
  if constexpr (Z <= 2 * kNT1) {
    const int tid = threadIdx.x;
    const int i0 = 2 * tid;
    if constexpr (Z / 2 >= 128) {
      s[i0] = a;
      s[i0 + 1] = b;
      __syncthreads();
      for (int stride = Z / 2; stride >= 128; stride >>= 1) {
        const int lo = 2 * tid - (tid & (stride - 1));
        const int hi = lo + stride;
        const bool up = (lo & Z) == 0;
        const KeyT x = s[lo];
        const KeyT y = s[hi];
        if ((x > y) == up) {
          s[lo] = y;
          s[hi] = x;
        }
        __syncthreads();
      }
      a = s[i0];
      b = s[i0 + 1];
      __syncthreads();
    }
    lane_steps<KeyT, Z, (Z / 2 < 64 ? Z / 2 : 64)>(a, b, i0);
    const bool up = (i0 & Z) == 0;
    if ((a > b) == up) {
      const KeyT t = a;
      a = b;
      b = t;
    }
    bitonic_from<KeyT, 2 * Z>(a, b, s);
  }
}

template <typename KeyT>
__device__ __forceinline__ void bitonic_sort_regs(KeyT& a, KeyT& b, KeyT* s) {
  bitonic_from<KeyT, 2>(a, b, s);
}

// ------------------------------------------------------------------ pass 1
// kMove: the fusion also performs the item's move (the prior is read from the
// source set through the shift).
template <typename KeyT, bool kMove = false>
__device__ __forceinline__ void chunk_body(const Item& it, int64_t chunk) {
  constexpr KeyT kNoKey = (KeyT)~(KeyT)0;
  __shared__ KeyT s_key[kChunk];
  __shared__ float s_w[kChunk];
  __shared__ float s_wz[kChunk];
  __shared__ uint32_t s_seg[kChunk];   // (tile << kSegBits | local) of record r
  __shared__ int s_isum[kNT1 / 64];

  const int tid = threadIdx.x;
  const int64_t base = chunk * kChunk;
  const int T = it.T;
  uint32_t* drow = it.fs.dir + chunk * (int64_t)T;
  for (int t = tid; t < T; t += kNT1) drow[t] = 0u;

  // ---- per-point decisions; thread t takes points t and t + kNT1
  KeyT key[2];
  int nmine = 0;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int p = j * kNT1 + tid;
    const int64_t i = base + p;
    key[j] = kNoKey;
    if (i < it.n) {
      const PointEval e = eval_point(it.P, it.c, it.x[i], it.y[i], it.z[i]);
      int cell = -1;
      bool acc = false;
      int ix = 0, iy = 0;
      if (e.valid && bin_xy(e.xm, e.ym, it.c, ix, iy)) {
        cell = iy * it.c.nx + ix;
        // the prior: the map's cell, or with a fused move the moved-in cell
        // of the source set (the prior values where the cell enters)
        const int64_t sc = kMove ? move_source(it, ix, iy) : cell;
        const Layers& P = kMove ? it.Lsrc : it.L;
        const float h0 = sc >= 0 ? P.h[sc] : it.c.h_init;
        const float v0 = sc >= 0 ? P.v[sc] : it.c.v_init;
        const float d = e.zm - h0;
        acc = (d * d) <= (it.c.k2 * (v0 + e.sp2));
        // wall/edge rule: in a crowded cell that holds an estimate, points
        // below the estimate are ignored (before the gate)
        if (it.fs.count && e.zm < h0 && it.fs.count[cell] > (uint32_t)it.c.wall && sc >= 0 &&
            P.valid[sc])
          acc = false;
      }
      if (it.out_cell) it.out_cell[i] = cell;
      if (it.out_accept) it.out_accept[i] = acc ? 1 : 0;
      if (acc) {
        const float w = 1.0f / e.sp2;
        s_w[p] = w;
        s_wz[p] = w * e.zm;
        const uint32_t tile = (uint32_t)((iy >> kTileLogY) * it.tiles_x + (ix >> kTileLogX));
        const uint32_t local =
            (uint32_t)(((iy & (kTileH - 1)) << kTileLogX) | (ix & (kTileW - 1)));
        const KeyT seg = ((KeyT)tile << kSegBits) | (KeyT)local;
        key[j] = (seg << kPBits) | (KeyT)p;
        ++nmine;
      }
    }
  }
  int nacc = 0;
  (void)block_exclusive_sum<kNT1>(nmine, nacc, s_isum);
  if (nacc == 0) return;  // uniform: the directory row stays zero

  // ---- sort by (tile, local, point); invalid keys sort last
  bitonic_sort_regs<KeyT>(key[0], key[1], s_key);
  s_key[2 * tid] = key[0];
  s_key[2 * tid + 1] = key[1];
  __syncthreads();

  // ---- one partial per (tile, local) run, by a segmented inclusive scan over
  // the sorted keys: within the thread, then across the wave's lanes, then a
  // carry across waves.  A run's sum is the scan value at its last key.  The
  // order of the additions is fixed by the chunk's sorted keys, which depend
  // only on the frame.
  const int lane = tid & 63;
  const int wid = tid >> 6;
  const int q0 = 2 * tid;
  const int q1 = q0 + 1;
  const uint32_t k0 = (uint32_t)(s_key[q0] >> kPBits);
  const uint32_t k1 = (uint32_t)(s_key[q1] >> kPBits);
  // run heads; keys past nacc start segments of their own and hold zero
  const bool f0 = q0 >= nacc || q0 == 0 || (uint32_t)(s_key[q0 - (q0 > 0)] >> kPBits) != k0;
  const bool f1 = q1 >= nacc || k0 != k1;
  float w0 = 0.0f, wz0 = 0.0f, w1 = 0.0f, wz1 = 0.0f;
  if (q0 < nacc) {
    const int p = (int)(s_key[q0] & (KeyT)(kChunk - 1));
    w0 = s_w[p];
    wz0 = s_wz[p];
  }
  if (q1 < nacc) {
    const int p = (int)(s_key[q1] & (KeyT)(kChunk - 1));
    w1 = s_w[p];
    wz1 = s_wz[p];
  }
  // the thread's two keys, then the wave: (flag, value) pairs combine as
  // earlier (+) later = later's flag ? later : earlier + later
  bool tf = f0 || f1;
  float tw = f1 ? w1 : w0 + w1;
  float twz = f1 ? wz1 : wz0 + wz1;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const bool pf = __shfl_up((int)tf, o, 64) != 0;
    const float pw = __shfl_up(tw, o, 64);
    const float pwz = __shfl_up(twz, o, 64);
    if (lane >= o) {
      if (!tf) {
        tw = pw + tw;
        twz = pwz + twz;
      }
      tf = tf || pf;
    }
  }
  __shared__ int s_wf[kNT1 / 64];
  __shared__ float s_ww[kNT1 / 64];
  __shared__ float s_wwz[kNT1 / 64];
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
  float pw, pwz;  // sum of the run's keys before q0
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
  const float i0w = f0 ? w0 : pw + w0;
  const float i0wz = f0 ? wz0 : pwz + wz0;
  const float i1w = f1 ? w1 : i0w + w1;
  const float i1wz = f1 ? wz1 : i0wz + wz1;
  // run tails, one record each, in run order
  const bool t0 = q0 < nacc && f1;
  const bool t1 = q1 < nacc &&
                  (q1 == nacc - 1 || (uint32_t)(s_key[q1 + (q1 + 1 < kChunk)] >> kPBits) != k1);
  int nrec = 0;
  int r = block_exclusive_sum<kNT1>((t0 ? 1 : 0) + (t1 ? 1 : 0), nrec, s_isum);
  if (t0) {
    const int64_t o = base + r;
    it.fs.rec_local[o] = (uint16_t)(k0 & (kTileCells - 1));
    it.fs.rec_w[o] = i0w;
    it.fs.rec_wz[o] = i0wz;
    s_seg[r] = k0;
    ++r;
  }
  if (t1) {
    const int64_t o = base + r;
    it.fs.rec_local[o] = (uint16_t)(k1 & (kTileCells - 1));
    it.fs.rec_w[o] = i1w;
    it.fs.rec_wz[o] = i1wz;
    s_seg[r] = k1;
  }
  __syncthreads();

  // ---- directory: first record and record count of each touched tile
  for (int r2 = tid; r2 < nrec; r2 += kNT1) {
    const uint32_t tile = s_seg[r2] >> kSegBits;
    if (r2 > 0 && (s_seg[r2 - 1] >> kSegBits) == tile) continue;
    int lo = r2, hi = nrec;  // first record of a later tile
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if ((s_seg[mid] >> kSegBits) == tile) lo = mid + 1;
      else hi = mid;
    }
    drow[tile] = ((uint32_t)r2 << 16) | (uint32_t)(lo - r2);
  }
}

// ------------------------------------------------------------------ pass 2
constexpr int kNT2 = kTileCells;           // pass-2 threads: one per cell of the tile
static_assert(kNT2 == kTileCells, "pass 2 gives each thread one cell of the tile");
constexpr int kCap = 8 * kNT2;             // partials staged per group
constexpr int kPer = kCap / kNT2;          // partials each thread loads per group
constexpr int kGroupChunks = 256;          // chunks per group
constexpr int kMaskWords = kGroupChunks / 32;
constexpr int kWin = kNT2;                 // directory entries read per window

__device__ __forceinline__ void tile_body(const Item& it, int t) {
  __shared__ uint32_t s_mask[kMaskWords][kTileCells];  // chunks of the group holding each cell
  __shared__ uint32_t s_start[kTileCells];             // per cell: count, then first slot
  __shared__ float s_w[kCap];                          // the group's partials by (cell, chunk)
  __shared__ float s_wz[kCap];
  __shared__ uint32_t e_chunk[kWin];                   // touching chunks of the window
  __shared__ uint32_t e_dir[kWin];                     // their directory words
  __shared__ uint32_t e_pre[kWin + 1];                 // prefix of their partial counts
  __shared__ int s_isum[kNT2 / 64];
  __shared__ int s_g1;

  const int l = threadIdx.x;  // the cell of the tile this thread owns
  const int B = it.B;
  const int T = it.T;
  float acc_w = 0.0f;
  float acc_wz = 0.0f;
  bool hit = false;
  const int tx = t % it.tiles_x;
  const int ty = t / it.tiles_x;
  const int ix = (tx << kTileLogX) + (l & (kTileW - 1));
  const int iy = (ty << kTileLogY) + (l >> kTileLogX);
  const int64_t cell = (int64_t)iy * it.c.nx + ix;
  // a fused move: every cell of the tile takes its moved-in values first (the
  // same thread updates it below, so the update sees them)
  float h0 = 0.0f, v0 = 0.0f;
  if (it.fuse_move && ix < it.c.nx && iy < it.c.ny) move_cell(it, ix, iy, h0, v0);

  for (int k0 = 0; k0 < B; k0 += kWin) {
    // compact the chunks of this window that touched the tile, in chunk order
    const int kk = k0 + l;
    const uint32_t d = (kk < B) ? it.fs.dir[(int64_t)kk * T + t] : 0u;
    int L = 0;
    const int pos = block_exclusive_sum<kNT2>(d != 0u ? 1 : 0, L, s_isum);
    if (d != 0u) {
      e_chunk[pos] = (uint32_t)kk;
      e_dir[pos] = d;
    }
    __syncthreads();
    if (L == 0) continue;
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
  if (!it.fuse_move) {
    h0 = it.L.h[cell];
    v0 = it.L.v[cell];
  }
  const float W = (1.0f / v0) + acc_w;
  const float v1 = 1.0f / W;
  const float h1 = ((h0 / v0) + acc_wz) * v1;
  it.L.h[cell] = h1;
  it.L.v[cell] = v1;
  it.L.t[cell] = it.t_now;
  it.L.valid[cell] = 1;
  if (it.c.var_t != 0.0f) it.L.mark[cell] = 1;  // updated: no time variance
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
    const uint32_t key = (uint32_t)iy * (uint32_t)it.c.nx + (uint32_t)ix + 1u;
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

// ------------------------------------------- time variance after a fusion
// Valid cells that the fusion did not update (not flagged in the mark layer)
// gain sigma_t^2; the flags are cleared, since clearing expects zero marks.
constexpr int kNTv = 256;

__device__ __forceinline__ void timevar_body(const Item& it, int64_t unit) {
  const int64_t i = unit * kNTv + threadIdx.x;
  if (i >= (int64_t)it.c.nx * it.c.ny) return;
  if (it.L.mark[i]) {
    it.L.mark[i] = 0;
  } else if (it.L.valid[i]) {
    it.L.v[i] = it.L.v[i] + it.c.var_t;
  }
}

__global__ __launch_bounds__(kNT1) void k_fuse_count(Item it) { count_body(it, blockIdx.x); }

__global__ __launch_bounds__(kNTv) void k_time_variance(Item it) { timevar_body(it, blockIdx.x); }

__global__ __launch_bounds__(256) void k_zero_u32(uint32_t* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// ---------------------------------------------------------------- launches
template <typename KeyT, bool kMove>
__global__ __launch_bounds__(kNT1) void k_fuse_chunk(Item it) {
  chunk_body<KeyT, kMove>(it, blockIdx.x);
}

__global__ __launch_bounds__(kNT2) void k_fuse_tile(Item it) { tile_body(it, blockIdx.x); }

template <typename KeyT>
__global__ __launch_bounds__(kNT1) void k_fuse_chunk_b(const Batch* bt) {
  const int64_t total = bt->off[kBChunk][bt->n];
  for (int64_t w = blockIdx.x; w < total; w += gridDim.x) {
    const int i = batch_item(bt, kBChunk, w);
    if (bt->items[i].fuse_move) chunk_body<KeyT, true>(bt->items[i], w - bt->off[kBChunk][i]);
    else chunk_body<KeyT, false>(bt->items[i], w - bt->off[kBChunk][i]);
    __syncthreads();
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
  const size_t o_dir = off;
  off = align256(off + (size_t)B * (size_t)T * sizeof(uint32_t));
  const size_t o_cnt = off;
  off = align256(off + (size_t)count_cells * sizeof(uint32_t));
  if (out && base) {
    out->rec_local = (uint16_t*)(base + o_local);
    out->rec_w = (float*)(base + o_w);
    out->rec_wz = (float*)(base + o_wz);
    out->dir = (uint32_t*)(base + o_dir);
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
      const bool k64 = fuse_needs_key64(it.T);
      if (it.fuse_move) {
        if (k64) hipLaunchKernelGGL((k_fuse_chunk<uint64_t, true>), dim3(it.B), dim3(kNT1), 0, stream, it);
        else hipLaunchKernelGGL((k_fuse_chunk<uint32_t, true>), dim3(it.B), dim3(kNT1), 0, stream, it);
      } else {
        if (k64) hipLaunchKernelGGL((k_fuse_chunk<uint64_t, false>), dim3(it.B), dim3(kNT1), 0, stream, it);
        else hipLaunchKernelGGL((k_fuse_chunk<uint32_t, false>), dim3(it.B), dim3(kNT1), 0, stream, it);
      }
    }
    if ((err = hipGetLastError()) != hipSuccess) return err;
    {
      TimedLaunch tl("k_fuse_tile", stream);
      hipLaunchKernelGGL(k_fuse_tile, dim3(it.T), dim3(kNT2), 0, stream, it);
    }
    if ((err = hipGetLastError()) != hipSuccess) return err;
  }
  if (it.c.var_t != 0.0f) {  // time variance, also after an empty frame
    TimedLaunch tl("k_time_variance", stream);
    hipLaunchKernelGGL(k_time_variance, dim3((unsigned)((cells + kNTv - 1) / kNTv)), dim3(kNTv),
                       0, stream, it);
    err = hipGetLastError();
  }
  return err;
}

hipError_t launch_fuse_batch(const Batch* d_batch, bool key64, int grid_chunk, int grid_tile,
                             hipStream_t stream) {
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
  return hipGetLastError();
}

}  // namespace emx
