// Visibility clean-up by ray casting (Sec. II-E, Eq. 3 and Eq. 4).
//
// The samples of a ray are q_k = o + (k/K) d for k = 1..K-1, in float32.
// Their number varies from 0 to a few hundred per ray, so one thread per ray
// leaves the long rays on the critical path.  The work is therefore split in
// two launches:
//
// setup, two roles in one grid:
//   - Block role: per block of 2^b x 2^b cells, the largest height of a cell
//     that a ray could still remove: valid, older than the minimum age, with a
//     normal.  It is -inf if there is none.  In blocks with such a cell the
//     same pass writes each cell's 8-byte clearing record {h, or -inf if no
//     ray may remove it, v}, so that the march's height test takes one load.
//     Other blocks prune every sample, so their records are never read.
//     The cells' loads come in two rounds, each issued at once: validity,
//     then the update time, normal z and height of valid cells (or the upper
//     bound of invalid ones).
//   - Ray role, one thread per point:
//       - the ray's exact in-map range of k.  A sample's cell is in the map over
//         a contiguous range of k, because q_k.x and q_k.y are monotone in k:
//         each is a correctly rounded chain of monotone operations.  The range
//         is found by binary search with the very sample evaluation the march
//         uses.
//       - the range is cut into segments of `seg` samples.  Each workgroup
//         reserves its segments with one integer atomic, in one of kSubQ
//         sub-queues, so no counter is contended.  An entry names the ray by
//         its point (8 bytes: the ray, the first sample and the count); the
//         march rebuilds the ray from the point, so no per-ray record is
//         written.  A ray that would overflow its bounded sub-queue goes whole
//         to an overflow list (one entry per ray at most, so the list cannot
//         overflow).
//   - Block 0 zeroes the counter set of the next plain call, and the block
//     role zeroes the caller's removed-cell mask.
// march: a persistent grid drains the queue, one segment per thread.
//   - A segment's consecutive samples mostly stay in one block: the block
//     maximum is loaded again only when the block changes.
//   - A sample at height q.z >= the block maximum passes above every cell that
//     could be removed, since removal needs h > q.z.  It is skipped without
//     reading the cell: exact pruning.
//   - Other samples read their cell's clearing record (and the normal only
//     if the height test passes).
//   - A sample that removes its cell resets the cell to the prior on the spot
//     (and flags it in the caller's mask).  The march reads only the setup's
//     records and the normals, never the heights, variances or validity it
//     resets, so every ray still sees the state as it was when the call
//     started.  Resets are idempotent stores of the same values, so the queue
//     order never shows in the result.
//   - The overflow list's rays are marched after the queue, whole.
// There is no separate pass to apply the removals.
//
// Upper bound layer (Sec. II-H), on maps that keep one: a sample in a cell
// without an estimate lowers the cell's bound to the sample height, by an
// integer atomic minimum (order-free, so deterministic).  Such cells count in
// the block maximum with their current bound, so pruning stays exact: a
// sample at or above it can neither remove a cell nor lower a bound.
#include "emx_kernels.h"

namespace emx {

namespace {

constexpr int kNTc = 256;

struct Ray {
  float ox, oy, oz;
  float dx, dy, dz;
  double rK;  // 1/K, correctly rounded in double
};

// t = float32(k / K), correctly rounded, without a float32 division.
// For integers 1 <= k < K < 2^24, k/K lies more than 2^-49 (relative) from
// every float32 rounding boundary: a boundary is an odd multiple of half an
// ulp, and k/K equal to one would need K > k >= 2^24.  The double product
// k * RN(1/K) carries at most 2^-52 relative error, so it rounds to the same
// float32 as k/K.
__device__ __forceinline__ float t_of(const Ray& r, int k) {
  return (float)((double)k * r.rK);
}

// f(k) = q_k.x * inv_r (or .y), exactly as binning computes it
template <bool kIsX>
__device__ __forceinline__ float f_of(const Ray& r, int k, float inv_r) {
  const float t = t_of(r, k);
  return kIsX ? (r.ox + t * r.dx) * inv_r : (r.oy + t * r.dy) * inv_r;
}

// Smallest k in [lo, hi] with p(k), for p false then true over [lo, hi];
// hi + 1 if p holds nowhere.  g is a guess of the answer: p is evaluated at g
// and its neighbour, and a binary search over the rest of the range runs only
// if the guess is off by more than one.  The answer never depends on g.
template <class Pred>
__device__ __forceinline__ int first_true(int lo, int hi, int g, Pred p) {
  g = min(max(g, lo), hi);
  int a, b;  // answer in [a, b]; b == hi + 1 stands for "nowhere"
  if (p(g)) {
    if (g == lo || !p(g - 1)) return g;
    a = lo;
    b = g - 1;
  } else {
    if (g == hi) return hi + 1;
    if (p(g + 1)) return g + 1;
    a = g + 2;
    b = hi + 1;
  }
  while (a < b) {
    const int m = (a + b) >> 1;
    if (p(m)) b = m;
    else a = m + 1;
  }
  return a;
}

// Guess of the first k at which o + (k/K) d crosses the line value w,
// rounded up; any int if the crossing is undefined.
__device__ __forceinline__ int crossing_guess(float o, float d, float w, int K) {
  const double k = ((double)w - (double)o) * (double)K / (double)d;
  return (k > -1.0 && k < 2.0e9) ? (int)ceil(k) : 1;
}

// Range [lo, hi] of k in [1, K-1] where 0 <= f(k) < lim, for f monotone in k
// (non-decreasing if inc).  Empty range: lo > hi.
template <bool kIsX>
__device__ __forceinline__ void axis_range(const Ray& r, int K, float inv_r, float lim, bool inc,
                                           int& lo, int& hi) {
  auto in = [&](int k) {
    const float v = f_of<kIsX>(r, k, inv_r);
    return v >= 0.0f && v < lim;
  };
  lo = 1;
  hi = K - 1;
  if (in(lo) && in(hi)) return;
  // "v >= 0" and "v < lim" are each monotone in k.  P(k) = (inc ? f >= 0 :
  // f < lim) turns true once; Q(k) = (inc ? f < lim : f >= 0) turns false
  // once.  The guesses come from the real line o + (k/K) d in metres.
  const float o = kIsX ? r.ox : r.oy;
  const float d = kIsX ? r.dx : r.dy;
  const float wlim = lim / inv_r;
  auto P = [&](int k) {
    const float v = f_of<kIsX>(r, k, inv_r);
    return inc ? (v >= 0.0f) : (v < lim);
  };
  auto notQ = [&](int k) {
    const float v = f_of<kIsX>(r, k, inv_r);
    return inc ? !(v < lim) : !(v >= 0.0f);
  };
  lo = first_true(1, K - 1, crossing_guess(o, d, inc ? 0.0f : wlim, K), P);
  hi = first_true(1, K - 1, crossing_guess(o, d, inc ? wlim : 0.0f, K), notQ) - 1;
}

// Lowers *a to v if v is smaller (v not NaN), as an integer atomic on the
// float's bits: non-negative floats order like their bits as signed
// integers, negative ones inversely to their bits as unsigned integers, and
// every negative float's bits exceed every non-negative one's.
__device__ __forceinline__ void atomic_min_f32(float* a, float v) {
  if (!signbit(v)) atomicMin(reinterpret_cast<int*>(a), __float_as_int(v));
  else atomicMax(reinterpret_cast<unsigned int*>(a), __float_as_uint(v));
}

// A cell can be removed only if it is valid, older than the minimum age and
// has a normal (its validity, update time and normal z given).
__device__ __forceinline__ bool clearable(const Item& it, uint8_t valid, int32_t t_upd, float nz) {
  return valid && (((int64_t)it.t_now - (int64_t)t_upd) > (int64_t)it.c.tau) && !isnan(nz);
}

// Removal of a cell: back to the prior, invalid (physical index pc); flagged
// in the caller's mask (logical index lc).
__device__ __forceinline__ void clear_cell(const Item& it, int64_t pc, int lc) {
  it.L.h[pc] = it.c.h_init;
  it.L.v[pc] = it.c.v_init;
  it.L.valid[pc] = 0;
  if (it.out_cleared) it.out_cleared[lc] = 1;
}

// The removal test of sample q (height qz) in cell c, from the cell's
// clearing record {h, v}, written by the setup: one 8-byte load for the height
// test (which most samples fail), and the normal only when it passes.  A cell
// no ray may clear holds -inf, which fails hd > 0 for every finite sample
// height.  On maps with an upper bound layer, a cell without an estimate holds
// NaN in place of the height (no other record does), which sends the sample
// to its bound.
__device__ __forceinline__ void test_cell_rec(const Item& it, const Ray& r, int lc, int64_t pc,
                                              float qz, float an2dd, const float2 k) {
  if (isnan(k.x)) {
    atomic_min_f32(it.L.ub + pc, qz);
    return;
  }
  const float hd = k.x - qz;
  if (!(hd > 0.0f) || !((hd * hd) > k.y)) return;
  const float dot = (r.dx * it.L.nx[pc] + r.dy * it.L.ny[pc]) + r.dz * it.L.nz[pc];
  if ((dot * dot) > an2dd) clear_cell(it, pc, lc);
}

// The ray of point i of the item: origin, direction, sample count K and the
// end point's cell (or -1 outside).  False if the point casts no ray (not
// valid, too long a ray, or K < 2: no samples).  The setup and the march both
// build rays here, so a queued ray is rebuilt bit for bit from its point.
__device__ __forceinline__ bool ray_of(const Item& it, int64_t i, Ray& r, int& K, int& end_cell) {
  r.ox = it.P.t[0];
  r.oy = it.P.t[1];
  r.oz = it.P.t[2];
  const PointEval e = eval_point(it.P, it.c, it.x[i], it.y[i], it.z[i]);
  r.dx = e.xm - r.ox;
  r.dy = e.ym - r.oy;
  r.dz = e.zm - r.oz;
  const float m = fmaxf(fabsf(r.dx), fabsf(r.dy));
  const float ks = m * it.c.inv_step;
  if (!e.valid || !(ks < 16777216.0f)) return false;
  K = (int)ceilf(ks);
  if (K < 2) return false;
  r.rK = 1.0 / (double)K;
  int ex, ey;
  end_cell = bin_xy(e.xm, e.ym, it.c, ex, ey) ? ey * it.c.nx + ex : -1;
  return true;
}

constexpr int kUnroll = 8;

// Test samples k in [ka, kb] of ray r against the map; cm holds the block
// maxima.  kUnroll samples at a time: their cells and blocks are found without
// branches, then the block maxima are loaded together, one load per change of
// block along the ray (a ray spends about five samples in a block of 8 x 8
// cells).  The per-sample work is kept to the sample itself.
__device__ __forceinline__ void march_range(const Item& it, const Ray& r, int ka, int kb,
                                            int end_cell, const float* cm) {
  const float an2dd = it.c.an2 * ((r.dx * r.dx + r.dy * r.dy) + r.dz * r.dz);
  const int bl = it.bl;
  const int bx = it.bx;
  const float inv_r = it.c.inv_r;
  const int nx = it.c.nx;
  uint32_t pblk = 0xFFFFFFFFu;  // the block of the previous sample, and its maximum
  float pm = 0.0f;
  for (int k = ka; k <= kb; k += kUnroll) {
    int cell[kUnroll];     // logical: the end-cell test, the records
    int64_t pc[kUnroll];   // physical: the layers
    uint32_t blk[kUnroll];
    float qz[kUnroll];
    float m[kUnroll];
    bool cand[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      // [ka, kb] lies in the ray's in-map range, which the setup found with
      // this very evaluation (f_of): qx * inv_r and qy * inv_r are in [0, nx)
      // and [0, ny), so truncation is floor and the cell is in the map.  The
      // unused slots past kb evaluate sample kb again, so they stay in the map
      // too; they are never candidates.
      const float t = t_of(r, min(k + u, kb));
      const float qx = r.ox + t * r.dx;
      const float qy = r.oy + t * r.dy;
      qz[u] = r.oz + t * r.dz;
      const int ix = (int)(qx * inv_r);
      const int iy = (int)(qy * inv_r);
      cell[u] = iy * nx + ix;
      pc[u] = pcell(it.c, ix, iy);
      blk[u] = (uint32_t)((iy >> bl) * bx + (ix >> bl));
    }
    // the block maxima where the block changes, every load issued before any
    // is used; the other slots take their predecessor's
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      m[u] = 0.0f;
      if (blk[u] != (u ? blk[u - 1] : pblk)) m[u] = cm[blk[u]];
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u)
      if (blk[u] == (u ? blk[u - 1] : pblk)) m[u] = u ? m[u - 1] : pm;
    pblk = blk[kUnroll - 1];
    pm = m[kUnroll - 1];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u)
      cand[u] = (k + u <= kb) & (qz[u] < m[u]) & (cell[u] != end_cell);
    // the candidates' records, all requested before any is tested
    float2 rec[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      rec[u] = make_float2(-INFINITY, 0.0f);
      if (cand[u]) rec[u] = it.L.clr[cell[u]];
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      if (!cand[u]) continue;
      test_cell_rec(it, r, cell[u], pc[u], qz[u], an2dd, rec[u]);
    }
  }
}

// Setup work unit `unit` of item `it`; `qsel` picks the sub-queue.
__device__ __forceinline__ void setup_body(const Item& it, int unit, int qsel) {
  const int lane = threadIdx.x & 63;
  // the next plain call's queue counters start from zero
  if (unit == 0 && it.cq.counter_next && threadIdx.x <= kSubQ)
    it.cq.counter_next[threadIdx.x * kCtrStride] = 0u;
  if (unit < it.nprep) {
    // ---- block role: each wave takes it.bpw (1 or 4) blocks of 8 x 8 cells,
    // one cell of each per lane, so their loads are in flight together
    const int b0 = (unit * (kNTc / 64) + (threadIdx.x >> 6)) * it.bpw;
    const int side = 1 << it.bl;
    int64_t c[kMaxBlocksPerWave];   // logical cell: the mask, the records
    int64_t p[kMaxBlocksPerWave];   // physical cell: the layers
    bool inside[kMaxBlocksPerWave], ok[kMaxBlocksPerWave];
    float h[kMaxBlocksPerWave], v[kMaxBlocksPerWave];
#pragma unroll
    for (int j = 0; j < kMaxBlocksPerWave; ++j) {
      const int b = b0 + j;
      const int ix = ((b % it.bx) << it.bl) + (lane & (side - 1));
      const int iy = ((b / it.bx) << it.bl) + (lane >> it.bl);
      inside[j] = j < it.bpw && b < it.nb && ix < it.c.nx && iy < it.c.ny;
      c[j] = inside[j] ? (int64_t)iy * it.c.nx + ix : 0;
      p[j] = inside[j] ? pcell(it.c, ix, iy) : 0;
    }
    // two rounds of loads for all of the wave's blocks, not one round per
    // test: first the validity, then what a valid cell's tests need (update
    // time, normal z, height), or a cell without an estimate's bound.  Cells
    // that cannot matter load nothing more (cell 0 stands in for cells
    // outside the map).
    uint8_t vd[kMaxBlocksPerWave];
    int32_t tu[kMaxBlocksPerWave];
    float nz[kMaxBlocksPerWave], ubv[kMaxBlocksPerWave];
#pragma unroll
    for (int j = 0; j < kMaxBlocksPerWave; ++j)
      vd[j] = (j < it.bpw && inside[j]) ? it.L.valid[p[j]] : 0;
#pragma unroll
    for (int j = 0; j < kMaxBlocksPerWave; ++j) {
      tu[j] = 0;
      nz[j] = 0.0f;
      h[j] = 0.0f;
      ubv[j] = INFINITY;
      if (vd[j]) {
        tu[j] = it.L.t[p[j]];
        nz[j] = it.L.nz[p[j]];
        h[j] = it.L.h[p[j]];
      } else if (it.L.ub && inside[j]) {
        ubv[j] = it.L.ub[p[j]];
      }
    }
#pragma unroll
    for (int j = 0; j < kMaxBlocksPerWave; ++j) {
      if (inside[j] && it.out_cleared) it.out_cleared[c[j]] = 0;  // the march sets removals
      ok[j] = inside[j] && clearable(it, vd[j], tu[j], nz[j]);
      v[j] = ok[j] ? h[j] : -INFINITY;
      // with an upper bound layer, a sample below the bound of a cell without
      // an estimate lowers it: such cells take part in the maximum too
      if (it.L.ub && inside[j] && !vd[j]) v[j] = ubv[j];
    }
#pragma unroll
    for (int j = 0; j < kMaxBlocksPerWave; ++j) {
      if (j >= it.bpw) break;
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) v[j] = fmaxf(v[j], __shfl_xor(v[j], o, 64));
      if (lane == 0 && b0 + j < it.nb) it.L.cmax[b0 + j] = v[j];
      // the march reads records only in blocks with a removable cell, where
      // some sample may pass below the block maximum
      if (v[j] > -INFINITY && inside[j]) {
        // a NaN height can never be cleared (hd > 0 fails), so -inf serves
        const bool bound = it.L.ub && !vd[j];
        const float hx = bound ? __builtin_nanf("") : (ok[j] && !isnan(h[j]) ? h[j] : -INFINITY);
        it.L.clr[c[j]] = make_float2(hx, it.L.v[p[j]]);
      }
    }
    return;
  }
  // ---- ray role: the ray's in-map sample range, queued in segments
  const int64_t i = (int64_t)(unit - it.nprep) * kNTc + threadIdx.x;
  int k0 = 1, k1 = 0;
  if (i < it.n) {
    Ray r;
    int K, end_cell;
    if (ray_of(it, i, r, K, end_cell)) {
      int lx, hx, ly, hy;
      axis_range<true>(r, K, it.c.inv_r, it.c.nxf, r.dx >= 0.0f, lx, hx);
      axis_range<false>(r, K, it.c.inv_r, it.c.nyf, r.dy >= 0.0f, ly, hy);
      k0 = max(lx, ly);
      k1 = min(hx, hy);
    }
  }
  const int seg = it.cq.seg;
  const int ns = k1 >= k0 ? k1 - k0 + 1 : 0;
  const int nseg = (ns + seg - 1) / seg;
  // one reservation per workgroup, in the sub-queue this workgroup maps to
  __shared__ int s_isum[kNTc / 64];
  __shared__ uint32_t s_base;
  int wtot = 0;
  const int off = block_exclusive_sum<kNTc>(nseg, wtot, s_isum);
  const int sub = qsel % kSubQ;
  const ClearQueue& cq = it.cq;
  if (threadIdx.x == 0)
    s_base = wtot > 0 ? atomicAdd(cq.counter + sub * kCtrStride, (uint32_t)wtot) : 0u;
  __syncthreads();
  if (nseg == 0) return;
  const int64_t first = (int64_t)s_base + off;
  uint2* q = cq.queue + (int64_t)sub * cq.qcap;
  const int64_t gray = it.ray_base + i;
  if (first + nseg <= cq.qcap) {
    for (int sgi = 0; sgi < nseg; ++sgi) {
      const int ka = k0 + sgi * seg;
      const int cnt = min(seg, k1 - ka + 1);
      q[first + sgi] = make_uint2((uint32_t)gray, ((uint32_t)ka << 8) | (uint32_t)cnt);
    }
  } else {
    // sub-queue full: leave empty entries in any reserved slots; the whole
    // ray goes to the overflow list, marched after the queue
    for (int64_t e = first; e < first + nseg && e < cq.qcap; ++e) q[e] = make_uint2(0u, 0u);
    const uint32_t o = atomicAdd(cq.counter + kOverCtr, 1u);
    cq.over[o] = make_uint4((uint32_t)gray, (uint32_t)k0, (uint32_t)k1, 0u);
  }
}

// Prefix of the sub-queue fill levels (kSubQ == 64: the first wave).
__device__ __forceinline__ void queue_prefix(const ClearQueue& cq, int64_t* s_qoff) {
  if (threadIdx.x < 64) {
    const int64_t c = min((int64_t)cq.counter[threadIdx.x * kCtrStride], cq.qcap);
    int64_t x = c;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int64_t y = __shfl_up(x, o, 64);
      if ((int)threadIdx.x >= o) x += y;
    }
    s_qoff[threadIdx.x + 1] = x;
    if (threadIdx.x == 0) s_qoff[0] = 0;
  }
}

// Queue entry g (over all sub-queues) and the ray it names.
__device__ __forceinline__ uint2 queue_entry(const ClearQueue& cq, const int64_t* s_qoff,
                                             int64_t g) {
  int lo = 0, hi = kSubQ - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (s_qoff[mid] <= g) lo = mid;
    else hi = mid - 1;
  }
  return cq.queue[(int64_t)lo * cq.qcap + (g - s_qoff[lo])];
}

// Samples [ka, kb] of queued ray g (the item's point g - ray_base).
__device__ __forceinline__ void march_ray(const Item& it, uint32_t g, int ka, int kb,
                                          const float* cm) {
  Ray r;
  int K, end_cell;
  if (!ray_of(it, (int64_t)g - it.ray_base, r, K, end_cell)) return;  // never for a queued ray
  march_range(it, r, ka, kb, end_cell, cm);
}

__device__ __forceinline__ void march_entry(const Item& it, uint2 e, const float* cm) {
  const int cnt = (int)(e.y & 255u);
  if (cnt == 0) return;
  const int ka = (int)(e.y >> 8);
  march_ray(it, e.x, ka, ka + cnt - 1, cm);
}

// Item of global ray g in a batch: the last item whose first ray is <= g
// (items without rays are skipped over).  s_rays holds the batch's prefix.
__device__ __forceinline__ int ray_item(const int64_t* s_rays, int n, int64_t g) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (s_rays[mid] <= g) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// ---------------------------------------------------------------- launches
__global__ __launch_bounds__(kNTc) void k_clear_setup(Item it) {
  setup_body(it, blockIdx.x, (int)blockIdx.x - it.nprep);
}

// The block maxima are read through the caches: they are small and shared by
// every workgroup, and staging them in LDS per workgroup costs more than it saves.
__global__ __launch_bounds__(kNTc) void k_clear_march(Item it) {
  __shared__ int64_t s_qoff[kSubQ + 1];
  queue_prefix(it.cq, s_qoff);
  __syncthreads();
  const int64_t total = s_qoff[kSubQ];
  for (int64_t g = (int64_t)blockIdx.x * kNTc + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * kNTc)
    march_entry(it, queue_entry(it.cq, s_qoff, g), it.L.cmax);
  // then the rays that overflowed their sub-queue, whole
  const uint32_t nover = it.cq.counter[kOverCtr];
  for (int64_t g = (int64_t)blockIdx.x * kNTc + threadIdx.x; g < nover;
       g += (int64_t)gridDim.x * kNTc) {
    const uint4 o = it.cq.over[g];
    march_ray(it, o.x, (int)o.y, (int)o.z, it.L.cmax);
  }
}


__global__ __launch_bounds__(kNTc) void k_clear_setup_b(const Batch* bt) {
  const int64_t total = bt->off[kBSetup][bt->n];
  for (int64_t w = blockIdx.x; w < total; w += gridDim.x) {
    const int i = batch_item(bt, kBSetup, w);
    setup_body(bt->items[i], (int)(w - bt->off[kBSetup][i]), (int)w);
    __syncthreads();
  }
}

// Every item of a batch shares one queue (the first item's view of it); a
// queue entry's global ray index names its item.
__global__ __launch_bounds__(kNTc) void k_clear_march_b(const Batch* bt) {
  __shared__ int64_t s_qoff[kSubQ + 1];
  __shared__ int64_t s_rays[kMaxItems + 1];
  const ClearQueue& cq = bt->items[0].cq;
  const int n = bt->n;
  queue_prefix(cq, s_qoff);
  for (int k = threadIdx.x; k <= n; k += kNTc) s_rays[k] = bt->rays[k];
  __syncthreads();
  const int64_t total = s_qoff[kSubQ];
  for (int64_t g = (int64_t)blockIdx.x * kNTc + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * kNTc) {
    const uint2 e = queue_entry(cq, s_qoff, g);
    if ((e.y & 255u) == 0) continue;
    const Item& it = bt->items[ray_item(s_rays, n, e.x)];
    march_entry(it, e, it.L.cmax);
  }
  const uint32_t nover = cq.counter[kOverCtr];
  for (int64_t g = (int64_t)blockIdx.x * kNTc + threadIdx.x; g < nover;
       g += (int64_t)gridDim.x * kNTc) {
    const uint4 o = cq.over[g];
    const Item& it = bt->items[ray_item(s_rays, n, o.x)];
    march_ray(it, o.x, (int)o.y, (int)o.z, it.L.cmax);
  }
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

// Room for kQueueSamplesPerRay samples per ray on average plus two partial
// segments per ray (a ray's range rarely ends on a segment boundary), and
// slack for uneven sub-queue fill.  A full sub-queue is not an error: its
// rays go to the overflow list (room for every ray) and are marched whole.
int64_t clear_queue_cap(int64_t max_points, int seg) {
  const int64_t segs = (max_points * kQueueSamplesPerRay + seg - 1) / seg + 2 * max_points;
  return (segs + segs / 8 + kSubQ - 1) / kSubQ;
}

size_t clear_scratch_layout(int64_t max_points, int seg, char* base, ClearQueue* out) {
  const size_t n = (size_t)max_points;
  const size_t qcap = (size_t)clear_queue_cap(max_points, seg);
  size_t off = 0;
  const size_t o_q = off;
  off = align256(off + (size_t)kSubQ * qcap * sizeof(uint2));
  const size_t o_over = off;
  off = align256(off + n * sizeof(uint4));
  if (out && base) {
    out->queue = (uint2*)(base + o_q);
    out->over = (uint4*)(base + o_over);
    out->qcap = (int64_t)qcap;
    out->seg = seg;
  }
  return off;
}

hipError_t launch_clear(const Item& it, int march_grid, hipStream_t stream, bool* ran) {
  *ran = false;
  // with no rays the setup still zeroes the caller's mask (block role only)
  if (it.n <= 0 && !it.out_cleared) return hipSuccess;
  const unsigned nray = it.n > 0 ? (unsigned)((it.n + kNTc - 1) / kNTc) : 0u;
  {
    TimedLaunch tl("k_clear_setup", stream);
    hipLaunchKernelGGL(k_clear_setup, dim3((unsigned)it.nprep + nray), dim3(kNTc), 0, stream, it);
  }
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  *ran = true;
  if (it.n <= 0) return hipSuccess;
  TimedLaunch tl("k_clear_march", stream);
  hipLaunchKernelGGL(k_clear_march, dim3((unsigned)march_grid), dim3(kNTc), 0, stream, it);
  return hipGetLastError();
}

int clear_setup_units(int64_t n, int nprep, bool mask) {
  return n > 0 ? nprep + (int)((n + kNTc - 1) / kNTc) : (mask ? nprep : 0);
}
int clear_blocks_per_wave(int nb) { return nb >= 4096 ? kMaxBlocksPerWave : 1; }
int clear_block_units(int nb) {
  const int per = (kNTc / 64) * clear_blocks_per_wave(nb);
  return (nb + per - 1) / per;
}

hipError_t launch_clear_batch(const Batch* d_batch, int grid_setup, int grid_march,
                              hipStream_t stream) {
  {
    TimedLaunch tl("k_clear_setup_b", stream);
    hipLaunchKernelGGL(k_clear_setup_b, dim3(grid_setup), dim3(kNTc), 0, stream, d_batch);
  }
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  {
    TimedLaunch tl("k_clear_march_b", stream);
    hipLaunchKernelGGL(k_clear_march_b, dim3(grid_march), dim3(kNTc), 0, stream, d_batch);
  }
  return hipGetLastError();
}

}  // namespace emx
