// Visibility clean-up by ray casting (Sec. II-E, Eq. 3 and Eq. 4).
//
// The samples of a ray are q_k = o + (k/K) d for k = 1..K-1, in float32.
// Their number varies from 0 to a few hundred per ray, so one thread per ray
// leaves the long rays on the critical path.  The work is therefore split in
// three launches:
//
// k_clear_setup, two roles in one grid:
//   - Block role: per block of 2^b x 2^b cells, the largest height of a cell
//     that a ray could still remove: valid, older than the minimum age, with a
//     normal.  It is -inf if there is none.
//   - Ray role, one thread per point:
//       - the ray's exact in-map range of k.  A sample's cell is in the map over
//         a contiguous range of k, because q_k.x and q_k.y are monotone in k:
//         each is a correctly rounded chain of monotone operations.  The range
//         is found by binary search with the very sample evaluation the march
//         uses.
//       - the range is cut into segments of kSeg samples.  Each workgroup
//         reserves its segments with one integer atomic, in one of kSubQ
//         sub-queues, so no counter is contended.  A ray that would overflow
//         its bounded sub-queue is marched in place instead.
// k_clear_march: a persistent grid drains the queue, one segment per thread.
//   - A sample at height q.z >= the block maximum passes above every cell that
//     could be removed, since removal needs h > q.z.  It is skipped without
//     reading the cell: exact pruning.
//   - Marks are idempotent byte stores, so the queue order never shows in the
//     result.
//   - The state is only read, so every ray sees the state as it was when the
//     call started.
// k_clear_apply: resets marked cells to the prior, reports and clears the
// marks, and rewinds the queue counters for the next call.
#include "emx_kernels.h"

namespace emx {

namespace {

constexpr int kNTc = 256;
constexpr int kSeg = 32;          // samples per queued segment
constexpr int kQueuePerRay = 4;   // queue capacity, in segments per point
constexpr int kSubQ = 64;         // sub-queues, each with its own counter
constexpr int kCtrStride = 32;    // counters 128 bytes apart

struct Ray {
  float ox, oy, oz;
  float dx, dy, dz;
  float Kf;
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
  // "v >= 0" and "v < lim" are each monotone in k: find where each holds.
  // P(k) = (inc ? f >= 0 : f < lim) turns true once; Q(k) = (inc ? f < lim :
  // f >= 0) turns false once.
  int a = 1, b = K;  // first k with P(k), K if none
  while (a < b) {
    const int m = (a + b) >> 1;
    const float v = f_of<kIsX>(r, m, inv_r);
    if (inc ? (v >= 0.0f) : (v < lim)) b = m;
    else a = m + 1;
  }
  lo = a;
  a = 0;
  b = K - 1;  // last k with Q(k), 0 if none
  while (a < b) {
    const int m = (a + b + 1) >> 1;
    const float v = f_of<kIsX>(r, m, inv_r);
    if (inc ? (v < lim) : (v >= 0.0f)) a = m;
    else b = m - 1;
  }
  hi = a;
}

// A cell can be removed only if it is valid, older than the minimum age and
// has a normal.
__device__ __forceinline__ bool clearable(const Layers& L, int64_t c, int32_t t_now, int32_t tau) {
  return L.valid[c] && (((int64_t)t_now - (int64_t)L.t[c]) > (int64_t)tau) && !isnan(L.nz[c]);
}

struct ClearArgs {
  const float* x;
  const float* y;
  const float* z;
  int64_t n;
  Pose32 P;
  Consts c;
  Layers L;
  int32_t t_now;
  int bl;          // block side 2^bl cells
  int bx, by, nb;  // blocks per map row / column / total
  int nprep;       // workgroups of the block role
  ClearScratch s;
  uint32_t* counter;  // kSubQ counters of queued segments, kCtrStride apart
  int64_t qcap;       // capacity of each sub-queue (segments)
};

// The full removal test of sample q (height qz) in cell c.
__device__ __forceinline__ void test_cell(const ClearArgs& a, const Ray& r, int c, float qz,
                                          float an2dd) {
  // one round trip: every field the test may need
  const uint8_t vc = a.L.valid[c];
  const int32_t tc = a.L.t[c];
  const float hc = a.L.h[c];
  const float varc = a.L.v[c];
  const float nxc = a.L.nx[c];
  const float nyc = a.L.ny[c];
  const float nzc = a.L.nz[c];
  const float hd = hc - qz;
  if (!vc || !(((int64_t)a.t_now - (int64_t)tc) > (int64_t)a.c.tau) || isnan(nzc)) return;
  if (!(hd > 0.0f) || !((hd * hd) > varc)) return;
  const float dot = (r.dx * nxc + r.dy * nyc) + r.dz * nzc;
  if ((dot * dot) > an2dd) a.L.mark[c] = 1;
}

constexpr int kUnroll = 4;

// Test samples k in [ka, kb] of ray r against the map.  cm holds the block
// maxima; with cm == nullptr every sample is tested (same result, no pruning).
// kUnroll samples at a time: their cells and block maxima are found without
// branches, so the block-maximum loads issue together.
__device__ __forceinline__ void march_range(const ClearArgs& a, const Ray& r, int ka, int kb,
                                            int end_cell, const float* cm) {
  const float an2dd = a.c.an2 * ((r.dx * r.dx + r.dy * r.dy) + r.dz * r.dz);
  const int bl = a.bl;
  for (int k = ka; k <= kb; k += kUnroll) {
    int cell[kUnroll];
    float qz[kUnroll];
    bool cand[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const float t = t_of(r, k + u);
      const float qx = r.ox + t * r.dx;
      const float qy = r.oy + t * r.dy;
      qz[u] = r.oz + t * r.dz;
      const float fx = qx * a.c.inv_r;
      const float fy = qy * a.c.inv_r;
      const bool in = (k + u <= kb) && fx >= 0.0f && fx < a.c.nxf && fy >= 0.0f && fy < a.c.nyf;
      const int ix = in ? (int)floorf(fx) : 0;
      const int iy = in ? (int)floorf(fy) : 0;
      cell[u] = iy * a.c.nx + ix;
      const float m = cm ? cm[(iy >> bl) * a.bx + (ix >> bl)] : INFINITY;
      cand[u] = in && (qz[u] < m) && cell[u] != end_cell;
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u)
      if (cand[u]) test_cell(a, r, cell[u], qz[u], an2dd);
  }
}

__global__ __launch_bounds__(kNTc) void k_clear_setup(ClearArgs a) {
  const int lane = threadIdx.x & 63;
  if ((int)blockIdx.x < a.nprep) {
    // ---- block role: one wave per block of cells
    const int b = blockIdx.x * (kNTc / 64) + (threadIdx.x >> 6);
    if (b >= a.nb) return;  // whole wave leaves together
    const int side = 1 << a.bl;
    const int x0 = (b % a.bx) << a.bl;
    const int y0 = (b / a.bx) << a.bl;
    float v = -INFINITY;
    for (int j = lane; j < side * side; j += 64) {
      const int ix = x0 + (j & (side - 1));
      const int iy = y0 + (j >> a.bl);
      if (ix < a.c.nx && iy < a.c.ny) {
        const int64_t c = (int64_t)iy * a.c.nx + ix;
        if (clearable(a.L, c, a.t_now, a.c.tau)) v = fmaxf(v, a.L.h[c]);
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    if (lane == 0) a.L.cmax[b] = v;
    return;
  }
  // ---- ray role
  const int64_t i = (int64_t)(blockIdx.x - a.nprep) * kNTc + threadIdx.x;
  Ray r;
  r.ox = a.P.t[0];
  r.oy = a.P.t[1];
  r.oz = a.P.t[2];
  r.dx = r.dy = r.dz = 0.0f;
  r.Kf = 1.0f;
  r.rK = 1.0;
  int k0 = 1, k1 = 0, end_cell = -1;
  if (i < a.n) {
    const PointEval e = eval_point(a.P, a.c, a.x[i], a.y[i], a.z[i]);
    r.dx = e.xm - r.ox;
    r.dy = e.ym - r.oy;
    r.dz = e.zm - r.oz;
    const float m = fmaxf(fabsf(r.dx), fabsf(r.dy));
    const float ks = m * a.c.inv_step;
    if (e.valid && ks < 16777216.0f) {
      const int K = (int)ceilf(ks);
      if (K >= 2) {
        r.Kf = (float)K;
        r.rK = 1.0 / (double)K;
        int ex, ey;
        if (bin_xy(e.xm, e.ym, a.c, ex, ey)) end_cell = ey * a.c.nx + ex;
        int lx, hx, ly, hy;
        axis_range<true>(r, K, a.c.inv_r, a.c.nxf, r.dx >= 0.0f, lx, hx);
        axis_range<false>(r, K, a.c.inv_r, a.c.nyf, r.dy >= 0.0f, ly, hy);
        k0 = max(lx, ly);
        k1 = min(hx, hy);
      }
    }
  }
  const int ns = k1 >= k0 ? k1 - k0 + 1 : 0;
  const int nseg = (ns + kSeg - 1) / kSeg;
  // one reservation per workgroup, in the sub-queue of this workgroup
  __shared__ int s_isum[kNTc / 64];
  __shared__ uint32_t s_base;
  int wtot = 0;
  const int off = block_exclusive_sum<kNTc>(nseg, wtot, s_isum);
  const int sub = (int)((blockIdx.x - a.nprep) % kSubQ);
  if (threadIdx.x == 0) s_base = wtot > 0 ? atomicAdd(a.counter + sub * kCtrStride, (uint32_t)wtot) : 0u;
  __syncthreads();
  if (nseg == 0) return;
  const int64_t first = (int64_t)s_base + off;
  uint2* q = a.s.queue + (int64_t)sub * a.qcap;
  if (first + nseg <= a.qcap) {
    a.s.ray[i] = make_float4(r.dx, r.dy, r.dz, r.Kf);
    a.s.ray_end[i] = end_cell;
    for (int sgi = 0; sgi < nseg; ++sgi) {
      const int ka = k0 + sgi * kSeg;
      const int cnt = min(kSeg, k1 - ka + 1);
      q[first + sgi] = make_uint2((uint32_t)i, ((uint32_t)ka << 8) | (uint32_t)cnt);
    }
  } else {
    // sub-queue full: leave empty entries in any reserved slots and march
    // here, unpruned (the block maxima are still being written by this launch)
    for (int64_t e = first; e < first + nseg && e < a.qcap; ++e) q[e] = make_uint2(0u, 0u);
    march_range(a, r, k0, k1, end_cell, nullptr);
  }
}

__global__ __launch_bounds__(kNTc) void k_clear_march(ClearArgs a) {
  extern __shared__ float s_cmax[];
  __shared__ int64_t s_qoff[kSubQ + 1];
  for (int j = threadIdx.x; j < a.nb; j += kNTc) s_cmax[j] = a.L.cmax[j];
  if (threadIdx.x < 64) {
    // prefix of the sub-queue fill levels (kSubQ == 64: one wave)
    const int64_t c = min((int64_t)a.counter[threadIdx.x * kCtrStride], a.qcap);
    int64_t x = c;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int64_t y = __shfl_up(x, o, 64);
      if ((int)threadIdx.x >= o) x += y;
    }
    s_qoff[threadIdx.x + 1] = x;
    if (threadIdx.x == 0) s_qoff[0] = 0;
  }
  __syncthreads();
  const int64_t total = s_qoff[kSubQ];
  Ray r;
  r.ox = a.P.t[0];
  r.oy = a.P.t[1];
  r.oz = a.P.t[2];
  for (int64_t g = (int64_t)blockIdx.x * kNTc + threadIdx.x; g < total;
       g += (int64_t)gridDim.x * kNTc) {
    int lo = 0, hi = kSubQ - 1;  // sub-queue holding global entry g
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (s_qoff[mid] <= g) lo = mid;
      else hi = mid - 1;
    }
    const uint2 e = a.s.queue[(int64_t)lo * a.qcap + (g - s_qoff[lo])];
    const int cnt = (int)(e.y & 255u);
    if (cnt == 0) continue;
    const int ka = (int)(e.y >> 8);
    const float4 d = a.s.ray[e.x];
    r.dx = d.x;
    r.dy = d.y;
    r.dz = d.z;
    r.Kf = d.w;
    r.rK = 1.0 / (double)d.w;
    march_range(a, r, ka, ka + cnt - 1, a.s.ray_end[e.x], s_cmax);
  }
}

struct ApplyArgs {
  Consts c;
  Layers L;
  int64_t cells;
  uint8_t* out;
  uint32_t* counter;
};

__global__ __launch_bounds__(kNTc) void k_clear_apply(ApplyArgs a) {
  const int64_t i = (int64_t)blockIdx.x * kNTc + threadIdx.x;
  if (i < kSubQ) a.counter[i * kCtrStride] = 0u;
  if (i >= a.cells) return;
  const uint8_t m = a.L.mark[i];
  if (a.out) a.out[i] = m;
  if (m) {
    a.L.h[i] = a.c.h_init;
    a.L.v[i] = a.c.v_init;
    a.L.valid[i] = 0;
    a.L.mark[i] = 0;
  }
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

size_t clear_scratch_layout(int64_t max_points, char* base, ClearScratch* out) {
  const size_t n = (size_t)max_points;
  size_t off = 0;
  const size_t o_ray = off;
  off = align256(off + n * sizeof(float4));
  const size_t o_end = off;
  off = align256(off + n * sizeof(int32_t));
  const size_t o_q = off;
  off = align256(off + (size_t)kSubQ * ((n * kQueuePerRay + kSubQ - 1) / kSubQ) * sizeof(uint2));
  if (out && base) {
    out->ray = (float4*)(base + o_ray);
    out->ray_end = (int32_t*)(base + o_end);
    out->queue = (uint2*)(base + o_q);
  }
  return off;
}

hipError_t launch_clear(const float* x, const float* y, const float* z, int64_t n,
                        const Pose32& P, const Consts& c, const Layers& L, int32_t t_now,
                        const ClearScratch& s, uint32_t* counter, uint8_t* out_cleared,
                        int march_grid, hipStream_t stream) {
  const int64_t cells = (int64_t)c.nx * c.ny;
  if (n > 0) {
    ClearArgs a;
    a.x = x;
    a.y = y;
    a.z = z;
    a.n = n;
    a.P = P;
    a.c = c;
    a.L = L;
    a.t_now = t_now;
    a.bl = block_log_of(c.nx, c.ny);
    a.bx = blocks_of(c.nx, a.bl);
    a.by = blocks_of(c.ny, a.bl);
    a.nb = a.bx * a.by;
    a.nprep = (a.nb + kNTc / 64 - 1) / (kNTc / 64);
    a.s = s;
    a.counter = counter;
    a.qcap = (n * kQueuePerRay + kSubQ - 1) / kSubQ;
    const unsigned nray = (unsigned)((n + kNTc - 1) / kNTc);
    hipLaunchKernelGGL(k_clear_setup, dim3((unsigned)a.nprep + nray), dim3(kNTc), 0, stream, a);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k_clear_march, dim3((unsigned)march_grid), dim3(kNTc),
                       (size_t)a.nb * sizeof(float), stream, a);
    err = hipGetLastError();
    if (err != hipSuccess) return err;
  }
  ApplyArgs b;
  b.c = c;
  b.L = L;
  b.cells = cells;
  b.out = out_cleared;
  b.counter = counter;
  hipLaunchKernelGGL(k_clear_apply, dim3((unsigned)((cells + kNTc - 1) / kNTc)), dim3(kNTc), 0,
                     stream, b);
  return hipGetLastError();
}

}  // namespace emx
