// Visibility clean-up by ray casting (Sec. II-E, Eq. 3 and Eq. 4).
//
// k_clear_march: one thread per point.  The thread walks the samples of the
// sensor->point ray and marks every cell that the ray passes below.
//   - The samples are q_k = o + (k/K) d for k = 1..K-1, in float32.
//   - A sample's cell is in the map over a contiguous range of k, because
//     q_k.x and q_k.y are monotone in k: each is a correctly rounded chain of
//     monotone operations.  So the thread first finds that range exactly,
//     using the very sample evaluation it then loops over.  Rays reaching far
//     beyond the map cost only their in-map samples.
//   - Marks are idempotent byte stores: no atomics, no ordering.
//   - The state is only read, so every ray sees the state as it was when the
//     call started.
// k_clear_apply: one pass over the cells.  It resets marked cells to the prior,
// reports the marks and clears them for the next call.
#include "emx_kernels.h"

namespace emx {

namespace {

constexpr int kNTc = 256;

struct Ray {
  float ox, oy, oz;
  float dx, dy, dz;
  float Kf;
};

__device__ __forceinline__ void sample(const Ray& r, int k, float& qx, float& qy, float& qz) {
  const float t = (float)k / r.Kf;
  qx = r.ox + t * r.dx;
  qy = r.oy + t * r.dy;
  qz = r.oz + t * r.dz;
}

// f(k) = q_k.x * inv_r, exactly as binning computes it
__device__ __forceinline__ float fx_of(const Ray& r, int k, float inv_r) {
  const float t = (float)k / r.Kf;
  return (r.ox + t * r.dx) * inv_r;
}
__device__ __forceinline__ float fy_of(const Ray& r, int k, float inv_r) {
  const float t = (float)k / r.Kf;
  return (r.oy + t * r.dy) * inv_r;
}

// Range [lo, hi] of k in [1, K-1] where 0 <= f(k) < lim, for f monotone in k
// (non-decreasing if inc).  Empty range: lo > hi.
template <bool kIsX>
__device__ __forceinline__ void axis_range(const Ray& r, int K, float inv_r, float lim, bool inc,
                                           int& lo, int& hi) {
  auto f = [&](int k) { return kIsX ? fx_of(r, k, inv_r) : fy_of(r, k, inv_r); };
  auto in = [&](int k) {
    const float v = f(k);
    return v >= 0.0f && v < lim;
  };
  lo = 1;
  hi = K - 1;
  if (in(lo) && in(hi)) return;
  // "v >= 0" and "v < lim" are each monotone; find where each holds.
  if (inc) {
    // v >= 0 turns true at some k; v < lim turns false at some k
    int a = 1, b = K;  // first k with f(k) >= 0, K if none
    while (a < b) {
      const int m = (a + b) >> 1;
      if (f(m) >= 0.0f) b = m;
      else a = m + 1;
    }
    lo = a;
    a = 0;
    b = K - 1;  // last k with f(k) < lim, 0 if none
    while (a < b) {
      const int m = (a + b + 1) >> 1;
      if (f(m) < lim) a = m;
      else b = m - 1;
    }
    hi = a;
  } else {
    int a = 1, b = K;  // first k with f(k) < lim
    while (a < b) {
      const int m = (a + b) >> 1;
      if (f(m) < lim) b = m;
      else a = m + 1;
    }
    lo = a;
    a = 0;
    b = K - 1;  // last k with f(k) >= 0
    while (a < b) {
      const int m = (a + b + 1) >> 1;
      if (f(m) >= 0.0f) a = m;
      else b = m - 1;
    }
    hi = a;
  }
}

struct MarchArgs {
  const float* x;
  const float* y;
  const float* z;
  int64_t n;
  Pose32 P;
  Consts c;
  Layers L;
  int32_t t_now;
  int bl;      // block side 2^bl cells
  int bx, nb;  // blocks per map row, blocks in the map
};

// A cell can be removed only if it is valid, older than the minimum age and
// has a normal.  cmax[b] is the largest height of such a cell in block b
// (-inf if none).  A sample at height q.z >= cmax[b] passes above every cell
// of the block that could be removed (removal needs h > q.z), so the march
// skips it without reading the cell.  This is exact pruning.
__device__ __forceinline__ bool clearable(const Layers& L, int64_t c, int32_t t_now, int32_t tau) {
  return L.valid[c] && (((int64_t)t_now - (int64_t)L.t[c]) > (int64_t)tau) && !isnan(L.nz[c]);
}

struct PrepArgs {
  Consts c;
  Layers L;
  int32_t t_now;
  int bl, bx, by;
};

// One wave per block of 2^bl x 2^bl cells.
__global__ __launch_bounds__(kNTc) void k_clear_prep(PrepArgs a) {
  const int lane = threadIdx.x & 63;
  const int b = blockIdx.x * (kNTc / 64) + (threadIdx.x >> 6);
  if (b >= a.bx * a.by) return;  // whole wave leaves together
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
}

constexpr int kUnroll = 4;

__global__ __launch_bounds__(kNTc) void k_clear_march(MarchArgs a) {
  extern __shared__ float s_cmax[];
  for (int j = threadIdx.x; j < a.nb; j += kNTc) s_cmax[j] = a.L.cmax[j];
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * kNTc + threadIdx.x;
  if (i >= a.n) return;
  const PointEval e = eval_point(a.P, a.c, a.x[i], a.y[i], a.z[i]);
  if (!e.valid) return;
  Ray r;
  r.ox = a.P.t[0];
  r.oy = a.P.t[1];
  r.oz = a.P.t[2];
  r.dx = e.xm - r.ox;
  r.dy = e.ym - r.oy;
  r.dz = e.zm - r.oz;
  const float m = fmaxf(fabsf(r.dx), fabsf(r.dy));
  const float ks = m * a.c.inv_step;
  if (!(ks < 16777216.0f)) return;
  const int K = (int)ceilf(ks);
  if (K < 2) return;
  r.Kf = (float)K;
  int ex = -1, ey = -1;
  const bool end_in = bin_xy(e.xm, e.ym, a.c, ex, ey);
  const int end_cell = end_in ? ey * a.c.nx + ex : -1;

  int lx, hx, ly, hy;
  axis_range<true>(r, K, a.c.inv_r, a.c.nxf, r.dx >= 0.0f, lx, hx);
  axis_range<false>(r, K, a.c.inv_r, a.c.nyf, r.dy >= 0.0f, ly, hy);
  const int k0 = max(lx, ly);
  const int k1 = min(hx, hy);

  const float an2dd = a.c.an2 * ((r.dx * r.dx + r.dy * r.dy) + r.dz * r.dz);
  const int bl = a.bl;
  for (int k = k0; k <= k1; k += kUnroll) {
    int cell[kUnroll];
    float qz[kUnroll];
    bool hit[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      float qx, qy;
      sample(r, k + u, qx, qy, qz[u]);
      int ix, iy;
      cell[u] = -1;
      hit[u] = false;
      if (k + u <= k1 && bin_xy(qx, qy, a.c, ix, iy)) {
        cell[u] = iy * a.c.nx + ix;
        hit[u] = qz[u] < s_cmax[(iy >> bl) * a.bx + (ix >> bl)];
      }
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      if (!hit[u] || cell[u] == end_cell) continue;
      const int c = cell[u];
      // one round trip: every field the test may need
      const uint8_t vc = a.L.valid[c];
      const int32_t tc = a.L.t[c];
      const float hc = a.L.h[c];
      const float varc = a.L.v[c];
      const float nxc = a.L.nx[c];
      const float nyc = a.L.ny[c];
      const float nzc = a.L.nz[c];
      const float hd = hc - qz[u];
      if (!vc || !(((int64_t)a.t_now - (int64_t)tc) > (int64_t)a.c.tau) || isnan(nzc)) continue;
      if (!(hd > 0.0f) || !((hd * hd) > varc)) continue;
      const float dot = (r.dx * nxc + r.dy * nyc) + r.dz * nzc;
      if ((dot * dot) > an2dd) a.L.mark[c] = 1;
    }
  }
}

struct ApplyArgs {
  Consts c;
  Layers L;
  int64_t cells;
  uint8_t* out;
};

__global__ __launch_bounds__(kNTc) void k_clear_apply(ApplyArgs a) {
  const int64_t i = (int64_t)blockIdx.x * kNTc + threadIdx.x;
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

}  // namespace

hipError_t launch_clear(const float* x, const float* y, const float* z, int64_t n,
                        const Pose32& P, const Consts& c, const Layers& L, int32_t t_now,
                        uint8_t* out_cleared, hipStream_t stream) {
  const int64_t cells = (int64_t)c.nx * c.ny;
  if (n > 0) {
    PrepArgs pa;
    pa.c = c;
    pa.L = L;
    pa.t_now = t_now;
    pa.bl = block_log_of(c.nx, c.ny);
    pa.bx = blocks_of(c.nx, pa.bl);
    pa.by = blocks_of(c.ny, pa.bl);
    const int nb = pa.bx * pa.by;
    hipLaunchKernelGGL(k_clear_prep, dim3((nb + kNTc / 64 - 1) / (kNTc / 64)), dim3(kNTc), 0,
                       stream, pa);
    hipError_t err0 = hipGetLastError();
    if (err0 != hipSuccess) return err0;
    MarchArgs a;
    a.x = x;
    a.y = y;
    a.z = z;
    a.n = n;
    a.P = P;
    a.c = c;
    a.L = L;
    a.t_now = t_now;
    a.bl = pa.bl;
    a.bx = pa.bx;
    a.nb = nb;
    hipLaunchKernelGGL(k_clear_march, dim3((unsigned)((n + kNTc - 1) / kNTc)), dim3(kNTc),
                       (size_t)nb * sizeof(float), stream, a);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
  }
  ApplyArgs b;
  b.c = c;
  b.L = L;
  b.cells = cells;
  b.out = out_cleared;
  hipLaunchKernelGGL(k_clear_apply, dim3((unsigned)((cells + kNTc - 1) / kNTc)), dim3(kNTc), 0,
                     stream, b);
  return hipGetLastError();
}

}  // namespace emx
