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
};

__global__ __launch_bounds__(kNTc) void k_clear_march(MarchArgs a) {
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
  const int32_t t_now = a.t_now;
  for (int k = k0; k <= k1; ++k) {
    float qx, qy, qz;
    sample(r, k, qx, qy, qz);
    int ix, iy;
    if (!bin_xy(qx, qy, a.c, ix, iy)) continue;
    const int cell = iy * a.c.nx + ix;
    if (cell == end_cell) continue;
    if (!a.L.valid[cell]) continue;
    const float hd = a.L.h[cell] - qz;
    if (!(hd > 0.0f)) continue;
    if (!((hd * hd) > a.L.v[cell])) continue;
    if (!(((int64_t)t_now - (int64_t)a.L.t[cell]) > (int64_t)a.c.tau)) continue;
    const float nz = a.L.nz[cell];
    if (isnan(nz)) continue;
    const float dot = (r.dx * a.L.nx[cell] + r.dy * a.L.ny[cell]) + r.dz * nz;
    if ((dot * dot) > an2dd) a.L.mark[cell] = 1;
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
    MarchArgs a;
    a.x = x;
    a.y = y;
    a.z = z;
    a.n = n;
    a.P = P;
    a.c = c;
    a.L = L;
    a.t_now = t_now;
    hipLaunchKernelGGL(k_clear_march, dim3((unsigned)((n + kNTc - 1) / kNTc)), dim3(kNTc), 0,
                       stream, a);
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
