// Height drift compensation (Sec. II-D).
//
// The map's heights are shifted by the mean error between a frame's points and
// the map on flat ground, measured before the frame is fused.  Three launches:
//   1. per 1024-point chunk, the float64 sum of the errors and their count,
//      each thread summing its four points in index order and the workgroup
//      combining them by a fixed binary tree;
//   2. one workgroup combines the chunk partials by a fixed tree and writes the
//      mean and the count (to scratch and the optional outputs);
//   3. every valid cell adds the mean, rounded once to float32.
// The order of every sum depends only on the number of points, so the result
// is the same on every call.  The point decisions (transform, validity,
// binning) are the fusion's own, from the shared device helpers.
#include "emx_kernels.h"

namespace emx {

namespace {

constexpr int kNTd = 256;                 // threads per chunk workgroup
constexpr int kPerD = kChunk / kNTd;      // points per thread
constexpr int kNTr = 1024;                // threads of the combining workgroup
constexpr int kNTs = 256;                 // threads per shift workgroup

struct DriftResult {
  double mean;
  int64_t n;
};

struct DriftArgs {
  Item it;
  float trav_min;
  double* part_sum;     // [B]
  uint32_t* part_cnt;   // [B]
  DriftResult* res;
  double* out_mean;     // optional
  int64_t* out_count;   // optional
};

// Fixed-shape tree over nthreads values in LDS; thread 0 ends with the total.
template <int N>
__device__ __forceinline__ void tree_sum(double* s_sum, int64_t* s_cnt, int tid) {
#pragma unroll
  for (int stride = N / 2; stride > 0; stride >>= 1) {
    __syncthreads();
    if (tid < stride) {
      s_sum[tid] = s_sum[tid] + s_sum[tid + stride];
      s_cnt[tid] = s_cnt[tid] + s_cnt[tid + stride];
    }
  }
  __syncthreads();
}

__global__ __launch_bounds__(kNTd) void k_drift_partial(DriftArgs a) {
  __shared__ double s_sum[kNTd];
  __shared__ int64_t s_cnt[kNTd];
  const Item& it = a.it;
  const int tid = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * kChunk;
  double sum = 0.0;
  int64_t cnt = 0;
#pragma unroll
  for (int j = 0; j < kPerD; ++j) {
    const int64_t i = base + (int64_t)tid * kPerD + j;  // a thread's points in order
    if (i >= it.n) break;
    const PointEval e = eval_point(it.P, it.c, it.x[i], it.y[i], it.z[i]);
    int ix, iy;
    if (!e.valid || !bin_xy(e.xm, e.ym, it.c, ix, iy)) continue;
    const int64_t cell = (int64_t)iy * it.c.nx + ix;
    if (!it.L.valid[cell]) continue;
    const float tr = it.L.trav[cell];
    if (!(tr > a.trav_min)) continue;  // NaN traversability never passes
    sum = sum + ((double)e.zm - (double)it.L.h[cell]);
    ++cnt;
  }
  s_sum[tid] = sum;
  s_cnt[tid] = cnt;
  tree_sum<kNTd>(s_sum, s_cnt, tid);
  if (tid == 0) {
    a.part_sum[blockIdx.x] = s_sum[0];
    a.part_cnt[blockIdx.x] = (uint32_t)s_cnt[0];
  }
}

__global__ __launch_bounds__(kNTr) void k_drift_combine(DriftArgs a) {
  __shared__ double s_sum[kNTr];
  __shared__ int64_t s_cnt[kNTr];
  const int tid = threadIdx.x;
  double sum = 0.0;
  int64_t cnt = 0;
  for (int64_t b = tid; b < a.it.B; b += kNTr) {
    sum = sum + a.part_sum[b];
    cnt += a.part_cnt[b];
  }
  s_sum[tid] = sum;
  s_cnt[tid] = cnt;
  tree_sum<kNTr>(s_sum, s_cnt, tid);
  if (tid == 0) {
    const int64_t n = s_cnt[0];
    const double mean = n > 0 ? s_sum[0] / (double)n : 0.0;
    a.res->mean = mean;
    a.res->n = n;
    if (a.out_mean) *a.out_mean = mean;
    if (a.out_count) *a.out_count = n;
  }
}

__global__ __launch_bounds__(kNTs) void k_drift_shift(Layers L, int64_t cells,
                                                      const DriftResult* res) {
  const int64_t i = (int64_t)blockIdx.x * kNTs + threadIdx.x;
  if (i >= cells) return;
  const int64_t n = res->n;
  if (n <= 0 || !L.valid[i]) return;
  L.h[i] = L.h[i] + (float)res->mean;
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

size_t drift_scratch_layout(int64_t max_points, char* base, DriftScratch* out) {
  const int64_t B = (max_points + kChunk - 1) / kChunk;
  size_t off = 0;
  const size_t o_res = off;
  off = align256(off + sizeof(DriftResult));
  const size_t o_sum = off;
  off = align256(off + (size_t)B * sizeof(double));
  const size_t o_cnt = off;
  off = align256(off + (size_t)B * sizeof(uint32_t));
  if (out && base) {
    out->res = base + o_res;
    out->part_sum = (double*)(base + o_sum);
    out->part_cnt = (uint32_t*)(base + o_cnt);
  }
  return off;
}

hipError_t launch_drift(const Item& it, float trav_min, const DriftScratch& ds,
                        double* out_mean, int64_t* out_count, hipStream_t stream) {
  DriftArgs a;
  a.it = it;
  a.trav_min = trav_min;
  a.part_sum = ds.part_sum;
  a.part_cnt = ds.part_cnt;
  a.res = (DriftResult*)ds.res;
  a.out_mean = out_mean;
  a.out_count = out_count;
  hipError_t err;
  if (it.B > 0) {
    TimedLaunch tl("k_drift_partial", stream);
    hipLaunchKernelGGL(k_drift_partial, dim3(it.B), dim3(kNTd), 0, stream, a);
  }
  if ((err = hipGetLastError()) != hipSuccess) return err;
  {
    TimedLaunch tl("k_drift_combine", stream);
    hipLaunchKernelGGL(k_drift_combine, dim3(1), dim3(kNTr), 0, stream, a);
  }
  if ((err = hipGetLastError()) != hipSuccess) return err;
  const int64_t cells = (int64_t)it.c.nx * it.c.ny;
  {
    TimedLaunch tl("k_drift_shift", stream);
    hipLaunchKernelGGL(k_drift_shift, dim3((unsigned)((cells + kNTs - 1) / kNTs)), dim3(kNTs),
                       0, stream, it.L, cells, (const DriftResult*)ds.res);
  }
  return hipGetLastError();
}

}  // namespace emx
