// Height drift compensation (Sec. II-D).
//
// The map's heights are shifted by the mean error between a frame's points and
// the map on flat ground, measured before the frame is fused.  Three launches:
//   1. per 1024-point chunk, the float64 sum of the errors and their count,
//      each thread summing its four points (256 apart) in index order and the
//      workgroup combining them by a fixed butterfly;
//   2. one workgroup combines the chunk partials in the same fixed way and
//      writes the mean and the count (to scratch and the optional outputs).
//      It is a launch of its own: handing the partials to a last workgroup
//      inside launch 1 needs an agent-scope release per workgroup, and on
//      this chip each one writes back the L2;
//   3. every valid cell adds the mean, rounded once to float32.
// The order of every sum depends only on the number of points, so the result
// is the same on every call.  The point decisions (transform, validity,
// binning) are the fusion's own, from the shared device helpers.
#include "emx_kernels.h"

namespace emx {

namespace {

constexpr int kNTd = 256;                 // threads per chunk workgroup
constexpr int kPerD = kChunk / kNTd;      // points per thread
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

// Fixed-shape sum over the workgroup: a butterfly within each wave, then the
// wave totals in wave order.  Thread 0 ends with the total; the order of the
// additions never changes.
__device__ __forceinline__ void block_sum(double& sum, int64_t& cnt, double* s_sum,
                                          int64_t* s_cnt) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    sum = sum + __shfl_xor(sum, o, 64);
    cnt = cnt + __shfl_xor(cnt, o, 64);
  }
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    s_sum[wave] = sum;
    s_cnt[wave] = cnt;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    sum = s_sum[0];
    cnt = s_cnt[0];
    for (int w = 1; w < kNTd / 64; ++w) {
      sum = sum + s_sum[w];
      cnt = cnt + s_cnt[w];
    }
  }
}

// The chunk partials of blocks 0..B-1 combined by one workgroup: strided
// sums in chunk order, then a fixed tree.
__device__ __forceinline__ void combine(const DriftArgs& a, double* s_sum, int64_t* s_cnt) {
  const int tid = threadIdx.x;
  double sum = 0.0;
  int64_t cnt = 0;
  for (int64_t b = tid; b < a.it.B; b += kNTd) {
    sum = sum + a.part_sum[b];
    cnt += a.part_cnt[b];
  }
  block_sum(sum, cnt, s_sum, s_cnt);
  if (tid == 0) {
    const int64_t n = cnt;
    const double mean = n > 0 ? sum / (double)n : 0.0;
    a.res->mean = mean;
    a.res->n = n;
    if (a.out_mean) *a.out_mean = mean;
    if (a.out_count) *a.out_count = n;
  }
}

__global__ __launch_bounds__(kNTd) void k_drift_partial(DriftArgs a) {
  __shared__ double s_sum[kNTd / 64];
  __shared__ int64_t s_cnt[kNTd / 64];
  const Item& it = a.it;
  const int tid = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * kChunk;
  double sum = 0.0;
  int64_t cnt = 0;
  // the four points' cells first, then their layers, so that the gathers of
  // all four are in flight together
  float zm[kPerD];
  int64_t cell[kPerD];
  bool use[kPerD];
#pragma unroll
  for (int j = 0; j < kPerD; ++j) {
    const int64_t i = base + (int64_t)j * kNTd + tid;  // a thread's points in index order
    use[j] = false;
    cell[j] = 0;
    zm[j] = 0.0f;
    if (i < it.n) {
      const PointEval e = eval_point(it.P, it.c, it.x[i], it.y[i], it.z[i]);
      int ix, iy;
      use[j] = e.valid && bin_xy(e.xm, e.ym, it.c, ix, iy);
      if (use[j]) cell[j] = pcell(it.c, ix, iy);  // physical: the layers
      zm[j] = e.zm;
    }
  }
#pragma unroll
  for (int j = 0; j < kPerD; ++j) {
    const uint8_t vc = it.L.valid[cell[j]];
    const float tr = it.L.trav[cell[j]];
    const float hc = it.L.h[cell[j]];
    // NaN traversability never passes
    if (use[j] && vc && tr > a.trav_min) {
      sum = sum + ((double)zm[j] - (double)hc);
      ++cnt;
    }
  }
  block_sum(sum, cnt, s_sum, s_cnt);
  if (tid == 0) {
    a.part_sum[blockIdx.x] = sum;
    a.part_cnt[blockIdx.x] = (uint32_t)cnt;
  }
}

__global__ __launch_bounds__(kNTd) void k_drift_combine(DriftArgs a) {
  __shared__ double s_sum[kNTd / 64];
  __shared__ int64_t s_cnt[kNTd / 64];
  combine(a, s_sum, s_cnt);
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
    hipLaunchKernelGGL(k_drift_combine, dim3(1), dim3(kNTd), 0, stream, a);
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
