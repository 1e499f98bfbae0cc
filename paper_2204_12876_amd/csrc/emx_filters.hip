// Post-processing filters for legged locomotion (Sec. II-I).
//
// Minimum-filter inpainting: the invalid cells form regions connected through
// their edge neighbours; each region takes the smallest height on its border.
// Five per-cell launches:
//   1. init: every invalid cell is its own parent; every region minimum is
//      "none";
//   2. union: each invalid cell joins its right and lower invalid
//      neighbours.  The union-find links the larger root below the smaller
//      one with an integer atomic minimum, so links only ever point to smaller
//      indices: no cycles, and each region ends with its smallest cell as the
//      root whatever the order of the unions;
//   3. flatten: each invalid cell points straight at its root;
//   4. border: each valid cell offers its height to the roots of its invalid
//      edge neighbours, by an integer atomic minimum over an order-preserving
//      key of the float;
//   5. fill: invalid cells read their root's minimum (NaN if none).
// Every step is order-free, so the output is deterministic.
//
// Smoothing (box, Gaussian, median) works on 16 x 16 output tiles.  A
// workgroup stages the tile and its mirrored halo in LDS; box and Gaussian
// then run a pass along x into LDS and a pass along y to the output, the
// median selects from the staged window.
#include "emx_kernels.h"

namespace emx {

namespace {

constexpr int kNTi = 256;

// Order-preserving key of a float: larger float, larger key.  The all-ones
// key is "none" and decodes to NaN.
__device__ __forceinline__ uint32_t f32_key(float f) {
  const uint32_t b = __float_as_uint(f);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float key_f32(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}
constexpr uint32_t kNoKey = 0xffffffffu;

struct InpaintArgs {
  Consts c;
  Layers L;
  int32_t* parent;  // [cells] root chain of invalid cells; -1 for valid ones
  uint32_t* best;   // [cells] per root: key of the smallest border height
  float* out;       // [cells]
};

__device__ __forceinline__ int32_t find_root(const int32_t* parent, int32_t x) {
  // parents change under concurrent unions: read them through the atomics path
  int32_t p = __atomic_load_n(parent + x, __ATOMIC_RELAXED);
  while (p != x) {
    x = p;
    p = __atomic_load_n(parent + x, __ATOMIC_RELAXED);
  }
  return x;
}

__device__ __forceinline__ void unite(int32_t* parent, int32_t a, int32_t b) {
  while (true) {
    a = find_root(parent, a);
    b = find_root(parent, b);
    if (a == b) return;
    if (a < b) {
      const int32_t t = a;
      a = b;
      b = t;
    }
    // link root a below b; if a is no longer a root, follow its new parent
    const int32_t old = atomicMin(parent + a, b);
    if (old == a) return;
    a = old;
  }
}

__global__ __launch_bounds__(kNTi) void k_inp_init(InpaintArgs a) {
  const int64_t i = (int64_t)blockIdx.x * kNTi + threadIdx.x;
  if (i >= (int64_t)a.c.nx * a.c.ny) return;
  a.parent[i] = a.L.valid[i] ? -1 : (int32_t)i;
  a.best[i] = kNoKey;
}

__global__ __launch_bounds__(kNTi) void k_inp_union(InpaintArgs a) {
  const int64_t i = (int64_t)blockIdx.x * kNTi + threadIdx.x;
  const int nx = a.c.nx;
  if (i >= (int64_t)nx * a.c.ny || a.L.valid[i]) return;
  const int iy = (int)(i / nx);
  const int ix = (int)(i - (int64_t)iy * nx);
  if (ix + 1 < nx && !a.L.valid[i + 1]) unite(a.parent, (int32_t)i, (int32_t)(i + 1));
  if (iy + 1 < a.c.ny && !a.L.valid[i + nx]) unite(a.parent, (int32_t)i, (int32_t)(i + nx));
}

__global__ __launch_bounds__(kNTi) void k_inp_flatten(InpaintArgs a) {
  const int64_t i = (int64_t)blockIdx.x * kNTi + threadIdx.x;
  if (i >= (int64_t)a.c.nx * a.c.ny || a.L.valid[i]) return;
  a.parent[i] = find_root(a.parent, (int32_t)i);
}

__global__ __launch_bounds__(kNTi) void k_inp_border(InpaintArgs a) {
  const int64_t i = (int64_t)blockIdx.x * kNTi + threadIdx.x;
  const int nx = a.c.nx;
  const int ny = a.c.ny;
  if (i >= (int64_t)nx * ny || !a.L.valid[i]) return;
  const int iy = (int)(i / nx);
  const int ix = (int)(i - (int64_t)iy * nx);
  const uint32_t k = f32_key(a.L.h[i]);
  int32_t last = -1;  // neighbours in one region share a root: offer it once
  const int64_t nb[4] = {ix > 0 ? i - 1 : -1, ix + 1 < nx ? i + 1 : -1,
                         iy > 0 ? i - nx : -1, iy + 1 < ny ? i + nx : -1};
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    if (nb[d] < 0 || a.L.valid[nb[d]]) continue;
    const int32_t r = a.parent[nb[d]];
    if (r == last) continue;
    last = r;
    if (k < a.best[r]) atomicMin(a.best + r, k);
  }
}

__global__ __launch_bounds__(kNTi) void k_inp_fill(InpaintArgs a) {
  const int64_t i = (int64_t)blockIdx.x * kNTi + threadIdx.x;
  if (i >= (int64_t)a.c.nx * a.c.ny) return;
  a.out[i] = a.L.valid[i] ? a.L.h[i] : key_f32(a.best[a.parent[i]]);
}

// -------------------------------------------------------------- smoothing
constexpr int kFT = 16;                      // output tile side
constexpr int kMaxR = 15;                    // largest radius (ksize 31)
constexpr int kFH = kFT + 2 * kMaxR;         // largest staged side

struct SmoothArgs {
  const float* in;
  float* out;
  int nx, ny;
  int r;                 // ksize / 2
  float w[2 * kMaxR + 1];  // per-axis weights (box: all 1)
  float scale;           // applied after both passes (box: 1/ksize^2)
};

// Index i mirrored into [0, n) about the edge cells.  Positions a partial
// tile stages beyond what its outputs read are clamped, to stay in bounds.
__device__ __forceinline__ int mirror(int i, int n) {
  i = i < 0 ? -i : i;
  i = i > n - 1 ? 2 * (n - 1) - i : i;
  return min(max(i, 0), n - 1);
}

// Stage the tile at (x0, y0) with a halo of r, mirrored at the grid's edges.
__device__ __forceinline__ void stage(float (*s)[kFH], const SmoothArgs& a, int x0, int y0) {
  const int side = kFT + 2 * a.r;
  for (int idx = threadIdx.x; idx < side * side; idx += kNTi) {
    const int ly = idx / side;
    const int lx = idx - ly * side;
    const int gx = mirror(x0 - a.r + lx, a.nx);
    const int gy = mirror(y0 - a.r + ly, a.ny);
    s[ly][lx] = a.in[(int64_t)gy * a.nx + gx];
  }
}

// Box and Gaussian: weighted sum along x (into LDS), then along y.
__global__ __launch_bounds__(kNTi) void k_smooth_sep(SmoothArgs a) {
  __shared__ float s[kFH][kFH];
  __shared__ float t[kFH][kFT + 1];
  __shared__ float w[2 * kMaxR + 1];  // the weights, indexed at run time
  const int x0 = blockIdx.x * kFT;
  const int y0 = blockIdx.y * kFT;
  if (threadIdx.x < 2 * kMaxR + 1) w[threadIdx.x] = a.w[threadIdx.x];
  stage(s, a, x0, y0);
  __syncthreads();
  const int k = 2 * a.r + 1;
  const int rows = kFT + 2 * a.r;
  for (int idx = threadIdx.x; idx < rows * kFT; idx += kNTi) {
    const int ly = idx / kFT;
    const int lx = idx - ly * kFT;
    float acc = 0.0f;
    for (int j = 0; j < k; ++j) acc = acc + w[j] * s[ly][lx + j];
    t[ly][lx] = acc;
  }
  __syncthreads();
  const int lx = threadIdx.x % kFT;
  const int ly = threadIdx.x / kFT;
  const int gx = x0 + lx;
  const int gy = y0 + ly;
  if (gx >= a.nx || gy >= a.ny) return;
  float acc = 0.0f;
  for (int j = 0; j < k; ++j) acc = acc + w[j] * t[ly + j][lx];
  a.out[(int64_t)gy * a.nx + gx] = acc * a.scale;
}

// Median of a K x K window: the value whose rank brackets the middle; NaN if
// the window holds a NaN.
template <int K>
__global__ __launch_bounds__(kNTi) void k_smooth_median(SmoothArgs a) {
  __shared__ float s[kFH][kFH];
  const int x0 = blockIdx.x * kFT;
  const int y0 = blockIdx.y * kFT;
  stage(s, a, x0, y0);
  __syncthreads();
  const int lx = threadIdx.x % kFT;
  const int ly = threadIdx.x / kFT;
  const int gx = x0 + lx;
  const int gy = y0 + ly;
  if (gx >= a.nx || gy >= a.ny) return;
  constexpr int N = K * K;
  constexpr int mid = N / 2;
  float v[N];
  bool nan = false;
#pragma unroll
  for (int dy = 0; dy < K; ++dy)
#pragma unroll
    for (int dx = 0; dx < K; ++dx) {
      v[dy * K + dx] = s[ly + dy][lx + dx];
      nan = nan || isnan(v[dy * K + dx]);
    }
  float med = __builtin_nanf("");
  if (!nan) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
      int less = 0, same = 0;
#pragma unroll
      for (int j = 0; j < N; ++j) {
        less += v[j] < v[i] ? 1 : 0;
        same += v[j] == v[i] ? 1 : 0;
      }
      if (less <= mid && less + same > mid) med = v[i];
    }
  }
  a.out[(int64_t)gy * a.nx + gx] = med;
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

size_t inpaint_scratch_bytes(int nx, int ny) {
  const size_t C = (size_t)nx * (size_t)ny;
  return align256(C * 4) + align256(C * 4);
}

hipError_t launch_inpaint(const Consts& c, const Layers& L, float* out, char* scratch,
                          hipStream_t stream) {
  const int64_t C = (int64_t)c.nx * c.ny;
  InpaintArgs a;
  a.c = c;
  a.L = L;
  a.parent = (int32_t*)scratch;
  a.best = (uint32_t*)(scratch + align256((size_t)C * 4));
  a.out = out;
  const dim3 grid((unsigned)((C + kNTi - 1) / kNTi));
  hipError_t e;
  {
    TimedLaunch tl("k_inp_init", stream);
    hipLaunchKernelGGL(k_inp_init, grid, dim3(kNTi), 0, stream, a);
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  {
    TimedLaunch tl("k_inp_union", stream);
    hipLaunchKernelGGL(k_inp_union, grid, dim3(kNTi), 0, stream, a);
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  {
    TimedLaunch tl("k_inp_flatten", stream);
    hipLaunchKernelGGL(k_inp_flatten, grid, dim3(kNTi), 0, stream, a);
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  {
    TimedLaunch tl("k_inp_border", stream);
    hipLaunchKernelGGL(k_inp_border, grid, dim3(kNTi), 0, stream, a);
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  {
    TimedLaunch tl("k_inp_fill", stream);
    hipLaunchKernelGGL(k_inp_fill, grid, dim3(kNTi), 0, stream, a);
  }
  return hipGetLastError();
}

// kind: 0 box, 1 Gaussian, 2 median (validated by the caller).
hipError_t launch_smooth(const float* in, float* out, int nx, int ny, int kind, int ksize,
                         float sigma, hipStream_t stream) {
  SmoothArgs a;
  a.in = in;
  a.out = out;
  a.nx = nx;
  a.ny = ny;
  a.r = ksize / 2;
  a.scale = 1.0f;
  for (int j = 0; j < 2 * kMaxR + 1; ++j) a.w[j] = 0.0f;
  if (kind == 0) {
    for (int j = 0; j < ksize; ++j) a.w[j] = 1.0f;
    a.scale = (float)(1.0 / ((double)ksize * (double)ksize));
  } else if (kind == 1) {
    double w[2 * kMaxR + 1], sum = 0.0;
    const double s = (double)sigma;
    for (int j = 0; j < ksize; ++j) {
      const double i = (double)(j - a.r);
      w[j] = exp(-(i * i) / (2.0 * s * s));
      sum += w[j];
    }
    for (int j = 0; j < ksize; ++j) a.w[j] = (float)(w[j] / sum);
  }
  const dim3 grid((unsigned)((nx + kFT - 1) / kFT), (unsigned)((ny + kFT - 1) / kFT));
  if (kind == 2) {
    TimedLaunch tl("k_smooth_median", stream);
    if (ksize == 3) hipLaunchKernelGGL(k_smooth_median<3>, grid, dim3(kNTi), 0, stream, a);
    else hipLaunchKernelGGL(k_smooth_median<5>, grid, dim3(kNTi), 0, stream, a);
  } else {
    TimedLaunch tl("k_smooth_sep", stream);
    hipLaunchKernelGGL(k_smooth_sep, grid, dim3(kNTi), 0, stream, a);
  }
  return hipGetLastError();
}

}  // namespace emx
