// Post-processing filters for legged locomotion (Sec. II-I).
//
// Minimum-filter inpainting: the invalid cells form regions connected through
// their edge neighbours; each region takes the smallest height on its border.
// A union-find over the grid labels the regions.  Links only ever point from
// a larger cell index to a smaller one (an integer atomic minimum), so there
// are no cycles and each region ends with its smallest cell as the root,
// whatever the order of the unions.  Four per-cell launches:
//   1. local: per 32 x 32 tile, in LDS, the union of the tile's invalid cells
//      and, per tile-local region, the minimum border height offered from
//      inside the tile.  Writes each invalid cell's parent (its local root)
//      and the local minimum at each local root;
//   2. merge: invalid cells on a tile edge unite with their invalid
//      neighbours across it, in the global parent array;
//   3. border: local roots pass their minimum to their final root, and valid
//      cells on a tile edge offer their height across it;
//   4. fill: invalid cells read their final root's minimum (NaN if none).
// Minima are integer atomics over an order-preserving key of the float, so
// the output is deterministic.
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
  int32_t* parent;  // [cells] parent chain of invalid cells (global indices)
  uint32_t* best;   // [cells] at local roots: key of the smallest border height
  float* out;       // [cells]
  int tiles_x;
};

constexpr int kIT = 32;                // inpainting tile side
constexpr int kNTl = kIT * kIT;        // one thread per tile cell

__device__ __forceinline__ int32_t find_root(const int32_t* parent, int32_t x) {
  // parents change under concurrent unions: read them through the atomics path
  int32_t p = __atomic_load_n(parent + x, __ATOMIC_RELAXED);
  while (p != x) {
    x = p;
    p = __atomic_load_n(parent + x, __ATOMIC_RELAXED);
  }
  return x;
}

// find_root that also halves the path: each visited cell is pointed at its
// grandparent.  The write is an atomic minimum, so it can never undo a link
// made meanwhile (parents only decrease, and stay ancestors).
__device__ __forceinline__ int32_t find_halve(int32_t* parent, int32_t x) {
  int32_t p = __atomic_load_n(parent + x, __ATOMIC_RELAXED);
  while (p != x) {
    const int32_t g = __atomic_load_n(parent + p, __ATOMIC_RELAXED);
    if (g != p) atomicMin(parent + x, g);
    x = p;
    p = g;
  }
  return x;
}

__device__ __forceinline__ void unite(int32_t* parent, int32_t a, int32_t b) {
  while (true) {
    a = find_halve(parent, a);
    b = find_halve(parent, b);
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

// The same union-find on a tile's LDS array of local indices.
__device__ __forceinline__ int lds_find(volatile int* par, int x) {
  int p = par[x];
  while (p != x) {
    x = p;
    p = par[x];
  }
  return x;
}

__device__ __forceinline__ void lds_unite(int* par, int a, int b) {
  volatile int* vp = par;
  while (true) {
    a = lds_find(vp, a);
    b = lds_find(vp, b);
    if (a == b) return;
    if (a < b) {
      const int t = a;
      a = b;
      b = t;
    }
    const int old = atomicMin(par + a, b);
    if (old == a) return;
    a = old;
  }
}

// Physical cell of logical cell i (the map's ring layout).  The union-find
// works on logical cells; only the map's layers are read through the ring.
__device__ __forceinline__ int64_t lphys(const Consts& c, int64_t i) {
  const int iy = (int)(i / c.nx);
  const int ix = (int)(i - (int64_t)iy * c.nx);
  return pcell(c, ix, iy);
}

__global__ __launch_bounds__(kNTl) void k_inp_local(InpaintArgs a) {
  __shared__ int s_par[kNTl];
  __shared__ uint32_t s_best[kNTl];
  const int nx = a.c.nx;
  const int ny = a.c.ny;
  const int tid = threadIdx.x;
  const int lx = tid % kIT;
  const int ly = tid / kIT;
  const int x0 = (int)(blockIdx.x % a.tiles_x) * kIT;
  const int y0 = (int)(blockIdx.x / a.tiles_x) * kIT;
  const int gx = x0 + lx;
  const int gy = y0 + ly;
  const bool in = gx < nx && gy < ny;
  const int64_t i = (int64_t)gy * nx + gx;
  const bool ok = in && a.L.valid[lphys(a.c, i)];
  const bool hole = in && !ok;
  // Rows first, without atomics: a hole's parent is the first cell of its
  // run of holes along the row (a tile row is half a wave: one ballot).
  const uint64_t bal = __ballot(hole);
  const uint32_t row = (uint32_t)(bal >> (tid & 32));
  const uint32_t gaps = ~row & ((1u << lx) - 1u);   // non-holes left of lx
  const int start = gaps ? 32 - __builtin_clz(gaps) : 0;
  s_par[tid] = hole ? ly * kIT + start : -1;
  s_best[tid] = kNoKey;
  __syncthreads();
  // Then columns: join a run to the run above where they first overlap.
  if (hole && ly > 0 && s_par[tid - kIT] >= 0 && (lx == start || s_par[tid - kIT - 1] < 0))
    lds_unite(s_par, ly * kIT + start, tid - kIT);
  __syncthreads();
  // offers from valid cells to holes of the same tile: per direction, the
  // lanes of a wave that offer to one region are reduced first, so that each
  // region takes one LDS atomic per wave
  {
    volatile int* vp = s_par;
    const uint32_t k = ok ? f32_key(a.L.h[lphys(a.c, i)]) : kNoKey;
    const int nb[4] = {lx > 0 ? tid - 1 : -1, lx + 1 < kIT && gx + 1 < nx ? tid + 1 : -1,
                       ly > 0 ? tid - kIT : -1, ly + 1 < kIT && gy + 1 < ny ? tid + kIT : -1};
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      int r = (ok && nb[d] >= 0 && vp[nb[d]] >= 0) ? lds_find(vp, nb[d]) : -1;
      uint64_t pend = __ballot(r >= 0);
      while (pend) {
        const int leader = __builtin_ctzll(pend);
        const int R = __shfl(r, leader, 64);
        uint32_t m = r == R ? k : kNoKey;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) m = min(m, (uint32_t)__shfl_xor((int)m, o, 64));
        if ((threadIdx.x & 63) == leader) atomicMin(s_best + R, m);
        if (r == R) r = -1;
        pend = __ballot(r >= 0);
      }
    }
  }
  __syncthreads();
  if (hole) {
    const int r = lds_find(s_par, tid);
    a.parent[i] = (int32_t)((int64_t)(y0 + r / kIT) * nx + x0 + r % kIT);
    a.best[i] = r == tid ? s_best[tid] : kNoKey;
  }
}

__global__ __launch_bounds__(kNTi) void k_inp_merge(InpaintArgs a) {
  const int64_t i = (int64_t)blockIdx.x * kNTi + threadIdx.x;
  const int nx = a.c.nx;
  if (i >= (int64_t)nx * a.c.ny) return;
  const int iy = (int)(i / nx);
  const int ix = (int)(i - (int64_t)iy * nx);
  const bool right = (ix % kIT) == kIT - 1 && ix + 1 < nx;
  const bool down = (iy % kIT) == kIT - 1 && iy + 1 < a.c.ny;
  if (!(right || down) || a.L.valid[lphys(a.c, i)]) return;
  // Along an edge, hole pairs next to each other are already joined on both
  // sides: only the first pair of each run of pairs unites.
  if (right && !a.L.valid[lphys(a.c, i + 1)] &&
      (iy % kIT == 0 || a.L.valid[lphys(a.c, i - nx)] || a.L.valid[lphys(a.c, i - nx + 1)]))
    unite(a.parent, (int32_t)i, (int32_t)(i + 1));
  if (down && !a.L.valid[lphys(a.c, i + nx)] && (ix % kIT == 0 || a.L.valid[lphys(a.c, i - 1)] || a.L.valid[lphys(a.c, i + nx - 1)]))
    unite(a.parent, (int32_t)i, (int32_t)(i + nx));
}

__global__ __launch_bounds__(kNTi) void k_inp_border(InpaintArgs a) {
  const int64_t i = (int64_t)blockIdx.x * kNTi + threadIdx.x;
  const int nx = a.c.nx;
  const int ny = a.c.ny;
  if (i >= (int64_t)nx * ny) return;
  const int iy = (int)(i / nx);
  const int ix = (int)(i - (int64_t)iy * nx);
  if (!a.L.valid[lphys(a.c, i)]) {
    // a local root hands its tile's minimum to the final root
    const uint32_t k = a.best[i];
    if (k == kNoKey) return;
    const int32_t r = find_root(a.parent, (int32_t)i);
    if (r != (int32_t)i) atomicMin(a.best + r, k);
    return;
  }
  // valid cells offer their height to holes across a tile edge
  const int tx = ix % kIT;
  const int ty = iy % kIT;
  if (tx != 0 && tx != kIT - 1 && ty != 0 && ty != kIT - 1) return;
  const uint32_t k = f32_key(a.L.h[lphys(a.c, i)]);
  if (tx == 0 && ix > 0 && !a.L.valid[lphys(a.c, i - 1)]) atomicMin(a.best + find_root(a.parent, (int32_t)(i - 1)), k);
  if (tx == kIT - 1 && ix + 1 < nx && !a.L.valid[lphys(a.c, i + 1)])
    atomicMin(a.best + find_root(a.parent, (int32_t)(i + 1)), k);
  if (ty == 0 && iy > 0 && !a.L.valid[lphys(a.c, i - nx)])
    atomicMin(a.best + find_root(a.parent, (int32_t)(i - nx)), k);
  if (ty == kIT - 1 && iy + 1 < ny && !a.L.valid[lphys(a.c, i + nx)])
    atomicMin(a.best + find_root(a.parent, (int32_t)(i + nx)), k);
}

__global__ __launch_bounds__(kNTi) void k_inp_fill(InpaintArgs a) {
  const int64_t i = (int64_t)blockIdx.x * kNTi + threadIdx.x;
  if (i >= (int64_t)a.c.nx * a.c.ny) return;
  a.out[i] = a.L.valid[lphys(a.c, i)] ? a.L.h[lphys(a.c, i)] : key_f32(a.best[find_root(a.parent, (int32_t)i)]);
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
  a.tiles_x = (c.nx + kIT - 1) / kIT;
  const unsigned tiles = (unsigned)(a.tiles_x * ((c.ny + kIT - 1) / kIT));
  const dim3 grid((unsigned)((C + kNTi - 1) / kNTi));
  hipError_t e;
  {
    TimedLaunch tl("k_inp_local", stream);
    hipLaunchKernelGGL(k_inp_local, dim3(tiles), dim3(kNTl), 0, stream, a);
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  {
    TimedLaunch tl("k_inp_merge", stream);
    hipLaunchKernelGGL(k_inp_merge, grid, dim3(kNTi), 0, stream, a);
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
