// Per-cell passes: prior fill, robot-centric move, 3x3 normals, conv traversability.
//
// The stencils (normals, traversability) stage a 34x34 halo tile of heights
// and validity in LDS.  Each 32x8 workgroup then produces a 32x32 output tile,
// four rows per thread, so every height is read from HBM about 1.13 times.
#include "emx_kernels.h"

namespace emx {

namespace {

constexpr int kNTf = 256;

// ------------------------------------------------------------------ prior fill
struct FillArgs {
  Consts c;
  Layers L;
  int64_t cells;
  uint32_t* ctl;
  int nctl;
};

__global__ __launch_bounds__(kNTf) void k_fill_prior(FillArgs a) {
  const int64_t i = (int64_t)blockIdx.x * kNTf + threadIdx.x;
  if (i < a.nctl) a.ctl[i] = 0u;
  if (i >= a.cells) return;
  const float qnan = __builtin_nanf("");
  a.L.h[i] = a.c.h_init;
  a.L.v[i] = a.c.v_init;
  a.L.t[i] = 0;
  a.L.nx[i] = qnan;
  a.L.ny[i] = qnan;
  a.L.nz[i] = qnan;
  a.L.trav[i] = qnan;
  a.L.valid[i] = 0;
  a.L.mark[i] = 0;
}

// ------------------------------------------------------------------------ move
struct MoveArgs {
  Consts c;
  Layers src;
  Layers dst;
  int sx, sy;
};

// dst(ix, iy) <- src(ix + sx, iy + sy), or the prior where that is outside.
__global__ __launch_bounds__(kNTf) void k_move(MoveArgs a) {
  const int ix = blockIdx.x * 64 + (threadIdx.x & 63);
  const int iy = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (ix >= a.c.nx || iy >= a.c.ny) return;
  const int64_t o = (int64_t)iy * a.c.nx + ix;
  const int jx = ix + a.sx;
  const int jy = iy + a.sy;
  if (jx >= 0 && jx < a.c.nx && jy >= 0 && jy < a.c.ny) {
    const int64_t s = (int64_t)jy * a.c.nx + jx;
    a.dst.h[o] = a.src.h[s];
    a.dst.v[o] = a.src.v[s];
    a.dst.t[o] = a.src.t[s];
    a.dst.nx[o] = a.src.nx[s];
    a.dst.ny[o] = a.src.ny[s];
    a.dst.nz[o] = a.src.nz[s];
    a.dst.trav[o] = a.src.trav[s];
    a.dst.valid[o] = a.src.valid[s];
  } else {
    const float qnan = __builtin_nanf("");
    a.dst.h[o] = a.c.h_init;
    a.dst.v[o] = a.c.v_init;
    a.dst.t[o] = 0;
    a.dst.nx[o] = qnan;
    a.dst.ny[o] = qnan;
    a.dst.nz[o] = qnan;
    a.dst.trav[o] = qnan;
    a.dst.valid[o] = 0;
  }
  a.dst.mark[o] = 0;
}

// ---------------------------------------------------------------- stencil tile
constexpr int kSW = 32;            // output tile width
constexpr int kSH = 32;            // output tile height
constexpr int kHW = kSW + 2;       // halo tile
constexpr int kHH = kSH + 2;

struct HaloTile {
  float h[kHH][kHW + 1];
  uint8_t ok[kHH][kHW + 2];
};

__device__ __forceinline__ void load_halo(HaloTile& s, const Consts& c, const Layers& L, int x0,
                                          int y0) {
  for (int idx = threadIdx.x; idx < kHH * kHW; idx += kNTf) {
    const int ly = idx / kHW;
    const int lx = idx - ly * kHW;
    const int gx = x0 - 1 + lx;
    const int gy = y0 - 1 + ly;
    float hv = 0.0f;
    uint8_t ok = 0;
    if (gx >= 0 && gx < c.nx && gy >= 0 && gy < c.ny) {
      const int64_t o = (int64_t)gy * c.nx + gx;
      ok = L.valid[o];
      hv = L.h[o];
    }
    s.h[ly][lx] = hv;
    s.ok[ly][lx] = ok;
  }
}

// the cell at halo position (lx, ly) is interior and its 3x3 window is valid
__device__ __forceinline__ bool window_ok(const HaloTile& s, const Consts& c, int gx, int gy,
                                          int lx, int ly) {
  if (gx < 1 || gy < 1 || gx > c.nx - 2 || gy > c.ny - 2) return false;
  bool ok = true;
#pragma unroll
  for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
    for (int dx = -1; dx <= 1; ++dx) ok = ok && (s.ok[ly + dy][lx + dx] != 0);
  return ok;
}

struct StencilArgs {
  Consts c;
  Layers L;
  const float* w;  // traversability weights (89)
};

__global__ __launch_bounds__(kNTf) void k_normals(StencilArgs a) {
  __shared__ HaloTile s;
  const int x0 = blockIdx.x * kSW;
  const int y0 = blockIdx.y * kSH;
  load_halo(s, a.c, a.L, x0, y0);
  __syncthreads();
  const int tx = threadIdx.x & (kSW - 1);
  const int ty0 = threadIdx.x / kSW;
  const float qnan = __builtin_nanf("");
#pragma unroll
  for (int j = 0; j < kSH / (kNTf / kSW); ++j) {
    const int ty = ty0 + j * (kNTf / kSW);
    const int gx = x0 + tx;
    const int gy = y0 + ty;
    if (gx >= a.c.nx || gy >= a.c.ny) continue;
    const int lx = tx + 1;
    const int ly = ty + 1;
    float nx = qnan, ny = qnan, nz = qnan;
    if (window_ok(s, a.c, gx, gy, lx, ly)) {
      const float dxm = s.h[ly - 1][lx + 1] - s.h[ly - 1][lx - 1];
      const float dx0 = s.h[ly][lx + 1] - s.h[ly][lx - 1];
      const float dxp = s.h[ly + 1][lx + 1] - s.h[ly + 1][lx - 1];
      const float dym = s.h[ly + 1][lx - 1] - s.h[ly - 1][lx - 1];
      const float dy0 = s.h[ly + 1][lx] - s.h[ly - 1][lx];
      const float dyp = s.h[ly + 1][lx + 1] - s.h[ly - 1][lx + 1];
      const float gxv = ((dxm + dx0) + dxp) * a.c.inv6r;
      const float gyv = ((dym + dy0) + dyp) * a.c.inv6r;
      const float q = (gxv * gxv + gyv * gyv) + 1.0f;
      const float inv = 1.0f / sqrtf(q);
      nx = -gxv * inv;
      ny = -gyv * inv;
      nz = inv;
    }
    const int64_t o = (int64_t)gy * a.c.nx + gx;
    a.L.nx[o] = nx;
    a.L.ny[o] = ny;
    a.L.nz[o] = nz;
  }
}

__global__ __launch_bounds__(kNTf) void k_trav(StencilArgs a) {
  __shared__ HaloTile s;
  __shared__ float sw[89];
  const int x0 = blockIdx.x * kSW;
  const int y0 = blockIdx.y * kSH;
  if (threadIdx.x < 89) sw[threadIdx.x] = a.w[threadIdx.x];
  load_halo(s, a.c, a.L, x0, y0);
  __syncthreads();
  const int tx = threadIdx.x & (kSW - 1);
  const int ty0 = threadIdx.x / kSW;
  const float qnan = __builtin_nanf("");
#pragma unroll
  for (int j = 0; j < kSH / (kNTf / kSW); ++j) {
    const int ty = ty0 + j * (kNTf / kSW);
    const int gx = x0 + tx;
    const int gy = y0 + ty;
    if (gx >= a.c.nx || gy >= a.c.ny) continue;
    const int lx = tx + 1;
    const int ly = ty + 1;
    float T = qnan;
    if (window_ok(s, a.c, gx, gy, lx, ly)) {
      float win[9];
#pragma unroll
      for (int dy = 0; dy < 3; ++dy)
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) win[dy * 3 + dx] = s.h[ly - 1 + dy][lx - 1 + dx];
      T = sw[88];
#pragma unroll
      for (int ch = 0; ch < 8; ++ch) {
        float acc = sw[72 + ch];
#pragma unroll
        for (int k = 0; k < 9; ++k) acc = fmaf(sw[ch * 9 + k], win[k], acc);
        T = fmaf(sw[80 + ch], fmaxf(acc, 0.0f), T);
      }
    }
    a.L.trav[(int64_t)gy * a.c.nx + gx] = T;
  }
}

}  // namespace

hipError_t launch_fill_prior(const Consts& c, const Layers& L, uint32_t* ctl, int nctl,
                             hipStream_t stream) {
  FillArgs a;
  a.c = c;
  a.L = L;
  a.cells = (int64_t)c.nx * c.ny;
  a.ctl = ctl;
  a.nctl = ctl ? nctl : 0;
  hipLaunchKernelGGL(k_fill_prior, dim3((unsigned)((a.cells + kNTf - 1) / kNTf)), dim3(kNTf), 0,
                     stream, a);
  return hipGetLastError();
}

hipError_t launch_move(const Consts& c, const Layers& src, const Layers& dst, int sx, int sy,
                       hipStream_t stream) {
  MoveArgs a;
  a.c = c;
  a.src = src;
  a.dst = dst;
  a.sx = sx;
  a.sy = sy;
  hipLaunchKernelGGL(k_move, dim3((c.nx + 63) / 64, (c.ny + 3) / 4), dim3(kNTf), 0, stream, a);
  return hipGetLastError();
}

hipError_t launch_normals(const Consts& c, const Layers& L, hipStream_t stream) {
  StencilArgs a;
  a.c = c;
  a.L = L;
  a.w = nullptr;
  hipLaunchKernelGGL(k_normals, dim3((c.nx + kSW - 1) / kSW, (c.ny + kSH - 1) / kSH), dim3(kNTf),
                     0, stream, a);
  return hipGetLastError();
}

hipError_t launch_trav(const Consts& c, const Layers& L, const float* weights,
                       hipStream_t stream) {
  StencilArgs a;
  a.c = c;
  a.L = L;
  a.w = weights;
  hipLaunchKernelGGL(k_trav, dim3((c.nx + kSW - 1) / kSW, (c.ny + kSH - 1) / kSH), dim3(kNTf), 0,
                     stream, a);
  return hipGetLastError();
}

}  // namespace emx
