// C ABI of libemx.so, plain per-map calls: argument checks, map handles, state
// layout and launch sequencing.  Everything device-side is enqueued on the
// caller's stream; the library never allocates device memory.
#include <math.h>
#include <stdarg.h>
#include <string.h>

#include <cstdio>
#include <mutex>
#include <new>
#include <string>

#include "emx_host.h"

namespace emx {

namespace {
thread_local std::string g_err;
constexpr int kMaxSide = 16384;
size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
bool finite_pos(double x) { return isfinite(x) && x > 0.0; }
}  // namespace

emx_status fail(emx_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

const char* last_error_text() { return g_err.c_str(); }

emx_status hip_fail(hipError_t e, const char* what) {
  return fail(EMX_EHIP, "%s: %s", what, hipGetErrorString(e));
}

emx_status check_params(const emx_params* p) {
  if (!p) return fail(EMX_EINVAL, "params is NULL");
  if (p->nx < 3 || p->ny < 3 || p->nx > kMaxSide || p->ny > kMaxSide)
    return fail(EMX_EINVAL, "nx, ny must lie in [3, %d] (got %d, %d)", kMaxSide, p->nx, p->ny);
  if (!isfinite(p->resolution) || p->resolution < 1e-6 || p->resolution > 1e6)
    return fail(EMX_EINVAL, "resolution must lie in [1e-6, 1e6] m");
  if (!isfinite(p->init_height)) return fail(EMX_EINVAL, "init_height must be finite");
  if (!finite_pos(p->init_variance)) return fail(EMX_EINVAL, "init_variance must be > 0");
  if (!finite_pos(p->noise_alpha)) return fail(EMX_EINVAL, "noise_alpha must be > 0");
  if (!finite_pos(p->min_range)) return fail(EMX_EINVAL, "min_range must be > 0");
  const float rmin2 = (float)((double)p->min_range * (double)p->min_range);
  const float sp2min = p->noise_alpha * rmin2;
  if (!(sp2min >= 1.17549435e-38f) || !isfinite(sp2min))
    return fail(EMX_EINVAL, "noise_alpha * min_range^2 must be a normal float32");
  if (!isfinite(p->gate_k) || p->gate_k < 0.0f) return fail(EMX_EINVAL, "gate_k must be >= 0");
  if (!finite_pos(p->ray_step)) return fail(EMX_EINVAL, "ray_step must be > 0");
  if (!isfinite((float)(1.0 / (double)p->ray_step)))
    return fail(EMX_EINVAL, "1/ray_step overflows float32");
  if (!isfinite(p->clear_normal_alpha) || p->clear_normal_alpha < 0.0f)
    return fail(EMX_EINVAL, "clear_normal_alpha must be >= 0");
  if (p->clear_min_age_ms < 0) return fail(EMX_EINVAL, "clear_min_age_ms must be >= 0");
  if (!isfinite(p->time_variance) || p->time_variance < 0.0f)
    return fail(EMX_EINVAL, "time_variance must be >= 0");
  if (p->wall_min_count < 0) return fail(EMX_EINVAL, "wall_min_count must be >= 0");
  if (p->upper_bound != 0 && p->upper_bound != 1)
    return fail(EMX_EINVAL, "upper_bound must be 0 or 1");
  if (p->excl_on != 0 && p->excl_on != 1) return fail(EMX_EINVAL, "excl_on must be 0 or 1");
  if (p->excl_on) {
    if (!isfinite(p->excl_theta) || p->excl_theta < 0.0f || p->excl_theta >= 1.5707963f)
      return fail(EMX_EINVAL, "excl_theta must lie in [0, pi/2)");
    if (!isfinite(p->excl_b) || !isfinite(p->excl_c) || !isfinite(p->excl_d))
      return fail(EMX_EINVAL, "excl_b, excl_c, excl_d must be finite");
    if (!isfinite((float)tan((double)p->excl_theta)))
      return fail(EMX_EINVAL, "tan(excl_theta) overflows float32");
  }
  if (!isfinite(p->outlier_variance) || p->outlier_variance < 0.0f)
    return fail(EMX_EINVAL, "outlier_variance must be >= 0");
  return EMX_OK;
}

Consts make_consts(const emx_params& p) {
  Consts c;
  c.inv_r = (float)(1.0 / p.resolution);
  c.rmin2 = (float)((double)p.min_range * (double)p.min_range);
  c.k2 = (float)((double)p.gate_k * (double)p.gate_k);
  c.alpha = p.noise_alpha;
  c.an2 = (float)((double)p.clear_normal_alpha * (double)p.clear_normal_alpha);
  c.inv_step = (float)(1.0 / (double)p.ray_step);
  c.inv6r = (float)(1.0 / (6.0 * p.resolution));
  c.h_init = p.init_height;
  c.v_init = p.init_variance;
  c.nx = p.nx;
  c.ny = p.ny;
  c.nxf = (float)p.nx;
  c.nyf = (float)p.ny;
  c.tau = p.clear_min_age_ms;
  c.var_t = p.time_variance;
  c.wall = p.wall_min_count;
  c.excl_on = p.excl_on;
  c.excl_slope = p.excl_on ? (float)tan((double)p.excl_theta) : 0.0f;
  c.excl_b = p.excl_b;
  c.excl_c = p.excl_c;
  c.excl_d = p.excl_d;
  c.var_o = p.outlier_variance;
  c.ox = 0;
  c.oy = 0;
  return c;
}

// One buffer set: seven 4-byte layers, two byte layers, the clearing block
// maxima, the upper bound layer if the map keeps one, then the fusion's four
// planes of fixed-point sums (8 bytes per cell each); each 256-aligned.
size_t set_layout(const emx_params& p, char* base, Layers* L) {
  const size_t C = (size_t)p.nx * (size_t)p.ny;
  const size_t l4 = align256(C * 4);
  const size_t l1 = align256(C);
  const int bl = block_log_of(p.nx, p.ny);
  const size_t lb = align256((size_t)blocks_of(p.nx, bl) * blocks_of(p.ny, bl) * 4);
  if (L && base) {
    L->h = (float*)(base + 0 * l4);
    L->v = (float*)(base + 1 * l4);
    L->t = (int32_t*)(base + 2 * l4);
    L->nx = (float*)(base + 3 * l4);
    L->ny = (float*)(base + 4 * l4);
    L->nz = (float*)(base + 5 * l4);
    L->trav = (float*)(base + 6 * l4);
    L->valid = (uint8_t*)(base + 7 * l4);
    L->mark = (uint8_t*)(base + 7 * l4 + l1);
    L->cmax = (float*)(base + 7 * l4 + 2 * l1);
    L->ub = p.upper_bound ? (float*)(base + 7 * l4 + 2 * l1 + lb) : nullptr;
    L->fx = (uint64_t*)(base + 7 * l4 + 2 * l1 + lb + (p.upper_bound ? l4 : 0));
    L->fxs = (int64_t)(align256(C * 8) / 8);
  }
  return 7 * l4 + 2 * l1 + lb + (p.upper_bound ? l4 : 0) + kFxWords * align256(C * 8);
}

size_t clr_bytes(const emx_params& p) { return align256((size_t)p.nx * (size_t)p.ny * 8); }

int tiles_of(const emx_params& p) { return tiles_x_of(p.nx) * tiles_y_of(p.ny); }

int64_t ctl_words(const emx_params& p) { return (int64_t)kCtlWords + tiles_of(p); }

// A persistent grid of per_cu workgroups per compute unit of the current device.
int persistent_grid(int per_cu) {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus <= 0)
    cus = 256;
  return per_cu * cus;
}

bool center_cell(double c, double r, int64_t* out) {
  const double q = floor(c / r);
  if (!isfinite(q) || fabs(q) > 1073741824.0) return false;
  *out = (int64_t)q;
  return true;
}

emx_status check_map(const emx_map* m) {
  if (!m) return fail(EMX_EINVAL, "map is NULL");
  if (!m->state) return fail(EMX_ESTATE, "map has no state");
  return EMX_OK;
}

emx_status check_frame(const emx_frame* f) {
  if (!f) return fail(EMX_EINVAL, "frame is NULL");
  if (f->n < 0 || f->n > 2147483647LL) return fail(EMX_EINVAL, "n must lie in [0, 2^31)");
  if (f->n > 0 && (!f->x || !f->y || !f->z)) return fail(EMX_EINVAL, "point arrays are NULL");
  return EMX_OK;
}

emx_status make_item(const emx_map* m, const emx_frame* f, Item* it) {
  memset(it, 0, sizeof(Item));
  it->c = m->c;
  it->L = m->L;
  it->tiles_x = tiles_x_of(m->p.nx);
  it->T = tiles_of(m->p);
  it->bl = block_log_of(m->p.nx, m->p.ny);
  it->bx = blocks_of(m->p.nx, it->bl);
  it->by = blocks_of(m->p.ny, it->bl);
  it->nb = it->bx * it->by;
  it->bpw = clear_blocks_per_wave(it->nb);
  it->nprep = clear_block_units(it->nb);
  it->fs.tcnt = m->ctl + kCtlWords;
  if (!f) return EMX_OK;
  for (int k = 0; k < 12; ++k)
    if (!isfinite(f->pose[k])) return fail(EMX_EINVAL, "pose has a non-finite entry");
  const double ox = (double)(m->cgx - m->p.nx / 2) * m->p.resolution;
  const double oy = (double)(m->cgy - m->p.ny / 2) * m->p.resolution;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) it->P.R[i * 3 + j] = (float)f->pose[i * 4 + j];
  it->P.t[0] = (float)(f->pose[3] - ox);
  it->P.t[1] = (float)(f->pose[7] - oy);
  it->P.t[2] = (float)f->pose[11];
  if (!isfinite(it->P.t[0]) || !isfinite(it->P.t[1]) || !isfinite(it->P.t[2]))
    return fail(EMX_EINVAL, "map-local translation overflows float32");
  const int64_t dt = f->t_ms - m->t0;
  if (dt < 0 || dt > 2147483647LL)
    return fail(EMX_EINVAL, "t_ms - t0 must lie in [0, 2^31) (got %lld)", (long long)dt);
  it->t_now = (int32_t)dt;
  it->x = f->x;
  it->y = f->y;
  it->z = f->z;
  it->n = f->n;
  it->B = (int)((f->n + kChunk - 1) / kChunk);
  fuse_fixed_shifts(it->c, it->P, f->n, &it->fxw, &it->fxz);
  return EMX_OK;
}

void turn_ring(const Consts& c, int sx, int sy, int* ox, int* oy) {
  *ox = (int)((((int64_t)c.ox + sx) % c.nx + c.nx) % c.nx);
  *oy = (int)((((int64_t)c.oy + sy) % c.ny + c.ny) % c.ny);
}

bool plan_move(const emx_map* m, double cx, double cy, int64_t* ngx, int64_t* ngy, int* sx,
               int* sy) {
  if (!center_cell(cx, m->p.resolution, ngx) || !center_cell(cy, m->p.resolution, ngy))
    return false;
  const int64_t dx = *ngx - m->cgx, dy = *ngy - m->cgy;
  const int64_t lim = (int64_t)kMaxSide + 1;
  *sx = (int)(dx > lim ? lim : (dx < -lim ? -lim : dx));
  *sy = (int)(dy > lim ? lim : (dy < -lim ? -lim : dy));
  return true;
}

}  // namespace emx

using namespace emx;

extern "C" {

const char* emx_version(void) { return "emx 0.2.0 gfx950"; }

const char* emx_last_error(void) { return last_error_text(); }

emx_status emx_params_check(const emx_params* params) { return check_params(params); }

size_t emx_state_bytes(const emx_params* params) {
  if (check_params(params) != EMX_OK) return 0;
  return align256(set_layout(*params, nullptr, nullptr) + clr_bytes(*params) +
                  ctl_words(*params) * sizeof(uint32_t));
}

size_t emx_scratch_bytes(const emx_params* params, int64_t max_points) {
  if (check_params(params) != EMX_OK) return 0;
  if (max_points < 0 || max_points > 2147483647LL) {
    fail(EMX_EINVAL, "max_points must lie in [0, 2^31)");
    return 0;
  }
  const int64_t count_cells =
      params->wall_min_count > 0 ? (int64_t)params->nx * params->ny : 0;
  const size_t f = fuse_scratch_layout(count_cells, nullptr, nullptr);
  const size_t c = clear_scratch_layout(max_points, kDefaultSeg, nullptr, nullptr);
  return f > c ? f : c;
}

size_t emx_export_bytes(const emx_params* params) {
  if (check_params(params) != EMX_OK) return 0;
  return (size_t)29 * (size_t)params->nx * (size_t)params->ny;
}

emx_status emx_init_map(const emx_params* params, double cx, double cy, int64_t t0_ms,
                        void* d_state, size_t state_bytes, void* stream, emx_map** out) {
  emx_status s = check_params(params);
  if (s != EMX_OK) return s;
  if (!out) return fail(EMX_EINVAL, "out is NULL");
  if (!d_state) return fail(EMX_EINVAL, "d_state is NULL");
  if (((uintptr_t)d_state & 255u) != 0) return fail(EMX_EINVAL, "d_state must be 256-byte aligned");
  const size_t need = emx_state_bytes(params);
  if (state_bytes < need)
    return fail(EMX_ENOMEM, "state buffer has %zu bytes, needs %zu", state_bytes, need);
  int64_t cgx, cgy;
  if (!center_cell(cx, params->resolution, &cgx) || !center_cell(cy, params->resolution, &cgy))
    return fail(EMX_EINVAL, "map centre out of range");
  emx_map* m = new (std::nothrow) emx_map;
  if (!m) return fail(EMX_ENOMEM, "host allocation failed");
  m->p = *params;
  m->c = make_consts(*params);
  m->cgx = cgx;
  m->cgy = cgy;
  m->t0 = t0_ms;
  m->state = (char*)d_state;
  const size_t set_bytes = set_layout(*params, m->state, &m->L);
  m->L.clr = (float2*)(m->state + set_bytes);
  m->ctr_sel = 0;
  m->ctl = (uint32_t*)(m->state + set_bytes + clr_bytes(*params));
  m->march_grid = persistent_grid(kMarchPerCU);
  hipError_t e =
      launch_fill_prior(m->c, m->L, m->ctl, (int)ctl_words(*params), (hipStream_t)stream);
  if (e != hipSuccess) {
    delete m;
    return hip_fail(e, "init_map");
  }
  *out = m;
  return EMX_OK;
}

emx_status emx_free_map(emx_map* map) {
  if (!map) return fail(EMX_EINVAL, "map is NULL");
  delete map;
  return EMX_OK;
}

emx_status emx_move_map(emx_map* m, double cx, double cy, void* stream) {
  emx_status s = check_map(m);
  if (s != EMX_OK) return s;
  int64_t ngx, ngy;
  int sx, sy;
  if (!plan_move(m, cx, cy, &ngx, &ngy, &sx, &sy))
    return fail(EMX_EINVAL, "map centre out of range");
  if (sx == 0 && sy == 0) return EMX_OK;
  emx_map moved = *m;
  turn_ring(m->c, sx, sy, &moved.c.ox, &moved.c.oy);
  Item it;
  make_item(&moved, nullptr, &it);
  it.sx = sx;
  it.sy = sy;
  hipError_t e = launch_move(it, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "move_map");
  m->c.ox = moved.c.ox;
  m->c.oy = moved.c.oy;
  m->cgx = ngx;
  m->cgy = ngy;
  return EMX_OK;
}

// fuse_points, optionally preceded by the move to (cx, cy).  Every argument
// is checked before anything is enqueued, so a refused call moves nothing.
static emx_status fuse_impl(emx_map* m, const emx_frame* f, bool move, double cx, double cy,
                            void* d_scratch, size_t scratch_bytes, int32_t* d_out_cell,
                            uint8_t* d_out_accept, void* stream) {
  emx_status s = check_map(m);
  if (s != EMX_OK) return s;
  if ((s = check_frame(f)) != EMX_OK) return s;
  int64_t ngx = m->cgx, ngy = m->cgy;
  int sx = 0, sy = 0;
  if (move && !plan_move(m, cx, cy, &ngx, &ngy, &sx, &sy))
    return fail(EMX_EINVAL, "map centre out of range");
  const bool shift = sx != 0 || sy != 0;
  // the item on the moved map: new centre, the ring turned
  emx_map moved = *m;
  if (shift) {
    moved.cgx = ngx;
    moved.cgy = ngy;
    turn_ring(m->c, sx, sy, &moved.c.ox, &moved.c.oy);
  }
  Item it;
  if ((s = make_item(&moved, f, &it)) != EMX_OK) return s;
  it.sx = sx;
  it.sy = sy;
  const bool run = f->n > 0 || m->p.time_variance != 0.0f;  // time variance: every call
  if (f->n > 0) {
    const int64_t count_cells = m->p.wall_min_count > 0 ? (int64_t)m->p.nx * m->p.ny : 0;
    const size_t need = fuse_scratch_layout(count_cells, nullptr, nullptr);
    if (need > 0) {
      if (!d_scratch) return fail(EMX_EINVAL, "d_scratch is NULL");
      if (((uintptr_t)d_scratch & 255u) != 0)
        return fail(EMX_EINVAL, "d_scratch must be 256-byte aligned");
      if (scratch_bytes < need)
        return fail(EMX_ENOMEM, "scratch has %zu bytes, needs %zu", scratch_bytes, need);
      fuse_scratch_layout(count_cells, (char*)d_scratch, &it.fs);
    }
  }
  it.out_cell = d_out_cell;
  it.out_accept = d_out_accept;
  it.stages = kStageFuse;
  hipError_t e = hipSuccess;
  if (shift) e = launch_move(it, (hipStream_t)stream);
  if (e == hipSuccess && run) e = launch_fuse(it, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, move ? "move_fuse_points" : "fuse_points");
  if (shift) {
    m->c.ox = moved.c.ox;
    m->c.oy = moved.c.oy;
    m->cgx = ngx;
    m->cgy = ngy;
  }
  return EMX_OK;
}

emx_status emx_fuse_points(emx_map* m, const emx_frame* f, void* d_scratch, size_t scratch_bytes,
                           int32_t* d_out_cell, uint8_t* d_out_accept, void* stream) {
  return fuse_impl(m, f, false, 0.0, 0.0, d_scratch, scratch_bytes, d_out_cell, d_out_accept,
                   stream);
}

}  // extern "C"

// Built-in fusion scratch for callers that cannot allocate.  Every GPU the
// library runs on holds its own copy of this array until the process ends.
// In host code the array's name is only a stand-in for the device address:
// the address is looked up once per device and kept in g_noalloc_ptr.
namespace {
constexpr size_t kNoallocScratchBytes = (size_t)16 << 20;
constexpr int kNoallocMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];
std::mutex g_noalloc_mu;
void* g_noalloc_ptr[kNoallocMaxDevices] = {};

// The current device's copy of the built-in scratch, looked up on first use.
emx_status noalloc_scratch(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kNoallocMaxDevices)
    return fail(EMX_EINVAL, "device %d is beyond the %d devices the built-in scratch serves", dev,
                kNoallocMaxDevices);
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!ptr) return fail(EMX_EHIP, "hipGetSymbolAddress(scratch) gave NULL");
    g_noalloc_ptr[dev] = ptr;
  }
  *out = g_noalloc_ptr[dev];
  return EMX_OK;
}
}  // namespace

extern "C" {

size_t emx_noalloc_scratch_limit(void) { return kNoallocScratchBytes; }

emx_status emx_fuse_points_noalloc(emx_map* m, const emx_frame* f, int32_t* d_out_cell,
                                   uint8_t* d_out_accept, void* stream) {
  emx_status s = check_map(m);
  if (s != EMX_OK) return s;
  if ((s = check_frame(f)) != EMX_OK) return s;
  const int64_t count_cells = m->p.wall_min_count > 0 ? (int64_t)m->p.nx * m->p.ny : 0;
  const size_t need = fuse_scratch_layout(count_cells, nullptr, nullptr);
  if (need > kNoallocScratchBytes)
    return fail(EMX_ENOMEM,
                "the wall rule's per-cell counts of this map need %zu bytes of fusion "
                "scratch; the built-in scratch holds %zu",
                need, kNoallocScratchBytes);
  void* d_scratch = nullptr;
  if ((s = noalloc_scratch(&d_scratch)) != EMX_OK) return s;
  return fuse_impl(m, f, false, 0.0, 0.0, d_scratch, kNoallocScratchBytes, d_out_cell,
                   d_out_accept, stream);
}

emx_status emx_move_fuse_points(emx_map* m, double cx, double cy, const emx_frame* f,
                                void* d_scratch, size_t scratch_bytes, int32_t* d_out_cell,
                                uint8_t* d_out_accept, void* stream) {
  return fuse_impl(m, f, true, cx, cy, d_scratch, scratch_bytes, d_out_cell, d_out_accept,
                   stream);
}

emx_status emx_clear_visibility(emx_map* m, const emx_frame* f, void* d_scratch,
                                size_t scratch_bytes, uint8_t* d_out_cleared, void* stream) {
  emx_status s = check_map(m);
  if (s != EMX_OK) return s;
  if ((s = check_frame(f)) != EMX_OK) return s;
  Item it;
  if ((s = make_item(m, f, &it)) != EMX_OK) return s;
  if (f->n > 0) {
    const size_t need = clear_scratch_layout(f->n, kDefaultSeg, nullptr, nullptr);
    if (!d_scratch) return fail(EMX_EINVAL, "d_scratch is NULL");
    if (((uintptr_t)d_scratch & 255u) != 0)
      return fail(EMX_EINVAL, "d_scratch must be 256-byte aligned");
    if (scratch_bytes < need)
      return fail(EMX_ENOMEM, "scratch has %zu bytes, needs %zu", scratch_bytes, need);
    clear_scratch_layout(f->n, kDefaultSeg, (char*)d_scratch, &it.cq);
  }
  it.cq.counter = m->ctl + m->ctr_sel * kCtrWords;
  it.cq.counter_next = m->ctl + (1 - m->ctr_sel) * kCtrWords;
  it.cq.seg = kDefaultSeg;
  it.out_cleared = d_out_cleared;
  it.stages = kStageClear;
  bool ran = false;
  hipError_t e = launch_clear(it, m->march_grid, (hipStream_t)stream, &ran);
  // once the setup ran, this call's counter set is spent and the other one
  // is being zeroed: switch, whatever happened after
  if (ran) m->ctr_sel = 1 - m->ctr_sel;
  if (e != hipSuccess) return hip_fail(e, "clear_visibility");
  return EMX_OK;
}

size_t emx_drift_scratch_bytes(int64_t max_points) {
  if (max_points < 0) return 0;
  return drift_scratch_layout(max_points, nullptr, nullptr);
}

emx_status emx_compensate_drift(emx_map* m, const emx_frame* f, float trav_min, void* d_scratch,
                                size_t scratch_bytes, double* d_out_mean, int64_t* d_out_count,
                                void* stream) {
  emx_status s = check_map(m);
  if (s != EMX_OK) return s;
  if ((s = check_frame(f)) != EMX_OK) return s;
  if (isnan(trav_min)) return fail(EMX_EINVAL, "trav_min is NaN");
  Item it;
  if ((s = make_item(m, f, &it)) != EMX_OK) return s;
  const size_t need = drift_scratch_layout(f->n, nullptr, nullptr);
  if (!d_scratch) return fail(EMX_EINVAL, "d_scratch is NULL");
  if (((uintptr_t)d_scratch & 255u) != 0)
    return fail(EMX_EINVAL, "d_scratch must be 256-byte aligned");
  if (scratch_bytes < need)
    return fail(EMX_ENOMEM, "scratch has %zu bytes, needs %zu", scratch_bytes, need);
  DriftScratch ds;
  drift_scratch_layout(f->n, (char*)d_scratch, &ds);
  hipError_t e = launch_drift(it, trav_min, ds, d_out_mean, d_out_count, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "compensate_drift");
  return EMX_OK;
}

emx_status emx_overlap_clear(emx_map* m, double rx, double ry, double rz, float radius,
                             float threshold, uint8_t* d_out_cleared, void* stream) {
  emx_status s = check_map(m);
  if (s != EMX_OK) return s;
  if (!isfinite(rx) || !isfinite(ry) || !isfinite(rz))
    return fail(EMX_EINVAL, "robot position must be finite");
  if (!isfinite(radius) || radius < 0.0f) return fail(EMX_EINVAL, "radius must be >= 0");
  if (!isfinite(threshold) || threshold < 0.0f)
    return fail(EMX_EINVAL, "threshold must be >= 0");
  const double ox = (double)(m->cgx - m->p.nx / 2) * m->p.resolution;
  const double oy = (double)(m->cgy - m->p.ny / 2) * m->p.resolution;
  OverlapArgs a;
  a.c = m->c;
  a.L = m->L;
  a.r32 = (float)m->p.resolution;
  a.rx = (float)(rx - ox);
  a.ry = (float)(ry - oy);
  a.rz = (float)rz;
  a.rad2 = (float)((double)radius * (double)radius);
  a.thr = threshold;
  a.out = d_out_cleared;
  if (!isfinite(a.rx) || !isfinite(a.ry) || !isfinite(a.rz))
    return fail(EMX_EINVAL, "map-local robot position overflows float32");
  hipError_t e = launch_overlap(a, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "overlap_clear");
  return EMX_OK;
}

size_t emx_inpaint_scratch_bytes(const emx_params* params) {
  if (!params || check_params(params) != EMX_OK) return 0;
  return inpaint_scratch_bytes(params->nx, params->ny);
}

emx_status emx_inpaint_min(emx_map* m, float* d_out, void* d_scratch, size_t scratch_bytes,
                           void* stream) {
  emx_status s = check_map(m);
  if (s != EMX_OK) return s;
  if (!d_out) return fail(EMX_EINVAL, "d_out is NULL");
  if (!d_scratch) return fail(EMX_EINVAL, "d_scratch is NULL");
  if (((uintptr_t)d_scratch & 255u) != 0)
    return fail(EMX_EINVAL, "d_scratch must be 256-byte aligned");
  const size_t need = inpaint_scratch_bytes(m->p.nx, m->p.ny);
  if (scratch_bytes < need)
    return fail(EMX_ENOMEM, "scratch has %zu bytes, needs %zu", scratch_bytes, need);
  hipError_t e =
      launch_inpaint(m->c, m->L, d_out, (char*)d_scratch, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "inpaint_min");
  return EMX_OK;
}

emx_status emx_smooth(const float* d_in, float* d_out, int32_t nx, int32_t ny, int32_t kind,
                      int32_t ksize, float sigma, void* stream) {
  if (!d_in || !d_out) return fail(EMX_EINVAL, "d_in or d_out is NULL");
  if (nx < 1 || ny < 1 || (int64_t)nx * ny > 2147483647LL)
    return fail(EMX_EINVAL, "grid %d x %d out of range", nx, ny);
  if (kind < EMX_SMOOTH_BOX || kind > EMX_SMOOTH_MEDIAN)
    return fail(EMX_EINVAL, "unknown filter kind %d", kind);
  if (ksize < 1 || (ksize & 1) == 0 || ksize > 31)
    return fail(EMX_EINVAL, "ksize must be odd, 1..31 (got %d)", ksize);
  if (kind == EMX_SMOOTH_MEDIAN && ksize != 3 && ksize != 5)
    return fail(EMX_EINVAL, "the median takes ksize 3 or 5 (got %d)", ksize);
  if (kind == EMX_SMOOTH_GAUSSIAN && !(isfinite(sigma) && sigma > 0.0f))
    return fail(EMX_EINVAL, "sigma must be > 0");
  if (nx <= ksize / 2 || ny <= ksize / 2)
    return fail(EMX_EINVAL, "grid %d x %d too small for ksize %d", nx, ny, ksize);
  const size_t bytes = (size_t)nx * (size_t)ny * sizeof(float);
  const char* a = (const char*)d_in;
  const char* b = (const char*)d_out;
  if (a < b + bytes && b < a + bytes) return fail(EMX_EINVAL, "d_out overlaps d_in");
  hipError_t e = launch_smooth(d_in, d_out, nx, ny, kind, ksize, sigma, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "smooth");
  return EMX_OK;
}

emx_status emx_compute_normals(emx_map* m, void* stream) {
  emx_status s = check_map(m);
  if (s != EMX_OK) return s;
  Item it;
  make_item(m, nullptr, &it);
  it.stages = kStageNormals;
  hipError_t e = launch_normals(it, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "compute_normals");
  return EMX_OK;
}

emx_status emx_traversability(emx_map* m, const float* d_weights, void* stream) {
  emx_status s = check_map(m);
  if (s != EMX_OK) return s;
  if (!d_weights) return fail(EMX_EINVAL, "d_weights is NULL");
  Item it;
  make_item(m, nullptr, &it);
  it.w = d_weights;
  it.stages = kStageTrav;
  hipError_t e = launch_trav(it, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "traversability");
  return EMX_OK;
}

emx_status emx_normals_traversability(emx_map* m, const float* d_weights, void* stream) {
  emx_status s = check_map(m);
  if (s != EMX_OK) return s;
  if (!d_weights) return fail(EMX_EINVAL, "d_weights is NULL");
  Item it;
  make_item(m, nullptr, &it);
  it.w = d_weights;
  it.stages = kStageNormals | kStageTrav;
  hipError_t e = launch_normals_trav(it, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "normals_traversability");
  return EMX_OK;
}

emx_status emx_layer(emx_map* m, int32_t layer, void** d_ptr) {
  emx_status s = check_map(m);
  if (s != EMX_OK) return s;
  if (!d_ptr) return fail(EMX_EINVAL, "d_ptr is NULL");
  const Layers& L = m->L;
  void* p = nullptr;
  switch (layer) {
    case EMX_LAYER_HEIGHT: p = L.h; break;
    case EMX_LAYER_VARIANCE: p = L.v; break;
    case EMX_LAYER_TIME: p = L.t; break;
    case EMX_LAYER_NORMAL_X: p = L.nx; break;
    case EMX_LAYER_NORMAL_Y: p = L.ny; break;
    case EMX_LAYER_NORMAL_Z: p = L.nz; break;
    case EMX_LAYER_TRAV: p = L.trav; break;
    case EMX_LAYER_VALID: p = L.valid; break;
    case EMX_LAYER_UPPER:
      if (!L.ub) return fail(EMX_EINVAL, "the map keeps no upper bound layer");
      p = L.ub;
      break;
    default: return fail(EMX_EINVAL, "unknown layer %d", layer);
  }
  *d_ptr = p;
  return EMX_OK;
}

emx_status emx_map_info(emx_map* m, int32_t* cgx, int32_t* cgy, int64_t* t0_ms) {
  emx_status s = check_map(m);
  if (s != EMX_OK) return s;
  if (cgx) *cgx = (int32_t)m->cgx;
  if (cgy) *cgy = (int32_t)m->cgy;
  if (t0_ms) *t0_ms = m->t0;
  return EMX_OK;
}

emx_status emx_map_origin(emx_map* m, int32_t* ox, int32_t* oy) {
  emx_status s = check_map(m);
  if (s != EMX_OK) return s;
  if (ox) *ox = m->c.ox;
  if (oy) *oy = m->c.oy;
  return EMX_OK;
}

// Between the packed logical layers and the ring: each layer is four
// rectangles, logical [0, nx-ox) x [0, ny-oy) at physical (ox, oy), and so on.
static emx_status copy_state(emx_map* m, char* packed, bool out, hipStream_t st) {
  const Layers& L = m->L;
  const int nx = m->p.nx, ny = m->p.ny, ox = m->c.ox, oy = m->c.oy;
  const size_t C = (size_t)nx * (size_t)ny;
  void* lay[8] = {L.h, L.v, L.t, L.nx, L.ny, L.nz, L.trav, L.valid};
  // logical start, physical start and extent of the two pieces of an axis
  const int lx[2] = {0, nx - ox}, px[2] = {ox, 0}, wx[2] = {nx - ox, ox};
  const int ly[2] = {0, ny - oy}, py[2] = {oy, 0}, hy[2] = {ny - oy, oy};
  size_t off = 0;
  for (int k = 0; k < 8; ++k) {
    const size_t es = k < 7 ? 4 : 1;
    char* pk = packed + off;
    char* ring = (char*)lay[k];
    for (int j = 0; j < 2; ++j)
      for (int i = 0; i < 2; ++i) {
        if (wx[i] == 0 || hy[j] == 0) continue;
        char* lp = pk + ((size_t)ly[j] * nx + lx[i]) * es;
        char* rp = ring + ((size_t)py[j] * nx + px[i]) * es;
        const size_t pitch = (size_t)nx * es;
        hipError_t e =
            out ? hipMemcpy2DAsync(lp, pitch, rp, pitch, (size_t)wx[i] * es, (size_t)hy[j],
                                   hipMemcpyDeviceToDevice, st)
                : hipMemcpy2DAsync(rp, pitch, lp, pitch, (size_t)wx[i] * es, (size_t)hy[j],
                                   hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return hip_fail(e, out ? "export_state" : "import_state");
      }
    off += es * C;
  }
  return EMX_OK;
}

emx_status emx_export_state(emx_map* m, void* d_dst, void* stream) {
  emx_status s = check_map(m);
  if (s != EMX_OK) return s;
  if (!d_dst) return fail(EMX_EINVAL, "d_dst is NULL");
  return copy_state(m, (char*)d_dst, true, (hipStream_t)stream);
}

emx_status emx_import_state(emx_map* m, const void* d_src, void* stream) {
  emx_status s = check_map(m);
  if (s != EMX_OK) return s;
  if (!d_src) return fail(EMX_EINVAL, "d_src is NULL");
  return copy_state(m, (char*)d_src, false, (hipStream_t)stream);
}

}  // extern "C"
