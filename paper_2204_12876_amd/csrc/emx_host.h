// Host-side internals shared by the plain and batched C ABI entry points.
#pragma once

#include <stdint.h>

#include "emx.h"
#include "emx_kernels.h"

namespace emx {

// Per-map control words after the layers: two sets of clearing
// queue counters, used by alternate plain calls (each call's setup zeroes the
// other set for the next call), then the fusion's per-tile flags (one word
// per tile, zero between calls).
constexpr int kCtlWords = 2 * kCtrWords;
int64_t ctl_words(const emx_params& p);

// Default clearing segment length (samples per queued segment) and march
// workgroups per compute unit, from a sweep of both on MI355X.
constexpr int kDefaultSeg = 16;
constexpr int kMarchPerCU = 16;

emx_status fail(emx_status code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
emx_status hip_fail(hipError_t e, const char* what);
const char* last_error_text();

emx_status check_params(const emx_params* p);
Consts make_consts(const emx_params& p);
size_t set_layout(const emx_params& p, char* base, Layers* L);
size_t clr_bytes(const emx_params& p);  // the per-map clearing record array
int tiles_of(const emx_params& p);
int persistent_grid(int per_cu);
bool center_cell(double c, double r, int64_t* out);

}  // namespace emx

struct emx_map {
  emx_params p;
  emx::Consts c;
  int64_t cgx, cgy;
  int64_t t0;
  char* state;
  emx::Layers L;  // the layers, in the ring layout with origin (c.ox, c.oy)
  uint32_t* ctl;
  int ctr_sel;  // the counter set the next clear_visibility uses
  int march_grid;
};

namespace emx {

emx_status check_map(const emx_map* m);
emx_status check_frame(const emx_frame* f);

// Item for map m and frame f (f may be NULL for per-cell calls), on the map's
// current buffer set.  Validates the pose and time; fills geometry, not scratch.
emx_status make_item(const emx_map* m, const emx_frame* f, Item* it);

// Plan the move of map m to centre (cx, cy): shift in cells, clamped; returns
// false if the centre is out of range.
bool plan_move(const emx_map* m, double cx, double cy, int64_t* ngx, int64_t* ngy, int* sx,
               int* sy);

// The ring origin after a move by (sx, sy): logical cell (0, 0) of the moved
// map is logical cell (sx, sy) of the map before the move.
void turn_ring(const Consts& c, int sx, int sy, int* ox, int* oy);

}  // namespace emx
