// Host-side launchers of the emx kernels (internal to libemx.so).
//
// Plain launchers take one Item by value and launch one workgroup per unit of
// work.  Batched launchers take a device-resident Batch and a fixed grid of
// persistent workgroups, so that a captured graph can be replayed for any
// batch that fits the table.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "emx_device.h"

namespace emx {

// Brackets one plain kernel launch with timing events on its stream while
// timing is on (emx_timing_begin); does nothing otherwise.
class TimedLaunch {
 public:
  TimedLaunch(const char* name, hipStream_t s);
  ~TimedLaunch();
  TimedLaunch(const TimedLaunch&) = delete;
  TimedLaunch& operator=(const TimedLaunch&) = delete;

 private:
  hipStream_t stream_;
  long idx_;
};

// ------------------------------------------------------------------ fusion
int tiles_x_of(int nx);
int tiles_y_of(int ny);
// The fixed-point shifts of a frame of n points (Item::fxw, Item::fxz).
void fuse_fixed_shifts(const Consts& c, const Pose32& P, int64_t n, int* fxw, int* fxz);
// count_cells: cells of the per-cell point counts of the wall/edge rule (0:
// none); the fusion's only scratch.  Sets out->count.
size_t fuse_scratch_layout(int64_t count_cells, char* base, FuseScratch* out);
// Runs the time variance pass even when it.n == 0.
hipError_t launch_fuse(const Item& it, hipStream_t stream);
// Work units of the batched count zeroing and per-cell variance stages.
int64_t zero_units(int64_t cells);
int64_t var_units(int64_t cells);
// grid: zero, count, chunk, tile, variance; a zero grid skips its stage.
hipError_t launch_fuse_batch(const Batch* d_batch, const int grid[5], hipStream_t stream);

// ---------------------------------------------------------------- clearing
int64_t clear_queue_cap(int64_t max_points, int seg);
size_t clear_scratch_layout(int64_t max_points, int seg, char* base, ClearQueue* out);
// Setup workgroups: block role, then one per 256 rays; with no rays, the
// block role alone if a removed-cell mask must be zeroed.
int clear_setup_units(int64_t n, int nprep, bool mask);
// Blocks per wave and workgroups of the setup's block role for nb pruning blocks.
int clear_blocks_per_wave(int nb);
int clear_block_units(int nb);
// The item's queue counters must be zero on entry; the setup zeroes
// it.cq.counter_next (if set) for the next call.  *ran: the setup was launched.
hipError_t launch_clear(const Item& it, int march_grid, hipStream_t stream, bool* ran);
hipError_t launch_clear_batch(const Batch* d_batch, int grid_setup, int grid_march,
                              hipStream_t stream);

// --------------------------------------------------------------- per cell
// Threads' worth of work of the move: the cells that enter the map.
int64_t move_units(const Item& it);
int64_t cells_units(int nx, int ny);
// Fills L with the prior and zeroes ctl[0..nctl).
hipError_t launch_fill_prior(const Consts& c, const Layers& L, uint32_t* ctl, int nctl,
                             hipStream_t stream);
hipError_t launch_move(const Item& it, hipStream_t stream);

// Overlap clearance on one map's current layers (map-local float32 geometry).
struct OverlapArgs {
  Consts c;
  Layers L;
  float r32;       // resolution
  float rx, ry;    // robot, map-local
  float rz;        // robot height
  float rad2;      // radius^2
  float thr;       // height threshold
  uint8_t* out;    // optional removed-cell flags
};
hipError_t launch_overlap(const OverlapArgs& a, hipStream_t stream);
hipError_t launch_normals(const Item& it, hipStream_t stream);
hipError_t launch_trav(const Item& it, hipStream_t stream);
hipError_t launch_normals_trav(const Item& it, hipStream_t stream);
hipError_t launch_move_batch(const Batch* d_batch, int grid, hipStream_t stream);
hipError_t launch_cells_batch(const Batch* d_batch, int grid, hipStream_t stream);

// ---------------------------------------------------------------- filters
size_t inpaint_scratch_bytes(int nx, int ny);
hipError_t launch_inpaint(const Consts& c, const Layers& L, float* out, char* scratch,
                          hipStream_t stream);
// kind: 0 box, 1 Gaussian, 2 median; arguments validated by the caller.
hipError_t launch_smooth(const float* in, float* out, int nx, int ny, int kind, int ksize,
                         float sigma, hipStream_t stream);

// ------------------------------------------------------------------ drift
struct DriftScratch {
  void* res;            // the mean (double) and count (int64) of the last call
  double* part_sum;     // [chunks] float64 partial sums of the errors
  uint32_t* part_cnt;   // [chunks] contributing points per chunk
};
size_t drift_scratch_layout(int64_t max_points, char* base, DriftScratch* out);
hipError_t launch_drift(const Item& it, float trav_min, const DriftScratch& ds,
                        double* out_mean, int64_t* out_count, hipStream_t stream);

}  // namespace emx
