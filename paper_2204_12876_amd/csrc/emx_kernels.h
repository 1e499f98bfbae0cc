// Host-side launchers of the emx kernels (internal to libemx.so).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "emx_device.h"

namespace emx {

// ------------------------------------------------------------------ fusion
struct FuseScratch {
  uint16_t* rec_local;  // [B * kChunk] cell within its tile of each per-chunk partial
  float* rec_w;         // [B * kChunk] chunk partial of sum 1/sp2
  float* rec_wz;        // [B * kChunk] chunk partial of sum zm/sp2
  uint32_t* dir;        // [B * T]  (start << 16 | count) of a tile's partials in a chunk
};

// Scratch layout for frames of up to max_points; returns total bytes.
size_t fuse_scratch_layout(int64_t max_points, int T, char* base, FuseScratch* out);

int tiles_x_of(int nx);
int tiles_y_of(int ny);

hipError_t launch_fuse(const float* x, const float* y, const float* z, int64_t n,
                       const Pose32& P, const Consts& c, const Layers& L, int32_t t_now,
                       int32_t* out_cell, uint8_t* out_accept, const FuseScratch& s,
                       hipStream_t stream);

// ---------------------------------------------------------------- clearing
struct ClearScratch {
  float4* ray;       // [n] (dx, dy, dz, K) of each queued ray
  int32_t* ray_end;  // [n] end point's cell or -1
  uint2* queue;      // ~[4n] (ray, k_start << 8 | count) segments, in sub-queues
};

size_t clear_scratch_layout(int64_t max_points, char* base, ClearScratch* out);

// `counter` (64 uint32 counters, 32 words apart, in the map's control block)
// must be zero on entry; the call leaves it zero.
hipError_t launch_clear(const float* x, const float* y, const float* z, int64_t n,
                        const Pose32& P, const Consts& c, const Layers& L, int32_t t_now,
                        const ClearScratch& s, uint32_t* counter, uint8_t* out_cleared,
                        int march_grid, hipStream_t stream);

// --------------------------------------------------------------- per cell
// Fills L with the prior and zeroes ctl[0..nctl).
hipError_t launch_fill_prior(const Consts& c, const Layers& L, uint32_t* ctl, int nctl,
                             hipStream_t stream);
hipError_t launch_move(const Consts& c, const Layers& src, const Layers& dst, int sx, int sy,
                       hipStream_t stream);
hipError_t launch_normals(const Consts& c, const Layers& L, hipStream_t stream);
hipError_t launch_trav(const Consts& c, const Layers& L, const float* weights,
                       hipStream_t stream);

}  // namespace emx
