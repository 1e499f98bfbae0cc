/*
 * emx.h - C ABI of the MI355X (gfx950) elevation-map fusion library (libemx.so).
 *
 * This is the data-parallel per-frame path of GPU elevation mapping (Miki et al.,
 * "Elevation Mapping for Locomotion and Navigation using GPU", arXiv 2204.12876):
 *   - rigid transform of a point cloud into the robot-centric map frame (Sec. II-A);
 *   - range-quadratic height noise (Sec. II-C);
 *   - binning into grid cells;
 *   - a Mahalanobis outlier gate against each cell's prior (Sec. II-C);
 *   - inverse-variance (Kalman) fusion of height and variance (Sec. II-C, Eq. 1, 2);
 *   - visibility ray clearing (Sec. II-E, Eq. 3, 4);
 *   - 3x3 surface normals (Sec. II-A);
 *   - a small convolutional traversability filter (Sec. II-G);
 * and the method's further per-frame steps: time variance and the wall/edge
 * rule in the fusion (Sec. II-C), height drift compensation (Sec. II-D),
 * overlap clearance (Sec. II-F), the upper bound layer (Sec. II-H), and the
 * locomotion filters: minimum-filter inpainting and smoothing (Sec. II-I).
 *
 * Conventions shared by every call:
 *   - Pointers named d_* are device (HBM) pointers.  All other pointers are host
 *     pointers, read synchronously during the call.
 *   - The caller owns every device buffer: points, map state, scratch and outputs.
 *     The library never allocates device memory.  It allocates host-side
 *     objects only: map handles, and batch executors with their pinned tables
 *     and capture stream.
 *   - `stream` is a hipStream_t passed as void*; NULL means the null stream.
 *     Device work is enqueued on it and the call returns without synchronising.
 *     Results are visible after the stream passes the call.  Buffers handed to a
 *     call must stay alive until then.
 *   - Arguments are checked on the host before anything is enqueued.  On an
 *     invalid argument a call returns a negative emx_status, enqueues nothing and
 *     sets a thread-local message readable with emx_last_error().
 *   - Kernel faults surface at the caller's next stream synchronisation.
 *   - A map must not be used from two streams at once.  Distinct maps are
 *     independent.
 *   - Floating point: every result is computed in IEEE float32 (drift
 *     compensation sums its errors in float64).  Decisions use a fixed
 *     operation order, round-to-nearest and no fused multiply-add.  Those
 *     decisions are the range check, cell index, gate, ray samples and clearing
 *     predicate; the order is stated below.  The fusion's sums are exact
 *     integer sums and every float sum has a fixed order, so results are the
 *     same from run to run.
 *
 * Map geometry (the paper is silent on it; these are this library's conventions):
 *   - Cells are half-open squares of side r.  Global cell (gx, gy) covers
 *     [gx*r, (gx+1)*r) x [gy*r, (gy+1)*r) of world x, y.
 *   - The map is centred on cell (cgx, cgy) = (floor(cx/r), floor(cy/r)),
 *     computed in double precision.
 *   - Local cell (ix, iy) is global (cgx - nx/2 + ix, cgy - ny/2 + iy), with
 *     integer division.  Layers are row-major [iy][ix], cell = iy*nx + ix.
 *   - The local origin O = ((cgx - nx/2)*r, (cgy - ny/2)*r), in double.
 *   - A pose is a row-major 3x4 sensor->world matrix [R | t] in double.  The
 *     library rounds R to float32 and forms t32 = float32(t - (O.x, O.y, 0)):
 *     the translation in map-local metres, subtracted in double.
 */
#ifndef EMX_H
#define EMX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t emx_status;
#define EMX_OK 0
#define EMX_EINVAL (-1)  /* invalid argument: nothing enqueued                     */
#define EMX_ENOMEM (-2)  /* a caller buffer is smaller than the size query demands */
#define EMX_EHIP (-3)    /* the HIP runtime refused a launch or copy               */
#define EMX_ESTATE (-5)  /* the map handle is not usable (e.g. freed state)        */

typedef struct emx_map emx_map; /* opaque host handle */

/* Map parameters.  Units are metres, milliseconds, square metres. */
typedef struct {
  int32_t nx, ny;            /* cells; 3..16384 each                                 */
  double resolution;         /* r, metres per cell, 1e-6..1e6                        */
  float init_height;         /* prior height h_init of a fresh or removed cell       */
  float init_variance;       /* prior variance, large (Sec. II-C), > 0               */
  float noise_alpha;         /* alpha_d in sigma_p^2 = alpha_d * d^2 (Sec. II-C), > 0 */
  float gate_k;              /* Mahalanobis gate k, in sigmas (Sec. II-C), >= 0       */
  float min_range;           /* points with d < min_range are dropped, > 0           */
  float ray_step;            /* clearing ray step (Sec. II-E), > 0                   */
  float clear_normal_alpha;  /* alpha_n of Eq. 4, >= 0                               */
  int32_t clear_min_age_ms;  /* clearing needs age > this (Sec. II-E), >= 0          */
  float time_variance;       /* sigma_t^2 (Sec. II-C): each fuse_points call adds it */
                             /* to every valid cell it does not update; >= 0, 0 off  */
  int32_t wall_min_count;    /* wall/edge rule (Sec. II-C): in a valid cell that     */
                             /* receives more than this many of a frame's points,    */
                             /* points below its height are ignored; >= 0, 0 off     */
  int32_t upper_bound;       /* 1: keep the upper bound layer (Sec. II-H), updated   */
                             /* by emx_clear_visibility; 0: no such layer            */
  int32_t excl_on;           /* 1: exclusion area (Sec. II-C, Fig. 3): fusion ignores */
                             /* points above the line below; 0 off                   */
  float excl_theta;          /* theta_a, the line's angle, rad, in [0, pi/2)         */
  float excl_b;              /* the line's height above the sensor near it, m        */
  float excl_c;              /* horizontal distance where the line starts to rise, m */
  float excl_d;              /* the line's greatest height above the sensor, m       */
  float outlier_variance;    /* sigma_o^2 (Sec. II-C: outlier detection raises the   */
                             /* cell's variance): added once per fuse call to each   */
                             /* cell that is valid when the call starts and gets a   */
                             /* gate-rejected point; >= 0, 0 off                     */
} emx_params;

/* One point cloud in the sensor frame, structure of arrays. */
typedef struct {
  const float* x;   /* d_x[n], d_y[n], d_z[n]: float32 sensor-frame coordinates  */
  const float* y;
  const float* z;
  int64_t n;        /* points; 0 makes every per-point call a no-op; < 2^31     */
  double pose[12];  /* row-major 3x4 sensor->world [R | t]; R, t finite         */
  int64_t t_ms;     /* frame time; t_ms - t0_ms must lie in [0, 2^31)           */
} emx_frame;

/* Layer identifiers for emx_layer().  Element types in brackets. */
#define EMX_LAYER_HEIGHT 0     /* [float]   h                                      */
#define EMX_LAYER_VARIANCE 1   /* [float]   sigma_m^2                              */
#define EMX_LAYER_TIME 2       /* [int32]   ms since t0 of the last fusion         */
#define EMX_LAYER_NORMAL_X 3   /* [float]   NaN where undefined                    */
#define EMX_LAYER_NORMAL_Y 4   /* [float]                                          */
#define EMX_LAYER_NORMAL_Z 5   /* [float]                                          */
#define EMX_LAYER_TRAV 6       /* [float]   traversability, NaN where undefined    */
#define EMX_LAYER_VALID 7      /* [uint8]   1 once a point has been fused          */
#define EMX_LAYER_UPPER 8      /* [float]   upper bound of the ground height, +inf  */
                               /* where no ray has passed; only with upper_bound=1, */
                               /* and not part of the export format                 */
#define EMX_NUM_LAYERS 8

/* Library version string (static storage). */
const char* emx_version(void);

/* Text of the last non-OK status returned on the calling thread. */
const char* emx_last_error(void);

/* Host-only check of a parameter block.  Returns EMX_OK or EMX_EINVAL. */
emx_status emx_params_check(const emx_params* params);

/* Device bytes of one map's state: one set of layers stored as a ring (see
 * emx_layer; with upper_bound = 1 it also holds the upper bound layer), the
 * fusion's fixed-point sums (32 bytes per cell, zero between calls), 8 bytes
 * of clearing scratch per cell and a small control block (the clearing queue
 * counters and one word per 32x16-cell fusion tile).  Returns 0 for invalid
 * parameters. */
size_t emx_state_bytes(const emx_params* params);

/* Device scratch bytes emx_fuse_points and emx_clear_visibility need for
 * frames of up to max_points points (one buffer serves both calls, which use
 * it in turn; the fusion's part is the wall rule's per-cell counts, 4 bytes
 * per cell with wall_min_count > 0, else none).  Returns 0 for invalid
 * parameters or max_points < 0. */
size_t emx_scratch_bytes(const emx_params* params, int64_t max_points);

/* Bytes of the packed export format: the layers in identifier order, each
 * nx*ny elements: h, v, t_upd, normal x, y, z, trav (4 bytes each), valid
 * (1 byte).  29*nx*ny. */
size_t emx_export_bytes(const emx_params* params);

/* Create a map centred on world (cx, cy).  Every cell starts at the prior:
 * h_init, init_variance, t_upd 0, invalid, NaN normals and traversability
 * (Sec. II-C starts the variance at a large value).
 *   d_state:      caller-owned device buffer of state_bytes >= emx_state_bytes(),
 *                 256-byte aligned; retained by the handle until emx_free_map.
 *   t0_ms:        the time origin of the int32 time layer.
 * The prior fill is enqueued on `stream`.  *out receives a new handle. */
emx_status emx_init_map(const emx_params* params, double cx, double cy, int64_t t0_ms,
                        void* d_state, size_t state_bytes, void* stream, emx_map** out);

/* Height drift compensation (Sec. II-D), meant to run just before
 * emx_fuse_points on the same frame.  In float32, as emx_fuse_points decides:
 * each valid point in the map whose cell is valid and has traversability
 * above trav_min (NaN never is) contributes e = zm - h[cell], with e formed in
 * float64.  Their mean, summed in float64 in a fixed order of the points, is
 * added in float32 to the height of every valid cell; with no contributing
 * point nothing changes.
 *   d_scratch:     >= emx_drift_scratch_bytes(frame->n) bytes, 256-aligned.
 *   d_out_mean:    optional double[1]: the mean (0 if none).
 *   d_out_count:   optional int64[1]: the number of contributing points. */
size_t emx_drift_scratch_bytes(int64_t max_points);
emx_status emx_compensate_drift(emx_map* map, const emx_frame* frame, float trav_min,
                                void* d_scratch, size_t scratch_bytes, double* d_out_mean,
                                int64_t* d_out_count, void* stream);

/* Release the host handle.  The caller frees d_state once the stream is idle. */
emx_status emx_free_map(emx_map* map);

/* Robot-centric re-centring (Sec. I; the map follows the robot).  The map
 * shifts by whole cells to centre cell (floor(cx/r), floor(cy/r)).
 *   - Cells that stay in the map keep every layer.
 *   - Cells that enter take the prior, as in emx_init_map.
 * The layers are a ring: the move turns it (emx_map_origin changes) and resets
 * only the entering rows and columns, so its cost is the strips, not the map.
 * A zero shift enqueues nothing.  Layer pointers from emx_layer() stay valid. */
emx_status emx_move_map(emx_map* map, double cx, double cy, void* stream);

/* Fuse one point cloud into the map (Sec. II-C, Eq. 1 and Eq. 2).
 *
 * Per point, in float32 and in this operation order:
 *   xm = ((R00*xs + R01*ys) + R02*zs) + t32.x   (likewise ym, zm)
 *   d2 = (xs*xs + ys*ys) + zs*zs;  sp2 = alpha * d2
 *   The point is valid iff xs, ys, zs, d2 and sp2 are finite and
 *   d2 >= float32(min_range^2).
 *   fx = xm*inv_r, fy = ym*inv_r, with inv_r = float32(1/r).  The point is in
 *   the map iff 0 <= fx < nx and 0 <= fy < ny; then cell = floor(fy)*nx +
 *   floor(fx).
 *   Gate: e = zm - h0[cell]; accept iff e*e <= k2*(v0[cell] + sp2), with
 *   k2 = float32(gate_k^2).  h0 and v0 are the map's values when the call
 *   starts.
 *   Exclusion area (excl_on = 1; the figure defining it is not in the text,
 *   so this is the library's reading of theta_a, b, c, d): with the sensor
 *   origin o = t32,
 *     rho = sqrt((xm-o.x)*(xm-o.x) + (ym-o.y)*(ym-o.y));  e = zm - o.z
 *     line = fminf(b + s*fmaxf(rho - c, 0), d),  s = float32(tan(theta_a))
 *   an in-map point with e > line is ignored: not counted, gated or fused
 *   (its cell is still reported in d_out_cell).
 *   Wall/edge rule (wall_min_count > 0): a cell that is valid when the call
 *   starts and receives more than wall_min_count of the frame's valid,
 *   not-ignored points ignores those with zm < h0, before the gate (they are
 *   not accepted).
 * Per cell c with a non-empty accepted set A:
 *   W = 1/v0 + sum_A 1/sp2;  v = 1/W;  h = (h0/v0 + sum_A zm/sp2) * v
 *   valid = 1, t_upd = t_ms - t0.
 *   This equals Eq. 1 and 2 applied point by point, in exact arithmetic.
 *   The sums are formed exactly, in fixed point.  A point's float32 terms
 *     w = 1/sp2;  u = w * rz,  rz = (R20*xs + R21*ys) + R22*zs  (zm = rz + tz)
 *   are rounded to integers at the scales 2^Sw and 2^Su (ties to even; a w
 *   that rounds to zero counts as one unit) and summed as integers.  The
 *   shifts are chosen per call so that no sum can overflow:
 *     Sw = 93 - ceil(log2 n) - Ew,  2^(Ew-1) <= wmax < 2^Ew,
 *     wmax = (1 + 2^-10) * float32(1 / float32(alpha * float32(min_range^2))),
 *   and Su likewise with umax = (1 + 2^-10) * (|R20| + |R21| + |R22|) /
 *   (alpha * sqrt(float32(min_range^2))), bounds of every accepted w and |u|.
 *   In float64, sum 1/sp2 = Iw * 2^-Sw and sum zm/sp2 = Iu * 2^-Su +
 *   tz * sum 1/sp2 (Iw, Iu: the integer sums); each is then rounded to
 *   float32 for the update above.  The integer sums do not depend on the
 *   order of the points, so results are identical from run to run and across
 *   batching.
 * Cells with no accepted point are left bitwise unchanged, except that with
 * time_variance > 0 each valid one gets v = v + float32(time_variance).
 * With outlier_variance > 0, each cell that is valid when the call starts and
 * gets a point that reaches the gate and fails it gets, after the above,
 * v = v + float32(outlier_variance), once per call.
 *   d_scratch:    >= emx_scratch_bytes(params, frame->n) bytes, 256-aligned.
 *                 The fusion reads it only with wall_min_count > 0 (per-cell
 *                 counts); otherwise it may be NULL.
 *   d_out_cell:   optional int32[n]: cell, or -1 (dropped or outside).
 *   d_out_accept: optional uint8[n]: 1 iff the point passed the gate. */
emx_status emx_fuse_points(emx_map* map, const emx_frame* frame, void* d_scratch,
                           size_t scratch_bytes, int32_t* d_out_cell,
                           uint8_t* d_out_accept, void* stream);

/* emx_fuse_points without a scratch argument and without any allocation.
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc).
 *   Scratch: a built-in device array of emx_noalloc_scratch_limit() bytes
 *   (16 MiB), one per GPU, held from the first call on that GPU until the
 *   process ends.  It holds the fusion's scratch: the wall rule's per-cell
 *   counts (4 bytes per cell with wall_min_count > 0; without the rule the
 *   fusion uses none).  A map whose counts exceed it (more than 4,194,304
 *   cells) is refused with EMX_ENOMEM and nothing is enqueued.
 *   Every call on one GPU shares that GPU's array.  Calls that overlap on one
 *   GPU (on different streams, or from different threads without ordering)
 *   race on it; calls in order on one stream do not.
 *   Results are those of emx_fuse_points, bit for bit.  The call allocates
 *   nothing on the device or through any library; its first call on a GPU
 *   looks up the array's device address (hipGetSymbolAddress).
 * Other arguments, checks and errors are as for emx_fuse_points. */
size_t emx_noalloc_scratch_limit(void);
emx_status emx_fuse_points_noalloc(emx_map* map, const emx_frame* frame, int32_t* d_out_cell,
                                   uint8_t* d_out_accept, void* stream);

/* emx_move_map(map, cx, cy) then emx_fuse_points(map, frame, ...), with the
 * results of the two calls bit for bit, checked as one call: everything is
 * checked before anything is enqueued, so a refused call moves nothing.  The
 * pose is taken relative to the moved map.  Arguments are as for the two
 * calls. */
emx_status emx_move_fuse_points(emx_map* map, double cx, double cy, const emx_frame* frame,
                                void* d_scratch, size_t scratch_bytes, int32_t* d_out_cell,
                                uint8_t* d_out_accept, void* stream);

/* Visibility clean-up by ray casting (Sec. II-E, Eq. 3 and Eq. 4).
 *
 * Every valid point casts a ray from the sensor origin o = t32.  This includes
 * gated-out points and points whose end lies outside the map.  In float32:
 *   (dx, dy, dz) = (xm, ym, zm) - o;  m = max(|dx|, |dy|)
 *   K = ceil(m * inv_step), with inv_step = float32(1/ray_step).
 *   The ray is skipped unless m*inv_step < 2^24.
 *   Samples k = 1..K-1: t = float(k)/float(K);
 *   q = (o.x + t*dx, o.y + t*dy, o.z + t*dz).
 * A sample in cell c (in the map, not the end point's own cell) marks c iff:
 *   - valid[c];
 *   - (t_ms - t0) - t_upd[c] > clear_min_age_ms;
 *   - hd = h[c] - q.z satisfies hd > 0 and hd*hd > v[c]  (Eq. 3, sigma = sqrt(v));
 *   - nz[c] is not NaN;
 *   - ((dx*nx + dy*ny) + dz*nz)^2 > an2 * ((dx*dx + dy*dy) + dz*dz), with
 *     an2 = float32(alpha_n^2)  (Eq. 4: |r.n| > alpha_n for unit r, n).
 * Rays test the state as it was when the call started.  Afterwards each
 * marked cell returns to (init_height, init_variance) and becomes invalid.
 * Normals and traversability are left for the next per-cell pass.
 * Upper bound (Sec. II-H, maps with upper_bound = 1): the same samples, in
 * cells that are invalid when the call starts, lower the cell's bound to q.z:
 * upper[c] = min(upper[c], q.z over those samples).  A minimum has no order,
 * so the layer is deterministic.  Cells enter with +inf (init, move).
 *   d_scratch:     >= emx_scratch_bytes(params, frame->n) bytes, 256-aligned;
 *                  may be NULL when n = 0.
 *   d_out_cleared: optional uint8[nx*ny], set to 1 for removed cells, 0 else. */
emx_status emx_clear_visibility(emx_map* map, const emx_frame* frame, void* d_scratch,
                                size_t scratch_bytes, uint8_t* d_out_cleared, void* stream);

/* Surface normal per cell (Sec. II-A, "normal calculation").
 *   The normal is the least-squares plane fit on the 3x3 window (Prewitt
 *   differences):
 *     gx = ((d(-1) + d(0)) + d(+1)) * float32(1/(6r)),
 *     with d(dy) = h[iy+dy][ix+1] - h[iy+dy][ix-1]; gy likewise over columns.
 *   n = (-gx, -gy, 1) / sqrt((gx*gx + gy*gy) + 1).
 *   It is NaN unless 1 <= ix <= nx-2, 1 <= iy <= ny-2 and all 9 cells are
 *   valid. */
emx_status emx_compute_normals(emx_map* map, void* stream);

/* Traversability filter (Sec. II-G).  The paper's trained network is not
 * given; this is a 3x3 cross-correlation 1->8 with bias, then ReLU, then a 1x1
 * conv 8->1 with bias, with no output activation.
 *   d_weights: device float32[89]: w1[8][1][3][3] (PyTorch conv layout),
 *              b1[8], w2[8], b2[1].
 *   T = b2 + sum_c w2[c] * max(b1[c] + sum_{dy,dx} w1[c][dy+1][dx+1]*h[iy+dy][ix+dx], 0)
 *   NaN where the normal is NaN (border or any of the 9 cells invalid). */
emx_status emx_traversability(emx_map* map, const float* d_weights, void* stream);

/* emx_compute_normals then emx_traversability in one pass over the map (one
 * launch; each tile's heights are staged once).  Results are bitwise those of
 * the two calls. */
emx_status emx_normals_traversability(emx_map* map, const float* d_weights, void* stream);

/* Overlap clearance (Sec. II-F): removes old estimates of another floor
 * near the robot.  In float32, in map-local metres (rx, ry are moved into
 * them in float64, as the pose is):
 *   dx = ((float)ix + 0.5f) * float32(r) - rx32,  dy likewise with iy, ry32;
 *   a cell is removed iff valid, dx*dx + dy*dy <= float32(radius^2) and
 *   |h - float32(rz)| > threshold.
 * Removed cells return to (init_height, init_variance) and become invalid, as
 * in emx_clear_visibility.
 *   rx, ry, rz:    robot position in the world; rz is the robot's height.
 *   radius:        horizontal radius in metres, >= 0.
 *   threshold:     height difference in metres, >= 0.
 *   d_out_cleared: optional uint8[nx*ny], 1 for removed cells, 0 else. */
emx_status emx_overlap_clear(emx_map* map, double rx, double ry, double rz, float radius,
                             float threshold, uint8_t* d_out_cleared, void* stream);

/* Minimum-filter inpainting (Sec. II-I).  The invalid cells form regions
 * connected through their four edge neighbours.  Each region takes the
 * smallest height among the valid cells that share an edge with it (the
 * minimum along its occlusion border); a region without such a cell is NaN.
 * Valid cells keep their height.  The map is not changed.
 *   d_out:     device float32[nx*ny], row-major like the layers.
 *   d_scratch: >= emx_inpaint_scratch_bytes(params) bytes, 256-aligned. */
size_t emx_inpaint_scratch_bytes(const emx_params* params);
emx_status emx_inpaint_min(emx_map* map, float* d_out, void* d_scratch, size_t scratch_bytes,
                           void* stream);

/* Smoothing filters on a float32 grid (Sec. II-I: Gaussian, box blur,
 * median).  Row-major [ny][nx] in and out; d_out must not overlap d_in.
 * The window is ksize x ksize (ksize odd); border cells read the grid
 * mirrored about the edge cell without repeating it (index -1 reads 1), so
 * nx and ny must exceed ksize/2.
 *   EMX_SMOOTH_BOX:      mean of the window; ksize 1..31.
 *   EMX_SMOOTH_GAUSSIAN: separable weights w_i = exp(-i*i / (2 sigma^2)),
 *                        i = -ksize/2..ksize/2, normalised to sum 1 (formed in
 *                        double, rounded to float); along x, then along y;
 *                        ksize 1..31, sigma > 0.
 *   EMX_SMOOTH_MEDIAN:   the middle of the window's values; ksize 3 or 5.
 * A NaN in the window makes the output NaN (box and Gaussian through the
 * arithmetic, median by rule).  sigma is ignored except for the Gaussian. */
#define EMX_SMOOTH_BOX 0
#define EMX_SMOOTH_GAUSSIAN 1
#define EMX_SMOOTH_MEDIAN 2
emx_status emx_smooth(const float* d_in, float* d_out, int32_t nx, int32_t ny, int32_t kind,
                      int32_t ksize, float sigma, void* stream);

/* Device pointer of a layer, [ny][nx] elements stored as a ring: local cell
 * (ix, iy) is element ((iy + oy) mod ny) * nx + (ix + ox) mod nx, with the
 * ring origin (ox, oy) of emx_map_origin.  A move turns the ring (the origin
 * changes) and resets only the cells that enter the map; the pointer stays
 * valid for the map's lifetime. */
emx_status emx_layer(emx_map* map, int32_t layer, void** d_ptr);

/* The ring origin of the map's layers (see emx_layer), as of the last call
 * enqueued on the map.  Out-pointers may be NULL. */
emx_status emx_map_origin(emx_map* map, int32_t* ox, int32_t* oy);

/* Host-side geometry of a map.  Out-pointers may be NULL. */
emx_status emx_map_info(emx_map* map, int32_t* cgx, int32_t* cgy, int64_t* t0_ms);

/* Copy the layers out to (or in from) a packed device buffer of
 * emx_export_bytes() bytes, in the format described there, in local cell
 * order (the ring is unrolled; the origin does not change). */
emx_status emx_export_state(emx_map* map, void* d_dst, void* stream);
emx_status emx_import_state(emx_map* map, const void* d_src, void* stream);


/* ------------------------------------------------------------------ batches
 * Many maps, each with its own frame, through the whole per-frame path in one
 * launch sequence (one graph launch when "graph" is on, the default).
 *   - Stages run in pipeline order for every item: move, fuse, clear, normals,
 *     traversability.  `stages` selects them per item.
 *   - Each item's results are bitwise identical to those of the plain calls
 *     run in the same order on that map: the per-point and per-cell
 *     arithmetic is the same, the fusion's sums are integer sums (any order
 *     gives the same bits), and every float32 sum has a fixed order.
 *   - The tuning selects only launch geometry (persistent grid sizes) and the
 *     clearing segment length.  It never changes results.
 *   - Every map option of the plain calls is served: time and outlier
 *     variance, the wall rule (its counts take scratch, see
 *     emx_batch_scratch_bytes), the upper bound layer and the exclusion area. */
#define EMX_STAGE_MOVE 1u
#define EMX_STAGE_FUSE 2u
#define EMX_STAGE_CLEAR 4u
#define EMX_STAGE_NORMALS 8u
#define EMX_STAGE_TRAV 16u
#define EMX_STAGE_ALL 31u
#define EMX_BATCH_MAX_ITEMS 64

typedef struct emx_batch emx_batch; /* opaque: tables, graphs and tuning */

typedef struct {
  emx_map* map;           /* each map at most once per batch                   */
  emx_frame frame;        /* points for FUSE and CLEAR (as emx_fuse_points)    */
  double cx, cy;          /* MOVE target centre (as emx_move_map)              */
  const float* d_weights; /* TRAV weights, device float32[89]                  */
  int32_t* d_out_cell;    /* optional, as emx_fuse_points                      */
  uint8_t* d_out_accept;  /* optional, as emx_fuse_points                      */
  uint8_t* d_out_cleared; /* optional, as emx_clear_visibility                 */
  uint32_t stages;        /* EMX_STAGE_* bits                                  */
} emx_batch_item;

/* Create a batch executor.  tuning_json: NULL, or a flat JSON object whose
 * optional integer keys are the persistent grid sizes in workgroups
 * ("grid_move", "grid_chunk", "grid_tile", "grid_setup", "grid_march",
 * "grid_cells"), the clearing segment length "seg" (1..255) and "graph" (0
 * runs the launches directly instead of a cached graph).  Other keys are
 * ignored.
 * The executor allocates two pinned host tables and a capture stream. */
emx_status emx_batch_create(const char* tuning_json, emx_batch** out);
emx_status emx_batch_destroy(emx_batch* batch); /* waits for its last batch */

/* The executor's tuning as JSON, written to buf (len bytes). */
emx_status emx_batch_tuning(const emx_batch* batch, char* buf, size_t len);

/* Batches run and graphs captured by this executor so far.  A capture
 * happens the first time a batch needs a (scratch, key width, grid sizes)
 * combination that is not in the executor's cache of 16 graphs. */
emx_status emx_batch_stats(const emx_batch* batch, int64_t* batches, int64_t* captures);

/* Device scratch bytes for this list of items (1..EMX_BATCH_MAX_ITEMS);
 * 0 if the list is invalid. */
size_t emx_batch_scratch_bytes(const emx_batch* batch, const emx_batch_item* items,
                               int32_t n);

/* An upper bound of emx_batch_scratch_bytes() over every batch of at most
 * max_items items (1..EMX_BATCH_MAX_ITEMS) whose maps have no more fusion
 * tiles than a map of `largest` and whose frames hold at most max_points
 * points together.  For callers that size one scratch buffer up front, as a
 * server under a fixed memory budget does.  0 if an argument is invalid. */
size_t emx_batch_scratch_bound(const emx_batch* batch, const emx_params* largest,
                               int32_t max_items, int64_t max_points);

/* Run the batch on `stream`.
 *   d_scratch: >= emx_batch_scratch_bytes(), 256-aligned.  Its first bytes
 *              hold the batch's device table.  Graphs are cached per scratch
 *              address, key width and grid sizes, so keep reusing the same
 *              buffer.  A scratch buffer must not be shared by batches in
 *              flight at the same time.
 *   Each stage's grid is the tuned size capped at the stage's work rounded
 *   up to a power of two (the march: about two threads per ray).
 *   Every item is checked before anything is enqueued; on an error no map
 *   changes.  Moves commit the maps' new centres when the call returns OK.
 *   The call may wait on the host for the batch before last to release its
 *   pinned table. */
emx_status emx_pipeline_batch(emx_batch* batch, const emx_batch_item* items, int32_t n,
                              void* d_scratch, size_t scratch_bytes, void* stream);

/* ---------------------------------------------------------------- timing
 * Per-kernel timing, for profiling.  Between begin and end, each kernel the
 * library launches directly (plain calls, and batches run with "graph": 0) is
 * bracketed by two timing events on its own stream; launches captured into a
 * graph are not timed.  Batched kernels carry the suffix "_b".  end waits for the
 * recorded events and writes a JSON object to buf (len bytes):
 *   {"<kernel>": [launches, total_ms], ...}
 * in order of first launch, then forgets them: a second end without a new
 * begin reports {}.  Meant for one host thread; the events add a
 * little time between kernels, not inside them. */
emx_status emx_timing_begin(void);
emx_status emx_timing_end(char* buf, size_t len);

#ifdef __cplusplus
}
#endif
#endif /* EMX_H */
