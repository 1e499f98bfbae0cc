// Batched pipeline: many maps, each with its own frame, through every stage
// in one launch sequence.
//
// The host fills a Batch table in pinned memory:
//   - each item's state pointers, geometry and constants;
//   - per stage, the prefix of work units over the items.
// Then, on the caller's stream:
//   - one copy of the table's header and its n items into the caller's
//     scratch;
//   - one graph of persistent launches: move, the wall rule's counts (zeroed,
//     then counted) if a map uses it, fusion pass 1 and pass 2, the per-cell
//     variances if a map uses time or outlier variance, clearing setup and
//     march, then normals + traversability.
// Every launch finds its work in the table, so a graph depends only on the
// scratch address and the grid sizes.  Each stage's grid
// is the tuned size capped at the stage's work rounded up to a power of two,
// so a small batch does not launch thousands of idle workgroups, and few
// distinct graphs arise.  Captured graphs are kept in a small LRU cache.
// Two pinned tables alternate: the host fills one while the other may still
// be read by the previous batch's copy.
//
// The work of each item runs through the same per-point and per-cell
// arithmetic as the plain calls (fusion pass 2 differs only in how cells are
// spread over threads), so every map's results equal those of the plain calls
// bit for bit.
#include <stdlib.h>
#include <string.h>

#include <cstddef>
#include <cstdio>
#include <new>

#include "emx_host.h"

using namespace emx;

namespace {

struct Tuning {
  int grid_move = 1024;
  int grid_chunk = 512;
  int grid_tile = 512;
  int grid_setup = 2048;
  int grid_march = 2048;
  int grid_cells = 1024;
  int seg = kDefaultSeg;
  int graph = 1;
};

// Value of "key": <number> in a flat JSON object; false if absent.
bool json_int(const char* js, const char* key, int* out) {
  char pat[64];
  snprintf(pat, sizeof pat, "\"%s\"", key);
  const char* p = strstr(js, pat);
  if (!p) return false;
  p = strchr(p + strlen(pat), ':');
  if (!p) return false;
  char* end = nullptr;
  const long v = strtol(p + 1, &end, 10);
  if (end == p + 1) return false;
  *out = (int)v;
  return true;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// grid: move, zero, count, chunk, tile, variance, setup, march, cells
constexpr int kGrids = 9;

struct GraphKey {
  void* scratch;
  int grid[kGrids];

  bool operator==(const GraphKey& o) const {
    if (scratch != o.scratch) return false;
    for (int i = 0; i < kGrids; ++i)
      if (grid[i] != o.grid[i]) return false;
    return true;
  }
};

int pow2_at_least(int64_t x) {
  int g = 1;
  while (g < x && g < (1 << 30)) g <<= 1;
  return g;
}

}  // namespace

struct emx_batch {
  Tuning tune;
  Batch* host[2];      // pinned tables, alternating
  hipEvent_t done[2];  // last launch that read host[i]
  bool used[2];
  int next;
  hipStream_t cap;     // private stream for graph capture
  static constexpr int kCache = 16;
  GraphKey keys[kCache];  // most recently used last
  hipGraphExec_t execs[kCache];
  int ncache;
  int64_t batches;    // batches run
  int64_t captures;   // graphs captured
};

namespace {

emx_status check_items(const emx_batch_item* items, int32_t n) {
  if (n < 1 || n > kMaxItems) return fail(EMX_EINVAL, "batch size must lie in [1, %d]", kMaxItems);
  if (!items) return fail(EMX_EINVAL, "items is NULL");
  for (int32_t i = 0; i < n; ++i) {
    emx_status s = check_map(items[i].map);
    if (s != EMX_OK) return s;
    if (items[i].stages & ~(uint32_t)EMX_STAGE_ALL)
      return fail(EMX_EINVAL, "item %d: unknown stage bits", i);
    if ((items[i].stages & (EMX_STAGE_FUSE | EMX_STAGE_CLEAR)) &&
        (s = check_frame(&items[i].frame)) != EMX_OK)
      return s;
    if ((items[i].stages & EMX_STAGE_TRAV) && !items[i].d_weights)
      return fail(EMX_EINVAL, "item %d: traversability needs weights", i);
    for (int32_t j = 0; j < i; ++j)
      if (items[j].map == items[i].map) return fail(EMX_EINVAL, "map appears twice in a batch");
  }
  return EMX_OK;
}

int64_t frame_points(const emx_batch_item& b) {
  return (b.stages & (EMX_STAGE_FUSE | EMX_STAGE_CLEAR)) ? b.frame.n : 0;
}

// Scratch layout: the device table, the clearing queue counters (zeroed by the
// batch's first launch), each item's fusion scratch, then one clearing queue
// shared by the batch.
constexpr size_t kCounterOffset = (sizeof(Batch) + 255) & ~(size_t)255;
constexpr size_t kCounterBytes = kCtrWords * sizeof(uint32_t);

size_t batch_layout(const emx_batch_item* items, int32_t n, int seg, char* base, Batch* tab) {
  size_t off = align256(kCounterOffset + kCounterBytes);
  int64_t rays = 0;
  for (int32_t i = 0; i < n; ++i) {
    const int64_t np = frame_points(items[i]);
    if (items[i].stages & EMX_STAGE_FUSE) {
      const emx_params& mp = items[i].map->p;
      const int64_t cc = mp.wall_min_count > 0 ? (int64_t)mp.nx * mp.ny : 0;
      const size_t f = fuse_scratch_layout(cc, nullptr, nullptr);
      if (tab && base) fuse_scratch_layout(cc, base + off, &tab->items[i].fs);
      off = align256(off + f);
    }
    if (tab) {
      tab->items[i].ray_base = rays;
      tab->rays[i] = rays;
    }
    if (items[i].stages & EMX_STAGE_CLEAR) rays += np;
  }
  if (tab) tab->rays[n] = rays;
  ClearQueue cq = {};
  const size_t c = clear_scratch_layout(rays, seg, base ? base + off : nullptr, &cq);
  if (tab && base)
    for (int32_t i = 0; i < n; ++i) {
      tab->items[i].cq = cq;
      tab->items[i].cq.counter = (uint32_t*)(base + kCounterOffset);
      tab->items[i].cq.counter_next = nullptr;  // zeroed by the batch's first launch
    }
  return off + c;
}

}  // namespace

extern "C" {

emx_status emx_batch_create(const char* tuning_json, emx_batch** out) {
  if (!out) return fail(EMX_EINVAL, "out is NULL");
  emx_batch* b = new (std::nothrow) emx_batch;
  if (!b) return fail(EMX_ENOMEM, "host allocation failed");
  b->tune = Tuning();
  b->tune.grid_march = persistent_grid(kMarchPerCU);
  b->tune.grid_setup = persistent_grid(8);
  if (tuning_json) {
    json_int(tuning_json, "grid_move", &b->tune.grid_move);
    json_int(tuning_json, "grid_chunk", &b->tune.grid_chunk);
    json_int(tuning_json, "grid_tile", &b->tune.grid_tile);
    json_int(tuning_json, "grid_setup", &b->tune.grid_setup);
    json_int(tuning_json, "grid_march", &b->tune.grid_march);
    json_int(tuning_json, "grid_cells", &b->tune.grid_cells);
    json_int(tuning_json, "seg", &b->tune.seg);
    json_int(tuning_json, "graph", &b->tune.graph);
  }
  const Tuning& t = b->tune;
  const int grids[] = {t.grid_move, t.grid_chunk, t.grid_tile, t.grid_setup,
                       t.grid_march, t.grid_cells};
  for (int g : grids)
    if (g < 1 || g > 65536) {
      delete b;
      return fail(EMX_EINVAL, "tuning: grid sizes must lie in [1, 65536]");
    }
  if (t.seg < 1 || t.seg > 255) {
    delete b;
    return fail(EMX_EINVAL, "tuning: seg must lie in [1, 255]");
  }
  b->ncache = 0;
  b->batches = 0;
  b->captures = 0;
  b->next = 0;
  b->host[0] = b->host[1] = nullptr;
  b->cap = nullptr;
  for (int i = 0; i < 2; ++i) {
    b->used[i] = false;
    b->done[i] = nullptr;
    hipError_t e = hipHostMalloc((void**)&b->host[i], sizeof(Batch), hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->done[i], hipEventDisableTiming);
    if (e != hipSuccess) {
      emx_batch_destroy(b);
      return hip_fail(e, "batch_create");
    }
  }
  hipError_t e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
  if (e != hipSuccess) {
    emx_batch_destroy(b);
    return hip_fail(e, "batch_create");
  }
  *out = b;
  return EMX_OK;
}

emx_status emx_batch_destroy(emx_batch* b) {
  if (!b) return fail(EMX_EINVAL, "batch is NULL");
  for (int i = 0; i < 2; ++i) {
    if (b->done[i]) {
      (void)hipEventSynchronize(b->done[i]);
      (void)hipEventDestroy(b->done[i]);
    }
    if (b->host[i]) (void)hipHostFree(b->host[i]);
  }
  for (int i = 0; i < b->ncache; ++i) (void)hipGraphExecDestroy(b->execs[i]);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  delete b;
  return EMX_OK;
}

emx_status emx_batch_tuning(const emx_batch* b, char* buf, size_t len) {
  if (!b || !buf) return fail(EMX_EINVAL, "NULL argument");
  const Tuning& t = b->tune;
  const int w = snprintf(buf, len,
                         "{\"grid_move\": %d, \"grid_chunk\": %d, \"grid_tile\": %d, "
                         "\"grid_setup\": %d, \"grid_march\": %d, "
                         "\"grid_cells\": %d, \"seg\": %d, \"graph\": %d}",
                         t.grid_move, t.grid_chunk, t.grid_tile, t.grid_setup, t.grid_march,
                         t.grid_cells, t.seg, t.graph);
  if (w < 0 || (size_t)w >= len) return fail(EMX_ENOMEM, "buffer too small");
  return EMX_OK;
}

emx_status emx_batch_stats(const emx_batch* b, int64_t* batches, int64_t* captures) {
  if (!b || !batches || !captures) return fail(EMX_EINVAL, "NULL argument");
  *batches = b->batches;
  *captures = b->captures;
  return EMX_OK;
}

size_t emx_batch_scratch_bytes(const emx_batch* b, const emx_batch_item* items, int32_t n) {
  if (!b || check_items(items, n) != EMX_OK) return 0;
  return batch_layout(items, n, b->tune.seg, nullptr, nullptr);
}

size_t emx_batch_scratch_bound(const emx_batch* b, const emx_params* largest, int32_t max_items,
                               int64_t max_points) {
  if (!b || check_params(largest) != EMX_OK) return 0;
  if (max_items < 1 || max_items > kMaxItems || max_points < 0 || max_points > 2147483647LL)
    return 0;
  // The fusion's scratch is each item's wall-rule counts, padded by under 256
  // bytes per item.
  const int64_t cc =
      largest->wall_min_count > 0 ? (int64_t)max_items * largest->nx * largest->ny : 0;
  const size_t fuse = fuse_scratch_layout(cc, nullptr, nullptr) + (size_t)max_items * 256;
  return align256(kCounterOffset + kCounterBytes) + fuse +
         clear_scratch_layout(max_points, b->tune.seg, nullptr, nullptr);
}

emx_status emx_pipeline_batch(emx_batch* b, const emx_batch_item* items, int32_t n,
                              void* d_scratch, size_t scratch_bytes, void* stream) {
  if (!b) return fail(EMX_EINVAL, "batch is NULL");
  emx_status s = check_items(items, n);
  if (s != EMX_OK) return s;
  if (!d_scratch) return fail(EMX_EINVAL, "d_scratch is NULL");
  if (((uintptr_t)d_scratch & 255u) != 0)
    return fail(EMX_EINVAL, "d_scratch must be 256-byte aligned");
  const size_t need = batch_layout(items, n, b->tune.seg, nullptr, nullptr);
  if (scratch_bytes < need)
    return fail(EMX_ENOMEM, "scratch has %zu bytes, needs %zu", scratch_bytes, need);

  // ---- validate every frame before any map is touched
  for (int32_t i = 0; i < n; ++i) {
    const emx_batch_item& bi = items[i];
    int64_t ngx, ngy;
    int sx, sy;
    if ((bi.stages & EMX_STAGE_MOVE) && !plan_move(bi.map, bi.cx, bi.cy, &ngx, &ngy, &sx, &sy))
      return fail(EMX_EINVAL, "item %d: map centre out of range", i);
  }

  // ---- fill the host table (wait until the copy that last read it is done)
  const int buf = b->next;
  b->next ^= 1;
  if (b->used[buf]) {
    hipError_t e = hipEventSynchronize(b->done[buf]);
    if (e != hipSuccess) return hip_fail(e, "pipeline_batch");
  }
  Batch* tab = b->host[buf];
  const size_t upload = offsetof(Batch, items) + (size_t)n * sizeof(Item);
  memset(tab, 0, upload);
  tab->n = n;
  Batch* d_tab = (Batch*)d_scratch;
  // plan every item on copies of the map geometry: no map changes until the
  // whole batch has been checked
  int ox[kMaxItems], oy[kMaxItems];
  int64_t cgx[kMaxItems], cgy[kMaxItems];
  for (int32_t i = 0; i < n; ++i) {
    const emx_batch_item& bi = items[i];
    emx_map tmp = *bi.map;
    Item& it = tab->items[i];
    int sx = 0, sy = 0;
    if (bi.stages & EMX_STAGE_MOVE) {
      int64_t ngx, ngy;
      plan_move(bi.map, bi.cx, bi.cy, &ngx, &ngy, &sx, &sy);
      if (sx != 0 || sy != 0) {
        turn_ring(bi.map->c, sx, sy, &tmp.c.ox, &tmp.c.oy);
        tmp.cgx = ngx;
        tmp.cgy = ngy;
      }
    }
    const bool pts = (bi.stages & (EMX_STAGE_FUSE | EMX_STAGE_CLEAR)) != 0;
    s = make_item(&tmp, pts ? &bi.frame : nullptr, &it);
    if (s != EMX_OK) return fail(s, "item %d: %s", i, last_error_text());
    it.sx = sx;
    it.sy = sy;
    it.stages = bi.stages;
    it.w = bi.d_weights;
    it.out_cell = bi.d_out_cell;
    it.out_accept = bi.d_out_accept;
    it.out_cleared = bi.d_out_cleared;
    it.index = i;
    ox[i] = tmp.c.ox;
    oy[i] = tmp.c.oy;
    cgx[i] = tmp.cgx;
    cgy[i] = tmp.cgy;
  }
  batch_layout(items, n, b->tune.seg, (char*)d_scratch, tab);
  int64_t clear_rays = 0;
  for (int32_t i = 0; i < n; ++i) {
    Item& it = tab->items[i];
    it.cq.seg = b->tune.seg;
    if (it.stages & EMX_STAGE_CLEAR) clear_rays += it.n;
    const uint32_t st = it.stages;
    const bool moved = (st & EMX_STAGE_MOVE) && (it.sx != 0 || it.sy != 0);
    const bool fuse = (st & EMX_STAGE_FUSE) && it.n > 0;
    const bool clear = (st & EMX_STAGE_CLEAR) != 0;
    const int64_t cells = (int64_t)it.c.nx * it.c.ny;
    const bool wall = fuse && it.fs.count != nullptr;
    // the per-cell variances, as the plain call runs them (time variance also
    // after an empty frame)
    const bool var = (st & EMX_STAGE_FUSE) &&
                     (it.c.var_t != 0.0f || (it.c.var_o != 0.0f && it.n > 0));
    tab->off[kBMove][i + 1] = tab->off[kBMove][i] + (moved ? move_units(it) : 0);
    tab->off[kBZero][i + 1] = tab->off[kBZero][i] + (wall ? zero_units(cells) : 0);
    tab->off[kBCount][i + 1] = tab->off[kBCount][i] + (wall ? it.B : 0);
    tab->off[kBChunk][i + 1] = tab->off[kBChunk][i] + (fuse ? it.B : 0);
    tab->off[kBTile][i + 1] = tab->off[kBTile][i] + (fuse ? it.T : 0);
    tab->off[kBVar][i + 1] = tab->off[kBVar][i] + (var ? var_units(cells) : 0);
    tab->off[kBSetup][i + 1] =
        tab->off[kBSetup][i] +
        (clear ? clear_setup_units(it.n, it.nprep, it.out_cleared != nullptr) : 0);
    tab->off[kBCells][i + 1] =
        tab->off[kBCells][i] +
        ((st & (EMX_STAGE_NORMALS | EMX_STAGE_TRAV)) ? cells_units(it.c.nx, it.c.ny) : 0);
  }

  // ---- grids: the tuned size, capped at the stage's work (power of two);
  // the march gets about two threads per ray
  const Tuning& t = b->tune;
  auto cap = [](int tuned, int64_t units) {
    return (int)(units < 1 ? 1 : (pow2_at_least(units) < tuned ? pow2_at_least(units) : tuned));
  };
  // stages that only some maps use are skipped (grid 0) when none does
  auto cap_opt = [&](int tuned, int64_t units) { return units < 1 ? 0 : cap(tuned, units); };
  GraphKey key;
  key.scratch = d_scratch;
  key.grid[0] = cap(t.grid_move, tab->off[kBMove][n]);
  key.grid[1] = cap_opt(t.grid_cells, tab->off[kBZero][n]);
  key.grid[2] = cap_opt(t.grid_chunk, tab->off[kBCount][n]);
  key.grid[3] = cap(t.grid_chunk, tab->off[kBChunk][n]);
  key.grid[4] = cap(t.grid_tile, tab->off[kBTile][n]);
  key.grid[5] = cap_opt(t.grid_cells, tab->off[kBVar][n]);
  key.grid[6] = cap(t.grid_setup, tab->off[kBSetup][n]);
  key.grid[7] = cap(t.grid_march, (2 * clear_rays + 255) / 256);
  key.grid[8] = cap(t.grid_cells, tab->off[kBCells][n]);

  // ---- enqueue: the table upload, then a cached graph or the same launches
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipSuccess;
  e = hipMemcpyAsync(d_tab, tab, upload, hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return hip_fail(e, "pipeline_batch: table upload");
  auto enqueue = [&](hipStream_t q) -> hipError_t {
    hipError_t r = launch_move_batch(d_tab, key.grid[0], q);
    if (r == hipSuccess) r = launch_fuse_batch(d_tab, key.grid + 1, q);
    if (r == hipSuccess) r = launch_clear_batch(d_tab, key.grid[6], key.grid[7], q);
    if (r == hipSuccess) r = launch_cells_batch(d_tab, key.grid[8], q);
    return r;
  };
  if (t.graph) {
    int slot = -1;
    for (int k = 0; k < b->ncache; ++k)
      if (b->keys[k] == key) slot = k;
    if (slot < 0) {
      hipGraph_t g = nullptr;
      hipGraphExec_t ex = nullptr;
      e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
      if (e == hipSuccess) {
        hipError_t e1 = enqueue(b->cap);
        e = hipStreamEndCapture(b->cap, &g);
        if (e1 != hipSuccess) e = e1;
      }
      if (e == hipSuccess) e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
      if (g) (void)hipGraphDestroy(g);
      if (e != hipSuccess) return hip_fail(e, "pipeline_batch: graph capture");
      if (b->ncache == emx_batch::kCache) {  // evict the least recently used
        (void)hipGraphExecDestroy(b->execs[0]);
        for (int k = 1; k < b->ncache; ++k) {
          b->keys[k - 1] = b->keys[k];
          b->execs[k - 1] = b->execs[k];
        }
        --b->ncache;
      }
      slot = b->ncache++;
      b->keys[slot] = key;
      b->execs[slot] = ex;
      ++b->captures;
    }
    // move the entry to the most recently used end
    const GraphKey k0 = b->keys[slot];
    hipGraphExec_t x0 = b->execs[slot];
    for (int k = slot + 1; k < b->ncache; ++k) {
      b->keys[k - 1] = b->keys[k];
      b->execs[k - 1] = b->execs[k];
    }
    b->keys[b->ncache - 1] = k0;
    b->execs[b->ncache - 1] = x0;
    e = hipGraphLaunch(x0, st);
  } else {
    e = enqueue(st);
  }
  if (e == hipSuccess) e = hipEventRecord(b->done[buf], st);
  if (e != hipSuccess) return hip_fail(e, "pipeline_batch");
  b->used[buf] = true;
  ++b->batches;
  // the moves are enqueued: commit the maps' new geometry
  for (int32_t i = 0; i < n; ++i) {
    items[i].map->c.ox = ox[i];
    items[i].map->c.oy = oy[i];
    items[i].map->cgx = cgx[i];
    items[i].map->cgy = cgy[i];
  }
  return EMX_OK;
}

}  // extern "C"
