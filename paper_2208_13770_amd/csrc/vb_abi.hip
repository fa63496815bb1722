// vb_abi.hip -- host implementation of the C ABI declared in include/vbuf.h.
//
// A context holds one batch of independent particle systems.  Each step queues
// three launches on the context's stream: the two broad-phase kernels, which
// return at once unless some system's list went invalid at the previous step
// (Def. autoverlet), and the fused step kernel.  The host never reads the
// validity flag.  It reads the overflow counters after every block of
// STATS_RING steps, one block behind the device, and waits on them only to
// take a snapshot (every SNAP_BLOCKS blocks) or at the end of a vb_run call; a
// Verlet-list row, cell bin or friction history that overflowed is grown and
// the steps since the last snapshot run again.  Every reorder_interval steps
// (and after a state is loaded) the host also queues a counting sort of the
// particle storage by cell, after which every row is rebuilt from the stored
// x0 and R_NL.  Blocks of STATS_RING steps that need nothing from the host run
// as one replayed HIP graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/vbuf.h"
#include "vb_device.h"

namespace vb {
hipError_t launch_step(const StepArgs &a, int64_t n_tiles, int unroll, int friction, int walls,
                       hipStream_t st, hipEvent_t t0, hipEvent_t t1);
hipError_t launch_broad_phase(const BroadArgs &a, int grid_bin, int grid_pairs, int nt, hipStream_t st,
                              hipEvent_t t0, hipEvent_t t1);
size_t pairs_lds_bytes(int width, int pmax, int nt);
int pairs_blocks_per_cu(int width, int pmax, int nt);
int64_t pairs_static_lds(int nt);
bool pairs_threads_supported(int nt);
hipError_t launch_get_history(const SysDev *sys, const int32_t *tile_sys, int64_t n_tiles,
                              const uint32_t *origs, const HistEntry *hist, const int32_t *hcnt,
                              int64_t stride, int32_t hcap, int32_t *partner, double *spring,
                              int32_t cap, int32_t *needed, hipStream_t st);
hipError_t launch_check_history(const SysDev &S, const int32_t *partner, const double *spring,
                                int32_t cap, int32_t *needed, int32_t *err, hipStream_t st);
hipError_t launch_set_history(const SysDev *sys, const int32_t *tile_sys, int64_t n_tiles,
                              const uint32_t *origs, const int32_t *partner, const double *spring,
                              int32_t cap, HistEntry *hist, int32_t *hcnt, int64_t stride,
                              hipStream_t st);
hipError_t launch_sort(const SortArgs &a, hipStream_t st);
int64_t scan_blocks(int64_t n_cells);
hipError_t launch_stats_reduce(const SysDev *sys, const TileStats *stats, const int32_t *ring,
                               int64_t n_tiles, int32_t n_sys, int32_t step0, int32_t nsteps,
                               RecordDev *out, hipStream_t st);
hipError_t launch_set_state(const SysDev &S, X3 *xs, V3 *vs, float2 *ri, uint32_t *origs,
                            const double *x, const double *v, const float *rc, const float *invm,
                            int32_t *err, int32_t *r_lo, int32_t *r_hi, hipStream_t st);
hipError_t launch_get_state(const SysDev *sys, const int32_t *tile_sys, int64_t n_tiles,
                            const X3 *xs, const V3 *vs, const uint32_t *origs, double *x, double *v,
                            hipStream_t st);
hipError_t launch_pairs(const SysDev &S, const X3 *xs, const float2 *ri, const uint32_t *origs,
                        const int32_t *cnt, const int32_t *nbr, int64_t stride,
                        int32_t contacts_only, int32_t *counts, int64_t *offsets, int64_t *total,
                        int64_t cap, int32_t *pairs, double *delta, hipStream_t st);
hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t st);
hipError_t launch_get_bp(const SysDev *sys, const int32_t *tile_sys, int64_t n_tiles,
                         const uint32_t *origs, const float4 *bp, float4 *x0r, hipStream_t st);
hipError_t launch_set_bp(const SysDev *sys, const int32_t *tile_sys, int64_t n_tiles,
                         const uint32_t *origs, const float2 *ri, const float4 *x0r, float4 *bp,
                         int32_t *err, hipStream_t st);
hipError_t launch_posq(const SysDev *sys, const int32_t *tile_sys, const int32_t *rrange, int n_sys,
                       const X3 *xs, const float2 *ri, uint64_t *posq, int64_t n, hipStream_t st);
}  // namespace vb

using namespace vb;

static_assert(sizeof(vb_step_record) == sizeof(RecordDev), "record layouts match");

// Scratch of the allocation-free pair export (vb_get_pairs_noalloc): the
// per-particle counts (int32), their exclusive prefix (int64) and the total
// (int64) for one system of at most VB_NOALLOC_MAX_N particles.  Every device
// the library runs on holds its own copy, from the first use of the library on
// that device until the process ends.  In host code `scratch` names no device
// address: the address of each device's copy is taken once, at the first
// context created on that device, and kept in g_scratch.
constexpr int64_t SCRATCH_BYTES = 12 * (int64_t)VB_NOALLOC_MAX_N + 256;
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];
constexpr int MAX_DEVICES = 64;
static void *g_scratch[MAX_DEVICES] = {};
static std::mutex g_scratch_mutex;

// Address of this device's scratch (the device is current); null on failure.
static void *device_scratch(int device) {
  if (device < 0 || device >= MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch[device]) {
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
    g_scratch[device] = ptr;
  }
  return g_scratch[device];
}

struct vb_ctx {
  hipStream_t stream = nullptr;
  int device = 0;
  int n_cu = 0;
  int32_t n_sys = 0;
  int64_t n_total = 0, slots = 0, n_tiles = 0, n_cells = 0;
  int32_t max_n = 0;
  std::vector<SysDev> sys_h;
  SysDev *sys_d = nullptr;
  int32_t *tile_sys = nullptr;
  // state, double-buffered every step (index cur)
  X3 *xs[2] = {nullptr, nullptr};
  V3 *vs[2] = {nullptr, nullptr};
  uint64_t *posq[2] = {nullptr, nullptr};  // coded positions of xs[0], xs[1]
  // (R_C, 1/m) and original index, double-buffered only by the storage sort (index scur)
  float2 *ri[2] = {nullptr, nullptr};
  uint32_t *orig[2] = {nullptr, nullptr};
  int scur = 0;
  int32_t *rrange = nullptr;               // [2][n_sys] smallest and largest R_C (FP32 bits)
  // friction history (allocated only when some system has friction)
  int any_friction = 0;
  int any_walls = 0;           // some system has planar or cylindrical walls
  int32_t hcap = 0;
  HistEntry *hist[2] = {nullptr, nullptr};
  int32_t *hcnt[2] = {nullptr, nullptr};
  HistEntry *hist_snap = nullptr;
  int32_t *hcnt_snap = nullptr;
  int32_t hist_snap_cap = 0;   // entries per slot hist_snap holds
  // snapshot of a step that a call can be run again from after an overflow
  // (state, x0 and R_NL, pending flags, friction history; the rows are rebuilt
  // from x0 and R_NL on restore), with the host's bookkeeping at that step
  X3 *snap_x = nullptr;
  V3 *snap_v = nullptr;
  float2 *snap_ri = nullptr;
  uint32_t *snap_orig = nullptr;
  float4 *snap_bp = nullptr;
  int32_t *snap_flags = nullptr;
  struct {
    int32_t at = 0;            // index of the step within the call
    int64_t step = 0, next_sort = 0;
    int first = 0, force = 0;
    int32_t hcap = 0;          // history columns the snapshot holds
  } snap;
  // overflow counters read back after each block of steps (pinned, two slots),
  // so that a call stops launching once a row, a bin or a history overflowed
  int32_t *ovf_host = nullptr;
  hipEvent_t ovf_ev[2] = {nullptr, nullptr};
  int32_t ovf_n = 0;    // read-backs requested in the current pass of vb_run
  float4 *bp = nullptr;
  float4 *bp_alt = nullptr;    // the storage sort moves bp here, then the two swap
  int32_t *cnt = nullptr, *nbr = nullptr;
  int32_t width = 0;
  int32_t *bin_count = nullptr;
  float4 *bins_bp = nullptr;
  int32_t *bins_og = nullptr;
  int32_t bin_cap = 0;
  int32_t *cellid = nullptr, *inv = nullptr;
  int32_t *act = nullptr;      // systems of the current broad phase (see BroadArgs)
  int64_t n_bricks = 0;
  int32_t pmax = 0;            // candidates k_pairs stages in LDS per workgroup
  int32_t xwindows = 1;        // k_pairs searches staged rows in x windows
  size_t lds_limit = 0;        // LDS bytes a workgroup may use on this device
  size_t lds_cu = 0;           // LDS bytes of one CU
  int pairs_grid = 0;
  int any_no_buffer = 0, any_fixed = 0;
  // counting sort of the storage
  int32_t *cell_count = nullptr, *cell_start = nullptr, *block_sum = nullptr;
  int32_t *inslot = nullptr, *perm0 = nullptr;
  // control
  int32_t *flags = nullptr, *go = nullptr, *overflow = nullptr, *err = nullptr;
  TileStats *stats = nullptr;
  int32_t *rebuilt_ring = nullptr;
  RecordDev *hist_d = nullptr;
  int64_t hist_cap = 0;
  int32_t *pair_counts = nullptr;
  int64_t *pair_offsets = nullptr, *pair_total = nullptr;
  int broad_grid = 0;
  int32_t row_limit = MAX_ROW;  // rows are sorted in LDS: TILE * width * 4 bytes
  int cur = 0;
  int64_t step = 0;
  int first = 1;
  int force_pending = 1;
  int relist_pending = 0;      // the next step rebuilds rows from x0 and R_NL (no broad phase)
  int have_list = 0;           // bp and the rows hold a list (a step ran, or a Verlet state was loaded)
  int64_t next_sort = 0;       // step at which the storage is re-sorted next (-1: never)
  int32_t sort_interval = 0;
  int loaded = 0;
  int fresh = 0;               // a state was loaded and no step has run since
  // launch shape (results do not depend on it): see Shape below
  int xcd_remap = 2;
  int step_unroll = 8;
  int pairs_t = PAIRS_T;
  int shape_fixed = 0;  // the shape was set by the environment: the tuned cache does not apply
  // replay of STATS_RING steps as one HIP graph (launch-bound small systems);
  // one cached graph per ping-pong parity, keyed by what the graph bakes in
  int use_graphs = 1;
  hipStream_t cap_stream = nullptr;
  int32_t *step_base_d = nullptr;  // first step of the replayed block
  int graph_mode = 0;              // queue_* build graph nodes: step = *step_base_d + graph_off
  int32_t graph_off = 0;
  hipGraphExec_t graph_exec[2] = {nullptr, nullptr};
  uint64_t graph_key[2] = {0, 0};
  // timing
  bool timing = false;
  std::vector<hipEvent_t> ev;
  double ms_rebuild = 0.0, ms_step = 0.0;
  int64_t t_steps = 0, t_rebuild_steps = 0;
  std::string msg;
};

static thread_local std::string g_create_error;

static vb_status fail(vb_ctx *c, vb_status code, const std::string &m) {
  if (c) c->msg = m;
  else g_create_error = m;
  return code;
}

#define HIP_OK(ctx, expr)                                                             \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail((ctx), e_ == hipErrorOutOfMemory ? VB_ENOMEM : VB_EDEVICE,          \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                 \
  } while (0)

template <typename T>
static hipError_t dalloc(T **p, int64_t count) {
  *p = nullptr;
  if (count <= 0) count = 1;
  return hipMalloc(reinterpret_cast<void **>(p), (size_t)count * sizeof(T));
}

static void free_all(vb_ctx *c) {
  void *ptrs[] = {c->sys_d, c->tile_sys, c->xs[0], c->xs[1], c->vs[0], c->vs[1], c->ri[0], c->ri[1],
                  c->orig[0], c->orig[1], c->posq[0],
                  c->posq[1], c->rrange, c->hist[0], c->hist[1], c->hcnt[0], c->hcnt[1], c->hist_snap,
                  c->hcnt_snap, c->snap_x, c->snap_v, c->snap_ri, c->snap_orig, c->snap_bp, c->snap_flags, c->bp, c->bp_alt, c->cnt, c->nbr, c->bin_count, c->bins_bp, c->bins_og,
                  c->act, c->cellid, c->inv,
                  c->cell_count, c->cell_start, c->block_sum, c->inslot, c->perm0, c->flags,
                  c->go, c->overflow, c->err, c->stats, c->rebuilt_ring, c->hist_d,
                  c->pair_counts, c->pair_offsets, c->pair_total};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  for (int b = 0; b < 2; ++b)
    if (c->graph_exec[b]) (void)hipGraphExecDestroy(c->graph_exec[b]);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  if (c->step_base_d) (void)hipFree(c->step_base_d);
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  c->ev.clear();
  for (hipEvent_t e : c->ovf_ev)
    if (e) (void)hipEventDestroy(e);
  if (c->ovf_host) (void)hipHostFree(c->ovf_host);
}

static std::string check_params(const vb_params &p, int64_t n) {
  if (n < 0) return "n < 0";
  // the step kernel addresses a system's 8-byte position codes with 32-bit
  // byte offsets
  if (n > ((int64_t)1 << 29) - TILE) return "n too large for one system (at most 2^29 - 256)";
  if (p.skin_mode < 0 || p.skin_mode > 3) return "skin_mode must be 0..3";
  if (p.cap_mode != 0 && p.cap_mode != 1) return "cap_mode must be 0 or 1";
  if (!(p.dt > 0.0) || !std::isfinite(p.dt)) return "dt must be positive";
  if (!(p.cell_size > 0.0) || !std::isfinite(p.cell_size)) return "cell_size must be positive";
  if (!(p.K >= 0.0) || !std::isfinite(p.K)) return "K must be >= 0";
  if (!(p.skin_uniform >= 0.0) || !std::isfinite(p.skin_uniform)) return "skin_uniform must be >= 0";
  if (!(p.kn >= 0.0) || !(p.gamma_n >= 0.0) || !std::isfinite(p.kn) || !std::isfinite(p.gamma_n))
    return "kn and gamma_n must be finite and >= 0";
  for (int a = 0; a < 3; ++a) {
    if (!std::isfinite(p.lo[a]) || !std::isfinite(p.hi[a]) || !(p.hi[a] > p.lo[a]))
      return "box must satisfy lo < hi";
    if (!std::isfinite(p.gravity[a])) return "gravity must be finite";
  }
  // the FP32 inclusion test of the broad phase returns a superset of the exact
  // list only with a positive margin: at least 16 FP32 ulps of the largest
  // coordinate (the rounding of the reference positions and of the distance)
  double xmax = 0.0;
  for (int a = 0; a < 3; ++a) xmax = std::max(xmax, std::max(std::fabs(p.lo[a]), std::fabs(p.hi[a])));
  if (!std::isfinite(p.eps) || !(p.eps >= std::ldexp(xmax, -19)))
    return "eps must be at least 2^-19 times the largest box coordinate";
  if (p.max_neighbors < 1 || p.max_neighbors > MAX_ROW) return "max_neighbors must be 1..128";
  if (p.skin_mode == VB_FIXED_INTERVAL && p.fixed_interval < 1) return "fixed_interval must be >= 1";
  if (p.reorder_interval < 0) return "reorder_interval must be >= 0";
  if (p.bin_capacity < 0 || p.bin_capacity > MAX_BIN) return "bin_capacity must be 0..256";
  if (!(p.kt >= 0.0) || !(p.gamma_t >= 0.0) || !(p.mu >= 0.0) || !std::isfinite(p.kt) ||
      !std::isfinite(p.gamma_t) || !std::isfinite(p.mu))
    return "kt, gamma_t and mu must be finite and >= 0";
  if (p.contact_capacity < 0 || p.contact_capacity > MAX_HIST) return "contact_capacity must be 0..64";
  if (p.n_planes < 0 || p.n_planes > VB_MAX_PLANES) return "n_planes must be 0..4";
  for (int w = 0; w < p.n_planes; ++w) {
    const double *pl = p.planes[w];
    for (int c = 0; c < 5; ++c)
      if (!std::isfinite(pl[c]) && !(c == 4 && pl[c] == -INFINITY)) return "plane values must be finite";
    const double nn = pl[0] * pl[0] + pl[1] * pl[1] + pl[2] * pl[2];
    if (std::fabs(nn - 1.0) > 1e-9) return "plane normals must have unit length";
  }
  if (p.n_cylinders < 0 || p.n_cylinders > VB_MAX_CYLINDERS) return "n_cylinders must be 0..2";
  for (int w = 0; w < p.n_cylinders; ++w) {
    const double *cy = p.cylinders[w];
    for (int c = 0; c < 4; ++c)
      if (!std::isfinite(cy[c]) && !(c == 3 && cy[c] == -INFINITY))
        return "cylinder values must be finite";
    if (!(cy[2] > 0.0)) return "cylinder radii must be positive";
  }
  return "";
}

// Cell grid of one system: cells of edge at least L_C (1 + 2^-10) + 2 eps per
// axis, so that every pair the FP32 inclusion test may accept lies in cells at
// most `ring` apart (Sec. 3.2: cells not smaller than the bounding spheres).
// Cells are numbered brick by brick (bricks of BRICK^3 cells); the numbering
// covers whole bricks, so a system uses nkeys >= nc[0] nc[1] nc[2] cell numbers.
static int64_t make_grid(const vb_params &p, SysDev &S) {
  const double edge_min = p.cell_size * (1.0 + 1.0 / 1024.0) + 2.0 * p.eps;
  int64_t nkeys = BRICK * BRICK * BRICK;
  for (int a = 0; a < 3; ++a) {
    const double len = p.hi[a] - p.lo[a];
    double k = std::floor(len / edge_min);
    if (k < 1) k = 1;
    if (k > 1 << 20) k = 1 << 20;
    S.nc[a] = (int32_t)k;
    S.nb[a] = (S.nc[a] + BRICK - 1) / BRICK;
    S.inv_edge[a] = k / len;
    nkeys *= S.nb[a];
  }
  S.nkeys = (int32_t)std::min<int64_t>(nkeys, INT32_MAX);
  return nkeys;
}

// LDS and grid of the pair search for the current row width and threads per
// workgroup.  LDS: rows plus staged candidates of 20 bytes; half the CU's LDS per
// workgroup (two resident per CU), less the kernel's static arrays
// (PAIRS_STATIC_LDS), unless wide rows need more; never beyond the device limit.  Grid: the pair
// search walks the bricks grid-stride with exactly the workgroups that are
// resident at once, so that at any time they work on one window of consecutive
// bricks, whose staged neighbourhoods overlap in L2.
static void size_pair_search(vb_ctx *c) {
  const int64_t rows = (int64_t)pairs_lds_bytes(c->width, 0, c->pairs_t);
  const int64_t budget = std::min<int64_t>((int64_t)c->lds_limit - PAIRS_STATIC_LDS,
                                           std::max<int64_t>((int64_t)c->lds_cu / 2 - PAIRS_STATIC_LDS,
                                                             rows + 1024 * 20));
  c->pmax = (int32_t)std::max<int64_t>(0, std::min<int64_t>(4096, (budget - rows) / 20));
  c->pairs_grid = (int)std::max<int64_t>(
      1, std::min<int64_t>(c->n_bricks,
                           (int64_t)pairs_blocks_per_cu(c->width, c->pmax, c->pairs_t) * c->n_cu));
}

static vb_status alloc_rows(vb_ctx *c, int32_t width) {
  if (c->nbr) (void)hipFree(c->nbr);
  c->nbr = nullptr;
  HIP_OK(c, dalloc(&c->nbr, c->slots * (int64_t)width));
  c->width = width;
  size_pair_search(c);
  return VB_OK;
}

// ------------------------------------------------------------------ launch shapes
// The launch shape of a context: the partner gathers each step-kernel thread
// keeps in flight (1, 2, 4 or 8), the step kernel's tile order (0: launch
// order, 1: each XCD a contiguous range, 2: each XCD runs of consecutive tiles
// inside one window) and the pair search's threads per
// workgroup (256, 384 or 512).  Results do not depend on it (the FP64 contact
// law and integration are rounded after every operation and summed in one
// order), so it may change between any two steps.
struct Shape {
  int unroll, xcd, pairs_t;
};

static bool shape_ok(const Shape &sh) {
  return (sh.unroll == 1 || sh.unroll == 2 || sh.unroll == 4 || sh.unroll == 8) &&
         (sh.xcd >= 0 && sh.xcd <= 2) && pairs_threads_supported(sh.pairs_t);
}

static Shape current_shape(const vb_ctx *c) { return Shape{c->step_unroll, c->xcd_remap, c->pairs_t}; }

static void apply_shape(vb_ctx *c, const Shape &sh) {
  c->step_unroll = sh.unroll;
  c->xcd_remap = sh.xcd;
  if (sh.pairs_t != c->pairs_t) {
    c->pairs_t = sh.pairs_t;
    size_pair_search(c);
  }
}

// Shapes chosen by vb_tune, kept for the life of the process and keyed by the
// batch's size (log2 of its particle count), its density (particles per cell, in
// quarters) and whether friction is on; vb_batch_create starts from the entry
// of its key.
using ShapeKey = std::tuple<int, int, int>;
static std::map<ShapeKey, Shape> g_shapes;
static std::mutex g_shapes_mutex;

static ShapeKey shape_key(const vb_ctx *c) {
  int64_t cells = 0;
  for (const SysDev &S : c->sys_h) cells += (int64_t)S.nc[0] * S.nc[1] * S.nc[2];
  const int lg = c->n_total > 0 ? (int)std::floor(std::log2((double)c->n_total)) : 0;
  const int dens = (int)std::lround(4.0 * (double)c->n_total / (double)std::max<int64_t>(cells, 1));
  return ShapeKey(lg, dens, c->any_friction);
}

// Friction history: cap entries per slot, double-buffered, plus the snapshot
// vb_run keeps to run a call again.  The contents are not kept (a regrow runs
// the call again from its snapshot, which is re-laid by copy_hist).
static vb_status alloc_hist_tables(vb_ctx *c, int32_t cap) {
  for (int b = 0; b < 2; ++b) {
    if (c->hist[b]) (void)hipFree(c->hist[b]);
    if (c->hcnt[b]) (void)hipFree(c->hcnt[b]);
    c->hist[b] = nullptr;
    c->hcnt[b] = nullptr;
    HIP_OK(c, dalloc(&c->hist[b], c->slots * (int64_t)cap));
    HIP_OK(c, dalloc(&c->hcnt[b], c->slots));
    HIP_OK(c, hipMemset(c->hcnt[b], 0, sizeof(int32_t) * c->slots));
  }
  c->hcap = cap;
  return VB_OK;
}

static vb_status alloc_bins(vb_ctx *c, int32_t cap) {
  if (c->bins_bp) (void)hipFree(c->bins_bp);
  if (c->bins_og) (void)hipFree(c->bins_og);
  c->bins_bp = nullptr;
  c->bins_og = nullptr;
  HIP_OK(c, dalloc(&c->bins_bp, c->n_cells * (int64_t)cap + BIN_PAD));
  HIP_OK(c, dalloc(&c->bins_og, c->n_cells * (int64_t)cap + BIN_PAD));
  c->bin_cap = cap;
  return VB_OK;
}

static vb_status alloc_hist(vb_ctx *c, int64_t steps) {
  const int64_t need = std::max<int64_t>(steps, STATS_RING) * c->n_sys;
  if (need <= c->hist_cap) return VB_OK;
  if (c->hist_d) (void)hipFree(c->hist_d);
  c->hist_d = nullptr;
  HIP_OK(c, dalloc(&c->hist_d, need));
  c->hist_cap = need;
  return VB_OK;
}

extern "C" vb_status vb_batch_create(const vb_params *h_params, const int64_t *h_n,
                                     int32_t n_sys, void *stream, vb_ctx **out) {
  if (!out) return fail(nullptr, VB_EINVAL, "out is NULL");
  *out = nullptr;
  if (!h_params || !h_n) return fail(nullptr, VB_EINVAL, "params or sizes NULL");
  if (n_sys < 1 || n_sys > MAX_SYS) return fail(nullptr, VB_EINVAL, "n_sys must be 1..1024");
  for (int s = 0; s < n_sys; ++s) {
    std::string m = check_params(h_params[s], h_n[s]);
    if (!m.empty()) return fail(nullptr, VB_EINVAL, "system " + std::to_string(s) + ": " + m);
  }
  vb_ctx *c = new (std::nothrow) vb_ctx();
  if (!c) return fail(nullptr, VB_ENOMEM, "host allocation failed");
  c->stream = reinterpret_cast<hipStream_t>(stream);
  const char *env = std::getenv("VBUF_XCD_REMAP");
  if (env) c->xcd_remap = std::min(2, std::max(0, std::atoi(env))), c->shape_fixed = 1;
  if ((env = std::getenv("VBUF_STEP_UNROLL"))) c->step_unroll = std::atoi(env), c->shape_fixed = 1;
  if ((env = std::getenv("VBUF_GRAPHS"))) c->use_graphs = std::atoi(env) != 0;
  if ((env = std::getenv("VBUF_PAIR_WINDOWS"))) c->xwindows = std::atoi(env) != 0;
  vb_status st = VB_OK;
  auto bail = [&](vb_status code) {
    g_create_error = c->msg;
    free_all(c);
    delete c;
    return code;
  };
  if (hipGetDevice(&c->device) != hipSuccess) {
    c->msg = "hipGetDevice failed";
    return bail(VB_EDEVICE);
  }
  if (!device_scratch(c->device)) {
    c->msg = "hipGetSymbolAddress of the export scratch failed";
    return bail(VB_EDEVICE);
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, c->device) != hipSuccess) {
    c->msg = "hipGetDeviceProperties failed";
    return bail(VB_EDEVICE);
  }
  c->n_cu = prop.multiProcessorCount;
  c->lds_limit = prop.sharedMemPerBlock;
  c->lds_cu = std::max(prop.maxSharedMemoryPerMultiProcessor, prop.sharedMemPerBlock);
  for (int nt : {256, 384, 512})
    if (pairs_static_lds(nt) < 0 || pairs_static_lds(nt) > PAIRS_STATIC_LDS) {
      c->msg = "pair search: static LDS above its reserve";
      return bail(VB_EDEVICE);
    }
  // rows are sorted in LDS: the widest row any pair-search shape (up to 512
  // threads per workgroup) can hold
  c->row_limit = (int32_t)std::min<size_t>(MAX_ROW, (c->lds_limit - PAIRS_STATIC_LDS - pairs_lds_bytes(0, 0, 512)) /
                                                         (512 * sizeof(uint16_t)));
  c->row_limit -= c->row_limit % ROW_GROUP;  // rows are stored in whole groups
  c->n_sys = n_sys;
  c->sys_h.resize(n_sys);
  c->sort_interval = h_params[0].reorder_interval;
  int64_t p_off = 0, t_off = 0, c_off = 0, o_off = 0, b_off = 0;
  int32_t width = 1, bcap = 1;
  for (int s = 0; s < n_sys; ++s) {
    const vb_params &p = h_params[s];
    SysDev &S = c->sys_h[s];
    std::memset(&S, 0, sizeof(S));
    S.n = (int32_t)h_n[s];
    S.n_tiles = (int32_t)((h_n[s] + TILE - 1) / TILE);
    S.p_off = p_off;
    S.tile_off = t_off;
    S.c_off = c_off;
    S.o_off = o_off;
    S.b_off = b_off;
    if (make_grid(p, S) > (1LL << 30)) {
      c->msg = "system " + std::to_string(s) + ": cell grid too fine for the box";
      return bail(VB_EINVAL);
    }
    S.dt = p.dt;
    S.K = p.K;
    S.kn = p.kn;
    S.gamma_n = p.gamma_n;
    S.skin_uniform = p.skin_uniform;
    S.cap = p.cap_mode == 0 ? 0.5 * p.cell_size : p.cell_size;
    for (int a = 0; a < 3; ++a) {
      S.lo[a] = p.lo[a];
      S.hi[a] = p.hi[a];
      S.g[a] = p.gravity[a];
    }
    S.eps = (float)p.eps;
    S.skin_mode = p.skin_mode;
    S.fixed_interval = p.fixed_interval < 1 ? 1 : p.fixed_interval;
    S.ring = p.cap_mode == 0 ? 1 : 2;
    S.kt = p.kt;
    S.gamma_t = p.gamma_t;
    S.mu = p.mu;
    S.friction = p.mu > 0.0 && (p.kt > 0.0 || p.gamma_t > 0.0);
    c->any_friction |= S.friction;
    c->hcap = std::max(c->hcap, p.contact_capacity > 0 ? p.contact_capacity : 16);
    S.n_planes = p.n_planes;
    for (int w = 0; w < p.n_planes; ++w)
      for (int c = 0; c < 5; ++c) S.planes[w][c] = p.planes[w][c];
    c->any_walls |= p.n_planes > 0 || p.n_cylinders > 0;
    S.n_cyl = p.n_cylinders;
    for (int w = 0; w < p.n_cylinders; ++w)
      for (int c = 0; c < 4; ++c) S.cyl[w][c] = p.cylinders[w][c];
    {  // grid of the coded positions: the box and two cells beyond each face,
       // 2^19 - 1 steps along its longest edge
      double span = 0.0;
      for (int a = 0; a < 3; ++a) {
        S.qlo[a] = p.lo[a] - 2.0 * p.cell_size;
        span = std::max(span, p.hi[a] - p.lo[a] + 4.0 * p.cell_size);
      }
      S.qinv = (double)((1 << 19) - 1) / span;
      S.qinv32 = (float)S.qinv;
    }
    p_off += (int64_t)S.n_tiles * TILE;
    t_off += S.n_tiles;
    c_off += S.nkeys;
    o_off += S.n;
    b_off += (int64_t)S.nb[0] * S.nb[1] * S.nb[2];
    c->any_no_buffer |= p.skin_mode == VB_NO_BUFFER;
    c->any_fixed |= p.skin_mode == VB_FIXED_INTERVAL;
    width = std::max(width, p.max_neighbors);
    bcap = std::max(bcap, p.bin_capacity > 0 ? p.bin_capacity : 16);
    c->max_n = std::max(c->max_n, S.n);
  }
  width = (width + ROW_GROUP - 1) / ROW_GROUP * ROW_GROUP;
  if (width > c->row_limit) {
    c->msg = "max_neighbors exceeds " + std::to_string(c->row_limit) + " on this device";
    return bail(VB_EINVAL);
  }
  c->slots = p_off;
  c->n_tiles = t_off;
  c->n_cells = c_off;
  c->n_total = o_off;
  c->n_bricks = b_off;
  if (c->slots > (int64_t)INT32_MAX || c->n_cells > (int64_t)INT32_MAX) {
    c->msg = "batch too large";
    return bail(VB_EINVAL);
  }
  // the broad-phase kernels walk the tiles grid-stride from a bounded grid, so
  // that a step without broad phase costs two short launches
  c->broad_grid = (int)std::max<int64_t>(1, std::min<int64_t>(c->n_tiles, 8LL * c->n_cu));
  std::vector<int32_t> ts(std::max<int64_t>(c->n_tiles, 1), 0);
  for (int s = 0; s < n_sys; ++s)
    for (int t = 0; t < c->sys_h[s].n_tiles; ++t) ts[c->sys_h[s].tile_off + t] = s;

#define ALLOC(ptr, count)                                         \
  if (dalloc(&(ptr), (count)) != hipSuccess) {                    \
    c->msg = "device allocation failed: " #ptr;                   \
    return bail(VB_ENOMEM);                                       \
  }
  ALLOC(c->sys_d, n_sys);
  ALLOC(c->tile_sys, c->n_tiles);
  for (int b = 0; b < 2; ++b) {
    ALLOC(c->xs[b], c->slots);
    ALLOC(c->vs[b], c->slots);
    ALLOC(c->ri[b], c->slots);
    ALLOC(c->orig[b], c->slots);
    ALLOC(c->posq[b], c->slots);
  }
  ALLOC(c->rrange, 2 * n_sys);
  ALLOC(c->bp, c->slots);
  ALLOC(c->bp_alt, c->slots);
  ALLOC(c->cnt, c->slots);
  ALLOC(c->bin_count, c->n_cells);
  ALLOC(c->act, 2 * MAX_SYS + 2);
  ALLOC(c->cellid, c->slots);
  ALLOC(c->inv, c->slots);
  ALLOC(c->cell_count, c->n_cells);
  ALLOC(c->cell_start, c->n_cells + 1);
  ALLOC(c->block_sum, scan_blocks(c->n_cells) + 1);
  ALLOC(c->inslot, c->slots);
  ALLOC(c->perm0, c->slots);
  ALLOC(c->flags, 2 * n_sys);
  ALLOC(c->go, n_sys);
  ALLOC(c->overflow, 3);
  ALLOC(c->step_base_d, 1);
  ALLOC(c->err, 2);
  ALLOC(c->stats, (int64_t)STATS_RING * std::max<int64_t>(c->n_tiles, 1));
  ALLOC(c->rebuilt_ring, (int64_t)STATS_RING * n_sys);
  ALLOC(c->pair_counts, std::max<int32_t>(c->max_n, 1));
  ALLOC(c->pair_offsets, std::max<int32_t>(c->max_n, 1));
  ALLOC(c->pair_total, 1);
#undef ALLOC
  if ((st = alloc_rows(c, width)) != VB_OK) return bail(st);
  if (c->any_friction && (st = alloc_hist_tables(c, c->hcap)) != VB_OK) return bail(st);
  if (hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
    c->msg = "stream creation failed";
    return bail(VB_EDEVICE);
  }
  if ((st = alloc_bins(c, bcap)) != VB_OK) return bail(st);
  if ((st = alloc_hist(c, STATS_RING)) != VB_OK) return bail(st);
  if (hipMemcpy(c->sys_d, c->sys_h.data(), sizeof(SysDev) * n_sys, hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemcpy(c->tile_sys, ts.data(), sizeof(int32_t) * ts.size(), hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemset(c->act, 0, sizeof(int32_t) * (2 * MAX_SYS + 2)) != hipSuccess ||
      hipMemset(c->bin_count, 0, sizeof(int32_t) * std::max<int64_t>(c->n_cells, 1)) !=
          hipSuccess ||
      hipMemset(c->cell_count, 0, sizeof(int32_t) * std::max<int64_t>(c->n_cells, 1)) !=
          hipSuccess ||
      hipMemset(c->cnt, 0, sizeof(int32_t) * c->slots) != hipSuccess ||
      hipMemset(c->flags, 0, sizeof(int32_t) * 2 * n_sys) != hipSuccess ||
      hipMemset(c->go, 0, sizeof(int32_t) * n_sys) != hipSuccess ||
      hipMemset(c->overflow, 0, sizeof(int32_t) * 3) != hipSuccess ||
      hipMemset(c->rebuilt_ring, 0, sizeof(int32_t) * STATS_RING * n_sys) != hipSuccess ||
      hipDeviceSynchronize() != hipSuccess) {
    c->msg = "device initialisation failed";
    return bail(VB_EDEVICE);
  }
  if (!c->shape_fixed) {
    // the default shape keeps 4 partner gathers in flight per thread, where the
    // step kernel runs five waves per SIMD; 8 with friction on batches of 2^20
    // particles or more, whose step kernel holds more registers (four waves)
    if (!(c->any_friction && c->n_total >= (int64_t)1 << 20)) c->step_unroll = 4;
    // a shape tuned earlier in this process for batches like this one
    std::lock_guard<std::mutex> lock(g_shapes_mutex);
    auto it = g_shapes.find(shape_key(c));
    if (it != g_shapes.end()) apply_shape(c, it->second);
  }
  *out = c;
  return VB_OK;
}

extern "C" vb_status vb_create(const vb_params *h_params, int64_t n, void *stream,
                               vb_ctx **out) {
  return vb_batch_create(h_params, &n, 1, stream, out);
}

// Coded positions of xs[b] for the step kernel's pre-test.
static hipError_t fill_posq(vb_ctx *c, int b) {
  return launch_posq(c->sys_d, c->tile_sys, c->rrange, c->n_sys, c->xs[b], c->ri[c->scur], c->posq[b], c->slots,
                     c->stream);
}

// Clears the per-run control state on the stream: no pending violation, no
// broad phase under way, empty bins, no overflow.
static vb_status reset_control(vb_ctx *c) {
  HIP_OK(c, launch_fill_i32(c->flags, 2 * c->n_sys, 0, c->stream));
  HIP_OK(c, launch_fill_i32(c->go, c->n_sys, 0, c->stream));
  HIP_OK(c, launch_fill_i32(c->bin_count, c->n_cells, 0, c->stream));
  HIP_OK(c, launch_fill_i32(c->overflow, 3, 0, c->stream));
  return VB_OK;
}

extern "C" vb_status vb_set_state(vb_ctx *c, const double *d_x, const double *d_v,
                                  const float *d_rc, const float *d_invm,
                                  int32_t v_is_half_step) {
  if (!c) return fail(nullptr, VB_EINVAL, "ctx is NULL");
  if (c->n_total > 0 && (!d_x || !d_v || !d_rc || !d_invm))
    return fail(c, VB_EINVAL, "state pointers must not be NULL");
  HIP_OK(c, launch_fill_i32(c->err, 1, 0, c->stream));
  HIP_OK(c, launch_fill_i32(c->rrange, c->n_sys, 0x7F800000, c->stream));  // +inf
  HIP_OK(c, launch_fill_i32(c->rrange + c->n_sys, c->n_sys, 0, c->stream));
  for (int s = 0; s < c->n_sys; ++s)
    HIP_OK(c, launch_set_state(c->sys_h[s], c->xs[0], c->vs[0], c->ri[0], c->orig[0], d_x, d_v,
                               d_rc, d_invm, c->err,
                               c->rrange + s, c->rrange + c->n_sys + s, c->stream));
  c->scur = 0;
  HIP_OK(c, launch_fill_i32(c->cnt, c->slots, 0, c->stream));
  HIP_OK(c, fill_posq(c, 0));
  if (c->any_friction) HIP_OK(c, launch_fill_i32(c->hcnt[0], c->slots, 0, c->stream));
  vb_status st = reset_control(c);
  if (st != VB_OK) return st;
  int32_t err = 0;
  HIP_OK(c, hipMemcpyAsync(&err, c->err, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
  HIP_OK(c, hipStreamSynchronize(c->stream));
  c->loaded = 0;
  if (err & 1) return fail(c, VB_ENONFINITE, "state holds NaN or Inf");
  if (err & 2) return fail(c, VB_EINVAL, "a radius is <= 0 or exceeds the cap of R_NL");
  if (err & 4) return fail(c, VB_EINVAL, "an inverse mass is <= 0");
  c->cur = 0;
  c->step = 0;
  c->first = v_is_half_step ? 0 : 1;
  c->force_pending = 1;
  c->relist_pending = 0;
  c->have_list = 0;
  c->next_sort = 0;
  c->loaded = 1;
  c->fresh = 1;
  return VB_OK;
}

static BroadArgs broad_args(vb_ctx *c, int force, int relist) {
  BroadArgs a;
  a.sys = c->sys_d;
  a.tile_sys = c->tile_sys;
  a.n_sys = c->n_sys;
  a.n_tiles = c->n_tiles;
  a.x = c->xs[c->cur];
  a.v = c->vs[c->cur];
  a.ri = c->ri[c->scur];
  a.orig = c->orig[c->scur];
  a.bp = c->bp;
  a.cnt = c->cnt;
  a.nbr = c->nbr;
  a.stride = c->slots;
  a.width = c->width;
  a.bin_count = c->bin_count;
  a.bins_bp = c->bins_bp;
  a.bins_og = c->bins_og;
  a.bin_cap = c->bin_cap;
  a.act = c->act;
  a.n_bricks = c->n_bricks;
  a.pmax = c->pmax;
  a.xwindows = c->xwindows;
  a.inv = c->inv;
  a.flags = c->flags;
  a.go = c->go;
  a.rebuilt_ring = c->rebuilt_ring;
  a.overflow = c->overflow;
  a.step = c->graph_mode ? c->graph_off : (int32_t)c->step;
  a.step_base = c->graph_mode ? c->step_base_d : nullptr;
  a.force = force;
  a.relist = relist;
  return a;
}

// Work that precedes the step kernel of the current step: the storage re-sort
// when it is due (x0 and R_NL move with their particles; the rows, which hold
// slots, are then rebuilt from them without a broad phase, so the schedule of
// broad phases does not change), and the conditional broad phase.
// t0/t1 (may be null) take the start and end of the broad-phase kernels.
static vb_status queue_broad_phase(vb_ctx *c, hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr) {
  if (c->next_sort >= 0 && c->step >= c->next_sort && c->n_tiles > 0) {
    SortArgs s;
    s.sys = c->sys_d;
    s.tile_sys = c->tile_sys;
    s.n_tiles = c->n_tiles;
    s.n_cells = c->n_cells;
    s.x_src = c->xs[c->cur];
    s.v_src = c->vs[c->cur];
    s.ri_src = c->ri[c->scur];
    s.orig_src = c->orig[c->scur];
    s.x_dst = c->xs[c->cur ^ 1];
    s.v_dst = c->vs[c->cur ^ 1];
    s.ri_dst = c->ri[c->scur ^ 1];
    s.orig_dst = c->orig[c->scur ^ 1];
    s.bp_src = c->bp;
    s.bp_dst = c->bp_alt;
    s.cell_count = c->cell_count;
    s.cell_start = c->cell_start;
    s.block_sum = c->block_sum;
    s.cellid = c->cellid;
    s.inslot = c->inslot;
    s.perm0 = c->perm0;
    s.hist_src = c->any_friction ? c->hist[c->cur] : nullptr;
    s.hcnt_src = c->any_friction ? c->hcnt[c->cur] : nullptr;
    s.hist_dst = c->any_friction ? c->hist[c->cur ^ 1] : nullptr;
    s.hcnt_dst = c->any_friction ? c->hcnt[c->cur ^ 1] : nullptr;
    s.hcap = c->hcap;
    s.stride = c->slots;
    HIP_OK(c, launch_sort(s, c->stream));
    c->cur ^= 1;
    c->scur ^= 1;
    std::swap(c->bp, c->bp_alt);
    HIP_OK(c, fill_posq(c, c->cur));
    c->relist_pending = 1;  // slots moved: every row must be rebuilt
    c->next_sort = c->sort_interval > 0 ? c->step + c->sort_interval : -1;
  }
  HIP_OK(c, launch_broad_phase(broad_args(c, c->force_pending, c->relist_pending), c->broad_grid,
                               c->pairs_grid, c->pairs_t, c->stream, t0, t1));
  c->force_pending = 0;
  c->relist_pending = 0;
  return VB_OK;
}

static vb_status queue_step(vb_ctx *c, hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr) {
  StepArgs a;
  a.sys = c->sys_d;
  a.tile_sys = c->tile_sys;
  a.x_cur = c->xs[c->cur];
  a.v_cur = c->vs[c->cur];
  a.x_dst = c->xs[c->cur ^ 1];
  a.v_dst = c->vs[c->cur ^ 1];
  a.ri = c->ri[c->scur];
  a.orig = c->orig[c->scur];
  a.posq_cur = c->posq[c->cur];
  a.posq_dst = c->posq[c->cur ^ 1];
  a.rrange = c->rrange;
  a.bp = c->bp;
  a.cnt = c->cnt;
  a.nbr = c->nbr;
  a.stride = c->slots;
  a.go = c->go;
  a.flags = c->flags;
  a.bin_count = c->bin_count;
  a.n_sys = c->n_sys;
  a.stats = c->stats;
  a.n_tiles = c->n_tiles;
  a.step = c->graph_mode ? c->graph_off : (int32_t)c->step;
  a.step_base = c->graph_mode ? c->step_base_d : nullptr;
  a.first = c->first;
  a.xcd_remap = c->xcd_remap;
  a.width = c->width;
  a.hist_cur = c->hist[c->cur];
  a.hcnt_cur = c->hcnt[c->cur];
  a.hist_dst = c->hist[c->cur ^ 1];
  a.hcnt_dst = c->hcnt[c->cur ^ 1];
  a.hcap = c->hcap;
  a.overflow = c->overflow;
  HIP_OK(c, launch_step(a, c->n_tiles, c->step_unroll, c->any_friction, c->any_walls, c->stream,
                        t0, t1));
  return VB_OK;
}

static vb_status ensure_events(vb_ctx *c, size_t n) {
  while (c->ev.size() < n) {
    hipEvent_t e;
    HIP_OK(c, hipEventCreate(&e));
    c->ev.push_back(e);
  }
  return VB_OK;
}

// Queues n_steps steps; records go to hist_d[r * n_sys + s].
// What a captured block of steps bakes in: buffers, sizes, launch shapes.
static uint64_t graph_key(const vb_ctx *c, int cur) {
  const uint64_t parts[] = {(uint64_t)(uintptr_t)c->xs[cur], (uint64_t)(uintptr_t)c->nbr,
                            (uint64_t)(uintptr_t)c->ri[c->scur], (uint64_t)(uintptr_t)c->orig[c->scur],
                            (uint64_t)(uintptr_t)c->bp,
                            (uint64_t)(uintptr_t)c->bins_bp, (uint64_t)(uintptr_t)c->bins_og,
                            (uint64_t)(uintptr_t)c->hist[cur], (uint64_t)(uintptr_t)c->hist[cur ^ 1],
                            (uint64_t)(uintptr_t)c->stream, (uint64_t)c->width, (uint64_t)c->pmax,
                            (uint64_t)c->bin_cap, (uint64_t)c->hcap, (uint64_t)c->step_unroll,
                            (uint64_t)c->xcd_remap, (uint64_t)c->pairs_t, (uint64_t)c->pairs_grid,
                            (uint64_t)cur};
  uint64_t h = 1469598103934665603ull;  // FNV-1a over the words
  for (uint64_t w : parts)
    for (int b = 0; b < 8; ++b) h = (h ^ ((w >> (8 * b)) & 0xff)) * 1099511628211ull;
  return h | 1;
}

// Captures STATS_RING steps (broad-phase gate, pair search, step kernel each)
// starting from ping-pong parity cur, with the step read from step_base_d.
static vb_status capture_block(vb_ctx *c, int cur) {
  if (c->graph_exec[cur]) (void)hipGraphExecDestroy(c->graph_exec[cur]);
  c->graph_exec[cur] = nullptr;
  c->graph_key[cur] = 0;
  const hipStream_t saved_stream = c->stream;
  const int saved_cur = c->cur;
  c->stream = c->cap_stream;
  c->cur = cur;
  c->graph_mode = 1;
  vb_status st = VB_OK;
  hipGraph_t g = nullptr;
  if (hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    st = fail(c, VB_EDEVICE, "hipStreamBeginCapture failed");
  } else {
    for (int32_t i = 0; i < STATS_RING && st == VB_OK; ++i) {
      c->graph_off = i;
      BroadArgs b = broad_args(c, 0, 0);
      if (launch_broad_phase(b, c->broad_grid, c->pairs_grid, c->pairs_t, c->stream, nullptr, nullptr) !=
          hipSuccess)
        st = fail(c, VB_EDEVICE, "capture of the broad phase failed");
      else if ((st = queue_step(c)) == VB_OK)
        c->cur ^= 1;
    }
    const hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
    if (st == VB_OK && e != hipSuccess) st = fail(c, VB_EDEVICE, "hipStreamEndCapture failed");
  }
  if (st == VB_OK && hipGraphInstantiate(&c->graph_exec[cur], g, nullptr, nullptr, 0) != hipSuccess)
    st = fail(c, VB_EDEVICE, "hipGraphInstantiate failed");
  if (g) (void)hipGraphDestroy(g);
  c->graph_mode = 0;
  c->graph_off = 0;
  c->stream = saved_stream;
  c->cur = saved_cur;
  if (st == VB_OK) c->graph_key[cur] = graph_key(c, cur);
  return st;
}

// Queues n_steps steps; records go to hist_d[r * n_sys + s].  Blocks of
// STATS_RING steps run as one replayed graph when nothing in them needs the
// host (no timing, first step, forced broad phase or storage re-sort).
// After a block of steps: requests the overflow counters and looks at those
// requested after the block before, which has finished by then (one block
// stays queued ahead, so the device does not wait).  *seen is set when they
// show a row, a bin or a history beyond its capacity: the rest of the call
// would be run again anyway.
static vb_status overflow_seen(vb_ctx *c, bool *seen) {
  *seen = false;
  if (!c->ovf_host) {
    HIP_OK(c, hipHostMalloc(reinterpret_cast<void **>(&c->ovf_host), 6 * sizeof(int32_t)));
    for (hipEvent_t &e : c->ovf_ev) HIP_OK(c, hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  if (c->ovf_n > 0) {
    const int prev = (c->ovf_n - 1) & 1;
    HIP_OK(c, hipEventSynchronize(c->ovf_ev[prev]));
    const int32_t *o = c->ovf_host + 3 * prev;
    if (o[0] > c->width || o[1] > c->bin_cap || o[2] > c->hcap) {
      *seen = true;
      return VB_OK;
    }
  }
  const int k = c->ovf_n & 1;
  HIP_OK(c, hipMemcpyAsync(c->ovf_host + 3 * k, c->overflow, 3 * sizeof(int32_t),
                           hipMemcpyDeviceToHost, c->stream));
  HIP_OK(c, hipEventRecord(c->ovf_ev[k], c->stream));
  ++c->ovf_n;
  return VB_OK;
}

// Blocks of STATS_RING steps between two snapshots of a call.  A call keeps a
// snapshot of its first step and of every SNAP_BLOCKS-th block boundary after
// it, each taken once every step before it is known free of overflow; a row, a
// bin or a history that outgrows its capacity runs the call again from the last
// snapshot, so at most SNAP_BLOCKS + 1 blocks run twice.
constexpr int SNAP_BLOCKS = 4;

// Keeps the state at the current step (call step index `at`): positions and
// velocities, x0 and R_NL, the pending validity flags, the friction history and
// the host's step bookkeeping.  The rows are not kept: a restore rebuilds them
// from x0 and R_NL.
static vb_status take_snapshot(vb_ctx *c, int32_t at) {
  if (!c->snap_x) {
    HIP_OK(c, dalloc(&c->snap_x, c->slots));
    HIP_OK(c, dalloc(&c->snap_v, c->slots));
    HIP_OK(c, dalloc(&c->snap_ri, c->slots));
    HIP_OK(c, dalloc(&c->snap_orig, c->slots));
    HIP_OK(c, dalloc(&c->snap_bp, c->slots));
    HIP_OK(c, dalloc(&c->snap_flags, 2 * (int64_t)c->n_sys));
  }
  HIP_OK(c, hipMemcpyAsync(c->snap_x, c->xs[c->cur], sizeof(X3) * c->slots,
                           hipMemcpyDeviceToDevice, c->stream));
  HIP_OK(c, hipMemcpyAsync(c->snap_v, c->vs[c->cur], sizeof(V3) * c->slots,
                           hipMemcpyDeviceToDevice, c->stream));
  HIP_OK(c, hipMemcpyAsync(c->snap_ri, c->ri[c->scur], sizeof(float2) * c->slots,
                           hipMemcpyDeviceToDevice, c->stream));
  HIP_OK(c, hipMemcpyAsync(c->snap_orig, c->orig[c->scur], sizeof(uint32_t) * c->slots,
                           hipMemcpyDeviceToDevice, c->stream));
  HIP_OK(c, hipMemcpyAsync(c->snap_bp, c->bp, sizeof(float4) * c->slots, hipMemcpyDeviceToDevice,
                           c->stream));
  HIP_OK(c, hipMemcpyAsync(c->snap_flags, c->flags, sizeof(int32_t) * 2 * c->n_sys,
                           hipMemcpyDeviceToDevice, c->stream));
  if (c->any_friction) {
    if (c->hist_snap_cap < c->hcap) {
      if (c->hist_snap) (void)hipFree(c->hist_snap);
      c->hist_snap = nullptr;
      HIP_OK(c, dalloc(&c->hist_snap, c->slots * (int64_t)c->hcap));
      c->hist_snap_cap = c->hcap;
    }
    if (!c->hcnt_snap) HIP_OK(c, dalloc(&c->hcnt_snap, c->slots));
    HIP_OK(c, hipMemcpyAsync(c->hist_snap, c->hist[c->cur], sizeof(HistEntry) * c->slots * c->hcap,
                             hipMemcpyDeviceToDevice, c->stream));
    HIP_OK(c, hipMemcpyAsync(c->hcnt_snap, c->hcnt[c->cur], sizeof(int32_t) * c->slots,
                             hipMemcpyDeviceToDevice, c->stream));
    c->snap.hcap = c->hcap;
  }
  c->snap.at = at;
  c->snap.step = c->step;
  c->snap.next_sort = c->next_sort;
  c->snap.first = c->first;
  c->snap.force = c->force_pending;
  return VB_OK;
}

// Back to the snapshot.  The rows are rebuilt at its step from its x0 and R_NL
// (a broad phase where one was pending there), so the run from it repeats the
// same schedule of broad phases, whatever capacities grew meanwhile.
static vb_status restore_snapshot(vb_ctx *c) {
  HIP_OK(c, hipMemcpyAsync(c->xs[0], c->snap_x, sizeof(X3) * c->slots, hipMemcpyDeviceToDevice,
                           c->stream));
  HIP_OK(c, hipMemcpyAsync(c->vs[0], c->snap_v, sizeof(V3) * c->slots, hipMemcpyDeviceToDevice,
                           c->stream));
  HIP_OK(c, hipMemcpyAsync(c->ri[0], c->snap_ri, sizeof(float2) * c->slots, hipMemcpyDeviceToDevice,
                           c->stream));
  HIP_OK(c, hipMemcpyAsync(c->orig[0], c->snap_orig, sizeof(uint32_t) * c->slots,
                           hipMemcpyDeviceToDevice, c->stream));
  c->scur = 0;
  HIP_OK(c, hipMemcpyAsync(c->bp, c->snap_bp, sizeof(float4) * c->slots, hipMemcpyDeviceToDevice,
                           c->stream));
  HIP_OK(c, launch_fill_i32(c->cnt, c->slots, 0, c->stream));
  HIP_OK(c, fill_posq(c, 0));
  if (c->any_friction) {  // entries c < snap.hcap sit at the same place in a wider table
    HIP_OK(c, hipMemcpyAsync(c->hist[0], c->hist_snap, sizeof(HistEntry) * c->slots * c->snap.hcap,
                             hipMemcpyDeviceToDevice, c->stream));
    HIP_OK(c, hipMemcpyAsync(c->hcnt[0], c->hcnt_snap, sizeof(int32_t) * c->slots,
                             hipMemcpyDeviceToDevice, c->stream));
  }
  vb_status st = reset_control(c);
  if (st != VB_OK) return st;
  HIP_OK(c, hipMemcpyAsync(c->flags, c->snap_flags, sizeof(int32_t) * 2 * c->n_sys,
                           hipMemcpyDeviceToDevice, c->stream));
  c->cur = 0;
  c->step = c->snap.step;
  c->next_sort = c->snap.next_sort;
  c->first = c->snap.first;
  c->force_pending = c->snap.force;
  c->relist_pending = 1;
  return VB_OK;
}

// Waits for every queued step and reads the overflow counters.
static vb_status overflow_now(vb_ctx *c, bool *seen) {
  int32_t ovf[3] = {0, 0, 0};
  HIP_OK(c, hipMemcpyAsync(ovf, c->overflow, sizeof(ovf), hipMemcpyDeviceToHost, c->stream));
  HIP_OK(c, hipStreamSynchronize(c->stream));
  *seen = ovf[0] > c->width || ovf[1] > c->bin_cap || ovf[2] > c->hcap;
  c->ovf_n = 0;  // nothing left to look at one block behind
  return VB_OK;
}

// Queues the steps i0 .. n_steps-1 of the call (records go to hist_d[i * n_sys
// + s]); *done receives the call index reached, and *seen is set when the
// overflow counters showed a row, a bin or a history beyond its capacity (the
// steps since the last snapshot are then to be run again).  With timing on,
// four events per step take the kernels' own start and end times: binning
// start and pair-search end, step-kernel start and end.
static vb_status run_steps(vb_ctx *c, int32_t i0, int32_t n_steps, int32_t *done, bool *seen) {
  vb_status st;
  *seen = false;
  c->ovf_n = 0;
  *done = i0;
  int32_t pending = 0;
  int blocks = 0;  // blocks queued since the last snapshot
  for (int32_t i = i0; i < n_steps;) {
    if (blocks >= SNAP_BLOCKS && pending == 0) {
      if ((st = overflow_now(c, seen)) != VB_OK) return st;
      if (*seen) return VB_OK;
      if ((st = take_snapshot(c, i)) != VB_OK) return st;
      blocks = 0;
    }
    const bool block = c->use_graphs && !c->timing && !c->first && !c->force_pending &&
                       !c->relist_pending && n_steps - i >= STATS_RING && c->n_tiles > 0 &&
                       (c->next_sort < 0 || c->next_sort >= c->step + STATS_RING);
    if (block && pending > 0) {  // close the records of the steps before the block
      HIP_OK(c, launch_stats_reduce(c->sys_d, c->stats, c->rebuilt_ring, c->n_tiles, c->n_sys,
                                    (int32_t)(c->step - pending), pending,
                                    c->hist_d + (int64_t)(i - pending) * c->n_sys, c->stream));
      pending = 0;
    }
    if (block) {
      const int cur = c->cur;
      if (!c->graph_exec[cur] || c->graph_key[cur] != graph_key(c, cur))
        if ((st = capture_block(c, cur)) != VB_OK) return st;
      HIP_OK(c, launch_fill_i32(c->step_base_d, 1, (int32_t)c->step, c->stream));
      HIP_OK(c, hipGraphLaunch(c->graph_exec[cur], c->stream));
      c->step += STATS_RING;  // an even count: the ping-pong parity is back to cur
      HIP_OK(c, launch_stats_reduce(c->sys_d, c->stats, c->rebuilt_ring, c->n_tiles, c->n_sys,
                                    (int32_t)(c->step - STATS_RING), STATS_RING,
                                    c->hist_d + (int64_t)i * c->n_sys, c->stream));
      i += STATS_RING;
      *done = i;
      ++blocks;
      if ((st = overflow_seen(c, seen)) != VB_OK) return st;
      if (*seen) return VB_OK;
      continue;
    }
    hipEvent_t *e = c->timing ? &c->ev[4 * (size_t)i] : nullptr;
    if ((st = queue_broad_phase(c, e ? e[0] : nullptr, e ? e[1] : nullptr)) != VB_OK) return st;
    if ((st = queue_step(c, e ? e[2] : nullptr, e ? e[3] : nullptr)) != VB_OK) return st;
    c->first = 0;
    c->cur ^= 1;
    c->step += 1;
    ++pending;
    if (pending == STATS_RING || i == n_steps - 1) {
      HIP_OK(c, launch_stats_reduce(c->sys_d, c->stats, c->rebuilt_ring, c->n_tiles, c->n_sys,
                                    (int32_t)(c->step - pending), pending,
                                    c->hist_d + (int64_t)(i + 1 - pending) * c->n_sys,
                                    c->stream));
      pending = 0;
      *done = i + 1;
      ++blocks;
      if (i + 1 < n_steps) {
        if ((st = overflow_seen(c, seen)) != VB_OK) return st;
        if (*seen) return VB_OK;
      }
    }
    ++i;
  }
  *done = n_steps;
  return VB_OK;
}

// Step records from the device.  A state that left the finite numbers (a time
// step far too large for the contact stiffness, say) shows in the kinetic
// energy of its step; the context then holds no usable state.
static vb_status read_records(vb_ctx *c, std::vector<vb_step_record> &rec, int32_t n_steps,
                              int64_t step0) {
  HIP_OK(c, hipMemcpy(rec.data(), c->hist_d, sizeof(vb_step_record) * rec.size(),
                      hipMemcpyDeviceToHost));
  for (int32_t r = 0; r < n_steps; ++r)
    for (int s = 0; s < c->n_sys; ++s)
      if (!std::isfinite(rec[(size_t)r * c->n_sys + s].kinetic_energy)) {
        c->loaded = 0;
        return fail(c, VB_ENONFINITE, "system " + std::to_string(s) + ": the kinetic energy "
                                      "is not finite at step " + std::to_string(step0 + r));
      }
  return VB_OK;
}

extern "C" vb_status vb_run(vb_ctx *c, int32_t n_steps, vb_step_record *h_hist) {
  if (!c) return fail(nullptr, VB_EINVAL, "ctx is NULL");
  if (!c->loaded) return fail(c, VB_EINVAL, "no state loaded (vb_set_state)");
  if (n_steps < 0) return fail(c, VB_EINVAL, "n_steps < 0");
  if (n_steps == 0) return VB_OK;
  if (c->step + n_steps > (int64_t)INT32_MAX) return fail(c, VB_EINVAL, "step counter overflow");
  c->fresh = 0;
  vb_status st;
  if ((st = alloc_hist(c, n_steps)) != VB_OK) return st;
  if (c->timing && (st = ensure_events(c, 4 * (size_t)n_steps)) != VB_OK) return st;
  const int64_t step0 = c->step;
  if ((st = take_snapshot(c, 0)) != VB_OK) return st;
  int32_t i0 = 0, retries = 0, last_restore = -1;
  for (;;) {
    int32_t done = 0;
    bool seen = false;
    if ((st = run_steps(c, i0, n_steps, &done, &seen)) != VB_OK) return st;
    int32_t ovf[3] = {0, 0, 0};
    HIP_OK(c, hipMemcpyAsync(ovf, c->overflow, sizeof(ovf), hipMemcpyDeviceToHost, c->stream));
    HIP_OK(c, hipStreamSynchronize(c->stream));
    if (ovf[0] <= c->width && ovf[1] <= c->bin_cap && ovf[2] <= c->hcap) {
      if (done != n_steps) return fail(c, VB_EDEVICE, "internal: a call stopped without overflow");
      break;
    }
    if (done > 0) {  // a diverged state piles up in the outermost cells: report that, not the bins
      std::vector<vb_step_record> rec((size_t)done * c->n_sys);
      if ((st = read_records(c, rec, done, step0)) != VB_OK) return st;
    }
    retries = c->snap.at == last_restore ? retries + 1 : 0;
    last_restore = c->snap.at;
    if (ovf[0] > c->row_limit || ovf[1] > MAX_BIN || ovf[2] > MAX_HIST || retries >= 4) {
      c->loaded = 0;
      return fail(c, VB_ECAPACITY,
                  "a Verlet-list row needs " + std::to_string(ovf[0]) + " entries (limit " +
                      std::to_string(c->row_limit) + "), a cell bin " + std::to_string(ovf[1]) +
                      " particles (limit 256) or a friction history " + std::to_string(ovf[2]) +
                      " contacts (limit " + std::to_string(MAX_HIST) + ")");
    }
    // grow, then run again from the last snapshot, which by construction lies
    // before the block that overflowed
    if (ovf[0] > c->width &&
        (st = alloc_rows(c, std::min<int32_t>(c->row_limit, (ovf[0] + ovf[0] / 4 + 7) / 8 * 8))) != VB_OK)
      return st;
    if (ovf[1] > c->bin_cap &&
        (st = alloc_bins(c, std::min<int32_t>(MAX_BIN, (ovf[1] + ovf[1] / 4 + 7) / 8 * 8))) != VB_OK)
      return st;
    if (ovf[2] > c->hcap &&
        (st = alloc_hist_tables(c, std::min<int32_t>(MAX_HIST, (ovf[2] + ovf[2] / 4 + 3) / 4 * 4))) != VB_OK)
      return st;
    if ((st = restore_snapshot(c)) != VB_OK) return st;
    i0 = c->snap.at;
  }
  c->have_list = 1;
  std::vector<vb_step_record> rec((size_t)n_steps * c->n_sys);
  if ((st = read_records(c, rec, n_steps, step0)) != VB_OK) return st;
  if (h_hist)
    for (int s = 0; s < c->n_sys; ++s)
      for (int32_t r = 0; r < n_steps; ++r)
        h_hist[(int64_t)s * n_steps + r] = rec[(size_t)r * c->n_sys + s];
  if (c->timing) {
    for (int32_t i = 0; i < n_steps; ++i) {
      float a = 0.f, b = 0.f;
      HIP_OK(c, hipEventElapsedTime(&a, c->ev[4 * (size_t)i], c->ev[4 * (size_t)i + 1]));
      HIP_OK(c, hipEventElapsedTime(&b, c->ev[4 * (size_t)i + 2], c->ev[4 * (size_t)i + 3]));
      c->ms_rebuild += a;
      c->ms_step += b;
      int any = 0;
      for (int s = 0; s < c->n_sys; ++s) any |= rec[(size_t)i * c->n_sys + s].rebuilt;
      c->t_rebuild_steps += any;
    }
    c->t_steps += n_steps;
  }
  return VB_OK;
}

extern "C" vb_status vb_get_state(vb_ctx *c, double *d_x, double *d_v,
                                  int32_t *h_v_is_half_step) {
  if (!c) return fail(nullptr, VB_EINVAL, "ctx is NULL");
  if (!c->loaded) return fail(c, VB_EINVAL, "no state loaded");
  HIP_OK(c, launch_get_state(c->sys_d, c->tile_sys, c->n_tiles, c->xs[c->cur], c->vs[c->cur],
                             c->orig[c->scur],
                             d_x, d_v, c->stream));
  HIP_OK(c, hipStreamSynchronize(c->stream));
  if (h_v_is_half_step) *h_v_is_half_step = c->first ? 0 : 1;
  return VB_OK;
}

extern "C" vb_status vb_get_verlet_state(vb_ctx *c, float *d_x0r, int32_t *h_pending,
                                         int64_t *h_step) {
  if (!c) return fail(nullptr, VB_EINVAL, "ctx is NULL");
  if (!c->loaded) return fail(c, VB_EINVAL, "no state loaded");
  if (!c->have_list) return fail(c, VB_EINVAL, "no list yet: run a step first");
  if (c->n_total > 0 && !d_x0r) return fail(c, VB_EINVAL, "d_x0r is NULL");
  if (c->n_total > 0)
    HIP_OK(c, launch_get_bp(c->sys_d, c->tile_sys, c->n_tiles, c->orig[c->scur], c->bp,
                            reinterpret_cast<float4 *>(d_x0r), c->stream));
  std::vector<int32_t> fl((size_t)c->n_sys, 0);
  HIP_OK(c, hipMemcpyAsync(fl.data(), c->flags + (c->step & 1) * c->n_sys, sizeof(int32_t) * c->n_sys,
                           hipMemcpyDeviceToHost, c->stream));
  HIP_OK(c, hipStreamSynchronize(c->stream));
  if (h_pending)
    for (int s = 0; s < c->n_sys; ++s) h_pending[s] = (fl[s] != 0 || c->force_pending) ? 1 : 0;
  if (h_step) *h_step = c->step;
  return VB_OK;
}

extern "C" vb_status vb_set_verlet_state(vb_ctx *c, const float *d_x0r, const int32_t *h_pending,
                                         int64_t step) {
  if (!c) return fail(nullptr, VB_EINVAL, "ctx is NULL");
  if (!c->loaded || !c->fresh)
    return fail(c, VB_EINVAL, "a Verlet state is loaded right after vb_set_state, before any step");
  if (!h_pending || (c->n_total > 0 && !d_x0r)) return fail(c, VB_EINVAL, "input pointer is NULL");
  if (step < 0 || step >= (int64_t)INT32_MAX) return fail(c, VB_EINVAL, "step out of range");
  std::vector<int32_t> fl((size_t)2 * c->n_sys, 0);
  for (int s = 0; s < c->n_sys; ++s) {
    if (h_pending[s] != 0 && h_pending[s] != 1) return fail(c, VB_EINVAL, "pending flags are 0 or 1");
    fl[(size_t)(step & 1) * c->n_sys + s] = h_pending[s];
  }
  HIP_OK(c, launch_fill_i32(c->err, 1, 0, c->stream));
  if (c->n_total > 0)
    HIP_OK(c, launch_set_bp(c->sys_d, c->tile_sys, c->n_tiles, c->orig[c->scur], c->ri[c->scur],
                            reinterpret_cast<const float4 *>(d_x0r), c->bp, c->err, c->stream));
  int32_t err = 0;
  HIP_OK(c, hipMemcpyAsync(&err, c->err, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
  HIP_OK(c, hipStreamSynchronize(c->stream));
  if (err & 1) return fail(c, VB_ENONFINITE, "x0 or R_NL holds NaN or Inf");
  if (err & 2) return fail(c, VB_EINVAL, "an R_NL is below its R_C or beyond the cap");
  HIP_OK(c, hipMemcpyAsync(c->flags, fl.data(), sizeof(int32_t) * fl.size(), hipMemcpyHostToDevice,
                           c->stream));
  HIP_OK(c, hipStreamSynchronize(c->stream));
  c->step = step;
  c->force_pending = 0;
  c->relist_pending = 1;
  c->have_list = 1;
  return VB_OK;
}

extern "C" vb_status vb_get_history(vb_ctx *c, int32_t *d_partner, double *d_spring, int32_t cap,
                                    int32_t *h_needed) {
  if (!c) return fail(nullptr, VB_EINVAL, "ctx is NULL");
  if (!c->any_friction) return fail(c, VB_EINVAL, "no system of this context has friction");
  if (!c->loaded) return fail(c, VB_EINVAL, "no state loaded");
  if (cap < 0 || (cap > 0 && (!d_partner || !d_spring)))
    return fail(c, VB_EINVAL, "bad output buffers");
  HIP_OK(c, launch_fill_i32(c->err, 1, 0, c->stream));
  HIP_OK(c, launch_get_history(c->sys_d, c->tile_sys, c->n_tiles, c->orig[c->scur], c->hist[c->cur],
                               c->hcnt[c->cur], c->slots, c->hcap, d_partner, d_spring, cap,
                               c->err, c->stream));
  int32_t needed = 0;
  HIP_OK(c, hipMemcpyAsync(&needed, c->err, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
  HIP_OK(c, hipStreamSynchronize(c->stream));
  if (h_needed) *h_needed = needed;
  if (needed > cap)
    return fail(c, VB_ECAPACITY, "a particle has " + std::to_string(needed) + " contacts, cap is " +
                                     std::to_string(cap));
  return VB_OK;
}

extern "C" vb_status vb_set_history(vb_ctx *c, const int32_t *d_partner, const double *d_spring,
                                    int32_t cap) {
  if (!c) return fail(nullptr, VB_EINVAL, "ctx is NULL");
  if (!c->any_friction) return fail(c, VB_EINVAL, "no system of this context has friction");
  if (!c->loaded || !c->fresh)
    return fail(c, VB_EINVAL, "a history is loaded right after vb_set_state, before any step");
  if (cap < 0 || (cap > 0 && (!d_partner || !d_spring))) return fail(c, VB_EINVAL, "bad input buffers");
  if (cap == 0) return VB_OK;
  // count and check first (err[0]: largest count, err[1]: faults), then grow
  // the tables if they are too small, then load
  HIP_OK(c, launch_fill_i32(c->err, 2, 0, c->stream));
  for (int s = 0; s < c->n_sys; ++s)
    if (c->sys_h[s].friction)
      HIP_OK(c, launch_check_history(c->sys_h[s], d_partner, d_spring, cap, c->err, c->err + 1,
                                     c->stream));
  int32_t chk[2] = {0, 0};
  HIP_OK(c, hipMemcpyAsync(chk, c->err, sizeof(chk), hipMemcpyDeviceToHost, c->stream));
  HIP_OK(c, hipStreamSynchronize(c->stream));
  if (chk[1] & 1) return fail(c, VB_ENONFINITE, "a spring holds NaN or Inf");
  if (chk[1] & 2)
    return fail(c, VB_EINVAL, "a partner is out of range, the particle itself, or out of order");
  if (chk[0] > MAX_HIST)
    return fail(c, VB_ECAPACITY, "a particle has " + std::to_string(chk[0]) + " contacts (limit " +
                                     std::to_string(MAX_HIST) + ")");
  vb_status st;
  if (chk[0] > c->hcap && (st = alloc_hist_tables(c, std::min(MAX_HIST, (chk[0] + 3) / 4 * 4))) != VB_OK)
    return st;
  HIP_OK(c, launch_set_history(c->sys_d, c->tile_sys, c->n_tiles, c->orig[c->scur], d_partner,
                               d_spring, cap, c->hist[c->cur], c->hcnt[c->cur], c->slots, c->stream));
  HIP_OK(c, hipStreamSynchronize(c->stream));
  return VB_OK;
}

extern "C" vb_status vb_get_pairs(vb_ctx *c, int32_t sys, int32_t which, int32_t *d_pairs,
                                  double *d_delta, int64_t cap, int64_t *h_n) {
  if (!c) return fail(nullptr, VB_EINVAL, "ctx is NULL");
  if (!c->loaded) return fail(c, VB_EINVAL, "no state loaded");
  if (sys < 0 || sys >= c->n_sys) return fail(c, VB_EINVAL, "sys out of range");
  if (which != 0 && which != 1) return fail(c, VB_EINVAL, "which must be 0 or 1");
  if (cap < 0 || (cap > 0 && !d_pairs)) return fail(c, VB_EINVAL, "bad output buffer");
  vb_status st;
  if (which == 1) {
    // the broad phase the next step would run, if any; the next step repeats it
    // when its flag is still set, so the bins are emptied again here
    if ((st = queue_broad_phase(c)) != VB_OK) return st;
    HIP_OK(c, launch_fill_i32(c->bin_count, c->n_cells, 0, c->stream));
    int32_t ovf[2] = {0, 0};
    HIP_OK(c, hipMemcpyAsync(ovf, c->overflow, sizeof(ovf), hipMemcpyDeviceToHost, c->stream));
    HIP_OK(c, hipStreamSynchronize(c->stream));
    if (ovf[0] > c->width || ovf[1] > c->bin_cap)
      return fail(c, VB_ECAPACITY, "list row or cell bin overflow in the broad phase; run a "
                                   "step first so that vb_run grows them");
  }
  HIP_OK(c, launch_pairs(c->sys_h[sys], c->xs[c->cur], c->ri[c->scur], c->orig[c->scur], c->cnt,
                         c->nbr, c->slots, which,
                         c->pair_counts, c->pair_offsets, c->pair_total, cap,
                         cap > 0 ? d_pairs : nullptr, cap > 0 ? d_delta : nullptr, c->stream));
  int64_t total = 0;
  HIP_OK(c, hipMemcpyAsync(&total, c->pair_total, sizeof(int64_t), hipMemcpyDeviceToHost,
                           c->stream));
  HIP_OK(c, hipStreamSynchronize(c->stream));
  if (c->sys_h[sys].n == 0) total = 0;
  if (h_n) *h_n = total;
  return VB_OK;
}

extern "C" vb_status vb_get_pairs_noalloc(vb_ctx *c, int32_t sys, int32_t which, int32_t *d_pairs,
                                          double *d_delta, int64_t cap, int64_t *h_n) {
  if (!c) return fail(nullptr, VB_EINVAL, "ctx is NULL");
  if (!c->loaded) return fail(c, VB_EINVAL, "no state loaded");
  if (sys < 0 || sys >= c->n_sys) return fail(c, VB_EINVAL, "sys out of range");
  if (which != 0 && which != 1) return fail(c, VB_EINVAL, "which must be 0 or 1");
  if (cap < 0 || (cap > 0 && !d_pairs)) return fail(c, VB_EINVAL, "bad output buffer");
  if (c->sys_h[sys].n > VB_NOALLOC_MAX_N)
    return fail(c, VB_EINVAL, "system " + std::to_string(sys) + " has " +
                                  std::to_string(c->sys_h[sys].n) + " particles; the allocation-free "
                                  "export takes at most " + std::to_string(VB_NOALLOC_MAX_N));
  unsigned char *base = static_cast<unsigned char *>(g_scratch[c->device]);
  if (!base) return fail(c, VB_EDEVICE, "no export scratch on this device");
  // counts [n] int32, offsets [n] int64 and the total, 8-byte aligned
  int32_t *counts = reinterpret_cast<int32_t *>(base);
  int64_t *offsets = reinterpret_cast<int64_t *>(base + 4 * (int64_t)VB_NOALLOC_MAX_N);
  int64_t *total_d = reinterpret_cast<int64_t *>(base + 12 * (int64_t)VB_NOALLOC_MAX_N);
  vb_status st;
  if (which == 1) {  // as vb_get_pairs: the broad phase the next step would run, if any
    if ((st = queue_broad_phase(c)) != VB_OK) return st;
    HIP_OK(c, launch_fill_i32(c->bin_count, c->n_cells, 0, c->stream));
    int32_t ovf[2] = {0, 0};
    HIP_OK(c, hipMemcpyAsync(ovf, c->overflow, sizeof(ovf), hipMemcpyDeviceToHost, c->stream));
    HIP_OK(c, hipStreamSynchronize(c->stream));
    if (ovf[0] > c->width || ovf[1] > c->bin_cap)
      return fail(c, VB_ECAPACITY, "list row or cell bin overflow in the broad phase; run a "
                                   "step first so that vb_run grows them");
  }
  HIP_OK(c, launch_pairs(c->sys_h[sys], c->xs[c->cur], c->ri[c->scur], c->orig[c->scur], c->cnt,
                         c->nbr, c->slots, which, counts,
                         offsets, total_d, cap, cap > 0 ? d_pairs : nullptr,
                         cap > 0 ? d_delta : nullptr, c->stream));
  int64_t total = 0;
  HIP_OK(c, hipMemcpyAsync(&total, total_d, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream));
  HIP_OK(c, hipStreamSynchronize(c->stream));
  if (c->sys_h[sys].n == 0) total = 0;
  if (h_n) *h_n = total;
  return VB_OK;
}

extern "C" vb_status vb_set_launch(vb_ctx *c, int32_t unroll, int32_t xcd_order, int32_t pairs_threads) {
  if (!c) return fail(nullptr, VB_EINVAL, "ctx is NULL");
  const Shape sh{unroll, xcd_order, pairs_threads};
  if (!shape_ok(sh))
    return fail(c, VB_EINVAL, "launch shape: unroll 1, 2, 4 or 8; xcd_order 0, 1 or 2; pairs_threads "
                              "256, 384 or 512");
  apply_shape(c, sh);
  return VB_OK;
}

extern "C" vb_status vb_get_launch(vb_ctx *c, int32_t *h_unroll, int32_t *h_xcd_order,
                                   int32_t *h_pairs_threads) {
  if (!c) return fail(nullptr, VB_EINVAL, "ctx is NULL");
  if (h_unroll) *h_unroll = c->step_unroll;
  if (h_xcd_order) *h_xcd_order = c->xcd_remap;
  if (h_pairs_threads) *h_pairs_threads = c->pairs_t;
  return VB_OK;
}

extern "C" vb_status vb_tune(vb_ctx *c, int32_t n_steps, vb_step_record *h_hist) {
  if (!c) return fail(nullptr, VB_EINVAL, "ctx is NULL");
  if (!c->loaded) return fail(c, VB_EINVAL, "no state loaded (vb_set_state)");
  const Shape step_cands[] = {{8, 2, 0}, {8, 0, 0}, {8, 1, 0}, {4, 2, 0}, {4, 0, 0},
                              {4, 1, 0}, {2, 2, 0}, {2, 0, 0}, {2, 1, 0}};
  const int pair_cands[] = {256, 384, 512};
  constexpr int N_STEP = 9, N_PAIR = 3, PAIR_REPS = 2;
  // trials: the starting shape and up to N_STEP others (the starting one may
  // lie outside the list), then the pair-search sizes
  const int32_t trial = std::max<int32_t>(2, n_steps / 16);
  if (n_steps < (N_STEP + 1) * trial + N_PAIR * PAIR_REPS)
    return fail(c, VB_EINVAL, "vb_tune needs at least " +
                                  std::to_string((N_STEP + 1) * 2 + N_PAIR * PAIR_REPS) + " steps");
  // the caller's timing totals are set aside while the tuner times its trials
  const bool timing0 = c->timing;
  const double ms_rebuild0 = c->ms_rebuild, ms_step0 = c->ms_step;
  const int64_t t_steps0 = c->t_steps, t_rebuild0 = c->t_rebuild_steps;
  std::vector<vb_step_record> part;
  int32_t done = 0;
  auto run = [&](int32_t steps) -> vb_status {
    part.assign((size_t)c->n_sys * steps, vb_step_record{});
    vb_status st = vb_run(c, steps, part.data());
    if (st != VB_OK) return st;
    if (h_hist)
      for (int s = 0; s < c->n_sys; ++s)
        for (int32_t r = 0; r < steps; ++r)
          h_hist[(int64_t)s * n_steps + done + r] = part[(size_t)s * steps + r];
    done += steps;
    return VB_OK;
  };
  auto restore_timing = [&]() {
    c->timing = timing0;
    c->ms_rebuild = ms_rebuild0;
    c->ms_step = ms_step0;
    c->t_steps = t_steps0;
    c->t_rebuild_steps = t_rebuild0;
  };
  vb_status st = VB_OK;
  const Shape start = current_shape(c);
  Shape best = start;
  // The shape the context starts from is timed first and kept unless another
  // is faster by more than SWITCH_MARGIN: trials are short, and a shape that
  // wins by less is within their noise.
  constexpr double SWITCH_MARGIN = 0.01;
  // 1) the step kernel: every gather count and tile order for `trial` steps,
  //    timed by HIP events on the kernel itself
  double best_ms = INFINITY;
  c->timing = true;
  for (int i = -1; i < N_STEP && st == VB_OK; ++i) {
    const Shape sh = i < 0 ? start : Shape{step_cands[i].unroll, step_cands[i].xcd, start.pairs_t};
    if (i >= 0 && sh.unroll == start.unroll && sh.xcd == start.xcd) continue;
    apply_shape(c, sh);
    c->ms_step = 0.0;
    c->t_steps = 0;
    if ((st = run(trial)) != VB_OK) break;
    const double ms = c->ms_step / trial;
    if (i < 0 || ms < best_ms * (1.0 - SWITCH_MARGIN)) {
      best_ms = ms;
      best.unroll = sh.unroll;
      best.xcd = sh.xcd;
    }
  }
  // 2) the pair search: every workgroup size on PAIR_REPS forced broad phases
  //    (which change no result, theorem of Sec. 4.2), timed from the start of the
  //    binning to the end of the pair search, the starting size first
  best_ms = INFINITY;
  for (int i = -1; i < N_PAIR && st == VB_OK; ++i) {
    const int nt = i < 0 ? start.pairs_t : pair_cands[i];
    if (i >= 0 && nt == start.pairs_t) continue;
    const Shape sh{best.unroll, best.xcd, nt};
    apply_shape(c, sh);
    c->ms_rebuild = 0.0;
    for (int r = 0; r < PAIR_REPS && st == VB_OK; ++r) {
      c->force_pending = 1;
      st = run(1);
    }
    if (st == VB_OK && (i < 0 || c->ms_rebuild < best_ms * (1.0 - SWITCH_MARGIN))) {
      best_ms = c->ms_rebuild;
      best.pairs_t = nt;
    }
  }
  restore_timing();
  if (st != VB_OK) return st;
  // 3) the rest of the steps with the chosen shape, which later contexts of
  //    this kind start from
  apply_shape(c, best);
  {
    std::lock_guard<std::mutex> lock(g_shapes_mutex);
    g_shapes[shape_key(c)] = best;
  }
  if (n_steps > done && (st = run(n_steps - done)) != VB_OK) return st;
  return VB_OK;
}

extern "C" vb_status vb_force_rebuild(vb_ctx *c) {
  if (!c) return fail(nullptr, VB_EINVAL, "ctx is NULL");
  c->force_pending = 1;
  return VB_OK;
}

extern "C" vb_status vb_set_K(vb_ctx *c, int32_t sys, double K) {
  if (!c) return fail(nullptr, VB_EINVAL, "ctx is NULL");
  if (!(K >= 0.0) || !std::isfinite(K)) return fail(c, VB_EINVAL, "K must be finite and >= 0");
  if (sys >= c->n_sys) return fail(c, VB_EINVAL, "sys out of range");
  for (int s = 0; s < c->n_sys; ++s)
    if (sys < 0 || s == sys) c->sys_h[s].K = K;
  // queued behind the work already on the stream, which still reads the old K
  HIP_OK(c, hipMemcpyAsync(c->sys_d, c->sys_h.data(), sizeof(SysDev) * c->n_sys,
                           hipMemcpyHostToDevice, c->stream));
  HIP_OK(c, hipStreamSynchronize(c->stream));
  return VB_OK;
}

extern "C" vb_status vb_set_timing(vb_ctx *c, int32_t on) {
  if (!c) return fail(nullptr, VB_EINVAL, "ctx is NULL");
  c->timing = on != 0;
  c->ms_rebuild = c->ms_step = 0.0;
  c->t_steps = c->t_rebuild_steps = 0;
  return VB_OK;
}

extern "C" vb_status vb_phase_times(vb_ctx *c, double *h_ms_rebuild, double *h_ms_step,
                                    int64_t *h_steps, int64_t *h_rebuild_steps) {
  if (!c) return fail(nullptr, VB_EINVAL, "ctx is NULL");
  if (h_ms_rebuild) *h_ms_rebuild = c->ms_rebuild;
  if (h_ms_step) *h_ms_step = c->ms_step;
  if (h_steps) *h_steps = c->t_steps;
  if (h_rebuild_steps) *h_rebuild_steps = c->t_rebuild_steps;
  return VB_OK;
}

extern "C" vb_status vb_get_info(vb_ctx *c, int64_t *h_n_total, int32_t *h_n_sys,
                                 int32_t *h_row_width, int64_t *h_step) {
  if (!c) return fail(nullptr, VB_EINVAL, "ctx is NULL");
  if (h_n_total) *h_n_total = c->n_total;
  if (h_n_sys) *h_n_sys = c->n_sys;
  if (h_row_width) *h_row_width = c->width;
  if (h_step) *h_step = c->step;
  return VB_OK;
}

extern "C" const char *vb_last_error(const vb_ctx *c) {
  return c ? c->msg.c_str() : g_create_error.c_str();
}

extern "C" void vb_destroy(vb_ctx *c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  free_all(c);
  delete c;
}
