// vb_device.h -- device-side data layout of libvbuf (internal).
//
// Particles live in "slots".  Each system of a batch owns a contiguous range of
// slots padded to a multiple of TILE, so a tile (one workgroup of the step
// kernel) never straddles two systems.  Slots are kept in cell-sorted order (by
// cell, then by original index), re-permuted at every broad phase; the original
// index travels inside the position record.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vb {

constexpr int TILE = 256;         // particles per tile = threads per workgroup
constexpr int WAVE = 64;          // CDNA wavefront
constexpr int MAX_SYS = 1024;     // systems per batch
constexpr int STATS_RING = 64;    // steps of per-tile statistics kept before reduction
constexpr int MAX_ROW = 128;      // largest Verlet-list row (rows are sorted in LDS)

// Position record, 32 B: FP64 centre, FP32 cut-off radius R_C, original index.
struct alignas(16) PX {
  double x, y, z;
  float rc;
  uint32_t orig;
};
// Velocity record, 32 B: FP64 velocity (the half-step velocity once running),
// FP32 inverse mass.
struct alignas(16) PV {
  double vx, vy, vz;
  float invm;
  uint32_t pad;
};
static_assert(sizeof(PX) == 32 && sizeof(PV) == 32, "records are 32 bytes");

// One system of the batch, as the kernels see it.
struct SysDev {
  int64_t p_off;      // first slot
  int64_t tile_off;   // first tile
  int64_t c_off;      // first cell of the system in the concatenated cell arrays
  int64_t o_off;      // first index of the system in the caller's concatenated order
  int32_t n;          // particles
  int32_t n_tiles;    // tiles
  int32_t nc[3];      // cells per axis
  int32_t ncell;      // nc[0] * nc[1] * nc[2]
  double inv_edge[3]; // 1 / cell edge per axis (binning is done in FP64)
  double dt, K, kn, gamma_n, skin_uniform, cap;
  double lo[3], hi[3], g[3];
  float eps;
  int32_t skin_mode;
  int32_t fixed_interval;
  int32_t ring;       // cell rings searched: 1 (cap mode 0) or 2 (cap mode 1)
};

// Per-tile statistics of one step (reduced per system later, in a fixed order).
struct TileStats {
  double ke;          // sum of m |v^n|^2 / 2
  int32_t rowsum;     // sum of row lengths (twice the unique pairs)
  int32_t contacts2;  // contacts counted from both sides
  int32_t violators;  // particles failing the validity test after the step
  float max_excess;   // max (|x^{n+1} - x0| - skin_eff)
};

// Per-system, per-step record as kept on the device (mirrors vb_step_record).
struct RecordDev {
  int32_t step, rebuilt;
  int64_t list_pairs, contacts, violators;
  float max_excess;
  int32_t reserved;
  double kinetic_energy;
};

// Arguments of the fused step kernel.
struct StepArgs {
  const SysDev *sys;
  const int32_t *tile_sys;
  const PX *px_cur;
  const PV *pv_cur;
  const PX *px_tmp;   // permuted state written by a broad phase at this step
  const PV *pv_tmp;
  PX *px_dst;
  PV *pv_dst;
  const float4 *bp;   // x0 (FP32) and R_NL of the last broad phase
  const int32_t *cnt; // row lengths
  const int32_t *nbr; // rows, column-major: entry q of slot k at nbr[q * stride + k]
  int64_t stride;
  const int32_t *rebuilt_at;  // [n_sys] step of the last broad phase
  int32_t *flags;     // [2][n_sys] validity-violation flags, slot (step & 1)
  int32_t n_sys;
  TileStats *stats;   // [STATS_RING][n_tiles_total]
  int64_t n_tiles;
  int32_t step;
  int32_t first;      // 1: the velocities are the full-step v^0 (no first half kick)
  int32_t xcd_remap;  // 1: give each XCD a contiguous range of tiles
};

// Arguments of the broad-phase (rebuild) kernel.
struct RebuildArgs {
  const SysDev *sys;
  const int32_t *tile_sys;
  int32_t n_sys;
  int64_t n_tiles;
  int64_t n_cells;    // total cells of the batch
  const PX *px_cur;
  const PV *pv_cur;
  PX *px_tmp;
  PV *pv_tmp;
  float4 *bp;
  int32_t *cnt;
  int32_t *nbr;
  int64_t stride;
  int32_t width;      // row capacity W
  int32_t *cell_count;  // [n_cells]
  int32_t *cell_start;  // [n_cells + 1]
  int32_t *block_sum;   // [grid]
  int32_t *cellid;      // [slots] cell of each slot (current order)
  int32_t *cellid_new;  // [slots] cell of each slot (new order)
  int32_t *inslot;      // [slots] arrival rank inside its cell
  int32_t *perm0;       // [slots] provisional new order
  int32_t *perm;        // [slots] new order: perm[new slot] = old local slot
  int32_t *inv;         // [slots] inv[p_off + orig] = new local slot
  int32_t *rebuilt_at;
  int32_t *flags;
  int32_t *overflow;    // [1] largest row length seen beyond W (0 if none)
  int32_t step;
  int32_t force;        // 1: broad phase for every system regardless of flags
};

}  // namespace vb
