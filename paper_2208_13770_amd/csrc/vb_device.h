// vb_device.h -- device-side data layout of libvbuf (internal).
//
// Particles live in "slots".  Each system of a batch owns a contiguous range of
// slots padded to a multiple of TILE, so a tile (one workgroup) never straddles
// two systems.  What a step changes (position, velocity) is kept apart from what
// only a storage sort moves (R_C, 1/m, original index), so that a step writes
// the 48 bytes of state it changes and nothing else.  The slot order is
// re-sorted by cell from time to time for locality (not at every broad phase),
// so rows of the Verlet list hold slots and are ordered by original index.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/vbuf.h"

namespace vb {

constexpr int TILE = 256;         // particles per tile = threads per workgroup
constexpr int WAVE = 64;          // CDNA wavefront
constexpr int MAX_SYS = 1024;     // systems per batch
constexpr int STATS_RING = 64;    // steps of per-tile statistics kept before reduction
constexpr int MAX_ROW = 128;      // largest Verlet-list row (rows are sorted in LDS)
constexpr int MAX_BIN = 256;      // largest cell-bin capacity
constexpr int MAX_HIST = 64;      // largest friction history per particle (contacts)
constexpr int SCAN_ITEMS = 16;    // cells per thread in the block-level scans
constexpr int BRICK = 4;          // cells per brick edge: cells are numbered brick by brick
constexpr int MAX_CAND = 24;      // row entries per segment of the step kernel's two-pass scan
                                  // (24 KB of LDS candidates: five workgroups per CU)
static_assert(MAX_CAND % 8 == 0, "segments start on a whole step of the largest unroll");
constexpr int CONTACT_UNROLL = 2; // candidates whose records are requested together (94 VGPRs
                                  // at U = 4: five waves per SIMD)
constexpr int PAIRS_T = 384;      // threads of a pair-search workgroup (one brick): a brick of
                                  // 64 cells at about 5 particles per cell in one pass
constexpr int BIN_PAD = 8;        // entries allocated past the last cell bin (read, never used)
constexpr int XRES = 8;           // sub-bins per cell edge along x that bound the pair
                                  // search's candidate windows
constexpr int PAIRS_STATIC_LDS = 13 * 1024;  // bound on the pair search's static LDS (bytes)
// Rows of the Verlet list are stored in groups of ROW_GROUP entries: group g of
// slot k is the int4 at nbr[(g * stride + k) * ROW_GROUP], entry q is component
// q % ROW_GROUP of group q / ROW_GROUP.  One 16-byte load fetches four entries of
// a row, and a wave's lanes read one group as 1 KB of consecutive memory.  Row
// widths are multiples of ROW_GROUP.
constexpr int ROW_GROUP = 4;
__host__ __device__ __forceinline__ int64_t row_index(int64_t stride, int64_t k, int q) {
  return ((int64_t)(q / ROW_GROUP) * stride + k) * ROW_GROUP + (q % ROW_GROUP);
}

// Position of a slot, 24 B: FP64 centre.  Double-buffered (a step reads one
// buffer and writes the other).
struct X3 {
  double x, y, z;
};
// Velocity of a slot, 24 B: FP64 velocity (the half-step velocity once running).
// Double-buffered like the position.
struct V3 {
  double vx, vy, vz;
};
static_assert(sizeof(X3) == 24 && sizeof(V3) == 24, "state records are 24 bytes");
// Per slot and constant between storage sorts: float2 (R_C, 1/m) and the
// original index (uint32), each in an array of its own.

// One system of the batch, as the kernels see it.
struct SysDev {
  int64_t p_off;      // first slot
  int64_t tile_off;   // first tile
  int64_t c_off;      // first cell of the system in the concatenated cell arrays
  int64_t o_off;      // first index of the system in the caller's concatenated order
  int32_t n;          // particles
  int32_t n_tiles;    // tiles
  int64_t b_off;      // first brick of the system in the concatenated brick list
  int32_t nc[3];      // cells per axis
  int32_t nb[3];      // bricks per axis, ceil(nc / BRICK)
  int32_t nkeys;      // cell numbers in use: nb[0] * nb[1] * nb[2] * BRICK^3
  double inv_edge[3]; // 1 / cell edge per axis (binning is done in FP64)
  double dt, K, kn, gamma_n, skin_uniform, cap;
  double lo[3], hi[3], g[3];
  float eps;
  int32_t skin_mode;
  int32_t fixed_interval;
  int32_t ring;       // cell rings searched: 1 (cap mode 0) or 2 (cap mode 1)
  // grid of the step kernel's coded positions: 19-bit coordinates of pitch
  // 1/qinv from qlo, covering the box and two cells beyond each face
  double qlo[3];
  double qinv;
  float qinv32;       // qinv rounded to FP32, for the pre-test
  int32_t n_planes;   // planar walls besides the box faces
  int32_t friction;   // 1: tangential spring-dashpot with Coulomb limit on the contacts
  double planes[VB_MAX_PLANES][5];  // (n_x, n_y, n_z, d, z_min) as in vb_params
  double kt, gamma_t, mu;           // friction law
  int32_t n_cyl;      // vertical cylindrical walls
  int32_t pad_cyl;
  double cyl[VB_MAX_CYLINDERS][4];  // (c_x, c_y, R, z_min) as in vb_params
};

// One entry of a particle's friction history: a contact of the previous step
// (partner's original index) and the tangential spring of that contact as seen
// from the particle.  Entries of a particle are ordered by partner.
struct alignas(16) HistEntry {
  double sx, sy, sz;
  uint32_t orig;
  uint32_t pad;
};
static_assert(sizeof(HistEntry) == 32, "history entries are 32 bytes");

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

// Arguments of the two broad-phase kernels (binning, pair search).
struct BroadArgs {
  const SysDev *sys;
  const int32_t *tile_sys;
  int32_t n_sys;
  int64_t n_tiles;
  const X3 *x;
  const V3 *v;
  const float2 *ri;     // [slots] (R_C, 1/m)
  const uint32_t *orig; // [slots] original index
  float4 *bp;           // [slots] x0 (FP32) and R_NL of the broad phase
  int32_t *cnt;         // [slots] row lengths
  int32_t *nbr;         // rows in groups of four entries: entry q of slot k at row_index(stride, k, q)
  int64_t stride;
  int32_t width;        // row capacity W
  int32_t *bin_count;   // [cells] particles binned per cell (zeroed by the step kernel)
  float4 *bins_bp;      // [cells][bin_cap] x0 and R_NL of the binned particles
  int32_t *bins_og;     // [cells][bin_cap] original index of the binned particles (slots via inv)
  int32_t bin_cap;
  // the systems that take part in this broad phase, written by the binning for
  // the pair search: act[0] = their count A, act[1 + i] = system i of them (in
  // index order), act[1 + MAX_SYS + i] = bricks of the systems before it (i <= A)
  int32_t *act;
  int64_t n_bricks;
  int32_t pmax;         // candidates a workgroup can stage in LDS
  int32_t xwindows;     // 1: staged rows are searched in x windows (0: whole rows)
  int32_t *inv;         // [slots] inv[p_off + orig] = local slot (written when force or relist is set)
  const int32_t *flags; // [2][n_sys] validity-violation flags; slot (step & 1) is read
  int32_t *go;          // [n_sys] 1 if the system runs a broad phase at this step
  int32_t *rebuilt_ring;  // [STATS_RING][n_sys]
  int32_t *overflow;    // [0] longest row beyond W, [1] fullest bin beyond bin_cap
  int32_t step;         // the step, or its offset from *step_base when step_base is set
  const int32_t *step_base;  // device step counter of a replayed graph (else null)
  int32_t force;        // 1: broad phase for every system regardless of flags
  int32_t relist;       // 1: every system without a broad phase at this step rebuilds its
                        //    rows from the stored x0 and R_NL (bp), keeping both
};

// Arguments of the fused step kernel.
struct StepArgs {
  const SysDev *sys;
  const int32_t *tile_sys;
  const X3 *x_cur;
  const V3 *v_cur;
  X3 *x_dst;
  V3 *v_dst;
  const float2 *ri;          // [slots] (R_C, 1/m)
  const uint32_t *orig;      // [slots] original index
  const uint64_t *posq_cur;  // coded positions and radius bounds of x_cur
  uint64_t *posq_dst;        // written with x_dst
  const int32_t *rrange;     // [2][n_sys] FP32 bits of each system's smallest and largest R_C
  const float4 *bp;
  const int32_t *cnt;
  const int32_t *nbr;
  int64_t stride;
  const int32_t *go;     // [n_sys] broad phase ran at this step
  int32_t *flags;        // [2][n_sys]
  int32_t *bin_count;    // cleared after a broad phase
  int32_t n_sys;
  TileStats *stats;      // [STATS_RING][n_tiles_total]
  int64_t n_tiles;
  int32_t step;          // the step, or its offset from *step_base when step_base is set
  const int32_t *step_base;  // device step counter of a replayed graph (else null)
  int32_t first;         // 1: the velocities are the full-step v^0 (no first half kick)
  int32_t xcd_remap;     // tile order: 0 launch order, 1 a contiguous range per XCD,
                         // 2 runs of consecutive tiles per XCD
  int32_t width;         // row capacity W (entries below it are allocated)
  // friction history (used only when some system has friction): column-major,
  // entry c of slot k at hist[c * stride + k]
  const HistEntry *hist_cur;
  const int32_t *hcnt_cur;
  HistEntry *hist_dst;
  int32_t *hcnt_dst;
  int32_t hcap;          // entries per slot
  int32_t *overflow;     // [2]: most contacts a particle had beyond hcap
};

// Arguments of the spatial re-sort (counting sort of the slots by cell).
struct SortArgs {
  const SysDev *sys;
  const int32_t *tile_sys;
  int64_t n_tiles;
  int64_t n_cells;
  const X3 *x_src;
  const V3 *v_src;
  const float2 *ri_src;
  const uint32_t *orig_src;
  X3 *x_dst;
  V3 *v_dst;
  float2 *ri_dst;
  uint32_t *orig_dst;
  const float4 *bp_src; // x0 and R_NL of the last broad phase move with their particle
  float4 *bp_dst;
  int32_t *cell_count;  // [cells] zero on entry, zero on exit
  int32_t *cell_start;  // [cells + 1]
  int32_t *block_sum;   // [scan blocks]
  int32_t *cellid;      // [slots]
  int32_t *inslot;      // [slots]
  int32_t *perm0;       // [slots]
  // friction history, moved with its particle (null when no system has friction)
  const HistEntry *hist_src;
  const int32_t *hcnt_src;
  HistEntry *hist_dst;
  int32_t *hcnt_dst;
  int32_t hcap;
  int64_t stride;       // slots
};

}  // namespace vb
