// vb_kernels.hip -- gfx950 kernels of the local Verlet buffer DEM step.
//
// Per time step three launches run on the context's stream:
//   k_bin    the start of the conditional broad phase (Def. autoverlet): for each
//            system whose list went invalid (Eq. update failed at the previous
//            step) or that is forced, the extended spheres of Eq. bounding_sphere
//            with the local skin of Eq. skin_formulus1 capped as in Eq.
//            skin_formulus_mincell, the reference positions x0, and the
//            binning of the particles into the uniform cells of Alg. 1;
//   k_pairs  the linked-cell pair search of Alg. 1 on those spheres, one
//            workgroup per brick of cells with the brick's neighbourhood staged
//            in LDS, one thread per particle, each row sorted by original index;
//   k_step   narrow phase (Eq. delta), normal spring-dashpot contact force (and
//            the tangential one with its per-contact history when friction is
//            on), box, planar and cylindrical walls, gravity, velocity-Verlet integration and
//            the displacement test of Eq. update for the next step, fused, one
//            thread per particle.
// Both broad-phase kernels return at once when no system needs a broad phase,
// so the host never waits on the validity flag.  A counting sort of the particle
// storage by cell (k_sort_*) runs when the host schedules it, for locality.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include "vb_device.h"

namespace vb {

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}
__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}
__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, WAVE));
  return v;
}

// Inclusive prefix sum over a TILE-thread block; *total receives the block sum.
template <int NT = TILE>
__device__ __forceinline__ int block_inclusive_scan(int v, int *total) {
  __shared__ int wsum[NT / WAVE];
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
#pragma unroll
  for (int o = 1; o < WAVE; o <<= 1) {
    int u = __shfl_up(v, o, WAVE);
    if (lane >= o) v += u;
  }
  if (lane == WAVE - 1) wsum[w] = v;
  __syncthreads();
  int before = 0, all = 0;
#pragma unroll
  for (int i = 0; i < NT / WAVE; ++i) {
    if (i < w) before += wsum[i];
    all += wsum[i];
  }
  __syncthreads();
  *total = all;
  return v + before;
}

__device__ __forceinline__ int64_t block_sum_i64(int64_t v) {
  __shared__ int64_t part[TILE / WAVE];
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
#pragma unroll
  for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  if (lane == 0) part[w] = v;
  __syncthreads();
  int64_t s = 0;
#pragma unroll
  for (int i = 0; i < TILE / WAVE; ++i) s += part[i];
  __syncthreads();
  return s;
}

// Overlap of two spheres, Eq. delta: delta = R_i + R_j - |x_i - x_j|, in FP64.
// Returns true iff delta > 0 (contact, Sec. 3.2), with the separation vector
// and distance for the force.  The cheap test on the squared distance only
// skips pairs whose overlap is certainly negative.
__device__ __forceinline__ bool overlap_positive(const X3 &a, float arc, const X3 &b, float brc,
                                                 double &dx, double &dy, double &dz, double &d,
                                                 double &delta) {
  dx = a.x - b.x;
  dy = a.y - b.y;
  dz = a.z - b.z;
  const double d2 = dx * dx + dy * dy + dz * dz;
  const double rs = (double)arc + (double)brc;
  if (!(d2 < rs * rs * (1.0 + 1e-12))) return false;
  d = sqrt(d2);
  delta = rs - d;
  return delta > 0.0;
}

// Coded positions of the step kernel's pre-test, 8 B per particle.  The centre
// is rounded to a grid of pitch h = 1/qinv (19 bits per axis: x in bits 0-18,
// y in 19-37, z in 38-56); bits 57-63 hold a code c whose bound
// rlo + c (rhi - rlo)/126, on the system's range [rlo, rhi] of R_C, is at
// least R_C.  Code 127 marks a centre off the grid or a radius without a code:
// such a particle passes every pre-test it takes part in.
constexpr int QBITS = 19;
constexpr uint32_t QMASK = (1u << QBITS) - 1u;
constexpr uint32_t QFREE = 127u;
// Margin of the pre-test in grid steps.  Rounding each centre moves the
// difference of two centres by at most sqrt(3) h; the FP32 arithmetic of the
// test adds under 0.1 h, since a reach is below 2^18 h (the grid spans at
// least four cells and R_C is at most one cell).
constexpr float QMARGIN = 2.5f;

__device__ __forceinline__ float radius_step(float rlo, float rhi) {
  return (rhi - rlo) * (1.0f / 126.0f);
}
__device__ __forceinline__ float radius_bound(float rlo, float step, uint32_t c) {
  return __fmaf_rn((float)c, step, rlo);
}

// The radius code of R_C = rc on the range [rlo, rhi]: the smallest c <= 126
// whose bound is at least rc, or QFREE if none is.
__device__ __forceinline__ uint32_t radius_code(float rlo, float rhi, float rc) {
  uint32_t c = QFREE;
  const float step = radius_step(rlo, rhi);
  if (rc <= rlo) {
    c = 0;
  } else if (step > 0.0f) {
    const float t = ceilf((rc - rlo) / step);
    uint32_t c0 = t < 126.0f ? (uint32_t)t : 126u;
    while (c0 < 126u && radius_bound(rlo, step, c0) < rc) ++c0;
    if (radius_bound(rlo, step, c0) >= rc) c = c0;
  }
  return c;
}

// The coded position of centre (x, y, z) with radius code c.
__device__ __forceinline__ uint64_t posq_encode_c(const SysDev &S, double x, double y, double z,
                                                  uint32_t c) {
  const double lim = (double)QMASK;  // t < 2^19 - 1 keeps floor(t + 1/2) within 19 bits
  const double tx = (x - S.qlo[0]) * S.qinv;
  const double ty = (y - S.qlo[1]) * S.qinv;
  const double tz = (z - S.qlo[2]) * S.qinv;
  if (!(tx >= 0.0 && tx < lim && ty >= 0.0 && ty < lim && tz >= 0.0 && tz < lim))
    return (uint64_t)QFREE << 57;
  const uint64_t qx = (uint32_t)(tx + 0.5), qy = (uint32_t)(ty + 0.5), qz = (uint32_t)(tz + 0.5);
  return qx | (qy << QBITS) | (qz << (2 * QBITS)) | ((uint64_t)c << 57);
}

__device__ __forceinline__ uint64_t posq_encode(const SysDev &S, float rlo, float rhi, double x,
                                                double y, double z, float rc) {
  return posq_encode_c(S, x, y, z, radius_code(rlo, rhi, rc));
}

// One side of the pre-test, decoded once per particle: grid coordinates and
// R_C in grid steps plus the margin (infinite for a particle without a code).
struct QSelf {
  int x, y, z;
  float reach0;
};
__device__ __forceinline__ QSelf posq_self(uint64_t q, float rc, float qinv32) {
  QSelf m;
  m.x = (int)(q & QMASK);
  m.y = (int)((q >> QBITS) & QMASK);
  m.z = (int)((q >> (2 * QBITS)) & QMASK);
  m.reach0 = (uint32_t)(q >> 57) == QFREE ? INFINITY : __fmaf_rn(rc, qinv32, QMARGIN);
  return m;
}

// Pre-test of a contact on coded positions: true whenever the exact FP64 test
// of Eq. delta can be.  rlo_q and step_q are the radius code's origin and step
// in grid steps.
__device__ __forceinline__ bool posq_candidate(const QSelf &m, uint2 o, float rlo_q,
                                               float step_q) {
  // the code's two 32-bit words: x in bits 0-18 of the low word, y across the
  // two, z in bits 6-24 of the high word, the radius code in its bits 25-31
  const float dx = (float)(m.x - (int)(o.x & QMASK));
  const float dy = (float)(m.y - (int)(__builtin_amdgcn_alignbit(o.y, o.x, QBITS) & QMASK));
  const float dz = (float)(m.z - (int)((o.y >> (2 * QBITS - 32)) & QMASK));
  const uint32_t c = o.y >> 25;
  const float reach = c == QFREE ? INFINITY : m.reach0 + __fmaf_rn((float)c, step_q, rlo_q);
  return __fmaf_rn(dx, dx, __fmaf_rn(dy, dy, dz * dz)) <= reach * reach;
}

// Tile of workgroup i of n in the step kernel's tile order.  The 8 XCDs receive
// workgroups round-robin (workgroup i on XCD i % 8), and each has its own L2.
//  0: tile i.  Tiles in flight at one time form one window of consecutive
//     tiles, spread over all XCDs.
//  1: each XCD walks a contiguous eighth of the tiles.
//  2: runs of XCD_RUN consecutive tiles go to one XCD, the 8 runs of a group
//     side by side, so that a tile's neighbours along the storage order are
//     mostly on its own XCD while the window stays one (a last group shorter
//     than 8 runs keeps order 0).
constexpr int64_t XCD_RUN = 32;
__device__ __forceinline__ int64_t xcd_tile(int64_t i, int64_t n, int order) {
  if (order == 1) {
    const int64_t x = i & 7, k = i >> 3;
    const int64_t q = n >> 3, r = n & 7;
    return x * q + (x < r ? x : r) + k;
  }
  if (order == 2) {
    const int64_t g = i / (8 * XCD_RUN);
    if ((g + 1) * 8 * XCD_RUN > n) return i;
    const int64_t r = i - g * 8 * XCD_RUN;
    return g * 8 * XCD_RUN + (r & 7) * XCD_RUN + (r >> 3);
  }
  return i;
}

// Cell number of integer cell coordinates.  Cells are numbered brick by brick
// (bricks of BRICK^3 cells, x fastest inside a brick and between bricks), so that
// cells close in space are close in memory.
__device__ __forceinline__ int cell_key(const SysDev &S, int cx, int cy, int cz) {
  const int brick = ((cz / BRICK) * S.nb[1] + (cy / BRICK)) * S.nb[0] + (cx / BRICK);
  return brick * (BRICK * BRICK * BRICK) +
         ((cz % BRICK) * BRICK + (cy % BRICK)) * BRICK + (cx % BRICK);
}

// Integer cell coordinates of a position (Alg. 1: uniform decomposition of the
// domain); positions outside the box fall in the border cells.
__device__ __forceinline__ void cell_coords(const SysDev &S, double x, double y, double z, int c[3]) {
  const double p[3] = {x, y, z};
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    double f = floor((p[ax] - S.lo[ax]) * S.inv_edge[ax]);
    f = fmin(fmax(f, 0.0), (double)(S.nc[ax] - 1));  // NaN -> 0, clamp to the grid
    c[ax] = (int)f;
  }
}

__device__ __forceinline__ int cell_of(const SysDev &S, double x, double y, double z) {
  int c[3];
  cell_coords(S, x, y, z, c);
  return cell_key(S, c[0], c[1], c[2]);
}

// Slot of each lane in its cell bin with one atomic per run of equal cells in
// the wave (the storage is sorted by cell, so neighbouring lanes mostly share a
// cell).  key < 0 marks a lane that bins nothing; returns the lane's slot.
__device__ __forceinline__ int wave_bin_slot(int32_t *count, int64_t key) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int64_t prev = __shfl_up(key, 1, WAVE);
  const bool head = lane == 0 || key != prev;
  const uint64_t heads = __ballot(head);
  const uint64_t upto = lane == WAVE - 1 ? ~0ull : ((2ull << lane) - 1ull);
  const int head_lane = 63 - __clzll((long long)(heads & upto));
  const uint64_t after = heads & ~upto;
  const int next = after ? __ffsll((long long)after) - 1 : WAVE;
  int base = 0;
  if (head && key >= 0) base = atomicAdd(&count[key], next - lane);
  base = __shfl(base, head_lane, WAVE);
  return base + (lane - head_lane);
}

// Does system s run a broad phase at this step?  (Def. autoverlet: when Eq.
// update failed after the previous step; always without buffer; every
// fixed_interval steps in the fixed-interval practice; when forced.)
__device__ __forceinline__ int needs_broad_phase(const SysDev &S, const int32_t *flags, int n_sys,
                                                 int s, int step, int force) {
  if (force || S.skin_mode == 2) return 1;
  if (S.skin_mode == 3) return (step % S.fixed_interval) == 0;
  return flags[(step & 1) * n_sys + s] != 0;
}

// Streaming accesses of the step kernel (the particle's own records, its row
// and its new state) carry the non-temporal hint, so that they do not evict the
// neighbour records the gathers reuse from L2.
typedef float vf4_t __attribute__((ext_vector_type(4)));
typedef double vd2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float4 nt_load(const float4 *p) {
  const vf4_t v = __builtin_nontemporal_load(reinterpret_cast<const vf4_t *>(p));
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ int32_t nt_load(const int32_t *p) { return __builtin_nontemporal_load(p); }
typedef int vi4_t __attribute__((ext_vector_type(4)));
// One group of four row entries (16 bytes), non-temporal.
__device__ __forceinline__ void nt_load_group(const int32_t *p, int32_t *out) {
  const vi4_t v = __builtin_nontemporal_load(reinterpret_cast<const vi4_t *>(p));
  out[0] = v.x;
  out[1] = v.y;
  out[2] = v.z;
  out[3] = v.w;
}
__device__ __forceinline__ void nt_store(float4 *p, const float4 &v) {
  const vf4_t w = {v.x, v.y, v.z, v.w};
  __builtin_nontemporal_store(w, reinterpret_cast<vf4_t *>(p));
}
// A 24-byte state record (three doubles, 8-byte aligned), non-temporal.
__device__ __forceinline__ void nt_store24(double *dst, double a, double b, double c) {
  __builtin_nontemporal_store(a, dst);
  __builtin_nontemporal_store(b, dst + 1);
  __builtin_nontemporal_store(c, dst + 2);
}

// ------------------------------------------------------------------ k_step

template <int UNROLL, bool FRIC, bool WALLS>
__global__ __launch_bounds__(TILE) void k_step(StepArgs a) {
  const int64_t t = xcd_tile(blockIdx.x, gridDim.x, a.xcd_remap);
  const int s = a.tile_sys[t];
  const SysDev &S = a.sys[s];
  const int lt = (int)(t - S.tile_off);
  const int local = lt * TILE + (int)threadIdx.x;
  const bool active = local < S.n;
  const int64_t k = S.p_off + local;
  const X3 *__restrict__ xs = a.x_cur;
  const V3 *__restrict__ vs = a.v_cur;
  const float *__restrict__ rcs = reinterpret_cast<const float *>(a.ri);  // R_C at 2k, 1/m at 2k+1
  const int step = a.step + (a.step_base ? *a.step_base : 0);
  __shared__ int32_t s_cand[MAX_CAND * TILE];  // per-thread lists of contact candidates

  // after a broad phase: empty this tile's share of the system's cell bins and
  // consume the flag that asked for it
  if (a.go[s]) {
    const int chunk = (S.nkeys + S.n_tiles - 1) / S.n_tiles;
    const int c1 = min(S.nkeys, (lt + 1) * chunk);
    for (int c = lt * chunk + (int)threadIdx.x; c < c1; c += TILE) a.bin_count[S.c_off + c] = 0;
    if (lt == 0 && threadIdx.x == 0) a.flags[(step & 1) * a.n_sys + s] = 0;
  }

  double ke = 0.0;
  int rowlen = 0, ncon = 0, viol = 0;
  float excess = -INFINITY;
  if (active) {
    // the particle's records and the first UNROLL row entries are requested
    // together: entries below the row width are always allocated, and an entry
    // is used only if it lies below the row length.  With UNROLL a multiple of
    // ROW_GROUP the row is read a group (four entries) per load.
    const int64_t st = a.stride;
    int32_t j[UNROLL];
    // entries q .. q+UNROLL-1 (q a multiple of UNROLL) that lie below limit
    auto load_entries = [&](int q, int limit, int32_t *dst) {
      if constexpr (UNROLL % ROW_GROUP == 0) {
#pragma unroll
        for (int g = 0; g < UNROLL / ROW_GROUP; ++g)
          if (q + g * ROW_GROUP < limit)
            nt_load_group(&a.nbr[row_index(st, k, q + g * ROW_GROUP)], dst + g * ROW_GROUP);
      } else {
#pragma unroll
        for (int u = 0; u < UNROLL; ++u)
          dst[u] = q + u < limit ? nt_load(&a.nbr[row_index(st, k, q + u)]) : 0;
      }
    };
    const int spec = min(UNROLL, a.width);
    load_entries(0, spec, j);
    const X3 me = xs[k];  // plain loads: the flushes of the neighbours gather them too
    const V3 mv = vs[k];
    const float2 mri = a.ri[k];
    const float mrc = mri.x;
    const float rlo = __int_as_float(a.rrange[s]), rhi = __int_as_float(a.rrange[a.n_sys + s]);
    const uint32_t mcode = radius_code(rlo, rhi, mrc);  // the same for both codes of this step
    const QSelf mq = posq_self(posq_encode_c(S, me.x, me.y, me.z, mcode), mrc, S.qinv32);
    const float rlo_q = rlo * S.qinv32, step_q = radius_step(rlo, rhi) * S.qinv32;
    const float4 b = nt_load(&a.bp[k]);
    rowlen = nt_load(&a.cnt[k]);
    double fx = 0.0, fy = 0.0, fz = 0.0;
    // friction history: this particle's contacts of the previous step (partner
    // ascending) are merged with this step's contacts, which come in the same
    // order; the new history holds exactly this step's contacts
    const bool fric = FRIC && S.friction;
    const int hn = fric ? a.hcnt_cur[k] : 0;
    int hp = 0, hc = 0;
    HistEntry hold;
    hold.orig = 0xFFFFFFFFu;
    if (hn > 0) hold = a.hist_cur[k];
    auto contact = [&](const X3 &o, float orc, const V3 &ov, uint32_t oorig) {
      double dx, dy, dz, d, delta;
      if (overlap_positive(me, mrc, o, orc, dx, dy, dz, d, delta)) {
        const double nx = dx / d, ny = dy / d, nz = dz / d;
        const double vn = (mv.vx - ov.vx) * nx + (mv.vy - ov.vy) * ny + (mv.vz - ov.vz) * nz;
        const double fm = S.kn * delta - S.gamma_n * vn;
        fx += fm * nx;
        fy += fm * ny;
        fz += fm * nz;
        ++ncon;
        if constexpr (FRIC) {
          if (fric) {
            // tangential linear spring-dashpot with a Coulomb limit: the spring
            // of the previous step, turned into the tangent plane, grows by
            // v_t dt; a force beyond mu F_n is cut back to the cone and the
            // spring set to the one that gives it
            while (hp < hn && hold.orig < oorig) {
              ++hp;
              if (hp < hn) hold = a.hist_cur[(int64_t)hp * st + k];
            }
            double sx = 0.0, sy = 0.0, sz = 0.0;
            if (hp < hn && hold.orig == oorig) {
              sx = hold.sx;
              sy = hold.sy;
              sz = hold.sz;
            }
            const double vtx = (mv.vx - ov.vx) - vn * nx;
            const double vty = (mv.vy - ov.vy) - vn * ny;
            const double vtz = (mv.vz - ov.vz) - vn * nz;
            const double sn = sx * nx + sy * ny + sz * nz;
            sx = (sx - sn * nx) + vtx * S.dt;
            sy = (sy - sn * ny) + vty * S.dt;
            sz = (sz - sn * nz) + vtz * S.dt;
            double ftx = -S.kt * sx - S.gamma_t * vtx;
            double fty = -S.kt * sy - S.gamma_t * vty;
            double ftz = -S.kt * sz - S.gamma_t * vtz;
            const double ftn = sqrt(ftx * ftx + fty * fty + ftz * ftz);
            const double lim = S.mu * (fm > 0.0 ? fm : 0.0);
            if (ftn > lim) {
              const double sc = lim / ftn;
              ftx *= sc;
              fty *= sc;
              ftz *= sc;
              sx = S.kt > 0.0 ? -(ftx + S.gamma_t * vtx) / S.kt : 0.0;
              sy = S.kt > 0.0 ? -(fty + S.gamma_t * vty) / S.kt : 0.0;
              sz = S.kt > 0.0 ? -(ftz + S.gamma_t * vtz) / S.kt : 0.0;
            }
            fx += ftx;
            fy += fty;
            fz += ftz;
            if (hc < a.hcap) {
              HistEntry e;
              e.sx = sx;
              e.sy = sy;
              e.sz = sz;
              e.orig = oorig;
              e.pad = 0;
              a.hist_dst[(int64_t)hc * st + k] = e;
            }
            ++hc;
          }
        }
      }
    };
    // Two passes over each segment of MAX_CAND row entries.  The scan walks the
    // row (ascending original index) with UNROLL gathers of the 8-byte coded
    // positions in flight, requesting the next chunk's row entries meanwhile,
    // and lists in LDS the partners that pass the conservative pre-test.  The
    // flush then requests the FP64 positions and the velocities of the listed
    // partners together, runs the exact test and adds the contact forces in
    // list (= row) order.
    // candidates whose records the flush requests together: one with friction,
    // whose contact law holds more registers
    constexpr int CU = FRIC ? 1 : CONTACT_UNROLL;
    for (int q0 = 0; q0 < rowlen; q0 += MAX_CAND) {
      const int q1 = min(rowlen, q0 + MAX_CAND);
      int nc = 0;
      for (int q = q0; q < q1; q += UNROLL) {
        // one gather per entry, issued for every lane: an entry past the
        // segment reads the system's first code instead of its stale index, so
        // no gather sits behind a branch and the compiler waits for each alone
        // (the extra requests all hit one line).  Codes are addressed from the
        // system's base, shared by the workgroup, with a 32-bit byte offset: a
        // system holds at most 2^29 - 256 particles, so 8 x index fits.
        uint2 o[UNROLL];
        const char *pq = reinterpret_cast<const char *>(a.posq_cur + S.p_off);
#pragma unroll
        for (int u = 0; u < UNROLL; ++u)
          o[u] = *reinterpret_cast<const uint2 *>(pq + (uint32_t)(q + u < q1 ? j[u] : 0) * 8u);
        int32_t jn[UNROLL];
        load_entries(q + UNROLL, rowlen, jn);
#pragma unroll
        for (int u = 0; u < UNROLL; ++u)
          if (q + u < q1 && posq_candidate(mq, o[u], rlo_q, step_q)) {
            s_cand[nc * TILE + threadIdx.x] = j[u];
            ++nc;
          }
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) j[u] = jn[u];
      }
      for (int i0 = 0; i0 < nc; i0 += CU) {
        int32_t jj[CU];
        X3 o[CU];
        V3 ov[CU];
        float orc[CU];
        uint32_t oo[CU];
#pragma unroll
        for (int u = 0; u < CU; ++u)
          jj[u] = i0 + u < nc ? s_cand[(i0 + u) * TILE + threadIdx.x] : 0;
#pragma unroll
        for (int u = 0; u < CU; ++u)
          if (i0 + u < nc) {
            const int64_t q = S.p_off + jj[u];
            o[u] = xs[q];
            orc[u] = rcs[2 * q];
            ov[u] = vs[q];
            oo[u] = FRIC ? a.orig[q] : 0u;
          }
#pragma unroll
        for (int u = 0; u < CU; ++u)
          if (i0 + u < nc) contact(o[u], orc[u], ov[u], oo[u]);
      }
    }
    if constexpr (FRIC) {
      if (fric) {
        a.hcnt_dst[k] = hc < a.hcap ? hc : a.hcap;
        if (hc > a.hcap) atomicMax(&a.overflow[2], hc);
      }
    }
    // walls: half-spaces of infinite mass at rest, normals into the box,
    // in the order -x, +x, -y, +y, -z, +z, then the planar and the cylindrical
    // walls
    const double pos[3] = {me.x, me.y, me.z};
    const double vel[3] = {mv.vx, mv.vy, mv.vz};
    double f[3] = {fx, fy, fz};
    // the overlap R_C - t is positive exactly when R_C > t (a difference of
    // doubles rounds to a positive value iff it is positive), so it is formed
    // only for the faces a particle touches
    const double rcd = (double)mrc;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const double tlo = pos[ax] - S.lo[ax];
      if (rcd > tlo) f[ax] += S.kn * (rcd - tlo) - S.gamma_n * vel[ax];
      const double thi = S.hi[ax] - pos[ax];
      if (rcd > thi) f[ax] -= S.kn * (rcd - thi) - S.gamma_n * (-vel[ax]);
    }
    // planar and cylindrical walls (instances for batches that have them: the
    // loops cost the step kernel time even when they run no iteration)
    if constexpr (WALLS) {
      // planar walls, in index order: the same law against the half-space n.x < d,
      // for centres above the wall's height bound
      for (int w = 0; w < S.n_planes; ++w) {
        const double *pl = S.planes[w];
        if (!(pos[2] > pl[4])) continue;
        const double sd = pl[0] * pos[0] + pl[1] * pos[1] + pl[2] * pos[2] - pl[3];
        if (rcd > sd) {  // overlap R_C - sd positive
          const double dw = rcd - sd;
          const double vn = vel[0] * pl[0] + vel[1] * pl[1] + vel[2] * pl[2];
          const double fm = S.kn * dw - S.gamma_n * vn;
          f[0] += fm * pl[0];
          f[1] += fm * pl[1];
          f[2] += fm * pl[2];
        }
      }
      // vertical cylindrical walls, in index order: the same law against the inside
      // of the cylinder, for centres above the wall's height bound; the overlap is
      // R_C less the distance R - rho of the centre from the wall, the normal
      // points to the axis
      for (int w = 0; w < S.n_cyl; ++w) {
        const double *cy = S.cyl[w];
        if (!(pos[2] > cy[3])) continue;
        const double dx = pos[0] - cy[0], dy = pos[1] - cy[1];
        const double rho = sqrt(dx * dx + dy * dy);
        const double tw = cy[2] - rho;
        if (rcd > tw && rho > 0.0) {  // overlap R_C - (R - rho) positive
          const double dw = rcd - tw;
          const double nx = -dx / rho, ny = -dy / rho;
          const double vn = vel[0] * nx + vel[1] * ny;
          const double fm = S.kn * dw - S.gamma_n * vn;
          f[0] += fm * nx;
          f[1] += fm * ny;
        }
      }
    }
    // velocity Verlet: v^n = v^{n-1/2} + dt/2 a^n, v^{n+1/2} = v^n + dt/2 a^n,
    // x^{n+1} = x^n + dt v^{n+1/2}
    const double hdt = 0.5 * S.dt, im = (double)mri.y;
    double vf[3], vn[3], xn[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const double acc = f[ax] * im + S.g[ax];
      vf[ax] = a.first ? vel[ax] : vel[ax] + hdt * acc;
      vn[ax] = vf[ax] + hdt * acc;
      xn[ax] = pos[ax] + S.dt * vn[ax];
    }
    nt_store24(&a.x_dst[k].x, xn[0], xn[1], xn[2]);
    nt_store24(&a.v_dst[k].vx, vn[0], vn[1], vn[2]);
    __builtin_nontemporal_store(posq_encode_c(S, xn[0], xn[1], xn[2], mcode), &a.posq_dst[k]);
    ke = 0.5 * (vf[0] * vf[0] + vf[1] * vf[1] + vf[2] * vf[2]) / im;
    // Eq. update for the next step: straight-line displacement since the last
    // broad phase against the skin left after the cap (R_NL - R_C)
    const float ddx = (float)(xn[0] - (double)b.x);
    const float ddy = (float)(xn[1] - (double)b.y);
    const float ddz = (float)(xn[2] - (double)b.z);
    const float disp = sqrtf(__fmaf_rn(ddx, ddx, __fmaf_rn(ddy, ddy, ddz * ddz)));
    const float skin_eff = b.w - mrc;
    viol = disp > skin_eff ? 1 : 0;
    excess = disp - skin_eff;
  }
  // per-tile statistics, reduced in a fixed order
  __shared__ double s_ke[TILE / WAVE];
  __shared__ int s_i[3][TILE / WAVE];
  __shared__ float s_x[TILE / WAVE];
  ke = wave_sum(ke);
  // row lengths and contacts summed together in the two halves of one word
  // (each is at most 64 x MAX_ROW < 2^16 per wave); violators counted by ballot
  static_assert(WAVE * MAX_ROW < (1 << 16), "a wave's row or contact sum fits 16 bits");
  const int rc_sum = wave_sum(rowlen | (ncon << 16));
  const int n_viol = (int)__popcll(__ballot(viol));
  excess = wave_max(excess);
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  if (lane == 0) {
    s_ke[w] = ke;
    s_i[0][w] = rc_sum & 0xFFFF;
    s_i[1][w] = rc_sum >> 16;
    s_i[2][w] = n_viol;
    s_x[w] = excess;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    TileStats stt;
    stt.ke = 0.0;
    stt.rowsum = stt.contacts2 = stt.violators = 0;
    stt.max_excess = -INFINITY;
#pragma unroll
    for (int i = 0; i < TILE / WAVE; ++i) {
      stt.ke += s_ke[i];
      stt.rowsum += s_i[0][i];
      stt.contacts2 += s_i[1][i];
      stt.violators += s_i[2][i];
      stt.max_excess = fmaxf(stt.max_excess, s_x[i]);
    }
    a.stats[(int64_t)(step % STATS_RING) * a.n_tiles + t] = stt;
    if (stt.violators > 0 && (S.skin_mode == 0 || S.skin_mode == 1))
      atomicOr(&a.flags[((step + 1) & 1) * a.n_sys + s], 1);
  }
}

// ------------------------------------------------------------------ broad phase

// Extended spheres, reference positions and cell bins of every system that needs
// a broad phase at this step; with relist set, the other systems bin their
// stored x0 and R_NL unchanged (their rows are then rebuilt by the pair search
// without a broad phase: after a storage sort, a resumed checkpoint or a retried
// block).  The systems that take part are listed first, in index order, with
// the prefix of their tiles; the grid then walks their tiles only, grid-stride,
// so that a batch in which few systems rebuild pays for those alone.
__global__ __launch_bounds__(TILE) void k_bin(BroadArgs a) {
  constexpr int SYS_PER = MAX_SYS / TILE;  // systems looked at by each thread
  __shared__ int32_t s_act[MAX_SYS];       // 2 s + 1 if system s runs a broad phase, else 2 s
  __shared__ int32_t s_tpre[MAX_SYS + 1];  // tiles of the listed systems before entry i
  const int tid = threadIdx.x;
  const int step = a.step + (a.step_base ? *a.step_base : 0);
  int code[SYS_PER];
  int n_act = 0;
#pragma unroll
  for (int q = 0; q < SYS_PER; ++q) {
    const int s = tid * SYS_PER + q;
    code[q] = -1;
    if (s < a.n_sys) {
      const int nd = needs_broad_phase(a.sys[s], a.flags, a.n_sys, s, step, a.force);
      if (blockIdx.x == 0) {
        a.go[s] = nd | a.relist;
        a.rebuilt_ring[(step % STATS_RING) * a.n_sys + s] = nd;
      }
      if (nd || a.relist) {
        code[q] = 2 * s + nd;
        n_act += 1;
      }
    }
  }
  // a step without broad phase (the common case) ends here, after one barrier
  if (!__syncthreads_or(n_act)) return;
  int n_tl = 0, n_bk = 0;
#pragma unroll
  for (int q = 0; q < SYS_PER; ++q)
    if (code[q] >= 0) {
      const SysDev &S = a.sys[code[q] >> 1];
      n_tl += S.n_tiles;
      n_bk += S.nb[0] * S.nb[1] * S.nb[2];
    }
  int tot_act, tot_tl, tot_bk;  // the same in every workgroup
  int i_act = block_inclusive_scan<TILE>(n_act, &tot_act) - n_act;
  int i_tl = block_inclusive_scan<TILE>(n_tl, &tot_tl) - n_tl;
  int i_bk = block_inclusive_scan<TILE>(n_bk, &tot_bk) - n_bk;
#pragma unroll
  for (int q = 0; q < SYS_PER; ++q)
    if (code[q] >= 0) {
      const int s = code[q] >> 1;
      const SysDev &S = a.sys[s];
      s_act[i_act] = code[q];
      s_tpre[i_act] = i_tl;
      if (blockIdx.x == 0) {
        a.act[1 + i_act] = s;
        a.act[1 + MAX_SYS + i_act] = i_bk;
      }
      ++i_act;
      i_tl += S.n_tiles;
      i_bk += S.nb[0] * S.nb[1] * S.nb[2];
    }
  if (tid == 0) {
    s_tpre[tot_act] = tot_tl;
    if (blockIdx.x == 0) {
      a.act[0] = tot_act;
      a.act[1 + MAX_SYS + tot_act] = tot_bk;
    }
  }
  __syncthreads();
  int e = 0;  // entry of the listed system that holds tile u
  for (int64_t u = blockIdx.x; u < tot_tl; u += gridDim.x) {
    while (s_tpre[e + 1] <= u) ++e;
    const int s = s_act[e] >> 1, nd = s_act[e] & 1;
    const SysDev &S = a.sys[s];
    const int local = (int)(u - s_tpre[e]) * TILE + tid;
    int64_t key = -1;
    float4 b = make_float4(0.f, 0.f, 0.f, 0.f);
    uint32_t orig = 0;
    if (local < S.n) {
      const int64_t k = S.p_off + local;
      const X3 x = a.x[k];
      if (nd) {
        const V3 v = a.v[k];
        double skin;
        if (S.skin_mode == 0) skin = S.K * sqrt(v.vx * v.vx + v.vy * v.vy + v.vz * v.vz) * S.dt;
        else if (S.skin_mode == 2) skin = 0.0;
        else skin = S.skin_uniform;
        const double r = (double)a.ri[k].x + skin;
        const double rnl = r < S.cap ? r : S.cap;
        b = make_float4((float)x.x, (float)x.y, (float)x.z, (float)rnl);
        a.bp[k] = b;
        key = S.c_off + cell_of(S, x.x, x.y, x.z);
      } else {
        // the list of the last broad phase is the set of pairs within reach of
        // the stored spheres; any binning that keeps pairs within reach in
        // neighbouring cells finds it, so binning x0 reproduces it exactly
        b = a.bp[k];
        key = S.c_off + cell_of(S, (double)b.x, (double)b.y, (double)b.z);
      }
      orig = a.orig[k];
      // slots move only when the state is set, the storage sorted or a snapshot
      // restored, and each of these forces a broad phase or a relist of every
      // system: the inverse permutation is rewritten then, not at every broad
      // phase (a scattered 4-byte write per particle)
      if (a.force || a.relist) a.inv[S.p_off + orig] = local;
    }
    const int slot = wave_bin_slot(a.bin_count, key);
    if (key >= 0) {
      if (slot < a.bin_cap) {
        a.bins_bp[key * a.bin_cap + slot] = b;
        a.bins_og[key * a.bin_cap + slot] = (int32_t)orig;
      } else {
        atomicMax(&a.overflow[1], slot + 1);
      }
    }
  }
}

// Inserts key into the sorted row of this thread (column threadIdx.x of a
// [W][ld] LDS array, threadIdx.x < ld) if the row has room; returns the new
// count (which may exceed W: overflow).  Entries are original indices.
__device__ __forceinline__ int row_insert(int32_t *s_row, int ld, int count, int W, int32_t key) {
  if (count < W) {
    int j = count;
    while (j > 0 && s_row[(j - 1) * ld + threadIdx.x] > key) {
      s_row[j * ld + threadIdx.x] = s_row[(j - 1) * ld + threadIdx.x];
      --j;
    }
    s_row[j * ld + threadIdx.x] = key;
  }
  return count + 1;
}

// Bitonic sort of N keys held in registers (all indices are compile-time
// constants after unrolling), ascending.
template <int N>
__device__ __forceinline__ void bitonic_sort(int32_t (&key)[N]) {
#pragma unroll
  for (int kk = 2; kk <= N; kk <<= 1)
#pragma unroll
    for (int j = kk >> 1; j > 0; j >>= 1)
#pragma unroll
      for (int i = 0; i < N; ++i) {
        const int l = i ^ j;
        if (l > i) {
          const int32_t lo = min(key[i], key[l]), hi = max(key[i], key[l]);
          const bool up = (i & kk) == 0;
          key[i] = up ? lo : hi;
          key[l] = up ? hi : lo;
        }
      }
}

// Writes this thread's row of n <= N staged-entry indices (column threadIdx.x
// of a [.][NT] LDS array) to the Verlet list as slots, ordered by original
// index: the original indices are sorted in registers, then turned into slots
// through inv (inv[orig] = slot of the system's particle orig).
template <int N, int NT>
__device__ __forceinline__ void row_write_sorted(const uint16_t *s_row, const int32_t *s_key,
                                                 const int32_t *__restrict__ inv, int n,
                                                 int32_t *nbr, int64_t stride, int64_t k) {
  static_assert(N % ROW_GROUP == 0, "whole groups");
  int32_t key[N];
#pragma unroll
  for (int q = 0; q < N; ++q) key[q] = q < n ? s_key[s_row[q * NT + threadIdx.x]] : INT32_MAX;
  bitonic_sort<N>(key);
#pragma unroll
  for (int q = 0; q < N; ++q) key[q] = q < n ? inv[key[q]] : 0;
  // whole groups: a group that holds an entry below n lies below the row width
  // (n <= W and W is a multiple of ROW_GROUP)
#pragma unroll
  for (int g = 0; g < N / ROW_GROUP; ++g)
    if (g * ROW_GROUP < n)
      *reinterpret_cast<int4 *>(&nbr[row_index(stride, k, g * ROW_GROUP)]) =
          make_int4(key[4 * g], key[4 * g + 1], key[4 * g + 2], key[4 * g + 3]);
}

// The same for a row of any length up to W: insertion sort in LDS.
template <int NT>
__device__ __forceinline__ void row_write_sorted_lds(uint16_t *s_row, const int32_t *s_key,
                                                     const int32_t *__restrict__ inv, int n,
                                                     int32_t *nbr, int64_t stride, int64_t k) {
  for (int i = 1; i < n; ++i) {
    const int e = s_row[i * NT + threadIdx.x];
    const int32_t key = s_key[e];
    int j = i;
    while (j > 0) {
      const int prev = s_row[(j - 1) * NT + threadIdx.x];
      if (s_key[prev] <= key) break;
      s_row[j * NT + threadIdx.x] = (uint16_t)prev;
      --j;
    }
    s_row[j * NT + threadIdx.x] = (uint16_t)e;
  }
  for (int q = 0; q < n; ++q) nbr[row_index(stride, k, q)] = inv[s_key[s_row[q * NT + threadIdx.x]]];
}

// The FP32 inclusion test of Alg. 1 on the extended spheres, |x_i - x_j| <=
// R_NL,i + R_NL,j + eps, on squares: me = (x0_i, R_NL,i), reach = R_NL,i + eps,
// o = (x0_j, R_NL,j).  One rounding sequence (explicit fused multiply-adds) for
// both the LDS-staged and the direct search, so that they find the same pairs.
__device__ __forceinline__ bool within_reach(const float4 &me, const float4 &o, float reach) {
  const float ex = me.x - o.x, ey = me.y - o.y, ez = me.z - o.z;
  const float lim = reach + o.w;
  return __fmaf_rn(ex, ex, __fmaf_rn(ey, ey, ez * ez)) <= lim * lim;
}

// Four staged entries e..e+3 against the particle `me` (position and R_NL +
// eps): each entry index is written at the row's end, and the row grows by NT
// for each entry within reach.  wofs keeps the exact length (times NT); the
// write position is capped once per group, at the first spare row wend (rows
// W to W+3 are spare: a group adds at most three hits before its last write).
// ix01 and ix23 hold the four entry indices as 16-bit pairs.  TAIL masks
// entries at or past e1; OWN masks the particle's own entry.
template <bool TAIL, bool OWN, int NT>
__device__ __forceinline__ void pair_test4(const float4 *s_pos, int e, int e1, int me_e,
                                           const float4 &me, float reach, uint16_t *myrow,
                                           unsigned wend, unsigned &wofs, uint32_t ix01,
                                           uint32_t ix23) {
  const float4 o[4] = {s_pos[e], s_pos[e + 1], s_pos[e + 2], s_pos[e + 3]};
  const uint16_t ix[4] = {(uint16_t)ix01, (uint16_t)(ix01 >> 16), (uint16_t)ix23,
                          (uint16_t)(ix23 >> 16)};
  uint16_t *const p0 = myrow + min(wofs, wend);
  uint16_t *p = p0;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    bool hit = within_reach(me, o[u], reach);
    if (TAIL) hit = hit && e + u < e1;
    if (OWN) hit = hit && e + u != me_e;
    *p = ix[u];
    p += hit ? NT : 0;
  }
  wofs += (unsigned)(p - p0);
}

// The staged range [e, e1): groups of four, the last one masked.
template <bool OWN, int NT>
__device__ __forceinline__ void pair_scan_range(const float4 *s_pos, int e, int e1, int me_e,
                                                const float4 &me, float reach, uint16_t *myrow,
                                                unsigned wend, unsigned &wofs) {
  // entry indices are below 2^16 (at most 4096 are staged): no carry between
  // the halves of a pair
  uint32_t ix01 = (uint32_t)e | ((uint32_t)(e + 1) << 16);
  uint32_t ix23 = (uint32_t)(e + 2) | ((uint32_t)(e + 3) << 16);
  for (; e + 4 <= e1; e += 4, ix01 += 0x40004u, ix23 += 0x40004u)
    pair_test4<false, OWN, NT>(s_pos, e, e1, me_e, me, reach, myrow, wend, wofs, ix01, ix23);
  if (e < e1) pair_test4<true, OWN, NT>(s_pos, e, e1, me_e, me, reach, myrow, wend, wofs, ix01, ix23);
}

// Sub-bin of a coordinate along a line of box cells, floor((x - xl) * qinv)
// clamped to [-1, nq] (NaN gives -1).  Every operation is non-decreasing in x,
// so the sub-bin is too: the candidate windows of the pair search rest on it.
__device__ __forceinline__ int xsub(float x, float xl, float qinv, int nq) {
  const float f = floorf((x - xl) * qinv);
  return (int)fminf(fmaxf(f, -1.f), (float)nq);
}

// Stages one cell of n <= NM entries (positions pb[0..n), original indices
// po[0..n)) at LDS entries off.. in x sub-bin order, and writes the
// starts of the cell's sub-bins [qlo, qlo + XRES) into tab.  The whole cell is
// loaded into registers at once (entries at or past n are read, not used: the
// bins are padded by BIN_PAD), then placed by a counting sort over the
// sub-bins, ties in bin order: byte q of `below` counts the entries below
// sub-bin qlo + q, byte q of `seen` those of sub-bin qlo + q placed so far.
// Within a cell, x order implies sub-bin order, since xsub is non-decreasing in
// x.  A sub-bin outside the cell's (a position outside the grid, rounded
// across a face, or NaN) sets nowin; rmax takes the largest R_NL as float bits.
template <int NM>
__device__ __forceinline__ void stage_cell(const float4 *pb, const int32_t *po, int n, int off,
                                           int qlo, float xl, float qinv, int nq, float4 *s_pos,
                                           int32_t *s_key, uint16_t *tab, int &nowin, int &rmax) {
  static_assert(NM <= BIN_PAD && NM < 256, "loads stay inside the padded bins; byte counters");
  float4 bp[NM];
  int32_t og[NM];
#pragma unroll
  for (int u = 0; u < NM; ++u) {
    bp[u] = pb[u];
    og[u] = po[u];
  }
  // every load above is issued before any of them is used (one round trip,
  // not one for the positions and one for the indices)
  __builtin_amdgcn_sched_barrier(0);
  int rb[NM];
  uint64_t below = 0, seen = 0;
#pragma unroll
  for (int u = 0; u < NM; ++u) {
    // entries past n count in the last sub-bin, which adds to no byte
    const bool in = u < n;
    const int bq = xsub(bp[u].x, xl, qinv, nq) - qlo;
    nowin |= (in && (unsigned)bq >= (unsigned)XRES) ? 1 : 0;
    rb[u] = in ? 8 * min(max(bq, 0), XRES - 1) : 8 * (XRES - 1);
    below += 0x0101010101010100ull << rb[u];
    rmax = max(rmax, in ? __float_as_int(bp[u].w) : 0);
  }
#pragma unroll
  for (int u = 0; u < NM; ++u)
    if (u < n) {
      const int e = off + (int)(((below >> rb[u]) & 255u) + ((seen >> rb[u]) & 255u));
      seen += 1ull << rb[u];
      s_pos[e] = bp[u];
      s_key[e] = og[u];
    }
#pragma unroll
  for (int qq = 0; qq < XRES; ++qq) tab[qlo + qq] = (uint16_t)(off + (int)((below >> (8 * qq)) & 255u));
}

// The same for a cell of 8 < n <= 64 entries, in chunks of eight: a first pass
// counts the sub-bins, a second places the entries (its loads mostly hit the
// cache).  Bins are padded by BIN_PAD >= 8, so a chunk's reads past n stay
// inside the allocation.
__device__ __forceinline__ void stage_cell_chunks(const float4 *pb, const int32_t *po, int n, int off,
                                                  int qlo, float xl, float qinv, int nq,
                                                  float4 *s_pos, int32_t *s_key, uint16_t *tab,
                                                  int &nowin, int &rmax) {
  static_assert(BIN_PAD >= 8, "a chunk reads up to seven entries past the cell");
  uint64_t below = 0, seen = 0;
  for (int i0 = 0; i0 < n; i0 += 8) {
    float xw[8][2];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      xw[u][0] = pb[i0 + u].x;
      xw[u][1] = pb[i0 + u].w;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const bool in = i0 + u < n;
      const int bq = xsub(xw[u][0], xl, qinv, nq) - qlo;
      nowin |= (in && (unsigned)bq >= (unsigned)XRES) ? 1 : 0;
      below += in ? (0x0101010101010100ull << (8 * min(max(bq, 0), XRES - 1))) : 0ull;
      rmax = max(rmax, in ? __float_as_int(xw[u][1]) : 0);
    }
  }
  for (int i0 = 0; i0 < n; i0 += 8) {
    float4 bp[8];
    int32_t og[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      bp[u] = pb[i0 + u];
      og[u] = po[i0 + u];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (i0 + u < n) {
        const int rb = 8 * min(max(xsub(bp[u].x, xl, qinv, nq) - qlo, 0), XRES - 1);
        const int e = off + (int)(((below >> rb) & 255u) + ((seen >> rb) & 255u));
        seen += 1ull << rb;
        s_pos[e] = bp[u];
        s_key[e] = og[u];
      }
  }
#pragma unroll
  for (int qq = 0; qq < XRES; ++qq) tab[qlo + qq] = (uint16_t)(off + (int)((below >> (8 * qq)) & 255u));
}

// Alg. 1 on the extended spheres, one workgroup per brick of cells: the bins of
// the brick and of the cells within `ring` cells around it are staged in LDS,
// then every particle of the brick is tested against the particles of the cells
// within `ring` cells of its own (|x_i - x_j| <= R_NL,i + R_NL,j, plus eps for
// FP32 rounding, tested on squares).  Matches are appended to the row in LDS;
// the row is then sorted by original index and stored as slots.  A
// neighbourhood too full for LDS is read from the bins directly, by half the
// workgroup.
// Staged cells are ordered by x sub-bin (XRES per cell edge), so each line of box
// cells along x is too, and a table gives where each sub-bin starts.  A
// particle tests, in each (dz, dy) row, only the sub-bins within
// R_NL,i + eps + max R_NL (plus a rounding margin) of its x: a window that holds
// every entry the test can pass, so the rows are the same as over the whole
// range, for about half the tests.
template <int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_pairs(BroadArgs a) {
  extern __shared__ __align__(16) unsigned char lds[];
  constexpr int HALF = NT / 2;
  const int W = a.width;
  float4 *s_pos = reinterpret_cast<float4 *>(lds);                          // [pmax + 4]
  int32_t *s_key = reinterpret_cast<int32_t *>(s_pos + a.pmax + 4);         // [pmax]
  unsigned char *rows = reinterpret_cast<unsigned char *>(s_key + a.pmax);
  uint16_t *s_row16 = reinterpret_cast<uint16_t *>(rows);                   // [W + 4][NT]
  int32_t *s_row32 = reinterpret_cast<int32_t *>(rows);                     // [W][HALF]
  __shared__ int s_cnt[8 * 8 * 8];
  __shared__ int s_off[8 * 8 * 8 + 1];
  __shared__ int s_home[BRICK * BRICK * BRICK + 1];
  __shared__ uint16_t s_xstart[8 * 8 * (8 * XRES + 1)];  // [line][sub-bin]: first staged entry
  __shared__ int s_rmax, s_nowin;  // largest staged R_NL (float bits); windows off
  static_assert(BRICK * BRICK * BRICK == WAVE, "one lane per cell of a brick");
  static_assert(2 * NT >= 8 * 8 * 8, "two box cells per thread in the prefix");
  static_assert(XRES == 8, "a cell's sub-bin counts are the eight bytes of one word");
  const int tid = threadIdx.x;
  int any = 0;
  for (int s = tid; s < a.n_sys; s += NT) any |= a.go[s];
  if (!__syncthreads_or(any)) return;
  // the bricks of the systems that take part, as the binning listed them
  const int n_act = a.act[0];
  const int32_t *act_sys = a.act + 1, *act_bpre = a.act + 1 + MAX_SYS;
  const int64_t n_bk = act_bpre[n_act];
  int e = 0;  // entry of the listed system that holds brick u
  for (int64_t u = blockIdx.x; u < n_bk; u += gridDim.x) {
    while (act_bpre[e + 1] <= u) ++e;
    const int s = act_sys[e];
    const SysDev &S = a.sys[s];
    const int r = S.ring, E = BRICK + 2 * r, V = E * E * E;
    const int lb = (int)(u - act_bpre[e]);
    const int bx = lb % S.nb[0], by = (lb / S.nb[0]) % S.nb[1], bz = lb / (S.nb[0] * S.nb[1]);
    const int ox = bx * BRICK - r, oy = by * BRICK - r, oz = bz * BRICK - r;
    // occupancy of every cell of the neighbourhood box (0 outside the grid)
    if (tid == 0) s_rmax = 0, s_nowin = a.xwindows ? 0 : 1;
    for (int v = tid; v < V; v += NT) {
      const int cx = ox + v % E, cy = oy + (v / E) % E, cz = oz + v / (E * E);
      int n = 0;
      if (cx >= 0 && cy >= 0 && cz >= 0 && cx < S.nc[0] && cy < S.nc[1] && cz < S.nc[2])
        n = min(a.bin_count[S.c_off + cell_key(S, cx, cy, cz)], a.bin_cap);
      s_cnt[v] = n;
    }
    __syncthreads();
    {  // exclusive prefix over the box cells, two per thread
      const int v0 = 2 * tid;
      const int c0 = v0 < V ? s_cnt[v0] : 0, c1 = v0 + 1 < V ? s_cnt[v0 + 1] : 0;
      int tot;
      const int incl = block_inclusive_scan<NT>(c0 + c1, &tot);
      if (v0 < V) s_off[v0] = incl - c0 - c1;
      if (v0 + 1 < V) s_off[v0 + 1] = incl - c1;
      if (tid == 0) s_off[V] = tot;
    }
    if (tid < WAVE) {  // particles of the brick itself: prefix over its cells, one lane each
      const int j = tid;
      const int v = ((r + j / (BRICK * BRICK)) * E + (r + (j / BRICK) % BRICK)) * E + r + j % BRICK;
      const int c = s_cnt[v];
      int incl = c;
#pragma unroll
      for (int o = 1; o < WAVE; o <<= 1) {
        const int u = __shfl_up(incl, o, WAVE);
        if (j >= o) incl += u;
      }
      s_home[j] = incl - c;
      if (j == WAVE - 1) s_home[WAVE] = incl;
    }
    __syncthreads();
    const bool staged = s_off[V] <= a.pmax;
    // x frame of the sub-bins: box cell t of a line holds sub-bins [t, t + 1) * XRES
    const int NQ = E * XRES;
    const float xl = (float)(S.lo[0] + (double)ox / S.inv_edge[0]);
    const float qinv = (float)(S.inv_edge[0] * XRES);
    if (staged) {
      // largest R_NL as float bits: every positive float orders as its bits,
      // and a NaN or infinite radius orders above every finite one
      int nowin = 0, rmax = 0;
      for (int v = tid; v < V; v += NT) {
        const int n = s_cnt[v], off = s_off[v], t = v % E, qlo = t * XRES;
        uint16_t *tab = s_xstart + (v / E) * (NQ + 1);
        if (t == E - 1) tab[NQ] = (uint16_t)(off + n);
        if (n == 0 || n > 64) {  // the starts of a cell without windows: its first entry
#pragma unroll
          for (int qq = 0; qq < XRES; ++qq) tab[qlo + qq] = (uint16_t)off;
          if (n == 0) continue;
        }
        const int cx = ox + t, cy = oy + (v / E) % E, cz = oz + v / (E * E);
        const int64_t base = (S.c_off + cell_key(S, cx, cy, cz)) * a.bin_cap;
        const float4 *pb = a.bins_bp + base;
        const int32_t *po = a.bins_og + base;
        if (n <= 8) {
          stage_cell<8>(pb, po, n, off, qlo, xl, qinv, NQ, s_pos, s_key, tab, nowin, rmax);
        } else if (n <= 64) {
          stage_cell_chunks(pb, po, n, off, qlo, xl, qinv, NQ, s_pos, s_key, tab, nowin, rmax);
        } else {
          // more than 64 in the cell: staged in bin order, and the brick tests
          // whole rows
          nowin = 1;
          for (int i0 = 0; i0 < n; i0 += 8) {  // eight loads in flight per thread
            float4 bp[8];
            int32_t og[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {  // entries past n re-read entry n - 1
              const int64_t q = base + min(i0 + u, n - 1);
              bp[u] = a.bins_bp[q];
              og[u] = a.bins_og[q];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u)
              if (i0 + u < n) {
                s_pos[off + i0 + u] = bp[u];
                s_key[off + i0 + u] = og[u];
              }
          }
        }
      }
      if (rmax > 0) atomicMax(&s_rmax, rmax);
      if (nowin) s_nowin = 1;
      __syncthreads();
    }
    const int H = s_home[WAVE];
    const int step_h = staged ? NT : HALF;
    if (staged || tid < HALF)
      for (int h = tid; h < H; h += step_h) {
        int lo = 0, hi = WAVE;  // home cell j: s_home[j] <= h < s_home[j+1]
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (s_home[mid] <= h) lo = mid;
          else hi = mid;
        }
        const int j = lo, i = h - s_home[j];
        const int ix = r + j % BRICK, iy = r + (j / BRICK) % BRICK, iz = r + j / (BRICK * BRICK);
        const int v = (iz * E + iy) * E + ix;
        int count = 0;
        int64_t k;
        if (staged) {
          const int me_e = s_off[v] + i;  // this particle's staged entry
          const float4 me = s_pos[me_e];
          const float reach = me.w + S.eps;
          k = S.p_off + a.inv[S.p_off + s_key[me_e]];  // the slot, from the original index
          // the sub-bins [q0, q1e) that can hold a partner: a pair that passes
          // the test below lies within (R_NL,i + eps + R_NL,j)(1 + 2^-22) in x,
          // and the margins also cover the rounding of x -+ bw
          int q0 = 0, q1e = NQ;
          const float rmx = __int_as_float(s_rmax);
          if (s_nowin == 0 && rmx <= __FLT_MAX__) {
            const float bw = (reach + rmx) * (1.f + 0x1p-19f) + fabsf(me.x) * 0x1p-21f;
            q0 = max(xsub(me.x - bw, xl, qinv, NQ), 0);
            q1e = min(xsub(me.x + bw, xl, qinv, NQ) + 1, NQ);
          }
          // box cells are numbered x fastest, so the 2r+1 cells of one (dz, dy)
          // row of the neighbourhood are one contiguous range of staged entries.
          // The test has no branch: every entry is written at the row's end,
          // and the row grows only by the entries that pass (rows W to W+3
          // are spare rows for overflow).  Ranges are read four entries at a time; the
          // last group of a range is masked (reads past its end stay inside
          // the staged array, which has four spare entries), and only the
          // particle's own row of cells can hold the particle itself.
          uint16_t *myrow = s_row16 + tid;
          const unsigned wend = (unsigned)W * NT;
          unsigned wofs = 0;  // count * NT
          for (int dz = -r; dz <= r; ++dz)
            for (int dy = -r; dy <= r; ++dy) {
              const int vrow = v + (dz * E + dy) * E;
              const uint16_t *tab = s_xstart + ((iz + dz) * E + iy + dy) * (NQ + 1);
              const int e0 = max(s_off[vrow - r], (int)tab[q0]);
              const int e1 = min(s_off[vrow + r + 1], (int)tab[q1e]);
              if (dz == 0 && dy == 0)
                pair_scan_range<true, NT>(s_pos, e0, e1, me_e, me, reach, myrow, wend, wofs);
              else
                pair_scan_range<false, NT>(s_pos, e0, e1, me_e, me, reach, myrow, wend, wofs);
            }
          count = (int)(wofs / NT);
          const int kept = count < W ? count : W;
          // one sort for the whole wave, sized by its longest row (no divergence)
          const int32_t *inv = a.inv + S.p_off;
          if (!__any(kept > 8))
            row_write_sorted<8, NT>(s_row16, s_key, inv, kept, a.nbr, a.stride, k);
          else if (!__any(kept > 16))
            row_write_sorted<16, NT>(s_row16, s_key, inv, kept, a.nbr, a.stride, k);
          else if (!__any(kept > 32))
            row_write_sorted<32, NT>(s_row16, s_key, inv, kept, a.nbr, a.stride, k);
          else
            row_write_sorted_lds<NT>(s_row16, s_key, inv, kept, a.nbr, a.stride, k);
        } else {
          const int64_t mybase = (S.c_off + cell_key(S, ox + ix, oy + iy, oz + iz)) * a.bin_cap;
          const float4 me = a.bins_bp[mybase + i];
          const float reach = me.w + S.eps;
          k = S.p_off + a.inv[S.p_off + a.bins_og[mybase + i]];
          for (int dz = -r; dz <= r; ++dz)
            for (int dy = -r; dy <= r; ++dy)
              for (int dx = -r; dx <= r; ++dx) {
                const int v2 = v + (dz * E + dy) * E + dx;
                const int n2 = s_cnt[v2];
                if (n2 == 0) continue;
                const int64_t base =
                    (S.c_off + cell_key(S, ox + ix + dx, oy + iy + dy, oz + iz + dz)) * a.bin_cap;
                for (int e = 0; e < n2; ++e) {
                  if (v2 == v && e == i) continue;
                  if (within_reach(me, a.bins_bp[base + e], reach))
                    count = row_insert(s_row32, HALF, count, W, a.bins_og[base + e]);
                }
              }
          const int kept = count < W ? count : W;
          for (int q = 0; q < kept; ++q)
            a.nbr[row_index(a.stride, k, q)] = a.inv[S.p_off + s_row32[q * HALF + tid]];
        }
        a.cnt[k] = count < W ? count : W;
        if (count > W) atomicMax(&a.overflow[0], count);
      }
    __syncthreads();  // the next brick reuses the LDS
  }
}

// ------------------------------------------------------------------ spatial sort

// Counting sort of every system's slots by cell, then by original index inside a
// cell (deterministic).  Scheduled by the host; every row is then rebuilt from
// the stored x0 and R_NL (no new broad phase: the schedule is kept).
__global__ __launch_bounds__(TILE) void k_sort_count(SortArgs a) {
  const int64_t t = blockIdx.x;
  const SysDev &S = a.sys[a.tile_sys[t]];
  const int local = (int)(t - S.tile_off) * TILE + (int)threadIdx.x;
  if (local >= S.n) return;
  const int64_t k = S.p_off + local;
  const X3 p = a.x_src[k];
  const int c = cell_of(S, p.x, p.y, p.z);
  a.cellid[k] = c;
  a.inslot[k] = atomicAdd(&a.cell_count[S.c_off + c], 1);
}

// Exclusive scan, stage 1: each workgroup scans TILE * SCAN_ITEMS cells.
__global__ __launch_bounds__(TILE) void k_scan_blocks(const int32_t *in, int64_t n, int32_t *out,
                                                      int32_t *block_sum) {
  const int64_t base = (int64_t)blockIdx.x * TILE * SCAN_ITEMS + (int64_t)threadIdx.x * SCAN_ITEMS;
  int v[SCAN_ITEMS];
  int sum = 0;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    v[i] = base + i < n ? in[base + i] : 0;
    sum += v[i];
  }
  int tot;
  const int incl = block_inclusive_scan(sum, &tot);
  int run = incl - sum;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    if (base + i < n) out[base + i] = run;
    run += v[i];
  }
  if (threadIdx.x == 0) block_sum[blockIdx.x] = tot;
}

// Stage 2: exclusive scan of the block sums in one workgroup; block_sum[nb] = total.
__global__ __launch_bounds__(TILE) void k_scan_top(int32_t *block_sum, int64_t nb) {
  __shared__ int carry_s;
  if (threadIdx.x == 0) carry_s = 0;
  __syncthreads();
  for (int64_t b0 = 0; b0 < nb; b0 += TILE) {
    const int64_t i = b0 + threadIdx.x;
    const int v = i < nb ? block_sum[i] : 0;
    int tot;
    const int incl = block_inclusive_scan(v, &tot);
    const int carry = carry_s;
    if (i < nb) block_sum[i] = carry + incl - v;
    __syncthreads();
    if (threadIdx.x == 0) carry_s = carry + tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) block_sum[nb] = carry_s;
}

// Stage 3: add the block offsets; out[n] = total.
__global__ __launch_bounds__(TILE) void k_scan_add(int32_t *out, int64_t n, const int32_t *block_sum,
                                                   int64_t nb) {
  const int64_t base = (int64_t)blockIdx.x * TILE * SCAN_ITEMS + (int64_t)threadIdx.x * SCAN_ITEMS;
  const int add = block_sum[blockIdx.x];
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i)
    if (base + i < n) out[base + i] += add;
  if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = block_sum[nb];
}

// Scatter every slot to a provisional place inside its cell; empty the counts.
__global__ __launch_bounds__(TILE) void k_sort_scatter(SortArgs a) {
  const int64_t t = blockIdx.x;
  const int64_t chunk = (a.n_cells + a.n_tiles - 1) / a.n_tiles;
  const int64_t c1 = min(a.n_cells, (t + 1) * chunk);
  for (int64_t c = t * chunk + threadIdx.x; c < c1; c += TILE) a.cell_count[c] = 0;
  const SysDev &S = a.sys[a.tile_sys[t]];
  const int local = (int)(t - S.tile_off) * TILE + (int)threadIdx.x;
  if (local >= S.n) return;
  const int64_t k = S.p_off + local;
  const int32_t base = a.cell_start[S.c_off];
  a.perm0[S.p_off + (a.cell_start[S.c_off + a.cellid[k]] - base) + a.inslot[k]] = local;
}

// Final place = cell start + rank of the original index among the cell's
// particles; move the state there.
__global__ __launch_bounds__(TILE) void k_sort_place(SortArgs a) {
  const int64_t t = blockIdx.x;
  const SysDev &S = a.sys[a.tile_sys[t]];
  const int local = (int)(t - S.tile_off) * TILE + (int)threadIdx.x;
  if (local >= S.n) return;
  const int64_t p = S.p_off + local;
  const int32_t q = a.perm0[p];
  const int c = a.cellid[S.p_off + q];
  const int32_t base = a.cell_start[S.c_off];
  const int64_t cs = S.p_off + (a.cell_start[S.c_off + c] - base);
  const int64_t ce = S.p_off + (a.cell_start[S.c_off + c + 1] - base);
  const uint32_t me = a.orig_src[S.p_off + q];
  int rank = 0;
  for (int64_t m = cs; m < ce; ++m) rank += a.orig_src[S.p_off + a.perm0[m]] < me;
  a.x_dst[cs + rank] = a.x_src[S.p_off + q];
  a.v_dst[cs + rank] = a.v_src[S.p_off + q];
  a.ri_dst[cs + rank] = a.ri_src[S.p_off + q];
  a.orig_dst[cs + rank] = me;
  a.bp_dst[cs + rank] = a.bp_src[S.p_off + q];
  if (a.hist_src) {  // the friction history moves with its particle
    const int hn = a.hcnt_src[S.p_off + q];
    a.hcnt_dst[cs + rank] = hn;
    for (int c = 0; c < hn; ++c)
      a.hist_dst[(int64_t)c * a.stride + cs + rank] = a.hist_src[(int64_t)c * a.stride + S.p_off + q];
  }
}

// ------------------------------------------------------------------ statistics

// One workgroup per (system, step): sums the system's tile statistics of that
// step in a fixed order.
__global__ __launch_bounds__(TILE) void k_stats_reduce(const SysDev *sys, const TileStats *stats,
                                                       const int32_t *rebuilt_ring, int64_t n_tiles,
                                                       int32_t n_sys, int32_t step0,
                                                       RecordDev *out) {
  const int s = blockIdx.x;
  const int r = blockIdx.y;
  const int step = step0 + r;
  const SysDev &S = sys[s];
  const TileStats *st = stats + (int64_t)(step % STATS_RING) * n_tiles + S.tile_off;
  double ke = 0.0;
  int64_t rows = 0, con = 0, vio = 0;
  float mx = -INFINITY;
  for (int i = threadIdx.x; i < S.n_tiles; i += TILE) {
    const TileStats q = st[i];
    ke += q.ke;
    rows += q.rowsum;
    con += q.contacts2;
    vio += q.violators;
    mx = fmaxf(mx, q.max_excess);
  }
  __shared__ double s_ke[TILE / WAVE];
  __shared__ float s_mx[TILE / WAVE];
  const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
  ke = wave_sum(ke);
  mx = wave_max(mx);
  if (lane == 0) {
    s_ke[w] = ke;
    s_mx[w] = mx;
  }
  rows = block_sum_i64(rows);
  con = block_sum_i64(con);
  vio = block_sum_i64(vio);
  if (threadIdx.x == 0) {
    double k2 = 0.0;
    float m2 = -INFINITY;
    for (int i = 0; i < TILE / WAVE; ++i) {
      k2 += s_ke[i];
      m2 = fmaxf(m2, s_mx[i]);
    }
    RecordDev rec;
    rec.step = step;
    rec.rebuilt = rebuilt_ring[(step % STATS_RING) * n_sys + s];
    rec.list_pairs = rows / 2;
    rec.contacts = con / 2;
    rec.violators = vio;
    rec.max_excess = S.n > 0 ? m2 : 0.0f;
    rec.reserved = 0;
    rec.kinetic_energy = k2;
    out[(int64_t)r * n_sys + s] = rec;
  }
}

// ------------------------------------------------------------------ state I/O

// Coded positions of every slot, for the step kernel's pre-test.
__global__ void k_posq(const SysDev *sys, const int32_t *tile_sys, const int32_t *rrange, int n_sys,
                       const X3 *xs, const float2 *ri, uint64_t *posq, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int s = tile_sys[i / TILE];
  const X3 p = xs[i];
  posq[i] = posq_encode(sys[s], __int_as_float(rrange[s]), __int_as_float(rrange[n_sys + s]), p.x,
                        p.y, p.z, ri[i].x);
}

// Load one system from the caller's original order; flags bad values in *err:
// bit 0 non-finite, bit 1 radius out of range, bit 2 non-positive inverse mass.
// The smallest and largest valid R_C go to *r_lo and *r_hi (FP32 bits; positive
// floats order like their bits).
__global__ void k_set_state(SysDev S, X3 *xs, V3 *vs, float2 *ri, uint32_t *origs, const double *x,
                            const double *v, const float *rc, const float *invm, int32_t *err,
                            int32_t *r_lo, int32_t *r_hi) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t padded = (int64_t)S.n_tiles * TILE;
  if (i >= padded) return;  // padded is a multiple of the block size: whole waves
  X3 p = {0.0, 0.0, 0.0};
  V3 q = {0.0, 0.0, 0.0};
  float2 r = make_float2(0.0f, 0.0f);
  uint32_t o = 0xFFFFFFFFu;
  float rmin = INFINITY, rmax = 0.0f;
  if (i < S.n) {
    const int64_t g = S.o_off + i;
    p.x = x[3 * g];
    p.y = x[3 * g + 1];
    p.z = x[3 * g + 2];
    q.vx = v[3 * g];
    q.vy = v[3 * g + 1];
    q.vz = v[3 * g + 2];
    r = make_float2(rc[g], invm[g]);
    o = (uint32_t)i;
    int e = 0;
    if (!isfinite(p.x) || !isfinite(p.y) || !isfinite(p.z) || !isfinite(q.vx) ||
        !isfinite(q.vy) || !isfinite(q.vz) || !isfinite(r.x) || !isfinite(r.y))
      e |= 1;
    else {
      if (!(r.x > 0.0f) || (double)r.x > S.cap) e |= 2;
      if (!(r.y > 0.0f)) e |= 4;
    }
    if (e) atomicOr(err, e);
    else rmin = rmax = r.x;
  }
  xs[S.p_off + i] = p;
  vs[S.p_off + i] = q;
  ri[S.p_off + i] = r;
  origs[S.p_off + i] = o;
  rmin = -wave_max(-rmin);
  rmax = wave_max(rmax);
  if ((threadIdx.x & (WAVE - 1)) == 0 && rmax > 0.0f) {
    atomicMin(r_lo, __float_as_int(rmin));
    atomicMax(r_hi, __float_as_int(rmax));
  }
}

// Friction history to the caller's original order: particle g's contacts of
// the last step (partner ascending) in partner[g][0..cap), -1 after the last,
// with their springs; *needed receives the largest count of any particle.
__global__ void k_get_history(const SysDev *sys, const int32_t *tile_sys, const uint32_t *origs,
                              const HistEntry *hist, const int32_t *hcnt, int64_t stride,
                              int32_t hcap, int32_t *partner, double *spring, int32_t cap,
                              int32_t *needed) {
  const int64_t t = blockIdx.x;
  const SysDev &S = sys[tile_sys[t]];
  const int local = (int)(t - S.tile_off) * TILE + (int)threadIdx.x;
  if (local >= S.n) return;
  const int64_t k = S.p_off + local;
  const int64_t g = S.o_off + origs[k];
  const int n = S.friction ? min(hcnt[k], hcap) : 0;
  if (n > 0) atomicMax(needed, n);
  for (int c = 0; c < cap; ++c) {
    int32_t who = -1;
    double sx = 0.0, sy = 0.0, sz = 0.0;
    if (c < n) {
      const HistEntry e = hist[(int64_t)c * stride + k];
      who = (int32_t)e.orig;
      sx = e.sx;
      sy = e.sy;
      sz = e.sz;
    }
    partner[g * cap + c] = who;
    spring[3 * (g * cap + c)] = sx;
    spring[3 * (g * cap + c) + 1] = sy;
    spring[3 * (g * cap + c) + 2] = sz;
  }
}

// Checks a history in original order for one system (partners ascending, in
// the system, not the particle itself; springs finite) and takes the largest
// count.  err: 1 for a spring that is not finite, 2 for a bad partner.
__global__ void k_check_history(SysDev S, const int32_t *partner, const double *spring,
                                int32_t cap, int32_t *needed, int32_t *err) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= S.n) return;
  const int64_t g = S.o_off + i;
  int n = 0, prev = -1, e = 0;
  for (int c = 0; c < cap; ++c) {
    const int32_t who = partner[g * cap + c];
    if (who < 0) break;
    if (who >= S.n || who == (int32_t)i || who <= prev) e |= 2;
    const double *sp = spring + 3 * (g * cap + c);
    if (!isfinite(sp[0]) || !isfinite(sp[1]) || !isfinite(sp[2])) e |= 1;
    prev = who;
    ++n;
  }
  if (n > 0) atomicMax(needed, n);
  if (e) atomicOr(err, e);
}

// Loads a checked history into the tables: each slot takes the contacts of
// the particle it holds (whatever the storage order).
__global__ void k_set_history(const SysDev *sys, const int32_t *tile_sys, const uint32_t *origs,
                              const int32_t *partner, const double *spring, int32_t cap,
                              HistEntry *hist, int32_t *hcnt, int64_t stride) {
  const int64_t t = blockIdx.x;
  const SysDev &S = sys[tile_sys[t]];
  const int local = (int)(t - S.tile_off) * TILE + (int)threadIdx.x;
  if (local >= S.n || !S.friction) return;
  const int64_t k = S.p_off + local;
  const int64_t g = S.o_off + origs[k];
  int n = 0;
  for (int c = 0; c < cap; ++c) {
    const int32_t who = partner[g * cap + c];
    if (who < 0) break;
    HistEntry e;
    e.sx = spring[3 * (g * cap + c)];
    e.sy = spring[3 * (g * cap + c) + 1];
    e.sz = spring[3 * (g * cap + c) + 2];
    e.orig = (uint32_t)who;
    e.pad = 0;
    hist[(int64_t)c * stride + k] = e;
    ++n;
  }
  hcnt[k] = n;
}

// The Verlet state in the caller's original order: x0 (FP32) and R_NL of the
// last broad phase, one float4 per particle.
__global__ void k_get_bp(const SysDev *sys, const int32_t *tile_sys, const uint32_t *origs,
                         const float4 *bp, float4 *x0r) {
  const int64_t t = blockIdx.x;
  const SysDev &S = sys[tile_sys[t]];
  const int local = (int)(t - S.tile_off) * TILE + (int)threadIdx.x;
  if (local >= S.n) return;
  const int64_t k = S.p_off + local;
  x0r[S.o_off + origs[k]] = bp[k];
}

// Loads a Verlet state given in original order into the slots; flags bad values
// in *err: bit 0 not finite, bit 1 R_NL below R_C or beyond the cap.
__global__ void k_set_bp(const SysDev *sys, const int32_t *tile_sys, const uint32_t *origs,
                         const float2 *ri, const float4 *x0r, float4 *bp, int32_t *err) {
  const int64_t t = blockIdx.x;
  const SysDev &S = sys[tile_sys[t]];
  const int local = (int)(t - S.tile_off) * TILE + (int)threadIdx.x;
  if (local >= S.n) return;
  const int64_t k = S.p_off + local;
  const float4 b = x0r[S.o_off + origs[k]];
  int e = 0;
  if (!isfinite(b.x) || !isfinite(b.y) || !isfinite(b.z) || !isfinite(b.w)) e |= 1;
  else if (!(b.w >= ri[k].x) || !(b.w <= (float)S.cap)) e |= 2;
  if (e) atomicOr(err, e);
  bp[k] = b;
}

// Copy the state back to the caller's original order.
__global__ void k_get_state(const SysDev *sys, const int32_t *tile_sys, const X3 *xs, const V3 *vs,
                            const uint32_t *origs, double *x, double *v) {
  const int64_t t = blockIdx.x;
  const SysDev &S = sys[tile_sys[t]];
  const int local = (int)(t - S.tile_off) * TILE + (int)threadIdx.x;
  if (local >= S.n) return;
  const int64_t k = S.p_off + local;
  const int64_t g = S.o_off + origs[k];
  if (x) {
    const X3 p = xs[k];
    x[3 * g] = p.x;
    x[3 * g + 1] = p.y;
    x[3 * g + 2] = p.z;
  }
  if (v) {
    const V3 q = vs[k];
    v[3 * g] = q.vx;
    v[3 * g + 1] = q.vy;
    v[3 * g + 2] = q.vz;
  }
}

// ------------------------------------------------------------------ pair export

// Per original index i of system S: how many row entries j have orig(j) > i
// (and positive overlap when contacts_only).
__global__ void k_pairs_count(SysDev S, const X3 *xs, const float2 *ri, const uint32_t *origs,
                              const int32_t *cnt, const int32_t *nbr, int64_t stride,
                              int32_t contacts_only, int32_t *counts) {
  const int local = blockIdx.x * blockDim.x + threadIdx.x;
  if (local >= S.n) return;
  const int64_t k = S.p_off + local;
  const X3 me = xs[k];
  const float mrc = ri[k].x;
  const uint32_t mo = origs[k];
  int c = 0;
  const int len = cnt[k];
  for (int q = 0; q < len; ++q) {
    const int64_t j = S.p_off + nbr[row_index(stride, k, q)];
    if (origs[j] <= mo) continue;
    if (contacts_only) {
      double dx, dy, dz, d, delta;
      if (!overlap_positive(me, mrc, xs[j], ri[j].x, dx, dy, dz, d, delta)) continue;
    }
    ++c;
  }
  counts[mo] = c;
}

__global__ void k_pairs_write(SysDev S, const X3 *xs, const float2 *ri, const uint32_t *origs,
                              const int32_t *cnt, const int32_t *nbr, int64_t stride,
                              int32_t contacts_only, const int64_t *offsets, int64_t cap,
                              int32_t *pairs, double *delta_out) {
  const int local = blockIdx.x * blockDim.x + threadIdx.x;
  if (local >= S.n) return;
  const int64_t k = S.p_off + local;
  const X3 me = xs[k];
  const float mrc = ri[k].x;
  const uint32_t mo = origs[k];
  int64_t off = offsets[mo];
  const int len = cnt[k];
  for (int q = 0; q < len; ++q) {
    const int64_t j = S.p_off + nbr[row_index(stride, k, q)];
    const uint32_t oo = origs[j];
    if (oo <= mo) continue;
    const X3 o = xs[j];
    const float orc = ri[j].x;
    double dx, dy, dz, d = 0.0, delta = 0.0;
    const bool touch = overlap_positive(me, mrc, o, orc, dx, dy, dz, d, delta);
    if (contacts_only && !touch) continue;
    if (!touch) {
      dx = me.x - o.x;
      dy = me.y - o.y;
      dz = me.z - o.z;
      delta = ((double)mrc + (double)orc) - sqrt(dx * dx + dy * dy + dz * dz);
    }
    if (off < cap) {
      pairs[2 * off] = (int32_t)mo;
      pairs[2 * off + 1] = (int32_t)oo;
      if (delta_out) delta_out[off] = delta;
    }
    ++off;
  }
}

// Exclusive prefix sum of n int32 counts into int64 offsets, one workgroup.
__global__ __launch_bounds__(TILE) void k_scan_single(const int32_t *in, int64_t n, int64_t *out,
                                                      int64_t *total) {
  __shared__ int64_t carry_s;
  if (threadIdx.x == 0) carry_s = 0;
  __syncthreads();
  for (int64_t base = 0; base < n; base += TILE) {
    const int64_t i = base + threadIdx.x;
    const int v = i < n ? in[i] : 0;
    int tot;
    const int incl = block_inclusive_scan(v, &tot);
    const int64_t carry = carry_s;
    if (i < n) out[i] = carry + incl - v;
    __syncthreads();
    if (threadIdx.x == 0) carry_s = carry + tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) *total = carry_s;
}

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace vb

// ------------------------------------------------------------------ launchers
// Host entry points of the kernels above (C++ linkage, internal to the library).
namespace vb {

// t0/t1 (both null, or both events): events that take the kernel's own start
// and end times.
template <typename K>
static void launch_timed(K kernel, dim3 g, dim3 b, uint32_t lds, hipStream_t st, hipEvent_t t0,
                         hipEvent_t t1, const StepArgs &a) {
  if (t0 || t1) hipExtLaunchKernelGGL(kernel, g, b, lds, st, t0, t1, 0, a);
  else hipLaunchKernelGGL(kernel, g, b, lds, st, a);
}

template <bool FRIC, bool WALLS>
static void launch_step_t(const StepArgs &a, int64_t n_tiles, int unroll, hipStream_t st,
                          hipEvent_t t0, hipEvent_t t1) {
  const dim3 g((unsigned)n_tiles), b(TILE);
  if (unroll >= 8) launch_timed(k_step<8, FRIC, WALLS>, g, b, 0, st, t0, t1, a);
  else if (unroll >= 4) launch_timed(k_step<4, FRIC, WALLS>, g, b, 0, st, t0, t1, a);
  else if (unroll >= 2) launch_timed(k_step<2, FRIC, WALLS>, g, b, 0, st, t0, t1, a);
  else launch_timed(k_step<1, FRIC, WALLS>, g, b, 0, st, t0, t1, a);
}

// friction: 1 if some system of the batch has friction (its history is kept);
// walls: 1 if some system has planar or cylindrical walls besides the box faces
hipError_t launch_step(const StepArgs &a, int64_t n_tiles, int unroll, int friction, int walls,
                       hipStream_t st, hipEvent_t t0, hipEvent_t t1) {
  if (n_tiles <= 0) return hipSuccess;
  if (friction && walls) launch_step_t<true, true>(a, n_tiles, unroll, st, t0, t1);
  else if (friction) launch_step_t<true, false>(a, n_tiles, unroll, st, t0, t1);
  else if (walls) launch_step_t<false, true>(a, n_tiles, unroll, st, t0, t1);
  else launch_step_t<false, false>(a, n_tiles, unroll, st, t0, t1);
  return hipGetLastError();
}

// Dynamic LDS of k_pairs<nt>: staged candidates (position and R_NL with four
// spare entries for the scan's reads past a range, and original index) and the
// rows (W + 4 rows of 16-bit staged indices, the last four spares for full rows,
// or W rows of 32-bit keys for half the threads in the fallback path).
size_t pairs_lds_bytes(int width, int pmax, int nt) {
  return (size_t)(pmax + 4) * sizeof(float4) + (size_t)pmax * sizeof(int32_t) +
         (size_t)nt * (size_t)(width + 4) * sizeof(uint16_t);
}

// Static LDS of the pair search with nt threads (bytes); -1 if not known.
int64_t pairs_static_lds(int nt) {
  hipFuncAttributes fa;
  hipError_t e;
  if (nt == 256) e = hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(k_pairs<256>));
  else if (nt == 512) e = hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(k_pairs<512>));
  else e = hipFuncGetAttributes(&fa, reinterpret_cast<const void *>(k_pairs<384>));
  return e == hipSuccess ? (int64_t)fa.sharedSizeBytes : -1;
}

// Threads per pair-search workgroup the library is built for.
bool pairs_threads_supported(int nt) { return nt == 256 || nt == 384 || nt == 512; }

// Workgroups of the pair search with nt threads resident on one CU at once (at
// least 1).
int pairs_blocks_per_cu(int width, int pmax, int nt) {
  int n = 0;
  const size_t lds = pairs_lds_bytes(width, pmax, nt);
  hipError_t e;
  if (nt == 256) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_pairs<256>, 256, lds);
  else if (nt == 512) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_pairs<512>, 512, lds);
  else e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_pairs<384>, 384, lds);
  if (e != hipSuccess) return 1;
  return n > 0 ? n : 1;
}

template <int NT>
static void launch_pairs_t(const BroadArgs &a, int grid_pairs, uint32_t lds, hipStream_t st,
                           hipEvent_t t1) {
  if (t1) hipExtLaunchKernelGGL(k_pairs<NT>, dim3(grid_pairs), dim3(NT), lds, st, nullptr, t1, 0, a);
  else hipLaunchKernelGGL(k_pairs<NT>, dim3(grid_pairs), dim3(NT), lds, st, a);
}

// t0 takes the start of the binning kernel, t1 the end of the pair search
// (both null, or both events).  The pair search runs nt threads per workgroup.
hipError_t launch_broad_phase(const BroadArgs &a, int grid_bin, int grid_pairs, int nt, hipStream_t st,
                              hipEvent_t t0, hipEvent_t t1) {
  if (grid_bin <= 0) return hipSuccess;
  const uint32_t lds = (uint32_t)pairs_lds_bytes(a.width, a.pmax, nt);
  if (t0 || t1)
    hipExtLaunchKernelGGL(k_bin, dim3(grid_bin), dim3(TILE), 0, st, t0, grid_pairs > 0 ? nullptr : t1,
                          0, a);
  else
    hipLaunchKernelGGL(k_bin, dim3(grid_bin), dim3(TILE), 0, st, a);
  if (grid_pairs > 0) {
    if (nt == 256) launch_pairs_t<256>(a, grid_pairs, lds, st, t1);
    else if (nt == 512) launch_pairs_t<512>(a, grid_pairs, lds, st, t1);
    else launch_pairs_t<384>(a, grid_pairs, lds, st, t1);
  }
  return hipGetLastError();
}

hipError_t launch_sort(const SortArgs &a, hipStream_t st) {
  if (a.n_tiles <= 0) return hipSuccess;
  const unsigned nt = (unsigned)a.n_tiles;
  const int64_t per = (int64_t)TILE * SCAN_ITEMS;
  const int64_t nb = (a.n_cells + per - 1) / per;
  hipLaunchKernelGGL(k_sort_count, dim3(nt), dim3(TILE), 0, st, a);
  hipLaunchKernelGGL(k_scan_blocks, dim3((unsigned)nb), dim3(TILE), 0, st, a.cell_count,
                     a.n_cells, a.cell_start, a.block_sum);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(TILE), 0, st, a.block_sum, nb);
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(TILE), 0, st, a.cell_start, a.n_cells,
                     a.block_sum, nb);
  hipLaunchKernelGGL(k_sort_scatter, dim3(nt), dim3(TILE), 0, st, a);
  hipLaunchKernelGGL(k_sort_place, dim3(nt), dim3(TILE), 0, st, a);
  return hipGetLastError();
}

int64_t scan_blocks(int64_t n_cells) {
  const int64_t per = (int64_t)TILE * SCAN_ITEMS;
  return (n_cells + per - 1) / per;
}

hipError_t launch_stats_reduce(const SysDev *sys, const TileStats *stats, const int32_t *ring,
                               int64_t n_tiles, int32_t n_sys, int32_t step0, int32_t nsteps,
                               RecordDev *out, hipStream_t st) {
  if (nsteps <= 0 || n_sys <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_stats_reduce, dim3(n_sys, nsteps), dim3(TILE), 0, st, sys, stats, ring,
                     n_tiles, n_sys, step0, out);
  return hipGetLastError();
}

hipError_t launch_set_state(const SysDev &S, X3 *xs, V3 *vs, float2 *ri, uint32_t *origs,
                            const double *x, const double *v, const float *rc, const float *invm,
                            int32_t *err, int32_t *r_lo, int32_t *r_hi, hipStream_t st) {
  const int64_t padded = (int64_t)S.n_tiles * TILE;
  if (padded == 0) return hipSuccess;
  hipLaunchKernelGGL(k_set_state, dim3((unsigned)(padded / 256)), dim3(256), 0, st, S, xs, vs, ri,
                     origs, x, v, rc, invm, err, r_lo, r_hi);
  return hipGetLastError();
}

hipError_t launch_get_state(const SysDev *sys, const int32_t *tile_sys, int64_t n_tiles,
                            const X3 *xs, const V3 *vs, const uint32_t *origs, double *x, double *v,
                            hipStream_t st) {
  if (n_tiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_get_state, dim3((unsigned)n_tiles), dim3(TILE), 0, st, sys, tile_sys, xs,
                     vs, origs, x, v);
  return hipGetLastError();
}

hipError_t launch_get_bp(const SysDev *sys, const int32_t *tile_sys, int64_t n_tiles,
                         const uint32_t *origs, const float4 *bp, float4 *x0r, hipStream_t st) {
  if (n_tiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_get_bp, dim3((unsigned)n_tiles), dim3(TILE), 0, st, sys, tile_sys, origs, bp,
                     x0r);
  return hipGetLastError();
}

hipError_t launch_set_bp(const SysDev *sys, const int32_t *tile_sys, int64_t n_tiles,
                         const uint32_t *origs, const float2 *ri, const float4 *x0r, float4 *bp,
                         int32_t *err, hipStream_t st) {
  if (n_tiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_set_bp, dim3((unsigned)n_tiles), dim3(TILE), 0, st, sys, tile_sys, origs, ri,
                     x0r, bp, err);
  return hipGetLastError();
}

hipError_t launch_get_history(const SysDev *sys, const int32_t *tile_sys, int64_t n_tiles,
                              const uint32_t *origs, const HistEntry *hist, const int32_t *hcnt,
                              int64_t stride, int32_t hcap, int32_t *partner, double *spring,
                              int32_t cap, int32_t *needed, hipStream_t st) {
  if (n_tiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_get_history, dim3((unsigned)n_tiles), dim3(TILE), 0, st, sys, tile_sys, origs,
                     hist, hcnt, stride, hcap, partner, spring, cap, needed);
  return hipGetLastError();
}

hipError_t launch_check_history(const SysDev &S, const int32_t *partner, const double *spring,
                                int32_t cap, int32_t *needed, int32_t *err, hipStream_t st) {
  if (S.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_check_history, dim3((unsigned)((S.n + 255) / 256)), dim3(256), 0, st, S,
                     partner, spring, cap, needed, err);
  return hipGetLastError();
}

hipError_t launch_set_history(const SysDev *sys, const int32_t *tile_sys, int64_t n_tiles,
                              const uint32_t *origs, const int32_t *partner, const double *spring,
                              int32_t cap, HistEntry *hist, int32_t *hcnt, int64_t stride,
                              hipStream_t st) {
  if (n_tiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_set_history, dim3((unsigned)n_tiles), dim3(TILE), 0, st, sys, tile_sys, origs,
                     partner, spring, cap, hist, hcnt, stride);
  return hipGetLastError();
}

hipError_t launch_pairs(const SysDev &S, const X3 *xs, const float2 *ri, const uint32_t *origs,
                        const int32_t *cnt, const int32_t *nbr, int64_t stride,
                        int32_t contacts_only, int32_t *counts, int64_t *offsets, int64_t *total,
                        int64_t cap, int32_t *pairs, double *delta, hipStream_t st) {
  if (S.n <= 0) return hipSuccess;
  const unsigned g = (unsigned)((S.n + 255) / 256);
  hipLaunchKernelGGL(k_pairs_count, dim3(g), dim3(256), 0, st, S, xs, ri, origs, cnt, nbr, stride,
                     contacts_only, counts);
  hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(TILE), 0, st, counts, (int64_t)S.n, offsets,
                     total);
  if (pairs)
    hipLaunchKernelGGL(k_pairs_write, dim3(g), dim3(256), 0, st, S, xs, ri, origs, cnt, nbr, stride,
                       contacts_only, offsets, cap, pairs, delta);
  return hipGetLastError();
}

hipError_t launch_posq(const SysDev *sys, const int32_t *tile_sys, const int32_t *rrange, int n_sys,
                       const X3 *xs, const float2 *ri, uint64_t *posq, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_posq, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, sys, tile_sys,
                     rrange, n_sys, xs, ri, posq, n);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

}  // namespace vb
