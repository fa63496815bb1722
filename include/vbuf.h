/*
 * vbuf.h -- C ABI of libvbuf.so: the local Verlet buffer DEM step on one AMD
 * Instinct MI355X (gfx950).
 *
 * The method (Mainassara Checkaraou, Besseron, Rousset, Qi, Peters, "Local Verlet
 * buffer approach for broad-phase interaction detection in Discrete Element
 * Method"):
 *   - every particle p carries a skin  skin_p = K |v_p| dt        (Sec. 4.1, Eq. skin_formulus1)
 *   - its broad-phase sphere is  R_NL,p = R_C,p + skin_p          (Sec. 4, Eq. bounding_sphere)
 *     capped by the cell size                                     (Sec. 5.1, Eq. skin_formulus_mincell)
 *   - the linked-cell broad phase on those spheres builds the Verlet list
 *                                                                 (Sec. 3.2, Alg. 1)
 *   - the list is reused while every particle's straight-line displacement since
 *     the last broad phase is within its skin, and rebuilt otherwise
 *                                                                 (Sec. 4.2, Eq. update, Def. autoverlet)
 *   - the narrow phase tests each listed pair for overlap         (Sec. 3.2, Eq. delta)
 *   - contact forces (normal linear spring-dashpot) and velocity-Verlet integration
 *                                                                 (Sec. 3.1, Sec. 5.1)
 * By the theorem of Sec. 4.2 the results equal those of running the broad phase
 * at every step; this library reproduces that bit for bit (forces are summed in
 * ascending original partner index whatever the list holds).
 *
 * Conventions common to every call:
 *   - Pointers named d_* are device pointers on the context's device (for example
 *     the data_ptr() of a PyTorch tensor); pointers named h_* are host pointers.
 *     The caller owns every pointer it passes; the library never frees them and
 *     keeps none of them after the call returns.
 *   - The library owns its workspace (state buffers, cell arrays, Verlet lists),
 *     allocated at create and grown when a list row overflows.
 *   - Particle order at the boundary is always the caller's original order, with
 *     the systems of a batch concatenated in creation order.  The internal
 *     cell-sorted order is invisible.
 *   - Every call returns a vb_status; on failure vb_last_error() gives a message
 *     for that context.  No exception or abort crosses the ABI.
 *   - All work of a context is queued on the HIP stream given at create; calls
 *     that return host data synchronise that stream.  One context is not safe to
 *     use from several host threads at once.
 *   - Units are the caller's; the synthetic workloads use box units (the longest
 *     box side is 1).
 *   - Environment variables read at create, for tuning: VBUF_GRAPHS=0 (results
 *     bit-identical) launches every step on its own instead of
 *     replaying blocks of 64 steps as one captured HIP graph; VBUF_STEP_UNROLL
 *     = 1, 2, 4 or 8 sets the partner gathers each thread of the step kernel
 *     keeps in flight; VBUF_XCD_REMAP = 0, 1 or 2 sets the step kernel's tile
 *     order (see vb_set_launch); VBUF_PAIR_WINDOWS=0 makes the pair search
 *     test whole rows of cells instead of the x windows within reach (the same
 *     lists).  VBUF_STEP_UNROLL or VBUF_XCD_REMAP fixes the
 *     launch shape of the context (vb_set_launch), which vb_tune then does not
 *     take from its cache.  Results are bit-identical for every setting: the
 *     FP64 contact law and integration round every operation (no contraction),
 *     in one fixed order.
 */
#ifndef VBUF_H
#define VBUF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t vb_status;
#define VB_OK 0
#define VB_EINVAL (-1)      /* invalid argument or parameter                       */
#define VB_ENOMEM (-2)      /* device or host allocation failed                    */
#define VB_EDEVICE (-3)     /* a HIP call failed                                   */
#define VB_ECAPACITY (-4)   /* a list row, cell bin or friction history exceeded its maximum */
#define VB_ENONFINITE (-5)  /* NaN or Inf in the state given, or reached during a run */

/* How the broad-phase sphere of each particle is extended. */
#define VB_SKIN_LOCAL 0     /* skin_p = K |v_p| dt, the paper's local skin (Eq. skin_formulus1)  */
#define VB_SKIN_UNIFORM 1   /* skin_p = skin_uniform, the classic global Verlet skin (Eq. skin_val) */
#define VB_NO_BUFFER 2      /* broad phase at every step with R_NL = R_C: the paper's plain baseline */
#define VB_FIXED_INTERVAL 3 /* broad phase every fixed_interval steps with the uniform skin; the  */
                            /* fixed-update practice the automatic scheme replaces (Sec. 1, 4.2)  */

#define VB_MAX_PLANES 4
#define VB_MAX_CYLINDERS 2

/* Parameters of one particle system.  Float fields are read as given; positions,
 * velocities and the contact law are evaluated in FP64. */
typedef struct vb_params {
  int32_t skin_mode;      /* VB_SKIN_LOCAL, VB_SKIN_UNIFORM, VB_NO_BUFFER or VB_FIXED_INTERVAL   */
  int32_t cap_mode;       /* 0: R_NL <= L_C/2, one-ring cell search (default);                   */
                          /* 1: R_NL <= L_C as printed in Eq. skin_formulus_mincell, two-ring    */
  double K;               /* skin factor of Eq. skin_formulus1: the steps a skin lasts (Sec. 4.1)  */
  double dt;              /* time step                                                            */
  double cell_size;       /* L_C: the uniform cell edge of the linked-cell grid (Sec. 3.2)        */
  double skin_uniform;    /* skin of VB_SKIN_UNIFORM and VB_FIXED_INTERVAL                        */
  double eps;             /* absolute margin of the FP32 broad-phase inclusion test, at least     */
                          /* 2^-19 max(|lo|, |hi|) (16 FP32 ulps of the largest coordinate)       */
  double lo[3], hi[3];    /* box corners; a planar wall on each face                               */
  double kn, gamma_n;     /* normal spring stiffness and dashpot coefficient                       */
  double gravity[3];      /* gravitational acceleration                                            */
  int32_t max_neighbors;  /* initial width of a Verlet-list row (grown on overflow), 1..128       */
  int32_t fixed_interval; /* broad-phase period of VB_FIXED_INTERVAL (>= 1)                        */
  int32_t reorder_interval; /* steps between re-sorts of the particle storage by cell, for memory */
                          /* locality (0: only after vb_set_state); the batch uses system 0's     */
  int32_t bin_capacity;   /* initial particles per cell bin (grown on overflow), 1..256; 0 = 16   */
  int32_t n_planes;       /* planar walls besides the box faces, 0..VB_MAX_PLANES                 */
  int32_t reserved_;
  double planes[VB_MAX_PLANES][5]; /* (n_x, n_y, n_z, d, z_min): unit normal n pointing into   */
                          /* the domain; the wall fills n.x < d and acts, with the contact law   */
                          /* of the box faces, on particles whose centre has z > z_min (a finite */
                          /* wall such as a hopper side above its outlet).  Walls act after the  */
                          /* box faces, in index order.                                           */
  double kt, gamma_t, mu; /* tangential spring, tangential dashpot and Coulomb coefficient of the */
                          /* particle-particle friction (translational; the spring of a contact   */
                          /* is kept while the contact lasts); mu = 0 or kt = gamma_t = 0: none   */
  int32_t contact_capacity; /* initial contacts per particle the friction history holds (grown  */
                          /* on overflow), 1..64; 0 = 16                                           */
  int32_t reserved2_;
  int32_t n_cylinders;    /* vertical cylindrical walls, 0..VB_MAX_CYLINDERS                      */
  int32_t reserved3_;
  double cylinders[VB_MAX_CYLINDERS][4]; /* (c_x, c_y, R, z_min): the domain is the inside of   */
                          /* the cylinder of radius R > 0 about the vertical axis through         */
                          /* (c_x, c_y) (a silo); the wall acts, with the contact law of the box  */
                          /* faces, on particles whose centre has z > z_min, with the normal      */
                          /* towards the axis (none for a centre on the axis).  Cylinders act     */
                          /* after the planar walls, in index order.                              */
} vb_params;

/* Diagnostics of one time step n of one system (the state x^n whose forces the
 * step evaluates, then its advance to x^{n+1}). */
typedef struct vb_step_record {
  int32_t step;           /* n                                                                    */
  int32_t rebuilt;        /* 1 if a broad phase ran at x^n (Def. autoverlet)                       */
  int64_t list_pairs;     /* unique pairs in the Verlet list used at x^n                           */
  int64_t contacts;       /* unique pairs with positive overlap at x^n (Eq. delta)                 */
  int64_t violators;      /* particles with |x^{n+1} - x0| > skin after the step (Eq. update)      */
  float max_excess;       /* max over particles of |x^{n+1} - x0| - skin (FP32)                    */
  int32_t reserved;
  double kinetic_energy;  /* sum of m |v^n|^2 / 2 with the full-step velocity v^n                 */
} vb_step_record;

typedef struct vb_ctx vb_ctx;

/* Create a context for one system of n particles (0 <= n <= 2^29 - 256): the inputs of the
 * method as the paper states them, the skin factor K and time step dt (Sec. 4.1,
 * Eq. skin_formulus1), the uniform cell size L_C of the linked-cell grid
 * (Sec. 3.2, Alg. 1; Sec. 5.1, Eq. skin_formulus_mincell) and the contact model
 * (Sec. 5.1).  stream is a hipStream_t (NULL for the default stream); *out
 * receives the context, which owns every device buffer the method needs.
 * Errors: VB_EINVAL for a bad parameter (checked before any device call),
 * VB_ENOMEM, VB_EDEVICE. */
vb_status vb_create(const vb_params *h_params, int64_t n, void *stream, vb_ctx **out);

/* Create a context for n_sys independent systems solved together, one launch per
 * phase for the whole batch (each system follows the method of Sec. 4 on its
 * own: its own K, cells, skins and broad-phase decisions).  h_params[s] and
 * h_n[s] describe system s.  Errors as vb_create, and VB_EINVAL for n_sys
 * outside 1..1024. */
vb_status vb_batch_create(const vb_params *h_params, const int64_t *h_n, int32_t n_sys,
                          void *stream, vb_ctx **out);

/* Load the state of the particles (Sec. 3.2: centre X_i and bounding radius R_C,i
 * of every particle; Sec. 4.1: its velocity v_p), in original order, all systems
 * concatenated:
 *   d_x    [N][3] FP64 positions x^n
 *   d_v    [N][3] FP64 velocities: the full-step velocity v^0 when v_is_half_step
 *                 is 0 (a fresh start: the first step applies half a kick), or the
 *                 half-step velocity v^{n-1/2} when 1 (a resume from vb_get_state)
 *   d_rc   [N]    FP32 cut-off (contact) radius R_C > 0, with 2 R_C <= L_C (cap 0)
 *                 or R_C <= L_C (cap 1)
 *   d_invm [N]    FP32 inverse mass > 0
 * The step counter restarts at 0 and the next step runs a broad phase (the
 * proof of Sec. 4.2 starts from one).  Synchronises the stream.
 * Errors: VB_ENONFINITE for NaN/Inf, VB_EINVAL for a radius or mass out of range. */
vb_status vb_set_state(vb_ctx *ctx, const double *d_x, const double *d_v, const float *d_rc,
                       const float *d_invm, int32_t v_is_half_step);

/* Advance every system n_steps time steps of the time loop with the Verlet check
 * (flow chart of Sec. 4; Sec. 4.2, Eq. update, Def. autoverlet): at each step a
 * system whose list failed the validity test after the previous step (and every
 * system at its first step) runs the broad phase on extended spheres, then every
 * system runs the narrow phase on its list (Eq. delta), the contact forces and
 * velocity-Verlet integration (Sec. 3.1, Sec. 5.1), and the validity test for the
 * next step.  h_hist, if not NULL, receives [n_sys][n_steps] records.
 * A Verlet-list row, a cell bin or a friction history that overflows is grown,
 * and the steps since the call's last snapshot run again: a call keeps its
 * starting state and, every 4 blocks of 64 steps, the state once every step
 * before it is known free of overflow.  A run from a snapshot rebuilds the rows
 * from the stored x0 and R_NL, so results, records and the schedule of broad
 * phases are those of a run that never overflowed.  The overflow counters are
 * read back after every block of 64 steps, one block behind the device.
 * Synchronises the stream at the end.
 * Errors: VB_ECAPACITY if a row needs more than 128 entries, a bin more than 256
 * or a friction history more than 64 contacts; VB_ENONFINITE if the state
 * becomes NaN or infinite (the context then needs vb_set_state again);
 * VB_ENOMEM, VB_EDEVICE. */
vb_status vb_run(vb_ctx *ctx, int32_t n_steps, vb_step_record *h_hist);

/* Copy the state out (the positions and velocities the integration of Sec. 3.1
 * advances), original order: d_x [N][3] positions x^n and d_v [N][3]
 * velocities (v^{n-1/2} after at least one step, else the loaded velocities).
 * Either pointer may be NULL.  *h_v_is_half_step (if not NULL) tells which.
 * Synchronises the stream.  Errors: VB_EINVAL without a loaded state. */
vb_status vb_get_state(vb_ctx *ctx, double *d_x, double *d_v, int32_t *h_v_is_half_step);

/* The Verlet state (what the automatic update of Sec. 4.2 carries from one step
 * to the next besides positions and velocities: Eq. update, Def. autoverlet),
 * for a checkpoint that resumes with the same schedule of broad phases:
 *   d_x0r     [N][4] FP32, original order: the reference position x0 of the last
 *             broad phase (x, y, z; Eq. update) and the extended radius R_NL of
 *             that broad phase (Eq. bounding_sphere, capped as in Eq.
 *             skin_formulus_mincell);
 *   h_pending [n_sys]: 1 if the system's list failed the validity test after the
 *             last step (or a broad phase was requested), so that the next step
 *             runs a broad phase;
 *   *h_step   the step counter (may be NULL).
 * Synchronises the stream.  Errors: VB_EINVAL without a loaded state or before
 * the first step (no list yet). */
vb_status vb_get_verlet_state(vb_ctx *ctx, float *d_x0r, int32_t *h_pending, int64_t *h_step);

/* Load a Verlet state in the layout of vb_get_verlet_state, right after
 * vb_set_state and before any vb_run.  The next step rebuilds each system's list
 * from the given x0 and R_NL (the set of pairs within reach of those spheres,
 * Alg. 1) without re-deriving skins, or runs a broad phase where h_pending says
 * so, and the step counter continues from step.  With vb_set_state(...,
 * v_is_half_step = 1) (and vb_set_history under friction) from one checkpoint,
 * the resumed run repeats the uninterrupted one: positions, velocities, the
 * broad-phase schedule and every record field (the kinetic energy up to its
 * summation order).  Synchronises the stream.
 * Errors: VB_EINVAL if a step ran since vb_set_state, for step outside
 * 0..2^31-2, a pending flag other than 0 or 1, or an R_NL below its R_C or beyond
 * the cap; VB_ENONFINITE for NaN or Inf. */
vb_status vb_set_verlet_state(vb_ctx *ctx, const float *d_x0r, const int32_t *h_pending,
                              int64_t step);

/* The friction history, for a checkpoint that resumes exactly: the contacts of
 * the last step with their tangential springs (the state a frictional step
 * carries besides positions and velocities; Sec. 5.1 names static friction,
 * whose spring lasts as long as its contact).  In original order, all systems
 * concatenated:
 *   d_partner [N][cap] int32: particle g's partners (original index local to its
 *             system), ascending, then -1 after the last one
 *   d_spring  [N][cap][3] FP64: the spring of each of those contacts as seen
 *             from particle g (0 after the last one)
 * Systems without friction export no contacts.  *h_needed (may be NULL)
 * receives the largest contact count of any particle.  Synchronises the stream.
 * Errors: VB_EINVAL if no system has friction or no state is loaded;
 * VB_ECAPACITY if a particle has more than cap contacts (then only the first
 * cap of each are written). */
vb_status vb_get_history(vb_ctx *ctx, int32_t *d_partner, double *d_spring, int32_t cap,
                         int32_t *h_needed);

/* Load a friction history (the per-contact springs of the static friction named
 * in Sec. 5.1) in the layout of vb_get_history, right after
 * vb_set_state and before any vb_run: with the state and the history of a
 * checkpoint (vb_get_state, vb_get_history; v_is_half_step = 1), the run goes on
 * bit for bit as the uninterrupted one.  Without it a resumed run starts every
 * spring at zero.  Tables grow to the largest count.  Synchronises the stream.
 * Errors: VB_EINVAL if no system has friction, if a step ran since vb_set_state,
 * or for a partner out of range, equal to the particle or out of order;
 * VB_ENONFINITE for a spring with NaN or Inf; VB_ECAPACITY beyond 64 contacts. */
vb_status vb_set_history(vb_ctx *ctx, const int32_t *d_partner, const double *d_spring,
                         int32_t cap);

/* The canonical unique list of one system as pairs (i, j), i < j, in original
 * indices local to the system, sorted lexicographically:
 *   which = 0: the Verlet list of the last broad phase (Def. verletlist);
 *   which = 1: the contacts (overlap > 0) at the current positions, after the
 *              broad phase that the next step would run if the list is invalid.
 * d_pairs [cap][2] int32, d_delta [cap] FP64 overlaps (may be NULL).  *h_n receives
 * the full count even if it exceeds cap (then only cap pairs are written).
 * Synchronises the stream. */
vb_status vb_get_pairs(vb_ctx *ctx, int32_t sys, int32_t which, int32_t *d_pairs,
                       double *d_delta, int64_t cap, int64_t *h_n);

/* vb_get_pairs for callers that cannot allocate device memory (code that must
 * not call hipMalloc, such as tight serving loops or harnesses that forbid it):
 * the same result, with the export's per-particle scratch taken from a fixed
 * array in the library (12 bytes per particle of the largest system it takes,
 * VB_NOALLOC_MAX_N, held on each device the library runs on until the process
 * ends) instead of the context's buffers.  This call allocates nothing.  Calls
 * on one device share that array: two calls that overlap on one device (from
 * several host threads or streams) race.  Synchronises the stream.
 * Errors: as vb_get_pairs, and VB_EINVAL for a system of more than
 * VB_NOALLOC_MAX_N particles. */
#define VB_NOALLOC_MAX_N 4194304
vb_status vb_get_pairs_noalloc(vb_ctx *ctx, int32_t sys, int32_t which, int32_t *d_pairs,
                               double *d_delta, int64_t cap, int64_t *h_n);

/* Launch shape of a context: the partner gathers each thread of the step kernel
 * keeps in flight (unroll 1, 2, 4 or 8), the step kernel's tile order (xcd_order
 * 0: launch order, 1: each of the 8 XCDs a contiguous range of tiles, 2: each
 * XCD runs of 32 consecutive tiles, the 8 runs of a group side by side) and the
 * threads of a pair-search workgroup (256, 384 or 512); a new context starts
 * from (4, 2, 384), or (8, 2, 384) for a batch with friction of 2^20 particles
 * or more, or from the shape vb_tune chose for its kind.  Results, records and
 * the schedule of broad phases do not depend on it (the steps are those of the
 * time loop of Sec. 3.1 whatever the shape), so it may change between any two
 * calls.  Errors: VB_EINVAL for a value outside those sets. */
vb_status vb_set_launch(vb_ctx *ctx, int32_t unroll, int32_t xcd_order, int32_t pairs_threads);
vb_status vb_get_launch(vb_ctx *ctx, int32_t *h_unroll, int32_t *h_xcd_order,
                        int32_t *h_pairs_threads);

/* Advance n_steps steps as vb_run does (the same positions and velocities)
 * while choosing the launch shape by measurement: the starting shape, then every
 * other gather count and tile order of the step kernel for n_steps/16 steps each
 * (at least 2), then every pair-search workgroup size on two forced broad phases
 * each (which change no result, theorem of Sec. 4.2, but show in the records'
 * rebuilt flags), each timed by HIP events on the kernels themselves; another
 * shape replaces the starting one only if it is more than 1 % faster.  The rest
 * of the steps run with the chosen shape.  The chosen shape stays with the context and, for the life
 * of the process, with its kind (log2 of its particle count, particles per cell,
 * friction on or off): a context of that kind created later starts from it.
 * h_hist as for vb_run.  Errors: VB_EINVAL for fewer than 26 steps; those of
 * vb_run. */
vb_status vb_tune(vb_ctx *ctx, int32_t n_steps, vb_step_record *h_hist);

/* Request a broad phase at the next step (all systems), as if a validity test
 * had failed (Def. autoverlet); by the theorem of Sec. 4.2 this changes no
 * result.  Errors: VB_EINVAL for a NULL ctx. */
vb_status vb_force_rebuild(vb_ctx *ctx);

/* Set the skin factor K of Eq. skin_formulus1 for system sys (every system when
 * sys < 0).  K is the method's one tuning parameter, with an optimum that
 * depends on the case (Sec. 5.4); by the theorem of Sec. 4.2 the results do not
 * depend on it, so it may change between two vb_run calls (a tuner does).  The
 * new K shapes the skins from the next broad phase on; the current list stays
 * valid until its own validity test fails.
 * Errors: VB_EINVAL if K is negative or not finite, or sys >= the system count. */
vb_status vb_set_K(vb_ctx *ctx, int32_t sys, double K);

/* Enable (1) or disable (0) per-kernel HIP-event timing of vb_run (the per-phase
 * split the paper reports, Sec. 5.4), and read the totals since timing was
 * enabled.  The events take the kernels' own start and
 * end times (as a kernel-trace profiler reports them, launch gaps excluded):
 * milliseconds from the start of the binning kernel to the end of the pair
 * search at every step (including the launches that found no system to rebuild;
 * storage re-sorts excluded), milliseconds in the step kernel, the number of
 * steps timed and the number of steps at which any system ran a broad phase. */
vb_status vb_set_timing(vb_ctx *ctx, int32_t on);
vb_status vb_phase_times(vb_ctx *ctx, double *h_ms_rebuild, double *h_ms_step,
                         int64_t *h_steps, int64_t *h_rebuild_steps);

/* Sizes: total particles N, systems, current row width (the longest Verlet-list
 * row it holds, Def. verletlist), current step counter (Sec. 3.1 time loop).
 * Any output pointer may be NULL.  Errors: VB_EINVAL for a NULL ctx. */
vb_status vb_get_info(vb_ctx *ctx, int64_t *h_n_total, int32_t *h_n_sys,
                      int32_t *h_row_width, int64_t *h_step);

/* Message of the last failed call on ctx (ctx may be NULL for a failed create).
 * The pointer stays valid until the next call on ctx. */
const char *vb_last_error(const vb_ctx *ctx);

/* Release every resource of ctx: the state, the Verlet lists and cell bins of
 * Alg. 1 and the friction history (NULL is ignored).  Synchronises the stream. */
void vb_destroy(vb_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* VBUF_H */
