/*
 * orc.h -- FP64 CPU oracle for the local Verlet buffer DEM step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may include, link or
 * call this code: only the test suite, the smoke check and the CPU baseline leg
 * of the benchmark use it.  It shares no code, header or constant with the HIP
 * library.
 *
 * What it computes (Mainassara Checkaraou et al., "Local Verlet buffer approach
 * for broad-phase interaction detection in Discrete Element Method"):
 *   - linked-cell broad phase on bounding spheres        (Sec. 3.2, Alg. 1)
 *   - sphere narrow phase, overlap delta                  (Sec. 3.2, Eq. delta)
 *   - extended spheres R_NL = R_C + skin                  (Sec. 4, Eq. bounding_sphere)
 *   - local skin  skin_p = K * |v_p| * dt                 (Sec. 4.1, Eq. skin_formulus1)
 *   - cap by the cell size                                (Sec. 5.1, Eq. skin_formulus_mincell)
 *   - validity test  dx_p <= skin_p, automatic update     (Sec. 4.2, Eq. update, Def. autoverlet)
 *   - velocity-Verlet integration, linear spring-dashpot  (Sec. 3.1, Sec. 5.1)
 * and, as the plain definition the method must reproduce exactly (Sec. 1 and
 * Sec. 4: results identical to running the broad phase every step), the naive
 * step whose contact set is found by brute force over all pairs.
 *
 * All arithmetic is IEEE double, no fused multiply-add, no reassociation.
 */
#ifndef ORC_H
#define ORC_H
#include <stdint.h>

#define ORC_MAX_PLANES 4
#define ORC_MAX_CYLINDERS 2

enum {
  ORC_SKIN_LOCAL = 0,      /* skin_p = K |v_p| dt (the paper's method)              */
  ORC_SKIN_UNIFORM = 1,    /* skin_p = skin_uniform for every particle               */
  ORC_NO_BUFFER = 2,       /* broad phase every step on R_NL = R_C (plain baseline) */
  ORC_FIXED_INTERVAL = 3,  /* broad phase every fixed_interval steps, uniform skin   */
  ORC_NAIVE = 4            /* no list at all: contacts by brute force every step     */
};

typedef struct {
  int32_t skin_mode;       /* one of the ORC_* modes above                                  */
  int32_t cap_mode;        /* 0: R_NL <= L_C/2, 1-ring search; 1: R_NL <= L_C, 2-ring search */
  int32_t ring;            /* 0 = derived from cap_mode; >0 forces the search ring (planted  */
                           /*     mistake for the negative test of the cap reading)          */
  int32_t fixed_interval;  /* period for ORC_FIXED_INTERVAL                                   */
  int32_t check_superset;  /* 1: every step, count brute-force contacts missing from the list */
  int32_t validity_uses_uncapped_skin; /* planted mistake for a negative test; 0 normally    */
  int32_t v_in_is_half_step; /* 1: v_in is a half-step velocity v^{n-1/2} (a resumed run): */
                             /*    the first step applies both half kicks                  */
  int32_t state_fp32;      /* 1: positions and velocities are rounded to FP32 after every     */
                           /*    step (a variant for the precision test; 0 normally)         */
  double K, dt, cell_size, skin_uniform, eps;
  double lo[3], hi[3];     /* box; a planar wall on each of the six faces                     */
  double kn, gamma_n;      /* normal linear spring-dashpot                                    */
  double g[3];             /* gravity acceleration                                            */
  int32_t n_planes;        /* planar walls besides the six box faces, 0..ORC_MAX_PLANES      */
  int32_t pad2_;
  double planes[ORC_MAX_PLANES][5]; /* (n_x, n_y, n_z, d, z_min): unit normal n into the      */
                           /*     domain; the wall fills n.x < d and acts on particles whose  */
                           /*     centre has z > z_min (a finite wall, e.g. a hopper side)     */
  double kt, gamma_t, mu;  /* tangential spring, tangential dashpot, Coulomb coefficient of   */
                           /*     particle-particle friction; all 0 = frictionless            */
  int32_t n_cylinders;     /* vertical cylindrical walls, 0..ORC_MAX_CYLINDERS               */
  int32_t pad3_;
  double cylinders[ORC_MAX_CYLINDERS][4]; /* (c_x, c_y, R, z_min): the domain is the inside  */
                           /*     of the cylinder of radius R about the vertical line through */
                           /*     (c_x, c_y); the wall acts on centres with z > z_min         */
} orc_params;

typedef struct {
  int32_t step;            /* n: the state x^n whose forces this record describes            */
  int32_t rebuilt;         /* 1 if a broad phase ran at x^n                                   */
  int64_t list_pairs;      /* unique pairs in the Verlet list used at x^n                    */
  int64_t contacts;        /* unique pairs with delta > 0 at x^n                             */
  int64_t violators;       /* particles with |x^{n+1} - x0| > skin_eff after this step      */
  int64_t missed;          /* contacts at x^n absent from the list (check_superset only)     */
  double max_excess;       /* max_p (|x^{n+1}_p - x0_p| - skin_eff_p)                        */
  double kinetic_energy;   /* sum_p m_p |v^n_p|^2 / 2                                        */
} orc_record;

/* Threads for the loops over particles (default 1).  Every result is bit-identical
 * whatever the count. */
void orc_set_threads(int n);
int orc_get_threads(void);

/* Broad phase by brute force: every pair i<j with |x_i - x_j| <= r_i + r_j + eps.
 * Writes up to cap pairs (int32 i, j) in lexicographic order; returns the count. */
int64_t orc_broadphase_brute(int64_t n, const double *x, const double *r, double eps,
                             int32_t *pairs, int64_t cap);

/* Broad phase by Alg. 1 (linked cells).  Cells of edge >= cell_edge_min tile
 * [lo,hi]; each cell is checked against the cells within `ring` cells of it
 * (its Moore neighbourhood for ring = 1) of smaller index, and against itself
 * for particle pairs of smaller index.  Same output convention as above. */
int64_t orc_broadphase_linked_cell(int64_t n, const double *x, const double *r, double eps,
                                   const double *lo, const double *hi, double cell_edge_min,
                                   int32_t ring, int32_t *pairs, int64_t cap);

/* Contact set by brute force: pairs i<j with delta = rc_i + rc_j - |x_i - x_j| > 0. */
int64_t orc_contacts_brute(int64_t n, const double *x, const double *rc, int32_t *pairs,
                           int64_t cap);

/* Extended radii at a broad phase: skin from the mode, R_NL capped, skin_eff = R_NL - R_C.
 * Returns 0, or -1 if some R_C exceeds the cap. */
int orc_rebuild_radii(const orc_params *p, int64_t n, const double *v, const double *rc,
                      double *rnl, double *skin_eff);

/* Forces on every particle from a canonical sorted contact list: pair terms summed
 * in ascending partner index, then the six walls, in the order -x,+x,-y,+y,-z,+z,
 * then the planar walls in index order.  Gravity is not included (it is added as
 * an acceleration by the integrator).  Normal forces only: the tangential
 * (friction) term needs the contact history that orc_run keeps. */
int orc_forces(const orc_params *p, int64_t n, const double *x, const double *v,
               const double *rc, int64_t ncontacts, const int32_t *contacts, double *F);

/* Run n_steps steps from (x_in, v_in) where v_in is the full-step velocity v^0
 * (or the half-step velocity v^{n-1/2} when v_in_is_half_step is set).
 * Outputs x^S and the half-step velocity v^{S-1/2} (v^0 if n_steps == 0).
 * hist (n_steps records) and the final list (list_out, cap, *list_n) are optional.
 * Returns 0, -1 bad parameters, -2 out of memory, -3 list_out too small. */
int orc_run(const orc_params *p, int64_t n, const double *x_in, const double *v_in,
            const double *rc, const double *invm, int32_t n_steps, double *x_out,
            double *v_out, orc_record *hist, int32_t *list_out, int64_t list_cap,
            int64_t *list_n);

/* Tangential springs of the last step's contacts (friction on): for particle i,
 * entries off[i] .. off[i+1]-1 hold its partners j (ascending) and the spring
 * xi (3 doubles each) of the pair as seen from i.  off has n + 1 entries; j and
 * xi hold cap entries; n is set to the number of entries. */
typedef struct {
  int64_t *off;
  int32_t *j;
  double *xi;
  int64_t cap;
  int64_t n;
} orc_springs;

/* orc_run that also exports the springs (spr may be NULL); -3 when they do
 * not fit in spr->cap entries (spr->n then holds the count). */
int orc_run_springs(const orc_params *p, int64_t n, const double *x_in, const double *v_in,
                    const double *rc, const double *invm, int32_t n_steps, double *x_out,
                    double *v_out, orc_record *hist, int32_t *list_out, int64_t list_cap,
                    int64_t *list_n, orc_springs *spr);

#endif
