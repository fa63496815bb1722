/*
 * orc.c -- FP64 CPU oracle for the local Verlet buffer DEM step.
 *
 * TEST INFRASTRUCTURE ONLY: used by the test suite, the smoke check and the CPU
 * baseline leg of the benchmark; never by the product path.  Plain and slow on
 * purpose (its loops over particles may use several host threads, with results
 * bit-identical to one thread).  Every function below names the passage of the
 * paper (Mainassara Checkaraou et al., local Verlet buffer for DEM) it follows.
 *
 * Readings taken where the paper is silent or ambiguous (each is listed with its
 * reason in the design notes of the repository):
 *   R1  v_p in skin_p = K v_p dt is the speed |v_p|.
 *   R2  skins are evaluated at a broad phase only, from the latest velocity
 *       available there (the half-step velocity v^{n-1/2}; v^0 at n = 0), and
 *       stay frozen until the next broad phase.
 *   R3  the cap: cap_mode 0 bounds R_NL by L_C/2 so that R_NL,i + R_NL,j <= L_C
 *       and the one-ring cell search of Alg. 1 is complete; cap_mode 1 takes the
 *       bound R_NL <= L_C literally and then needs a two-ring search.
 *   R4  the validity test compares the displacement with skin_eff = R_NL - R_C,
 *       the skin after the cap (the proof of the theorem needs R_NL = R_C + skin).
 *   R5  Alg. 1 also pairs particles inside the same cell (P_b before P_a), and
 *       the neighbour cells of Alg. 1 are the 26 Moore neighbours.
 *   R6  inequalities exactly as printed: broad phase <=, contact iff delta > 0,
 *       list invalid iff displacement > skin.
 *   R7  a broad phase always runs at step 0.
 *   R10 the broad-phase inclusion test is inflated by an absolute eps.
 *   R12 the contact law is a normal linear spring-dashpot (Sec. 5.1 names the
 *       model, not its constants, which are inputs here), against particles and
 *       against the walls (box faces, planar and cylindrical walls) alike.
 *   R13 the dashpot uses the half-step velocity available when forces are evaluated.
 *   R14 the forces on a particle are summed in ascending partner index, then
 *       the box faces (-x, +x, -y, +y, -z, +z), then the planar walls in order,
 *       then the cylindrical walls in order, so that the sum does not depend on
 *       what the Verlet list holds.
 *   R16 friction, when on, is a translational tangential spring-dashpot capped
 *       by Coulomb's law, with a spring per contact that starts at zero when the
 *       contact forms (Sec. 5.1 names static friction without its form).
 */
#include "orc.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Threads.  Loops over particles whose iterations are independent may run on
 * several threads; every result is the same as on one thread, bit for bit:
 * each iteration writes only its own particle, a list is built as pieces of
 * consecutive iterations joined in iteration order (or sorted afterwards),
 * maxima and counts are order-free, and the one sum (the kinetic energy) is
 * taken in particle order on one thread. */
static int g_threads = 1;
/* smallest loop that runs on several threads: below it one thread is faster */
#define ORC_PAR_MIN 16384

void orc_set_threads(int n) { g_threads = n < 1 ? 1 : n; }

int orc_get_threads(void) { return g_threads; }

/* ------------------------------------------------------------------ helpers */

static double dist3(const double *a, const double *b) {
  double dx = a[0] - b[0], dy = a[1] - b[1], dz = a[2] - b[2];
  return sqrt(dx * dx + dy * dy + dz * dz);
}

static double norm3(const double *a) { return sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]); }

static int cmp_pair(const void *pa, const void *pb) {
  const int32_t *a = (const int32_t *)pa, *b = (const int32_t *)pb;
  if (a[0] != b[0]) return a[0] < b[0] ? -1 : 1;
  if (a[1] != b[1]) return a[1] < b[1] ? -1 : 1;
  return 0;
}

/* A growable array of (i, j) pairs. */
typedef struct {
  int32_t *p;
  int64_t n, cap;
  int oom;
} pairvec;

static void pv_push(pairvec *v, int32_t i, int32_t j) {
  if (v->oom) return;
  if (v->n == v->cap) {
    int64_t nc = v->cap ? 2 * v->cap : 1024;
    int32_t *np = (int32_t *)realloc(v->p, (size_t)nc * 2 * sizeof(int32_t));
    if (!np) {
      v->oom = 1;
      return;
    }
    v->p = np;
    v->cap = nc;
  }
  v->p[2 * v->n] = i;
  v->p[2 * v->n + 1] = j;
  v->n++;
}

/* Appends the pieces a[0..np) to v in order and frees them. */
static void pv_join(pairvec *v, pairvec *a, int np) {
  for (int t = 0; t < np; t++) {
    if (a[t].oom) v->oom = 1;
    for (int64_t k = 0; k < a[t].n; k++) pv_push(v, a[t].p[2 * k], a[t].p[2 * k + 1]);
    free(a[t].p);
  }
}

static int64_t pv_export(const pairvec *v, int32_t *out, int64_t cap) {
  if (out) {
    int64_t m = v->n < cap ? v->n : cap;
    memcpy(out, v->p, (size_t)m * 2 * sizeof(int32_t));
  }
  return v->n;
}

/* ----------------------------------------------- broad phase, brute force */

/* All pairs, the O(n^2) approach the paper lists among broad-phase algorithms
 * (Sec. 1).  Inclusion test of Alg. 1: |X_a - X_b| <= r_a + r_b (plus eps, R10). */
static void broad_brute(int64_t n, const double *x, const double *r, double eps, pairvec *out) {
  for (int64_t i = 0; i < n; i++)
    for (int64_t j = i + 1; j < n; j++)
      if (dist3(x + 3 * i, x + 3 * j) <= r[i] + r[j] + eps) pv_push(out, (int32_t)i, (int32_t)j);
}

int64_t orc_broadphase_brute(int64_t n, const double *x, const double *r, double eps,
                             int32_t *pairs, int64_t cap) {
  pairvec v = {0};
  broad_brute(n, x, r, eps, &v);
  int64_t m = v.oom ? -2 : pv_export(&v, pairs, cap);
  free(v.p);
  return m;
}

/* ----------------------------------------------- broad phase, linked cells */

/* Alg. 1 (Sec. 3.2): uniform decomposition of the domain into cells; for every
 * cell C_a and every neighbour cell C_b of smaller index, every particle pair
 * (P_a, P_b) whose bounding spheres intersect is added to the list.  Pairs inside
 * one cell are checked once with P_b < P_a (R5).  Cells are not smaller than
 * cell_edge_min along any axis (Sec. 3.2: not smaller than the largest bounding
 * sphere).  Coordinates outside [lo, hi] are clamped to the border cells. */
static int broad_linked_cell(int64_t n, const double *x, const double *r, double eps,
                             const double *lo, const double *hi, double cell_edge_min,
                             int32_t ring, pairvec *out) {
  int64_t nc[3];
  double edge[3];
  for (int a = 0; a < 3; a++) {
    double len = hi[a] - lo[a];
    int64_t k = (int64_t)floor(len / cell_edge_min);
    nc[a] = k < 1 ? 1 : k;
    edge[a] = len / (double)nc[a];
  }
  int64_t ncell = nc[0] * nc[1] * nc[2];
  int64_t *cell = (int64_t *)malloc((size_t)(n ? n : 1) * sizeof(int64_t));
  int64_t *start = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
  int64_t *fill = (int64_t *)calloc((size_t)ncell + 1, sizeof(int64_t));
  int64_t *member = (int64_t *)malloc((size_t)(n ? n : 1) * sizeof(int64_t));
  if (!cell || !start || !fill || !member) {
    free(cell), free(start), free(fill), free(member);
    return -2;
  }
  for (int64_t i = 0; i < n; i++) {
    int64_t c[3];
    for (int a = 0; a < 3; a++) {
      double f = floor((x[3 * i + a] - lo[a]) / edge[a]);
      int64_t k = f < 0 ? 0 : (f > (double)(nc[a] - 1) ? nc[a] - 1 : (int64_t)f);
      c[a] = k;
    }
    cell[i] = (c[2] * nc[1] + c[1]) * nc[0] + c[0];
    start[cell[i] + 1]++;
  }
  for (int64_t c = 0; c < ncell; c++) start[c + 1] += start[c];
  /* members of each cell in ascending particle index */
  for (int64_t i = 0; i < n; i++) member[start[cell[i]] + fill[cell[i]]++] = i;

  /* every thread collects the pairs of its own cells; the list is sorted below */
  pairvec *part = (pairvec *)calloc((size_t)g_threads, sizeof(pairvec));
  if (!part) {
    free(cell), free(start), free(fill), free(member);
    return -2;
  }
#pragma omp parallel for collapse(2) schedule(dynamic) num_threads(g_threads) if (n >= ORC_PAR_MIN)
  for (int64_t cz = 0; cz < nc[2]; cz++)
    for (int64_t cy = 0; cy < nc[1]; cy++)
      for (int64_t cx = 0; cx < nc[0]; cx++) {
#ifdef _OPENMP
        pairvec *mine = &part[omp_get_thread_num()];
#else
        pairvec *mine = &part[0];
#endif
        int64_t ca = (cz * nc[1] + cy) * nc[0] + cx;
        for (int64_t dz = -ring; dz <= ring; dz++)
          for (int64_t dy = -ring; dy <= ring; dy++)
            for (int64_t dx = -ring; dx <= ring; dx++) {
              int64_t bx = cx + dx, by = cy + dy, bz = cz + dz;
              if (bx < 0 || by < 0 || bz < 0 || bx >= nc[0] || by >= nc[1] || bz >= nc[2])
                continue;
              int64_t cb = (bz * nc[1] + by) * nc[0] + bx;
              if (cb > ca) continue; /* each pair of cells once: index(C_b) < index(C_a) */
              for (int64_t ia = start[ca]; ia < start[ca + 1]; ia++) {
                int64_t pa = member[ia];
                for (int64_t ib = start[cb]; ib < start[cb + 1]; ib++) {
                  int64_t pb = member[ib];
                  if (cb == ca && pb >= pa) continue; /* same cell: P_b < P_a */
                  if (dist3(x + 3 * pa, x + 3 * pb) <= r[pa] + r[pb] + eps) {
                    int64_t i = pa < pb ? pa : pb, j = pa < pb ? pb : pa;
                    pv_push(mine, (int32_t)i, (int32_t)j);
                  }
                }
              }
            }
      }
  pv_join(out, part, g_threads);
  free(part);
  free(cell), free(start), free(fill), free(member);
  if (out->oom) return -2;
  qsort(out->p, (size_t)out->n, 2 * sizeof(int32_t), cmp_pair);
  return 0;
}

int64_t orc_broadphase_linked_cell(int64_t n, const double *x, const double *r, double eps,
                                   const double *lo, const double *hi, double cell_edge_min,
                                   int32_t ring, int32_t *pairs, int64_t cap) {
  pairvec v = {0};
  int rc = broad_linked_cell(n, x, r, eps, lo, hi, cell_edge_min, ring, &v);
  int64_t m = rc < 0 ? rc : pv_export(&v, pairs, cap);
  free(v.p);
  return m;
}

/* ----------------------------------------------------- narrow phase, naive */

/* Overlap of two spheres, Eq. delta (Sec. 3.2): delta = r_i + r_j - |X_i - X_j|. */
static double overlap(const double *xi, const double *xj, double ri, double rj) {
  return ri + rj - dist3(xi, xj);
}

/* The contact set by definition: every pair whose overlap exceeds zero (Eq. delta,
 * Sec. 3.2: such a pair collides, one with zero or negative overlap does not). */
static void contacts_brute(int64_t n, const double *x, const double *rc, pairvec *out) {
  int np = g_threads;
  pairvec *part = (pairvec *)calloc((size_t)np, sizeof(pairvec));
  if (!part) {
    out->oom = 1;
    return;
  }
  /* piece t holds the pairs of the particles i in [t n / np, (t+1) n / np) */
#pragma omp parallel for schedule(static, 1) num_threads(np) if (n >= 512)
  for (int t = 0; t < np; t++)
    for (int64_t i = t * n / np; i < (t + 1) * n / np; i++)
      for (int64_t j = i + 1; j < n; j++)
        if (overlap(x + 3 * i, x + 3 * j, rc[i], rc[j]) > 0.0) pv_push(&part[t], (int32_t)i, (int32_t)j);
  pv_join(out, part, np);
  free(part);
}

int64_t orc_contacts_brute(int64_t n, const double *x, const double *rc, int32_t *pairs,
                           int64_t cap) {
  pairvec v = {0};
  contacts_brute(n, x, rc, &v);
  int64_t m = v.oom ? -2 : pv_export(&v, pairs, cap);
  free(v.p);
  return m;
}

/* ------------------------------------------------------------- extended radii */

static double cap_of(const orc_params *p) {
  /* Eq. skin_formulus_mincell bounds R_NL by the cell size; R3 for the half. */
  return p->cap_mode == 0 ? 0.5 * p->cell_size : p->cell_size;
}

/* Eq. skin_formulus1 (local skin), Eq. bounding_sphere (R_NL = R_C + skin) and
 * Eq. skin_formulus_mincell (cap by the cell size). */
int orc_rebuild_radii(const orc_params *p, int64_t n, const double *v, const double *rc,
                      double *rnl, double *skin_eff) {
  double cap = cap_of(p);
  int bad = 0;
#pragma omp parallel for reduction(|| : bad) num_threads(g_threads) if (n >= ORC_PAR_MIN)
  for (int64_t i = 0; i < n; i++) {
    double skin;
    switch (p->skin_mode) {
      case ORC_SKIN_LOCAL: skin = p->K * norm3(v + 3 * i) * p->dt; break;
      case ORC_SKIN_UNIFORM:
      case ORC_FIXED_INTERVAL: skin = p->skin_uniform; break;
      default: skin = 0.0; break; /* no buffer: R_NL = R_C */
    }
    if (rc[i] > cap) bad = 1;
    double r = rc[i] + skin;
    rnl[i] = r < cap ? r : cap;
    skin_eff[i] = rnl[i] - rc[i];
  }
  return bad ? -1 : 0;
}

/* --------------------------------------------------------------------- forces */

/* History of the tangential springs: for every particle i, its contacts of
 * the previous step, partner index ascending, with the spring elongation xi of
 * the pair as seen from i (i's partner holds the opposite vector). */
typedef struct {
  int64_t *off; /* [n + 1] */
  int32_t *j;
  double *xi;   /* 3 per entry */
  int64_t cap;
} history;

static int friction_on(const orc_params *p) {
  return p->mu > 0.0 && (p->kt > 0.0 || p->gamma_t > 0.0);
}

/* The pair and wall forces of one step.  With a history (friction on), each
 * contact also gets the tangential linear spring-dashpot with a Coulomb limit
 * (the "LSD" law with static friction named in Sec. 5.1, translational part):
 *   xi <- xi_old projected on the tangent plane + v_t dt,
 *   F_t = -kt xi - gamma_t v_t, capped at mu max(F_n, 0), xi then set to the
 *   elongation of the capped force;
 * a contact absent from the previous step starts with xi = 0, and the new
 * history holds exactly this step's contacts. */
static int forces_core(const orc_params *p, int64_t n, const double *x, const double *v,
                       const double *rc, int64_t ncontacts, const int32_t *contacts, double *F,
                       const history *old, history *neu) {
  int64_t *deg = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  int32_t *adj = (int32_t *)malloc((size_t)(2 * ncontacts + 1) * sizeof(int32_t));
  int64_t *fill = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  if (!deg || !adj || !fill) {
    free(deg), free(adj), free(fill);
    return -2;
  }
  for (int64_t k = 0; k < ncontacts; k++) {
    deg[contacts[2 * k] + 1]++;
    deg[contacts[2 * k + 1] + 1]++;
  }
  for (int64_t i = 0; i < n; i++) deg[i + 1] += deg[i];
  for (int64_t k = 0; k < ncontacts; k++) {
    int32_t i = contacts[2 * k], j = contacts[2 * k + 1];
    adj[deg[i] + fill[i]++] = j;
    adj[deg[j] + fill[j]++] = i;
  }
#pragma omp parallel for num_threads(g_threads) if (n >= ORC_PAR_MIN)
  for (int64_t i = 0; i < n; i++) { /* ascending partner order (insertion sort) */
    for (int64_t a = deg[i] + 1; a < deg[i + 1]; a++) {
      int32_t key = adj[a];
      int64_t b = a - 1;
      while (b >= deg[i] && adj[b] > key) {
        adj[b + 1] = adj[b];
        b--;
      }
      adj[b + 1] = key;
    }
  }
  if (neu) {
    if (neu->cap < 2 * ncontacts + 1) {
      int32_t *nj = (int32_t *)realloc(neu->j, (size_t)(2 * ncontacts + 1) * sizeof(int32_t));
      double *nx = (double *)realloc(neu->xi, (size_t)(2 * ncontacts + 1) * 3 * sizeof(double));
      if (nj) neu->j = nj;
      if (nx) neu->xi = nx;
      if (!nj || !nx) {
        free(deg), free(adj), free(fill);
        return -2;
      }
      neu->cap = 2 * ncontacts + 1;
    }
    memcpy(neu->off, deg, (size_t)(n + 1) * sizeof(int64_t));
  }
#pragma omp parallel for num_threads(g_threads) if (n >= ORC_PAR_MIN)
  for (int64_t i = 0; i < n; i++) {
    const double *xi = x + 3 * i, *vi = v + 3 * i;
    double f[3] = {0.0, 0.0, 0.0};
    int64_t h = old ? old->off[i] : 0, h_end = old ? old->off[i + 1] : 0;
    for (int64_t a = deg[i]; a < deg[i + 1]; a++) {
      int64_t j = adj[a];
      const double *xj = x + 3 * j, *vj = v + 3 * j;
      double d = dist3(xi, xj);
      double delta = rc[i] + rc[j] - d;
      double nrm[3] = {(xi[0] - xj[0]) / d, (xi[1] - xj[1]) / d, (xi[2] - xj[2]) / d};
      double vn = (vi[0] - vj[0]) * nrm[0] + (vi[1] - vj[1]) * nrm[1] + (vi[2] - vj[2]) * nrm[2];
      double fm = p->kn * delta - p->gamma_n * vn;
      f[0] += fm * nrm[0];
      f[1] += fm * nrm[1];
      f[2] += fm * nrm[2];
      if (neu) {
        double s[3] = {0.0, 0.0, 0.0}; /* the pair's spring from the previous step, if any */
        while (h < h_end && old->j[h] < j) h++;
        if (h < h_end && old->j[h] == j)
          for (int c = 0; c < 3; c++) s[c] = old->xi[3 * h + c];
        double vt[3], sn = s[0] * nrm[0] + s[1] * nrm[1] + s[2] * nrm[2];
        for (int c = 0; c < 3; c++) {
          vt[c] = (vi[c] - vj[c]) - vn * nrm[c];
          s[c] = (s[c] - sn * nrm[c]) + vt[c] * p->dt;
        }
        double ft[3], ftn = 0.0;
        for (int c = 0; c < 3; c++) {
          ft[c] = -p->kt * s[c] - p->gamma_t * vt[c];
          ftn += ft[c] * ft[c];
        }
        ftn = sqrt(ftn);
        double lim = p->mu * (fm > 0.0 ? fm : 0.0);
        if (ftn > lim) { /* sliding: the force on the cone, the spring that gives it */
          double sc = lim / ftn;
          for (int c = 0; c < 3; c++) {
            ft[c] *= sc;
            s[c] = p->kt > 0.0 ? -(ft[c] + p->gamma_t * vt[c]) / p->kt : 0.0;
          }
        }
        f[0] += ft[0];
        f[1] += ft[1];
        f[2] += ft[2];
        neu->j[a] = (int32_t)j;
        for (int c = 0; c < 3; c++) neu->xi[3 * a + c] = s[c];
      }
    }
    for (int ax = 0; ax < 3; ax++) {
      double dlo = rc[i] - (xi[ax] - p->lo[ax]); /* wall at lo, normal +e_ax */
      if (dlo > 0.0) f[ax] += p->kn * dlo - p->gamma_n * vi[ax];
      double dhi = rc[i] - (p->hi[ax] - xi[ax]); /* wall at hi, normal -e_ax */
      if (dhi > 0.0) f[ax] -= p->kn * dhi - p->gamma_n * (-vi[ax]);
    }
    /* planar walls: the same law against a half-space of infinite mass at rest,
     * overlap = R_C minus the signed distance of the centre from the plane */
    for (int w = 0; w < p->n_planes; w++) {
      const double *pl = p->planes[w];
      if (!(xi[2] > pl[4])) continue;
      double s = pl[0] * xi[0] + pl[1] * xi[1] + pl[2] * xi[2] - pl[3];
      double delta = rc[i] - s;
      if (delta > 0.0) {
        double vn = vi[0] * pl[0] + vi[1] * pl[1] + vi[2] * pl[2];
        double fm = p->kn * delta - p->gamma_n * vn;
        f[0] += fm * pl[0];
        f[1] += fm * pl[1];
        f[2] += fm * pl[2];
      }
    }
    /* vertical cylindrical walls (a silo): the same law against the inside of a
     * cylinder; the centre lies rho from the axis, so R - rho from the wall, and
     * the wall pushes towards the axis.  A centre on the axis has no normal. */
    for (int w = 0; w < p->n_cylinders; w++) {
      const double *cyl = p->cylinders[w];
      if (!(xi[2] > cyl[3])) continue;
      double ex = xi[0] - cyl[0];
      double ey = xi[1] - cyl[1];
      double rho = sqrt(ex * ex + ey * ey);
      double delta = rc[i] - (cyl[2] - rho);
      if (delta > 0.0 && rho > 0.0) {
        double nx = -ex / rho;
        double ny = -ey / rho;
        double vn = vi[0] * nx + vi[1] * ny;
        double fm = p->kn * delta - p->gamma_n * vn;
        f[0] += fm * nx;
        f[1] += fm * ny;
      }
    }
    F[3 * i] = f[0];
    F[3 * i + 1] = f[1];
    F[3 * i + 2] = f[2];
  }
  free(deg), free(adj), free(fill);
  return 0;
}

/* Linear spring-dashpot (Sec. 5.1) on the contact pairs (i < j), normal part:
 * pair terms summed in ascending partner index, then the walls -x,+x,-y,+y,-z,+z,
 * then the planar walls, then the cylindrical walls. */
int orc_forces(const orc_params *p, int64_t n, const double *x, const double *v,
               const double *rc, int64_t ncontacts, const int32_t *contacts, double *F) {
  return forces_core(p, n, x, v, rc, ncontacts, contacts, F, NULL, NULL);
}

/* ------------------------------------------------------------------- the run */

static int pair_in(const pairvec *L, int32_t i, int32_t j) {
  int64_t a = 0, b = L->n - 1;
  while (a <= b) {
    int64_t m = (a + b) / 2;
    const int32_t *q = L->p + 2 * m;
    if (q[0] == i && q[1] == j) return 1;
    if (q[0] < i || (q[0] == i && q[1] < j)) a = m + 1;
    else b = m - 1;
  }
  return 0;
}

/* One run of the time loop of Sec. 3.1 with the Verlet check of Sec. 4
 * (flow chart of the modified code): at each step n,
 *   1. decide whether the list is still valid (Eq. update; Def. autoverlet),
 *   2. if not (or n = 0, R7), broad phase on the extended spheres (Alg. 1 with
 *      Eq. bounding_sphere, skin_formulus1, skin_formulus_mincell),
 *   3. narrow phase on the list (Eq. delta),
 *   4. forces (linear spring-dashpot, walls, gravity),
 *   5. velocity-Verlet integration:
 *        v^n     = v^{n-1/2} + dt/2 a^n        (skipped at n = 0, where v^0 is given)
 *        v^{n+1/2} = v^n + dt/2 a^n,   x^{n+1} = x^n + dt v^{n+1/2},
 *   6. displacement of every particle since the last broad phase, a straight
 *      line (Sec. 2), compared with its skin for step n+1.
 * In ORC_NAIVE mode steps 1-2 are skipped and step 3 tests every pair. */
int orc_run(const orc_params *p, int64_t n, const double *x_in, const double *v_in,
            const double *rc, const double *invm, int32_t n_steps, double *x_out,
            double *v_out, orc_record *hist, int32_t *list_out, int64_t list_cap,
            int64_t *list_n) {
  return orc_run_springs(p, n, x_in, v_in, rc, invm, n_steps, x_out, v_out, hist, list_out,
                         list_cap, list_n, NULL);
}

int orc_run_springs(const orc_params *p, int64_t n, const double *x_in, const double *v_in,
                    const double *rc, const double *invm, int32_t n_steps, double *x_out,
                    double *v_out, orc_record *hist, int32_t *list_out, int64_t list_cap,
                    int64_t *list_n, orc_springs *spr) {
  if (n < 0 || n_steps < 0 || !(p->dt > 0.0) || !(p->cell_size > 0.0) || p->eps < 0.0) return -1;
  if (p->skin_mode == ORC_FIXED_INTERVAL && p->fixed_interval < 1) return -1;
  if (p->n_planes < 0 || p->n_planes > ORC_MAX_PLANES) return -1;
  if (p->n_cylinders < 0 || p->n_cylinders > ORC_MAX_CYLINDERS) return -1;
  for (int w = 0; w < p->n_cylinders; w++)
    if (!(p->cylinders[w][2] > 0.0)) return -1;
  int32_t ring = p->ring > 0 ? p->ring : (p->cap_mode == 0 ? 1 : 2);
  /* the smallest cell edge that keeps Alg. 1 complete for the chosen cap: every
     reach R_NL,i + R_NL,j + eps is at most ring * edge */
  double edge_min = p->cell_size * (1.0 + 1e-9) + p->eps;
  size_t n3 = (size_t)n * 3, a3 = n3 ? n3 : 3;
  double *x = (double *)malloc(a3 * sizeof(double));
  double *vh = (double *)malloc(a3 * sizeof(double));
  double *x0 = (double *)calloc(a3, sizeof(double));
  double *F = (double *)malloc(a3 * sizeof(double));
  double *rnl = (double *)calloc((size_t)(n ? n : 1), sizeof(double));
  double *skin_eff = (double *)calloc((size_t)(n ? n : 1), sizeof(double));
  double *skin_test = (double *)calloc((size_t)(n ? n : 1), sizeof(double));
  double *kin = (double *)calloc((size_t)(n ? n : 1), sizeof(double));
  pairvec L = {0}, C = {0}, B = {0};
  history H[2] = {{0}, {0}};
  const int fric = friction_on(p);
  int cur_h = 0;
  int ret = 0;
  if (fric) {
    for (int b = 0; b < 2; b++) H[b].off = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!H[0].off || !H[1].off) {
      ret = -2;
      goto done;
    }
  }
  if (!x || !vh || !x0 || !F || !rnl || !skin_eff || !skin_test || !kin) {
    ret = -2;
    goto done;
  }
  memcpy(x, x_in, n3 * sizeof(double));
  memcpy(vh, v_in, n3 * sizeof(double));
  int violated = 0;
  int64_t list_pairs = 0;
  for (int32_t step = 0; step < n_steps; step++) {
    /* 1-2. validity and broad phase */
    int rebuild = 0;
    if (p->skin_mode == ORC_NAIVE) rebuild = 0;
    else if (p->skin_mode == ORC_NO_BUFFER) rebuild = 1;
    else if (p->skin_mode == ORC_FIXED_INTERVAL) rebuild = (step % p->fixed_interval) == 0;
    else rebuild = (step == 0) || violated;
    if (rebuild) {
      if (orc_rebuild_radii(p, n, vh, rc, rnl, skin_eff) != 0) {
        ret = -1;
        goto done;
      }
      for (int64_t i = 0; i < n; i++) {
        skin_test[i] = skin_eff[i]; /* R4 */
        if (p->validity_uses_uncapped_skin && p->skin_mode == ORC_SKIN_LOCAL)
          skin_test[i] = p->K * norm3(vh + 3 * i) * p->dt; /* planted mistake */
      }
      memcpy(x0, x, n3 * sizeof(double));
      L.n = 0;
      if (broad_linked_cell(n, x, rnl, p->eps, p->lo, p->hi, edge_min, ring, &L) != 0) {
        ret = -2;
        goto done;
      }
      list_pairs = L.n;
    }
    /* 3. narrow phase */
    C.n = 0;
    if (p->skin_mode == ORC_NAIVE) {
      contacts_brute(n, x, rc, &C);
    } else {
      /* piece t filters the list entries [t L.n / np, (t+1) L.n / np), joined in order */
      int np = g_threads;
      pairvec *part = (pairvec *)calloc((size_t)np, sizeof(pairvec));
      if (!part) {
        ret = -2;
        goto done;
      }
#pragma omp parallel for schedule(static, 1) num_threads(np) if (L.n >= ORC_PAR_MIN)
      for (int t = 0; t < np; t++) {
        pairvec *Ct = &part[t];
        for (int64_t k = t * L.n / np; k < (t + 1) * L.n / np; k++) {
          int32_t i = L.p[2 * k], j = L.p[2 * k + 1];
          if (overlap(x + 3 * i, x + 3 * j, rc[i], rc[j]) > 0.0) pv_push(Ct, i, j);
        }
      }
      pv_join(&C, part, np);
      free(part);
    }
    int64_t missed = 0;
    if (p->check_superset && p->skin_mode != ORC_NAIVE) {
      B.n = 0;
      contacts_brute(n, x, rc, &B);
      for (int64_t k = 0; k < B.n; k++)
        if (!pair_in(&L, B.p[2 * k], B.p[2 * k + 1])) missed++;
    }
    if (C.oom || B.oom) {
      ret = -2;
      goto done;
    }
    /* 4. forces */
    if (forces_core(p, n, x, vh, rc, C.n, C.p, F, fric ? &H[cur_h] : NULL,
                    fric ? &H[cur_h ^ 1] : NULL) != 0) {
      ret = -2;
      goto done;
    }
    cur_h ^= 1;
    /* 5. integration */
    double hdt = 0.5 * p->dt;
#pragma omp parallel for num_threads(g_threads) if (n >= ORC_PAR_MIN)
    for (int64_t i = 0; i < n; i++) {
      double vfull[3];
      for (int a = 0; a < 3; a++) {
        double acc = F[3 * i + a] * invm[i] + p->g[a];
        vfull[a] = (step == 0 && !p->v_in_is_half_step) ? vh[3 * i + a] : vh[3 * i + a] + hdt * acc;
        vh[3 * i + a] = vfull[a] + hdt * acc;
        x[3 * i + a] = x[3 * i + a] + p->dt * vh[3 * i + a];
      }
      kin[i] = 0.5 * (vfull[0] * vfull[0] + vfull[1] * vfull[1] + vfull[2] * vfull[2]) / invm[i];
      if (p->state_fp32)
        for (int a = 0; a < 3; a++) {
          x[3 * i + a] = (double)(float)x[3 * i + a];
          vh[3 * i + a] = (double)(float)vh[3 * i + a];
        }
    }
    double ke = 0.0;
    for (int64_t i = 0; i < n; i++) ke += kin[i]; /* in particle order */
    /* 6. displacement test for the next step */
    int64_t viol = 0;
    double max_excess = -INFINITY;
    if (p->skin_mode != ORC_NAIVE) {
#pragma omp parallel for reduction(max : max_excess) reduction(+ : viol) num_threads(g_threads) \
    if (n >= ORC_PAR_MIN)
      for (int64_t i = 0; i < n; i++) {
        double disp = dist3(x + 3 * i, x0 + 3 * i);
        double excess = disp - skin_test[i];
        if (excess > max_excess) max_excess = excess;
        if (disp > skin_test[i]) viol++;
      }
    }
    if (n == 0 || p->skin_mode == ORC_NAIVE) max_excess = 0.0;
    violated = viol > 0;
    if (hist) {
      orc_record *r = hist + step;
      r->step = step;
      r->rebuilt = rebuild;
      r->list_pairs = p->skin_mode == ORC_NAIVE ? 0 : list_pairs;
      r->contacts = C.n;
      r->violators = viol;
      r->missed = missed;
      r->max_excess = max_excess;
      r->kinetic_energy = ke;
    }
  }
  memcpy(x_out, x, n3 * sizeof(double));
  memcpy(v_out, vh, n3 * sizeof(double));
  if (spr) { /* the springs of the last step's contacts, as the next step would read them */
    spr->n = fric ? H[cur_h].off[n] : 0;
    if (spr->off) {
      if (fric) memcpy(spr->off, H[cur_h].off, (size_t)(n + 1) * sizeof(int64_t));
      else memset(spr->off, 0, (size_t)(n + 1) * sizeof(int64_t));
    }
    if (spr->n > spr->cap) ret = -3;
    else if (spr->n > 0 && spr->j && spr->xi) {
      memcpy(spr->j, H[cur_h].j, (size_t)spr->n * sizeof(int32_t));
      memcpy(spr->xi, H[cur_h].xi, (size_t)spr->n * 3 * sizeof(double));
    }
  }
  if (list_n) {
    *list_n = L.n;
    if (list_out) {
      if (L.n > list_cap) ret = -3;
      else memcpy(list_out, L.p, (size_t)L.n * 2 * sizeof(int32_t));
    }
  }
done:
  free(x), free(vh), free(x0), free(F), free(rnl), free(skin_eff), free(skin_test), free(kin);
  free(L.p), free(C.p), free(B.p);
  for (int b = 0; b < 2; b++) free(H[b].off), free(H[b].j), free(H[b].xi);
  return ret;
}
