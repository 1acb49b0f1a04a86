/*
 * DSMC oracle: a plain, sequential, FP64 implementation of one time step of
 * unsteady DSMC -- Generation, Motion, Enumeration/Indexing, Interaction and
 * Sampling -- in the order of the sequential algorithm of Sec. 1.1 (Fig. 1)
 * of Bogdanov, Bykov,
 * Grishin, Khanlarov, Lukianov and Zakharov, "Algorithms of Two-Level
 * Parallelization for DSMC of Unsteady Flows in Molecular Gasdynamics".
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke entry point and
 * the CPU-baseline leg of the benchmark may load this library.  It shares no
 * code, header, table or constant generator with the GPU library.
 *
 * What the paper fixes (Sec. 1.1): the step order; the particle array P
 * (coordinates, velocity); the readdressing array LCR built from the cell of
 * every particle after the particle stage; the cell array C; removal of
 * particles that leave the domain and insertion of generated ones each step;
 * runs made independent by shifting the random number generator.  The
 * kinetics the paper leaves to the DSMC literature it cites (Bird 1994) are
 * written here from the mathematics:
 *   - no-time-counter (NTC) pair selection with a per-cell remainder and an
 *     immediate update of (sigma*c_r)_max;
 *   - hard-sphere / variable-hard-sphere cross sections, isotropic scattering;
 *   - specular and diffuse (full accommodation) walls, vacuum outflow, and
 *     inflow of a drifting Maxwellian through the -x face;
 *   - an optional obstacle made of solid cells (voxels of the cell grid) with
 *     diffuse faces: the straight path is followed from cell to cell in the
 *     time order of its plane crossings (the voxel traversal of Amanatides
 *     and Woo, 1987) and the first solid cell it enters is hit on the face it
 *     crosses.
 * Random numbers come from the counter-based generator Philox4x32-10 of
 * Salmon, Moraes, Dror and Shaw (SC'11), written from its published
 * definition.  Build with -O2 -ffp-contract=off (no fast-math).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_BC_SPECULAR 0
#define OR_BC_DIFFUSE 1
#define OR_BC_INFLOW 2
#define OR_BC_OUTFLOW 3

#define OR_OK 0
#define OR_EINVAL -1
#define OR_ECAPACITY -3
#define OR_EBOUNCE -7
#define OR_EREJECT -8
#define OR_ENOMEM -9
#define OR_EUNSUPPORTED -6

#define PURPOSE_INIT 0u
#define PURPOSE_GEN 1u
#define PURPOSE_WALL 2u
#define PURPOSE_COLL 3u

#define MAX_WALL_HITS 64
#define MAX_GEN_ATTEMPTS 1000
/* Each inflow particle draws from its own stretch of its face element's
 * stream: particle k starts at uniform k * GEN_UNIFORMS (at most
 * 4 * MAX_GEN_ATTEMPTS + 5 are used), so particles are independent of one
 * another's rejections.  The 32-bit block counter bounds k below 2^21; runs
 * expecting 2^20 or more entrants per face element per step are refused. */
#define GEN_UNIFORMS 4096
#define MAX_GEN_PER_FACE 1048576.0
#define MAX_INIT_ATTEMPTS 100

static const double TWO_PI = 6.283185307179586476925286766559;
static const double SQRT_PI = 1.7724538509055160272981674833411;

typedef struct {
    int32_t dim, nx, ny, nz;
    double lx, ly, lz;
    double dt;
    double fnum_sigma;
    double omega, c_ref;
    int32_t face_bc[6];
    double face_T[6];
    double inflow_n, inflow_U, inflow_T;
    const uint8_t *solid;
    double solid_T;
    int64_t capacity;
    int64_t n_init;
    double init_U[3];
    double init_T;
    uint32_t run_id, seed;
    int32_t subcells;    /* collision partners from sub-cells: k per axis (0 or 1 = none) */
    int32_t pad;
    double nbar_alpha;   /* 0: NTC count from N(N-1)/2; in (0, 1]: from N * Nbar / 2, Nbar a running
                            mean of the cell's count with weight nbar_alpha */
} or_spec;

typedef struct {
    or_spec sp;
    int64_t nc;          /* cells */
    int64_t sub;         /* sub-cells per axis (1 = none) */
    int64_t S;           /* sub-cells per cell, sub^dim */
    int64_t nbin;        /* Indexing bins (sub-cells), nc * S; the DEAD bin is nbin */
    double inv_f[3];     /* sub-cells per unit length along each axis */
    int64_t nface;       /* inflow face elements, 0 without inflow */
    double L[3];
    double inv_d[3];     /* cells per unit length along each axis */
    double coef;         /* Fnum*sigma_ref*dt/V_c */
    double vhs_exp;      /* 1 - 2 omega */
    double gmax0;
    double mbar;         /* mean number entering through one face element per step */
    double beta, s_inf, p_branch, dy, dz;
    int64_t n;           /* particles in P */
    double *p[6];        /* x, y, z, u, v, w (z is 0 in 2-D) */
    double *q[6];        /* scratch for the permutation */
    int32_t *cell;       /* bin (sub-cell) of each slot after Motion (nbin = DEAD) */
    int32_t *lcr;        /* readdressing array */
    int64_t n_sorted;    /* number of entries of lcr (particles before removal) */
    int64_t *cstart;     /* nbin + 2 bin starts */
    int64_t *ccount;     /* nbin + 1 */
    double *rem_c, *gmax;
    double *nbar;        /* running mean of each cell's particle count (with nbar_alpha > 0) */
    int64_t *ncoll;
    double *rem_f;
    uint32_t step;
    int32_t err;
    int64_t last_ncoll, last_ngen, last_nremoved, last_nmoved;
    uint8_t *solid;      /* [nc] 1 = solid cell (copy of the spec's mask), or NULL */
    int has_solid;       /* at least one solid cell */
    int64_t last_nsolid; /* solid faces hit in the last Motion */
    double d[3];         /* cell size along each axis */
} or_run;

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon et al., SC'11)                                       */
/* ------------------------------------------------------------------------- */

void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Uniform in (0,1) from two 32-bit words: 52 random bits, centred. */
double or_u01(uint32_t a, uint32_t b)
{
    uint64_t m = ((uint64_t)a << 20) | (uint64_t)(b >> 12);
    return ((double)m + 0.5) * 0x1p-52;
}

/* Index in [0, n) from one 32-bit word. */
uint32_t or_index(uint32_t a, uint32_t n)
{
    return (uint32_t)(((uint64_t)a * (uint64_t)n) >> 32);
}

/* A stream of uniforms for one (key, step, purpose, index): uniform number k
 * comes from block k/2, words 2(k%2) and 2(k%2)+1. */
typedef struct {
    uint32_t key[2];
    uint32_t c0, c1, c2;
    uint64_t next;
} ustream;

static double us_next(ustream *s)
{
    uint32_t ctr[4] = {s->c0, s->c1, s->c2, (uint32_t)(s->next >> 1)};
    uint32_t blk[4];
    or_philox4x32_10(ctr, s->key, blk);
    int h = (int)(s->next & 1u);
    s->next++;
    return or_u01(blk[2 * h], blk[2 * h + 1]);
}

static void box_muller(double u1, double u2, double *n0, double *n1)
{
    double r = sqrt(-2.0 * log(u1));
    double th = TWO_PI * u2;
    *n0 = r * cos(th);
    *n1 = r * sin(th);
}

/* ------------------------------------------------------------------------- */
/* Run set-up                                                                 */
/* ------------------------------------------------------------------------- */

static int64_t axis_index(double x, double inv, int32_t n)
{
    double f = floor(x * inv);
    if (!(f > 0.0)) return 0;
    if (f >= (double)(n - 1)) return n - 1;
    return (int64_t)f;
}

static int64_t cell_of(const or_run *R, const double pos[3])
{
    int64_t ix = axis_index(pos[0], R->inv_d[0], R->sp.nx);
    int64_t iy = axis_index(pos[1], R->inv_d[1], R->sp.ny);
    int64_t iz = (R->sp.dim == 3) ? axis_index(pos[2], R->inv_d[2], R->sp.nz) : 0;
    return (iz * R->sp.ny + iy) * R->sp.nx + ix;
}

/* The Indexing bin of a position: its cell when there are no sub-cells;
 * otherwise the sub-cell grid (sub per axis) is indexed cell by cell, bin =
 * cell * S + (sz * sub + sy) * sub + sx, the cell being the sub-cell index
 * divided by sub along each axis. */
static int64_t bin_of(const or_run *R, const double pos[3])
{
    if (R->sub == 1) return cell_of(R, pos);
    const int64_t k = R->sub;
    int64_t fx = axis_index(pos[0], R->inv_f[0], (int32_t)(R->sp.nx * k));
    int64_t fy = axis_index(pos[1], R->inv_f[1], (int32_t)(R->sp.ny * k));
    int64_t fz = (R->sp.dim == 3) ? axis_index(pos[2], R->inv_f[2], (int32_t)(R->sp.nz * k)) : 0;
    int64_t c = ((fz / k) * R->sp.ny + fy / k) * R->sp.nx + fx / k;
    int64_t s = ((fz % k) * k + fy % k) * k + fx % k;
    return c * R->S + s;
}

/* g = sigma(c_r)/sigma_ref * c_r for HS / VHS. */
static double g_of(const or_run *R, double cr)
{
    if (R->sp.omega == 0.5) return cr;
    if (!(cr > 0.0)) return 0.0;
    return cr * pow(cr / R->sp.c_ref, R->vhs_exp);
}

void or_run_free(or_run *R)
{
    if (!R) return;
    for (int a = 0; a < 6; ++a) {
        free(R->p[a]);
        free(R->q[a]);
    }
    free(R->cell); free(R->lcr); free(R->cstart); free(R->ccount);
    free(R->rem_c); free(R->gmax); free(R->nbar); free(R->ncoll); free(R->rem_f);
    free(R->solid);
    free(R);
}

or_run *or_run_new(const or_spec *sp, int32_t *status)
{
    *status = OR_OK;
    if (sp->dim != 2 && sp->dim != 3) { *status = OR_EINVAL; return NULL; }
    if (sp->nx < 1 || sp->ny < 1 || sp->nz < 1 || (sp->dim == 2 && sp->nz != 1)) {
        *status = OR_EINVAL; return NULL;
    }
    if (!(sp->dt > 0.0) || sp->capacity < sp->n_init || sp->n_init < 0) {
        *status = OR_EINVAL; return NULL;
    }
    if (sp->solid && !(sp->solid_T > 0.0)) { *status = OR_EINVAL; return NULL; }
    for (int f = 0; f < 6; ++f) {
        int bc = sp->face_bc[f];
        if (bc < 0 || bc > 3) { *status = OR_EINVAL; return NULL; }
        if (bc == OR_BC_INFLOW && f != 0) { *status = OR_EINVAL; return NULL; }
    }
    if (sp->subcells < 0 || sp->subcells > 4) { *status = OR_EINVAL; return NULL; }
    if (sp->subcells > 1 && sp->solid) { *status = OR_EUNSUPPORTED; return NULL; }
    if (!(sp->nbar_alpha >= 0.0 && sp->nbar_alpha <= 1.0)) { *status = OR_EINVAL; return NULL; }
    or_run *R = (or_run *)calloc(1, sizeof(or_run));
    if (!R) { *status = OR_ENOMEM; return NULL; }
    R->sp = *sp;
    R->sp.solid = NULL;
    R->nc = (int64_t)sp->nx * sp->ny * sp->nz;
    R->sub = sp->subcells > 1 ? sp->subcells : 1;
    R->S = R->sub * R->sub * (sp->dim == 3 ? R->sub : 1);
    R->nbin = R->nc * R->S;
    R->inv_f[0] = (double)(sp->nx * R->sub) / sp->lx;
    R->inv_f[1] = (double)(sp->ny * R->sub) / sp->ly;
    R->inv_f[2] = (double)(sp->nz * R->sub) / sp->lz;
    R->L[0] = sp->lx; R->L[1] = sp->ly; R->L[2] = sp->lz;
    R->inv_d[0] = (double)sp->nx / sp->lx;
    R->inv_d[1] = (double)sp->ny / sp->ly;
    R->inv_d[2] = (double)sp->nz / sp->lz;
    R->d[0] = sp->lx / sp->nx;
    R->d[1] = sp->ly / sp->ny;
    R->d[2] = sp->lz / sp->nz;
    if (sp->solid) {
        R->solid = (uint8_t *)malloc((size_t)R->nc);
        if (!R->solid) { or_run_free(R); *status = OR_ENOMEM; return NULL; }
        for (int64_t c = 0; c < R->nc; ++c) {
            R->solid[c] = sp->solid[c] ? 1 : 0;
            if (R->solid[c]) R->has_solid = 1;
            /* inflow enters through the first layer of cells: it must be fluid */
            if (R->solid[c] && sp->face_bc[0] == OR_BC_INFLOW && c % sp->nx == 0) {
                or_run_free(R); *status = OR_EINVAL; return NULL;
            }
        }
    }
    double vc = (sp->lx / sp->nx) * (sp->ly / sp->ny) * (sp->lz / sp->nz);
    R->coef = sp->fnum_sigma * sp->dt / vc;
    R->vhs_exp = 1.0 - 2.0 * sp->omega;

    /* initial (sigma c_r)_max: g at c0 = |U| + 3 sqrt(2 T_max) */
    int inflow = (sp->face_bc[0] == OR_BC_INFLOW);
    double U0 = inflow ? sp->inflow_U : 0.0;
    double Ui = sqrt(sp->init_U[0] * sp->init_U[0] + sp->init_U[1] * sp->init_U[1] +
                     sp->init_U[2] * sp->init_U[2]);
    if (Ui > U0) U0 = Ui;
    double Tmax = sp->init_T;
    if (inflow && sp->inflow_T > Tmax) Tmax = sp->inflow_T;
    for (int f = 0; f < 2 * sp->dim; ++f)
        if (sp->face_bc[f] == OR_BC_DIFFUSE && sp->face_T[f] > Tmax) Tmax = sp->face_T[f];
    if (R->has_solid && sp->solid_T > Tmax) Tmax = sp->solid_T;
    double c0 = U0 + 3.0 * sqrt(2.0 * Tmax);
    R->gmax0 = g_of(R, c0);

    R->dy = sp->ly / sp->ny;
    R->dz = sp->lz / sp->nz;
    if (inflow) {
        R->nface = (int64_t)sp->ny * sp->nz;
        R->beta = 1.0 / sqrt(2.0 * sp->inflow_T);
        R->s_inf = sp->inflow_U * R->beta;
        R->p_branch = 1.0 / (1.0 + SQRT_PI * R->s_inf);
        double s = R->s_inf;
        double flux = sp->inflow_n / (2.0 * SQRT_PI * R->beta) *
                      (exp(-s * s) + SQRT_PI * s * (1.0 + erf(s)));
        R->mbar = flux * (R->dy * R->dz) * sp->dt;
        if (!(R->mbar < MAX_GEN_PER_FACE)) { or_run_free(R); *status = OR_EINVAL; return NULL; }
    }

    int64_t cap = sp->capacity > 0 ? sp->capacity : 1;
    for (int a = 0; a < 6; ++a) {
        R->p[a] = (double *)calloc((size_t)cap, sizeof(double));
        R->q[a] = (double *)calloc((size_t)cap, sizeof(double));
    }
    R->cell = (int32_t *)calloc((size_t)cap, sizeof(int32_t));
    R->lcr = (int32_t *)calloc((size_t)cap, sizeof(int32_t));
    R->cstart = (int64_t *)calloc((size_t)(R->nbin + 2), sizeof(int64_t));
    R->ccount = (int64_t *)calloc((size_t)(R->nbin + 1), sizeof(int64_t));
    R->rem_c = (double *)calloc((size_t)R->nc, sizeof(double));
    R->gmax = (double *)calloc((size_t)R->nc, sizeof(double));
    R->nbar = (double *)calloc((size_t)R->nc, sizeof(double));
    R->ncoll = (int64_t *)calloc((size_t)R->nc, sizeof(int64_t));
    R->rem_f = (double *)calloc((size_t)(R->nface > 0 ? R->nface : 1), sizeof(double));
    int ok = R->cell && R->lcr && R->cstart && R->ccount && R->rem_c && R->gmax && R->nbar &&
             R->ncoll && R->rem_f;
    for (int a = 0; a < 6; ++a) ok = ok && R->p[a] && R->q[a];
    if (!ok) { or_run_free(R); *status = OR_ENOMEM; return NULL; }
    /* the running mean starts at the expected count of the initial fill */
    for (int64_t c = 0; c < R->nc; ++c) {
        R->gmax[c] = R->gmax0;
        R->nbar[c] = (double)sp->n_init / (double)R->nc;
    }
    return R;
}

/* Initial uniform Maxwellian fill: slot i draws from (step 0, INIT, i).
 * Uniforms 0..3 give the three velocity normals (two Box-Muller pairs, the
 * last output unused), uniforms 4.. give the position: three at a time, drawn
 * again while the position lies in a solid cell (uniform over the fluid). */
void or_init(or_run *R)
{
    const or_spec *sp = &R->sp;
    double st = sqrt(sp->init_T);
    for (int64_t i = 0; i < sp->n_init; ++i) {
        ustream s = {{sp->run_id, sp->seed}, 0u, PURPOSE_INIT, (uint32_t)i, 0};
        double u0 = us_next(&s), u1 = us_next(&s), u2 = us_next(&s), u3 = us_next(&s);
        double n0, n1, n2, n3;
        box_muller(u0, u1, &n0, &n1);
        box_muller(u2, u3, &n2, &n3);
        (void)n3;
        R->p[3][i] = sp->init_U[0] + st * n0;
        R->p[4][i] = sp->init_U[1] + st * n1;
        R->p[5][i] = sp->init_U[2] + st * n2;
        double pos[3];
        for (int att = 0;; ++att) {
            if (att == MAX_INIT_ATTEMPTS) { R->err = OR_EREJECT; return; }
            double ux = us_next(&s), uy = us_next(&s), uz = us_next(&s);
            pos[0] = ux * sp->lx;
            pos[1] = uy * sp->ly;
            pos[2] = (sp->dim == 3) ? uz * sp->lz : 0.0;
            if (!R->has_solid || !R->solid[cell_of(R, pos)]) break;
        }
        R->p[0][i] = pos[0];
        R->p[1][i] = pos[1];
        R->p[2][i] = pos[2];
    }
    R->n = sp->n_init;
    R->step = 0;
}

/* ------------------------------------------------------------------------- */
/* Generation: inflow of a drifting Maxwellian through the -x face            */
/* ------------------------------------------------------------------------- */

void or_generation(or_run *R)
{
    const or_spec *sp = &R->sp;
    R->last_ngen = 0;
    if (R->nface == 0) return;
    double st = sqrt(sp->inflow_T);
    for (int64_t j = 0; j < R->nface; ++j) {
        double M = R->mbar + R->rem_f[j];
        double fl = floor(M);
        int64_t nemit = (int64_t)fl;
        R->rem_f[j] = M - fl;
        int64_t iy = j % sp->ny, iz = j / sp->ny;
        ustream s = {{sp->run_id, sp->seed}, R->step, PURPOSE_GEN, (uint32_t)j, 0};
        for (int64_t k = 0; k < nemit; ++k) {
            s.next = (uint64_t)k * GEN_UNIFORMS;
            /* normal velocity: z = beta*u has density ~ z exp(-(z-s)^2), z > 0 */
            double z = 0.0;
            int att;
            for (att = 0; att < MAX_GEN_ATTEMPTS; ++att) {
                double ub = us_next(&s), up = us_next(&s), uq = us_next(&s), ua = us_next(&s);
                double r = sqrt(-log(up));
                double x = (ub < R->p_branch) ? ((uq < 0.5) ? -r : r) : r * cos(TWO_PI * uq);
                z = R->s_inf + x;
                if (z > 0.0 && ua < z / (R->s_inf + fabs(x))) break;
            }
            if (att == MAX_GEN_ATTEMPTS) { R->err = OR_EREJECT; return; }
            double u = z / R->beta;
            double t0, t1;
            double v1 = us_next(&s), v2 = us_next(&s);
            box_muller(v1, v2, &t0, &t1);
            double y = ((double)iy + us_next(&s)) * R->dy;
            double zc = (sp->dim == 3) ? ((double)iz + us_next(&s)) * R->dz : 0.0;
            double ut = us_next(&s);
            double x0 = -(u * sp->dt) * (1.0 - ut);
            if (R->n >= sp->capacity) { R->err = OR_ECAPACITY; return; }
            int64_t d = R->n++;
            R->p[0][d] = x0; R->p[1][d] = y; R->p[2][d] = zc;
            R->p[3][d] = u; R->p[4][d] = st * t0; R->p[5][d] = st * t1;
            R->last_ngen++;
        }
    }
}

/* ------------------------------------------------------------------------- */
/* Motion + Enumeration                                                       */
/* ------------------------------------------------------------------------- */

static int64_t cell_at(const or_run *R, const int64_t v[3])
{
    return (v[2] * R->sp.ny + v[1]) * R->sp.nx + v[0];
}

/* Follows the straight path from pos (in cell vox) with velocity vel for a
 * time tlim, crossing cell planes in time order (ties: lower axis first).
 * Returns the axis of the face of the first solid cell entered and its time
 * in *th, or -1 if none is entered; vox follows the path up to that face (or
 * up to tlim).  A plane is at k * d (k = 0..n). */
static int solid_walk(const or_run *R, const double pos[3], const double vel[3], double tlim,
                      int64_t vox[3], double *th)
{
    const int32_t n[3] = {R->sp.nx, R->sp.ny, R->sp.nz};
    for (;;) {
        double tn = INFINITY;
        int ax = -1;
        for (int a = 0; a < R->sp.dim; ++a) {
            double t;
            if (vel[a] > 0.0) t = ((double)(vox[a] + 1) * R->d[a] - pos[a]) / vel[a];
            else if (vel[a] < 0.0) t = ((double)vox[a] * R->d[a] - pos[a]) / vel[a];
            else continue;
            if (t < tn) { tn = t; ax = a; }
        }
        if (ax < 0 || !(tn < tlim)) return -1;
        int64_t next[3] = {vox[0], vox[1], vox[2]};
        next[ax] += (vel[ax] > 0.0) ? 1 : -1;
        if (next[ax] < 0 || next[ax] >= n[ax]) return -1; /* a domain face: not this walk's */
        if (R->solid[cell_at(R, next)]) {
            *th = tn > 0.0 ? tn : 0.0;
            return ax;
        }
        vox[ax] = next[ax];
    }
}

/* Coordinate x moved by rounding steps only until axis_index puts it in cell
 * i along axis a (used when a position rounds into a solid cell next to the
 * fluid cell the path ended in). */
static double snap_into(const or_run *R, int a, double x, int64_t i)
{
    const int32_t n[3] = {R->sp.nx, R->sp.ny, R->sp.nz};
    if (axis_index(x, R->inv_d[a], n[a]) > i) {
        x = (double)(i + 1) * R->d[a];
        while (axis_index(x, R->inv_d[a], n[a]) > i) x = nextafter(x, -INFINITY);
    } else {
        x = (double)i * R->d[a];
        while (axis_index(x, R->inv_d[a], n[a]) < i) x = nextafter(x, INFINITY);
    }
    return x;
}

/* Re-emission from a diffuse surface at temperature Tw whose normal is axis
 * ax (side 1: the particle arrived moving +, so it leaves moving -): normal
 * speed sqrt(-2 Tw ln U), tangentials sqrt(Tw) N(0,1), from the WALL stream
 * of the slot at uniforms 4h .. 4h+2 for the h-th wall interaction. */
static void diffuse_emit(ustream *ws, int hits, double Tw, int ax, int side, double vel[3])
{
    ws->next = 4u * (uint64_t)hits;
    double w0 = us_next(ws), w1 = us_next(ws), w2 = us_next(ws);
    double vn = sqrt(-2.0 * Tw * log(w0));
    double n0, n1;
    box_muller(w1, w2, &n0, &n1);
    double stw = sqrt(Tw);
    int t1 = (ax == 0) ? 1 : 0, t2 = (ax == 2) ? 1 : 2;
    vel[ax] = side ? -vn : vn;
    vel[t1] = stw * n0;
    vel[t2] = stw * n1;
}

/* Moves one particle for dt; returns its new cell or nc (DEAD). */
static int64_t move_one(or_run *R, int64_t slot, double pos[3], double vel[3])
{
    const or_spec *sp = &R->sp;
    const int dim = sp->dim;
    double trem = sp->dt;
    int hits = 0;
    ustream ws = {{sp->run_id, sp->seed}, R->step, PURPOSE_WALL, (uint32_t)slot, 0};
    int64_t vox[3] = {axis_index(pos[0], R->inv_d[0], sp->nx), axis_index(pos[1], R->inv_d[1], sp->ny),
                      (dim == 3) ? axis_index(pos[2], R->inv_d[2], sp->nz) : 0};
    for (;;) {
        double tmin = INFINITY;
        int ax = -1, side = 0;
        for (int a = 0; a < dim; ++a) {
            double th;
            int sd;
            if (vel[a] > 0.0) { th = (R->L[a] - pos[a]) / vel[a]; sd = 1; }
            else if (vel[a] < 0.0) { th = (0.0 - pos[a]) / vel[a]; sd = 0; }
            else continue;
            if (th < 0.0) th = 0.0;
            if (th < tmin) { tmin = th; ax = a; side = sd; }
        }
        if (R->has_solid) {
            /* a solid cell entered before the domain face (or the end of the step) */
            double ts;
            int sa = solid_walk(R, pos, vel, (ax < 0 || tmin >= trem) ? trem : tmin, vox, &ts);
            if (sa >= 0) {
                int up = vel[sa] > 0.0;
                double plane = (double)(up ? vox[sa] + 1 : vox[sa]) * R->d[sa];
                for (int a = 0; a < dim; ++a) pos[a] = (a == sa) ? plane : pos[a] + vel[a] * ts;
                trem = trem - ts;
                diffuse_emit(&ws, hits, sp->solid_T, sa, up, vel);
                R->last_nsolid++;
                if (++hits == MAX_WALL_HITS) { R->err = OR_EBOUNCE; break; }
                continue;
            }
        }
        if (ax < 0 || tmin >= trem) {
            for (int a = 0; a < dim; ++a) pos[a] = pos[a] + vel[a] * trem;
            break;
        }
        for (int a = 0; a < dim; ++a)
            pos[a] = (a == ax) ? (side ? R->L[a] : 0.0) : pos[a] + vel[a] * tmin;
        trem = trem - tmin;
        int f = 2 * ax + side;
        int bc = sp->face_bc[f];
        if (bc == OR_BC_SPECULAR) {
            vel[ax] = -vel[ax];
        } else if (bc == OR_BC_DIFFUSE) {
            diffuse_emit(&ws, hits, sp->face_T[f], ax, side, vel);
        } else {
            return R->nc; /* inflow plane crossed outward, or outflow */
        }
        if (++hits == MAX_WALL_HITS) { R->err = OR_EBOUNCE; break; }
    }
    if (pos[0] < 0.0) return R->nc; /* a generated particle that never entered */
    int64_t c = cell_of(R, pos);
    if (R->has_solid && R->solid[c]) {
        /* rounding put the end point across the face of a solid cell: it
         * belongs to the fluid cell the path ended in */
        for (int a = 0; a < dim; ++a)
            if (axis_index(pos[a], R->inv_d[a], (a == 0) ? sp->nx : (a == 1) ? sp->ny : sp->nz) != vox[a])
                pos[a] = snap_into(R, a, pos[a], vox[a]);
        c = cell_of(R, pos);
    }
    return c;
}

void or_motion(or_run *R)
{
    int64_t removed = 0;
    R->last_nsolid = 0;
    for (int64_t i = 0; i < R->n; ++i) {
        double pos[3] = {R->p[0][i], R->p[1][i], R->p[2][i]};
        double vel[3] = {R->p[3][i], R->p[4][i], R->p[5][i]};
        int64_t c = move_one(R, i, pos, vel);
        R->p[0][i] = pos[0]; R->p[1][i] = pos[1]; R->p[2][i] = pos[2];
        R->p[3][i] = vel[0]; R->p[4][i] = vel[1]; R->p[5][i] = vel[2];
        /* Enumeration: the particle's bin (its sub-cell, or its cell) */
        R->cell[i] = (int32_t)(c == R->nc ? R->nbin : (R->sub == 1 ? c : bin_of(R, pos)));
        if (c == R->nc) removed++;
    }
    R->last_nremoved = removed;
    R->last_nmoved = R->n;
}

/* ------------------------------------------------------------------------- */
/* Indexing: stable counting sort of slots by cell (DEAD last)                */
/* ------------------------------------------------------------------------- */

/* The textbook stable counting sort: count, exclusive prefix sum, then place
 * the slots in ascending order.  start has nbins+1 entries. */
void or_counting_sort(const int32_t *key, int64_t n, int64_t nbins, int32_t *lcr,
                      int64_t *start, int64_t *count)
{
    for (int64_t b = 0; b < nbins; ++b) count[b] = 0;
    for (int64_t i = 0; i < n; ++i) count[key[i]]++;
    start[0] = 0;
    for (int64_t b = 0; b < nbins; ++b) start[b + 1] = start[b] + count[b];
    int64_t *cursor = (int64_t *)malloc((size_t)(nbins > 0 ? nbins : 1) * sizeof(int64_t));
    for (int64_t b = 0; b < nbins; ++b) cursor[b] = start[b];
    for (int64_t i = 0; i < n; ++i) lcr[cursor[key[i]]++] = (int32_t)i;
    free(cursor);
}

void or_indexing(or_run *R)
{
    or_counting_sort(R->cell, R->n, R->nbin + 1, R->lcr, R->cstart, R->ccount);
    R->n_sorted = R->n;
}

/* P <- P[LCR[0 : n - #DEAD]]: P becomes cell-sorted and the DEAD bin drops. */
void or_permute(or_run *R)
{
    int64_t keep = R->n - R->ccount[R->nbin];
    for (int a = 0; a < 6; ++a) {
        for (int64_t p = 0; p < keep; ++p) R->q[a][p] = R->p[a][R->lcr[p]];
        double *t = R->p[a];
        R->p[a] = R->q[a];
        R->q[a] = t;
    }
    R->n = keep;
}

/* ------------------------------------------------------------------------- */
/* Interaction: NTC collisions in one cell                                    */
/* ------------------------------------------------------------------------- */

/* The second partner of selection k given the first, i: with sub-cells
 * (off = the S + 1 sub-cell starts of the cell, relative to its first
 * particle) another particle of i's sub-cell when it holds two or more,
 * drawn uniformly; otherwise, and without sub-cells, another particle of the
 * cell, drawn uniformly.  Either way one index draw, from word a. */
static int64_t second_partner(uint32_t a, int64_t i, int64_t N, const int64_t *off)
{
    if (off) {
        int64_t s = 0;
        while (off[s + 1] <= i) s++;
        int64_t ns = off[s + 1] - off[s];
        if (ns >= 2) {
            int64_t jp = off[s] + or_index(a, (uint32_t)(ns - 1));
            return jp + (jp >= i ? 1 : 0);
        }
    }
    int64_t jp = or_index(a, (uint32_t)(N - 1));
    return jp + (jp >= i ? 1 : 0);
}

/* Collides the N particles whose velocities are u[0..N), v[..], w[..]; off
 * (NULL without sub-cells) holds the S + 1 sub-cell starts.  The number of
 * selections (NTC, Bird): M = pairs * Fnum sigma_ref dt / V_c * (sigma
 * c_r)_max + the cell's remainder, pairs = N(N-1)/2, or with nbar (not NULL)
 * N * Nbar / 2 where the running mean Nbar is first moved towards this
 * step's N by the weight nbar_alpha.
 * trace (optional) receives (i, j, accepted) per selection, at most
 * trace_cap selections. Returns the number of accepted collisions. */
static int64_t collide_cell(const or_run *R, uint32_t cell, int64_t N, double *u, double *v,
                            double *w, double *gmax, double *rem, double *nbar, const int64_t *off,
                            int32_t *trace, int64_t trace_cap, int64_t *nsel_out)
{
    double npairs;
    if (nbar) {
        *nbar = *nbar + R->sp.nbar_alpha * ((double)N - *nbar);
        npairs = 0.5 * (double)N * (*nbar);
    } else {
        npairs = 0.5 * (double)(N * (N - 1));
    }
    double M = npairs * R->coef * (*gmax) + *rem;
    double fl = floor(M);
    int64_t nsel = (int64_t)fl;
    *rem = M - fl;
    if (N < 2) nsel = 0;
    if (nsel_out) *nsel_out = nsel;
    int64_t ncol = 0;
    for (int64_t k = 0; k < nsel; ++k) {
        uint32_t c0[4] = {R->step, PURPOSE_COLL, cell, (uint32_t)(2 * k)};
        uint32_t c1[4] = {R->step, PURPOSE_COLL, cell, (uint32_t)(2 * k + 1)};
        uint32_t b0[4], b1[4];
        or_philox4x32_10(c0, (const uint32_t[2]){R->sp.run_id, R->sp.seed}, b0);
        or_philox4x32_10(c1, (const uint32_t[2]){R->sp.run_id, R->sp.seed}, b1);
        int64_t i = or_index(b0[0], (uint32_t)N);
        int64_t j = second_partner(b0[1], i, N, off);
        double du = u[i] - u[j], dv = v[i] - v[j], dw = w[i] - w[j];
        double cr = sqrt(du * du + dv * dv + dw * dw);
        double g = g_of(R, cr);
        if (g > *gmax) *gmax = g;
        int acc = or_u01(b0[2], b0[3]) < g / *gmax;
        if (trace && k < trace_cap) {
            trace[3 * k] = (int32_t)i;
            trace[3 * k + 1] = (int32_t)j;
            trace[3 * k + 2] = acc;
        }
        if (!acc) continue;
        double cosx = 2.0 * or_u01(b1[0], b1[1]) - 1.0;
        double sinx = sqrt(1.0 - cosx * cosx);
        double eps = TWO_PI * or_u01(b1[2], b1[3]);
        double rx = cr * cosx, ry = cr * sinx * cos(eps), rz = cr * sinx * sin(eps);
        double mx = 0.5 * (u[i] + u[j]), my = 0.5 * (v[i] + v[j]), mz = 0.5 * (w[i] + w[j]);
        u[i] = mx + 0.5 * rx; v[i] = my + 0.5 * ry; w[i] = mz + 0.5 * rz;
        u[j] = mx - 0.5 * rx; v[j] = my - 0.5 * ry; w[j] = mz - 0.5 * rz;
        ncol++;
    }
    return ncol;
}

void or_interaction(or_run *R)
{
    int64_t total = 0;
    int64_t *off = (int64_t *)malloc((size_t)(R->S + 1) * sizeof(int64_t));
    for (int64_t c = 0; c < R->nc; ++c) {
        /* the cell's particles: its S bins, consecutive in LCR order */
        int64_t b = R->cstart[c * R->S], N = R->cstart[(c + 1) * R->S] - b;
        for (int64_t s = 0; s <= R->S; ++s) off[s] = R->cstart[c * R->S + s] - b;
        int64_t k = collide_cell(R, (uint32_t)c, N, R->p[3] + b, R->p[4] + b, R->p[5] + b,
                                 &R->gmax[c], &R->rem_c[c], R->sp.nbar_alpha > 0.0 ? &R->nbar[c] : NULL,
                                 R->sub > 1 ? off : NULL, NULL, 0, NULL);
        R->ncoll[c] += k;
        total += k;
    }
    free(off);
    R->last_ncoll = total;
}

/* Stand-alone single-cell interaction for brute-force tests: the velocities
 * are updated in place, (gmax, rem) are in/out, trace as in collide_cell;
 * the count is always the N(N-1)/2 form (no running mean). */
int64_t or_collide_cell(const or_spec *sp, uint32_t step, uint32_t cell, int64_t N, double *u,
                        double *v, double *w, double *gmax, double *rem, const int64_t *sub_off,
                        int32_t *trace, int64_t trace_cap, int64_t *nsel_out)
{
    int32_t st;
    or_spec s2 = *sp;
    s2.capacity = 1; s2.n_init = 0; s2.solid = NULL;
    s2.face_bc[0] = OR_BC_SPECULAR;
    or_run *R = or_run_new(&s2, &st);
    if (!R) return st;
    R->step = step;
    int64_t k = collide_cell(R, cell, N, u, v, w, gmax, rem, NULL, R->sub > 1 ? sub_off : NULL, trace,
                             trace_cap, nsel_out);
    or_run_free(R);
    return k;
}

/* ------------------------------------------------------------------------- */
/* Sampling                                                                   */
/* ------------------------------------------------------------------------- */

/* out[c][7] = N, sum u, sum v, sum w, sum u^2, sum v^2, sum w^2 over cell c. */
void or_sample(const or_run *R, double *out)
{
    for (int64_t c = 0; c < R->nc; ++c) {
        double s[7] = {0, 0, 0, 0, 0, 0, 0};
        int64_t b = R->cstart[c * R->S], N = R->cstart[(c + 1) * R->S] - b;
        for (int64_t k = b; k < b + N; ++k) {
            double u = R->p[3][k], v = R->p[4][k], w = R->p[5][k];
            s[0] += 1.0;
            s[1] += u; s[2] += v; s[3] += w;
            s[4] += u * u; s[5] += v * v; s[6] += w * w;
        }
        for (int f = 0; f < 7; ++f) out[7 * c + f] = s[f];
    }
}

/* ------------------------------------------------------------------------- */
/* One time step and accessors                                                */
/* ------------------------------------------------------------------------- */

void or_step(or_run *R)
{
    R->step++;
    or_generation(R);
    or_motion(R);
    or_indexing(R);
    or_permute(R);
    or_interaction(R);
}

void or_step_begin(or_run *R) { R->step++; }

/* info: n, step, err, nc, n_sorted, last_ncoll, last_ngen, last_nremoved, last_nmoved, nface,
 * nbin */
void or_get_info(const or_run *R, int64_t info[11])
{
    info[0] = R->n; info[1] = R->step; info[2] = R->err; info[3] = R->nc;
    info[4] = R->n_sorted; info[5] = R->last_ncoll; info[6] = R->last_ngen;
    info[7] = R->last_nremoved; info[8] = R->last_nmoved; info[9] = R->nface;
    info[10] = R->nbin;
}

/* derived constants: coef, vhs_exp, gmax0, mbar, beta, s_inf, p_branch */
void or_get_consts(const or_run *R, double out[7])
{
    out[0] = R->coef; out[1] = R->vhs_exp; out[2] = R->gmax0; out[3] = R->mbar;
    out[4] = R->beta; out[5] = R->s_inf; out[6] = R->p_branch;
}

void or_get_state(const or_run *R, double *out /* [6][n] */)
{
    for (int a = 0; a < 6; ++a) memcpy(out + a * R->n, R->p[a], (size_t)R->n * sizeof(double));
}

int32_t or_set_state(or_run *R, int64_t n, const double *in /* [6][n] */)
{
    if (n < 0 || n > R->sp.capacity) return OR_EINVAL;
    for (int a = 0; a < 6; ++a) memcpy(R->p[a], in + a * n, (size_t)n * sizeof(double));
    R->n = n;
    return OR_OK;
}

void or_set_step(or_run *R, uint32_t step) { R->step = step; }

void or_get_cells(const or_run *R, int32_t *cell /* n_sorted */, int32_t *lcr /* n_sorted */,
                  int64_t *cstart /* nbin+2 */, int64_t *ccount /* nbin+1 */)
{
    if (cell) memcpy(cell, R->cell, (size_t)R->n_sorted * sizeof(int32_t));
    if (lcr) memcpy(lcr, R->lcr, (size_t)R->n_sorted * sizeof(int32_t));
    if (cstart) memcpy(cstart, R->cstart, (size_t)(R->nbin + 2) * sizeof(int64_t));
    if (ccount) memcpy(ccount, R->ccount, (size_t)(R->nbin + 1) * sizeof(int64_t));
}

void or_get_cell_state(const or_run *R, double *rem, double *gmax, int64_t *ncoll)
{
    if (rem) memcpy(rem, R->rem_c, (size_t)R->nc * sizeof(double));
    if (gmax) memcpy(gmax, R->gmax, (size_t)R->nc * sizeof(double));
    if (ncoll) memcpy(ncoll, R->ncoll, (size_t)R->nc * sizeof(int64_t));
}

void or_set_cell_state(or_run *R, const double *rem, const double *gmax)
{
    if (rem) memcpy(R->rem_c, rem, (size_t)R->nc * sizeof(double));
    if (gmax) memcpy(R->gmax, gmax, (size_t)R->nc * sizeof(double));
}

void or_get_nbar(const or_run *R, double *nbar) { memcpy(nbar, R->nbar, (size_t)R->nc * sizeof(double)); }

void or_set_nbar(or_run *R, const double *nbar) { memcpy(R->nbar, nbar, (size_t)R->nc * sizeof(double)); }

int64_t or_get_solid_hits(const or_run *R) { return R->last_nsolid; }

void or_get_face_rem(const or_run *R, double *rem)
{
    memcpy(rem, R->rem_f, (size_t)R->nface * sizeof(double));
}

/* ------------------------------------------------------------------------- */
/* Ensemble of independent runs (the outer loop), one thread per group        */
/* ------------------------------------------------------------------------- */

typedef struct {
    const or_spec *specs;
    int32_t n_runs, n_steps, n_samples, n_groups, n_threads, tid;
    const int32_t *slot_of;   /* [n_steps]: sample slot of step s (index s - 1), or -1 */
    double *acc;              /* [n_samples][n_groups][nc][7] */
    int64_t nc;
    int64_t psteps, ncoll;
    int32_t status;
} ens_job;

static void *ens_worker(void *arg)
{
    ens_job *J = (ens_job *)arg;
    double *tmp = (double *)malloc((size_t)J->nc * 7 * sizeof(double));
    for (int32_t g = J->tid; g < J->n_groups; g += J->n_threads) {
        for (int32_t r = g; r < J->n_runs; r += J->n_groups) {
            int32_t st;
            or_run *R = or_run_new(&J->specs[r], &st);
            if (!R) { J->status = st; free(tmp); return NULL; }
            or_init(R);
            for (int32_t s = 1; s <= J->n_steps; ++s) {
                or_step(R);
                J->psteps += R->last_nmoved;
                J->ncoll += R->last_ncoll;
                if (R->err) { J->status = R->err; or_run_free(R); free(tmp); return NULL; }
                const int32_t ks = J->slot_of[s - 1];
                if (ks >= 0) {
                    or_sample(R, tmp);
                    double *dst = J->acc + ((size_t)ks * J->n_groups + g) * J->nc * 7;
                    for (int64_t e = 0; e < J->nc * 7; ++e) dst[e] += tmp[e];
                }
            }
            or_run_free(R);
        }
    }
    free(tmp);
    return NULL;
}

/* Runs every run from its initial state for n_steps steps; run r adds its
 * per-cell sample sums into group r % n_groups, runs taken in ascending order
 * inside a group (so the result does not depend on n_threads).  All runs must
 * share one grid.  stats[0] = particle-steps (particles moved), stats[1] =
 * collisions.
 *
 * Sample slot k holds the snapshots taken after the steps
 * sample_steps[k] - j * stride, j = 0 .. window - 1 (those >= 1 and
 * <= n_steps): with window = 1 one moment of the unsteady process (Sec. 1.1,
 * Fig. 1); with a longer window the time average of a steady flow (an
 * averaging time much longer than dt, Sec. 1.1) on top of the average over
 * the runs (end of Sec. 3).  A step may belong to one slot only.  nsnap[k]
 * receives the number of snapshots each run adds to slot k. */
int32_t or_ensemble(const or_spec *specs, int32_t n_runs, int32_t n_steps,
                    const int32_t *sample_steps, int32_t n_samples, int32_t window,
                    int32_t stride, int32_t n_groups, int32_t n_threads, double *acc,
                    int64_t *nsnap, int64_t stats[2])
{
    if (n_runs < 1 || n_groups < 1 || n_threads < 1 || n_steps < 0 || window < 1 || stride < 1)
        return OR_EINVAL;
    int64_t nc = (int64_t)specs[0].nx * specs[0].ny * specs[0].nz;
    for (int32_t r = 1; r < n_runs; ++r)
        if ((int64_t)specs[r].nx * specs[r].ny * specs[r].nz != nc) return OR_EINVAL;
    int32_t *slot_of = (int32_t *)malloc((size_t)(n_steps > 0 ? n_steps : 1) * sizeof(int32_t));
    for (int32_t s = 0; s < n_steps; ++s) slot_of[s] = -1;
    for (int32_t k = 0; k < n_samples; ++k) {
        nsnap[k] = 0;
        for (int32_t j = 0; j < window; ++j) {
            const int64_t s = (int64_t)sample_steps[k] - (int64_t)j * stride;
            if (s < 1 || s > n_steps) continue;
            if (slot_of[s - 1] >= 0) { free(slot_of); return OR_EINVAL; }
            slot_of[s - 1] = k;
            nsnap[k]++;
        }
    }
    memset(acc, 0, (size_t)n_samples * n_groups * nc * 7 * sizeof(double));
    if (n_threads > n_groups) n_threads = n_groups;
    ens_job *jobs = (ens_job *)calloc((size_t)n_threads, sizeof(ens_job));
    pthread_t *th = (pthread_t *)calloc((size_t)n_threads, sizeof(pthread_t));
    for (int32_t t = 0; t < n_threads; ++t) {
        ens_job *J = &jobs[t];
        J->specs = specs; J->n_runs = n_runs; J->n_steps = n_steps;
        J->n_samples = n_samples; J->n_groups = n_groups; J->n_threads = n_threads;
        J->tid = t; J->slot_of = slot_of; J->acc = acc; J->nc = nc;
        pthread_create(&th[t], NULL, ens_worker, J);
    }
    int32_t status = OR_OK;
    stats[0] = stats[1] = 0;
    for (int32_t t = 0; t < n_threads; ++t) {
        pthread_join(th[t], NULL);
        if (jobs[t].status) status = jobs[t].status;
        stats[0] += jobs[t].psteps;
        stats[1] += jobs[t].ncoll;
    }
    free(jobs);
    free(th);
    free(slot_of);
    return status;
}
