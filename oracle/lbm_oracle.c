/*
 * FP64 CPU oracle for the D3Q19 lattice-Boltzmann time step with the adaptive
 * volumetric-flux inlet of McClure, Li, Sheppard and Miller, "An Adaptive
 * Volumetric Flux Boundary Condition for Lattice Boltzmann Methods"
 * (arXiv:1806.10589).
 *
 * TEST INFRASTRUCTURE ONLY. The test suite, the smoke check and the CPU
 * baseline leg of the benchmark are the only users of this file. It shares no
 * code, header, table or helper with the HIP library: the velocity set, the
 * weights and every formula below are written out here on their own, in the
 * order the paper gives them, with no blocking, fusion or reordering.
 *
 * Layout: dense array-of-structures over every voxel of the box,
 *   f[((z*ny + y)*nx + x)*19 + q],
 * solid voxels hold zeros and are skipped. Streaming is the push form of the
 * lattice Boltzmann equation (Methods, eq. LBE): the post-collision value at x
 * moves to x + xi_q.
 *
 * One step (Methods, the paragraph after eq. potential: the boundary
 * condition is applied after streaming and before collision):
 *   a. push-stream with halfway bounce-back at solid voxels and at
 *      non-periodic side faces;
 *   b. inlet (plane z = 0): integrate the consistency condition over the
 *      inlet pore sites to get the uniform inlet density (eq. potential),
 *      then apply the pressure condition with that density (Appendix B);
 *   c. outlet (plane z = nz-1): the same pressure condition with the fixed
 *      outlet density (Methods, last paragraph; Appendix B, last sentence);
 *   d. BGK collision at every pore site;
 *   e. record rho_in, Q_in, Q_out, total mass and max |u|.
 *
 * Readings where the paper is silent or garbled (all listed in the design
 * notes of the repository):
 *   - sign order inside each +/- group of eq. d3q19 is the one App. B's x- and
 *     y-momentum equations imply; weights 1/3, 1/18, 1/36 are the ones the
 *     bounce-back coefficients 1/3 and 1/6 of App. B imply;
 *   - the equilibrium's last term is -3/2 u.u (printed with a plus sign,
 *     which breaks sum f_eq = rho);
 *   - u_x = u_y = 0 at the inlet and outlet pore sites;
 *   - the Hecht-Harting closure uses the simplified rows of App. B;
 *   - the inlet area A is the number of pore sites of plane z = 0 (dr = 1);
 *   - walls are halfway (link) bounce-back;
 *   - a population whose source lies beyond z = 0 or z = nz-1 is an unknown,
 *     whatever else that source is (solid side, wall).
 *
 * Floating point: IEEE double, sums in site order, built with
 * -ffp-contract=off so no fused multiply-add changes the rounding.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define Q19 19

/* Methods, eq. d3q19: the 19 discrete velocities, grouped as the paper lists
 * them; signs inside the groups follow App. B (x-momentum: +1,7,9,11,13 and
 * -2,8,10,12,14; y-momentum: +3,7,10,15,17 and -4,8,9,16,18; z: inlet unknowns
 * 5,11,14,15,18 have xi_z = +1). */
static const int CX[Q19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
static const int CY[Q19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
static const int CZ[Q19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

/* The opposite direction: xi_opp(q) = -xi_q. Computed from the table rather
 * than listed, so that it cannot disagree with it. */
static int OPP[Q19];

/* D3Q19 weights, App. B: f_5 - f_6 = 6 rho0 w (xi.u) with coefficient 1/3
 * gives w = 1/18 for the six axis directions; the 1/6 coefficients of the
 * simplified Hecht-Harting rows give w = 1/36 for the twelve diagonals; the
 * rest weight is what makes the weights sum to one. */
static double W[Q19];

static int tables_ready = 0;

static void init_tables(void)
{
    if (tables_ready) return;
    for (int q = 0; q < Q19; ++q) {
        int n2 = CX[q] * CX[q] + CY[q] * CY[q] + CZ[q] * CZ[q];
        W[q] = (n2 == 0) ? 1.0 / 3.0 : (n2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
        OPP[q] = -1;
        for (int p = 0; p < Q19; ++p)
            if (CX[p] == -CX[q] && CY[p] == -CY[q] && CZ[p] == -CZ[q]) OPP[q] = p;
    }
    tables_ready = 1;
}

/* z-direction treatment of the box. */
enum { ORC_Z_FLUX = 0, ORC_Z_PERIODIC = 1, ORC_Z_WALL = 2 };

typedef struct orc_lattice {
    int nx, ny, nz;
    int periodic_x, periodic_y, z_mode;
    double tau, rho0, q_target, rho_out;
    int collide;
    long ncell;
    unsigned char *solid; /* [nz][ny][nx], 1 = solid */
    double *f;            /* [cell][19], post-collision state */
    double *ft;           /* streamed values of the step in progress */
    long step;
    int a_in, a_out;      /* pore sites on planes z = 0 and z = nz-1 */
} orc_lattice;

static long cell_index(const orc_lattice *L, int x, int y, int z)
{
    return ((long)z * L->ny + y) * L->nx + x;
}

void orc_velocity_set(int *cx, int *cy, int *cz, double *w, int *opp)
{
    init_tables();
    for (int q = 0; q < Q19; ++q) {
        cx[q] = CX[q];
        cy[q] = CY[q];
        cz[q] = CZ[q];
        w[q] = W[q];
        opp[q] = OPP[q];
    }
}

/* App. B, the equilibrium of the incompressible D3Q19 model:
 *   f_eq_q = w_q [ rho + rho0 (3 xi.u + 9/2 (xi.u)^2 - 3/2 u.u) ],
 * with the sign of the last term read as minus. */
void orc_equilibrium(double rho, double rho0, double ux, double uy, double uz, double *feq)
{
    init_tables();
    double uu = ux * ux + uy * uy + uz * uz;
    for (int q = 0; q < Q19; ++q) {
        double cu = CX[q] * ux + CY[q] * uy + CZ[q] * uz;
        feq[q] = W[q] * (rho + rho0 * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu));
    }
}

/* Methods eq. m0 and eq. m357: rho = sum f, j = rho0 u = sum f xi. */
static void moments(const double *f, double *rho, double *jx, double *jy, double *jz)
{
    double r = 0.0, x = 0.0, y = 0.0, z = 0.0;
    for (int q = 0; q < Q19; ++q) {
        r += f[q];
        x += f[q] * CX[q];
        y += f[q] * CY[q];
        z += f[q] * CZ[q];
    }
    *rho = r;
    *jx = x;
    *jy = y;
    *jz = z;
}

/* Methods eq. inlet: the weighted sum of the 14 known populations at an inlet
 * site, K = f0+f1+f2+f3+f4+f7+f8+f9+f10 + 2(f6+f12+f13+f16+f17). */
static double inlet_known_sum(const double *f)
{
    return f[0] + f[1] + f[2] + f[3] + f[4] + f[7] + f[8] + f[9] + f[10] +
           2.0 * (f[6] + f[12] + f[13] + f[16] + f[17]);
}

/* The outlet's consistency sum: the same argument as eq. inlet with the roles
 * of xi_z = +1 and xi_z = -1 exchanged, K' = in-plane + 2(f5+f11+f14+f15+f18),
 * so that u_z = (K' - rho)/rho0. */
static double outlet_known_sum(const double *f)
{
    return f[0] + f[1] + f[2] + f[3] + f[4] + f[7] + f[8] + f[9] + f[10] +
           2.0 * (f[5] + f[11] + f[14] + f[15] + f[18]);
}

/* Pressure condition at an inlet site with density rho (App. B):
 *   u_z from the consistency condition, u_x = u_y = 0;
 *   f5 by bounce-back of the non-equilibrium part: f5 = f6 + rho0 u_z / 3;
 *   the Hecht-Harting transverse corrections
 *     N_x = 1/2 [f1+f7+f9 - (f2+f10+f8)] - rho0 u_x / 3,
 *     N_y = 1/2 [f3+f7+f10 - (f4+f9+f8)] - rho0 u_y / 3;
 *   the simplified closure rows
 *     f11 = f12 + rho0 (u_x+u_z)/6 - N_x,  f14 = f13 + rho0 (-u_x+u_z)/6 + N_x,
 *     f15 = f16 + rho0 (u_y+u_z)/6 - N_y,  f18 = f17 + rho0 (-u_y+u_z)/6 + N_y.
 * Returns u_z. */
double orc_inlet_bc_site(double *f, double rho, double rho0)
{
    const double ux = 0.0, uy = 0.0;
    double uz = rho / rho0 - inlet_known_sum(f) / rho0;
    double nx = 0.5 * (f[1] + f[7] + f[9] - (f[2] + f[10] + f[8])) - rho0 * ux / 3.0;
    double ny = 0.5 * (f[3] + f[7] + f[10] - (f[4] + f[9] + f[8])) - rho0 * uy / 3.0;
    f[5] = f[6] + rho0 * uz / 3.0;
    f[11] = f[12] + rho0 * (ux + uz) / 6.0 - nx;
    f[14] = f[13] + rho0 * (-ux + uz) / 6.0 + nx;
    f[15] = f[16] + rho0 * (uy + uz) / 6.0 - ny;
    f[18] = f[17] + rho0 * (-uy + uz) / 6.0 + ny;
    return uz;
}

/* The same pressure condition at an outlet site (App. B, last sentence: the
 * closure rows rearranged for the outlet unknowns 6, 12, 13, 16, 17).
 * Returns u_z. */
double orc_outlet_bc_site(double *f, double rho, double rho0)
{
    const double ux = 0.0, uy = 0.0;
    double uz = outlet_known_sum(f) / rho0 - rho / rho0;
    double nx = 0.5 * (f[1] + f[7] + f[9] - (f[2] + f[10] + f[8])) - rho0 * ux / 3.0;
    double ny = 0.5 * (f[3] + f[7] + f[10] - (f[4] + f[9] + f[8])) - rho0 * uy / 3.0;
    f[6] = f[5] - rho0 * uz / 3.0;
    f[12] = f[11] - rho0 * (ux + uz) / 6.0 + nx;
    f[13] = f[14] - rho0 * (-ux + uz) / 6.0 - nx;
    f[16] = f[15] - rho0 * (uy + uz) / 6.0 + ny;
    f[17] = f[18] - rho0 * (-uy + uz) / 6.0 - ny;
    return uz;
}

orc_lattice *orc_create(int nx, int ny, int nz, const unsigned char *solid, int periodic_x,
                        int periodic_y, int z_mode, double tau, double rho0, double q_target,
                        double rho_out)
{
    init_tables();
    if (nx < 1 || ny < 1 || nz < 3 || !solid || tau <= 0.5 || rho0 <= 0.0) return NULL;
    if (z_mode < ORC_Z_FLUX || z_mode > ORC_Z_WALL) return NULL;
    orc_lattice *L = (orc_lattice *)calloc(1, sizeof(orc_lattice));
    if (!L) return NULL;
    L->nx = nx;
    L->ny = ny;
    L->nz = nz;
    L->periodic_x = periodic_x;
    L->periodic_y = periodic_y;
    L->z_mode = z_mode;
    L->tau = tau;
    L->rho0 = rho0;
    L->q_target = q_target;
    L->rho_out = rho_out;
    L->collide = 1;
    L->ncell = (long)nx * ny * nz;
    L->solid = (unsigned char *)malloc((size_t)L->ncell);
    L->f = (double *)calloc((size_t)L->ncell * Q19, sizeof(double));
    L->ft = (double *)calloc((size_t)L->ncell * Q19, sizeof(double));
    if (!L->solid || !L->f || !L->ft) {
        free(L->solid);
        free(L->f);
        free(L->ft);
        free(L);
        return NULL;
    }
    memcpy(L->solid, solid, (size_t)L->ncell);
    L->a_in = L->a_out = 0;
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            if (!L->solid[cell_index(L, x, y, 0)]) L->a_in++;
            if (!L->solid[cell_index(L, x, y, nz - 1)]) L->a_out++;
        }
    if (z_mode == ORC_Z_FLUX && L->a_in == 0) {
        free(L->solid);
        free(L->f);
        free(L->ft);
        free(L);
        return NULL;
    }
    return L;
}

void orc_destroy(orc_lattice *L)
{
    if (!L) return;
    free(L->solid);
    free(L->f);
    free(L->ft);
    free(L);
}

void orc_set_collision(orc_lattice *L, int on) { L->collide = on; }
void orc_set_target_flux(orc_lattice *L, double q) { L->q_target = q; }
void orc_set_outlet_density(orc_lattice *L, double rho) { L->rho_out = rho; }
long orc_step_count(const orc_lattice *L) { return L->step; }
int orc_inlet_area(const orc_lattice *L) { return L->a_in; }
int orc_outlet_area(const orc_lattice *L) { return L->a_out; }

void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Rest (or uniform) equilibrium at every pore site. */
void orc_init_equilibrium(orc_lattice *L, double rho, double ux, double uy, double uz)
{
    double feq[Q19];
    orc_equilibrium(rho, L->rho0, ux, uy, uz, feq);
    for (long c = 0; c < L->ncell; ++c)
        for (int q = 0; q < Q19; ++q) L->f[c * Q19 + q] = L->solid[c] ? 0.0 : feq[q];
    L->step = 0;
}

void orc_set_f(orc_lattice *L, const double *f)
{
    for (long c = 0; c < L->ncell; ++c)
        for (int q = 0; q < Q19; ++q) L->f[c * Q19 + q] = L->solid[c] ? 0.0 : f[c * Q19 + q];
}

void orc_get_f(const orc_lattice *L, double *f)
{
    memcpy(f, L->f, (size_t)L->ncell * Q19 * sizeof(double));
}

/* Dense density and velocity fields of the stored (post-collision) state.
 * Collision conserves rho and j, so these are also the post-boundary moments
 * of the last step. Solid voxels get zeros. */
void orc_fields(const orc_lattice *L, double *rho, double *ux, double *uy, double *uz)
{
    for (long c = 0; c < L->ncell; ++c) {
        if (L->solid[c]) {
            rho[c] = ux[c] = uy[c] = uz[c] = 0.0;
            continue;
        }
        double r, jx, jy, jz;
        moments(&L->f[c * Q19], &r, &jx, &jy, &jz);
        rho[c] = r;
        ux[c] = jx / L->rho0;
        uy[c] = jy / L->rho0;
        uz[c] = jz / L->rho0;
    }
}

/* a. Push streaming with halfway bounce-back. Every slot of ft that no
 * population reaches is left NaN: those are exactly the boundary unknowns,
 * which the inlet/outlet conditions fill; a NaN surviving them would expose a
 * streaming error. */
static void stream_push(orc_lattice *L)
{
    const int nx = L->nx, ny = L->ny, nz = L->nz;
    const double nan_value = NAN;
#pragma omp parallel for schedule(static)
    for (long c = 0; c < L->ncell; ++c)
        for (int q = 0; q < Q19; ++q) L->ft[c * Q19 + q] = L->solid[c] ? 0.0 : nan_value;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long c = cell_index(L, x, y, z);
                if (L->solid[c]) continue;
                for (int q = 0; q < Q19; ++q) {
                    int tx = x + CX[q], ty = y + CY[q], tz = z + CZ[q];
                    int leaves = 0, blocked = 0;
                    /* The z faces take precedence: a population that crosses
                     * z = 0 or z = nz-1 of an open box leaves the domain. */
                    if (tz < 0 || tz >= nz) {
                        if (L->z_mode == ORC_Z_PERIODIC)
                            tz = (tz + nz) % nz;
                        else if (L->z_mode == ORC_Z_WALL)
                            blocked = 1;
                        else
                            leaves = 1;
                    }
                    if (leaves) continue;
                    if (tx < 0 || tx >= nx) {
                        if (L->periodic_x)
                            tx = (tx + nx) % nx;
                        else
                            blocked = 1;
                    }
                    if (ty < 0 || ty >= ny) {
                        if (L->periodic_y)
                            ty = (ty + ny) % ny;
                        else
                            blocked = 1;
                    }
                    if (!blocked && L->solid[cell_index(L, tx, ty, tz)]) blocked = 1;
                    double v = L->f[c * Q19 + q];
                    if (blocked)
                        L->ft[c * Q19 + OPP[q]] = v;
                    else
                        L->ft[cell_index(L, tx, ty, tz) * Q19 + q] = v;
                }
            }
}

/* d. BGK collision with relaxation time tau: f <- f - (f - f_eq)/tau
 * (Methods: nu = c_s^2 (tau - 1/2)). */
static void collide_bgk(orc_lattice *L)
{
    const double omega = L->collide ? 1.0 / L->tau : 0.0;
    const double rho0 = L->rho0;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < L->nz; ++z) {
        double feq[Q19];
        for (long c = (long)z * L->ny * L->nx; c < (long)(z + 1) * L->ny * L->nx; ++c) {
            if (L->solid[c]) continue;
            double *f = &L->ft[c * Q19];
            double rho, jx, jy, jz;
            moments(f, &rho, &jx, &jy, &jz);
            orc_equilibrium(rho, rho0, jx / rho0, jy / rho0, jz / rho0, feq);
            for (int q = 0; q < Q19; ++q) f[q] = f[q] - omega * (f[q] - feq[q]);
        }
    }
}

/* One time step. hist (may be NULL) receives, in this order:
 * rho_in, Q_in, Q_out, total mass, max |u|.
 * Returns 0, or -1 if a slot was left unset (a streaming error). */
static int step_once(orc_lattice *L, double *hist)
{
    const int nx = L->nx, ny = L->ny, nz = L->nz;
    const double rho0 = L->rho0;
    stream_push(L);

    double rho_in = NAN, q_in = 0.0, q_out = 0.0;
    if (L->z_mode == ORC_Z_FLUX) {
        /* b. eq. potential: rho = rho0 Q_z / A + (1/A) sum_i K_i over the
         * inlet pore sites, summed in site order. */
        double ksum = 0.0;
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long c = cell_index(L, x, y, 0);
                if (L->solid[c]) continue;
                ksum += inlet_known_sum(&L->ft[c * Q19]);
            }
        rho_in = rho0 * L->q_target / (double)L->a_in + ksum / (double)L->a_in;
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long c = cell_index(L, x, y, 0);
                if (L->solid[c]) continue;
                q_in += orc_inlet_bc_site(&L->ft[c * Q19], rho_in, rho0);
            }
        /* c. pressure outlet with rho_out. */
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long c = cell_index(L, x, y, nz - 1);
                if (L->solid[c]) continue;
                q_out += orc_outlet_bc_site(&L->ft[c * Q19], L->rho_out, rho0);
            }
    }

    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (long c = 0; c < L->ncell; ++c) {
        if (L->solid[c]) continue;
        for (int q = 0; q < Q19; ++q)
            if (isnan(L->ft[c * Q19 + q])) bad |= 1;
    }

    double mass = 0.0, umax = 0.0;
    if (hist) {
        /* e. max |u| over the post-boundary moments (collision keeps them). */
        for (long c = 0; c < L->ncell; ++c) {
            if (L->solid[c]) continue;
            double rho, jx, jy, jz;
            moments(&L->ft[c * Q19], &rho, &jx, &jy, &jz);
            double u = sqrt(jx * jx + jy * jy + jz * jz) / rho0;
            if (u > umax || isnan(u)) umax = u;
        }
    }

    collide_bgk(L);

    if (hist) {
        for (long c = 0; c < L->ncell; ++c) {
            if (L->solid[c]) continue;
            for (int q = 0; q < Q19; ++q) mass += L->ft[c * Q19 + q];
        }
        hist[0] = rho_in;
        hist[1] = q_in;
        hist[2] = q_out;
        hist[3] = mass;
        hist[4] = umax;
    }
    double *t = L->f;
    L->f = L->ft;
    L->ft = t;
    L->step++;
    return bad ? -1 : 0;
}

/* Advance n steps; hist (may be NULL) gets 5 values per step. */
int orc_step(orc_lattice *L, int n, double *hist)
{
    for (int i = 0; i < n; ++i) {
        int rc = step_once(L, hist ? hist + 5 * (long)i : NULL);
        if (rc) return rc;
    }
    return 0;
}
