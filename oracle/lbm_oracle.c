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
    double rho_offset;    /* added to the inlet density of eq. potential (controller tests) */
    int collide;
    int mrt;              /* 1: MRT collision of Appendix A instead of BGK */
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

/* a. Push streaming with halfway bounce-back of the first nq velocities
 * (19 for D3Q19; 7 for the D3Q7 mass transport, whose velocities are q = 0..6
 * of the same set, App. A), src and dst with stride nq. Every slot of dst that
 * no population reaches is left NaN: those are exactly the boundary unknowns,
 * which the inlet/outlet conditions fill; a NaN surviving them would expose a
 * streaming error. */
static void stream_push_n(const orc_lattice *L, const double *src, double *dst, int nq)
{
    const int nx = L->nx, ny = L->ny, nz = L->nz;
    const double nan_value = NAN;
#pragma omp parallel for schedule(static)
    for (long c = 0; c < L->ncell; ++c)
        for (int q = 0; q < nq; ++q) dst[c * nq + q] = L->solid[c] ? 0.0 : nan_value;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long c = cell_index(L, x, y, z);
                if (L->solid[c]) continue;
                for (int q = 0; q < nq; ++q) {
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
                    double v = src[c * nq + q];
                    if (blocked)
                        dst[c * nq + OPP[q]] = v;
                    else
                        dst[cell_index(L, tx, ty, tz) * nq + q] = v;
                }
            }
}

static void stream_push(orc_lattice *L) { stream_push_n(L, L->f, L->ft, Q19); }

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

/* b, c. The flux inlet and the pressure outlet on the streamed values ft.
 * uz_in / uz_out (may be NULL) receive the boundary velocity of every site of
 * plane z = 0 / z = nz-1 (index x + nx*y; solid sites untouched). */
static void apply_momentum_bc(orc_lattice *L, double *uz_in, double *uz_out, double *rho_in_out,
                              double *q_in_out, double *q_out_out)
{
    const int nx = L->nx, ny = L->ny, nz = L->nz;
    const double rho0 = L->rho0;
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
        rho_in = rho0 * L->q_target / (double)L->a_in + ksum / (double)L->a_in + L->rho_offset;
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long c = cell_index(L, x, y, 0);
                if (L->solid[c]) continue;
                double uz = orc_inlet_bc_site(&L->ft[c * Q19], rho_in, rho0);
                if (uz_in) uz_in[x + nx * y] = uz;
                q_in += uz;
            }
        /* c. pressure outlet with rho_out. */
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long c = cell_index(L, x, y, nz - 1);
                if (L->solid[c]) continue;
                double uz = orc_outlet_bc_site(&L->ft[c * Q19], L->rho_out, rho0);
                if (uz_out) uz_out[x + nx * y] = uz;
                q_out += uz;
            }
    }
    *rho_in_out = rho_in;
    *q_in_out = q_in;
    *q_out_out = q_out;
}

/* 1 if a pore slot of a (stride nq) is NaN: a slot no population reached. */
static int any_unset(const orc_lattice *L, const double *a, int nq)
{
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (long c = 0; c < L->ncell; ++c) {
        if (L->solid[c]) continue;
        for (int q = 0; q < nq; ++q)
            if (isnan(a[c * nq + q])) bad |= 1;
    }
    return bad;
}

/* max |u| over the pore sites of a state (collision keeps rho and j). */
static double max_speed(const orc_lattice *L, const double *f)
{
    double umax = 0.0;
    for (long c = 0; c < L->ncell; ++c) {
        if (L->solid[c]) continue;
        double rho, jx, jy, jz;
        moments(&f[c * Q19], &rho, &jx, &jy, &jz);
        double u = sqrt(jx * jx + jy * jy + jz * jz) / L->rho0;
        if (u > umax || isnan(u)) umax = u;
    }
    return umax;
}

static double total_mass(const orc_lattice *L, const double *a, int nq)
{
    double m = 0.0;
    for (long c = 0; c < L->ncell; ++c) {
        if (L->solid[c]) continue;
        for (int q = 0; q < nq; ++q) m += a[c * nq + q];
    }
    return m;
}

void orc_mrt_collide_site(double *f, double rho0, double tau, double alpha, double gx, double gy,
                          double gz);

/* Single-fluid MRT collision (Appendix A without the interfacial stress) of
 * every pore cell of the streamed values. */
static void collide_mrt(orc_lattice *L)
{
#pragma omp parallel for schedule(static)
    for (int z = 0; z < L->nz; ++z)
        for (long c = (long)z * L->ny * L->nx; c < (long)(z + 1) * L->ny * L->nx; ++c)
            if (!L->solid[c]) orc_mrt_collide_site(&L->ft[c * Q19], L->rho0, L->tau, 0.0, 0.0, 0.0, 0.0);
}

void orc_set_mrt(orc_lattice *L, int on) { L->mrt = on; }

/* One time step. hist (may be NULL) receives, in this order:
 * rho_in, Q_in, Q_out, total mass, max |u|.
 * Returns 0, or -1 if a slot was left unset (a streaming error). */
static int step_once(orc_lattice *L, double *hist)
{
    stream_push(L);
    double rho_in, q_in, q_out;
    apply_momentum_bc(L, NULL, NULL, &rho_in, &q_in, &q_out);
    int bad = any_unset(L, L->ft, Q19);
    double umax = hist ? max_speed(L, L->ft) : 0.0;
    if (L->mrt && L->collide)
        collide_mrt(L);
    else
        collide_bgk(L);
    if (hist) {
        hist[0] = rho_in;
        hist[1] = q_in;
        hist[2] = q_out;
        hist[3] = total_mass(L, L->ft, Q19);
        hist[4] = umax;
    }
    double *t = L->f;
    L->f = L->ft;
    L->ft = t;
    L->step++;
    return bad ? -1 : 0;
}

/* An offset added to the inlet density of eq. potential in every following
 * step (0 for the paper's method; the tests of the inlet controller use it). */
void orc_set_inlet_offset(orc_lattice *L, double d) { L->rho_offset = d; }

/* The inlet density eq. potential gives for the next step, without the
 * offset: stream the current state (into the scratch buffer, which the next
 * step overwrites anyway) and sum K_i over the inlet pore sites. */
double orc_plain_inlet_density(orc_lattice *L)
{
    stream_push(L);
    double ksum = 0.0;
    for (int y = 0; y < L->ny; ++y)
        for (int x = 0; x < L->nx; ++x) {
            long c = cell_index(L, x, y, 0);
            if (L->solid[c]) continue;
            ksum += inlet_known_sum(&L->ft[c * Q19]);
        }
    return (L->rho0 * L->q_target + ksum) / (double)L->a_in;
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

/* ======================================================================
 * Two-fluid colour-gradient model (Appendix A).
 *
 * Momentum: D3Q19 MRT. Moments m = M f in the basis of d'Humieres et al.
 * (2002), in the order Appendix A lists them:
 *   (rho, e, eps, j_x, q_x, j_y, q_y, j_z, q_z, 3p_xx, 3pi_xx, p_ww, pi_ww,
 *    p_xy, p_yz, p_xz, m_x, m_y, m_z),
 * built here from the basis polynomials of that paper (the matrix is not
 * printed in the text). Relaxation m* = m - S (m - m_eq) with
 *   S = diag(0, s_e, s_eps, 0, s_q, 0, s_q, 0, s_q, s_nu, s_pi, s_nu, s_pi,
 *            s_nu, s_nu, s_nu, s_m, s_m, s_m),
 *   s_e = s_eps = s_pi = s_nu = 1/tau,  s_q = s_m = 8 (2 - s_nu)/(8 - s_nu).
 * Equilibrium moments: the projections M f_eq(rho, j) plus the interfacial
 * stress of Appendix A, alpha |C| times
 *   e: 19 (the paper's e is the density-independent part scaled by 1/19),
 *   3p_xx: (2n_x^2 - n_y^2 - n_z^2)/2,  p_ww: (n_y^2 - n_z^2)/2,
 *   p_xy: n_x n_y/2,  p_yz: n_y n_z/2,  p_xz: n_x n_z/2.
 * C = grad phi by the isotropic stencil C = 3 sum_q w_q xi_q phi(x + xi_q),
 * n = C/|C| (n = 0 where |C| <= 1e-6).
 *
 * Mass transport: D3Q7 (q = 0..6 of the same velocity set, weights 1/3 and
 * 1/9) for the two colours A (non-wetting) and B (wetting), streamed with
 * halfway bounce-back and then fully relaxed to the recoloured equilibrium
 *   A_q = w_q N_A [1 + 9/2 u.xi_q + beta N_B n.xi_q],
 *   B_q = w_q N_B [1 + 9/2 u.xi_q - beta N_A n.xi_q],
 * with N_A = sum A_q, N_B = sum B_q, phi = (N_A - N_B)/(N_A + N_B).
 *
 * Readings (where Appendix A is silent): phi at a solid neighbour or beyond a
 * non-periodic side is phi_solid (wetting); phi beyond z = 0 or z = nz-1 of an
 * open box is the site's own phi; inlet injects pure A: A_5 = w_5 (1 + 9/2 u_z),
 * B_5 = 0; the outlet unknowns A_6, B_6 are the equilibrium of the site's
 * previous-step densities with the boundary velocity:
 *   A_6 = w_6 N_A^prev (1 - 9/2 u_z), B_6 = w_6 N_B^prev (1 - 9/2 u_z).
 * ====================================================================== */

#define Q7 7
static const double W7[Q7] = {1.0 / 3.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                              1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0};

static double MB[Q19][Q19]; /* MB[k][q]: moment k of direction q */
static double MB_NORM2[Q19];
static int mrt_ready = 0;

static void init_mrt(void)
{
    if (mrt_ready) return;
    init_tables();
    for (int q = 0; q < Q19; ++q) {
        const double x = CX[q], y = CY[q], z = CZ[q];
        const double c2 = x * x + y * y + z * z;
        MB[0][q] = 1.0;
        MB[1][q] = 19.0 * c2 - 30.0;
        MB[2][q] = (21.0 * c2 * c2 - 53.0 * c2 + 24.0) / 2.0;
        MB[3][q] = x;
        MB[4][q] = (5.0 * c2 - 9.0) * x;
        MB[5][q] = y;
        MB[6][q] = (5.0 * c2 - 9.0) * y;
        MB[7][q] = z;
        MB[8][q] = (5.0 * c2 - 9.0) * z;
        MB[9][q] = 3.0 * x * x - c2;
        MB[10][q] = (3.0 * c2 - 5.0) * (3.0 * x * x - c2);
        MB[11][q] = y * y - z * z;
        MB[12][q] = (3.0 * c2 - 5.0) * (y * y - z * z);
        MB[13][q] = x * y;
        MB[14][q] = y * z;
        MB[15][q] = x * z;
        MB[16][q] = (y * y - z * z) * x;
        MB[17][q] = (z * z - x * x) * y;
        MB[18][q] = (x * x - y * y) * z;
    }
    for (int k = 0; k < Q19; ++k) {
        double s = 0.0;
        for (int q = 0; q < Q19; ++q) s += MB[k][q] * MB[k][q];
        MB_NORM2[k] = s;
    }
    mrt_ready = 1;
}

void orc_mrt_matrix(double *m19x19)
{
    init_mrt();
    for (int k = 0; k < Q19; ++k)
        for (int q = 0; q < Q19; ++q) m19x19[k * Q19 + q] = MB[k][q];
}

/* MRT collision of one site with relaxation rates S[19] and the colour
 * stress of gradient (gx, gy, gz) (alpha = 0 or C = 0: plain MRT). */
void orc_mrt_collide_site_rates(double *f, double rho0, const double *S, double alpha, double gx,
                                double gy, double gz)
{
    init_mrt();
    double m[Q19], meq[Q19], feq[Q19];
    double rho, jx, jy, jz;
    moments(f, &rho, &jx, &jy, &jz);
    orc_equilibrium(rho, rho0, jx / rho0, jy / rho0, jz / rho0, feq);
    for (int k = 0; k < Q19; ++k) {
        double a = 0.0, b = 0.0;
        for (int q = 0; q < Q19; ++q) {
            a += MB[k][q] * f[q];
            b += MB[k][q] * feq[q];
        }
        m[k] = a;
        meq[k] = b;
    }
    const double cmag = sqrt(gx * gx + gy * gy + gz * gz);
    if (alpha != 0.0 && cmag > 1e-6) {
        const double nx = gx / cmag, ny = gy / cmag, nz = gz / cmag;
        const double ac = alpha * cmag;
        meq[1] += 19.0 * ac;
        meq[9] += 0.5 * ac * (2.0 * nx * nx - ny * ny - nz * nz);
        meq[11] += 0.5 * ac * (ny * ny - nz * nz);
        meq[13] += 0.5 * ac * nx * ny;
        meq[14] += 0.5 * ac * ny * nz;
        meq[15] += 0.5 * ac * nx * nz;
    }
    for (int k = 0; k < Q19; ++k) m[k] = m[k] - S[k] * (m[k] - meq[k]);
    for (int q = 0; q < Q19; ++q) {
        double v = 0.0;
        for (int k = 0; k < Q19; ++k) v += MB[k][q] * m[k] / MB_NORM2[k];
        f[q] = v;
    }
}

/* The paper's rates: s_e = s_eps = s_pi = s_nu = 1/tau, s_q = s_m =
 * 8 (2 - s_nu)/(8 - s_nu); density and momentum are not relaxed. */
void orc_mrt_collide_site(double *f, double rho0, double tau, double alpha, double gx, double gy,
                          double gz)
{
    const double snu = 1.0 / tau;
    const double sq = 8.0 * (2.0 - snu) / (8.0 - snu);
    const double S[Q19] = {0.0, snu, snu, 0.0, sq, 0.0, sq, 0.0, sq, snu,
                           snu, snu, snu, snu, snu, snu, sq,  sq,  sq};
    orc_mrt_collide_site_rates(f, rho0, S, alpha, gx, gy, gz);
}

typedef struct orc_colour {
    orc_lattice *L;
    double alpha, beta, phi_solid;
    double *A, *B, *At, *Bt; /* [cell][7] */
    double *na, *nb, *phi;   /* [cell] after streaming of the step in progress */
    double *uz_in, *uz_out;  /* [ny][nx] boundary velocities */
} orc_colour;

void orc_colour_destroy(orc_colour *C);

orc_colour *orc_colour_create(int nx, int ny, int nz, const unsigned char *solid, int periodic_x,
                              int periodic_y, int z_mode, double tau, double rho0,
                              double q_target, double rho_out, double alpha, double beta,
                              double phi_solid)
{
    init_mrt();
    orc_lattice *L = orc_create(nx, ny, nz, solid, periodic_x, periodic_y, z_mode, tau, rho0,
                                q_target, rho_out);
    if (!L) return NULL;
    orc_colour *C = (orc_colour *)calloc(1, sizeof(orc_colour));
    if (!C) {
        orc_destroy(L);
        return NULL;
    }
    C->L = L;
    C->alpha = alpha;
    C->beta = beta;
    C->phi_solid = phi_solid;
    size_t n7 = (size_t)L->ncell * Q7;
    C->A = (double *)calloc(n7, sizeof(double));
    C->B = (double *)calloc(n7, sizeof(double));
    C->At = (double *)calloc(n7, sizeof(double));
    C->Bt = (double *)calloc(n7, sizeof(double));
    C->na = (double *)calloc((size_t)L->ncell, sizeof(double));
    C->nb = (double *)calloc((size_t)L->ncell, sizeof(double));
    C->phi = (double *)calloc((size_t)L->ncell, sizeof(double));
    C->uz_in = (double *)calloc((size_t)nx * ny, sizeof(double));
    C->uz_out = (double *)calloc((size_t)nx * ny, sizeof(double));
    if (!C->A || !C->B || !C->At || !C->Bt || !C->na || !C->nb || !C->phi || !C->uz_in ||
        !C->uz_out) {
        orc_colour_destroy(C); /* frees whatever was allocated, and the lattice */
        return NULL;
    }
    return C;
}

void orc_colour_destroy(orc_colour *C)
{
    if (!C) return;
    orc_destroy(C->L);
    free(C->A);
    free(C->B);
    free(C->At);
    free(C->Bt);
    free(C->na);
    free(C->nb);
    free(C->phi);
    free(C->uz_in);
    free(C->uz_out);
    free(C);
}

/* Rest momentum state (rho = 1, u = 0) and colour densities na, nb (dense
 * [cell]) as D3Q7 equilibria at rest. */
void orc_colour_init(orc_colour *C, const double *na, const double *nb)
{
    orc_lattice *L = C->L;
    orc_init_equilibrium(L, 1.0, 0.0, 0.0, 0.0);
    for (long c = 0; c < L->ncell; ++c)
        for (int q = 0; q < Q7; ++q) {
            C->A[c * Q7 + q] = L->solid[c] ? 0.0 : W7[q] * na[c];
            C->B[c * Q7 + q] = L->solid[c] ? 0.0 : W7[q] * nb[c];
        }
}

void orc_colour_set_state(orc_colour *C, const double *f, const double *A, const double *B)
{
    orc_lattice *L = C->L;
    orc_set_f(L, f);
    for (long c = 0; c < L->ncell; ++c)
        for (int q = 0; q < Q7; ++q) {
            C->A[c * Q7 + q] = L->solid[c] ? 0.0 : A[c * Q7 + q];
            C->B[c * Q7 + q] = L->solid[c] ? 0.0 : B[c * Q7 + q];
        }
}

void orc_colour_get_state(const orc_colour *C, double *f, double *A, double *B)
{
    orc_get_f(C->L, f);
    memcpy(A, C->A, (size_t)C->L->ncell * Q7 * sizeof(double));
    memcpy(B, C->B, (size_t)C->L->ncell * Q7 * sizeof(double));
}

/* phi of the neighbour x + xi_q of pore cell (x, y, z) in the dense phase
 * field phi, with the readings above for solids, sides and the open z
 * faces. */
static double neighbour_phi(const orc_colour *C, const double *phi, int x, int y, int z, int q)
{
    const orc_lattice *L = C->L;
    int tx = x + CX[q], ty = y + CY[q], tz = z + CZ[q];
    if (tz < 0 || tz >= L->nz) {
        if (L->z_mode == ORC_Z_PERIODIC)
            tz = (tz + L->nz) % L->nz;
        else if (L->z_mode == ORC_Z_WALL)
            return C->phi_solid;
        else
            return phi[cell_index(L, x, y, z)];
    }
    if (tx < 0 || tx >= L->nx) {
        if (!L->periodic_x) return C->phi_solid;
        tx = (tx + L->nx) % L->nx;
    }
    if (ty < 0 || ty >= L->ny) {
        if (!L->periodic_y) return C->phi_solid;
        ty = (ty + L->ny) % L->ny;
    }
    long t = cell_index(L, tx, ty, tz);
    return L->solid[t] ? C->phi_solid : phi[t];
}

/* Colour gradient at pore cell (x, y, z) by the isotropic D3Q19 stencil
 * C = 3 sum_q w_q xi_q phi(x + xi_q) (Appendix A names the gradient of the
 * phase field but prints no stencil; this one is exact for fields up to
 * quadratic order away from solids and faces). */
static void colour_gradient_site(const orc_colour *C, const double *phi, int x, int y, int z,
                                 double *gx, double *gy, double *gz)
{
    double ax = 0.0, ay = 0.0, az = 0.0;
    for (int q = 1; q < Q19; ++q) {
        const double p = neighbour_phi(C, phi, x, y, z, q);
        ax += 3.0 * W[q] * CX[q] * p;
        ay += 3.0 * W[q] * CY[q] * p;
        az += 3.0 * W[q] * CZ[q] * p;
    }
    *gx = ax;
    *gy = ay;
    *gz = az;
}

/* The colour gradient of a given dense phase field phi [cell] at every pore
 * cell, grad [cell][3] (zero at solid cells): the stencil the step uses. */
void orc_colour_gradient(const orc_colour *C, const double *phi, double *grad)
{
    const orc_lattice *L = C->L;
    for (int z = 0; z < L->nz; ++z)
        for (int y = 0; y < L->ny; ++y)
            for (int x = 0; x < L->nx; ++x) {
                long c = cell_index(L, x, y, z);
                grad[c * 3] = grad[c * 3 + 1] = grad[c * 3 + 2] = 0.0;
                if (L->solid[c]) continue;
                colour_gradient_site(C, phi, x, y, z, &grad[c * 3], &grad[c * 3 + 1],
                                     &grad[c * 3 + 2]);
            }
}

/* One two-fluid step. hist (may be NULL): rho_in, Q_in, Q_out, mass, max|u|,
 * sum N_A, sum N_B. */
static int colour_step_once(orc_colour *C, double *hist)
{
    orc_lattice *L = C->L;
    const int nx = L->nx, ny = L->ny, nz = L->nz;
    const double rho0 = L->rho0;

    /* previous colour densities at the outlet sites (stored state) */
    double *na_prev = (double *)malloc((size_t)nx * ny * sizeof(double));
    double *nb_prev = (double *)malloc((size_t)nx * ny * sizeof(double));
    if (!na_prev || !nb_prev) {
        free(na_prev);
        free(nb_prev);
        return -2;
    }
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            long c = cell_index(L, x, y, nz - 1);
            double a = 0.0, b = 0.0;
            for (int q = 0; q < Q7; ++q) {
                a += C->A[c * Q7 + q];
                b += C->B[c * Q7 + q];
            }
            na_prev[x + nx * y] = a;
            nb_prev[x + nx * y] = b;
        }

    /* 1. stream f, A, B */
    stream_push_n(L, L->f, L->ft, Q19);
    stream_push_n(L, C->A, C->At, Q7);
    stream_push_n(L, C->B, C->Bt, Q7);

    /* 2. momentum boundary conditions (as for the single fluid) */
    double rho_in, q_in, q_out;
    apply_momentum_bc(L, C->uz_in, C->uz_out, &rho_in, &q_in, &q_out);

    /* 3. mass-transport boundary unknowns */
    if (L->z_mode == ORC_Z_FLUX) {
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long c = cell_index(L, x, y, 0);
                if (L->solid[c]) continue;
                const double uz = C->uz_in[x + nx * y];
                C->At[c * Q7 + 5] = W7[5] * 1.0 * (1.0 + 4.5 * uz);
                C->Bt[c * Q7 + 5] = 0.0;
            }
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long c = cell_index(L, x, y, nz - 1);
                if (L->solid[c]) continue;
                const double uz = C->uz_out[x + nx * y];
                C->At[c * Q7 + 6] = W7[6] * na_prev[x + nx * y] * (1.0 - 4.5 * uz);
                C->Bt[c * Q7 + 6] = W7[6] * nb_prev[x + nx * y] * (1.0 - 4.5 * uz);
            }
    }
    free(na_prev);
    free(nb_prev);

    int bad = any_unset(L, L->ft, Q19) | any_unset(L, C->At, Q7) | any_unset(L, C->Bt, Q7);

    /* 4. phase field at every pore site */
#pragma omp parallel for schedule(static)
    for (long c = 0; c < L->ncell; ++c) {
        if (L->solid[c]) continue;
        double a = 0.0, b = 0.0;
        for (int q = 0; q < Q7; ++q) {
            a += C->At[c * Q7 + q];
            b += C->Bt[c * Q7 + q];
        }
        C->na[c] = a;
        C->nb[c] = b;
        C->phi[c] = (a + b) != 0.0 ? (a - b) / (a + b) : 0.0;
    }

    double umax = hist ? max_speed(L, L->ft) : 0.0;

    /* 5-7. colour gradient, MRT with the interfacial stress, recolouring */
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long c = cell_index(L, x, y, z);
                if (L->solid[c]) continue;
                double gx, gy, gz;
                colour_gradient_site(C, C->phi, x, y, z, &gx, &gy, &gz);
                double *f = &L->ft[c * Q19];
                double rho, jx, jy, jz;
                moments(f, &rho, &jx, &jy, &jz);
                const double ux = jx / rho0, uy = jy / rho0, uz = jz / rho0;
                if (!L->collide) continue; /* testing aid: pure streaming */
                orc_mrt_collide_site(f, rho0, L->tau, C->alpha, gx, gy, gz);
                const double cmag = sqrt(gx * gx + gy * gy + gz * gz);
                double nxv = 0.0, nyv = 0.0, nzv = 0.0;
                if (cmag > 1e-6) {
                    nxv = gx / cmag;
                    nyv = gy / cmag;
                    nzv = gz / cmag;
                }
                const double na = C->na[c], nb = C->nb[c];
                for (int q = 0; q < Q7; ++q) {
                    const double cu = CX[q] * ux + CY[q] * uy + CZ[q] * uz;
                    const double cn = CX[q] * nxv + CY[q] * nyv + CZ[q] * nzv;
                    C->At[c * Q7 + q] = W7[q] * na * (1.0 + 4.5 * cu + C->beta * nb * cn);
                    C->Bt[c * Q7 + q] = W7[q] * nb * (1.0 + 4.5 * cu - C->beta * na * cn);
                }
            }

    if (hist) {
        hist[0] = rho_in;
        hist[1] = q_in;
        hist[2] = q_out;
        hist[3] = total_mass(L, L->ft, Q19);
        hist[4] = umax;
        hist[5] = total_mass(L, C->At, Q7);
        hist[6] = total_mass(L, C->Bt, Q7);
    }
    double *t = L->f;
    L->f = L->ft;
    L->ft = t;
    t = C->A;
    C->A = C->At;
    C->At = t;
    t = C->B;
    C->B = C->Bt;
    C->Bt = t;
    L->step++;
    return bad ? -1 : 0;
}

int orc_colour_step(orc_colour *C, int n, double *hist)
{
    for (int i = 0; i < n; ++i) {
        int rc = colour_step_once(C, hist ? hist + 7 * (long)i : NULL);
        if (rc) return rc;
    }
    return 0;
}

/* Dense fields of the stored state: rho, u, and phi from the stored A, B. */
void orc_colour_fields(const orc_colour *C, double *rho, double *ux, double *uy, double *uz,
                       double *phi)
{
    const orc_lattice *L = C->L;
    orc_fields(L, rho, ux, uy, uz);
    for (long c = 0; c < L->ncell; ++c) {
        if (L->solid[c]) {
            phi[c] = 0.0;
            continue;
        }
        double a = 0.0, b = 0.0;
        for (int q = 0; q < Q7; ++q) {
            a += C->A[c * Q7 + q];
            b += C->B[c * Q7 + q];
        }
        phi[c] = (a + b) != 0.0 ? (a - b) / (a + b) : 0.0;
    }
}

void orc_colour_set_collision(orc_colour *C, int on) { C->L->collide = on; }
