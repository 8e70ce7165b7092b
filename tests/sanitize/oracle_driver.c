/* Host driver of the FP64 oracle for the sanitizer build (test
 * infrastructure): exercises streaming with every z treatment and side
 * periodicity, the flux inlet and pressure outlet, BGK and MRT collision,
 * the plain inlet density, the two-fluid step, its colour gradient and the
 * field read-outs on small random boxes, then frees everything. Built with
 * -fsanitize=address,undefined by tests/test_host_sanitizers.py; exits
 * non-zero when a conservation check fails. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct orc_lattice orc_lattice;
typedef struct orc_colour orc_colour;
orc_lattice *orc_create(int nx, int ny, int nz, const unsigned char *solid, int periodic_x, int periodic_y,
                        int z_mode, double tau, double rho0, double q_target, double rho_out);
void orc_destroy(orc_lattice *L);
void orc_set_mrt(orc_lattice *L, int on);
void orc_init_equilibrium(orc_lattice *L, double rho, double ux, double uy, double uz);
void orc_set_f(orc_lattice *L, const double *f);
void orc_get_f(const orc_lattice *L, double *f);
void orc_fields(const orc_lattice *L, double *rho, double *ux, double *uy, double *uz);
int orc_step(orc_lattice *L, int n, double *hist);
double orc_plain_inlet_density(orc_lattice *L);
void orc_set_inlet_offset(orc_lattice *L, double d);
orc_colour *orc_colour_create(int nx, int ny, int nz, const unsigned char *solid, int periodic_x, int periodic_y,
                              int z_mode, double tau, double rho0, double q_target, double rho_out, double alpha,
                              double beta, double phi_solid);
void orc_colour_destroy(orc_colour *C);
void orc_colour_init(orc_colour *C, const double *na, const double *nb);
int orc_colour_step(orc_colour *C, int n, double *hist);
void orc_colour_gradient(const orc_colour *C, const double *phi, double *grad);
void orc_colour_fields(const orc_colour *C, double *rho, double *ux, double *uy, double *uz, double *phi);

static unsigned long long rng = 88172645463325252ULL;
static double uni(void)
{
    rng ^= rng << 13;
    rng ^= rng >> 7;
    rng ^= rng << 17;
    return (double)(rng >> 11) * (1.0 / 9007199254740992.0);
}

static int single_fluid(int nx, int ny, int nz, int px, int py, int z_mode, int mrt)
{
    const long n = (long)nx * ny * nz;
    unsigned char *solid = (unsigned char *)malloc((size_t)n);
    for (long c = 0; c < n; ++c) solid[c] = uni() < 0.25;
    for (long c = 0; c < (long)nx * ny; ++c) solid[c] = 0; /* an open inlet plane */
    orc_lattice *L = orc_create(nx, ny, nz, solid, px, py, z_mode, 0.8, 1.0, 0.02 * nx * ny, 1.0);
    if (!L) {
        free(solid);
        return 1;
    }
    orc_set_mrt(L, mrt);
    double *f = (double *)malloc((size_t)n * 19 * sizeof(double));
    orc_init_equilibrium(L, 1.0, 0.0, 0.0, 0.01);
    orc_get_f(L, f);
    for (long i = 0; i < n * 19; ++i) f[i] *= 1.0 + 0.02 * (uni() - 0.5);
    orc_set_f(L, f);
    double hist[5 * 12];
    int bad = 0;
    if (orc_step(L, 12, hist) != 0) bad = 1;
    if (z_mode == 0) {
        const double rp = orc_plain_inlet_density(L);
        orc_set_inlet_offset(L, 0.0);
        double h[5];
        if (orc_step(L, 1, h) != 0 || fabs(h[0] - rp) > 1e-12) bad = 1;
    } else if (!(fabs(hist[11 * 5 + 3] - hist[3]) <= 1e-10 * fabs(hist[3]))) {
        bad = 1; /* closed box: the mass of step 12 equals that of step 1 */
    }
    double *rho = (double *)malloc((size_t)n * 4 * sizeof(double));
    orc_fields(L, rho, rho + n, rho + 2 * n, rho + 3 * n);
    free(rho);
    free(f);
    orc_destroy(L);
    free(solid);
    return bad;
}

static int two_fluid(int nx, int ny, int nz, int px, int py, int z_mode)
{
    const long n = (long)nx * ny * nz;
    unsigned char *solid = (unsigned char *)malloc((size_t)n);
    for (long c = 0; c < n; ++c) solid[c] = uni() < 0.2;
    for (long c = 0; c < (long)nx * ny; ++c) solid[c] = 0;
    orc_colour *C = orc_colour_create(nx, ny, nz, solid, px, py, z_mode, 1.0, 1.0, 0.01 * nx * ny, 1.0, 0.0157,
                                      0.7, -0.7071);
    if (!C) {
        free(solid);
        return 1;
    }
    double *na = (double *)malloc((size_t)n * sizeof(double)), *nb = (double *)malloc((size_t)n * sizeof(double));
    for (long c = 0; c < n; ++c) {
        na[c] = (c < 2L * nx * ny) ? 1.0 : 0.0;
        nb[c] = 1.0 - na[c];
    }
    orc_colour_init(C, na, nb);
    double hist[7 * 10];
    int bad = orc_colour_step(C, 10, hist) != 0;
    if (z_mode != 0 && !(fabs(hist[9 * 7 + 5] - hist[5]) <= 1e-10 * fabs(hist[5]))) bad = 1; /* colour conserved */
    double *fld = (double *)malloc((size_t)n * 5 * sizeof(double));
    orc_colour_fields(C, fld, fld + n, fld + 2 * n, fld + 3 * n, fld + 4 * n);
    double *grad = (double *)malloc((size_t)n * 3 * sizeof(double));
    orc_colour_gradient(C, fld + 4 * n, grad);
    free(grad);
    free(fld);
    free(na);
    free(nb);
    orc_colour_destroy(C);
    free(solid);
    return bad;
}

int main(void)
{
    int fails = 0;
    for (int z_mode = 0; z_mode < 3; ++z_mode)
        for (int p = 0; p < 4; ++p) {
            fails += single_fluid(5 + p, 4 + (p & 1), 6 + z_mode, p & 1, (p >> 1) & 1, z_mode, p == 3);
            fails += two_fluid(6, 5 + p, 7, p & 1, (p >> 1) & 1, z_mode);
        }
    if (orc_create(0, 4, 4, NULL, 1, 1, 0, 0.8, 1.0, 0.0, 1.0) != NULL) ++fails; /* rejected arguments */
    printf("oracle driver: %d failures\n", fails);
    return fails ? 1 : 0;
}
