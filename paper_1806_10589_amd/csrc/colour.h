// gfx950 kernels of the two-fluid colour-gradient step (Appendix A).
//
// State: momentum distributions f (D3Q19, deviations g = f - w_q, as for the
// single fluid) and the two colours' D3Q7 distributions A (non-wetting) and B
// (wetting), absolute values, [7][n_pad] each. One step is two launches:
//   k_phase   pull A, B (halfway bounce-back, inlet/outlet unknowns) and write
//             N_A, N_B and the phase field phi = (N_A - N_B)/(N_A + N_B);
//   k_colour  pull f with the flux inlet / pressure outlet, colour gradient
//             C = 3 sum_q w_q xi_q phi(x + xi_q) from the neighbours' phi,
//             MRT collision with the interfacial stress, recolouring of A and
//             B, store.
// The colour gradient needs phi at every neighbour after this step's
// streaming, which is why the phase field is its own pass.
#pragma once
#include "kernels.h"

namespace flbm {

// Storage of the colour state (A, B, N_A, N_B, phi): the momentum storage
// type, except that the FP16-deviation mode keeps the colours in FP32
// (absolute colour fractions in FP16 would break colour conservation at the
// 1e-4 level every step).
template <typename T> struct ColourStore { using type = T; };
template <> struct ColourStore<_Float16> { using type = float; };

// phi of the neighbour that pull direction p reads from, decoded from the
// pull index: a regular pull q*n_pad + src gives phi[src]; bounce-back (a
// solid or a non-periodic side) gives the wetting value phi_solid; a source
// beyond the open z faces gives the site's own phi.
template <typename T>
__device__ __forceinline__ double neighbour_phi(const T *__restrict__ phi, int32_t idx, int p, int64_t npad,
                                                int64_t sentinel, double own, double phi_solid)
{
    const int64_t lo = (int64_t)p * npad;
    if (idx >= lo && idx < lo + npad) return (double)phi[idx - lo];
    return idx == sentinel ? own : phi_solid;
}

struct PhaseArgs {
    int64_t n, npad, a_in, out0, sentinel;
    int32_t flux_mode, rd;
    double rho0;
    DevState *st;
    const int32_t *nbr;
    const void *fin;                // momentum state (storage type)
    const void *ain, *bin;          // colour state read this step
    void *aout, *bout;              // written only when collision is off
    void *na, *nb, *phi;            // phase field outputs [n_pad]
};

// Phase pass: one site per thread.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_phase(PhaseArgs p)
{
    using R = typename Compute<T>::type;
    using C = typename ColourStore<T>::type;
    const int64_t s = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    const int64_t npad = p.npad;
    const C *ain = (const C *)p.ain, *bin = (const C *)p.bin;
    R a[7], b[7];
    a[0] = (R)ain[s];
    b[0] = (R)bin[s];
#pragma unroll
    for (int q = 1; q < 7; ++q) {
        const int32_t idx = p.nbr[(int64_t)(q - 1) * npad + s];
        const bool known = idx < (int64_t)7 * npad;  // the sentinel marks a boundary unknown
        a[q] = known ? (R)ain[idx] : (R)0;
        b[q] = known ? (R)bin[idx] : (R)0;
    }
    if (p.flux_mode && (s < p.a_in || (s >= p.out0 && s < p.n))) {
        // the site's boundary velocity, from the pulled momentum knowns
        const T *fin = (const T *)p.fin;
        R g[19];
        g[0] = Codec<T>::dec(fin[s], 0);
#pragma unroll
        for (int q = 1; q < 19; ++q) {
            const int32_t idx = p.nbr[(int64_t)(q - 1) * npad + s];
            g[q] = idx == p.sentinel ? (R)0 : Codec<T>::dec(fin[idx], q);
        }
        const DevState *st = p.st;
        if (s < p.a_in) {
            // pure non-wetting injection: A_5 = w_5 (1 + 9/2 u_z), B_5 = 0
            const double drho_in = inlet_drho(st, p.rd, p.rho0, p.a_in);
            const double uz = inlet_velocity(g, drho_in, p.rho0);
            a[5] = (R)(d3q19::weight7(5) * (1.0 + 4.5 * uz));
            b[5] = (R)0;
        } else {
            // outflow: equilibrium of the site's previous colour densities
            const double uz = outlet_velocity(g, st->drho_out, p.rho0);
            double na_prev = 0.0, nb_prev = 0.0;
#pragma unroll
            for (int q = 0; q < 7; ++q) {
                na_prev += (double)ain[(int64_t)q * npad + s];
                nb_prev += (double)bin[(int64_t)q * npad + s];
            }
            a[6] = (R)(d3q19::weight7(6) * na_prev * (1.0 - 4.5 * uz));
            b[6] = (R)(d3q19::weight7(6) * nb_prev * (1.0 - 4.5 * uz));
        }
    }
    R na = 0, nb = 0;
#pragma unroll
    for (int q = 0; q < 7; ++q) {
        na += a[q];
        nb += b[q];
    }
    const R tot = na + nb;
    // non-temporal: the colour step reads these once per site (phi also from
    // the neighbours), after the whole pass has been written
    __builtin_nontemporal_store((C)na, &((C *)p.na)[s]);
    __builtin_nontemporal_store((C)nb, &((C *)p.nb)[s]);
    __builtin_nontemporal_store((C)(tot != (R)0 ? (na - nb) / tot : (R)0), &((C *)p.phi)[s]);
    if (p.st->omega == 0.0) {
        // testing aid (collision off): keep the streamed colours
#pragma unroll
        for (int q = 0; q < 7; ++q) {
            ((C *)p.aout)[(int64_t)q * npad + s] = (C)a[q];
            ((C *)p.bout)[(int64_t)q * npad + s] = (C)b[q];
        }
    }
}

struct ColourStepArgs {
    double alpha, beta, phi_solid;
    int64_t sentinel;
    const void *na, *nb, *phi;
    void *aout, *bout;
};

// Colour step: TILE threads per tile, one site per thread.
template <typename T, bool OBS>
__global__ __launch_bounds__(TILE, (sizeof(T) <= 4 && !OBS) ? 6 : 1) void k_colour(const T *__restrict__ fin, T *__restrict__ fout,
                                                 const int32_t *__restrict__ nbr, StepArgs a,
                                                 ColourStepArgs c)
{
    using R = typename Compute<T>::type;
    using C = typename ColourStore<T>::type;
    const int tile = (int)blockIdx.x;
    const int64_t s = (int64_t)tile * TILE + threadIdx.x;
    const int64_t npad = a.npad;
    const C *phi = (const C *)c.phi;

    // pull f, and with the same indices the colour gradient: the neighbour
    // x + xi_q is the source of pull direction opp(q), so
    // C = -3 sum_p w_p xi_p phi(source of p)
    R g[19];
    g[0] = Codec<T>::dec(fin[s], 0);
    const double own = (double)phi[s];
    R gx = 0, gy = 0, gz = 0;
#pragma unroll
    for (int q = 1; q < 19; ++q) {
        const int32_t idx = nbr[(int64_t)(q - 1) * npad + s];
        g[q] = Codec<T>::dec(fin[idx], q);
        const R ph = (R)neighbour_phi(phi, idx, q, npad, c.sentinel, own, c.phi_solid);
        const R w3 = (R)(3.0 * d3q19::weight(q));
        if (d3q19::cx[q]) gx -= d3q19::cx[q] * w3 * ph;
        if (d3q19::cy[q]) gy -= d3q19::cy[q] * w3 * ph;
        if (d3q19::cz[q]) gz -= d3q19::cz[q] * w3 * ph;
    }

    double uz_in = 0.0, uz_out = 0.0;
    if (tile < a.nt_in && s < a.a_in) {
        const double drho_in = inlet_drho(a.st, a.rd, a.rho0, a.a_in);
        uz_in = inlet_condition(g, drho_in, a.rho0);
    }
    if (tile >= a.tout0 && s >= a.out0 && s < a.n) uz_out = outlet_condition(g, a.st->drho_out, a.rho0);

    const R snu = (R)a.st->omega;
    const bool collide = snu != (R)0;
    R drho, ux, uy, uz;
    if (collide) {
        mrt_collide<true>(g, snu, (R)a.rho0, (R)a.inv_rho0, (R)c.alpha, gx, gy, gz, drho, ux, uy, uz);
        conserve_mass<T>(g, drho, (uint32_t)s);
    } else {
        drho = ux = uy = uz = 0;
#pragma unroll
        for (int q = 0; q < 19; ++q) drho += g[q];
    }

    // the next inlet sum (as in the single-fluid kernel)
    double s_next = 0.0;
    if (tile < a.nt01 && s < a.n01) {
        const uint64_t cw = a.kcoef[s];
#pragma unroll
        for (int q = 0; q < 19; ++q) {
            const uint32_t cc = (uint32_t)(cw >> (2 * q)) & 3u;
            if (cc) s_next += (double)cc * (double)Codec<T>::dec(Codec<T>::enc(g[q], q, (uint32_t)s), q);
        }
    }

#pragma unroll
    for (int q = 0; q < 19; ++q)
        __builtin_nontemporal_store(Codec<T>::enc(g[q], q, (uint32_t)s), &fout[(int64_t)q * npad + s]);

    // recolouring: full relaxation of A and B to
    //   w_q N_A [1 + 9/2 u.xi_q + beta N_B n.xi_q],  w_q N_B [1 + 9/2 u.xi_q - beta N_A n.xi_q]
    const R na = (R)((const C *)c.na)[s], nb = (R)((const C *)c.nb)[s];
    if (collide) {
        const R cm2 = gx * gx + gy * gy + gz * gz;
        R nx = 0, ny = 0, nz = 0;
        if (cm2 > (R)1e-12) {
            const R inv = (R)1 / sqrt(cm2);
            nx = gx * inv;
            ny = gy * inv;
            nz = gz * inv;
        }
        const R bab = (R)c.beta * na * nb;
        C *aout = (C *)c.aout, *bout = (C *)c.bout;
#pragma unroll
        for (int q = 0; q < 7; ++q) {
            R cu = 0, cn = 0;
            if (d3q19::cx[q]) {
                cu += d3q19::cx[q] > 0 ? ux : -ux;
                cn += d3q19::cx[q] > 0 ? nx : -nx;
            }
            if (d3q19::cy[q]) {
                cu += d3q19::cy[q] > 0 ? uy : -uy;
                cn += d3q19::cy[q] > 0 ? ny : -ny;
            }
            if (d3q19::cz[q]) {
                cu += d3q19::cz[q] > 0 ? uz : -uz;
                cn += d3q19::cz[q] > 0 ? nz : -nz;
            }
            const R w = (R)d3q19::weight7(q);
            const R adv = (R)1 + (R)4.5 * cu;
            __builtin_nontemporal_store((C)(w * (na * adv + bab * cn)), &aout[(int64_t)q * npad + s]);
            __builtin_nontemporal_store((C)(w * (nb * adv - bab * cn)), &bout[(int64_t)q * npad + s]);
        }
    }

    double m = 0.0;
    float u2max = 0.f;
    uint32_t bad = 0;
    if (OBS) {
        m = (double)drho;
        u2max = (float)(ux * ux + uy * uy + uz * uz);
        bad = !isfinite((double)drho + (double)ux + (double)uy + (double)uz + (double)na + (double)nb);
    }
    step_epilogue<TILE, OBS, true>(tile, uz_in, uz_out, s_next, m, u2max, bad, a, (double)na, (double)nb);
}

// Phase field of a stored colour state (for readout): phi from the stored A, B.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_phase_of_state(const T *__restrict__ A, const T *__restrict__ B,
                                                          int64_t n, int64_t npad, double *__restrict__ out)
{
    const int64_t s = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (s >= n) return;
    double na = 0.0, nb = 0.0;
#pragma unroll
    for (int q = 0; q < 7; ++q) {
        na += (double)A[(int64_t)q * npad + s];
        nb += (double)B[(int64_t)q * npad + s];
    }
    out[s] = (na + nb) != 0.0 ? (na - nb) / (na + nb) : 0.0;
}

}  // namespace flbm
