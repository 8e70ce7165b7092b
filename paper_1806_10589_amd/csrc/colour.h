// gfx950 kernels of the two-fluid colour-gradient step (Appendix A).
//
// State: momentum distributions f (D3Q19, deviations g = f - w_q, as for the
// single fluid) and the two colours' D3Q7 distributions A (non-wetting) and B
// (wetting), absolute values, stored as pairs (A_q, B_q) in [7][n_pad]: the
// two colours of one direction and site are always read together (pulled
// from the same source) and written together, so one pair access replaces
// two. One step is two launches:
//   k_phase   pull A, B (halfway bounce-back, inlet/outlet unknowns) and write
//             the pair (N_A, N_B) and the phase field
//             phi = (N_A - N_B)/(N_A + N_B);
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

// A pair of colour values (A then B; N_A then N_B) as one vector access.
template <typename C> struct Pair { typedef C type __attribute__((ext_vector_type(2))); };

// Stores of a colour pair (A, B) never exceed 8 bytes per lane: on gfx950 a
// 16-byte vector store whose data registers the very next instruction
// overwrites has stored the overwriting value in some lanes (the last four
// of each group of sixteen), and the compiler emitted exactly that order for
// FP64 pairs. Such a pair is stored as its two halves, with a compiler
// barrier between them so that they are not merged back; FP32 pairs (8
// bytes) stay one store.
template <typename C>
__device__ __forceinline__ void store_pair(typename Pair<C>::type *dst, C a, C b, bool nt)
{
    if constexpr (sizeof(C) <= 4) {
        if (nt)
            __builtin_nontemporal_store(typename Pair<C>::type{a, b}, dst);
        else
            *dst = typename Pair<C>::type{a, b};
    } else {
        C *d = (C *)dst;
        if (nt)
            __builtin_nontemporal_store(a, d);
        else
            d[0] = a;
        __asm__ __volatile__("" ::: "memory");
        if (nt)
            __builtin_nontemporal_store(b, d + 1);
        else
            d[1] = b;
    }
}

// The same through a buffer descriptor (non-temporal), pair element i of
// the array the descriptor covers, row offset soff in bytes.
template <typename C>
__device__ __forceinline__ void buf_store_pair_nt(__amdgpu_buffer_rsrc_t r, uint32_t i, uint32_t soff, C a, C b)
{
    typedef typename RawBits<sizeof(C)>::type CB;
    if constexpr (sizeof(C) <= 4) {
        typedef typename RawBits<2 * sizeof(C)>::type CB2;
        buf_store_raw_nt<2 * sizeof(C)>(__builtin_bit_cast(CB2, typename Pair<C>::type{a, b}), r,
                                        i * 2u * (uint32_t)sizeof(C), soff);
    } else {
        buf_store_raw_nt<sizeof(C)>(__builtin_bit_cast(CB, a), r, i * 2u * (uint32_t)sizeof(C), soff);
        __asm__ __volatile__("" ::: "memory");
        buf_store_raw_nt<sizeof(C)>(__builtin_bit_cast(CB, b), r, i * 2u * (uint32_t)sizeof(C) + (uint32_t)sizeof(C),
                                    soff);
    }
}

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
    const void *abin;               // colour pairs read this step [7][n_pad]
    void *about;                    // written only when collision is off
    void *nab, *phi;                // outputs: (N_A, N_B) pairs and phi, [n_pad]
};

// Phase pass: one site per thread.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_phase(PhaseArgs p)
{
    using R = typename Compute<T>::type;
    using C = typename ColourStore<T>::type;
    typedef typename Pair<C>::type C2;
    const int64_t s = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    const int64_t npad = p.npad;
    const C2 *abin = (const C2 *)p.abin;
    R a[7], b[7];
    {
        const C2 v = abin[s];
        a[0] = (R)v[0];
        b[0] = (R)v[1];
    }
#pragma unroll
    for (int q = 1; q < 7; ++q) {
        const int32_t idx = p.nbr[(int64_t)(q - 1) * npad + s];
        const bool known = idx < (int64_t)7 * npad;  // the sentinel marks a boundary unknown
        const C2 v = abin[known ? (int64_t)idx : s];
        a[q] = known ? (R)v[0] : (R)0;
        b[q] = known ? (R)v[1] : (R)0;
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
            // (s_carry[rd] holds the inlet sum: the colour model ends every
            // step in a launch of its own)
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
                const C2 v = abin[(int64_t)q * npad + s];
                na_prev += (double)v[0];
                nb_prev += (double)v[1];
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
    store_pair<C>(&((C2 *)p.nab)[s], (C)na, (C)nb, true);
    __builtin_nontemporal_store((C)(tot != (R)0 ? (na - nb) / tot : (R)0), &((C *)p.phi)[s]);
    if (p.st->omega == 0.0) {
        // testing aid (collision off): keep the streamed colours
#pragma unroll
        for (int q = 0; q < 7; ++q) store_pair<C>(&((C2 *)p.about)[(int64_t)q * npad + s], (C)a[q], (C)b[q], false);
    }
}

struct ColourStepArgs {
    double alpha, beta, phi_solid;
    int64_t sentinel;
    const void *nab, *phi;          // (N_A, N_B) pairs and phi of this step, [n_pad]
    void *about;                    // recoloured pairs (A_q, B_q) [7][n_pad]
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
    const double drho_in = step_begin<TILE>(tile, a, a.rd);

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
    if (tile < a.nt_in && s < a.a_in) uz_in = inlet_condition(g, drho_in, a.rho0);
    if (tile >= a.tout0 && s >= a.out0 && s < a.n) uz_out = outlet_condition(g, cst(a.st)->drho_out, a.rho0);

    const R snu = (R)cst(a.st)->omega;
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
    typedef typename Pair<C>::type C2;
    const C2 nv = ((const C2 *)c.nab)[s];
    const R na = (R)nv[0], nb = (R)nv[1];
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
        C2 *about = (C2 *)c.about;
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
            store_pair<C>(&about[(int64_t)q * npad + s], (C)(w * (na * adv + bab * cn)), (C)(w * (nb * adv - bab * cn)),
                          true);
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
    step_epilogue<TILE, OBS, true>(tile, uz_in, uz_out, s_next, m, u2max, bad, a, a.rd, (double)na, (double)nb);
}

// ---------------------------------------------------------------- buffer path
//
// The two passes on the path the single-fluid step takes when every buffer is
// below 4 GiB: raw buffer instructions (base and size in an SGPR descriptor,
// 32-bit lane offsets), non-temporal stores, and the compact pull table (8-bit
// or 16-bit codes per 512-site tile, or the int32 rows; every form addresses
// the same slots). The colour step's collision is written in two-rate form
// (see trt_stress_collide below), which needs a fraction of the registers of
// the moment transform.

// How a pulled population is reached: a regular source, the boundary unknown
// of an open z face, or halfway bounce-back off a solid or a wall.
enum { PULL_REG = 0, PULL_UNK = 1, PULL_BB = 2 };

// Flat pull index (into a [rows][n_pad] array) and kind of direction q for a
// site at position p of its tile, from a code of the tile's form; bb is the
// site's own slot of direction opp(q), sent the open-face sentinel.
template <int FORM>
__device__ __forceinline__ uint32_t decode_pull(uint32_t code, uint32_t base, uint32_t p, uint32_t bb,
                                                uint32_t sent, uint32_t q, uint32_t npad, int &kind)
{
    if constexpr (FORM == PULL_TILE_BYTE) {
        kind = code <= PULL_MAX_BYTE ? PULL_REG : (code == PULL_BYTE_BOUNCE ? PULL_BB : PULL_UNK);
        return code <= PULL_MAX_BYTE ? base + p + code : (code == PULL_BYTE_BOUNCE ? bb : sent);
    } else if constexpr (FORM == PULL_TILE_HALF) {
        kind = code <= PULL_MAX_CODE ? PULL_REG : (code == PULL_BOUNCE ? PULL_BB : PULL_UNK);
        return code <= PULL_MAX_CODE ? base + code : (code == PULL_BOUNCE ? bb : sent);
    } else {
        // int32 row: code is the flat index itself
        const uint32_t rel = code - q * npad;
        kind = rel < npad ? PULL_REG : (code == sent ? PULL_UNK : PULL_BB);
        return code;
    }
}

// The code of direction q (1..18) of this thread's site from the words of
// its tile's form, loaded once per site.
template <int FORM>
__device__ __forceinline__ uint32_t pull_code(const uint32_t (&w)[9], uint32_t tail, int q)
{
    if constexpr (FORM == PULL_TILE_BYTE)
        return q <= 16 ? (w[(q - 1) >> 2] >> (((q - 1) & 3) * 8)) & 0xFFu : (tail >> ((q - 17) * 8)) & 0xFFu;
    else if constexpr (FORM == PULL_TILE_HALF)
        return ((q - 1) & 1) ? (w[(q - 1) >> 1] >> 16) : (w[(q - 1) >> 1] & 0xFFFFu);
    else
        return 0u;  // int32 rows are loaded per direction
}

// Load the code words of directions 1..Q1 for the site at s (lane offset
// 4 s) from the tile's form.
template <int FORM, int Q1>
__device__ __forceinline__ void load_pull_words(const StepArgs &a, uint32_t s, uint32_t npad, uint32_t (&w)[9],
                                                uint32_t &tail)
{
    constexpr int AUX = SC_IDX_AUX;
    if constexpr (FORM == PULL_TILE_BYTE) {
        const __amdgpu_buffer_rsrc_t rb = make_rsrc(a.pull_bytes, a.bytes_bytes);
#pragma unroll
        for (int k = 0; k < (Q1 + 3) / 4 && k < 4; ++k)
            w[k] = buf_load_raw<4, AUX>(rb, s * 4u, (uint32_t)k * npad * 4u);
        if constexpr (Q1 > 16) tail = buf_load_raw<2, AUX>(rb, s * 2u, 16u * npad);
    } else if constexpr (FORM == PULL_TILE_HALF) {
        const __amdgpu_buffer_rsrc_t rc = make_rsrc(a.pull_codes, a.codes_bytes);
#pragma unroll
        for (int k = 0; k < (Q1 + 1) / 2; ++k) w[k] = buf_load_raw<4, AUX>(rc, s * 4u, (uint32_t)k * npad * 4u);
    }
}

// Two-rate form of the colour step's collision (Appendix A). With the rates
// of Appendix A every even moment that is not conserved relaxes at s_nu and
// every odd one at s_q; conserved moments have no non-equilibrium part. The
// even moments span the part of g symmetric under xi -> -xi, the odd ones
// the antisymmetric part, so the moment-space relaxation
//   g += M^T diag(1/|M_k|^2) (-S (M g - m_eq - dm))
// is, direction by direction,
//   g_q += -s_nu (g_q^+ - e_q - d_q) - s_q (g_q^- - o_q),
// g^+- the symmetric / antisymmetric parts (g_q +- g_opp(q))/2, e_q and o_q
// the even and odd parts of the incompressible equilibrium in deviation form
// (w_q [rho - 1 + rho0 (9/2 (xi.u)^2 - 3/2 u.u)] and 3 w_q rho0 xi.u), and
// d = M^T diag(1/|M_k|^2) dm the interfacial stress alpha |C| (19,
// (2n_x^2 - n_y^2 - n_z^2)/2, (n_y^2 - n_z^2)/2, n_x n_y/2, n_y n_z/2,
// n_x n_z/2) on (e, 3p_xx, p_ww, p_xy, p_yz, p_xz) taken back to directions
// (even, so d_q = d_opp(q)). Equal to mrt_collide<true> up to rounding.
template <typename R>
__device__ __forceinline__ void trt_stress_collide(R (&g)[19], R snu, R rho0, R inv_rho0, R alpha, R gx, R gy,
                                                   R gz, R &drho, R &ux, R &uy, R &uz)
{
    R d = g[0], jx = 0, jy = 0, jz = 0;
#pragma unroll
    for (int q = 1; q < 19; q += 2) {
        const R sum = g[q] + g[q + 1], dif = g[q] - g[q + 1];
        d += sum;
        if (d3q19::cx[q]) jx += d3q19::cx[q] > 0 ? dif : -dif;
        if (d3q19::cy[q]) jy += d3q19::cy[q] > 0 ? dif : -dif;
        if (d3q19::cz[q]) jz += d3q19::cz[q] > 0 ? dif : -dif;
    }
    drho = d;
    ux = jx * inv_rho0;
    uy = jy * inv_rho0;
    uz = jz * inv_rho0;

    // stress moments alpha C_a C_b / |C| (zero where |C| <= 1e-6)
    const R cm2 = gx * gx + gy * gy + gz * gz;
    R ac = 0, sxx = 0, syy = 0, szz = 0, sxy = 0, syz = 0, sxz = 0;
    if (cm2 > (R)1e-12) {
        const R cmag = sqrt(cm2);
        ac = alpha * cmag;
        const R f = alpha / cmag;
        sxx = f * gx * gx;
        syy = f * gy * gy;
        szz = f * gz * gz;
        sxy = f * gx * gy;
        syz = f * gy * gz;
        sxz = f * gx * gz;
    }
    const R dm1 = (R)19 * ac, dm9 = (R)0.5 * ((R)2 * sxx - syy - szz), dm11 = (R)0.5 * (syy - szz);
    const R dm13 = (R)0.5 * sxy, dm14 = (R)0.5 * syz, dm15 = (R)0.5 * sxz;

    const R sq = (R)8 * ((R)2 - snu) / ((R)8 - snu);
    const R base = d - rho0 * (R)1.5 * (ux * ux + uy * uy + uz * uz);
    // rest direction: symmetric only
    {
        const double c1 = (double)d3q19::mb(1, 0) / d3q19::mb_norm2(1);
        const R e0 = (R)(1.0 / 3.0) * base;
        g[0] -= snu * (g[0] - e0 - (R)c1 * dm1);
    }
#pragma unroll
    for (int q = 1; q < 19; q += 2) {
        R cu = 0;
        if (d3q19::cx[q]) cu += d3q19::cx[q] > 0 ? ux : -ux;
        if (d3q19::cy[q]) cu += d3q19::cy[q] > 0 ? uy : -uy;
        if (d3q19::cz[q]) cu += d3q19::cz[q] > 0 ? uz : -uz;
        const R w = (R)d3q19::weight(q);
        // d_q from the stress moments: basis entry over the row's squared norm
        const double k1 = (double)d3q19::mb(1, q) / d3q19::mb_norm2(1);
        const double k9 = (double)d3q19::mb(9, q) / d3q19::mb_norm2(9);
        const double k11 = (double)d3q19::mb(11, q) / d3q19::mb_norm2(11);
        const double k13 = (double)d3q19::mb(13, q) / d3q19::mb_norm2(13);
        const double k14 = (double)d3q19::mb(14, q) / d3q19::mb_norm2(14);
        const double k15 = (double)d3q19::mb(15, q) / d3q19::mb_norm2(15);
        R dq = (R)k1 * dm1;
        if (k9 != 0.0) dq += (R)k9 * dm9;
        if (k11 != 0.0) dq += (R)k11 * dm11;
        if (k13 != 0.0) dq += (R)k13 * dm13;
        if (k14 != 0.0) dq += (R)k14 * dm14;
        if (k15 != 0.0) dq += (R)k15 * dm15;
        const R even = w * (base + rho0 * (R)4.5 * cu * cu) + dq;
        const R odd = w * rho0 * (R)3 * cu;
        const R sp = (R)0.5 * (g[q] + g[q + 1]), sm = (R)0.5 * (g[q] - g[q + 1]);
        const R rp = snu * (sp - even), rm = sq * (sm - odd);
        g[q] -= rp + rm;
        g[q + 1] -= rp - rm;
    }
}

#ifndef FLBM_PHASE_V
#define FLBM_PHASE_V 1
#endif
#ifndef FLBM_COLOUR_NSUM
#define FLBM_COLOUR_NSUM 1
#endif
// Sites per thread of the phase pass (TILE / PHASE_V threads per tile). Two
// sites per thread take 77 VGPRs instead of 58 and were measured slower on a
// 256^3 pack (105 vs 98 us), as were 256- and 1024-thread blocks of one site
// per thread.
constexpr int PHASE_V = FLBM_PHASE_V;
// The phase pass hands the colour step N = N_A + N_B and phi instead of the
// pair (N_A, N_B): the colour step reads phi at the site anyway (its gradient
// reads the neighbours' phi), and recovers N_A = N (1 + phi)/2, N_B =
// N (1 - phi)/2, which equal the pair up to rounding; 4 bytes less written
// and 4 less read per site.
constexpr bool COLOUR_NSUM = FLBM_COLOUR_NSUM;

// The colour densities of a site from what the phase pass stored.
template <typename R, typename C>
__device__ __forceinline__ void colour_densities(const void *nab, const void *phi, uint32_t s, uint32_t npad,
                                                 R &na, R &nb)
{
    constexpr uint32_t ES = sizeof(C);
    if constexpr (COLOUR_NSUM) {
        const R n = (R)__builtin_bit_cast(C, buf_load_raw<ES>(make_rsrc(nab, npad * ES), s * ES, 0u));
        const R ph = (R)__builtin_bit_cast(C, buf_load_raw<ES>(make_rsrc(phi, npad * ES), s * ES, 0u));
        na = (R)0.5 * n * ((R)1 + ph);
        nb = (R)0.5 * n * ((R)1 - ph);
    } else {
        typedef typename Pair<C>::type C2;
        const C2 v = __builtin_bit_cast(C2, buf_load_raw<2 * ES>(make_rsrc(nab, npad * 2 * ES), s * 2 * ES, 0u));
        na = (R)v[0];
        nb = (R)v[1];
    }
}

// Phase pass, buffer path: PHASE_V sites per thread, TILE sites per block.
template <typename T>
__global__ __launch_bounds__(TILE / PHASE_V) void k_phase_buf(PhaseArgs p, StepArgs a)
{
    using R = typename Compute<T>::type;
    using C = typename ColourStore<T>::type;
    typedef typename Pair<C>::type C2;
    constexpr int V = PHASE_V, NT = TILE / PHASE_V;
    constexpr int PB = 2 * sizeof(C);  // bytes of a colour pair
    const uint32_t npad = (uint32_t)p.npad;
    const int tile = (int)blockIdx.x;
    const uint32_t pos0 = threadIdx.x;
    const __amdgpu_buffer_rsrc_t rab = make_rsrc(p.abin, 7u * npad * (uint32_t)PB);
    const uint32_t esz = (uint32_t)sizeof(C);
    const int32_t *hdr = a.pull_hdr ? a.pull_hdr + (int64_t)tile * PULL_HDR : nullptr;
    const int form = hdr ? (int)hdr_entry(hdr, PULL_HDR_FORM) : PULL_TILE_INT32;
    const uint32_t sent = 19u * npad;
    uint32_t pos[V], s[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
        pos[v] = pos0 + (uint32_t)(v * NT);
        s[v] = (uint32_t)tile * TILE + pos[v];
    }
    R av[V][7], bv[V][7];
#pragma unroll
    for (int v = 0; v < V; ++v) {
        const C2 x = __builtin_bit_cast(C2, buf_load_raw<PB>(rab, s[v] * (uint32_t)PB, 0u));
        av[v][0] = (R)x[0];
        bv[v][0] = (R)x[1];
    }
    auto gather = [&](auto form_tag) {
        constexpr int FORM = decltype(form_tag)::value;
        uint32_t w[V][9], tail[V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
#pragma unroll
            for (int k = 0; k < 9; ++k) w[v][k] = 0;
            tail[v] = 0;
            load_pull_words<FORM, 6>(a, s[v], npad, w[v], tail[v]);
        }
        const __amdgpu_buffer_rsrc_t rn = make_rsrc(p.nbr, a.nbr_bytes);
#pragma unroll
        for (int q = 1; q < 7; ++q) {
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const uint32_t code =
                    FORM == PULL_TILE_INT32
                        ? (uint32_t)buf_load_raw<4, SC_IDX_AUX>(rn, s[v] * 4u, (uint32_t)(q - 1) * npad * 4u)
                        : pull_code<FORM>(w[v], tail[v], q);
                int kind;
                const uint32_t base = FORM == PULL_TILE_INT32 ? 0u : hdr_entry(hdr, q - 1);
                const uint32_t idx = decode_pull<FORM>(code, base, pos[v], (uint32_t)d3q19::opp(q) * npad + s[v],
                                                       sent, (uint32_t)q, npad, kind);
                // the colour array has 7 rows: an unknown reads the site's own
                // slot and is replaced by zero (the boundary fills it below)
                const uint32_t off = (kind == PULL_UNK ? s[v] : idx) * (uint32_t)PB;
                const C2 x = __builtin_bit_cast(C2, buf_load_raw<PB>(rab, off, 0u));
                av[v][q] = kind == PULL_UNK ? (R)0 : (R)x[0];
                bv[v][q] = kind == PULL_UNK ? (R)0 : (R)x[1];
            }
        }
    };
    if (form == PULL_TILE_BYTE)
        gather(std::integral_constant<int, PULL_TILE_BYTE>{});
    else if (form == PULL_TILE_HALF)
        gather(std::integral_constant<int, PULL_TILE_HALF>{});
    else
        gather(std::integral_constant<int, PULL_TILE_INT32>{});

    const bool boundary_tile = p.flux_mode && (tile < a.nt_in || tile >= a.tout0);
#pragma unroll
    for (int v = 0; v < V; ++v) {
        const int64_t sv = (int64_t)s[v];
        if (boundary_tile && (sv < p.a_in || (sv >= p.out0 && sv < p.n))) {
            // the site's boundary velocity, from the pulled momentum knowns
            // (few sites: plain loads of the int32 table)
            const T *fin = (const T *)p.fin;
            R g[19];
            g[0] = Codec<T>::dec(fin[sv], 0);
#pragma unroll
            for (int q = 1; q < 19; ++q) {
                const int32_t idx = p.nbr[(int64_t)(q - 1) * npad + sv];
                g[q] = idx == p.sentinel ? (R)0 : Codec<T>::dec(fin[idx], q);
            }
            const DevState *st = p.st;
            const C2 *abin = (const C2 *)p.abin;
            if (sv < p.a_in) {
                // pure non-wetting injection: A_5 = w_5 (1 + 9/2 u_z), B_5 = 0
                // (s_carry[rd] holds the inlet sum: the colour model ends
                // every step in a launch of its own)
                const double drho_in = inlet_drho(st, p.rd, p.rho0, p.a_in);
                const double uz = inlet_velocity(g, drho_in, p.rho0);
                av[v][5] = (R)(d3q19::weight7(5) * (1.0 + 4.5 * uz));
                bv[v][5] = (R)0;
            } else {
                // outflow: equilibrium of the site's previous colour densities
                const double uz = outlet_velocity(g, st->drho_out, p.rho0);
                double na_prev = 0.0, nb_prev = 0.0;
#pragma unroll
                for (int q = 0; q < 7; ++q) {
                    const C2 x = abin[(int64_t)q * npad + sv];
                    na_prev += (double)x[0];
                    nb_prev += (double)x[1];
                }
                av[v][6] = (R)(d3q19::weight7(6) * na_prev * (1.0 - 4.5 * uz));
                bv[v][6] = (R)(d3q19::weight7(6) * nb_prev * (1.0 - 4.5 * uz));
            }
        }
    }
    typedef typename RawBits<sizeof(C)>::type CB;
    const __amdgpu_buffer_rsrc_t rph = make_rsrc(p.phi, npad * esz);
#pragma unroll
    for (int v = 0; v < V; ++v) {
        R na = 0, nb = 0;
#pragma unroll
        for (int q = 0; q < 7; ++q) {
            na += av[v][q];
            nb += bv[v][q];
        }
        const R tot = na + nb;
        if constexpr (COLOUR_NSUM) {
            buf_store_raw_nt<sizeof(C)>(__builtin_bit_cast(CB, (C)tot), make_rsrc(p.nab, npad * esz), s[v] * esz, 0u);
        } else {
            buf_store_pair_nt<C>(make_rsrc(p.nab, npad * (uint32_t)PB), s[v], 0u, (C)na, (C)nb);
        }
        buf_store_raw_nt<sizeof(C)>(__builtin_bit_cast(CB, (C)(tot != (R)0 ? (na - nb) / tot : (R)0)), rph,
                                    s[v] * esz, 0u);
        if (p.st->omega == 0.0) {
            // testing aid (collision off): keep the streamed colours
#pragma unroll
            for (int q = 0; q < 7; ++q)
                store_pair<C>(&((C2 *)p.about)[(int64_t)q * npad + s[v]], (C)av[v][q], (C)bv[v][q], false);
        }
    }
}

// Colour step, buffer path: TILE threads per tile, one site per thread.
#ifndef FLBM_COLOUR_WAVES
#define FLBM_COLOUR_WAVES 6
#endif

// Minimum waves per SIMD the colour step is compiled for (FP32 and FP16
// storage): left to itself the compiler hoists all 36 gathers of a site and
// takes 105 VGPRs (4 waves); with this bound it takes 72 (7 waves) without
// spilling, where a bound of 8 waves spills.
constexpr int COLOUR_WAVES = FLBM_COLOUR_WAVES;

template <typename T, bool OBS>
__global__ __launch_bounds__(TILE, sizeof(T) <= 4 ? COLOUR_WAVES : 1) void k_colour_buf(const T *__restrict__ fin, T *__restrict__ fout,
                                                     const int32_t *__restrict__ nbr, StepArgs a, ColourStepArgs c)
{
    using R = typename Compute<T>::type;
    using C = typename ColourStore<T>::type;
    const uint32_t npad = (uint32_t)a.npad;
    const int tile = (int)blockIdx.x;
    const uint32_t s = (uint32_t)tile * TILE + threadIdx.x;
    const uint32_t esz = (uint32_t)sizeof(C), fsz = (uint32_t)sizeof(T);
    const __amdgpu_buffer_rsrc_t rf = make_rsrc(fin, a.f_bytes);
    const __amdgpu_buffer_rsrc_t rph = make_rsrc(c.phi, npad * esz);

    // pull f, and with the same decoded indices the colour gradient: the
    // neighbour x + xi_q is the source of pull direction opp(q), so
    // C = -3 sum_p w_p xi_p phi(source of p); a solid or wall source reads
    // phi_solid, an open-face source the site's own phi.
    R g[19];
    g[0] = Codec<T>::dec(__builtin_bit_cast(T, buf_load_raw<sizeof(T)>(rf, s * fsz, 0u)), 0);
    R gx = 0, gy = 0, gz = 0;
    const R phs = (R)c.phi_solid;
    const int32_t *hdr = a.pull_hdr ? a.pull_hdr + (int64_t)tile * PULL_HDR : nullptr;
    const int form = hdr ? (int)hdr_entry(hdr, PULL_HDR_FORM) : PULL_TILE_INT32;
    const uint32_t sent = 19u * npad, pos = threadIdx.x;
    // FORM_RUN: a tile of 8-bit codes read as run codes (see pull_format.h)
    constexpr int FORM_RUN = 3;
    auto gather = [&](auto form_tag) {
        constexpr int FORM = decltype(form_tag)::value;
        constexpr int CODES = FORM == FORM_RUN ? PULL_TILE_BYTE : FORM;
        uint32_t w[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, tail = 0;
        RunWave rw{0u, 0u, 0u, false};
        uint32_t off = 0;
        if constexpr (FORM == FORM_RUN) {
            const __amdgpu_buffer_rsrc_t rr = make_rsrc(a.pull_runs, a.runs_bytes);
            rw = load_runs(rr, s);
            load_runs_wide(rw, rr, s, npad);
        } else {
            load_pull_words<FORM, 18>(a, s, npad, w, tail);
        }
        const __amdgpu_buffer_rsrc_t rn = make_rsrc(nbr, a.nbr_bytes);
#pragma unroll
        for (int q = 1; q < 19; ++q) {
            const uint32_t code = FORM == PULL_TILE_INT32
                                      ? (uint32_t)buf_load_raw<4, SC_IDX_AUX>(rn, s * 4u, (uint32_t)(q - 1) * npad * 4u)
                                  : FORM == FORM_RUN ? run_code(rw, q, off)
                                                     : pull_code<CODES>(w, tail, q);
            int kind;
            const uint32_t base = FORM == PULL_TILE_INT32 ? 0u : hdr_entry(hdr, q - 1);
            const uint32_t idx = decode_pull<CODES>(code, base, pos, (uint32_t)d3q19::opp(q) * npad + s, sent,
                                                    (uint32_t)q, npad, kind);
            g[q] = Codec<T>::dec(__builtin_bit_cast(T, buf_load_raw<sizeof(T)>(rf, idx * fsz, 0u)), q);
            const uint32_t src = kind == PULL_REG ? idx - (uint32_t)q * npad : s;
            const R pv = (R)__builtin_bit_cast(C, buf_load_raw<sizeof(C)>(rph, src * esz, 0u));
            const R ph = kind == PULL_BB ? phs : pv;
            const R w3 = (R)(3.0 * d3q19::weight(q));
            if (d3q19::cx[q]) gx -= d3q19::cx[q] * w3 * ph;
            if (d3q19::cy[q]) gy -= d3q19::cy[q] * w3 * ph;
            if (d3q19::cz[q]) gz -= d3q19::cz[q] * w3 * ph;
        }
    };
    // run codes where the table has them, except in FP16 storage: 2 % off
    // the FP32 colour step, 1-3 % onto the FP16 one (whose decode lengthens a
    // latency chain the single-fluid FP16 step has shortened enough to gain)
    if (form == PULL_TILE_BYTE && !std::is_same<T, _Float16>::value && a.pull_runs && hdr_entry(hdr, PULL_HDR_RUNS))
        gather(std::integral_constant<int, FORM_RUN>{});
    else if (form == PULL_TILE_BYTE)
        gather(std::integral_constant<int, PULL_TILE_BYTE>{});
    else if (form == PULL_TILE_HALF)
        gather(std::integral_constant<int, PULL_TILE_HALF>{});
    else
        gather(std::integral_constant<int, PULL_TILE_INT32>{});

    double uz_in = 0.0, uz_out = 0.0;
    // after the gathers are issued (as in the single-fluid step)
    const double drho_in = step_begin<TILE>(tile, a, a.rd);
    if (tile < a.nt_in && (int64_t)s < a.a_in) uz_in = inlet_condition(g, drho_in, a.rho0);
    if (tile >= a.tout0 && (int64_t)s >= a.out0 && (int64_t)s < a.n)
        uz_out = outlet_condition(g, cst(a.st)->drho_out, a.rho0);

    const R snu = (R)cst(a.st)->omega;
    const bool collide = snu != (R)0;
    R drho, ux, uy, uz;
    if (collide) {
        trt_stress_collide(g, snu, (R)a.rho0, (R)a.inv_rho0, (R)c.alpha, gx, gy, gz, drho, ux, uy, uz);
        conserve_mass<T>(g, drho, s);
    } else {
        drho = ux = uy = uz = 0;
#pragma unroll
        for (int q = 0; q < 19; ++q) drho += g[q];
    }

    // the next inlet sum (as in the single-fluid kernel)
    double s_next = 0.0;
    if (tile < a.nt01 && (int64_t)s < a.n01) {
        const uint64_t cw = a.kcoef[s];
#pragma unroll
        for (int q = 0; q < 19; ++q) {
            const uint32_t cc = (uint32_t)(cw >> (2 * q)) & 3u;
            if (cc) s_next += (double)cc * (double)Codec<T>::dec(Codec<T>::enc(g[q], q, s), q);
        }
    }

    {
        const __amdgpu_buffer_rsrc_t ro = make_rsrc(fout, a.f_bytes);
        typedef typename RawBits<sizeof(T)>::type TB;
#pragma unroll
        for (int q = 0; q < 19; ++q)
            buf_store_raw_nt<sizeof(T)>(__builtin_bit_cast(TB, Codec<T>::enc(g[q], q, s)), ro, s * fsz,
                                        (uint32_t)q * npad * fsz);
    }

    // recolouring: full relaxation of A and B to
    //   w_q N_A [1 + 9/2 u.xi_q + beta N_B n.xi_q],  w_q N_B [1 + 9/2 u.xi_q - beta N_A n.xi_q]
    constexpr int PB = 2 * sizeof(C);
    R na, nb;
    colour_densities<R, C>(c.nab, c.phi, s, npad, na, nb);
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
        const __amdgpu_buffer_rsrc_t rabo = make_rsrc(c.about, 7u * npad * (uint32_t)PB);
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
            buf_store_pair_nt<C>(rabo, s, (uint32_t)q * npad * (uint32_t)PB, (C)(w * (na * adv + bab * cn)),
                                 (C)(w * (nb * adv - bab * cn)));
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
    step_epilogue<TILE, OBS, true>(tile, uz_in, uz_out, s_next, m, u2max, bad, a, a.rd, (double)na, (double)nb);
}

// Phase field of a stored colour state (for readout): phi from the stored A, B.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_phase_of_state(const typename Pair<T>::type *__restrict__ AB, int64_t n,
                                                          int64_t npad, double *__restrict__ out)
{
    const int64_t s = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (s >= n) return;
    double na = 0.0, nb = 0.0;
#pragma unroll
    for (int q = 0; q < 7; ++q) {
        const typename Pair<T>::type v = AB[(int64_t)q * npad + s];
        na += (double)v[0];
        nb += (double)v[1];
    }
    out[s] = (na + nb) != 0.0 ? (na - nb) / (na + nb) : 0.0;
}

}  // namespace flbm
