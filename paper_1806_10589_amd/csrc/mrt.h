// D3Q19 multiple-relaxation-time collision in the moment basis of
// d'Humieres et al. (2002) that Appendix A lists; shared by the single-fluid
// MRT step and the two-fluid colour step.
#pragma once
#include <hip/hip_runtime.h>

#include "d3q19.h"

namespace flbm {

// MRT collision (Appendix A) in deviation variables, with (STRESS) or
// without the interfacial stress of colour gradient (gx, gy, gz):
//   m = M g;  m_eq = projections of the incompressible equilibrium plus
//   alpha |C| (19, (2n_x^2 - n_y^2 - n_z^2)/2, (n_y^2 - n_z^2)/2, n_x n_y/2,
//   n_y n_z/2, n_x n_z/2) on (e, 3p_xx, p_ww, p_xy, p_yz, p_xz);
//   g += M^T diag(1/|row|^2) (-S (m - m_eq)),
//   S: s_e = s_eps = s_pi = s_nu, s_q = s_m = 8 (2 - s_nu)/(8 - s_nu).
// Returns the moments (rho - 1, u).
template <bool STRESS, typename R>
__device__ __forceinline__ void mrt_collide(R (&g)[19], R snu, R rho0, R inv_rho0, R alpha, R gx, R gy, R gz,
                                            R &drho, R &ux, R &uy, R &uz)
{
    R d = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
    for (int q = 0; q < 19; ++q) {
        d += g[q];
        if (d3q19::cx[q]) jx += d3q19::cx[q] > 0 ? g[q] : -g[q];
        if (d3q19::cy[q]) jy += d3q19::cy[q] > 0 ? g[q] : -g[q];
        if (d3q19::cz[q]) jz += d3q19::cz[q] > 0 ? g[q] : -g[q];
    }
    drho = d;
    ux = jx * inv_rho0;
    uy = jy * inv_rho0;
    uz = jz * inv_rho0;

    R m[19];
#pragma unroll
    for (int k = 0; k < 19; ++k) {
        R acc = 0;
        if (k == 0 || k == 3 || k == 5 || k == 7) {
            m[k] = 0;  // conserved: not relaxed
            continue;
        }
#pragma unroll
        for (int q = 0; q < 19; ++q) {
            const int c = d3q19::mb(k, q);
            if (c == 1)
                acc += g[q];
            else if (c == -1)
                acc -= g[q];
            else if (c != 0)
                acc += (R)c * g[q];
        }
        m[k] = acc;
    }

    const R xx = jx * jx, yy = jy * jy, zz = jz * jz;
    const R jj = (xx + yy + zz) * inv_rho0;
    const R cm2 = gx * gx + gy * gy + gz * gz;
    // alpha |C| n_a n_b = alpha C_a C_b / |C|; zero where |C| <= 1e-6
    R ac = 0, sxx = 0, syy = 0, szz = 0, sxy = 0, syz = 0, sxz = 0;
    if (STRESS && cm2 > (R)1e-12) {
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
    R meq[19];
    meq[0] = meq[3] = meq[5] = meq[7] = 0;
    meq[1] = (R)-11 * d + (R)19 * jj + (R)19 * ac;
    meq[2] = (R)3 * d - (R)5.5 * jj;
    meq[4] = (R)(-2.0 / 3.0) * jx;
    meq[6] = (R)(-2.0 / 3.0) * jy;
    meq[8] = (R)(-2.0 / 3.0) * jz;
    const R pxx = ((R)2 * xx - yy - zz) * inv_rho0;
    const R pww = (yy - zz) * inv_rho0;
    meq[9] = pxx + (R)0.5 * ((R)2 * sxx - syy - szz);
    meq[10] = (R)-0.5 * pxx;
    meq[11] = pww + (R)0.5 * (syy - szz);
    meq[12] = (R)-0.5 * pww;
    meq[13] = jx * jy * inv_rho0 + (R)0.5 * sxy;
    meq[14] = jy * jz * inv_rho0 + (R)0.5 * syz;
    meq[15] = jx * jz * inv_rho0 + (R)0.5 * sxz;
    meq[16] = meq[17] = meq[18] = 0;

    const R sq = (R)8 * ((R)2 - snu) / ((R)8 - snu);
    R dm[19];
#pragma unroll
    for (int k = 0; k < 19; ++k) {
        const bool cons = (k == 0 || k == 3 || k == 5 || k == 7);
        const bool rate_q = (k == 4 || k == 6 || k == 8 || k >= 16);
        const R s = cons ? (R)0 : (rate_q ? sq : snu);
        dm[k] = cons ? (R)0 : -s * (m[k] - meq[k]) * (R)(1.0 / d3q19::mb_norm2(k));
    }
#pragma unroll
    for (int q = 0; q < 19; ++q) {
        R acc = 0;
#pragma unroll
        for (int k = 0; k < 19; ++k) {
            if (k == 0 || k == 3 || k == 5 || k == 7) continue;
            const int c = d3q19::mb(k, q);
            if (c == 1)
                acc += dm[k];
            else if (c == -1)
                acc -= dm[k];
            else if (c != 0)
                acc += (R)c * dm[k];
        }
        g[q] += acc;
    }
}

}  // namespace flbm
