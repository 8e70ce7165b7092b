// D3Q19 velocity set used by the HIP library (host and device).
//
// Numbering follows the groups of eq. d3q19; the sign order inside each group
// is the one implied by Appendix B's momentum equations (x: +1,7,9,11,13 and
// -2,8,10,12,14; y: +3,7,10,15,17 and -4,8,9,16,18) and by its inlet
// unknowns {5,11,14,15,18} (xi_z = +1). Opposite pairs are (1,2), (3,4), ...,
// (17,18). Weights 1/3, 1/18, 1/36 follow from the bounce-back coefficients
// 1/3 and 1/6 of Appendix B.
#pragma once
#include <stdint.h>

#if defined(__HIPCC__)
#define FLBM_HD __host__ __device__
#else
#define FLBM_HD
#endif

namespace d3q19 {

constexpr int Q = 19;

constexpr int cx[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int cy[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int cz[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

FLBM_HD constexpr int opp(int q) { return q == 0 ? 0 : ((q & 1) ? q + 1 : q - 1); }

FLBM_HD constexpr double weight(int q)
{
    return q == 0 ? 1.0 / 3.0 : (q <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
}

// Coefficient of f_q in the consistency sums: eq. inlet weights the in-plane
// populations by 1 and the ones leaving through the inlet (xi_z = -1) by 2;
// the outlet sum mirrors it. The unknowns get 0.
FLBM_HD constexpr int inlet_coeff(int q) { return cz[q] == 0 ? 1 : (cz[q] < 0 ? 2 : 0); }
FLBM_HD constexpr int outlet_coeff(int q) { return cz[q] == 0 ? 1 : (cz[q] > 0 ? 2 : 0); }

}  // namespace d3q19

namespace d3q19 {

// Moment basis of d'Humieres et al. (2002), rows in the order Appendix A
// lists the moments: (rho, e, eps, j_x, q_x, j_y, q_y, j_z, q_z, 3p_xx,
// 3pi_xx, p_ww, pi_ww, p_xy, p_yz, p_xz, m_x, m_y, m_z). Entry (k, q) is the
// basis polynomial k evaluated at xi_q; evaluated at compile time.
FLBM_HD constexpr int mb(int k, int q)
{
    const int x = cx[q], y = cy[q], z = cz[q];
    const int c2 = x * x + y * y + z * z;
    switch (k) {
    case 0: return 1;
    case 1: return 19 * c2 - 30;
    case 2: return (21 * c2 * c2 - 53 * c2 + 24) / 2;
    case 3: return x;
    case 4: return (5 * c2 - 9) * x;
    case 5: return y;
    case 6: return (5 * c2 - 9) * y;
    case 7: return z;
    case 8: return (5 * c2 - 9) * z;
    case 9: return 3 * x * x - c2;
    case 10: return (3 * c2 - 5) * (3 * x * x - c2);
    case 11: return y * y - z * z;
    case 12: return (3 * c2 - 5) * (y * y - z * z);
    case 13: return x * y;
    case 14: return y * z;
    case 15: return x * z;
    case 16: return (y * y - z * z) * x;
    case 17: return (z * z - x * x) * y;
    default: return (x * x - y * y) * z;
    }
}

// Squared norms of the basis rows (the basis is orthogonal, so the inverse
// transform is the transpose divided by these).
FLBM_HD constexpr int mb_norm2(int k)
{
    int s = 0;
    for (int q = 0; q < Q; ++q) s += mb(k, q) * mb(k, q);
    return s;
}

// FP16 storage of deviations: h_q = (f_q - w_q) 2^half_shift(q), a power of
// two per weight class, so that deviations up to about 1.5 w_q (rest) and
// 2.25 w_q (moving directions) stay below the FP16 maximum and small ones stay
// out of its subnormal range; scaling by a power of two is exact.
FLBM_HD constexpr int half_shift(int q) { return q == 0 ? 17 : (q <= 6 ? 19 : 20); }

// D3Q7 mass transport (Appendix A): velocities q = 0..6 of the set above,
// weights 1/3 and 1/9.
constexpr int Q7 = 7;
FLBM_HD constexpr double weight7(int q) { return q == 0 ? 1.0 / 3.0 : 1.0 / 9.0; }

}  // namespace d3q19
