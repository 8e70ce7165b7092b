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
