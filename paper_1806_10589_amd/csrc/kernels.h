// gfx950 kernels of one D3Q19 step on the sparse pore lattice.
//
// Storage: distributions are kept as deviations from the rest weights,
// g_q = f_q - w_q, in [19][n_pad] structure-of-arrays (row q holds direction q
// for every site), so a wave's 64 lanes touch 64 consecutive sites of one row.
// Because the consistency weights of eq. inlet sum to one against the
// weights, the inlet sum becomes sum_i Kt_i with Kt the same weighted sum of
// deviations, and rho_in - 1 = (rho0 Q* + sum_i Kt_i) / A (eq. potential)
// needs no cancellation of O(1) terms.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "d3q19.h"
#include "mrt.h"
#include "pull_format.h"

namespace flbm {

// Launch shape of the fused step kernel: SC_BLOCK threads, SC_V consecutive
// sites per thread (vector loads of the pull indices and the rest
// population, vector stores), TILE sites per block.
#ifndef FLBM_SC_BLOCK
#define FLBM_SC_BLOCK 512
#endif
#ifndef FLBM_SC_V
#define FLBM_SC_V 1
#endif
#ifndef FLBM_SC_NT
#define FLBM_SC_NT 1
#endif
constexpr int SC_BLOCK = FLBM_SC_BLOCK;
constexpr bool SC_NT = FLBM_SC_NT;  // non-temporal stores of the new state
#ifndef FLBM_SC_IDX_NT
#define FLBM_SC_IDX_NT 1
#endif
constexpr int SC_IDX_AUX = FLBM_SC_IDX_NT ? 2 : 0;  // cache policy of the pull-table loads (codes or indices)
constexpr int SC_V = FLBM_SC_V;
constexpr int TILE = SC_BLOCK * SC_V;
constexpr int PAD_SITES = 1024;  // n_pad is a multiple of this (>= every TILE used)
static_assert(PAD_SITES % TILE == 0, "tile must divide the site padding");

constexpr int BLOCK = 256;       // threads per block of the other kernels
constexpr int HIST_STRIDE = 8;   // doubles per history record
constexpr int PLANE_MAX_BLOCKS = 1024;

// FP64 scalars shared by the kernels of a step. Written by single threads
// with vector stores; read by every block.
struct DevState {
    double q_target;      // Q*
    double drho_out;      // rho_out - 1
    double s_carry[2];    // inlet consistency sum (deviation form) for the next step,
                          // slot = index of the buffer that step reads
    double omega;         // 1/tau (0 turns collision off)
    double ctrl_delta;    // controller's offset at its last decision (reporting only)
    double obs_mass;      // on-demand observables
    double obs_umax;
    int64_t step;         // steps completed
    uint32_t k_ticket;    // last-block ticket of the inlet-plane reduction
    uint32_t unstable;    // sticky watchdog flag
    uint32_t obs_bad;
    int64_t ctrl_steps;   // controller decisions taken
    uint32_t ctrl_released;  // sticky: plain update from now on (tolerance met, or no progress)
    uint32_t ovr_on;      // 1: the inlet density override below is in force
    double ctrl_best;     // smallest outlet-flux error seen at a 10% improvement
    int64_t ctrl_best_n;  // decision count at that improvement
    double ovr_rho;       // inlet density override (absolute)
    double ovr_limit;     // its bound on |rho_in - rho_plain|
    double ctrl_rho;      // the controller's held proposal (absolute inlet density)
    double ctrl_limit;    // its bound on |rho_in - rho_plain| until the next decision
    double ctrl_gain;
    double ctrl_acc;      // sum of the outlet flux over the current decision period
    int64_t ctrl_periods; // decision periods completed (entries pushed to the period ring)
    uint32_t ctrl_on;     // 1: the held proposal is in force
    uint32_t pad2_;
    double rin[2];        // inlet density minus one used by the step that wrote buffer i
    uint32_t pend[2];     // 1: the end of the step that wrote buffer i (history record,
                          // step counter, its inlet sum into s_carry[i]) is still to come
};

// Inlet density minus one for the step that reads parity rd: the update of
// eq. potential, rho_in = (rho0 Q* + sum_i K_i) / A in deviation form, moved
// towards a caller's override or the learned controller's held proposal by
// at most the bound that comes with it (the plain update judges both).
// DevState as the step kernels read it: through the constant address space,
// so that every field read is a scalar load. Tile 0 of a step kernel writes
// a few fields (step_begin), and with a store through the same pointer in the
// kernel the compiler would read the others -- omega in every tile -- with
// vector loads, which wait behind the gathers in flight (3-4 % of the FP16
// step). The fields read this way are not written while the kernel runs.
typedef const DevState __attribute__((address_space(4))) *CDevState;
__device__ __forceinline__ CDevState cst(const DevState *p) { return (CDevState)p; }

// carry: the inlet consistency sum sum_i K_i (deviation form).
template <typename SP>
__device__ __forceinline__ double inlet_drho_from(SP st, double carry, double rho0, int64_t a_in)
{
    const double plain = (rho0 * st->q_target + carry) / (double)a_in;
    if (st->ovr_on) {
        // a caller's inlet density, judged by the plain update: at most
        // ovr_limit away from it
        const double d = st->ovr_rho - 1.0 - plain;
        return plain + fmin(st->ovr_limit, fmax(-st->ovr_limit, d));
    }
    if (st->ctrl_on) {
        // the learned controller's held proposal, judged the same way
        const double d = st->ctrl_gain * (st->ctrl_rho - 1.0 - plain);
        return plain + fmin(st->ctrl_limit, fmax(-st->ctrl_limit, d));
    }
    return plain;
}

// The same from the sum held in s_carry[rd] (valid once the previous step
// has ended, see step_begin).
__device__ __forceinline__ double inlet_drho_plain(const DevState *st, int rd, double rho0, int64_t a_in)
{
    return (rho0 * st->q_target + st->s_carry[rd]) / (double)a_in;
}

__device__ __forceinline__ double inlet_drho(const DevState *st, int rd, double rho0, int64_t a_in)
{
    return inlet_drho_from(st, st->s_carry[rd], rho0, a_in);
}

struct StepArgs {
    int64_t n, npad;
    uint32_t f_bytes, nbr_bytes;  // buffer sizes for the descriptors (BUF path)
    int64_t a_in;         // inlet sites [0, a_in)
    int64_t out0;         // outlet sites [out0, n)
    int64_t n01;          // sites of planes z = 0 and 1: they feed the next inlet sum
    int32_t nt_in;        // tiles holding inlet sites: [0, nt_in)
    int32_t nt01;         // tiles holding planes 0 and 1: [0, nt01)
    int32_t tout0;        // tiles holding outlet sites: [tout0, tiles)
    int32_t hist_cap;
    int32_t flux_mode;
    int32_t rd;           // s_carry slot this step reads (its input buffer)
    int32_t part_stride;  // the boundary partials are [2][part_stride]: slot i holds those
                          // of the step that wrote buffer i
    double rho0, inv_rho0;
    DevState *st;
    const uint64_t *kcoef;          // per site of planes 0-1: 2-bit weight of each post-collision
                                    // population in the next step's inlet sum
    double *spart;                  // per-tile partial of that sum      [2][part_stride]
    double *bpart_in, *bpart_out;   // per-tile sums of u_z               [2][part_stride]
    double *obs_mass;               // per-tile sums of rho - 1
    float *obs_umax2;               // per-tile max |u|^2
    uint32_t *obs_bad;              // per-tile non-finite flag
    double *obs_na, *obs_nb;        // per-tile colour sums (two-fluid model)
    double *hist;
    const uint32_t *pull_codes;     // compact pull table: 16-bit codes ([9][npad] words)
    const uint32_t *pull_bytes;     // byte codes ([4][npad] words, then [npad] 16-bit)
    const int32_t *pull_hdr;        // per-tile header ([tiles][PULL_HDR]); null: int32 table only
    const uint32_t *pull_runs;      // run codes ([npad][2] words, then [npad]); null: byte codes only
    uint32_t codes_bytes, bytes_bytes;  // sizes of the code arrays for the descriptors
    uint32_t runs_bytes, pad2_;
};

struct PlaneArgs {
    int64_t npad, a_in;
    int32_t slot;         // s_carry slot to fill
    int32_t pad_;
    DevState *st;
    double *kpart;
};

// Storage codec: how a stored population of direction q at site `site`
// becomes the arithmetic value (the deviation g_q = f_q - w_q) and back.
// FP32 and FP64 store g directly; FP16 stores g 2^half_shift(q) (exact
// power-of-two scaling, arithmetic in FP32) with dithered rounding: a fixed
// amount, uniform in [0, 1) of the FP16 spacing, is added to the magnitude
// before truncating to the FP16 grid (unbiased: the value rounds up with a
// probability equal to its distance from the grid point below). Equal values
// at neighbouring sites -- a reservoir in plug flow holds thousands of them
// -- then round up or down at random instead of all the same way, so their
// rounding errors do not add up to a mass source across a plane (without it
// the outlet flux of a 256^3 pack at Darcy velocity 1e-5 ends 7 % low).
// In the FP16 normal range the FP16 grid is the FP32 values whose 13 low
// significand bits are zero, so the dither is an integer add of 13 random
// bits to the FP32 pattern and a mask. gfx950's stochastic-rounding
// conversion (v_cvt_sr_f16_f32) does exactly that in one instruction: it adds
// the top 13 bits of its 32-bit random operand to the 13 dropped bits and
// truncates (checked bit for bit against the add-and-mask form on a million
// FP16-normal values); below the FP16 normal range it rounds onto the
// subnormal grid the same way. The random word comes from one integer hash
// of the site (shared by its 19 populations), xored with a constant per
// direction and multiplied by an odd constant: the top bits of the product
// differ between the directions of a site in no fixed pattern. (Offsets that
// differ between directions by a fixed amount at every site -- a Weyl step
// -- bias the steady flux by 1 % on a test pack; independent ones leave
// 0.1-0.2 %.) They depend on nothing else, so runs stay deterministic.
// The site hash is the published 32-bit integer mix known as "lowbias32"
// (xorshift-multiply rounds with the multipliers 0x7feb352d and 0x846ca68b,
// from C. Wellons' hash-prospector search); the per-direction constants are
// the golden-ratio increment 0x9e3779b9 and the MurmurHash3 finalizer
// multiplier 0x85ebca6b.
__device__ __forceinline__ uint32_t dither_hash(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}

template <typename T> struct Codec {
    typedef T R;
    static __device__ __forceinline__ R dec(T v, int) { return v; }
    static __device__ __forceinline__ T enc(R v, int, uint32_t) { return v; }
};
template <> struct Codec<_Float16> {
    typedef float R;
    typedef _Float16 h2 __attribute__((ext_vector_type(2)));
    static __device__ __forceinline__ float scale(int q) { return (float)(1u << d3q19::half_shift(q)); }
    static __device__ __forceinline__ float dec(_Float16 v, int q) { return (float)v * (1.0f / scale(q)); }
    // x: the value already scaled, g_q 2^half_shift(q)
    static __device__ __forceinline__ _Float16 enc_scaled(float x, int q, uint32_t site)
    {
        const uint32_t r = (dither_hash(site) ^ ((uint32_t)q * 0x9e3779b9u)) * 0x85ebca6bu;
        return __builtin_amdgcn_cvt_sr_f16_f32(h2{0, 0}, x, r, false)[0];
    }
    static __device__ __forceinline__ _Float16 enc(float v, int q, uint32_t site)
    {
        return enc_scaled(v * scale(q), q, site);
    }
};
template <typename T> struct Compute { using type = typename Codec<T>::R; };

typedef int32_t i32x2 __attribute__((ext_vector_type(2)));
typedef int32_t i32x4 __attribute__((ext_vector_type(4)));

template <typename T, int V> struct Vec;
template <typename T> struct Vec<T, 1> { typedef T type; };
template <typename T> struct Vec<T, 2> { typedef T type __attribute__((ext_vector_type(2))); };
template <typename T> struct Vec<T, 4> { typedef T type __attribute__((ext_vector_type(4))); };


// Buffer-resource access (CDNA raw buffer instructions): the base address
// and byte size live in an SGPR descriptor, each lane supplies a 32-bit byte
// offset, and a uniform row offset goes in the scalar offset field. No
// per-lane 64-bit address arithmetic, and the hardware drops accesses beyond
// the size. Used when every buffer of the step is below 4 GiB (checked on the
// host); otherwise the kernel falls back to plain 64-bit global addressing.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *p, uint32_t bytes)
{
    // third descriptor word 0x00020000: raw (untyped) 32-bit data format, gfx9 family
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}

template <int BYTES> struct RawBits;
template <> struct RawBits<2> { typedef uint16_t type; };
template <> struct RawBits<4> { typedef uint32_t type; };
template <> struct RawBits<8> { typedef uint32_t type __attribute__((ext_vector_type(2))); };
template <> struct RawBits<16> { typedef uint32_t type __attribute__((ext_vector_type(4))); };

template <int BYTES, int AUX = 0>
__device__ __forceinline__ typename RawBits<BYTES>::type buf_load_raw(__amdgpu_buffer_rsrc_t r, uint32_t voff,
                                                                      uint32_t soff)
{
    if constexpr (BYTES == 2)
        return __builtin_amdgcn_raw_buffer_load_b16(r, (int)voff, (int)soff, AUX);
    else if constexpr (BYTES == 4)
        return __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, AUX);
    else if constexpr (BYTES == 8)
        return __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, AUX);
    else
        return __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, AUX);
}

// aux = 2: non-temporal (gfx940-family cache policy bit "nt")
template <int BYTES>
__device__ __forceinline__ void buf_store_raw_nt(typename RawBits<BYTES>::type v, __amdgpu_buffer_rsrc_t r,
                                                 uint32_t voff, uint32_t soff)
{
    constexpr int aux = SC_NT ? 2 : 0;
    if constexpr (BYTES == 2)
        __builtin_amdgcn_raw_buffer_store_b16(v, r, (int)voff, (int)soff, aux);
    else if constexpr (BYTES == 4)
        __builtin_amdgcn_raw_buffer_store_b32(v, r, (int)voff, (int)soff, aux);
    else if constexpr (BYTES == 8)
        __builtin_amdgcn_raw_buffer_store_b64(v, r, (int)voff, (int)soff, aux);
    else
        __builtin_amdgcn_raw_buffer_store_b128(v, r, (int)voff, (int)soff, aux);
}

// V consecutive elements of type T at byte offset voff + soff (one load of
// up to 16 bytes, two when V * sizeof(T) is 32).
template <int V, typename T, typename R, int AUX = 0>
__device__ __forceinline__ void buf_load_v(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, R (&o)[V])
{
    constexpr int BYTES = V * (int)sizeof(T);
    if constexpr (BYTES > 16) {
        R lo[V / 2], hi[V / 2];
        buf_load_v<V / 2, T, R, AUX>(r, voff, soff, lo);
        buf_load_v<V / 2, T, R, AUX>(r, voff + (uint32_t)(BYTES / 2), soff, hi);
#pragma unroll
        for (int v = 0; v < V / 2; ++v) {
            o[v] = lo[v];
            o[v + V / 2] = hi[v];
        }
    } else {
        typedef typename Vec<T, V>::type VT;
        const VT x = __builtin_bit_cast(VT, buf_load_raw<BYTES, AUX>(r, voff, soff));
        if constexpr (V == 1) {
            o[0] = (R)x;
        } else {
#pragma unroll
            for (int v = 0; v < V; ++v) o[v] = (R)x[v];
        }
    }
}

template <int V, typename T, typename R>
__device__ __forceinline__ void buf_store_v_nt(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff,
                                               const R (&val)[V])
{
    constexpr int BYTES = V * (int)sizeof(T);
    if constexpr (BYTES > 16) {
        R lo[V / 2], hi[V / 2];
#pragma unroll
        for (int v = 0; v < V / 2; ++v) {
            lo[v] = val[v];
            hi[v] = val[v + V / 2];
        }
        buf_store_v_nt<V / 2, T>(r, voff, soff, lo);
        buf_store_v_nt<V / 2, T>(r, voff + (uint32_t)(BYTES / 2), soff, hi);
    } else {
        typedef typename Vec<T, V>::type VT;
        VT x;
        if constexpr (V == 1) {
            x = (T)val[0];
        } else {
#pragma unroll
            for (int v = 0; v < V; ++v) x[v] = (T)val[v];
        }
        buf_store_raw_nt<BYTES>(__builtin_bit_cast(typename RawBits<BYTES>::type, x), r, voff, soff);
    }
}

// Load V consecutive elements (one vector load when V > 1; p is aligned to
// V elements because site tiles start at multiples of V).
template <int V, typename T, typename R>
__device__ __forceinline__ void load_v(const T *__restrict__ p, R (&o)[V])
{
    if constexpr (V == 1) {
        o[0] = (R)p[0];
    } else {
        const typename Vec<T, V>::type x = *(const typename Vec<T, V>::type *)p;
#pragma unroll
        for (int v = 0; v < V; ++v) o[v] = (R)x[v];
    }
}

// Non-temporal store of V consecutive elements.
template <int V, typename T, typename R>
__device__ __forceinline__ void store_v_nt(T *__restrict__ p, const R (&val)[V])
{
    if constexpr (V == 1) {
        __builtin_nontemporal_store((T)val[0], p);
    } else {
        typename Vec<T, V>::type x;
#pragma unroll
        for (int v = 0; v < V; ++v) x[v] = (T)val[v];
        __builtin_nontemporal_store(x, (typename Vec<T, V>::type *)p);
    }
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ float wave_max(float v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ uint32_t wave_or(uint32_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o, 64);
    return v;
}

// Deterministic block sum (fixed butterfly inside waves, waves in order).
template <int NT>
__device__ __forceinline__ double block_sum(double v, double *lds)
{
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) lds[w] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) s += lds[i];
    __syncthreads();
    return s;
}

// --------------------------------------------------------------- boundary

// Pressure condition at an inlet site with inlet density 1 + drho_in
// (Appendix B; u_x = u_y = 0): u_z from the consistency condition eq. inlet,
// f5 by non-equilibrium bounce-back, f11, f14, f15, f18 from the simplified
// Hecht-Harting rows. Arithmetic in FP64. Returns u_z.
// u_z at an inlet site from the consistency condition (eq. inlet) with the
// known populations (deviations) and inlet density 1 + drho_in.
template <typename R>
__device__ __forceinline__ double inlet_velocity(const R (&g)[19], double drho_in, double rho0)
{
    double k = 0.0;
#pragma unroll
    for (int q = 0; q < 19; ++q)
        if (d3q19::inlet_coeff(q)) k += d3q19::inlet_coeff(q) * (double)g[q];
    return (drho_in - k) / rho0;
}

// u_z at an outlet site with outlet density 1 + drho_out.
template <typename R>
__device__ __forceinline__ double outlet_velocity(const R (&g)[19], double drho_out, double rho0)
{
    double k = 0.0;
#pragma unroll
    for (int q = 0; q < 19; ++q)
        if (d3q19::outlet_coeff(q)) k += d3q19::outlet_coeff(q) * (double)g[q];
    return (k - drho_out) / rho0;
}

template <typename R>
__device__ __forceinline__ double inlet_condition(R (&g)[19], double drho_in, double rho0)
{
    const double uz = inlet_velocity(g, drho_in, rho0);
    const double nx = 0.5 * ((double)g[1] + (double)g[7] + (double)g[9] -
                             ((double)g[2] + (double)g[10] + (double)g[8]));
    const double ny = 0.5 * ((double)g[3] + (double)g[7] + (double)g[10] -
                             ((double)g[4] + (double)g[9] + (double)g[8]));
    const double r3 = rho0 * uz / 3.0;
    const double r6 = 0.5 * r3;  // equals rho0 uz / 6 rounded: halving is exact
    g[5] = (R)((double)g[6] + r3);
    g[11] = (R)((double)g[12] + r6 - nx);
    g[14] = (R)((double)g[13] + r6 + nx);
    g[15] = (R)((double)g[16] + r6 - ny);
    g[18] = (R)((double)g[17] + r6 + ny);
    return uz;
}

// The same condition at an outlet site with density 1 + drho_out, the
// closure rows solved for the outlet unknowns 6, 12, 13, 16, 17.
template <typename R>
__device__ __forceinline__ double outlet_condition(R (&g)[19], double drho_out, double rho0)
{
    const double uz = outlet_velocity(g, drho_out, rho0);
    const double nx = 0.5 * ((double)g[1] + (double)g[7] + (double)g[9] -
                             ((double)g[2] + (double)g[10] + (double)g[8]));
    const double ny = 0.5 * ((double)g[3] + (double)g[7] + (double)g[10] -
                             ((double)g[4] + (double)g[9] + (double)g[8]));
    const double r3 = rho0 * uz / 3.0;
    const double r6 = 0.5 * r3;
    g[6] = (R)((double)g[5] - r3);
    g[12] = (R)((double)g[11] - r6 + nx);
    g[13] = (R)((double)g[14] - r6 - nx);
    g[16] = (R)((double)g[15] - r6 + ny);
    g[17] = (R)((double)g[18] - r6 - ny);
    return uz;
}

// --------------------------------------------------------------- collision

// BGK relaxation toward the incompressible equilibrium
//   f_eq = w_q [rho + rho0 (3 xi.u + 9/2 (xi.u)^2 - 3/2 u.u)],  u = j/rho0,
// written for deviations: g_eq = w_q [(rho - 1) + rho0 (...)], and
//   g <- g + omega (g_eq - g) = (1 - omega) g + omega g_eq.
// Opposite directions share xi.u up to sign, so each pair (q, opp q) forms
// the even part omega w (base + rho0 9/2 (xi.u)^2) once and adds / subtracts
// the odd part omega w rho0 3 xi.u; omega and the weights are folded into
// per-class coefficients.
// On return g holds the post-collision deviations; drho, u the moments.
// SCALED: g holds the FP16 storage scaling of the deviations, g_q
// 2^half_shift(q), on entry and on return; the moment sums take the inverse
// powers of two and the relaxation coefficients the powers of two. Scaling by
// a power of two commutes with rounding, so the result is the unscaled
// computation's, scaled, without a multiply per population on either side.
template <typename R, bool SCALED = false>
__device__ __forceinline__ void bgk_collide(R (&g)[19], R omega, R rho0, R inv_rho0, R &drho,
                                            R &ux, R &uy, R &uz)
{
    // per weight class (rest, axis, diagonal): the storage scale, 1 unless SCALED
    constexpr double c0 = SCALED ? (double)(1u << d3q19::half_shift(0)) : 1.0;
    constexpr double c1 = SCALED ? (double)(1u << d3q19::half_shift(1)) : 1.0;
    constexpr double c2 = SCALED ? (double)(1u << d3q19::half_shift(7)) : 1.0;
    R d = g[0] * (R)(1.0 / c0);
    R jx = 0, jy = 0, jz = 0;
#pragma unroll
    for (int q = 1; q < 19; q += 2) {
        const R inv = (R)(1.0 / (q <= 6 ? c1 : c2));
        const R sum = g[q] + g[q + 1], dif = g[q] - g[q + 1];
        d += sum * inv;
        if (d3q19::cx[q]) jx += (d3q19::cx[q] > 0 ? dif : -dif) * inv;
        if (d3q19::cy[q]) jy += (d3q19::cy[q] > 0 ? dif : -dif) * inv;
        if (d3q19::cz[q]) jz += (d3q19::cz[q] > 0 ? dif : -dif) * inv;
    }
    ux = jx * inv_rho0;
    uy = jy * inv_rho0;
    uz = jz * inv_rho0;
    drho = d;
    const R keep = (R)1 - omega;
    const R base = d - rho0 * (R)1.5 * (ux * ux + uy * uy + uz * uz);
    // omega * w * base for the three weight classes, omega * w * rho0 * {9/2, 3}
    const R ob0 = omega * (R)(c0 / 3.0) * base;
    const R ob1 = omega * (R)(c1 / 18.0) * base, ob2 = omega * (R)(c2 / 36.0) * base;
    const R oe1 = omega * rho0 * (R)(c1 * 4.5 / 18.0), oe2 = omega * rho0 * (R)(c2 * 4.5 / 36.0);
    const R oo1 = omega * rho0 * (R)(c1 * 3.0 / 18.0), oo2 = omega * rho0 * (R)(c2 * 3.0 / 36.0);
    g[0] = keep * g[0] + ob0;
#pragma unroll
    for (int q = 1; q < 19; q += 2) {  // q has positive orientation, q + 1 = opp(q)
        R cu = 0;
        if (d3q19::cx[q]) cu += d3q19::cx[q] > 0 ? ux : -ux;
        if (d3q19::cy[q]) cu += d3q19::cy[q] > 0 ? uy : -uy;
        if (d3q19::cz[q]) cu += d3q19::cz[q] > 0 ? uz : -uz;
        const bool axis = q <= 6;
        const R even = (axis ? oe1 : oe2) * cu * cu + (axis ? ob1 : ob2);
        const R odd = (axis ? oo1 : oo2) * cu;
        g[q] = keep * g[q] + (even + odd);
        g[q + 1] = keep * g[q + 1] + (even - odd);
    }
}

// --------------------------------------------------------------- kernels

// Inlet plane reduction (eq. potential) of the current state: each thread
// sums the consistency sums of its inlet sites from the pulled values; blocks
// write FP64 partials; the last block to finish sums them in block order into
// s_carry[slot]. The fused step kernel turns it into rho_in, and each step's
// end (step_begin, finalize_step) hands the sum of the following step over, so
// this kernel runs only when a run of steps starts from a state the step
// kernels did not produce.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_inlet_plane(const T *__restrict__ fin,
                                                       const int32_t *__restrict__ nbr,
                                                       PlaneArgs a)
{
    __shared__ double lds[BLOCK / 64];
    __shared__ int is_last;
    double k = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < a.a_in;
         i += (int64_t)gridDim.x * BLOCK) {
        double ki = (double)Codec<T>::dec(fin[i], 0);
#pragma unroll
        for (int q = 1; q < 19; ++q)
            if (d3q19::inlet_coeff(q))
                ki += d3q19::inlet_coeff(q) *
                      (double)Codec<T>::dec(fin[nbr[(int64_t)(q - 1) * a.npad + i]], q);
        k += ki;
    }
    k = block_sum<BLOCK>(k, lds);
    if (threadIdx.x == 0) {
        a.kpart[blockIdx.x] = k;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // the partial before the ticket
        const uint32_t prev = atomicAdd(&a.st->k_ticket, 1u);
        is_last = (prev == gridDim.x - 1);
    }
    __syncthreads();
    if (!is_last) return;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // every block's partial after its ticket
    double s = 0.0;
    for (int i = threadIdx.x; i < (int)gridDim.x; i += BLOCK) s += a.kpart[i];
    s = block_sum<BLOCK>(s, lds);
    if (threadIdx.x == 0) {
        a.st->s_carry[a.slot] = s;
        a.st->pend[a.slot] = 0;  // the next step starts from this sum
        a.st->k_ticket = 0;
    }
}

// Shared tail of the step kernels (NT threads per tile). OBS: write the
// tile's watchdog partials (sum of rho - 1, max |u|^2, non-finite flag).
// Boundary tiles (planes 0-1 and the outlet plane) reduce their u_z sums and
// their share of the next inlet sum into the partials' slot rd ^ 1 (the
// buffer the step writes), for the end of the step (see step_begin).
// COLOUR: also the tile's sums of the two colour densities.
template <int NT, bool OBS, bool COLOUR = false>
__device__ __forceinline__ void step_epilogue(int tile, double uz_in, double uz_out, double s_next, double m,
                                              float u2max, uint32_t bad, const StepArgs &a, int rd,
                                              double na_sum = 0.0, double nb_sum = 0.0)
{
    __shared__ double lds[NT / 64];
    __shared__ float ldsf[NT / 64];
    __shared__ uint32_t ldsu[NT / 64];
    if (OBS && COLOUR) {
        na_sum = block_sum<NT>(na_sum, lds);
        nb_sum = block_sum<NT>(nb_sum, lds);
        if (threadIdx.x == 0) {
            a.obs_na[tile] = na_sum;
            a.obs_nb[tile] = nb_sum;
        }
    }
    if (OBS) {
        m = block_sum<NT>(m, lds);
        const float wm = wave_max(u2max);
        const uint32_t wb = wave_or(bad);
        const int w = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) {
            ldsf[w] = wm;
            ldsu[w] = wb;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            float mm = 0.f;
            uint32_t bb = 0;
#pragma unroll
            for (int i = 0; i < NT / 64; ++i) {
                mm = fmaxf(mm, ldsf[i]);
                bb |= ldsu[i];
            }
            a.obs_mass[tile] = m;
            a.obs_umax2[tile] = mm;
            a.obs_bad[tile] = bb;
        }
    }

    if (!a.flux_mode || !(tile < a.nt01 || tile >= a.tout0)) return;
    const double si = block_sum<NT>(uz_in, lds);
    const double so = block_sum<NT>(uz_out, lds);
    const double sn = block_sum<NT>(s_next, lds);
    if (threadIdx.x == 0) {
        const int64_t w = (int64_t)(rd ^ 1) * a.part_stride;
        if (tile < a.nt_in) a.bpart_in[w + tile] = si;
        if (tile < a.nt01) a.spart[w + tile] = sn;
        if (tile >= a.tout0) a.bpart_out[w + tile - a.tout0] = so;
    }
}

// End of a step: the sums of its boundary tiles' partials give Q_in, Q_out
// and the inlet consistency sum the next step starts from; the step goes into
// the history and the step counter advances. It runs either in a launch of
// its own after the step kernel (k_step_finalize: the kernel boundary orders
// every tile's partial before these reads) or, inside a run of steps, in the
// next step kernel (step_begin), where the inlet tiles also sum the partials
// themselves instead of waiting for s_carry. Both sum in one fixed order
// (partials_sum), so a step's results do not depend on which end it had.
// (The first form was the last boundary tile to finish, found by a ticket:
// the release fence each boundary tile then needs writes that XCD's L2 back,
// and cost about 7 % of the step on a 256^3 pack.)
constexpr int FIN_BLOCK = 256;  // threads of a finalize: the partials in one round of loads

// Sum of n partials in a fixed order for any block of NT >= FIN_BLOCK threads:
// threads below FIN_BLOCK add every FIN_BLOCK-th entry, the rest add nothing.
template <int NT>
__device__ __forceinline__ double partials_sum(const double *p, int n, double *lds)
{
    static_assert(NT >= FIN_BLOCK && NT % 64 == 0, "a whole number of waves, at least FIN_BLOCK threads");
    double v = 0.0;
    if ((int)threadIdx.x < FIN_BLOCK)
        for (int i = (int)threadIdx.x; i < n; i += FIN_BLOCK) v += p[i];
    return block_sum<NT>(v, lds);
}

// Record the end of the step that wrote buffer w (thread 0 only): ti, to the
// inlet and outlet u_z sums, tn the next inlet sum.
__device__ __forceinline__ void end_step_record(const StepArgs &a, int w, double ti, double to, double tn)
{
    DevState *st = a.st;
    const int64_t t = st->step;
    const double nan = __builtin_nan("");
    const double r[HIST_STRIDE] = {a.flux_mode ? 1.0 + st->rin[w] : nan, a.flux_mode ? ti : nan,
                                   a.flux_mode ? to : nan, nan, nan, (double)(t + 1), nan, nan};
    double *h = a.hist + (t % a.hist_cap) * HIST_STRIDE;
    // one 8-byte store each, kept apart by a compiler barrier (see store_pair
    // in colour.h); plain stores, since a volatile one is followed by a wait
    // for every memory operation of the wave in flight (in a step kernel, the
    // tile's gathers)
#pragma unroll
    for (int i = 0; i < HIST_STRIDE; ++i) {
        h[i] = r[i];
        __asm__ __volatile__("" ::: "memory");
    }
    if (a.flux_mode) st->s_carry[w] = tn;
    st->step = t + 1;
}

// Sums of the partials in slot w (the step that wrote buffer w).
template <int NT>
__device__ __forceinline__ void end_step_sums(const StepArgs &a, int w, double *lds, double &ti, double &to)
{
    const int64_t o = (int64_t)w * a.part_stride;
    const int nt_out = (int)((a.npad / TILE) - a.tout0);
    ti = partials_sum<NT>(a.bpart_in + o, a.nt_in, lds);
    to = partials_sum<NT>(a.bpart_out + o, nt_out, lds);
}

// The end of the step that read buffer rd, in a launch of its own.
__device__ __forceinline__ void finalize_step(const StepArgs &a, const int rd)
{
    __shared__ double lds[FIN_BLOCK / 64];
    const int w = rd ^ 1;
    double ti = 0.0, to = 0.0, tn = 0.0;
    if (a.flux_mode) {
        end_step_sums<FIN_BLOCK>(a, w, lds, ti, to);
        tn = partials_sum<FIN_BLOCK>(a.spart + (int64_t)w * a.part_stride, a.nt01, lds);
    }
    if (threadIdx.x == 0) {
        end_step_record(a, w, ti, to, tn);
        a.st->pend[w] = 0;
    }
}

// Start of a step that reads buffer rd, for the tile `tile` (block-uniform;
// every thread of the tile calls it). Returns the inlet density minus one on
// the inlet tiles (0 elsewhere). When the step that wrote buffer rd has not
// ended yet (pend[rd]: runs of steps launch no k_step_finalize in between),
// the inlet tiles sum its partials themselves and tile 0 records its end. Tile
// 0 then marks this step's end as pending, with its inlet density for the
// record. pend[rd] and s_carry[rd] are not written by this kernel while it
// reads them (tile 0 writes s_carry[rd] only when pend[rd] is set, and then
// nobody reads it).
template <int NT>
__device__ __forceinline__ double step_begin(int tile, const StepArgs &a, int rd)
{
    __shared__ double lds[NT / 64];
    const bool inlet = a.flux_mode && tile < a.nt_in;
    if (!inlet && tile != 0) return 0.0;
    DevState *st = a.st;
    const bool pend = cst(st)->pend[rd] != 0;
    double drho = 0.0, carry = 0.0;
    if (inlet) {
        carry = pend ? partials_sum<NT>(a.spart + (int64_t)rd * a.part_stride, a.nt01, lds) : cst(st)->s_carry[rd];
        drho = inlet_drho_from(cst(st), carry, a.rho0, a.a_in);
    }
    if (tile == 0) {
        if (pend) {
            double ti = 0.0, to = 0.0;
            if (a.flux_mode) end_step_sums<NT>(a, rd, lds, ti, to);
            if (threadIdx.x == 0) end_step_record(a, rd, ti, to, carry);
        }
        if (threadIdx.x == 0) {
            st->rin[rd ^ 1] = drho;
            st->pend[rd ^ 1] = 1;
        }
    }
    return drho;
}

__global__ __launch_bounds__(FIN_BLOCK) void k_step_finalize(StepArgs a)
{
    finalize_step(a, a.rd);
}

// Fused step for every site: pull the 19 populations, apply the inlet or
// outlet pressure condition where the site lies on z = 0 or z = nz-1, BGK
// collide, store. Each thread owns SC_V consecutive sites. Tiles holding
// boundary sites also reduce sum u_z (FP64) and their share of the next inlet
// sum, which the step's end (step_begin of the next step kernel, or
// k_step_finalize) turns into Q_in, Q_out and the next step's start.
// OBS: also write per-tile partials of mass, max |u|^2 and a non-finite flag.
// Mass-exact store of a collided site in reduced precision: the rest
// population takes the site's pre-collision mass minus what the other 18
// populations will hold once stored, so the coherent part of the rounding --
// the weight coefficients rounded to the working precision, the storage
// format -- creates no mass at the site (what is left is rounding of a few
// sums, whose sign varies from site to site). Without it a reduced-precision
// state settles to a fixed point with a small mass source at every site
// proportional to the local density deviation, which adds up along the flow
// direction to a systematic outlet-flux error growing with the domain length
// (about 1e-3 of Q* over the 268 planes of a 256^3 pack in FP32). FP64
// storage keeps its arithmetic unchanged.
// Encode a collided site for storage, mass-exact (see above): h[q] for
// q >= 1 first, then the rest population from the pre-collision mass minus
// what the others hold as stored.
// SCALED: g holds the FP16 storage scaling (see bgk_collide).
template <typename T, bool SCALED = false, typename R>
__device__ __forceinline__ void encode_site(const R (&g)[19], T (&h)[19], R pre, uint32_t site)
{
#pragma unroll
    for (int q = 1; q < 19; ++q) {
        if constexpr (SCALED)
            h[q] = Codec<T>::enc_scaled(g[q], q, site);
        else
            h[q] = Codec<T>::enc(g[q], q, site);
    }
    if constexpr (!std::is_same<T, double>::value) {
        R s = 0;
#pragma unroll
        for (int q = 1; q < 19; ++q) s += Codec<T>::dec(h[q], q);
        h[0] = Codec<T>::enc(pre - s, 0, site);
    } else {
        h[0] = g[0];
    }
}

template <typename T, typename R>
__device__ __forceinline__ void conserve_mass(R (&g)[19], R pre, uint32_t site)
{
    if constexpr (!std::is_same<T, double>::value) {
        R s = 0;
#pragma unroll
        for (int q = 1; q < 19; ++q) s += Codec<T>::dec(Codec<T>::enc(g[q], q, site), q);
        g[0] = pre - s;
    }
}

// A loaded population as the step's arithmetic holds it: decoded, or for
// SCALED only widened (it keeps the storage scaling).
template <typename T, bool SCALED>
__device__ __forceinline__ typename Compute<T>::type load_pop(T v, int q)
{
    if constexpr (SCALED)
        return (typename Compute<T>::type)v;
    else
        return Codec<T>::dec(v, q);
}

// SCALED populations to deviations (UP false) and back (UP true), around the
// boundary conditions of the few inlet and outlet sites; exact.
template <typename T, bool SCALED, bool UP, typename R>
__device__ __forceinline__ void rescale_pops(R (&g)[19])
{
    if constexpr (SCALED) {
#pragma unroll
        for (int q = 0; q < 19; ++q) g[q] *= UP ? Codec<T>::scale(q) : (R)1 / Codec<T>::scale(q);
    }
}

// Entry i of a tile header, read as the uniform value it is: through the
// constant address space (the header is never written while a step runs),
// so that it is a scalar load even where the pointer itself was read from
// memory (the batched kernels), and through readfirstlane, a convergent
// operation the compiler cannot sink into the branch of the one code kind
// that uses it. As a vector load sunk into that branch, followed by a wait
// for every load in flight, it cost the batched step a quarter of its time.
typedef const int32_t __attribute__((address_space(4))) *ConstI32;
__device__ __forceinline__ uint32_t hdr_entry(const int32_t *hdr, int i)
{
    return (uint32_t)__builtin_amdgcn_readfirstlane(((ConstI32)hdr)[i]);
}

// The byte codes of V consecutive sites from s0 (see pull_format.h):
// directions 1..16 in four words per site (w[k] holds 4k+1..4k+4), 17 and
// 18 in a 16-bit tail.
template <int V>
__device__ __forceinline__ void load_byte_codes(__amdgpu_buffer_rsrc_t rb, uint32_t s0, uint32_t npad,
                                                uint32_t (&w)[4][V], uint16_t (&tl)[V])
{
#pragma unroll
    for (int k = 0; k < 4; ++k)
        buf_load_v<V, uint32_t, uint32_t, SC_IDX_AUX>(rb, s0 * 4u, (uint32_t)k * npad * 4u, w[k]);
    buf_load_v<V, uint16_t, uint16_t, SC_IDX_AUX>(rb, s0 * 2u, 16u * npad, tl);
}

// Run codes of a 64-site wave, one site per lane (see pull_format.h): this
// lane's mask and its words of the wave's list of changed codes.
struct RunWave {
    uint32_t mask, w0, w1;
    bool wide;  // the list is longer than 256 bytes (the same on every lane)
};

__device__ __forceinline__ RunWave load_runs(__amdgpu_buffer_rsrc_t rr, uint32_t s)
{
    const auto x = buf_load_raw<8, SC_IDX_AUX>(rr, s * 8u, 0u);
    return RunWave{x[0], x[1], 0u, false};
}

// The second word of the list, for the waves that have one (a branch taken
// by the whole wave).
__device__ __forceinline__ void load_runs_wide(RunWave &r, __amdgpu_buffer_rsrc_t rr, uint32_t s, uint32_t npad)
{
    r.wide = (__builtin_amdgcn_readfirstlane(r.mask) & PULL_RUN_WIDE) != 0u;
    if (r.wide) r.w1 = buf_load_raw<4, SC_IDX_AUX>(rr, s * 4u, 8u * npad);
}

// Byte code of direction q from the wave's run codes; directions are taken
// in order 1..18 with off (0 before direction 1) counting the listed codes
// of the directions before q. Entry k of the list sits in byte k % 4 of
// lane (k / 4) % 64's first (k < 256) or second word.
__device__ __forceinline__ uint32_t run_code(const RunWave &r, int q, uint32_t &off)
{
    const uint32_t e = (r.mask >> (q - 1)) & 1u;
    const uint64_t m = __builtin_amdgcn_ballot_w64(e != 0u);
    const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
    const uint32_t k = off + below + e - 1u;  // the wave's first site lists every direction
    off += (uint32_t)__builtin_popcountll(m);
    const int addr = (int)(k & 0xFCu);
    uint32_t d = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)r.w0);
    if (r.wide) {
        const uint32_t d1 = (uint32_t)__builtin_amdgcn_ds_bpermute(addr, (int)r.w1);
        d = k >= 256u ? d1 : d;
    }
    return (d >> ((k & 3u) * 8u)) & 0xFFu;
}

// The work of one tile (SC_BLOCK threads), shared by the single-lattice
// kernel (one tile per block) and the batched kernel (a work list of tiles
// of many lattices per block).
template <typename T, bool OBS, bool BUF, bool MRT>
__device__ __forceinline__ void stream_collide_tile(const int tile, const T *__restrict__ fin,
                                                    T *__restrict__ fout, const int32_t *__restrict__ nbr,
                                                    const StepArgs &a, const int rd)
{
    using R = typename Compute<T>::type;
    constexpr int V = SC_V;
    // FP16 with BGK keeps the populations in their storage scaling from load
    // to store (see bgk_collide)
    constexpr bool SCALED = std::is_same<T, _Float16>::value && !MRT;
    const int64_t s0 = ((int64_t)tile * SC_BLOCK + threadIdx.x) * V;
    const int64_t npad = a.npad;

    R g[V][19];
    if constexpr (BUF) {
        const __amdgpu_buffer_rsrc_t rf = make_rsrc(fin, a.f_bytes);
        const __amdgpu_buffer_rsrc_t rn = make_rsrc(nbr, a.nbr_bytes);
        const uint32_t vo = (uint32_t)s0 * (uint32_t)sizeof(T);
        const uint32_t vi = (uint32_t)s0 * 4u;
        {
            T r[V];
            buf_load_v<V, T, T>(rf, vo, 0u, r);
#pragma unroll
            for (int v = 0; v < V; ++v) g[v][0] = load_pop<T, SCALED>(r[v], 0);
        }
        const int32_t *hdr = a.pull_hdr ? a.pull_hdr + (int64_t)tile * PULL_HDR : nullptr;
        // FP16 loads the codes (run codes where the table has them, else
        // byte codes) before the tile's form is known, so that their latency
        // overlaps the header's (wasted on the few tiles of another form):
        // 6 % off the FP16 step, which waits on latency, and 1 % onto the
        // FP32 step and the colour passes, which wait on bandwidth
        constexpr bool SPEC = std::is_same<T, _Float16>::value;
        // run codes: one site per lane, where the table carries them. The 10
        // bytes per site they save take 4 % off the FP32 step, which waits on
        // bandwidth, and 3 % off the FP16 step, whose latency chain their
        // decode (a ballot, a lane count and a cross-lane read per direction)
        // lengthens: that made it 3 % slower as long as its last gather
        // waited for all the others (see build.py)
        const bool runs_on = V == 1 && a.pull_runs != nullptr;
        const __amdgpu_buffer_rsrc_t rr = make_rsrc(a.pull_runs, a.runs_bytes);
        uint32_t w[4][V];
        uint16_t tl[V];
        RunWave rw{0u, 0u, 0u, false};
        if constexpr (SPEC) {
            if (hdr) {
                if (runs_on)
                    rw = load_runs(rr, (uint32_t)s0);
                else
                    load_byte_codes<V>(make_rsrc(a.pull_bytes, a.bytes_bytes), (uint32_t)s0, (uint32_t)npad, w, tl);
            }
        }
        const int form = hdr ? (int)hdr_entry(hdr, PULL_HDR_FORM) : PULL_TILE_INT32;
        const uint32_t sent = 19u * (uint32_t)npad;
        // position of each of this thread's sites in the tile
        const uint32_t p0 = (uint32_t)(s0 - (int64_t)tile * TILE);
        // byte code c of direction q: flat index = base + position + code
        auto pull_byte = [&](int q, int v, uint32_t c) {
            const uint32_t base = hdr_entry(hdr, q - 1);
            const uint32_t bb = (uint32_t)d3q19::opp(q) * (uint32_t)npad + (uint32_t)s0;
            const uint32_t idx = c <= PULL_MAX_BYTE ? base + p0 + (uint32_t)v + c
                                 : (c == PULL_BYTE_BOUNCE ? bb + (uint32_t)v : sent);
            T r[1];
            buf_load_v<1, T, T>(rf, idx * (uint32_t)sizeof(T), 0u, r);
            g[v][q] = load_pop<T, SCALED>(r[0], q);
        };
        if (form == PULL_TILE_BYTE && runs_on && hdr_entry(hdr, PULL_HDR_RUNS)) {
            if constexpr (!SPEC) rw = load_runs(rr, (uint32_t)s0);
            load_runs_wide(rw, rr, (uint32_t)s0, (uint32_t)npad);
            uint32_t off = 0;
#pragma unroll
            for (int q = 1; q < 19; ++q) pull_byte(q, 0, run_code(rw, q, off));
        } else if (form == PULL_TILE_BYTE) {
            // byte codes: directions 1..16 in four words, 17 and 18 in a
            // 16-bit tail
            if (!SPEC || runs_on)
                load_byte_codes<V>(make_rsrc(a.pull_bytes, a.bytes_bytes), (uint32_t)s0, (uint32_t)npad, w, tl);
#pragma unroll
            for (int q = 1; q < 19; ++q) {
#pragma unroll
                for (int v = 0; v < V; ++v)
                    pull_byte(q, v, q <= 16 ? (w[(q - 1) >> 2][v] >> (((q - 1) & 3) * 8)) & 0xFFu
                                            : ((uint32_t)tl[v] >> ((q - 17) * 8)) & 0xFFu);
            }
        } else if (form == PULL_TILE_HALF) {
            // 16-bit codes, two per word; flat index = base + code
            const __amdgpu_buffer_rsrc_t rc = make_rsrc(a.pull_codes, a.codes_bytes);
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                uint32_t w[V];
                buf_load_v<V, uint32_t, uint32_t, SC_IDX_AUX>(rc, vi, (uint32_t)k * (uint32_t)npad * 4u, w);
#pragma unroll
                for (int half = 0; half < 2; ++half) {
                    const int q = 2 * k + 1 + half;
                    const uint32_t base = hdr_entry(hdr, q - 1);
                    const uint32_t bb = (uint32_t)d3q19::opp(q) * (uint32_t)npad + (uint32_t)s0;
#pragma unroll
                    for (int v = 0; v < V; ++v) {
                        const uint32_t c = half ? (w[v] >> 16) : (w[v] & 0xFFFFu);
                        const uint32_t idx = c <= PULL_MAX_CODE ? base + c
                                             : (c == PULL_BOUNCE ? bb + (uint32_t)v : sent);
                        T r[1];
                        buf_load_v<1, T, T>(rf, idx * (uint32_t)sizeof(T), 0u, r);
                        g[v][q] = load_pop<T, SCALED>(r[0], q);
                    }
                }
            }
        } else {
#pragma unroll
            for (int q = 1; q < 19; ++q) {
                int32_t idx[V];
                buf_load_v<V, int32_t, int32_t, SC_IDX_AUX>(rn, vi, (uint32_t)(q - 1) * (uint32_t)npad * 4u, idx);
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    T r[1];
                    buf_load_v<1, T, T>(rf, (uint32_t)idx[v] * (uint32_t)sizeof(T), 0u, r);
                    g[v][q] = load_pop<T, SCALED>(r[0], q);
                }
            }
        }
    } else {
        {
            T r[V];
            load_v<V>(fin + s0, r);
#pragma unroll
            for (int v = 0; v < V; ++v) g[v][0] = load_pop<T, SCALED>(r[v], 0);
        }
#pragma unroll
        for (int q = 1; q < 19; ++q) {
            int32_t idx[V];
            load_v<V>(nbr + (int64_t)(q - 1) * npad + s0, idx);
#pragma unroll
            for (int v = 0; v < V; ++v) g[v][q] = load_pop<T, SCALED>(fin[idx[v]], q);
        }
    }

    // after the gathers are issued: the inlet tiles' sums and tile 0's
    // record then wait with them, and every other tile starts as before
    const double drho_in = step_begin<SC_BLOCK>(tile, a, rd);
    double uz_in = 0.0, uz_out = 0.0;
    if (tile < a.nt_in) {
#pragma unroll
        for (int v = 0; v < V; ++v)
            if (s0 + v < a.a_in) {
                rescale_pops<T, SCALED, false>(g[v]);
                uz_in += inlet_condition(g[v], drho_in, a.rho0);
                rescale_pops<T, SCALED, true>(g[v]);
            }
    }
    if (tile >= a.tout0) {
#pragma unroll
        for (int v = 0; v < V; ++v)
            if (s0 + v >= a.out0 && s0 + v < a.n) {
                rescale_pops<T, SCALED, false>(g[v]);
                uz_out += outlet_condition(g[v], cst(a.st)->drho_out, a.rho0);
                rescale_pops<T, SCALED, true>(g[v]);
            }
    }

    const R omega = (R)cst(a.st)->omega;
    double m = 0.0;
    float u2max = 0.f;
    uint32_t bad = 0;
    T h[V][19];  // the post-collision populations as stored
#pragma unroll
    for (int v = 0; v < V; ++v) {
        R drho, ux, uy, uz;
        if constexpr (MRT) {
            if (omega != (R)0) {
                mrt_collide<false>(g[v], omega, (R)a.rho0, (R)a.inv_rho0, (R)0, (R)0, (R)0, (R)0, drho, ux, uy, uz);
            } else {
                bgk_collide(g[v], omega, (R)a.rho0, (R)a.inv_rho0, drho, ux, uy, uz);
            }
        } else {
            bgk_collide<R, SCALED>(g[v], omega, (R)a.rho0, (R)a.inv_rho0, drho, ux, uy, uz);
        }
        encode_site<T, SCALED>(g[v], h[v], drho, (uint32_t)(s0 + v));  // drho: the pre-collision mass
        if (OBS) {
            m += (double)drho;
            u2max = fmaxf(u2max, (float)(ux * ux + uy * uy + uz * uz));
            bad |= !isfinite((double)drho + (double)ux + (double)uy + (double)uz);
        }
    }

    // Contribution of this tile's post-collision populations to the next
    // step's inlet sum: the pull table is a bijection, so each population of
    // planes 0-1 that an inlet site will pull carries one fixed weight. The
    // sum is taken over the values exactly as stored, so that it equals what
    // the next step's inlet sites will read.
    double s_next = 0.0;
    if (tile < a.nt01) {
#pragma unroll
        for (int v = 0; v < V; ++v)
            if (s0 + v < a.n01) {
                const uint64_t cw = a.kcoef[s0 + v];
#pragma unroll
                for (int q = 0; q < 19; ++q) {
                    const uint32_t c = (uint32_t)(cw >> (2 * q)) & 3u;
                    if (c) s_next += (double)c * (double)Codec<T>::dec(h[v][q], q);
                }
            }
    }

    if constexpr (BUF) {
        const __amdgpu_buffer_rsrc_t ro = make_rsrc(fout, a.f_bytes);
        const uint32_t vo = (uint32_t)s0 * (uint32_t)sizeof(T);
#pragma unroll
        for (int q = 0; q < 19; ++q) {
            T out[V];
#pragma unroll
            for (int v = 0; v < V; ++v) out[v] = h[v][q];
            buf_store_v_nt<V, T>(ro, vo, (uint32_t)q * (uint32_t)npad * (uint32_t)sizeof(T), out);
        }
    } else {
#pragma unroll
        for (int q = 0; q < 19; ++q) {
            T out[V];
#pragma unroll
            for (int v = 0; v < V; ++v) out[v] = h[v][q];
            store_v_nt<V>(fout + (int64_t)q * npad + s0, out);
        }
    }

    step_epilogue<SC_BLOCK, OBS>(tile, uz_in, uz_out, s_next, m, u2max, bad, a, rd);
}

template <typename T, bool OBS, bool BUF, bool MRT = false>
__global__ __launch_bounds__(SC_BLOCK) void k_stream_collide(const T *__restrict__ fin,
                                                             T *__restrict__ fout,
                                                             const int32_t *__restrict__ nbr,
                                                             StepArgs a)
{
    stream_collide_tile<T, OBS, BUF, MRT>((int)blockIdx.x, fin, fout, nbr, a, a.rd);
}

// The FP16 step, held to 80 scalar registers: it waits on latency, and the
// inlet tiles' sums and tile 0's record of the previous step (step_begin)
// took it from 78 to 83 scalar registers and its step from 130 to 134 us on
// a 256^3 pack; at 80 (the few values beyond go to VGPR lanes) it takes
// 131 us. The FP32 step gains nothing from such a bound.
template <bool OBS, bool BUF, bool MRT = false>
__global__ __launch_bounds__(SC_BLOCK) __attribute__((amdgpu_num_sgpr(80))) void k_stream_collide_h(
    const _Float16 *__restrict__ fin, _Float16 *__restrict__ fout, const int32_t *__restrict__ nbr, StepArgs a)
{
    stream_collide_tile<_Float16, OBS, BUF, MRT>((int)blockIdx.x, fin, fout, nbr, a, a.rd);
}

// Batched step: many lattices in one launch. Each lattice keeps its own
// buffers, pull table, state and partials (its StepArgs); a work list of
// (lattice, tile range) items is walked by a persistent grid, block b taking
// items b, b + gridDim.x, ... Every tile does exactly the single-lattice work,
// so each lattice's step is the same as a launch of its own.
struct BatchSample {
    StepArgs a;                 // rd holds the slot read at batch parity 0
    const void *f0, *f1;        // f0: the buffer read at batch parity 0
    const int32_t *nbr;
};

struct BatchItem {
    int32_t sample, t0, t1, pad_;
};

template <typename T, bool OBS, bool BUF, bool MRT>
__global__ __launch_bounds__(SC_BLOCK) void k_batch_step(const BatchSample *__restrict__ tab,
                                                         const BatchItem *__restrict__ work, int32_t n_work,
                                                         int32_t parity)
{
    for (int w = (int)blockIdx.x; w < n_work; w += (int)gridDim.x) {
        const BatchItem it = work[w];
        const BatchSample *S = tab + it.sample;
        const StepArgs a = S->a;
        const int rd = a.rd ^ parity;
        const T *fin = (const T *)(parity ? S->f1 : S->f0);
        T *fout = (T *)(parity ? S->f0 : S->f1);
        for (int t = it.t0; t < it.t1; ++t) {
            stream_collide_tile<T, OBS, BUF, MRT>(t, fin, fout, S->nbr, a, rd);
            __syncthreads();  // the tile's LDS reductions are reused by the next tile
        }
    }
}

// The same work with one single-tile item per block and no loop: the
// arguments then stay in scalar registers as in the single-lattice kernel
// (the loop of the persistent form costs registers and occupancy). Two
// register budgets: the compiler's choice, or at most 64 VGPRs (8 waves per
// SIMD, at the price of a few spilled registers); the autotuner picks.
template <typename T, bool OBS, bool BUF, bool MRT>
__device__ __forceinline__ void batch_tile_body(const BatchSample *__restrict__ tab,
                                                const BatchItem *__restrict__ work, int32_t parity)
{
    const BatchItem it = work[blockIdx.x];
    const BatchSample *S = tab + it.sample;
    const StepArgs a = S->a;
    const T *fin = (const T *)(parity ? S->f1 : S->f0);
    T *fout = (T *)(parity ? S->f0 : S->f1);
    stream_collide_tile<T, OBS, BUF, MRT>(it.t0, fin, fout, S->nbr, a, a.rd ^ parity);
}

template <typename T, bool OBS, bool BUF, bool MRT>
__global__ __launch_bounds__(SC_BLOCK) void k_batch_tile(const BatchSample *__restrict__ tab,
                                                         const BatchItem *__restrict__ work, int32_t parity)
{
    batch_tile_body<T, OBS, BUF, MRT>(tab, work, parity);
}

template <typename T, bool OBS, bool BUF, bool MRT>
__global__ __launch_bounds__(SC_BLOCK, 8) void k_batch_tile8(const BatchSample *__restrict__ tab,
                                                             const BatchItem *__restrict__ work, int32_t parity)
{
    batch_tile_body<T, OBS, BUF, MRT>(tab, work, parity);
}

// End of a batched step: one block per sample, as k_step_finalize.
__global__ __launch_bounds__(FIN_BLOCK) void k_batch_finalize(const BatchSample *__restrict__ tab, int32_t parity)
{
    const StepArgs a = tab[blockIdx.x].a;
    finalize_step(a, a.rd ^ parity);
}

// Reduce the per-tile observables of the last step into its history record
// (mass, max |u|) and raise the sticky watchdog flag when a value is not
// finite or |u| exceeds the limit. One block.
struct ObsArgs {
    int64_t n;
    int32_t tiles, hist_cap;   // tiles: number of per-tile partials to reduce
    double umax_limit;
    int32_t to_history;   // 1: record into the last step's history slot
    int32_t raise_flag;   // 1: a bad state sets the sticky watchdog flag
    DevState *st;
    const double *obs_mass;
    const float *obs_umax2;
    const uint32_t *obs_bad;
    const double *obs_na, *obs_nb;  // null for the single-fluid model
    double *hist;
};

constexpr int OBS_BLOCK = 1024;

__global__ __launch_bounds__(OBS_BLOCK) void k_obs_finalize(ObsArgs a)
{
    __shared__ double lds[OBS_BLOCK / 64];
    __shared__ float ldsf[OBS_BLOCK / 64];
    __shared__ uint32_t ldsu[OBS_BLOCK / 64];
    double m = 0.0;
    float u2 = 0.f;
    uint32_t bad = 0;
    for (int i = threadIdx.x; i < a.tiles; i += OBS_BLOCK) {
        m += a.obs_mass[i];
        u2 = fmaxf(u2, a.obs_umax2[i]);
        bad |= a.obs_bad[i];
    }
    m = block_sum<OBS_BLOCK>(m, lds);
    double sa = 0.0, sb = 0.0;
    if (a.obs_na) {
        for (int i = threadIdx.x; i < a.tiles; i += OBS_BLOCK) {
            sa += a.obs_na[i];
            sb += a.obs_nb[i];
        }
        sa = block_sum<OBS_BLOCK>(sa, lds);
        sb = block_sum<OBS_BLOCK>(sb, lds);
    }
    u2 = wave_max(u2);
    bad = wave_or(bad);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        ldsf[w] = u2;
        ldsu[w] = bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        float mm = 0.f;
        uint32_t bb = 0;
        for (int i = 0; i < OBS_BLOCK / 64; ++i) {
            mm = fmaxf(mm, ldsf[i]);
            bb |= ldsu[i];
        }
        DevState *st = a.st;
        const double mass = (double)a.n + m;
        const double umax = bb ? __builtin_nan("") : sqrt((double)mm);
        if (a.raise_flag && (bb || umax > a.umax_limit)) st->unstable = 1u;
        st->obs_mass = mass;
        st->obs_umax = umax;
        st->obs_bad = bb;
        if (a.to_history) {
            volatile double *h = a.hist + ((st->step - 1) % a.hist_cap) * HIST_STRIDE;
            h[3] = mass;
            h[4] = umax;
            if (a.obs_na) {
                h[6] = sa;
                h[7] = sb;
            }
        }
    }
}

// Per-tile observables of a stored state (no step): rho - 1, |u|^2, finiteness.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_state_observables(const T *__restrict__ f, int64_t npad,
                                                             double inv_rho0, double *obs_mass,
                                                             float *obs_umax2, uint32_t *obs_bad)
{
    __shared__ double lds[BLOCK / 64];
    __shared__ float ldsf[BLOCK / 64];
    __shared__ uint32_t ldsu[BLOCK / 64];
    const int64_t s = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    double d = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
    for (int q = 0; q < 19; ++q) {
        const double v = (double)Codec<T>::dec(f[(int64_t)q * npad + s], q);
        d += v;
        jx += d3q19::cx[q] * v;
        jy += d3q19::cy[q] * v;
        jz += d3q19::cz[q] * v;
    }
    const double m = block_sum<BLOCK>(d, lds);
    const double u2 = (jx * jx + jy * jy + jz * jz) * inv_rho0 * inv_rho0;
    float wm = wave_max((float)u2);
    uint32_t wb = wave_or(!isfinite(d + jx + jy + jz));
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        ldsf[w] = wm;
        ldsu[w] = wb;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        float mm = 0.f;
        uint32_t bb = 0;
        for (int i = 0; i < BLOCK / 64; ++i) {
            mm = fmaxf(mm, ldsf[i]);
            bb |= ldsu[i];
        }
        obs_mass[blockIdx.x] = m;
        obs_umax2[blockIdx.x] = mm;
        obs_bad[blockIdx.x] = bb;
    }
}

// Density and velocity of every site (FP64 [4][npad]: rho, ux, uy, uz).
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_moments(const T *__restrict__ f, int64_t n, int64_t npad,
                                                   double inv_rho0, double *__restrict__ out)
{
    const int64_t s = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (s >= n) return;
    double d = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
    for (int q = 0; q < 19; ++q) {
        const double v = (double)Codec<T>::dec(f[(int64_t)q * npad + s], q);
        d += v;
        jx += d3q19::cx[q] * v;
        jy += d3q19::cy[q] * v;
        jz += d3q19::cz[q] * v;
    }
    out[s] = 1.0 + d;
    out[npad + s] = jx * inv_rho0;
    out[2 * npad + s] = jy * inv_rho0;
    out[3 * npad + s] = jz * inv_rho0;
}

struct Dev19 {
    double v[19];
};

// Fill a distribution buffer: rows q < 19, sites < n get dev.v[q]; padding
// sites and the zero pad behind the rows get 0.
template <typename T>
__global__ __launch_bounds__(BLOCK) void k_fill(T *__restrict__ f, int64_t n, int64_t npad,
                                                int64_t total, Dev19 dev)
{
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < total;
         i += (int64_t)gridDim.x * BLOCK) {
        const int64_t q = i / npad, s = i - q * npad;
        T v = 0;
        if (q < 19 && s < n) {
            double x = 0;
#pragma unroll
            for (int k = 0; k < 19; ++k)
                if (k == q) x = dev.v[k];
            v = Codec<T>::enc((typename Codec<T>::R)x, (int)q, (uint32_t)s);
        }
        f[i] = v;
    }
}

__global__ void k_set_f64(double *p, double v) { *p = v; }
__global__ void k_set_u32(uint32_t *p, uint32_t v) { *p = v; }

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Streaming copy, one 16-byte element per thread (calibration of attainable
// HBM bandwidth). Non-temporal loads and stores: the fastest of the copy
// forms measured (plain loads, four elements per thread and plain stores
// are 5-20 % slower).
__global__ __launch_bounds__(BLOCK) void k_copy16(const u32x4 *__restrict__ src, u32x4 *__restrict__ dst,
                                                  int64_t n16)
{
    const int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i < n16) __builtin_nontemporal_store(__builtin_nontemporal_load(&src[i]), &dst[i]);
}

}  // namespace flbm
