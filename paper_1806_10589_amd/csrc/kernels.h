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

#include "d3q19.h"

namespace flbm {

constexpr int BLOCK = 256;       // sites per block of the step kernel (4 waves)
constexpr int HIST_STRIDE = 8;   // doubles per history record
constexpr int NUM_XCD = 8;       // MI355X: 8 XCDs, blocks dealt round-robin
constexpr int PLANE_MAX_BLOCKS = 1024;

// FP64 scalars shared by the kernels of a step. Written by single threads
// with vector stores; read by every block.
struct DevState {
    double q_target;      // Q*
    double drho_out;      // rho_out - 1
    double drho_in;       // rho_in - 1 of the step in progress
    double omega;         // 1/tau (0 turns collision off)
    double obs_mass;      // on-demand observables
    double obs_umax;
    int64_t step;         // steps completed
    uint32_t k_ticket;    // last-block tickets of the two reductions
    uint32_t b_ticket;
    uint32_t unstable;    // sticky watchdog flag
    uint32_t obs_bad;
};

struct StepArgs {
    int64_t n, npad;
    int64_t a_in;         // inlet sites [0, a_in)
    int64_t out0;         // outlet sites [out0, n)
    int32_t nt_in;        // tiles holding inlet sites: [0, nt_in)
    int32_t tout0;        // tiles holding outlet sites: [tout0, tiles)
    int32_t n_bnd;        // tiles taking part in the boundary ticket
    int32_t hist_cap;
    int32_t flux_mode;
    int32_t pad_;
    double rho0, inv_rho0;
    DevState *st;
    double *bpart_in, *bpart_out;   // per-tile sums of u_z
    double *obs_mass;               // per-tile sums of rho - 1
    float *obs_umax2;               // per-tile max |u|^2
    uint32_t *obs_bad;              // per-tile non-finite flag
    double *hist;
};

struct PlaneArgs {
    int64_t npad, a_in;
    int32_t hist_cap;
    int32_t pad_;
    double rho0;
    DevState *st;
    double *kpart;
    double *hist;
};

template <typename T> struct Compute;
template <> struct Compute<float> { using type = float; };
template <> struct Compute<double> { using type = double; };

// Block index -> tile: the hardware deals consecutive blocks round-robin to
// the 8 XCDs; this map gives each XCD one contiguous run of tiles, so the
// cache lines that neighbouring tiles share stay in one XCD's L2.
__device__ __forceinline__ int xcd_tile(int b, int nb)
{
    const int q = nb / NUM_XCD, r = nb % NUM_XCD;
    const int x = b % NUM_XCD, k = b / NUM_XCD;
    return x * q + (x < r ? x : r) + k;
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
template <typename R>
__device__ __forceinline__ double inlet_condition(R (&g)[19], double drho_in, double rho0)
{
    double k = 0.0;
#pragma unroll
    for (int q = 0; q < 19; ++q)
        if (d3q19::inlet_coeff(q)) k += d3q19::inlet_coeff(q) * (double)g[q];
    const double uz = (drho_in - k) / rho0;
    const double nx = 0.5 * ((double)g[1] + (double)g[7] + (double)g[9] -
                             ((double)g[2] + (double)g[10] + (double)g[8]));
    const double ny = 0.5 * ((double)g[3] + (double)g[7] + (double)g[10] -
                             ((double)g[4] + (double)g[9] + (double)g[8]));
    const double ru = rho0 * uz;
    g[5] = (R)((double)g[6] + ru / 3.0);
    g[11] = (R)((double)g[12] + ru / 6.0 - nx);
    g[14] = (R)((double)g[13] + ru / 6.0 + nx);
    g[15] = (R)((double)g[16] + ru / 6.0 - ny);
    g[18] = (R)((double)g[17] + ru / 6.0 + ny);
    return uz;
}

// The same condition at an outlet site with density 1 + drho_out, the
// closure rows solved for the outlet unknowns 6, 12, 13, 16, 17.
template <typename R>
__device__ __forceinline__ double outlet_condition(R (&g)[19], double drho_out, double rho0)
{
    double k = 0.0;
#pragma unroll
    for (int q = 0; q < 19; ++q)
        if (d3q19::outlet_coeff(q)) k += d3q19::outlet_coeff(q) * (double)g[q];
    const double uz = (k - drho_out) / rho0;
    const double nx = 0.5 * ((double)g[1] + (double)g[7] + (double)g[9] -
                             ((double)g[2] + (double)g[10] + (double)g[8]));
    const double ny = 0.5 * ((double)g[3] + (double)g[7] + (double)g[10] -
                             ((double)g[4] + (double)g[9] + (double)g[8]));
    const double ru = rho0 * uz;
    g[6] = (R)((double)g[5] - ru / 3.0);
    g[12] = (R)((double)g[11] - ru / 6.0 + nx);
    g[13] = (R)((double)g[14] - ru / 6.0 - nx);
    g[16] = (R)((double)g[15] - ru / 6.0 + ny);
    g[17] = (R)((double)g[18] - ru / 6.0 - ny);
    return uz;
}

// --------------------------------------------------------------- collision

// BGK relaxation toward the incompressible equilibrium
//   f_eq = w_q [rho + rho0 (3 xi.u + 9/2 (xi.u)^2 - 3/2 u.u)],  u = j/rho0,
// written for deviations: g_eq = w_q [(rho - 1) + rho0 (...)].
// On return g holds the post-collision deviations; drho, u the moments.
template <typename R>
__device__ __forceinline__ void bgk_collide(R (&g)[19], R omega, R rho0, R inv_rho0, R &drho,
                                            R &ux, R &uy, R &uz)
{
    R d = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
    for (int q = 0; q < 19; ++q) {
        d += g[q];
        if (d3q19::cx[q]) jx += d3q19::cx[q] > 0 ? g[q] : -g[q];
        if (d3q19::cy[q]) jy += d3q19::cy[q] > 0 ? g[q] : -g[q];
        if (d3q19::cz[q]) jz += d3q19::cz[q] > 0 ? g[q] : -g[q];
    }
    ux = jx * inv_rho0;
    uy = jy * inv_rho0;
    uz = jz * inv_rho0;
    drho = d;
    const R base = d - rho0 * (R)1.5 * (ux * ux + uy * uy + uz * uz);
#pragma unroll
    for (int q = 0; q < 19; ++q) {
        R cu = 0;
        if (d3q19::cx[q]) cu += d3q19::cx[q] > 0 ? ux : -ux;
        if (d3q19::cy[q]) cu += d3q19::cy[q] > 0 ? uy : -uy;
        if (d3q19::cz[q]) cu += d3q19::cz[q] > 0 ? uz : -uz;
        const R geq = (R)d3q19::weight(q) * (base + rho0 * cu * ((R)3 + (R)4.5 * cu));
        g[q] += omega * (geq - g[q]);
    }
}

// --------------------------------------------------------------- kernels

// Inlet plane reduction (eq. potential). Each thread sums the consistency
// sums of its inlet sites from the streamed (pulled) values; blocks write
// FP64 partials; the last block to finish sums them in block order and sets
// rho_in - 1 = (rho0 Q* + sum_i Kt_i) / A for the step kernel.
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
        double ki = (double)fin[i];
#pragma unroll
        for (int q = 1; q < 19; ++q)
            if (d3q19::inlet_coeff(q))
                ki += d3q19::inlet_coeff(q) * (double)fin[nbr[(int64_t)(q - 1) * a.npad + i]];
        k += ki;
    }
    k = block_sum<BLOCK>(k, lds);
    if (threadIdx.x == 0) {
        a.kpart[blockIdx.x] = k;
        __threadfence();
        const uint32_t prev = atomicAdd(&a.st->k_ticket, 1u);
        is_last = (prev == gridDim.x - 1);
    }
    __syncthreads();
    if (!is_last) return;
    __threadfence();
    double s = 0.0;
    for (int i = threadIdx.x; i < (int)gridDim.x; i += BLOCK) s += a.kpart[i];
    s = block_sum<BLOCK>(s, lds);
    if (threadIdx.x == 0) {
        DevState *st = a.st;
        const double drho = (a.rho0 * st->q_target + s) / (double)a.a_in;
        st->drho_in = drho;
        const int64_t slot = st->step % a.hist_cap;
        a.hist[slot * HIST_STRIDE + 0] = 1.0 + drho;
        st->k_ticket = 0;
    }
}

// Fused step for every site: pull the 19 populations, apply the inlet or
// outlet pressure condition where the site lies on z = 0 or z = nz-1, BGK
// collide, store. Tiles holding boundary sites also reduce sum u_z (FP64)
// and the last of them records Q_in, Q_out and advances the step counter.
// OBS: also write per-tile partials of mass, max |u|^2 and a non-finite flag.
template <typename T, bool OBS>
__global__ __launch_bounds__(BLOCK) void k_stream_collide(const T *__restrict__ fin,
                                                          T *__restrict__ fout,
                                                          const int32_t *__restrict__ nbr,
                                                          StepArgs a)
{
    using R = typename Compute<T>::type;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int64_t s = (int64_t)tile * BLOCK + threadIdx.x;
    const int64_t npad = a.npad;

    R g[19];
    g[0] = (R)fin[s];
#pragma unroll
    for (int q = 1; q < 19; ++q) g[q] = (R)fin[nbr[(int64_t)(q - 1) * npad + s]];

    double uz_in = 0.0, uz_out = 0.0;
    if (tile < a.nt_in && s < a.a_in) uz_in = inlet_condition(g, a.st->drho_in, a.rho0);
    if (tile >= a.tout0 && s >= a.out0 && s < a.n)
        uz_out = outlet_condition(g, a.st->drho_out, a.rho0);

    R drho, ux, uy, uz;
    bgk_collide(g, (R)a.st->omega, (R)a.rho0, (R)a.inv_rho0, drho, ux, uy, uz);

#pragma unroll
    for (int q = 0; q < 19; ++q) __builtin_nontemporal_store((T)g[q], &fout[(int64_t)q * npad + s]);

    __shared__ double lds[BLOCK / 64];
    __shared__ float ldsf[BLOCK / 64];
    __shared__ uint32_t ldsu[BLOCK / 64];
    if (OBS) {
        const double m = block_sum<BLOCK>((double)drho, lds);
        const float u2 = (float)(ux * ux + uy * uy + uz * uz);
        const uint32_t bad = !isfinite((double)drho + (double)ux + (double)uy + (double)uz);
        float wm = wave_max(u2);
        uint32_t wb = wave_or(bad);
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
            for (int i = 0; i < BLOCK / 64; ++i) {
                mm = fmaxf(mm, ldsf[i]);
                bb |= ldsu[i];
            }
            a.obs_mass[tile] = m;
            a.obs_umax2[tile] = mm;
            a.obs_bad[tile] = bb;
        }
    }

    const bool bnd_tile = a.flux_mode ? (tile < a.nt_in || tile >= a.tout0) : (tile == 0);
    if (!bnd_tile) return;
    __shared__ int is_last;
    const double si = block_sum<BLOCK>(uz_in, lds);
    const double so = block_sum<BLOCK>(uz_out, lds);
    if (threadIdx.x == 0) {
        if (tile < a.nt_in) a.bpart_in[tile] = si;
        if (a.flux_mode && tile >= a.tout0) a.bpart_out[tile - a.tout0] = so;
        __threadfence();
        const uint32_t prev = atomicAdd(&a.st->b_ticket, 1u);
        is_last = (prev == (uint32_t)a.n_bnd - 1);
    }
    __syncthreads();
    if (!is_last) return;
    __threadfence();
    const int nt_out = a.flux_mode ? (int)((a.npad / BLOCK) - a.tout0) : 0;
    double ti = 0.0, to = 0.0;
    for (int i = threadIdx.x; i < a.nt_in; i += BLOCK) ti += a.bpart_in[i];
    for (int i = threadIdx.x; i < nt_out; i += BLOCK) to += a.bpart_out[i];
    ti = block_sum<BLOCK>(ti, lds);
    to = block_sum<BLOCK>(to, lds);
    if (threadIdx.x == 0) {
        DevState *st = a.st;
        const int64_t t = st->step;
        double *h = a.hist + (t % a.hist_cap) * HIST_STRIDE;
        if (!a.flux_mode) h[0] = __builtin_nan("");
        h[1] = a.flux_mode ? ti : __builtin_nan("");
        h[2] = a.flux_mode ? to : __builtin_nan("");
        h[3] = __builtin_nan("");
        h[4] = __builtin_nan("");
        h[5] = (double)(t + 1);
        st->step = t + 1;
        st->b_ticket = 0;
    }
}

// Reduce the per-tile observables of the last step into its history record
// (mass, max |u|) and raise the sticky watchdog flag when a value is not
// finite or |u| exceeds the limit. One block.
struct ObsArgs {
    int64_t n;
    int32_t tiles, hist_cap;
    double umax_limit;
    int32_t to_history;   // 1: record into the last step's history slot
    int32_t raise_flag;   // 1: a bad state sets the sticky watchdog flag
    DevState *st;
    const double *obs_mass;
    const float *obs_umax2;
    const uint32_t *obs_bad;
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
            double *h = a.hist + ((st->step - 1) % a.hist_cap) * HIST_STRIDE;
            h[3] = mass;
            h[4] = umax;
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
        const double v = (double)f[(int64_t)q * npad + s];
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
        const double v = (double)f[(int64_t)q * npad + s];
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
            v = (T)x;
        }
        f[i] = v;
    }
}

__global__ void k_set_f64(double *p, double v) { *p = v; }
__global__ void k_set_u32(uint32_t *p, uint32_t v) { *p = v; }

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Streaming copy, 16-byte lanes (calibration of attainable HBM bandwidth).
__global__ __launch_bounds__(BLOCK) void k_copy16(const u32x4 *__restrict__ src, u32x4 *__restrict__ dst,
                                                  int64_t n16)
{
    for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n16;
         i += (int64_t)gridDim.x * BLOCK)
        __builtin_nontemporal_store(src[i], &dst[i]);
}

}  // namespace flbm
