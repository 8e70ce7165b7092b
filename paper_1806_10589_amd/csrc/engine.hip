// C-ABI of the library: context, device memory, step orchestration, the
// learned inlet controller and batched stepping.
//
// One single-fluid step is one launch on the caller's stream (Methods, the
// paragraph after eq. potential: the inlet density is found from the
// streamed knowns, then the pressure condition is applied, then collision):
// k_stream_collide pulls, applies the boundary conditions with the inlet
// density of eq. potential, collides (BGK or MRT), stores, and writes per-tile
// partials of Q_in, Q_out and of the inlet sum that the next step's inlet
// sites will pull; the next step kernel reduces them (step_begin), and after
// the last step of a run k_step_finalize (one block) does. With pull streaming
// the "streamed" values of a step are gathers of the stored state, so no
// grid-wide barrier is needed inside a step; k_inlet_plane computes the sum
// from the state only after the host has written it. The colour model adds
// a phase pass before its step kernel. The buffers alternate every step.
// Runs of steps are captured once per starting buffer as a HIP graph and
// replayed; the last step of each run also reduces the watchdog observables.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/fluxlbm.h"
#include "colour.h"
#include "kernels.h"
#include "lattice.h"
#include "markers.h"
#include "mlp.h"
#include "mlp_ctx.h"

using namespace flbm;

namespace {

constexpr int HIST_CAP = 8192;
constexpr int64_t SENT_PAD = 64;

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

struct flbm_ctx {
    flbm_params p{};
    LatticeSpec spec;
    Lattice lat;
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    std::string err;

    // launch geometry
    int tiles = 0, nt_in = 0, nt01 = 0, tout0 = 0, plane_blocks = 0;
    int blocks256 = 0;  // n_pad / BLOCK: grid of the one-site-per-thread kernels
    bool use_buf = false; // f and nbr each below 4 GiB: buffer-instruction path
    bool need_plane = true; // the carried inlet sum is stale (state set from the host)
    int obs_slots = 0;  // per-tile observable partials: max(tiles, blocks256)
    size_t elem = 4;  // bytes per stored population

    // device memory
    void *dmem = nullptr;
    size_t dbytes = 0;
    bool owned = false, ready = false;
    void *f[2] = {nullptr, nullptr};
    int cur = 0;
    int32_t *nbr = nullptr;
    // compact pull table (buffer path)
    CompactPull pull;
    int pull_format = FLBM_PULL_INT32;
    uint32_t *pull_codes = nullptr, *pull_bytes = nullptr, *pull_runs = nullptr;
    int32_t *pull_hdr = nullptr;
    DevState *st = nullptr;
    double *kpart = nullptr, *bpart_in = nullptr, *bpart_out = nullptr, *spart = nullptr;
    uint64_t *kcoef = nullptr;
    double *obs_mass = nullptr;
    float *obs_umax2 = nullptr;
    uint32_t *obs_bad = nullptr;
    double *hist = nullptr;
    double *fields = nullptr;
    // two-fluid colour model
    bool colour = false;
    void *cab[2] = {nullptr, nullptr};  // colour pairs (A_q, B_q) [7][n_pad]
    void *nab = nullptr;                // (N_A, N_B) pairs [n_pad]
    void *phi = nullptr;                // phase field [n_pad]
    double *obs_na = nullptr, *obs_nb = nullptr;
    // learned inlet controller
    bool ctrl_on = false;
    const flbm_mlp *ctrl_net = nullptr;
    flbm_controller_params ctrl{};
    float *ctrl_feat = nullptr;   // [16] geometry inputs on the device
    float *ctrl_trace = nullptr;  // [HIST_CAP][CTRL_REC] decision records
    double *ctrl_ring = nullptr;  // [256] period-mean outlet fluxes

    // host bookkeeping
    int64_t steps = 0;
    int collide = 1;
    int chunk = 0;
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    bool use_graph = true;
    bool markers = false;  // FLBM_PROFILE=1: roctx ranges per launch, direct launches (no graphs)
};

namespace {

flbm_status fail(flbm_ctx *c, flbm_status code, const std::string &msg)
{
    if (c) c->err = msg;
    return code;
}

#define HIPCHK(c, expr)                                                                       \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail((c), FLBM_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));  \
    } while (0)

bool is_fp64(const flbm_ctx *c) { return c->p.precision == FLBM_FP64; }
// element size of the colour state (A, B, N_A, N_B, phi): FP64, else FP32
size_t colour_elem(const flbm_ctx *c) { return is_fp64(c) ? 8 : 4; }

// Call fn(T{}) with T the storage type of the distributions.
template <typename Fn>
void with_storage(const flbm_ctx *c, Fn &&fn)
{
    if (c->p.precision == FLBM_FP64)
        fn(double{});
    else if (c->p.precision == FLBM_FP16DEV)
        fn(_Float16{});
    else
        fn(float{});
}

// Host-side codec of the stored deviations (the device codec's mirror).
template <typename T> double host_dec(T v, int) { return (double)v; }
template <typename T> T host_enc(double g, int) { return (T)g; }
template <> double host_dec<_Float16>(_Float16 v, int q)
{
    return (double)v / (double)(1u << d3q19::half_shift(q));
}
template <> _Float16 host_enc<_Float16>(double g, int q)
{
    return (_Float16)(float)(g * (double)(1u << d3q19::half_shift(q)));
}

// byte codes: [4][n_pad] words, then the [n_pad] 16-bit row
size_t pull_bytes_size(const flbm_ctx *c)
{
    return c->pull.bytes.size() * sizeof(uint32_t) + c->pull.tail.size() * sizeof(uint16_t);
}

// run codes: [n_pad][2] words, then the [n_pad] second words
size_t pull_runs_size(const flbm_ctx *c)
{
    return (c->pull.runs.size() + c->pull.runs_hi.size()) * sizeof(uint32_t);
}

flbm_status upload_pull(flbm_ctx *c)
{
    HIPCHK(c, hipMemcpyAsync(c->pull_codes, c->pull.codes.data(), c->pull.codes.size() * sizeof(uint32_t),
                             hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->pull_bytes, c->pull.bytes.data(), c->pull.bytes.size() * sizeof(uint32_t),
                             hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync((char *)c->pull_bytes + c->pull.bytes.size() * sizeof(uint32_t), c->pull.tail.data(),
                             c->pull.tail.size() * sizeof(uint16_t), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->pull_runs, c->pull.runs.data(), c->pull.runs.size() * sizeof(uint32_t),
                             hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->pull_runs + c->pull.runs.size(), c->pull.runs_hi.data(),
                             c->pull.runs_hi.size() * sizeof(uint32_t), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(c->pull_hdr, c->pull.hdr.data(), c->pull.hdr.size() * sizeof(int32_t),
                             hipMemcpyHostToDevice, c->stream));
    return FLBM_OK;
}

size_t f_bytes(const flbm_ctx *c) { return (size_t)(19 * c->lat.n_pad + SENT_PAD) * c->elem; }

// Carve the device slab. With base == nullptr only the size is computed.
size_t carve(flbm_ctx *c, char *base)
{
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        char *p = base ? base + off : nullptr;
        off += align256(bytes);
        return p;
    };
    const int64_t npad = c->lat.n_pad;
    char *f0 = take(f_bytes(c));
    char *f1 = take(f_bytes(c));
    char *nb = take((size_t)18 * npad * sizeof(int32_t));
    char *pcw = c->pull.tiles ? take(c->pull.codes.size() * sizeof(uint32_t)) : nullptr;
    char *pcb = c->pull.tiles ? take(pull_bytes_size(c)) : nullptr;
    char *pch = c->pull.tiles ? take(c->pull.hdr.size() * sizeof(int32_t)) : nullptr;
    char *pcr = c->pull.tiles ? take(pull_runs_size(c)) : nullptr;
    char *st = take(sizeof(DevState));
    char *kp = take(PLANE_MAX_BLOCKS * sizeof(double));
    // boundary partials: two slots (the step that wrote buffer 0, 1) of one per tile
    char *bi = take((size_t)2 * c->tiles * sizeof(double));
    char *bo = take((size_t)2 * c->tiles * sizeof(double));
    char *sp = take((size_t)2 * c->tiles * sizeof(double));
    char *kc = take((size_t)std::max<int64_t>(1, (int64_t)c->lat.kcoef.size()) * sizeof(uint64_t));
    char *om = take((size_t)c->obs_slots * sizeof(double));
    char *ou = take((size_t)c->obs_slots * sizeof(float));
    char *ob = take((size_t)c->obs_slots * sizeof(uint32_t));
    char *hi = take((size_t)HIST_CAP * HIST_STRIDE * sizeof(double));
    char *fl = take((size_t)4 * npad * sizeof(double));
    char *cf = take(16 * sizeof(float));
    char *ct = take((size_t)HIST_CAP * 40 * sizeof(float));
    char *cr = take(256 * sizeof(double));
    char *cc[4] = {nullptr, nullptr, nullptr, nullptr};
    char *on = nullptr, *ob2 = nullptr;
    if (c->colour) {
        for (int i = 0; i < 2; ++i) cc[i] = take((size_t)7 * npad * 2 * colour_elem(c));
        cc[2] = take((size_t)npad * 2 * colour_elem(c));
        cc[3] = take((size_t)npad * colour_elem(c));
        on = take((size_t)c->obs_slots * sizeof(double));
        ob2 = take((size_t)c->obs_slots * sizeof(double));
    }
    if (base) {
        c->f[0] = f0;
        c->f[1] = f1;
        c->nbr = (int32_t *)nb;
        c->pull_codes = (uint32_t *)pcw;
        c->pull_bytes = (uint32_t *)pcb;
        c->pull_hdr = (int32_t *)pch;
        c->pull_runs = (uint32_t *)pcr;
        c->st = (DevState *)st;
        c->kpart = (double *)kp;
        c->bpart_in = (double *)bi;
        c->bpart_out = (double *)bo;
        c->spart = (double *)sp;
        c->kcoef = (uint64_t *)kc;
        c->obs_mass = (double *)om;
        c->obs_umax2 = (float *)ou;
        c->obs_bad = (uint32_t *)ob;
        c->hist = (double *)hi;
        c->fields = (double *)fl;
        c->ctrl_feat = (float *)cf;
        c->ctrl_trace = (float *)ct;
        c->ctrl_ring = (double *)cr;
        if (c->colour) {
            c->cab[0] = cc[0];
            c->cab[1] = cc[1];
            c->nab = cc[2];
            c->phi = cc[3];
            c->obs_na = (double *)on;
            c->obs_nb = (double *)ob2;
        }
    }
    return off;
}

StepArgs step_args(const flbm_ctx *c)
{
    StepArgs a{};
    a.n = c->lat.n;
    a.npad = c->lat.n_pad;
    a.f_bytes = c->use_buf ? (uint32_t)f_bytes(c) : 0u;
    a.nbr_bytes = c->use_buf ? (uint32_t)((uint64_t)18 * c->lat.n_pad * 4) : 0u;
    const bool flux = c->p.z_mode == FLBM_Z_FLUX;
    a.a_in = flux ? c->lat.a_in : 0;
    a.out0 = flux ? c->lat.n - c->lat.a_out : c->lat.n;
    a.n01 = flux ? c->lat.n01 : 0;
    a.nt_in = flux ? c->nt_in : 0;
    a.nt01 = flux ? c->nt01 : 0;
    a.kcoef = c->kcoef;
    a.spart = c->spart;
    a.tout0 = flux ? c->tout0 : c->tiles;
    a.hist_cap = HIST_CAP;
    const bool compact = c->pull_format != FLBM_PULL_INT32 && c->use_buf && c->pull.tiles > 0;
    a.pull_codes = compact ? c->pull_codes : nullptr;
    a.pull_bytes = compact ? c->pull_bytes : nullptr;
    a.pull_hdr = compact ? c->pull_hdr : nullptr;
    a.codes_bytes = compact ? (uint32_t)(c->pull.codes.size() * sizeof(uint32_t)) : 0u;
    a.bytes_bytes = compact ? (uint32_t)pull_bytes_size(c) : 0u;
    const bool runs = compact && c->pull_format == FLBM_PULL_RUN && c->pull.tiles_run > 0;
    a.pull_runs = runs ? c->pull_runs : nullptr;
    a.runs_bytes = runs ? (uint32_t)pull_runs_size(c) : 0u;
    a.flux_mode = flux;
    a.rho0 = c->p.rho0;
    a.inv_rho0 = 1.0 / c->p.rho0;
    a.st = c->st;
    a.bpart_in = c->bpart_in;
    a.bpart_out = c->bpart_out;
    a.part_stride = c->tiles;
    a.obs_mass = c->obs_mass;
    a.obs_umax2 = c->obs_umax2;
    a.obs_bad = c->obs_bad;
    a.obs_na = c->obs_na;
    a.obs_nb = c->obs_nb;
    a.hist = c->hist;
    return a;
}

PlaneArgs plane_args(const flbm_ctx *c, int slot)
{
    PlaneArgs a{};
    a.npad = c->lat.n_pad;
    a.a_in = c->lat.a_in;
    a.slot = slot;
    a.st = c->st;
    a.kpart = c->kpart;
    return a;
}

ObsArgs obs_args(const flbm_ctx *c, int to_history, int partials)
{
    ObsArgs a{};
    a.n = c->lat.n;
    a.tiles = partials;
    a.hist_cap = HIST_CAP;
    a.umax_limit = c->p.umax_limit;
    a.to_history = to_history;
    a.raise_flag = c->p.watchdog_every > 0;
    a.st = c->st;
    a.obs_mass = c->obs_mass;
    a.obs_umax2 = c->obs_umax2;
    a.obs_bad = c->obs_bad;
    a.obs_na = to_history ? c->obs_na : nullptr;
    a.obs_nb = to_history ? c->obs_nb : nullptr;
    a.hist = c->hist;
    return a;
}

// The two launches of a colour step from buffer `from`.
template <typename T>
void launch_colour_step(flbm_ctx *c, hipStream_t s, int from, bool obs)
{
    PhaseArgs p{};
    p.n = c->lat.n;
    p.npad = c->lat.n_pad;
    const bool flux = c->p.z_mode == FLBM_Z_FLUX;
    p.a_in = flux ? c->lat.a_in : 0;
    p.out0 = flux ? c->lat.n - c->lat.a_out : c->lat.n;
    p.sentinel = c->lat.sentinel;
    p.flux_mode = flux;
    p.rd = from;
    p.rho0 = c->p.rho0;
    p.st = c->st;
    p.nbr = c->nbr;
    p.fin = c->f[from];
    p.abin = c->cab[from];
    p.about = c->cab[from ^ 1];
    p.nab = c->nab;
    p.phi = c->phi;
    StepArgs a = step_args(c);
    a.rd = from;
    {
        Range r(c->markers, "flbm phase pass");
        if (c->use_buf)
            hipLaunchKernelGGL(k_phase_buf<T>, dim3(c->tiles), dim3(TILE / PHASE_V), 0, s, p, a);
        else
            hipLaunchKernelGGL(k_phase<T>, dim3(c->blocks256), dim3(BLOCK), 0, s, p);
    }
    ColourStepArgs cs{};
    cs.alpha = c->p.alpha;
    cs.beta = c->p.beta;
    cs.phi_solid = c->p.phi_solid;
    cs.sentinel = c->lat.sentinel;
    cs.nab = c->nab;
    cs.phi = c->phi;
    cs.about = c->cab[from ^ 1];
    const T *fin = (const T *)c->f[from];
    T *fout = (T *)c->f[from ^ 1];
    Range r(c->markers, "flbm colour step");
    if (c->use_buf) {
        const dim3 grid(c->tiles);
        if (obs)
            hipLaunchKernelGGL((k_colour_buf<T, true>), grid, dim3(TILE), 0, s, fin, fout, c->nbr, a, cs);
        else
            hipLaunchKernelGGL((k_colour_buf<T, false>), grid, dim3(TILE), 0, s, fin, fout, c->nbr, a, cs);
    } else if (obs) {
        hipLaunchKernelGGL((k_colour<T, true>), dim3(c->tiles), dim3(TILE), 0, s, fin, fout, c->nbr, a, cs);
    } else {
        hipLaunchKernelGGL((k_colour<T, false>), dim3(c->tiles), dim3(TILE), 0, s, fin, fout, c->nbr, a, cs);
    }
}

// The fused kernel in its variants: with or without the watchdog partials;
// buffer instructions (buffers below 4 GiB) or 64-bit addressing; BGK or
// single-fluid MRT collision.
template <typename T, bool OBS, bool BUF, bool MRT>
void launch_sc(dim3 grid, hipStream_t s, const T *fin, T *fout, const int32_t *nbr, const StepArgs &a)
{
    if constexpr (std::is_same<T, _Float16>::value)
        hipLaunchKernelGGL((k_stream_collide_h<OBS, BUF, MRT>), grid, dim3(SC_BLOCK), 0, s, fin, fout, nbr, a);
    else
        hipLaunchKernelGGL((k_stream_collide<T, OBS, BUF, MRT>), grid, dim3(SC_BLOCK), 0, s, fin, fout, nbr, a);
}

template <typename T, bool MRT>
void launch_stream_collide_c(flbm_ctx *c, hipStream_t s, const T *fin, T *fout, bool obs, const StepArgs &a)
{
    Range r(c->markers, "flbm stream-collide");
    const dim3 grid(c->tiles);
    if (c->use_buf) {
        if (obs)
            launch_sc<T, true, true, MRT>(grid, s, fin, fout, c->nbr, a);
        else
            launch_sc<T, false, true, MRT>(grid, s, fin, fout, c->nbr, a);
    } else {
        if (obs)
            launch_sc<T, true, false, MRT>(grid, s, fin, fout, c->nbr, a);
        else
            launch_sc<T, false, false, MRT>(grid, s, fin, fout, c->nbr, a);
    }
}

template <typename T>
void launch_stream_collide(flbm_ctx *c, hipStream_t s, const T *fin, T *fout, bool obs)
{
    StepArgs a = step_args(c);
    a.rd = fin == (const T *)c->f[1] ? 1 : 0;
    if (c->p.model == FLBM_MRT)
        launch_stream_collide_c<T, true>(c, s, fin, fout, obs, a);
    else
        launch_stream_collide_c<T, false>(c, s, fin, fout, obs, a);
}

// The end of a step read from buffer `from` (after its step kernel): Q_in,
// Q_out, the next inlet sum, the history record and the step counter.
void launch_finalize(flbm_ctx *c, hipStream_t s, int from)
{
    Range r(c->markers, "flbm step finalize");
    StepArgs a = step_args(c);
    a.rd = from;
    hipLaunchKernelGGL(k_step_finalize, dim3(1), dim3(FIN_BLOCK), 0, s, a);
}

// Enqueue one step from buffer `from` on stream s; fin: end it with
// k_step_finalize (else the next step kernel ends it, see step_begin).
template <typename T>
void launch_step(flbm_ctx *c, hipStream_t s, int from, bool obs, bool fin)
{
    const T *fin_buf = (const T *)c->f[from];
    T *fout = (T *)c->f[from ^ 1];
    launch_stream_collide<T>(c, s, fin_buf, fout, obs);
    if (fin || obs) launch_finalize(c, s, from);
    if (obs) {
        Range r(c->markers, "flbm observables");
        hipLaunchKernelGGL(k_obs_finalize, dim3(1), dim3(OBS_BLOCK), 0, s, obs_args(c, 1, c->tiles));
    }
}

void launch_step_plain(flbm_ctx *c, hipStream_t s, int from, bool obs, bool fin)
{
    if (c->colour) {
        with_storage(c, [&](auto tag) { launch_colour_step<decltype(tag)>(c, s, from, obs); });
        launch_finalize(c, s, from);
        if (obs) {
            Range r(c->markers, "flbm observables");
            hipLaunchKernelGGL(k_obs_finalize, dim3(1), dim3(OBS_BLOCK), 0, s, obs_args(c, 1, c->tiles));
        }
        return;
    }
    with_storage(c, [&](auto tag) { launch_step<decltype(tag)>(c, s, from, obs, fin); });
}

// Learned inlet controller (one workgroup, launched after every step
// kernel). Every step it adds the outlet flux to the current period's sum;
// every `period` steps it closes the period (pushing its mean outlet flux into
// a ring) and decides: it builds the network's inputs -- 15 geometry values,
// the period-mean outlet-flux errors at 16 log-spaced lags (in periods) and
// the scale of the current inlet-outlet density difference -- runs the
// network (MFMA, BF16 operands, FP32 accumulation) and holds the proposed
// inlet density with the decaying trust bound for the next period; the step
// kernel moves the plain density of eq. potential towards it by at most that
// bound every step. No proposal once the outlet flux has met the release
// tolerance or stopped improving (for good), for Q* <= 0, or when the output
// is not finite. With the period scaled to the charging time of the sample
// (which grows as its length squared), the inputs look alike across sizes.
constexpr int CTRL_LAGS[16] = {1, 2, 3, 4, 6, 8, 11, 16, 22, 32, 45, 64, 90, 128, 180, 250};
constexpr int CTRL_RING = 256;  // period means kept (> the longest lag)
constexpr int CTRL_REC = 40;    // floats per trace record: x[32], then 4 doubles

struct CtrlArgs {
    DevState *st;
    const double *hist;
    double *ring;  // [CTRL_RING] period-mean outlet fluxes
    float *trace;  // [HIST_CAP][CTRL_REC], one record per decision
    int32_t hist_cap;
    int32_t trust_decisions;
    int32_t rd_next;
    int32_t relative;
    int32_t stall_decisions;
    int32_t period;
    const float *params;
    const float *geometry;
    double rho0, a_in, drho_ref, gain, trust0, release_tol, margin;
};

__global__ __launch_bounds__(256) void k_controller(CtrlArgs c)
{
    __shared__ float x[mlp::N_IN];
    __shared__ float h1[mlp::N_HID], h2[mlp::N_HID];
    DevState *st = c.st;
    const int64_t t = st->step;  // steps completed; the last one has index t - 1
    if (t < 1) return;
    const bool decide = (t % c.period) == 0;
    if (threadIdx.x == 0) {
        const double q = c.hist[((t - 1) % c.hist_cap) * HIST_STRIDE + 2];
        double acc = st->ctrl_acc + (isfinite(q) ? q : 0.0);
        if (decide) {
            c.ring[st->ctrl_periods % CTRL_RING] = acc / (double)c.period;
            st->ctrl_periods += 1;
            acc = 0.0;
        }
        st->ctrl_acc = acc;
    }
    if (!decide) return;
    __syncthreads();
    const int64_t np = st->ctrl_periods;
    const double qs = st->q_target;
    const double qn = qs != 0.0 ? fabs(qs) : 1.0;
    auto qbar = [&](int64_t k) -> double {  // mean outlet flux of period k; rest before the first
        return k >= 0 ? c.ring[k % CTRL_RING] : 0.0;
    };
    const double rin = c.hist[((t - 1) % c.hist_cap) * HIST_STRIDE + 0];
    const double drho = rin - 1.0 - st->drho_out;
    if (threadIdx.x < mlp::N_IN) {
        const int i = threadIdx.x;
        float v;
        if (i < 15) {
            v = c.geometry[i];
        } else if (i < 31) {
            const double e = (qbar(np - CTRL_LAGS[i - 15]) - qs) / qn;
            v = (float)fmin(2.0, fmax(-2.0, e));
        } else {
            const double lg = drho > 0.0 ? log10(drho / c.drho_ref) / 3.0 : -1.0;
            v = isfinite(lg) ? (float)fmin(1.0, fmax(-1.0, lg)) : -1.0f;
        }
        x[i] = v;
    }
    __syncthreads();
    const float y = mlp::forward_one(c.params, x, h1, h2);
    const int64_t n = st->ctrl_steps;  // decisions taken before this one
    float *rec = c.trace + (size_t)(n % c.hist_cap) * CTRL_REC;
    if (threadIdx.x < mlp::N_IN) rec[threadIdx.x] = x[threadIdx.x];
    if (threadIdx.x == 0) {
        const double e = fabs(qbar(np - 1) - qs) / qn;
        if (np >= 2 && e <= c.release_tol) st->ctrl_released = 1u;
        // progress judge: the error must fall by 10 % within stall_decisions decisions
        if (n == 0 || e < 0.9 * st->ctrl_best) {
            // two 8-byte stores (a merged 16-byte store is avoided, see
            // store_pair in colour.h)
            st->ctrl_best = e;
            __asm__ __volatile__("" ::: "memory");
            st->ctrl_best_n = n;
        } else if (c.stall_decisions > 0 && n - st->ctrl_best_n >= c.stall_decisions) {
            st->ctrl_released = 1u;
        }
        const double bound =
            c.trust_decisions > 0 ? c.trust0 * fmax(0.0, 1.0 - (double)n / (double)c.trust_decisions) : 0.0;
        const double limit = bound * c.rho0 * qn / c.a_in;
        const double rho_plain = 1.0 + inlet_drho_plain(st, c.rd_next, c.rho0, (int64_t)c.a_in);
        const double r = c.relative ? fmin(3.0, fmax(-2.0, (double)y)) : fmin(4.0, fmax(-4.0, (double)y));
        const double rho_hat = 1.0 + st->drho_out + (c.relative ? drho : c.drho_ref) * exp(r - c.margin);
        // a non-finite output is dropped before clipping (fmin/fmax would
        // turn a NaN into a bound)
        const bool on = isfinite(y) && isfinite(rho_hat) && qs > 0.0 && !st->ctrl_released &&
                        !(c.relative && !(drho > 0.0)) && limit > 0.0;
        double delta = 0.0;
        if (on) delta = fmin(limit, fmax(-limit, c.gain * (rho_hat - rho_plain)));
        // 8-byte stores, kept apart (as above)
        st->ctrl_rho = on ? rho_hat : 0.0;
        __asm__ __volatile__("" ::: "memory");
        st->ctrl_limit = on ? limit : 0.0;
        __asm__ __volatile__("" ::: "memory");
        st->ctrl_gain = c.gain;
        st->ctrl_on = on ? 1u : 0u;
        st->ctrl_delta = delta;
        __asm__ __volatile__("" ::: "memory");
        st->ctrl_steps = n + 1;
        volatile double *aux = (double *)(rec + 32);
        aux[0] = drho;
        aux[1] = rho_plain;
        aux[2] = (double)y;
        aux[3] = delta;
    }
}

void launch_controller(flbm_ctx *c, hipStream_t s, int rd_next)
{
    CtrlArgs a{};
    a.st = c->st;
    a.hist = c->hist;
    a.ring = c->ctrl_ring;
    a.trace = c->ctrl_trace;
    a.hist_cap = HIST_CAP;
    a.trust_decisions = c->ctrl.trust_decisions;
    a.rd_next = rd_next;
    a.relative = c->ctrl.relative;
    a.stall_decisions = c->ctrl.stall_decisions;
    a.period = c->ctrl.period;
    a.params = c->ctrl_net->params;
    a.geometry = c->ctrl_feat;
    a.rho0 = c->p.rho0;
    a.a_in = (double)c->lat.a_in;
    a.drho_ref = c->ctrl.drho_ref;
    a.gain = c->ctrl.gain;
    a.trust0 = c->ctrl.trust0;
    a.release_tol = c->ctrl.release_tol;
    a.margin = c->ctrl.margin;
    hipLaunchKernelGGL(k_controller, dim3(1), dim3(256), 0, s, a);
}

// One step of a run; last: the run's last step (it records the watchdog's
// observables and ends in a launch of its own). Inside a run the next step
// kernel ends each single-fluid step (step_begin), which saves a launch per
// step; the controller reads every step's outlet flux from its end, so with
// it each step ends in its own launch, as in the colour model.
void launch_step_any(flbm_ctx *c, hipStream_t s, int from, bool last)
{
    launch_step_plain(c, s, from, last, last || c->ctrl_on);
    if (c->ctrl_on) {
        Range r(c->markers, "flbm controller");
        launch_controller(c, s, from ^ 1);
    }
}

void drop_graphs(flbm_ctx *c)
{
    for (int i = 0; i < 2; ++i)
        if (c->graph[i]) {
            (void)hipGraphExecDestroy(c->graph[i]);
            c->graph[i] = nullptr;
        }
}

flbm_status capture_graph(flbm_ctx *c, int parity)
{
    if (!c->cap_stream) HIPCHK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    HIPCHK(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    for (int i = 0; i < c->chunk; ++i) launch_step_any(c, c->cap_stream, parity ^ (i & 1), i == c->chunk - 1);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
    if (e != hipSuccess) return fail(c, FLBM_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&c->graph[parity], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        c->graph[parity] = nullptr;
        return fail(c, FLBM_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e));
    }
    return FLBM_OK;
}

// The step kernel carries the inlet consistency sum from one step to the
// next; when the state was set from the host, recompute it from the state.
flbm_status refresh_inlet_sum(flbm_ctx *c)
{
    if (!c->need_plane || c->p.z_mode != FLBM_Z_FLUX) return FLBM_OK;
    with_storage(c, [&](auto tag) {
        using T = decltype(tag);
        hipLaunchKernelGGL(k_inlet_plane<T>, dim3(c->plane_blocks), dim3(BLOCK), 0, c->stream,
                           (const T *)c->f[c->cur], c->nbr, plane_args(c, c->cur));
    });
    HIPCHK(c, hipGetLastError());
    c->need_plane = false;
    return FLBM_OK;
}

flbm_status reset_state(flbm_ctx *c)
{
    DevState h{};
    h.q_target = c->p.q_target;
    h.drho_out = c->p.rho_out - 1.0;
    h.omega = c->collide ? 1.0 / c->p.tau : 0.0;
    h.step = 0;
    HIPCHK(c, hipMemcpyAsync(c->st, &h, sizeof(h), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemsetAsync(c->hist, 0xff, (size_t)HIST_CAP * HIST_STRIDE * sizeof(double), c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->steps = 0;
    c->need_plane = true;
    return FLBM_OK;
}

template <typename T>
void launch_fill(flbm_ctx *c, int which, const Dev19 &dev)
{
    const int64_t total = 19 * c->lat.n_pad + SENT_PAD;
    const int blocks = (int)std::min<int64_t>((total + BLOCK - 1) / BLOCK, 65536);
    hipLaunchKernelGGL(k_fill<T>, dim3(blocks), dim3(BLOCK), 0, c->stream, (T *)c->f[which],
                       c->lat.n, c->lat.n_pad, total, dev);
}

flbm_status fill_equilibrium(flbm_ctx *c, double rho, double ux, double uy, double uz)
{
    Dev19 dev{};
    const double uu = ux * ux + uy * uy + uz * uz;
    for (int q = 0; q < 19; ++q) {
        const double cu = d3q19::cx[q] * ux + d3q19::cy[q] * uy + d3q19::cz[q] * uz;
        dev.v[q] = d3q19::weight(q) * ((rho - 1.0) + c->p.rho0 * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu));
    }
    Dev19 zero{};
    for (int w = 0; w < 2; ++w)
        with_storage(c, [&](auto tag) { launch_fill<decltype(tag)>(c, w, w == c->cur ? dev : zero); });
    HIPCHK(c, hipGetLastError());
    return reset_state(c);
}

flbm_status setup_device(flbm_ctx *c, void *mem)
{
    c->dmem = mem;
    carve(c, (char *)mem);
    HIPCHK(c, hipMemcpyAsync(c->nbr, c->lat.nbr.data(), c->lat.nbr.size() * sizeof(int32_t),
                             hipMemcpyHostToDevice, c->stream));
    if (c->pull.tiles) {
        flbm_status rc = upload_pull(c);
        if (rc) return rc;
    }
    if (!c->lat.kcoef.empty())
        HIPCHK(c, hipMemcpyAsync(c->kcoef, c->lat.kcoef.data(), c->lat.kcoef.size() * sizeof(uint64_t),
                                 hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemsetAsync(c->kpart, 0, PLANE_MAX_BLOCKS * sizeof(double), c->stream));
    if (c->colour) {
        for (int i = 0; i < 2; ++i)
            HIPCHK(c, hipMemsetAsync(c->cab[i], 0, (size_t)14 * c->lat.n_pad * colour_elem(c), c->stream));
        HIPCHK(c, hipMemsetAsync(c->nab, 0, (size_t)2 * c->lat.n_pad * colour_elem(c), c->stream));
        HIPCHK(c, hipMemsetAsync(c->phi, 0, (size_t)c->lat.n_pad * colour_elem(c), c->stream));
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->ready = true;
    c->cur = 0;
    return fill_equilibrium(c, c->p.rho_out, 0.0, 0.0, 0.0);
}

flbm_status ensure_device(flbm_ctx *c)
{
    HIPCHK(c, hipSetDevice(c->device));
    if (c->ready) return FLBM_OK;
    void *mem = nullptr;
    hipError_t e = hipMalloc(&mem, c->dbytes);
    if (e != hipSuccess) return fail(c, FLBM_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    c->owned = true;
    return setup_device(c, mem);
}

flbm_status check_params(const flbm_params *p, std::string &why)
{
    if (p->nx < 1 || p->ny < 1 || p->nz < 3) return why = "dimensions must be nx, ny >= 1, nz >= 3", FLBM_EINVAL;
    if (p->reservoir_layers < 0 || 2 * p->reservoir_layers > p->nz)
        return why = "reservoir layers exceed the box", FLBM_EINVAL;
    if (!(p->tau > 0.5)) return why = "tau must exceed 1/2", FLBM_EINVAL;
    if (!(p->rho0 > 0.0)) return why = "rho0 must be positive", FLBM_EINVAL;
    if (p->z_mode < FLBM_Z_FLUX || p->z_mode > FLBM_Z_WALL) return why = "unknown z_mode", FLBM_EINVAL;
    if (p->precision != FLBM_FP64 && p->precision != FLBM_FP32 && p->precision != FLBM_FP16DEV)
        return why = "unknown precision", FLBM_EINVAL;
    if (p->model != FLBM_BGK && p->model != FLBM_COLOUR && p->model != FLBM_MRT)
        return why = "unknown model", FLBM_EINVAL;
    if (p->model == FLBM_COLOUR && (!std::isfinite(p->alpha) || !std::isfinite(p->beta) ||
                                    !std::isfinite(p->phi_solid)))
        return why = "colour parameters must be finite", FLBM_EINVAL;
    if (p->watchdog_every < 0) return why = "watchdog_every must be >= 0", FLBM_EINVAL;
    if (!std::isfinite(p->q_target) || !std::isfinite(p->rho_out) || !(p->rho_out > 0.0))
        return why = "q_target and rho_out must be finite, rho_out positive", FLBM_EINVAL;
    return FLBM_OK;
}

}  // namespace

extern "C" {

flbm_status flbm_default_params(flbm_params *p)
{
    if (!p) return FLBM_EINVAL;
    std::memset(p, 0, sizeof(*p));
    p->periodic_x = 1;
    p->periodic_y = 1;
    p->z_mode = FLBM_Z_FLUX;
    p->precision = FLBM_FP32;
    p->model = FLBM_BGK;
    p->watchdog_every = 1000;
    p->tau = 0.8;
    p->rho0 = 1.0;
    p->q_target = 0.0;
    p->rho_out = 1.0;
    p->alpha = 0.005;
    p->beta = 0.7;
    p->phi_solid = 0.0;
    p->umax_limit = 0.1;
    return FLBM_OK;
}

flbm_status flbm_create(const uint8_t *solid_mask, const flbm_params *p, void *hip_stream, flbm_ctx **out)
{
    if (!solid_mask || !p || !out) return FLBM_EINVAL;
    *out = nullptr;
    std::string why;
    flbm_status rc = check_params(p, why);
    if (rc != FLBM_OK) return rc;
    flbm_ctx *c = new (std::nothrow) flbm_ctx();
    if (!c) return FLBM_ENOMEM;
    c->p = *p;
    if (!(c->p.umax_limit > 0.0)) c->p.umax_limit = 0.1;
    c->spec.nx = p->nx;
    c->spec.ny = p->ny;
    c->spec.nz = p->nz;
    c->spec.periodic_x = p->periodic_x != 0;
    c->spec.periodic_y = p->periodic_y != 0;
    c->spec.z_mode = p->z_mode;
    c->spec.reservoir_layers = p->reservoir_layers;
    c->stream = (hipStream_t)hip_stream;
    c->elem = p->precision == FLBM_FP64 ? 8 : (p->precision == FLBM_FP16DEV ? 2 : 4);
    c->colour = p->model == FLBM_COLOUR;
    int code = FLBM_OK;
    std::string e = build_lattice(solid_mask, c->spec, c->lat, code);
    if (!e.empty()) {
        delete c;
        return code;
    }
    e = check_pull_bijection(c->lat, c->spec);
    if (!e.empty()) {
        delete c;
        return FLBM_EINVAL;
    }
    c->tiles = (int)(c->lat.n_pad / TILE);
    c->use_buf = f_bytes(c) < (1ull << 32) && (uint64_t)18 * c->lat.n_pad * 4 < (1ull << 32);
    // testing aid: FLBM_NO_BUF=1 takes the 64-bit addressing path (that of
    // lattices past 4 GiB) for a context of any size
    const char *nobuf = std::getenv("FLBM_NO_BUF");
    if (nobuf && nobuf[0] == '1') c->use_buf = false;
    if (c->use_buf) {
        // the step (and both passes of the colour step) reads the compact pull
        // table where it fits
        e = build_compact_pull(c->lat, TILE, (int32_t)PULL_MAX_CODE, (int32_t)PULL_MAX_BYTE, c->pull);
        if (!e.empty()) {
            delete c;
            return FLBM_ENOMEM;
        }
        e = check_compact_pull(c->lat, c->pull);
        if (!e.empty()) {
            delete c;
            return FLBM_EINVAL;
        }
        c->pull_format = FLBM_PULL_RUN;
    }
    c->blocks256 = (int)(c->lat.n_pad / BLOCK);
    c->obs_slots = std::max(c->tiles, c->blocks256);
    const bool flux = p->z_mode == FLBM_Z_FLUX;
    c->nt_in = flux ? (int)((c->lat.a_in + TILE - 1) / TILE) : 0;
    c->nt01 = flux ? (int)((c->lat.n01 + TILE - 1) / TILE) : 0;
    c->tout0 = flux ? (int)((c->lat.n - c->lat.a_out) / TILE) : c->tiles;
    c->plane_blocks = flux ? (int)std::min<int64_t>((c->lat.a_in + BLOCK - 1) / BLOCK, PLANE_MAX_BLOCKS) : 0;
    const int w = p->watchdog_every > 0 ? std::min(p->watchdog_every, 256) : 256;
    c->chunk = std::max(2, w + (w & 1));
    const char *ng = std::getenv("FLBM_NO_GRAPH");
    c->use_graph = !(ng && ng[0] == '1');
    // FLBM_PROFILE=1: a roctx range around every kernel launch of a step,
    // which therefore launches directly instead of replaying graphs
    const char *pf = std::getenv("FLBM_PROFILE");
    c->markers = pf && pf[0] == '1';
    if (c->markers) c->use_graph = false;
    c->dbytes = carve(c, nullptr);
    // No usable device is not an error yet: the host-side lattice queries
    // work without one, and the first device call reports the HIP error.
    if (hipGetDevice(&c->device) != hipSuccess) c->device = 0;
    *out = c;
    return FLBM_OK;
}

flbm_status flbm_destroy(flbm_ctx *c)
{
    if (!c) return FLBM_EINVAL;
    (void)hipSetDevice(c->device);
    if (c->ready) (void)hipStreamSynchronize(c->stream);
    drop_graphs(c);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->owned && c->dmem) (void)hipFree(c->dmem);
    delete c;
    return FLBM_OK;
}

flbm_status flbm_device_bytes(const flbm_ctx *c, size_t *bytes)
{
    if (!c || !bytes) return FLBM_EINVAL;
    *bytes = c->dbytes;
    return FLBM_OK;
}

flbm_status flbm_bind_device_memory(flbm_ctx *c, void *dev_ptr, size_t bytes)
{
    if (!c || !dev_ptr) return FLBM_EINVAL;
    if (c->ready) return fail(c, FLBM_ESTATE, "device memory already in use");
    if (((uintptr_t)dev_ptr & 255) != 0) return fail(c, FLBM_EINVAL, "device memory must be 256-byte aligned");
    if (bytes < c->dbytes) return fail(c, FLBM_EBOUND, "device buffer smaller than flbm_device_bytes");
    HIPCHK(c, hipSetDevice(c->device));
    c->owned = false;
    return setup_device(c, dev_ptr);
}

flbm_status flbm_num_sites(const flbm_ctx *c, int64_t *n_sites, int64_t *a_in, int64_t *a_out)
{
    if (!c) return FLBM_EINVAL;
    if (n_sites) *n_sites = c->lat.n;
    if (a_in) *a_in = c->lat.a_in;
    if (a_out) *a_out = c->lat.a_out;
    return FLBM_OK;
}

flbm_status flbm_get_site_coords(const flbm_ctx *c, int32_t *xyz)
{
    if (!c || !xyz) return FLBM_EINVAL;
    std::memcpy(xyz, c->lat.coords.data(), c->lat.coords.size() * sizeof(int32_t));
    return FLBM_OK;
}

flbm_status flbm_set_controller(flbm_ctx *c, const flbm_mlp *net, const flbm_controller_params *p)
{
    if (!c) return FLBM_EINVAL;
    if (net && !p) return FLBM_EINVAL;
    if (c->p.z_mode != FLBM_Z_FLUX && net) return fail(c, FLBM_ESTATE, "the controller needs the flux inlet");
    flbm_status rc = ensure_device(c);
    if (rc) return rc;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    drop_graphs(c);
    if (net) {
        if (!(p->trust0 >= 0.0) || !std::isfinite(p->gain) || p->trust_decisions < 0 || !(p->release_tol >= 0.0) ||
            !(p->drho_ref > 0.0) || !std::isfinite(p->drho_ref) || p->stall_decisions < 0 ||
            (p->relative != 0 && p->relative != 1) || p->period < 1 || !(p->margin >= 0.0f) ||
            !std::isfinite(p->margin))
            return fail(c, FLBM_EINVAL, "bad controller parameters");
        c->ctrl = *p;
        c->ctrl_net = net;
        float g[16] = {0};
        std::memcpy(g, p->geometry, sizeof(p->geometry));
        HIPCHK(c, hipMemcpy(c->ctrl_feat, g, sizeof(g), hipMemcpyHostToDevice));
    }
    c->ctrl_on = net != nullptr;
    // fresh controller state: no offset, not released, no decisions taken
    const double zero = 0.0;
    const int64_t z64 = 0;
    const uint32_t z32 = 0;
    HIPCHK(c, hipMemcpy(&c->st->ctrl_delta, &zero, sizeof(zero), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(&c->st->ctrl_steps, &z64, sizeof(z64), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(&c->st->ctrl_released, &z32, sizeof(z32), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(&c->st->ctrl_best, &zero, sizeof(zero), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(&c->st->ctrl_best_n, &z64, sizeof(z64), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(&c->st->ctrl_on, &z32, sizeof(z32), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(&c->st->ctrl_acc, &zero, sizeof(zero), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(&c->st->ctrl_periods, &z64, sizeof(z64), hipMemcpyHostToDevice));
    return FLBM_OK;
}

flbm_status flbm_set_inlet_density_override(flbm_ctx *c, const double *rho_in_or_null, double trust)
{
    if (!c) return FLBM_EINVAL;
    if (rho_in_or_null && (!std::isfinite(*rho_in_or_null) || !(trust >= 0.0) || !std::isfinite(trust)))
        return FLBM_EINVAL;
    if (c->p.z_mode != FLBM_Z_FLUX && rho_in_or_null) return fail(c, FLBM_ESTATE, "the override needs the flux inlet");
    flbm_status rc = ensure_device(c);
    if (rc) return rc;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const uint32_t on = rho_in_or_null ? 1u : 0u;
    const double rho = rho_in_or_null ? *rho_in_or_null : 0.0;
    const double limit = trust * c->p.rho0 * std::fabs(c->p.q_target) / (double)c->lat.a_in;
    HIPCHK(c, hipMemcpy(&c->st->ovr_rho, &rho, sizeof(rho), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(&c->st->ovr_limit, &limit, sizeof(limit), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(&c->st->ovr_on, &on, sizeof(on), hipMemcpyHostToDevice));
    return FLBM_OK;
}

flbm_status flbm_controller_state(flbm_ctx *c, int32_t *active, int32_t *released, double *delta, int64_t *decisions)
{
    if (!c) return FLBM_EINVAL;
    if (active) *active = c->ctrl_on ? 1 : 0;
    if (!c->ready) {
        if (released) *released = 0;
        if (delta) *delta = 0.0;
        if (decisions) *decisions = 0;
        return FLBM_OK;
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    DevState d{};
    HIPCHK(c, hipMemcpy(&d, c->st, sizeof(d), hipMemcpyDeviceToHost));
    if (released) *released = (int32_t)d.ctrl_released;
    if (delta) *delta = d.ctrl_delta;
    if (decisions) *decisions = d.ctrl_steps;
    return FLBM_OK;
}

flbm_status flbm_controller_trace(flbm_ctx *c, int32_t n, float *x, double *aux)
{
    if (!c || n < 0 || (n > 0 && (!x || !aux))) return FLBM_EINVAL;
    if (n == 0) return FLBM_OK;
    if (!c->ready || n > HIST_CAP) return fail(c, FLBM_EBOUND, "more records than the ring holds");
    HIPCHK(c, hipStreamSynchronize(c->stream));
    DevState d{};
    HIPCHK(c, hipMemcpy(&d, c->st, sizeof(d), hipMemcpyDeviceToHost));
    if (n > d.ctrl_steps) return fail(c, FLBM_EBOUND, "fewer decisions taken than requested");
    std::vector<float> rec((size_t)HIST_CAP * CTRL_REC);
    HIPCHK(c, hipMemcpy(rec.data(), c->ctrl_trace, rec.size() * sizeof(float), hipMemcpyDeviceToHost));
    for (int32_t i = 0; i < n; ++i) {
        const int64_t k = d.ctrl_steps - n + i;  // decision number
        const float *r = rec.data() + (size_t)(k % HIST_CAP) * CTRL_REC;
        std::memcpy(x + (size_t)i * 32, r, 32 * sizeof(float));
        std::memcpy(aux + (size_t)i * 4, r + 32, 4 * sizeof(double));
    }
    return FLBM_OK;
}

flbm_status flbm_get_pull_table(const flbm_ctx *c, int32_t *nbr)
{
    if (!c || !nbr) return FLBM_EINVAL;
    const int64_t n = c->lat.n, npad = c->lat.n_pad;
    for (int q = 0; q < 18; ++q)
        std::memcpy(nbr + q * n, c->lat.nbr.data() + q * npad, n * sizeof(int32_t));
    return FLBM_OK;
}

flbm_status flbm_set_pull_format(flbm_ctx *c, int32_t format, int32_t limit16, int32_t limit8)
{
    if (!c) return FLBM_EINVAL;
    if (format != FLBM_PULL_INT32 && format != FLBM_PULL_HALF && format != FLBM_PULL_COMPACT &&
        format != FLBM_PULL_RUN)
        return fail(c, FLBM_EINVAL, "unknown pull format");
    if (limit16 < 0 || (uint32_t)limit16 > PULL_MAX_CODE || limit8 < 0 || (uint32_t)limit8 > PULL_MAX_BYTE)
        return fail(c, FLBM_EINVAL, "code limit out of range");
    if (format != FLBM_PULL_INT32 && !c->pull.tiles)
        return fail(c, FLBM_ESTATE, "no compact pull table (a lattice past the 4 GiB buffer path)");
    const int32_t l16 = limit16 ? limit16 : (int32_t)PULL_MAX_CODE;
    const bool bytes_on = format == FLBM_PULL_COMPACT || format == FLBM_PULL_RUN;
    const int32_t l8 = bytes_on ? (limit8 ? limit8 : (int32_t)PULL_MAX_BYTE) : 0;
    if (c->ready) {
        HIPCHK(c, hipSetDevice(c->device));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    drop_graphs(c);
    if (format != FLBM_PULL_INT32 && (l16 != c->pull.limit16 || l8 != c->pull.limit8)) {
        std::string e = build_compact_pull(c->lat, TILE, l16, l8, c->pull);
        if (!e.empty()) return fail(c, FLBM_ENOMEM, e);
        e = check_compact_pull(c->lat, c->pull);
        if (!e.empty()) return fail(c, FLBM_EINVAL, e);
        if (c->ready) {
            flbm_status rc = upload_pull(c);
            if (rc) return rc;
            HIPCHK(c, hipStreamSynchronize(c->stream));
        }
    }
    c->pull_format = format;
    return FLBM_OK;
}

flbm_status flbm_pull_format_info(const flbm_ctx *c, int32_t *format, int64_t *tiles8, int64_t *tiles16,
                                  int64_t *tiles)
{
    if (!c) return FLBM_EINVAL;
    const bool on = c->pull_format != FLBM_PULL_INT32 && c->pull.tiles > 0;
    if (format) *format = on ? c->pull_format : FLBM_PULL_INT32;
    if (tiles8) *tiles8 = on ? c->pull.tiles8 : 0;
    if (tiles16) *tiles16 = on ? c->pull.tiles16 : 0;
    if (tiles) *tiles = c->tiles;
    return FLBM_OK;
}

flbm_status flbm_pull_run_info(const flbm_ctx *c, int64_t *tiles_run, int64_t *waves_wide)
{
    if (!c) return FLBM_EINVAL;
    if (tiles_run) *tiles_run = c->pull.tiles ? c->pull.tiles_run : 0;
    if (waves_wide) *waves_wide = c->pull.tiles ? c->pull.waves_wide : 0;
    return FLBM_OK;
}

flbm_status flbm_get_pull_runs(const flbm_ctx *c, uint32_t *runs, uint32_t *runs_hi)
{
    if (!c) return FLBM_EINVAL;
    if (!c->pull.tiles) return fail(const_cast<flbm_ctx *>(c), FLBM_ESTATE, "no compact pull table");
    if (runs) std::memcpy(runs, c->pull.runs.data(), c->pull.runs.size() * sizeof(uint32_t));
    if (runs_hi) std::memcpy(runs_hi, c->pull.runs_hi.data(), c->pull.runs_hi.size() * sizeof(uint32_t));
    return FLBM_OK;
}

flbm_status flbm_get_compact_pull(const flbm_ctx *c, uint32_t *codes16, uint32_t *codes8, uint16_t *codes8_tail,
                                  int32_t *hdr)
{
    if (!c) return FLBM_EINVAL;
    if (!c->pull.tiles) return fail(const_cast<flbm_ctx *>(c), FLBM_ESTATE, "no compact pull table");
    if (codes16) std::memcpy(codes16, c->pull.codes.data(), c->pull.codes.size() * sizeof(uint32_t));
    if (codes8) std::memcpy(codes8, c->pull.bytes.data(), c->pull.bytes.size() * sizeof(uint32_t));
    if (codes8_tail) std::memcpy(codes8_tail, c->pull.tail.data(), c->pull.tail.size() * sizeof(uint16_t));
    if (hdr) std::memcpy(hdr, c->pull.hdr.data(), c->pull.hdr.size() * sizeof(int32_t));
    return FLBM_OK;
}

// Distributions in a checkpoint: f, then the colour pairs (A_q, B_q) for the
// colour model.
static size_t state_f_bytes(const flbm_ctx *c)
{
    return (size_t)19 * c->lat.n_pad * c->elem + (c->colour ? (size_t)14 * c->lat.n_pad * colour_elem(c) : 0);
}

flbm_status flbm_state_bytes(const flbm_ctx *c, size_t *bytes)
{
    if (!c || !bytes) return FLBM_EINVAL;
    *bytes = state_f_bytes(c) + 3 * sizeof(int64_t);
    return FLBM_OK;
}

// Checkpoint trailer after the distributions: step count, a flag telling
// whether the carried inlet sum is valid, and that sum.
struct StateTrailer {
    int64_t steps;
    int64_t carry_valid;
    double s_carry;
};

flbm_status flbm_save_state(flbm_ctx *c, void *host, size_t bytes)
{
    if (!c || !host) return FLBM_EINVAL;
    const size_t fb = state_f_bytes(c), f19 = (size_t)19 * c->lat.n_pad * c->elem;
    if (bytes < fb + sizeof(StateTrailer)) return fail(c, FLBM_EBOUND, "host buffer too small");
    flbm_status rc = ensure_device(c);
    if (rc) return rc;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(host, c->f[c->cur], f19, hipMemcpyDeviceToHost));
    if (c->colour) {
        const size_t c14 = (size_t)14 * c->lat.n_pad * colour_elem(c);
        HIPCHK(c, hipMemcpy((char *)host + f19, c->cab[c->cur], c14, hipMemcpyDeviceToHost));
    }
    DevState d{};
    HIPCHK(c, hipMemcpy(&d, c->st, sizeof(d), hipMemcpyDeviceToHost));
    StateTrailer tr{c->steps, c->need_plane ? 0 : 1, d.s_carry[c->cur]};
    std::memcpy((char *)host + fb, &tr, sizeof(tr));
    return FLBM_OK;
}

flbm_status flbm_load_state(flbm_ctx *c, const void *host, size_t bytes)
{
    if (!c || !host) return FLBM_EINVAL;
    const size_t fb = state_f_bytes(c), f19 = (size_t)19 * c->lat.n_pad * c->elem;
    if (bytes < fb + sizeof(StateTrailer)) return fail(c, FLBM_EBOUND, "host buffer too small");
    flbm_status rc = ensure_device(c);
    if (rc) return rc;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(c->f[c->cur], host, f19, hipMemcpyHostToDevice));
    if (c->colour) {
        const size_t c14 = (size_t)14 * c->lat.n_pad * colour_elem(c);
        HIPCHK(c, hipMemcpy(c->cab[c->cur], (const char *)host + f19, c14, hipMemcpyHostToDevice));
    }
    rc = reset_state(c);
    if (rc) return rc;
    StateTrailer tr{};
    std::memcpy(&tr, (const char *)host + fb, sizeof(tr));
    // Restore the step counter on both sides so history slots line up, and
    // the carried inlet sum so the resumed run is bitwise the same.
    c->steps = tr.steps;
    HIPCHK(c, hipMemcpy(&c->st->step, &tr.steps, sizeof(int64_t), hipMemcpyHostToDevice));
    if (tr.carry_valid) {
        HIPCHK(c, hipMemcpy(&c->st->s_carry[c->cur], &tr.s_carry, sizeof(double), hipMemcpyHostToDevice));
        c->need_plane = false;
    }
    return FLBM_OK;
}

// Host [7][n] FP64 colour distributions A and B <-> device pairs (A_q, B_q)
// [7][n_pad] in the colour storage type.
extern "C++" {
template <typename C>
static flbm_status write_colour_pairs_t(flbm_ctx *c, void *dst, const double *A, const double *B)
{
    const int64_t n = c->lat.n, npad = c->lat.n_pad;
    std::vector<C> h((size_t)14 * npad, (C)0);
    for (int q = 0; q < 7; ++q)
        for (int64_t s = 0; s < n; ++s) {
            h[2 * (q * npad + s)] = (C)A[q * n + s];
            h[2 * (q * npad + s) + 1] = (C)B[q * n + s];
        }
    HIPCHK(c, hipMemcpy(dst, h.data(), h.size() * sizeof(C), hipMemcpyHostToDevice));
    return FLBM_OK;
}

template <typename C>
static flbm_status read_colour_pairs_t(flbm_ctx *c, const void *src, double *A, double *B)
{
    const int64_t n = c->lat.n, npad = c->lat.n_pad;
    std::vector<C> h((size_t)14 * npad);
    HIPCHK(c, hipMemcpy(h.data(), src, h.size() * sizeof(C), hipMemcpyDeviceToHost));
    for (int q = 0; q < 7; ++q)
        for (int64_t s = 0; s < n; ++s) {
            A[q * n + s] = (double)h[2 * (q * npad + s)];
            B[q * n + s] = (double)h[2 * (q * npad + s) + 1];
        }
    return FLBM_OK;
}
}  // extern "C++"

static flbm_status write_colour_pairs(flbm_ctx *c, void *dst, const double *A, const double *B)
{
    return is_fp64(c) ? write_colour_pairs_t<double>(c, dst, A, B) : write_colour_pairs_t<float>(c, dst, A, B);
}

static flbm_status read_colour_pairs(flbm_ctx *c, const void *src, double *A, double *B)
{
    return is_fp64(c) ? read_colour_pairs_t<double>(c, src, A, B) : read_colour_pairs_t<float>(c, src, A, B);
}

flbm_status flbm_init_colour(flbm_ctx *c, const double *na, const double *nb)
{
    if (!c || !na || !nb) return FLBM_EINVAL;
    if (!c->colour) return fail(c, FLBM_ESTATE, "not a colour-model context");
    flbm_status rc = ensure_device(c);
    if (rc) return rc;
    rc = fill_equilibrium(c, 1.0, 0.0, 0.0, 0.0);
    if (rc) return rc;
    const int64_t n = c->lat.n;
    std::vector<double> a((size_t)7 * n), b((size_t)7 * n);
    for (int q = 0; q < 7; ++q)
        for (int64_t s = 0; s < n; ++s) {
            a[q * n + s] = d3q19::weight7(q) * na[s];
            b[q * n + s] = d3q19::weight7(q) * nb[s];
        }
    return write_colour_pairs(c, c->cab[c->cur], a.data(), b.data());
}

flbm_status flbm_read_colour(flbm_ctx *c, double *A, double *B)
{
    if (!c || !A || !B) return FLBM_EINVAL;
    if (!c->colour) return fail(c, FLBM_ESTATE, "not a colour-model context");
    flbm_status rc = ensure_device(c);
    if (rc) return rc;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return read_colour_pairs(c, c->cab[c->cur], A, B);
}

flbm_status flbm_write_colour(flbm_ctx *c, const double *A, const double *B)
{
    if (!c || !A || !B) return FLBM_EINVAL;
    if (!c->colour) return fail(c, FLBM_ESTATE, "not a colour-model context");
    flbm_status rc = ensure_device(c);
    if (rc) return rc;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    rc = write_colour_pairs(c, c->cab[c->cur], A, B);
    if (rc) return rc;
    return reset_state(c);
}

flbm_status flbm_read_phase(flbm_ctx *c, double *phi)
{
    if (!c || !phi) return FLBM_EINVAL;
    if (!c->colour) return fail(c, FLBM_ESTATE, "not a colour-model context");
    flbm_status rc = ensure_device(c);
    if (rc) return rc;
    if (is_fp64(c))
        hipLaunchKernelGGL(k_phase_of_state<double>, dim3(c->blocks256), dim3(BLOCK), 0, c->stream,
                           (const Pair<double>::type *)c->cab[c->cur], c->lat.n, c->lat.n_pad, c->fields);
    else
        hipLaunchKernelGGL(k_phase_of_state<float>, dim3(c->blocks256), dim3(BLOCK), 0, c->stream,
                           (const Pair<float>::type *)c->cab[c->cur], c->lat.n, c->lat.n_pad, c->fields);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(c->stream));
    HIPCHK(c, hipMemcpy(phi, c->fields, c->lat.n * sizeof(double), hipMemcpyDeviceToHost));
    return FLBM_OK;
}

flbm_status flbm_init_equilibrium(flbm_ctx *c, double rho, double ux, double uy, double uz)
{
    if (!c) return FLBM_EINVAL;
    flbm_status rc = ensure_device(c);
    if (rc) return rc;
    return fill_equilibrium(c, rho, ux, uy, uz);
}

flbm_status flbm_set_target_flux(flbm_ctx *c, double q_target)
{
    if (!c || !std::isfinite(q_target)) return FLBM_EINVAL;
    c->p.q_target = q_target;
    if (!c->ready) return FLBM_OK;
    HIPCHK(c, hipSetDevice(c->device));
    hipLaunchKernelGGL(k_set_f64, dim3(1), dim3(1), 0, c->stream, &c->st->q_target, q_target);
    HIPCHK(c, hipGetLastError());
    return FLBM_OK;
}

flbm_status flbm_set_outlet_density(flbm_ctx *c, double rho_out)
{
    if (!c || !std::isfinite(rho_out) || !(rho_out > 0.0)) return FLBM_EINVAL;
    c->p.rho_out = rho_out;
    if (!c->ready) return FLBM_OK;
    HIPCHK(c, hipSetDevice(c->device));
    hipLaunchKernelGGL(k_set_f64, dim3(1), dim3(1), 0, c->stream, &c->st->drho_out, rho_out - 1.0);
    HIPCHK(c, hipGetLastError());
    return FLBM_OK;
}

flbm_status flbm_debug_set_collision(flbm_ctx *c, int32_t enabled)
{
    if (!c) return FLBM_EINVAL;
    c->collide = enabled ? 1 : 0;
    if (!c->ready) return FLBM_OK;
    HIPCHK(c, hipSetDevice(c->device));
    hipLaunchKernelGGL(k_set_f64, dim3(1), dim3(1), 0, c->stream, &c->st->omega,
                       c->collide ? 1.0 / c->p.tau : 0.0);
    HIPCHK(c, hipGetLastError());
    return FLBM_OK;
}

flbm_status flbm_step(flbm_ctx *c, int32_t n)
{
    if (!c || n < 0) return FLBM_EINVAL;
    Range r(c->markers, "flbm_step");
    flbm_status rc = ensure_device(c);
    if (rc) return rc;
    if (n > 0) {
        rc = refresh_inlet_sum(c);
        if (rc) return rc;
    }
    int32_t left = n;
    while (left > 0) {
        if (c->use_graph && left >= c->chunk) {
            if (!c->graph[c->cur]) {
                rc = capture_graph(c, c->cur);
                if (rc) return rc;
            }
            HIPCHK(c, hipGraphLaunch(c->graph[c->cur], c->stream));
            left -= c->chunk;
            c->steps += c->chunk;
        } else {
            const int k = std::min(left, c->chunk);
            for (int i = 0; i < k; ++i) {
                launch_step_any(c, c->stream, c->cur, i == k - 1);
                c->cur ^= 1;
            }
            HIPCHK(c, hipGetLastError());
            left -= k;
            c->steps += k;
        }
    }
    return FLBM_OK;
}

flbm_status flbm_sync(flbm_ctx *c)
{
    if (!c) return FLBM_EINVAL;
    if (!c->ready) return FLBM_OK;
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    uint32_t unstable = 0;
    HIPCHK(c, hipMemcpy(&unstable, &c->st->unstable, sizeof(unstable), hipMemcpyDeviceToHost));
    if (unstable) return fail(c, FLBM_EUNSTABLE, "watchdog: non-finite value or |u| above the limit");
    return FLBM_OK;
}

flbm_status flbm_history_capacity(const flbm_ctx *c, int32_t *cap)
{
    if (!c || !cap) return FLBM_EINVAL;
    *cap = HIST_CAP;
    return FLBM_OK;
}

flbm_status flbm_step_count(const flbm_ctx *c, int64_t *steps)
{
    if (!c || !steps) return FLBM_EINVAL;
    *steps = c->steps;
    return FLBM_OK;
}

flbm_status flbm_get_history(flbm_ctx *c, double *buf, int32_t n)
{
    if (!c || !buf || n < 0 || n > HIST_CAP || n > c->steps) return FLBM_EINVAL;
    if (n == 0) return FLBM_OK;
    flbm_status rc = ensure_device(c);
    if (rc) return rc;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    std::vector<double> h((size_t)HIST_CAP * HIST_STRIDE);
    HIPCHK(c, hipMemcpy(h.data(), c->hist, h.size() * sizeof(double), hipMemcpyDeviceToHost));
    for (int32_t i = 0; i < n; ++i) {
        const int64_t t = c->steps - n + i;  // 0-based step index
        const double *r = &h[(size_t)(t % HIST_CAP) * HIST_STRIDE];
        for (int k = 0; k < 5; ++k) buf[7 * (size_t)i + k] = r[k];
        buf[7 * (size_t)i + 5] = r[6];
        buf[7 * (size_t)i + 6] = r[7];
    }
    return FLBM_OK;
}

flbm_status flbm_get_boundary(flbm_ctx *c, double *q_in, double *q_out, double *rho_in, double *rho_out)
{
    if (!c) return FLBM_EINVAL;
    if (rho_out) *rho_out = c->p.rho_out;
    if (c->steps == 0) {
        if (q_in) *q_in = NAN;
        if (q_out) *q_out = NAN;
        if (rho_in) *rho_in = NAN;
        return FLBM_OK;
    }
    double r[7];
    flbm_status rc = flbm_get_history(c, r, 1);
    if (rc) return rc;
    if (rho_in) *rho_in = r[0];
    if (q_in) *q_in = r[1];
    if (q_out) *q_out = r[2];
    return FLBM_OK;
}

flbm_status flbm_read_fields(flbm_ctx *c, double *rho, double *ux, double *uy, double *uz)
{
    if (!c) return FLBM_EINVAL;
    flbm_status rc = ensure_device(c);
    if (rc) return rc;
    const int64_t n = c->lat.n, npad = c->lat.n_pad;
    with_storage(c, [&](auto tag) {
        using T = decltype(tag);
        hipLaunchKernelGGL(k_moments<T>, dim3(c->blocks256), dim3(BLOCK), 0, c->stream,
                           (const T *)c->f[c->cur], n, npad, 1.0 / c->p.rho0, c->fields);
    });
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(c->stream));
    double *dst[4] = {rho, ux, uy, uz};
    for (int k = 0; k < 4; ++k)
        if (dst[k]) HIPCHK(c, hipMemcpy(dst[k], c->fields + k * npad, n * sizeof(double), hipMemcpyDeviceToHost));
    return FLBM_OK;
}

flbm_status flbm_read_distributions(flbm_ctx *c, double *f)
{
    if (!c || !f) return FLBM_EINVAL;
    flbm_status rc = ensure_device(c);
    if (rc) return rc;
    const int64_t n = c->lat.n, npad = c->lat.n_pad;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    hipError_t e = hipSuccess;
    with_storage(c, [&](auto tag) {
        using T = decltype(tag);
        std::vector<T> h((size_t)19 * npad);
        e = hipMemcpy(h.data(), c->f[c->cur], h.size() * sizeof(T), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return;
        for (int q = 0; q < 19; ++q)
            for (int64_t s = 0; s < n; ++s) f[q * n + s] = d3q19::weight(q) + host_dec<T>(h[q * npad + s], q);
    });
    HIPCHK(c, e);
    return FLBM_OK;
}

flbm_status flbm_write_distributions(flbm_ctx *c, const double *f)
{
    if (!c || !f) return FLBM_EINVAL;
    flbm_status rc = ensure_device(c);
    if (rc) return rc;
    const int64_t n = c->lat.n, npad = c->lat.n_pad;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    hipError_t e = hipSuccess;
    with_storage(c, [&](auto tag) {
        using T = decltype(tag);
        std::vector<T> h((size_t)19 * npad, (T)0);
        for (int q = 0; q < 19; ++q)
            for (int64_t s = 0; s < n; ++s) h[q * npad + s] = host_enc<T>(f[q * n + s] - d3q19::weight(q), q);
        e = hipMemcpy(c->f[c->cur], h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice);
    });
    HIPCHK(c, e);
    return reset_state(c);
}

flbm_status flbm_get_observables(flbm_ctx *c, double *mass, double *umax, int32_t *nonfinite)
{
    if (!c) return FLBM_EINVAL;
    flbm_status rc = ensure_device(c);
    if (rc) return rc;
    with_storage(c, [&](auto tag) {
        using T = decltype(tag);
        hipLaunchKernelGGL(k_state_observables<T>, dim3(c->blocks256), dim3(BLOCK), 0, c->stream,
                           (const T *)c->f[c->cur], c->lat.n_pad, 1.0 / c->p.rho0, c->obs_mass,
                           c->obs_umax2, c->obs_bad);
    });
    hipLaunchKernelGGL(k_obs_finalize, dim3(1), dim3(OBS_BLOCK), 0, c->stream, obs_args(c, 0, c->blocks256));
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(c->stream));
    DevState h{};
    HIPCHK(c, hipMemcpy(&h, c->st, sizeof(h), hipMemcpyDeviceToHost));
    if (mass) *mass = h.obs_mass;
    if (umax) *umax = h.obs_umax;
    if (nonfinite) *nonfinite = (int32_t)h.obs_bad;
    return FLBM_OK;
}

flbm_status flbm_device_layout(const flbm_ctx *c, void **f_cur, void **nbr, int64_t *n_pad)
{
    if (!c) return FLBM_EINVAL;
    if (f_cur) *f_cur = c->ready ? c->f[c->cur] : nullptr;
    if (nbr) *nbr = c->ready ? (void *)c->nbr : nullptr;
    if (n_pad) *n_pad = c->lat.n_pad;
    return FLBM_OK;
}

flbm_status flbm_profile_kernels(flbm_ctx *c, int32_t n, double *ms_plane, double *ms_step)
{
    if (!c || n < 1) return FLBM_EINVAL;
    flbm_status rc = ensure_device(c);
    if (rc) return rc;
    hipEvent_t ev[2];
    for (auto &e : ev) HIPCHK(c, hipEventCreate(&e));
    double tp = 0.0, ts = 0.0;
    float ms = 0.f;
    if (c->p.z_mode == FLBM_Z_FLUX) {
        c->need_plane = true;
        HIPCHK(c, hipEventRecord(ev[0], c->stream));
        rc = refresh_inlet_sum(c);
        if (rc) return rc;
        HIPCHK(c, hipEventRecord(ev[1], c->stream));
        HIPCHK(c, hipEventSynchronize(ev[1]));
        HIPCHK(c, hipEventElapsedTime(&ms, ev[0], ev[1]));
        tp = ms;
    }
    for (int32_t i = 0; i < n; ++i) {
        const int from = c->cur;
        HIPCHK(c, hipEventRecord(ev[0], c->stream));
        if (c->colour) {
            // both launches of a colour step (phase pass and colour step)
            with_storage(c, [&](auto tag) { launch_colour_step<decltype(tag)>(c, c->stream, from, false); });
        } else {
            with_storage(c, [&](auto tag) {
                using T = decltype(tag);
                launch_stream_collide<T>(c, c->stream, (const T *)c->f[from], (T *)c->f[from ^ 1], false);
            });
        }
        HIPCHK(c, hipEventRecord(ev[1], c->stream));
        launch_finalize(c, c->stream, from);  // outside the timed step kernel
        HIPCHK(c, hipGetLastError());
        HIPCHK(c, hipEventSynchronize(ev[1]));
        HIPCHK(c, hipEventElapsedTime(&ms, ev[0], ev[1]));
        ts += ms;
        c->cur ^= 1;
        c->steps += 1;
    }
    for (auto &e : ev) (void)hipEventDestroy(e);
    if (ms_plane) *ms_plane = tp;
    if (ms_step) *ms_step = ts / n;
    return FLBM_OK;
}

flbm_status flbm_copy_kernel(const void *src, void *dst, size_t bytes, void *hip_stream)
{
    if (!src || !dst || (bytes & 15) != 0) return FLBM_EINVAL;
    if ((((uintptr_t)src) & 15) || (((uintptr_t)dst) & 15)) return FLBM_EINVAL;
    const int64_t n16 = (int64_t)(bytes / 16);
    if (n16 == 0) return FLBM_OK;
    const int64_t blocks = (n16 + BLOCK - 1) / BLOCK;
    if (blocks > INT32_MAX) return FLBM_EINVAL;
    hipLaunchKernelGGL(k_copy16, dim3((unsigned)blocks), dim3(BLOCK), 0, (hipStream_t)hip_stream,
                       (const u32x4 *)src, (u32x4 *)dst, n16);
    return hipGetLastError() == hipSuccess ? FLBM_OK : FLBM_EHIP;
}

const char *flbm_status_string(flbm_status s)
{
    switch (s) {
    case FLBM_OK: return "ok";
    case FLBM_EINVAL: return "invalid argument";
    case FLBM_ENOINLET: return "no pore site on the inlet plane";
    case FLBM_ENOMEM: return "out of memory";
    case FLBM_EHIP: return "HIP runtime error";
    case FLBM_EUNSTABLE: return "watchdog: unstable state";
    case FLBM_EINDEX: return "lattice too large for 32-bit indices";
    case FLBM_EBOUND: return "device buffer too small";
    case FLBM_ESTATE: return "call not valid in the current state";
    case FLBM_ESCRATCH: return "input larger than the allocation-free scratch holds (67,108,864 padded sites)";
    default: return "unknown status";
    }
}

const char *flbm_last_error(const flbm_ctx *c) { return c ? c->err.c_str() : ""; }

}  // extern "C"

// ======================================================================
// Batched stepping of many lattices (samples of uneven size, each with its
// own target flux, outlet density and state) by one launch per step (and a
// finalize launch with one block per sample).

struct flbm_batch {
    std::vector<flbm_ctx *> s;
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;
    int device = 0;
    bool use_buf = false;
    int precision = 0, model = 0;
    bool tile8_ok = false;  // the 64-VGPR tile kernel of this batch runs without scratch
    flbm_schedule sched{};
    BatchSample *d_tab = nullptr;
    BatchItem *d_work = nullptr;
    int n_work = 0, work_cap = 0;
    std::vector<BatchSample> tab_host;   // last uploaded table
    hipGraphExec_t graph = nullptr;
    std::string err;
};

namespace {

flbm_status bfail(flbm_batch *b, flbm_status s, const std::string &msg)
{
    b->err = msg;
    return s;
}

#define BHIPCHK(b, expr)                                                                        \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return bfail((b), FLBM_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));    \
    } while (0)

void batch_drop_graph(flbm_batch *b)
{
    if (b->graph) {
        (void)hipGraphExecDestroy(b->graph);
        b->graph = nullptr;
    }
}

// Work list in the schedule's order.
flbm_status batch_build_work(flbm_batch *b)
{
    const int tpi = std::max(1, b->sched.tiles_per_item);
    const int ns = (int)b->s.size();
    std::vector<std::vector<BatchItem>> per(ns);
    for (int i = 0; i < ns; ++i)
        for (int t = 0; t < b->s[i]->tiles; t += tpi)
            per[i].push_back(BatchItem{i, t, std::min(t + tpi, b->s[i]->tiles), 0});
    std::vector<int> order(ns);
    for (int i = 0; i < ns; ++i) order[i] = i;
    if (b->sched.order == FLBM_ORDER_LARGEST)
        std::stable_sort(order.begin(), order.end(),
                         [&](int x, int y) { return b->s[x]->tiles > b->s[y]->tiles; });
    std::vector<BatchItem> work;
    if (b->sched.order == FLBM_ORDER_SAMPLE) {
        for (int i : order) work.insert(work.end(), per[i].begin(), per[i].end());
    } else {
        size_t longest = 0;
        for (auto &v : per) longest = std::max(longest, v.size());
        for (size_t k = 0; k < longest; ++k)
            for (int i : order)
                if (k < per[i].size()) work.push_back(per[i][k]);
    }
    if ((int)work.size() > b->work_cap) {
        if (b->d_work) (void)hipFree(b->d_work);
        b->d_work = nullptr;
        BHIPCHK(b, hipMalloc(&b->d_work, work.size() * sizeof(BatchItem)));
        b->work_cap = (int)work.size();
    }
    BHIPCHK(b, hipMemcpy(b->d_work, work.data(), work.size() * sizeof(BatchItem), hipMemcpyHostToDevice));
    b->n_work = (int)work.size();
    batch_drop_graph(b);
    return FLBM_OK;
}

// Per-sample table relative to each sample's current buffer; uploaded only
// when it changed (an odd number of steps flips every sample's buffers).
flbm_status batch_refresh(flbm_batch *b)
{
    std::vector<BatchSample> t(b->s.size());
    for (size_t i = 0; i < b->s.size(); ++i) {
        flbm_ctx *c = b->s[i];
        flbm_status rc = refresh_inlet_sum(c);
        if (rc) return bfail(b, rc, "sample " + std::to_string(i) + ": " + c->err);
        std::memset(&t[i], 0, sizeof(BatchSample));
        t[i].a = step_args(c);
        t[i].a.rd = c->cur;
        t[i].f0 = c->f[c->cur];
        t[i].f1 = c->f[c->cur ^ 1];
        t[i].nbr = c->nbr;
    }
    if (t.size() != b->tab_host.size() ||
        std::memcmp(t.data(), b->tab_host.data(), t.size() * sizeof(BatchSample)) != 0) {
        BHIPCHK(b, hipMemcpyAsync(b->d_tab, t.data(), t.size() * sizeof(BatchSample), hipMemcpyHostToDevice,
                                  b->stream));
        BHIPCHK(b, hipStreamSynchronize(b->stream));  // the host copy must outlive the transfer
        b->tab_host = std::move(t);
    }
    return FLBM_OK;
}

// Whether the 64-VGPR tile kernel (the step without observables) of this
// precision, model and address path fits its budget without scratch. Where
// it spills it is not used: besides the cost of scratch, register spills are
// 16-byte stores whose registers are reused at once, the order that has
// stored wrong values on gfx950 (see store_pair in colour.h).
template <typename T, bool MRT>
bool tile8_fits(bool use_buf)
{
    hipFuncAttributes fa{};
    const hipError_t e = use_buf ? hipFuncGetAttributes(&fa, (const void *)k_batch_tile8<T, false, true, MRT>)
                                 : hipFuncGetAttributes(&fa, (const void *)k_batch_tile8<T, false, false, MRT>);
    return e == hipSuccess && fa.localSizeBytes == 0;
}

bool batch_tile8_fits(const flbm_batch *b)
{
    const bool mrt = b->model == FLBM_MRT;
    if (b->precision == FLBM_FP64) return mrt ? tile8_fits<double, true>(b->use_buf) : tile8_fits<double, false>(b->use_buf);
    if (b->precision == FLBM_FP16DEV)
        return mrt ? tile8_fits<_Float16, true>(b->use_buf) : tile8_fits<_Float16, false>(b->use_buf);
    return mrt ? tile8_fits<float, true>(b->use_buf) : tile8_fits<float, false>(b->use_buf);
}

template <typename T, bool MRT>
void batch_launch_t(flbm_batch *b, hipStream_t s, int parity, bool obs)
{
    const int grid = b->sched.grid > 0 ? std::min(b->sched.grid, b->n_work) : b->n_work;
    if (b->sched.grid == 0 && b->sched.tiles_per_item == 1) {
        // one tile per block: the loop-free kernel, in the chosen register budget.
        // The observable step always takes the compiler's budget: squeezed to
        // 64 VGPRs it spills to scratch, and a scratch-using launch inside a
        // captured chunk costs far more than the step itself.
        const dim3 g(b->n_work), blk(SC_BLOCK);
        const bool o8 = b->sched.occupancy == 8 && !obs && b->tile8_ok;
#define FLBM_BATCH_TILE(OB, BU)                                                                           \
    do {                                                                                                  \
        if (o8)                                                                                           \
            hipLaunchKernelGGL((k_batch_tile8<T, OB, BU, MRT>), g, blk, 0, s, b->d_tab, b->d_work, parity); \
        else                                                                                              \
            hipLaunchKernelGGL((k_batch_tile<T, OB, BU, MRT>), g, blk, 0, s, b->d_tab, b->d_work, parity);  \
    } while (0)
        if (b->use_buf) {
            if (obs)
                FLBM_BATCH_TILE(true, true);
            else
                FLBM_BATCH_TILE(false, true);
        } else {
            if (obs)
                FLBM_BATCH_TILE(true, false);
            else
                FLBM_BATCH_TILE(false, false);
        }
#undef FLBM_BATCH_TILE
    } else if (b->use_buf) {
        if (obs)
            hipLaunchKernelGGL((k_batch_step<T, true, true, MRT>), dim3(grid), dim3(SC_BLOCK), 0, s, b->d_tab,
                               b->d_work, b->n_work, parity);
        else
            hipLaunchKernelGGL((k_batch_step<T, false, true, MRT>), dim3(grid), dim3(SC_BLOCK), 0, s, b->d_tab,
                               b->d_work, b->n_work, parity);
    } else {
        if (obs)
            hipLaunchKernelGGL((k_batch_step<T, true, false, MRT>), dim3(grid), dim3(SC_BLOCK), 0, s, b->d_tab,
                               b->d_work, b->n_work, parity);
        else
            hipLaunchKernelGGL((k_batch_step<T, false, false, MRT>), dim3(grid), dim3(SC_BLOCK), 0, s, b->d_tab,
                               b->d_work, b->n_work, parity);
    }
    hipLaunchKernelGGL(k_batch_finalize, dim3((unsigned)b->s.size()), dim3(FIN_BLOCK), 0, s, b->d_tab, parity);
    if (obs)
        for (flbm_ctx *c : b->s)
            hipLaunchKernelGGL(k_obs_finalize, dim3(1), dim3(OBS_BLOCK), 0, s, obs_args(c, 1, c->tiles));
}

void batch_launch(flbm_batch *b, hipStream_t s, int parity, bool obs)
{
    flbm_ctx *c0 = b->s[0];
    const bool mrt = b->model == FLBM_MRT;
    with_storage(c0, [&](auto tag) {
        using T = decltype(tag);
        if (mrt)
            batch_launch_t<T, true>(b, s, parity, obs);
        else
            batch_launch_t<T, false>(b, s, parity, obs);
    });
}

flbm_status batch_capture(flbm_batch *b)
{
    if (!b->cap_stream) BHIPCHK(b, hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
    BHIPCHK(b, hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
    for (int i = 0; i < b->sched.chunk; ++i) batch_launch(b, b->cap_stream, i & 1, i == b->sched.chunk - 1);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
    if (e != hipSuccess) return bfail(b, FLBM_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        b->graph = nullptr;
        return bfail(b, FLBM_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e));
    }
    return FLBM_OK;
}

void batch_advance(flbm_batch *b, int k)
{
    for (flbm_ctx *c : b->s) {
        c->steps += k;
        c->cur ^= (k & 1);
    }
}

flbm_status batch_check_schedule(const flbm_schedule *s)
{
    if (!s || s->grid < 0 || s->tiles_per_item < 1 || s->chunk < 1 || s->order < FLBM_ORDER_SAMPLE ||
        s->order > FLBM_ORDER_LARGEST || (s->occupancy != 0 && s->occupancy != 8))
        return FLBM_EINVAL;
    return FLBM_OK;
}

}  // namespace

extern "C" {

flbm_status flbm_batch_create(int32_t n, flbm_ctx *const *samples, flbm_batch **out)
{
    if (!out || n < 1 || !samples) return FLBM_EINVAL;
    *out = nullptr;
    for (int32_t i = 0; i < n; ++i)
        if (!samples[i]) return FLBM_EINVAL;
    flbm_ctx *c0 = samples[0];
    for (int32_t i = 0; i < n; ++i) {
        flbm_ctx *c = samples[i];
        if (ensure_device(c)) return FLBM_ENOMEM;
        if (c->stream != c0->stream || c->device != c0->device) return FLBM_EINVAL;
        if (c->p.precision != c0->p.precision || c->p.model != c0->p.model || c->use_buf != c0->use_buf)
            return FLBM_EINVAL;
        if (c->colour || c->ctrl_on) return FLBM_ESTATE;
        for (int32_t j = 0; j < i; ++j)
            if (samples[j] == c) return FLBM_EINVAL;
    }
    flbm_batch *b = new (std::nothrow) flbm_batch();
    if (!b) return FLBM_ENOMEM;
    b->s.assign(samples, samples + n);
    b->stream = c0->stream;
    b->device = c0->device;
    b->use_buf = c0->use_buf;
    b->precision = c0->p.precision;
    b->model = c0->p.model;
    b->sched = flbm_schedule{0, FLBM_ORDER_INTERLEAVE, 4, 64, 0};
    (void)hipSetDevice(b->device);
    b->tile8_ok = batch_tile8_fits(b);
    if (hipSetDevice(b->device) != hipSuccess || hipMalloc(&b->d_tab, n * sizeof(BatchSample)) != hipSuccess) {
        delete b;
        return FLBM_ENOMEM;
    }
    if (batch_build_work(b) != FLBM_OK) {
        (void)hipFree(b->d_tab);
        if (b->d_work) (void)hipFree(b->d_work);
        delete b;
        return FLBM_EHIP;
    }
    *out = b;
    return FLBM_OK;
}

flbm_status flbm_batch_destroy(flbm_batch *b)
{
    if (!b) return FLBM_EINVAL;
    (void)hipSetDevice(b->device);
    (void)hipStreamSynchronize(b->stream);
    batch_drop_graph(b);
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    if (b->d_tab) (void)hipFree(b->d_tab);
    if (b->d_work) (void)hipFree(b->d_work);
    delete b;
    return FLBM_OK;
}

flbm_status flbm_batch_set_schedule(flbm_batch *b, const flbm_schedule *s)
{
    if (!b || batch_check_schedule(s)) return FLBM_EINVAL;
    BHIPCHK(b, hipSetDevice(b->device));
    BHIPCHK(b, hipStreamSynchronize(b->stream));
    b->sched = *s;
    return batch_build_work(b);
}

flbm_status flbm_batch_get_schedule(const flbm_batch *b, flbm_schedule *s)
{
    if (!b || !s) return FLBM_EINVAL;
    *s = b->sched;
    return FLBM_OK;
}

flbm_status flbm_batch_step(flbm_batch *b, int32_t n)
{
    if (!b || n < 0) return FLBM_EINVAL;
    if (n == 0) return FLBM_OK;
    Range r(!b->s.empty() && b->s[0]->markers, "flbm_batch_step");
    BHIPCHK(b, hipSetDevice(b->device));
    flbm_status rc = batch_refresh(b);
    if (rc) return rc;
    int32_t left = n;
    int parity = 0;
    while (left > 0) {
        if (left >= b->sched.chunk && (b->sched.chunk & 1) == 0) {
            // a graph of an even number of steps starts and ends at parity 0
            if (!b->graph) {
                rc = batch_capture(b);
                if (rc) return rc;
            }
            BHIPCHK(b, hipGraphLaunch(b->graph, b->stream));
            left -= b->sched.chunk;
        } else {
            const int k = std::min(left, b->sched.chunk);
            for (int i = 0; i < k; ++i) batch_launch(b, b->stream, (parity + i) & 1, i == k - 1);
            BHIPCHK(b, hipGetLastError());
            parity = (parity + k) & 1;
            left -= k;
        }
    }
    batch_advance(b, n);
    return FLBM_OK;
}

flbm_status flbm_batch_sync(flbm_batch *b, int32_t *first_unstable)
{
    if (!b) return FLBM_EINVAL;
    if (first_unstable) *first_unstable = -1;
    BHIPCHK(b, hipSetDevice(b->device));
    BHIPCHK(b, hipStreamSynchronize(b->stream));
    for (size_t i = 0; i < b->s.size(); ++i) {
        uint32_t u = 0;
        BHIPCHK(b, hipMemcpy(&u, &b->s[i]->st->unstable, sizeof(u), hipMemcpyDeviceToHost));
        if (u) {
            if (first_unstable) *first_unstable = (int32_t)i;
            return bfail(b, FLBM_EUNSTABLE, "watchdog tripped in sample " + std::to_string(i));
        }
    }
    return FLBM_OK;
}

flbm_status flbm_batch_time(flbm_batch *b, int32_t n, double *ms_per_step)
{
    if (!b || n < 1 || !ms_per_step) return FLBM_EINVAL;
    BHIPCHK(b, hipSetDevice(b->device));
    flbm_status rc = batch_refresh(b);
    if (rc) return rc;
    hipEvent_t e0, e1;
    BHIPCHK(b, hipEventCreate(&e0));
    BHIPCHK(b, hipEventCreate(&e1));
    BHIPCHK(b, hipEventRecord(e0, b->stream));
    for (int i = 0; i < n; ++i) batch_launch(b, b->stream, i & 1, false);
    BHIPCHK(b, hipEventRecord(e1, b->stream));
    BHIPCHK(b, hipEventSynchronize(e1));
    float ms = 0.f;
    BHIPCHK(b, hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    batch_advance(b, n);
    *ms_per_step = (double)ms / n;
    return FLBM_OK;
}

flbm_status flbm_batch_autotune(flbm_batch *b, const char *cache_path, int32_t trial_steps, flbm_schedule *best,
                                double *best_ms)
{
    if (!b || trial_steps < 1) return FLBM_EINVAL;
    BHIPCHK(b, hipSetDevice(b->device));
    hipDeviceProp_t prop;
    BHIPCHK(b, hipGetDeviceProperties(&prop, b->device));
    std::string arch = prop.gcnArchName;
    const size_t colon = arch.find(':');
    if (colon != std::string::npos) arch = arch.substr(0, colon);
    int64_t sites = 0;
    for (flbm_ctx *c : b->s) sites += c->lat.n;
    int bucket = 0;
    while ((int64_t{1} << (bucket + 1)) <= sites) ++bucket;
    const int prec = b->precision;
    // the collision model and the pull-table formats in use change the
    // kernels, so they are part of the key: bit 0 int32 table, bit 1 16-bit
    // codes, bit 2 compact (8- and 16-bit) codes, bit 3 compact codes with
    // run codes
    const int model = b->s.empty() ? 0 : b->s[0]->p.model;
    int formats = 0;
    for (flbm_ctx *c : b->s) {
        const bool coded = c->use_buf && c->pull.tiles > 0 && c->pull_format != FLBM_PULL_INT32;
        formats |= !coded ? 1 : c->pull_format == FLBM_PULL_HALF ? 2 : c->pull_format == FLBM_PULL_COMPACT ? 4 : 8;
    }
    const int chunk = b->sched.chunk;
    // a cached choice for this architecture, precision, model, formats and
    // size bucket; lines of other layouts (no "v2" tag) never match
    if (cache_path) {
        FILE *fp = std::fopen(cache_path, "r");
        if (fp) {
            char line[256];
            while (std::fgets(line, sizeof(line), fp)) {
                char tag[8], a[64];
                int p, m, fm, bk, g, o, t, occ;
                double ms;
                if (std::sscanf(line, "%7s %63s %d %d %d %d %d %d %d %d %lf", tag, a, &p, &m, &fm, &bk, &g, &o, &t,
                                &occ, &ms) != 11 ||
                    std::strcmp(tag, "v2") != 0)
                    continue;
                if (arch == a && p == prec && m == model && fm == formats && bk == bucket) {
                    std::fclose(fp);
                    flbm_schedule s{g, o, t, chunk, occ};
                    flbm_status rc = flbm_batch_set_schedule(b, &s);
                    if (rc) return rc;
                    if (best) *best = s;
                    if (best_ms) *best_ms = ms;
                    return FLBM_OK;
                }
            }
            std::fclose(fp);
        }
    }
    const int cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    const int grids[] = {0, 2 * cus, 4 * cus, 8 * cus, 16 * cus};
    const int orders[] = {FLBM_ORDER_SAMPLE, FLBM_ORDER_INTERLEAVE, FLBM_ORDER_LARGEST};
    const int tpis[] = {1, 4, 16};
    flbm_schedule bs = b->sched;
    double bms = 1e300;
    for (int g : grids)
        for (int o : orders)
            for (int t : tpis)
                for (int occ : {0, 8}) {
                    if (occ == 8 && !(g == 0 && t == 1)) continue;  // a budget only the loop-free kernel has
                    if (occ == 8 && !b->tile8_ok) continue;         // that kernel spills here
                    flbm_schedule s{g, o, t, chunk, occ};
                    flbm_status rc = flbm_batch_set_schedule(b, &s);
                    if (rc) return rc;
                    double ms = 0.0;
                    rc = flbm_batch_time(b, 1, &ms);  // warm-up
                    if (rc) return rc;
                    rc = flbm_batch_time(b, trial_steps, &ms);
                    if (rc) return rc;
                    if (ms < bms) {
                        bms = ms;
                        bs = s;
                    }
                }
    flbm_status rc = flbm_batch_set_schedule(b, &bs);
    if (rc) return rc;
    if (cache_path) {
        FILE *fp = std::fopen(cache_path, "a");
        if (fp) {
            std::fprintf(fp, "v2 %s %d %d %d %d %d %d %d %d %.6f\n", arch.c_str(), prec, model, formats, bucket,
                         bs.grid, bs.order, bs.tiles_per_item, bs.occupancy, bms);
            std::fclose(fp);
        }
    }
    if (best) *best = bs;
    if (best_ms) *best_ms = bms;
    return FLBM_OK;
}

const char *flbm_batch_last_error(const flbm_batch *b) { return b ? b->err.c_str() : ""; }

}  // extern "C"

// ======================================================================
// Observables of a caller-held state without allocating: the two kernels of
// flbm_get_observables (per-block partials, then one block reducing them)
// with their partials and result record in a file-scope device array.

namespace {

constexpr int NOALLOC_MAX_BLOCKS = 1 << 18;  // partial slots: 256-site blocks, 67,108,864 sites
constexpr size_t NOALLOC_STATE_BYTES = (sizeof(DevState) + 255) / 256 * 256;
constexpr size_t NOALLOC_BYTES =
    NOALLOC_STATE_BYTES + (size_t)NOALLOC_MAX_BLOCKS * (sizeof(double) + sizeof(float) + sizeof(uint32_t));

// One copy per device, held until the process ends. Host code never uses
// this name as an address: the device address comes from
// hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// The device address of `scratch` on the current device (looked up on the
// first call there).
hipError_t scratch_address(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace

extern "C" {

flbm_status flbm_state_observables_noalloc(const void *f_dev, int32_t precision, int64_t n_sites, int64_t n_pad,
                                           double rho0, void *hip_stream, double *mass, double *umax,
                                           int32_t *nonfinite)
{
    if (!f_dev || n_sites < 0 || n_pad < 1 || n_sites > n_pad || n_pad % BLOCK != 0 || !(rho0 > 0.0) ||
        (precision != FLBM_FP64 && precision != FLBM_FP32 && precision != FLBM_FP16DEV))
        return FLBM_EINVAL;
    const int64_t blocks = n_pad / BLOCK;
    if (blocks > NOALLOC_MAX_BLOCKS) return FLBM_ESCRATCH;
    void *base = nullptr;
    if (scratch_address(&base) != hipSuccess) return FLBM_EHIP;
    hipStream_t s = (hipStream_t)hip_stream;
    char *sp = (char *)base;
    DevState *st = (DevState *)sp;
    double *pm = (double *)(sp + NOALLOC_STATE_BYTES);
    float *pu = (float *)(pm + NOALLOC_MAX_BLOCKS);
    uint32_t *pb = (uint32_t *)(pu + NOALLOC_MAX_BLOCKS);
    // every call writes the partials of all its blocks and the result fields
    // before reading them: nothing needs clearing
    const dim3 grid((unsigned)blocks), block(BLOCK);
    if (precision == FLBM_FP64)
        hipLaunchKernelGGL(k_state_observables<double>, grid, block, 0, s, (const double *)f_dev, n_pad, 1.0 / rho0,
                           pm, pu, pb);
    else if (precision == FLBM_FP32)
        hipLaunchKernelGGL(k_state_observables<float>, grid, block, 0, s, (const float *)f_dev, n_pad, 1.0 / rho0,
                           pm, pu, pb);
    else
        hipLaunchKernelGGL(k_state_observables<_Float16>, grid, block, 0, s, (const _Float16 *)f_dev, n_pad,
                           1.0 / rho0, pm, pu, pb);
    ObsArgs a{};
    a.n = n_sites;
    a.tiles = (int32_t)blocks;
    a.hist_cap = 1;
    a.umax_limit = 0.0;
    a.to_history = 0;
    a.raise_flag = 0;
    a.st = st;
    a.obs_mass = pm;
    a.obs_umax2 = pu;
    a.obs_bad = pb;
    hipLaunchKernelGGL(k_obs_finalize, dim3(1), dim3(OBS_BLOCK), 0, s, a);
    if (hipGetLastError() != hipSuccess) return FLBM_EHIP;
    double res[2];
    uint32_t bad = 0;
    if (hipMemcpyAsync(res, &st->obs_mass, 2 * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(&bad, &st->obs_bad, sizeof(uint32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return FLBM_EHIP;
    if (mass) *mass = res[0];
    if (umax) *umax = res[1];
    if (nonfinite) *nonfinite = (int32_t)bad;
    return FLBM_OK;
}

}  // extern "C"
