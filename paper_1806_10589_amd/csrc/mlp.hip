// C-ABI of the controller network: create, set/get FP32 master weights,
// forward, gradients and Adam training steps on caller-owned device buffers.
#include <hip/hip_runtime.h>

#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/fluxlbm.h"
#include "mlp.h"
#include "mlp_ctx.h"

using namespace flbm;
using namespace flbm::mlp;

namespace {

struct GemmArgs {
    View A, B;          // A: M x K, B: K x N
    float *C;           // C[i * c_rs + j], M x N
    int64_t c_rs;
    const float *bias;  // per column, or null
    int act;            // 0: none, 1: tanh
    int M, N, K;
};

constexpr int GEMM_WAVES = 4;

// C = act(A B + bias); one 16x16 tile per wave.
__global__ __launch_bounds__(64 * GEMM_WAVES) void k_gemm(GemmArgs g)
{
    const int tiles_n = (g.N + 15) / 16;
    const int tiles = ((g.M + 15) / 16) * tiles_n;
    const int t = blockIdx.x * GEMM_WAVES + (threadIdx.x >> 6);
    if (t >= tiles) return;
    const int ti = t / tiles_n, tj = t % tiles_n;
    const v4f32 d = wave_tile(g.A, g.B, ti, tj, g.K);
    const int l = threadIdx.x & 63;
    const int col = tj * 16 + (l & 15);
    if (col >= g.N) return;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int row = ti * 16 + 4 * (l >> 4) + r;
        if (row >= g.M) continue;
        float v = d[r] + (g.bias ? g.bias[col] : 0.0f);
        if (g.act == 1) v = tanhf(v);
        g.C[(int64_t)row * g.c_rs + col] = v;
    }
}

// Mean squared error and its gradient 2 (y - t) / B; one block, fixed order.
__global__ __launch_bounds__(256) void k_mse(const float *y, const float *t, float *dy, int batch, float *loss)
{
    __shared__ float red[256];
    float s = 0.f;
    for (int i = threadIdx.x; i < batch; i += 256) {
        const float e = y[i] - t[i];
        dy[i] = 2.0f * e / (float)batch;
        s += e * e;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = red[0] / (float)batch;
}

// dz = dh (1 - h^2) (tanh backward), n elements.
__global__ __launch_bounds__(256) void k_tanh_back(const float *dh, const float *h, float *dz, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) dz[i] = dh[i] * (1.0f - h[i] * h[i]);
}

// db[j] = sum_i dz[i][j] (rows summed in order), one thread per column.
__global__ __launch_bounds__(256) void k_colsum(const float *dz, int rows, int cols, float *db)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= cols) return;
    float s = 0.f;
    for (int i = 0; i < rows; ++i) s += dz[(int64_t)i * cols + j];
    db[j] = s;
}

// Adam on FP32 master weights.
__global__ __launch_bounds__(256) void k_adam(float *p, const float *g, float *m, float *v, int n, float lr,
                                              float beta1, float beta2, float eps, float c1, float c2)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = beta1 * m[i] + (1.0f - beta1) * gi;
    const float vi = beta2 * v[i] + (1.0f - beta2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

inline size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

void launch_gemm(hipStream_t s, const View &A, const View &B, float *C, int64_t c_rs, const float *bias, int act,
                 int M, int N, int K)
{
    GemmArgs g{A, B, C, c_rs, bias, act, M, N, K};
    const int tiles = ((M + 15) / 16) * ((N + 15) / 16);
    const int blocks = (tiles + GEMM_WAVES - 1) / GEMM_WAVES;
    hipLaunchKernelGGL(k_gemm, dim3(blocks), dim3(64 * GEMM_WAVES), 0, s, g);
}

// Forward pass of a batch; keeps H1, H2, Y in the context's scratch.
void forward(flbm_mlp *m, const float *x, int B)
{
    const float *P = m->params;
    const View X{x, N_IN, 1, B, N_IN};
    launch_gemm(m->stream, X, View{P + OFF_W1, 1, N_IN, N_IN, N_HID}, m->h1, N_HID, P + OFF_B1, 1, B, N_HID, N_IN);
    launch_gemm(m->stream, View{m->h1, N_HID, 1, B, N_HID}, View{P + OFF_W2, 1, N_HID, N_HID, N_HID}, m->h2, N_HID,
                P + OFF_B2, 1, B, N_HID, N_HID);
    launch_gemm(m->stream, View{m->h2, N_HID, 1, B, N_HID}, View{P + OFF_W3, 1, 1, N_HID, 1}, m->y, 1, P + OFF_B3, 0,
                B, 1, N_HID);
}

// Backward pass of the mean squared error against t; gradients into m->grads.
void backward(flbm_mlp *m, const float *x, const float *t, int B)
{
    const float *P = m->params;
    float *G = m->grads;
    hipStream_t s = m->stream;
    hipLaunchKernelGGL(k_mse, dim3(1), dim3(256), 0, s, m->y, t, m->dy, B, m->loss);
    // layer 3: dW3 = dY^T H2, db3 = sum dY, dH2 = dY W3
    launch_gemm(s, View{m->dy, 0, 1, 1, B}, View{m->h2, N_HID, 1, B, N_HID}, G + OFF_W3, N_HID, nullptr, 0, 1, N_HID,
                B);
    hipLaunchKernelGGL(k_colsum, dim3(1), dim3(256), 0, s, m->dy, B, 1, G + OFF_B3);
    launch_gemm(s, View{m->dy, 1, 0, B, 1}, View{P + OFF_W3, 0, 1, 1, N_HID}, m->dh, N_HID, nullptr, 0, B, N_HID, 1);
    const int64_t nh = (int64_t)B * N_HID;
    const int eb = (int)((nh + 255) / 256);
    hipLaunchKernelGGL(k_tanh_back, dim3(eb), dim3(256), 0, s, m->dh, m->h2, m->dz, nh);
    // layer 2: dW2 = dZ2^T H1, db2 = colsum dZ2, dH1 = dZ2 W2
    launch_gemm(s, View{m->dz, 1, N_HID, N_HID, B}, View{m->h1, N_HID, 1, B, N_HID}, G + OFF_W2, N_HID, nullptr, 0,
                N_HID, N_HID, B);
    hipLaunchKernelGGL(k_colsum, dim3(1), dim3(256), 0, s, m->dz, B, N_HID, G + OFF_B2);
    launch_gemm(s, View{m->dz, N_HID, 1, B, N_HID}, View{P + OFF_W2, N_HID, 1, N_HID, N_HID}, m->dh, N_HID, nullptr,
                0, B, N_HID, N_HID);
    hipLaunchKernelGGL(k_tanh_back, dim3(eb), dim3(256), 0, s, m->dh, m->h1, m->dz, nh);
    // layer 1: dW1 = dZ1^T X, db1 = colsum dZ1
    launch_gemm(s, View{m->dz, 1, N_HID, N_HID, B}, View{x, N_IN, 1, B, N_IN}, G + OFF_W1, N_IN, nullptr, 0, N_HID,
                N_IN, B);
    hipLaunchKernelGGL(k_colsum, dim3(1), dim3(256), 0, s, m->dz, B, N_HID, G + OFF_B1);
}

flbm_status check(hipError_t e) { return e == hipSuccess ? FLBM_OK : FLBM_EHIP; }

}  // namespace

extern "C" {

flbm_status flbm_mlp_create(int32_t max_batch, void *hip_stream, flbm_mlp **out)
{
    if (!out || max_batch < 1) return FLBM_EINVAL;
    *out = nullptr;
    flbm_mlp *m = new (std::nothrow) flbm_mlp();
    if (!m) return FLBM_ENOMEM;
    m->stream = (hipStream_t)hip_stream;
    m->max_batch = max_batch;
    const size_t np = al(N_PARAMS * sizeof(float));
    const size_t bh = al((size_t)max_batch * N_HID * sizeof(float));
    const size_t b1 = al((size_t)max_batch * sizeof(float));
    m->bytes = 4 * np + 4 * bh + 2 * b1 + al(sizeof(float));
    if (hipMalloc(&m->mem, m->bytes) != hipSuccess) {
        delete m;
        return FLBM_ENOMEM;
    }
    char *p = (char *)m->mem;
    auto take = [&](size_t b) {
        char *r = p;
        p += b;
        return (float *)r;
    };
    m->params = take(np);
    m->grads = take(np);
    m->adam_m = take(np);
    m->adam_v = take(np);
    m->h1 = take(bh);
    m->h2 = take(bh);
    m->dh = take(bh);
    m->dz = take(bh);
    m->y = take(b1);
    m->dy = take(b1);
    m->loss = take(al(sizeof(float)));
    if (hipMemset(m->mem, 0, m->bytes) != hipSuccess) {
        (void)hipFree(m->mem);
        delete m;
        return FLBM_EHIP;
    }
    *out = m;
    return FLBM_OK;
}

flbm_status flbm_mlp_destroy(flbm_mlp *m)
{
    if (!m) return FLBM_EINVAL;
    (void)hipStreamSynchronize(m->stream);
    (void)hipFree(m->mem);
    delete m;
    return FLBM_OK;
}

flbm_status flbm_mlp_num_params(int32_t *n)
{
    if (!n) return FLBM_EINVAL;
    *n = N_PARAMS;
    return FLBM_OK;
}

flbm_status flbm_mlp_set_params(flbm_mlp *m, const float *host, int32_t n)
{
    if (!m || !host || n != N_PARAMS) return FLBM_EINVAL;
    flbm_status rc = check(hipStreamSynchronize(m->stream));
    if (rc) return rc;
    rc = check(hipMemcpy(m->params, host, N_PARAMS * sizeof(float), hipMemcpyHostToDevice));
    if (rc) return rc;
    rc = check(hipMemset(m->adam_m, 0, N_PARAMS * sizeof(float)));
    if (rc) return rc;
    rc = check(hipMemset(m->adam_v, 0, N_PARAMS * sizeof(float)));
    m->adam_t = 0;
    return rc;
}

flbm_status flbm_mlp_get_params(flbm_mlp *m, float *host, int32_t n)
{
    if (!m || !host || n != N_PARAMS) return FLBM_EINVAL;
    flbm_status rc = check(hipStreamSynchronize(m->stream));
    if (rc) return rc;
    return check(hipMemcpy(host, m->params, N_PARAMS * sizeof(float), hipMemcpyDeviceToHost));
}

flbm_status flbm_mlp_forward(flbm_mlp *m, const float *dev_x, float *dev_y, int32_t batch)
{
    if (!m || !dev_x || !dev_y || batch < 1 || batch > m->max_batch) return FLBM_EINVAL;
    forward(m, dev_x, batch);
    flbm_status rc = check(hipMemcpyAsync(dev_y, m->y, batch * sizeof(float), hipMemcpyDeviceToDevice, m->stream));
    if (rc) return rc;
    return check(hipGetLastError());
}

flbm_status flbm_mlp_gradients(flbm_mlp *m, const float *dev_x, const float *dev_t, int32_t batch, float *host_grads,
                               float *host_loss)
{
    if (!m || !dev_x || !dev_t || batch < 1 || batch > m->max_batch) return FLBM_EINVAL;
    forward(m, dev_x, batch);
    backward(m, dev_x, dev_t, batch);
    flbm_status rc = check(hipGetLastError());
    if (rc) return rc;
    rc = check(hipStreamSynchronize(m->stream));
    if (rc) return rc;
    if (host_grads) rc = check(hipMemcpy(host_grads, m->grads, N_PARAMS * sizeof(float), hipMemcpyDeviceToHost));
    if (rc) return rc;
    if (host_loss) rc = check(hipMemcpy(host_loss, m->loss, sizeof(float), hipMemcpyDeviceToHost));
    return rc;
}

flbm_status flbm_mlp_train_step(flbm_mlp *m, const float *dev_x, const float *dev_t, int32_t batch, float lr,
                                float *host_loss)
{
    if (!m || !dev_x || !dev_t || batch < 1 || batch > m->max_batch || !(lr > 0.0f)) return FLBM_EINVAL;
    forward(m, dev_x, batch);
    backward(m, dev_x, dev_t, batch);
    m->adam_t += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.0f - powf(b1, (float)m->adam_t), c2 = 1.0f - powf(b2, (float)m->adam_t);
    hipLaunchKernelGGL(k_adam, dim3((N_PARAMS + 255) / 256), dim3(256), 0, m->stream, m->params, m->grads, m->adam_m,
                       m->adam_v, N_PARAMS, lr, b1, b2, 1e-8f, c1, c2);
    flbm_status rc = check(hipGetLastError());
    if (rc || !host_loss) return rc;
    rc = check(hipStreamSynchronize(m->stream));
    if (rc) return rc;
    return check(hipMemcpy(host_loss, m->loss, sizeof(float), hipMemcpyDeviceToHost));
}

flbm_status flbm_gemm_bf16(const float *A, int64_t a_rs, int64_t a_cs, const float *B, int64_t b_rs, int64_t b_cs,
                           float *C, int64_t c_rs, int32_t M, int32_t N, int32_t K, void *hip_stream)
{
    if (!A || !B || !C || M < 1 || N < 1 || K < 1) return FLBM_EINVAL;
    launch_gemm((hipStream_t)hip_stream, View{A, a_rs, a_cs, M, K}, View{B, b_rs, b_cs, K, N}, C, c_rs, nullptr, 0, M,
                N, K);
    return check(hipGetLastError());
}

}  // extern "C"
