// Small multilayer perceptron on gfx950 matrix cores: 32 -> 128 -> 128 -> 1,
// tanh hidden activations, BF16 operands with FP32 accumulation
// (v_mfma_f32_16x16x16_bf16), FP32 master weights updated by Adam.
//
// It is the learned inlet controller's network: it predicts, from inlet-slice
// statistics and the recent outlet-flux error history, how far the inlet
// density still has to rise before the flow is steady.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace flbm {
namespace mlp {

constexpr int N_IN = 32;
constexpr int N_HID = 128;
// parameter layout (FP32): W1 [N_HID][N_IN], b1 [N_HID], W2 [N_HID][N_HID],
// b2 [N_HID], W3 [1][N_HID], b3 [1]
constexpr int OFF_W1 = 0;
constexpr int OFF_B1 = OFF_W1 + N_HID * N_IN;
constexpr int OFF_W2 = OFF_B1 + N_HID;
constexpr int OFF_B2 = OFF_W2 + N_HID * N_HID;
constexpr int OFF_W3 = OFF_B2 + N_HID;
constexpr int OFF_B3 = OFF_W3 + N_HID;
constexpr int N_PARAMS = OFF_B3 + 1;

typedef short v4i16 __attribute__((ext_vector_type(4)));
typedef float v4f32 __attribute__((ext_vector_type(4)));

// FP32 -> BF16 bits, round to nearest even (NaN kept quiet).
__host__ __device__ inline uint16_t bf16_bits(float x)
{
    uint32_t u = __builtin_bit_cast(uint32_t, x);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// Strided FP32 matrix view: element (r, c) at p[r * rs + c * cs]; rows x cols.
struct View {
    const float *p;
    int64_t rs, cs;
    int rows, cols;
    __device__ __forceinline__ float at(int r, int c) const
    {
        return (r < rows && c < cols) ? p[(int64_t)r * rs + (int64_t)c * cs] : 0.0f;
    }
};

// One wave computes the 16x16 tile (ti, tj) of A (M x K) times B (K x N),
// operands rounded to BF16, FP32 accumulation. Lane l holds, per the
// 16x16x16 BF16 MFMA layout, A rows l % 16 and B columns l % 16 with
// k = 4 (l / 16) + j, and returns D column l % 16, rows 4 (l / 16) + r.
__device__ __forceinline__ v4f32 wave_tile(const View &A, const View &B, int ti, int tj, int K)
{
    const int l = threadIdx.x & 63;
    const int row = ti * 16 + (l & 15), col = tj * 16 + (l & 15), kq = 4 * (l >> 4);
    v4f32 acc = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += 16) {
        v4i16 a, b;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            a[j] = (short)bf16_bits(A.at(row, k0 + kq + j));
            b[j] = (short)bf16_bits(B.at(k0 + kq + j, col));
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
    }
    return acc;
}

// Forward pass of one feature vector inside a single workgroup of 4 waves
// (the controller's inference), through the same MFMA tile routine as
// training: the batch is padded to 16 rows of which row 0 is the input.
// x and the hidden layers live in LDS. Returns y on every thread.
__device__ inline float forward_one(const float *params, const float *x_lds, float *h1_lds, float *h2_lds)
{
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const View X{x_lds, N_IN, 1, 1, N_IN};
    const View W1t{params + OFF_W1, 1, N_IN, N_IN, N_HID};
    for (int tj = w; tj < N_HID / 16; tj += 4) {
        const v4f32 d = wave_tile(X, W1t, 0, tj, N_IN);
        const int col = tj * 16 + (l & 15);
        if ((l >> 4) == 0) h1_lds[col] = tanhf(d[0] + params[OFF_B1 + col]);
    }
    __syncthreads();
    const View H1{h1_lds, N_HID, 1, 1, N_HID};
    const View W2t{params + OFF_W2, 1, N_HID, N_HID, N_HID};
    for (int tj = w; tj < N_HID / 16; tj += 4) {
        const v4f32 d = wave_tile(H1, W2t, 0, tj, N_HID);
        const int col = tj * 16 + (l & 15);
        if ((l >> 4) == 0) h2_lds[col] = tanhf(d[0] + params[OFF_B2 + col]);
    }
    __syncthreads();
    // output layer (N = 1): the first wave's tile, column 0
    __shared__ float y_lds;
    if (w == 0) {
        const View H2{h2_lds, N_HID, 1, 1, N_HID};
        const View W3t{params + OFF_W3, 1, 1, N_HID, 1};
        const v4f32 d = wave_tile(H2, W3t, 0, 0, N_HID);
        if (l == 0) y_lds = d[0] + params[OFF_B3];
    }
    __syncthreads();
    return y_lds;
}

}  // namespace mlp
}  // namespace flbm
