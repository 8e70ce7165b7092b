// Host-side state of a controller network (shared by the network's C-ABI and
// the step engine, which reads the device weights for inference).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

struct flbm_mlp {
    hipStream_t stream = nullptr;
    int max_batch = 0;
    void *mem = nullptr;
    size_t bytes = 0;
    float *params = nullptr, *grads = nullptr, *adam_m = nullptr, *adam_v = nullptr;
    float *h1 = nullptr, *h2 = nullptr, *dh = nullptr, *dz = nullptr, *y = nullptr, *dy = nullptr;
    float *loss = nullptr;
    int64_t adam_t = 0;
};
