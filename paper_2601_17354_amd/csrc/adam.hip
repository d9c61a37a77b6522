// Adam on the canonical parameter layout: parameters, gradients and both
// moments share one [rows][n] layout that is never permuted, so the moments
// stay aligned with their parameters (PocketGS index-mapping subsection).
// One pass: reads p, g, m, v and writes p, m, v (28 B per element).
#include <math.h>

#include "common.hpp"

namespace {

struct LR {
    float v[64];
};

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v, int rows,
                                              int n, LR lr, float b1, float b2, float eps, float bc1,
                                              float bc2) {
    const size_t total = (size_t)rows * n;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
         i += (size_t)gridDim.x * blockDim.x) {
        const int row = (int)(i / (size_t)n);
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr.v[row] * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    }
}

// Step counter and bias corrections on the device, so that a captured
// graph advances the step on every replay: state[0] = step (uint32),
// state[1], state[2] = 1 - beta1^step, 1 - beta2^step (float32 bits).
__global__ void k_adam_advance(uint32_t* state, float b1, float b2) {
    if (threadIdx.x != 0) return;
    const uint32_t step = state[0] + 1u;
    state[0] = step;
    state[1] = __float_as_uint((float)(1.0 - pow((double)b1, (double)step)));
    state[2] = __float_as_uint((float)(1.0 - pow((double)b2, (double)step)));
}

__global__ __launch_bounds__(256) void k_adam_dev(float* __restrict__ p, const float* __restrict__ g,
                                                  float* __restrict__ m, float* __restrict__ v, int rows, int n,
                                                  LR lr, float b1, float b2, float eps,
                                                  const uint32_t* __restrict__ state) {
    const float bc1 = __uint_as_float(state[1]), bc2 = __uint_as_float(state[2]);
    const size_t total = (size_t)rows * n;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
         i += (size_t)gridDim.x * blockDim.x) {
        const int row = (int)(i / (size_t)n);
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr.v[row] * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    }
}

}  // namespace

extern "C" pgs_status pgs_adam_step_dev(float* params_dev, const float* grads_dev, float* m_dev, float* v_dev,
                                        int32_t rows, int32_t n, const float* lr_host, uint32_t* state_dev,
                                        float beta1, float beta2, float eps, void* stream) {
    PGS_REQUIRE(rows > 0 && rows <= 64 && n >= 0, "pgs_adam_step_dev: bad sizes");
    PGS_REQUIRE(lr_host != nullptr && state_dev != nullptr, "pgs_adam_step_dev: null pointer");
    PGS_REQUIRE(n == 0 || (params_dev && grads_dev && m_dev && v_dev), "pgs_adam_step_dev: null pointer");
    LR lr{};
    for (int r = 0; r < rows; ++r) lr.v[r] = lr_host[r];
    hipStream_t s = pgs::as_stream(stream);
    k_adam_advance<<<1, 64, 0, s>>>(state_dev, beta1, beta2);
    PGS_CHECK_LAUNCH("pgs_adam_step_dev advance");
    if (n == 0) return PGS_OK;
    const size_t total = (size_t)rows * n;
    size_t blocks = (total + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    k_adam_dev<<<(unsigned)blocks, 256, 0, s>>>(params_dev, grads_dev, m_dev, v_dev, rows, n, lr, beta1, beta2,
                                                eps, state_dev);
    PGS_CHECK_LAUNCH("pgs_adam_step_dev");
    return PGS_OK;
}

extern "C" pgs_status pgs_adam_step(float* params_dev, const float* grads_dev, float* m_dev, float* v_dev,
                                    int32_t rows, int32_t n, const float* lr_host, int32_t step,
                                    float beta1, float beta2, float eps, void* stream) {
    PGS_REQUIRE(rows > 0 && rows <= 64 && n >= 0 && step >= 1, "pgs_adam_step: bad sizes");
    PGS_REQUIRE(lr_host != nullptr, "pgs_adam_step: null learning rates");
    if (n == 0) return PGS_OK;
    PGS_REQUIRE(params_dev && grads_dev && m_dev && v_dev, "pgs_adam_step: null pointer");
    LR lr{};
    for (int r = 0; r < rows; ++r) lr.v[r] = lr_host[r];
    const float bc1 = (float)(1.0 - pow((double)beta1, step));
    const float bc2 = (float)(1.0 - pow((double)beta2, step));
    const size_t total = (size_t)rows * n;
    size_t blocks = (total + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    k_adam<<<(unsigned)blocks, 256, 0, pgs::as_stream(stream)>>>(params_dev, grads_dev, m_dev, v_dev, rows, n,
                                                                 lr, beta1, beta2, eps, bc1, bc2);
    PGS_CHECK_LAUNCH("pgs_adam_step");
    return PGS_OK;
}
