// Photometric loss L = (1 - lambda) L1 + lambda (1 - SSIM) and dL/dx.
//
// The paper does not state its loss; this is the 3D Gaussian Splatting form.
// SSIM (Wang et al. 2004): 11x11 Gaussian window (sigma 1.5), C1 = 1e-4,
// C2 = 9e-4, zero padding, mean over pixels and channels.
//
// Both SSIM kernels walk a strip of 64 output columns (one lane each) down
// 32 rows per workgroup of one wave.  Each input row (with a 5-column halo)
// is loaded once, prefetched one row ahead into registers, placed in LDS and
// blurred horizontally; the horizontal results of the last 11 rows sit in a
// register ring, from which the vertical pass forms the 11x11 window sums.
// Forward: mu_x, mu_y, E[x^2], E[y^2], E[xy] -> the SSIM map's partial
// derivatives m1 = dS/dmu_x, m2 = dS/dE[x^2], m3 = dS/dE[xy] and the strip's
// SSIM sum.  Backward: the same windowed pass over (m1, m2, m3) gives
//     dSSIM/dx_p = (1/N) (w*m1 + 2 x_p w*m2 + y_p w*m3)(p),
// the adjoint of the zero-padded blur being the zero-padded blur.
#include <math.h>

#include "common.hpp"

namespace {

constexpr int kHalo = 5;
constexpr int kSW = 64;                    // output columns per strip (one lane each)
constexpr int kRH = 32;                    // output rows per workgroup
constexpr int kRowW = kSW + 2 * kHalo;     // 74 input columns per row
constexpr float kC1 = 1e-4f, kC2 = 9e-4f;

struct Win {
    float w[11];
};

inline Win gaussian_window() {
    Win win;
    double g[11], s = 0;
    for (int i = 0; i < 11; ++i) {
        const double d = i - 5;
        g[i] = exp(-d * d / (2.0 * 1.5 * 1.5));
        s += g[i];
    }
    for (int i = 0; i < 11; ++i) win.w[i] = (float)(g[i] / s);
    return win;
}

__device__ __forceinline__ float block_sum(float v, float* red) {
    // wave sums to lane 63, then the 4 wave totals
    const float w = wave_sum_to_lane63(v);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 63) red[wv] = w;
    __syncthreads();
    float tot = 0.f;
    if (threadIdx.x == 0) tot = red[0] + red[1] + red[2] + red[3];
    __syncthreads();
    return tot;
}

__global__ __launch_bounds__(256) void k_l1(const float* __restrict__ x, const float* __restrict__ y,
                                            size_t N, float scale, float* __restrict__ dl,
                                            float* __restrict__ part) {
    __shared__ float red[4];
    float s = 0.f;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < N; i += (size_t)gridDim.x * blockDim.x) {
        const float d = x[i] - y[i];
        s += fabsf(d);
        dl[i] = d > 0.f ? scale : (d < 0.f ? -scale : 0.f);
    }
    const float tot = block_sum(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// Row ii of a strip (input row r0 - 5 + ii) of up to NQ planes, loaded by
// the 64 lanes: lane l takes columns l and (for l < 10) l + 64.
template <int NQ>
struct RowLoad {
    float v[NQ][2];
    __device__ __forceinline__ void load(const float* const* planes, int W, int H, int c0, int gy, int l) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int q = l + 64 * h, gx = c0 - kHalo + q;
            const bool in = q < kRowW && gy >= 0 && gy < H && gx >= 0 && gx < W;
#pragma unroll
            for (int f = 0; f < NQ; ++f) v[f][h] = in ? planes[f][(size_t)gy * W + gx] : 0.f;
        }
    }
    __device__ __forceinline__ void store(float (*lds)[kRowW + 2], int l) const {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int q = l + 64 * h;
            if (q < kRowW) {
#pragma unroll
                for (int f = 0; f < NQ; ++f) lds[f][q] = v[f][h];
            }
        }
    }
};

__global__ __launch_bounds__(64) void k_ssim_fwd(const float* __restrict__ x, const float* __restrict__ y,
                                                 int W, int H, Win win, float* __restrict__ m,
                                                 float* __restrict__ part) {
    __shared__ float rows[2][2][kRowW + 2];
    const int l = threadIdx.x, ch = blockIdx.z, c0 = blockIdx.x * kSW, r0 = blockIdx.y * kRH;
    const size_t plane = (size_t)W * H;
    const float* planes[2] = {x + ch * plane, y + ch * plane};
    const int col = c0 + l;
    const int rows_in = min(kRH, H - r0) + 2 * kHalo;
    float ring[11][5];
    float ssum = 0.f;
    RowLoad<2> next;
    next.load(planes, W, H, c0, r0 - kHalo, l);
    for (int base = 0; base < rows_in; base += 11) {
#pragma unroll
        for (int k = 0; k < 11; ++k) {
            const int ii = base + k;
            if (ii < rows_in) {
            const int buf = ii & 1;
            next.store(rows[buf], l);
            if (ii + 1 < rows_in) next.load(planes, W, H, c0, r0 - kHalo + ii + 1, l);
            __syncthreads();
            float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f, a4 = 0.f;
#pragma unroll
            for (int t = 0; t < 11; ++t) {
                const float w = win.w[t], xv = rows[buf][0][l + t], yv = rows[buf][1][l + t];
                a0 += w * xv;
                a1 += w * yv;
                a2 += w * xv * xv;
                a3 += w * yv * yv;
                a4 += w * xv * yv;
            }
            ring[k][0] = a0;
            ring[k][1] = a1;
            ring[k][2] = a2;
            ring[k][3] = a3;
            ring[k][4] = a4;
            if (ii >= 2 * kHalo) {
                const int o = r0 + ii - 2 * kHalo;   // output row
                float q[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int t = 0; t < 11; ++t)
#pragma unroll
                    for (int f = 0; f < 5; ++f) q[f] += win.w[t] * ring[(k + 1 + t) % 11][f];
                if (col < W && o < H) {
                    const float mx = q[0], my = q[1];
                    const float vx = q[2] - mx * mx, vy = q[3] - my * my, cxy = q[4] - mx * my;
                    const float N1 = 2.f * mx * my + kC1, N2 = 2.f * cxy + kC2;
                    const float D1 = mx * mx + my * my + kC1, D2 = vx + vy + kC2;
                    const float inv = 1.f / (D1 * D2);
                    const float S = N1 * N2 * inv;
                    const float m1 = (2.f * my * N2 - 2.f * my * N1) * inv - S * (2.f * mx / D1 - 2.f * mx / D2);
                    const float m2 = -S / D2;
                    const float m3 = 2.f * N1 * inv;
                    const size_t pix = (size_t)o * W + col;
                    m[(size_t)(3 * ch + 0) * plane + pix] = m1;
                    m[(size_t)(3 * ch + 1) * plane + pix] = m2;
                    m[(size_t)(3 * ch + 2) * plane + pix] = m3;
                    ssum += S;
                }
            }
            }
        }
    }
    const float tot = wave_sum_to_lane63(ssum);
    if (l == 63) part[(blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = tot;
}

__global__ __launch_bounds__(64) void k_ssim_bwd(const float* __restrict__ x, const float* __restrict__ y,
                                                 int W, int H, Win win, const float* __restrict__ m,
                                                 float l1_scale, float ssim_scale,
                                                 float* __restrict__ dl, float* __restrict__ part) {
    __shared__ float rows[2][3][kRowW + 2];
    const int l = threadIdx.x, ch = blockIdx.z, c0 = blockIdx.x * kSW, r0 = blockIdx.y * kRH;
    const size_t plane = (size_t)W * H;
    const float* planes[3] = {m + (size_t)(3 * ch) * plane, m + (size_t)(3 * ch + 1) * plane,
                              m + (size_t)(3 * ch + 2) * plane};
    const int col = c0 + l;
    const int rows_in = min(kRH, H - r0) + 2 * kHalo;
    float ring[11][3];
    float l1sum = 0.f;
    RowLoad<3> next;
    next.load(planes, W, H, c0, r0 - kHalo, l);
    for (int base = 0; base < rows_in; base += 11) {
#pragma unroll
        for (int k = 0; k < 11; ++k) {
            const int ii = base + k;
            if (ii < rows_in) {
            const int buf = ii & 1;
            next.store(rows[buf], l);
            if (ii + 1 < rows_in) next.load(planes, W, H, c0, r0 - kHalo + ii + 1, l);
            __syncthreads();
            float a[3] = {0.f, 0.f, 0.f};
#pragma unroll
            for (int t = 0; t < 11; ++t)
#pragma unroll
                for (int f = 0; f < 3; ++f) a[f] += win.w[t] * rows[buf][f][l + t];
#pragma unroll
            for (int f = 0; f < 3; ++f) ring[k][f] = a[f];
            if (ii >= 2 * kHalo) {
                const int o = r0 + ii - 2 * kHalo;
                float b[3] = {0.f, 0.f, 0.f};
#pragma unroll
                for (int t = 0; t < 11; ++t)
#pragma unroll
                    for (int f = 0; f < 3; ++f) b[f] += win.w[t] * ring[(k + 1 + t) % 11][f];
                if (col < W && o < H) {
                    const size_t i = ch * plane + (size_t)o * W + col;
                    const float xv = x[i], yv = y[i], d = xv - yv;
                    l1sum += fabsf(d);
                    const float sgn = d > 0.f ? 1.f : (d < 0.f ? -1.f : 0.f);
                    dl[i] = l1_scale * sgn - ssim_scale * (b[0] + 2.f * xv * b[1] + yv * b[2]);
                }
            }
            }
        }
    }
    const float tot = wave_sum_to_lane63(l1sum);
    if (l == 63) part[(blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = tot;
}

// Sums the per-block partials in a fixed order (deterministic, no atomics):
// 1024 lanes, eight independent accumulators each so the loads overlap.
constexpr int kFinalThreads = 1024;

__device__ __forceinline__ float strided_sum(const float* __restrict__ p, int n) {
    float acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int base = threadIdx.x; base < n; base += 8 * kFinalThreads) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = base + u * kFinalThreads;
            if (i < n) acc[u] += p[i];
        }
    }
    return ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
}

__device__ __forceinline__ float block_sum_1024(float v, float* red) {
    const float w = wave_sum_to_lane63(v);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 63) red[wv] = w;
    __syncthreads();
    float tot = 0.f;
    if (threadIdx.x == 0)
        for (int k = 0; k < kFinalThreads / 64; ++k) tot += red[k];
    __syncthreads();
    return tot;
}

__global__ __launch_bounds__(kFinalThreads) void k_loss_final(const float* __restrict__ part_l1, int nl,
                                                              const float* __restrict__ part_s, int ns,
                                                              float lambda, float invN,
                                                              float* __restrict__ out) {
    __shared__ float red[kFinalThreads / 64];
    const float l1 = block_sum_1024(strided_sum(part_l1, nl), red) * invN;
    const float ss = block_sum_1024(strided_sum(part_s, ns), red) * invN;
    if (threadIdx.x == 0) out[0] = lambda > 0.f ? (1.f - lambda) * l1 + lambda * (1.f - ss) : l1;
}

constexpr int kL1Blocks = 1024;

// Squared error of the two images clamped to [0, 1], per-block partials.
__global__ __launch_bounds__(256) void k_sq_err(const float* __restrict__ x, const float* __restrict__ y,
                                                size_t N, float* __restrict__ part) {
    __shared__ float red[4];
    float s = 0.f;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < N; i += (size_t)gridDim.x * blockDim.x) {
        const float d = fminf(fmaxf(x[i], 0.f), 1.f) - fminf(fmaxf(y[i], 0.f), 1.f);
        s += d * d;
    }
    const float tot = block_sum(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// out[0] = MSE, out[1] = 10 log10(1 / MSE) (infinite for identical images).
__global__ __launch_bounds__(kFinalThreads) void k_psnr_final(const float* __restrict__ part, int np,
                                                              double invN, float* __restrict__ out) {
    __shared__ float red[kFinalThreads / 64];
    const float sse = block_sum_1024(strided_sum(part, np), red);
    if (threadIdx.x == 0) {
        const double mse = (double)sse * invN;
        out[0] = (float)mse;
        out[1] = mse > 0.0 ? (float)(10.0 * log10(1.0 / mse)) : INFINITY;
    }
}

inline int ssim_blocks(int W, int H) { return ((W + kSW - 1) / kSW) * ((H + kRH - 1) / kRH) * 3; }

inline size_t part_bytes(int W, int H) {
    const int nb = ssim_blocks(W, H) > kL1Blocks ? ssim_blocks(W, H) : kL1Blocks;
    return (((size_t)2 * nb * sizeof(float)) + 255) & ~(size_t)255;
}

}  // namespace

extern "C" pgs_status pgs_psnr(const float* x_dev, const float* y_dev, int32_t width, int32_t height,
                               float* out_dev, void* workspace_dev, size_t workspace_bytes, void* stream) {
    PGS_REQUIRE(width > 0 && height > 0, "pgs_psnr: bad size");
    PGS_REQUIRE(x_dev && y_dev && out_dev && workspace_dev, "pgs_psnr: null pointer");
    PGS_REQUIRE(workspace_bytes >= kL1Blocks * sizeof(float), "pgs_psnr: workspace too small");
    hipStream_t s = pgs::as_stream(stream);
    const size_t N = (size_t)3 * width * height;
    float* part = static_cast<float*>(workspace_dev);
    k_sq_err<<<kL1Blocks, 256, 0, s>>>(x_dev, y_dev, N, part);
    k_psnr_final<<<1, kFinalThreads, 0, s>>>(part, kL1Blocks, 1.0 / (double)N, out_dev);
    PGS_CHECK_LAUNCH("pgs_psnr");
    return PGS_OK;
}

extern "C" size_t pgs_loss_workspace(int32_t width, int32_t height) {
    if (width <= 0 || height <= 0) return 256;
    return part_bytes(width, height) + (size_t)9 * width * height * sizeof(float);
}

extern "C" pgs_status pgs_loss_l1_dssim(const float* x_dev, const float* y_dev, int32_t width,
                                        int32_t height, float lambda, float* loss_dev, float* dl_dx_dev,
                                        void* workspace_dev, size_t workspace_bytes, void* stream) {
    PGS_REQUIRE(width > 0 && height > 0, "pgs_loss_l1_dssim: bad size");
    PGS_REQUIRE(lambda >= 0.f && lambda <= 1.f, "pgs_loss_l1_dssim: lambda %g", (double)lambda);
    PGS_REQUIRE(x_dev && y_dev && loss_dev && dl_dx_dev && workspace_dev, "pgs_loss_l1_dssim: null pointer");
    const size_t need = lambda > 0.f ? pgs_loss_workspace(width, height) : part_bytes(width, height);
    PGS_REQUIRE(workspace_bytes >= need, "pgs_loss_l1_dssim: workspace %zu < %zu", workspace_bytes, need);
    hipStream_t s = pgs::as_stream(stream);
    const int npart = (int)(part_bytes(width, height) / (2 * sizeof(float)));
    float* part_l1 = static_cast<float*>(workspace_dev);
    float* part_s = part_l1 + npart;
    float* m = reinterpret_cast<float*>(static_cast<char*>(workspace_dev) + part_bytes(width, height));
    const size_t N = (size_t)3 * width * height;
    const float invN = (float)(1.0 / (double)N);
    int nl = kL1Blocks, ns = 0;
    if (lambda == 0.f) {
        k_l1<<<kL1Blocks, 256, 0, s>>>(x_dev, y_dev, N, invN, dl_dx_dev, part_l1);
    } else {
        const Win win = gaussian_window();
        const dim3 grid((width + kSW - 1) / kSW, (height + kRH - 1) / kRH, 3);
        nl = ns = ssim_blocks(width, height);
        k_ssim_fwd<<<grid, 64, 0, s>>>(x_dev, y_dev, width, height, win, m, part_s);
        k_ssim_bwd<<<grid, 64, 0, s>>>(x_dev, y_dev, width, height, win, m, (1.f - lambda) * invN,
                                       lambda * invN, dl_dx_dev, part_l1);
    }
    k_loss_final<<<1, kFinalThreads, 0, s>>>(part_l1, nl, part_s, ns, lambda, invN, loss_dev);
    PGS_CHECK_LAUNCH("pgs_loss_l1_dssim");
    return PGS_OK;
}
