// Seeding network 64 -> 64 -> 64 -> 64 -> 8 (exact-erf GELU after the hidden
// layers) on bfloat16 matrix cores with float32 accumulation: inference,
// training backward (weight gradients), and the log-Euclidean seed loss.
//
// The network is this project's stand-in for PocketGS's seeding operator
// (Sec. "Prior-Conditioned Gaussian Parameterization"); it is not in the
// paper.  Weights are one float32 vector [W1 (64x64, out-major), b1, W2, b2,
// W3, b3, W4 (8x64), b4] of 13000 values; every product rounds both operands
// to bfloat16 (nearest, ties to even) and accumulates in float32.
//
// Tiling.  A block of 4 waves owns tiles of 64 rows.  Every product is a
// 16x16 output tile of v_mfma_f32_16x16x32_bf16 (one 16x16x16 for the
// 16-wide K of the output layer's backward).  Operand layout of that
// instruction: lane l supplies A[l%16][8(l/16)+j] and B[8(l/16)+j][l%16]
// (j < 8) and receives D[4(l/16)+j][l%16] (j < 4).  Forward tiles compute
// Z^T = W H^T, so A rows are weight rows and B columns are activation rows:
// both read 16 contiguous bytes from LDS, and each lane receives 4
// consecutive outputs of one row, stored as one 8-byte write.  Wave w owns
// outputs 16w..16w+15 of every hidden layer for all 64 rows; in the backward
// pass the same wave owns inputs 16w..16w+15 of dH = dZ W, so GELU'(Z) stays
// in the registers that produced it.  Weight gradients dW = dZ^T H reduce
// over rows, so the kernel keeps transposed copies (rows contiguous) of H
// and dZ in LDS and accumulates each block's dW in registers across all its
// tiles; one partial per block goes to the workspace and a second kernel
// sums the partials in block order (deterministic for a given row count).
#include <math.h>

#include "common.hpp"

namespace {

typedef short bf16x8 __attribute__((ext_vector_type(8)));
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16;

constexpr int kRows = 64;       // rows per tile
constexpr int kThreads = 256;   // 4 waves
constexpr int kS = 72;          // LDS row stride (elements) of 64-wide operands
constexpr int kS4 = 24;         // LDS row stride of 16-wide operands
constexpr int kNW = 13000;      // weights
constexpr int kLayerStride = 64 * 64 + 64;   // W_l then b_l, hidden layers
constexpr int kOffW4 = 3 * kLayerStride;     // 12480
constexpr int kOffB4 = kOffW4 + 8 * 64;      // 12992
constexpr int kMaxBwdBlocks = 256;
constexpr int kLossThreads = 256;

__device__ __forceinline__ u16 to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (u16)((u >> 16) | 0x40u);   // quiet NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return (u16)(u >> 16);
}

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float z) {
    return 0.5f * (1.f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

__device__ __forceinline__ bf16x8 ld8(const u16* p) { return *reinterpret_cast<const bf16x8*>(p); }
__device__ __forceinline__ bf16x4 ld4(const u16* p) { return *reinterpret_cast<const bf16x4*>(p); }
__device__ __forceinline__ void st4(u16* p, const u16 v[4]) {
    uint2 w;
    w.x = (uint32_t)v[0] | ((uint32_t)v[1] << 16);
    w.y = (uint32_t)v[2] | ((uint32_t)v[3] << 16);
    *reinterpret_cast<uint2*>(p) = w;
}
__device__ __forceinline__ f32x4 mfma32(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// Weights into LDS as bfloat16: W holds W1..W3 (rows 0..191) and W4 padded
// to 16 rows (rows 192..207), stride kS.  Wt (optional) holds W2^T, W3^T
// (stride kS) and W4^T (64 x 16, stride kS4, at element 128 * kS).
__device__ void load_weights(const float* __restrict__ w, u16* W, u16* Wt, float* bias) {
    const int tid = threadIdx.x;
    for (int e = tid; e < 3 * 4096; e += kThreads) {
        const int l = e >> 12, k = e & 4095, o = k >> 6, i = k & 63;
        const u16 v = to_bf16(w[l * kLayerStride + k]);
        W[(l * 64 + o) * kS + i] = v;
        if (Wt && l > 0) Wt[((l - 1) * 64 + i) * kS + o] = v;
    }
    for (int e = tid; e < 16 * 64; e += kThreads) {
        const int o = e >> 6, i = e & 63;
        const u16 v = o < 8 ? to_bf16(w[kOffW4 + o * 64 + i]) : (u16)0;
        W[(192 + o) * kS + i] = v;
        if (Wt) Wt[128 * kS + i * kS4 + o] = v;
    }
    for (int e = tid; e < 200; e += kThreads)
        bias[e] = e < 192 ? w[(e >> 6) * kLayerStride + 4096 + (e & 63)] : w[kOffB4 + e - 192];
}

// Input rows row0..row0+63 (zeros past m) as bfloat16, row-major into H0
// and (optional) transposed into HT0.
__device__ void load_x(const float* __restrict__ x, int m, int row0, u16* H0, u16* HT0) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const int f = tid + kThreads * p, r = f >> 4, c = (f & 15) * 4;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (row0 + r < m) v = *reinterpret_cast<const float4*>(x + (size_t)(row0 + r) * 64 + c);
        const u16 b[4] = {to_bf16(v.x), to_bf16(v.y), to_bf16(v.z), to_bf16(v.w)};
        st4(H0 + r * kS + c, b);
        if (HT0) {
#pragma unroll
            for (int j = 0; j < 4; ++j) HT0[(c + j) * kS + r] = b[j];
        }
    }
}

// Hidden layer l: Hout = bf16(GELU(Hin W_l^T + b_l)).  Wave w computes
// outputs 16w..16w+15 for the four 16-row tiles; gp (optional) receives
// GELU'(Z) in the accumulator layout.
__device__ __forceinline__ void hidden_layer(int l, const u16* Hin, u16* Hout, u16* HTout, const u16* W,
                                             const float* bias, float gp[4][4], bool keep) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, lr = lane & 15, lg = lane >> 4;
    const int o = 16 * wave + 4 * lg;
    const u16* Wl = W + (l * 64 + 16 * wave + lr) * kS + 8 * lg;
    const bf16x8 a0 = ld8(Wl), a1 = ld8(Wl + 32);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int r = 16 * t + lr;
        const u16* Hr = Hin + r * kS + 8 * lg;
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = mfma32(a0, ld8(Hr), acc);
        acc = mfma32(a1, ld8(Hr + 32), acc);
        u16 hb[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const float z = acc[j] + bias[l * 64 + o + j];
            hb[j] = to_bf16(gelu(z));
            if (keep) gp[t][j] = gelu_grad(z);
        }
        st4(Hout + r * kS + o, hb);
        if (HTout) {
#pragma unroll
            for (int j = 0; j < 4; ++j) HTout[(o + j) * kS + r] = hb[j];
        }
    }
}

__global__ __launch_bounds__(kThreads) void k_mlp_forward(const float* __restrict__ w,
                                                          const float* __restrict__ x, int m,
                                                          float* __restrict__ y) {
    __shared__ __align__(16) u16 W[208 * kS];
    __shared__ __align__(16) u16 H[2][64 * kS];
    __shared__ float bias[200];
    load_weights(w, W, nullptr, bias);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, lr = lane & 15, lg = lane >> 4;
    const int tiles = (m + kRows - 1) / kRows;
    float unused[4][4];
    for (int tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const int row0 = tile * kRows;
        __syncthreads();
        load_x(x, m, row0, H[0], nullptr);
        __syncthreads();
        hidden_layer(0, H[0], H[1], nullptr, W, bias, unused, false);
        __syncthreads();
        hidden_layer(1, H[1], H[0], nullptr, W, bias, unused, false);
        __syncthreads();
        hidden_layer(2, H[0], H[1], nullptr, W, bias, unused, false);
        __syncthreads();
        // output layer: wave w takes rows 16w..16w+15; lanes with l/16 < 2
        // receive the 8 real outputs (rows 8..15 of W4 are zero padding)
        const u16* Wr = W + (192 + lr) * kS + 8 * lg;
        const u16* Hr = H[1] + (16 * wave + lr) * kS + 8 * lg;
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = mfma32(ld8(Wr), ld8(Hr), acc);
        acc = mfma32(ld8(Wr + 32), ld8(Hr + 32), acc);
        const int row = row0 + 16 * wave + lr;
        if (lg < 2 && row < m) {
            const int o = 4 * lg;
            *reinterpret_cast<float4*>(y + (size_t)row * 8 + o) =
                make_float4(acc[0] + bias[192 + o], acc[1] + bias[193 + o], acc[2] + bias[194 + o],
                            acc[3] + bias[195 + o]);
        }
    }
}

__global__ __launch_bounds__(kThreads) void k_mlp_backward(const float* __restrict__ w,
                                                           const float* __restrict__ x, int m,
                                                           const float* __restrict__ dy,
                                                           float* __restrict__ partial) {
    __shared__ __align__(16) u16 W[208 * kS];
    __shared__ __align__(16) u16 Wt[128 * kS + 64 * kS4];
    __shared__ __align__(16) u16 H[2][64 * kS];
    __shared__ __align__(16) u16 HT[4][64 * kS];
    __shared__ __align__(16) u16 dZ[64 * kS];
    __shared__ __align__(16) u16 dZT[64 * kS];
    __shared__ __align__(16) u16 dZ4[64 * kS4];
    __shared__ __align__(16) u16 dZ4T[16 * kS];
    __shared__ float bias[200];
    __shared__ float db4[kThreads];
    load_weights(w, W, Wt, bias);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, lr = lane & 15, lg = lane >> 4;
    const int tiles = (m + kRows - 1) / kRows;

    f32x4 accW[3][4];       // dW_l[16 wave + 4 lg + j][16 c + lr]
    f32x4 accW4 = {0.f, 0.f, 0.f, 0.f};    // dW4[4 lg + j][16 wave + lr]
    float dbh[3][4];        // bias gradient partials of outputs 16 wave + 4 lg + j
    float db4acc = 0.f;     // output bias gradient partial of output tid % 16
#pragma unroll
    for (int l = 0; l < 3; ++l)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            accW[l][c] = {0.f, 0.f, 0.f, 0.f};
            dbh[l][c] = 0.f;
        }
    float gp[3][4][4];

    for (int tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const int row0 = tile * kRows;
        __syncthreads();
        load_x(x, m, row0, H[0], HT[0]);
        __syncthreads();
        hidden_layer(0, H[0], H[1], HT[1], W, bias, gp[0], true);
        __syncthreads();
        hidden_layer(1, H[1], H[0], HT[2], W, bias, gp[1], true);
        __syncthreads();
        hidden_layer(2, H[0], H[1], HT[3], W, bias, gp[2], true);
        // output gradient rows: bfloat16 copies (16 columns, 8..15 zero)
        for (int e = tid; e < 64 * 16; e += kThreads) {
            const int r = e >> 4, o = e & 15;
            float v = 0.f;
            if (o < 8 && row0 + r < m) v = dy[(size_t)(row0 + r) * 8 + o];
            db4acc += v;
            const u16 b = to_bf16(v);
            dZ4[r * kS4 + o] = b;
            dZ4T[o * kS + r] = b;
        }
        __syncthreads();

        // output layer: dW4 += dZ4^T H3 (wave w: inputs 16w..16w+15);
        // dH3 = dZ4 W4 with K = 16 outputs
        {
            const u16* A = dZ4T + lr * kS + 8 * lg;
            const u16* Bm = HT[3] + (16 * wave + lr) * kS + 8 * lg;
            accW4 = mfma32(ld8(A), ld8(Bm), accW4);
            accW4 = mfma32(ld8(A + 32), ld8(Bm + 32), accW4);
            const bf16x4 a = ld4(Wt + 128 * kS + (16 * wave + lr) * kS4 + 4 * lg);
            const int o = 16 * wave + 4 * lg;
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                f32x4 dh = {0.f, 0.f, 0.f, 0.f};
                dh = mfma16(a, ld4(dZ4 + (16 * t + lr) * kS4 + 4 * lg), dh);
                const int r = 16 * t + lr;
                u16 b[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const float dz = dh[j] * gp[2][t][j];
                    dbh[2][j] += dz;
                    b[j] = to_bf16(dz);
                }
                st4(dZ + r * kS + o, b);
#pragma unroll
                for (int j = 0; j < 4; ++j) dZT[(o + j) * kS + r] = b[j];
            }
        }
        __syncthreads();

        // hidden layers 2, 1, 0: dW_l += dZ_l^T H_l; dH_l = dZ_l W_l feeds
        // dZ_{l-1} = dH_l * GELU'(Z_{l-1})
#pragma unroll
        for (int l = 2; l >= 0; --l) {
            const u16* A = dZT + (16 * wave + lr) * kS + 8 * lg;
            const bf16x8 a0 = ld8(A), a1 = ld8(A + 32);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const u16* Bm = HT[l] + (16 * c + lr) * kS + 8 * lg;
                accW[l][c] = mfma32(a0, ld8(Bm), accW[l][c]);
                accW[l][c] = mfma32(a1, ld8(Bm + 32), accW[l][c]);
            }
            if (l > 0) {
                const u16* Wl = Wt + ((l - 1) * 64 + 16 * wave + lr) * kS + 8 * lg;
                const bf16x8 w0 = ld8(Wl), w1 = ld8(Wl + 32);
                f32x4 dh[4];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const u16* Bm = dZ + (16 * t + lr) * kS + 8 * lg;
                    dh[t] = {0.f, 0.f, 0.f, 0.f};
                    dh[t] = mfma32(w0, ld8(Bm), dh[t]);
                    dh[t] = mfma32(w1, ld8(Bm + 32), dh[t]);
                }
                __syncthreads();   // every wave has read dZ_l and dZ_l^T
                const int o = 16 * wave + 4 * lg;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const int r = 16 * t + lr;
                    u16 b[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const float dz = dh[t][j] * gp[l - 1][t][j];
                        dbh[l - 1][j] += dz;
                        b[j] = to_bf16(dz);
                    }
                    st4(dZ + r * kS + o, b);
#pragma unroll
                    for (int j = 0; j < 4; ++j) dZT[(o + j) * kS + r] = b[j];
                }
                __syncthreads();
            }
        }
    }

    // block partial: weight gradients straight from the accumulators
    float* out = partial + (size_t)blockIdx.x * kNW;
#pragma unroll
    for (int l = 0; l < 3; ++l)
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                out[l * kLayerStride + (16 * wave + 4 * lg + j) * 64 + 16 * c + lr] = accW[l][c][j];
    if (lg < 2) {
#pragma unroll
        for (int j = 0; j < 4; ++j) out[kOffW4 + (4 * lg + j) * 64 + 16 * wave + lr] = accW4[j];
    }
    // hidden biases: sum the 16 lanes that share an output (fixed order)
#pragma unroll
    for (int l = 0; l < 3; ++l)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            float v = dbh[l][j];
            v += __shfl_xor(v, 1);
            v += __shfl_xor(v, 2);
            v += __shfl_xor(v, 4);
            v += __shfl_xor(v, 8);
            if (lr == 0) out[l * kLayerStride + 4096 + 16 * wave + 4 * lg + j] = v;
        }
    db4[tid] = db4acc;
    __syncthreads();
    if (tid < 8) {
        float v = 0.f;
        for (int k = 0; k < kThreads / 16; ++k) v += db4[16 * k + tid];
        out[kOffB4 + tid] = v;
    }
}

__global__ __launch_bounds__(256) void k_mlp_reduce(const float* __restrict__ partial, int blocks,
                                                    float* __restrict__ dw) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= kNW) return;
    float s = 0.f;
    for (int b = 0; b < blocks; ++b) s += partial[(size_t)b * kNW + k];
    dw[k] = s;
}

// ---------------------------------------------------------------- seed loss
// Per row: q = y[3:7]/|y[3:7]|, R = R_base R(q), s = logs_base + y[0:3],
// L = R diag(2 s) R^T; loss = ||L - M*||_F^2 + (logit(0.1) + y[7] - logit*)^2.
// base row: R (9, row-major), log-scales (3), quaternion (4).
// target row: M*00, M*11, M*22, M*01, M*02, M*12, logit*, unused.

__device__ void rot_of_quat(const double q[4], double R[3][3]) {
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0][0] = 1 - 2 * (y * y + z * z); R[0][1] = 2 * (x * y - w * z); R[0][2] = 2 * (x * z + w * y);
    R[1][0] = 2 * (x * y + w * z); R[1][1] = 1 - 2 * (x * x + z * z); R[1][2] = 2 * (y * z - w * x);
    R[2][0] = 2 * (x * z - w * y); R[2][1] = 2 * (y * z + w * x); R[2][2] = 1 - 2 * (x * x + y * y);
}

__global__ __launch_bounds__(kLossThreads) void k_seed_loss(const float* __restrict__ y,
                                                            const float* __restrict__ base,
                                                            const float* __restrict__ target, int m,
                                                            double scale, double* __restrict__ partial,
                                                            float* __restrict__ dy) {
    __shared__ double red[kLossThreads];
    const int i = blockIdx.x * kLossThreads + threadIdx.x;
    double per = 0.0;
    if (i < m) {
        double Y[8], Rb[3][3], ls[3], M[3][3];
        for (int k = 0; k < 8; ++k) Y[k] = y[(size_t)i * 8 + k];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) Rb[a][b] = base[(size_t)i * 16 + 3 * a + b];
        for (int a = 0; a < 3; ++a) ls[a] = base[(size_t)i * 16 + 9 + a];
        const float* T = target + (size_t)i * 8;
        M[0][0] = T[0]; M[1][1] = T[1]; M[2][2] = T[2];
        M[0][1] = M[1][0] = T[3];
        M[0][2] = M[2][0] = T[4];
        M[1][2] = M[2][1] = T[5];
        const double qn = sqrt(Y[3] * Y[3] + Y[4] * Y[4] + Y[5] * Y[5] + Y[6] * Y[6]);
        const double q[4] = {Y[3] / qn, Y[4] / qn, Y[5] / qn, Y[6] / qn};
        double Ro[3][3], Rh[3][3];
        rot_of_quat(q, Ro);
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) Rh[a][b] = Rb[a][0] * Ro[0][b] + Rb[a][1] * Ro[1][b] + Rb[a][2] * Ro[2][b];
        double s2[3];
        for (int k = 0; k < 3; ++k) s2[k] = 2.0 * (ls[k] + Y[k]);
        double G[3][3];   // 2 (L - M)
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                const double L = Rh[a][0] * s2[0] * Rh[b][0] + Rh[a][1] * s2[1] * Rh[b][1] +
                                 Rh[a][2] * s2[2] * Rh[b][2];
                const double d = L - M[a][b];
                per += d * d;
                G[a][b] = 2.0 * d;
            }
        const double dl = log(1.0 / 9.0) + Y[7] - T[6];   // logit(0.1) = log(1/9)
        per += dl * dl;
        if (dy) {
            // dper/ds_k = 2 r_k^T G r_k;  dper/dRh = 2 G Rh diag(2 s)
            double GR[3][3];
            for (int a = 0; a < 3; ++a)
                for (int k = 0; k < 3; ++k) GR[a][k] = G[a][0] * Rh[0][k] + G[a][1] * Rh[1][k] + G[a][2] * Rh[2][k];
            double ds[3], dRh[3][3];
            for (int k = 0; k < 3; ++k) {
                ds[k] = 2.0 * (Rh[0][k] * GR[0][k] + Rh[1][k] * GR[1][k] + Rh[2][k] * GR[2][k]);
                for (int a = 0; a < 3; ++a) dRh[a][k] = 2.0 * GR[a][k] * s2[k];
            }
            double E[3][3];   // dper/dRo = Rb^T dRh
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) E[a][b] = Rb[0][a] * dRh[0][b] + Rb[1][a] * dRh[1][b] + Rb[2][a] * dRh[2][b];
            const double w = q[0], x = q[1], yq = q[2], z = q[3];
            double dq[4];
            dq[0] = 2 * (-z * E[0][1] + yq * E[0][2] + z * E[1][0] - x * E[1][2] - yq * E[2][0] + x * E[2][1]);
            dq[1] = 2 * (yq * E[0][1] + z * E[0][2] + yq * E[1][0] - 2 * x * E[1][1] - w * E[1][2] + z * E[2][0] +
                         w * E[2][1] - 2 * x * E[2][2]);
            dq[2] = 2 * (-2 * yq * E[0][0] + x * E[0][1] + w * E[0][2] + x * E[1][0] + z * E[1][2] - w * E[2][0] +
                         z * E[2][1] - 2 * yq * E[2][2]);
            dq[3] = 2 * (-2 * z * E[0][0] - w * E[0][1] + x * E[0][2] + w * E[1][0] - 2 * z * E[1][1] +
                         yq * E[1][2] + x * E[2][0] + yq * E[2][1]);
            const double qd = q[0] * dq[0] + q[1] * dq[1] + q[2] * dq[2] + q[3] * dq[3];
            float* D = dy + (size_t)i * 8;
            for (int k = 0; k < 3; ++k) D[k] = (float)(scale * ds[k]);
            for (int k = 0; k < 4; ++k) D[3 + k] = (float)(scale * (dq[k] - q[k] * qd) / qn);
            D[7] = (float)(scale * 2.0 * dl);
        }
    }
    red[threadIdx.x] = per;
    __syncthreads();
    for (int s = kLossThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(1024) void k_seed_loss_final(const double* __restrict__ partial, int blocks,
                                                          double scale, float* __restrict__ loss) {
    __shared__ double red[1024];
    double s = 0.0;
    for (int b = threadIdx.x; b < blocks; b += 1024) s += partial[b];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 512; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = (float)(scale * red[0]);
}

int bwd_blocks(int m) {
    const int tiles = (m + kRows - 1) / kRows;
    return tiles < kMaxBwdBlocks ? tiles : kMaxBwdBlocks;
}

bool aligned16(const void* p) { return ((uintptr_t)p & 15u) == 0; }

}  // namespace

extern "C" int32_t pgs_mlp_weight_count(void) { return kNW; }

extern "C" pgs_status pgs_mlp_forward(const float* weights_dev, const float* x_dev, int32_t m, float* y_dev,
                                      void* stream) {
    PGS_REQUIRE(m >= 0, "pgs_mlp_forward: m must be >= 0 (m=%d)", m);
    if (m == 0) return PGS_OK;
    PGS_REQUIRE(weights_dev && x_dev && y_dev, "pgs_mlp_forward: null pointer");
    PGS_REQUIRE(aligned16(x_dev) && aligned16(y_dev), "pgs_mlp_forward: x and y must be 16-byte aligned");
    const int tiles = (m + kRows - 1) / kRows;
    const int grid = tiles < 512 ? tiles : 512;   // persistent: each block converts the weights once
    k_mlp_forward<<<grid, kThreads, 0, pgs::as_stream(stream)>>>(weights_dev, x_dev, m, y_dev);
    PGS_CHECK_LAUNCH("pgs_mlp_forward");
    return PGS_OK;
}

extern "C" size_t pgs_mlp_backward_workspace(int32_t m) {
    if (m <= 0) return 0;
    return (size_t)bwd_blocks(m) * kNW * sizeof(float);
}

extern "C" pgs_status pgs_mlp_backward(const float* weights_dev, const float* x_dev, int32_t m,
                                       const float* dy_dev, float* dweights_dev, void* workspace_dev,
                                       size_t workspace_bytes, void* stream) {
    PGS_REQUIRE(m >= 0, "pgs_mlp_backward: m must be >= 0 (m=%d)", m);
    PGS_REQUIRE(weights_dev && dweights_dev, "pgs_mlp_backward: null pointer");
    hipStream_t s = pgs::as_stream(stream);
    if (m == 0) {   // no rows: the reduction over zero partials writes zeros
        k_mlp_reduce<<<(kNW + 255) / 256, 256, 0, s>>>(nullptr, 0, dweights_dev);
        PGS_CHECK_LAUNCH("pgs_mlp_backward");
        return PGS_OK;
    }
    PGS_REQUIRE(x_dev && dy_dev && workspace_dev, "pgs_mlp_backward: null pointer");
    PGS_REQUIRE(aligned16(x_dev), "pgs_mlp_backward: x must be 16-byte aligned");
    PGS_REQUIRE(workspace_bytes >= pgs_mlp_backward_workspace(m),
                "pgs_mlp_backward: workspace too small (%zu < %zu)", workspace_bytes,
                pgs_mlp_backward_workspace(m));
    const int blocks = bwd_blocks(m);
    float* partial = static_cast<float*>(workspace_dev);
    k_mlp_backward<<<blocks, kThreads, 0, s>>>(weights_dev, x_dev, m, dy_dev, partial);
    PGS_CHECK_LAUNCH("pgs_mlp_backward");
    k_mlp_reduce<<<(kNW + 255) / 256, 256, 0, s>>>(partial, blocks, dweights_dev);
    PGS_CHECK_LAUNCH("pgs_mlp_backward reduce");
    return PGS_OK;
}

extern "C" size_t pgs_seed_loss_workspace(int32_t m) {
    if (m <= 0) return 0;
    return (size_t)((m + kLossThreads - 1) / kLossThreads) * sizeof(double);
}

extern "C" pgs_status pgs_seed_loss(const float* y_dev, const float* base_dev, const float* target_dev,
                                    int32_t m, float scale, float* loss_dev, float* dy_dev, void* workspace_dev,
                                    size_t workspace_bytes, void* stream) {
    PGS_REQUIRE(m > 0, "pgs_seed_loss: m must be > 0 (m=%d)", m);
    PGS_REQUIRE(y_dev && base_dev && target_dev && loss_dev && workspace_dev, "pgs_seed_loss: null pointer");
    PGS_REQUIRE(workspace_bytes >= pgs_seed_loss_workspace(m), "pgs_seed_loss: workspace too small (%zu < %zu)",
                workspace_bytes, pgs_seed_loss_workspace(m));
    hipStream_t s = pgs::as_stream(stream);
    const int blocks = (m + kLossThreads - 1) / kLossThreads;
    double* partial = static_cast<double*>(workspace_dev);
    k_seed_loss<<<blocks, kLossThreads, 0, s>>>(y_dev, base_dev, target_dev, m, (double)scale, partial, dy_dev);
    PGS_CHECK_LAUNCH("pgs_seed_loss");
    k_seed_loss_final<<<1, 1024, 0, s>>>(partial, blocks, (double)scale, loss_dev);
    PGS_CHECK_LAUNCH("pgs_seed_loss final");
    return PGS_OK;
}
