// EWA projection of 3D Gaussians and its backward (one thread per Gaussian).
//
// PocketGS composites "depth-sorted visible Gaussians" (Sec. "Explicit
// Computation Graph") and inherits the projection from 3D Gaussian Splatting.
// Reading used: near plane 0.2, Sigma2D = (J W) Sigma (J W)^T + 0.3 I,
// J clamped at 1.3x the half field of view, radius ceil(3 sqrt(lambda_max))
// with lambda_max = m + sqrt(max(0.1, m^2 - det)), inclusive tile rectangle
// [floor((u-r)/TW), floor((u+r)/TW)] clipped to the image, real SH colour
// + 1/2 clamped at 0, sigmoid opacity.
//
// All per-Gaussian maths runs in float64 and is rounded once to float32.
// The work is bound by the canonical-parameter reads (56 B/Gaussian at SH
// degree 0, 236 B at degree 3), so the float64 ALU cost is hidden; in
// exchange every integer decision (culling, radius, rectangle, depth-key
// bits) is taken on values accurate to ~1e-16 relative.
#include <math.h>

#include "common.hpp"

namespace {

using pgs::CamD;

// Real SH normalisation constants (textbook values, Condon-Shortley phase):
constexpr double kY00 = 0.28209479177387814;   // 1/(2 sqrt(pi))
constexpr double kY1 = 0.4886025119029199;     // sqrt(3/(4 pi))
constexpr double kY2a = 1.0925484305920792;    // sqrt(15/(4 pi))
constexpr double kY2b = 0.31539156525252005;   // sqrt(5/(16 pi))
constexpr double kY2c = 0.5462742152960396;    // sqrt(15/(16 pi))
constexpr double kY3a = 0.5900435899266435;    // sqrt(35/(32 pi))
constexpr double kY3b = 2.890611442640554;     // sqrt(105/(4 pi))
constexpr double kY3c = 0.4570457994644658;    // sqrt(21/(32 pi))
constexpr double kY3d = 0.3731763325901154;    // sqrt(7/(16 pi))
constexpr double kY3e = 1.445305721320277;     // sqrt(105/(16 pi))

// Basis values Y[k], k = l*l + l + m, at unit direction (x, y, z).
template <int D>
__device__ __forceinline__ void sh_eval(double x, double y, double z, double* Y) {
    Y[0] = kY00;
    if (D >= 1) {
        Y[1] = -kY1 * y;
        Y[2] = kY1 * z;
        Y[3] = -kY1 * x;
    }
    if (D >= 2) {
        Y[4] = kY2a * x * y;
        Y[5] = -kY2a * y * z;
        Y[6] = kY2b * (3.0 * z * z - 1.0);
        Y[7] = -kY2a * x * z;
        Y[8] = kY2c * (x * x - y * y);
    }
    if (D >= 3) {
        Y[9] = -kY3a * y * (3.0 * x * x - y * y);
        Y[10] = kY3b * x * y * z;
        Y[11] = -kY3c * y * (5.0 * z * z - 1.0);
        Y[12] = kY3d * z * (5.0 * z * z - 3.0);
        Y[13] = -kY3c * x * (5.0 * z * z - 1.0);
        Y[14] = kY3e * z * (x * x - y * y);
        Y[15] = -kY3a * x * (x * x - 3.0 * y * y);
    }
}

// Gradient of polynomial Y[k] with respect to (x, y, z) (any extension off
// the sphere works: the chain through normalisation removes the radial
// part); k is a constant wherever this is called, so the switch folds away.
__device__ __forceinline__ void sh_grad_k(int k, double x, double y, double z, double& gx, double& gy,
                                          double& gz) {
    switch (k) {
        case 1: gx = 0.0; gy = -kY1; gz = 0.0; break;
        case 2: gx = 0.0; gy = 0.0; gz = kY1; break;
        case 3: gx = -kY1; gy = 0.0; gz = 0.0; break;
        case 4: gx = kY2a * y; gy = kY2a * x; gz = 0.0; break;
        case 5: gx = 0.0; gy = -kY2a * z; gz = -kY2a * y; break;
        case 6: gx = 0.0; gy = 0.0; gz = 6.0 * kY2b * z; break;
        case 7: gx = -kY2a * z; gy = 0.0; gz = -kY2a * x; break;
        case 8: gx = 2.0 * kY2c * x; gy = -2.0 * kY2c * y; gz = 0.0; break;
        case 9: gx = -6.0 * kY3a * x * y; gy = -3.0 * kY3a * (x * x - y * y); gz = 0.0; break;
        case 10: gx = kY3b * y * z; gy = kY3b * x * z; gz = kY3b * x * y; break;
        case 11: gx = 0.0; gy = -kY3c * (5.0 * z * z - 1.0); gz = -10.0 * kY3c * y * z; break;
        case 12: gx = 0.0; gy = 0.0; gz = kY3d * (15.0 * z * z - 3.0); break;
        case 13: gx = -kY3c * (5.0 * z * z - 1.0); gy = 0.0; gz = -10.0 * kY3c * x * z; break;
        case 14: gx = 2.0 * kY3e * x * z; gy = -2.0 * kY3e * y * z; gz = kY3e * (x * x - y * y); break;
        case 15: gx = -3.0 * kY3a * (x * x - y * y); gy = 6.0 * kY3a * x * y; gz = 0.0; break;
        default: gx = gy = gz = 0.0; break;
    }
}

// Geometry shared by the forward and the backward kernels: the part that
// does not depend on the view (rotation, scales, 3D covariance) and the
// per-view part (camera-space mean, Jacobian, 2D covariance).
struct Shape {
    double qn[4], qlen;      // normalised quaternion and |q|
    double R[9];             // rotation of the Gaussian
    double s[3];             // exp(log-scale)
    double Sig[6];           // 3D covariance xx, xy, xz, yy, yz, zz
};

struct Geo {
    double x, y, z;          // camera-space mean
    double tx, ty;           // clamped x/z, y/z
    bool clx, cly;           // J clamp active
    double T0[3], T1[3];     // rows of J W
    double a, b, c, det;     // Sigma2D with dilation
};

__device__ __forceinline__ double prow(const float* P, int r, int n, int i) {
    return (double)P[(size_t)r * n + i];
}

__device__ __forceinline__ void shape_of(const float* __restrict__ P, int n, int i, Shape& S3) {
    const double qw = prow(P, 6, n, i), qx = prow(P, 7, n, i), qy = prow(P, 8, n, i),
                 qz = prow(P, 9, n, i);
    S3.qlen = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
    const double w = qw / S3.qlen, x = qx / S3.qlen, y = qy / S3.qlen, z = qz / S3.qlen;
    S3.qn[0] = w; S3.qn[1] = x; S3.qn[2] = y; S3.qn[3] = z;
    double* R = S3.R;
    R[0] = 1.0 - 2.0 * (y * y + z * z); R[1] = 2.0 * (x * y - w * z); R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z); R[4] = 1.0 - 2.0 * (x * x + z * z); R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y); R[7] = 2.0 * (y * z + w * x); R[8] = 1.0 - 2.0 * (x * x + y * y);
    for (int k = 0; k < 3; ++k) S3.s[k] = exp(prow(P, 3 + k, n, i));
    // Sigma = R diag(s^2) R^T
    const double s0 = S3.s[0] * S3.s[0], s1 = S3.s[1] * S3.s[1], s2 = S3.s[2] * S3.s[2];
    auto sig = [&](int r, int c) { return R[3 * r] * R[3 * c] * s0 + R[3 * r + 1] * R[3 * c + 1] * s1 + R[3 * r + 2] * R[3 * c + 2] * s2; };
    S3.Sig[0] = sig(0, 0); S3.Sig[1] = sig(0, 1); S3.Sig[2] = sig(0, 2);
    S3.Sig[3] = sig(1, 1); S3.Sig[4] = sig(1, 2); S3.Sig[5] = sig(2, 2);
}

__device__ __forceinline__ void view_geometry(const float* __restrict__ P, int n, int i, const Shape& S3,
                                              const CamD& cam, Geo& G) {
    const double mx = prow(P, 0, n, i), my = prow(P, 1, n, i), mz = prow(P, 2, n, i);
    G.x = cam.R[0] * mx + cam.R[1] * my + cam.R[2] * mz + cam.t[0];
    G.y = cam.R[3] * mx + cam.R[4] * my + cam.R[5] * mz + cam.t[1];
    G.z = cam.R[6] * mx + cam.R[7] * my + cam.R[8] * mz + cam.t[2];
    const double xz = G.x / G.z, yz = G.y / G.z;
    G.clx = (xz < -cam.lim_x) || (xz > cam.lim_x);
    G.cly = (yz < -cam.lim_y) || (yz > cam.lim_y);
    G.tx = fmin(cam.lim_x, fmax(-cam.lim_x, xz));
    G.ty = fmin(cam.lim_y, fmax(-cam.lim_y, yz));
    const double j00 = cam.fx / G.z, j02 = -cam.fx * G.tx / G.z;
    const double j11 = cam.fy / G.z, j12 = -cam.fy * G.ty / G.z;
    for (int k = 0; k < 3; ++k) {
        G.T0[k] = j00 * cam.R[k] + j02 * cam.R[6 + k];
        G.T1[k] = j11 * cam.R[3 + k] + j12 * cam.R[6 + k];
    }
    const double* S = S3.Sig;
    const double U0 = S[0] * G.T0[0] + S[1] * G.T0[1] + S[2] * G.T0[2];
    const double U1 = S[1] * G.T0[0] + S[3] * G.T0[1] + S[4] * G.T0[2];
    const double U2 = S[2] * G.T0[0] + S[4] * G.T0[1] + S[5] * G.T0[2];
    const double V0 = S[0] * G.T1[0] + S[1] * G.T1[1] + S[2] * G.T1[2];
    const double V1 = S[1] * G.T1[0] + S[3] * G.T1[1] + S[4] * G.T1[2];
    const double V2 = S[2] * G.T1[0] + S[4] * G.T1[1] + S[5] * G.T1[2];
    G.a = G.T0[0] * U0 + G.T0[1] * U1 + G.T0[2] * U2 + 0.3;
    G.b = G.T0[0] * V0 + G.T0[1] * V1 + G.T0[2] * V2;
    G.c = G.T1[0] * V0 + G.T1[1] * V1 + G.T1[2] * V2 + 0.3;
    G.det = G.a * G.c - G.b * G.b;
}

// Half-extents (x, y) of the pixel region where the compositing kernels can
// find alpha >= 1/255 for a splat with the float32 conic (A, B, C) and
// opacity o that they read.  The region is the ellipse
// A dx^2 + 2B dx dy + C dy^2 <= tau, tau = 2 ln(255 o), enlarged so that it
// also covers the float32 evaluation of the quadratic form (relative error
// below 20 * 2^-24 / (1 - rho), rho = |B| / sqrt(AC)) and of exp (1e-3 added
// to tau).  (-1, -1) when o is below the threshold (no pixel qualifies);
// (inf, inf) when the conic is too close to degenerate (1 - rho < 1e-3) for
// the bound, so that nothing is skipped.
__device__ void alpha_extent(float A, float B, float C, float o, float& hx, float& hy) {
    if (o < pgs::kAlphaMin * (1.0f - 1e-6f)) {
        hx = hy = -1.f;
        return;
    }
    const double a = A, b = B, c = C;
    const double det = a * c - b * b;
    const double one_m_rho = 1.0 - fabs(b) / sqrt(a * c);
    if (!(det > 0.0) || !(a > 0.0) || !(c > 0.0) || !(one_m_rho >= 1e-3)) {
        hx = hy = INFINITY;
        return;
    }
    const double tau = 2.0 * log(255.0 * fmax((double)o, 1.0 / 255.0));
    const double eta = 20.0 * 0x1p-24 / one_m_rho;
    const double t = (tau + 1e-3) / (1.0 - eta);
    hx = (float)(sqrt(t * c / det) * (1.0 + 1e-5) + 1e-2);
    hy = (float)(sqrt(t * a / det) * (1.0 + 1e-5) + 1e-2);
}

// Projection of Gaussian i into one view (record, radius, rectangle and
// tile count at index i of that view's arrays).
template <int D>
__device__ __forceinline__ void project_view(const float* __restrict__ P, int n, int i, const Shape& S3,
                                             const CamD& cam, int tw, int th, int TX, int TY,
                                             float* __restrict__ out, int* __restrict__ radius,
                                             uint32_t* __restrict__ rect, uint32_t* __restrict__ touched) {
    constexpr int K = (D + 1) * (D + 1);
    Geo G;
    view_geometry(P, n, i, S3, cam, G);
    bool ok = G.z > 0.2 && G.det > 0.0;
    double u = 0, v = 0, r = 0, x0 = 0, x1 = -1, y0 = 0, y1 = -1;
    if (ok) {
        u = cam.fx * G.x / G.z + cam.cx;
        v = cam.fy * G.y / G.z + cam.cy;
        const double mid = 0.5 * (G.a + G.c);
        const double lam = mid + sqrt(fmax(0.1, mid * mid - G.det));
        r = ceil(3.0 * sqrt(lam));
        x0 = fmin(fmax(floor((u - r) / tw), 0.0), (double)TX);
        x1 = fmin(fmax(floor((u + r) / tw), -1.0), (double)(TX - 1));
        y0 = fmin(fmax(floor((v - r) / th), 0.0), (double)TY);
        y1 = fmin(fmax(floor((v + r) / th), -1.0), (double)(TY - 1));
        ok = isfinite(u) && isfinite(v) && x0 <= x1 && y0 <= y1;
    }
    if (!ok) {
        float4* rec = reinterpret_cast<float4*>(out + (size_t)i * PGS_PROJ_STRIDE);
        const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
        rec[0] = z;
        rec[1] = z;
        rec[2] = z;
        rec[3] = z;
        radius[i] = 0;
        rect[i] = 0;
        rect[(size_t)n + i] = 0;
        touched[i] = 0;
        return;
    }
    // colour from the view direction
    double d0 = prow(P, 0, n, i) - cam.campos[0];
    double d1 = prow(P, 1, n, i) - cam.campos[1];
    double d2 = prow(P, 2, n, i) - cam.campos[2];
    const double dl = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
    d0 /= dl; d1 /= dl; d2 /= dl;
    double Y[K];
    sh_eval<D>(d0, d1, d2, Y);
    double col[3];
    for (int ch = 0; ch < 3; ++ch) {
        double acc = 0.5;
        for (int k = 0; k < K; ++k) acc += Y[k] * prow(P, 11 + 3 * k + ch, n, i);
        col[ch] = fmax(acc, 0.0);
    }
    const double o = 1.0 / (1.0 + exp(-prow(P, 10, n, i)));
    static_assert(PGS_PROJ_U == 0 && PGS_PROJ_V == 1 && PGS_PROJ_DEPTH == 2 && PGS_PROJ_A == 3 &&
                      PGS_PROJ_B == 4 && PGS_PROJ_C == 5 && PGS_PROJ_OPACITY == 6 && PGS_PROJ_R == 7 &&
                      PGS_PROJ_G == 8 && PGS_PROJ_BLUE == 9 && PGS_PROJ_STRIDE == 16,
                  "record layout");
    float4* rec = reinterpret_cast<float4*>(out + (size_t)i * PGS_PROJ_STRIDE);
    const float A32 = (float)(G.c / G.det), B32 = (float)(-G.b / G.det), C32 = (float)(G.a / G.det);
    const float o32 = (float)o;
    float hx, hy;
    alpha_extent(A32, B32, C32, o32, hx, hy);
    rec[0] = make_float4((float)u, (float)v, (float)G.z, A32);
    rec[1] = make_float4(B32, C32, o32, (float)col[0]);
    rec[2] = make_float4((float)col[1], (float)col[2], hx, hy);
    rec[3] = make_float4(0.f, 0.f, 0.f, 0.f);
    radius[i] = (int)r;
    const uint32_t ix0 = (uint32_t)x0, ix1 = (uint32_t)x1, iy0 = (uint32_t)y0, iy1 = (uint32_t)y1;
    rect[i] = ix0 | (iy0 << 16);
    rect[(size_t)n + i] = ix1 | (iy1 << 16);
    touched[i] = (ix1 - ix0 + 1) * (iy1 - iy0 + 1);
}

template <int D>
__global__ __launch_bounds__(256) void k_project(const float* __restrict__ P, int n, CamD cam,
                                                 int tw, int th, int TX, int TY,
                                                 float* __restrict__ out, int* __restrict__ radius,
                                                 uint32_t* __restrict__ rect,
                                                 uint32_t* __restrict__ touched) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    Shape S3;
    shape_of(P, n, i, S3);
    project_view<D>(P, n, i, S3, cam, tw, th, TX, TY, out, radius, rect, touched);
}

// Up to kLaunchViews views per multi-view launch, cameras by value.
constexpr int kLaunchViews = 8;
struct LaunchViews {
    int nv, v0;  // views in this launch, index of the first
    CamD cam[kLaunchViews];
    int TX[kLaunchViews], TY[kLaunchViews];
};

// Every view of a launch for one Gaussian: the view-independent shape once,
// the parameters read once from HBM (the views re-read them from cache).
template <int D>
__global__ __launch_bounds__(256) void k_project_views(const float* __restrict__ P, int n, LaunchViews lv,
                                                       int tw, int th, float* __restrict__ out_all,
                                                       int* __restrict__ radius_all,
                                                       uint32_t* __restrict__ rect_all,
                                                       uint32_t* __restrict__ touched_all) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    Shape S3;
    shape_of(P, n, i, S3);
    for (int k = 0; k < lv.nv; ++k) {
        const size_t v = (size_t)(lv.v0 + k);
        project_view<D>(P, n, i, S3, lv.cam[k], tw, th, lv.TX[k], lv.TY[k], out_all + v * n * PGS_PROJ_STRIDE,
                        radius_all + v * n, rect_all + 2 * v * n, touched_all + v * n);
    }
}

// Backward: exact derivative of k_project's outputs (u, v, A, B, C, o, rgb)
// with every discrete decision frozen, accumulated into the canonical
// gradient rows.
// The gradient contributions of one view to Gaussian i's canonical rows,
// handed to acc(row, value) (float64).
template <int D, class Acc>
__device__ __forceinline__ void project_bwd_view(const float* __restrict__ P, int n, int i, const Shape& S3,
                                                 const CamD& cam, const float* __restrict__ g2d_row, Acc&& acc) {
    constexpr int K = (D + 1) * (D + 1);
    auto gin = [&](int f) { return (double)g2d_row[f]; };
    const double gu = gin(0), gv = gin(1), gA = gin(2), gB = gin(3), gC = gin(4), go = gin(5);
    const double gcol[3] = {gin(6), gin(7), gin(8)};

    double gmu[3], glog[3], gqraw[4];
    Geo G;
    view_geometry(P, n, i, S3, cam, G);
    const double a = G.a, b = G.b, c = G.c, det2 = G.det * G.det;
    // conic (A, B, C) = (c, -b, a) / det  ->  Sigma2D entries
    const double ga = (-c * c * gA + b * c * gB - b * b * gC) / det2;
    const double gb = (2.0 * b * c * gA - (a * c + b * b) * gB + 2.0 * a * b * gC) / det2;
    const double gc = (-b * b * gA + a * b * gB - a * a * gC) / det2;
    // symmetric 2x2 gradient of Sigma2D
    const double G00 = ga, G01 = 0.5 * gb, G11 = gc;
    const double* S = S3.Sig;
    double Sm[3][3] = {{S[0], S[1], S[2]}, {S[1], S[3], S[4]}, {S[2], S[4], S[5]}};
    // dL/dSigma = T^T G2 T (3x3 symmetric)
    double GS[3][3];
    for (int r = 0; r < 3; ++r)
        for (int q = 0; q < 3; ++q)
            GS[r][q] = G.T0[r] * (G00 * G.T0[q] + G01 * G.T1[q]) +
                       G.T1[r] * (G01 * G.T0[q] + G11 * G.T1[q]);
    // dL/dT = 2 G2 T Sigma (2x3)
    double TS0[3], TS1[3];
    for (int q = 0; q < 3; ++q) {
        TS0[q] = G.T0[0] * Sm[0][q] + G.T0[1] * Sm[1][q] + G.T0[2] * Sm[2][q];
        TS1[q] = G.T1[0] * Sm[0][q] + G.T1[1] * Sm[1][q] + G.T1[2] * Sm[2][q];
    }
    double dT0[3], dT1[3];
    for (int q = 0; q < 3; ++q) {
        dT0[q] = 2.0 * (G00 * TS0[q] + G01 * TS1[q]);
        dT1[q] = 2.0 * (G01 * TS0[q] + G11 * TS1[q]);
    }
    // T = J W: dL/dJ = dL/dT W^T; only J00, J02, J11, J12 are non-zero
    const double* W = cam.R;
    const double gJ00 = dT0[0] * W[0] + dT0[1] * W[1] + dT0[2] * W[2];
    const double gJ02 = dT0[0] * W[6] + dT0[1] * W[7] + dT0[2] * W[8];
    const double gJ11 = dT1[0] * W[3] + dT1[1] * W[4] + dT1[2] * W[5];
    const double gJ12 = dT1[0] * W[6] + dT1[1] * W[7] + dT1[2] * W[8];
    const double z = G.z, z2 = z * z;
    double gx = 0, gy = 0, gz = 0;
    // J00 = fx/z, J02 = -fx tx/z (tx = x/z unless clamped), same in y
    gz += -cam.fx / z2 * gJ00 - cam.fy / z2 * gJ11;
    gz += cam.fx * G.tx / z2 * gJ02 + cam.fy * G.ty / z2 * gJ12;
    if (!G.clx) {
        gx += -cam.fx / z2 * gJ02;
        gz += cam.fx * G.x / (z2 * z) * gJ02;
    }
    if (!G.cly) {
        gy += -cam.fy / z2 * gJ12;
        gz += cam.fy * G.y / (z2 * z) * gJ12;
    }
    // pixel mean
    gx += gu * cam.fx / z;
    gy += gv * cam.fy / z;
    gz += -gu * cam.fx * G.x / z2 - gv * cam.fy * G.y / z2;
    // x_c = W mu + t
    for (int k = 0; k < 3; ++k) gmu[k] = W[k] * gx + W[3 + k] * gy + W[6 + k] * gz;

    // Sigma = M M^T, M = R diag(s): dL/dM = 2 dL/dSigma M
    double M[3][3], gM[3][3];
    for (int r = 0; r < 3; ++r)
        for (int q = 0; q < 3; ++q) M[r][q] = S3.R[3 * r + q] * S3.s[q];
    for (int r = 0; r < 3; ++r)
        for (int q = 0; q < 3; ++q)
            gM[r][q] = 2.0 * (GS[r][0] * M[0][q] + GS[r][1] * M[1][q] + GS[r][2] * M[2][q]);
    double gR[9];
    for (int q = 0; q < 3; ++q) {
        double a_ = 0.0;
        for (int r = 0; r < 3; ++r) {
            a_ += gM[r][q] * S3.R[3 * r + q];
            gR[3 * r + q] = gM[r][q] * S3.s[q];
        }
        glog[q] = a_ * S3.s[q];
    }
    const double w = S3.qn[0], x = S3.qn[1], y = S3.qn[2], zq = S3.qn[3];
    double gq[4];
    gq[0] = 2.0 * (-zq * gR[1] + y * gR[2] + zq * gR[3] - x * gR[5] - y * gR[6] + x * gR[7]);
    gq[1] = 2.0 * (y * gR[1] + zq * gR[2] + y * gR[3] - 2.0 * x * gR[4] - w * gR[5] +
                   zq * gR[6] + w * gR[7] - 2.0 * x * gR[8]);
    gq[2] = 2.0 * (-2.0 * y * gR[0] + x * gR[1] + w * gR[2] + x * gR[3] + zq * gR[5] -
                   w * gR[6] + zq * gR[7] - 2.0 * y * gR[8]);
    gq[3] = 2.0 * (-2.0 * zq * gR[0] - w * gR[1] + x * gR[2] + w * gR[3] - 2.0 * zq * gR[4] +
                   y * gR[5] + x * gR[6] + y * gR[7]);
    const double dotq = gq[0] * w + gq[1] * x + gq[2] * y + gq[3] * zq;
    for (int k = 0; k < 4; ++k) gqraw[k] = (gq[k] - S3.qn[k] * dotq) / S3.qlen;
    // colour: c = max(0, sum_k Y_k(d) f_k + 1/2), d = unit(mu - campos)
    double d0 = prow(P, 0, n, i) - cam.campos[0];
    double d1 = prow(P, 1, n, i) - cam.campos[1];
    double d2 = prow(P, 2, n, i) - cam.campos[2];
    const double dl = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
    d0 /= dl; d1 /= dl; d2 /= dl;
    double Y[K];
    sh_eval<D>(d0, d1, d2, Y);
    double graw[3];
    for (int ch = 0; ch < 3; ++ch) {
        double c_ = 0.5;
        for (int k = 0; k < K; ++k) c_ += Y[k] * prow(P, 11 + 3 * k + ch, n, i);
        graw[ch] = c_ >= 0.0 ? gcol[ch] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) acc(11 + 3 * k + ch, Y[k] * graw[ch]);
    if (D >= 1) {
        double gd[3] = {0, 0, 0};
#pragma unroll
        for (int k = 1; k < K; ++k) {
            const double gy_k = prow(P, 11 + 3 * k, n, i) * graw[0] +
                                prow(P, 12 + 3 * k, n, i) * graw[1] +
                                prow(P, 13 + 3 * k, n, i) * graw[2];
            double dx, dy, dz;
            sh_grad_k(k, d0, d1, d2, dx, dy, dz);
            gd[0] += gy_k * dx;
            gd[1] += gy_k * dy;
            gd[2] += gy_k * dz;
        }
        const double dd = gd[0] * d0 + gd[1] * d1 + gd[2] * d2;
        gmu[0] += (gd[0] - d0 * dd) / dl;
        gmu[1] += (gd[1] - d1 * dd) / dl;
        gmu[2] += (gd[2] - d2 * dd) / dl;
    }
    const double o = 1.0 / (1.0 + exp(-prow(P, 10, n, i)));
#pragma unroll
    for (int k = 0; k < 3; ++k) acc(k, gmu[k]);
#pragma unroll
    for (int k = 0; k < 3; ++k) acc(3 + k, glog[k]);
#pragma unroll
    for (int k = 0; k < 4; ++k) acc(6 + k, gqraw[k]);
    acc(10, go * o * (1.0 - o));
}

template <int D>
__global__ __launch_bounds__(256) void k_project_bwd(const float* __restrict__ P, int n, CamD cam,
                                                     const int* __restrict__ radius,
                                                     const float* __restrict__ g2d,
                                                     float* __restrict__ grads) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || radius[i] == 0) return;
    Shape S3;
    shape_of(P, n, i, S3);
    project_bwd_view<D>(P, n, i, S3, cam, g2d + (size_t)i * PGS_GRAD2D_STRIDE, [&](int r, double g) {
        float* dst = &grads[(size_t)r * n + i];
        *dst = (float)((double)*dst + g);
    });
}

// Every view of a launch for one Gaussian, its canonical rows accumulated
// in registers: each view adds in float64 and rounds to float32, in view
// order, as launching the one-view kernel per view would; the rows are read
// and written once.
template <int D>
__global__ __launch_bounds__(256) void k_project_bwd_views(const float* __restrict__ P, int n, LaunchViews lv,
                                                           const int* __restrict__ radius_all,
                                                           const float* __restrict__ g2d_all,
                                                           float* __restrict__ grads) {
    constexpr int F = 11 + 3 * (D + 1) * (D + 1);
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    bool any = false;
    for (int k = 0; k < lv.nv; ++k) any |= radius_all[(size_t)(lv.v0 + k) * n + i] != 0;
    if (!any) return;
    float acc[F];
#pragma unroll
    for (int r = 0; r < F; ++r) acc[r] = grads[(size_t)r * n + i];
    Shape S3;
    shape_of(P, n, i, S3);
    for (int k = 0; k < lv.nv; ++k) {
        const size_t v = (size_t)(lv.v0 + k);
        if (radius_all[v * n + i] == 0) continue;
        // the parameter pointer made opaque per view: the parameters are
        // re-read (from cache) by every view instead of being held in
        // registers across the loop
        const float* Pv = P;
        asm volatile("" : "+s"(Pv));
        project_bwd_view<D>(Pv, n, i, S3, lv.cam[k], g2d_all + (v * n + i) * PGS_GRAD2D_STRIDE,
                            [&](int r, double g) { acc[r] = (float)((double)acc[r] + g); });
    }
#pragma unroll
    for (int r = 0; r < F; ++r) grads[(size_t)r * n + i] = acc[r];
}

}  // namespace

extern "C" pgs_status pgs_project(const float* params_dev, int32_t n, int32_t sh_degree,
                                  const pgs_camera* cam_host, int32_t tile_w, int32_t tile_h,
                                  float* proj_dev, int32_t* radius_dev, uint32_t* rect_dev,
                                  uint32_t* touched_dev, void* stream) {
    PGS_REQUIRE(n >= 0, "pgs_project: n < 0");
    PGS_REQUIRE(sh_degree >= 0 && sh_degree <= 3, "pgs_project: sh_degree %d", sh_degree);
    PGS_REQUIRE(cam_host != nullptr, "pgs_project: null camera");
    PGS_REQUIRE(cam_host->width > 0 && cam_host->height > 0 && tile_w > 0 && tile_h > 0,
                "pgs_project: bad image/tile size");
    const int TX = (cam_host->width + tile_w - 1) / tile_w;
    const int TY = (cam_host->height + tile_h - 1) / tile_h;
    PGS_REQUIRE(TX <= 65535 && TY <= 65535, "pgs_project: too many tiles");
    if (n == 0) return PGS_OK;
    PGS_REQUIRE(params_dev && proj_dev && radius_dev && rect_dev && touched_dev,
                "pgs_project: null pointer");
    const pgs::CamD cam = pgs::make_cam(*cam_host);
    const dim3 grid((n + 255) / 256), block(256);
    hipStream_t s = pgs::as_stream(stream);
    switch (sh_degree) {
        case 0: k_project<0><<<grid, block, 0, s>>>(params_dev, n, cam, tile_w, tile_h, TX, TY, proj_dev, radius_dev, rect_dev, touched_dev); break;
        case 1: k_project<1><<<grid, block, 0, s>>>(params_dev, n, cam, tile_w, tile_h, TX, TY, proj_dev, radius_dev, rect_dev, touched_dev); break;
        case 2: k_project<2><<<grid, block, 0, s>>>(params_dev, n, cam, tile_w, tile_h, TX, TY, proj_dev, radius_dev, rect_dev, touched_dev); break;
        default: k_project<3><<<grid, block, 0, s>>>(params_dev, n, cam, tile_w, tile_h, TX, TY, proj_dev, radius_dev, rect_dev, touched_dev); break;
    }
    PGS_CHECK_LAUNCH("pgs_project");
    return PGS_OK;
}

extern "C" pgs_status pgs_project_bwd(const float* params_dev, int32_t n, int32_t sh_degree,
                                      const pgs_camera* cam_host, const int32_t* radius_dev,
                                      const float* grad2d_dev, float* grads_dev, void* stream) {
    PGS_REQUIRE(n >= 0, "pgs_project_bwd: n < 0");
    PGS_REQUIRE(sh_degree >= 0 && sh_degree <= 3, "pgs_project_bwd: sh_degree %d", sh_degree);
    PGS_REQUIRE(cam_host != nullptr, "pgs_project_bwd: null camera");
    if (n == 0) return PGS_OK;
    PGS_REQUIRE(params_dev && radius_dev && grad2d_dev && grads_dev, "pgs_project_bwd: null pointer");
    const pgs::CamD cam = pgs::make_cam(*cam_host);
    const dim3 grid((n + 255) / 256), block(256);
    hipStream_t s = pgs::as_stream(stream);
    switch (sh_degree) {
        case 0: k_project_bwd<0><<<grid, block, 0, s>>>(params_dev, n, cam, radius_dev, grad2d_dev, grads_dev); break;
        case 1: k_project_bwd<1><<<grid, block, 0, s>>>(params_dev, n, cam, radius_dev, grad2d_dev, grads_dev); break;
        case 2: k_project_bwd<2><<<grid, block, 0, s>>>(params_dev, n, cam, radius_dev, grad2d_dev, grads_dev); break;
        default: k_project_bwd<3><<<grid, block, 0, s>>>(params_dev, n, cam, radius_dev, grad2d_dev, grads_dev); break;
    }
    PGS_CHECK_LAUNCH("pgs_project_bwd");
    return PGS_OK;
}

namespace {

// Cameras of views [v0, v0 + nv) of a batch, for one multi-view launch.
LaunchViews launch_views(const pgs_view_batch& vb, int v0, int nv) {
    LaunchViews lv{};
    lv.nv = nv;
    lv.v0 = v0;
    for (int k = 0; k < nv; ++k) {
        const pgs_camera& c = vb.cams[v0 + k];
        lv.cam[k] = pgs::make_cam(c);
        lv.TX[k] = (c.width + vb.tile_w - 1) / vb.tile_w;
        lv.TY[k] = (c.height + vb.tile_h - 1) / vb.tile_h;
    }
    return lv;
}

}  // namespace

extern "C" pgs_status pgs_project_views(const pgs_view_batch* views, const float* params_dev, int32_t n,
                                        int32_t sh_degree, float* proj_all_dev, int32_t* radius_all_dev,
                                        uint32_t* rect_all_dev, uint32_t* touched_all_dev, void* stream) {
    if (pgs_status st = pgs::check_views(views, "pgs_project_views")) return st;
    PGS_REQUIRE(n >= 0, "pgs_project_views: n < 0");
    PGS_REQUIRE(sh_degree >= 0 && sh_degree <= 3, "pgs_project_views: sh_degree %d", sh_degree);
    if (n == 0) return PGS_OK;
    PGS_REQUIRE(params_dev && proj_all_dev && radius_all_dev && rect_all_dev && touched_all_dev,
                "pgs_project_views: null pointer");
    const dim3 grid((n + 255) / 256), block(256);
    hipStream_t s = pgs::as_stream(stream);
    const int tw = views->tile_w, th = views->tile_h;
    for (int v0 = 0; v0 < views->n_views; v0 += kLaunchViews) {
        const LaunchViews lv = launch_views(*views, v0, min(kLaunchViews, views->n_views - v0));
        switch (sh_degree) {
            case 0: k_project_views<0><<<grid, block, 0, s>>>(params_dev, n, lv, tw, th, proj_all_dev, radius_all_dev, rect_all_dev, touched_all_dev); break;
            case 1: k_project_views<1><<<grid, block, 0, s>>>(params_dev, n, lv, tw, th, proj_all_dev, radius_all_dev, rect_all_dev, touched_all_dev); break;
            case 2: k_project_views<2><<<grid, block, 0, s>>>(params_dev, n, lv, tw, th, proj_all_dev, radius_all_dev, rect_all_dev, touched_all_dev); break;
            default: k_project_views<3><<<grid, block, 0, s>>>(params_dev, n, lv, tw, th, proj_all_dev, radius_all_dev, rect_all_dev, touched_all_dev); break;
        }
    }
    PGS_CHECK_LAUNCH("pgs_project_views");
    return PGS_OK;
}

extern "C" pgs_status pgs_project_bwd_views(const pgs_view_batch* views, const float* params_dev, int32_t n,
                                            int32_t sh_degree, const int32_t* radius_all_dev,
                                            const float* grad2d_all_dev, float* grads_dev, void* stream) {
    if (pgs_status st = pgs::check_views(views, "pgs_project_bwd_views")) return st;
    PGS_REQUIRE(n >= 0, "pgs_project_bwd_views: n < 0");
    PGS_REQUIRE(sh_degree >= 0 && sh_degree <= 3, "pgs_project_bwd_views: sh_degree %d", sh_degree);
    if (n == 0) return PGS_OK;
    PGS_REQUIRE(params_dev && radius_all_dev && grad2d_all_dev && grads_dev, "pgs_project_bwd_views: null pointer");
    const dim3 grid((n + 255) / 256), block(256);
    hipStream_t s = pgs::as_stream(stream);
    for (int v0 = 0; v0 < views->n_views; v0 += kLaunchViews) {
        const LaunchViews lv = launch_views(*views, v0, min(kLaunchViews, views->n_views - v0));
        switch (sh_degree) {
            case 0: k_project_bwd_views<0><<<grid, block, 0, s>>>(params_dev, n, lv, radius_all_dev, grad2d_all_dev, grads_dev); break;
            case 1: k_project_bwd_views<1><<<grid, block, 0, s>>>(params_dev, n, lv, radius_all_dev, grad2d_all_dev, grads_dev); break;
            case 2: k_project_bwd_views<2><<<grid, block, 0, s>>>(params_dev, n, lv, radius_all_dev, grad2d_all_dev, grads_dev); break;
            default: k_project_bwd_views<3><<<grid, block, 0, s>>>(params_dev, n, lv, radius_all_dev, grad2d_all_dev, grads_dev); break;
        }
    }
    PGS_CHECK_LAUNCH("pgs_project_bwd_views");
    return PGS_OK;
}
