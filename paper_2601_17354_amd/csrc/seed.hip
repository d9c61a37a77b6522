// KNN local surface statistics and disc-like covariance seeding (PocketGS
// Sec. "Prior-Conditioned Gaussian Parameterization").
//
// pgs_knn: exact brute force.  One lane per query point; the workgroup stages
// 256 candidate points at a time in LDS and every lane keeps its k best
// (squared distance, index) pairs sorted in registers.  Squared distances
// are ((dx*dx) + (dy*dy)) + (dz*dz) in float64 with contraction off, which
// fixes every rounding, so neighbour sets and their order are reproducible
// bit for bit.  Candidates arrive in increasing index order, so a candidate
// only displaces strictly larger distances: ties keep the smaller index.
//
// pgs_pca_seed: per point, in float64: covariance of the 16 neighbours about
// their centroid, cyclic Jacobi eigen-decomposition of the 3x3 matrix,
// normal = eigenvector of the smallest eigenvalue, s_t = mean distance to
// the 3 nearest, s_n = r_normal s_t; rotation [t1 t2 n] with the tangent
// basis of Duff et al. (2017) and its quaternion by Shepperd's method.
#include <math.h>

#include "common.hpp"

namespace {

constexpr int kKnnThreads = 256;
constexpr int kMaxK = 32;

__device__ __forceinline__ double sqdist(double qx, double qy, double qz, double px, double py, double pz) {
#pragma clang fp contract(off)
    const double dx = px - qx, dy = py - qy, dz = pz - qz;
    return (dx * dx + dy * dy) + dz * dz;
}

template <int K>
__global__ __launch_bounds__(kKnnThreads) void k_knn(const float* __restrict__ pts, int m,
                                                     int* __restrict__ nbr, double* __restrict__ d2out) {
    __shared__ float sp[3][kKnnThreads];
    const int q = blockIdx.x * kKnnThreads + threadIdx.x;
    const bool live = q < m;
    double qx = 0, qy = 0, qz = 0;
    if (live) {
        qx = pts[q];
        qy = pts[(size_t)m + q];
        qz = pts[2 * (size_t)m + q];
    }
    double bd[K];
    int bi[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        bd[k] = INFINITY;
        bi[k] = -1;
    }
    for (int base = 0; base < m; base += kKnnThreads) {
        const int c = base + threadIdx.x;
        __syncthreads();
        if (c < m) {
            sp[0][threadIdx.x] = pts[c];
            sp[1][threadIdx.x] = pts[(size_t)m + c];
            sp[2][threadIdx.x] = pts[2 * (size_t)m + c];
        }
        __syncthreads();
        const int nc = min(kKnnThreads, m - base);
        if (!live) continue;
        for (int j = 0; j < nc; ++j) {
            const int idx = base + j;
            if (idx == q) continue;
            const double d = sqdist(qx, qy, qz, sp[0][j], sp[1][j], sp[2][j]);
            if (!(d < bd[K - 1])) continue;
            // shift strictly larger entries down one slot (the last drops
            // out) and place d after every entry with distance <= d
            bool placed = false;
#pragma unroll
            for (int k = K - 1; k >= 0; --k) {
                if (!placed) {
                    if (k > 0 && bd[k - 1] > d) {
                        bd[k] = bd[k - 1];
                        bi[k] = bi[k - 1];
                    } else {
                        bd[k] = d;
                        bi[k] = idx;
                        placed = true;
                    }
                }
            }
        }
    }
    if (!live) return;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        nbr[(size_t)k * m + q] = bi[k];
        d2out[(size_t)k * m + q] = bd[k];
    }
}

// Eigen-decomposition of a symmetric 3x3 matrix by cyclic Jacobi rotations.
// On return A's diagonal holds the eigenvalues and V's columns the vectors.
__device__ void jacobi3(double A[3][3], double V[3][3]) {
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) V[r][c] = r == c ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 30; ++sweep) {
        const double off = fabs(A[0][1]) + fabs(A[0][2]) + fabs(A[1][2]);
        const double scale = fabs(A[0][0]) + fabs(A[1][1]) + fabs(A[2][2]);
        if (off <= 1e-300 || off <= 1e-18 * scale) break;
        for (int p = 0; p < 2; ++p)
            for (int q = p + 1; q < 3; ++q) {
                const double apq = A[p][q];
                if (apq == 0.0) continue;
                const double theta = (A[q][q] - A[p][p]) / (2.0 * apq);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                // A <- J^T A J with J the rotation in the (p, q) plane
                for (int k = 0; k < 3; ++k) {
                    const double akp = A[k][p], akq = A[k][q];
                    A[k][p] = c * akp - s * akq;
                    A[k][q] = s * akp + c * akq;
                }
                for (int k = 0; k < 3; ++k) {
                    const double apk = A[p][k], aqk = A[q][k];
                    A[p][k] = c * apk - s * aqk;
                    A[q][k] = s * apk + c * aqk;
                }
                for (int k = 0; k < 3; ++k) {
                    const double vkp = V[k][p], vkq = V[k][q];
                    V[k][p] = c * vkp - s * vkq;
                    V[k][q] = s * vkp + c * vkq;
                }
            }
    }
}

__global__ __launch_bounds__(256) void k_pca_seed(const float* __restrict__ pts, const float* __restrict__ col,
                                                  int m, const int* __restrict__ nbr,
                                                  const double* __restrict__ d2, int k, double r_normal,
                                                  float* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    constexpr int KN = 16, KS = 3;
    double P[KN][3];
    double cen[3] = {0, 0, 0};
    for (int j = 0; j < KN; ++j) {
        const int id = nbr[(size_t)j * m + i];
        for (int a = 0; a < 3; ++a) {
            P[j][a] = pts[(size_t)a * m + id];
            cen[a] += P[j][a];
        }
    }
    for (int a = 0; a < 3; ++a) cen[a] /= KN;
    double A[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int j = 0; j < KN; ++j) {
        const double d[3] = {P[j][0] - cen[0], P[j][1] - cen[1], P[j][2] - cen[2]};
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) A[a][b] += d[a] * d[b];
    }
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) A[a][b] /= KN;
    double V[3][3];
    jacobi3(A, V);
    int imin = 0;
    if (A[1][1] < A[imin][imin]) imin = 1;
    if (A[2][2] < A[imin][imin]) imin = 2;
    double nx = V[0][imin], ny = V[1][imin], nz = V[2][imin];
    const double nl = sqrt(nx * nx + ny * ny + nz * nz);
    nx /= nl; ny /= nl; nz /= nl;
    double st = 0.0;
    for (int j = 0; j < KS; ++j) st += sqrt(d2[(size_t)j * m + i]);
    st /= KS;
    const double sn = r_normal * st;
    // right-handed tangent frame (t1, t2, n), Duff et al. 2017
    const double sg = nz >= 0.0 ? 1.0 : -1.0;
    const double a = -1.0 / (sg + nz), b = nx * ny * a;
    const double t1[3] = {1.0 + sg * nx * nx * a, sg * b, -sg * nx};
    const double t2[3] = {b, sg + ny * ny * a, -ny};
    const double R[3][3] = {{t1[0], t2[0], nx}, {t1[1], t2[1], ny}, {t1[2], t2[2], nz}};
    // quaternion (w, x, y, z) of R, Shepperd's method
    double qw, qx, qy, qz;
    const double tr = R[0][0] + R[1][1] + R[2][2];
    if (tr >= R[0][0] && tr >= R[1][1] && tr >= R[2][2]) {
        qw = 0.5 * sqrt(1.0 + tr);
        qx = (R[2][1] - R[1][2]) / (4.0 * qw);
        qy = (R[0][2] - R[2][0]) / (4.0 * qw);
        qz = (R[1][0] - R[0][1]) / (4.0 * qw);
    } else if (R[0][0] >= R[1][1] && R[0][0] >= R[2][2]) {
        qx = 0.5 * sqrt(1.0 + R[0][0] - R[1][1] - R[2][2]);
        qw = (R[2][1] - R[1][2]) / (4.0 * qx);
        qy = (R[0][1] + R[1][0]) / (4.0 * qx);
        qz = (R[0][2] + R[2][0]) / (4.0 * qx);
    } else if (R[1][1] >= R[2][2]) {
        qy = 0.5 * sqrt(1.0 - R[0][0] + R[1][1] - R[2][2]);
        qw = (R[0][2] - R[2][0]) / (4.0 * qy);
        qx = (R[0][1] + R[1][0]) / (4.0 * qy);
        qz = (R[1][2] + R[2][1]) / (4.0 * qy);
    } else {
        qz = 0.5 * sqrt(1.0 - R[0][0] - R[1][1] + R[2][2]);
        qw = (R[1][0] - R[0][1]) / (4.0 * qz);
        qx = (R[0][2] + R[2][0]) / (4.0 * qz);
        qy = (R[1][2] + R[2][1]) / (4.0 * qz);
    }
    const double y00 = 0.28209479177387814;  // 1/(2 sqrt(pi))
    float vals[14];
    for (int a2 = 0; a2 < 3; ++a2) vals[a2] = pts[(size_t)a2 * m + i];
    vals[3] = (float)log(st);
    vals[4] = (float)log(st);
    vals[5] = (float)log(sn);
    vals[6] = (float)qw;
    vals[7] = (float)qx;
    vals[8] = (float)qy;
    vals[9] = (float)qz;
    vals[10] = (float)log(0.1 / 0.9);
    for (int c = 0; c < 3; ++c) vals[11 + c] = (float)(((double)col[(size_t)c * m + i] - 0.5) / y00);
    for (int r = 0; r < 14; ++r) out[(size_t)r * m + i] = vals[r];
}

}  // namespace

extern "C" pgs_status pgs_knn(const float* points_dev, int32_t m, int32_t k, int32_t* nbr_dev,
                              double* d2_dev, void* stream) {
    PGS_REQUIRE(k == 4 || k == 8 || k == 16 || k == kMaxK, "pgs_knn: k must be 4, 8, 16 or 32 (k=%d)", k);
    PGS_REQUIRE(m > k, "pgs_knn: need m > k (k=%d m=%d)", k, m);
    PGS_REQUIRE(points_dev && nbr_dev && d2_dev, "pgs_knn: null pointer");
    hipStream_t s = pgs::as_stream(stream);
    const dim3 grid((m + kKnnThreads - 1) / kKnnThreads), block(kKnnThreads);
    switch (k) {
        case 4: k_knn<4><<<grid, block, 0, s>>>(points_dev, m, nbr_dev, d2_dev); break;
        case 8: k_knn<8><<<grid, block, 0, s>>>(points_dev, m, nbr_dev, d2_dev); break;
        case 16: k_knn<16><<<grid, block, 0, s>>>(points_dev, m, nbr_dev, d2_dev); break;
        default: k_knn<kMaxK><<<grid, block, 0, s>>>(points_dev, m, nbr_dev, d2_dev); break;
    }
    PGS_CHECK_LAUNCH("pgs_knn");
    return PGS_OK;
}

extern "C" pgs_status pgs_pca_seed(const float* points_dev, const float* colours_dev, int32_t m,
                                   const int32_t* nbr_dev, const double* d2_dev, int32_t k, float r_normal,
                                   float* params_dev, void* stream) {
    PGS_REQUIRE(m > 16 && k >= 16, "pgs_pca_seed: need m > 16 and k >= 16");
    PGS_REQUIRE(r_normal > 0.f, "pgs_pca_seed: r_normal must be positive");
    PGS_REQUIRE(points_dev && colours_dev && nbr_dev && d2_dev && params_dev, "pgs_pca_seed: null pointer");
    k_pca_seed<<<(m + 255) / 256, 256, 0, pgs::as_stream(stream)>>>(points_dev, colours_dev, m, nbr_dev, d2_dev,
                                                                  k, (double)r_normal, params_dev);
    PGS_CHECK_LAUNCH("pgs_pca_seed");
    return PGS_OK;
}
