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

constexpr int kKn = 16;

// The 16 neighbours of point i in float64 and their covariance about the
// neighbourhood centroid (PocketGS, equation for C_i).
__device__ void neighbourhood(const float* __restrict__ pts, int m, const int* __restrict__ nbr, int i,
                              double P[kKn][3], double A[3][3]) {
    double cen[3] = {0, 0, 0};
    for (int j = 0; j < kKn; ++j) {
        const int id = nbr[(size_t)j * m + i];
        for (int a = 0; a < 3; ++a) {
            P[j][a] = pts[(size_t)a * m + id];
            cen[a] += P[j][a];
        }
    }
    for (int a = 0; a < 3; ++a) cen[a] /= kKn;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) A[a][b] = 0.0;
    for (int j = 0; j < kKn; ++j) {
        const double d[3] = {P[j][0] - cen[0], P[j][1] - cen[1], P[j][2] - cen[2]};
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) A[a][b] += d[a] * d[b];
    }
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) A[a][b] /= kKn;
}

// Unit quaternion (w, x, y, z) of a rotation matrix, Shepperd's method: the
// branch follows the largest of the trace and the three diagonal entries.
__device__ void quat_of_rot(const double R[3][3], double q[4]) {
    const double tr = R[0][0] + R[1][1] + R[2][2];
    if (tr >= R[0][0] && tr >= R[1][1] && tr >= R[2][2]) {
        q[0] = 0.5 * sqrt(1.0 + tr);
        q[1] = (R[2][1] - R[1][2]) / (4.0 * q[0]);
        q[2] = (R[0][2] - R[2][0]) / (4.0 * q[0]);
        q[3] = (R[1][0] - R[0][1]) / (4.0 * q[0]);
    } else if (R[0][0] >= R[1][1] && R[0][0] >= R[2][2]) {
        q[1] = 0.5 * sqrt(1.0 + R[0][0] - R[1][1] - R[2][2]);
        q[0] = (R[2][1] - R[1][2]) / (4.0 * q[1]);
        q[2] = (R[0][1] + R[1][0]) / (4.0 * q[1]);
        q[3] = (R[0][2] + R[2][0]) / (4.0 * q[1]);
    } else if (R[1][1] >= R[2][2]) {
        q[2] = 0.5 * sqrt(1.0 - R[0][0] + R[1][1] - R[2][2]);
        q[0] = (R[0][2] - R[2][0]) / (4.0 * q[2]);
        q[1] = (R[0][1] + R[1][0]) / (4.0 * q[2]);
        q[3] = (R[1][2] + R[2][1]) / (4.0 * q[2]);
    } else {
        q[3] = 0.5 * sqrt(1.0 - R[0][0] - R[1][1] + R[2][2]);
        q[0] = (R[1][0] - R[0][1]) / (4.0 * q[3]);
        q[1] = (R[0][2] + R[2][0]) / (4.0 * q[3]);
        q[2] = (R[1][2] + R[2][1]) / (4.0 * q[3]);
    }
}

__device__ void rot_of_quat(const double qin[4], double R[3][3]) {
    const double n = sqrt(qin[0] * qin[0] + qin[1] * qin[1] + qin[2] * qin[2] + qin[3] * qin[3]);
    const double w = qin[0] / n, x = qin[1] / n, y = qin[2] / n, z = qin[3] / n;
    R[0][0] = 1 - 2 * (y * y + z * z); R[0][1] = 2 * (x * y - w * z); R[0][2] = 2 * (x * z + w * y);
    R[1][0] = 2 * (x * y + w * z); R[1][1] = 1 - 2 * (x * x + z * z); R[1][2] = 2 * (y * z - w * x);
    R[2][0] = 2 * (x * z - w * y); R[2][1] = 2 * (y * z + w * x); R[2][2] = 1 - 2 * (x * x + y * y);
}

__global__ __launch_bounds__(256) void k_pca_seed(const float* __restrict__ pts, const float* __restrict__ col,
                                                  int m, const int* __restrict__ nbr,
                                                  const double* __restrict__ d2, int k, double r_normal,
                                                  float* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    constexpr int KS = 3;
    double P[kKn][3], A[3][3];
    neighbourhood(pts, m, nbr, i, P, A);
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
    double q[4];
    quat_of_rot(R, q);
    const double y00 = 0.28209479177387814;  // 1/(2 sqrt(pi))
    float vals[14];
    for (int a2 = 0; a2 < 3; ++a2) vals[a2] = pts[(size_t)a2 * m + i];
    vals[3] = (float)log(st);
    vals[4] = (float)log(st);
    vals[5] = (float)log(sn);
    for (int c = 0; c < 4; ++c) vals[6 + c] = (float)q[c];
    vals[10] = (float)log(0.1 / 0.9);
    for (int c = 0; c < 3; ++c) vals[11 + c] = (float)(((double)col[(size_t)c * m + i] - 0.5) / y00);
    for (int r = 0; r < 14; ++r) out[(size_t)r * m + i] = vals[r];
}

// Features of the seeding network for point i.  Frame R = [e1 e2 e3]:
// eigenvectors of C_i for the largest and middle eigenvalue, each signed so
// that the third moment of the offsets p_k - p_i along it is >= 0, and
// e3 = e1 x e2.  x = offsets in the frame / s_t (16 x 3), R^T C_i R / s_t^2
// (3 x 3), seven zeros.  base = R (row-major), plain-seed log-scales,
// quaternion of R.
__global__ __launch_bounds__(256) void k_mlp_features(const float* __restrict__ pts, int m,
                                                      const int* __restrict__ nbr,
                                                      const double* __restrict__ d2, double r_normal,
                                                      float* __restrict__ x, float* __restrict__ base) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    double P[kKn][3], A[3][3], C[3][3], V[3][3];
    neighbourhood(pts, m, nbr, i, P, A);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) C[a][b] = A[a][b];
    jacobi3(A, V);
    int ord[3] = {0, 1, 2};   // eigenvalue indices, largest first
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2 - a; ++b)
            if (A[ord[b + 1]][ord[b + 1]] > A[ord[b]][ord[b]]) {
                const int t = ord[b];
                ord[b] = ord[b + 1];
                ord[b + 1] = t;
            }
    const double p[3] = {pts[i], pts[(size_t)m + i], pts[2 * (size_t)m + i]};
    for (int j = 0; j < kKn; ++j)
        for (int a = 0; a < 3; ++a) P[j][a] -= p[a];   // offsets from the point
    double e[3][3];
    for (int c = 0; c < 2; ++c) {
        const int col = ord[c];
        const double nl = sqrt(V[0][col] * V[0][col] + V[1][col] * V[1][col] + V[2][col] * V[2][col]);
        double v[3] = {V[0][col] / nl, V[1][col] / nl, V[2][col] / nl};
        double m3 = 0.0;
        for (int j = 0; j < kKn; ++j) {
            const double d = P[j][0] * v[0] + P[j][1] * v[1] + P[j][2] * v[2];
            m3 += d * d * d;
        }
        const double sg = m3 < 0.0 ? -1.0 : 1.0;
        for (int a = 0; a < 3; ++a) e[c][a] = sg * v[a];
    }
    e[2][0] = e[0][1] * e[1][2] - e[0][2] * e[1][1];
    e[2][1] = e[0][2] * e[1][0] - e[0][0] * e[1][2];
    e[2][2] = e[0][0] * e[1][1] - e[0][1] * e[1][0];
    double st = 0.0;
    for (int j = 0; j < 3; ++j) st += sqrt(d2[(size_t)j * m + i]);
    st /= 3.0;
    float* xr = x + (size_t)i * 64;
    for (int j = 0; j < kKn; ++j)
        for (int c = 0; c < 3; ++c)
            xr[3 * j + c] = (float)((P[j][0] * e[c][0] + P[j][1] * e[c][1] + P[j][2] * e[c][2]) / st);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double v = 0.0;
            for (int u = 0; u < 3; ++u)
                for (int w = 0; w < 3; ++w) v += e[a][u] * C[u][w] * e[b][w];
            xr[48 + 3 * a + b] = (float)(v / (st * st));
        }
    for (int k = 57; k < 64; ++k) xr[k] = 0.f;
    double R[3][3];
    for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c) R[a][c] = e[c][a];
    double q[4];
    quat_of_rot(R, q);
    float* br = base + (size_t)i * 16;
    for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c) br[3 * a + c] = (float)R[a][c];
    br[9] = (float)log(st);
    br[10] = (float)log(st);
    br[11] = (float)log(r_normal * st);
    for (int c = 0; c < 4; ++c) br[12 + c] = (float)q[c];
}

// Training target of Gaussian i: log S = R diag(2 s) R^T (6 entries), logit.
__global__ __launch_bounds__(256) void k_seed_targets(const float* __restrict__ params, int n,
                                                      float* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double q[4], R[3][3], s2[3];
    for (int c = 0; c < 4; ++c) q[c] = params[(size_t)(6 + c) * n + i];
    for (int c = 0; c < 3; ++c) s2[c] = 2.0 * (double)params[(size_t)(3 + c) * n + i];
    rot_of_quat(q, R);
    auto M = [&](int a, int b) { return R[a][0] * s2[0] * R[b][0] + R[a][1] * s2[1] * R[b][1] + R[a][2] * s2[2] * R[b][2]; };
    float* o = out + (size_t)i * 8;
    o[0] = (float)M(0, 0);
    o[1] = (float)M(1, 1);
    o[2] = (float)M(2, 2);
    o[3] = (float)M(0, 1);
    o[4] = (float)M(0, 2);
    o[5] = (float)M(1, 2);
    o[6] = params[(size_t)10 * n + i];
    o[7] = 0.f;
}

// Seed from network outputs y with the fall back to the plain seed (pca
// columns): y not finite, |q_out| < 1e-6, a |d log-scale| > 2, or the axis
// of the smallest predicted scale more than 60 degrees from the plain
// normal (e3).  `pca` and `out` may be the same buffer.
__global__ __launch_bounds__(256) void k_seed_apply(const float* __restrict__ y, const float* __restrict__ base,
                                                    const float* pca, int m, float* out,
                                                    uint8_t* __restrict__ flags, uint32_t* __restrict__ count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    bool fb = false;
    if (i < m) {
        float vals[14];
        for (int r = 0; r < 14; ++r) vals[r] = pca[(size_t)r * m + i];
        double Y[8];
        for (int k = 0; k < 8; ++k) {
            const float v = y[(size_t)i * 8 + k];
            fb = fb || !isfinite(v);
            Y[k] = v;
        }
        const double qn = fb ? 0.0 : sqrt(Y[3] * Y[3] + Y[4] * Y[4] + Y[5] * Y[5] + Y[6] * Y[6]);
        fb = fb || qn < 1e-6;
        if (!fb) {
            double dl = 0.0;
            for (int k = 0; k < 3; ++k) dl = fmax(dl, fabs(Y[k]));
            double Ro[3][3], s[3];
            const double qo[4] = {Y[3] / qn, Y[4] / qn, Y[5] / qn, Y[6] / qn};
            rot_of_quat(qo, Ro);
            for (int k = 0; k < 3; ++k) s[k] = (double)base[(size_t)i * 16 + 9 + k] + Y[k];
            int kmin = 0;
            if (s[1] < s[kmin]) kmin = 1;
            if (s[2] < s[kmin]) kmin = 2;
            // (Rb Ro e_kmin) . (Rb e3) = (Ro e_kmin) . e3 = Ro[2][kmin]
            const double c = fabs(Ro[2][kmin]);
            fb = dl > 2.0 || c < 0.5;
            if (!fb) {
                double qb[4];
                for (int k = 0; k < 4; ++k) qb[k] = base[(size_t)i * 16 + 12 + k];
                const double w = qb[0] * qo[0] - qb[1] * qo[1] - qb[2] * qo[2] - qb[3] * qo[3];
                const double qx = qb[0] * qo[1] + qo[0] * qb[1] + qb[2] * qo[3] - qb[3] * qo[2];
                const double qy = qb[0] * qo[2] + qo[0] * qb[2] + qb[3] * qo[1] - qb[1] * qo[3];
                const double qz = qb[0] * qo[3] + qo[0] * qb[3] + qb[1] * qo[2] - qb[2] * qo[1];
                for (int k = 0; k < 3; ++k) vals[3 + k] = (float)s[k];
                vals[6] = (float)w;
                vals[7] = (float)qx;
                vals[8] = (float)qy;
                vals[9] = (float)qz;
                vals[10] = (float)(log(1.0 / 9.0) + Y[7]);
            }
        }
        for (int r = 0; r < 14; ++r) out[(size_t)r * m + i] = vals[r];
        if (flags) flags[i] = fb ? 1 : 0;
    }
    const unsigned long long b = __ballot(fb);
    if (count && (threadIdx.x & 63) == 0 && b) atomicAdd(count, (uint32_t)__popcll(b));
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

extern "C" pgs_status pgs_mlp_features(const float* points_dev, int32_t m, const int32_t* nbr_dev,
                                       const double* d2_dev, int32_t k, float r_normal, float* x_dev,
                                       float* base_dev, void* stream) {
    PGS_REQUIRE(m > 16 && k >= 16, "pgs_mlp_features: need m > 16 and k >= 16");
    PGS_REQUIRE(r_normal > 0.f, "pgs_mlp_features: r_normal must be positive");
    PGS_REQUIRE(points_dev && nbr_dev && d2_dev && x_dev && base_dev, "pgs_mlp_features: null pointer");
    k_mlp_features<<<(m + 255) / 256, 256, 0, pgs::as_stream(stream)>>>(points_dev, m, nbr_dev, d2_dev,
                                                                      (double)r_normal, x_dev, base_dev);
    PGS_CHECK_LAUNCH("pgs_mlp_features");
    return PGS_OK;
}

extern "C" pgs_status pgs_seed_targets(const float* params_dev, int32_t n, float* targets_dev, void* stream) {
    PGS_REQUIRE(n >= 0, "pgs_seed_targets: n must be >= 0");
    if (n == 0) return PGS_OK;
    PGS_REQUIRE(params_dev && targets_dev, "pgs_seed_targets: null pointer");
    k_seed_targets<<<(n + 255) / 256, 256, 0, pgs::as_stream(stream)>>>(params_dev, n, targets_dev);
    PGS_CHECK_LAUNCH("pgs_seed_targets");
    return PGS_OK;
}

extern "C" pgs_status pgs_seed_apply(const float* y_dev, const float* base_dev, const float* pca_params_dev,
                                     int32_t m, float* params_dev, uint8_t* fallback_dev,
                                     uint32_t* fallback_count_dev, void* stream) {
    PGS_REQUIRE(m >= 0, "pgs_seed_apply: m must be >= 0");
    if (m == 0) return PGS_OK;
    PGS_REQUIRE(y_dev && base_dev && pca_params_dev && params_dev, "pgs_seed_apply: null pointer");
    k_seed_apply<<<(m + 255) / 256, 256, 0, pgs::as_stream(stream)>>>(y_dev, base_dev, pca_params_dev, m,
                                                                    params_dev, fallback_dev, fallback_count_dev);
    PGS_CHECK_LAUNCH("pgs_seed_apply");
    return PGS_OK;
}
