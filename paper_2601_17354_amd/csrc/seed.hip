// KNN local surface statistics and disc-like covariance seeding (PocketGS
// Sec. "Prior-Conditioned Gaussian Parameterization").
//
// pgs_knn: exact k nearest neighbours through a uniform grid.  The points'
// bounding box is cut into cubic cells (at most 128 along its longest side);
// points are counted per cell, the counts scanned into cell starts and the
// points' coordinates and indices gathered in cell order.  One lane per query
// (queries in cell order, so a wave searches neighbouring cells) visits the
// cells in shells of growing Chebyshev distance r around its own cell and
// keeps its k best (squared distance, index) pairs sorted in registers,
// ordered by distance and then index.  Every point of a cell r + 1 or more
// cells away is farther than r cell widths, so the search stops after shell
// r once the k-th distance is at most (r h)^2: no unvisited point can enter
// or tie.  Squared distances are ((dx*dx) + (dy*dy)) + (dz*dz) in float64
// with contraction off, which fixes every rounding, so the neighbour sets and
// their order equal a brute-force search with ties broken by the smaller
// index, bit for bit, whatever order the cells are visited in.
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

// Grid of a KNN search: cubic cells of width h from the box corner lo,
// dims[3] cells per axis (at most kGridMax).
constexpr int kGridMax = 128;
constexpr int kBoxBlocks = 256;

struct GridDesc {
    double lo[3];
    double h;
    int dims[3];
};

__device__ __forceinline__ int cell_axis(double v, double lo, double h, int dim) {
    int c = (int)floor((v - lo) / h);
    return c < 0 ? 0 : (c >= dim ? dim - 1 : c);
}

// Per-block partial bounding boxes: part[b][0..2] minima, [3..5] maxima.
__global__ __launch_bounds__(256) void k_box_partial(const float* __restrict__ pts, int m, float* __restrict__ part) {
    __shared__ float red[6][256];
    float mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x)
        for (int a = 0; a < 3; ++a) {
            const float v = pts[(size_t)a * m + i];
            mn[a] = fminf(mn[a], v);
            mx[a] = fmaxf(mx[a], v);
        }
    for (int a = 0; a < 3; ++a) {
        red[a][threadIdx.x] = mn[a];
        red[3 + a][threadIdx.x] = mx[a];
    }
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off)
            for (int a = 0; a < 3; ++a) {
                red[a][threadIdx.x] = fminf(red[a][threadIdx.x], red[a][threadIdx.x + off]);
                red[3 + a][threadIdx.x] = fmaxf(red[3 + a][threadIdx.x], red[3 + a][threadIdx.x + off]);
            }
        __syncthreads();
    }
    if (threadIdx.x < 6) part[blockIdx.x * 6 + threadIdx.x] = red[threadIdx.x][0];
}

// The grid from the partial boxes (every thread computes the same value).
__device__ GridDesc grid_of(const float* __restrict__ part) {
    float mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int b = 0; b < kBoxBlocks; ++b)
        for (int a = 0; a < 3; ++a) {
            mn[a] = fminf(mn[a], part[b * 6 + a]);
            mx[a] = fmaxf(mx[a], part[b * 6 + 3 + a]);
        }
    GridDesc g;
    double ext = 0.0;
    for (int a = 0; a < 3; ++a) ext = fmax(ext, (double)mx[a] - (double)mn[a]);
    g.h = ext > 0.0 ? ext / kGridMax : 1.0;
    for (int a = 0; a < 3; ++a) {
        g.lo[a] = mn[a];
        const int d = (int)floor(((double)mx[a] - (double)mn[a]) / g.h) + 1;
        g.dims[a] = d < 1 ? 1 : (d > kGridMax ? kGridMax : d);
    }
    return g;
}

__global__ __launch_bounds__(256) void k_cell_count(const float* __restrict__ pts, int m,
                                                    const float* __restrict__ part, uint32_t* __restrict__ counts,
                                                    uint32_t* __restrict__ cell_of) {
    __shared__ GridDesc sg;
    if (threadIdx.x == 0) sg = grid_of(part);
    __syncthreads();
    const GridDesc g = sg;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
        const int cx = cell_axis(pts[i], g.lo[0], g.h, g.dims[0]);
        const int cy = cell_axis(pts[(size_t)m + i], g.lo[1], g.h, g.dims[1]);
        const int cz = cell_axis(pts[2 * (size_t)m + i], g.lo[2], g.h, g.dims[2]);
        const uint32_t c = ((uint32_t)cz * g.dims[1] + cy) * g.dims[0] + cx;
        cell_of[i] = c;
        atomicAdd(&counts[c], 1u);
    }
}

// Exclusive scan of the cell counts into starts (one chunk of 4096 per
// workgroup; the chunk totals are added up by each workgroup itself).
constexpr int kCellScanItems = 4096;

__global__ __launch_bounds__(256) void k_cell_total(const uint32_t* __restrict__ counts, uint32_t n,
                                                    uint32_t* __restrict__ totals) {
    __shared__ uint32_t red[256];
    uint32_t s = 0;
    for (uint32_t i = blockIdx.x * kCellScanItems + threadIdx.x; i < min(n, (blockIdx.x + 1) * kCellScanItems);
         i += 256)
        s += counts[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) totals[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_cell_starts(const uint32_t* __restrict__ counts, uint32_t n,
                                                     const uint32_t* __restrict__ totals,
                                                     uint32_t* __restrict__ starts, uint32_t* __restrict__ cursor) {
    __shared__ uint32_t sc[256];
    __shared__ uint32_t s_before;
    uint32_t b = 0;
    for (uint32_t k = threadIdx.x; k < blockIdx.x; k += 256) b += totals[k];
    sc[threadIdx.x] = b;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int k = 0; k < 256; ++k) t += sc[k];
        s_before = t;
    }
    __syncthreads();
    // 16 consecutive cells per thread
    const uint32_t base = blockIdx.x * kCellScanItems + threadIdx.x * 16;
    uint32_t loc[16], sum = 0;
    for (int k = 0; k < 16; ++k) {
        loc[k] = base + k < n ? counts[base + k] : 0u;
        sum += loc[k];
    }
    sc[threadIdx.x] = sum;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const uint32_t add = threadIdx.x >= (unsigned)off ? sc[threadIdx.x - off] : 0u;
        __syncthreads();
        sc[threadIdx.x] += add;
        __syncthreads();
    }
    uint32_t run = s_before + sc[threadIdx.x] - sum;
    for (int k = 0; k < 16; ++k) {
        if (base + k < n) {
            starts[base + k] = run;
            cursor[base + k] = run;
        }
        run += loc[k];
    }
}

__global__ __launch_bounds__(256) void k_cell_end(const uint32_t* __restrict__ counts, uint32_t n,
                                                  uint32_t* __restrict__ starts) {
    if (blockIdx.x == 0 && threadIdx.x == 0) starts[n] = starts[n - 1] + counts[n - 1];
}

// Points in cell order (order inside a cell is arbitrary: the search's
// tie rule does not depend on it).
__global__ __launch_bounds__(256) void k_cell_scatter(const float* __restrict__ pts, int m,
                                                      const uint32_t* __restrict__ cell_of,
                                                      uint32_t* __restrict__ cursor, float4* __restrict__ sorted) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
        const uint32_t at = atomicAdd(&cursor[cell_of[i]], 1u);
        sorted[at] = make_float4(pts[i], pts[(size_t)m + i], pts[2 * (size_t)m + i], __int_as_float(i));
    }
}

template <int K>
__device__ __forceinline__ void knn_insert(double d, int idx, double (&bd)[K], int (&bi)[K]) {
    // (d, idx) enters when it precedes the last entry in (distance, index)
    // order; entries it precedes shift down one slot
    if (!(d < bd[K - 1] || (d == bd[K - 1] && idx < bi[K - 1]))) return;
    bool placed = false;
#pragma unroll
    for (int k = K - 1; k >= 0; --k) {
        if (!placed) {
            if (k > 0 && (bd[k - 1] > d || (bd[k - 1] == d && bi[k - 1] > idx))) {
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

template <int K>
__global__ __launch_bounds__(kKnnThreads) void k_knn_grid(const float4* __restrict__ sorted, int m,
                                                          const float* __restrict__ part,
                                                          const uint32_t* __restrict__ starts,
                                                          int* __restrict__ nbr, double* __restrict__ d2out) {
    __shared__ GridDesc sg;
    if (threadIdx.x == 0) sg = grid_of(part);
    __syncthreads();
    const GridDesc g = sg;
    const int j = blockIdx.x * kKnnThreads + threadIdx.x;
    if (j >= m) return;
    const float4 qp = sorted[j];
    const int q = __float_as_int(qp.w);
    const double qx = qp.x, qy = qp.y, qz = qp.z;
    const int cx = cell_axis(qx, g.lo[0], g.h, g.dims[0]);
    const int cy = cell_axis(qy, g.lo[1], g.h, g.dims[1]);
    const int cz = cell_axis(qz, g.lo[2], g.h, g.dims[2]);
    double bd[K];
    int bi[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        bd[k] = INFINITY;
        bi[k] = 0x7fffffff;
    }
    const int rmax = max(g.dims[0], max(g.dims[1], g.dims[2]));
    for (int r = 0; r <= rmax; ++r) {
        for (int dz = -r; dz <= r; ++dz) {
            const int z = cz + dz;
            if (z < 0 || z >= g.dims[2]) continue;
            for (int dy = -r; dy <= r; ++dy) {
                const int y = cy + dy;
                if (y < 0 || y >= g.dims[1]) continue;
                const bool face = dz == -r || dz == r || dy == -r || dy == r;
                // on the shell: every x of a face row, else only x = -r and x = +r
                for (int dx = -r; dx <= r; dx += (face || r == 0) ? 1 : 2 * r) {
                    const int x = cx + dx;
                    if (x < 0 || x >= g.dims[0]) continue;
                    const uint32_t c = ((uint32_t)z * g.dims[1] + y) * g.dims[0] + x;
                    const uint32_t e = starts[c + 1];
                    for (uint32_t t = starts[c]; t < e; ++t) {
                        const float4 p = sorted[t];
                        const int idx = __float_as_int(p.w);
                        if (idx == q) continue;
                        knn_insert<K>(sqdist(qx, qy, qz, p.x, p.y, p.z), idx, bd, bi);
                    }
                }
            }
        }
        // cells r + 1 or more away hold only points farther than r h
        const double reach = (double)r * g.h;
        if (bi[K - 1] != 0x7fffffff && bd[K - 1] <= reach * reach * (1.0 - 1e-12)) break;
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        nbr[(size_t)k * m + q] = bi[k];
        d2out[(size_t)k * m + q] = bd[k];
    }
}

// Workspace of pgs_knn for m points.
struct KnnWs {
    float* part;
    uint32_t* counts;
    uint32_t* starts;
    uint32_t* cursor;
    uint32_t* totals;
    uint32_t* cell_of;
    float4* sorted;
    size_t bytes;
};

constexpr uint32_t kGridCells = (uint32_t)kGridMax * kGridMax * kGridMax;

KnnWs knn_layout(void* base, int m) {
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    KnnWs w{};
    char* p = static_cast<char*>(base);
    size_t off = 0;
    w.part = reinterpret_cast<float*>(p + off); off += up((size_t)kBoxBlocks * 6 * 4);
    w.counts = reinterpret_cast<uint32_t*>(p + off); off += up((size_t)kGridCells * 4);
    w.starts = reinterpret_cast<uint32_t*>(p + off); off += up(((size_t)kGridCells + 1) * 4);
    w.cursor = reinterpret_cast<uint32_t*>(p + off); off += up((size_t)kGridCells * 4);
    w.totals = reinterpret_cast<uint32_t*>(p + off); off += up((size_t)(kGridCells / kCellScanItems + 1) * 4);
    w.cell_of = reinterpret_cast<uint32_t*>(p + off); off += up((size_t)m * 4);
    w.sorted = reinterpret_cast<float4*>(p + off); off += up((size_t)m * 16);
    w.bytes = off;
    return w;
}

__global__ void k_clear_cells(uint32_t* __restrict__ p, uint32_t n) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0u;
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

extern "C" size_t pgs_knn_workspace(int32_t m) { return knn_layout(nullptr, m > 0 ? m : 0).bytes; }

extern "C" pgs_status pgs_knn(const float* points_dev, int32_t m, int32_t k, int32_t* nbr_dev,
                              double* d2_dev, void* workspace_dev, size_t workspace_bytes, void* stream) {
    PGS_REQUIRE(k == 4 || k == 8 || k == 16 || k == kMaxK, "pgs_knn: k must be 4, 8, 16 or 32 (k=%d)", k);
    PGS_REQUIRE(m > k, "pgs_knn: need m > k (k=%d m=%d)", k, m);
    PGS_REQUIRE(points_dev && nbr_dev && d2_dev && workspace_dev, "pgs_knn: null pointer");
    const KnnWs w = knn_layout(workspace_dev, m);
    PGS_REQUIRE(workspace_bytes >= w.bytes, "pgs_knn: workspace %zu < %zu", workspace_bytes, w.bytes);
    hipStream_t s = pgs::as_stream(stream);
    const int gm = (m + 255) / 256 < 4096 ? (m + 255) / 256 : 4096;
    k_box_partial<<<kBoxBlocks, 256, 0, s>>>(points_dev, m, w.part);
    k_clear_cells<<<1024, 256, 0, s>>>(w.counts, kGridCells);
    k_cell_count<<<gm, 256, 0, s>>>(points_dev, m, w.part, w.counts, w.cell_of);
    const uint32_t chunks = (kGridCells + kCellScanItems - 1) / kCellScanItems;
    k_cell_total<<<chunks, 256, 0, s>>>(w.counts, kGridCells, w.totals);
    k_cell_starts<<<chunks, 256, 0, s>>>(w.counts, kGridCells, w.totals, w.starts, w.cursor);
    k_cell_end<<<1, 64, 0, s>>>(w.counts, kGridCells, w.starts);
    k_cell_scatter<<<gm, 256, 0, s>>>(points_dev, m, w.cell_of, w.cursor, w.sorted);
    const dim3 grid((m + kKnnThreads - 1) / kKnnThreads), block(kKnnThreads);
    switch (k) {
        case 4: k_knn_grid<4><<<grid, block, 0, s>>>(w.sorted, m, w.part, w.starts, nbr_dev, d2_dev); break;
        case 8: k_knn_grid<8><<<grid, block, 0, s>>>(w.sorted, m, w.part, w.starts, nbr_dev, d2_dev); break;
        case 16: k_knn_grid<16><<<grid, block, 0, s>>>(w.sorted, m, w.part, w.starts, nbr_dev, d2_dev); break;
        default: k_knn_grid<kMaxK><<<grid, block, 0, s>>>(w.sorted, m, w.part, w.starts, nbr_dev, d2_dev); break;
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
