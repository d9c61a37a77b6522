// Robust bundle adjustment with the reduced camera system (PocketGS
// subsection "GPU-Native Global BA as Mobile MAP Refinement": the robustified
// reprojection objective of equation ba_obj, scale-aware gauge fixing, and
// the Schur complement over the block-diagonal point blocks).
//
// Everything is float64.  One Levenberg-Marquardt step (pgs_ba_step):
//   k_ba_points   one thread per point, over its observations: residual,
//                 Huber weight, Jacobians; the point block H_pp + lambda
//                 diag(H_pp) inverted in place (3x3, adjugate), v = H_pp^-1 b_p,
//                 and per observation the pose-point block H_tp (6x3) and the
//                 observation's pose block and gradient (21 + 6 values);
//   k_ba_cameras  16 workgroups per camera, each over a slice of its
//                 observations: partial row blocks of the reduced system
//                 S = H_tt - H_tp H_pp^-1 H_pt (its blocks (i, k), k <= i:
//                 the solve reads the lower triangle) and g = b_t - H_tp v
//                 accumulated in LDS over every pair of observations that
//                 share a point (float64 LDS atomics); the first slice adds
//                 the camera's damped pose block and gradient, summed over
//                 its observations in a fixed order; k_ba_rows sums the
//                 slices in order;
//   k_ba_solve /  the gauge-free rows and columns of S (camera 0's six
//   k_ba_syrk     parameters and camera 1's centre coordinate along the gauge
//                 axis removed), a panel-blocked Cholesky (each panel
//                 factored by one workgroup in LDS, the right-hand side
//                 carried as an extra row so the forward substitution comes
//                 with the factor; the trailing update over many
//                 workgroups), and the blocked back substitution -> the
//                 pose step;
//   k_ba_backsub  one thread per point: dP = v - H_pp^-1 sum H_tp^T dt.
// The cost (sum of Huber terms) is reduced per block in a fixed order.
#include <math.h>

#include "common.hpp"

namespace {

constexpr int kCamThreads = 256;
constexpr int kSolveThreads = 1024;
constexpr int kCostThreads = 256;

// Per-observation record in the workspace: H_tp (6x3 row-major), then the
// observation's pose block (upper triangle of 6x6, row-major, 21 values)
// and its gradient contribution (6).
constexpr int kObsRec = 18 + 21 + 6;
// Per-point record: damped H_pp^-1 (3x3 row-major) and v (3).
constexpr int kPtRec = 12;

struct Obs {
    double r[2];        // residual
    double w;           // Huber weight
    double Jt[2][6];    // d r / d(dphi, dc)
    double Jp[2][3];    // d r / dP
};

__device__ __forceinline__ void observe(const pgs_ba_problem& pb, const double* __restrict__ rot,
                                        const double* __restrict__ centre, const double* __restrict__ pts,
                                        int o, int j, Obs& ob) {
    const int i = (int)pb.obs_cam_dev[o];
    const double* R = rot + 9 * (size_t)i;
    const double d0 = pts[3 * (size_t)j] - centre[3 * i], d1 = pts[3 * (size_t)j + 1] - centre[3 * i + 1],
                 d2 = pts[3 * (size_t)j + 2] - centre[3 * i + 2];
    const double x0 = R[0] * d0 + R[1] * d1 + R[2] * d2;
    const double x1 = R[3] * d0 + R[4] * d1 + R[5] * d2;
    const double x2 = R[6] * d0 + R[7] * d1 + R[8] * d2;
    const double iz = 1.0 / x2;
    ob.r[0] = pb.fx * x0 * iz + pb.cx - pb.obs_uv_dev[2 * (size_t)o];
    ob.r[1] = pb.fy * x1 * iz + pb.cy - pb.obs_uv_dev[2 * (size_t)o + 1];
    const double s = ob.r[0] * ob.r[0] + ob.r[1] * ob.r[1];
    const double nrm = sqrt(s);
    ob.w = nrm <= pb.huber_delta ? 1.0 : pb.huber_delta / nrm;
    // d pi / d x
    const double a00 = pb.fx * iz, a02 = -pb.fx * x0 * iz * iz;
    const double a11 = pb.fy * iz, a12 = -pb.fy * x1 * iz * iz;
    // A R (2x3): d r / dP; d r / dc = -A R; d r / ddphi = -A R [d]x
    double AR[2][3];
    for (int k = 0; k < 3; ++k) {
        AR[0][k] = a00 * R[k] + a02 * R[6 + k];
        AR[1][k] = a11 * R[3 + k] + a12 * R[6 + k];
    }
    for (int r = 0; r < 2; ++r) {
        // (A R) [d]x with [d]x = [[0,-d2,d1],[d2,0,-d0],[-d1,d0,0]]
        const double m0 = AR[r][1] * d2 - AR[r][2] * d1;
        const double m1 = -AR[r][0] * d2 + AR[r][2] * d0;
        const double m2 = AR[r][0] * d1 - AR[r][1] * d0;
        ob.Jt[r][0] = -m0;
        ob.Jt[r][1] = -m1;
        ob.Jt[r][2] = -m2;
        for (int k = 0; k < 3; ++k) {
            ob.Jt[r][3 + k] = -AR[r][k];
            ob.Jp[r][k] = AR[r][k];
        }
    }
}

__device__ __forceinline__ int tri6(int a, int b) {  // index of (a, b), a <= b, in the 6x6 upper triangle
    return a * 6 - a * (a - 1) / 2 + (b - a);
}

__global__ __launch_bounds__(256) void k_ba_points(pgs_ba_problem pb, const double* __restrict__ rot,
                                                   const double* __restrict__ centre,
                                                   const double* __restrict__ pts, double lam,
                                                   double* __restrict__ obs_rec, double* __restrict__ pt_rec) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= pb.n_points) return;
    double Hp[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, bp[3] = {0, 0, 0};
    const uint32_t o0 = pb.point_start_dev[j], o1 = pb.point_start_dev[j + 1];
    for (uint32_t o = o0; o < o1; ++o) {
        Obs ob;
        observe(pb, rot, centre, pts, (int)o, j, ob);
        double* rec = obs_rec + (size_t)o * kObsRec;
        for (int a = 0; a < 3; ++a) {
            for (int b = 0; b < 3; ++b) Hp[a][b] += ob.w * (ob.Jp[0][a] * ob.Jp[0][b] + ob.Jp[1][a] * ob.Jp[1][b]);
            bp[a] -= ob.w * (ob.Jp[0][a] * ob.r[0] + ob.Jp[1][a] * ob.r[1]);
        }
        for (int a = 0; a < 6; ++a)
            for (int b = 0; b < 3; ++b)
                rec[3 * a + b] = ob.w * (ob.Jt[0][a] * ob.Jp[0][b] + ob.Jt[1][a] * ob.Jp[1][b]);
        for (int a = 0; a < 6; ++a) {
            for (int b = a; b < 6; ++b)
                rec[18 + tri6(a, b)] = ob.w * (ob.Jt[0][a] * ob.Jt[0][b] + ob.Jt[1][a] * ob.Jt[1][b]);
            rec[39 + a] = -ob.w * (ob.Jt[0][a] * ob.r[0] + ob.Jt[1][a] * ob.r[1]);
        }
    }
    // damped point block and its inverse (adjugate / determinant)
    for (int a = 0; a < 3; ++a) Hp[a][a] += lam * Hp[a][a];
    const double c00 = Hp[1][1] * Hp[2][2] - Hp[1][2] * Hp[2][1];
    const double c01 = Hp[1][2] * Hp[2][0] - Hp[1][0] * Hp[2][2];
    const double c02 = Hp[1][0] * Hp[2][1] - Hp[1][1] * Hp[2][0];
    const double det = Hp[0][0] * c00 + Hp[0][1] * c01 + Hp[0][2] * c02;
    const double id = 1.0 / det;
    double Ai[3][3];
    Ai[0][0] = c00 * id;
    Ai[1][0] = c01 * id;
    Ai[2][0] = c02 * id;
    Ai[0][1] = (Hp[0][2] * Hp[2][1] - Hp[0][1] * Hp[2][2]) * id;
    Ai[1][1] = (Hp[0][0] * Hp[2][2] - Hp[0][2] * Hp[2][0]) * id;
    Ai[2][1] = (Hp[0][1] * Hp[2][0] - Hp[0][0] * Hp[2][1]) * id;
    Ai[0][2] = (Hp[0][1] * Hp[1][2] - Hp[0][2] * Hp[1][1]) * id;
    Ai[1][2] = (Hp[0][2] * Hp[1][0] - Hp[0][0] * Hp[1][2]) * id;
    Ai[2][2] = (Hp[0][0] * Hp[1][1] - Hp[0][1] * Hp[1][0]) * id;
    double* pr = pt_rec + (size_t)j * kPtRec;
    for (int a = 0; a < 3; ++a) {
        for (int b = 0; b < 3; ++b) pr[3 * a + b] = Ai[a][b];
        pr[9 + a] = Ai[a][0] * bp[0] + Ai[a][1] * bp[1] + Ai[a][2] * bp[2];
    }
}

__device__ __forceinline__ double wave_sum_f64(double v) {
    for (int k = 32; k > 0; k >>= 1) {
        const long long b = __double_as_longlong(v);
        const int lo = __shfl_xor((int)(b & 0xffffffffll), k), hi = __shfl_xor((int)(b >> 32), k);
        v += __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
    }
    return v;
}

// Workgroup (i, s): split s of camera i's observations.  Partial row block
// i of the reduced system over those observations (pair products of
// observations that share a point, float64 LDS atomics); split 0 also adds
// the camera's damped pose block and gradient, summed over all its
// observations in a fixed order.  Partials go to part[i][s][6 n6 + 6].
constexpr int kCamSplit = 16;

__global__ __launch_bounds__(kCamThreads) void k_ba_cameras(pgs_ba_problem pb, double lam,
                                                            const double* __restrict__ obs_rec,
                                                            const double* __restrict__ pt_rec,
                                                            double* __restrict__ part) {
    extern __shared__ double lds[];
    constexpr int NW = kCamThreads / 64;
    const int i = blockIdx.x, split = blockIdx.y, t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int n6 = 6 * pb.n_cams;
    double* row = lds;                 // [6][n6]
    double* wsum = row + 6 * n6;       // [NW][27] per-wave pose block sums
    double* gi = wsum + NW * 27;       // [6]
    const uint32_t c0 = pb.cam_start_dev[i], c1 = pb.cam_start_dev[i + 1];
    for (int e = t; e < 6 * n6; e += kCamThreads) row[e] = 0.0;
    if (t < 6) gi[t] = 0.0;
    if (split == 0) {
        // pose block and gradient of camera i: per-lane sums over its
        // observations, then wave sums and the waves' totals in a fixed order
        double acc[27];
        for (int k = 0; k < 27; ++k) acc[k] = 0.0;
        for (uint32_t q = c0 + t; q < c1; q += kCamThreads) {
            const double* rec = obs_rec + (size_t)pb.cam_obs_dev[q] * kObsRec + 18;
            for (int k = 0; k < 27; ++k) acc[k] += rec[k];
        }
        for (int k = 0; k < 27; ++k) {
            const double v = wave_sum_f64(acc[k]);
            if (lane == 0) wsum[wv * 27 + k] = v;
        }
        __syncthreads();
        if (t < 36) {
            const int a = t / 6, b = t % 6, k = a <= b ? tri6(a, b) : tri6(b, a);
            double h = 0.0;
            for (int w = 0; w < NW; ++w) h += wsum[w * 27 + k];
            if (a == b) h += lam * h;
            row[a * n6 + 6 * i + b] = h;
        }
        if (t < 6) {
            double h = 0.0;
            for (int w = 0; w < NW; ++w) h += wsum[w * 27 + 21 + t];
            gi[t] = h;
        }
    }
    __syncthreads();
    // - H_tp H_pp^-1 H_pt and - H_tp v over this split of camera i's observations
    const uint32_t chunk = (c1 - c0 + kCamSplit - 1) / kCamSplit;
    const uint32_t q0 = c0 + split * chunk, q1 = min(c1, q0 + chunk);
    double gl[6] = {0, 0, 0, 0, 0, 0};  // this lane's share of - H_tp v
    for (uint32_t q = q0 + t; q < q1; q += kCamThreads) {
        const uint32_t o = pb.cam_obs_dev[q];
        const uint32_t j = pb.obs_pt_dev[o];
        const double* Htp = obs_rec + (size_t)o * kObsRec;
        const double* pr = pt_rec + (size_t)j * kPtRec;
        double T[6][3];  // H_tp(i, j) H_pp(j)^-1
        for (int a = 0; a < 6; ++a)
            for (int b = 0; b < 3; ++b)
                T[a][b] = Htp[3 * a] * pr[b] + Htp[3 * a + 1] * pr[3 + b] + Htp[3 * a + 2] * pr[6 + b];
        for (int a = 0; a < 6; ++a) gl[a] -= Htp[3 * a] * pr[9] + Htp[3 * a + 1] * pr[10] + Htp[3 * a + 2] * pr[11];
        // the track is walked from a lane-dependent start so that the lanes
        // of a wave add into different camera blocks at the same time
        const uint32_t s0 = pb.point_start_dev[j], nt = pb.point_start_dev[j + 1] - s0;
        for (uint32_t r = 0; r < nt; ++r) {
            uint32_t o2 = s0 + r + (uint32_t)lane % nt;
            if (o2 >= s0 + nt) o2 -= nt;
            const int k = (int)pb.obs_cam_dev[o2];
            if (k > i) continue;  // the solve reads the lower triangle only
            const double* H2 = obs_rec + (size_t)o2 * kObsRec;
            for (int a = 0; a < 6; ++a)
                for (int b = 0; b < 6; ++b)
                    atomicAdd(&row[a * n6 + 6 * k + b],
                              -(T[a][0] * H2[3 * b] + T[a][1] * H2[3 * b + 1] + T[a][2] * H2[3 * b + 2]));
        }
    }
    for (int a = 0; a < 6; ++a) {
        const double v = wave_sum_f64(gl[a]);
        if (lane == 0) atomicAdd(&gi[a], v);
    }
    __syncthreads();
    double* out = part + ((size_t)i * kCamSplit + split) * (6 * n6 + 6);
    for (int e = t; e < 6 * n6; e += kCamThreads) out[e] = row[e];
    if (t < 6) out[6 * n6 + t] = gi[t];
}

// Row blocks of S and g: the camera splits' partials summed in split order.
__global__ __launch_bounds__(256) void k_ba_rows(int n_cams, const double* __restrict__ part,
                                                 double* __restrict__ S, double* __restrict__ g) {
    const int n6 = 6 * n_cams, per = 6 * n6 + 6;
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (size_t)n_cams * per) return;
    const int i = (int)(e / per), k = (int)(e - (size_t)i * per);
    double acc = 0.0;
    for (int sp = 0; sp < kCamSplit; ++sp) acc += part[((size_t)i * kCamSplit + sp) * per + k];
    if (k < 6 * n6) S[(size_t)(6 * i) * n6 + k] = acc;
    else g[6 * i + (k - 6 * n6)] = acc;
}

// Free (moving) pose parameter k of nf: skips camera 0's six and camera 1's
// centre coordinate along the gauge axis.
__device__ __forceinline__ int free_param(int k, int gauge_axis) {
    const int p = k + 6;                        // past camera 0
    return p >= 9 + gauge_axis ? p + 1 : p;     // past camera 1's fixed centre coordinate
}

// Broadcast of a double from lane `src` of the wave.
__device__ __forceinline__ double lane_bcast(double v, int src) {
    const long long b = __double_as_longlong(v);
    const int lo = __shfl((int)(b & 0xffffffffll), src), hi = __shfl((int)(b >> 32), src);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// One workgroup solves the gauge-free reduced camera system.  A holds nf + 1
// rows of nf: the system's rows, then the right-hand side as an extra row,
// so that the Cholesky factorisation A = L L^T of the rows computes the
// forward substitution L y = g as that row's entries of L.  Right-looking,
// in panels of PW columns: the panel's rows (from the panel's diagonal down,
// right-hand side included) are staged in LDS; the PW x PW diagonal block is
// factored with one thread per entry; the rows below are the triangular
// solves x L11^T = a, one thread per row; the trailing lower triangle is
// updated in 4 x 4 register blocks from the panel in LDS.  Back substitution
// L^T x = y then runs panel by panel from the last: the products with the
// solved entries below a panel are summed over 1024 / PW row slices in a
// fixed order, and one wave solves the PW x PW triangle with lane broadcasts.
// The step is scattered to the free pose entries; the fixed ones are 0.
// `flags` and [k_begin, k_end) select the part one launch does (gather,
// panels, in-kernel trailing updates, back substitution).
constexpr int kSolveGather = 1, kSolveTrailing = 2, kSolveBack = 4;

template <int PW>
__global__ __launch_bounds__(kSolveThreads) void k_ba_solve(int n_cams, int gauge_axis,
                                                            const double* __restrict__ S,
                                                            const double* __restrict__ g, double* __restrict__ A,
                                                            double* __restrict__ dpose, int k_begin, int k_end,
                                                            int flags) {
    extern __shared__ double lds[];
    constexpr int T = kSolveThreads, PS = PW + 1, NS = T / PW;
    const int n6 = 6 * n_cams, nf = n6 - 7, t = threadIdx.x;
    double* col = lds;                  // [PW] the column being eliminated
    double* inv = col + PW;             // [PW] 1 / L_pp of the panel
    double* dd = inv + PW;              // [1]  the pivot
    double* P = dd + 2;                 // panel [nf + 1][PS]; later red [NS][PW], L11 [PW][PS], x [nf]
    if (flags & kSolveGather) {
        for (int e = t; e < nf * nf; e += T) {
            const int r = e / nf, c = e - r * nf;
            if (c <= r) A[e] = S[(size_t)free_param(r, gauge_axis) * n6 + free_param(c, gauge_axis)];
        }
        for (int c = t; c < nf; c += T) A[(size_t)nf * nf + c] = g[free_param(c, gauge_axis)];
        __syncthreads();
    }
    for (int k0 = k_begin; k0 < nf && k0 < k_end; k0 += PW) {
        const int nb = min(PW, nf - k0), m = nf + 1 - k0;  // panel rows, the right-hand side last
        for (int e = t; e < m * nb; e += T) {
            const int r = e / nb, c = e - r * nb;
            P[r * PS + c] = (r >= nb || c <= r) ? A[(size_t)(k0 + r) * nf + k0 + c] : 0.0;
        }
        __syncthreads();
        // diagonal block: thread (r, c), c <= r < nb, keeps its entry in a register
        const int dr = t / PW, dc = t % PW;
        const bool own = t < PW * PW && dr < nb && dc <= dr;
        double a = own ? P[dr * PS + dc] : 0.0;
        for (int p = 0; p < nb; ++p) {
            if (own && dr == p && dc == p) dd[0] = a;
            __syncthreads();
            if (own && dc == p) {
                const double d = sqrt(dd[0]);
                a = dr == p ? d : a / d;
                col[dr] = a;
                if (dr == p) inv[p] = 1.0 / d;
            }
            __syncthreads();
            if (own && dc > p) a -= col[dr] * col[dc];
        }
        if (own) P[dr * PS + dc] = a;
        __syncthreads();
        // rows below the block: x L11^T = a, x_p = (a_p - sum_{q<p} x_q L_pq) / L_pp
        for (int r = nb + t; r < m; r += T) {
            double x[PW];
#pragma unroll
            for (int p = 0; p < PW; ++p) x[p] = p < nb ? P[r * PS + p] : 0.0;
#pragma unroll
            for (int p = 0; p < PW; ++p) {
                if (p < nb) {
                    double v = x[p];
#pragma unroll
                    for (int q = 0; q < p; ++q) v -= x[q] * P[p * PS + q];
                    x[p] = v * inv[p];
                }
            }
#pragma unroll
            for (int p = 0; p < PW; ++p)
                if (p < nb) P[r * PS + p] = x[p];
        }
        __syncthreads();
        for (int e = t; e < m * nb; e += T) {
            const int r = e / nb, c = e - r * nb;
            if (r >= nb || c <= r) A[(size_t)(k0 + r) * nf + k0 + c] = P[r * PS + c];
        }
        // trailing update of rows nb..m-1 (right-hand side last), columns
        // nb..nf-k0-1, lower triangle: A_ij -= sum_p L_ip L_jp (here, or by
        // k_ba_syrk over many workgroups)
        const int mt = m - nb, mc = mt - 1, bi_n = (mt + 3) >> 2, bj_n = (mc + 3) >> 2;
        for (int e = t; e < ((flags & kSolveTrailing) ? bi_n * bj_n : 0); e += T) {
            const int bi = e / bj_n, bj = e - bi * bj_n;
            if (bj > bi) continue;
            double acc[4][4];
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] = 0.0;
            int ri[4], rj[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                ri[u] = nb + min(4 * bi + u, mt - 1);
                rj[u] = nb + min(4 * bj + u, mc - 1);
            }
            for (int p = 0; p < nb; ++p) {
                double li[4], lj[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    li[u] = P[ri[u] * PS + p];
                    lj[u] = P[rj[u] * PS + p];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int v = 0; v < 4; ++v) acc[u][v] = fma(li[u], lj[v], acc[u][v]);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int ii = 4 * bi + u;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int jj = 4 * bj + v;
                    if (ii < mt && jj < mc && jj <= ii) A[(size_t)(k0 + nb + ii) * nf + k0 + nb + jj] -= acc[u][v];
                }
            }
        }
        __syncthreads();
    }
    if (!(flags & kSolveBack)) return;
    // back substitution L^T x = y, y = row nf of A
    double* red = P;                    // [NS][PW]
    double* L11 = red + NS * PW;        // [PW][PS]
    double* xs = L11 + PW * PS;         // [nf]
    const int lane = t & 63;
    for (int k0 = ((nf - 1) / PW) * PW; k0 >= 0; k0 -= PW) {
        const int nb = min(PW, nf - k0), cc = t % PW, sl = t / PW;
        double v = 0.0;
        if (cc < nb)
            for (int r = k0 + nb + sl; r < nf; r += NS) v += A[(size_t)r * nf + k0 + cc] * xs[r];
        red[sl * PW + cc] = v;
        for (int e = t; e < nb * nb; e += T) {
            const int r = e / nb, c = e - r * nb;
            if (c <= r) L11[r * PS + c] = A[(size_t)(k0 + r) * nf + k0 + c];
        }
        __syncthreads();
        if (t < 64) {
            double w = 0.0;
            if (lane < nb) {
                w = A[(size_t)nf * nf + k0 + lane];
                for (int q = 0; q < NS; ++q) w -= red[q * PW + lane];
            }
            for (int q = nb - 1; q >= 0; --q) {
                const double xq = lane_bcast(w / L11[q * PS + q], q);
                if (lane == q) w = xq;
                else if (lane < q) w -= L11[q * PS + lane] * xq;
            }
            if (lane < nb) xs[k0 + lane] = w;
        }
        __syncthreads();
    }
    for (int e = t; e < n6; e += T) dpose[e] = 0.0;
    __syncthreads();
    for (int r = t; r < nf; r += T) dpose[free_param(r, gauge_axis)] = xs[r];
}

// Trailing update after panel k0 over many workgroups: one 32 x 32 tile of
// the lower triangle of rows k0 + nb .. nf (the right-hand side row last)
// and columns k0 + nb .. nf - 1 per workgroup, A_ij -= sum_p L_ip L_jp with
// the panel's columns of both row ranges staged in LDS; each thread a 2 x 2
// block, the sum over p in order.
constexpr int kSyrkTile = 32;

template <int PW>
__global__ __launch_bounds__(256) void k_ba_syrk(int nf, int k0, double* __restrict__ A) {
    __shared__ double Li[kSyrkTile][PW + 1], Lj[kSyrkTile][PW + 1];
    const int t = threadIdx.x, nb = min(PW, nf - k0), r0 = k0 + nb;
    const int mt = nf + 1 - r0, mc = nf - r0;
    const int e = (int)blockIdx.x;
    int ti = 0;
    while ((ti + 1) * (ti + 2) / 2 <= e) ++ti;
    const int tj = e - ti * (ti + 1) / 2, i0 = ti * kSyrkTile, j0 = tj * kSyrkTile;
    if (j0 >= mc) return;
    for (int q = t; q < kSyrkTile * nb; q += 256) {
        const int r = q / nb, p = q - r * nb;
        Li[r][p] = i0 + r < mt ? A[(size_t)(r0 + i0 + r) * nf + k0 + p] : 0.0;
        Lj[r][p] = j0 + r < mc ? A[(size_t)(r0 + j0 + r) * nf + k0 + p] : 0.0;
    }
    __syncthreads();
    const int ty = t >> 4, tx = t & 15;
    double acc[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
    for (int p = 0; p < nb; ++p) {
        const double a0 = Li[2 * ty][p], a1 = Li[2 * ty + 1][p], b0 = Lj[2 * tx][p], b1 = Lj[2 * tx + 1][p];
        acc[0][0] = fma(a0, b0, acc[0][0]);
        acc[0][1] = fma(a0, b1, acc[0][1]);
        acc[1][0] = fma(a1, b0, acc[1][0]);
        acc[1][1] = fma(a1, b1, acc[1][1]);
    }
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v) {
            const int ii = i0 + 2 * ty + u, jj = j0 + 2 * tx + v;
            if (ii < mt && jj < mc && jj <= ii) A[(size_t)(r0 + ii) * nf + r0 + jj] -= acc[u][v];
        }
}

__global__ __launch_bounds__(256) void k_ba_backsub(pgs_ba_problem pb, const double* __restrict__ obs_rec,
                                                    const double* __restrict__ pt_rec,
                                                    const double* __restrict__ dpose,
                                                    double* __restrict__ dpoint) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= pb.n_points) return;
    double s[3] = {0, 0, 0};
    for (uint32_t o = pb.point_start_dev[j]; o < pb.point_start_dev[j + 1]; ++o) {
        const double* Htp = obs_rec + (size_t)o * kObsRec;
        const double* dt = dpose + 6 * (size_t)pb.obs_cam_dev[o];
        for (int b = 0; b < 3; ++b)
            for (int a = 0; a < 6; ++a) s[b] += Htp[3 * a + b] * dt[a];
    }
    const double* pr = pt_rec + (size_t)j * kPtRec;
    for (int a = 0; a < 3; ++a)
        dpoint[3 * (size_t)j + a] = pr[9 + a] - (pr[3 * a] * s[0] + pr[3 * a + 1] * s[1] + pr[3 * a + 2] * s[2]);
}

// Robust cost: per-block partial sums of rho over the observations.
__global__ __launch_bounds__(kCostThreads) void k_ba_cost(pgs_ba_problem pb, const double* __restrict__ rot,
                                                          const double* __restrict__ centre,
                                                          const double* __restrict__ pts,
                                                          double* __restrict__ part) {
    __shared__ double s[kCostThreads];
    double acc = 0.0;
    for (int j = blockIdx.x * kCostThreads + threadIdx.x; j < pb.n_points; j += gridDim.x * kCostThreads) {
        for (uint32_t o = pb.point_start_dev[j]; o < pb.point_start_dev[j + 1]; ++o) {
            Obs ob;
            observe(pb, rot, centre, pts, (int)o, j, ob);
            const double q = ob.r[0] * ob.r[0] + ob.r[1] * ob.r[1];
            const double n = sqrt(q);
            acc += n <= pb.huber_delta ? q : 2.0 * pb.huber_delta * n - pb.huber_delta * pb.huber_delta;
        }
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int k = kCostThreads / 2; k > 0; k >>= 1) {
        if (threadIdx.x < k) s[threadIdx.x] += s[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

__global__ void k_ba_cost_final(const double* __restrict__ part, int n, double* __restrict__ out) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        double acc = 0.0;
        for (int k = 0; k < n; ++k) acc += part[k];
        *out = acc;
    }
}

__global__ __launch_bounds__(256) void k_ba_apply(int n_cams, int n_points, const double* __restrict__ rot,
                                                  const double* __restrict__ centre,
                                                  const double* __restrict__ pts, const double* __restrict__ dpose,
                                                  const double* __restrict__ dpoint, double* __restrict__ rot_out,
                                                  double* __restrict__ centre_out, double* __restrict__ pts_out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n_points)
        for (int a = 0; a < 3; ++a) pts_out[3 * (size_t)k + a] = pts[3 * (size_t)k + a] + dpoint[3 * (size_t)k + a];
    if (k < n_cams) {
        const double* w = dpose + 6 * k;
        const double th = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
        // exp([w]x) = I + a [w]x + b [w]x^2 (Rodrigues; series below 1e-8)
        const double a = th < 1e-8 ? 1.0 - th * th / 6.0 : sin(th) / th;
        const double b = th < 1e-8 ? 0.5 - th * th / 24.0 : (1.0 - cos(th)) / (th * th);
        const double K[9] = {0, -w[2], w[1], w[2], 0, -w[0], -w[1], w[0], 0};
        double E[9];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                double kk = 0.0;
                for (int m = 0; m < 3; ++m) kk += K[3 * r + m] * K[3 * m + c];
                E[3 * r + c] = (r == c ? 1.0 : 0.0) + a * K[3 * r + c] + b * kk;
            }
        const double* R = rot + 9 * k;
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c)
                rot_out[9 * k + 3 * r + c] = R[3 * r] * E[c] + R[3 * r + 1] * E[3 + c] + R[3 * r + 2] * E[6 + c];
        for (int a2 = 0; a2 < 3; ++a2) centre_out[3 * k + a2] = centre[3 * k + a2] + w[3 + a2];
    }
}

// ------------------------------------------------------------ refinement

// Thread per point: the least-squares intersection of its observation rays
// (sum (I - d d^T) P = sum (I - d d^T) c, d the unit world ray of the
// measured pixel, solved by the adjugate when det > 1e-12 trace^3), then
// over its observations in front of their cameras the mean reprojection
// error and the smallest cosine between two camera-to-point rays; the point
// is kept with >= 2 such observations, mean error <= max_err and smallest
// cosine <= cos_min; an observation is kept when its point is and it lies
// in front of its camera.
__global__ __launch_bounds__(256) void k_ba_refine(pgs_ba_problem pb, const double* __restrict__ rot,
                                                   const double* __restrict__ centre, double max_err,
                                                   double cos_min, double* __restrict__ pts_out,
                                                   uint8_t* __restrict__ keep_pt, uint8_t* __restrict__ keep_obs) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= pb.n_points) return;
    const uint32_t o0 = pb.point_start_dev[j], o1 = pb.point_start_dev[j + 1];
    double A[6] = {0, 0, 0, 0, 0, 0}, b[3] = {0, 0, 0};  // A00 A01 A02 A11 A12 A22
    for (uint32_t o = o0; o < o1; ++o) {
        const int i = (int)pb.obs_cam_dev[o];
        const double* R = rot + 9 * (size_t)i;
        const double* c = centre + 3 * (size_t)i;
        const double q0 = (pb.obs_uv_dev[2 * (size_t)o] - pb.cx) / pb.fx;
        const double q1 = (pb.obs_uv_dev[2 * (size_t)o + 1] - pb.cy) / pb.fy;
        double d[3];
        for (int a = 0; a < 3; ++a) d[a] = R[a] * q0 + R[3 + a] * q1 + R[6 + a];  // R^T (q0, q1, 1)
        const double inv = 1.0 / sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        for (int a = 0; a < 3; ++a) d[a] *= inv;
        const double dc = d[0] * c[0] + d[1] * c[1] + d[2] * c[2];
        A[0] += 1.0 - d[0] * d[0];
        A[1] -= d[0] * d[1];
        A[2] -= d[0] * d[2];
        A[3] += 1.0 - d[1] * d[1];
        A[4] -= d[1] * d[2];
        A[5] += 1.0 - d[2] * d[2];
        for (int a = 0; a < 3; ++a) b[a] += c[a] - d[a] * dc;
    }
    const double c00 = A[3] * A[5] - A[4] * A[4], c01 = A[2] * A[4] - A[1] * A[5], c02 = A[1] * A[4] - A[2] * A[3];
    const double c11 = A[0] * A[5] - A[2] * A[2], c12 = A[1] * A[2] - A[0] * A[4], c22 = A[0] * A[3] - A[1] * A[1];
    const double det = A[0] * c00 + A[1] * c01 + A[2] * c02;
    const double tr = A[0] + A[3] + A[5];
    const bool solvable = det > 1e-12 * tr * tr * tr;
    double P[3] = {0.0, 0.0, 0.0};
    if (solvable) {
        const double id = 1.0 / det;
        P[0] = (c00 * b[0] + c01 * b[1] + c02 * b[2]) * id;
        P[1] = (c01 * b[0] + c11 * b[1] + c12 * b[2]) * id;
        P[2] = (c02 * b[0] + c12 * b[1] + c22 * b[2]) * id;
    }
    int cnt = 0;
    double esum = 0.0, mincos = 2.0;
    for (uint32_t o = o0; o < o1 && solvable; ++o) {
        const int i = (int)pb.obs_cam_dev[o];
        const double* R = rot + 9 * (size_t)i;
        const double* c = centre + 3 * (size_t)i;
        const double v0 = P[0] - c[0], v1 = P[1] - c[1], v2 = P[2] - c[2];
        const double x0 = R[0] * v0 + R[1] * v1 + R[2] * v2, x1 = R[3] * v0 + R[4] * v1 + R[5] * v2,
                     x2 = R[6] * v0 + R[7] * v1 + R[8] * v2;
        if (!(x2 > 0.0)) continue;
        const double du = pb.fx * x0 / x2 + pb.cx - pb.obs_uv_dev[2 * (size_t)o];
        const double dv = pb.fy * x1 / x2 + pb.cy - pb.obs_uv_dev[2 * (size_t)o + 1];
        esum += sqrt(du * du + dv * dv);
        ++cnt;
        const double n0 = 1.0 / sqrt(v0 * v0 + v1 * v1 + v2 * v2);
        for (uint32_t o2 = o + 1; o2 < o1; ++o2) {
            const int k = (int)pb.obs_cam_dev[o2];
            const double* R2 = rot + 9 * (size_t)k;
            const double* c2 = centre + 3 * (size_t)k;
            const double w0 = P[0] - c2[0], w1 = P[1] - c2[1], w2 = P[2] - c2[2];
            if (!(R2[6] * w0 + R2[7] * w1 + R2[8] * w2 > 0.0)) continue;
            const double cs = (v0 * w0 + v1 * w1 + v2 * w2) * n0 / sqrt(w0 * w0 + w1 * w1 + w2 * w2);
            mincos = fmin(mincos, cs);
        }
    }
    const bool keep = solvable && cnt >= 2 && esum / (double)(cnt > 0 ? cnt : 1) <= max_err && mincos <= cos_min;
    for (int a = 0; a < 3; ++a) pts_out[3 * (size_t)j + a] = P[a];
    keep_pt[j] = keep ? 1 : 0;
    for (uint32_t o = o0; o < o1; ++o) {
        bool front = false;
        if (keep) {
            const int i = (int)pb.obs_cam_dev[o];
            const double* R = rot + 9 * (size_t)i;
            const double* c = centre + 3 * (size_t)i;
            front = R[6] * (P[0] - c[0]) + R[7] * (P[1] - c[1]) + R[8] * (P[2] - c[2]) > 0.0;
        }
        keep_obs[o] = front ? 1 : 0;
    }
}

// Exclusive scan of 0/1 flags (optionally read through a permutation) into
// idx[0..n] (idx[n] = total): per-block sums, one workgroup over the block
// sums, then per-block prefixes.
constexpr int kFlagBlock = 1024;

__device__ __forceinline__ uint32_t flag_at(const uint8_t* f, const uint32_t* perm, uint32_t i) {
    return f[perm ? perm[i] : i] ? 1u : 0u;
}

__global__ __launch_bounds__(256) void k_flag_sums(const uint8_t* __restrict__ f, const uint32_t* __restrict__ perm,
                                                   uint32_t n, uint32_t* __restrict__ bsum) {
    __shared__ uint32_t s[4];
    const uint32_t base = blockIdx.x * kFlagBlock;
    uint32_t c = 0;
    for (uint32_t i = base + threadIdx.x; i < min(n, base + kFlagBlock); i += 256) c += flag_at(f, perm, i);
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) bsum[blockIdx.x] = s[0] + s[1] + s[2] + s[3];
}

__global__ __launch_bounds__(1024) void k_flag_top(uint32_t* __restrict__ bsum, uint32_t nb) {
    __shared__ uint32_t s[1024];
    uint32_t carry = 0;
    for (uint32_t base = 0; base < nb; base += 1024) {
        const uint32_t i = base + threadIdx.x;
        const uint32_t v = i < nb ? bsum[i] : 0u;
        s[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            const uint32_t add = threadIdx.x >= (unsigned)o ? s[threadIdx.x - o] : 0u;
            __syncthreads();
            s[threadIdx.x] += add;
            __syncthreads();
        }
        if (i < nb) bsum[i] = carry + s[threadIdx.x] - v;
        carry += s[1023];
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_flag_apply(const uint8_t* __restrict__ f, const uint32_t* __restrict__ perm,
                                                    uint32_t n, const uint32_t* __restrict__ bsum,
                                                    uint32_t* __restrict__ idx) {
    __shared__ uint32_t s[4];
    const uint32_t base = blockIdx.x * kFlagBlock;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint32_t run = bsum[blockIdx.x];
    for (uint32_t c0 = base; c0 < min(n, base + kFlagBlock); c0 += 256) {
        const uint32_t i = c0 + threadIdx.x;
        const uint32_t v = i < n ? flag_at(f, perm, i) : 0u;
        const uint64_t bal = __ballot(v != 0u);
        if (lane == 0) s[wv] = (uint32_t)__popcll(bal);
        __syncthreads();
        uint32_t before = 0, all = 0;
        for (int w = 0; w < 4; ++w) {
            before += w < wv ? s[w] : 0u;
            all += s[w];
        }
        if (i < n) idx[i] = run + before + (uint32_t)__popcll(bal & ((1ull << lane) - 1ull));
        run += all;
        __syncthreads();
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) idx[n] = run;
}

pgs_status flag_scan(const uint8_t* f, const uint32_t* perm, uint32_t n, uint32_t* idx, uint32_t* bsum,
                     hipStream_t s) {
    const uint32_t nb = (n + kFlagBlock - 1) / kFlagBlock;
    if (nb == 0) return PGS_OK;
    k_flag_sums<<<nb, 256, 0, s>>>(f, perm, n, bsum);
    k_flag_top<<<1, 1024, 0, s>>>(bsum, nb);
    k_flag_apply<<<nb, 256, 0, s>>>(f, perm, n, bsum, idx);
    return PGS_OK;
}

// Points: kept ones renumbered, their first observation's new index.
__global__ __launch_bounds__(256) void k_compact_points(int M, const uint8_t* __restrict__ keep_pt,
                                                        const uint32_t* __restrict__ pidx,
                                                        const uint32_t* __restrict__ oidx,
                                                        const uint32_t* __restrict__ point_start,
                                                        const double* __restrict__ pts, double* __restrict__ pts_out,
                                                        uint32_t* __restrict__ point_start_out, int O,
                                                        uint32_t* __restrict__ counts) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < M && keep_pt[j]) {
        const uint32_t n = pidx[j];
        for (int a = 0; a < 3; ++a) pts_out[3 * (size_t)n + a] = pts[3 * (size_t)j + a];
        point_start_out[n] = oidx[point_start[j]];
    }
    if (j == 0) {
        point_start_out[pidx[M]] = oidx[point_start[M]];
        counts[0] = pidx[M];
        counts[1] = oidx[O];
    }
}

__global__ __launch_bounds__(256) void k_compact_obs(pgs_ba_problem pb, const uint8_t* __restrict__ keep_obs,
                                                     const uint32_t* __restrict__ oidx,
                                                     const uint32_t* __restrict__ pidx, const uint32_t* __restrict__ qidx,
                                                     uint32_t* __restrict__ cam_out, uint32_t* __restrict__ pt_out,
                                                     double* __restrict__ uv_out, uint32_t* __restrict__ cam_obs_out,
                                                     uint32_t* __restrict__ cam_start_out) {
    const uint32_t o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o < (uint32_t)pb.n_obs) {
        if (keep_obs[o]) {
            const uint32_t n = oidx[o];
            cam_out[n] = pb.obs_cam_dev[o];
            pt_out[n] = pidx[pb.obs_pt_dev[o]];
            uv_out[2 * (size_t)n] = pb.obs_uv_dev[2 * (size_t)o];
            uv_out[2 * (size_t)n + 1] = pb.obs_uv_dev[2 * (size_t)o + 1];
        }
        // o is a position in the by-camera list here
        const uint32_t ob = pb.cam_obs_dev[o];
        if (keep_obs[ob]) cam_obs_out[qidx[o]] = oidx[ob];
    }
    if (o <= (uint32_t)pb.n_cams) cam_start_out[o] = qidx[pb.cam_start_dev[o]];
}

// Workspace layout of one problem size.
struct BaWs {
    double *obs_rec, *pt_rec, *cam_part, *S, *g, *A, *part;
    size_t bytes;
};

inline size_t al(size_t x) { return (x + 255) & ~(size_t)255; }
constexpr int kCostBlocks = 1024;

BaWs ba_layout(void* base, int C, int M, int O) {
    BaWs w{};
    char* p = static_cast<char*>(base);
    size_t off = 0;
    const size_t n6 = 6 * (size_t)C, nf = n6 > 7 ? n6 - 7 : 0;
    auto take = [&](size_t n) { double* q = reinterpret_cast<double*>(p + off); off += al(n * 8); return q; };
    w.obs_rec = take((size_t)O * kObsRec);
    w.pt_rec = take((size_t)M * kPtRec);
    w.cam_part = take((size_t)C * kCamSplit * (6 * n6 + 6));
    w.S = take(n6 * n6);
    w.g = take(n6);
    w.A = take((nf + 1) * nf);
    w.part = take(kCostBlocks);
    w.bytes = off;
    return w;
}

// Panel width of the solve and its LDS: the panel's nf + 1 rows padded to
// PW + 1 doubles (32 columns up to nf = 400: at most 106 KB; 16 beyond, up
// to nf = 6 PGS_BA_MAX_CAMS - 7: about 104 KB).
constexpr int kSolveWide = 400;
template <int PW>
inline size_t solve_lds(int nf) {
    const size_t panel = (size_t)(nf + 1) * (PW + 1), back = (size_t)kSolveThreads + PW * (PW + 1) + nf;
    return (2 * PW + 2 + (panel > back ? panel : back)) * sizeof(double);
}
template <int PW>
bool solve_lds_reserved(int nf) {
    static const bool ok = hipFuncSetAttribute(reinterpret_cast<const void*>(k_ba_solve<PW>),
                                               hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)solve_lds<PW>(PW == 32 ? kSolveWide : 6 * PGS_BA_MAX_CAMS - 7)) ==
                           hipSuccess;
    return ok && solve_lds<PW>(nf) <= solve_lds<PW>(PW == 32 ? kSolveWide : 6 * PGS_BA_MAX_CAMS - 7);
}

// The solve as a chain of launches: the gather and the first panel, then
// per panel the trailing update over many workgroups and the next panel's
// factorisation (one workgroup), then the back substitution.
template <int PW>
void solve_panels(int C, int gauge_axis, const BaWs& w, double* dpose, hipStream_t s) {
    const int nf = 6 * C - 7;
    const size_t lds = solve_lds<PW>(nf);
    for (int k0 = 0; k0 < nf; k0 += PW) {
        k_ba_solve<PW><<<1, kSolveThreads, lds, s>>>(C, gauge_axis, w.S, w.g, w.A, dpose, k0, k0 + PW,
                                                     k0 == 0 ? kSolveGather : 0);
        const int nb = min(PW, nf - k0), mt = nf + 1 - k0 - nb;
        if (nf - k0 - nb > 0) {
            const int tiles = (mt + kSyrkTile - 1) / kSyrkTile;
            k_ba_syrk<PW><<<tiles * (tiles + 1) / 2, 256, 0, s>>>(nf, k0, w.A);
        }
    }
    k_ba_solve<PW><<<1, kSolveThreads, lds, s>>>(C, gauge_axis, w.S, w.g, w.A, dpose, nf, nf, kSolveBack);
}

pgs_status check_problem(const pgs_ba_problem* pb, const char* who) {
    PGS_REQUIRE(pb != nullptr, "%s: null problem", who);
    PGS_REQUIRE(pb->n_cams >= 2 && pb->n_cams <= PGS_BA_MAX_CAMS, "%s: n_cams %d not in 2..%d", who, pb->n_cams,
                PGS_BA_MAX_CAMS);
    PGS_REQUIRE(pb->n_points >= 1 && pb->n_obs >= 1, "%s: empty problem", who);
    PGS_REQUIRE(pb->gauge_axis >= 0 && pb->gauge_axis <= 2, "%s: gauge_axis %d", who, pb->gauge_axis);
    PGS_REQUIRE(pb->huber_delta > 0.0, "%s: huber_delta must be > 0", who);
    PGS_REQUIRE(pb->obs_cam_dev && pb->obs_pt_dev && pb->obs_uv_dev && pb->point_start_dev && pb->cam_obs_dev &&
                    pb->cam_start_dev, "%s: null pointer in the problem", who);
    return PGS_OK;
}

}  // namespace

extern "C" size_t pgs_ba_workspace(int32_t n_cams, int32_t n_points, int32_t n_obs) {
    if (n_cams < 0 || n_points < 0 || n_obs < 0) return 0;
    return ba_layout(nullptr, n_cams, n_points, n_obs).bytes;
}

extern "C" pgs_status pgs_ba_cost(const pgs_ba_problem* problem, const double* rot_dev, const double* centre_dev,
                                  const double* points_dev, double* cost_dev, void* workspace_dev,
                                  size_t workspace_bytes, void* stream) {
    if (pgs_status st = check_problem(problem, "pgs_ba_cost")) return st;
    PGS_REQUIRE(rot_dev && centre_dev && points_dev && cost_dev && workspace_dev, "pgs_ba_cost: null pointer");
    const BaWs w = ba_layout(workspace_dev, problem->n_cams, problem->n_points, problem->n_obs);
    PGS_REQUIRE(workspace_bytes >= w.bytes, "pgs_ba_cost: workspace %zu < %zu", workspace_bytes, w.bytes);
    hipStream_t s = pgs::as_stream(stream);
    const int blocks = min(kCostBlocks, (problem->n_points + kCostThreads - 1) / kCostThreads);
    k_ba_cost<<<blocks, kCostThreads, 0, s>>>(*problem, rot_dev, centre_dev, points_dev, w.part);
    k_ba_cost_final<<<1, 64, 0, s>>>(w.part, blocks, cost_dev);
    PGS_CHECK_LAUNCH("pgs_ba_cost");
    return PGS_OK;
}

extern "C" pgs_status pgs_ba_step(const pgs_ba_problem* problem, const double* rot_dev, const double* centre_dev,
                                  const double* points_dev, double lambda, double* dpose_dev, double* dpoint_dev,
                                  void* workspace_dev, size_t workspace_bytes, void* stream) {
    if (pgs_status st = check_problem(problem, "pgs_ba_step")) return st;
    PGS_REQUIRE(lambda >= 0.0, "pgs_ba_step: lambda < 0");
    PGS_REQUIRE(rot_dev && centre_dev && points_dev && dpose_dev && dpoint_dev && workspace_dev,
                "pgs_ba_step: null pointer");
    const int C = problem->n_cams, M = problem->n_points;
    const BaWs w = ba_layout(workspace_dev, C, M, problem->n_obs);
    PGS_REQUIRE(workspace_bytes >= w.bytes, "pgs_ba_step: workspace %zu < %zu", workspace_bytes, w.bytes);
    hipStream_t s = pgs::as_stream(stream);
    k_ba_points<<<(M + 255) / 256, 256, 0, s>>>(*problem, rot_dev, centre_dev, points_dev, lambda, w.obs_rec,
                                                w.pt_rec);
    const size_t lds = (size_t)(6 * 6 * C + (kCamThreads / 64) * 27 + 6) * sizeof(double);
    k_ba_cameras<<<dim3(C, kCamSplit), kCamThreads, lds, s>>>(*problem, lambda, w.obs_rec, w.pt_rec, w.cam_part);
    const size_t rows = (size_t)C * (36 * C + 6);
    k_ba_rows<<<(unsigned)((rows + 255) / 256), 256, 0, s>>>(C, w.cam_part, w.S, w.g);
    const int nf = 6 * C - 7;
    if (nf <= kSolveWide) {
        PGS_REQUIRE(solve_lds_reserved<32>(nf), "pgs_ba_step: cannot reserve LDS for the solve");
        solve_panels<32>(C, problem->gauge_axis, w, dpose_dev, s);
    } else {
        PGS_REQUIRE(solve_lds_reserved<16>(nf), "pgs_ba_step: cannot reserve LDS for the solve");
        solve_panels<16>(C, problem->gauge_axis, w, dpose_dev, s);
    }
    k_ba_backsub<<<(M + 255) / 256, 256, 0, s>>>(*problem, w.obs_rec, w.pt_rec, dpose_dev, dpoint_dev);
    PGS_CHECK_LAUNCH("pgs_ba_step");
    return PGS_OK;
}

extern "C" pgs_status pgs_ba_apply(int32_t n_cams, int32_t n_points, const double* rot_dev,
                                   const double* centre_dev, const double* points_dev, const double* dpose_dev,
                                   const double* dpoint_dev, double* rot_out_dev, double* centre_out_dev,
                                   double* points_out_dev, void* stream) {
    PGS_REQUIRE(n_cams >= 0 && n_points >= 0, "pgs_ba_apply: negative size");
    PGS_REQUIRE(rot_dev && centre_dev && points_dev && dpose_dev && dpoint_dev && rot_out_dev && centre_out_dev &&
                    points_out_dev, "pgs_ba_apply: null pointer");
    const int n = max(n_cams, n_points);
    if (n == 0) return PGS_OK;
    k_ba_apply<<<(n + 255) / 256, 256, 0, pgs::as_stream(stream)>>>(n_cams, n_points, rot_dev, centre_dev,
                                                                   points_dev, dpose_dev, dpoint_dev, rot_out_dev,
                                                                   centre_out_dev, points_out_dev);
    PGS_CHECK_LAUNCH("pgs_ba_apply");
    return PGS_OK;
}

extern "C" pgs_status pgs_ba_refine(const pgs_ba_problem* problem, const double* rot_dev, const double* centre_dev,
                                    double max_err, double min_angle, double* points_out_dev,
                                    uint8_t* keep_point_dev, uint8_t* keep_obs_dev, void* stream) {
    if (pgs_status st = check_problem(problem, "pgs_ba_refine")) return st;
    PGS_REQUIRE(rot_dev && centre_dev && points_out_dev && keep_point_dev && keep_obs_dev,
                "pgs_ba_refine: null pointer");
    PGS_REQUIRE(max_err >= 0.0 && min_angle >= 0.0, "pgs_ba_refine: negative threshold");
    const int M = problem->n_points;
    k_ba_refine<<<(M + 255) / 256, 256, 0, pgs::as_stream(stream)>>>(*problem, rot_dev, centre_dev, max_err,
                                                                     cos(min_angle), points_out_dev, keep_point_dev,
                                                                     keep_obs_dev);
    PGS_CHECK_LAUNCH("pgs_ba_refine");
    return PGS_OK;
}

extern "C" size_t pgs_ba_compact_workspace(int32_t n_points, int32_t n_obs) {
    if (n_points < 0 || n_obs < 0) return 0;
    const size_t nb = ((size_t)(n_points > n_obs ? n_points : n_obs) + kFlagBlock - 1) / kFlagBlock + 1;
    return al(((size_t)n_points + 1) * 4) + 2 * al(((size_t)n_obs + 1) * 4) + 3 * al(nb * 4);
}

extern "C" pgs_status pgs_ba_compact(const pgs_ba_problem* problem, const uint8_t* keep_point_dev,
                                     const uint8_t* keep_obs_dev, const double* points_dev,
                                     uint32_t* obs_cam_out_dev, uint32_t* obs_pt_out_dev, double* obs_uv_out_dev,
                                     uint32_t* point_start_out_dev, uint32_t* cam_obs_out_dev,
                                     uint32_t* cam_start_out_dev, double* points_out_dev, uint32_t* counts_out_dev,
                                     void* workspace_dev, size_t workspace_bytes, void* stream) {
    if (pgs_status st = check_problem(problem, "pgs_ba_compact")) return st;
    PGS_REQUIRE(keep_point_dev && keep_obs_dev && points_dev && obs_cam_out_dev && obs_pt_out_dev &&
                    obs_uv_out_dev && point_start_out_dev && cam_obs_out_dev && cam_start_out_dev &&
                    points_out_dev && counts_out_dev && workspace_dev, "pgs_ba_compact: null pointer");
    const int M = problem->n_points, O = problem->n_obs;
    PGS_REQUIRE(workspace_bytes >= pgs_ba_compact_workspace(M, O), "pgs_ba_compact: workspace %zu < %zu",
                workspace_bytes, pgs_ba_compact_workspace(M, O));
    hipStream_t s = pgs::as_stream(stream);
    char* p = static_cast<char*>(workspace_dev);
    const size_t nb = ((size_t)(M > O ? M : O) + kFlagBlock - 1) / kFlagBlock + 1;
    uint32_t* pidx = reinterpret_cast<uint32_t*>(p);
    p += al(((size_t)M + 1) * 4);
    uint32_t* oidx = reinterpret_cast<uint32_t*>(p);
    p += al(((size_t)O + 1) * 4);
    uint32_t* qidx = reinterpret_cast<uint32_t*>(p);
    p += al(((size_t)O + 1) * 4);
    uint32_t* b0 = reinterpret_cast<uint32_t*>(p);
    p += al(nb * 4);
    uint32_t* b1 = reinterpret_cast<uint32_t*>(p);
    p += al(nb * 4);
    uint32_t* b2 = reinterpret_cast<uint32_t*>(p);
    flag_scan(keep_point_dev, nullptr, (uint32_t)M, pidx, b0, s);
    flag_scan(keep_obs_dev, nullptr, (uint32_t)O, oidx, b1, s);
    flag_scan(keep_obs_dev, problem->cam_obs_dev, (uint32_t)O, qidx, b2, s);
    k_compact_points<<<(M + 255) / 256, 256, 0, s>>>(M, keep_point_dev, pidx, oidx, problem->point_start_dev,
                                                     points_dev, points_out_dev, point_start_out_dev, O,
                                                     counts_out_dev);
    const int n = (O > problem->n_cams + 1 ? O : problem->n_cams + 1);
    k_compact_obs<<<(n + 255) / 256, 256, 0, s>>>(*problem, keep_obs_dev, oidx, pidx, qidx, obs_cam_out_dev,
                                                  obs_pt_out_dev, obs_uv_out_dev, cam_obs_out_dev,
                                                  cam_start_out_dev);
    PGS_CHECK_LAUNCH("pgs_ba_compact");
    return PGS_OK;
}
