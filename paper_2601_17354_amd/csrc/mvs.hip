// Single-reference cost-volume multi-view stereo on gfx950 (subsection
// "Single-Reference Cost-Volume MVS": probabilistic depth range, reference
// score S_ref, Census plane-sweep cost, SGM aggregation, confidence filter,
// fusion into the dense cloud).
//
// Kernels:
//   k_mvs_depths / k_mvs_range  camera depths of the sparse points that
//       project into each view as float64 bit patterns (all ones for the
//       others), then per view (one workgroup) the ranks that define the 5%
//       and 95% quantiles found by radix selection; range =
//       [0.5 q_.05, 1.5 q_.95];
//   k_mvs_ref     per target view the candidate maximising
//       exp(-(b - b_target)^2 / (2 sigma_b^2)) max(alpha / alpha_min, 1);
//   k_census      7 x 7 Census (48 bits) from a 22 x 22 LDS tile;
//   k_cost<D>     one thread per (pixel slot, plane) over 128 pixels per
//       workgroup: the plane-sweep pixel in the
//       reference view from float32 arithmetic in a fixed order without
//       contraction (the nearest-pixel decision is reproducible), Hamming
//       distance of the Census strings; cost volume [y][x][plane] bytes;
//   k_sgm<KPL, COLS>  one wave per image line sweeps it forward (path costs
//       stored as bytes) and back: lane l holds the KPL consecutive planes
//       KPL l .. (one load per step of each operand, prefetched 8 steps
//       ahead); per step the previous costs' minimum is a DPP wave reduction
//       and the neighbouring planes come from DPP wave shifts.  The row
//       kernel writes the two row paths' sum; the column kernel adds both
//       column paths to it, stages the totals of 32 steps in an LDS ring and
//       lets two lanes per pixel take the winner, the confidence test and the refined
//       depth of one of those pixels, without storing the total;
//   k_fuse_*      per-row counts, one scan over rows and the back-projection
//       of the kept pixels in row-major order.

#include <math.h>

#include "common.hpp"

namespace {

constexpr int kCensusR = 3;
constexpr int kCensusBits = (2 * kCensusR + 1) * (2 * kCensusR + 1) - 1;  // 48
constexpr int kCostOut = kCensusBits;
constexpr int kTile = 16;
constexpr int kHalo = kTile + 2 * kCensusR;

struct Cam64 {
    double fx, fy, cx, cy, R[9], t[3];
};

__device__ __forceinline__ Cam64 cam64(const pgs_camera& c) {
    Cam64 d;
    d.fx = c.fx;
    d.fy = c.fy;
    d.cx = c.cx;
    d.cy = c.cy;
    for (int r = 0; r < 3; ++r) {
        for (int k = 0; k < 3; ++k) d.R[3 * r + k] = c.viewmat[4 * r + k];
        d.t[r] = c.viewmat[4 * r + 3];
    }
    return d;
}

// ---------------------------------------------------------------- census

__global__ __launch_bounds__(256) void k_census(const uint8_t* __restrict__ grey, int W, int H,
                                                uint64_t* __restrict__ out) {
    __shared__ int tile[kHalo][kHalo];
    const size_t off = (size_t)blockIdx.z * W * H;
    const int x0 = blockIdx.x * kTile - kCensusR, y0 = blockIdx.y * kTile - kCensusR;
    for (int e = threadIdx.x; e < kHalo * kHalo; e += 256) {
        const int ty = e / kHalo, tx = e - ty * kHalo;
        const int gx = min(max(x0 + tx, 0), W - 1), gy = min(max(y0 + ty, 0), H - 1);
        tile[ty][tx] = grey[off + (size_t)gy * W + gx];
    }
    __syncthreads();
    const int lx = threadIdx.x % kTile, ly = threadIdx.x / kTile;
    const int x = blockIdx.x * kTile + lx, y = blockIdx.y * kTile + ly;
    if (x >= W || y >= H) return;
    const int c = tile[ly + kCensusR][lx + kCensusR];
    uint64_t v = 0;
    int b = 0;
#pragma unroll
    for (int dy = -kCensusR; dy <= kCensusR; ++dy)
#pragma unroll
        for (int dx = -kCensusR; dx <= kCensusR; ++dx) {
            if (dy == 0 && dx == 0) continue;
            v |= (uint64_t)(tile[ly + kCensusR + dy][lx + kCensusR + dx] < c) << b;
            ++b;
        }
    out[off + (size_t)y * W + x] = v;
}

// ---------------------------------------------------------------- range

__global__ __launch_bounds__(256) void k_mvs_clear(uint32_t* __restrict__ p, int n) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// Key of point j in view v: the float64 bit pattern of its camera depth when
// it projects into the view (positive, so the patterns order like the
// values), all ones otherwise (after every valid key).
__global__ __launch_bounds__(256) void k_mvs_depths(const pgs_camera* __restrict__ cams, int W, int H,
                                                    const double* __restrict__ pts, int M,
                                                    uint64_t* __restrict__ keys) {
#pragma clang fp contract(off)
    const int v = blockIdx.y, j = blockIdx.x * 256 + threadIdx.x;
    if (j >= M) return;
    const Cam64 c = cam64(cams[v]);
    const double P0 = pts[3 * (size_t)j], P1 = pts[3 * (size_t)j + 1], P2 = pts[3 * (size_t)j + 2];
    const double x = c.R[0] * P0 + c.R[1] * P1 + c.R[2] * P2 + c.t[0];
    const double y = c.R[3] * P0 + c.R[4] * P1 + c.R[5] * P2 + c.t[1];
    const double z = c.R[6] * P0 + c.R[7] * P1 + c.R[8] * P2 + c.t[2];
    const double u = c.fx * (x / z) + c.cx, w = c.fy * (y / z) + c.cy;
    const bool in = z > 0.0 && u >= -0.5 && u < (double)W - 0.5 && w >= -0.5 && w < (double)H - 0.5;
    keys[(size_t)v * M + j] = in ? (uint64_t)__double_as_longlong(z) : ~0ull;
}

struct RangeLds {
    uint32_t hist[256];
    uint32_t wsum[16];
    uint64_t wmin[16];
    uint64_t prefix;
    uint32_t rank;
};

__device__ __forceinline__ uint32_t block_sum_u32(uint32_t v, RangeLds& L) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if ((threadIdx.x & 63) == 0) L.wsum[threadIdx.x >> 6] = v;
    __syncthreads();
    uint32_t s = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += L.wsum[w];
    __syncthreads();
    return s;
}

__device__ __forceinline__ uint64_t block_min_u64(uint64_t v, RangeLds& L) {
    for (int o = 32; o > 0; o >>= 1) {
        const uint64_t u = ((uint64_t)(uint32_t)__shfl_xor((int)(v >> 32), o) << 32) |
                           (uint32_t)__shfl_xor((int)(uint32_t)v, o);
        v = u < v ? u : v;
    }
    if ((threadIdx.x & 63) == 0) L.wmin[threadIdx.x >> 6] = v;
    __syncthreads();
    uint64_t m = ~0ull;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) m = L.wmin[w] < m ? L.wmin[w] : m;
    __syncthreads();
    return m;
}

// The rank-th smallest of the keys (one workgroup), by radix selection over
// 8-bit digits from the most significant; the digit is found by one wave
// (four bins per lane, a lane prefix sum and a ballot).
__device__ uint64_t select_rank(const uint64_t* __restrict__ keys, uint32_t n, uint32_t rank, RangeLds& L) {
    const int t = threadIdx.x, lane = t & 63;
    uint64_t prefix = 0, mask = 0;
    uint32_t r = rank;
    for (int shift = 56; shift >= 0; shift -= 8) {
        if (t < 256) L.hist[t] = 0u;
        __syncthreads();
        for (uint32_t i = t; i < n; i += blockDim.x) {
            const uint64_t k = keys[i];
            if ((k & mask) == prefix) atomicAdd(&L.hist[(k >> shift) & 255u], 1u);
        }
        __syncthreads();
        if (t < 64) {
            const uint32_t h0 = L.hist[4 * lane], h1 = L.hist[4 * lane + 1], h2 = L.hist[4 * lane + 2],
                           h3 = L.hist[4 * lane + 3];
            const uint32_t own = h0 + h1 + h2 + h3;
            uint32_t inc = own;
            for (int o = 1; o < 64; o <<= 1) {
                const uint32_t u = __shfl_up(inc, o);
                if (lane >= o) inc += u;
            }
            const uint32_t exc = inc - own;
            const uint64_t hit = __ballot(inc > r);
            const int q = __ffsll((long long)hit) - 1;  // first lane whose bins reach past r
            if (lane == q) {
                uint32_t acc = exc, d = 4 * lane + 3;
                const uint32_t hs[4] = {h0, h1, h2, h3};
                for (int e = 0; e < 4; ++e) {
                    if (acc + hs[e] > r) {
                        d = 4 * lane + e;
                        break;
                    }
                    acc += hs[e];
                }
                L.prefix = prefix | ((uint64_t)d << shift);
                L.rank = r - acc;
            }
        }
        __syncthreads();
        prefix = L.prefix;
        r = L.rank;
        mask |= 255ull << shift;
        __syncthreads();
    }
    return prefix;
}

// q(p) = z_i + (z_{i+1} - z_i)(h - i), h = (n - 1) p: z_i by selection, z_{i+1}
// is z_i when more than i + 1 keys are <= z_i, else the smallest key above.
__device__ double quantile_of(const uint64_t* keys, uint32_t M, uint32_t n, double p, RangeLds& L) {
#pragma clang fp contract(off)
    const double h = (double)(n - 1) * p;
    const uint32_t i = (uint32_t)floor(h);
    const uint64_t ki = select_rank(keys, M, i, L);
    const double zi = __longlong_as_double((long long)ki);
    if (i + 1 >= n) return zi;
    uint32_t le = 0;
    uint64_t above = ~0ull;
    for (uint32_t e = threadIdx.x; e < M; e += blockDim.x) {
        const uint64_t k = keys[e];
        le += k <= ki;
        if (k > ki && k < above) above = k;
    }
    le = block_sum_u32(le, L);
    above = block_min_u64(above, L);
    const double zj = le >= i + 2 ? zi : __longlong_as_double((long long)above);
    return zi + (zj - zi) * (h - (double)i);
}

__global__ __launch_bounds__(1024) void k_mvs_range(int M, const uint64_t* __restrict__ keys,
                                                    double* __restrict__ range) {
#pragma clang fp contract(off)
    __shared__ RangeLds L;
    const int v = blockIdx.x;
    const uint64_t* k = keys + (size_t)v * M;
    uint32_t c = 0;
    for (int e = threadIdx.x; e < M; e += blockDim.x) c += k[e] != ~0ull;
    const uint32_t n = block_sum_u32(c, L);
    double lo = 0.0, hi = 0.0;
    if (n > 0) {
        lo = 0.5 * quantile_of(k, M, n, 0.05, L);
        hi = 1.5 * quantile_of(k, M, n, 0.95, L);
    }
    if (threadIdx.x == 0) {
        range[2 * v] = lo;
        range[2 * v + 1] = hi;
    }
}

// ---------------------------------------------------------------- reference

__global__ __launch_bounds__(64) void k_mvs_ref(const pgs_camera* __restrict__ cams, int V, double b_target,
                                                double sigma_b, double alpha_min, int32_t* __restrict__ ref) {
    const int tv = blockIdx.x * 64 + threadIdx.x;
    if (tv >= V) return;
    const Cam64 a = cam64(cams[tv]);
    double ca[3];
    for (int k = 0; k < 3; ++k) ca[k] = -(a.R[k] * a.t[0] + a.R[3 + k] * a.t[1] + a.R[6 + k] * a.t[2]);
    double best = -1.0;
    int arg = -1;
    for (int c = 0; c < V; ++c) {
        if (c == tv) continue;
        const Cam64 b = cam64(cams[c]);
        double d2 = 0.0, dot = 0.0;
        for (int k = 0; k < 3; ++k) {
            const double cb = -(b.R[k] * b.t[0] + b.R[3 + k] * b.t[1] + b.R[6 + k] * b.t[2]);
            d2 += (cb - ca[k]) * (cb - ca[k]);
            dot += a.R[6 + k] * b.R[6 + k];
        }
        const double base = sqrt(d2), alpha = acos(fmin(1.0, fmax(-1.0, dot)));
        const double s = exp(-(base - b_target) * (base - b_target) / (2.0 * sigma_b * sigma_b)) *
                         fmax(alpha / alpha_min, 1.0);
        if (arg < 0 || s > best) {
            best = s;
            arg = c;
        }
    }
    ref[tv] = arg;
}

// ---------------------------------------------------------------- cost volume

constexpr int kCostPix = 128;  // pixels per cost workgroup

// Workgroup: kCostPix consecutive pixels of one target, all D planes; thread
// (slot, k) handles plane k for pixels slot, slot + 256/D, ...  The relative
// pose, the plane depth d_k and the pixel rays are float64 values rounded
// to float32 (d_k once per thread, the rays once per pixel in LDS); the per
// pixel-plane sweep is unfused float32 in a fixed order.
template <int D>
__global__ __launch_bounds__(256) void k_cost(const pgs_camera* __restrict__ cams, int W, int H,
                                              const uint64_t* __restrict__ census,
                                              const int32_t* __restrict__ targets, const int32_t* __restrict__ refs,
                                              const double* __restrict__ range, uint8_t* __restrict__ cost) {
#pragma clang fp contract(off)
    constexpr int SL = 256 / D > 0 ? 256 / D : 1;  // pixel slots per pass
    __shared__ float s_pose[16];  // M, m, the reference intrinsics
    __shared__ float s_a[kCostPix], s_b[kCostPix];
    __shared__ uint64_t s_cen[kCostPix];
    const int t = threadIdx.x, ti = blockIdx.y, tv = targets[ti], rv = refs[tv];
    const uint32_t npix = (uint32_t)W * (uint32_t)H, base = blockIdx.x * kCostPix;
    // every lane reads the pose below, so it is defined without a reference too
    if (rv < 0 && t < 16) s_pose[t] = 0.0f;
    if (t == 0 && rv >= 0) {
        const Cam64 ct = cam64(cams[tv]), cr = cam64(cams[rv]);
        double M[9];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                M[3 * i + j] = cr.R[3 * i] * ct.R[3 * j] + cr.R[3 * i + 1] * ct.R[3 * j + 1] +
                               cr.R[3 * i + 2] * ct.R[3 * j + 2];
        for (int i = 0; i < 9; ++i) s_pose[i] = (float)M[i];
        for (int i = 0; i < 3; ++i)
            s_pose[9 + i] =
                (float)(cr.t[i] - (M[3 * i] * ct.t[0] + M[3 * i + 1] * ct.t[1] + M[3 * i + 2] * ct.t[2]));
        s_pose[12] = cams[rv].fx;
        s_pose[13] = cams[rv].fy;
        s_pose[14] = cams[rv].cx;
        s_pose[15] = cams[rv].cy;
    }
    for (int q = t; q < kCostPix; q += blockDim.x) {
        if (base + q >= npix) {  // the ragged tail's slots are masked but still read
            s_a[q] = s_b[q] = 0.0f;
            s_cen[q] = 0;
            continue;
        }
        const pgs_camera& c = cams[tv];
        const uint32_t pix = base + q, y = pix / (uint32_t)W, x = pix - y * (uint32_t)W;
        s_a[q] = (float)(((double)x - (double)c.cx) / (double)c.fx);
        s_b[q] = (float)(((double)y - (double)c.cy) / (double)c.fy);
        s_cen[q] = census[(size_t)tv * npix + pix];
    }
    __syncthreads();
    if (t >= SL * D) return;
    const int k = t % D, slot = t / D;
    const double d_min = range[2 * tv], d_max = range[2 * tv + 1];
    // no reference (a single view) or an empty range: every cost is the out cost
    const bool ranged = rv >= 0 && d_min > 0.0 && d_max > d_min;
    float d = 0.0f;
    if (ranged) {
        const double inv_far = 1.0 / d_max;
        const double h = (1.0 / d_min - inv_far) / (double)(D - 1);
        d = (float)(1.0 / (inv_far + (double)k * h));
    }
    const float* M = s_pose;
    const float wmax = (float)(W - 1), hmax = (float)(H - 1);
    const uint64_t* rc = census + (size_t)(rv >= 0 ? rv : tv) * npix;
    uint8_t* out = cost + ((size_t)ti * npix + base) * D + k;
    // four pixels per round with their gathers issued together: an invalid
    // sample reads the reference's pixel 0 and is replaced by the out cost
    static_assert(kCostPix % (4 * SL) == 0, "pixel rounds must tile the workgroup");
    for (int i0 = slot; i0 < kCostPix; i0 += 4 * SL) {
        uint64_t g[4];
        bool ok[4];
#pragma unroll
        for (int u4 = 0; u4 < 4; ++u4) {
            const int i = i0 + u4 * SL;
            // evaluated everywhere and masked (no divergent branch)
            const float X = d * s_a[i], Y = d * s_b[i], Z = d;
            const float xr = M[0] * X + M[1] * Y + M[2] * Z + M[9];
            const float yr = M[3] * X + M[4] * Y + M[5] * Z + M[10];
            const float zr = M[6] * X + M[7] * Y + M[8] * Z + M[11];
            const float u = floorf(M[12] * (xr / zr) + M[14] + 0.5f);
            const float v = floorf(M[13] * (yr / zr) + M[15] + 0.5f);
            ok[u4] = ranged && base + i < npix && zr > 0.0f && u >= 0.0f && u <= wmax && v >= 0.0f && v <= hmax;
            const size_t idx = (size_t)(uint32_t)(ok[u4] ? v : 0.0f) * W + (size_t)(uint32_t)(ok[u4] ? u : 0.0f);
            g[u4] = rc[idx];
        }
#pragma unroll
        for (int u4 = 0; u4 < 4; ++u4) {
            const int i = i0 + u4 * SL;
            if (base + i < npix) out[(size_t)i * D] = (uint8_t)(ok[u4] ? __popcll(s_cen[i] ^ g[u4]) : kCostOut);
        }
    }
}

// ---------------------------------------------------------------- SGM

constexpr int kIntMax = 0x7fffffff;

// Minimum over the wave, returned to every lane: an inclusive min-scan
// inside each row of 16 lanes (DPP row shifts), folded across rows with
// row broadcasts (lane 63 ends with the total), then read from lane 63.
__device__ __forceinline__ int wave_min_all(int v) {
    v = min(v, __builtin_amdgcn_update_dpp(kIntMax, v, 0x111, 0xf, 0xf, false));
    v = min(v, __builtin_amdgcn_update_dpp(kIntMax, v, 0x112, 0xf, 0xf, false));
    v = min(v, __builtin_amdgcn_update_dpp(kIntMax, v, 0x114, 0xf, 0xf, false));
    v = min(v, __builtin_amdgcn_update_dpp(kIntMax, v, 0x118, 0xf, 0xf, false));
    v = min(v, __builtin_amdgcn_update_dpp(kIntMax, v, 0x142, 0xa, 0xf, false));
    v = min(v, __builtin_amdgcn_update_dpp(kIntMax, v, 0x143, 0xc, 0xf, false));
    return __builtin_amdgcn_readlane(v, 63);
}

// Value of lane l - 1 (wave shift right by one), `edge` in lane 0.
__device__ __forceinline__ int from_lower_lane(int v, int edge) {
    return __builtin_amdgcn_update_dpp(edge, v, 0x138, 0xf, 0xf, false);
}

// Value of lane l + 1 (wave shift left by one), `edge` in lane 63.
__device__ __forceinline__ int from_upper_lane(int v, int edge) {
    return __builtin_amdgcn_update_dpp(edge, v, 0x130, 0xf, 0xf, false);
}

struct SgmArgs {
    const uint8_t* cost;
    uint8_t* lbuf;       // forward path costs of the line being swept [T][H][W][D]
    uint16_t* agg;       // path-cost sum [T][H][W][D]
    bool agg_total;      // the last pass also stores the full sum
    const int32_t* targets;
    const double* range;
    float* depth;        // [T][H][W]
    float* conf;
    int W, H, p1, p2;
    double keep_ratio;   // 1 - confidence threshold
};

// Lane l holds planes KPL l .. KPL l + KPL - 1 of a pixel: its costs are KPL
// consecutive bytes and its sums KPL consecutive uint16, loaded as one word
// where KPL allows and kept packed until used.
template <int KPL> struct SumWord { typedef uint64_t type; };
template <> struct SumWord<1> { typedef uint32_t type; };
template <> struct SumWord<2> { typedef uint32_t type; };

template <int KPL>
struct LanePack {
    typedef typename SumWord<KPL>::type G;
    __device__ static void load(const uint8_t* c, const uint16_t* g, bool with_g, uint32_t& cw, G& gw) {
        if (KPL == 2) {
            cw = *reinterpret_cast<const uint16_t*>(c);
            gw = with_g ? *reinterpret_cast<const uint32_t*>(g) : 0u;
        } else if (KPL == 4) {
            cw = *reinterpret_cast<const uint32_t*>(c);
            gw = with_g ? (G)*reinterpret_cast<const uint64_t*>(g) : (G)0;
        } else {
            cw = 0;
            gw = 0;
#pragma unroll
            for (int j = 0; j < KPL; ++j) {
                cw |= (uint32_t)c[j] << (8 * j);
                if (with_g) gw |= (G)g[j] << (16 * j);
            }
        }
    }
    __device__ static uint32_t load_bytes(const uint8_t* c) {
        if (KPL == 2) return *reinterpret_cast<const uint16_t*>(c);
        if (KPL == 4) return *reinterpret_cast<const uint32_t*>(c);
        uint32_t w = 0;
#pragma unroll
        for (int j = 0; j < KPL; ++j) w |= (uint32_t)c[j] << (8 * j);
        return w;
    }
    __device__ static void store_bytes(uint8_t* c, const int (&v)[KPL]) {
        if (KPL == 2) {
            *reinterpret_cast<uint16_t*>(c) = (uint16_t)((uint32_t)v[0] | ((uint32_t)v[1] << 8));
        } else if (KPL == 4) {
            *reinterpret_cast<uint32_t*>(c) =
                (uint32_t)v[0] | ((uint32_t)v[1] << 8) | ((uint32_t)v[2] << 16) | ((uint32_t)v[3] << 24);
        } else {
#pragma unroll
            for (int j = 0; j < KPL; ++j) c[j] = (uint8_t)v[j];
        }
    }
    __device__ static G load_sums(const uint16_t* g) {
        if (KPL == 2) return *reinterpret_cast<const uint32_t*>(g);
        if (KPL == 4) return (G)*reinterpret_cast<const uint64_t*>(g);
        G w = 0;
#pragma unroll
        for (int j = 0; j < KPL; ++j) w |= (G)g[j] << (16 * j);
        return w;
    }
    __device__ static int cost(uint32_t cw, int j) { return (int)((cw >> (8 * j)) & 255u); }
    __device__ static int sum(G gw, int j) { return (int)((gw >> (16 * j)) & 0xffffu); }
    __device__ static void store(uint16_t* g, const int (&v)[KPL]) {
        if (KPL == 2) {
            *reinterpret_cast<uint32_t*>(g) = (uint32_t)v[0] | ((uint32_t)v[1] << 16);
        } else if (KPL == 4) {
            *reinterpret_cast<uint64_t*>(g) = (uint64_t)(uint32_t)v[0] | ((uint64_t)(uint32_t)v[1] << 16) |
                                              ((uint64_t)(uint32_t)v[2] << 32) | ((uint64_t)(uint32_t)v[3] << 48);
        } else {
#pragma unroll
            for (int j = 0; j < KPL; ++j) g[j] = (uint16_t)v[j];
        }
    }
};

// One sweep of a wave along its line.  kForward: path costs to lbuf (bytes,
// every value <= 48 + p2 <= 255 is checked on the host); kRowsBack: the
// opposite direction, the two rows' path costs summed into agg; kColsBack:
// the opposite column direction added to the row sum and lbuf's forward
// column costs, then per pixel the winner and the confidence-test sums
// (recorded in lane step mod 64 and turned into refined depths 64 pixels
// at a time).
enum SweepMode { kForward = 0, kRowsBack = 1, kColsBack = 2 };
constexpr int kSgmRing = 32;  // column steps staged in LDS per wave

template <int KPL, int MODE>
__device__ __forceinline__ void sgm_sweep(const SgmArgs& a, int line, int ti, bool rows, bool rev,
                                          uint16_t* ring) {
#pragma clang fp contract(off)
    constexpr int D = 64 * KPL;
    constexpr int kBig = 1 << 28;
    constexpr int PF = 8;
    typedef LanePack<KPL> LP;
    typedef typename LP::G G;
    const int lane = threadIdx.x & 63;
    const int n = rows ? a.W : a.H;
    const size_t npix = (size_t)a.W * a.H;
    const long long p0 = rows ? (long long)line * a.W + (rev ? a.W - 1 : 0)
                              : (long long)(rev ? a.H - 1 : 0) * a.W + line;
    const long long dp = rows ? (rev ? -1 : 1) : (rev ? -(long long)a.W : (long long)a.W);
    const size_t off = (size_t)ti * npix * D + KPL * lane;
    const uint8_t* cbase = a.cost + off;
    uint8_t* lbase = a.lbuf + off;
    uint16_t* abase = a.agg + off;
    double inv_far = 0.0, h = 0.0;
    if (MODE == kColsBack) {
        const int tv = a.targets[ti];
        const double d_min = a.range[2 * tv], d_max = a.range[2 * tv + 1];
        inv_far = 1.0 / d_max;
        h = (1.0 / d_min - inv_far) / (double)(D - 1);
    }
    int L[KPL];
    uint32_t cc[PF], cn[PF], fc[PF], fn[PF];
    G ac[PF], an[PF];
    auto load = [&](int s, uint32_t& c, uint32_t& f, G& g) {
        if (s < n) {
            const size_t e = (size_t)(p0 + dp * s) * D;
            c = LP::load_bytes(cbase + e);
            if (MODE != kForward) f = LP::load_bytes(lbase + e);
            if (MODE == kColsBack) g = LP::load_sums(abase + e);
        }
    };
    // column back sweep: the full sums of kSgmRing consecutive steps sit in
    // this wave's LDS ring (row = step mod kSgmRing, D + 2 uint16 per row so
    // that the lanes' rows fall in different banks); lanes p and p + 32 then
    // take the winner, the second minimum two planes away and the winner's
    // neighbours of step p over one half of the planes each, combined by a
    // lane swap, and lane p writes that pixel's depth and confidence
    constexpr int RS = D + 2;
    constexpr int RING = kSgmRing;
    auto flush = [&](int s_first, int count) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // lanes p and p + 32 take step p, each over half of the planes
        const int px = lane & 31, half = lane >> 5;
        const bool act = px < count;
        const uint32_t* r = reinterpret_cast<const uint32_t*>(ring + px * RS) + half * (D / 4);
        const int k0 = half * (D / 2);
        int key = kBig;  // (sum << 8) | plane, smallest first
        if (act) {
#pragma unroll 4
            for (int c = 0; c < D / 4; ++c) {
                const uint32_t w = r[c];
                key = min(key, (int)((w & 0xffffu) << 8) | (k0 + 2 * c));
                key = min(key, (int)((w >> 16) << 8) | (k0 + 2 * c + 1));
            }
        }
        key = min(key, __shfl_xor(key, 32));
        const int s1 = key >> 8, kw = key & 255;
        int s2 = kBig;
        if (act) {
#pragma unroll 4
            for (int c = 0; c < D / 4; ++c) {
                const uint32_t w = r[c];
                const int ka = k0 + 2 * c, kb = ka + 1;
                if (ka - kw >= 2 || kw - ka >= 2) s2 = min(s2, (int)(w & 0xffffu));
                if (kb - kw >= 2 || kw - kb >= 2) s2 = min(s2, (int)(w >> 16));
            }
        }
        s2 = min(s2, __shfl_xor(s2, 32));
        if (act && half == 0) {
            const uint16_t* rh = ring + px * RS;
            const int vm = rh[kw > 0 ? kw - 1 : 0], vq = rh[kw < D - 1 ? kw + 1 : D - 1];
            const bool keep = kw > 0 && kw < D - 1 && s2 > 0 && (double)s1 <= a.keep_ratio * (double)s2;
            float dout = 0.0f;
            if (keep) {
                const int den = vm - 2 * s1 + vq;
                const double delta = den > 0 ? (double)(vm - vq) / (2.0 * (double)den) : 0.0;
                dout = (float)(1.0 / (inv_far + ((double)kw + delta) * h));
            }
            const size_t o = (size_t)ti * npix + (size_t)(p0 + dp * (s_first + px));
            a.depth[o] = dout;
            a.conf[o] = s2 > 0 ? (float)(1.0 - (double)s1 / (double)s2) : 0.0f;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
#pragma unroll
    for (int q = 0; q < PF; ++q) load(q, cc[q], fc[q], ac[q]);
    for (int s0 = 0; s0 < n; s0 += PF) {
#pragma unroll
        for (int q = 0; q < PF; ++q) load(s0 + PF + q, cn[q], fn[q], an[q]);
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            const int s = s0 + q;
            if (s >= n) break;
            if (s == 0) {
#pragma unroll
                for (int j = 0; j < KPL; ++j) L[j] = LP::cost(cc[q], j);
            } else {
                int m = L[0];
#pragma unroll
                for (int j = 1; j < KPL; ++j) m = min(m, L[j]);
                m = wave_min_all(m);
                // plane k - 1 of the lane's first plane is the previous
                // lane's last; k + 1 of its last is the next lane's first
                const int below = from_lower_lane(L[KPL - 1], kBig);
                const int above = from_upper_lane(L[0], kBig);
                int Ln[KPL];
#pragma unroll
                for (int j = 0; j < KPL; ++j) {
                    const int km1 = j > 0 ? L[j - 1] : below;
                    const int kp1 = j + 1 < KPL ? L[j + 1] : above;
                    const int best = min(min(L[j], km1 + a.p1), min(kp1 + a.p1, m + a.p2));
                    Ln[j] = LP::cost(cc[q], j) + best - m;
                }
#pragma unroll
                for (int j = 0; j < KPL; ++j) L[j] = Ln[j];
            }
            const size_t e = (size_t)(p0 + dp * s) * D;
            if (MODE == kForward) {
                LP::store_bytes(lbase + e, L);
            } else if (MODE == kRowsBack) {
                int S[KPL];
#pragma unroll
                for (int j = 0; j < KPL; ++j) S[j] = LP::cost(fc[q], j) + L[j];
                LP::store(abase + e, S);
            } else {
                int S[KPL];
#pragma unroll
                for (int j = 0; j < KPL; ++j) S[j] = LP::sum(ac[q], j) + LP::cost(fc[q], j) + L[j];
                if (a.agg_total) LP::store(abase + e, S);
                uint16_t* rw = ring + (s & (RING - 1)) * RS + KPL * lane;
                if (KPL == 2) {
                    *reinterpret_cast<uint32_t*>(rw) = (uint32_t)S[0] | ((uint32_t)S[1] << 16);
                } else {
#pragma unroll
                    for (int j = 0; j < KPL; ++j) rw[j] = (uint16_t)S[j];
                }
                if ((s & (RING - 1)) == RING - 1 || s == n - 1) flush(s & ~(RING - 1), (s & (RING - 1)) + 1);
            }
        }
#pragma unroll
        for (int q = 0; q < PF; ++q) {
            cc[q] = cn[q];
            fc[q] = fn[q];
            ac[q] = an[q];
        }
    }
}

// Rows (COLS = false): left to right into lbuf, then right to left summed
// with it into agg.  Columns (COLS = true): top to bottom into lbuf, then
// bottom to top with the winner.  One wave per line, four lines per
// workgroup; the second sweep reads what the same wave stored.
template <int KPL, bool COLS>
__global__ __launch_bounds__(256) void k_sgm(SgmArgs a) {
    extern __shared__ uint16_t sgm_ring[];  // columns: [4 waves][kSgmRing steps][64 KPL + 2]
    const int line = blockIdx.x * 4 + (threadIdx.x >> 6), ti = blockIdx.y;
    if (line >= (COLS ? a.W : a.H)) return;
    uint16_t* ring = sgm_ring + (threadIdx.x >> 6) * kSgmRing * (64 * KPL + 2);
    sgm_sweep<KPL, kForward>(a, line, ti, !COLS, false, ring);
    if (COLS) sgm_sweep<KPL, kColsBack>(a, line, ti, false, true, ring);
    else sgm_sweep<KPL, kRowsBack>(a, line, ti, true, true, ring);
}

template <int KPL>
constexpr size_t sgm_ring_bytes() { return (size_t)4 * kSgmRing * (64 * KPL + 2) * sizeof(uint16_t); }

// ---------------------------------------------------------------- fusion

__global__ __launch_bounds__(256) void k_fuse_count(const float* __restrict__ depth, int W,
                                                    uint32_t* __restrict__ rowcnt) {
    const size_t row = blockIdx.x;
    const float* d = depth + row * W;
    int c = 0;
    for (int x = threadIdx.x; x < W; x += 256) c += d[x] > 0.0f;
    __shared__ int s[256];
    s[threadIdx.x] = c;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) rowcnt[row] = (uint32_t)s[0];
}

// Exclusive scan of the row counts (one workgroup); total to *total.
__global__ __launch_bounds__(1024) void k_fuse_scan(uint32_t* __restrict__ rows, int n, uint32_t* __restrict__ total) {
    __shared__ uint32_t s[1024];
    uint32_t carry = 0;
    for (int base = 0; base < n; base += 1024) {
        const int i = base + threadIdx.x;
        const uint32_t v = i < n ? rows[i] : 0u;
        s[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            const uint32_t add = threadIdx.x >= (unsigned)o ? s[threadIdx.x - o] : 0u;
            __syncthreads();
            s[threadIdx.x] += add;
            __syncthreads();
        }
        if (i < n) rows[i] = carry + s[threadIdx.x] - v;
        carry += s[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = carry;
}

// Kept pixel number idx (row-major over the targets) becomes point idx / stride
// when idx is a multiple of stride: world position into out [3][capacity]
// and, with grey given, its intensity / 255 into colour [3][capacity].
__global__ __launch_bounds__(256) void k_fuse_write(const pgs_camera* __restrict__ cams,
                                                    const int32_t* __restrict__ targets, int W, int H,
                                                    const float* __restrict__ depth,
                                                    const uint32_t* __restrict__ rowoff, const uint8_t* __restrict__ grey,
                                                    uint32_t stride, float* __restrict__ out,
                                                    float* __restrict__ colour, uint32_t capacity) {
    __shared__ uint32_t wcnt[4];
    const size_t row = blockIdx.x;
    const int ti = (int)(row / H), y = (int)(row - (size_t)ti * H);
    const Cam64 c = cam64(cams[targets[ti]]);
    const float* d = depth + row * W;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint32_t base = rowoff[row];
    for (int x0 = 0; x0 < W; x0 += 256) {
        const int x = x0 + threadIdx.x;
        const float z = x < W ? d[x] : 0.0f;
        const bool keep = z > 0.0f;
        const uint64_t b = __ballot(keep);
        if (lane == 0) wcnt[wv] = (uint32_t)__popcll(b);
        __syncthreads();
        uint32_t before = 0, all = 0;
        for (int w = 0; w < 4; ++w) {
            before += w < wv ? wcnt[w] : 0u;
            all += wcnt[w];
        }
        const uint32_t idx = base + before + (uint32_t)__popcll(b & ((1ull << lane) - 1ull));
        const uint32_t o = idx / stride;
        if (keep && idx == o * stride && o < capacity) {
            const double zz = z;
            const double X = zz * (((double)x - c.cx) / c.fx) - c.t[0];
            const double Y = zz * (((double)y - c.cy) / c.fy) - c.t[1];
            const double Z = zz - c.t[2];
            for (int k = 0; k < 3; ++k)
                out[(size_t)k * capacity + o] = (float)(c.R[k] * X + c.R[3 + k] * Y + c.R[6 + k] * Z);
            if (colour) {
                const float v = (float)grey[((size_t)targets[ti] * H + y) * W + x] / 255.0f;
                for (int k = 0; k < 3; ++k) colour[(size_t)k * capacity + o] = v;
            }
        }
        base += all;
        __syncthreads();
    }
}

inline size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

pgs_status check_params(const pgs_mvs_params* p, const char* who) {
    PGS_REQUIRE(p, "%s: null params", who);
    PGS_REQUIRE(p->n_planes == 64 || p->n_planes == 128 || p->n_planes == 192 || p->n_planes == 256,
                "%s: n_planes %d not 64, 128, 192 or 256", who, p->n_planes);
    PGS_REQUIRE(p->p1 >= 0 && p->p2 >= 0 && p->p1 <= 1000 && p->p2 <= 1000, "%s: penalties %d, %d not in 0..1000",
                who, p->p1, p->p2);
    PGS_REQUIRE(p->conf_min >= 0.0 && p->conf_min <= 1.0, "%s: conf_min not in [0, 1]", who);
    return PGS_OK;
}

template <int KPL>
pgs_status launch_sgm(SgmArgs a, int n_targets, hipStream_t s) {
    static const bool lds_ok = hipFuncSetAttribute(reinterpret_cast<const void*>(k_sgm<KPL, true>),
                                                   hipFuncAttributeMaxDynamicSharedMemorySize,
                                                   (int)sgm_ring_bytes<KPL>()) == hipSuccess;
    PGS_REQUIRE(lds_ok, "pgs_mvs_sgm: cannot reserve %zu bytes of LDS", sgm_ring_bytes<KPL>());
    k_sgm<KPL, false><<<dim3((a.H + 3) / 4, n_targets), 256, 0, s>>>(a);
    k_sgm<KPL, true><<<dim3((a.W + 3) / 4, n_targets), 256, sgm_ring_bytes<KPL>(), s>>>(a);
    PGS_CHECK_LAUNCH("pgs_mvs_sgm");
    return PGS_OK;
}

}  // namespace

extern "C" pgs_status pgs_mvs_census(const uint8_t* grey_dev, int32_t n_views, int32_t width, int32_t height,
                                     uint64_t* census_dev, void* stream) {
    PGS_REQUIRE(n_views >= 0 && width >= 0 && height >= 0, "pgs_mvs_census: negative size");
    if (n_views == 0 || width == 0 || height == 0) return PGS_OK;
    PGS_REQUIRE(grey_dev && census_dev, "pgs_mvs_census: null pointer");
    PGS_REQUIRE(n_views <= 65535, "pgs_mvs_census: more than 65535 views");
    const dim3 grid((width + kTile - 1) / kTile, (height + kTile - 1) / kTile, n_views);
    k_census<<<grid, 256, 0, pgs::as_stream(stream)>>>(grey_dev, width, height, census_dev);
    PGS_CHECK_LAUNCH("pgs_mvs_census");
    return PGS_OK;
}

extern "C" size_t pgs_mvs_range_workspace(int32_t n_views, int32_t n_points) {
    if (n_views <= 0 || n_points < 0) return 0;
    return al256((size_t)n_views * n_points * 8);
}

extern "C" pgs_status pgs_mvs_depth_range(const pgs_camera* cams_dev, int32_t n_views, int32_t width, int32_t height,
                                          const double* points_dev, int32_t n_points, double* range_dev,
                                          void* workspace_dev, size_t workspace_bytes, void* stream) {
    PGS_REQUIRE(n_views >= 0 && n_points >= 0 && width > 0 && height > 0, "pgs_mvs_depth_range: bad size");
    if (n_views == 0) return PGS_OK;
    PGS_REQUIRE(n_views <= 65535, "pgs_mvs_depth_range: more than 65535 views");
    PGS_REQUIRE(cams_dev && range_dev && (points_dev || n_points == 0) && workspace_dev,
                "pgs_mvs_depth_range: null pointer");
    PGS_REQUIRE(workspace_bytes >= pgs_mvs_range_workspace(n_views, n_points),
                "pgs_mvs_depth_range: workspace %zu < %zu", workspace_bytes,
                pgs_mvs_range_workspace(n_views, n_points));
    hipStream_t s = pgs::as_stream(stream);
    uint64_t* keys = static_cast<uint64_t*>(workspace_dev);
    if (n_points > 0)
        k_mvs_depths<<<dim3((n_points + 255) / 256, n_views), 256, 0, s>>>(cams_dev, width, height, points_dev,
                                                                           n_points, keys);
    k_mvs_range<<<n_views, 1024, 0, s>>>(n_points, keys, range_dev);
    PGS_CHECK_LAUNCH("pgs_mvs_depth_range");
    return PGS_OK;
}

extern "C" pgs_status pgs_mvs_select_ref(const pgs_camera* cams_dev, int32_t n_views, const pgs_mvs_params* params,
                                         int32_t* ref_dev, void* stream) {
    PGS_REQUIRE(n_views >= 0, "pgs_mvs_select_ref: negative size");
    if (n_views == 0) return PGS_OK;
    PGS_REQUIRE(cams_dev && ref_dev && params, "pgs_mvs_select_ref: null pointer");
    PGS_REQUIRE(params->sigma_b > 0.0 && params->alpha_min > 0.0, "pgs_mvs_select_ref: sigma_b, alpha_min must be > 0");
    k_mvs_ref<<<(n_views + 63) / 64, 64, 0, pgs::as_stream(stream)>>>(cams_dev, n_views, params->b_target,
                                                                      params->sigma_b, params->alpha_min, ref_dev);
    PGS_CHECK_LAUNCH("pgs_mvs_select_ref");
    return PGS_OK;
}

extern "C" pgs_status pgs_mvs_cost(const pgs_camera* cams_dev, int32_t width, int32_t height,
                                   const uint64_t* census_dev, const int32_t* targets_dev, int32_t n_targets,
                                   const int32_t* ref_dev, const double* range_dev, const pgs_mvs_params* params,
                                   uint8_t* cost_dev, void* stream) {
    if (pgs_status st = check_params(params, "pgs_mvs_cost")) return st;
    PGS_REQUIRE(n_targets >= 0 && width > 0 && height > 0, "pgs_mvs_cost: bad size");
    if (n_targets == 0) return PGS_OK;
    PGS_REQUIRE(n_targets <= 65535, "pgs_mvs_cost: more than 65535 targets");
    PGS_REQUIRE(cams_dev && census_dev && targets_dev && ref_dev && range_dev && cost_dev, "pgs_mvs_cost: null pointer");
    const int D = params->n_planes;
    const long long npix = (long long)width * height;
    PGS_REQUIRE(npix < (1ll << 31), "pgs_mvs_cost: image too large");
    hipStream_t s = pgs::as_stream(stream);
    const dim3 grid((unsigned)((npix + kCostPix - 1) / kCostPix), n_targets);
    switch (D) {
        case 64: k_cost<64><<<grid, 256, 0, s>>>(cams_dev, width, height, census_dev, targets_dev, ref_dev, range_dev, cost_dev); break;
        case 128: k_cost<128><<<grid, 256, 0, s>>>(cams_dev, width, height, census_dev, targets_dev, ref_dev, range_dev, cost_dev); break;
        case 192: k_cost<192><<<grid, 256, 0, s>>>(cams_dev, width, height, census_dev, targets_dev, ref_dev, range_dev, cost_dev); break;
        default: k_cost<256><<<grid, 256, 0, s>>>(cams_dev, width, height, census_dev, targets_dev, ref_dev, range_dev, cost_dev); break;
    }
    PGS_CHECK_LAUNCH("pgs_mvs_cost");
    return PGS_OK;
}

extern "C" size_t pgs_mvs_sgm_workspace(int32_t n_targets, int32_t width, int32_t height, int32_t n_planes) {
    if (n_targets <= 0 || width <= 0 || height <= 0 || n_planes <= 0) return 0;
    const size_t e = (size_t)n_targets * width * height * n_planes;
    return al256(e) + al256(e * 2);
}

extern "C" pgs_status pgs_mvs_sgm(const uint8_t* cost_dev, int32_t width, int32_t height, const int32_t* targets_dev,
                                  int32_t n_targets, const double* range_dev, const pgs_mvs_params* params,
                                  float* depth_dev, float* conf_dev, uint16_t* agg_out_dev, void* workspace_dev,
                                  size_t workspace_bytes, void* stream) {
    if (pgs_status st = check_params(params, "pgs_mvs_sgm")) return st;
    PGS_REQUIRE(n_targets >= 0 && width > 0 && height > 0, "pgs_mvs_sgm: bad size");
    if (n_targets == 0) return PGS_OK;
    PGS_REQUIRE(n_targets <= 65535, "pgs_mvs_sgm: more than 65535 targets");
    PGS_REQUIRE(cost_dev && targets_dev && range_dev && depth_dev && conf_dev, "pgs_mvs_sgm: null pointer");
    PGS_REQUIRE(workspace_dev && workspace_bytes >= pgs_mvs_sgm_workspace(n_targets, width, height,
                                                                           params->n_planes),
                "pgs_mvs_sgm: workspace too small");
    PGS_REQUIRE(48 + params->p2 <= 255, "pgs_mvs_sgm: path costs up to %d do not fit a byte", 48 + params->p2);
    const size_t e = (size_t)n_targets * width * height * params->n_planes;
    SgmArgs a{};
    a.cost = cost_dev;
    a.lbuf = static_cast<uint8_t*>(workspace_dev);
    a.agg = agg_out_dev ? agg_out_dev : reinterpret_cast<uint16_t*>(static_cast<char*>(workspace_dev) + al256(e));
    a.agg_total = agg_out_dev != nullptr;
    a.targets = targets_dev;
    a.range = range_dev;
    a.depth = depth_dev;
    a.conf = conf_dev;
    a.W = width;
    a.H = height;
    a.p1 = params->p1;
    a.p2 = params->p2;
    a.keep_ratio = 1.0 - params->conf_min;
    hipStream_t s = pgs::as_stream(stream);
    switch (params->n_planes) {
        case 64: return launch_sgm<1>(a, n_targets, s);
        case 128: return launch_sgm<2>(a, n_targets, s);
        case 192: return launch_sgm<3>(a, n_targets, s);
        default: return launch_sgm<4>(a, n_targets, s);
    }
}

extern "C" size_t pgs_mvs_fuse_workspace(int32_t n_targets, int32_t height) {
    if (n_targets <= 0 || height <= 0) return 0;
    return al256((size_t)n_targets * height * 4);
}

extern "C" pgs_status pgs_mvs_fuse(const pgs_camera* cams_dev, const int32_t* targets_dev, int32_t n_targets,
                                   int32_t width, int32_t height, const float* depth_dev, const uint8_t* grey_dev,
                                   uint32_t stride, float* points_dev, float* colour_dev, uint32_t capacity,
                                   uint32_t* count_dev, void* workspace_dev, size_t workspace_bytes, void* stream) {
    PGS_REQUIRE(n_targets >= 0 && width > 0 && height > 0 && stride >= 1, "pgs_mvs_fuse: bad size or stride");
    PGS_REQUIRE(count_dev, "pgs_mvs_fuse: null count");
    PGS_REQUIRE(!colour_dev || grey_dev, "pgs_mvs_fuse: colours need the grey images");
    hipStream_t s = pgs::as_stream(stream);
    if (n_targets == 0) {
        k_mvs_clear<<<1, 256, 0, s>>>(count_dev, 1);
        PGS_CHECK_LAUNCH("pgs_mvs_fuse");
        return PGS_OK;
    }
    PGS_REQUIRE(cams_dev && targets_dev && depth_dev && (points_dev || capacity == 0) && workspace_dev,
                "pgs_mvs_fuse: null pointer");
    PGS_REQUIRE(workspace_bytes >= pgs_mvs_fuse_workspace(n_targets, height), "pgs_mvs_fuse: workspace too small");
    const long long rows = (long long)n_targets * height;
    PGS_REQUIRE(rows < (1ll << 31), "pgs_mvs_fuse: too many rows");
    uint32_t* rowcnt = static_cast<uint32_t*>(workspace_dev);
    k_fuse_count<<<(unsigned)rows, 256, 0, s>>>(depth_dev, width, rowcnt);
    k_fuse_scan<<<1, 1024, 0, s>>>(rowcnt, (int)rows, count_dev);
    k_fuse_write<<<(unsigned)rows, 256, 0, s>>>(cams_dev, targets_dev, width, height, depth_dev, rowcnt, grey_dev,
                                                stride, points_dev, colour_dev, capacity);
    PGS_CHECK_LAUNCH("pgs_mvs_fuse");
    return PGS_OK;
}
