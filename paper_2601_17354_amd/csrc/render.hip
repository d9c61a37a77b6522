// Per-tile compositing forward and its backward.
//
// Forward (PocketGS Sec. "Explicit Computation Graph", "Bandwidth-Efficient
// Forward Replay Cache"): one workgroup per tile, one lane per pixel.  The
// tile's sorted splat list is staged through LDS in batches (one splat per
// lane per batch, 36 B of 2D attributes each) and every wave steps through
// the batch in lockstep, each lane compositing its pixel front to back.  A
// barrier with a live-lane count ends the tile once every pixel terminated.
//
// Replay trace.  S = {id, C_in, alpha} is recorded per wave of 64 pixels as
// groups, one per sorted splat id that at least one of the wave's pixels
// composited: a 64-bit ballot mask of those pixels (stored at the id's slot)
// followed by their entries, appended contiguously in lane order to the
// wave's entry region.  The id of an entry is thus the slot of its group,
// its pixel the lane of its mask bit, and a pixel's entries in group order
// are its contributors front to back.  Entry regions have the exact worst
// case size (64 entries per wave and listed splat), so nothing overflows;
// a per-wave step counter bounds the valid groups, so masks of earlier
// iterations are never read and nothing is cleared between iterations.
// Entries are written as one coalesced run per group.  After the front to
// back pass the kernel walks each wave's groups back to front with the
// splat colours re-staged in LDS and replaces alpha-only entries by
// (C_in, alpha): C_in is the colour of everything behind the splat, the
// over-recursion C_out = C_in (1 - alpha) + alpha c run from the background.
//
// Backward (equation "backward_chain"), two variants:
//   cached     steps through each wave's groups front to back, visiting only
//              non-empty masks; a lane with a bit set reads its entry, takes
//              dL/dC_out (starts at dL/dC, times (1 - alpha) after each own
//              entry), dL/dalpha = <dL/dC_out, c - C_in> and dL/dc =
//              alpha dL/dC_out, chains them to the nine 2D parameters, and the
//              wave reduces them with DPP (a lone lane writes directly).
//   recompute  walks the list back to front from n_contrib, re-evaluates
//              alpha with the forward's exact arithmetic, recovers
//              T_k = T_{k+1} / (1 - alpha_k) from T_final and accumulates the
//              colour behind as it goes (the 3D Gaussian Splatting backward).
// Per-wave partial sums meet in LDS and leave with one float atomic per
// field and (tile, splat), scattered to the canonical index values[id]
// (index-mapping equation).
#include "common.hpp"

// Trace groups whose entries a wave loads before consuming the first one.
#ifndef PGS_TRACE_GROUPS
#define PGS_TRACE_GROUPS 4
#endif

namespace {

using pgs::kAlphaMax;
using pgs::kAlphaMin;
using pgs::kTMin;

struct Splat {
    float u, v, A, B, C, o, r, g, b;
};

// Alpha of a splat at pixel centre (px, py).  Evaluated with contraction off
// so that the forward and the recompute backward produce identical bits.
__device__ __forceinline__ bool splat_alpha(const Splat& s, float px, float py, float& alpha,
                                            float& gauss, float& dx, float& dy) {
#pragma clang fp contract(off)
    dx = s.u - px;
    dy = s.v - py;
    const float power = -0.5f * (s.A * dx * dx + s.C * dy * dy) - s.B * dx * dy;
    if (power > 0.f) return false;
    gauss = __expf(power);
    alpha = fminf(kAlphaMax, s.o * gauss);
    return alpha >= kAlphaMin;
}

__device__ __forceinline__ void stage_splat(const float* __restrict__ proj, int n, uint32_t g,
                                            float4* sa, float4* sb, float* sc, int slot) {
    sa[slot] = make_float4(proj[(size_t)PGS_PROJ_U * n + g], proj[(size_t)PGS_PROJ_V * n + g],
                           proj[(size_t)PGS_PROJ_A * n + g], proj[(size_t)PGS_PROJ_B * n + g]);
    sb[slot] = make_float4(proj[(size_t)PGS_PROJ_C * n + g], proj[(size_t)PGS_PROJ_OPACITY * n + g],
                           proj[(size_t)PGS_PROJ_R * n + g], proj[(size_t)PGS_PROJ_G * n + g]);
    sc[slot] = proj[(size_t)PGS_PROJ_BLUE * n + g];
}

__device__ __forceinline__ Splat load_splat(const float4* sa, const float4* sb, const float* sc, int k) {
    const float4 a = sa[k], b = sb[k];
    return Splat{a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w, sc[k]};
}

__device__ __forceinline__ uint32_t lane_rank(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ __forceinline__ uint64_t read_lane64(uint64_t v, int lane) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
    return ((uint64_t)hi << 32) | lo;
}

struct Trace {
    uint64_t* mask;    // [pair_cap][NW]
    uint32_t* steps;   // [n_tiles][NW]
    float4* entry;     // [entry_cap] (C_in r, g, b, alpha)
    uint32_t* count;   // [H*W]
    size_t entry_cap;
    uint32_t pair_cap;
};

template <int TW, int TH, bool CACHED>
__global__ __launch_bounds__(TW* TH) void k_render_fwd(
    int W, int H, int TX, int tile_offset, int n_tiles_total, const float* __restrict__ proj, int n,
    const uint32_t* __restrict__ values, const uint32_t* __restrict__ ranges, float bg0, float bg1,
    float bg2, float* __restrict__ image, float* __restrict__ t_final,
    uint32_t* __restrict__ n_contrib, Trace tr, uint32_t* __restrict__ flags,
    const uint32_t* __restrict__ order) {
    constexpr int NT = TW * TH;
    constexpr int NW = NT / 64;
    __shared__ float4 s_a[NT];
    __shared__ float4 s_b[NT];
    __shared__ float s_c[NT];
    __shared__ uint32_t s_steps;
    const int tile = order ? (int)order[blockIdx.x] : (int)blockIdx.x;
    const int tx = tile % TX, ty = tile / TX;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int px = tx * TW + (t % TW), py = ty * TH + (t / TW);
    const bool inside = px < W && py < H;
    const int gt = tile_offset + tile;
    const uint32_t start = ranges[gt], end = ranges[n_tiles_total + gt];
    const float fpx = (float)px + 0.5f, fpy = (float)py + 0.5f;

    // the trace is recorded only if this tile's pairs fit the trace buffers
    const bool rec = CACHED && end <= tr.pair_cap;
    if (CACHED && !rec && t == 0) atomicOr(flags, PGS_FLAG_CACHE_OVERFLOW);
    const size_t ebase = (size_t)NT * start + (size_t)64 * (end - start) * wv;
    uint32_t cursor = 0, steps = 0, cnt = 0;

    float T = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f;
    bool done = !inside;
    uint32_t last = 0;

    for (uint32_t base = start; base < end; base += NT) {
        if (__syncthreads_count(!done) == 0) break;
        if (base + t < end) stage_splat(proj, n, values[base + t], s_a, s_b, s_c, t);
        __syncthreads();
        const int nb = (int)min((uint32_t)NT, end - base);
        for (int k = 0; k < nb; ++k) {
            if (__ballot(!done) == 0) break;  // the whole wave has terminated
            bool contrib = false;
            float alpha = 0.f;
            if (!done) {
                const Splat s = load_splat(s_a, s_b, s_c, k);
                float gauss, dx, dy;
                if (splat_alpha(s, fpx, fpy, alpha, gauss, dx, dy)) {
                    const float test_T = T * (1.f - alpha);
                    if (test_T < kTMin) {
                        done = true;
                    } else {
                        contrib = true;
                        const float w = alpha * T;
                        C0 += w * s.r;
                        C1 += w * s.g;
                        C2 += w * s.b;
                        T = test_T;
                        last = base + k - start + 1;
                    }
                }
            }
            if (rec) {
                const uint64_t m = __ballot(contrib);
                if (lane == 0) tr.mask[(size_t)(base + k) * NW + wv] = m;
                cursor += __popcll(m);
                cnt += contrib ? 1u : 0u;
                steps = base + k - start + 1;
            }
        }
    }
    if (inside) {
        const size_t pix = (size_t)py * W + px, plane = (size_t)W * H;
        image[pix] = C0 + T * bg0;
        image[plane + pix] = C1 + T * bg1;
        image[2 * plane + pix] = C2 + T * bg2;
        t_final[pix] = T;
        n_contrib[pix] = last;
        if (CACHED) tr.count[pix] = rec ? cnt : 0u;
    }
    if (!rec) return;  // uniform for the block
    if (lane == 0) tr.steps[(size_t)gt * NW + wv] = steps;

    // Entry pass: back to front over each wave's groups with the splats
    // re-staged in LDS batch by batch (the forward batches in reverse).  Each
    // set lane re-evaluates alpha with the same arithmetic as above (same
    // bits) and writes its entry (C_in, alpha) once, C_in being the colour
    // accumulated behind the splat so far.
    if (t == 0) s_steps = 0;
    __syncthreads();
    if (lane == 0) atomicMax(&s_steps, steps);
    __syncthreads();
    const uint32_t smax = s_steps;
    float a0 = bg0, a1 = bg1, a2 = bg2;
    uint32_t cur = cursor;
    if (smax == 0) return;
    const int64_t top = (int64_t)((smax - 1) / NT) * NT;  // first position of the last batch
    for (int64_t lo = top; lo >= 0; lo -= NT) {
        const uint32_t hi = min((uint32_t)lo + NT, smax);
        __syncthreads();
        if ((uint32_t)lo + t < hi) stage_splat(proj, n, values[start + lo + t], s_a, s_b, s_c, t);
        __syncthreads();
        const uint32_t whi = min(hi, steps);
        if (whi <= (uint32_t)lo) continue;
        // chunks of 64 steps, last chunk first; one vector load fetches a
        // chunk's masks, then the non-empty ones are visited last to first
        for (int64_t c0 = lo + (int64_t)((whi - 1 - lo) / 64) * 64; c0 >= lo; c0 -= 64) {
            const uint32_t cn = min(64u, whi - (uint32_t)c0);
            const uint64_t mv = (uint32_t)lane < cn ? tr.mask[(size_t)(start + c0 + lane) * NW + wv] : 0ull;
            uint64_t any = __ballot(mv != 0ull);
            while (any) {
                const int i = 63 - __clzll(any);
                any &= ~(1ull << i);
                const uint64_t m = read_lane64(mv, i);
                cur -= __popcll(m);
                if ((m >> lane) & 1ull) {
                    const Splat s = load_splat(s_a, s_b, s_c, (int)(c0 + i - lo));
                    float a = 0.f, gauss, dx, dy;
                    splat_alpha(s, fpx, fpy, a, gauss, dx, dy);
                    tr.entry[ebase + cur + lane_rank(m)] = make_float4(a0, a1, a2, a);
                    a0 = a * s.r + (1.f - a) * a0;
                    a1 = a * s.g + (1.f - a) * a1;
                    a2 = a * s.b + (1.f - a) * a2;
                }
            }
        }
    }
}

// Nine 2D gradients of one splat at one pixel from dL/dalpha and dL/dc.
__device__ __forceinline__ void chain_2d(const Splat& s, float dx, float dy, float alpha,
                                         float dgauss_do, bool clamped, float dl_dalpha,
                                         float dc0, float dc1, float dc2, float* v) {
    float dpow = 0.f, d_o = 0.f;
    if (!clamped) {
        dpow = alpha * dl_dalpha;
        d_o = dgauss_do * dl_dalpha;
    }
    v[0] = -(s.A * dx + s.B * dy) * dpow;
    v[1] = -(s.B * dx + s.C * dy) * dpow;
    v[2] = -0.5f * dx * dx * dpow;
    v[3] = -dx * dy * dpow;
    v[4] = -0.5f * dy * dy * dpow;
    v[5] = d_o;
    v[6] = dc0;
    v[7] = dc1;
    v[8] = dc2;
}

// Adds one wave's nine gradients of splat jj into the workgroup's LDS
// accumulator: a lone contributing lane adds its own values, otherwise the
// wave sums with DPP and lane 63 adds (LDS float atomics, ds_add_f32).
template <int BG>
__device__ __forceinline__ void accumulate(const float* v, float (*acc)[BG], int lane, int jj, bool lone,
                                           bool mine) {
    if (lone) {
        if (mine) {
#pragma unroll
            for (int f = 0; f < 9; ++f) atomicAdd(&acc[f][jj], v[f]);
        }
        return;
    }
#pragma unroll
    for (int f = 0; f < 9; ++f) {
        const float sum = wave_sum_to_lane63(v[f]);
        if (lane == 63) atomicAdd(&acc[f][jj], sum);
    }
}

// One float atomic per field and splat of the batch into the canonical
// 2D-gradient rows (index map values[id]).
template <int BG>
__device__ __forceinline__ void flush_batch(float (*acc)[BG], const uint32_t* gid, int nb, int n,
                                            float* __restrict__ grad2d, int t, int NT) {
    for (int idx = t; idx < nb * 9; idx += NT) {
        const int f = idx / nb, jj = idx - f * nb;
        const float s = acc[f][jj];
        if (s != 0.f) unsafeAtomicAdd(&grad2d[(size_t)f * n + gid[jj]], s);
    }
}

template <int BG>
__device__ __forceinline__ void zero_acc(float (*acc)[BG], int t, int NT) {
    for (int idx = t; idx < 9 * BG; idx += NT) (&acc[0][0])[idx] = 0.f;
}

template <int TW, int TH>
__global__ __launch_bounds__(TW* TH) void k_render_bwd_cached(
    int W, int H, int TX, int tile_offset, int n_tiles_total, const float* __restrict__ proj, int n,
    const uint32_t* __restrict__ values, const uint32_t* __restrict__ ranges, Trace tr,
    const float* __restrict__ dl_dimage, float* __restrict__ grad2d, const uint32_t* __restrict__ order) {
    constexpr int NT = TW * TH;
    constexpr int NW = NT / 64;
    constexpr int BG = NT;
    __shared__ float4 s_a[BG];
    __shared__ float4 s_b[BG];
    __shared__ float s_c[BG];
    __shared__ uint32_t s_g[BG];
    __shared__ float s_acc[9][BG];
    __shared__ uint32_t s_steps;
    const int tile = order ? (int)order[blockIdx.x] : (int)blockIdx.x;
    const int tx = tile % TX, ty = tile / TX;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int px = tx * TW + (t % TW), py = ty * TH + (t / TW);
    const bool inside = px < W && py < H;
    const int gt = tile_offset + tile;
    const uint32_t start = ranges[gt], end = ranges[n_tiles_total + gt];
    if (end > tr.pair_cap) return;  // no trace was recorded for this tile
    const float fpx = (float)px + 0.5f, fpy = (float)py + 0.5f;
    const size_t pix = (size_t)py * W + px, plane = (size_t)W * H;
    const size_t ebase = (size_t)NT * start + (size_t)64 * (end - start) * wv;

    float g0 = 0.f, g1 = 0.f, g2 = 0.f;  // dL/dC_out of this pixel's next entry
    if (inside) {
        g0 = dl_dimage[pix];
        g1 = dl_dimage[plane + pix];
        g2 = dl_dimage[2 * plane + pix];
    }
    const uint32_t steps = tr.steps[(size_t)gt * NW + wv];
    if (t == 0) s_steps = 0;
    __syncthreads();
    if (lane == 0) atomicMax(&s_steps, steps);
    __syncthreads();
    const uint32_t smax = s_steps;
    uint32_t cursor = 0;

    for (uint32_t base = 0; base < smax; base += BG) {
        const int nb = (int)min((uint32_t)BG, smax - base);
        if (t < nb) {
            const uint32_t g = values[start + base + t];
            s_g[t] = g;
            stage_splat(proj, n, g, s_a, s_b, s_c, t);
        }
        zero_acc<BG>(s_acc, t, NT);
        __syncthreads();
        const uint32_t whi = min(base + (uint32_t)nb, steps);
        for (uint32_t c0 = base; c0 < whi; c0 += 64) {
            const uint32_t cn = min(64u, whi - c0);
            const uint64_t mv = (uint32_t)lane < cn ? tr.mask[(size_t)(start + c0 + lane) * NW + wv] : 0ull;
            uint64_t any = __ballot(mv != 0ull);
            while (any) {
                // take up to kG groups and issue all their trace loads before
                // any of them is consumed (memory-level parallelism per wave)
                constexpr int kG = PGS_TRACE_GROUPS;
                int gi[kG];
                uint64_t gm[kG];
                uint32_t gc[kG];
                uint32_t cur = cursor;
#pragma unroll
                for (int q = 0; q < kG; ++q) {
                    gi[q] = 0;
                    gm[q] = 0ull;
                    gc[q] = cur;
                    if (any) {
                        const int i = __ffsll((unsigned long long)any) - 1;
                        any &= any - 1;
                        gi[q] = i;
                        gm[q] = read_lane64(mv, i);
                        cur += __popcll(gm[q]);
                    }
                }
                float4 ent[kG];
#pragma unroll
                for (int q = 0; q < kG; ++q) {
                    ent[q] = make_float4(0.f, 0.f, 0.f, 0.f);
                    if ((gm[q] >> lane) & 1ull) ent[q] = tr.entry[ebase + gc[q] + lane_rank(gm[q])];
                }
#pragma unroll
                for (int q = 0; q < kG; ++q) {
                    const uint64_t m = gm[q];
                    if (m == 0ull) continue;  // uniform: fewer than kG groups left
                    const int jj = (int)(c0 - base) + gi[q];
                    const bool mine = (m >> lane) & 1ull;
                    float v[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
                    if (mine) {
                        const Splat s = load_splat(s_a, s_b, s_c, jj);
                        const float dx = s.u - fpx, dy = s.v - fpy;
                        const float a = ent[q].w;
                        // dL/dalpha = <dL/dC_out, c - C_in>, dL/dc = alpha dL/dC_out
                        const float dla =
                            g0 * (s.r - ent[q].x) + g1 * (s.g - ent[q].y) + g2 * (s.b - ent[q].z);
                        const bool clamped = a >= kAlphaMax;
                        chain_2d(s, dx, dy, a, clamped ? 0.f : a / s.o, clamped, dla, a * g0, a * g1,
                                 a * g2, v);
                        // dL/dC_in = dL/dC_out (1 - alpha): the next entry's dL/dC_out
                        const float om = 1.f - a;
                        g0 *= om;
                        g1 *= om;
                        g2 *= om;
                    }
                    accumulate<BG>(v, s_acc, lane, jj, __popcll(m) == 1, mine);
                }
                cursor = cur;
            }
        }
        __syncthreads();
        flush_batch<BG>(s_acc, s_g, nb, n, grad2d, t, NT);
        __syncthreads();
    }
}

template <int TW, int TH>
__global__ __launch_bounds__(TW* TH) void k_render_bwd_recompute(
    int W, int H, int TX, int tile_offset, int n_tiles_total, const float* __restrict__ proj, int n,
    const uint32_t* __restrict__ values, const uint32_t* __restrict__ ranges, float bg0, float bg1,
    float bg2, const float* __restrict__ t_final, const uint32_t* __restrict__ n_contrib,
    const float* __restrict__ dl_dimage, float* __restrict__ grad2d, const uint32_t* __restrict__ order) {
    constexpr int NT = TW * TH;
    constexpr int NW = NT / 64;
    constexpr int BG = NT;
    __shared__ float4 s_a[BG];
    __shared__ float4 s_b[BG];
    __shared__ float s_c[BG];
    __shared__ uint32_t s_g[BG];
    __shared__ float s_acc[9][BG];
    __shared__ uint32_t s_last;
    const int tile = order ? (int)order[blockIdx.x] : (int)blockIdx.x;
    const int tx = tile % TX, ty = tile / TX;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int px = tx * TW + (t % TW), py = ty * TH + (t / TW);
    const bool inside = px < W && py < H;
    const int gt = tile_offset + tile;
    const uint32_t start = ranges[gt];
    const float fpx = (float)px + 0.5f, fpy = (float)py + 0.5f;
    const size_t pix = (size_t)py * W + px, plane = (size_t)W * H;

    uint32_t last = 0;
    float T = 1.f, G0 = 0.f, G1 = 0.f, G2 = 0.f;
    if (inside) {
        last = n_contrib[pix];
        T = t_final[pix];
        G0 = dl_dimage[pix];
        G1 = dl_dimage[plane + pix];
        G2 = dl_dimage[2 * plane + pix];
    }
    float a0 = bg0, a1 = bg1, a2 = bg2;  // colour behind the current splat
    if (t == 0) s_last = 0;
    __syncthreads();
    if (last) atomicMax(&s_last, last);
    __syncthreads();
    const uint32_t top = s_last;

    for (uint32_t hi = top; hi > 0;) {
        const uint32_t lo = hi > (uint32_t)BG ? hi - BG : 0u;
        const int nb = (int)(hi - lo);
        if (t < nb) {
            const uint32_t g = values[start + lo + t];
            s_g[t] = g;
            stage_splat(proj, n, g, s_a, s_b, s_c, t);
        }
        zero_acc<BG>(s_acc, t, NT);
        __syncthreads();
        for (int jj = nb - 1; jj >= 0; --jj) {
            const uint32_t jrel = lo + jj;
            bool ok = false;
            float alpha = 0.f, gauss = 0.f, dx = 0.f, dy = 0.f;
            Splat s{};
            if (jrel < last) {
                s = load_splat(s_a, s_b, s_c, jj);
                ok = splat_alpha(s, fpx, fpy, alpha, gauss, dx, dy);
            }
            const uint64_t m = __ballot(ok);
            if (m == 0) continue;
            float v[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
            if (ok) {
                const float Tk = T / (1.f - alpha);
                const float q0 = Tk * G0, q1 = Tk * G1, q2 = Tk * G2;
                const float dla = q0 * (s.r - a0) + q1 * (s.g - a1) + q2 * (s.b - a2);
                const bool clamped = s.o * gauss > kAlphaMax;
                chain_2d(s, dx, dy, alpha, gauss, clamped, dla, alpha * q0, alpha * q1,
                         alpha * q2, v);
                a0 = alpha * s.r + (1.f - alpha) * a0;
                a1 = alpha * s.g + (1.f - alpha) * a1;
                a2 = alpha * s.b + (1.f - alpha) * a2;
                T = Tk;
            }
            accumulate<BG>(v, s_acc, lane, jj, __popcll(m) == 1, ok);
        }
        __syncthreads();
        flush_batch<BG>(s_acc, s_g, nb, n, grad2d, t, NT);
        __syncthreads();
        hi = lo;
    }
}

bool tile_ok(int tw, int th) { return tw == 16 && th == 16; }

}  // namespace

extern "C" size_t pgs_trace_entries(uint32_t pair_capacity, int32_t tile_w, int32_t tile_h) {
    return (size_t)pair_capacity * (size_t)(tile_w > 0 ? tile_w : 0) * (size_t)(tile_h > 0 ? tile_h : 0);
}

static pgs_status make_trace(const pgs_replay* c, int tile_w, int tile_h, Trace& tr, const char* who) {
    PGS_REQUIRE(c->mask_dev && c->steps_dev && c->entry_dev && c->count_dev, "%s: null trace pointer", who);
    PGS_REQUIRE(((uintptr_t)c->entry_dev % 16) == 0, "%s: trace entries must be 16-byte aligned", who);
    PGS_REQUIRE(c->entry_capacity >= pgs_trace_entries(c->pair_capacity, tile_w, tile_h),
                "%s: trace entry capacity %llu below %u pairs x %d pixels", who,
                (unsigned long long)c->entry_capacity, c->pair_capacity, tile_w * tile_h);
    tr = Trace{c->mask_dev, c->steps_dev, reinterpret_cast<float4*>(c->entry_dev), c->count_dev,
               (size_t)c->entry_capacity, c->pair_capacity};
    return PGS_OK;
}

extern "C" pgs_status pgs_render_fwd(int32_t width, int32_t height, int32_t tile_w, int32_t tile_h,
                                     const float* proj_dev, int32_t n, const uint32_t* values_dev,
                                     const uint32_t* ranges_dev, int32_t view_tile_offset,
                                     const float* bg_host, float* image_dev, float* t_final_dev,
                                     uint32_t* n_contrib_dev, const pgs_replay* cache,
                                     uint32_t* flags_dev, const uint32_t* tile_order_dev, void* stream) {
    PGS_REQUIRE(width > 0 && height > 0 && n >= 0 && view_tile_offset >= 0, "pgs_render_fwd: bad sizes");
    PGS_REQUIRE(tile_ok(tile_w, tile_h), "pgs_render_fwd: unsupported tile %dx%d", tile_w, tile_h);
    PGS_REQUIRE(bg_host && ranges_dev && image_dev && t_final_dev && n_contrib_dev,
                "pgs_render_fwd: null pointer");
    PGS_REQUIRE(n == 0 || (proj_dev && values_dev), "pgs_render_fwd: null pointer");
    const int TX = (width + tile_w - 1) / tile_w, TY = (height + tile_h - 1) / tile_h;
    const int n_tiles_total = view_tile_offset + TX * TY;
    Trace tr{};
    if (cache) {
        PGS_REQUIRE(flags_dev != nullptr, "pgs_render_fwd: a trace needs the flags word");
        pgs_status st = make_trace(cache, tile_w, tile_h, tr, "pgs_render_fwd");
        if (st != PGS_OK) return st;
    }
    hipStream_t s = pgs::as_stream(stream);
    const dim3 grid(TX * TY), block(256);
    if (cache)
        k_render_fwd<16, 16, true><<<grid, block, 0, s>>>(width, height, TX, view_tile_offset, n_tiles_total,
                                                          proj_dev, n, values_dev, ranges_dev, bg_host[0],
                                                          bg_host[1], bg_host[2], image_dev, t_final_dev,
                                                          n_contrib_dev, tr, flags_dev, tile_order_dev);
    else
        k_render_fwd<16, 16, false><<<grid, block, 0, s>>>(width, height, TX, view_tile_offset, n_tiles_total,
                                                           proj_dev, n, values_dev, ranges_dev, bg_host[0],
                                                           bg_host[1], bg_host[2], image_dev, t_final_dev,
                                                           n_contrib_dev, tr, flags_dev, tile_order_dev);
    PGS_CHECK_LAUNCH("pgs_render_fwd");
    return PGS_OK;
}

extern "C" pgs_status pgs_render_bwd(int32_t width, int32_t height, int32_t tile_w, int32_t tile_h,
                                     const float* proj_dev, int32_t n, const uint32_t* values_dev,
                                     const uint32_t* ranges_dev, int32_t view_tile_offset,
                                     const float* bg_host, const float* t_final_dev,
                                     const uint32_t* n_contrib_dev, const pgs_replay* cache,
                                     const float* dl_dimage_dev, float* grad2d_dev,
                                     const uint32_t* tile_order_dev, void* stream) {
    PGS_REQUIRE(width > 0 && height > 0 && n >= 0 && view_tile_offset >= 0, "pgs_render_bwd: bad sizes");
    PGS_REQUIRE(tile_ok(tile_w, tile_h), "pgs_render_bwd: unsupported tile %dx%d", tile_w, tile_h);
    PGS_REQUIRE(bg_host && ranges_dev && dl_dimage_dev, "pgs_render_bwd: null pointer");
    if (n == 0) return PGS_OK;
    PGS_REQUIRE(proj_dev && values_dev && grad2d_dev, "pgs_render_bwd: null pointer");
    const int TX = (width + tile_w - 1) / tile_w, TY = (height + tile_h - 1) / tile_h;
    const int n_tiles_total = view_tile_offset + TX * TY;
    hipStream_t s = pgs::as_stream(stream);
    const dim3 grid(TX * TY), block(256);
    if (cache) {
        Trace tr{};
        pgs_status st = make_trace(cache, tile_w, tile_h, tr, "pgs_render_bwd");
        if (st != PGS_OK) return st;
        k_render_bwd_cached<16, 16><<<grid, block, 0, s>>>(width, height, TX, view_tile_offset, n_tiles_total,
                                                           proj_dev, n, values_dev, ranges_dev, tr,
                                                           dl_dimage_dev, grad2d_dev, tile_order_dev);
    } else {
        PGS_REQUIRE(t_final_dev && n_contrib_dev, "pgs_render_bwd: null pointer");
        k_render_bwd_recompute<16, 16><<<grid, block, 0, s>>>(width, height, TX, view_tile_offset,
                                                              n_tiles_total, proj_dev, n, values_dev,
                                                              ranges_dev, bg_host[0], bg_host[1], bg_host[2],
                                                              t_final_dev, n_contrib_dev, dl_dimage_dev,
                                                              grad2d_dev, tile_order_dev);
    }
    PGS_CHECK_LAUNCH("pgs_render_bwd");
    return PGS_OK;
}
