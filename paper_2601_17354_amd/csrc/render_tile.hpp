// Per-tile compositing forward and backward, shared by the single-view
// kernels (one workgroup per tile) and the multi-view persistent kernels
// (workgroups pull (view, tile) items from a queue).
//
// Forward (PocketGS Sec. "Explicit Computation Graph", "Bandwidth-Efficient
// Forward Replay Cache"): one lane per pixel of a TW x TH tile.  The tile's
// sorted splat list is staged through LDS in batches of BG splats (36 B of
// 2D attributes each) and every wave steps through the batch in lockstep,
// each lane compositing its pixel front to back.  A barrier with a live-lane
// count ends the tile once every pixel terminated.
//
// Replay trace.  S = {id, C_in, alpha} is recorded per wave of 64 pixels as
// groups, one per sorted splat id that at least one of the wave's pixels
// composited: a 64-bit ballot mask of those pixels (stored at the id's slot)
// followed by their entries in lane order.  The id of an entry is thus the
// slot of its group, its pixel the lane of its mask bit, and a pixel's
// entries in group order are its contributors front to back.  After the
// front to back pass each wave knows how many entries it recorded and takes
// a region of exactly that size from a device-wide bump counter (one 64-bit
// atomic per tile, split among its waves in order); a wave whose region does
// not fit the entry capacity is left unrecorded and the overflow flag is
// raised, the counter then holding the demand the caller needs.  A per-wave
// step counter bounds the valid groups, so masks of earlier iterations are
// never read and nothing is cleared between iterations.  The tile's groups
// are then walked back to front with the splats re-staged in LDS, and each
// entry is written once, one coalesced run per group: C_in (12 bytes; the
// backward recomputes alpha) or (C_in, alpha) (16 bytes), C_in being the
// colour of everything behind the splat, the over-recursion
// C_out = C_in (1 - alpha) + alpha c run from the background.
//
// Backward (equation "backward_chain"), two variants:
//   cached     steps through each wave's groups front to back, visiting only
//              non-empty masks, four groups at a time with the next four's
//              entries in flight; a lane with a bit set reads its entry, takes
//              dL/dC_out (starts at dL/dC, times (1 - alpha) after each own
//              entry), dL/dalpha = <dL/dC_out, c - C_in> and dL/dc =
//              alpha dL/dC_out, forms the nine per-pixel terms that the
//              splat's 2D gradients are linear in, and the wave reduces the
//              four groups' terms together (lane swaps and DPP).
//   recompute  walks the list back to front from n_contrib, re-evaluates
//              alpha with the forward's exact arithmetic, recovers
//              T_k = T_{k+1} / (1 - alpha_k) from T_final and accumulates the
//              colour behind as it goes (the 3D Gaussian Splatting backward).
// Per-wave partial sums meet in LDS; once per batch the splat's conic and
// opacity turn them into its nine 2D gradients, which leave with one float
// atomic per field and (tile, splat), scattered to the canonical index
// values[id] (index-mapping equation).
#pragma once

#include "common.hpp"

// Splats a wave composites between two termination checks.
#ifndef FWD_UNROLL
#define FWD_UNROLL 8
#endif

namespace pgs {

// A splat as staged in LDS: mean (u, v), the conic (A, B, C) held as
// hA = -A/2, nB = -B, hC = -C/2 (scalings by powers of two and a sign, so
// exact), opacity and colour.
struct Splat {
    float u, v, hA, nB, hC, o, r, g, b;
};

// Alpha of a splat at pixel centre (px, py).  Evaluated with contraction off
// so that the forward and the recompute backward produce identical bits.
__device__ __forceinline__ bool splat_alpha(const Splat& s, float px, float py, float& alpha,
                                            float& gauss, float& dx, float& dy) {
#pragma clang fp contract(off)
    dx = s.u - px;
    dy = s.v - py;
    // power = -(A dx^2 + 2 B dx dy + C dy^2) / 2 = (hA dx + nB dy) dx + hC dy^2
    const float power = __builtin_fmaf(__builtin_fmaf(s.hA, dx, s.nB * dy), dx, s.hC * dy * dy);
    gauss = __expf(power);
    alpha = fminf(kAlphaMax, s.o * gauss);
    return !(power > 0.f) && alpha >= kAlphaMin;
}

// One splat's record (u, v, depth, A | B, C, o, r | g, b, ex, ey) is one
// 64-byte line: three 16-byte loads.  (The compositing kernels decide which
// waves a splat can reach from its conic instead of the half-extents
// (ex, ey).)
__device__ __forceinline__ void stage_splat(const float* __restrict__ proj, int n, uint32_t g,
                                            float4* sa, float4* sb, float* sc, int slot) {
    (void)n;
    const float4* rec = reinterpret_cast<const float4*>(proj + (size_t)g * PGS_PROJ_STRIDE);
    const float4 r0 = rec[0], r1 = rec[1], r2 = rec[2];
    sa[slot] = make_float4(r0.x, r0.y, -0.5f * r0.w, -r1.x);   // u, v, hA, nB
    sb[slot] = make_float4(-0.5f * r1.y, r1.z, r1.w, r2.x);    // hC, o, r, g
    sc[slot] = r2.y;                                  // b
}

__device__ __forceinline__ Splat load_splat(const float4* sa, const float4* sb, const float* sc, int k) {
    const float4 a = sa[k], b = sb[k];
    return Splat{a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w, sc[k]};
}

// Mean, conic and opacity of a staged splat (colour left zero).
__device__ __forceinline__ Splat load_shape(const float4* sa, const float4* sb, int k) {
    const float4 a = sa[k];
    const float2 b = *reinterpret_cast<const float2*>(&sb[k]);
    return Splat{a.x, a.y, a.z, a.w, b.x, b.y, 0.f, 0.f, 0.f};
}

// Set bits of m below this lane: its rank among the lanes of m.
__device__ __forceinline__ uint32_t lane_rank(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Whether this lane's bit is set in the wave-uniform mask m (the mask
// becomes the execution mask directly).
__device__ __forceinline__ bool lane_in(uint64_t m) { return __builtin_amdgcn_inverse_ballot_w64(m); }

// A wave's trace entries are addressed through a buffer resource on the
// start of its region (kept in scalar registers) with 32-bit byte offsets:
// a run's start as the scalar offset and the lane's rank in it as the vector
// one, so an access takes no 64-bit per-lane address arithmetic.  A region
// stays far below 4 GiB: a pixel composites at most ln(1e-4) / ln(1 - 1/255)
// < 2400 splats before its transmittance ends it, so a wave's region holds
// fewer than 64 * 2400 entries.  Word 3 of the resource selects the 32-bit
// data format (value 4 in bits 15-18), which untyped buffer access on this
// GPU family expects; the record count is left at its maximum.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t region_rsrc(const void* region) {
    const uint64_t a = reinterpret_cast<uint64_t>(region);
    const uint64_t u = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(a >> 32)) << 32) |
                       (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)a);
    return __builtin_amdgcn_make_buffer_rsrc(reinterpret_cast<void*>(u), (short)0, -1, 0x00020000);
}

typedef uint32_t u32x3 __attribute__((ext_vector_type(3)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Entry `rank` (< 64) of the run of EW-word entries that starts `first`
// entries into the region.
template <int EW>
__device__ __forceinline__ float4 load_entry(__amdgpu_buffer_rsrc_t rs, uint32_t first, uint32_t rank) {
    // first is the same in every lane; saying so keeps the offset scalar
    const uint32_t voff = rank * (4u * EW),
                   soff = (uint32_t)__builtin_amdgcn_readfirstlane((int)(first * (4u * EW)));
    if constexpr (EW == 4) {
        const u32x4 r = __builtin_amdgcn_raw_buffer_load_b128(rs, voff, soff, 0);
        return make_float4(__uint_as_float(r.x), __uint_as_float(r.y), __uint_as_float(r.z), __uint_as_float(r.w));
    } else {
        const u32x3 r = __builtin_amdgcn_raw_buffer_load_b96(rs, voff, soff, 0);
        return make_float4(__uint_as_float(r.x), __uint_as_float(r.y), __uint_as_float(r.z), 0.f);
    }
}

// Stores take the whole offset in the vector operand and a zero scalar
// offset: the compiler inserts the wait that a store of more than 8 bytes
// needs before its data registers are overwritten only for that form, and
// with a register scalar offset the store was measured to pick up the next
// value of its data registers.
template <int EW>
__device__ __forceinline__ void store_entry(__amdgpu_buffer_rsrc_t rs, uint32_t first, uint32_t rank, float c0,
                                            float c1, float c2, float alpha) {
    const uint32_t voff = (first + rank) * (4u * EW);
    if constexpr (EW == 4) {
        u32x4 d = {__float_as_uint(c0), __float_as_uint(c1), __float_as_uint(c2), __float_as_uint(alpha)};
        __builtin_amdgcn_raw_buffer_store_b128(d, rs, voff, 0, 0);
    } else {
        u32x3 d = {__float_as_uint(c0), __float_as_uint(c1), __float_as_uint(c2)};
        __builtin_amdgcn_raw_buffer_store_b96(d, rs, voff, 0, 0);
        (void)alpha;
    }
}

__device__ __forceinline__ uint64_t read_lane64(uint64_t v, int lane) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
    return ((uint64_t)hi << 32) | lo;
}

// Transposes the 64 x 64 bit matrix whose row r is lane r's h: afterwards
// lane s holds bit s of every lane's h, bit r from lane r.  Six block-swap
// stages; stage j exchanges the j x j blocks between lanes r and r ^ j.
__device__ __forceinline__ uint64_t transpose64(uint64_t h, int lane) {
    constexpr uint64_t kMask[6] = {0x00000000FFFFFFFFull, 0x0000FFFF0000FFFFull, 0x00FF00FF00FF00FFull,
                                   0x0F0F0F0F0F0F0F0Full, 0x3333333333333333ull, 0x5555555555555555ull};
#pragma unroll
    for (int l = 0; l < 6; ++l) {
        const int j = 32 >> l;
        const uint32_t plo = (uint32_t)__shfl_xor((int)(uint32_t)h, j);
        const uint32_t phi = (uint32_t)__shfl_xor((int)(uint32_t)(h >> 32), j);
        const uint64_t p = ((uint64_t)phi << 32) | plo;
        const bool low = (lane & j) == 0;
        const uint64_t d = low ? (((h >> j) ^ p) & kMask[l]) : (((p >> j) ^ h) & kMask[l]);
        h ^= low ? (d << j) : d;
    }
    return h;
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
    for (int j = 32; j > 0; j >>= 1) v += (uint32_t)__shfl_xor((int)v, j);
    return v;
}

struct Trace {
    uint64_t* mask;             // [NW][pair_cap]
    uint32_t* steps;            // [n_tiles][NW]
    uint32_t* base;             // [n_tiles][NW] first entry of the wave's region
    unsigned long long* used;   // entries handed out in this forward
    float* entry;               // [entry_cap][EW]: (C_in r, g, b[, alpha])
    uint32_t* count;            // [pixels]
    size_t entry_cap;
    uint32_t pair_cap;
    int words;                  // EW of the launch: 4 with alpha, 3 without
};

// A trace entry holds EW words: (C_in r, g, b, alpha) as one 16-byte record,
// or (C_in r, g, b) as one 12-byte record when the backward recomputes alpha
// from the staged splat with the forward's arithmetic (same bits).

// One tile of one view.  Pixel arrays (image planes, t_final, n_contrib,
// count) are the view's own; gt is the tile's global index in the ranges.
struct TileJob {
    int W, H, tx, ty, gt;
    const float* proj;
    float* image;
    float* t_final;
    uint32_t* n_contrib;
    uint32_t* count;
};

// LDS of a tile pass: one batch of BG staged splats (forward), plus their
// canonical ids and the gradient accumulator (backward); declared by each
// kernel and handed to the tile functions.
template <int BG>
struct FwdLds {
    float4 a[BG];
    float4 b[BG];
    float c[BG];
    uint8_t reach[BG];  // bit w: the splat can reach a pixel of wave w
    uint32_t steps;
    // per wave of the tile: entries, steps, fit flag and region start
    uint32_t wcur[4], wsteps[4], wfit[4];
    unsigned long long wbase[4];
};

template <int BG>
struct TileLds {
    float4 a[BG];
    float4 b[BG];
    float c[BG];
    uint32_t g[BG];
    float io[BG];  // 1 / opacity
    uint8_t reach[BG];  // bit w: the splat can reach a pixel of wave w (recompute backward)
    float acc[9][BG + 1];  // one word of padding per row: a splat's nine terms fall in nine banks
    uint32_t steps;
};

// Stages splats base .. base+nb-1 of the sorted list into LDS slots 0..nb-1.
template <int NT, bool KEEP_IDS, class Lds>
__device__ __forceinline__ void stage_batch(Lds& L, const float* __restrict__ proj, int n,
                                            const uint32_t* __restrict__ values, uint32_t base, int nb,
                                            int t) {
    for (int q = t; q < nb; q += NT) {
        const uint32_t g = values[base + q];
        stage_splat(proj, n, g, L.a, L.b, L.c, q);
        if constexpr (KEEP_IDS) {
            L.g[q] = g;
            L.io[q] = 1.f / L.b[q].y;
        }
    }
}

// Which waves of a TW x TH tile a splat can reach: bit w is cleared only if
// splat_alpha gives alpha < 1/255 at every pixel centre of wave w's rows
// (the wave's pixel-centre rectangle R_w).  Alpha reaches 1/255 only where
// q = A dx^2 + 2 B dx dy + C dy^2 <= 2 ln(255 o).  The minimum of q over R_w
// is zero if the centre lies inside R_w, else the least of the four edge
// minima, each the minimum of a convex quadratic in one variable, clamped to
// the edge.  Rounding: with rho = |B| / sqrt(A C), the magnitudes of q's
// three terms sum to at most q (1 + rho) / (1 - rho), and each term carries
// a relative error of a few units of roundoff u in float32, both in
// splat_alpha and here (an error in the position of an edge minimum changes q
// only to second order), so both evaluations are within
// kappa = 64 u (1 + rho) / (1 - rho) of q relative to it.  A wave is dropped
// when the computed minimum, shrunk by 2 kappa, still exceeds 2 ln(255 o) by
// 1e-4, which also covers the rounding of the exponential, the opacity
// product and the threshold; and never when kappa >= 1/8.
template <int TW, int TH>
__device__ __forceinline__ uint32_t reach_waves(float u, float v, float A, float B, float C, float o, int tx,
                                                int ty) {
    constexpr int NW = TW * TH / 64;
    constexpr int R = 64 / TW;  // pixel rows per wave
    constexpr uint32_t kAll = (1u << NW) - 1u;
    if (!(o > kAlphaMin * 0.5f)) return 0u;  // alpha = o e^power <= o < 1/255 everywhere
    if (!(A > 0.f && C > 0.f)) return kAll;
    const float ac = A * C;
    const float rho = fabsf(B) * __frsqrt_rn(ac);
    // 1 - rho = (A C - B^2) / (A C (1 + rho)), the determinant taken with one rounding
    const float det = __builtin_fmaf(A, C, -B * B);
    const float omr = det / (ac * (1.f + rho));
    const float kappa = 64.f * 0x1p-24f * (1.f + rho) / omr;
    if (!(omr > 0.f && kappa < 0.125f)) return kAll;
    const float thr = 2.f * __logf(255.f * o) + 1e-4f;
    const float shrink = 1.f - 2.f * kappa;
    const float ra = 1.f / A, rc = 1.f / C;
    const float xlo = (float)(tx * TW) + 0.5f, xhi = xlo + (float)(TW - 1);
    // dx over the rectangle's columns, dy over its rows (d = centre - pixel)
    const float dxa = u - xhi, dxb = u - xlo;
    const float ma = -B * dxa * rc, mb = -B * dxb * rc;  // best dy on the columns x = xhi, xlo
    auto q = [&](float dx, float dy) { return A * dx * dx + 2.f * B * dx * dy + C * dy * dy; };
    uint32_t bits = 0u;
#pragma unroll 1
    for (int w = 0; w < NW; ++w) {
        const float ylo = (float)(ty * TH + w * R) + 0.5f, yhi = ylo + (float)(R - 1);
        const float dya = v - yhi, dyb = v - ylo;
        float m = 0.f;
        if (!(dxa <= 0.f && dxb >= 0.f && dya <= 0.f && dyb >= 0.f)) {
            m = fminf(q(dxa, fminf(fmaxf(ma, dya), dyb)), q(dxb, fminf(fmaxf(mb, dya), dyb)));
            // rows y = yhi, ylo: dx minimising q at fixed dy is -B dy / A
            m = fminf(m, q(fminf(fmaxf(-B * dya * ra, dxa), dxb), dya));
            m = fminf(m, q(fminf(fmaxf(-B * dyb * ra, dxa), dxb), dyb));
        }
        if (!(m * shrink > thr)) bits |= 1u << w;
    }
    return bits;
}

// Stages splats base .. base+nb-1 of the sorted list into LDS slots 0..nb-1
// with the waves each can reach (and, for the backward, their canonical ids
// and 1 / opacity).
template <int TW, int TH, int NT, bool KEEP_IDS, class Lds>
__device__ __forceinline__ void stage_batch_reach(Lds& L, const float* __restrict__ proj,
                                                  const uint32_t* __restrict__ values, uint32_t base, int nb,
                                                  int t, int tx, int ty) {
    for (int q = t; q < nb; q += NT) {
        const uint32_t g = values[base + q];
        const float4* rec = reinterpret_cast<const float4*>(proj + (size_t)g * PGS_PROJ_STRIDE);
        const float4 r0 = rec[0], r1 = rec[1], r2 = rec[2];
        L.a[q] = make_float4(r0.x, r0.y, -0.5f * r0.w, -r1.x);   // u, v, hA, nB
        L.b[q] = make_float4(-0.5f * r1.y, r1.z, r1.w, r2.x);    // hC, o, r, g
        L.c[q] = r2.y;                                           // b
        L.reach[q] = (uint8_t)reach_waves<TW, TH>(r0.x, r0.y, r0.w, r1.x, r1.y, r1.z, tx, ty);
        if constexpr (KEEP_IDS) {
            L.g[q] = g;
            L.io[q] = 1.f / r1.z;
        }
    }
}

template <int TW, int TH, int BG, bool CACHED, int EW = 4>
__device__ __forceinline__ void fwd_tile(const TileJob& j, int n_tiles_total, int n,
                                         const uint32_t* __restrict__ values,
                                         const uint32_t* __restrict__ ranges, float bg0, float bg1,
                                         float bg2, const Trace& tr, uint32_t* __restrict__ flags,
                                         FwdLds<BG>& L) {
    constexpr int NT = TW * TH;
    constexpr int NW = NT / 64;
    static_assert((BG & (BG - 1)) == 0 && BG % FWD_UNROLL == 0, "batch: a power of two, whole groups");
    static_assert(NW <= 4, "at most four waves per tile");
    const int t = threadIdx.x, lane = t & 63, wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const int px = j.tx * TW + (t % TW), py = j.ty * TH + (t / TW);
    const bool inside = px < j.W && py < j.H;
    const uint32_t start = ranges[j.gt], end = ranges[n_tiles_total + j.gt];
    const float fpx = (float)px + 0.5f, fpy = (float)py + 0.5f;

    // the trace is recorded only if this tile's pairs fit the trace buffers
    const bool rec = CACHED && end <= tr.pair_cap;
    if (CACHED && !rec && t == 0) atomicOr(flags, PGS_FLAG_CACHE_OVERFLOW);
    // Each lane keeps the composited bits of the current window of 64
    // steps (bit s: this pixel took step s); a window is transposed over the
    // wave into its 64 step masks and written as one coalesced 512-byte run
    // (wave-major mask layout).  The lane's entry count and last
    // contributing step come from the same bits.
    uint64_t* wmask = tr.mask + (size_t)wv * tr.pair_cap + start;
    uint64_t hist = 0ull;
    uint32_t steps = 0, cnt = 0, last = 0;
    auto flush_chunk = [&](uint32_t c0, uint32_t cn) {
        cnt += (uint32_t)__popcll(hist);
        if (hist) last = c0 + 64u - (uint32_t)__clzll(hist);
        if (rec) {
            const uint64_t m = transpose64(hist, lane);
            if ((uint32_t)lane < cn) wmask[c0 + lane] = m;
        }
        hist = 0ull;
    };

    float T = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f;
    bool done = !inside;

    for (uint32_t base = start; base < end; base += BG) {
        if (__syncthreads_count(!done) == 0) break;
        const int nb = (int)min((uint32_t)BG, end - base);
        stage_batch_reach<TW, TH, NT, false>(L, j.proj, values, base, nb, t, j.tx, j.ty);
        __syncthreads();
        // Windows of 64 steps.  Of a window the wave visits only the steps
        // whose splat can reach one of its pixels (a wave-uniform bit set,
        // walked with scalar bit scans), FWD_UNROLL at a time: their LDS
        // loads and alphas first, straight-line, then the steps in order,
        // with a termination check per group.  Every step it skips has alpha
        // < 1/255 at all of its pixels, so its mask bits are zero as if it
        // had been visited.
        for (int c0 = 0; c0 < nb; c0 += 64) {
            if (__ballot(!done) == 0) break;  // the whole wave has terminated
            const int cn = min(64, nb - c0);
            uint64_t todo = __ballot(lane < cn && ((L.reach[c0 + lane] >> wv) & 1u) != 0u);
            while (todo) {
                if (__ballot(!done) == 0) break;
                int kq[FWD_UNROLL];
                bool val[FWD_UNROLL];
#pragma unroll
                for (int u = 0; u < FWD_UNROLL; ++u) {
                    val[u] = todo != 0ull;
                    kq[u] = val[u] ? (int)__builtin_ctzll(todo) : 0;
                    todo &= todo - 1ull;
                }
                // geometry and opacity only; the colours are read by the
                // steps that composite
                Splat sp[FWD_UNROLL];
#pragma unroll
                for (int u = 0; u < FWD_UNROLL; ++u) sp[u] = load_shape(L.a, L.b, c0 + kq[u]);
                float al[FWD_UNROLL];
                bool hit[FWD_UNROLL];
#pragma unroll
                for (int u = 0; u < FWD_UNROLL; ++u) {
                    float gauss, dx, dy;
                    hit[u] = splat_alpha(sp[u], fpx, fpy, al[u], gauss, dx, dy) && val[u];
                }
#pragma unroll
                for (int u = 0; u < FWD_UNROLL; ++u) {
                    // exec-masked: a step none of the wave's pixels takes is
                    // skipped by the whole wave
                    if (hit[u] && !done) {
                        const float alpha = al[u];
                        const float test_T = T * (1.f - alpha);
                        if (test_T < kTMin) {
                            done = true;
                        } else {
                            const int k = c0 + kq[u];
                            const float2 rg = *reinterpret_cast<const float2*>(&L.b[k].z);
                            const float w = alpha * T;
                            C0 += w * rg.x;
                            C1 += w * rg.y;
                            C2 += w * L.c[k];
                            T = test_T;
                            hist |= 1ull << kq[u];
                        }
                    }
                }
            }
            const uint32_t rel0 = base + (uint32_t)c0 - start;
            flush_chunk(rel0, (uint32_t)cn);
            steps = rel0 + (uint32_t)cn;
        }
    }
    uint32_t cursor = 0;
    if (rec) cursor = (uint32_t)__builtin_amdgcn_readfirstlane((int)wave_sum_u32(cnt));  // the same in every lane
    // Entry regions: one bump-counter atomic per tile (a single device-wide
    // address, so per-wave atomics would queue there), split among the
    // waves in order.  A wave whose region does not fit the entry capacity
    // is left unrecorded (its step count becomes 0, so the backward reads
    // nothing of it) and the overflow flag is raised; the counter keeps the
    // demand either way.
    size_t ebase = 0;
    bool wrec = rec;
    uint32_t smax = 0;
    if (rec) {  // uniform for the block
        if (lane == 0) {
            L.wcur[wv] = cursor;
            L.wsteps[wv] = steps;
        }
        __syncthreads();
        if (t == 0) {
            unsigned long long total = 0;
            for (int w = 0; w < NW; ++w) total += L.wcur[w];
            unsigned long long b = total ? atomicAdd(tr.used, total) : 0ull;
            uint32_t sm = 0;
            bool lost = false;
            for (int w = 0; w < NW; ++w) {
                const bool fit = L.wcur[w] == 0 || b + L.wcur[w] <= tr.entry_cap;
                L.wfit[w] = fit;
                L.wbase[w] = fit ? b : 0ull;
                if (fit) sm = max(sm, L.wsteps[w]);
                lost |= !fit;
                b += L.wcur[w];
            }
            if (lost) atomicOr(flags, PGS_FLAG_CACHE_OVERFLOW);
            L.steps = sm;
        }
        __syncthreads();
        wrec = L.wfit[wv] != 0;
        ebase = (size_t)L.wbase[wv];
        smax = L.steps;
        if (!wrec) steps = 0;
    }
    if (inside) {
        const size_t pix = (size_t)py * j.W + px, plane = (size_t)j.W * j.H;
        j.image[pix] = C0 + T * bg0;
        j.image[plane + pix] = C1 + T * bg1;
        j.image[2 * plane + pix] = C2 + T * bg2;
        j.t_final[pix] = T;
        j.n_contrib[pix] = last;
        if (CACHED) j.count[pix] = wrec ? cnt : 0u;
    }
    if (!rec) return;  // uniform for the block
    if (lane == 0) {
        tr.steps[(size_t)j.gt * NW + wv] = steps;
        tr.base[(size_t)j.gt * NW + wv] = (uint32_t)ebase;
    }

    // Entry pass: back to front over each wave's groups with the splats
    // re-staged in LDS batch by batch (the forward batches in reverse).  Each
    // set lane re-evaluates alpha with the same arithmetic as above (same
    // bits) and writes its entry (C_in, alpha) once, C_in being the colour
    // accumulated behind the splat so far.
    float a0 = bg0, a1 = bg1, a2 = bg2;
    uint32_t cur = cursor;
    if (smax == 0) return;
    const int64_t top = (int64_t)((smax - 1) / BG) * BG;  // first position of the last batch
    // Windows of 64 steps per batch.  A batch's masks are loaded together
    // with its splats: a wait on a vector load also waits for the entry
    // stores issued before it, so this costs one such wait per batch rather
    // than one per window.
    constexpr int kWin = BG >= 64 ? BG / 64 : 1;
    const uint64_t* wm = tr.mask + (size_t)wv * tr.pair_cap + start;
    const __amdgpu_buffer_rsrc_t went = region_rsrc(tr.entry + ebase * EW);
    for (int64_t lo = top; lo >= 0; lo -= BG) {
        const uint32_t hi = min((uint32_t)lo + BG, smax);
        __syncthreads();
        stage_batch<NT, false>(L, j.proj, n, values, start + (uint32_t)lo, (int)(hi - (uint32_t)lo), t);
        const uint32_t whi = min(hi, steps);
        uint64_t mw[kWin];
#pragma unroll
        for (int w = 0; w < kWin; ++w) {
            const uint32_t c0 = (uint32_t)lo + 64u * w;
            mw[w] = c0 + (uint32_t)lane < whi ? wm[c0 + lane] : 0ull;
        }
        __syncthreads();
        // windows last to first; the non-empty groups of a window are taken
        // last to first, four at a time: their splats' loads and alphas
        // first, then each set lane writes its entries in order
#pragma unroll
        for (int w = kWin - 1; w >= 0; --w) {
            const uint32_t c0 = (uint32_t)lo + 64u * w;
            if (c0 >= whi) continue;  // uniform
            const uint64_t mv = mw[w];
            uint64_t any = __ballot(mv != 0ull);
            while (any) {
                int gi[4];
                uint64_t gm[4];
                uint32_t gc[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    gi[q] = 0;
                    gm[q] = 0ull;
                    if (any) {
                        const int i = 63 - __clzll(any);
                        any &= ~(1ull << i);
                        gi[q] = i;
                        gm[q] = read_lane64(mv, i);
                        cur -= __popcll(gm[q]);
                    }
                    gc[q] = cur;
                }
                Splat sq[4];
                float al[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    sq[q] = load_splat(L.a, L.b, L.c, 64 * w + gi[q]);
                    float gauss, dx, dy;
                    splat_alpha(sq[q], fpx, fpy, al[q], gauss, dx, dy);
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (lane_in(gm[q])) {
                        const float a = al[q];
                        store_entry<EW>(went, gc[q], lane_rank(gm[q]), a0, a1, a2, a);
                        a0 = a * sq[q].r + (1.f - a) * a0;
                        a1 = a * sq[q].g + (1.f - a) * a1;
                        a2 = a * sq[q].b + (1.f - a) * a2;
                    }
                }
            }
        }
    }
}

// Per-pixel terms of one splat's nine 2D gradients, all linear in what the
// wave and the tile sum: with p = dL/dpower = alpha dL/dalpha (0 where alpha
// is clamped) and d = (dx, dy) the offset from the pixel to the mean, the
// terms are p dx, p dy, p dx^2, p dx dy, p dy^2, p and dL/dc = alpha dL/dC_out.
// The splat's conic and opacity, the same for every pixel, are applied once
// per splat and tile to the sums (grad2d_from_sums).
__device__ __forceinline__ void raw_terms(float dx, float dy, float alpha, bool clamped, float dl_dalpha,
                                          float dc0, float dc1, float dc2, float* v) {
    const float p = clamped ? 0.f : alpha * dl_dalpha;
    const float px = p * dx, py = p * dy;
    v[0] = px;
    v[1] = py;
    v[2] = px * dx;
    v[3] = px * dy;
    v[4] = py * dy;
    v[5] = p;
    v[6] = dc0;
    v[7] = dc1;
    v[8] = dc2;
}

// The nine 2D gradients from the summed terms of raw_terms.  With
// power = hA dx^2 + nB dx dy + hC dy^2 (hA = -A/2, nB = -B, hC = -C/2) and
// alpha = o e^power: dL/du = 2 hA S(p dx) + nB S(p dy),
// dL/dv = nB S(p dx) + 2 hC S(p dy), dL/dA = -S(p dx^2) / 2,
// dL/dB = -S(p dx dy), dL/dC = -S(p dy^2) / 2, dL/do = S(p) / o (the
// derivative of o e^power by o is alpha / o), dL/dc unchanged.
__device__ __forceinline__ void grad2d_from_sums(float hA, float nB, float hC, float inv_o, float* f) {
    const float spx = f[0], spy = f[1];
    f[0] = __builtin_fmaf(2.f * hA, spx, nB * spy);
    f[1] = __builtin_fmaf(2.f * hC, spy, nB * spx);
    f[2] = -0.5f * f[2];
    f[3] = -f[3];
    f[4] = -0.5f * f[4];
    f[5] = f[5] * inv_o;
}

// x + y taken from the lane that the DPP control CTRL names inside a 16-lane
// row (every control used here names a lane of the same row).
template <int CTRL>
__device__ __forceinline__ float dpp_add(float x, float y) {
    return x + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(y), CTRL, 0xf, 0xf, false));
}

// One transposing step for two values a and b with the partner lane that CTRL
// names: lanes with lo set keep the sum of a over the pair of lanes, the
// others the sum of b.
template <int CTRL>
__device__ __forceinline__ float fold_pair(float a, float b, bool lo) {
    return dpp_add<CTRL>(lo ? a : b, lo ? b : a);
}

// The term that lane i of a 16-lane row holds after wave_reduce36: 8 in odd
// lanes; in even lanes of quad k (k = i / 4) term (0, 2, 1, 3)[k] where bit 1
// of i is clear, else term (4, 6, 5, 7)[k] (the first step leaves the even
// terms of each pair in lanes 0-7, the second the first pair of each pair of
// pairs in quads 0 and 2).
__device__ __forceinline__ int term_of_lane(int i) {
    if (i & 1) return 8;
    const int k = i >> 2;
    const int base = (i & 2) ? 4 : 0;
    return base + (k == 0 ? 0 : k == 1 ? 2 : k == 2 ? 1 : 3);
}

// Sums the nine terms of each of four groups over the wave (v[9q + f] is term
// f of group q at this lane).  v_permlane32_swap meets lanes 0-31 of one
// register with lanes 32-63 of another: pairing group q with group q + 2
// leaves groups 0 and 1 in the lower half and groups 2 and 3 in the upper
// one.  v_permlane16_swap does the same between neighbouring 16-lane rows:
// pairing group q with q + 1 leaves row r holding group r, each lane a sum
// over four lanes.  Inside the row four transposing steps follow (partner
// lane i ^ 8 by a rotation of 8, the mirror lane inside each half, then
// i ^ 2 and i ^ 1 inside each quad): each step halves the number of values
// a lane holds and doubles the lanes each value covers, so the row's nine
// values take 27 instructions instead of the 36 of a scan of each.
// Afterwards lane i of row r holds the row total of term term_of_lane(i) of
// group r.
__device__ __forceinline__ float wave_reduce36(const float* v, int lane) {
    float s[18];
#pragma unroll
    for (int f = 0; f < 9; ++f) {
        const auto r02 = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[f]), __float_as_uint(v[18 + f]),
                                                          false, false);
        const auto r13 = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[9 + f]), __float_as_uint(v[27 + f]),
                                                          false, false);
        s[2 * f] = __uint_as_float(r02[0]) + __uint_as_float(r02[1]);
        s[2 * f + 1] = __uint_as_float(r13[0]) + __uint_as_float(r13[1]);
    }
    float x[9];
#pragma unroll
    for (int f = 0; f < 9; ++f) {
        const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(s[2 * f]), __float_as_uint(s[2 * f + 1]),
                                                        false, false);
        x[f] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
    constexpr int kRor8 = 0x128, kHalfMirror = 0x141, kSwap2 = 0x4e, kSwap1 = 0xb1;
    const bool lo8 = (lane & 8) == 0, lo4 = (lane & 4) == 0, lo2 = (lane & 2) == 0, lo1 = (lane & 1) == 0;
    // each value covers lanes {i, i ^ 8}: pairs (0, 1), (2, 3), (4, 5), (6, 7)
    const float p0 = fold_pair<kRor8>(x[0], x[1], lo8), p1 = fold_pair<kRor8>(x[2], x[3], lo8);
    const float p2 = fold_pair<kRor8>(x[4], x[5], lo8), p3 = fold_pair<kRor8>(x[6], x[7], lo8);
    float t8 = dpp_add<kRor8>(x[8], x[8]);
    // four lanes each
    const float q0 = fold_pair<kHalfMirror>(p0, p1, lo4), q1 = fold_pair<kHalfMirror>(p2, p3, lo4);
    t8 = dpp_add<kHalfMirror>(t8, t8);
    // eight lanes each
    const float r0 = fold_pair<kSwap2>(q0, q1, lo2);
    t8 = dpp_add<kSwap2>(t8, t8);
    // the whole row; kept outside the adding lanes' branch, where the shifted
    // move folds into the add
    const float total = fold_pair<kSwap1>(r0, t8, lo1);
    asm volatile("" : : "v"(total));
    return total;
}

// Adds the wave's nine gradient terms of each of KG = 4 groups (splat slots
// slot0 + gi[q]; an empty group, whose mask is 0, adds nothing) into the LDS
// accumulator: one combined reduction, then one LDS add in which lane i of
// row r (i even, or i = 1) adds term term_of_lane(i) of group r.
template <int BG, int KG>
__device__ __forceinline__ void accumulate_groups(const float* v, float (*acc)[BG + 1], int lane, uint32_t slot0,
                                                  const int* gi, const uint64_t* gm) {
    static_assert(KG * 9 == 36, "the combined reduction takes four groups");
    const float x = wave_reduce36(v, lane);
    // row r takes group r's slot, or -1 for an empty group (lane selects
    // of the uniform values, no branch)
    int sq[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) sq[q] = gm[q] != 0ull ? (int)slot0 + gi[q] : -1;
    const int s01 = (lane & 16) ? sq[1] : sq[0];
    const int s23 = (lane & 16) ? sq[3] : sq[2];
    const int slot = (lane & 32) ? s23 : s01;
    const int i = lane & 15;
    if (((i & 1) == 0 || i == 1) && slot >= 0) atomicAdd(&acc[term_of_lane(i)][slot], x);
}

// The batch's summed terms become its splats' 2D gradients (one thread per
// splat), then one float atomic per field and splat goes into the canonical
// 2D-gradient records (index map values[id]); the nine fields of a splat
// share one 64-byte record, so consecutive lanes hit the same line.  Each
// accumulator word is cleared as it is read, so the next batch starts from
// zeros (slots past nb are never written).
template <int BG>
__device__ __forceinline__ void flush_batch(TileLds<BG>& L, int nb, int n, float* __restrict__ grad2d, int t,
                                            int NT) {
    (void)n;
    float (*acc)[BG + 1] = L.acc;
    const uint32_t* gid = L.g;
    for (int jj = t; jj < nb; jj += NT) {
        float f[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) f[k] = acc[k][jj];
        grad2d_from_sums(L.a[jj].z, L.a[jj].w, L.b[jj].x, L.io[jj], f);
#pragma unroll
        for (int k = 0; k < 6; ++k) acc[k][jj] = f[k];
    }
    __syncthreads();
    for (int idx = t; idx < nb * 9; idx += NT) {
        const int jj = idx / 9, f = idx - jj * 9;
        const float s = acc[f][jj];
        acc[f][jj] = 0.f;
        if (s != 0.f) unsafeAtomicAdd(&grad2d[(size_t)gid[jj] * PGS_GRAD2D_STRIDE + f], s);
    }
}

template <int BG>
__device__ __forceinline__ void zero_acc(float (*acc)[BG + 1], int t, int NT) {
    for (int idx = t; idx < 9 * (BG + 1); idx += NT) (&acc[0][0])[idx] = 0.f;
}

// Up to four non-empty groups of a 64-step window, front to back: the
// step within the window, the lane mask and the first entry (relative to the
// wave's region) of each; an unused slot has an empty mask.
struct TraceGroups {
    int gi[4];
    uint64_t gm[4];
    uint32_t gc[4];
};

__device__ __forceinline__ void take_groups(uint64_t& any, uint64_t mv, uint32_t& cursor, TraceGroups& g) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        g.gi[q] = 0;
        g.gm[q] = 0ull;
        g.gc[q] = cursor;
        if (any) {
            const int i = __ffsll((unsigned long long)any) - 1;
            any &= any - 1;
            g.gi[q] = i;
            g.gm[q] = read_lane64(mv, i);
            cursor = (uint32_t)__builtin_amdgcn_readfirstlane((int)(cursor + __popcll(g.gm[q])));  // uniform
        }
    }
}

// Every lane loads: its own entry where it has one, else the wave's first
// entry (the region is not empty when a group exists); alpha is taken as 0
// for the latter in bwd_groups.
template <int EW>
__device__ __forceinline__ void load_groups(__amdgpu_buffer_rsrc_t went, const TraceGroups& g, float4* e) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        // an empty group (unused slot) reads the region's first entry
        e[q] = load_entry<EW>(went, g.gm[q] != 0ull ? g.gc[q] : 0u, lane_in(g.gm[q]) ? lane_rank(g.gm[q]) : 0u);
    }
}

// Gradients of four groups at this lane's pixel, reduced over the wave into
// the batch accumulator; a lane without an entry in a group contributes
// exact zeros there and keeps its dL/dC_out.
template <int BG, int EW, class Lds>
__device__ __forceinline__ void bwd_groups(const TraceGroups& g, const float4* e, Lds& L, uint32_t slot0, float fpx,
                                           float fpy, int lane, float& g0, float& g1, float& g2) {
    float v[36];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int jj = (int)slot0 + g.gi[q];
        const Splat s = load_splat(L.a, L.b, L.c, jj);
        float dx = s.u - fpx, dy = s.v - fpy;
        float a;
        if constexpr (EW == 4) {
            a = lane_in(g.gm[q]) ? e[q].w : 0.f;
        } else {
            // the entry's alpha, recomputed with the forward's arithmetic
            float ar, gauss;
            splat_alpha(s, fpx, fpy, ar, gauss, dx, dy);
            a = lane_in(g.gm[q]) ? ar : 0.f;
        }
        // dL/dalpha = <dL/dC_out, c - C_in>, dL/dc = alpha dL/dC_out
        const float dla = g0 * (s.r - e[q].x) + g1 * (s.g - e[q].y) + g2 * (s.b - e[q].z);
        const bool clamped = a >= kAlphaMax;
        raw_terms(dx, dy, a, clamped, dla, a * g0, a * g1, a * g2, &v[q * 9]);
        // dL/dC_in = dL/dC_out (1 - alpha): the next entry's dL/dC_out
        const float om = 1.f - a;
        g0 *= om;
        g1 *= om;
        g2 *= om;
    }
    accumulate_groups<BG, 4>(v, L.acc, lane, slot0, g.gi, g.gm);
}

template <int TW, int TH, int BG, int EW = 4>
__device__ __forceinline__ void bwd_cached_tile(const TileJob& j, int n_tiles_total, int n,
                                                const uint32_t* __restrict__ values,
                                                const uint32_t* __restrict__ ranges, const Trace& tr,
                                                const float* __restrict__ dl_dimage,
                                                float* __restrict__ grad2d, TileLds<BG>& L) {
    constexpr int NT = TW * TH;
    constexpr int NW = NT / 64;
    const int t = threadIdx.x, lane = t & 63, wv = __builtin_amdgcn_readfirstlane(t >> 6);
    const int px = j.tx * TW + (t % TW), py = j.ty * TH + (t / TW);
    const bool inside = px < j.W && py < j.H;
    const uint32_t start = ranges[j.gt], end = ranges[n_tiles_total + j.gt];
    if (end > tr.pair_cap) return;  // no trace was recorded for this tile (uniform)
    const float fpx = (float)px + 0.5f, fpy = (float)py + 0.5f;
    const size_t pix = (size_t)py * j.W + px, plane = (size_t)j.W * j.H;
    const size_t ebase = tr.base[(size_t)j.gt * NW + wv];
    const __amdgpu_buffer_rsrc_t went = region_rsrc(tr.entry + ebase * EW);

    float g0 = 0.f, g1 = 0.f, g2 = 0.f;  // dL/dC_out of this pixel's next entry
    if (inside) {
        g0 = dl_dimage[pix];
        g1 = dl_dimage[plane + pix];
        g2 = dl_dimage[2 * plane + pix];
    }
    const uint32_t steps = tr.steps[(size_t)j.gt * NW + wv];
    __syncthreads();
    if (t == 0) L.steps = 0;
    __syncthreads();
    if (lane == 0) atomicMax(&L.steps, steps);
    __syncthreads();
    const uint32_t smax = L.steps;
    uint32_t cursor = 0;
    zero_acc<BG>(L.acc, t, NT);  // once: each flush leaves the accumulator cleared

    for (uint32_t base = 0; base < smax; base += BG) {
        const int nb = (int)min((uint32_t)BG, smax - base);
        stage_batch<NT, true>(L, j.proj, n, values, start + base, nb, t);
        __syncthreads();
        const uint32_t whi = min(base + (uint32_t)nb, steps);
        for (uint32_t c0 = base; c0 < whi; c0 += 64) {
            const uint32_t cn = min(64u, whi - c0);
            const uint64_t mv = (uint32_t)lane < cn ? tr.mask[(size_t)wv * tr.pair_cap + start + c0 + lane] : 0ull;
            uint64_t any = __ballot(mv != 0ull);
            if (!any) continue;  // uniform
            // Groups are taken four at a time and software-pipelined: the
            // next four groups' trace entries are loaded while the current
            // four are reduced.  Every lane loads (a lane without an entry in
            // a group reads the wave's first entry and takes alpha = 0 there),
            // so the count of loads in flight is fixed and the wait for the
            // current four leaves the next four outstanding.
            TraceGroups ga, gb;
            float4 ea[4], eb[4];
            take_groups(any, mv, cursor, ga);
            load_groups<EW>(went, ga, ea);
            for (;;) {
                if (!any) {
                    bwd_groups<BG, EW>(ga, ea, L, c0 - base, fpx, fpy, lane, g0, g1, g2);
                    break;
                }
                take_groups(any, mv, cursor, gb);
                load_groups<EW>(went, gb, eb);
                bwd_groups<BG, EW>(ga, ea, L, c0 - base, fpx, fpy, lane, g0, g1, g2);
                if (!any) {
                    bwd_groups<BG, EW>(gb, eb, L, c0 - base, fpx, fpy, lane, g0, g1, g2);
                    break;
                }
                take_groups(any, mv, cursor, ga);
                load_groups<EW>(went, ga, ea);
                bwd_groups<BG, EW>(gb, eb, L, c0 - base, fpx, fpy, lane, g0, g1, g2);
            }
        }
        __syncthreads();
        flush_batch<BG>(L, nb, n, grad2d, t, NT);
        __syncthreads();
    }
}

template <int TW, int TH, int BG>
__device__ __forceinline__ void bwd_recompute_tile(const TileJob& j, int n,
                                                   const uint32_t* __restrict__ values,
                                                   const uint32_t* __restrict__ ranges, float bg0,
                                                   float bg1, float bg2, const float* __restrict__ dl_dimage,
                                                   float* __restrict__ grad2d, TileLds<BG>& L) {
    constexpr int NT = TW * TH;
    const int t = threadIdx.x, lane = t & 63;
    const int px = j.tx * TW + (t % TW), py = j.ty * TH + (t / TW);
    const bool inside = px < j.W && py < j.H;
    const uint32_t start = ranges[j.gt];
    const float fpx = (float)px + 0.5f, fpy = (float)py + 0.5f;
    const size_t pix = (size_t)py * j.W + px, plane = (size_t)j.W * j.H;

    uint32_t last = 0;
    float T = 1.f, G0 = 0.f, G1 = 0.f, G2 = 0.f;
    if (inside) {
        last = j.n_contrib[pix];
        T = j.t_final[pix];
        G0 = dl_dimage[pix];
        G1 = dl_dimage[plane + pix];
        G2 = dl_dimage[2 * plane + pix];
    }
    float a0 = bg0, a1 = bg1, a2 = bg2;  // colour behind the current splat
    __syncthreads();
    if (t == 0) L.steps = 0;
    __syncthreads();
    if (last) atomicMax(&L.steps, last);
    __syncthreads();
    const uint32_t top = L.steps;
    const int wv = t >> 6;
    zero_acc<BG>(L.acc, t, NT);  // once: each flush leaves the accumulator cleared

    for (uint32_t hi = top; hi > 0;) {
        const uint32_t lo = hi > (uint32_t)BG ? hi - BG : 0u;
        const int nb = (int)(hi - lo);
        stage_batch_reach<TW, TH, NT, true>(L, j.proj, values, start + lo, nb, t, j.tx, j.ty);
        __syncthreads();
        // back to front over the steps whose splat can reach one of the
        // wave's pixels (windows of 64 last to first, scalar bit scans); the
        // gradients of four splats that some lane uses are reduced over the
        // wave together
        int cw = (nb - 1) >> 6;
        auto window = [&](int w) {
            const int k = 64 * w + lane;
            return __ballot(k < nb && ((L.reach[k] >> wv) & 1u) != 0u);
        };
        uint64_t todo = window(cw);
        bool more = true;
        while (more) {
            float v[36];
            int gi[4];
            uint64_t gm[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                gi[q] = 0;
                gm[q] = 0ull;
#pragma unroll
                for (int f = 0; f < 9; ++f) v[q * 9 + f] = 0.f;
                while (more) {
                    while (todo == 0ull && cw > 0) todo = window(--cw);
                    if (todo == 0ull) {
                        more = false;
                        break;
                    }
                    const int bit = 63 - __clzll(todo);
                    todo &= ~(1ull << bit);
                    const int k = 64 * cw + bit;
                    bool ok = false;
                    float alpha = 0.f, gauss = 0.f, dx = 0.f, dy = 0.f;
                    Splat s{};
                    if (lo + (uint32_t)k < last) {
                        s = load_splat(L.a, L.b, L.c, k);
                        ok = splat_alpha(s, fpx, fpy, alpha, gauss, dx, dy);
                    }
                    const uint64_t m = __ballot(ok);
                    if (m == 0) continue;
                    if (ok) {
                        // T_k = T_{k+1} / (1 - alpha_k), with the hardware reciprocal
                        // (about one unit of roundoff, the size of the product's own)
                        const float Tk = T * __builtin_amdgcn_rcpf(1.f - alpha);
                        const float q0 = Tk * G0, q1 = Tk * G1, q2 = Tk * G2;
                        const float dla = q0 * (s.r - a0) + q1 * (s.g - a1) + q2 * (s.b - a2);
                        const bool clamped = s.o * gauss > kAlphaMax;
                        raw_terms(dx, dy, alpha, clamped, dla, alpha * q0, alpha * q1, alpha * q2, &v[q * 9]);
                        a0 = alpha * s.r + (1.f - alpha) * a0;
                        a1 = alpha * s.g + (1.f - alpha) * a1;
                        a2 = alpha * s.b + (1.f - alpha) * a2;
                        T = Tk;
                    }
                    gi[q] = k;
                    gm[q] = m;
                    break;
                }
            }
            accumulate_groups<BG, 4>(v, L.acc, lane, 0u, gi, gm);
        }
        __syncthreads();
        flush_batch<BG>(L, nb, n, grad2d, t, NT);
        __syncthreads();
        hi = lo;
    }
}

// Checks a replay-trace descriptor and wraps it.
pgs_status make_trace(const pgs_replay* c, Trace& tr, const char* who);

// Zeroes the trace's entry counter ahead of a forward (a kernel, so that the
// call can be captured in a graph).
void reset_trace_counter(const Trace& tr, hipStream_t s);

// Tile shapes the kernels are built for (one lane per pixel, whole waves).
inline bool tile_shape_ok(int tw, int th) {
    return (tw == 16 && th == 16) || (tw == 8 && th == 8) || (tw == 16 && th == 8) ||
           (tw == 32 && th == 8) || (tw == 8 && th == 32);
}

}  // namespace pgs
