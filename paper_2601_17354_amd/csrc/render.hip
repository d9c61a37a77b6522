// Per-tile compositing forward and its backward.
//
// Forward (PocketGS Sec. "Explicit Computation Graph", "Bandwidth-Efficient
// Forward Replay Cache"): one workgroup per tile, one lane per pixel.  The
// tile's sorted splat list is staged through LDS in batches (one splat per
// lane per batch, 36 B of 2D attributes each); every lane composites the
// batch front to back.  A barrier with a live-lane count ends the tile once
// every pixel has terminated.  In cached mode each contributing splat appends
// {id, alpha, c} to the pixel's trace slot count(u); after the pass the lane
// walks its own entries back to front and overwrites c with C_in, the colour
// behind the splat (the over-recursion C_out = C_in (1 - alpha) + alpha c run
// from the background), so the backward reads C_in directly.
//
// Backward (equation "backward_chain"), two variants:
//   cached     walks each pixel's trace front to back.  The workgroup steps
//              through the tile's list in lockstep; a lane consumes its next
//              trace entry when the entry's id equals the current list
//              position, so all lanes of a wave work on the same splat and
//              the wave reduces its nine 2D gradients with DPP before LDS
//              accumulation and one float atomic per field and tile.
//              dL/dC_out starts at dL/dC and is multiplied by (1 - alpha)
//              after every entry (dL/dC_in = dL/dC_out (1 - alpha)).
//   recompute  walks the list back to front from n_contrib, re-evaluates
//              alpha with the forward's exact arithmetic, recovers
//              T_k = T_{k+1} / (1 - alpha_k) from T_final and accumulates the
//              colour behind as it goes.
// Gradients are scattered to the canonical index values[j] (index-mapping
// equation).
#include "common.hpp"

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

struct Trace {
    uint32_t* id;
    float* alpha;
    float* c_in;
    uint32_t* count;
    int k_max;
    size_t slots;
};

template <int TW, int TH, bool CACHED>
__global__ __launch_bounds__(TW* TH) void k_render_fwd(
    int W, int H, int TX, int tile_offset, int n_tiles_total, const float* __restrict__ proj, int n,
    const uint32_t* __restrict__ values, const uint32_t* __restrict__ ranges, float bg0, float bg1,
    float bg2, float* __restrict__ image, float* __restrict__ t_final,
    uint32_t* __restrict__ n_contrib, Trace tr, uint32_t* __restrict__ flags) {
    constexpr int NT = TW * TH;
    __shared__ float4 s_a[NT];
    __shared__ float4 s_b[NT];
    __shared__ float s_c[NT];
    const int tile = blockIdx.x;
    const int tx = tile % TX, ty = tile / TX;
    const int t = threadIdx.x;
    const int px = tx * TW + (t % TW), py = ty * TH + (t / TW);
    const bool inside = px < W && py < H;
    const int gt = tile_offset + tile;
    const uint32_t start = ranges[gt], end = ranges[n_tiles_total + gt];
    const float fpx = (float)px + 0.5f, fpy = (float)py + 0.5f;

    float T = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f;
    bool done = !inside;
    uint32_t last = 0, cnt = 0;
    const size_t tbase = (size_t)gt * (size_t)(CACHED ? tr.k_max : 0);

    for (uint32_t base = start; base < end; base += NT) {
        if (__syncthreads_count(!done) == 0) break;
        if (base + t < end) stage_splat(proj, n, values[base + t], s_a, s_b, s_c, t);
        __syncthreads();
        const int nb = (int)min((uint32_t)NT, end - base);
        for (int k = 0; k < nb && !done; ++k) {
            const Splat s = load_splat(s_a, s_b, s_c, k);
            float alpha, gauss, dx, dy;
            if (!splat_alpha(s, fpx, fpy, alpha, gauss, dx, dy)) continue;
            const float test_T = T * (1.f - alpha);
            if (test_T < kTMin) {
                done = true;
                break;
            }
            const float w = alpha * T;
            C0 += w * s.r;
            C1 += w * s.g;
            C2 += w * s.b;
            if (CACHED) {
                if (cnt < (uint32_t)tr.k_max) {
                    const size_t e = (tbase + cnt) * NT + t;
                    tr.id[e] = base + k;
                    tr.alpha[e] = alpha;
                    tr.c_in[e] = s.r;
                    tr.c_in[tr.slots + e] = s.g;
                    tr.c_in[2 * tr.slots + e] = s.b;
                }
                ++cnt;
            }
            T = test_T;
            last = base + k - start + 1;
        }
    }
    if (!inside) return;
    const size_t pix = (size_t)py * W + px, plane = (size_t)W * H;
    image[pix] = C0 + T * bg0;
    image[plane + pix] = C1 + T * bg1;
    image[2 * plane + pix] = C2 + T * bg2;
    t_final[pix] = T;
    n_contrib[pix] = last;
    if (CACHED) {
        uint32_t kept = cnt;
        if (cnt > (uint32_t)tr.k_max) {
            kept = (uint32_t)tr.k_max;
            atomicOr(flags, PGS_FLAG_CACHE_OVERFLOW);
        }
        tr.count[pix] = kept;
        // C_in of each entry: everything behind it, from the background forward
        float a0 = bg0, a1 = bg1, a2 = bg2;
        for (int k = (int)kept - 1; k >= 0; --k) {
            const size_t e = (tbase + k) * NT + t;
            const float al = tr.alpha[e];
            const float r = tr.c_in[e], g = tr.c_in[tr.slots + e], b = tr.c_in[2 * tr.slots + e];
            tr.c_in[e] = a0;
            tr.c_in[tr.slots + e] = a1;
            tr.c_in[2 * tr.slots + e] = a2;
            a0 = al * r + (1.f - al) * a0;
            a1 = al * g + (1.f - al) * a1;
            a2 = al * b + (1.f - al) * a2;
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

template <int NW, int BG>
__device__ __forceinline__ void reduce_to_lds(float* v, float (*acc)[9][BG], int wv, int lane, int jj) {
#pragma unroll
    for (int f = 0; f < 9; ++f) {
        const float sum = wave_sum_to_lane63(v[f]);
        if (lane == 63) acc[wv][f][jj] = sum;
    }
}

template <int NW, int BG>
__device__ __forceinline__ void flush_batch(float (*acc)[9][BG], const uint32_t* gid, int nb, int n,
                                            float* __restrict__ grad2d, int t, int NT) {
    for (int idx = t; idx < nb * 9; idx += NT) {
        const int f = idx / nb, jj = idx - f * nb;
        float s = 0.f;
#pragma unroll
        for (int w = 0; w < NW; ++w) s += acc[w][f][jj];
        if (s != 0.f) unsafeAtomicAdd(&grad2d[(size_t)f * n + gid[jj]], s);
    }
}

template <int TW, int TH>
__global__ __launch_bounds__(TW* TH) void k_render_bwd_cached(
    int W, int H, int TX, int tile_offset, int n_tiles_total, const float* __restrict__ proj, int n,
    const uint32_t* __restrict__ values, const uint32_t* __restrict__ ranges, Trace tr,
    const float* __restrict__ dl_dimage, float* __restrict__ grad2d) {
    constexpr int NT = TW * TH;
    constexpr int NW = NT / 64;
    constexpr int BG = NT;
    __shared__ float4 s_a[BG];
    __shared__ float4 s_b[BG];
    __shared__ float s_c[BG];
    __shared__ uint32_t s_g[BG];
    __shared__ float s_acc[NW][9][BG];
    __shared__ uint32_t s_end;
    const int tile = blockIdx.x;
    const int tx = tile % TX, ty = tile / TX;
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    const int px = tx * TW + (t % TW), py = ty * TH + (t / TW);
    const bool inside = px < W && py < H;
    const int gt = tile_offset + tile;
    const uint32_t start = ranges[gt];
    const float fpx = (float)px + 0.5f, fpy = (float)py + 0.5f;
    const size_t tbase = (size_t)gt * (size_t)tr.k_max;
    const size_t pix = (size_t)py * W + px, plane = (size_t)W * H;

    uint32_t cnt = 0;
    float g0 = 0.f, g1 = 0.f, g2 = 0.f;
    if (inside) {
        cnt = tr.count[pix];
        g0 = dl_dimage[pix];
        g1 = dl_dimage[plane + pix];
        g2 = dl_dimage[2 * plane + pix];
    }
    // current entry in registers
    uint32_t k = 0, cur_id = 0xffffffffu;
    float cur_a = 0.f, cur_c0 = 0.f, cur_c1 = 0.f, cur_c2 = 0.f;
    auto fetch = [&](uint32_t kk) {
        if (kk < cnt) {
            const size_t e = (tbase + kk) * NT + t;
            cur_id = tr.id[e];
            cur_a = tr.alpha[e];
            cur_c0 = tr.c_in[e];
            cur_c1 = tr.c_in[tr.slots + e];
            cur_c2 = tr.c_in[2 * tr.slots + e];
        } else {
            cur_id = 0xffffffffu;
        }
    };
    if (t == 0) s_end = 0;
    uint32_t my_end = 0;
    if (cnt > 0) my_end = tr.id[(tbase + cnt - 1) * NT + t] + 1;
    fetch(0);
    __syncthreads();
    if (my_end) atomicMax(&s_end, my_end);
    __syncthreads();
    const uint32_t end = s_end;

    for (uint32_t base = start; base < end; base += BG) {
        const int nb = (int)min((uint32_t)BG, end - base);
        if (t < nb) {
            const uint32_t g = values[base + t];
            s_g[t] = g;
            stage_splat(proj, n, g, s_a, s_b, s_c, t);
        }
        for (int idx = t; idx < NW * 9 * BG; idx += NT) (&s_acc[0][0][0])[idx] = 0.f;
        __syncthreads();
        for (int jj = 0; jj < nb; ++jj) {
            const bool match = cur_id == base + jj;
            if (__ballot(match) == 0) continue;
            float v[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
            if (match) {
                const Splat s = load_splat(s_a, s_b, s_c, jj);
                const float dx = s.u - fpx, dy = s.v - fpy;
                const float al = cur_a;
                // dL/dalpha = <dL/dC_out, c - C_in>, dL/dc = alpha dL/dC_out
                const float dla = g0 * (s.r - cur_c0) + g1 * (s.g - cur_c1) + g2 * (s.b - cur_c2);
                const bool clamped = al >= kAlphaMax;
                chain_2d(s, dx, dy, al, clamped ? 0.f : al / s.o, clamped, dla, al * g0, al * g1,
                         al * g2, v);
                // dL/dC_in = dL/dC_out (1 - alpha) is the next entry's dL/dC_out
                const float om = 1.f - al;
                g0 *= om;
                g1 *= om;
                g2 *= om;
                ++k;
                fetch(k);
            }
            reduce_to_lds<NW, BG>(v, s_acc, wv, lane, jj);
        }
        __syncthreads();
        flush_batch<NW, BG>(s_acc, s_g, nb, n, grad2d, t, NT);
        __syncthreads();
    }
}

template <int TW, int TH>
__global__ __launch_bounds__(TW* TH) void k_render_bwd_recompute(
    int W, int H, int TX, int tile_offset, int n_tiles_total, const float* __restrict__ proj, int n,
    const uint32_t* __restrict__ values, const uint32_t* __restrict__ ranges, float bg0, float bg1,
    float bg2, const float* __restrict__ t_final, const uint32_t* __restrict__ n_contrib,
    const float* __restrict__ dl_dimage, float* __restrict__ grad2d) {
    constexpr int NT = TW * TH;
    constexpr int NW = NT / 64;
    constexpr int BG = NT;
    __shared__ float4 s_a[BG];
    __shared__ float4 s_b[BG];
    __shared__ float s_c[BG];
    __shared__ uint32_t s_g[BG];
    __shared__ float s_acc[NW][9][BG];
    __shared__ uint32_t s_last;
    const int tile = blockIdx.x;
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
        for (int idx = t; idx < NW * 9 * BG; idx += NT) (&s_acc[0][0][0])[idx] = 0.f;
        __syncthreads();
        for (int jj = nb - 1; jj >= 0; --jj) {
            const uint32_t jrel = lo + jj;
            bool ok = false;
            float alpha = 0.f, gauss = 0.f, dx = 0.f, dy = 0.f;
            Splat s;
            if (jrel < last) {
                s = load_splat(s_a, s_b, s_c, jj);
                ok = splat_alpha(s, fpx, fpy, alpha, gauss, dx, dy);
            }
            if (__ballot(ok) == 0) continue;
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
            reduce_to_lds<NW, BG>(v, s_acc, wv, lane, jj);
        }
        __syncthreads();
        flush_batch<NW, BG>(s_acc, s_g, nb, n, grad2d, t, NT);
        __syncthreads();
        hi = lo;
    }
}

bool tile_ok(int tw, int th) { return tw == 16 && th == 16; }

}  // namespace

extern "C" pgs_status pgs_render_fwd(int32_t width, int32_t height, int32_t tile_w, int32_t tile_h,
                                     const float* proj_dev, int32_t n, const uint32_t* values_dev,
                                     const uint32_t* ranges_dev, int32_t view_tile_offset,
                                     const float* bg_host, float* image_dev, float* t_final_dev,
                                     uint32_t* n_contrib_dev, const pgs_replay* cache,
                                     uint32_t* flags_dev, void* stream) {
    PGS_REQUIRE(width > 0 && height > 0 && n >= 0 && view_tile_offset >= 0, "pgs_render_fwd: bad sizes");
    PGS_REQUIRE(tile_ok(tile_w, tile_h), "pgs_render_fwd: unsupported tile %dx%d", tile_w, tile_h);
    PGS_REQUIRE(bg_host && ranges_dev && image_dev && t_final_dev && n_contrib_dev,
                "pgs_render_fwd: null pointer");
    PGS_REQUIRE(n == 0 || (proj_dev && values_dev), "pgs_render_fwd: null pointer");
    const int TX = (width + tile_w - 1) / tile_w, TY = (height + tile_h - 1) / tile_h;
    const int n_tiles_total = view_tile_offset + TX * TY;
    Trace tr{};
    if (cache) {
        PGS_REQUIRE(cache->id_dev && cache->alpha_dev && cache->c_in_dev && cache->count_dev &&
                        cache->k_max > 0 && flags_dev, "pgs_render_fwd: bad trace");
        tr = Trace{cache->id_dev, cache->alpha_dev, cache->c_in_dev, cache->count_dev, cache->k_max,
                   (size_t)n_tiles_total * cache->k_max * tile_w * tile_h};
    }
    hipStream_t s = pgs::as_stream(stream);
    const dim3 grid(TX * TY), block(256);
    if (cache)
        k_render_fwd<16, 16, true><<<grid, block, 0, s>>>(width, height, TX, view_tile_offset, n_tiles_total,
                                                          proj_dev, n, values_dev, ranges_dev, bg_host[0],
                                                          bg_host[1], bg_host[2], image_dev, t_final_dev,
                                                          n_contrib_dev, tr, flags_dev);
    else
        k_render_fwd<16, 16, false><<<grid, block, 0, s>>>(width, height, TX, view_tile_offset, n_tiles_total,
                                                           proj_dev, n, values_dev, ranges_dev, bg_host[0],
                                                           bg_host[1], bg_host[2], image_dev, t_final_dev,
                                                           n_contrib_dev, tr, flags_dev);
    PGS_CHECK_LAUNCH("pgs_render_fwd");
    return PGS_OK;
}

extern "C" pgs_status pgs_render_bwd(int32_t width, int32_t height, int32_t tile_w, int32_t tile_h,
                                     const float* proj_dev, int32_t n, const uint32_t* values_dev,
                                     const uint32_t* ranges_dev, int32_t view_tile_offset,
                                     const float* bg_host, const float* t_final_dev,
                                     const uint32_t* n_contrib_dev, const pgs_replay* cache,
                                     const float* dl_dimage_dev, float* grad2d_dev, void* stream) {
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
        PGS_REQUIRE(cache->id_dev && cache->alpha_dev && cache->c_in_dev && cache->count_dev &&
                        cache->k_max > 0, "pgs_render_bwd: bad trace");
        Trace tr{cache->id_dev, cache->alpha_dev, cache->c_in_dev, cache->count_dev, cache->k_max,
                 (size_t)n_tiles_total * cache->k_max * tile_w * tile_h};
        k_render_bwd_cached<16, 16><<<grid, block, 0, s>>>(width, height, TX, view_tile_offset, n_tiles_total,
                                                           proj_dev, n, values_dev, ranges_dev, tr,
                                                           dl_dimage_dev, grad2d_dev);
    } else {
        PGS_REQUIRE(t_final_dev && n_contrib_dev, "pgs_render_bwd: null pointer");
        k_render_bwd_recompute<16, 16><<<grid, block, 0, s>>>(width, height, TX, view_tile_offset,
                                                              n_tiles_total, proj_dev, n, values_dev,
                                                              ranges_dev, bg_host[0], bg_host[1], bg_host[2],
                                                              t_final_dev, n_contrib_dev, dl_dimage_dev,
                                                              grad2d_dev);
    }
    PGS_CHECK_LAUNCH("pgs_render_bwd");
    return PGS_OK;
}
