// Single-view compositing kernels: one workgroup per TW x TH tile (the tile
// pass itself, its replay trace and both backward variants are described in
// render_tile.hpp).  Splats are staged in batches of one per lane.
#include <type_traits>

#include "render_tile.hpp"

namespace {

using pgs::Trace;
using pgs::TileJob;
using pgs::TileLds;

template <int TW, int TH, bool CACHED, int EW = 4>
__global__ __launch_bounds__(TW* TH) void k_render_fwd(
    int W, int H, int TX, int tile_offset, int n_tiles_total, const float* __restrict__ proj, int n,
    const uint32_t* __restrict__ values, const uint32_t* __restrict__ ranges, float bg0, float bg1,
    float bg2, float* __restrict__ image, float* __restrict__ t_final,
    uint32_t* __restrict__ n_contrib, Trace tr, uint32_t* __restrict__ flags,
    const uint32_t* __restrict__ order) {
    constexpr int BG = TW * TH;
    __shared__ pgs::FwdLds<BG> L;
    const int tile = order ? (int)order[blockIdx.x] : (int)blockIdx.x;
    const TileJob j{W, H, tile % TX, tile / TX, tile_offset + tile, proj, image, t_final, n_contrib, tr.count};
    pgs::fwd_tile<TW, TH, BG, CACHED, EW>(j, n_tiles_total, n, values, ranges, bg0, bg1, bg2, tr, flags, L);
}

template <int TW, int TH, int EW>
__global__ __launch_bounds__(TW* TH) __attribute__((amdgpu_waves_per_eu(EW == 3 ? 6 : 1))) void k_render_bwd_cached(
    int W, int H, int TX, int tile_offset, int n_tiles_total, const float* __restrict__ proj, int n,
    const uint32_t* __restrict__ values, const uint32_t* __restrict__ ranges, Trace tr,
    const float* __restrict__ dl_dimage, float* __restrict__ grad2d, const uint32_t* __restrict__ order) {
    constexpr int BG = TW * TH;
    __shared__ TileLds<BG> L;
    const int tile = order ? (int)order[blockIdx.x] : (int)blockIdx.x;
    const TileJob j{W, H, tile % TX, tile / TX, tile_offset + tile, proj, nullptr, nullptr, nullptr, nullptr};
    pgs::bwd_cached_tile<TW, TH, BG, EW>(j, n_tiles_total, n, values, ranges, tr, dl_dimage, grad2d, L);
}

template <int TW, int TH>
__global__ __launch_bounds__(TW* TH) __attribute__((amdgpu_waves_per_eu(6))) void k_render_bwd_recompute(
    int W, int H, int TX, int tile_offset, const float* __restrict__ proj, int n,
    const uint32_t* __restrict__ values, const uint32_t* __restrict__ ranges, float bg0, float bg1,
    float bg2, const float* __restrict__ t_final, const uint32_t* __restrict__ n_contrib,
    const float* __restrict__ dl_dimage, float* __restrict__ grad2d, const uint32_t* __restrict__ order) {
    constexpr int BG = TW * TH;
    __shared__ TileLds<BG> L;
    const int tile = order ? (int)order[blockIdx.x] : (int)blockIdx.x;
    const TileJob j{W, H, tile % TX, tile / TX, tile_offset + tile, proj, nullptr, const_cast<float*>(t_final),
                    const_cast<uint32_t*>(n_contrib), nullptr};
    pgs::bwd_recompute_tile<TW, TH, BG>(j, n, values, ranges, bg0, bg1, bg2, dl_dimage, grad2d, L);
}

// Launches `body` with the kernel instance of the tile shape (TW, TH).
template <class F>
void with_tile(int tw, int th, F&& body) {
    if (tw == 16 && th == 16) body(std::integral_constant<int, 16>{}, std::integral_constant<int, 16>{});
    else if (tw == 8 && th == 8) body(std::integral_constant<int, 8>{}, std::integral_constant<int, 8>{});
    else if (tw == 16 && th == 8) body(std::integral_constant<int, 16>{}, std::integral_constant<int, 8>{});
    else if (tw == 32 && th == 8) body(std::integral_constant<int, 32>{}, std::integral_constant<int, 8>{});
    else body(std::integral_constant<int, 8>{}, std::integral_constant<int, 32>{});
}

}  // namespace

extern "C" size_t pgs_trace_entries(uint32_t pair_capacity, int32_t tile_w, int32_t tile_h) {
    return (size_t)pair_capacity * (size_t)(tile_w > 0 ? tile_w : 0) * (size_t)(tile_h > 0 ? tile_h : 0);
}

namespace {
__global__ void k_clear_u64(unsigned long long* p) {
    if (threadIdx.x == 0) *p = 0ull;
}
}  // namespace

pgs_status pgs::make_trace(const pgs_replay* c, Trace& tr, const char* who) {
    PGS_REQUIRE(c->mask_dev && c->steps_dev && c->base_dev && c->used_dev && c->entry_dev && c->count_dev,
                "%s: null trace pointer", who);
    PGS_REQUIRE(((uintptr_t)c->entry_dev % 16) == 0, "%s: trace entries must be 16-byte aligned", who);
    PGS_REQUIRE(c->entry_capacity <= 0xffffffffull, "%s: entry capacity %llu above 2^32 - 1", who,
                (unsigned long long)c->entry_capacity);
    PGS_REQUIRE(c->entry_words == 3 || c->entry_words == 4, "%s: entry_words %u is neither 3 nor 4", who,
                c->entry_words);
    tr = Trace{c->mask_dev, c->steps_dev, c->base_dev, reinterpret_cast<unsigned long long*>(c->used_dev),
               c->entry_dev, c->count_dev, (size_t)c->entry_capacity, c->pair_capacity, (int)c->entry_words};
    return PGS_OK;
}

void pgs::reset_trace_counter(const Trace& tr, hipStream_t s) { k_clear_u64<<<1, 64, 0, s>>>(tr.used); }

extern "C" pgs_status pgs_render_fwd(int32_t width, int32_t height, int32_t tile_w, int32_t tile_h,
                                     const float* proj_dev, int32_t n, const uint32_t* values_dev,
                                     const uint32_t* ranges_dev, int32_t view_tile_offset,
                                     const float* bg_host, float* image_dev, float* t_final_dev,
                                     uint32_t* n_contrib_dev, const pgs_replay* cache,
                                     uint32_t* flags_dev, const uint32_t* tile_order_dev, void* stream) {
    PGS_REQUIRE(width > 0 && height > 0 && n >= 0 && view_tile_offset >= 0, "pgs_render_fwd: bad sizes");
    PGS_REQUIRE(pgs::tile_shape_ok(tile_w, tile_h), "pgs_render_fwd: unsupported tile %dx%d", tile_w, tile_h);
    PGS_REQUIRE(bg_host && ranges_dev && image_dev && t_final_dev && n_contrib_dev,
                "pgs_render_fwd: null pointer");
    PGS_REQUIRE(n == 0 || (proj_dev && values_dev), "pgs_render_fwd: null pointer");
    const int TX = (width + tile_w - 1) / tile_w, TY = (height + tile_h - 1) / tile_h;
    const int n_tiles_total = view_tile_offset + TX * TY;
    Trace tr{};
    if (cache) {
        PGS_REQUIRE(flags_dev != nullptr, "pgs_render_fwd: a trace needs the flags word");
        pgs_status st = pgs::make_trace(cache, tr, "pgs_render_fwd");
        if (st != PGS_OK) return st;
    }
    hipStream_t s = pgs::as_stream(stream);
    if (cache) pgs::reset_trace_counter(tr, s);
    with_tile(tile_w, tile_h, [&](auto TWc, auto THc) {
        constexpr int TW = decltype(TWc)::value, TH = decltype(THc)::value;
        const dim3 grid(TX * TY), block(TW * TH);
        if (cache && tr.words == 3)
            k_render_fwd<TW, TH, true, 3><<<grid, block, 0, s>>>(width, height, TX, view_tile_offset,
                                                                 n_tiles_total, proj_dev, n, values_dev, ranges_dev,
                                                                 bg_host[0], bg_host[1], bg_host[2], image_dev,
                                                                 t_final_dev, n_contrib_dev, tr, flags_dev,
                                                                 tile_order_dev);
        else if (cache)
            k_render_fwd<TW, TH, true, 4><<<grid, block, 0, s>>>(width, height, TX, view_tile_offset,
                                                                 n_tiles_total, proj_dev, n, values_dev, ranges_dev,
                                                                 bg_host[0], bg_host[1], bg_host[2], image_dev,
                                                                 t_final_dev, n_contrib_dev, tr, flags_dev,
                                                                 tile_order_dev);
        else
            k_render_fwd<TW, TH, false><<<grid, block, 0, s>>>(width, height, TX, view_tile_offset,
                                                               n_tiles_total, proj_dev, n, values_dev, ranges_dev,
                                                               bg_host[0], bg_host[1], bg_host[2], image_dev,
                                                               t_final_dev, n_contrib_dev, tr, flags_dev,
                                                               tile_order_dev);
    });
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
    PGS_REQUIRE(pgs::tile_shape_ok(tile_w, tile_h), "pgs_render_bwd: unsupported tile %dx%d", tile_w, tile_h);
    PGS_REQUIRE(bg_host && ranges_dev && dl_dimage_dev, "pgs_render_bwd: null pointer");
    if (n == 0) return PGS_OK;
    PGS_REQUIRE(proj_dev && values_dev && grad2d_dev, "pgs_render_bwd: null pointer");
    const int TX = (width + tile_w - 1) / tile_w, TY = (height + tile_h - 1) / tile_h;
    const int n_tiles_total = view_tile_offset + TX * TY;
    hipStream_t s = pgs::as_stream(stream);
    Trace tr{};
    if (cache) {
        pgs_status st = pgs::make_trace(cache, tr, "pgs_render_bwd");
        if (st != PGS_OK) return st;
    } else {
        PGS_REQUIRE(t_final_dev && n_contrib_dev, "pgs_render_bwd: null pointer");
    }
    with_tile(tile_w, tile_h, [&](auto TWc, auto THc) {
        constexpr int TW = decltype(TWc)::value, TH = decltype(THc)::value;
        const dim3 grid(TX * TY), block(TW * TH);
        if (cache && tr.words == 3)
            k_render_bwd_cached<TW, TH, 3><<<grid, block, 0, s>>>(width, height, TX, view_tile_offset,
                                                                  n_tiles_total, proj_dev, n, values_dev, ranges_dev,
                                                                  tr, dl_dimage_dev, grad2d_dev, tile_order_dev);
        else if (cache)
            k_render_bwd_cached<TW, TH, 4><<<grid, block, 0, s>>>(width, height, TX, view_tile_offset,
                                                                  n_tiles_total, proj_dev, n, values_dev, ranges_dev,
                                                                  tr, dl_dimage_dev, grad2d_dev, tile_order_dev);
        else
            k_render_bwd_recompute<TW, TH><<<grid, block, 0, s>>>(width, height, TX, view_tile_offset, proj_dev, n,
                                                                  values_dev, ranges_dev, bg_host[0], bg_host[1],
                                                                  bg_host[2], t_final_dev, n_contrib_dev,
                                                                  dl_dimage_dev, grad2d_dev, tile_order_dev);
    });
    PGS_CHECK_LAUNCH("pgs_render_bwd");
    return PGS_OK;
}
