// Several views of uneven resolution in one launch.
//
// Tiles of all views share one global numbering (view v's tiles start at
// tile_offset[v]), so one key sort orders every (view, tile, depth) pair and
// one ranges array indexes them.  The compositing forward and both backward
// variants run as persistent launches: each workgroup pulls global tile
// indices from an atomic queue (in the heavy-first order of pgs_tile_order
// when given) until the queue is exhausted, and runs the same tile pass as
// the single-view kernels on the view that owns the tile.  Tile shape and
// the number of splats staged per LDS batch are template parameters so that
// a tuner can pick them per workload.
#include <type_traits>

#include "render_tile.hpp"

namespace {

using pgs::TileJob;
using pgs::Trace;

constexpr int kMaxViews = PGS_MAX_VIEWS;

struct ViewTable {
    int n_views;
    int W[kMaxViews], H[kMaxViews], TX[kMaxViews];
    int tile_off[kMaxViews + 1];
    long long pix_off[kMaxViews + 1];
    float bg[3];
};

__device__ __forceinline__ int view_of(const ViewTable& vt, int gt) {
    int v = 0;
    while (v + 1 < vt.n_views && gt >= vt.tile_off[v + 1]) ++v;
    return v;
}

// Next queue item for the whole workgroup (one atomic per tile).
__device__ __forceinline__ uint32_t next_item(uint32_t* queue, uint32_t* s_item) {
    __syncthreads();  // the previous tile's LDS and *s_item are no longer read
    if (threadIdx.x == 0) *s_item = atomicAdd(queue, 1u);
    __syncthreads();
    return *s_item;
}

__device__ __forceinline__ TileJob job_of(const ViewTable& vt, int gt, const float* proj_all, int n,
                                          float* image_all, float* t_final_all, uint32_t* n_contrib_all,
                                          uint32_t* count_all, int& v) {
    v = view_of(vt, gt);
    const int tile = gt - vt.tile_off[v];
    const size_t p0 = (size_t)vt.pix_off[v];
    return TileJob{vt.W[v], vt.H[v], tile % vt.TX[v], tile / vt.TX[v], gt,
                   proj_all + (size_t)v * PGS_PROJ_STRIDE * n,
                   image_all ? image_all + 3 * p0 : nullptr, t_final_all ? t_final_all + p0 : nullptr,
                   n_contrib_all ? n_contrib_all + p0 : nullptr, count_all ? count_all + p0 : nullptr};
}

__global__ void k_clear_queue(uint32_t* queue) {
    if (threadIdx.x == 0) *queue = 0u;
}

template <int TW, int TH, int BG, bool CACHED, int EW = 4>
__global__ __launch_bounds__(TW* TH) __attribute__((amdgpu_waves_per_eu(CACHED ? 5 : 1))) void k_render_fwd_views(
    ViewTable vt, int n_tiles_total, const float* __restrict__ proj_all, int n,
    const uint32_t* __restrict__ values, const uint32_t* __restrict__ ranges, float* __restrict__ image_all,
    float* __restrict__ t_final_all, uint32_t* __restrict__ n_contrib_all, Trace tr,
    uint32_t* __restrict__ flags, const uint32_t* __restrict__ order, uint32_t* __restrict__ queue) {
    __shared__ pgs::FwdLds<BG> L;
    __shared__ uint32_t s_item;
    for (;;) {
        const uint32_t item = next_item(queue, &s_item);
        if (item >= (uint32_t)n_tiles_total) break;
        const int gt = order ? (int)order[item] : (int)item;
        int v;
        const TileJob j = job_of(vt, gt, proj_all, n, image_all, t_final_all, n_contrib_all,
                                 CACHED ? tr.count : nullptr, v);
        pgs::fwd_tile<TW, TH, BG, CACHED, EW>(j, n_tiles_total, n, values, ranges, vt.bg[0], vt.bg[1], vt.bg[2],
                                              tr, flags, L);
    }
}

template <int TW, int TH, int BG, bool CACHED, int EW = 4>
__global__ __launch_bounds__(TW* TH) void k_render_bwd_views(
    ViewTable vt, int n_tiles_total, const float* __restrict__ proj_all, int n,
    const uint32_t* __restrict__ values, const uint32_t* __restrict__ ranges,
    const float* __restrict__ t_final_all, const uint32_t* __restrict__ n_contrib_all, Trace tr,
    const float* __restrict__ dl_all, float* __restrict__ grad2d_all, const uint32_t* __restrict__ order,
    uint32_t* __restrict__ queue) {
    __shared__ pgs::TileLds<BG> L;
    __shared__ uint32_t s_item;
    for (;;) {
        const uint32_t item = next_item(queue, &s_item);
        if (item >= (uint32_t)n_tiles_total) break;
        const int gt = order ? (int)order[item] : (int)item;
        int v;
        const TileJob j = job_of(vt, gt, proj_all, n, nullptr, const_cast<float*>(t_final_all),
                                 const_cast<uint32_t*>(n_contrib_all), nullptr, v);
        const float* dl = dl_all + 3 * (size_t)vt.pix_off[v];
        float* g2 = grad2d_all + (size_t)v * PGS_GRAD2D_STRIDE * n;
        if constexpr (CACHED)
            pgs::bwd_cached_tile<TW, TH, BG, EW>(j, n_tiles_total, n, values, ranges, tr, dl, g2, L);
        else
            pgs::bwd_recompute_tile<TW, TH, BG>(j, n, values, ranges, vt.bg[0], vt.bg[1], vt.bg[2], dl, g2, L);
    }
}

template <int V>
using IC = std::integral_constant<int, V>;

// Calls body(TW, TH, BG) with the compile-time configuration.
template <class F>
void with_config(int tw, int th, int bg, F&& body) {
    auto with_bg = [&](auto TWc, auto THc) {
        switch (bg) {
            case 32: body(TWc, THc, IC<32>{}); break;
            case 64: body(TWc, THc, IC<64>{}); break;
            case 128: body(TWc, THc, IC<128>{}); break;
            default: body(TWc, THc, IC<256>{}); break;
        }
    };
    if (tw == 16 && th == 16) with_bg(IC<16>{}, IC<16>{});
    else if (tw == 8 && th == 8) with_bg(IC<8>{}, IC<8>{});
    else if (tw == 16 && th == 8) with_bg(IC<16>{}, IC<8>{});
    else if (tw == 32 && th == 8) with_bg(IC<32>{}, IC<8>{});
    else with_bg(IC<8>{}, IC<32>{});
}

bool batch_ok(int bg) { return bg == 32 || bg == 64 || bg == 128 || bg == 256; }

pgs_status check_batch(const pgs_view_batch* vb, const char* who) {
    pgs_status st = pgs::check_views(vb, who);
    if (st != PGS_OK) return st;
    PGS_REQUIRE(pgs::tile_shape_ok(vb->tile_w, vb->tile_h), "%s: unsupported tile %dx%d", who, vb->tile_w,
                vb->tile_h);
    PGS_REQUIRE(batch_ok(vb->batch), "%s: batch %d not in {32, 64, 128, 256}", who, vb->batch);
    PGS_REQUIRE(vb->blocks >= 0, "%s: blocks must be >= 0", who);
    return PGS_OK;
}

ViewTable make_table(const pgs_view_batch* vb, const float* bg) {
    const pgs::ViewsLayout lay = pgs::views_layout(*vb);
    ViewTable vt{};
    vt.n_views = vb->n_views;
    for (int v = 0; v < vb->n_views; ++v) {
        vt.W[v] = vb->cams[v].width;
        vt.H[v] = vb->cams[v].height;
        vt.TX[v] = lay.TX[v];
    }
    for (int v = 0; v <= vb->n_views; ++v) {
        vt.tile_off[v] = lay.tile_off[v];
        vt.pix_off[v] = lay.pix_off[v];
    }
    for (int c = 0; c < 3; ++c) vt.bg[c] = bg ? bg[c] : 0.f;
    return vt;
}

// Workgroups of a persistent launch: as many as the device keeps resident.
template <class K>
int resident_blocks(K kernel, int threads, int requested, int items) {
    int blocks = requested;
    if (blocks <= 0) {
        int per_cu = 0, dev = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess || per_cu < 1)
            per_cu = 1;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
            cus = 256;
        blocks = per_cu * cus;
    }
    return blocks < items ? blocks : items;
}

}  // namespace

extern "C" int32_t pgs_views_layout(const pgs_view_batch* vb, int32_t* tile_offsets, int64_t* pixel_offsets) {
    if (check_batch(vb, "pgs_views_layout") != PGS_OK) return -1;
    const ViewTable vt = make_table(vb, nullptr);
    for (int v = 0; v <= vb->n_views; ++v) {
        if (tile_offsets) tile_offsets[v] = vt.tile_off[v];
        if (pixel_offsets) pixel_offsets[v] = vt.pix_off[v];
    }
    return vt.tile_off[vb->n_views];
}

extern "C" pgs_status pgs_render_fwd_views(const pgs_view_batch* vb, const float* proj_all_dev, int32_t n,
                                           const uint32_t* values_dev, const uint32_t* ranges_dev,
                                           const float* bg_host, float* image_all_dev, float* t_final_all_dev,
                                           uint32_t* n_contrib_all_dev, const pgs_replay* cache,
                                           uint32_t* flags_dev, const uint32_t* tile_order_dev,
                                           uint32_t* queue_dev, void* stream) {
    pgs_status st = check_batch(vb, "pgs_render_fwd_views");
    if (st != PGS_OK) return st;
    PGS_REQUIRE(n >= 0, "pgs_render_fwd_views: n must be >= 0");
    PGS_REQUIRE(bg_host && ranges_dev && image_all_dev && t_final_all_dev && n_contrib_all_dev && queue_dev,
                "pgs_render_fwd_views: null pointer");
    PGS_REQUIRE(n == 0 || (proj_all_dev && values_dev), "pgs_render_fwd_views: null pointer");
    const ViewTable vt = make_table(vb, bg_host);
    const int total = vt.tile_off[vb->n_views];
    Trace tr{};
    if (cache) {
        PGS_REQUIRE(flags_dev != nullptr, "pgs_render_fwd_views: a trace needs the flags word");
        st = pgs::make_trace(cache, tr, "pgs_render_fwd_views");
        if (st != PGS_OK) return st;
    }
    hipStream_t s = pgs::as_stream(stream);
    k_clear_queue<<<1, 64, 0, s>>>(queue_dev);
    if (cache) pgs::reset_trace_counter(tr, s);
    with_config(vb->tile_w, vb->tile_h, vb->batch, [&](auto TWc, auto THc, auto BGc) {
        constexpr int TW = decltype(TWc)::value, TH = decltype(THc)::value, BG = decltype(BGc)::value;
        if (cache && tr.words == 3) {
            auto k = k_render_fwd_views<TW, TH, BG, true, 3>;
            const int blocks = resident_blocks(k, TW * TH, vb->blocks, total);
            k<<<blocks, TW * TH, 0, s>>>(vt, total, proj_all_dev, n, values_dev, ranges_dev, image_all_dev,
                                         t_final_all_dev, n_contrib_all_dev, tr, flags_dev, tile_order_dev,
                                         queue_dev);
        } else if (cache) {
            auto k = k_render_fwd_views<TW, TH, BG, true, 4>;
            const int blocks = resident_blocks(k, TW * TH, vb->blocks, total);
            k<<<blocks, TW * TH, 0, s>>>(vt, total, proj_all_dev, n, values_dev, ranges_dev, image_all_dev,
                                         t_final_all_dev, n_contrib_all_dev, tr, flags_dev, tile_order_dev,
                                         queue_dev);
        } else {
            auto k = k_render_fwd_views<TW, TH, BG, false>;
            const int blocks = resident_blocks(k, TW * TH, vb->blocks, total);
            k<<<blocks, TW * TH, 0, s>>>(vt, total, proj_all_dev, n, values_dev, ranges_dev, image_all_dev,
                                         t_final_all_dev, n_contrib_all_dev, tr, flags_dev, tile_order_dev,
                                         queue_dev);
        }
    });
    PGS_CHECK_LAUNCH("pgs_render_fwd_views");
    return PGS_OK;
}

extern "C" pgs_status pgs_render_bwd_views(const pgs_view_batch* vb, const float* proj_all_dev, int32_t n,
                                           const uint32_t* values_dev, const uint32_t* ranges_dev,
                                           const float* bg_host, const float* t_final_all_dev,
                                           const uint32_t* n_contrib_all_dev, const pgs_replay* cache,
                                           const float* dl_all_dev, float* grad2d_all_dev,
                                           const uint32_t* tile_order_dev, uint32_t* queue_dev, void* stream) {
    pgs_status st = check_batch(vb, "pgs_render_bwd_views");
    if (st != PGS_OK) return st;
    PGS_REQUIRE(n >= 0, "pgs_render_bwd_views: n must be >= 0");
    PGS_REQUIRE(bg_host && ranges_dev && dl_all_dev && queue_dev, "pgs_render_bwd_views: null pointer");
    if (n == 0) return PGS_OK;
    PGS_REQUIRE(proj_all_dev && values_dev && grad2d_all_dev, "pgs_render_bwd_views: null pointer");
    const ViewTable vt = make_table(vb, bg_host);
    const int total = vt.tile_off[vb->n_views];
    Trace tr{};
    if (cache) {
        st = pgs::make_trace(cache, tr, "pgs_render_bwd_views");
        if (st != PGS_OK) return st;
    } else {
        PGS_REQUIRE(t_final_all_dev && n_contrib_all_dev, "pgs_render_bwd_views: null pointer");
    }
    hipStream_t s = pgs::as_stream(stream);
    k_clear_queue<<<1, 64, 0, s>>>(queue_dev);
    with_config(vb->tile_w, vb->tile_h, vb->batch, [&](auto TWc, auto THc, auto BGc) {
        constexpr int TW = decltype(TWc)::value, TH = decltype(THc)::value, BG = decltype(BGc)::value;
        if (cache && tr.words == 3) {
            auto k = k_render_bwd_views<TW, TH, BG, true, 3>;
            const int blocks = resident_blocks(k, TW * TH, vb->blocks, total);
            k<<<blocks, TW * TH, 0, s>>>(vt, total, proj_all_dev, n, values_dev, ranges_dev, t_final_all_dev,
                                         n_contrib_all_dev, tr, dl_all_dev, grad2d_all_dev, tile_order_dev,
                                         queue_dev);
        } else if (cache) {
            auto k = k_render_bwd_views<TW, TH, BG, true, 4>;
            const int blocks = resident_blocks(k, TW * TH, vb->blocks, total);
            k<<<blocks, TW * TH, 0, s>>>(vt, total, proj_all_dev, n, values_dev, ranges_dev, t_final_all_dev,
                                         n_contrib_all_dev, tr, dl_all_dev, grad2d_all_dev, tile_order_dev,
                                         queue_dev);
        } else {
            auto k = k_render_bwd_views<TW, TH, BG, false>;
            const int blocks = resident_blocks(k, TW * TH, vb->blocks, total);
            k<<<blocks, TW * TH, 0, s>>>(vt, total, proj_all_dev, n, values_dev, ranges_dev, t_final_all_dev,
                                         n_contrib_all_dev, tr, dl_all_dev, grad2d_all_dev, tile_order_dev,
                                         queue_dev);
        }
    });
    PGS_CHECK_LAUNCH("pgs_render_bwd_views");
    return PGS_OK;
}
