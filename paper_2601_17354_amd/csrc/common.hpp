// Internal helpers shared by the gfx950 kernels of libpocketgs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pocketgs.h"

namespace pgs {

void set_error(const char* fmt, ...);

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Thresholds of the compositing loop: alpha is clamped to 0.99, splats below
// 1/255 are skipped and a pixel stops before transmittance would fall below
// 1e-4 (conventions inherited from 3D Gaussian Splatting).
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kAlphaMax = 0.99f;
constexpr float kTMin = 1e-4f;

// Camera in float64 for the per-Gaussian projection maths.
struct CamD {
    double R[9];
    double t[3];
    double fx, fy, cx, cy;
    double campos[3];  // camera centre -R^T t
    double lim_x, lim_y;
    int W, H;
};

inline CamD make_cam(const pgs_camera& c) {
    CamD d;
    for (int r = 0; r < 3; ++r) {
        for (int k = 0; k < 3; ++k) d.R[3 * r + k] = c.viewmat[4 * r + k];
        d.t[r] = c.viewmat[4 * r + 3];
    }
    d.fx = c.fx;
    d.fy = c.fy;
    d.cx = c.cx;
    d.cy = c.cy;
    for (int k = 0; k < 3; ++k)
        d.campos[k] = -(d.R[k] * d.t[0] + d.R[3 + k] * d.t[1] + d.R[6 + k] * d.t[2]);
    d.W = c.width;
    d.H = c.height;
    d.lim_x = 1.3 * (double)c.width / (2.0 * (double)c.fx);
    d.lim_y = 1.3 * (double)c.height / (2.0 * (double)c.fy);
    return d;
}

// Tile and pixel offsets of a batch of views (tiles numbered view by view,
// row-major inside a view; pixel arrays concatenated view by view).
struct ViewsLayout {
    int TX[PGS_MAX_VIEWS];
    int tile_off[PGS_MAX_VIEWS + 1];
    long long pix_off[PGS_MAX_VIEWS + 1];
};

inline ViewsLayout views_layout(const pgs_view_batch& vb) {
    ViewsLayout l{};
    for (int v = 0; v < vb.n_views; ++v) {
        const int W = vb.cams[v].width, H = vb.cams[v].height;
        l.TX[v] = (W + vb.tile_w - 1) / vb.tile_w;
        const int TY = (H + vb.tile_h - 1) / vb.tile_h;
        l.tile_off[v + 1] = l.tile_off[v] + l.TX[v] * TY;
        l.pix_off[v + 1] = l.pix_off[v] + (long long)W * H;
    }
    return l;
}

// Validates the view list of a batch (shape checks are the caller's).
pgs_status check_views(const pgs_view_batch* vb, const char* who);

}  // namespace pgs

#define PGS_REQUIRE(cond, ...)                 \
    do {                                       \
        if (!(cond)) {                         \
            pgs::set_error(__VA_ARGS__);       \
            return PGS_ERR_INVALID_ARG;        \
        }                                      \
    } while (0)

#define PGS_CHECK_LAUNCH(what)                                                       \
    do {                                                                             \
        hipError_t e_ = hipGetLastError();                                           \
        if (e_ != hipSuccess) {                                                      \
            pgs::set_error("%s: %s (%s:%d)", what, hipGetErrorString(e_), __FILE__, \
                           __LINE__);                                                \
            return PGS_ERR_HIP;                                                      \
        }                                                                            \
    } while (0)

// Wave-wide float sum on wave64 with DPP: an inclusive scan inside each row of
// 16 lanes (row_shr 1, 2, 4, 8), then row_bcast:15 and row_bcast:31 fold the
// rows together.  Lane 63 ends up holding the sum of all 64 inputs.
__device__ __forceinline__ float wave_sum_to_lane63(float v) {
    int x = __float_as_int(v);
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false));
    x = __float_as_int(v);
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false));
    x = __float_as_int(v);
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false));
    x = __float_as_int(v);
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false));
    x = __float_as_int(v);
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false));
    x = __float_as_int(v);
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false));
    return v;
}
