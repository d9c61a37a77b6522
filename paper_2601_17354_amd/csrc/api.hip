// Version and error reporting of the C ABI.
#include <stdarg.h>
#include <stdio.h>

#include "common.hpp"

namespace pgs {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

pgs_status check_views(const pgs_view_batch* vb, const char* who) {
    PGS_REQUIRE(vb != nullptr && vb->cams != nullptr, "%s: null view batch", who);
    PGS_REQUIRE(vb->n_views >= 1 && vb->n_views <= PGS_MAX_VIEWS, "%s: n_views %d not in 1..%d", who,
                vb->n_views, PGS_MAX_VIEWS);
    PGS_REQUIRE(vb->tile_w > 0 && vb->tile_h > 0, "%s: bad tile %dx%d", who, vb->tile_w, vb->tile_h);
    long long tiles = 0;
    for (int v = 0; v < vb->n_views; ++v) {
        const int W = vb->cams[v].width, H = vb->cams[v].height;
        PGS_REQUIRE(W > 0 && H > 0 && W < 65536 * vb->tile_w && H < 65536 * vb->tile_h,
                    "%s: view %d size %dx%d", who, v, W, H);
        tiles += (long long)((W + vb->tile_w - 1) / vb->tile_w) * ((H + vb->tile_h - 1) / vb->tile_h);
    }
    PGS_REQUIRE(tiles < (1ll << 31), "%s: %lld tiles", who, tiles);
    return PGS_OK;
}

}  // namespace pgs

extern "C" const char* pgs_version(void) { return "pocketgs-gfx950 0.1"; }

extern "C" const char* pgs_last_error(void) { return pgs::g_err; }
