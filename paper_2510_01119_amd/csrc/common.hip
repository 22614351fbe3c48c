// Library-wide plumbing: error reporting, view validation, fills, version.
#include "common.hpp"

#include <cstring>

namespace gs4d {

namespace {
thread_local char g_last_error[512] = "";
}

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
    va_end(ap);
}

int make_view_pack(const gs4d_view *views, int32_t n_views, ViewPack *pack) {
    GS4D_REQUIRE(views != nullptr, "views is NULL");
    GS4D_REQUIRE(n_views >= 1 && n_views <= GS4D_MAX_VIEWS, "n_views must be in [1, %d], got %d",
                 GS4D_MAX_VIEWS, n_views);
    std::memset(pack, 0, sizeof(*pack));
    const int32_t W = views[0].width, H = views[0].height;
    GS4D_REQUIRE(W > 0 && H > 0, "view size must be positive (%d x %d)", W, H);
    GS4D_REQUIRE((int64_t)W * H <= ((int64_t)1 << 28), "view too large");
    for (int32_t i = 0; i < n_views; ++i) {
        const gs4d_view &v = views[i];
        GS4D_REQUIRE(v.width == W && v.height == H, "all views of a call must share width and height");
        GS4D_REQUIRE(v.fx > 0.0f && v.fy > 0.0f, "focal lengths must be positive");
        GS4D_REQUIRE(v.near_z > 0.0f, "near_z must be positive");
        pack->v[i] = v;
    }
    pack->n_views = n_views;
    pack->width = W;
    pack->height = H;
    pack->tiles_x = (W + GS4D_TILE - 1) / GS4D_TILE;
    pack->tiles_y = (H + GS4D_TILE - 1) / GS4D_TILE;
    pack->tiles_per_view = pack->tiles_x * pack->tiles_y;
    return GS4D_OK;
}

}  // namespace gs4d

using namespace gs4d;

extern "C" const char *gs4d_last_error(void) { return g_last_error; }

extern "C" const char *gs4d_status_string(int status) {
    switch (status) {
        case GS4D_OK: return "ok";
        case GS4D_ERR_INVALID_ARG: return "invalid argument";
        case GS4D_ERR_CAPACITY: return "capacity exceeded";
        case GS4D_ERR_HIP: return "HIP runtime error";
        case GS4D_ERR_UNSUPPORTED: return "unsupported";
        default: return "unknown status";
    }
}

extern "C" int gs4d_version(void) { return 1; }

extern "C" int gs4d_fill_f32(float *dst, float value, int64_t count, void *stream) {
    GS4D_REQUIRE(count >= 0 && (count == 0 || dst), "gs4d_fill_f32: bad arguments");
    return launch_fill<float>(dst, value, count, as_stream(stream));
}

extern "C" int gs4d_fill_u32(uint32_t *dst, uint32_t value, int64_t count, void *stream) {
    GS4D_REQUIRE(count >= 0 && (count == 0 || dst), "gs4d_fill_u32: bad arguments");
    return launch_fill<uint32_t>(dst, value, count, as_stream(stream));
}
