// Internal (not part of the C ABI): the pieces of an fg_render workspace that
// the blend backward reads when the forward ran with save_state.
#pragma once
#include "fg.h"
#include <cstddef>
#include <cstdint>

namespace fgr {

struct RenderWsView {
    const uint32_t* nch;       // [n_tiles] chunks per tile
    const uint32_t* mfirst;    // [n_tiles] first chunk item of a tile with more than one chunk
    const uint32_t* mitem;     // [max_items] chunk item -> tile
    const uint32_t* counters;  // [2]: number of chunk items (clamped to max_items)
    const float* state;        // [max_items][4][256]: T, C0, C1, C2 per pixel after the chunk
    int chunk;                 // splats per chunk
    int64_t max_items;
};

// Carves ws as fg_render does for (cam, cap_pairs, tune); false if ws is too
// small or tune does not ask for saved state.
bool render_ws_view(const void* ws, size_t ws_bytes, const fg_camera* cam, int64_t cap_pairs, const fg_tune* tune,
                    RenderWsView* v);

}  // namespace fgr
