// Runtime tuning knobs of the library (rad_tuning_get / rad_tuning_set).
#include <hip/hip_runtime.h>

#include "gemm.h"

namespace rad {
namespace {
GemmTuning g_gemm{{0, 0}, 0};
int g_lookahead = 1;
}
GemmTuning& gemm_tuning() { return g_gemm; }
bool lookahead_enabled() { return g_lookahead != 0; }
}  // namespace rad

extern "C" int32_t rad_tuning_get(rad_tuning* out) {
  rad::clear_error();
  if (!out) {
    rad::set_error("rad_tuning_get: NULL output");
    return RAD_EINVAL;
  }
  *out = rad_tuning{};
  out->small_tile_below_f64 = rad::g_gemm.small_tile_below[0];
  out->small_tile_below_f32 = rad::g_gemm.small_tile_below[1];
  out->lookahead = rad::g_lookahead;
  out->side_chunk_tiles = rad::g_gemm.side_chunk_tiles;
  return RAD_OK;
}

extern "C" int32_t rad_tuning_set(const rad_tuning* in) {
  rad::clear_error();
  if (!in || in->small_tile_below_f64 < 0 || in->small_tile_below_f32 < 0 || in->lookahead < 0 ||
      in->lookahead > 1 || in->side_chunk_tiles < 0) {
    rad::set_error("rad_tuning_set: NULL or out-of-range field");
    return RAD_EINVAL;
  }
  rad::g_gemm.small_tile_below[0] = in->small_tile_below_f64;
  rad::g_gemm.small_tile_below[1] = in->small_tile_below_f32;
  rad::g_lookahead = in->lookahead;
  rad::g_gemm.side_chunk_tiles = in->side_chunk_tiles;
  return RAD_OK;
}
