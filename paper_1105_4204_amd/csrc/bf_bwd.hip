// Adjoint kernel of the trigonometric bilateral filter (placeholder until the
// fused backward lands).
#include "bf_internal.h"

namespace bf {

bf_status plan_bwd_tiles(int64_t, int64_t, const SpatialParams&, int, int, TileGeom*) {
    set_error("backward not implemented yet");
    return BF_EUNSUPPORTED;
}

bf_status launch_bwd(const float*, const float*, const float*, const float*, float*, int64_t,
                     int64_t, const RangeParams&, const SpatialParams&, const TileGeom&,
                     hipStream_t) {
    set_error("backward not implemented yet");
    return BF_EUNSUPPORTED;
}

}  // namespace bf
