// Host launcher of the look-ahead frame-set kernel (k_estimate.hip), used by
// rt_frameset_ahead.
#pragma once

#include "rt_internal.h"

namespace rc {

// One launch of the look-ahead frame-set loop: the apply of frame-set t
// (fa, ba; NULL fa: none) and the band statistics, estimate and tables of
// frame-set t + 1 with the clearing of its whole-frame statistics (fe, be;
// NULL fe: none).
hipError_t launch_frameset_ahead(const Geo& g, const FramePtrs* fa, const Bufs& ba, const FramePtrs* fe,
                                 const Bufs& be, hipStream_t st);

}  // namespace rc
