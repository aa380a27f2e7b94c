// Float32 collision and push streaming with a given force: the steps a
// closure network drives (collide_f32.hip).
#pragma once

#include "mlb_internal.h"

namespace mlb {

// f[parity ^ 1] = streamed post-collision populations of f[parity] with the
// force S.Nf, every system and species of the per-site block map
void launch_collide_f32(const SysDesc<float> *sys, const int2 *map, int nblk, int maxM, int parity, hipStream_t st);

}  // namespace mlb
