// Choice of render options against an accuracy target (autotune.cpp).
#pragma once

#include <vector>

#include "scene.h"

namespace dc {

// Sampled pixels of a viewport for the accuracy check: a stride grid and
// pixels along the chords that cross the viewport (about `want` in all).
void tune_sample_pixels(const Geometry& G, const dc_viewport& vp, int want,
                        std::vector<int>& rows, std::vector<int>& cols);

// dc_autotune on a scene with densities; seg_w are the segment weights of
// the resident densities (for the direct-sum reference).  Synchronous.
void autotune_scene(dc_scene_s& s, const dc_viewport* vps, int n, const dc_tune_opts& t,
                    const double* seg_w, dc_tune_report& rep, hipStream_t st);

}  // namespace dc
