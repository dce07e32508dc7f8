// Anti-aliased render (aa.cpp).
#pragma once

#include <vector>

#include "scene.h"

namespace dc {

// Does the closed segment a + t (b - a), t in [0, 1], meet the closed box
// [xa, xb] x [ya, yb]?
bool segment_meets_box(double ax, double ay, double bx, double by, double xa, double xb,
                       double ya, double yb);

// mask[r * W + k] = 1 when the closed square of pixel (r, k) meets a chord
// segment of the scene (closed segment), else 0.
void aa_edge_pixels(const Geometry& G, const dc_viewport& vp, std::vector<unsigned char>& mask);

// dc_render_aa (synchronous).
void render_aa(dc_scene_s& s, const dc_viewport& vp, const dc_eval_opts& o, int aa,
               int out_dtype, void* out, dc_aa_report* rep, hipStream_t st);

}  // namespace dc
