// Kernel arguments of the learned denoiser, shared by its kernels and the host code.
#pragma once

#include "vdamp_internal.h"

namespace vdamp {
namespace cnn {

typedef unsigned short u16;  // BF16 bits

enum ConvMode : int {
  CV_RELU = 0,      // z = acc + bias (+ per-slice bias); out = relu(z)
  CV_MASK = 1,      // out = acc * (mask > 0)             (tangent, input gradient)
  CV_LAST = 2,      // img_out = resid - s0 * (acc + bias) (channels 0, 1)
  CV_LAST_TAN = 3   // img_out = resid - acc
};

struct ConvArgs {
  const SliceDev* slices;
  const int2* tiles;    // (slice, tile) with tile = ty * (nx / 16) + tx
  int ntiles;
  const u16* in;        // [pixel][CIN]
  const u16* w;         // [MT * 16][KSTEPS * 32]
  const float* bias;    // [Cout] or null (none)
  const float* sbias;   // [B][48] per-slice bias (layer 1) or null
  const u16* mask;      // [pixel][48] or null
  u16* out;             // [pixel][48]
  // ReLU pattern, [pixel] of 4 16-bit words: bit 4 g + i of word t is channel
  // 16 t + 4 g + i (word 3 unused).  CV_RELU writes it when bits_out is set; CV_MASK
  // reads it instead of mask when bits is set.
  uint2* bits_out;
  const uint2* bits;
  const float2* resid;  // complex image (last layer)
  const float* s0;      // [B]
  float2* img_out;      // complex image (last layer)
};

// First-stage groups of the weight-gradient reduction (the workspace holds their sums).
constexpr int kWgradReduceGroups = 16;

struct WgradArgs {
  const SliceDev* slices;
  const int2* tiles;
  int ntiles;
  const u16* dz;       // [pixel][DZC]
  int dzc;             // channel stride of dz (48 or 8)
  int cout;            // valid gradient channels (48 or 2)
  const u16* h;        // [pixel][CIN]
  float* part;         // [gridDim.x][MT * 16][NT * 16]
  float* part_bias;    // [gridDim.x][MT * 16]
  float* tile_sums;    // [ntiles][48] or null
};

}  // namespace cnn
}  // namespace vdamp
