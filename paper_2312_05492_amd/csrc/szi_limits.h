// szi_limits.h -- limits shared by the kernels, the host code and the blob
// layout.  No HIP here: the blob code builds without it.
#pragma once

namespace szi {

constexpr int kMaxLevels = 9;      // 1D: strides 256 .. 1
constexpr int kLmax = 24;          // Huffman length limit
constexpr int kMaxRadius = 1024;   // LDS histogram holds 2R <= 2048 bins

}  // namespace szi
