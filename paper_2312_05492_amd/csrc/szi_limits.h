// szi_limits.h -- limits shared by the kernels, the host code and the blob
// layout.  No HIP here: the blob code builds without it.
#pragma once

namespace szi {

constexpr int kMaxLevels = 9;      // 1D: strides 256 .. 1
constexpr int kLmax = 24;          // Huffman length limit
constexpr int kMaxRadius = 1024;   // LDS histogram holds 2R <= 2048 bins
// other windows than the defaults: at most this many block points (window
// plus far faces, one wave's LDS), at most kGenMaxExtent along a dimension
constexpr int kGenMaxBlock = 4096;
constexpr int kGenMaxExtent = 1024;

}  // namespace szi
