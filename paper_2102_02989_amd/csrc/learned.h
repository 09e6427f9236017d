// learned.h -- parameter layout of the screening network (FP32, host and device).
#pragma once

namespace rsgdf {

constexpr int kMlpF = 16;  // input features (11 used, zero padded)
constexpr int kMlpH = 64;  // hidden width
constexpr int kMlpOffMean = 0;                        // feature means [16]
constexpr int kMlpOffIstd = kMlpOffMean + kMlpF;      // 1 / feature std [16]
constexpr int kMlpOffW1 = kMlpOffIstd + kMlpF;        // [64][16]
constexpr int kMlpOffB1 = kMlpOffW1 + kMlpH * kMlpF;  // [64]
constexpr int kMlpOffW2 = kMlpOffB1 + kMlpH;          // [64][64]
constexpr int kMlpOffB2 = kMlpOffW2 + kMlpH * kMlpH;  // [64]
constexpr int kMlpOffW3 = kMlpOffB2 + kMlpH;          // [64]
constexpr int kMlpOffB3 = kMlpOffW3 + kMlpH;          // [1]
constexpr int kMlpOffLo = kMlpOffB3 + 1;              // training range, raw features [16]
constexpr int kMlpOffHi = kMlpOffLo + kMlpF;          // [16]
constexpr int kMlpNParam = kMlpOffHi + kMlpF;         // 5377
constexpr int kMlpNTrain = kMlpOffB3 + 1 - kMlpOffW1; // trainable: W1 .. b3 (5313)

}  // namespace rsgdf
