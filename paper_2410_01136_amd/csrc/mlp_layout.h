// Byte layout of the packed coordinate-MLP (device buffer and its LDS copy).
#pragma once

namespace sm {

constexpr int kMlpFourier = 16;
constexpr int kMlpOffFourier = 0;                       // float [16][3] (turns per unit x^)
constexpr int kMlpOffW0 = 256;                          // fp16 [rb 4][t 2][lane 64][8]
constexpr int kMlpW0Bytes = 4 * 2 * 64 * 8 * 2;         // 8 KiB
constexpr int kMlpOffW1 = kMlpOffW0 + kMlpW0Bytes;      // fp16 [layer 3][rb 4][t 8][lane 64][8]
constexpr int kMlpHiddenBytes = 4 * 8 * 64 * 8 * 2;     // 32 KiB per layer
constexpr int kMlpOffWout = kMlpOffW1 + 3 * kMlpHiddenBytes;  // fp16 [t 8][lane 64][8]
constexpr int kMlpWoutBytes = 8 * 64 * 8 * 2;           // 8 KiB
constexpr int kMlpOffBias = kMlpOffWout + kMlpWoutBytes;  // float [layer 4][rb 4][h 2][r 16]
constexpr int kMlpBiasPerLayer = 4 * 2 * 16;
constexpr int kMlpOffBout = kMlpOffBias + 4 * kMlpBiasPerLayer * 4;  // float [5] (+pad)
constexpr int kMlpBytes = kMlpOffBout + 64;

static_assert(kMlpBytes % 16 == 0, "packed MLP must be a whole number of 16-byte words");
static_assert(kMlpBytes <= 160 * 1024, "packed MLP must fit in LDS");

}  // namespace sm
