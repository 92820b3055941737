// Eigenbound network 12 -> 64 -> 64 -> 2 (ReLU): dense kernels on the matrix cores.
#pragma once

#include "common.hpp"

namespace blk {

constexpr int kMlpIn = 12, kMlpHid = 64, kMlpOut = 2;
// flat parameter layout: W1 [12][64], b1 [64], W2 [64][64], b2 [64], W3 [64][2], b3 [2]
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kMlpIn * kMlpHid;
constexpr int kOffW2 = kOffB1 + kMlpHid;
constexpr int kOffB2 = kOffW2 + kMlpHid * kMlpHid;
constexpr int kOffW3 = kOffB2 + kMlpHid;
constexpr int kOffB3 = kOffW3 + kMlpHid * kMlpOut;
constexpr int kMlpParams = kOffB3 + kMlpOut;  // 5122
// a deployable model: parameters, then feature mean[12], std[12], target mean[2], std[2]
constexpr int kMlpModel = kMlpParams + 2 * kMlpIn + 2 * kMlpOut;

// H1 = relu(X W1 + b1), H2 = relu(H1 W2 + b2), Y = H2 W3 + b3 for X [n][12]
void mlp_forward_dev(const float* theta, const float* x, int n, float* h1, float* h2, float* y, hipStream_t s);

}  // namespace blk
