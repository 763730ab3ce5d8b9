// Shape and packed layout of the learned branching policy's parameters.
#pragma once

namespace mcs {

constexpr int kPolicyF = 16;   // features per candidate vertex
constexpr int kPolicyH = 64;   // width of both hidden layers
constexpr int kOffW1 = 0;                                // W1[64][16]
constexpr int kOffB1 = kOffW1 + kPolicyH * kPolicyF;     // b1[64]
constexpr int kOffW2 = kOffB1 + kPolicyH;                // W2[64][64]
constexpr int kOffB2 = kOffW2 + kPolicyH * kPolicyH;     // b2[64]
constexpr int kOffW3 = kOffB2 + kPolicyH;                // w3[64]
constexpr int kOffB3 = kOffW3 + kPolicyH;                // b3
constexpr int kPolicyParams = kOffB3 + 1;                // 5313

}  // namespace mcs
