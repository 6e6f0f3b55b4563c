// Lattice tables for the device code (compile-time constants, folded after loop unrolling).
//
// D3Q19 velocities are the columns of the paper's matrix M (Sec. II.A) with the rest vector
// last; weights from eq. (d3q19_weight_function). The D3Q7 species lattice uses the six face
// directions in the same order as D3Q19 directions 0..5, then rest.
#pragma once

#include <cstdint>

namespace lbm {

struct D3Q19 {
  static constexpr int Q = 19;
  static constexpr int cx[19] = {1, -1, 0, 0, 0, 0, 1, 1, 1, 1, -1, -1, -1, -1, 0, 0, 0, 0, 0};
  static constexpr int cy[19] = {0, 0, 1, -1, 0, 0, 1, -1, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0};
  static constexpr int cz[19] = {0, 0, 0, 0, 1, -1, 0, 0, 1, -1, 0, 0, 1, -1, 1, -1, 1, -1, 0};
  static constexpr int opp[19] = {1, 0, 3, 2, 5, 4, 11, 10, 13, 12, 7, 6, 9, 8, 17, 16, 15, 14, 18};
  // Nine directions whose opposites complete the moving set (pair-difference stencils).
  static constexpr int half[9] = {0, 2, 4, 6, 7, 8, 9, 14, 15};
  static constexpr int c2(int i) { return cx[i] * cx[i] + cy[i] * cy[i] + cz[i] * cz[i]; }
  static constexpr double w(int i) { return c2(i) == 0 ? 1.0 / 3.0 : (c2(i) == 1 ? 1.0 / 18.0 : 1.0 / 36.0); }
  // w_i / |c_i| (recolouring weight), zero for the rest vector.
  static constexpr double w_over_len(int i) {
    return c2(i) == 0 ? 0.0 : (c2(i) == 1 ? 1.0 / 18.0 : 1.0 / (36.0 * 1.4142135623730950488));
  }
};

struct D3Q7 {
  static constexpr int Q = 7;
  static constexpr int opp[7] = {1, 0, 3, 2, 5, 4, 6};
  static constexpr double w(int i) { return i == 6 ? 0.25 : 0.125; }
};

// Bits of the per-node info word.
enum : uint32_t {
  kLinkMask = (1u << 18) - 1,  // fluid: bit i set if x - c_i is solid; solid: bit i set if x + c_i is fluid
  kFluid = 1u << 18,
  kWet = 1u << 19,             // fluid node with at least one solid neighbour (wetting applies)
  kRnnShift = 20,              // bits 20..22: r(x) * NN(x)
  kRnnMask = 7u << 20,
  kExtrap = 1u << 23,          // solid node whose colour is extrapolated (has a fluid neighbour)
  kInlet = 1u << 24,           // species inlet plane x = 0
  kOutlet = 1u << 25,          // species outflow plane x = nx - 1
};

}  // namespace lbm
