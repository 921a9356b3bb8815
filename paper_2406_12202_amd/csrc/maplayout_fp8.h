// Packed map-weight layout for the FP8 map path of the 8x256 map.
//
// Products of hidden activations with hidden weights run on
// v_mfma_scale_f32_32x32x64_f8f6f4 with OCP E4M3 operands; products with the
// encodings gamma(x) (input layer, skip layer) and gamma(d) (direction layer)
// stay on v_mfma_f32_32x32x16_bf16.  Both accumulate in the same float32
// registers: the FP8 instruction's per-operand power-of-two scales undo the
// per-layer scaling of weights (2^ew) and activations (2^ea), so the
// accumulator holds the unscaled product and biases are added unscaled.
//
// FP8 operand of k-block kb8 (64 inputs) in lane (n, h): 32 bytes.  A
// finished 32-row output tile mt leaves, in lane (n, h), rows
// 8 (v / 4) + 4 h + v % 4 (v = 0..15) of its tile; quantised in that order,
// tile 2 kb8 fills bytes 0..15 and tile 2 kb8 + 1 bytes 16..31 of k-block kb8
// of the next layer's input, so byte j of half h carries feature
// 64 kb8 + 32 (j / 16) + 8 ((j % 16) / 4) + 4 h + j % 4.  The weight operand
// of lane (m, h) holds the same features of row m (the instruction pairs
// byte j of half h of both operands).
//
// Weights are stored per (layer, 32-row output tile) as chunks of 1 KB units
// in execution order: an FP8 k-block is two units (lane bytes 0..15, 16..31),
// then the BF16 encoding k-blocks follow as one unit each (layout of
// maplayout_bf16.h).  Biases use the BF16 layout.  The density and colour
// heads stay float32 in natural row order and act on the float32 accumulators.
#pragma once

#include "maplayout_bf16.h"

namespace fl {

template <class SB>
struct ShapeF8 {
  using BS = SB;
  static constexpr int W = SB::W, D = SB::D, SKIP = SB::SKIP, DW = SB::DW, LX = SB::LX, LD = SB::LD;
  static constexpr int K8 = W / 64;                // FP8 k-blocks of a hidden input
  static constexpr int KBX = SB::KBX, KBD = SB::KBD, MT = SB::MT, MTD = SB::MTD;
  static constexpr int NL = SB::NL;                // execution order: 0..D-1 trunk, D feature, D+1 dir
  static_assert(W % 64 == 0 && DW > 0, "FP8 layout needs width % 64 == 0 and a direction layer");

  static constexpr int fp8_units(int l) { return l == 0 ? 0 : 2 * K8; }
  static constexpr int enc_units(int l) { return l == 0 ? KBX : (l == SKIP ? KBX : (l == D + 1 ? KBD : 0)); }
  static constexpr int layer_units(int l) { return fp8_units(l) + enc_units(l); }
  static constexpr int layer_mt(int l) { return SB::layer_mt(l); }
  static constexpr long unit_base(int l) {
    long o = 0;
    for (int i = 0; i < l; ++i) o += (long)layer_mt(i) * layer_units(i);
    return o;
  }
  static constexpr long UNITS = unit_base(NL);
  static constexpr int max_units() {
    int m = 0;
    for (int l = 0; l < NL; ++l) m = layer_units(l) > m ? layer_units(l) : m;
    return m;
  }
  static constexpr int MAX_U = max_units();
  static constexpr long BIASES = SB::BIASES;
  static constexpr long SIG_OFF = 0;               // W floats + bias (padded to 4)
  static constexpr long RGB_OFF = W + 4;           // 3 x DW floats + 3 biases
  static constexpr long HEADS = RGB_OFF + 3L * DW + 4;
  static constexpr int N_SCALED = D + 1;           // FP8 layers 1..D+1
};

using NerfMapF8 = ShapeF8<NerfMapB>;

inline int chain_feature_f8(int kb8, int h, int j) {
  return 64 * kb8 + 32 * (j / 16) + 8 * ((j % 16) / 4) + 4 * h + j % 4;
}

}  // namespace fl
