// Packed map-weight layout for the BF16 MFMA MLP (v_mfma_f32_32x32x16_bf16).
//
// A wave evaluates 64 samples as two 32-column tiles that share every weight
// fragment.  Lane l owns samples n = l % 32 of both tiles and half h = l / 32.
// In a k-block (the 16 inputs of one instruction) half h supplies inputs
// 8 h .. 8 h + 7 as eight bf16 values.  The accumulator of output m-tile mt
// holds, in lane (n, h), rows 8 (v / 4) + 4 h + v % 4 (v = 0..15); after bias,
// activation and rounding to bf16, values v = 0..7 form the lane's operand of
// k-block 2 mt and v = 8..15 that of k-block 2 mt + 1, so k-block kb of a
// chained input carries, in half h and slot q, feature
// 16 kb + 8 (q / 4) + 4 h + q % 4.
//
// Encoding inputs: pseudo-pair p = 0 .. 3L+1 as in the FP32 layout ((sin, cos)
// of band p / 3 and coordinate p % 3, then (x0, x1) and (x2, 0)); pair p sits
// in k-block p / 8, half (p / 4) % 2, slots 2 (p % 4) and 2 (p % 4) + 1.
//
// Weights are stored as "chunks", one per (layer, output m-tile) in execution
// order; a chunk is kb 1 KB blocks, block k holding the 64 lanes' 16-byte A
// operands of k-block k.  Biases stay float32.  The heads are MFMA tiles too,
// stored after the layers ("tail tiles") with 32 biases each after the
// layers' biases: a map without direction layer has one tile, rows 0
// (density, over the trunk output) and 1..3 (colour, over the trunk output
// and gamma(d)), KBH + KBD blocks; a map with a direction layer has a density
// tile (row 0 over the trunk output, KBH blocks) and a colour tile (rows 0..2
// over the direction layer's output, DW / 16 blocks).  A head weight w is
// stored as hi = bf16(w) in its row r and lo = bf16(w - hi) in row r + 8
// (bias 0), so a head output is the sum of two accumulator rows (values v and
// v + 4 of lane half 0) and the head weights keep 16 significant bits.
#pragma once

namespace fl {

template <int W_, int D_, int SKIP_, int LX_, int LD_, int DW_>
struct ShapeB {
  static constexpr int W = W_, D = D_, SKIP = SKIP_, LX = LX_, LD = LD_, DW = DW_;
  static constexpr int IN_X = 3 + 6 * LX, IN_D = 3 + 6 * LD;
  static constexpr int MT = W / 32;
  static constexpr int KBH = W / 16;
  static constexpr int KBX = (3 * LX + 2 + 7) / 8;
  static constexpr int KBD = (3 * LD + 2 + 7) / 8;
  static constexpr int MTD = DW / 32;
  static constexpr int KBG = DW > 0 ? DW / 16 : KBH + KBD;
  static constexpr int NL = D + (DW > 0 ? 2 : 0);   // MFMA layers in execution order
  static_assert(W % 32 == 0 && DW % 32 == 0, "widths must be multiples of 32");

  // layer l in execution order: hidden 0..D-1, then feature (D) and dir (D+1)
  static constexpr int layer_kb(int l) {
    return l == 0 ? KBX : (l < D ? (l == SKIP ? KBH + KBX : KBH) : (l == D ? KBH : KBH + KBD));
  }
  static constexpr int layer_mt(int l) { return l <= D ? MT : MTD; }
  static constexpr long block_base(int l) {       // first 1 KB block of layer l
    long o = 0;
    for (int i = 0; i < l; ++i) o += (long)layer_mt(i) * layer_kb(i);
    return o;
  }
  static constexpr long bias_base(int l) {        // first bias float of layer l
    long o = 0;
    for (int i = 0; i < l; ++i) o += 32L * layer_mt(i);
    return o;
  }
  static constexpr int SIG_KB = DW > 0 ? KBH : KBH + KBD;   // first tail tile
  static constexpr int RGB_KB = DW > 0 ? DW / 16 : 0;         // second tail tile (maps with a direction layer)
  static constexpr long SIG_BLOCK = block_base(NL);
  static constexpr long RGB_BLOCK = SIG_BLOCK + SIG_KB;
  static constexpr long SIG_BIAS = bias_base(NL);
  static constexpr long RGB_BIAS = SIG_BIAS + 32;
  static constexpr long BLOCKS = RGB_BLOCK + RGB_KB;
  static constexpr long BIASES = SIG_BIAS + (DW > 0 ? 64 : 32);
  // the single head tile of a map without direction layer
  static constexpr int HEAD_KB = DW > 0 ? 0 : SIG_KB;
  static constexpr long HEAD_BLOCK = SIG_BLOCK;
  static constexpr long HEAD_BIAS = SIG_BIAS;
  static constexpr int MAX_KB = (KBH + KBX) > (KBH + KBD) ? (KBH + KBX) : (KBH + KBD);
  static constexpr long SIG_OFF = 0;              // float offsets in the head buffer
  static constexpr long SIG_SIZE = 16L * KBH + 4;
  static constexpr long RGB_OFF = SIG_SIZE;
  static constexpr long RGB_SIZE = 48L * KBG + 4;
  static constexpr long HEADS = RGB_OFF + RGB_SIZE;
};

using SmallMapB = ShapeB<64, 4, -1, 6, 2, 0>;
using NerfMapB = ShapeB<256, 8, 5, 10, 4, 128>;

inline int chain_feature_b(int kb, int h, int q) { return 16 * kb + 8 * (q / 4) + 4 * h + (q % 4); }

inline int posenc_feature_b(int L, int kb, int h, int q) {
  const int p = 8 * kb + 4 * h + q / 2, e = q % 2;
  if (p < 3 * L) return 3 + 6 * (p / 3) + 3 * e + p % 3;
  if (p == 3 * L) return e;
  if (p == 3 * L + 1) return e ? -1 : 2;
  return -1;
}

}  // namespace fl
