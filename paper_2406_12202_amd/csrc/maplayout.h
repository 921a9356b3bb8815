// Packed map-weight layout for the register-chained MFMA MLP (host packer and
// device kernels both read it).
//
// The MLP runs as D^T = W X^T on v_mfma_f32_16x16x4_f32: weights are the A
// operand (16 output rows x 4 input features per instruction), activations of
// 16 samples the B operand.  Lane l of a wave owns sample n = l % 16 and lane
// group g = l / 16; in a k-block (the 4 inputs of one instruction) group g
// supplies input position g.  The accumulator of output m-tile mt holds, in
// lane (n, g), rows 16 mt + 4 g + r (r = 0..3) of sample n; after bias and
// activation those 4 values are exactly the B operands of k-blocks 4 mt + r of
// the next layer, so activations never leave registers.  Weight columns are
// permuted to match: k-block kb of a chained input carries, in group g,
// feature 16 (kb / 4) + 4 g + kb % 4.
//
// Positional-encoding inputs: the encoding terms are grouped into pseudo-pairs
// p = 0 .. 3L+1 -- pair p < 3L is (sin, cos)(2^{p/3} pi x_{p%3}), pair 3L is
// (x_0, x_1), pair 3L+1 is (x_2, 0) -- and pair p goes to group p % 4 at
// k-blocks 2 (p / 4) and 2 (p / 4) + 1, so every lane evaluates whole sin/cos
// pairs.  Block counts are padded to multiples of 4 so that a lane reads the A
// operands of 4 k-blocks with one 16-byte load.
#pragma once

namespace fl {

constexpr int round4(int x) { return (x + 3) & ~3; }
constexpr int posenc_kb(int L) { return round4(2 * ((3 * L + 2 + 3) / 4)); }

template <int W_, int D_, int SKIP_, int LX_, int LD_, int DW_>
struct Shape {
  static constexpr int W = W_, D = D_, SKIP = SKIP_, LX = LX_, LD = LD_, DW = DW_;
  static constexpr int IN_X = 3 + 6 * LX, IN_D = 3 + 6 * LD;
  static constexpr int MT = W / 16;            // output m-tiles of a hidden layer
  static constexpr int KBH = W / 4;            // k-blocks of a hidden activation
  static constexpr int KBX = posenc_kb(LX);
  static constexpr int KBD = posenc_kb(LD);
  static constexpr int MTD = DW / 16;          // m-tiles of the direction layer
  static constexpr int KBG = DW > 0 ? DW / 4 : KBH + KBD;  // k-blocks into the rgb head
  static_assert(W % 16 == 0 && DW % 16 == 0, "widths must be multiples of 16");

  // float offsets of each block of the packed buffer
  static constexpr long dense_size(int mt, int kb) { return (long)mt * kb * 64 + (long)mt * 16; }
  static constexpr int layer_kb(int l) { return l == 0 ? KBX : (l == SKIP ? KBH + KBX : KBH); }
  static constexpr long layer_off(int l) {
    long o = 0;
    for (int i = 0; i < l; ++i) o += dense_size(MT, layer_kb(i));
    return o;
  }
  static constexpr long SIG_OFF = layer_off(D);
  static constexpr long SIG_SIZE = 4L * KBH + 4;
  static constexpr long FEAT_OFF = SIG_OFF + SIG_SIZE;
  static constexpr long DIR_OFF = FEAT_OFF + (DW > 0 ? dense_size(MT, KBH) : 0);
  static constexpr long RGB_OFF = DIR_OFF + (DW > 0 ? dense_size(MTD, KBH + KBD) : 0);
  static constexpr long RGB_SIZE = 12L * KBG + 4;
  static constexpr long TOTAL = RGB_OFF + RGB_SIZE;

  // multiply-accumulates per sample of the unpadded network
  static constexpr long macs() {
    long m = (long)W * IN_X;
    for (int l = 1; l < D; ++l) m += (long)W * (l == SKIP ? W + IN_X : W);
    m += W;
    if (DW > 0) m += (long)W * W + (long)DW * (W + IN_D) + 3L * DW;
    else m += 3L * (W + IN_D);
    return m;
  }
};

// the map shapes compiled into the library
using SmallMap = Shape<64, 4, -1, 6, 2, 0>;
using NerfMap = Shape<256, 8, 5, 10, 4, 128>;

// feature index (within its segment) of a chained k-block in group g
inline int chain_feature(int kb, int g) { return 16 * (kb / 4) + 4 * g + (kb % 4); }

// encoding term index of k-block kb in group g, -1 for padding
inline int posenc_feature(int L, int kb, int g) {
  const int p = 4 * (kb / 2) + g, e = kb % 2;
  if (p < 3 * L) return 3 + 6 * (p / 3) + 3 * e + p % 3;
  if (p == 3 * L) return e;             // x_0 | x_1
  if (p == 3 * L + 1) return e ? -1 : 2; // x_2 | pad
  return -1;
}

}  // namespace fl
