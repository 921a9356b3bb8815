// bf16 operand tiles of v_mfma_f32_32x32x16_bf16 for the training kernels
// (proposal and map): a 32 x 32 output tile holds, in lane (n, h) = lane
// n + 32 h and register v, row 8 (v / 4) + 4 h + v % 4 of column n.
// Registers 0..7 and 8..15, rounded to bf16, are the next product's operands
// of its k-blocks 2 mt and 2 mt + 1 ("chained" order: k-block kb carries in
// half h and slot q the row chain_row(kb, h, q)).  Products that contract
// over the columns (weight gradients) read their operands from per-wave LDS
// tables laid out [row][column] in bf16, kTabRow entries per row.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fl {

typedef float pf32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 pbf16x8 __attribute__((ext_vector_type(8)));
typedef float pf32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 pbf16x2 __attribute__((ext_vector_type(2)));

// LDS table row stride in bf16 entries: 32 columns and 8 of padding, which
// keeps 16-byte reads aligned and spreads rows over the banks
constexpr int kTabRow = 40;

// row of register v in lane half h of an output tile
__device__ __forceinline__ int tile_row(int v, int h) { return 8 * (v >> 2) + 4 * h + (v & 3); }

__device__ __forceinline__ int chain_row(int kb, int h, int q) { return 16 * kb + 8 * (q >> 2) + 4 * h + (q & 3); }

__device__ __forceinline__ uint32_t pack2_bf16(float a, float b) {
  const pf32x2 f = {a, b};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(f, pbf16x2));
}

// rounded bf16 operands of k-blocks 2 mt and 2 mt + 1 from an output tile
__device__ __forceinline__ void tile_operands_bf16(const pf32x16& t, pbf16x8& k0, pbf16x8& k1) {
  uint4 u0, u1;
  u0.x = pack2_bf16(t[0], t[1]); u0.y = pack2_bf16(t[2], t[3]);
  u0.z = pack2_bf16(t[4], t[5]); u0.w = pack2_bf16(t[6], t[7]);
  u1.x = pack2_bf16(t[8], t[9]); u1.y = pack2_bf16(t[10], t[11]);
  u1.z = pack2_bf16(t[12], t[13]); u1.w = pack2_bf16(t[14], t[15]);
  k0 = __builtin_bit_cast(pbf16x8, u0);
  k1 = __builtin_bit_cast(pbf16x8, u1);
}

// a 32-row output tile (rows row0 + tile_row(v, h) of column n) into a
// [row][column] table as bf16, the same rounding as tile_operands_bf16
__device__ __forceinline__ void tile_to_table(const pf32x16& t, __bf16* tab, const int row0, const int n,
                                              const int h) {
#pragma unroll
  for (int v = 0; v < 16; ++v) tab[(row0 + tile_row(v, h)) * kTabRow + n] = (__bf16)t[v];
}

// operand slots of k-block kb (columns 16 kb + 8 h .. + 7) of table row `row`
__device__ __forceinline__ pbf16x8 table_operand(const __bf16* tab, const int row, const int kb, const int h) {
  return __builtin_bit_cast(pbf16x8, *reinterpret_cast<const uint4*>(tab + row * kTabRow + 16 * kb + 8 * h));
}

}  // namespace fl
