// BF16 MFMA building blocks of the learned SGS closure (12-64-64-64-2 SiLU
// network): fragment conversion and the 16x16x16 bf16 matrix instruction.
//
// v_mfma_f32_16x16x16_bf16 operand layout (wave64, lane l):
//   A (16 x 16, rows x k): lane holds A[l % 16][4 (l / 16) + q], q = 0..3
//   B (16 x 16, k x cols): lane holds B[4 (l / 16) + q][l % 16]
//   D (16 x 16):           lane holds D[4 (l / 16) + q][l % 16]
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace cm {

constexpr int MLP_NI = 12, MLP_NH = 64, MLP_NO = 2;
constexpr int MLP_NPARAM = MLP_NH * MLP_NI + MLP_NH + 2 * (MLP_NH * MLP_NH + MLP_NH) + MLP_NO * MLP_NH + MLP_NO;
// offsets of the layer blocks in the parameter vector: W [out][in] then bias
constexpr int OFF_W1 = 0;
constexpr int OFF_B1 = OFF_W1 + MLP_NH * MLP_NI;
constexpr int OFF_W2 = OFF_B1 + MLP_NH;
constexpr int OFF_B2 = OFF_W2 + MLP_NH * MLP_NH;
constexpr int OFF_W3 = OFF_B2 + MLP_NH;
constexpr int OFF_B3 = OFF_W3 + MLP_NH * MLP_NH;
constexpr int OFF_W4 = OFF_B3 + MLP_NH;
constexpr int OFF_B4 = OFF_W4 + MLP_NO * MLP_NH;

// packed A fragments (weight tiles) of the four layers for the fused
// inference in transposed form, counted in units of 64 lanes x 4 bf16: layer
// 1 one 16x16x16 tile per output tile; layers 2-4 one 16x16x32 tile (two
// units, 64 lanes x 8 bf16) per (output tile, 32-wide k chunk)
constexpr int FRAG_L1 = 4, FRAG_L2 = 16, FRAG_L3 = 16, FRAG_L4 = 4;
constexpr int FRAG_TOTAL = FRAG_L1 + FRAG_L2 + FRAG_L3 + FRAG_L4;

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// float -> bfloat16 bits, round to nearest even (NaN/Inf kept)
__host__ __device__ inline uint16_t f2bf(float f)
{
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__host__ __device__ inline float bf2f(uint16_t b) { return __builtin_bit_cast(float, (uint32_t)b << 16); }

__device__ inline f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// v_mfma_f32_16x16x32_bf16: A and B hold 8 bf16 per lane, lane l covering
// rows (A) / columns (B) l % 16 and one eighth of k selected by l / 16, with
// the same lane-and-slot to k correspondence in A and B; D as above.  A k
// chunk may therefore be ordered freely, provided that A and B agree: the
// fused forward feeds B as two 16x16x16 D tiles side by side (slot s < 4:
// unit 4 (l / 16) + s, slot s >= 4: unit 16 + 4 (l / 16) + s - 4 of the
// chunk) and packs the weights in the same order.
typedef short bf16x8s __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8v __attribute__((ext_vector_type(8)));

__device__ inline f32x4 mfma32(bf16x8s a, bf16x4 b_lo, bf16x4 b_hi, f32x4 c)
{
    const bf16x8s b = __builtin_shufflevector(b_lo, b_hi, 0, 1, 2, 3, 4, 5, 6, 7);
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8v, a), __builtin_bit_cast(bf16x8v, b), c,
                                                   0, 0, 0);
}

// k index within a 32-wide chunk of lane group g (= lane / 16), slot s
__host__ __device__ constexpr int k32_unit(int g, int s) { return s < 4 ? 4 * g + s : 16 + 4 * g + (s - 4); }

__device__ inline float silu_f(float z) { return z / (1.0f + expf(-z)); }
__device__ inline float dsilu_f(float z)
{
    const float s = 1.0f / (1.0f + expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

}  // namespace cm
