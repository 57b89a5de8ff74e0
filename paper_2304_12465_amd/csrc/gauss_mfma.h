// Gaussian kernel entries on the matrix cores: operand layouts and
// per-precision traits shared by the product tiles and the KRILL sketch.
// ||x - y||^2 = ||x||^2 + ||y||^2 - 2 x.y over centred points, with the
// contraction on v_mfma_f64_16x16x4f64 (FP64) or v_mfma_f32_16x16x4f32
// (FP32); exp on the VALU.
#pragma once
#include <hip/hip_runtime.h>
#include "exp64.h"
#include <type_traits>

namespace krr {
namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Operand layouts (wave64, lane l, g = l / 16, li = l % 16):
//   A (16 x 4): lane l holds A[li][g];  B (4 x 16): lane l holds B[g][li]
//   D (16 x 16), element t of lane l:
//     v_mfma_f64_16x16x4f64: D[4 t + g][li]
//     v_mfma_f32_16x16x4f32: D[4 g + t][li]
// col(t, g) names that row index of D.
template <typename T>
struct GT;
template <>
struct GT<double> {
  typedef f64x4 acc_t;
  static __device__ __forceinline__ acc_t mfma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int col(int t, int g) { return 4 * t + g; }
  // exponents in units of ln2/1024 (the scale 1024/ln2 is folded into s);
  // the expansion guard bounds them far inside exp64_u's range
  static __device__ __forceinline__ double ex(double x, const double* tab) { return exp64_u(x, tab); }
  static constexpr double kFar = -1.0e7;     // exponent of columns past the range (2^-9766 -> 0)
  static constexpr int kTable = kExpTableU;  // entries of the exp table in LDS
  static __device__ __forceinline__ void fill(double* tab) { exp64u_table_fill(tab); }
  static constexpr double kExpScale = kExpUScale;
  // expansion error bound (d + 3) eps s (max||x||^2 + max||y||^2) at most
  // 400 eps = 8.9e-14, else direct differences
  static constexpr double kBound = 400.0;
};
template <>
struct GT<float> {
  typedef f32x4 acc_t;
  static __device__ __forceinline__ acc_t mfma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int col(int t, int g) { return 4 * g + t; }
  static __device__ __forceinline__ float ex(float x, const double*) {
    return __builtin_amdgcn_exp2f(x);
  }
  static constexpr float kFar = -3.0e38f;
  static constexpr double kExpScale = 1.4426950408889634;  // log2(e): v_exp_f32 is base 2
  static constexpr int kTable = 1;                          // no table
  static __device__ __forceinline__ void fill(double*) {}
  // 200 eps_32 = 1.2e-5 relative per entry at most (the FP32 tile tolerance
  // is 2e-5 of sum |K||V|), else direct differences
  static constexpr double kBound = 200.0;
};

// Three-slice bf16 contraction of FP32 points (padded dimension a multiple
// of 8 up to 32): every coordinate x is split by round-to-nearest bf16
// conversions into h + m + l (each remainder is exact in FP32; the last has
// at most 8 significant bits, so the three hold x exactly), and the six
// slice products of weight down to 2^-16 (hh, hm, mh, hl, lh, mm) run on
// v_mfma_f32_16x16x32_bf16 with FP32 accumulation.  Each product is exact
// in FP32; the dropped ones (ml, lm, ll) are below 2^-24 |x||y| together.
// K index 32 st + 8 g + e of MFMA step st is coordinate d0 + e of product p,
// for the 8-coordinate group G = 4 st + g: p = G / (D/8), d0 = 8 (G % (D/8));
// groups with p >= 6 pad the last step (zero B slices).  The A operand (the
// staged columns) and the B operand (the rows held in registers) take the
// slices s3_aslice(p) and s3_bslice(p) (h = 0, m = 1, l = 2).
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <typename T, int D>
constexpr bool s3_split() {
  return std::is_same<T, float>::value && D % 8 == 0 && D <= 32;
}
__device__ __forceinline__ int s3_aslice(int p) { return p == 2 || p == 5 ? 1 : p == 4 ? 2 : 0; }
__device__ __forceinline__ int s3_bslice(int p) { return p == 1 || p == 5 ? 1 : p == 3 ? 2 : 0; }
// MFMA steps (K = 32 each) over the 6 D slice coordinates
template <int D>
constexpr int s3_steps() {
  return (6 * D + 31) / 32;
}
// LDS row pitch (bf16) of staged split points: 3 D, plus 8 when 3 D / 8 is
// even, so the 16-byte reads of 8 consecutive rows fall in distinct banks
template <int D>
constexpr int s3_pitch() {
  return (3 * D / 8) % 2 ? 3 * D : 3 * D + 8;
}

// Two coordinates -> their h, m and l bf16 slices, each pair packed in a
// 32-bit word (low half: a).
__device__ __forceinline__ void split3_pair(float a, float b, uint32_t& h, uint32_t& m,
                                            uint32_t& l) {
  h = __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{a, b}, bf16x2));
  a -= __builtin_bit_cast(float, h << 16);
  b -= __builtin_bit_cast(float, h & 0xffff0000u);
  m = __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{a, b}, bf16x2));
  a -= __builtin_bit_cast(float, m << 16);
  b -= __builtin_bit_cast(float, m & 0xffff0000u);
  l = __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{a, b}, bf16x2));
}

// B operand of step st for lane group g from a row x of D FP32 coordinates
template <int D>
__device__ __forceinline__ bf16x8 s3_b_operand(const float* __restrict__ x, int st, int g) {
  const int G = 4 * st + g, p = G / (D / 8), d0 = 8 * (G % (D / 8));
  u32x4 w = {0u, 0u, 0u, 0u};
  if (p < 6) {
    const int bs = s3_bslice(p);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      uint32_t h, m, l;
      split3_pair(x[d0 + 2 * e], x[d0 + 2 * e + 1], h, m, l);
      w[e] = bs == 0 ? h : bs == 1 ? m : l;
    }
  }
  return __builtin_bit_cast(bf16x8, w);
}
// LDS offset (bf16) of the A operand of step st for lane group g in a row
// of split points (h | m | l, D each)
template <int D>
__device__ __forceinline__ int s3_a_offset(int st, int g) {
  const int G = 4 * st + g, p = G / (D / 8), d0 = 8 * (G % (D / 8));
  return p < 6 ? s3_aslice(p) * D + d0 : 0;
}
// Coordinates 4 q .. 4 q + 3 of a point into its LDS row of slices
template <int D>
__device__ __forceinline__ void s3_store_quad(const f32x4& v, int q, __bf16* row) {
  uint32_t h0, m0, l0, h1, m1, l1;
  split3_pair(v[0], v[1], h0, m0, l0);
  split3_pair(v[2], v[3], h1, m1, l1);
  *reinterpret_cast<uint2*>(row + 4 * q) = make_uint2(h0, h1);
  *reinterpret_cast<uint2*>(row + D + 4 * q) = make_uint2(m0, m1);
  *reinterpret_cast<uint2*>(row + 2 * D + 4 * q) = make_uint2(l0, l1);
}

__device__ __forceinline__ double fma_g(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_g(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// The expansion puts an error of up to (dpad + 3) eps s (max||x||^2 +
// max||y||^2) into the exponent; above GT<T>::kBound eps the direct
// differences are used instead.
template <typename T>
__device__ __forceinline__ bool gauss_expansion_too_coarse(double s_nat, double xmax, double ymax,
                                                           int dpad) {
  return s_nat * (xmax + ymax) * (dpad + 3) > GT<T>::kBound;
}

}  // namespace
}  // namespace krr
