// Gaussian kernel entries on the matrix cores: operand layouts and
// per-precision traits shared by the product tiles and the KRILL sketch.
// ||x - y||^2 = ||x||^2 + ||y||^2 - 2 x.y over centred points, with the
// contraction on v_mfma_f64_16x16x4f64 (FP64) or v_mfma_f32_16x16x4f32
// (FP32); exp on the VALU.
#pragma once
#include <hip/hip_runtime.h>
#include "exp64.h"

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
