// FP64 exp for the kernel tiles: table-driven argument reduction after
// P. T. P. Tang, "Table-driven implementation of the exponential function in
// IEEE floating-point arithmetic", ACM TOMS 15(2), 1989.
//
// x = (64 m + j) ln2/64 + r with |r| <= ln2/128, so exp(x) = 2^m 2^(j/64) e^r.
// ln2/64 is split in two doubles (the FMA form of the reduction keeps r to a
// few ulps of r); e^r - 1 is its degree-5 Taylor polynomial, whose truncation
// error on |r| <= ln2/128 is below 3.6e-17.  2^(j/64) comes from a 64-entry
// table the calling kernel keeps in LDS (exp64_table_fill).  The result is
// within about one ulp; x below -745.2 (and -inf) gives 0, NaN gives NaN.
#pragma once
#include <hip/hip_runtime.h>

namespace krr {

constexpr int kExpTable = 64;

// Threads 0..63 of the block fill the table; the caller synchronises.
__device__ __forceinline__ void exp64_table_fill(double* tab) {
  if (threadIdx.x < kExpTable) tab[threadIdx.x] = exp2((double)threadIdx.x / kExpTable);
}

__device__ __forceinline__ double exp64(double x, const double* __restrict__ tab) {
  constexpr double kInvL = 92.33248261689366;                  // 64 / ln 2
  constexpr double kL1 = 0x1.62e42fefa39efp-7;                 // ln2/64, leading part
  constexpr double kL2 = 0x1.abc9e3b39803fp-62;                // ln2/64 - kL1
  // below -1e4 the result is 0; the clamp keeps the reduction exact for
  // arbitrarily negative (and -inf) arguments, and passes NaN through
  x = x < -1.0e4 ? -1.0e4 : x;
  const double n = __builtin_rint(x * kInvL);
  double r = __builtin_fma(-n, kL1, x);
  r = __builtin_fma(-n, kL2, r);
  const int k = (int)n;
  const double t = tab[k & (kExpTable - 1)];
  double p = __builtin_fma(r, 1.0 / 120.0, 1.0 / 24.0);
  p = __builtin_fma(r, p, 1.0 / 6.0);
  p = __builtin_fma(r, p, 0.5);
  p = __builtin_fma(r * r, p, r);  // e^r - 1
  return ldexp(__builtin_fma(t, p, t), k >> 6);
}

// The exponential for an argument given in units of ln2/1024 (the kernel
// tiles' form): exp64_u(a * 1024/ln2) = exp(a).  Callers fold the factor
// 1024/ln2 into the multiply-add that forms the exponent, so the reduction
// is n = rint(u), v = u - n (exact, |v| <= 1/2); 2^(j/1024) comes from a
// 1024-entry table in LDS (exp64u_table_fill) and e^r - 1, r = v ln2/1024,
// from a degree-3 polynomial in v whose coefficients carry the powers of
// ln2/1024 (truncation below 5.5e-16 on |r| <= ln2/2048, about 2.5 ulp: the
// tiles allow 1e-13 of sum |K||V|).  Forming u rounds it to about 3 eps |a|
// more than the exponent itself carries.  Precondition: |u| < 2^30 or u = NaN
// (no clamp: callers whose exponents are bounded use this form); larger
// magnitudes saturate the conversion and are not supported.
constexpr int kExpTableU = 1024;
constexpr double kExpUScale = 1477.3197218702985;  // 1024 / ln2

// The block's threads fill the table; the caller synchronises.
__device__ __forceinline__ void exp64u_table_fill(double* tab) {
  for (int j = threadIdx.x; j < kExpTableU; j += blockDim.x)
    tab[j] = exp2((double)j / kExpTableU);
}

__device__ __forceinline__ double exp64_u(double u, const double* __restrict__ tab) {
  constexpr double kC1 = 0x1.62e42fefa39efp-11;  // (ln2/1024)
  constexpr double kC2 = 0x1.ebfbdff82c58fp-23;  // (ln2/1024)^2 / 2
  constexpr double kC3 = 0x1.c6b08d704a0cp-35;   // (ln2/1024)^3 / 6
  const double n = __builtin_rint(u);
  const double v = u - n;
  const int k = (int)n;
  const double t = tab[k & (kExpTableU - 1)];
  double p = __builtin_fma(v, kC3, kC2);
  p = __builtin_fma(v, p, kC1);
  return ldexp(__builtin_fma(t, p * v, t), k >> 10);
}

}  // namespace krr
