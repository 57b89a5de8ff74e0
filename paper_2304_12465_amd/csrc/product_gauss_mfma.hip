// Gaussian kernel tiles on the matrix cores in FP64 (precision KRR_FP64,
// v_mfma_f64_16x16x4f64) and FP32 (precision KRR_FP32, v_mfma_f32_16x16x4f32).
//
// ||x - y||^2 = ||x||^2 + ||y||^2 - 2 x.y with the contraction on the MFMA
// over centred points (centring keeps the expansion's cancellation at
// ~eps ||x||^2).  The distance MFMA starts from -||x||^2 / 2, so one FMA
// gives the exponent; exp runs on the VALU (FP64: the table-driven exp64_u
// on an exponent scaled by 1024/ln2; FP32: v_exp_f32 on an exponent scaled
// by log2 e).  FP32 points of padded dimension 8, 16 or 32 run the
// contraction as three bf16 slices per coordinate on
// v_mfma_f32_16x16x32_bf16 (gauss_mfma.h: exact slices, six slice products,
// the dropped ones below 2^-24 |x||y|), other FP32 dimensions on
// v_mfma_f32_16x16x4f32.  The reduction against V
// is a second MFMA for more than 4 right-hand sides: the distance output
// layout (lane l holds, for t = 0..3, column col(t, l/16) of row l % 16) is
// the A-operand layout of K-step t of the 16x16x4 MFMA with K index l / 16
// standing for that column, so no lane exchange is needed.  For up to 4
// right-hand sides E.V runs on the VALU and the four lanes of a row are
// added at the end.  FP64 sums throughout (FP32 partial sums fold into FP64
// every 256 columns); per-split partials go to fixed slots (bitwise
// reproducible).
#include "product.h"
#include "gauss_mfma.h"
#include <algorithm>
#include <type_traits>

namespace krr {

namespace {

constexpr int kRTg = 2;      // 16-row tiles per wave
constexpr int kColsG = 64;   // columns per LDS chunk (four 16-column tiles)
constexpr int kFoldG = 4;    // FP32: chunks per FP64 fold (256 columns)

template <typename T>
__device__ __forceinline__ bool needs_direct(const GJob<T>& J) {
  if (J.route) return J.route == 2;  // decided on the host from known norms
  return gauss_expansion_too_coarse<T>(J.s_nat, (double)*J.xmax, (double)*J.ymax, J.dpad);
}

// Per-thread staging of the next 64-column chunk (points, squared norms, V),
// loaded into registers while the current chunk is computed.  A chunk inside
// the column range reads with linear addresses; the last chunk of a range
// repeats its last column in the positions past the end, whose exponent is
// set to kFar when the norms are stored, so their kernel values are exactly
// 0.  No value is tested when it is loaded: the loads stay in flight across
// the current chunk's MFMAs.
// The product tiles take the three-slice bf16 contraction at padded
// dimension 8, 16 and 32 (at 24 its slices spill 30-160 registers at 4 waves
// per SIMD, against 0-36 for the FP32 contraction).
template <typename T, int D>
constexpr bool g_uses_split() {
  return s3_split<T, D>() && D != 24;
}

template <typename T, int D, int VS>
struct StageG {
  static constexpr bool kSplit = g_uses_split<T, D>();
  // point values per thread; split path: 4-coordinate segments instead
  static constexpr int kY = kSplit ? 1 : kColsG * D / 256;
  static constexpr int kSegs = kColsG * D / 4;
  static constexpr int kSegPT = kSplit ? (kSegs + 255) / 256 : 1;
  // V: 64 columns x VS right-hand-side slots (16 for the MFMA reduction,
  // the m used for the VALU one), at most one value per thread below 256
  static constexpr int kV = VS > 0 ? (kColsG * VS + 255) / 256 : 1;  // VS = 0: no V (store)
  T y[kY];
  f32x4 y4[kSegPT];  // split path: coordinates 4 (seg % (D/4)) .. + 3 of column seg / (D/4)
  T v[kV];
  T yn;        // threads 0..63: squared norm of their column
  bool valid;  // threads 0..63: the column is in range
};

template <typename T, int D, int VS>
__device__ __forceinline__ void stage_fetch(const GJob<T>& J, int64_t jb, int64_t j1, int tid,
                                            StageG<T, D, VS>& st) {
  constexpr int kVals = kColsG * VS;  // V values of a chunk
  typedef StageG<T, D, VS> S;
  if (jb + kColsG <= j1) {
    if constexpr (S::kSplit) {
#pragma unroll
      for (int q = 0; q < S::kSegPT; ++q) {
        const int seg = tid + q * 256;
        if (S::kSegs % 256 == 0 || seg < S::kSegs)
          st.y4[q] = *reinterpret_cast<const f32x4*>(J.yc + (jb + seg / (D / 4)) * D +
                                                      4 * (seg % (D / 4)));
      }
    } else {
#pragma unroll
      for (int q = 0; q < S::kY; ++q) st.y[q] = J.yc[jb * D + tid + q * 256];
    }
    if constexpr (VS > 0) {
#pragma unroll
      for (int q = 0; q < StageG<T, D, VS>::kV; ++q) {
        const int e = tid + q * 256;
        if (e < kVals) st.v[q] = J.v[(jb + e / VS) * 16 + e % VS];
      }
    }
    if (tid < kColsG) {
      st.yn = J.yn[jb + tid];
      st.valid = true;
    }
  } else {
    const int64_t last = j1 - 1;
    if constexpr (S::kSplit) {
#pragma unroll
      for (int q = 0; q < S::kSegPT; ++q) {
        const int seg = tid + q * 256;
        if (S::kSegs % 256 == 0 || seg < S::kSegs) {
          const int64_t col = jb + seg / (D / 4) < last ? jb + seg / (D / 4) : last;
          st.y4[q] = *reinterpret_cast<const f32x4*>(J.yc + col * D + 4 * (seg % (D / 4)));
        }
      }
    } else {
#pragma unroll
      for (int q = 0; q < S::kY; ++q) {
        const int e = tid + q * 256;
        const int64_t col = jb + e / D < last ? jb + e / D : last;
        st.y[q] = J.yc[col * D + e % D];
      }
    }
    if constexpr (VS > 0) {
#pragma unroll
      for (int q = 0; q < StageG<T, D, VS>::kV; ++q) {
        const int e = tid + q * 256;
        const int64_t col = jb + e / VS < last ? jb + e / VS : last;
        if (e < kVals) st.v[q] = J.v[col * 16 + e % VS];
      }
    }
    if (tid < kColsG) {
      const int64_t col = jb + tid < last ? jb + tid : last;
      st.yn = J.yn[col];
      st.valid = jb + tid < j1;
    }
  }
}

template <typename T, int D, int MV>
__device__ __forceinline__ void g_item(const GJob<T>& J, int64_t rg, int split,
                                       const double* __restrict__ etab) {
  typedef typename GT<T>::acc_t acc_t;
  constexpr bool kF32 = std::is_same<T, float>::value;
  constexpr int KS = D / 4;
  constexpr int NT = kColsG / 16;
  constexpr bool kSplit = g_uses_split<T, D>();
  constexpr int NC = s3_steps<D>();  // bf16 MFMA steps of the split path
  constexpr int PY = s3_pitch<D>();
  // the chunk's points: their values, or (split path) their slices h | m | l
  // per row; the form not used keeps one element
  __shared__ T sY[kSplit ? 1 : kColsG][D + 1];
  __shared__ __attribute__((aligned(16))) __bf16 sYb[kSplit ? kColsG : 1][PY];
  __shared__ T sAy[kColsG];
  __shared__ T sV[kColsG][17];  // [column][rhs]

  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int g = lane >> 4, li = lane & 15;
  const int64_t nr = J.nr, nc = J.nc;
  const int64_t row0 = (rg * 4 + wave) * (16 * kRTg);

  T xb[kRTg][kSplit ? 1 : KS];  // B operand: X[i0 + li][4 ks + g]
  bf16x8 xbb[kRTg][kSplit ? NC : 1];  // split path: B operand of step st
  int aoff[kSplit ? NC : 1];          // split path: LDS offset of the A operand in a row
  acc_t cinit[kRTg];
#pragma unroll
  for (int rt = 0; rt < kRTg; ++rt) {
    int64_t i = row0 + rt * 16 + li;
    if (i > nr - 1) i = nr - 1;
    if constexpr (kSplit) {
#pragma unroll
      for (int st = 0; st < NC; ++st) {
        xbb[rt][st] = s3_b_operand<D>(J.xc + i * D, st, g);
        if (rt == 0) aoff[st] = s3_a_offset<D>(st, g);
      }
    } else {
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) xb[rt][ks] = J.xc[i * D + 4 * ks + g];
    }
    const T h = T(-0.5) * J.xn[i];
    cinit[rt] = acc_t{h, h, h, h};
  }
  // E.V on the matrix cores (MV = 0): two accumulators per row tile (even /
  // odd K steps) keep independent MFMA chains in flight.  On the VALU
  // (MV = 1, 2, 4, 8 right-hand sides): lane l sums E[li][col] V[col][c] over
  // its columns.
  // MV < 0: the store variant (the kernel values go to J.store, no V)
  constexpr bool kStore = MV < 0;
  constexpr int MA = MV == 0 ? 2 : 1;
  constexpr int MC = MV <= 0 ? 1 : MV;
  acc_t acc[kRTg][MA];
  T accv[kRTg][MC];
  double fold[kRTg][4];  // FP32 only: FP64 running sums of the output entries
#pragma unroll
  for (int rt = 0; rt < kRTg; ++rt) {
#pragma unroll
    for (int a = 0; a < MA; ++a) acc[rt][a] = acc_t{T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int c = 0; c < MC; ++c) accv[rt][c] = T(0);
#pragma unroll
    for (int u = 0; u < 4; ++u) fold[rt][u] = 0.0;
  }
  const T s2 = T(2) * J.s;

  const int64_t j0 = (int64_t)split * J.per;
  int64_t j1 = j0 + J.per;
  if (j1 > nc) j1 = nc;
  constexpr int VS = MV == 0 ? 16 : kStore ? 0 : MV;  // V slots staged per column
  StageG<T, D, VS> st;
  if (j0 < j1) stage_fetch<T, D, VS>(J, j0, j1, tid, st);
  int chunk = 0;
  for (int64_t jb = j0; jb < j1; jb += kColsG, ++chunk) {
    __syncthreads();  // the previous chunk's LDS reads are done
    if constexpr (kSplit) {
      typedef StageG<T, D, VS> S;
#pragma unroll
      for (int q = 0; q < S::kSegPT; ++q) {
        const int seg = tid + q * 256;
        if (S::kSegs % 256 == 0 || seg < S::kSegs)
          s3_store_quad<D>(st.y4[q], seg % (D / 4), sYb[seg / (D / 4)]);
      }
    } else {
#pragma unroll
      for (int q = 0; q < StageG<T, D, VS>::kY; ++q) {
        const int e = tid + q * 256;
        sY[e / D][e % D] = st.y[q];
      }
    }
    if constexpr (VS > 0) {
#pragma unroll
      for (int q = 0; q < StageG<T, D, VS>::kV; ++q) {
        const int e = tid + q * 256;
        if (e < kColsG * VS) sV[e / VS][e % VS] = st.v[q];
      }
    }
    if (tid < kColsG) sAy[tid] = st.valid ? -J.s * st.yn : GT<T>::kFar;
    __syncthreads();
    if (jb + kColsG < j1) stage_fetch<T, D, VS>(J, jb + kColsG, j1, tid, st);
    if (row0 >= nr) continue;
    acc_t dot[2][kRTg];
    auto distance = [&](int ct, acc_t* dd) {
      if constexpr (kSplit) {
        bf16x8 ya[NC];  // A operand: slices of Y[ct*16 + li]
#pragma unroll
        for (int st = 0; st < NC; ++st)
          ya[st] = *reinterpret_cast<const bf16x8*>(&sYb[ct * 16 + li][aoff[st]]);
#pragma unroll
        for (int rt = 0; rt < kRTg; ++rt)
          dd[rt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ya[0], xbb[rt][0], cinit[rt], 0, 0, 0);
#pragma unroll
        for (int st = 1; st < NC; ++st)
#pragma unroll
          for (int rt = 0; rt < kRTg; ++rt)
            dd[rt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ya[st], xbb[rt][st], dd[rt], 0, 0, 0);
      } else {
        T ya[KS];  // A operand: Y[ct*16 + li][4 ks + g]
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) ya[ks] = sY[ct * 16 + li][4 * ks + g];
        // the first K step reads the -||x||^2 / 2 start from cinit directly
#pragma unroll
        for (int rt = 0; rt < kRTg; ++rt) dd[rt] = GT<T>::mfma(ya[0], xb[rt][0], cinit[rt]);
#pragma unroll
        for (int ks = 1; ks < KS; ++ks)
#pragma unroll
          for (int rt = 0; rt < kRTg; ++rt) dd[rt] = GT<T>::mfma(ya[ks], xb[rt][ks], dd[rt]);
      }
    };
    // FP32: the distance MFMAs of column tile ct + 1 are issued before the
    // exp work of tile ct, which does not depend on them (the FP32 matrix
    // cores run beside the VALU).  FP64 matrix and vector instructions do
    // not overlap, so the FP64 tile computes one tile's distances at a time
    // and spends the registers on occupancy instead.
    constexpr bool kAhead = std::is_same<T, float>::value;
    if (kAhead) distance(0, dot[0]);
#pragma unroll
    for (int ct = 0; ct < NT; ++ct) {
      if (!kAhead) distance(ct, dot[ct & 1]);
      else if (ct + 1 < NT) distance(ct + 1, dot[(ct + 1) & 1]);
      T ay[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) ay[t] = sAy[ct * 16 + GT<T>::col(t, g)];
      // dot[rt][t] = y_{col(t,g)} . x_{li} - ||x_{li}||^2 / 2
      T e[kRTg][4];
#pragma unroll
      for (int rt = 0; rt < kRTg; ++rt)
#pragma unroll
        for (int t = 0; t < 4; ++t)
          e[rt][t] = GT<T>::ex(fma_g(dot[ct & 1][rt][t], s2, ay[t]), etab);
      if constexpr (kStore) {
        // entry (row i0 + li, column col(t, g)) of the block; FP32 lanes
        // hold four consecutive columns (col = 4 g + t): one 16-byte store
        // (aligned: chunks start at multiples of 64 columns, ld is a
        // multiple of 8)
#pragma unroll
        for (int rt = 0; rt < kRTg; ++rt) {
          const int64_t i = row0 + rt * 16 + li;
          if (i >= nr) continue;
          if constexpr (kF32) {
            const int64_t jc = jb + ct * 16 + 4 * g;
            if (jc + 3 < j1) {
              *reinterpret_cast<f32x4*>(&J.store[i * J.ld + jc]) =
                  f32x4{e[rt][0], e[rt][1], e[rt][2], e[rt][3]};
              continue;
            }
          }
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const int64_t j = jb + ct * 16 + GT<T>::col(t, g);
            if (j < j1) J.store[i * J.ld + j] = e[rt][t];
          }
        }
      } else if constexpr (MV == 0) {
        // A of E.V step t: lane l holds E[li][col(t, g)] (K index g)
        T vb[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) vb[t] = sV[ct * 16 + GT<T>::col(t, g)][li];  // V[col][c = li]
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int rt = 0; rt < kRTg; ++rt)
            acc[rt][t & 1] = GT<T>::mfma(e[rt][t], vb[t], acc[rt][t & 1]);
      } else {
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int c = 0; c < MV; ++c) {
            const T v = sV[ct * 16 + GT<T>::col(t, g)][c];
#pragma unroll
            for (int rt = 0; rt < kRTg; ++rt) accv[rt][c] = fma_g(e[rt][t], v, accv[rt][c]);
          }
      }
    }
    if constexpr (kF32 && !kStore) {
      if ((chunk + 1) % kFoldG == 0) {
#pragma unroll
        for (int rt = 0; rt < kRTg; ++rt) {
          if constexpr (MV == 0) {
#pragma unroll
            for (int u = 0; u < 4; ++u) fold[rt][u] += (double)acc[rt][0][u] + (double)acc[rt][1][u];
            acc[rt][0] = acc_t{0.f, 0.f, 0.f, 0.f};
            acc[rt][1] = acc_t{0.f, 0.f, 0.f, 0.f};
          } else {
#pragma unroll
            for (int c = 0; c < MC; ++c) {
              fold[rt][c] += (double)accv[rt][c];
              accv[rt][c] = 0.f;
            }
          }
        }
      }
    }
  }
  if (kStore || row0 >= nr) return;
  // partial slots: split-major, rows of J.M values (the product's columns)
  double* __restrict__ out = J.part + (int64_t)split * nr * J.M;
  if constexpr (MV == 0) {
#pragma unroll
    for (int rt = 0; rt < kRTg; ++rt)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        // E.V output: lane l, element t holds W[i0 + col(t, g)][c = li]
        const int64_t i = row0 + rt * 16 + GT<T>::col(t, g);
        const double w = kF32 ? fold[rt][t] + ((double)acc[rt][0][t] + (double)acc[rt][1][t])
                              : (double)acc[rt][0][t] + (double)acc[rt][1][t];
        if (i < nr && li < J.M) out[i * J.M + li] = w;
      }
  } else {
#pragma unroll
    for (int rt = 0; rt < kRTg; ++rt)
#pragma unroll
      for (int c = 0; c < MV; ++c) {
        // lanes li, li+16, li+32, li+48 hold partial sums of row li: add in
        // a fixed pairing ((g0 + g1) + (g2 + g3))
        double a = kF32 ? fold[rt][c] + (double)accv[rt][c] : (double)accv[rt][c];
        a += __shfl_xor(a, 16);
        a += __shfl_xor(a, 32);
        const int64_t i = row0 + rt * 16 + li;
        if (g == 0 && i < nr && c < J.M) out[i * J.M + c] = a;
      }
  }
}

constexpr int kMaxGJobs = 8;
template <typename T>
struct GTable {
  GJob<T> job[kMaxGJobs];
  int njobs;
  int64_t total;
};

// Occupancy floors.  FP64 tiles up to 16 padded dimensions are held to 128
// VGPRs, 4 waves per SIMD (no spill up to 2 right-hand sides: the distance
// of one column tile at a time and V staged for the m columns used; the
// 2,000,000 x 10,000 product 17.2-18.7 -> 16.6-16.8 ms together with the
// XCD item order; 5 waves spill 28+ registers and lose 1-50%; with 4 to 16
// right-hand sides they spill 14-43 registers and are still 1-6% faster
// than at 3 waves, measured at d = 8 and 16 on 200,000 x 100,000).  Up to 48
// padded dimensions they are held to 168 VGPRs, 3 waves instead of 2, at the
// price of a register spill (at d = 32, up to 44 registers, outside the
// inner loop); measured on N = 200,000: d = 32 with 1 / 8 right-hand sides
// 26% / 9% faster, d = 24 and 48 5-13%; 4 waves at d = 32 lose 1-11%; at
// d = 64 the spill passes 800 bytes and costs 20%, so those keep the
// compiler's choice.  FP32 tiles up to
// 32 padded dimensions are held to 128 VGPRs (4 waves instead of 3; d = 32
// spills 52-184 bytes): 2-12% faster over 1-8 right-hand sides.
// The FP64 store variant (MV < 0: kernel values written out, bound by the
// writes) keeps 2 waves per SIMD, where 3-4 would spill its store addresses.
template <typename T, int D, int MV>
constexpr int g_waves_per_eu() {
  if (std::is_same<T, double>::value && MV < 0) return D <= 48 ? 2 : 1;
  return std::is_same<T, double>::value ? (D <= 16 ? 4 : D <= 48 ? 3 : 1) : (D <= 32 ? 4 : 1);
}

template <typename T, int D, int MV>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(g_waves_per_eu<T, D, MV>())))
void tile_gauss_mfma(const GTable<T> tab) {
  __shared__ double etab[GT<T>::kTable];  // FP64 exp table (one unused entry for FP32 tiles)
  if constexpr (std::is_same<T, double>::value) {
    GT<T>::fill(etab);
    __syncthreads();
  }
  for (int64_t w = blockIdx.x; w < xcd_slots(tab.total); w += gridDim.x) {
    const int64_t item = xcd_item(w, tab.total);
    if (item >= tab.total) continue;
    int jn = 0;
    while (jn + 1 < tab.njobs && item >= tab.job[jn + 1].item0) ++jn;
    const GJob<T>& J = tab.job[jn];
    if (needs_direct(J)) continue;  // uniform over the workgroup
    // row groups of one column split are consecutive items
    const int64_t local = item - J.item0;
    const int64_t nrg = (J.nr + 4 * 16 * kRTg - 1) / (4 * 16 * kRTg);
    g_item<T, D, MV>(J, local % nrg, (int)(local / nrg), etab);
  }
}

// Direct-difference Gaussian tile for the jobs the expansion cannot serve to
// the precision's accuracy: same items and partial-sum layout as
// tile_gauss_mfma.  Thread t owns row t % 128 of the item and every other
// column (t / 128 picks the parity); the column points and V are
// wave-uniform (scalar loads).  FP32 sums fold into FP64 every 256 columns;
// the two parities are added in a fixed order.
template <typename T, int D>
__global__ __launch_bounds__(256) void tile_gauss_direct(const GTable<T> tab) {
  constexpr bool kF32 = std::is_same<T, float>::value;
  __shared__ double etab[kExpTable];
  __shared__ double sW[128][17];
  if constexpr (!kF32) exp64_table_fill(etab);
  __syncthreads();
  const int tid = threadIdx.x;
  const int r = tid & 127, h = tid >> 7;
  for (int64_t w = blockIdx.x; w < xcd_slots(tab.total); w += gridDim.x) {
    const int64_t item = xcd_item(w, tab.total);
    if (item >= tab.total) continue;
    int jn = 0;
    while (jn + 1 < tab.njobs && item >= tab.job[jn + 1].item0) ++jn;
    const GJob<T>& J = tab.job[jn];
    if (!needs_direct(J)) continue;  // uniform over the workgroup
    const int64_t local = item - J.item0;
    const int64_t nrg = (J.nr + 4 * 16 * kRTg - 1) / (4 * 16 * kRTg);
    const int64_t rg = local % nrg;
    const int split = (int)(local / nrg);
    const int64_t nr = J.nr;
    const int64_t i = rg * (4 * 16 * kRTg) + r;
    const int64_t ic = i < nr ? i : nr - 1;
    T x[D];
#pragma unroll
    for (int k = 0; k < D; ++k) x[k] = J.xc[ic * D + k];
    double acc64[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) acc64[c] = 0.0;
    const int64_t j0 = (int64_t)split * J.per;
    int64_t j1 = j0 + J.per;
    if (j1 > J.nc) j1 = J.nc;
    for (int64_t jb = j0; jb < j1; jb += 2 * 256) {
      const int64_t je = jb + 2 * 256 < j1 ? jb + 2 * 256 : j1;
      T acc[16];
#pragma unroll
      for (int c = 0; c < 16; ++c) acc[c] = T(0);
      for (int64_t j = jb + h; j < je; j += 2) {
        const T* __restrict__ y = J.yc + j * D;
        T s = T(0);
#pragma unroll
        for (int k = 0; k < D; ++k) {
          const T t = x[k] - y[k];
          s = fma_g(t, t, s);
        }
        // direct differences serve unbounded exponents: the clamped exp64
        T e;
        if constexpr (kF32) e = GT<T>::ex(-J.s * s, etab);
        else e = exp64(-J.s_nat * s, etab);
        const T* __restrict__ v = J.v + j * 16;
#pragma unroll
        for (int c = 0; c < 16; ++c) acc[c] = fma_g(e, v[c], acc[c]);
      }
#pragma unroll
      for (int c = 0; c < 16; ++c) acc64[c] += (double)acc[c];
    }
    __syncthreads();  // sW of the previous item is consumed
    if (h == 1) {
#pragma unroll
      for (int c = 0; c < 16; ++c) sW[r][c] = acc64[c];
    }
    __syncthreads();
    if (h == 0 && i < nr) {
      double* __restrict__ out = J.part + ((int64_t)split * nr + i) * J.M;
      for (int c = 0; c < J.M; ++c) out[c] = acc64[c] + sW[r][c];
    }
  }
}

template <typename T>
__global__ void zero_scalar(T* p) {
  *p = T(0);
}

// centred copy and squared norms (formed in FP64 from the rounded centred
// coordinates); the largest norm goes to *xmax (wave maximum, then an integer
// atomic max on the bits: the norms are >= 0, whose IEEE bit patterns order
// like the values)
template <typename T>
__global__ void pack_centred(const double* __restrict__ X, int64_t n, int d, int dpad,
                             const double* __restrict__ centre, T* __restrict__ xc,
                             T* __restrict__ xn, T* __restrict__ xmax) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double s = 0.0;
  if (i < n) {
    for (int k = 0; k < dpad; ++k) {
      const T v = k < d ? (T)(X[i * d + k] - centre[k]) : T(0);
      xc[i * dpad + k] = v;
      s += (double)v * (double)v;
    }
    xn[i] = (T)s;
  }
  T m = (T)s;
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
  if ((threadIdx.x & 63) == 0) {
    if constexpr (std::is_same<T, double>::value)
      atomicMax(reinterpret_cast<unsigned long long*>(xmax), (unsigned long long)__double_as_longlong(m));
    else
      atomicMax(reinterpret_cast<unsigned int*>(xmax), (unsigned int)__float_as_uint(m));
  }
}

template <typename T>
__global__ void pack_v16(VecView V, int64_t n, int c0, int mc, T* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * 16) return;
  const int64_t j = t / 16;
  const int c = (int)(t % 16);
  out[t] = c < mc ? (T)V.p[j * V.rs + (int64_t)(c0 + c) * V.cs] : T(0);
}

struct GSplit {
  int nsplit;
  int64_t per;
};

GSplit g_split(int64_t nr, int64_t nc) {
  const int64_t ns = split_count(nr, nc, 4 * 16 * kRTg, 256);
  int64_t per = ceil_div(std::max<int64_t>(nc, 1), ns);
  per = ceil_div(per, kColsG) * kColsG;
  return {(int)ns, per};
}

// E.V reduction variant for m right-hand sides.  Per 16 x 16 tile the MFMA
// reduction costs four 16x16x4 MFMAs whatever m is, the VALU one m FMAs per
// entry: FP64 (64-cycle MFMA) keeps the VALU up to 8 right-hand sides, FP32
// (32-cycle MFMA, and a tile already bound by the matrix cores) up to 4.
template <typename T>
int g_variant(int m) {
  const int vmax = std::is_same<T, double>::value ? 8 : 4;
  if (m > vmax) return 0;
  return m <= 1 ? 1 : m <= 2 ? 2 : m <= 4 ? 4 : 8;
}

template <typename T, int D>
void launch_d(int mv, unsigned grid, const GTable<T>& tab, hipStream_t s) {
  switch (mv) {
    case 1: tile_gauss_mfma<T, D, 1><<<grid, 256, 0, s>>>(tab); break;
    case 2: tile_gauss_mfma<T, D, 2><<<grid, 256, 0, s>>>(tab); break;
    case 4: tile_gauss_mfma<T, D, 4><<<grid, 256, 0, s>>>(tab); break;
    case 8:
      if constexpr (std::is_same<T, double>::value) {
        tile_gauss_mfma<T, D, 8><<<grid, 256, 0, s>>>(tab);
        break;
      }
      [[fallthrough]];
    default: tile_gauss_mfma<T, D, 0><<<grid, 256, 0, s>>>(tab); break;
  }
}

template <typename T>
int carve_centred(int64_t n, int32_t dpad, Arena& arena, PointSet* out, const T** xc,
                  const T** xn, const T** xmax) {
  *xc = arena.take<T>((size_t)n * dpad);
  *xn = arena.take<T>(n);
  *xmax = arena.take<T>(1);
  if (!out->centre) {
    out->centre = arena.take<double>(64);
    out->cpart = arena.take<double>(256 * 64);
  }
  return KRR_OK;
}

template <typename T>
int fill_centred(const double* X, const double* centre, const PointSet& ps, const T* xc,
                 const T* xn, const T* xmax, hipStream_t s) {
  const int64_t n = ps.n;
  zero_scalar<T><<<1, 1, 0, s>>>(const_cast<T*>(xmax));
  KRR_LAUNCH_CHECK("zero_scalar");
  if (n == 0) return KRR_OK;
  double* c = const_cast<double*>(ps.centre);
  if (centre) {
    if (centre != c)
      KRR_TRY(hip_check(hipMemcpyAsync(c, centre, sizeof(double) * ps.d, hipMemcpyDeviceToDevice, s),
                        "centre copy"));
  } else {
    KRR_TRY(compute_centre(X, n, ps.d, c, ps.cpart, s));
  }
  pack_centred<T><<<(unsigned)ceil_div(n, 256), 256, 0, s>>>(X, n, ps.d, ps.dpad, c,
                                                             const_cast<T*>(xc), const_cast<T*>(xn),
                                                             const_cast<T*>(xmax));
  KRR_LAUNCH_CHECK("pack_centred");
  return KRR_OK;
}

template <typename T>
size_t g_scratch_bytes(int64_t nr, int64_t nc) {
  GSplit sp = g_split(nr, nc);
  Arena a;
  a.take<T>((size_t)std::max<int64_t>(nc, 1) * 16);
  a.take<double>((size_t)sp.nsplit * std::max<int64_t>(nr, 1) * 16);
  return a.used;
}

template <typename T>
int g_prepare(double sigma, const T* rxc, const T* rxn, const T* rxmax, const T* cxc,
              const T* cxn, const T* cxmax, int64_t nr, int64_t nc, int dpad, VecView V, int c0,
              int mc, double rmax_host, double cmax_host, Arena& scratch, GJob<T>* out,
              hipStream_t s) {
  GSplit sp = g_split(nr, nc);
  T* v = scratch.take<T>((size_t)std::max<int64_t>(nc, 1) * 16);
  double* part = scratch.take<double>((size_t)sp.nsplit * nr * 16);
  if (!scratch.ok()) {
    set_error("Gaussian MFMA product scratch too small");
    return KRR_EWORKSPACE;
  }
  if (nc > 0) {
    pack_v16<T><<<(unsigned)ceil_div(nc * 16, 256), 256, 0, s>>>(V, nc, c0, mc, v);
    KRR_LAUNCH_CHECK("pack_v16");
  }
  const double s_nat = 1.0 / (2.0 * sigma * sigma);
  GJob<T>& j = *out;
  j.xc = rxc;
  j.xn = rxn;
  j.xmax = rxmax;
  j.ymax = cxmax;
  j.yc = cxc;
  j.yn = cxn;
  j.v = v;
  j.part = part;
  j.nr = nr;
  j.nc = nc;
  j.per = sp.per;
  j.item0 = 0;
  // exponents in the units of the tile's exp: base 2 for FP32 (v_exp_f32),
  // ln2/1024 for FP64 (exp64_u)
  j.s = (T)(GT<T>::kExpScale * s_nat);
  j.s_nat = s_nat;
  j.nsplit = sp.nsplit;
  j.M = mc;
  j.dpad = dpad;
  // the device's guard on the host, in the same arithmetic, when both
  // maxima are known
  j.route = 0;
  if (rmax_host >= 0.0 && cmax_host >= 0.0)
    j.route = s_nat * (rmax_host + cmax_host) * (dpad + 3) > GT<T>::kBound ? 2 : 1;
  return KRR_OK;
}

template <typename T>
int g_launch(const std::vector<GJob<T>>& jobs, hipStream_t s) {
  for (int D : {4, 8, 16, 20, 24, 32, 48, 64}) {
    for (int mv : {1, 2, 4, 8, 0}) {
      std::vector<GJob<T>> sel;
      for (const GJob<T>& j : jobs)
        if (j.dpad == D && g_variant<T>(j.M) == mv) sel.push_back(j);
      for (size_t j0 = 0; j0 < sel.size(); j0 += kMaxGJobs) {
        GTable<T> tab{};
        int64_t total = 0;
        int nj = 0;
        for (size_t j = j0; j < sel.size() && nj < kMaxGJobs; ++j, ++nj) {
          tab.job[nj] = sel[j];
          tab.job[nj].item0 = total;
          total += ceil_div(sel[j].nr, (int64_t)4 * 16 * kRTg) * sel[j].nsplit;
        }
        tab.njobs = nj;
        tab.total = total;
        if (total == 0) continue;
        const unsigned grid = (unsigned)std::min<int64_t>(xcd_slots(total), kGridCap);
        // kernels no job of the table needs are not launched
        bool any_mfma = false, any_direct = false;
        for (int q = 0; q < nj; ++q) {
          any_mfma = any_mfma || tab.job[q].route != 2;
          any_direct = any_direct || tab.job[q].route != 1;
        }
        void* tok = tile_timer_start(s, mv);
        if (any_mfma) switch (D) {
          case 4: launch_d<T, 4>(mv, grid, tab, s); break;
          case 8: launch_d<T, 8>(mv, grid, tab, s); break;
          case 16: launch_d<T, 16>(mv, grid, tab, s); break;
          case 20: launch_d<T, 20>(mv, grid, tab, s); break;
          case 24: launch_d<T, 24>(mv, grid, tab, s); break;
          case 32: launch_d<T, 32>(mv, grid, tab, s); break;
          case 48: launch_d<T, 48>(mv, grid, tab, s); break;
          default: launch_d<T, 64>(mv, grid, tab, s); break;
        }
        KRR_LAUNCH_CHECK("tile_gauss_mfma");
        // the direct tile serves the jobs the MFMA tile skipped (the choice is
        // made on the device when the norms are not known on the host, so the
        // launch stays asynchronous)
        if (any_direct) switch (D) {
          case 4: tile_gauss_direct<T, 4><<<grid, 256, 0, s>>>(tab); break;
          case 8: tile_gauss_direct<T, 8><<<grid, 256, 0, s>>>(tab); break;
          case 16: tile_gauss_direct<T, 16><<<grid, 256, 0, s>>>(tab); break;
          case 20: tile_gauss_direct<T, 20><<<grid, 256, 0, s>>>(tab); break;
          case 24: tile_gauss_direct<T, 24><<<grid, 256, 0, s>>>(tab); break;
          case 32: tile_gauss_direct<T, 32><<<grid, 256, 0, s>>>(tab); break;
          case 48: tile_gauss_direct<T, 48><<<grid, 256, 0, s>>>(tab); break;
          default: tile_gauss_direct<T, 64><<<grid, 256, 0, s>>>(tab); break;
        }
        KRR_LAUNCH_CHECK("tile_gauss_direct");
        tile_timer_stop(tok, s);
      }
    }
  }
  return KRR_OK;
}

}  // namespace

int carve_f64c(int64_t n, int32_t dpad, Arena& arena, PointSet* out) {
  return carve_centred<double>(n, dpad, arena, out, &out->xc64, &out->xn64, &out->xmax64);
}
int fill_f64c(const double* X, const double* centre, const PointSet& ps, hipStream_t s) {
  return fill_centred<double>(X, centre, ps, ps.xc64, ps.xn64, ps.xmax64, s);
}
int carve_f32c(int64_t n, int32_t dpad, Arena& arena, PointSet* out) {
  return carve_centred<float>(n, dpad, arena, out, &out->xc32, &out->xn32, &out->xmax32);
}
int fill_f32c(const double* X, const double* centre, const PointSet& ps, hipStream_t s) {
  return fill_centred<float>(X, centre, ps, ps.xc32, ps.xn32, ps.xmax32, s);
}

namespace {

template <typename T>
__global__ __launch_bounds__(256) void zero_pad_cols(T* __restrict__ out, int64_t nr, int64_t nc,
                                                     int64_t ld) {
  const int64_t w = ld - nc;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= nr * w) return;
  out[(e / w) * ld + nc + e % w] = T(0);
}

template <typename T>
int g_block_store(double sigma, const T* rxc, const T* rxn, const T* rxmax, const T* cxc,
                  const T* cxn, const T* cxmax, int64_t nr, int64_t nc, int dpad,
                  double rmax_host, double cmax_host, T* out, int64_t ld, bool* done,
                  hipStream_t s) {
  *done = false;
  const double s_nat = 1.0 / (2.0 * sigma * sigma);
  // the products' guard, on the host: unknown maxima or too coarse an
  // expansion leave the block to direct differences
  if (rmax_host < 0.0 || cmax_host < 0.0) return KRR_OK;
  if (s_nat * (rmax_host + cmax_host) * (dpad + 3) > GT<T>::kBound) return KRR_OK;
  const GSplit sp = g_split(nr, nc);
  GTable<T> tab{};
  GJob<T>& j = tab.job[0];
  j.xc = rxc;
  j.xn = rxn;
  j.xmax = rxmax;
  j.ymax = cxmax;
  j.yc = cxc;
  j.yn = cxn;
  j.nr = nr;
  j.nc = nc;
  j.per = sp.per;
  j.s = (T)(GT<T>::kExpScale * s_nat);
  j.s_nat = s_nat;
  j.nsplit = sp.nsplit;
  j.dpad = dpad;
  j.route = 1;
  j.store = out;
  j.ld = ld;
  tab.njobs = 1;
  tab.total = ceil_div(nr, (int64_t)4 * 16 * kRTg) * sp.nsplit;
  if (tab.total > 0 && nc > 0) {
    const unsigned grid = (unsigned)std::min<int64_t>(xcd_slots(tab.total), kGridCap);
    switch (dpad) {
      case 4: tile_gauss_mfma<T, 4, -1><<<grid, 256, 0, s>>>(tab); break;
      case 8: tile_gauss_mfma<T, 8, -1><<<grid, 256, 0, s>>>(tab); break;
      case 16: tile_gauss_mfma<T, 16, -1><<<grid, 256, 0, s>>>(tab); break;
      case 20: tile_gauss_mfma<T, 20, -1><<<grid, 256, 0, s>>>(tab); break;
      case 24: tile_gauss_mfma<T, 24, -1><<<grid, 256, 0, s>>>(tab); break;
      case 32: tile_gauss_mfma<T, 32, -1><<<grid, 256, 0, s>>>(tab); break;
      case 48: tile_gauss_mfma<T, 48, -1><<<grid, 256, 0, s>>>(tab); break;
      default: tile_gauss_mfma<T, 64, -1><<<grid, 256, 0, s>>>(tab); break;
    }
    KRR_LAUNCH_CHECK("tile_gauss_mfma (store)");
  }
  if (ld > nc && nr > 0) {
    zero_pad_cols<T><<<(unsigned)ceil_div(nr * (ld - nc), 256), 256, 0, s>>>(out, nr, nc, ld);
    KRR_LAUNCH_CHECK("zero_pad_cols");
  }
  *done = true;
  return KRR_OK;
}

}  // namespace

int gauss_block_store(krr_precision prec, double sigma, const PointSet& rows,
                      const PointSet& cols, void* out, int64_t ld, bool* done, hipStream_t s) {
  if (prec == KRR_FP64) {
    if (!rows.xc64 || !cols.xc64) {
      *done = false;
      return KRR_OK;
    }
    return g_block_store<double>(sigma, rows.xc64, rows.xn64, rows.xmax64, cols.xc64, cols.xn64,
                                 cols.xmax64, rows.n, cols.n, rows.dpad, rows.max_host,
                                 cols.max_host, static_cast<double*>(out), ld, done, s);
  }
  if (!rows.xc32 || !cols.xc32) {
    *done = false;
    return KRR_OK;
  }
  return g_block_store<float>(sigma, rows.xc32, rows.xn32, rows.xmax32, cols.xc32, cols.xn32,
                              cols.xmax32, rows.n, cols.n, rows.dpad, rows.max_host,
                              cols.max_host, static_cast<float*>(out), ld, done, s);
}

int learn_norm_max(PointSet& ps, hipStream_t s) {
  if (ps.n == 0) return KRR_OK;
  if (ps.xmax64) {
    double v = 0.0;
    KRR_TRY(hip_check(hipMemcpyAsync(&v, ps.xmax64, sizeof(double), hipMemcpyDeviceToHost, s),
                      "norm max"));
    KRR_TRY(hip_check(hipStreamSynchronize(s), "sync"));
    ps.max_host = v;
  } else if (ps.xmax32) {
    float v = 0.0f;
    KRR_TRY(hip_check(hipMemcpyAsync(&v, ps.xmax32, sizeof(float), hipMemcpyDeviceToHost, s),
                      "norm max"));
    KRR_TRY(hip_check(hipStreamSynchronize(s), "sync"));
    ps.max_host = (double)v;
  }
  return KRR_OK;
}

size_t product_f64mfma_scratch_bytes(int64_t nr, int64_t nc) { return g_scratch_bytes<double>(nr, nc); }
size_t product_f32mfma_scratch_bytes(int64_t nr, int64_t nc) { return g_scratch_bytes<float>(nr, nc); }

int f64_prepare(double sigma, const PointSet& rows, const PointSet& cols, VecView V, int c0, int mc,
                Arena& scratch, F64Job* out, hipStream_t s) {
  if (!rows.xc64 || !cols.xc64 || rows.dpad != cols.dpad) {
    set_error("FP64 Gaussian product: centred layouts missing or inconsistent");
    return KRR_EINVAL;
  }
  return g_prepare<double>(sigma, rows.xc64, rows.xn64, rows.xmax64, cols.xc64, cols.xn64,
                           cols.xmax64, rows.n, cols.n, rows.dpad, V, c0, mc, rows.max_host,
                           cols.max_host, scratch, out, s);
}
int f32_prepare(double sigma, const PointSet& rows, const PointSet& cols, VecView V, int c0, int mc,
                Arena& scratch, F32Job* out, hipStream_t s) {
  if (!rows.xc32 || !cols.xc32 || rows.dpad != cols.dpad) {
    set_error("FP32 Gaussian product: centred layouts missing or inconsistent");
    return KRR_EINVAL;
  }
  return g_prepare<float>(sigma, rows.xc32, rows.xn32, rows.xmax32, cols.xc32, cols.xn32,
                          cols.xmax32, rows.n, cols.n, rows.dpad, V, c0, mc, rows.max_host,
                          cols.max_host, scratch, out, s);
}
int f64_launch(const std::vector<F64Job>& jobs, hipStream_t s) { return g_launch<double>(jobs, s); }
int f32_launch(const std::vector<F32Job>& jobs, hipStream_t s) { return g_launch<float>(jobs, s); }

}  // namespace krr
