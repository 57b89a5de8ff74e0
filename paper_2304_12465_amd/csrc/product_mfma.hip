// Gaussian kernel tiles on the bf16 matrix cores (precision KRR_MIXED).
//
// The squared distance is ||x||^2 + ||y||^2 - 2 x.y with the contraction x.y
// on v_mfma_f32_16x16x32_bf16 using a hi/lo split of each coordinate
// (x = hi + lo, three products hi.hi + hi.lo + lo.hi, FP32 accumulation),
// after centring the points (distances are translation invariant; centring
// shrinks ||x|| and with it the cancellation).  exp runs on the VALU in FP32.
// The reduction against V is a second split-bf16 contraction on the matrix
// cores: the output layout of the distance MFMA (lane l holds rows
// 4(l/16)..4(l/16)+3 of a 16-column tile, column l%16) is, up to a fixed
// permutation of the K index, the A-operand layout of the 16x16x32 MFMA,
// so the exponentiated tile feeds the second MFMA without any lane shuffle.
// FP32 partial sums fold into FP64 every 256 columns; per-split partials
// go to fixed slots, so results are bitwise reproducible.
#include "product.h"
#include <algorithm>

namespace krr {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

// (a, b) -> bf16 hi parts (one v_cvt_pk_bf16_f32) and bf16 lo parts of the
// remainders, packed as two 32-bit words.
__device__ __forceinline__ void split_pair(float a, float b, uint32_t& hi, uint32_t& lo) {
  const bf16x2 h = __builtin_convertvector(f32x2{a, b}, bf16x2);
  hi = __builtin_bit_cast(uint32_t, h);
  const float ha = __builtin_bit_cast(float, hi << 16);
  const float hb = __builtin_bit_cast(float, hi & 0xffff0000u);
  const bf16x2 l = __builtin_convertvector(f32x2{a - ha, b - hb}, bf16x2);
  lo = __builtin_bit_cast(uint32_t, l);
}

constexpr int kRT = 4;       // 16-row tiles per wave
constexpr int kCols = 64;    // columns per LDS chunk (four 16-column MFMA tiles)
constexpr int kFoldChunks = 4;  // FP32 chunks per FP64 fold (256 columns)

__device__ __forceinline__ __bf16 to_bf16(float x) { return (__bf16)x; }
__device__ __forceinline__ float from_bf16(__bf16 x) { return (float)x; }

// Column permutation of the V-reduction MFMA's K index: slot v (0..7) of
// lane group g holds column (v < 4 ? 4g + v : 16 + 4g + v - 4) of the chunk.
__device__ __forceinline__ int slot_col(int g, int v) { return v < 4 ? 4 * g + v : 16 + 4 * g + (v - 4); }

// Per-thread staging of one 64-column chunk: the next chunk's points, its
// -s ||y||^2 and its V tile are loaded into registers while the current
// chunk is computed, and written to LDS after the next barrier.
template <int KP>
struct Stage {
  static constexpr int kSeg = KP / 32;  // 16-byte point segments per thread and array
  bf16x8 yh[kSeg], yl[kSeg];
  bf16x8 v;    // one 16-byte V segment (hi for threads 0..127, lo for 128..255)
  float yn;    // threads 0..63: squared norm of their column
  bool valid;  // threads 0..63: the column is in range
};

// A chunk inside the column range reads with linear addresses; the last
// chunk of a range repeats its last column past the end, and those columns
// get a huge distance when the norms are stored (exp -> 0).  No loaded value
// is tested here, so the loads stay in flight across the current chunk.
template <int KP>
__device__ __forceinline__ void stage_fetch(const MfmaJob& J, int64_t jb, int64_t j1, int tid,
                                            Stage<KP>& st) {
  constexpr int SPR = KP / 8;  // segments per column
  const int64_t last = j1 - 1;
  const bool full = jb + kCols <= j1;
#pragma unroll
  for (int q = 0; q < Stage<KP>::kSeg; ++q) {
    const int e = tid + q * 256;
    const int jj = e / SPR, seg = e % SPR;
    const int64_t col = full || jb + jj < last ? jb + jj : last;
    st.yh[q] = *reinterpret_cast<const bf16x8*>(J.yhi + col * KP + seg * 8);
    st.yl[q] = *reinterpret_cast<const bf16x8*>(J.ylo + col * KP + seg * 8);
  }
  // V is stored pre-permuted in 32-column groups of 16 x 32 slots, zero
  // padded to whole 64-column chunks: a chunk is 2 x 512 contiguous values
  const uint16_t* vsrc = tid < 128 ? J.vh : J.vl;
  st.v = *reinterpret_cast<const bf16x8*>(vsrc + jb * 16 + (tid & 127) * 8);
  if (tid < kCols) {
    const int64_t col = full || jb + tid < last ? jb + tid : last;
    st.yn = J.yn[col];
    st.valid = full || jb + tid < j1;
  }
}

template <int KP>
__device__ __forceinline__ void stage_store(const Stage<KP>& st, int tid, float s,
                                            __bf16 (*sYh)[KP + 8], __bf16 (*sYl)[KP + 8],
                                            float* sAy, __bf16 (*sVh)[16][40],
                                            __bf16 (*sVl)[16][40]) {
  constexpr int SPR = KP / 8;
#pragma unroll
  for (int q = 0; q < Stage<KP>::kSeg; ++q) {
    const int e = tid + q * 256;
    const int jj = e / SPR, seg = e % SPR;
    *reinterpret_cast<bf16x8*>(&sYh[jj][seg * 8]) = st.yh[q];
    *reinterpret_cast<bf16x8*>(&sYl[jj][seg * 8]) = st.yl[q];
  }
  const int vs = tid & 127;  // (group, rhs, 8-slot segment)
  __bf16(*dst)[16][40] = tid < 128 ? sVh : sVl;
  *reinterpret_cast<bf16x8*>(&dst[vs >> 6][(vs >> 2) & 15][(vs & 3) * 8]) = st.v;
  // columns past the range get a huge distance: exp -> 0
  if (tid < kCols) sAy[tid] = st.valid ? -s * st.yn : -3.0e38f;
}

template <int KP>
__device__ __forceinline__ void mfma_item(const MfmaJob& J, int64_t rg, int split) {
  const uint16_t* __restrict__ Xhi = J.xhi;
  const uint16_t* __restrict__ Xlo = J.xlo;
  const float* __restrict__ Xn = J.xn;
  const int64_t nr = J.nr;
  const int64_t nc = J.nc;
  const float s = J.s;
  constexpr int KS = KP / 32;       // MFMA K steps of the distance contraction
  constexpr int YP = KP + 8;        // LDS row pitch (bf16) of the column points
  constexpr int NG = kCols / 32;    // 32-column groups per chunk (V-reduction K)
  __shared__ __attribute__((aligned(16))) __bf16 sYh[kCols][YP];
  __shared__ __attribute__((aligned(16))) __bf16 sYl[kCols][YP];
  __shared__ __attribute__((aligned(16))) float sAy[kCols];
  __shared__ __attribute__((aligned(16))) __bf16 sVh[NG][16][32 + 8];  // [group][c][slot]
  __shared__ __attribute__((aligned(16))) __bf16 sVl[NG][16][32 + 8];
  // FP64 running sums of each lane's outputs (each lane touches only its own
  // entries, so no barrier is involved)
  __shared__ double sAcc[4][kRT * 4][64];

  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int g = lane >> 4, li = lane & 15;
  const int64_t row0 = (rg * 4 + wave) * (16 * kRT);

  // Row operands (B of the distance MFMA): X[i0 + li][8g .. 8g+8] per K
  // step.  The distance MFMA starts from -||x||^2 / 2 (accumulator init), so
  // its result is x.y - ||x||^2 / 2 and one FMA gives the exponent
  // 2 s (x.y - ||x||^2/2) - s ||y||^2 = -s ||x - y||^2.
  bf16x8 xh[kRT][KS], xl[kRT][KS];
  f32x4 cinit[kRT];
#pragma unroll
  for (int rt = 0; rt < kRT; ++rt) {
    int64_t i = row0 + rt * 16 + li;
    if (i > nr - 1) i = nr - 1;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      xh[rt][ks] = *reinterpret_cast<const bf16x8*>(Xhi + i * KP + ks * 32 + g * 8);
      xl[rt][ks] = *reinterpret_cast<const bf16x8*>(Xlo + i * KP + ks * 32 + g * 8);
    }
    const float h = -0.5f * Xn[i];
    cinit[rt] = f32x4{h, h, h, h};
  }
  f32x4 acc[kRT];
#pragma unroll
  for (int rt = 0; rt < kRT; ++rt) {
    acc[rt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int u = 0; u < 4; ++u) sAcc[wave][rt * 4 + u][lane] = 0.0;
  }
  const float s2 = 2.0f * s;

  const int64_t j0 = (int64_t)split * J.per;
  int64_t j1 = j0 + J.per;
  if (j1 > nc) j1 = nc;
  Stage<KP> st;
  if (j0 < j1) stage_fetch<KP>(J, j0, j1, tid, st);
  int chunk = 0;
  for (int64_t jb = j0; jb < j1; jb += kCols, ++chunk) {
    __syncthreads();  // the previous chunk's LDS reads are done
    stage_store<KP>(st, tid, J.s, sYh, sYl, sAy, sVh, sVl);
    __syncthreads();
    if (jb + kCols < j1) stage_fetch<KP>(J, jb + kCols, j1, tid, st);
    if (row0 >= nr) continue;  // idle wave still joins the barriers
#pragma unroll
    for (int gi = 0; gi < NG; ++gi) {
      // A operands of the distance MFMA for the group's two column tiles
      bf16x8 yh[2][KS], yl[2][KS];
#pragma unroll
      for (int ct = 0; ct < 2; ++ct)
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
          yh[ct][ks] = *reinterpret_cast<const bf16x8*>(&sYh[gi * 32 + ct * 16 + li][ks * 32 + g * 8]);
          yl[ct][ks] = *reinterpret_cast<const bf16x8*>(&sYl[gi * 32 + ct * 16 + li][ks * 32 + g * 8]);
        }
      float ay[2][4];
#pragma unroll
      for (int ct = 0; ct < 2; ++ct)
#pragma unroll
        for (int u = 0; u < 4; ++u) ay[ct][u] = sAy[gi * 32 + ct * 16 + 4 * g + u];
      const bf16x8 vh = *reinterpret_cast<const bf16x8*>(&sVh[gi][li][g * 8]);
      const bf16x8 vl = *reinterpret_cast<const bf16x8*>(&sVl[gi][li][g * 8]);
      // Software pipeline over the row tiles: the distance MFMAs of tile
      // rt + 1 are independent of the exp / split VALU work of tile rt, so
      // the two overlap.
      f32x4 dot[2][2];  // [row tile parity][column tile]
      auto distance = [&](int rt, f32x4* d) {
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
          f32x4 t = cinit[rt];
#pragma unroll
          for (int ks = 0; ks < KS; ++ks) {
            t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(yh[ct][ks], xh[rt][ks], t, 0, 0, 0);
            t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(yh[ct][ks], xl[rt][ks], t, 0, 0, 0);
            t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(yl[ct][ks], xh[rt][ks], t, 0, 0, 0);
          }
          d[ct] = t;
        }
      };
      distance(0, dot[0]);
#pragma unroll
      for (int rt = 0; rt < kRT; ++rt) {
        if (rt + 1 < kRT) distance(rt + 1, dot[(rt + 1) & 1]);
        uint32_t eh[4], el[4];  // 8 bf16 each: K slots 8g .. 8g+7
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
          // dot[u] = y_{4g+u} . x_{li} - ||x_{li}||^2 / 2; the exponent is left
          // unclamped: rounding can make it ~1e-6 positive, within the
          // split's error budget.
          const f32x4 dd = dot[rt & 1][ct];
          float e[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) e[u] = __builtin_amdgcn_exp2f(__builtin_fmaf(dd[u], s2, ay[ct][u]));
          split_pair(e[0], e[1], eh[ct * 2 + 0], el[ct * 2 + 0]);
          split_pair(e[2], e[3], eh[ct * 2 + 1], el[ct * 2 + 1]);
        }
        const bf16x8 EH = __builtin_bit_cast(bf16x8, eh);
        const bf16x8 EL = __builtin_bit_cast(bf16x8, el);
        // W[i][c] += sum_j E[i][j] V[j][c]: A = E (rows li, K slots 8g..8g+7)
        acc[rt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(EH, vh, acc[rt], 0, 0, 0);
        acc[rt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(EH, vl, acc[rt], 0, 0, 0);
        acc[rt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(EL, vh, acc[rt], 0, 0, 0);
      }
    }
    if ((chunk + 1) % kFoldChunks == 0) {
#pragma unroll
      for (int rt = 0; rt < kRT; ++rt) {
#pragma unroll
        for (int u = 0; u < 4; ++u) sAcc[wave][rt * 4 + u][lane] += (double)acc[rt][u];
        acc[rt] = f32x4{0.f, 0.f, 0.f, 0.f};
      }
    }
  }
  if (row0 >= nr) return;
  // partial slots: split-major, rows of J.M values (the product's columns)
  double* __restrict__ out = J.part + (int64_t)split * nr * J.M;
#pragma unroll
  for (int rt = 0; rt < kRT; ++rt) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      // E.V output: lane l holds W[i0 + 4g + u][c = li]
      const int64_t i = row0 + rt * 16 + 4 * g + u;
      if (i < nr && li < J.M)
        out[i * J.M + li] = sAcc[wave][rt * 4 + u][lane] + (double)acc[rt][u];
    }
  }
}

constexpr int kMaxMJobs = 8;
struct MJobTable {
  MfmaJob job[kMaxMJobs];
  int njobs;
  int64_t total;
};

// Expansion guard.  hi + lo keeps 16 significant bits of each centred
// coordinate (|x - hi - lo| <= 2^-16 |x|) and lo.lo is dropped, so each
// coordinate product is off by at most 3 2^-16 |x_l||y_l|; FP32 sums of the
// 3 kp products and the FP32 norms add about (3 kp + 2) 2^-24.  With
// 2 |x.y| <= ||x||^2 + ||y||^2 the exponent error is at most
//   s (max||x||^2 + max||y||^2) (3 2^-16 + (3 kp + 2) 2^-24),
// s = 1 / (2 sigma^2).  Above 2^-9 (a relative error of 0.2% per entry)
// the job goes to direct differences on the FP32 centred points instead.
__host__ __device__ __forceinline__ bool mixed_bound_exceeded(float s_nat, float xmax, float ymax,
                                                              int kp) {
  const float gfac = 3.0f * 0x1p-16f + (float)(3 * kp + 2) * 0x1p-24f;
  return s_nat * (xmax + ymax) * gfac > 0x1p-9f;
}
__device__ __forceinline__ bool mixed_too_coarse(const MfmaJob& J) {
  if (J.route) return J.route == 2;  // decided on the host from known norms
  return mixed_bound_exceeded(J.s_nat, *J.xmax, *J.ymax, J.kp);
}

template <int KP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(KP == 32 ? 3 : 2)))
void tile_mfma_gauss(const MJobTable tab) {
  for (int64_t w = blockIdx.x; w < xcd_slots(tab.total); w += gridDim.x) {
    const int64_t item = xcd_item(w, tab.total);
    if (item >= tab.total) continue;
    int jn = 0;
    while (jn + 1 < tab.njobs && item >= tab.job[jn + 1].item0) ++jn;
    const MfmaJob& J = tab.job[jn];
    if (mixed_too_coarse(J)) continue;  // uniform over the workgroup
    // row groups of one column split are consecutive items
    const int64_t local = item - J.item0;
    const int64_t nrg = (J.nr + 4 * 16 * kRT - 1) / (4 * 16 * kRT);
    mfma_item<KP>(J, local % nrg, (int)(local / nrg));
  }
}

// V(j, c) from the split copy in the V-reduction's permuted order (the
// inverse of slot_col within each 32-column group), as hi + lo in FP32.
__device__ __forceinline__ float vsplit_at(const MfmaJob& J, int64_t j, int c) {
  const int jj = (int)(j & 31);
  const int slot = 8 * ((jj & 15) >> 2) + (jj < 16 ? 0 : 4) + (jj & 3);
  const int64_t t = (j >> 5) * 512 + c * 32 + slot;
  return from_bf16(__builtin_bit_cast(__bf16, J.vh[t])) +
         from_bf16(__builtin_bit_cast(__bf16, J.vl[t]));
}

// Direct-difference tile for the jobs the guard refuses: FP32 differences
// of the centred FP32 points, v_exp_f32, FP32 sums folded into FP64 every
// 256 columns; the same work items (256 rows x one column split) and the
// same partial-sum slots as tile_mfma_gauss.  Thread t owns row t of the
// item; column points and V are wave-uniform.
template <int D>
__global__ __launch_bounds__(256) void tile_mixed_direct(const MJobTable tab) {
  const int tid = threadIdx.x;
  for (int64_t w = blockIdx.x; w < xcd_slots(tab.total); w += gridDim.x) {
    const int64_t item = xcd_item(w, tab.total);
    if (item >= tab.total) continue;
    int jn = 0;
    while (jn + 1 < tab.njobs && item >= tab.job[jn + 1].item0) ++jn;
    const MfmaJob& J = tab.job[jn];
    if (J.dpad != D || !mixed_too_coarse(J)) continue;  // uniform over the workgroup
    const int64_t local = item - J.item0;
    const int64_t nrg = (J.nr + 4 * 16 * kRT - 1) / (4 * 16 * kRT);
    const int64_t rg = local % nrg;
    const int split = (int)(local / nrg);
    const int64_t nr = J.nr;
    const int64_t i = rg * (4 * 16 * kRT) + tid;
    const int64_t ic = i < nr ? i : nr - 1;
    float x[D];
#pragma unroll
    for (int k = 0; k < D; ++k) x[k] = J.xf[ic * D + k];
    double acc64[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) acc64[c] = 0.0;
    const int64_t j0 = (int64_t)split * J.per;
    int64_t j1 = j0 + J.per;
    if (j1 > J.nc) j1 = J.nc;
    for (int64_t jb = j0; jb < j1; jb += kFoldChunks * kCols) {
      const int64_t je = jb + kFoldChunks * kCols < j1 ? jb + kFoldChunks * kCols : j1;
      float acc[16];
#pragma unroll
      for (int c = 0; c < 16; ++c) acc[c] = 0.f;
      for (int64_t j = jb; j < je; ++j) {
        const float* __restrict__ y = J.yf + j * D;
        float s2 = 0.f;
#pragma unroll
        for (int k = 0; k < D; ++k) {
          const float t = x[k] - y[k];
          s2 = __builtin_fmaf(t, t, s2);
        }
        const float e = __builtin_amdgcn_exp2f(-J.s * s2);
#pragma unroll
        for (int c = 0; c < 16; ++c)
          if (c < J.M) acc[c] = __builtin_fmaf(e, vsplit_at(J, j, c), acc[c]);
      }
#pragma unroll
      for (int c = 0; c < 16; ++c) acc64[c] += (double)acc[c];
    }
    if (i < nr) {
      double* __restrict__ out = J.part + ((int64_t)split * nr + i) * J.M;
      for (int c = 0; c < J.M; ++c) out[c] = acc64[c];
    }
  }
}

}  // namespace

}  // namespace krr

namespace krr {

namespace {

// centre = mean of the points, in fixed-order stages: a workgroup sums a
// chunk of rows, thread t taking coordinate t % d of rows t / d, t / d + Q,
// ... (Q = 256 / d row lanes; consecutive threads read consecutive
// addresses), then the Q lanes of each coordinate are added in lane order
__global__ __launch_bounds__(256) void centre_part(const double* __restrict__ X, int64_t n, int d,
                                                   int64_t chunk, double* __restrict__ part) {
  __shared__ double red[256];
  const int t = threadIdx.x;
  const int Q = 256 / d;
  const int q = t / d, k = t % d;
  const int64_t i0 = (int64_t)blockIdx.x * chunk;
  const int64_t i1 = (i0 + chunk < n) ? i0 + chunk : n;
  double s = 0.0;
  if (q < Q)
    for (int64_t i = i0 + q; i < i1; i += Q) s += X[i * d + k];
  red[t] = s;
  __syncthreads();
  if (t < d) {
    double v = 0.0;
    for (int r = 0; r < Q; ++r) v += red[r * d + t];
    part[(int64_t)blockIdx.x * d + t] = v;
  }
}

__global__ void centre_final(const double* __restrict__ part, int nb, int d, int64_t n,
                             double* __restrict__ c) {
  const int k = threadIdx.x;
  if (k >= d) return;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += part[(int64_t)b * d + k];
  c[k] = s / (double)n;
}

// hi/lo bf16 split of the centred coordinates and FP32 squared norms
__global__ void pack_split(const double* __restrict__ X, int64_t n, int d, int kp,
                           const double* __restrict__ centre, uint16_t* __restrict__ hi,
                           uint16_t* __restrict__ lo) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * kp) return;
  const int64_t i = t / kp;
  const int k = (int)(t % kp);
  double v = 0.0;
  if (k < d) v = X[i * d + k] - (centre ? centre[k] : 0.0);
  const __bf16 h = (__bf16)(float)v;
  const __bf16 l = (__bf16)(float)(v - (double)(float)h);
  hi[t] = __builtin_bit_cast(uint16_t, h);
  lo[t] = __builtin_bit_cast(uint16_t, l);
}

__global__ void pack_norms(const double* __restrict__ X, int64_t n, int d,
                           const double* __restrict__ centre, float* __restrict__ nrm) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int k = 0; k < d; ++k) {
    const double v = X[i * d + k] - (centre ? centre[k] : 0.0);
    s += v * v;
  }
  nrm[i] = (float)s;
}

// V (n x m, strided) -> hi/lo bf16 in the V-reduction MFMA's operand order:
// 32-column groups of 16 rhs x 32 K slots, slot (8g + v) holding column
// slot_col(g, v) of the group; columns c0 .. c0+mc, zero padded to 16 rhs
// and to whole 64-column chunks (npad = 64 ceil(n / 64)).
__global__ void pack_vsplit(VecView V, int64_t n, int64_t npad, int c0, int mc,
                            uint16_t* __restrict__ hi, uint16_t* __restrict__ lo) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= npad * 16) return;
  const int64_t q = t / 512;
  const int r = (int)(t % 512);
  const int c = r / 32, slot = r % 32;
  const int64_t j = q * 32 + slot_col(slot / 8, slot % 8);
  float v = 0.f;
  double vd = 0.0;
  if (j < n && c < mc) {
    vd = V.p[j * V.rs + (int64_t)(c0 + c) * V.cs];
    v = (float)vd;
  }
  const __bf16 h = (__bf16)v;
  const __bf16 l = (__bf16)(float)(vd - (double)(float)h);
  hi[t] = __builtin_bit_cast(uint16_t, h);
  lo[t] = __builtin_bit_cast(uint16_t, l);
}

struct MSplit {
  int nsplit;
  int64_t per;
};

MSplit mfma_split(int64_t nr, int64_t nc) {
  const int64_t ns = split_count(nr, nc, 4 * 16 * kRT, 256);
  int64_t per = ceil_div(std::max<int64_t>(nc, 1), ns);
  per = ceil_div(per, kCols) * kCols;  // whole chunks per split
  return {(int)ns, per};
}

}  // namespace

int carve_mixed(int64_t n, int32_t d, Arena& arena, PointSet* out) {
  const int kp = mfma_kdim(d);
  if (kp > 64) {
    set_error("MIXED Gaussian tiles support d <= 64");
    return KRR_EINVAL;
  }
  out->kpad = kp;
  out->xhi = arena.take<uint16_t>((size_t)n * kp);
  out->xlo = arena.take<uint16_t>((size_t)n * kp);
  out->nrm = arena.take<float>(n);
  out->centre = arena.take<double>(64);
  out->cpart = arena.take<double>(256 * 64);
  return KRR_OK;
}

int compute_centre(const double* X, int64_t n, int32_t d, double* centre, double* part,
                   hipStream_t s) {
  if (n <= 0) return hip_check(hipMemsetAsync(centre, 0, sizeof(double) * d, s), "centre");
  const int nb = (int)std::min<int64_t>(256, n);
  const int64_t chunk = ceil_div(n, nb);
  const int nbe = (int)ceil_div(n, chunk);
  centre_part<<<nbe, 256, 0, s>>>(X, n, d, chunk, part);
  KRR_LAUNCH_CHECK("centre_part");
  centre_final<<<1, 64, 0, s>>>(part, nbe, d, n, centre);
  KRR_LAUNCH_CHECK("centre_final");
  return KRR_OK;
}

int fill_mixed(const double* X, const double* centre, const PointSet& ps, hipStream_t s) {
  const int64_t n = ps.n;
  if (n == 0) return KRR_OK;
  if (!X || !ps.xhi) {
    set_error("fill_mixed: NULL points or layout");
    return KRR_EINVAL;
  }
  if (centre && centre != ps.centre)
    KRR_TRY(hip_check(hipMemcpyAsync(const_cast<double*>(ps.centre), centre, sizeof(double) * ps.d,
                                     hipMemcpyDeviceToDevice, s), "centre copy"));
  if (!centre) KRR_TRY(compute_centre(X, n, ps.d, const_cast<double*>(ps.centre), ps.cpart, s));
  const double* c = ps.centre;
  pack_split<<<(unsigned)ceil_div(n * ps.kpad, 256), 256, 0, s>>>(
      X, n, ps.d, ps.kpad, c, const_cast<uint16_t*>(ps.xhi), const_cast<uint16_t*>(ps.xlo));
  KRR_LAUNCH_CHECK("pack_split");
  pack_norms<<<(unsigned)ceil_div(n, 256), 256, 0, s>>>(X, n, ps.d, c, const_cast<float*>(ps.nrm));
  KRR_LAUNCH_CHECK("pack_norms");
  return KRR_OK;
}

size_t product_mfma_scratch_bytes(int64_t nr, int64_t nc) {
  MSplit sp = mfma_split(nr, nc);
  Arena a;
  const int64_t npad = ceil_div(std::max<int64_t>(nc, 1), kCols) * kCols;
  a.take<uint16_t>((size_t)npad * 16);
  a.take<uint16_t>((size_t)npad * 16);
  a.take<double>((size_t)sp.nsplit * std::max<int64_t>(nr, 1) * 16);
  return a.used;
}

int mfma_prepare(double sigma, const PointSet& rows, const PointSet& cols, VecView V, int c0,
                 int mc, Arena& scratch, MfmaJob* out, hipStream_t s) {
  const int64_t nr = rows.n, nc = cols.n;
  if (rows.kpad != cols.kpad || !rows.xhi || !cols.xhi) {
    set_error("MIXED product: point layouts missing or inconsistent");
    return KRR_EINVAL;
  }
  MSplit sp = mfma_split(nr, nc);
  const int64_t npad = ceil_div(std::max<int64_t>(nc, 1), kCols) * kCols;
  uint16_t* vh = scratch.take<uint16_t>((size_t)npad * 16);
  uint16_t* vl = scratch.take<uint16_t>((size_t)npad * 16);
  double* part = scratch.take<double>((size_t)sp.nsplit * nr * 16);
  if (!scratch.ok()) {
    set_error("MIXED product scratch too small");
    return KRR_EWORKSPACE;
  }
  if (nc > 0) {
    pack_vsplit<<<(unsigned)ceil_div(npad * 16, 256), 256, 0, s>>>(V, nc, npad, c0, mc, vh, vl);
    KRR_LAUNCH_CHECK("pack_vsplit");
  }
  if (!rows.xc32 || !cols.xc32 || rows.dpad != cols.dpad) {
    set_error("MIXED product: FP32 centred layouts missing or inconsistent");
    return KRR_EINVAL;
  }
  MfmaJob& j = *out;
  j.xf = rows.xc32;
  j.yf = cols.xc32;
  j.xmax = rows.xmax32;
  j.ymax = cols.xmax32;
  j.s_nat = (float)(1.0 / (2.0 * sigma * sigma));
  j.dpad = rows.dpad;
  j.xhi = rows.xhi;
  j.xlo = rows.xlo;
  j.xn = rows.nrm;
  j.yhi = cols.xhi;
  j.ylo = cols.xlo;
  j.yn = cols.nrm;
  j.vh = vh;
  j.vl = vl;
  j.part = part;
  j.nr = nr;
  j.nc = nc;
  j.per = sp.per;
  j.item0 = 0;
  j.s = (float)(1.4426950408889634 / (2.0 * sigma * sigma));
  j.nsplit = sp.nsplit;
  j.M = mc;
  j.kp = rows.kpad;
  j.route = 0;
  if (rows.max_host >= 0.0 && cols.max_host >= 0.0)
    j.route = mixed_bound_exceeded(j.s_nat, (float)rows.max_host, (float)cols.max_host, j.kp) ? 2 : 1;
  return KRR_OK;
}

int mfma_launch(const std::vector<MfmaJob>& jobs, hipStream_t s) {
  for (int kp : {32, 64}) {
    std::vector<MfmaJob> sel;
    for (const MfmaJob& j : jobs)
      if (j.kp == kp) sel.push_back(j);
    for (size_t j0 = 0; j0 < sel.size(); j0 += kMaxMJobs) {
      MJobTable tab{};
      int64_t total = 0;
      int nj = 0;
      for (size_t j = j0; j < sel.size() && nj < kMaxMJobs; ++j, ++nj) {
        tab.job[nj] = sel[j];
        tab.job[nj].item0 = total;
        total += ceil_div(sel[j].nr, (int64_t)4 * 16 * kRT) * sel[j].nsplit;
      }
      tab.njobs = nj;
      tab.total = total;
      if (total == 0) continue;
      const unsigned grid = (unsigned)std::min<int64_t>(xcd_slots(total), kGridCap);
      bool any_mfma = false;
      for (int q = 0; q < nj; ++q) any_mfma = any_mfma || tab.job[q].route != 2;
      void* tok = tile_timer_start(s);
      if (any_mfma) {
        if (kp == 32) tile_mfma_gauss<32><<<grid, 256, 0, s>>>(tab);
        else tile_mfma_gauss<64><<<grid, 256, 0, s>>>(tab);
        KRR_LAUNCH_CHECK("tile_mfma_gauss");
      }
      // the direct tile serves the jobs the guard refused (decided on the
      // device, so the launch stays asynchronous); one launch per padded
      // dimension present
      int dseen[kMaxMJobs], nd = 0;
      for (int q = 0; q < nj; ++q) {
        if (tab.job[q].route == 1) continue;  // known to stay on the expansion tile
        bool seen = false;
        for (int u = 0; u < nd; ++u) seen = seen || dseen[u] == tab.job[q].dpad;
        if (!seen) dseen[nd++] = tab.job[q].dpad;
      }
      for (int u = 0; u < nd; ++u) {
        switch (dseen[u]) {
          case 4: tile_mixed_direct<4><<<grid, 256, 0, s>>>(tab); break;
          case 8: tile_mixed_direct<8><<<grid, 256, 0, s>>>(tab); break;
          case 16: tile_mixed_direct<16><<<grid, 256, 0, s>>>(tab); break;
          case 20: tile_mixed_direct<20><<<grid, 256, 0, s>>>(tab); break;
          case 24: tile_mixed_direct<24><<<grid, 256, 0, s>>>(tab); break;
          case 32: tile_mixed_direct<32><<<grid, 256, 0, s>>>(tab); break;
          case 48: tile_mixed_direct<48><<<grid, 256, 0, s>>>(tab); break;
          default: tile_mixed_direct<64><<<grid, 256, 0, s>>>(tab); break;
        }
        KRR_LAUNCH_CHECK("tile_mixed_direct");
      }
      tile_timer_stop(tok, s);
    }
  }
  return KRR_OK;
}

}  // namespace krr
