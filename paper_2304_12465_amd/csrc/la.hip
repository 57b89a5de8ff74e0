// FP64 dense linear algebra for the build steps of the method: the Woodbury
// core F^T F + mu I (Alg. 1 preconditioner), its Cholesky factor, the KRILL
// matrix B^T B + H and its Cholesky factor (Alg. 2), and the triangular
// solves that apply them.  GEMM runs on the FP64 matrix cores.
#include "la.h"
#include <algorithm>
#include <vector>

namespace krr {

namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kKStep = 16;          // K slice staged in LDS per iteration
constexpr int kPad = kKStep + 1;    // LDS row pitch in doubles
constexpr int kUE = kKStep / 4;     // entries per thread and operand per 64 tile rows

// v_mfma_f64_16x16x4f64 operand layout (wave64):
//   A (16 x 4): lane l holds A[l % 16][l / 16]
//   B (4 x 16): lane l holds B[l / 16][l % 16]
//   D (16 x 16): lane l, element t holds D[4 t + l / 16][l % 16]
//
// Output tiles in the order the workgroups take them: column by column
// (all row tiles of one column tile together), or, for the lower triangle
// of a square product, row by row over the tiles on or below the diagonal.
// Consecutive workgroups go to the eight XCDs in turn (workgroup L to XCD
// L mod 8), so each XCD is given a contiguous run of that order: tiles that
// read the same operand slab then share one L2.
__host__ __device__ inline int64_t tile_count(int64_t gx, int64_t gy, int lower) {
  return lower ? gy * (gy + 1) / 2 : gx * gy;
}
__device__ inline bool tile_of(int64_t L, int64_t gx, int64_t gy, int lower, int64_t& ty,
                               int64_t& tx) {
  const int64_t T = tile_count(gx, gy, lower);
  const int64_t per = (T + 7) / 8;
  const int64_t t = (L % 8) * per + L / 8;
  if (t >= T) return false;
  if (lower) {
    int64_t y = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
    while (y * (y + 1) / 2 > t) --y;
    while ((y + 1) * (y + 2) / 2 <= t) ++y;
    ty = y;
    tx = t - y * (y + 1) / 2;
  } else {
    tx = t / gy;
    ty = t % gy;
  }
  return true;
}

// C = alpha op(A) op(B) + beta C on a TM x TN output tile per workgroup
// (TM, TN in {64, 128}); the four waves split it 2 x 2, each wave holding
// (TM / 32) x (TN / 32) MFMA accumulators.  A 128 x 128 tile does twice
// the MFMA work of a 64 x 64 tile per byte staged, which the FP64 matrix
// rate needs when the operands stream from memory.
template <bool AT, bool BT, int TM, int TN>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(TM * TN > 64 * 64 ? 2 : 4)))
void gemm_f64_kernel(int64_t M, int64_t N, int64_t K, double alpha, const double* __restrict__ A,
                     int64_t lda, const double* __restrict__ B, int64_t ldb, double beta,
                     double* __restrict__ C, int64_t ldc, int64_t kchunk,
                     double* __restrict__ slots, int lower) {
  constexpr int FM = TM / 32, FN = TN / 32;  // MFMA blocks per wave
  constexpr int RA = TM / 64, RB = TN / 64;  // 64-row loader passes
  // two LDS buffers: the next K step is stored into one while the MFMAs read
  // the other, so each step needs one barrier
  __shared__ double As[2][TM][kPad];  // [buffer][m][k]
  __shared__ double Bs[2][TN][kPad];  // [buffer][n][k]
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  int64_t ty, tx;
  if (!tile_of(blockIdx.x, (N + TN - 1) / TN, (M + TM - 1) / TM, lower, ty, tx)) return;
  const int64_t m0 = ty * TM, n0 = tx * TN;
  const int wm = (wave >> 1) * (TM / 2), wn = (wave & 1) * (TN / 2);
  f64x4 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};

  // Tile loaders: per K step every thread fetches kKStep / 4 entries of A per
  // 64 tile rows, and the same of B, all in flight at once; the next step's
  // loads are issued before this step's MFMAs.  A row-major operand reads
  // through per-thread row pointers clamped to the last row (the values of
  // rows past the end are replaced by zero), so every step but the last
  // needs no per-element checks; a K-major operand takes that path when its
  // whole tile is in range.  The last step of a K range, and K-major tiles
  // at the edge, clamp every address instead.
  // row-major operand: 64 rows x kKStep k, kUE consecutive k per thread;
  // K-major operand: lane l of wave w takes row l at k = kUE w .. kUE w + kUE
  // - 1, so each load instruction reads 64 consecutive values and each LDS
  // store writes 64 consecutive rows of one k (consecutive banks; the
  // transposing store of kUE rows per thread hit every fourth bank)
  const int ar = tid >> 2, ak = (tid & 3) * kUE;
  const int km = tid & 63, kq = (tid >> 6) * kUE;
  // split K: this workgroup covers [kb, ke); the bounds checks below use ke
  const int64_t kb = (int64_t)blockIdx.z * kchunk;
  const int64_t ke = (kb + kchunk < K) ? kb + kchunk : K;
  const double* arow[RA];
  bool aok[RA];
#pragma unroll
  for (int r = 0; r < RA; ++r) {
    const int64_t gm = m0 + 64 * r + ar;
    aok[r] = gm < M;
    arow[r] = A + (aok[r] ? gm : M - 1) * lda;
  }
  const double* brow[RB];
  bool bok[RB];
#pragma unroll
  for (int r = 0; r < RB; ++r) {
    const int64_t gn = n0 + 64 * r + ar;
    bok[r] = gn < N;
    brow[r] = B + (bok[r] ? gn : N - 1) * ldb;
  }
  const bool afull = !AT || m0 + TM <= M, bfull = BT || n0 + TN <= N;
  // raw loaded values; the zero mask (bit 4 r + u, A in the low half, B in
  // the high half) is applied only when they are stored to LDS, so nothing
  // waits on the loads before the MFMAs of the current step
  double ra[RA][kUE], rb[RB][kUE];
  uint32_t okm = 0;
  auto fetch = [&](int64_t k0) {
    okm = 0;
    if (k0 + kKStep <= ke && afull && bfull) {
#pragma unroll
      for (int r = 0; r < RA; ++r)
#pragma unroll
        for (int u = 0; u < kUE; ++u) {
          if (!AT) {
            ra[r][u] = arow[r][k0 + ak + u];
            okm |= (aok[r] ? 1u : 0u) << (kUE * r + u);
          } else {
            ra[r][u] = A[(k0 + kq + u) * lda + m0 + 64 * r + km];
            okm |= 1u << (kUE * r + u);
          }
        }
#pragma unroll
      for (int r = 0; r < RB; ++r)
#pragma unroll
        for (int u = 0; u < kUE; ++u) {
          if (BT) {
            rb[r][u] = brow[r][k0 + ak + u];
            okm |= (bok[r] ? 1u : 0u) << (16 + kUE * r + u);
          } else {
            rb[r][u] = B[(k0 + kq + u) * ldb + n0 + 64 * r + km];
            okm |= 1u << (16 + kUE * r + u);
          }
        }
      return;
    }
    // past the end of the range (the last prefetch) every k reads ke - 1
#pragma unroll
    for (int r = 0; r < RA; ++r)
#pragma unroll
      for (int u = 0; u < kUE; ++u) {
        int64_t gm, gk;
        if (!AT) {
          gm = m0 + 64 * r + ar;
          gk = k0 + ak + u;
        } else {
          gm = m0 + 64 * r + km;
          gk = k0 + kq + u;
        }
        const bool ok = gm < M && gk < ke;
        const int64_t cm = gm < M ? gm : M - 1, ck = gk < ke ? gk : ke - 1;
        ra[r][u] = AT ? A[ck * lda + cm] : A[cm * lda + ck];
        okm |= (ok ? 1u : 0u) << (kUE * r + u);
      }
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
      for (int u = 0; u < kUE; ++u) {
        int64_t gn, gk;
        if (BT) {
          gn = n0 + 64 * r + ar;
          gk = k0 + ak + u;
        } else {
          gn = n0 + 64 * r + km;
          gk = k0 + kq + u;
        }
        const bool ok = gn < N && gk < ke;
        const int64_t cn = gn < N ? gn : N - 1, ck = gk < ke ? gk : ke - 1;
        rb[r][u] = BT ? B[cn * ldb + ck] : B[ck * ldb + cn];
        okm |= (ok ? 1u : 0u) << (16 + kUE * r + u);
      }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int r = 0; r < RA; ++r)
#pragma unroll
      for (int u = 0; u < kUE; ++u) {
        const double v = (okm >> (kUE * r + u)) & 1u ? ra[r][u] : 0.0;
        if (!AT)
          As[buf][64 * r + ar][ak + u] = v;
        else
          As[buf][64 * r + km][kq + u] = v;
      }
#pragma unroll
    for (int r = 0; r < RB; ++r)
#pragma unroll
      for (int u = 0; u < kUE; ++u) {
        const double v = (okm >> (16 + kUE * r + u)) & 1u ? rb[r][u] : 0.0;
        if (BT)
          Bs[buf][64 * r + ar][ak + u] = v;
        else
          Bs[buf][64 * r + km][kq + u] = v;
      }
  };
  int cur = 0;
  if (kb < ke) {
    fetch(kb);
    store(0);
    __syncthreads();
    fetch(kb + kKStep);  // clamped addresses: harmless past the end
  }
  for (int64_t k0 = kb; k0 < ke; k0 += kKStep) {
#pragma unroll
    for (int ks = 0; ks < kKStep; ks += 4) {
      double a[FM], b[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) a[i] = As[cur][wm + i * 16 + (lane & 15)][ks + (lane >> 4)];
#pragma unroll
      for (int j = 0; j < FN; ++j) b[j] = Bs[cur][wn + j * 16 + (lane & 15)][ks + (lane >> 4)];
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    // the other buffer was last read before the previous barrier
    if (k0 + kKStep < ke) {
      store(cur ^ 1);
      fetch(k0 + 2 * kKStep);
    }
    __syncthreads();
    cur ^= 1;
  }
  // epilogue, one block row at a time: the old values of C are fetched
  // together (clamped addresses) before any store
  const bool use_c = !slots && beta != 0.0;
#pragma unroll
  for (int i = 0; i < FM; ++i) {
    double old[FN][4] = {};
    if (use_c) {
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int64_t gm = m0 + wm + i * 16 + 4 * t + (lane >> 4);
          const int64_t gn = n0 + wn + j * 16 + (lane & 15);
          const int64_t cm = gm < M ? gm : M - 1, cn = gn < N ? gn : N - 1;
          old[j][t] = C[cm * ldc + cn];
        }
    }
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int64_t gm = m0 + wm + i * 16 + 4 * t + (lane >> 4);
        const int64_t gn = n0 + wn + j * 16 + (lane & 15);
        if (gm < M && gn < N) {
          double v = alpha * acc[i][j][t];
          if (slots) {
            slots[((int64_t)blockIdx.z * M + gm) * N + gn] = v;
          } else {
            if (use_c) v += beta * old[j][t];
            C[gm * ldc + gn] = v;
          }
        }
      }
  }
}

// C = sum_z slots[z] (fixed order) + beta C; with `lower`, only the square
// tiles (tile x tile) on or below the diagonal, as the GEMM wrote them
__global__ __launch_bounds__(256) void splitk_reduce(const double* __restrict__ slots, int nz,
                                                     int64_t M, int64_t N, double beta,
                                                     double* __restrict__ C, int64_t ldc,
                                                     int lower, int tile) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= M * N) return;
  const int64_t m = t / N, n = t % N;
  if (lower && n / tile > m / tile) return;  // tile skipped by the GEMM
  double v = 0.0;
  for (int z = 0; z < nz; ++z) v += slots[((int64_t)z * M + m) * N + n];
  if (beta != 0.0) v += beta * C[m * ldc + n];
  C[m * ldc + n] = v;
}

// Output tile shape: 128 x 128 for large products, 128 x 64 when all of a
// short M (65 .. 128 rows) fits one tile row over many columns (each
// column block of B is then read once), else 64 x 64.
struct TileShape {
  int tm, tn;
};
TileShape choose_tile(int64_t M, int64_t N, int64_t K, bool lower) {
  if (M >= 2048 && N >= 2048 && K >= 1024) return {128, 128};
  if (!lower && M > 64 && M <= 128 && N >= 8192) return {128, 64};
  return {64, 64};
}

// K split for outputs with few tiles and a long K: as many K slices as fit
// one full round of resident workgroups on every XCD (each XCD takes a
// contiguous run of ceil(tiles / 8) tiles per slice; a CU holds four 64 x 64
// or two larger tiles), so no second, mostly idle round follows.
int choose_ksplit(int64_t M, int64_t N, int64_t K, bool lower) {
  const TileShape ts = choose_tile(M, N, K, lower);
  const int64_t gx = ceil_div(N, ts.tn), gy = ceil_div(M, ts.tm);
  const int64_t per_xcd = ceil_div(tile_count(gx, gy, lower ? 1 : 0), 8);
  const int64_t slots = 32 * (ts.tm == 64 ? 4 : 2);  // per XCD
  if (per_xcd >= slots / 2 || K < 8192) return 1;
  int64_t z = slots / per_xcd;
  z = std::min<int64_t>(z, K / 2048);
  return (int)std::max<int64_t>(1, std::min<int64_t>(z, 4096));
}

template <bool AT, bool BT>
void launch_gemm(TileShape ts, dim3 grid, hipStream_t s, int64_t M, int64_t N, int64_t K,
                 double alpha, const double* A, int64_t lda, const double* B, int64_t ldb,
                 double beta, double* C, int64_t ldc, int64_t kchunk, double* slots, int lower) {
  if (ts.tm == 128 && ts.tn == 128)
    gemm_f64_kernel<AT, BT, 128, 128><<<grid, 256, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta,
                                                            C, ldc, kchunk, slots, lower);
  else if (ts.tm == 128)
    gemm_f64_kernel<AT, BT, 128, 64><<<grid, 256, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C,
                                                           ldc, kchunk, slots, lower);
  else
    gemm_f64_kernel<AT, BT, 64, 64><<<grid, 256, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C,
                                                          ldc, kchunk, slots, lower);
}

constexpr int kNb = 64;  // block size of the blocked factorisation and solves

// Cholesky of one nb x nb diagonal block (nb <= kNb), right-looking, one
// quad of lanes per row (256 threads): lane c of row i keeps entries
// j = 4 u + c (u < kNb / 4) in registers (the loops are unrolled, so every
// index is a constant).  Step k: every lane forms y = 1 / sqrt(p) of the
// pivot p (passed through LDS), the lane holding entry (i, k) stores the
// multiplier l_i = A(i, k) y into LDS, and after the barrier every lane
// updates its entries j > k by A(i, j) -= l_i l_j; the lane holding (k + 1,
// k + 1) then passes the next pivot.  Each entry takes the same multiply-adds
// in the same order as with one lane per row, at a quarter of the
// multiply-adds per lane per step.  Whole rows are read and written: the
// entries above the diagonal start with whatever A holds there and collect
// values of no meaning, but no entry on or below the diagonal ever reads one
// (entry (i, j), j <= i, takes the multipliers of columns k < j from rows i
// and j).  Rows and columns past nb stay zero and take pivot 1.  A
// non-positive pivot is replaced by 1 so the sweep stays finite; `info`
// reports the first one.
__global__ __launch_bounds__(256) void potrf_diag(double* __restrict__ A, int64_t lda, int nb,
                                                  int64_t col0, int* __restrict__ info) {
  constexpr int kU = kNb / 4;
  __shared__ double colv[kNb];
  __shared__ double piv;
  const int i = threadIdx.x >> 2, c = threadIdx.x & 3;
  const bool row = i < nb;
  double t[kU];
#pragma unroll
  for (int u = 0; u < kU; ++u) t[u] = (row && 4 * u + c < nb) ? A[i * lda + 4 * u + c] : 0.0;
  if (threadIdx.x == 0) piv = t[0];
  __syncthreads();
  int bad = 0;
#pragma unroll
  for (int k = 0; k < kNb; ++k) {
    __builtin_amdgcn_sched_barrier(0);  // one column at a time: bounds the live LDS reads
    const double p = piv;
    // y = 1 / sqrt(p): v_rsq_f64 and two Newton steps (each doubles the
    // correct bits), so the column takes one multiply instead of a square
    // root and a division on the step's dependent chain; row k gets p y =
    // sqrt(p) to within an ulp or two.  Pivots below 2^-960 (none in a
    // well-posed factor) take the square root.
    double y = 1.0;
    if (k < nb) {
      if (p >= 0x1p-960) {
        y = __builtin_amdgcn_rsq(p);
        const double h = 0.5 * p;
        y = __builtin_fma(y, __builtin_fma(-h * y, y, 0.5), y);
        y = __builtin_fma(y, __builtin_fma(-h * y, y, 0.5), y);
      } else if (p > 0.0) {
        y = 1.0 / sqrt(p);
      } else if (!bad) {
        bad = (int)(col0 + k + 1);
      }
    }
    if (c == (k & 3)) {
      const double l = t[k >> 2] * y;
      t[k >> 2] = l;
      colv[i] = l;
    }
    __syncthreads();
    const double li = colv[i];
#pragma unroll
    for (int u = k >> 2; u < kU; ++u)
      if (4 * u + c > k) t[u] = __builtin_fma(-li, colv[4 * u + c], t[u]);
    if (k + 1 < kNb && i == k + 1 && c == ((k + 1) & 3)) piv = t[(k + 1) >> 2];
    __syncthreads();
  }
  if (row) {
#pragma unroll
    for (int u = 0; u < kU; ++u)
      if (4 * u + c < nb) A[i * lda + 4 * u + c] = t[u];
  }
  if (threadIdx.x == 0 && bad && *info == 0) *info = bad;
}

// A lower-triangular nb x nb block (nb <= kNb) staged in LDS, padded to
// kNb x kNb with the identity, plus the reciprocals of its diagonal.
__device__ __forceinline__ void stage_tri(const double* __restrict__ L, int64_t lda, int nb,
                                          double (*T)[kNb + 1], double* tinv) {
  const int tid = threadIdx.x;
  for (int e = tid; e < kNb * kNb; e += blockDim.x) {
    const int q = e / kNb, p = e % kNb;
    T[q][p] = (q < nb && p < nb) ? L[q * lda + p] : (q == p ? 1.0 : 0.0);
  }
  __syncthreads();
  if (tid < kNb) tinv[tid] = 1.0 / T[tid][tid];
  __syncthreads();
}

// x <- T^{-1} x by forward substitution, four lanes per vector: lane c of a
// quad (c = lane & 3) holds entries 4 i + c in x[i] (fully unrolled, so x
// stays in registers).  For each row q every lane sums the terms of its own
// entries below q, the quad adds the four sums (two lane exchanges; IEEE
// addition is commutative, so all four lanes get the same bits), and the
// lane that owns entry q keeps its solved value.  Against one lane per
// vector this takes a quarter of the FMAs and LDS reads per lane at the same
// dependent depth: the 64-wide panel solve 38-40 -> 19-21 us.
__device__ __forceinline__ void tri_forward4(const double (*T)[kNb + 1], const double* tinv,
                                             double (&x)[kNb / 4], int c) {
  const int base = (int)(threadIdx.x & 63) & ~3;
#pragma unroll
  for (int q = 0; q < kNb; ++q) {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < kNb / 4; ++i)
      if (4 * i + c < q) s = __builtin_fma(T[q][4 * i + c], x[i], s);
    s += __shfl_xor(s, 1);
    s += __shfl_xor(s, 2);
    const double orig = __shfl(x[q >> 2], base | (q & 3));
    const double xq = (orig - s) * tinv[q];
    if ((q & 3) == c) x[q >> 2] = xq;
  }
}

// The quad's entries of one vector of nb <= kNb entries at stride `stride`:
// entries q >= nb alias entry nb - 1 (loaded, solved against the identity
// padding, never stored and never affecting entries < nb).
__device__ __forceinline__ void load_quad(const double* __restrict__ base, int64_t stride, int nb,
                                          int c, double (&x)[kNb / 4]) {
#pragma unroll
  for (int i = 0; i < kNb / 4; ++i) {
    const int q = 4 * i + c;
    x[i] = base[(int64_t)(q < nb ? q : nb - 1) * stride];
  }
}
__device__ __forceinline__ void store_quad(double* __restrict__ base, int64_t stride, int nb,
                                           int c, const double (&x)[kNb / 4]) {
#pragma unroll
  for (int i = 0; i < kNb / 4; ++i) {
    const int q = 4 * i + c;
    if (q < nb) base[(int64_t)q * stride] = x[i];
  }
}

// X <- X L^{-T} for X (nrows x nb, ld ldx) and an nb x nb (nb <= kNb) lower
// factor L, one quad per row (the row solve is a forward substitution with
// L), 64 rows per workgroup.  In the factorisation X is the panel below the
// diagonal block.
__global__ __launch_bounds__(256) void potrf_panel(const double* __restrict__ L, int64_t lda,
                                                   int nb, double* __restrict__ X, int64_t ldx,
                                                   int64_t nrows) {
  __shared__ double T[kNb][kNb + 1];
  __shared__ double tinv[kNb];
  stage_tri(L, lda, nb, T, tinv);
  const int c = threadIdx.x & 3;
  const int64_t r = (int64_t)blockIdx.x * (blockDim.x / 4) + (threadIdx.x >> 2);
  // quads past the end solve the last row again and store nothing (every
  // lane takes part in the quad exchanges)
  double* row = X + (r < nrows ? r : nrows - 1) * ldx;
  double x[kNb / 4];
  load_quad(row, 1, nb, c, x);
  tri_forward4(T, tinv, x, c);
  if (r < nrows) store_quad(row, 1, nb, c, x);
}

// One block of a lower-triangular solve with many right-hand sides:
// B_blk <- L_blk^{-1} B_blk, one quad per right-hand-side column, 64
// columns per workgroup.
__global__ __launch_bounds__(256) void trsm_diag(const double* __restrict__ L, int64_t lda, int nb,
                                                 double* __restrict__ B, int64_t ldb,
                                                 int64_t ncols) {
  __shared__ double T[kNb][kNb + 1];
  __shared__ double tinv[kNb];
  stage_tri(L, lda, nb, T, tinv);
  const int c = threadIdx.x & 3;
  const int64_t col = (int64_t)blockIdx.x * (blockDim.x / 4) + (threadIdx.x >> 2);
  double* base = B + (col < ncols ? col : ncols - 1);
  double x[kNb / 4];
  load_quad(base, ldb, nb, c, x);
  tri_forward4(T, tinv, x, c);
  if (col < ncols) store_quad(base, ldb, nb, c, x);
}

// C[M x N] = alpha A B^T + beta C for M <= MM rows of A (row-major M x K)
// and B given as N x K rows: each output is a dot product of two contiguous
// rows.  One workgroup per output column streams row j of B (coalesced)
// against the M rows of A (L2-resident); lanes, then the four waves, are
// added in a fixed order, so the result is reproducible.  Used by the
// preconditioner applies, whose first product has one row per right-hand
// side.
template <int MM>
__global__ __launch_bounds__(256) void gemm_rowdot(int64_t M, int64_t N, int64_t K, double alpha,
                                                   const double* __restrict__ A, int64_t lda,
                                                   const double* __restrict__ B, int64_t ldb,
                                                   double beta, double* __restrict__ C,
                                                   int64_t ldc) {
  __shared__ double red[4][MM];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t j = blockIdx.x;
  double acc[MM];
#pragma unroll
  for (int c = 0; c < MM; ++c) acc[c] = 0.0;
  const double* __restrict__ b = B + j * ldb;
  for (int64_t k = tid; k < K; k += 256) {
    const double bv = b[k];
#pragma unroll
    for (int c = 0; c < MM; ++c)
      if (c < M) acc[c] = __builtin_fma(A[c * lda + k], bv, acc[c]);
  }
#pragma unroll
  for (int c = 0; c < MM; ++c) {
    double v = acc[c];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (lane == 0) red[wave][c] = v;
  }
  __syncthreads();
  if (tid < MM && tid < M) {
    const int c = tid;
    const double v = (red[0][c] + red[1][c]) + (red[2][c] + red[3][c]);
    const double old = beta != 0.0 ? beta * C[c * ldc + j] : 0.0;
    C[c * ldc + j] = alpha * v + old;
  }
}

// C[M x N] = alpha A B + beta C for M <= MM rows of A (row-major M x K) and
// B row-major K x N: a workgroup owns 64 output columns; its four waves take
// the k = w mod 4 rows of B (each load of a wave reads 64 consecutive
// columns) and their partial sums are added in wave order through LDS.
// Used for the second product of each preconditioner apply on large
// problems (one row per right-hand side, B = Q^T).
template <int MM>
__global__ __launch_bounds__(256) void gemm_colsum(int64_t M, int64_t N, int64_t K, double alpha,
                                                   const double* __restrict__ A, int64_t lda,
                                                   const double* __restrict__ B, int64_t ldb,
                                                   double beta, double* C, int64_t ldc,
                                                   const double* Cin) {
  __shared__ double red[4][MM][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t j = (int64_t)blockIdx.x * 64 + lane;
  const int64_t jj = j < N ? j : N - 1;
  double acc[MM];
#pragma unroll
  for (int c = 0; c < MM; ++c) acc[c] = 0.0;
#pragma unroll 4
  for (int64_t k = wave; k < K; k += 4) {
    const double bv = B[k * ldb + jj];
#pragma unroll
    for (int c = 0; c < MM; ++c)
      if (c < M) acc[c] = __builtin_fma(A[c * lda + k], bv, acc[c]);
  }
#pragma unroll
  for (int c = 0; c < MM; ++c) red[wave][c][lane] = acc[c];
  __syncthreads();
  if (wave == 0 && j < N) {
#pragma unroll
    for (int c = 0; c < MM; ++c)
      if (c < M) {
        const double v = (red[0][c][lane] + red[1][c][lane]) + (red[2][c][lane] + red[3][c][lane]);
        const double old = beta != 0.0 ? beta * Cin[c * ldc + j] : 0.0;
        C[c * ldc + j] = alpha * v + old;
      }
  }
}

// Products of at most 8 rows against a long dimension (the preconditioner
// applies of large full-data problems: the point count N runs to millions,
// the rank to thousands), on the FP64 matrix cores.  The A operand's 16 MFMA
// rows hold the (zero-padded) right-hand sides; each 16-index step of the
// contraction is four k-steps whose slot g takes the indices 4g + s
// (s = 0..3), so each lane reads 32 contiguous bytes per operand row.  Both
// are HBM-bound: the MFMA work (16 rows for at most 8 used) stays below the
// time of the streamed operand.
typedef double d4u __attribute__((ext_vector_type(4), aligned(8)));
constexpr int64_t kLongK = 65536;  // contraction length from which long_nt_partial runs
constexpr int64_t kLongN = 65536;  // output width from which long_nn runs
constexpr int kLongTiles = 4;                      // 16-column output tiles per wave
constexpr int kLongCols = 4 * kLongTiles * 16;     // output columns per workgroup

__device__ __forceinline__ d4u load4(const double* p, bool ok) {
  if (ok) return *reinterpret_cast<const d4u*>(p);
  return d4u{0.0, 0.0, 0.0, 0.0};
}

// part[z][c][j] = sum over k in [z kc, min(K, (z + 1) kc)) of A[c][k] B[j][k]
// for c < M <= 8, j < N (A row-major M x K, B given as N rows of K).  A wave
// owns 64 output columns; the workgroup's four waves share the K chunk, so
// the chunk of A is read from L2 once per workgroup and B once overall.
__global__ __launch_bounds__(256) void long_nt_partial(int M, int64_t N, int64_t K,
                                                       const double* __restrict__ A, int64_t lda,
                                                       const double* __restrict__ B, int64_t ldb,
                                                       int64_t kc, double* __restrict__ part) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, li = lane & 15;
  const int64_t j0 = ((int64_t)blockIdx.x * 4 + wave) * (16 * kLongTiles);
  if (j0 >= N) return;
  const int64_t z = blockIdx.y;
  const int64_t kb = z * kc, ke = std::min<int64_t>(K, kb + kc);
  const bool arow = li < M;
  const double* ap = A + (arow ? (int64_t)li : 0) * lda;
  const double* bp[kLongTiles];
  bool bok[kLongTiles];
#pragma unroll
  for (int t = 0; t < kLongTiles; ++t) {
    const int64_t j = j0 + 16 * t + li;
    bok[t] = j < N;
    bp[t] = B + (bok[t] ? j : 0) * ldb;
  }
  f64x4 acc[kLongTiles];
#pragma unroll
  for (int t = 0; t < kLongTiles; ++t) acc[t] = f64x4{0.0, 0.0, 0.0, 0.0};
  int64_t k = kb;
#pragma unroll 2
  for (; k + 16 <= ke; k += 16) {
    const int64_t o = k + 4 * g;
    const d4u a = load4(ap + o, arow);
    d4u b[kLongTiles];
#pragma unroll
    for (int t = 0; t < kLongTiles; ++t) b[t] = load4(bp[t] + o, bok[t]);
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int t = 0; t < kLongTiles; ++t)
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q], b[t][q], acc[t], 0, 0, 0);
  }
  if (k < ke) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t i = k + 4 * g + q;
      const bool in = i < ke;
      const double a = (arow && in) ? ap[i] : 0.0;
#pragma unroll
      for (int t = 0; t < kLongTiles; ++t) {
        const double b = (bok[t] && in) ? bp[t][i] : 0.0;
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[t], 0, 0, 0);
      }
    }
  }
  // element r of acc[t] is D[4 r + g][li]: right-hand side 4 r + g, column
  // j0 + 16 t + li
  double* out = part + z * (int64_t)M * N;
#pragma unroll
  for (int t = 0; t < kLongTiles; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int c = 4 * r + g;
      const int64_t j = j0 + 16 * t + li;
      if (c < M && j < N) out[(int64_t)c * N + j] = acc[t][r];
    }
}

// C[c][j] = alpha * sum_z part[z][c][j] + beta C[c][j]: a workgroup takes 64
// outputs, wave w adds the chunks of its quarter in increasing order, and
// the quarters are added in wave order (fixed order: reproducible).
__global__ __launch_bounds__(256) void long_nt_reduce(int M, int64_t N, int Z,
                                                      const double* __restrict__ part,
                                                      double alpha, double beta, double* C,
                                                      int64_t ldc) {
  __shared__ double red[4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t MN = (int64_t)M * N;
  const int64_t i = (int64_t)blockIdx.x * 64 + lane;
  const int64_t ii = i < MN ? i : MN - 1;
  const int zq = (Z + 3) / 4;
  const int zb = wave * zq, ze = std::min(Z, zb + zq);
  double v = 0.0;
#pragma unroll 8
  for (int z = zb; z < ze; ++z) v += part[(int64_t)z * MN + ii];
  red[wave][lane] = v;
  __syncthreads();
  if (wave == 0 && i < MN) {
    const int64_t c = i / N, j = i - c * N;
    const double sum = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
    const double old = beta != 0.0 ? beta * C[c * ldc + j] : 0.0;
    C[c * ldc + j] = alpha * sum + old;
  }
}

// C[c][n] = alpha sum_k A[c][k] B[k][n] + beta Cin[c][n] for c < M <= 8 (A
// row-major M x K, B row-major K x N).  A workgroup owns 64 output columns
// as four tiles: lane li of tile t stands for column n0 + 4 li + t, so one
// 32-byte load per lane and row of B feeds all four tiles and the lane's
// outputs for one right-hand side are four adjacent columns (one 32-byte
// store).  The four waves take the 16-row steps of K in turn (wave w: steps
// w, w + 4, ...); wave 0 adds the others' sums in wave order (fixed order).
__global__ __launch_bounds__(256) void long_nn(int M, int64_t N, int64_t K, double alpha,
                                               const double* __restrict__ A, int64_t lda,
                                               const double* __restrict__ B, int64_t ldb,
                                               double beta, const double* Cin, double* C,
                                               int64_t ldc) {
  // waves 1..3: element r < 2 of each tile (right-hand sides 4 r + g < 8)
  __shared__ double red[3][2][4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, li = lane & 15;
  const int64_t n0 = (int64_t)blockIdx.x * 64;
  const int64_t nc = n0 + 4 * li;
  const bool full = n0 + 64 <= N;
  const bool arow = li < M;
  const double* ap = A + (arow ? (int64_t)li : 0) * lda;
  f64x4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = f64x4{0.0, 0.0, 0.0, 0.0};
  const int64_t kfull = full ? K / 16 * 16 : 0;  // steps read with 32-byte loads
  int64_t k = 16 * (int64_t)wave;
#pragma unroll 2
  for (; k < kfull; k += 64) {
    const d4u a = load4(ap + k + 4 * g, arow);
    d4u b[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) b[q] = load4(B + (k + 4 * g + q) * ldb + nc, true);
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int t = 0; t < 4; ++t)
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q], b[q][t], acc[t], 0, 0, 0);
  }
  // the K tail, and every step of a workgroup whose columns run past N
  for (; k < K; k += 64) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t row = k + 4 * g + q;
      const bool in = row < K;
      const double a = (arow && in) ? ap[row] : 0.0;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const double b = (in && nc + t < N) ? B[row * ldb + nc + t] : 0.0;
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[t], 0, 0, 0);
      }
    }
  }
  if (wave > 0) {
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int t = 0; t < 4; ++t) red[wave - 1][r][t][lane] = acc[t][r];
  }
  __syncthreads();
  if (wave > 0) return;
  // element r of acc[t] is D[4 r + g][li]: right-hand side 4 r + g, column nc + t
#pragma unroll
  for (int r = 0; r < 2; ++r) {
    const int c = 4 * r + g;
    if (c >= M) continue;
    double v[4];
#pragma unroll
    for (int t = 0; t < 4; ++t)
      v[t] = alpha * (((acc[t][r] + red[0][r][t][lane]) + red[1][r][t][lane]) + red[2][r][t][lane]);
    double* out = C + (int64_t)c * ldc + nc;
    const double* in = Cin + (int64_t)c * ldc + nc;
    if (full) {
      d4u w{v[0], v[1], v[2], v[3]};
      if (beta != 0.0) w += beta * *reinterpret_cast<const d4u*>(in);
      *reinterpret_cast<d4u*>(out) = w;
    } else {
#pragma unroll
      for (int t = 0; t < 4; ++t)
        if (nc + t < N) out[t] = v[t] + (beta != 0.0 ? beta * in[t] : 0.0);
    }
  }
}

// chunks of the long contraction for long_nt_partial: about 1024
// workgroups, chunks of at least 512 indices, at most 256 of them
int long_nt_chunks(int64_t N, int64_t K) {
  const int64_t gx = ceil_div(N, kLongCols);
  int64_t z = std::max<int64_t>(1, 1024 / gx);
  z = std::min<int64_t>(z, std::max<int64_t>(1, K / 512));
  return (int)std::min<int64_t>(z, 256);
}

int launch_long_nt(int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda,
                   const double* B, int64_t ldb, double beta, double* C, int64_t ldc,
                   double* part, int Z, hipStream_t s) {
  const int64_t kc = ceil_div(ceil_div(K, Z), 16) * 16;
  const int z = (int)ceil_div(K, kc);
  long_nt_partial<<<dim3((unsigned)ceil_div(N, kLongCols), (unsigned)z), 256, 0, s>>>(
      (int)M, N, K, A, lda, B, ldb, kc, part);
  KRR_LAUNCH_CHECK("long_nt_partial");
  long_nt_reduce<<<(unsigned)ceil_div(M * N, 64), 256, 0, s>>>((int)M, N, z, part, alpha, beta, C,
                                                               ldc);
  KRR_LAUNCH_CHECK("long_nt_reduce");
  return KRR_OK;
}

int launch_long_nn(int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda,
                   const double* B, int64_t ldb, double beta, const double* Cin, double* C,
                   int64_t ldc, hipStream_t s) {
  long_nn<<<(unsigned)ceil_div(N, 64), 256, 0, s>>>((int)M, N, K, alpha, A, lda, B, ldb, beta,
                                                   Cin, C, ldc);
  KRR_LAUNCH_CHECK("long_nn");
  return KRR_OK;
}

}  // namespace

int gemm_colsum_into(int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda,
                     const double* B, int64_t ldb, double beta, const double* Cin, double* C,
                     int64_t ldc, hipStream_t s) {
  if (M < 1 || M > 8 || N < 1) {
    set_error("gemm_colsum_into: M=%lld N=%lld out of range", (long long)M, (long long)N);
    return KRR_EINVAL;
  }
  if (N >= kLongN) return launch_long_nn(M, N, K, alpha, A, lda, B, ldb, beta, Cin, C, ldc, s);
  const unsigned g = (unsigned)ceil_div(N, 64);
  if (M == 1)
    gemm_colsum<1><<<g, 256, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, Cin);
  else if (M <= 2)
    gemm_colsum<2><<<g, 256, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, Cin);
  else if (M <= 4)
    gemm_colsum<4><<<g, 256, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, Cin);
  else
    gemm_colsum<8><<<g, 256, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, Cin);
  KRR_LAUNCH_CHECK("gemm_colsum");
  return KRR_OK;
}

size_t gemm_scratch_bytes(int64_t M, int64_t N, int64_t K, bool lower_only) {
  const int z = choose_ksplit(M, N, K, lower_only);
  size_t need = z > 1 ? align_up((size_t)z * M * N * sizeof(double)) : 0;
  // long_nt_chunks(n, K) * n <= min(1024 * kLongCols, 256 n) for every n <= N
  // (at most 1024 / ceil(n / kLongCols) chunks): a product with fewer
  // columns than this one still fits.  Sized for min(M, 8) rows, so a
  // caller sizing for up to M > 8 right-hand sides can run its products
  // with 8 or fewer on the long-contraction kernels.
  if (K >= kLongK && !lower_only)
    need = std::max(need, align_up((size_t)std::min<int64_t>(1024 * kLongCols, 256 * N) *
                                   std::min<int64_t>(M, 8) * sizeof(double)));
  return need;
}

int gemm_f64(bool b_trans, int64_t M, int64_t N, int64_t K, double alpha, const double* A,
             int64_t lda, const double* B, int64_t ldb, double beta, double* C, int64_t ldc,
             hipStream_t s, Arena* scratch) {
  return gemm_f64_ex(false, b_trans, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, s, scratch);
}

int gemm_f64_ex(bool a_trans, bool b_trans, int64_t M, int64_t N, int64_t K, double alpha,
                const double* A, int64_t lda, const double* B, int64_t ldb, double beta, double* C,
                int64_t ldc, hipStream_t s, Arena* scratch, bool lower_only) {
  if (M <= 0 || N <= 0) return KRR_OK;
  if (!a_trans && !b_trans && M <= 8 && !lower_only && (N >= 65536 || K <= 1024)) {
    // enough columns for ~1000 workgroups, or a short K (little work per
    // workgroup, where the tiled GEMM's staging and 64-row tiles cost more
    // than they save); otherwise the tiled GEMM's K split keeps more of the
    // chip busy
    if (N >= kLongN) return launch_long_nn(M, N, K, alpha, A, lda, B, ldb, beta, C, C, ldc, s);
    const unsigned g = (unsigned)ceil_div(N, 64);
    if (M == 1)
      gemm_colsum<1><<<g, 256, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, C);
    else if (M <= 2)
      gemm_colsum<2><<<g, 256, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, C);
    else if (M <= 4)
      gemm_colsum<4><<<g, 256, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, C);
    else
      gemm_colsum<8><<<g, 256, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, C);
    KRR_LAUNCH_CHECK("gemm_colsum");
    return KRR_OK;
  }
  if (!a_trans && b_trans && M <= 8 && !lower_only) {
    if (K >= kLongK && scratch) {
      // a long contraction: one workgroup per output column would stream
      // A's rows once per column (they leave L2 at these lengths), so
      // chunks of K go to the matrix cores instead
      const int Z = long_nt_chunks(N, K);
      const size_t mark = scratch->used;
      double* part = scratch->take<double>((size_t)Z * M * N);
      if (scratch->ok()) {
        const int rc = launch_long_nt(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, part, Z, s);
        scratch->used = mark;
        return rc;
      }
      scratch->used = mark;
    }
    const unsigned g = (unsigned)N;
    if (M == 1)
      gemm_rowdot<1><<<g, 256, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
    else if (M <= 2)
      gemm_rowdot<2><<<g, 256, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
    else if (M <= 4)
      gemm_rowdot<4><<<g, 256, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
    else
      gemm_rowdot<8><<<g, 256, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
    KRR_LAUNCH_CHECK("gemm_rowdot");
    return KRR_OK;
  }
  const TileShape ts = choose_tile(M, N, K, lower_only);
  const int64_t gx = ceil_div(N, ts.tn), gy = ceil_div(M, ts.tm);
  if (lower_only && M != N) {
    set_error("gemm_f64: the lower-triangle product needs a square C (M=%lld, N=%lld)",
              (long long)M, (long long)N);
    return KRR_EINVAL;
  }
  if (tile_count(gx, gy, lower_only ? 1 : 0) > ((int64_t)1 << 30)) {
    set_error("gemm_f64: %lld x %lld output too large for the grid", (long long)M, (long long)N);
    return KRR_EINVAL;
  }
  int z = scratch ? choose_ksplit(M, N, K, lower_only) : 1;
  double* slots = nullptr;
  const size_t mark = scratch ? scratch->used : 0;
  if (z > 1) {
    slots = scratch->take<double>((size_t)z * M * N);
    if (!scratch->ok()) {
      scratch->used = mark;
      z = 1;
      slots = nullptr;
    }
  }
  const int64_t kchunk = z > 1 ? ceil_div(ceil_div(K, z), kKStep) * kKStep : std::max<int64_t>(K, 1);
  z = (int)std::max<int64_t>(1, ceil_div(K, kchunk));
  if (z == 1 && slots) {
    slots = nullptr;
    scratch->used = mark;
  }
  const int64_t tiles = tile_count(gx, gy, lower_only ? 1 : 0);
  dim3 grid((unsigned)(ceil_div(tiles, 8) * 8), 1, (unsigned)z);
  const int lw = lower_only ? 1 : 0;
  if (a_trans) {
    if (b_trans)
      launch_gemm<true, true>(ts, grid, s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, kchunk,
                              slots, lw);
    else
      launch_gemm<true, false>(ts, grid, s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, kchunk,
                               slots, lw);
  } else {
    if (b_trans)
      launch_gemm<false, true>(ts, grid, s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, kchunk,
                               slots, lw);
    else
      launch_gemm<false, false>(ts, grid, s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, kchunk,
                                slots, lw);
  }
  KRR_LAUNCH_CHECK("gemm_f64");
  if (slots) {
    splitk_reduce<<<(unsigned)ceil_div(M * N, 256), 256, 0, s>>>(slots, z, M, N, beta, C, ldc,
                                                                  lw, ts.tm);
    KRR_LAUNCH_CHECK("splitk_reduce");
    scratch->used = mark;
  }
  return KRR_OK;
}

namespace {

constexpr int64_t kNbOuter = 512;  // outer block of the two-level factorisation and solves

// Cholesky of an n x n block (n <= kNbOuter) in kNb steps: diagonal block in
// one wave, the panel below it row by row, then the lower-triangle trailing
// update (K = kNb).  col0 is the block's first column in the whole matrix.
int potrf_block(int64_t n, double* A, int64_t lda, int* info, int64_t col0, hipStream_t s) {
  for (int64_t k = 0; k < n; k += kNb) {
    const int nb = (int)std::min<int64_t>(kNb, n - k);
    double* Akk = A + k * lda + k;
    potrf_diag<<<1, 256, 0, s>>>(Akk, lda, nb, col0 + k, info);
    KRR_LAUNCH_CHECK("potrf_diag");
    const int64_t rest = n - k - nb;
    if (rest > 0) {
      potrf_panel<<<(unsigned)ceil_div(rest, 64), 256, 0, s>>>(Akk, lda, nb, Akk + nb * lda, lda,
                                                                 rest);
      KRR_LAUNCH_CHECK("potrf_panel");
      double* L21 = A + (k + nb) * lda + k;
      double* A22 = A + (k + nb) * lda + (k + nb);
      KRR_TRY(gemm_f64_ex(false, true, rest, rest, nb, -1.0, L21, lda, L21, lda, 1.0, A22, lda, s,
                          nullptr, true));
    }
  }
  return KRR_OK;
}

// X <- X L^{-T} for X (rows x nb) and the nb x nb lower factor L, left-looking
// over kNb-column blocks: one GEMM with the columns already solved, then the
// row-wise substitution.
int panel_trsm(int64_t rows, int64_t nb, const double* L, int64_t lda, double* X, int64_t ldx,
               hipStream_t s) {
  for (int64_t j = 0; j < nb; j += kNb) {
    const int jb = (int)std::min<int64_t>(kNb, nb - j);
    if (j > 0)
      KRR_TRY(gemm_f64(true, rows, jb, j, -1.0, X, ldx, L + j * lda, lda, 1.0, X + j, ldx, s));
    potrf_panel<<<(unsigned)ceil_div(rows, 64), 256, 0, s>>>(L + j * lda + j, lda, jb, X + j, ldx,
                                                               rows);
    KRR_LAUNCH_CHECK("potrf_panel");
  }
  return KRR_OK;
}

// B <- L^{-1} B for an n x n (n <= kNbOuter) lower L, left-looking in kNb
// steps: B_k -= L[k, 0:k] B[0:k], then the block substitution.
int trsm_block(int64_t n, int64_t ncols, const double* L, int64_t lda, double* B, int64_t ldb,
               hipStream_t s) {
  for (int64_t k = 0; k < n; k += kNb) {
    const int nb = (int)std::min<int64_t>(kNb, n - k);
    if (k > 0)
      KRR_TRY(gemm_f64(false, nb, ncols, k, -1.0, L + k * lda, lda, B, ldb, 1.0, B + k * ldb, ldb,
                       s));
    trsm_diag<<<(unsigned)ceil_div(ncols, 64), 256, 0, s>>>(L + k * lda + k, lda, nb,
                                                                    B + k * ldb, ldb, ncols);
    KRR_LAUNCH_CHECK("trsm_diag");
  }
  return KRR_OK;
}

}  // namespace

// Two levels of blocking: kNbOuter-wide outer steps whose GEMMs have
// K = kNbOuter (the MFMA work dominates the C traffic), and kNb-wide inner
// steps inside each diagonal block.

int potrf_lower(int64_t n, double* A, int64_t lda, int* info, hipStream_t s) {
  KRR_TRY(hip_check(hipMemsetAsync(info, 0, sizeof(int), s), "potrf info reset"));
  for (int64_t k = 0; k < n; k += kNbOuter) {
    const int64_t nb = std::min<int64_t>(kNbOuter, n - k);
    double* Akk = A + k * lda + k;
    KRR_TRY(potrf_block(nb, Akk, lda, info, k, s));
    const int64_t rest = n - k - nb;
    if (rest > 0) {
      // panel L21 = A21 L11^{-T}, then A22 -= L21 L21^T on the lower-triangle
      // tiles (the factorisation reads nothing above the diagonal)
      double* L21 = A + (k + nb) * lda + k;
      double* A22 = A + (k + nb) * lda + (k + nb);
      KRR_TRY(panel_trsm(rest, nb, Akk, lda, L21, lda, s));
      KRR_TRY(gemm_f64_ex(false, true, rest, rest, nb, -1.0, L21, lda, L21, lda, 1.0, A22, lda, s,
                          nullptr, true));
    }
  }
  return KRR_OK;
}

namespace {

// Block row k (nb rows) of the right-looking blocked forward substitution
// on X = I: solve it against L_kk, then update the rows below at once (one
// GEMM with many tiles).  Block row k of L^{-1} is zero right of column
// k + nb, so the step touches only columns 0 .. k + nb, and it reads only
// block column k of L.
int tri_inv_step(int64_t n, int64_t k, const double* L, int64_t lda, double* X, int64_t ldx,
                 hipStream_t s) {
  const int64_t nb = std::min<int64_t>(kNbOuter, n - k);
  const int64_t ncols = k + nb;
  KRR_TRY(trsm_block(nb, ncols, L + k * lda + k, lda, X + k * ldx, ldx, s));
  const int64_t below = n - k - nb;
  if (below > 0)
    KRR_TRY(gemm_f64(false, below, ncols, nb, -1.0, L + (k + nb) * lda + k, lda, X + k * ldx,
                     ldx, 1.0, X + (k + nb) * ldx, ldx, s));
  return KRR_OK;
}

// A second stream for potrf_inverse_lower and its events, released on
// every path (the stream is synchronised first).
struct SideStream {
  hipStream_t st = nullptr;
  std::vector<hipEvent_t> ev;
  ~SideStream() {
    if (st) (void)hipStreamSynchronize(st);
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
    if (st) (void)hipStreamDestroy(st);
  }
};

}  // namespace

int tri_inv_lower(int64_t n, const double* L, int64_t lda, double* X, int64_t ldx,
                  hipStream_t s) {
  for (int64_t k = 0; k < n; k += kNbOuter) KRR_TRY(tri_inv_step(n, k, L, lda, X, ldx, s));
  return KRR_OK;
}

int potrf_inverse_lower(int64_t n, double* A, int64_t lda, int* info, double* X, int64_t ldx,
                        hipStream_t s) {
  // The factorisation runs on s; block row k of the inverse needs only block
  // column k of L, final once the factorisation's panel of step k is
  // solved, so it runs on a second stream behind an event recorded there,
  // while s goes on with the trailing update and the later block columns.
  // Both are chains of small latency-bound launches that leave most of the
  // chip idle; the two overlap.
  const int64_t nblk = ceil_div(n, kNbOuter);
  if (nblk <= 1) {  // one block: nothing to overlap
    KRR_TRY(potrf_lower(n, A, lda, info, s));
    return tri_inv_lower(n, A, lda, X, ldx, s);
  }
  SideStream side;
  KRR_TRY(hip_check(hipStreamCreateWithFlags(&side.st, hipStreamNonBlocking), "side stream"));
  side.ev.assign((size_t)nblk + 2, nullptr);
  for (hipEvent_t& e : side.ev)
    KRR_TRY(hip_check(hipEventCreateWithFlags(&e, hipEventDisableTiming), "event"));
  KRR_TRY(hip_check(hipMemsetAsync(info, 0, sizeof(int), s), "potrf info reset"));
  // the side stream starts behind everything queued on s so far (A, X = I)
  KRR_TRY(hip_check(hipEventRecord(side.ev[nblk], s), "event record"));
  KRR_TRY(hip_check(hipStreamWaitEvent(side.st, side.ev[nblk], 0), "stream wait"));
  for (int64_t b = 0, k = 0; k < n; ++b, k += kNbOuter) {
    const int64_t nb = std::min<int64_t>(kNbOuter, n - k);
    double* Akk = A + k * lda + k;
    KRR_TRY(potrf_block(nb, Akk, lda, info, k, s));
    const int64_t rest = n - k - nb;
    double* L21 = A + (k + nb) * lda + k;
    if (rest > 0) KRR_TRY(panel_trsm(rest, nb, Akk, lda, L21, lda, s));
    KRR_TRY(hip_check(hipEventRecord(side.ev[b], s), "event record"));
    if (rest > 0)
      KRR_TRY(gemm_f64_ex(false, true, rest, rest, nb, -1.0, L21, lda, L21, lda, 1.0,
                          A + (k + nb) * lda + (k + nb), lda, s, nullptr, true));
    KRR_TRY(hip_check(hipStreamWaitEvent(side.st, side.ev[b], 0), "stream wait"));
    KRR_TRY(tri_inv_step(n, k, A, lda, X, ldx, side.st));
  }
  KRR_TRY(hip_check(hipEventRecord(side.ev[nblk + 1], side.st), "event record"));
  return hip_check(hipStreamWaitEvent(s, side.ev[nblk + 1], 0), "stream join");
}

int trsm_lower_left(int64_t n, int64_t ncols, const double* L, int64_t lda, double* B,
                    int64_t ldb, hipStream_t s) {
  if (ncols <= 0 || n <= 0) return KRR_OK;
  for (int64_t k = 0; k < n; k += kNbOuter) {
    const int64_t nb = std::min<int64_t>(kNbOuter, n - k);
    // B_k -= L[k, 0:k] B[0:k], then the block solve
    if (k > 0)
      KRR_TRY(gemm_f64(false, nb, ncols, k, -1.0, L + k * lda, lda, B, ldb, 1.0, B + k * ldb, ldb,
                       s));
    KRR_TRY(trsm_block(nb, ncols, L + k * lda + k, lda, B + k * ldb, ldb, s));
  }
  return KRR_OK;
}

}  // namespace krr
