// FP64 dense linear algebra for the build steps of the method: the Woodbury
// core F^T F + mu I (Alg. 1 preconditioner), its Cholesky factor, the KRILL
// matrix B^T B + H and its Cholesky factor (Alg. 2), and the triangular
// solves that apply them.  GEMM runs on the FP64 matrix cores.
#include "la.h"
#include <algorithm>

namespace krr {

namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kTile = 64;   // output tile per workgroup (64 x 64)
constexpr int kKStep = 16;  // K slice staged in LDS per iteration
constexpr int kPad = 17;    // LDS row pitch in doubles

// v_mfma_f64_16x16x4f64 operand layout (wave64):
//   A (16 x 4): lane l holds A[l % 16][l / 16]
//   B (4 x 16): lane l holds B[l / 16][l % 16]
//   D (16 x 16): lane l, element t holds D[4 t + l / 16][l % 16]
template <bool AT, bool BT>
__global__ __launch_bounds__(256) void gemm_f64_kernel(int64_t M, int64_t N, int64_t K,
                                                       double alpha, const double* __restrict__ A,
                                                       int64_t lda, const double* __restrict__ B,
                                                       int64_t ldb, double beta,
                                                       double* __restrict__ C, int64_t ldc,
                                                       int64_t kchunk, double* __restrict__ slots,
                                                       int lower) {
  __shared__ double As[kTile][kPad];  // [m][k]
  __shared__ double Bs[kTile][kPad];  // [n][k]
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int64_t m0 = (int64_t)blockIdx.y * kTile, n0 = (int64_t)blockIdx.x * kTile;
  if (lower && n0 > m0) return;  // tile strictly above the diagonal: not wanted
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  f64x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};

  const int ar = tid >> 2, ak = (tid & 3) * 4;  // A tile loader: 64 rows x 16 k
  // split K: this workgroup covers [kb, ke); the bounds checks below use ke
  const int64_t kb = (int64_t)blockIdx.z * kchunk;
  const int64_t ke = (kb + kchunk < K) ? kb + kchunk : K;
  for (int64_t k0 = kb; k0 < ke; k0 += kKStep) {
    if (!AT) {
      const int64_t gm = m0 + ar;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t gk = k0 + ak + u;
        As[ar][ak + u] = (gm < M && gk < ke) ? A[gm * lda + gk] : 0.0;
      }
    } else {
      const int kk = tid >> 4, mm = (tid & 15) * 4;  // A is K x M: 16 k x 64 m
      const int64_t gk = k0 + kk;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t gm = m0 + mm + u;
        As[mm + u][kk] = (gk < ke && gm < M) ? A[gk * lda + gm] : 0.0;
      }
    }
    if (BT) {
      const int64_t gn = n0 + ar;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t gk = k0 + ak + u;
        Bs[ar][ak + u] = (gn < N && gk < ke) ? B[gn * ldb + gk] : 0.0;
      }
    } else {
      const int kk = tid >> 4, nn = (tid & 15) * 4;  // 16 k x 64 n
      const int64_t gk = k0 + kk;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t gn = n0 + nn + u;
        Bs[nn + u][kk] = (gk < ke && gn < N) ? B[gk * ldb + gn] : 0.0;
      }
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < kKStep; ks += 4) {
      double a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = As[wm + i * 16 + (lane & 15)][ks + (lane >> 4)];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = Bs[wn + j * 16 + (lane & 15)][ks + (lane >> 4)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int64_t gm = m0 + wm + i * 16 + 4 * t + (lane >> 4);
        const int64_t gn = n0 + wn + j * 16 + (lane & 15);
        if (gm < M && gn < N) {
          double v = alpha * acc[i][j][t];
          if (slots) {
            slots[((int64_t)blockIdx.z * M + gm) * N + gn] = v;
          } else {
            if (beta != 0.0) v += beta * C[gm * ldc + gn];
            C[gm * ldc + gn] = v;
          }
        }
      }
}

// C = sum_z slots[z] (fixed order) + beta C
__global__ __launch_bounds__(256) void splitk_reduce(const double* __restrict__ slots, int nz,
                                                     int64_t M, int64_t N, double beta,
                                                     double* __restrict__ C, int64_t ldc,
                                                     int lower) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= M * N) return;
  const int64_t m = t / N, n = t % N;
  if (lower && n / kTile > m / kTile) return;  // tile skipped by the GEMM
  double v = 0.0;
  for (int z = 0; z < nz; ++z) v += slots[((int64_t)z * M + m) * N + n];
  if (beta != 0.0) v += beta * C[m * ldc + n];
  C[m * ldc + n] = v;
}

int choose_ksplit(int64_t M, int64_t N, int64_t K) {
  const int64_t tiles = ceil_div(M, kTile) * ceil_div(N, kTile);
  if (tiles >= 512 || K < 8192) return 1;
  int64_t z = ceil_div(1024, tiles);
  z = std::min<int64_t>(z, K / 2048);
  return (int)std::max<int64_t>(1, std::min<int64_t>(z, 4096));
}

constexpr int kNb = 64;  // block size of the blocked factorisation and solves

// Cholesky of one nb x nb diagonal block held in LDS (right-looking).
__global__ __launch_bounds__(256) void potrf_diag(double* __restrict__ A, int64_t lda, int nb,
                                                  int64_t col0, int* __restrict__ info) {
  __shared__ double T[kNb][kNb + 1];
  __shared__ int bad;
  const int tid = threadIdx.x;
  for (int e = tid; e < nb * nb; e += blockDim.x) T[e / nb][e % nb] = A[(e / nb) * lda + e % nb];
  if (tid == 0) bad = 0;
  __syncthreads();
  for (int k = 0; k < nb; ++k) {
    if (tid == 0) {
      const double p = T[k][k];
      if (!(p > 0.0)) {
        if (!bad) bad = (int)(col0 + k + 1);
        T[k][k] = 1.0;  // keep going with finite values; info reports the failure
      } else {
        T[k][k] = sqrt(p);
      }
    }
    __syncthreads();
    const double piv = T[k][k];
    for (int i = k + 1 + tid; i < nb; i += blockDim.x) T[i][k] /= piv;
    __syncthreads();
    const int rem = nb - k - 1;
    for (int e = tid; e < rem * rem; e += blockDim.x) {
      const int i = k + 1 + e / rem, j = k + 1 + e % rem;
      if (j <= i) T[i][j] -= T[i][k] * T[j][k];
    }
    __syncthreads();
  }
  for (int e = tid; e < nb * nb; e += blockDim.x) {
    const int i = e / nb, j = e % nb;
    if (j <= i) A[i * lda + j] = T[i][j];
  }
  if (tid == 0 && bad && *info == 0) *info = bad;
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

// x <- T^{-1} x by forward substitution, fully unrolled so that x stays in
// registers; two partial sums per row halve the dependent FMA chain.  The
// scheduling barriers keep the compiler from hoisting the whole triangle's
// LDS reads into registers at once.
__device__ __forceinline__ void tri_forward(const double (*T)[kNb + 1], const double* tinv,
                                            double (&x)[kNb]) {
#pragma unroll
  for (int q = 0; q < kNb; ++q) {
    double s0 = x[q], s1 = 0.0;
#pragma unroll
    for (int p = 0; p + 1 < q; p += 2) {
      s0 = __builtin_fma(-T[q][p], x[p], s0);
      s1 = __builtin_fma(-T[q][p + 1], x[p + 1], s1);
      if ((p & 15) == 14) __builtin_amdgcn_sched_barrier(0);
    }
    if (q & 1) s0 = __builtin_fma(-T[q][q - 1], x[q - 1], s0);
    x[q] = (s0 + s1) * tinv[q];
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Branch-free strided access to the nb <= kNb entries of one column: entries
// q >= nb alias entry nb - 1 (they are loaded, solved against the identity
// padding and never affect entries < nb).  The store runs from q = kNb - 1
// down, so entry nb - 1 is written last with its solved value.
__device__ __forceinline__ void load_col(const double* __restrict__ base, int64_t stride, int nb,
                                         double (&x)[kNb]) {
#pragma unroll
  for (int q = 0; q < kNb; ++q) x[q] = base[(int64_t)(q < nb ? q : nb - 1) * stride];
}
__device__ __forceinline__ void store_col(double* __restrict__ base, int64_t stride, int nb,
                                          const double (&x)[kNb]) {
  // a fresh copy of the stride: the store addresses are recomputed rather
  // than kept live across the solve
  __asm__ volatile("" : "+s"(stride));
#pragma unroll
  for (int q = kNb - 1; q >= 0; --q) base[(int64_t)(q < nb ? q : nb - 1) * stride] = x[q];
}

// Rows below the diagonal block: L_i = A_i L_kk^{-T}, one thread per row
// (the row solve is a forward substitution with L_kk).
__global__ __launch_bounds__(256) void potrf_panel(double* __restrict__ A, int64_t lda, int nb,
                                                   int64_t nrows) {
  __shared__ double T[kNb][kNb + 1];
  __shared__ double tinv[kNb];
  // A points at the diagonal block; panel rows start nb rows below
  stage_tri(A, lda, nb, T, tinv);
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  double* row = A + (nb + r) * lda;
  double x[kNb];
  load_col(row, 1, nb, x);
  tri_forward(T, tinv, x);
  store_col(row, 1, nb, x);
}

// One block of a lower-triangular solve with many right-hand sides:
// B_blk <- L_blk^{-1} B_blk, one thread per right-hand-side column.
__global__ __launch_bounds__(256) void trsm_diag(const double* __restrict__ L, int64_t lda, int nb,
                                                 double* __restrict__ B, int64_t ldb,
                                                 int64_t ncols) {
  __shared__ double T[kNb][kNb + 1];
  __shared__ double tinv[kNb];
  stage_tri(L, lda, nb, T, tinv);
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncols) return;
  double x[kNb];
  load_col(B + c, ldb, nb, x);
  tri_forward(T, tinv, x);
  store_col(B + c, ldb, nb, x);
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
                                                   double beta, double* __restrict__ C,
                                                   int64_t ldc) {
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
        const double old = beta != 0.0 ? beta * C[c * ldc + j] : 0.0;
        C[c * ldc + j] = alpha * v + old;
      }
  }
}

}  // namespace

size_t gemm_scratch_bytes(int64_t M, int64_t N, int64_t K) {
  const int z = choose_ksplit(M, N, K);
  return z > 1 ? align_up((size_t)z * M * N * sizeof(double)) : 0;
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
  if (!a_trans && !b_trans && M <= 8 && !lower_only && N >= 65536) {
    // enough columns for ~1000 workgroups; below that the tiled GEMM (with
    // its K split) keeps more of the chip busy
    const unsigned g = (unsigned)ceil_div(N, 64);
    if (M == 1)
      gemm_colsum<1><<<g, 256, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
    else if (M <= 2)
      gemm_colsum<2><<<g, 256, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
    else if (M <= 4)
      gemm_colsum<4><<<g, 256, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
    else
      gemm_colsum<8><<<g, 256, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
    KRR_LAUNCH_CHECK("gemm_colsum");
    return KRR_OK;
  }
  if (!a_trans && b_trans && M <= 8 && !lower_only) {
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
  const int64_t gx = ceil_div(N, kTile), gy = ceil_div(M, kTile);
  if (gy > 65535) {
    set_error("gemm_f64: M=%lld too large for the grid", (long long)M);
    return KRR_EINVAL;
  }
  int z = scratch ? choose_ksplit(M, N, K) : 1;
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
  dim3 grid((unsigned)gx, (unsigned)gy, (unsigned)z);
  if (a_trans) {
    if (b_trans)
      gemm_f64_kernel<true, true><<<grid, 256, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C,
                                                       ldc, kchunk, slots, lower_only ? 1 : 0);
    else
      gemm_f64_kernel<true, false><<<grid, 256, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C,
                                                        ldc, kchunk, slots, lower_only ? 1 : 0);
  } else {
    if (b_trans)
      gemm_f64_kernel<false, true><<<grid, 256, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C,
                                                        ldc, kchunk, slots, lower_only ? 1 : 0);
    else
      gemm_f64_kernel<false, false><<<grid, 256, 0, s>>>(M, N, K, alpha, A, lda, B, ldb, beta, C,
                                                         ldc, kchunk, slots, lower_only ? 1 : 0);
  }
  KRR_LAUNCH_CHECK("gemm_f64");
  if (slots) {
    splitk_reduce<<<(unsigned)ceil_div(M * N, 256), 256, 0, s>>>(slots, z, M, N, beta, C, ldc,
                                                                  lower_only ? 1 : 0);
    KRR_LAUNCH_CHECK("splitk_reduce");
    scratch->used = mark;
  }
  return KRR_OK;
}

int potrf_lower(int64_t n, double* A, int64_t lda, int* info, hipStream_t s) {
  KRR_TRY(hip_check(hipMemsetAsync(info, 0, sizeof(int), s), "potrf info reset"));
  for (int64_t k = 0; k < n; k += kNb) {
    const int nb = (int)std::min<int64_t>(kNb, n - k);
    double* Akk = A + k * lda + k;
    potrf_diag<<<1, 256, 0, s>>>(Akk, lda, nb, k, info);
    KRR_LAUNCH_CHECK("potrf_diag");
    const int64_t rest = n - k - nb;
    if (rest > 0) {
      potrf_panel<<<(unsigned)ceil_div(rest, 256), 256, 0, s>>>(Akk, lda, nb, rest);
      KRR_LAUNCH_CHECK("potrf_panel");
      // trailing update A22 -= L21 L21^T on the lower-triangle tiles (the
      // factorisation reads nothing above the diagonal)
      double* L21 = A + (k + nb) * lda + k;
      double* A22 = A + (k + nb) * lda + (k + nb);
      KRR_TRY(gemm_f64_ex(false, true, rest, rest, nb, -1.0, L21, lda, L21, lda, 1.0, A22, lda, s,
                          nullptr, true));
    }
  }
  return KRR_OK;
}

int tri_inv_lower(int64_t n, const double* L, int64_t lda, double* X, int64_t ldx,
                  hipStream_t s) {
  // right-looking blocked forward substitution on X = I: after block row k
  // is solved, the rows below are updated at once (one GEMM with many
  // tiles).  Block row k of L^{-1} is zero right of column k + nb, so every
  // step touches only columns 0 .. k + nb.
  for (int64_t k = 0; k < n; k += kNb) {
    const int nb = (int)std::min<int64_t>(kNb, n - k);
    const int64_t ncols = k + nb;
    trsm_diag<<<(unsigned)ceil_div(ncols, 256), 256, 0, s>>>(L + k * lda + k, lda, nb, X + k * ldx,
                                                             ldx, ncols);
    KRR_LAUNCH_CHECK("trsm_diag");
    const int64_t below = n - k - nb;
    if (below > 0)
      KRR_TRY(gemm_f64(false, below, ncols, nb, -1.0, L + (k + nb) * lda + k, lda, X + k * ldx,
                       ldx, 1.0, X + (k + nb) * ldx, ldx, s));
  }
  return KRR_OK;
}

int trsm_lower_left(int64_t n, int64_t ncols, const double* L, int64_t lda, double* B,
                    int64_t ldb, hipStream_t s) {
  if (ncols <= 0 || n <= 0) return KRR_OK;
  for (int64_t k = 0; k < n; k += kNb) {
    const int nb = (int)std::min<int64_t>(kNb, n - k);
    if (k > 0) {
      // B_k -= L[k, 0:k] B[0:k]
      KRR_TRY(gemm_f64(false, nb, ncols, k, -1.0, L + k * lda, lda, B, ldb, 1.0, B + k * ldb, ldb,
                       s));
    }
    trsm_diag<<<(unsigned)ceil_div(ncols, 256), 256, 0, s>>>(L + k * lda + k, lda, nb,
                                                                    B + k * ldb, ldb, ncols);
    KRR_LAUNCH_CHECK("trsm_diag");
  }
  return KRR_OK;
}

}  // namespace krr
