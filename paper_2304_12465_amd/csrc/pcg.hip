// Preconditioned conjugate gradient (zero initial iterate, relative-residual
// stop; Sec. 3, eq. psd_system) with m independent right-hand sides, and the
// operator / preconditioner applications it calls (Alg. 1 and Alg. 2).
//
// Vectors live column-major in HBM (vector c of length n at p + c*n) so
// every update and dot product streams contiguous memory.  Dot products are
// two-stage with fixed per-block slots and a fixed-order final sum, so the
// recurrence is bitwise reproducible run to run and independent of what
// else shares the GPU.  CG scalars are FP64.
#include "solver.h"
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

namespace krr {

namespace {

constexpr int kThreads = 256;
constexpr int kMaxRefine = 6;  // refinement rounds for FP32 / MIXED tiles
// A step carries x beside p (FP64 tiles) when its recursive residual is
// predicted at most this many times the target.  A step that carries x and
// does not converge costs one more vector in the product (the FP64 Gaussian
// tile over 2,000,000 x 10,000 entries: 18.0 ms with two vectors against
// 16.9 ms with one); a converging one that does not carry it costs a whole
// operator product for the true residual, 15 times more.  The generous
// margin absorbs a contraction that slows from one step to the next (the
// 2,000,000-point KRILL solve to 1e-6: 0.02, 0.04, 0.08, 0.17, 0.16).
constexpr double kSpecReach = 5.0;

// Products of at most this many kernel entries take well under 0.1 ms, so a
// host round trip per iteration would cost as much as the iteration: such
// solves run in bursts, and their exit check is no cheaper carried.
constexpr double kBurstEntries = 1.6e7;

// Kernel entries of one operator application to m vectors.
double operator_entries(const Precond& P, int m) {
  return P.type == kRPChol ? (double)P.N * (double)P.N * m : 2.0 * (double)P.N * (double)P.k * m;
}

__device__ __forceinline__ double block_sum(double v, double* sh) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (tid < w) sh[tid] += sh[tid + w];
    __syncthreads();
  }
  return sh[0];
}

enum FinalOp { kFinPW = 0, kFinRR = 1, kFinRZ = 2, kFinInit = 3, kFinSum = 4, kFinActivate = 5 };

// The scalar step of the recurrence for column c, given the column's sum s.
__device__ __forceinline__ void final_op(int op, int c, double s, int m_max, double tol2, int slot,
                                         double* __restrict__ S) {
  const bool act = S[kActive * m_max + c] != 0.0;
  switch (op) {
    case kFinPW:
      S[kPW * m_max + c] = s;
      S[kAlpha * m_max + c] = act ? S[kRZ * m_max + c] / s : 0.0;
      break;
    case kFinRR:
      S[kRR * m_max + c] = s;
      S[kActivePrev * m_max + c] = act ? 1.0 : 0.0;
      S[kActive * m_max + c] = (act && s > tol2 * S[kBB * m_max + c]) ? 1.0 : 0.0;
      break;
    case kFinActivate:  // restart from a true residual with ||r||^2 = s
      S[kRR * m_max + c] = s;
      S[kActive * m_max + c] = (S[kBB * m_max + c] > 0.0 && s > tol2 * S[kBB * m_max + c]) ? 1.0 : 0.0;
      break;
    case kFinRZ:
      S[kRZnew * m_max + c] = s;
      S[kBeta * m_max + c] = act ? s / S[kRZ * m_max + c] : 0.0;
      if (act) S[kRZ * m_max + c] = s;
      break;
    case kFinInit:  // s = ||b||^2
      S[kBB * m_max + c] = s;
      S[kRR * m_max + c] = s;
      S[kActive * m_max + c] = s > 0.0 ? 1.0 : 0.0;
      break;
    default:
      S[slot * m_max + c] = s;
  }
}

// Where a reduction's block sums go: partial slots for finalize, or, when
// the whole column is one block (fin >= 0), straight into the scalar step
// (the sum 0 + s is what finalize would form from the single slot).
struct RedOut {
  double* part;
  int fin;  // FinalOp, or -1
  int m_max;
  double tol2;
  int slot;
  double* scal;
};
__device__ __forceinline__ void red_store(const RedOut& o, int c, int nblk, int blk, double s) {
  if (o.fin >= 0)
    final_op(o.fin, c, 0.0 + s, o.m_max, o.tol2, o.slot, o.scal);
  else
    o.part[(int64_t)c * nblk + blk] = s;
}

// One thread per column: sums the partial slots in a fixed order and applies
// the scalar step of the recurrence.
__global__ void finalize(const double* __restrict__ part, int nblk, int m, int m_max, int op,
                         double tol2, int slot, double* __restrict__ scal) {
  const int c = threadIdx.x;
  if (c >= m) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += part[(int64_t)c * nblk + b];
  final_op(op, c, s, m_max, tol2, slot, scal);
}

// part[c*nblk + blk] = sum over this block's rows of A_c * B_c
__global__ __launch_bounds__(kThreads) void dot_part(const double* __restrict__ A,
                                                     const double* __restrict__ B, int64_t n,
                                                     int64_t chunk, int nblk, const RedOut out) {
  __shared__ double sh[kThreads];
  const int c = blockIdx.y, blk = blockIdx.x;
  const int64_t i0 = (int64_t)blk * chunk;
  const int64_t i1 = (i0 + chunk < n) ? i0 + chunk : n;
  const double* a = A + (int64_t)c * n;
  const double* b = B + (int64_t)c * n;
  double s = 0.0;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += kThreads) s += a[i] * b[i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) red_store(out, c, nblk, blk, s);
}

// x += alpha p; r -= alpha w; partial sums of r^2 (new r); scal is read
// here and, for a one-block column, written by the scalar step
__global__ __launch_bounds__(kThreads) void update_xr(double* __restrict__ x,
                                                      double* __restrict__ r,
                                                      const double* __restrict__ p,
                                                      const double* __restrict__ w,
                                                      const double* scal, int m_max,
                                                      int64_t n, int64_t chunk, int nblk,
                                                      const RedOut out) {
  __shared__ double sh[kThreads];
  const int c = blockIdx.y, blk = blockIdx.x;
  const double alpha = scal[kAlpha * m_max + c];
  const int64_t i0 = (int64_t)blk * chunk;
  const int64_t i1 = (i0 + chunk < n) ? i0 + chunk : n;
  const int64_t off = (int64_t)c * n;
  double s = 0.0;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += kThreads) {
    x[off + i] += alpha * p[off + i];
    const double rv = r[off + i] - alpha * w[off + i];
    r[off + i] = rv;
    s += rv * rv;
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) red_store(out, c, nblk, blk, s);
}

// One block per column (n <= 16,384 rows): p.w, the step length, x += alpha p,
// r -= alpha w and r.r in one launch, with the same sums in the same order as
// dot_part followed by update_xr (so the iterates are bitwise those of the
// two launches).
__global__ __launch_bounds__(kThreads) void pw_update_xr(double* __restrict__ x,
                                                         double* __restrict__ r,
                                                         const double* __restrict__ p,
                                                         const double* __restrict__ w, int m_max,
                                                         int64_t n, double tol2,
                                                         double* __restrict__ scal,
                                                         int log_row = -1) {
  __shared__ double sh[kThreads];
  const int c = blockIdx.x;
  const int64_t off = (int64_t)c * n;
  const bool act = scal[kActive * m_max + c] != 0.0;
  const double rz = scal[kRZ * m_max + c];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += kThreads) s += p[off + i] * w[off + i];
  s = 0.0 + block_sum(s, sh);
  const double alpha = act ? rz / s : 0.0;
  double q = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += kThreads) {
    x[off + i] += alpha * p[off + i];
    const double rv = r[off + i] - alpha * w[off + i];
    r[off + i] = rv;
    q += rv * rv;
  }
  __syncthreads();  // sh is reused
  q = block_sum(q, sh);
  if (threadIdx.x == 0) {
    scal[kPW * m_max + c] = s;
    scal[kAlpha * m_max + c] = alpha;
    final_op(kFinRR, c, 0.0 + q, m_max, tol2, 0, scal);
    if (log_row >= 0) {
      scal[log_row * m_max + c] = scal[kRR * m_max + c];
      scal[(log_row + 1) * m_max + c] = scal[kActivePrev * m_max + c];
      scal[(log_row + 2) * m_max + c] = scal[kActive * m_max + c];
    }
  }
}

// One block per column (n <= 16,384 rows): r.z, beta and p = z + beta p in
// one launch (the sums and updates of dot_part + update_p, same order).
__global__ __launch_bounds__(kThreads) void rz_update_p(const double* __restrict__ r,
                                                        const double* __restrict__ z,
                                                        double* __restrict__ p, int m_max,
                                                        int64_t n, double* __restrict__ scal) {
  __shared__ double sh[kThreads];
  const int c = blockIdx.x;
  const int64_t off = (int64_t)c * n;
  const bool act = scal[kActive * m_max + c] != 0.0;
  const double rz_old = scal[kRZ * m_max + c];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += kThreads) s += r[off + i] * z[off + i];
  s = 0.0 + block_sum(s, sh);
  const double beta = act ? s / rz_old : 0.0;
  for (int64_t i = threadIdx.x; i < n; i += kThreads)
    p[off + i] = act ? z[off + i] + beta * p[off + i] : 0.0;
  if (threadIdx.x == 0) final_op(kFinRZ, c, s, m_max, 0.0, 0, scal);
}

// p = active ? z + beta p : 0
__global__ __launch_bounds__(kThreads) void update_p(double* __restrict__ p,
                                                     const double* __restrict__ z,
                                                     const double* __restrict__ scal, int m_max,
                                                     int64_t n) {
  const int c = blockIdx.y;
  const double beta = scal[kBeta * m_max + c];
  const bool act = scal[kActive * m_max + c] != 0.0;
  const int64_t off = (int64_t)c * n;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads)
    p[off + i] = act ? z[off + i] + beta * p[off + i] : 0.0;
}

__global__ void colmajor_from_rowmajor(const double* __restrict__ src, int64_t n, int m,
                                       double* __restrict__ dst) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * m) return;
  const int64_t i = t / m;
  const int c = (int)(t % m);
  dst[(int64_t)c * n + i] = src[t];
}

__global__ void rowmajor_from_colmajor(const double* __restrict__ src, int64_t n, int m,
                                       double* __restrict__ dst) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * m) return;
  const int64_t i = t / m;
  const int c = (int)(t % m);
  dst[t] = src[(int64_t)c * n + i];
}

__global__ void axpby(double* __restrict__ y, const double* __restrict__ x, double a, double b,
                      int64_t len) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < len) y[t] = a * x[t] + b * y[t];
}

// True residual of x + alpha p from the product of x and of p taken in the
// same step: wx <- (b - M x) - alpha (M p), column c at offset c n (wx holds
// M x on entry; alpha = 0 for a column that was not active, whose x did not
// move).
__global__ void carried_residual(const double* __restrict__ b, const double* __restrict__ w,
                                 double* __restrict__ wx, const double* __restrict__ scal,
                                 int m_max, int64_t n) {
  const int c = blockIdx.y;
  const double alpha = scal[kAlpha * m_max + c];
  const int64_t off = (int64_t)c * n;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    wx[off + i] = (b[off + i] - wx[off + i]) - alpha * w[off + i];
}

__global__ void fill(double* __restrict__ y, double v, int64_t len) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < len) y[t] = v;
}

// one block per column up to 16,384 rows (its sum then goes straight into
// the scalar step, one launch instead of two), else 2,048 rows per block
int blocks_for(int64_t n) {
  if (n <= 16384) return 1;
  return (int)std::min<int64_t>(512, ceil_div(n, 2048));
}

struct Red {
  int nblk;
  int64_t chunk;
};
Red red_for(int64_t n) {
  Red r;
  r.nblk = blocks_for(n);
  r.chunk = ceil_div(std::max<int64_t>(n, 1), r.nblk);
  return r;
}

// Residual gap on the sampled rows, one block per column c:
//   scal[kGap][c] = sum_q ((b - mu x - W)_i - r_i)^2,  i = gap_row(q, n, ns),
// with W = K(sampled rows, :) x in FP64: the squared distance between the
// FP64 residual and the recursive one on the sample, in a fixed order.
__global__ __launch_bounds__(kThreads) void gap_sums(const double* __restrict__ b,
                                                     const double* __restrict__ x,
                                                     const double* __restrict__ r,
                                                     const double* __restrict__ W, double mu,
                                                     int64_t n, int64_t ns, int m_max,
                                                     double* __restrict__ scal) {
  __shared__ double sh[kThreads];
  const int c = blockIdx.x;
  const int64_t o = (int64_t)c * n;
  double acc = 0.0;
  for (int64_t q = threadIdx.x; q < ns; q += kThreads) {
    const int64_t i = o + gap_row(q, n, ns);
    const double g = ((b[i] - mu * x[i]) - W[(int64_t)c * ns + q]) - r[i];
    acc += g * g;
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) scal[kGap * m_max + c] = acc;
}

int dot_cols(const PcgState& st, const double* A, const double* B, int m, int op, double tol2,
             int slot, hipStream_t s) {
  const Red rd = red_for(st.n);
  dim3 g((unsigned)rd.nblk, (unsigned)m);
  const RedOut out{st.part, rd.nblk == 1 ? op : -1, st.m_max, tol2, slot, st.scal};
  dot_part<<<g, kThreads, 0, s>>>(A, B, st.n, rd.chunk, rd.nblk, out);
  KRR_LAUNCH_CHECK("dot_part");
  if (rd.nblk > 1) {
    finalize<<<1, 64, 0, s>>>(st.part, rd.nblk, m, st.m_max, op, tol2, slot, st.scal);
    KRR_LAUNCH_CHECK("finalize");
  }
  return KRR_OK;
}

}  // namespace

int to_colmajor(const double* src, int64_t n, int32_t m, double* dst, hipStream_t s) {
  if (n * m == 0) return KRR_OK;
  colmajor_from_rowmajor<<<(unsigned)ceil_div(n * m, 256), 256, 0, s>>>(src, n, m, dst);
  KRR_LAUNCH_CHECK("colmajor_from_rowmajor");
  return KRR_OK;
}

int to_rowmajor(const double* src, int64_t n, int32_t m, double* dst, hipStream_t s) {
  if (n * m == 0) return KRR_OK;
  rowmajor_from_colmajor<<<(unsigned)ceil_div(n * m, 256), 256, 0, s>>>(src, n, m, dst);
  KRR_LAUNCH_CHECK("rowmajor_from_colmajor");
  return KRR_OK;
}

size_t pcg_bytes(int64_t n, int32_t m_max, int64_t N_restricted, int32_t rank, int32_t spec_m) {
  Arena a;
  PcgState st;
  pcg_carve(a, st, n, m_max, N_restricted, rank, spec_m);
  return a.used;
}

void pcg_carve(Arena& a, PcgState& st, int64_t n, int32_t m_max, int64_t N_restricted,
               int32_t rank, int32_t spec_m) {
  st.m_max = m_max;
  st.n = n;
  const size_t v = (size_t)std::max<int64_t>(n, 1) * m_max;
  // p and w also hold the columns of x (and of M x) that a product may carry
  const size_t v2 = (size_t)std::max<int64_t>(n, 1) * (m_max + spec_m);
  st.x = a.take<double>(v);
  st.r = a.take<double>(v);
  st.z = a.take<double>(v);
  st.p = a.take<double>(v2);
  st.w = a.take<double>(v2);
  st.b = a.take<double>(v);
  st.scal = a.take<double>((size_t)kScalars * m_max);
  st.nblk = blocks_for(n);
  st.part = a.take<double>((size_t)st.nblk * m_max);
  st.tmpN = N_restricted > 0 ? a.take<double>((size_t)N_restricted * (m_max + spec_m)) : nullptr;
  st.tmpR = rank > 0 ? a.take<double>((size_t)rank * m_max) : nullptr;
}

int apply_operator(Precond& P, VecBlock V, int32_t m, VecBlock W, bool force64, hipStream_t s) {
  const krr_precision pr = force64 ? KRR_FP64 : P.prec;
  if (P.type == kRPChol) {
    const PointSet& ps = force64 ? P.pts64 : P.pts;
    return product(P.kind, P.sigma, pr, ps, ps, V.view(), m, P.mu, V.view(), W.out(), P.scratch,
                   s);
  }
  // restricted: t = K_NS V, W = K_SN t + H V
  VecBlock t{P.pcg.tmpN, P.N};
  if (P.stored && (!force64 || P.kns_es == 8)) {
    // over the stored A(:,S) (FP64 storage serves the FP64 checks too)
    KRR_TRY(stored_operator(P, V.p, m, t.p, W.p, s));
  } else {
    const PointSet& xs = force64 ? P.pts64 : P.pts;
    const PointSet& cs = force64 ? P.cpts64 : P.cpts;
    KRR_TRY(product(P.kind, P.sigma, pr, xs, cs, V.view(), m, 0.0, V.view(), t.out(), P.scratch, s));
    KRR_TRY(product(P.kind, P.sigma, pr, cs, xs, t.view(), m, 0.0, t.view(), W.out(), P.scratch, s));
  }
  // W^T (m x k) += V^T (m x k) H  (H symmetric)
  return gemm_f64(false, m, P.k, P.k, 1.0, V.p, P.k, P.H, P.k, 1.0, W.p, P.k, s, &P.scratch);
}

int apply_precond(Precond& P, VecBlock R, int32_t m, VecBlock Z, hipStream_t s) {
  if (P.type == kRPChol) {
    // Woodbury form of (F F^T + mu I)^{-1}:  z = (r - Q (Q^T r)) / mu.
    const int64_t N = P.N;
    const int32_t rk = P.rank;
    const double imu = 1.0 / P.mu;
    // the short-K column-sum product reads R itself for its beta term
    const bool colsum = m <= 8 && rk > 0 && (N >= 65536 || rk <= 1024);
    if (Z.p != R.p && !colsum)
      KRR_TRY(hip_check(hipMemcpyAsync(Z.p, R.p, sizeof(double) * N * m, hipMemcpyDeviceToDevice, s),
                        "copy r"));
    if (rk == 0) {
      axpby<<<(unsigned)ceil_div(N * m, 256), 256, 0, s>>>(Z.p, Z.p, imu, 0.0, N * m);
      KRR_LAUNCH_CHECK("axpby");
      return KRR_OK;
    }
    double* TT = P.pcg.tmpR;  // m x rank: T^T = R^T Q
    KRR_TRY(gemm_f64(true, m, rk, N, 1.0, R.p, N, P.QT, N, 0.0, TT, rk, s, &P.scratch));
    // Z^T = R^T / mu - (1/mu) T^T Q^T
    if (colsum) return gemm_colsum_into(m, N, rk, -imu, TT, rk, P.QT, N, imu, R.p, Z.p, N, s);
    return gemm_f64(false, m, N, rk, -imu, TT, rk, P.QT, N, imu, Z.p, N, s, &P.scratch);
  }
  // KRILL: z = C^{-1} C^{-T} r with P = C^T C, C = L^T, i.e. z = L^{-T} (L^{-1} r),
  // as two products with the stored L^{-1} (vectors column-major: r^T is m x k).
  const int64_t k = P.k;
  double* tmp = P.pcg.tmpN;  // m x k (tmpN holds N >= k rows x m)
  KRR_TRY(gemm_f64(true, m, k, k, 1.0, R.p, k, P.Linv, k, 0.0, tmp, k, s, &P.scratch));  // (L^{-1} r)^T
  return gemm_f64(false, m, k, k, 1.0, tmp, k, P.Linv, k, 0.0, Z.p, k, s, &P.scratch);
}

int system_rhs(Precond& P, const double* Y, int32_t m, VecBlock B, hipStream_t s) {
  if (P.type == kRPChol) return to_colmajor(Y, P.N, m, B.p, s);
  // b = A(S,:) y, evaluated in FP64 (Alg. 2, last step)
  if (P.stored && P.kns_es == 8) return stored_rhs(P, Y, m, B.p, s);
  VecView y{Y, m, 1};
  return product(P.kind, P.sigma, KRR_FP64, P.cpts64, P.pts64, y, m, 0.0, y, B.out(), P.scratch,
                 s);
}

namespace {

int pull_async(Solve& S, hipStream_t s) {
  PcgState& st = S.P->pcg;
  return hip_check(hipMemcpyAsync(st.host, st.scal, sizeof(double) * kScalars * st.m_max,
                                  hipMemcpyDeviceToHost, s),
                   "scalars D2H");
}

void fail(Solve& S, int code) {
  S.err = code;
  S.phase = kPhaseDone;
  S.errmsg = last_error();
}

// z = P^{-1} r; rz = r.z (fresh, no beta); p = z
int restart_direction(Solve& S, hipStream_t s) {
  Precond& P = *S.P;
  PcgState& st = P.pcg;
  const int64_t n = st.n;
  VecBlock R{st.r, n}, Z{st.z, n};
  KRR_TRY(apply_precond(P, R, S.m, Z, s));
  KRR_TRY(dot_cols(st, st.r, st.z, S.m, kFinSum, 0, kRZ, s));
  return hip_check(hipMemcpyAsync(st.p, st.z, sizeof(double) * n * S.m, hipMemcpyDeviceToDevice, s),
                   "p = z");
}

}  // namespace

int solve_begin(Solve& S, Precond& P, const double* Y, int32_t m, double tol, int32_t max_iter,
                hipStream_t s) {
  S = Solve();
  S.P = &P;
  S.m = m;
  S.tol = tol;
  S.tol_inner = tol;
  S.max_iter = max_iter;
  S.t0 = std::chrono::steady_clock::now();
  S.iters.assign(m, 0);
  S.active.assign(m, 0);
  S.true_rel.assign(m, 0.0);
  PcgState& st = P.pcg;
  const int64_t n = st.n;
  const int64_t len = n * m;
  VecBlock Bv{st.b, n};
  KRR_TRY(system_rhs(P, Y, m, Bv, s));
  fill<<<(unsigned)ceil_div(len, 256), 256, 0, s>>>(st.x, 0.0, len);
  KRR_LAUNCH_CHECK("fill");
  KRR_TRY(hip_check(hipMemcpyAsync(st.r, st.b, sizeof(double) * len, hipMemcpyDeviceToDevice, s),
                    "r = b"));
  KRR_TRY(dot_cols(st, st.b, st.b, m, kFinInit, 0, 0, s));
  KRR_TRY(restart_direction(S, s));
  KRR_TRY(pull_async(S, s));
  KRR_TRY(hip_check(hipStreamSynchronize(s), "stream sync"));
  const int mm = st.m_max;
  bool any = false;
  for (int c = 0; c < m; ++c) {
    if (!std::isfinite(st.host[kBB * mm + c]) || !std::isfinite(st.host[kRZ * mm + c])) {
      set_error("NaN/Inf in the right-hand side or its preconditioned residual, column %d", c);
      return KRR_ENAN;
    }
    S.active[c] = st.host[kActive * mm + c] != 0.0;
    any = any || S.active[c];
  }
  S.phase = (any && max_iter > 0) ? kPhaseIterate : kPhaseCheck;
  // MIXED full-data solves estimate the residual gap each time the worst
  // relative recursive residual has halved since the last estimate (one
  // FP64 product of the sampled rows, ~1% of an iteration's product)
  if (P.type == kRPChol && P.nsamp > 0) S.gap_next = 0.5;
  return KRR_OK;
}

namespace {

// The decision after a true residual (wres: b - M x, column c at offset
// c n): done, or a restart of the recurrence from it.
void check_decision(Solve& S, const double* h, const double* wres, hipStream_t s) {
  Precond& P = *S.P;
  PcgState& st = P.pcg;
  const int mm = st.m_max;
  S.worst_true = 0.0;
  bool replace = false, bad = false;
  for (int c = 0; c < S.m; ++c) {
    const double bb = h[kBB * mm + c];
    S.true_rel[c] = 0.0;
    if (bb <= 0) continue;
    const double rt = std::sqrt(h[kTrue * mm + c] / bb);
    S.true_rel[c] = rt;
    if (!std::isfinite(rt)) bad = true;
    S.worst_true = std::max(S.worst_true, rt);
    // FP64 tiles: replace when the recurrence drifted (> 10 tol).
    // FP32 / MIXED tiles: iterative refinement with the FP64 residual
    // until it meets tol (the lower-precision operator limits the
    // recurrence).
    if (rt > (P.prec == KRR_FP64 ? 10.0 * S.tol : S.tol)) replace = true;
  }
  if (bad) {
    set_error("NaN/Inf in the true residual");
    fail(S, KRR_ENAN);
    return;
  }
  const int max_restarts = P.prec == KRR_FP64 ? 1 : kMaxRefine;
  if (!replace || S.restarts >= max_restarts || S.it >= S.max_iter) {
    S.phase = kPhaseDone;
    return;
  }
  ++S.restarts;
  // A refinement round aims below tol: the lower-precision operator
  // leaves part of each round's correction in the true residual.  That
  // part scales with the round's starting residual; the last round's
  // contraction of the true residual (rho, which includes it) bounds the
  // coming round's share by rho * worst_true.  Where that is at most
  // tol / 10 the round only has to reach tol / 2 (the true residual then
  // ends near or below 0.6 tol); otherwise it aims at tol / 10.
  if (P.prec != KRR_FP64) {
    const double rho = S.prev_true > 0.0 ? S.worst_true / S.prev_true : 1.0;
    S.tol_inner = (rho * S.worst_true <= 0.1 * S.tol ? 0.5 : 0.1) * S.tol;
  }
  S.prev_true = S.worst_true;
  S.gap_read = S.gap_pending = false;
  if (P.nsamp > 0) S.gap_next = 0.5 * S.worst_true;
  const int64_t len = st.n * S.m;
  int rc = hip_check(hipMemcpyAsync(st.r, wres, sizeof(double) * len, hipMemcpyDeviceToDevice, s),
                     "r = true residual");
  if (rc == KRR_OK)
    rc = dot_cols(st, st.r, st.r, S.m, kFinActivate, S.tol_inner * S.tol_inner, 0, s);
  if (rc == KRR_OK) rc = restart_direction(S, s);
  if (rc < 0) {
    fail(S, rc);
    return;
  }
  S.phase = kPhaseIterate;
}

}  // namespace

int solve_step(Solve* const* solves, int n, hipStream_t s) {
  // 1. products: direction products of iterating solves (their precision)
  //    and FP64 true-residual products of checking solves, one group.
  std::vector<ProductReq> reqs;
  std::vector<int> owner;
  for (int q = 0; q < n; ++q) {
    Solve& S = *solves[q];
    if (S.phase == kPhaseDone) continue;
    Precond& P = *S.P;
    PcgState& st = P.pcg;
    const bool check = S.phase == kPhaseCheck;
    // a step predicted to converge carries x beside p (columns m .. 2m - 1)
    S.spec_now = !check && S.spec_next && P.spec_m >= S.m;
    S.spec_next = false;
    if (check) ++S.check_products;
    const int32_t mc = S.spec_now ? 2 * S.m : S.m;
    if (S.spec_now) {
      const int rc = hip_check(hipMemcpyAsync(st.p + (int64_t)S.m * st.n, st.x,
                                              sizeof(double) * st.n * S.m,
                                              hipMemcpyDeviceToDevice, s),
                               "carry x");
      if (rc < 0) {
        fail(S, rc);
        continue;
      }
    }
    VecBlock src{check ? st.x : st.p, st.n}, dst{st.w, st.n};
    if (P.type == kRPChol) {
      ProductReq r;
      r.kind = P.kind;
      r.sigma = P.sigma;
      r.prec = check ? KRR_FP64 : P.prec;
      r.rows = check ? &P.pts64 : &P.pts;
      r.cols = r.rows;
      r.V = src.view();
      r.m = mc;
      r.shift = P.mu;
      r.Vs = src.view();
      r.W = dst.out();
      r.scratch = &P.scratch;
      reqs.push_back(r);
      owner.push_back(q);
    } else {
      const int rc = apply_operator(P, src, mc, dst, check, s);
      if (rc < 0) fail(S, rc);
    }
  }
  if (!reqs.empty()) {
    const int rc = product_group(reqs.data(), (int)reqs.size(), s);
    if (rc < 0) {
      for (int q : owner) fail(*solves[q], rc);
    }
  }
  // residual-gap estimates: FP64 rows of the sample against all points, on
  // x and r before this step's update (the solve's own scratch, after its
  // direction product in stream order)
  for (int q = 0; q < n; ++q) {
    Solve& S = *solves[q];
    if (S.phase != kPhaseIterate || !S.gap_pending) continue;
    S.gap_pending = false;
    Precond& P = *S.P;
    PcgState& st = P.pcg;
    VecBlock X{st.x, st.n}, Ws{P.samp_w, P.nsamp};
    int rc = product(P.kind, P.sigma, KRR_FP64, P.spts64, P.pts64, X.view(), S.m, 0.0, X.view(),
                     Ws.out(), P.scratch, s);
    if (rc == KRR_OK) {
      gap_sums<<<(unsigned)S.m, kThreads, 0, s>>>(st.b, st.x, st.r, P.samp_w, P.mu, st.n, P.nsamp,
                                                  st.m_max, st.scal);
      rc = hip_check(hipGetLastError(), "gap_sums");
    }
    if (rc < 0) {
      fail(S, rc);
      continue;
    }
    S.gap_read = true;
  }
  // 2. post-product kernels and scalar read-back
  for (int q = 0; q < n; ++q) {
    Solve& S = *solves[q];
    if (S.phase == kPhaseDone) continue;
    PcgState& st = S.P->pcg;
    const int64_t nn = st.n;
    const int mm = st.m_max;
    int rc = KRR_OK;
    if (S.phase == kPhaseIterate && red_for(nn).nblk == 1) {
      // short vectors: the dot product and the update in one launch
      pw_update_xr<<<(unsigned)S.m, kThreads, 0, s>>>(st.x, st.r, st.p, st.w, mm, nn,
                                                      S.tol_inner * S.tol_inner, st.scal);
      rc = hip_check(hipGetLastError(), "pw_update_xr");
    } else if (S.phase == kPhaseIterate) {
      rc = dot_cols(st, st.p, st.w, S.m, kFinPW, 0, 0, s);
      if (rc == KRR_OK) {
        const Red rd = red_for(nn);
        const double tol2 = S.tol_inner * S.tol_inner;
        const RedOut out{st.part, rd.nblk == 1 ? (int)kFinRR : -1, mm, tol2, 0, st.scal};
        update_xr<<<dim3((unsigned)rd.nblk, (unsigned)S.m), kThreads, 0, s>>>(
            st.x, st.r, st.p, st.w, st.scal, mm, nn, rd.chunk, rd.nblk, out);
        rc = hip_check(hipGetLastError(), "update_xr");
        if (rc == KRR_OK && rd.nblk > 1) {
          finalize<<<1, 64, 0, s>>>(st.part, rd.nblk, S.m, mm, kFinRR, tol2, 0, st.scal);
          rc = hip_check(hipGetLastError(), "finalize rr");
        }
      }
    } else {
      const int64_t len = nn * S.m;
      axpby<<<(unsigned)ceil_div(len, 256), 256, 0, s>>>(st.w, st.b, 1.0, -1.0, len);
      rc = hip_check(hipGetLastError(), "axpby");
      if (rc == KRR_OK) rc = dot_cols(st, st.w, st.w, S.m, kFinSum, 0, kTrue, s);
    }
    if (rc == KRR_OK && S.phase == kPhaseIterate && S.spec_now) {
      // the true residual of the updated x, from the product's x columns
      double* wx = st.w + (int64_t)S.m * nn;
      carried_residual<<<dim3((unsigned)std::min<int64_t>(ceil_div(nn, 256), 4096), (unsigned)S.m),
                         256, 0, s>>>(st.b, st.w, wx, st.scal, mm, nn);
      rc = hip_check(hipGetLastError(), "carried_residual");
      if (rc == KRR_OK) rc = dot_cols(st, wx, wx, S.m, kFinSum, 0, kTrue, s);
    }
    if (rc == KRR_OK) rc = pull_async(S, s);
    if (rc < 0) fail(S, rc);
  }
  KRR_TRY(hip_check(hipStreamSynchronize(s), "stream sync"));
  // 3. host decisions, then the next direction
  for (int q = 0; q < n; ++q) {
    Solve& S = *solves[q];
    if (S.phase == kPhaseDone) continue;
    Precond& P = *S.P;
    PcgState& st = P.pcg;
    const int mm = st.m_max;
    const double* h = st.host;
    if (S.phase == kPhaseIterate) {
      ++S.it;
      double worst = 0.0;
      bool any = false, bad = false;
      for (int c = 0; c < S.m; ++c) {
        if (h[kActivePrev * mm + c] != 0.0) S.iters[c] = S.it;
        const double rr = h[kRR * mm + c], bb = h[kBB * mm + c];
        if (!std::isfinite(rr)) bad = true;
        if (bb > 0) worst = std::max(worst, std::sqrt(rr / bb));
        S.active[c] = h[kActive * mm + c] != 0.0;
        any = any || S.active[c];
      }
      if (bad) {
        set_error("NaN/Inf in a residual at iteration %d", S.it);
        fail(S, KRR_ENAN);
        continue;
      }
      S.history.push_back(worst);
      if (!any || S.it >= S.max_iter) {
        // a step that carried x has its true residual in hand already
        if (S.spec_now)
          check_decision(S, h, st.w + (int64_t)S.m * st.n, s);
        else
          S.phase = kPhaseCheck;
        continue;
      }
      if (P.spec_m >= S.m && operator_entries(P, S.m) > kBurstEntries) {
        // carry x in the next step when its recursive residual, predicted
        // by this step's contraction applied once more, is within
        // kSpecReach of the target, or when it is the last step allowed
        const size_t nh = S.history.size();
        const double prev = nh >= 2 ? S.history[nh - 2] : 1.0;
        const double rho = prev > 0.0 ? std::min(1.0, worst / prev) : 1.0;
        S.spec_next = worst * rho <= kSpecReach * S.tol_inner || S.it + 1 >= S.max_iter;
      }
      if (S.gap_read) {
        // The recursive residual r tracks b - A_mixed x; the FP64 residual
        // differs from it by the sampled gap g (scaled to all N rows), which
        // stays nearly constant once the round has passed it.  Once
        // |r| <= |g| / 2 in every active column, further steps can lower the
        // FP64 residual by ~10% (sqrt(1 + 1/4) for r and g uncorrelated):
        // the round ends at this floor.
        S.gap_read = false;
        const double scale = (double)st.n / (double)P.nsamp;
        bool floor = true;
        for (int c = 0; c < S.m; ++c)
          if (S.active[c] && 4.0 * h[kRR * mm + c] > scale * h[kGap * mm + c]) floor = false;
        if (floor) {
          S.phase = kPhaseCheck;
          continue;
        }
      }
      if (S.gap_next > 0.0 && worst <= S.gap_next) {
        S.gap_pending = true;
        S.gap_next = 0.5 * worst;
      }
      VecBlock R{st.r, st.n}, Z{st.z, st.n};
      int rc = apply_precond(P, R, S.m, Z, s);
      if (rc == KRR_OK && red_for(st.n).nblk == 1) {
        rz_update_p<<<(unsigned)S.m, kThreads, 0, s>>>(st.r, st.z, st.p, mm, st.n, st.scal);
        rc = hip_check(hipGetLastError(), "rz_update_p");
      } else {
        if (rc == KRR_OK) rc = dot_cols(st, st.r, st.z, S.m, kFinRZ, 0, 0, s);
        if (rc == KRR_OK) {
          update_p<<<dim3((unsigned)std::min<int64_t>(ceil_div(st.n, 256), 4096), (unsigned)S.m),
                     kThreads, 0, s>>>(st.p, st.z, st.scal, mm, st.n);
          rc = hip_check(hipGetLastError(), "update_p");
        }
      }
      if (rc < 0) fail(S, rc);
    } else {
      check_decision(S, h, st.w, s);
    }
  }
  return KRR_OK;
}

int solve_end(Solve& S, double* beta, krr_solve_info* info, hipStream_t s) {
  Precond& P = *S.P;
  PcgState& st = P.pcg;
  if (S.err < 0) {
    set_error("%s", S.errmsg.c_str());
    return S.err;
  }
  KRR_TRY(to_rowmajor(st.x, st.n, S.m, beta, s));
  KRR_TRY(hip_check(hipStreamSynchronize(s), "stream sync"));
  const int mm = st.m_max;
  double worst_rec = 0.0;
  int conv = 0;
  // A column has converged when the FP64 true residual confirms it: FP32 and
  // MIXED tiles need ||b - M x|| <= tol ||b|| itself (the recurrence follows
  // the lower-precision operator); FP64 tiles stop on the recursive residual
  // and accept a drift of the true one up to 10 tol.
  const bool fp64 = P.prec == KRR_FP64;
  for (int c = 0; c < S.m; ++c) {
    const double bb = st.host[kBB * mm + c];
    const double rr = st.host[kRR * mm + c];
    const double rel = bb > 0 ? std::sqrt(rr / bb) : 0.0;
    worst_rec = std::max(worst_rec, rel);
    const double rt = S.true_rel[c];
    if (fp64 ? (rel <= S.tol && rt <= 10.0 * S.tol) : rt <= S.tol) ++conv;
  }
  if (info) {
    info->iters = S.m > 0 ? *std::max_element(S.iters.begin(), S.iters.end()) : 0;
    info->converged_cols = conv;
    info->relres_recursive = worst_rec;
    info->relres_true = S.worst_true;
    info->products = S.it + S.check_products;
    info->build_seconds = P.build_seconds;
    info->solve_seconds =
        std::chrono::duration<double>(std::chrono::steady_clock::now() - S.t0).count();
    if (info->history) {
      info->history_len = 0;
      for (size_t i = 0; i < S.history.size() && info->history_len < info->history_cap; ++i)
        info->history[info->history_len++] = S.history[i];
    }
  }
  return conv == S.m ? KRR_OK : KRR_NOT_CONVERGED;
}

namespace {

bool burst_eligible(const Solve& S) {
  const Precond& P = *S.P;
  if (S.phase != kPhaseIterate || S.gap_next > 0.0 || S.gap_pending || S.gap_read) return false;
  if (red_for(P.pcg.n).nblk != 1) return false;  // the one-launch short-vector kernels
  return operator_entries(P, S.m) <= kBurstEntries && S.max_iter - S.it >= 2;
}

// Up to kBurst iterations of one solve between two host synchronisations.
// The device already freezes a converged column (alpha = 0, then p = 0), so
// the iterations of a burst after its last active one change neither x nor
// r; each iteration logs ||r||^2 and the column activity (pw_update_xr), and
// the host replays them in order, exactly as solve_step would have decided
// one iteration at a time (same kernels, same arguments: same results).
int solve_burst(Solve& S, hipStream_t s) {
  Precond& P = *S.P;
  PcgState& st = P.pcg;
  const int mm = st.m_max;
  const int64_t nn = st.n;
  const int k = (int)std::min<int64_t>(kBurst, (int64_t)S.max_iter - S.it);
  const double tol2 = S.tol_inner * S.tol_inner;
  VecBlock Pv{st.p, nn}, Wv{st.w, nn}, R{st.r, nn}, Z{st.z, nn};
  for (int i = 0; i < k; ++i) {
    if (P.type == kRPChol) {
      ProductReq r;
      r.kind = P.kind;
      r.sigma = P.sigma;
      r.prec = P.prec;
      r.rows = &P.pts;
      r.cols = r.rows;
      r.V = Pv.view();
      r.m = S.m;
      r.shift = P.mu;
      r.Vs = Pv.view();
      r.W = Wv.out();
      r.scratch = &P.scratch;
      KRR_TRY(product_group(&r, 1, s));
    } else {
      KRR_TRY(apply_operator(P, Pv, S.m, Wv, false, s));
    }
    pw_update_xr<<<(unsigned)S.m, kThreads, 0, s>>>(st.x, st.r, st.p, st.w, mm, nn, tol2,
                                                    st.scal, kLog0 + 3 * i);
    KRR_TRY(hip_check(hipGetLastError(), "pw_update_xr"));
    if (i + 1 < k) {
      KRR_TRY(apply_precond(P, R, S.m, Z, s));
      rz_update_p<<<(unsigned)S.m, kThreads, 0, s>>>(st.r, st.z, st.p, mm, nn, st.scal);
      KRR_TRY(hip_check(hipGetLastError(), "rz_update_p"));
    }
  }
  KRR_TRY(pull_async(S, s));
  KRR_TRY(hip_check(hipStreamSynchronize(s), "stream sync"));
  const double* h = st.host;
  for (int i = 0; i < k; ++i) {
    const int row = kLog0 + 3 * i;
    ++S.it;
    double worst = 0.0;
    bool any = false, bad = false;
    for (int c = 0; c < S.m; ++c) {
      if (h[(row + 1) * mm + c] != 0.0) S.iters[c] = S.it;
      const double rr = h[row * mm + c], bb = h[kBB * mm + c];
      if (!std::isfinite(rr)) bad = true;
      if (bb > 0) worst = std::max(worst, std::sqrt(rr / bb));
      S.active[c] = h[(row + 2) * mm + c] != 0.0;
      any = any || S.active[c];
    }
    if (bad) {
      set_error("NaN/Inf in a residual at iteration %d", S.it);
      fail(S, KRR_ENAN);
      return KRR_OK;
    }
    S.history.push_back(worst);
    if (!any || S.it >= S.max_iter) {
      S.phase = kPhaseCheck;
      return KRR_OK;
    }
  }
  // still iterating: the next direction, as at the end of a step
  KRR_TRY(apply_precond(P, R, S.m, Z, s));
  rz_update_p<<<(unsigned)S.m, kThreads, 0, s>>>(st.r, st.z, st.p, mm, nn, st.scal);
  return hip_check(hipGetLastError(), "rz_update_p");
}

}  // namespace

int run_pcg(Precond& P, const double* Y, int32_t m, double tol, int32_t max_iter, double* beta,
            krr_solve_info* info, hipStream_t s) {
  Solve S;
  KRR_TRY(solve_begin(S, P, Y, m, tol, max_iter, s));
  Solve* one = &S;
  while (S.phase != kPhaseDone) {
    if (burst_eligible(S))
      KRR_TRY(solve_burst(S, s));
    else
      KRR_TRY(solve_step(&one, 1, s));
  }
  return solve_end(S, beta, info, s);
}

}  // namespace krr
