// Direct solve of the restricted KRR equations (Sec. 2.2, eq.
// restricted_krr_eqn): form the k x k matrix
//   M = A(S,:) A(:,S) + H,   H = mu A(S,S) + N eps tr(A(S,S)) I
// (the shifted regulariser of Alg. 2, so the system is the one KRILL's PCG
// solves), factor it and solve -- the direct method that Sec. 4.2 weighs
// against KRILL, with its O(N k^2) Gram matrix.  FP64 throughout: kernel
// blocks K(X_blk, S) of nb rows, the Gram update as a lower-triangle GEMM
// over each block, A(S,:) y over the same blocks, the blocked Cholesky,
// L^{-1} and two products.
#include "solver.h"
#include <algorithm>
#include <cmath>
#include <vector>

namespace krr {

namespace {

constexpr int64_t kBlockBytes = int64_t(1) << 30;  // one kernel block K(X_blk, S)
constexpr int64_t kMaxBlockRows = 65535 * 16;       // kernel_block64's row limit

__global__ void gather_centres(const double* __restrict__ X, int d,
                               const int64_t* __restrict__ idx, int64_t k,
                               double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < k * d) out[t] = X[idx[t / d] * d + t % d];
}

// Lower triangle of M += mu A_SS, diagonal += shift.
__global__ void add_regulariser(double* __restrict__ M, const double* __restrict__ Ass,
                                int64_t k, double mu, double shift) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= k * k) return;
  const int64_t i = t / k, j = t % k;
  if (j > i) return;
  M[t] += mu * Ass[t] + (i == j ? shift : 0.0);
}

__global__ void set_identity(double* __restrict__ X, int64_t k) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < k * k) X[t] = (t / k == t % k) ? 1.0 : 0.0;
}

struct Direct {
  PointSet pts, cpts;
  double* craw = nullptr;  // k x d centre points
  double* M = nullptr;     // k x k: Gram + H, then its Cholesky factor (lower)
  double* Linv = nullptr;  // k x k: A(S,S) first, then L^{-1}
  double* Kb = nullptr;    // nb x k kernel block
  double* b = nullptr;     // k x m: A(S,:) y
  double* t = nullptr;     // k x m: L^{-1} b
  int* info = nullptr;
  int64_t nb = 0;
  Arena scratch;
};

int direct_layout(Arena& a, krr_kernel_kind kind, int64_t N, int32_t d, int64_t k, int32_t m,
                  Direct& D) {
  KRR_TRY(carve_points(kind, KRR_FP64, N, d, a, &D.pts));
  KRR_TRY(carve_points(kind, KRR_FP64, k, d, a, &D.cpts));
  D.nb = std::max<int64_t>(1, std::min<int64_t>({N, kMaxBlockRows, kBlockBytes / (8 * k)}));
  D.craw = a.take<double>((size_t)k * d);
  D.M = a.take<double>((size_t)k * k);
  D.Linv = a.take<double>((size_t)k * k);
  D.Kb = a.take<double>((size_t)D.nb * k);
  D.b = a.take<double>((size_t)k * m);
  D.t = a.take<double>((size_t)k * m);
  D.info = a.take<int>(4);
  const size_t sb = std::max({gemm_scratch_bytes(k, k, D.nb, true), gemm_scratch_bytes(k, m, D.nb),
                              gemm_scratch_bytes(k, m, k)}) +
                    kAlign;
  char* sc = a.take<char>(sb);
  D.scratch = Arena(sc, sb);
  return KRR_OK;
}

int validate(krr_kernel_kind kind, double sigma, int64_t N, int32_t d, int32_t k, int32_t m) {
  if (kind != KRR_GAUSSIAN && kind != KRR_LAPLACE) {
    set_error("unknown kernel kind %d", (int)kind);
    return KRR_EINVAL;
  }
  if (!(sigma > 0.0) || !std::isfinite(sigma)) {
    set_error("sigma must be positive and finite");
    return KRR_EINVAL;
  }
  if (N < 1 || d < 1 || d > 64 || k < 1 || k > N || k > 32768 || m < 1 || m > 64) {
    set_error("invalid direct restricted shape N=%lld d=%d k=%d m=%d", (long long)N, d, k, m);
    return KRR_EINVAL;
  }
  return KRR_OK;
}

}  // namespace

extern "C" int krr_restricted_direct_ws(krr_kernel_kind kind, int64_t N, int32_t d, int32_t k,
                                        int32_t m, size_t* bytes) {
  KRR_TRY(validate(kind, 1.0, N, d, k, m));
  if (!bytes) {
    set_error("bytes is NULL");
    return KRR_EINVAL;
  }
  Arena a;
  Direct D;
  KRR_TRY(direct_layout(a, kind, N, d, k, m, D));
  *bytes = a.used;
  return KRR_OK;
}

extern "C" int krr_restricted_direct(krr_kernel_kind kind, double sigma, const double* X,
                                     int64_t N, int32_t d, double mu, const int64_t* centers,
                                     int32_t k, const double* Y, int32_t m, double* beta,
                                     void* ws, size_t ws_bytes, hipStream_t s) {
  KRR_TRY(validate(kind, sigma, N, d, k, m));
  if (!(mu > 0.0) || !std::isfinite(mu)) {
    set_error("mu must be positive and finite");
    return KRR_EINVAL;
  }
  if (!X || !centers || !Y || !beta) {
    set_error("NULL array argument");
    return KRR_EINVAL;
  }
  Arena meas;
  Direct D;
  KRR_TRY(direct_layout(meas, kind, N, d, k, m, D));
  KRR_TRY(check_ws(ws, ws_bytes, meas.used));
  Arena a(ws, ws_bytes);
  D = Direct();
  KRR_TRY(direct_layout(a, kind, N, d, k, m, D));
  // centre indices are read back once and checked
  std::vector<int64_t> hc((size_t)k);
  KRR_TRY(hip_check(hipMemcpyAsync(hc.data(), centers, sizeof(int64_t) * k,
                                   hipMemcpyDeviceToHost, s), "centres D2H"));
  KRR_TRY(hip_check(hipStreamSynchronize(s), "sync"));
  for (int64_t i = 0; i < k; ++i)
    if (hc[i] < 0 || hc[i] >= N) {
      set_error("centre index %lld out of range", (long long)hc[i]);
      return KRR_EINVAL;
    }
  // point layouts (the centres share the full set's shared parameters)
  KRR_TRY(fill_points(kind, KRR_FP64, X, nullptr, D.pts, s));
  gather_centres<<<(unsigned)ceil_div((int64_t)k * d, 256), 256, 0, s>>>(X, d, centers, k, D.craw);
  KRR_LAUNCH_CHECK("gather_centres");
  KRR_TRY(fill_points(kind, KRR_FP64, D.craw, shared_params(kind, KRR_FP64, D.pts), D.cpts, s));
  // Gram matrix (lower triangle) and right-hand side over row blocks
  for (int64_t r0 = 0; r0 < N; r0 += D.nb) {
    const int64_t nr = std::min(D.nb, N - r0);
    PointSet rows = D.pts;
    rows.n = nr;
    rows.x64 = D.pts.x64 + r0 * D.pts.dpad;
    KRR_TRY(kernel_block64(kind, sigma, rows, D.cpts, D.Kb, k, s));
    const double beta0 = r0 == 0 ? 0.0 : 1.0;
    KRR_TRY(gemm_f64_ex(true, false, k, k, nr, 1.0, D.Kb, k, D.Kb, k, beta0, D.M, k, s, &D.scratch,
                        true));
    KRR_TRY(gemm_f64_ex(true, false, k, m, nr, 1.0, D.Kb, k, Y + r0 * m, m, beta0, D.b, m, s,
                        &D.scratch));
  }
  // + H: both kernels are 1 on the diagonal, so tr(A(S,S)) = k
  KRR_TRY(kernel_block64(kind, sigma, D.cpts, D.cpts, D.Linv, k, s));
  const double shift = (double)N * kEps * (double)k;
  add_regulariser<<<(unsigned)ceil_div((int64_t)k * k, 256), 256, 0, s>>>(D.M, D.Linv, k, mu, shift);
  KRR_LAUNCH_CHECK("add_regulariser");
  set_identity<<<(unsigned)ceil_div((int64_t)k * k, 256), 256, 0, s>>>(D.Linv, k);
  KRR_LAUNCH_CHECK("set_identity");
  KRR_TRY(potrf_inverse_lower(k, D.M, k, D.info, D.Linv, k, s));
  int info = 0;
  KRR_TRY(hip_check(hipMemcpyAsync(&info, D.info, sizeof(int), hipMemcpyDeviceToHost, s), "info"));
  KRR_TRY(hip_check(hipStreamSynchronize(s), "sync"));
  if (info != 0) {
    set_error("Cholesky of the restricted matrix failed at column %d", info);
    return KRR_ENOTSPD;
  }
  // beta = L^{-T} (L^{-1} b)
  KRR_TRY(gemm_f64(false, k, m, k, 1.0, D.Linv, k, D.b, m, 0.0, D.t, m, s, &D.scratch));
  KRR_TRY(gemm_f64_ex(true, false, k, m, k, 1.0, D.Linv, k, D.t, m, 0.0, beta, m, s, &D.scratch));
  return hip_check(hipStreamSynchronize(s), "sync");
}

}  // namespace krr
