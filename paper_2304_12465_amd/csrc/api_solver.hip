// C ABI: preconditioner builds, applications and the PCG solve.
#include "solver.h"
#include <cmath>
#include <new>

using namespace krr;

struct krr_precond_s {
  Precond P;
};

namespace {

int check_kernel(int kind, double sigma, int prec) {
  if (kind != KRR_GAUSSIAN && kind != KRR_LAPLACE) {
    set_error("unknown kernel kind %d", kind);
    return KRR_EINVAL;
  }
  if (prec != KRR_FP64 && prec != KRR_FP32 && prec != KRR_MIXED) {
    set_error("unknown precision %d", prec);
    return KRR_EINVAL;
  }
  if (!(sigma > 0.0) || !std::isfinite(sigma)) {
    set_error("sigma must be positive and finite");
    return KRR_EINVAL;
  }
  return KRR_OK;
}

int rp_params(Precond& P, krr_kernel_kind kind, krr_precision prec, int64_t N, int32_t d,
              int32_t r, int32_t B, int32_t m_max) {
  if (N < 1 || d < 1 || d > 64 || r < 1 || r > N || B < 0 || B > kBmax || m_max < 1 ||
      m_max > 64) {
    set_error("invalid RPCholesky shape N=%lld d=%d r=%d B=%d m_max=%d", (long long)N, d, r, B,
              m_max);
    return KRR_EINVAL;
  }
  if (prec == KRR_MIXED && kind == KRR_GAUSSIAN && padded_dim(d) == 0) return KRR_EINVAL;
  P.type = kRPChol;
  P.kind = kind;
  P.prec = prec;
  P.N = N;
  P.d = d;
  P.r_req = r;
  P.B = B > 0 ? B : std::min(100, (r + 9) / 10);
  P.m_max = m_max;
  return KRR_OK;
}

int finish_carve(Precond& P, void* ws, size_t ws_bytes, size_t need) {
  KRR_TRY(check_ws(ws, ws_bytes, need));
  P.ws_used = need;
  // one pinned block: the PCG scalar mirror, then the build's staging bytes
  const size_t scal = align_up(sizeof(double) * kScalars * P.m_max);
  KRR_TRY(hip_check(hipHostMalloc((void**)&P.pcg.host, scal + kHostStage, hipHostMallocDefault),
                    "pinned host scalars"));
  P.rp.hstage = reinterpret_cast<char*>(P.pcg.host) + scal;
  return KRR_OK;
}

int valid_precond(krr_precond P) {
  if (!P) {
    set_error("NULL precond");
    return KRR_EINVAL;
  }
  return KRR_OK;
}

// Calls that use the PCG vectors of the workspace are refused while a
// stepped solve holds them.
int precond_idle(krr_precond P) {
  KRR_TRY(valid_precond(P));
  if (P->P.solving) {
    set_error("the precond is running a stepped solve (end or free it first)");
    return KRR_EINVAL;
  }
  return KRR_OK;
}

}  // namespace

extern "C" int krr_rpchol_ws(krr_kernel_kind kind, krr_precision prec, int64_t N, int32_t d,
                             int32_t r, int32_t B, int32_t m_max, size_t* bytes) {
  KRR_TRY(check_kernel(kind, 1.0, prec));
  if (!bytes) {
    set_error("bytes is NULL");
    return KRR_EINVAL;
  }
  Precond P;
  KRR_TRY(rp_params(P, kind, prec, N, d, r, B, m_max));
  Arena a;
  KRR_TRY(rpchol_layout(a, P));
  *bytes = a.used;
  return KRR_OK;
}

extern "C" int krr_nystrom_build(krr_kernel_kind kind, double sigma, krr_precision prec,
                                 const double* X, int64_t N, int32_t d, double mu, int32_t r,
                                 int32_t B, uint64_t seed, krr_pivot_rule rule, int32_t m_max,
                                 void* ws, size_t ws_bytes, krr_precond* out,
                                 hipStream_t stream) {
  KRR_TRY(check_kernel(kind, sigma, prec));
  if (rule != KRR_PIVOT_RPCHOL && rule != KRR_PIVOT_UNIFORM && rule != KRR_PIVOT_GREEDY) {
    set_error("unknown pivot rule %d", (int)rule);
    return KRR_EINVAL;
  }
  if (!out || !X) {
    set_error("NULL argument");
    return KRR_EINVAL;
  }
  if (!(mu > 0.0) || !std::isfinite(mu)) {
    set_error("mu must be positive and finite");
    return KRR_EINVAL;
  }
  *out = nullptr;
  krr_precond h = new (std::nothrow) krr_precond_s;
  if (!h) {
    set_error("out of host memory");
    return KRR_EINVAL;
  }
  Precond& P = h->P;
  int rc = rp_params(P, kind, prec, N, d, r, B, m_max);
  if (rc == KRR_OK) {
    P.sigma = sigma;
    P.mu = mu;
    P.seed = seed;
    P.rule = rule;
    if (rule == KRR_PIVOT_GREEDY) P.B = 1;  // one pivot per step
    Arena meas;
    rc = rpchol_layout(meas, P);
    if (rc == KRR_OK) rc = finish_carve(P, ws, ws_bytes, meas.used);
    if (rc == KRR_OK) {
      Arena a(ws, ws_bytes);
      rc = rpchol_layout(a, P);
    }
    if (rc == KRR_OK) rc = rpchol_build(P, X, stream);
  }
  if (rc != KRR_OK) {
    krr_precond_free(h);
    return rc;
  }
  *out = h;
  return KRR_OK;
}

extern "C" int krr_rpchol_build(krr_kernel_kind kind, double sigma, krr_precision prec,
                                const double* X, int64_t N, int32_t d, double mu, int32_t r,
                                int32_t B, uint64_t seed, int32_t m_max, void* ws,
                                size_t ws_bytes, krr_precond* out, hipStream_t stream) {
  return krr_nystrom_build(kind, sigma, prec, X, N, d, mu, r, B, seed, KRR_PIVOT_RPCHOL, m_max, ws,
                           ws_bytes, out, stream);
}

namespace {
__global__ void lower_copy(const double* __restrict__ L, int64_t n, double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * n) return;
  const int64_t i = t / n, j = t % n;
  out[t] = j <= i ? L[t] : 0.0;
}

// Clears the strict upper triangle of an n x n row-major matrix.
__global__ void zero_upper(double* __restrict__ L, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * n) return;
  if (t % n > t / n) L[t] = 0.0;
}
}  // namespace

extern "C" int krr_rpchol_factor(krr_precond h, double* FT, hipStream_t stream) {
  KRR_TRY(valid_precond(h));
  Precond& P = h->P;
  if (P.type != kRPChol) {
    set_error("not an RPCholesky preconditioner");
    return KRR_EINVAL;
  }
  const int64_t rk = P.rank;
  if (rk == 0) return KRR_OK;
  if (!FT) {
    set_error("NULL output");
    return KRR_EINVAL;
  }
  // L (the lower Cholesky factor of mu I + F^T F) lives in P.core, whose
  // strict upper triangle holds values of no meaning and is read by nothing
  // after the build: clear it in place, then F^T = L Q^T
  zero_upper<<<(unsigned)ceil_div(rk * rk, 256), 256, 0, stream>>>(P.core, rk);
  KRR_LAUNCH_CHECK("zero_upper");
  return gemm_f64(false, rk, P.N, rk, 1.0, P.core, rk, P.QT, P.N, 0.0, FT, P.N, stream);
}

extern "C" int krr_precond_dims(krr_precond h, int32_t* rank, int64_t* n) {
  KRR_TRY(valid_precond(h));
  const Precond& P = h->P;
  if (rank) *rank = P.type == kRPChol ? P.rank : P.k;
  if (n) *n = P.pcg.n;
  return KRR_OK;
}

extern "C" int krr_precond_pivots(krr_precond h, int64_t* host_out, int32_t cap, int32_t* count) {
  KRR_TRY(valid_precond(h));
  const Precond& P = h->P;
  const std::vector<int64_t>& v = P.type == kRPChol ? P.pivots : P.centers_host;
  const int32_t n = (int32_t)v.size();
  if (count) *count = n;
  if (host_out)
    for (int32_t i = 0; i < n && i < cap; ++i) host_out[i] = v[i];
  return KRR_OK;
}

extern "C" int krr_precond_apply(krr_precond h, const double* Z, int32_t m, double* OUT,
                                 hipStream_t stream) {
  KRR_TRY(precond_idle(h));
  Precond& P = h->P;
  if (m < 1 || m > P.m_max || !Z || !OUT) {
    set_error("invalid arguments (m=%d, m_max=%d)", m, P.m_max);
    return KRR_EINVAL;
  }
  const int64_t n = P.pcg.n;
  VecBlock R{P.pcg.r, n}, Zb{P.pcg.z, n};
  KRR_TRY(to_colmajor(Z, n, m, R.p, stream));
  KRR_TRY(apply_precond(P, R, m, Zb, stream));
  return to_rowmajor(Zb.p, n, m, OUT, stream);
}

extern "C" int krr_precond_operator(krr_precond h, const double* V, int32_t m, double* OUT,
                                    hipStream_t stream) {
  KRR_TRY(precond_idle(h));
  Precond& P = h->P;
  if (m < 1 || m > P.m_max || !V || !OUT) {
    set_error("invalid arguments (m=%d, m_max=%d)", m, P.m_max);
    return KRR_EINVAL;
  }
  const int64_t n = P.pcg.n;
  VecBlock Pv{P.pcg.p, n}, W{P.pcg.w, n};
  KRR_TRY(to_colmajor(V, n, m, Pv.p, stream));
  KRR_TRY(apply_operator(P, Pv, m, W, false, stream));
  return to_rowmajor(W.p, n, m, OUT, stream);
}

extern "C" void krr_precond_free(krr_precond h) {
  if (!h) return;
  if (h->P.pcg.host) (void)hipHostFree(h->P.pcg.host);
  delete h;
}

extern "C" int krr_pcg_solve(krr_precond h, const double* Y, int32_t m, double tol,
                             int32_t max_iter, double* beta, krr_solve_info* info,
                             hipStream_t stream) {
  KRR_TRY(precond_idle(h));
  Precond& P = h->P;
  if (m < 1 || m > P.m_max || !Y || !beta || !(tol > 0.0) || max_iter < 0) {
    set_error("invalid arguments (m=%d, m_max=%d, tol=%g, max_iter=%d)", m, P.m_max, tol,
              max_iter);
    return KRR_EINVAL;
  }
  return run_pcg(P, Y, m, tol, max_iter, beta, info, stream);
}

namespace {

int krill_params(Precond& P, krr_kernel_kind kind, krr_precision prec, int64_t N, int32_t d,
                 int32_t k, int32_t sketch_rows, int32_t zeta, int32_t m_max) {
  if (N < 1 || d < 1 || d > 64 || k < 1 || k > N || k > 65536 || m_max < 1 || m_max > 64 ||
      sketch_rows < 0 || zeta < 0) {
    set_error("invalid KRILL shape N=%lld d=%d k=%d sketch_rows=%d zeta=%d m_max=%d",
              (long long)N, d, k, sketch_rows, zeta, m_max);
    return KRR_EINVAL;
  }
  const int32_t ds = sketch_rows > 0 ? sketch_rows : 2 * k;
  const int32_t z = zeta > 0 ? zeta : (int32_t)std::ceil(std::log((double)k + 1.0));
  if (z > ds) {
    set_error("zeta=%d exceeds the sketch rows %d", z, ds);
    return KRR_EINVAL;
  }
  P.type = kKrill;
  P.kind = kind;
  // KRR_MIXED: FP64 restricted products, right-hand side and checks, FP32
  // sketch tiles
  P.prec = prec == KRR_MIXED ? KRR_FP64 : prec;
  P.sketch_prec = prec == KRR_MIXED ? KRR_FP32 : prec;
  P.N = N;
  P.d = d;
  P.k = k;
  P.sketch_rows = ds;
  P.zeta = z;
  P.m_max = m_max;
  return KRR_OK;
}

__global__ void widen_signs(const int* __restrict__ neg, int64_t n, int* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) out[t] = neg[t] ? -1 : 1;
}

}  // namespace

namespace {

int krill_ws_impl(krr_kernel_kind kind, krr_precision prec, int64_t N, int32_t d, int32_t k,
                  int32_t sketch_rows, int32_t zeta, int32_t m_max, bool stored, size_t* bytes) {
  KRR_TRY(check_kernel(kind, 1.0, prec));
  if (!bytes) {
    set_error("bytes is NULL");
    return KRR_EINVAL;
  }
  Precond P;
  KRR_TRY(krill_params(P, kind, prec, N, d, k, sketch_rows, zeta, m_max));
  P.stored = stored;
  Arena a;
  KRR_TRY(krill_layout(a, P));
  *bytes = a.used;
  return KRR_OK;
}

int krill_build_impl(krr_kernel_kind kind, double sigma, krr_precision prec, const double* X,
                     int64_t N, int32_t d, double mu, const int64_t* centers, int32_t k,
                     int32_t sketch_rows, int32_t zeta, uint64_t seed, int32_t m_max, void* ws,
                     size_t ws_bytes, bool stored, krr_precond* out, hipStream_t stream) {
  KRR_TRY(check_kernel(kind, sigma, prec));
  if (!out || !X) {
    set_error("NULL argument");
    return KRR_EINVAL;
  }
  if (!(mu > 0.0) || !std::isfinite(mu)) {
    set_error("mu must be positive and finite");
    return KRR_EINVAL;
  }
  *out = nullptr;
  krr_precond h = new (std::nothrow) krr_precond_s;
  if (!h) {
    set_error("out of host memory");
    return KRR_EINVAL;
  }
  Precond& P = h->P;
  int rc = krill_params(P, kind, prec, N, d, k, sketch_rows, zeta, m_max);
  if (rc == KRR_OK) {
    P.sigma = sigma;
    P.mu = mu;
    P.seed = seed;
    P.stored = stored;
    Arena meas;
    rc = krill_layout(meas, P);
    if (rc == KRR_OK) rc = finish_carve(P, ws, ws_bytes, meas.used);
    if (rc == KRR_OK) {
      Arena a(ws, ws_bytes);
      rc = krill_layout(a, P);
    }
    if (rc == KRR_OK) rc = krill_build(P, X, centers, stream);
  }
  if (rc != KRR_OK) {
    krr_precond_free(h);
    return rc;
  }
  *out = h;
  return KRR_OK;
}

}  // namespace

extern "C" int krr_krill_ws(krr_kernel_kind kind, krr_precision prec, int64_t N, int32_t d,
                            int32_t k, int32_t sketch_rows, int32_t zeta, int32_t m_max,
                            size_t* bytes) {
  return krill_ws_impl(kind, prec, N, d, k, sketch_rows, zeta, m_max, false, bytes);
}

extern "C" int krr_krill_build(krr_kernel_kind kind, double sigma, krr_precision prec,
                               const double* X, int64_t N, int32_t d, double mu,
                               const int64_t* centers, int32_t k, int32_t sketch_rows,
                               int32_t zeta, uint64_t seed, int32_t m_max, void* ws,
                               size_t ws_bytes, krr_precond* out, hipStream_t stream) {
  return krill_build_impl(kind, sigma, prec, X, N, d, mu, centers, k, sketch_rows, zeta, seed,
                          m_max, ws, ws_bytes, false, out, stream);
}

extern "C" int krr_krill_stored_ws(krr_kernel_kind kind, krr_precision prec, int64_t N,
                                   int32_t d, int32_t k, int32_t sketch_rows, int32_t zeta,
                                   int32_t m_max, size_t* bytes) {
  return krill_ws_impl(kind, prec, N, d, k, sketch_rows, zeta, m_max, true, bytes);
}

extern "C" int krr_krill_build_stored(krr_kernel_kind kind, double sigma, krr_precision prec,
                                      const double* X, int64_t N, int32_t d, double mu,
                                      const int64_t* centers, int32_t k, int32_t sketch_rows,
                                      int32_t zeta, uint64_t seed, int32_t m_max, void* ws,
                                      size_t ws_bytes, krr_precond* out, hipStream_t stream) {
  return krill_build_impl(kind, sigma, prec, X, N, d, mu, centers, k, sketch_rows, zeta, seed,
                          m_max, ws, ws_bytes, true, out, stream);
}

extern "C" int krr_krill_export(krr_precond h, int32_t what, void* dst, size_t bytes,
                                hipStream_t stream) {
  KRR_TRY(valid_precond(h));
  Precond& P = h->P;
  if (P.type != kKrill) {
    set_error("not a KRILL preconditioner");
    return KRR_EINVAL;
  }
  const int64_t nz = P.N * P.zeta, kk = (int64_t)P.k * P.k;
  size_t need = 0;
  switch (what) {
    case 0:
    case 1: need = sizeof(int) * nz; break;
    case 2: need = sizeof(double) * (size_t)P.sketch_rows * P.k; break;
    case 3:
    case 4: need = sizeof(double) * kk; break;
    case 5:
      if (!P.stored) {
        set_error("export 5 needs a stored build (krr_krill_build_stored)");
        return KRR_EINVAL;
      }
      need = sizeof(double) * (size_t)P.N * P.k;
      break;
    default:
      set_error("unknown export %d", what);
      return KRR_EINVAL;
  }
  if (!dst || bytes < need) {
    set_error("export buffer too small: %zu < %zu", bytes, need);
    return KRR_EINVAL;
  }
  switch (what) {
    case 0:
      return hip_check(hipMemcpyAsync(dst, P.kw.rows, need, hipMemcpyDeviceToDevice, stream), "export");
    case 1:
      widen_signs<<<(unsigned)ceil_div(nz, 256), 256, 0, stream>>>(P.kw.neg, nz, (int*)dst);
      KRR_LAUNCH_CHECK("widen_signs");
      return KRR_OK;
    case 2:
      return hip_check(hipMemcpyAsync(dst, P.kw.B, need, hipMemcpyDeviceToDevice, stream), "export");
    case 3:
      return hip_check(hipMemcpyAsync(dst, P.H, need, hipMemcpyDeviceToDevice, stream), "export");
    case 5:
      return stored_export(P, static_cast<double*>(dst), stream);
    default:
      lower_copy<<<(unsigned)ceil_div(kk, 256), 256, 0, stream>>>(P.C, P.k, (double*)dst);
      KRR_LAUNCH_CHECK("lower_copy");
      return KRR_OK;
  }
}

struct krr_solve_s {
  Solve S;
};

extern "C" int krr_solve_begin(krr_precond h, const double* Y, int32_t m, double tol,
                               int32_t max_iter, krr_solve* out, hipStream_t stream) {
  KRR_TRY(precond_idle(h));
  Precond& P = h->P;
  if (!out || m < 1 || m > P.m_max || !Y || !(tol > 0.0) || max_iter < 0) {
    set_error("invalid arguments (m=%d, m_max=%d, tol=%g, max_iter=%d)", m, P.m_max, tol,
              max_iter);
    return KRR_EINVAL;
  }
  *out = nullptr;
  krr_solve q = new (std::nothrow) krr_solve_s;
  if (!q) {
    set_error("out of host memory");
    return KRR_EINVAL;
  }
  const int rc = solve_begin(q->S, P, Y, m, tol, max_iter, stream);
  if (rc < 0) {
    delete q;
    return rc;
  }
  P.solving = true;
  *out = q;
  return KRR_OK;
}

namespace {
void release_solve(krr_solve q) {
  if (q->S.P) q->S.P->solving = false;
  delete q;
}
}  // namespace

extern "C" int krr_solve_step(krr_solve* solves, int32_t n, int32_t* state, hipStream_t stream) {
  if (n < 0 || (n > 0 && (!solves || !state))) {
    set_error("invalid arguments");
    return KRR_EINVAL;
  }
  std::vector<Solve*> v;
  v.reserve(n);
  for (int32_t i = 0; i < n; ++i) {
    if (!solves[i]) {
      set_error("NULL solve at %d", i);
      return KRR_EINVAL;
    }
    v.push_back(&solves[i]->S);
  }
  const int rc = solve_step(v.data(), n, stream);
  for (int32_t i = 0; i < n; ++i)
    state[i] = v[i]->err < 0 ? v[i]->err : (v[i]->phase == kPhaseDone ? 1 : 0);
  return rc;
}

extern "C" int krr_solve_end(krr_solve q, double* beta, krr_solve_info* info, hipStream_t stream) {
  if (!q) {
    set_error("NULL solve");
    return KRR_EINVAL;
  }
  int rc = KRR_OK;
  if (q->S.err >= 0 && q->S.phase != kPhaseDone) {
    set_error("solve has not finished");
    rc = KRR_EINVAL;
  } else if (q->S.err >= 0 && !beta) {
    set_error("NULL beta");
    rc = KRR_EINVAL;
  } else {
    rc = solve_end(q->S, beta, info, stream);
  }
  release_solve(q);
  return rc;
}

extern "C" void krr_solve_free(krr_solve q) {
  if (q) release_solve(q);
}

// ---- out-of-sample prediction -------------------------------------------

namespace {
__global__ void gather_rows(const double* __restrict__ X, int d, const int64_t* __restrict__ idx,
                            int64_t k, double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < k * d) out[t] = X[idx[t / d] * d + t % d];
}

// bytes of the centre copy ahead of the product's own workspace
size_t predict_prefix(const Precond& P) {
  return P.type == kRPChol ? 0 : align_up(sizeof(double) * (size_t)P.k * P.d);
}
}  // namespace

extern "C" int krr_predict_ws(krr_precond h, krr_precision prec, int64_t ntest, int32_t m,
                              size_t* bytes) {
  KRR_TRY(valid_precond(h));
  const Precond& P = h->P;
  const int64_t nc = P.type == kRPChol ? P.N : P.k;
  KRR_TRY(validate_matvec(P.kind, P.sigma, prec, ntest, nc, P.d, m));
  if (!bytes) {
    set_error("bytes is NULL");
    return KRR_EINVAL;
  }
  *bytes = predict_prefix(P) + matvec_bytes(P.kind, prec, ntest, nc, P.d, m);
  return KRR_OK;
}

extern "C" int krr_predict(krr_precond h, krr_precision prec, const double* X,
                           const double* Xtest, int64_t ntest, const double* beta, int32_t m,
                           double* out, void* ws, size_t ws_bytes, hipStream_t stream) {
  KRR_TRY(valid_precond(h));
  const Precond& P = h->P;
  const int64_t nc = P.type == kRPChol ? P.N : P.k;
  KRR_TRY(validate_matvec(P.kind, P.sigma, prec, ntest, nc, P.d, m));
  if (ntest == 0) return KRR_OK;
  if (!X || !Xtest || !beta || !out) {
    set_error("NULL array argument");
    return KRR_EINVAL;
  }
  const size_t pre = predict_prefix(P);
  KRR_TRY(check_ws(ws, ws_bytes, pre + matvec_bytes(P.kind, prec, ntest, nc, P.d, m)));
  const double* Xc = X;
  if (P.type != kRPChol) {
    // restricted KRR predicts from the centres x^(s_1) .. x^(s_k)
    double* C = static_cast<double*>(ws);
    gather_rows<<<(unsigned)ceil_div(P.k * P.d, 256), 256, 0, stream>>>(X, P.d, P.centers, P.k, C);
    KRR_LAUNCH_CHECK("gather_rows");
    Xc = C;
  }
  return matvec_impl(P.kind, P.sigma, prec, Xtest, ntest, Xc, nc, P.d, beta, m, 0.0, out,
                     static_cast<char*>(ws) + pre, ws_bytes - pre, stream);
}
