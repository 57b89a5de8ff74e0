// Restricted products over a stored kernel block.  Sec. 4.1 keeps the N x k
// matrix A(:,S) in memory and applies it in every iteration; here it is
// evaluated once at build time into the caller's workspace (FP64, or FP32
// for FP32 tiles), after which each application of the restricted operator
// streams it from HBM instead of recomputing its entries:
//
//   w = A(S,:) (A(:,S) v)   (the caller adds H v)
//
// With one right-hand side and a row that fits a workgroup's registers, one
// pass reads every stored entry once: a 1024-thread workgroup owns a block of
// rows; for each row it forms t_i = A(i,:) v (fixed-order block reduction)
// and, with the row still in registers, adds A(i,:)^T t_i into its own
// partial column sums.  Otherwise two passes: t = A(:,S) v (one wave per
// row), then the column sums of A(:,S)^T t over row blocks.  Partial sums go
// to fixed slots and are added in a fixed order: bitwise reproducible.
//
// Layout: row i (point i) holds the k centre entries, zero padded to ld, a
// multiple of 8 (16-byte aligned rows in both element types).
#include "solver.h"
#include "exp64.h"
#include <algorithm>
#include <type_traits>

namespace krr {

namespace {

constexpr int kFillRows = 64;       // rows per workgroup of the fill kernel
constexpr int kFusedThreads = 1024; // threads of the single-pass workgroup
constexpr int kColsThreads = 256;

template <typename T>
struct Vec;
template <>
struct Vec<double> {
  static constexpr int kN = 2;
  typedef double2 type;
  static __device__ __forceinline__ double get(const double2& v, int e) { return e == 0 ? v.x : v.y; }
};
template <>
struct Vec<float> {
  static constexpr int kN = 4;
  typedef float4 type;
  static __device__ __forceinline__ double get(const float4& v, int e) {
    return (double)(e == 0 ? v.x : e == 1 ? v.y : e == 2 ? v.z : v.w);
  }
};

// A(i, c) = K(x_i, s_c) by direct differences: FP64 entries through the
// table-driven exp64, FP32 entries (FP32 points) through v_exp_f32.  Row
// points are wave-uniform; each thread owns one centre.
template <int KIND, typename T, int D>
__global__ __launch_bounds__(256) void kns_fill(const T* __restrict__ X, int64_t N,
                                                const T* __restrict__ C, int64_t k, int64_t ld,
                                                int64_t rows_per_block, double scale,
                                                T* __restrict__ out) {
  __shared__ double etab[kExpTable];
  if constexpr (std::is_same<T, double>::value) {
    exp64_table_fill(etab);
    __syncthreads();
  }
  const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (c >= ld) return;
  const int64_t cc = c < k ? c : k - 1;
  T y[D];
#pragma unroll
  for (int q = 0; q < D; ++q) y[q] = C[cc * D + q];
  const int64_t r0 = (int64_t)blockIdx.y * rows_per_block;
  const int64_t r1 = r0 + rows_per_block < N ? r0 + rows_per_block : N;
  for (int64_t i = r0; i < r1; ++i) {
    const T* __restrict__ x = X + i * D;
    T s = T(0);
#pragma unroll
    for (int q = 0; q < D; ++q) {
      const T t = x[q] - y[q];
      if (KIND == KRR_LAPLACE) s += __builtin_fabs(t);
      else s = t * t + s;
    }
    T e;
    if constexpr (std::is_same<T, double>::value) e = exp64(s * scale, etab);
    else e = __builtin_amdgcn_exp2f(s * (float)scale);
    out[i * ld + c] = c < k ? e : T(0);
  }
}

template <int KIND, typename T>
void* fill_pick(int D) {
  switch (D) {
    case 4: return (void*)&kns_fill<KIND, T, 4>;
    case 8: return (void*)&kns_fill<KIND, T, 8>;
    case 16: return (void*)&kns_fill<KIND, T, 16>;
    case 20: return (void*)&kns_fill<KIND, T, 20>;
    case 24: return (void*)&kns_fill<KIND, T, 24>;
    case 32: return (void*)&kns_fill<KIND, T, 32>;
    case 48: return (void*)&kns_fill<KIND, T, 48>;
    default: return (void*)&kns_fill<KIND, T, 64>;
  }
}

// Single pass, one right-hand side: U vectors of Vec<T>::kN columns per
// thread (column index (u * 1024 + tid) * kN + e), rows [r0, r1) of block g,
// v staged in LDS.  part[g * ld + j] = sum over the block's rows i of
// A(i, j) t_i with t_i = sum_j A(i, j) v_j (v has k entries, t has N).
constexpr int kFusedMaxLd = 16384;   // v in LDS: 128 KB of gfx950's 160 KB
template <typename T, int U>
__global__ __launch_bounds__(kFusedThreads) void kns_fused(const T* __restrict__ A, int64_t N,
                                                            int64_t k, int64_t ld,
                                                            int64_t rows_per_block,
                                                            const double* __restrict__ v,
                                                            double* __restrict__ t,
                                                            double* __restrict__ part) {
  typedef typename Vec<T>::type VT;
  constexpr int E = Vec<T>::kN;
  __shared__ double sv[kFusedMaxLd];
  __shared__ double red[2][kFusedThreads / 64];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  for (int64_t j = tid; j < ld; j += kFusedThreads) sv[j] = j < k ? v[j] : 0.0;
  double acc[U][E];
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int e = 0; e < E; ++e) acc[u][e] = 0.0;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
  const int64_t r1 = r0 + rows_per_block < N ? r0 + rows_per_block : N;
  // the next row's entries are loaded while the current row is reduced
  VT cur[U], nxt[U];
  auto load = [&](int64_t i, VT* dst) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t j = (int64_t)(u * kFusedThreads + tid) * E;
      dst[u] = j < ld ? *reinterpret_cast<const VT*>(A + i * ld + j) : VT{};
    }
  };
  if (r0 < r1) load(r0, cur);
  __syncthreads();  // sv is filled
  int par = 0;
  for (int64_t i = r0; i < r1; ++i) {
    if (i + 1 < r1) load(i + 1, nxt);
    double s = 0.0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = (u * kFusedThreads + tid) * E;
      if (j < ld) {
#pragma unroll
        for (int e = 0; e < E; ++e) s = __builtin_fma(Vec<T>::get(cur[u], e), sv[j + e], s);
      }
    }
    // fixed-order reduction: butterfly within the wave, then the waves in order
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if (lane == 0) red[par][wave] = s;
    __syncthreads();
    double ti = 0.0;
#pragma unroll
    for (int w = 0; w < kFusedThreads / 64; ++w) ti += red[par][w];
    par ^= 1;  // the other buffer is free: every thread passed this barrier
    if (tid == 0) t[i] = ti;
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int e = 0; e < E; ++e) acc[u][e] = __builtin_fma(Vec<T>::get(cur[u], e), ti, acc[u][e]);
#pragma unroll
    for (int u = 0; u < U; ++u) cur[u] = nxt[u];
  }
  double* __restrict__ out = part + (int64_t)blockIdx.x * ld;
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int64_t j = (int64_t)(u * kFusedThreads + tid) * E + e;
      if (j < ld) out[j] = acc[u][e];
    }
}

// Two passes, pass 1: t[c][i] = sum_j A(i, j) v[c][j] for c < m, one wave
// per row (grid-stride), lanes over columns, fixed butterfly reduction.
template <typename T, int M>
__global__ __launch_bounds__(256) void kns_rows(const T* __restrict__ A, int64_t N, int64_t k,
                                                int64_t ld, const double* __restrict__ v,
                                                int64_t ldv, int m, double* __restrict__ t,
                                                int64_t ldt) {
  typedef typename Vec<T>::type VT;
  constexpr int E = Vec<T>::kN;
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t i = wave; i < N; i += nw) {
    double s[M];
#pragma unroll
    for (int c = 0; c < M; ++c) s[c] = 0.0;
    for (int64_t j0 = (int64_t)lane * E; j0 < ld; j0 += 64 * E) {
      const VT a = *reinterpret_cast<const VT*>(A + i * ld + j0);
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int64_t j = j0 + e;
        if (j < k) {
          const double av = Vec<T>::get(a, e);
#pragma unroll
          for (int c = 0; c < M; ++c)
            if (c < m) s[c] = __builtin_fma(av, v[c * ldv + j], s[c]);
        }
      }
    }
#pragma unroll
    for (int c = 0; c < M; ++c) {
      double x = s[c];
      for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
      if (lane == 0 && c < m) t[c * ldt + i] = x;
    }
  }
}

// Two passes, pass 2 (and the FP64 right-hand side): column sums over row
// blocks, part[(g * M + c) * ld + j] = sum over rows i of block g of
// A(i, j) t(i, c), with t(i, c) = tp[i * trs + c * tcs] (any strides).
template <typename T, int M>
__global__ __launch_bounds__(kColsThreads) void kns_cols(const T* __restrict__ A, int64_t N,
                                                         int64_t ld, int64_t rows_per_block,
                                                         const double* __restrict__ tp,
                                                         int64_t trs, int64_t tcs, int m,
                                                         double* __restrict__ part) {
  typedef typename Vec<T>::type VT;
  constexpr int E = Vec<T>::kN;
  const int64_t j0 = ((int64_t)blockIdx.x * kColsThreads + threadIdx.x) * E;
  const int64_t g = blockIdx.y;
  const int64_t r0 = g * rows_per_block;
  const int64_t r1 = r0 + rows_per_block < N ? r0 + rows_per_block : N;
  double acc[E][M];
#pragma unroll
  for (int e = 0; e < E; ++e)
#pragma unroll
    for (int c = 0; c < M; ++c) acc[e][c] = 0.0;
  if (j0 < ld) {
    for (int64_t i = r0; i < r1; ++i) {
      const VT a = *reinterpret_cast<const VT*>(A + i * ld + j0);
#pragma unroll
      for (int c = 0; c < M; ++c) {
        if (c < m) {
          const double tv = tp[i * trs + c * tcs];
#pragma unroll
          for (int e = 0; e < E; ++e) acc[e][c] = __builtin_fma(Vec<T>::get(a, e), tv, acc[e][c]);
        }
      }
    }
#pragma unroll
    for (int c = 0; c < M; ++c)
      if (c < m)
#pragma unroll
        for (int e = 0; e < E; ++e) part[(g * M + c) * ld + j0 + e] = acc[e][c];
  }
}

// w[c * ldw + j] = sum over g = 0 .. G-1 of part[(g * Ms + c) * ld + j]
// (fixed order), j < k, c < m.
__global__ void kns_reduce(const double* __restrict__ part, int64_t G, int Ms, int64_t ld,
                           int64_t k, int m, double* __restrict__ w, int64_t ldw) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= k * m) return;
  const int c = (int)(t / k);
  const int64_t j = t % k;
  double s = 0.0;
  for (int64_t g = 0; g < G; ++g) s += part[(g * Ms + c) * ld + j];
  w[c * ldw + j] = s;
}

__global__ void kns_to_f64(const float* __restrict__ A, int64_t N, int64_t k, int64_t ld,
                           double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N * k) return;
  out[t] = (double)A[(t / k) * ld + t % k];
}
__global__ void kns_copy_f64(const double* __restrict__ A, int64_t N, int64_t k, int64_t ld,
                             double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= N * k) return;
  out[t] = A[(t / k) * ld + t % k];
}

// Shapes of the passes (functions of N, k and the element size only).
struct StoredPlan {
  int64_t ld;         // padded row length
  int fused_u;        // U of the single pass (0: the row does not fit; two passes)
  int64_t g1, rpb1;   // single pass: row blocks (one per CU) and rows per block
  int64_t g2, rpb2;   // column pass: row blocks and rows per block
};

int ms_of(int mc) { return mc == 1 ? 1 : mc <= 4 ? 4 : 16; }

StoredPlan stored_plan(int64_t N, int64_t k, int es) {
  StoredPlan p;
  p.ld = (k + 7) / 8 * 8;
  const int E = es == 8 ? 2 : 4;
  const int64_t u = ceil_div(p.ld, (int64_t)kFusedThreads * E);
  p.fused_u = (u <= 8 && p.ld <= kFusedMaxLd) ? (int)u : 0;
  const int64_t n = std::max<int64_t>(N, 1);
  p.rpb1 = ceil_div(n, std::min<int64_t>(n, 256));
  p.g1 = ceil_div(n, p.rpb1);
  // the column pass spreads about 2048 workgroups over the column chunks
  const int64_t chunks = ceil_div(p.ld, (int64_t)kColsThreads * E);
  p.rpb2 = ceil_div(n, std::max<int64_t>(1, std::min<int64_t>(n, ceil_div(2048, chunks))));
  p.g2 = ceil_div(n, p.rpb2);
  return p;
}

template <typename T, int U>
void fused_u(const T* A, const Precond& P, const StoredPlan& pl, const double* v, double* t,
             hipStream_t s) {
  kns_fused<T, U><<<(unsigned)pl.g1, kFusedThreads, 0, s>>>(A, P.N, P.k, pl.ld, pl.rpb1, v, t,
                                                            P.kns_part);
}

template <typename T>
int launch_fused(const Precond& P, const StoredPlan& pl, const double* v, double* t, hipStream_t s) {
  const T* A = static_cast<const T*>(P.kns);
  switch (pl.fused_u) {
    case 1: fused_u<T, 1>(A, P, pl, v, t, s); break;
    case 2: fused_u<T, 2>(A, P, pl, v, t, s); break;
    case 3: fused_u<T, 3>(A, P, pl, v, t, s); break;
    case 4: fused_u<T, 4>(A, P, pl, v, t, s); break;
    case 5: fused_u<T, 5>(A, P, pl, v, t, s); break;
    case 6: fused_u<T, 6>(A, P, pl, v, t, s); break;
    case 7: fused_u<T, 7>(A, P, pl, v, t, s); break;
    default: fused_u<T, 8>(A, P, pl, v, t, s); break;
  }
  KRR_LAUNCH_CHECK("kns_fused");
  return KRR_OK;
}

template <typename T, int M>
void launch_rows_m(const T* A, const Precond& P, const StoredPlan& pl, const double* v,
                   int64_t ldv, int m, double* t, int64_t ldt, hipStream_t s) {
  const unsigned grid = (unsigned)std::min<int64_t>(ceil_div(P.N, 4), 8192);
  kns_rows<T, M><<<grid, 256, 0, s>>>(A, P.N, P.k, pl.ld, v, ldv, m, t, ldt);
}

template <typename T, int M>
void launch_cols_m(const T* A, const Precond& P, const StoredPlan& pl, const double* tp,
                   int64_t trs, int64_t tcs, int m, hipStream_t s) {
  constexpr int E = Vec<T>::kN;
  dim3 g((unsigned)ceil_div(pl.ld, (int64_t)kColsThreads * E), (unsigned)pl.g2);
  kns_cols<T, M><<<g, kColsThreads, 0, s>>>(A, P.N, pl.ld, pl.rpb2, tp, trs, tcs, m, P.kns_part);
}

// w (k x mc, column stride ldw) = A^T (t), t column-major N x mc (or any strides)
template <typename T>
int cols_pass(const Precond& P, const StoredPlan& pl, const double* tp, int64_t trs, int64_t tcs,
              int mc, double* w, int64_t ldw, hipStream_t s) {
  const T* A = static_cast<const T*>(P.kns);
  const int Ms = ms_of(mc);
  if (Ms == 1) launch_cols_m<T, 1>(A, P, pl, tp, trs, tcs, mc, s);
  else if (Ms == 4) launch_cols_m<T, 4>(A, P, pl, tp, trs, tcs, mc, s);
  else launch_cols_m<T, 16>(A, P, pl, tp, trs, tcs, mc, s);
  KRR_LAUNCH_CHECK("kns_cols");
  kns_reduce<<<(unsigned)ceil_div(P.k * mc, 256), 256, 0, s>>>(P.kns_part, pl.g2, Ms, pl.ld, P.k,
                                                              mc, w, ldw);
  KRR_LAUNCH_CHECK("kns_reduce");
  return KRR_OK;
}

template <typename T>
int two_pass(const Precond& P, const StoredPlan& pl, const double* v, int64_t ldv, int m,
             double* t, double* w, int64_t ldw, hipStream_t s) {
  const T* A = static_cast<const T*>(P.kns);
  for (int c0 = 0; c0 < m; c0 += 16) {
    const int mc = std::min(16, m - c0);
    const double* vc = v + (int64_t)c0 * ldv;
    double* tc = t + (int64_t)c0 * P.N;
    if (mc == 1) launch_rows_m<T, 1>(A, P, pl, vc, ldv, mc, tc, P.N, s);
    else if (mc <= 4) launch_rows_m<T, 4>(A, P, pl, vc, ldv, mc, tc, P.N, s);
    else launch_rows_m<T, 16>(A, P, pl, vc, ldv, mc, tc, P.N, s);
    KRR_LAUNCH_CHECK("kns_rows");
    KRR_TRY(cols_pass<T>(P, pl, tc, 1, P.N, mc, w + (int64_t)c0 * ldw, ldw, s));
  }
  return KRR_OK;
}

}  // namespace

size_t stored_bytes(int64_t N, int64_t k, int es, int32_t m_max, size_t* part_bytes) {
  const StoredPlan pl = stored_plan(N, k, es);
  const int64_t g = std::max(pl.g1, pl.g2);
  if (part_bytes) *part_bytes = sizeof(double) * (size_t)g * ms_of(std::min(m_max, 16)) * pl.ld;
  return (size_t)N * pl.ld * es;
}

int stored_fill(Precond& P, hipStream_t s) {
  const bool f64 = P.kns_es == 8;
  const StoredPlan pl = stored_plan(P.N, P.k, P.kns_es);
  PointSet& X = f64 ? P.pts64 : P.pts;
  PointSet& C = f64 ? P.cpts64 : P.cpts;
  if (P.kind == KRR_GAUSSIAN) {
    // the product tiles' expansion writes the block where its guard admits
    // the problem (the same entries the recomputing tiles evaluate); the
    // norm maxima are learned here for that choice
    KRR_TRY(learn_norm_max(X, s));
    KRR_TRY(learn_norm_max(C, s));
    bool done = false;
    KRR_TRY(gauss_block_store(f64 ? KRR_FP64 : KRR_FP32, P.sigma, X, C, P.kns, pl.ld, &done, s));
    if (done) return KRR_OK;
  }
  const int D = X.dpad;
  const double log2e = 1.4426950408889634;
  const double scale = P.kind == KRR_LAPLACE ? -1.0 / P.sigma : -1.0 / (2.0 * P.sigma * P.sigma);
  int64_t rpb = std::max<int64_t>(kFillRows, ceil_div(P.N, 65535));
  dim3 g((unsigned)ceil_div(pl.ld, 256), (unsigned)ceil_div(P.N, rpb));
  if (f64) {
    void* fn = P.kind == KRR_LAPLACE ? fill_pick<KRR_LAPLACE, double>(D) : fill_pick<KRR_GAUSSIAN, double>(D);
    using Fn = void (*)(const double*, int64_t, const double*, int64_t, int64_t, int64_t, double, double*);
    reinterpret_cast<Fn>(fn)<<<g, 256, 0, s>>>(X.x64, P.N, C.x64, P.k, pl.ld, rpb, scale,
                                               static_cast<double*>(P.kns));
  } else {
    if (!X.x32 || !C.x32) {
      set_error("stored kernel block: FP32 point layouts missing");
      return KRR_EINVAL;
    }
    void* fn = P.kind == KRR_LAPLACE ? fill_pick<KRR_LAPLACE, float>(D) : fill_pick<KRR_GAUSSIAN, float>(D);
    using Fn = void (*)(const float*, int64_t, const float*, int64_t, int64_t, int64_t, double, float*);
    reinterpret_cast<Fn>(fn)<<<g, 256, 0, s>>>(X.x32, P.N, C.x32, P.k, pl.ld, rpb, scale * log2e,
                                               static_cast<float*>(P.kns));
  }
  KRR_LAUNCH_CHECK("kns_fill");
  return KRR_OK;
}

int stored_operator(const Precond& P, const double* v, int32_t m, double* t, double* w,
                    hipStream_t s) {
  const StoredPlan pl = stored_plan(P.N, P.k, P.kns_es);
  const bool f64 = P.kns_es == 8;
  void* tok = tile_timer_start(s);
  if (m == 1 && pl.fused_u) {
    KRR_TRY(f64 ? launch_fused<double>(P, pl, v, t, s) : launch_fused<float>(P, pl, v, t, s));
    kns_reduce<<<(unsigned)ceil_div(P.k, 256), 256, 0, s>>>(P.kns_part, pl.g1, 1, pl.ld, P.k, 1,
                                                           w, P.k);
    KRR_LAUNCH_CHECK("kns_reduce");
  } else {
    KRR_TRY(f64 ? two_pass<double>(P, pl, v, P.k, m, t, w, P.k, s)
                : two_pass<float>(P, pl, v, P.k, m, t, w, P.k, s));
  }
  tile_timer_stop(tok, s);
  return KRR_OK;
}

int stored_rhs(const Precond& P, const double* Y, int32_t m, double* B, hipStream_t s) {
  // B (k x m, column-major) = A(S,:) Y with Y row-major N x m; FP64 storage only
  const StoredPlan pl = stored_plan(P.N, P.k, 8);
  for (int c0 = 0; c0 < m; c0 += 16) {
    const int mc = std::min(16, m - c0);
    KRR_TRY(cols_pass<double>(P, pl, Y + c0, m, 1, mc, B + (int64_t)c0 * P.k, P.k, s));
  }
  return KRR_OK;
}

int stored_export(const Precond& P, double* dst, hipStream_t s) {
  const StoredPlan pl = stored_plan(P.N, P.k, P.kns_es);
  const int64_t tot = P.N * P.k;
  if (P.kns_es == 8)
    kns_copy_f64<<<(unsigned)ceil_div(tot, 256), 256, 0, s>>>(static_cast<const double*>(P.kns), P.N,
                                                              P.k, pl.ld, dst);
  else
    kns_to_f64<<<(unsigned)ceil_div(tot, 256), 256, 0, s>>>(static_cast<const float*>(P.kns), P.N,
                                                            P.k, pl.ld, dst);
  KRR_LAUNCH_CHECK("kns export");
  return KRR_OK;
}

}  // namespace krr
