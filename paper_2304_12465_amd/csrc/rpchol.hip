// Blocked RPCholesky (Appendix A, Alg. 3) on gfx950, the Woodbury factor of
// the Nystrom preconditioner of Alg. 1, and the FP64 kernel-column tile used
// by the build steps.
//
// Readings of the algorithm (identical rules are written out independently in
// the CPU reference):
//  * draws are i.i.d. with replacement: draw t of block b uses
//    u = u53(sm(sm(sm(seed, 1), b), t)) and picks the smallest index whose
//    inclusive prefix sum exceeds u*T; prefix sums follow a fixed order
//    (chunks of 1024 summed left to right, then a left-to-right running sum
//    of chunk totals) so both implementations round identically;
//  * the distinct draws are taken in ascending index order;
//  * the small Cholesky proceeds pivot by pivot and drops a pivot whose Schur
//    diagonal is <= eps * tr(A); dropped pivots create no column;
//  * after each block the drawn entries of the residual diagonal are set to
//    zero and the diagonal is clamped at zero;
//  * the loop stops early once the residual trace is <= eps * tr(A).
// The uniform and greedy pivot rules (Sec. 3.1) change only the block's
// draws: uniform draws through the same prefix rule on 0/1 pool weights
// (indices never drawn) and budgets r distinct draws; greedy takes the one
// index of the largest residual diagonal entry (smallest index among equal
// maxima) and stops once that entry is <= eps * tr(A).
#include "solver.h"
#include "exp64.h"
#include <algorithm>
#include <chrono>
#include <cmath>

namespace krr {

namespace {

constexpr int kChunk = 1024;
constexpr int kOffLds = 4096;  // chunk offsets staged in LDS up to this many

__global__ void fill_d(double* __restrict__ d, double v, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) d[t] = v;
}

// S[c] = ((0 + d[c*1024]) + d[c*1024+1]) + ... : one workgroup per chunk
// stages it in LDS (coalesced), then one thread adds it in index order.
__global__ __launch_bounds__(256) void chunk_sums(const double* __restrict__ d, int64_t n,
                                                  int64_t nch, double* __restrict__ S) {
  __shared__ double v[kChunk];
  const int64_t c = blockIdx.x;
  const int64_t i0 = c * kChunk;
  const int len = (int)((i0 + kChunk < n) ? kChunk : n - i0);
  for (int e = threadIdx.x; e < len; e += blockDim.x) v[e] = d[i0 + e];
  __syncthreads();
  if (threadIdx.x != 0) return;
  // the chain of additions is sequential; its operands are read from LDS
  // sixteen at a time ahead of it
  double s = 0.0;
  int e = 0;
  for (; e + 16 <= len; e += 16) {
    double w[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) w[u] = v[e + u];
#pragma unroll
    for (int u = 0; u < 16; ++u) s = __dadd_rn(s, w[u]);
  }
  for (; e < len; ++e) s = __dadd_rn(s, v[e]);
  S[c] = s;
}

// Largest d_i of each 1024-entry chunk and its index (the smallest among
// equal maxima): V[c], I[c].  The maximum is exact, so the result does not
// depend on the reduction order.
__device__ __forceinline__ bool arg_better(double v, int64_t i, double bv, int64_t bi) {
  return v > bv || (v == bv && i < bi);
}
__global__ __launch_bounds__(256) void chunk_argmax(const double* __restrict__ d, int64_t n,
                                                    double* __restrict__ V,
                                                    int64_t* __restrict__ I) {
  __shared__ double sv[256];
  __shared__ int64_t si[256];
  const int64_t c = blockIdx.x;
  const int64_t i0 = c * kChunk;
  const int64_t i1 = (i0 + kChunk < n) ? i0 + kChunk : n;
  double bv = -1.0;
  int64_t bi = n;
  for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x)
    if (arg_better(d[i], i, bv, bi)) {
      bv = d[i];
      bi = i;
    }
  sv[threadIdx.x] = bv;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w && arg_better(sv[threadIdx.x + w], si[threadIdx.x + w], sv[threadIdx.x],
                                      si[threadIdx.x])) {
      sv[threadIdx.x] = sv[threadIdx.x + w];
      si[threadIdx.x] = si[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    V[c] = sv[0];
    I[c] = si[0];
  }
}

// Over the chunks: out[0] = index of the largest d, vmax[0] = its value.
__global__ __launch_bounds__(256) void argmax_final(const double* __restrict__ V,
                                                    const int64_t* __restrict__ I, int64_t nch,
                                                    int64_t* __restrict__ out,
                                                    double* __restrict__ vmax) {
  __shared__ double sv[256];
  __shared__ int64_t si[256];
  double bv = -1.0;
  int64_t bi = INT64_MAX;
  for (int64_t c = threadIdx.x; c < nch; c += blockDim.x)
    if (arg_better(V[c], I[c], bv, bi)) {
      bv = V[c];
      bi = I[c];
    }
  sv[threadIdx.x] = bv;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w && arg_better(sv[threadIdx.x + w], si[threadIdx.x + w], sv[threadIdx.x],
                                      si[threadIdx.x])) {
      sv[threadIdx.x] = sv[threadIdx.x + w];
      si[threadIdx.x] = si[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = si[0];
    vmax[0] = sv[0];
  }
}

// O[0] = 0, O[c+1] = O[c] + S[c] (sequential, one thread).
__global__ void chunk_offsets(const double* __restrict__ S, int64_t nch, double* __restrict__ O) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double o = 0.0;
  O[0] = 0.0;
  for (int64_t c = 0; c < nch; ++c) {
    o = __dadd_rn(o, S[c]);
    O[c + 1] = o;
  }
}

__global__ __launch_bounds__(256) void draw_pivots(const double* __restrict__ d, int64_t n,
                                                   const double* __restrict__ O, int64_t nch,
                                                   uint64_t block_key, int count,
                                                   int64_t* __restrict__ out) {
  // one workgroup per draw t: binary search over the chunk offsets (staged
  // in LDS when they fit), then the chunk staged in LDS and scanned in index
  // order by one thread
  __shared__ double v[kChunk];
  __shared__ double so[kOffLds];
  __shared__ int64_t found;
  __shared__ int64_t last[256];
  const int t = blockIdx.x;
  const int tid = threadIdx.x;
  const bool staged = nch + 1 <= kOffLds;
  if (staged)
    for (int64_t c = tid; c <= nch; c += blockDim.x) so[c] = O[c];
  __syncthreads();
  const double* __restrict__ off = staged ? so : O;
  const double T = off[nch];
  const double u = u53(sm64(block_key, (uint64_t)t));
  const double thr = __dmul_rn(u, T);
  // smallest chunk c with O[c+1] > thr (every thread finds the same one)
  int64_t lo = 0, hi = nch;  // search in [lo, hi)
  while (lo < hi) {
    const int64_t mid = (lo + hi) / 2;
    if (off[mid + 1] > thr) hi = mid;
    else lo = mid + 1;
  }
  if (tid == 0) found = -1;
  if (lo < nch) {
    const int64_t i0 = lo * kChunk;
    const int len = (int)((i0 + kChunk < n) ? kChunk : n - i0);
    for (int e = tid; e < len; e += blockDim.x) v[e] = d[i0 + e];
    __syncthreads();
    if (tid == 0) {
      // the running sum is sequential; its operands are read from LDS
      // sixteen at a time ahead of it
      const double base = off[lo];
      double p = 0.0;
      int64_t hit = -1;
      for (int e = 0; e < len && hit < 0; e += 16) {
        double w[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) w[q] = e + q < len ? v[e + q] : 0.0;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          if (hit < 0 && e + q < len) {
            p = __dadd_rn(p, w[q]);
            if (__dadd_rn(base, p) > thr) hit = i0 + e + q;
          }
        }
      }
      found = hit;
    }
  }
  __syncthreads();
  if (found < 0) {
    // u*T rounded up to T: the last index with positive mass (0 if none)
    int64_t mine = -1;
    for (int64_t i = n - 1 - tid; i >= 0; i -= blockDim.x)
      if (d[i] > 0.0) {
        mine = i;
        break;
      }
    last[tid] = mine;
    __syncthreads();
    if (tid == 0) {
      int64_t best = -1;
      for (int q = 0; q < (int)blockDim.x; ++q) best = last[q] > best ? last[q] : best;
      found = best < 0 ? 0 : best;
    }
    __syncthreads();
  }
  if (tid == 0) out[t] = found;
}

// out[q][j] = K(A_q, B_j) in FP64, direct differences.  One thread per j;
// the row points A_q are wave-uniform (scalar loads).
template <int KIND, int D>
__global__ __launch_bounds__(256) void kblock64(const double* __restrict__ A, int64_t na,
                                                const double* __restrict__ B, int64_t nb,
                                                double scale, double* __restrict__ out,
                                                int64_t ld) {
  __shared__ double etab[kExpTable];
  exp64_table_fill(etab);
  __syncthreads();
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t jj = j < nb ? j : nb - 1;
  double y[D];
#pragma unroll
  for (int k = 0; k < D; ++k) y[k] = B[jj * D + k];
  const int64_t q0 = (int64_t)blockIdx.y * 16;
  const int64_t q1 = (q0 + 16 < na) ? q0 + 16 : na;
  for (int64_t q = q0; q < q1; ++q) {
    const double* __restrict__ a = A + q * D;
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const double t = a[k] - y[k];
      if (KIND == KRR_LAPLACE) s += __builtin_fabs(t);
      else s = __builtin_fma(t, t, s);
    }
    if (j < nb) out[q * ld + j] = exp64(s * scale, etab);
  }
}

template <int KIND>
void* kblock_pick(int D) {
  switch (D) {
    case 4: return (void*)&kblock64<KIND, 4>;
    case 8: return (void*)&kblock64<KIND, 8>;
    case 16: return (void*)&kblock64<KIND, 16>;
    case 20: return (void*)&kblock64<KIND, 20>;
    case 24: return (void*)&kblock64<KIND, 24>;
    case 32: return (void*)&kblock64<KIND, 32>;
    case 48: return (void*)&kblock64<KIND, 48>;
    default: return (void*)&kblock64<KIND, 64>;
  }
}
using KBlockFn = void (*)(const double*, int64_t, const double*, int64_t, double, double*, int64_t);

__global__ void gather_points(const double* __restrict__ X, int D, const int64_t* __restrict__ idx,
                              int64_t cnt, double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= cnt * D) return;
  const int64_t q = t / D;
  const int k = (int)(t % D);
  out[t] = X[idx[q] * D + k];
}

// out[q][k] = X[gap_row(q, N, ns)][k]  (ns x d, row-major)
__global__ void gather_strided(const double* __restrict__ X, int64_t N, int d, int64_t ns,
                               double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ns * d) return;
  const int64_t q = t / d;
  out[t] = X[gap_row(q, N, ns) * d + t % d];
}

// Fs[q][p] = FT[p][idx[q]]  (cnt x i, row-major)
__global__ void gather_cols(const double* __restrict__ FT, int64_t ldf, int64_t i,
                            const int64_t* __restrict__ idx, int64_t cnt,
                            double* __restrict__ Fs) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= cnt * i) return;
  const int64_t q = t / i, p = t % i;
  Fs[t] = FT[p * ldf + idx[q]];
}

// Pivot-by-pivot Cholesky of G(S',S') with the drop rule, in LDS.
// One array M holds G in its upper triangle (diagonal included); below the
// diagonal it holds, transposed, the rows of R of the accepted pivots
// (R(acc[a], q) at M[q][a], q >= acc[a] >= a) and the running Schur sums
// S(q3, q2) = sum_a R(a, q3) R(a, q2) at M[q3][q2] for the rows not yet
// reached (q < q2 < q3); the diagonal sums sit in dsum.  Each accepted
// pivot adds its rank-1 term to every sum at once (right-looking), so no
// thread runs a chain as long as the pivot count; each sum still takes its
// terms in acceptance order, one rounding per product and per addition,
// which is the left-looking order term for term.  Rows beyond the current
// pivot never overlap the R columns (a < na <= q < q2).  Outputs the lower
// factor of the accepted pivots, Lacc = R_acc^T (acc x acc, ld = ldl), the
// accepted positions and their count.
constexpr int kCholThreads = 1024;  // 32 x 32 threads over the Schur sums
static_assert(kBmax <= kCholThreads, "chol_drop: one thread per column");
__global__ __launch_bounds__(kCholThreads) void chol_drop(const double* __restrict__ GT, int64_t ldg,
                                                 const int64_t* __restrict__ sp, int bp,
                                                 double thresh, double* __restrict__ Lacc,
                                                 int ldl, int* __restrict__ acc_out,
                                                 int* __restrict__ acc_count) {
  __shared__ double M[kBmax][kBmax + 1];
  __shared__ double dsum[kBmax];
  __shared__ int64_t spl[kBmax];
  __shared__ int acc[kBmax];
  const int tid = threadIdx.x;
  for (int q = tid; q < bp; q += blockDim.x) {
    spl[q] = sp[q];
    dsum[q] = 0.0;
  }
  __syncthreads();
  // G(S'_q, S'_q2) for q2 >= q, zero below; eight loads in flight per thread
  const int nn = bp * bp;
  for (int e0 = 0; e0 < nn; e0 += 8 * kCholThreads) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * kCholThreads + tid;
      const int ec = e < nn ? e : nn - 1;
      v[u] = GT[(int64_t)(ec / bp) * ldg + spl[ec % bp]];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * kCholThreads + tid;
      if (e < nn) {
        const int q = e / bp, q2 = e % bp;
        M[q][q2] = q2 >= q ? v[u] : 0.0;
      }
    }
  }
  __syncthreads();
  const int ty = tid >> 5, tx = tid & 31;
  int na = 0;
  for (int q = 0; q < bp; ++q) {
    // every thread reads the same finished values, so all take the same
    // branch
    const double sd = __dsub_rn(M[q][q], dsum[q]);
    if (!(sd > thresh)) continue;
    const double r = sqrt(sd);
    for (int q2 = q + 1 + tid; q2 < bp; q2 += blockDim.x)
      M[q2][na] = __ddiv_rn(__dsub_rn(M[q][q2], M[q2][q]), r);  // M[q2][q] = S(q2, q)
    __syncthreads();
    // rank-1 update of the sums of the rows after q: thread (ty, tx) takes
    // rows i = q + 1 + ty (+32) and, in each, columns j = q + 1 + tx (+32)
    // up to i
    for (int i = q + 1 + ty; i < bp; i += 32) {
      const double ri = M[i][na];
      for (int j = q + 1 + tx; j <= i; j += 32) {
        const double t = __dmul_rn(ri, M[j][na]);
        if (j == i)
          dsum[i] = __dadd_rn(dsum[i], t);
        else
          M[i][j] = __dadd_rn(M[i][j], t);
      }
    }
    if (tid == 0) {
      M[q][na] = r;
      acc[na] = q;
    }
    __syncthreads();
    ++na;
  }
  // Lacc[a][b] = R(acc[b], acc[a]) = M[acc[a]][b] for b <= a
  for (int e = tid; e < na * na; e += blockDim.x) {
    const int a = e / na, b2 = e % na;
    Lacc[a * ldl + b2] = (b2 <= a) ? M[acc[a]][b2] : 0.0;
  }
  for (int a = tid; a < na; a += blockDim.x) acc_out[a] = acc[a];
  if (tid == 0) *acc_count = na;
}

// FT[i0 + a][j] = GT[acc[a]][j]
__global__ void copy_rows(const double* __restrict__ GT, int64_t ld, const int* __restrict__ acc,
                          int na, int64_t n, double* __restrict__ dst) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)na * n) return;
  const int64_t a = t / n, j = t % n;
  dst[a * n + j] = GT[(int64_t)acc[a] * ld + j];
}

// d[j] = max(d[j] - sum_a Fnew[a][j]^2, 0)
__global__ void d_update(double* __restrict__ d, const double* __restrict__ Fnew, int na,
                         int64_t n) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double s = 0.0;
  for (int a = 0; a < na; ++a) {
    const double f = Fnew[(int64_t)a * n + j];
    s += f * f;
  }
  const double v = d[j] - s;
  d[j] = v > 0.0 ? v : 0.0;
}

__global__ void zero_at(double* __restrict__ d, const int64_t* __restrict__ idx, int cnt) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < cnt) d[idx[t]] = 0.0;
}

__global__ void add_diag(double* __restrict__ A, int64_t n, int64_t lda, double v) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) A[t * lda + t] += v;
}

}  // namespace

int kernel_block64(krr_kernel_kind kind, double sigma, const PointSet& A, const PointSet& B,
                   double* out, int64_t ld, hipStream_t s) {
  if (A.n == 0 || B.n == 0) return KRR_OK;
  const double scale = kind == KRR_LAPLACE ? -1.0 / sigma : -1.0 / (2.0 * sigma * sigma);
  const int D = A.dpad;
  void* fn = kind == KRR_LAPLACE ? kblock_pick<KRR_LAPLACE>(D) : kblock_pick<KRR_GAUSSIAN>(D);
  dim3 g((unsigned)ceil_div(B.n, 256), (unsigned)ceil_div(A.n, 16));
  if (g.y > 65535) {
    set_error("kernel_block64: too many rows");
    return KRR_EINVAL;
  }
  reinterpret_cast<KBlockFn>(fn)<<<g, 256, 0, s>>>(A.x64, A.n, B.x64, B.n, scale, out, ld);
  KRR_LAUNCH_CHECK("kblock64");
  return KRR_OK;
}

int rpchol_layout(Arena& a, Precond& P) {
  KRR_TRY(carve_points(P.kind, KRR_FP64, P.N, P.d, a, &P.pts64));
  if (P.prec != KRR_FP64)
    KRR_TRY(carve_points(P.kind, P.prec, P.N, P.d, a, &P.pts));
  else
    P.pts = P.pts64;
  const int64_t N = P.N;
  P.QT = a.take<double>((size_t)P.r_req * N);
  P.core = a.take<double>((size_t)P.r_req * P.r_req);
  P.spec_m = spec_columns(P);
  pcg_carve(a, P.pcg, N, P.m_max, 0, P.r_req, P.spec_m);
  // MIXED: sampled rows for the residual-gap estimate of the refinement
  P.nsamp = P.prec == KRR_MIXED ? std::min<int64_t>(N, kGapRows) : 0;
  if (P.nsamp > 0) {
    P.samp_x = a.take<double>((size_t)P.nsamp * P.d);
    KRR_TRY(carve_points(P.kind, KRR_FP64, P.nsamp, P.d, a, &P.spts64));
    P.samp_w = a.take<double>((size_t)P.nsamp * P.m_max);
  }
  RPWork& w = P.rp;
  const int64_t nch = ceil_div(N, kChunk);
  w.d = a.take<double>(N);
  w.S = a.take<double>(nch);
  w.O = a.take<double>(nch + 1);
  w.draws = a.take<int64_t>(kBmax);
  w.sp = a.take<int64_t>(kBmax);
  w.GT = a.take<double>((size_t)P.B * N);
  w.Fs = a.take<double>((size_t)P.B * P.r_req);
  w.Lacc = a.take<double>((size_t)kBmax * kBmax);
  w.acc = a.take<int>(kBmax);
  w.ints = a.take<int>(4);
  w.spx = a.take<double>((size_t)kBmax * 64);
  w.pool = a.take<double>(N);
  w.S2 = a.take<double>(nch);
  w.O2 = a.take<double>(nch + 1);
  w.gi = a.take<int64_t>(nch);
  w.vmax = a.take<double>(1);
  // scratch for products, split-K GEMMs of the build and of the applies
  // iteration products take up to m_max + spec_m columns
  const size_t ps = product_scratch_bytes(P.prec, N, N, P.m_max + P.spec_m);
  const size_t ps64 = std::max(product_scratch_bytes(KRR_FP64, N, N, P.m_max),
                               product_scratch_bytes(KRR_FP64, P.nsamp, N, P.m_max));
  const size_t gs = std::max(gemm_scratch_bytes(P.m_max, P.r_req, N),
                             std::max(gemm_scratch_bytes(P.r_req, P.r_req, N, true),
                                      gemm_scratch_bytes(P.B, N, P.r_req)));
  const size_t sb = std::max(std::max(ps, ps64), gs) + kAlign;
  char* sc = a.take<char>(sb);
  P.scratch = Arena(sc, sb);
  return KRR_OK;
}

int rpchol_build(Precond& P, const double* X, hipStream_t s) {
  using clk = std::chrono::steady_clock;
  const auto t0 = clk::now();
  const int64_t N = P.N;
  const int64_t nch = ceil_div(N, kChunk);
  RPWork& w = P.rp;
  // fill the point layouts carved by rpchol_layout
  KRR_TRY(fill_points(P.kind, KRR_FP64, X, nullptr, P.pts64, s));
  if (P.prec != KRR_FP64) KRR_TRY(fill_points(P.kind, P.prec, X, nullptr, P.pts, s));
  if (P.nsamp > 0) {
    gather_strided<<<(unsigned)ceil_div(P.nsamp * P.d, 256), 256, 0, s>>>(X, N, P.d, P.nsamp,
                                                                         P.samp_x);
    KRR_LAUNCH_CHECK("gather_strided");
    KRR_TRY(fill_points(P.kind, KRR_FP64, P.samp_x, shared_params(P.kind, KRR_FP64, P.pts64),
                        P.spts64, s));
  }
  // d = diag(A): both kernels equal exp(0) = 1 on the diagonal
  fill_d<<<(unsigned)ceil_div(N, 256), 256, 0, s>>>(w.d, 1.0, N);
  KRR_LAUNCH_CHECK("fill_d");
  const int rule = P.rule;
  if (rule == KRR_PIVOT_UNIFORM) {
    fill_d<<<(unsigned)ceil_div(N, 256), 256, 0, s>>>(w.pool, 1.0, N);
    KRR_LAUNCH_CHECK("fill_d pool");
  }
  const double trA = (double)N;
  const double thresh = kEps * trA;
  const uint64_t kpiv = sm64(P.seed, kTagPivot);
  const int D = P.pts64.dpad;
  P.pivots.clear();
  int64_t i = 0;
  int64_t b = 0;
  std::vector<int64_t> sp;
  // pinned staging: [0, 64) total T, [64, 64 + 8 kBmax) draws, then the
  // accepted count and list, then the distinct draws for the upload
  double* hT = reinterpret_cast<double*>(w.hstage);
  int64_t* hdraws = reinterpret_cast<int64_t*>(w.hstage + 64);
  int* hints = reinterpret_cast<int*>(w.hstage + 64 + 8 * kBmax);
  int* hacc = hints + 16;
  int64_t* hsp = reinterpret_cast<int64_t*>(w.hstage + 128 + 8 * kBmax + 4 * kBmax);
  static_assert(128 + 8 * kBmax + 4 * kBmax + 8 * kBmax <= kHostStage, "staging bytes");
  int64_t ndrawn = 0;  // uniform rule: distinct indices drawn so far
  while ((rule == KRR_PIVOT_UNIFORM ? ndrawn : i) < P.r_req && b <= N) {
    // prefix tables, then the block's draws (they read the total on the
    // device); one readback of the total(s) and the draws
    chunk_sums<<<(unsigned)nch, 256, 0, s>>>(w.d, N, nch, w.S);
    KRR_LAUNCH_CHECK("chunk_sums");
    chunk_offsets<<<1, 1, 0, s>>>(w.S, nch, w.O);
    KRR_LAUNCH_CHECK("chunk_offsets");
    const int cnt = rule == KRR_PIVOT_GREEDY
                        ? 1
                        : (int)std::min<int64_t>(P.B, P.r_req - (rule == KRR_PIVOT_UNIFORM ? ndrawn : i));
    const double* aux = nullptr;  // pool total (uniform) or largest d (greedy)
    if (rule == KRR_PIVOT_UNIFORM) {
      chunk_sums<<<(unsigned)nch, 256, 0, s>>>(w.pool, N, nch, w.S2);
      KRR_LAUNCH_CHECK("chunk_sums pool");
      chunk_offsets<<<1, 1, 0, s>>>(w.S2, nch, w.O2);
      KRR_LAUNCH_CHECK("chunk_offsets pool");
      draw_pivots<<<(unsigned)cnt, 256, 0, s>>>(w.pool, N, w.O2, nch, sm64(kpiv, (uint64_t)b),
                                                             cnt, w.draws);
      KRR_LAUNCH_CHECK("draw_pivots pool");
      aux = w.O2 + nch;
    } else if (rule == KRR_PIVOT_GREEDY) {
      // w.S is free again once the offsets are formed
      chunk_argmax<<<(unsigned)nch, 256, 0, s>>>(w.d, N, w.S, w.gi);
      KRR_LAUNCH_CHECK("chunk_argmax");
      argmax_final<<<1, 256, 0, s>>>(w.S, w.gi, nch, w.draws, w.vmax);
      KRR_LAUNCH_CHECK("argmax_final");
      aux = w.vmax;
    } else {
      draw_pivots<<<(unsigned)cnt, 256, 0, s>>>(w.d, N, w.O, nch, sm64(kpiv, (uint64_t)b),
                                                             cnt, w.draws);
      KRR_LAUNCH_CHECK("draw_pivots");
    }
    KRR_TRY(hip_check(hipMemcpyAsync(hT, w.O + nch, sizeof(double), hipMemcpyDeviceToHost, s), "T"));
    if (aux)
      KRR_TRY(hip_check(hipMemcpyAsync(hT + 1, aux, sizeof(double), hipMemcpyDeviceToHost, s),
                        "rule total"));
    KRR_TRY(hip_check(hipMemcpyAsync(hdraws, w.draws, sizeof(int64_t) * cnt, hipMemcpyDeviceToHost, s),
                      "draws"));
    KRR_TRY(hip_check(hipStreamSynchronize(s), "sync"));
    if (!(hT[0] > thresh)) break;  // residual exhausted (exact recovery): the draws are unused
    if (rule == KRR_PIVOT_UNIFORM && !(hT[1] > 0.0)) break;     // every index drawn
    if (rule == KRR_PIVOT_GREEDY && !(hT[1] > thresh)) break;   // no pivot can be accepted
    sp.assign(hdraws, hdraws + cnt);
    std::sort(sp.begin(), sp.end());
    sp.erase(std::unique(sp.begin(), sp.end()), sp.end());
    const int bp = (int)sp.size();
    std::copy(sp.begin(), sp.end(), hsp);
    KRR_TRY(hip_check(hipMemcpyAsync(w.sp, hsp, sizeof(int64_t) * bp, hipMemcpyHostToDevice, s),
                      "S'"));
    // G^T = A(S', :) - F(S', 1:i) F(:, 1:i)^T
    gather_points<<<(unsigned)ceil_div((int64_t)bp * D, 256), 256, 0, s>>>(P.pts64.x64, D, w.sp, bp,
                                                                          w.spx);
    KRR_LAUNCH_CHECK("gather_points");
    PointSet sps;
    sps.n = bp;
    sps.d = P.d;
    sps.dpad = D;
    sps.x64 = w.spx;
    KRR_TRY(kernel_block64(P.kind, P.sigma, sps, P.pts64, w.GT, N, s));
    if (i > 0) {
      gather_cols<<<(unsigned)ceil_div((int64_t)bp * i, 256), 256, 0, s>>>(P.QT, N, i, w.sp, bp,
                                                                          w.Fs);
      KRR_LAUNCH_CHECK("gather_cols");
      KRR_TRY(gemm_f64(false, bp, N, i, -1.0, w.Fs, i, P.QT, N, 1.0, w.GT, N, s, &P.scratch));
    }
    chol_drop<<<1, kCholThreads, 0, s>>>(w.GT, N, w.sp, bp, thresh, w.Lacc, kBmax, w.acc, w.ints);
    KRR_LAUNCH_CHECK("chol_drop");
    KRR_TRY(hip_check(hipMemcpyAsync(hints, w.ints, sizeof(int), hipMemcpyDeviceToHost, s), "acc"));
    KRR_TRY(hip_check(hipMemcpyAsync(hacc, w.acc, sizeof(int) * bp, hipMemcpyDeviceToHost, s),
                      "acc list"));
    KRR_TRY(hip_check(hipStreamSynchronize(s), "sync"));
    const int na = hints[0];
    if (na > 0) {
      double* Fnew = P.QT + i * N;
      copy_rows<<<(unsigned)ceil_div((int64_t)na * N, 256), 256, 0, s>>>(w.GT, N, w.acc, na, N, Fnew);
      KRR_LAUNCH_CHECK("copy_rows");
      // F_new^T = R_acc^{-T} G_acc^T
      KRR_TRY(trsm_lower_left(na, N, w.Lacc, kBmax, Fnew, N, s));
      d_update<<<(unsigned)ceil_div(N, 256), 256, 0, s>>>(w.d, Fnew, na, N);
      KRR_LAUNCH_CHECK("d_update");
    }
    zero_at<<<1, kBmax, 0, s>>>(w.d, w.sp, bp);
    KRR_LAUNCH_CHECK("zero_at");
    if (rule == KRR_PIVOT_UNIFORM) {
      zero_at<<<1, kBmax, 0, s>>>(w.pool, w.sp, bp);
      KRR_LAUNCH_CHECK("zero_at pool");
    }
    for (int a2 = 0; a2 < na; ++a2) P.pivots.push_back(sp[hacc[a2]]);
    i += na;
    ndrawn += bp;
    ++b;
  }
  P.rank = (int32_t)i;
  const int64_t rk = i;
  if (rk > 0) {
    // core = mu I + F^T F (its lower triangle: the Cholesky factorisation
    // reads nothing else), its Cholesky factor L, then Q^T = L^{-1} F^T in
    // place
    KRR_TRY(gemm_f64_ex(false, true, rk, rk, N, 1.0, P.QT, N, P.QT, N, 0.0, P.core, rk, s,
                        &P.scratch, true));
    add_diag<<<(unsigned)ceil_div(rk, 256), 256, 0, s>>>(P.core, rk, rk, P.mu);
    KRR_LAUNCH_CHECK("add_diag");
    KRR_TRY(potrf_lower(rk, P.core, rk, w.ints + 1, s));
    int info = 0;
    KRR_TRY(hip_check(hipMemcpyAsync(&info, w.ints + 1, sizeof(int), hipMemcpyDeviceToHost, s),
                      "info"));
    KRR_TRY(hip_check(hipStreamSynchronize(s), "sync"));
    if (info != 0) {
      set_error("Cholesky of mu I + F^T F failed at column %d", info);
      return KRR_ENOTSPD;
    }
    KRR_TRY(trsm_lower_left(rk, N, P.core, rk, P.QT, N, s));
  }
  KRR_TRY(hip_check(hipStreamSynchronize(s), "sync"));
  // the largest centred norms on the host: the solve's products choose
  // their tile there (no launch of the tile they do not need)
  KRR_TRY(learn_norm_max(P.pts64, s));
  if (P.prec != KRR_FP64) KRR_TRY(learn_norm_max(P.pts, s));
  else P.pts = P.pts64;
  if (P.nsamp > 0) KRR_TRY(learn_norm_max(P.spts64, s));
  P.build_seconds = std::chrono::duration<double>(clk::now() - t0).count();
  return KRR_OK;
}

}  // namespace krr
