// Restricted KRR with KRILL preconditioning (Sec. 2.2, Alg. 2) on gfx950:
// uniform centres, the sparse sign embedding, the sketch B = Phi A(:,S),
// the k x k matrix P = B^T B + H and its Cholesky factor.
//
// Readings (written out independently in the CPU reference):
//  * centres: the k indices with the smallest keys sm(sm(seed,2), i), ties
//    by index, in ascending index order (uniform without replacement);
//  * Phi column j: candidate rows below(sm(sm(sm(seed,3), j), t), d) for
//    t = 0, 1, ..., keeping the first zeta distinct ones; the sign of its
//    q-th nonzero is the top bit of sm(sm(sm(seed,4), j), q) (0 -> +);
//    values +-zeta^{-1/2};
//  * H = mu A(S,S) + N eps tr(A(S,S)) I with eps = 2^-52.
//
// B is formed without atomics on floating-point data: Phi is transposed
// into per-row lists sorted by point index, and each B row is a fixed-order
// signed sum of kernel rows, so the build is bitwise reproducible.
#include "solver.h"
#include "exp64.h"
#include "gauss_mfma.h"
#include <algorithm>
#include <chrono>
#include <cmath>

namespace krr {

namespace {

constexpr int kBlk = 1024;  // elements per block in the compaction passes
constexpr int kMaxCand = 1 << 16;
constexpr int kMaxDraws = 1 << 16;

__device__ __forceinline__ uint64_t mulhi64(uint64_t a, uint64_t b) { return __umul64hi(a, b); }

// ---- centres -------------------------------------------------------------

__global__ void key_flags(uint64_t ckey, int64_t N, uint64_t thresh, int* __restrict__ flags) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) flags[i] = sm64(ckey, (uint64_t)i) <= thresh ? 1 : 0;
}

// counts[b] = number of flags set in block b of kBlk elements
__global__ __launch_bounds__(256) void block_counts(const int* __restrict__ flags, int64_t n,
                                                    int* __restrict__ counts) {
  __shared__ int sh[256];
  const int64_t b0 = (int64_t)blockIdx.x * kBlk;
  int c = 0;
  for (int u = threadIdx.x; u < kBlk; u += 256) {
    const int64_t i = b0 + u;
    if (i < n) c += flags[i];
  }
  sh[threadIdx.x] = c;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) counts[blockIdx.x] = sh[0];
}

// exclusive scan of n ints into out[0..n] (out[n] = total) by one
// workgroup: thread t sums a contiguous segment, the 1024 segment sums are
// scanned in LDS, then each thread writes its segment's prefixes (integer
// sums: the result does not depend on the order)
constexpr int kScanThreads = 1024;
__global__ __launch_bounds__(kScanThreads) void scan_excl(const int* __restrict__ in, int64_t n,
                                                          int64_t* __restrict__ out) {
  __shared__ int64_t sh[kScanThreads];
  const int t = threadIdx.x;
  const int64_t per = (n + kScanThreads - 1) / kScanThreads;
  const int64_t b = t * per;
  const int64_t e = b + per < n ? b + per : n;
  int64_t seg = 0;
  for (int64_t i = b; i < e; ++i) seg += in[i];
  sh[t] = seg;
  __syncthreads();
  for (int w = 1; w < kScanThreads; w <<= 1) {
    const int64_t v = t >= w ? sh[t - w] : 0;
    __syncthreads();
    sh[t] += v;
    __syncthreads();
  }
  int64_t run = t > 0 ? sh[t - 1] : 0;
  for (int64_t i = b; i < e; ++i) {
    out[i] = run;
    run += in[i];
  }
  if (t == kScanThreads - 1) out[n] = sh[t];
}

// Stable compaction: out[offset[b] + rank within block] = i for flagged i.
__global__ __launch_bounds__(256) void compact(const int* __restrict__ flags, int64_t n,
                                               const int64_t* __restrict__ offs,
                                               int64_t* __restrict__ out) {
  __shared__ int sh[256];
  const int64_t b0 = (int64_t)blockIdx.x * kBlk;
  int64_t base = offs[blockIdx.x];
  for (int u0 = 0; u0 < kBlk; u0 += 256) {
    const int64_t i = b0 + u0 + threadIdx.x;
    const int f = (i < n) ? flags[i] : 0;
    sh[threadIdx.x] = f;
    __syncthreads();
    // inclusive scan in LDS (Hillis-Steele)
    for (int w = 1; w < 256; w <<= 1) {
      const int v = threadIdx.x >= w ? sh[threadIdx.x - w] : 0;
      __syncthreads();
      sh[threadIdx.x] += v;
      __syncthreads();
    }
    if (f) out[base + sh[threadIdx.x] - 1] = i;
    const int tot = sh[255];
    __syncthreads();
    base += tot;
  }
}

// keys[a] = the sampling key of candidate a
__global__ void cand_keys(const int64_t* __restrict__ cand, int64_t nc, uint64_t ckey,
                          uint64_t* __restrict__ keys) {
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (a < nc) keys[a] = sm64(ckey, (uint64_t)cand[a]);
}

// keep[a] = 1 if candidate a is among the k smallest (key, index) pairs: its
// rank counted against all candidates, staged through LDS 1024 at a time
constexpr int kRankStage = 1024;
__global__ __launch_bounds__(256) void rank_select(const int64_t* __restrict__ cand,
                                                   const uint64_t* __restrict__ keys, int64_t nc,
                                                   int64_t k, int* __restrict__ keep) {
  __shared__ uint64_t sk[kRankStage];
  __shared__ int64_t si[kRankStage];
  const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = a < nc;
  const uint64_t ka = valid ? keys[a] : 0;
  const int64_t ia = valid ? cand[a] : 0;
  int64_t rank = 0;
  for (int64_t b0 = 0; b0 < nc; b0 += kRankStage) {
    const int64_t L = nc - b0 < kRankStage ? nc - b0 : kRankStage;
    __syncthreads();  // the previous stage's reads are done
    for (int64_t u = threadIdx.x; u < L; u += blockDim.x) {
      sk[u] = keys[b0 + u];
      si[u] = cand[b0 + u];
    }
    __syncthreads();
    for (int64_t u = 0; u < L; ++u) rank += (sk[u] < ka || (sk[u] == ka && si[u] < ia)) ? 1 : 0;
  }
  if (valid) keep[a] = rank < k ? 1 : 0;
}

__global__ void gather_i64(const int64_t* __restrict__ src, const int64_t* __restrict__ pos,
                           int64_t n, int64_t* __restrict__ dst) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) dst[t] = src[pos[t]];
}

__global__ void gather_raw(const double* __restrict__ X, int d, const int64_t* __restrict__ idx,
                           int64_t cnt, double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= cnt * d) return;
  out[t] = X[idx[t / d] * d + t % d];
}

// ---- sparse sign embedding -----------------------------------------------

// rows[j*zeta + q], neg[j*zeta + q]; counts per sketch row (integer atomics:
// the totals do not depend on order).  err[0] is set if a column runs out of
// candidates.
__global__ void sketch_gen(int64_t N, int d_rows, int zeta, uint64_t rkey, uint64_t skey,
                           int* __restrict__ rows, int* __restrict__ neg,
                           int* __restrict__ row_count, int* __restrict__ err) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  const uint64_t kj = sm64(rkey, (uint64_t)j);
  const uint64_t ks = sm64(skey, (uint64_t)j);
  int* rj = rows + j * zeta;
  int got = 0;
  for (int t = 0; t < kMaxDraws && got < zeta; ++t) {
    const int r = (int)mulhi64(sm64(kj, (uint64_t)t), (uint64_t)d_rows);
    bool dup = false;
    for (int q = 0; q < got; ++q) dup |= (rj[q] == r);
    if (!dup) rj[got++] = r;
  }
  if (got < zeta) {
    atomicExch(err, 1);
    for (int q = got; q < zeta; ++q) rj[q] = 0;
  }
  for (int q = 0; q < zeta; ++q) {
    neg[j * zeta + q] = (int)(sm64(ks, (uint64_t)q) >> 63);
    atomicAdd(row_count + rj[q], 1);
  }
}

// entries[pos] = 2 j + neg for every nonzero, placed in its row's segment
// (order within a segment fixed afterwards by seg_sort).
__global__ void sketch_fill(int64_t N, int zeta, const int* __restrict__ rows,
                            const int* __restrict__ neg, const int64_t* __restrict__ offs,
                            int* __restrict__ cursor, int64_t* __restrict__ entries) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  for (int q = 0; q < zeta; ++q) {
    const int r = rows[j * zeta + q];
    const int slot = atomicAdd(cursor + r, 1);
    entries[offs[r] + slot] = 2 * j + neg[j * zeta + q];
  }
}

// Sorts each row segment ascending (entries are distinct): rank sort.
constexpr int kSegLds = 4096;
__global__ __launch_bounds__(256) void seg_sort(const int64_t* __restrict__ offs,
                                                int64_t* __restrict__ entries,
                                                int64_t* __restrict__ tmp) {
  __shared__ int64_t sh[kSegLds];
  const int64_t r = blockIdx.x;
  const int64_t b = offs[r], e = offs[r + 1];
  const int64_t L = e - b;
  if (L == 0) return;
  if (L == 1) {
    if (threadIdx.x == 0) tmp[b] = entries[b];
    return;
  }
  if (L <= kSegLds) {
    for (int64_t u = threadIdx.x; u < L; u += 256) sh[u] = entries[b + u];
    __syncthreads();
    for (int64_t u = threadIdx.x; u < L; u += 256) {
      const int64_t v = sh[u];
      int64_t rank = 0;
      for (int64_t w = 0; w < L; ++w) rank += sh[w] < v ? 1 : 0;
      tmp[b + rank] = v;
    }
  } else {
    for (int64_t u = threadIdx.x; u < L; u += 256) {
      const int64_t v = entries[b + u];
      int64_t rank = 0;
      for (int64_t w = 0; w < L; ++w) rank += entries[b + w] < v ? 1 : 0;
      tmp[b + rank] = v;
    }
  }
}

// row_of[e] = r for every entry of row r (one workgroup per row)
__global__ void entry_rows(const int64_t* __restrict__ offs, int* __restrict__ row_of) {
  const int64_t r = blockIdx.x;
  for (int64_t e = offs[r] + threadIdx.x; e < offs[r + 1]; e += blockDim.x) row_of[e] = (int)r;
}

// ---- sketch B = Phi A(:,S) ---------------------------------------------
// Lanes own centres (R per lane, in registers); the workgroup walks a range
// of sketch rows; each row's entries (point index and sign) are
// wave-uniform, read with scalar loads, and their points enter the VALU as
// SGPR operands.  B[r][c] = zeta^{-1/2} sum_e s_e K(x_{j_e}, c).
// Gaussian sketches run here only when the matrix-core sketch cannot serve
// them to the precision's accuracy (guard: the largest centred squared norms
// of points and centres; null for Laplace).
template <int KIND, typename T, int D, int R>
__global__ __launch_bounds__(256) void sketch_apply(const T* __restrict__ C, int64_t k,
                                                    const T* __restrict__ X,
                                                    const int64_t* __restrict__ offs,
                                                    const int64_t* __restrict__ entries,
                                                    int64_t d_rows, int rows_per_wg, T scale,
                                                    double inv_sqrt_zeta,
                                                    double* __restrict__ Bout,
                                                    const T* __restrict__ gmax_x,
                                                    const T* __restrict__ gmax_c, double s_nat) {
  __shared__ double etab[kExpTable];  // FP64 exp table (unused by FP32 sketches)
  if (gmax_x && !gauss_expansion_too_coarse<T>(s_nat, (double)*gmax_x, (double)*gmax_c, D)) return;
  if constexpr (sizeof(T) == 8) {
    exp64_table_fill(etab);
    __syncthreads();
  }
  const int lane = threadIdx.x;
  const int64_t c0 = (int64_t)blockIdx.x * 256 * R;
  T x[R][D];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    int64_t c = c0 + lane + 256 * q;
    if (c > k - 1) c = k - 1;
#pragma unroll
    for (int t = 0; t < D; ++t) x[q][t] = C[c * D + t];
  }
  const int64_t r0 = (int64_t)blockIdx.y * rows_per_wg;
  const int64_t r1 = (r0 + rows_per_wg < d_rows) ? r0 + rows_per_wg : d_rows;
  for (int64_t r = r0; r < r1; ++r) {
    const int64_t eb = offs[r], ee = offs[r + 1];
    double acc64[R];
#pragma unroll
    for (int q = 0; q < R; ++q) acc64[q] = 0.0;
    for (int64_t e0 = eb; e0 < ee; e0 += 64) {
      const int64_t e1 = (e0 + 64 < ee) ? e0 + 64 : ee;
      T acc[R];
#pragma unroll
      for (int q = 0; q < R; ++q) acc[q] = T(0);
      for (int64_t e = e0; e < e1; ++e) {
        const int64_t code = entries[e];
        const int64_t j = code >> 1;
        const T sgn = (code & 1) ? T(-1) : T(1);
        const T* __restrict__ y = X + j * D;
        T yv[D];
#pragma unroll
        for (int t = 0; t < D; ++t) yv[t] = y[t];
#pragma unroll
        for (int q = 0; q < R; ++q) {
          T s0 = T(0);
#pragma unroll
          for (int t = 0; t < D; ++t) {
            const T df = x[q][t] - yv[t];
            if (KIND == KRR_LAPLACE) s0 += (sizeof(T) == 4 ? (T)__builtin_fabsf((float)df) : (T)__builtin_fabs((double)df));
            else s0 += df * df;
          }
          T ev;
          if constexpr (sizeof(T) == 4) ev = __builtin_amdgcn_exp2f(s0 * scale);
          else ev = exp64(s0 * scale, etab);
          acc[q] += sgn * ev;
        }
      }
#pragma unroll
      for (int q = 0; q < R; ++q) acc64[q] += (double)acc[q];
    }
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const int64_t c = c0 + lane + 256 * q;
      if (c < k) Bout[r * k + c] = acc64[q] * inv_sqrt_zeta;
    }
  }
}

template <int KIND, typename T>
void* sketch_pick(int D) {
  switch (D) {
    case 4: return (void*)&sketch_apply<KIND, T, 4, 2>;
    case 8: return (void*)&sketch_apply<KIND, T, 8, 2>;
    case 16: return (void*)&sketch_apply<KIND, T, 16, 2>;
    case 20: return (void*)&sketch_apply<KIND, T, 20, 2>;
    case 24: return (void*)&sketch_apply<KIND, T, 24, 1>;
    case 32: return (void*)&sketch_apply<KIND, T, 32, 1>;
    case 48: return (void*)&sketch_apply<KIND, T, 48, 1>;
    default: return (void*)&sketch_apply<KIND, T, 64, 1>;
  }
}
int sketch_rpl(int D) { return D <= 20 ? 2 : 1; }

__global__ void set_identity(double* __restrict__ A, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n * n) A[t] = (t / n == t % n) ? 1.0 : 0.0;
}

__global__ void scale_add_diag(double* __restrict__ A, int64_t n, double a, double diag) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * n) return;
  double v = a * A[t];
  if (t / n == t % n) v += diag;
  A[t] = v;
}

}  // namespace

int krill_layout(Arena& a, Precond& P) {
  const int64_t N = P.N, k = P.k;
  KRR_TRY(carve_points(P.kind, KRR_FP64, N, P.d, a, &P.pts64));
  if (P.prec != KRR_FP64) KRR_TRY(carve_points(P.kind, P.prec, N, P.d, a, &P.pts));
  else P.pts = P.pts64;
  KRR_TRY(carve_points(P.kind, KRR_FP64, k, P.d, a, &P.cpts64));
  if (P.prec != KRR_FP64) KRR_TRY(carve_points(P.kind, P.prec, k, P.d, a, &P.cpts));
  else P.cpts = P.cpts64;
  if (P.sketch_prec != P.prec) {
    KRR_TRY(carve_points(P.kind, P.sketch_prec, N, P.d, a, &P.skpts));
    KRR_TRY(carve_points(P.kind, P.sketch_prec, k, P.d, a, &P.skcpts));
  }
  P.centers = a.take<int64_t>(k);
  P.H = a.take<double>((size_t)k * k);
  P.C = a.take<double>((size_t)k * k);
  P.Linv = a.take<double>((size_t)k * k);
  P.spec_m = spec_columns(P);
  pcg_carve(a, P.pcg, k, P.m_max, N, 0, P.spec_m);
  KrillWork& w = P.kw;
  const int64_t nblk = ceil_div(N, kBlk);
  w.flags = a.take<int>(N);
  w.counts = a.take<int>(nblk);
  w.offs = a.take<int64_t>(std::max<int64_t>(nblk, P.sketch_rows) + 1);
  w.cand = a.take<int64_t>(kMaxCand);
  w.craw = a.take<double>((size_t)k * P.d);
  w.rows = a.take<int>((size_t)N * P.zeta);
  w.neg = a.take<int>((size_t)N * P.zeta);
  w.row_count = a.take<int>(P.sketch_rows + 1);
  w.entries = a.take<int64_t>((size_t)N * P.zeta);
  w.tmp = a.take<int64_t>((size_t)N * P.zeta);
  w.B = a.take<double>((size_t)P.sketch_rows * k);
  w.ints = a.take<int>(4);
  if (P.stored) {
    P.kns_es = P.prec == KRR_FP64 ? 8 : 4;
    size_t part = 0;
    const size_t kb = stored_bytes(N, k, P.kns_es, P.m_max, &part);
    P.kns = a.take<char>(kb);
    P.kns_part = a.take<double>(part / sizeof(double));
  }
  // operator products take up to m_max + spec_m columns
  const int32_t mc = P.m_max + P.spec_m;
  const size_t ps = std::max(product_scratch_bytes(P.prec, N, k, mc),
                             product_scratch_bytes(P.prec, k, N, mc));
  const size_t ps64 = std::max(product_scratch_bytes(KRR_FP64, N, k, P.m_max),
                               product_scratch_bytes(KRR_FP64, k, N, P.m_max));
  const size_t gs = std::max(gemm_scratch_bytes(k, k, P.sketch_rows, true),
                             gemm_scratch_bytes(mc, k, k));
  const size_t sb = std::max(std::max(ps, ps64), gs) + kAlign;
  char* sc = a.take<char>(sb);
  P.scratch = Arena(sc, sb);
  return KRR_OK;
}

int krill_build(Precond& P, const double* X, const int64_t* centers, hipStream_t s) {
  using clk = std::chrono::steady_clock;
  const auto t0 = clk::now();
  const int64_t N = P.N, k = P.k;
  KrillWork& w = P.kw;
  KRR_TRY(fill_points(P.kind, KRR_FP64, X, nullptr, P.pts64, s));
  if (P.prec != KRR_FP64) KRR_TRY(fill_points(P.kind, P.prec, X, nullptr, P.pts, s));
  const bool own_sketch = P.sketch_prec != P.prec;
  if (own_sketch) KRR_TRY(fill_points(P.kind, P.sketch_prec, X, nullptr, P.skpts, s));

  // 1. centres
  if (centers) {
    KRR_TRY(hip_check(hipMemcpyAsync(P.centers, centers, sizeof(int64_t) * k,
                                     hipMemcpyDeviceToDevice, s), "centres"));
  } else {
    const uint64_t ckey = sm64(P.seed, kTagCenter);
    const int64_t nblk = ceil_div(N, kBlk);
    // expected count below the threshold: k + 6 sqrt(k) + 64 (never < k in practice)
    double want = (double)k + 6.0 * std::sqrt((double)k) + 64.0;
    int64_t nc = 0;
    for (int attempt = 0; attempt < 8; ++attempt) {
      const double frac = std::min(1.0, want / (double)N);
      const double tf = frac * 18446744073709551616.0;
      const uint64_t thresh = tf >= 18446744073709549568.0 ? ~0ull : (uint64_t)tf;
      key_flags<<<(unsigned)ceil_div(N, 256), 256, 0, s>>>(ckey, N, thresh, w.flags);
      KRR_LAUNCH_CHECK("key_flags");
      block_counts<<<(unsigned)nblk, 256, 0, s>>>(w.flags, N, w.counts);
      KRR_LAUNCH_CHECK("block_counts");
      scan_excl<<<1, kScanThreads, 0, s>>>(w.counts, nblk, w.offs);
      KRR_LAUNCH_CHECK("scan_excl");
      KRR_TRY(hip_check(hipMemcpyAsync(&nc, w.offs + nblk, sizeof(int64_t), hipMemcpyDeviceToHost, s),
                        "count"));
      KRR_TRY(hip_check(hipStreamSynchronize(s), "sync"));
      if (nc >= k || frac >= 1.0) break;
      want *= 1.5;
    }
    if (nc < k || nc > kMaxCand) {
      set_error("centre sampling: %lld candidates for k=%lld (limit %d)", (long long)nc,
                (long long)k, kMaxCand);
      return KRR_EINVAL;
    }
    compact<<<(unsigned)nblk, 256, 0, s>>>(w.flags, N, w.offs, w.cand);
    KRR_LAUNCH_CHECK("compact");
    // the keys go to w.tmp, which holds the selected positions only afterwards
    uint64_t* keys = reinterpret_cast<uint64_t*>(w.tmp);
    cand_keys<<<(unsigned)ceil_div(nc, 256), 256, 0, s>>>(w.cand, nc, ckey, keys);
    KRR_LAUNCH_CHECK("cand_keys");
    rank_select<<<(unsigned)ceil_div(nc, 256), 256, 0, s>>>(w.cand, keys, nc, k, w.flags);
    KRR_LAUNCH_CHECK("rank_select");
    const int64_t nb2 = ceil_div(nc, kBlk);
    block_counts<<<(unsigned)nb2, 256, 0, s>>>(w.flags, nc, w.counts);
    KRR_LAUNCH_CHECK("block_counts 2");
    scan_excl<<<1, kScanThreads, 0, s>>>(w.counts, nb2, w.offs);
    KRR_LAUNCH_CHECK("scan_excl 2");
    compact<<<(unsigned)nb2, 256, 0, s>>>(w.flags, nc, w.offs, w.tmp);  // positions in cand
    KRR_LAUNCH_CHECK("compact 2");
    gather_i64<<<(unsigned)ceil_div(k, 256), 256, 0, s>>>(w.cand, w.tmp, k, P.centers);
    KRR_LAUNCH_CHECK("gather centres");
  }
  P.centers_host.resize(k);
  KRR_TRY(hip_check(hipMemcpyAsync(P.centers_host.data(), P.centers, sizeof(int64_t) * k,
                                   hipMemcpyDeviceToHost, s), "centres D2H"));
  KRR_TRY(hip_check(hipStreamSynchronize(s), "sync"));
  for (int64_t i = 0; i < k; ++i)
    if (P.centers_host[i] < 0 || P.centers_host[i] >= N) {
      set_error("centre index %lld out of range", (long long)P.centers_host[i]);
      return KRR_EINVAL;
    }
  gather_raw<<<(unsigned)ceil_div(k * P.d, 256), 256, 0, s>>>(X, P.d, P.centers, k, w.craw);
  KRR_LAUNCH_CHECK("gather_raw");
  KRR_TRY(fill_points(P.kind, KRR_FP64, w.craw, shared_params(P.kind, KRR_FP64, P.pts64),
                      P.cpts64, s));
  if (P.prec != KRR_FP64)
    KRR_TRY(fill_points(P.kind, P.prec, w.craw, shared_params(P.kind, P.prec, P.pts), P.cpts, s));
  if (own_sketch)
    KRR_TRY(fill_points(P.kind, P.sketch_prec, w.craw,
                        shared_params(P.kind, P.sketch_prec, P.skpts), P.skcpts, s));
  // the point layouts of the sketch tiles
  const PointSet& skp = own_sketch ? P.skpts : P.pts;
  const PointSet& skc = own_sketch ? P.skcpts : P.cpts;
  const bool sk64 = P.sketch_prec == KRR_FP64;

  // 2. H = mu A_SS + N eps tr(A_SS) I  (tr(A_SS) = k: unit diagonal)
  KRR_TRY(kernel_block64(P.kind, P.sigma, P.cpts64, P.cpts64, P.H, k, s));
  P.shift = (double)N * kEps * (double)k;
  scale_add_diag<<<(unsigned)ceil_div(k * k, 256), 256, 0, s>>>(P.H, k, P.mu, P.shift);
  KRR_LAUNCH_CHECK("scale_add_diag");

  // stored mode: A(:,S) evaluated once, in the tile precision
  if (P.stored) KRR_TRY(stored_fill(P, s));

  // 3. sparse sign embedding and its row lists
  const int ds = P.sketch_rows, z = P.zeta;
  KRR_TRY(hip_check(hipMemsetAsync(w.row_count, 0, sizeof(int) * (ds + 1), s), "row counts"));
  KRR_TRY(hip_check(hipMemsetAsync(w.ints, 0, sizeof(int) * 4, s), "err"));
  sketch_gen<<<(unsigned)ceil_div(N, 256), 256, 0, s>>>(N, ds, z, sm64(P.seed, kTagSketchRow),
                                                         sm64(P.seed, kTagSketchSign), w.rows,
                                                         w.neg, w.row_count, w.ints);
  KRR_LAUNCH_CHECK("sketch_gen");
  scan_excl<<<1, kScanThreads, 0, s>>>(w.row_count, ds, w.offs);
  KRR_LAUNCH_CHECK("scan rows");
  KRR_TRY(hip_check(hipMemsetAsync(w.row_count, 0, sizeof(int) * (ds + 1), s), "cursor"));
  sketch_fill<<<(unsigned)ceil_div(N, 256), 256, 0, s>>>(N, z, w.rows, w.neg, w.offs,
                                                          w.row_count, w.entries);
  KRR_LAUNCH_CHECK("sketch_fill");
  seg_sort<<<(unsigned)ds, 256, 0, s>>>(w.offs, w.entries, w.tmp);
  KRR_LAUNCH_CHECK("seg_sort");
  int err = 0;
  KRR_TRY(hip_check(hipMemcpyAsync(&err, w.ints, sizeof(int), hipMemcpyDeviceToHost, s), "err"));
  KRR_TRY(hip_check(hipStreamSynchronize(s), "sync"));
  if (err) {
    set_error("sparse sign embedding: a column ran out of candidate rows");
    return KRR_EINVAL;
  }
  // the sorted row lists are in tmp

  // 4. B = Phi A(:, S)  (d_rows x k)
  {
    const int D = P.pts64.dpad;
    const int R = sketch_rpl(D);
    const int rows_per_wg = 8;
    dim3 g((unsigned)ceil_div(k, 256 * R), (unsigned)ceil_div(ds, rows_per_wg));
    const double log2e = 1.4426950408889634;
    const double izeta = 1.0 / std::sqrt((double)z);
    const bool gauss = P.kind == KRR_GAUSSIAN;
    const double s_nat = 1.0 / (2.0 * P.sigma * P.sigma);
    // Gaussian: the matrix-core sketch, unless its device-side guard sends
    // the problem to the direct differences below (each kernel skips the
    // other's case)
    if (gauss) {
      // the unsorted entries are no longer needed: their space holds row_of
      int* row_of = reinterpret_cast<int*>(w.entries);
      entry_rows<<<(unsigned)ds, 256, 0, s>>>(w.offs, row_of);
      KRR_LAUNCH_CHECK("entry_rows");
      KRR_TRY(sketch_gauss_mfma_launch(sk64 ? KRR_FP64 : KRR_FP32, P.sigma, skp, skc, w.offs,
                                       w.tmp, row_of, ds, izeta, w.B, s));
    }
    if (sk64) {
      const double sc = P.kind == KRR_LAPLACE ? -1.0 / P.sigma : -s_nat;
      void* fn = P.kind == KRR_LAPLACE ? sketch_pick<KRR_LAPLACE, double>(D)
                                       : sketch_pick<KRR_GAUSSIAN, double>(D);
      using Fn = void (*)(const double*, int64_t, const double*, const int64_t*, const int64_t*,
                          int64_t, int, double, double, double*, const double*, const double*,
                          double);
      reinterpret_cast<Fn>(fn)<<<g, 256, 0, s>>>(
          skc.x64, k, skp.x64, w.offs, w.tmp, ds, rows_per_wg, sc, izeta, w.B,
          gauss ? skp.xmax64 : nullptr, gauss ? skc.xmax64 : nullptr, s_nat);
    } else {
      const float sc = (float)(P.kind == KRR_LAPLACE ? -log2e / P.sigma : -log2e * s_nat);
      void* fn = P.kind == KRR_LAPLACE ? sketch_pick<KRR_LAPLACE, float>(D)
                                       : sketch_pick<KRR_GAUSSIAN, float>(D);
      using Fn = void (*)(const float*, int64_t, const float*, const int64_t*, const int64_t*,
                          int64_t, int, float, double, double*, const float*, const float*,
                          double);
      reinterpret_cast<Fn>(fn)<<<g, 256, 0, s>>>(
          skc.x32, k, skp.x32, w.offs, w.tmp, ds, rows_per_wg, sc, izeta, w.B,
          gauss ? skp.xmax32 : nullptr, gauss ? skc.xmax32 : nullptr, s_nat);
    }
    KRR_LAUNCH_CHECK("sketch_apply");
  }
  // 5. P = B^T B + H, 6. C = chol(P) (lower factor L, P = L L^T, C = L^T)
  KRR_TRY(hip_check(hipMemcpyAsync(P.C, P.H, sizeof(double) * k * k, hipMemcpyDeviceToDevice, s),
                    "P = H"));
  // lower-triangle tiles only: the Cholesky reads nothing above the diagonal
  KRR_TRY(gemm_f64_ex(true, false, k, k, ds, 1.0, w.B, k, w.B, k, 1.0, P.C, k, s, &P.scratch, true));
  // 7. with L^{-1} by a right-looking blocked solve on the identity, each
  // block row formed as soon as its block column of L is final (a second
  // stream): each apply of P^{-1} = L^{-T} L^{-1} is then two dense k x k
  // products streamed from HBM instead of two sequential triangular solves
  set_identity<<<(unsigned)ceil_div(k * k, 256), 256, 0, s>>>(P.Linv, k);
  KRR_LAUNCH_CHECK("set_identity");
  KRR_TRY(potrf_inverse_lower(k, P.C, k, w.ints + 1, P.Linv, k, s));
  int info = 0;
  KRR_TRY(hip_check(hipMemcpyAsync(&info, w.ints + 1, sizeof(int), hipMemcpyDeviceToHost, s), "info"));
  KRR_TRY(hip_check(hipStreamSynchronize(s), "sync"));
  if (info != 0) {
    set_error("Cholesky of the KRILL matrix failed at column %d", info);
    return KRR_ENOTSPD;
  }
  // the largest centred norms on the host: the solve's products choose
  // their tile there (no launch of the tile they do not need)
  KRR_TRY(learn_norm_max(P.pts64, s));
  KRR_TRY(learn_norm_max(P.cpts64, s));
  if (P.prec != KRR_FP64) {
    KRR_TRY(learn_norm_max(P.pts, s));
    KRR_TRY(learn_norm_max(P.cpts, s));
  } else {
    P.pts = P.pts64;
    P.cpts = P.cpts64;
  }
  P.build_seconds = std::chrono::duration<double>(clk::now() - t0).count();
  return KRR_OK;
}

}  // namespace krr
