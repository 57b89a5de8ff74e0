// VALU kernel tiles for the matrix-free product W = K(Xr, Xc) V (+ shift V).
//
// Design (gfx950, wave64):
//  * Each lane owns R rows of the output.  Its R points stay in VGPRs for
//    the whole launch; the wave sweeps a contiguous range of columns.
//  * A column's point and its V row are wave-uniform, so they are read with
//    scalar loads and enter VALU instructions as SGPR operands: no LDS
//    traffic and no VGPRs for column data.  Four waves of a workgroup walk
//    the same columns at the same time and share the scalar cache.
//  * Entries are computed by direct differences (Laplace: |x-y| summed;
//    Gaussian: (x-y)^2 summed), exponentiated and reduced against V at once:
//    the kernel matrix is never stored.
//  * FP32 tiles sum at most 256 columns in FP32, then fold into FP64
//    accumulators.  Per-split partial sums go to fixed slots and a second
//    kernel adds them in a fixed order, so results are bitwise reproducible
//    and independent of scheduling.
#include "product.h"
#include "exp64.h"
#include <algorithm>
#include <mutex>
#include <type_traits>
#include <vector>

namespace krr {

namespace {

constexpr int kWaves = 4;           // waves per workgroup

__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float abs_t(float a) { return __builtin_fabsf(a); }
__device__ __forceinline__ double abs_t(double a) { return __builtin_fabs(a); }
constexpr int kFold = 256;          // FP32 columns per FP64 fold

// One work item: row group rg (kWaves waves x 64 lanes x R rows) against
// column split `split` of one product.
template <typename T>
struct TileJob {
  const T* Xr;
  const T* Xc;
  const T* Vc;
  const uint32_t* Qr;  // quantised points (Laplace FP32 / MIXED tiles)
  const uint32_t* Qc;
  const double* qp;    // [lo, S]
  double* part;
  int64_t nr, nc, per;
  int64_t item0;  // first work item of this job in the launch
  T scale;
  int nsplit;
};

constexpr int kMaxJobs = 8;  // products per launch (kernel-argument table)

template <typename T>
struct JobTable {
  TileJob<T> job[kMaxJobs];
  int njobs;
  int64_t total;
};

template <int KIND, typename T, int D, int M, int R>
__device__ __forceinline__ void tile_item(const T* __restrict__ Xr, int64_t nr,
                                          const T* __restrict__ Xc, const T* __restrict__ Vc,
                                          int64_t nc, T scale, int split, int64_t cols_per_split,
                                          int64_t rg, double* __restrict__ part, int nsplit,
                                          const double* __restrict__ etab) {
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int64_t row0 = (rg * kWaves + wave) * 64 * R;
  if (row0 >= nr) return;  // whole wave idle (wave-uniform)

  T x[R][D];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    int64_t i = row0 + lane + 64 * r;
    if (i > nr - 1) i = nr - 1;
#pragma unroll
    for (int k = 0; k < D; ++k) x[r][k] = Xr[i * D + k];
  }
  double acc64[R][M];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int c = 0; c < M; ++c) acc64[r][c] = 0.0;

  const int64_t j0 = (int64_t)split * cols_per_split;
  int64_t j1 = j0 + cols_per_split;
  if (j1 > nc) j1 = nc;

  for (int64_t jb = j0; jb < j1; jb += kFold) {
    const int64_t je = (jb + kFold < j1) ? jb + kFold : j1;
    T acc[R][M];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int c = 0; c < M; ++c) acc[r][c] = T(0);
#pragma unroll 2
    for (int64_t j = jb; j < je; ++j) {
      const T* __restrict__ xc = Xc + j * D;
      const T* __restrict__ vc = Vc + j * M;
      T y[D];
#pragma unroll
      for (int k = 0; k < D; ++k) y[k] = xc[k];
      T v[M];
#pragma unroll
      for (int c = 0; c < M; ++c) v[c] = vc[c];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        // two interleaved partial sums break the dependency chain
        T s0, s1 = T(0);
#pragma unroll
        for (int k = 0; k < D; k += 2) {
          const T t0 = x[r][k] - y[k];
          const T a0 = KIND == KRR_LAPLACE ? abs_t(t0) : t0 * t0;
          s0 = k == 0 ? a0 : (KIND == KRR_LAPLACE ? s0 + a0 : fma_t(t0, t0, s0));
          if (k + 1 < D) {
            const T t1 = x[r][k + 1] - y[k + 1];
            const T a1 = KIND == KRR_LAPLACE ? abs_t(t1) : t1 * t1;
            s1 = k == 0 ? a1 : (KIND == KRR_LAPLACE ? s1 + a1 : fma_t(t1, t1, s1));
          }
        }
        T e;
        if constexpr (sizeof(T) == 4) e = __builtin_amdgcn_exp2f((s0 + s1) * scale);
        else e = exp64((s0 + s1) * scale, etab);
#pragma unroll
        for (int c = 0; c < M; ++c) acc[r][c] = fma_t(e, v[c], acc[r][c]);
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int c = 0; c < M; ++c) acc64[r][c] += (double)acc[r][c];
  }
  double* __restrict__ out = part + (int64_t)split * nr * M;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    int64_t i = row0 + lane + 64 * r;
    if (i < nr) {
#pragma unroll
      for (int c = 0; c < M; ++c) out[i * M + c] = acc64[r][c];
    }
  }
}

// Occupancy floors for the VALU tiles (waves per SIMD the register budget
// must allow), set where the compiler's own budget leaves 1-2 waves and a
// same-box A/B on 100,000 points showed the floor to pay despite a register
// spill of 12-292 bytes per lane:
//   quantised Laplace, 16 right-hand sides, d = 16-24: 1 -> 2 waves, 46-49%
//   faster; d = 8 and 32 with 16, d = 16 with 8: 2 -> 3 waves, 10-21%;
//   FP64 Laplace, 16 right-hand sides, d >= 32: 1 -> 2 waves, 48%; d = 16
//   with 16 and d = 32 with 4: 2 -> 3 waves, 14-18%; d = 16 with 8: 3 -> 4
//   waves, 5%.
// Other shapes keep the compiler's budget (FP64 d = 8 with 16 and quantised
// d = 8 with 8 measured no gain; FP64 d = 32 with 8 would spill 676 bytes,
// with 1-2 over 560).
template <int D, int M>
constexpr int lapq_waves() {
  if ((D == 32 && M == 16) || (D == 16 && M == 8) || (D == 8 && M == 16)) return 3;
  if (M == 16 && D >= 16 && D <= 24) return 2;
  return 1;
}
template <typename T, int D, int M>
constexpr int valu_waves() {
  if (!std::is_same<T, double>::value) return 1;
  if (M == 16) return D >= 32 ? 2 : D == 16 ? 3 : 1;
  if (D == 16 && M == 8) return 4;
  return D == 32 && M == 4 ? 3 : 1;
}

template <int KIND, typename T, int D, int M, int R>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(valu_waves<T, D, M>())))
void tile_valu(const JobTable<T> tab) {
  __shared__ double etab[kExpTable];  // FP64 exp table (unused by FP32 tiles)
  if constexpr (sizeof(T) == 8) {
    exp64_table_fill(etab);
    __syncthreads();
  }
  for (int64_t w = blockIdx.x; w < xcd_slots(tab.total); w += gridDim.x) {
    const int64_t item = xcd_item(w, tab.total);
    if (item >= tab.total) continue;
    int jn = 0;
    while (jn + 1 < tab.njobs && item >= tab.job[jn + 1].item0) ++jn;
    const TileJob<T>& J = tab.job[jn];
    // row groups of one column split are consecutive items
    const int64_t local = item - J.item0;
    const int64_t nrg = (J.nr + kWaves * 64 * R - 1) / (kWaves * 64 * R);
    const int split = (int)(local / nrg);
    const int64_t rg = local % nrg;
    tile_item<KIND, T, D, M, R>(J.Xr, J.nr, J.Xc, J.Vc, J.nc, J.scale, split, J.per, rg, J.part,
                                J.nsplit, etab);
  }
}

// |x - y| + acc as one v_sad_u32: the empty asm keeps the compiler from
// reassociating the integer chain into max/min/sub/add3 sequences.
__device__ __forceinline__ uint32_t sad_u32(uint32_t x, uint32_t y, uint32_t acc) {
  uint32_t r = (x > y ? x - y : y - x) + acc;
  __asm__("" : "+v"(r));
  return r;
}

// Laplace tile on quantised coordinates: the l1 distance of a pair is the
// exact 32-bit sum of |q_x - q_y| (v_sad_u32, one instruction per
// coordinate with the column coordinate as an SGPR operand), converted to
// FP32 once and scaled by -log2(e) / (sigma S) inside exp2.
template <int D, int M, int R>
__device__ __forceinline__ void tile_item_q(const uint32_t* __restrict__ Qr, int64_t nr,
                                            const uint32_t* __restrict__ Qc,
                                            const float* __restrict__ Vc, int64_t nc,
                                            float scale, int split, int64_t cols_per_split,
                                            int64_t rg, double* __restrict__ part) {
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int64_t row0 = (rg * kWaves + wave) * 64 * R;
  if (row0 >= nr) return;
  uint32_t x[R][D];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    int64_t i = row0 + lane + 64 * r;
    if (i > nr - 1) i = nr - 1;
#pragma unroll
    for (int k = 0; k < D; ++k) x[r][k] = Qr[i * D + k];
  }
  double acc64[R][M];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int c = 0; c < M; ++c) acc64[r][c] = 0.0;
  const int64_t j0 = (int64_t)split * cols_per_split;
  int64_t j1 = j0 + cols_per_split;
  if (j1 > nc) j1 = nc;
  for (int64_t jb = j0; jb < j1; jb += kFold) {
    const int64_t je = (jb + kFold < j1) ? jb + kFold : j1;
    float acc[R][M];
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int c = 0; c < M; ++c) acc[r][c] = 0.f;
#pragma unroll 2
    for (int64_t j = jb; j < je; ++j) {
      const uint32_t* __restrict__ yc = Qc + j * D;
      const float* __restrict__ vc = Vc + j * M;
      uint32_t y[D];
#pragma unroll
      for (int k = 0; k < D; ++k) y[k] = yc[k];
      float v[M];
#pragma unroll
      for (int c = 0; c < M; ++c) v[c] = vc[c];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        // one chain per row (R rows give R independent chains); it starts
        // from an opaque zero so that every step stays a v_sad_u32
        uint32_t s0 = 0;
        __asm__("" : "+v"(s0));
#pragma unroll
        for (int k = 0; k < D; ++k) s0 = sad_u32(x[r][k], y[k], s0);
        const float e = __builtin_amdgcn_exp2f((float)s0 * scale);
#pragma unroll
        for (int c = 0; c < M; ++c) acc[r][c] = __builtin_fmaf(e, v[c], acc[r][c]);
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int c = 0; c < M; ++c) acc64[r][c] += (double)acc[r][c];
  }
  double* __restrict__ out = part + (int64_t)split * nr * M;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    int64_t i = row0 + lane + 64 * r;
    if (i < nr) {
#pragma unroll
      for (int c = 0; c < M; ++c) out[i * M + c] = acc64[r][c];
    }
  }
}

template <int D, int M, int R>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(lapq_waves<D, M>())))
void tile_lapq(const JobTable<float> tab) {
  for (int64_t w = blockIdx.x; w < xcd_slots(tab.total); w += gridDim.x) {
    const int64_t item = xcd_item(w, tab.total);
    if (item >= tab.total) continue;
    int jn = 0;
    while (jn + 1 < tab.njobs && item >= tab.job[jn + 1].item0) ++jn;
    const TileJob<float>& J = tab.job[jn];
    const int64_t local = item - J.item0;
    const int64_t nrg = (J.nr + kWaves * 64 * R - 1) / (kWaves * 64 * R);
    const float sc = (float)((double)J.scale / J.qp[1]);
    tile_item_q<D, M, R>(J.Qr, J.nr, J.Qc, J.Vc, J.nc, sc, (int)(local / nrg), J.per,
                         local % nrg, J.part);
  }
}

// W[i, c0+c] = sum_s part[s, i, c] + shift * Vs[i, c0+c], fixed order over s.
__global__ __launch_bounds__(256) void reduce_splits(const double* __restrict__ part, int nsplit,
                                                     int64_t nr, int M, int mc, int c0,
                                                     double shift, VecView Vs, VecOut W) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nr * mc) return;
  const int64_t i = t / mc;
  const int c = (int)(t % mc);
  double s = 0.0;
  for (int q = 0; q < nsplit; ++q) s += part[((int64_t)q * nr + i) * M + c];
  if (shift != 0.0) s += shift * Vs.p[i * Vs.rs + (int64_t)(c0 + c) * Vs.cs];
  W.p[i * W.rs + (int64_t)(c0 + c) * W.cs] = s;
}

// per-block min / max of all coordinates of up to two point sets
__global__ __launch_bounds__(256) void minmax_part(const double* __restrict__ X1, int64_t len1,
                                                   const double* __restrict__ X2, int64_t len2,
                                                   int64_t chunk, double* __restrict__ part) {
  __shared__ double smin[256], smax[256];
  const int64_t tot = len1 + len2;
  const int64_t b0 = (int64_t)blockIdx.x * chunk;
  const int64_t b1 = (b0 + chunk < tot) ? b0 + chunk : tot;
  double lo = 1.0e308, hi = -1.0e308;
  for (int64_t t = b0 + threadIdx.x; t < b1; t += 256) {
    const double v = t < len1 ? X1[t] : X2[t - len1];
    lo = v < lo ? v : lo;
    hi = v > hi ? v : hi;
  }
  smin[threadIdx.x] = lo;
  smax[threadIdx.x] = hi;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + w]);
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = smin[0];
    part[2 * blockIdx.x + 1] = smax[0];
  }
}

__global__ void minmax_final(const double* __restrict__ part, int nb, double qmax,
                             double* __restrict__ qp) {
  double lo = 1.0e308, hi = -1.0e308;
  for (int b = 0; b < nb; ++b) {
    lo = fmin(lo, part[2 * b]);
    hi = fmax(hi, part[2 * b + 1]);
  }
  const double range = hi - lo;
  qp[0] = lo;
  qp[1] = range > 0.0 ? qmax / range : 1.0;
}

// q = round((x - lo) S), clamped to [0, 2^qbits - 1]; padding stays 0
__global__ void pack_quant(const double* __restrict__ X, int64_t n, int d, int dpad,
                           const double* __restrict__ qp, double qmax,
                           uint32_t* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * dpad) return;
  const int64_t i = t / dpad;
  const int k = (int)(t % dpad);
  uint32_t q = 0;
  if (k < d) {
    double v = rint((X[i * d + k] - qp[0]) * qp[1]);
    v = v < 0.0 ? 0.0 : (v > qmax ? qmax : v);
    q = (uint32_t)v;
  }
  out[t] = q;
}

template <typename T>
__global__ void pack_pts(const double* __restrict__ X, int64_t n, int d, int dpad,
                         const double* __restrict__ centre, T* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * dpad) return;
  const int64_t i = t / dpad;
  const int k = (int)(t % dpad);
  double v = 0.0;
  if (k < d) v = X[i * d + k] - (centre ? centre[k] : 0.0);
  out[t] = (T)v;
}

// Vp[j, c] = V[j, c0 + c] for c < mc, 0 for mc <= c < M.
template <typename T>
__global__ void pack_vec(VecView V, int64_t n, int c0, int mc, int M, T* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * M) return;
  const int64_t j = t / M;
  const int c = (int)(t % M);
  out[t] = (c < mc) ? (T)V.p[j * V.rs + (int64_t)(c0 + c) * V.cs] : T(0);
}

constexpr int kDims[] = {4, 8, 16, 20, 24, 32, 48, 64};
constexpr int kMs[] = {1, 2, 4, 8, 16};

template <int D>
constexpr int rows_per_lane() { return D <= 32 ? 2 : 1; }

template <int KIND, typename T, int D, int M>
void* tile_ptr() {
  return reinterpret_cast<void*>(&tile_valu<KIND, T, D, M, rows_per_lane<D>()>);
}
template <typename T>
using TileFn = void (*)(const JobTable<T>);

// quantised tiles: more rows per lane give more independent SAD chains
// (dependent v_sad_u32 issued back to back need a wait state on gfx950)
template <int D>
constexpr int rows_per_lane_q() { return D <= 24 ? 4 : (D <= 48 ? 2 : 1); }
int rows_for_q(int D) { return D <= 24 ? 4 : (D <= 48 ? 2 : 1); }

template <int D, int M>
void* tileq_ptr() {
  return reinterpret_cast<void*>(&tile_lapq<D, M, rows_per_lane_q<D>()>);
}
template <int D>
void* pickq_m(int M) {
  switch (M) {
    case 1: return tileq_ptr<D, 1>();
    case 2: return tileq_ptr<D, 2>();
    case 4: return tileq_ptr<D, 4>();
    case 8: return tileq_ptr<D, 8>();
    default: return tileq_ptr<D, 16>();
  }
}
void* pickq_d(int D, int M) {
  switch (D) {
    case 4: return pickq_m<4>(M);
    case 8: return pickq_m<8>(M);
    case 16: return pickq_m<16>(M);
    case 20: return pickq_m<20>(M);
    case 24: return pickq_m<24>(M);
    case 32: return pickq_m<32>(M);
    case 48: return pickq_m<48>(M);
    default: return pickq_m<64>(M);
  }
}

template <int KIND, typename T, int D>
void* pick_m(int M) {
  switch (M) {
    case 1: return tile_ptr<KIND, T, D, 1>();
    case 2: return tile_ptr<KIND, T, D, 2>();
    case 4: return tile_ptr<KIND, T, D, 4>();
    case 8: return tile_ptr<KIND, T, D, 8>();
    default: return tile_ptr<KIND, T, D, 16>();
  }
}

template <int KIND, typename T>
void* pick_d(int D, int M) {
  switch (D) {
    case 4: return pick_m<KIND, T, 4>(M);
    case 8: return pick_m<KIND, T, 8>(M);
    case 16: return pick_m<KIND, T, 16>(M);
    case 20: return pick_m<KIND, T, 20>(M);
    case 24: return pick_m<KIND, T, 24>(M);
    case 32: return pick_m<KIND, T, 32>(M);
    case 48: return pick_m<KIND, T, 48>(M);
    default: return pick_m<KIND, T, 64>(M);
  }
}

int mpad(int m) { return m <= 1 ? 1 : m <= 2 ? 2 : m <= 4 ? 4 : m <= 8 ? 8 : 16; }

struct Split {
  int nsplit;
  int64_t per;
};

Split choose_split(int64_t nr, int64_t nc, int R) {
  const int64_t ns = split_count(nr, nc, (int64_t)kWaves * 64 * R, 128);
  return {(int)ns, ceil_div(std::max<int64_t>(nc, 1), ns)};
}

int rows_for_dpad(int D) { return D <= 32 ? 2 : 1; }

// Optional HIP-event timing of the product tiles (the dominant kernel).
struct TileTimer {
  std::mutex mu;
  bool on = false;
  struct Rec {
    hipEvent_t e0, e1;
    int vectors;
  };
  std::vector<Rec> ev;
  std::vector<hipEvent_t> pool;
  hipEvent_t get() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
};
TileTimer& timer() {
  static TileTimer t;
  return t;
}

}  // namespace

void* tile_timer_start(hipStream_t s, int vectors) {
  TileTimer& tt = timer();
  std::lock_guard<std::mutex> g(tt.mu);
  if (!tt.on) return nullptr;
  hipEvent_t e0 = tt.get(), e1 = tt.get();
  if (!e0 || !e1) return nullptr;
  (void)hipEventRecord(e0, s);
  tt.ev.push_back({e0, e1, vectors});
  return reinterpret_cast<void*>(tt.ev.size());  // 1-based index
}

void tile_timer_stop(void* token, hipStream_t s) {
  if (!token) return;
  TileTimer& tt = timer();
  std::lock_guard<std::mutex> g(tt.mu);
  const size_t i = reinterpret_cast<size_t>(token) - 1;
  if (i < tt.ev.size()) (void)hipEventRecord(tt.ev[i].e1, s);
}

void tile_timing_enable(bool on) {
  TileTimer& t = timer();
  std::lock_guard<std::mutex> g(t.mu);
  t.on = on;
}

int tile_timing_read(double* total_ms, int64_t* launches, int vectors, double* match_ms,
                     int64_t* match_launches) {
  TileTimer& t = timer();
  std::lock_guard<std::mutex> g(t.mu);
  double tot = 0.0, mt = 0.0;
  int64_t mn = 0;
  for (auto& rec : t.ev) {
    KRR_TRY(hip_check(hipEventSynchronize(rec.e1), "timing sync"));
    float ms = 0.f;
    KRR_TRY(hip_check(hipEventElapsedTime(&ms, rec.e0, rec.e1), "elapsed"));
    tot += ms;
    if (rec.vectors == vectors) {
      mt += ms;
      ++mn;
    }
    t.pool.push_back(rec.e0);
    t.pool.push_back(rec.e1);
  }
  if (total_ms) *total_ms = tot;
  if (launches) *launches = (int64_t)t.ev.size();
  if (match_ms) *match_ms = mt;
  if (match_launches) *match_launches = mn;
  t.ev.clear();
  return KRR_OK;
}

int padded_dim(int32_t d) {
  for (int D : kDims)
    if (d <= D) return D;
  return 0;
}

int mfma_kdim(int32_t d) { return (int)((d + 31) / 32 * 32); }

size_t pointset_bytes(krr_kernel_kind kind, krr_precision prec, int64_t n, int32_t d) {
  Arena a;
  PointSet ps;
  if (carve_points(kind, prec, n, d, a, &ps) != KRR_OK) return 0;
  return a.used;
}

int quant_bits(int D) {
  int lg = 0;
  while ((1 << lg) < D) ++lg;
  return std::min(30, 32 - lg);
}

int carve_points(krr_kernel_kind kind, krr_precision prec, int64_t n, int32_t d, Arena& arena,
                 PointSet* out) {
  const int D = padded_dim(d);
  if (D == 0) {
    set_error("dimension d=%d unsupported (1 <= d <= 64)", d);
    return KRR_EINVAL;
  }
  *out = PointSet();
  out->n = n;
  out->d = d;
  out->dpad = D;
  if (prec == KRR_FP64) {
    out->x64 = arena.take<double>((size_t)n * D);
    if (kind == KRR_GAUSSIAN) KRR_TRY(carve_f64c(n, D, arena, out));
    return KRR_OK;
  }
  if (prec == KRR_MIXED && kind == KRR_GAUSSIAN) {
    // the bf16 split, and the FP32 centred copy (same centre) that serves
    // the jobs whose expansion error bound is too coarse for the split
    KRR_TRY(carve_mixed(n, d, arena, out));
    return carve_f32c(n, D, arena, out);
  }
  out->x32 = arena.take<float>((size_t)n * D);
  if (prec == KRR_FP32 && kind == KRR_GAUSSIAN) KRR_TRY(carve_f32c(n, D, arena, out));
  if (kind == KRR_LAPLACE) {
    out->qbits = quant_bits(D);
    out->xq = arena.take<uint32_t>((size_t)n * D);
    out->qp = arena.take<double>(4);
    out->qpart = arena.take<double>(2 * 256);
  }
  return KRR_OK;
}

const double* shared_params(krr_kernel_kind kind, krr_precision prec, const PointSet& ps) {
  if (kind == KRR_LAPLACE) return prec == KRR_FP64 ? nullptr : ps.qp;
  return ps.centre;  // Gaussian FP64 (centred MFMA layout) and MIXED
}

int quant_params(const double* X1, int64_t n1, const double* X2, int64_t n2, int32_t d,
                 int32_t qbits, double* qpart, double* qp, hipStream_t s) {
  const int64_t tot = (n1 + n2) * d;
  const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(256, ceil_div(tot, 4096)));
  const int64_t chunk = ceil_div(std::max<int64_t>(tot, 1), nb);
  minmax_part<<<nb, 256, 0, s>>>(X1, n1 * d, X2, n2 * d, chunk, qpart);
  KRR_LAUNCH_CHECK("minmax_part");
  minmax_final<<<1, 1, 0, s>>>(qpart, nb, (double)((1u << qbits) - 1u), qp);
  KRR_LAUNCH_CHECK("minmax_final");
  return KRR_OK;
}

int fill_points(krr_kernel_kind kind, krr_precision prec, const double* X, const double* shared,
                const PointSet& ps, hipStream_t s) {
  const int64_t n = ps.n;
  if (n == 0) return KRR_OK;
  const int D = ps.dpad;
  const int64_t tot = n * D;
  if (X == nullptr) {
    set_error("fill_points: NULL points");
    return KRR_EINVAL;
  }
  if (prec == KRR_FP64) {
    if (!ps.x64) {
      set_error("fill_points: layout not carved");
      return KRR_EINVAL;
    }
    pack_pts<double><<<(unsigned)ceil_div(tot, 256), 256, 0, s>>>(X, n, ps.d, D, nullptr,
                                                                   const_cast<double*>(ps.x64));
    KRR_LAUNCH_CHECK("pack_pts<double>");
    if (kind == KRR_GAUSSIAN) return fill_f64c(X, shared, ps, s);
    return KRR_OK;
  }
  if (prec == KRR_MIXED && kind == KRR_GAUSSIAN) {
    if (!ps.xhi || !ps.xc32) {
      set_error("fill_points: layout not carved");
      return KRR_EINVAL;
    }
    KRR_TRY(fill_mixed(X, shared, ps, s));
    return fill_f32c(X, ps.centre, ps, s);
  }
  if (!ps.x32) {
    set_error("fill_points: layout not carved");
    return KRR_EINVAL;
  }
  // uncentred FP32 copy (KRILL's sketch); Gaussian tiles use the centred copy
  pack_pts<float><<<(unsigned)ceil_div(tot, 256), 256, 0, s>>>(X, n, ps.d, D, nullptr,
                                                                const_cast<float*>(ps.x32));
  KRR_LAUNCH_CHECK("pack_pts<float>");
  if (kind == KRR_LAPLACE) {
    double* qp = const_cast<double*>(ps.qp);
    if (shared) {
      if (shared != qp)
        KRR_TRY(hip_check(hipMemcpyAsync(qp, shared, 2 * sizeof(double), hipMemcpyDeviceToDevice, s),
                          "quant params"));
    } else {
      KRR_TRY(quant_params(X, n, nullptr, 0, ps.d, ps.qbits, ps.qpart, qp, s));
    }
    pack_quant<<<(unsigned)ceil_div(tot, 256), 256, 0, s>>>(
        X, n, ps.d, D, qp, (double)((1u << ps.qbits) - 1u), const_cast<uint32_t*>(ps.xq));
    KRR_LAUNCH_CHECK("pack_quant");
    return KRR_OK;
  }
  return fill_f32c(X, shared, ps, s);  // FP32 Gaussian: centred MFMA layout
}

int pack_points(krr_kernel_kind kind, krr_precision prec, const double* X, int64_t n, int32_t d,
                const double* centre, Arena& arena, PointSet* out, hipStream_t s) {
  KRR_TRY(carve_points(kind, prec, n, d, arena, out));
  if (arena.base == nullptr) return KRR_OK;  // measuring
  if (!arena.ok()) {
    set_error("workspace too small for the point layout");
    return KRR_EWORKSPACE;
  }
  return fill_points(kind, prec, X, centre, *out, s);
}

size_t product_scratch_bytes(krr_precision prec, int64_t nr, int64_t nc, int32_t m) {
  const size_t es = prec == KRR_FP64 ? 8 : 4;
  const int M = mpad(std::min(m, 16));
  // worst case over the row-per-lane choices (more rows per lane -> fewer
  // row groups -> more column splits)
  int64_t ns = 1;
  for (int R = 1; R <= 4; ++R) ns = std::max<int64_t>(ns, choose_split(nr, nc, R).nsplit);
  Arena a;
  a.take<char>((size_t)std::max<int64_t>(nc, 1) * M * es);
  a.take<double>((size_t)ns * std::max<int64_t>(nr, 1) * M);
  if (prec == KRR_MIXED) return std::max(a.used, product_mfma_scratch_bytes(nr, nc));
  if (prec == KRR_FP64) return std::max(a.used, product_f64mfma_scratch_bytes(nr, nc));
  if (prec == KRR_FP32) return std::max(a.used, product_f32mfma_scratch_bytes(nr, nc));
  return a.used;
}

namespace {

struct Family {
  bool f64;
  void* fn;
  std::vector<TileJob<float>> j32;
  std::vector<TileJob<double>> j64;
  int R;
};

template <typename T>
int launch_jobs(void* fn, const std::vector<TileJob<T>>& jobs, int R, hipStream_t s) {
  for (size_t j0 = 0; j0 < jobs.size(); j0 += kMaxJobs) {
    JobTable<T> tab{};
    int64_t total = 0;
    int nj = 0;
    for (size_t j = j0; j < jobs.size() && nj < kMaxJobs; ++j, ++nj) {
      tab.job[nj] = jobs[j];
      tab.job[nj].item0 = total;
      total += ceil_div(jobs[j].nr, (int64_t)kWaves * 64 * R) * jobs[j].nsplit;
    }
    tab.njobs = nj;
    tab.total = total;
    if (total == 0) continue;
    const unsigned grid = (unsigned)std::min<int64_t>(xcd_slots(total), kGridCap);
    void* tok = tile_timer_start(s);
    reinterpret_cast<TileFn<T>>(fn)<<<grid, 256, 0, s>>>(tab);
    KRR_LAUNCH_CHECK("tile_valu");
    tile_timer_stop(tok, s);
  }
  return KRR_OK;
}

}  // namespace

int product_group(const ProductReq* reqs, int n, hipStream_t s) {
  int mmax = 0;
  for (int q = 0; q < n; ++q) {
    const ProductReq& r = reqs[q];
    if (r.rows->dpad != r.cols->dpad) {
      set_error("row and column point sets differ in dimension");
      return KRR_EINVAL;
    }
    if (r.rows->n > 0) mmax = std::max(mmax, r.m);
  }
  std::vector<size_t> marks(n);
  for (int q = 0; q < n; ++q) marks[q] = reqs[q].scratch->used;
  const double log2e = 1.4426950408889634;
  for (int c0 = 0; c0 < mmax; c0 += 16) {
    std::vector<Family> fams;
    auto family = [&](bool f64, void* fn, int R) -> Family& {
      for (auto& f : fams)
        if (f.fn == fn) return f;
      fams.push_back(Family{f64, fn, {}, {}, R});
      return fams.back();
    };
    std::vector<MfmaJob> mjobs;
    std::vector<F64Job> fjobs;
    std::vector<F32Job> gjobs;
    std::vector<int> mreq;
    struct Pending {
      int q;
      double* part;
      int nsplit;
      int M;
      int mc;
      bool mfma;
    };
    std::vector<Pending> pend;
    for (int q = 0; q < n; ++q) {
      const ProductReq& r = reqs[q];
      const int64_t nr = r.rows->n, nc = r.cols->n;
      if (nr == 0 || r.m <= c0) continue;
      Arena& sc = *r.scratch;
      sc.used = marks[q];
      const int mc = std::min(16, r.m - c0);
      if (r.prec == KRR_FP64 && r.kind == KRR_GAUSSIAN) {
        F64Job fj;
        KRR_TRY(f64_prepare(r.sigma, *r.rows, *r.cols, r.V, c0, mc, sc, &fj, s));
        pend.push_back(Pending{q, fj.part, nc > 0 ? fj.nsplit : 0, mc, mc, true});
        if (nc > 0) fjobs.push_back(fj);
        continue;
      }
      if (r.prec == KRR_FP32 && r.kind == KRR_GAUSSIAN) {
        F32Job gj;
        KRR_TRY(f32_prepare(r.sigma, *r.rows, *r.cols, r.V, c0, mc, sc, &gj, s));
        pend.push_back(Pending{q, gj.part, nc > 0 ? gj.nsplit : 0, mc, mc, true});
        if (nc > 0) gjobs.push_back(gj);
        continue;
      }
      if (r.prec == KRR_MIXED && r.kind == KRR_GAUSSIAN) {
        MfmaJob mj;
        KRR_TRY(mfma_prepare(r.sigma, *r.rows, *r.cols, r.V, c0, mc, sc, &mj, s));
        pend.push_back(Pending{q, mj.part, nc > 0 ? mj.nsplit : 0, mc, mc, true});
        if (nc > 0) {
          mjobs.push_back(mj);
          mreq.push_back(q);
        }
        continue;
      }
      const int D = r.rows->dpad;
      const bool f64 = r.prec == KRR_FP64;
      const bool quantised = !f64 && r.kind == KRR_LAPLACE;
      const int R = quantised ? rows_for_q(D) : rows_for_dpad(D);
      const int M = mpad(mc);
      Split sp = choose_split(nr, nc, R);
      void* vp = f64 ? (void*)sc.take<double>((size_t)std::max<int64_t>(nc, 1) * M)
                     : (void*)sc.take<float>((size_t)std::max<int64_t>(nc, 1) * M);
      double* part = sc.take<double>((size_t)sp.nsplit * nr * M);
      if (!sc.ok()) {
        set_error("product scratch too small");
        return KRR_EWORKSPACE;
      }
      pend.push_back(Pending{q, part, nc > 0 ? sp.nsplit : 0, M, mc, false});
      if (nc == 0) continue;
      const int64_t tot = nc * M;
      if (f64) {
        pack_vec<double><<<(unsigned)ceil_div(tot, 256), 256, 0, s>>>(r.V, nc, c0, mc, M, (double*)vp);
        KRR_LAUNCH_CHECK("pack_vec");
        const double sc64 = r.kind == KRR_LAPLACE ? -1.0 / r.sigma : -1.0 / (2.0 * r.sigma * r.sigma);
        void* fn = pick_d<KRR_LAPLACE, double>(D, M);  // Gaussian FP64 runs on the MFMA tile
        TileJob<double> j{};
        j.Xr = r.rows->x64;
        j.Xc = r.cols->x64;
        j.Vc = (const double*)vp;
        j.part = part;
        j.nr = nr;
        j.nc = nc;
        j.per = sp.per;
        j.scale = sc64;
        j.nsplit = sp.nsplit;
        family(true, fn, R).j64.push_back(j);
      } else {
        pack_vec<float><<<(unsigned)ceil_div(tot, 256), 256, 0, s>>>(r.V, nc, c0, mc, M, (float*)vp);
        KRR_LAUNCH_CHECK("pack_vec");
        // Laplace under FP32 / MIXED: rows and columns share one quantisation
        // (the same qp buffer or identical copies); the row set's is used
        if (!r.rows->xq || !r.cols->xq) {
          set_error("Laplace FP32 tiles: quantised layout missing");
          return KRR_EINVAL;
        }
        const float sc32 = (float)(-log2e / r.sigma);
        void* fn = pickq_d(D, M);  // Gaussian FP32 runs on the MFMA tile
        TileJob<float> j{};
        j.Qr = r.rows->xq;
        j.Qc = r.cols->xq;
        j.qp = r.rows->qp;
        j.Xr = r.rows->x32;
        j.Xc = r.cols->x32;
        j.Vc = (const float*)vp;
        j.part = part;
        j.nr = nr;
        j.nc = nc;
        j.per = sp.per;
        j.scale = sc32;
        j.nsplit = sp.nsplit;
        family(false, fn, R).j32.push_back(j);
      }
    }
    for (auto& f : fams) {
      if (f.f64) KRR_TRY(launch_jobs<double>(f.fn, f.j64, f.R, s));
      else KRR_TRY(launch_jobs<float>(f.fn, f.j32, f.R, s));
    }
    if (!mjobs.empty()) KRR_TRY(mfma_launch(mjobs, s));
    if (!fjobs.empty()) KRR_TRY(f64_launch(fjobs, s));
    if (!gjobs.empty()) KRR_TRY(f32_launch(gjobs, s));
    for (const Pending& pd : pend) {
      const ProductReq& r = reqs[pd.q];
      const int64_t nr = r.rows->n;
      const int64_t tot = nr * pd.mc;
      reduce_splits<<<(unsigned)ceil_div(tot, 256), 256, 0, s>>>(pd.part, pd.nsplit, nr, pd.M,
                                                                 pd.mc, c0, r.shift, r.Vs, r.W);
      KRR_LAUNCH_CHECK("reduce_splits");
    }
  }
  for (int q = 0; q < n; ++q) reqs[q].scratch->used = marks[q];
  return KRR_OK;
}

int product(krr_kernel_kind kind, double sigma, krr_precision prec, const PointSet& rows,
            const PointSet& cols, VecView V, int32_t m, double shift, VecView Vs, VecOut W,
            Arena& scratch, hipStream_t s) {
  ProductReq r;
  r.kind = kind;
  r.sigma = sigma;
  r.prec = prec;
  r.rows = &rows;
  r.cols = &cols;
  r.V = V;
  r.m = m;
  r.shift = shift;
  r.Vs = Vs;
  r.W = W;
  r.scratch = &scratch;
  return product_group(&r, 1, s);
}

}  // namespace krr
