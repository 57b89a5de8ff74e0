// Gaussian kernel tiles in FP64 on the matrix cores (precision KRR_FP64).
//
// ||x - y||^2 = ||x||^2 + ||y||^2 - 2 x.y with the contraction on
// v_mfma_f64_16x16x4f64 over centred points (centring keeps the expansion's
// cancellation at ~2^-52 ||x||^2, far below the FP64 tolerance).  The
// distance MFMA starts from -||x||^2 / 2, so one FMA gives the exponent.
// exp runs on the VALU in FP64.  The reduction against V is a second f64
// MFMA: the distance output layout (lane l holds columns 4t + l/16 of row
// l % 16, t = 0..3) is exactly the A-operand layout of K-step t of the
// 16x16x4 MFMA, so no lane exchange is needed.  Sums stay FP64 throughout;
// per-split partials go to fixed slots (bitwise reproducible).
#include "product.h"
#include <algorithm>

namespace krr {

namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kRT64 = 2;     // 16-row tiles per wave
constexpr int kCols64 = 64;  // columns per LDS chunk (four 16-column tiles)

// v_mfma_f64_16x16x4f64 operand layout (wave64):
//   A (16 x 4): lane l holds A[l % 16][l / 16]
//   B (4 x 16): lane l holds B[l / 16][l % 16]
//   D (16 x 16): lane l, element t holds D[4 t + l / 16][l % 16]
template <int D>
__device__ __forceinline__ void f64_item(const F64Job& J, int64_t rg, int split) {
  constexpr int KS = D / 4;
  __shared__ double sY[kCols64][D + 1];
  __shared__ double sAy[kCols64];
  __shared__ double sV[kCols64][17];  // [column][rhs]

  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int g = lane >> 4, li = lane & 15;
  const int64_t nr = J.nr, nc = J.nc;
  const int M = J.M;
  const int64_t row0 = (rg * 4 + wave) * (16 * kRT64);

  double xb[kRT64][KS];  // B operand: X[i0 + li][4 ks + g]
  f64x4 cinit[kRT64];
#pragma unroll
  for (int rt = 0; rt < kRT64; ++rt) {
    int64_t i = row0 + rt * 16 + li;
    if (i > nr - 1) i = nr - 1;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) xb[rt][ks] = J.xc[i * D + 4 * ks + g];
    const double h = -0.5 * J.xn[i];
    cinit[rt] = f64x4{h, h, h, h};
  }
  // two accumulators per row tile (even / odd K steps of the V reduction)
  // keep independent MFMA chains in flight
  f64x4 acc[kRT64][2];
#pragma unroll
  for (int rt = 0; rt < kRT64; ++rt) {
    acc[rt][0] = f64x4{0.0, 0.0, 0.0, 0.0};
    acc[rt][1] = f64x4{0.0, 0.0, 0.0, 0.0};
  }
  const double s2 = 2.0 * J.s;

  const int64_t j0 = (int64_t)split * J.per;
  int64_t j1 = j0 + J.per;
  if (j1 > nc) j1 = nc;
  for (int64_t jb = j0; jb < j1; jb += kCols64) {
    const int ncol = (int)((j1 - jb < kCols64) ? j1 - jb : kCols64);
    __syncthreads();
    for (int e = tid; e < kCols64 * D; e += 256) {
      const int jj = e / D, k = e % D;
      sY[jj][k] = jj < ncol ? J.yc[(jb + jj) * D + k] : 0.0;
    }
    if (tid < kCols64) sAy[tid] = tid < ncol ? -J.s * J.yn[jb + tid] : -1.0e300;
    for (int e = tid; e < kCols64 * 16; e += 256) {
      const int jj = e / 16, c = e % 16;
      sV[jj][c] = (jj < ncol && c < M) ? J.v[(jb + jj) * 16 + c] : 0.0;
    }
    __syncthreads();
    if (row0 >= nr) continue;
#pragma unroll 1
    for (int ct = 0; ct < kCols64 / 16; ++ct) {
      double ya[KS];  // A operand: Y[j0 + li][4 ks + g]
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) ya[ks] = sY[ct * 16 + li][4 * ks + g];
      double ay[4], vb[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        ay[t] = sAy[ct * 16 + 4 * t + g];
        vb[t] = sV[ct * 16 + 4 * t + g][li];  // B of E.V step t: V[4t + g][c = li]
      }
      // distance chains of the row tiles, interleaved
      f64x4 dot[kRT64];
#pragma unroll
      for (int rt = 0; rt < kRT64; ++rt) dot[rt] = cinit[rt];
#pragma unroll
      for (int ks = 0; ks < KS; ++ks)
#pragma unroll
        for (int rt = 0; rt < kRT64; ++rt)
          dot[rt] = __builtin_amdgcn_mfma_f64_16x16x4f64(ya[ks], xb[rt][ks], dot[rt], 0, 0, 0);
      // dot[rt][t] = y_{4t+g} . x_{li} - ||x_{li}||^2 / 2
      double e[kRT64][4];
#pragma unroll
      for (int rt = 0; rt < kRT64; ++rt)
#pragma unroll
        for (int t = 0; t < 4; ++t) e[rt][t] = exp(__builtin_fma(dot[rt][t], s2, ay[t]));
      // A of E.V step t: lane l holds E[li][4t + g] (K index g)
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int rt = 0; rt < kRT64; ++rt)
          acc[rt][t & 1] = __builtin_amdgcn_mfma_f64_16x16x4f64(e[rt][t], vb[t], acc[rt][t & 1], 0, 0, 0);
    }
  }
  if (row0 >= nr) return;
  double* __restrict__ out = J.part + (int64_t)split * nr * 16;
#pragma unroll
  for (int rt = 0; rt < kRT64; ++rt)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      // E.V output: lane l, element t holds W[i0 + 4t + g][c = li]
      const int64_t i = row0 + rt * 16 + 4 * t + g;
      if (i < nr && li < M) out[i * 16 + li] = acc[rt][0][t] + acc[rt][1][t];
    }
}

constexpr int kMaxF64Jobs = 8;
struct F64Table {
  F64Job job[kMaxF64Jobs];
  int njobs;
  int64_t total;
};

template <int D>
__global__ __launch_bounds__(256) void tile_f64_gauss(const F64Table tab) {
  for (int64_t item = blockIdx.x; item < tab.total; item += gridDim.x) {
    int jn = 0;
    while (jn + 1 < tab.njobs && item >= tab.job[jn + 1].item0) ++jn;
    const F64Job& J = tab.job[jn];
    const int64_t local = item - J.item0;
    f64_item<D>(J, local / J.nsplit, (int)(local % J.nsplit));
  }
}

__global__ void pack_centred64(const double* __restrict__ X, int64_t n, int d, int dpad,
                               const double* __restrict__ centre, double* __restrict__ xc,
                               double* __restrict__ xn) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int k = 0; k < dpad; ++k) {
    const double v = k < d ? X[i * d + k] - centre[k] : 0.0;
    xc[i * dpad + k] = v;
    s += v * v;
  }
  xn[i] = s;
}

__global__ void pack_v64(VecView V, int64_t n, int c0, int mc, double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * 16) return;
  const int64_t j = t / 16;
  const int c = (int)(t % 16);
  out[t] = c < mc ? V.p[j * V.rs + (int64_t)(c0 + c) * V.cs] : 0.0;
}

struct FSplit {
  int nsplit;
  int64_t per;
};

FSplit f64_split(int64_t nr, int64_t nc) {
  const int64_t ns = split_count(nr, nc, 4 * 16 * kRT64, 256);
  int64_t per = ceil_div(std::max<int64_t>(nc, 1), ns);
  per = ceil_div(per, kCols64) * kCols64;
  return {(int)ns, per};
}

}  // namespace

int carve_f64c(int64_t n, int32_t dpad, Arena& arena, PointSet* out) {
  out->xc64 = arena.take<double>((size_t)n * dpad);
  out->xn64 = arena.take<double>(n);
  if (!out->centre) {
    out->centre = arena.take<double>(64);
    out->cpart = arena.take<double>(256 * 64);
  }
  return KRR_OK;
}

int fill_f64c(const double* X, const double* centre, const PointSet& ps, hipStream_t s) {
  const int64_t n = ps.n;
  if (n == 0) return KRR_OK;
  double* c = const_cast<double*>(ps.centre);
  if (centre) {
    if (centre != c)
      KRR_TRY(hip_check(hipMemcpyAsync(c, centre, sizeof(double) * ps.d, hipMemcpyDeviceToDevice, s),
                        "centre copy"));
  } else {
    KRR_TRY(compute_centre(X, n, ps.d, c, ps.cpart, s));
  }
  pack_centred64<<<(unsigned)ceil_div(n, 256), 256, 0, s>>>(X, n, ps.d, ps.dpad, c,
                                                            const_cast<double*>(ps.xc64),
                                                            const_cast<double*>(ps.xn64));
  KRR_LAUNCH_CHECK("pack_centred64");
  return KRR_OK;
}

size_t product_f64mfma_scratch_bytes(int64_t nr, int64_t nc) {
  FSplit sp = f64_split(nr, nc);
  Arena a;
  a.take<double>((size_t)std::max<int64_t>(nc, 1) * 16);
  a.take<double>((size_t)sp.nsplit * std::max<int64_t>(nr, 1) * 16);
  return a.used;
}

int f64_prepare(double sigma, const PointSet& rows, const PointSet& cols, VecView V, int c0, int mc,
                Arena& scratch, F64Job* out, hipStream_t s) {
  const int64_t nr = rows.n, nc = cols.n;
  if (!rows.xc64 || !cols.xc64 || rows.dpad != cols.dpad) {
    set_error("FP64 Gaussian product: centred layouts missing or inconsistent");
    return KRR_EINVAL;
  }
  FSplit sp = f64_split(nr, nc);
  double* v = scratch.take<double>((size_t)std::max<int64_t>(nc, 1) * 16);
  double* part = scratch.take<double>((size_t)sp.nsplit * nr * 16);
  if (!scratch.ok()) {
    set_error("FP64 product scratch too small");
    return KRR_EWORKSPACE;
  }
  if (nc > 0) {
    pack_v64<<<(unsigned)ceil_div(nc * 16, 256), 256, 0, s>>>(V, nc, c0, mc, v);
    KRR_LAUNCH_CHECK("pack_v64");
  }
  F64Job& j = *out;
  j.xc = rows.xc64;
  j.xn = rows.xn64;
  j.yc = cols.xc64;
  j.yn = cols.xn64;
  j.v = v;
  j.part = part;
  j.nr = nr;
  j.nc = nc;
  j.per = sp.per;
  j.item0 = 0;
  j.s = 1.0 / (2.0 * sigma * sigma);
  j.nsplit = sp.nsplit;
  j.M = mc;
  j.dpad = rows.dpad;
  return KRR_OK;
}

int f64_launch(const std::vector<F64Job>& jobs, hipStream_t s) {
  for (int D : {4, 8, 16, 20, 24, 32, 48, 64}) {
    std::vector<F64Job> sel;
    for (const F64Job& j : jobs)
      if (j.dpad == D) sel.push_back(j);
    for (size_t j0 = 0; j0 < sel.size(); j0 += kMaxF64Jobs) {
      F64Table tab{};
      int64_t total = 0;
      int nj = 0;
      for (size_t j = j0; j < sel.size() && nj < kMaxF64Jobs; ++j, ++nj) {
        tab.job[nj] = sel[j];
        tab.job[nj].item0 = total;
        total += ceil_div(sel[j].nr, (int64_t)4 * 16 * kRT64) * sel[j].nsplit;
      }
      tab.njobs = nj;
      tab.total = total;
      if (total == 0) continue;
      const unsigned grid = (unsigned)std::min<int64_t>(total, kGridCap);
      void* tok = tile_timer_start(s);
      switch (D) {
        case 4: tile_f64_gauss<4><<<grid, 256, 0, s>>>(tab); break;
        case 8: tile_f64_gauss<8><<<grid, 256, 0, s>>>(tab); break;
        case 16: tile_f64_gauss<16><<<grid, 256, 0, s>>>(tab); break;
        case 20: tile_f64_gauss<20><<<grid, 256, 0, s>>>(tab); break;
        case 24: tile_f64_gauss<24><<<grid, 256, 0, s>>>(tab); break;
        case 32: tile_f64_gauss<32><<<grid, 256, 0, s>>>(tab); break;
        case 48: tile_f64_gauss<48><<<grid, 256, 0, s>>>(tab); break;
        default: tile_f64_gauss<64><<<grid, 256, 0, s>>>(tab); break;
      }
      KRR_LAUNCH_CHECK("tile_f64_gauss");
      tile_timer_stop(tok, s);
    }
  }
  return KRR_OK;
}

}  // namespace krr
