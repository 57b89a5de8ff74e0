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
#include "exp64.h"
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
//
// Per-thread staging of the next 64-column chunk (points, -s ||y||^2, V),
// loaded into registers while the current chunk is computed.
template <int D>
struct Stage64 {
  static constexpr int kY = kCols64 * D / 256;  // doubles of points per thread
  double y[kY];
  double v[4];  // V: 64 columns x 16 rhs / 256 threads
  double ay;    // threads 0..63
};

template <int D>
__device__ __forceinline__ void stage64_fetch(const F64Job& J, int64_t jb, int64_t j1, int tid,
                                              Stage64<D>& st) {
#pragma unroll
  for (int q = 0; q < Stage64<D>::kY; ++q) {
    const int e = tid + q * 256;
    const int jj = e / D;
    st.y[q] = (jb + jj < j1) ? J.yc[jb * D + e] : 0.0;
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int e = tid + q * 256;
    st.v[q] = (jb + e / 16 < j1) ? J.v[jb * 16 + e] : 0.0;
  }
  if (tid < kCols64) st.ay = (jb + tid < j1) ? -J.s * J.yn[jb + tid] : -1.0e300;
}

// The expansion ||x||^2 + ||y||^2 - 2 x.y carries an absolute error of at
// most about (d + 3) eps s (||x||^2 + ||y||^2) into the exponent, i.e. into
// the relative error of each entry.  Jobs where that bound (with the largest
// centred norms of rows and columns) could exceed ~9e-14 -- a bandwidth
// small against the spread of the points -- take direct differences instead
// (tile_f64_direct).
constexpr double kDirectBound = 400.0;  // x eps = 8.9e-14
__device__ __forceinline__ bool needs_direct(const F64Job& J) {
  return J.s * (*J.xmax + *J.ymax) * (J.dpad + 3) > kDirectBound;
}

template <int D, int MV>
__device__ __forceinline__ void f64_item(const F64Job& J, int64_t rg, int split,
                                         const double* __restrict__ etab) {
  constexpr int KS = D / 4;
  constexpr int NT = kCols64 / 16;
  __shared__ double sY[kCols64][D + 1];
  __shared__ double sAy[kCols64];
  __shared__ double sV[kCols64][17];  // [column][rhs]

  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int g = lane >> 4, li = lane & 15;
  const int64_t nr = J.nr, nc = J.nc;
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
  // E.V on the matrix cores (MV = 0): two accumulators per row tile (even /
  // odd K steps) keep independent MFMA chains in flight.  On the VALU
  // (MV = 1, 2, 4 right-hand sides): lane l sums E[li][4t + g] V[4t + g][c]
  // over its columns; the four lanes of a row are added at the end.
  constexpr int MA = MV == 0 ? 2 : 1;
  constexpr int MC = MV == 0 ? 1 : MV;
  f64x4 acc[kRT64][MA];
  double accv[kRT64][MC];
#pragma unroll
  for (int rt = 0; rt < kRT64; ++rt) {
#pragma unroll
    for (int a = 0; a < MA; ++a) acc[rt][a] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int c = 0; c < MC; ++c) accv[rt][c] = 0.0;
  }
  const double s2 = 2.0 * J.s;

  const int64_t j0 = (int64_t)split * J.per;
  int64_t j1 = j0 + J.per;
  if (j1 > nc) j1 = nc;
  Stage64<D> st;
  if (j0 < j1) stage64_fetch<D>(J, j0, j1, tid, st);
  for (int64_t jb = j0; jb < j1; jb += kCols64) {
    __syncthreads();  // the previous chunk's LDS reads are done
#pragma unroll
    for (int q = 0; q < Stage64<D>::kY; ++q) {
      const int e = tid + q * 256;
      sY[e / D][e % D] = st.y[q];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + q * 256;
      sV[e / 16][e % 16] = st.v[q];
    }
    if (tid < kCols64) sAy[tid] = st.ay;
    __syncthreads();
    if (jb + kCols64 < j1) stage64_fetch<D>(J, jb + kCols64, j1, tid, st);
    if (row0 >= nr) continue;
    // distance MFMAs of column tile ct + 1 are issued before the exp work
    // of tile ct, which does not depend on them
    f64x4 dot[2][kRT64];
    auto distance = [&](int ct, f64x4* d) {
      double ya[KS];  // A operand: Y[ct*16 + li][4 ks + g]
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) ya[ks] = sY[ct * 16 + li][4 * ks + g];
#pragma unroll
      for (int rt = 0; rt < kRT64; ++rt) d[rt] = cinit[rt];
#pragma unroll
      for (int ks = 0; ks < KS; ++ks)
#pragma unroll
        for (int rt = 0; rt < kRT64; ++rt)
          d[rt] = __builtin_amdgcn_mfma_f64_16x16x4f64(ya[ks], xb[rt][ks], d[rt], 0, 0, 0);
    };
    distance(0, dot[0]);
#pragma unroll
    for (int ct = 0; ct < NT; ++ct) {
      if (ct + 1 < NT) distance(ct + 1, dot[(ct + 1) & 1]);
      double ay[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) ay[t] = sAy[ct * 16 + 4 * t + g];
      // dot[rt][t] = y_{4t+g} . x_{li} - ||x_{li}||^2 / 2
      double e[kRT64][4];
#pragma unroll
      for (int rt = 0; rt < kRT64; ++rt)
#pragma unroll
        for (int t = 0; t < 4; ++t)
          e[rt][t] = exp64(__builtin_fma(dot[ct & 1][rt][t], s2, ay[t]), etab);
      if constexpr (MV == 0) {
        // A of E.V step t: lane l holds E[li][4t + g] (K index g)
        double vb[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) vb[t] = sV[ct * 16 + 4 * t + g][li];  // V[4t + g][c = li]
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int rt = 0; rt < kRT64; ++rt)
            acc[rt][t & 1] = __builtin_amdgcn_mfma_f64_16x16x4f64(e[rt][t], vb[t], acc[rt][t & 1], 0, 0, 0);
      } else {
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int c = 0; c < MV; ++c) {
            const double v = sV[ct * 16 + 4 * t + g][c];
#pragma unroll
            for (int rt = 0; rt < kRT64; ++rt) accv[rt][c] = __builtin_fma(e[rt][t], v, accv[rt][c]);
          }
      }
    }
  }
  if (row0 >= nr) return;
  double* __restrict__ out = J.part + (int64_t)split * nr * 16;
  if constexpr (MV == 0) {
#pragma unroll
    for (int rt = 0; rt < kRT64; ++rt)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        // E.V output: lane l, element t holds W[i0 + 4t + g][c = li]
        const int64_t i = row0 + rt * 16 + 4 * t + g;
        if (i < nr && li < J.M) out[i * 16 + li] = acc[rt][0][t] + acc[rt][1][t];
      }
  } else {
#pragma unroll
    for (int rt = 0; rt < kRT64; ++rt)
#pragma unroll
      for (int c = 0; c < MV; ++c) {
        // lanes li, li+16, li+32, li+48 hold partial sums of row li: add in
        // a fixed pairing ((g0 + g1) + (g2 + g3))
        double a = accv[rt][c];
        a += __shfl_xor(a, 16);
        a += __shfl_xor(a, 32);
        const int64_t i = row0 + rt * 16 + li;
        if (g == 0 && i < nr && c < J.M) out[i * 16 + c] = a;
      }
  }
}

constexpr int kMaxF64Jobs = 8;
struct F64Table {
  F64Job job[kMaxF64Jobs];
  int njobs;
  int64_t total;
};

template <int D, int MV>
__global__ __launch_bounds__(256) void tile_f64_gauss(const F64Table tab) {
  __shared__ double etab[kExpTable];
  exp64_table_fill(etab);
  __syncthreads();
  for (int64_t item = blockIdx.x; item < tab.total; item += gridDim.x) {
    int jn = 0;
    while (jn + 1 < tab.njobs && item >= tab.job[jn + 1].item0) ++jn;
    const F64Job& J = tab.job[jn];
    if (needs_direct(J)) continue;  // uniform over the workgroup
    const int64_t local = item - J.item0;
    f64_item<D, MV>(J, local / J.nsplit, (int)(local % J.nsplit), etab);
  }
}

// Direct-difference FP64 Gaussian tile for the jobs the expansion cannot
// serve to FP64 accuracy: same items and partial-sum layout as
// tile_f64_gauss.  Thread t owns row t % 128 of the item and every other
// column (t / 128 picks the parity); the column points and V are
// wave-uniform (scalar loads).  The two parities are added in a fixed order.
template <int D>
__global__ __launch_bounds__(256) void tile_f64_direct(const F64Table tab) {
  __shared__ double etab[kExpTable];
  __shared__ double sW[128][17];
  exp64_table_fill(etab);
  __syncthreads();
  const int tid = threadIdx.x;
  const int r = tid & 127, h = tid >> 7;
  for (int64_t item = blockIdx.x; item < tab.total; item += gridDim.x) {
    int jn = 0;
    while (jn + 1 < tab.njobs && item >= tab.job[jn + 1].item0) ++jn;
    const F64Job& J = tab.job[jn];
    if (!needs_direct(J)) continue;  // uniform over the workgroup
    const int64_t local = item - J.item0;
    const int64_t rg = local / J.nsplit;
    const int split = (int)(local % J.nsplit);
    const int64_t nr = J.nr;
    const int64_t i = rg * (4 * 16 * kRT64) + r;
    const int64_t ic = i < nr ? i : nr - 1;
    double x[D];
#pragma unroll
    for (int k = 0; k < D; ++k) x[k] = J.xc[ic * D + k];
    double acc[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) acc[c] = 0.0;
    const int64_t j0 = (int64_t)split * J.per;
    int64_t j1 = j0 + J.per;
    if (j1 > J.nc) j1 = J.nc;
    for (int64_t j = j0 + h; j < j1; j += 2) {
      const double* __restrict__ y = J.yc + j * D;
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < D; ++k) {
        const double t = x[k] - y[k];
        s = __builtin_fma(t, t, s);
      }
      const double e = exp64(-J.s * s, etab);
      const double* __restrict__ v = J.v + j * 16;
#pragma unroll
      for (int c = 0; c < 16; ++c) acc[c] = __builtin_fma(e, v[c], acc[c]);
    }
    __syncthreads();  // sW of the previous item is consumed
    if (h == 1) {
#pragma unroll
      for (int c = 0; c < 16; ++c) sW[r][c] = acc[c];
    }
    __syncthreads();
    if (h == 0 && i < nr) {
      double* __restrict__ out = J.part + (int64_t)split * nr * 16 + i * 16;
      for (int c = 0; c < J.M; ++c) out[c] = acc[c] + sW[r][c];
    }
  }
}

__global__ void zero_scalar(double* p) { *p = 0.0; }

// centred copy and squared norms; the largest norm goes to *xmax (wave
// maximum, then an integer atomic max on the bits: the norms are >= 0, whose
// IEEE bit patterns order like the values)
__global__ void pack_centred64(const double* __restrict__ X, int64_t n, int d, int dpad,
                               const double* __restrict__ centre, double* __restrict__ xc,
                               double* __restrict__ xn, double* __restrict__ xmax) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double s = 0.0;
  if (i < n) {
    for (int k = 0; k < dpad; ++k) {
      const double v = k < d ? X[i * d + k] - centre[k] : 0.0;
      xc[i * dpad + k] = v;
      s += v * v;
    }
    xn[i] = s;
  }
  for (int off = 32; off > 0; off >>= 1) s = fmax(s, __shfl_xor(s, off));
  if ((threadIdx.x & 63) == 0)
    atomicMax(reinterpret_cast<unsigned long long*>(xmax), (unsigned long long)__double_as_longlong(s));
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
  out->xmax64 = arena.take<double>(1);
  if (!out->centre) {
    out->centre = arena.take<double>(64);
    out->cpart = arena.take<double>(256 * 64);
  }
  return KRR_OK;
}

int fill_f64c(const double* X, const double* centre, const PointSet& ps, hipStream_t s) {
  const int64_t n = ps.n;
  zero_scalar<<<1, 1, 0, s>>>(const_cast<double*>(ps.xmax64));
  KRR_LAUNCH_CHECK("zero_scalar");
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
                                                            const_cast<double*>(ps.xn64),
                                                            const_cast<double*>(ps.xmax64));
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
  j.xmax = rows.xmax64;
  j.ymax = cols.xmax64;
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

namespace {

// E.V reduction variant for m right-hand sides: VALU for m <= 4, MFMA above
int f64_variant(int m) { return m <= 1 ? 1 : m <= 2 ? 2 : m <= 4 ? 4 : 0; }

template <int D>
void launch_d(int mv, unsigned grid, const F64Table& tab, hipStream_t s) {
  switch (mv) {
    case 1: tile_f64_gauss<D, 1><<<grid, 256, 0, s>>>(tab); break;
    case 2: tile_f64_gauss<D, 2><<<grid, 256, 0, s>>>(tab); break;
    case 4: tile_f64_gauss<D, 4><<<grid, 256, 0, s>>>(tab); break;
    default: tile_f64_gauss<D, 0><<<grid, 256, 0, s>>>(tab); break;
  }
}

}  // namespace

int f64_launch(const std::vector<F64Job>& jobs, hipStream_t s) {
  for (int D : {4, 8, 16, 20, 24, 32, 48, 64}) {
    for (int mv : {1, 2, 4, 0}) {
      std::vector<F64Job> sel;
      for (const F64Job& j : jobs)
        if (j.dpad == D && f64_variant(j.M) == mv) sel.push_back(j);
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
          case 4: launch_d<4>(mv, grid, tab, s); break;
          case 8: launch_d<8>(mv, grid, tab, s); break;
          case 16: launch_d<16>(mv, grid, tab, s); break;
          case 20: launch_d<20>(mv, grid, tab, s); break;
          case 24: launch_d<24>(mv, grid, tab, s); break;
          case 32: launch_d<32>(mv, grid, tab, s); break;
          case 48: launch_d<48>(mv, grid, tab, s); break;
          default: launch_d<64>(mv, grid, tab, s); break;
        }
        KRR_LAUNCH_CHECK("tile_f64_gauss");
        // the direct tile serves the jobs the MFMA tile skipped (the choice is
        // made on the device, so the launch stays asynchronous)
        switch (D) {
          case 4: tile_f64_direct<4><<<grid, 256, 0, s>>>(tab); break;
          case 8: tile_f64_direct<8><<<grid, 256, 0, s>>>(tab); break;
          case 16: tile_f64_direct<16><<<grid, 256, 0, s>>>(tab); break;
          case 20: tile_f64_direct<20><<<grid, 256, 0, s>>>(tab); break;
          case 24: tile_f64_direct<24><<<grid, 256, 0, s>>>(tab); break;
          case 32: tile_f64_direct<32><<<grid, 256, 0, s>>>(tab); break;
          case 48: tile_f64_direct<48><<<grid, 256, 0, s>>>(tab); break;
          default: tile_f64_direct<64><<<grid, 256, 0, s>>>(tab); break;
        }
        KRR_LAUNCH_CHECK("tile_f64_direct");
        tile_timer_stop(tok, s);
      }
    }
  }
  return KRR_OK;
}

}  // namespace krr
