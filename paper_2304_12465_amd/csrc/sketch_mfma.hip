// KRILL's sketch B = Phi A(:, S) (Alg. 2) for the Gaussian kernel on the
// matrix cores.  B[r][c] = zeta^{-1/2} sum over the nonzeros e of row r of
// Phi of sign_e K(x_{j_e}, s_c).
//
// Orientation: the centres are the rows of an MFMA tile (held in registers
// as the B operand, 128 per workgroup), the nonzeros of a range of sketch
// rows are its columns, 64 at a time, with their points gathered into LDS.
// The distance contraction runs on v_mfma_f64_16x16x4f64 as in the FP64
// product tile.  FP32 points (padded dimension 8, 16, 24 or 32) run it as the
// three-slice bf16 contraction of the FP32 product tiles (gauss_mfma.h): at
// d = 16 three 16-cycle MFMAs per 256 entries against four 32-cycle FP32
// ones.  Other padded dimensions use v_mfma_f32_16x16x4f32.  Instead of a
// product with V, each lane adds the exponentials of its columns (signed)
// into the running sum of the current sketch row, and a row's sum is
// completed across the four lanes that share a centre when the nonzeros
// move on to the next row.  The nonzeros of a row are in ascending point
// order and every workgroup owns whole rows, so each entry of B is a
// fixed-order sum written once (bitwise reproducible, no atomics).
#include "product.h"
#include "gauss_mfma.h"
#include <algorithm>
#include <type_traits>

namespace krr {

namespace {

constexpr int kSkRT = 2;     // 16-centre tiles per wave (128 centres per workgroup)
constexpr int kSkCols = 64;  // nonzeros per LDS chunk (four 16-column tiles)

template <typename T>
struct SketchJob {
  const T* cc;    // centres, centred, k x dpad
  const T* cn;    // their squared norms
  const T* cmax;  // largest squared norm (device scalar)
  int64_t k;
  const T* yc;    // all points, centred with the same centre, N x dpad
  const T* yn;
  const T* ymax;
  const int64_t* offs;     // ds + 1 row offsets into entries
  const int64_t* entries;  // 2 j + (sign < 0), ascending j within a row
  const int* row_of;       // sketch row of every entry
  int64_t ds;
  int rows_per_wg;
  T s;           // exponent scale: 1024/ln2 s_nat (FP64, exp64_u) or log2(e) s_nat (FP32, exp2)
  double s_nat;  // 1 / (2 sigma^2)
  int dpad;
  double inv_sqrt_zeta;
  double* B;     // ds x k
};

// The FP64 sketch up to 16 padded dimensions is held to 128 VGPRs: 4 waves
// per SIMD (2 waves: the 2,000,000-point, k = 10,000 FP64 sketch in 0.280 s
// of build; 3 waves, no spill: 146.9 ms; 4 waves, 15 registers spilled
// outside the inner loop: 143.6 ms).  Ordering its workgroups in XCD runs
// (each row range's centre blocks on one XCD) doubled its time: the
// workgroups of a row range then gather the same points at the same moment
// through one L2.
template <typename T, int D>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(std::is_same<T, double>::value && D <= 16 ? 4 : 1)))
void sketch_gauss_mfma(const SketchJob<T> J) {
  typedef typename GT<T>::acc_t acc_t;
  constexpr int KS = D / 4;
  constexpr int NT = kSkCols / 16;
  constexpr int kY = kSkCols * D / 256;
  constexpr bool kSplit = s3_split<T, D>();
  constexpr int NC = s3_steps<D>();        // bf16 MFMA steps
  constexpr int PY = s3_pitch<D>();
  constexpr int kSegs = kSkCols * D / 4;   // 4-coordinate segments of a chunk's points
  constexpr int kSegPT = (kSegs + 255) / 256;
  __shared__ double etab[GT<T>::kTable];  // FP64 exp table (one unused entry for FP32)
  // a chunk's points: their values, or (kSplit) their bf16 slices h | m | l
  // per row; the form not used keeps one element
  __shared__ T sY[kSplit ? 1 : kSkCols][D + 1];
  __shared__ __attribute__((aligned(16))) __bf16 sYb[kSplit ? kSkCols : 1][PY];
  __shared__ T sAy[kSkCols];
  __shared__ T sSg[kSkCols];
  __shared__ int sRow[kSkCols];
  __shared__ int64_t sJn[kSkCols];  // points of the next chunk's nonzeros
  // the direct-difference sketch serves this problem (uniform decision)
  if (gauss_expansion_too_coarse<T>(J.s_nat, (double)*J.cmax, (double)*J.ymax, J.dpad)) return;
  if constexpr (std::is_same<T, double>::value) GT<T>::fill(etab);

  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int g = lane >> 4, li = lane & 15;
  const int64_t k = J.k;
  const int64_t c0 = (int64_t)blockIdx.x * (4 * 16 * kSkRT) + wave * (16 * kSkRT);
  T xb[kSkRT][kSplit ? 1 : KS];  // B operand: centre c0 + 16 rt + li, coordinates 4 ks + g
  // kSplit: K index 32 st + 8 g + e of step st is coordinate d0 + e of slice
  // product p, with 8-coordinate group G = 4 st + g, p = G / (D/8) and d0 =
  // 8 (G % (D/8)); groups with p >= 6 pad the last step (zero centre slices)
  bf16x8 xbb[kSkRT][kSplit ? NC : 1];
  int aoff[kSplit ? NC : 1];  // LDS offset of the lane's point slice in a row
  acc_t cinit[kSkRT];
#pragma unroll
  for (int rt = 0; rt < kSkRT; ++rt) {
    int64_t c = c0 + rt * 16 + li;
    if (c > k - 1) c = k - 1;
    if constexpr (kSplit) {
#pragma unroll
      for (int st = 0; st < NC; ++st) {
        xbb[rt][st] = s3_b_operand<D>(J.cc + c * D, st, g);
        if (rt == 0) aoff[st] = s3_a_offset<D>(st, g);
      }
    } else {
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) xb[rt][ks] = J.cc[c * D + 4 * ks + g];
    }
    const T h = T(-0.5) * J.cn[c];
    cinit[rt] = acc_t{h, h, h, h};
  }
  const int64_t r0 = (int64_t)blockIdx.y * J.rows_per_wg;
  const int64_t r1 = r0 + J.rows_per_wg < J.ds ? r0 + J.rows_per_wg : J.ds;
  const int64_t eb = J.offs[r0], ee = J.offs[r1];
  const T s2 = T(2) * J.s;

  double cur[kSkRT];
#pragma unroll
  for (int rt = 0; rt < kSkRT; ++rt) cur[rt] = 0.0;
  // completes row rho: the four lanes of a centre are added in a fixed
  // pairing ((g0 + g1) + (g2 + g3))
  auto flush = [&](int64_t rho) {
#pragma unroll
    for (int rt = 0; rt < kSkRT; ++rt) {
      double v = cur[rt];
      v += __shfl_xor(v, 16);
      v += __shfl_xor(v, 32);
      const int64_t c = c0 + rt * 16 + li;
      if (g == 0 && c < k) J.B[rho * k + c] = v * J.inv_sqrt_zeta;
      cur[rt] = 0.0;
    }
  };
  auto zero_row = [&](int64_t rho) {
#pragma unroll
    for (int rt = 0; rt < kSkRT; ++rt) {
      const int64_t c = c0 + rt * 16 + li;
      if (g == 0 && c < k) J.B[rho * k + c] = 0.0;
    }
  };

  // Two-stage pipeline over 64-nonzero chunks: while chunk i is computed
  // from LDS, the point data of chunk i + 1 (indices from LDS) and the
  // codes of chunk i + 2 are in flight in registers.
  auto load_code = [&](int64_t base) -> int64_t {
    const int64_t e = base + tid;
    return J.entries[e < ee ? e : ee - 1];
  };
  T y_st[kSplit ? 1 : kY];
  f32x4 y4_st[kSplit ? kSegPT : 1];  // kSplit: coordinates 4 part .. 4 part + 3 of a point
  T ay_st = T(0), sg_st = T(0);
  int row_st = 0;
  auto stage_points = [&](int64_t base, int64_t code) {
    if constexpr (kSplit) {
#pragma unroll
      for (int q = 0; q < kSegPT; ++q) {
        const int seg = tid + q * 256;
        if (kSegs % 256 == 0 || seg < kSegs)
          y4_st[q] = *reinterpret_cast<const f32x4*>(J.yc + sJn[seg / (D / 4)] * D +
                                                      4 * (seg % (D / 4)));
      }
    } else {
#pragma unroll
      for (int q = 0; q < kY; ++q) {
        const int idx = tid + q * 256;
        y_st[q] = J.yc[sJn[idx / D] * D + idx % D];
      }
    }
    if (tid < kSkCols) {
      const int64_t e = base + tid;
      const bool valid = e < ee;
      const int64_t j = code >> 1;
      ay_st = valid ? -J.s * J.yn[j] : GT<T>::kFar;
      sg_st = valid ? ((code & 1) ? T(-1) : T(1)) : T(0);
      row_st = J.row_of[valid ? e : ee - 1];  // padding keeps the last row: no false boundary
    }
  };
  int64_t code_n = 0;
  if (eb < ee) {
    if (tid < kSkCols) {
      code_n = load_code(eb);
      sJn[tid] = code_n >> 1;
    }
    __syncthreads();
    stage_points(eb, code_n);
    if (tid < kSkCols) code_n = load_code(eb + kSkCols);
  }

  int64_t rc = r0;  // row whose sum is being formed (uniform)
  for (int64_t e0 = eb; e0 < ee; e0 += kSkCols) {
    __syncthreads();  // the previous chunk's LDS reads are done
    if constexpr (kSplit) {
#pragma unroll
      for (int q = 0; q < kSegPT; ++q) {
        const int seg = tid + q * 256;
        if (kSegs % 256 == 0 || seg < kSegs)
          s3_store_quad<D>(y4_st[q], seg % (D / 4), sYb[seg / (D / 4)]);
      }
    } else {
#pragma unroll
      for (int q = 0; q < kY; ++q) {
        const int idx = tid + q * 256;
        sY[idx / D][idx % D] = y_st[q];
      }
    }
    if (tid < kSkCols) {
      sAy[tid] = ay_st;
      sSg[tid] = sg_st;
      sRow[tid] = row_st;
      sJn[tid] = code_n >> 1;
    }
    __syncthreads();
    if (e0 + kSkCols < ee) {
      const int64_t code = code_n;
      stage_points(e0 + kSkCols, code);
      if (tid < kSkCols) code_n = load_code(e0 + 2 * kSkCols);
    }
    acc_t dot[2][kSkRT];
    auto distance = [&](int ct, acc_t* dv) {
#pragma unroll
      for (int rt = 0; rt < kSkRT; ++rt) dv[rt] = cinit[rt];
      if constexpr (kSplit) {
        bf16x8 ya[NC];  // A operand: slices of the point of nonzero ct*16 + li
#pragma unroll
        for (int st = 0; st < NC; ++st)
          ya[st] = *reinterpret_cast<const bf16x8*>(&sYb[ct * 16 + li][aoff[st]]);
#pragma unroll
        for (int st = 0; st < NC; ++st)
#pragma unroll
          for (int rt = 0; rt < kSkRT; ++rt)
            dv[rt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ya[st], xbb[rt][st], dv[rt], 0, 0, 0);
      } else {
        T ya[KS];  // A operand: point of nonzero ct*16 + li, coordinates 4 ks + g
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) ya[ks] = sY[ct * 16 + li][4 * ks + g];
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
#pragma unroll
          for (int rt = 0; rt < kSkRT; ++rt) dv[rt] = GT<T>::mfma(ya[ks], xb[rt][ks], dv[rt]);
      }
    };
    distance(0, dot[0]);
#pragma unroll
    for (int ct = 0; ct < NT; ++ct) {
      if (ct + 1 < NT) distance(ct + 1, dot[(ct + 1) & 1]);
      // dot[rt][t] = y_col . c_li - ||c_li||^2 / 2 for col = ct*16 + col(t, g)
      // ex: the kernel values (FP64: signed).  FP32: w is the signed sum of
      // the lane's four columns (one multiply, then a chain of multiply-adds
      // in a fixed order) for a tile that stays within the current row; the
      // FP64 tile keeps the signed values and adds them pairwise (the chain's
      // extra registers would spill at 128 VGPRs)
      constexpr bool kChain = std::is_same<T, float>::value;
      T ex[kSkRT][4], w[kSkRT];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int col = ct * 16 + GT<T>::col(t, g);
        const T ay = sAy[col], sg = sSg[col];
#pragma unroll
        for (int rt = 0; rt < kSkRT; ++rt) {
          const T e = GT<T>::ex(fma_g(dot[ct & 1][rt][t], s2, ay), etab);
          if constexpr (kChain) {
            ex[rt][t] = e;
            w[rt] = t == 0 ? sg * e : fma_g(sg, e, w[rt]);
          } else {
            ex[rt][t] = sg * e;
          }
        }
      }
      const int64_t rf = sRow[ct * 16], rl = sRow[ct * 16 + 15];
      if (rf == rc && rl == rc) {
#pragma unroll
        for (int rt = 0; rt < kSkRT; ++rt) {
          if constexpr (kChain)
            cur[rt] += (double)w[rt];
          else
            cur[rt] += (double)((ex[rt][0] + ex[rt][1]) + (ex[rt][2] + ex[rt][3]));
        }
      } else {
        // the tile reaches into later rows: finish them in order
        int64_t rho = rc;
        while (true) {
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const int col = ct * 16 + GT<T>::col(t, g);
            if (sRow[col] == rho) {
              const T sg = kChain ? sSg[col] : T(1);
#pragma unroll
              for (int rt = 0; rt < kSkRT; ++rt) cur[rt] += (double)(sg * ex[rt][t]);
            }
          }
          if (rho == rl) break;
          flush(rho);
          int64_t nx = rl;  // next row present in this tile
          for (int u = 0; u < 16; ++u) {
            const int64_t r = sRow[ct * 16 + u];
            if (r > rho && r < nx) nx = r;
          }
          for (int64_t z = rho + 1; z < nx; ++z) zero_row(z);
          rho = nx;
        }
        rc = rl;
      }
    }
  }
  flush(rc);
  for (int64_t z = rc + 1; z < r1; ++z) zero_row(z);
}

template <typename T>
void* sketch_mfma_pick(int D) {
  switch (D) {
    case 4: return (void*)&sketch_gauss_mfma<T, 4>;
    case 8: return (void*)&sketch_gauss_mfma<T, 8>;
    case 16: return (void*)&sketch_gauss_mfma<T, 16>;
    case 20: return (void*)&sketch_gauss_mfma<T, 20>;
    case 24: return (void*)&sketch_gauss_mfma<T, 24>;
    case 32: return (void*)&sketch_gauss_mfma<T, 32>;
    case 48: return (void*)&sketch_gauss_mfma<T, 48>;
    case 64: return (void*)&sketch_gauss_mfma<T, 64>;
    default: return nullptr;
  }
}

template <typename T>
int launch_sketch(double sigma, int dpad, const T* cc, const T* cn, const T* cmax, int64_t k,
                  const T* yc, const T* yn, const T* ymax, const int64_t* offs,
                  const int64_t* entries, const int* row_of, int64_t ds, double inv_sqrt_zeta,
                  double* B, hipStream_t s) {
  void* fn = sketch_mfma_pick<T>(dpad);
  if (!fn) {
    set_error("sketch: unsupported padded dimension %d", dpad);
    return KRR_EINVAL;
  }
  SketchJob<T> J;
  J.cc = cc;
  J.cn = cn;
  J.cmax = cmax;
  J.k = k;
  J.yc = yc;
  J.yn = yn;
  J.ymax = ymax;
  J.offs = offs;
  J.entries = entries;
  J.row_of = row_of;
  J.ds = ds;
  J.rows_per_wg = (int)std::max<int64_t>(8, ceil_div(ds, 65535));
  J.s_nat = 1.0 / (2.0 * sigma * sigma);
  J.s = (T)(GT<T>::kExpScale * J.s_nat);
  J.dpad = dpad;
  J.inv_sqrt_zeta = inv_sqrt_zeta;
  J.B = B;
  // centre blocks vary fastest: the workgroups that share a row range (and
  // so gather the same points) run together
  dim3 grid((unsigned)ceil_div(k, 4 * 16 * kSkRT), (unsigned)ceil_div(ds, J.rows_per_wg));
  using Fn = void (*)(const SketchJob<T>);
  reinterpret_cast<Fn>(fn)<<<grid, 256, 0, s>>>(J);
  KRR_LAUNCH_CHECK("sketch_gauss_mfma");
  return KRR_OK;
}

}  // namespace

int sketch_gauss_mfma_launch(krr_precision prec, double sigma, const PointSet& pts,
                             const PointSet& cpts, const int64_t* offs, const int64_t* entries,
                             const int* row_of, int64_t ds, double inv_sqrt_zeta, double* B,
                             hipStream_t s) {
  if (cpts.n <= 0 || ds <= 0) return KRR_OK;
  if (prec == KRR_FP64)
    return launch_sketch<double>(sigma, pts.dpad, cpts.xc64, cpts.xn64, cpts.xmax64, cpts.n,
                                 pts.xc64, pts.xn64, pts.xmax64, offs, entries, row_of, ds,
                                 inv_sqrt_zeta, B, s);
  return launch_sketch<float>(sigma, pts.dpad, cpts.xc32, cpts.xn32, cpts.xmax32, cpts.n,
                              pts.xc32, pts.xn32, pts.xmax32, offs, entries, row_of, ds,
                              inv_sqrt_zeta, B, s);
}

}  // namespace krr
