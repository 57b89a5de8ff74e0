// Internal interface of the matrix-free kernel product engine.
#pragma once
#include <algorithm>
#include <vector>
#include "common.h"

namespace krr {

// Work items of a product are (row group, column split) pairs of equal
// size, dealt to the resident workgroups of 256 CUs.  About 10,240 items
// (some 40 per CU) keep the imbalance of the last round within a few
// percent.  A split count of 8 or more is a multiple of 8, so the items of
// one split share an XCD (workgroup id mod 8) when the grid covers them.
inline int64_t split_count(int64_t nr, int64_t nc, int64_t rows_per_wg, int64_t min_cols) {
  constexpr int64_t kTargetItems = 10240;
  const int64_t rg = std::max<int64_t>(1, ceil_div(nr, rows_per_wg));
  int64_t ns = (kTargetItems + rg / 2) / rg;
  ns = std::min<int64_t>(ns, std::max<int64_t>(1, nc / min_cols));
  if (ns >= 8) ns = ns / 8 * 8;
  return std::max<int64_t>(1, std::min<int64_t>(ns, 4096));
}

// Largest grid of a product launch (items beyond it are taken by a
// grid-stride loop).
constexpr int64_t kGridCap = 65536;

// XCD-contiguous item order for a grid-stride loop over `total` items:
// loop index w (w = blockIdx.x, blockIdx.x + gridDim.x, ... below
// xcd_slots(total); gridDim.x a multiple of 8) runs on XCD w mod 8 and takes
// item xcd_item(w, total), so XCD x works through the x-th of eight
// contiguous runs of items (indices at or past `total` are padding, skipped).
// With the row groups of a column split numbered consecutively, the
// workgroups of one XCD then read the same columns at about the same time
// and share them in that XCD's L2.
__host__ __device__ inline int64_t xcd_slots(int64_t total) { return (total + 7) / 8 * 8; }
__host__ __device__ inline int64_t xcd_item(int64_t w, int64_t total) {
  return (w % 8) * ((total + 7) / 8) + w / 8;
}

// A point set in the compute layout of one precision: n x dpad, zero padded
// from d to dpad (zero coordinates add nothing to either distance).
struct PointSet {
  int64_t n = 0;
  int32_t d = 0;
  int32_t dpad = 0;
  const double* x64 = nullptr;  // FP64 layout (KRR_FP64)
  const float* x32 = nullptr;   // FP32 layout (KRR_FP32, Laplace under KRR_MIXED)
  // bf16 hi/lo split and FP32 squared norms (Gaussian under KRR_MIXED)
  // (a MIXED Gaussian layout also holds the FP32 centred copy xc32 / xn32 /
  // xmax32 below, which serves jobs the split expansion cannot)
  const uint16_t* xhi = nullptr;  // n x kpad bf16 bits
  const uint16_t* xlo = nullptr;
  const float* nrm = nullptr;     // n, ||x||^2 in FP32 of the centred point
  const double* centre = nullptr; // d doubles subtracted before the split
  double* cpart = nullptr;        // 256 x 64 partial sums for the centre
  int32_t kpad = 0;
  // Laplace tiles under FP32 / MIXED: coordinates quantised to `qbits`-bit
  // unsigned fixed point, q = round((x - lo) S); the l1 sums of a tile are
  // then exact 32-bit integer sums of |q_x - q_y| (one v_sad_u32 each).
  const double* xc64 = nullptr;   // FP64 Gaussian: centred points n x dpad
  const double* xn64 = nullptr;   // FP64 Gaussian: ||x - centre||^2
  const double* xmax64 = nullptr; // FP64 Gaussian: max ||x - centre||^2 (one device double)
  const float* xc32 = nullptr;    // FP32 Gaussian: centred points n x dpad
  const float* xn32 = nullptr;    // FP32 Gaussian: ||x - centre||^2
  const float* xmax32 = nullptr;  // FP32 Gaussian: max ||x - centre||^2 (one device float)
  const uint32_t* xq = nullptr;   // n x dpad
  const double* qp = nullptr;     // [lo, S] (device), shared by rows and columns
  double* qpart = nullptr;        // 256 x 2 partial min/max
  int32_t qbits = 0;
  // Gaussian layouts: the largest centred squared norm (the value behind
  // xmax64 / xmax32) once it has been read back to the host, else -1; with
  // both point sets known, products choose between the expansion tile and
  // direct differences on the host and launch only that kernel
  double max_host = -1.0;
};

// Reads a filled Gaussian layout's largest centred squared norm back to
// ps.max_host (synchronises `s`); a no-op for other layouts.
int learn_norm_max(PointSet& ps, hipStream_t s);

// Quantisation range of a point set (or of two): qp[0] = lo, qp[1] = S.
int quant_params(const double* X1, int64_t n1, const double* X2, int64_t n2, int32_t d,
                 int32_t qbits, double* qpart, double* qp, hipStream_t s);

int padded_dim(int32_t d);                       // 0 if d unsupported
int mfma_kdim(int32_t d);                        // bf16 K padding (multiple of 32)

// Bytes of the packed layout for one precision and kernel.
size_t pointset_bytes(krr_kernel_kind kind, krr_precision prec, int64_t n, int32_t d);
// Carves the layout `prec` needs for n points of dimension d from `arena`
// (no GPU work; with a measuring arena only the size is recorded).
int carve_points(krr_kernel_kind kind, krr_precision prec, int64_t n, int32_t d, Arena& arena,
                 PointSet* out);
// Fills a carved layout from FP64 points X (n x d, row-major, device).
// `shared` carries parameters that several point sets of one problem must
// agree on (device, or null to derive them from X): the centre (d doubles)
// of MIXED Gaussian layouts, the quantisation [lo, S] of Laplace FP32 /
// MIXED layouts.
int fill_points(krr_kernel_kind kind, krr_precision prec, const double* X, const double* shared,
                const PointSet& ps, hipStream_t s);
const double* shared_params(krr_kernel_kind kind, krr_precision prec, const PointSet& ps);
// carve_points + fill_points.
int pack_points(krr_kernel_kind kind, krr_precision prec, const double* X, int64_t n, int32_t d,
                const double* centre, Arena& arena, PointSet* out, hipStream_t s);

// KRILL sketch B = Phi A(:, S) for the Gaussian kernel on the matrix cores
// (FP64 or FP32 tiles, FP64 sums): B[r][c] = inv_sqrt_zeta * sum over the
// nonzeros of row r (entries[offs[r] .. offs[r+1]), each 2 j + (sign < 0),
// ascending j; row_of[e] = r) of sign K(x_j, s_c).  pts: all points, cpts:
// the centres, both packed centred with one centre.  The kernel checks the
// expansion guard on the device and does nothing when the direct-difference
// sketch must serve the problem instead.
int sketch_gauss_mfma_launch(krr_precision prec, double sigma, const PointSet& pts,
                             const PointSet& cpts, const int64_t* offs, const int64_t* entries,
                             const int* row_of, int64_t ds, double inv_sqrt_zeta, double* B,
                             hipStream_t s);

// Scratch bytes for product(rows=nr, cols=nc, m).
size_t product_scratch_bytes(krr_precision prec, int64_t nr, int64_t nc, int32_t m);

// Strided view of a block of m vectors: element (i, c) at p[i*rs + c*cs].
struct VecView {
  const double* p = nullptr;
  int64_t rs = 1, cs = 1;
};
struct VecOut {
  double* p = nullptr;
  int64_t rs = 1, cs = 1;
};

// W = K(rows, cols) V + shift * Vs  (V: cols.n x m, Vs and W: rows.n x m).
// Deterministic reduction order.
int product(krr_kernel_kind kind, double sigma, krr_precision prec, const PointSet& rows,
            const PointSet& cols, VecView V, int32_t m, double shift, VecView Vs, VecOut W,
            Arena& scratch, hipStream_t s);

// One product of a group: W = K(rows, cols) V + shift Vs, scratch from the
// request's own arena.
struct ProductReq {
  krr_kernel_kind kind = KRR_GAUSSIAN;
  double sigma = 1.0;
  krr_precision prec = KRR_FP64;
  const PointSet* rows = nullptr;
  const PointSet* cols = nullptr;
  VecView V;
  int32_t m = 1;
  double shift = 0.0;
  VecView Vs;
  VecOut W;
  Arena* scratch = nullptr;
};
// Several products at once: tiles of products that use the same kernel
// instantiation share launches.  Each product's tile decomposition depends
// only on its own shapes, so results are bitwise identical to product().
int product_group(const ProductReq* reqs, int n, hipStream_t s);

// A prepared bf16-split MFMA job (V packed, partial slots carved).
struct MfmaJob {
  const uint16_t* xhi;
  const uint16_t* xlo;
  const float* xn;
  const uint16_t* yhi;
  const uint16_t* ylo;
  const float* yn;
  const uint16_t* vh;
  const uint16_t* vl;
  double* part;
  int route;    // 0: the kernels evaluate the guard; 1: expansion tile; 2: direct differences
  // FP32 centred points (nr x dpad / nc x dpad) and the largest centred
  // squared norms (device), for the expansion guard and its fallback tile
  const float* xf;
  const float* yf;
  const float* xmax;
  const float* ymax;
  int64_t nr, nc, per, item0;
  float s;      // exponent scale in base 2: log2(e) / (2 sigma^2)
  float s_nat;  // 1 / (2 sigma^2)
  int nsplit, M, kp, dpad;
};
int mfma_prepare(double sigma, const PointSet& rows, const PointSet& cols, VecView V, int c0,
                 int mc, Arena& scratch, MfmaJob* out, hipStream_t s);
int mfma_launch(const std::vector<MfmaJob>& jobs, hipStream_t s);

// A prepared Gaussian MFMA job in FP64 or FP32 (product_gauss_mfma.hip).
template <typename T>
struct GJob {
  const T* xc;      // centred rows, nr x dpad
  const T* xn;      // their squared norms
  const T* xmax;    // max ||x||^2 of the rows / columns (device)
  const T* ymax;
  const T* yc;      // centred columns, nc x dpad
  const T* yn;
  const T* v;       // nc x 16
  double* part;     // nsplit x nr x 16
  int64_t nr, nc, per, item0;
  T s;              // exponent scale (FP32: in base 2)
  double s_nat;     // 1 / (2 sigma^2)
  int nsplit, M, dpad;
  int route;        // 0: the kernels evaluate the guard; 1: expansion tile; 2: direct differences
  T* store;         // store variant: the kernel values, nr x ld (row-major), else null
  int64_t ld;
};
typedef GJob<double> F64Job;
typedef GJob<float> F32Job;
int carve_f64c(int64_t n, int32_t dpad, Arena& arena, PointSet* out);
int fill_f64c(const double* X, const double* centre, const PointSet& ps, hipStream_t s);
int carve_f32c(int64_t n, int32_t dpad, Arena& arena, PointSet* out);
int fill_f32c(const double* X, const double* centre, const PointSet& ps, hipStream_t s);
size_t product_f64mfma_scratch_bytes(int64_t nr, int64_t nc);
size_t product_f32mfma_scratch_bytes(int64_t nr, int64_t nc);
int f64_prepare(double sigma, const PointSet& rows, const PointSet& cols, VecView V, int c0, int mc,
                Arena& scratch, F64Job* out, hipStream_t s);
int f32_prepare(double sigma, const PointSet& rows, const PointSet& cols, VecView V, int c0, int mc,
                Arena& scratch, F32Job* out, hipStream_t s);
int f64_launch(const std::vector<F64Job>& jobs, hipStream_t s);
// Writes the Gaussian kernel block K(rows, cols) (nr x nc, row-major with
// leading dimension ld >= nc, zero in columns nc .. ld - 1) with the
// expansion tiles in `prec` (KRR_FP64: FP64 values, KRR_FP32: FP32), when
// the expansion's guard, taken on the host from the norm maxima the point
// sets hold (learn_norm_max), admits it; *done tells whether it did (else
// the caller evaluates the block by direct differences).
int gauss_block_store(krr_precision prec, double sigma, const PointSet& rows,
                      const PointSet& cols, void* out, int64_t ld, bool* done, hipStream_t s);
int f32_launch(const std::vector<F32Job>& jobs, hipStream_t s);

// bf16-split MFMA path for Gaussian tiles (product_mfma.hip).
int carve_mixed(int64_t n, int32_t d, Arena& arena, PointSet* out);
int compute_centre(const double* X, int64_t n, int32_t d, double* centre, double* part,
                   hipStream_t s);
int fill_mixed(const double* X, const double* centre, const PointSet& ps, hipStream_t s);
size_t product_mfma_scratch_bytes(int64_t nr, int64_t nc);

// The standalone product W = K(Xr, Xc) V + shift V with its own point layouts
// carved from a caller workspace (api_matvec.hip); also serves predictions.
int validate_matvec(int kind, double sigma, int prec, int64_t nr, int64_t nc, int32_t d,
                    int32_t m);
size_t matvec_bytes(int kind, int prec, int64_t nr, int64_t nc, int32_t d, int32_t m);
int matvec_impl(int kind, double sigma, int prec, const double* Xr, int64_t nr, const double* Xc,
                int64_t nc, int32_t d, const double* V, int32_t m, double shift, double* W,
                void* ws, size_t ws_bytes, hipStream_t stream);

// Tile timer hooks: start returns a token (or null when timing is off).
// vectors: the right-hand-side vectors the launched Gaussian matrix-core
// tile instantiation carries (0: its 9-16-vector form; -1 for other tiles)
void* tile_timer_start(hipStream_t s, int vectors = -1);
void tile_timer_stop(void* token, hipStream_t s);

// Event timing of the product tile kernel launches (process-wide).
void tile_timing_enable(bool on);
// All recorded launches, and those whose tile carried `vectors` vectors
// (match_*, optional); clears the record.
int tile_timing_read(double* total_ms, int64_t* launches, int vectors = -1,
                     double* match_ms = nullptr, int64_t* match_launches = nullptr);

}  // namespace krr
