// Internal: preconditioner objects and the PCG driver.
#pragma once
#include <chrono>
#include <string>
#include <vector>
#include "product.h"
#include "la.h"

namespace krr {

// SplitMix64 (Steele, Lea & Flood 2014) used as a counter-based generator:
// sm(s, n) is the n-th output of the generator seeded with s.
__host__ __device__ inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__host__ __device__ inline uint64_t sm64(uint64_t seed, uint64_t n) {
  return mix64(seed + (n + 1) * 0x9E3779B97F4A7C15ull);
}
enum : uint64_t { kTagPivot = 1, kTagCenter = 2, kTagSketchRow = 3, kTagSketchSign = 4 };
__host__ __device__ inline double u53(uint64_t x) { return (double)(x >> 11) * 0x1.0p-53; }

constexpr double kEps = 0x1.0p-52;  // FP64 machine epsilon
constexpr int kBmax = 128;          // largest RPCholesky block

enum PrecondType { kRPChol = 0, kKrill = 1 };

// Column-major block of m vectors of length n (vector c at p + c*n).
struct VecBlock {
  double* p = nullptr;
  int64_t n = 0;
  VecView view() const { return VecView{p, 1, n}; }
  VecOut out() const { return VecOut{p, 1, n}; }
};

struct PcgState {
  int32_t m_max = 0;
  int64_t n = 0;                            // system size: N (full) or k (restricted)
  double *x = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *w = nullptr, *b = nullptr;
  double* scal = nullptr;                   // per-column scalars, kScalars x m_max
  double* part = nullptr;                   // reduction partials
  int nblk = 0;                             // reduction blocks per column
  double* host = nullptr;                   // pinned host mirror of scal
  double* tmpN = nullptr;                   // N x (m_max + spec) (restricted: K_NS p)
  double* tmpR = nullptr;                   // rank x m_max (Woodbury: Q^T r)
};

// Build-time buffers of RPCholesky (part of the workspace footprint).
// Pinned host bytes for the build's small readbacks (totals, draws, accepted lists).
constexpr size_t kHostStage = 4096;

struct RPWork {
  double* d = nullptr;      // residual diagonal, N
  double* S = nullptr;      // chunk totals
  double* O = nullptr;      // chunk offsets
  int64_t* draws = nullptr; // block draws
  int64_t* sp = nullptr;    // distinct draws (ascending)
  double* GT = nullptr;     // B x N: G^T of the block
  double* Fs = nullptr;     // B x r: F(S', 1:i)
  double* Lacc = nullptr;   // kBmax x kBmax
  int* acc = nullptr;       // accepted positions
  int* ints = nullptr;      // [0] accepted count, [1] Cholesky info
  double* spx = nullptr;    // pivot points, kBmax x dpad
  char* hstage = nullptr;   // pinned host staging of the per-block readbacks (kHostStage bytes)
  // uniform rule: pool weights (1 = never drawn), their chunk totals and
  // offsets; greedy rule: per-chunk argmax indices and the maximum
  double* pool = nullptr;   // N
  double* S2 = nullptr;     // chunk totals of pool
  double* O2 = nullptr;     // chunk offsets of pool
  int64_t* gi = nullptr;    // per-chunk index of the largest d
  double* vmax = nullptr;   // largest d (one double)
};

// Build-time buffers of KRILL.
struct KrillWork {
  int* flags = nullptr;       // N
  int* counts = nullptr;      // per 1024-block counts
  int64_t* offs = nullptr;    // block offsets / sketch row offsets
  int64_t* cand = nullptr;    // centre candidates
  double* craw = nullptr;     // k x d centre points
  int* rows = nullptr;        // N x zeta sketch rows
  int* neg = nullptr;         // N x zeta sign bits
  int* row_count = nullptr;   // d_rows + 1
  int64_t* entries = nullptr; // N zeta: 2 j + neg, grouped by row
  int64_t* tmp = nullptr;     // N zeta: sorted row lists
  double* B = nullptr;        // d_rows x k sketch
  int* ints = nullptr;        // [0] error flag, [1] Cholesky info
};

struct Precond {
  PrecondType type = kRPChol;
  krr_kernel_kind kind = KRR_GAUSSIAN;
  double sigma = 1.0;
  krr_precision prec = KRR_FP64;
  double mu = 0.0;
  int64_t N = 0;
  int32_t d = 0;
  int32_t m_max = 1;
  PointSet pts64;  // FP64 layout of X (build steps, true residuals)
  PointSet pts;    // layout of the product precision (== pts64 for FP64)
  // MIXED full-data solves: FP64 layout of a fixed strided sample of the rows
  // (row gap_row(q, N, nsamp) for q < nsamp) and the sampled product output
  // (nsamp x m_max, column-major), for estimating the operator's residual gap
  int64_t nsamp = 0;
  double* samp_x = nullptr;  // nsamp x d
  PointSet spts64;
  double* samp_w = nullptr;
  // RPCholesky: Q^T (rank x N, row-major) with Q Q^T = F (mu I + F^T F)^{-1} F^T,
  // and the lower Cholesky factor L of mu I + F^T F (rank x rank).
  int32_t r_req = 0, B = 0, rank = 0;
  int32_t rule = KRR_PIVOT_RPCHOL;  // pivot rule of the block loop
  uint64_t seed = 0;
  double* QT = nullptr;
  double* core = nullptr;
  std::vector<int64_t> pivots;
  RPWork rp;
  // KRILL
  int32_t k = 0, sketch_rows = 0, zeta = 0;
  double shift = 0.0;             // N eps tr(A_SS)
  int64_t* centers = nullptr;     // device, k
  PointSet cpts64, cpts;          // centres in both layouts
  // precision of the sketch tiles: prec, or FP32 under FP64 products (a
  // KRR_MIXED build), which then keeps FP32 layouts of X and the centres
  krr_precision sketch_prec = KRR_FP64;
  PointSet skpts, skcpts;
  double* H = nullptr;            // k x k: mu A_SS + shift I
  double* C = nullptr;            // k x k: lower Cholesky factor of P = B^T B + H
  double* Linv = nullptr;         // k x k: L^{-1} (the apply is two dense products)
  std::vector<int64_t> centers_host;
  KrillWork kw;
  // stored mode (Sec. 4.1 keeps A(:,S) in memory): A(:,S), N x ld row-major,
  // FP64 (kns_es = 8) or FP32 (4), and the partial column sums of its passes
  bool stored = false;
  void* kns = nullptr;
  int kns_es = 8;
  double* kns_part = nullptr;
  // PCG state and scratch
  PcgState pcg;
  // FP64 tiles: the columns of x that an iteration's operator product may
  // carry beside p (p and w hold m_max + spec_m columns; 0 = none)
  int32_t spec_m = 0;
  Arena scratch;
  size_t ws_used = 0;
  double build_seconds = 0.0;
  bool solving = false;  // a stepped solve owns the PCG vectors (krr_solve_begin .. end/free)
};

// Fixed-order reductions and vector updates (pcg.hip).  The rows from kLog0
// hold, for each iteration of a burst (several iterations between host
// synchronisations, short solves only), its ||r||^2, previous and new
// activity per column: rows kLog0 + 3 i + {0, 1, 2}.
constexpr int kBurst = 8;
enum ScalarSlot {
  kRZ = 0, kPW, kAlpha, kBeta, kRR, kBB, kActive, kRZnew, kTrue, kTmp, kActivePrev, kGap, kLog0
};
constexpr int kScalars = kLog0 + 3 * kBurst;

// Rows sampled for the residual-gap estimate of MIXED solves: at most
// kGapRows, evenly strided over the N rows.
constexpr int64_t kGapRows = 1024;
__host__ __device__ inline int64_t gap_row(int64_t q, int64_t N, int64_t nsamp) {
  return q * N / nsamp;
}

size_t pcg_bytes(int64_t n, int32_t m_max, int64_t N_for_restricted, int32_t rank,
                 int32_t spec_m = 0);
void pcg_carve(Arena& a, PcgState& st, int64_t n, int32_t m_max, int64_t N_for_restricted,
               int32_t rank, int32_t spec_m = 0);
// Columns of x carried beside p by the iteration products (FP64 tiles, up
// to kSpecMax right-hand sides, not over a stored block): the iteration
// expected to converge also forms M x, so that its true residual needs no
// product of its own.  Set before the layout is carved.
constexpr int32_t kSpecMax = 4;
inline int32_t spec_columns(const Precond& P) {
  return (P.prec == KRR_FP64 && !P.stored && P.m_max <= kSpecMax) ? P.m_max : 0;
}

// System operator M V (full: K V + mu V; restricted: K_SN K_NS V + H V) in the
// product precision `prec` (or FP64 when force64).
int apply_operator(Precond& P, VecBlock V, int32_t m, VecBlock W, bool force64, hipStream_t s);
// Preconditioner Z = P^{-1} R.
int apply_precond(Precond& P, VecBlock R, int32_t m, VecBlock Z, hipStream_t s);
// Right-hand side of the system for targets Y (N x m, row-major).
int system_rhs(Precond& P, const double* Y, int32_t m, VecBlock B, hipStream_t s);

int run_pcg(Precond& P, const double* Y, int32_t m, double tol, int32_t max_iter, double* beta,
            krr_solve_info* info, hipStream_t s);

// PCG as a state machine, so that several solves advance together (one
// host synchronisation per step, direction products grouped into shared
// launches).
enum SolvePhase { kPhaseIterate = 0, kPhaseCheck = 1, kPhaseDone = 2 };
struct Solve {
  Precond* P = nullptr;
  int32_t m = 0;
  double tol = 0.0;
  double tol_inner = 0.0;  // recursive-residual target of the current PCG run
  int32_t max_iter = 0;
  int it = 0;
  int restarts = 0;
  int phase = kPhaseIterate;
  int err = 0;
  std::string errmsg;
  std::vector<int32_t> iters;
  std::vector<char> active;
  std::vector<double> history;
  double worst_true = 0.0;
  double prev_true = 1.0;  // worst true residual at the previous check (x = 0: 1)
  std::vector<double> true_rel;  // per column: ||b - M x|| / ||b|| at the last check
  // residual-gap estimates (MIXED full-data solves): the next one is taken
  // once the worst relative recursive residual is at or below gap_next
  // (0: none); pending = its product runs in the next step, read = its sums
  // arrive with this step's scalars
  double gap_next = 0.0;
  bool gap_pending = false, gap_read = false;
  // true residual carried by an iteration: spec_next = the next step's
  // product also takes x (its recursive residual is predicted within reach
  // of tol); spec_now = this step's did
  bool spec_next = false, spec_now = false;
  int check_products = 0;  // operator products spent on true residuals
  std::chrono::steady_clock::time_point t0;
};
int solve_begin(Solve& S, Precond& P, const double* Y, int32_t m, double tol, int32_t max_iter,
                hipStream_t s);
int solve_step(Solve* const* solves, int n, hipStream_t s);
int solve_end(Solve& S, double* beta, krr_solve_info* info, hipStream_t s);

// Stored kernel block of restricted KRR (stored.hip): bytes of A(:,S) (and of
// its partial sums), its evaluation at build time, the operator
// w = A(S,:)(A(:,S) v) over it (t: N x m scratch; v, w: k x m, column-major),
// the FP64 right-hand side B = A(S,:) Y (Y row-major N x m, FP64 storage
// only) and its export as FP64 N x k.
size_t stored_bytes(int64_t N, int64_t k, int es, int32_t m_max, size_t* part_bytes);
int stored_fill(Precond& P, hipStream_t s);
int stored_operator(const Precond& P, const double* v, int32_t m, double* t, double* w,
                    hipStream_t s);
int stored_rhs(const Precond& P, const double* Y, int32_t m, double* B, hipStream_t s);
int stored_export(const Precond& P, double* dst, hipStream_t s);

// Layout helpers used for both measuring and carving.
int rpchol_layout(Arena& a, Precond& P);
int rpchol_build(Precond& P, const double* X, hipStream_t s);
int krill_layout(Arena& a, Precond& P);
int krill_build(Precond& P, const double* X, const int64_t* centers, hipStream_t s);

// Dense kernel block out[q][j] = K(A_q, B_j) in FP64 (out: na x nb, ld).
int kernel_block64(krr_kernel_kind kind, double sigma, const PointSet& A, const PointSet& B,
                   double* out, int64_t ld, hipStream_t s);

// Layout conversions between the ABI's row-major blocks and column-major.
int to_colmajor(const double* src, int64_t n, int32_t m, double* dst, hipStream_t s);
int to_rowmajor(const double* src, int64_t n, int32_t m, double* dst, hipStream_t s);

}  // namespace krr
