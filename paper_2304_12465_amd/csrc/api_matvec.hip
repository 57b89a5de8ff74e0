// C ABI: error state and the standalone kernel product.
#include "product.h"
#include <cmath>
#include <cstring>
#include <mutex>

namespace krr {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

int validate_matvec(int kind, double sigma, int prec, int64_t nr, int64_t nc, int32_t d,
                           int32_t m) {
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
  if (nr < 0 || nc < 0 || d < 1 || d > 64 || m < 1 || m > 64) {
    set_error("invalid shape nr=%lld nc=%lld d=%d m=%d (need nr,nc >= 0, 1<=d<=64, 1<=m<=64)",
              (long long)nr, (long long)nc, d, m);
    return KRR_EINVAL;
  }
  return KRR_OK;
}

size_t matvec_bytes(int kind, int prec, int64_t nr, int64_t nc, int32_t d, int32_t m) {
  return pointset_bytes((krr_kernel_kind)kind, (krr_precision)prec, nr, d) +
         pointset_bytes((krr_kernel_kind)kind, (krr_precision)prec, nc, d) +
         product_scratch_bytes((krr_precision)prec, nr, nc, m);
}

const char* last_error() { return g_err; }

}  // namespace krr

using namespace krr;

extern "C" const char* krr_last_error(void) { return g_err; }

extern "C" int krr_kernel_matvec_ws(krr_precision prec, int64_t nr, int64_t nc, int32_t d,
                                    int32_t m, size_t* bytes) {
  KRR_TRY(validate_matvec(KRR_LAPLACE, 1.0, prec, nr, nc, d, m));
  if (!bytes) {
    set_error("bytes is NULL");
    return KRR_EINVAL;
  }
  // the Gaussian layout is at least as large as the Laplace one
  size_t a = matvec_bytes(KRR_GAUSSIAN, prec, nr, nc, d, m);
  size_t b = matvec_bytes(KRR_LAPLACE, prec, nr, nc, d, m);
  *bytes = a > b ? a : b;
  return KRR_OK;
}

namespace krr {

int matvec_impl(int kind, double sigma, int prec,
                const double* Xr, int64_t nr, const double* Xc, int64_t nc, int32_t d,
                const double* V, int32_t m, double shift, double* W, void* ws, size_t ws_bytes,
                hipStream_t stream) {
  const krr_kernel_kind kk = (krr_kernel_kind)kind;
  const krr_precision pp = (krr_precision)prec;
  KRR_TRY(validate_matvec(kind, sigma, prec, nr, nc, d, m));
  if (shift != 0.0 && nr != nc) {
    set_error("shift != 0 needs a square product (nr == nc)");
    return KRR_EINVAL;
  }
  if (!std::isfinite(shift)) {
    set_error("shift must be finite");
    return KRR_EINVAL;
  }
  if (nr == 0) return KRR_OK;
  if (!W || (nc > 0 && (!Xc || !V)) || !Xr || (shift != 0.0 && !V)) {
    set_error("NULL array argument");
    return KRR_EINVAL;
  }
  const size_t need = matvec_bytes(kind, prec, nr, nc, d, m);
  KRR_TRY(check_ws(ws, ws_bytes, need));
  Arena arena(ws, ws_bytes);
  PointSet rows, cols;
  const bool same = (Xc == Xr && nc == nr);
  KRR_TRY(carve_points(kk, pp, nr, d, arena, &rows));
  if (same) cols = rows;
  else KRR_TRY(carve_points(kk, pp, nc, d, arena, &cols));
  if (!arena.ok()) {
    set_error("workspace too small for the point layouts");
    return KRR_EWORKSPACE;
  }
  if (same) {
    KRR_TRY(fill_points(kk, pp, Xr, nullptr, rows, stream));
  } else if (kk == KRR_LAPLACE && pp != KRR_FP64) {
    // one quantisation over both sets
    KRR_TRY(quant_params(Xr, nr, Xc, nc, d, rows.qbits, rows.qpart, const_cast<double*>(rows.qp),
                         stream));
    KRR_TRY(fill_points(kk, pp, Xr, rows.qp, rows, stream));
    KRR_TRY(fill_points(kk, pp, Xc, rows.qp, cols, stream));
  } else {
    // columns first: MIXED Gaussian rows share the columns' centre
    KRR_TRY(fill_points(kk, pp, Xc, nullptr, cols, stream));
    KRR_TRY(fill_points(kk, pp, Xr, nc > 0 ? shared_params(kk, pp, cols) : nullptr, rows,
                        stream));
  }
  VecView v{V, m, 1};
  VecOut w{W, m, 1};
  return product(kk, sigma, pp, rows, cols, v, m, shift, v, w, arena, stream);
}

}  // namespace krr


extern "C" int krr_kernel_matvec(krr_kernel_kind kind, double sigma, krr_precision prec,
                                 const double* Xr, int64_t nr, const double* Xc, int64_t nc,
                                 int32_t d, const double* V, int32_t m, double shift, double* W,
                                 void* ws, size_t ws_bytes, hipStream_t stream) {
  return matvec_impl(kind, sigma, prec, Xr, nr, Xc, nc, d, V, m, shift, W, ws, ws_bytes, stream);
}

// ---- allocation-free product ------------------------------------------------
// A fixed scratch array in device memory for krr_kernel_matvec_noalloc: every
// GPU the library runs on holds its own copy for the life of the process.
// Host code never uses the array's name as an address: the device address is
// looked up once per device (hipGetSymbolAddress, with that device current)
// and kept per device.
constexpr size_t kNoAllocScratchBytes = size_t(256) << 20;
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

int device_scratch(void** out) {
  int dev = -1;
  KRR_TRY(hip_check(hipGetDevice(&dev), "hipGetDevice"));
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device %d out of range for the fixed scratch table", dev);
    return KRR_EINVAL;
  }
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    KRR_TRY(hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)),
                      "hipGetSymbolAddress(scratch)"));
    if (!p) {
      set_error("hipGetSymbolAddress(scratch) returned NULL");
      return KRR_EHIP;
    }
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return KRR_OK;
}
}  // namespace

extern "C" int krr_kernel_matvec_noalloc(krr_kernel_kind kind, double sigma, krr_precision prec,
                                         const double* Xr, int64_t nr, const double* Xc,
                                         int64_t nc, int32_t d, const double* V, int32_t m,
                                         double shift, double* W, hipStream_t stream) {
  KRR_TRY(validate_matvec(kind, sigma, prec, nr, nc, d, m));
  const size_t need = matvec_bytes(kind, prec, nr, nc, d, m);
  if (need > kNoAllocScratchBytes) {
    set_error("product needs %zu bytes of scratch; the fixed scratch holds %zu "
              "(use krr_kernel_matvec with a workspace)", need, kNoAllocScratchBytes);
    return KRR_EWORKSPACE;
  }
  if (nr == 0) return KRR_OK;
  void* ws = nullptr;
  KRR_TRY(device_scratch(&ws));
  return matvec_impl(kind, sigma, prec, Xr, nr, Xc, nc, d, V, m, shift, W, ws,
                     kNoAllocScratchBytes, stream);
}

extern "C" int krr_timing_enable(int on) {
  tile_timing_enable(on != 0);
  return KRR_OK;
}

extern "C" int krr_timing_read(double* total_ms, int64_t* launches) {
  return tile_timing_read(total_ms, launches);
}

extern "C" int krr_timing_read_vectors(int32_t vectors, double* total_ms, int64_t* launches,
                                       double* match_ms, int64_t* match_launches) {
  if (vectors < 0) {
    set_error("krr_timing_read_vectors: vectors must be >= 0");
    return KRR_EINVAL;
  }
  return tile_timing_read(total_ms, launches, vectors, match_ms, match_launches);
}
