// Internal helpers shared by the library's translation units: error state,
// a bump allocator over the caller's workspace, and launch checking.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstddef>
#include <cstdio>
#include <cstdarg>
#include <string>
#include "../../include/krr.h"

namespace krr {

void set_error(const char* fmt, ...);
const char* last_error();

// Returns KRR_EHIP (and records the message) when a HIP call failed.
inline int hip_check(hipError_t e, const char* what) {
  if (e == hipSuccess) return KRR_OK;
  set_error("%s: %s", what, hipGetErrorString(e));
  return KRR_EHIP;
}

#define KRR_TRY(expr)                 \
  do {                                \
    int _rc = (expr);                 \
    if (_rc < 0) return _rc;          \
  } while (0)

#define KRR_LAUNCH_CHECK(name) KRR_TRY(::krr::hip_check(hipGetLastError(), name))

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Bump allocator: the same call sequence gives the same layout, so a
// "measuring" arena (base == nullptr) computes the footprint that a real
// arena later carves out of the caller's workspace.
struct Arena {
  char* base = nullptr;
  size_t cap = 0;
  size_t used = 0;
  Arena() = default;
  Arena(void* b, size_t c) : base(static_cast<char*>(b)), cap(c) {}
  template <class T>
  T* take(size_t count) {
    size_t off = used;
    used += align_up(count * sizeof(T) + (count == 0 ? 1 : 0));
    return base ? reinterpret_cast<T*>(base + off) : nullptr;
  }
  bool ok() const { return base == nullptr || used <= cap; }
};

inline int check_ws(void* ws, size_t ws_bytes, size_t need) {
  if (ws == nullptr || ws_bytes < need) {
    set_error("workspace too small: %zu bytes given, %zu needed", ws == nullptr ? (size_t)0 : ws_bytes, need);
    return KRR_EWORKSPACE;
  }
  if ((reinterpret_cast<uintptr_t>(ws) % kAlign) != 0) {
    set_error("workspace must be %zu-byte aligned", kAlign);
    return KRR_EWORKSPACE;
  }
  return KRR_OK;
}

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace krr
