// Error reporting and device-buffer helpers shared by the C-ABI sources.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "ietidp.h"

namespace ieti {
namespace rt {

// thread-local message behind ieti_last_error()
inline std::string& last_error() {
  thread_local std::string msg;
  return msg;
}

inline int fail(int code, const std::string& msg) {
  last_error() = msg;
  return code;
}

#define HIP_TRY(expr)                                                                           \
  do {                                                                                          \
    hipError_t e_ = (expr);                                                                     \
    if (e_ != hipSuccess)                                                                       \
      return ::ieti::rt::fail(IETI_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

template <class T>
struct DBuf {
  T* ptr = nullptr;
  int64_t n = 0;
  void release() {
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    n = 0;
  }
};

template <class T>
int dalloc(DBuf<T>& b, int64_t n) {
  b.release();
  b.n = n;
  if (n <= 0) return IETI_OK;
  HIP_TRY(hipMalloc(&b.ptr, size_t(n) * sizeof(T)));
  return IETI_OK;
}

template <class T>
int dupload(DBuf<T>& b, const std::vector<T>& h) {
  int rc = dalloc(b, int64_t(h.size()));
  if (rc) return rc;
  if (!h.empty()) HIP_TRY(hipMemcpy(b.ptr, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  return IETI_OK;
}

template <class T>
int dupload(DBuf<T>& b, const T* h, int64_t n) {
  int rc = dalloc(b, n);
  if (rc) return rc;
  if (n > 0) HIP_TRY(hipMemcpy(b.ptr, h, size_t(n) * sizeof(T), hipMemcpyHostToDevice));
  return IETI_OK;
}

}  // namespace rt
}  // namespace ieti
