// Host-side helpers shared by the library's C++ sources: error type, HIP call
// checks, device buffers and host/device pointer handling.
#pragma once
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstring>
#include <string>
#include <vector>

#include "msdd.h"

namespace msdd_host {

struct MsddError {
  int code;
  std::string msg;
};

#define HIPCHK(x)                                                                       \
  do {                                                                                  \
    hipError_t e_ = (x);                                                                \
    if (e_ != hipSuccess)                                                               \
      throw MsddError{MSDD_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_)};    \
  } while (0)

#define REQUIRE(cond, msg)                                     \
  do {                                                         \
    if (!(cond)) throw MsddError{MSDD_EINVAL, std::string(msg)}; \
  } while (0)

inline double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

template <class T>
struct DVec {
  T* p = nullptr;
  size_t n = 0;
  DVec() = default;
  DVec(const DVec&) = delete;
  DVec& operator=(const DVec&) = delete;
  DVec(DVec&& o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
  DVec& operator=(DVec&& o) noexcept {
    if (this != &o) { release(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
    return *this;
  }
  ~DVec() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  void alloc(size_t cnt) {
    release();
    if (cnt == 0) return;
    if (hipMalloc((void**)&p, cnt * sizeof(T)) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
      throw MsddError{MSDD_ENOMEM, "device allocation of " + std::to_string(cnt * sizeof(T)) + " bytes failed"};
    }
    n = cnt;
  }
  void zero(hipStream_t s) {
    if (n) HIPCHK(hipMemsetAsync(p, 0, n * sizeof(T), s));
  }
  void upload(const std::vector<T>& v, hipStream_t s) {
    alloc(v.size());
    if (n) HIPCHK(hipMemcpyAsync(p, v.data(), n * sizeof(T), hipMemcpyHostToDevice, s));
  }
  std::vector<T> download(hipStream_t s, size_t cnt = (size_t)-1) const {
    if (cnt == (size_t)-1) cnt = n;
    std::vector<T> v(cnt);
    if (cnt) {
      HIPCHK(hipMemcpyAsync(v.data(), p, cnt * sizeof(T), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
    }
    return v;
  }
};

inline bool is_device_ptr(const void* ptr) {
  if (!ptr) return false;
  hipPointerAttribute_t a;
  hipError_t e = hipPointerGetAttributes(&a, ptr);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return a.type == hipMemoryTypeDevice || a.isManaged;
}

template <class T>
std::vector<T> to_host(const T* ptr, size_t cnt) {
  std::vector<T> v(cnt);
  if (cnt == 0) return v;
  REQUIRE(ptr != nullptr, "null array argument");
  if (is_device_ptr(ptr)) {
    HIPCHK(hipMemcpy(v.data(), ptr, cnt * sizeof(T), hipMemcpyDeviceToHost));
  } else {
    std::memcpy(v.data(), ptr, cnt * sizeof(T));
  }
  return v;
}

// device copy owned by the context (from host or device source)
template <class T>
void to_device(DVec<T>& dst, const T* src, size_t cnt, hipStream_t s) {
  dst.alloc(cnt);
  if (!cnt) return;
  REQUIRE(src != nullptr, "null array argument");
  HIPCHK(hipMemcpyAsync(dst.p, src, cnt * sizeof(T),
                        is_device_ptr(src) ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
}

}  // namespace msdd_host
