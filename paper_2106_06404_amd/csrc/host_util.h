// Host-side helpers shared by the library's C++ sources: error type, HIP call
// checks, device buffers and host/device pointer handling.
#pragma once
#include <hip/hip_runtime.h>

#include <chrono>
#include <cstring>
#include <map>
#include <mutex>
#include <thread>
#include <string>
#include <unordered_map>
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

// Pinned host staging for uploads.  hipMemcpyAsync from pageable memory blocks the
// host until the runtime has copied the data through its own bounce buffers; copied
// into pinned memory first, an upload becomes an asynchronous DMA that overlaps the
// host work after it.  The staged copies stay valid (chunks are only handed out
// again) until the next reset, taken at the same device-wide safe points as the
// device memory cache, when no copy can still be in flight; one arena per device.
class PinnedArena {
 public:
  static PinnedArena& get() {
    static PinnedArena arenas[kMaxDev];
    int dev = 0;
    (void)hipGetDevice(&dev);
    return arenas[dev >= 0 && dev < kMaxDev ? dev : 0];
  }
  // uninitialised pinned space for bytes (valid until the next reset), or nullptr
  void* alloc(size_t bytes) {
    std::lock_guard<std::mutex> lk(mu_);
    const size_t need = (bytes + 255) & ~(size_t)255;
    while (cur_ < chunks_.size() && off_ + need > chunks_[cur_].second) {
      ++cur_;
      off_ = 0;
    }
    if (cur_ == chunks_.size()) {
      const size_t sz = need > kChunk ? need : kChunk;
      void* p = nullptr;
      if (hipHostMalloc(&p, sz, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
      }
      chunks_.push_back({static_cast<char*>(p), sz});
      off_ = 0;
    }
    char* dst = chunks_[cur_].first + off_;
    off_ += need;
    return dst;
  }
  // a pinned copy of [src, src + bytes), or nullptr (then the caller copies directly)
  void* stage(const void* src, size_t bytes) {
    char* dst = static_cast<char*>(alloc(bytes));
    if (!dst) return nullptr;
    copy_bytes(dst, src, bytes);
    return dst;
  }
  // memcpy; large blocks by several threads (a single thread moves only a few GB/s)
  static void copy_bytes(void* dstv, const void* src, size_t bytes) {
    constexpr size_t kPar = (size_t)4 << 20;
    char* dst = static_cast<char*>(dstv);
    if (bytes >= kPar) {
      constexpr int kThr = 8;
      const size_t part = ((bytes + kThr - 1) / kThr + 255) & ~(size_t)255;
      const char* s = static_cast<const char*>(src);
      std::vector<std::thread> th;
      for (size_t a = part; a < bytes; a += part) {
        const size_t len = a + part < bytes ? part : bytes - a;
        th.emplace_back([dst, s, a, len] { std::memcpy(dst + a, s + a, len); });
      }
      std::memcpy(dst, s, part < bytes ? part : bytes);
      for (auto& t : th) t.join();
    } else {
      std::memcpy(dst, src, bytes);
    }
  }
  void reset() {
    std::lock_guard<std::mutex> lk(mu_);
    cur_ = 0;
    off_ = 0;
  }

 private:
  static constexpr int kMaxDev = 64;
  static constexpr size_t kChunk = (size_t)64 << 20;
  std::mutex mu_;
  std::vector<std::pair<char*, size_t>> chunks_;
  size_t cur_ = 0, off_ = 0;
};

// Device memory cache shared by all contexts of the process.  A setup allocates and
// frees hundreds of buffers; hipMalloc and hipFree are slow and hipFree waits for the
// device, so freed blocks are kept for reuse.  A freed block is quarantined until the
// next safe point (a device-wide synchronisation, taken at the start of every setup and
// when a context is destroyed): until then a kernel still in flight may read it, and
// another stream or host thread must not receive it.  Blocks are matched by size,
// rounded up to 256 bytes below 64 KiB and to eighths of a power of two above.
class DevicePool {
 public:
  static DevicePool& get() {
    static DevicePool pool;
    return pool;
  }
  void* alloc(size_t bytes) {
    const size_t sz = round(bytes);
    int dev = 0;
    (void)hipGetDevice(&dev);
    {
      std::lock_guard<std::mutex> lk(mu_);
      auto it = free_.find(Key{dev, sz});
      if (it != free_.end()) {
        void* p = it->second;
        free_.erase(it);
        live_[p] = Key{dev, sz};
        return p;
      }
    }
    void* p = nullptr;
    if (hipMalloc(&p, sz) != hipSuccess) {
      (void)hipGetLastError();
      drop_free(dev);  // give the cached blocks back and try once more
      if (hipMalloc(&p, sz) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
      }
    }
    std::lock_guard<std::mutex> lk(mu_);
    live_[p] = Key{dev, sz};
    return p;
  }
  void release(void* p) {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = live_.find(p);
    if (it == live_.end()) return;
    quarantine_.push_back({it->second, p});
    live_.erase(it);
  }
  // the device has no work in flight: the current device's quarantined blocks become
  // reusable
  void safe_point() {
    int dev = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceSynchronize();
    PinnedArena::get().reset();
    std::lock_guard<std::mutex> lk(mu_);
    std::vector<std::pair<Key, void*>> keep;
    for (auto& q : quarantine_) {
      if (q.first.dev == dev)
        free_.emplace(q.first, q.second);
      else
        keep.push_back(q);
    }
    quarantine_.swap(keep);
  }

 private:
  struct Key {
    int dev;
    size_t bytes;
    bool operator<(const Key& o) const { return dev != o.dev ? dev < o.dev : bytes < o.bytes; }
  };
  static size_t round(size_t b) {
    if (b < 65536) return (b + 255) & ~(size_t)255;
    size_t p = 65536;
    while (p * 2 <= b) p *= 2;
    const size_t step = p / 8;
    return (b + step - 1) / step * step;
  }
  void drop_free(int dev) {
    std::lock_guard<std::mutex> lk(mu_);
    for (auto it = free_.begin(); it != free_.end();) {
      if (it->first.dev == dev) {
        (void)hipFree(it->second);
        it = free_.erase(it);
      } else {
        ++it;
      }
    }
  }
  std::mutex mu_;
  std::multimap<Key, void*> free_;
  std::unordered_map<void*, Key> live_;
  std::vector<std::pair<Key, void*>> quarantine_;
};

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
    if (p) DevicePool::get().release(p);
    p = nullptr;
    n = 0;
  }
  void alloc(size_t cnt) {
    release();
    if (cnt == 0) return;
    p = static_cast<T*>(DevicePool::get().alloc(cnt * sizeof(T)));
    if (!p)
      throw MsddError{MSDD_ENOMEM, "device allocation of " + std::to_string(cnt * sizeof(T)) + " bytes failed"};
    n = cnt;
  }
  void zero(hipStream_t s) {
    if (n) HIPCHK(hipMemsetAsync(p, 0, n * sizeof(T), s));
  }
  void upload(const std::vector<T>& v, hipStream_t s) {
    alloc(v.size());
    if (!n) return;
    const size_t bytes = n * sizeof(T);
    const void* src = bytes >= ((size_t)64 << 10) ? PinnedArena::get().stage(v.data(), bytes) : nullptr;
    HIPCHK(hipMemcpyAsync(p, src ? src : v.data(), bytes, hipMemcpyHostToDevice, s));
  }
  // upload from host memory that stays valid until the copy has run (pinned staging
  // space, or pageable memory, which the runtime copies before returning)
  void upload_raw(const T* src, size_t cnt, hipStream_t s) {
    alloc(cnt);
    if (n) HIPCHK(hipMemcpyAsync(p, src, n * sizeof(T), hipMemcpyHostToDevice, s));
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

// host copy into v (resized to cnt; its storage is reused when v already holds that many)
// (device sources through pinned staging space, in pieces of at most 16 MB)
template <class T>
void to_host_into(std::vector<T>& v, const T* ptr, size_t cnt) {
  v.resize(cnt);
  if (cnt == 0) return;
  REQUIRE(ptr != nullptr, "null array argument");
  const size_t bytes = cnt * sizeof(T);
  if (is_device_ptr(ptr)) {
    constexpr size_t kPiece = (size_t)16 << 20;
    char* st = bytes >= ((size_t)64 << 10)
                   ? static_cast<char*>(PinnedArena::get().alloc(bytes < kPiece ? bytes : kPiece))
                   : nullptr;
    if (!st) {
      HIPCHK(hipMemcpy(v.data(), ptr, bytes, hipMemcpyDeviceToHost));
      return;
    }
    for (size_t a = 0; a < bytes; a += kPiece) {
      const size_t len = bytes - a < kPiece ? bytes - a : kPiece;
      HIPCHK(hipMemcpy(st, reinterpret_cast<const char*>(ptr) + a, len, hipMemcpyDeviceToHost));
      PinnedArena::copy_bytes(reinterpret_cast<char*>(v.data()) + a, st, len);
    }
  } else {
    PinnedArena::copy_bytes(v.data(), ptr, bytes);
  }
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

// Host array built only to be uploaded: placed in the pinned staging arena (no zeroing,
// no first-touch page faults, asynchronous upload), or in an owned vector when pinned
// memory is not available.  Contents start uninitialised.
template <class T>
struct HostBuf {
  T* p = nullptr;
  size_t n = 0;
  std::vector<T> fallback;
  explicit HostBuf(size_t cnt) : n(cnt) {
    p = cnt ? static_cast<T*>(PinnedArena::get().alloc(cnt * sizeof(T))) : nullptr;
    if (!p && cnt) {
      fallback.resize(cnt);
      p = fallback.data();
    }
  }
  T& operator[](size_t i) { return p[i]; }
  T* begin() { return p; }
};

}  // namespace msdd_host
