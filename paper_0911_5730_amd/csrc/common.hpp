// Shared host-side definitions of libbddc: error type, HIP checks, device arena.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <functional>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/bddc.h"

namespace bddc {

struct Error {
  bddc_status status;
  std::string msg;
};

[[noreturn]] inline void fail(bddc_status s, const std::string& msg) { throw Error{s, msg}; }

#define BDDC_HIP(call)                                                                   \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      ::bddc::fail(BDDC_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));    \
  } while (0)

// Device memory of the library: blocks from hipMalloc are kept in a
// process-wide cache per device after release and reused (best fit, at most
// twice the request) by later allocations, so repeated set-ups allocate and
// free nothing.  Release only memory that no queued work still uses.
void* device_acquire(size_t bytes);
void device_release(void* p);

// One device allocation carved into aligned pieces.  Pieces are laid out by a
// sizing pass (base == nullptr) and then a second pass after allocation.
class Arena {
 public:
  void reset_sizing() { base_ = nullptr; used_ = 0; }
  template <class T>
  T* take(size_t count) {
    size_t bytes = ((count * sizeof(T)) + 255) & ~size_t(255);
    size_t off = used_;
    used_ += bytes;
    if (!base_) return nullptr;
    return reinterpret_cast<T*>(base_ + off);
  }
  size_t used() const { return used_; }
  void allocate(hipStream_t st) {
    (void)st;
    size_t n = used_ ? used_ : 256;
    base_ = static_cast<char*>(device_acquire(n));
    size_ = n;
    used_ = 0;
  }
  // the caller has synchronised the stream that used the memory
  void release(hipStream_t st) {
    (void)st;
    if (base_) device_release(base_);
    base_ = nullptr;
  }
  size_t size() const { return size_; }
  // lay pieces out in memory the arena does not own (its size checked by the
  // caller against used() of a sizing pass); detach() forgets it again
  void attach(void* base) {
    base_ = static_cast<char*>(base);
    used_ = 0;
  }
  void detach() { base_ = nullptr; }

 private:
  char* base_ = nullptr;
  size_t used_ = 0;
  size_t size_ = 0;
};

// body(begin, end) over [0, n) in chunks of `chunk`, on a persistent pool of
// up to 8 host threads (the caller takes part).  The body must not throw and
// must write disjoint data for disjoint ranges.
void parallel_for(int n, int chunk, const std::function<void(int, int)>& body);

// Pinned host buffers, reused across handles: hipHostMalloc is slow and
// hipHostFree synchronises the device, so buffers stay in a process-wide pool.
void* pinned_acquire(size_t bytes);
void pinned_release(void* p);

// Host-to-device uploads staged through one pinned buffer.  add() records a
// source that must stay alive until flush(); flush() packs the sources into a
// pinned buffer laid out like their destinations and enqueues one copy per run
// of destinations separated only by arena alignment padding (< 256 bytes, which
// no other piece can occupy).  At destruction the buffer goes to `deferred`
// (released by the owner after a later stream synchronisation) or, without
// one, back to the pool once the copies are done.
class Staging {
 public:
  explicit Staging(hipStream_t st, std::vector<void*>* deferred = nullptr) : st_(st), deferred_(deferred) {}
  Staging(const Staging&) = delete;
  Staging& operator=(const Staging&) = delete;
  ~Staging();
  void add(void* dst, const void* src, size_t bytes) {
    if (bytes) items_.push_back({static_cast<char*>(dst), static_cast<const char*>(src), bytes});
  }
  template <class T>
  void add(T* dst, const std::vector<T>& v) {
    add(dst, v.data(), v.size() * sizeof(T));
  }
  void flush();

 private:
  struct Item {
    char* dst;
    const char* src;
    size_t bytes;
  };
  hipStream_t st_;
  std::vector<void*>* deferred_;
  std::vector<Item> items_;
  void* buf_ = nullptr;
};

template <class T>
void h2d(T* dst, const std::vector<T>& src, hipStream_t st) {
  if (!src.empty())
    BDDC_HIP(hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, st));
}

}  // namespace bddc
