// Common definitions for the two-site DMRG sigma library (gfx950).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <vector>

namespace dmrg {

// Quantum numbers of the U(1)xU(1) symmetry: particle number N and 2*Sz.
struct QN {
  int n = 0, s = 0;
};
inline bool operator==(QN a, QN b) { return a.n == b.n && a.s == b.s; }
inline bool operator!=(QN a, QN b) { return !(a == b); }
inline bool operator<(QN a, QN b) { return a.n < b.n || (a.n == b.n && a.s < b.s); }
inline QN operator+(QN a, QN b) { return {a.n + b.n, a.s + b.s}; }
inline QN operator-(QN a, QN b) { return {a.n - b.n, a.s - b.s}; }
inline QN operator-(QN a) { return {-a.n, -a.s}; }

// Local basis of one spatial orbital: |0>, |up>, |dn>, |updn> = a+_up a+_dn |0>.
static const QN kSiteQN[4] = {{0, 0}, {1, 1}, {1, -1}, {2, 0}};
static const int kSiteN[4] = {0, 1, 1, 2};

// Errors raised inside the library; the C-ABI turns them into status codes.
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

enum : int {
  kOk = 0,
  kWarnNotConverged = 1,
  kErrInvalidArg = -1,
  kErrShape = -2,
  kErrHip = -3,
  kErrOom = -4,
  kErrNoDevice = -5,
  kErrUnimplemented = -6,
  kErrState = -7,
};

#define DMRG_HIP(call)                                                                  \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess) {                                                             \
      if (e_ == hipErrorOutOfMemory)                                                    \
        throw ::dmrg::Error(::dmrg::kErrOom, std::string("out of device memory at ") + \
                                                 #call);                                \
      throw ::dmrg::Error(::dmrg::kErrHip, std::string(hipGetErrorString(e_)) + " at " + \
                                               #call);                                  \
    }                                                                                   \
  } while (0)

#define DMRG_REQUIRE(cond, code, msg) \
  do {                                \
    if (!(cond)) throw ::dmrg::Error((code), (msg)); \
  } while (0)

// Owning device buffer (hipMalloc / hipFree).
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  explicit DevBuf(size_t n) { alloc(n); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes) { o.p = nullptr; o.bytes = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) { release(); p = o.p; bytes = o.bytes; o.p = nullptr; o.bytes = 0; }
    return *this;
  }
  ~DevBuf() { release(); }
  void alloc(size_t n) {
    release();
    if (n == 0) return;
    DMRG_HIP(hipMalloc(&p, n));
    bytes = n;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  template <class T> T* as() const { return static_cast<T*>(p); }
};

}  // namespace dmrg
