// Shared host/device utilities: error handling, device buffers, bfloat16.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/mfmg.h"

namespace mfmg {

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define MFMG_HIP(call)                                                                       \
  do {                                                                                       \
    hipError_t e_ = (call);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      throw ::mfmg::Error(e_ == hipErrorOutOfMemory ? MFMG_ERR_OOM : MFMG_ERR_HIP,           \
                          std::string(#call) + ": " + hipGetErrorString(e_));                \
  } while (0)

#define MFMG_REQUIRE(cond, code, msg)                                                        \
  do {                                                                                       \
    if (!(cond)) throw ::mfmg::Error((code), (msg));                                         \
  } while (0)

// Owning device allocation.
template <typename T>
struct DeviceArray {
  T* ptr = nullptr;
  size_t n = 0;
  DeviceArray() = default;
  explicit DeviceArray(size_t count) { alloc(count); }
  DeviceArray(const DeviceArray&) = delete;
  DeviceArray& operator=(const DeviceArray&) = delete;
  DeviceArray(DeviceArray&& o) noexcept : ptr(o.ptr), n(o.n) { o.ptr = nullptr; o.n = 0; }
  DeviceArray& operator=(DeviceArray&& o) noexcept {
    if (this != &o) { release(); ptr = o.ptr; n = o.n; o.ptr = nullptr; o.n = 0; }
    return *this;
  }
  ~DeviceArray() { release(); }
  void alloc(size_t count) {
    release();
    n = count;
    if (count) MFMG_HIP(hipMalloc(&ptr, count * sizeof(T)));
  }
  void release() {
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    n = 0;
  }
  void upload(const std::vector<T>& h) {
    alloc(h.size());
    if (n) MFMG_HIP(hipMemcpy(ptr, h.data(), n * sizeof(T), hipMemcpyHostToDevice));
  }
  void upload(const T* h, size_t count) {
    alloc(count);
    if (n) MFMG_HIP(hipMemcpy(ptr, h, n * sizeof(T), hipMemcpyHostToDevice));
  }
  std::vector<T> download() const {
    std::vector<T> h(n);
    if (n) MFMG_HIP(hipMemcpy(h.data(), ptr, n * sizeof(T), hipMemcpyDeviceToHost));
    return h;
  }
  size_t bytes() const { return n * sizeof(T); }
};

// bfloat16 stored as raw bits; conversion with round-to-nearest-even.
struct bf16 {
  uint16_t bits;
};

__host__ __device__ inline float bf16_to_float(bf16 v) {
  uint32_t u = static_cast<uint32_t>(v.bits) << 16;
  float f;
  __builtin_memcpy(&f, &u, 4);
  return f;
}

__host__ __device__ inline bf16 float_to_bf16(float f) {
  uint32_t u;
  __builtin_memcpy(&u, &f, 4);
  bf16 r;
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) {  // NaN stays NaN
    r.bits = static_cast<uint16_t>((u >> 16) | 0x0040u);
    return r;
  }
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  r.bits = static_cast<uint16_t>(u >> 16);
  return r;
}

// Storage <-> compute conversions.  Acc<S>::type is the arithmetic type used
// for a vector stored as S (bf16 vectors are computed in FP32).
template <typename S> struct Acc { using type = S; };
template <> struct Acc<bf16> { using type = float; };

template <typename C, typename S> __host__ __device__ inline C load_as(const S& v) {
  return static_cast<C>(v);
}
template <> __host__ __device__ inline float load_as<float, bf16>(const bf16& v) {
  return bf16_to_float(v);
}
template <> __host__ __device__ inline double load_as<double, bf16>(const bf16& v) {
  return bf16_to_float(v);
}
template <typename S, typename C> __host__ __device__ inline S store_as(C v) {
  return static_cast<S>(v);
}
template <> __host__ __device__ inline bf16 store_as<bf16, float>(float v) {
  return float_to_bf16(v);
}
template <> __host__ __device__ inline bf16 store_as<bf16, double>(double v) {
  return float_to_bf16(static_cast<float>(v));
}

inline size_t dtype_size(int dt) { return dt == MFMG_F64 ? 8 : dt == MFMG_F32 ? 4 : 2; }

// dtype code of a storage type
template <typename S> constexpr int dtype_of();
template <> constexpr int dtype_of<double>() { return MFMG_F64; }
template <> constexpr int dtype_of<float>() { return MFMG_F32; }
template <> constexpr int dtype_of<bf16>() { return MFMG_BF16; }

}  // namespace mfmg
