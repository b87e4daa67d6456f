// Shared definitions of the gfx950 kernels and the host runtime.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <tuple>

namespace mpofit {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex2 __attribute__((ext_vector_type(2)));

// Global-memory views of generic pointers: accesses through them use the
// global instructions, whose completion is tracked apart from LDS traffic
// (generic "flat" accesses make every LDS wait also wait for memory).
#define GAS __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ const GAS T* gload_ptr(const T* p) { return (const GAS T*)p; }
template <typename T>
__device__ __forceinline__ GAS T* gstore_ptr(T* p) { return (GAS T*)p; }
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// Arithmetic of a GEMM launch.
enum class Mode : int { F64 = 0, F32 = 1, BF16 = 2, BF16X3 = 3 };
// Element type of an operand or result in memory.
enum class DType : int { F64 = 0, F32 = 1 };

// Device status flags (bit set in a device int).
enum : int {
  FLAG_NONFINITE = 1,
  FLAG_CHOL = 2,      // non-positive pivot in a Cholesky factorization
  FLAG_GUARD = 4,     // unused (small singular values are truncated, not flagged)
  FLAG_EIG = 8,       // eigenvalue search did not bracket
};

struct Error {
  int status;
  std::string msg;
};

#define HIP_OK(expr)                                                             \
  do {                                                                           \
    hipError_t e_ = (expr);                                                      \
    if (e_ != hipSuccess)                                                        \
      throw ::mpofit::Error{4, std::string(#expr) + ": " + hipGetErrorString(e_)}; \
  } while (0)

inline int ceil_div(long long a, long long b) { return (int)((a + b - 1) / b); }

}  // namespace mpofit
