// Internal declarations of libhhg (host + device).  Not part of the ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/hhg.h"
#include "fe.h"

namespace hhg {

// ------------------------------------------------------------------ errors
void set_error(const std::string& msg);
struct Error {
  hhg_status code;
  std::string msg;
};
#define HHG_CHECK_HIP(expr)                                                                  \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      throw ::hhg::Error{HHG_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)};    \
  } while (0)
#define HHG_REQUIRE(cond, code, msg)                          \
  do {                                                        \
    if (!(cond)) throw ::hhg::Error{(code), std::string(msg)}; \
  } while (0)

// Boundary class of a coordinate: 0 low face, 1 inside, 2 high face.
inline int bclass3(int c, int N) { return c == 0 ? 0 : (c == N ? 2 : 1); }
inline int bclass(int i, int j, int k, int N) { return bclass3(i, N) + 3 * bclass3(j, N) + 9 * bclass3(k, N); }
constexpr int kInteriorClass = 13;

// ------------------------------------------------------------- device side
// Stencil table of one row type in device memory: n entries of offsets (in
// elements, relative to the row's own array position) and weights (nw per
// entry, stored entry-major).
template <typename T>
struct DStencil {
  const int* off;
  const T* w;
  int n;
};

constexpr int kMaxClasses = 27;

}  // namespace hhg
