// Internal declarations of libhhg (host + device).  Not part of the ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/hhg.h"

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

// ------------------------------------------------------------- stencils
// One stencil entry in lattice terms: source group g (velocity groups 0..7,
// or 0 for P1 arrays), index offset (di, dj, dk), and up to three weights
// (three velocity components for B / B^T, one otherwise).
struct Entry {
  int g, di, dj, dk;
  double w[3];
};
using Row = std::vector<Entry>;

// Element matrices of the six Kuhn tetrahedra at h = 1, built from the
// barycentric calculus (host, float64).  vorder 1 or 2.
struct ElementSet {
  int vorder;
  int nloc;                         // 4 or 10
  double K[6][10][10];              // velocity stiffness
  double M[6][10][10];              // velocity consistent mass
  double D[6][3][4][10];            // -int psi_k d_d phi_a
  double Kp[6][4][4];               // P1 stiffness (pressure)
  double Mp[6][4][4];               // P1 mass (pressure)
  int vpos[6][10][3];               // local velocity DoF positions, site units
  int ppos[6][4][3];                // local vertex positions, P1 units
};
void build_elements(int vorder, ElementSet* es);

// Row stencils around a row DoF, summed over the lattice elements that lie in
// the box [0, Nbox]^3 (P1 units).  kind: 'A' stiffness (velocity row ->
// velocity cols), 'M' velocity mass, 'T' B^T (velocity row -> pressure cols,
// 3 weights), 'B' (pressure row -> velocity cols, 3 weights), 'C' pressure
// stiffness, 'P' pressure mass.  Row position: group g and index (i, j, k).
Row row_stencil(const ElementSet& es, char kind, int g, int i, int j, int k, int Nbox);

// Boundary class of a coordinate: 0 low face, 1 inside, 2 high face.
inline int bclass3(int c, int N) { return c == 0 ? 0 : (c == N ? 2 : 1); }
inline int bclass(int i, int j, int k, int N) { return bclass3(i, N) + 3 * bclass3(j, N) + 9 * bclass3(k, N); }
constexpr int kInteriorClass = 13;

// Dense symmetric pseudo-inverse by cyclic Jacobi rotations (host, float64):
// eigen-decomposition K = Q L Q^T, eigenvalues below rcond * max |L| dropped.
// Returns the numerical rank.
int sym_pinv(int n, const std::vector<double>& K, std::vector<double>& Kp, double rcond);

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
