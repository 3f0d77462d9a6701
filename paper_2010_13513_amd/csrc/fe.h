// Host-side finite-element setup shared by the library and the build-time
// stencil generator (plain C++, no HIP).
#pragma once
#include <tuple>
#include <vector>

namespace hhg {

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

// Velocity group (0: vertex, 1..7: edge directions) of a doubled-lattice parity.
int group_of_parity(int px, int py, int pz);
// Point location in the Kuhn cube: t in [0,1]^3 -> vertices V (offsets from
// the cube origin) and barycentric coordinates lam of the containing tet.
void kuhn_locate(const double t[3], int V[4][3], double lam[4]);
// Interpolation weights of a coarse element function at a point of a fine
// class: entries (coarse group, offset from cube origin in coarse index
// units, weight); order 1: P1 (group 0), order 2: P2 (groups).
std::vector<std::tuple<int, int, int, int, double>> interp_weights(int order, const double t[3]);
// Restriction (transpose of the interpolation): per coarse velocity group the
// (fine group, fine offset from 2 (i,j,k), weight) entries; the linear P1
// pressure restriction (offsets from 2 (i,j,k)).
struct RestrictEntry {
  int g, di, dj, dk;
  double w;
};
void restriction_entries(int vorder, std::vector<std::vector<RestrictEntry>>& vel, std::vector<RestrictEntry>& pres);

// Dense symmetric pseudo-inverse by cyclic Jacobi rotations (host, float64):
// eigen-decomposition K = Q L Q^T, eigenvalues below rcond * max |L| dropped.
// Returns the numerical rank.
int sym_pinv(int n, const std::vector<double>& K, std::vector<double>& Kp, double rcond);
// Pseudo-inverse of a symmetric K whose null space is exactly span{z} (|z| = 1):
// K^+ = (K + z z^T)^{-1} - z z^T, the inverse by Gauss-Jordan elimination with
// partial pivoting.  Returns false if a pivot vanishes (then K has a larger
// null space and sym_pinv is needed).
bool sym_pinv_null1(int n, const std::vector<double>& K, const std::vector<double>& z, std::vector<double>& Kp);

}  // namespace hhg
