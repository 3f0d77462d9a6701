// Unstructured macro meshes (Sec. 2, 2.1): declarations shared by the host
// builder (umesh.hip), the kernels (ukernels.hip) and the C ABI (api.hip).
//
// Every macro cell c of T_0, vertices sorted by id v0 < v1 < v2 < v3, is
// refined by Bey's rule l times.  In path coordinates (i, j, k), n >= i >= j
// >= k >= 0 with n = 2^l, the barycentric weights of a refined node are
// (n - i, i - j, j - k, k) / n, so the refined cell is the affine image of the
// Kuhn simplex conv{0, n e_x, n (e_x + e_y), n (1,1,1)} and its nodes are the
// Freudenthal lattice points inside it: every node has the same 15-point
// neighbourhood (the centre and +-(1,0,0), (0,1,0), (0,0,1), (1,1,0), (1,0,1),
// (0,1,1), (1,1,1)), and its row depends only on the cell and on which of the
// four faces of the cell the node lies on (class m: bit 0 i = n, bit 1 i = j,
// bit 2 j = k, bit 3 k = 0; bit t set <=> barycentric weight t is zero).
//
// Storage (float64): each cell holds its closed lattice packed slab by slab
// (k), row by row (j), i fastest: slot(i, j, k) = S(k) + R(k, j) + i - j with
// S(k) = T(n + 1) - T(n + 1 - k), T(m) = m (m + 1) (m + 2) / 6, R(k, j) =
// (j - k)(n + 1) - (j (j - 1) - k (k - 1)) / 2; P = T(n + 1) slots per cell,
// cell c at c P.  A node on a vertex, edge or face of T_0 (an interface
// node) has a copy in every cell that contains it; all copies hold the same
// value at all times: kernels that write an interface node write every copy.
// A vector is [u1 | u2 | u3 | p], each `vs` words (cells times P, rounded up).
#pragma once
#include <array>

#include "kernels.h"

namespace hhg {

constexpr int kUPoints = 15;
// Stencil point e: 0 the centre, 1..7 the direction with bits (e & 1, e >> 1
// & 1, e >> 2 & 1) in (i, j, k), 8..14 the negative of direction e - 7.
__host__ __device__ constexpr int udir(int e, int a) {
  return e == 0 ? 0 : (e < 8 ? ((e >> a) & 1) : -(((e - 7) >> a) & 1));
}
// Packed slot of (i, j, k) inside a cell with n intervals (int: n <= 512).
__host__ __device__ inline int utet(int m) { return m * (m + 1) * (m + 2) / 6; }
__host__ __device__ inline int uslot(int i, int j, int k, int n) {
  return utet(n + 1) - utet(n + 1 - k) + (j - k) * (n + 1) - (j * (j - 1) - k * (k - 1)) / 2 + (i - j);
}
// Class of (i, j, k): bit 0 i = n, bit 1 i = j, bit 2 j = k, bit 3 k = 0.
__host__ __device__ inline int uclass(int i, int j, int k, int n) {
  return (i == n) | ((i == j) << 1) | ((j == k) << 2) | ((k == 0) << 3);
}
__host__ __device__ inline int upack(int i, int j, int k) { return i | (j << 10) | (k << 20); }

// Row weights of one macro cell at one level, per class m (index 15 unused
// except for the centre-only class of a level-0 vertex).
struct UCell {
  double A[16][kUPoints];      // stiffness (velocity row -> velocity columns)
  double M[16][kUPoints];      // consistent mass
  double B[16][kUPoints][3];   // pressure row -> velocity columns (three components)
  double BT[16][kUPoints][3];  // velocity row -> pressure columns
  double ml[16];               // lumped mass (int psi over the cell's elements at the node)
  double cfac;                 // PSPG: C = cfac A (delta |T|^(2/3), |T| equal for all elements of the cell)
  double ainv0;                // 1 / A[0][0]
  unsigned inside[16];         // bit e: stencil point e lies in the closed cell
  unsigned owned;              // bit m: this cell owns the primitive of class m (the first cell containing it)
  unsigned bnd;                // bit m: the primitive of class m lies on the Dirichlet boundary
};

// One level as a kernel argument.
struct ULev {
  int n, ncell;
  long P, vs;
  const UCell* cs;
};

// Interface nodes of one level: node q has occurrences off[q] .. off[q + 1]
// (cell, i | j << 10 | k << 20), the owner's first.  Nodes [0, nfree) are
// free (not Dirichlet), ordered by Gauss-Seidel colour; [nfree, n) Dirichlet.
struct UList {
  const int* off;
  const int2* occ;
  const double* ainv;  // 1 / assembled A diagonal, free nodes
  int nfree, n;
  int maxocc;          // most occurrences of one node
};

// Row segments (i0, j, k, count) of up to lps points, one lane per point
// (lps a power of two <= 64: several short rows share a wavefront): stride 1
// for the apply and transfer lists, stride 4 for one interior colour.
struct USegs {
  const int4* s;
  int n;
  long pts;  // points in all segments (timer work units)
  int lps;
};

// Host-side state of one level of an unstructured hierarchy.
struct ULevelData {
  ULev L{};
  int nnodes = 0;
  int ncol_if = 0;               // interface colours K (colours K..K+3: cell interiors)
  std::vector<int> col_off;      // K + 1 offsets into the free interface nodes
  std::vector<int> col_maxocc;   // per interface colour: most occurrences of one of its nodes
  int* col_off_d = nullptr;      // device copies: col_off, occurrence slots per colour (if_slots)
  int* col_sl_d = nullptr;
  UList lst{};
  USegs all{}, inner{}, colour[4]{};
  USegs zitems{};                // k-marching items (j, i0, ka, kb) of the interior apply
  double* dinv = nullptr;        // per slot: 1 / Schur diagonal of its node
  double* ml_own = nullptr;      // per slot: lumped mass of its node at the owner slot, else 0
  unsigned char* flags = nullptr;  // per slot: bit 0 owner, bit 1 Dirichlet
  int* canon = nullptr;          // per slot: canonical index of its node (-1: padding)
  double ml_total = 0.0;         // sum of the lumped masses (domain volume)
  std::vector<UCell> hcs;        // host copy of the cell rows
  std::vector<int> h_off;        // host copies of the interface lists (coarse assembly)
  std::vector<int2> h_occ;
  std::vector<int> h_canon;
};

// Occurrence slots per interface node (1, 2 or 4: 16, 32 or 64 lanes) of a
// launch over n nodes whose nodes lie in at most maxocc cells each.
int if_slots(int maxocc, int n);

// Launchers (ukernels.hip), float64, asynchronous on s.
// y = [b -] op x at every node: opmask 1 A, 2 B^T (velocity rows), 4 B, 8 C
// (pressure rows B u - C p; 16: + C p instead), Dirichlet velocity rows zero;
// mass: the consistent mass on all four fields (every row) instead.  wv / wp:
// write the velocity / pressure rows (the others are left as they are).
// zitems: the k-marching items (j, i0, ka, kb) of the interior rows (used
// unless mass; n = 0: the row-segment kernel).
void launch_u_apply_rows(hipStream_t s, const ULev& L, USegs inner, USegs zitems, const UList& lst, const double* x,
                         const double* b, double* y, int opmask, bool has_b, bool mass, bool wv, bool wp);
void launch_u_gs_inner(hipStream_t s, const ULev& L, USegs seg, double* x, const double* b);
// Free interface nodes [first, first + count) of one colour; maxocc: the
// most occurrences of one of them (sets the lanes per node).
void launch_u_gs_iface(hipStream_t s, const ULev& L, const UList& lst, int first, int count, int maxocc, double* x,
                       const double* b);
void launch_u_pstep(hipStream_t s, const ULev& L, const double* dinv, double* x, const double* r, double omega);
// A whole smoothing call (iters Uzawa iterations: xi sweeps of every colour,
// also reversed when sym, then r_p = g - B u + C p into r and the pressure
// step) in one workgroup, every value computed as by the per-colour
// launches; false (nothing launched) when the level has more cells or
// colours than the kernel holds.
bool launch_u_smooth_small(hipStream_t s, const ULevelData& U, double* x, const double* b, double* r, int iters,
                           int xi, bool sym, double omega);
void launch_u_restrict(hipStream_t s, const ULev& Lf, const ULev& Lc, USegs inner_c, const UList& lst_c,
                       const double* rf, double* rc);
void launch_u_prolong(hipStream_t s, const ULev& Lc, const ULev& Lf, USegs all_f, const double* xc, double* xf,
                      bool add, bool skip_bnd);
void launch_u_inject(hipStream_t s, const ULev& Lf, const ULev& Lc, USegs all_c, const double* xf, double* xc);
void launch_u_copy_bnd(hipStream_t s, const ULev& L, const unsigned char* flags, const double* src, double* dst);
// Zero the Dirichlet velocity rows and every pressure row of b.
void launch_u_rhs_fix(hipStream_t s, const ULev& L, const unsigned char* flags, double* b);
void launch_u_from_canon(hipStream_t s, const ULev& L, const int* canon, int nnodes, const double* src, double* dst);
void launch_u_to_canon(hipStream_t s, const ULev& L, const int* canon, const unsigned char* flags, int nnodes,
                       const double* src, double* dst);
void launch_u_pfrom_canon(hipStream_t s, const ULev& L, const int* canon, const double* src, double* p);
// sums[out] = sum over the owner slots s and the `nf` fields f from f0 of
// w[s] x_f[s] y_f[s] (w = null: 1; y = null: 1).
void launch_u_dot(hipStream_t s, const ULev& L, const unsigned char* flags, const double* w, const double* x,
                  const double* y, int f0, int nf, double* partial, double* sums, int out);
// p -= sums[slot] / denom on every slot of the pressure field.
void launch_u_shift(hipStream_t s, const ULev& L, double* p, const double* sums, int slot, double denom);
// p *= 1 / sqrt(sums[slot]) on every slot of the pressure field.
void launch_u_pscale(hipStream_t s, const ULev& L, double* p, const double* sums, int slot);
// Copy the owner value of every interface node to its other copies (all four fields).
void launch_u_sync(hipStream_t s, const ULev& L, const UList& lst, double* x);

// Host side (umesh.hip).
// Checks (xyz, tet) as a tetrahedral mesh: indices in range, every vertex
// used, no degenerate or repeated tetrahedron, no face in more than two
// tetrahedra, the two at a shared face on opposite sides of it (HHG_ERR_ARG
// naming the first violation otherwise).
void validate_tet_mesh(const double* xyz, int nv, const int* tet, int nt);
// Boundary faces (sorted vertex triples) lying on the listed planes of the
// unit cube (bit f: 0 x = 0, 1 x = 1, 2 y = 0, 3 y = 1, 4 z = 0, 5 z = 1).
std::vector<std::array<int, 3>> boundary_faces_on_cube(const double* xyz, int nv, const int* tet, int nt,
                                                       unsigned faces);
// Every outflow face a boundary face of the mesh, at least one boundary face
// left Dirichlet (HHG_ERR_ARG otherwise).
void check_outflow_faces(const int* tet, int nt, const std::vector<std::array<int, 3>>& outflow);

// Levels lmin..lmax of an unstructured hierarchy (device tables in `mem`).
struct UHier {
  int lmin = 0, lmax = 0, ncell = 0;
  std::vector<ULevelData> lv;
  std::vector<void*> mem;
  ULevelData& L(int l) { return lv[l - lmin]; }
  ~UHier();
};
// Builds every level (cell rows, slot tables, interface lists and colours,
// segments, the Schur diagonal of option `schur`); `outflow`: boundary
// faces (sorted vertex triples) with the natural outflow condition, the
// other boundary faces (and their closure) Dirichlet.  Synchronous.
UHier* u_build(const double* xyz, int nv, const int* tet, int nt, const std::vector<std::array<int, 3>>& outflow,
               int lmin, int lmax, int schur);
// Coarse unknowns of level lmin (array positions of the free velocity nodes'
// owner slots in three components, then of every pressure node) and the
// operator calA restricted to them (row-major, n x n), assembled on the host
// from the cell rows; K is left empty when there are more than max_n unknowns.
void u_coarse_system(UHier& u, std::vector<int>& unk, std::vector<double>& K, int max_n);
// Host-only view of one level's tables (hhg_query_umesh).
void u_query(const double* xyz, int nv, const int* tet, int nt, unsigned cube_outflow, int level, int schur,
             int max_unknowns, int* nnodes, int* ncolours, int* nunk, double* pos, int* colour, double* sdiag,
             double* K);

}  // namespace hhg
