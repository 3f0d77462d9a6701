// Kernel-side declarations shared by the launchers (host) and kernels.hip.
#pragma once
#include "hhg_internal.h"

namespace hhg {

// Geometry of one level: N intervals, n1 = N + 1 nodes per edge, nn = n1^3
// words per lattice array, G velocity groups (1: P1, 8: P2), vstride = G nn,
// nf = faces with the natural outflow condition (bit f: face f of the unit
// cube, 0: x = 0, 1: x = 1, 2: y = 0, 3: y = 1, 4: z = 0, 5: z = 1; the
// others are Dirichlet).
struct Geom {
  int N, n1, nn, G, vstride, nf;
};

// Gauss-Seidel colours of the lattice velocity: the vertex group (P1: every
// node) in two classes by (i + j + k) mod 2, then one colour per P2 edge
// group.  Two vertex classes suffice: on the Kuhn lattice the stiffness
// couples two vertex nodes only along a lattice axis (for the other edges of
// a Kuhn tetrahedron the barycentric gradients are orthogonal, so their
// entries vanish).
constexpr int kGsVertexColours = 2;
__host__ __device__ constexpr int gs_colours(int G) { return G == 1 ? kGsVertexColours : kGsVertexColours + 7; }

// Outflow-face velocity rows (Sec. 2, natural boundary condition): sites on
// Neumann faces (off the closed Dirichlet part) are unknowns whose rows are
// the element sums inside the cube, i.e. the boundary-class rows of their
// group.  Tables per (group, boundary class) = g * 27 + cls (cls = c_x + 3 c_y
// + 9 c_z with c = 0 low face, 1 inside, 2 high face, for the site's doubled
// coordinates): A rows (offsets relative to the site's array position,
// weights scaled to the level), B^T rows (offsets relative to the group-0
// index, three weights), 1 / a_ii, and the restriction rows from the next
// finer level (offsets relative to the fine group-0 index of 2 (i, j, k),
// fine group shift included) of the coarse sites of that level's list.
constexpr int kNeuSlots = 8 * 27;
template <typename T>
struct NeuTables {
  DStencil<T> A[kNeuSlots];
  DStencil<T> BT[kNeuSlots];
  DStencil<T> R[kNeuSlots];
  T adiag_inv[kNeuSlots];
};
// One list of outflow sites of a level, ordered by Gauss-Seidel colour: site
// q has array position pos[q] (group g nn + index) and table slot slot[q].
struct NeuList {
  const int* pos;
  const int* slot;
};

// Per-level constants of the generated interior stencils (weights at h = 1):
// A scales by h, B and B^T by h^2, PSPG C by delta (1/6)^(2/3) h^3, masses by
// h^3; ainv[g] = 1 / (a * A_gg).
// Variable viscosity: nu (P1 nodes, nn words) and ainv_site (1 / a_ii per
// velocity site, G nn words); both null for the constant-coefficient rows.
template <typename T>
struct LevelConst {
  T a, b, c, m;
  T ainv[8];
  const T* nu;
  const T* ainv_site;
};

// Stencil tables of one level in one precision (device pointers inside).
// Velocity rows exist only at interior velocity sites and use the unbounded
// lattice stencil; pressure rows use one of 27 boundary classes.
template <typename T>
struct Tables {
  DStencil<T> A[8];     // velocity row, group g -> velocity cols (offsets include group shift)
  DStencil<T> BT[8];    // velocity row, group g -> pressure cols, 3 weights/entry
  DStencil<T> Mv[8];    // velocity mass, interior rows
  DStencil<T> B[27];    // pressure row, class -> velocity cols (offset from group-0 index), 3 weights
  DStencil<T> C[27];    // pressure row, class -> pressure cols (PSPG; n = 0 for Taylor-Hood)
  const int* Bcode[27]; // packed (g, di+2, dj+2, dk+2) of the B entries (setup only)
  T adiag_inv[8];       // 1 / A_gg
  T mclass[27];         // int psi_k per boundary class
  const T* dinv;        // per pressure node 1 / D_k (Schur diagonal), nn words
  DStencil<T> Mfull[8 * 27];  // velocity mass rows of every group and boundary class
  DStencil<T> Pm[27];         // P1 pressure mass rows per boundary class
};

// Kernel families for the event timer (hhg_timer_*).
enum KernelFamily {
  KF_APPLY = 0,     // stencil apply / residual (interior pressure and all velocity rows)
  KF_PROW_BND = 1,  // boundary pressure rows (now extra blocks of the apply launches: no launches of their own)
  KF_GS_VERTEX = 2, // Gauss-Seidel colour of the vertex group
  KF_GS_EDGE = 3,   // Gauss-Seidel colour of one P2 edge group
  KF_PSTEP = 4,     // Uzawa pressure step
  KF_RESTRICT = 5,
  KF_PROLONG = 6,
  KF_COARSE = 7,
  KF_REDUCE = 8,
  KF_OTHER = 9,
  KF_MLP = 10,      // MLP matrix products (work units: flops)
  KF_SMALL = 11,    // one-workgroup V-cycle over the small levels
  KF_NEUMANN = 12,  // outflow-face rows, Gauss-Seidel and transfers
  KF_IFACE = 13,    // interface-node rows, Gauss-Seidel and copies of unstructured meshes
  KF_COUNT = 14
};
void timer_set_mask(unsigned mask);
bool timer_enabled();
// Records HIP events on the launch stream around one kernel launch when its
// family is enabled (kernels.hip).
struct KScope {
  hipStream_t s_;
  hipEvent_t b_ = nullptr;
  // packet = true: the events are left to the launch (launch_timed), which
  // has the dispatch packet stamp the kernel's own start and end -- the
  // kernel's execution time without the event and queue overhead around a
  // launch (for kernels of a few microseconds that overhead is most of a
  // bracketed measurement).  Not while the stream is being captured.
  hipEvent_t a_ = nullptr;
  bool packet_ = false;
  KScope(hipStream_t s, int fam, double units, bool packet = false);
  ~KScope();
};
// Sum of event-measured durations (ms), launches and work units of one family
// since the last read; synchronises the recorded events.
void timer_read(int family, double* total_ms, int* launches, double* units);

// Prolongation tables between level l-1 (coarse) and l (fine): fine class
// (S & 3 per coordinate, 64 classes for quadratic, 8 for linear on the P1
// lattice) -> 10 (coarse offset, weight) slots, offsets relative to the coarse
// cube (S >> 2 or S >> 1) position in group 0; slots past the class's weights
// hold offset 0 and weight 0.  (The restriction is generated code.)
template <typename T>
struct TransferTables {
  const int* vp_off;   // velocity prolongation [ncls][10], ncls = 64 (P2) or 8 (P1)
  const T* vp_w;
  const int* pp_off;   // P1 pressure prolongation [8][10]
  const T* pp_w;
};

// A V-cycle over the small levels lmin..ltop run by one workgroup (one
// launch; the phases are separated by workgroup barriers instead of kernel
// boundaries).  lv (device array) describes the levels from lmin: lv[q] is
// level lmin + q, its tt the transfer tables between levels lmin + q - 1 and
// lmin + q; the work vectors r, cx, cb of the levels below ltop are used, and
// x, b of the call replace cx, cb on ltop.
template <typename T>
struct SmallLevel {
  Geom g;
  LevelConst<T> lc;
  const Tables<T>* tb;
  const TransferTables<T>* tt;
  const T* dinv;
  const int* bnd;
  int nbnd;
  T *r, *cx, *cb;
  int lds_off;  // LDS element offset of this level's [cx | cb | r] copy, -1: none
};
template <typename T>
struct SmallCycle {
  int nlev;                 // ltop - lmin + 1 (>= 2)
  int G;
  int pre0, post0, inc;     // smoothing on level lmin + q: pre0 + (nlev - 1 - q) inc (post likewise)
  int gs_sym, xi, full_mask;
  T omega;
  T* x;                     // ltop vectors
  const T* b;
  const double* Kp;         // coarse pseudo-inverse (nunk x nunk, nunk <= 2048), unknown positions unk
  const int* unk;
  int nunk;
  int lds_words;            // > 0: every level's vectors live in LDS (x, b copied in and x out)
  int q16;                  // levels lmin + q, q < q16, hold bfloat16 values (float32 only)
};
// LDS available for the level vectors of the one-workgroup V-cycle (bytes).
constexpr int kSmallLdsBytes = 128 * 1024;
template <typename T>
void launch_vcycle_small(hipStream_t s, const SmallLevel<T>* lv, const SmallCycle<T>& sc);
// Allow kSmallLdsBytes of dynamic LDS for the one-workgroup V-cycle kernels.
void small_kernel_attributes();

// Uzawa pressure step fused into the pressure rows of a residual launch:
// with p set, a pressure row's residual r_k is not stored but applied as
// p_k -= omega dinv_k r_k (eq. uzawa-pressure).  Only for operators whose
// pressure rows do not read p (no C block: Taylor-Hood), so that the update
// in place races with no read.
template <typename T>
struct PStep {
  T* p = nullptr;
  const T* dinv = nullptr;
  T omega = T(0);
};

// Launchers (kernels.hip).  All asynchronous on `s`.
template <typename T>
void launch_apply(hipStream_t s, const Geom& g, const LevelConst<T>& lc, const Tables<T>* tb, const T* x, const T* b,
                  T* y, int opmask, bool has_b, bool vel_rows, bool p_rows, const int* bnd, int nbnd,
                  const PStep<T>& ps = PStep<T>{});
template <typename T>
void launch_gs_colour(hipStream_t s, const Geom& g, const LevelConst<T>& lc, T* x, const T* b, int colour);
template <typename T>
void launch_pressure_step(hipStream_t s, const Geom& g, const T* dinv, T* x, const T* rp, T omega);
template <typename T>
void launch_schur_diag(hipStream_t s, const Geom& g, const Tables<T>* tb, const T* ainv_site, int mode, T* dinv,
                       const NeuTables<T>* nt);
// Outflow-face kernels over the sites [first, first + n) of a level's list.
// Rows: y = [b -] (A (opmask 1) + B^T (opmask 2)) x at the sites.
template <typename T>
void launch_neu_rows(hipStream_t s, const Geom& g, const NeuTables<T>* nt, NeuList L, int first, int n, const T* x,
                     const T* b, T* y, int opmask, bool has_b);
// One Gauss-Seidel colour at the sites (the caller passes that colour's range).
template <typename T>
void launch_neu_gs(hipStream_t s, const Geom& g, const NeuTables<T>* nt, NeuList L, int first, int n, T* x,
                   const T* b);
// b = M f at the sites (boundary-class velocity mass rows of tb).
template <typename T>
void launch_neu_rhs(hipStream_t s, const Geom& g, const Tables<T>* tb, NeuList L, int n, const T* f, T* b);
// Coarse sites (list and tables of the coarse level): rc = R rf.
template <typename T>
void launch_neu_restrict(hipStream_t s, const Geom& gf, const Geom& gc, const NeuTables<T>* ntc, NeuList Lc, int n,
                         const T* rf, T* rc);
// Fine sites (list of the fine level): xf += I xc (interpolation tables of the fine level).
template <typename T>
void launch_neu_prolong(hipStream_t s, const Geom& gc, const Geom& gf, const TransferTables<T>* tt, NeuList Lf, int n,
                        const T* xc, T* xf);
template <typename T>
void launch_nu_diag(hipStream_t s, const Geom& g, const LevelConst<T>& lc, T* ainv_site);
template <typename T>
void launch_rhs(hipStream_t s, const Geom& g, const LevelConst<T>& lc, const T* fnod, T* b);
template <typename T>
void launch_mass(hipStream_t s, const Geom& g, const Tables<T>* tb, const T* x, T* y);
template <typename T>
void launch_dot(hipStream_t s, const T* x, const T* y, size_t n, double* partial, double* out);
template <typename T>
// zero_x (optional): a coarse vector set to zero word for word by the same
// threads (the coarse correction's start value), every word of the level.
void launch_restrict(hipStream_t s, const Geom& gf, const Geom& gc, const TransferTables<T>* tt, const T* rf, T* rc,
                     T* zero_x = nullptr);
template <typename T>
void launch_prolong(hipStream_t s, const Geom& gc, const Geom& gf, const TransferTables<T>* tt, const T* xc, T* xf,
                    bool add, bool skip_boundary);
template <typename T>
void launch_inject_boundary(hipStream_t s, const Geom& gf, const Geom& gc, const T* xf, T* xc);
template <typename T>
void launch_copy_boundary(hipStream_t s, const Geom& g, const T* src, T* dst);
template <typename T>
void launch_from_lattice(hipStream_t s, const Geom& g, const double* src, T* dst);
template <typename T>
void launch_to_lattice(hipStream_t s, const Geom& g, const T* src, double* dst);
// sum over pressure nodes of (weights per class) * p, or of p^2, into out[slot]
template <typename T>
void launch_psum(hipStream_t s, const Geom& g, const Tables<T>* tb, const T* p, double* partial, double* out,
                 int mode);
template <typename T>
void launch_pshift(hipStream_t s, const Geom& g, T* p, const double* sums, int mode);
// p -= (weighted, mode 0, or plain, mode 1) mean of p: launch_psum + launch_pshift,
// or one workgroup for levels with at most kMeanOneBlock pressure nodes.
constexpr int kMeanOneBlock = 65536;
template <typename T>
void launch_mean_zero(hipStream_t s, const Geom& g, const Tables<T>* tb, T* p, double* partial, double* sums,
                      int mode);
template <typename T>
void launch_vsumsq(hipStream_t s, const Geom& g, const T* x, int nwords, double* partial, double* out);
template <typename T>
void launch_coarse(hipStream_t s, const double* Kp, const int* unk, int nunk, const T* r, T* x);
void launch_unit_columns(hipStream_t s, double* E, size_t stride, const int* unk, int n);
void launch_to_f32(hipStream_t s, const double* x, float* y, size_t n);
void launch_coarse_features(hipStream_t s, const double* r, const int* unk, int nunk, const double* nu, int nn,
                            float* f, double* norm);
void launch_coarse_scatter(hipStream_t s, const float* y, const int* unk, int nunk, const double* norm, double* x,
                           float* out);
void launch_gather_rows(hipStream_t s, const float* src, const int* idx, int B, int w, float* dst);
void launch_add_f32_to_f64(hipStream_t s, double* y, const float* e, size_t n);
// Round to bfloat16 (nearest, ties to even) in place, stored as float32:
// x[s stride + off + t] for s < nseg, t < n.
void launch_round_bf16(hipStream_t s, float* x, size_t stride, size_t off, size_t n, int nseg);
template <typename T>
void launch_scale(hipStream_t s, T* x, size_t n, const double* sums, int slot);
template <typename T>
void launch_fill(hipStream_t s, T* x, size_t n, T v);
template <typename T>
void launch_scaled_copy(hipStream_t s, T* y, const T* x, const T* d, size_t n, T a);
template <typename T>
void launch_axpy(hipStream_t s, T* y, const T* x, size_t n, T a);

constexpr int kPartials = 1024;   // reduction partial slots

}  // namespace hhg
