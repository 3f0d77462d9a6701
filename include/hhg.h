/*
 * hhg.h -- C ABI of libhhg: matrix-free hierarchical-hybrid-grid multigrid for
 * the Stokes system on MI355X (gfx950).
 *
 * Method: Kohl & Ruede, "Textbook efficiency: massively parallel matrix-free
 * multigrid for the Stokes system".  Discrete problem: Sec. 2, eq.
 * stokes-discrete (calA = [[A, B^T], [B, -C]], A = diag(A, A, A)), PSPG
 * stabilisation eq. pspg (P1-P1) or C = 0 (P2-P1 Taylor-Hood).  Smoother:
 * Sec. 3.2, eq. uzawa-iteration.  Transfer: Sec. 3.3.  Cycles: Alg. fmg.
 *
 * Domain and hierarchy.  The macro mesh (hhg_mesh) is the unit cube split into
 * the six Kuhn tetrahedra (macro_refine = 0) or the 48 tetrahedra of one Bey
 * step of it (macro_refine = 1).  Bey refinement keeps Kuhn simplices, so
 * level l is the Freudenthal lattice with N = 2^(l + macro_refine) intervals
 * per cube edge and every macro-primitive's refined DoFs are sub-lattices of
 * it.  Velocity is
 * Dirichlet on the whole boundary; the pressure is fixed by int p = 0.
 *
 * Unstructured macro meshes (Sec. 2, 2.1: HHG on any T_0): hhg_mesh_create
 * with a tetrahedral mesh that is not a Kuhn partition of the cube gives the
 * per-cell path, P1-P1 PSPG in float64.  Each macro cell (vertices sorted by
 * id, v0 < v1 < v2 < v3) is refined by Bey's rule; level l has n = 2^l
 * intervals per macro edge.  Velocity is Dirichlet on the faces of T_0 that
 * belong to one tetrahedron (and on their edges and vertices).  Nodes are
 * numbered in "canonical order": nodes on vertices of T_0, then on edges,
 * faces and cells; within one kind by the sorted vertex ids of the
 * primitive, then lexicographically by the node's barycentric weights on
 * those vertices (in vertex-id order).  Gauss-Seidel colours: nodes on
 * vertices, edges and faces greedily in canonical order (the smallest colour
 * that no earlier node sharing an element with it has), K colours, then the
 * cell interiors in four colours K + (i + j + k) mod 4, (i, j, k) = (n - a0,
 * n - a0 - a1, a3) from the weights a.  The library stores each cell's
 * closed lattice with copies of the interface nodes; callers see the layout
 * only through hhg_vec_layout and the conversions.
 *
 * Vectors.  All vectors are caller-owned device buffers holding every DoF of a
 * level, Dirichlet velocity DoFs included (they carry the boundary data; the
 * lifting of Sec. 2 comes from applying the operator to them).  Layout (in
 * elements of the chosen precision), with n1 = N + 1 and nn = n1^3:
 *   P1-P1: [u1 | u2 | u3 | p], each nn words, index i + n1 (j + n1 k).
 *   P2-P1: [u1 | u2 | u3 | p], each velocity component 8 groups of nn words:
 *          group 0 = vertex DoFs (doubled-lattice position 2(i,j,k)), groups
 *          1..7 = edge DoFs of direction (1,0,0), (0,1,0), (0,0,1), (1,1,0),
 *          (1,0,1), (0,1,1), (1,1,1) at position 2(i,j,k) + dir; entries whose
 *          position leaves [0, 2N]^3 are padding and stay zero.
 * hhg_vec_layout() reports the sizes; hhg_vec_from_lattice / _to_lattice
 * convert to and from the plain lattice order (u1, u2, u3 over the velocity
 * lattice X + (M+1)(Y + (M+1) Z), M = N or 2N, then p over the P1 lattice);
 * on an unstructured mesh the plain order is [u1 | u2 | u3 | p], each over
 * the nodes in canonical order.
 *
 * Outputs: boundary velocity rows of every operator output are zero; pressure
 * rows exist at every pressure node.
 *
 * Precision: HHG_F64 (double storage and arithmetic) and HHG_F32 (float
 * storage, float accumulation).  Calls are asynchronous on the context's HIP
 * stream unless they return host values.
 *
 * Errors: every call returns an hhg_status; hhg_last_error() gives a message for
 * the calling thread.  No C++ exception crosses this interface.
 */
#ifndef HHG_H
#define HHG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int hhg_status;
enum {
  HHG_OK = 0,
  HHG_ERR_ARG = 1,            /* bad level, pointer, size or enum value          */
  HHG_ERR_PREC = 2,           /* precision not supported for this call          */
  HHG_ERR_HIP = 3,            /* a HIP runtime call failed                      */
  HHG_ERR_OOM = 4,            /* device allocation failed                       */
  HHG_ERR_NOT_CONVERGED = 5,  /* stopping test not met (stats still filled)     */
  HHG_ERR_STATE = 6           /* call needs setup that has not been done        */
};

typedef struct hhg_ctx_s* hhg_ctx;
typedef struct hhg_mesh_s* hhg_mesh;
typedef struct hhg_hier_s* hhg_hier;
typedef struct hhg_mlp_s* hhg_mlp;

typedef enum { HHG_P1P1 = 0, HHG_P2P1 = 1 } hhg_disc;
/* Storage precision of a vector.  HHG_BF16 (bfloat16 words) is accepted only
 * where a call says so; elsewhere it is refused with HHG_ERR_PREC. */
typedef enum { HHG_F64 = 0, HHG_F32 = 1, HHG_BF16 = 2 } hhg_prec;
/* Operator blocks of eq. stokes-discrete; MASS = consistent velocity mass and
 * P1 pressure mass (used for right-hand sides and error norms). */
typedef enum { HHG_OP_FULL = 0, HHG_OP_A = 1, HHG_OP_BT = 2, HHG_OP_B = 3, HHG_OP_C = 4, HHG_OP_MASS = 5 } hhg_op;
/* Velocity relaxation of eq. uzawa-velocity: A_f (forward Gauss-Seidel) or A_s
 * (forward then backward). */
typedef enum { HHG_GS_FWD = 0, HHG_GS_SYM = 1 } hhg_gs;
/* Diagonal D of S_hat = omega^{-1} D in eq. uzawa-pressure.  SD: diag(C + B
 * diag(A)^{-1} B^T) over interior velocity DoFs; ML: lumped P1 mass. */
typedef enum { HHG_SCHUR_SD = 0, HHG_SCHUR_ML = 1 } hhg_schur;

/* FMG(nu_pre, nu_post, nu_inc, kappa, A_hat, xi) of Alg. fmg plus omega^{-1}. */
typedef struct {
  int nu_pre, nu_post, nu_inc, kappa;
  hhg_gs gs;
  int xi;
  double omega_inv;       /* S_hat = omega_inv * D                          */
  int extra_cycles;       /* V-cycles on the finest level after FMG          */
  double rtol;            /* > 0: instead of extra_cycles, cycle until
                             ||r||_2 <= rtol ||b||_2 (max_cycles bound)       */
  int max_cycles;
  int coarse_smooth;      /* > 0: no coarse solve; the coarsest level gets this
                             many Uzawa iterations instead (comparison point
                             for the learned coarse solve); 0: exact solve, or
                             the attached network                           */
} hhg_solver_params;

typedef struct {
  int cycles;             /* V-cycles on the finest level (FMG's included)  */
  double res_u, res_p;    /* Euclidean norms of the final residual blocks    */
  double rel_res;         /* ||r|| / ||b||                                   */
  double work_units;      /* Sec. 4 model, in W(calA_L)                      */
  double seconds;         /* device time of the call on the context stream
                             (HIP events around its work)                   */
  int fallbacks;          /* learned coarse solve switched off (hhg_hier_set_mlp),
                             or float32 corrections given up (hhg_dc_solve) */
} hhg_stats;

/* ---------------------------------------------------------------- context */
/* Select device `device`; `stream` is a hipStream_t (NULL: the null stream).
 * The context owns nothing else; destroy it after every hierarchy made on it. */
hhg_status hhg_ctx_create(int device, void* stream, hhg_ctx* out);
hhg_status hhg_ctx_set_stream(hhg_ctx ctx, void* stream);
hhg_status hhg_ctx_destroy(hhg_ctx ctx);
const char* hhg_last_error(void);

/* ------------------------------------------------------------ macro mesh */
/* The macro mesh T_0 of Sec. 2 (host data; no device memory).
 *
 * hhg_mesh_cube: the unit cube split into the six Kuhn tetrahedra sharing the
 * diagonal (0,0,0)-(1,1,1) (macro_refine = 0), or the 48 tetrahedra of one
 * Bey refinement step of them (macro_refine = 1, the six Kuhn tetrahedra of
 * each of the eight half-size sub-cubes).
 *
 * hhg_mesh_create: an explicit T_0.  xyz: host, nv x 3 doubles (vertex
 * coordinates); tet: host, nt x 4 vertex indices (any vertex order within a
 * tetrahedron, any order of the tetrahedra).  Copied.  The lattice layout of
 * this library needs a T_0 whose uniform refinement is one Freudenthal
 * lattice: the call accepts a partition of the unit cube into the Kuhn
 * tetrahedra of its N^3 sub-cubes, N = 1 or 2 (6 or 48 tetrahedra; every
 * vertex on the lattice within 1e-9, no duplicate or unused vertex, every
 * tetrahedron a Kuhn simplex, no tetrahedron twice) as the lattice path; any
 * other conforming tetrahedral mesh becomes an unstructured mesh (per-cell
 * path; hhg_mesh_info reports macro_refine = -1).  Checked: indices in range,
 * every vertex used, no tetrahedron with a repeated vertex, degenerate
 * (|det| <= 1e-10 of its extent cubed) or given twice, no face in more than
 * two tetrahedra, the two tetrahedra at a shared face on opposite sides of
 * it; HHG_ERR_ARG with a message naming the first violation otherwise.
 * Conformity (faces meet whole faces) and the absence of overlaps between
 * tetrahedra that share no face are the caller's to ensure.
 *
 * A hierarchy copies what it needs: the mesh may be destroyed after
 * hhg_hier_create.  hhg_mesh_info: vertex and tetrahedron counts and the
 * macro refinement (N = 2^macro_refine sub-cubes per edge). */
hhg_status hhg_mesh_cube(hhg_ctx ctx, int macro_refine, hhg_mesh* out);
hhg_status hhg_mesh_create(hhg_ctx ctx, const double* xyz, int nv, const int* tet, int nt, hhg_mesh* out);
hhg_status hhg_mesh_info(hhg_mesh mesh, int* nv, int* nt, int* macro_refine);
/* Natural outflow boundary (Sec. 2: du/dn = n p on the Neumann part of the
 * boundary, u = w on the Dirichlet part).  faces: bit f marks face f of the
 * unit cube as outflow (0: x = 0, 1: x = 1, 2: y = 0, 3: y = 1, 4: z = 0,
 * 5: z = 1); the others stay Dirichlet, and the Dirichlet part is closed (a
 * site on an edge or corner of a Dirichlet face is Dirichlet).  Default 0 (all
 * Dirichlet); 63 is refused (HHG_ERR_ARG: the velocity would have a null
 * space).  Applies to hierarchies created afterwards.  On such a hierarchy the
 * outflow sites are unknowns of every operator, smoother, transfer and solve;
 * the pressure is determined, so the solvers do no mean-zero projection
 * (hhg_project_mean_zero still projects when called); the vectors keep their
 * layout (the outflow sites hold values, not boundary data:
 * hhg_copy_boundary skips them); variable viscosity is refused
 * (HHG_ERR_STATE) and the one-workgroup small-level V-cycle is not used.
 * Unstructured meshes: the boundary triangles of the mesh lying on those
 * planes of the unit cube (within 1e-12) become outflow faces (HHG_ERR_ARG if
 * there is none, or if no boundary face would stay Dirichlet); the other
 * boundary faces and their closure stay Dirichlet. */
hhg_status hhg_mesh_set_outflow(hhg_mesh mesh, unsigned faces);
/* Unstructured meshes: outflow faces given as boundary triangles, tri = ntri
 * x 3 vertex indices (host, any vertex order; ntri = 0 clears them).  Every
 * triangle must be a face of exactly one tetrahedron and at least one
 * boundary face must stay Dirichlet, else HHG_ERR_ARG; Kuhn-partition meshes
 * refuse the call (they take hhg_mesh_set_outflow).  As there, the solvers
 * then do no mean-zero projection.  Applies to hierarchies created
 * afterwards. */
hhg_status hhg_mesh_set_outflow_faces(hhg_mesh mesh, const int* tri, int ntri);
hhg_status hhg_mesh_destroy(hhg_mesh mesh);

/* ------------------------------------------------------------- hierarchy */
/* Build levels lmin..lmax (lmin is the coarsest, solved directly when it has
 * at most 2048 unknowns; otherwise hhg_coarse_solve, hhg_vcycle and
 * hhg_fmg_solve report HHG_ERR_STATE and the hierarchy serves operators and
 * transfers only) of one
 * discretisation: lattice sizes, stencil weights (computed on the host from
 * the element matrices of the six Kuhn tetrahedra, Sec. 2.1: constant per
 * macro-primitive), the dense pseudo-inverse of the coarsest operator, and
 * library work vectors (one residual per level plus the V-cycle and FMG
 * vectors of the coarser levels), all in the given working precision.
 * Level l of a mesh with macro refinement r has N = 2^(l + r) intervals per
 * cube edge.  Limits: 0 <= lmin < lmax, N(lmax) <= 512 (P1-P1) or 256
 * (P2-P1); Taylor-Hood needs N(lmin) >= 2 (a level-0 Taylor-Hood system on
 * six tetrahedra has spurious pressure modes).  The hierarchy runs on the
 * mesh's context.  Ownership: the hierarchy.
 *
 * Unstructured mesh: disc must be HHG_P1P1 and 0 <= lmin < lmax <= 9 (the
 * whole vector under 2^31 words); every call on the hierarchy takes HHG_F64
 * vectors (HHG_ERR_PREC otherwise); variable viscosity, defect correction,
 * bfloat16 levels, the learned coarse solve and its recorder report
 * HHG_ERR_STATE.  Work units are those of the P1-P1 model of Sec. 4. */
hhg_status hhg_hier_create(hhg_mesh mesh, hhg_disc disc, int lmin, int lmax, hhg_schur schur, hhg_hier* out);
hhg_status hhg_hier_destroy(hhg_hier h);

/* Sizes of one level: N, words per lattice array (nn = (N+1)^3), words of a
 * whole vector, words of the plain lattice-order vector. */
hhg_status hhg_vec_layout(hhg_hier h, int level, int* N, size_t* nn, size_t* vec_words,
                          size_t* lattice_words);

/* Device-to-device conversion between the plain lattice order (always double)
 * and the library layout in precision `prec` (double -> float rounds to
 * nearest even).  Padding entries are written as zero. */
hhg_status hhg_vec_from_lattice(hhg_hier h, int level, const double* src_lattice, void* dst, hhg_prec prec);
hhg_status hhg_vec_to_lattice(hhg_hier h, int level, const void* src, double* dst_lattice, hhg_prec prec);

/* Variable viscosity nu(x) on one level (not in the paper's experiments):
 * the A block becomes sum_T nu_T int_T grad phi_i . grad phi_j per velocity
 * component, nu_T the mean of nu at the four vertices of T.  nu: device,
 * double, nn words, the nodal values at the P1 nodes of `level` (lattice
 * order); copied.  Rebuilds the Gauss-Seidel diagonals, the Schur diagonal D
 * and, on the coarsest level, the coarse pseudo-inverse.  Set it on every
 * level of a solve.  Synchronous. */
hhg_status hhg_set_viscosity(hhg_hier h, int level, const double* nu);

/* ------------------------------------------------------------- operators */
/* y = op x on `level` (eq. stokes-discrete blocks; FULL = calA).  A and BT
 * fill the velocity part of y and zero its pressure part, B and C the
 * reverse (C = the PSPG matrix, i.e. minus the block of calA).  MASS: the
 * consistent velocity mass on every velocity DoF (boundary rows included) and
 * the P1 pressure mass.  x and y must not overlap. */
hhg_status hhg_apply(hhg_hier h, int level, hhg_op op, const void* x, void* y, hhg_prec prec);
/* r = b - calA x (Alg. fmg defect; boundary velocity rows zero). */
hhg_status hhg_residual(hhg_hier h, int level, const void* x, const void* b, void* r, hhg_prec prec);
/* b = (M I(f) on interior velocity rows, 0 on pressure rows): the load vector
 * of Sec. 2 with f given by its nodal values f_nodal (velocity part used). */
hhg_status hhg_rhs(hhg_hier h, int level, const void* f_nodal, void* b, hhg_prec prec);
/* `iters` inexact Uzawa iterations (eq. uzawa-iteration) in place on x:
 * xi multicolour Gauss-Seidel sweeps (gs) on A u = f - B^T p_k, then
 * p <- p - omega D^{-1} (g - B u + C p_k) with omega = 1 / omega_inv. */
hhg_status hhg_smooth(hhg_hier h, int level, void* x, const void* b, int iters, hhg_gs gs, int xi,
                      double omega_inv, hhg_prec prec);
/* r_coarse = restriction of r_fine (transpose of hhg_prolong_add's
 * interpolation, Sec. 3.3); fine boundary velocity rows are ignored, coarse
 * boundary velocity rows set to zero, the coarse pressure part shifted to
 * zero sum. */
hhg_status hhg_restrict(hhg_hier h, int fine_level, const void* r_fine, void* r_coarse, hhg_prec prec);
/* x_fine += I x_coarse: quadratic interpolation of P2 velocity, linear of
 * P1 fields (Sec. 3.3). */
hhg_status hhg_prolong_add(hhg_hier h, int coarse_level, const void* x_coarse, void* x_fine, hhg_prec prec);
/* x <- x + calA_lmin^+ (b - calA x) on the unknowns of the coarsest level,
 * then zero pressure mean.  F64 only. */
hhg_status hhg_coarse_solve(hhg_hier h, void* x, const void* b, hhg_prec prec);
/* p <- p - (m^T p / m^T 1), m_k = int psi_k (Sec. 2 mean-zero pressure). */
hhg_status hhg_project_mean_zero(hhg_hier h, int level, void* x, hhg_prec prec);
/* Copy the boundary velocity values of `src` (level `level`) into the
 * boundary velocity DoFs of `dst` on level `level` (same level) */
hhg_status hhg_copy_boundary(hhg_hier h, int level, const void* src, void* dst, hhg_prec prec);

/* Largest eigenvalue of D^{-1}(C + B A_s^{-1} B^T) by `iters` power
 * iterations (eq. omega-eigenvalue-problem; A_s^{-1}: one forward + one
 * backward sweep from zero).  v0: caller-drawn start vector on the pressure
 * nodes (device, double, nn words, P1 lattice order).  Synchronous. */
hhg_status hhg_estimate_omega(hhg_hier h, int level, const double* v0, int iters, double* omega_inv);

/* Dot products x.y of the velocity parts and of the pressure parts
 * (synchronous); with y = hhg_apply(MASS) of x they are squared M-norms. */
hhg_status hhg_dots(hhg_hier h, int level, const void* x, const void* y, double* dot_u, double* dot_p,
                    hhg_prec prec);

/* Kernel event timer (process-wide, for measurement).  hhg_timer_start
 * enables HIP events around every launch of the kernel families in the mask
 * (bit f = family f: 0 apply/residual, 1 boundary pressure rows, 2 vertex
 * Gauss-Seidel colour, 3 edge-group Gauss-Seidel colour, 4 Uzawa pressure
 * step, 5 restriction, 6 prolongation, 7 coarse solve, 8 reductions, 9 other,
 * 10 MLP matrix products, 11 one-workgroup small-level V-cycle, 12
 * outflow-face rows, Gauss-Seidel sites and transfers, 13 interface-node
 * rows, Gauss-Seidel colours and copies of unstructured meshes; on those
 * meshes family 0 is the cell-interior rows and 2 the interior colours)
 * and clears earlier records; mask 0 disables it.  hhg_timer_read synchronises
 * and returns, for one family since the last read, the summed event time in
 * ms, the launches and the work units (sites processed: P2 sites or P1
 * nodes for apply/transfers, updated sites for Gauss-Seidel colours). */
hhg_status hhg_timer_start(unsigned family_mask);
hhg_status hhg_timer_read(int family, double* total_ms, int* launches, double* units);

/* Euclidean norms of the velocity and pressure parts of x (synchronous). */
hhg_status hhg_norms(hhg_hier h, int level, const void* x, double* norm_u, double* norm_p, hhg_prec prec);

/* ------------------------------------------------------ host-only queries */
/* The row stencil the library applies, at h = 1, computed on the host from
 * the element matrices (no device needed).  kind: 'A' stiffness, 'M' velocity
 * mass, 'T' B^T (velocity row -> pressure columns), 'B' (pressure row ->
 * velocity columns), 'C' P1 stiffness (PSPG C = C-row * delta h_T^2 / h), 'P'
 * P1 mass.  Row: velocity group `group` (0 for P1 / pressure rows) at index
 * (i, j, k), summed over the lattice elements inside [0, nbox]^3.  Output
 * entries: code[4 e .. 4 e + 3] = (column group, di, dj, dk), w[3 e .. 3 e +
 * 2] = weights (three for 'T' and 'B', else w[3 e] only).  *n = number of
 * entries; HHG_ERR_ARG if more than max_entries. */
hhg_status hhg_query_stencil(hhg_disc disc, char kind, int group, int i, int j, int k, int nbox, int max_entries,
                             int* n, int* code, double* w);
/* Host-only view of level `level` (0..6) of an unstructured mesh (xyz, tet
 * as for hhg_mesh_create; any valid tetrahedral mesh, Kuhn partitions
 * included; cube_outflow: outflow faces as for hhg_mesh_set_outflow on an
 * unstructured mesh, 0 for none): the number of nodes, of Gauss-Seidel colours and of coarse
 * unknowns (free velocity nodes times three, then every pressure node); per
 * node in canonical order (arrays of nnodes entries, or NULL): position
 * (3 doubles), colour, Schur diagonal D of option `schur`; and calA on the
 * unknowns (nunk x nunk, row-major; velocity unknowns component-major, nodes
 * ascending, then the pressure nodes) if nunk <= max_unknowns and K is not
 * NULL.  Call once with NULL arrays for the sizes. */
hhg_status hhg_query_umesh(const double* xyz, int nv, const int* tet, int nt, unsigned cube_outflow, int level,
                           hhg_schur schur, int max_unknowns, int* nnodes, int* ncolours, int* nunk, double* pos,
                           int* colour, double* schur_diag, double* K);
/* Interpolation weights of Sec. 3.3 at a fine position inside one coarse
 * lattice cube: t = (tx, ty, tz) / q with q = 2 (linear) or 4 (quadratic)
 * and order 1 or 2.  Output: code[4 e ..] = (coarse group, di, dj, dk) from the
 * cube origin, w[e]; at most 10 entries. */
hhg_status hhg_query_interpolation(int order, int tx, int ty, int tz, int q, int* n, int* code, double* w);

/* ----------------------------------------------------------------- cycles */
/* One variable V-cycle of Alg. fmg on x (finest level `level`,
 * l_fine = level), storage and arithmetic in `prec` (the coarsest-level
 * pseudo-inverse is applied in float64 either way; the learned coarse solve
 * and the training-pair recorder act on float64 cycles only). */
hhg_status hhg_vcycle(hhg_hier h, int level, void* x, const void* b, const hhg_solver_params* prm, hhg_prec prec);
/* Alg. fmg on lmin..lmax.  b_levels[l - lmin]: right-hand sides of every level
 * (hhg_rhs); x: finest-level vector whose boundary velocity DoFs hold the
 * boundary data (interpolated to coarser levels by injection), overwritten by
 * the solution.  Then extra_cycles V-cycles (or cycles to rtol).  Stats
 * optional (NULL).  F64. */
hhg_status hhg_fmg_solve(hhg_hier h, void* x, const void* const* b_levels, const hhg_solver_params* prm,
                         hhg_stats* stats);

/* Defect correction (iterative refinement) in float64 around inner cycles in
 * `inner_prec`: repeat r = b - calA x (float64); stop when ||r||_2 <= rtol
 * ||b||_2 or after max_outer corrections; otherwise convert r to the inner
 * precision (round to nearest even), run inner_cycles variable V-cycles
 * (prm's smoothing parameters, arithmetic and storage in inner_prec, the
 * coarsest-level pseudo-inverse applied in float64) on calA e = r from e = 0,
 * x += e in float64 and project the pressure to zero mean in float64.  x holds
 * the boundary data and the start vector.  Fallback: when a float32
 * correction does not reduce the float64 residual norm (or makes it not
 * finite), it is undone and the remaining corrections use float64 inner
 * cycles (stats->fallbacks = 1).  Stats: cycles = inner V-cycles in total
 * (an undone correction's included), residual norms of the final x.
 * HHG_ERR_NOT_CONVERGED if rtol is not reached. */
hhg_status hhg_dc_solve(hhg_hier h, void* x, const void* b, const hhg_solver_params* prm, hhg_prec inner_prec,
                        int inner_cycles, double rtol, int max_outer, hhg_stats* stats);

/* ------------------------------------------------ learned coarse solve */
/* Not in the paper: a dense network n_in -> H -> H -> H -> n_out (ReLU)
 * that stands in for the exact coarse solve of Alg. fmg.  Weights and layer
 * inputs are bfloat16 (round to nearest even), products run on the matrix
 * cores with float32 accumulation, master weights and Adam moments are float32.
 * Parameter order (host, float32): W1 (H x n_in, row-major), b1, W2, b2, W3,
 * b3, W4 (n_out x H), b4.  max_batch bounds every batch.  The MLP belongs to a
 * context; destroy it before the context. */
hhg_status hhg_mlp_create(hhg_ctx ctx, int n_in, int n_hidden, int n_out, int max_batch, hhg_mlp* out);
hhg_status hhg_mlp_destroy(hhg_mlp m);
hhg_status hhg_mlp_num_params(hhg_mlp m, size_t* n);
/* Copy parameters in (resets the Adam state) or out. */
hhg_status hhg_mlp_set_params(hhg_mlp m, const float* host_params);
hhg_status hhg_mlp_get_params(hhg_mlp m, float* host_params);
/* y = net(x); x, y device float32, batch x n_in and batch x n_out. */
hhg_status hhg_mlp_forward(hhg_mlp m, const float* x, int batch, float* y);
/* Mean squared error over the n_out outputs of the batch and its gradient
 * (host float32, parameter order) -- synchronous. */
hhg_status hhg_mlp_loss_grad(hhg_mlp m, const float* x, const float* y, int batch, float* grad_host, double* loss);
/* Adam (beta 0.9 / 0.999, eps 1e-8) over minibatches: for epoch e the samples
 * order[e n_samples + i] (host, caller-drawn) are taken batch by batch; x, y
 * device float32 datasets (n_samples rows).  last_loss: mean batch loss of the
 * final epoch. */
hhg_status hhg_mlp_train(hhg_mlp m, const float* x, const float* y, int n_samples, int batch, int epochs, float lr,
                         const int* order, double* last_loss);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving or training loops, harnesses that forbid hipMalloc):
 * hhg_mlp_train without allocation.  Same arguments, arithmetic and results
 * as hhg_mlp_train (bit for bit), but the device copy of the sample order and
 * the per-epoch loss accumulators live in a static device array of the
 * library (one per GPU, 8 MiB + 32 KiB, held until the process ends) instead
 * of memory allocated per call; the call makes no hipMalloc / hipFree.
 * Limits: epochs * n_samples <= 2^21 and epochs <= 4096, else HHG_ERR_ARG.
 * Every call on a GPU shares that array: calls that overlap on one GPU (other
 * threads, other contexts or streams of the same device) race and must be
 * serialised by the caller.  Synchronous. */
hhg_status hhg_mlp_train_noalloc(hhg_mlp m, const float* x, const float* y, int n_samples, int batch, int epochs,
                                 float lr, const int* order, double* last_loss);
/* Feature and output sizes of the learned coarse solve of this hierarchy:
 * n_out = coarse unknowns (interior velocity, then pressure), n_in = n_out +
 * P1 nodes of the coarsest level. */
hhg_status hhg_mlp_dims(hhg_hier h, int* n_in, int* n_out);
/* One training pair from a coarsest-level vector r (device, float64, library
 * layout): features = [r_unk / ||r_unk||, log nu at the coarse P1 nodes (0
 * without viscosity)], target = (exact coarse correction)_unk / ||r_unk|| with
 * the pressure at zero mean.  Outputs device float32. */
hhg_status hhg_coarse_pair(hhg_hier h, const double* r, float* features, float* target);
/* Cycles on the small levels: a V-cycle whose top level has at most
 * max_sites velocity sites per component ((N+1)^3 for P1-P1, (2N+1)^3 for
 * P2-P1) runs from that level down to the coarse solve and back up in one
 * single-workgroup kernel (phases separated by workgroup barriers instead of
 * kernel launches; same arithmetic, sums in a different order), with the
 * level vectors held in LDS when the levels up to the top fit in 128 KB.
 * Applies to V-cycles with the exact coarse solve (not with a network
 * attached, the recorder on or coarse_smooth > 0).  Default 800; 0 turns it
 * off.  On an unstructured macro mesh the same bound is on a level's slots
 * (cells times points per cell) and applies to every smoothing call
 * (hhg_smooth and the smoothing inside cycles): one workgroup runs the whole
 * call, every value computed as by the per-colour launches; default 300
 * (the cube benchmark's level 1), meshes of at most 64 cells. */
hhg_status hhg_hier_set_fused_sites(hhg_hier h, long max_sites);
/* Not in the paper: bfloat16 storage on the coarse levels of float32
 * cycles.  The n coarsest levels (lmin .. lmin + n - 1, 0 <= n <= number of
 * levels; default 0) hold bfloat16 values: every float32 operation that
 * writes a vector of such a level -- apply, residual, rhs, mass, lattice
 * conversion, smoother (per colour and pressure step), restriction,
 * prolongation, coarse solve, mean-zero projection, and the inner cycles of
 * hhg_dc_solve -- rounds the words it writes to the nearest bfloat16 (ties
 * to even).  The values stay in the float32 vectors (layout unchanged):
 * bfloat16 to float32 is exact, so the arithmetic is that of bfloat16 storage
 * with float32 computation.  hhg_copy_boundary moves words unchanged; float64
 * operations are not affected. */
hhg_status hhg_hier_set_bf16_levels(hhg_hier h, int n);

/* Training-pair recorder: while capacity > 0, every exact float64 coarse
 * solve (inside hhg_vcycle, hhg_fmg_solve, hhg_dc_solve with F64 inner
 * cycles) also writes the pair of its residual, as hhg_coarse_pair does, into
 * row k of features (capacity x n_in) and targets (capacity x n_out), k = 0,
 * 1, ... until capacity rows are filled.  Device float32 buffers owned by the
 * caller and kept until recording stops (capacity 0).  Each call restarts the
 * count; solves run eagerly (no HIP-graph replay) while recording. */
hhg_status hhg_record_pairs(hhg_hier h, float* features, float* targets, int capacity);
hhg_status hhg_recorded_pairs(hhg_hier h, int* count);
/* Attach (or detach with m = NULL) a network as the coarse solve of float64
 * cycles: correction = ||r_unk|| net(features), then zero pressure mean.
 * Fallback (hhg_fmg_solve with rtol > 0): a finest-level cycle whose residual
 * ratio exceeds rho_plain (1 + tau), or is not finite, is undone and the rest
 * of that solve uses the exact coarse solve (counted in stats->fallbacks).
 * While a network is attached, hhg_set_viscosity on the coarsest level defers
 * the pseudo-inverse rebuild to the first exact coarse solve. */
hhg_status hhg_hier_set_mlp(hhg_hier h, hhg_mlp m, double rho_plain, double tau);

#ifdef __cplusplus
}
#endif
#endif /* HHG_H */
