// C ABI of libhhg: contexts, hierarchies, operators, cycles (include/hhg.h).
//
// Host-side driver of the paper's solver: Alg. fmg (FMG + variable V-cycle),
// eq. uzawa-iteration (inexact Uzawa relaxation in multicolour order),
// Sec. 3.3 (transfer), Sec. 2 (discrete Stokes operator).  Every numerical
// step runs in the kernels of kernels.hip; this file builds tables, owns work
// memory and sequences launches on the context stream.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <tuple>
#include <type_traits>
#include <unordered_map>

#include "kernels.h"
#include "mlp.h"
#include "umesh.h"

namespace hhg {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }

namespace {

const int kGroupDir[8][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1},
                             {1, 1, 0}, {1, 0, 1}, {0, 1, 1}, {1, 1, 1}};

// Device memory arena owned by a hierarchy.
struct Arena {
  std::vector<void*> ptrs;
  template <typename T>
  T* alloc(size_t n) {
    void* p = nullptr;
    if (n == 0) n = 1;
    hipError_t e = hipMalloc(&p, n * sizeof(T));
    if (e != hipSuccess) throw Error{HHG_ERR_OOM, std::string("hipMalloc: ") + hipGetErrorString(e)};
    ptrs.push_back(p);
    return (T*)p;
  }
  template <typename T>
  T* upload(const std::vector<T>& v) {
    T* p = alloc<T>(v.size());
    if (!v.empty()) HHG_CHECK_HIP(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return p;
  }
  ~Arena() {
    for (void* p : ptrs) (void)hipFree(p);
  }
};

// Host staging of one stencil set before upload.
struct HostStencil {
  std::vector<int> off;
  std::vector<double> w;  // nw per entry
  std::vector<int> code;
};

template <typename T>
DStencil<T> upload_stencil(Arena& a, const HostStencil& hs) {
  std::vector<T> wt(hs.w.begin(), hs.w.end());
  DStencil<T> d;
  d.off = a.upload(hs.off);
  d.w = a.upload(wt);
  d.n = (int)hs.off.size();
  return d;
}

int lin(int di, int dj, int dk, int n1) { return di + n1 * (dj + n1 * dk); }

}  // namespace

struct Level {
  int l = 0;
  Geom g{};
  double h = 1.0;
  int nbnd = 0;
  int* bnd = nullptr;  // boundary pressure node list
  Tables<double>* tb64 = nullptr;
  Tables<float>* tb32 = nullptr;
  TransferTables<double>* tt64 = nullptr;  // transfer from level l-1 to l
  TransferTables<float>* tt32 = nullptr;
  double* dinv64 = nullptr;
  float* dinv32 = nullptr;
  LevelConst<double> lc64{};
  LevelConst<float> lc32{};
  // variable viscosity (allocated by hhg_set_viscosity)
  double *nu64 = nullptr, *ainvs64 = nullptr;
  float *nu32 = nullptr, *ainvs32 = nullptr;
  size_t vec_words = 0;
  // work vectors (float64): residual, V-cycle correction / rhs, FMG iterate, boundary data
  double *r = nullptr, *cx = nullptr, *cb = nullptr, *xs = nullptr, *w = nullptr;
  float* r32 = nullptr;
  // float32 V-cycle vectors (allocated on first mixed-precision use)
  float *cx32 = nullptr, *cb32 = nullptr;
  // finest-level correction and right-hand side of a float64 inner solve;
  // the iterate before a float32 correction (undone if it does not help)
  double *dc_e = nullptr, *dc_r = nullptr, *dc_bk = nullptr;
  // host copies of the double tables (coarse assembly)
  std::vector<HostStencil> hA, hBT, hB, hC;
  double adiag[8] = {0};
  // outflow-face sites (ordered by colour; neu_coff[c] .. neu_coff[c + 1] is
  // colour c) and their row / restriction tables
  int neu_n = 0;
  int *neu_pos = nullptr, *neu_slot = nullptr;
  std::vector<int> neu_coff;
  NeuTables<double>* neu64 = nullptr;
  NeuTables<float>* neu32 = nullptr;
  NeuList neu() const { return NeuList{neu_pos, neu_slot}; }
};

}  // namespace hhg

struct hhg_mlp_s {
  hhg_ctx ctx = nullptr;
  hhg::Mlp net;
  int* idx = nullptr;       // device minibatch indices
  float *bx = nullptr, *by = nullptr;  // device minibatch
};

struct hhg_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;
  hipStream_t capture = nullptr;  // private stream for HIP-graph capture
  unsigned char* scratch = nullptr;  // this device's address of the static scratch array
};

// Static device scratch of the allocation-free entry point
// (hhg_mlp_train_noalloc): loss accumulators of up to kScratchEpochs epochs,
// then the sample order of up to kScratchOrder minibatch slots.  One copy per
// device, held until the process ends; in host code `scratch` is only a
// symbol: its device address comes from hipGetSymbolAddress (hhg_ctx_create).
constexpr size_t kScratchEpochs = 4096;
constexpr size_t kScratchOrder = (size_t)1 << 21;
constexpr size_t kScratchBytes = kScratchEpochs * sizeof(double) + kScratchOrder * sizeof(int);
// Default bound of the one-workgroup smoothing calls on unstructured meshes
// (slots of a level; hhg_hier_set_fused_sites).  An interface node's update
// is three dependent round trips (records, rows, own value), so one
// workgroup only wins where a colour is a single pass of its threads: on
// the cube benchmark (24 cells) level 1 (240 slots) gains, level 2 (840)
// loses (FMG solve: off 26.4 ms, up to level 1 25.8, up to level 2 28.2,
// up to level 3 47.6).
constexpr long kUFusedSlots = 300;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Macro mesh T_0 (host data): vertex coordinates, tetrahedra, and the number
// of Bey steps between the six-tetrahedron Kuhn cube and it.
struct hhg_mesh_s {
  hhg_ctx ctx = nullptr;
  int mr = 0;
  unsigned nf = 0;   // outflow faces (hhg_mesh_set_outflow)
  bool general = false;  // not a Kuhn partition of the cube: unstructured path
  std::vector<std::array<int, 3>> outflow;  // unstructured path: outflow boundary faces (sorted vertex triples)
  std::vector<double> xyz;
  std::vector<int> tet;
};

struct hhg_hier_s {
  hhg_ctx ctx = nullptr;
  int disc = 0, mr = 0, lmin = 0, lmax = 0, schur = 0;
  int nf = 0;        // outflow faces of the domain (Geom::nf)
  int G = 1;
  hhg::Arena arena;
  std::vector<hhg::Level> levels;
  // unstructured macro mesh: level tables of the per-cell path (null on the lattice path)
  std::unique_ptr<hhg::UHier> um;
  double* Kp = nullptr;
  int* unk = nullptr;
  int nunk = 0, rank = 0;
  std::vector<int> unk_host;
  double* partial = nullptr;
  double* sums = nullptr;   // device scratch for reductions (16 doubles)
  double* hsums = nullptr;  // pinned host copy
  // learned coarse solve (optional)
  hhg_mlp mlp = nullptr;
  double rho_plain = 0.0, tau = 0.0;
  bool mlp_off = false;      // fallback taken in the current solve
  bool kp_stale = false;     // coarse pseudo-inverse not rebuilt for the current viscosity
  bool kp_ready = false;     // coarse pseudo-inverse computed (lazily, ensure_coarse)
  float *feat = nullptr, *mlp_out = nullptr;
  double* norm = nullptr;
  double* bk = nullptr;      // copy of x before a monitored V-cycle
  // training-pair recorder of exact coarse solves (hhg_record_pairs)
  float *rec_f = nullptr, *rec_t = nullptr;
  int rec_cap = 0, rec_n = 0;
  double* rc = nullptr;      // coarse correction of a recorded solve
  double *ce = nullptr, *cy = nullptr;  // coarse-operator assembly scratch
  // one-workgroup V-cycle over the small levels: level descriptors on the
  // device (rebuilt when stale), levels with at most fused_sites velocity
  // sites per component are cycled that way (0: never)
  hhg::SmallLevel<double>* slv64 = nullptr;
  hhg::SmallLevel<float>* slv32 = nullptr;
  bool slv_stale = true;
  long fused_sites = 800;
  // unstructured meshes: levels with at most ufused_slots slots (cells times
  // points per cell) run each smoothing call in one workgroup (0: never)
  long ufused_slots = kUFusedSlots;
  std::vector<int> lds_end64, lds_end32;  // LDS words of levels lmin..l (0: level not in LDS)
  // levels lmin .. lmin + bf16_levels - 1 hold bfloat16 values in their
  // float32 vectors (hhg_hier_set_bf16_levels)
  int bf16_levels = 0;
  // cached HIP graph of a fixed-work FMG solve (key: vectors + parameters)
  hipGraphExec_t fmg_exec = nullptr;
  std::vector<unsigned char> fmg_key;
  // events bracketing a call that reports statistics (hhg_stats.seconds)
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  hhg::Level& L(int l) { return levels[l - lmin]; }
};

namespace hhg {
namespace {

hipStream_t S(hhg_hier h) { return h->ctx->stream; }

template <typename T>
const Tables<T>* tables(Level& lv);
template <>
const Tables<double>* tables<double>(Level& lv) {
  return lv.tb64;
}
template <>
const Tables<float>* tables<float>(Level& lv) {
  return lv.tb32;
}
template <typename T>
const TransferTables<T>* ttables(Level& lv);
template <>
const TransferTables<double>* ttables<double>(Level& lv) {
  return lv.tt64;
}
template <>
const TransferTables<float>* ttables<float>(Level& lv) {
  return lv.tt32;
}
template <typename T>
const LevelConst<T>& lconst(Level& lv);
template <>
const LevelConst<double>& lconst<double>(Level& lv) {
  return lv.lc64;
}
template <>
const LevelConst<float>& lconst<float>(Level& lv) {
  return lv.lc32;
}
template <typename T>
const NeuTables<T>* neutab(Level& lv);
template <>
const NeuTables<double>* neutab<double>(Level& lv) {
  return lv.neu64;
}
template <>
const NeuTables<float>* neutab<float>(Level& lv) {
  return lv.neu32;
}
template <typename T>
const T* dinv(Level& lv);
template <>
const double* dinv<double>(Level& lv) {
  return lv.dinv64;
}
template <>
const float* dinv<float>(Level& lv) {
  return lv.dinv32;
}

// --------------------------------------------------------- table building
void build_level_tables(hhg_hier h, Level& lv, const ElementSet& es) {
  const Geom& g = lv.g;
  const int G = g.G, n1 = g.n1, nn = g.nn;
  const double hh = lv.h;
  const double sA = hh, sB = hh * hh, sM = hh * hh * hh;
  const double sC = (h->disc == HHG_P1P1) ? (1.0 / 12.0) * std::pow(1.0 / 6.0, 2.0 / 3.0) * hh * hh * hh : 0.0;
  lv.lc64.a = sA, lv.lc64.b = sB, lv.lc64.c = sC, lv.lc64.m = sM;
  lv.lc32.a = (float)sA, lv.lc32.b = (float)sB, lv.lc32.c = (float)sC, lv.lc32.m = (float)sM;
  auto prune = [](Row r, int nw) {
    double mx = 0.0;
    for (auto& e : r)
      for (int d = 0; d < nw; ++d) mx = std::max(mx, std::fabs(e.w[d]));
    Row out;
    for (auto& e : r) {
      bool keep = false;
      for (int d = 0; d < nw; ++d) keep |= std::fabs(e.w[d]) > 1e-13 * mx;
      if (keep) out.push_back(e);
    }
    return out;
  };
  Tables<double> t64{};
  Tables<float> t32{};
  Arena& a = h->arena;
  const int rep[3] = {0, 2, 4};
  lv.hA.assign(G, {});
  lv.hBT.assign(G, {});
  lv.hB.assign(27, {});
  lv.hC.assign(27, {});
  for (int gr = 0; gr < G; ++gr) {
    const int c = 3;
    HostStencil A, BT, Mv;
    for (auto& e : prune(row_stencil(es, 'A', gr, c, c, c, 7), 1)) {
      A.off.push_back((e.g - gr) * nn + lin(e.di, e.dj, e.dk, n1));
      A.w.push_back(e.w[0] * sA);
      if (e.g == gr && e.di == 0 && e.dj == 0 && e.dk == 0) lv.adiag[gr] = e.w[0] * sA;
    }
    for (auto& e : prune(row_stencil(es, 'T', gr, c, c, c, 7), 3)) {
      BT.off.push_back(lin(e.di, e.dj, e.dk, n1));
      for (int d = 0; d < 3; ++d) BT.w.push_back(e.w[d] * sB);
    }
    for (auto& e : prune(row_stencil(es, 'M', gr, c, c, c, 7), 1)) {
      Mv.off.push_back((e.g - gr) * nn + lin(e.di, e.dj, e.dk, n1));
      Mv.w.push_back(e.w[0] * sM);
    }
    HHG_REQUIRE(lv.adiag[gr] > 0.0, HHG_ERR_STATE, "stencil setup: missing diagonal");
    t64.A[gr] = upload_stencil<double>(a, A);
    t32.A[gr] = upload_stencil<float>(a, A);
    t64.BT[gr] = upload_stencil<double>(a, BT);
    t32.BT[gr] = upload_stencil<float>(a, BT);
    t64.Mv[gr] = upload_stencil<double>(a, Mv);
    t32.Mv[gr] = upload_stencil<float>(a, Mv);
    t64.adiag_inv[gr] = 1.0 / lv.adiag[gr];
    t32.adiag_inv[gr] = (float)(1.0 / lv.adiag[gr]);
    lv.lc64.ainv[gr] = 1.0 / lv.adiag[gr];
    lv.lc32.ainv[gr] = (float)(1.0 / lv.adiag[gr]);
    lv.hA[gr] = A;
    lv.hBT[gr] = BT;
  }
  for (int cls = 0; cls < 27; ++cls) {
    const int ci = rep[cls % 3], cj = rep[(cls / 3) % 3], ck = rep[cls / 9];
    HostStencil B, C;
    for (auto& e : prune(row_stencil(es, 'B', 0, ci, cj, ck, 4), 3)) {
      B.off.push_back(e.g * nn + lin(e.di, e.dj, e.dk, n1));
      for (int d = 0; d < 3; ++d) B.w.push_back(e.w[d] * sB);
      B.code.push_back(e.g | ((e.di + 2) << 4) | ((e.dj + 2) << 8) | ((e.dk + 2) << 12));
    }
    if (h->disc == HHG_P1P1) {
      for (auto& e : prune(row_stencil(es, 'C', 0, ci, cj, ck, 4), 1)) {
        C.off.push_back(lin(e.di, e.dj, e.dk, n1));
        C.w.push_back(e.w[0] * sC);
      }
    }
    double m = 0.0;
    for (auto& e : row_stencil(es, 'P', 0, ci, cj, ck, 4)) m += e.w[0] * sM;
    t64.B[cls] = upload_stencil<double>(a, B);
    t32.B[cls] = upload_stencil<float>(a, B);
    t64.C[cls] = upload_stencil<double>(a, C);
    t32.C[cls] = upload_stencil<float>(a, C);
    const int* code = a.upload(B.code);
    t64.Bcode[cls] = code;
    t32.Bcode[cls] = code;
    t64.mclass[cls] = m;
    t32.mclass[cls] = (float)m;
    lv.hB[cls] = B;
    lv.hC[cls] = C;
  }
  // full mass rows: velocity groups x boundary classes, pressure classes
  for (int gr = 0; gr < G; ++gr)
    for (int cls = 0; cls < 27; ++cls) {
      const int cc[3] = {cls % 3, (cls / 3) % 3, cls / 9};
      const int dir[3] = {G == 1 ? 0 : kGroupDir[gr][0], G == 1 ? 0 : kGroupDir[gr][1], G == 1 ? 0 : kGroupDir[gr][2]};
      bool valid = true;
      for (int d = 0; d < 3; ++d) valid &= !(dir[d] && cc[d] != 1);
      HostStencil Mc;
      if (valid) {
        for (auto& e : prune(row_stencil(es, 'M', gr, rep[cc[0]], rep[cc[1]], rep[cc[2]], 4), 1)) {
          Mc.off.push_back((e.g - gr) * nn + lin(e.di, e.dj, e.dk, n1));
          Mc.w.push_back(e.w[0] * sM);
        }
      }
      t64.Mfull[gr * 27 + cls] = upload_stencil<double>(a, Mc);
      t32.Mfull[gr * 27 + cls] = upload_stencil<float>(a, Mc);
    }
  for (int cls = 0; cls < 27; ++cls) {
    HostStencil Pc;
    for (auto& e : prune(row_stencil(es, 'P', 0, rep[cls % 3], rep[(cls / 3) % 3], rep[cls / 9], 4), 1)) {
      Pc.off.push_back(lin(e.di, e.dj, e.dk, n1));
      Pc.w.push_back(e.w[0] * sM);
    }
    t64.Pm[cls] = upload_stencil<double>(a, Pc);
    t32.Pm[cls] = upload_stencil<float>(a, Pc);
  }
  lv.dinv64 = a.alloc<double>(nn);
  lv.dinv32 = a.alloc<float>(nn);
  t64.dinv = lv.dinv64;
  t32.dinv = lv.dinv32;
  lv.tb64 = a.alloc<Tables<double>>(1);
  lv.tb32 = a.alloc<Tables<float>>(1);
  HHG_CHECK_HIP(hipMemcpy(lv.tb64, &t64, sizeof(t64), hipMemcpyHostToDevice));
  HHG_CHECK_HIP(hipMemcpy(lv.tb32, &t32, sizeof(t32), hipMemcpyHostToDevice));
  // boundary pressure nodes, grouped by boundary class (lattice order inside
  // a class): each node's row is the generated row of its class, so a
  // wavefront of one class runs one branch instead of several
  std::vector<std::pair<int, int>> bcl;
  auto bc3 = [&](int c) { return c == 0 ? 0 : (c == g.N ? 2 : 1); };
  for (int k = 0; k < n1; ++k)
    for (int j = 0; j < n1; ++j)
      for (int i = 0; i < n1; ++i)
        if (i == 0 || j == 0 || k == 0 || i == g.N || j == g.N || k == g.N)
          bcl.push_back({bc3(i) + 3 * bc3(j) + 9 * bc3(k), lin(i, j, k, n1)});
  std::stable_sort(bcl.begin(), bcl.end(),
                   [](const std::pair<int, int>& a, const std::pair<int, int>& b) { return a.first < b.first; });
  std::vector<int> bnd;
  for (auto& e : bcl) bnd.push_back(e.second);
  lv.nbnd = (int)bnd.size();
  lv.bnd = a.upload(bnd);
}

// Outflow faces: the site lists of every level (sites on Neumann faces off the
// closed Dirichlet part, ordered by Gauss-Seidel colour), their boundary-class
// A and B^T rows, and for every coarse level the restriction rows of its
// sites (the interior restriction row -- transpose of the interpolation --
// without the fine sites outside the cube).
void build_neumann(hhg_hier h, const ElementSet& es) {
  const int G = h->G;
  const int rep[3] = {0, 2, 4};
  std::vector<std::vector<RestrictEntry>> rvel;
  std::vector<RestrictEntry> rpres;
  restriction_entries(G == 1 ? 1 : 2, rvel, rpres);
  for (int l = h->lmin; l <= h->lmax; ++l) {
    Level& lv = h->L(l);
    const Geom& g = lv.g;
    const int N = g.N, n1 = g.n1, nn = g.nn;
    const int M = G == 1 ? N : 2 * N;
    const int ncol = gs_colours(G);
    std::vector<std::vector<std::pair<int, int>>> bycol(ncol);  // (pos, slot)
    std::vector<char> used(kNeuSlots, 0);
    for (int gr = 0; gr < G; ++gr)
      for (int k = 0; k < n1; ++k)
        for (int j = 0; j < n1; ++j)
          for (int i = 0; i < n1; ++i) {
            const int dir[3] = {G == 1 ? 0 : kGroupDir[gr][0], G == 1 ? 0 : kGroupDir[gr][1],
                                G == 1 ? 0 : kGroupDir[gr][2]};
            const int c[3] = {i, j, k};
            int X[3], faces = 0, cls = 0, mul = 1;
            bool exists = true;
            for (int d = 0; d < 3; ++d) {
              X[d] = G == 1 ? c[d] : 2 * c[d] + dir[d];
              exists = exists && X[d] <= M;
              faces |= (X[d] == 0 ? 1 : 0) << (2 * d);
              faces |= (X[d] == M ? 1 : 0) << (2 * d + 1);
              cls += mul * (X[d] == 0 ? 0 : (X[d] == M ? 2 : 1));
              mul *= 3;
            }
            if (!exists || faces == 0 || (faces & ~h->nf)) continue;
            const int colour = gr == 0 ? (i + j + k) % kGsVertexColours : kGsVertexColours - 1 + gr;
            bycol[colour].push_back({gr * nn + lin(i, j, k, n1), gr * 27 + cls});
            used[gr * 27 + cls] = 1;
          }
    std::vector<int> pos, slot;
    lv.neu_coff.assign(1, 0);
    for (int c = 0; c < ncol; ++c) {
      for (auto& ps : bycol[c]) pos.push_back(ps.first), slot.push_back(ps.second);
      lv.neu_coff.push_back((int)pos.size());
    }
    lv.neu_n = (int)pos.size();
    lv.neu_pos = h->arena.upload(pos);
    lv.neu_slot = h->arena.upload(slot);
    const double sA = lv.h, sB = lv.h * lv.h;
    NeuTables<double> t64{};
    NeuTables<float> t32{};
    for (int sl = 0; sl < kNeuSlots; ++sl) {
      if (!used[sl]) continue;
      const int gr = sl / 27, cls = sl % 27;
      const int ci = rep[cls % 3], cj = rep[(cls / 3) % 3], ck = rep[cls / 9];
      HostStencil A, BT;
      double diag = 0.0;
      // entries that vanish mathematically (vertex pairs off the lattice
      // axes) carry rounding residue of the element sums: dropped, as in the
      // generated interior rows, so no Gauss-Seidel colour reads its own sites
      const auto arow = row_stencil(es, 'A', gr, ci, cj, ck, 4);
      double amax = 0.0;
      for (auto& e : arow) amax = std::max(amax, std::fabs(e.w[0]));
      for (auto& e : arow) {
        if (std::fabs(e.w[0]) <= 1e-13 * amax) continue;
        A.off.push_back((e.g - gr) * nn + lin(e.di, e.dj, e.dk, n1));
        A.w.push_back(e.w[0] * sA);
        if (e.g == gr && e.di == 0 && e.dj == 0 && e.dk == 0) diag = e.w[0] * sA;
      }
      for (auto& e : row_stencil(es, 'T', gr, ci, cj, ck, 4)) {
        if (e.w[0] == 0.0 && e.w[1] == 0.0 && e.w[2] == 0.0) continue;
        BT.off.push_back(lin(e.di, e.dj, e.dk, n1));
        for (int d = 0; d < 3; ++d) BT.w.push_back(e.w[d] * sB);
      }
      HHG_REQUIRE(diag > 0.0, HHG_ERR_STATE, "outflow setup: missing diagonal");
      t64.A[sl] = upload_stencil<double>(h->arena, A);
      t32.A[sl] = upload_stencil<float>(h->arena, A);
      t64.BT[sl] = upload_stencil<double>(h->arena, BT);
      t32.BT[sl] = upload_stencil<float>(h->arena, BT);
      t64.adiag_inv[sl] = 1.0 / diag;
      t32.adiag_inv[sl] = (float)(1.0 / diag);
      if (l < h->lmax) {  // restriction rows from level l + 1 to these sites
        const Level& fl = h->L(l + 1);
        const int n1f = fl.g.n1, nnf = fl.g.nn;
        const int cc[3] = {cls % 3, (cls / 3) % 3, cls / 9};
        HostStencil R;
        for (const auto& e : rvel[gr]) {
          const int fo[3] = {e.di, e.dj, e.dk};
          bool inside = true;
          for (int d = 0; d < 3; ++d) {
            // fine position relative to the coarse site, in fine site units
            const int delta = G == 1 ? fo[d] : 2 * fo[d] + kGroupDir[e.g][d] - 2 * kGroupDir[gr][d];
            if (cc[d] == 0 && delta < 0) inside = false;
            if (cc[d] == 2 && delta > 0) inside = false;
          }
          if (!inside || e.w == 0.0) continue;
          R.off.push_back(e.g * nnf + lin(e.di, e.dj, e.dk, n1f));
          R.w.push_back(e.w);
        }
        t64.R[sl] = upload_stencil<double>(h->arena, R);
        t32.R[sl] = upload_stencil<float>(h->arena, R);
      }
    }
    lv.neu64 = h->arena.alloc<NeuTables<double>>(1);
    lv.neu32 = h->arena.alloc<NeuTables<float>>(1);
    HHG_CHECK_HIP(hipMemcpy(lv.neu64, &t64, sizeof(t64), hipMemcpyHostToDevice));
    HHG_CHECK_HIP(hipMemcpy(lv.neu32, &t32, sizeof(t32), hipMemcpyHostToDevice));
  }
}


void build_transfer(hhg_hier h, Level& lc, Level& lf) {
  Arena& a = h->arena;
  const int G = lf.g.G;
  const int n1c = lc.g.n1, nnc = lc.g.nn;
  // velocity prolongation classes
  const int vorder = G == 1 ? 1 : 2;
  const int vq = vorder == 1 ? 2 : 4;  // fine positions per coarse cube edge
  const int ncls = vq * vq * vq;
  std::vector<int> vp_off(ncls * 10, 0);
  std::vector<double> vp_w(ncls * 10, 0.0);
  for (int cz = 0; cz < vq; ++cz)
    for (int cy = 0; cy < vq; ++cy)
      for (int cx = 0; cx < vq; ++cx) {
        const int cls = cx + vq * (cy + vq * cz);
        const double t[3] = {(double)cx / vq, (double)cy / vq, (double)cz / vq};
        auto ws = interp_weights(vorder, t);
        HHG_REQUIRE(ws.size() <= 10, HHG_ERR_STATE, "transfer setup: too many weights");
        int e = 0;
        for (auto& w : ws) {
          const int gc = std::get<0>(w), oi = std::get<1>(w), oj = std::get<2>(w), ok = std::get<3>(w);
          vp_off[cls * 10 + e] = gc * nnc + lin(oi, oj, ok, n1c);
          vp_w[cls * 10 + e] = std::get<4>(w);
          ++e;
        }
      }
  // pressure (linear) prolongation classes
  std::vector<int> pp_off(80, 0);
  std::vector<double> pp_w(80, 0.0);
  for (int cz = 0; cz < 2; ++cz)
    for (int cy = 0; cy < 2; ++cy)
      for (int cx = 0; cx < 2; ++cx) {
        const int cls = cx + 2 * (cy + 2 * cz);
        const double t[3] = {cx / 2.0, cy / 2.0, cz / 2.0};
        auto ws = interp_weights(1, t);
        int e = 0;
        for (auto& w : ws) {
          const int oi = std::get<1>(w), oj = std::get<2>(w), ok = std::get<3>(w);
          pp_off[cls * 10 + e] = lin(oi, oj, ok, n1c);
          pp_w[cls * 10 + e] = std::get<4>(w);
          ++e;
        }
      }
  auto mk = [&](auto& tt, auto tag) {
    using T = decltype(tag);
    std::vector<T> vw(vp_w.begin(), vp_w.end()), pw(pp_w.begin(), pp_w.end());
    tt.vp_off = a.upload(vp_off);
    tt.vp_w = a.upload(vw);
    tt.pp_off = a.upload(pp_off);
    tt.pp_w = a.upload(pw);
  };
  TransferTables<double> t64{};
  TransferTables<float> t32{};
  mk(t64, double());
  mk(t32, float());
  lf.tt64 = a.alloc<TransferTables<double>>(1);
  lf.tt32 = a.alloc<TransferTables<float>>(1);
  HHG_CHECK_HIP(hipMemcpy(lf.tt64, &t64, sizeof(t64), hipMemcpyHostToDevice));
  HHG_CHECK_HIP(hipMemcpy(lf.tt32, &t32, sizeof(t32), hipMemcpyHostToDevice));
}

int full_mask(hhg_hier h);

// Coarse unknowns (interior velocity DoFs, all pressure DoFs) of the
// coarsest level and the device buffer of the pseudo-inverse; the
// pseudo-inverse itself is computed on first use (ensure_coarse), so a
// hierarchy that never solves on its coarsest level (an error-evaluation
// pair of levels, say) does not pay for the host decomposition.
void build_coarse(hhg_hier h) {
  Level& lv = h->L(h->lmin);
  const Geom& g = lv.g;
  const int N = g.N, n1 = g.n1, nn = g.nn, G = g.G;
  std::vector<int> unk;
  std::unordered_map<int, int> pos2u;
  // velocity unknowns: sites that exist and lie on no Dirichlet face
  auto vint = [&](int gr, int i, int j, int k) {
    const int dir[3] = {G == 1 ? 0 : kGroupDir[gr][0], G == 1 ? 0 : kGroupDir[gr][1], G == 1 ? 0 : kGroupDir[gr][2]};
    const int c[3] = {i, j, k}, M = G == 1 ? N : 2 * N;
    int faces = 0;
    for (int d = 0; d < 3; ++d) {
      const int X = G == 1 ? c[d] : 2 * c[d] + dir[d];
      if (X > M) return false;
      faces |= (X == 0 ? 1 : 0) << (2 * d);
      faces |= (X == M ? 1 : 0) << (2 * d + 1);
    }
    return (faces & ~h->nf) == 0;
  };
  for (int d = 0; d < 3; ++d)
    for (int gr = 0; gr < G; ++gr)
      for (int k = 0; k < n1; ++k)
        for (int j = 0; j < n1; ++j)
          for (int i = 0; i < n1; ++i)
            if (vint(gr, i, j, k)) {
              const int p = d * g.vstride + gr * nn + lin(i, j, k, n1);
              pos2u[p] = (int)unk.size();
              unk.push_back(p);
            }
  for (int k = 0; k < n1; ++k)
    for (int j = 0; j < n1; ++j)
      for (int i = 0; i < n1; ++i) {
        const int p = 3 * g.vstride + lin(i, j, k, n1);
        pos2u[p] = (int)unk.size();
        unk.push_back(p);
      }
  const int n = (int)unk.size();
  if (n > 2048) {  // no dense coarse solve: the hierarchy still applies operators and transfers
    h->nunk = 0;
    return;
  }
  h->nunk = n;
  h->Kp = h->arena.alloc<double>((size_t)n * n);
  h->unk = h->arena.upload(unk);
  h->unk_host = unk;
  h->kp_ready = false;
}

// Dense coarse operator on the unknowns from the host stencil tables
// (constant coefficients), and its pseudo-inverse into h->Kp.
void build_coarse_pinv(hhg_hier h) {
  Level& lv = h->L(h->lmin);
  const Geom& g = lv.g;
  const int N = g.N, n1 = g.n1, nn = g.nn;
  const int n = h->nunk;
  const std::vector<int>& unk = h->unk_host;
  std::unordered_map<int, int> pos2u;
  for (int r = 0; r < n; ++r) pos2u[unk[r]] = r;
  std::vector<double> K((size_t)n * n, 0.0);
  auto add = [&](int r, int pos, double w) {
    auto it = pos2u.find(pos);
    if (it != pos2u.end()) K[(size_t)r * n + it->second] += w;
  };
  for (int r = 0; r < n; ++r) {
    const int p = unk[r];
    if (p < 3 * g.vstride) {
      const int d = p / g.vstride, rem = p % g.vstride, gr = rem / nn, idx = rem % nn;
      const HostStencil& A = lv.hA[gr];
      for (size_t e = 0; e < A.off.size(); ++e) add(r, p + A.off[e], A.w[e]);
      const HostStencil& BT = lv.hBT[gr];
      for (size_t e = 0; e < BT.off.size(); ++e) add(r, 3 * g.vstride + idx + BT.off[e], BT.w[3 * e + d]);
    } else {
      const int idx = p - 3 * g.vstride;
      const int i = idx % n1, j = (idx / n1) % n1, k = idx / (n1 * n1);
      const int cls = bclass(i, j, k, N);
      const HostStencil& B = lv.hB[cls];
      for (size_t e = 0; e < B.off.size(); ++e)
        for (int d = 0; d < 3; ++d) add(r, d * g.vstride + idx + B.off[e], B.w[3 * e + d]);
      const HostStencil& C = lv.hC[cls];
      for (size_t e = 0; e < C.off.size(); ++e) add(r, p + C.off[e], -C.w[e]);
    }
  }
  for (int r = 0; r < n; ++r)
    for (int c = r + 1; c < n; ++c) {
      const double s = 0.5 * (K[(size_t)r * n + c] + K[(size_t)c * n + r]);
      K[(size_t)r * n + c] = K[(size_t)c * n + r] = s;
    }
  std::vector<double> Kp;
  h->rank = sym_pinv(n, K, Kp, 1e-12);
  HHG_CHECK_HIP(hipMemcpy(h->Kp, Kp.data(), Kp.size() * sizeof(double), hipMemcpyHostToDevice));
  h->kp_ready = true;
}

void build_coarse_device(hhg_hier h);

// The coarse pseudo-inverse of the current operator, computed now if it has
// not been (host work: call outside graph capture).
void ensure_coarse(hhg_hier h) {
  if (h->nunk == 0) return;
  if (!h->kp_ready && h->um) {
    HHG_CHECK_HIP(hipStreamSynchronize(S(h)));
    std::vector<int> unk;
    std::vector<double> K, Kp;
    u_coarse_system(*h->um, unk, K, 2048);
    const int n = h->nunk;
    for (int r = 0; r < n; ++r)
      for (int c = r + 1; c < n; ++c) {
        const double sym = 0.5 * (K[(size_t)r * n + c] + K[(size_t)c * n + r]);
        K[(size_t)r * n + c] = K[(size_t)c * n + r] = sym;
      }
    h->rank = sym_pinv(n, K, Kp, 1e-12);
    HHG_CHECK_HIP(hipMemcpy(h->Kp, Kp.data(), Kp.size() * sizeof(double), hipMemcpyHostToDevice));
    h->kp_ready = true;
    return;
  }
  if (!h->kp_ready) {
    HHG_CHECK_HIP(hipStreamSynchronize(S(h)));
    if (h->L(h->lmin).nu64 || h->nf)  // rows the host tables do not hold: from the device operator
      build_coarse_device(h);
    else
      build_coarse_pinv(h);
  }
}

template <typename T>
void op_apply(hhg_hier h, int l, int opmask, const T* x, const T* b, T* y, bool has_b, bool vel, bool prs);

// ------------------------------------------------ unstructured-mesh ops
// The per-cell path of an unstructured T_0 (umesh.h), float64 only.
template <typename T>
void u_f64() {
  if (!std::is_same<T, double>::value) throw Error{HHG_ERR_PREC, "unstructured macro meshes: float64 only"};
}
ULevelData& UL(hhg_hier h, int l) { return h->um->L(l); }
void u_colour(hhg_hier h, int l, int c, double* x, const double* b) {
  ULevelData& U = UL(h, l);
  const int K = U.ncol_if;
  if (c < K)
    launch_u_gs_iface(S(h), U.L, U.lst, U.col_off[c], U.col_off[c + 1] - U.col_off[c], U.col_maxocc[c], x, b);
  else
    launch_u_gs_inner(S(h), U.L, U.colour[c - K], x, b);
}
void u_smooth(hhg_hier h, int l, double* x, const double* b, int iters, int gs, int xi, double omega) {
  ULevelData& U = UL(h, l);
  const int ncol = U.ncol_if + 4;
  double* r = h->L(l).r;
  if ((long)U.L.ncell * U.L.P <= h->ufused_slots &&
      launch_u_smooth_small(S(h), U, x, b, r, iters, xi, gs == HHG_GS_SYM, omega))
    return;
  for (int it = 0; it < iters; ++it) {
    for (int s = 0; s < xi; ++s) {
      for (int c = 0; c < ncol; ++c) u_colour(h, l, c, x, b);
      if (gs == HHG_GS_SYM)
        for (int c = ncol - 1; c >= 0; --c) u_colour(h, l, c, x, b);
    }
    // r_p = g - B u + C p, then p -= omega D^{-1} r_p
    launch_u_apply_rows(S(h), U.L, U.inner, U.zitems, U.lst, x, b, r, 12, true, false, false, true);
    launch_u_pstep(S(h), U.L, U.dinv, x, r, omega);
  }
}
// p -= (m^T p / m^T 1), m the lumped mass, over the nodes (owner slots)
void u_mean_zero(hhg_hier h, int l, double* x) {
  ULevelData& U = UL(h, l);
  launch_u_dot(S(h), U.L, U.flags, U.ml_own, x, nullptr, 3, 1, h->partial, h->sums, 0);
  launch_u_shift(S(h), U.L, x + 3 * U.L.vs, h->sums, 0, U.ml_total);
}
void u_norms_launch(hhg_hier h, int l, const double* x, const double* y) {
  ULevelData& U = UL(h, l);
  launch_u_dot(S(h), U.L, U.flags, nullptr, x, y, 0, 3, h->partial, h->sums, 0);
  launch_u_dot(S(h), U.L, U.flags, nullptr, x, y, 3, 1, h->partial + 2 * kPartials, h->sums, 2);
}
// Boundary copies of Alg. fmg (Dirichlet velocity values) on either path.
void op_copy_boundary(hhg_hier h, int l, const double* src, double* dst) {
  if (h->um)
    launch_u_copy_bnd(S(h), UL(h, l).L, UL(h, l).flags, src, dst);
  else
    launch_copy_boundary<double>(S(h), h->L(l).g, src, dst);
}
void op_inject(hhg_hier h, int lf, const double* xf, double* xc) {
  if (h->um)
    launch_u_inject(S(h), UL(h, lf).L, UL(h, lf - 1).L, UL(h, lf - 1).all, xf, xc);
  else
    launch_inject_boundary<double>(S(h), h->L(lf).g, h->L(lf - 1).g, xf, xc);
}

// Dense coarse operator from the device operator itself (columns = calA e_c
// restricted to the unknowns, all n columns applied back to back), used when
// the coarsest level's rows depend on data such as a variable viscosity; then
// its pseudo-inverse replaces Kp.  When the first (eigenvalue) pseudo-inverse
// found exactly one null vector, that vector is the constant pressure (Sec. 2:
// the pressure is fixed only up to a constant) and the rebuild uses
// K^+ = (K + z z^T)^{-1} - z z^T instead of a new eigen-decomposition.
void build_coarse_device(hhg_hier h) {
  if (h->nunk == 0) return;
  Level& lv = h->L(h->lmin);
  const int n = h->nunk;
  const size_t vw = lv.vec_words;
  if (!h->ce) {  // private vectors: callers may hold the coarse work vectors
    h->ce = h->arena.alloc<double>((size_t)n * vw);
    h->cy = h->arena.alloc<double>((size_t)n * vw);
  }
  launch_fill<double>(S(h), h->ce, (size_t)n * vw, 0.0);
  launch_unit_columns(S(h), h->ce, vw, h->unk, n);
  for (int c = 0; c < n; ++c)
    op_apply<double>(h, h->lmin, full_mask(h), h->ce + c * vw, nullptr, h->cy + c * vw, false, true, true);
  std::vector<double> cols((size_t)n * vw), K((size_t)n * n);
  HHG_CHECK_HIP(hipMemcpyAsync(cols.data(), h->cy, cols.size() * sizeof(double), hipMemcpyDeviceToHost, S(h)));
  HHG_CHECK_HIP(hipStreamSynchronize(S(h)));
  for (int c = 0; c < n; ++c)
    for (int r = 0; r < n; ++r) K[(size_t)r * n + c] = cols[c * vw + h->unk_host[r]];
  for (int r = 0; r < n; ++r)
    for (int c = r + 1; c < n; ++c) {
      const double sym = 0.5 * (K[(size_t)r * n + c] + K[(size_t)c * n + r]);
      K[(size_t)r * n + c] = K[(size_t)c * n + r] = sym;
    }
  std::vector<double> Kp;
  bool done = false;
  if (h->kp_ready && h->rank == n - 1) {
    const size_t pbase = 3 * (size_t)lv.g.vstride;
    int np = 0;
    for (int r = 0; r < n; ++r) np += (size_t)h->unk_host[r] >= pbase;
    std::vector<double> z(n, 0.0);
    for (int r = 0; r < n; ++r)
      if ((size_t)h->unk_host[r] >= pbase) z[r] = 1.0 / std::sqrt((double)np);
    done = sym_pinv_null1(n, K, z, Kp);
  }
  if (!done) h->rank = sym_pinv(n, K, Kp, 1e-12);
  HHG_CHECK_HIP(hipMemcpy(h->Kp, Kp.data(), Kp.size() * sizeof(double), hipMemcpyHostToDevice));
  h->kp_ready = true;
}

// ---------------------------------------------------------------- ops
// Levels that hold bfloat16 values: a float32 operation writing a vector of
// such a level rounds the words it wrote, v[s stride + off + t] for s < nseg,
// t < n, to the nearest bfloat16 right after the kernel that wrote them --
// within one kernel no site reads another site's output, so this gives the
// values of bfloat16 storage with float32 arithmetic.
template <typename T>
void round_out(hhg_hier h, int l, T* v, size_t stride, size_t off, size_t n, int nseg) {
  if constexpr (std::is_same<T, float>::value) {
    if (l - h->lmin < h->bf16_levels) launch_round_bf16(S(h), v, stride, off, n, nseg);
  } else {
    (void)h, (void)l, (void)v, (void)stride, (void)off, (void)n, (void)nseg;
  }
}

template <typename T>
void op_apply(hhg_hier h, int l, int opmask, const T* x, const T* b, T* y, bool has_b, bool vel, bool prs) {
  if (h->um) {
    u_f64<T>();
    ULevelData& U = UL(h, l);
    launch_u_apply_rows(S(h), U.L, U.inner, U.zitems, U.lst, (const double*)x, (const double*)b, (double*)y, opmask, has_b,
                        false, vel, prs);
    return;
  }
  Level& lv = h->L(l);
  launch_apply<T>(S(h), lv.g, lconst<T>(lv), tables<T>(lv), x, b, y, opmask, has_b, vel, prs, lv.bnd, lv.nbnd);
  if (vel && lv.neu_n)  // outflow-face velocity rows (boundary rows to the grid-wide kernels)
    launch_neu_rows<T>(S(h), lv.g, neutab<T>(lv), lv.neu(), 0, lv.neu_n, x, b, y, opmask & 3, has_b);
  round_out<T>(h, l, y, 0, 0, lv.vec_words, 1);
}

int full_mask(hhg_hier h) { return h->disc == HHG_P1P1 ? 15 : 7; }

template <typename T>
T* rbuf(Level& lv);
template <>
double* rbuf<double>(Level& lv) {
  return lv.r;
}
template <>
float* rbuf<float>(Level& lv) {
  return lv.r32;
}

template <typename T>
void op_smooth(hhg_hier h, int l, T* x, const T* b, int iters, int gs, int xi, double omega) {
  if (h->um) {
    u_f64<T>();
    u_smooth(h, l, (double*)x, (const double*)b, iters, gs, xi, omega);
    return;
  }
  Level& lv = h->L(l);
  const int ncol = gs_colours(h->G);
  T* r = rbuf<T>(lv);
  auto colour = [&](int c) {  // a vertex colour writes the vertex group, the others edge group c - 1
    launch_gs_colour<T>(S(h), lv.g, lconst<T>(lv), x, b, c);
    if (lv.neu_n)
      launch_neu_gs<T>(S(h), lv.g, neutab<T>(lv), lv.neu(), lv.neu_coff[c], lv.neu_coff[c + 1] - lv.neu_coff[c], x, b);
    round_out<T>(h, l, x, lv.g.vstride, c < kGsVertexColours ? 0 : (size_t)(c - kGsVertexColours + 1) * lv.g.nn,
                 lv.g.nn, 3);
  };
  for (int it = 0; it < iters; ++it) {
    for (int s = 0; s < xi; ++s) {
      for (int c = 0; c < ncol; ++c) colour(c);
      if (gs == HHG_GS_SYM)
        for (int c = ncol - 1; c >= 0; --c) colour(c);
    }
    // r_p = g - B u + C p, then p -= omega D^{-1} r_p.  With constant
    // coefficients the k-marching apply in its pressure-rows-only form (a
    // few loads per lattice point, no velocity rows written).  Taylor-Hood
    // pressure rows read no p (C = 0): the step is applied in place by the
    // residual launch itself (no residual stored, one launch less per
    // iteration), except where the residual is rounded to bfloat16 first.
    const bool bf16_level = std::is_same<T, float>::value && l - h->lmin < h->bf16_levels;
    if (!lv.nu64 && h->disc == HHG_P2P1 && !bf16_level) {
      PStep<T> ps;
      ps.p = x + 3 * (size_t)lv.g.vstride;
      ps.dinv = dinv<T>(lv);
      ps.omega = (T)omega;
      launch_apply<T>(S(h), lv.g, lconst<T>(lv), tables<T>(lv), x, b, r, full_mask(h), true, false, true, lv.bnd,
                      lv.nbnd, ps);
    } else {
      if (!lv.nu64)
        op_apply<T>(h, l, full_mask(h), x, b, r, true, false, true);
      else
        op_apply<T>(h, l, full_mask(h) & 12, x, b, r, true, false, true);
      launch_pressure_step<T>(S(h), lv.g, dinv<T>(lv), x, r, (T)omega);
    }
    round_out<T>(h, l, x, 0, 3 * (size_t)lv.g.vstride, lv.g.nn, 1);
  }
}

// Zero pressure mean (int p = 0, Sec. 2), the normalisation of the pressure
// inside the solvers; with an outflow face the pressure is determined and
// nothing is done.  hhg_project_mean_zero always projects (op_mean_zero_always).
template <typename T>
void op_mean_zero_always(hhg_hier h, int l, T* x) {
  if (h->um) {
    u_f64<T>();
    u_mean_zero(h, l, (double*)x);
    return;
  }
  Level& lv = h->L(l);
  T* p = x + 3 * (size_t)lv.g.vstride;
  launch_mean_zero<T>(S(h), lv.g, tables<T>(lv), p, h->partial, h->sums, 0);
  round_out<T>(h, l, p, 0, 0, lv.g.nn, 1);
}
template <typename T>
void op_mean_zero(hhg_hier h, int l, T* x) {
  if (h->nf) return;
  if (h->um) {
    u_f64<T>();
    u_mean_zero(h, l, (double*)x);
    return;
  }
  Level& lv = h->L(l);
  T* p = x + 3 * (size_t)lv.g.vstride;
  launch_mean_zero<T>(S(h), lv.g, tables<T>(lv), p, h->partial, h->sums, 0);
  round_out<T>(h, l, p, 0, 0, lv.g.nn, 1);
}

template <typename T>
void op_restrict(hhg_hier h, int lf, const T* rf, T* rc, T* zero_x = nullptr) {
  if (h->um) {
    if (zero_x) launch_fill<T>(S(h), zero_x, h->L(lf - 1).vec_words, T(0));
    u_f64<T>();
    ULevelData& F = UL(h, lf);
    ULevelData& C = UL(h, lf - 1);
    launch_u_restrict(S(h), F.L, C.L, C.inner, C.lst, (const double*)rf, (double*)rc);
    if (h->nf) return;  // outflow faces: no null vector, no compatibility shift
    // compatibility with the null vector (0, 1): plain mean of the pressure nodes
    launch_u_dot(S(h), C.L, C.flags, nullptr, (const double*)rc, nullptr, 3, 1, h->partial, h->sums, 0);
    launch_u_shift(S(h), C.L, (double*)rc + 3 * C.L.vs, h->sums, 0, (double)C.nnodes);
    return;
  }
  Level& f = h->L(lf);
  Level& c = h->L(lf - 1);
  launch_restrict<T>(S(h), f.g, c.g, ttables<T>(f), rf, rc, zero_x);
  if (c.neu_n) launch_neu_restrict<T>(S(h), f.g, c.g, neutab<T>(c), c.neu(), c.neu_n, rf, rc);
  round_out<T>(h, lf - 1, rc, 0, 0, c.vec_words, 1);
  if (h->nf) return;  // no null vector: no compatibility shift
  T* p = rc + 3 * (size_t)c.g.vstride;
  launch_mean_zero<T>(S(h), c.g, tables<T>(c), p, h->partial, h->sums, 1);
  round_out<T>(h, lf - 1, p, 0, 0, c.g.nn, 1);
}

template <typename T>
void op_prolong(hhg_hier h, int lc, const T* xc, T* xf, bool add, bool skip_bnd) {
  if (h->um) {
    u_f64<T>();
    launch_u_prolong(S(h), UL(h, lc).L, UL(h, lc + 1).L, UL(h, lc + 1).all, (const double*)xc, (double*)xf, add,
                     skip_bnd);
    return;
  }
  Level& c = h->L(lc);
  Level& f = h->L(lc + 1);
  launch_prolong<T>(S(h), c.g, f.g, ttables<T>(f), xc, xf, add, skip_bnd);
  if (add && skip_bnd && f.neu_n)  // the outflow sites the grid-wide kernel skipped as boundary
    launch_neu_prolong<T>(S(h), c.g, f.g, ttables<T>(f), f.neu(), f.neu_n, xc, xf);
  round_out<T>(h, lc + 1, xf, 0, 0, f.vec_words, 1);
}

template <typename T>
T* cxbuf(Level& lv);
template <>
double* cxbuf<double>(Level& lv) {
  return lv.cx;
}
template <>
float* cxbuf<float>(Level& lv) {
  return lv.cx32;
}
template <typename T>
T* cbbuf(Level& lv);
template <>
double* cbbuf<double>(Level& lv) {
  return lv.cb;
}
template <>
float* cbbuf<float>(Level& lv) {
  return lv.cb32;
}

// Device descriptors of every level for the one-workgroup V-cycle (host
// copies uploaded with a synchronous copy: called outside graph capture).
template <typename T>
void fill_small(hhg_hier h, std::vector<SmallLevel<T>>& out, std::vector<int>& lds_end) {
  out.resize(h->levels.size());
  lds_end.assign(h->levels.size(), 0);
  size_t off = 0;
  bool fits = true;
  for (int l = h->lmin; l <= h->lmax; ++l) {
    Level& lv = h->L(l);
    SmallLevel<T>& s = out[l - h->lmin];
    s.g = lv.g;
    s.lc = lconst<T>(lv);
    s.tb = tables<T>(lv);
    s.tt = l > h->lmin ? ttables<T>(lv) : nullptr;
    s.dinv = dinv<T>(lv);
    s.bnd = lv.bnd;
    s.nbnd = lv.nbnd;
    s.r = rbuf<T>(lv);
    s.cx = cxbuf<T>(lv);
    s.cb = cbbuf<T>(lv);
    // LDS copies of [x | b | r] for the lowest levels, as long as they fit
    fits = fits && (off + 3 * lv.vec_words) * sizeof(T) <= (size_t)kSmallLdsBytes;
    s.lds_off = fits ? (int)off : -1;
    if (fits) {
      off += 3 * lv.vec_words;
      lds_end[l - h->lmin] = (int)off;
    }
  }
}
void refresh_small(hhg_hier h) {
  if (!h->slv_stale || h->um) return;  // no one-workgroup cycle on unstructured meshes
  if (!h->slv64) {
    h->slv64 = h->arena.alloc<SmallLevel<double>>(h->levels.size());
    h->slv32 = h->arena.alloc<SmallLevel<float>>(h->levels.size());
  }
  std::vector<SmallLevel<double>> a;
  std::vector<SmallLevel<float>> b;
  fill_small<double>(h, a, h->lds_end64);
  fill_small<float>(h, b, h->lds_end32);
  HHG_CHECK_HIP(hipMemcpy(h->slv64, a.data(), a.size() * sizeof(a[0]), hipMemcpyHostToDevice));
  HHG_CHECK_HIP(hipMemcpy(h->slv32, b.data(), b.size() * sizeof(b[0]), hipMemcpyHostToDevice));
  h->slv_stale = false;
}
template <typename T>
const SmallLevel<T>* slv(hhg_hier h);
template <>
const SmallLevel<double>* slv<double>(hhg_hier h) {
  return h->slv64;
}
template <>
const SmallLevel<float>* slv<float>(hhg_hier h) {
  return h->slv32;
}
long vel_sites(const Level& lv) {
  const long m = lv.g.G == 1 ? lv.g.N + 1 : 2 * (long)lv.g.N + 1;
  return m * m * m;
}

// Coarse solve x <- x + A0^+ (b - A0 x) on the unknowns (float64 GEMV for
// either storage precision), then zero pressure mean.
void build_coarse_device(hhg_hier h);

// Coarse solve x <- x + A0^+ (b - A0 x) on the unknowns (float64 GEMV for
// either storage precision), then zero pressure mean.  With an MLP attached
// (float64 solves), the correction is ||r|| net([r / ||r||, log nu]) instead,
// unless the fallback monitor has switched it off for this solve.  With
// p->coarse_smooth > 0 the coarsest level is only relaxed (that many Uzawa
// iterations), the comparison point without any coarse solve.  While the
// recorder is on, every exact float64 solve also stores its training pair.
template <typename T>
void op_coarse(hhg_hier h, T* x, const T* b, bool allow_mlp = true, const hhg_solver_params* p = nullptr) {
  Level& lv = h->L(h->lmin);
  if (p && p->coarse_smooth > 0) {
    op_smooth<T>(h, h->lmin, x, b, p->coarse_smooth, p->gs, p->xi, 1.0 / p->omega_inv);
    op_mean_zero<T>(h, h->lmin, x);
    return;
  }
  HHG_REQUIRE(h->nunk > 0, HHG_ERR_STATE, "coarsest level has more than 2048 unknowns: no dense coarse solve");
  T* r = rbuf<T>(lv);
  op_apply<T>(h, h->lmin, full_mask(h), x, b, r, true, true, true);
  if constexpr (std::is_same<T, double>::value) {
    if (allow_mlp && h->mlp && !h->mlp_off) {
      launch_coarse_features(S(h), r, h->unk, h->nunk, lv.nu64, lv.g.nn, h->feat, h->norm);
      h->mlp->net.forward(S(h), h->feat, 1, h->mlp_out);
      launch_coarse_scatter(S(h), h->mlp_out, h->unk, h->nunk, h->norm, x, nullptr);
      op_mean_zero<T>(h, h->lmin, x);
      return;
    }
  }
  if (h->kp_stale) {
    HHG_CHECK_HIP(hipStreamSynchronize(S(h)));
    build_coarse_device(h);
    h->kp_stale = false;
  }
  ensure_coarse(h);
  if constexpr (std::is_same<T, double>::value) {
    if (h->rec_n < h->rec_cap) {
      const size_t ni = (size_t)h->nunk + lv.g.nn;
      launch_coarse_features(S(h), r, h->unk, h->nunk, lv.nu64, lv.g.nn, h->rec_f + h->rec_n * ni, h->norm);
      launch_fill<double>(S(h), h->rc, lv.vec_words, 0.0);
      launch_coarse<double>(S(h), h->Kp, h->unk, h->nunk, r, h->rc);
      op_mean_zero<double>(h, h->lmin, h->rc);
      launch_coarse_scatter(S(h), nullptr, h->unk, h->nunk, h->norm, h->rc, h->rec_t + h->rec_n * (size_t)h->nunk);
      launch_axpy<double>(S(h), x, h->rc, lv.vec_words, 1.0);
      op_mean_zero<double>(h, h->lmin, x);
      ++h->rec_n;
      return;
    }
  }
  launch_coarse<T>(S(h), h->Kp, h->unk, h->nunk, r, x);
  if (h->um) launch_u_sync(S(h), UL(h, h->lmin).L, UL(h, h->lmin).lst, (double*)x);
  round_out<T>(h, h->lmin, x, 0, 0, lv.vec_words, 1);
  op_mean_zero<T>(h, h->lmin, x);
}

// Variable V-cycle of Alg. fmg in storage/arithmetic precision T.
template <typename T>
void vcycle_t(hhg_hier h, int lf, int l, T* x, const T* b, const hhg_solver_params& p) {
  if (l == h->lmin) {
    op_coarse<T>(h, x, b, true, &p);
    return;
  }
  // the whole cycle from a small level down in one workgroup (plain exact
  // coarse solve only: no network, recorder, relaxation-only mode or pending
  // pseudo-inverse rebuild)
  const bool mlp_on = std::is_same<T, double>::value && h->mlp && !h->mlp_off;
  if (vel_sites(h->L(l)) <= h->fused_sites && !h->slv_stale && p.coarse_smooth == 0 && h->nunk > 0 && !mlp_on &&
      h->rec_n >= h->rec_cap && !h->kp_stale && h->kp_ready && h->nf == 0 && !h->um &&
      (std::is_same<T, double>::value || h->L(h->lmin).cx32)) {
    SmallCycle<T> sc{};
    sc.nlev = l - h->lmin + 1;
    sc.G = h->G;
    sc.pre0 = p.nu_pre + (lf - l) * p.nu_inc;
    sc.post0 = p.nu_post + (lf - l) * p.nu_inc;
    sc.inc = p.nu_inc;
    sc.gs_sym = p.gs == HHG_GS_SYM;
    sc.xi = p.xi;
    sc.full_mask = full_mask(h);
    sc.omega = (T)(1.0 / p.omega_inv);
    sc.x = x;
    sc.b = b;
    sc.Kp = h->Kp;
    sc.unk = h->unk;
    sc.nunk = h->nunk;
    sc.lds_words = (std::is_same<T, double>::value ? h->lds_end64 : h->lds_end32)[l - h->lmin];
    sc.q16 = std::is_same<T, float>::value ? h->bf16_levels : 0;
    launch_vcycle_small<T>(S(h), slv<T>(h), sc);
    return;
  }
  Level& lv = h->L(l);
  Level& lc = h->L(l - 1);
  const double om = 1.0 / p.omega_inv;
  T* r = rbuf<T>(lv);
  op_smooth<T>(h, l, x, b, p.nu_pre + (lf - l) * p.nu_inc, p.gs, p.xi, om);
  op_apply<T>(h, l, full_mask(h), x, b, r, true, true, true);
  op_restrict<T>(h, l, r, cbbuf<T>(lc), cxbuf<T>(lc));  // and the coarse start value 0
  vcycle_t<T>(h, lf, l - 1, cxbuf<T>(lc), cbbuf<T>(lc), p);
  op_prolong<T>(h, l - 1, cxbuf<T>(lc), x, true, true);
  op_smooth<T>(h, l, x, b, p.nu_post + (lf - l) * p.nu_inc, p.gs, p.xi, om);
}

void vcycle(hhg_hier h, int lf, int l, double* x, const double* b, const hhg_solver_params& p) {
  vcycle_t<double>(h, lf, l, x, b, p);
}

void ensure_f32_vectors(hhg_hier h) {
  for (int l = h->lmin; l < h->lmax; ++l) {
    Level& lv = h->L(l);
    if (!lv.cx32) {
      h->slv_stale = true;
      lv.cx32 = h->arena.alloc<float>(lv.vec_words);
      lv.cb32 = h->arena.alloc<float>(lv.vec_words);
      launch_fill<float>(S(h), lv.cx32, lv.vec_words, 0.0f);
      launch_fill<float>(S(h), lv.cb32, lv.vec_words, 0.0f);
    }
  }
  Level& top = h->L(h->lmax);
  if (!top.cx32) {  // finest level: correction and right-hand side of the inner solve
    top.cx32 = h->arena.alloc<float>(top.vec_words);
    top.cb32 = h->arena.alloc<float>(top.vec_words);
    launch_fill<float>(S(h), top.cx32, top.vec_words, 0.0f);
    launch_fill<float>(S(h), top.cb32, top.vec_words, 0.0f);
  }
}

// Euclidean norms of velocity and pressure parts (synchronous).
template <typename T>
void norms(hhg_hier h, int l, const T* x, double* nu, double* np_) {
  Level& lv = h->L(l);
  if (h->um) {
    u_f64<T>();
    u_norms_launch(h, l, (const double*)x, (const double*)x);
  } else {
    launch_vsumsq<T>(S(h), lv.g, x, 3 * lv.g.vstride, h->partial, h->sums);
    launch_vsumsq<T>(S(h), lv.g, x + 3 * (size_t)lv.g.vstride, lv.g.nn, h->partial + 2 * kPartials, h->sums + 2);
  }
  HHG_CHECK_HIP(hipMemcpyAsync(h->hsums, h->sums, 4 * sizeof(double), hipMemcpyDeviceToHost, S(h)));
  HHG_CHECK_HIP(hipStreamSynchronize(S(h)));
  *nu = std::sqrt(h->hsums[0]);
  *np_ = std::sqrt(h->hsums[2]);
}

double fmg_work_units(const hhg_hier h, const hhg_solver_params& p) {
  // Sec. 4: W(P^-1) = sweeps * W_A + 2 W_B + W_C (normalised), variable V-cycle
  // bound 8/7 W(V_L^L) + 16/49 nu_inc W(P^-1), FMG bound 8 kappa / 7 W*.
  double a, bb, c;
  if (h->disc == HHG_P2P1) {
    a = 46.0 / 72.0, bb = 13.0 / 72.0, c = 0.0;
  } else {
    a = 0.3, bb = 0.3, c = 0.1;
  }
  const double sweeps = p.xi * (p.gs == HHG_GS_SYM ? 2.0 : 1.0);
  const double wp = sweeps * a + 2 * bb + c;
  const double wv = (p.nu_pre + p.nu_post) * wp + 1.0;
  const double wstar = 8.0 / 7.0 * wv + 16.0 / 49.0 * p.nu_inc * wp;
  return 8.0 * p.kappa / 7.0 * wstar;
}

double vcycle_work_units(const hhg_hier h, const hhg_solver_params& p) {
  double a, bb, c;
  if (h->disc == HHG_P2P1) {
    a = 46.0 / 72.0, bb = 13.0 / 72.0, c = 0.0;
  } else {
    a = 0.3, bb = 0.3, c = 0.1;
  }
  const double sweeps = p.xi * (p.gs == HHG_GS_SYM ? 2.0 : 1.0);
  const double wp = sweeps * a + 2 * bb + c;
  const double wv = (p.nu_pre + p.nu_post) * wp + 1.0;
  return 8.0 / 7.0 * wv + 16.0 / 49.0 * p.nu_inc * wp;
}

// Alg. fmg without stopping test: boundary data injected to every level,
// coarse solve, then per level FMG interpolation, boundary reset and kappa
// V-cycles (each followed by the mean-zero projection), then extra_cycles
// V-cycles on the finest level (when rtol <= 0).
template <typename BL>
void fmg_body(hhg_hier h, double* x, BL bl, const hhg_solver_params& p) {
  hipStream_t s = S(h);
  Level& top = h->L(h->lmax);
  op_copy_boundary(h, h->lmax, x, top.w);
  for (int l = h->lmax - 1; l >= h->lmin; --l) op_inject(h, l + 1, h->L(l + 1).w, h->L(l).w);
  Level& bot = h->L(h->lmin);
  launch_fill<double>(s, bot.xs, bot.vec_words, 0.0);
  op_copy_boundary(h, h->lmin, bot.w, bot.xs);
  op_coarse<double>(h, bot.xs, bl(h->lmin), true, &p);
  for (int l = h->lmin + 1; l <= h->lmax; ++l) {
    Level& lv = h->L(l);
    double* X = l == h->lmax ? x : lv.xs;
    op_prolong<double>(h, l - 1, h->L(l - 1).xs, X, false, false);
    op_copy_boundary(h, l, lv.w, X);
    for (int c = 0; c < p.kappa; ++c) {
      vcycle(h, l, l, X, bl(l), p);
      op_mean_zero<double>(h, l, X);
    }
  }
  if (p.rtol <= 0.0)
    for (int c = 0; c < p.extra_cycles; ++c) {
      vcycle(h, h->lmax, h->lmax, x, bl(h->lmax), p);
      op_mean_zero<double>(h, h->lmax, x);
    }
}

// The six Kuhn simplices of the cube [0,1]^3: vertices 0, e_a, e_a + e_b,
// (1,1,1) for the permutations (a, b, c) of the axes.
const int kPerm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

// Kuhn partition of the unit cube into N^3 sub-cubes of 6 tetrahedra each.
void kuhn_cube_mesh(int N, std::vector<double>& xyz, std::vector<int>& tet) {
  const int n1 = N + 1;
  xyz.clear();
  tet.clear();
  for (int k = 0; k <= N; ++k)
    for (int j = 0; j <= N; ++j)
      for (int i = 0; i <= N; ++i) {
        xyz.push_back((double)i / N);
        xyz.push_back((double)j / N);
        xyz.push_back((double)k / N);
      }
  for (int k = 0; k < N; ++k)
    for (int j = 0; j < N; ++j)
      for (int i = 0; i < N; ++i)
        for (const auto& pm : kPerm) {
          int c[3] = {i, j, k};
          tet.push_back(c[0] + n1 * (c[1] + n1 * c[2]));
          for (int s = 0; s < 3; ++s) {
            ++c[pm[s]];
            tet.push_back(c[0] + n1 * (c[1] + n1 * c[2]));
          }
        }
}

// N if (xyz, tet) is the Kuhn partition of the unit cube into N^3 sub-cubes
// (N = 1 or 2) in any vertex and tetrahedron order; otherwise throws
// HHG_ERR_ARG naming the first violation.
int kuhn_cube_refinement(const double* xyz, int nv, const int* tet, int nt) {
  HHG_REQUIRE(nt == 6 || nt == 48, HHG_ERR_ARG,
              "mesh: only the Kuhn partitions of the unit cube (6 or 48 tetrahedra) are supported, got " +
                  std::to_string(nt) + " tetrahedra");
  const int N = nt == 6 ? 1 : 2, n1 = N + 1;
  HHG_REQUIRE(nv == n1 * n1 * n1, HHG_ERR_ARG,
              "mesh: expected " + std::to_string(n1 * n1 * n1) + " vertices, got " + std::to_string(nv));
  std::vector<int> lat(nv);
  std::vector<int> seen(nv, 0);
  for (int v = 0; v < nv; ++v) {
    int c[3];
    for (int d = 0; d < 3; ++d) {
      const double t = xyz[3 * v + d] * N;
      c[d] = (int)std::lround(t);
      HHG_REQUIRE(std::isfinite(t) && std::fabs(t - c[d]) <= 1e-9 && c[d] >= 0 && c[d] <= N, HHG_ERR_ARG,
                  "mesh: vertex " + std::to_string(v) + " is not a point of the unit-cube lattice");
    }
    lat[v] = c[0] + n1 * (c[1] + n1 * c[2]);
    HHG_REQUIRE(!seen[lat[v]], HHG_ERR_ARG, "mesh: vertex " + std::to_string(v) + " duplicates another vertex");
    seen[lat[v]] = 1;
  }
  std::vector<int> used(nv, 0), cell_perm(6 * N * N * N, 0);
  for (int t = 0; t < nt; ++t) {
    int p[4][3];
    for (int q = 0; q < 4; ++q) {
      const int v = tet[4 * t + q];
      HHG_REQUIRE(v >= 0 && v < nv, HHG_ERR_ARG, "mesh: tetrahedron " + std::to_string(t) + " has a bad vertex index");
      used[v] = 1;
      const int L = lat[v];
      p[q][0] = L % n1, p[q][1] = (L / n1) % n1, p[q][2] = L / (n1 * n1);
    }
    // sort the corners by coordinate sum: a Kuhn simplex has one corner at
    // each sum b, b+1, b+2, b+3, each a unit step from the one before
    int ord[4] = {0, 1, 2, 3};
    std::sort(ord, ord + 4, [&](int a, int b) {
      return p[a][0] + p[a][1] + p[a][2] < p[b][0] + p[b][1] + p[b][2];
    });
    int axis[3];
    bool ok = true;
    for (int s = 0; s < 3 && ok; ++s) {
      int nd = 0, ax = -1;
      for (int d = 0; d < 3; ++d) {
        const int df = p[ord[s + 1]][d] - p[ord[s]][d];
        if (df == 1) ++nd, ax = d;
        else if (df != 0) ok = false;
      }
      ok = ok && nd == 1;
      axis[s] = ax;
    }
    ok = ok && axis[0] != axis[1] && axis[1] != axis[2] && axis[0] != axis[2];
    HHG_REQUIRE(ok, HHG_ERR_ARG, "mesh: tetrahedron " + std::to_string(t) + " is not a Kuhn simplex of a sub-cube");
    int perm = -1;
    for (int q = 0; q < 6; ++q)
      if (kPerm[q][0] == axis[0] && kPerm[q][1] == axis[1]) perm = q;
    const int* b = p[ord[0]];
    const int cell = b[0] + N * (b[1] + N * b[2]);
    HHG_REQUIRE(!cell_perm[6 * cell + perm], HHG_ERR_ARG,
                "mesh: tetrahedron " + std::to_string(t) + " appears twice");
    cell_perm[6 * cell + perm] = 1;
  }
  for (int v = 0; v < nv; ++v)
    HHG_REQUIRE(used[v], HHG_ERR_ARG, "mesh: vertex " + std::to_string(v) + " belongs to no tetrahedron");
  return N;
}

// Device time of a call: start() records an event on the context stream,
// seconds() records the end event and waits for it.
struct CallClock {
  hhg_hier h;
  explicit CallClock(hhg_hier hh) : h(hh) {
    if (!h->ev0) {
      HHG_CHECK_HIP(hipEventCreate(&h->ev0));
      HHG_CHECK_HIP(hipEventCreate(&h->ev1));
    }
    HHG_CHECK_HIP(hipEventRecord(h->ev0, h->ctx->stream));
  }
  double seconds() {
    HHG_CHECK_HIP(hipEventRecord(h->ev1, h->ctx->stream));
    HHG_CHECK_HIP(hipEventSynchronize(h->ev1));
    float ms = 0.f;
    HHG_CHECK_HIP(hipEventElapsedTime(&ms, h->ev0, h->ev1));
    return 1e-3 * ms;
  }
};

hhg_hier check_level(hhg_hier h, int l) {
  HHG_REQUIRE(h != nullptr, HHG_ERR_ARG, "null hierarchy");
  HHG_REQUIRE(l >= h->lmin && l <= h->lmax, HHG_ERR_ARG, "level out of range");
  return h;
}

template <typename F>
hhg_status guard(F&& f) {
  try {
    f();
    return HHG_OK;
  } catch (const Error& e) {
    set_error(e.msg);
    return e.code;
  } catch (const std::exception& e) {
    set_error(e.what());
    return HHG_ERR_STATE;
  } catch (...) {
    set_error("unknown error");
    return HHG_ERR_STATE;
  }
}

// Hierarchy on an unstructured T_0 (P1-P1 only): the level tables of the
// per-cell path, the work vectors of every level and the coarse unknowns.
hhg_hier u_hier_create(hhg_mesh mesh, hhg_disc disc, int lmin, int lmax, hhg_schur schur) {
  hhg_ctx ctx = mesh->ctx;
  HHG_REQUIRE(disc == HHG_P1P1, HHG_ERR_ARG, "unstructured macro meshes: P1-P1 only");
  HHG_REQUIRE(lmin >= 0 && lmin < lmax && lmax <= 9, HHG_ERR_ARG, "need 0 <= lmin < lmax <= 9");
  HHG_REQUIRE(schur == HHG_SCHUR_SD || schur == HHG_SCHUR_ML, HHG_ERR_ARG, "unknown Schur option");
  HHG_CHECK_HIP(hipSetDevice(ctx->device));
  std::unique_ptr<hhg_hier_s> h(new hhg_hier_s);
  h->ctx = ctx;
  h->disc = disc;
  h->mr = -1;
  h->lmin = lmin;
  h->lmax = lmax;
  h->schur = schur;
  h->G = 1;
  h->nf = mesh->outflow.empty() ? 0 : 1;  // the pressure is determined: no mean-zero steps
  h->um.reset(u_build(mesh->xyz.data(), (int)(mesh->xyz.size() / 3), mesh->tet.data(), (int)(mesh->tet.size() / 4),
                      mesh->outflow, lmin, lmax, schur));
  h->partial = h->arena.alloc<double>(4 * kPartials);
  h->sums = h->arena.alloc<double>(16);
  HHG_CHECK_HIP(hipHostMalloc((void**)&h->hsums, 16 * sizeof(double), hipHostMallocDefault));
  h->levels.resize(lmax - lmin + 1);
  for (int l = lmin; l <= lmax; ++l) {
    Level& lv = h->L(l);
    ULevelData& U = UL(h.get(), l);
    lv.l = l;
    lv.g.N = U.L.n;
    lv.g.n1 = U.L.n + 1;
    lv.g.nn = U.nnodes;
    lv.g.G = 1;
    lv.g.vstride = (int)U.L.vs;
    lv.vec_words = 4 * (size_t)U.L.vs;
    lv.r = h->arena.alloc<double>(lv.vec_words);
    lv.w = h->arena.alloc<double>(lv.vec_words);
    lv.xs = h->arena.alloc<double>(lv.vec_words);
    if (l < lmax) {
      lv.cx = h->arena.alloc<double>(lv.vec_words);
      lv.cb = h->arena.alloc<double>(lv.vec_words);
      launch_fill<double>(ctx->stream, lv.cx, lv.vec_words, 0.0);
      launch_fill<double>(ctx->stream, lv.cb, lv.vec_words, 0.0);
    }
    launch_fill<double>(ctx->stream, lv.r, lv.vec_words, 0.0);
    launch_fill<double>(ctx->stream, lv.w, lv.vec_words, 0.0);
    launch_fill<double>(ctx->stream, lv.xs, lv.vec_words, 0.0);
  }
  std::vector<int> unk;
  std::vector<double> K;
  u_coarse_system(*h->um, unk, K, 0);
  if (unk.size() <= 2048) {
    h->nunk = (int)unk.size();
    h->Kp = h->arena.alloc<double>(unk.size() * unk.size());
    h->unk = h->arena.upload(unk);
    h->unk_host = unk;
  }
  HHG_CHECK_HIP(hipGetLastError());
  HHG_CHECK_HIP(hipStreamSynchronize(ctx->stream));
  return h.release();
}

// Largest eigenvalue of D^{-1}(C + B A_s^{-1} B^T) by power iteration on the
// per-cell path (eq. omega-eigenvalue-problem); v0 in canonical node order.
double u_estimate_omega(hhg_hier h, int l, const double* v0, int iters) {
  Level& lv = h->L(l);
  ULevelData& U = UL(h, l);
  const size_t vs = U.L.vs, vs3 = 3 * vs;
  double* v = lv.xs;  // pressure part holds v
  double* z = lv.w;   // velocity part: sweep iterate; pressure part: -v for C
  double* y = lv.r;
  hipStream_t s = S(h);
  launch_fill<double>(s, v, lv.vec_words, 0.0);
  launch_u_pfrom_canon(s, U.L, U.canon, v0, v + vs3);
  op_mean_zero<double>(h, l, v);
  launch_u_dot(s, U.L, U.flags, nullptr, v, v, 3, 1, h->partial, h->sums, 0);
  launch_u_pscale(s, U.L, v + vs3, h->sums, 0);
  const int ncol = U.ncol_if + 4;
  for (int it = 0; it < iters; ++it) {
    launch_u_apply_rows(s, U.L, U.inner, U.zitems, U.lst, v, nullptr, y, 2, false, false, true, false);  // B^T v
    launch_fill<double>(s, z, lv.vec_words, 0.0);
    for (int c = 0; c < ncol; ++c) u_colour(h, l, c, z, y);
    for (int c = ncol - 1; c >= 0; --c) u_colour(h, l, c, z, y);
    launch_scaled_copy<double>(s, z + vs3, v + vs3, nullptr, vs, -1.0);
    launch_u_apply_rows(s, U.L, U.inner, U.zitems, U.lst, z, nullptr, y, 12, false, false, false, true);  // B z + C v
    launch_scaled_copy<double>(s, v + vs3, y + vs3, U.dinv, vs, 1.0);
    launch_u_dot(s, U.L, U.flags, nullptr, v, v, 3, 1, h->partial, h->sums, 0);
    if (it + 1 < iters) launch_u_pscale(s, U.L, v + vs3, h->sums, 0);
  }
  HHG_CHECK_HIP(hipMemcpyAsync(h->hsums, h->sums, sizeof(double), hipMemcpyDeviceToHost, s));
  HHG_CHECK_HIP(hipStreamSynchronize(s));
  return std::sqrt(h->hsums[0]);
}

// Calls that exist for the lattice path only.
void lattice_only(hhg_hier h, const char* what) {
  HHG_REQUIRE(!h || !h->um, HHG_ERR_STATE, std::string(what) + " is not available on unstructured macro meshes");
}

}  // namespace
}  // namespace hhg

using namespace hhg;

extern "C" {

const char* hhg_last_error(void) { return g_err.c_str(); }

hhg_status hhg_ctx_create(int device, void* stream, hhg_ctx* out) {
  return guard([&] {
    HHG_REQUIRE(out != nullptr, HHG_ERR_ARG, "null output");
    int n = 0;
    HHG_CHECK_HIP(hipGetDeviceCount(&n));
    HHG_REQUIRE(device >= 0 && device < n, HHG_ERR_ARG, "device out of range");
    HHG_CHECK_HIP(hipSetDevice(device));
    void* sp = nullptr;  // the scratch array's address on this device
    HHG_CHECK_HIP(hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch)));
    auto* c = new hhg_ctx_s;
    c->device = device;
    c->stream = (hipStream_t)stream;
    c->scratch = (unsigned char*)sp;
    *out = c;
  });
}

hhg_status hhg_ctx_set_stream(hhg_ctx ctx, void* stream) {
  return guard([&] {
    HHG_REQUIRE(ctx != nullptr, HHG_ERR_ARG, "null context");
    ctx->stream = (hipStream_t)stream;
  });
}

hhg_status hhg_ctx_destroy(hhg_ctx ctx) {
  return guard([&] {
    if (ctx && ctx->capture) (void)hipStreamDestroy(ctx->capture);
    delete ctx;
  });
}

hhg_status hhg_mesh_cube(hhg_ctx ctx, int macro_refine, hhg_mesh* out) {
  return guard([&] {
    HHG_REQUIRE(ctx && out, HHG_ERR_ARG, "null argument");
    HHG_REQUIRE(macro_refine == 0 || macro_refine == 1, HHG_ERR_ARG, "macro_refine must be 0 or 1");
    std::unique_ptr<hhg_mesh_s> m(new hhg_mesh_s);
    m->ctx = ctx;
    m->mr = macro_refine;
    kuhn_cube_mesh(1 << macro_refine, m->xyz, m->tet);
    *out = m.release();
  });
}

hhg_status hhg_mesh_create(hhg_ctx ctx, const double* xyz, int nv, const int* tet, int nt, hhg_mesh* out) {
  return guard([&] {
    HHG_REQUIRE(ctx && out && xyz && tet && nv > 0 && nt > 0, HHG_ERR_ARG, "null or empty argument");
    int N = 0;
    try {
      N = kuhn_cube_refinement(xyz, nv, tet, nt);
    } catch (const Error& e) {
      if (e.code != HHG_ERR_ARG) throw;
      validate_tet_mesh(xyz, nv, tet, nt);  // a general T_0: the per-cell path
    }
    std::unique_ptr<hhg_mesh_s> m(new hhg_mesh_s);
    m->ctx = ctx;
    m->general = N == 0;
    m->mr = N == 0 ? -1 : (N == 1 ? 0 : 1);
    m->xyz.assign(xyz, xyz + 3 * (size_t)nv);
    m->tet.assign(tet, tet + 4 * (size_t)nt);
    *out = m.release();
  });
}

hhg_status hhg_mesh_set_outflow(hhg_mesh mesh, unsigned faces) {
  return guard([&] {
    HHG_REQUIRE(mesh, HHG_ERR_ARG, "null mesh");
    HHG_REQUIRE(faces < 63u, HHG_ERR_ARG, "outflow faces: a mask of faces 0..5 with at least one Dirichlet face");
    if (mesh->general) {  // the boundary triangles on those planes of the unit cube
      const int nv = (int)(mesh->xyz.size() / 3), nt = (int)(mesh->tet.size() / 4);
      std::vector<std::array<int, 3>> of = boundary_faces_on_cube(mesh->xyz.data(), nv, mesh->tet.data(), nt, faces);
      HHG_REQUIRE(faces == 0 || !of.empty(), HHG_ERR_ARG, "outflow: no boundary face of the mesh on those planes");
      check_outflow_faces(mesh->tet.data(), nt, of);
      mesh->outflow = of;
    }
    mesh->nf = faces;
  });
}

hhg_status hhg_mesh_set_outflow_faces(hhg_mesh mesh, const int* tri, int ntri) {
  return guard([&] {
    HHG_REQUIRE(mesh && (tri || ntri == 0) && ntri >= 0, HHG_ERR_ARG, "bad arguments");
    HHG_REQUIRE(mesh->general, HHG_ERR_ARG,
                "explicit outflow faces: unstructured meshes only (Kuhn partitions: hhg_mesh_set_outflow)");
    std::vector<std::array<int, 3>> of(ntri);
    for (int q = 0; q < ntri; ++q) {
      for (int a = 0; a < 3; ++a) of[q][a] = tri[3 * q + a];
      std::sort(of[q].begin(), of[q].end());
    }
    std::sort(of.begin(), of.end());
    of.erase(std::unique(of.begin(), of.end()), of.end());
    check_outflow_faces(mesh->tet.data(), (int)(mesh->tet.size() / 4), of);
    mesh->outflow = of;
    mesh->nf = of.empty() ? 0u : 64u;  // bit 6: explicit faces
  });
}

hhg_status hhg_mesh_info(hhg_mesh mesh, int* nv, int* nt, int* macro_refine) {
  return guard([&] {
    HHG_REQUIRE(mesh, HHG_ERR_ARG, "null mesh");
    if (nv) *nv = (int)(mesh->xyz.size() / 3);
    if (nt) *nt = (int)(mesh->tet.size() / 4);
    if (macro_refine) *macro_refine = mesh->mr;
  });
}

hhg_status hhg_mesh_destroy(hhg_mesh mesh) {
  return guard([&] { delete mesh; });
}

hhg_status hhg_hier_create(hhg_mesh mesh, hhg_disc disc, int lmin, int lmax, hhg_schur schur, hhg_hier* out) {
  return guard([&] {
    HHG_REQUIRE(mesh && out, HHG_ERR_ARG, "null argument");
    if (mesh->general) {
      *out = u_hier_create(mesh, disc, lmin, lmax, schur);
      return;
    }
    hhg_ctx ctx = mesh->ctx;
    const int macro_refine = mesh->mr;
    HHG_REQUIRE(disc == HHG_P1P1 || disc == HHG_P2P1, HHG_ERR_ARG, "unknown discretisation");
    HHG_REQUIRE(lmin >= 0 && lmin < lmax, HHG_ERR_ARG, "need 0 <= lmin < lmax");
    HHG_REQUIRE((1 << (lmax + macro_refine)) <= (disc == HHG_P1P1 ? 512 : 256), HHG_ERR_ARG,
                "finest level too large (N <= 512 for P1-P1, N <= 256 for P2-P1)");
    HHG_REQUIRE(schur == HHG_SCHUR_SD || schur == HHG_SCHUR_ML, HHG_ERR_ARG, "unknown Schur option");
    HHG_REQUIRE(disc == HHG_P1P1 || (1 << (lmin + macro_refine)) >= 2, HHG_ERR_ARG,
                "Taylor-Hood needs at least 2 intervals on the coarsest level");
    HHG_CHECK_HIP(hipSetDevice(ctx->device));
    std::unique_ptr<hhg_hier_s> h(new hhg_hier_s);
    h->ctx = ctx;
    h->nf = (int)mesh->nf;
    h->disc = disc;
    h->mr = macro_refine;
    h->lmin = lmin;
    h->lmax = lmax;
    h->schur = schur;
    h->G = disc == HHG_P1P1 ? 1 : 8;
    ElementSet es;
    build_elements(disc == HHG_P1P1 ? 1 : 2, &es);
    h->partial = h->arena.alloc<double>(4 * kPartials);
    h->sums = h->arena.alloc<double>(16);
    HHG_CHECK_HIP(hipHostMalloc((void**)&h->hsums, 16 * sizeof(double), hipHostMallocDefault));
    h->levels.resize(lmax - lmin + 1);
    for (int l = lmin; l <= lmax; ++l) {
      Level& lv = h->L(l);
      lv.l = l;
      const int N = 1 << (l + macro_refine);
      lv.g.N = N;
      lv.g.n1 = N + 1;
      lv.g.nn = (N + 1) * (N + 1) * (N + 1);
      lv.g.G = h->G;
      lv.g.vstride = h->G * lv.g.nn;
      lv.g.nf = h->nf;
      lv.h = 1.0 / N;
      lv.vec_words = 3 * (size_t)lv.g.vstride + lv.g.nn;
      build_level_tables(h.get(), lv, es);
      lv.r = h->arena.alloc<double>(lv.vec_words);
      lv.r32 = h->arena.alloc<float>(lv.vec_words);
      lv.w = h->arena.alloc<double>(lv.vec_words);
      lv.xs = h->arena.alloc<double>(lv.vec_words);
      if (l < lmax) {
        lv.cx = h->arena.alloc<double>(lv.vec_words);
        lv.cb = h->arena.alloc<double>(lv.vec_words);
      }
      launch_fill<double>(ctx->stream, lv.r, lv.vec_words, 0.0);
      launch_fill<float>(ctx->stream, lv.r32, lv.vec_words, 0.0f);
      launch_fill<double>(ctx->stream, lv.w, lv.vec_words, 0.0);
      launch_fill<double>(ctx->stream, lv.xs, lv.vec_words, 0.0);
    }
    for (int l = lmin + 1; l <= lmax; ++l) build_transfer(h.get(), h->L(l - 1), h->L(l));
    if (h->nf) build_neumann(h.get(), es);
    for (int l = lmin; l <= lmax; ++l) {  // Schur diagonal per pressure node
      Level& lv = h->L(l);
      launch_schur_diag<double>(ctx->stream, lv.g, lv.tb64, nullptr, schur, lv.dinv64, lv.neu64);
      launch_schur_diag<float>(ctx->stream, lv.g, lv.tb32, nullptr, schur, lv.dinv32, lv.neu32);
    }
    HHG_CHECK_HIP(hipGetLastError());
    build_coarse(h.get());
    small_kernel_attributes();
    refresh_small(h.get());
    HHG_CHECK_HIP(hipStreamSynchronize(ctx->stream));
    *out = h.release();
  });
}

hhg_status hhg_hier_destroy(hhg_hier h) {
  return guard([&] {
    if (!h) return;
    (void)hipStreamSynchronize(h->ctx->stream);
    if (h->fmg_exec) (void)hipGraphExecDestroy(h->fmg_exec);
    if (h->ev0) (void)hipEventDestroy(h->ev0);
    if (h->ev1) (void)hipEventDestroy(h->ev1);
    if (h->hsums) (void)hipHostFree(h->hsums);
    delete h;
  });
}

hhg_status hhg_vec_layout(hhg_hier h, int level, int* N, size_t* nn, size_t* vec_words, size_t* lattice_words) {
  return guard([&] {
    check_level(h, level);
    Level& lv = h->L(level);
    if (N) *N = lv.g.N;
    if (nn) *nn = lv.g.nn;
    if (vec_words) *vec_words = lv.vec_words;
    const size_t m1 = (h->G == 1 ? lv.g.N : 2 * lv.g.N) + 1;
    if (lattice_words) *lattice_words = h->um ? 4 * (size_t)lv.g.nn : 3 * m1 * m1 * m1 + lv.g.nn;
  });
}

#define HHG_DISPATCH(prec, F)                                              \
  do {                                                                     \
    if ((prec) == HHG_F64) {                                               \
      using T = double;                                                    \
      F;                                                                   \
    } else if ((prec) == HHG_F32) {                                        \
      using T = float;                                                     \
      F;                                                                   \
    } else {                                                               \
      throw Error{HHG_ERR_PREC, "unsupported precision"};                  \
    }                                                                      \
  } while (0)

hhg_status hhg_vec_from_lattice(hhg_hier h, int level, const double* src, void* dst, hhg_prec prec) {
  return guard([&] {
    check_level(h, level);
    HHG_REQUIRE(src && dst, HHG_ERR_ARG, "null vector");
    Level& lv = h->L(level);
    if (h->um) {
      HHG_REQUIRE(prec == HHG_F64, HHG_ERR_PREC, "unstructured macro meshes: float64 only");
      ULevelData& U = UL(h, level);
      launch_fill<double>(S(h), (double*)dst, lv.vec_words, 0.0);
      launch_u_from_canon(S(h), U.L, U.canon, U.nnodes, src, (double*)dst);
      HHG_CHECK_HIP(hipGetLastError());
      return;
    }
    HHG_DISPATCH(prec, {
      launch_fill<T>(S(h), (T*)dst, lv.vec_words, T(0));
      launch_from_lattice<T>(S(h), lv.g, src, (T*)dst);
      round_out<T>(h, level, (T*)dst, 0, 0, lv.vec_words, 1);
    });
    HHG_CHECK_HIP(hipGetLastError());
  });
}

hhg_status hhg_vec_to_lattice(hhg_hier h, int level, const void* src, double* dst, hhg_prec prec) {
  return guard([&] {
    check_level(h, level);
    HHG_REQUIRE(src && dst, HHG_ERR_ARG, "null vector");
    Level& lv = h->L(level);
    if (h->um) {
      HHG_REQUIRE(prec == HHG_F64, HHG_ERR_PREC, "unstructured macro meshes: float64 only");
      ULevelData& U = UL(h, level);
      launch_u_to_canon(S(h), U.L, U.canon, U.flags, U.nnodes, (const double*)src, dst);
      HHG_CHECK_HIP(hipGetLastError());
      return;
    }
    HHG_DISPATCH(prec, launch_to_lattice<T>(S(h), lv.g, (const T*)src, dst));
    HHG_CHECK_HIP(hipGetLastError());
  });
}

hhg_status hhg_apply(hhg_hier h, int level, hhg_op op, const void* x, void* y, hhg_prec prec) {
  return guard([&] {
    check_level(h, level);
    HHG_REQUIRE(x && y && x != y, HHG_ERR_ARG, "bad vectors");
    Level& lv = h->L(level);
    int mask = 0;
    switch (op) {
      case HHG_OP_FULL: mask = full_mask(h); break;
      case HHG_OP_A: mask = 1; break;
      case HHG_OP_BT: mask = 2; break;
      case HHG_OP_B: mask = 4; break;
      case HHG_OP_C: mask = 8 | 16; break;
      case HHG_OP_MASS: mask = -1; break;
      default: throw Error{HHG_ERR_ARG, "operator not supported"};
    }
    if (mask < 0 && h->um) {
      HHG_REQUIRE(prec == HHG_F64, HHG_ERR_PREC, "unstructured macro meshes: float64 only");
      ULevelData& U = UL(h, level);
      launch_u_apply_rows(S(h), U.L, U.inner, U.zitems, U.lst, (const double*)x, nullptr, (double*)y, 0, false, true, true, true);
      HHG_CHECK_HIP(hipGetLastError());
      return;
    }
    if (mask < 0) {
      HHG_DISPATCH(prec, {
        launch_mass<T>(S(h), lv.g, tables<T>(lv), (const T*)x, (T*)y);
        round_out<T>(h, level, (T*)y, 0, 0, lv.vec_words, 1);
      });
      HHG_CHECK_HIP(hipGetLastError());
      return;
    }
    if (op == HHG_OP_C && h->disc == HHG_P2P1) mask = 0;
    HHG_DISPATCH(prec, {
      op_apply<T>(h, level, mask, (const T*)x, nullptr, (T*)y, false, true, true);
      (void)lv;
    });
    HHG_CHECK_HIP(hipGetLastError());
  });
}

hhg_status hhg_residual(hhg_hier h, int level, const void* x, const void* b, void* r, hhg_prec prec) {
  return guard([&] {
    check_level(h, level);
    HHG_REQUIRE(x && b && r && x != r && b != r, HHG_ERR_ARG, "bad vectors");
    HHG_DISPATCH(prec, op_apply<T>(h, level, full_mask(h), (const T*)x, (const T*)b, (T*)r, true, true, true));
    HHG_CHECK_HIP(hipGetLastError());
  });
}

hhg_status hhg_rhs(hhg_hier h, int level, const void* f, void* b, hhg_prec prec) {
  return guard([&] {
    check_level(h, level);
    HHG_REQUIRE(f && b && f != b, HHG_ERR_ARG, "bad vectors");
    Level& lv = h->L(level);
    if (h->um) {  // b = M I(f) on the free velocity rows, zero elsewhere
      HHG_REQUIRE(prec == HHG_F64, HHG_ERR_PREC, "unstructured macro meshes: float64 only");
      ULevelData& U = UL(h, level);
      launch_u_apply_rows(S(h), U.L, U.inner, U.zitems, U.lst, (const double*)f, nullptr, (double*)b, 0, false, true, true, true);
      launch_u_rhs_fix(S(h), U.L, U.flags, (double*)b);
      HHG_CHECK_HIP(hipGetLastError());
      return;
    }
    HHG_DISPATCH(prec, {
      launch_rhs<T>(S(h), lv.g, lconst<T>(lv), (const T*)f, (T*)b);
      if (lv.neu_n) launch_neu_rhs<T>(S(h), lv.g, tables<T>(lv), lv.neu(), lv.neu_n, (const T*)f, (T*)b);
      round_out<T>(h, level, (T*)b, 0, 0, lv.vec_words, 1);
    });
    HHG_CHECK_HIP(hipGetLastError());
  });
}

hhg_status hhg_smooth(hhg_hier h, int level, void* x, const void* b, int iters, hhg_gs gs, int xi, double omega_inv,
                      hhg_prec prec) {
  return guard([&] {
    check_level(h, level);
    HHG_REQUIRE(x && b && x != b, HHG_ERR_ARG, "bad vectors");
    HHG_REQUIRE(iters >= 0 && xi >= 1 && omega_inv > 0.0, HHG_ERR_ARG, "bad smoother parameters");
    HHG_REQUIRE(gs == HHG_GS_FWD || gs == HHG_GS_SYM, HHG_ERR_ARG, "bad Gauss-Seidel variant");
    HHG_DISPATCH(prec, op_smooth<T>(h, level, (T*)x, (const T*)b, iters, gs, xi, 1.0 / omega_inv));
    HHG_CHECK_HIP(hipGetLastError());
  });
}

hhg_status hhg_restrict(hhg_hier h, int fine_level, const void* rf, void* rc, hhg_prec prec) {
  return guard([&] {
    check_level(h, fine_level);
    HHG_REQUIRE(fine_level > h->lmin, HHG_ERR_ARG, "no coarser level");
    HHG_REQUIRE(rf && rc, HHG_ERR_ARG, "null vector");
    HHG_DISPATCH(prec, op_restrict<T>(h, fine_level, (const T*)rf, (T*)rc));
    HHG_CHECK_HIP(hipGetLastError());
  });
}

hhg_status hhg_prolong_add(hhg_hier h, int coarse_level, const void* xc, void* xf, hhg_prec prec) {
  return guard([&] {
    check_level(h, coarse_level);
    HHG_REQUIRE(coarse_level < h->lmax, HHG_ERR_ARG, "no finer level");
    HHG_REQUIRE(xc && xf, HHG_ERR_ARG, "null vector");
    HHG_DISPATCH(prec, op_prolong<T>(h, coarse_level, (const T*)xc, (T*)xf, true, false));
    HHG_CHECK_HIP(hipGetLastError());
  });
}

hhg_status hhg_coarse_solve(hhg_hier h, void* x, const void* b, hhg_prec prec) {
  return guard([&] {
    HHG_REQUIRE(h && x && b && x != b, HHG_ERR_ARG, "bad arguments");
    HHG_REQUIRE(prec == HHG_F64, HHG_ERR_PREC, "coarse solve is float64");
    ensure_coarse(h);
    op_coarse<double>(h, (double*)x, (const double*)b);
    HHG_CHECK_HIP(hipGetLastError());
  });
}

hhg_status hhg_project_mean_zero(hhg_hier h, int level, void* x, hhg_prec prec) {
  return guard([&] {
    check_level(h, level);
    HHG_REQUIRE(x, HHG_ERR_ARG, "null vector");
    HHG_DISPATCH(prec, op_mean_zero_always<T>(h, level, (T*)x));
    HHG_CHECK_HIP(hipGetLastError());
  });
}

hhg_status hhg_copy_boundary(hhg_hier h, int level, const void* src, void* dst, hhg_prec prec) {
  return guard([&] {
    check_level(h, level);
    HHG_REQUIRE(src && dst, HHG_ERR_ARG, "null vector");
    Level& lv = h->L(level);
    if (h->um) {
      HHG_REQUIRE(prec == HHG_F64, HHG_ERR_PREC, "unstructured macro meshes: float64 only");
      op_copy_boundary(h, level, (const double*)src, (double*)dst);
      HHG_CHECK_HIP(hipGetLastError());
      return;
    }
    HHG_DISPATCH(prec, launch_copy_boundary<T>(S(h), lv.g, (const T*)src, (T*)dst));
    HHG_CHECK_HIP(hipGetLastError());
  });
}

hhg_status hhg_norms(hhg_hier h, int level, const void* x, double* nu, double* np_, hhg_prec prec) {
  return guard([&] {
    check_level(h, level);
    HHG_REQUIRE(x && nu && np_, HHG_ERR_ARG, "null argument");
    HHG_DISPATCH(prec, norms<T>(h, level, (const T*)x, nu, np_));
  });
}

hhg_status hhg_estimate_omega(hhg_hier h, int level, const double* v0, int iters, double* omega_inv) {
  return guard([&] {
    check_level(h, level);
    HHG_REQUIRE(v0 && omega_inv && iters >= 1, HHG_ERR_ARG, "bad arguments");
    Level& lv = h->L(level);
    if (h->um) {
      *omega_inv = u_estimate_omega(h, level, v0, iters);
      return;
    }
    const Geom& g = lv.g;
    const size_t vs3 = 3 * (size_t)g.vstride;
    double* v = lv.xs;   // pressure part holds v; velocity part zero
    double* z = lv.w;    // velocity part: sweep iterate; pressure part: -v for C
    double* y = lv.r;    // B^T v (velocity rows), then (B z + C v) (pressure rows)
    hipStream_t s = S(h);
    launch_fill<double>(s, v, lv.vec_words, 0.0);
    HHG_CHECK_HIP(hipMemcpyAsync(v + vs3, v0, g.nn * sizeof(double), hipMemcpyDeviceToDevice, s));
    op_mean_zero<double>(h, level, v);
    auto normalise = [&]() {
      launch_vsumsq<double>(s, g, v + vs3, g.nn, h->partial, h->sums);
      launch_scale<double>(s, v + vs3, g.nn, h->sums, 0);
    };
    normalise();
    const int ncol = gs_colours(h->G);
    for (int it = 0; it < iters; ++it) {
      op_apply<double>(h, level, 2, v, nullptr, y, false, true, false);   // B^T v
      launch_fill<double>(s, z, lv.vec_words, 0.0);
      auto colour = [&](int c) {
        launch_gs_colour<double>(s, g, lv.lc64, z, y, c);
        if (lv.neu_n)
          launch_neu_gs<double>(s, g, lv.neu64, lv.neu(), lv.neu_coff[c], lv.neu_coff[c + 1] - lv.neu_coff[c], z, y);
      };
      for (int c = 0; c < ncol; ++c) colour(c);
      for (int c = ncol - 1; c >= 0; --c) colour(c);
      launch_scaled_copy<double>(s, z + vs3, v + vs3, nullptr, g.nn, -1.0);
      op_apply<double>(h, level, full_mask(h) & 12, z, nullptr, y, false, false, true);  // B z + C v
      launch_scaled_copy<double>(s, v + vs3, y + vs3, lv.dinv64, g.nn, 1.0);         // w = D^{-1}(...)
      launch_vsumsq<double>(s, g, v + vs3, g.nn, h->partial, h->sums);
      if (it + 1 < iters) launch_scale<double>(s, v + vs3, g.nn, h->sums, 0);
    }
    HHG_CHECK_HIP(hipMemcpyAsync(h->hsums, h->sums, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    HHG_CHECK_HIP(hipStreamSynchronize(s));
    *omega_inv = std::sqrt(h->hsums[0]);
  });
}

hhg_status hhg_dots(hhg_hier h, int level, const void* x, const void* y, double* dot_u, double* dot_p,
                    hhg_prec prec) {
  return guard([&] {
    check_level(h, level);
    HHG_REQUIRE(x && y && dot_u && dot_p, HHG_ERR_ARG, "null argument");
    Level& lv = h->L(level);
    const size_t nv = 3 * (size_t)lv.g.vstride;
    if (h->um) {
      HHG_REQUIRE(prec == HHG_F64, HHG_ERR_PREC, "unstructured macro meshes: float64 only");
      u_norms_launch(h, level, (const double*)x, (const double*)y);
    } else
    HHG_DISPATCH(prec, {
      launch_dot<T>(S(h), (const T*)x, (const T*)y, nv, h->partial, h->sums);
      launch_dot<T>(S(h), (const T*)x + nv, (const T*)y + nv, lv.g.nn, h->partial + 2 * kPartials, h->sums + 2);
    });
    HHG_CHECK_HIP(hipMemcpyAsync(h->hsums, h->sums, 4 * sizeof(double), hipMemcpyDeviceToHost, S(h)));
    HHG_CHECK_HIP(hipStreamSynchronize(S(h)));
    *dot_u = h->hsums[0];
    *dot_p = h->hsums[2];
  });
}

hhg_status hhg_timer_start(unsigned family_mask) {
  return guard([&] {
    timer_set_mask(family_mask);
    for (int f = 0; f < KF_COUNT; ++f) timer_read(f, nullptr, nullptr, nullptr);
  });
}

hhg_status hhg_timer_read(int family, double* total_ms, int* launches, double* units) {
  return guard([&] {
    HHG_REQUIRE(family >= 0 && family < KF_COUNT, HHG_ERR_ARG, "unknown kernel family");
    timer_read(family, total_ms, launches, units);
  });
}

hhg_status hhg_set_viscosity(hhg_hier h, int level, const double* nu) {
  return guard([&] {
    check_level(h, level);
    HHG_REQUIRE(nu, HHG_ERR_ARG, "null viscosity");
    lattice_only(h, "variable viscosity");
    HHG_REQUIRE(h->nf == 0, HHG_ERR_STATE, "variable viscosity with an outflow face is not supported");
    Level& lv = h->L(level);
    hipStream_t s = S(h);
    const size_t nn = lv.g.nn;
    if (!lv.nu64) {
      lv.nu64 = h->arena.alloc<double>(nn);
      lv.nu32 = h->arena.alloc<float>(nn);
      lv.ainvs64 = h->arena.alloc<double>((size_t)lv.g.vstride);
      lv.ainvs32 = h->arena.alloc<float>((size_t)lv.g.vstride);
    }
    HHG_CHECK_HIP(hipMemcpyAsync(lv.nu64, nu, nn * sizeof(double), hipMemcpyDeviceToDevice, s));
    launch_to_f32(s, lv.nu64, lv.nu32, nn);
    lv.lc64.nu = lv.nu64;
    lv.lc32.nu = lv.nu32;
    lv.lc64.ainv_site = lv.ainvs64;
    lv.lc32.ainv_site = lv.ainvs32;
    launch_nu_diag<double>(s, lv.g, lv.lc64, lv.ainvs64);
    launch_nu_diag<float>(s, lv.g, lv.lc32, lv.ainvs32);
    launch_schur_diag<double>(s, lv.g, lv.tb64, lv.ainvs64, h->schur, lv.dinv64, lv.neu64);
    launch_schur_diag<float>(s, lv.g, lv.tb32, lv.ainvs32, h->schur, lv.dinv32, lv.neu32);
    h->slv_stale = true;
    if (h->fmg_exec) {  // a captured solve holds the old operator
      HHG_CHECK_HIP(hipGraphExecDestroy(h->fmg_exec));
      h->fmg_exec = nullptr;
      h->fmg_key.clear();
    }
    if (level == h->lmin) {
      if (h->mlp) {
        h->kp_stale = true;  // rebuilt only if the plain coarse solve is needed
      } else {
        build_coarse_device(h);
      }
    }
    HHG_CHECK_HIP(hipStreamSynchronize(s));
  });
}

hhg_status hhg_dc_solve(hhg_hier h, void* xv, const void* bv, const hhg_solver_params* prm, hhg_prec inner_prec,
                        int inner_cycles, double rtol, int max_outer, hhg_stats* stats) {
  return guard([&] {
    HHG_REQUIRE(h && xv && bv && prm, HHG_ERR_ARG, "null argument");
    lattice_only(h, "defect correction");
    HHG_REQUIRE(inner_prec == HHG_F64 || inner_prec == HHG_F32, HHG_ERR_PREC, "inner precision must be F64 or F32");
    HHG_REQUIRE(inner_cycles >= 1 && rtol > 0.0 && max_outer >= 1, HHG_ERR_ARG, "bad iteration parameters");
    HHG_REQUIRE(prm->omega_inv > 0.0 && prm->xi >= 1, HHG_ERR_ARG, "bad solver parameters");
    HHG_REQUIRE(h->nunk > 0, HHG_ERR_STATE, "no dense coarse solve on this hierarchy");
    const int L = h->lmax;
    Level& top = h->L(L);
    hipStream_t s = S(h);
    double* x = (double*)xv;
    const double* b = (const double*)bv;
    if (inner_prec == HHG_F32) ensure_f32_vectors(h);
    ensure_coarse(h);
    refresh_small(h);
    CallClock clock(h);
    double bu, bp, ru = 0, rp = 0;
    norms<double>(h, L, b, &bu, &bp);
    const double bn = std::sqrt(bu * bu + bp * bp);
    int outer = 0, cycles = 0, fallbacks = 0;
    bool f32 = inner_prec == HHG_F32;
    auto ensure_f64_work = [&]() {
      if (!top.dc_e) {
        top.dc_e = h->arena.alloc<double>(top.vec_words);
        top.dc_r = h->arena.alloc<double>(top.vec_words);
      }
    };
    if (!f32) ensure_f64_work();
    if (f32 && !top.dc_bk) top.dc_bk = h->arena.alloc<double>(top.vec_words);
    double prev = -1.0;
    for (;;) {
      op_apply<double>(h, L, full_mask(h), x, b, top.r, true, true, true);   // r = b - A x (float64)
      norms<double>(h, L, top.r, &ru, &rp);
      const double rn = std::sqrt(ru * ru + rp * rp);
      if (f32 && prev >= 0.0 && !(rn < prev)) {
        // the last float32 correction did not reduce the float64 residual (or
        // made it non-finite): undo it, finish with float64 inner cycles
        HHG_CHECK_HIP(hipMemcpyAsync(x, top.dc_bk, top.vec_words * sizeof(double), hipMemcpyDeviceToDevice, s));
        f32 = false;
        ++fallbacks;
        ensure_f64_work();
        continue;
      }
      if (rn <= rtol * bn || outer >= max_outer) break;
      prev = rn;
      if (f32) {
        HHG_CHECK_HIP(hipMemcpyAsync(top.dc_bk, x, top.vec_words * sizeof(double), hipMemcpyDeviceToDevice, s));
        launch_to_f32(s, top.r, top.cb32, top.vec_words);                     // RNE
        round_out<float>(h, L, top.cb32, 0, 0, top.vec_words, 1);
        launch_fill<float>(s, top.cx32, top.vec_words, 0.0f);
        for (int c = 0; c < inner_cycles; ++c) vcycle_t<float>(h, L, L, top.cx32, top.cb32, *prm);
        launch_add_f32_to_f64(s, x, top.cx32, top.vec_words);
      } else {  // the V-cycle uses top.r as its own residual vector: keep the rhs apart
        HHG_CHECK_HIP(hipMemcpyAsync(top.dc_r, top.r, top.vec_words * sizeof(double), hipMemcpyDeviceToDevice, s));
        launch_fill<double>(s, top.dc_e, top.vec_words, 0.0);
        for (int c = 0; c < inner_cycles; ++c) vcycle_t<double>(h, L, L, top.dc_e, top.dc_r, *prm);
        launch_axpy<double>(s, x, top.dc_e, top.vec_words, 1.0);
      }
      op_mean_zero<double>(h, L, x);
      ++outer;
      cycles += inner_cycles;
    }
    HHG_CHECK_HIP(hipGetLastError());
    if (stats) {
      stats->cycles = cycles;
      stats->res_u = ru;
      stats->res_p = rp;
      stats->rel_res = bn > 0 ? std::sqrt(ru * ru + rp * rp) / bn : 0.0;
      stats->work_units = cycles * vcycle_work_units(h, *prm);
      stats->seconds = clock.seconds();
      stats->fallbacks = fallbacks;
    }
    if (std::sqrt(ru * ru + rp * rp) > rtol * bn)
      throw Error{HHG_ERR_NOT_CONVERGED, "relative residual above rtol after max_outer corrections"};
  });
}

hhg_status hhg_mlp_create(hhg_ctx ctx, int n_in, int n_hidden, int n_out, int max_batch, hhg_mlp* out) {
  return guard([&] {
    HHG_REQUIRE(ctx && out, HHG_ERR_ARG, "null argument");
    HHG_REQUIRE(n_in >= 1 && n_out >= 1 && n_hidden >= 16 && n_hidden % 16 == 0 && max_batch >= 1, HHG_ERR_ARG,
                "bad MLP sizes (hidden width a multiple of 16)");
    HHG_CHECK_HIP(hipSetDevice(ctx->device));
    std::unique_ptr<hhg_mlp_s> m(new hhg_mlp_s);
    m->ctx = ctx;
    m->net.init(n_in, n_hidden, n_out, max_batch);
    HHG_CHECK_HIP(hipMalloc(&m->idx, sizeof(int) * max_batch));
    HHG_CHECK_HIP(hipMalloc(&m->bx, sizeof(float) * (size_t)max_batch * n_in));
    HHG_CHECK_HIP(hipMalloc(&m->by, sizeof(float) * (size_t)max_batch * n_out));
    *out = m.release();
  });
}

hhg_status hhg_mlp_destroy(hhg_mlp m) {
  return guard([&] {
    if (!m) return;
    (void)hipDeviceSynchronize();
    (void)hipFree(m->idx);
    (void)hipFree(m->bx);
    (void)hipFree(m->by);
    delete m;
  });
}

hhg_status hhg_mlp_num_params(hhg_mlp m, size_t* n) {
  return guard([&] {
    HHG_REQUIRE(m && n, HHG_ERR_ARG, "null argument");
    *n = (size_t)m->net.host_params();
  });
}

hhg_status hhg_mlp_set_params(hhg_mlp m, const float* host) {
  return guard([&] {
    HHG_REQUIRE(m && host, HHG_ERR_ARG, "null argument");
    m->net.set_params(host);
  });
}

hhg_status hhg_mlp_get_params(hhg_mlp m, float* host) {
  return guard([&] {
    HHG_REQUIRE(m && host, HHG_ERR_ARG, "null argument");
    HHG_CHECK_HIP(hipStreamSynchronize(m->ctx->stream));
    m->net.unpack(m->net.P, host);
  });
}

hhg_status hhg_mlp_forward(hhg_mlp m, const float* x, int batch, float* y) {
  return guard([&] {
    HHG_REQUIRE(m && x && y, HHG_ERR_ARG, "null argument");
    HHG_REQUIRE(batch >= 1 && batch <= m->net.max_batch, HHG_ERR_ARG, "batch out of range");
    m->net.forward(m->ctx->stream, x, batch, y);
    HHG_CHECK_HIP(hipGetLastError());
  });
}

hhg_status hhg_mlp_loss_grad(hhg_mlp m, const float* x, const float* y, int batch, float* grad_host, double* loss) {
  return guard([&] {
    HHG_REQUIRE(m && x && y && grad_host && loss, HHG_ERR_ARG, "null argument");
    HHG_REQUIRE(batch >= 1 && batch <= m->net.max_batch, HHG_ERR_ARG, "batch out of range");
    *loss = m->net.loss_grad(m->ctx->stream, x, y, batch);
    HHG_CHECK_HIP(hipStreamSynchronize(m->ctx->stream));
    m->net.unpack(m->net.Gr, grad_host);
  });
}

namespace hhg {
namespace {
// Checks of a training call; returns the number of order entries.
size_t check_train_args(hhg_mlp m, const float* x, const float* y, int n_samples, int batch, int epochs, float lr,
                        const int* order) {
  HHG_REQUIRE(m && x && y && order, HHG_ERR_ARG, "null argument");
  HHG_REQUIRE(n_samples >= 1 && epochs >= 1 && lr > 0.f && batch >= 1 && batch <= m->net.max_batch, HHG_ERR_ARG,
              "bad training parameters");
  HHG_REQUIRE(n_samples / batch >= 1, HHG_ERR_ARG, "batch larger than the data set");
  const size_t nord = (size_t)epochs * n_samples;
  for (size_t q = 0; q < nord; ++q)
    HHG_REQUIRE(order[q] >= 0 && order[q] < n_samples, HHG_ERR_ARG, "sample index out of range");
  return nord;
}
// The Adam steps of every full minibatch of every epoch, enqueued on the
// context stream: dord = the order on the device, dloss[e] += batch losses of
// epoch e (zeroed by the caller).
void train_steps(hhg_mlp m, const float* x, const float* y, int n_samples, int batch, int epochs, float lr,
                 const int* dord, double* dloss) {
  hipStream_t s = m->ctx->stream;
  const int nb = n_samples / batch;
  for (int e = 0; e < epochs; ++e)
    for (int q = 0; q < nb; ++q) {
      const int* idx = dord + (size_t)e * n_samples + (size_t)q * batch;
      m->net.train_step_dev(s, x, y, idx, batch, lr, dloss + e);
    }
}
}  // namespace
}  // namespace hhg

hhg_status hhg_mlp_train(hhg_mlp m, const float* x, const float* y, int n_samples, int batch, int epochs, float lr,
                         const int* order, double* last_loss) {
  return guard([&] {
    const size_t nord = check_train_args(m, x, y, n_samples, batch, epochs, lr, order);
    hipStream_t s = m->ctx->stream;
    const int nb = n_samples / batch;  // full minibatches per epoch
    // the whole order and one loss accumulator per epoch on the device: the
    // steps are enqueued without host round trips
    int* dord = nullptr;
    double* dloss = nullptr;
    HHG_CHECK_HIP(hipMalloc(&dord, nord * sizeof(int)));
    hipError_t e0 = hipMalloc(&dloss, (size_t)epochs * sizeof(double));
    if (e0 != hipSuccess) {
      (void)hipFree(dord);
      HHG_CHECK_HIP(e0);
    }
    std::vector<double> hloss(epochs, 0.0);
    hipError_t err = hipMemcpyAsync(dord, order, nord * sizeof(int), hipMemcpyHostToDevice, s);
    if (err == hipSuccess) err = hipMemcpyAsync(dloss, hloss.data(), epochs * sizeof(double), hipMemcpyHostToDevice, s);
    if (err == hipSuccess) train_steps(m, x, y, n_samples, batch, epochs, lr, dord, dloss);
    if (err == hipSuccess) err = hipMemcpyAsync(hloss.data(), dloss, epochs * sizeof(double), hipMemcpyDeviceToHost, s);
    if (err == hipSuccess) err = hipStreamSynchronize(s);
    (void)hipFree(dord);
    (void)hipFree(dloss);
    HHG_CHECK_HIP(err);
    HHG_CHECK_HIP(hipGetLastError());
    if (last_loss) *last_loss = hloss[epochs - 1] / nb;
  });
}

hhg_status hhg_mlp_train_noalloc(hhg_mlp m, const float* x, const float* y, int n_samples, int batch, int epochs,
                                 float lr, const int* order, double* last_loss) {
  return guard([&] {
    const size_t nord = check_train_args(m, x, y, n_samples, batch, epochs, lr, order);
    HHG_REQUIRE((size_t)epochs <= kScratchEpochs && nord <= kScratchOrder, HHG_ERR_ARG,
                "hhg_mlp_train_noalloc: epochs * n_samples must be at most " + std::to_string(kScratchOrder) +
                    " and epochs at most " + std::to_string(kScratchEpochs) + " (static scratch); got " +
                    std::to_string(nord) + " and " + std::to_string(epochs));
    hipStream_t s = m->ctx->stream;
    double* dloss = (double*)m->ctx->scratch;
    int* dord = (int*)(m->ctx->scratch + kScratchEpochs * sizeof(double));
    launch_fill<double>(s, dloss, (size_t)epochs, 0.0);  // the previous call left its losses here
    HHG_CHECK_HIP(hipMemcpyAsync(dord, order, nord * sizeof(int), hipMemcpyHostToDevice, s));
    train_steps(m, x, y, n_samples, batch, epochs, lr, dord, dloss);
    double last = 0.0;
    HHG_CHECK_HIP(hipMemcpyAsync(&last, dloss + (epochs - 1), sizeof(double), hipMemcpyDeviceToHost, s));
    HHG_CHECK_HIP(hipStreamSynchronize(s));
    HHG_CHECK_HIP(hipGetLastError());
    if (last_loss) *last_loss = last / (n_samples / batch);
  });
}

hhg_status hhg_mlp_dims(hhg_hier h, int* n_in, int* n_out) {
  return guard([&] {
    HHG_REQUIRE(h && n_in && n_out, HHG_ERR_ARG, "null argument");
    lattice_only(h, "the learned coarse solve");
    HHG_REQUIRE(h->nunk > 0, HHG_ERR_STATE, "no dense coarse solve on this hierarchy");
    *n_in = h->nunk + h->L(h->lmin).g.nn;
    *n_out = h->nunk;
  });
}

static void ensure_coarse_buffers(hhg_hier h) {
  if (!h->feat) {
    h->feat = h->arena.alloc<float>((size_t)h->nunk + h->L(h->lmin).g.nn);
    h->mlp_out = h->arena.alloc<float>(h->nunk);
    h->norm = h->arena.alloc<double>(2);
  }
}

hhg_status hhg_coarse_pair(hhg_hier h, const double* r, float* features, float* target) {
  return guard([&] {
    HHG_REQUIRE(h && r && features && target, HHG_ERR_ARG, "null argument");
    lattice_only(h, "the learned coarse solve");
    HHG_REQUIRE(h->nunk > 0, HHG_ERR_STATE, "no dense coarse solve on this hierarchy");
    ensure_coarse_buffers(h);
    Level& lv = h->L(h->lmin);
    HHG_REQUIRE(r != lv.r && r != lv.cx, HHG_ERR_ARG, "r must be a caller vector");
    launch_coarse_features(S(h), r, h->unk, h->nunk, lv.nu64, lv.g.nn, features, h->norm);
    double* c = lv.cx;
    launch_fill<double>(S(h), c, lv.vec_words, 0.0);
    op_coarse<double>(h, c, r, false);  // exact correction (plain coarse solve)
    launch_coarse_scatter(S(h), nullptr, h->unk, h->nunk, h->norm, c, target);
    HHG_CHECK_HIP(hipGetLastError());
  });
}

hhg_status hhg_hier_set_bf16_levels(hhg_hier h, int n) {
  return guard([&] {
    HHG_REQUIRE(h && n >= 0 && n <= h->lmax - h->lmin + 1, HHG_ERR_ARG, "bad number of levels");
    lattice_only(h, "bfloat16 levels");
    h->bf16_levels = n;
  });
}

hhg_status hhg_hier_set_fused_sites(hhg_hier h, long max_sites) {
  return guard([&] {
    HHG_REQUIRE(h && max_sites >= 0, HHG_ERR_ARG, "bad arguments");
    h->fused_sites = max_sites;
    h->ufused_slots = max_sites;
    if (h->fmg_exec) {  // a captured solve holds the old launch sequence
      HHG_CHECK_HIP(hipGraphExecDestroy(h->fmg_exec));
      h->fmg_exec = nullptr;
      h->fmg_key.clear();
    }
  });
}

hhg_status hhg_record_pairs(hhg_hier h, float* features, float* targets, int capacity) {
  return guard([&] {
    HHG_REQUIRE(h && capacity >= 0, HHG_ERR_ARG, "bad arguments");
    lattice_only(h, "the training-pair recorder");
    HHG_REQUIRE(capacity == 0 || (features && targets), HHG_ERR_ARG, "null buffers");
    HHG_REQUIRE(capacity == 0 || h->nunk > 0, HHG_ERR_STATE, "no dense coarse solve on this hierarchy");
    if (capacity > 0) {
      ensure_coarse_buffers(h);
      ensure_coarse(h);
    }
    if (capacity > 0 && !h->rc) h->rc = h->arena.alloc<double>(h->L(h->lmin).vec_words);
    h->rec_f = capacity ? features : nullptr;
    h->rec_t = capacity ? targets : nullptr;
    h->rec_cap = capacity;
    h->rec_n = 0;
  });
}

hhg_status hhg_recorded_pairs(hhg_hier h, int* count) {
  return guard([&] {
    HHG_REQUIRE(h && count, HHG_ERR_ARG, "null argument");
    *count = h->rec_n;
  });
}

hhg_status hhg_hier_set_mlp(hhg_hier h, hhg_mlp m, double rho_plain, double tau) {
  return guard([&] {
    HHG_REQUIRE(h, HHG_ERR_ARG, "null hierarchy");
    if (m) lattice_only(h, "the learned coarse solve");
    if (m) {
      HHG_REQUIRE(h->nunk > 0, HHG_ERR_STATE, "no dense coarse solve on this hierarchy");
      HHG_REQUIRE(m->net.n_in == h->nunk + h->L(h->lmin).g.nn && m->net.n_out == h->nunk, HHG_ERR_ARG,
                  "MLP sizes do not match the coarsest level");
      HHG_REQUIRE(rho_plain > 0.0 && tau >= -1.0, HHG_ERR_ARG, "bad monitor parameters");
      ensure_coarse_buffers(h);
    }
    h->mlp = m;
    h->rho_plain = rho_plain;
    h->tau = tau;
    h->mlp_off = false;
    if (h->fmg_exec) {
      HHG_CHECK_HIP(hipGraphExecDestroy(h->fmg_exec));
      h->fmg_exec = nullptr;
      h->fmg_key.clear();
    }
  });
}

hhg_status hhg_query_stencil(hhg_disc disc, char kind, int group, int i, int j, int k, int nbox, int max_entries,
                             int* n, int* code, double* w) {
  return guard([&] {
    HHG_REQUIRE(disc == HHG_P1P1 || disc == HHG_P2P1, HHG_ERR_ARG, "unknown discretisation");
    HHG_REQUIRE(n && code && w, HHG_ERR_ARG, "null output");
    HHG_REQUIRE(std::strchr("AMTBCP", kind) != nullptr && kind != 0, HHG_ERR_ARG, "unknown stencil kind");
    ElementSet es;
    build_elements(disc == HHG_P1P1 ? 1 : 2, &es);
    Row r = row_stencil(es, kind, group, i, j, k, nbox);
    *n = (int)r.size();
    HHG_REQUIRE((int)r.size() <= max_entries, HHG_ERR_ARG, "output too small");
    for (size_t e = 0; e < r.size(); ++e) {
      code[4 * e] = r[e].g, code[4 * e + 1] = r[e].di, code[4 * e + 2] = r[e].dj, code[4 * e + 3] = r[e].dk;
      for (int d = 0; d < 3; ++d) w[3 * e + d] = r[e].w[d];
    }
  });
}

hhg_status hhg_query_umesh(const double* xyz, int nv, const int* tet, int nt, unsigned cube_outflow, int level,
                           hhg_schur schur, int max_unknowns, int* nnodes, int* ncolours, int* nunk, double* pos,
                           int* colour, double* schur_diag, double* K) {
  return guard([&] {
    HHG_REQUIRE(xyz && tet, HHG_ERR_ARG, "null mesh");
    HHG_REQUIRE(schur == HHG_SCHUR_SD || schur == HHG_SCHUR_ML, HHG_ERR_ARG, "unknown Schur option");
    HHG_REQUIRE(cube_outflow < 64u, HHG_ERR_ARG, "outflow faces: a mask of faces 0..5");
    u_query(xyz, nv, tet, nt, cube_outflow, level, schur, max_unknowns, nnodes, ncolours, nunk, pos, colour,
            schur_diag, K);
  });
}

hhg_status hhg_query_interpolation(int order, int tx, int ty, int tz, int q, int* n, int* code, double* w) {
  return guard([&] {
    HHG_REQUIRE(order == 1 || order == 2, HHG_ERR_ARG, "order must be 1 or 2");
    HHG_REQUIRE(q >= 1 && tx >= 0 && ty >= 0 && tz >= 0 && tx <= q && ty <= q && tz <= q, HHG_ERR_ARG,
                "position outside the cube");
    HHG_REQUIRE(n && code && w, HHG_ERR_ARG, "null output");
    const double t[3] = {(double)tx / q, (double)ty / q, (double)tz / q};
    auto ws = interp_weights(order, t);
    *n = (int)ws.size();
    for (size_t e = 0; e < ws.size(); ++e) {
      code[4 * e] = std::get<0>(ws[e]);
      code[4 * e + 1] = std::get<1>(ws[e]);
      code[4 * e + 2] = std::get<2>(ws[e]);
      code[4 * e + 3] = std::get<3>(ws[e]);
      w[e] = std::get<4>(ws[e]);
    }
  });
}

hhg_status hhg_vcycle(hhg_hier h, int level, void* x, const void* b, const hhg_solver_params* prm, hhg_prec prec) {
  return guard([&] {
    check_level(h, level);
    HHG_REQUIRE(x && b && prm && prm->omega_inv > 0.0 && prm->xi >= 1, HHG_ERR_ARG, "bad arguments");
    HHG_REQUIRE(prec == HHG_F64 || prec == HHG_F32, HHG_ERR_PREC, "bad precision");
    HHG_REQUIRE(!h->um || prec == HHG_F64, HHG_ERR_PREC, "unstructured macro meshes: float64 only");
    ensure_coarse(h);
    if (prec == HHG_F32) {
      HHG_REQUIRE(h->nunk > 0 || prm->coarse_smooth > 0, HHG_ERR_STATE, "no dense coarse solve on this hierarchy");
      ensure_f32_vectors(h);
      refresh_small(h);
      vcycle_t<float>(h, level, level, (float*)x, (const float*)b, *prm);
    } else {
      refresh_small(h);
      vcycle(h, level, level, (double*)x, (const double*)b, *prm);
    }
    HHG_CHECK_HIP(hipGetLastError());
  });
}

hhg_status hhg_fmg_solve(hhg_hier h, void* xv, const void* const* b_levels, const hhg_solver_params* prm,
                         hhg_stats* stats) {
  hhg_status st = guard([&] {
    HHG_REQUIRE(h && xv && b_levels && prm, HHG_ERR_ARG, "null argument");
    HHG_REQUIRE(prm->omega_inv > 0.0 && prm->xi >= 1 && prm->kappa >= 1, HHG_ERR_ARG, "bad solver parameters");
    HHG_REQUIRE(prm->nu_pre >= 0 && prm->nu_post >= 0 && prm->nu_inc >= 0 && prm->extra_cycles >= 0, HHG_ERR_ARG,
                "bad solver parameters");
    for (int l = h->lmin; l <= h->lmax; ++l) HHG_REQUIRE(b_levels[l - h->lmin], HHG_ERR_ARG, "null rhs");
    HHG_REQUIRE(h->nunk > 0 || prm->coarse_smooth > 0, HHG_ERR_STATE, "no dense coarse solve on this hierarchy");
    HHG_REQUIRE(prm->coarse_smooth >= 0, HHG_ERR_ARG, "bad solver parameters");
    const hhg_solver_params& p = *prm;
    double* x = (double*)xv;
    auto bl = [&](int l) { return (const double*)b_levels[l - h->lmin]; };
    if (!(h->mlp && h->kp_stale)) ensure_coarse(h);
    refresh_small(h);
    // Fixed work (no stopping test, no statistics): the whole solve is one
    // replayed HIP graph, captured on the first call with these vectors and
    // parameters.  The event timer needs per-launch events, so it runs eagerly.
    const bool fixed = stats == nullptr && p.rtol <= 0.0 && !timer_enabled() && h->rec_cap == 0;
    if (fixed && h->kp_stale && !h->mlp && p.coarse_smooth == 0) {  // no host work inside a capture
      build_coarse_device(h);
      h->kp_stale = false;
    }
    if (fixed) {
      std::vector<unsigned char> key(sizeof(hhg_solver_params) + sizeof(void*) * (h->lmax - h->lmin + 2));
      std::memcpy(key.data(), &p, sizeof p);
      std::memcpy(key.data() + sizeof p, &xv, sizeof(void*));
      for (int l = h->lmin; l <= h->lmax; ++l)
        std::memcpy(key.data() + sizeof p + sizeof(void*) * (l - h->lmin + 1), &b_levels[l - h->lmin], sizeof(void*));
      if (!(h->fmg_exec && key == h->fmg_key)) {
        if (h->fmg_exec) {
          HHG_CHECK_HIP(hipGraphExecDestroy(h->fmg_exec));
          h->fmg_exec = nullptr;
        }
        hhg_ctx c = h->ctx;
        if (!c->capture) HHG_CHECK_HIP(hipStreamCreateWithFlags(&c->capture, hipStreamNonBlocking));
        hipStream_t user = c->stream;
        c->stream = c->capture;
        hipGraph_t graph = nullptr;
        HHG_CHECK_HIP(hipStreamBeginCapture(c->capture, hipStreamCaptureModeThreadLocal));
        try {
          fmg_body(h, x, bl, p);
        } catch (...) {
          (void)hipStreamEndCapture(c->capture, &graph);
          if (graph) (void)hipGraphDestroy(graph);
          c->stream = user;
          throw;
        }
        HHG_CHECK_HIP(hipStreamEndCapture(c->capture, &graph));
        c->stream = user;
        hipError_t e = hipGraphInstantiate(&h->fmg_exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        HHG_CHECK_HIP(e);
        h->fmg_key = key;
      }
      HHG_CHECK_HIP(hipGraphLaunch(h->fmg_exec, S(h)));
      return;
    }
    CallClock clock(h);
    fmg_body(h, x, bl, p);
    Level& top = h->L(h->lmax);
    int cycles = p.kappa + (p.rtol > 0.0 ? 0 : p.extra_cycles);
    int fallbacks = 0;
    double bu = 0, bp = 0, ru = 0, rp = 0;
    const double* b = bl(h->lmax);
    norms<double>(h, h->lmax, b, &bu, &bp);
    const double bn = std::sqrt(bu * bu + bp * bp);
    // Fallback monitor: with the learned coarse solve, a cycle whose residual
    // reduction is worse than rho_plain (1 + tau) (or not finite) is undone and
    // the rest of the solve uses the plain coarse solve.
    const bool monitor = h->mlp && p.rtol > 0.0;
    if (monitor && !h->bk) h->bk = h->arena.alloc<double>(top.vec_words);
    double prev = -1.0;
    for (;;) {
      op_apply<double>(h, h->lmax, full_mask(h), x, b, top.r, true, true, true);
      norms<double>(h, h->lmax, top.r, &ru, &rp);
      const double rn = std::sqrt(ru * ru + rp * rp);
      if (monitor && !h->mlp_off &&
          (!std::isfinite(rn) || (prev > 0.0 && rn > h->rho_plain * (1.0 + h->tau) * prev))) {
        h->mlp_off = true;
        ++fallbacks;
        if (prev > 0.0) {  // undo the last cycle
          HHG_CHECK_HIP(hipMemcpyAsync(x, h->bk, top.vec_words * sizeof(double), hipMemcpyDeviceToDevice, S(h)));
        } else {           // the FMG start itself is unusable: redo it with the exact coarse solve
          fmg_body(h, x, bl, p);
        }
        continue;
      }
      if (p.rtol <= 0.0 || rn <= p.rtol * bn || cycles >= p.max_cycles) break;
      if (monitor && !h->mlp_off)
        HHG_CHECK_HIP(hipMemcpyAsync(h->bk, x, top.vec_words * sizeof(double), hipMemcpyDeviceToDevice, S(h)));
      prev = rn;
      vcycle(h, h->lmax, h->lmax, x, b, p);
      op_mean_zero<double>(h, h->lmax, x);
      ++cycles;
    }
    h->mlp_off = false;
    HHG_CHECK_HIP(hipGetLastError());
    if (stats) {
      stats->cycles = cycles;
      stats->res_u = ru;
      stats->res_p = rp;
      stats->rel_res = bn > 0 ? std::sqrt(ru * ru + rp * rp) / bn : 0.0;
      stats->work_units = fmg_work_units(h, p) + (cycles - p.kappa) * vcycle_work_units(h, p);
      stats->seconds = clock.seconds();
      stats->fallbacks = fallbacks;
    }
    if (p.rtol > 0.0 && std::sqrt(ru * ru + rp * rp) > p.rtol * bn)
      throw Error{HHG_ERR_NOT_CONVERGED, "relative residual above rtol after max_cycles"};
  });
  return st;
}

}  // extern "C"
