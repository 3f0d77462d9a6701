// Build-time generator of the interior stencil code (host program).
//
// Paper Sec. 2.1: with constant coefficients the stencil of a row is the same
// at every inner node of a macro-primitive.  On the Kuhn-cube hierarchy the
// inner rows of every level share one stencil per row type up to a power of
// h, so their weights (at h = 1, from the element matrices of fe_host.cpp)
// are emitted as literals into fully unrolled device functions; kernels scale
// the sums by h, h^2 or h^3.  Usage: gen_stencils <output file>.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <string>
#include <vector>

#include "fe.h"

using namespace hhg;

namespace {

Row pruned(const ElementSet& es, char kind, int g, int nw) {
  Row r = row_stencil(es, kind, g, 3, 3, 3, 7);
  double mx = 0.0;
  for (auto& e : r)
    for (int d = 0; d < nw; ++d) mx = std::max(mx, std::fabs(e.w[d]));
  Row out;
  for (auto& e : r) {
    bool keep = false;
    for (int d = 0; d < nw; ++d) keep |= std::fabs(e.w[d]) > 1e-13 * mx;
    if (keep) out.push_back(e);
  }
  std::sort(out.begin(), out.end(), [](const Entry& a, const Entry& b) {
    if (a.dk != b.dk) return a.dk < b.dk;
    if (a.dj != b.dj) return a.dj < b.dj;
    if (a.g != b.g) return a.g < b.g;
    return a.di < b.di;
  });
  return out;
}

std::string off_expr(const Entry& e, int row_group, bool group_shift) {
  char buf[160];
  const int gs = group_shift ? e.g - row_group : 0;
  std::snprintf(buf, sizeof buf, "(%d) * nn + (%d) + (%d) * s1 + (%d) * s2", gs, e.di, e.dj, e.dk);
  return buf;
}

std::string lit(double w) {
  char buf[64];
  std::snprintf(buf, sizeof buf, "%.17g", w);
  return buf;
}

// velocity row -> velocity columns, three components with one weight
void emit_vv(FILE* f, const char* name, const Row& r, int g) {
  std::fprintf(f,
               "template <typename T>\n__device__ __forceinline__ void %s(const T* __restrict__ u0, const T* "
               "__restrict__ u1, const T* __restrict__ u2, int pos, int s1, int s2, int nn, T& a0, T& a1, T& a2) {\n",
               name);
  for (auto& e : r)
    std::fprintf(f, "  { const int o = pos + %s; const T w = T(%s); a0 += w * u0[o]; a1 += w * u1[o]; a2 += w * u2[o]; }\n",
                 off_expr(e, g, true).c_str(), lit(e.w[0]).c_str());
  std::fprintf(f, "}\n// %zu entries\n\n", r.size());
}

// velocity row -> pressure columns, three weights
void emit_vp(FILE* f, const char* name, const Row& r) {
  std::fprintf(f,
               "template <typename T>\n__device__ __forceinline__ void %s(const T* __restrict__ p, int pos, int s1, "
               "int s2, T& a0, T& a1, T& a2) {\n  const int nn = 0;\n",
               name);
  for (auto& e : r)
    std::fprintf(f, "  { const T v = p[pos + %s]; a0 += T(%s) * v; a1 += T(%s) * v; a2 += T(%s) * v; }\n",
                 off_expr(e, 0, false).c_str(), lit(e.w[0]).c_str(), lit(e.w[1]).c_str(), lit(e.w[2]).c_str());
  std::fprintf(f, "  (void)nn;\n}\n// %zu entries\n\n", r.size());
}

// pressure row -> velocity columns (three weights, one sum)
void emit_pv(FILE* f, const char* name, const Row& r) {
  std::fprintf(f,
               "template <typename T>\n__device__ __forceinline__ void %s(const T* __restrict__ u0, const T* "
               "__restrict__ u1, const T* __restrict__ u2, int pos, int s1, int s2, int nn, T& a) {\n",
               name);
  for (auto& e : r) {
    std::string o = "pos + " + off_expr(e, 0, true);
    std::fprintf(f, "  { const int o = %s;", o.c_str());
    const char* c[3] = {"u0", "u1", "u2"};
    for (int d = 0; d < 3; ++d)
      if (e.w[d] != 0.0) std::fprintf(f, " a += T(%s) * %s[o];", lit(e.w[d]).c_str(), c[d]);
    std::fprintf(f, " }\n");
  }
  std::fprintf(f, "}\n// %zu entries\n\n", r.size());
}

// pressure row -> pressure columns
void emit_pp(FILE* f, const char* name, const Row& r) {
  std::fprintf(f,
               "template <typename T>\n__device__ __forceinline__ void %s(const T* __restrict__ p, int pos, int s1, "
               "int s2, T& a) {\n  const int nn = 0;\n",
               name);
  for (auto& e : r)
    std::fprintf(f, "  a += T(%s) * p[pos + %s];\n", lit(e.w[0]).c_str(), off_expr(e, 0, false).c_str());
  std::fprintf(f, "  (void)nn;\n}\n// %zu entries\n\n", r.size());
}

// Variable viscosity (A weighted by nu_T = mean of nu at the element's four
// vertices): the row of velocity group g at index (i,j,k) summed element by
// element over the lattice elements containing it.  nu is read at P1 indices
// relative to idx = i + s1 j + s2 k; u at group arrays relative to pos.
struct ElemRow {
  int vo[4][3];                 // element vertices, P1 offsets from (i,j,k)
  std::vector<Entry> cols;      // element-local row: column (group, offset), weight
  double diag;                  // K[a][a]
};

std::vector<ElemRow> element_rows(const ElementSet& es, int g) {
  const int kDir[8][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {1, 1, 0}, {1, 0, 1}, {0, 1, 1}, {1, 1, 1}};
  const int vs = es.vorder;
  const int i = 3, j = 3, k = 3;
  int rpos[3];
  for (int d = 0; d < 3; ++d) rpos[d] = vs == 1 ? 3 : 2 * 3 + kDir[g][d];
  std::vector<ElemRow> out;
  for (int ck = k - 1; ck <= k + 1; ++ck)
    for (int cj = j - 1; cj <= j + 1; ++cj)
      for (int ci = i - 1; ci <= i + 1; ++ci)
        for (int t = 0; t < 6; ++t) {
          const int org[3] = {ci, cj, ck};
          int a = -1;
          for (int q = 0; q < es.nloc; ++q) {
            bool m = true;
            for (int d = 0; d < 3; ++d) m &= org[d] * vs + es.vpos[t][q][d] == rpos[d];
            if (m) a = q;
          }
          if (a < 0) continue;
          ElemRow er;
          for (int v = 0; v < 4; ++v)
            for (int d = 0; d < 3; ++d) er.vo[v][d] = org[d] + es.ppos[t][v][d] - (d == 0 ? i : d == 1 ? j : k);
          er.diag = es.K[t][a][a];
          for (int b = 0; b < es.nloc; ++b) {
            if (es.K[t][a][b] == 0.0) continue;
            Entry e{};
            int sp[3];
            for (int d = 0; d < 3; ++d) sp[d] = org[d] * vs + es.vpos[t][b][d];
            if (vs == 1) {
              e.g = 0;
              e.di = sp[0] - i, e.dj = sp[1] - j, e.dk = sp[2] - k;
            } else {
              int par[3] = {sp[0] & 1, sp[1] & 1, sp[2] & 1};
              for (int q = 0; q < 8; ++q)
                if (kDir[q][0] == par[0] && kDir[q][1] == par[1] && kDir[q][2] == par[2]) e.g = q;
              e.di = (sp[0] >> 1) - i, e.dj = (sp[1] >> 1) - j, e.dk = (sp[2] >> 1) - k;
            }
            e.w[0] = es.K[t][a][b];
            er.cols.push_back(e);
          }
          out.push_back(er);
        }
  return out;
}

void emit_anu(FILE* f, const char* name, const std::vector<ElemRow>& rows, int g) {
  std::fprintf(f,
               "template <typename T>\n__device__ __forceinline__ void %s(const T* __restrict__ u0, const T* "
               "__restrict__ u1, const T* __restrict__ u2, const T* __restrict__ nu, int pos, int idx, int s1, int s2, "
               "int nn, T& a0, T& a1, T& a2) {\n",
               name);
  for (auto& er : rows) {
    std::fprintf(f, "  {\n    const T nt = T(0.25) * (");
    for (int v = 0; v < 4; ++v)
      std::fprintf(f, "%snu[idx + (%d) + (%d) * s1 + (%d) * s2]", v ? " + " : "", er.vo[v][0], er.vo[v][1],
                   er.vo[v][2]);
    std::fprintf(f, ");\n    T b0 = 0, b1 = 0, b2 = 0;\n");
    for (auto& e : er.cols)
      std::fprintf(f, "    { const int o = pos + %s; const T w = T(%s); b0 += w * u0[o]; b1 += w * u1[o]; b2 += w * u2[o]; }\n",
                   off_expr(e, g, true).c_str(), lit(e.w[0]).c_str());
    std::fprintf(f, "    a0 += nt * b0; a1 += nt * b1; a2 += nt * b2;\n  }\n");
  }
  std::fprintf(f, "}\n// %zu elements\n\n", rows.size());
}

void emit_anu_diag(FILE* f, const char* name, const std::vector<ElemRow>& rows) {
  std::fprintf(f,
               "template <typename T>\n__device__ __forceinline__ T %s(const T* __restrict__ nu, int idx, int s1, int s2) "
               "{\n  T d = 0;\n",
               name);
  for (auto& er : rows) {
    std::fprintf(f, "  d += T(%s) * T(0.25) * (", lit(er.diag).c_str());
    for (int v = 0; v < 4; ++v)
      std::fprintf(f, "%snu[idx + (%d) + (%d) * s1 + (%d) * s2]", v ? " + " : "", er.vo[v][0], er.vo[v][1],
                   er.vo[v][2]);
    std::fprintf(f, ");\n");
  }
  std::fprintf(f, "  return d;\n}\n\n");
}

// k-marching form of the constant-coefficient operator calA (A, B^T, B and
// -C together) for one velocity component d and one loaded k-plane of the
// input.  A wavefront owns 64 consecutive lattice columns (i, j) and walks k;
// for every (array, dj) that component d's rows need it loads the word of
// column (i, j + dj) once -- the i -+ 1 neighbours come from the adjacent
// lanes (from_prev / from_next, wavefront lane shifts) -- and scatters it
// into the rows of the lane's own column at k = kp - dk, kept in three
// rotating accumulator planes (slot = relative plane index mod 3; Q =
// relative index of the loaded plane mod 3).  Loads are buffer loads: ru
// addresses velocity component d (group c at byte offset c nnb), rp the
// pressure; vo[dj + 1] is the byte offset of column (i, j + dj) in plane kp,
// which the caller clamps into the lattice, and the caller discards the first
// and last lane of the wavefront (their shifted neighbours are missing).  A clamped or wrapped
// word only reaches rows that are not interior -- an interior row references
// positions inside the cube only -- and those rows are written as zero.
// Accumulator row g < G: velocity row of component d, group g; row G: the
// part of the pressure row that comes from u_d (and, for d = 0, from -C p).
// Every weight at h = 1 is a rational k / den with a small integer k and one
// denominator per block (A, B^T, B, C; {D}_zm_den), so the code multiplies by
// the integer k -- an f64 literal with a zero low word, which needs no scalar
// register -- and the denominators and the h scales sa, sb, sc are applied
// once: velocity rows are in units of sa / den_A and pressure rows in units
// of sb / den_B (the caller scales them when it writes), and each loaded
// pressure word is pre-scaled once, by rt = sb den_A / (sa den_T) for the
// B^T entries, by rc = sc den_B / (sb den_C) for the C entries.
struct ZmUse {
  int row, dk;
  double w;
  int kind;  // 0: A, 1: B^T or B (by the array), 2: C (negated weight)
};
// Smallest denominator (<= 10^4) that makes every weight an integer to
// rounding; generation fails if there is none.
int common_den(const std::vector<double>& ws) {
  for (int den = 1; den <= 10000; ++den) {
    bool ok = true;
    for (double w : ws) ok = ok && std::fabs(w * den - std::nearbyint(w * den)) <= 1e-9 * std::max(1.0, std::fabs(w * den));
    if (ok) return den;
  }
  std::fprintf(stderr, "gen_stencils: zm weights are not small rationals\n");
  std::exit(1);
}
void emit_zm(FILE* f, const ElementSet& es, const char* D, int G) {
  auto slot = [](int Q, int dk) { return ((Q - dk) % 3 + 3) % 3; };
  // denominators per block, over all components
  std::vector<double> wa, wt, wb, wc;
  for (int r = 0; r < G; ++r) {
    for (auto& e : pruned(es, 'A', r, 1)) wa.push_back(e.w[0]);
    for (auto& e : pruned(es, 'T', r, 3))
      for (int d = 0; d < 3; ++d) wt.push_back(e.w[d]);
  }
  for (auto& e : pruned(es, 'B', 0, 3))
    for (int d = 0; d < 3; ++d) wb.push_back(e.w[d]);
  if (G == 1)
    for (auto& e : pruned(es, 'C', 0, 1)) wc.push_back(e.w[0]);
  const int den[4] = {common_den(wa), common_den(wt), common_den(wb), wc.empty() ? 1 : common_den(wc)};
  std::fprintf(f, "// denominators of the k-marching weights: A, B^T, B, C\nconstexpr int %s_zm_den[4] = {%d, %d, %d, %d};\n\n",
               D, den[0], den[1], den[2], den[3]);
  auto kw = [&](const ZmUse& u, int a) {
    const int dn = u.kind == 0 ? den[0] : (u.kind == 2 ? den[3] : (a == G ? den[1] : den[2]));
    return lit(std::nearbyint(u.w * dn));
  };
  for (int d = 0; d < 3; ++d) {
    // array a (velocity group c: a = c; pressure: a = G), dj + 1, di + 1 -> uses
    std::vector<std::vector<ZmUse>> use((G + 1) * 9);
    auto at = [&](int a, int di, int dj) -> std::vector<ZmUse>& { return use[a * 9 + (dj + 1) * 3 + (di + 1)]; };
    for (int r = 0; r < G; ++r) {
      for (auto& e : pruned(es, 'A', r, 1)) at(e.g, e.di, e.dj).push_back({r, e.dk, e.w[0], 0});
      for (auto& e : pruned(es, 'T', r, 3))
        if (e.w[d] != 0.0) at(G, e.di, e.dj).push_back({r, e.dk, e.w[d], 1});
    }
    for (auto& e : pruned(es, 'B', 0, 3))
      if (e.w[d] != 0.0) at(e.g, e.di, e.dj).push_back({G, e.dk, e.w[d], 1});
    if (G == 1 && d == 0)
      for (auto& e : pruned(es, 'C', 0, 1)) at(G, e.di, e.dj).push_back({G, e.dk, -e.w[0], 2});
    for (int Q = 0; Q < 3; ++Q) {
      std::fprintf(f,
                   "template <typename T>\n__device__ __forceinline__ void %s_zm%d_q%d(__amdgpu_buffer_rsrc_t ru, "
                   "__amdgpu_buffer_rsrc_t rp, const int (&vo)[3], int nnb, T rt, T rc, T (&acc)[3][%d]) {\n"
                   "  (void)rc; (void)nnb;\n",
                   D, d, Q, G + 1);
      // all loads of the plane first, then the words one by one in a fixed
      // order (zm_order / zm_word): a word's lane-shifted copies die before
      // the next word's are made
      int nload = 0;
      for (int a = 0; a <= G; ++a)
        for (int dj = -1; dj <= 1; ++dj) {
          bool any = false;
          for (int di = -1; di <= 1; ++di) any |= !at(a, di, dj).empty();
          if (!any) continue;
          if (a < G)
            std::fprintf(f, "  const T l%d = buffer_word<T>(ru, vo[%d], %d * nnb);\n", nload, dj + 1, a);
          else
            std::fprintf(f, "  const T l%d = buffer_word<T>(rp, vo[%d], 0);\n", nload, dj + 1);
          ++nload;
        }
      int iw = 0;
      for (int a = 0; a <= G; ++a)
        for (int dj = -1; dj <= 1; ++dj) {
          bool any = false;
          for (int di = -1; di <= 1; ++di) any |= !at(a, di, dj).empty();
          if (!any) continue;
          // pressure words: one scaled copy per kind that uses them
          bool kinds[3] = {false, false, false};
          for (int di = -1; di <= 1; ++di)
            for (auto& u : at(a, di, dj)) kinds[u.kind] = true;
          std::fprintf(f, "  zm_order(acc);\n");
          if (a < G) {
            std::fprintf(f, "  { const T v0 = zm_word(l%d);\n", iw);
          } else {
            std::fprintf(f, "  { const T w0 = zm_word(l%d);\n", iw);
            if (kinds[1]) std::fprintf(f, "    const T v0 = rt * w0;\n");
            if (kinds[2]) std::fprintf(f, "    const T c0 = rc * w0;\n");
          }
          ++iw;
          for (int di = -1; di <= 1; ++di) {
            const auto& us = at(a, di, dj);
            if (us.empty()) continue;
            const char* sh = di == -1 ? "from_prev" : (di == 1 ? "from_next" : "");
            std::fprintf(f, "    {\n");
            if (a < G || kinds[1]) std::fprintf(f, "      const T v = %s(v0);\n", sh);
            if (a == G && kinds[2]) std::fprintf(f, "      const T c = %s(c0);\n", sh);
            for (auto& u : us)
              std::fprintf(f, "      acc[%d][%d] = fma(T(%s), %s, acc[%d][%d]);\n", slot(Q, u.dk), u.row, kw(u, a).c_str(),
                           u.kind == 2 ? "c" : "v", slot(Q, u.dk), u.row);
            std::fprintf(f, "    }\n");
          }
          std::fprintf(f, "  }\n");
        }
      std::fprintf(f, "}\n// %d loads per plane\n\n", nload);
    }
  }
}

// Pressure rows at boundary nodes, one function per boundary class (cls =
// c_i + 3 c_j + 9 c_k, c = 0 low face, 1 inside, 2 high face; 13 is the
// interior): the row summed over the lattice elements inside the cube only,
// taken at a representative node of the class in a box of 4 intervals.
Row pruned_at(const ElementSet& es, char kind, int ci, int cj, int ck, int nw) {
  Row r = row_stencil(es, kind, 0, ci, cj, ck, 4);
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
}
// One velocity component's part of a boundary-class pressure row.
void emit_pv_comp(FILE* f, const char* name, const Row& r, int d) {
  std::fprintf(f,
               "template <typename T>\n__device__ __forceinline__ void %s(const T* __restrict__ ud, int pos, int s1, "
               "int s2, int nn, T& a) {\n",
               name);
  size_t n = 0;
  for (auto& e : r) {
    if (e.w[d] == 0.0) continue;
    std::string o = "pos + " + off_expr(e, 0, true);
    std::fprintf(f, "  a += T(%s) * ud[%s];\n", lit(e.w[d]).c_str(), o.c_str());
    ++n;
  }
  std::fprintf(f, "}\n// %zu entries\n\n", n);
}

void emit_boundary_rows(FILE* f, const ElementSet& es, const char* D, int G) {
  const int rep[3] = {0, 2, 4};
  for (int cls = 0; cls < 27; ++cls) {
    if (cls == 13) continue;
    const int ci = rep[cls % 3], cj = rep[(cls / 3) % 3], ck = rep[cls / 9];
    char name[64];
    std::snprintf(name, sizeof name, "%s_Bc%d", D, cls);
    const Row brow = pruned_at(es, 'B', ci, cj, ck, 3);
    emit_pv(f, name, brow);
    for (int d = 0; d < 3; ++d) {
      std::snprintf(name, sizeof name, "%s_Bc%d_d%d", D, cls, d);
      emit_pv_comp(f, name, brow, d);
    }
    if (G == 1) {
      std::snprintf(name, sizeof name, "%s_Cc%d", D, cls);
      emit_pp(f, name, pruned_at(es, 'C', ci, cj, ck, 1));
    }
  }
}

// Restriction (transpose of the interpolation) gathered at coarse index
// (i, j, k): per coarse velocity group the three components from the fine
// residual around fine index fb = 2 (i, j, k) (fine strides s1, s2, group
// stride nn, component stride vs); and the P1 pressure with every entry
// clipped to the fine lattice [0, Nf]^3.
void emit_restriction(FILE* f, const char* D, int vorder) {
  std::vector<std::vector<RestrictEntry>> vel;
  std::vector<RestrictEntry> pres;
  restriction_entries(vorder, vel, pres);
  for (size_t gc = 0; gc < vel.size(); ++gc) {
    std::fprintf(f,
                 "template <typename T>\n__device__ __forceinline__ void %s_R_g%zu(const T* __restrict__ rf, int fb, int "
                 "s1, int s2, int nn, int vs, T& a0, T& a1, T& a2) {\n",
                 D, gc);
    for (auto& e : vel[gc])
      std::fprintf(f,
                   "  { const int o = fb + (%d) * nn + (%d) + (%d) * s1 + (%d) * s2; const T w = T(%s); a0 += w * rf[o]; "
                   "a1 += w * rf[vs + o]; a2 += w * rf[2 * vs + o]; }\n",
                   e.g, e.di, e.dj, e.dk, lit(e.w).c_str());
    std::fprintf(f, "}\n// %zu entries\n\n", vel[gc].size());
  }
  std::fprintf(f,
               "template <typename T>\n__device__ __forceinline__ T %s_RP(const T* __restrict__ p, int fb, int fi, int fj, "
               "int fk, int Nf, int s1, int s2) {\n  T a = 0;\n",
               D);
  // Entries outside the fine lattice drop out.  Each word is read at its
  // position clamped into the lattice (always a valid address) and the entry's
  // weight is zeroed when the position was outside: the loads carry no branch,
  // so they issue as one batch instead of one round trip each.
  for (auto& e : pres)
    std::fprintf(f,
                 "  { const int ci = min(max(fi + (%d), 0), Nf), cj = min(max(fj + (%d), 0), Nf), "
                 "ck = min(max(fk + (%d), 0), Nf);\n"
                 "    const T v = p[fb + (ci - fi) + (cj - fj) * s1 + (ck - fk) * s2];\n"
                 "    a += (ci == fi + (%d) && cj == fj + (%d) && ck == fk + (%d) ? T(%s) : T(0)) * v; }\n",
                 e.di, e.dj, e.dk, e.di, e.dj, e.dk, lit(e.w).c_str());
  std::fprintf(f, "  return a;\n}\n// %zu entries\n\n", pres.size());
}

// k-marching velocity restriction (P2-P1): a wavefront owns 64 consecutive
// coarse columns (i, j) of one component and walks the coarse planes; step q
// (coarse plane kq) loads the fine planes 2 kq (P = 0) and 2 kq + 1 (P = 1).
// A lane holds the fine words at 2 i (even) and 2 i + 1 (odd) of every fine
// row 2 j + dj (dj = -2 .. 1) and fine group the plane's entries use; the
// offsets di = -1, -2 are the previous lane's odd and even words.  An entry
// (coarse group gc, fine group g, di, dj, dk) of a plane of parity P = dk mod
// 2 adds to coarse plane kq (dk >= 0, accumulator slot Q) or kq + 1 (dk < 0,
// slot 1 - Q).  ro_e / ro_o: byte offsets of the even / odd word of fine row
// dj + 2 in the plane, group g at soffset g nnb.
void emit_restriction_zm(FILE* f, const char* D, int vorder) {
  std::vector<std::vector<RestrictEntry>> vel;
  std::vector<RestrictEntry> pres;
  restriction_entries(vorder, vel, pres);
  const int G = (int)vel.size();
  for (int P = 0; P < 2; ++P)
    for (int Q = 0; Q < 2; ++Q) {
      std::fprintf(f,
                   "template <typename T>\n__device__ __forceinline__ void %s_Rzm_p%d_q%d(__amdgpu_buffer_rsrc_t ru, "
                   "const int (&ro_e)[4], const int (&ro_o)[4], int nnb, T (&acc)[2][%d]) {\n",
                   D, P, Q, G);
      // the (fine group, row) pairs this plane parity uses, in a fixed order
      std::vector<std::pair<int, int>> pairs;
      for (int g = 0; g < 8; ++g)
        for (int dj = -2; dj <= 1; ++dj) {
          bool any = false;
          for (int gc = 0; gc < G; ++gc)
            for (auto& e : vel[gc]) any |= e.g == g && e.dj == dj && (((e.dk % 2) + 2) % 2) == P;
          if (any) pairs.push_back({g, dj});
        }
      for (size_t w = 0; w < pairs.size(); ++w)
        std::fprintf(f,
                     "  const T e%zu = buffer_word<T>(ru, ro_e[%d], %d * nnb);\n"
                     "  const T o%zu = buffer_word<T>(ru, ro_o[%d], %d * nnb);\n",
                     w, pairs[w].second + 2, pairs[w].first, w, pairs[w].second + 2, pairs[w].first);
      for (size_t w = 0; w < pairs.size(); ++w) {
        const int g = pairs[w].first, dj = pairs[w].second;
        bool need[4] = {false, false, false, false};  // di + 2
        for (int gc = 0; gc < G; ++gc)
          for (auto& e : vel[gc])
            if (e.g == g && e.dj == dj && (((e.dk % 2) + 2) % 2) == P) need[e.di + 2] = true;
        std::fprintf(f, "  {\n");
        if (need[0]) std::fprintf(f, "    const T m2 = from_prev(e%zu);\n", w);
        if (need[1]) std::fprintf(f, "    const T m1 = from_prev(o%zu);\n", w);
        for (int gc = 0; gc < G; ++gc)
          for (auto& e : vel[gc]) {
            if (!(e.g == g && e.dj == dj && (((e.dk % 2) + 2) % 2) == P)) continue;
            const char* word = e.di == -2 ? "m2" : (e.di == -1 ? "m1" : nullptr);
            char buf[32];
            if (!word) {
              std::snprintf(buf, sizeof buf, "%c%zu", e.di == 0 ? 'e' : 'o', w);
              word = buf;
            }
            const int slot = e.dk >= 0 ? Q : 1 - Q;
            std::fprintf(f, "    acc[%d][%d] = fma(T(%s), %s, acc[%d][%d]);\n", slot, gc, lit(e.w).c_str(), word, slot,
                         gc);
          }
        std::fprintf(f, "  }\n");
      }
      std::fprintf(f, "}\n// %zu word pairs per plane\n\n", pairs.size());
    }
}

// Interpolation by coarse cubes: the coarse element functions of cube (i, j,
// k) at its fine sites 2 (i, j, k) + (pi, pj, pk) of fine group g.  c holds
// the coarse words at the doubled positions (a, b, c) in {0, 1, 2}^3 of the
// cube, index a + 3 b + 9 c (coarse group of parity (a & 1, b & 1, c & 1) at
// coarse index (i, j, k) + (a, b, c) / 2; P1 uses the corners a, b, c in {0,
// 2} only); v[pi + 2 pj + 4 pk] receives the eight values.
void emit_prolongation_cube(FILE* f, const char* D, int vorder) {
  const int G = vorder == 1 ? 1 : 8;
  const int vq = vorder == 1 ? 2 : 4;  // fine positions per coarse cube edge
  int dir[8][3] = {};  // parity of each group
  for (int p = 0; p < 8; ++p) {
    const int g = group_of_parity(p & 1, (p >> 1) & 1, p >> 2);
    for (int d = 0; d < 3; ++d) dir[g][d] = (p >> d) & 1;
  }
  for (int g = 0; g < G; ++g) {
    std::fprintf(f, "template <typename T>\n__device__ __forceinline__ void %s_Pc_g%d(const T (&c)[27], T (&v)[8]) {\n",
                 D, g);
    for (int p = 0; p < 8; ++p) {
      double t[3];
      for (int d = 0; d < 3; ++d) {
        const int par = (p >> d) & 1;
        t[d] = (double)(vorder == 2 ? 2 * par + dir[g][d] : par) / vq;
      }
      std::string sum;
      for (auto& w : interp_weights(vorder, t)) {
        const int gc = std::get<0>(w);
        const int o[3] = {std::get<1>(w), std::get<2>(w), std::get<3>(w)};
        int idx = 0, mul = 1;
        for (int d = 0; d < 3; ++d, mul *= 3) idx += mul * (2 * o[d] + (vorder == 2 ? dir[gc][d] : 0));
        if (!sum.empty()) sum += " + ";
        sum += "T(" + lit(std::get<4>(w)) + ") * c[" + std::to_string(idx) + "]";
      }
      std::fprintf(f, "  v[%d] = %s;\n", p, sum.empty() ? "T(0)" : sum.c_str());
    }
    std::fprintf(f, "}\n");
  }
  std::fprintf(f, "template <typename T>\n__device__ __forceinline__ void %s_Pc(int g, const T (&c)[27], T (&v)[8]) {\n",
               D);
  if (G == 1) {
    std::fprintf(f, "  (void)g;\n  %s_Pc_g0(c, v);\n}\n\n", D);
    return;
  }
  std::fprintf(f, "  switch (g) {\n");
  for (int g = 0; g < G; ++g) std::fprintf(f, "    case %d: %s_Pc_g%d(c, v); break;\n", g, D, g);
  std::fprintf(f, "    default: break;\n  }\n}\n\n");
}

double diag_of(const Row& r, int g) {
  for (auto& e : r)
    if (e.g == g && e.di == 0 && e.dj == 0 && e.dk == 0) return e.w[0];
  return 0.0;
}

}  // namespace

int main(int argc, char** argv) {
  if (argc < 2) {
    std::fprintf(stderr, "usage: gen_stencils <output>\n");
    return 2;
  }
  FILE* f = std::fopen(argv[1], "w");
  if (!f) return 1;
  std::fprintf(f,
               "// Generated by gen_stencils.cpp from the element matrices of the six Kuhn tetrahedra.\n"
               "// Interior row stencils at h = 1; do not edit.\n#pragma once\nnamespace hhg {\nnamespace gen {\n\n");
  for (int vorder = 1; vorder <= 2; ++vorder) {
    ElementSet es;
    build_elements(vorder, &es);
    const char* D = vorder == 1 ? "p1" : "p2";
    const int G = vorder == 1 ? 1 : 8;
    char name[64];
    for (int g = 0; g < G; ++g) {
      Row A = pruned(es, 'A', g, 1), M = pruned(es, 'M', g, 1), BT = pruned(es, 'T', g, 3);
      std::snprintf(name, sizeof name, "%s_A_g%d", D, g);
      emit_vv(f, name, A, g);
      std::snprintf(name, sizeof name, "%s_M_g%d", D, g);
      emit_vv(f, name, M, g);
      std::snprintf(name, sizeof name, "%s_BT_g%d", D, g);
      emit_vp(f, name, BT);
      std::fprintf(f, "constexpr double %s_ADIAG_g%d = %s;\n\n", D, g, lit(diag_of(A, g)).c_str());
      auto er = element_rows(es, g);
      std::snprintf(name, sizeof name, "%s_Anu_g%d", D, g);
      emit_anu(f, name, er, g);
      std::snprintf(name, sizeof name, "%s_Anudiag_g%d", D, g);
      emit_anu_diag(f, name, er);
    }
    Row B = pruned(es, 'B', 0, 3);
    std::snprintf(name, sizeof name, "%s_B", D);
    emit_pv(f, name, B);
    for (int d = 0; d < 3; ++d) {
      std::snprintf(name, sizeof name, "%s_B_d%d", D, d);
      emit_pv_comp(f, name, B, d);
    }
    if (vorder == 1) {
      Row C = pruned(es, 'C', 0, 1);
      emit_pp(f, "p1_C", C);
    }
    emit_zm(f, es, D, G);
    emit_boundary_rows(f, es, D, G);
    emit_restriction(f, D, vorder);
    if (vorder == 2) emit_restriction_zm(f, D, vorder);
    emit_prolongation_cube(f, D, vorder);
  }
  std::fprintf(f, "}  // namespace gen\n}  // namespace hhg\n");
  std::fclose(f);
  return 0;
}
