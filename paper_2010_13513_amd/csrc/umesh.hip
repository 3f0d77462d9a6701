// Host builder of the unstructured-mesh path (Sec. 2, 2.1, 3.2): macro
// primitives of T_0, node numbering, the rows of every macro cell per node
// class, interface lists with their Gauss-Seidel colours, and the Schur
// diagonal.  All of it float64 host arithmetic done once per hierarchy.
//
// Node numbering ("canonical order", the order of hhg_vec_from_lattice /
// _to_lattice on such a hierarchy): nodes on vertices of T_0, then on edges,
// faces, cells; within one kind by the primitive's sorted vertex ids, then by
// the barycentric weights on those vertices (in vertex-id order),
// lexicographically.
//
// Gauss-Seidel colours: interface nodes greedily in canonical order (the
// smallest colour no earlier coupled node has; coupled = sharing an element),
// K colours; cell-interior nodes K + (i + j + k) mod 4, conflict-free because
// the 14 lattice neighbours differ in i + j + k by 1, 2 or 3.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <set>

#include "umesh.h"

namespace hhg {
namespace {

using Tup = std::vector<int>;

long binom(long n, long k) {
  if (k < 0 || n < k) return 0;
  long r = 1;
  for (long t = 1; t <= k; ++t) r = r * (n - k + t) / t;
  return r;
}

// Rank of the composition w[0..d) of n (all parts >= 1) among all such
// compositions in lexicographic order.
long comp_rank(const int* w, int d, int n) {
  long r = 0;
  int R = n;
  for (int t = 0; t + 1 < d; ++t) {
    const int s = d - t - 2;
    r += binom(R - 1, s + 1) - binom(R - w[t], s + 1);
    R -= w[t];
  }
  return r;
}

// Volume and barycentric gradients of the tetrahedron Y.
double tet_geometry(const double Y[4][3], double g[4][3]) {
  double J[3][3];
  for (int a = 0; a < 3; ++a)
    for (int d = 0; d < 3; ++d) J[d][a] = Y[a + 1][d] - Y[0][d];
  const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                     J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                     J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
  // rows of J^{-1} are the gradients of the barycentric coordinates 1..3
  double inv[3][3];
  inv[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
  inv[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
  inv[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
  inv[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
  inv[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
  inv[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
  inv[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
  inv[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
  inv[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
  for (int a = 0; a < 3; ++a)
    for (int d = 0; d < 3; ++d) g[a + 1][d] = inv[a][d];
  for (int d = 0; d < 3; ++d) g[0][d] = -(g[1][d] + g[2][d] + g[3][d]);
  return std::fabs(det) / 6.0;
}

int stencil_index(int di, int dj, int dk) {
  for (int e = 0; e < kUPoints; ++e)
    if (udir(e, 0) == di && udir(e, 1) == dj && udir(e, 2) == dk) return e;
  throw Error{HHG_ERR_STATE, "internal: not a lattice neighbour"};
}

// Vertices (lattice offsets) of the Freudenthal simplex of axis order p:
// 0, e_p0, e_p0 + e_p1, (1, 1, 1).
const int kPerm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
void simplex_offsets(int p, int V[4][3]) {
  int c[3] = {0, 0, 0};
  for (int d = 0; d < 3; ++d) V[0][d] = 0;
  for (int s = 0; s < 3; ++s) {
    ++c[kPerm[p][s]];
    for (int d = 0; d < 3; ++d) V[s + 1][d] = c[d];
  }
}

// Rows of one cell (vertices X in sorted-id order) at n intervals, for every
// class: the elements of the cell around a node of class m are the lattice
// simplices at a representative node (weights 0 where m has a bit, 3
// elsewhere) that lie in the closed cell.
void cell_rows(const double X[4][3], int n, UCell& u) {
  std::memset(&u, 0, sizeof u);
  double e[3][3];  // lattice steps in (i, j, k)
  for (int a = 0; a < 3; ++a)
    for (int d = 0; d < 3; ++d) e[a][d] = (X[a + 1][d] - X[a][d]) / n;
  // element matrices of the six simplex types (translation invariant)
  double K[6][4][4], Mm[6][4][4], G[6][4][3], vol = 0.0;
  int V[6][4][3];
  for (int p = 0; p < 6; ++p) {
    simplex_offsets(p, V[p]);
    double Y[4][3];
    for (int t = 0; t < 4; ++t)
      for (int d = 0; d < 3; ++d) Y[t][d] = V[p][t][0] * e[0][d] + V[p][t][1] * e[1][d] + V[p][t][2] * e[2][d];
    vol = tet_geometry(Y, G[p]);
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) {
        K[p][a][b] = vol * (G[p][a][0] * G[p][b][0] + G[p][a][1] * G[p][b][1] + G[p][a][2] * G[p][b][2]);
        Mm[p][a][b] = vol / 20.0 * (a == b ? 2.0 : 1.0);
      }
  }
  u.cfac = (1.0 / 12.0) * std::pow(vol, 2.0 / 3.0);
  for (int m = 0; m < 16; ++m) {
    int a[4];
    for (int t = 0; t < 4; ++t) a[t] = (m >> t) & 1 ? 0 : 3;
    const int nr = a[0] + a[1] + a[2] + a[3];
    if (nr == 0) continue;
    const int P[3] = {nr - a[0], nr - a[0] - a[1], a[3]};
    auto inside = [&](const int q[3]) { return nr >= q[0] && q[0] >= q[1] && q[1] >= q[2] && q[2] >= 0; };
    for (int p = 0; p < 6; ++p)
      for (int t = 0; t < 4; ++t) {  // the node is vertex t of the element
        int Q[4][3];
        bool in = true;
        for (int s = 0; s < 4; ++s) {
          for (int d = 0; d < 3; ++d) Q[s][d] = P[d] - V[p][t][d] + V[p][s][d];
          in = in && inside(Q[s]);
        }
        if (!in) continue;
        for (int s = 0; s < 4; ++s) {
          const int ei = stencil_index(Q[s][0] - P[0], Q[s][1] - P[1], Q[s][2] - P[2]);
          u.inside[m] |= 1u << ei;
          u.A[m][ei] += K[p][t][s];
          u.M[m][ei] += Mm[p][t][s];
          for (int d = 0; d < 3; ++d) {
            u.B[m][ei][d] += -(vol / 4.0) * G[p][s][d];   // pressure row t, velocity column s
            u.BT[m][ei][d] += -(vol / 4.0) * G[p][t][d];  // velocity row t, pressure column s
          }
        }
        u.ml[m] += vol / 4.0;
      }
  }
  u.ainv0 = 1.0 / u.A[0][0];
}

struct Prims {
  std::vector<std::vector<Tup>> list;        // [d] sorted primitives of d + 1 vertices
  std::vector<std::array<long, 16>> rank;    // [cell][class] rank of the primitive within its kind
  std::vector<unsigned> owned, bnd;          // [cell] class bits
};

Tup sub_tuple(const std::array<int, 4>& v, int m) {
  Tup t;
  for (int q = 0; q < 4; ++q)
    if (!((m >> q) & 1)) t.push_back(v[q]);
  return t;
}

Prims primitives(const std::vector<std::array<int, 4>>& cells, const std::vector<std::array<int, 3>>& outflow) {
  Prims P;
  P.list.resize(4);
  std::vector<std::map<Tup, int>> first(4);
  std::map<Tup, int> face_count;
  for (size_t c = 0; c < cells.size(); ++c)
    for (int m = 0; m < 15; ++m) {
      const Tup t = sub_tuple(cells[c], m);
      first[t.size() - 1].emplace(t, (int)c);
      if (t.size() == 3) ++face_count[t];
    }
  std::vector<std::map<Tup, long>> rk(4);
  for (int d = 0; d < 4; ++d) {
    long r = 0;
    for (auto& kv : first[d]) {
      P.list[d].push_back(kv.first);
      rk[d][kv.first] = r++;
    }
  }
  std::set<Tup> outf;
  for (const auto& f : outflow) outf.insert(Tup(f.begin(), f.end()));
  // Dirichlet: sub-primitives of the faces that belong to one cell and are
  // not outflow faces
  std::set<Tup> dirichlet;
  for (auto& kv : face_count)
    if (kv.second == 1 && !outf.count(kv.first)) {
      const Tup& f = kv.first;
      for (int mask = 1; mask < 8; ++mask) {
        Tup t;
        for (int q = 0; q < 3; ++q)
          if ((mask >> q) & 1) t.push_back(f[q]);
        dirichlet.insert(t);
      }
    }
  P.rank.resize(cells.size());
  P.owned.assign(cells.size(), 0u);
  P.bnd.assign(cells.size(), 0u);
  for (size_t c = 0; c < cells.size(); ++c)
    for (int m = 0; m < 15; ++m) {
      const Tup t = sub_tuple(cells[c], m);
      P.rank[c][m] = rk[t.size() - 1][t];
      if (first[t.size() - 1][t] == (int)c) P.owned[c] |= 1u << m;
      if (dirichlet.count(t)) P.bnd[c] |= 1u << m;
    }
  return P;
}

// Lanes per segment: the smallest power of two >= the longest row (at most
// 64), so that short rows on the small levels share a wavefront.
int lanes_for(int longest) {
  int l = 1;
  while (l < longest && l < 64) l <<= 1;
  return l;
}
void push_segments(std::vector<int4>& out, int i0, int count, int j, int k, int stride, int lps) {
  for (int a = 0; a < count; a += lps) out.push_back(int4{i0 + a * stride, j, k, std::min(lps, count - a)});
}

template <typename T>
T* upload(UHier& u, const std::vector<T>& v) {
  void* p = nullptr;
  const size_t bytes = std::max<size_t>(1, v.size()) * sizeof(T);
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) throw Error{HHG_ERR_OOM, std::string("hipMalloc: ") + hipGetErrorString(e)};
  u.mem.push_back(p);
  if (!v.empty()) HHG_CHECK_HIP(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return (T*)p;
}

USegs upload_segs(UHier& u, const std::vector<int4>& v, int lps) {
  long pts = 0;
  for (const int4& q : v) pts += q.w;
  return USegs{upload(u, v), (int)v.size(), pts, lps};
}

}  // namespace

UHier::~UHier() {
  for (void* p : mem) (void)hipFree(p);
}

std::vector<std::array<int, 3>> boundary_faces_on_cube(const double* xyz, int nv, const int* tet, int nt,
                                                       unsigned faces) {
  (void)nv;
  std::map<std::array<int, 3>, int> count;
  for (int t = 0; t < nt; ++t)
    for (int drop = 0; drop < 4; ++drop) {
      std::array<int, 3> f;
      int w = 0;
      for (int q = 0; q < 4; ++q)
        if (q != drop) f[w++] = tet[4 * t + q];
      std::sort(f.begin(), f.end());
      ++count[f];
    }
  std::vector<std::array<int, 3>> out;
  for (const auto& kv : count) {
    if (kv.second != 1) continue;
    for (int face = 0; face < 6; ++face) {
      if (!((faces >> face) & 1)) continue;
      const int d = face / 2;
      const double val = face % 2;
      bool on = true;
      for (int v : kv.first) on = on && std::fabs(xyz[3 * v + d] - val) < 1e-12;
      if (on) {
        out.push_back(kv.first);
        break;
      }
    }
  }
  return out;
}

void check_outflow_faces(const int* tet, int nt, const std::vector<std::array<int, 3>>& outflow) {
  std::map<std::array<int, 3>, int> count;
  for (int t = 0; t < nt; ++t)
    for (int drop = 0; drop < 4; ++drop) {
      std::array<int, 3> f;
      int w = 0;
      for (int q = 0; q < 4; ++q)
        if (q != drop) f[w++] = tet[4 * t + q];
      std::sort(f.begin(), f.end());
      ++count[f];
    }
  long nbnd = 0;
  for (const auto& kv : count) nbnd += kv.second == 1;
  std::set<std::array<int, 3>> seen;
  for (const auto& f : outflow) {
    auto it = count.find(f);
    HHG_REQUIRE(it != count.end() && it->second == 1, HHG_ERR_ARG,
                "outflow face (" + std::to_string(f[0]) + ", " + std::to_string(f[1]) + ", " + std::to_string(f[2]) +
                    ") is not a boundary face of the mesh");
    seen.insert(f);
  }
  HHG_REQUIRE((long)seen.size() < nbnd, HHG_ERR_ARG,
              "outflow faces: at least one boundary face must stay Dirichlet (the velocity would have a null space)");
}

void validate_tet_mesh(const double* xyz, int nv, const int* tet, int nt) {
  HHG_REQUIRE(nv >= 4 && nt >= 1, HHG_ERR_ARG, "mesh: need at least 4 vertices and one tetrahedron");
  std::vector<int> used(nv, 0);
  std::set<std::array<int, 4>> seen;
  std::map<std::array<int, 3>, int> faces;  // face -> opposite vertex, -1 once shared
  double scale = 0.0;
  for (int v = 0; v < 3 * nv; ++v) {
    HHG_REQUIRE(std::isfinite(xyz[v]), HHG_ERR_ARG, "mesh: vertex " + std::to_string(v / 3) + " is not finite");
    scale = std::max(scale, std::fabs(xyz[v]));
  }
  for (int t = 0; t < nt; ++t) {
    std::array<int, 4> s;
    for (int q = 0; q < 4; ++q) {
      s[q] = tet[4 * t + q];
      HHG_REQUIRE(s[q] >= 0 && s[q] < nv, HHG_ERR_ARG, "mesh: tetrahedron " + std::to_string(t) + " has a bad vertex index");
      used[s[q]] = 1;
    }
    std::sort(s.begin(), s.end());
    HHG_REQUIRE(s[0] != s[1] && s[1] != s[2] && s[2] != s[3], HHG_ERR_ARG,
                "mesh: tetrahedron " + std::to_string(t) + " repeats a vertex");
    HHG_REQUIRE(seen.insert(s).second, HHG_ERR_ARG, "mesh: tetrahedron " + std::to_string(t) + " appears twice");
    double Y[4][3], g[4][3];
    for (int q = 0; q < 4; ++q)
      for (int d = 0; d < 3; ++d) Y[q][d] = xyz[3 * s[q] + d];
    double ext = 0.0;
    for (int q = 1; q < 4; ++q)
      for (int d = 0; d < 3; ++d) ext = std::max(ext, std::fabs(Y[q][d] - Y[0][d]));
    double J[3][3];
    for (int a = 0; a < 3; ++a)
      for (int d = 0; d < 3; ++d) J[d][a] = Y[a + 1][d] - Y[0][d];
    const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                       J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                       J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    HHG_REQUIRE(std::fabs(det) > 1e-10 * ext * ext * ext && ext > 1e-12 * std::max(scale, 1.0), HHG_ERR_ARG,
                "mesh: tetrahedron " + std::to_string(t) + " is degenerate");
    (void)g;
    for (int drop = 0; drop < 4; ++drop) {
      std::array<int, 3> f;
      int w = 0;
      for (int q = 0; q < 4; ++q)
        if (q != drop) f[w++] = s[q];
      auto it = faces.find(f);
      if (it == faces.end()) {
        faces.emplace(f, s[drop]);  // the vertex opposite the face in its first tetrahedron
        continue;
      }
      HHG_REQUIRE(it->second >= 0, HHG_ERR_ARG,
                  "mesh: a face of tetrahedron " + std::to_string(t) + " belongs to more than two tetrahedra");
      // the two tetrahedra sharing a face lie on opposite sides of it
      auto side = [&](int v) {
        double J[3][3];
        for (int a = 0; a < 3; ++a)
          for (int d = 0; d < 3; ++d) J[a][d] = xyz[3 * (a < 2 ? f[a + 1] : v) + d] - xyz[3 * f[0] + d];
        return J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
               J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
      };
      HHG_REQUIRE(side(it->second) * side(s[drop]) < 0.0, HHG_ERR_ARG,
                  "mesh: tetrahedron " + std::to_string(t) + " overlaps its neighbour across a shared face");
      it->second = -1;  // shared by two tetrahedra
    }
  }
  for (int v = 0; v < nv; ++v)
    HHG_REQUIRE(used[v], HHG_ERR_ARG, "mesh: vertex " + std::to_string(v) + " belongs to no tetrahedron");
}

namespace {

// Host tables of one level before upload.
struct UHostLevel {
  std::vector<int> canon, col;
  std::vector<unsigned char> flags;
  std::vector<double> ainv, dinv, mlown;
  std::vector<int4> all, inner, cseg[4];
  int lps_all = 64, lps_inner = 64, lps_col = 64;  // lanes per segment of each list
  int nfree = 0, nlist = 0;
};

struct UMeshPrims {
  std::vector<std::array<int, 4>> cells;  // vertex ids sorted
  Prims pr;
  long nprim[4];
};

UMeshPrims mesh_prims(const int* tet, int nt, const std::vector<std::array<int, 3>>& outflow) {
  UMeshPrims M;
  M.cells.resize(nt);
  for (int c = 0; c < nt; ++c) {
    for (int q = 0; q < 4; ++q) M.cells[c][q] = tet[4 * c + q];
    std::sort(M.cells[c].begin(), M.cells[c].end());
  }
  M.pr = primitives(M.cells, outflow);
  for (int d = 0; d < 4; ++d) M.nprim[d] = (long)M.pr.list[d].size();
  return M;
}

// Host part of level l: cell rows, slot tables, interface lists and colours,
// Schur diagonal, segments (lv.hcs, lv.h_off, lv.h_occ, lv.col_off, counts).
void u_level_host(const UMeshPrims& M, const double* xyz, int l, int schur, ULevelData& lv, UHostLevel& H) {
  const std::vector<std::array<int, 4>>& cells = M.cells;
  const Prims& pr = M.pr;
  const long* nprim = M.nprim;
  const int nt = (int)cells.size();
  const int n = 1 << l;
  const long P = utet(n + 1);
  const long nslots = (long)nt * P;
  const long vs = (nslots + 63) / 64 * 64;
  HHG_REQUIRE(4 * vs < (1L << 31), HHG_ERR_ARG, "unstructured mesh: finest level too large");
  // nodes per primitive of d + 1 vertices, and the start of each kind
  long per[4], base[5];
  base[0] = 0;
  for (int d = 0; d < 4; ++d) {
    per[d] = binom(n - 1, d);
    base[d + 1] = base[d] + nprim[d] * per[d];
  }
  const long nnodes = base[4], nif = base[3];
  HHG_REQUIRE(nnodes < (1L << 31), HHG_ERR_ARG, "unstructured mesh: too many nodes");
  lv.nnodes = (int)nnodes;
  // cell rows
  lv.hcs.resize(nt);
  for (int c = 0; c < nt; ++c) {
    double X[4][3];
    for (int q = 0; q < 4; ++q)
      for (int d = 0; d < 3; ++d) X[q][d] = xyz[3 * cells[c][q] + d];
    cell_rows(X, n, lv.hcs[c]);
    lv.hcs[c].owned = pr.owned[c];
    lv.hcs[c].bnd = pr.bnd[c];
  }
  // slot tables
  H.canon.assign(vs, -1);
  std::vector<int>& canon = H.canon;
  H.flags.assign(vs, 0);
  std::vector<unsigned char>& flags = H.flags;
  std::vector<std::vector<int2>> occ(nif);
  for (int c = 0; c < nt; ++c)
    for (int k = 0; k <= n; ++k)
      for (int j = k; j <= n; ++j)
        for (int i = j; i <= n; ++i) {
          const int a[4] = {n - i, i - j, j - k, k};
          const int m = uclass(i, j, k, n);
          int w[4], d = 0;
          for (int t = 0; t < 4; ++t)
            if (a[t] > 0) w[d++] = a[t];
          const long q = base[d - 1] + pr.rank[c][m] * per[d - 1] + comp_rank(w, d, n);
          const long s = (long)c * P + uslot(i, j, k, n);
          canon[s] = (int)q;
          flags[s] = (unsigned char)(((pr.owned[c] >> m) & 1) | (((pr.bnd[c] >> m) & 1) << 1));
          if (m) occ[q].push_back(int2{c, upack(i, j, k)});
        }
  // assembled diagonal, lumped mass, Dirichlet flag of the interface nodes
  std::vector<double> adiag(nif, 0.0), mlif(nif, 0.0);
  std::vector<char> ifd(nif, 0);
  for (long q = 0; q < nif; ++q) {
    HHG_REQUIRE(!occ[q].empty(), HHG_ERR_STATE, "internal: interface node without a cell");
    for (const int2& o : occ[q]) {  // cells ascending: the owner first
      const int i = o.y & 1023, j = (o.y >> 10) & 1023, k = o.y >> 20, m = uclass(i, j, k, n);
      adiag[q] += lv.hcs[o.x].A[m][0];
      mlif[q] += lv.hcs[o.x].ml[m];
      ifd[q] = (char)((lv.hcs[o.x].bnd >> m) & 1);
    }
  }
  // neighbours (canonical indices) of one occurrence
  auto for_neighbours = [&](const int2& o, auto&& fn) {
    const int i = o.y & 1023, j = (o.y >> 10) & 1023, k = o.y >> 20, m = uclass(i, j, k, n);
    const UCell& cs = lv.hcs[o.x];
    for (int e = 0; e < kUPoints; ++e)
      if ((cs.inside[m] >> e) & 1) {
        const long s = (long)o.x * P + uslot(i + udir(e, 0), j + udir(e, 1), k + udir(e, 2), n);
        fn(e, m, cs, canon[s]);
      }
  };
  // greedy colours of the interface nodes in canonical order
  H.col.assign(nif, 0);
  std::vector<int>& col = H.col;
  int K = 0;
  std::vector<char> used;
  for (long q = 0; q < nif; ++q) {
    used.assign(K + 2, 0);
    for (const int2& o : occ[q])
      for_neighbours(o, [&](int, int, const UCell&, int r) {
        if (r < q && r < nif && col[r] < (int)used.size()) used[col[r]] = 1;
      });
    int cq = 0;
    while (used[cq]) ++cq;
    col[q] = cq;
    K = std::max(K, cq + 1);
  }
  lv.ncol_if = K;
  // interface list: free nodes by colour, then the Dirichlet ones; inside a
  // group by the owner copy's slot (cell, then i fastest), so that the
  // threads of a launch read neighbouring memory (the order inside a colour
  // does not change the result: its nodes are not coupled)
  auto owner_slot = [&](long q) {
    const int2 o = occ[q][0];
    return (long)o.x * P + uslot(o.y & 1023, (o.y >> 10) & 1023, o.y >> 20, n);
  };
  std::vector<long> order;
  auto append_sorted = [&](std::vector<long>& grp) {
    std::sort(grp.begin(), grp.end(), [&](long a, long b) { return owner_slot(a) < owner_slot(b); });
    order.insert(order.end(), grp.begin(), grp.end());
  };
  std::vector<std::vector<long>> by_col(K);
  std::vector<long> dir_nodes;
  for (long q = 0; q < nif; ++q) {
    if (ifd[q])
      dir_nodes.push_back(q);
    else
      by_col[col[q]].push_back(q);
  }
  lv.col_off.assign(K + 1, 0);
  for (int cc = 0; cc < K; ++cc) {
    append_sorted(by_col[cc]);
    lv.col_off[cc + 1] = (int)order.size();
  }
  const int nfree = (int)order.size();
  append_sorted(dir_nodes);
  lv.h_off.assign(1, 0);
  lv.h_occ.clear();
  H.ainv.assign(order.size(), 0.0);
  std::vector<double>& ainv = H.ainv;
  for (size_t t = 0; t < order.size(); ++t) {
    const long q = order[t];
    for (const int2& o : occ[q]) lv.h_occ.push_back(o);
    lv.h_off.push_back((int)lv.h_occ.size());
    if ((int)t < nfree) ainv[t] = 1.0 / adiag[q];
  }
  // Schur diagonal per node: ML, or C_qq + sum_d sum_r B_d[q, r]^2 / A_rr
  // over free velocity nodes r
  auto adiag_of = [&](int r, int cell) -> double { return r < nif ? adiag[r] : lv.hcs[cell].A[0][0]; };
  auto free_node = [&](int r) { return r >= nif || !ifd[r]; };
  auto sd_node = [&](const std::vector<int2>& occs) {
    std::map<int, std::array<double, 3>> brow;
    double cqq = 0.0;
    std::map<int, int> cell_of;
    for (const int2& o : occs)
      for_neighbours(o, [&](int e, int m, const UCell& cs, int r) {
        auto& w = brow[r];
        for (int d = 0; d < 3; ++d) w[d] += cs.B[m][e][d];
        cell_of[r] = o.x;
        if (e == 0) cqq += cs.cfac * cs.A[m][0];
      });
    double d = cqq;
    for (auto& kv : brow)
      if (free_node(kv.first)) {
        const double a = adiag_of(kv.first, cell_of[kv.first]);
        d += (kv.second[0] * kv.second[0] + kv.second[1] * kv.second[1] + kv.second[2] * kv.second[2]) / a;
      }
    return d;
  };
  std::vector<double> dnode_if(nif);
  for (long q = 0; q < nif; ++q) dnode_if[q] = schur == HHG_SCHUR_ML ? mlif[q] : sd_node(occ[q]);
  H.dinv.assign(vs, 0.0);
  H.mlown.assign(vs, 0.0);
  std::vector<double>&dinv = H.dinv, &mlown = H.mlown;
  double mltot = 0.0;
  for (int c = 0; c < nt; ++c) {
    const UCell& cs = lv.hcs[c];
    // deep interior nodes (all neighbours interior): one value per cell
    double dcell = cs.cfac * cs.A[0][0];
    for (int e = 0; e < kUPoints; ++e)
      dcell += (cs.B[0][e][0] * cs.B[0][e][0] + cs.B[0][e][1] * cs.B[0][e][1] + cs.B[0][e][2] * cs.B[0][e][2]) /
               cs.A[0][0];
    for (int k = 0; k <= n; ++k)
      for (int j = k; j <= n; ++j)
        for (int i = j; i <= n; ++i) {
          const long s = (long)c * P + uslot(i, j, k, n);
          const int q = canon[s];
          double dq, mq;
          if (q < nif) {
            dq = dnode_if[q];
            mq = mlif[q];
          } else {
            mq = cs.ml[0];
            if (schur == HHG_SCHUR_ML) dq = mq;
            else if (i <= n - 2 && i >= j + 2 && j >= k + 2 && k >= 2) dq = dcell;
            else dq = sd_node(std::vector<int2>{int2{c, upack(i, j, k)}});
          }
          dinv[s] = 1.0 / dq;
          if (flags[s] & 1) {
            mlown[s] = mq;
            mltot += mq;
          }
        }
  }
  lv.ml_total = mltot;
  // segments
  std::vector<int4>&all = H.all, &inner = H.inner, *cseg = H.cseg;
  H.lps_all = lanes_for(n + 1);
  H.lps_inner = lanes_for(n - 2);
  H.lps_col = lanes_for((n - 2 + 3) / 4);
  for (int k = 0; k <= n; ++k)
    for (int j = k; j <= n; ++j) push_segments(all, j, n - j + 1, j, k, 1, H.lps_all);
  for (int k = 1; k <= n; ++k)
    for (int j = k + 1; j <= n; ++j) {
      const int i0 = j + 1, i1 = n - 1;
      if (i0 > i1) continue;
      push_segments(inner, i0, i1 - i0 + 1, j, k, 1, H.lps_inner);
      for (int r = 0; r < 4; ++r) {
        const int f = i0 + ((((r - i0 - j - k) % 4) + 4) % 4);
        if (f <= i1) push_segments(cseg[r], f, (i1 - f) / 4 + 1, j, k, 4, H.lps_col);
      }
    }
  H.nfree = nfree;
  H.nlist = (int)order.size();
  lv.L.n = n;
  lv.L.ncell = nt;
  lv.L.P = P;
  lv.L.vs = vs;
}

}  // namespace

UHier* u_build(const double* xyz, int nv, const int* tet, int nt, const std::vector<std::array<int, 3>>& outflow,
               int lmin, int lmax, int schur) {
  (void)nv;
  std::unique_ptr<UHier> u(new UHier);
  u->lmin = lmin;
  u->lmax = lmax;
  u->ncell = nt;
  const UMeshPrims M = mesh_prims(tet, nt, outflow);
  u->lv.resize(lmax - lmin + 1);
  for (int l = lmin; l <= lmax; ++l) {
    ULevelData& lv = u->L(l);
    UHostLevel H;
    u_level_host(M, xyz, l, schur, lv, H);
    lv.L.cs = upload(*u, lv.hcs);
    lv.all = upload_segs(*u, H.all, H.lps_all);
    lv.inner = upload_segs(*u, H.inner, H.lps_inner);
    {
      // k-marching items of the interior apply: row j, window i0 .. i0 + 61,
      // output planes [ka, kb) in chunks of kUZmChunk
      constexpr int kUZmChunk = 16;  // level 7 of the cube benchmark: 8 0.361 ms, 16 0.343, 32 0.344, 64 0.414
      const int n = lv.L.n;
      std::vector<int4> zi;
      for (int j = 2; j <= n - 2; ++j)
        for (int i0 = j + 1; i0 <= n - 1; i0 += 62)
          for (int ka = 1; ka <= j - 1; ka += kUZmChunk) zi.push_back(make_int4(j, i0, ka, std::min(ka + kUZmChunk, j)));
      if (!zi.empty()) lv.zitems = USegs{upload(*u, zi), (int)zi.size(), 0, 64};
    }
    for (int r = 0; r < 4; ++r) lv.colour[r] = upload_segs(*u, H.cseg[r], H.lps_col);
    lv.lst.off = upload(*u, lv.h_off);
    lv.lst.occ = upload(*u, lv.h_occ);
    lv.lst.ainv = upload(*u, H.ainv);
    lv.lst.nfree = H.nfree;
    lv.lst.n = H.nlist;
    lv.lst.maxocc = 0;
    for (int q = 0; q < H.nlist; ++q) lv.lst.maxocc = std::max(lv.lst.maxocc, lv.h_off[q + 1] - lv.h_off[q]);
    lv.col_maxocc.assign(lv.col_off.size() > 0 ? lv.col_off.size() - 1 : 0, 0);
    std::vector<int> col_sl(lv.col_maxocc.size(), 1);
    for (size_t cc = 0; cc + 1 < lv.col_off.size(); ++cc) {
      for (int q = lv.col_off[cc]; q < lv.col_off[cc + 1]; ++q)
        lv.col_maxocc[cc] = std::max(lv.col_maxocc[cc], lv.h_off[q + 1] - lv.h_off[q]);
      col_sl[cc] = if_slots(lv.col_maxocc[cc], lv.col_off[cc + 1] - lv.col_off[cc]);
    }
    if (!lv.col_off.empty()) {
      lv.col_off_d = upload(*u, lv.col_off);
      if (!col_sl.empty()) lv.col_sl_d = upload(*u, col_sl);
    }
    lv.dinv = upload(*u, H.dinv);
    lv.ml_own = upload(*u, H.mlown);
    lv.flags = upload(*u, H.flags);
    lv.canon = upload(*u, H.canon);
    if (l == lmin) lv.h_canon = std::move(H.canon);
  }
  return u.release();
}

namespace {
// calA on the unknowns of one level (see u_coarse_system), from its host rows
// and slot numbering.
void u_level_system(const ULevelData& lv, const std::vector<int>& canon, std::vector<int>& unk,
                    std::vector<double>& K, int max_n) {
  const int n = lv.L.n;
  const long P = lv.L.P, vs = lv.L.vs;
  const int nn = lv.nnodes;
  // owner slot, Dirichlet flag and occurrences of every node
  std::vector<long> own(nn, -1);
  std::vector<char> dir(nn, 0);
  std::vector<std::vector<int2>> occ(nn);
  for (int c = 0; c < lv.L.ncell; ++c)
    for (int k = 0; k <= n; ++k)
      for (int j = k; j <= n; ++j)
        for (int i = j; i <= n; ++i) {
          const long s = (long)c * P + uslot(i, j, k, n);
          const int q = canon[s];
          const int m = uclass(i, j, k, n);
          if ((lv.hcs[c].owned >> m) & 1) own[q] = s;
          dir[q] = (char)((lv.hcs[c].bnd >> m) & 1);
          occ[q].push_back(int2{c, upack(i, j, k)});
        }
  std::vector<int> vrow(nn, -1), prow(nn, -1);
  unk.clear();
  for (int d = 0; d < 3; ++d)
    for (int q = 0; q < nn; ++q)
      if (!dir[q]) {
        if (d == 0) vrow[q] = (int)unk.size();
        unk.push_back((int)(d * vs + own[q]));
      }
  int nv = 0;
  for (int q = 0; q < nn; ++q) nv += !dir[q];
  for (int q = 0; q < nn; ++q) {
    prow[q] = (int)unk.size();
    unk.push_back((int)(3 * vs + own[q]));
  }
  const int N = (int)unk.size();
  K.clear();
  if (N > max_n) return;
  K.assign((size_t)N * N, 0.0);
  auto vidx = [&](int q, int d) { return d * nv + vrow[q]; };
  for (int q = 0; q < nn; ++q)
    for (const int2& o : occ[q]) {
      const int i = o.y & 1023, j = (o.y >> 10) & 1023, k = o.y >> 20, m = uclass(i, j, k, n);
      const UCell& cs = lv.hcs[o.x];
      for (int e = 0; e < kUPoints; ++e) {
        if (!((cs.inside[m] >> e) & 1)) continue;
        const long s = (long)o.x * P + uslot(i + udir(e, 0), j + udir(e, 1), k + udir(e, 2), n);
        const int r = canon[s];
        for (int d = 0; d < 3; ++d) {
          if (!dir[q]) {
            if (!dir[r]) K[(size_t)vidx(q, d) * N + vidx(r, d)] += cs.A[m][e];
            K[(size_t)vidx(q, d) * N + prow[r]] += cs.BT[m][e][d];
          }
          if (!dir[r]) K[(size_t)prow[q] * N + vidx(r, d)] += cs.B[m][e][d];
        }
        K[(size_t)prow[q] * N + prow[r]] -= cs.cfac * cs.A[m][e];
      }
    }
}
}  // namespace

void u_coarse_system(UHier& u, std::vector<int>& unk, std::vector<double>& K, int max_n) {
  ULevelData& lv = u.L(u.lmin);
  u_level_system(lv, lv.h_canon, unk, K, max_n);
}

void u_query(const double* xyz, int nv, const int* tet, int nt, unsigned cube_outflow, int level, int schur,
             int max_unknowns, int* nnodes, int* ncolours, int* nunk, double* pos, int* colour, double* sdiag,
             double* Kout) {
  validate_tet_mesh(xyz, nv, tet, nt);
  HHG_REQUIRE(level >= 0 && level <= 6, HHG_ERR_ARG, "query: level must be 0..6");
  const UMeshPrims M = mesh_prims(tet, nt, boundary_faces_on_cube(xyz, nv, tet, nt, cube_outflow));
  ULevelData lv;
  UHostLevel H;
  u_level_host(M, xyz, level, schur, lv, H);
  const int n = lv.L.n;
  const long nif = (long)H.col.size();
  if (nnodes) *nnodes = lv.nnodes;
  if (ncolours) *ncolours = lv.ncol_if + 4;
  for (int c = 0; c < nt; ++c)
    for (int k = 0; k <= n; ++k)
      for (int j = k; j <= n; ++j)
        for (int i = j; i <= n; ++i) {
          const long s = (long)c * lv.L.P + uslot(i, j, k, n);
          if (!(H.flags[s] & 1)) continue;
          const int q = H.canon[s];
          const double a[4] = {(double)(n - i), (double)(i - j), (double)(j - k), (double)k};
          if (pos)
            for (int d = 0; d < 3; ++d) {
              double v = 0.0;
              for (int t = 0; t < 4; ++t) v += a[t] * xyz[3 * M.cells[c][t] + d];
              pos[3 * (size_t)q + d] = v / n;
            }
          if (colour) colour[q] = q < nif ? H.col[q] : lv.ncol_if + (i + j + k) % 4;
          if (sdiag) sdiag[q] = 1.0 / H.dinv[s];
        }
  std::vector<int> unk;
  std::vector<double> K;
  u_level_system(lv, H.canon, unk, K, max_unknowns);
  if (nunk) *nunk = (int)unk.size();
  if (Kout && !K.empty()) std::copy(K.begin(), K.end(), Kout);
}

}  // namespace hhg
