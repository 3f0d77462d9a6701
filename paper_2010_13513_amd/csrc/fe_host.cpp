// Host-side finite-element setup: element matrices of the six Kuhn
// tetrahedra, row stencils on the lattice, dense symmetric pseudo-inverse.
//
// Paper Sec. 2 (eq. stokes-discrete, eq. pspg) and Sec. 2.1: on uniformly
// refined macro-cells the stencil of a row is the same at every node of one
// primitive, so rows are assembled once per row type from the element
// matrices and then applied matrix-free.
#include <algorithm>
#include <cmath>
#include <map>
#include <tuple>

#include "fe.h"

namespace hhg {
namespace {

const int kPerm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
const int kEdge[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
// parity class of each velocity group (group 0 = vertex)
const int kGroupDir[8][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1},
                             {1, 1, 0}, {1, 0, 1}, {0, 1, 1}, {1, 1, 1}};

// Affine function of the barycentric coordinates: c0 + sum_n c[n] lam_n.
struct Aff {
  double c0 = 0.0;
  double c[4] = {0, 0, 0, 0};
};

double sum4(const double* c) { return c[0] + c[1] + c[2] + c[3]; }

// int_T f g for affine f, g:  |T| [f0 g0 + (f0 S_g + g0 S_f)/4 + (S_f S_g + f.g)/20]
double int_aff_aff(const Aff& f, const Aff& g, double vol) {
  double sf = sum4(f.c), sg = sum4(g.c);
  double dot = f.c[0] * g.c[0] + f.c[1] * g.c[1] + f.c[2] * g.c[2] + f.c[3] * g.c[3];
  return vol * (f.c0 * g.c0 + (f.c0 * sg + g.c0 * sf) / 4.0 + (sf * sg + dot) / 20.0);
}

// int_T lam_k f for affine f: |T| [f0/4 + (S_f + f_k)/20]
double int_lam_aff(int k, const Aff& f, double vol) { return vol * (f.c0 / 4.0 + (sum4(f.c) + f.c[k]) / 20.0); }

double fact(int n) {
  double r = 1.0;
  for (int i = 2; i <= n; ++i) r *= i;
  return r;
}

// int_T lam_a lam_b lam_c lam_d = |T| prod(multiplicity!) / 840
double int_quartic(int a, int b, int c, int d, double vol) {
  int m[4] = {0, 0, 0, 0};
  m[a]++, m[b]++, m[c]++, m[d]++;
  return vol * fact(m[0]) * fact(m[1]) * fact(m[2]) * fact(m[3]) * 6.0 / fact(7);
}

// d phi / d lam_m for the local basis (affine in lam)
void basis_derivs(int vorder, Aff dphi[10][4]) {
  for (int a = 0; a < 10; ++a)
    for (int m = 0; m < 4; ++m) dphi[a][m] = Aff();
  if (vorder == 1) {
    for (int a = 0; a < 4; ++a) dphi[a][a].c0 = 1.0;
    return;
  }
  for (int i = 0; i < 4; ++i) {  // lam_i (2 lam_i - 1): derivative 4 lam_i - 1
    dphi[i][i].c0 = -1.0;
    dphi[i][i].c[i] = 4.0;
  }
  for (int e = 0; e < 6; ++e) {  // 4 lam_i lam_j
    int i = kEdge[e][0], j = kEdge[e][1];
    dphi[4 + e][i].c[j] = 4.0;
    dphi[4 + e][j].c[i] = 4.0;
  }
}

// P2 basis as homogeneous quadratic forms lam^T Q lam (so products integrate
// with the quartic formula).
void basis_quadratic(double Q[10][4][4]) {
  for (int a = 0; a < 10; ++a)
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) Q[a][i][j] = 0.0;
  for (int i = 0; i < 4; ++i) {  // lam_i^2 - lam_i * sum_{p != i} lam_p
    Q[i][i][i] = 1.0;
    for (int p = 0; p < 4; ++p)
      if (p != i) Q[i][i][p] = Q[i][p][i] = -0.5;
  }
  for (int e = 0; e < 6; ++e) {
    int i = kEdge[e][0], j = kEdge[e][1];
    Q[4 + e][i][j] = Q[4 + e][j][i] = 2.0;
  }
}

}  // namespace

void build_elements(int vorder, ElementSet* es) {
  es->vorder = vorder;
  es->nloc = vorder == 1 ? 4 : 10;
  const double vol = 1.0 / 6.0;
  Aff dphi[10][4];
  basis_derivs(vorder, dphi);
  double Q[10][4][4];
  basis_quadratic(Q);
  for (int t = 0; t < 6; ++t) {
    int v[4][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}, {1, 1, 1}};
    v[1][kPerm[t][0]] = 1;
    for (int d = 0; d < 3; ++d) v[2][d] = v[1][d];
    v[2][kPerm[t][1]] += 1;
    // grad lam: J = [v1-v0, v2-v0, v3-v0] (columns); grad lam_{1..3} = rows of J^{-1}
    double J[3][3];
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) J[r][c] = v[c + 1][r] - v[0][r];
    double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                 J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
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
    double g[4][3];
    for (int d = 0; d < 3; ++d) {
      g[1][d] = inv[0][d];
      g[2][d] = inv[1][d];
      g[3][d] = inv[2][d];
      g[0][d] = -(g[1][d] + g[2][d] + g[3][d]);
    }
    double G[4][4];
    for (int m = 0; m < 4; ++m)
      for (int q = 0; q < 4; ++q) G[m][q] = g[m][0] * g[q][0] + g[m][1] * g[q][1] + g[m][2] * g[q][2];
    const int n = es->nloc;
    for (int a = 0; a < n; ++a)
      for (int b = 0; b < n; ++b) {
        double s = 0.0;
        for (int m = 0; m < 4; ++m)
          for (int q = 0; q < 4; ++q) s += G[m][q] * int_aff_aff(dphi[a][m], dphi[b][q], vol);
        es->K[t][a][b] = s;
        double mass = 0.0;
        if (vorder == 1) {
          mass = vol * (a == b ? 2.0 : 1.0) / 20.0;
        } else {
          for (int i0 = 0; i0 < 4; ++i0)
            for (int i1 = 0; i1 < 4; ++i1) {
              if (Q[a][i0][i1] == 0.0) continue;
              for (int i2 = 0; i2 < 4; ++i2)
                for (int i3 = 0; i3 < 4; ++i3)
                  if (Q[b][i2][i3] != 0.0) mass += Q[a][i0][i1] * Q[b][i2][i3] * int_quartic(i0, i1, i2, i3, vol);
            }
        }
        es->M[t][a][b] = mass;
      }
    for (int d = 0; d < 3; ++d)
      for (int k = 0; k < 4; ++k)
        for (int a = 0; a < n; ++a) {
          double s = 0.0;
          for (int m = 0; m < 4; ++m) s += g[m][d] * int_lam_aff(k, dphi[a][m], vol);
          es->D[t][d][k][a] = -s;
        }
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) {
        es->Kp[t][a][b] = vol * G[a][b];
        es->Mp[t][a][b] = vol * (a == b ? 2.0 : 1.0) / 20.0;
      }
    for (int a = 0; a < 4; ++a)
      for (int d = 0; d < 3; ++d) es->ppos[t][a][d] = v[a][d];
    if (vorder == 1) {
      for (int a = 0; a < 4; ++a)
        for (int d = 0; d < 3; ++d) es->vpos[t][a][d] = v[a][d];
    } else {
      for (int a = 0; a < 4; ++a)
        for (int d = 0; d < 3; ++d) es->vpos[t][a][d] = 2 * v[a][d];
      for (int e = 0; e < 6; ++e)
        for (int d = 0; d < 3; ++d) es->vpos[t][4 + e][d] = v[kEdge[e][0]][d] + v[kEdge[e][1]][d];
    }
  }
}

Row row_stencil(const ElementSet& es, char kind, int g, int i, int j, int k, int Nbox) {
  const bool prow = (kind == 'B' || kind == 'C' || kind == 'P');
  const bool pcol = (kind == 'T' || kind == 'C' || kind == 'P');
  const int vs = es.vorder;  // site units per P1 unit
  int rpos[3];
  if (prow || vs == 1) {
    rpos[0] = i, rpos[1] = j, rpos[2] = k;
  } else {
    rpos[0] = 2 * i + kGroupDir[g][0], rpos[1] = 2 * j + kGroupDir[g][1], rpos[2] = 2 * k + kGroupDir[g][2];
  }
  std::map<std::tuple<int, int, int, int>, Entry> acc;
  for (int ck = k - 1; ck <= k + 1; ++ck)
    for (int cj = j - 1; cj <= j + 1; ++cj)
      for (int ci = i - 1; ci <= i + 1; ++ci) {
        if (ci < 0 || cj < 0 || ck < 0 || ci >= Nbox || cj >= Nbox || ck >= Nbox) continue;
        const int org[3] = {ci, cj, ck};
        for (int t = 0; t < 6; ++t) {
          // local index of the row DoF in this element
          int a = -1;
          int nrow = prow ? 4 : es.nloc;
          for (int q = 0; q < nrow; ++q) {
            const int* lp = prow ? es.ppos[t][q] : es.vpos[t][q];
            int sc = prow ? 1 : vs;
            if (org[0] * sc + lp[0] == rpos[0] && org[1] * sc + lp[1] == rpos[1] && org[2] * sc + lp[2] == rpos[2]) a = q;
          }
          if (a < 0) continue;
          int ncol = pcol ? 4 : es.nloc;
          for (int b = 0; b < ncol; ++b) {
            int cg, cidx[3];
            if (pcol || vs == 1) {
              const int* lp = pcol ? es.ppos[t][b] : es.vpos[t][b];
              cg = 0;
              for (int d = 0; d < 3; ++d) cidx[d] = org[d] + lp[d];
            } else {
              int sp[3];
              for (int d = 0; d < 3; ++d) sp[d] = 2 * org[d] + es.vpos[t][b][d];
              int par[3] = {sp[0] & 1, sp[1] & 1, sp[2] & 1};
              cg = -1;
              for (int q = 0; q < 8; ++q)
                if (kGroupDir[q][0] == par[0] && kGroupDir[q][1] == par[1] && kGroupDir[q][2] == par[2]) cg = q;
              for (int d = 0; d < 3; ++d) cidx[d] = sp[d] >> 1;
            }
            auto key = std::make_tuple(cg, cidx[2] - k, cidx[1] - j, cidx[0] - i);
            Entry& e = acc[key];
            e.g = cg;
            e.di = cidx[0] - i, e.dj = cidx[1] - j, e.dk = cidx[2] - k;
            switch (kind) {
              case 'A': e.w[0] += es.K[t][a][b]; break;
              case 'M': e.w[0] += es.M[t][a][b]; break;
              case 'C': e.w[0] += es.Kp[t][a][b]; break;
              case 'P': e.w[0] += es.Mp[t][a][b]; break;
              case 'T':
                for (int d = 0; d < 3; ++d) e.w[d] += es.D[t][d][b][a];
                break;
              case 'B':
                for (int d = 0; d < 3; ++d) e.w[d] += es.D[t][d][a][b];
                break;
            }
          }
        }
      }
  Row row;
  for (auto& kv : acc) row.push_back(kv.second);
  return row;
}

int sym_pinv(int n, const std::vector<double>& Kin, std::vector<double>& Kp, double rcond) {
  // cyclic Jacobi: A <- R^T A R until off-diagonal mass is negligible
  std::vector<double> A(Kin), V((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
  auto a = [&](int r, int c) -> double& { return A[(size_t)r * n + c]; };
  double fro = 0.0;
  for (double x : A) fro += x * x;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += a(p, q) * a(p, q);
    if (off <= 1e-32 * fro) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        double apq = a(p, q);
        if (std::fabs(apq) < 1e-300) continue;
        double theta = (a(q, q) - a(p, p)) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int r = 0; r < n; ++r) {  // columns p, q
          double arp = a(r, p), arq = a(r, q);
          a(r, p) = c * arp - s * arq;
          a(r, q) = s * arp + c * arq;
        }
        for (int r = 0; r < n; ++r) {  // rows p, q
          double apr = a(p, r), aqr = a(q, r);
          a(p, r) = c * apr - s * aqr;
          a(q, r) = s * apr + c * aqr;
        }
        for (int r = 0; r < n; ++r) {
          double vrp = V[(size_t)r * n + p], vrq = V[(size_t)r * n + q];
          V[(size_t)r * n + p] = c * vrp - s * vrq;
          V[(size_t)r * n + q] = s * vrp + c * vrq;
        }
      }
  }
  double lmax = 0.0;
  for (int i = 0; i < n; ++i) lmax = std::max(lmax, std::fabs(a(i, i)));
  Kp.assign((size_t)n * n, 0.0);
  int rank = 0;
  for (int m = 0; m < n; ++m) {
    double lam = a(m, m);
    if (std::fabs(lam) <= rcond * lmax) continue;
    ++rank;
    double il = 1.0 / lam;
    for (int r = 0; r < n; ++r) {
      double vr = V[(size_t)r * n + m] * il;
      if (vr == 0.0) continue;
      for (int c = 0; c < n; ++c) Kp[(size_t)r * n + c] += vr * V[(size_t)c * n + m];
    }
  }
  return rank;
}

bool sym_pinv_null1(int n, const std::vector<double>& K, const std::vector<double>& z, std::vector<double>& Kp) {
  // [M | I] -> [I | M^{-1}] with M = K + z z^T, row-major, n x 2n
  const size_t w = 2 * (size_t)n;
  std::vector<double> a((size_t)n * w, 0.0);
  double scale = 0.0;
  for (int r = 0; r < n; ++r) {
    for (int c = 0; c < n; ++c) {
      a[r * w + c] = K[(size_t)r * n + c] + z[r] * z[c];
      scale = std::max(scale, std::fabs(a[r * w + c]));
    }
    a[r * w + n + r] = 1.0;
  }
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(a[r * w + c]) > std::fabs(a[piv * w + c])) piv = r;
    if (!(std::fabs(a[piv * w + c]) > 1e-13 * scale)) return false;
    if (piv != c)
      for (size_t q = 0; q < w; ++q) std::swap(a[c * w + q], a[piv * w + q]);
    const double inv = 1.0 / a[c * w + c];
    for (size_t q = c; q < w; ++q) a[c * w + q] *= inv;
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const double f = a[r * w + c];
      if (f == 0.0) continue;
      double* ar = &a[r * w];
      const double* ac = &a[c * w];
      for (size_t q = c; q < w; ++q) ar[q] -= f * ac[q];
    }
  }
  Kp.assign((size_t)n * n, 0.0);
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < n; ++c) Kp[(size_t)r * n + c] = a[r * w + n + c] - z[r] * z[c];
  return true;
}

int group_of_parity(int px, int py, int pz) {
  for (int g = 0; g < 8; ++g)
    if (kGroupDir[g][0] == px && kGroupDir[g][1] == py && kGroupDir[g][2] == pz) return g;
  return -1;
}

// Kuhn point location inside the unit cube at t (in [0,1]^3): vertices (P1
// offsets from the cube origin) and barycentric coordinates.
void kuhn_locate(const double t[3], int V[4][3], double lam[4]) {
  int ord[3] = {0, 1, 2};
  std::stable_sort(ord, ord + 3, [&](int a, int b) { return t[a] > t[b]; });
  lam[0] = 1.0 - t[ord[0]];
  lam[1] = t[ord[0]] - t[ord[1]];
  lam[2] = t[ord[1]] - t[ord[2]];
  lam[3] = t[ord[2]];
  for (int d = 0; d < 3; ++d) V[0][d] = 0;
  for (int s = 0; s < 3; ++s) {
    for (int d = 0; d < 3; ++d) V[s + 1][d] = V[s][d];
    V[s + 1][ord[s]] += 1;
  }
}

// Interpolation weights of a coarse element function at a point of a fine class.
// order 1: P1 (coarse DoFs on the P1 lattice, group 0); order 2: P2 (groups).
// Returns entries (coarse group, offset from cube origin in coarse index units, weight).
std::vector<std::tuple<int, int, int, int, double>> interp_weights(int order, const double t[3]) {
  int V[4][3];
  double lam[4];
  kuhn_locate(t, V, lam);
  std::map<std::tuple<int, int, int, int>, double> acc;
  if (order == 1) {
    for (int a = 0; a < 4; ++a)
      if (lam[a] != 0.0) acc[std::make_tuple(0, V[a][0], V[a][1], V[a][2])] += lam[a];
  } else {
    const int E[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
    for (int a = 0; a < 4; ++a) {
      const double v = lam[a] * (2.0 * lam[a] - 1.0);
      if (v != 0.0) acc[std::make_tuple(0, V[a][0], V[a][1], V[a][2])] += v;
    }
    for (int e = 0; e < 6; ++e) {
      const int p = E[e][0], q = E[e][1];
      const double v = 4.0 * lam[p] * lam[q];
      if (v == 0.0) continue;
      int S[3];
      for (int d = 0; d < 3; ++d) S[d] = V[p][d] + V[q][d];  // doubled coarse position rel. to 2*cube
      const int gr = group_of_parity(S[0] & 1, S[1] & 1, S[2] & 1);
      acc[std::make_tuple(gr, S[0] >> 1, S[1] >> 1, S[2] >> 1)] += v;
    }
  }
  std::vector<std::tuple<int, int, int, int, double>> out;
  for (auto& kv : acc)
    if (std::fabs(kv.second) > 1e-15)
      out.emplace_back(std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first), std::get<3>(kv.first),
                       kv.second);
  return out;
}

void restriction_entries(int vorder, std::vector<std::vector<RestrictEntry>>& vel, std::vector<RestrictEntry>& pres) {
  const int G = vorder == 1 ? 1 : 8;
  const int vq = vorder == 1 ? 2 : 4;  // fine positions per coarse cube edge
  std::vector<std::map<std::tuple<int, int, int, int>, double>> racc(G);
  for (int cz = 0; cz < vq; ++cz)
    for (int cy = 0; cy < vq; ++cy)
      for (int cx = 0; cx < vq; ++cx) {
        const double t[3] = {(double)cx / vq, (double)cy / vq, (double)cz / vq};
        for (auto& w : interp_weights(vorder, t)) {
          const int gc = std::get<0>(w);
          const int c[3] = {cx, cy, cz};
          const int o[3] = {std::get<1>(w), std::get<2>(w), std::get<3>(w)};
          int fofs[3], fpar[3];
          for (int d = 0; d < 3; ++d) {
            if (vorder == 2) {
              const int delta = c[d] - 4 * o[d] - 2 * kGroupDir[gc][d];  // fine doubled, rel. to 2 S_c
              fpar[d] = delta & 1;
              fofs[d] = kGroupDir[gc][d] + (delta >> 1);  // fine index rel. to 2 (i,j,k)
            } else {
              fpar[d] = 0;
              fofs[d] = c[d] - 2 * o[d];
            }
          }
          const int fg = vorder == 2 ? group_of_parity(fpar[0], fpar[1], fpar[2]) : 0;
          racc[gc][std::make_tuple(fg, fofs[0], fofs[1], fofs[2])] += std::get<4>(w);
        }
      }
  vel.assign(G, {});
  for (int gc = 0; gc < G; ++gc)
    for (auto& kv : racc[gc])
      vel[gc].push_back({std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first), std::get<3>(kv.first),
                         kv.second});
  std::map<std::tuple<int, int, int>, double> pracc;
  for (int cz = 0; cz < 2; ++cz)
    for (int cy = 0; cy < 2; ++cy)
      for (int cx = 0; cx < 2; ++cx) {
        const double t[3] = {cx / 2.0, cy / 2.0, cz / 2.0};
        for (auto& w : interp_weights(1, t))
          pracc[std::make_tuple(cx - 2 * std::get<1>(w), cy - 2 * std::get<2>(w), cz - 2 * std::get<3>(w))] +=
              std::get<4>(w);
      }
  pres.clear();
  for (auto& kv : pracc)
    pres.push_back({0, std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first), kv.second});
}

}  // namespace hhg
