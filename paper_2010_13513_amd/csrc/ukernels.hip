// Kernels of the unstructured-mesh path (Sec. 2, 2.1, 3.2, 3.3), float64.
//
// Cell interiors run as lattice kernels: a workgroup of four wavefronts
// takes 256 / lps row segments of one cell (grid.y = cell), one lane per point,
// with the cell's interior rows staged in LDS; neighbours are the 14
// Freudenthal neighbours in the cell's packed slot order.  On the large
// levels the interior rows of the apply walk k instead (k_u_apply_zm).
// Interface nodes (on vertices, edges and faces of T_0) run 16, 32 or 64
// lanes per node, one per stencil point and occurrence slot: the row is the
// sum, over the cells containing the node, of that cell's row of the node's
// class, and the result goes to every copy of the node.  The smoothing calls
// of the smallest levels run in one workgroup (k_u_smooth_small).
#include <type_traits>

#include "lanes.h"
#include "umesh.h"

namespace hhg {
namespace {

constexpr int kUBlock = 256;

__device__ __forceinline__ void unpack(int v, int& i, int& j, int& k) {
  i = v & 1023;
  j = (v >> 10) & 1023;
  k = v >> 20;
}

// Slot offsets of the 15 stencil points relative to the centre.
__device__ __forceinline__ void offsets(int i, int j, int k, int n, int (&off)[kUPoints]) {
  const int c = uslot(i, j, k, n);
#pragma unroll
  for (int e = 0; e < kUPoints; ++e) off[e] = uslot(i + udir(e, 0), j + udir(e, 1), k + udir(e, 2), n) - c;
}

// Interior rows of cell c (class 0) into LDS: A, B^T (3), B (3), M.
__device__ __forceinline__ void stage_inner(const UCell* __restrict__ cs, double (*w)[kUPoints]) {
  for (int t = threadIdx.x; t < 8 * kUPoints; t += kUBlock) {
    const int q = t / kUPoints, e = t % kUPoints;
    double v;
    if (q == 0) v = cs->A[0][e];
    else if (q < 4) v = cs->BT[0][e][q - 1];
    else if (q < 7) v = cs->B[0][e][q - 4];
    else v = cs->M[0][e];
    w[q][e] = v;
  }
  __syncthreads();
}

// ------------------------------------------------------------------ apply
// opmask bits: 1 A, 2 B^T, 4 B, 8 C, 16 C with + sign (the C block alone);
// wv / wp: write the velocity / pressure rows.
// Interior point (i, j, k) of cell c, its rows w (class 0, staged in LDS).
template <bool HB, bool MASS>
__device__ __forceinline__ void apply_inner_pt(const ULev& L, int c, const double (*w)[kUPoints], double cf, int i,
                                               int j, int k, const double* __restrict__ x,
                                               const double* __restrict__ b, double* __restrict__ y, int opmask,
                                               int wv, int wp) {
  const int n = L.n;
  int off[kUPoints];
  offsets(i, j, k, n, off);
  const size_t t = (size_t)c * L.P + uslot(i, j, k, n);
  const size_t vs = L.vs;
  if (MASS) {
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      const double* xf = x + f * vs + t;
      double a = 0.0;
#pragma unroll
      for (int e = 0; e < kUPoints; ++e) a += w[7][e] * xf[off[e]];
      y[f * vs + t] = a;
    }
    return;
  }
  const bool dA = opmask & 1, dBT = opmask & 2, dB = opmask & 4, dC = opmask & 24;
  double au[3] = {0.0, 0.0, 0.0}, bp[3] = {0.0, 0.0, 0.0}, bu = 0.0, cp = 0.0;
  const double *u0 = x + t, *u1 = x + vs + t, *u2 = x + 2 * vs + t, *p = x + 3 * vs + t;
#pragma unroll
  for (int e = 0; e < kUPoints; ++e) {
    if (dA || dB) {
      const double v0 = u0[off[e]], v1 = u1[off[e]], v2 = u2[off[e]];
      if (dA) {
        au[0] += w[0][e] * v0;
        au[1] += w[0][e] * v1;
        au[2] += w[0][e] * v2;
      }
      if (dB) bu += w[4][e] * v0 + w[5][e] * v1 + w[6][e] * v2;
    }
    if (dBT || dC) {
      const double pe = p[off[e]];
      if (dBT) {
        bp[0] += w[1][e] * pe;
        bp[1] += w[2][e] * pe;
        bp[2] += w[3][e] * pe;
      }
      if (dC) cp += w[0][e] * pe;
    }
  }
  const double yp = bu + ((opmask & 16) ? cf * cp : -(cf * cp));
  if (wv)
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double v = au[d] + bp[d];
      y[d * vs + t] = HB ? b[d * vs + t] - v : v;
    }
  if (wp) y[3 * vs + t] = HB ? b[3 * vs + t] - yp : yp;
}

template <bool HB, bool MASS>
__global__ void __launch_bounds__(kUBlock) k_u_apply_inner(ULev L, USegs sg, const double* __restrict__ x,
                                                           const double* __restrict__ b, double* __restrict__ y,
                                                           int opmask, int wv, int wp) {
  __shared__ double w[8][kUPoints];
  const int c = blockIdx.y;
  const UCell* cs = L.cs + c;
  stage_inner(cs, w);
  const int sid = blockIdx.x * (kUBlock / sg.lps) + threadIdx.x / sg.lps, lane = threadIdx.x % sg.lps;
  if (sid >= sg.n) return;
  const int4 s = sg.s[sid];
  if (lane >= s.w) return;
  apply_inner_pt<HB, MASS>(L, c, w, cs->cfac, s.x + lane, s.y, s.z, x, b, y, opmask, wv, wp);
}

// k-marching apply of the interior rows (class 0) of cell c: a wavefront owns
// the points (i0 - 1 .. i0 + 62, j) of one row j of the cell and the output
// planes [ka, kb), and walks k = ka - 1 .. kb; at each plane it loads rows
// j - 1, j, j + 1 of the four fields once (12 loads), takes the i -+ 1
// neighbours from the adjacent lanes, and adds each word into the rows of
// its lane's point at k - 1, k, k + 1 (three rotating accumulator planes);
// the row at k - 1 is complete after plane k and is written.  Per interior
// point this issues 12 loads per plane for 62 points instead of 60 gathers
// per point.  Lanes outside the row load its nearest point: an interior row
// only reads points inside the closed cell, so such words reach only rows
// that are not written.  Same products as apply_inner_pt, summed in another
// order.  Velocity row d: A u_d + B^T_d p; pressure row: B u -+ C p.
template <int Q, bool HB>
__device__ __forceinline__ void uzm_step(const ULev& L, const double (*w)[kUPoints], double csign, size_t base, int i,
                                         int j, int kp, bool out, int ka, int kb, const double* __restrict__ x,
                                         const double* __restrict__ b, double* __restrict__ y, bool dA, bool dBT,
                                         bool dB, bool dC, int wv, int wp, double (&acc)[3][4]) {
  const int n = L.n;
  const size_t vs = L.vs;
  // the rows are read from LDS at every plane: an opaque zero offset keeps
  // the compiler from hoisting all 105 weights into registers for the loop
  int z = 0;
  asm volatile("" : "+v"(z));
  const double* wz = &w[0][0] + z;
  double v[3][4];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const int jj = max(j - 1 + r, kp);  // row j - 1 at plane j is not in the cell (its words reach row k = j only)
    const size_t sl = base + uslot(min(max(i, jj), n), jj, kp, n);
#pragma unroll
    for (int f = 0; f < 4; ++f) v[r][f] = x[f * vs + sl];
  }
#pragma unroll
  for (int e = 0; e < kUPoints; ++e) {
    const int di = udir(e, 0), dj = udir(e, 1), dk = udir(e, 2);
    const int sl = ((Q - dk) % 3 + 3) % 3;  // accumulator plane of the row at k = kp - dk
    double u[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      const double a = v[dj + 1][f];
      u[f] = di < 0 ? gen::from_prev(a) : (di > 0 ? gen::from_next(a) : a);
    }
    auto W = [&](int q) { return wz[q * kUPoints + e]; };
    if (dA)
#pragma unroll
      for (int d = 0; d < 3; ++d) acc[sl][d] += W(0) * u[d];
    if (dBT)
#pragma unroll
      for (int d = 0; d < 3; ++d) acc[sl][d] += W(1 + d) * u[3];
    if (dB) acc[sl][3] += W(4) * u[0] + W(5) * u[1] + W(6) * u[2];
    if (dC) acc[sl][3] += csign * (W(0) * u[3]);
  }
  constexpr int S = (Q + 2) % 3;  // the row at k = kp - 1
  const int kr = kp - 1;
  if (out && kr >= ka && kr < kb) {
    const size_t t = base + uslot(i, j, kr, n);
    if (wv)
#pragma unroll
      for (int d = 0; d < 3; ++d) y[d * vs + t] = HB ? b[d * vs + t] - acc[S][d] : acc[S][d];
    if (wp) y[3 * vs + t] = HB ? b[3 * vs + t] - acc[S][3] : acc[S][3];
  }
#pragma unroll
  for (int f = 0; f < 4; ++f) acc[S][f] = 0.0;
}

template <bool HB>
__global__ void __launch_bounds__(kUBlock) k_u_apply_zm(ULev L, const int4* __restrict__ items, int nitems,
                                                        const double* __restrict__ x, const double* __restrict__ b,
                                                        double* __restrict__ y, int opmask, int wv, int wp) {
  __shared__ double w[8][kUPoints];
  const int c = blockIdx.y;
  const UCell* cs = L.cs + c;
  stage_inner(cs, w);
  const int it = blockIdx.x * (kUBlock / 64) + (int)threadIdx.x / 64, lane = (int)threadIdx.x % 64;
  if (it >= nitems) return;  // whole wavefront
  const int4 item = items[it];  // (j, i0, ka, kb)
  const int j = item.x, ka = item.z, kb = item.w, n = L.n;
  const int i = item.y - 1 + lane;
  const bool out = lane >= 1 && lane <= 62 && i <= n - 1;
  const bool dA = opmask & 1, dBT = opmask & 2, dB = opmask & 4, dC = opmask & 24;
  const double csign = (opmask & 16) ? cs->cfac : -cs->cfac;
  const size_t base = (size_t)c * L.P;
  double acc[3][4];
#pragma unroll
  for (int q = 0; q < 3; ++q)
#pragma unroll
    for (int f = 0; f < 4; ++f) acc[q][f] = 0.0;
  const int nq = kb - ka + 2;
  for (int q = 0; q < nq; q += 3) {
    const int kp = ka - 1 + q;
    uzm_step<0, HB>(L, w, csign, base, i, j, kp, out, ka, kb, x, b, y, dA, dBT, dB, dC, wv, wp, acc);
    if (q + 1 < nq) uzm_step<1, HB>(L, w, csign, base, i, j, kp + 1, out, ka, kb, x, b, y, dA, dBT, dB, dC, wv, wp, acc);
    if (q + 2 < nq) uzm_step<2, HB>(L, w, csign, base, i, j, kp + 2, out, ka, kb, x, b, y, dA, dBT, dB, dC, wv, wp, acc);
  }
}

// Interface nodes: a group of 16 SL lanes per node (SL = 1, 2 or 4 slots,
// set per launch by the most occurrences of one of its nodes).  Lane l
// takes stencil point e = l mod 16 (e < 15) of the node's occurrences (cells)
// l / 16, l / 16 + SL, ...; the lane sums are combined by shuffles within
// the group.  Points outside an occurrence's closed cell add nothing.  (Face
// nodes follow each other in node order, so neighbouring groups read
// neighbouring rows; one lane per node would leave most compute units idle
// on the few thousand nodes of one colour, and a node in many cells -- the
// vertices and edges of T_0 -- would walk them one after the other.)
constexpr int kIfPts = 16;

__host__ __device__ constexpr int if_nodes(int sl) { return kUBlock / (kIfPts * sl); }
constexpr int kIfManyNodes = 8192;  // see if_launch

template <int GW>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
  for (int off = GW / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, GW);
  return v;
}
__device__ __forceinline__ size_t occ_centre(const ULev& L, int2 oc) {
  int i, j, k;
  unpack(oc.y, i, j, k);
  return (size_t)oc.x * L.P + uslot(i, j, k, L.n);
}
// The occurrences of a node are taken in batches of 16 SL: lane l of the
// node's group loads the record of occurrence base + l (cell, packed point,
// class, the class's inside mask), then the group walks the batch in order,
// SL occurrences at a time, with the records passed round by shuffles.  The
// loads of one occurrence then depend on no load of another, and a node in
// many cells costs one batch of round trips instead of a chain of three per
// occurrence.
struct OccRec {
  int cell, pt, m;
  unsigned in;
};
__device__ __forceinline__ OccRec occ_record(const ULev& L, const UList& lst, int o0, int no, int idx) {
  OccRec r{0, 0, 0, 0u};
  if (idx < no) {
    const int2 oc = lst.occ[o0 + idx];
    int i, j, k;
    unpack(oc.y, i, j, k);
    r.cell = oc.x;
    r.pt = oc.y;
    r.m = uclass(i, j, k, L.n);
    r.in = L.cs[oc.x].inside[r.m];
  }
  return r;
}
template <int GW>
__device__ __forceinline__ OccRec occ_share(const OccRec& r, int u) {
  return OccRec{__shfl(r.cell, u, GW), __shfl(r.pt, u, GW), __shfl(r.m, u, GW), (unsigned)__shfl((int)r.in, u, GW)};
}
// Stencil point e of occurrence r: ok (a real occurrence and the point
// inside its closed cell) and its slot; otherwise the slot of the centre (a
// valid address whose words are then weighted by zero) -- no branch, so the
// loads of consecutive occurrences can be in flight together.
__device__ __forceinline__ long occ_slot(const ULev& L, const OccRec& r, int e, bool real, bool& ok) {
  ok = real && e < kUPoints && ((r.in >> e) & 1u);
  const int ee = ok ? e : 0;
  int i, j, k;
  unpack(r.pt, i, j, k);
  return (long)r.cell * L.P + uslot(i + udir(ee, 0), j + udir(ee, 1), k + udir(ee, 2), L.n);
}

// Rows of interface node q, lane l of its group of 16 SL lanes (the whole
// group calls it).
template <bool HB, bool MASS, int SL>
__device__ __forceinline__ void apply_iface_node(const ULev& L, const UList& lst, int q, int l,
                                                 const double* __restrict__ x, const double* __restrict__ b,
                                                 double* __restrict__ y, int opmask, int wv, int wp) {
  constexpr int GW = kIfPts * SL;
  const int e = l % kIfPts;
  const size_t vs = L.vs;
  const int o0 = lst.off[q], o1 = lst.off[q + 1], no = o1 - o0;
  double acc[4] = {0.0, 0.0, 0.0, 0.0}, bp[3] = {0.0, 0.0, 0.0}, cp = 0.0;
  const bool dA = opmask & 1, dBT = opmask & 2, dB = opmask & 4, dC = opmask & 24;
  const int ew = e < kUPoints ? e : 0;  // weight column of the lane (lane 15: weighted by zero)
  for (int base = 0; base < no; base += GW) {
    const OccRec mine = occ_record(L, lst, o0, no, base + l);
    const int cnt = min(GW, no - base);
    for (int u0 = 0; u0 < cnt; u0 += SL) {
      const int u = u0 + l / kIfPts;
      const OccRec r = occ_share<GW>(mine, u);
      bool ok;
      const long sl = occ_slot(L, r, e, u < cnt, ok);
      const double z = ok ? 1.0 : 0.0;
      const UCell* cs = L.cs + r.cell;
      const int m = r.m;
      if (MASS) {
        const double mw = z * cs->M[m][ew];
        for (int f = 0; f < 4; ++f) acc[f] += mw * x[f * vs + sl];
        continue;
      }
      if (dA || dB) {
        const double v0 = x[sl], v1 = x[vs + sl], v2 = x[2 * vs + sl];
        if (dA) {
          const double a = z * cs->A[m][ew];
          acc[0] += a * v0;
          acc[1] += a * v1;
          acc[2] += a * v2;
        }
        if (dB)
          acc[3] += (z * cs->B[m][ew][0]) * v0 + (z * cs->B[m][ew][1]) * v1 + (z * cs->B[m][ew][2]) * v2;
      }
      if (dBT || dC) {
        const double pe = x[3 * vs + sl];
        if (dBT) {
          bp[0] += (z * cs->BT[m][ew][0]) * pe;
          bp[1] += (z * cs->BT[m][ew][1]) * pe;
          bp[2] += (z * cs->BT[m][ew][2]) * pe;
        }
        if (dC) cp += cs->cfac * (z * cs->A[m][ew]) * pe;
      }
    }
  }
  double out[4];
  const size_t own = occ_centre(L, lst.occ[o0]);
  if (MASS) {
    for (int f = 0; f < 4; ++f) out[f] = group_sum<GW>(acc[f]);
  } else {
    const bool dir = q >= lst.nfree;
    for (int d = 0; d < 3; ++d) {
      const double v = group_sum<GW>(acc[d] + bp[d]);
      out[d] = dir ? 0.0 : (HB ? b[d * vs + own] - v : v);
    }
    const double yp = group_sum<GW>(acc[3] + ((opmask & 16) ? cp : -cp));
    out[3] = HB ? b[3 * vs + own] - yp : yp;
  }
  for (int o = o0 + l; o < o1; o += GW) {
    const size_t sl = occ_centre(L, lst.occ[o]);
    if (MASS || wv)
      for (int d = 0; d < 3; ++d) y[d * vs + sl] = out[d];
    if (MASS || wp) y[3 * vs + sl] = out[3];
  }
}

template <bool HB, bool MASS, int SL>
__global__ void __launch_bounds__(kUBlock) k_u_apply_iface(ULev L, UList lst, const double* __restrict__ x,
                                                           const double* __restrict__ b, double* __restrict__ y,
                                                           int opmask, int wv, int wp) {
  constexpr int GW = kIfPts * SL;
  const int q = blockIdx.x * if_nodes(SL) + (threadIdx.x / GW);
  if (q >= lst.n) return;
  apply_iface_node<HB, MASS, SL>(L, lst, q, threadIdx.x % GW, x, b, y, opmask, wv, wp);
}

// ----------------------------------------------------------- Gauss-Seidel
// One interior colour: points (i, j, k) of the cell interiors with i + j + k
// = colour (mod 4), segments of stride 4; u_d += (f_d - A u_d - B^T_d p) / a_00.
__device__ __forceinline__ void gs_inner_pt(const ULev& L, int c, const double (*w)[kUPoints], double ai, int i,
                                            int j, int k, double* __restrict__ x, const double* __restrict__ b) {
  const int n = L.n;
  int off[kUPoints];
  offsets(i, j, k, n, off);
  const size_t t = (size_t)c * L.P + uslot(i, j, k, n);
  const size_t vs = L.vs;
  const double* p = x + 3 * vs + t;
  double r[3] = {b[t], b[vs + t], b[2 * vs + t]};
#pragma unroll
  for (int e = 0; e < kUPoints; ++e) {
    const double pe = p[off[e]];
    r[0] -= w[0][e] * x[t + off[e]] + w[1][e] * pe;
    r[1] -= w[0][e] * x[vs + t + off[e]] + w[2][e] * pe;
    r[2] -= w[0][e] * x[2 * vs + t + off[e]] + w[3][e] * pe;
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) x[d * vs + t] += r[d] * ai;
}

__global__ void __launch_bounds__(kUBlock) k_u_gs_inner(ULev L, USegs sg, double* __restrict__ x,
                                                        const double* __restrict__ b) {
  __shared__ double w[8][kUPoints];
  const int c = blockIdx.y;
  const UCell* cs = L.cs + c;
  stage_inner(cs, w);
  const int sid = blockIdx.x * (kUBlock / sg.lps) + threadIdx.x / sg.lps, lane = threadIdx.x % sg.lps;
  if (sid >= sg.n) return;
  const int4 s = sg.s[sid];
  if (lane >= s.w) return;
  gs_inner_pt(L, c, w, cs->ainv0, s.x + 4 * lane, s.y, s.z, x, b);
}

// Free interface nodes [first, first + count) of one colour, a group of
// 16 SL lanes per node as in k_u_apply_iface.  Every lane of a group reads the
// node's old value before any lane writes a copy (one wavefront, program
// order).
template <int SL>
__device__ __forceinline__ void gs_iface_node(const ULev& L, const UList& lst, int q, int l, double* __restrict__ x,
                                              const double* __restrict__ b) {
  constexpr int GW = kIfPts * SL;
  const int e = l % kIfPts;
  const size_t vs = L.vs;
  const int o0 = lst.off[q], o1 = lst.off[q + 1], no = o1 - o0;
  double r[3] = {0.0, 0.0, 0.0};
  const int ew = e < kUPoints ? e : 0;
  for (int base = 0; base < no; base += GW) {
    const OccRec mine = occ_record(L, lst, o0, no, base + l);
    const int cnt = min(GW, no - base);
    for (int u0 = 0; u0 < cnt; u0 += SL) {
      const int u = u0 + l / kIfPts;
      const OccRec rc = occ_share<GW>(mine, u);
      bool ok;
      const long sl = occ_slot(L, rc, e, u < cnt, ok);
      const double z = ok ? 1.0 : 0.0;
      const UCell* cs = L.cs + rc.cell;
      const int m = rc.m;
      const double a = z * cs->A[m][ew], pe = x[3 * vs + sl];
      r[0] += a * x[sl] + (z * cs->BT[m][ew][0]) * pe;
      r[1] += a * x[vs + sl] + (z * cs->BT[m][ew][1]) * pe;
      r[2] += a * x[2 * vs + sl] + (z * cs->BT[m][ew][2]) * pe;
    }
  }
  const size_t own = occ_centre(L, lst.occ[o0]);
  const double ai = lst.ainv[q];
  double v[3];
  for (int d = 0; d < 3; ++d) v[d] = x[d * vs + own] + (b[d * vs + own] - group_sum<GW>(r[d])) * ai;
  for (int o = o0 + l; o < o1; o += GW) {
    const size_t sl = occ_centre(L, lst.occ[o]);
    for (int d = 0; d < 3; ++d) x[d * vs + sl] = v[d];
  }
}

template <int SL>
__global__ void __launch_bounds__(kUBlock) k_u_gs_iface(ULev L, UList lst, int first, int count,
                                                        double* __restrict__ x, const double* __restrict__ b) {
  constexpr int GW = kIfPts * SL;
  const int t = blockIdx.x * if_nodes(SL) + (threadIdx.x / GW);
  if (t >= count) return;
  gs_iface_node<SL>(L, lst, first + t, threadIdx.x % GW, x, b);
}

// p -= omega r_p dinv on every real slot (copies stay equal: same inputs).
__global__ void __launch_bounds__(kUBlock) k_u_pstep(long nslots, long vs, const double* __restrict__ dinv,
                                                     double* __restrict__ x, const double* __restrict__ r,
                                                     double omega) {
  const long t = (long)blockIdx.x * kUBlock + threadIdx.x;
  if (t >= nslots) return;
  x[3 * vs + t] -= omega * r[3 * vs + t] * dinv[t];
}

// --------------------------------------------------------------- transfer
// Restriction at coarse interior points: r_c = r_f(2 p) + 1/2 sum of the 14
// fine neighbours of 2 p (the midpoints of the coarse edges at p).
__global__ void __launch_bounds__(kUBlock) k_u_restrict_inner(ULev Lf, ULev Lc, USegs sg,
                                                              const double* __restrict__ rf,
                                                              double* __restrict__ rc) {
  const int c = blockIdx.y;
  const int sid = blockIdx.x * (kUBlock / sg.lps) + threadIdx.x / sg.lps, lane = threadIdx.x % sg.lps;
  if (sid >= sg.n) return;
  const int4 s = sg.s[sid];
  if (lane >= s.w) return;
  const int i = s.x + lane, j = s.y, k = s.z;
  int off[kUPoints];
  offsets(2 * i, 2 * j, 2 * k, Lf.n, off);
  const size_t tf = (size_t)c * Lf.P + uslot(2 * i, 2 * j, 2 * k, Lf.n);
  const size_t tc = (size_t)c * Lc.P + uslot(i, j, k, Lc.n);
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    const double* r = rf + f * Lf.vs + tf;
    double a = 0.0;
#pragma unroll
    for (int e = 1; e < kUPoints; ++e) a += r[off[e]];
    rc[f * Lc.vs + tc] = r[0] + 0.5 * a;
  }
}

// Restriction at coarse interface nodes: the fine node at 2 q, plus half of
// every fine midpoint next to it, each midpoint taken once (from the cell
// that owns the primitive it lies on); fine Dirichlet velocity values count
// as zero and the coarse Dirichlet velocity rows are zero.  A group of 16 SL
// lanes per node, lane l the midpoint in direction l mod 16 of the node's
// occurrences l / 16, l / 16 + SL, ..., records in batches as in the
// interface rows above.
template <int SL>
__global__ void __launch_bounds__(kUBlock) k_u_restrict_iface(ULev Lf, ULev Lc, UList lst,
                                                              const double* __restrict__ rf,
                                                              double* __restrict__ rc) {
  constexpr int GW = kIfPts * SL;
  const int q = blockIdx.x * if_nodes(SL) + (threadIdx.x / GW), l = threadIdx.x % GW, e = l % kIfPts;
  if (q >= lst.n) return;
  const int nc = Lc.n, nf = Lf.n;
  const int o0 = lst.off[q], o1 = lst.off[q + 1], no = o1 - o0;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const bool lane_pt = e >= 1 && e < kUPoints;
  const int ee = lane_pt ? e : 1;
  for (int base = 0; base < no; base += GW) {
    // record of occurrence base + l: cell, coarse point, and the fine cell's
    // inside mask of the coarse class, ownership and Dirichlet masks
    int mc = 0, mp = 0;
    unsigned mi = 0u, mo = 0u, mb = 0u;
    if (base + l < no) {
      const int2 oc = lst.occ[o0 + base + l];
      int i, j, k;
      unpack(oc.y, i, j, k);
      const UCell* cs = Lf.cs + oc.x;
      mc = oc.x;
      mp = oc.y;
      mi = cs->inside[uclass(i, j, k, nc)];
      mo = cs->owned;
      mb = cs->bnd;
    }
    const int cnt = min(GW, no - base);
    for (int u0 = 0; u0 < cnt; u0 += SL) {
      const int u = u0 + l / kIfPts;
      const int cell = __shfl(mc, u, GW), pt = __shfl(mp, u, GW);
      const unsigned ins = (unsigned)__shfl((int)mi, u, GW), own = (unsigned)__shfl((int)mo, u, GW),
                     bnd = (unsigned)__shfl((int)mb, u, GW);
      int i, j, k;
      unpack(pt, i, j, k);
      const int I = 2 * i + udir(ee, 0), J = 2 * j + udir(ee, 1), K = 2 * k + udir(ee, 2);
      const int mf = uclass(I, J, K, nf);
      const bool take = u < cnt && lane_pt && ((ins >> e) & 1) && ((own >> mf) & 1);
      const size_t sl = (size_t)cell * Lf.P + (take ? uslot(I, J, K, nf) : uslot(2 * i, 2 * j, 2 * k, nf));
      const bool fd = (bnd >> mf) & 1;
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        const double v = rf[f * Lf.vs + sl];
        acc[f] += (take && !(f < 3 && fd)) ? 0.5 * v : 0.0;
      }
    }
  }
#pragma unroll
  for (int f = 0; f < 4; ++f) acc[f] = group_sum<GW>(acc[f]);
  int i, j, k;
  unpack(lst.occ[o0].y, i, j, k);
  const size_t fown = (size_t)lst.occ[o0].x * Lf.P + uslot(2 * i, 2 * j, 2 * k, nf);
  const bool dir = q >= lst.nfree;
  double out[4];
  for (int f = 0; f < 4; ++f) out[f] = (f < 3 && dir) ? 0.0 : rf[f * Lf.vs + fown] + acc[f];
  for (int o = o0 + l; o < o1; o += GW) {
    const int2 oc = lst.occ[o];
    unpack(oc.y, i, j, k);
    const size_t sl = (size_t)oc.x * Lc.P + uslot(i, j, k, nc);
    for (int f = 0; f < 4; ++f) rc[f * Lc.vs + sl] = out[f];
  }
}

// Linear interpolation at every fine slot of a cell (copies of interface
// nodes included: every cell computes the same value for them).
__global__ void __launch_bounds__(kUBlock) k_u_prolong(ULev Lc, ULev Lf, USegs sg, const double* __restrict__ xc,
                                                       double* __restrict__ xf, int add, int skip_bnd) {
  const int c = blockIdx.y;
  const int sid = blockIdx.x * (kUBlock / sg.lps) + threadIdx.x / sg.lps, lane = threadIdx.x % sg.lps;
  if (sid >= sg.n) return;
  const int4 s = sg.s[sid];
  if (lane >= s.w) return;
  const int I = s.x + lane, J = s.y, K = s.z;
  const int nf = Lf.n, nc = Lc.n;
  const size_t tf = (size_t)c * Lf.P + uslot(I, J, K, nf);
  const size_t ta = (size_t)c * Lc.P + uslot(I >> 1, J >> 1, K >> 1, nc);
  const size_t tb = (size_t)c * Lc.P + uslot((I + 1) >> 1, (J + 1) >> 1, (K + 1) >> 1, nc);
  const bool even = !((I | J | K) & 1);
  const bool fd = skip_bnd && ((Lf.cs[c].bnd >> uclass(I, J, K, nf)) & 1);
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    const double v = even ? xc[f * Lc.vs + ta] : 0.5 * (xc[f * Lc.vs + ta] + xc[f * Lc.vs + tb]);
    double* o = xf + f * Lf.vs + tf;
    if (!add) *o = v;
    else if (!(f < 3 && fd)) *o += v;
  }
}

// Dirichlet velocity slots of the coarse level <- the fine value at 2 (i, j, k).
__global__ void __launch_bounds__(kUBlock) k_u_inject(ULev Lf, ULev Lc, USegs sg, const double* __restrict__ xf,
                                                      double* __restrict__ xc) {
  const int c = blockIdx.y;
  const int sid = blockIdx.x * (kUBlock / sg.lps) + threadIdx.x / sg.lps, lane = threadIdx.x % sg.lps;
  if (sid >= sg.n) return;
  const int4 s = sg.s[sid];
  if (lane >= s.w) return;
  const int i = s.x + lane, j = s.y, k = s.z;
  if (!((Lc.cs[c].bnd >> uclass(i, j, k, Lc.n)) & 1)) return;
  const size_t tc = (size_t)c * Lc.P + uslot(i, j, k, Lc.n);
  const size_t tf = (size_t)c * Lf.P + uslot(2 * i, 2 * j, 2 * k, Lf.n);
  for (int d = 0; d < 3; ++d) xc[d * Lc.vs + tc] = xf[d * Lf.vs + tf];
}

// ------------------------------------------------------------ flat kernels
__global__ void __launch_bounds__(kUBlock) k_u_copy_bnd(long nslots, long vs, const unsigned char* __restrict__ fl,
                                                        const double* __restrict__ src, double* __restrict__ dst) {
  const long t = (long)blockIdx.x * kUBlock + threadIdx.x;
  if (t >= nslots || !(fl[t] & 2)) return;
  for (int d = 0; d < 3; ++d) dst[d * vs + t] = src[d * vs + t];
}

// Load vector of the right-hand side: zero Dirichlet velocity rows and the pressure rows.
__global__ void __launch_bounds__(kUBlock) k_u_rhs_fix(long nslots, long vs, const unsigned char* __restrict__ fl,
                                                       double* __restrict__ b) {
  const long t = (long)blockIdx.x * kUBlock + threadIdx.x;
  if (t >= nslots) return;
  if (fl[t] & 2)
    for (int d = 0; d < 3; ++d) b[d * vs + t] = 0.0;
  b[3 * vs + t] = 0.0;
}

__global__ void __launch_bounds__(kUBlock) k_u_from_canon(long nslots, long vs, const int* __restrict__ canon,
                                                          int nnodes, const double* __restrict__ src,
                                                          double* __restrict__ dst) {
  const long t = (long)blockIdx.x * kUBlock + threadIdx.x;
  if (t >= nslots) return;
  const int q = canon[t];
  for (int f = 0; f < 4; ++f) dst[f * vs + t] = src[(size_t)f * nnodes + q];
}

__global__ void __launch_bounds__(kUBlock) k_u_to_canon(long nslots, long vs, const int* __restrict__ canon,
                                                        const unsigned char* __restrict__ fl, int nnodes,
                                                        const double* __restrict__ src, double* __restrict__ dst) {
  const long t = (long)blockIdx.x * kUBlock + threadIdx.x;
  if (t >= nslots || !(fl[t] & 1)) return;
  const int q = canon[t];
  for (int f = 0; f < 4; ++f) dst[(size_t)f * nnodes + q] = src[f * vs + t];
}

__global__ void __launch_bounds__(kUBlock) k_u_pfrom_canon(long nslots, const int* __restrict__ canon,
                                                           const double* __restrict__ src, double* __restrict__ p) {
  const long t = (long)blockIdx.x * kUBlock + threadIdx.x;
  if (t >= nslots) return;
  p[t] = src[canon[t]];
}

template <bool W, bool Y>
__global__ void __launch_bounds__(kUBlock) k_u_dot(long nslots, long vs, const unsigned char* __restrict__ fl,
                                                   const double* __restrict__ w, const double* __restrict__ x,
                                                   const double* __restrict__ y, int f0, int nf,
                                                   double* __restrict__ partial) {
  __shared__ double sa[kUBlock];
  double a = 0.0;
  for (long t = (long)blockIdx.x * kUBlock + threadIdx.x; t < nslots; t += (long)gridDim.x * kUBlock) {
    if (!(fl[t] & 1)) continue;
    for (int f = f0; f < f0 + nf; ++f) {
      const double v = x[f * vs + t] * (Y ? y[f * vs + t] : 1.0);
      a += W ? w[t] * v : v;
    }
  }
  sa[threadIdx.x] = a;
  __syncthreads();
  for (int s = kUBlock / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sa[threadIdx.x] += sa[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sa[0];
}

__global__ void __launch_bounds__(kUBlock) k_u_final(const double* __restrict__ partial, int nparts,
                                                     double* __restrict__ out) {
  __shared__ double sa[kUBlock];
  double a = 0.0;
  for (int q = threadIdx.x; q < nparts; q += kUBlock) a += partial[q];
  sa[threadIdx.x] = a;
  __syncthreads();
  for (int s = kUBlock / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sa[threadIdx.x] += sa[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sa[0];
}

__global__ void __launch_bounds__(kUBlock) k_u_shift(long nslots, double* __restrict__ p,
                                                     const double* __restrict__ sums, int slot, double denom) {
  const long t = (long)blockIdx.x * kUBlock + threadIdx.x;
  if (t >= nslots) return;
  p[t] -= sums[slot] / denom;
}

__global__ void __launch_bounds__(kUBlock) k_u_pscale(long nslots, double* __restrict__ p,
                                                      const double* __restrict__ sums, int slot) {
  const long t = (long)blockIdx.x * kUBlock + threadIdx.x;
  if (t >= nslots) return;
  p[t] *= 1.0 / sqrt(sums[slot]);
}

__global__ void __launch_bounds__(kUBlock) k_u_sync(ULev L, UList lst, double* __restrict__ x) {
  const int q = blockIdx.x * kUBlock + threadIdx.x;
  if (q >= lst.n) return;
  const int o0 = lst.off[q], o1 = lst.off[q + 1];
  int i, j, k;
  unpack(lst.occ[o0].y, i, j, k);
  const size_t own = (size_t)lst.occ[o0].x * L.P + uslot(i, j, k, L.n);
  double v[4];
  for (int f = 0; f < 4; ++f) v[f] = x[f * L.vs + own];
  for (int o = o0 + 1; o < o1; ++o) {
    const int2 oc = lst.occ[o];
    unpack(oc.y, i, j, k);
    const size_t sl = (size_t)oc.x * L.P + uslot(i, j, k, L.n);
    for (int f = 0; f < 4; ++f) x[f * L.vs + sl] = v[f];
  }
}

unsigned ublocks(long n) { return (unsigned)((n + kUBlock - 1) / kUBlock); }

// ---------------------------------------------------------- small levels
// One workgroup runs a whole smoothing call (iters Uzawa iterations, Sec.
// 3.2) on a small level: the phases of the launch-per-colour path -- every
// interface colour, then the four interior colours (xi sweeps, each also
// reversed for the symmetric variant), the pressure residual rows, the
// pressure step -- each a block-strided loop over the same per-node and
// per-point functions with the same lanes per node, phases separated by
// workgroup barriers, so every value is computed as there.  The cells'
// interior rows are staged in LDS once.  On the small levels a launch per
// phase is almost all launch latency.
constexpr int kUSmall = 1024;
constexpr int kUSmallCells = 64;  // LDS: 8 x 15 words per cell

struct USmallArgs {
  ULev L;
  UList lst;
  USegs inner, colour[4];
  const int* col_off;  // K + 1 offsets of the interface colours
  const int* col_sl;   // K occurrence slots per interface colour
  int K, list_sl;      // list_sl: occurrence slots of the whole list (residual rows)
  const double* dinv;
  double omega;
  int iters, xi, sym;
};

template <int SL>
__device__ void small_gs_iface(const ULev& L, const UList& lst, int first, int count, double* __restrict__ x,
                               const double* __restrict__ b) {
  constexpr int GW = kIfPts * SL;
  for (int t0 = 0; t0 < count; t0 += kUSmall / GW) {
    const int t = t0 + (int)threadIdx.x / GW;
    if (t < count) gs_iface_node<SL>(L, lst, first + t, (int)threadIdx.x % GW, x, b);
  }
}
template <int SL>
__device__ void small_presid_iface(const ULev& L, const UList& lst, const double* __restrict__ x,
                                   const double* __restrict__ b, double* __restrict__ r) {
  constexpr int GW = kIfPts * SL;
  for (int t0 = 0; t0 < lst.n; t0 += kUSmall / GW) {
    const int q = t0 + (int)threadIdx.x / GW;
    if (q < lst.n) apply_iface_node<true, false, SL>(L, lst, q, (int)threadIdx.x % GW, x, b, r, 12, 0, 1);
  }
}

__global__ void __launch_bounds__(kUSmall) k_u_smooth_small(USmallArgs a, double* __restrict__ x,
                                                            const double* __restrict__ b, double* __restrict__ r) {
  extern __shared__ double wall[];  // [cell][8][15]: A, B^T (3), B (3), M of class 0
  const ULev& L = a.L;
  const int ncell = L.ncell;
  for (int t = threadIdx.x; t < ncell * 8 * kUPoints; t += kUSmall) {
    const int c = t / (8 * kUPoints), q = (t / kUPoints) % 8, e = t % kUPoints;
    const UCell* cs = L.cs + c;
    double v;
    if (q == 0) v = cs->A[0][e];
    else if (q < 4) v = cs->BT[0][e][q - 1];
    else if (q < 7) v = cs->B[0][e][q - 4];
    else v = cs->M[0][e];
    wall[t] = v;
  }
  __syncthreads();
  auto rows = [&](int c) { return reinterpret_cast<const double(*)[kUPoints]>(wall + c * 8 * kUPoints); };
  auto colour = [&](int c) {
    if (c < a.K) {
      const int first = a.col_off[c], count = a.col_off[c + 1] - first, sl = a.col_sl[c];
      if (sl == 1)
        small_gs_iface<1>(L, a.lst, first, count, x, b);
      else if (sl == 2)
        small_gs_iface<2>(L, a.lst, first, count, x, b);
      else
        small_gs_iface<4>(L, a.lst, first, count, x, b);
    } else {
      const USegs sg = a.colour[c - a.K];
      const int lps = sg.lps, tot = ncell * sg.n;
      for (int w0 = 0; w0 < tot; w0 += kUSmall / lps) {
        const int w = w0 + (int)threadIdx.x / lps, lane = (int)threadIdx.x % lps;
        if (w < tot) {
          const int cc = w / sg.n;
          const int4 s = sg.s[w - cc * sg.n];
          if (lane < s.w) gs_inner_pt(L, cc, rows(cc), L.cs[cc].ainv0, s.x + 4 * lane, s.y, s.z, x, b);
        }
      }
    }
    __syncthreads();
  };
  const int ncol = a.K + 4;
  for (int it = 0; it < a.iters; ++it) {
    for (int sw = 0; sw < a.xi; ++sw) {
      for (int c = 0; c < ncol; ++c) colour(c);
      if (a.sym)
        for (int c = ncol - 1; c >= 0; --c) colour(c);
    }
    // r_p = g - B u + C p: interior points and interface nodes (disjoint slots)
    {
      const USegs sg = a.inner;
      const int lps = sg.lps, tot = ncell * sg.n;
      for (int w0 = 0; w0 < tot; w0 += kUSmall / lps) {
        const int w = w0 + (int)threadIdx.x / lps, lane = (int)threadIdx.x % lps;
        if (w < tot) {
          const int cc = w / sg.n;
          const int4 s = sg.s[w - cc * sg.n];
          if (lane < s.w)
            apply_inner_pt<true, false>(L, cc, rows(cc), L.cs[cc].cfac, s.x + lane, s.y, s.z, x, b, r, 12, 0, 1);
        }
      }
    }
    if (a.list_sl == 1)
      small_presid_iface<1>(L, a.lst, x, b, r);
    else if (a.list_sl == 2)
      small_presid_iface<2>(L, a.lst, x, b, r);
    else
      small_presid_iface<4>(L, a.lst, x, b, r);
    __syncthreads();
    // p -= omega r_p D^-1 on every slot
    const long ns = (long)ncell * L.P;
    for (long t = threadIdx.x; t < ns; t += kUSmall) x[3 * L.vs + t] -= a.omega * r[3 * L.vs + t] * a.dinv[t];
    __syncthreads();
  }
}
dim3 seg_grid(const USegs& s, int ncell) {
  const int per = kUBlock / s.lps;
  return dim3((unsigned)((s.n + per - 1) / per), (unsigned)ncell);
}
long real_slots(const ULev& L) { return (long)L.ncell * L.P; }
constexpr int kUPartials = 512;

}  // namespace

// Occurrence slots per node from the most occurrences of one node (1: 16
// lanes, 2: 32, more: 64, one wavefront).  Launches of many nodes are mostly
// face nodes (2 cells) and throughput-bound: 2 slots, whatever a few edge
// and vertex nodes of T_0 need (cube benchmark, interface rows of a level-7
// apply: 4 slots 0.374 ms, 2 slots 0.245 ms; the level-6 FMG solve 26.9 ->
// 26.4 ms with this rule at 8192 nodes, 26.5 at 4096, 26.6 at 32768).
int if_slots(int maxocc, int n) { return maxocc <= 1 ? 1 : ((maxocc <= 2 || n >= kIfManyNodes) ? 2 : 4); }

// Interface launch over n nodes with if_slots slots per node:
// f(std::integral_constant<int, SL>, grid).
template <typename F>
void if_launch(int maxocc, int n, F&& f) {
  auto grid = [n](int sl) { return dim3((unsigned)((n + if_nodes(sl) - 1) / if_nodes(sl))); };
  const int sl = if_slots(maxocc, n);
  if (sl == 1)
    f(std::integral_constant<int, 1>{}, grid(1));
  else if (sl == 2)
    f(std::integral_constant<int, 2>{}, grid(2));
  else
    f(std::integral_constant<int, 4>{}, grid(4));
}

void launch_u_apply_rows(hipStream_t s, const ULev& L, USegs inner, USegs zitems, const UList& lst, const double* x,
                         const double* b, double* y, int opmask, bool has_b, bool mass, bool wv, bool wp) {
  // k-marching from n = 64 on (cube benchmark FMG solve: from 32 26.2 ms,
  // from 64 25.6, from 128 25.8, never 25.8; on the small levels its chains
  // of dependent plane steps cost more than the row-segment gathers)
  if (inner.n > 0 && !mass && zitems.n > 0 && L.n >= 64) {
    KScope ks(s, KF_APPLY, (double)inner.pts * L.ncell);
    const dim3 g((unsigned)((zitems.n + kUBlock / 64 - 1) / (kUBlock / 64)), (unsigned)L.ncell);
    if (has_b)
      hipLaunchKernelGGL((k_u_apply_zm<true>), g, dim3(kUBlock), 0, s, L, zitems.s, zitems.n, x, b, y, opmask, (int)wv,
                         (int)wp);
    else
      hipLaunchKernelGGL((k_u_apply_zm<false>), g, dim3(kUBlock), 0, s, L, zitems.s, zitems.n, x, b, y, opmask,
                         (int)wv, (int)wp);
  } else if (inner.n > 0) {
    KScope ks(s, KF_APPLY, (double)inner.pts * L.ncell);
    const dim3 g = seg_grid(inner, L.ncell);
    if (mass)
      hipLaunchKernelGGL((k_u_apply_inner<false, true>), g, dim3(kUBlock), 0, s, L, inner, x, b, y, opmask, 1, 1);
    else if (has_b)
      hipLaunchKernelGGL((k_u_apply_inner<true, false>), g, dim3(kUBlock), 0, s, L, inner, x, b, y, opmask, (int)wv,
                         (int)wp);
    else
      hipLaunchKernelGGL((k_u_apply_inner<false, false>), g, dim3(kUBlock), 0, s, L, inner, x, b, y, opmask, (int)wv,
                         (int)wp);
  }
  if (lst.n > 0) {
    KScope ks(s, KF_IFACE, (double)lst.n);
    if_launch(lst.maxocc, lst.n, [&](auto sl, dim3 g) {
      constexpr int SL = decltype(sl)::value;
      if (mass)
        hipLaunchKernelGGL((k_u_apply_iface<false, true, SL>), g, dim3(kUBlock), 0, s, L, lst, x, b, y, opmask, 1, 1);
      else if (has_b)
        hipLaunchKernelGGL((k_u_apply_iface<true, false, SL>), g, dim3(kUBlock), 0, s, L, lst, x, b, y, opmask,
                           (int)wv, (int)wp);
      else
        hipLaunchKernelGGL((k_u_apply_iface<false, false, SL>), g, dim3(kUBlock), 0, s, L, lst, x, b, y, opmask,
                           (int)wv, (int)wp);
    });
  }
}

void launch_u_gs_inner(hipStream_t s, const ULev& L, USegs seg, double* x, const double* b) {
  if (seg.n == 0) return;
  KScope ks(s, KF_GS_VERTEX, (double)seg.pts * L.ncell);
  hipLaunchKernelGGL(k_u_gs_inner, seg_grid(seg, L.ncell), dim3(kUBlock), 0, s, L, seg, x, b);
}

void launch_u_gs_iface(hipStream_t s, const ULev& L, const UList& lst, int first, int count, int maxocc, double* x,
                       const double* b) {
  if (count <= 0) return;
  KScope ks(s, KF_IFACE, (double)count);
  if_launch(maxocc, count, [&](auto sl, dim3 g) {
    hipLaunchKernelGGL((k_u_gs_iface<decltype(sl)::value>), g, dim3(kUBlock), 0, s, L, lst, first, count, x, b);
  });
}

bool launch_u_smooth_small(hipStream_t s, const ULevelData& U, double* x, const double* b, double* r, int iters,
                           int xi, bool sym, double omega) {
  if (U.L.ncell > kUSmallCells || U.ncol_if > 64 || !U.col_off_d) return false;
  if (iters <= 0) return true;
  KScope ks(s, KF_SMALL, (double)real_slots(U.L));
  USmallArgs a{};
  a.L = U.L;
  a.lst = U.lst;
  a.inner = U.inner;
  for (int c = 0; c < 4; ++c) a.colour[c] = U.colour[c];
  a.col_off = U.col_off_d;
  a.col_sl = U.col_sl_d;
  a.K = U.ncol_if;
  a.list_sl = if_slots(U.lst.maxocc, U.lst.n);
  a.dinv = U.dinv;
  a.omega = omega;
  a.iters = iters;
  a.xi = xi;
  a.sym = sym;
  const size_t lds = (size_t)U.L.ncell * 8 * kUPoints * sizeof(double);
  hipLaunchKernelGGL(k_u_smooth_small, dim3(1), dim3(kUSmall), lds, s, a, x, b, r);
  return true;
}

void launch_u_pstep(hipStream_t s, const ULev& L, const double* dinv, double* x, const double* r, double omega) {
  const long n = real_slots(L);
  KScope ks(s, KF_PSTEP, (double)n);
  hipLaunchKernelGGL(k_u_pstep, dim3(ublocks(n)), dim3(kUBlock), 0, s, n, L.vs, dinv, x, r, omega);
}

void launch_u_restrict(hipStream_t s, const ULev& Lf, const ULev& Lc, USegs inner_c, const UList& lst_c,
                       const double* rf, double* rc) {
  KScope ks(s, KF_RESTRICT, (double)real_slots(Lc));
  if (inner_c.n > 0)
    hipLaunchKernelGGL(k_u_restrict_inner, seg_grid(inner_c, Lc.ncell), dim3(kUBlock), 0, s, Lf, Lc, inner_c, rf,
                       rc);
  if (lst_c.n > 0)
    if_launch(lst_c.maxocc, lst_c.n, [&](auto sl, dim3 g) {
      hipLaunchKernelGGL((k_u_restrict_iface<decltype(sl)::value>), g, dim3(kUBlock), 0, s, Lf, Lc, lst_c, rf, rc);
    });
}

void launch_u_prolong(hipStream_t s, const ULev& Lc, const ULev& Lf, USegs all_f, const double* xc, double* xf,
                      bool add, bool skip_bnd) {
  if (all_f.n == 0) return;
  KScope ks(s, KF_PROLONG, (double)real_slots(Lf));
  hipLaunchKernelGGL(k_u_prolong, seg_grid(all_f, Lf.ncell), dim3(kUBlock), 0, s, Lc, Lf, all_f, xc, xf, (int)add,
                     (int)skip_bnd);
}

void launch_u_inject(hipStream_t s, const ULev& Lf, const ULev& Lc, USegs all_c, const double* xf, double* xc) {
  if (all_c.n == 0) return;
  KScope ks(s, KF_OTHER, (double)real_slots(Lc));
  hipLaunchKernelGGL(k_u_inject, seg_grid(all_c, Lc.ncell), dim3(kUBlock), 0, s, Lf, Lc, all_c, xf, xc);
}

void launch_u_copy_bnd(hipStream_t s, const ULev& L, const unsigned char* flags, const double* src, double* dst) {
  const long n = real_slots(L);
  KScope ks(s, KF_OTHER, (double)n);
  hipLaunchKernelGGL(k_u_copy_bnd, dim3(ublocks(n)), dim3(kUBlock), 0, s, n, L.vs, flags, src, dst);
}

void launch_u_rhs_fix(hipStream_t s, const ULev& L, const unsigned char* flags, double* b) {
  const long n = real_slots(L);
  KScope ks(s, KF_OTHER, (double)n);
  hipLaunchKernelGGL(k_u_rhs_fix, dim3(ublocks(n)), dim3(kUBlock), 0, s, n, L.vs, flags, b);
}

void launch_u_from_canon(hipStream_t s, const ULev& L, const int* canon, int nnodes, const double* src, double* dst) {
  const long n = real_slots(L);
  KScope ks(s, KF_OTHER, (double)n);
  hipLaunchKernelGGL(k_u_from_canon, dim3(ublocks(n)), dim3(kUBlock), 0, s, n, L.vs, canon, nnodes, src, dst);
}

void launch_u_to_canon(hipStream_t s, const ULev& L, const int* canon, const unsigned char* flags, int nnodes,
                       const double* src, double* dst) {
  const long n = real_slots(L);
  KScope ks(s, KF_OTHER, (double)n);
  hipLaunchKernelGGL(k_u_to_canon, dim3(ublocks(n)), dim3(kUBlock), 0, s, n, L.vs, canon, flags, nnodes, src, dst);
}

void launch_u_pfrom_canon(hipStream_t s, const ULev& L, const int* canon, const double* src, double* p) {
  const long n = real_slots(L);
  KScope ks(s, KF_OTHER, (double)n);
  hipLaunchKernelGGL(k_u_pfrom_canon, dim3(ublocks(n)), dim3(kUBlock), 0, s, n, canon, src, p);
}

void launch_u_dot(hipStream_t s, const ULev& L, const unsigned char* flags, const double* w, const double* x,
                  const double* y, int f0, int nf, double* partial, double* sums, int out) {
  const long n = real_slots(L);
  const unsigned nb = std::min<unsigned>(ublocks(n), kUPartials);
  KScope ks(s, KF_REDUCE, (double)n);
  if (w && y)
    hipLaunchKernelGGL((k_u_dot<true, true>), dim3(nb), dim3(kUBlock), 0, s, n, L.vs, flags, w, x, y, f0, nf, partial);
  else if (w)
    hipLaunchKernelGGL((k_u_dot<true, false>), dim3(nb), dim3(kUBlock), 0, s, n, L.vs, flags, w, x, y, f0, nf,
                       partial);
  else if (y)
    hipLaunchKernelGGL((k_u_dot<false, true>), dim3(nb), dim3(kUBlock), 0, s, n, L.vs, flags, w, x, y, f0, nf,
                       partial);
  else
    hipLaunchKernelGGL((k_u_dot<false, false>), dim3(nb), dim3(kUBlock), 0, s, n, L.vs, flags, w, x, y, f0, nf,
                       partial);
  hipLaunchKernelGGL(k_u_final, dim3(1), dim3(kUBlock), 0, s, partial, (int)nb, sums + out);
}

void launch_u_shift(hipStream_t s, const ULev& L, double* p, const double* sums, int slot, double denom) {
  const long n = real_slots(L);
  KScope ks(s, KF_OTHER, (double)n);
  hipLaunchKernelGGL(k_u_shift, dim3(ublocks(n)), dim3(kUBlock), 0, s, n, p, sums, slot, denom);
}

void launch_u_pscale(hipStream_t s, const ULev& L, double* p, const double* sums, int slot) {
  const long n = real_slots(L);
  KScope ks(s, KF_OTHER, (double)n);
  hipLaunchKernelGGL(k_u_pscale, dim3(ublocks(n)), dim3(kUBlock), 0, s, n, p, sums, slot);
}

void launch_u_sync(hipStream_t s, const ULev& L, const UList& lst, double* x) {
  if (lst.n == 0) return;
  KScope ks(s, KF_IFACE, (double)lst.n);
  hipLaunchKernelGGL(k_u_sync, dim3(ublocks(lst.n)), dim3(kUBlock), 0, s, L, lst, x);
}

}  // namespace hhg
