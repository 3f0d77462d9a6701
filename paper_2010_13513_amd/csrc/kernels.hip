// HIP kernels of libhhg for gfx950: matrix-free stencil application,
// multicolour Gauss-Seidel, Uzawa pressure step, grid transfer, reductions.
//
// Data layout (see include/hhg.h): every lattice array has nn = (N+1)^3 words
// indexed i + n1 (j + n1 k); one thread per array index, consecutive threads
// along i, so every stencil neighbour load of a wavefront is a contiguous run.
// Stencil weights are constant per row type (paper Sec. 2.1) and are read from
// small device tables with wavefront-uniform addresses (scalar loads).
#include <type_traits>
#include <vector>

#include <hip/hip_ext.h>

#include "kernels.h"
#include "lanes.h"

namespace hhg {
namespace gen {
// One word of a buffer (raw buffer load, bounds-checked by the resource: an
// offset outside it reads 0).
template <typename T>
__device__ __forceinline__ T buffer_word(__amdgpu_buffer_rsrc_t r, int voff, int soff);
template <>
__device__ __forceinline__ double buffer_word<double>(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
template <>
__device__ __forceinline__ float buffer_word<float>(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
// Buffer resource over n bytes from p (gfx9 word 3: 32-bit data format).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, unsigned n) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)n, 0x00020000);
}
}  // namespace gen
}  // namespace hhg

namespace hhg {
namespace gen {
// Order points of the k-marching plane step.  The compiler otherwise makes
// the lane-shifted copies of every loaded word right after the loads and the
// multiply-adds much later, holding all copies at once (about 40 registers).
// An empty volatile asm that takes the accumulators (zm_order) and the next
// word (zm_word) as in/out register operands fixes the order word by word:
// it emits no instruction and touches no memory.
template <typename T, int R>
__device__ __forceinline__ void zm_order(T (&acc)[3][R]) {
#pragma unroll
  for (int s = 0; s < 3; ++s)
#pragma unroll
    for (int r = 0; r < R; ++r) asm volatile("" : "+v"(acc[s][r]));
}
template <typename T>
__device__ __forceinline__ T zm_word(T v) {
  asm volatile("" : "+v"(v));
  return v;
}
}  // namespace gen
}  // namespace hhg

#include "generated/stencils.inc"

namespace hhg {
namespace {

constexpr int kBlock = 256;

__device__ __forceinline__ void decode(int t, int n1, int& i, int& j, int& k) {
  i = t % n1;
  const int r = t / n1;
  j = r % n1;
  k = r / n1;
}
// parity class of velocity group g (0: vertex, 1..7: edge directions)
__device__ __forceinline__ int gdx(int g) { return (0xB2 >> g) & 1; }
__device__ __forceinline__ int gdy(int g) { return (0xD4 >> g) & 1; }
__device__ __forceinline__ int gdz(int g) { return (0xE8 >> g) & 1; }

template <int G>
__device__ __forceinline__ bool vel_interior(int g, int i, int j, int k, int N) {
  const int dx = G == 1 ? 0 : gdx(g), dy = G == 1 ? 0 : gdy(g), dz = G == 1 ? 0 : gdz(g);
  return i >= 1 - dx && j >= 1 - dy && k >= 1 - dz && i <= N - 1 && j <= N - 1 && k <= N - 1;
}
// velocity site exists (not padding): doubled position 2(i,j,k) + dir inside [0, 2N]
template <int G>
__device__ __forceinline__ bool vel_exists(int g, int i, int j, int k, int N) {
  if (G == 1) return true;
  return i + gdx(g) <= N && j + gdy(g) <= N && k + gdz(g) <= N;
}
__device__ __forceinline__ int bcls3(int c, int N) { return c == 0 ? 0 : (c == N ? 2 : 1); }

// Faces of the cube a velocity site lies on (bit f as in Geom::nf), from its
// position in site units (doubled for P2).
__device__ __forceinline__ int site_faces(int X, int Y, int Z, int M) {
  return (X == 0) | ((X == M) << 1) | ((Y == 0) << 2) | ((Y == M) << 3) | ((Z == 0) << 4) | ((Z == M) << 5);
}
// The velocity site is an unknown: it exists and lies on no Dirichlet face
// (interior sites, and sites whose faces are all outflow faces).
template <int G>
__device__ __forceinline__ bool vel_unknown(const Geom& g, int gr, int i, int j, int k) {
  if (!vel_exists<G>(gr, i, j, k, g.N)) return false;
  const int f = G == 1 ? site_faces(i, j, k, g.N)
                       : site_faces(2 * i + gdx(gr), 2 * j + gdy(gr), 2 * k + gdz(gr), 2 * g.N);
  return (f & ~g.nf) == 0;
}

unsigned nblocks(size_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// ------------------------------------------------------------ event timer
struct TimerRec {
  int fam;
  hipEvent_t a, b;
  double units;
};
struct Timer {
  unsigned mask = 0;
  std::vector<TimerRec> recs;
};
Timer& timer() {
  static Timer t;
  return t;
}
}  // namespace

KScope::KScope(hipStream_t s, int fam, double units, bool packet) : s_(s) {
  Timer& t = timer();
  if (!((t.mask >> fam) & 1u)) return;
  TimerRec r{fam, nullptr, nullptr, units};
  if (hipEventCreate(&r.a) != hipSuccess || hipEventCreate(&r.b) != hipSuccess) return;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  packet_ = packet && hipStreamIsCapturing(s, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone;
  if (packet_)
    a_ = r.a;
  else
    (void)hipEventRecord(r.a, s);
  b_ = r.b;
  t.recs.push_back(r);
}
KScope::~KScope() {
  if (b_ && !packet_) (void)hipEventRecord(b_, s_);
}

namespace {

// ------------------------------------------------------- generated stencils
// Dispatch of the generated interior row stencils by velocity group (the group
// is uniform per workgroup, so the switch is a scalar branch).
template <typename T, int G>
struct Rows;

template <typename T>
struct Rows<T, 1> {
  static __device__ __forceinline__ void A(int, const T* u0, const T* u1, const T* u2, int pos, int s1, int s2, int nn,
                                           T& a0, T& a1, T& a2) {
    gen::p1_A_g0<T>(u0, u1, u2, pos, s1, s2, nn, a0, a1, a2);
  }
  static __device__ __forceinline__ void M(int, const T* u0, const T* u1, const T* u2, int pos, int s1, int s2, int nn,
                                           T& a0, T& a1, T& a2) {
    gen::p1_M_g0<T>(u0, u1, u2, pos, s1, s2, nn, a0, a1, a2);
  }
  static __device__ __forceinline__ void BT(int, const T* p, int pos, int s1, int s2, T& a0, T& a1, T& a2) {
    gen::p1_BT_g0<T>(p, pos, s1, s2, a0, a1, a2);
  }
  static __device__ __forceinline__ void B(const T* u0, const T* u1, const T* u2, int pos, int s1, int s2, int nn,
                                           T& a) {
    gen::p1_B<T>(u0, u1, u2, pos, s1, s2, nn, a);
  }
  static __device__ __forceinline__ void C(const T* p, int pos, int s1, int s2, T& a) {
    gen::p1_C<T>(p, pos, s1, s2, a);
  }
  static __device__ __forceinline__ void Anu(int, const T* u0, const T* u1, const T* u2, const T* nu, int pos, int idx,
                                             int s1, int s2, int nn, T& a0, T& a1, T& a2) {
    gen::p1_Anu_g0<T>(u0, u1, u2, nu, pos, idx, s1, s2, nn, a0, a1, a2);
  }
  static __device__ __forceinline__ T Anudiag(int, const T* nu, int idx, int s1, int s2) {
    return gen::p1_Anudiag_g0<T>(nu, idx, s1, s2);
  }
};

#define HHG_P2_CASES(F, ...)        \
  switch (g) {                      \
    case 0: gen::F##_g0<T>(__VA_ARGS__); break; \
    case 1: gen::F##_g1<T>(__VA_ARGS__); break; \
    case 2: gen::F##_g2<T>(__VA_ARGS__); break; \
    case 3: gen::F##_g3<T>(__VA_ARGS__); break; \
    case 4: gen::F##_g4<T>(__VA_ARGS__); break; \
    case 5: gen::F##_g5<T>(__VA_ARGS__); break; \
    case 6: gen::F##_g6<T>(__VA_ARGS__); break; \
    default: gen::F##_g7<T>(__VA_ARGS__); break; \
  }

template <typename T>
struct Rows<T, 8> {
  static __device__ __forceinline__ void A(int g, const T* u0, const T* u1, const T* u2, int pos, int s1, int s2,
                                           int nn, T& a0, T& a1, T& a2) {
    HHG_P2_CASES(p2_A, u0, u1, u2, pos, s1, s2, nn, a0, a1, a2)
  }
  static __device__ __forceinline__ void M(int g, const T* u0, const T* u1, const T* u2, int pos, int s1, int s2,
                                           int nn, T& a0, T& a1, T& a2) {
    HHG_P2_CASES(p2_M, u0, u1, u2, pos, s1, s2, nn, a0, a1, a2)
  }
  static __device__ __forceinline__ void BT(int g, const T* p, int pos, int s1, int s2, T& a0, T& a1, T& a2) {
    HHG_P2_CASES(p2_BT, p, pos, s1, s2, a0, a1, a2)
  }
  static __device__ __forceinline__ void B(const T* u0, const T* u1, const T* u2, int pos, int s1, int s2, int nn,
                                           T& a) {
    gen::p2_B<T>(u0, u1, u2, pos, s1, s2, nn, a);
  }
  static __device__ __forceinline__ void C(const T*, int, int, int, T&) {}
  static __device__ __forceinline__ void Anu(int g, const T* u0, const T* u1, const T* u2, const T* nu, int pos,
                                             int idx, int s1, int s2, int nn, T& a0, T& a1, T& a2) {
    HHG_P2_CASES(p2_Anu, u0, u1, u2, nu, pos, idx, s1, s2, nn, a0, a1, a2)
  }
  static __device__ __forceinline__ T Anudiag(int g, const T* nu, int idx, int s1, int s2) {
    T d = 0;
    switch (g) {
      case 0: d = gen::p2_Anudiag_g0<T>(nu, idx, s1, s2); break;
      case 1: d = gen::p2_Anudiag_g1<T>(nu, idx, s1, s2); break;
      case 2: d = gen::p2_Anudiag_g2<T>(nu, idx, s1, s2); break;
      case 3: d = gen::p2_Anudiag_g3<T>(nu, idx, s1, s2); break;
      case 4: d = gen::p2_Anudiag_g4<T>(nu, idx, s1, s2); break;
      case 5: d = gen::p2_Anudiag_g5<T>(nu, idx, s1, s2); break;
      case 6: d = gen::p2_Anudiag_g6<T>(nu, idx, s1, s2); break;
      default: d = gen::p2_Anudiag_g7<T>(nu, idx, s1, s2); break;
    }
    return d;
  }
};

// ---------------------------------------------------------------- apply
// Logical block index with a contiguous range of blocks per XCD: the 8 XCDs
// receive workgroups round-robin, so block b runs on XCD b % 8; remapping
// gives each XCD one contiguous slab of the lattice, and the k +- 1 planes a
// stencil reads stay in that XCD's L2.  grid must be a multiple of 8.
__device__ __forceinline__ int xcd_block() {
  const int per = gridDim.x >> 3;
  return (blockIdx.x & 7) * per + (blockIdx.x >> 3);
}
unsigned nblocks8(size_t n) { return (unsigned)(((n + kBlock - 1) / kBlock + 7) & ~(size_t)7); }
// The same remap over the first nmain blocks of a grid (nmain a multiple of 8).
__device__ __forceinline__ int xcd_block_of(int nmain) {
  const int per = nmain >> 3;
  return (blockIdx.x & 7) * per + (blockIdx.x >> 3);
}

// Pressure rows of the boundary nodes, run by the extra blocks appended to an
// apply launch (blocks nmain.. of the grid, block size bs): they overlap the
// interior rows instead of taking a launch of their own.
template <typename T, int G>
__device__ __forceinline__ void prow_bnd_block(const Geom& g, const LevelConst<T>& lc, const T* __restrict__ x,
                                               const T* __restrict__ b, T* __restrict__ y, int opmask, int has_b,
                                               const int* __restrict__ bnd, int nbnd, int nmain, int bs,
                                               PStep<T> ps);

// Pressure row value at any node t = (i, j, k): interior rows from the
// generated interior stencils, boundary rows from the generated per-class
// stencils (cls = c_i + 3 c_j + 9 c_k, c = 0 low face, 1 inside, 2 high
// face): B u (opmask 4) and -C p (8) or +C p (8 | 16) for PSPG, summed over
// the elements inside the cube.
#define HHG_BCLS_CASES(D, X)                                                                              \
  switch (cls) {                                                                                          \
    case 0: X(D, 0); break;   case 1: X(D, 1); break;   case 2: X(D, 2); break;   case 3: X(D, 3); break;   \
    case 4: X(D, 4); break;   case 5: X(D, 5); break;   case 6: X(D, 6); break;   case 7: X(D, 7); break;   \
    case 8: X(D, 8); break;   case 9: X(D, 9); break;   case 10: X(D, 10); break; case 11: X(D, 11); break; \
    case 12: X(D, 12); break; case 14: X(D, 14); break; case 15: X(D, 15); break; case 16: X(D, 16); break; \
    case 17: X(D, 17); break; case 18: X(D, 18); break; case 19: X(D, 19); break; case 20: X(D, 20); break; \
    case 21: X(D, 21); break; case 22: X(D, 22); break; case 23: X(D, 23); break; case 24: X(D, 24); break; \
    case 25: X(D, 25); break; default: X(D, 26); break;                                                   \
  }
#define HHG_BROW(D, C) gen::D##_Bc##C<T>(u0, u1, u2, t, s1, s2, nn, ab)
#define HHG_CROW(D, C) gen::D##_Cc##C<T>(p, t, s1, s2, ac)
#define HHG_BROW_D0(D, C) gen::D##_Bc##C##_d0<T>(ud, t, s1, s2, nn, ab)
#define HHG_BROW_D1(D, C) gen::D##_Bc##C##_d1<T>(ud, t, s1, s2, nn, ab)
#define HHG_BROW_D2(D, C) gen::D##_Bc##C##_d2<T>(ud, t, s1, s2, nn, ab)
template <typename T, int G>
__device__ __forceinline__ T prow_value(const Geom& g, const LevelConst<T>& lc, const T* __restrict__ x, int opmask,
                                        int t, int i, int j, int k) {
  const int N = g.N, s1 = g.n1, s2 = g.n1 * g.n1, nn = g.nn;
  const T* __restrict__ u0 = x;
  const T* __restrict__ u1 = x + g.vstride;
  const T* __restrict__ u2 = x + 2 * g.vstride;
  const T* __restrict__ p = x + 3 * g.vstride;
  T ab = 0, ac = 0;
  if (i >= 1 && j >= 1 && k >= 1 && i <= N - 1 && j <= N - 1 && k <= N - 1) {
    if (opmask & 4) Rows<T, G>::B(u0, u1, u2, t, s1, s2, nn, ab);
    if (opmask & 24) Rows<T, G>::C(p, t, s1, s2, ac);
  } else {
    const int cls = bcls3(i, N) + 3 * bcls3(j, N) + 9 * bcls3(k, N);
    if (opmask & 4) {
      if constexpr (G == 1) {
        HHG_BCLS_CASES(p1, HHG_BROW)
      } else {
        HHG_BCLS_CASES(p2, HHG_BROW)
      }
    }
    if constexpr (G == 1)
      if (opmask & 24) HHG_BCLS_CASES(p1, HHG_CROW)
  }
  return lc.b * ab + ((opmask & 16) ? lc.c * ac : -lc.c * ac);
}
#undef HHG_BROW

// One velocity row type (group GR) of the apply at array index t.
template <typename T, int G, int GR, bool VAR>
__device__ __forceinline__ void apply_vrow(const Geom& g, const LevelConst<T>& lc, const T* __restrict__ x,
                                           const T* __restrict__ b, T* __restrict__ y, int opmask, int has_b, int t,
                                           int i, int j, int k) {
  const int s1 = g.n1, s2 = g.n1 * g.n1, nn = g.nn;
  const T* __restrict__ u0 = x;
  const T* __restrict__ u1 = x + g.vstride;
  const T* __restrict__ u2 = x + 2 * g.vstride;
  const T* __restrict__ p = x + 3 * g.vstride;
  const bool in = vel_interior<G>(GR, i, j, k, g.N);
  const int pos = GR * nn + t;
  T r0 = 0, r1 = 0, r2 = 0;
  if (in) {
    T a0 = 0, a1 = 0, a2 = 0, c0 = 0, c1 = 0, c2 = 0;
    if (opmask & 1) {
      if constexpr (VAR)
        Rows<T, G>::Anu(GR, u0, u1, u2, lc.nu, pos, t, s1, s2, nn, a0, a1, a2);
      else
        Rows<T, G>::A(GR, u0, u1, u2, pos, s1, s2, nn, a0, a1, a2);
    }
    if (opmask & 2) Rows<T, G>::BT(GR, p, t, s1, s2, c0, c1, c2);
    r0 = lc.a * a0 + lc.b * c0;
    r1 = lc.a * a1 + lc.b * c1;
    r2 = lc.a * a2 + lc.b * c2;
    if (has_b) {
      r0 = b[pos] - r0;
      r1 = b[g.vstride + pos] - r1;
      r2 = b[2 * g.vstride + pos] - r2;
    }
  }
  y[pos] = r0;
  y[g.vstride + pos] = r1;
  y[2 * g.vstride + pos] = r2;
}

template <typename T, int G, int GR, bool VAR>
__device__ __forceinline__ void apply_vrows(const Geom& g, const LevelConst<T>& lc, const T* x, const T* b, T* y,
                                            int opmask, int has_b, int t, int i, int j, int k) {
  apply_vrow<T, G, GR, VAR>(g, lc, x, b, y, opmask, has_b, t, i, j, k);
  if constexpr (GR + 1 < G) apply_vrows<T, G, GR + 1, VAR>(g, lc, x, b, y, opmask, has_b, t, i, j, k);
}

// y = [b -] op x on every row type at array index t: the G velocity groups
// (zero rows where the site is not an interior velocity DoF) and the interior
// pressure row (boundary pressure rows: extra blocks, prow_bnd_block).  opmask bits: 1 A, 2 B^T,
// 4 B, 8 -C (block of calA), 16: +C instead.
template <typename T, int G, bool VAR>
__device__ __forceinline__ void apply_site(const Geom& g, const LevelConst<T>& lc, const T* __restrict__ x,
                                           const T* __restrict__ b, T* __restrict__ y, int opmask, int has_b,
                                           int vel_rows, int p_rows, int t) {
  int i, j, k;
  decode(t, g.n1, i, j, k);
  const int N = g.N;
  if (vel_rows) apply_vrows<T, G, 0, VAR>(g, lc, x, b, y, opmask, has_b, t, i, j, k);
  if (p_rows && i >= 1 && j >= 1 && k >= 1 && i <= N - 1 && j <= N - 1 && k <= N - 1) {  // boundary: prow_bnd_block
    const T acc = prow_value<T, G>(g, lc, x, opmask, t, i, j, k);
    const int pp = 3 * g.vstride + t;
    y[pp] = has_b ? b[pp] - acc : acc;
  }
}
template <typename T, int G, bool VAR>
__global__ void __launch_bounds__(kBlock) k_apply(Geom g, LevelConst<T> lc, const T* __restrict__ x,
                                                  const T* __restrict__ b, T* __restrict__ y, int opmask, int has_b,
                                                  int vel_rows, int p_rows, const int* __restrict__ bnd, int nbnd,
                                                  int nmain) {
  if ((int)blockIdx.x >= nmain) {
    prow_bnd_block<T, G>(g, lc, x, b, y, opmask, has_b, bnd, nbnd, nmain, kBlock, PStep<T>{});
    return;
  }
  const int t = xcd_block_of(nmain) * kBlock + threadIdx.x;
  if (t >= g.nn) return;
  apply_site<T, G, VAR>(g, lc, x, b, y, opmask, has_b, vel_rows, p_rows, t);
}

// k-marching apply of the whole constant-coefficient operator (A, B^T, B and
// -C; y = calA x or b - calA x).  A block is three wavefronts over the same
// 64 consecutive lattice columns (linear index i + n1 j) of one chunk of
// k-planes [k0, k1); wavefront d computes the velocity rows of component d.
// For kp = k0 - 1 .. k1 each wavefront loads the words of columns (i, j + dj)
// its rows need, takes the i -+ 1 neighbours from the adjacent lanes, and
// scatters them into the rows of its lane's column at k = kp - dk, kept in
// three rotating accumulator planes; the row plane kp - 1 is complete after
// plane kp and is written.  The first and last lane lack a shifted
// neighbour, so windows overlap by two columns and only lanes 1..62 write.
// The pressure row is the sum of the three wavefronts' parts, added through
// LDS.  Per P2 site this issues 69 / 8 loads instead of one per stencil entry.
constexpr int kZmCols = 64;
#ifndef HHG_ZM_KC
#define HHG_ZM_KC 20  // k-planes per chunk (the chunk re-reads 2 halo planes); 20 measured best of 8..48
#endif
constexpr int kZmOut = kZmCols - 2;  // columns written per window
constexpr unsigned kZmF32Lds = 50000;  // dynamic LDS of the large-lattice P2-P1 launch: 3 workgroups per CU

template <typename T, int G, int D, int Q>
__device__ __forceinline__ void zm_plane(__amdgpu_buffer_rsrc_t ru, __amdgpu_buffer_rsrc_t rp, const int (&vo)[3],
                                         int nnb, T rt, T rc, T (&acc)[3][G + 1]) {
#define HHG_ZM(P) gen::P<T>(ru, rp, vo, nnb, rt, rc, acc)
  if constexpr (G == 1) {
    if constexpr (D == 0 && Q == 0) HHG_ZM(p1_zm0_q0);
    if constexpr (D == 0 && Q == 1) HHG_ZM(p1_zm0_q1);
    if constexpr (D == 0 && Q == 2) HHG_ZM(p1_zm0_q2);
    if constexpr (D == 1 && Q == 0) HHG_ZM(p1_zm1_q0);
    if constexpr (D == 1 && Q == 1) HHG_ZM(p1_zm1_q1);
    if constexpr (D == 1 && Q == 2) HHG_ZM(p1_zm1_q2);
    if constexpr (D == 2 && Q == 0) HHG_ZM(p1_zm2_q0);
    if constexpr (D == 2 && Q == 1) HHG_ZM(p1_zm2_q1);
    if constexpr (D == 2 && Q == 2) HHG_ZM(p1_zm2_q2);
  } else {
    if constexpr (D == 0 && Q == 0) HHG_ZM(p2_zm0_q0);
    if constexpr (D == 0 && Q == 1) HHG_ZM(p2_zm0_q1);
    if constexpr (D == 0 && Q == 2) HHG_ZM(p2_zm0_q2);
    if constexpr (D == 1 && Q == 0) HHG_ZM(p2_zm1_q0);
    if constexpr (D == 1 && Q == 1) HHG_ZM(p2_zm1_q1);
    if constexpr (D == 1 && Q == 2) HHG_ZM(p2_zm1_q2);
    if constexpr (D == 2 && Q == 0) HHG_ZM(p2_zm2_q0);
    if constexpr (D == 2 && Q == 1) HHG_ZM(p2_zm2_q1);
    if constexpr (D == 2 && Q == 2) HHG_ZM(p2_zm2_q2);
  }
#undef HHG_ZM
}

// Column of a lane: nb[dj + 1] = array index of column (i, j + dj) clamped
// into the array, so every load stays in it; rows fed by a clamped (or
// row-wrapped) word are never interior.  `valid`: the lane writes its column.
template <typename T>
struct ZmCol {
  int col, i, j, k0, k1;
  int nb[3];
  bool valid;
  T rt, rc;  // pressure-word scales of the B^T and C entries
  T sv, sp;  // units of the accumulated velocity and pressure rows
};

template <typename T, int G, int D, int Q, bool VEL, bool HB>
__device__ __forceinline__ void zm_step(const Geom& g, const LevelConst<T>& lc, const T* __restrict__ x,
                                        const T* __restrict__ b, T* __restrict__ y, const ZmCol<T>& c, int q,
                                        T (&acc)[3][G + 1], T (*pshare)[3][kZmCols], const PStep<T>& ps) {
  constexpr int S = (Q + 2) % 3;  // slot of the row plane completed by this step
  const int N = g.N, s1 = g.n1, s2 = g.n1 * g.n1, nn = g.nn, vs = g.vstride;
  const int kp = c.k0 - 1 + q;
  const int kr = kp - 1;
  const int kps = min(max(kp, 0), N) * s2;
  const int vo[3] = {(c.nb[0] + kps) * (int)sizeof(T), (c.nb[1] + kps) * (int)sizeof(T),
                     (c.nb[2] + kps) * (int)sizeof(T)};
  const __amdgpu_buffer_rsrc_t ru = gen::make_rsrc(x + (size_t)D * vs, (unsigned)((size_t)vs * sizeof(T)));
  const __amdgpu_buffer_rsrc_t rp = gen::make_rsrc(x + (size_t)3 * vs, (unsigned)((size_t)nn * sizeof(T)));
  // residual: the b words of the row this step completes are loaded before
  // the plane's multiply-adds, so their latency hides behind them instead of
  // adding a round trip before the stores (address clamped into the lattice;
  // only the rows written use them)
  T bv[G + 1];
  if constexpr (HB) {
    const int atc = c.nb[1] + min(max(kr, 0), N) * s2;
#pragma unroll
    for (int gr = 0; gr < G; ++gr) bv[gr] = VEL ? b[D * vs + gr * nn + atc] : T(0);
    bv[G] = D == 0 ? b[3 * vs + atc] : T(0);
  }
  zm_plane<T, G, D, Q>(ru, rp, vo, nn * (int)sizeof(T), c.rt, c.rc, acc);
  if constexpr (HB) {
#pragma unroll
    for (int r = 0; r <= G; ++r) asm volatile("" : "+v"(bv[r]));  // keep the loads above (not sunk to the stores)
  }
  (void)s1;
  const int lane = threadIdx.x & (kZmCols - 1);
  if (kr >= c.k0 && kr < c.k1) {  // uniform over the block
    const int at = c.col + kr * s2;
    if (VEL && c.valid) {
#pragma unroll
      for (int gr = 0; gr < G; ++gr) {
        const int pos = D * vs + gr * nn + at;
        const T v = c.sv * acc[S][gr];
        y[pos] = vel_interior<G>(gr, c.i, c.j, kr, N) ? (HB ? bv[gr] - v : v) : T(0);
      }
    }
    pshare[q & 1][D][lane] = acc[S][G];
    __syncthreads();
    if (D == 0 && c.valid && c.i >= 1 && c.j >= 1 && kr >= 1 && c.i <= N - 1 && c.j <= N - 1 && kr <= N - 1) {
      const T v = c.sp * (pshare[q & 1][0][lane] + pshare[q & 1][1][lane] + pshare[q & 1][2][lane]);
      const int pp = 3 * vs + at;
      const T r = HB ? bv[G] - v : v;
      if (HB && !VEL && ps.p)
        ps.p[at] -= ps.omega * ps.dinv[at] * r;
      else
        y[pp] = r;
    }
  }
#pragma unroll
  for (int r = 0; r <= G; ++r) acc[S][r] = T(0);
}

template <typename T, int G, int D, bool VEL, bool HB>
__device__ __forceinline__ void zm_run(const Geom& g, const LevelConst<T>& lc, const T* __restrict__ x,
                                       const T* __restrict__ b, T* __restrict__ y, const ZmCol<T>& c,
                                       T (*pshare)[3][kZmCols], const PStep<T>& ps) {
  T acc[3][G + 1];
#pragma unroll
  for (int s = 0; s < 3; ++s)
#pragma unroll
    for (int r = 0; r <= G; ++r) acc[s][r] = T(0);
  const int nq = c.k1 - c.k0 + 2;
  for (int q = 0; q < nq; q += 3) {
    zm_step<T, G, D, 0, VEL, HB>(g, lc, x, b, y, c, q, acc, pshare, ps);
    if (q + 1 < nq) zm_step<T, G, D, 1, VEL, HB>(g, lc, x, b, y, c, q + 1, acc, pshare, ps);
    if (q + 2 < nq) zm_step<T, G, D, 2, VEL, HB>(g, lc, x, b, y, c, q + 2, acc, pshare, ps);
  }
}

template <typename T, int G>
__device__ __forceinline__ void prow_bnd_split(const Geom& g, const LevelConst<T>& lc, const T* __restrict__ x,
                                               const T* __restrict__ b, T* __restrict__ y, int has_b,
                                               const int* __restrict__ bnd, int nbnd, int nmain, PStep<T> ps,
                                               T (*red)[kZmCols]);

template <typename T, int G, bool VEL, bool HB>
__global__ void __launch_bounds__(3 * kZmCols) k_apply_zm(Geom g, LevelConst<T> lc, const T* __restrict__ x,
                                                          const T* __restrict__ b, T* __restrict__ y, int kc, int ncb,
                                                          const int* __restrict__ bnd, int nbnd, int nmain,
                                                          PStep<T> ps) {
  __shared__ T pshare[2][3][kZmCols];
  if ((int)blockIdx.x >= nmain) {
    prow_bnd_split<T, G>(g, lc, x, b, y, (int)HB, bnd, nbnd, nmain, ps, pshare[0]);
    return;
  }
  const int lin = xcd_block_of(nmain);
  const int cb = lin % ncb, chunk = lin / ncb;
  const int n1 = g.n1, N = g.N;
  ZmCol<T> c;
  {
    const int* den = G == 1 ? gen::p1_zm_den : gen::p2_zm_den;  // A, B^T, B, C
    c.rt = (lc.b * T(den[0])) / (lc.a * T(den[1]));
    c.rc = (lc.c * T(den[2])) / (lc.b * T(den[3]));
    c.sv = lc.a / T(den[0]);
    c.sp = lc.b / T(den[2]);
  }
  const int lane = threadIdx.x & (kZmCols - 1);
  c.col = cb * kZmOut - 1 + lane;
  c.k0 = chunk * kc;
  if (c.k0 >= n1) return;  // whole block: grid padding
  c.k1 = min(c.k0 + kc, n1);
  const int ncol = n1 * n1;
  c.valid = lane >= 1 && lane <= kZmOut && c.col < ncol;
  c.i = c.col % n1;
  c.j = c.col / n1;
#pragma unroll
  for (int dj = -1; dj <= 1; ++dj) c.nb[dj + 1] = min(max(c.col + dj * n1, 0), ncol - 1);
  const int wave = threadIdx.x / kZmCols;  // velocity component
  if (wave == 0)
    zm_run<T, G, 0, VEL, HB>(g, lc, x, b, y, c, pshare, ps);
  else if (wave == 1)
    zm_run<T, G, 1, VEL, HB>(g, lc, x, b, y, c, pshare, ps);
  else
    zm_run<T, G, 2, VEL, HB>(g, lc, x, b, y, c, pshare, ps);
}

// Pressure rows at boundary nodes (list), boundary-class stencils.
template <typename T, int G>
__device__ __forceinline__ void prow_bnd_block(const Geom& g, const LevelConst<T>& lc, const T* __restrict__ x,
                                               const T* __restrict__ b, T* __restrict__ y, int opmask, int has_b,
                                               const int* __restrict__ bnd, int nbnd, int nmain, int bs,
                                               PStep<T> ps) {
  const int q = ((int)blockIdx.x - nmain) * bs + (int)threadIdx.x;
  if (q >= nbnd) return;
  const int t = bnd[q];
  int i, j, k;
  decode(t, g.n1, i, j, k);
  const T acc = prow_value<T, G>(g, lc, x, opmask, t, i, j, k);
  const int pp = 3 * g.vstride + t;
  const T r = has_b ? b[pp] - acc : acc;
  if (ps.p)
    ps.p[t] -= ps.omega * ps.dinv[t] * r;
  else
    y[pp] = r;
}



// The boundary pressure rows of a k-marching launch, one component per
// wavefront: the block's three wavefronts take the same 64 nodes, wavefront d
// sums the B_d part of each node's class row, and wavefront 0 adds the three
// partial sums (and C p for PSPG) after a block barrier -- a third of the
// loads of a whole row per thread.  red: 3 x 64 words of LDS.
template <typename T, int G>
__device__ __forceinline__ void prow_bnd_split(const Geom& g, const LevelConst<T>& lc, const T* __restrict__ x,
                                               const T* __restrict__ b, T* __restrict__ y, int has_b,
                                               const int* __restrict__ bnd, int nbnd, int nmain, PStep<T> ps,
                                               T (*red)[kZmCols]) {
  const int lane = (int)threadIdx.x % kZmCols, d = (int)threadIdx.x / kZmCols;
  const int q = ((int)blockIdx.x - nmain) * kZmCols + lane;
  const int N = g.N, s1 = g.n1, s2 = g.n1 * g.n1, nn = g.nn;
  int t = 0, cls = 0;
  T ab = 0;
  if (q < nbnd) {
    t = bnd[q];
    int i, j, k;
    decode(t, g.n1, i, j, k);
    cls = bcls3(i, N) + 3 * bcls3(j, N) + 9 * bcls3(k, N);
    const T* __restrict__ ud = x + (size_t)d * g.vstride;
    if (d == 0) {
      if constexpr (G == 1) {
        HHG_BCLS_CASES(p1, HHG_BROW_D0)
      } else {
        HHG_BCLS_CASES(p2, HHG_BROW_D0)
      }
    } else if (d == 1) {
      if constexpr (G == 1) {
        HHG_BCLS_CASES(p1, HHG_BROW_D1)
      } else {
        HHG_BCLS_CASES(p2, HHG_BROW_D1)
      }
    } else {
      if constexpr (G == 1) {
        HHG_BCLS_CASES(p1, HHG_BROW_D2)
      } else {
        HHG_BCLS_CASES(p2, HHG_BROW_D2)
      }
    }
  }
  red[d][lane] = ab;
  __syncthreads();
  if (d != 0 || q >= nbnd) return;
  T ac = 0;
  if constexpr (G == 1) {
    const T* __restrict__ p = x + 3 * (size_t)g.vstride;
    HHG_BCLS_CASES(p1, HHG_CROW)
  }
  // opmask of the k-marching launch: B and -C p (PSPG) / B only (Taylor-Hood)
  const T acc = lc.b * (red[0][lane] + red[1][lane] + red[2][lane]) - lc.c * ac;
  const int pp = 3 * g.vstride + t;
  const T r = has_b ? b[pp] - acc : acc;
  if (ps.p)
    ps.p[t] -= ps.omega * ps.dinv[t] * r;
  else
    y[pp] = r;
}
#undef HHG_CROW
#undef HHG_BROW_D0
#undef HHG_BROW_D1
#undef HHG_BROW_D2

// Taylor-Hood pressure residual rows r_p = g - B u on the small grid-wide
// levels, one velocity component per wavefront as in prow_bnd_split: block
// = 64 pressure nodes x 3 components, the interior nodes (1..N-1)^3 in the
// first ninner blocks (generated interior row split by component), the
// boundary list after them; with ps the pressure step is applied in place
// (Taylor-Hood rows read no p).  One round trip of independent loads per
// thread instead of the k-marching form's chain of dependent plane steps.
template <typename T>
__global__ void __launch_bounds__(3 * kZmCols) k_prow_split(Geom g, LevelConst<T> lc, const T* __restrict__ x,
                                                            const T* __restrict__ b, T* __restrict__ y,
                                                            const int* __restrict__ bnd, int nbnd, int ninner,
                                                            PStep<T> ps) {
  __shared__ T red[3][kZmCols];
  if ((int)blockIdx.x >= ninner) {
    prow_bnd_split<T, 8>(g, lc, x, b, y, 1, bnd, nbnd, ninner, ps, red);
    return;
  }
  const int lane = (int)threadIdx.x % kZmCols, d = (int)threadIdx.x / kZmCols;
  const int nr = g.N - 1, q = (int)blockIdx.x * kZmCols + lane;
  const bool on = q < nr * nr * nr;
  const int s1 = g.n1, s2 = g.n1 * g.n1, nn = g.nn;
  int t = 0;
  T ab = 0;
  if (on) {
    const int i = 1 + q % nr, j = 1 + (q / nr) % nr, k = 1 + q / (nr * nr);
    t = i + s1 * j + s2 * k;
    const T* __restrict__ ud = x + (size_t)d * g.vstride;
    if (d == 0)
      gen::p2_B_d0<T>(ud, t, s1, s2, nn, ab);
    else if (d == 1)
      gen::p2_B_d1<T>(ud, t, s1, s2, nn, ab);
    else
      gen::p2_B_d2<T>(ud, t, s1, s2, nn, ab);
  }
  red[d][lane] = ab;
  __syncthreads();
  if (d != 0 || !on) return;
  const T acc = lc.b * (red[0][lane] + red[1][lane] + red[2][lane]);
  const int pp = 3 * g.vstride + t;
  const T r = b[pp] - acc;
  if (ps.p)
    ps.p[t] -= ps.omega * ps.dinv[t] * r;
  else
    y[pp] = r;
}

// ---------------------------------------------------------- Gauss-Seidel
// The generated row functions accumulate three components at once; the
// Gauss-Seidel kernels give each velocity component its own thread
// (blockIdx.y) so a colour of a small level spreads over three times as many
// waves.  Component d reads u_d, p and writes u_d only (A is block diagonal).
template <typename T, int G, bool VAR>
__device__ __forceinline__ void gs_update(const Geom& g, const LevelConst<T>& lc, T* __restrict__ x,
                                          const T* __restrict__ b, int gr, int idx, int d) {
  const int s1 = g.n1, s2 = g.n1 * g.n1, nn = g.nn;
  const int pos = gr * nn + idx;
  T* ud = x + d * g.vstride;
  const T* p = x + 3 * g.vstride;
  T a0 = 0, a1 = 0, a2 = 0, c0 = 0, c1 = 0, c2 = 0;
  // same pointer for the three component slots: only slot d is used
  T ai;
  if constexpr (VAR) {
    Rows<T, G>::Anu(gr, ud, ud, ud, lc.nu, pos, idx, s1, s2, nn, a0, a1, a2);
    ai = lc.ainv_site[pos];
  } else {
    Rows<T, G>::A(gr, ud, ud, ud, pos, s1, s2, nn, a0, a1, a2);
    ai = lc.ainv[gr];
  }
  Rows<T, G>::BT(gr, p, idx, s1, s2, c0, c1, c2);
  const T c = d == 0 ? c0 : (d == 1 ? c1 : c2);
  ud[pos] += (b[d * g.vstride + pos] - lc.a * a0 - lc.b * c) * ai;
}

// One colour of the vertex group: interior nodes with (i+j+k) mod 2 == c.
// u_d += (f_d - (A u_d) - (B^T p)_d) / a_gg.
__host__ __device__ __forceinline__ int gs_vertex_count(const Geom& g) {
  const int nr = g.N - 1, ni = (nr + 1) >> 1;
  return ni * nr * nr;
}
template <typename T, int G, bool VAR>
__device__ __forceinline__ void gs_vertex_site(const Geom& g, const LevelConst<T>& lc, T* __restrict__ x,
                                               const T* __restrict__ b, int c, int t, int d) {
  const int N = g.N, nr = N - 1, ni = (nr + 1) >> 1;
  const int ip = t % ni, row = t / ni;
  const int j = 1 + row % nr, k = 1 + row / nr;
  const int i = 1 + ((c + 1 + j + k) & 1) + 2 * ip;
  if (i > N - 1) return;
  gs_update<T, G, VAR>(g, lc, x, b, 0, i + g.n1 * j + g.n1 * g.n1 * k, d);
}
template <typename T, int G, bool VAR>
__global__ void __launch_bounds__(kBlock) k_gs_vertex(Geom g, LevelConst<T> lc, T* __restrict__ x,
                                                      const T* __restrict__ b, int c) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= gs_vertex_count(g)) return;
  gs_vertex_site<T, G, VAR>(g, lc, x, b, c, t, blockIdx.y);
}

// One edge group (one colour) of the P2 velocity: all interior sites of group gr.
__host__ __device__ __forceinline__ int gs_edge_count(const Geom& g, int gr) {
  return (g.N - 1 + ((0xB2 >> gr) & 1)) * (g.N - 1 + ((0xD4 >> gr) & 1)) * (g.N - 1 + ((0xE8 >> gr) & 1));
}
template <typename T, bool VAR>
__device__ __forceinline__ void gs_edge_site(const Geom& g, const LevelConst<T>& lc, T* __restrict__ x,
                                             const T* __restrict__ b, int gr, int t, int d) {
  const int N = g.N;
  const int dx = gdx(gr), dy = gdy(gr), dz = gdz(gr);
  const int cx = N - 1 + dx, cy = N - 1 + dy;
  const int i = 1 - dx + t % cx;
  const int r = t / cx;
  const int j = 1 - dy + r % cy;
  const int k = 1 - dz + r / cy;
  gs_update<T, 8, VAR>(g, lc, x, b, gr, i + g.n1 * j + g.n1 * g.n1 * k, d);
}
// One instantiation per edge group: with the group a compile-time constant
// the A-row and B^T-row loads form one straight-line batch (one memory round
// trip); behind a runtime switch on the group they were two.
template <typename T, bool VAR, int GR>
__global__ void __launch_bounds__(kBlock) k_gs_edge(Geom g, LevelConst<T> lc, T* __restrict__ x,
                                                    const T* __restrict__ b) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= gs_edge_count(g, GR)) return;
  gs_edge_site<T, VAR>(g, lc, x, b, GR, t, blockIdx.y);
}

// p <- p - omega * dinv * rp (eq. uzawa-pressure with S_hat = omega^{-1} D).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_pstep(int nn, const T* __restrict__ dinv, T* __restrict__ p,
                                                  const T* __restrict__ rp, T omega) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= nn) return;
  p[t] -= omega * dinv[t] * rp[t];
}

// Schur diagonal per pressure node: mode 0: C_kk + sum_d sum_{j interior}
// B_dkj^2 / A_jj; mode 1: int psi_k.  Writes 1 / D_k.
template <typename T, int G>
__global__ void __launch_bounds__(kBlock) k_schur_diag(Geom g, const Tables<T>* __restrict__ tb,
                                                       const T* __restrict__ ainv_site, int mode,
                                                       T* __restrict__ dinv, const NeuTables<T>* __restrict__ nt) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= g.nn) return;
  int i, j, k;
  decode(t, g.n1, i, j, k);
  const int N = g.N;
  const int cls = bcls3(i, N) + 3 * bcls3(j, N) + 9 * bcls3(k, N);
  double d = 0.0;
  if (mode == 1) {
    d = (double)tb->mclass[cls];
  } else {
    const DStencil<T> c = tb->C[cls];
    for (int e = 0; e < c.n; ++e)
      if (c.off[e] == 0) d += (double)c.w[e];
    const DStencil<T> s = tb->B[cls];
    const int* code = tb->Bcode[cls];
    for (int e = 0; e < s.n; ++e) {
      const int cc = code[e];
      const int gr = cc & 15;
      const int ii = i + ((cc >> 4) & 15) - 2, jj = j + ((cc >> 8) & 15) - 2, kk = k + ((cc >> 12) & 15) - 2;
      if (!vel_unknown<G>(g, gr, ii, jj, kk)) continue;
      const double w0 = s.w[3 * e], w1 = s.w[3 * e + 1], w2 = s.w[3 * e + 2];
      double ai;
      if (!vel_interior<G>(gr, ii, jj, kk, N)) {  // outflow-face site: its boundary-class row
        const int sx = G == 1 ? bcls3(ii, N) : (gdx(gr) ? 1 : bcls3(ii, N));
        const int sy = G == 1 ? bcls3(jj, N) : (gdy(gr) ? 1 : bcls3(jj, N));
        const int sz = G == 1 ? bcls3(kk, N) : (gdz(gr) ? 1 : bcls3(kk, N));
        ai = (double)nt->adiag_inv[gr * 27 + sx + 3 * sy + 9 * sz];
      } else {
        ai = ainv_site ? (double)ainv_site[gr * g.nn + ii + g.n1 * (jj + g.n1 * kk)] : (double)tb->adiag_inv[gr];
      }
      d += (w0 * w0 + w1 * w1 + w2 * w2) * ai;
    }
  }
  dinv[t] = (T)(1.0 / d);
}

// 1 / a_ii for every interior velocity site with variable viscosity (0 elsewhere).
template <typename T, int G>
__global__ void __launch_bounds__(kBlock) k_nu_diag(Geom g, LevelConst<T> lc, T* __restrict__ ainv_site) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= g.nn) return;
  int i, j, k;
  decode(t, g.n1, i, j, k);
  for (int gr = 0; gr < G; ++gr) {
    T v = 0;
    if (vel_interior<G>(gr, i, j, k, g.N))
      v = T(1) / (lc.a * Rows<T, G>::Anudiag(gr, lc.nu, t, g.n1, g.n1 * g.n1));
    ainv_site[gr * g.nn + t] = v;
  }
}

// b = M f on interior velocity rows (velocity mass, interior stencil), 0 on
// boundary rows and on the pressure part.
template <typename T, int G>
__global__ void __launch_bounds__(kBlock) k_rhs(Geom g, LevelConst<T> lc, const T* __restrict__ f,
                                                T* __restrict__ b) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= g.nn) return;
  int i, j, k;
  decode(t, g.n1, i, j, k);
  const int s1 = g.n1, s2 = g.n1 * g.n1, nn = g.nn;
#pragma unroll 1
  for (int gr = 0; gr < G; ++gr) {
    const bool in = vel_interior<G>(gr, i, j, k, g.N);
    const int pos = gr * nn + t;
    T a0 = 0, a1 = 0, a2 = 0;
    if (in) Rows<T, G>::M(gr, f, f + g.vstride, f + 2 * g.vstride, pos, s1, s2, nn, a0, a1, a2);
    b[pos] = lc.m * a0;
    b[g.vstride + pos] = lc.m * a1;
    b[2 * g.vstride + pos] = lc.m * a2;
  }
  b[3 * g.vstride + t] = 0;
}

// y = M x: consistent velocity mass on every velocity site (boundary rows
// included, boundary-class stencils) and P1 pressure mass on every node.
template <typename T, int G>
__global__ void __launch_bounds__(kBlock) k_mass(Geom g, const Tables<T>* __restrict__ tb, const T* __restrict__ x,
                                                 T* __restrict__ y) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= g.nn) return;
  int i, j, k;
  decode(t, g.n1, i, j, k);
  const int N = g.N;
#pragma unroll
  for (int gr = 0; gr < G; ++gr) {
    const int pos = gr * g.nn + t;
    if (!vel_exists<G>(gr, i, j, k, N)) {
      y[pos] = 0;
      y[g.vstride + pos] = 0;
      y[2 * g.vstride + pos] = 0;
      continue;
    }
    const int dx = G == 1 ? 0 : gdx(gr), dy = G == 1 ? 0 : gdy(gr), dz = G == 1 ? 0 : gdz(gr);
    const int cls = (dx ? 1 : bcls3(i, N)) + 3 * (dy ? 1 : bcls3(j, N)) + 9 * (dz ? 1 : bcls3(k, N));
    const DStencil<T> st = tb->Mfull[gr * 27 + cls];
    T a0 = 0, a1 = 0, a2 = 0;
    for (int e = 0; e < st.n; ++e) {
      const int o = pos + st.off[e];
      a0 += st.w[e] * x[o];
      a1 += st.w[e] * x[g.vstride + o];
      a2 += st.w[e] * x[2 * g.vstride + o];
    }
    y[pos] = a0;
    y[g.vstride + pos] = a1;
    y[2 * g.vstride + pos] = a2;
  }
  const int cls = bcls3(i, N) + 3 * bcls3(j, N) + 9 * bcls3(k, N);
  const DStencil<T> st = tb->Pm[cls];
  T a = 0;
  const T* p = x + 3 * g.vstride;
  for (int e = 0; e < st.n; ++e) a += st.w[e] * p[t + st.off[e]];
  y[3 * g.vstride + t] = a;
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_dot(const T* __restrict__ x, const T* __restrict__ y, long n,
                                                double* __restrict__ partial) {
  __shared__ double sa[kBlock];
  double a = 0.0;
  for (long t = (long)blockIdx.x * kBlock + threadIdx.x; t < n; t += (long)gridDim.x * kBlock)
    a += (double)x[t] * (double)y[t];
  sa[threadIdx.x] = a;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sa[threadIdx.x] += sa[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = sa[0];
    partial[2 * blockIdx.x + 1] = 0.0;
  }
}

// ---------------------------------------------------------------- transfer
// Restriction (transpose of the prolongation, generated gathers): one coarse
// node t and one slice sl per thread -- velocity group sl / 3 < G, component
// sl % 3, or the P1 pressure for sl = 3 G (entries clipped at the domain
// boundary).  One component per thread: the small levels are latency-bound,
// and a vertex-group gather of all three components is ~375 dependent-ish
// loads.  Coarse boundary velocity rows are zero.
template <typename T, int G>
__device__ __forceinline__ void restrict_site(const Geom& gf, const Geom& gc, const T* __restrict__ rf,
                                              T* __restrict__ rc, int t, int sl, T* __restrict__ zx = nullptr) {
  int i, j, k;
  decode(t, gc.n1, i, j, k);
  const int fb = 2 * i + gf.n1 * (2 * j + gf.n1 * 2 * k);
  const int s1 = gf.n1, s2 = gf.n1 * gf.n1, nn = gf.nn, vs = gf.vstride;
  if (sl == 3 * G) {
    const T* pf = rf + 3 * (size_t)vs;
    rc[3 * gc.vstride + t] = G == 1 ? gen::p1_RP<T>(pf, fb, 2 * i, 2 * j, 2 * k, gf.N, s1, s2)
                                    : gen::p2_RP<T>(pf, fb, 2 * i, 2 * j, 2 * k, gf.N, s1, s2);
    if (zx) zx[3 * gc.vstride + t] = T(0);
    return;
  }
  const int gr = sl / 3, d = sl - 3 * gr;
  const T* rd = rf + (size_t)d * vs;  // component d; the other two outputs of the gather are unused
  T a0 = 0, a1 = 0, a2 = 0;
  if (vel_interior<G>(gr, i, j, k, gc.N)) {
    if constexpr (G == 1) {
      gen::p1_R_g0<T>(rd, fb, s1, s2, nn, 0, a0, a1, a2);
    } else {
      const int g = gr;
      HHG_P2_CASES(p2_R, rd, fb, s1, s2, nn, 0, a0, a1, a2)
    }
  }
  (void)a1, (void)a2;
  rc[(size_t)d * gc.vstride + gr * gc.nn + t] = a0;
  if (zx) zx[(size_t)d * gc.vstride + gr * gc.nn + t] = T(0);
}
template <typename T, int G>
__global__ void __launch_bounds__(kBlock) k_restrict(Geom gf, Geom gc, const T* __restrict__ rf, T* __restrict__ rc,
                                                     int sl0, T* __restrict__ zx) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= gc.nn) return;
  restrict_site<T, G>(gf, gc, rf, rc, t, sl0 + (int)blockIdx.y, zx);
}

// k-marching velocity restriction, P2-P1: a block is three wavefronts (the
// velocity components) over the same 64 consecutive coarse columns (linear
// index i + n1 j) of one chunk of coarse planes [k0, k1).  Step q (coarse
// plane kq = k0 - 1 + q) loads the fine planes 2 kq and 2 kq + 1: each lane
// the fine words at 2 i and 2 i + 1 of the fine rows 2 j - 2 .. 2 j + 1 of
// every fine group the plane's restriction entries use (one batch of loads,
// coalesced pairs instead of one gather per entry), the offsets 2 i - 1 and
// 2 i - 2 from the previous lane; the entries add into coarse planes kq and
// kq + 1 (two rotating accumulator planes), and plane kq is complete after
// step q and written.  Windows overlap by two columns (the end lanes lack a
// neighbour); clamped words reach only boundary coarse rows, which are
// written as zero.  Same entries as restrict_site, summed in another order.
constexpr int kRzmCols = 64;
#ifndef HHG_RZM_KC
#define HHG_RZM_KC 8  // coarse planes per chunk
#endif
template <typename T, int Q>
__device__ __forceinline__ void rzm_step(const Geom& gf, const Geom& gc, __amdgpu_buffer_rsrc_t ru, int fcol_e,
                                         int fcol_o, const int (&frow)[4], int kq, int k0, int k1, bool valid, int ic,
                                         int jc, int col, T* __restrict__ rc, int d, T (&acc)[2][8],
                                         T* __restrict__ zx) {
  const int n1f = gf.n1, s2f = n1f * n1f, nnb = gf.nn * (int)sizeof(T);
#pragma unroll
  for (int P = 0; P < 2; ++P) {
    const int F = min(max(2 * kq + P, 0), n1f - 1) * s2f;
    int ro_e[4], ro_o[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      ro_e[r] = (F + frow[r] + fcol_e) * (int)sizeof(T);
      ro_o[r] = (F + frow[r] + fcol_o) * (int)sizeof(T);
    }
    if (P == 0) {
      if constexpr (Q == 0) gen::p2_Rzm_p0_q0<T>(ru, ro_e, ro_o, nnb, acc);
      else gen::p2_Rzm_p0_q1<T>(ru, ro_e, ro_o, nnb, acc);
    } else {
      if constexpr (Q == 0) gen::p2_Rzm_p1_q0<T>(ru, ro_e, ro_o, nnb, acc);
      else gen::p2_Rzm_p1_q1<T>(ru, ro_e, ro_o, nnb, acc);
    }
    // keep the next plane's loads below this plane's multiply-adds (left
    // alone, the compiler issues both planes' 106 words at once: 256 VGPRs)
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int g = 0; g < 8; ++g) asm volatile("" : "+v"(acc[q][g]));
  }
  if (valid && kq >= k0 && kq < k1) {
    const int at = col + kq * gc.n1 * gc.n1;
#pragma unroll
    for (int g = 0; g < 8; ++g)
      rc[(size_t)d * gc.vstride + g * gc.nn + at] = vel_interior<8>(g, ic, jc, kq, gc.N) ? acc[Q][g] : T(0);
    if (zx)
#pragma unroll
      for (int g = 0; g < 8; ++g) zx[(size_t)d * gc.vstride + g * gc.nn + at] = T(0);
  }
#pragma unroll
  for (int g = 0; g < 8; ++g) acc[Q][g] = T(0);
}

template <typename T>
__global__ void __launch_bounds__(3 * kRzmCols) k_restrict_zm(Geom gf, Geom gc, const T* __restrict__ rf,
                                                              T* __restrict__ rc, int kc, int ncb, int nmain,
                                                              T* __restrict__ zx) {
  const int lin = xcd_block_of(nmain);
  const int cb = lin % ncb, chunk = lin / ncb;
  const int k0 = chunk * kc;
  if (k0 >= gc.n1) return;  // whole block: grid padding
  const int k1 = min(k0 + kc, gc.n1);
  const int lane = threadIdx.x & (kRzmCols - 1), d = threadIdx.x / kRzmCols;
  const int ncol = gc.n1 * gc.n1;
  const int col = cb * (kRzmCols - 2) - 1 + lane;
  const bool valid = lane >= 1 && lane <= kRzmCols - 2 && col < ncol;
  const int cc = min(max(col, 0), ncol - 1);
  const int ic = cc % gc.n1, jc = cc / gc.n1;
  const int n1f = gf.n1;
  const int fcol_e = 2 * ic, fcol_o = min(2 * ic + 1, n1f - 1);
  int frow[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) frow[r] = min(max(2 * jc - 2 + r, 0), n1f - 1) * n1f;
  const __amdgpu_buffer_rsrc_t ru =
      gen::make_rsrc(rf + (size_t)d * gf.vstride, (unsigned)((size_t)gf.vstride * sizeof(T)));
  T acc[2][8];
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int g = 0; g < 8; ++g) acc[q][g] = T(0);
  const int nq = k1 - k0 + 1;
  for (int q = 0; q < nq; q += 2) {
    rzm_step<T, 0>(gf, gc, ru, fcol_e, fcol_o, frow, k0 - 1 + q, k0, k1, valid, ic, jc, col, rc, d, acc, zx);
    if (q + 1 < nq)
      rzm_step<T, 1>(gf, gc, ru, fcol_e, fcol_o, frow, k0 + q, k0, k1, valid, ic, jc, col, rc, d, acc, zx);
  }
}

// Prolongation: a fine thread evaluates the coarse function at its site of
// one slice sl -- velocity group sl / 3 < G, component sl % 3, or the
// pressure for sl = 3 G (or every slice for sl < 0, the one-workgroup
// V-cycle's form).
template <typename T, int G>
__device__ __forceinline__ void prolong_slice(const Geom& gc, const Geom& gf, const TransferTables<T>* __restrict__ tt,
                                              const T* __restrict__ xc, T* __restrict__ xf, int add,
                                              int skip_boundary, int t, int i, int j, int k, int sl) {
  if (sl == 3 * G) {
    const int cls = (i & 1) + 2 * (j & 1) + 4 * (k & 1);
    const int base = (i >> 1) + gc.n1 * ((j >> 1) + gc.n1 * (k >> 1));
    T a = 0;
    // all 10 table slots: the slots past a class's count hold weight 0 and
    // offset 0 (the class's own coarse node, a valid index), so every load is
    // unconditional and the table and value loads go out as two batches
    // instead of two round trips per entry; the sum is unchanged
#pragma unroll
    for (int e = 0; e < 10; ++e) a += tt->pp_w[cls * 10 + e] * xc[3 * gc.vstride + base + tt->pp_off[cls * 10 + e]];
    const int pp = 3 * gf.vstride + t;
    xf[pp] = add ? xf[pp] + a : a;
    return;
  }
  const int gr = sl / 3, d = sl - 3 * gr;
  const int Nf = gf.N;
  if (!vel_exists<G>(gr, i, j, k, Nf)) return;
  if (skip_boundary && !vel_interior<G>(gr, i, j, k, Nf)) return;
  int cls, base;
  if (G == 1) {
    cls = (i & 1) + 2 * (j & 1) + 4 * (k & 1);
    base = (i >> 1) + gc.n1 * ((j >> 1) + gc.n1 * (k >> 1));
  } else {
    const int X = 2 * i + gdx(gr), Y = 2 * j + gdy(gr), Z = 2 * k + gdz(gr);
    cls = (X & 3) + 4 * (Y & 3) + 16 * (Z & 3);
    base = (X >> 2) + gc.n1 * ((Y >> 2) + gc.n1 * (Z >> 2));
  }
  const T* xd = xc + (size_t)d * gc.vstride;
  T a = 0;
#pragma unroll
  for (int e = 0; e < 10; ++e) a += tt->vp_w[cls * 10 + e] * xd[base + tt->vp_off[cls * 10 + e]];  // as above
  const int pos = d * gf.vstride + gr * gf.nn + t;
  xf[pos] = add ? xf[pos] + a : a;
}
// One velocity group of one fine site, its three components together (one
// table walk for the three).
template <typename T, int G>
__device__ __forceinline__ void prolong_group(const Geom& gc, const Geom& gf, const TransferTables<T>* __restrict__ tt,
                                              const T* __restrict__ xc, T* __restrict__ xf, int add, int skip_boundary,
                                              int t, int i, int j, int k, int gr) {
  const int Nf = gf.N;
  {
    if (!vel_exists<G>(gr, i, j, k, Nf)) return;
    if (skip_boundary && !vel_interior<G>(gr, i, j, k, Nf)) return;
    int cls, base;
    if (G == 1) {
      cls = (i & 1) + 2 * (j & 1) + 4 * (k & 1);
      base = (i >> 1) + gc.n1 * ((j >> 1) + gc.n1 * (k >> 1));
    } else {
      const int X = 2 * i + gdx(gr), Y = 2 * j + gdy(gr), Z = 2 * k + gdz(gr);
      cls = (X & 3) + 4 * (Y & 3) + 16 * (Z & 3);
      base = (X >> 2) + gc.n1 * ((Y >> 2) + gc.n1 * (Z >> 2));
    }
    T a0 = 0, a1 = 0, a2 = 0;
#pragma unroll
    for (int e = 0; e < 10; ++e) {  // all slots, as in prolong_slice
      const int o = base + tt->vp_off[cls * 10 + e];
      const T w = tt->vp_w[cls * 10 + e];
      a0 += w * xc[o];
      a1 += w * xc[gc.vstride + o];
      a2 += w * xc[2 * gc.vstride + o];
    }
    const int pos = gr * gf.nn + t;
    xf[pos] = add ? xf[pos] + a0 : a0;
    xf[gf.vstride + pos] = add ? xf[gf.vstride + pos] + a1 : a1;
    xf[2 * gf.vstride + pos] = add ? xf[2 * gf.vstride + pos] + a2 : a2;
  }
}
// Every slice of one fine site (the one-workgroup V-cycle's form: same sums
// as prolong_slice).
template <typename T, int G>
__device__ __forceinline__ void prolong_site(const Geom& gc, const Geom& gf, const TransferTables<T>* __restrict__ tt,
                                             const T* __restrict__ xc, T* __restrict__ xf, int add, int skip_boundary,
                                             int t) {
  int i, j, k;
  decode(t, gf.n1, i, j, k);
#pragma unroll
  for (int gr = 0; gr < G; ++gr) prolong_group<T, G>(gc, gf, tt, xc, xf, add, skip_boundary, t, i, j, k, gr);
  prolong_slice<T, G>(gc, gf, tt, xc, xf, add, skip_boundary, t, i, j, k, 3 * G);
}
template <typename T, int G>
__global__ void __launch_bounds__(kBlock) k_prolong(Geom gc, Geom gf, const TransferTables<T>* __restrict__ tt,
                                                    const T* __restrict__ xc, T* __restrict__ xf, int add,
                                                    int skip_boundary) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= gf.nn) return;
  int i, j, k;
  decode(t, gf.n1, i, j, k);
  prolong_slice<T, G>(gc, gf, tt, xc, xf, add, skip_boundary, t, i, j, k, blockIdx.y);
}

// Prolongation by coarse cubes (large levels): a thread owns coarse cube (i,
// j, k) and one slice -- velocity component blockIdx.y < 3, or the pressure
// (blockIdx.y == 3, the P1 function on the vertex lattice) -- loads the
// cube's coarse words once (27 for P2, its 8 corners for P1) and writes the
// fine sites 2 (i, j, k) + {0, 1}^3 of every fine group with the generated
// interpolation (no table walk, no per-site class).  A fine group's eight
// words are read as one batch before its eight stores; a word's address is
// clamped to the cube's own site when the site is not written, so every load
// is in bounds and unconditional.
template <typename T, int G, bool ADD>
__global__ void __launch_bounds__(kBlock) k_prolong_cube(Geom gc, Geom gf, const T* __restrict__ xc,
                                                         T* __restrict__ xf, int skip_boundary) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= gc.nn) return;
  int i, j, k;
  decode(t, gc.n1, i, j, k);
  const int sl = blockIdx.y;
  const bool pres = sl == 3;
  const int n1c = gc.n1;
  const int oi = min(i + 1, n1c - 1) - i, oj = (min(j + 1, n1c - 1) - j) * n1c,
            ok = (min(k + 1, n1c - 1) - k) * n1c * n1c;
  const T* src = xc + (size_t)(pres ? 3 : sl) * gc.vstride + t;
  T c[27];
#pragma unroll
  for (int q = 0; q < 27; ++q) c[q] = T(0);
  if (G == 8 && !pres) {
#pragma unroll
    for (int q = 0; q < 27; ++q) {
      const int a = q % 3, b = (q / 3) % 3, e = q / 9;
      const int gr = (a & 1) + 2 * (b & 1) + 4 * (e & 1);  // parity -> group below
      constexpr int kGroupOfParity[8] = {0, 1, 2, 4, 3, 5, 6, 7};
      c[q] = src[kGroupOfParity[gr] * gc.nn + (a == 2 ? oi : 0) + (b == 2 ? oj : 0) + (e == 2 ? ok : 0)];
    }
  } else {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int a = q & 1, b = (q >> 1) & 1, e = q >> 2;
      c[2 * a + 6 * b + 18 * e] = src[(a ? oi : 0) + (b ? oj : 0) + (e ? ok : 0)];
    }
  }
  const int n1f = gf.n1, Nf = gf.N;
  const int fi = 2 * i, fj = 2 * j, fk = 2 * k;
  T* dst = xf + (size_t)(pres ? 3 : sl) * gf.vstride + (fi + n1f * (fj + n1f * fk));
  if (pres || G == 1) {
    T v[8], old[8];
    gen::p1_Pc_g0<T>(c, v);
    bool w[8];
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      const int pi = p & 1, pj = (p >> 1) & 1, pk = p >> 2;
      w[p] = fi + pi <= Nf && fj + pj <= Nf && fk + pk <= Nf &&
             (pres || !skip_boundary || vel_interior<1>(0, fi + pi, fj + pj, fk + pk, Nf));
      if (ADD) old[p] = dst[w[p] ? pi + n1f * (pj + n1f * pk) : 0];
    }
#pragma unroll
    for (int p = 0; p < 8; ++p)
      if (w[p]) dst[(p & 1) + n1f * (((p >> 1) & 1) + n1f * (p >> 2))] = ADD ? old[p] + v[p] : v[p];
    return;
  }
#pragma unroll
  for (int g = 0; g < 8; ++g) {
    T v[8], old[8];
    gen::p2_Pc<T>(g, c, v);
    bool w[8];
#pragma unroll
    for (int p = 0; p < 8; ++p) {
      const int pi = p & 1, pj = (p >> 1) & 1, pk = p >> 2;
      w[p] = vel_exists<8>(g, fi + pi, fj + pj, fk + pk, Nf) &&
             (!skip_boundary || vel_interior<8>(g, fi + pi, fj + pj, fk + pk, Nf));
      if (ADD) old[p] = dst[g * gf.nn + (w[p] ? pi + n1f * (pj + n1f * pk) : 0)];
    }
#pragma unroll
    for (int p = 0; p < 8; ++p)
      if (w[p]) {
        const int o = g * gf.nn + (p & 1) + n1f * (((p >> 1) & 1) + n1f * (p >> 2));
        dst[o] = ADD ? old[p] + v[p] : v[p];
      }
  }
}

// Boundary velocity values of the coarse level from the coincident fine nodes.
template <typename T, int G>
__global__ void __launch_bounds__(kBlock) k_inject_boundary(Geom gf, Geom gc, const T* __restrict__ xf,
                                                            T* __restrict__ xc) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= gc.nn) return;
  int i, j, k;
  decode(t, gc.n1, i, j, k);
#pragma unroll
  for (int gr = 0; gr < G; ++gr) {
    if (!vel_exists<G>(gr, i, j, k, gc.N) || vel_unknown<G>(gc, gr, i, j, k)) continue;
    int fi, fj, fk;
    if (G == 1) {
      fi = 2 * i, fj = 2 * j, fk = 2 * k;
    } else {  // coarse doubled position S -> fine vertex index S
      fi = 2 * i + gdx(gr), fj = 2 * j + gdy(gr), fk = 2 * k + gdz(gr);
    }
    const int fpos = fi + gf.n1 * (fj + gf.n1 * fk);
    const int pos = gr * gc.nn + t;
    xc[pos] = xf[fpos];
    xc[gc.vstride + pos] = xf[gf.vstride + fpos];
    xc[2 * gc.vstride + pos] = xf[2 * gf.vstride + fpos];
  }
}

template <typename T, int G>
__global__ void __launch_bounds__(kBlock) k_copy_boundary(Geom g, const T* __restrict__ src, T* __restrict__ dst) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= g.nn) return;
  int i, j, k;
  decode(t, g.n1, i, j, k);
#pragma unroll
  for (int gr = 0; gr < G; ++gr) {
    if (!vel_exists<G>(gr, i, j, k, g.N) || vel_unknown<G>(g, gr, i, j, k)) continue;
    const int pos = gr * g.nn + t;
    dst[pos] = src[pos];
    dst[g.vstride + pos] = src[g.vstride + pos];
    dst[2 * g.vstride + pos] = src[2 * g.vstride + pos];
  }
}

// ------------------------------------------------------------ conversions
// Plain lattice order: velocity components over (M+1)^3, M = N (P1) or 2N (P2),
// then pressure over (N+1)^3.
template <typename T, int G>
__global__ void __launch_bounds__(kBlock) k_lattice(Geom g, const double* __restrict__ lat, T* __restrict__ vec,
                                                    double* __restrict__ lat_out, const T* __restrict__ vec_in,
                                                    int to_lattice) {
  const int M = G == 1 ? g.N : 2 * g.N;
  const int m1 = M + 1;
  const long nv = (long)m1 * m1 * m1;
  const long tot = 3 * nv + g.nn;
  const long t = (long)blockIdx.x * kBlock + threadIdx.x;
  if (t >= tot) return;
  long vpos;
  if (t < 3 * nv) {
    const int d = (int)(t / nv);
    const int s = (int)(t % nv);
    const int X = s % m1, r = s / m1, Y = r % m1, Z = r / m1;
    int gr = 0, i = X, j = Y, k = Z;
    if (G == 8) {
      const int par = (X & 1) | ((Y & 1) << 1) | ((Z & 1) << 2);
      // parity bits (x | y<<1 | z<<2) -> group index: only 3 <-> 4 differ
      gr = par == 3 ? 4 : (par == 4 ? 3 : par);
      i = X >> 1, j = Y >> 1, k = Z >> 1;
    }
    vpos = (long)d * g.vstride + (long)gr * g.nn + i + (long)g.n1 * (j + (long)g.n1 * k);
  } else {
    vpos = 3L * g.vstride + (t - 3 * nv);
  }
  if (to_lattice)
    lat_out[t] = (double)vec_in[vpos];
  else
    vec[vpos] = (T)lat[t];
}

// ------------------------------------------------------------- reductions
// Block partial sums of pressure quantities.  mode 0: sum m_cls p and sum
// m_cls (two slots); mode 1: sum p; mode 2: sum p^2.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_psum(Geom g, const Tables<T>* __restrict__ tb, const T* __restrict__ p,
                                                 double* __restrict__ partial, int mode) {
  __shared__ double sa[kBlock], sb[kBlock];
  double a = 0.0, bsum = 0.0;
  for (int t = blockIdx.x * kBlock + threadIdx.x; t < g.nn; t += gridDim.x * kBlock) {
    const double v = (double)p[t];
    if (mode == 0) {
      int i, j, k;
      decode(t, g.n1, i, j, k);
      const double m = (double)tb->mclass[bcls3(i, g.N) + 3 * bcls3(j, g.N) + 9 * bcls3(k, g.N)];
      a += m * v;
      bsum += m;
    } else if (mode == 1) {
      a += v;
    } else {
      a += v * v;
    }
  }
  sa[threadIdx.x] = a;
  sb[threadIdx.x] = bsum;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      sa[threadIdx.x] += sa[threadIdx.x + s];
      sb[threadIdx.x] += sb[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = sa[0];
    partial[2 * blockIdx.x + 1] = sb[0];
  }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_sumsq(const T* __restrict__ x, long n, double* __restrict__ partial) {
  __shared__ double sa[kBlock];
  double a = 0.0;
  for (long t = (long)blockIdx.x * kBlock + threadIdx.x; t < n; t += (long)gridDim.x * kBlock) {
    const double v = (double)x[t];
    a += v * v;
  }
  sa[threadIdx.x] = a;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sa[threadIdx.x] += sa[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = sa[0];
    partial[2 * blockIdx.x + 1] = 0.0;
  }
}

// Fixed-order final sum of the block partials into out[0], out[1].
__global__ void __launch_bounds__(kBlock) k_final_sum(const double* __restrict__ partial, int nparts,
                                                      double* __restrict__ out) {
  __shared__ double sa[kBlock], sb[kBlock];
  double a = 0.0, b = 0.0;
  for (int q = threadIdx.x; q < nparts; q += kBlock) {
    a += partial[2 * q];
    b += partial[2 * q + 1];
  }
  sa[threadIdx.x] = a;
  sb[threadIdx.x] = b;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      sa[threadIdx.x] += sa[threadIdx.x + s];
      sb[threadIdx.x] += sb[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = sa[0];
    out[1] = sb[0];
  }
}

// mode 0: p -= s0 / s1 (weighted mean); mode 1: p -= s0 / nn (plain mean).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_pshift(int nn, T* __restrict__ p, const double* __restrict__ sums,
                                                   int mode) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= nn) return;
  const double mean = mode == 0 ? sums[0] / sums[1] : sums[0] / (double)nn;
  p[t] = (T)((double)p[t] - mean);
}

// The whole mean-zero shift of a small level in one workgroup: the sums of
// k_psum (mode 0 or 1), a tree reduction, then p -= mean; sums[0], sums[1]
// as k_final_sum leaves them.  Three launches become one.
constexpr int kMeanBlock = 1024;
template <typename T>
__global__ void __launch_bounds__(kMeanBlock) k_mean_zero_1b(Geom g, const Tables<T>* __restrict__ tb,
                                                             T* __restrict__ p, double* __restrict__ sums, int mode) {
  constexpr int kWaves = kMeanBlock / 64;
  __shared__ double mc[27], sa[kWaves], sb[kWaves], smean;
  if (mode == 0 && threadIdx.x < 27) mc[threadIdx.x] = (double)tb->mclass[threadIdx.x];
  __syncthreads();
  // (i, j, k) from t by float reciprocals: exact for the one-block sizes
  // (n1 <= 40, t < 65536: the quotients stay far from integer boundaries)
  const float inv = 1.0f / (float)g.n1;
  double a = 0.0, bsum = 0.0;
  for (int t = threadIdx.x; t < g.nn; t += kMeanBlock) {
    const double v = (double)p[t];
    if (mode == 0) {
      const int r = (int)(((float)t + 0.5f) * inv);
      const int i = t - r * g.n1;
      const int k = (int)(((float)r + 0.5f) * inv);
      const int j = r - k * g.n1;
      const double m = mc[bcls3(i, g.N) + 3 * bcls3(j, g.N) + 9 * bcls3(k, g.N)];
      a += m * v;
      bsum += m;
    } else {
      a += v;
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_down(a, o);
    bsum += __shfl_down(bsum, o);
  }
  const int w = (int)threadIdx.x / 64, lane = (int)threadIdx.x % 64;
  if (lane == 0) {
    sa[w] = a;
    sb[w] = bsum;
  }
  __syncthreads();
  if (w == 0) {
    double x = lane < kWaves ? sa[lane] : 0.0, y = lane < kWaves ? sb[lane] : 0.0;
    for (int o = 32; o > 0; o >>= 1) {
      x += __shfl_down(x, o);
      y += __shfl_down(y, o);
    }
    if (lane == 0) {
      smean = mode == 0 ? x / y : x / (double)g.nn;
      sums[0] = x;
      sums[1] = y;
    }
  }
  __syncthreads();
  const double mean = smean;
  for (int t = threadIdx.x; t < g.nn; t += kMeanBlock) p[t] = (T)((double)p[t] - mean);
}

// x *= 1 / sqrt(sums[slot])
template <typename T>
__global__ void __launch_bounds__(kBlock) k_scale(T* __restrict__ x, long n, const double* __restrict__ sums,
                                                  int slot) {
  const long t = (long)blockIdx.x * kBlock + threadIdx.x;
  if (t >= n) return;
  x[t] = (T)((double)x[t] / sqrt(sums[slot]));
}

// y = a * x (.* d if d != nullptr)
template <typename T>
__global__ void __launch_bounds__(kBlock) k_scaled_copy(T* __restrict__ y, const T* __restrict__ x,
                                                        const T* __restrict__ d, long n, T a) {
  const long t = (long)blockIdx.x * kBlock + threadIdx.x;
  if (t >= n) return;
  y[t] = d ? a * x[t] * d[t] : a * x[t];
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_fill(T* __restrict__ x, long n, T v) {
  const long t = (long)blockIdx.x * kBlock + threadIdx.x;
  if (t < n) x[t] = v;
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_axpy(T* __restrict__ y, const T* __restrict__ x, long n, T a) {
  const long t = (long)blockIdx.x * kBlock + threadIdx.x;
  if (t < n) y[t] += a * x[t];
}

// ------------------------------------------------- outflow faces
// Sites of a Neumann face (Sec. 2, natural outflow condition) are unknowns
// with truncated rows: the elements outside the cube are missing.  Few sites
// (O(N^2)), so the rows are table-driven (NeuTables, one per group and
// boundary class); the grid-wide kernels treat these sites as boundary sites
// and these kernels fill in their rows afterwards.  blockIdx.y = velocity
// component d; every table offset stays inside the cube.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_neu_rows(Geom g, const NeuTables<T>* __restrict__ nt, NeuList L,
                                                     int first, int n, const T* __restrict__ x,
                                                     const T* __restrict__ b, T* __restrict__ y, int opmask,
                                                     int has_b) {
  const int q = blockIdx.x * kBlock + threadIdx.x;
  if (q >= n) return;
  const int d = blockIdx.y;
  const int pos = L.pos[first + q], sl = L.slot[first + q];
  const int t = pos % g.nn;
  const T* ud = x + (size_t)d * g.vstride;
  const T* p = x + 3 * (size_t)g.vstride;
  T r = 0;
  if (opmask & 1) {
    const DStencil<T> A = nt->A[sl];
    for (int e = 0; e < A.n; ++e) r += A.w[e] * ud[pos + A.off[e]];
  }
  if (opmask & 2) {
    const DStencil<T> BT = nt->BT[sl];
    for (int e = 0; e < BT.n; ++e) r += BT.w[3 * e + d] * p[t + BT.off[e]];
  }
  const size_t o = (size_t)d * g.vstride + pos;
  y[o] = has_b ? b[o] - r : r;
}

// u_d += (f_d - A u_d - (B^T p)_d) / a_ii at the sites of one colour (no two
// sites of a colour are coupled, so the order inside the launch is free).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_neu_gs(Geom g, const NeuTables<T>* __restrict__ nt, NeuList L, int first,
                                                   int n, T* __restrict__ x, const T* __restrict__ b) {
  const int q = blockIdx.x * kBlock + threadIdx.x;
  if (q >= n) return;
  const int d = blockIdx.y;
  const int pos = L.pos[first + q], sl = L.slot[first + q];
  const int t = pos % g.nn;
  T* ud = x + (size_t)d * g.vstride;
  const T* p = x + 3 * (size_t)g.vstride;
  const DStencil<T> A = nt->A[sl];
  const DStencil<T> BT = nt->BT[sl];
  T r = b[(size_t)d * g.vstride + pos];
  for (int e = 0; e < A.n; ++e) r -= A.w[e] * ud[pos + A.off[e]];
  for (int e = 0; e < BT.n; ++e) r -= BT.w[3 * e + d] * p[t + BT.off[e]];
  ud[pos] += r * nt->adiag_inv[sl];
}

// b = M f at the sites: the consistent velocity mass rows of the boundary
// classes (Tables::Mfull, same slot numbering).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_neu_rhs(Geom g, const Tables<T>* __restrict__ tb, NeuList L, int n,
                                                    const T* __restrict__ f, T* __restrict__ b) {
  const int q = blockIdx.x * kBlock + threadIdx.x;
  if (q >= n) return;
  const int d = blockIdx.y;
  const int pos = L.pos[q];
  const DStencil<T> M = tb->Mfull[L.slot[q]];
  const T* fd = f + (size_t)d * g.vstride;
  T a = 0;
  for (int e = 0; e < M.n; ++e) a += M.w[e] * fd[pos + M.off[e]];
  b[(size_t)d * g.vstride + pos] = a;
}

// Coarse outflow sites: rc = sum of R-weights times the fine residual (the
// transpose of the interpolation, limited to fine sites inside the cube).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_neu_restrict(Geom gf, Geom gc, const NeuTables<T>* __restrict__ ntc,
                                                         NeuList Lc, int n, const T* __restrict__ rf,
                                                         T* __restrict__ rc) {
  const int q = blockIdx.x * kBlock + threadIdx.x;
  if (q >= n) return;
  const int d = blockIdx.y;
  const int pos = Lc.pos[q];
  const int t = pos % gc.nn;
  int i, j, k;
  decode(t, gc.n1, i, j, k);
  const int fb = 2 * i + gf.n1 * (2 * j + gf.n1 * 2 * k);
  const DStencil<T> R = ntc->R[Lc.slot[q]];
  const T* r = rf + (size_t)d * gf.vstride;
  T a = 0;
  for (int e = 0; e < R.n; ++e) a += R.w[e] * r[fb + R.off[e]];
  rc[(size_t)d * gc.vstride + pos] = a;
}

// Fine outflow sites: xf += I xc, the interpolation of the grid-wide
// prolongation at these sites (which it skips as boundary sites).
template <typename T, int G>
__global__ void __launch_bounds__(kBlock) k_neu_prolong(Geom gc, Geom gf, const TransferTables<T>* __restrict__ tt,
                                                        NeuList Lf, int n, const T* __restrict__ xc,
                                                        T* __restrict__ xf) {
  const int q = blockIdx.x * kBlock + threadIdx.x;
  if (q >= n) return;
  const int pos = Lf.pos[q];
  const int gr = pos / gf.nn, t = pos - gr * gf.nn;
  int i, j, k;
  decode(t, gf.n1, i, j, k);
  prolong_slice<T, G>(gc, gf, tt, xc, xf, 1, 0, t, i, j, k, 3 * gr + (int)blockIdx.y);
}

// ------------------------------------------------- small-level V-cycle
// Table-driven form of the boundary pressure rows: the generated per-class
// rows are fastest in grid-wide launches, but in the one-workgroup cycle
// this compact loop measured faster (its many phases run a lot of distinct
// code).  The restriction, the Gauss-Seidel and the interior rows there are
// the generated forms, whose independent unrolled loads win over table loops.
template <typename T>
__device__ __forceinline__ T prow_bnd_table(const Geom& g, const Tables<T>* __restrict__ tb, const T* __restrict__ x,
                                            int opmask, int node) {
  int i, j, k;
  decode(node, g.n1, i, j, k);
  const int cls = bcls3(i, g.N) + 3 * bcls3(j, g.N) + 9 * bcls3(k, g.N);
  const T* u0 = x;
  const T* u1 = x + g.vstride;
  const T* u2 = x + 2 * g.vstride;
  const T* p = x + 3 * g.vstride;
  T acc = 0;
  if (opmask & 4) {
    // four entries per pass into four partial sums: the entries' table and
    // vector loads are independent, so a pass waits for memory once
    const DStencil<T> s = tb->B[cls];
    T a4[4] = {0, 0, 0, 0};
    int e = 0;
    for (; e + 4 <= s.n; e += 4) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int o = node + s.off[e + q];
        const T* w = s.w + 3 * (e + q);
        a4[q] += w[0] * u0[o] + w[1] * u1[o] + w[2] * u2[o];
      }
    }
    for (; e < s.n; ++e) {
      const int o = node + s.off[e];
      a4[0] += s.w[3 * e] * u0[o] + s.w[3 * e + 1] * u1[o] + s.w[3 * e + 2] * u2[o];
    }
    acc = (a4[0] + a4[1]) + (a4[2] + a4[3]);
  }
  if (opmask & 8) {
    const DStencil<T> s = tb->C[cls];
    T c = 0;
    for (int e = 0; e < s.n; ++e) c += s.w[e] * p[node + s.off[e]];
    acc += (opmask & 16) ? c : -c;
  }
  return acc;
}


// Round a float32 value to the nearest bfloat16 (ties to even), kept as a
// float32 whose low 16 bits are zero; NaN stays NaN.
__device__ __forceinline__ float round_bf16(float v) {
  unsigned u = __float_as_uint(v);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x7fffffu)) return __uint_as_float((u | 0x400000u) & 0xffff0000u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xffff0000u);
}

// One workgroup runs the whole variable V-cycle of Alg. fmg below and at the
// level lmin + nlev - 1: the same site bodies as the grid-wide kernels, each
// phase a block-strided loop, phases separated by barriers.  On the small
// levels a grid-wide launch is almost all launch latency; here a phase costs
// a few hundred nanoseconds.
#ifndef HHG_SMALL_BLOCK
#define HHG_SMALL_BLOCK 256
#endif
constexpr int kSmallBlock = HHG_SMALL_BLOCK;

template <typename T>
__device__ double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int s = kSmallBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  const double out = red[0];
  __syncthreads();
  return out;
}

// Pointer type of the level vectors in the one-workgroup V-cycle: LDS
// pointers when every level lives in LDS.  The helpers below are real calls
// (too large to inline at every use); with an LDS-typed parameter their
// stencil loads compile to LDS reads instead of generic (flat) loads.
template <typename T, bool LDS>
struct SmallVec {
  using type = T*;
};
template <typename T>
struct SmallVec<T, true> {
  typedef __attribute__((address_space(3))) T* type;
};

// Levels stored as bfloat16 (float32 only): round what a phase wrote,
// v[s stride + off + t] for s < nseg, t < n, then a barrier.
template <typename T, typename V>
__device__ void small_round(bool on, V v, int stride, int off, int n, int nseg) {
  if constexpr (std::is_same<T, float>::value) {
    if (!on) return;
    for (int t = threadIdx.x; t < n * nseg; t += kSmallBlock) {
      const int sg = t / n, at = sg * stride + off + (t - sg * n);
      v[at] = round_bf16(v[at]);
    }
    __syncthreads();
  } else {
    (void)on, (void)v, (void)stride, (void)off, (void)n, (void)nseg;
  }
}

template <typename T, int G, bool VAR, typename V>
__device__ void small_apply(const SmallLevel<T>& L, int opmask, V x, V b, V y, int vel_rows) {
  for (int t = threadIdx.x; t < L.g.nn; t += kSmallBlock)
    apply_site<T, G, VAR>(L.g, L.lc, (const T*)x, (const T*)b, (T*)y, opmask, 1, vel_rows, 1, t);
  // boundary pressure rows from the last thread down: on the levels where
  // nn < kSmallBlock they go to the threads the loop above left idle
  for (int q = kSmallBlock - 1 - (int)threadIdx.x; q < L.nbnd; q += kSmallBlock) {
    const int t = L.bnd[q];
    const int pp = 3 * L.g.vstride + t;
    y[pp] = b[pp] - prow_bnd_table<T>(L.g, L.tb, (const T*)x, opmask, t);
  }
  __syncthreads();
}

template <typename T, int G, bool VAR, typename V>
__device__ void small_colour(const SmallLevel<T>& L, V x, V b, int c, bool q16) {
  if (c < kGsVertexColours) {
    const int n = gs_vertex_count(L.g);
    for (int w = threadIdx.x; w < 3 * n; w += kSmallBlock)
      gs_vertex_site<T, G, VAR>(L.g, L.lc, (T*)x, (const T*)b, c, w % n, w / n);
  } else {
    if constexpr (G == 8) {
      const int gr = c - kGsVertexColours + 1, n = gs_edge_count(L.g, gr);
      for (int w = threadIdx.x; w < 3 * n; w += kSmallBlock)
        gs_edge_site<T, VAR>(L.g, L.lc, (T*)x, (const T*)b, gr, w % n, w / n);
    }
  }
  __syncthreads();
  small_round<T>(q16, x, L.g.vstride, c < kGsVertexColours ? 0 : (c - kGsVertexColours + 1) * L.g.nn, L.g.nn,
                 3);  // the group the colour wrote
}

template <typename T, int G, bool VAR, typename V>
__device__ void small_smooth(const SmallCycle<T>& sc, const SmallLevel<T>& L, V x, V b, V r, int iters, bool q16) {
  if (L.g.N < 2) return;
  constexpr int ncol = gs_colours(G);
  for (int it = 0; it < iters; ++it) {
    for (int s = 0; s < sc.xi; ++s) {
      for (int c = 0; c < ncol; ++c) small_colour<T, G, VAR>(L, x, b, c, q16);
      if (sc.gs_sym)
        for (int c = ncol - 1; c >= 0; --c) small_colour<T, G, VAR>(L, x, b, c, q16);
    }
    const int vs = L.g.vstride;
    small_apply<T, G, VAR>(L, sc.full_mask & 12, x, b, r, 0);
    small_round<T>(q16, r, 0, 3 * vs, L.g.nn, 1);
    for (int t = threadIdx.x; t < L.g.nn; t += kSmallBlock) x[3 * vs + t] -= sc.omega * L.dinv[t] * r[3 * vs + t];
    __syncthreads();
    small_round<T>(q16, x, 0, 3 * vs, L.g.nn, 1);
  }
}

template <typename T, int G, typename V>
__device__ void small_smooth_any(const SmallCycle<T>& sc, const SmallLevel<T>& L, V x, V b, V r, int iters, bool q16) {
  if (L.lc.nu)
    small_smooth<T, G, true>(sc, L, x, b, r, iters, q16);
  else
    small_smooth<T, G, false>(sc, L, x, b, r, iters, q16);
}

template <typename T, int G, typename V>
__device__ void small_residual(const SmallCycle<T>& sc, const SmallLevel<T>& L, V x, V b, V r) {
  if (L.lc.nu)
    small_apply<T, G, true>(L, sc.full_mask, x, b, r, 1);
  else
    small_apply<T, G, false>(L, sc.full_mask, x, b, r, 1);
}

// p -= sum_k w_k p_k / sum_k w_k with w_k = int psi_k (mode 0) or 1 (mode 1)
template <typename T, typename V>
__device__ void small_pshift(const SmallLevel<T>& L, V p, int mode, double* red) {
  double a = 0.0, m = 0.0;
  for (int t = threadIdx.x; t < L.g.nn; t += kSmallBlock) {
    double w = 1.0;
    if (mode == 0) {
      int i, j, k;
      decode(t, L.g.n1, i, j, k);
      w = (double)L.tb->mclass[bcls3(i, L.g.N) + 3 * bcls3(j, L.g.N) + 9 * bcls3(k, L.g.N)];
    }
    a += w * (double)p[t];
    m += w;
  }
  const double sa = block_sum<T>(a, red);
  const double sm = block_sum<T>(m, red);
  const double mean = sa / sm;
  for (int t = threadIdx.x; t < L.g.nn; t += kSmallBlock) p[t] = (T)((double)p[t] - mean);
  __syncthreads();
}

// LDS: every level's vectors live in LDS (sc.lds_words > 0).  A separate
// instantiation, so that every level pointer derives from the LDS array and
// the stencil loads compile to LDS reads rather than generic (flat) loads.
template <typename T, int G, bool LDS>
__global__ void __launch_bounds__(kSmallBlock) k_vcycle_small(const SmallLevel<T>* __restrict__ lv, SmallCycle<T> sc) {
  __shared__ double red[kSmallBlock];
  __shared__ double rs[2048];
  extern __shared__ __align__(16) unsigned char lds_raw[];
  T* const sm = reinterpret_cast<T*>(lds_raw);
  constexpr bool lds = LDS;
  using V = typename SmallVec<T, LDS>::type;
  const int top = sc.nlev - 1;
  // the level vectors: LDS copies, or the work vectors (x, b of the call on top)
  auto vw = [&](int q) { return 3 * lv[q].g.vstride + lv[q].g.nn; };
  auto X = [&](int q) -> V {
    if constexpr (LDS) return (V)(sm + lv[q].lds_off);
    else return q == top ? sc.x : lv[q].cx;
  };
  auto B = [&](int q) -> V {
    if constexpr (LDS) return (V)(sm + lv[q].lds_off + vw(q));
    else return q == top ? const_cast<T*>(sc.b) : lv[q].cb;
  };
  auto R = [&](int q) -> V {
    if constexpr (LDS) return (V)(sm + lv[q].lds_off + 2 * vw(q));
    else return lv[q].r;
  };
  if (lds) {
    V xs = X(top);
    V bs = B(top);
    for (int t = threadIdx.x; t < vw(top); t += kSmallBlock) {
      xs[t] = sc.x[t];
      bs[t] = sc.b[t];
    }
    __syncthreads();
  }
  // descend: smooth, residual, restrict (+ zero-sum pressure), zero correction
  for (int q = top; q >= 1; --q) {
    const SmallLevel<T>& L = lv[q];
    const SmallLevel<T>& C = lv[q - 1];
    V x = X(q);
    V b = B(q);
    small_smooth_any<T, G>(sc, L, x, b, R(q), sc.pre0 + (top - q) * sc.inc, q < sc.q16);
    small_residual<T, G>(sc, L, x, b, R(q));
    small_round<T>(q < sc.q16, R(q), 0, 0, vw(q), 1);
    V cb = B(q - 1);
    V r = R(q);
    for (int w = threadIdx.x; w < (3 * G + 1) * C.g.nn; w += kSmallBlock)
      restrict_site<T, G>(L.g, C.g, (const T*)r, (T*)cb, w % C.g.nn, w / C.g.nn);
    __syncthreads();
    small_round<T>(q - 1 < sc.q16, cb, 0, 0, vw(q - 1), 1);
    small_pshift<T>(C, cb + 3 * (size_t)C.g.vstride, 1, red);
    small_round<T>(q - 1 < sc.q16, cb, 0, 3 * C.g.vstride, C.g.nn, 1);
    V cx = X(q - 1);
    for (int t = threadIdx.x; t < vw(q - 1); t += kSmallBlock) cx[t] = T(0);
    __syncthreads();
  }
  // coarsest level: x += K^+ (b - calA x) on the unknowns, zero pressure mean
  {
    const SmallLevel<T>& L = lv[0];
    V x = X(0);
    V r = R(0);
    small_residual<T, G>(sc, L, x, B(0), R(0));
    small_round<T>(0 < sc.q16, R(0), 0, 0, vw(0), 1);
    for (int c = threadIdx.x; c < sc.nunk; c += kSmallBlock) rs[c] = (double)r[sc.unk[c]];
    __syncthreads();
    for (int row = threadIdx.x; row < sc.nunk; row += kSmallBlock) {
      const double* kr = sc.Kp + (size_t)row * sc.nunk;
      double acc = 0.0;
      for (int c = 0; c < sc.nunk; ++c) acc += kr[c] * rs[c];
      x[sc.unk[row]] = (T)((double)x[sc.unk[row]] + acc);
    }
    __syncthreads();
    small_round<T>(0 < sc.q16, x, 0, 0, vw(0), 1);
    small_pshift<T>(L, x + 3 * (size_t)L.g.vstride, 0, red);
    small_round<T>(0 < sc.q16, x, 0, 3 * L.g.vstride, L.g.nn, 1);
  }
  // ascend: prolongate and add, post-smooth
  for (int q = 1; q <= top; ++q) {
    const SmallLevel<T>& L = lv[q];
    const SmallLevel<T>& C = lv[q - 1];
    V x = X(q);
    V xc = X(q - 1);
    for (int t = threadIdx.x; t < L.g.nn; t += kSmallBlock)
      prolong_site<T, G>(C.g, L.g, L.tt, (const T*)xc, (T*)x, 1, 1, t);
    __syncthreads();
    small_round<T>(q < sc.q16, x, 0, 0, vw(q), 1);
    small_smooth_any<T, G>(sc, L, x, B(q), R(q), sc.post0 + (top - q) * sc.inc, q < sc.q16);
  }
  if (lds) {
    V xs = X(top);
    for (int t = threadIdx.x; t < vw(top); t += kSmallBlock) sc.x[t] = xs[t];
  }
}

// E[c stride + unk[c]] = 1 for c < n: the unit vectors of the coarse unknowns
// (columns of the dense coarse operator), E zero-filled by the caller.
__global__ void __launch_bounds__(kBlock) k_unit_columns(double* __restrict__ E, long stride,
                                                         const int* __restrict__ unk, int n) {
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c < n) E[c * stride + unk[c]] = 1.0;
}

// Coarsest level: x[unk] += Kp r[unk] (one workgroup, unknowns staged in LDS,
// float64 arithmetic whatever the storage type T).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_coarse(const double* __restrict__ Kp, const int* __restrict__ unk, int n,
                                                   const T* __restrict__ r, T* __restrict__ x) {
  __shared__ double rs[2048];
  for (int c = threadIdx.x; c < n; c += kBlock) rs[c] = (double)r[unk[c]];
  __syncthreads();
  for (int row = threadIdx.x; row < n; row += kBlock) {
    const double* kr = Kp + (size_t)row * n;
    double acc = 0.0;
    for (int c = 0; c < n; ++c) acc += kr[c] * rs[c];
    x[unk[row]] = (T)((double)x[unk[row]] + acc);
  }
}

// Coarse-level MLP features: f[c] = r[unk[c]] / ||r_unk||, c < nunk, then
// log nu at the nn P1 nodes (0 without a viscosity); norm[0] = ||r_unk||.
__global__ void __launch_bounds__(kBlock) k_coarse_features(const double* __restrict__ r, const int* __restrict__ unk,
                                                            int nunk, const double* __restrict__ nu, int nn,
                                                            float* __restrict__ f, double* __restrict__ norm) {
  __shared__ double s[kBlock];
  double a = 0.0;
  for (int c = threadIdx.x; c < nunk; c += kBlock) {
    const double v = r[unk[c]];
    a += v * v;
  }
  s[threadIdx.x] = a;
  __syncthreads();
  for (int k = kBlock / 2; k > 0; k >>= 1) {
    if (threadIdx.x < k) s[threadIdx.x] += s[threadIdx.x + k];
    __syncthreads();
  }
  const double nr = sqrt(s[0]);
  const double inv = nr > 0.0 ? 1.0 / nr : 0.0;
  for (int c = threadIdx.x; c < nunk; c += kBlock) f[c] = (float)(r[unk[c]] * inv);
  for (int q = threadIdx.x; q < nn; q += kBlock) f[nunk + q] = nu ? (float)log(nu[q]) : 0.f;
  if (threadIdx.x == 0) norm[0] = nr;
}

// x[unk[c]] += norm * y[c] (the learned correction), or out[c] = x[unk[c]] / norm.
__global__ void __launch_bounds__(kBlock) k_coarse_scatter(const float* __restrict__ y, const int* __restrict__ unk,
                                                           int nunk, const double* __restrict__ norm,
                                                           double* __restrict__ x, float* __restrict__ out) {
  for (int c = blockIdx.x * kBlock + threadIdx.x; c < nunk; c += gridDim.x * kBlock) {
    if (out)
      out[c] = norm[0] > 0.0 ? (float)(x[unk[c]] / norm[0]) : 0.f;
    else
      x[unk[c]] += norm[0] * (double)y[c];
  }
}

// Rows idx[0..B) of src (n x w floats) -> dst (B x w).
__global__ void k_gather_rows(const float* __restrict__ src, const int* __restrict__ idx, int B, int w,
                              float* __restrict__ dst) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long)B * w) return;
  dst[t] = src[(long)idx[t / w] * w + t % w];
}

// y (precision Y) = x (precision X), round to nearest even when narrowing.
template <typename X, typename Y>
__global__ void __launch_bounds__(kBlock) k_convert(const X* __restrict__ x, Y* __restrict__ y, long n) {
  const long t = (long)blockIdx.x * kBlock + threadIdx.x;
  if (t < n) y[t] = (Y)x[t];
}

// x[s * stride + off + t] = round_bf16(...) for s < nseg, t < n.
__global__ void __launch_bounds__(kBlock) k_round_bf16(float* __restrict__ x, long stride, long off, long n,
                                                       int nseg) {
  const long t = (long)blockIdx.x * kBlock + threadIdx.x;
  if (t >= n * nseg) return;
  const long seg = t / n, i = t - seg * n;
  float* p = x + seg * stride + off + i;
  *p = round_bf16(*p);
}

// y += (double) e
template <typename X>
__global__ void __launch_bounds__(kBlock) k_add_to_f64(double* __restrict__ y, const X* __restrict__ e, long n) {
  const long t = (long)blockIdx.x * kBlock + threadIdx.x;
  if (t < n) y[t] += (double)e[t];
}

}  // namespace

// ---------------------------------------------------------------- launchers
#define HHG_LAUNCH(kernel, grid, stream, ...) hipLaunchKernelGGL(kernel, dim3(grid), dim3(kBlock), 0, stream, __VA_ARGS__)

static double p_sites(const Geom& g) {
  const double m = g.G == 1 ? g.N + 1 : 2 * g.N + 1;
  return m * m * m;
}

template <typename T>
void launch_apply(hipStream_t s, const Geom& g, const LevelConst<T>& lc, const Tables<T>* tb, const T* x, const T* b,
                  T* y, int opmask, bool has_b, bool vel_rows, bool p_rows, const int* bnd, int nbnd,
                  const PStep<T>& ps) {
  if (!(vel_rows || p_rows)) return;
  KScope ks(s, KF_APPLY, p_sites(g));
  const int hb = has_b, vr = vel_rows, pr = p_rows;
  const int full = g.G == 1 ? 15 : 7;
  const int nb_bnd = p_rows ? nbnd : 0;
  if (!lc.nu && opmask == full && p_rows) {
    // k-marching form: 62 output columns per block, k in chunks of kc planes;
    // the boundary pressure rows in extra blocks of 192 threads
    // chunk length: HHG_ZM_KC planes, halved (down to 2) while the grid has
    // fewer than ~1000 blocks -- on the small levels a chunk is a chain of
    // dependent plane steps, so short chunks (more blocks) win over the
    // re-read halo planes
    const int ncb = (g.n1 * g.n1 + kZmOut - 1) / kZmOut;
    int kc = std::min(HHG_ZM_KC, g.n1);
    while (kc > 2 && ncb * ((g.n1 + kc - 1) / kc) < 1024) kc = (kc + 1) / 2;
    const int nch = (g.n1 + kc - 1) / kc;
    const int nmain = (ncb * nch + 7) & ~7;
    const int nextra = (nb_bnd + kZmCols - 1) / kZmCols;  // 64 boundary nodes per block
    const dim3 grid(nmain + nextra), block(3 * kZmCols);
    // float32 P2-P1: the kernel's registers allow 8 resident workgroups per
    // CU, but the columns of more than 3 workgroups in flight evict each
    // other's j-neighbour rows from L2 before they are re-read (measured on
    // the 48-tet level-7 lattice: 8 -> 1.23 ms, 4 -> 1.16 ms, 3 -> 1.14 ms,
    // 2 -> 1.36 ms).  Unused dynamic LDS caps residency at 3 of the CU's
    // 160 KiB, for float64 too (below).  The cap pays on that lattice only (n1 = 257); on the
    // smaller ones the columns in flight fit the L2 anyway (n1 = 65: 0.034 ->
    // 0.028 ms uncapped; n1 = 129: 0.193 -> 0.188).  P1-P1 loads a third of
    // the words per plane and needs the waves to hide their latency: no cap
    // (n1 = 257, float32: 3 workgroups 0.381 ms, 4 0.383, 6 0.278, uncapped
    // 0.215).
    // vel_rows false: the pressure rows only (the Uzawa pressure residual):
    // the velocity words are still loaded for B u, the velocity rows are
    // neither accumulated nor written and their b words not read
    // float64 at 114 VGPRs would hold 5 workgroups per CU; the same cap to 3
    // measured 2.158 -> 2.102 ms on the n1 = 257 lattice (4: 2.135 ms)
    const unsigned dyn = g.G == 8 && g.n1 >= 200 ? kZmF32Lds : 0;
    // the fused pressure step: the pressure-residual form only
    const bool fused = ps.p && !vel_rows && has_b;
    // Taylor-Hood pressure residual on lattices up to 33 nodes per edge: the
    // per-node split form (6-tet FMG to level 5: 3.206 -> 3.187 ms; the same
    // up to 65 nodes: 3.186 ms)
    if (g.G == 8 && !vel_rows && has_b && g.n1 <= 33) {
      const int nr = g.N - 1;
      const int ninner = (nr * nr * nr + kZmCols - 1) / kZmCols;
      const int nbb = (nb_bnd + kZmCols - 1) / kZmCols;
      hipLaunchKernelGGL((k_prow_split<T>), dim3(ninner + nbb), dim3(3 * kZmCols), 0, s, g, lc, x, b, y, bnd, nb_bnd,
                         ninner, ps);
      return;
    }
    auto go = [&](auto gg, auto vel, auto hbc) {
      constexpr int GG = decltype(gg)::value;
      constexpr bool V = decltype(vel)::value, H = decltype(hbc)::value;
      hipLaunchKernelGGL((k_apply_zm<T, GG, V, H>), grid, block, dyn, s, g, lc, x, b, y, kc, ncb, bnd, nb_bnd, nmain,
                         fused ? ps : PStep<T>{});
    };
    using I1 = std::integral_constant<int, 1>;
    using I8 = std::integral_constant<int, 8>;
    using BT = std::true_type;
    using BF = std::false_type;
    if (g.G == 1) {
      if (vel_rows)
        hb ? go(I1{}, BT{}, BT{}) : go(I1{}, BT{}, BF{});
      else
        hb ? go(I1{}, BF{}, BT{}) : go(I1{}, BF{}, BF{});
    } else {
      if (vel_rows)
        hb ? go(I8{}, BT{}, BT{}) : go(I8{}, BT{}, BF{});
      else
        hb ? go(I8{}, BF{}, BT{}) : go(I8{}, BF{}, BF{});
    }
    if (ps.p && !fused)
      HHG_LAUNCH((k_pstep<T>), nblocks(g.nn), s, g.nn, ps.dinv, ps.p, y + 3 * (size_t)g.vstride, ps.omega);
  } else {
    const int nmain = (int)nblocks8(g.nn);
    const unsigned nb = (unsigned)(nmain + (nb_bnd + kBlock - 1) / kBlock);
    if (g.G == 1) {
      if (lc.nu)
        HHG_LAUNCH((k_apply<T, 1, true>), nb, s, g, lc, x, b, y, opmask, hb, vr, pr, bnd, nb_bnd, nmain);
      else
        HHG_LAUNCH((k_apply<T, 1, false>), nb, s, g, lc, x, b, y, opmask, hb, vr, pr, bnd, nb_bnd, nmain);
    } else {
      if (lc.nu)
        HHG_LAUNCH((k_apply<T, 8, true>), nb, s, g, lc, x, b, y, opmask, hb, vr, pr, bnd, nb_bnd, nmain);
      else
        HHG_LAUNCH((k_apply<T, 8, false>), nb, s, g, lc, x, b, y, opmask, hb, vr, pr, bnd, nb_bnd, nmain);
    }
    if (ps.p)  // the per-site form stores the residual; the step follows
      HHG_LAUNCH((k_pstep<T>), nblocks(g.nn), s, g.nn, ps.dinv, ps.p, y + 3 * (size_t)g.vstride, ps.omega);
  }
  (void)tb;
}

// Launch, with the packet-stamped events of a KScope opened with packet = true.
template <typename K, typename... Args>
void launch_timed(const KScope& ks, K kernel, dim3 grid, dim3 block, hipStream_t s, Args... args) {
  if (ks.packet_)
    hipExtLaunchKernelGGL(kernel, grid, block, 0, s, ks.a_, ks.b_, 0, args...);
  else
    hipLaunchKernelGGL(kernel, grid, block, 0, s, args...);
}

template <typename T>
void launch_gs_colour(hipStream_t s, const Geom& g, const LevelConst<T>& lc, T* x, const T* b, int colour) {
  const int N = g.N;
  if (N < 2) return;
  if (colour < kGsVertexColours) {
    const int nr = N - 1, ni = (nr + 1) / 2;
    double cnt = 0;
    if (timer().mask & (1u << KF_GS_VERTEX))
      for (int k = 1; k <= nr; ++k)
        for (int j = 1; j <= nr; ++j) {
          const int i0 = 1 + ((colour + 1 + j + k) & 1);
          if (i0 <= nr) cnt += (nr - i0) / 2 + 1;
        }
    KScope ks(s, KF_GS_VERTEX, cnt, true);
    const dim3 grid(nblocks((size_t)ni * nr * nr), 3), block(kBlock);
    if (g.G == 1) {
      if (lc.nu)
        launch_timed(ks, k_gs_vertex<T, 1, true>, grid, block, s, g, lc, x, b, colour);
      else
        launch_timed(ks, k_gs_vertex<T, 1, false>, grid, block, s, g, lc, x, b, colour);
    } else {
      if (lc.nu)
        launch_timed(ks, k_gs_vertex<T, 8, true>, grid, block, s, g, lc, x, b, colour);
      else
        launch_timed(ks, k_gs_vertex<T, 8, false>, grid, block, s, g, lc, x, b, colour);
    }
  } else {
    const int gr = colour - kGsVertexColours + 1;
    const size_t n = (size_t)gs_edge_count(g, gr);
    KScope ks(s, KF_GS_EDGE, (double)n, true);
    const dim3 grid(nblocks(n), 3), block(kBlock);
#define HHG_GS_EDGE(GR)                                                               \
  case GR:                                                                            \
    if (lc.nu)                                                                        \
      launch_timed(ks, k_gs_edge<T, true, GR>, grid, block, s, g, lc, x, b);          \
    else                                                                              \
      launch_timed(ks, k_gs_edge<T, false, GR>, grid, block, s, g, lc, x, b);         \
    break
    switch (gr) {
      HHG_GS_EDGE(1); HHG_GS_EDGE(2); HHG_GS_EDGE(3); HHG_GS_EDGE(4);
      HHG_GS_EDGE(5); HHG_GS_EDGE(6); HHG_GS_EDGE(7);
      default: break;
    }
#undef HHG_GS_EDGE
  }
}

template <typename T>
void launch_pressure_step(hipStream_t s, const Geom& g, const T* dinv, T* x, const T* rp, T omega) {
  KScope ks(s, KF_PSTEP, g.nn);
  HHG_LAUNCH((k_pstep<T>), nblocks(g.nn), s, g.nn, dinv, x + 3 * (size_t)g.vstride, rp + 3 * (size_t)g.vstride, omega);
}

template <typename T>
void launch_schur_diag(hipStream_t s, const Geom& g, const Tables<T>* tb, const T* ainv_site, int mode, T* dinv,
                       const NeuTables<T>* nt) {
  if (g.G == 1)
    HHG_LAUNCH((k_schur_diag<T, 1>), nblocks(g.nn), s, g, tb, ainv_site, mode, dinv, nt);
  else
    HHG_LAUNCH((k_schur_diag<T, 8>), nblocks(g.nn), s, g, tb, ainv_site, mode, dinv, nt);
}

template <typename T>
void launch_neu_rows(hipStream_t s, const Geom& g, const NeuTables<T>* nt, NeuList L, int first, int n, const T* x,
                     const T* b, T* y, int opmask, bool has_b) {
  if (n <= 0 || !(opmask & 3)) return;
  KScope ks(s, KF_NEUMANN, n);
  hipLaunchKernelGGL((k_neu_rows<T>), dim3(nblocks(n), 3), dim3(kBlock), 0, s, g, nt, L, first, n, x, b, y, opmask,
                     (int)has_b);
}

template <typename T>
void launch_neu_gs(hipStream_t s, const Geom& g, const NeuTables<T>* nt, NeuList L, int first, int n, T* x,
                   const T* b) {
  if (n <= 0) return;
  KScope ks(s, KF_NEUMANN, n);
  hipLaunchKernelGGL((k_neu_gs<T>), dim3(nblocks(n), 3), dim3(kBlock), 0, s, g, nt, L, first, n, x, b);
}

template <typename T>
void launch_neu_rhs(hipStream_t s, const Geom& g, const Tables<T>* tb, NeuList L, int n, const T* f, T* b) {
  if (n <= 0) return;
  hipLaunchKernelGGL((k_neu_rhs<T>), dim3(nblocks(n), 3), dim3(kBlock), 0, s, g, tb, L, n, f, b);
}

template <typename T>
void launch_neu_restrict(hipStream_t s, const Geom& gf, const Geom& gc, const NeuTables<T>* ntc, NeuList Lc, int n,
                         const T* rf, T* rc) {
  if (n <= 0) return;
  KScope ks(s, KF_NEUMANN, n);
  hipLaunchKernelGGL((k_neu_restrict<T>), dim3(nblocks(n), 3), dim3(kBlock), 0, s, gf, gc, ntc, Lc, n, rf, rc);
}

template <typename T>
void launch_neu_prolong(hipStream_t s, const Geom& gc, const Geom& gf, const TransferTables<T>* tt, NeuList Lf, int n,
                        const T* xc, T* xf) {
  if (n <= 0) return;
  KScope ks(s, KF_NEUMANN, n);
  if (gf.G == 1)
    hipLaunchKernelGGL((k_neu_prolong<T, 1>), dim3(nblocks(n), 3), dim3(kBlock), 0, s, gc, gf, tt, Lf, n, xc, xf);
  else
    hipLaunchKernelGGL((k_neu_prolong<T, 8>), dim3(nblocks(n), 3), dim3(kBlock), 0, s, gc, gf, tt, Lf, n, xc, xf);
}

template <typename T>
void launch_nu_diag(hipStream_t s, const Geom& g, const LevelConst<T>& lc, T* ainv_site) {
  if (g.G == 1)
    HHG_LAUNCH((k_nu_diag<T, 1>), nblocks(g.nn), s, g, lc, ainv_site);
  else
    HHG_LAUNCH((k_nu_diag<T, 8>), nblocks(g.nn), s, g, lc, ainv_site);
}

template <typename T>
void launch_rhs(hipStream_t s, const Geom& g, const LevelConst<T>& lc, const T* f, T* b) {
  if (g.G == 1)
    HHG_LAUNCH((k_rhs<T, 1>), nblocks(g.nn), s, g, lc, f, b);
  else
    HHG_LAUNCH((k_rhs<T, 8>), nblocks(g.nn), s, g, lc, f, b);
}

template <typename T>
void launch_mass(hipStream_t s, const Geom& g, const Tables<T>* tb, const T* x, T* y) {
  KScope ks(s, KF_OTHER, p_sites(g));
  if (g.G == 1)
    HHG_LAUNCH((k_mass<T, 1>), nblocks(g.nn), s, g, tb, x, y);
  else
    HHG_LAUNCH((k_mass<T, 8>), nblocks(g.nn), s, g, tb, x, y);
}

template <typename T>
void launch_dot(hipStream_t s, const T* x, const T* y, size_t n, double* partial, double* out) {
  size_t b = (n + kBlock - 1) / kBlock;
  const int nb = (int)(b < (size_t)kPartials ? (b == 0 ? 1 : b) : kPartials);
  KScope ks(s, KF_REDUCE, (double)n);
  HHG_LAUNCH((k_dot<T>), nb, s, x, y, (long)n, partial);
  HHG_LAUNCH(k_final_sum, 1, s, partial, nb, out);
}

template <typename T>
void launch_restrict(hipStream_t s, const Geom& gf, const Geom& gc, const TransferTables<T>* tt, const T* rf, T* rc,
                     T* zero_x) {
  KScope ks(s, KF_RESTRICT, p_sites(gf));
  (void)tt;
  // grid.y: (velocity group, component) slices and the pressure
  if (gc.G == 1) {
    hipLaunchKernelGGL((k_restrict<T, 1>), dim3(nblocks(gc.nn), 4), dim3(kBlock), 0, s, gf, gc, rf, rc, 0, zero_x);
  } else if (gc.n1 >= 33) {
    // velocity: the k-marching form; the pressure slice as before.  From a
    // coarse lattice of 33 nodes per edge on (48-tet cube, level 7 -> 6:
    // 3.52 -> 1.05 ms in float64, 13.5 % -> 45 % of HBM; level 6 -> 5 0.350
    // -> 0.147 ms); on the FMG's small levels the per-site gather is as fast
    // (6-tet cube, FMG to level 5 with it on every level: 4.21 -> 4.25 ms)
    const int ncb = (gc.n1 * gc.n1 + kRzmCols - 3) / (kRzmCols - 2);
    int kc = std::min(HHG_RZM_KC, gc.n1);
    while (kc > 2 && ncb * ((gc.n1 + kc - 1) / kc) < 1024) kc = (kc + 1) / 2;
    const int nch = (gc.n1 + kc - 1) / kc;
    const int nmain = (ncb * nch + 7) & ~7;
    hipLaunchKernelGGL((k_restrict_zm<T>), dim3(nmain), dim3(3 * kRzmCols), 0, s, gf, gc, rf, rc, kc, ncb, nmain,
                       zero_x);
    hipLaunchKernelGGL((k_restrict<T, 8>), dim3(nblocks(gc.nn), 1), dim3(kBlock), 0, s, gf, gc, rf, rc, 24, zero_x);
  } else {
    hipLaunchKernelGGL((k_restrict<T, 8>), dim3(nblocks(gc.nn), 25), dim3(kBlock), 0, s, gf, gc, rf, rc, 0, zero_x);
  }
}

template <typename T>
void launch_prolong(hipStream_t s, const Geom& gc, const Geom& gf, const TransferTables<T>* tt, const T* xc, T* xf,
                    bool add, bool skip_boundary) {
  KScope ks(s, KF_PROLONG, p_sites(gf));
  const dim3 block(kBlock);
  // From a fine lattice of 65 nodes per edge on: a thread per (coarse cube,
  // slice), generated interpolation (48-tet cube, level 6 -> 7, float64:
  // P2-P1 4.06 -> 1.47 ms, 22 % -> 61 % of 8 TB/s; P1-P1 0.73 -> 0.25 ms);
  // on the FMG's small levels the per-site slices keep more threads in
  // flight (6-tet FMG to level 5 with cubes everywhere: 4.20 -> 4.27 ms)
  if (gf.n1 >= 65) {
    const dim3 grid(nblocks(gc.nn), 4);
    if (gf.G == 1) {
      if (add)
        hipLaunchKernelGGL((k_prolong_cube<T, 1, true>), grid, block, 0, s, gc, gf, xc, xf, (int)skip_boundary);
      else
        hipLaunchKernelGGL((k_prolong_cube<T, 1, false>), grid, block, 0, s, gc, gf, xc, xf, (int)skip_boundary);
    } else {
      if (add)
        hipLaunchKernelGGL((k_prolong_cube<T, 8, true>), grid, block, 0, s, gc, gf, xc, xf, (int)skip_boundary);
      else
        hipLaunchKernelGGL((k_prolong_cube<T, 8, false>), grid, block, 0, s, gc, gf, xc, xf, (int)skip_boundary);
    }
  } else if (gf.G == 1)
    hipLaunchKernelGGL((k_prolong<T, 1>), dim3(nblocks(gf.nn), 4), block, 0, s, gc, gf, tt, xc, xf, (int)add,
                       (int)skip_boundary);
  else
    hipLaunchKernelGGL((k_prolong<T, 8>), dim3(nblocks(gf.nn), 25), block, 0, s, gc, gf, tt, xc, xf, (int)add,
                       (int)skip_boundary);
}

template <typename T>
void launch_inject_boundary(hipStream_t s, const Geom& gf, const Geom& gc, const T* xf, T* xc) {
  if (gc.G == 1)
    HHG_LAUNCH((k_inject_boundary<T, 1>), nblocks(gc.nn), s, gf, gc, xf, xc);
  else
    HHG_LAUNCH((k_inject_boundary<T, 8>), nblocks(gc.nn), s, gf, gc, xf, xc);
}

template <typename T>
void launch_copy_boundary(hipStream_t s, const Geom& g, const T* src, T* dst) {
  if (g.G == 1)
    HHG_LAUNCH((k_copy_boundary<T, 1>), nblocks(g.nn), s, g, src, dst);
  else
    HHG_LAUNCH((k_copy_boundary<T, 8>), nblocks(g.nn), s, g, src, dst);
}

template <typename T>
static size_t lattice_words(const Geom& g) {
  const size_t m1 = (g.G == 1 ? g.N : 2 * g.N) + 1;
  return 3 * m1 * m1 * m1 + (size_t)g.nn;
}

template <typename T>
void launch_from_lattice(hipStream_t s, const Geom& g, const double* src, T* dst) {
  const size_t n = lattice_words<T>(g);
  if (g.G == 1)
    HHG_LAUNCH((k_lattice<T, 1>), nblocks(n), s, g, src, dst, nullptr, nullptr, 0);
  else
    HHG_LAUNCH((k_lattice<T, 8>), nblocks(n), s, g, src, dst, nullptr, nullptr, 0);
}

template <typename T>
void launch_to_lattice(hipStream_t s, const Geom& g, const T* src, double* dst) {
  const size_t n = lattice_words<T>(g);
  if (g.G == 1)
    HHG_LAUNCH((k_lattice<T, 1>), nblocks(n), s, g, nullptr, nullptr, dst, src, 1);
  else
    HHG_LAUNCH((k_lattice<T, 8>), nblocks(n), s, g, nullptr, nullptr, dst, src, 1);
}

static int reduce_grid(size_t n) {
  size_t b = (n + kBlock - 1) / kBlock;
  return (int)(b < (size_t)kPartials ? (b == 0 ? 1 : b) : kPartials);
}

template <typename T>
void launch_psum(hipStream_t s, const Geom& g, const Tables<T>* tb, const T* p, double* partial, double* out,
                 int mode) {
  const int nb = reduce_grid(g.nn);
  KScope ks(s, KF_REDUCE, g.nn);
  HHG_LAUNCH((k_psum<T>), nb, s, g, tb, p, partial, mode);
  HHG_LAUNCH(k_final_sum, 1, s, partial, nb, out);
}

template <typename T>
void launch_mean_zero(hipStream_t s, const Geom& g, const Tables<T>* tb, T* p, double* partial, double* sums,
                      int mode) {
  if (g.nn <= kMeanOneBlock) {
    KScope ks(s, KF_REDUCE, g.nn);
    hipLaunchKernelGGL((k_mean_zero_1b<T>), dim3(1), dim3(kMeanBlock), 0, s, g, tb, p, sums, mode);
  } else {
    launch_psum<T>(s, g, tb, p, partial, sums, mode);
    launch_pshift<T>(s, g, p, sums, mode);
  }
}

template <typename T>
void launch_pshift(hipStream_t s, const Geom& g, T* p, const double* sums, int mode) {
  KScope ks(s, KF_REDUCE, g.nn);
  HHG_LAUNCH((k_pshift<T>), nblocks(g.nn), s, g.nn, p, sums, mode);
}

template <typename T>
void launch_vsumsq(hipStream_t s, const Geom&, const T* x, int nwords, double* partial, double* out) {
  const int nb = reduce_grid((size_t)nwords);
  KScope ks(s, KF_REDUCE, nwords);
  HHG_LAUNCH((k_sumsq<T>), nb, s, x, (long)nwords, partial);
  HHG_LAUNCH(k_final_sum, 1, s, partial, nb, out);
}

template <typename T>
void launch_coarse(hipStream_t s, const double* Kp, const int* unk, int nunk, const T* r, T* x) {
  KScope ks(s, KF_COARSE, nunk);
  HHG_LAUNCH((k_coarse<T>), 1, s, Kp, unk, nunk, r, x);
}

template <typename T>
void launch_vcycle_small(hipStream_t s, const SmallLevel<T>* lv, const SmallCycle<T>& sc) {
  KScope ks(s, KF_SMALL, sc.nlev);
  const size_t lds = (size_t)sc.lds_words * sizeof(T);
  const dim3 grid(1), block(kSmallBlock);
  if (sc.G == 1) {
    if (lds)
      hipLaunchKernelGGL((k_vcycle_small<T, 1, true>), grid, block, lds, s, lv, sc);
    else
      hipLaunchKernelGGL((k_vcycle_small<T, 1, false>), grid, block, 0, s, lv, sc);
  } else {
    if (lds)
      hipLaunchKernelGGL((k_vcycle_small<T, 8, true>), grid, block, lds, s, lv, sc);
    else
      hipLaunchKernelGGL((k_vcycle_small<T, 8, false>), grid, block, 0, s, lv, sc);
  }
}

template <typename T, int G>
void small_attributes_of(int bytes) {
  (void)hipFuncSetAttribute((const void*)k_vcycle_small<T, G, true>, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}
void small_kernel_attributes() {
  small_attributes_of<double, 1>(kSmallLdsBytes);
  small_attributes_of<double, 8>(kSmallLdsBytes);
  small_attributes_of<float, 1>(kSmallLdsBytes);
  small_attributes_of<float, 8>(kSmallLdsBytes);
}

void launch_unit_columns(hipStream_t s, double* E, size_t stride, const int* unk, int n) {
  if (n > 0) HHG_LAUNCH(k_unit_columns, nblocks(n), s, E, (long)stride, unk, n);
}

void launch_coarse_features(hipStream_t s, const double* r, const int* unk, int nunk, const double* nu, int nn,
                            float* f, double* norm) {
  KScope ks(s, KF_COARSE, nunk);
  HHG_LAUNCH(k_coarse_features, 1, s, r, unk, nunk, nu, nn, f, norm);
}

void launch_coarse_scatter(hipStream_t s, const float* y, const int* unk, int nunk, const double* norm, double* x,
                           float* out) {
  KScope ks(s, KF_COARSE, nunk);
  HHG_LAUNCH(k_coarse_scatter, nblocks(nunk), s, y, unk, nunk, norm, x, out);
}

void launch_gather_rows(hipStream_t s, const float* src, const int* idx, int B, int w, float* dst) {
  if ((long)B * w > 0) HHG_LAUNCH(k_gather_rows, nblocks((size_t)B * w), s, src, idx, B, w, dst);
}

void launch_to_f32(hipStream_t s, const double* x, float* y, size_t n) {
  if (n) HHG_LAUNCH((k_convert<double, float>), nblocks(n), s, x, y, (long)n);
}

void launch_round_bf16(hipStream_t s, float* x, size_t stride, size_t off, size_t n, int nseg) {
  if (n && nseg) HHG_LAUNCH(k_round_bf16, nblocks(n * (size_t)nseg), s, x, (long)stride, (long)off, (long)n, nseg);
}

void launch_add_f32_to_f64(hipStream_t s, double* y, const float* e, size_t n) {
  if (n) HHG_LAUNCH((k_add_to_f64<float>), nblocks(n), s, y, e, (long)n);
}

template <typename T>
void launch_scale(hipStream_t s, T* x, size_t n, const double* sums, int slot) {
  HHG_LAUNCH((k_scale<T>), nblocks(n), s, x, (long)n, sums, slot);
}

template <typename T>
void launch_scaled_copy(hipStream_t s, T* y, const T* x, const T* d, size_t n, T a) {
  if (n) HHG_LAUNCH((k_scaled_copy<T>), nblocks(n), s, y, x, d, (long)n, a);
}

template <typename T>
void launch_fill(hipStream_t s, T* x, size_t n, T v) {
  if (n) HHG_LAUNCH((k_fill<T>), nblocks(n), s, x, (long)n, v);
}

template <typename T>
void launch_axpy(hipStream_t s, T* y, const T* x, size_t n, T a) {
  if (n) HHG_LAUNCH((k_axpy<T>), nblocks(n), s, y, x, (long)n, a);
}

#define HHG_INSTANTIATE(T)                                                                                          \
  template void launch_apply<T>(hipStream_t, const Geom&, const LevelConst<T>&, const Tables<T>*, const T*,        \
                                const T*, T*, int, bool, bool, bool, const int*, int, const PStep<T>&);             \
  template void launch_gs_colour<T>(hipStream_t, const Geom&, const LevelConst<T>&, T*, const T*, int);             \
  template void launch_pressure_step<T>(hipStream_t, const Geom&, const T*, T*, const T*, T);                       \
  template void launch_schur_diag<T>(hipStream_t, const Geom&, const Tables<T>*, const T*, int, T*,                 \
                                     const NeuTables<T>*);                                                          \
  template void launch_neu_rows<T>(hipStream_t, const Geom&, const NeuTables<T>*, NeuList, int, int, const T*,      \
                                   const T*, T*, int, bool);                                                        \
  template void launch_neu_gs<T>(hipStream_t, const Geom&, const NeuTables<T>*, NeuList, int, int, T*, const T*);   \
  template void launch_neu_rhs<T>(hipStream_t, const Geom&, const Tables<T>*, NeuList, int, const T*, T*);          \
  template void launch_neu_restrict<T>(hipStream_t, const Geom&, const Geom&, const NeuTables<T>*, NeuList, int,    \
                                       const T*, T*);                                                               \
  template void launch_neu_prolong<T>(hipStream_t, const Geom&, const Geom&, const TransferTables<T>*, NeuList,     \
                                      int, const T*, T*);                                                           \
  template void launch_nu_diag<T>(hipStream_t, const Geom&, const LevelConst<T>&, T*);                              \
  template void launch_rhs<T>(hipStream_t, const Geom&, const LevelConst<T>&, const T*, T*);                        \
  template void launch_mass<T>(hipStream_t, const Geom&, const Tables<T>*, const T*, T*);                           \
  template void launch_dot<T>(hipStream_t, const T*, const T*, size_t, double*, double*);                           \
  template void launch_restrict<T>(hipStream_t, const Geom&, const Geom&, const TransferTables<T>*, const T*, T*,  \
                                   T*);                                                                             \
  template void launch_prolong<T>(hipStream_t, const Geom&, const Geom&, const TransferTables<T>*, const T*, T*,    \
                                  bool, bool);                                                                      \
  template void launch_inject_boundary<T>(hipStream_t, const Geom&, const Geom&, const T*, T*);                     \
  template void launch_copy_boundary<T>(hipStream_t, const Geom&, const T*, T*);                                    \
  template void launch_from_lattice<T>(hipStream_t, const Geom&, const double*, T*);                                \
  template void launch_to_lattice<T>(hipStream_t, const Geom&, const T*, double*);                                  \
  template void launch_psum<T>(hipStream_t, const Geom&, const Tables<T>*, const T*, double*, double*, int);        \
  template void launch_pshift<T>(hipStream_t, const Geom&, T*, const double*, int);                                 \
  template void launch_mean_zero<T>(hipStream_t, const Geom&, const Tables<T>*, T*, double*, double*, int);         \
  template void launch_vsumsq<T>(hipStream_t, const Geom&, const T*, int, double*, double*);                        \
  template void launch_scale<T>(hipStream_t, T*, size_t, const double*, int);                                       \
  template void launch_fill<T>(hipStream_t, T*, size_t, T);                                                         \
  template void launch_coarse<T>(hipStream_t, const double*, const int*, int, const T*, T*);                        \
  template void launch_scaled_copy<T>(hipStream_t, T*, const T*, const T*, size_t, T);                              \
  template void launch_axpy<T>(hipStream_t, T*, const T*, size_t, T);                                              \
  template void launch_vcycle_small<T>(hipStream_t, const SmallLevel<T>*, const SmallCycle<T>&);

HHG_INSTANTIATE(double)
HHG_INSTANTIATE(float)

void timer_set_mask(unsigned mask) {
  Timer& t = timer();
  t.mask = mask;
}

bool timer_enabled() { return timer().mask != 0; }

void timer_read(int family, double* total_ms, int* launches, double* units) {
  Timer& t = timer();
  double ms = 0.0, u = 0.0;
  int n = 0;
  std::vector<TimerRec> keep;
  for (auto& r : t.recs) {
    if (r.fam != family) {
      keep.push_back(r);
      continue;
    }
    float e = 0.0f;
    if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&e, r.a, r.b) == hipSuccess) {
      ms += e;
      u += r.units;
      ++n;
    }
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  t.recs.swap(keep);
  if (total_ms) *total_ms = ms;
  if (launches) *launches = n;
  if (units) *units = u;
}

}  // namespace hhg
