// Refinement with connectivity (Sections 3.1-3.4): one level of the 12-subtet red
// refinement that also emits the refined mesh's edge and face numbering -- the numbering
// NumEdges / FacesUp would compute on the refined mesh -- derived in closed form from the
// coarse mesh's numbering, with no sort.
//
// Symbols of one coarse tet t: corners V0..V3 (0..3), edge midpoints M0..M5 (4..9, local
// edges IJ IK IL JK JL KL), centroid C (10).  Child c (RedRefine's vertex lists) lives at
// row(t, c) = t for c = 0 and nE + 11 t + c - 1 otherwise, so all first children precede
// all others, which are ordered by (t, c).  Positions are 6 row + local edge (edges) and
// 4 row + local face (faces); a refined edge/face is numbered by the rank of its first
// position (edges) or of its owner's slot (faces), as in the paper.
//
// First occurrence of a refined edge:
//  (M_j, C)  inside t only: the first octahedron child holding it (fixed per j);
//  (M_i, M_j) on a coarse face: the corner child of the shared vertex, in t or in the
//            neighbour across that face, whichever position is smaller (within a tet the
//            corner child precedes the octahedron children);
//  (V, M_j)  half of coarse edge e at node v: the corner child of v in every tet around e;
//            first is child 0 of the lowest tet whose local vertex I is v (a per-edge
//            atomicMin over the coarse tets), else the corner child of v in the first tet
//            of e (edge_first_tet, with the local edge and orientation kept per edge).
// Faces have at most two occurrences: inside t (fixed partner child) or across a coarse
// face (corner child or middle-triangle child of the neighbour).  Two passes over the
// coarse tets (per-row masks and counts; then ids and outputs) around two scans.
#include <climits>
#include <utility>

#include "common.hpp"

namespace ph {

// ---------------------------------------------------------------- compile-time tables
// child c, vertex p -> symbol (RedRefine's vertex lists), 4-bit packed
__host__ __device__ constexpr uint64_t chw(int w) {
  return w == 0 ? 0x6893975284716540ull : (w == 1 ? 0xa689a975a847a654ull : 0xa879a864a695a574ull);
}
__host__ __device__ constexpr int ch(int c, int p) { return (int)((chw(c >> 2) >> (4 * (4 * (c & 3) + p))) & 15ull); }
static_assert(ch(0, 0) == 0 && ch(0, 1) == 4 && ch(0, 3) == 6, "child 0 = [I m0 m1 m2]");
static_assert(ch(1, 0) == 1 && ch(1, 1) == 7 && ch(1, 2) == 4 && ch(1, 3) == 8, "child 1 = [J m3 m0 m4]");
static_assert(ch(3, 1) == 9 && ch(3, 3) == 6, "child 3 = [L m5 m4 m2]");
static_assert(ch(7, 0) == 9 && ch(7, 3) == 10 && ch(8, 1) == 7 && ch(11, 0) == 9 && ch(11, 2) == 8, "octahedron");

// position (1..3) of midpoint M_j in corner child v, 0 if absent
__host__ __device__ constexpr int posv(int v, int j) {
  return ch(v, 1) == 4 + j ? 1 : (ch(v, 2) == 4 + j ? 2 : (ch(v, 3) == 4 + j ? 3 : 0));
}
// runtime forms of posv and eidx (one shift of a packed constant instead of a chain of
// compares): posv_r(v, j) for corner child v < 4, eidx_r(i, j) for local vertices i != j
__host__ __device__ constexpr uint64_t posv_pack() {
  uint64_t r = 0;
  for (int v = 0; v < 4; ++v)
    for (int j = 0; j < 6; ++j) r |= (uint64_t)posv(v, j) << (2 * (6 * v + j));
  return r;
}
__device__ __forceinline__ int posv_r(int v, int j) { return (int)((posv_pack() >> (2 * (6 * v + j))) & 3ull); }
__host__ __device__ constexpr uint64_t eidx_pack() {
  uint64_t r = 0;
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) r |= (uint64_t)(i == j ? 15 : eidx(i, j)) << (4 * (4 * i + j));
  return r;
}
__device__ __forceinline__ int eidx_r(int i, int j) { return (int)((eidx_pack() >> (4 * (4 * i + j))) & 15ull); }
static_assert(((posv_pack() >> (2 * (6 * 1 + 3))) & 3) == (uint64_t)posv(1, 3), "posv pack");

// local face of corner child v that lies on coarse face k (15 if none)
__host__ __device__ constexpr int cornerface(int v, int k) {
  return (int)((0x12f1f2021f0f210ull >> (4 * (4 * v + k))) & 15ull);
}
static_assert(cornerface(0, 0) == 0 && cornerface(0, 2) == 2 && cornerface(1, 2) == 1 && cornerface(2, 1) == 2 &&
                  cornerface(3, 3) == 0 && cornerface(0, 3) == 15,
              "corner faces");

__host__ __device__ constexpr int common_v(int i, int j) {
  return (ev0(i) == ev0(j) || ev0(i) == ev1(j)) ? ev0(i) : ev1(i);
}
__host__ __device__ constexpr int other_end(int i, int v) { return ev0(i) == v ? ev1(i) : ev0(i); }
// coarse face holding three distinct local vertices = face opposite the fourth
__host__ __device__ constexpr int face_with(int a, int b, int c) { return opp(6 - a - b - c); }

__host__ __device__ constexpr int esym_lo(int c, int jj) {
  return ch(c, ev0(jj)) < ch(c, ev1(jj)) ? ch(c, ev0(jj)) : ch(c, ev1(jj));
}
__host__ __device__ constexpr int esym_hi(int c, int jj) {
  return ch(c, ev0(jj)) < ch(c, ev1(jj)) ? ch(c, ev1(jj)) : ch(c, ev0(jj));
}
// edge kind: 1 (V, M), 2 (M, M), 3 (M, C)
__host__ __device__ constexpr int ekind(int c, int jj) { return esym_hi(c, jj) == 10 ? 3 : (esym_lo(c, jj) < 4 ? 1 : 2); }

// first octahedron child / local edge holding (M_j, C)
__host__ __device__ constexpr int first3(int j, bool want_edge) {
  for (int c = 4; c < 12; ++c)
    for (int jj = 0; jj < 6; ++jj)
      if (esym_lo(c, jj) == 4 + j && esym_hi(c, jj) == 10) return want_edge ? jj : c;
  return -1;
}

// faces: kind 0 inside t, 1 corner triangle on a coarse face, 2 middle triangle of a coarse face
__host__ __device__ constexpr int fs(int c, int kk, int m) { return ch(c, fv(kk, m)); }
__host__ __device__ constexpr int nverts(int c, int kk) {
  return (fs(c, kk, 0) < 4) + (fs(c, kk, 1) < 4) + (fs(c, kk, 2) < 4);
}
__host__ __device__ constexpr bool has_c(int c, int kk) {
  return fs(c, kk, 0) == 10 || fs(c, kk, 1) == 10 || fs(c, kk, 2) == 10;
}
__host__ __device__ constexpr int vmask_of(int s) {
  return s < 4 ? (1 << s) : (s < 10 ? ((1 << ev0(s - 4)) | (1 << ev1(s - 4))) : 0);
}
__host__ __device__ constexpr int span(int c, int kk) {
  return vmask_of(fs(c, kk, 0)) | vmask_of(fs(c, kk, 1)) | vmask_of(fs(c, kk, 2));
}
__host__ __device__ constexpr int popc4(int m) { return (m & 1) + ((m >> 1) & 1) + ((m >> 2) & 1) + ((m >> 3) & 1); }
__host__ __device__ constexpr int fkind(int c, int kk) {
  return has_c(c, kk) ? 0 : (nverts(c, kk) == 1 ? 1 : (popc4(span(c, kk)) == 3 ? 2 : 0));
}
// coarse face of a kind-1/2 face: the face opposite the vertex it does not span
__host__ __device__ constexpr int fcoarse(int c, int kk) {
  return opp((span(c, kk) & 1) == 0 ? 0 : ((span(c, kk) & 2) == 0 ? 1 : ((span(c, kk) & 4) == 0 ? 2 : 3)));
}
__host__ __device__ constexpr int symset(int c, int kk) {
  return (1 << fs(c, kk, 0)) | (1 << fs(c, kk, 1)) | (1 << fs(c, kk, 2));
}
// partner (child * 4 + local face) of a kind-0 face inside t
__host__ __device__ constexpr int fpartner(int c, int kk) {
  for (int c2 = 0; c2 < 12; ++c2)
    for (int k2 = 0; k2 < 4; ++k2)
      if (c2 != c && symset(c2, k2) == symset(c, kk)) return 4 * c2 + k2;
  return -1;
}
static_assert(fkind(0, 3) == 0 && fpartner(0, 3) == 4 * 4 + 0, "cut triangle at I shared with child 4");
static_assert(fkind(8, 0) == 2 && fcoarse(8, 0) == 0 && fkind(11, 0) == 2 && fcoarse(11, 0) == 3, "middles");
static_assert(fkind(1, 1) == 1 && fcoarse(1, 1) == 2 && fkind(2, 2) == 1 && fcoarse(2, 2) == 1, "corners");
static_assert(first3(0, false) == 4 && first3(3, false) == 5, "first (M, C)");

// Element i of an array addressed as its (wave-uniform) base plus an unsigned 32-bit byte
// offset: the hardware adds the offset to a scalar base, so no 64-bit address arithmetic is
// spent per access.  Stores (every one of them a write-once output) carry the nontemporal
// hint.  Valid while i * sizeof(T) < 2^32 (every array indexed this way holds at most
// 16 nE' bytes < 2^32 by the entry point's size limits; two-dimensional outputs
// take a per-row base).
template <class T>
__device__ __forceinline__ T ldu(const T* p, uint32_t i) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(p) + i * (uint32_t)sizeof(T));
}
template <class T>
__device__ __forceinline__ void stu(T* p, uint32_t i, T v) {
  st_nt(reinterpret_cast<T*>(reinterpret_cast<char*>(p) + i * (uint32_t)sizeof(T)), v);
}

constexpr int RCT = 256;

struct RCArgs {
  int64_t nC, nE, nE2, nEd, nEd2, nF2;
  const int4* T4;  // AoS copies of the coarse tets, faces, neighbours, edges (e0..e3 | e4 e5 - -)
  const int4* F4;
  const int4* N4;
  const int4* E8;
  const int32_t* eft;
  const int32_t* pre;
  const int32_t* minI;  // [2 nEd]: (t << 2 | j) of the lowest tet whose vertex I is that end
  const int32_t* efp;   // [nEd]: (6 t0 + j0) << 1 | (node at ev0(j0) is the larger end)
  // per refined row, written by pass 1: (prefix within its workgroup's row range) << 6 |
  // first-edge mask and << 4 | owned-face mask; the ranges' offsets are in tpre
  uint32_t* recE;
  uint32_t* recF;
  uint32_t* tagg;  // [4][ntiles] per-workgroup totals: edges of the child-0 rows, of the other
  uint32_t* tpre;  // rows, faces of the child-0 rows, of the other rows; tpre = their offsets
  int64_t ntiles;  // (one exclusive scan over all four; a face offset is tpre[.] - tpre[2 ntiles],
                   // the edge total), then the grand total
  int32_t* edges2;
  int32_t* t2e2;
  int32_t* eft2;
  int32_t* pre2;
  int32_t* faces2;
  int32_t* t2f2;
  int8_t* sig2;
  int32_t* f2t2;
  int32_t* nbr2;
  // the level's check, done by pass 2's first workgroup (the flag and the totals are final
  // before pass 2 starts): chk_flag = input ids out of range, chk_etot / chk_all = the edge
  // total and edges + faces; a code is ORed into *status, and chk_out (when not null) gets
  // {edges, faces, flag} for the synchronous check
  const uint32_t* chk_etot;
  const uint32_t* chk_all;
  const uint32_t* chk_flag;
  int32_t* status;
  int64_t* chk_out;
};

__global__ __launch_bounds__(RCT) void k_rc_prep(int64_t nE, int64_t nEd, const int32_t* __restrict__ tet,
                                                 const int32_t* __restrict__ t2e, const int32_t* __restrict__ eft,
                                                 const int32_t* __restrict__ t2f, const int32_t* __restrict__ nbr,
                                                 int32_t* __restrict__ minI, int32_t* __restrict__ efp,
                                                 int4* __restrict__ T4, int4* __restrict__ F4, int4* __restrict__ N4,
                                                 int4* __restrict__ E8, uint32_t* __restrict__ bad) {
  int64_t t = (int64_t)blockIdx.x * RCT + threadIdx.x;
  if (t >= nE) return;
  int n[4], e[6];
#pragma unroll
  for (int i = 0; i < 4; ++i) n[i] = tet[i * nE + t];
  bool oob = false;
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    e[j] = t2e[j * nE + t];
    if ((uint32_t)e[j] >= (uint64_t)nEd) {  // edge ids index the per-edge tables below
      oob = true;
      e[j] = 0;
    }
  }
  if (oob) atomicOr(bad, 1u);
  T4[t] = make_int4(n[0], n[1], n[2], n[3]);
  F4[t] = make_int4(t2f[t], t2f[nE + t], t2f[2 * nE + t], t2f[3 * nE + t]);
  int nb4[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int v = nbr[i * nE + t];
    nb4[i] = (v >= nE) ? -1 : v;  // inputs are trusted; clamps only keep later loads in range
  }
  N4[t] = make_int4(nb4[0], nb4[1], nb4[2], nb4[3]);
  E8[2 * t] = make_int4(e[0], e[1], e[2], e[3]);
  E8[2 * t + 1] = make_int4(e[4], e[5], 0, 0);
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    const int a = n[ev0(j)], b = n[ev1(j)];
    const int lo = a < b ? a : b;
    if (eft[e[j]] == t) efp[e[j]] = (int32_t)(((6 * t + j) << 1) | (a != lo ? 1 : 0));
    if (j < 3) atomicMin(&minI[2 * e[j] + (n[0] == lo ? 0 : 1)], (int32_t)((t << 2) | j));
  }
}

// Row arithmetic is 32-bit: the entry point guarantees 6 nE' < 2^31, so rows, 6 row + j and
// 4 row + k all fit in int32.
__device__ __forceinline__ int rowof(int nE, int tt, int c) { return c == 0 ? tt : nE + 11 * tt + (c - 1); }
template <int C>
__device__ __forceinline__ int rowc(int nE, int tt) { return C == 0 ? tt : nE + 11 * tt + (C - 1); }
// order of the rows of one tet's children: child 0 first, then 1..11
__host__ __device__ constexpr int rord(int c) { return c == 0 ? -1 : c; }

// Both passes run one workgroup per RCW coarse tets: wave c handles child c of all of them,
// so the child index is uniform across a wave and every rule above resolves at compile time
// (one specialised code path per child, selected by a scalar branch).  A workgroup's rows
// are rows [t0, t0 + RCW) and [nE + 11 t0, nE + 11 (t0 + RCW)): per-row outputs are staged
// in LDS and written out as two contiguous ranges.  The lookups below are branch-free
// (clamped indices, selects), so a lane issues all loads of one stage back to back instead
// of waiting for each in turn.
constexpr int RCW = 64;
constexpr int RCB = 12 * RCW;
constexpr int RCS = 13;  // LDS stride of one tet's 12 child slots (odd: no bank conflicts)

template <class F, int... I>
__device__ __forceinline__ void sfor_(F& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void sfor(F&& f) {
  sfor_(f, std::make_integer_sequence<int, N>{});
}

// Values of a coarse tet that several of its 12 child rows look up, gathered once per
// workgroup into LDS (item q of the workgroup's tet l at sh[q RCW + l]) rather than by each of
// the 12 waves:
//  QM + k       coarse face k: bits 2i, 2i+1 = position of local vertex i in the tet across
//               face k (the tet itself on the boundary), bits 8, 9 = position of face k there
//  QMI + 2j + s minI[2 e_j + s]
//  QEF + j      efp[e_j]
//  QFT + j      eft[e_j]       (pass 2 only)
//  QPR          pre[t]         (pass 2 only)
constexpr int QM = 0, QMI = 4, QEF = 16, QFT = 22, QPR = 28;
constexpr int NQ1 = 22, NQ2 = 29;  // items of pass 1 and pass 2

// coarse tet data of one lane
struct CT {
  int t;
  int n[4], f[4], nb[4], e[6];
  const int* sh;  // this tet's column of the shared items
  __device__ __forceinline__ int item(int q) const { return sh[q * RCW]; }
};
__device__ __forceinline__ void load_ct(const RCArgs& A, int t, const int* sh, CT& T) {
  const uint32_t u = (uint32_t)t;
  const int4 a = ldu(A.T4, u), b = ldu(A.F4, u), c = ldu(A.N4, u), d = ldu(A.E8, 2 * u), e = ldu(A.E8, 2 * u + 1);
  T.t = t;
  T.sh = sh;
  T.n[0] = a.x, T.n[1] = a.y, T.n[2] = a.z, T.n[3] = a.w;
  T.f[0] = b.x, T.f[1] = b.y, T.f[2] = b.z, T.f[3] = b.w;
  T.nb[0] = c.x, T.nb[1] = c.y, T.nb[2] = c.z, T.nb[3] = c.w;
  T.e[0] = d.x, T.e[1] = d.y, T.e[2] = d.z, T.e[3] = d.w, T.e[4] = e.x, T.e[5] = e.y;
}
// the neighbour across coarse face k, or the tet itself (a valid address) on the boundary
__device__ __forceinline__ int nb_or_self(const CT& T, int k) { return T.nb[k] >= 0 ? T.nb[k] : T.t; }
__device__ __forceinline__ int loc4v(const int4& v, int x) { return v.x == x ? 0 : (v.y == x ? 1 : (v.z == x ? 2 : 3)); }

// the first NQ shared items of the workgroup's tets: wave w fills items w, w + 12, ...
template <int NQ>
__device__ __forceinline__ void gather_items(const RCArgs& A, int t0, int nb, int* sh) {
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  if (lane >= nb) return;
  const uint32_t t = (uint32_t)(t0 + lane);
  const int32_t* E = reinterpret_cast<const int32_t*>(A.E8);  // e_j at 8 t + j
#pragma unroll
  for (int i = 0; i < (NQ + RCB / 64 - 1) / (RCB / 64); ++i) {
    const int q = w + i * (RCB / 64);
    if (q >= NQ) break;
    int v;
    if (q < QMI) {
      const int k = q;
      const int nk = ldu(reinterpret_cast<const int32_t*>(A.N4), 4 * t + k);
      const uint32_t tn = nk >= 0 ? (uint32_t)nk : t;
      const int4 own = ldu(A.T4, t), nn = ldu(A.T4, tn), nf = ldu(A.F4, tn);
      const int fk = ldu(reinterpret_cast<const int32_t*>(A.F4), 4 * t + k);
      v = loc4v(nn, own.x) | (loc4v(nn, own.y) << 2) | (loc4v(nn, own.z) << 4) | (loc4v(nn, own.w) << 6) |
          (loc4v(nf, fk) << 8);
    } else if (q < QEF) {
      const int j = (q - QMI) >> 1, s = (q - QMI) & 1;
      v = ldu(A.minI, (uint32_t)(2 * ldu(E, 8 * t + j) + s));
    } else if (q < QFT) {
      v = ldu(A.efp, (uint32_t)ldu(E, 8 * t + (q - QEF)));
    } else if (q < QPR) {
      v = ldu(A.eft, (uint32_t)ldu(E, 8 * t + (q - QFT)));
    } else {
      v = ldu(A.pre, t);
    }
    sh[q * RCW + lane] = v;
  }
}

// first occurrence (row, local edge) of local edge J of child C
template <int C, int J>
__device__ __forceinline__ void efirst(const RCArgs& A, const CT& T, int& er, int& ej) {
  constexpr int s0 = ch(C, ev0(J)), s1 = ch(C, ev1(J));
  constexpr int lo = s0 < s1 ? s0 : s1, hi = s0 < s1 ? s1 : s0;
  const int nE = (int)A.nE;
  if constexpr (hi == 10) {  // (M_j, C): inside t
    er = rowc<first3(lo - 4, false)>(nE, T.t);
    ej = first3(lo - 4, true);
  } else if constexpr (lo < 4) {  // (V_lo, M_j): half of coarse edge e_j at node v
    constexpr int j = hi - 4;
    const int v = T.n[lo];
    const int na = T.n[ev0(j)], nb = T.n[ev1(j)];
    const bool vlo = v == (na < nb ? na : nb);
    const int mi = T.sh[(QMI + 2 * j + (vlo ? 0 : 1)) * RCW];  // minI of that end of e_j
    const int p0 = T.item(QEF + j);
    // child 0 of the lowest tet whose vertex I is v (local edge j of (I, m_j)), else the
    // corner child of v in the first tet of e
    const int flip = p0 & 1, p = p0 >> 1;
    const int t0 = p / 6, j0 = p - 6 * t0;
    const int vl = (vlo != (flip != 0)) ? ev0(j0) : ev1(j0);
    const bool ok = p0 >= 0 && t0 < nE;  // unset only for inconsistent input
    const bool use_mi = mi != INT_MAX && (mi >> 2) < nE;
    er = use_mi ? (mi >> 2) : (ok ? rowof(nE, t0, vl) : rowc<C>(nE, T.t));
    ej = use_mi ? (mi & 3) : (ok ? posv_r(vl, j0) - 1 : J);
  } else {  // (M_i, M_j) on a coarse face: corner child of the shared vertex, here or in the neighbour
    constexpr int i = lo - 4, j = hi - 4;
    constexpr int v = common_v(i, j), a = other_end(i, v), b = other_end(j, v);
    constexpr int k = face_with(v, a, b);
    constexpr int jr = eidx(posv(v, i), posv(v, j));
    const int rr = rowc<v>(nE, T.t);
    const int mp = T.item(QM + k);  // positions of V_v, V_a, V_b in the tet across face k
    const int v2 = (mp >> (2 * v)) & 3, a2 = (mp >> (2 * a)) & 3, b2 = (mp >> (2 * b)) & 3;
    const int le2 = eidx_r(posv_r(v2, eidx_r(v2, a2)), posv_r(v2, eidx_r(v2, b2)));
    const int r2 = rowof(nE, nb_or_self(T, k), v2);
    const bool there = T.nb[k] >= 0 && 6 * r2 + le2 < 6 * rr + jr;
    er = there ? r2 : rr;
    ej = there ? le2 : jr;
  }
}

// is local edge J of child C first seen in this row?
template <int C, int J>
__device__ __forceinline__ bool efirst_here(const RCArgs& A, const CT& T) {
  constexpr int s0 = ch(C, ev0(J)), s1 = ch(C, ev1(J));
  constexpr int lo = s0 < s1 ? s0 : s1, hi = s0 < s1 ? s1 : s0;
  if constexpr (hi == 10) {
    return first3(lo - 4, false) == C && first3(lo - 4, true) == J;
  } else if constexpr (lo >= 4 && common_v(lo - 4, hi - 4) != C) {
    return false;  // an octahedron child never holds the first (M, M) occurrence
  } else {
    int er, ej;
    efirst<C, J>(A, T, er, ej);
    return er == rowc<C>((int)A.nE, T.t) && ej == J;
  }
}

// other occurrence (row, local face) of local face K of child C; row -1 on the boundary
template <int C, int K>
__device__ __forceinline__ void fother(const RCArgs& A, const CT& T, int& fr, int& fk) {
  constexpr int kind = fkind(C, K);
  const int nE = (int)A.nE;
  if constexpr (kind == 0) {
    constexpr int p = fpartner(C, K);
    fr = rowc<(p >> 2)>(nE, T.t);
    fk = p & 3;
  } else {
    constexpr int k = fcoarse(C, K);
    const int tn = nb_or_self(T, k);
    const int mp = T.item(QM + k);
    const int k2 = (mp >> 8) & 3;
    if constexpr (kind == 2) {
      fr = rowof(nE, tn, 8 + k2);
      fk = 0;
    } else {
      const int v2 = (mp >> (2 * C)) & 3;  // corner child C holds vertex V_C
      fr = rowof(nE, tn, v2);
      fk = cornerface(v2, k2);
    }
    if (T.nb[k] < 0) fr = -1, fk = 0;
  }
}

template <int C, int K>
__device__ __forceinline__ bool fown(const RCArgs& A, const CT& T, int r, int& fr, int& fk) {
  fother<C, K>(A, T, fr, fk);
  if constexpr (fkind(C, K) == 0)
    return rord(fpartner(C, K) >> 2) > rord(C);
  else
    return fr < 0 || 4 * fr + fk > 4 * r + K;
}

template <int S>
__device__ __forceinline__ int sym_node(const RCArgs& A, const CT& T) {
  if constexpr (S < 4) {
    return T.n[S];
  } else if constexpr (S < 10) {
    const int e = T.e[S - 4];
    return (int)A.nC + T.item(QFT + S - 4) + e + 1;
  } else {
    return (int)A.nC + T.t + T.item(QPR);
  }
}

// the rows of a workgroup: LDS slot l * RCS + c of (lane l, child c) <-> global row
struct RCBlock {
  int t0;
  int nb;  // tets in this workgroup
};
__device__ __forceinline__ RCBlock rc_block(const RCArgs& A) {
  RCBlock B;
  B.t0 = (int)blockIdx.x * RCW;
  const int rest = (int)A.nE - B.t0;
  B.nb = rest < RCW ? rest : RCW;
  return B;
}
// flush slot of thread i: row and LDS slot, or false
__device__ __forceinline__ bool rc_flush_slot(const RCArgs& A, const RCBlock& B, int i, int& row, int& slot) {
  if (i < 11 * B.nb) {  // children 1..11, rows nE + 11 t0 + i
    const int l = i / 11;
    row = (int)A.nE + 11 * B.t0 + i;
    slot = l * RCS + 1 + (i - 11 * l);
    return true;
  }
  if (i >= 11 * RCW && i - 11 * RCW < B.nb) {  // child 0, rows t0 + l
    const int l = i - 11 * RCW;
    row = B.t0 + l;
    slot = l * RCS;
    return true;
  }
  return false;
}

// pass 1: the first-edge and owned-face masks of every refined row with their prefix counts
// inside the workgroup's two row ranges, and the ranges' totals
__global__ __launch_bounds__(RCB) void k_rc_pass1(RCArgs A) {
  __shared__ uint32_t sE[RCW * RCS], sF[RCW * RCS];
  __shared__ uint32_t lw[RCB / 64];
  __shared__ int sh[NQ1 * RCW];
  const RCBlock B = rc_block(A);
  const int lane = threadIdx.x & 63;
  const int c = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  CT T;  // loaded before the shared items so that both gathers are in flight together
  if (lane < B.nb) load_ct(A, B.t0 + lane, sh + lane, T);
  gather_items<NQ1>(A, B.t0, B.nb, sh);
  __syncthreads();
  if (lane < B.nb) {
    sfor<12>([&](auto Cc) {
      constexpr int C = decltype(Cc)::value;
      if (c != C) return;
      const int r = rowc<C>((int)A.nE, T.t);
      int me = 0, mf = 0;
      sfor<6>([&](auto Jc) {
        constexpr int J = decltype(Jc)::value;
        if (efirst_here<C, J>(A, T)) me |= 1 << J;
      });
      sfor<4>([&](auto Kc) {
        constexpr int K = decltype(Kc)::value;
        int fr, fk;
        if (fown<C, K>(A, T, r, fr, fk)) mf |= 1 << K;
      });
      sE[lane * RCS + C] = (uint32_t)me;
      sF[lane * RCS + C] = (uint32_t)mf;
    });
  }
  __syncthreads();
  // rows in flush order: threads 0 .. 11 RCW - 1 the other rows, the last RCW the child-0 rows
  int row, slot;
  const bool has = rc_flush_slot(A, B, threadIdx.x, row, slot);
  const uint32_t me = has ? sE[slot] : 0u, mf = has ? sF[slot] : 0u;
  const bool first = threadIdx.x >= 11 * RCW;
  const uint32_t pk = (uint32_t)__popc(me) | ((uint32_t)__popc(mf) << 16);  // < 2^16 each per block
  uint32_t agg1, agg2;
  const uint32_t p2 = block_excl_scan<RCB / 64>(first ? 0u : pk, lw, agg2);
  const uint32_t p1 = block_excl_scan<RCB / 64>(first ? pk : 0u, lw, agg1);
  if (has) {
    const uint32_t p = first ? p1 : p2;
    stu(A.recE, (uint32_t)row, ((p & 0xffffu) << 6) | me);
    stu(A.recF, (uint32_t)row, ((p >> 16) << 4) | mf);
  }
  if (threadIdx.x == 0) {
    const int64_t b = blockIdx.x, n = A.ntiles;
    A.tagg[b] = agg1 & 0xffffu;
    A.tagg[n + b] = agg2 & 0xffffu;
    A.tagg[2 * n + b] = agg1 >> 16;
    A.tagg[3 * n + b] = agg2 >> 16;
  }
}

// absolute prefix of a row's record: its workgroup range's offset + the in-range prefix
__device__ __forceinline__ int row_tile(int nE, int row) {
  return (row < nE ? row : (int)((uint32_t)(row - nE) / 11u)) / RCW;
}
__device__ __forceinline__ uint32_t pre_e(const RCArgs& A, int row, uint32_t rec) {
  const int nE = (int)A.nE;
  return ldu(A.tpre, (uint32_t)((row < nE ? 0 : 1) * (int)A.ntiles + row_tile(nE, row))) + (rec >> 6);
}
__device__ __forceinline__ uint32_t pre_f(const RCArgs& A, int row, uint32_t rec) {
  const int nE = (int)A.nE, n = (int)A.ntiles;
  return ldu(A.tpre, (uint32_t)((row < nE ? 2 : 3) * n + row_tile(nE, row))) - ldu(A.tpre, (uint32_t)(2 * n)) +
         (rec >> 4);
}

// pass 2: ids of the refined edges and faces of every row, and all outputs.  Phase 1 stages
// the per-row outputs in LDS and writes them as two contiguous row ranges; phase 2 reuses
// the LDS for the records of the edges and faces first seen in the workgroup's rows, whose
// ids form one contiguous range per row range, and writes those out contiguously too.
constexpr int RCO = 20;  // staged words per row: pre, 6 edges, 4 faces, 4 neighbours, 4 packed signs,
                         // and (not written out) the node ids of the row's 4 vertices
constexpr int RCL = RCO * RCW * RCS;  // LDS words
// phase-2 capacities (entities per row range): child-0 rows exactly (<= 6 edges, 4 faces
// each), the other rows about 1.2 edges and 2 faces per row; overflow goes out directly
constexpr int CE1 = 6 * RCW, CF1 = 4 * RCW, CE2 = 1024;
constexpr int CF2 = (RCL - 3 * CE1 - 5 * CF1 - 3 * CE2) / 5;
static_assert(CF2 >= 2 * 11 * RCW + 64, "room for the typical face count of a workgroup");
constexpr int OE1 = 0, OF1 = OE1 + 3 * CE1, OE2 = OF1 + 5 * CF1, OF2 = OE2 + 3 * CE2;  // SoA blocks

struct RCRange {  // one row range's first-seen edges and faces: [e0, e0 + ne), [f0, f0 + nf)
  int e0, f0;      // < nEd' < 2^26, < nF' < 2^28
  int ne, nf;
};

// input ids out of range (flag) and refined totals against the recurrences (one thread)
__device__ __forceinline__ void rc_check_level(const RCArgs& A) {
  const int64_t ne = *A.chk_etot, nf = (int64_t)*A.chk_all - ne;
  const uint32_t flag = *A.chk_flag;
  int32_t code = 0;
  if (flag) code |= 1;
  if (ne != A.nEd2 || nf != A.nF2) code |= 2;
  if (code && A.status) atomicOr(A.status, code);
  if (A.chk_out) {
    A.chk_out[0] = ne;
    A.chk_out[1] = nf;
    A.chk_out[2] = flag;
  }
}

__global__ __launch_bounds__(RCB) __attribute__((amdgpu_waves_per_eu(6))) void k_rc_pass2(RCArgs A) {
  if (blockIdx.x == 0 && threadIdx.x == 0) rc_check_level(A);
  __shared__ int32_t sW[RCL];
  __shared__ RCRange sR[2];
  __shared__ int sh[NQ2 * RCW];
  const RCBlock B = rc_block(A);
  const int lane = threadIdx.x & 63;
  const int c = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int nE = (int)A.nE;
  const int64_t nEd2 = A.nEd2, nF2 = A.nF2;
  if (threadIdx.x < 2) {  // ranges from the prefix records (exact for consistent input)
    const bool r2 = threadIdx.x == 1;
    const int lo = r2 ? nE + 11 * B.t0 : B.t0;
    const int hi = r2 ? nE + 11 * (B.t0 + B.nb) : B.t0 + B.nb;  // row after the range
    const bool last = r2 && hi == A.nE2;
    const int64_t e0 = pre_e(A, lo, ldu(A.recE, (uint32_t)lo)), f0 = pre_f(A, lo, ldu(A.recF, (uint32_t)lo));
    const int64_t e1 = last ? nEd2 : (int64_t)pre_e(A, hi, ldu(A.recE, (uint32_t)hi));
    const int64_t f1 = last ? nF2 : (int64_t)pre_f(A, hi, ldu(A.recF, (uint32_t)hi));
    RCRange R;
    R.e0 = (int)e0;
    R.f0 = (int)f0;
    R.ne = (int)(e1 > e0 ? e1 - e0 : 0);
    R.nf = (int)(f1 > f0 ? f1 - f0 : 0);
    sR[threadIdx.x] = R;
  }
  // kept in registers from phase 1 to phase 2: this row's masks and the f2t slot across each
  // owned face (its edge and face ids and vertex node ids are read back from LDS)
  int me = 0, mf = 0, r = 0;
  int fnb[4];
  CT T;
  if (lane < B.nb) load_ct(A, B.t0 + lane, sh + lane, T);
  gather_items<NQ2>(A, B.t0, B.nb, sh);
  __syncthreads();
  if (lane < B.nb) {
    sfor<12>([&](auto Cc) {
      constexpr int C = decltype(Cc)::value;
      if (c != C) return;
      r = rowc<C>(nE, T.t);
      // stage 1: this row's records, every first occurrence / other side, the vertex ids
      const uint32_t oe = ldu(A.recE, (uint32_t)r), of = ldu(A.recF, (uint32_t)r);
      int er[6], ej[6], fr[4], fk[4];
      sfor<6>([&](auto Jc) {
        constexpr int J = decltype(Jc)::value;
        efirst<C, J>(A, T, er[J], ej[J]);
      });
      sfor<4>([&](auto Kc) {
        constexpr int K = decltype(Kc)::value;
        fother<C, K>(A, T, fr[K], fk[K]);
      });
      int32_t* w = sW + lane * RCS + C;
      sfor<4>([&](auto Pc) {
        constexpr int Q = decltype(Pc)::value;
        w[(16 + Q) * RCW * RCS] = sym_node<ch(C, Q)>(A, T);
      });
      // stage 2: the records of those rows (a first-seen edge's row is this row)
      uint32_t oE[6], oF[4];
      sfor<6>([&](auto Jc) {
        constexpr int J = decltype(Jc)::value;
        oE[J] = ldu(A.recE, (uint32_t)(er[J]));
      });
      sfor<4>([&](auto Kc) {
        constexpr int K = decltype(Kc)::value;
        oF[K] = ldu(A.recF, (uint32_t)(fr[K] >= 0 ? fr[K] : r));
      });
      // stage 3: ids = workgroup offset + in-workgroup prefix + rank inside the row
      me = (int)(oe & 63);
      mf = (int)(of & 15);
      const uint32_t pf = pre_f(A, r, of);
      w[0] = (int32_t)pre_e(A, r, oe);
      sfor<6>([&](auto Jc) {
        constexpr int J = decltype(Jc)::value;
        w[(1 + J) * RCW * RCS] = (int)(pre_e(A, er[J], oE[J]) + __popc((oE[J] & 63) & ((1u << ej[J]) - 1)));
      });
      uint32_t sg = 0;
      sfor<4>([&](auto Kc) {
        constexpr int K = decltype(Kc)::value;
        const bool own = (mf >> K) & 1;
        const int idn = (int)(pre_f(A, fr[K], oF[K]) + __popc((oF[K] & 15) & ((1u << fk[K]) - 1)));
        fnb[K] = fr[K] < 0 ? -1 : 4 * fr[K] + fk[K];
        w[(7 + K) * RCW * RCS] = own ? (int)(pf + __popc(mf & ((1 << K) - 1))) : (fr[K] >= 0 ? idn : -1);  // -1: bad input
        w[(11 + K) * RCW * RCS] = fr[K] < 0 ? -1 : fr[K];
        sg |= (own ? 0x01u : 0xffu) << (8 * K);
      });
      w[15 * RCW * RCS] = (int32_t)sg;
    });
  }
  __syncthreads();
  int row, slot;
  if (rc_flush_slot(A, B, threadIdx.x, row, slot)) {
    const int64_t n2 = A.nE2;
    const int32_t* v = sW + slot;
    const uint32_t u = (uint32_t)row;
    stu(A.pre2, u, v[0]);
#pragma unroll
    for (int j = 0; j < 6; ++j) stu(A.t2e2 + j * n2, u, v[(1 + j) * RCW * RCS]);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      stu(A.t2f2 + k * n2, u, v[(7 + k) * RCW * RCS]);
      stu(A.nbr2 + k * n2, u, v[(11 + k) * RCW * RCS]);
      stu(A.sig2 + k * n2, u, (int8_t)(((uint32_t)v[15 * RCW * RCS] >> (8 * k)) & 0xffu));
    }
  }
  int eid[6], fid[4], nd[4];
  if (lane < B.nb) {
    const int32_t* w = sW + lane * RCS + c;
#pragma unroll
    for (int j = 0; j < 6; ++j) eid[j] = w[(1 + j) * RCW * RCS];
#pragma unroll
    for (int k = 0; k < 4; ++k) fid[k] = w[(7 + k) * RCW * RCS];
#pragma unroll
    for (int q = 0; q < 4; ++q) nd[q] = w[(16 + q) * RCW * RCS];
  }
  __syncthreads();
  // phase 2: records of the edges and faces first seen in these rows
  if (lane < B.nb) {
    sfor<12>([&](auto Cc) {
      constexpr int C = decltype(Cc)::value;
      if (c != C) return;
      const RCRange R = sR[C == 0 ? 0 : 1];
      constexpr int oe_ = C == 0 ? OE1 : OE2, ce = C == 0 ? CE1 : CE2;
      constexpr int of_ = C == 0 ? OF1 : OF2, cf = C == 0 ? CF1 : CF2;
      sfor<6>([&](auto Jc) {
        constexpr int J = decltype(Jc)::value;
        if (!((me >> J) & 1)) return;
        const int id = eid[J];
        const int na = nd[ev0(J)], nb = nd[ev1(J)];
        const int lo = na < nb ? na : nb, hi = na < nb ? nb : na;
        const int li = id - R.e0;
        if (li >= 0 && li < ce && li < R.ne) {
          sW[oe_ + li] = lo;
          sW[oe_ + ce + li] = hi;
          sW[oe_ + 2 * ce + li] = r;
        } else if (id >= 0 && id < nEd2) {
          stu(A.edges2, (uint32_t)id, lo);
          stu(A.edges2 + nEd2, (uint32_t)id, hi);
          stu(A.eft2, (uint32_t)id, r);
        }
      });
      sfor<4>([&](auto Kc) {
        constexpr int K = decltype(Kc)::value;
        if (!((mf >> K) & 1)) return;
        const int id = fid[K];
        const int n0 = nd[fv(K, 0)], n1 = nd[fv(K, 1)], n2 = nd[fv(K, 2)];
        const int li = id - R.f0;
        if (li >= 0 && li < cf && li < R.nf) {
          sW[of_ + li] = 4 * r + K;
          sW[of_ + cf + li] = fnb[K];
          sW[of_ + 2 * cf + li] = n0;
          sW[of_ + 3 * cf + li] = n1;
          sW[of_ + 4 * cf + li] = n2;
        } else if (id >= 0 && id < nF2) {
          stu(A.f2t2, (uint32_t)id, 4 * r + K);
          stu(A.f2t2 + nF2, (uint32_t)id, fnb[K]);
          stu(A.faces2, (uint32_t)id, n0);
          stu(A.faces2 + nF2, (uint32_t)id, n1);
          stu(A.faces2 + 2 * nF2, (uint32_t)id, n2);
        }
      });
    });
  }
  __syncthreads();
#pragma unroll
  for (int g = 0; g < 2; ++g) {
    const RCRange R = sR[g];
    const int oe_ = g == 0 ? OE1 : OE2, ce = g == 0 ? CE1 : CE2;
    const int of_ = g == 0 ? OF1 : OF2, cf = g == 0 ? CF1 : CF2;
    int ne = R.ne < ce ? R.ne : ce, nf = R.nf < cf ? R.nf : cf;
    if (R.e0 + ne > nEd2) ne = R.e0 < nEd2 ? (int)(nEd2 - R.e0) : 0;  // inconsistent input only
    if (R.f0 + nf > nF2) nf = R.f0 < nF2 ? (int)(nF2 - R.f0) : 0;
    int32_t *ed0 = A.edges2 + R.e0, *ed1 = A.edges2 + nEd2 + R.e0, *ef = A.eft2 + R.e0;
    for (int i = threadIdx.x; i < ne; i += RCB) {
      stu(ed0, (uint32_t)i, sW[oe_ + i]);
      stu(ed1, (uint32_t)i, sW[oe_ + ce + i]);
      stu(ef, (uint32_t)i, sW[oe_ + 2 * ce + i]);
    }
    int32_t *ft0 = A.f2t2 + R.f0, *ft1 = A.f2t2 + nF2 + R.f0, *fa0 = A.faces2 + R.f0, *fa1 = A.faces2 + nF2 + R.f0,
            *fa2 = A.faces2 + 2 * nF2 + R.f0;
    for (int i = threadIdx.x; i < nf; i += RCB) {
      stu(ft0, (uint32_t)i, sW[of_ + i]);
      stu(ft1, (uint32_t)i, sW[of_ + cf + i]);
      stu(fa0, (uint32_t)i, sW[of_ + 2 * cf + i]);
      stu(fa1, (uint32_t)i, sW[of_ + 3 * cf + i]);
      stu(fa2, (uint32_t)i, sW[of_ + 4 * cf + i]);
    }
  }
}

// every per-call buffer that must start from a known value, in one launch: minI = INT_MAX
// [2 nEd], efp = -1 [nEd], the input-check flag and both scans' status words = 0 [nz]
__global__ __launch_bounds__(RCT) void k_rc_init(int64_t nEd, int32_t* __restrict__ minI, int32_t* __restrict__ efp,
                                                 int64_t nz, uint32_t* __restrict__ z) {
  const int64_t stride = (int64_t)gridDim.x * RCT;
  for (int64_t i = (int64_t)blockIdx.x * RCT + threadIdx.x; i < 2 * nEd; i += stride) {
    minI[i] = INT_MAX;
    if (i < nEd) efp[i] = -1;
  }
  for (int64_t i = (int64_t)blockIdx.x * RCT + threadIdx.x; i < nz; i += stride) z[i] = 0;
}


struct RCWS {
  int32_t *minI, *efp;
  int4 *T4, *F4, *N4, *E8;
  uint32_t *recE, *recF;
  uint32_t* z;  // zeroed by the init kernel: 4 words (input flag z[2]), the scans' status
  uint64_t* st;
  uint32_t *tagg, *tpre;
  int64_t ntiles, nz;
  int64_t* chk;  // {edges, faces, flag} read back by the synchronous check
  size_t sub;
};

static void rc_layout(Arena& a, int64_t nE, int64_t nEd, RCWS& w) {
  const int64_t n2 = 12 * nE;
  w.minI = a.take<int32_t>(2 * nEd);
  w.efp = a.take<int32_t>(nEd);
  w.T4 = a.take<int4>(nE);
  w.F4 = a.take<int4>(nE);
  w.N4 = a.take<int4>(nE);
  w.E8 = a.take<int4>(2 * nE);
  w.recE = a.take<uint32_t>(n2);
  w.recF = a.take<uint32_t>(n2);
  w.ntiles = (nE + RCW - 1) / RCW;
  const int64_t sw = scan_status_words(4 * w.ntiles);
  w.z = a.take<uint32_t>(4 + 2 * sw);
  w.st = w.z ? reinterpret_cast<uint64_t*>(w.z + 4) : nullptr;  // (a size query lays out from null)
  w.nz = 4 + 2 * sw;
  w.tagg = a.take<uint32_t>(4 * w.ntiles);
  w.tpre = a.take<uint32_t>(4 * w.ntiles + 2);
  w.chk = a.take<int64_t>(4);
  w.sub = a.size();
}

int launch_refine(int64_t nC, const double* coord, int64_t nE, const int32_t* tetra, const int32_t* t2e,
                  const int32_t* eft, const int32_t* pre, int64_t nCo, double* coord_out, int32_t* tetra_out,
                  hipStream_t s, uint32_t* bad);

}  // namespace ph

using namespace ph;

extern "C" size_t phfem_refine_connected_workspace(int64_t nE, int64_t nEd) {
  if (nE <= 0 || nEd <= 0) return 0;
  Arena a;
  RCWS w;
  rc_layout(a, nE, nEd, w);
  return w.sub;
}

extern "C" int phfem_refine_connected(int64_t nC, const double* coord, int64_t nE, const int32_t* tetra, int64_t nEd,
                                      int64_t nF, const int32_t* tet2edge, const int32_t* edge_first_tet,
                                      const int32_t* tet_edge_prefix, const int32_t* tet2face, const int32_t* nbr,
                                      void* work, size_t work_bytes, double* coord_out, int32_t* tetra_out,
                                      int32_t* edges_out, int32_t* tet2edge_out, int32_t* edge_first_tet_out,
                                      int32_t* tet_edge_prefix_out, int32_t* faces_out, int32_t* tet2face_out,
                                      int8_t* sigma_out, int32_t* face2tet_out, int32_t* nbr_out, int64_t* counts,
                                      int32_t* status, phfem_stream_t stream_) {
  clear_error();
  hipStream_t s = (hipStream_t)stream_;
  if (nC <= 0 || nE <= 0 || nEd <= 0 || nF <= 0) return err(PHFEM_EINVAL, "bad sizes");
  const int64_t nE2 = 12 * nE, nC2 = nC + nEd + nE;
  const int64_t nEd2 = 2 * nEd + 3 * nF + 6 * nE, nF2 = 4 * nF + 16 * nE;
  // int32 positions; the per-row records pack the edge prefix in 26 bits, the face prefix in 28
  if (nEd2 >= (int64_t(1) << 26) || nF2 >= (int64_t(1) << 28) || 6 * nE2 >= (int64_t(1) << 31) ||
      nC2 >= (int64_t(1) << 31))
    return err(PHFEM_EINVAL, "refined mesh exceeds the index ranges (nEd' < 2^26, nF' < 2^28, 6 nE' < 2^31)");
  if (!coord || !tetra || !tet2edge || !edge_first_tet || !tet_edge_prefix || !tet2face || !nbr || !coord_out ||
      !tetra_out || !edges_out || !tet2edge_out || !edge_first_tet_out || !tet_edge_prefix_out || !faces_out ||
      !tet2face_out || !sigma_out || !face2tet_out || !nbr_out || !counts)
    return err(PHFEM_EINVAL, "null argument");
  if (!work || work_bytes < phfem_refine_connected_workspace(nE, nEd))
    return err(PHFEM_EWORKSPACE, "refine_connected workspace too small");
  Arena a(work, work_bytes);
  RCWS w;
  rc_layout(a, nE, nEd, w);
  PH_LAUNCH_B("rc_init", 12.0 * nEd + 4.0 * w.nz, k_rc_init,
              (unsigned)std::min<int64_t>(grid_for(std::max<int64_t>(2 * nEd, w.nz), RCT), 4096), RCT, 0, s, nEd,
              w.minI, w.efp, w.nz, w.z);
  int rc = launch_refine(nC, coord, nE, tetra, tet2edge, edge_first_tet, tet_edge_prefix, nC2, coord_out, tetra_out,
                         s, w.z + 2);
  if (rc) return rc;
  PH_LAUNCH_B("rc_prep", 60.0 * nE + 12.0 * nEd + 80.0 * nE, k_rc_prep, grid_for(nE, RCT), RCT, 0, s, nE, nEd, tetra,
              tet2edge, edge_first_tet, tet2face, nbr, w.minI, w.efp, w.T4, w.F4, w.N4, w.E8, w.z + 2);
  RCArgs A;
  A.nC = nC;
  A.nE = nE;
  A.nE2 = nE2;
  A.nEd = nEd;
  A.nEd2 = nEd2;
  A.nF2 = nF2;
  A.T4 = w.T4;
  A.F4 = w.F4;
  A.N4 = w.N4;
  A.E8 = w.E8;
  A.eft = edge_first_tet;
  A.pre = tet_edge_prefix;
  A.minI = w.minI;
  A.efp = w.efp;
  A.recE = w.recE;
  A.recF = w.recF;
  A.tagg = w.tagg;
  A.tpre = w.tpre;
  A.ntiles = w.ntiles;
  A.edges2 = edges_out;
  A.t2e2 = tet2edge_out;
  A.eft2 = edge_first_tet_out;
  A.pre2 = tet_edge_prefix_out;
  A.faces2 = faces_out;
  A.t2f2 = tet2face_out;
  A.sig2 = sigma_out;
  A.f2t2 = face2tet_out;
  A.nbr2 = nbr_out;
  A.chk_etot = w.tpre + 2 * w.ntiles;
  A.chk_all = w.tpre + 4 * w.ntiles;
  A.chk_flag = w.z + 2;
  A.status = status;
  A.chk_out = status ? nullptr : w.chk;
  // pass 1 reads the coarse AoS data once (cache-shared by the 12 rows of a tet) and writes
  // one record word per refined row and count
  PH_LAUNCH_B("refconn_pass1", 80.0 * nE + 12.0 * nEd + 8.0 * nE2, k_rc_pass1, (unsigned)w.ntiles, RCB, 0, s, A);
  // offsets of the workgroups' row ranges: other rows after all child-0 rows
  rc = scan_exclusive(w.tagg, w.tpre, 4 * w.ntiles, w.tpre + 4 * w.ntiles, a, s, w.st);
  if (rc) return rc;
  // pass 2 writes every refined connectivity array once
  PH_LAUNCH_B("refconn_pass2", 80.0 * nE + 12.0 * nEd + 8.0 * nE2 + (24.0 + 4 + 16 + 1 * 4 + 16) * nE2 + 12.0 * nEd2 +
                                   20.0 * nF2,
              k_rc_pass2, (unsigned)w.ntiles, RCB, 0, s, A);
  if (!status) {  // synchronous check
    int64_t chk[3] = {0, 0, 0};
    PH_HIP(hipMemcpyAsync(chk, w.chk, 3 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    PH_HIP(hipStreamSynchronize(s));
    if (chk[2]) return err(PHFEM_EINVAL, "an input id lies outside the mesh (vertex, edge or refined node)");
    if (chk[0] != nEd2 || chk[1] != nF2)
      return err(PHFEM_EINVAL, "input connectivity is not the first-appearance numbering of a conforming, "
                               "consistently oriented mesh (refined counts differ from 2nEd+3nF+6nE, 4nF+16nE)");
  }
  counts[0] = nEd2;
  counts[1] = nF2;
  counts[2] = 2 * nF2 - 4 * nE2;
  return PHFEM_OK;
}

// ---------------------------------------------------------------- several levels in one call
namespace ph {

struct MeshSizes {
  int64_t nC, nE, nEd, nF;
};
static MeshSizes refined(const MeshSizes& m) {
  return {m.nC + m.nEd + m.nE, 12 * m.nE, 2 * m.nEd + 3 * m.nF + 6 * m.nE, 4 * m.nF + 16 * m.nE};
}

// the arrays of one mesh with its connectivity, carved from an arena
struct MeshBufs {
  double* coord;
  int32_t *tetra, *edges, *t2e, *eft, *pre, *faces, *t2f, *f2t, *nbr;
  int8_t* sigma;
};
static void mesh_layout(Arena& a, const MeshSizes& m, MeshBufs& b) {
  b.coord = a.take<double>(3 * m.nC);
  b.tetra = a.take<int32_t>(4 * m.nE);
  b.edges = a.take<int32_t>(2 * m.nEd);
  b.t2e = a.take<int32_t>(6 * m.nE);
  b.eft = a.take<int32_t>(m.nEd);
  b.pre = a.take<int32_t>(m.nE);
  b.faces = a.take<int32_t>(3 * m.nF);
  b.t2f = a.take<int32_t>(4 * m.nE);
  b.sigma = a.take<int8_t>(4 * m.nE);
  b.f2t = a.take<int32_t>(2 * m.nF);
  b.nbr = a.take<int32_t>(4 * m.nE);
}

__global__ void k_zero_i32(int32_t* __restrict__ p) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0;
}

struct LevelsWS {
  MeshBufs m[2];  // ping-pong intermediate meshes (levels 1 .. L-1), sized for level L-1
  int32_t* status;
  void* sub;
  size_t sub_bytes;
};
static size_t levels_layout(Arena& a, MeshSizes m, int L, LevelsWS* w) {
  MeshSizes mid = m;  // largest intermediate: level L-1
  size_t inner = 0;
  for (int l = 0; l < L; ++l) {
    inner = std::max(inner, phfem_refine_connected_workspace(mid.nE, mid.nEd));
    if (l < L - 1) mid = refined(mid);
  }
  MeshBufs b[2];
  for (int i = 0; i < 2; ++i) mesh_layout(a, L > 1 ? mid : MeshSizes{0, 0, 0, 0}, b[i]);
  int32_t* st = a.take<int32_t>(64);
  void* sub = a.take<uint8_t>(inner);
  if (w) {
    w->m[0] = b[0];
    w->m[1] = b[1];
    w->status = st;
    w->sub = sub;
    w->sub_bytes = inner;
  }
  return a.size();
}

}  // namespace ph

extern "C" int phfem_refined_sizes(int64_t nC, int64_t nE, int64_t nEd, int64_t nF, int32_t levels, int64_t* out) {
  clear_error();
  if (!out || levels < 0 || nC <= 0 || nE <= 0 || nEd <= 0 || nF <= 0) return err(PHFEM_EINVAL, "bad arguments");
  MeshSizes m{nC, nE, nEd, nF};
  for (int l = 0; l < levels; ++l) {
    m = refined(m);
    if (m.nE > (int64_t(1) << 40)) return err(PHFEM_EINVAL, "sizes overflow");
  }
  out[0] = m.nC;
  out[1] = m.nE;
  out[2] = m.nEd;
  out[3] = m.nF;
  return PHFEM_OK;
}

extern "C" size_t phfem_refine_connected_levels_workspace(int64_t nC, int64_t nE, int64_t nEd, int64_t nF,
                                                          int32_t levels) {
  if (nC <= 0 || nE <= 0 || nEd <= 0 || nF <= 0 || levels < 1 || levels > 16) return 0;
  Arena a;
  return levels_layout(a, MeshSizes{nC, nE, nEd, nF}, levels, nullptr);
}

extern "C" int phfem_refine_connected_levels(
    int64_t nC, const double* coord, int64_t nE, const int32_t* tetra, int64_t nEd, int64_t nF,
    const int32_t* tet2edge, const int32_t* edge_first_tet, const int32_t* tet_edge_prefix, const int32_t* tet2face,
    const int32_t* nbr, int32_t levels, void* work, size_t work_bytes, double* coord_out, int32_t* tetra_out,
    int32_t* edges_out, int32_t* tet2edge_out, int32_t* edge_first_tet_out, int32_t* tet_edge_prefix_out,
    int32_t* faces_out, int32_t* tet2face_out, int8_t* sigma_out, int32_t* face2tet_out, int32_t* nbr_out,
    int64_t* counts, int32_t* status, phfem_stream_t stream_) {
  clear_error();
  hipStream_t s = (hipStream_t)stream_;
  if (levels < 1 || levels > 16) return err(PHFEM_EINVAL, "levels must be in [1, 16]");
  if (nC <= 0 || nE <= 0 || nEd <= 0 || nF <= 0) return err(PHFEM_EINVAL, "bad sizes");
  const size_t need = phfem_refine_connected_levels_workspace(nC, nE, nEd, nF, levels);
  if (!work || work_bytes < need) return err(PHFEM_EWORKSPACE, "refine_connected_levels workspace too small");
  Arena a(work, work_bytes);
  LevelsWS w;
  levels_layout(a, MeshSizes{nC, nE, nEd, nF}, levels, &w);
  int32_t* st = status ? status : w.status;
  if (!status) PH_LAUNCH("zero_i32", k_zero_i32, 1, 64, 0, s, st);
  MeshSizes m{nC, nE, nEd, nF};
  MeshBufs in{const_cast<double*>(coord), const_cast<int32_t*>(tetra), nullptr, const_cast<int32_t*>(tet2edge),
              const_cast<int32_t*>(edge_first_tet), const_cast<int32_t*>(tet_edge_prefix), nullptr,
              const_cast<int32_t*>(tet2face), nullptr, const_cast<int32_t*>(nbr), nullptr};
  for (int l = 0; l < levels; ++l) {
    const bool last = l == levels - 1;
    MeshBufs out = last ? MeshBufs{coord_out, tetra_out, edges_out, tet2edge_out, edge_first_tet_out,
                                   tet_edge_prefix_out, faces_out, tet2face_out, face2tet_out, nbr_out, sigma_out}
                        : w.m[l & 1];
    int64_t c3[3];
    int rc = phfem_refine_connected(m.nC, in.coord, m.nE, in.tetra, m.nEd, m.nF, in.t2e, in.eft, in.pre, in.t2f,
                                    in.nbr, w.sub, w.sub_bytes, out.coord, out.tetra, out.edges, out.t2e, out.eft,
                                    out.pre, out.faces, out.t2f, out.sigma, out.f2t, out.nbr, c3, st, stream_);
    if (rc) return rc;
    m = refined(m);
    in = out;
    if (last && counts) {
      counts[0] = c3[0];
      counts[1] = c3[1];
      counts[2] = c3[2];
    }
  }
  if (!status) {
    int32_t h = 0;
    PH_HIP(hipMemcpyAsync(&h, st, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    PH_HIP(hipStreamSynchronize(s));
    if (h) return err(PHFEM_EINVAL, "input connectivity check failed (ids out of range or not a first-appearance "
                                    "numbering of a conforming, consistently oriented mesh)");
  }
  return PHFEM_OK;
}
