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
// local face of corner child v that lies on coarse face k (15 if none)
__host__ __device__ constexpr int cornerface(int v, int k) { return (int)((0x12f1f2021f0f210ull >> (4 * (4 * v + k))) & 15ull); }
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
__host__ __device__ constexpr int nverts(int c, int kk) { return (fs(c, kk, 0) < 4) + (fs(c, kk, 1) < 4) + (fs(c, kk, 2) < 4); }
__host__ __device__ constexpr bool has_c(int c, int kk) { return fs(c, kk, 0) == 10 || fs(c, kk, 1) == 10 || fs(c, kk, 2) == 10; }
__host__ __device__ constexpr int vmask_of(int s) { return s < 4 ? (1 << s) : (s < 10 ? ((1 << ev0(s - 4)) | (1 << ev1(s - 4))) : 0); }
__host__ __device__ constexpr int span(int c, int kk) { return vmask_of(fs(c, kk, 0)) | vmask_of(fs(c, kk, 1)) | vmask_of(fs(c, kk, 2)); }
__host__ __device__ constexpr int popc4(int m) { return (m & 1) + ((m >> 1) & 1) + ((m >> 2) & 1) + ((m >> 3) & 1); }
__host__ __device__ constexpr int fkind(int c, int kk) {
  return has_c(c, kk) ? 0 : (nverts(c, kk) == 1 ? 1 : (popc4(span(c, kk)) == 3 ? 2 : 0));
}
// coarse face of a kind-1/2 face: the face opposite the vertex it does not span
__host__ __device__ constexpr int fcoarse(int c, int kk) {
  return opp((span(c, kk) & 1) == 0 ? 0 : ((span(c, kk) & 2) == 0 ? 1 : ((span(c, kk) & 4) == 0 ? 2 : 3)));
}
__host__ __device__ constexpr int symset(int c, int kk) { return (1 << fs(c, kk, 0)) | (1 << fs(c, kk, 1)) | (1 << fs(c, kk, 2)); }
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

__device__ __forceinline__ int loc4(const int a[4], int x) { return a[0] == x ? 0 : (a[1] == x ? 1 : (a[2] == x ? 2 : 3)); }

// Run-time tables (a thread handles one refined row, so the child index is a run-time value)
struct RuleTables {
  int8_t f3c[6], f3j[6];  // first (octahedron child, local edge) holding (M_j, C)
  int8_t fkind[48];       // per child*4 + local face: 0 inside, 1 corner triangle, 2 middle triangle
  int8_t fco[48];         // coarse face of a kind-1/2 face
  int8_t fpart[48];       // partner child*4 + local face of a kind-0 face
};
__host__ __device__ constexpr RuleTables make_tables() {
  RuleTables T{};
  for (int j = 0; j < 6; ++j) {
    T.f3c[j] = (int8_t)first3(j, false);
    T.f3j[j] = (int8_t)first3(j, true);
  }
  for (int c = 0; c < 12; ++c)
    for (int kk = 0; kk < 4; ++kk) {
      T.fkind[4 * c + kk] = (int8_t)fkind(c, kk);
      T.fco[4 * c + kk] = (int8_t)(fkind(c, kk) ? fcoarse(c, kk) : 0);
      T.fpart[4 * c + kk] = (int8_t)(fkind(c, kk) ? 0 : fpartner(c, kk));
    }
  return T;
}
__constant__ RuleTables c_rt = make_tables();

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
  uint32_t* inE;        // pass 1: count | first-edge mask << 8 per refined row
  uint32_t* inF;        // pass 1: count | owned-face mask << 8
  const uint32_t* recE; // after the scans: prefix << 6 | first-edge mask
  const uint32_t* recF; // prefix << 4 | owned-face mask
  int32_t* edges2;
  int32_t* t2e2;
  int32_t* eft2;
  int32_t* pre2;
  int32_t* faces2;
  int32_t* t2f2;
  int8_t* sig2;
  int32_t* f2t2;
  int32_t* nbr2;
};

__global__ __launch_bounds__(RCT) void k_rc_prep(int64_t nE, const int32_t* __restrict__ tet,
                                                 const int32_t* __restrict__ t2e, const int32_t* __restrict__ eft,
                                                 const int32_t* __restrict__ t2f, const int32_t* __restrict__ nbr,
                                                 int32_t* __restrict__ minI, int32_t* __restrict__ efp,
                                                 int4* __restrict__ T4, int4* __restrict__ F4, int4* __restrict__ N4,
                                                 int4* __restrict__ E8) {
  int64_t t = (int64_t)blockIdx.x * RCT + threadIdx.x;
  if (t >= nE) return;
  int n[4], e[6];
#pragma unroll
  for (int i = 0; i < 4; ++i) n[i] = tet[i * nE + t];
#pragma unroll
  for (int j = 0; j < 6; ++j) e[j] = t2e[j * nE + t];
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

__device__ __forceinline__ int64_t rowof(int64_t nE, int64_t tt, int c) { return c == 0 ? tt : nE + 11 * tt + (c - 1); }
__device__ __forceinline__ int get4(const int4& v, int i) { return i == 0 ? v.x : (i == 1 ? v.y : (i == 2 ? v.z : v.w)); }
__device__ __forceinline__ int loc4v(const int4& v, int x) { return v.x == x ? 0 : (v.y == x ? 1 : (v.z == x ? 2 : 3)); }

// One refined row: its coarse tet and child, the coarse data it needs.
struct RCRow {
  int64_t r, t;
  int c;
  int4 n, f, nb, e0, e1;  // e0 = edges 0..3, e1.xy = edges 4, 5
};
__device__ __forceinline__ int edge_of(const RCRow& R, int j) { return j < 4 ? get4(R.e0, j) : (j == 4 ? R.e1.x : R.e1.y); }

__device__ __forceinline__ void rc_row(const RCArgs& A, int64_t r, RCRow& R) {
  const int64_t nE = A.nE;
  R.r = r;
  if (r < nE) {
    R.t = r;
    R.c = 0;
  } else {
    const int64_t q = r - nE;
    R.t = q / 11;
    R.c = 1 + (int)(q - 11 * R.t);
  }
  R.n = A.T4[R.t];
  R.f = A.F4[R.t];
  R.nb = A.N4[R.t];
  R.e0 = A.E8[2 * R.t];
  R.e1 = A.E8[2 * R.t + 1];
}

__device__ __forceinline__ int ech(int c, int p) { return ch(c, p); }  // run-time c: shifts of packed constants

// first occurrence (row, local edge) of local edge jj of this row's child
__device__ __forceinline__ void edge_first_rt(const RCArgs& A, const RCRow& R, int jj, int64_t& er, int& ej) {
  const int64_t nE = A.nE, t = R.t;
  const int c = R.c;
  const int s0 = ech(c, ev0(jj)), s1 = ech(c, ev1(jj));
  const int lo = s0 < s1 ? s0 : s1, hi = s0 < s1 ? s1 : s0;
  if (hi == 10) {  // (M_j, C): inside t
    er = rowof(nE, t, c_rt.f3c[lo - 4]);
    ej = c_rt.f3j[lo - 4];
    return;
  }
  if (lo < 4) {  // (V_a, M_j): half of coarse edge e_j at node v
    const int j = hi - 4;
    const int e = edge_of(R, j);
    const int v = get4(R.n, lo);
    const int na = get4(R.n, ev0(j)), nb = get4(R.n, ev1(j));
    const int lon = na < nb ? na : nb;
    const int mi = A.minI[2 * e + (v == lon ? 0 : 1)];
    if (mi != INT_MAX && (mi >> 2) < nE) {
      er = mi >> 2;  // child 0 of that tet, local edge j of (I, m_j)
      ej = mi & 3;
      return;
    }
    const int p0 = A.efp[e];
    const int flip = p0 & 1, p = p0 >> 1;
    const int t0 = p / 6, j0 = p - 6 * t0;
    const int vl = ((v == lon) != (flip != 0)) ? ev0(j0) : ev1(j0);
    const bool ok = p0 >= 0 && t0 < nE;  // unset only for inconsistent input
    er = ok ? rowof(nE, t0, vl) : R.r;
    ej = ok ? posv(vl, j0) - 1 : jj;
    return;
  }
  // (M_i, M_j) on a coarse face: corner child of the shared vertex, here or in the neighbour
  const int i = lo - 4, j = hi - 4;
  const int v = common_v(i, j), a = other_end(i, v), b = other_end(j, v);
  const int k = face_with(v, a, b);
  int64_t rr = rowof(nE, t, v);
  int jr = eidx(posv(v, i), posv(v, j));
  const int tn = get4(R.nb, k);
  if (tn >= 0) {
    const int4 nn = A.T4[tn];
    const int v2 = loc4v(nn, get4(R.n, v)), a2 = loc4v(nn, get4(R.n, a)), b2 = loc4v(nn, get4(R.n, b));
    const int le2 = eidx(posv(v2, eidx(v2, a2)), posv(v2, eidx(v2, b2)));
    const int64_t r2 = rowof(nE, tn, v2);
    if (6 * r2 + le2 < 6 * rr + jr) {
      rr = r2;
      jr = le2;
    }
  }
  er = rr;
  ej = jr;
}

// other occurrence (row, local face) of local face kk of this row's child; row -1 on the boundary
__device__ __forceinline__ void face_other_rt(const RCArgs& A, const RCRow& R, int kk, int64_t& fr, int& fk) {
  const int64_t nE = A.nE;
  const int idx = 4 * R.c + kk;
  const int kind = c_rt.fkind[idx];
  if (kind == 0) {
    const int p = c_rt.fpart[idx];
    fr = rowof(nE, R.t, p >> 2);
    fk = p & 3;
    return;
  }
  const int k = c_rt.fco[idx];
  const int tn = get4(R.nb, k);
  if (tn < 0) {
    fr = -1;
    fk = 0;
    return;
  }
  const int k2 = loc4v(A.F4[tn], get4(R.f, k));
  if (kind == 2) {
    fr = rowof(nE, tn, 8 + k2);
    fk = 0;
  } else {
    const int v2 = loc4v(A.T4[tn], get4(R.n, R.c & 3));  // corner child c holds vertex V_c
    fr = rowof(nE, tn, v2);
    fk = cornerface(v2, k2);
  }
}

// pass 1: count | mask << 8 of first edges and owned faces for every refined row
__global__ __launch_bounds__(RCT) void k_rc_pass1(RCArgs A) {
  const int64_t r = (int64_t)blockIdx.x * RCT + threadIdx.x;
  if (r >= A.nE2) return;
  RCRow R;
  rc_row(A, r, R);
  int me = 0, mf = 0;
#pragma unroll
  for (int jj = 0; jj < 6; ++jj) {
    int64_t er;
    int ej;
    edge_first_rt(A, R, jj, er, ej);
    me |= (er == r && ej == jj) ? (1 << jj) : 0;
  }
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    int64_t fr;
    int fk;
    face_other_rt(A, R, kk, fr, fk);
    mf |= (fr < 0 || 4 * fr + fk > 4 * r + kk) ? (1 << kk) : 0;
  }
  A.inE[r] = (uint32_t)__popc(me) | ((uint32_t)me << 8);
  A.inF[r] = (uint32_t)__popc(mf) | ((uint32_t)mf << 8);
}

__device__ __forceinline__ int sym_node(const RCArgs& A, const RCRow& R, int sym) {
  if (sym < 4) return get4(R.n, sym);
  if (sym < 10) {
    const int e = edge_of(R, sym - 4);
    return (int)(A.nC + A.eft[e] + e + 1);
  }
  return (int)(A.nC + R.t + A.pre[R.t]);
}

// pass 2: ids of the refined edges and faces of every row, and all outputs
__global__ __launch_bounds__(RCT) void k_rc_pass2(RCArgs A) {
  const int64_t r = (int64_t)blockIdx.x * RCT + threadIdx.x;
  if (r >= A.nE2) return;
  RCRow R;
  rc_row(A, r, R);
  const int c = R.c;
  const uint32_t oe = A.recE[r], of = A.recF[r];
  const int me = oe & 63, mf = of & 15;
  A.pre2[r] = (int32_t)(oe >> 6);
#pragma unroll
  for (int jj = 0; jj < 6; ++jj) {
    int32_t id;
    if ((me >> jj) & 1) {
      id = (int32_t)((oe >> 6) + __popc(me & ((1 << jj) - 1)));
      const int na = sym_node(A, R, ech(c, ev0(jj))), nb = sym_node(A, R, ech(c, ev1(jj)));
      A.edges2[id] = na < nb ? na : nb;
      A.edges2[A.nEd2 + id] = na < nb ? nb : na;
      A.eft2[id] = (int32_t)r;
    } else {
      int64_t er;
      int ej;
      edge_first_rt(A, R, jj, er, ej);
      const uint32_t o = A.recE[er];
      id = (int32_t)((o >> 6) + __popc((o & 63) & ((1u << ej) - 1)));
    }
    A.t2e2[jj * A.nE2 + r] = id;
  }
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    int64_t fr;
    int fk;
    face_other_rt(A, R, kk, fr, fk);
    const bool own = (mf >> kk) & 1;
    int32_t id;
    if (own) {
      id = (int32_t)((of >> 4) + __popc(mf & ((1 << kk) - 1)));
      A.f2t2[id] = (int32_t)(4 * r + kk);
      A.f2t2[A.nF2 + id] = fr < 0 ? -1 : (int32_t)(4 * fr + fk);
#pragma unroll
      for (int m = 0; m < 3; ++m) A.faces2[m * A.nF2 + id] = sym_node(A, R, ech(c, fv(kk, m)));
    } else {
      const uint32_t o = A.recF[fr];
      id = (int32_t)((o >> 4) + __popc((o & 15) & ((1u << fk) - 1)));
    }
    A.t2f2[kk * A.nE2 + r] = id;
    A.sig2[kk * A.nE2 + r] = own ? 1 : -1;
    A.nbr2[kk * A.nE2 + r] = fr < 0 ? -1 : (int32_t)fr;
  }
}

__global__ __launch_bounds__(RCT) void k_fill_i32(int64_t n, int32_t v, int32_t* __restrict__ a) {
  for (int64_t i = (int64_t)blockIdx.x * RCT + threadIdx.x; i < n; i += (int64_t)gridDim.x * RCT) a[i] = v;
}

struct RCWS {
  int32_t *minI, *efp;
  int4 *T4, *F4, *N4, *E8;
  uint32_t *inE, *inF, *recF, *tot;
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
  w.inE = a.take<uint32_t>(n2);
  w.inF = a.take<uint32_t>(n2);
  w.recF = a.take<uint32_t>(n2);
  w.tot = a.take<uint32_t>(16);
  w.sub = a.size();
}

int launch_refine(int64_t nC, const double* coord, int64_t nE, const int32_t* tetra, const int32_t* t2e,
                  const int32_t* eft, const int32_t* pre, int64_t nCo, double* coord_out, int32_t* tetra_out,
                  hipStream_t s);

}  // namespace ph

using namespace ph;

extern "C" size_t phfem_refine_connected_workspace(int64_t nE, int64_t nEd) {
  if (nE <= 0 || nEd <= 0) return 0;
  Arena a;
  RCWS w;
  rc_layout(a, nE, nEd, w);
  return w.sub + scan_workspace(12 * nE);
}

extern "C" int phfem_refine_connected(int64_t nC, const double* coord, int64_t nE, const int32_t* tetra, int64_t nEd,
                                      int64_t nF, const int32_t* tet2edge, const int32_t* edge_first_tet,
                                      const int32_t* tet_edge_prefix, const int32_t* tet2face, const int32_t* nbr,
                                      void* work, size_t work_bytes, double* coord_out, int32_t* tetra_out,
                                      int32_t* edges_out, int32_t* tet2edge_out, int32_t* edge_first_tet_out,
                                      int32_t* tet_edge_prefix_out, int32_t* faces_out, int32_t* tet2face_out,
                                      int8_t* sigma_out, int32_t* face2tet_out, int32_t* nbr_out, int64_t* counts,
                                      phfem_stream_t stream_) {
  clear_error();
  hipStream_t s = (hipStream_t)stream_;
  if (nC <= 0 || nE <= 0 || nEd <= 0 || nF <= 0) return err(PHFEM_EINVAL, "bad sizes");
  const int64_t nE2 = 12 * nE, nC2 = nC + nEd + nE;
  const int64_t nEd2 = 2 * nEd + 3 * nF + 6 * nE, nF2 = 4 * nF + 16 * nE;
  if (6 * nE2 >= (int64_t(1) << 31) || nC2 >= (int64_t(1) << 31) || 4 * nF2 >= (int64_t(1) << 31))
    return err(PHFEM_EINVAL, "refined mesh exceeds int32 positions");
  if (!coord || !tetra || !tet2edge || !edge_first_tet || !tet_edge_prefix || !tet2face || !nbr || !coord_out ||
      !tetra_out || !edges_out || !tet2edge_out || !edge_first_tet_out || !tet_edge_prefix_out || !faces_out ||
      !tet2face_out || !sigma_out || !face2tet_out || !nbr_out || !counts)
    return err(PHFEM_EINVAL, "null argument");
  if (!work || work_bytes < phfem_refine_connected_workspace(nE, nEd))
    return err(PHFEM_EWORKSPACE, "refine_connected workspace too small");
  Arena a(work, work_bytes);
  RCWS w;
  rc_layout(a, nE, nEd, w);
  int rc = launch_refine(nC, coord, nE, tetra, tet2edge, edge_first_tet, tet_edge_prefix, nC2, coord_out, tetra_out,
                         s);
  if (rc) return rc;
  PH_LAUNCH("fill_i32", k_fill_i32, (unsigned)std::min<int64_t>(grid_for(2 * nEd, RCT), 4096), RCT, 0, s, 2 * nEd,
            (int32_t)INT_MAX, w.minI);
  PH_LAUNCH("fill_i32", k_fill_i32, (unsigned)std::min<int64_t>(grid_for(nEd, RCT), 4096), RCT, 0, s, nEd, -1, w.efp);
  PH_LAUNCH_B("rc_prep", 60.0 * nE + 12.0 * nEd + 80.0 * nE, k_rc_prep, grid_for(nE, RCT), RCT, 0, s, nE, tetra,
              tet2edge, edge_first_tet, tet2face, nbr, w.minI, w.efp, w.T4, w.F4, w.N4, w.E8);
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
  A.inE = w.inE;
  A.inF = w.inF;
  A.recE = w.inE;  // the edge scan writes its records in place
  A.recF = w.recF;
  A.edges2 = edges_out;
  A.t2e2 = tet2edge_out;
  A.eft2 = edge_first_tet_out;
  A.pre2 = tet_edge_prefix_out;
  A.faces2 = faces_out;
  A.t2f2 = tet2face_out;
  A.sig2 = sigma_out;
  A.f2t2 = face2tet_out;
  A.nbr2 = nbr_out;
  // pass 1 reads the coarse AoS data once (cache-shared by the 12 rows of a tet) and writes
  // two words per refined row
  PH_LAUNCH_B("refconn_pass1", 80.0 * nE + 12.0 * nEd + 8.0 * nE2, k_rc_pass1, grid_for(nE2, RCT), RCT, 0, s, A);
  a.off = w.sub;
  rc = scan_packed(w.inE, w.inE, nE2, 6, w.tot, a, s);
  if (rc) return rc;
  a.off = w.sub;
  rc = scan_packed(w.inF, w.recF, nE2, 4, w.tot + 1, a, s);
  if (rc) return rc;
  // pass 2 writes every refined connectivity array once
  PH_LAUNCH_B("refconn_pass2", 80.0 * nE + 12.0 * nEd + 8.0 * nE2 + (24.0 + 4 + 16 + 1 * 4 + 16) * nE2 + 12.0 * nEd2 +
                                   20.0 * nF2,
              k_rc_pass2, grid_for(nE2, RCT), RCT, 0, s, A);
  uint32_t tot[2] = {0, 0};
  PH_HIP(hipMemcpyAsync(tot, w.tot, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  PH_HIP(hipStreamSynchronize(s));
  if ((int64_t)tot[0] != nEd2 || (int64_t)tot[1] != nF2)
    return err(PHFEM_EINVAL, "input connectivity is not the first-appearance numbering of a conforming, "
                             "consistently oriented mesh (refined counts differ from 2nEd+3nF+6nE, 4nF+16nE)");
  counts[0] = nEd2;
  counts[1] = nF2;
  counts[2] = 2 * nF2 - 4 * nE2;
  return PHFEM_OK;
}
