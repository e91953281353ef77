// Oracle for the primal hybrid FEM hot path of "Vectorized 3D mesh refinement and
// implementation of primal hybrid FEM in MATLAB" (Nagula Mallesham, Gaddam, Valdman,
// Acharya, arXiv 2509.11133).
//
// TEST INFRASTRUCTURE ONLY.  Plain, slow, single-threaded code written so that it can be
// checked against the paper by eye.  Only the tests, the smoke check and the CPU baseline
// leg of the benchmark may load it.  It shares no code, header or table with the GPU
// library; the two only agree on data layout (0-based int32 indices, SoA arrays: the k-th
// column of an n x m MATLAB array is the k-th contiguous block of length n).
//
// Arithmetic: FP64 throughout, long double for the 4x4 inverses (A(T)^-1 through the exact
// split of its constant mode, see element_inverse) and the brute-force dense
// solve.  Every function names the passage of the paper it follows.
//
// Readings of the paper taken here (the paper is silent, ambiguous or garbled there):
//  * The operator is -div(kappa grad u) + c u = f with c > 0 (the paper: kappa = c = 1);
//    c <= 0 makes the element matrices singular and is rejected.
//  * |T| in eq. (K(T)) is det of the 4x4 vertex matrix (= 6 vol), so K_ij = vol grad_i.grad_j.
//  * Row 4 of eq. (C(T)) reads sigma_4|F_4| r_4 (the printed sigma_3 is a typo).
//  * sigma = +1 on the occurrence of a face in its owner (the lowest tet index holding it),
//    -1 on the other occurrence; all faces use the FacesUp numbering.
//  * The face system is solved in the SPD form S+ = C A^-1 C', r+ = b_D - C A^-1 B
//    (the paper's S = -C A^-1 C' times -1).
//  * All boundary faces are Dirichlet faces (no Neumann faces on the hot path).

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <set>
#include <string>
#include <vector>

namespace {

enum { ORC_OK = 0, ORC_EINVAL = 1, ORC_EORIENT = 2, ORC_EDEGEN = 3, ORC_ESINGULAR = 4, ORC_ENOCONV = 5 };

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

// ---------------------------------------------------------------------------------------
// Local numbering of a tetrahedron T = [a b c d] (= [I J K L] in the listings).
// Edges in NumEdges order: IJ, IK, IL, JK, JL, KL (Section 3.1, Listing 2).
const int EDGE_V[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
// Oriented faces [a b c], [a c d], [a d b], [d c b] (Section 2.2).
const int FACE_V[4][3] = {{0, 1, 2}, {0, 2, 3}, {0, 3, 1}, {3, 2, 1}};
// Triples inserted into Edges2Tetra (Listing 3): (I,J,K), (I,L,J), (I,K,L), (J,L,K).
const int E2T_TRIPLE[4][3] = {{0, 1, 2}, {0, 3, 1}, {0, 2, 3}, {1, 3, 2}};

typedef std::pair<int, int> Key2;

int tet_node(const int32_t* tet, int64_t nE, int64_t t, int i) { return tet[i * nE + t]; }

int check_mesh(int64_t nC, int64_t nE, const int32_t* tet) {
  if (nC <= 0 || nE <= 0 || tet == nullptr) return fail(ORC_EINVAL, "empty mesh or null pointer");
  for (int64_t t = 0; t < nE; ++t) {
    int v[4];
    for (int i = 0; i < 4; ++i) {
      v[i] = tet_node(tet, nE, t, i);
      if (v[i] < 0 || v[i] >= nC) return fail(ORC_EINVAL, "node index out of range in tet " + std::to_string(t));
    }
    for (int i = 0; i < 4; ++i)
      for (int j = i + 1; j < 4; ++j)
        if (v[i] == v[j]) return fail(ORC_EINVAL, "repeated node in tet " + std::to_string(t));
  }
  return ORC_OK;
}

// NumEdges (Listing 2): edges of all tets in (tet, local edge) order, each row sorted,
// then a stable unique: global edge number = rank of first appearance.
struct EdgeData {
  std::map<Key2, int> id;
  std::vector<int> a, b, first_tet;
  std::vector<int> tet2edge;  // [6][nE]
  std::vector<int> prefix;    // edges first appearing in tets before t
};

void build_edges(int64_t nE, const int32_t* tet, EdgeData& E) {
  E.tet2edge.assign(6 * nE, -1);
  E.prefix.assign(nE, 0);
  for (int64_t t = 0; t < nE; ++t) {
    E.prefix[t] = (int)E.a.size();
    for (int j = 0; j < 6; ++j) {
      int p = tet_node(tet, nE, t, EDGE_V[j][0]);
      int q = tet_node(tet, nE, t, EDGE_V[j][1]);
      Key2 k(std::min(p, q), std::max(p, q));
      auto it = E.id.find(k);
      int e;
      if (it == E.id.end()) {
        e = (int)E.a.size();
        E.id[k] = e;
        E.a.push_back(k.first);
        E.b.push_back(k.second);
        E.first_tet.push_back((int)t);
      } else {
        e = it->second;
      }
      E.tet2edge[j * nE + t] = e;
    }
  }
}

int edge_of(const EdgeData& E, int p, int q) {
  auto it = E.id.find(Key2(std::min(p, q), std::max(p, q)));
  return it == E.id.end() ? -1 : it->second;
}

// EdgeNum2Tetra (Listing 3, Remark 1): for the oriented face (i,j,k) of tet m the directed
// edge pairs (e_jk,e_ij), (e_ki,e_jk), (e_ij,e_ki) map to m.  The MATLAB sparse() call
// would add colliding entries; a collision means the same oriented face occurs twice,
// i.e. the tets are not consistently oriented (or a face has more than two tets).
int build_e2t(int64_t nE, const int32_t* tet, const EdgeData& E, std::map<Key2, int>& E2T) {
  for (int64_t m = 0; m < nE; ++m) {
    for (int f = 0; f < 4; ++f) {
      int i = tet_node(tet, nE, m, E2T_TRIPLE[f][0]);
      int j = tet_node(tet, nE, m, E2T_TRIPLE[f][1]);
      int k = tet_node(tet, nE, m, E2T_TRIPLE[f][2]);
      int eij = edge_of(E, i, j), ejk = edge_of(E, j, k), eki = edge_of(E, k, i);
      const Key2 keys[3] = {Key2(ejk, eij), Key2(eki, ejk), Key2(eij, eki)};
      for (const Key2& key : keys) {
        if (E2T.count(key))
          return fail(ORC_EORIENT, "oriented face seen twice (tets " + std::to_string(E2T[key]) + " and " +
                                       std::to_string(m) + "): mesh not consistently oriented");
        E2T[key] = (int)m;
      }
    }
  }
  return ORC_OK;
}

// FacesUp (Listing 4) + fullFaces: the neighbour across face [i j k] is Edges2Tetra(e_ij,e_jk)
// (0 = none).  A face is stored when it has no neighbour or the neighbour index is larger,
// so the owner is the lowest tet index holding the face and the face number is the rank by
// (owner, local face).  tet2face is fullFaces' g_ind; sigma = +1 at the owner, -1 at the
// repeated occurrence (IVRF).
struct FaceData {
  std::vector<std::array<int, 3>> tuple;  // Faces rows
  std::vector<int> owner_slot, nbr_slot;  // slots 4t+k, -1 = boundary
  std::vector<int> tet2face;              // [4][nE]
  std::vector<int8_t> sigma;              // [4][nE]
  std::vector<int> nbr;                   // [4][nE]
};

int build_faces(int64_t nE, const int32_t* tet, const EdgeData& E, const std::map<Key2, int>& E2T, FaceData& F) {
  F.tet2face.assign(4 * nE, -1);
  F.sigma.assign(4 * nE, 0);
  F.nbr.assign(4 * nE, -1);
  std::map<std::array<int, 3>, int> by_nodes;
  for (int64_t t = 0; t < nE; ++t) {
    for (int k = 0; k < 4; ++k) {
      int i = tet_node(tet, nE, t, FACE_V[k][0]);
      int j = tet_node(tet, nE, t, FACE_V[k][1]);
      int l = tet_node(tet, nE, t, FACE_V[k][2]);
      auto it = E2T.find(Key2(edge_of(E, i, j), edge_of(E, j, l)));
      int nb = (it == E2T.end()) ? -1 : it->second;
      if (nb == (int)t) return fail(ORC_EORIENT, "face probe returned the tet itself");
      std::array<int, 3> s = {i, j, l};
      std::sort(s.begin(), s.end());
      F.nbr[k * nE + t] = nb;
      if (nb < 0 || (int)t < nb) {
        int id = (int)F.tuple.size();
        F.tuple.push_back({i, j, l});
        F.owner_slot.push_back((int)(4 * t + k));
        F.nbr_slot.push_back(-1);
        if (by_nodes.count(s)) return fail(ORC_EORIENT, "face stored twice");
        by_nodes[s] = id;
        F.tet2face[k * nE + t] = id;
        F.sigma[k * nE + t] = 1;
      } else {
        auto jt = by_nodes.find(s);
        if (jt == by_nodes.end()) return fail(ORC_EORIENT, "neighbour does not hold the face");
        int id = jt->second;
        if (F.owner_slot[id] / 4 != nb || F.nbr_slot[id] != -1)
          return fail(ORC_EORIENT, "face with more than two tets or inconsistent neighbour");
        F.nbr_slot[id] = (int)(4 * t + k);
        F.tet2face[k * nE + t] = id;
        F.sigma[k * nE + t] = -1;
      }
    }
  }
  // every interior face must have been seen from both sides
  for (size_t id = 0; id < F.tuple.size(); ++id) {
    int ot = F.owner_slot[id] / 4, ok = F.owner_slot[id] % 4;
    int nb = F.nbr[ok * nE + ot];
    if (nb >= 0 && F.nbr_slot[id] < 0) return fail(ORC_EORIENT, "interior face seen from one side only");
  }
  return ORC_OK;
}

// ---------------------------------------------------------------------------------------
// Scalars: long double and a forward-mode dual number (value + one directional derivative),
// used to differentiate the per-tet functional of the adjoint with respect to coordinates.
struct Dual {
  long double v, d;
  Dual() : v(0), d(0) {}
  Dual(long double a) : v(a), d(0) {}
  Dual(long double a, long double b) : v(a), d(b) {}
};
inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(Dual a, Dual b) { return Dual(a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)); }
inline Dual& operator+=(Dual& a, Dual b) { a = a + b; return a; }
inline Dual& operator-=(Dual& a, Dual b) { a = a - b; return a; }
inline Dual sqrt(Dual a) { long double s = sqrtl(a.v); return Dual(s, a.d / (2 * s)); }
inline Dual sin(Dual a) { return Dual(sinl(a.v), a.d * cosl(a.v)); }
inline Dual fabs(Dual a) { return a.v < 0 ? -a : a; }
inline long double val(Dual a) { return a.v; }
inline long double val(long double a) { return a; }
inline long double sqrt(long double a) { return sqrtl(a); }
inline long double sin(long double a) { return sinl(a); }
inline long double fabs(long double a) { return fabsl(a); }

const long double PI_L = 3.141592653589793238462643383279502884L;

// Data functions f, u_D (and exact solutions in the error norms).
enum { FUN_ZERO = 0, FUN_CONST = 1, FUN_SIN3 = 2, FUN_LINEAR = 3, FUN_X2Y2Z2 = 4, FUN_X2Y2Z2_LOAD = 5 };

template <class R>
R fun_eval(int kind, const double* p, R x, R y, R z) {
  switch (kind) {
    case FUN_ZERO: return R(0.0L);
    case FUN_CONST: return R((long double)p[0]);
    case FUN_SIN3: return R((long double)p[0]) * sin(R(PI_L) * x) * sin(R(PI_L) * y) * sin(R(PI_L) * z);
    case FUN_LINEAR:
      return R((long double)p[0]) + R((long double)p[1]) * x + R((long double)p[2]) * y + R((long double)p[3]) * z;
    case FUN_X2Y2Z2: return R((long double)p[0]) * x * x * y * y * z * z;
    case FUN_X2Y2Z2_LOAD:  // -kappa Lap(x^2y^2z^2) + c x^2y^2z^2 with kappa = p[0], c = p[1]
      return R(-2.0L * p[0]) * (y * y * z * z + x * x * z * z + x * x * y * y) + R((long double)p[1]) * x * x * y * y * z * z;
    default: return R(0.0L);
  }
}

// gradient of the exact solutions (error norms and linear-solution checks)
void fun_grad(int kind, const double* p, long double x, long double y, long double z, long double g[3]) {
  g[0] = g[1] = g[2] = 0;
  switch (kind) {
    case FUN_SIN3: {
      long double sx = sinl(PI_L * x), sy = sinl(PI_L * y), sz = sinl(PI_L * z);
      long double cx = cosl(PI_L * x), cy = cosl(PI_L * y), cz = cosl(PI_L * z);
      g[0] = p[0] * PI_L * cx * sy * sz;
      g[1] = p[0] * PI_L * sx * cy * sz;
      g[2] = p[0] * PI_L * sx * sy * cz;
      break;
    }
    case FUN_LINEAR: g[0] = p[1]; g[1] = p[2]; g[2] = p[3]; break;
    case FUN_X2Y2Z2:
      g[0] = p[0] * 2 * x * y * y * z * z;
      g[1] = p[0] * 2 * x * x * y * z * z;
      g[2] = p[0] * 2 * x * x * y * y * z;
      break;
    default: break;
  }
}

struct Params {
  double c;
  double kappa_const;
  int32_t f_kind;
  double f_par[4];
  int32_t ud_kind;
  double ud_par[4];
  int32_t quad;  // 0: face-centroid rule of StiffMassPH, 1: P1 interpolation b = M f(x_i)
  // Neumann data on Gamma_N: g = kappa_T grad(u_g) . nu with u_g = fun(g_kind, g_par) and nu
  // the outward unit normal (the paper's example prescribes the flux of its exact solution)
  int32_t g_kind;
  double g_par[4];
};

// ---------------------------------------------------------------------------------------
// Local quantities of one tet (Section 4.2, Listing 6, Listing 7).
template <class R>
struct Local {
  R x[4][3];
  R detP;     // det [1 1 1 1; x; y; z] = 6 * signed volume
  R vol;      // |detP| / 6
  R g[4][3];  // gradients of the barycentric basis: columns 2..4 of the inverse vertex matrix
  R area[4];  // |F_k| = 0.5 |(x3 - x1) x (x2 - x1)| for the face tuple [x1 x2 x3]
};

// Gauss-Jordan inverse with partial pivoting; returns the determinant.
template <class R>
R invert4(R A[4][4], R Ainv[4][4]) {
  R M[4][8];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      M[i][j] = A[i][j];
      M[i][4 + j] = R(i == j ? 1.0L : 0.0L);
    }
  R det(1.0L);
  for (int col = 0; col < 4; ++col) {
    int piv = col;
    for (int r = col + 1; r < 4; ++r)
      if (fabsl(val(M[r][col])) > fabsl(val(M[piv][col]))) piv = r;
    if (val(M[piv][col]) == 0) return R(0.0L);
    if (piv != col) {
      for (int j = 0; j < 8; ++j) std::swap(M[piv][j], M[col][j]);
      det = -det;
    }
    R pv = M[col][col];
    det = det * pv;
    for (int j = 0; j < 8; ++j) M[col][j] = M[col][j] / pv;
    for (int r = 0; r < 4; ++r) {
      if (r == col) continue;
      R f = M[r][col];
      for (int j = 0; j < 8; ++j) M[r][j] = M[r][j] - f * M[col][j];
    }
  }
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) Ainv[i][j] = M[i][4 + j];
  return det;
}

template <class R>
bool local_geometry(Local<R>& L) {
  R P[4][4], Pi[4][4];
  for (int j = 0; j < 4; ++j) {
    P[0][j] = R(1.0L);
    for (int d = 0; d < 3; ++d) P[1 + d][j] = L.x[j][d];
  }
  L.detP = invert4(P, Pi);
  if (val(L.detP) == 0) return false;
  L.vol = fabs(L.detP) / R(6.0L);
  for (int i = 0; i < 4; ++i)
    for (int d = 0; d < 3; ++d) L.g[i][d] = Pi[i][1 + d];
  for (int k = 0; k < 4; ++k) {
    const R* x1 = L.x[FACE_V[k][0]];
    const R* x2 = L.x[FACE_V[k][1]];
    const R* x3 = L.x[FACE_V[k][2]];
    R u[3], w[3];
    for (int d = 0; d < 3; ++d) {
      u[d] = x3[d] - x1[d];
      w[d] = x2[d] - x1[d];
    }
    R cx = u[1] * w[2] - u[2] * w[1];
    R cy = u[2] * w[0] - u[0] * w[2];
    R cz = u[0] * w[1] - u[1] * w[0];
    L.area[k] = R(0.5L) * sqrt(cx * cx + cy * cy + cz * cz);
  }
  return true;
}

// Load vector of one tet.  quad 0 follows StiffMassPH: f at the four face centroids
// Ct1=(P1+P2+P3)/3, Ct2=(P1+P3+P4)/3, Ct3=(P1+P4+P2)/3, Ct4=(P2+P4+P3)/3, weight |T|/4,
// phi_j(Ct_i) = 1/3 for the three vertices of face i.  quad 1: b = M(T) f(x_i) (exact for
// linear f).
template <class R>
void local_load(const Local<R>& L, const Params& P, R B[4]) {
  if (P.quad == 1) {
    R fx[4];
    for (int i = 0; i < 4; ++i) fx[i] = fun_eval<R>(P.f_kind, P.f_par, L.x[i][0], L.x[i][1], L.x[i][2]);
    for (int i = 0; i < 4; ++i) {
      R s(0.0L);
      for (int j = 0; j < 4; ++j) s = s + R(i == j ? 2.0L : 1.0L) * fx[j];
      B[i] = L.vol / R(20.0L) * s;
    }
    return;
  }
  const int CT[4][3] = {{0, 1, 2}, {0, 2, 3}, {0, 3, 1}, {1, 3, 2}};
  R fc[4];
  for (int k = 0; k < 4; ++k) {
    R c[3];
    for (int d = 0; d < 3; ++d) c[d] = (L.x[CT[k][0]][d] + L.x[CT[k][1]][d] + L.x[CT[k][2]][d]) / R(3.0L);
    fc[k] = fun_eval<R>(P.f_kind, P.f_par, c[0], c[1], c[2]);
  }
  B[0] = L.vol * (fc[0] + fc[1] + fc[2]) / R(12.0L);
  B[1] = L.vol * (fc[0] + fc[2] + fc[3]) / R(12.0L);
  B[2] = L.vol * (fc[0] + fc[3] + fc[1]) / R(12.0L);
  B[3] = L.vol * (fc[1] + fc[3] + fc[2]) / R(12.0L);
}

// r_k of eq. (C(T)): 1/3 on the three vertices of face k.
long double rmat(int k, int i) {
  for (int m = 0; m < 3; ++m)
    if (FACE_V[k][m] == i) return 1.0L / 3.0L;
  return 0.0L;
}

// A(T) = kappa K(T) + c M(T) (eq. K(T), eq. M(T)); C(T) row k = sigma_k |F_k| r_k (eq. C(T)).
template <class R>
void local_AC(const Local<R>& L, R kappa, const Params& P, const int sig[4], R A[4][4], R K[4][4], R C[4][4]) {
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      R gg = L.g[i][0] * L.g[j][0] + L.g[i][1] * L.g[j][1] + L.g[i][2] * L.g[j][2];
      K[i][j] = L.vol * gg;
      R m = R((long double)P.c) * L.vol / R(20.0L) * R(i == j ? 2.0L : 1.0L);
      A[i][j] = kappa * K[i][j] + m;
    }
  for (int k = 0; k < 4; ++k)
    for (int i = 0; i < 4; ++i) C[k][i] = R((long double)sig[k]) * L.area[k] * R(rmat(k, i));
}

struct TetIn {
  long double kappa;
  int sig[4];
};

int load_tet(int64_t nC, const double* X, int64_t nE, const int32_t* tet, int64_t t, Local<long double>& L) {
  for (int i = 0; i < 4; ++i) {
    int v = tet_node(tet, nE, t, i);
    for (int d = 0; d < 3; ++d) L.x[i][d] = X[d * nC + v];
  }
  if (!local_geometry(L)) return fail(ORC_EDEGEN, "zero-volume tet " + std::to_string(t));
  return ORC_OK;
}

// A(T)^-1 by the exact split of the constant mode.  Section 4.2's K(T) has zero row sums and
// M(T) = (c|T|/20)(1 + delta_ij), so A(T) 1 = (c|T|/4) 1: with the projector P1 = 1 1'/4,
// A = A_perp + (c|T|/4) P1, where A_perp = kappa K + (c|T|/20)(I - P1) annihilates 1 and acts
// on its complement.  Hence A^-1 = A_perp^+ + 1 1'/(c|T|), and A_perp^+ = (A_perp + a P1)^-1
// - P1/a for any a > 0; a = trace(A_perp)/3 makes that matrix as well conditioned as A_perp
// on the complement.  Inverting A itself loses digits as |K|/(c|T|) ~ h^-2 grows (about 1e-12
// relative after six 12-subtet refinements of the unit cube, even in long double).
long double element_inverse(const long double K[4][4], long double kappa, long double c, long double vol,
                            long double Ainv[4][4]) {
  const long double m = c * vol / 20.0L;
  long double As[4][4], Asi[4][4];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) As[i][j] = kappa * K[i][j] + m * ((i == j ? 1.0L : 0.0L) - 0.25L);
  const long double a = (As[0][0] + As[1][1] + As[2][2] + As[3][3]) / 3.0L;
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) As[i][j] += 0.25L * a;
  const long double det = invert4(As, Asi);
  if (det == 0) return 0;
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) Ainv[i][j] = Asi[i][j] - 0.25L / a + 1.0L / (c * vol);
  return det;
}

// Element Schur complement (Algorithm 1, eq. schur): S(T) = C A^-1 C', r(T) = C A^-1 B.
struct Elem {
  bool neu[4];  // local face on Gamma_N
  long double A[4][4], Ainv[4][4], K[4][4], C[4][4], B[4];
  long double S[4][4], r[4];
  long double vol;
  long double area[4];
};

// Outward unit normal of the tet on its local face k (away from the opposite vertex).
void outward_normal(const Local<long double>& L, int k, long double nu[3]) {
  const long double* x1 = L.x[FACE_V[k][0]];
  const long double* x2 = L.x[FACE_V[k][1]];
  const long double* x3 = L.x[FACE_V[k][2]];
  long double a[3], b[3];
  for (int d = 0; d < 3; ++d) {
    a[d] = x2[d] - x1[d];
    b[d] = x3[d] - x1[d];
  }
  long double n[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
  const int opp = 6 - FACE_V[k][0] - FACE_V[k][1] - FACE_V[k][2];
  long double s = 0;
  for (int d = 0; d < 3; ++d) s += n[d] * (L.x[opp][d] - x1[d]);
  const long double nl = sqrtl(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
  for (int d = 0; d < 3; ++d) nu[d] = (s > 0 ? -n[d] : n[d]) / nl;
}

// g at the centroid of local face k: kappa grad(u_g) . nu (outward)
long double neumann_g(const Local<long double>& L, int k, long double kappa, const Params& P) {
  long double c[3], nu[3], gu[3];
  for (int d = 0; d < 3; ++d)
    c[d] = (L.x[FACE_V[k][0]][d] + L.x[FACE_V[k][1]][d] + L.x[FACE_V[k][2]][d]) / 3.0L;
  outward_normal(L, k, nu);
  fun_grad(P.g_kind, P.g_par, c[0], c[1], c[2], gu);
  return kappa * (gu[0] * nu[0] + gu[1] * nu[1] + gu[2] * nu[2]);
}

// tet2face / neumann (nF flags, 1 = Neumann face) may be null: then no Neumann face.  A
// Neumann face adds LN_j = |F| g(Ct_F) phi_j(Ct_F) = |F| g(Ct_F) / 3 for its three vertices
// to the load (Section 4.3, Multiplier's LN).
int element(int64_t nC, const double* X, int64_t nE, const int32_t* tet, const int8_t* sigma, const double* kappa,
            const Params& P, int64_t t, Elem& E, const int32_t* tet2face = nullptr,
            const uint8_t* neumann = nullptr) {
  Local<long double> L;
  int rc = load_tet(nC, X, nE, tet, t, L);
  if (rc) return rc;
  int sig[4];
  for (int k = 0; k < 4; ++k) sig[k] = sigma ? sigma[k * nE + t] : 1;
  long double kap = kappa ? kappa[t] : P.kappa_const;
  local_AC(L, kap, P, sig, E.A, E.K, E.C);
  local_load(L, P, E.B);
  for (int k = 0; k < 4; ++k) {
    E.neu[k] = neumann && tet2face && neumann[tet2face[k * nE + t]];
    if (!E.neu[k]) continue;
    const long double g = neumann_g(L, k, kap, P);
    for (int m = 0; m < 3; ++m) E.B[FACE_V[k][m]] += L.area[k] * g / 3.0L;
  }
  if (element_inverse(E.K, kap, (long double)P.c, L.vol, E.Ainv) == 0)
    return fail(ORC_ESINGULAR, "singular element matrix");
  long double AiCt[4][4], AiB[4];
  for (int i = 0; i < 4; ++i) {
    for (int l = 0; l < 4; ++l) {
      long double s = 0;
      for (int j = 0; j < 4; ++j) s += E.Ainv[i][j] * E.C[l][j];
      AiCt[i][l] = s;
    }
    long double s = 0;
    for (int j = 0; j < 4; ++j) s += E.Ainv[i][j] * E.B[j];
    AiB[i] = s;
  }
  for (int k = 0; k < 4; ++k) {
    for (int l = 0; l < 4; ++l) {
      long double s = 0;
      for (int i = 0; i < 4; ++i) s += E.C[k][i] * AiCt[i][l];
      E.S[k][l] = s;
    }
    long double s = 0;
    for (int i = 0; i < 4; ++i) s += E.C[k][i] * AiB[i];
    E.r[k] = s;
  }
  E.vol = L.vol;
  for (int k = 0; k < 4; ++k) E.area[k] = L.area[k];
  return ORC_OK;
}

int check_params(const Params* P) {
  if (!P) return fail(ORC_EINVAL, "null params");
  if (!(P->c > 0)) return fail(ORC_ESINGULAR, "reaction coefficient c must be > 0");
  return ORC_OK;
}

// b_D of the face system: |F| u_D(Ct_F) on Dirichlet faces (Section 4.3).
long double face_bD(int64_t nC, const double* X, const int32_t* tri, const Params& P) {
  long double x[3][3];
  for (int m = 0; m < 3; ++m)
    for (int d = 0; d < 3; ++d) x[m][d] = X[d * nC + tri[m]];
  long double u[3], w[3];
  for (int d = 0; d < 3; ++d) {
    u[d] = x[2][d] - x[0][d];
    w[d] = x[1][d] - x[0][d];
  }
  long double cx = u[1] * w[2] - u[2] * w[1], cy = u[2] * w[0] - u[0] * w[2], cz = u[0] * w[1] - u[1] * w[0];
  long double area = 0.5L * sqrtl(cx * cx + cy * cy + cz * cz);
  long double c[3];
  for (int d = 0; d < 3; ++d) c[d] = (x[0][d] + x[1][d] + x[2][d]) / 3.0L;
  return area * fun_eval<long double>(P.ud_kind, P.ud_par, c[0], c[1], c[2]);
}

// Gauss-Legendre nodes/weights on [0,1] by Newton iteration on P_n.
void gauss_legendre01(int n, std::vector<long double>& x, std::vector<long double>& w) {
  x.assign(n, 0);
  w.assign(n, 0);
  for (int i = 0; i < n; ++i) {
    long double z = cosl(PI_L * (i + 0.75L) / (n + 0.5L)), dp = 1;
    for (int it = 0; it < 100; ++it) {
      long double p0 = 1, p1 = z;  // P_0, P_1; after the loop p1 = P_n, p0 = P_{n-1}
      for (int k = 2; k <= n; ++k) {
        long double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1);
      long double dz = p1 / dp;
      z -= dz;
      if (fabsl(dz) < 1e-19L) break;
    }
    x[i] = (1 - z) / 2;
    w[i] = 1 / ((1 - z * z) * dp * dp);  // 2 / ((1 - z^2) P_n'(z)^2), halved for [0, 1]
  }
}

// Collapsed-coordinate (Duffy) product rule on the unit tet {xi,eta,zeta >= 0, sum <= 1}:
// xi = u, eta = v(1-u), zeta = w(1-u)(1-v), Jacobian (1-u)^2 (1-v).  Exact for total
// degree <= 2n-3.
void tet_rule(int n, std::vector<std::array<long double, 4>>& q) {
  std::vector<long double> x, w;
  gauss_legendre01(n, x, w);
  q.clear();
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b)
      for (int c = 0; c < n; ++c) {
        long double u = x[a], v = x[b], s = x[c];
        long double xi = u, eta = v * (1 - u), zeta = s * (1 - u) * (1 - v);
        long double wt = w[a] * w[b] * w[c] * (1 - u) * (1 - u) * (1 - v);
        q.push_back({xi, eta, zeta, wt});
      }
}

// The same collapse on the unit triangle: u, v(1-u), Jacobian (1-u).  Exact for total degree
// <= 2n-2.
void tri_rule(int n, std::vector<std::array<long double, 3>>& q) {
  std::vector<long double> x, w;
  gauss_legendre01(n, x, w);
  q.clear();
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) {
      long double u = x[a], v = x[b];
      q.push_back({u, v * (1 - u), w[a] * w[b] * (1 - u)});
    }
}

// CSR in the face numbering, rows sorted by column, diagonal included.
struct CSR {
  std::vector<int> rowptr, col;
  std::vector<double> val;
};

void csr_matvec(const CSR& A, const std::vector<double>& x, std::vector<double>& y) {
  int n = (int)A.rowptr.size() - 1;
  y.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double s = 0;
    for (int p = A.rowptr[i]; p < A.rowptr[i + 1]; ++p) s += A.val[p] * x[A.col[p]];
    y[i] = s;
  }
}

// Jacobi-preconditioned conjugate gradients, x0 = 0, stop at ||r|| <= tol ||b||.
int pcg(const CSR& A, const std::vector<double>& b, double tol, int maxit, std::vector<double>& x, int* iters,
        double* relres) {
  int n = (int)b.size();
  std::vector<double> dinv(n), r(b), z(n), p(n), q(n);
  for (int i = 0; i < n; ++i) {
    double d = 0;
    for (int k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k)
      if (A.col[k] == i) d = A.val[k];
    if (!(d > 0)) return fail(ORC_ESINGULAR, "non-positive diagonal in face system");
    dinv[i] = 1.0 / d;
  }
  x.assign(n, 0.0);
  double bn = 0;
  for (int i = 0; i < n; ++i) bn += b[i] * b[i];
  bn = std::sqrt(bn);
  if (bn == 0) {
    *iters = 0;
    *relres = 0;
    return ORC_OK;
  }
  double rz = 0;
  for (int i = 0; i < n; ++i) {
    z[i] = r[i] * dinv[i];
    p[i] = z[i];
    rz += r[i] * z[i];
  }
  int it = 0;
  double rn = bn;
  while (it < maxit && rn > tol * bn) {
    csr_matvec(A, p, q);
    double pq = 0;
    for (int i = 0; i < n; ++i) pq += p[i] * q[i];
    double alpha = rz / pq;
    double rr = 0, rzn = 0;
    for (int i = 0; i < n; ++i) {
      x[i] += alpha * p[i];
      r[i] -= alpha * q[i];
      z[i] = r[i] * dinv[i];
      rr += r[i] * r[i];
      rzn += r[i] * z[i];
    }
    double beta = rzn / rz;
    rz = rzn;
    for (int i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
    rn = std::sqrt(rr);
    ++it;
  }
  *iters = it;
  *relres = rn / bn;
  if (rn > tol * bn) return fail(ORC_ENOCONV, "PCG did not converge");
  return ORC_OK;
}

// The face system over the faces not on Gamma_N (the paper's RFaces: Neumann rows and columns
// removed, Section 4.4), numbered in face order; rfaces[f] = its row, or -1 on Gamma_N.
// neumann may be null (every boundary face Dirichlet).
int build_csr(int64_t nC, const double* X, int64_t nE, const int32_t* tet, int64_t nF, const int32_t* tet2face,
              const int8_t* sigma, const int32_t* face2tet, const int32_t* faces, const double* kappa, const Params& P,
              const uint8_t* neumann, CSR& A, std::vector<double>& rhs, std::vector<int>& rfaces) {
  rfaces.assign(nF, -1);
  int64_t L = 0;
  for (int64_t f = 0; f < nF; ++f)
    if (!(neumann && neumann[f])) rfaces[f] = (int)L++;
  std::vector<std::map<int, double>> rows(L);
  rhs.assign(L, 0.0);
  for (int64_t f = 0; f < nF; ++f) {
    if (face2tet[nF + f] < 0 && rfaces[f] >= 0) {
      int tri[3] = {faces[f], faces[nF + f], faces[2 * nF + f]};
      rhs[rfaces[f]] = (double)face_bD(nC, X, tri, P);
    }
  }
  for (int64_t t = 0; t < nE; ++t) {  // tets in order: owners before neighbours
    Elem E;
    int rc = element(nC, X, nE, tet, sigma, kappa, P, t, E, tet2face, neumann);
    if (rc) return rc;
    int F[4];
    for (int k = 0; k < 4; ++k) F[k] = rfaces[tet2face[k * nE + t]];
    for (int k = 0; k < 4; ++k) {
      if (F[k] < 0) continue;
      for (int l = 0; l < 4; ++l)
        if (F[l] >= 0) rows[F[k]][F[l]] += (double)E.S[k][l];
      rhs[F[k]] -= (double)E.r[k];
    }
  }
  A.rowptr.assign(L + 1, 0);
  A.col.clear();
  A.val.clear();
  for (int64_t f = 0; f < L; ++f) {
    for (auto& kv : rows[f]) {
      A.col.push_back(kv.first);
      A.val.push_back(kv.second);
    }
    A.rowptr[f + 1] = (int)A.col.size();
  }
  return ORC_OK;
}

// U(T) = A(T)^-1 (B(T) + C(T)' Lambda(T))   (Algorithm 1, recovery step)
// On Gamma_N the multiplier is not an unknown: its faces contribute LN through B instead.
int recover(int64_t nC, const double* X, int64_t nE, const int32_t* tet, const int32_t* tet2face, const int8_t* sigma,
            const double* kappa, const Params& P, const double* lambda, const double* Bsrc, double* U,
            const uint8_t* neumann = nullptr) {
  for (int64_t t = 0; t < nE; ++t) {
    Elem E;
    int rc = element(nC, X, nE, tet, sigma, kappa, P, t, E, tet2face, neumann);
    if (rc) return rc;
    long double rhsT[4];
    for (int i = 0; i < 4; ++i) {
      long double s = Bsrc ? (long double)Bsrc[i * nE + t] : E.B[i];
      if (lambda)
        for (int k = 0; k < 4; ++k)
          if (!E.neu[k]) s += E.C[k][i] * lambda[tet2face[k * nE + t]];
      rhsT[i] = s;
    }
    for (int i = 0; i < 4; ++i) {
      long double s = 0;
      for (int j = 0; j < 4; ++j) s += E.Ainv[i][j] * rhsT[j];
      U[i * nE + t] = (double)s;
    }
  }
  return ORC_OK;
}

// Per-tet adjoint functional (hand-free: differentiated by dual numbers)
//   Phi_T = P'A U - lambda'C P - P'B - Q'C U + sum_{boundary faces} Q_F b_D,F
// with P, U, lambda, Q held fixed; dJ/dX = -dPhi/dX.
template <class R>
R adjoint_phi(const R x[4][3], long double kappa, const Params& Pm, const int sig[4], const bool bnd[4],
              const long double Pv[4], const long double Uv[4], const long double lam[4], const long double Qv[4]) {
  Local<R> L;
  for (int i = 0; i < 4; ++i)
    for (int d = 0; d < 3; ++d) L.x[i][d] = x[i][d];
  local_geometry(L);
  R A[4][4], K[4][4], C[4][4], B[4];
  local_AC(L, R(kappa), Pm, sig, A, K, C);
  local_load(L, Pm, B);
  R phi(0.0L);
  for (int i = 0; i < 4; ++i) {
    for (int j = 0; j < 4; ++j) phi += R(Pv[i]) * A[i][j] * R(Uv[j]);
    phi -= R(Pv[i]) * B[i];
  }
  for (int k = 0; k < 4; ++k)
    for (int i = 0; i < 4; ++i) phi -= C[k][i] * (R(lam[k]) * R(Pv[i]) + R(Qv[k]) * R(Uv[i]));
  for (int k = 0; k < 4; ++k) {
    if (!bnd[k]) continue;
    const R* x1 = L.x[FACE_V[k][0]];
    const R* x2 = L.x[FACE_V[k][1]];
    const R* x3 = L.x[FACE_V[k][2]];
    R c[3];
    for (int d = 0; d < 3; ++d) c[d] = (x1[d] + x2[d] + x3[d]) / R(3.0L);
    phi += R(Qv[k]) * L.area[k] * fun_eval<R>(Pm.ud_kind, Pm.ud_par, c[0], c[1], c[2]);
  }
  return phi;
}

}  // namespace

// =======================================================================================
extern "C" {

const char* orc_last_error(void) { return g_err.c_str(); }

// NumEdges (Listing 2).  edges: [2][nEd] packed (row stride nEd), capacity 12 nE.
int orc_edges(int64_t nC, int64_t nE, const int32_t* tet, int32_t* edges, int32_t* tet2edge, int32_t* edge_first_tet,
              int32_t* tet_edge_prefix, int64_t* nEd_out) {
  int rc = check_mesh(nC, nE, tet);
  if (rc) return rc;
  EdgeData E;
  build_edges(nE, tet, E);
  int64_t nEd = (int64_t)E.a.size();
  for (int64_t e = 0; e < nEd; ++e) {
    edges[e] = E.a[e];
    edges[nEd + e] = E.b[e];
    if (edge_first_tet) edge_first_tet[e] = E.first_tet[e];
  }
  std::memcpy(tet2edge, E.tet2edge.data(), sizeof(int32_t) * 6 * nE);
  if (tet_edge_prefix) std::memcpy(tet_edge_prefix, E.prefix.data(), sizeof(int32_t) * nE);
  *nEd_out = nEd;
  return ORC_OK;
}

// Edges2Tetra (Listing 3) as sorted (row, col, tet) triplets; capacity 12 nE.
int orc_edges2tetra(int64_t nC, int64_t nE, const int32_t* tet, int32_t* rows, int32_t* cols, int32_t* tets,
                    int64_t* nnz) {
  int rc = check_mesh(nC, nE, tet);
  if (rc) return rc;
  EdgeData E;
  build_edges(nE, tet, E);
  std::map<Key2, int> E2T;
  rc = build_e2t(nE, tet, E, E2T);
  if (rc) return rc;
  int64_t n = 0;
  for (auto& kv : E2T) {
    rows[n] = kv.first.first;
    cols[n] = kv.first.second;
    tets[n] = kv.second;
    ++n;
  }
  *nnz = n;
  return ORC_OK;
}

// FacesUp (Listing 4) + fullFaces.  faces [3][nF], face2tet [2][nF] as slots 4t+k (-1 = none),
// tet2face/sigma/nbr [4][nE].  counts[0] = nF, counts[1] = number of boundary faces.
int orc_faces(int64_t nC, int64_t nE, const int32_t* tet, int32_t* faces, int32_t* tet2face, int8_t* sigma,
              int32_t* face2tet, int32_t* nbr, int64_t* counts) {
  int rc = check_mesh(nC, nE, tet);
  if (rc) return rc;
  EdgeData E;
  build_edges(nE, tet, E);
  std::map<Key2, int> E2T;
  rc = build_e2t(nE, tet, E, E2T);
  if (rc) return rc;
  FaceData F;
  rc = build_faces(nE, tet, E, E2T, F);
  if (rc) return rc;
  int64_t nF = (int64_t)F.tuple.size(), nB = 0;
  for (int64_t f = 0; f < nF; ++f) {
    for (int m = 0; m < 3; ++m) faces[m * nF + f] = F.tuple[f][m];
    face2tet[f] = F.owner_slot[f];
    face2tet[nF + f] = F.nbr_slot[f];
    if (F.nbr_slot[f] < 0) ++nB;
  }
  std::memcpy(tet2face, F.tet2face.data(), sizeof(int32_t) * 4 * nE);
  std::memcpy(sigma, F.sigma.data(), 4 * nE);
  std::memcpy(nbr, F.nbr.data(), sizeof(int32_t) * 4 * nE);
  counts[0] = nF;
  counts[1] = nB;
  return ORC_OK;
}

// Red refinement (Section 3.4).  Every tet gets seven new nodes, its centroid
// (((x_I + x_J) + x_K) + x_L) / 4 and the midpoints (x_a + x_b) / 2 of its six edges; a
// midpoint is shared by all tets holding the edge, a centroid belongs to one tet.  New nodes
// are numbered after the old ones in the order they first occur when the tets are visited in
// order, each tet listing its centroid and then the midpoints of its edges IJ, IK, IL, JK, JL,
// KL (the coordinate-keyed stable unique of the section's construction; in a conforming mesh a
// midpoint is identified by its edge's node pair, a centroid by its tet).  Each tet becomes 12:
// four corner tets (a vertex and the midpoints of its three edges) and the eight tets joining
// the centroid to the faces of the inner octahedron, in the vertex order of CHILD below; child
// 1 keeps row t, children 2..12 go to rows nE + 11 t + (c - 2).  A boundary triangle
// [n1 n2 n3] splits into its three corner triangles and the middle one (SPLIT below), keeping
// its orientation; triangle 1 keeps row f, 2..4 go to rows n + 3 f + (c - 2).
// Xo: [3][nC + nEd + nE] (stride = the new node count); To: [4][12 nE]; dbo/nbo: [3][4 n].
namespace {
// point labels: 0..3 = vertices I J K L, 4 + j = midpoint of local edge j (IJ IK IL JK JL KL),
// 10 = centroid
const int CHILD[12][4] = {{0, 4, 5, 6}, {1, 7, 4, 8}, {2, 5, 7, 9}, {3, 9, 8, 6},   // corner tets
                          {4, 5, 6, 10}, {7, 4, 8, 10}, {5, 7, 9, 10}, {9, 8, 6, 10},
                          {4, 7, 5, 10}, {5, 9, 6, 10}, {4, 6, 8, 10}, {9, 7, 8, 10}};  // octahedron
// triangle labels: 0..2 = n1 n2 n3, 3 = mid(n1 n2), 4 = mid(n2 n3), 5 = mid(n1 n3)
const int SPLIT[4][3] = {{0, 3, 5}, {1, 4, 3}, {2, 5, 4}, {3, 4, 5}};
}  // namespace

int orc_refine(int64_t nC, const double* X, int64_t nE, const int32_t* tet, int64_t nDb, const int32_t* db,
               int64_t nNb, const int32_t* nb, double* Xo, int32_t* To, int32_t* dbo, int32_t* nbo, int64_t* nC_out) {
  int rc = check_mesh(nC, nE, tet);
  if (rc) return rc;
  auto coord = [&](int v, int d) { return X[d * nC + v]; };
  // first-appearance numbering of the new nodes and their coordinates
  std::map<std::pair<int, int>, int64_t> mid_id;  // edge (sorted node pair) -> new node id
  std::vector<int64_t> cent_id(nE);
  std::vector<std::array<double, 3>> newpts;
  std::vector<std::array<int64_t, 11>> label(nE);  // per tet: node id of every point label
  for (int64_t t = 0; t < nE; ++t) {
    int v[4];
    for (int i = 0; i < 4; ++i) v[i] = tet_node(tet, nE, t, i);
    std::array<double, 3> ct;
    for (int d = 0; d < 3; ++d) ct[d] = (((coord(v[0], d) + coord(v[1], d)) + coord(v[2], d)) + coord(v[3], d)) / 4.0;
    cent_id[t] = nC + (int64_t)newpts.size();
    newpts.push_back(ct);
    for (int i = 0; i < 4; ++i) label[t][i] = v[i];
    label[t][10] = cent_id[t];
    for (int j = 0; j < 6; ++j) {
      const int a = v[EDGE_V[j][0]], b = v[EDGE_V[j][1]];
      const std::pair<int, int> key(std::min(a, b), std::max(a, b));
      auto it = mid_id.find(key);
      if (it == mid_id.end()) {
        std::array<double, 3> m;
        for (int d = 0; d < 3; ++d) m[d] = (coord(a, d) + coord(b, d)) / 2.0;
        it = mid_id.emplace(key, nC + (int64_t)newpts.size()).first;
        newpts.push_back(m);
      }
      label[t][4 + j] = it->second;
    }
  }
  const int64_t nCo = nC + (int64_t)newpts.size();
  for (int d = 0; d < 3; ++d) {
    for (int64_t v = 0; v < nC; ++v) Xo[d * nCo + v] = X[d * nC + v];
    for (size_t m = 0; m < newpts.size(); ++m) Xo[d * nCo + nC + (int64_t)m] = newpts[m][d];
  }
  const int64_t nEo = 12 * nE;
  for (int64_t t = 0; t < nE; ++t)
    for (int c = 0; c < 12; ++c) {
      const int64_t row = c == 0 ? t : nE + 11 * t + (c - 1);
      for (int i = 0; i < 4; ++i) To[i * nEo + row] = (int32_t)label[t][CHILD[c][i]];
    }
  auto refine_faces = [&](int64_t n, const int32_t* Fin, int32_t* Fout) -> int {
    const int64_t n4 = 4 * n;
    for (int64_t f = 0; f < n; ++f) {
      const int c3[3] = {Fin[f], Fin[n + f], Fin[2 * n + f]};
      int64_t lab[6] = {c3[0], c3[1], c3[2], -1, -1, -1};
      const int ends[3][2] = {{0, 1}, {1, 2}, {0, 2}};
      for (int m = 0; m < 3; ++m) {
        const int a = c3[ends[m][0]], b = c3[ends[m][1]];
        auto it = mid_id.find(std::pair<int, int>(std::min(a, b), std::max(a, b)));
        if (it == mid_id.end()) return fail(ORC_EINVAL, "boundary face is not a mesh face");
        lab[3 + m] = it->second;
      }
      for (int c = 0; c < 4; ++c) {
        const int64_t row = c == 0 ? f : n + 3 * f + (c - 1);
        for (int m = 0; m < 3; ++m) Fout[m * n4 + row] = (int32_t)lab[SPLIT[c][m]];
      }
    }
    return ORC_OK;
  };
  if (nDb > 0) {
    rc = refine_faces(nDb, db, dbo);
    if (rc) return rc;
  }
  if (nNb > 0) {
    rc = refine_faces(nNb, nb, nbo);
    if (rc) return rc;
  }
  *nC_out = nCo;
  return ORC_OK;
}

// Local matrices of every tet (Listings 6-7, eqs. K(T), M(T), C(T)) and the element Schur
// blocks (eq. schur).  Outputs (any may be null):
//   vol [nE]; K [16][nE] = kappa K(T) row-major; d [4][nE] = sigma_k |F_k|;
//   B [4][nE]; S [16][nE] = C A^-1 C'; r [4][nE] = C A^-1 B.
int orc_local(int64_t nC, const double* X, int64_t nE, const int32_t* tet, const int8_t* sigma, const double* kappa,
              const Params* P, double* vol, double* K, double* d, double* B, double* S, double* r) {
  int rc = check_mesh(nC, nE, tet);
  if (rc) return rc;
  rc = check_params(P);
  if (rc) return rc;
  for (int64_t t = 0; t < nE; ++t) {
    Elem E;
    rc = element(nC, X, nE, tet, sigma, kappa, *P, t, E);
    if (rc) return rc;
    long double kap = kappa ? kappa[t] : P->kappa_const;
    if (vol) vol[t] = (double)E.vol;
    for (int k = 0; k < 4; ++k) {
      if (d) d[k * nE + t] = (double)((sigma ? sigma[k * nE + t] : 1) * E.area[k]);
      if (B) B[k * nE + t] = (double)E.B[k];
      if (r) r[k * nE + t] = (double)E.r[k];
      for (int l = 0; l < 4; ++l) {
        if (K) K[(4 * k + l) * nE + t] = (double)(kap * E.K[k][l]);
        if (S) S[(4 * k + l) * nE + t] = (double)E.S[k][l];
      }
    }
  }
  return ORC_OK;
}

// Condensed face system (Algorithm 1 / Listing 8 assembly): full CSR (diagonal included,
// columns ascending), S+ = sum_T P_T' S(T) P_T, rhs = b_D - sum_T P_T' r(T).
// Capacities: col/val 7 nF.  nnz_out = number of stored entries.
int orc_condense(int64_t nC, const double* X, int64_t nE, const int32_t* tet, int64_t nF, const int32_t* tet2face,
                 const int8_t* sigma, const int32_t* face2tet, const int32_t* faces, const double* kappa,
                 const Params* P, const uint8_t* neumann, int32_t* rowptr, int32_t* col, double* val, double* rhs,
                 int32_t* rfaces, int64_t* nnz_out, int64_t* L_out) {
  int rc = check_mesh(nC, nE, tet);
  if (rc) return rc;
  rc = check_params(P);
  if (rc) return rc;
  CSR A;
  std::vector<double> b;
  std::vector<int> rf;
  rc = build_csr(nC, X, nE, tet, nF, tet2face, sigma, face2tet, faces, kappa, *P, neumann, A, b, rf);
  if (rc) return rc;
  const int64_t L = (int64_t)b.size();
  std::memcpy(rowptr, A.rowptr.data(), sizeof(int32_t) * (L + 1));
  std::memcpy(col, A.col.data(), sizeof(int32_t) * A.col.size());
  std::memcpy(val, A.val.data(), sizeof(double) * A.val.size());
  std::memcpy(rhs, b.data(), sizeof(double) * L);
  if (rfaces) std::memcpy(rfaces, rf.data(), sizeof(int32_t) * nF);
  *nnz_out = (int64_t)A.col.size();
  if (L_out) *L_out = L;
  return ORC_OK;
}

// Face solve with Jacobi-PCG on a full CSR.  stats: iterations and final relative residual.
int orc_pcg(int64_t n, const int32_t* rowptr, const int32_t* col, const double* val, const double* rhs, double tol,
            int32_t maxit, double* x, int32_t* iters, double* relres) {
  CSR A;
  A.rowptr.assign(rowptr, rowptr + n + 1);
  A.col.assign(col, col + rowptr[n]);
  A.val.assign(val, val + rowptr[n]);
  std::vector<double> b(rhs, rhs + n), xv;
  int it = 0;
  double rr = 0;
  int rc = pcg(A, b, tol, maxit, xv, &it, &rr);
  std::memcpy(x, xv.data(), sizeof(double) * n);
  *iters = it;
  *relres = rr;
  return rc;
}

// Recovery U(T) = A(T)^-1 (B(T) + C(T)' Lambda(T)).  U: [4][nE].
int orc_recover(int64_t nC, const double* X, int64_t nE, const int32_t* tet, const int32_t* tet2face,
                const int8_t* sigma, const double* kappa, const Params* P, const uint8_t* neumann,
                const double* lambda, double* U) {
  int rc = check_mesh(nC, nE, tet);
  if (rc) return rc;
  rc = check_params(P);
  if (rc) return rc;
  return recover(nC, X, nE, tet, tet2face, sigma, kappa, *P, lambda, nullptr, U, neumann);
}

// Brute force: the full (N+L) block system of eq. (VectorForm)
//   [K+M  -C'; -C  0] [U; Lambda] = [b + LN; -b_D]
// assembled dense and solved by LU with partial pivoting in long double.  Tiny meshes only.
// Faces on Gamma_N carry no multiplier: their rows are lambda_F = 0 and couple to nothing.
int orc_dense_solve(int64_t nC, const double* X, int64_t nE, const int32_t* tet, int64_t nF, const int32_t* tet2face,
                    const int8_t* sigma, const int32_t* face2tet, const int32_t* faces, const double* kappa,
                    const Params* P, const uint8_t* neumann, double* U, double* lambda) {
  int rc = check_mesh(nC, nE, tet);
  if (rc) return rc;
  rc = check_params(P);
  if (rc) return rc;
  int64_t N = 4 * nE, L = nF, n = N + L;
  if (n > 6000) return fail(ORC_EINVAL, "dense solve is for tiny meshes only");
  std::vector<long double> M(n * n, 0.0L), rhs(n, 0.0L);
  for (int64_t t = 0; t < nE; ++t) {
    Elem E;
    rc = element(nC, X, nE, tet, sigma, kappa, *P, t, E, tet2face, neumann);
    if (rc) return rc;
    for (int i = 0; i < 4; ++i) {
      for (int j = 0; j < 4; ++j) M[(4 * t + i) * n + 4 * t + j] += E.A[i][j];
      rhs[4 * t + i] += E.B[i];
      for (int k = 0; k < 4; ++k) {
        if (E.neu[k]) continue;
        int64_t f = tet2face[k * nE + t];
        M[(4 * t + i) * n + N + f] -= E.C[k][i];
        M[(N + f) * n + 4 * t + i] -= E.C[k][i];
      }
    }
  }
  for (int64_t f = 0; f < nF; ++f)
    if (neumann && neumann[f]) M[(N + f) * n + N + f] = 1.0L;
  for (int64_t f = 0; f < nF; ++f)
    if (face2tet[nF + f] < 0 && !(neumann && neumann[f])) {
      int tri[3] = {faces[f], faces[nF + f], faces[2 * nF + f]};
      rhs[N + f] = -face_bD(nC, X, tri, *P);
    }
  std::vector<int64_t> perm(n);
  for (int64_t i = 0; i < n; ++i) perm[i] = i;
  for (int64_t c = 0; c < n; ++c) {
    int64_t piv = c;
    for (int64_t r = c + 1; r < n; ++r)
      if (fabsl(M[r * n + c]) > fabsl(M[piv * n + c])) piv = r;
    if (M[piv * n + c] == 0) return fail(ORC_ESINGULAR, "singular block system");
    if (piv != c) {
      for (int64_t j = 0; j < n; ++j) std::swap(M[piv * n + j], M[c * n + j]);
      std::swap(rhs[piv], rhs[c]);
    }
    for (int64_t r = c + 1; r < n; ++r) {
      long double f = M[r * n + c] / M[c * n + c];
      if (f == 0) continue;
      for (int64_t j = c; j < n; ++j) M[r * n + j] -= f * M[c * n + j];
      rhs[r] -= f * rhs[c];
    }
  }
  std::vector<long double> x(n);
  for (int64_t r = n - 1; r >= 0; --r) {
    long double s = rhs[r];
    for (int64_t j = r + 1; j < n; ++j) s -= M[r * n + j] * x[j];
    x[r] = s / M[r * n + r];
  }
  for (int64_t t = 0; t < nE; ++t)
    for (int i = 0; i < 4; ++i) U[i * nE + t] = (double)x[4 * t + i];
  for (int64_t f = 0; f < nF; ++f) lambda[f] = (double)x[N + f];
  return ORC_OK;
}

// Adjoint of J with dJ/dU = gbar (U [4][nE] is the forward solution, lambda its multiplier):
//   S+ Q = -C A^-1 gbar,  P = A^-1 (gbar + C'Q),
//   dJ/dlog kappa_T = -kappa_T P_T' K_T U_T,
//   dJ/dX = -d/dX [ P'A U - lambda'C P - P'B - Q'C U + Q'b_D ]   (P, U, lambda, Q fixed),
// the coordinate derivative taken per tet with dual numbers.  Outputs (any may be null):
// dlogk [nE], dX [3][nC], Q [nF], Pout [4][nE].
int orc_adjoint(int64_t nC, const double* X, int64_t nE, const int32_t* tet, int64_t nF, const int32_t* tet2face,
                const int8_t* sigma, const int32_t* face2tet, const int32_t* faces, const double* kappa,
                const Params* Pm, const double* U, const double* lambda, const double* gbar, double tol, int32_t maxit,
                double* dlogk, double* dX, double* Qout, double* Pout, int32_t* iters) {
  int rc = check_mesh(nC, nE, tet);
  if (rc) return rc;
  rc = check_params(Pm);
  if (rc) return rc;
  CSR A;
  std::vector<double> b;
  std::vector<int> rf;
  rc = build_csr(nC, X, nE, tet, nF, tet2face, sigma, face2tet, faces, kappa, *Pm, nullptr, A, b, rf);
  if (rc) return rc;
  // adjoint right-hand side -C A^-1 gbar
  std::vector<double> w(4 * nE), radj(nF, 0.0);
  Params P0 = *Pm;
  rc = recover(nC, X, nE, tet, tet2face, sigma, kappa, P0, nullptr, gbar, w.data());
  if (rc) return rc;
  for (int64_t t = 0; t < nE; ++t) {
    Elem E;
    rc = element(nC, X, nE, tet, sigma, kappa, *Pm, t, E);
    if (rc) return rc;
    for (int k = 0; k < 4; ++k) {
      long double s = 0;
      for (int i = 0; i < 4; ++i) s += E.C[k][i] * w[i * nE + t];
      radj[tet2face[k * nE + t]] -= (double)s;
    }
  }
  std::vector<double> Q;
  int it = 0;
  double rr = 0;
  rc = pcg(A, radj, tol, maxit, Q, &it, &rr);
  if (iters) *iters = it;
  if (rc) return rc;
  std::vector<double> Pv(4 * nE);
  rc = recover(nC, X, nE, tet, tet2face, sigma, kappa, P0, Q.data(), gbar, Pv.data());
  if (rc) return rc;
  if (Qout) std::memcpy(Qout, Q.data(), sizeof(double) * nF);
  if (Pout) std::memcpy(Pout, Pv.data(), sizeof(double) * 4 * nE);
  if (dX)
    for (int64_t i = 0; i < 3 * nC; ++i) dX[i] = 0;
  for (int64_t t = 0; t < nE; ++t) {
    long double kap = kappa ? kappa[t] : Pm->kappa_const;
    long double Pt[4], Ut[4], lt[4], Qt[4];
    int sig[4];
    bool bnd[4];
    for (int i = 0; i < 4; ++i) {
      Pt[i] = Pv[i * nE + t];
      Ut[i] = U[i * nE + t];
    }
    for (int k = 0; k < 4; ++k) {
      int f = tet2face[k * nE + t];
      lt[k] = lambda[f];
      Qt[k] = Q[f];
      sig[k] = sigma[k * nE + t];
      bnd[k] = face2tet[nF + f] < 0;
    }
    if (dlogk) {
      Elem E;
      rc = element(nC, X, nE, tet, sigma, kappa, *Pm, t, E);
      if (rc) return rc;
      long double s = 0;
      for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) s += Pt[i] * E.K[i][j] * Ut[j];
      dlogk[t] = (double)(-kap * s);
    }
    if (dX) {
      long double xb[4][3];
      int v[4];
      for (int i = 0; i < 4; ++i) {
        v[i] = tet_node(tet, nE, t, i);
        for (int d = 0; d < 3; ++d) xb[i][d] = X[d * nC + v[i]];
      }
      for (int i = 0; i < 4; ++i)
        for (int d = 0; d < 3; ++d) {
          Dual x[4][3];
          for (int a = 0; a < 4; ++a)
            for (int e = 0; e < 3; ++e) x[a][e] = Dual(xb[a][e], (a == i && e == d) ? 1.0L : 0.0L);
          Dual phi = adjoint_phi<Dual>(x, kap, *Pm, sig, bnd, Pt, Ut, lt, Qt);
          dX[d * nC + v[i]] -= (double)phi.d;
        }
    }
  }
  return ORC_OK;
}

// Error norms against an exact solution u (kind/params): out[0] = sum_T ||grad(u-u_h)||^2,
// out[1] = sum_T ||u-u_h||^2, out[2] = sum_T h sum_{F in dT \ Gamma_N} ||kappa grad u . nu_F - lambda_F||^2_F
// (nu_F: outward normal of the face's owner; the h-norm of eq. (eMnorm) without the root).
// With out[0..2], ||u - u_h||_Y = sqrt(out[0] + out[1] / h^2) and ||kappa - kappa_h||_h = sqrt(out[2]).
// Quadrature: collapsed Gauss-Legendre product rules with nq points per direction.
int orc_errors(int64_t nC, const double* X, int64_t nE, const int32_t* tet, const int32_t* tet2face,
               const int8_t* sigma, const double* kappa, const Params* P, const uint8_t* neumann, const double* U,
               const double* lambda, int32_t u_kind, const double* u_par, double h, int32_t nq, double* out) {
  int rc = check_mesh(nC, nE, tet);
  if (rc) return rc;
  std::vector<std::array<long double, 4>> qt;
  std::vector<std::array<long double, 3>> qf;
  tet_rule(nq, qt);
  tri_rule(nq, qf);
  long double e_grad = 0, e_l2 = 0, e_lam = 0;
  for (int64_t t = 0; t < nE; ++t) {
    Local<long double> L;
    rc = load_tet(nC, X, nE, tet, t, L);
    if (rc) return rc;
    long double kap = kappa ? kappa[t] : P->kappa_const;
    long double Ut[4], guh[3] = {0, 0, 0};
    for (int i = 0; i < 4; ++i) {
      Ut[i] = U[i * nE + t];
      for (int d = 0; d < 3; ++d) guh[d] += Ut[i] * L.g[i][d];
    }
    for (auto& q : qt) {
      long double lam[4] = {1 - q[0] - q[1] - q[2], q[0], q[1], q[2]};
      long double x[3] = {0, 0, 0};
      long double uh = 0;
      for (int i = 0; i < 4; ++i) {
        uh += lam[i] * Ut[i];
        for (int d = 0; d < 3; ++d) x[d] += lam[i] * L.x[i][d];
      }
      long double w = q[3] * fabsl(L.detP);
      long double u = fun_eval<long double>(u_kind, u_par, x[0], x[1], x[2]);
      long double gu[3];
      fun_grad(u_kind, u_par, x[0], x[1], x[2], gu);
      long double dg = 0;
      for (int d = 0; d < 3; ++d) dg += (gu[d] - guh[d]) * (gu[d] - guh[d]);
      e_grad += w * dg;
      e_l2 += w * (u - uh) * (u - uh);
    }
    for (int k = 0; k < 4; ++k) {
      if (neumann && neumann[tet2face[k * nE + t]]) continue;  // the h-norm runs over dT \ Gamma_N
      const long double* x1 = L.x[FACE_V[k][0]];
      const long double* x2 = L.x[FACE_V[k][1]];
      const long double* x3 = L.x[FACE_V[k][2]];
      // outward normal of this tet on face k, flipped to the owner's orientation by sigma
      long double nrm[3];
      long double a[3], b[3];
      for (int d = 0; d < 3; ++d) {
        a[d] = x2[d] - x1[d];
        b[d] = x3[d] - x1[d];
      }
      nrm[0] = a[1] * b[2] - a[2] * b[1];
      nrm[1] = a[2] * b[0] - a[0] * b[2];
      nrm[2] = a[0] * b[1] - a[1] * b[0];
      long double nl = sqrtl(nrm[0] * nrm[0] + nrm[1] * nrm[1] + nrm[2] * nrm[2]);
      // make it point away from the opposite vertex
      int opp = 6 - FACE_V[k][0] - FACE_V[k][1] - FACE_V[k][2];
      long double s = 0;
      for (int d = 0; d < 3; ++d) s += nrm[d] * (L.x[opp][d] - x1[d]);
      long double sgn = (s > 0 ? -1.0L : 1.0L) * sigma[k * nE + t];
      for (int d = 0; d < 3; ++d) nrm[d] *= sgn / nl;
      long double area = L.area[k];
      long double lh = lambda[tet2face[k * nE + t]];
      for (auto& q : qf) {
        long double x[3];
        for (int d = 0; d < 3; ++d) x[d] = x1[d] + q[0] * (x2[d] - x1[d]) + q[1] * (x3[d] - x1[d]);
        long double gu[3];
        fun_grad(u_kind, u_par, x[0], x[1], x[2], gu);
        long double le = kap * (gu[0] * nrm[0] + gu[1] * nrm[1] + gu[2] * nrm[2]);
        e_lam += h * 2 * area * q[2] * (le - lh) * (le - lh);
      }
    }
  }
  out[0] = (double)e_grad;
  out[1] = (double)e_l2;
  out[2] = (double)e_lam;
  return ORC_OK;
}

// Quadrature rule on the unit tet (for pinning the rule itself): pts [3][m], wts [m], m = n^3.
int orc_tet_rule(int32_t n, double* pts, double* wts) {
  std::vector<std::array<long double, 4>> q;
  tet_rule(n, q);
  int64_t m = (int64_t)q.size();
  for (int64_t i = 0; i < m; ++i) {
    for (int d = 0; d < 3; ++d) pts[d * m + i] = (double)q[i][d];
    wts[i] = (double)q[i][3];
  }
  return ORC_OK;
}

// Quadrature rule on the unit triangle {u, v >= 0, u + v <= 1} (for pinning the rule itself):
// pts [2][m], wts [m], m = n^2.
int orc_tri_rule(int32_t n, double* pts, double* wts) {
  std::vector<std::array<long double, 3>> q;
  tri_rule(n, q);
  int64_t m = (int64_t)q.size();
  for (int64_t i = 0; i < m; ++i) {
    for (int d = 0; d < 2; ++d) pts[d * m + i] = (double)q[i][d];
    wts[i] = (double)q[i][2];
  }
  return ORC_OK;
}

}  // extern "C"
