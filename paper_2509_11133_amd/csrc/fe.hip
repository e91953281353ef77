// Local matrices, element Schur complement and condensed face system (Sections 4.2-4.6,
// Algorithm 1), the matrix-free FP64 recovery / residual, and the adjoint VJP.
//
// Element algebra (one tet, R = double or float):
//   A = kappa K + c M with K = vol g_i.g_j and M = c vol/20 (1 + delta_ij).  K 1 = 0 and
//   M 1 = vol/4 1, so 1 is an eigenvector of A with eigenvalue c vol/4 and
//       A^-1 = 1 1' / (c vol) + W,   W = (A restricted to 1-perp)^-1  (W 1 = 0).
//   W is formed in the orthonormal basis q1 = (1,1,-1,-1)/2, q2 = (1,-1,1,-1)/2,
//   q3 = (1,-1,-1,1)/2 of 1-perp: N = kappa vol Gh Gh' + (c vol/20) I_3 with Gh = Q'G
//   (3x3 SPD, conditioned like the tet's shape), W = Q N^-1 Q'.
//   C row k = d_k r_k with d_k = sigma_k |F_k| and r_k = (1 1' - Pi)/3 row k, Pi the
//   face -> opposite-vertex permutation; with W 1 = 0 this gives
//       S_kl = d_k d_l (1/(c vol) + W[opp k][opp l] / 9),
//       r_k  = d_k (sum B / (c vol) - (W B)[opp k] / 3),
//       U    = 1 (sum B + sum mu) / (c vol) + W (B - Pi' mu / 3),   mu_k = d_k lambda_k.
//   This split keeps the FP32 path accurate: A itself has cond ~ h^-2, N does not.
#include <climits>

#include "common.hpp"

namespace ph {

constexpr int FT = 256;

template <class R>
struct Elem {
  double det, vol;  // FP64 in both precisions
  R g[4][3];        // barycentric gradients
  R d[4];           // sigma_k |F_k|
  R W[4][4];
  R icv;            // 1 / (c vol)
  R kappa, c;

  // x: vertex coordinates (FP64).  Returns false for a zero-volume tet; its d (and with it
  // every S_kl and r_k) is then zero and the other members are finite placeholders.
  __device__ __forceinline__ bool init(const double x[4][3], double kap, double cc, const int sig[4]) {
    double v[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int e = 0; e < 3; ++e) v[i][e] = x[i + 1][e] - x[0][e];
    det = v[0][0] * (v[1][1] * v[2][2] - v[1][2] * v[2][1]) - v[0][1] * (v[1][0] * v[2][2] - v[1][2] * v[2][0]) +
          v[0][2] * (v[1][0] * v[2][1] - v[1][1] * v[2][0]);
    const bool ok = det != 0.0;
    if (!ok) det = 1.0;
    vol = fabs(det) * (1.0 / 6.0);
    kappa = (R)kap;
    c = (R)cc;
    R w[4][3];  // vertex positions relative to vertex 0
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      w[0][e] = (R)0;
      w[1][e] = (R)v[0][e];
      w[2][e] = (R)v[1][e];
      w[3][e] = (R)v[2][e];
    }
    const R idet = (R)(1.0 / det);
    // g_b = (v2 x v3)/det, g_c = (v3 x v1)/det, g_d = (v1 x v2)/det, g_a = -(g_b + g_c + g_d)
#pragma unroll
    for (int i = 1; i < 4; ++i) {
      const R* p = w[i == 1 ? 2 : (i == 2 ? 3 : 1)];
      const R* q = w[i == 1 ? 3 : (i == 2 ? 1 : 2)];
      g[i][0] = (p[1] * q[2] - p[2] * q[1]) * idet;
      g[i][1] = (p[2] * q[0] - p[0] * q[2]) * idet;
      g[i][2] = (p[0] * q[1] - p[1] * q[0]) * idet;
    }
#pragma unroll
    for (int e = 0; e < 3; ++e) g[0][e] = -(g[1][e] + g[2][e] + g[3][e]);
    // face k lies opposite vertex opp(k), and |grad lambda_i| = |F_i| / (3 |T|), so
    // |F_k| = 3 |T| |g_opp(k)|
    const R v3 = ok ? (R)(3.0 * vol) : (R)0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const R* gk = g[opp(k)];
      d[k] = (R)sig[k] * v3 * sqrt(gk[0] * gk[0] + gk[1] * gk[1] + gk[2] * gk[2]);
    }
    // W = Q N^-1 Q'
    R gh[3][3];
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      gh[0][e] = (R)0.5 * (g[0][e] + g[1][e] - g[2][e] - g[3][e]);
      gh[1][e] = (R)0.5 * (g[0][e] - g[1][e] + g[2][e] - g[3][e]);
      gh[2][e] = (R)0.5 * (g[0][e] - g[1][e] - g[2][e] + g[3][e]);
    }
    const R kv = kappa * (R)vol, mv = c * (R)vol * (R)(1.0 / 20.0);
    R N[3][3];
#pragma unroll
    for (int m = 0; m < 3; ++m)
#pragma unroll
      for (int n = m; n < 3; ++n) {
        R s = kv * (gh[m][0] * gh[n][0] + gh[m][1] * gh[n][1] + gh[m][2] * gh[n][2]);
        if (m == n) s += mv;
        N[m][n] = s;
        N[n][m] = s;
      }
    R A00 = N[1][1] * N[2][2] - N[1][2] * N[2][1];
    R A01 = N[0][2] * N[2][1] - N[0][1] * N[2][2];
    R A02 = N[0][1] * N[1][2] - N[0][2] * N[1][1];
    R A11 = N[0][0] * N[2][2] - N[0][2] * N[2][0];
    R A12 = N[0][2] * N[1][0] - N[0][0] * N[1][2];
    R A22 = N[0][0] * N[1][1] - N[0][1] * N[1][0];
    R idn = (R)1 / (N[0][0] * A00 + N[0][1] * (N[1][2] * N[2][0] - N[1][0] * N[2][2]) +
                    N[0][2] * (N[1][0] * N[2][1] - N[1][1] * N[2][0]));
    R Ni[3][3] = {{A00 * idn, A01 * idn, A02 * idn},
                  {A01 * idn, A11 * idn, A12 * idn},
                  {A02 * idn, A12 * idn, A22 * idn}};
    // Y = Q Ni (4x3), q_m[i] = 0.5 * sign pattern
    const int sg[3][4] = {{1, 1, -1, -1}, {1, -1, 1, -1}, {1, -1, -1, 1}};
    R Y[4][3];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int n = 0; n < 3; ++n) {
        R s = (R)0;
#pragma unroll
        for (int m = 0; m < 3; ++m) s += sg[m][i] > 0 ? Ni[m][n] : -Ni[m][n];
        Y[i][n] = (R)0.5 * s;
      }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = i; j < 4; ++j) {
        R s = (R)0;
#pragma unroll
        for (int n = 0; n < 3; ++n) s += sg[n][j] > 0 ? Y[i][n] : -Y[i][n];
        W[i][j] = (R)0.5 * s;
        W[j][i] = W[i][j];
      }
    icv = (R)(1.0 / (cc * vol));
    return ok;
  }

  // the 10 distinct entries of the symmetric S(T), row-major upper triangle
  __device__ __forceinline__ void Supper(R s[10]) const {
    int n = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int l = k; l < 4; ++l) s[n++] = S(k, l);
  }

  __device__ __forceinline__ R S(int k, int l) const {
    return d[k] * d[l] * (icv + W[opp(k)][opp(l)] * (R)(1.0 / 9.0));
  }

  // r_k = (C A^-1 y)_k for a load-like vector y
  __device__ __forceinline__ void CAinv(const R y[4], R r[4]) const {
    R sy = (y[0] + y[1]) + (y[2] + y[3]);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int o = opp(k);
      R wy = W[o][0] * y[0] + W[o][1] * y[1] + W[o][2] * y[2] + W[o][3] * y[3];
      r[k] = d[k] * (sy * icv - wy * (R)(1.0 / 3.0));
    }
  }
};

// load vector of one tet (StiffMassPH's face-centroid rule or b = M f(x_i)); the points are
// formed in the working precision R
template <class R>
__device__ __forceinline__ void load_vec(const double x[4][3], double vol, const DevParams& P, R B[4]) {
  R xr[4][3];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int e = 0; e < 3; ++e) xr[i][e] = (R)x[i][e];
  if (P.quad == PHFEM_QUAD_P1_INTERP) {
    R f[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) f[i] = fun_at<R>(P.fk, P.fp, xr[i][0], xr[i][1], xr[i][2]);
    R sf = (f[0] + f[1]) + (f[2] + f[3]);
#pragma unroll
    for (int i = 0; i < 4; ++i) B[i] = (R)vol * (R)(1.0 / 20.0) * (sf + f[i]);
    return;
  }
  R fc[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int a = fv(k, 0), b = fv(k, 1), c = fv(k, 2);
    R cx = (xr[a][0] + xr[b][0] + xr[c][0]) * (R)(1.0 / 3.0);
    R cy = (xr[a][1] + xr[b][1] + xr[c][1]) * (R)(1.0 / 3.0);
    R cz = (xr[a][2] + xr[b][2] + xr[c][2]) * (R)(1.0 / 3.0);
    fc[k] = fun_at<R>(P.fk, P.fp, cx, cy, cz);
  }
  // vertex i lies on the three faces other than the one opposite it (opp(i))
  const R w = (R)vol * (R)(1.0 / 12.0);
#pragma unroll
  for (int i = 0; i < 4; ++i) B[i] = w * (((fc[0] + fc[1]) + (fc[2] + fc[3])) - fc[opp(i)]);
}

// AoS copy of the coordinates, one 32-byte (x, y, z, 0) record per node: a tet's gather
// then touches 4 cache lines instead of 12

__device__ __forceinline__ void gather_xa(const double4* __restrict__ XA, const int v[4], double x[4][3]) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const double4 p = XA[v[i]];
    x[i][0] = p.x;
    x[i][1] = p.y;
    x[i][2] = p.z;
  }
}

__device__ __forceinline__ void gather_x(int64_t nC, const double* __restrict__ X, const int v[4], double x[4][3]) {
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int e = 0; e < 3; ++e) x[i][e] = X[e * nC + v[i]];
}

// Neumann flux at the centroid of local face k: kappa grad(u_g) . nu, nu the outward unit
// normal = -grad(lambda_opp(k)) / |grad(lambda_opp(k))| (the barycentric coordinate of the
// opposite vertex grows inward).  LN adds |F_k| g / 3 to the three vertices of face k, which
// is d_k g / 3 with d_k = |F_k| on a boundary face (sigma = +1).
template <class R>
__device__ __forceinline__ double neumann_flux(const Elem<R>& E, const double x[4][3], int k, double kap,
                                               const DevParams& P) {
  const int a = fv(k, 0), b = fv(k, 1), c = fv(k, 2), o = opp(k);
  const double g0 = (double)E.g[o][0], g1 = (double)E.g[o][1], g2 = (double)E.g[o][2];
  const double gl = sqrt(g0 * g0 + g1 * g1 + g2 * g2);
  double gu[3];
  fun_grad(P.gk, P.gp, (x[a][0] + x[b][0] + x[c][0]) / 3.0, (x[a][1] + x[b][1] + x[c][1]) / 3.0,
           (x[a][2] + x[b][2] + x[c][2]) / 3.0, gu);
  return -kap * (gu[0] * g0 + gu[1] * g1 + gu[2] * g2) / gl;
}

// ---------------------------------------------------------------- assemble (inspection)
template <class R>
__global__ __launch_bounds__(FT) void k_assemble(int64_t nC, const double* __restrict__ X, int64_t nE,
                                                 const int32_t* __restrict__ tet, const int8_t* __restrict__ sigma,
                                                 const double* __restrict__ kappa, DevParams P, double* vol,
                                                 double* K, double* dd, double* Bo, double* So, double* ro) {
  int64_t t = (int64_t)blockIdx.x * FT + threadIdx.x;
  if (t >= nE) return;
  int v[4], sig[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    v[i] = tet[i * nE + t];
    sig[i] = sigma ? sigma[i * nE + t] : 1;
  }
  double x[4][3];
  gather_x(nC, X, v, x);
  const double kap = kappa ? kappa[t] : P.kc;
  Elem<R> E;
  if (!E.init(x, kap, P.c, sig)) return;
  R B[4], r[4];
  load_vec<R>(x, E.vol, P, B);
  E.CAinv(B, r);
  if (vol) vol[t] = E.vol;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (dd) dd[k * nE + t] = (double)E.d[k];
    if (Bo) Bo[k * nE + t] = (double)B[k];
    if (ro) ro[k * nE + t] = (double)r[k];
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      if (K)
        K[(4 * k + l) * nE + t] =
            (double)(E.kappa * (R)E.vol * (E.g[k][0] * E.g[l][0] + E.g[k][1] * E.g[l][1] + E.g[k][2] * E.g[l][2]));
      if (So) So[(4 * k + l) * nE + t] = (double)E.S(k, l);
    }
  }
}

// ---------------------------------------------------------------- condense
// per face: off-diagonal count (6 interior, 3 boundary) for the row-pointer scan, diagonal
// cleared, rhs = b_D on boundary faces (|F| u_D(centroid)), 0 inside.
__global__ __launch_bounds__(FT) void k_face_init(int64_t nF, int64_t nC, const double* __restrict__ X,
                                                  const int32_t* __restrict__ faces,
                                                  const int32_t* __restrict__ face2tet, DevParams P,
                                                  uint32_t* __restrict__ cnt, double* __restrict__ diag,
                                                  double* __restrict__ rhs, int* __restrict__ flags) {
  int64_t f = (int64_t)blockIdx.x * FT + threadIdx.x;
  if (f > nF) return;
  if (f == nF) {
    if (cnt) cnt[nF] = 0;
    return;
  }
  const bool interior = face2tet[nF + f] >= 0;
  if (cnt) cnt[f] = interior ? 6u : 3u;
  if (diag) diag[f] = 0.0;
  if (!rhs) return;
  double b = 0.0;
  if (!interior && P.uk != PHFEM_FUN_ZERO && !(P.nm && P.nm[f])) {
    double x[3][3];
    bool inr = true;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      int v = faces[m * nF + f];
      if ((uint32_t)v >= (uint64_t)nC) {
        inr = false;
        v = 0;
      }
#pragma unroll
      for (int e = 0; e < 3; ++e) x[m][e] = X[e * nC + v];
    }
    if (!inr && flags) atomicOr(flags, DEV_BADNODE);
    double u0 = x[2][0] - x[0][0], u1 = x[2][1] - x[0][1], u2 = x[2][2] - x[0][2];
    double s0 = x[1][0] - x[0][0], s1 = x[1][1] - x[0][1], s2 = x[1][2] - x[0][2];
    double n0 = u1 * s2 - u2 * s1, n1 = u2 * s0 - u0 * s2, n2 = u0 * s1 - u1 * s0;
    double area = 0.5 * sqrt(n0 * n0 + n1 * n1 + n2 * n2);
    double cx = (x[0][0] + x[1][0] + x[2][0]) / 3.0, cy = (x[0][1] + x[1][1] + x[2][1]) / 3.0,
           cz = (x[0][2] + x[1][2] + x[2][2]) / 3.0;
    b = area * fun_at<double>(P.uk, P.up, cx, cy, cz);
  }
  rhs[f] = b;
}

// Condensation (no atomics), tiles of CT consecutive tets (the workgroup).  A face is numbered
// at its owner (lowest tet index), so the faces owned by a tile's tets form one contiguous id
// range, and in the meshes the refinement produces about three quarters of the interior
// faces have their second tet in the owner's tile as well (siblings are numbered close
// together).  Two passes:
//  k_cond_cross: every tet computes its element block; a tet whose face is owned by a tet of
//                another tile writes that face's row of its block (S_kk, (C A^-1 B)_k, the
//                three S_kl and their face ids) as a 32-byte record at slot 4t+k;
//  k_cond_tile:  the tile recomputes its tets' blocks into LDS and writes the rows of the
//                faces it owns: owner's row and, for the second tet, its row from LDS when it
//                lies in the tile, else its record; off-diagonals sorted by column, diagonal
//                S_owner + S_neighbour and rhs (b_D - r_owner) - r_neighbour in that order.
// The element arithmetic is done twice (it is cheap next to the memory traffic); what
// crosses HBM is the input once per pass, one record per cross-tile face and the rows.
// Neumann faces (params.neumann): LN in the load, the face's row becomes lambda_F = g (S_kk
// = 1, r_k = -g, no coupling), and its coupling entries in every other row are zero (S_kl =
// S_lk = 0), the paper's system over the other faces without renumbering.

// position of S_kl (either order) in the row-major upper triangle of a 4x4 matrix
__host__ __device__ constexpr int uidx(int k, int l) {
  return k <= l ? (k * (7 - k)) / 2 + l : (l * (7 - l)) / 2 + k;
}
static_assert(uidx(0, 0) == 0 && uidx(0, 3) == 3 && uidx(1, 1) == 4 && uidx(2, 1) == 5 && uidx(2, 2) == 7 &&
                  uidx(3, 3) == 9,
              "upper-triangle index");

constexpr int CT = 256;  // tets per tile = threads per workgroup of both passes

template <class R>
struct SlotRec {  // row k of one tet's element Schur block S(T) and (C A^-1 B)_k
  R d;            // S_kk
  R r;            // (C A^-1 B)_k
  R o[3];         // S_kl for the three l != k, ascending l
  int32_t c[3];   // face ids of those three l
};
static_assert(sizeof(SlotRec<float>) == 32 && sizeof(SlotRec<double>) == 56, "packed slot records");

// a record as whole 16-byte stores (32 B in FP32, 56 B in FP64)
template <class R>
__device__ __forceinline__ void store_rec(SlotRec<R>* p, const SlotRec<R>& q) {
  constexpr int W = sizeof(SlotRec<R>) / 8;
  union {
    SlotRec<R> rec;
    uint2 w[W];
  } u;
  u.rec = q;
  uint2* d = reinterpret_cast<uint2*>(p);
  if (W % 2 == 0) {
#pragma unroll
    for (int m = 0; m < W; m += 2)
      *reinterpret_cast<uint4*>(d + m) = make_uint4(u.w[m].x, u.w[m].y, u.w[m + 1].x, u.w[m + 1].y);
  } else {
#pragma unroll
    for (int m = 0; m < W; ++m) d[m] = u.w[m];
  }
}

// One tet's element Schur block (upper triangle su) and r = C A^-1 B, with the Neumann rows
// and columns of its faces set as described above.  F: its face ids (nF bounds the flag reads).
template <class R>
__device__ __forceinline__ void elem_block(const double (&x)[4][3], const int (&sig)[4], const int (&F)[4], double kap,
                                           const DevParams& P, int64_t nF, R (&su)[10], R (&r)[4]) {
  Elem<R> E;
  E.init(x, kap, P.c, sig);
  R B[4];
  load_vec<R>(x, E.vol, P, B);
  bool neu[4] = {false, false, false, false};
  double gN[4] = {0, 0, 0, 0};
  if (P.nm) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      neu[k] = (uint32_t)F[k] < (uint64_t)nF && P.nm[F[k]];
      if (!neu[k]) continue;
      gN[k] = neumann_flux(E, x, k, kap, P);
      const R ln = E.d[k] * (R)gN[k] * (R)(1.0 / 3.0);
#pragma unroll
      for (int i = 0; i < 4; ++i)
        if (i != opp(k)) B[i] += ln;
    }
  }
  E.CAinv(B, r);
  E.Supper(su);
  if (P.nm) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (!neu[k]) continue;
      r[k] = (R)(-gN[k]);
#pragma unroll
      for (int l = 0; l < 4; ++l) su[uidx(k, l)] = l == k ? (R)1 : (R)0;
    }
  }
}

// An empty register barrier on the coordinates: the element arithmetic of one field cannot be
// hoisted out of a loop over fields (holding its geometric intermediates in registers across
// the loop would cost more, in occupancy, than recomputing them).
__device__ __forceinline__ void opaque_coords(double (&x)[4][3]) {
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int e = 0; e < 3; ++e) asm volatile("" : "+v"(x[i][e]));
}

// the tet's vertex ids (clamped into range: invalid input gives garbage, never a read out of
// range), sigma, face ids and coordinates
__device__ __forceinline__ void elem_inputs(int64_t nC, const double4* __restrict__ XA, int64_t nE, int64_t t,
                                            const int32_t* __restrict__ tet, const int32_t* __restrict__ t2f,
                                            const int8_t* __restrict__ sigma, int (&sig)[4], int (&F)[4],
                                            double (&x)[4][3]) {
  int v[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    v[i] = tet[i * nE + t];
    if ((uint32_t)v[i] >= (uint64_t)nC) v[i] = 0;
    sig[i] = sigma[i * nE + t];
    F[i] = t2f[i * nE + t];
  }
  gather_xa(XA, v, x);
}

// A workgroup scans CX consecutive tets for cross-tile faces and computes the element blocks
// of the ones that have any (about a third in refined meshes) from a compacted LDS list, so
// the element arithmetic runs only where a record is written.
constexpr int CXK = 4;
constexpr int CX = CT * CXK;

// Records are stored densely per workgroup of this pass: workgroup b's region starts at
// 4 CX b, a tet's records follow each other in local-face order at its offset, the offsets in
// tet order (an exclusive scan of the cross-face counts); cinfo[t] = offset << 4 | mask of
// the tet's cross faces, so the tile pass finds the record of slot 4t+k at
// rec_index(t, k, cinfo[t]).  A field's records take rec_stride(nE) slots.
__host__ __device__ __forceinline__ int64_t rec_stride(int64_t nE) { return 4 * CX * ((nE + CX - 1) / CX); }
__device__ __forceinline__ int64_t rec_index(int t, int k, uint32_t ci) {
  return (int64_t)(t / CX) * 4 * CX + (ci >> 4) + __popc((ci & 15u) & ((1u << k) - 1u));
}

template <class R>
__global__ __launch_bounds__(CT) void k_cond_cross(int64_t nC, const double4* __restrict__ XA, int64_t nE,
                                                   const int32_t* __restrict__ tet, const int32_t* __restrict__ t2f,
                                                   const int8_t* __restrict__ sigma, const int32_t* __restrict__ nbr,
                                                   int nk, const double* __restrict__ kappa, DevParams P, int64_t nF,
                                                   SlotRec<R>* __restrict__ recs, uint16_t* __restrict__ cinfo) {
  __shared__ int32_t lt[CX];
  __shared__ int32_t lcnt;
  __shared__ uint32_t lw[CT / 64];
  const int64_t T0 = (int64_t)blockIdx.x * CX;
  __builtin_amdgcn_s_setprio(2);  // raised while loads are issued (as in the tile pass)
  if (threadIdx.x == 0) lcnt = 0;
  __syncthreads();
  int nbv[CXK][4], sgv[CXK][4];
#pragma unroll
  for (int j = 0; j < CXK; ++j) {
    const int64_t t = T0 + j * CT + threadIdx.x;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      nbv[j][k] = t < nE ? nbr[k * nE + t] : -1;
      sgv[j][k] = t < nE ? sigma[k * nE + t] : 1;
    }
  }
  int cm[CXK];
#pragma unroll
  for (int j = 0; j < CXK; ++j) {
    const int64_t t = T0 + j * CT + threadIdx.x;
    const int64_t tile = t / CT;
    cm[j] = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (sgv[j][k] < 0 && nbv[j][k] >= 0 && nbv[j][k] / CT != tile) cm[j] |= 1 << k;
  }
  // the tets' record offsets in tet order (j major, then thread)
  uint32_t run = 0, off[CXK];
#pragma unroll
  for (int j = 0; j < CXK; ++j) {
    uint32_t tot;
    off[j] = run + block_excl_scan<CT / 64>((uint32_t)__popc(cm[j]), lw, tot);
    run += tot;
  }
#pragma unroll
  for (int j = 0; j < CXK; ++j) {
    const int64_t t = T0 + j * CT + threadIdx.x;
    if (t < nE) cinfo[t] = (uint16_t)(off[j] << 4 | cm[j]);
    if (cm[j]) lt[atomicAdd(&lcnt, 1)] = (int32_t)(off[j] << 14 | (uint32_t)(t - T0) << 4 | cm[j]);
  }
  __syncthreads();
  const int n = lcnt;
  const int64_t rs = rec_stride(nE), base = (int64_t)blockIdx.x * 4 * CX;
  for (int i = threadIdx.x; i < n; i += CT) {
    const int w = lt[i];
    const int64_t t = T0 + ((w >> 4) & (CX - 1));
    const int cross = w & 15;
    const int64_t tb = base + (w >> 14);
    int sig[4], F[4];
    double x[4][3];
    __builtin_amdgcn_s_setprio(2);
    elem_inputs(nC, XA, nE, t, tet, t2f, sigma, sig, F, x);
    __builtin_amdgcn_s_setprio(0);
    for (int j = 0; j < nk; ++j) {  // field j of the group: kappa + j nE, records at recs + j rs
      opaque_coords(x);
      R su[10], r[4];
      elem_block<R>(x, sig, F, kappa ? kappa[j * nE + t] : P.kc, P, nF, su, r);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (!(cross & (1 << k))) continue;
        SlotRec<R> q;
        q.d = su[uidx(k, k)];
        q.r = r[k];
        int m = 0;
#pragma unroll
        for (int l = 0; l < 4; ++l) {
          if (l == k) continue;
          q.o[m] = su[uidx(k, l)];
          q.c[m] = F[l];
          ++m;
        }
        store_rec(recs + j * rs + tb + __popc(cross & ((1 << k) - 1)), q);
      }
    }
  }
}

__global__ __launch_bounds__(FT) void k_coords_aos(int64_t nC, const double* __restrict__ X, double4* __restrict__ XA) {
  const int64_t v = (int64_t)blockIdx.x * FT + threadIdx.x;
  if (v >= nC) return;
  XA[v] = make_double4(X[v], X[nC + v], X[2 * nC + v], 0.0);
}

// rank of each of the 6 columns (ties by position; pads last)
__device__ __forceinline__ void col_ranks(const int (&cf)[6], int (&rk)[6]) {
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    int rank = 0;
#pragma unroll
    for (int m = 0; m < 6; ++m) rank += (cf[m] < cf[i] || (cf[m] == cf[i] && m < i)) ? 1 : 0;
    rk[i] = rank;
  }
}

// b_D = |F| u_D(centroid) of a Dirichlet boundary face (0 elsewhere)
__device__ __forceinline__ double face_bD(int64_t nF, int64_t nC, const double* __restrict__ X,
                                          const int32_t* __restrict__ faces, const DevParams& P, int64_t f, int q1) {
  if (q1 >= 0 || P.uk == PHFEM_FUN_ZERO || (P.nm && P.nm[f])) return 0.0;
  double xx[3][3];
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    int vv = faces[m * nF + f];
    if ((uint32_t)vv >= (uint64_t)nC) vv = 0;  // invalid input: no read out of range
#pragma unroll
    for (int e = 0; e < 3; ++e) xx[m][e] = X[e * nC + vv];
  }
  double u0 = xx[2][0] - xx[0][0], u1 = xx[2][1] - xx[0][1], u2 = xx[2][2] - xx[0][2];
  double s0 = xx[1][0] - xx[0][0], s1 = xx[1][1] - xx[0][1], s2 = xx[1][2] - xx[0][2];
  double n0 = u1 * s2 - u2 * s1, n1 = u2 * s0 - u0 * s2, n2 = u0 * s1 - u1 * s0;
  double area = 0.5 * sqrt(n0 * n0 + n1 * n1 + n2 * n2);
  return area * fun_at<double>(P.uk, P.up, (xx[0][0] + xx[1][0] + xx[2][0]) / 3.0,
                               (xx[0][1] + xx[1][1] + xx[2][1]) / 3.0, (xx[0][2] + xx[1][2] + xx[2][2]) / 3.0);
}

// Rows of the faces owned by tile blockIdx.x.  Faces are numbered in owner order, so the tile
// owns one id range, found from its tets' owned faces right after their first loads; the
// face-to-tet slots of the first NPF chunks of CT faces of that range, and the records of
// their cross-tile second tets, are then requested before the element arithmetic, so that
// their latency overlaps it instead of following it.  PATTERN: also rowptr and col
// (values-only re-assembly leaves them to an earlier call).
template <class R, bool PATTERN>
__global__ __launch_bounds__(CT) void k_cond_tile(int64_t nC, const double4* __restrict__ XA,
                                                  const double* __restrict__ X, int64_t nE,
                                                  const int32_t* __restrict__ tet, const int32_t* __restrict__ t2f,
                                                  const int8_t* __restrict__ sigma, const double* __restrict__ kappa,
                                                  DevParams P, int64_t nF, const int32_t* __restrict__ faces,
                                                  const int32_t* __restrict__ face2tet,
                                                  const SlotRec<R>* __restrict__ recs,
                                                  const uint16_t* __restrict__ cinfo, int32_t* __restrict__ rowptr,
                                                  int32_t* __restrict__ col, double* __restrict__ val,
                                                  double* __restrict__ diag, double* __restrict__ rhs) {
  constexpr int NPF = 2;  // (4 waves per SIMD in FP32, 3 in FP64 either way)
  __shared__ R lS[10][CT];
  __shared__ R lr[4][CT];
  __shared__ int32_t lF[4][CT];
  __shared__ __align__(16) int32_t lcol[PATTERN ? 6 * CT : 2];
  __shared__ __align__(16) double lval[6 * CT];
  __shared__ int32_t lrange[2];
  const int64_t T0 = (int64_t)blockIdx.x * CT;
  const int nb = nE - T0 < CT ? (int)(nE - T0) : CT;
  const int o = threadIdx.x;
  // a raised wave priority while the tile's loads are issued, back to normal for the element
  // arithmetic, so that other waves' loads start ahead of it
  __builtin_amdgcn_s_setprio(2);
  if (o == 0) {
    lrange[0] = INT_MAX;
    lrange[1] = -1;
  }
  const int64_t t = T0 + o;
  int v[4], sig[4], F[4];
  double kap = P.kc;
  int fmin = INT_MAX, fmax = -1;
  if (o < nb) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      v[i] = tet[i * nE + t];
      if ((uint32_t)v[i] >= (uint64_t)nC) v[i] = 0;  // invalid input: no read out of range
      sig[i] = sigma[i * nE + t];
      F[i] = t2f[i * nE + t];
      if (sig[i] > 0) {
        fmin = min(fmin, F[i]);
        fmax = max(fmax, F[i]);
      }
    }
    if (kappa) kap = kappa[t];
  }
  double x[4][3];
  if (o < nb) gather_xa(XA, v, x);
  // the tile's owned face range
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) {
    fmin = min(fmin, __shfl_xor(fmin, d, 64));
    fmax = max(fmax, __shfl_xor(fmax, d, 64));
  }
  __syncthreads();
  if ((o & 63) == 0) {
    atomicMin(&lrange[0], fmin);
    atomicMax(&lrange[1], fmax);
  }
  __syncthreads();
  const int64_t F0 = lrange[0] < 0 ? 0 : lrange[0];  // (a negative id: invalid input)
  int64_t F1 = (int64_t)lrange[1] + 1;
  if (F1 > nF) F1 = nF;                    // invalid input: stay in range
  if (F1 - F0 > 4 * CT) F1 = F0 + 4 * CT;  // (a tile owns at most 4 CT faces)
  // the slot of the second tet of a face is a record when that tet lies outside the tile
  auto cross_slot = [&](int q1) {
    const int o2 = (q1 >> 2) - (int)T0;
    return q1 >= 0 && (uint64_t)q1 < (uint64_t)(4 * nE) && !(o2 >= 0 && o2 < nb);
  };
  int pq0[NPF], pq1[NPF];
#pragma unroll
  for (int c = 0; c < NPF; ++c) {
    const int64_t f = F0 + c * CT + o;
    pq0[c] = f < F1 ? face2tet[f] : -1;
    pq1[c] = f < F1 ? face2tet[nF + f] : -1;
  }
  SlotRec<R> prec[NPF];
#pragma unroll
  for (int c = 0; c < NPF; ++c)
    if (cross_slot(pq1[c])) prec[c] = recs[rec_index(pq1[c] >> 2, pq1[c] & 3, cinfo[pq1[c] >> 2])];
  __builtin_amdgcn_s_setprio(0);
  if (o < nb) {
    R su[10], r[4];
    elem_block<R>(x, sig, F, kap, P, nF, su, r);
#pragma unroll
    for (int j = 0; j < 10; ++j) lS[j][o] = su[j];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      lr[k][o] = r[k];
      lF[k][o] = F[k];
    }
  }
  __syncthreads();
  // one chunk of CT faces from `base`: rows built into LDS, then stored as contiguous ranges.
  // pre: q0, q1 (and the record, for a cross-tile second tet) were loaded above.
  auto chunk = [&](int64_t base, bool pre, int q0, int q1, SlotRec<R> rec) __attribute__((always_inline)) {
    const int nloc = F1 - base < CT ? (int)(F1 - base) : CT;
    const int64_t f = base + o;
    if (o < nloc) {
      if (!pre) {
        q0 = face2tet[f];
        q1 = face2tet[nF + f];
      }
      const int oo = (q0 >> 2) - (int)T0, k = q0 & 3;
      int cf[6], rk[6];
      double cv[6];
      double dg = 0.0, rh = 0.0;
      if (q0 >= 0 && oo >= 0 && oo < nb) {
        dg = (double)lS[uidx(k, k)][oo];
        rh = face_bD(nF, nC, X, faces, P, f, q1) - (double)lr[k][oo];
        int n = 0;
#pragma unroll
        for (int l = 0; l < 4; ++l) {
          if (l == k) continue;
          cf[n] = lF[l][oo];
          cv[n] = (double)lS[uidx(k, l)][oo];
          ++n;
        }
      } else {  // not owned here: invalid input (the row is written as zeros)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          cf[i] = INT_MAX;
          cv[i] = 0.0;
        }
      }
      if (q1 >= 0 && (uint64_t)q1 < (uint64_t)(4 * nE)) {
        const int o2 = (q1 >> 2) - (int)T0, k2 = q1 & 3;
        if (o2 >= 0 && o2 < nb) {  // second tet in the tile
          dg += (double)lS[uidx(k2, k2)][o2];
          rh -= (double)lr[k2][o2];
          int n = 3;
#pragma unroll
          for (int l = 0; l < 4; ++l) {
            if (l == k2) continue;
            cf[n] = lF[l][o2];
            cv[n] = (double)lS[uidx(k2, l)][o2];
            ++n;
          }
        } else {  // its record
          const SlotRec<R> b = pre ? rec : recs[rec_index(q1 >> 2, k2, cinfo[q1 >> 2])];
          dg += (double)b.d;
          rh -= (double)b.r;
#pragma unroll
          for (int i = 0; i < 3; ++i) {
            cf[3 + i] = b.c[i];
            cv[3 + i] = (double)b.o[i];
          }
        }
      } else {
#pragma unroll
        for (int i = 3; i < 6; ++i) {
          cf[i] = INT_MAX;  // sorts last; written as column f with value 0
          cv[i] = 0.0;
        }
      }
      col_ranks(cf, rk);
#pragma unroll
      for (int i = 0; i < 6; ++i) {
        if (PATTERN) lcol[6 * o + rk[i]] = cf[i] == INT_MAX ? (int32_t)f : cf[i];
        lval[6 * o + rk[i]] = cv[i];
      }
      st_nt(diag + f, dg);
      st_nt(rhs + f, rh);
      if (PATTERN) {
        st_nt(rowptr + f, (int32_t)(6 * f));
        if (f == nF - 1) rowptr[nF] = (int32_t)(6 * nF);
      }
    }
    __syncthreads();
    // as 16-byte value pairs and 8-byte column pairs (val + 48 base bytes is 16-byte aligned,
    // col + 24 base bytes 8-byte aligned, given the alignment the entry point checks)
    {
      typedef double d2 __attribute__((ext_vector_type(2)));
      typedef int32_t i2 __attribute__((ext_vector_type(2)));
      const d2* lv2 = reinterpret_cast<const d2*>(lval);
      d2* gv2 = reinterpret_cast<d2*>(val + 6 * base);
      for (int i = o; i < 3 * nloc; i += CT) {
        __builtin_nontemporal_store(lv2[i], gv2 + i);
        if (PATTERN)
          __builtin_nontemporal_store(reinterpret_cast<const i2*>(lcol)[i], reinterpret_cast<i2*>(col + 6 * base) + i);
      }
    }
    __syncthreads();
  };
  int64_t base = F0;
#pragma unroll
  for (int c = 0; c < NPF; ++c)
    if (base < F1) {
      chunk(base, true, pq0[c], pq1[c], prec[c]);
      base += CT;
    }
  for (; base < F1; base += CT) chunk(base, false, -1, -1, prec[0]);
}

// ---------------------------------------------------------------- recovery / residual (FP64)
// hi + lo = a + b exactly (Knuth's two-sum)
__device__ __forceinline__ void two_sum(double a, double b, double& hi, double& lo) {
  hi = a + b;
  const double bb = hi - a;
  lo = (a - (hi - bb)) + (b - bb);
}

// sum_i B_i + sum_k d_k f_k rounded once from a double-double accumulation (each product
// enters with its exact rounding error from an fma)
__device__ __forceinline__ double dd_mean_sum(const double (&B)[4], const double (&d)[4], const double (&f)[4]) {
  double hi = B[0], lo = 0.0, h, l;
#pragma unroll
  for (int i = 1; i < 4; ++i) {
    two_sum(hi, B[i], h, l);
    hi = h;
    lo += l;
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double p = d[k] * f[k];
    two_sum(hi, p, h, l);
    hi = h;
    lo += l + fma(d[k], f[k], -p);
  }
  return hi + lo;
}

// U(T) = A^-1 (Bsrc + C' lambda) with Bsrc = load vector (gsrc == null) or gsrc[4][nE].
// cu != null: cu[4t+k] = (C U)_k, the term local face k of tet t takes off the residual of
// its face (a Neumann row lambda_F = g takes lambda_F - g); k_face_residual then forms each
// face's residual from its owner's and neighbour's slots in that order, so the sums do not
// depend on scheduling.  A vertex or face id out of range sets DEV_BADNODE (nothing of that
// tet is read or written), a zero volume DEV_DEGEN.
__global__ __launch_bounds__(FT) void k_recover(int64_t nC, const double* __restrict__ X, int64_t nE, int64_t nF,
                                                const int32_t* __restrict__ tet, const int32_t* __restrict__ t2f,
                                                const int8_t* __restrict__ sigma, const double* __restrict__ kappa,
                                                DevParams P, const double* __restrict__ lambda,
                                                const double* __restrict__ gsrc, double* __restrict__ U,
                                                double* __restrict__ cu, int* __restrict__ flags) {
  int64_t t = (int64_t)blockIdx.x * FT + threadIdx.x;
  if (t >= nE) return;
  int v[4], sig[4], F[4];
  bool inr = true;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    v[i] = tet[i * nE + t];
    sig[i] = sigma[i * nE + t];
    F[i] = t2f[i * nE + t];
    inr = inr && (uint32_t)v[i] < (uint64_t)nC && (uint32_t)F[i] < (uint64_t)nF;
  }
  if (!inr) {
    if (flags) atomicOr(flags, DEV_BADNODE);
    return;
  }
  double x[4][3];
  gather_x(nC, X, v, x);
  const double kap = kappa ? kappa[t] : P.kc;
  Elem<double> E;
  if (!E.init(x, kap, P.c, sig)) {
    if (flags) atomicOr(flags, DEV_DEGEN);
    return;
  }
  double B[4];
  if (gsrc) {
#pragma unroll
    for (int i = 0; i < 4; ++i) B[i] = gsrc[i * nE + t];
  } else {
    load_vec<double>(x, E.vol, P, B);
  }
  double mu[4] = {0, 0, 0, 0}, gN[4] = {0, 0, 0, 0};
  bool neu[4] = {false, false, false, false};
  if (P.nm && !gsrc) {  // Neumann faces: LN = C_k' g in place of C_k' lambda_F
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      neu[k] = P.nm[F[k]];
      if (neu[k]) gN[k] = neumann_flux(E, x, k, kap, P);
    }
  }
  double fac[4];  // mu_k = d_k fac_k: the multiplier, g on a Neumann face
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    fac[k] = neu[k] ? gN[k] : (lambda ? lambda[F[k]] : 0.0);
    mu[k] = E.d[k] * fac[k];
  }
  // The mean mode s = (sum B + sum mu) / (c vol): the four mu_k = sigma_k |F_k| lambda_k nearly
  // cancel (their sum is the flux balance of the tet, O(h) smaller than the terms), so the sum
  // is carried in double-double (error-free products and sums); otherwise its rounding,
  // amplified by 1 / (c vol), sets the floor of the true residual (about 1e-12 relative at
  // h = 1/32 with lognormal kappa).
  const double dk[4] = {E.d[0], E.d[1], E.d[2], E.d[3]};
  const double s = dd_mean_sum(B, dk, fac) * E.icv;
  double y[4], u[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) y[i] = B[i] - mu[opp(i)] / 3.0;  // face opposite vertex i is opp(i)
#pragma unroll
  for (int i = 0; i < 4; ++i) u[i] = s + (E.W[i][0] * y[0] + E.W[i][1] * y[1] + E.W[i][2] * y[2] + E.W[i][3] * y[3]);
  if (U) {
#pragma unroll
    for (int i = 0; i < 4; ++i) U[i * nE + t] = u[i];
  }
  if (cu) {
    const double su = (u[0] + u[1]) + (u[2] + u[3]);
    double c4[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)  // a Neumann row is lambda_F = g
      c4[k] = neu[k] ? (lambda ? lambda[F[k]] : 0.0) - gN[k] : E.d[k] * (su - u[opp(k)]) / 3.0;
    reinterpret_cast<double4*>(cu)[t] = make_double4(c4[0], c4[1], c4[2], c4[3]);
  }
}

// res[F] = b_D[F] - cu[owner slot] - cu[neighbour slot] (b_D null: 0), the two terms in that
// order; a slot out of range sets DEV_BADNODE and leaves res[F] unwritten.
__global__ __launch_bounds__(FT) void k_face_residual(int64_t nF, int64_t nE, const int32_t* __restrict__ face2tet,
                                                      const double* __restrict__ bD, const double* __restrict__ cu,
                                                      double* __restrict__ res, int* __restrict__ flags) {
  const int64_t f = (int64_t)blockIdx.x * FT + threadIdx.x;
  if (f >= nF) return;
  const int q0 = face2tet[f], q1 = face2tet[nF + f];
  if ((uint32_t)q0 >= (uint64_t)(4 * nE) || (q1 != -1 && (uint32_t)q1 >= (uint64_t)(4 * nE))) {
    if (flags) atomicOr(flags, DEV_BADNODE);
    return;
  }
  double r = (bD ? bD[f] : 0.0) - cu[q0];
  if (q1 >= 0) r -= cu[q1];
  res[f] = r;
}

// ---------------------------------------------------------------- adjoint VJP (FP64)
// G_i = dPhi_T/dx_i for Phi_T = P'A U - lambda'C P - P'B - Q'C U + sum_bnd Q_F b_D,F;
// dJ/dX_v -= G_i, dJ/dlog kappa_T = -kappa vol gP.gU.
// A vertex or face id out of range sets DEV_BADNODE, a zero volume DEV_DEGEN (that tet then
// contributes nothing).
__global__ __launch_bounds__(FT) void k_vjp(int64_t nC, const double* __restrict__ X, int64_t nE, int64_t nF,
                                            const int32_t* __restrict__ tet, const int32_t* __restrict__ t2f,
                                            const int8_t* __restrict__ sigma, const int32_t* __restrict__ nbr,
                                            const double* __restrict__ kappa, DevParams P,
                                            const double* __restrict__ Uu, const double* __restrict__ Pp,
                                            const double* __restrict__ lambda, const double* __restrict__ Q,
                                            double* __restrict__ dlogk, double* __restrict__ dX,
                                            int* __restrict__ flags) {
  int64_t t = (int64_t)blockIdx.x * FT + threadIdx.x;
  if (t >= nE) return;
  int v[4], sig[4], Fi[4];
  double U[4], Pv[4], lam[4], Qf[4];
  bool bnd[4], inr = true;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    v[i] = tet[i * nE + t];
    Fi[i] = t2f[i * nE + t];
    inr = inr && (uint32_t)v[i] < (uint64_t)nC && (uint32_t)Fi[i] < (uint64_t)nF;
  }
  if (!inr) {
    atomicOr(flags, DEV_BADNODE);
    return;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    sig[i] = sigma[i * nE + t];
    lam[i] = lambda[Fi[i]];
    Qf[i] = Q[Fi[i]];
    bnd[i] = nbr[i * nE + t] < 0;
    U[i] = Uu[i * nE + t];
    Pv[i] = Pp[i * nE + t];
  }
  double x[4][3];
  gather_x(nC, X, v, x);
  const double kap = kappa ? kappa[t] : P.kc;
  Elem<double> E;
  if (!E.init(x, kap, P.c, sig)) {
    atomicOr(flags, DEV_DEGEN);
    return;
  }
  const double vol = E.vol, c = P.c;
  double gU[3] = {0, 0, 0}, gP[3] = {0, 0, 0};
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      gU[e] += U[i] * E.g[i][e];
      gP[e] += Pv[i] * E.g[i][e];
    }
  const double gPU = gP[0] * gU[0] + gP[1] * gU[1] + gP[2] * gU[2];
  if (dlogk) dlogk[t] = -kap * vol * gPU;
  if (!dX) return;
  double G[4][3];
  const double sP = (Pv[0] + Pv[1]) + (Pv[2] + Pv[3]), sU = (U[0] + U[1]) + (U[2] + U[3]);
  const double PU = Pv[0] * U[0] + Pv[1] * U[1] + Pv[2] * U[2] + Pv[3] * U[3];
  // (1) P'A U: stiffness and mass parts
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const double giU = E.g[i][0] * gU[0] + E.g[i][1] * gU[1] + E.g[i][2] * gU[2];
    const double giP = E.g[i][0] * gP[0] + E.g[i][1] * gP[1] + E.g[i][2] * gP[2];
#pragma unroll
    for (int e = 0; e < 3; ++e)
      G[i][e] = kap * vol * (gPU * E.g[i][e] - giU * gP[e] - giP * gU[e]) + c * vol / 20.0 * (PU + sP * sU) * E.g[i][e];
  }
  // (3) -P'B
  if (P.quad == PHFEM_QUAD_P1_INTERP) {
    double f[4], gf[4][3];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      f[i] = fun_at<double>(P.fk, P.fp, x[i][0], x[i][1], x[i][2]);
      fun_grad(P.fk, P.fp, x[i][0], x[i][1], x[i][2], gf[i]);
    }
    const double Pf = Pv[0] * f[0] + Pv[1] * f[1] + Pv[2] * f[2] + Pv[3] * f[3];
    const double sf = (f[0] + f[1]) + (f[2] + f[3]);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int e = 0; e < 3; ++e)
        G[i][e] -= vol / 20.0 * ((Pf + sP * sf) * E.g[i][e] + (Pv[i] + sP) * gf[i][e]);
  } else {
    double fc[4], gfc[4][3], sPk[4];
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int a = fv(k, 0), b = fv(k, 1), cc = fv(k, 2);
      double cx = (x[a][0] + x[b][0] + x[cc][0]) / 3.0, cy = (x[a][1] + x[b][1] + x[cc][1]) / 3.0,
             cz = (x[a][2] + x[b][2] + x[cc][2]) / 3.0;
      fc[k] = fun_at<double>(P.fk, P.fp, cx, cy, cz);
      fun_grad(P.fk, P.fp, cx, cy, cz, gfc[k]);
      sPk[k] = sP - Pv[opp(k)];
      acc += fc[k] * sPk[k];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int e = 0; e < 3; ++e) {
        double s = vol / 12.0 * acc * E.g[i][e];
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if (opp(k) != i) s += vol / 36.0 * sPk[k] * gfc[k][e];
        G[i][e] -= s;
      }
  }
  // (2) -lambda'C P - Q'C U  and  (4) + Q_F b_D,F on boundary faces: area derivatives
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int a = fv(k, 0), b = fv(k, 1), cc = fv(k, 2);
    double n[3];
    {
      double p0 = x[b][0] - x[a][0], p1 = x[b][1] - x[a][1], p2 = x[b][2] - x[a][2];
      double q0 = x[cc][0] - x[a][0], q1 = x[cc][1] - x[a][1], q2 = x[cc][2] - x[a][2];
      n[0] = p1 * q2 - p2 * q1;
      n[1] = p2 * q0 - p0 * q2;
      n[2] = p0 * q1 - p1 * q0;
    }
    const double nn = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    const double area = 0.5 * nn;
    double coef = -(double)sig[k] * (lam[k] * (sP - Pv[opp(k)]) + Qf[k] * (sU - U[opp(k)])) / 3.0;
    double gud[3] = {0, 0, 0};
    if (bnd[k]) {
      double cx = (x[a][0] + x[b][0] + x[cc][0]) / 3.0, cy = (x[a][1] + x[b][1] + x[cc][1]) / 3.0,
             cz = (x[a][2] + x[b][2] + x[cc][2]) / 3.0;
      coef += Qf[k] * fun_at<double>(P.uk, P.up, cx, cy, cz);
      fun_grad(P.uk, P.up, cx, cy, cz, gud);
    }
    // d|F|/dx_a = 0.5 nhat x (x_c - x_b), cyclic
    const int vv[3] = {a, b, cc};
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      const int p = vv[m], q = vv[(m + 1) % 3], r = vv[(m + 2) % 3];
      double e0 = x[r][0] - x[q][0], e1 = x[r][1] - x[q][1], e2 = x[r][2] - x[q][2];
      double dA0 = 0.5 * (n[1] * e2 - n[2] * e1) / nn, dA1 = 0.5 * (n[2] * e0 - n[0] * e2) / nn,
             dA2 = 0.5 * (n[0] * e1 - n[1] * e0) / nn;
      G[p][0] += coef * dA0;
      G[p][1] += coef * dA1;
      G[p][2] += coef * dA2;
      if (bnd[k]) {
#pragma unroll
        for (int e = 0; e < 3; ++e) G[p][e] += Qf[k] * area * gud[e] / 3.0;
      }
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int e = 0; e < 3; ++e) atomicAdd(&dX[e * nC + v[i]], -G[i][e]);
}

// instantiations used by the solver / grad drivers (solve.hip)
// U = A^-1 (Bsrc + C' lambda) per tet and, with res, res = b_D - C U per face (b_D null: 0);
// cu is a 4 nE scratch array of per-slot terms (required with res)
int launch_recover(int64_t nC, const double* X, int64_t nE, int64_t nF, const int32_t* tet, const int32_t* t2f,
                   const int8_t* sigma, const int32_t* face2tet, const double* kappa, const DevParams& P,
                   const double* lambda, const double* gsrc, const double* bD, double* U, double* cu, double* res,
                   int* flags, hipStream_t s) {
  const double bytes = (36.0 + (kappa ? 8.0 : 0.0) + (gsrc ? 32.0 : 0.0) + (U ? 32.0 : 0.0)) * nE + 24.0 * nC +
                       (lambda ? 8.0 : 0.0) * nE + (res ? 32.0 : 0.0) * nE;
  PH_LAUNCH_B("recover", bytes, k_recover, grid_for(nE, FT), FT, 0, s, nC, X, nE, nF, tet, t2f, sigma, kappa, P, lambda,
              gsrc, U, res ? cu : nullptr, flags);
  if (res)
    PH_LAUNCH_B("face_residual", (8.0 + (bD ? 8.0 : 0.0) + 16.0 + 8.0) * nF, k_face_residual, grid_for(nF, FT), FT, 0,
                s, nF, nE, face2tet, bD, (const double*)cu, res, flags);
  return PHFEM_OK;
}

int launch_face_init(int64_t nF, int64_t nC, const double* X, const int32_t* faces, const int32_t* face2tet,
                     const DevParams& P, uint32_t* cnt, double* diag, double* rhs, int* flags, hipStream_t s) {
  PH_LAUNCH_B("face_init", (8.0 + (cnt ? 4.0 : 0.0) + (diag ? 8.0 : 0.0) + (rhs ? 8.0 : 0.0)) * nF, k_face_init,
              grid_for(nF + 1, FT), FT, 0, s, nF, nC, X, faces, face2tet, P, cnt, diag, rhs, flags);
  return PHFEM_OK;
}

int launch_vjp(int64_t nC, const double* X, int64_t nE, int64_t nF, const int32_t* tet, const int32_t* t2f,
               const int8_t* sigma, const int32_t* nbr, const double* kappa, const DevParams& P, const double* U,
               const double* Pp, const double* lambda, const double* Q, double* dlogk, double* dX, int* flags,
               hipStream_t s) {
  PH_LAUNCH_B("vjp", (124.0 + (kappa ? 8.0 : 0.0)) * nE + 16.0 * nE + 72.0 * nC, k_vjp, grid_for(nE, FT), FT, 0, s, nC,
              X, nE, nF, tet, t2f, sigma, nbr, kappa, P, U, Pp, lambda, Q, dlogk, dX, flags);
  return PHFEM_OK;
}

}  // namespace ph

using namespace ph;

extern "C" int phfem_assemble(int64_t nC, const double* coord, int64_t nE, const int32_t* tetra, const int8_t* sigma,
                              const double* kappa, const phfem_params* p, double* vol, double* K, double* d,
                              double* B, double* S, double* r, phfem_stream_t stream_) {
  clear_error();
  hipStream_t s = (hipStream_t)stream_;
  int rc = check_params(p);
  if (rc) return rc;
  if (nC <= 0 || nE <= 0 || !coord || !tetra) return err(PHFEM_EINVAL, "bad mesh arguments");
  DevParams P = to_dev(*p);
  if (p->precision == PHFEM_MIXED)
    PH_LAUNCH("assemble_f32", k_assemble<float>, grid_for(nE, FT), FT, 0, s, nC, coord, nE, tetra, sigma, kappa, P,
              vol, K, d, B, S, r);
  else
    PH_LAUNCH("assemble_f64", k_assemble<double>, grid_for(nE, FT), FT, 0, s, nC, coord, nE, tetra, sigma, kappa, P,
              vol, K, d, B, S, r);
  return PHFEM_OK;
}

// fields per cross pass (it loops over them, reading each cross tet's inputs once)
constexpr int COND_GROUP = 4;

extern "C" size_t phfem_condense_batch_workspace(int64_t nC, int64_t nE, int64_t nF, int32_t precision,
                                                 int32_t nk) {
  (void)nF;
  if (nk < 1) return 0;
  Arena a;  // the AoS coordinates and one group's cross-tile records (the groups run in turn)
  a.take<double4>(nC);
  const int64_t g = std::min<int64_t>(nk, COND_GROUP);
  a.take<uint16_t>(nE);
  if (precision == PHFEM_MIXED)
    a.take<SlotRec<float>>(g * rec_stride(nE) + 4);
  else
    a.take<SlotRec<double>>(g * rec_stride(nE) + 4);
  return a.size();
}

extern "C" size_t phfem_condense_workspace(int64_t nC, int64_t nE, int64_t nF, int32_t precision) {
  return phfem_condense_batch_workspace(nC, nE, nF, precision, 1);
}

extern "C" int phfem_condense_batch(int64_t nC, const double* coord, int64_t nE, const int32_t* tetra, int64_t nF,
                                    const int32_t* faces, const int32_t* tet2face, const int8_t* sigma,
                                    const int32_t* nbr, const int32_t* face2tet, int32_t nk, const double* kappa,
                                    const phfem_params* p, void* work, size_t work_bytes, int32_t* rowptr,
                                    int32_t* col, double* val, double* diag, double* rhs, phfem_stream_t stream_) {
  clear_error();
  hipStream_t s = (hipStream_t)stream_;
  int rc = check_params(p);
  if (rc) return rc;
  if (nC <= 0 || nE <= 0 || nF <= 0 || !coord || !tetra || !faces || !tet2face || !sigma || !nbr || !face2tet || !val ||
      !diag || !rhs)
    return err(PHFEM_EINVAL, "bad condense arguments");
  if (nk < 1 || (nk > 1 && !kappa)) return err(PHFEM_EINVAL, "nk >= 1 coefficient fields (kappa required for nk > 1)");
  if ((rowptr == nullptr) != (col == nullptr)) return err(PHFEM_EINVAL, "rowptr and col: both or neither");
  if (6 * nF >= (int64_t(1) << 31) || 4 * nE >= (int64_t(1) << 31))
    return err(PHFEM_EINVAL, "face system exceeds int32 indexing");
  if ((reinterpret_cast<uintptr_t>(val) & 15) || (col && (reinterpret_cast<uintptr_t>(col) & 7)))
    return err(PHFEM_EINVAL, "val must be 16-byte and col 8-byte aligned");
  if (!work || work_bytes < phfem_condense_batch_workspace(nC, nE, nF, p->precision, nk))
    return err(PHFEM_EWORKSPACE, "condense workspace too small");
  Arena a(work, work_bytes);
  const bool mixed = p->precision == PHFEM_MIXED;
  double4* XA = a.take<double4>(nC);
  const int64_t grp = std::min<int64_t>(nk, COND_GROUP), rs = rec_stride(nE);
  uint16_t* cinfo = a.take<uint16_t>(nE);
  // (4 slots of slack: for invalid input a record index may run 3 past its region)
  void* recs = mixed ? (void*)a.take<SlotRec<float>>(grp * rs + 4) : (void*)a.take<SlotRec<double>>(grp * rs + 4);
  DevParams P = to_dev(*p);
  // algorithmic bytes per field.  cross: tets, tet2face, sigma, nbr (+ kappa) once (each
  // further field of its group adds its kappa only); tile: tets, tet2face, sigma (+ kappa)
  // once, face2tet once, off-diagonal values, diagonal and rhs written once, the pattern (col +
  // row pointer) once when written; coordinates once per pass (the records crossing tiles are
  // left out: an intermediate of this design)
  const double kb = kappa ? 8.0 : 0.0;
  const double cb = (52.0 + kb) * nE + 32.0 * nC;
  const double tbv = (36.0 + kb) * nE + 32.0 * nC + 8.0 * nF + (8.0 * 6.0 + 16.0) * nF, tbp = 4.0 * 7.0 * nF;
  const unsigned gt = grid_for(nE, CT), gx = grid_for(nE, CX);
  PH_LAUNCH_B("coords_aos", 56.0 * nC, k_coords_aos, grid_for(nC, FT), FT, 0, s, nC, coord, XA);
  for (int j0 = 0; j0 < nk; j0 += COND_GROUP) {
    // fields j0 .. j0 + g - 1: one cross pass writes their records, then one tile pass per field;
    // the pattern (when asked for) with the first field only
    const int g = std::min(COND_GROUP, nk - j0);
    const double* kg = kappa ? kappa + j0 * nE : nullptr;
    if (mixed)
      PH_LAUNCH_B("cond_cross_f32", cb + (g - 1) * kb * nE, k_cond_cross<float>, gx, CT, 0, s, nC, XA, nE, tetra,
                  tet2face, sigma, nbr, g, kg, P, nF, (SlotRec<float>*)recs, cinfo);
    else
      PH_LAUNCH_B("cond_cross_f64", cb + (g - 1) * kb * nE, k_cond_cross<double>, gx, CT, 0, s, nC, XA, nE, tetra,
                  tet2face, sigma, nbr, g, kg, P, nF, (SlotRec<double>*)recs, cinfo);
    for (int jj = 0; jj < g; ++jj) {
      const int j = j0 + jj;
      const double* kj = kappa ? kappa + j * nE : nullptr;
      int32_t* rp = j == 0 ? rowptr : nullptr;
      int32_t* cl = j == 0 ? col : nullptr;
      double *vj = val + j * 6 * nF, *dj = diag + j * nF, *rj = rhs + j * nF;
      const double tby = tbv + (cl ? tbp : 0.0);
      if (mixed) {
        const auto* rc32 = (const SlotRec<float>*)recs + jj * rs;
        if (cl)
          PH_LAUNCH_B("cond_tile_f32", tby, (k_cond_tile<float, true>), gt, CT, 0, s, nC, XA, coord, nE, tetra,
                      tet2face, sigma, kj, P, nF, faces, face2tet, rc32, cinfo, rp, cl, vj, dj, rj);
        else
          PH_LAUNCH_B("cond_tile_f32", tby, (k_cond_tile<float, false>), gt, CT, 0, s, nC, XA, coord, nE, tetra,
                      tet2face, sigma, kj, P, nF, faces, face2tet, rc32, cinfo, rp, cl, vj, dj, rj);
      } else {
        const auto* rc64 = (const SlotRec<double>*)recs + jj * rs;
        if (cl)
          PH_LAUNCH_B("cond_tile_f64", tby, (k_cond_tile<double, true>), gt, CT, 0, s, nC, XA, coord, nE, tetra,
                      tet2face, sigma, kj, P, nF, faces, face2tet, rc64, cinfo, rp, cl, vj, dj, rj);
        else
          PH_LAUNCH_B("cond_tile_f64", tby, (k_cond_tile<double, false>), gt, CT, 0, s, nC, XA, coord, nE, tetra,
                      tet2face, sigma, kj, P, nF, faces, face2tet, rc64, cinfo, rp, cl, vj, dj, rj);
      }
    }
  }
  return PHFEM_OK;
}

extern "C" int phfem_condense(int64_t nC, const double* coord, int64_t nE, const int32_t* tetra, int64_t nF,
                              const int32_t* faces, const int32_t* tet2face, const int8_t* sigma, const int32_t* nbr,
                              const int32_t* face2tet, const double* kappa, const phfem_params* p, void* work,
                              size_t work_bytes, int32_t* rowptr, int32_t* col, double* val, double* diag,
                              double* rhs, phfem_stream_t stream) {
  if (!rowptr || !col) {
    clear_error();
    return err(PHFEM_EINVAL, "bad condense arguments");
  }
  return phfem_condense_batch(nC, coord, nE, tetra, nF, faces, tet2face, sigma, nbr, face2tet, 1, kappa, p, work,
                              work_bytes, rowptr, col, val, diag, rhs, stream);
}
