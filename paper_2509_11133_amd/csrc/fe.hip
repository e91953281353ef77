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
constexpr int ET64 = 128;

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
__global__ __launch_bounds__(FT) void k_coords_aos(int64_t nC, const double* __restrict__ X, double4* __restrict__ XA) {
  const int64_t v = (int64_t)blockIdx.x * FT + threadIdx.x;
  if (v >= nC) return;
  XA[v] = make_double4(X[v], X[nC + v], X[2 * nC + v], 0.0);
}

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
                                                  double* __restrict__ rhs) {
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
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      int v = faces[m * nF + f];
#pragma unroll
      for (int e = 0; e < 3; ++e) x[m][e] = X[e * nC + v];
    }
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

// Condensation in two passes (no atomics):
//  k_elem_rec: one tet -> four slot records (slot 4t+k: row k of S(T), (C A^-1 B)_k and the
//              ids of the other three faces), staged in LDS and stored with coalesced
//              full-line writes;
//  k_face_rows: one face -> its whole CSR row from the slots of its owner and neighbour
//              (face2tet): off-diagonals sorted by column, diagonal S_owner + S_neighbour
//              and rhs (b_D - r_owner) - r_neighbour in that order.
// The neighbour slot is a random read; scattering the records to face order instead would
// turn it into a random partial-line write, which costs more.
// position of S_kl (either order) in the row-major upper triangle of a 4x4 matrix
__host__ __device__ constexpr int uidx(int k, int l) {
  return k <= l ? (k * (7 - k)) / 2 + l : (l * (7 - l)) / 2 + k;
}
static_assert(uidx(0, 0) == 0 && uidx(0, 3) == 3 && uidx(1, 1) == 4 && uidx(2, 1) == 5 && uidx(2, 2) == 7 &&
                  uidx(3, 3) == 9,
              "upper-triangle index");

template <class R>
struct SlotRec {  // row k of one tet's element Schur block S(T) and (C A^-1 B)_k
  R d;            // S_kk
  R r;            // (C A^-1 B)_k
  R o[3];         // S_kl for the three l != k, ascending l
  int32_t c[3];   // face ids of those three l
};
static_assert(sizeof(SlotRec<float>) == 32 && sizeof(SlotRec<double>) == 56, "packed slot records");

// the four slot records of one tet for one coefficient value, into the thread's LDS slots
template <class R>
__device__ __forceinline__ void elem_records(const double (&x)[4][3], const int (&sig)[4], const int (&F)[4],
                                             double kap, const DevParams& P, int64_t nF, uint2* lrec) {
  constexpr int W = sizeof(SlotRec<R>) / 8;
  Elem<R> E;
  E.init(x, kap, P.c, sig);
  R B[4], r[4], su[10];
  load_vec<R>(x, E.vol, P, B);
  bool neu[4] = {false, false, false, false};
  double gN[4] = {0, 0, 0, 0};
  if (P.nm) {  // Neumann faces: LN in the load; their rows become lambda_F = g
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
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    union {
      SlotRec<R> rec;
      uint2 w[W];
    } u;
    u.rec.d = neu[k] ? (R)1 : su[uidx(k, k)];
    u.rec.r = neu[k] ? (R)(-gN[k]) : r[k];
    int n = 0;
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      if (l == k) continue;
      u.rec.o[n] = neu[k] ? (R)0 : su[uidx(k, l)];
      u.rec.c[n] = neu[l] ? (int32_t)((uint32_t)F[l] | 0x80000000u) : F[l];  // a Neumann column: no coupling
      ++n;
    }
#pragma unroll
    for (int m = 0; m < W; ++m) lrec[k * W + m] = u.w[m];
  }
}

// workgroup size of k_elem_rec: FP64 records (56 B) stage 4 x 56 B per thread, so FP64 takes
// smaller workgroups to keep several resident per CU
template <class R>
constexpr int elem_threads() {
  return sizeof(R) == 8 ? ET64 : FT;
}

template <class R>
__global__ __launch_bounds__(elem_threads<R>()) void k_elem_rec(int64_t nC, const double4* __restrict__ XA, int64_t nE,
                                                 const int32_t* __restrict__ tet, const int32_t* __restrict__ t2f,
                                                 const int8_t* __restrict__ sigma, const double* __restrict__ kappa,
                                                 DevParams P, int64_t nF, SlotRec<R>* __restrict__ recs) {
  constexpr int W = sizeof(SlotRec<R>) / 8;
  constexpr int NT = elem_threads<R>();
  __shared__ uint2 lrec[4 * NT * W];
  const int64_t t0 = (int64_t)blockIdx.x * NT;
  const int64_t t = t0 + threadIdx.x;
  if (t < nE) {
    int v[4], sig[4], F[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      v[i] = tet[i * nE + t];
      if ((uint32_t)v[i] >= (uint64_t)nC) v[i] = 0;
      sig[i] = sigma[i * nE + t];
      F[i] = t2f[i * nE + t];
    }
    double x[4][3];
    gather_xa(XA, v, x);
    elem_records<R>(x, sig, F, kappa ? kappa[t] : P.kc, P, nF, lrec + 4 * threadIdx.x * W);
  }
  __syncthreads();
  const int64_t nb = nE - t0 < NT ? nE - t0 : NT;
  uint2* out = reinterpret_cast<uint2*>(recs + 4 * t0);
  for (int i = threadIdx.x; i < 4 * nb * W; i += NT) out[i] = lrec[i];
}

// One face's row from its owner's slot q0 and its neighbour's slot q1 (-1 on the boundary):
// the 6 (column, value) pairs unsorted (boundary: 3 pads INT_MAX / 0), diagonal, and the rhs
// b_D - r_owner - r_neighbour.
template <class R>
__device__ __forceinline__ void face_row(const SlotRec<R>* __restrict__ recs, int q0, int q1, double bD,
                                         const DevParams& P, int (&cf)[6], double (&cv)[6], double& dg,
                                         double& rh) {
  const SlotRec<R> a = recs[q0];  // owner's slot: row k of its element block
  dg = (double)a.d;
  rh = bD - (double)a.r;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    cf[i] = a.c[i];
    cv[i] = (double)a.o[i];
  }
  if (q1 >= 0) {
    const SlotRec<R> bq = recs[q1];  // neighbour's slot
    dg += (double)bq.d;
    rh -= (double)bq.r;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      cf[3 + i] = bq.c[i];
      cv[3 + i] = (double)bq.o[i];
    }
  } else {
#pragma unroll
    for (int i = 3; i < 6; ++i) {
      cf[i] = INT_MAX;  // sorts last; written as column F with value 0
      cv[i] = 0.0;
    }
  }
  if (P.nm) {  // columns of Neumann faces carry no coupling
#pragma unroll
    for (int i = 0; i < 6; ++i)
      if (cf[i] != INT_MAX && (cf[i] & 0x80000000)) {
        cf[i] &= 0x7fffffff;
        cv[i] = 0.0;
      }
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

// rowptr and col are written only when given (null: the pattern an earlier call wrote for the
// same connectivity is reused).
template <class R>
__global__ __launch_bounds__(FT) void k_face_rows(int64_t nF, int64_t nC, const double* __restrict__ X,
                                                  const int32_t* __restrict__ faces,
                                                  const int32_t* __restrict__ face2tet, DevParams P,
                                                  const SlotRec<R>* __restrict__ recs, int32_t* __restrict__ rowptr,
                                                  int32_t* __restrict__ col, double* __restrict__ val,
                                                  double* __restrict__ diag, double* __restrict__ rhs) {
  __shared__ int32_t lcol[6 * FT];
  __shared__ double lval[6 * FT];
  const int64_t f0 = (int64_t)blockIdx.x * FT;
  const int64_t f = f0 + threadIdx.x;
  const int nb = nF - f0 < FT ? (int)(nF - f0) : FT;
  const int base = 6 * (int)(f - f0);
  if (f < nF) {
    const int q0 = face2tet[f], q1 = face2tet[nF + f];
    const double bD = face_bD(nF, nC, X, faces, P, f, q1);
    int cf[6], rk[6];
    double cv[6], dg, rh;
    face_row<R>(recs, q0, q1, bD, P, cf, cv, dg, rh);
    col_ranks(cf, rk);
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      lcol[base + rk[i]] = cf[i] == INT_MAX ? (int32_t)f : cf[i];
      lval[base + rk[i]] = cv[i];
    }
    st_nt(diag + f, dg);
    st_nt(rhs + f, rh);
    if (rowptr) {
      st_nt(rowptr + f, (int32_t)(6 * f));
      if (f == nF - 1) rowptr[nF] = (int32_t)(6 * nF);
    }
  }
  __syncthreads();
  if (col) {
    for (int i = threadIdx.x; i < 6 * nb; i += FT) {
      st_nt(col + 6 * f0 + i, lcol[i]);
      st_nt(val + 6 * f0 + i, lval[i]);
    }
  } else {
    for (int i = threadIdx.x; i < 6 * nb; i += FT) st_nt(val + 6 * f0 + i, lval[i]);
  }
}

// ---------------------------------------------------------------- recovery / residual (FP64)
// U(T) = A^-1 (Bsrc + C' lambda) with Bsrc = load vector (gsrc == null) or gsrc[4][nE];
// res[F] -= (C U)_k for every local face when res != null (res preset to b_D or 0).
__global__ __launch_bounds__(FT) void k_recover(int64_t nC, const double* __restrict__ X, int64_t nE,
                                                const int32_t* __restrict__ tet, const int32_t* __restrict__ t2f,
                                                const int8_t* __restrict__ sigma, const double* __restrict__ kappa,
                                                DevParams P, const double* __restrict__ lambda,
                                                const double* __restrict__ gsrc, double* __restrict__ U,
                                                double* __restrict__ res, int* __restrict__ flags) {
  int64_t t = (int64_t)blockIdx.x * FT + threadIdx.x;
  if (t >= nE) return;
  int v[4], sig[4], F[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    v[i] = tet[i * nE + t];
    sig[i] = sigma[i * nE + t];
    F[i] = t2f[i * nE + t];
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
  if (lambda) {
#pragma unroll
    for (int k = 0; k < 4; ++k) mu[k] = E.d[k] * (neu[k] ? gN[k] : lambda[F[k]]);
  } else {
#pragma unroll
    for (int k = 0; k < 4; ++k) mu[k] = neu[k] ? E.d[k] * gN[k] : 0.0;
  }
  const double s = ((B[0] + B[1]) + (B[2] + B[3]) + ((mu[0] + mu[1]) + (mu[2] + mu[3]))) * E.icv;
  double y[4], u[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) y[i] = B[i] - mu[opp(i)] / 3.0;  // face opposite vertex i is opp(i)
#pragma unroll
  for (int i = 0; i < 4; ++i) u[i] = s + (E.W[i][0] * y[0] + E.W[i][1] * y[1] + E.W[i][2] * y[2] + E.W[i][3] * y[3]);
  if (U) {
#pragma unroll
    for (int i = 0; i < 4; ++i) U[i * nE + t] = u[i];
  }
  if (res) {
    const double su = (u[0] + u[1]) + (u[2] + u[3]);
#pragma unroll
    for (int k = 0; k < 4; ++k)  // a Neumann row is lambda_F = g
      atomicAdd(&res[F[k]], neu[k] ? gN[k] - (lambda ? lambda[F[k]] : 0.0) : -E.d[k] * (su - u[opp(k)]) / 3.0);
  }
}

// ---------------------------------------------------------------- adjoint VJP (FP64)
// G_i = dPhi_T/dx_i for Phi_T = P'A U - lambda'C P - P'B - Q'C U + sum_bnd Q_F b_D,F;
// dJ/dX_v -= G_i, dJ/dlog kappa_T = -kappa vol gP.gU.
__global__ __launch_bounds__(FT) void k_vjp(int64_t nC, const double* __restrict__ X, int64_t nE,
                                            const int32_t* __restrict__ tet, const int32_t* __restrict__ t2f,
                                            const int8_t* __restrict__ sigma, const int32_t* __restrict__ nbr,
                                            const double* __restrict__ kappa, DevParams P,
                                            const double* __restrict__ Uu, const double* __restrict__ Pp,
                                            const double* __restrict__ lambda, const double* __restrict__ Q,
                                            double* __restrict__ dlogk, double* __restrict__ dX) {
  int64_t t = (int64_t)blockIdx.x * FT + threadIdx.x;
  if (t >= nE) return;
  int v[4], sig[4];
  double U[4], Pv[4], lam[4], Qf[4];
  bool bnd[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    v[i] = tet[i * nE + t];
    sig[i] = sigma[i * nE + t];
    int Fi = t2f[i * nE + t];
    lam[i] = lambda[Fi];
    Qf[i] = Q[Fi];
    bnd[i] = nbr[i * nE + t] < 0;
    U[i] = Uu[i * nE + t];
    Pv[i] = Pp[i * nE + t];
  }
  double x[4][3];
  gather_x(nC, X, v, x);
  const double kap = kappa ? kappa[t] : P.kc;
  Elem<double> E;
  if (!E.init(x, kap, P.c, sig)) return;
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
int launch_recover(int64_t nC, const double* X, int64_t nE, const int32_t* tet, const int32_t* t2f,
                   const int8_t* sigma, const double* kappa, const DevParams& P, const double* lambda,
                   const double* gsrc, double* U, double* res, int* flags, hipStream_t s) {
  const double bytes = (36.0 + (kappa ? 8.0 : 0.0) + (gsrc ? 32.0 : 0.0) + (U ? 32.0 : 0.0)) * nE + 24.0 * nC +
                       (lambda ? 8.0 : 0.0) * nE + (res ? 16.0 : 0.0) * nE;
  PH_LAUNCH_B("recover", bytes, k_recover, grid_for(nE, FT), FT, 0, s, nC, X, nE, tet, t2f, sigma, kappa, P, lambda,
              gsrc, U, res, flags);
  return PHFEM_OK;
}

int launch_face_init(int64_t nF, int64_t nC, const double* X, const int32_t* faces, const int32_t* face2tet,
                     const DevParams& P, uint32_t* cnt, double* diag, double* rhs, hipStream_t s) {
  PH_LAUNCH_B("face_init", (8.0 + (cnt ? 4.0 : 0.0) + (diag ? 8.0 : 0.0) + (rhs ? 8.0 : 0.0)) * nF, k_face_init,
              grid_for(nF + 1, FT), FT, 0, s, nF, nC, X, faces, face2tet, P, cnt, diag, rhs);
  return PHFEM_OK;
}

int launch_vjp(int64_t nC, const double* X, int64_t nE, const int32_t* tet, const int32_t* t2f, const int8_t* sigma,
               const int32_t* nbr, const double* kappa, const DevParams& P, const double* U, const double* Pp,
               const double* lambda, const double* Q, double* dlogk, double* dX, hipStream_t s) {
  PH_LAUNCH_B("vjp", (124.0 + (kappa ? 8.0 : 0.0)) * nE + 16.0 * nE + 72.0 * nC, k_vjp, grid_for(nE, FT), FT, 0, s, nC,
              X, nE, tet, t2f, sigma, nbr, kappa, P, U, Pp, lambda, Q, dlogk, dX);
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

extern "C" size_t phfem_condense_batch_workspace(int64_t nC, int64_t nE, int64_t nF, int32_t precision,
                                                 int32_t nk) {
  (void)nF;
  if (nk < 1) return 0;
  Arena a;  // the AoS coordinates and one field's slot records (the fields run in turn)
  a.take<double4>(nC);
  if (precision == PHFEM_MIXED)
    a.take<SlotRec<float>>(4 * nE);
  else
    a.take<SlotRec<double>>(4 * nE);
  return a.size();
}

extern "C" size_t phfem_condense_workspace(int64_t nC, int64_t nE, int64_t nF, int32_t precision) {
  return phfem_condense_batch_workspace(nC, nE, nF, precision, 1);
}

extern "C" int phfem_condense_batch(int64_t nC, const double* coord, int64_t nE, const int32_t* tetra, int64_t nF,
                                    const int32_t* faces, const int32_t* tet2face, const int8_t* sigma,
                                    const int32_t* face2tet, int32_t nk, const double* kappa, const phfem_params* p,
                                    void* work, size_t work_bytes, int32_t* rowptr, int32_t* col, double* val,
                                    double* diag, double* rhs, phfem_stream_t stream_) {
  clear_error();
  hipStream_t s = (hipStream_t)stream_;
  int rc = check_params(p);
  if (rc) return rc;
  if (nC <= 0 || nE <= 0 || nF <= 0 || !coord || !tetra || !faces || !tet2face || !sigma || !face2tet || !val ||
      !diag || !rhs)
    return err(PHFEM_EINVAL, "bad condense arguments");
  if (nk < 1 || (nk > 1 && !kappa)) return err(PHFEM_EINVAL, "nk >= 1 coefficient fields (kappa required for nk > 1)");
  if ((rowptr == nullptr) != (col == nullptr)) return err(PHFEM_EINVAL, "rowptr and col: both or neither");
  if (6 * nF >= (int64_t(1) << 31)) return err(PHFEM_EINVAL, "face system exceeds int32 indexing");
  if (!work || work_bytes < phfem_condense_batch_workspace(nC, nE, nF, p->precision, nk))
    return err(PHFEM_EWORKSPACE, "condense workspace too small");
  Arena a(work, work_bytes);
  const bool mixed = p->precision == PHFEM_MIXED;
  double4* XA = a.take<double4>(nC);
  void* recs = mixed ? (void*)a.take<SlotRec<float>>(4 * nE) : (void*)a.take<SlotRec<double>>(4 * nE);
  DevParams P = to_dev(*p);
  // algorithmic bytes per field: tets, faces, sigma (+ kappa) once per tet, four records per
  // tet written once and read once, face2tet once, every off-diagonal value, diagonal and rhs
  // written once, the pattern (col + row pointer) once when written; coordinates once per call
  const double rb = 4.0 * (double)(mixed ? sizeof(SlotRec<float>) : sizeof(SlotRec<double>));
  const double eb = (36.0 + (kappa ? 8.0 : 0.0)) * nE + 24.0 * nC + rb * nE;
  const double fbv = rb * nE + 8.0 * nF + (8.0 * 6.0 + 16.0) * nF, fbp = 4.0 * 7.0 * nF;
  const unsigned gf = grid_for(nF, FT);
  PH_LAUNCH_B("coords_aos", 56.0 * nC, k_coords_aos, grid_for(nC, FT), FT, 0, s, nC, coord, XA);
  for (int j = 0; j < nk; ++j) {
    // field j; the pattern (when asked for) with the first field only
    const double* kj = kappa ? kappa + j * nE : nullptr;
    int32_t* rp = j == 0 ? rowptr : nullptr;
    int32_t* cl = j == 0 ? col : nullptr;
    double *vj = val + j * 6 * nF, *dj = diag + j * nF, *rj = rhs + j * nF;
    const double fb = fbv + (cl ? fbp : 0.0);
    if (mixed) {
      PH_LAUNCH_B("elem_rec_f32", eb, k_elem_rec<float>, grid_for(nE, elem_threads<float>()), elem_threads<float>(), 0,
                  s, nC, XA, nE, tetra, tet2face, sigma, kj, P, nF, (SlotRec<float>*)recs);
      PH_LAUNCH_B("face_rows_f32", fb, k_face_rows<float>, gf, FT, 0, s, nF, nC, coord, faces, face2tet, P,
                  (const SlotRec<float>*)recs, rp, cl, vj, dj, rj);
    } else {
      PH_LAUNCH_B("elem_rec_f64", eb, k_elem_rec<double>, grid_for(nE, elem_threads<double>()), elem_threads<double>(),
                  0, s, nC, XA, nE, tetra, tet2face, sigma, kj, P, nF, (SlotRec<double>*)recs);
      PH_LAUNCH_B("face_rows_f64", fb, k_face_rows<double>, gf, FT, 0, s, nF, nC, coord, faces, face2tet, P,
                  (const SlotRec<double>*)recs, rp, cl, vj, dj, rj);
    }
  }
  return PHFEM_OK;
}

extern "C" int phfem_condense(int64_t nC, const double* coord, int64_t nE, const int32_t* tetra, int64_t nF,
                              const int32_t* faces, const int32_t* tet2face, const int8_t* sigma, const int32_t* nbr,
                              const int32_t* face2tet, const double* kappa, const phfem_params* p, void* work,
                              size_t work_bytes, int32_t* rowptr, int32_t* col, double* val, double* diag,
                              double* rhs, phfem_stream_t stream) {
  (void)nbr;
  if (!rowptr || !col) {
    clear_error();
    return err(PHFEM_EINVAL, "bad condense arguments");
  }
  return phfem_condense_batch(nC, coord, nE, tetra, nF, faces, tet2face, sigma, face2tet, 1, kappa, p, work,
                              work_bytes, rowptr, col, val, diag, rhs, stream);
}
