// Several right-hand sides on one face system (Algorithm 1: one condensed matrix S serves
// every load; the loads differ in f, u_D, g).  NK independent Jacobi-PCG recurrences run in
// lockstep on the Jacobi-scaled FP64 copy of the system, so each iteration reads the matrix
// (6 column ids and 6 values per row) once for all of them: the vectors are interleaved
// ([nF][NK]), so a column's NK entries arrive together.  Each recurrence keeps its own
// alpha and beta; one that has met its tolerance is frozen (alpha = 0).  Then, as in
// phfem_solve's FP64 mode, the true residual b_D - C U(lambda) of every right-hand side is
// evaluated per tet in FP64 and correction solves (again all columns in lockstep) run while
// any stays above tol.  The right-hand sides r+ = b_D - C A^-1 B themselves are the true
// residuals at lambda = 0 unless the caller passes them.
#include <algorithm>
#include <cmath>
#include <string>

#include "common.hpp"

namespace ph {

int launch_recover(int64_t nC, const double* X, int64_t nE, int64_t nF, const int32_t* tet, const int32_t* t2f,
                   const int8_t* sigma, const int32_t* face2tet, const double* kappa, const DevParams& P,
                   const double* lambda, const double* gsrc, const double* bD, double* U, double* cu, double* res,
                   int* flags, hipStream_t s);
int launch_face_init(int64_t nF, int64_t nC, const double* X, const int32_t* faces, const int32_t* face2tet,
                     const DevParams& P, uint32_t* cnt, double* diag, double* rhs, int* flags, hipStream_t s);

constexpr int MT = 256;
constexpr int MG = 1024;        // at most MG workgroups (grid-stride)
constexpr int MAX_NK = 8;
constexpr int MCHECK = 16;      // iterations between host reads of the residual norms
constexpr int MREFRESH = 256;   // iterations between exact products q = A p

static unsigned mgrid(int64_t n) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + MT - 1) / MT, MG));
}

// NK block sums of one value per thread each, fixed order; results valid in all threads
template <int NK>
__device__ __forceinline__ void block_sums(double (&v)[NK], double* lds) {
#pragma unroll
  for (int j = 0; j < NK; ++j) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v[j] += __shfl_down(v[j], o, 64);
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) {
#pragma unroll
    for (int j = 0; j < NK; ++j) lds[j * (MT / 64) + w] = v[j];
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < NK; ++j) {
    const double* l = lds + j * (MT / 64);
    v[j] = (l[0] + l[1]) + (l[2] + l[3]);
  }
  __syncthreads();
}

// column sums of part[G][NK] (fixed order), in every thread
template <int NK>
__device__ __forceinline__ void sum_cols(const double* __restrict__ part, int G, double (&v)[NK], double* lds) {
#pragma unroll
  for (int j = 0; j < NK; ++j) v[j] = 0.0;
  for (int i = threadIdx.x; i < G; i += MT) {
#pragma unroll
    for (int j = 0; j < NK; ++j) v[j] += part[i * NK + j];
  }
  block_sums<NK>(v, lds);
}

template <int NK>
__device__ __forceinline__ void store_partials(double (&v)[NK], double* __restrict__ part) {
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < NK; ++j) part[blockIdx.x * NK + j] = v[j];
  }
}

// scalars (device, double): rz[2][NK] (current / previous r.r of the scaled system), act[NK]
// (1 = still iterating), rr[NK] (unscaled ||r||^2 of the update before), bb[NK] (||b||^2)
struct MScal {
  double* rz;
  double* act;
  double* rr;
  double* bb;
};

// r = D^-1/2 b (b: NK arrays of nF, or null for zero), x = 0, p = r; partial r.r and b.b
template <int NK>
__global__ __launch_bounds__(MT) void k_minit(int64_t n, const double* __restrict__ b, int64_t bstride,
                                              const double* __restrict__ diag, double* __restrict__ x,
                                              double* __restrict__ r, double* __restrict__ p,
                                              double* __restrict__ part_rz, double* __restrict__ part_bb) {
  __shared__ double lds[MT / 64 * NK];
  double arz[NK], abb[NK];
#pragma unroll
  for (int j = 0; j < NK; ++j) arz[j] = abb[j] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * MT + threadIdx.x; i < n; i += (int64_t)gridDim.x * MT) {
    const double sd = std::sqrt(diag[i]);
#pragma unroll
    for (int j = 0; j < NK; ++j) {
      const double bi = b[j * bstride + i];
      const double ri = bi / sd;
      x[i * NK + j] = 0.0;
      r[i * NK + j] = ri;
      p[i * NK + j] = ri;
      arz[j] += ri * ri;
      abb[j] += bi * bi;
    }
  }
  block_sums<NK>(arz, lds);
  store_partials<NK>(arz, part_rz);
  block_sums<NK>(abb, lds);
  store_partials<NK>(abb, part_bb);
}

// after init: rz[0] = sum part_rz, bb = sum part_bb, act = (bb > 0)
template <int NK>
__global__ __launch_bounds__(MT) void k_mscal0(int G, const double* __restrict__ part_rz,
                                               const double* __restrict__ part_bb, MScal S) {
  __shared__ double lds[MT / 64 * NK];
  double a[NK], b[NK];
  sum_cols<NK>(part_rz, G, a, lds);
  sum_cols<NK>(part_bb, G, b, lds);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < NK; ++j) {
      S.rz[j] = a[j];
      S.rz[NK + j] = a[j];
      S.bb[j] = b[j];
      S.rr[j] = b[j];
      S.act[j] = b[j] > 0.0 ? 1.0 : 0.0;
    }
  }
}

// the fused direction step: p = r + beta p and q = A r + beta q (A the scaled system, unit
// diagonal), partial p.q; beta_j = rz_new / rz_old from the update's partials (0 first)
// rz[slot] holds r.r of the previous residual; rz[slot ^ 1] receives the current one (block 0)
template <int NK, bool FUSED>
__global__ __launch_bounds__(MT) void k_mdir(int64_t n, const int32_t* __restrict__ col, const double* __restrict__ val,
                                             const double* __restrict__ r, double* __restrict__ p,
                                             double* __restrict__ q, int G, const double* __restrict__ part_rz,
                                             MScal S, int slot, int first, double* __restrict__ part_pq) {
  __shared__ double lds[MT / 64 * NK];
  double rzn[NK], beta[NK], apq[NK];
  const double* rzo = S.rz + slot * NK;
  if (first) {
#pragma unroll
    for (int j = 0; j < NK; ++j) rzn[j] = rzo[j];
  } else {
    sum_cols<NK>(part_rz, G, rzn, lds);
  }
#pragma unroll
  for (int j = 0; j < NK; ++j) {
    beta[j] = first || S.act[j] == 0.0 || rzo[j] == 0.0 ? 0.0 : rzn[j] / rzo[j];
    apq[j] = 0.0;
  }
  for (int64_t i = (int64_t)blockIdx.x * MT + threadIdx.x; i < n; i += (int64_t)gridDim.x * MT) {
    double pi[NK];
#pragma unroll
    for (int j = 0; j < NK; ++j) pi[j] = first ? r[i * NK + j] : r[i * NK + j] + beta[j] * p[i * NK + j];
    if (!FUSED) {
#pragma unroll
      for (int j = 0; j < NK; ++j) p[i * NK + j] = pi[j];
      continue;
    }
    const int2* c2 = reinterpret_cast<const int2*>(col + 6 * i);
    const double2* v2 = reinterpret_cast<const double2*>(val + 6 * i);
    const int2 c01 = c2[0], c23 = c2[1], c45 = c2[2];
    const double2 v01 = v2[0], v23 = v2[1], v45 = v2[2];
    const int cc[6] = {c01.x, c01.y, c23.x, c23.y, c45.x, c45.y};
    const double vv[6] = {v01.x, v01.y, v23.x, v23.y, v45.x, v45.y};
    double s[NK];
#pragma unroll
    for (int j = 0; j < NK; ++j) s[j] = r[i * NK + j];
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      const double* rc = r + (int64_t)cc[m] * NK;
#pragma unroll
      for (int j = 0; j < NK; ++j) s[j] += vv[m] * rc[j];
    }
#pragma unroll
    for (int j = 0; j < NK; ++j) {
      const double qi = first ? s[j] : s[j] + beta[j] * q[i * NK + j];
      p[i * NK + j] = pi[j];
      q[i * NK + j] = qi;
      apq[j] += pi[j] * qi;
    }
  }
  if (FUSED) {
    block_sums<NK>(apq, lds);
    store_partials<NK>(apq, part_pq);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < NK; ++j) S.rz[(slot ^ 1) * NK + j] = rzn[j];
  }
}

// q = A p exactly (the refresh of the fused recurrence), partial p.q
template <int NK>
__global__ __launch_bounds__(MT) void k_mspmv(int64_t n, const int32_t* __restrict__ col, const double* __restrict__ val,
                                              const double* __restrict__ p, double* __restrict__ q,
                                              double* __restrict__ part_pq) {
  __shared__ double lds[MT / 64 * NK];
  double apq[NK];
#pragma unroll
  for (int j = 0; j < NK; ++j) apq[j] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * MT + threadIdx.x; i < n; i += (int64_t)gridDim.x * MT) {
    const int2* c2 = reinterpret_cast<const int2*>(col + 6 * i);
    const double2* v2 = reinterpret_cast<const double2*>(val + 6 * i);
    const int2 c01 = c2[0], c23 = c2[1], c45 = c2[2];
    const double2 v01 = v2[0], v23 = v2[1], v45 = v2[2];
    const int cc[6] = {c01.x, c01.y, c23.x, c23.y, c45.x, c45.y};
    const double vv[6] = {v01.x, v01.y, v23.x, v23.y, v45.x, v45.y};
    double s[NK];
#pragma unroll
    for (int j = 0; j < NK; ++j) s[j] = p[i * NK + j];
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      const double* pc = p + (int64_t)cc[m] * NK;
#pragma unroll
      for (int j = 0; j < NK; ++j) s[j] += vv[m] * pc[j];
    }
#pragma unroll
    for (int j = 0; j < NK; ++j) {
      q[i * NK + j] = s[j];
      apq[j] += p[i * NK + j] * s[j];
    }
  }
  block_sums<NK>(apq, lds);
  store_partials<NK>(apq, part_pq);
}

// alpha_j = rz_j / pq_j (0 for a frozen column); x += alpha p, r -= alpha q; partial r.r and
// the unscaled sum d_i r_i^2
template <int NK>
__global__ __launch_bounds__(MT) void k_mupdate(int64_t n, int G, const double* __restrict__ part_pq, MScal S,
                                                int slot, double* __restrict__ x, double* __restrict__ r,
                                                const double* __restrict__ p, const double* __restrict__ q,
                                                const double* __restrict__ diag, double* __restrict__ part_rz,
                                                double* __restrict__ part_rr) {
  __shared__ double lds[MT / 64 * NK];
  double pq[NK], alpha[NK], arz[NK], arr[NK];
  sum_cols<NK>(part_pq, G, pq, lds);
#pragma unroll
  for (int j = 0; j < NK; ++j) {
    alpha[j] = S.act[j] != 0.0 && pq[j] != 0.0 ? S.rz[slot * NK + j] / pq[j] : 0.0;
    arz[j] = arr[j] = 0.0;
  }
  for (int64_t i = (int64_t)blockIdx.x * MT + threadIdx.x; i < n; i += (int64_t)gridDim.x * MT) {
    const double d = diag[i];
#pragma unroll
    for (int j = 0; j < NK; ++j) {
      x[i * NK + j] += alpha[j] * p[i * NK + j];
      const double ri = r[i * NK + j] - alpha[j] * q[i * NK + j];
      r[i * NK + j] = ri;
      arz[j] += ri * ri;
      arr[j] += d * (ri * ri);
    }
  }
  block_sums<NK>(arz, lds);
  store_partials<NK>(arz, part_rz);
  block_sums<NK>(arr, lds);
  store_partials<NK>(arr, part_rr);
}

// rr_j = sum of the update's unscaled partials (for the host's convergence check)
template <int NK>
__global__ __launch_bounds__(MT) void k_mrr(int G, const double* __restrict__ part_rr, MScal S) {
  __shared__ double lds[MT / 64 * NK];
  double a[NK];
  sum_cols<NK>(part_rr, G, a, lds);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < NK; ++j) S.rr[j] = a[j];
  }
}

// out_j = D^-1/2 x_j, de-interleaved (add: out_j += ...)
template <int NK, bool ADD>
__global__ __launch_bounds__(MT) void k_munscale(int64_t n, const double* __restrict__ diag,
                                                 const double* __restrict__ x, double* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * MT + threadIdx.x; i < n; i += (int64_t)gridDim.x * MT) {
    const double sd = std::sqrt(diag[i]);
#pragma unroll
    for (int j = 0; j < NK; ++j) {
      const double v = x[i * NK + j] / sd;
      if (ADD)
        out[j * n + i] += v;
      else
        out[j * n + i] = v;
    }
  }
}

__global__ __launch_bounds__(MT) void k_mnorm2(int64_t n, const double* __restrict__ v, double* __restrict__ part) {
  __shared__ double lds[MT / 64];
  double a[1] = {0.0};
  for (int64_t i = (int64_t)blockIdx.x * MT + threadIdx.x; i < n; i += (int64_t)gridDim.x * MT) a[0] += v[i] * v[i];
  block_sums<1>(a, lds);
  store_partials<1>(a, part);
}

__global__ __launch_bounds__(MT) void k_msum1(int G, const double* __restrict__ part, double* __restrict__ out) {
  __shared__ double lds[MT / 64];
  double a[1];
  sum_cols<1>(part, G, a, lds);
  if (threadIdx.x == 0) *out = a[0];
}

__global__ __launch_bounds__(MT) void k_mscale_f64(int64_t n, const int32_t* __restrict__ col,
                                                   const double* __restrict__ val, const double* __restrict__ diag,
                                                   double* __restrict__ vals) {
  for (int64_t k = (int64_t)blockIdx.x * MT + threadIdx.x; k < 6 * n; k += (int64_t)gridDim.x * MT)
    vals[k] = val[k] / std::sqrt(diag[k / 6] * diag[col[k]]);
}

__global__ __launch_bounds__(MT) void k_mcheck_pattern(int64_t n, const int32_t* __restrict__ rowptr,
                                                       const int32_t* __restrict__ col, int* __restrict__ flag) {
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * MT + threadIdx.x; i <= n; i += (int64_t)gridDim.x * MT) {
    bad = bad || (int64_t)rowptr[i] != 6 * i;
    if (i < n)
      for (int m = 0; m < 6; ++m) bad = bad || (uint32_t)col[6 * i + m] >= (uint64_t)n;
  }
  if (bad) atomicOr(flag, 1);
}

struct MWS {
  double *x, *r, *p, *q;       // interleaved [nF][NK]
  double *part_pq, *part_rz, *part_rr, *part_bb;
  double* scal;                // rz[2 NK], act[NK], rr[NK], bb[NK], norms[NK + 1]
  double *vals, *bD, *b, *e;   // scaled copy 6 nF; b_D [NK][nF]; rhs / residual [NK][nF]; corrections [NK][nF]
  double* cu;                  // per-slot residual terms, 4 nE
  int* flags;
};

static void mlayout(Arena& a, int64_t nE, int64_t nF, int nk, MWS& w) {
  w.x = a.take<double>(nk * nF);
  w.r = a.take<double>(nk * nF);
  w.p = a.take<double>(nk * nF);
  w.q = a.take<double>(nk * nF);
  w.part_pq = a.take<double>(MG * MAX_NK);
  w.part_rz = a.take<double>(MG * MAX_NK);
  w.part_rr = a.take<double>(MG * MAX_NK);
  w.part_bb = a.take<double>(MG * MAX_NK);
  w.scal = a.take<double>(6 * MAX_NK + 1);
  w.vals = a.take<double>(6 * nF);
  w.bD = a.take<double>(nk * nF);
  w.b = a.take<double>(nk * nF);
  w.e = a.take<double>(nk * nF);
  w.cu = a.take<double>(4 * nE);
  w.flags = a.take<int>(16);
}

struct MCtx {
  int64_t nC, nE, nF;
  const double* X;
  const int32_t* faces;
  const int32_t* tet;
  const int32_t* t2f;
  const int8_t* sigma;
  const int32_t* face2tet;
  const double* kappa;
  const int32_t* col;
  const double* diag;
  hipStream_t s;
};

static int mread(const double* d, double* h, int n, hipStream_t s) {
  PH_HIP(hipMemcpyAsync(h, d, sizeof(double) * n, hipMemcpyDeviceToHost, s));
  PH_HIP(hipStreamSynchronize(s));
  return PHFEM_OK;
}

static int mnorm(const MCtx& c, const double* v, MWS& w, double* out) {
  const unsigned G = mgrid(c.nF);
  PH_LAUNCH("mnorm2", k_mnorm2, G, MT, 0, c.s, c.nF, v, w.part_pq);
  PH_LAUNCH("msum1", k_msum1, 1, MT, 0, c.s, (int)G, (const double*)w.part_pq, w.scal + 6 * MAX_NK);
  double h = 0;
  int rc = mread(w.scal + 6 * MAX_NK, &h, 1, c.s);
  *out = std::sqrt(h);
  return rc;
}

// Lockstep Jacobi-PCG of NK columns: solves A y_j = b_j (b: [NK][nF]) from y = 0 to
// ||r_j|| <= tol_j ||b_j|| (unscaled 2-norms) or maxit; writes (ADD: adds) D^-1/2 y_j to
// out[j]; iters = lockstep iterations run.
template <int NK, bool ADD>
static int mpcg(const MCtx& c, MWS& w, const double* b, const double* tol, int maxit, double* out, int* iters) {
  const int64_t n = c.nF;
  const unsigned G = mgrid(n);
  MScal S{w.scal, w.scal + 2 * NK, w.scal + 3 * NK, w.scal + 4 * NK};
  PH_LAUNCH("mpcg_init", k_minit<NK>, G, MT, 0, c.s, n, b, n, c.diag, w.x, w.r, w.p, w.part_rz, w.part_bb);
  PH_LAUNCH("mpcg_scal", k_mscal0<NK>, 1, MT, 0, c.s, (int)G, (const double*)w.part_rz, (const double*)w.part_bb, S);
  double h[5 * MAX_NK];
  int rc = mread(w.scal, h, 5 * NK, c.s);
  if (rc) return rc;
  double bb[NK], act[NK];
  bool any = false;
  for (int j = 0; j < NK; ++j) {
    bb[j] = h[4 * NK + j];
    act[j] = h[2 * NK + j] != 0.0 && tol[j] < 1.0 ? 1.0 : 0.0;  // tol >= 1: a column left out
    any = any || act[j] != 0.0;
  }
  PH_HIP(hipMemcpyAsync(S.act, act, sizeof(double) * NK, hipMemcpyHostToDevice, c.s));
  int it = 0, slot = 0;
  while (any && it < maxit) {
    const bool first = it == 0;
    const double bytes = (double)n * (6.0 * 12.0 + NK * 8.0 * 5.0);  // matrix once, 5 vector streams per column
    if (!first && it % MREFRESH == 0) {
      PH_LAUNCH("mpcg_dir", (k_mdir<NK, false>), G, MT, 0, c.s, n, c.col, (const double*)w.vals,
                (const double*)w.r, w.p, w.q, (int)G, (const double*)w.part_rz, S, slot, 0, w.part_pq);
      PH_LAUNCH("mpcg_spmv", k_mspmv<NK>, G, MT, 0, c.s, n, c.col, (const double*)w.vals, (const double*)w.p, w.q,
                w.part_pq);
    } else {
      PH_LAUNCH_B("mpcg_spmv_dir", bytes, (k_mdir<NK, true>), G, MT, 0, c.s, n, c.col, (const double*)w.vals,
                  (const double*)w.r, w.p, w.q, (int)G, (const double*)w.part_rz, S, slot, first ? 1 : 0,
                  w.part_pq);
    }
    PH_LAUNCH_B("mpcg_update", (double)n * (8.0 + NK * 8.0 * 6.0), k_mupdate<NK>, G, MT, 0, c.s, n, (int)G,
                (const double*)w.part_pq, S, slot ^ 1, w.x, w.r, (const double*)w.p, (const double*)w.q, c.diag,
                w.part_rz, w.part_rr);
    slot ^= 1;
    ++it;
    if (it % MCHECK == 0 || it == maxit) {
      PH_LAUNCH("mpcg_rr", k_mrr<NK>, 1, MT, 0, c.s, (int)G, (const double*)w.part_rr, S);
      rc = mread(S.rr, h, NK, c.s);
      if (rc) return rc;
      any = false;
      bool changed = false;
      for (int j = 0; j < NK; ++j) {
        if (act[j] != 0.0 && !(std::sqrt(h[j]) > tol[j] * std::sqrt(bb[j]))) {  // also stops on NaN
          act[j] = 0.0;
          changed = true;
        }
        any = any || act[j] != 0.0;
      }
      if (changed) PH_HIP(hipMemcpyAsync(S.act, act, sizeof(double) * NK, hipMemcpyHostToDevice, c.s));
    }
  }
  PH_LAUNCH("mpcg_unscale", (k_munscale<NK, ADD>), G, MT, 0, c.s, n, c.diag, (const double*)w.x, out);
  *iters = it;
  return PHFEM_OK;
}

template <int NK>
static int msolve(const MCtx& c, const DevParams* P, const double* rhs, double tol, int maxit, MWS& w,
                  double* lambda, double* U, phfem_solve_stats* st) {
  const int64_t nF = c.nF;
  // b_D of each right-hand side, the right-hand sides (given, or the true residuals at
  // lambda = 0) and their norms
  PH_HIP(hipMemsetAsync(w.flags, 0, 2 * sizeof(int), c.s));
  for (int j = 0; j < NK; ++j) {
    int rc = launch_face_init(nF, c.nC, c.X, c.faces, c.face2tet, P[j], nullptr, nullptr, w.bD + j * nF, w.flags,
                              c.s);
    if (rc) return rc;
  }
  double bn[NK];
  for (int j = 0; j < NK; ++j) {
    double* bj = w.b + j * nF;
    if (rhs) {
      PH_HIP(hipMemcpyAsync(bj, rhs + j * nF, sizeof(double) * nF, hipMemcpyDeviceToDevice, c.s));
    } else {
      int rc = launch_recover(c.nC, c.X, c.nE, nF, c.tet, c.t2f, c.sigma, c.face2tet, c.kappa, P[j], nullptr, nullptr,
                              w.bD + j * nF, nullptr, w.cu, bj, w.flags, c.s);
      if (rc) return rc;
    }
    int rc = mnorm(c, bj, w, &bn[j]);
    if (rc) return rc;
    st[j] = phfem_solve_stats{0, 0, 0.0, bn[j], 0, 0};
  }
  double tolj[NK], rn[NK] = {}, prev[NK] = {};
  for (int j = 0; j < NK; ++j) tolj[j] = tol;
  int its = 0;
  int rc = mpcg<NK, false>(c, w, w.b, tolj, maxit, lambda, &its);
  if (rc) return rc;
  int total = its;
  for (int j = 0; j < NK; ++j) st[j].iters = its;
  for (int steps = 0;; ++steps) {
    // true residuals (FP64, matrix-free), U on the way
    bool more = false;
    for (int j = 0; j < NK; ++j) {
      rc = launch_recover(c.nC, c.X, c.nE, nF, c.tet, c.t2f, c.sigma, c.face2tet, c.kappa, P[j], lambda + j * nF,
                          nullptr, w.bD + j * nF, U + j * 4 * c.nE, w.cu, w.b + j * nF, w.flags, c.s);
      if (rc) return rc;
      prev[j] = rn[j];
      rc = mnorm(c, w.b + j * nF, w, &rn[j]);
      if (rc) return rc;
      st[j].rel_res = bn[j] > 0 ? rn[j] / bn[j] : rn[j];
      // another correction while above tol, gaining, and within the budgets
      const bool need = rn[j] > tol * bn[j] && (steps == 0 || rn[j] < 0.5 * prev[j]);
      tolj[j] = need ? std::max(0.5 * tol * bn[j] / rn[j], 1e-12) : 2.0;  // 2: a column left out
      more = more || need;
    }
    int hf[2] = {0, 0};
    PH_HIP(hipMemcpyAsync(hf, w.flags, 2 * sizeof(int), hipMemcpyDeviceToHost, c.s));
    PH_HIP(hipStreamSynchronize(c.s));
    if (hf[0]) return dev_flags_to_status(hf[0]);
    if (!more || steps == 8 || total >= maxit) break;
    // corrections of every column still above tol (the others enter with tol 2, i.e. frozen)
    rc = mpcg<NK, true>(c, w, w.b, tolj, maxit - total, lambda, &its);
    if (rc) return rc;
    total += its;
    for (int j = 0; j < NK; ++j)
      if (tolj[j] < 1.0) {
        st[j].iters += its;
        st[j].ir_steps += 1;
      }
  }
  bool ok = true;
  for (int j = 0; j < NK; ++j) ok = ok && !(st[j].rel_res > tol);
  if (!ok) return err(PHFEM_ENOCONV, "a right-hand side stopped above tol (stats hold each one's rel_res)");
  return PHFEM_OK;
}

}  // namespace ph

using namespace ph;

extern "C" size_t phfem_solve_multi_workspace(int64_t nE, int64_t nF, int32_t nk) {
  if (nE <= 0 || nF <= 0 || nk < 1 || nk > MAX_NK) return 0;
  Arena a;
  MWS w;
  mlayout(a, nE, nF, nk, w);
  return a.size();
}

extern "C" int phfem_solve_multi(int64_t nC, const double* coord, int64_t nE, const int32_t* tetra, int64_t nF,
                                 const int32_t* faces, const int32_t* tet2face, const int8_t* sigma,
                                 const int32_t* face2tet,
                                 const double* kappa, int32_t nk, const phfem_params* p, const int32_t* rowptr,
                                 const int32_t* col, const double* val, const double* diag, const double* rhs,
                                 double tol, int32_t max_iter, void* work, size_t work_bytes, double* lambda, double* U,
                                 phfem_solve_stats* stats, phfem_stream_t stream_) {
  clear_error();
  hipStream_t s = (hipStream_t)stream_;
  if (nk < 1 || nk > MAX_NK || !p) return err(PHFEM_EINVAL, "nk must be in [1, 8] with nk params");
  for (int j = 0; j < nk; ++j) {
    int rc = check_params(p + j);
    if (rc) return rc;
    if (p[j].c != p[0].c || p[j].kappa_const != p[0].kappa_const || p[j].neumann != p[0].neumann ||
        p[j].precision != p[0].precision)
      return err(PHFEM_EINVAL, "the right-hand sides must share c, kappa, the Neumann flags and the precision "
                               "(one face system)");
  }
  if (p[0].neumann) return err(PHFEM_EINVAL, "phfem_solve_multi covers Dirichlet boundaries (params.neumann NULL)");
  if (nC <= 0 || nE <= 0 || nF <= 0 || !coord || !tetra || !faces || !tet2face || !sigma || !face2tet || !rowptr ||
      !col ||
      !val || !diag || !lambda || !U || !stats)
    return err(PHFEM_EINVAL, "bad solve arguments");
  if (!(tol >= 0) || max_iter <= 0) return err(PHFEM_EINVAL, "bad tolerance or max_iter");
  if ((reinterpret_cast<uintptr_t>(col) & 7) || (reinterpret_cast<uintptr_t>(val) & 15))
    return err(PHFEM_EINVAL, "col must be 8-byte and val 16-byte aligned");
  if (!work || work_bytes < phfem_solve_multi_workspace(nE, nF, nk))
    return err(PHFEM_EWORKSPACE, "solve_multi workspace too small");
  Arena a(work, work_bytes);
  MWS w;
  mlayout(a, nE, nF, nk, w);
  PH_HIP(hipMemsetAsync(w.flags, 0, 2 * sizeof(int), s));
  PH_LAUNCH("mcheck_pattern", k_mcheck_pattern, mgrid(nF + 1), MT, 0, s, nF, rowptr, col, w.flags + 1);
  int hf = 0;
  PH_HIP(hipMemcpyAsync(&hf, w.flags + 1, sizeof(int), hipMemcpyDeviceToHost, s));
  PH_HIP(hipStreamSynchronize(s));
  if (hf) return err(PHFEM_EINVAL, "face system is not the 6-slot layout of phfem_condense");
  PH_LAUNCH("mscale_f64", k_mscale_f64, mgrid(6 * nF), MT, 0, s, nF, col, val, diag, w.vals);
  DevParams P[MAX_NK];
  for (int j = 0; j < nk; ++j) P[j] = to_dev(p[j]);
  MCtx c{nC, nE, nF, coord, faces, tetra, tet2face, sigma, face2tet, kappa, col, diag, s};
  switch (nk) {
    case 1: return msolve<1>(c, P, rhs, tol, max_iter, w, lambda, U, stats);
    case 2: return msolve<2>(c, P, rhs, tol, max_iter, w, lambda, U, stats);
    case 3: return msolve<3>(c, P, rhs, tol, max_iter, w, lambda, U, stats);
    case 4: return msolve<4>(c, P, rhs, tol, max_iter, w, lambda, U, stats);
    case 5: return msolve<5>(c, P, rhs, tol, max_iter, w, lambda, U, stats);
    case 6: return msolve<6>(c, P, rhs, tol, max_iter, w, lambda, U, stats);
    case 7: return msolve<7>(c, P, rhs, tol, max_iter, w, lambda, U, stats);
    default: return msolve<8>(c, P, rhs, tol, max_iter, w, lambda, U, stats);
  }
}
