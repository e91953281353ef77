// Face-system solve (Jacobi-PCG; the paper uses a sparse direct solve, Listing 8), the
// mixed-precision iterative refinement, recovery (Algorithm 1) and the adjoint driver.
//
// PCG scalars never leave the device: every block of a consumer kernel re-sums the fixed
// array of per-block partial dot products in a fixed order, so alpha and beta are
// bitwise identical across blocks and runs.  The host reads one residual norm every
// CHECK iterations.
#include <cmath>

#include "common.hpp"

namespace ph {

int launch_recover(int64_t nC, const double* X, int64_t nE, int64_t nF, const int32_t* tet, const int32_t* t2f,
                   const int8_t* sigma, const int32_t* face2tet, const double* kappa, const DevParams& P,
                   const double* lambda, const double* gsrc, const double* bD, double* U, double* cu, double* res,
                   int* flags, hipStream_t s);
int launch_face_init(int64_t nF, int64_t nC, const double* X, const int32_t* faces, const int32_t* face2tet,
                     const DevParams& P, uint32_t* cnt, double* diag, double* rhs, int* flags, hipStream_t s);
int launch_vjp(int64_t nC, const double* X, int64_t nE, int64_t nF, const int32_t* tet, const int32_t* t2f,
               const int8_t* sigma, const int32_t* nbr, const double* kappa, const DevParams& P, const double* U,
               const double* Pp, const double* lambda, const double* Q, double* dlogk, double* dX, int* flags,
               hipStream_t s);

constexpr int ST = 256;
constexpr int MAXG = 1024;
constexpr int CHECK = 16;
constexpr int REFRESH = 256;  // iterations between exact products q = A p (fused recurrence)
constexpr int FORCE = 2048;  // iterations after which a residual replacement is forced
constexpr int POLISH_MIN = 1;      // FP64 correction solves after the mixed refinement (at least)
constexpr int POLISH_MAX = 3;      // (at most; each must halve the true residual to continue)
constexpr double POLISH_TOL = 0.1;  // relative tolerance of each FP64 correction solve

static unsigned pcg_grid(int64_t n) {
  int64_t g = (n + ST - 1) / ST;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, MAXG));
}

// block-wide sum of one double per thread, fixed order; result valid in all threads
__device__ __forceinline__ double block_sum(double v, double* lds) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) lds[w] = v;
  __syncthreads();
  double s = (lds[0] + lds[1]) + (lds[2] + lds[3]);
  __syncthreads();
  return s;
}

__device__ __forceinline__ double sum_partials(const double* __restrict__ part, int G, double* lds) {
  double v = 0.0;
  for (int i = threadIdx.x; i < G; i += ST) v += part[i];
  return block_sum(v, lds);
}

// The face system's fixed 6-slot rows (rowptr[i] = 6 i, as phfem_condense writes them):
// y = (D + offdiag) x and the partial dots x.y (UNIT: a unit diagonal, not read).  A row's 6
// column ids and values are read as three 8-byte (int2) and three 16- or 8-byte (double2 /
// float2) vector loads; the products are summed in slot order, as a plain CSR loop would.
template <class T>
struct Vec2;
template <>
struct Vec2<double> {
  using type = double2;
};
template <>
struct Vec2<float> {
  using type = float2;
};

template <class T, bool UNIT>
__global__ __launch_bounds__(ST) void k_spmv_dot(int64_t n, const int32_t* __restrict__ col,
                                                 const T* __restrict__ val, const T* __restrict__ diag,
                                                 const T* __restrict__ x, T* __restrict__ y,
                                                 double* __restrict__ part) {
  using V2 = typename Vec2<T>::type;
  __shared__ double lds[ST / 64];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * ST + threadIdx.x; i < n; i += (int64_t)gridDim.x * ST) {
    const int2* c2 = reinterpret_cast<const int2*>(col + 6 * i);
    const V2* v2 = reinterpret_cast<const V2*>(val + 6 * i);
    const int2 c01 = c2[0], c23 = c2[1], c45 = c2[2];
    const V2 v01 = v2[0], v23 = v2[1], v45 = v2[2];
    const T xi = x[i];
    T s = UNIT ? xi : diag[i] * xi;
    s += v01.x * x[c01.x];
    s += v01.y * x[c01.y];
    s += v23.x * x[c23.x];
    s += v23.y * x[c23.y];
    s += v45.x * x[c45.x];
    s += v45.y * x[c45.y];
    y[i] = s;
    acc += (double)xi * (double)s;
  }
  double b = block_sum(acc, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = b;
}

// the pattern check run once per solve: rowptr[i] = 6 i and every column id in [0, nF)
__global__ __launch_bounds__(ST) void k_check_pattern(int64_t n, const int32_t* __restrict__ rowptr,
                                                      const int32_t* __restrict__ col, int* __restrict__ flags) {
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * ST + threadIdx.x; i <= n; i += (int64_t)gridDim.x * ST) {
    bad = bad || (int64_t)rowptr[i] != 6 * i;
    if (i < n)
      for (int q = 0; q < 6; ++q) bad = bad || (uint32_t)col[6 * i + q] >= (uint64_t)n;
  }
  if (bad) atomicOr(flags + 1, 1);
}

template <class T>
__global__ __launch_bounds__(ST) void k_pcg_init(int64_t n, const T* __restrict__ b, const T* __restrict__ diag,
                                                 T* __restrict__ x, T* __restrict__ r, T* __restrict__ z,
                                                 T* __restrict__ p, double* __restrict__ part_rz,
                                                 double* __restrict__ part_rr) {
  __shared__ double lds[ST / 64];
  double arz = 0.0, arr = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * ST + threadIdx.x; i < n; i += (int64_t)gridDim.x * ST) {
    T ri = b[i];
    T zi = ri / diag[i];
    x[i] = (T)0;
    r[i] = ri;
    z[i] = zi;
    p[i] = zi;
    arz += (double)ri * (double)zi;
    arr += (double)ri * (double)ri;
  }
  double s1 = block_sum(arz, lds);
  double s2 = block_sum(arr, lds);
  if (threadIdx.x == 0) {
    part_rz[blockIdx.x] = s1;
    part_rr[blockIdx.x] = s2;
  }
}

// the same start on the Jacobi-scaled system: r = D^-1/2 b, x = 0, p = r; partial r.r and
// the unscaled b.b (= sum d_i r_i^2)
template <class T>
__global__ __launch_bounds__(ST) void k_pcg_init_scaled(int64_t n, const T* __restrict__ b, const T* __restrict__ diag,
                                                        T* __restrict__ x, T* __restrict__ r, T* __restrict__ p,
                                                        double* __restrict__ part_rz, double* __restrict__ part_rr) {
  __shared__ double lds[ST / 64];
  double arz = 0.0, arr = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * ST + threadIdx.x; i < n; i += (int64_t)gridDim.x * ST) {
    const T bi = b[i];
    const T ri = bi / std::sqrt(diag[i]);
    x[i] = (T)0;
    r[i] = ri;
    p[i] = ri;
    arz += (double)ri * (double)ri;
    arr += (double)bi * (double)bi;
  }
  double s1 = block_sum(arz, lds);
  double s2 = block_sum(arr, lds);
  if (threadIdx.x == 0) {
    part_rz[blockIdx.x] = s1;
    part_rr[blockIdx.x] = s2;
  }
}

// x = D^-1/2 x (a scaled solution back in the original unknowns)
template <class T>
__global__ __launch_bounds__(ST) void k_unscale(int64_t n, const T* __restrict__ diag, T* __restrict__ x) {
  for (int64_t i = (int64_t)blockIdx.x * ST + threadIdx.x; i < n; i += (int64_t)gridDim.x * ST)
    x[i] = x[i] / std::sqrt(diag[i]);
}

// scal[slot] = sum part_rz, scal[2] = sum part_rr (single block)
__global__ __launch_bounds__(ST) void k_scalars(int G, const double* __restrict__ part_rz,
                                                const double* __restrict__ part_rr, double* __restrict__ scal,
                                                int slot) {
  __shared__ double lds[ST / 64];
  double a = sum_partials(part_rz, G, lds);
  double b = sum_partials(part_rr, G, lds);
  if (threadIdx.x == 0) {
    scal[slot] = a;
    scal[2] = b;
  }
}

// UNIT: the system has a unit diagonal (Jacobi-scaled), so z = r is not stored; the partial
// r.r is then weighted by diag when diag is given (the unscaled residual's 2-norm, sum d_i r_i^2)
template <class T, bool UNIT>
__global__ __launch_bounds__(ST) void k_pcg_update(int64_t n, int G, const double* __restrict__ part_pq,
                                                   const double* __restrict__ scal, int slot, T* __restrict__ x,
                                                   T* __restrict__ r, const T* __restrict__ p,
                                                   const T* __restrict__ q, const T* __restrict__ diag,
                                                   T* __restrict__ z, double* __restrict__ part_rz,
                                                   double* __restrict__ part_rr) {
  __shared__ double lds[ST / 64];
  const double pq = sum_partials(part_pq, G, lds);
  const double rz = scal[slot];
  const T alpha = (T)(rz / pq);
  double arz = 0.0, arr = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * ST + threadIdx.x; i < n; i += (int64_t)gridDim.x * ST) {
    x[i] += alpha * p[i];
    T ri = r[i] - alpha * q[i];
    r[i] = ri;
    T zi = ri;
    if (!UNIT) {
      zi = ri / diag[i];
      z[i] = zi;
    }
    arz += (double)ri * (double)zi;
    const double wi = (UNIT && diag) ? (double)diag[i] : 1.0;
    arr += wi * ((double)ri * (double)ri);
  }
  double s1 = block_sum(arz, lds);
  double s2 = block_sum(arr, lds);
  if (threadIdx.x == 0) {
    part_rz[blockIdx.x] = s1;
    part_rr[blockIdx.x] = s2;
  }
}

template <class T>
__global__ __launch_bounds__(ST) void k_pcg_dir(int64_t n, int G, const double* __restrict__ part_rz,
                                                const double* __restrict__ part_rr, double* __restrict__ scal,
                                                int slot_old, const T* __restrict__ z, T* __restrict__ p) {
  __shared__ double lds[ST / 64];
  const double rzn = sum_partials(part_rz, G, lds);
  const double rr = sum_partials(part_rr, G, lds);
  const T beta = (T)(rzn / scal[slot_old]);
  for (int64_t i = (int64_t)blockIdx.x * ST + threadIdx.x; i < n; i += (int64_t)gridDim.x * ST) p[i] = z[i] + beta * p[i];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    scal[slot_old ^ 1] = rzn;
    scal[2] = rr;
  }
}

// The direction update fused into the product: p = z + beta p and q = A z + beta q (= A p
// by linearity, A p_old being the q of the previous iteration) in one pass over the rows,
// with the partial dots p.q.  beta = (r.z)_new / (r.z)_old from the update kernel's
// partials, 0 on the first iteration; block 0 stores (r.z)_new in scal[slot_old ^ 1] and
// r.r in scal[2].  One kernel instead of two per iteration; the recurrence for q drifts
// from A p by rounding, so the solver recomputes q = A p exactly at intervals.
template <class T, bool UNIT>
__global__ __launch_bounds__(ST) void k_spmv_dir(int64_t n, const int32_t* __restrict__ col,
                                                 const T* __restrict__ val, const T* __restrict__ diag,
                                                 const T* __restrict__ z, T* __restrict__ p, T* __restrict__ q, int G,
                                                 const double* __restrict__ part_rz,
                                                 const double* __restrict__ part_rr, double* __restrict__ scal,
                                                 int slot_old, int first, double* __restrict__ part_pq) {
  using V2 = typename Vec2<T>::type;
  __shared__ double lds[ST / 64];
  const double rzn = sum_partials(part_rz, G, lds);
  const double rr = sum_partials(part_rr, G, lds);
  const T beta = first ? (T)0 : (T)(rzn / scal[slot_old]);
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * ST + threadIdx.x; i < n; i += (int64_t)gridDim.x * ST) {
    const int2* c2 = reinterpret_cast<const int2*>(col + 6 * i);
    const V2* v2 = reinterpret_cast<const V2*>(val + 6 * i);
    const int2 c01 = c2[0], c23 = c2[1], c45 = c2[2];
    const V2 v01 = v2[0], v23 = v2[1], v45 = v2[2];
    const T zi = z[i];
    T s = UNIT ? zi : diag[i] * zi;
    s += v01.x * z[c01.x];
    s += v01.y * z[c01.y];
    s += v23.x * z[c23.x];
    s += v23.y * z[c23.y];
    s += v45.x * z[c45.x];
    s += v45.y * z[c45.y];
    const T pi = first ? zi : zi + beta * p[i];
    const T qi = first ? s : s + beta * q[i];
    p[i] = pi;
    q[i] = qi;
    acc += (double)pi * (double)qi;
  }
  double b = block_sum(acc, lds);
  if (threadIdx.x == 0) part_pq[blockIdx.x] = b;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    scal[slot_old ^ 1] = rzn;
    scal[2] = rr;
  }
}

__global__ __launch_bounds__(ST) void k_norm2(int64_t n, const double* __restrict__ v, double* __restrict__ part) {
  __shared__ double lds[ST / 64];
  double a = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * ST + threadIdx.x; i < n; i += (int64_t)gridDim.x * ST) a += v[i] * v[i];
  double s = block_sum(a, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(ST) void k_sum1(int G, const double* __restrict__ part, double* __restrict__ out) {
  __shared__ double lds[ST / 64];
  double a = sum_partials(part, G, lds);
  if (threadIdx.x == 0) *out = a;
}

// The Jacobi-scaled FP32 copy of the system, D^-1/2 (D + offdiag) D^-1/2 with its unit
// diagonal implied: val32[6 i + q] = val[6 i + q] / sqrt(d_i d_col), rounded once from FP64.
// CG on it is Jacobi-PCG on the original system (iterates scaled by D^1/2) without the
// diagonal reads and the z vector.
__global__ __launch_bounds__(ST) void k_scale_f32(int64_t n, const int32_t* __restrict__ col,
                                                  const double* __restrict__ val, const double* __restrict__ diag,
                                                  float* __restrict__ val32) {
  for (int64_t k = (int64_t)blockIdx.x * ST + threadIdx.x; k < 6 * n; k += (int64_t)gridDim.x * ST) {
    const int64_t i = k / 6;
    val32[k] = (float)(val[k] / std::sqrt(diag[i] * diag[col[k]]));
  }
}

// the Jacobi-scaled FP64 copy, val64s[6 i + q] = val[6 i + q] / sqrt(d_i d_col)
__global__ __launch_bounds__(ST) void k_scale_f64(int64_t n, const int32_t* __restrict__ col,
                                                  const double* __restrict__ val, const double* __restrict__ diag,
                                                  double* __restrict__ vals) {
  for (int64_t k = (int64_t)blockIdx.x * ST + threadIdx.x; k < 6 * n; k += (int64_t)gridDim.x * ST) {
    const int64_t i = k / 6;
    vals[k] = val[k] / std::sqrt(diag[i] * diag[col[k]]);
  }
}

__global__ __launch_bounds__(ST) void k_add_f32(int64_t n, const float* __restrict__ d, double* __restrict__ x) {
  for (int64_t i = (int64_t)blockIdx.x * ST + threadIdx.x; i < n; i += (int64_t)gridDim.x * ST) x[i] += (double)d[i];
}

__global__ __launch_bounds__(ST) void k_add_f64(int64_t n, const double* __restrict__ d, double* __restrict__ x) {
  for (int64_t i = (int64_t)blockIdx.x * ST + threadIdx.x; i < n; i += (int64_t)gridDim.x * ST) x[i] += d[i];
}

// residual replacement of the scaled FP32 recurrence: r32 = (float) D^-1/2 r64; with init
// also p = r32, x32 = 0.  Partial r.r (= r.z of the unscaled system) into both partial
// arrays, as k_pcg_update<float, true> leaves them.
template <bool INIT>
__global__ __launch_bounds__(ST) void k_replace(int64_t n, const double* __restrict__ r64,
                                                const double* __restrict__ diag, float* __restrict__ r,
                                                float* __restrict__ p, float* __restrict__ x32,
                                                double* __restrict__ part_rz, double* __restrict__ part_rr) {
  __shared__ double lds[ST / 64];
  double arr = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * ST + threadIdx.x; i < n; i += (int64_t)gridDim.x * ST) {
    const float ri = (float)(r64[i] / std::sqrt(diag[i]));
    r[i] = ri;
    if (INIT) {
      p[i] = ri;
      x32[i] = 0.0f;
    }
    arr += (double)ri * (double)ri;
  }
  double s2 = block_sum(arr, lds);
  if (threadIdx.x == 0) {
    part_rz[blockIdx.x] = s2;
    part_rr[blockIdx.x] = s2;
  }
}

// x += D^-1/2 x32 (the scaled iterate back in the original unknowns), x32 = 0
__global__ __launch_bounds__(ST) void k_flush_x(int64_t n, const double* __restrict__ diag, float* __restrict__ x32,
                                                double* __restrict__ x) {
  for (int64_t i = (int64_t)blockIdx.x * ST + threadIdx.x; i < n; i += (int64_t)gridDim.x * ST) {
    x[i] += (double)x32[i] / std::sqrt(diag[i]);
    x32[i] = 0.0f;
  }
}

__global__ __launch_bounds__(ST) void k_fill0(int64_t n, double* __restrict__ x) {
  for (int64_t i = (int64_t)blockIdx.x * ST + threadIdx.x; i < n; i += (int64_t)gridDim.x * ST) x[i] = 0.0;
}

// ---------------------------------------------------------------- workspace
struct PcgWS {
  void *r, *z, *p, *q;
  double *part_pq, *part_rz, *part_rr, *scal;
};

template <class T>
static void pcg_layout(Arena& a, int64_t n, PcgWS& w) {
  w.r = a.take<T>(n);
  w.z = a.take<T>(n);
  w.p = a.take<T>(n);
  w.q = a.take<T>(n);
  w.part_pq = a.take<double>(MAXG);
  w.part_rz = a.take<double>(MAXG);
  w.part_rr = a.take<double>(MAXG);
  w.scal = a.take<double>(8);
}

struct SolveWS {
  PcgWS pcg, pcg64;  // pcg64: FP64 vectors of the mixed mode's FP64 polish
  double *bD, *r64, *e64, *val64s, *cu;
  float *val32, *x32;
  int* flags;
};

static void solve_layout(Arena& a, int64_t nE, int64_t nF, int32_t mode, SolveWS& w) {
  if (mode == PHFEM_SOLVE_FP32_PCG_FP64_IR)
    pcg_layout<float>(a, nF, w.pcg);
  else
    pcg_layout<double>(a, nF, w.pcg);
  w.bD = a.take<double>(nF);
  w.r64 = a.take<double>(nF);
  w.e64 = a.take<double>(nF);
  w.val64s = a.take<double>(6 * nF);
  if (mode == PHFEM_SOLVE_FP32_PCG_FP64_IR) {
    pcg_layout<double>(a, nF, w.pcg64);
    w.val32 = a.take<float>(6 * nF);
    w.x32 = a.take<float>(nF);
  } else {
    w.pcg64 = w.pcg;
    w.val32 = w.x32 = nullptr;
  }
  w.cu = a.take<double>(4 * nE);
  w.flags = a.take<int>(16);
}

static int read_scalar(const double* d, double* h, hipStream_t s) {
  PH_HIP(hipMemcpyAsync(h, d, sizeof(double), hipMemcpyDeviceToHost, s));
  PH_HIP(hipStreamSynchronize(s));
  return PHFEM_OK;
}

static int norm2(int64_t n, const double* v, PcgWS& w, double* out, hipStream_t s) {
  unsigned G = pcg_grid(n);
  PH_LAUNCH("norm2", k_norm2, G, ST, 0, s, n, v, w.part_pq);
  PH_LAUNCH("sum1", k_sum1, 1, ST, 0, s, (int)G, (const double*)w.part_pq, w.scal + 4);
  double h = 0;
  int rc = read_scalar(w.scal + 4, &h, s);
  *out = std::sqrt(h);
  return rc;
}

// Direction step of iteration it (before its update): p = z + beta p and q = A p, fused
// (k_spmv_dir) or, when `exact`, as the direction update followed by the plain product
// (resets the drift of the fused recurrence).  scal[slot] receives the new r.z.
template <class T, bool UNIT>
static int pcg_direction(int64_t n, const int32_t* col, const T* val, const T* diag, PcgWS& w, int slot, bool first,
                         bool exact, hipStream_t s) {
  const unsigned G = pcg_grid(n);
  T *z = UNIT ? (T*)w.r : (T*)w.z, *p = (T*)w.p, *q = (T*)w.q;
  if (exact && !first) {
    PH_LAUNCH_B("pcg_dir", 3.0 * sizeof(T) * n, k_pcg_dir<T>, G, ST, 0, s, n, (int)G, (const double*)w.part_rz,
                (const double*)w.part_rr, w.scal, slot ^ 1, (const T*)z, p);
    PH_LAUNCH_B("spmv_dot", (double)n * ((UNIT ? 2 : 3) * sizeof(T)) + 6.0 * n * (4 + sizeof(T)), (k_spmv_dot<T, UNIT>),
                G, ST, 0, s, n,
                col, val, diag, (const T*)p, q, w.part_pq);
  } else {
    PH_LAUNCH_B("spmv_dir", (double)n * ((UNIT ? 5 : 6) * sizeof(T)) + 6.0 * n * (4 + sizeof(T)), (k_spmv_dir<T, UNIT>),
                G, ST, 0, s, n, col,
                val, diag, (const T*)z, p, q, (int)G, (const double*)w.part_rz, (const double*)w.part_rr, w.scal,
                slot ^ 1, first ? 1 : 0, w.part_pq);
  }
  return PHFEM_OK;
}

// Jacobi-PCG on the 6-slot system (col, val, diag) from x0 = 0; stops at ||r|| <= tol ||b||
// (2-norm of the unscaled residual) or maxit.  SCALED: val is the Jacobi-scaled copy
// D^-1/2 (offdiag) D^-1/2 with the unit diagonal implied, and the iteration is CG on that
// system -- the same iterates in exact arithmetic, without the diagonal in the product and
// without the z vector; x is scaled back on exit.
template <class T, bool SCALED>
static int pcg(int64_t n, const int32_t* col, const T* val, const T* diag, const T* b, T* x,
               double tol, int maxit, PcgWS& w, int* iters, double* relres, hipStream_t s) {
  const unsigned G = pcg_grid(n);
  T *r = (T*)w.r, *z = (T*)w.z, *p = (T*)w.p, *q = (T*)w.q;
  if (SCALED)
    PH_LAUNCH("pcg_init", k_pcg_init_scaled<T>, G, ST, 0, s, n, b, diag, x, r, p, w.part_rz, w.part_rr);
  else
    PH_LAUNCH("pcg_init", k_pcg_init<T>, G, ST, 0, s, n, b, diag, x, r, z, p, w.part_rz, w.part_rr);
  PH_LAUNCH("pcg_scalars", k_scalars, 1, ST, 0, s, (int)G, (const double*)w.part_rz, (const double*)w.part_rr, w.scal,
            0);
  double rr0 = 0;
  int rc = read_scalar(w.scal + 2, &rr0, s);
  if (rc) return rc;
  const double bn = std::sqrt(rr0);
  *iters = 0;
  *relres = 0;
  if (bn == 0) return PHFEM_OK;  // x = 0 either way
  int slot = 0, it = 0;
  double rel = 1.0;
  while (it < maxit) {
    rc = pcg_direction<T, SCALED>(n, col, val, SCALED ? nullptr : diag, w, slot, it == 0,
                                  it > 0 && it % REFRESH == 0, s);
    if (rc) return rc;
    PH_LAUNCH_B("pcg_update", (SCALED ? 7.0 : 8.0) * sizeof(T) * n, (k_pcg_update<T, SCALED>), G, ST, 0, s, n, (int)G,
                (const double*)w.part_pq, (const double*)w.scal, slot, x, r, (const T*)p, (const T*)q, diag, z,
                w.part_rz, w.part_rr);
    slot ^= 1;
    ++it;
    // scal[2] holds r.r of the residual before this iteration's update (one iteration behind)
    if (it % CHECK == 0 || it == maxit) {
      double rr = 0;
      rc = read_scalar(w.scal + 2, &rr, s);
      if (rc) return rc;
      rel = std::sqrt(rr) / bn;
      if (!(rel > tol)) break;  // also stops on NaN
    }
  }
  if (SCALED) PH_LAUNCH("unscale", k_unscale<T>, G, ST, 0, s, n, diag, x);
  *iters = it;
  *relres = rel;
  return PHFEM_OK;
}

// Mesh-side data of the matrix-free FP64 operator b_D - C A^-1 (Bsrc + C'lambda).
struct MeshOp {
  int64_t nC, nE, nF;
  const double* X;
  const int32_t* tet;
  const int32_t* t2f;
  const int8_t* sigma;
  const int32_t* face2tet;
  const double* kappa;
  DevParams P;
  const double* gsrc;  // null: load vector of f
  const double* bD;    // null: zero
};

// r64 = b_D - C U(lambda) per face (owner term, then neighbour term) and U on the way
static int residual(const MeshOp& m, const double* lambda, double* U, double* cu, double* r64, int* flags,
                    hipStream_t s) {
  return launch_recover(m.nC, m.X, m.nE, m.nF, m.tet, m.t2f, m.sigma, m.face2tet, m.kappa, m.P, lambda, m.gsrc, m.bD,
                        U, cu, r64, flags, s);
}

static int check_flags(int* dflags, hipStream_t s) {
  int h = 0;
  PH_HIP(hipMemcpyAsync(&h, dflags, sizeof(int), hipMemcpyDeviceToHost, s));
  PH_HIP(hipStreamSynchronize(s));
  return h ? dev_flags_to_status(h) : PHFEM_OK;
}

// Solve S+ x = r+ (FP64 PCG on the stored system) or by FP64 iterative refinement with
// FP32 PCG corrections; U = A^-1 (Bsrc + C'x) in FP64 on exit; stats filled.
static int face_solve(const MeshOp& m, const int32_t* rowptr, const int32_t* col, const double* val,
                      const double* diag, const double* rhs, int32_t mode, double tol, double inner_tol, int maxit,
                      SolveWS& w, double* x, double* U, phfem_solve_stats* st, hipStream_t s) {
  const int64_t nF = m.nF;
  int rc;
  if ((reinterpret_cast<uintptr_t>(col) & 7) || (reinterpret_cast<uintptr_t>(val) & 15))
    return err(PHFEM_EINVAL, "col must be 8-byte and val 16-byte aligned");
  {
    PH_LAUNCH("check_pattern", k_check_pattern, pcg_grid(nF + 1), ST, 0, s, nF, rowptr, col, w.flags);
    int hf[2] = {0, 0};
    PH_HIP(hipMemcpyAsync(hf, w.flags, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
    PH_HIP(hipStreamSynchronize(s));
    if (hf[1]) return err(PHFEM_EINVAL, "face system is not the 6-slot layout of phfem_condense (rowptr[F] = 6 F, "
                                        "column ids in [0, nF))");
  }
  phfem_solve_stats loc = {0, 0, 0.0, 0.0, 0, 0};
  if (mode == PHFEM_SOLVE_FP64_PCG) {
    // PCG on the stored system stops on its recurrence residual; the stored system differs
    // from the matrix-free FP64 operator by assembly rounding, so the true residual can level
    // off above tol (about 3.5e-11 at Kuhn L5 with lognormal kappa, growing with the
    // condition number).  Each time the true residual b_D - C U(x) is still above tol, the
    // stored system is solved again for the correction e (S+ e = that residual, to the
    // relative accuracy still missing) and x += e: iterative refinement in FP64 that
    // converges on the true residual, as the mixed mode does.
    double rel = 0, bn = 0, rn = 0;
    int it = 0, total = 0;
    rc = norm2(nF, rhs, w.pcg, &bn, s);
    if (rc) return rc;
    loc.rhs_norm = bn;
    // the Jacobi-scaled copy the PCG iterates on (every solve below uses it)
    PH_LAUNCH("scale_f64", k_scale_f64, pcg_grid(6 * nF), ST, 0, s, nF, col, val, diag, w.val64s);
    rc = pcg<double, true>(nF, col, w.val64s, diag, rhs, x, tol, maxit, w.pcg, &it, &rel, s);
    if (rc) return rc;
    total = it;
    for (int steps = 0;; ++steps) {
      // true residual in FP64, matrix-free; also writes U
      rc = residual(m, x, U, w.cu, w.r64, w.flags, s);
      if (rc) return rc;
      rc = check_flags(w.flags, s);
      if (rc) return rc;
      const double prev = rn;
      rc = norm2(nF, w.r64, w.pcg, &rn, s);
      if (rc) return rc;
      loc.ir_steps = steps;
      if (!(rn > tol * bn) || total >= maxit || steps == 8 || (steps > 0 && !(rn < 0.5 * prev))) break;
      rc = pcg<double, true>(nF, col, w.val64s, diag, w.r64, w.e64, std::max(0.5 * tol * bn / rn, 1e-12),
                             maxit - total, w.pcg, &it, &rel, s);
      if (rc) return rc;
      total += it;
      PH_LAUNCH("add_f64", k_add_f64, pcg_grid(nF), ST, 0, s, nF, (const double*)w.e64, x);
    }
    loc.iters = total;
    loc.rel_res = bn > 0 ? rn / bn : rn;
    *st = loc;
    if (!(rn <= tol * bn))  // max_iter, or the corrections stopped gaining (attainable accuracy)
      return err(PHFEM_ENOCONV, total >= maxit ? "PCG reached max_iter above tolerance"
                                               : "FP64 refinement stagnated above tolerance (attainable accuracy "
                                                 "reached; stats.rel_res holds it)");
    return PHFEM_OK;
  }
  // mixed: the Jacobi-scaled FP32 copy of the system (6 nF off-diagonal slots, unit diagonal)
  PH_LAUNCH("scale_f32", k_scale_f32, pcg_grid(6 * nF), ST, 0, s, nF, col, val, diag, w.val32);
  // Iterative refinement without restarts: one FP32 CG recurrence on the scaled FP32 system
  // (Jacobi-PCG in scaled unknowns) whose residual is replaced by the scaled true FP64
  // residual D^-1/2 (b_D - C U(x)) (matrix-free, per tet, from the geometry) whenever the
  // recurrence residual has dropped by REPLACE since the last replacement (both in the
  // scaled 2-norm); the accumulated FP32 iterate is then folded into the FP64 solution.  The
  // search direction is kept, so the Krylov space is not rebuilt as restarted refinement
  // would; convergence is declared on the true FP64 residual only.
  const double REPLACE = inner_tol;
  const unsigned G = pcg_grid(nF);
  PcgWS& pw = w.pcg;
  float *r32 = (float*)pw.r, *p = (float*)pw.p, *q = (float*)pw.q;
  PH_LAUNCH("fill0", k_fill0, G, ST, 0, s, nF, x);
  rc = residual(m, x, U, w.cu, w.r64, w.flags, s);
  if (rc) return rc;
  rc = check_flags(w.flags, s);
  if (rc) return rc;
  double r0 = 0;
  rc = norm2(nF, w.r64, pw, &r0, s);
  if (rc) return rc;
  loc.rhs_norm = r0;
  if (r0 == 0) {
    *st = loc;
    return PHFEM_OK;
  }
  PH_LAUNCH("replace", k_replace<true>, G, ST, 0, s, nF, (const double*)w.r64, diag, r32, p, w.x32, pw.part_rz,
            pw.part_rr);
  PH_LAUNCH("pcg_scalars", k_scalars, 1, ST, 0, s, (int)G, (const double*)pw.part_rz, (const double*)pw.part_rr,
            pw.scal, 0);
  double ref = 0;  // scaled norm of the recurrence residual at the last replacement
  rc = read_scalar(pw.scal + 2, &ref, s);
  if (rc) return rc;
  ref = std::sqrt(ref);
  double rel = 1.0, best = r0;
  int slot = 0, it = 0, steps = 0, stall = 0, last = 0;
  bool replace = false, done = false, exact = false;
  while (!done) {
    // below the attainable accuracy the true residual stops falling: 6 replacements in a row
    // without a 10 % gain end the solve early (as max_iter would, with the same error)
    if (it >= maxit || stall >= 6) break;
    // direction step (exact product after a replacement and every REFRESH iterations)
    rc = pcg_direction<float, true>(nF, col, w.val32, nullptr, pw, slot, it == 0, exact || (it > 0 && it % REFRESH == 0),
                                    s);
    if (rc) return rc;
    exact = false;
    PH_LAUNCH_B("pcg_update", 6.0 * 4 * nF, (k_pcg_update<float, true>), G, ST, 0, s, nF, (int)G,
                (const double*)pw.part_pq, (const double*)pw.scal, slot, w.x32, r32, (const float*)p, (const float*)q,
                (const float*)nullptr, (float*)nullptr, pw.part_rz, pw.part_rr);
    if (replace) {
      PH_LAUNCH("flush_x", k_flush_x, G, ST, 0, s, nF, diag, w.x32, x);
      rc = residual(m, x, U, w.cu, w.r64, w.flags, s);
      if (rc) return rc;
      double rn = 0;
      rc = norm2(nF, w.r64, pw, &rn, s);
      if (rc) return rc;
      ++steps;
      rel = rn / r0;
      if (rn < 0.9 * best) {
        best = rn;
        stall = 0;
      } else {
        ++stall;
      }
      if (!(rel > tol)) {
        done = true;  // x and U are the converged FP64 solution
      } else {
        PH_LAUNCH("replace", k_replace<false>, G, ST, 0, s, nF, (const double*)w.r64, diag, r32, p, w.x32,
                  pw.part_rz, pw.part_rr);
        PH_LAUNCH("sum1", k_sum1, 1, ST, 0, s, (int)G, (const double*)pw.part_rr, pw.scal + 4);
        rc = read_scalar(pw.scal + 4, &ref, s);
        if (rc) return rc;
        ref = std::sqrt(ref);
        exact = true;
      }
      replace = false;
      last = it;
    }
    slot ^= 1;
    ++it;
    if (!done && it % CHECK == 0) {
      double rr = 0;
      rc = read_scalar(pw.scal + 2, &rr, s);
      if (rc) return rc;
      // replace when the recurrence has gained the factor, and also after FORCE iterations
      // without that gain (a recurrence that has stopped descending, near the attainable
      // accuracy, would otherwise never reach the stagnation test)
      if (!(std::sqrt(rr) > REPLACE * ref) || !(rr == rr) || it - last >= FORCE) replace = true;
    }
  }
  // FP64 polish.  The FP32 corrections leave the smoothest error modes (where cond x eps32
  // approaches 1) barely resolved: at an equal true residual the mixed iterate's error is about
  // ten times the FP64 solve's.  Correction solves on the stored FP64 system (its Jacobi-scaled
  // copy) from the true residual remove that part; they start from a small residual and stop
  // at a modest relative tolerance, so they cost a fraction of the FP32 iterations.
  if (it < maxit) {
    PH_LAUNCH("scale_f64", k_scale_f64, pcg_grid(6 * nF), ST, 0, s, nF, col, val, diag, w.val64s);
    double rn = rel * r0;
    for (int c = 0; c < POLISH_MAX && it < maxit; ++c) {
      int pit = 0;
      double prel = 0;
      rc = pcg<double, true>(nF, col, w.val64s, diag, w.r64, w.e64, POLISH_TOL, maxit - it, w.pcg64, &pit, &prel, s);
      if (rc) return rc;
      it += pit;
      loc.polish_iters += pit;
      PH_LAUNCH("add_f64", k_add_f64, G, ST, 0, s, nF, (const double*)w.e64, x);
      rc = residual(m, x, U, w.cu, w.r64, w.flags, s);
      if (rc) return rc;
      const double prev = rn;
      rc = norm2(nF, w.r64, w.pcg64, &rn, s);
      if (rc) return rc;
      ++loc.polish_steps;
      rel = rn / r0;
      if (!(rel > tol) && c + 1 >= POLISH_MIN) break;
      if (!(rn < 0.5 * prev) && c + 1 >= POLISH_MIN) break;
    }
  }
  loc.iters = it;
  loc.ir_steps = steps;
  loc.rel_res = rel;
  *st = loc;
  if (rel > tol)
    return err(PHFEM_ENOCONV, it >= maxit ? "mixed refinement reached max_iter above tolerance"
                                          : "mixed refinement stagnated above tolerance (attainable accuracy "
                                            "reached; stats.rel_res holds it)");
  return PHFEM_OK;
}

}  // namespace ph

using namespace ph;

extern "C" size_t phfem_solve_workspace(int64_t nE, int64_t nF, int32_t mode) {
  (void)nE;
  Arena a;
  SolveWS w;
  solve_layout(a, nE, nF, mode, w);
  return a.size();
}

static int solve_args_ok(int64_t nC, const double* coord, int64_t nE, const int32_t* tetra, int64_t nF,
                         const int32_t* faces, const int32_t* tet2face, const int8_t* sigma, const int32_t* face2tet,
                         const int32_t* rowptr, const int32_t* col, const double* val, const double* diag,
                         int32_t mode, double tol, int32_t max_iter) {
  if (nC <= 0 || nE <= 0 || nF <= 0 || !coord || !tetra || !faces || !tet2face || !sigma || !face2tet || !rowptr ||
      !col || !val || !diag)
    return err(PHFEM_EINVAL, "bad solve arguments");
  if (mode != PHFEM_SOLVE_FP64_PCG && mode != PHFEM_SOLVE_FP32_PCG_FP64_IR) return err(PHFEM_EINVAL, "bad mode");
  if (!(tol >= 0) || max_iter <= 0) return err(PHFEM_EINVAL, "bad tolerance or max_iter");
  return PHFEM_OK;
}

extern "C" int phfem_solve(int64_t nC, const double* coord, int64_t nE, const int32_t* tetra, int64_t nF,
                           const int32_t* faces, const int32_t* tet2face, const int8_t* sigma, const int32_t* face2tet,
                           const double* kappa, const phfem_params* p, const int32_t* rowptr, const int32_t* col,
                           const double* val, const double* diag, const double* rhs, int32_t mode, double tol,
                           double inner_tol, int32_t max_iter, void* work, size_t work_bytes, double* lambda,
                           double* U, phfem_solve_stats* stats, phfem_stream_t stream_) {
  clear_error();
  hipStream_t s = (hipStream_t)stream_;
  int rc = check_params(p);
  if (rc) return rc;
  rc = solve_args_ok(nC, coord, nE, tetra, nF, faces, tet2face, sigma, face2tet, rowptr, col, val, diag, mode, tol,
                     max_iter);
  if (rc) return rc;
  if (!rhs || !lambda || !U || !stats) return err(PHFEM_EINVAL, "null rhs/lambda/U/stats");
  if (!work || work_bytes < phfem_solve_workspace(nE, nF, mode)) return err(PHFEM_EWORKSPACE, "solve workspace too small");
  Arena a(work, work_bytes);
  SolveWS w;
  solve_layout(a, nE, nF, mode, w);
  MeshOp m{nC, nE, nF, coord, tetra, tet2face, sigma, face2tet, kappa, to_dev(*p), nullptr, w.bD};
  PH_HIP(hipMemsetAsync(w.flags, 0, 2 * sizeof(int), s));
  rc = launch_face_init(nF, nC, coord, faces, face2tet, m.P, nullptr, nullptr, w.bD, w.flags, s);
  if (rc) return rc;
  if (!(inner_tol > 0 && inner_tol < 1)) inner_tol = 0.9;
  return face_solve(m, rowptr, col, val, diag, rhs, mode, tol, inner_tol, max_iter, w, lambda, U, stats, s);
}

extern "C" size_t phfem_grad_workspace(int64_t nE, int64_t nF, int32_t mode) {
  Arena a;
  a.take<double>(nF);      // adjoint rhs
  a.take<double>(nF);      // Q
  a.take<double>(4 * nE);  // P
  return a.size() + phfem_solve_workspace(nE, nF, mode);
}

extern "C" int phfem_grad(int64_t nC, const double* coord, int64_t nE, const int32_t* tetra, int64_t nF,
                          const int32_t* faces, const int32_t* tet2face, const int8_t* sigma, const int32_t* face2tet,
                          const int32_t* nbr, const double* kappa, const phfem_params* p, const int32_t* rowptr,
                          const int32_t* col, const double* val, const double* diag, const double* U,
                          const double* lambda, const double* dJdU, int32_t mode, double tol, double inner_tol,
                          int32_t max_iter, void* work, size_t work_bytes, double* dJ_dlogkappa, double* dJ_dcoord,
                          phfem_solve_stats* stats, phfem_stream_t stream_) {
  clear_error();
  hipStream_t s = (hipStream_t)stream_;
  int rc = check_params(p);
  if (rc) return rc;
  rc = solve_args_ok(nC, coord, nE, tetra, nF, faces, tet2face, sigma, face2tet, rowptr, col, val, diag, mode, tol,
                     max_iter);
  if (rc) return rc;
  if (!nbr || !U || !lambda || !dJdU || !stats) return err(PHFEM_EINVAL, "null nbr/U/lambda/dJdU/stats");
  if (p->neumann) return err(PHFEM_EINVAL, "the gradient covers Dirichlet boundaries only (params.neumann must be NULL)");
  if (!work || work_bytes < phfem_grad_workspace(nE, nF, mode)) return err(PHFEM_EWORKSPACE, "grad workspace too small");
  Arena a(work, work_bytes);
  double* radj = a.take<double>(nF);
  double* Q = a.take<double>(nF);
  double* Pv = a.take<double>(4 * nE);
  SolveWS w;
  solve_layout(a, nE, nF, mode, w);
  DevParams P = to_dev(*p);
  PH_HIP(hipMemsetAsync(w.flags, 0, 2 * sizeof(int), s));
  // adjoint right-hand side -C A^-1 dJdU (recovery with lambda = 0 and the load replaced by dJdU)
  rc = launch_recover(nC, coord, nE, nF, tetra, tet2face, sigma, face2tet, kappa, P, nullptr, dJdU, nullptr, Pv, w.cu,
                      radj, w.flags, s);
  if (rc) return rc;
  rc = check_flags(w.flags, s);
  if (rc) return rc;
  MeshOp m{nC, nE, nF, coord, tetra, tet2face, sigma, face2tet, kappa, P, dJdU, nullptr};
  if (!(inner_tol > 0 && inner_tol < 1)) inner_tol = 0.9;
  // Pv = A^-1 (dJdU + C'Q) on exit; an adjoint solve that stopped above tol (ENOCONV) still
  // yields the gradient of its last iterate, and the call returns ENOCONV
  const int solve_rc = face_solve(m, rowptr, col, val, diag, radj, mode, tol, inner_tol, max_iter, w, Q, Pv, stats, s);
  if (solve_rc != PHFEM_OK && solve_rc != PHFEM_ENOCONV) return solve_rc;
  const std::string solve_msg = phfem_last_error();
  if (dJ_dcoord) PH_HIP(hipMemsetAsync(dJ_dcoord, 0, sizeof(double) * 3 * nC, s));
  rc = launch_vjp(nC, coord, nE, nF, tetra, tet2face, sigma, nbr, kappa, P, U, Pv, lambda, Q, dJ_dlogkappa, dJ_dcoord,
                  w.flags, s);
  if (rc) return rc;
  rc = check_flags(w.flags, s);
  if (rc) return rc;
  return solve_rc == PHFEM_OK ? PHFEM_OK : err(solve_rc, solve_msg);
}
