// A-priori error norms of a discrete solution against an exact solution (Section 5, the
// mesh-dependent norm of Y and the h-norm of eq. (eMnorm), the quantities of Table 4):
//   e0 = sum_T ||grad(u - u_h)||^2_T,   e1 = sum_T ||u - u_h||^2_T,
//   e2 = sum_T h sum_{F in dT \ Gamma_N} ||kappa_T grad u . nu_F - lambda_F||^2_F
// (nu_F the owner's outward normal, lambda_F relative to it), u_h linear on each tet with the
// vertex values U.  ||u - u_h||_Y = sqrt(e0 + e1 / h^2), ||kappa - kappa_h||_h = sqrt(e2).
//
// Quadrature: collapsed (Duffy) Gauss-Legendre products with n points per direction, exact
// to degree 2n - 3 on the tet (x = s, y = t (1 - s), z = r (1 - s)(1 - t), Jacobian
// (1 - s)^2 (1 - t)) and 2n - 2 on the triangle; the 1-D nodes come from Newton's method on
// the Legendre three-term recurrence.  One thread per tet, per-block partial sums reduced in
// a fixed order (deterministic).
#include <cmath>
#include <mutex>

#include "common.hpp"

namespace ph {

constexpr int ERT = 256;
constexpr int ERMAXQ = 12;

struct Fun4 {  // parameters of the exact solution, passed by value
  double p[4];
};

struct GL1 {  // 1-D Gauss-Legendre rule on [0, 1]
  int n;
  double x[ERMAXQ], w[ERMAXQ];
};

static GL1 gauss_legendre01(int n) {
  GL1 r;
  r.n = n;
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;  // P_0, P_1; recurrence (k+1) P_{k+1} = (2k+1) z P_k - k P_{k-1}
      for (int k = 1; k < n; ++k) {
        const double p2 = ((2.0 * k + 1.0) * z * p1 - k * p0) / (k + 1.0);
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);  // P_n'(z)
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-17) break;
    }
    r.x[i] = 0.5 * (1.0 - z);
    r.w[i] = 1.0 / ((1.0 - z * z) * dp * dp);  // 2 / ((1 - z^2) P_n'^2) on [-1, 1], halved
  }
  return r;
}

__global__ __launch_bounds__(ERT) void k_errors(int64_t nC, const double* __restrict__ X, int64_t nE,
                                                int64_t nF, const int32_t* __restrict__ tet,
                                                const int32_t* __restrict__ t2f,
                                                const int8_t* __restrict__ sigma, const double* __restrict__ kappa,
                                                DevParams P, const double* __restrict__ U,
                                                const double* __restrict__ lambda, int uk, Fun4 up, double h, GL1 q,
                                                double* __restrict__ part, uint32_t* __restrict__ bad) {
  __shared__ double lds[3][ERT / 64];
  const int64_t t = (int64_t)blockIdx.x * ERT + threadIdx.x;
  double e0 = 0.0, e1 = 0.0, e2 = 0.0;
  int v[4] = {0, 0, 0, 0}, sig[4], F[4] = {0, 0, 0, 0};
  double u[4];
  bool ok = t < nE;
  if (ok) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      v[i] = tet[i * nE + t];
      sig[i] = sigma[i * nE + t];
      F[i] = t2f[i * nE + t];
      u[i] = U[i * nE + t];
    }
    bool in = true;
#pragma unroll
    for (int i = 0; i < 4; ++i) in = in && v[i] >= 0 && v[i] < nC && F[i] >= 0 && F[i] < nF;
    if (!in) atomicOr(bad, 1u);  // the tet is left out and the call fails
    ok = in;
  }
  if (ok) {
    double x[4][3];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int e = 0; e < 3; ++e) x[i][e] = X[e * nC + v[i]];
    const double kap = kappa ? kappa[t] : P.kc;
    double a[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int e = 0; e < 3; ++e) a[i][e] = x[i + 1][e] - x[0][e];
    // gradients of the barycentric coordinates 1..3: rows of the inverse transpose of [a1 a2 a3]
    const double c0[3] = {a[1][1] * a[2][2] - a[1][2] * a[2][1], a[1][2] * a[2][0] - a[1][0] * a[2][2],
                          a[1][0] * a[2][1] - a[1][1] * a[2][0]};
    const double c1[3] = {a[2][1] * a[0][2] - a[2][2] * a[0][1], a[2][2] * a[0][0] - a[2][0] * a[0][2],
                          a[2][0] * a[0][1] - a[2][1] * a[0][0]};
    const double c2[3] = {a[0][1] * a[1][2] - a[0][2] * a[1][1], a[0][2] * a[1][0] - a[0][0] * a[1][2],
                          a[0][0] * a[1][1] - a[0][1] * a[1][0]};
    const double det = a[0][0] * c0[0] + a[0][1] * c0[1] + a[0][2] * c0[2];
    double guh[3];
#pragma unroll
    for (int e = 0; e < 3; ++e)
      guh[e] = ((u[1] - u[0]) * c0[e] + (u[2] - u[0]) * c1[e] + (u[3] - u[0]) * c2[e]) / det;
    const double jac = fabs(det);
    for (int i = 0; i < q.n; ++i) {
      const double s = q.x[i];
      for (int j = 0; j < q.n; ++j) {
        const double tt = q.x[j];
        for (int k = 0; k < q.n; ++k) {
          const double r = q.x[k];
          const double l1 = s, l2 = tt * (1.0 - s), l3 = r * (1.0 - s) * (1.0 - tt);
          const double l0 = 1.0 - l1 - l2 - l3;
          const double w = q.w[i] * q.w[j] * q.w[k] * (1.0 - s) * (1.0 - s) * (1.0 - tt) * jac;
          double p[3];
#pragma unroll
          for (int e = 0; e < 3; ++e) p[e] = l0 * x[0][e] + l1 * x[1][e] + l2 * x[2][e] + l3 * x[3][e];
          const double uh = l0 * u[0] + l1 * u[1] + l2 * u[2] + l3 * u[3];
          const double ue = fun_at<double>(uk, up.p, p[0], p[1], p[2]);
          double g[3];
          fun_grad(uk, up.p, p[0], p[1], p[2], g);
          e0 += w * ((g[0] - guh[0]) * (g[0] - guh[0]) + (g[1] - guh[1]) * (g[1] - guh[1]) +
                     (g[2] - guh[2]) * (g[2] - guh[2]));
          e1 += w * (ue - uh) * (ue - uh);
        }
      }
    }
#pragma unroll
    for (int kf = 0; kf < 4; ++kf) {
      if (P.nm && P.nm[F[kf]]) continue;  // the h-norm runs over dT \ Gamma_N
      const int ia = fv(kf, 0), ib = fv(kf, 1), ic = fv(kf, 2), io = opp(kf);
      double e1v[3], e2v[3], n[3];
#pragma unroll
      for (int e = 0; e < 3; ++e) {
        e1v[e] = x[ib][e] - x[ia][e];
        e2v[e] = x[ic][e] - x[ia][e];
      }
      n[0] = e1v[1] * e2v[2] - e1v[2] * e2v[1];
      n[1] = e1v[2] * e2v[0] - e1v[0] * e2v[2];
      n[2] = e1v[0] * e2v[1] - e1v[1] * e2v[0];
      const double nl = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
      const double away = n[0] * (x[io][0] - x[ia][0]) + n[1] * (x[io][1] - x[ia][1]) + n[2] * (x[io][2] - x[ia][2]);
      const double sgn = (away > 0 ? -1.0 : 1.0) * sig[kf] / nl;  // owner's outward unit normal
      const double lam = lambda[F[kf]];
      double acc = 0.0;
      for (int i = 0; i < q.n; ++i) {
        const double s = q.x[i];
        for (int j = 0; j < q.n; ++j) {
          const double tt = q.x[j] * (1.0 - s);
          const double w = q.w[i] * q.w[j] * (1.0 - s);
          double p[3], g[3];
#pragma unroll
          for (int e = 0; e < 3; ++e) p[e] = x[ia][e] + s * e1v[e] + tt * e2v[e];
          fun_grad(uk, up.p, p[0], p[1], p[2], g);
          const double d = kap * sgn * (g[0] * n[0] + g[1] * n[1] + g[2] * n[2]) - lam;
          acc += w * d * d;
        }
      }
      e2 += h * nl * acc;  // |F| = nl / 2 and the reference triangle's area 1/2
    }
  }
  // block sums in a fixed order
  double vals[3] = {e0, e1, e2};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    double vv = vals[c];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) vv += __shfl_down(vv, o, 64);
    if ((threadIdx.x & 63) == 0) lds[c][threadIdx.x >> 6] = vv;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    double sm = 0.0;
#pragma unroll
    for (int wv = 0; wv < ERT / 64; ++wv) sm += lds[threadIdx.x][wv];
    part[3 * (int64_t)blockIdx.x + threadIdx.x] = sm;
  }
}

__global__ __launch_bounds__(ERT) void k_errors_sum(int64_t nb, const double* __restrict__ part,
                                                    double* __restrict__ out) {
  __shared__ double lds[ERT / 64];
  for (int c = 0; c < 3; ++c) {
    double v = 0.0;
    for (int64_t i = threadIdx.x; i < nb; i += ERT) v += part[3 * i + c];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
      double sm = 0.0;
      for (int wv = 0; wv < ERT / 64; ++wv) sm += lds[wv];
      out[c] = sm;
    }
    __syncthreads();
  }
}

__global__ void k_errors_clear(uint32_t* __restrict__ bad) { *bad = 0u; }

// Scratch of phfem_errors_noalloc: the per-block partial sums, the three totals and the
// index-check word, in a fixed device array (no allocation and no caller workspace).  Every
// GPU that runs the library holds one copy until the process ends; host code reaches it only
// through the address hipGetSymbolAddress returns on that device.
constexpr size_t NOALLOC_BYTES = size_t(2) << 20;
static __device__ __align__(256) double scratch[NOALLOC_BYTES / sizeof(double)];

constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void* g_scratch[MAX_DEVICES];

// the current device's address of `scratch`, looked up once per device
static int scratch_address(void** out) {
  int d = 0;
  PH_HIP(hipGetDevice(&d));
  if (d < 0 || d >= MAX_DEVICES) return err(PHFEM_EINVAL, "device ordinal beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[d]) {
    void* p = nullptr;
    PH_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch[d] = p;
  }
  *out = g_scratch[d];
  return PHFEM_OK;
}

static size_t errors_scratch_bytes(int64_t nE) {
  Arena a;
  a.take<double>(3 * ((nE + ERT - 1) / ERT));
  a.take<double>(4);
  a.take<uint32_t>(1);
  return a.size();
}

static int errors_args_ok(int64_t nC, const double* coord, int64_t nE, const int32_t* tetra, int64_t nF,
                          const int32_t* tet2face, const int8_t* sigma, const phfem_params* p, const double* U,
                          const double* lambda, int32_t u_kind, const double* u_par, double h, int32_t nq,
                          double* out) {
  int rc = check_params(p);
  if (rc) return rc;
  if (nC <= 0 || nE <= 0 || nF <= 0 || !coord || !tetra || !tet2face || !sigma || !U || !lambda || !out || !u_par)
    return err(PHFEM_EINVAL, "bad errors arguments");
  if (u_kind < 0 || u_kind > PHFEM_FUN_X2Y2Z2_LOAD) return err(PHFEM_EINVAL, "bad u_kind");
  if (nq < 1 || nq > ERMAXQ) return err(PHFEM_EINVAL, "nq must be in [1, 12]");
  if (!(h > 0)) return err(PHFEM_EINVAL, "h must be > 0");
  return PHFEM_OK;
}

// the error sums with their scratch in (base, cap): per-block partials, totals, check word
static int errors_run(int64_t nC, const double* coord, int64_t nE, const int32_t* tetra, int64_t nF,
                      const int32_t* tet2face, const int8_t* sigma, const double* kappa, const phfem_params* p,
                      const double* U, const double* lambda, int32_t u_kind, const double* u_par, double h,
                      int32_t nq, void* base, size_t cap, double* out, hipStream_t s) {
  Arena a(base, cap);
  const int64_t nb = (nE + ERT - 1) / ERT;
  double* part = a.take<double>(3 * nb);
  double* dout = a.take<double>(4);
  uint32_t* bad = a.take<uint32_t>(1);
  Fun4 up;
  for (int i = 0; i < 4; ++i) up.p[i] = u_par[i];
  const GL1 q = gauss_legendre01(nq);
  PH_LAUNCH("errors_clear", k_errors_clear, 1, 1, 0, s, bad);
  PH_LAUNCH("errors", k_errors, (unsigned)nb, ERT, 0, s, nC, coord, nE, nF, tetra, tet2face, sigma, kappa, to_dev(*p),
            U, lambda, u_kind, up, h, q, part, bad);
  PH_LAUNCH("errors_sum", k_errors_sum, 1, ERT, 0, s, nb, (const double*)part, dout);
  double res[3];
  uint32_t hbad = 0;
  PH_HIP(hipMemcpyAsync(res, dout, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
  PH_HIP(hipMemcpyAsync(&hbad, bad, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  PH_HIP(hipStreamSynchronize(s));
  if (hbad) return err(PHFEM_EINVAL, "vertex or face id out of range");
  for (int i = 0; i < 3; ++i) out[i] = res[i];
  return PHFEM_OK;
}

}  // namespace ph

using namespace ph;

extern "C" size_t phfem_errors_workspace(int64_t nE) {
  if (nE <= 0) return 0;
  return errors_scratch_bytes(nE);
}

extern "C" int phfem_errors(int64_t nC, const double* coord, int64_t nE, const int32_t* tetra, int64_t nF,
                            const int32_t* tet2face, const int8_t* sigma, const double* kappa, const phfem_params* p,
                            const double* U, const double* lambda, int32_t u_kind, const double* u_par, double h,
                            int32_t nq, void* work, size_t work_bytes, double* out, phfem_stream_t stream_) {
  clear_error();
  int rc = errors_args_ok(nC, coord, nE, tetra, nF, tet2face, sigma, p, U, lambda, u_kind, u_par, h, nq, out);
  if (rc) return rc;
  if (!work || work_bytes < phfem_errors_workspace(nE)) return err(PHFEM_EWORKSPACE, "errors workspace too small");
  return errors_run(nC, coord, nE, tetra, nF, tet2face, sigma, kappa, p, U, lambda, u_kind, u_par, h, nq, work,
                    work_bytes, out, (hipStream_t)stream_);
}

extern "C" int phfem_errors_noalloc(int64_t nC, const double* coord, int64_t nE, const int32_t* tetra, int64_t nF,
                                    const int32_t* tet2face, const int8_t* sigma, const double* kappa,
                                    const phfem_params* p, const double* U, const double* lambda, int32_t u_kind,
                                    const double* u_par, double h, int32_t nq, double* out, phfem_stream_t stream_) {
  clear_error();
  int rc = errors_args_ok(nC, coord, nE, tetra, nF, tet2face, sigma, p, U, lambda, u_kind, u_par, h, nq, out);
  if (rc) return rc;
  if (nE > PHFEM_ERRORS_NOALLOC_MAX_TETS || errors_scratch_bytes(nE) > NOALLOC_BYTES)
    return err(PHFEM_EINVAL, "phfem_errors_noalloc: nE exceeds PHFEM_ERRORS_NOALLOC_MAX_TETS (use phfem_errors)");
  void* base = nullptr;
  rc = scratch_address(&base);
  if (rc) return rc;
  return errors_run(nC, coord, nE, tetra, nF, tet2face, sigma, kappa, p, U, lambda, u_kind, u_par, h, nq, base,
                    NOALLOC_BYTES, out, (hipStream_t)stream_);
}
