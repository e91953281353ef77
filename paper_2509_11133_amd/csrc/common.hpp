// Internal helpers shared by the library's HIP sources (not part of the C-ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <string>

#include "../../include/phfem.h"

namespace ph {

// ------------------------------------------------------------------ error state
void set_error(const std::string& msg);
void clear_error();

struct Fail {
  int code;
};

inline int err(int code, const std::string& msg) {
  set_error(msg);
  return code;
}

#define PH_HIP(call)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (call);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return ::ph::err(PHFEM_EHIP, std::string(#call) + ": " + hipGetErrorString(e_));    \
  } while (0)

// device error flags (OR-ed into one int in the workspace)
enum : int { DEV_BADNODE = 1, DEV_ORIENT = 2, DEV_DEGEN = 4, DEV_NOFACE = 8 };

int dev_flags_to_status(int flags);

// ------------------------------------------------------------------ workspace arena
// Bump allocator over the caller's workspace; with base == nullptr it only measures.
struct Arena {
  char* base;
  size_t cap, off;
  explicit Arena(void* b = nullptr, size_t c = 0) : base((char*)b), cap(c), off(0) {}
  template <class T>
  T* take(size_t n) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? (T*)(base + off) : nullptr;
    off += n * sizeof(T);
    return p;
  }
  size_t size() const { return (off + 255) & ~size_t(255); }
};

// ------------------------------------------------------------------ launches + profiling
bool profiling();
void prof_begin(const char* name, hipStream_t s, double bytes);
void prof_end(hipStream_t s);

inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

// Launch with an algorithmic byte count (each input read once, each output written once)
// recorded by the profiler; PH_LAUNCH for kernels without a meaningful count.
#define PH_LAUNCH_B(name, bytes, kernel, grid, block, shmem, stream, ...)             \
  do {                                                                                \
    if ((grid) > 0) {                                                                 \
      if (::ph::profiling()) ::ph::prof_begin(name, stream, (double)(bytes));         \
      hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), shmem, stream, __VA_ARGS__); \
      if (::ph::profiling()) ::ph::prof_end(stream);                                  \
      hipError_t e_ = hipGetLastError();                                              \
      if (e_ != hipSuccess)                                                           \
        return ::ph::err(PHFEM_EHIP, std::string("launch ") + name + ": " + hipGetErrorString(e_)); \
    }                                                                                 \
  } while (0)
#define PH_LAUNCH(name, kernel, grid, block, shmem, stream, ...) \
  PH_LAUNCH_B(name, 0, kernel, grid, block, shmem, stream, __VA_ARGS__)

// ------------------------------------------------------------------ device helpers
__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// Store of a write-once output stream: the nontemporal hint keeps these lines from displacing
// the kernel's re-read working set in L2 (measured: the refinement's pass 2 1.07 -> 0.88 ms,
// its output written as 27 row and entity streams).
template <class T>
__device__ __forceinline__ void st_nt(T* p, T v) {
  __builtin_nontemporal_store(v, p);
}
__device__ __forceinline__ void st_nt(uint2* p, uint2 v) {
  typedef uint32_t u2 __attribute__((ext_vector_type(2)));
  __builtin_nontemporal_store(u2{v.x, v.y}, reinterpret_cast<u2*>(p));
}
__device__ __forceinline__ void st_nt(int4* p, int4 v) {
  typedef int32_t i4 __attribute__((ext_vector_type(4)));
  __builtin_nontemporal_store(i4{v.x, v.y, v.z, v.w}, reinterpret_cast<i4*>(p));
}
__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

// Local numbering of tet [a b c d] as packed nibbles (no memory tables):
//  edges j = IJ IK IL JK JL KL -> vertices (ev0(j), ev1(j));
//  faces k = [a b c], [a c d], [a d b], [d c b] -> vertices fv(k, 0..2);
//  opp(k) = local vertex opposite face k (also: the face opposite vertex i is opp(i));
//  eidx(i, j) = local edge joining local vertices i != j.
__host__ __device__ __forceinline__ constexpr int ev0(int j) { return (int)((0x211000u >> (4 * j)) & 15u); }
__host__ __device__ __forceinline__ constexpr int ev1(int j) { return (int)((0x332321u >> (4 * j)) & 15u); }
__host__ __device__ __forceinline__ constexpr int fv(int k, int m) {
  return (int)((0x123130320210ull >> (12 * k + 4 * m)) & 15ull);
}
__host__ __device__ __forceinline__ constexpr int opp(int k) { return (int)((0x0213u >> (4 * k)) & 15u); }
__host__ __device__ __forceinline__ constexpr int eidx(int i, int j) {
  return (i < j ? i : j) == 0 ? (i > j ? i : j) - 1 : ((i < j ? i : j) == 1 ? (i > j ? i : j) + 1 : 5);
}
static_assert(fv(0, 0) == 0 && fv(0, 1) == 1 && fv(0, 2) == 2 && fv(1, 1) == 2 && fv(1, 2) == 3, "fv");
static_assert(fv(2, 1) == 3 && fv(2, 2) == 1 && fv(3, 0) == 3 && fv(3, 1) == 2 && fv(3, 2) == 1, "fv");
static_assert(ev0(3) == 1 && ev1(3) == 2 && ev0(5) == 2 && ev1(5) == 3 && ev1(2) == 3, "ev");
static_assert(opp(0) == 3 && opp(1) == 1 && opp(2) == 2 && opp(3) == 0, "opp");
static_assert(eidx(0, 1) == 0 && eidx(2, 0) == 1 && eidx(0, 3) == 2 && eidx(1, 2) == 3 && eidx(3, 1) == 4 &&
                  eidx(2, 3) == 5,
              "eidx");

// ------------------------------------------------------------------ problem data
struct DevParams {
  double c, kc;
  int fk;
  double fp[4];
  int uk;
  double up[4];
  int quad;
  int gk;
  double gp[4];
  const uint8_t* nm;  // Neumann flags per face, or null
};

inline DevParams to_dev(const phfem_params& p) {
  DevParams d;
  d.c = p.c;
  d.kc = p.kappa_const;
  d.fk = p.f_kind;
  d.uk = p.ud_kind;
  for (int i = 0; i < 4; ++i) {
    d.fp[i] = p.f_par[i];
    d.up[i] = p.ud_par[i];
    d.gp[i] = p.g_par[i];
  }
  d.quad = p.quad;
  d.gk = p.g_kind;
  d.nm = p.neumann;
  return d;
}

int check_params(const phfem_params* p);

template <class R>
__device__ __forceinline__ R sinpi_r(R x);
template <>
__device__ __forceinline__ double sinpi_r<double>(double x) { return sinpi(x); }
// FP32 sin(pi x): reduce x exactly to r in [-1, 1] (x - 2 rint(x / 2) is exact in FP32), then
// the hardware sine, which takes its argument in revolutions: sin(pi r) = v_sin(r / 2).
// Max abs error about 1.3e-7 on [0, 1] (against FP64 sinpi), against 5e-8 for the library
// sinpif at about 20x the instructions; the FP32 path only feeds the preconditioned inner
// solve, whose result is corrected with FP64 residuals.
template <>
__device__ __forceinline__ float sinpi_r<float>(float x) {
  const float r = x - 2.0f * rintf(0.5f * x);
  return __builtin_amdgcn_sinf(0.5f * r);
}
template <class R>
__device__ __forceinline__ R cospi_r(R x);
template <>
__device__ __forceinline__ double cospi_r<double>(double x) { return cospi(x); }
template <>
__device__ __forceinline__ float cospi_r<float>(float x) { return cospif(x); }

// f or u_D at a point (kinds of phfem.h)
template <class R>
__device__ __forceinline__ R fun_at(int kind, const double* p, R x, R y, R z) {
  switch (kind) {
    case PHFEM_FUN_CONST: return (R)p[0];
    case PHFEM_FUN_SIN3: return (R)p[0] * sinpi_r<R>(x) * sinpi_r<R>(y) * sinpi_r<R>(z);
    case PHFEM_FUN_LINEAR: return (R)p[0] + (R)p[1] * x + (R)p[2] * y + (R)p[3] * z;
    case PHFEM_FUN_X2Y2Z2: return (R)p[0] * x * x * y * y * z * z;
    case PHFEM_FUN_X2Y2Z2_LOAD: {
      R x2 = x * x, y2 = y * y, z2 = z * z;
      return (R)(-2.0 * p[0]) * (y2 * z2 + x2 * z2 + x2 * y2) + (R)p[1] * x2 * y2 * z2;
    }
    default: return (R)0;
  }
}

// gradient of the data functions (adjoint)
__device__ __forceinline__ void fun_grad(int kind, const double* p, double x, double y, double z, double g[3]) {
  g[0] = g[1] = g[2] = 0.0;
  switch (kind) {
    case PHFEM_FUN_SIN3: {
      const double pi = 3.14159265358979323846;
      double sx = sinpi(x), sy = sinpi(y), sz = sinpi(z), cx = cospi(x), cy = cospi(y), cz = cospi(z);
      g[0] = p[0] * pi * cx * sy * sz;
      g[1] = p[0] * pi * sx * cy * sz;
      g[2] = p[0] * pi * sx * sy * cz;
      break;
    }
    case PHFEM_FUN_LINEAR: g[0] = p[1]; g[1] = p[2]; g[2] = p[3]; break;
    case PHFEM_FUN_X2Y2Z2:
      g[0] = p[0] * 2 * x * y * y * z * z;
      g[1] = p[0] * 2 * x * x * y * z * z;
      g[2] = p[0] * 2 * x * x * y * y * z;
      break;
    case PHFEM_FUN_X2Y2Z2_LOAD: {
      double x2 = x * x, y2 = y * y, z2 = z * z;
      g[0] = -2 * p[0] * (2 * x * z2 + 2 * x * y2) + p[1] * 2 * x * y2 * z2;
      g[1] = -2 * p[0] * (2 * y * z2 + 2 * x2 * y) + p[1] * 2 * x2 * y * z2;
      g[2] = -2 * p[0] * (2 * y2 * z + 2 * x2 * z) + p[1] * 2 * x2 * y2 * z;
      break;
    }
    default: break;
  }
}

// ------------------------------------------------------------------ decoupled look-back
// Chained-scan tile protocol (Merrill & Garland 2016): st[tile] = flag << 32 | value with
// flag 1 = tile total published, 2 = inclusive prefix published; st[ntiles] = tile counter.
// All words start at zero.  A workgroup takes its tile index from the counter (so every
// earlier tile is already running), and wave 0 calls lookback_wave with the tile total:
// it publishes the total, sums the predecessors' published values 64 tiles at a time back
// to the nearest inclusive prefix, publishes its own inclusive prefix and returns the
// exclusive prefix (in every lane of wave 0).  Every wait ends: tile 0 publishes an
// inclusive prefix at once and every tile does after a finite walk.
constexpr uint64_t LB_AGG = 1ull << 32, LB_INC = 2ull << 32;

__device__ __forceinline__ uint32_t lookback_tile(uint64_t* st, int64_t ntiles) {
  return atomicAdd(reinterpret_cast<unsigned int*>(st + ntiles), 1u);
}

__device__ __forceinline__ uint32_t lookback_wave(uint64_t* st, int64_t b, uint32_t agg) {
  const int lane = threadIdx.x & 63;
  if (lane == 0)
    __hip_atomic_store(st + b, (b == 0 ? LB_INC : LB_AGG) | agg, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  uint32_t excl = 0;
  int64_t j = b - 1 - lane;
  while (b > 0) {
    uint64_t sv;
    for (;;) {
      sv = j >= 0 ? __hip_atomic_load(st + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : LB_INC;
      if (__ballot((sv >> 32) == 0) == 0) break;
      __builtin_amdgcn_s_sleep(1);
    }
    const uint64_t incm = __ballot((sv >> 32) == 2);
    const int stop = incm ? __ffsll((unsigned long long)incm) - 1 : 63;  // nearest inclusive prefix
    uint32_t x = lane <= stop ? (uint32_t)sv : 0u;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    excl += x;
    if (incm) break;
    j -= 64;
  }
  if (lane == 0 && b > 0)
    __hip_atomic_store(st + b, LB_INC | (excl + agg), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return excl;
}

// Block-wide exclusive scan of one value per thread (blockDim.x = 64 * NW); returns the
// thread's exclusive prefix, *agg = block total.  lw: NW words of LDS.  Contains barriers.
template <int NW>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* lw, uint32_t& agg) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t inc = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t u = __shfl_up(inc, o, 64);
    if (lane >= o) inc += u;
  }
  if (lane == 63) lw[w] = inc;
  __syncthreads();
  uint32_t pre = 0;
  agg = 0;
#pragma unroll
  for (int q = 0; q < NW; ++q) {
    const uint32_t t = lw[q];
    pre += q < w ? t : 0u;
    agg += t;
  }
  __syncthreads();
  return pre + inc - v;
}

// ------------------------------------------------------------------ primitives (prims.hip)
// Exclusive scan of n uint32 (in may alias out); *total (device) = sum, may be null.
// Status: scan_status_words(n) uint64 words, taken from ws and zeroed by the scan, or
// `cleared` (already zero on the stream, e.g. by a fill fused into an earlier kernel).
size_t scan_workspace(int64_t n);
int64_t scan_status_words(int64_t n);
int scan_exclusive(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total, Arena& ws, hipStream_t s,
                   uint64_t* cleared = nullptr);

// Packed scan: in = count (bits 0..7) | payload << 8, out = exclusive prefix << pb | payload.
int scan_packed(const uint32_t* in, uint32_t* out, int64_t n, int pb, uint32_t* total, Arena& ws, hipStream_t s,
                uint64_t* cleared = nullptr);

// Stable LSD radix sort of (uint64 key, int32 value) pairs on key bits [0, bits).
// vals_in == nullptr means values = index.  Result ends in (*keys_out, *vals_out), which
// point into one of the two buffer pairs.
size_t sort_workspace(int64_t n);
int radix_sort(uint64_t* keysA, int32_t* valsA, uint64_t* keysB, int32_t* valsB, const int32_t* vals_in, int64_t n,
               int bits, uint64_t** keys_out, int32_t** vals_out, Arena& ws, hipStream_t s);

}  // namespace ph
