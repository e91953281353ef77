// Library-wide state (error text, profiler) and the device primitives used by the
// connectivity kernels: a device-wide exclusive scan and a stable LSD radix sort of
// (uint64 key, int32 value) pairs.  Written for gfx950: wave64 ballots for the in-tile
// ranking, 256-thread workgroups (4 waves), one 4096-element tile per workgroup.
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"

namespace ph {

static thread_local std::string g_error;

void set_error(const std::string& msg) { g_error = msg; }
void clear_error() { g_error.clear(); }

int dev_flags_to_status(int f) {
  if (f & DEV_BADNODE) return err(PHFEM_EINVAL, "node, face or slot index out of range, or repeated node in a tet");
  if (f & DEV_ORIENT) return err(PHFEM_EORIENT, "a face occurs twice with the same orientation or in more than two tets");
  if (f & DEV_DEGEN) return err(PHFEM_EDEGEN, "zero-volume tet");
  if (f & DEV_NOFACE) return err(PHFEM_EINVAL, "boundary face is not a face of the mesh");
  return PHFEM_OK;
}

int check_params(const phfem_params* p) {
  if (!p) return err(PHFEM_EINVAL, "params is NULL");
  if (!(p->c > 0)) return err(PHFEM_ESINGULAR, "reaction coefficient c must be > 0 (kappa K + c M singular)");
  if (p->quad != PHFEM_QUAD_FACE_CENTROID && p->quad != PHFEM_QUAD_P1_INTERP) return err(PHFEM_EINVAL, "bad quad");
  if (p->precision != PHFEM_FP64 && p->precision != PHFEM_MIXED) return err(PHFEM_EINVAL, "bad precision");
  if (p->f_kind < 0 || p->f_kind > PHFEM_FUN_X2Y2Z2_LOAD || p->ud_kind < 0 || p->ud_kind > PHFEM_FUN_X2Y2Z2_LOAD ||
      p->g_kind < 0 || p->g_kind > PHFEM_FUN_X2Y2Z2_LOAD)
    return err(PHFEM_EINVAL, "bad function kind");
  return PHFEM_OK;
}

// ------------------------------------------------------------------ profiler
struct ProfRec {
  const char* name;
  hipEvent_t a, b;
  double bytes;
};
static bool g_prof = false;
static std::vector<ProfRec> g_recs;
static std::vector<hipEvent_t> g_pool;
static size_t g_pool_used = 0;
static std::mutex g_prof_mu;

static hipEvent_t pool_event() {
  if (g_pool_used == g_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    g_pool.push_back(e);
  }
  return g_pool[g_pool_used++];
}

bool profiling() { return g_prof; }

void prof_begin(const char* name, hipStream_t s, double bytes) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  ProfRec r{name, pool_event(), pool_event(), bytes};
  if (r.a) (void)hipEventRecord(r.a, s);
  g_recs.push_back(r);
}

void prof_end(hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (!g_recs.empty() && g_recs.back().b) (void)hipEventRecord(g_recs.back().b, s);
}

// ------------------------------------------------------------------ scan
// Single-pass exclusive scan with decoupled look-back (Merrill & Garland, "Single-pass
// Parallel Prefix Scan with Decoupled Look-back", 2016).  A workgroup takes the next tile
// index from a counter (so every earlier tile is already running), loads its 4096 items with
// coalesced loads, transposes them through LDS to 16 consecutive items per thread, publishes
// its tile total, and one wave walks back over the predecessors' published totals / inclusive
// prefixes, 64 tiles at a time, until it meets an inclusive prefix.  Results go back through
// LDS and out with coalesced stores: one read and one write of the data.
constexpr int SC_THREADS = 256;
constexpr int SC_ITEMS = 16;
constexpr int SC_TILE = SC_THREADS * SC_ITEMS;

__device__ __forceinline__ int sc_pad(int k) { return k + (k >> 5); }  // one pad word per 32

__global__ __launch_bounds__(SC_THREADS) void k_scan_clear(int64_t nw, uint64_t* __restrict__ st) {
  for (int64_t i = (int64_t)blockIdx.x * SC_THREADS + threadIdx.x; i < nw; i += (int64_t)gridDim.x * SC_THREADS)
    st[i] = 0;
}

// PACKED: in = count (bits 0..7) | payload << 8, out = prefix << pb | payload; else plain sums
template <bool PACKED>
__global__ __launch_bounds__(SC_THREADS) void k_scan_lookback(const uint32_t* in, int64_t n, int64_t ntiles,
                                                              uint64_t* __restrict__ st, int pb, uint32_t* out,
                                                              uint32_t* __restrict__ total) {
  __shared__ uint32_t tile[SC_TILE + SC_TILE / 32];
  __shared__ uint32_t lw[SC_THREADS / 64];
  __shared__ uint32_t s_tile, s_excl;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if (tid == 0) s_tile = lookback_tile(st, ntiles);
  __syncthreads();
  const int64_t b = s_tile;
  const int64_t base = b * SC_TILE;
#pragma unroll
  for (int i = 0; i < SC_ITEMS; ++i) {
    const int k = i * SC_THREADS + tid;
    tile[sc_pad(k)] = base + k < n ? in[base + k] : 0u;
  }
  __syncthreads();
  uint32_t v[SC_ITEMS];
  uint32_t sum = 0;
#pragma unroll
  for (int i = 0; i < SC_ITEMS; ++i) {
    v[i] = tile[sc_pad(tid * SC_ITEMS + i)];
    sum += PACKED ? (v[i] & 0xffu) : v[i];
  }
  uint32_t agg;
  const uint32_t tpre = block_excl_scan<SC_THREADS / 64>(sum, lw, agg);
  if (w == 0) {
    const uint32_t excl = lookback_wave(st, b, agg);
    if (lane == 0) {
      s_excl = excl;
      if (total && b == ntiles - 1) *total = excl + agg;
    }
  }
  __syncthreads();
  uint32_t run = s_excl + tpre;
#pragma unroll
  for (int i = 0; i < SC_ITEMS; ++i) {
    const uint32_t c = PACKED ? (v[i] & 0xffu) : v[i];
    tile[sc_pad(tid * SC_ITEMS + i)] = PACKED ? ((run << pb) | (v[i] >> 8)) : run;
    run += c;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < SC_ITEMS; ++i) {
    const int k = i * SC_THREADS + tid;
    if (base + k < n) out[base + k] = tile[sc_pad(k)];
  }
}

size_t scan_workspace(int64_t n) {
  Arena a;
  a.take<uint64_t>((size_t)((n + SC_TILE - 1) / SC_TILE) + 1);
  return a.size();
}

int64_t scan_status_words(int64_t n) { return (n + SC_TILE - 1) / SC_TILE + 1; }

static int scan_run(bool packed, const uint32_t* in, uint32_t* out, int64_t n, int pb, uint32_t* total, Arena& ws,
                    hipStream_t s, uint64_t* cleared) {
  const int64_t nt = (n + SC_TILE - 1) / SC_TILE;
  // per-tile status words, then the tile counter: zeroed here, or by the caller (cleared)
  uint64_t* st = cleared ? cleared : ws.take<uint64_t>((size_t)nt + 1);
  if (n == 0) return PHFEM_OK;
  if (!cleared)
    PH_LAUNCH("scan_clear", k_scan_clear, (unsigned)std::min<int64_t>((nt + SC_THREADS) / SC_THREADS, 1024),
              SC_THREADS, 0, s, nt + 1, st);
  if (packed)
    PH_LAUNCH_B("scanp", 8.0 * n, k_scan_lookback<true>, (unsigned)nt, SC_THREADS, 0, s, in, n, nt, st, pb, out,
                total);
  else
    PH_LAUNCH_B("scan", 8.0 * n, k_scan_lookback<false>, (unsigned)nt, SC_THREADS, 0, s, in, n, nt, st, 0, out,
                total);
  return PHFEM_OK;
}

int scan_exclusive(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* total, Arena& ws, hipStream_t s,
                   uint64_t* cleared) {
  return scan_run(false, in, out, n, 0, total, ws, s, cleared);
}

// Packed variant: in[i] = count (bits 0..7) | payload << 8; out[i] = (exclusive prefix of
// the counts) << pb | payload.  Used for per-row (first-appearance prefix, mask) records.
int scan_packed(const uint32_t* in, uint32_t* out, int64_t n, int pb, uint32_t* total, Arena& ws, hipStream_t s,
                uint64_t* cleared) {
  return scan_run(true, in, out, n, pb, total, ws, s, cleared);
}

// ------------------------------------------------------------------ radix sort
constexpr int RS_BITS = 8;
constexpr int RS_RADIX = 1 << RS_BITS;
constexpr int RS_THREADS = 256;
constexpr int RS_WAVES = RS_THREADS / 64;
constexpr int RS_ITEMS = 16;
constexpr int RS_TILE = RS_THREADS * RS_ITEMS;
static_assert(RS_RADIX == RS_THREADS, "one digit per thread in the offset pass");

// per-tile digit histogram, digit-major: hist[d * nblocks + b]
__global__ __launch_bounds__(RS_THREADS) void k_rs_hist(const uint64_t* __restrict__ keys, int64_t n, int shift,
                                                        uint32_t* __restrict__ hist, int64_t nblocks) {
  __shared__ uint32_t cnt[RS_WAVES][RS_RADIX];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int i = threadIdx.x; i < RS_WAVES * RS_RADIX; i += RS_THREADS) (&cnt[0][0])[i] = 0;
  __syncthreads();
  // wave-contiguous chunks; peers with the same digit aggregate before the LDS atomic
  int64_t wbase = (int64_t)blockIdx.x * RS_TILE + (int64_t)w * 64 * RS_ITEMS;
#pragma unroll 4
  for (int i = 0; i < RS_ITEMS; ++i) {
    int64_t idx = wbase + i * 64 + lane;
    bool valid = idx < n;
    uint32_t d = valid ? (uint32_t)((keys[idx] >> shift) & (RS_RADIX - 1)) : 0u;
    uint64_t peers = ballot(valid);
#pragma unroll
    for (int b = 0; b < RS_BITS; ++b) {
      uint64_t bb = ballot(valid && ((d >> b) & 1u));
      peers &= ((d >> b) & 1u) ? bb : ~bb;
    }
    if (valid && lane == __ffsll((unsigned long long)peers) - 1) atomicAdd(&cnt[w][d], (uint32_t)__popcll(peers));
  }
  __syncthreads();
  uint32_t s = 0;
#pragma unroll
  for (int ww = 0; ww < RS_WAVES; ++ww) s += cnt[ww][threadIdx.x];
  hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = s;
}

// Stable scatter: element order inside a tile is (wave, item, lane); each wave ranks its
// items with ballot-based peer masks and a per-wave digit counter in LDS.
__global__ __launch_bounds__(RS_THREADS) void k_rs_scatter(const uint64_t* __restrict__ kin,
                                                           const int32_t* __restrict__ vin, int64_t n, int shift,
                                                           const uint32_t* __restrict__ offs, int64_t nblocks,
                                                           uint64_t* __restrict__ kout, int32_t* __restrict__ vout) {
  __shared__ uint32_t wh[RS_WAVES][RS_RADIX];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int i = threadIdx.x; i < RS_WAVES * RS_RADIX; i += RS_THREADS) (&wh[0][0])[i] = 0;
  __syncthreads();
  const int64_t wbase = (int64_t)blockIdx.x * RS_TILE + (int64_t)w * 64 * RS_ITEMS;
  const uint64_t lt = (1ull << lane) - 1ull;
  uint64_t key[RS_ITEMS];
  int32_t val[RS_ITEMS];
  uint32_t rank[RS_ITEMS];
#pragma unroll
  for (int i = 0; i < RS_ITEMS; ++i) {
    int64_t idx = wbase + i * 64 + lane;
    bool valid = idx < n;
    key[i] = valid ? kin[idx] : 0ull;
    val[i] = valid ? (vin ? vin[idx] : (int32_t)idx) : 0;
  }
#pragma unroll
  for (int i = 0; i < RS_ITEMS; ++i) {
    int64_t idx = wbase + i * 64 + lane;
    bool valid = idx < n;
    uint32_t d = (uint32_t)((key[i] >> shift) & (RS_RADIX - 1));
    uint64_t peers = ballot(valid);
#pragma unroll
    for (int b = 0; b < RS_BITS; ++b) {
      uint64_t bb = ballot(valid && ((d >> b) & 1u));
      peers &= ((d >> b) & 1u) ? bb : ~bb;
    }
    int leader = valid ? __ffsll((unsigned long long)peers) - 1 : lane;
    uint32_t base = 0;
    if (valid && lane == leader) base = atomicAdd(&wh[w][d], (uint32_t)__popcll(peers));
    base = __shfl(base, leader, 64);
    rank[i] = base + (uint32_t)__popcll(peers & lt);
  }
  __syncthreads();
  {
    const int d = threadIdx.x;
    uint32_t run = offs[(int64_t)d * nblocks + blockIdx.x];
#pragma unroll
    for (int ww = 0; ww < RS_WAVES; ++ww) {
      uint32_t c = wh[ww][d];
      wh[ww][d] = run;
      run += c;
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < RS_ITEMS; ++i) {
    int64_t idx = wbase + i * 64 + lane;
    if (idx < n) {
      uint32_t d = (uint32_t)((key[i] >> shift) & (RS_RADIX - 1));
      uint32_t pos = wh[w][d] + rank[i];
      kout[pos] = key[i];
      vout[pos] = val[i];
    }
  }
}

size_t sort_workspace(int64_t n) {
  int64_t nb = (n + RS_TILE - 1) / RS_TILE;
  Arena a;
  a.take<uint32_t>((size_t)(nb * RS_RADIX));
  size_t s = a.size() + scan_workspace(nb * RS_RADIX);
  return s;
}

int radix_sort(uint64_t* keysA, int32_t* valsA, uint64_t* keysB, int32_t* valsB, const int32_t* vals_in, int64_t n,
               int bits, uint64_t** keys_out, int32_t** vals_out, Arena& ws, hipStream_t s) {
  if (n >= (int64_t(1) << 32)) return err(PHFEM_EINVAL, "sort size exceeds 2^32");
  int64_t nb = (n + RS_TILE - 1) / RS_TILE;
  uint32_t* hist = ws.take<uint32_t>((size_t)(nb * RS_RADIX));
  size_t mark = ws.off;
  // input keys in keysA, values in vals_in (identity when null; must not be valsB)
  uint64_t* kbuf[2] = {keysA, keysB};
  int32_t* vbuf[2] = {valsA, valsB};
  int cur = 0;
  const int32_t* vsrc = vals_in;
  if (bits <= 0) bits = RS_BITS;  // still run one pass so values are materialised
  for (int shift = 0; shift < bits; shift += RS_BITS) {
    ws.off = mark;
    PH_LAUNCH_B("rs_hist", 8.0 * n, k_rs_hist, (unsigned)nb, RS_THREADS, 0, s, (const uint64_t*)kbuf[cur], n, shift,
                hist, nb);
    int rc = scan_exclusive(hist, hist, nb * RS_RADIX, nullptr, ws, s);
    if (rc) return rc;
    PH_LAUNCH_B("rs_scatter", (vsrc ? 24.0 : 20.0) * n, k_rs_scatter, (unsigned)nb, RS_THREADS, 0, s,
                (const uint64_t*)kbuf[cur], vsrc, n, shift, (const uint32_t*)hist, nb, kbuf[cur ^ 1], vbuf[cur ^ 1]);
    cur ^= 1;
    vsrc = vbuf[cur];
  }
  *keys_out = kbuf[cur];
  *vals_out = vbuf[cur];
  return PHFEM_OK;
}

// ------------------------------------------------------------------ counter calibration
// Streams of known size for scaling the HBM traffic counters (FETCH_SIZE, WRITE_SIZE):
// read n doubles (16-byte loads, one partial sum per workgroup written), write n doubles,
// copy n doubles, or gather n 32-byte records at scattered positions of an array of m.
constexpr int CALT = 256;

__global__ __launch_bounds__(CALT) void k_cal_read(int64_t n2, const double2* __restrict__ src,
                                                   double* __restrict__ part) {
  double a = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * CALT + threadIdx.x; i < n2; i += (int64_t)gridDim.x * CALT) {
    const double2 v = src[i];
    a += v.x + v.y;
  }
  __shared__ double l[CALT / 64];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) a += __shfl_down(a, o, 64);
  if ((threadIdx.x & 63) == 0) l[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (l[0] + l[1]) + (l[2] + l[3]);
}

__global__ __launch_bounds__(CALT) void k_cal_write(int64_t n2, double2* __restrict__ dst, double v) {
  for (int64_t i = (int64_t)blockIdx.x * CALT + threadIdx.x; i < n2; i += (int64_t)gridDim.x * CALT)
    dst[i] = make_double2(v, v + 1.0);
}

__global__ __launch_bounds__(CALT) void k_cal_copy(int64_t n2, const double2* __restrict__ src,
                                                   double2* __restrict__ dst) {
  for (int64_t i = (int64_t)blockIdx.x * CALT + threadIdx.x; i < n2; i += (int64_t)gridDim.x * CALT) dst[i] = src[i];
}

// record j of the gather: (j * 2654435761) mod m, an odd multiplier over a power-of-two m
// (a permutation of the records); each 32-byte record read with two 16-byte loads
__global__ __launch_bounds__(CALT) void k_cal_gather(int64_t n, int64_t m, const double4* __restrict__ src,
                                                     double* __restrict__ part) {
  double a = 0.0;
  for (int64_t j = (int64_t)blockIdx.x * CALT + threadIdx.x; j < n; j += (int64_t)gridDim.x * CALT) {
    const uint64_t q = ((uint64_t)j * 2654435761ull) & (uint64_t)(m - 1);
    const double4 v = src[q];
    a += (v.x + v.y) + (v.z + v.w);
  }
  __shared__ double l[CALT / 64];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) a += __shfl_down(a, o, 64);
  if ((threadIdx.x & 63) == 0) l[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (l[0] + l[1]) + (l[2] + l[3]);
}

}  // namespace ph

// ------------------------------------------------------------------ C-ABI: errors, profiler
extern "C" {

const char* phfem_last_error(void) { return ph::g_error.c_str(); }
int phfem_abi_version(void) { return 2; }

void phfem_profile_enable(int32_t on) { ph::g_prof = on != 0; }

int phfem_profile_stream(int32_t op, const double* src, double* dst, int64_t n, int64_t m, phfem_stream_t stream_) {
  using namespace ph;
  clear_error();
  hipStream_t s = (hipStream_t)stream_;
  const unsigned G = 4096;  // grid-stride: partial sums of the read kernels fit dst[G]
  if (n <= 0 || (op != 3 && (n & 1))) return err(PHFEM_EINVAL, "n must be positive (and even for streams)");
  if (reinterpret_cast<uintptr_t>(src) & 31 || reinterpret_cast<uintptr_t>(dst) & 15)
    return err(PHFEM_EINVAL, "src 32-byte and dst 16-byte aligned");
  switch (op) {
    case 0:
      if (!src || !dst) return err(PHFEM_EINVAL, "null src/dst");
      PH_LAUNCH_B("cal_read", 8.0 * n, k_cal_read, G, CALT, 0, s, n / 2, (const double2*)src, dst);
      return PHFEM_OK;
    case 1:
      if (!dst) return err(PHFEM_EINVAL, "null dst");
      PH_LAUNCH_B("cal_write", 8.0 * n, k_cal_write, G, CALT, 0, s, n / 2, (double2*)dst, 1.0);
      return PHFEM_OK;
    case 2:
      if (!src || !dst) return err(PHFEM_EINVAL, "null src/dst");
      PH_LAUNCH_B("cal_copy", 16.0 * n, k_cal_copy, G, CALT, 0, s, n / 2, (const double2*)src, (double2*)dst);
      return PHFEM_OK;
    case 3:
      if (!src || !dst || m <= 0 || (m & (m - 1))) return err(PHFEM_EINVAL, "gather: m must be a power of two");
      PH_LAUNCH_B("cal_gather", 32.0 * n, k_cal_gather, G, CALT, 0, s, n, m, (const double4*)src, dst);
      return PHFEM_OK;
    default:
      return err(PHFEM_EINVAL, "op must be 0 (read), 1 (write), 2 (copy) or 3 (gather)");
  }
}

void phfem_profile_reset(void) {
  std::lock_guard<std::mutex> lk(ph::g_prof_mu);
  ph::g_recs.clear();
  ph::g_pool_used = 0;
}

int phfem_profile_query(const char* name, int64_t* launches, double* total_ms, double* total_bytes) {
  std::lock_guard<std::mutex> lk(ph::g_prof_mu);
  int64_t n = 0;
  double ms = 0, by = 0;
  for (auto& r : ph::g_recs) {
    if (std::strcmp(r.name, name) != 0 || !r.a || !r.b) continue;
    if (hipEventSynchronize(r.b) != hipSuccess) return ph::err(PHFEM_EHIP, "event sync");
    float t = 0;
    if (hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) return ph::err(PHFEM_EHIP, "event elapsed");
    ms += t;
    by += r.bytes;
    ++n;
  }
  *launches = n;
  *total_ms = ms;
  if (total_bytes) *total_bytes = by;
  return PHFEM_OK;
}

int phfem_profile_names(char* buf, size_t buf_bytes) {
  std::lock_guard<std::mutex> lk(ph::g_prof_mu);
  std::vector<std::string> seen;
  for (auto& r : ph::g_recs) {
    bool have = false;
    for (auto& s : seen) have = have || s == r.name;
    if (!have) seen.push_back(r.name);
  }
  std::string out;
  for (size_t i = 0; i < seen.size(); ++i) out += (i ? "," : "") + seen[i];
  if (buf_bytes == 0) return PHFEM_EINVAL;
  std::strncpy(buf, out.c_str(), buf_bytes - 1);
  buf[buf_bytes - 1] = 0;
  return PHFEM_OK;
}

}  // extern "C"
