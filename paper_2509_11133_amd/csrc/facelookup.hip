// Boundary-face lookup: which faces of the mesh numbering are the triangles of a boundary
// face list (the Multiplier routine of Section 4.4 finds its Neumann faces g_NFs this way
// before the load LN and the reduced face space are formed).
//
// A triangle list is small next to the mesh (boundary faces are O(nF^(2/3))), so the
// triangles go into an open-addressing hash table in the workspace (one int32 slot per entry,
// at most half full, keyed by the sorted node triple), and one pass over the faces probes it
// with every boundary face.  Three kernels, one readback; no sort.
#include "common.hpp"

namespace ph {

constexpr int LT = 256;

__device__ __forceinline__ void sort3(int& a, int& b, int& c) {
  if (a > b) {
    int t = a;
    a = b;
    b = t;
  }
  if (b > c) {
    int t = b;
    b = c;
    c = t;
  }
  if (a > b) {
    int t = a;
    a = b;
    b = t;
  }
}

// 64-bit mix of the sorted triple (splitmix64 finalizer), reduced to the table size
__device__ __forceinline__ uint32_t tri_hash(int a, int b, int c, uint32_t mask) {
  uint64_t h = (uint64_t)(uint32_t)a * 0x9E3779B97F4A7C15ull ^ (uint64_t)(uint32_t)b * 0xC2B2AE3D27D4EB4Full ^
               (uint64_t)(uint32_t)c * 0x165667B19E3779F9ull;
  h ^= h >> 30;
  h *= 0xBF58476D1CE4E5B9ull;
  h ^= h >> 27;
  h *= 0x94D049BB133111EBull;
  h ^= h >> 31;
  return (uint32_t)h & mask;
}

__global__ __launch_bounds__(LT) void k_lookup_init(uint32_t H, int64_t n, int32_t* __restrict__ tab,
                                                    int32_t* __restrict__ match, int* __restrict__ flag) {
  const int64_t i = (int64_t)blockIdx.x * LT + threadIdx.x;
  if (i < H) tab[i] = -1;
  if (i < n) match[i] = -1;
  if (i == 0) *flag = 0;
}

// triangle j into the table (invalid triangles -- a node out of range or repeated -- are
// flagged and left out)
__global__ __launch_bounds__(LT) void k_lookup_insert(int64_t n, int64_t nC, const int32_t* __restrict__ tris,
                                                      uint32_t mask, int32_t* __restrict__ tab, int* __restrict__ flag) {
  const int64_t j = (int64_t)blockIdx.x * LT + threadIdx.x;
  if (j >= n) return;
  int a = tris[j], b = tris[n + j], c = tris[2 * n + j];
  if ((uint32_t)a >= (uint64_t)nC || (uint32_t)b >= (uint64_t)nC || (uint32_t)c >= (uint64_t)nC || a == b ||
      b == c || a == c) {
    atomicOr(flag, 1);
    return;
  }
  sort3(a, b, c);
  uint32_t h = tri_hash(a, b, c, mask);
  while (atomicCAS(&tab[h], -1, (int32_t)j) != -1) h = (h + 1) & mask;
}

// face f: flags[f] = 1 when it is a boundary face listed in the table, and match[j] = f for
// every listed triangle j with its node set (the walk ends at the first empty slot; the table
// is at most half full)
__global__ __launch_bounds__(LT) void k_lookup_probe(int64_t nF, const int32_t* __restrict__ faces,
                                                     const int32_t* __restrict__ face2tet, int64_t n,
                                                     const int32_t* __restrict__ tris, uint32_t mask,
                                                     const int32_t* __restrict__ tab, uint8_t* __restrict__ flags,
                                                     int32_t* __restrict__ match) {
  const int64_t f = (int64_t)blockIdx.x * LT + threadIdx.x;
  if (f >= nF) return;
  bool hit = false;
  if (face2tet[nF + f] < 0) {
    int a = faces[f], b = faces[nF + f], c = faces[2 * nF + f];
    sort3(a, b, c);
    for (uint32_t h = tri_hash(a, b, c, mask);; h = (h + 1) & mask) {
      const int j = tab[h];
      if (j < 0) break;
      int p = tris[j], q = tris[n + j], r = tris[2 * n + j];
      sort3(p, q, r);
      if (p == a && q == b && r == c) {
        match[j] = (int32_t)f;
        hit = true;
      }
    }
  }
  flags[f] = hit ? 1 : 0;
}

__global__ __launch_bounds__(LT) void k_lookup_check(int64_t n, const int32_t* __restrict__ match,
                                                     int32_t* __restrict__ face_of, int* __restrict__ flag) {
  const int64_t j = (int64_t)blockIdx.x * LT + threadIdx.x;
  if (j >= n) return;
  const int32_t f = match[j];
  if (f < 0) atomicOr(flag, 2);
  if (face_of) face_of[j] = f;
}

static uint32_t table_size(int64_t n) {
  uint32_t H = 64;
  while ((int64_t)H < 2 * n) H <<= 1;
  return H;
}

}  // namespace ph

using namespace ph;

extern "C" size_t phfem_face_lookup_workspace(int64_t n) {
  if (n <= 0 || n > (int64_t(1) << 29)) return 0;
  Arena a;
  a.take<int32_t>(table_size(n));
  a.take<int32_t>(n);
  a.take<int>(1);
  return a.size();
}

extern "C" int phfem_face_lookup(int64_t nC, int64_t nF, const int32_t* faces, const int32_t* face2tet, int64_t n,
                                 const int32_t* tris, void* work, size_t work_bytes, uint8_t* flags, int32_t* face_of,
                                 phfem_stream_t stream_) {
  clear_error();
  hipStream_t s = (hipStream_t)stream_;
  if (nC <= 0 || nF <= 0 || nF >= (int64_t(1) << 31) || !faces || !face2tet || !flags)
    return err(PHFEM_EINVAL, "bad face lookup arguments");
  if (n < 0 || n > (int64_t(1) << 29) || (n > 0 && !tris)) return err(PHFEM_EINVAL, "bad triangle list");
  if (n == 0) {  // nothing listed: every flag 0
    PH_HIP(hipMemsetAsync(flags, 0, (size_t)nF, s));
    return PHFEM_OK;
  }
  if (!work || work_bytes < phfem_face_lookup_workspace(n))
    return err(PHFEM_EWORKSPACE, "face lookup workspace too small");
  Arena a(work, work_bytes);
  const uint32_t H = table_size(n);
  int32_t* tab = a.take<int32_t>(H);
  int32_t* match = a.take<int32_t>(n);
  int* dflag = a.take<int>(1);
  PH_LAUNCH("lookup_init", k_lookup_init, grid_for(std::max<int64_t>(H, n), LT), LT, 0, s, H, n, tab, match, dflag);
  PH_LAUNCH("lookup_insert", k_lookup_insert, grid_for(n, LT), LT, 0, s, n, nC, tris, H - 1, tab, dflag);
  PH_LAUNCH_B("lookup_probe", 5.0 * nF, k_lookup_probe, grid_for(nF, LT), LT, 0, s, nF, faces, face2tet, n, tris, H - 1,
              (const int32_t*)tab, flags, match);
  PH_LAUNCH("lookup_check", k_lookup_check, grid_for(n, LT), LT, 0, s, n, (const int32_t*)match, face_of, dflag);
  int h = 0;
  PH_HIP(hipMemcpyAsync(&h, dflag, sizeof(int), hipMemcpyDeviceToHost, s));
  PH_HIP(hipStreamSynchronize(s));
  if (h & 1) return err(PHFEM_EINVAL, "a listed triangle has a node out of range or a repeated node");
  if (h & 2) return err(PHFEM_EINVAL, "a listed triangle is not a boundary face of the mesh");
  return PHFEM_OK;
}
