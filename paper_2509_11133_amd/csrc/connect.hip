// Connectivity on the device (Sections 3.1-3.3): Nodes-to-Edge numbering (NumEdges),
// the neighbour across every face (the role of Edges2Tetra) and the face numbering of
// FacesUp / fullFaces.
//
// Both numberings are "rank of first appearance" over a position order (edges: 6t + j,
// faces: 4t + k): find each occurrence's first appearance (head), count heads per tet and
// scan -> per-tet prefix, then every occurrence takes the id prefix(t_head) + (heads of
// t_head before j_head).  Three ways to find the heads, with identical outputs:
//  * meshes of at most SMALL_NE tets: one workgroup, every occurrence compared with the
//    earlier ones in LDS;
//  * the general path: occurrences bucketed by their lowest node (counting sort), each bucket
//    resolved in LDS (node buckets, below);
//  * the fallback for a node in thousands of tets (or on request): a stable radix sort of
//    (key, position), segment heads found with wave64 ballots over the sorted keys.
#include "common.hpp"

namespace ph {

constexpr int CT = 256;  // threads per workgroup for the element-wise kernels

static inline int bits_for(int64_t n) {  // bits needed for values in [0, n)
  int b = 1;
  while ((int64_t(1) << b) < n) ++b;
  return b;
}

// ---------------------------------------------------------------- edges
// keys[6t+j] = (min << nb) | max of local edge j of tet t; validates node ids.
__global__ __launch_bounds__(CT) void k_edge_keys(int64_t nE, int64_t nC, const int32_t* __restrict__ tet, int nb,
                                                  uint64_t* __restrict__ keys, int* __restrict__ flags) {
  int64_t t = (int64_t)blockIdx.x * CT + threadIdx.x;
  if (t >= nE) return;
  int v[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) v[i] = tet[i * nE + t];
  bool bad = false;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    bad |= v[i] < 0 || v[i] >= nC;
#pragma unroll
    for (int j = i + 1; j < 4; ++j) bad |= v[i] == v[j];
  }
  if (bad) atomicOr(flags, DEV_BADNODE);
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    uint32_t a = (uint32_t)v[ev0(j)], b = (uint32_t)v[ev1(j)];
    uint32_t lo = a < b ? a : b, hi = a < b ? b : a;
    keys[6 * t + j] = ((uint64_t)lo << nb) | hi;
  }
}

// first[pos] = 1 if the sorted element s starts a segment of equal keys
__global__ __launch_bounds__(CT) void k_mark_heads(int64_t n, const uint64_t* __restrict__ sk,
                                                   const int32_t* __restrict__ sv, uint32_t vmask,
                                                   uint8_t* __restrict__ first) {
  int64_t s = (int64_t)blockIdx.x * CT + threadIdx.x;
  if (s >= n) return;
  bool head = s == 0 || sk[s] != sk[s - 1];
  first[(uint32_t)sv[s] & vmask] = head ? 1 : 0;
}

// cnt[t] = number of first appearances among the `per` positions of tet t
template <int PER>
__global__ __launch_bounds__(CT) void k_count_heads(int64_t nE, const uint8_t* __restrict__ first,
                                                    uint32_t* __restrict__ cnt) {
  int64_t t = (int64_t)blockIdx.x * CT + threadIdx.x;
  if (t > nE) return;
  uint32_t c = 0;
  if (t < nE) {
#pragma unroll
    for (int j = 0; j < PER; ++j) c += first[PER * t + j];
  }
  cnt[t] = c;  // cnt[nE] = 0 (room for the total)
}

// id of the first appearance at position p = PER*t + j
template <int PER>
__device__ __forceinline__ int32_t head_id(int64_t p, const uint8_t* __restrict__ first,
                                           const uint32_t* __restrict__ prefix) {
  int64_t t = p / PER;
  int j = (int)(p - PER * t);
  uint32_t id = prefix[t];
  for (int i = 0; i < j; ++i) id += first[PER * t + i];
  return (int32_t)id;
}

// Position of the segment head of sorted element s: nearest head at or below this lane in
// the wave (ballot), else walk back in memory (segments are a few elements long).
__device__ __forceinline__ int64_t find_head(int64_t s, bool valid, uint64_t key, bool head,
                                             const uint64_t* __restrict__ sk) {
  const int lane = lane_id();
  uint64_t hm = ballot(head);
  if (!valid) return s;
  uint64_t le = (lane == 63) ? ~0ull : ((2ull << lane) - 1ull);
  uint64_t m = hm & le;
  if (m) {
    int hl = 63 - __clzll((long long)m);
    return s - (lane - hl);
  }
  int64_t h = s - lane;  // first element of this wave's window; its head lies before it
  while (h > 0 && sk[h - 1] == key) --h;
  return h;
}

// nEd is read from the device (the scan total)
__global__ __launch_bounds__(CT) void k_edge_assign(int64_t n, int64_t nE, const uint32_t* __restrict__ nEdp, int nb,
                                                    const uint64_t* __restrict__ sk, const int32_t* __restrict__ sv,
                                                    const uint8_t* __restrict__ first,
                                                    const uint32_t* __restrict__ prefix,
                                                    int32_t* __restrict__ tet2edge, int32_t* __restrict__ edges,
                                                    int32_t* __restrict__ eft, uint32_t* __restrict__ headflag) {
  int64_t s = (int64_t)blockIdx.x * CT + threadIdx.x;
  bool valid = s < n;
  uint64_t key = valid ? sk[s] : 0;
  bool head = valid && (s == 0 || sk[s - 1] != key);
  int64_t h = find_head(s, valid, key, head, sk);
  if (!valid) return;
  int64_t ph = (int64_t)sv[h];
  int32_t id = head_id<6>(ph, first, prefix);
  int64_t p = (int64_t)sv[s];
  int64_t t = p / 6;
  int j = (int)(p - 6 * t);
  tet2edge[j * nE + t] = id;
  if (head) {
    const int64_t nEd = *nEdp;
    edges[id] = (int32_t)(key >> nb);
    edges[nEd + id] = (int32_t)(key & ((1ull << nb) - 1ull));
    eft[id] = (int32_t)t;
  }
  if (headflag) headflag[s] = head ? 1u : 0u;
}

// Nodes2Edge (upper triangle) CSR from the sorted unique keys; uidx = exclusive scan of
// the head flags in sorted order (= rank of the key among the distinct keys).
__global__ __launch_bounds__(CT) void k_n2e_fill(int64_t n, int nb, const uint64_t* __restrict__ sk,
                                                 const int32_t* __restrict__ sv, const uint32_t* __restrict__ uidx,
                                                 int64_t nE, const int32_t* __restrict__ tet2edge,
                                                 int32_t* __restrict__ col, int32_t* __restrict__ eid,
                                                 uint32_t* __restrict__ rowcnt) {
  int64_t s = (int64_t)blockIdx.x * CT + threadIdx.x;
  if (s >= n) return;
  uint64_t key = sk[s];
  if (s > 0 && sk[s - 1] == key) return;
  uint32_t u = uidx[s];
  int64_t p = sv[s];
  int64_t t = p / 6;
  int j = (int)(p - 6 * t);
  col[u] = (int32_t)(key & ((1ull << nb) - 1ull));
  eid[u] = tet2edge[j * nE + t];
  atomicAdd(&rowcnt[key >> nb], 1u);
}

// ---------------------------------------------------------------- faces
// key of local face k = (min node << eb) | edge opposite to that node within the face;
// value = slot 4t+k with the parity of the tuple's node order in bit 30.
__global__ __launch_bounds__(CT) void k_face_keys(int64_t nE, const int32_t* __restrict__ tet,
                                                  const int32_t* __restrict__ t2e, int eb,
                                                  uint64_t* __restrict__ keys, int32_t* __restrict__ vals) {
  int64_t t = (int64_t)blockIdx.x * CT + threadIdx.x;
  if (t >= nE) return;
  int v[4], e[6];
#pragma unroll
  for (int i = 0; i < 4; ++i) v[i] = tet[i * nE + t];
#pragma unroll
  for (int j = 0; j < 6; ++j) e[j] = t2e[j * nE + t];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int a = fv(k, 0), b = fv(k, 1), c = fv(k, 2);
    int na = v[a], nb_ = v[b], nc = v[c];
    int lo, oe;
    if (na < nb_ && na < nc) {
      lo = na;
      oe = e[eidx(b, c)];
    } else if (nb_ < nc) {
      lo = nb_;
      oe = e[eidx(a, c)];
    } else {
      lo = nc;
      oe = e[eidx(a, b)];
    }
    int parity = ((na > nb_) + (na > nc) + (nb_ > nc)) & 1;
    keys[4 * t + k] = ((uint64_t)(uint32_t)lo << eb) | (uint32_t)oe;
    vals[4 * t + k] = (int32_t)((4 * t + k) | ((int64_t)parity << 30));
  }
}

constexpr uint32_t SLOT_MASK = (1u << 30) - 1u;

// nF is read from the device (the scan total), so the host need not wait for it
__global__ __launch_bounds__(CT) void k_face_assign(int64_t n, int64_t nE, const uint32_t* __restrict__ nFp,
                                                    const uint64_t* __restrict__ sk, const int32_t* __restrict__ sv,
                                                    const uint8_t* __restrict__ first,
                                                    const uint32_t* __restrict__ prefix,
                                                    const int32_t* __restrict__ tet, int32_t* __restrict__ faces,
                                                    int32_t* __restrict__ tet2face, int8_t* __restrict__ sigma,
                                                    int32_t* __restrict__ face2tet, int32_t* __restrict__ nbr,
                                                    int* __restrict__ flags) {
  int64_t s = (int64_t)blockIdx.x * CT + threadIdx.x;
  if (s >= n) return;
  const int64_t nF = *nFp;
  uint64_t key = sk[s];
  bool head = s == 0 || sk[s - 1] != key;
  if (head) {
    uint32_t v0 = (uint32_t)sv[s];
    int64_t q0 = v0 & SLOT_MASK;
    int64_t t0 = q0 >> 2;
    int k0 = (int)(q0 & 3);
    int32_t id = head_id<4>(q0, first, prefix);
#pragma unroll
    for (int m = 0; m < 3; ++m) faces[m * nF + id] = tet[fv(k0, m) * nE + t0];
    face2tet[id] = (int32_t)q0;
    tet2face[k0 * nE + t0] = id;
    sigma[k0 * nE + t0] = 1;
    bool two = s + 1 < n && sk[s + 1] == key;
    if (two) {
      uint32_t v1 = (uint32_t)sv[s + 1];
      int64_t q1 = v1 & SLOT_MASK;
      face2tet[nF + id] = (int32_t)q1;
      if (nbr) nbr[k0 * nE + t0] = (int32_t)(q1 >> 2);
      bool three = s + 2 < n && sk[s + 2] == key;
      if (three || ((v0 >> 30) == (v1 >> 30))) atomicOr(flags, DEV_ORIENT);
    } else {
      face2tet[nF + id] = -1;
      if (nbr) nbr[k0 * nE + t0] = -1;
    }
  } else {
    if (s >= 2 && sk[s - 2] == key) return;  // third occurrence: flagged by the head
    int64_t q0 = (uint32_t)sv[s - 1] & SLOT_MASK;
    int64_t q1 = (uint32_t)sv[s] & SLOT_MASK;
    int64_t t1 = q1 >> 2;
    int k1 = (int)(q1 & 3);
    int32_t id = head_id<4>(q0, first, prefix);
    tet2face[k1 * nE + t1] = id;
    sigma[k1 * nE + t1] = -1;
    if (nbr) nbr[k1 * nE + t1] = (int32_t)(q0 >> 2);
  }
}

// ---------------------------------------------------------------- small meshes
// A mesh of at most SMALL_NE tets in one workgroup with everything in LDS: the same keys and
// the same numberings (rank of first appearance over positions 6t + j and 4t + k), with each
// occurrence's first appearance found by comparing it with the earlier positions instead of
// by a sort -- one launch instead of about twenty small ones (the level-0 mesh of a
// refinement chain).  out3 = {nEd, nF, device flags}.
constexpr int SMALL_NE = 256;
constexpr int SMT = 1024;

// exclusive prefix over positions [0, n) of flag(p), n <= 2 SMT, positions in chunks of two
template <class F>
__device__ __forceinline__ uint32_t small_scan(int n, F flag, int* spre, uint32_t* lw) {
  const int p0 = 2 * (int)threadIdx.x;
  const uint32_t f0 = p0 < n ? flag(p0) : 0u, f1 = p0 + 1 < n ? flag(p0 + 1) : 0u;
  uint32_t total;
  const uint32_t pre = block_excl_scan<SMT / 64>(f0 + f1, lw, total);
  if (p0 < n) spre[p0] = (int)pre;
  if (p0 + 1 < n) spre[p0 + 1] = (int)(pre + f0);
  return total;
}

__global__ __launch_bounds__(SMT) void k_connect_small(int nC, int nE, const int32_t* __restrict__ tet, int want_faces,
                                                       int32_t* __restrict__ edges, int32_t* __restrict__ tet2edge,
                                                       int32_t* __restrict__ eft, int32_t* __restrict__ pre,
                                                       int32_t* __restrict__ faces, int32_t* __restrict__ tet2face,
                                                       int8_t* __restrict__ sigma, int32_t* __restrict__ face2tet,
                                                       int32_t* __restrict__ nbr, uint32_t* __restrict__ out3) {
  __shared__ int sv[4 * SMALL_NE];       // node ids, 4 t + i
  __shared__ uint64_t sk[6 * SMALL_NE];  // keys in position order (edges, then faces)
  __shared__ int sh[6 * SMALL_NE];       // position of the first occurrence of the same key
  __shared__ int spre[6 * SMALL_NE];     // exclusive count of first occurrences before a position
  __shared__ int sid[6 * SMALL_NE];      // edge id per edge position
  __shared__ uint8_t spar[4 * SMALL_NE];
  __shared__ uint32_t lw[SMT / 64];
  __shared__ int sflag;
  const int n6 = 6 * nE, n4 = 4 * nE;
  if (threadIdx.x == 0) sflag = 0;
  __syncthreads();
  for (int t = threadIdx.x; t < nE; t += SMT) {
    int v[4];
    bool bad = false;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      v[i] = tet[i * nE + t];
      sv[4 * t + i] = v[i];
      bad |= v[i] < 0 || v[i] >= nC;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = i + 1; j < 4; ++j) bad |= v[i] == v[j];
    if (bad) atomicOr(&sflag, DEV_BADNODE);
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      const uint32_t a = (uint32_t)v[ev0(j)], b = (uint32_t)v[ev1(j)];
      sk[6 * t + j] = ((uint64_t)(a < b ? a : b) << 32) | (a < b ? b : a);
    }
  }
  __syncthreads();
  // edges: first occurrence of every key, ranks of the first occurrences in position order
  for (int p = threadIdx.x; p < n6; p += SMT) {
    const uint64_t key = sk[p];
    int h = p;
    for (int q = 0; q < p; ++q)
      if (sk[q] == key) {
        h = q;
        break;
      }
    sh[p] = h;
  }
  __syncthreads();
  const uint32_t nEd = small_scan(n6, [&](int p) { return sh[p] == p ? 1u : 0u; }, spre, lw);
  __syncthreads();
  for (int p = threadIdx.x; p < n6; p += SMT) {
    const int t = p / 6, j = p - 6 * t, id = spre[sh[p]];
    sid[p] = id;
    tet2edge[j * nE + t] = id;
    if (sh[p] == p) {
      edges[id] = (int32_t)(sk[p] >> 32);
      edges[nEd + id] = (int32_t)(sk[p] & 0xffffffffu);
      eft[id] = t;
    }
    if (j == 0) pre[t] = spre[p];
  }
  __syncthreads();
  uint32_t nF = 0;
  if (want_faces) {
    // faces: key (min node, id of the edge opposite it within the face), parity of the tuple
    for (int p = threadIdx.x; p < n4; p += SMT) {
      const int t = p >> 2, k = p & 3;
      const int a = fv(k, 0), b = fv(k, 1), c = fv(k, 2);
      const int na = sv[4 * t + a], nb_ = sv[4 * t + b], nc = sv[4 * t + c];
      int lo, oe;
      if (na < nb_ && na < nc) {
        lo = na;
        oe = sid[6 * t + eidx(b, c)];
      } else if (nb_ < nc) {
        lo = nb_;
        oe = sid[6 * t + eidx(a, c)];
      } else {
        lo = nc;
        oe = sid[6 * t + eidx(a, b)];
      }
      sk[p] = ((uint64_t)(uint32_t)lo << 32) | (uint32_t)oe;
      spar[p] = (uint8_t)(((na > nb_) + (na > nc) + (nb_ > nc)) & 1);
    }
    __syncthreads();
    for (int p = threadIdx.x; p < n4; p += SMT) {
      const uint64_t key = sk[p];
      int h = p;
      for (int q = 0; q < p; ++q)
        if (sk[q] == key) {
          h = q;
          break;
        }
      sh[p] = h;
    }
    __syncthreads();
    nF = small_scan(n4, [&](int p) { return sh[p] == p ? 1u : 0u; }, spre, lw);
    __syncthreads();
    for (int p = threadIdx.x; p < n4; p += SMT) {
      const int h = sh[p], t = p >> 2, k = p & 3, id = spre[h];
      const uint64_t key = sk[p];
      if (h == p) {  // owner: the later occurrences give the neighbour and the orientation check
        int q1 = -1, more = 0;
        for (int q = p + 1; q < n4; ++q)
          if (sk[q] == key) {
            if (q1 < 0)
              q1 = q;
            else
              more = 1;
          }
        if (more || (q1 >= 0 && spar[q1] == spar[p])) atomicOr(&sflag, DEV_ORIENT);
#pragma unroll
        for (int m = 0; m < 3; ++m) faces[m * nF + id] = sv[4 * t + fv(k, m)];
        face2tet[id] = p;
        face2tet[nF + id] = q1;
        tet2face[k * nE + t] = id;
        sigma[k * nE + t] = 1;
        if (nbr) nbr[k * nE + t] = q1 >= 0 ? (q1 >> 2) : -1;
      } else {
        bool second = true;  // a third occurrence is left to the owner's check
        for (int q = h + 1; q < p; ++q) second = second && sk[q] != key;
        if (second) {
          tet2face[k * nE + t] = id;
          sigma[k * nE + t] = -1;
          if (nbr) nbr[k * nE + t] = h >> 2;
        }
      }
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    out3[0] = nEd;
    out3[1] = nF;
    out3[2] = (uint32_t)sflag;
  }
}

// ---------------------------------------------------------------- node buckets
// The general path for meshes above SMALL_NE tets.  Equal keys share their lowest node (an
// edge's smaller node, a face's smallest node), so the occurrences are bucketed by that node
// with a counting sort (each workgroup aggregates its occurrences per node in an LDS hash
// table, then takes one global atomic per distinct node), and each bucket -- a few dozen
// occurrences in a mesh of bounded vertex degree -- is resolved in LDS by comparing every
// occurrence with the rest of its bucket:
//   edges: the first appearance is the least position among the bucket's occurrences with
//          the same other node;
//   faces: the first appearance is the least slot among the occurrences with the same edge
//          opposite the lowest node; the other one is the neighbour.
// The head flags then give per-tet counts, a scan gives the ids, and every output is written
// in position order (tet-major, coalesced) instead of in a sort order.  The order of the
// entries inside a bucket depends on atomics, but nothing read from a bucket does (minima,
// counts, ranks), so the outputs are deterministic.  A bucket above BK_BIG occurrences (a
// node in thousands of tets) sends the call to the radix-sort path below.
constexpr int BK_T = 256;            // threads per workgroup
constexpr int BK_LOGHS = 11;         // LDS hash slots per workgroup: 2048 > 6 BK_T occurrences
constexpr int BK_HS = 1 << BK_LOGHS;
constexpr uint32_t BK_EMPTY = 0xffffffffu;
constexpr int BK_BPW = 16;           // buckets per workgroup in the resolve pass
constexpr int BK_CAP = 2048;         // occurrences of those buckets staged in LDS
constexpr int BK_BIG = 8192;         // largest bucket resolved here
constexpr int BK_RHS = 2048;         // resolve: LDS hash slots of a workgroup's distinct keys
constexpr int BK_HCAP = 1536;        // resolve: entries of a workgroup resolved by hashing (load <= 3/4)
constexpr int BK_HE = BK_HCAP / BK_T;  // (entries per thread)
enum : int { DEV_BUCKET = 16 };      // internal: a bucket above BK_BIG occurrences
static_assert(BK_HS > 6 * BK_T, "every probe sequence finds a free slot");
static_assert((BK_BPW & (BK_BPW - 1)) == 0, "bucket search by halving");

__device__ __forceinline__ bool tet_ok(const int v[4], int64_t nC) {
  bool ok = true;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    ok &= v[i] >= 0 && v[i] < nC;
#pragma unroll
    for (int j = i + 1; j < 4; ++j) ok &= v[i] != v[j];
  }
  return ok;
}

// occurrence o of tet t: bucket node and entry.
//   edges (o = j):  entry = other node << 32 | position 6t+j
//   faces (o = k):  entry = opposite edge << 32 | (slot 4t+k) << 1 | parity of the tuple's node order
template <bool FACES>
__device__ __forceinline__ void bk_occ(int o, const int v[4], const int e[6], int64_t t, uint32_t& lo,
                                       uint64_t& ent) {
  if (!FACES) {
    const uint32_t a = (uint32_t)v[ev0(o)], b = (uint32_t)v[ev1(o)];
    lo = a < b ? a : b;
    ent = ((uint64_t)(a < b ? b : a) << 32) | (uint32_t)(6 * t + o);
  } else {
    const int na = v[fv(o, 0)], nb_ = v[fv(o, 1)], nc = v[fv(o, 2)];
    int oe;
    if (na < nb_ && na < nc) {
      lo = (uint32_t)na;
      oe = e[eidx(fv(o, 1), fv(o, 2))];
    } else if (nb_ < nc) {
      lo = (uint32_t)nb_;
      oe = e[eidx(fv(o, 0), fv(o, 2))];
    } else {
      lo = (uint32_t)nc;
      oe = e[eidx(fv(o, 0), fv(o, 1))];
    }
    const uint32_t par = (uint32_t)(((na > nb_) + (na > nc) + (nb_ > nc)) & 1);
    ent = ((uint64_t)(uint32_t)oe << 32) | ((uint32_t)(4 * t + o) << 1) | par;
  }
}

// LDS hash slot of node `key` (linear probing; the table never fills)
__device__ __forceinline__ int bk_slot(uint32_t* hk, uint32_t key) {
  uint32_t h = (key * 2654435761u) >> (32 - BK_LOGHS);
  for (;;) {
    const uint32_t prev = atomicCAS(&hk[h], BK_EMPTY, key);
    if (prev == BK_EMPTY || prev == key) return (int)h;
    h = (h + 1) & (BK_HS - 1);
  }
}

// bcnt[node] += occurrences in the node's bucket (tets with a bad node id are left out and
// flagged)
template <bool FACES>
__global__ __launch_bounds__(BK_T) void k_bk_count(int64_t nE, int64_t nC, const int32_t* __restrict__ tet,
                                                   uint32_t* __restrict__ bcnt, int* __restrict__ flags) {
  constexpr int N = FACES ? 4 : 6;
  __shared__ uint32_t hk[BK_HS], hc[BK_HS];
  for (int i = threadIdx.x; i < BK_HS; i += BK_T) {
    hk[i] = BK_EMPTY;
    hc[i] = 0;
  }
  __syncthreads();
  const int64_t t = (int64_t)blockIdx.x * BK_T + threadIdx.x;
  if (t < nE) {
    int v[4], e[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = tet[i * nE + t];
    if (tet_ok(v, nC)) {
#pragma unroll
      for (int o = 0; o < N; ++o) {
        uint32_t lo;
        uint64_t ent;
        bk_occ<FACES>(o, v, e, t, lo, ent);
        atomicAdd(&hc[bk_slot(hk, lo)], 1u);
      }
    } else {
      atomicOr(flags, DEV_BADNODE);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < BK_HS; i += BK_T)
    if (hk[i] != BK_EMPTY) atomicAdd(&bcnt[hk[i]], hc[i]);
}

// Entries into their buckets: bucket b spans [boff[b], boff[b+1]); each workgroup claims a
// run per node it holds by decrementing bcnt (which ends at zero again).  A tet with a bad
// node id has no entries; its positions are marked as their own heads so that the later
// passes stay in bounds (the call then fails with the flag set by the count pass).
template <bool FACES>
__global__ __launch_bounds__(BK_T) void k_bk_fill(int64_t nE, int64_t nC, const int32_t* __restrict__ tet,
                                                  const int32_t* __restrict__ t2e, const uint32_t* __restrict__ boff,
                                                  uint32_t* __restrict__ bcnt, uint64_t* __restrict__ bent,
                                                  int32_t* __restrict__ hp, int32_t* __restrict__ pp) {
  constexpr int N = FACES ? 4 : 6;
  __shared__ uint32_t hk[BK_HS], hc[BK_HS];
  for (int i = threadIdx.x; i < BK_HS; i += BK_T) {
    hk[i] = BK_EMPTY;
    hc[i] = 0;
  }
  __syncthreads();
  const int64_t t = (int64_t)blockIdx.x * BK_T + threadIdx.x;
  int slot[N];
  uint32_t rk[N];
  uint64_t ent[N];
  bool ok = false;
  if (t < nE) {
    int v[4], e[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = tet[i * nE + t];
    ok = tet_ok(v, nC);
    if (ok) {
      if (FACES) {
#pragma unroll
        for (int j = 0; j < 6; ++j) e[j] = t2e[j * nE + t];
      }
#pragma unroll
      for (int o = 0; o < N; ++o) {
        uint32_t lo;
        bk_occ<FACES>(o, v, e, t, lo, ent[o]);
        slot[o] = bk_slot(hk, lo);
        rk[o] = atomicAdd(&hc[slot[o]], 1u);
      }
    } else {
#pragma unroll
      for (int o = 0; o < N; ++o) {
        hp[N * t + o] = (int32_t)(N * t + o);
        if (FACES) pp[N * t + o] = -1;
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < BK_HS; i += BK_T) {
    const uint32_t key = hk[i];
    if (key != BK_EMPTY) {
      const uint32_t c = hc[i];
      const uint32_t old = atomicSub(&bcnt[key], c);
      hc[i] = boff[key] + old - c;
    }
  }
  __syncthreads();
  if (ok) {
#pragma unroll
    for (int o = 0; o < N; ++o) bent[hc[slot[o]] + rk[o]] = ent[o];
  }
}

// One entry against its bucket B[0, m) (LDS or global), written at global bucket start g.
//   edges: hp[pos] = least position with the same other node; SORTED also writes the
//          bucket in ascending (other node, position) order to bsort and the head flags in
//          that order to dfl (Nodes2Edge).
//   faces: hp[slot] = least slot with the same opposite edge, pp[slot] = the other slot or
//          -1; three occurrences, or two with the same parity, are flagged.
template <bool FACES, bool SORTED>
__device__ __forceinline__ void bk_resolve_one(uint64_t mine, const uint64_t* B, int m, int64_t g,
                                               int32_t* __restrict__ hp, int32_t* __restrict__ pp,
                                               uint64_t* __restrict__ bsort, uint32_t* __restrict__ dfl,
                                               int* __restrict__ flags) {
  const uint32_t key = (uint32_t)(mine >> 32), w = (uint32_t)mine;
  if (!FACES) {
    uint32_t hmin = w, rank = 0;
#pragma unroll 4
    for (int j = 0; j < m; ++j) {
      const uint64_t o = B[j];
      if ((uint32_t)(o >> 32) == key) hmin = min(hmin, (uint32_t)o);
      if (SORTED) rank += o < mine ? 1u : 0u;
    }
    hp[w] = (int32_t)hmin;
    if (SORTED) {
      bsort[g + rank] = mine;
      dfl[g + rank] = hmin == w ? 1u : 0u;
    }
  } else {
    uint32_t hmin = w >> 1, cnt = 0, pw = BK_EMPTY;
#pragma unroll 4
    for (int j = 0; j < m; ++j) {
      const uint64_t o = B[j];
      if ((uint32_t)(o >> 32) == key) {
        const uint32_t ow = (uint32_t)o;
        ++cnt;
        hmin = min(hmin, ow >> 1);
        if (ow != w) pw = ow;
      }
    }
    hp[w >> 1] = (int32_t)hmin;
    pp[w >> 1] = cnt == 2 ? (int32_t)(pw >> 1) : -1;
    if (cnt > 2 || (cnt == 2 && (pw & 1u) == (w & 1u))) atomicOr(flags, DEV_ORIENT);
  }
}

// Buckets [b0, b0 + BK_BPW) per workgroup.  Without the sorted output, when their entries fit
// BK_HCAP: every entry goes into an LDS hash table keyed by (bucket, key part) whose slots keep
// the least position (edges) or the least slot and one 64-bit sum of (slot, 1 << 32, odd
// parity << 48) (faces: the other slot of a pair is the sum less this one) -- one insertion per
// entry instead of a scan of its bucket.  Otherwise the
// entries are staged in LDS when they fit BK_CAP (each scans its bucket), else one bucket at a
// time from global memory; a bucket above BK_BIG is flagged DEV_BUCKET and its entries are
// given in-bounds placeholders (own head, no partner, no Nodes2Edge entry).  Every path
// writes the same values.
template <bool FACES, bool SORTED>
__global__ __launch_bounds__(BK_T) void k_bk_resolve(int64_t nB, const uint32_t* __restrict__ boff,
                                                     const uint64_t* __restrict__ bent, int32_t* __restrict__ hp,
                                                     int32_t* __restrict__ pp, uint64_t* __restrict__ bsort,
                                                     uint32_t* __restrict__ dfl, int* __restrict__ flags) {
  constexpr int HS = SORTED ? 1 : BK_RHS, HF = FACES && !SORTED ? BK_RHS : 1;
  __shared__ uint64_t E[BK_CAP];  // staged entries, or the hash table's keys
  __shared__ uint32_t hmin[HS];
  __shared__ uint64_t hsc[HF];
  __shared__ uint32_t bs[BK_BPW + 1];
  const int64_t b0 = (int64_t)blockIdx.x * BK_BPW;
  const int nb = (int)min((int64_t)BK_BPW, nB - b0);
  const uint32_t s0 = boff[b0], total = boff[b0 + nb] - s0;
  static_assert(BK_RHS <= BK_CAP && BK_HCAP < BK_RHS && BK_HCAP % BK_T == 0, "hash table in the staging array");
  if (!SORTED && total <= (uint32_t)BK_HCAP) {
    constexpr uint64_t EMPTY64 = ~0ull;
    for (int i = threadIdx.x; i < BK_RHS; i += BK_T) {
      E[i] = EMPTY64;
      hmin[i] = 0xffffffffu;
      if (FACES) hsc[i] = 0ull;
    }
    for (int i = threadIdx.x; i <= nb; i += BK_T) bs[i] = boff[b0 + i] - s0;
    __syncthreads();
    int slot[BK_HE];
    uint32_t wv[BK_HE];
#pragma unroll
    for (int u = 0; u < BK_HE; ++u) {
      const uint32_t e = threadIdx.x + u * BK_T;
      slot[u] = -1;
      wv[u] = 0u;
      if (e < total) {
        const uint64_t x = bent[s0 + e];
        int k = 0;
#pragma unroll
        for (int step = BK_BPW / 2; step > 0; step >>= 1)
          if (k + step < nb && bs[k + step] <= e) k += step;
        const uint64_t key = ((uint64_t)k << 32) | (x >> 32);
        uint32_t h = (uint32_t)((key * 0x9E3779B97F4A7C15ull) >> 53) & (BK_RHS - 1);  // table never full
        for (;;) {
          const uint64_t prev = atomicCAS((unsigned long long*)&E[h], EMPTY64, key);
          if (prev == EMPTY64 || prev == key) break;
          h = (h + 1) & (BK_RHS - 1);
        }
        slot[u] = (int)h;
        wv[u] = (uint32_t)x;
        if (!FACES) {
          atomicMin(&hmin[h], wv[u]);
        } else {
          const uint32_t q = wv[u] >> 1;
          atomicMin(&hmin[h], q);
          const uint64_t inc = (uint64_t)q | (1ull << 32) | ((uint64_t)(wv[u] & 1u) << 48);
          atomicAdd((unsigned long long*)&hsc[h], (unsigned long long)inc);
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < BK_HE; ++u) {
      if (slot[u] < 0) continue;
      const int h = slot[u];
      if (!FACES) {
        hp[wv[u]] = (int32_t)hmin[h];
      } else {
        const uint64_t c = hsc[h];
        const uint32_t q = wv[u] >> 1, mn = hmin[h], n = (uint32_t)(c >> 32) & 0xffffu;
        hp[q] = (int32_t)mn;
        pp[q] = n == 2 ? (int32_t)((uint32_t)c - q) : -1;
        if (n > 2 || (n == 2 && (c >> 48) != 1u)) atomicOr(flags, DEV_ORIENT);
      }
    }
  } else if (total <= (uint32_t)BK_CAP) {
    for (int i = threadIdx.x; i <= nb; i += BK_T) bs[i] = boff[b0 + i] - s0;
    for (uint32_t e = threadIdx.x; e < total; e += BK_T) E[e] = bent[s0 + e];
    __syncthreads();
    for (uint32_t e = threadIdx.x; e < total; e += BK_T) {
      // the entry's bucket: the last k with bs[k] <= e (binary search over the nb + 1 starts)
      int k = 0;
#pragma unroll
      for (int step = BK_BPW / 2; step > 0; step >>= 1)
        if (k + step < nb && bs[k + step] <= e) k += step;
      const uint32_t j0 = bs[k];
      bk_resolve_one<FACES, SORTED>(E[e], E + j0, (int)(bs[k + 1] - j0), (int64_t)s0 + j0, hp, pp, bsort, dfl,
                                    flags);
    }
  } else {
    for (int k = 0; k < nb; ++k) {
      const uint32_t j0 = boff[b0 + k];
      const int m = (int)(boff[b0 + k + 1] - j0);
      if (m > BK_BIG) {
        if (threadIdx.x == 0) atomicOr(flags, DEV_BUCKET);
        for (int e = threadIdx.x; e < m; e += BK_T) {
          const uint64_t mine = bent[j0 + e];
          const uint32_t w = (uint32_t)mine;
          if (!FACES) {
            hp[w] = (int32_t)w;
            if (SORTED) {
              bsort[j0 + e] = mine;
              dfl[j0 + e] = 0u;
            }
          } else {
            hp[w >> 1] = (int32_t)(w >> 1);
            pp[w >> 1] = -1;
          }
        }
        continue;
      }
      for (int e = threadIdx.x; e < m; e += BK_T)
        bk_resolve_one<FACES, SORTED>(bent[j0 + e], bent + j0, m, (int64_t)j0, hp, pp, bsort, dfl, flags);
    }
  }
}

// cnt[t] = first appearances among the N positions of tet t (cnt[nE] = 0)
template <int N>
__global__ __launch_bounds__(BK_T) void k_bk_heads(int64_t nE, const int32_t* __restrict__ hp,
                                                   uint32_t* __restrict__ cnt) {
  const int64_t t = (int64_t)blockIdx.x * BK_T + threadIdx.x;
  if (t > nE) return;
  uint32_t c = 0;
  if (t < nE) {
#pragma unroll
    for (int o = 0; o < N; ++o) c += hp[N * t + o] == (int32_t)(N * t + o) ? 1u : 0u;
  }
  cnt[t] = c;
}

// id of the first appearance at position h = N th + oh: prefix of th + heads of th before oh
// (tet th's N head records read as vectors: 3 x 8 bytes for edges, 16 bytes for faces)
template <int N>
__device__ __forceinline__ int32_t bk_head_id(int32_t h, const int32_t* __restrict__ hp,
                                              const uint32_t* __restrict__ pre) {
  static_assert(N == 4 || N == 6, "edges or faces");
  const int64_t th = h / N;
  const int oh = (int)(h - N * th);
  uint32_t id = pre[th];
  int w[N];
  if constexpr (N == 4) {
    const int4 x = reinterpret_cast<const int4*>(hp)[th];
    w[0] = x.x;
    w[1] = x.y;
    w[2] = x.z;
    w[3] = x.w;
  } else {
    const int2* p = reinterpret_cast<const int2*>(hp + 6 * th);  // 24 th bytes: 8-byte aligned
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const int2 x = p[i];
      w[2 * i] = x.x;
      w[2 * i + 1] = x.y;
    }
  }
#pragma unroll
  for (int i = 0; i < N - 1; ++i) id += (i < oh && w[i] == (int32_t)(N * th + i)) ? 1u : 0u;
  return (int32_t)id;
}

// edge outputs in tet order; pre = exclusive scan of k_bk_heads<6> (nE + 1 entries), *nEdp
// its total.  The edges first seen in a workgroup's tets have the consecutive ids
// [pre[t0], pre[t0 + BK_T]): their node pairs and first tets are staged in LDS and stored as
// contiguous ranges.
__global__ __launch_bounds__(BK_T) void k_bk_edge_assign(int64_t nE, const int32_t* __restrict__ tet,
                                                         const int32_t* __restrict__ hp,
                                                         const uint32_t* __restrict__ pre,
                                                         const uint32_t* __restrict__ nEdp,
                                                         int32_t* __restrict__ tet2edge, int32_t* __restrict__ edges,
                                                         int32_t* __restrict__ eft,
                                                         int32_t* __restrict__ tet_edge_prefix) {
  __shared__ int32_t slo[6 * BK_T], shi[6 * BK_T], sft[6 * BK_T];
  const int64_t t0 = (int64_t)blockIdx.x * BK_T, t = t0 + threadIdx.x;
  const int nb = nE - t0 < BK_T ? (int)(nE - t0) : BK_T;
  const int64_t nEd = *nEdp;
  const uint32_t base = pre[t0], nh = pre[t0 + nb] - base;  // this workgroup's first-seen edges
  if (t < nE) {
    int v[4], h[6];
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = tet[i * nE + t];
    const int2* h2 = reinterpret_cast<const int2*>(hp + 6 * t);  // 24 t bytes: 8-byte aligned
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const int2 x = h2[i];
      h[2 * i] = x.x;
      h[2 * i + 1] = x.y;
    }
    const uint32_t pt = pre[t];
    uint32_t r = 0;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      const int32_t p = (int32_t)(6 * t + j);
      int32_t id;
      if (h[j] == p) {
        id = (int32_t)(pt + r++);
        const int a = v[ev0(j)], b = v[ev1(j)];
        const uint32_t l = (uint32_t)id - base;  // < 6 BK_T: heads of this workgroup's tets
        if (l < 6u * BK_T) {
          slo[l] = a < b ? a : b;
          shi[l] = a < b ? b : a;
          sft[l] = (int32_t)t;
        }
      } else {
        id = bk_head_id<6>(h[j], hp, pre);
      }
      tet2edge[j * nE + t] = id;
    }
    tet_edge_prefix[t] = (int32_t)pt;
  }
  __syncthreads();
  for (uint32_t l = threadIdx.x; l < nh && l < 6u * BK_T; l += BK_T) {
    edges[base + l] = slo[l];
    edges[nEd + base + l] = shi[l];
    eft[base + l] = sft[l];
  }
}

// face outputs in tet order; pre = exclusive scan of k_bk_heads<4> (nE + 1 entries), *nFp its
// total.  The faces owned by a workgroup's tets have the consecutive ids
// [pre[t0], pre[t0 + BK_T]): their rows of faces and face2tet are staged in LDS and stored as
// contiguous ranges.
__global__ __launch_bounds__(BK_T) void k_bk_face_assign(int64_t nE, const int32_t* __restrict__ tet,
                                                         const int32_t* __restrict__ hp,
                                                         const int32_t* __restrict__ pp,
                                                         const uint32_t* __restrict__ pre,
                                                         const uint32_t* __restrict__ nFp,
                                                         int32_t* __restrict__ faces, int32_t* __restrict__ tet2face,
                                                         int8_t* __restrict__ sigma, int32_t* __restrict__ face2tet,
                                                         int32_t* __restrict__ nbr) {
  __shared__ int32_t sfa[3][4 * BK_T], sft[2][4 * BK_T];
  const int64_t t0 = (int64_t)blockIdx.x * BK_T, t = t0 + threadIdx.x;
  const int nb = nE - t0 < BK_T ? (int)(nE - t0) : BK_T;
  const int64_t nF = *nFp;
  const uint32_t base = pre[t0], nh = pre[t0 + nb] - base;  // this workgroup's owned faces
  if (t < nE) {
    int v[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = tet[i * nE + t];
    const int4 h4 = reinterpret_cast<const int4*>(hp)[t], p4 = reinterpret_cast<const int4*>(pp)[t];
    const int h[4] = {h4.x, h4.y, h4.z, h4.w}, pr[4] = {p4.x, p4.y, p4.z, p4.w};
    const uint32_t pt = pre[t];
    uint32_t r = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int32_t q = (int32_t)(4 * t + k);
      if (h[k] == q) {
        const int32_t id = (int32_t)(pt + r++);
        const uint32_t l = (uint32_t)id - base;  // < 4 BK_T: faces owned by this workgroup's tets
        if (l < 4u * BK_T) {
#pragma unroll
          for (int m = 0; m < 3; ++m) sfa[m][l] = v[fv(k, m)];
          sft[0][l] = q;
          sft[1][l] = pr[k];
        }
        tet2face[k * nE + t] = id;
        sigma[k * nE + t] = 1;
        if (nbr) nbr[k * nE + t] = pr[k] >= 0 ? (pr[k] >> 2) : -1;
      } else {
        tet2face[k * nE + t] = bk_head_id<4>(h[k], hp, pre);
        sigma[k * nE + t] = -1;
        if (nbr) nbr[k * nE + t] = h[k] >> 2;
      }
    }
  }
  __syncthreads();
  for (uint32_t l = threadIdx.x; l < nh && l < 4u * BK_T; l += BK_T) {
#pragma unroll
    for (int m = 0; m < 3; ++m) faces[m * nF + base + l] = sfa[m][l];
    face2tet[base + l] = sft[0][l];
    face2tet[nF + base + l] = sft[1][l];
  }
}

// Nodes2Edge from the sorted buckets: u = exclusive scan of the head flags in sorted order
// (the rank of the node pair among all distinct pairs, i.e. the CSR slot); *nup its total.
__global__ __launch_bounds__(BK_T) void k_bk_n2e_fill(int64_t n, int64_t nE, const uint64_t* __restrict__ bsort,
                                                      const uint32_t* __restrict__ u,
                                                      const uint32_t* __restrict__ nup,
                                                      const int32_t* __restrict__ tet2edge, int32_t* __restrict__ col,
                                                      int32_t* __restrict__ eid) {
  const int64_t s = (int64_t)blockIdx.x * BK_T + threadIdx.x;
  if (s >= n) return;
  const uint32_t us = u[s], un = s + 1 < n ? u[s + 1] : *nup;
  if (un == us) return;
  const uint64_t ent = bsort[s];
  const uint32_t pos = (uint32_t)ent;
  const int64_t t = pos / 6;
  const int j = (int)(pos - 6 * t);
  col[us] = (int32_t)(ent >> 32);
  eid[us] = tet2edge[j * nE + t];
}

// row pointers: the CSR slot of each node's first entry (its bucket start), total at nC
__global__ __launch_bounds__(BK_T) void k_bk_n2e_rows(int64_t nC, int64_t n, const uint32_t* __restrict__ boff,
                                                      const uint32_t* __restrict__ u,
                                                      const uint32_t* __restrict__ nup,
                                                      int32_t* __restrict__ rowptr) {
  const int64_t b = (int64_t)blockIdx.x * BK_T + threadIdx.x;
  if (b > nC) return;
  const uint32_t s = boff[b];
  rowptr[b] = (int32_t)(s < n ? u[s] : *nup);
}

// ---------------------------------------------------------------- workspace layouts
struct ConnWS {  // radix-sort path
  uint64_t *kA, *kB;
  int32_t *vA, *vB;
  uint8_t* first;
  uint32_t* cnt;   // nE + 1
  uint32_t* flag;  // head flags / ranks in sorted order (Nodes2Edge only)
  uint32_t* rowcnt;
  int* dflags;
  uint32_t* total;
  size_t sub;  // offset where the sort/scan scratch starts
};

static void conn_layout(Arena& a, int64_t nC, int64_t nE, int32_t flags, ConnWS& w) {
  int64_t n = 6 * nE;
  w.kA = a.take<uint64_t>(n);
  w.kB = a.take<uint64_t>(n);
  w.vA = a.take<int32_t>(n);
  w.vB = a.take<int32_t>(n);
  w.first = a.take<uint8_t>(n);
  w.cnt = a.take<uint32_t>(nE + 1);
  w.flag = (flags & PHFEM_CONNECT_NODES2EDGE) ? a.take<uint32_t>(n) : nullptr;  // head flags, then ranks
  w.rowcnt = (flags & PHFEM_CONNECT_NODES2EDGE) ? a.take<uint32_t>(nC + 1) : nullptr;
  w.dflags = a.take<int>(16);
  w.total = a.take<uint32_t>(16);
  w.sub = a.size();
}

static size_t radix_workspace(int64_t nC, int64_t nE, int32_t flags) {
  Arena a;
  ConnWS w;
  conn_layout(a, nC, nE, flags, w);
  size_t extra = sort_workspace(6 * nE);
  extra = std::max(extra, scan_workspace(6 * nE + 1));
  extra = std::max(extra, scan_workspace(nC + 1));
  return w.sub + extra;
}

struct BkWS {  // node-bucket path
  uint32_t *bcnt, *boff;  // nC + 1 each
  uint64_t* bent;         // bucket entries, 6 nE
  uint64_t* bsort;        // sorted buckets (Nodes2Edge only)
  uint32_t* dfl;          // head flags in sorted order, then CSR slots (Nodes2Edge only)
  int32_t *hp, *pp;       // head position per position (6 nE); partner slot per face slot (4 nE)
  uint32_t* cnt;          // nE + 1
  int* dflags;
  uint32_t* total;        // [0] nEd, [1] nF, [2] distinct node pairs
  size_t sub;
};

static void bk_layout(Arena& a, int64_t nC, int64_t nE, int32_t flags, BkWS& w) {
  const int64_t n = 6 * nE;
  const bool n2e = flags & PHFEM_CONNECT_NODES2EDGE, faces = flags & PHFEM_CONNECT_FACES;
  w.bcnt = a.take<uint32_t>(nC + 1);
  w.boff = a.take<uint32_t>(nC + 1);
  w.bent = a.take<uint64_t>(n);
  w.bsort = n2e ? a.take<uint64_t>(n) : nullptr;
  w.dfl = n2e ? a.take<uint32_t>(n) : nullptr;
  w.hp = a.take<int32_t>(n);
  w.pp = faces ? a.take<int32_t>(4 * nE) : nullptr;
  w.cnt = a.take<uint32_t>(nE + 1);
  w.dflags = a.take<int>(16);
  w.total = a.take<uint32_t>(16);
  w.sub = a.size();
}

static size_t bucket_workspace(int64_t nC, int64_t nE, int32_t flags) {
  Arena a;
  BkWS w;
  bk_layout(a, nC, nE, flags, w);
  size_t extra = scan_workspace(nC + 1);
  extra = std::max(extra, scan_workspace(nE + 1));
  if (flags & PHFEM_CONNECT_NODES2EDGE) extra = std::max(extra, scan_workspace(6 * nE));
  return w.sub + extra;
}

// counts[0..2] from the device totals and flags; one readback.  *redo: a bucket was too large
// for the bucket path (nothing else went wrong), so the caller runs the radix path instead.
static int bk_finish(const BkWS& w, int64_t nE, bool faces, int64_t* counts, bool* redo, hipStream_t s) {
  uint32_t tot[2] = {0, 0};
  int hf = 0;
  PH_HIP(hipMemcpyAsync(tot, w.total, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  PH_HIP(hipMemcpyAsync(&hf, w.dflags, sizeof(int), hipMemcpyDeviceToHost, s));
  PH_HIP(hipStreamSynchronize(s));
  if (hf & ~DEV_BUCKET) return dev_flags_to_status(hf & ~DEV_BUCKET);
  if (hf & DEV_BUCKET) {
    *redo = true;
    return PHFEM_OK;
  }
  counts[0] = tot[0];
  counts[1] = faces ? tot[1] : 0;
  counts[2] = faces ? 2 * (int64_t)tot[1] - 4 * nE : 0;  // 4 nE = 2 nI + nB and nF = nI + nB
  return PHFEM_OK;
}

static int connect_bucket(int64_t nC, int64_t nE, const int32_t* tetra, int32_t flags, Arena& a, int32_t* edges,
                          int32_t* tet2edge, int32_t* edge_first_tet, int32_t* tet_edge_prefix, int32_t* n2e_rowptr,
                          int32_t* n2e_col, int32_t* n2e_edge, int32_t* faces, int32_t* tet2face, int8_t* sigma,
                          int32_t* face2tet, int32_t* nbr, int64_t* counts, bool* redo, hipStream_t s) {
  const bool want_faces = flags & PHFEM_CONNECT_FACES, want_n2e = flags & PHFEM_CONNECT_NODES2EDGE;
  BkWS w;
  bk_layout(a, nC, nE, flags, w);
  const size_t sub = w.sub;
  const int64_t n6 = 6 * nE, n4 = 4 * nE;
  const unsigned gt = grid_for(nE, BK_T), gb = grid_for(nC, BK_BPW);
  PH_HIP(hipMemsetAsync(w.dflags, 0, sizeof(int), s));
  PH_HIP(hipMemsetAsync(w.bcnt, 0, sizeof(uint32_t) * (nC + 1), s));

  // ---- edges, bucketed by their smaller node
  PH_LAUNCH_B("bk_count", 16.0 * nE, k_bk_count<false>, gt, BK_T, 0, s, nE, nC, tetra, w.bcnt, w.dflags);
  if (want_n2e) {  // Nodes2Edge writes rows by node id: a bad id stops the call here
    int hf = 0;
    PH_HIP(hipMemcpyAsync(&hf, w.dflags, sizeof(int), hipMemcpyDeviceToHost, s));
    PH_HIP(hipStreamSynchronize(s));
    if (hf) return dev_flags_to_status(hf);
  }
  a.off = sub;
  int rc = scan_exclusive(w.bcnt, w.boff, nC + 1, nullptr, a, s);
  if (rc) return rc;
  PH_LAUNCH_B("bk_fill", 16.0 * nE + 8.0 * n6, k_bk_fill<false>, gt, BK_T, 0, s, nE, nC, tetra, nullptr,
              (const uint32_t*)w.boff, w.bcnt, w.bent, w.hp, nullptr);
  if (want_n2e)
    PH_LAUNCH_B("bk_resolve", 24.0 * n6, (k_bk_resolve<false, true>), gb, BK_T, 0, s, nC, (const uint32_t*)w.boff,
                (const uint64_t*)w.bent, w.hp, nullptr, w.bsort, w.dfl, w.dflags);
  else
    PH_LAUNCH_B("bk_resolve", 12.0 * n6, (k_bk_resolve<false, false>), gb, BK_T, 0, s, nC, (const uint32_t*)w.boff,
                (const uint64_t*)w.bent, w.hp, nullptr, nullptr, nullptr, w.dflags);
  PH_LAUNCH_B("bk_heads", 4.0 * n6 + 4.0 * nE, k_bk_heads<6>, grid_for(nE + 1, BK_T), BK_T, 0, s, nE,
              (const int32_t*)w.hp, w.cnt);
  a.off = sub;
  rc = scan_exclusive(w.cnt, w.cnt, nE + 1, w.total, a, s);
  if (rc) return rc;
  // unique edges ~ 1.2 nE on a tet mesh: 12 bytes each (node pair, first tet)
  PH_LAUNCH_B("edge_assign", 16.0 * nE + 4.0 * n6 + 4.0 * nE + 4.0 * n6 + 4.0 * nE + 12.0 * 1.2 * nE,
              k_bk_edge_assign, gt, BK_T, 0, s, nE, tetra, (const int32_t*)w.hp, (const uint32_t*)w.cnt,
              (const uint32_t*)w.total, tet2edge, edges, edge_first_tet, tet_edge_prefix);
  if (want_n2e) {
    a.off = sub;
    rc = scan_exclusive(w.dfl, w.dfl, n6, w.total + 2, a, s);  // in place: head flag -> CSR slot
    if (rc) return rc;
    PH_LAUNCH("n2e_fill", k_bk_n2e_fill, grid_for(n6, BK_T), BK_T, 0, s, n6, nE, (const uint64_t*)w.bsort,
              (const uint32_t*)w.dfl, (const uint32_t*)(w.total + 2), (const int32_t*)tet2edge, n2e_col, n2e_edge);
    PH_LAUNCH("n2e_rows", k_bk_n2e_rows, grid_for(nC + 1, BK_T), BK_T, 0, s, nC, n6, (const uint32_t*)w.boff,
              (const uint32_t*)w.dfl, (const uint32_t*)(w.total + 2), n2e_rowptr);
  }
  if (!want_faces) return bk_finish(w, nE, false, counts, redo, s);

  // ---- faces, bucketed by their smallest node (bcnt is back at zero after the fill)
  PH_LAUNCH_B("bk_count", 16.0 * nE, k_bk_count<true>, gt, BK_T, 0, s, nE, nC, tetra, w.bcnt, w.dflags);
  a.off = sub;
  rc = scan_exclusive(w.bcnt, w.boff, nC + 1, nullptr, a, s);
  if (rc) return rc;
  PH_LAUNCH_B("bk_fill", 40.0 * nE + 8.0 * n4, k_bk_fill<true>, gt, BK_T, 0, s, nE, nC, tetra,
              (const int32_t*)tet2edge, (const uint32_t*)w.boff, w.bcnt, w.bent, w.hp, w.pp);
  PH_LAUNCH_B("bk_resolve", 16.0 * n4, (k_bk_resolve<true, false>), gb, BK_T, 0, s, nC, (const uint32_t*)w.boff,
              (const uint64_t*)w.bent, w.hp, w.pp, nullptr, nullptr, w.dflags);
  PH_LAUNCH_B("bk_heads", 4.0 * n4 + 4.0 * nE, k_bk_heads<4>, grid_for(nE + 1, BK_T), BK_T, 0, s, nE,
              (const int32_t*)w.hp, w.cnt);
  a.off = sub;
  rc = scan_exclusive(w.cnt, w.cnt, nE + 1, w.total + 1, a, s);
  if (rc) return rc;
  // unique faces ~ 2 nE: 20 bytes each (node triple, two slots)
  PH_LAUNCH_B("face_assign", 16.0 * nE + 8.0 * n4 + 4.0 * nE + 9.0 * n4 + 20.0 * 2 * nE, k_bk_face_assign, gt, BK_T,
              0, s, nE, tetra, (const int32_t*)w.hp, (const int32_t*)w.pp, (const uint32_t*)w.cnt,
              (const uint32_t*)(w.total + 1), faces, tet2face, sigma, face2tet, nbr);
  return bk_finish(w, nE, true, counts, redo, s);
}

// The radix-sort path: stable LSD sort of the occurrence keys (node pair; lowest node and
// opposite edge), segment heads, per-tet counts and a scan give the same numbering.
static int connect_radix(int64_t nC, int64_t nE, const int32_t* tetra, int32_t flags, Arena& a, int32_t* edges,
                         int32_t* tet2edge, int32_t* edge_first_tet, int32_t* tet_edge_prefix, int32_t* n2e_rowptr,
                         int32_t* n2e_col, int32_t* n2e_edge, int32_t* faces, int32_t* tet2face, int8_t* sigma,
                         int32_t* face2tet, int32_t* nbr, int64_t* counts, hipStream_t s) {
  const bool want_faces = flags & PHFEM_CONNECT_FACES, want_n2e = flags & PHFEM_CONNECT_NODES2EDGE;
  ConnWS w;
  conn_layout(a, nC, nE, flags, w);
  const size_t sub = w.sub;
  const int64_t n6 = 6 * nE, n4 = 4 * nE;
  const int nb = bits_for(nC);
  PH_HIP(hipMemsetAsync(w.dflags, 0, sizeof(int), s));

  // ---- edges.  The node-id check is read back with the last count: until then a bad id only
  // makes key values wrong, never an address (Nodes2Edge, which indexes rows by node id, is
  // the exception and reads it at once).
  PH_LAUNCH_B("edge_keys", 64.0 * nE, k_edge_keys, grid_for(nE, CT), CT, 0, s, nE, nC, tetra, nb, w.kA, w.dflags);
  int hflags = 0;
  if (want_n2e) {
    PH_HIP(hipMemcpyAsync(&hflags, w.dflags, sizeof(int), hipMemcpyDeviceToHost, s));
    PH_HIP(hipStreamSynchronize(s));
    if (hflags) return dev_flags_to_status(hflags);
  }

  uint64_t* sk;
  int32_t* sv;
  a.off = sub;
  int rc = radix_sort(w.kA, w.vA, w.kB, w.vB, nullptr, n6, 2 * nb, &sk, &sv, a, s);
  if (rc) return rc;
  PH_LAUNCH_B("mark_heads", 13.0 * n6, k_mark_heads, grid_for(n6, CT), CT, 0, s, n6, (const uint64_t*)sk,
              (const int32_t*)sv,
            0xffffffffu, w.first);
  PH_LAUNCH_B("count_heads", 10.0 * nE, k_count_heads<6>, grid_for(nE + 1, CT), CT, 0, s, nE, (const uint8_t*)w.first,
              w.cnt);
  a.off = sub;
  rc = scan_exclusive(w.cnt, w.cnt, nE + 1, w.total, a, s);
  if (rc) return rc;
  // The edge count sizes the face keys' edge field.  A small mesh takes a bound instead
  // (min(6 nE, nC (nC - 1) / 2) distinct node pairs) and reads the count back with the face
  // count at the end, one host round trip fewer; a large mesh reads it here, since a loose
  // bound could add a radix pass there.
  const bool small = nE <= (int64_t(1) << 16);
  int64_t nEd = -1;
  if (!small) {
    uint32_t nEd32 = 0;
    PH_HIP(hipMemcpyAsync(&nEd32, w.total, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    PH_HIP(hipStreamSynchronize(s));
    nEd = nEd32;
  }
  PH_HIP(hipMemcpyAsync(tet_edge_prefix, w.cnt, sizeof(int32_t) * nE, hipMemcpyDeviceToDevice, s));
  PH_LAUNCH_B("edge_assign", 17.0 * n6 + 12.0 * (nEd >= 0 ? nEd : 1.2 * nE) + 4.0 * nE, k_edge_assign,
              grid_for(n6, CT), CT, 0, s, n6, nE, (const uint32_t*)w.total, nb, (const uint64_t*)sk, (const int32_t*)sv,
              (const uint8_t*)w.first, (const uint32_t*)w.cnt, tet2edge, edges, edge_first_tet, w.flag);
  if (want_n2e) {
    a.off = sub;
    rc = scan_exclusive(w.flag, w.flag, n6, nullptr, a, s);  // in place: head flag -> unique rank
    if (rc) return rc;
    PH_HIP(hipMemsetAsync(w.rowcnt, 0, sizeof(uint32_t) * (nC + 1), s));
    PH_LAUNCH("n2e_fill", k_n2e_fill, grid_for(n6, CT), CT, 0, s, n6, nb, (const uint64_t*)sk, (const int32_t*)sv,
              (const uint32_t*)w.flag, nE, (const int32_t*)tet2edge, n2e_col, n2e_edge, w.rowcnt);
    a.off = sub;
    rc = scan_exclusive(w.rowcnt, (uint32_t*)n2e_rowptr, nC + 1, nullptr, a, s);
    if (rc) return rc;
  }
  if (!want_faces) {
    uint32_t nEd32 = 0;
    PH_HIP(hipMemcpyAsync(&nEd32, w.total, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    PH_HIP(hipMemcpyAsync(&hflags, w.dflags, sizeof(int), hipMemcpyDeviceToHost, s));
    PH_HIP(hipStreamSynchronize(s));
    if (hflags) return dev_flags_to_status(hflags);
    counts[0] = nEd32;
    counts[1] = 0;
    counts[2] = 0;
    return PHFEM_OK;
  }

  // ---- faces: key = (min node, opposite edge) of every local face
  const int eb = bits_for(nEd >= 0 ? nEd : std::min<int64_t>(n6, nC * (nC - 1) / 2));
  PH_LAUNCH_B("face_keys", 88.0 * nE, k_face_keys, grid_for(nE, CT), CT, 0, s, nE, tetra, (const int32_t*)tet2edge, eb,
              w.kA,
            w.vA);
  a.off = sub;
  rc = radix_sort(w.kA, w.vA, w.kB, w.vB, w.vA, n4, nb + eb, &sk, &sv, a, s);
  if (rc) return rc;
  PH_LAUNCH_B("mark_heads", 13.0 * n4, k_mark_heads, grid_for(n4, CT), CT, 0, s, n4, (const uint64_t*)sk,
              (const int32_t*)sv,
            SLOT_MASK, w.first);
  PH_LAUNCH_B("count_heads", 8.0 * nE, k_count_heads<4>, grid_for(nE + 1, CT), CT, 0, s, nE, (const uint8_t*)w.first,
              w.cnt);
  a.off = sub;
  rc = scan_exclusive(w.cnt, w.cnt, nE + 1, w.total + 1, a, s);
  if (rc) return rc;
  PH_LAUNCH_B("face_assign", 22.0 * n4 + 20.0 * nE + 20.0 * 2 * nE, k_face_assign, grid_for(n4, CT), CT, 0, s, n4, nE,
              (const uint32_t*)(w.total + 1), (const uint64_t*)sk, (const int32_t*)sv, (const uint8_t*)w.first,
              (const uint32_t*)w.cnt, tetra, faces, tet2face, sigma, face2tet, nbr, w.dflags);
  // one readback for the counts and every device-side check
  uint32_t tot[2] = {0, 0};
  PH_HIP(hipMemcpyAsync(tot, w.total, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  PH_HIP(hipMemcpyAsync(&hflags, w.dflags, sizeof(int), hipMemcpyDeviceToHost, s));
  PH_HIP(hipStreamSynchronize(s));
  if (hflags) return dev_flags_to_status(hflags);
  const int64_t nF = tot[1];
  counts[0] = tot[0];
  counts[1] = nF;
  counts[2] = 2 * nF - 4 * nE;  // 4 nE = 2 nI + nB and nF = nI + nB
  return PHFEM_OK;
}

}  // namespace ph

using namespace ph;

extern "C" size_t phfem_connect_workspace(int64_t nC, int64_t nE, int32_t flags) {
  if (nC <= 0 || nE <= 0) return 0;
  return std::max(radix_workspace(nC, nE, flags), bucket_workspace(nC, nE, flags));
}

extern "C" int phfem_connect(int64_t nC, int64_t nE, const int32_t* tetra, int32_t flags, void* work,
                             size_t work_bytes, int32_t* edges, int32_t* tet2edge, int32_t* edge_first_tet,
                             int32_t* tet_edge_prefix, int32_t* n2e_rowptr, int32_t* n2e_col, int32_t* n2e_edge,
                             int32_t* faces, int32_t* tet2face, int8_t* sigma, int32_t* face2tet, int32_t* nbr,
                             int64_t* counts, phfem_stream_t stream_) {
  clear_error();
  hipStream_t s = (hipStream_t)stream_;
  if (nC <= 0 || nE <= 0) return err(PHFEM_EINVAL, "nC and nE must be positive");
  if (nE > (int64_t(1) << 26) || nC > (int64_t(1) << 28)) return err(PHFEM_EINVAL, "mesh too large for int32 ids");
  if (!tetra || !edges || !tet2edge || !edge_first_tet || !tet_edge_prefix || !counts)
    return err(PHFEM_EINVAL, "null edge output");
  const bool want_faces = flags & PHFEM_CONNECT_FACES, want_n2e = flags & PHFEM_CONNECT_NODES2EDGE;
  if (want_faces && (!faces || !tet2face || !sigma || !face2tet)) return err(PHFEM_EINVAL, "null face output");
  if (want_n2e && (!n2e_rowptr || !n2e_col || !n2e_edge)) return err(PHFEM_EINVAL, "null Nodes2Edge output");
  if (!work || work_bytes < phfem_connect_workspace(nC, nE, flags))
    return err(PHFEM_EWORKSPACE, "connect workspace too small");

  Arena a(work, work_bytes);
  if (nE <= SMALL_NE && !want_n2e) {
    ConnWS w;
    conn_layout(a, nC, nE, flags, w);
    PH_LAUNCH_B("connect_small", 16.0 * nE + 36.0 * nE + 3.6 * nE * 4 + (want_faces ? 26.0 * 4 * nE : 0.0),
                k_connect_small, 1, SMT, 0, s, (int)nC, (int)nE, tetra, want_faces ? 1 : 0, edges, tet2edge,
                edge_first_tet, tet_edge_prefix, faces, tet2face, sigma, face2tet, nbr, w.total);
    uint32_t h3[3] = {0, 0, 0};
    PH_HIP(hipMemcpyAsync(h3, w.total, sizeof(h3), hipMemcpyDeviceToHost, s));
    PH_HIP(hipStreamSynchronize(s));
    if (h3[2]) return dev_flags_to_status((int)h3[2]);
    counts[0] = h3[0];
    counts[1] = want_faces ? h3[1] : 0;
    counts[2] = want_faces ? 2 * (int64_t)h3[1] - 4 * nE : 0;
    return PHFEM_OK;
  }
  if (!(flags & PHFEM_CONNECT_RADIX)) {
    bool redo = false;
    const int rc = connect_bucket(nC, nE, tetra, flags, a, edges, tet2edge, edge_first_tet, tet_edge_prefix,
                                  n2e_rowptr, n2e_col, n2e_edge, faces, tet2face, sigma, face2tet, nbr, counts,
                                  &redo, s);
    if (rc || !redo) return rc;
    a.off = 0;
  }
  return connect_radix(nC, nE, tetra, flags, a, edges, tet2edge, edge_first_tet, tet_edge_prefix, n2e_rowptr,
                       n2e_col, n2e_edge, faces, tet2face, sigma, face2tet, nbr, counts, s);
}
