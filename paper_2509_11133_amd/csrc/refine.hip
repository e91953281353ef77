// 12-subtet red refinement on the device (Section 3.4, RedRefine and refineFaces).
//
// The paper numbers the new nodes by a coordinate-keyed stable unique over
// (tet; centroid, IJ, IK, IL, JK, JL, KL).  Every tet contributes its centroid and the
// midpoints of the edges that first appear in it, so that order has a closed form given
// the NumEdges outputs (first-appearance edge numbering, first tet of every edge, prefix
// count of edges first seen before every tet):
//     centroid(t) = nC + t + prefix(t),     midpoint(e) = nC + first_tet(e) + e + 1.
// Each tet writes its own new nodes (a contiguous id range) and its 12 children, so the
// kernel needs no sort and no comparison of floating-point coordinates.
#include "common.hpp"

namespace ph {

constexpr int RT = 256;

// one tet: its new coordinates (written directly) and its children (into the LDS rows)
__device__ __forceinline__ void refine_tet(int64_t nC, const double* __restrict__ X, int64_t nE,
                                           const int32_t* __restrict__ tet, const int32_t* __restrict__ t2e,
                                           const int32_t* __restrict__ eft, const int32_t* __restrict__ pre,
                                           int64_t nCo, double* __restrict__ Xo, uint32_t* __restrict__ bad, int64_t t,
                                           int32_t (*sT)[12 * RT], int l) {
  const int64_t nEd = nCo - nC - nE;
  int v[4], e[6], m[6];
  bool ok = true;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    v[i] = tet[i * nE + t];
    ok = ok && (uint32_t)v[i] < (uint64_t)nC;
  }
  const int64_t C64 = nC + t + pre[t];
  ok = ok && C64 >= nC && C64 < nCo;
  const int C = (int)C64;
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    e[j] = t2e[j * nE + t];
    const bool eok = (uint32_t)e[j] < (uint64_t)nEd;
    const int ft = eok ? eft[e[j]] : 0;
    const int64_t mj = nC + (int64_t)ft + e[j] + 1;
    ok = ok && eok && mj > nC && mj < nCo;
    m[j] = (int)mj;
    e[j] = (ft == t) ? 1 : 0;  // reuse: does the edge first appear in this tet?
  }
  if (!ok) {  // ids outside the mesh: no coordinates, children rows -1, and the call fails
    if (bad) atomicOr(bad, 1u);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int c = 0; c < 12; ++c) sT[i][c == 0 ? l : RT + 11 * l + c - 1] = -1;
    return;
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double x0 = X[d * nC + v[0]], x1 = X[d * nC + v[1]], x2 = X[d * nC + v[2]], x3 = X[d * nC + v[3]];
    Xo[d * nCo + C] = (((x0 + x1) + x2) + x3) / 4.0;
    const double xs[4] = {x0, x1, x2, x3};
#pragma unroll
    for (int j = 0; j < 6; ++j)
      if (e[j]) Xo[d * nCo + m[j]] = (xs[ev0(j)] + xs[ev1(j)]) / 2.0;
  }
  // children (RedRefine's vertex lists; m0..m5 = midpoints of IJ IK IL JK JL KL)
  const int I = v[0], J = v[1], K = v[2], L = v[3];
  const int ch[12][4] = {{I, m[0], m[1], m[2]},    {J, m[3], m[0], m[4]},    {K, m[1], m[3], m[5]},
                         {L, m[5], m[4], m[2]},    {m[0], m[1], m[2], C},    {m[3], m[0], m[4], C},
                         {m[1], m[3], m[5], C},    {m[5], m[4], m[2], C},    {m[0], m[3], m[1], C},
                         {m[1], m[5], m[2], C},    {m[0], m[2], m[4], C},    {m[5], m[3], m[4], C}};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    sT[i][l] = ch[0][i];
#pragma unroll
    for (int c = 1; c < 12; ++c) sT[i][RT + 11 * l + (c - 1)] = ch[c][i];
  }
}

// The children of a workgroup's RT tets are rows [t0, t0 + RT) (child 0) and
// [nE + 11 t0, nE + 11 (t0 + RT)) (children 1..11): staged in LDS and stored as two
// contiguous ranges per vertex array (full cache lines instead of stride-11 stores).  The
// grid covers max(nE, nC): thread g also copies the old node g's coordinates.
__global__ __launch_bounds__(RT) void k_refine(int64_t nC, const double* __restrict__ X, int64_t nE,
                                               const int32_t* __restrict__ tet, const int32_t* __restrict__ t2e,
                                               const int32_t* __restrict__ eft, const int32_t* __restrict__ pre,
                                               int64_t nCo, double* __restrict__ Xo, int32_t* __restrict__ To,
                                               uint32_t* __restrict__ bad) {
  __shared__ int32_t sT[4][12 * RT];
  const int64_t t0 = (int64_t)blockIdx.x * RT;
  const int nb = nE - t0 < RT ? (nE > t0 ? (int)(nE - t0) : 0) : RT;
  const int l = threadIdx.x;
  if (t0 + l < nC) {
#pragma unroll
    for (int d = 0; d < 3; ++d) Xo[d * nCo + t0 + l] = X[d * nC + t0 + l];
  }
  if (l < nb) refine_tet(nC, X, nE, tet, t2e, eft, pre, nCo, Xo, bad, t0 + l, sT, l);
  __syncthreads();
  const int64_t nEo = 12 * nE;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    int32_t* o = To + i * nEo;
    for (int k = l; k < nb; k += RT) st_nt(o + t0 + k, sT[i][k]);
    for (int k = l; k < 11 * nb; k += RT) st_nt(o + nE + 11 * t0 + k, sT[i][RT + k]);
  }
}

// edge id of the node pair (a, b) from the Nodes2Edge CSR (row min(a,b), column max(a,b))
__device__ __forceinline__ int n2e_lookup(int a, int b, int64_t nC, const int32_t* __restrict__ rp,
                                          const int32_t* __restrict__ col, const int32_t* __restrict__ eid) {
  int lo = a < b ? a : b, hi = a < b ? b : a;
  if (lo < 0 || hi >= nC) return -1;
  for (int q = rp[lo]; q < rp[lo + 1]; ++q)
    if (col[q] == hi) return eid[q];
  return -1;
}

__global__ __launch_bounds__(RT) void k_refine_faces(int64_t n, const int32_t* __restrict__ F, int64_t nC,
                                                     const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                                                     const int32_t* __restrict__ eid, const int32_t* __restrict__ eft,
                                                     int32_t* __restrict__ Fo, int* __restrict__ flags) {
  int64_t f = (int64_t)blockIdx.x * RT + threadIdx.x;
  if (f >= n) return;
  int n1 = F[f], n2 = F[n + f], n3 = F[2 * n + f];
  if ((uint32_t)n1 >= (uint64_t)nC || (uint32_t)n2 >= (uint64_t)nC || (uint32_t)n3 >= (uint64_t)nC) {
    atomicOr(flags, DEV_NOFACE);
    return;
  }
  int e12 = n2e_lookup(n1, n2, nC, rp, col, eid), e23 = n2e_lookup(n2, n3, nC, rp, col, eid),
      e13 = n2e_lookup(n1, n3, nC, rp, col, eid);
  if (e12 < 0 || e23 < 0 || e13 < 0) {
    atomicOr(flags, DEV_NOFACE);
    return;
  }
  int m12 = (int)(nC + eft[e12] + e12 + 1), m23 = (int)(nC + eft[e23] + e23 + 1), m13 = (int)(nC + eft[e13] + e13 + 1);
  const int rows[4][3] = {{n1, m12, m13}, {n2, m23, m12}, {n3, m13, m23}, {m12, m23, m13}};
  const int64_t n4 = 4 * n;
#pragma unroll
  for (int mm = 0; mm < 3; ++mm) {
    Fo[mm * n4 + f] = rows[0][mm];
#pragma unroll
    for (int c = 1; c < 4; ++c) Fo[mm * n4 + n + 3 * f + (c - 1)] = rows[c][mm];
  }
}

int launch_refine(int64_t nC, const double* coord, int64_t nE, const int32_t* tetra, const int32_t* t2e,
                  const int32_t* eft, const int32_t* pre, int64_t nCo, double* coord_out, int32_t* tetra_out,
                  hipStream_t s, uint32_t* bad) {
  const int64_t nEd = nCo - nC - nE;
  PH_LAUNCH_B("refine", 44.0 * nE + 4.0 * nEd + 24.0 * nC + 192.0 * nE + 24.0 * (nE + nEd) + 48.0 * nC, k_refine,
              grid_for(std::max(nE, nC), RT), RT, 0, s, nC, coord, nE, tetra, t2e, eft, pre, nCo, coord_out, tetra_out,
              bad);
  return PHFEM_OK;
}

}  // namespace ph

using namespace ph;

extern "C" size_t phfem_refine_workspace(int64_t nDb, int64_t nNb) {
  if (nDb < 0 || nNb < 0 || nDb + nNb == 0) return 0;
  Arena a;  // the face lookups' error word
  a.take<int>(1);
  return a.size();
}

extern "C" int phfem_refine(int64_t nC, const double* coord, int64_t nE, const int32_t* tetra, int64_t nEd,
                            const int32_t* tet2edge, const int32_t* edge_first_tet, const int32_t* tet_edge_prefix,
                            const int32_t* n2e_rowptr, const int32_t* n2e_col, const int32_t* n2e_edge, int64_t nDb,
                            const int32_t* db, int64_t nNb, const int32_t* nb, void* work, size_t work_bytes,
                            double* coord_out, int32_t* tetra_out, int32_t* db_out, int32_t* nb_out,
                            phfem_stream_t stream_) {
  clear_error();
  hipStream_t s = (hipStream_t)stream_;
  if (nC <= 0 || nE <= 0 || nEd <= 0 || nDb < 0 || nNb < 0) return err(PHFEM_EINVAL, "bad sizes");
  const int64_t nCo = nC + nEd + nE;
  if (12 * nE >= (int64_t(1) << 31) || nCo >= (int64_t(1) << 31)) return err(PHFEM_EINVAL, "refined mesh exceeds int32");
  if (!coord || !tetra || !tet2edge || !edge_first_tet || !tet_edge_prefix || !coord_out || !tetra_out)
    return err(PHFEM_EINVAL, "null argument");
  const bool faces = nDb + nNb > 0;
  if (faces && (!n2e_rowptr || !n2e_col || !n2e_edge)) return err(PHFEM_EINVAL, "boundary faces need Nodes2Edge");
  if ((nDb > 0 && (!db || !db_out)) || (nNb > 0 && (!nb || !nb_out))) return err(PHFEM_EINVAL, "null face list");
  if (faces && (!work || work_bytes < phfem_refine_workspace(nDb, nNb)))
    return err(PHFEM_EWORKSPACE, "refine workspace too small");
  int rc = launch_refine(nC, coord, nE, tetra, tet2edge, edge_first_tet, tet_edge_prefix, nCo, coord_out, tetra_out, s,
                         nullptr);
  if (rc) return rc;
  if (!faces) return PHFEM_OK;
  // error flag of the face lookups, in the caller's workspace
  Arena a(work, work_bytes);
  int* dflag = a.take<int>(1);
  PH_HIP(hipMemsetAsync(dflag, 0, sizeof(int), s));
  if (nDb > 0)
    PH_LAUNCH("refine_faces", k_refine_faces, grid_for(nDb, RT), RT, 0, s, nDb, db, nC, n2e_rowptr, n2e_col,
              n2e_edge, edge_first_tet, db_out, dflag);
  if (nNb > 0)
    PH_LAUNCH("refine_faces", k_refine_faces, grid_for(nNb, RT), RT, 0, s, nNb, nb, nC, n2e_rowptr, n2e_col,
              n2e_edge, edge_first_tet, nb_out, dflag);
  int h = 0;
  PH_HIP(hipMemcpyAsync(&h, dflag, sizeof(int), hipMemcpyDeviceToHost, s));
  PH_HIP(hipStreamSynchronize(s));
  if (h) return dev_flags_to_status(h);
  return PHFEM_OK;
}
