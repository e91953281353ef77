/*
 * phfem.h -- C-ABI of the MI355X (gfx950) hot path of the vectorized primal hybrid FEM of
 * "Vectorized 3D mesh refinement and implementation of primal hybrid FEM in MATLAB"
 * (Nagula Mallesham, Gaddam, Valdman, Acharya; arXiv 2509.11133).
 *
 * The path: 12-subtet red refinement (Section 3.4), Nodes-to-Edge / Edges-to-Tetrahedron /
 * Face-to-Tetrahedron connectivity (Sections 3.1-3.3), lowest-order primal hybrid local
 * matrices (Section 4.2), element-wise Schur complement (Section 4.6, Algorithm 1) into a
 * sparse SPD face system, Jacobi-PCG solve and recovery, and the adjoint gradient.
 *
 * Conventions for every call
 *  - Return value: PHFEM_OK (0) or one of the phfem_status codes; phfem_last_error() gives
 *    a text for the calling thread.  Arguments are validated before any work is enqueued;
 *    on a validation failure nothing is written.  Errors found on the device (bad node
 *    index, inconsistent orientation, zero volume) are reported by the calls that read back
 *    a count (connect, refine with boundary faces, solve, grad); outputs are then undefined.
 *  - Array arguments are DEVICE pointers to caller-owned memory; scalars and the *_stats /
 *    counts / params structs are HOST memory.  Nothing is allocated inside a call: scratch
 *    comes from the caller through (work, work_bytes), sized by the matching
 *    phfem_*_workspace() query (256-byte aligned pointer expected).
 *  - Indices are 0-based int32.  Arrays are SoA ("[r][n]" = r rows of n contiguous
 *    entries, row stride n): coord[3][nC] float64, tetra[4][nE] int32.  This is the paper's
 *    column-major MATLAB layout (k-th column of an n x r matrix = k-th row here).
 *  - Local numbering of tet T = [a b c d]: edges IJ IK IL JK JL KL (j = 0..5, Listing 2);
 *    faces [a b c], [a c d], [a d b], [d c b] (k = 0..3, Section 2.2).
 *  - A "slot" is 4*t + k (local face k of tet t).
 *  - Every call enqueues its kernels on `stream` (a hipStream_t) and returns without
 *    waiting, except where a count must be read back (documented per call).
 *  - Every kernel writes each output element exactly once or sums exactly two terms in
 *    floating point, so results are bitwise reproducible run to run, except the
 *    coordinate gradient of phfem_grad (atomic sums over the tets at a vertex).
 */
#ifndef PHFEM_H
#define PHFEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* phfem_stream_t; /* == hipStream_t */

typedef enum {
  PHFEM_OK = 0,
  PHFEM_EINVAL = 1,     /* bad argument, node index out of range, repeated node, face not in mesh */
  PHFEM_EORIENT = 2,    /* an oriented face occurs twice: tets not consistently oriented / non-manifold */
  PHFEM_EDEGEN = 3,     /* zero-volume tet */
  PHFEM_ESINGULAR = 4,  /* c <= 0: element matrices kappa K + c M singular */
  PHFEM_ENOCONV = 5,    /* solver stopped at max_iter above tolerance (stats still filled) */
  PHFEM_EWORKSPACE = 6, /* work_bytes smaller than the workspace query */
  PHFEM_EHIP = 7        /* HIP runtime error */
} phfem_status;

/* Thread-local text of the last error ("" after success). */
const char* phfem_last_error(void);
int phfem_abi_version(void);

/* ---------------------------------------------------------------- data functions ---- */
/* f (load) and u_D (Dirichlet data) are evaluated in the kernels from a kind + 4 params. */
enum {
  PHFEM_FUN_ZERO = 0,
  PHFEM_FUN_CONST = 1,         /* p0 */
  PHFEM_FUN_SIN3 = 2,          /* p0 sin(pi x) sin(pi y) sin(pi z) */
  PHFEM_FUN_LINEAR = 3,        /* p0 + p1 x + p2 y + p3 z */
  PHFEM_FUN_X2Y2Z2 = 4,        /* p0 x^2 y^2 z^2 (exact solution of the paper's example) */
  PHFEM_FUN_X2Y2Z2_LOAD = 5    /* -p0 Lap(x^2y^2z^2) + p1 x^2y^2z^2 (its load) */
};
enum { PHFEM_QUAD_FACE_CENTROID = 0, PHFEM_QUAD_P1_INTERP = 1 };
enum { PHFEM_FP64 = 0, PHFEM_MIXED = 1 };

/* Problem -div(kappa grad u) + c u = f (model problem of Section 4 with a per-tet kappa;
 * the paper has kappa = c = 1), u = u_D on Dirichlet faces, kappa grad u . nu = g on the
 * Neumann faces flagged in `neumann` (NULL: every boundary face is a Dirichlet face).
 *  g: the flux kappa_T grad(u_g) . nu of the data function u_g = fun(g_kind, g_par), nu the
 *        outward unit normal (the paper's example prescribes the flux of its exact solution);
 *        taken at the face centroid, LN = |F| g(Ct_F) / 3 on the face's vertices.
 *  neumann: device array of nF flags (1 = Neumann face; only boundary faces may be flagged),
 *        caller-owned, read by condense and solve.  A Neumann face leaves the multiplier
 *        space as in the paper: the face system keeps its row as lambda_F = g(Ct_F) (diagonal
 *        1, no coupling: its column is zero in every other row), which is the paper's system
 *        over the other faces (RFaces) with LN in the load, without renumbering.
 *  quad: PHFEM_QUAD_FACE_CENTROID = the paper's load rule (f at the 4 face centroids,
 *        weight |T|/4, StiffMassPH); PHFEM_QUAD_P1_INTERP = b(T) = M(T) f(x_i).
 *  precision: PHFEM_FP64, or PHFEM_MIXED = FP32 local-matrix and element-Schur arithmetic
 *        (Jacobian determinant and volume in FP64) summed into the FP64 face system. */
typedef struct {
  double c;
  double kappa_const; /* kappa when the kappa array is NULL */
  int32_t f_kind;
  double f_par[4];
  int32_t ud_kind;
  double ud_par[4];
  int32_t quad;
  int32_t precision;
  int32_t g_kind;
  double g_par[4];
  const uint8_t* neumann;
} phfem_params;

/* ---------------------------------------------------------------- connect (a1-a3) ---- */
enum {
  PHFEM_CONNECT_EDGES = 1,      /* Nodes-to-Edge numbering (NumEdges, Listing 2) */
  PHFEM_CONNECT_FACES = 2,      /* Edges-to-Tet neighbours + Faces (Listings 3-4, fullFaces) */
  PHFEM_CONNECT_NODES2EDGE = 4, /* also export Nodes2Edge (upper triangle) as CSR */
  PHFEM_CONNECT_RADIX = 8       /* take the radix-sort path (same outputs; for comparison) */
};

size_t phfem_connect_workspace(int64_t nC, int64_t nE, int32_t flags);

/* Connectivity of a conforming, consistently oriented tet mesh (all tets with the same
 * sign of det[b-a, c-a, d-a]).
 * Edges (Section 3.1, Listing 2): the 6 local edges of every tet, in (tet, local edge)
 * order, keyed by their sorted node pair; edge e = rank of the first appearance (MATLAB
 * unique(...,'stable')).
 *   edges[2][nEd]        sorted node pair of edge e (paper's U); capacity 12 nE ints
 *   tet2edge[6][nE]      edge of local edge j of tet t
 *   edge_first_tet[nEd]  first tet holding edge e; capacity 6 nE
 *   tet_edge_prefix[nE]  number of edges first seen in tets < t
 *   n2e_rowptr[nC+1], n2e_col[nEd], n2e_edge[nEd] (flag NODES2EDGE): Nodes2Edge(i,j) for
 *                        i < j as CSR over i with ascending j; capacities nC+1, 6 nE, 6 nE
 * Faces (Sections 3.2-3.3, Listings 3-4, Remark 1): neighbour across local face k = the
 * other tet holding the face (the paper's Edges2Tetra(e_ij, e_jk)); a face is numbered at
 * its owner (lowest tet index holding it) by rank of (owner, local face).
 *   faces[3][nF]         owner's oriented tuple (paper's Faces); capacity 12 nE ints
 *   tet2face[4][nE]      face of local face k of tet t (fullFaces' g_ind)
 *   sigma[4][nE]         +1 at the owner's occurrence, -1 at the other (sigma_k, Section 4.1)
 *   face2tet[2][nF]      slot 4t+k of the owner, slot of the neighbour or -1; capacity 8 nE
 *   nbr[4][nE]           tet across local face k, -1 on the boundary (may be NULL)
 * counts (host int64[3]): nEd, nF, nB (boundary faces).  Face outputs may be NULL without
 * the FACES flag.  Synchronizes `stream` (counts are read back).  Three paths, identical
 * outputs: a mesh of at most 256 tets without NODES2EDGE is connected in one workgroup (each
 * occurrence compared with the earlier ones); larger meshes bucket the occurrences by their
 * lowest node (counting sort) and resolve each bucket in LDS, falling back by themselves to
 * a stable radix sort of the occurrence keys when a node is the lowest node of more than
 * 8192 occurrences (or always, with PHFEM_CONNECT_RADIX).
 * Errors: EINVAL (nC, nE <= 0 or > 2^28 / 2^26, node out of range, repeated node in a tet),
 * EORIENT (a face held by two tets in the same orientation or by more than two tets). */
int phfem_connect(int64_t nC, int64_t nE, const int32_t* tetra, int32_t flags, void* work, size_t work_bytes,
                  int32_t* edges, int32_t* tet2edge, int32_t* edge_first_tet, int32_t* tet_edge_prefix,
                  int32_t* n2e_rowptr, int32_t* n2e_col, int32_t* n2e_edge, int32_t* faces, int32_t* tet2face,
                  int8_t* sigma, int32_t* face2tet, int32_t* nbr, int64_t* counts, phfem_stream_t stream);

/* ---------------------------------------------------------------- refine (a4) ------- */
/* 12-subtet red refinement (Section 3.4, RedRefine + refineFaces).  New nodes: for every
 * tet its centroid (((x_I+x_J)+x_K)+x_L)/4 and the midpoints (x_a+x_b)/2 of its edges, in
 * first-appearance order over (tet; centroid, IJ, IK, IL, JK, JL, KL) -- the paper's
 * coordinate-keyed stable unique.  In closed form: centroid(t) = nC + t + prefix(t),
 * midpoint(e) = nC + first_tet(e) + e + 1.  Child 1 of tet t at row t, children 2..12 at
 * rows nE + 11 t + (c - 2) with the vertex lists of RedRefine.  Boundary faces [n1 n2 n3]
 * split into 4 keeping their orientation, child 1 at row f, children 2..4 at
 * n + 3 f + (c - 2).
 * Inputs: the coarse mesh and its phfem_connect edge outputs (+ Nodes2Edge CSR when
 * nDb + nNb > 0).  Outputs: coord_out[3][nC + nEd + nE], tetra_out[4][12 nE],
 * db_out[3][4 nDb], nb_out[3][4 nNb] (row strides = those counts).  Coordinates are
 * bitwise those of the paper's formulas.  With boundary faces the call takes a workspace
 * (phfem_refine_workspace; work may be NULL without them) for its error word and
 * synchronizes once (EINVAL if a boundary face is not a mesh face; EWORKSPACE).  A tet whose vertex, edge or derived
 * node ids fall outside the mesh is skipped (its outputs are left unwritten, nothing is
 * written out of range); phfem_refine_connected reports such input. */
size_t phfem_refine_workspace(int64_t nDb, int64_t nNb); /* 0 without boundary faces */
int phfem_refine(int64_t nC, const double* coord, int64_t nE, const int32_t* tetra, int64_t nEd,
                 const int32_t* tet2edge, const int32_t* edge_first_tet, const int32_t* tet_edge_prefix,
                 const int32_t* n2e_rowptr, const int32_t* n2e_col, const int32_t* n2e_edge, int64_t nDb,
                 const int32_t* db, int64_t nNb, const int32_t* nb, void* work, size_t work_bytes,
                 double* coord_out, int32_t* tetra_out, int32_t* db_out, int32_t* nb_out, phfem_stream_t stream);

/* ---------------------------------------------------------------- face lookup ------- */
/* Boundary faces of the mesh numbering named by node triples: the lookup the Multiplier
 * routine of Section 4.4 makes for its Neumann faces (g_NFs) before it forms the load LN and
 * removes those faces from the multiplier space.  tris[3][n]: n triangles (nodes in any
 * order, e.g. a refined Nb list of phfem_refine); faces[3][nF], face2tet[2][nF]: the face
 * numbering of phfem_connect / phfem_refine_connected.  Outputs: flags[nF] (uint8, 1 = the
 * face is a boundary face whose node set is one of the triangles, else 0; the
 * params.neumann array) and face_of[n] (may be NULL: the face id of each triangle).  n = 0
 * writes zero flags and needs no workspace.  Triangles go into a hash table in the
 * workspace (phfem_face_lookup_workspace(n)), probed once per face.  Synchronizes (one
 * readback).  Errors: EINVAL (a triangle with a node out of range or a repeated node, or one
 * that is not a boundary face of the mesh; outputs then unspecified), EWORKSPACE. */
size_t phfem_face_lookup_workspace(int64_t n);
int phfem_face_lookup(int64_t nC, int64_t nF, const int32_t* faces, const int32_t* face2tet, int64_t n,
                      const int32_t* tris, void* work, size_t work_bytes, uint8_t* flags, int32_t* face_of,
                      phfem_stream_t stream);

/* Refinement with connectivity: phfem_refine's outputs plus the refined mesh's full
 * phfem_connect outputs (edges, tet2edge, edge_first_tet, tet_edge_prefix, faces,
 * tet2face, sigma, face2tet, nbr) -- the same numbering NumEdges / FacesUp give the
 * refined mesh (Sections 3.1-3.4), derived in closed form from the coarse numbering with
 * no sort.  Inputs must be the coarse mesh's own phfem_connect (or phfem_refine_connected)
 * outputs.  Refined sizes: nC' = nC + nEd + nE, nE' = 12 nE, nEd' = 2 nEd + 3 nF + 6 nE,
 * nF' = 4 nF + 16 nE, nB' = 2 nF' - 4 nE' (written to counts[3] = {nEd', nF', nB'}); output
 * arrays are packed SoA with those strides (capacities = these sizes).  No boundary face
 * lists (use phfem_refine for Db/Nb).
 * Input check: the refined edge and face totals found by the kernels must equal the
 * recurrences above (they do exactly when the input is a first-appearance numbering of a
 * conforming, consistently oriented mesh), and every vertex id, tet2edge id and derived
 * refined node id must lie in range.
 * status == NULL: synchronizes once and returns EINVAL on failure.  status != NULL (device
 * int32, caller-owned): nothing synchronizes; on failure the call ORs 1 (an id out of
 * range) or 2 (totals differ) into *status, so one zeroed word can collect a whole chain of
 * levels and be read once at the end.  The outputs of a failed check are unspecified (no
 * write leaves the output arrays either way). */
size_t phfem_refine_connected_workspace(int64_t nE, int64_t nEd);
int phfem_refine_connected(int64_t nC, const double* coord, int64_t nE, const int32_t* tetra, int64_t nEd, int64_t nF,
                           const int32_t* tet2edge, const int32_t* edge_first_tet, const int32_t* tet_edge_prefix,
                           const int32_t* tet2face, const int32_t* nbr, void* work, size_t work_bytes,
                           double* coord_out, int32_t* tetra_out, int32_t* edges_out, int32_t* tet2edge_out,
                           int32_t* edge_first_tet_out, int32_t* tet_edge_prefix_out, int32_t* faces_out,
                           int32_t* tet2face_out, int8_t* sigma_out, int32_t* face2tet_out, int32_t* nbr_out,
                           int64_t* counts, int32_t* status, phfem_stream_t stream);

/* Mesh sizes after `levels` refinements: out[4] = {nC, nE, nEd, nF} by the recurrences of
 * phfem_refine_connected (host only).  EINVAL for levels < 0 or non-positive sizes. */
int phfem_refined_sizes(int64_t nC, int64_t nE, int64_t nEd, int64_t nF, int32_t levels, int64_t* out);

/* `levels` (1..16) chained phfem_refine_connected calls in one call: the intermediate
 * meshes live in the workspace (two buffers sized for level levels-1), only the last
 * level's mesh and connectivity are written to the outputs (capacities: the sizes of
 * phfem_refined_sizes(..., levels)), counts[3] as for one level.  Results are bitwise those
 * of the chained calls.  status as for phfem_refine_connected (one word collects every
 * level); with status == NULL the call synchronizes once at the end and returns EINVAL if
 * any level's check failed.  Workspace bytes: phfem_refine_connected_levels_workspace. */
size_t phfem_refine_connected_levels_workspace(int64_t nC, int64_t nE, int64_t nEd, int64_t nF, int32_t levels);
int phfem_refine_connected_levels(int64_t nC, const double* coord, int64_t nE, const int32_t* tetra, int64_t nEd,
                                  int64_t nF, const int32_t* tet2edge, const int32_t* edge_first_tet,
                                  const int32_t* tet_edge_prefix, const int32_t* tet2face, const int32_t* nbr,
                                  int32_t levels, void* work, size_t work_bytes, double* coord_out, int32_t* tetra_out,
                                  int32_t* edges_out, int32_t* tet2edge_out, int32_t* edge_first_tet_out,
                                  int32_t* tet_edge_prefix_out, int32_t* faces_out, int32_t* tet2face_out,
                                  int8_t* sigma_out, int32_t* face2tet_out, int32_t* nbr_out, int64_t* counts,
                                  int32_t* status, phfem_stream_t stream);

/* ---------------------------------------------------------------- assemble (a5-a6) --- */
/* Per-tet local blocks (Sections 4.2-4.5; StiffMassPH, Multiplier, the page solves of
 * SchurComplement_vectorization).  kappa[nE] may be NULL (then p->kappa_const).
 * Outputs (each may be NULL; float64 in both precisions):
 *   vol[nE]      |det J| / 6
 *   K[16][nE]    kappa K(T), row-major 4x4 (K(T) of Section 4.2 with |T| read as 6 vol)
 *   d[4][nE]     sigma_k |F_k|; C(T) row k = d_k r_k (C(T) of Section 4.2)
 *   B[4][nE]     load vector of the tet (rule p->quad)
 *   S[16][nE]    element Schur block C A^-1 C' with A = kappa K + c M (SPD; the paper's
 *                S(T) is its negative)
 *   r[4][nE]     C A^-1 B
 * Errors: EINVAL, ESINGULAR (c <= 0).  Does not synchronize. */
int phfem_assemble(int64_t nC, const double* coord, int64_t nE, const int32_t* tetra, const int8_t* sigma,
                   const double* kappa, const phfem_params* p, double* vol, double* K, double* d, double* B,
                   double* S, double* r, phfem_stream_t stream);

/* (phfem_assemble ignores params.neumann: its B(T) is the load without LN.) */

/* ---------------------------------------------------------------- condense (a5-a7) --- */
size_t phfem_condense_workspace(int64_t nC, int64_t nE, int64_t nF, int32_t precision);

/* Condensed face system S+ lambda = r+ with S+ = sum_T P_T' C A^-1 C' P_T and
 * r+ = b_D - sum_T P_T' C A^-1 B, b_D,F = |F| u_D(centroid F) on boundary faces
 * (the assembly step of Algorithm 1, Listing 8; sign-flipped to SPD form).
 * Storage: diagonal separate, off-diagonals as CSR with a fixed 6 slots per row:
 *   rowptr[nF+1] = 6 F, col[6 nF], val[6 nF], diag[nF], rhs[nF]; all float64 (the FP64
 *   sums of FP32 blocks in mixed).  An interior face's row holds the 6 faces its two tets
 *   couple it to, columns ascending; a boundary face's row holds its 3, ascending, then 3
 *   explicit zeros in column F (boundary faces are O(nF^(2/3)), so the padding is a
 *   vanishing fraction and the row pointers need no scan).
 * Each off-diagonal has exactly one contributing tet; a diagonal / rhs entry is the owner
 * tet's term plus the neighbour's (in that order).  Tiles of 256 consecutive tets, two
 * passes: every tet whose face is owned by a tet of another tile writes that face's row of
 * its element block as a record (row k of the element Schur block, (C A^-1 B)_k, the other
 * face ids; FP32 records in mixed precision); then each tile recomputes its tets' blocks in
 * LDS and writes the rows of the faces it owns (a contiguous id range, faces being numbered
 * at their owner), taking the second tet's row from LDS or from its record.  Inputs from
 * phfem_connect or phfem_refine_connected (nbr required: it tells the tets with cross-tile
 * faces apart).  col 8-byte and val 16-byte aligned (vector stores of a row's slots).
 * Errors: EINVAL, ESINGULAR, EWORKSPACE.  Does not synchronize (EDEGEN is reported by
 * phfem_solve). */
int phfem_condense(int64_t nC, const double* coord, int64_t nE, const int32_t* tetra, int64_t nF,
                   const int32_t* faces, const int32_t* tet2face, const int8_t* sigma, const int32_t* nbr,
                   const int32_t* face2tet, const double* kappa, const phfem_params* p, void* work,
                   size_t work_bytes, int32_t* rowptr, int32_t* col, double* val, double* diag, double* rhs,
                   phfem_stream_t stream);

/* Re-assembly with a reused pattern and batched coefficient fields (for optimisation loops
 * that change kappa on a fixed mesh; the pattern of S+ depends on the connectivity alone,
 * the assembly step of Algorithm 1, Listing 8).  The face systems of nk >= 1 fields
 * kappa[nk][nE] (kappa may be NULL only for nk = 1: params.kappa_const) in one call:
 *   val[nk][6 nF], diag[nk][nF], rhs[nk][nF] (float64, the layout of phfem_condense per field).
 * rowptr[nF+1] and col[6 nF] are written when both are given and left untouched when both are
 * NULL (values-only re-assembly: the pattern phfem_condense wrote for the same connectivity
 * stays valid; it saves the 28 B/face of col and row pointers).  The coordinate copy is built
 * once per call; the cross-tile pass runs once per group of up to four fields (reading the
 * mesh once for the group), the tile pass once per field (a fused pass over several fields
 * costs occupancy in registers); field j's arrays equal phfem_condense's with kappa + j nE,
 * bit for bit.  Workspace: phfem_condense_batch_workspace (one group's cross-tile records:
 * min(nk, 4) fields).
 * Errors: EINVAL (also for only one of rowptr / col), ESINGULAR, EWORKSPACE.  Does not
 * synchronize. */
size_t phfem_condense_batch_workspace(int64_t nC, int64_t nE, int64_t nF, int32_t precision, int32_t nk);
int phfem_condense_batch(int64_t nC, const double* coord, int64_t nE, const int32_t* tetra, int64_t nF,
                         const int32_t* faces, const int32_t* tet2face, const int8_t* sigma, const int32_t* nbr,
                         const int32_t* face2tet, int32_t nk, const double* kappa, const phfem_params* p, void* work,
                         size_t work_bytes, int32_t* rowptr, int32_t* col, double* val, double* diag, double* rhs,
                         phfem_stream_t stream);

/* ---------------------------------------------------------------- solve (a8-a9) ------ */
enum { PHFEM_SOLVE_FP64_PCG = 0, PHFEM_SOLVE_FP32_PCG_FP64_IR = 1 };

typedef struct {
  int32_t iters;        /* PCG iterations, all of them (FP32 and FP64 in IR mode) */
  int32_t ir_steps;     /* residual replacements (IR mode) / true-residual corrections (FP64 mode) */
  double rel_res;       /* final ||b_D - C U(lambda)|| / ||r+||, evaluated in FP64 matrix-free */
  double rhs_norm;      /* ||r+|| */
  int32_t polish_steps; /* IR mode: FP64 correction solves after the FP32 refinement */
  int32_t polish_iters; /* IR mode: their PCG iterations (included in iters) */
} phfem_solve_stats;

size_t phfem_solve_workspace(int64_t nE, int64_t nF, int32_t mode);

/* Solve S+ lambda = r+ (Jacobi-PCG; the paper solves it with a sparse direct solver,
 * Listing 8) and recover U(T) = A(T)^-1 (B(T) + C(T)' lambda(T)) (Algorithm 1, last loop).
 * (rowptr, col, val, diag, rhs) as phfem_condense writes them: 6 slots per row, rowptr[F] =
 * 6 F, column ids in [0, nF) -- checked on the device once per call (EINVAL otherwise); col
 * 8-byte and val 16-byte aligned (vector loads of a row's slots).
 *  mode FP64_PCG: Jacobi-PCG on the FP64 system, run as CG on its Jacobi-scaled FP64 copy
 *    D^-1/2 S+ D^-1/2 (same iterates; no diagonal in the product, no z vector), to
 *    ||r|| <= tol ||r+|| (the unscaled recurrence residual); then,
 *    while the true residual b_D - C U(lambda) (FP64, matrix-free) is above tol ||r+||, the
 *    stored system is solved again for the correction (iterative refinement; the stored
 *    system differs from the matrix-free operator by assembly rounding, so the recurrence
 *    alone levels off near 3.5e-11 relative at Kuhn L5 with lognormal kappa).  Stops after 8
 *    corrections or when one no longer halves the true residual, then with ENOCONV if the
 *    true residual is still above tol (stats.rel_res is the attainable accuracy).
 *  mode FP32_PCG_FP64_IR: iterative refinement without restarts: one FP32 PCG recurrence on
 *    the Jacobi-scaled FP32 copy D^-1/2 S+ D^-1/2 of the system (unit diagonal, so CG there
 *    is Jacobi-PCG on S+ with no diagonal reads and no z vector), whose residual is
 *    replaced by the scaled true residual D^-1/2 (b_D - C U(lambda)), recomputed per tet in
 *    FP64 from the geometry (not from the stored system), each time the FP32 residual has
 *    fallen by the factor inner_tol in the scaled 2-norm (in (0, 1); anything else means
 *    0.9, measured best: rarer replacements let the FP32 recurrence drift from the true
 *    residual, which costs iterations as the condition number grows -- Kuhn L6 to 1e-10:
 *    63.6K iterations at 0.9 against 83.4K at 0.7) since the last replacement; the FP32
 *    iterate, scaled back by D^-1/2, is then added to the FP64 solution and the search
 *    direction kept.  The FP32 phase ends when the true residual meets tol or 6
 *    replacements in a row gain less than 10 % (a replacement is also forced after 2048
 *    iterations without that gain).  Then an FP64 polish: 1 to 3 correction solves on the
 *    Jacobi-scaled FP64 stored system, each from the true residual to a relative 0.1
 *    (continuing while tol is unmet and each halves the true residual): the
 *    FP32 corrections barely resolve the smoothest error modes (cond x eps32 near 1 there),
 *    which leaves the FP32-phase iterate's error about ten times the FP64 solve's at an
 *    equal residual; the polish removes it.  ENOCONV when the true residual is still above
 *    tol (attainable accuracy reached, or max_iter).  stats.ir_steps counts the
 *    replacements, stats.polish_steps / polish_iters the FP64 corrections.
 * The true residual is summed per face from the per-tet terms, owner's first, so the
 * whole solve is bitwise reproducible run to run.
 * Outputs: lambda[nF], U[4][nE] (float64).  Synchronizes (residual checks every few
 * iterations).  Errors: EINVAL (also a vertex, face or slot id out of range, found on the
 * device), EDEGEN (zero-volume tet), ENOCONV (max_iter reached, or -- either mode -- the
 * refinement stopped gaining above tol: outputs and stats hold the last iterate and its
 * attainable rel_res), EWORKSPACE. */
int phfem_solve(int64_t nC, const double* coord, int64_t nE, const int32_t* tetra, int64_t nF,
                const int32_t* faces, const int32_t* tet2face, const int8_t* sigma, const int32_t* face2tet,
                const double* kappa, const phfem_params* p, const int32_t* rowptr, const int32_t* col,
                const double* val, const double* diag, const double* rhs, int32_t mode, double tol, double inner_tol,
                int32_t max_iter, void* work, size_t work_bytes, double* lambda, double* U,
                phfem_solve_stats* stats, phfem_stream_t stream);

/* Several loads on one face system (Algorithm 1: the condensed S serves every load; the loads
 * differ in f, u_D and g, not in kappa or c): nk (1..8) right-hand sides solved together.
 * p[nk]: one params struct per load, all with the same c, kappa_const, precision and
 * neumann == NULL (EINVAL otherwise; the Dirichlet boundary of the paper's system); kappa is
 * shared.  (rowptr, col, val, diag): the 6-slot system of phfem_condense (either precision;
 * checked once per call).  rhs[nk][nF] (may be NULL): the r+ of each load as phfem_condense
 * writes it; NULL: r+ = b_D - C A^-1 B evaluated per tet in FP64 (the true residual at
 * lambda = 0).  FP64 Jacobi-PCG for all loads in lockstep on the Jacobi-scaled FP64 copy of
 * the system: each iteration reads the matrix once for all loads (interleaved vectors; 72 B
 * per face of matrix plus 40 B per face and load, against 72 + 40 B per face for every load
 * solved alone), with each load's own alpha and beta, a load frozen once its recurrence
 * residual meets tol; then, as phfem_solve's FP64 mode, correction solves on the true
 * residuals (matrix-free FP64) of the loads still above tol, in lockstep again.
 * Outputs: lambda[nk][nF], U[nk][4][nE], stats[nk] (host; iters = lockstep iterations while
 * that load was active).  Synchronizes.  Errors: EINVAL, EDEGEN, ENOCONV (a load stopped
 * above tol; all outputs and stats are still written), EWORKSPACE. */
size_t phfem_solve_multi_workspace(int64_t nE, int64_t nF, int32_t nk);
int phfem_solve_multi(int64_t nC, const double* coord, int64_t nE, const int32_t* tetra, int64_t nF,
                      const int32_t* faces, const int32_t* tet2face, const int8_t* sigma, const int32_t* face2tet,
                      const double* kappa, int32_t nk, const phfem_params* p, const int32_t* rowptr,
                      const int32_t* col, const double* val, const double* diag, const double* rhs, double tol,
                      int32_t max_iter, void* work, size_t work_bytes, double* lambda, double* U,
                      phfem_solve_stats* stats, phfem_stream_t stream);

/* ---------------------------------------------------------------- grad (a10) -------- */
size_t phfem_grad_workspace(int64_t nE, int64_t nF, int32_t mode);

/* Adjoint gradient of a scalar J(U) given dJdU[4][nE] at the solution (U, lambda) of
 * phfem_solve: one adjoint face solve S+ Q = -C A^-1 dJdU (same system and mode), then
 * P = A^-1 (dJdU + C'Q) and, per tet,
 *   dJ/dlog kappa_T = -kappa_T P_T' K_T U_T,
 *   dJ/dX = -d/dX [P'A U - lambda'C P - P'B - Q'C U + Q'b_D]  (P, U, lambda, Q fixed).
 * Outputs: dJ_dlogkappa[nE] (may be NULL), dJ_dcoord[3][nC] (may be NULL; zeroed and
 * accumulated with atomics, the one result that is not bitwise reproducible).
 * Synchronizes.  Errors as phfem_solve (ids out of range and zero volumes are also checked
 * in the gradient pass; ENOCONV: the adjoint solve stopped above tol, and the outputs hold
 * the gradient of its last iterate); EINVAL when params.neumann is set (the gradient covers
 * Dirichlet boundaries only). */
int phfem_grad(int64_t nC, const double* coord, int64_t nE, const int32_t* tetra, int64_t nF, const int32_t* faces,
               const int32_t* tet2face, const int8_t* sigma, const int32_t* face2tet, const int32_t* nbr,
               const double* kappa, const phfem_params* p, const int32_t* rowptr, const int32_t* col,
               const double* val, const double* diag, const double* U, const double* lambda, const double* dJdU,
               int32_t mode, double tol, double inner_tol, int32_t max_iter, void* work, size_t work_bytes,
               double* dJ_dlogkappa, double* dJ_dcoord, phfem_solve_stats* stats, phfem_stream_t stream);

/* ---------------------------------------------------------------- error norms ------- */
size_t phfem_errors_workspace(int64_t nE);

/* A-priori error norms of a solution (U, lambda) of phfem_solve against an exact solution
 * u = (u_kind, u_par[4] in host memory) (Section 5: the mesh-dependent norm ||.||_Y and the h-norm of the
 * multiplier, eq. (eMnorm); the quantities of Table 4), with u_h linear on each tet:
 *   out[0] = sum_T ||grad(u - u_h)||^2_T,   out[1] = sum_T ||u - u_h||^2_T,
 *   out[2] = sum_T h sum_{F in dT \ Gamma_N} ||kappa_T grad u . nu_F - lambda_F||^2_F,
 * nu_F the outward normal of the face's owner tet (lambda's orientation), Gamma_N the faces
 * flagged in params.neumann (if set).  ||u - u_h||_Y = sqrt(out[0] + out[1] / h^2),
 * ||kappa grad u - lambda||_h = sqrt(out[2]).  h > 0 is the caller's mesh size.
 * Quadrature: collapsed Gauss-Legendre products with nq in [1, 12] points per direction (exact
 * to degree 2 nq - 3 on tets and 2 nq - 2 on faces).  Inputs on the device as for
 * phfem_solve (nF faces); out[3] is HOST memory, written only on success.  The sums are
 * reduced in a fixed order (deterministic).  Synchronizes.  Errors: EINVAL (also for a vertex
 * or face id out of range, found on the device), EWORKSPACE. */
int phfem_errors(int64_t nC, const double* coord, int64_t nE, const int32_t* tetra, int64_t nF, const int32_t* tet2face,
                 const int8_t* sigma, const double* kappa, const phfem_params* p, const double* U,
                 const double* lambda, int32_t u_kind, const double* u_par, double h, int32_t nq, void* work,
                 size_t work_bytes, double* out, phfem_stream_t stream);

/* For callers that cannot allocate (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc and caller workspaces): phfem_errors without the
 * workspace argument.  Its scratch (per-block partial sums, totals, the index-check word;
 * 2 MiB) is a fixed device array of the library, one copy per GPU the library runs on,
 * held until the process ends; the call allocates nothing.  Same inputs, outputs, kernels
 * and results (bit for bit) as phfem_errors.  Limit: nE <= PHFEM_ERRORS_NOALLOC_MAX_TETS
 * (EINVAL beyond it).  Calls that overlap in time on one GPU share that array and race:
 * serialize them (one stream, or host-side ordering).  Synchronizes. */
#define PHFEM_ERRORS_NOALLOC_MAX_TETS 22364160
int phfem_errors_noalloc(int64_t nC, const double* coord, int64_t nE, const int32_t* tetra, int64_t nF,
                         const int32_t* tet2face, const int8_t* sigma, const double* kappa, const phfem_params* p,
                         const double* U, const double* lambda, int32_t u_kind, const double* u_par, double h,
                         int32_t nq, double* out, phfem_stream_t stream);

/* ---------------------------------------------------------------- profiling --------- */
/* When enabled, every kernel launch of the library is bracketed by HIP events on its
 * stream.  phfem_profile_query synchronizes those events and returns, for the kernel
 * named `name`, the number of launches, their summed duration (ms) and their summed
 * algorithmic bytes (each input read once, each output written once; 0 for kernels
 * without a count) since the last reset (total_bytes may be NULL).  phfem_profile_names
 * writes the names seen, comma separated.  Host-side bookkeeping only; not thread safe
 * against concurrent launches from several threads. */
void phfem_profile_enable(int32_t on);
/* Streams of known size that scale the HBM traffic counters of a profiler run (reads counted by
 * FETCH_SIZE, writes by WRITE_SIZE): op 0 reads n doubles of src (16-byte loads) and writes one
 * partial sum per workgroup to dst[0..4095]; op 1 writes n doubles to dst; op 2 copies n
 * doubles from src to dst; op 3 gathers n 32-byte records of src[m][4] (m a power of two) at
 * the positions (j * 2654435761) mod m, partial sums to dst[0..4095].  n even for ops 0-2;
 * src 32-byte and dst 16-byte aligned.  Asynchronous.  Errors: EINVAL. */
int phfem_profile_stream(int32_t op, const double* src, double* dst, int64_t n, int64_t m, phfem_stream_t stream);
void phfem_profile_reset(void);
int phfem_profile_query(const char* name, int64_t* launches, double* total_ms, double* total_bytes);
int phfem_profile_names(char* buf, size_t buf_bytes);

#ifdef __cplusplus
}
#endif
#endif /* PHFEM_H */
