/*
 * fem.h -- C ABI of the MI355X cell-wise matrix-free Q_p Laplacian library.
 *
 * The library keeps continuous high-order finite-element fields in redundant
 * cell-wise storage (every hexahedral cell owns all (p+1)^3 of its nodal
 * values; Section 2.2 of the paper) and provides, on that storage:
 *
 *   fe_apply       the local Laplace operator A: V_cell -> V_cell^*
 *                  (Eq. "Laplace operator" of Section 2.3; Section 3.1),
 *   fe_mass_apply  the local mass operator (Eq. "mass operator", Section 2.3),
 *   fem_dss        direct stiffness summation S = G G^T (Section 3.3) by the
 *                  dimensionally-split cascade of Section 4.1,
 *   patch_inverse  one additive Schwarz application over 2x2x2-cell vertex
 *                  patches, each patch operator inverted by fast
 *                  diagonalisation (the overlapping Schwarz patch smoothers of
 *                  the Remark "Beyond DSS", Section 3.2),
 *   smoother_step  damped Richardson sweeps on that Schwarz operator,
 *   pcg_solve      the primal-dual (flexible) preconditioned CG of the
 *                  Algorithm "Communication-Free (F)PCG" (Section 3.2),
 * plus batched launches over many independent problems and a continuous-
 * batching solve server.
 *
 * Conventions shared by every call
 * --------------------------------
 * Mesh.    A box [0,Lx]x[0,Ly]x[0,Lz] split into n[0] x n[1] x n[2]
 *          axis-aligned cells with per-direction widths.  Q_p Lagrange
 *          elements on Gauss-Lobatto-Legendre nodes, (p+1)-point Gauss
 *          quadrature (exact for these operators on boxes).
 * Global.  Global node (I,J,K), 0 <= I <= n[0] p, is numbered
 *          g = I + (n[0]p+1) (J + (n[1]p+1) K).  Cell (i,j,k) is numbered
 *          e = i + n[0] (j + n[1] k); its local node (a,b,c) (a along x) is
 *          l = a + (p+1)(b + (p+1) c) and sits at global node
 *          (i p + a, j p + b, k p + c).
 * Cell-wise vectors.  fem_cell_len() elements of the precision in use
 *          (FEM_F64: double, FEM_F32: float, FEM_BF16: bfloat16 bit pattern
 *          in uint16_t, FEM_F16: IEEE binary16 bit pattern in uint16_t; the
 *          two 16-bit formats are computed in FP32 and rounded to nearest
 *          even when stored).  The order inside is private to the library; use
 *          fem_pack/fem_unpack (canonical [cell][local node] order) or
 *          fem_gather/fem_scatter/fem_extract (global order) to move data in
 *          and out.  Padding entries are kept at zero by every call.
 * Primal/dual.  A primal (continuous) cell-wise vector holds equal values in
 *          all copies of a node; a dual vector holds unassembled per-cell
 *          contributions (Section 3.1).
 * Boundary. FEM_BC_DIRICHLET imposes homogeneous Dirichlet conditions by
 *          masking: copies on the domain boundary are read as zero and
 *          written as zero (A_D = P_I A P_I).  FEM_BC_NEUMANN applies the
 *          plain operator.
 * Memory.  Every vector argument is a device pointer to caller-owned memory,
 *          256-byte aligned.  The library owns only its handle-internal
 *          workspace (geometry, patch eigen-data, temporaries).
 * Streams. Calls are asynchronous on the handle's stream unless stated.
 *          Calls on one handle must not overlap (they share its workspace).
 * Errors.  Every call returns fem_status; fem_last_error() returns a
 *          thread-local message for the most recent failure.  No C++
 *          exception crosses this ABI.
 */
#ifndef FEM_MI355X_H
#define FEM_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum fem_status {
    FEM_OK = 0,
    FEM_EINVAL = 1,       /* bad argument (degree, sizes, pointers, aliasing)  */
    FEM_ENOMEM = 2,       /* device allocation failed / request exceeds budget */
    FEM_EHIP = 3,         /* HIP runtime error (message in fem_last_error)     */
    FEM_ENOTCONV = 4,     /* pcg_solve reached maxit without converging        */
    FEM_EBREAKDOWN = 5,   /* pcg_solve: non-finite or non-positive <q,p>       */
    FEM_EAGAIN = 6,       /* server: result not ready / request queued         */
    FEM_ENOTFOUND = 7     /* server: unknown ticket                            */
} fem_status;

typedef enum fem_prec { FEM_F64 = 0, FEM_F32 = 1, FEM_BF16 = 2, FEM_F16 = 3 } fem_prec;
typedef enum fem_bc { FEM_BC_DIRICHLET = 0, FEM_BC_NEUMANN = 1 } fem_bc;
typedef enum fem_cg_variant { FEM_CG_AUTO = 0, FEM_CG_PCG = 1, FEM_CG_FCG = 2 } fem_cg_variant;
/* Preconditioners of the solver: the additive Schwarz smoother over vertex
 * patches; the two simple ones of Section 3.3, the trivial P = S
 * (Eq. "dss_operator") and Jacobi P = D_cell^{-1} S; and the two-level
 * method (smoother plus an exact coarse correction on the trilinear
 * functions of the same mesh), the multigrid family the Remark after the
 * Theorem "Equivalence of Communication-Free FCG" names (fem_two_level). */
typedef enum fem_precond {
    FEM_PC_SCHWARZ = 0, FEM_PC_DSS = 1, FEM_PC_JACOBI = 2, FEM_PC_TWO_LEVEL = 3
} fem_precond;

/* Problem description.  p in 1..7, n[d] >= 1 (>= 2 for patch_inverse to be
 * non-trivial).  widths[d]: host array of n[d] positive cell widths along
 * direction d, copied at create time; NULL means n[d] equal cells of width
 * 1/n[d]. */
typedef struct fem_desc {
    int p;
    int n[3];
    const double* widths[3];
    int bc;                  /* fem_bc */
} fem_desc;

typedef struct fem_problem fem_problem;

/* Result record of pcg_solve and of the server. */
typedef struct fem_solve_info {
    int iters;               /* iterations performed                       */
    int status;              /* fem_status of the solve                    */
    double relres;           /* ||G^T r_k||_2 / ||G^T b||_2 at exit        */
    double seconds;          /* wall time of the solve (host clock)        */
} fem_solve_info;

/* ---------------------------------------------------------------- setup */

/* Create a problem on the current HIP device.  Copies the widths, builds
 * the 1D reference matrices and the per-vertex-line fast-diagonalisation
 * data on the host, uploads them, and allocates the handle's workspace.
 * stream: a hipStream_t (NULL = default stream).
 * Errors: FEM_EINVAL (p outside 1..7, n < 1, non-positive width),
 * FEM_ENOMEM, FEM_EHIP. */
fem_status fem_problem_create(const fem_desc* desc, void* stream, fem_problem** out);
fem_status fem_problem_destroy(fem_problem* P);
fem_status fem_set_stream(fem_problem* P, void* stream);

size_t fem_cell_len(const fem_problem* P);     /* elements per cell-wise vector (with padding) */
size_t fem_global_len(const fem_problem* P);   /* (n0 p+1)(n1 p+1)(n2 p+1)                      */
size_t fem_num_cells(const fem_problem* P);
size_t fem_num_patches(const fem_problem* P);  /* (n0-1)(n1-1)(n2-1) interior vertices          */
/* Device bytes a problem's handle plus a pcg_solve with the given smoother
 * precision needs (handle workspace + solver vectors), for admission. */
size_t fem_footprint_bytes(const fem_desc* desc, int smoother_prec);
/* Bytes one element of a precision occupies (8, 4, 2). */
size_t fem_prec_bytes(int prec);

/* ----------------------------------------------------------- converters */

/* x_cell = G x_glob (primal gather).  x_glob: device double[global_len]. */
fem_status fem_gather(fem_problem* P, const double* x_glob, void* x_cell, int prec);
/* y_glob = G^T y_cell (dual assembly: sums all copies of each node). */
fem_status fem_scatter(fem_problem* P, const void* y_cell, double* y_glob, int prec);
/* u_glob[g] = the copy of node g held by the lowest-numbered cell containing
 * it (reads a primal vector back to global order). */
fem_status fem_extract(fem_problem* P, const void* u_cell, double* u_glob, int prec);
/* Canonical cell-major order [num_cells][(p+1)^3] <-> library layout. */
fem_status fem_pack(fem_problem* P, const double* canon, void* v_cell, int prec);
fem_status fem_unpack(fem_problem* P, const void* v_cell, double* canon, int prec);
/* out = G^T r / m per copy (m = number of cells sharing the node): the
 * assembled residual spread evenly over its copies, summed in FP64 and then
 * rounded to `prec`.  r: dual FP64 vector.  Use it to hand a residual to a
 * reduced-precision smoother: a converging solve's unassembled residual has
 * per-copy values that cancel under assembly, and rounding them before
 * assembly would put an absolute error floor into the smoother's input.
 * smoother_step and patch_inverse see r only through G^T r, so the result
 * is the same operator input. */
fem_status fem_distribute_assembled(fem_problem* P, const double* r, void* out, int prec);
/* dst = src converted between precisions (round to nearest even). */
fem_status fem_convert(fem_problem* P, const void* src, int src_prec, void* dst, int dst_prec);

/* ------------------------------------------------------------ operators */

/* y = A x: per-cell sum-factorised Laplace apply (Eq. "Laplace operator",
 * Section 2.3) with per-cell coefficients hy hz/hx, hx hz/hy, hx hy/hz.
 * x primal (read), y dual (written).  x == y is FEM_EINVAL. */
fem_status fe_apply(fem_problem* P, const void* x_cell, void* y_cell, int prec);
/* y = M x: per-cell sum-factorised mass apply (Eq. "mass operator").  With
 * Dirichlet conditions x is read in full and y's boundary copies are zero
 * (P_I M), so fe_mass_apply(G f) is the load vector of nodal values f. */
fem_status fe_mass_apply(fem_problem* P, const void* x_cell, void* y_cell, int prec);
/* s = G G^T v: every copy receives the sum of all copies of its node
 * (Section 3.3), computed by three axis passes z, y, x (Algorithm
 * "Dimensionally-Split Structured Summation").  s may equal v (in place). */
fem_status fem_dss(fem_problem* P, const void* v, void* s, int prec);
/* One in-place axis pass of that cascade (axis 0 = x, 1 = y, 2 = z): each
 * pair of coincident face copies across interfaces normal to the axis is
 * replaced by its sum on both sides. */
fem_status fem_dss_axis(fem_problem* P, void* v, int axis, int prec);
/* z = sum_P R_P^T A_P^{-1} R_P G^T r: one additive Schwarz application over
 * all interior-vertex patches.  r dual (read), z primal (written), zero on
 * the Dirichlet boundary, every copy of a node bitwise equal.  r == z is
 * FEM_EINVAL. */
fem_status patch_inverse(fem_problem* P, const void* r_cell, void* z_cell, int prec);
/* z = Richardson(r): z_0 = 0, z_{j+1} = z_j + omega P_AS (r - A z_j), for
 * `sweeps` sweeps (>= 1).  r dual, z primal, both in `prec`. */
fem_status smoother_step(fem_problem* P, const void* r_cell, void* z_cell, int prec,
                         int sweeps, double omega);

/* z = B r, one application of the two-level preconditioner (the multigrid
 * V-cycle of the Remark after the Theorem "Equivalence of Communication-Free
 * FCG" with two levels, the coarse one solved exactly): z_0 = 0, `sweeps`
 * damped Richardson sweeps z <- z + omega P_AS (r - A z), the coarse
 * correction z <- z + P_0 A_0^{-1} P_0^T (r - A z), `sweeps` more sweeps.
 * The coarse space is the trilinear (Q1) functions on the interior vertices
 * of the same mesh; P_0 interpolates them at the nodes of every cell, A_0 is
 * the Q1 Laplacian of the mesh (the Galerkin operator of the nested spaces)
 * and its inverse is applied in FP64 by fast diagonalisation.  r dual, z
 * primal (continuous bit for bit), both in `prec`; the input is used only
 * through G^T r.  r == z is FEM_EINVAL; omega in (0, 1/4) keeps the
 * smoother convergent (the Schwarz operator's spectrum lies in (0, 8]). */
fem_status fem_two_level(fem_problem* P, const void* r_cell, void* z_cell, int prec, int sweeps, double omega);

/* ------------------------------------------------------------ reductions */

/* *result = <a, b> over all cell-wise entries, accumulated in FP64 with a
 * fixed reduction order.  Synchronises the stream.  prec_a/prec_b may
 * differ. */
fem_status fem_dot(fem_problem* P, const void* a, int prec_a, const void* b, int prec_b,
                   double* result);
/* *result = ||G^T r||_2 (assembled l2 norm of a dual vector).  Synchronises. */
fem_status fem_assembled_norm(fem_problem* P, const void* r, int prec, double* result);

/* --------------------------------------------------------------- solver */

/* Solve A u = b with the (F)PCG of the paper's Algorithm "Communication-Free
 * (F)PCG", preconditioned by smoother_step(sweeps, omega) in
 * `smoother_prec`.  b: dual FP64 cell-wise vector (read); u: primal FP64
 * cell-wise vector, initial guess in and solution out.  All vectors, pairings
 * and scalars stay on the device in FP64; the stopping test is
 * ||G^T r_k||_2 <= rtol ||G^T b||_2.  variant FEM_CG_AUTO uses PCG for an
 * FP64 smoother and FCG otherwise.  With an FP16 smoother the residual
 * copies handed to the smoother are scaled by a power of two that brings
 * the root-mean-square entry of G^T r_k into [2^-10, 2^-9) (late
 * residuals lie far below FP16's normal range, and the patch inverse
 * multiplies them by up to about 10^3 before z is stored in FP16);
 * the direction z then carries the same factor, which the step lengths of
 * (F)PCG absorb, so the iterates are those of the unscaled method up to
 * rounding.  Synchronises the stream at exit.  Returns FEM_ENOTCONV at
 * maxit, FEM_EBREAKDOWN on a non-finite ||G^T b|| (before iterating) or a
 * non-finite or non-positive <q,p>; info (may be NULL) is filled in every
 * case. */
fem_status pcg_solve(fem_problem* P, const double* b_cell, double* u_cell, double rtol,
                     int maxit, int smoother_prec, int sweeps, double omega, int variant,
                     fem_solve_info* info);

/* pcg_solve with a choice of preconditioner (fem_precond).  FEM_PC_SCHWARZ
 * is pcg_solve itself.  FEM_PC_DSS and FEM_PC_JACOBI apply z = S r or
 * z = D_cell^{-1} S r (Section 3.3: the assembled residual on every copy,
 * divided for Jacobi by the diagonal of the assembled operator, zero on a
 * Dirichlet boundary) in one pass that also yields ||G^T r||, in precision
 * smoother_prec; sweeps and omega are then unused (sweeps must still be >= 1).
 * FEM_PC_TWO_LEVEL applies fem_two_level(sweeps, omega) in smoother_prec.
 * FEM_CG_AUTO picks PCG for FP64 and for the static simple preconditioners,
 * FCG otherwise.  Same buffers,
 * workspace, synchronisation and errors as pcg_solve. */
fem_status pcg_solve_pc(fem_problem* P, const double* b_cell, double* u_cell, double rtol, int maxit,
                        int precond, int smoother_prec, int sweeps, double omega, int variant,
                        fem_solve_info* info);
/* One application of a simple preconditioner of Section 3.3: z = S r
 * (precond FEM_PC_DSS) or z = D_cell^{-1} S r (FEM_PC_JACOBI), where D_cell
 * holds on every copy of a node the diagonal of the assembled operator
 * (the identity G D_CG^{-1} = D_cell^{-1} G after Eq. "dss_operator").
 * r: dual FP64 cell-wise vector (read); z: primal cell-wise vector in `prec`
 * (written), every copy of a node bitwise equal, zero on a Dirichlet
 * boundary.  r == z is FEM_EINVAL. */
fem_status fem_precond_apply(fem_problem* P, int precond, const void* r_cell, void* z_cell, int prec);

/* pcg_solve_pc for callers that cannot allocate device memory (code under
 * stream capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same solve, bit for bit, with the solver's own vectors (r, p, q in FP64,
 * z and the smoother's residual copy in smoother_prec, 24 + 2 x
 * fem_prec_bytes(smoother_prec) bytes per cell-wise entry) taken from one
 * device array of fem_noalloc_scratch_bytes() bytes (64 MiB) that the
 * library holds on every device it runs on until the process ends, instead
 * of the handle's lazily allocated workspace.  It calls no allocator; the
 * problem handle (created beforehand) supplies everything else.  Call it
 * with the problem's device current.  Calls on one device share that array:
 * calls that overlap on one GPU (from several threads or streams) race and
 * must be serialised by the caller; the array keeps the last call's contents
 * and every vector is written before it is read.  FEM_EINVAL when the
 * vectors exceed the array (the message gives both sizes) or the current
 * device is not the problem's; otherwise as pcg_solve_pc. */
fem_status pcg_solve_noalloc(fem_problem* P, const double* b_cell, double* u_cell, double rtol, int maxit,
                             int precond, int smoother_prec, int sweeps, double omega, int variant,
                             fem_solve_info* info);
size_t fem_noalloc_scratch_bytes(void);

/* ------------------------------------------------------- batched launches */

typedef struct fem_batch fem_batch;

/* A batch of independent problems sharing one stream.  Batched calls run
 * every kernel phase either as one launch per degree present (each covering
 * all problems of that degree), or, when the degrees are two or three of
 * {2, 3, 7}, as one mixed-degree launch per phase: a grid whose workgroups
 * each run one item (one workgroup's work of that degree's own kernel) of
 * one degree.  Mixed launches use the default kernel shapes, so every
 * problem's result equals its single-problem call bit for bit; they are the
 * default until fem_batch_autotune decides (see there). */
fem_status fem_batch_create(int count, const fem_desc* descs, void* stream, fem_batch** out);
fem_status fem_batch_destroy(fem_batch* B);
/* Borrow problem i of the batch (owned by the batch) for per-problem calls. */
fem_status fem_batch_problem(fem_batch* B, int i, fem_problem** out);
/* y[i] = A x[i] for every problem i; x, y: host arrays of `count` device
 * pointers, each a cell-wise vector of that problem in `prec`. */
fem_status fem_batch_apply(fem_batch* B, void* const* x, void* const* y, int prec);
/* z[i] = P_AS r[i] for every problem i. */
fem_status fem_batch_patch_inverse(fem_batch* B, void* const* r, void* const* z, int prec);
/* Tile-shape autotuner: for each degree present in the batch, time the
 * candidate kernel shapes on the batch's own problems (apply: register
 * (p <= 3) or plane-streamed (p >= 4; for p = 7 in FP64 the matrix-core
 * kernel) kernel, or the LDS line kernel, and for p = 7 also the
 * plane-streamed kernel, each x two persistent grid caps; patch inverse for p <= 3: two launches through
 * the patch buffer, fused sweep from the cell copies, fused sweep from the
 * assembled residual, or solves with the in-tile x-combine; for p >= 4: MFMA
 * or line patch solves; each x two grid caps) and keep the fastest for later
 * batched calls.  choice (may be
 * NULL): int[14], choice[2(p-1)] = apply candidate index, choice[2(p-1)+1]
 * = patch-inverse candidate index of degree p, candidates in the order
 * listed with the grid cap varying fastest (untouched for absent degrees).
 * Where mixed-degree launches are possible it then times a whole pass
 * (apply + patch inverse) with the tuned per-degree launches and with the
 * mixed launches and keeps the faster (fem_batch_mixed reports which).
 * Synchronises the stream; allocates and frees its own scratch vectors. */
fem_status fem_batch_autotune(fem_batch* B, int prec, int* choice);
/* mixed = 1: mixed-degree launches where the batch's degrees allow them;
 * 0: one launch per degree (with the autotuned shapes). */
fem_status fem_batch_set_mixed(fem_batch* B, int mixed);
/* 1 if the batch's calls currently run as mixed-degree launches. */
int fem_batch_mixed(const fem_batch* B);

/* ------------------------------------------------- multi-block meshes */

/* Direct stiffness summation on a multi-block mesh (Section 4.2, Algorithm
 * "Unstructured Inter-Block Summation"): blocks of n[0] x n[1] x n[2] cells
 * of degree p, each in its own local axes, glued along whole block faces in
 * any relative orientation (rotations and reflections), so that a block
 * edge or corner may be shared by any number of blocks.
 *
 * fem_mb_create: block_n = int[3 * nblocks] (cells per local direction),
 * corners = int[8 * nblocks] vertex ids of each block's corners in local
 * order cx + 2 cy + 4 cz (ids only identify shared corners; no coordinates
 * are needed).  Two faces with the same four corner ids are glued; their
 * cell counts along matching directions must agree (FEM_EINVAL otherwise,
 * and for a face named by more than two blocks).  The plan derives each
 * glued face's orientation bits and the sharing lists of the nodes on cell
 * edges and corners of the inter-block skeleton (one representative copy per
 * block) on the host, uploads them and owns them.
 * The cell-wise vector of the mesh is the blocks' cell-wise vectors one
 * after another, block b starting at element fem_mb_block_offset(b), each in
 * the library's layout; fem_mb_pack/fem_mb_unpack convert from/to canonical
 * order (blocks in order, [cell][local node] within each). */
typedef struct fem_mb_plan fem_mb_plan;
fem_status fem_mb_create(int p, int nblocks, const int* block_n, const int* corners, void* stream,
                         fem_mb_plan** out);
fem_status fem_mb_destroy(fem_mb_plan* M);
size_t fem_mb_cell_len(const fem_mb_plan* M);
size_t fem_mb_block_offset(const fem_mb_plan* M, int block);
fem_status fem_mb_pack(fem_mb_plan* M, const double* canon, void* v_cell, int prec);
fem_status fem_mb_unpack(fem_mb_plan* M, const void* v_cell, double* canon, int prec);
/* v <- S v in place, S = G G^T of the multi-block mesh: stage 1 (stages & 1)
 * the structured cascade inside every block (three axis passes per block),
 * stage 2 (stages & 2) the inter-block skeleton in three launches on
 * disjoint copies: cell-face interiors (one pairwise exchange per node, the
 * index on the far side computed from the face orientation bits), cell-edge
 * interiors and cell corners (one representative per block summed, the sum
 * written to every copy).  stages = 3 is the whole summation; stage 2
 * alone assumes stage 1 has run.  Asynchronous on the plan's stream. */
fem_status fem_mb_dss(fem_mb_plan* M, void* v_cell, int prec, int stages);
/* out[0..n): glued faces, face-pass threads, line entities, widest line
 * sharing list, vertex entities, widest vertex sharing list. */
fem_status fem_mb_stats(const fem_mb_plan* M, int* out, int n);

/* ------------------------------------------------------- layout study */

/* The storage block size B of the blocked element-fastest layout (Section
 * 5.1) swept over powers of two, for the study of Section 6.1 ("Layout
 * study", Figure "Block-size sweep"): cell e's local node l sits at
 * (e / B) (p+1)^3 B + l B + e % B (the library's own vectors use B = 64).
 * FP64 device vectors, a uniform mesh of the unit cube with n[3] cells,
 * degrees 2..5, B in {1, 2, ..., 128}; FEM_EINVAL otherwise.  All
 * asynchronous on `stream`.
 * fem_layout_len: elements of such a vector (whole blocks).
 * fem_layout_pack: canonical [cell][local node] (ncells (p+1)^3 values) ->
 *   layout B (padding zeroed), or back when unpack != 0.
 * fem_layout_mass: y = M x per cell, the volumetric mass operator (Eq. "mass
 *   operator", no boundary conditions), `tile` = 16 or 32 cells staged in
 *   LDS per workgroup tile (the launch shape of the sweep).
 * fem_layout_dss: v <- G G^T v in place by the three structured axis passes
 *   (Algorithm "Dimensionally-Split Structured Summation"). */
size_t fem_layout_len(int p, const int* n, int B);
fem_status fem_layout_pack(int p, const int* n, int B, const double* src, double* dst, int unpack, void* stream);
fem_status fem_layout_mass(int p, const int* n, int B, int tile, const double* x, double* y, void* stream);
fem_status fem_layout_dss(int p, const int* n, int B, double* v, void* stream);

/* ---------------------------------------------------- solve server */

typedef struct fem_server fem_server;

/* A continuous-batching solve server on the current device.  hbm_budget:
 * bytes of device memory its active solves may hold (allocated once, as the
 * arena the solves are carved from); max_active: slot count.
 * smoother_prec/sweeps/omega: smoother of every solve.  Kernels run on
 * `stream`; the server also creates a stream of its own (default priority)
 * for request uploads and solution downloads, ordered by events.
 * Threads: one host thread drives fem_server_step; fem_server_submit,
 * fem_server_poll, fem_server_finished, fem_server_memory and
 * fem_server_stats may be called concurrently from other threads (they take
 * the server's lock); create and destroy must not overlap any other call. */
fem_status fem_server_create(size_t hbm_budget, int max_active, int smoother_prec, int sweeps,
                             double omega, void* stream, fem_server** out);
/* fem_server_create with a choice of preconditioner for every solve:
 * FEM_PC_SCHWARZ (the smoother, as fem_server_create) or FEM_PC_TWO_LEVEL
 * (fem_two_level with `sweeps` pre- and post-sweeps, batched over the
 * active solves like every other phase).  Other values are FEM_EINVAL. */
fem_status fem_server_create_pc(size_t hbm_budget, int max_active, int precond, int smoother_prec, int sweeps,
                                double omega, void* stream, fem_server** out);
fem_status fem_server_destroy(fem_server* S);
/* Queue a solve of A u = P_I M f (f: host double[global_len] nodal source
 * values, copied).  Returns FEM_ENOMEM if the request can never fit the
 * budget, FEM_OK otherwise (it is admitted when memory and a slot free up). */
fem_status fem_server_submit(fem_server* S, const fem_desc* desc, const double* f_glob,
                             double rtol, int maxit, uint64_t* ticket);
/* Admit queued requests that fit, then advance every active solve by at
 * least one iteration (a solve smaller than the largest active one takes up
 * to 8, as many as its size fits into the largest one's), every kernel phase
 * as one launch over all active solves (mixed-degree launches, see
 * fem_batch_create, or one launch per degree), retire converged ones.
 * n_active/n_queued/n_done (may be NULL) report the counts after the step. */
fem_status fem_server_step(fem_server* S, int* n_active, int* n_queued, int* n_done);
/* mixed = 1 (the default): the step's degree-dependent kernels run as
 * mixed-degree launches where the active degrees allow; 0: one launch per
 * degree.  Results are the same either way.  May be called from any thread;
 * takes effect at the next step. */
fem_status fem_server_set_mixed(fem_server* S, int mixed);
/* FEM_OK and the solution (global order, host double[global_len]; may be
 * NULL) if the ticket's solve has finished; FEM_EAGAIN if not yet;
 * FEM_ENOTFOUND for an unknown or already collected ticket. */
fem_status fem_server_poll(fem_server* S, uint64_t ticket, double* u_glob, fem_solve_info* info);
/* Device bytes currently held by admitted solves, and the high-water mark. */
fem_status fem_server_memory(fem_server* S, size_t* in_use, size_t* high_water);
/* Tickets whose solves have finished and are not collected yet, in
 * ascending order: writes at most max_tickets into out (may be NULL to
 * count) and returns how many there are. */
int fem_server_finished(fem_server* S, uint64_t* out, int max_tickets);
/* Host-side accounting of fem_server_step (for tuning): out[0..n) receives,
 * as far as n reaches, the seconds spent in admission, in queuing the
 * iteration's launches, waiting for the solves' scalars, handing finished
 * solutions over, starting retirements, and the number of steps. */
fem_status fem_server_stats(fem_server* S, double* out, int n);

/* ------------------------------------------------------- host utilities */

/* Host-only (no device use): the 1D reference mass and stiffness matrices
 * of degree p on [0,1] (row-major (p+1)x(p+1)), and the fast-diagonalisation
 * data of the 1D patch operator of two cells of widths h0, h1 restricted to
 * the 2p-1 interior nodes: S (row-major (2p-1)x(2p-1), columns are
 * eigenvectors) and lambda (2p-1) with S^T M S = I, S^T K S = diag(lambda). */
fem_status fem_host_1d_matrices(int p, double* mass, double* stiff);
/* Host-only: the p+1 Gauss-Lobatto-Legendre nodes of [0,1] the element uses
 * (ascending), e.g. to place nodal source values. */
fem_status fem_host_gll_nodes(int p, double* nodes);
fem_status fem_host_fd_1d(int p, double h0, double h1, double* S, double* lambda);

/* Process-wide kernel-variant switches (for comparisons; the batch
 * autotuner picks per batch instead).  FEM_OPT_PI_FUSED: patch_inverse for
 * p <= 3 as 0 two launches through the patch buffer, 1 one fused sweep
 * summing the residual's cell copies on chip, 2 assembly plus one fused
 * sweep reading the assembled residual, 3 assembly plus solves that add the
 * x-overlaps of neighbouring patches in the workgroup and write one run of
 * global x-nodes per patch line (a buffer about 3/5 of the patch buffer at
 * p = 3), then a combine by global node rows, 4 the same with one wavefront
 * per tile of floor(64 / (2p-1)) patches (x and y contractions on a lane's
 * patch plane in registers, two transposes through LDS instead of four);
 * for p >= 4, 2 selects line (VALU) patch solves instead of MFMA; -1
 * (default) picks by degree and precision only (4 for p = 2, 3 for p = 3
 * in FP64, else 0).  The p <= 3 combine of the two-launch
 * form runs by global node rows (FP64, every mesh with at least 48 cells
 * along x) or by (block, node plane), with identical results;
 * FEM_OPT_COMBINE_PER_CELL = 1 makes it use one wavefront per 64-cell block
 * (all node planes) instead.  For p >= 4 the combine runs by global node
 * rows in FP64 and per (64-cell block, node plane) otherwise, with
 * identical results; FEM_OPT_COMBINE_PER_CELL = 1 selects the latter and 2
 * the former for every precision (0, the default, picks by precision).  FEM_OPT_RESTRICT_FROM_CELLS = 1 makes
 * the p <= 3 patch solves sum the residual copies from the cell vector
 * instead of reading the assembled global-node array.  FEM_OPT_PI_SLAB_MB =
 * m > 0 runs the p <= 3 two-launch patch inverse of a single problem in
 * z-slabs of about m MB of patch results each (solve, then combine what is
 * complete), so the results are re-read from the Infinity Cache; 0 (default)
 * launches each phase once.  FEM_OPT_APPLY_PLANES_P7 = 1 runs the p = 7
 * FP64 Laplace and residual applies on the plane-streamed VALU kernel
 * instead of the matrix-core (MFMA) one.  Every variant gives
 * the same result up to the rounding of the summation order (bitwise
 * continuous in all cases).  Unknown options or values are FEM_EINVAL. */
typedef enum fem_option {
    FEM_OPT_PI_FUSED = 1,
    FEM_OPT_COMBINE_PER_CELL = 2,
    FEM_OPT_RESTRICT_FROM_CELLS = 3,
    FEM_OPT_PI_SLAB_MB = 4,
    FEM_OPT_APPLY_PLANES_P7 = 5
} fem_option;
fem_status fem_set_option(int option, int value);

/* Launch trace (for measurement).  fem_trace_enable(1) starts recording:
 * every kernel launch of the library's hot operations (apply, the patch
 * inverse phases, DSS, reductions, CG updates) is bracketed by a pair of HIP
 * events on the stream it is launched on; fem_trace_enable(0) stops, and
 * either call discards what was recorded.  fem_trace_read waits for the
 * recorded events, aggregates them per (label, p, precision) into out[0..),
 * writing at most max_recs records, clears the record list and returns the
 * number of distinct records (which may exceed max_recs; out may be NULL to
 * count).  Tracing adds one event record before and after each launch;
 * calls from several host threads are serialised by a lock. */
typedef struct fem_trace_rec {
    char label[48];      /* e.g. "apply", "pi_assemble", "pi_solve", "pi_combine" */
    int p;
    int prec;            /* fem_prec of the launch (the kernel's storage type) */
    int launches;
    double total_ms;     /* summed event-to-event durations */
} fem_trace_rec;
fem_status fem_trace_enable(int on);
int fem_trace_read(fem_trace_rec* out, int max_recs);

const char* fem_last_error(void);
const char* fem_version(void);

#ifdef __cplusplus
}
#endif
#endif /* FEM_MI355X_H */
