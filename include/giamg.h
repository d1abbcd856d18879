/*
 * giamg.h -- C ABI of the MI355X (gfx950) GIAMG-PCG solver library.
 *
 * The library solves A x = b for the high-order finite-element operator
 * A = K + lambda M (stiffness plus lambda times mass) of GLL-nodal hexahedra,
 * with conjugate gradients preconditioned by one GIAMG V-cycle per
 * iteration.  The method is that of Xu, Rasouli, Kirby, Moxey and Sundar,
 * "A geometrically informed algebraic multigrid preconditioned iterative
 * approach for solving high-order finite element systems" (arXiv 2512.15121):
 *
 *   - problem statement A x = b (Section 2);
 *   - the V-cycle of Algorithm 1 with Jacobi-accelerated Chebyshev smoothing,
 *     Galerkin coarse operators R A P with R = P^T and a direct solve on the
 *     coarsest level (Section 2.1);
 *   - p-coarsening driven by the element-to-dof map l2g (Section 2.2,
 *     Algorithms 2-4; prolongation, Algorithm 7, nodal variant);
 *   - smoothed-aggregation h-coarsening below order 1 (Section 2.5);
 *   - CG preconditioned by the V-cycle, stopped on the relative residual
 *     (Section 2.1, end; Section 3.1.1).
 *
 * Conventions shared by every entry point
 *   - Return value: GIAMG_OK (0) on success, a negative GIAMG_E* code on
 *     error, GIAMG_ENOTCONV (> 0) as a warning when the iteration cap was
 *     reached.  giamg_last_error() returns a thread-local message describing
 *     the last error on the calling thread.
 *   - "host" pointers are ordinary CPU memory; "device" pointers are HIP
 *     device memory of the GPU that was current at giamg_setup.  The caller
 *     owns every array it passes; nothing is retained after a call returns.
 *   - Work is enqueued on the HIP stream given at setup.  Calls that return
 *     results to the host synchronise that stream before returning.
 *   - A handle is not thread-safe: calls on one handle must not overlap.
 *     Distinct handles are independent.
 */
#ifndef GIAMG_H
#define GIAMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ------------------------------------------------------ */
#define GIAMG_OK          0
#define GIAMG_ENOTCONV    1   /* warning: iteration cap reached; x holds the last iterate */
#define GIAMG_EINVAL     (-1) /* bad argument (sizes, indices, geometry, options) */
#define GIAMG_ENOMEM     (-2) /* device or host allocation failed; no handle is created */
#define GIAMG_EHIP       (-3) /* a HIP runtime call failed */
#define GIAMG_EBREAKDOWN (-4) /* CG breakdown: p^T A p <= 0 or a non-finite value */
#define GIAMG_ENOTSUP    (-5) /* valid input outside what the library supports */

/* ---- options ----------------------------------------------------------- */
#define GIAMG_SMOOTHER_CHEBYSHEV 0
#define GIAMG_SMOOTHER_JACOBI    1
#define GIAMG_BC_DIRICHLET       0  /* nodes on faces owned by one element are constrained */
#define GIAMG_BC_PIN             1  /* only pin_node is constrained (pure Neumann + pin) */
#define GIAMG_PREC_FP64          0  /* everything in double precision, standard PCG */
#define GIAMG_PREC_MIXED         1  /* FP32 V-cycle (coarsest in FP64) inside FP64 flexible CG */
#define GIAMG_BATCH_AUTO  0   /* batch_kernel: fastest shape, timed per operator */
#define GIAMG_BATCH_LANES 1   /* 8 to 64 lanes per row, each lane loads its own (column, value) */
#define GIAMG_BATCH_WAVE  2   /* one row per wavefront, (column, value) pairs shared by readlane */
#define GIAMG_BATCH_GROUP 3   /* one group of rows with identical column lists per wavefront */
#define GIAMG_PRECOND_VCYCLE     0  /* one GIAMG V-cycle per CG iteration (the method) */
#define GIAMG_PRECOND_JACOBI     1  /* the inverse diagonal: the diagonally preconditioned CG
                                       the paper compares against (Section 3.2) */
#define GIAMG_ASSEMBLY_AUTO      0  /* fine operator assembled on the device where it fits */
#define GIAMG_ASSEMBLY_DEVICE    1  /* on the device, or GIAMG_ENOTSUP */
#define GIAMG_ASSEMBLY_HOST      2  /* on the host, then copied to the device */
#define GIAMG_BASIS_NODAL        0  /* tensor Lagrange on Gauss-Lobatto-Legendre points */
#define GIAMG_BASIS_MODAL        1  /* hierarchical modal basis of the paper's appendix:
                                       1-D modes (1-a)/2, (1+a)/2, then bubbles
                                       (1-a)/2 (1+a)/2 P^{1,1}_{n-2}(a); p-transfers
                                       inject the low modes (Algorithm 7) */

typedef struct giamg_opts {
    int32_t  smoother;     /* GIAMG_SMOOTHER_*; default Chebyshev */
    int32_t  degree;       /* Chebyshev degree or Jacobi sweeps, per pre- and post-smoothing; default 2 */
    double   omega;        /* Jacobi weight; default 2/3 */
    int32_t  coarse_max;   /* h-coarsen while a level has more rows than this; default 2000 */
    int32_t  max_levels;   /* hierarchy depth cap, fine level included; default 10 */
    int32_t  bc;           /* GIAMG_BC_*; default Dirichlet */
    int64_t  pin_node;     /* constrained node for GIAMG_BC_PIN; default 0 */
    int32_t  precision;    /* GIAMG_PREC_*; default FP64 */
    int32_t  maxit;        /* CG iteration cap; default 500 */
    uint64_t agg_seed;     /* SplitMix64 seed of the aggregation priorities; default 0 */
    int32_t  power_iters;  /* power iterations for lambda_max(D^-1 A); default 20 */
    double   cheb_lo;      /* Chebyshev interval [cheb_lo, cheb_hi] * lambda_max estimate; */
    double   cheb_hi;      /* defaults 0.1 and 1.1 */
    int32_t  direct_gathers; /* 1: products gather the vector straight from memory instead of
                                staging each block's columns in LDS first (same results, bit
                                for bit; 2 bytes less device memory per nonzero); default 0 */
    int32_t  graph_launch; /* 1: one CG iteration is captured as a HIP graph at the handle's
                              first solve and replayed (same kernels, same results, bit for
                              bit; less host work per iteration); default 0: the host launches
                              every kernel, which measured slightly faster on the device */
    int32_t  basis;        /* GIAMG_BASIS_*; default nodal */
    int32_t  schedule[8];  /* coarse p-orders after p, decreasing, zero-terminated (e.g.
                              {4,3,2,1} for p = 5: the by-one schedule); all zero (the
                              default): q = p / (smallest prime factor of p) down to 1.
                              A nodal step q < p that does not divide p numbers each
                              coarse node by the fine node at the nearest lattice
                              position and interpolates from the order-q GLL points */
    int32_t  batch_kernel; /* GIAMG_BATCH_*: kernel shape of the block products in
                              giamg_solve_batch.  AUTO (the default) times every shape on
                              an operator's first batched product and keeps the fastest;
                              LANES, WAVE and GROUP force one.  All give the same results,
                              bit for bit */
    int32_t  row_groups;   /* 1: an operator whose rows share column lists in groups (in
                              a high-order mesh the interior, face and edge nodes of an
                              element, face or edge) is multiplied in the grouped form:
                              one list of 16-bit LDS slots per group of up to 8 rows,
                              values reordered into per-block planes, the row sums in the
                              order of the CSR form (same rows, bit for bit; the block
                              partial sums of CG dot products add the rows in another
                              order).  Built where it removes at least a fifth of the
                              slots; needs direct_gathers = 0.  Default 0 (CSR form
                              only): the grouped form moves fewer bytes but measured
                              slower on gfx950 */
    int32_t  pad;
    int64_t  lean_max_nnz; /* operators with at most this many nonzeros (and no row longer
                              than 8192) are multiplied by a kernel that reads each row
                              straight from memory: a shorter chain of dependent loads
                              than the blocked, staged form, for the small coarse levels
                              (same rows, bit for bit; CG dot partials over other
                              blocks).  0: never.  Default 2000000 */
    int32_t  keep_boundary; /* 1: the coarse p-levels keep the constrained nodes (the fine
                              identity rows enter the Galerkin products as P_B^T P_B): the
                              reading under which 2^3 elements at p = 8 give the coarsest
                              level of Table 1, 27 rows / 343 nonzeros.  Default 0: coarse
                              levels hold the free nodes only */
    int32_t  pad2;
    double   theta;        /* strength threshold of the smoothed-aggregation graph (Section
                              2.5): j is a strong neighbour of i when |a_ij| >= theta
                              sqrt(|a_ii a_jj|), an edge found in either direction kept in
                              both; MIS-2 roots and aggregates are taken on that graph, the
                              SPAI-0 smoothing of the tentative prolongation uses all of A.
                              In [0, 1]; default 0: every stored off-diagonal entry */
    int32_t  preconditioner; /* GIAMG_PRECOND_*; default the V-cycle.  JACOBI builds the fine
                              level only (no coarse levels) and needs precision FP64;
                              giamg_solve and giamg_solve_noalloc only (batched solves,
                              sessions and the V-cycle steps of giamg_apply return
                              GIAMG_ENOTSUP) */
    int32_t  assembly;     /* GIAMG_ASSEMBLY_*: where the fine operator A = K + lambda M
                              (Section 3.1's element integrals) and the p-transfer
                              operators P, R = P^T (Algorithms 2-4, 7) are built.  AUTO
                              (the default): each on the device when its rows fit the
                              kernels' LDS lists (p <= 9 on hexahedral meshes with at
                              most 8 elements per node), else on the host; DEVICE: on
                              the device or GIAMG_ENOTSUP; HOST: on the host (C++
                              threads), then copied.  Same patterns; P and R bit for bit,
                              A's element integrals are contracted in another order, so
                              its values agree to rounding */
} giamg_opts;

/* Fill *opts with the defaults listed above. */
void giamg_default_opts(giamg_opts* opts);

/*
 * giamg_set_allocator -- route the library's device memory through the
 * caller's allocator (e.g. the caching allocator of a framework that owns
 * the device memory of the process).
 *
 * alloc(bytes, stream, ctx) returns device memory of at least `bytes` bytes
 * (256-byte aligned) or NULL; `stream` is the hipStream_t of the handle
 * whose call allocates (NULL = the null stream).  release(ptr, ctx) returns
 * a block; the library first synchronises the block's stream, so a block
 * comes back only when no work of the library on that stream uses it.  Both
 * may be called from the library's own threads (the server's loop and
 * setup worker).  alloc == NULL restores hipMalloc / hipFree.  The
 * registration is process-wide and applies to allocations made after it;
 * every block is released through the allocator it came from.  Returns
 * GIAMG_OK, or GIAMG_EINVAL when exactly one of alloc and release is NULL.
 */
typedef void* (*giamg_alloc_fn)(size_t bytes, void* stream, void* ctx);
typedef void (*giamg_release_fn)(void* ptr, void* ctx);
int giamg_set_allocator(giamg_alloc_fn alloc, giamg_release_fn release, void* ctx);

typedef struct giamg_s* giamg_handle;   /* opaque, owned by the library */

typedef struct giamg_info {
    int32_t iters;         /* CG iterations performed (A p products) */
    int32_t status;        /* return code of the solve for this right-hand side */
    double  relres;        /* ||r_k|| / ||b|| of the recursively updated residual at exit */
    double  true_relres;   /* ||b - A x|| / ||b|| recomputed at exit, FP64 */
    double  solve_ms;      /* GPU time of the whole solve, HIP events on the handle's stream */
    double  bytes;         /* algorithmic HBM bytes of every kernel the solve launched: each
                              CSR operator, gathered vector and row-local vector counted once
                              per launch */
} giamg_info;

/*
 * giamg_setup -- build the hierarchy for A = K + lambda M.
 *
 * coords   host, double [n_nodes][3]: node coordinates.  Only the eight corner
 *          dofs of each element are read: an element is the trilinear image
 *          of its corners (local (i,j,k) in {0,p}^3 for the nodal basis, in
 *          {0,1}^3 -- the vertex modes -- for the modal basis).
 * l2g      host, int32 [n_elem][(p+1)^3]: the element-to-dof map of
 *          Section 2.2.  Column (p+1)^2 i + (p+1) j + k holds the dof with
 *          basis index i along the first, j along the second and k along the
 *          third reference direction (the tensor ordering of the paper's
 *          appendix; modal index 0 and 1 are the vertex modes at -1 and +1,
 *          2..p the bubbles).  Shared modal dofs must have the same
 *          orientation in every element that holds them.  Every dof must
 *          belong to at least one element.
 * p        order, 1 <= p <= 10.   lambda >= 0 (lambda = 0 needs at least one
 *          constrained node).
 * opts     NULL for defaults.
 * stream   hipStream_t for all work of this handle (NULL = default stream); it
 *          must stay valid until giamg_free.
 * out      receives the handle; left untouched on error.
 *
 * Discretisation: tensor Lagrange basis on Gauss-Lobatto-Legendre points
 * (or the modal basis, opts->basis), Gauss-Legendre quadrature with p+2
 * points per direction.  Constrained
 * nodes get identity rows and columns.  Coarse orders follow opts->schedule,
 * by default q = p / (smallest prime factor of p) down to 1; coarse levels
 * hold free nodes only.  Errors: GIAMG_EINVAL, GIAMG_ENOMEM, GIAMG_EHIP, GIAMG_ENOTSUP.
 */
int giamg_setup(const double* coords, int64_t n_nodes,
                const int32_t* l2g, int64_t n_elem, int32_t p,
                double lambda, const giamg_opts* opts, void* stream,
                giamg_handle* out);

/* Release every resource of the handle (NULL is ignored).  Free the
 * handle's sessions (giamg_session_free) first: they use its hierarchy. */
void giamg_free(giamg_handle h);

/*
 * giamg_solve -- GIAMG-preconditioned CG (Section 2.1) to ||r||/||b|| < tol.
 *
 * b        device, double [n_nodes].
 * x        device, double [n_nodes]: initial guess on entry, solution on exit.
 * info     host, may be NULL.
 * FP64 mode runs standard PCG; mixed mode runs flexible CG (Polak-Ribiere
 * beta) around an FP32 V-cycle whose coarsest solve stays FP64.
 * Returns GIAMG_OK, GIAMG_ENOTCONV (cap reached), GIAMG_EBREAKDOWN or an
 * error.  Synchronises the stream.
 */
int giamg_solve(giamg_handle h, const double* b, double* x, double tol,
                giamg_info* info);

/*
 * giamg_solve_noalloc -- giamg_solve for callers that cannot allocate device
 * memory (code under HIP graph capture elsewhere in the program, serving
 * loops, harnesses that forbid hipMalloc): the same solve, the same kernels
 * and results bit for bit, but the CG vectors, block partial sums, device
 * scalars and control block it works in come from a fixed scratch array of
 * 32 MiB per GPU inside the library instead of the handle.  The call makes no
 * device or host allocation; the hierarchy and its level vectors were
 * allocated by giamg_setup.
 *
 * Limit: 7 n_nodes doubles plus the hierarchy's partial sums must fit the
 * 32 MiB (about 590,000 nodes at p = 4); a larger problem returns GIAMG_EINVAL with
 * the sizes in giamg_last_error() and touches nothing.  graph_launch is
 * ignored (an instantiated graph would allocate).
 * Sharing: every call on one GPU uses that GPU's single scratch array, whose
 * contents persist between calls (the solve clears what must start at zero).
 * Calls that overlap on one GPU -- from two threads, or on two streams
 * without ordering -- race on it and give wrong results; serialise them.
 * Arguments, return codes and synchronisation as giamg_solve.
 */
int giamg_solve_noalloc(giamg_handle h, const double* b, double* x, double tol,
                        giamg_info* info);

/*
 * giamg_solve_batch -- k independent solves against one hierarchy.
 *
 * B, X     device, double [n_nodes][k] row-major (right-hand side j is
 *          column j); X holds initial guesses on entry.
 * infos    host, k entries, may be NULL.
 * Each column runs its own CG scalars and stops on its own; the V-cycle of
 * all active columns runs as block sparse-matrix times dense-block products
 * in the handle's precision.  Returns the worst per-column code.
 */
int giamg_solve_batch(giamg_handle h, const double* B, double* X, int32_t k,
                      double tol, giamg_info* infos);

/* ---- profiling ------------------------------------------------------------
 * Phase breakdown of the solve in the categories of the paper's detailed
 * analysis (Section 3.2: first-level smoothing, smoothing, residual,
 * restriction and prolongation, V-cycle, CG matrix-vector product, CG dot
 * products, whole PCG iterations), measured with HIP events on the handle's
 * stream around each phase of every solve while profiling is on.  Phases
 * nest (a V-cycle contains its smoothing, residuals and transfers), so the
 * totals overlap.  GIAMG_PHASE_FINE_STEP times every launch of the fine-level
 * Chebyshev step (the dominant kernel) by events its dispatch records
 * itself.  Work queued past convergence (kernels that return at once on the
 * device stop flag) is not counted. */
#define GIAMG_PHASE_FIRST_SMOOTH 0  /* pre- and post-smoothing on the finest level */
#define GIAMG_PHASE_SMOOTH       1  /* smoothing on every level, the finest included */
#define GIAMG_PHASE_RESIDUAL     2  /* V-cycle residuals f - A x on every level */
#define GIAMG_PHASE_TRANSFER     3  /* restriction and prolongation ("PR transfer") */
#define GIAMG_PHASE_COARSE       4  /* direct solve on the coarsest level */
#define GIAMG_PHASE_VCYCLE       5  /* whole V-cycles (the preconditioner applications) */
#define GIAMG_PHASE_CG_MATVEC    6  /* CG product q = A p (with its dot-product partials) */
#define GIAMG_PHASE_CG_DOT       7  /* CG reductions and dot products */
#define GIAMG_PHASE_CG_UPDATE    8  /* CG vector updates: iterate, residual, direction */
#define GIAMG_PHASE_PCG          9  /* whole PCG iterations */
#define GIAMG_PHASE_FINE_STEP   10  /* single launches of the fine-level Chebyshev step */
#define GIAMG_PHASE_COUNT       11

typedef struct giamg_profile {
    double  ms[GIAMG_PHASE_COUNT];     /* summed GPU milliseconds per phase */
    int64_t count[GIAMG_PHASE_COUNT];  /* intervals summed per phase */
    int64_t solves;                    /* solves profiled */
    int64_t iterations;                /* their CG iterations */
} giamg_profile;

/* on = 1: profile every phase of the following giamg_solve calls of the
 * handle; on = 2: time only the launches of the fine-level Chebyshev step
 * (GIAMG_PHASE_FINE_STEP: no markers between the other kernels, so the
 * solve runs as unprofiled); on = 0: stop.  Profiled solves launch every
 * kernel from the host (as with graph_launch = 0) and create HIP events as
 * needed; giamg_solve_noalloc is never profiled.  Returns GIAMG_OK or
 * GIAMG_EINVAL. */
int giamg_profile_enable(giamg_handle h, int32_t on);
/* Copy the accumulated breakdown into *out (host); reset = 1 clears it. */
int giamg_profile_read(giamg_handle h, giamg_profile* out, int32_t reset);

/*
 * giamg_read_bandwidth -- attainable HBM read bandwidth of the current
 * device: a streaming kernel reads a fresh, zeroed buffer of `bytes` bytes
 * (contiguous 64 KB per block, 16-byte non-temporal loads, nothing written
 * for a zero buffer) once untimed and then `reps` times; *gbs
 * receives the median over the launches of bytes / duration (HIP events
 * recorded by the dispatches).  The buffer comes from the registered
 * allocator and is released before returning.  bytes >= 1 MiB, reps in
 * [1, 1000]; GIAMG_EINVAL otherwise, GIAMG_ENOMEM if the buffer cannot be
 * allocated.  Synchronises the device's null stream.
 */
int giamg_read_bandwidth(int64_t bytes, int32_t reps, double* gbs);

/* ---- hierarchy introspection (host outputs; synchronise the stream) ---- */
#define GIAMG_LEVEL_P        0   /* p-coarsened level (or the fine level) */
#define GIAMG_LEVEL_H        1   /* smoothed-aggregation level */
#define GIAMG_MAT_A          0
#define GIAMG_MAT_P          1   /* prolongation to the next coarser level */
#define GIAMG_MAT_R          2   /* restriction R = P^T */
#define GIAMG_MAT_AP         3   /* A P, the left factor of the Galerkin product (rows of
                                    this level, columns of the next); the post-smoother
                                    uses it for its first residual after the correction */

typedef struct giamg_level_desc {
    int32_t kind;        /* GIAMG_LEVEL_* */
    int32_t order;       /* polynomial order of the level (1 for h-levels) */
    int32_t coarsest;    /* 1 on the last level */
    int32_t device_assembly;  /* fine level: 1 if A was assembled on the device; else 0 */
    int64_t rows;        /* rows of A on this level */
    int64_t nnz_A, nnz_P, nnz_R;   /* P/R are 0 on the coarsest level */
    double  lam_hat;     /* lambda_max(D^-1 A) estimate (0 on the coarsest level) */
    int64_t nnz_AP;      /* 0 on the coarsest level */
    int64_t staged_nnz_A;  /* nonzeros of A in row blocks with staged gathers (0: all direct,
                              or A runs in the grouped form) */
    int64_t runs_A;        /* column runs those blocks stage */
    int64_t groups_A;      /* grouped form of A (see row_groups): row groups, 0 if not built */
    int64_t group_entries_A; /* 16-bit slots of that form (sum of the groups' row lengths) */
    int64_t lean_A;        /* 1: A is multiplied in the lean form (see lean_max_nnz) */
} giamg_level_desc;

/*
 * giamg_hierarchy_info -- sizes of the hierarchy's operators: the levels of
 * the V-cycle of Algorithm 1 (p-levels from the element map of Section 2.2,
 * then the smoothed-aggregation levels of Section 2.5), fine level first.
 *
 * n_levels host out: number of levels.
 * rows     host out, int64 [cap]: rows of A on level l, for l < min(cap, levels).
 * nnz      host out, int64 [cap]: stored nonzeros of A on level l.
 * cap      entries the caller's arrays hold (>= 0; 0 with NULL arrays queries
 *          the level count only).
 * Returns GIAMG_OK, or GIAMG_EINVAL for a null handle, a null n_levels, a
 * negative cap, or a null array with cap > 0.  Levels beyond cap are not
 * written; the call reads host-side metadata only (no synchronisation).
 */
int giamg_hierarchy_info(giamg_handle h, int32_t* n_levels, int64_t* rows, int64_t* nnz,
                         int32_t cap);

int giamg_num_levels(giamg_handle h);
int giamg_level_describe(giamg_handle h, int32_t level, giamg_level_desc* out);

/* Copy one CSR operator of a level to host arrays sized from the level
 * description: row_ptr int64 [rows+1], col int32 [nnz] (ascending within a
 * row), val double [nnz].  Any pointer may be NULL to skip it. */
int giamg_level_csr(giamg_handle h, int32_t level, int32_t which,
                    int64_t* row_ptr, int32_t* col, double* val);

/* p-levels: copy the level's element map, int32 [n_elem][(order+1)^3], -1
 * for constrained nodes (coarse levels hold free nodes only).  h-levels:
 * copy the aggregate id of each row of the level above, int32 [rows of the
 * finer level]; pass the h-level's finer level index. */
int giamg_level_l2g(giamg_handle h, int32_t level, int32_t* out);
int giamg_level_aggregates(giamg_handle h, int32_t level, int32_t* out);

/* Constrained-node mask of the fine level, uint8 [n_nodes] (host). */
int giamg_constrained(giamg_handle h, uint8_t* mask);

/*
 * giamg_apply -- run one step of the V-cycle on device vectors of a level
 * (double precision operators), for step-by-step checking.
 *   GIAMG_OP_SPMV        out = A_l a
 *   GIAMG_OP_RESIDUAL    out = a - A_l b              (a = f, b = x)
 *   GIAMG_OP_RESTRICT    out = R_l a                  (out on level l+1)
 *   GIAMG_OP_PROLONG_ADD out = out + P_l a            (a on level l+1)
 *   GIAMG_OP_PRESMOOTH   out = pre-smoothing of A_l x = a from x = 0
 *   GIAMG_OP_POSTSMOOTH  out = post-smoothing of A_l x = a from x = out
 *   GIAMG_OP_COARSE      out = A_l^-1 a               (coarsest level only)
 *   GIAMG_OP_VCYCLE      out = V-cycle from level l applied to a
 * Add GIAMG_OP_FP32 to run the FP32 operators of a mixed-precision handle
 * on float vectors.  Vectors are sized by the level they live on; a and out
 * must be non-NULL, b only for the residual (else GIAMG_EINVAL).
 * Synchronises the stream.
 */
#define GIAMG_OP_SPMV         0
#define GIAMG_OP_RESIDUAL     1
#define GIAMG_OP_RESTRICT     2
#define GIAMG_OP_PROLONG_ADD  3
#define GIAMG_OP_PRESMOOTH    4
#define GIAMG_OP_POSTSMOOTH   5
#define GIAMG_OP_COARSE       6
#define GIAMG_OP_VCYCLE       7
#define GIAMG_OP_FP32         256
int giamg_apply(giamg_handle h, int32_t op, int32_t level,
                const void* a, const void* b, void* out);

/* Physical coordinates of the fine-level quadrature points, host double
 * [n_elem][(p+2)^3][3] (tensor Gauss points, first direction slowest). */
int giamg_quadrature_points(giamg_handle h, double* xq);

/* Load vector b_i = sum_e sum_q w_q |J| f_q phi_i(x_q) from values of f at
 * those points (host double [n_elem][(p+2)^3]); b = 0 on constrained nodes.
 * host out b [n_nodes]. */
int giamg_load_vector(giamg_handle h, const double* fq, double* b);

/* Setup timings in milliseconds: [0] host assembly, [1] p-transfers,
 * [2] aggregation, [3] device Galerkin products, [4] coarsest factor,
 * [5] grouped product forms and smoother parameters, [6] total.
 * host out double[7]. */
int giamg_setup_times(giamg_handle h, double* ms);


/* ---- host-side setup steps (CPU only; no GPU or handle needed) ---------
 * The setup stages that run on the host, exposed for checking.  Results are
 * returned as a host CSR object owned by the library: query its sizes, copy
 * it into caller arrays, then free it. */
typedef struct giamg_hcsr_s* giamg_hcsr;

int  giamg_hcsr_size(giamg_hcsr m, int64_t* rows, int64_t* cols, int64_t* nnz);
int  giamg_hcsr_copy(giamg_hcsr m, int64_t* row_ptr, int32_t* col, double* val);
void giamg_hcsr_free(giamg_hcsr m);

/* Constrained-node mask of giamg_setup's boundary rule (faces owned by one
 * element), uint8 [n_nodes]; basis GIAMG_BASIS_*. */
int giamg_host_boundary(const int32_t* l2g, int64_t n_elem, int32_t p, int64_t n_nodes,
                        int32_t basis, uint8_t* mask);

/* Fine-level assembly exactly as giamg_setup performs it (bc, pin_node and
 * basis as in giamg_opts). */
int giamg_host_assemble(const double* coords, int64_t n_nodes, const int32_t* l2g,
                        int64_t n_elem, int32_t p, double lambda, int32_t bc,
                        int64_t pin_node, int32_t basis, giamg_hcsr* A_out);

/* One p-coarsening step p -> q < p of Algorithms 2-4 and 7 (nodal:
 * interpolation; modal: injection):
 * free_mask uint8 [n_fine] marks the free fine nodes, l2g may hold -1 for
 * constrained nodes; writes l2g_next int32 [n_elem][(q+1)^3] (-1 for
 * constrained coarse nodes), the coarse size, and P. */
int giamg_host_p_transfer(const int32_t* l2g, int64_t n_elem, int32_t p, int32_t q,
                          int64_t n_fine, const uint8_t* free_mask, int32_t basis,
                          int32_t* l2g_next, int64_t* n_coarse, giamg_hcsr* P_out);

/* Smoothed-aggregation transfer of Section 2.5 for a CSR operator (host
 * arrays, ascending columns; row_ptr[0] = 0 and non-decreasing, columns in
 * [0, n), else GIAMG_EINVAL) with aggregation seed and strength threshold
 * theta as in giamg_opts: writes agg int32 [n], returns P. */
int giamg_host_aggregate(const int64_t* row_ptr, const int32_t* col, const double* val,
                         int64_t n, uint64_t seed, double theta, int32_t* agg, int64_t* n_agg,
                         giamg_hcsr* P_out);

/* Dense inverse of the coarsest operator as giamg_setup forms it for the
 * direct solve on the last level of Algorithm 1 (Section 2.1): Cholesky
 * factor A = L L^T, the columns of A^-1 by forward and back substitution,
 * then the result symmetrised exactly.  A: host double [n][n], row-major,
 * symmetric positive definite (only its lower triangle and diagonal are
 * read); inv: host double [n][n], written in full.  1 <= n <= 16384 (the
 * coarsest size giamg_setup accepts); GIAMG_EINVAL if a pivot is not
 * positive (A not positive definite, or NaN), inv then undefined. */
int giamg_host_coarse_inverse(const double* A, int64_t n, double* inv);

/*
 * giamg_time_kernel -- time one device kernel of a level in the launch
 * configuration the solve uses: `reps` (1 to 100000) launches on the handle's stream, each
 * between its own pair of HIP events (contents of the level's work vectors
 * are overwritten).  kernel:
 *   GIAMG_KERNEL_CHEB_STEP  fused Chebyshev step on A_l (FP64; FP32 with GIAMG_OP_FP32)
 *   GIAMG_KERNEL_SPMV       plain y = A_l v
 *   GIAMG_KERNEL_RESTRICT   y = R_l v
 *   GIAMG_KERNEL_PROLONG    x += P_l v
 *   GIAMG_KERNEL_CG_PRODUCT q = A_l p with per-block partial sums of p.q
 *                           (the outer CG's product, FP64)
 * ms receives the mean duration of one launch, bytes its algorithmic HBM
 * bytes (values, column ids or 16-bit slots and run tables, row pointers,
 * the gathered vector once, row-local vectors).
 */
#define GIAMG_KERNEL_CHEB_STEP 0
#define GIAMG_KERNEL_SPMV      1
#define GIAMG_KERNEL_RESTRICT  2
#define GIAMG_KERNEL_PROLONG   3
#define GIAMG_KERNEL_CG_PRODUCT 4
int giamg_time_kernel(giamg_handle h, int32_t kernel, int32_t level, int32_t reps,
                      double* ms, double* bytes);


/* ---- continuous batching ------------------------------------------------
 * A session holds `slots` right-hand sides of one handle, each with its own
 * CG state (the block products of giamg_solve_batch; one CG iteration is a
 * captured HIP graph).  Columns join (admit) and leave (retire) between
 * steps without disturbing the others: a right-hand side gives the same
 * bits whatever else shares the session.  Work runs on a stream of the
 * session's own, ordered after the handle's stream at creation. */
typedef struct giamg_session_s* giamg_session;

int  giamg_session_create(giamg_handle h, int32_t slots, double tol, giamg_session* out);
/* Start `count` columns: b[i] (device, n_nodes doubles) into slot slots[i],
 * zero initial guess.  Asynchronous. */
int  giamg_session_admit(giamg_session s, int32_t count, const int32_t* slots,
                         const double* const* b);
/* Enqueue `iters` CG iterations of every running column.  Asynchronous. */
int  giamg_session_step(giamg_session s, int32_t iters);
/* Synchronise; running[j] = 1 while slot j iterates; infos (may be NULL)
 * get each slot's iterations, status and recursive relative residual. */
int  giamg_session_poll(giamg_session s, int32_t* running, giamg_info* infos);
/* Copy slot's solution into x (device, n_nodes doubles) and free the slot. */
int  giamg_session_retire(giamg_session s, int32_t slot, double* x);
void giamg_session_free(giamg_session s);

/* ---- serving -------------------------------------------------------------
 * A request loop on a background thread: requests for registered problems
 * are continuously batched into sessions (one per resident hierarchy, each
 * on its own stream, so different hierarchies overlap on the device);
 * hierarchies stay cached on the device and are set up on a worker thread
 * when the HBM budget allows, evicting idle ones least recently used first.
 * Latency runs from giamg_server_submit to the solution being in x. */
typedef struct giamg_server_s* giamg_server;

typedef struct giamg_server_opts {
    int64_t hbm_budget;   /* bytes of device memory for hierarchies and slots */
    int32_t slots;        /* concurrent right-hand sides per hierarchy */
    int32_t chunk;        /* CG iterations between admission points */
    double  tol;          /* relative residual target of every request */
    int32_t hold_ms;      /* 0 (default): requests join a hierarchy's free slots at the
                             next chunk boundary; > 0: they join only once they fill the
                             free slots or the oldest has waited hold_ms, or, once a
                             request has finished on that hierarchy, the shorter of
                             hold_ms and that request's admission-to-completion time
                             (fuller batches, longer latency) */
    int32_t pad;
} giamg_server_opts;

typedef struct giamg_server_stats {
    int64_t submitted, completed, setups, evictions, cache_hits;
    int64_t peak_bytes, resident_bytes;
    int32_t groups_resident, pad;
} giamg_server_statistics;

int  giamg_server_create(const giamg_server_opts* opts, giamg_server* out);
/* Register a problem (arguments as giamg_setup; host arrays are copied). */
int  giamg_server_add_problem(giamg_server s, const double* coords, int64_t n_nodes,
                              const int32_t* l2g, int64_t n_elem, int32_t p, double lambda,
                              const giamg_opts* opts, int32_t* problem);
/* Submit b (host, copied) for `problem`; x (host, n_nodes doubles) receives
 * the solution and must stay valid until giamg_server_wait returns. */
int  giamg_server_submit(giamg_server s, int32_t problem, const double* b, double* x,
                         int64_t* request);
/* Block until the request finishes; returns its status. */
int  giamg_server_wait(giamg_server s, int64_t request, giamg_info* info, double* latency_ms);
int  giamg_server_stats(giamg_server s, giamg_server_statistics* out);
void giamg_server_free(giamg_server s);

/* Thread-local message of the last failing call on this thread. */
const char* giamg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* GIAMG_H */
