/*
 * hmat.h -- C ABI of the MI355X H-matrix library for 3D elastodynamic
 * Green's tensors (Chaillat, Desiderio, Ciarlet, arXiv 1706.09384).
 *
 * The library assembles an H-matrix approximation of the dense complex
 * 3Nx x 3Ny matrix of eq. (syst_a), whose 3x3 block (i, j) is the Green's
 * tensor U_w(x_i, y_j) (eq. elasto_U) or its traction T_w(x_i, y_j)
 * (eq. elasto_T, normal taken at y_j) -- or of the P1 collocation matrix of
 * the single-layer equation on a triangle mesh (Section 4, hm_build_colloc)
 * -- and applies it in matrix-vector products (Section 3.1), in restarted
 * GMRES, and in the H-LU direct solver with its certification estimator
 * (Sections 3.2, 3.3).
 *
 * Assembly (hm_build) runs: geometric-bisection cluster trees (Section 2.1),
 * the block partition with the box admissibility condition (Section 6.1,
 * eq. admissibility_cond_bis), dense near-field tiles for non-admissible
 * leaf pairs, partially pivoted vector ACA with rank-3 updates and the
 * largest-sigma_3 pivot rule (Sections 2.2 and 2.3, stopping test eq.
 * stop_part), and recompression of every ACA block by QR + truncated SVD
 * (Section 3.2).  Everything after the trees runs in HIP kernels on the GPU.
 *
 * Conventions shared by all calls
 * -------------------------------
 * Points, normals: (n, 3) row-major float64 arrays.
 * Vectors: 3 degrees of freedom per point, interleaved (row 3i + alpha is
 *   component alpha at point i, original point order), nrhs columns stored
 *   row-major: element (row, c) at row * nrhs + c.  Complex numbers are
 *   interleaved (re, im) pairs: complex64 = 2 x float32, complex128 =
 *   2 x float64.
 * Streams: a hipStream_t passed as void*; NULL is the default stream.
 * Errors: every call returns an hm_status; nothing is thrown across the ABI.
 *   On error a message is available from hm_last_error() (thread-local) and
 *   output handles are left NULL.  No call leaks memory on error.
 * Threading: distinct matrices may be used from distinct threads; calls on
 *   one matrix must not overlap (it owns one set of work buffers).
 */
#ifndef HMAT_H
#define HMAT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HM_OK = 0,
    HM_ERR_ARG = 1,       /* invalid argument (sizes, NaN coordinates, parameters) */
    HM_ERR_ALLOC = 2,     /* device or host allocation failed */
    HM_ERR_HIP = 3,       /* a HIP runtime call or kernel launch failed */
    HM_ERR_SINGULAR = 4,  /* kernel evaluated at coincident points x_i == y_j (r = 0) */
    HM_ERR_NOCONV = 5,    /* GMRES reached maxit before tol; info is filled */
    HM_ERR_STATE = 6      /* call not valid for this object (e.g. matvec on a plan-only build) */
} hm_status;

typedef enum { HM_KERNEL_U = 0, HM_KERNEL_T = 1 } hm_kernel;

/* Storage and compute precision of the operator. */
typedef enum {
    HM_C128 = 0,  /* complex128 everywhere (the plain FP64 form) */
    HM_C64 = 1    /* complex64 kernel evaluation, ACA updates, storage and matvec;
                     ACA norm recurrences, recompression and GMRES refinement in FP64 */
} hm_prec;

typedef struct {
    int32_t kernel;        /* hm_kernel */
    int32_t prec;          /* hm_prec */
    double omega;          /* circular frequency (>= 0), Section 1 */
    double lambda, mu;     /* Lame parameters (mu > 0, lambda + 2 mu > 0) */
    double rho;            /* density (> 0); kappa_s^2 = rho w^2/mu, kappa_p^2 = rho w^2/(lambda+2mu) */
    double eta;            /* admissibility parameter eta-hat (>= 0), eq. admissibility_cond_bis */
    double eps;            /* ACA and recompression tolerance, 0 < eps < 1 (Sections 2.2, 3.2) */
    int32_t leaf;          /* maximum number of points in a leaf cluster (>= 1) */
    int32_t same;          /* 1: the column cloud is the row cloud (y ignored, one tree) */
    double self_re;        /* when same: the 3x3 diagonal blocks i == j are (self_re + i self_im) I3 */
    double self_im;
    int32_t points_on_host;/* 1: x, y, normals are host pointers; 0: device pointers */
    int32_t plan_only;     /* 1: build trees and block list only (no GPU work, no GPU needed) */
    int32_t rank_budget;   /* initial ACA column budget per block, 0 = library default */
    int32_t recompress;    /* 1: recompress ACA blocks (default); 0: keep the ACA factors */
    double tau_piv;        /* singular-pivot threshold on sigma_3/|M|_F, 0 = default per precision */
    const float *rank_model;   /* optional host pointer to rank-model weights
                                  (HM_RANK_MODEL_PARAMS floats), NULL = none */
    int32_t matvec_graph;  /* 1: hm_matvec replays a captured HIP graph of its launches
                              (re-captured when x, y or nrhs change) */
    int32_t unbatched;     /* 1: assembly launches its kernels once per block (the
                              comparison baseline of the batched default) */
    int32_t aca_scratch_mb;/* cap on the first-pass ACA factor scratch of one chunk of
                              admissible blocks, MiB; 0 = 40% of the device memory
                              free when the chunk starts (see hm_build) */
    int32_t rsvd;          /* 1: T-kernel admissible blocks whose 3x3 sub-blocks are all
                              singular by construction (both clusters in one coordinate
                              plane x_a = c, every column normal +-e_a: the planar
                              pattern of Section 2.3) are compressed by the randomized
                              range finder (the remark closing Section 2.3) instead of
                              the vector ACA with its singular-pivot fallback; the
                              range keeps |A - Q Q^* A|_F <= (eps/2)|A|_F and the
                              recompression truncates to eps (default 1: with the
                              fallback, single coplanar blocks of a cube missed eps by
                              up to 1,200 times); 0: vector ACA for every block */
    int32_t reserved[4];
} hm_params;

/* Fill p with the defaults: U kernel, complex128, w = 1, lambda = 2, mu = rho = 1,
 * eta = 3, eps = 1e-4, leaf = 32, same = 1, recompress = 1, rsvd = 1, everything
 * else 0 / NULL. */
hm_status hm_params_default(hm_params *p);

typedef struct hm_matrix hm_matrix;   /* opaque; owns all device memory it allocates */

/*
 * Assemble the H-matrix.
 *   x        (nx, 3) float64 row points
 *   y        (ny, 3) float64 column points, ignored when p->same (then ny must equal nx)
 *   normals  (ny, 3) float64 unit normals at the column points; required for
 *            HM_KERNEL_T, ignored (may be NULL) for HM_KERNEL_U
 *   stream   HIP stream for all device work; the call synchronizes it before returning
 *   out      receives the new matrix
 * Errors: HM_ERR_ARG for nx < 1, ny < 1, non-finite coordinates, leaf < 1,
 *   eta < 0, eps outside (0, 1), mu <= 0, rho <= 0, lambda + 2 mu <= 0,
 *   omega < 0, missing normals for T; HM_ERR_SINGULAR if a non-self block
 *   pairs two coincident points; HM_ERR_ALLOC / HM_ERR_HIP on device failure.
 * The library copies everything it needs; no caller pointer is retained.
 * Memory: the admissible blocks are compressed in chunks (dealt round-robin
 * in longest-ACA-first order); a chunk holds about aca_scratch_mb of
 * first-pass ACA factors, and its recompressed factors are final before the
 * next chunk starts.  Each chunk's factors stay in their own buffer, so peak
 * device memory is about the near field + the compressed factors + one
 * chunk's scratch.
 */
hm_status hm_build(const double *x, int64_t nx, const double *y, int64_t ny, const double *normals,
                   const hm_params *p, void *stream, hm_matrix **out);

/*
 * Assemble the H-matrix of the P1 collocation matrix of the single-layer
 * equation (Section 4, eqs. EFIE and discre_syst): a mesh of flat triangles,
 * continuous piecewise-linear hat functions v_j on its vertices, collocation
 * at the vertices.  Block (i, j) is
 *     sum over the elements E around vertex j of  int_E U_w(x_i, y) v_j(y) dS(y),
 * each element integral a collapsed (Duffy) Gauss-Legendre product rule with
 * q x q points: collapsed onto x_i with q_sing points when x_i is a vertex of
 * E (the surface Jacobian's factor cancels the 1/r singularity of U), onto
 * the element's first vertex with q_reg points otherwise.  The clusters, the
 * admissibility condition, the ACA and the recompression run on the vertices
 * as in hm_build, with the entry blocks above in place of U_w(x_i, y_j); every
 * other call (matvec, GMRES, H-LU, hm_frob_error) works on the result.
 *   nodes   (nc, 3) float64 vertices (the collocation points)
 *   tri     (ne, 3) int32 vertex indices of the elements, 0-based
 *   q_reg, q_sing  Gauss-Legendre points per direction, 1 .. 32 (the paper
 *           names no rule; 3 and 6 are the defaults of the Python binding)
 *   p       as for hm_build; kernel must be HM_KERNEL_U; same, self_re,
 *           self_im and rsvd are ignored (the operator is square on the
 *           vertices and has no point self blocks).  nodes and tri are host
 *           pointers when p->points_on_host, device pointers otherwise.
 * Errors: HM_ERR_ARG for a T kernel, nc < 3, ne < 1, an element vertex out of
 *   range or repeated, a vertex in no element, quadrature orders outside
 *   1 .. 32, and every hm_build argument error; HM_ERR_ALLOC / HM_ERR_HIP on
 *   device failure.  Nothing is retained from the caller's arrays.
 */
hm_status hm_build_colloc(const double *nodes, int64_t nc, const int32_t *tri, int64_t ne,
                          int32_t q_reg, int32_t q_sing, const hm_params *p, void *stream,
                          hm_matrix **out);

/*
 * y = A_H x, Section 3.1 (leaf blocks: dense O(mn), low-rank O(r(m+n))).
 *   x  device, (3 ny, nrhs), complex64 for HM_C64 or complex128 for HM_C128
 *   y  device, (3 nx, nrhs), same type; overwritten.  x and y must not overlap.
 * Both are row-major: entry (3i + a, c) is at index (3i + a) * nrhs + c.
 * Complex64 operators with nrhs >= 8 run on panels of 64 right-hand sides
 * with FP32 matrix-core products (the first such call allocates the panel
 * workspaces: 3 ny x 64 and sum(rank) x 64 complex64); other cases apply one
 * column at a time.  Calls that overlap on one matrix race on its workspaces.
 * Asynchronous on stream.  HM_ERR_ARG for nrhs < 1 or NULL pointers.
 */
hm_status hm_matvec(const hm_matrix *A, const void *x, void *y, int32_t nrhs, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * product as hm_matvec, y = A_H x, with its work vectors (x in cluster order,
 * the projections t = V^* x, the projection partial sums) taken from a fixed
 * 64 MiB device array that the library holds on each GPU it runs on until
 * the process ends, instead of the matrix's own workspaces.  It calls no
 * hipMalloc, hipFree or allocating library routine.
 *   x, y   as in hm_matvec (device, operator's complex type, row-major
 *          (3 ny, nrhs) / (3 nx, nrhs)); columns are applied one at a time
 *          with the one-column kernels (never the 64-column matrix-core
 *          panels), so for those columns the result equals hm_matvec's
 *          bit for bit.
 * HM_ERR_ARG when 3 ny + sum(rank) + 64 * (projection slots) complex
 * entries (each part rounded up to 256 bytes) exceed the 64 MiB, that is
 * 8,388,608 complex64 or 4,194,304 complex128 entries, for NULL pointers or
 * nrhs < 1;
 * HM_ERR_STATE for a plan-only matrix.  Every entry of the array is written
 * before it is read within one call.  All calls on one GPU share its array:
 * calls that overlap on one GPU (any matrices, any streams) race.
 * Asynchronous on stream.
 */
hm_status hm_matvec_noalloc(const hm_matrix *A, const void *x, void *y, int32_t nrhs, void *stream);

/*
 * r = b - A_H x evaluated with FP64 arithmetic from the stored factors
 * (complex64 or complex128 storage): the residual of the linear system
 * eq. syst_a with the H-matrix product of Section 3.1, used as the outer
 * residual of iterative refinement and to confirm GMRES convergence.
 *   b, x, r  device complex128, (3 nx, nrhs) / (3 ny, nrhs) / (3 nx, nrhs),
 *            row-major as in hm_matvec; r must not overlap b or x.
 * Asynchronous on stream.  HM_ERR_ARG for nrhs < 1 or NULL pointers,
 * HM_ERR_STATE for a plan-only matrix.
 */
hm_status hm_residual(const hm_matrix *A, const void *b, const void *x, void *r, int32_t nrhs,
                      void *stream);

typedef struct {
    int32_t iters;         /* total inner Krylov iterations (max over right-hand sides) */
    int32_t restarts;      /* GMRES cycles started */
    int32_t refinements;   /* outer FP64 refinement steps (0 for complex128 operators) */
    int32_t converged;     /* number of right-hand sides that met tol */
    double relres;         /* max over columns of |b - A_H x| / |b|, recomputed in FP64 */
    double relres_inner;   /* last inner recursive residual estimate (max over columns) */
} hm_gmres_info;

/*
 * Solve A_H x = b, the system eq. syst_a with the H-matrix operator, by
 * restarted GMRES(restart), the iterative solver of Section 1 whose cost is
 * dominated by the H-matrix-vector products of Section 3.1; x0 = 0, no
 * preconditioner (the paper leaves preconditioning open).
 * Each of the nrhs columns is an independent GMRES run; all columns share
 * one multi-right-hand-side H-matvec per iteration.  Complex128 operators
 * iterate in FP64 until the recursive residual is below tol, then confirm
 * with an explicit residual.  Complex64 operators run iterative refinement:
 * an FP64 residual (hm_residual), an inner complex64 GMRES on it, an FP64
 * update, until |b - A_H x| / |b| <= tol in FP64.
 *   b, x   device complex128, (3 nx, nrhs); x is overwritten.
 * Synchronous.  HM_ERR_NOCONV when maxit total inner iterations pass without
 * reaching tol (x then holds the last iterate and info is filled).
 */
hm_status hm_gmres(const hm_matrix *A, const void *b, void *x, int32_t nrhs, double tol,
                   int32_t restart, int32_t maxit, void *stream, hm_gmres_info *info);

typedef struct {
    int64_t nx, ny;                    /* points */
    int32_t nodes_x, nodes_y;          /* cluster tree sizes */
    int32_t leaves_x, leaves_y;
    int32_t levels_x, levels_y;        /* depth + 1 */
    int64_t n_blocks, n_dense, n_lowrank;
    int32_t c_sp;                      /* sparsity constant C_sp (Section 2.1) */
    int32_t prec;
    int64_t dense_entries;             /* complex entries in dense tiles */
    int64_t lowrank_entries;           /* complex entries in low-rank factors U, V */
    int64_t storage_bytes;             /* dense + low-rank bytes as stored */
    int32_t max_rank_aca, max_rank;    /* largest ACA rank, largest rank after recompression */
    int64_t sum_rank_aca, sum_rank;
    int32_t n_overflow;                /* budget continuations: a block that outgrows its column
                                          budget continues from where it stopped with a larger one
                                          (counted once per continuation) */
    int32_t n_fallback;                /* ACA steps that used the singular-pivot fallback */
    int32_t n_model_hits;              /* blocks whose predicted budget sufficed */
    double t_tree, t_upload, t_nearfield, t_aca, t_recompress, t_plan, t_total; /* seconds; the
                                          recompression of the blocks with few points can run inside
                                          t_aca, beside the ACA of the blocks with many points */
    int64_t matvec_bytes;              /* algorithmic bytes of one 1-RHS matvec */
    int64_t aca_scratch_bytes;         /* first-pass ACA factor scratch, summed over chunks */
    int32_t aca_chunks;                /* chunks the admissible blocks were assembled in */
    int32_t acc_waves, proj_rows;      /* 1-RHS matvec launch shape (hm_autotune may change it) */
    int32_t n_capped;                  /* admissible blocks whose ACA reached the rank cap (852
                                          columns in complex64, 639 in complex128) before its
                                          stopping test held: they keep the capped factors, which
                                          may miss eps; 0 on every workload of the test suite */
    int32_t n_rsvd;                    /* admissible blocks compressed by the randomized range
                                          finder (params.rsvd); their rank_aca is the number of
                                          samples */
} hm_stats;

hm_status hm_info(const hm_matrix *A, hm_stats *s);

/*
 * Measurement helper: runs the 1-RHS matvec kernels (gather, project,
 * accumulate) `reps` times on `stream` with HIP events between the launches.
 *   x, y          device vectors of the operator's type, (3 ny) and (3 nx)
 *   kernel_ms     host double[3]: mean duration of each kernel (ms)
 *   kernel_bytes  host int64[3]: algorithmic HBM bytes of each kernel
 *                 (x read; V factors; dense tiles + U factors + y write)
 * Synchronous.
 */
hm_status hm_profile_matvec(const hm_matrix *A, const void *x, void *y, int32_t reps, void *stream,
                            double *kernel_ms, int64_t *kernel_bytes);

/*
 * Measurement helper for the multi-RHS panels (complex64 operators only):
 * runs one 64-column panel product `reps` times on `stream` with HIP events
 * between the gather, project (+ reduction) and accumulate passes.
 *   x, y          device complex64, (3 ny, 64) and (3 nx, 64), row-major
 *   kernel_ms     host double[3]: mean duration of each pass (ms)
 *   kernel_flops  host double[3]: algorithmic flops of each pass (8 per
 *                 complex multiply-add: 0; 64 * 8 * sum 3 n r; 64 * 8 *
 *                 (sum 9 m n + sum 3 m r))
 * Synchronous.  HM_ERR_STATE for complex128 operators.
 */
hm_status hm_profile_matvec_multi(const hm_matrix *A, const void *x, void *y, int32_t reps,
                                  void *stream, double *kernel_ms, double *kernel_flops);

/*
 * Autotuner of the 1-RHS matvec launch shape: times every combination of
 * waves per accumulation workgroup {4, 8, 16} and projection row chunk
 * {256, 512, 1024} (`reps` timed products each, HIP events on `stream`) and
 * keeps the fastest for later hm_matvec calls.
 *   ms_table  host double[9] (may be NULL): mean ms, index 3 * chunk + waves
 * Synchronous; allocates two temporary vectors.  The products change only in
 * their floating-point summation order.
 */
hm_status hm_autotune(hm_matrix *A, int32_t reps, void *stream, double *ms_table);

/*
 * Copy a cluster tree to host buffers (which = 0: row tree, 1: column tree).
 *   perm   int32[n]: cluster position -> original point index
 *   nodes  int32[nodes * 5]: begin, end, left child, right child (-1 for
 *          leaves), depth; nodes numbered in pre-order
 *   boxes  float64[nodes * 6]: lo[3], hi[3] tight bounding boxes
 * Any pointer may be NULL to skip it.
 */
hm_status hm_export_tree(const hm_matrix *A, int32_t which, int32_t *perm, int32_t *nodes,
                         double *boxes);

/*
 * Copy the block partition to host buffers, in the order of a depth-first
 * traversal of the block cluster tree.
 *   blocks    int32[n_blocks * 3]: row node, column node, kind (0 dense, 1 low-rank)
 *   rank      int32[n_blocks]: stored rank (-1 for dense blocks)
 *   rank_aca  int32[n_blocks]: rank produced by ACA before recompression (-1 dense)
 */
hm_status hm_export_blocklist(const hm_matrix *A, int32_t *blocks, int32_t *rank,
                              int32_t *rank_aca);

/*
 * Copy one stored block to a host buffer in the operator's complex type,
 * rows/columns in cluster-local order (row 3p + alpha = point perm[begin + p]):
 * dense: the 3m x 3n tile, column-major; low-rank: U (3m x r, column-major)
 * followed by V (3n x r, column-major), block = U V^*.
 */
hm_status hm_export_block(const hm_matrix *A, int64_t block, void *host_buf);

void hm_destroy(hm_matrix *A);

/* ---------------------------------------------------------------------
 * H-LU direct solver (Section 3.2) and its certification (Section 3.3).
 * ------------------------------------------------------------------- */
typedef struct hm_lu hm_lu;   /* opaque; owns the factors' device memory */

typedef struct {
    double t_import;          /* seconds: copy of A_H into the factor blocks */
    double t_factor;          /* seconds: the recursive factorisation (synchronous) */
    int64_t storage_entries;  /* complex entries of L_H and U_H: m n per dense block,
                                 (m + n) k per low-rank block */
    int64_t device_bytes;     /* device memory held by the factors and their workspaces */
    int32_t max_rank;         /* largest rank of a low-rank factor block */
    int32_t n_nodes;          /* blocks of the block cluster tree (leaves and inner) */
    int32_t n_diag;           /* dense diagonal leaves factorised */
    int32_t n_recompressed;   /* low-rank blocks recompressed at eps_LU */
    int32_t n_batches;        /* batches those recompressions ran in */
    int32_t n_gemm;           /* matrix-core GEMM launches of the recursion */
    double gemm_flops;        /* their flops, 8 per complex multiply-add */
    int32_t n_sampled;        /* recompressions whose stacked factors (more than 64 columns)
                                 went through the randomized range finder first */
    int32_t reserved;
} hm_lu_stats;

/*
 * Factorise A_H = L_H U_H (Section 3.2): the recursive 2 x 2 block LU over
 * the block cluster tree, steps (1) A11 = L11 U11, (2) U12 = L11^-1 A12,
 * (3) L21 = A21 U11^-1, (4) A22 - L21 U12 = L22 U22, every block in the
 * dense, low-rank or subdivided format, without pivoting.  Sums that reach a
 * low-rank block are recompressed (QR of both factors, truncated SVD of
 * R_U R_V^*) at eps_lu, keeping the singular values whose Frobenius tail
 * exceeds eps_lu times the total; when the stacked factors hold more than 64
 * columns and eps_lu >= 1e-6, a randomized range finder (Liberty et al. 2007,
 * range error at most eps_lu / 2 in the Frobenius norm) reduces them first.  Dense diagonal leaves are eliminated
 * without pivoting.  Arithmetic is complex128 whatever A's precision.
 * Independent branches of the recursion (steps 2 and 3, the block columns or
 * rows of a substitution, the target blocks of an update) run on up to four
 * streams: the caller's and three created for the call (default priority),
 * joined back into the caller's stream by events; the environment variable
 * HM_LU_STREAMS (1 .. 4, default 4) sets the number.  The factors do not
 * depend on it.
 *   A       an assembled square operator (params.same = 1); read only, and
 *           not needed by the factors afterwards
 *   eps_lu  >= 0; values below 1e-13 act as 1e-13 (singular values at the
 *           rounding level of a block are never kept), so eps_lu = 0 gives
 *           the LU of A_H up to that floor
 *   out     receives the factors; free with hm_lu_destroy
 * Synchronous on stream.  HM_ERR_ARG for bad arguments or same = 0,
 * HM_ERR_STATE for a plan-only matrix, HM_ERR_NOCONV if a diagonal leaf
 * meets a zero pivot, HM_ERR_ALLOC when device memory runs out.
 */
hm_status hm_lu_factor(const hm_matrix *A, double eps_lu, void *stream, hm_lu **out);

/*
 * x0 = U_H^-1 L_H^-1 b: block forward then backward substitution over the
 * block tree (Section 3.2, direct solver).
 *   b, x  device complex128, row-major (3N, nrhs), original point order;
 *         b and x may not overlap
 * Asynchronous on stream.  HM_ERR_ARG for NULL pointers or nrhs < 1.
 */
hm_status hm_lu_solve(hm_lu *F, const void *b, void *x, int32_t nrhs, void *stream);

hm_status hm_lu_get_stats(const hm_lu *F, hm_lu_stats *s);

/*
 * The factors as one dense matrix, L_H strictly below the diagonal (unit
 * diagonal implied) and U_H on and above it, 3N x 3N column-major complex128
 * in cluster order (row 3p + a is point perm[p], component a), to a host
 * buffer.  For checks on small problems: HM_ERR_ARG when 3N > 20000.
 */
hm_status hm_lu_export_dense(hm_lu *F, void *host_buf);

void hm_lu_destroy(hm_lu *F);

/*
 * delta_H,F = |A_H - A|_F and |A|_F (Section 3.3): every stored block is
 * compared with the kernel re-evaluated in FP64 at its point pairs (dense
 * tiles entry by entry, low-rank blocks through their factors).
 * Synchronous on stream.  HM_ERR_STATE for a plan-only matrix.
 */
hm_status hm_frob_error(const hm_matrix *A, void *stream, double *diff_fro, double *a_fro);

/*
 * Sampled rows of the exact operator times x, the reference for the error of
 * the H-matrix product (Section 3.1) on those rows: for each sampled row
 * point i, y(3r + a, c) = sum_j sum_b K_ab(x_i, y_j) x(3j + b, c), every
 * entry block evaluated again in FP64 (the Green's tensor of eq. elasto_U /
 * elasto_T with the self blocks of hm_params, or the collocation operator's
 * element quadrature of Section 4) and never stored.  O(nrows * ny) kernel
 * evaluations.
 *   rows   host, nrows row point indices in the caller's order (0 .. nx - 1)
 *   x      device complex128, (3 ny, nrhs) row-major, the caller's point order
 *   y      device complex128, (3 nrows, nrhs) row-major: rows 3r .. 3r + 2 for rows[r]
 * Whatever the operator's precision, the evaluation and the sums are FP64;
 * partial sums over column chunks are added in a fixed order (deterministic).
 * Synchronizes the stream.  Errors: HM_ERR_ARG for NULL pointers, nrows
 * outside 1 .. 2^20, nrhs outside 1 .. 256, a row index out of range;
 * HM_ERR_STATE for a plan-only matrix.
 */
hm_status hm_exact_rows(const hm_matrix *A, const int64_t *rows, int64_t nrows, const void *x,
                        int32_t nrhs, void *y, void *stream);

typedef struct {
    double delta;      /* |b - A_H x0|_2 (FP64 residual with the H-matvec) */
    double delta_h;    /* the delta_H passed in */
    double b_norm, x0_norm;
    double estimate;   /* I = (delta + delta_H |x0|) / |b|, eq. est_direct */
} hm_lu_estimate_t;

/*
 * The estimator of eq. est_direct for one right-hand side:
 * |b - A x0| / |b| <= (delta + delta_H |x0|) / |b| with delta = |b - A_H x0|.
 *   b, x0    device complex128 vectors (3N), original point order
 *   delta_h  |A_H - A| in a norm that bounds the 2-norm (hm_frob_error's
 *            diff_fro)
 * Synchronous on stream.
 */
hm_status hm_lu_estimate(const hm_matrix *A, const void *b, const void *x0, double delta_h,
                         void *stream, hm_lu_estimate_t *est);

/*
 * Return the library's cached device memory to the driver.  Buffers of
 * 32 MiB or more that the library releases (build temporaries, destroyed
 * matrices) are kept for reuse, because freeing and re-allocating tens of GB
 * costs the driver up to seconds per build; they stay allocated until this
 * call or process exit.  Call it only when no library call is running.
 */
void hm_release_cache(void);

/* Thread-local description of the last error, "" if none. */
const char *hm_last_error(void);

/* ---------------------------------------------------------------------
 * Rank model: a 6 -> 64 -> 64 -> 1 ReLU network predicting the ACA rank of
 * an admissible block from (log|X|, log|Y|, k_s diam X, k_s diam Y,
 * k_s dist(X,Y), log10 eps), diam/dist from the bounding boxes.  The
 * target is log2(1 + r_ACA/3).  A prediction only sizes the first ACA
 * budget of a block; ACA's own stopping test still decides the rank.
 * Weights are float32, packed W1(64x6) b1(64) W2(64x64) b2(64) W3(1x64) b3(1).
 * --------------------------------------------------------------------- */
#define HM_RANK_MODEL_PARAMS (64 * 6 + 64 + 64 * 64 + 64 + 64 + 1)

/* Features and ACA ranks of every admissible block of a built matrix, in
 * block-list order: feats float32[n_lowrank * 6], ranks int32[n_lowrank]
 * (host buffers).  ln is the natural logarithm; diam and dist are the
 * bounding-box diameter and box distance of the admissibility test
 * (Section 7.1).  For a plan_only matrix the ranks are -1. */
hm_status hm_rank_samples(const hm_matrix *A, float *feats, int32_t *ranks);

/*
 * Train the rank model on the GPU with the library's own FP32 forward,
 * backward and Adam kernels (mean squared error on log2(1 + r/3)).
 *   feats    host float32[n * 6];  ranks  host int32[n]
 *   weights  host float32[HM_RANK_MODEL_PARAMS], in: initial, out: trained
 *   loss_out host float32[epochs] (may be NULL): mean loss per epoch
 */
hm_status hm_rank_model_train(const float *feats, const int32_t *ranks, int64_t n,
                              float *weights, int32_t epochs, int32_t batch, float lr,
                              uint64_t seed, float *loss_out, void *stream);

/* Forward pass on device: feats (n x 6) -> pred (n), all device float32. */
hm_status hm_rank_model_predict(const float *weights_host, const float *feats, float *pred,
                                int64_t n, void *stream);

/* One forward+backward pass on device for checking gradients: device
 * feats (n x 6), device targets (n), host weights; returns the loss and the
 * gradient (host float32[HM_RANK_MODEL_PARAMS]). */
hm_status hm_rank_model_grad(const float *weights_host, const float *feats, const float *targets,
                             int64_t n, float *loss, float *grad_host, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* HMAT_H */
