/*
 * ba.h -- C ABI of the MI355X bundle-adjustment hot path.
 *
 * Exact Levenberg-Marquardt bundle adjustment through the reduced camera
 * system (RCS), following "Distributed bundle adjustment with block-based
 * sparse matrix compression for super large scale datasets":
 *   normal equations (J^T J + lambda D^T D) dx = -J^T e ............ Sec. 3.1, Eq. (1)
 *   camera / point partition U, V, W, l_c, l_p ...................... Eq. (3)
 *   RCS  (U - W V^-1 W^T) dx_c = l_c - W V^-1 l_p ................... Eq. (4)
 *   points  V dx_p = l_p - W^T dx_c .................................. Eq. (5)
 *   block-diagonal preconditioned CG on the RCS ...................... Sec. 3.2, Eq. (6)-(7)
 *   RCS kept as upper-triangle 9x9 blocks (BSMC idea) ................ Sec. 4, Eq. (9)
 *   RCS formed point by point and summed ............................. Sec. 5
 *
 * Conventions
 *   - Camera i has 9 parameters [w(3) axis-angle, t(3), f, k1, k2]; a world
 *     point X projects as P = R(w) X + t, (x, y) = (P_x, P_y) / P_z,
 *     d = 1 + k1 r^2 + k2 r^4, pixel = f d (x, y).  Residual e = pixel - observed.
 *   - D^T D = diag(J^T J) (Marquardt scaling): U* = U + lambda diag(U),
 *     V* = V + lambda diag(V).
 *   - RCS rows are the free cameras (cam_fixed[i] == 0) in camera order; the
 *     camera-side vectors dxc and rhs are laid out [n_rows][9].
 *   - RCS blocks: row_ptr[n_rows+1] (int64), col_idx[n_blk] (int32) ascending
 *     within a row with the diagonal block first, blocks [n_blk][9][9] FP64
 *     row-major.  Only blocks (r, s) with r <= s are stored; block (r, s),
 *     r < s, exists iff the two cameras observe a common point.
 *   - "device" pointers are HIP device memory of the device current when
 *     ba_create was called; "host" pointers are ordinary host memory.
 *   - Every call is ordered on the context's stream.  Calls that return host
 *     values (cost, info structs, getters) synchronise that stream.
 *   - No exception crosses the ABI.  A context is not thread-safe; distinct
 *     contexts are independent.
 */
#ifndef BA_H
#define BA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum ba_status {
    BA_OK = 0,
    BA_ERR_INVALID_ARG = 1,    /* bad sizes, indices, non-finite data, duplicate observations */
    BA_ERR_STATE = 2,          /* call out of order (e.g. form_rcs before linearize) */
    BA_ERR_NOT_SPD = 3,        /* a damped V_p, an RCS diagonal block or d^T S d was not positive */
    BA_ERR_NOT_CONVERGED = 4,  /* warning: PCG hit max_iter; its result is still returned */
    BA_ERR_OUT_OF_MEMORY = 5,  /* device allocation failed (or the workspace cap was exceeded) */
    BA_ERR_DEVICE = 6,         /* a HIP runtime call failed */
    BA_ERR_RANGE = 7           /* a Jacobian entry does not fit the record type (above 3.4e38 for
                                  the FP32 records of mixed precision) or a residual is not finite */
} ba_status;

enum { BA_FP64 = 0, BA_MIXED = 1 };
/* Preconditioners of ba_pcg_solve / ba_lm_step:
 *   BLOCK_JACOBI: M = blockdiag(S_ii) (Sec. 3.2);
 *   LEARNED: the learned correction of block-Jacobi (ba_set_preconditioner_net);
 *   FSAI: factorised sparse approximate inverse M^-1 = G^T G, G block-lower-
 *     triangular on the lower RCS pattern (at most 27 lower neighbours per
 *     row, those with the most common points), recomputed after every
 *     formation from local FP32 factorisations; see ba_get_fsai;
 *   LEARNED_FSAI: the same pattern and apply, with G emitted by the learned
 *     network's factorised head (ba_set_preconditioner_net). */
enum { BA_PRECOND_BLOCK_JACOBI = 0, BA_PRECOND_LEARNED = 1, BA_PRECOND_FSAI = 2, BA_PRECOND_LEARNED_FSAI = 3 };

typedef struct ba_ctx ba_ctx;

typedef struct ba_problem_desc {
    int32_t n_cams;             /* cameras, > 0 */
    int32_t n_pts;              /* points, > 0 */
    int64_t n_obs;              /* observations, 0 < n_obs < 2^31 */
    const int32_t* obs_cam;     /* device [n_obs]: camera of each observation */
    const int32_t* obs_pt;      /* device [n_obs]: point of each observation */
    const double* obs_uv;       /* device [2][n_obs]: observed u (row 0) and v (row 1), pixels */
    const uint8_t* cam_fixed;   /* device [n_cams] or NULL: non-zero = camera held fixed */
    int32_t precision;          /* BA_FP64 or BA_MIXED (FP32 Jacobian / Schur operands) */
    int32_t reserved;
    void* stream;               /* hipStream_t for all work of this context (NULL = default) */
    size_t workspace_cap;       /* max device bytes the context may allocate, 0 = unlimited */
} ba_problem_desc;

/* Validates the observations and builds the co-visibility pattern once
 * (Sec. 4: block (i, j) is non-zero iff cameras i and j share a point).
 * Requirements: indices in range, finite pixels, no repeated (camera, point)
 * pair, every point observed at least twice (Eq. (3) needs two views).
 * Tracks of up to 64 observations are handled one wave per chunk of tracks,
 * longer ones one workgroup per point, with the same results to rounding.
 * The context copies the observations (the caller may free them on return)
 * and owns all workspace.  The host part of the build runs on up to 16
 * threads (BA_THREADS in the environment sets the count; the result does not
 * depend on it); BA_TIMING=1 prints the duration of each phase to stderr.
 * Errors: BA_ERR_INVALID_ARG, BA_ERR_OUT_OF_MEMORY, BA_ERR_DEVICE; *out is
 * NULL on error and the message is available from ba_last_error(NULL). */
ba_status ba_create(const ba_problem_desc* desc, ba_ctx** out);

/* Shared intrinsics (Sec. 4.1 counts c = 11 unknowns per camera, 6 exterior
 * and 5 interior; Table 2's datasets have fewer physical cameras than
 * images): image i has exterior parameters [w (3) axis-angle, t (3)] and is
 * taken by physical camera img_cam[i], whose interior parameters
 * [f, cx, cy, k1, k2] all its images share; pixel = (f d x + cx, f d y + cy)
 * with x, y, d as above.  In a context made by ba_create_shared the
 * parameter array `cams` of ba_linearize and ba_lm_step is device
 * [n_imgs * 6 + n_phys * 5]: the exterior parameters of every image, then the
 * interior parameters of every physical camera.  RCS rows are the free
 * images (exterior block in slots 0..5 of the row's 9) followed by the
 * physical cameras (interior block in slots 0..4); the unused slots carry an
 * identity diagonal and a zero right-hand side, so their solution is 0.
 * Block (u, v) is present iff a point is observed through both rows (an
 * image's row and its camera's row always are).  FP64 only; PCG with
 * block-Jacobi or FSAI (no deflation, no learned network), no
 * re-triangulation, no ba_get_jacobians or ba_triangulate.  Other fields and
 * errors as in ba_problem_desc / ba_create; img_cam entries outside
 * [0, n_phys) give BA_ERR_INVALID_ARG. */
typedef struct ba_shared_desc {
    int32_t n_imgs;             /* images, > 0 */
    int32_t n_phys;             /* physical cameras, > 0 */
    int32_t n_pts;              /* points, > 0 */
    int32_t reserved;           /* 0 */
    int64_t n_obs;              /* observations, 0 < n_obs < 2^30 */
    const int32_t* obs_img;     /* device [n_obs]: image of each observation */
    const int32_t* obs_pt;      /* device [n_obs] */
    const double* obs_uv;       /* device [2][n_obs] */
    const int32_t* img_cam;     /* device [n_imgs]: physical camera of each image */
    const uint8_t* img_fixed;   /* device [n_imgs] or NULL: exterior held fixed */
    void* stream;
    size_t workspace_cap;
} ba_shared_desc;

ba_status ba_create_shared(const ba_shared_desc* desc, ba_ctx** out);

/* Frees the context and its device workspace.  NULL is a no-op. */
void ba_destroy(ba_ctx* ctx);

/* Sec. 3.1: residuals e and Jacobian blocks J_c (2x9) and J_p (2x3) of every
 * observation at cams (device [n_cams][9]) and pts (device [n_pts][3]);
 * cost F = 1/2 sum |e|^2 in FP64 is written to *cost_host when non-NULL
 * (this synchronises; then BA_ERR_RANGE is returned if a Jacobian entry
 * does not fit the record type or a residual is not finite, and
 * ba_form_rcs reports it in any case).  The parameters are read during the
 * call only. */
ba_status ba_linearize(ba_ctx* ctx, const double* cams, const double* pts, double* cost_host);

/* Eq. (3)-(4), Sec. 5: forms the RCS S = U* - W V*^-1 W^T and its right-hand
 * side b = l_c - W V*^-1 l_p from the last linearization with damping
 * lambda >= 0, plus the block-Jacobi factors of its diagonal blocks.
 * Errors: BA_ERR_STATE (no linearization), BA_ERR_INVALID_ARG (lambda < 0 or
 * not finite), BA_ERR_RANGE (the linearization did not fit the records),
 * BA_ERR_NOT_SPD (a V*_p or S_ii is not positive definite). */
ba_status ba_form_rcs(ba_ctx* ctx, double lambda);

typedef struct ba_pcg_opts {
    double tol;                 /* stop when |r_k| / |r_0| <= tol (default 1e-6) */
    int32_t max_iter;           /* iteration cap (default 1000) */
    int32_t precond;            /* BA_PRECOND_BLOCK_JACOBI, _LEARNED, _FSAI or _LEARNED_FSAI */
    const double* x0;           /* device [n_rows][9] initial guess or NULL (zero) */
    int32_t deflate;            /* 1: deflate the similarity gauge (see ba_get_gauge) */
    int32_t solver_fp32;        /* 1: the products with S read an FP32 copy of S (rounded
                                   once from the FP64 RCS); vectors, scalar products and
                                   the stop test stay FP64.  PCG then solves the system of
                                   that rounded S (relative entry error <= 2^-24). */
    int32_t product;            /* layout of the iteration's product S z (Sec. 6.2):
                                   BA_PRODUCT_AUTO (0), _FULL or _UPPER, see below */
    int32_t reserved;           /* 0 */
} ba_pcg_opts;

/* The product S z of a PCG iteration.  FULL: every block row of both
 * triangles (a copy of S made after each formation) is gathered by its own
 * wave, so each stored block is read twice.  UPPER: each stored upper block
 * S_rs (s >= r) is read once; its wave forms S_rs z_s for row r and
 * S_rs^T z_r for row s, the latter is written per block and a second kernel
 * sums them per row in a fixed order (72 extra bytes written and read per
 * block, against 648 (FP64) or 324 (FP32) bytes of a second block read).
 * Both are deterministic; they differ only in the summation order.  AUTO
 * takes UPPER when the copy of both triangles would exceed 256 MiB (about
 * the GPU's last-level cache), FULL otherwise (one kernel less per
 * iteration on small systems).  A factorised preconditioner (FSAI or the
 * learned factor, M^-1 = G^T G) is applied with the same layout: FULL reads
 * G (FP32) by rows and a transposed copy; UPPER reads each block of G once
 * from an FP16 copy (G D^-1 with D = diag(S)^-1/2, one FP32 scale per
 * block), so the preconditioner differs from FULL's by that rounding (M
 * stays SPD; PCG converges to the same solution). */
enum { BA_PRODUCT_AUTO = 0, BA_PRODUCT_FULL = 1, BA_PRODUCT_UPPER = 2, BA_PRODUCT_CSR = 3 };

typedef struct ba_pcg_info {
    int32_t iters;              /* CG iterations (matrix-vector products) done */
    int32_t status;             /* BA_OK, BA_ERR_NOT_CONVERGED or BA_ERR_NOT_SPD */
    double relres;              /* final |r| / |r_0| */
    double ms;                  /* device time of the solve */
    int32_t precond_fallback;   /* 1: the learned preconditioner failed (d^T S d <= 0 or a
                                   non-finite residual) and the result is block-Jacobi's */
    int32_t reserved;
} ba_pcg_info;

/* Sec. 3.2, Eq. (6)-(7): preconditioned CG on S dxc = b with M = the
 * block-diagonal of S (or the learned preconditioner, see below); result in
 * dxc (device [n_rows][9]).  opts may be NULL for the defaults.  Returns
 * BA_ERR_NOT_CONVERGED (dxc still valid) or BA_ERR_NOT_SPD as warnings/errors;
 * BA_ERR_STATE without a formed RCS.  A learned preconditioner that fails
 * (d^T S d <= 0, or a non-finite residual) is replaced by block-Jacobi for
 * the same solve, reported in info->precond_fallback. */
ba_status ba_pcg_solve(ba_ctx* ctx, const ba_pcg_opts* opts, double* dxc, ba_pcg_info* info_host);

/* Sec. 6.2: y = S x with the RCS formed last, computed as one product of a
 * PCG iteration (layout `product`, BA_PRODUCT_*, and with solver_fp32 = 1
 * the FP32 copy of S).  BA_PRODUCT_CSR instead multiplies with a scalar
 * CSR copy of both triangles (the format of Sec. 4.1 Eq. (8) that BSMC is
 * compared with; built from the blocks on first use after each formation,
 * FP64 only, one wave per scalar row; not a PCG layout).  x, y: distinct
 * device arrays [n_rows][9], owned by the caller.  Synchronises the context
 * stream.  Errors: BA_ERR_STATE (no RCS), BA_ERR_INVALID_ARG (null or
 * identical arrays, unknown layout, CSR with solver_fp32). */
ba_status ba_rcs_product(ba_ctx* ctx, const double* x, double* y, int32_t product, int32_t solver_fp32);

/* Eq. (5): dxp = V*^-1 (l_p - sum_i W_ip^T dxc_i) for every point (device
 * [n_pts][3]) from the RCS formed last.  dxc: device [n_rows][9]. */
ba_status ba_back_substitute(ba_ctx* ctx, const double* dxc, double* dxp);

typedef struct ba_lm_state {    /* caller-owned; it is the checkpoint of an LM run */
    double lambda;              /* damping; start e.g. at 1e-4 */
    double nu;                  /* rejection multiplier; start at 2 */
    int32_t iter;               /* attempts made so far */
    int32_t flags;              /* bit 0: the context's linearization is current for the
                                   parameters passed next (set by ba_lm_step after a
                                   rejection; clear it whenever the parameters change) */
} ba_lm_state;

typedef struct ba_lm_opts {
    double pcg_tol;             /* default 1e-6 */
    int32_t pcg_max_iter;       /* default 1000 */
    int32_t precond;            /* BA_PRECOND_BLOCK_JACOBI, _LEARNED, _FSAI or _LEARNED_FSAI */
    int32_t deflate;            /* 1: deflated PCG on the similarity gauge */
    int32_t solver_fp32;        /* 1: PCG products with an FP32 copy of S (see ba_pcg_opts) */
    int32_t product;            /* BA_PRODUCT_AUTO, _FULL or _UPPER (see ba_pcg_opts) */
    int32_t retriangulate;      /* 0: points by Eq. (5); k in 1..100: after Eq. (5) the points
                                   are re-triangulated with the candidate cameras (ba_triangulate,
                                   k Gauss-Newton steps from the Eq. (5) points); the gain ratio
                                   and the update then use those points */
} ba_lm_opts;

typedef struct ba_lm_info {
    double cost;                /* F at the parameters passed in */
    double cost_new;            /* F at the candidate x + dx */
    double rho;                 /* gain ratio (F - F') / (dx^T l - 1/2 |J dx|^2) */
    double model_decrease;      /* dx^T l - 1/2 |J dx|^2 */
    double pcg_relres;
    int32_t pcg_iters;
    int32_t pcg_status;
    int32_t accepted;           /* 1 if the step was taken */
    int32_t stop;               /* 1 if an accepted step lowered F by < 1e-12 relative */
    double ms_linearize, ms_form_rcs, ms_pcg, ms_back_substitute, ms_evaluate, ms_total;
    double ms_precond;          /* learned preconditioner inference (0 for block-Jacobi) */
    int32_t precond_fallback;   /* 1: the learned preconditioner failed on this step's RCS
                                   (d^T S d <= 0 or a non-finite residual) and the step was
                                   solved again with block-Jacobi */
    int32_t tri_failed;         /* points whose re-triangulation failed (they keep their last
                                   iterate; 0 without retriangulate) */
} ba_lm_info;

/* One LM iteration (Eq. (1) solved through Eq. (4)-(7) and (5)): linearize
 * (skipped when state->flags bit 0 is set), form the RCS with state->lambda,
 * PCG, back-substitute, evaluate F at x + dx and the predicted decrease.
 * Accepted iff the predicted decrease is positive and F' < F; then cams and
 * pts (device, updated in place) take the step and
 * lambda *= max(1/3, 1 - (2 rho - 1)^3), nu = 2; otherwise lambda *= nu,
 * nu *= 2 and the parameters are untouched.  Every attempt counts one
 * iteration.  A learned preconditioner that fails on the step's RCS is
 * replaced by block-Jacobi within the step (info->precond_fallback).
 * BA_ERR_RANGE: the linearization did not fit the records (see
 * ba_linearize); no step is taken and state is unchanged.
 * opts may be NULL for the defaults. */
ba_status ba_lm_step(ba_ctx* ctx, double* cams, double* pts, ba_lm_state* state,
                     const ba_lm_opts* opts, ba_lm_info* info_host);

/* Re-triangulation, the alternative to Eq. (5) of Sec. 3.1 (points
 * re-estimated from the camera poses): every point of the context is
 * re-estimated from its observations with the cameras cams (device
 * [n_cams][9]) held fixed.  Start: the given pts (device [n_pts][3]), or
 * with linear_init = 1 a linear multi-view solve (each pixel undistorted by
 * Newton's method on r (1 + k1 r^2 + k2 r^4) = |pixel| / f, then the
 * least-squares point of the equations (x R_3 - R_1) X = t_1 - x t_3,
 * (y R_3 - R_2) X = t_2 - y t_3); then n_gn (0..100) Gauss-Newton steps on
 * the point's reprojection error.  pts is overwritten with the result; a
 * point whose 3x3 normal matrix is not positive definite keeps its start
 * (its last iterate) and is counted in *n_failed (host, may be NULL).
 * Synchronises the context stream. */
ba_status ba_triangulate(ba_ctx* ctx, const double* cams, double* pts, int32_t linear_init, int32_t n_gn,
                         int64_t* n_failed);

/* Projection of Sec. 3.1's camera model, without a context: uv (device
 * [2][n_obs]) = pixel of point obs_pt[k] in camera obs_cam[k] (+ noise
 * (device [2][n_obs]) when not NULL).  All pointers are device memory; no
 * validation beyond n_obs >= 0. */
ba_status ba_project(const double* cams, const double* pts, const int32_t* obs_cam,
                     const int32_t* obs_pt, int64_t n_obs, const double* noise,
                     double* uv, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the cost
 * F = 1/2 sum |e|^2 that ba_linearize returns, without a context.  All
 * pointers are device memory: cams [n_cams][9], pts [n_pts][3], obs_cam and
 * obs_pt [n_obs], uv [2][n_obs]; *cost (one double) receives F.  The work is
 * enqueued on stream (NULL = default) and nothing is allocated: the partial
 * sums (one per 1,024 observations) go to a 1 MiB device buffer that the
 * library holds on each GPU until the process ends and that every call on
 * that GPU overwrites, so calls that overlap on one GPU race.  Errors:
 * BA_ERR_INVALID_ARG for n_obs < 0, n_obs > 134,217,728 (the buffer's
 * limit), a NULL cost or a NULL input with n_obs > 0; BA_ERR_DEVICE if the
 * buffer's address cannot be taken or the launch fails. */
ba_status ba_cost_noalloc(const double* cams, const double* pts, const int32_t* obs_cam, const int32_t* obs_pt,
                          const double* uv, int64_t n_obs, double* cost, void* stream);

typedef struct ba_sizes {
    int32_t n_cams, n_pts, n_rows, precision;
    int64_t n_obs, n_blk, n_pairs;      /* n_pairs: off-diagonal co-observations (triples) */
    int64_t device_bytes;               /* device workspace held by the context */
} ba_sizes;

ba_status ba_get_sizes(const ba_ctx* ctx, ba_sizes* out);

/* Host copies of the pattern: row_ptr [n_rows+1], col_idx [n_blk]; either may be NULL. */
ba_status ba_get_pattern(ba_ctx* ctx, int64_t* row_ptr, int32_t* col_idx);

/* Host copies of the last formed RCS: blocks [n_blk][81], rhs [n_rows][9]; either may be NULL. */
ba_status ba_get_rcs(ba_ctx* ctx, double* blk, double* rhs);

/* Bytes of the RCS in each storage layout (Sec. 4.1): bsmc_bytes = the
 * upper 9x9 blocks (FP64) + one column index per block + the block-row
 * pointer (Eq. (9) counts three indices per block); full_bytes = the
 * two-triangle copy of the FULL product (blocks, column and source index
 * per entry, row pointer); csr_nnz = 81 (2 n_blk - n_rows) scalar
 * non-zeros of both triangles and csr_bytes = 12 bytes per non-zero + the
 * scalar row pointer (exactly Eq. (8) with c = 9). */
typedef struct ba_store_sizes {
    int64_t bsmc_bytes, full_bytes, csr_nnz, csr_bytes;
} ba_store_sizes;
ba_status ba_get_store_sizes(const ba_ctx* ctx, ba_store_sizes* out);

/* Host copy of the CSR copy of the last formed RCS (built if needed):
 * row_ptr [9 n_rows + 1], col [nnz] ascending within each scalar row, val
 * [nnz] FP64; *nnz receives the count.  Any pointer may be NULL. */
ba_status ba_get_csr(ba_ctx* ctx, int32_t* row_ptr, int32_t* col, double* val, int64_t* nnz);

/* Host copies of the last linearization in the caller's observation order:
 * J [n_obs][24] = J_c row 0 (9), J_c row 1 (9), J_p row 0 (3), J_p row 1 (3)
 * (converted to FP64 in mixed precision), e [n_obs][2]; either may be NULL.
 * After ba_lm_step J_p is formed as K L^T from the stored K = J_p L^-T and
 * the point's Cholesky factor L (the step's linearization does not store
 * J_p), so it equals the Jacobian to rounding. */
ba_status ba_get_jacobians(ba_ctx* ctx, double* J, double* e);

/* Host copy (FP32, [n_blk][81], row-major 9x9) of the factor G used by the
 * last FSAI or LEARNED_FSAI solve on the current RCS, in the slots of the
 * RCS blocks: the slot of upper block
 * (s, c), s < c, holds G_cs; a diagonal slot holds G_ss (lower triangular,
 * positive diagonal); slots of lower neighbours beyond the per-row limit
 * hold zeros.  Definition (Kolotilina-Yeremin): row i of G is zero outside
 * its set J_i and satisfies (G S)_ij = 0 for j in J_i, j != i, and
 * (G S G^T)_ii = I (for FSAI).  BA_ERR_STATE before the first such solve. */
ba_status ba_get_fsai(ba_ctx* ctx, float* G);

/* Gauge deflation.  A similarity transform of the whole scene leaves every
 * projection of Eq. (1) unchanged, so its seven generators (three rotations,
 * three translations, one scale) are null vectors of J; their camera parts
 * W [n_rows][7][9] (column order: rotation x, y, z, translation x, y, z,
 * scale) are null vectors of the undamped RCS of Eq. (4):
 *   rotation k:    dw = -J_r(w)^-1 e_k  (J_r: right Jacobian of the
 *                  axis-angle map), dt = 0;
 *   translation k: dt = -R(w) e_k;   scale: dt = t;   f, k1, k2 fixed.
 * With deflate = 1, PCG is the deflated CG of Saad, Yeung, Erhel and
 * Guyomarc'h on span(W): the start is corrected so that W^T r_0 = 0 and
 * every search direction is kept S-orthogonal to W.  The iterate converges
 * to the same S^-1 b; with small damping the gauge directions are the
 * slowest ones, so deflation removes most of the iterations they cost.
 * ba_get_gauge copies W (FP64) for the camera parameters of the last
 * linearization.  BA_ERR_STATE without a formed RCS. */
ba_status ba_get_gauge(ba_ctx* ctx, double* W);

/* Device time in ms of the stages of the last formation:
 * [0] linearize, [1] point stage, [2] off-diagonal pair stage, [3] diagonal stage. */
ba_status ba_get_stage_ms(ba_ctx* ctx, double* ms4);

/* ------------------------------------------------------------------------
 * Learned correction to block-Jacobi (extension of Sec. 3.2's block-diagonal
 * preconditioner).  A message-passing network over the camera-pair graph of
 * the RCS (blocks (i, j) non-zero iff cameras share points, Sec. 4) outputs
 * per camera a lower-triangular Lt_i with exp(.) diagonal; the preconditioner
 * blocks are P_i = L_i^-T Lt_i Lt_i^T L_i^-1 with S_ii = L_i L_i^T, SPD by
 * construction, and equal to S_ii^-1 (block-Jacobi) when Lt_i = I.
 * Parameters: a flat FP32 vector of ba_gnn_param_count() values in the order
 *   Wn[64][64], bn[64], We[96][64], be[64],
 *   3 x (M_l[192][64], c_l[64], U_l[128][64], u_l[64]), Wd[64][48], bd[48],
 *   Wo1[192][128], bo1[128], Wo2[128][96], bo2[96], ao[96] (factorised head,
 *   below); 112,496 values in all
 * (row-major, y = x W + b).  Node input (64): the 36 strictly-upper entries
 * of diag(S_ii)^-1/2 S_ii diag(S_ii)^-1/2, then log S_ii[r][r] minus their
 * mean (9), zero padding.  Edge input i->j (96): L_i^-1 S_ij L_j^-T
 * row-major (81), zero padding.  Layers: h = relu(x Wn + bn),
 * g = relu(e We + be); 3 x { m_ij = relu([h_i, h_j, g_ij] M_l + c_l),
 * a_i = mean_j m_ij, h_i += relu([h_i, a_i] U_l + u_l) }; o = h Wd + bd;
 * Lt diagonal exp(o[0..8]), strict lower row-major o[9..44].  Dense layers
 * use bf16 operands with FP32 accumulation.  Loss (training): Hutchinson
 * estimate of |B A - I|_F^2 / (9 n) with A = blockdiag(L)^-1 S blockdiag(L)^-T,
 * B = blockdiag(Lt Lt^T) and Rademacher probes.
 * Factorised head (edge variant, FSAI pattern): M^-1 = G^T G with G block-
 * lower-triangular on the sets J_i of BA_PRECOND_FSAI; in normalised
 * coordinates Ghat = G blockdiag(L), Ghat_ii = Lt_i and, for j in J_i, j < i,
 *   z_ij = relu([h_i, h_j, g_ij] Wo1 + bo1)                (128 values),
 *   Ghat_ij = reshape(z_ij Wo2 + bo2)[:81] - ao[:81] (elementwise) L_i^-1 S_ij L_j^-T,
 * (h after the third layer), with Wo1[192][128], bo1[128], Wo2[128][96],
 * bo2[96], ao[96] at the end of the parameters above (Wo2, bo2 and ao
 * zero: block-Jacobi).  Its loss is the Kaporin functional
 * (1/(9n)) sum_i [tr(Ghat_i Ahat[J_i,J_i] Ghat_i^T) - 2 log det Ghat_ii],
 * minimised over the pattern by the exact FSAI factor.
 * A ba_gnn runs its work on its stream (NULL = default); a network and the
 * graphs it is used with must not be used concurrently from two threads.
 * ------------------------------------------------------------------------ */
typedef struct ba_gnn ba_gnn;
typedef struct ba_gnn_graph ba_gnn_graph;

int64_t ba_gnn_param_count(void);

/* Copies params (host FP32, ba_gnn_param_count() values); Adam state zero. */
ba_status ba_gnn_create(const float* params, void* stream, ba_gnn** out);
void ba_gnn_destroy(ba_gnn* net);
/* Replaces the parameters (host FP32) and resets the optimiser state. */
ba_status ba_gnn_set_params(ba_gnn* net, const float* params);
/* Host copy of the FP32 master parameters. */
ba_status ba_gnn_get_params(ba_gnn* net, float* params);

/* Network input of one RCS instance: from the context's last formed RCS
 * (device work on the context stream), or from host arrays row_ptr
 * [n_rows+1] (int64), col_idx [n_blk] (diagonal first in each row), blocks
 * [n_blk][81] FP64 and, optionally, blk_pairs [n_blk] (common points of
 * each block; needed by the factorised head, NULL otherwise).
 * BA_ERR_NOT_SPD if a diagonal block is not SPD. */
ba_status ba_gnn_graph_from_ctx(ba_ctx* ctx, ba_gnn_graph** out);
ba_status ba_gnn_graph_from_host(int32_t n_rows, const int64_t* row_ptr, const int32_t* col_idx,
                                 const double* blk, const int32_t* blk_pairs, ba_gnn_graph** out);
void ba_gnn_graph_destroy(ba_gnn_graph* graph);

/* Loss and (if grad is not NULL) its gradient (host FP32, param order) for
 * n_probes Rademacher probes: host probes [n_probes][n_rows][9] (+-1), or
 * NULL to draw them on the device from seed.  Parameters are unchanged. */
ba_status ba_gnn_loss_grad(ba_gnn* net, ba_gnn_graph* graph, int32_t n_probes, const float* probes,
                           uint64_t seed, double* loss, float* grad);

/* One Adam step (beta 0.9 / 0.999, eps 1e-8, FP32 master weights) on the mean
 * gradient over n_graphs graphs, probes drawn from seed; *loss = mean loss
 * before the step. */
ba_status ba_gnn_train_step(ba_gnn* net, ba_gnn_graph* const* graphs, int32_t n_graphs, int32_t n_probes,
                            uint64_t seed, float lr, double* loss);

/* Host copy of the preconditioner blocks P [n_rows][81] for a graph. */
ba_status ba_gnn_preconditioner(ba_gnn* net, ba_gnn_graph* graph, double* P);

/* Factorised head: Kaporin loss and (if grad is not NULL) its gradient;
 * one Adam step on the mean over n_graphs graphs; and the factor G of a
 * graph (host FP32 [n_blk][81] in the RCS block slots, as ba_get_fsai).
 * BA_ERR_STATE for a graph built without common-point counts. */
ba_status ba_gnn_fsai_loss_grad(ba_gnn* net, ba_gnn_graph* graph, double* loss, float* grad);
ba_status ba_gnn_fsai_train_step(ba_gnn* net, ba_gnn_graph* const* graphs, int32_t n_graphs, float lr, double* loss);
ba_status ba_gnn_fsai_factor(ba_gnn* net, ba_gnn_graph* graph, float* G);

/* Uses net (not copied; must outlive its use) for BA_PRECOND_LEARNED and
 * BA_PRECOND_LEARNED_FSAI in ba_pcg_solve and ba_lm_step of ctx: after each formation the network runs
 * on the RCS on the context stream.  NULL detaches. */
ba_status ba_set_preconditioner_net(ba_ctx* ctx, ba_gnn* net);

/* C[M][N] = A[M][K] B[K][N] on the device's bf16 matrix cores (FP32
 * accumulation); host row-major arrays, A and B as bf16 bit patterns. */
ba_status ba_gemm_bf16(int32_t M, int32_t N, int32_t K, const uint16_t* A, const uint16_t* B, float* C);

const char* ba_gnn_last_error(void);

const char* ba_status_str(ba_status s);

/* Last error message of ctx, or of the last failed ba_create when ctx is NULL. */
const char* ba_last_error(const ba_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* BA_H */
