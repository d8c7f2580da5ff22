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
    BA_ERR_DEVICE = 6          /* a HIP runtime call failed */
} ba_status;

enum { BA_FP64 = 0, BA_MIXED = 1 };
enum { BA_PRECOND_BLOCK_JACOBI = 0, BA_PRECOND_LEARNED = 1 };

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
 * pair, every point observed 2..64 times.  The context copies the
 * observations (the caller may free them on return) and owns all workspace.
 * Errors: BA_ERR_INVALID_ARG, BA_ERR_OUT_OF_MEMORY, BA_ERR_DEVICE; *out is
 * NULL on error and the message is available from ba_last_error(NULL). */
ba_status ba_create(const ba_problem_desc* desc, ba_ctx** out);

/* Frees the context and its device workspace.  NULL is a no-op. */
void ba_destroy(ba_ctx* ctx);

/* Sec. 3.1: residuals e and Jacobian blocks J_c (2x9) and J_p (2x3) of every
 * observation at cams (device [n_cams][9]) and pts (device [n_pts][3]);
 * cost F = 1/2 sum |e|^2 in FP64 is written to *cost_host when non-NULL
 * (this synchronises).  The parameters are read during the call only. */
ba_status ba_linearize(ba_ctx* ctx, const double* cams, const double* pts, double* cost_host);

/* Eq. (3)-(4), Sec. 5: forms the RCS S = U* - W V*^-1 W^T and its right-hand
 * side b = l_c - W V*^-1 l_p from the last linearization with damping
 * lambda >= 0, plus the block-Jacobi factors of its diagonal blocks.
 * Errors: BA_ERR_STATE (no linearization), BA_ERR_INVALID_ARG (lambda < 0 or
 * not finite), BA_ERR_NOT_SPD (a V*_p or S_ii is not positive definite). */
ba_status ba_form_rcs(ba_ctx* ctx, double lambda);

typedef struct ba_pcg_opts {
    double tol;                 /* stop when |r_k| / |r_0| <= tol (default 1e-6) */
    int32_t max_iter;           /* iteration cap (default 1000) */
    int32_t precond;            /* BA_PRECOND_BLOCK_JACOBI or BA_PRECOND_LEARNED */
    const double* x0;           /* device [n_rows][9] initial guess or NULL (zero) */
} ba_pcg_opts;

typedef struct ba_pcg_info {
    int32_t iters;              /* CG iterations (matrix-vector products) done */
    int32_t status;             /* BA_OK, BA_ERR_NOT_CONVERGED or BA_ERR_NOT_SPD */
    double relres;              /* final |r| / |r_0| */
    double ms;                  /* device time of the solve */
} ba_pcg_info;

/* Sec. 3.2, Eq. (6)-(7): preconditioned CG on S dxc = b with M = the
 * block-diagonal of S (or the learned preconditioner, see below); result in
 * dxc (device [n_rows][9]).  opts may be NULL for the defaults.  Returns
 * BA_ERR_NOT_CONVERGED (dxc still valid) or BA_ERR_NOT_SPD as warnings/errors;
 * BA_ERR_STATE without a formed RCS. */
ba_status ba_pcg_solve(ba_ctx* ctx, const ba_pcg_opts* opts, double* dxc, ba_pcg_info* info_host);

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
    int32_t precond;            /* BA_PRECOND_BLOCK_JACOBI or BA_PRECOND_LEARNED */
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
} ba_lm_info;

/* One LM iteration (Eq. (1) solved through Eq. (4)-(7) and (5)): linearize
 * (skipped when state->flags bit 0 is set), form the RCS with state->lambda,
 * PCG, back-substitute, evaluate F at x + dx and the predicted decrease.
 * Accepted iff the predicted decrease is positive and F' < F; then cams and
 * pts (device, updated in place) take the step and
 * lambda *= max(1/3, 1 - (2 rho - 1)^3), nu = 2; otherwise lambda *= nu,
 * nu *= 2 and the parameters are untouched.  Every attempt counts one
 * iteration.  opts may be NULL for the defaults. */
ba_status ba_lm_step(ba_ctx* ctx, double* cams, double* pts, ba_lm_state* state,
                     const ba_lm_opts* opts, ba_lm_info* info_host);

/* Projection of Sec. 3.1's camera model, without a context: uv (device
 * [2][n_obs]) = pixel of point obs_pt[k] in camera obs_cam[k] (+ noise
 * (device [2][n_obs]) when not NULL).  All pointers are device memory; no
 * validation beyond n_obs >= 0. */
ba_status ba_project(const double* cams, const double* pts, const int32_t* obs_cam,
                     const int32_t* obs_pt, int64_t n_obs, const double* noise,
                     double* uv, void* stream);

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

/* Host copies of the last linearization in the caller's observation order:
 * J [n_obs][24] = J_c row 0 (9), J_c row 1 (9), J_p row 0 (3), J_p row 1 (3)
 * (converted to FP64 in mixed precision), e [n_obs][2]; either may be NULL. */
ba_status ba_get_jacobians(ba_ctx* ctx, double* J, double* e);

/* Device time in ms of the stages of the last formation:
 * [0] linearize, [1] point stage, [2] off-diagonal pair stage, [3] diagonal stage. */
ba_status ba_get_stage_ms(ba_ctx* ctx, double* ms4);

const char* ba_status_str(ba_status s);

/* Last error message of ctx, or of the last failed ba_create when ctx is NULL. */
const char* ba_last_error(const ba_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif /* BA_H */
