/*
 * oracle.c -- plain FP64 CPU reference for exact Levenberg-Marquardt bundle
 * adjustment with the Schur-complement reduced camera system (RCS).
 *
 * TEST INFRASTRUCTURE ONLY.  It is called by the test-suite, by the smoke
 * check and by the CPU-baseline leg of the benchmark; the product library
 * never links, loads or calls it, and the two share no code.
 *
 * It is written to be checked by eye against the paper:
 *   - normal equations with Marquardt damping, Sec. 3.1 Eq. (1);
 *   - camera/point split U, V, W, l_c, l_p, Sec. 3.1 Eq. (3);
 *   - reduced camera system S = U - W V^-1 W^T, b = l_c - W V^-1 l_p, Eq. (4);
 *   - point back-substitution V dx_p = l_p - W^T dx_c, Eq. (5);
 *   - point-by-point RCS formation: per 3D point compute its Jacobian,
 *     Hessian and Schur complement and add the resulting sub-RCS, Sec. 5
 *     steps (1)-(3); points split into equal-size groups whose sub-RCSs are
 *     summed, Sec. 6.1;
 *   - block storage of the upper triangle only (BSMC), Sec. 4, located by
 *     (row, column) with a binary search inside the row, Table 1;
 *   - block-diagonal preconditioned CG with the recurrence of Sec. 3.2;
 *   - BSMC matrix-vector product split over block groups whose partial
 *     results are summed, Sec. 6.2.
 *
 * Readings where the paper is silent (camera model, damping form, PCG stop
 * test, LM schedule) are stated next to the code that takes them.
 *
 * Jacobians are computed by forward-mode dual numbers through the projection
 * function (no hand-derived derivative formulas).
 *
 * Camera: 9 parameters [w(3) axis-angle, t(3), f, k1, k2].  P = R(w) X + t,
 * x = P_x / P_z, y = P_y / P_z, r2 = x^2 + y^2, d = 1 + k1 r2 + k2 r2^2,
 * predicted pixel (f d x, f d y), residual e = predicted - observed.
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC oracle.c -o liboracle.so -lm
 * (no fast-math: IEEE semantics are part of the reference).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NCP 9   /* camera parameters */
#define ND 12   /* dual directions: 9 camera + 3 point */

/* ------------------------------------------------------------------------ */
/* forward-mode dual numbers                                                 */
/* ------------------------------------------------------------------------ */
typedef struct { double v; double d[ND]; } dual;

static dual dconst(double v) { dual r; r.v = v; memset(r.d, 0, sizeof r.d); return r; }
static dual dvar(double v, int k) { dual r = dconst(v); r.d[k] = 1.0; return r; }
static dual dadd(dual a, dual b) { dual r; r.v = a.v + b.v; for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] + b.d[k]; return r; }
static dual dsub(dual a, dual b) { dual r; r.v = a.v - b.v; for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] - b.d[k]; return r; }
static dual dmul(dual a, dual b) { dual r; r.v = a.v * b.v; for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k]; return r; }
static dual dscale(dual a, double s) { dual r; r.v = a.v * s; for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] * s; return r; }
static dual ddiv(dual a, dual b) {
    dual r; r.v = a.v / b.v;
    for (int k = 0; k < ND; ++k) r.d[k] = (a.d[k] - r.v * b.d[k]) / b.v;
    return r;
}
static dual dsin(dual a) { dual r; r.v = sin(a.v); double c = cos(a.v); for (int k = 0; k < ND; ++k) r.d[k] = c * a.d[k]; return r; }
static dual dsqrt(dual a) { dual r; r.v = sqrt(a.v); for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] / (2.0 * r.v); return r; }

static void dcross(const dual a[3], const dual b[3], dual out[3]) {
    dual o0 = dsub(dmul(a[1], b[2]), dmul(a[2], b[1]));
    dual o1 = dsub(dmul(a[2], b[0]), dmul(a[0], b[2]));
    dual o2 = dsub(dmul(a[0], b[1]), dmul(a[1], b[0]));
    out[0] = o0; out[1] = o1; out[2] = o2;
}

/* R(w) X by the Rodrigues formula R = I + sin(th) K + (1 - cos(th)) K^2 with
 * K the cross-product matrix of the unit axis k = w / th; 1 - cos(th) is
 * written 2 sin^2(th/2) to avoid cancellation.  Below th = 1e-8 the
 * second-order Taylor form R = I + [w]x + [w]x^2 / 2 is used (its error is
 * O(th^3)). */
static void rotate(const dual w[3], const dual X[3], dual out[3]) {
    double th2 = w[0].v * w[0].v + w[1].v * w[1].v + w[2].v * w[2].v;
    dual wx[3], wwx[3];
    if (sqrt(th2) < 1e-8) {
        dcross(w, X, wx);
        dcross(w, wx, wwx);
        for (int i = 0; i < 3; ++i) out[i] = dadd(dadd(X[i], wx[i]), dscale(wwx[i], 0.5));
        return;
    }
    dual s = dadd(dadd(dmul(w[0], w[0]), dmul(w[1], w[1])), dmul(w[2], w[2]));
    dual th = dsqrt(s);
    dual k[3] = { ddiv(w[0], th), ddiv(w[1], th), ddiv(w[2], th) };
    dual kx[3], kkx[3];
    dcross(k, X, kx);
    dcross(k, kx, kkx);
    dual sn = dsin(th);
    dual sh = dsin(dscale(th, 0.5));
    dual omc = dscale(dmul(sh, sh), 2.0);
    for (int i = 0; i < 3; ++i) out[i] = dadd(dadd(X[i], dmul(sn, kx[i])), dmul(omc, kkx[i]));
}

/* predicted pixel of point X in camera c, as duals in the 12 directions */
static void project_dual(const double* c, const double* Xv, dual out[2]) {
    dual w[3], X[3], P[3];
    for (int i = 0; i < 3; ++i) w[i] = dvar(c[i], i);
    for (int i = 0; i < 3; ++i) X[i] = dvar(Xv[i], 9 + i);
    rotate(w, X, P);
    for (int i = 0; i < 3; ++i) P[i] = dadd(P[i], dvar(c[3 + i], 3 + i));
    dual f = dvar(c[6], 6), k1 = dvar(c[7], 7), k2 = dvar(c[8], 8);
    dual x = ddiv(P[0], P[2]);
    dual y = ddiv(P[1], P[2]);
    dual r2 = dadd(dmul(x, x), dmul(y, y));
    dual d = dadd(dadd(dconst(1.0), dmul(k1, r2)), dmul(k2, dmul(r2, r2)));
    dual fd = dmul(f, d);
    out[0] = dmul(fd, x);
    out[1] = dmul(fd, y);
}

/* ------------------------------------------------------------------------ */
/* stateless entry points                                                     */
/* ------------------------------------------------------------------------ */

/* uv[0][k], uv[1][k] = projection of point obs_pt[k] in camera obs_cam[k]
 * (+ noise[.][k] if noise is not NULL). */
void orc_project(int64_t n_obs, const double* cams, const double* pts,
                 const int32_t* obs_cam, const int32_t* obs_pt,
                 const double* noise, double* uv) {
    #pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n_obs; ++k) {
        dual p[2];
        project_dual(cams + (int64_t)obs_cam[k] * NCP, pts + (int64_t)obs_pt[k] * 3, p);
        uv[k] = p[0].v + (noise ? noise[k] : 0.0);
        uv[n_obs + k] = p[1].v + (noise ? noise[n_obs + k] : 0.0);
    }
}

/* residuals e[k][2], Jacobians Jc[k][2][9] = de/dc, Jp[k][2][3] = de/dX
 * (any output may be NULL); returns F = 1/2 sum |e|^2. */
double orc_linearize(int64_t n_obs, const double* cams, const double* pts,
                     const int32_t* obs_cam, const int32_t* obs_pt, const double* uv,
                     double* e, double* Jc, double* Jp) {
    double F = 0.0;
    #pragma omp parallel for schedule(static) reduction(+:F)
    for (int64_t k = 0; k < n_obs; ++k) {
        dual p[2];
        project_dual(cams + (int64_t)obs_cam[k] * NCP, pts + (int64_t)obs_pt[k] * 3, p);
        double eu = p[0].v - uv[k], ev = p[1].v - uv[n_obs + k];
        if (e) { e[2 * k] = eu; e[2 * k + 1] = ev; }
        for (int r = 0; r < 2; ++r) {
            if (Jc) for (int j = 0; j < 9; ++j) Jc[k * 18 + r * 9 + j] = p[r].d[j];
            if (Jp) for (int j = 0; j < 3; ++j) Jp[k * 6 + r * 3 + j] = p[r].d[9 + j];
        }
        F += 0.5 * (eu * eu + ev * ev);
    }
    return F;
}

/* ------------------------------------------------------------------------ */
/* problem object                                                            */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t n_cams, n_pts;
    int64_t n_obs;
    int32_t *obs_cam, *obs_pt;
    double *uv;                 /* [2][n_obs] */
    int32_t n_rows;             /* RCS block rows = free cameras */
    int32_t *cam_row;           /* camera -> RCS row, -1 for fixed cameras */
    int64_t *pt_ptr, *pt_obs;   /* observations of each point */
    int64_t n_blk;
    int64_t *row_ptr;           /* BSMC: blocks of row r are row_ptr[r]..row_ptr[r+1] */
    int32_t *col_idx;           /* column of each block, ascending, diagonal first */
    double *e, *Jc, *Jp;        /* last linearization */
    double cost;
    int have_lin;
    double *blk, *rhs;          /* RCS blocks [n_blk][81] row-major, rhs [n_rows][9] */
    double *Vinv, *lp;          /* per point: (V*)^-1 [9], l_p [3] */
    int have_rcs;
    double lambda;
    int n_threads;
} orc_problem;

static int cmp_i64(const void* a, const void* b) {
    int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
    return (x > y) - (x < y);
}

void orc_destroy(orc_problem* P) {
    if (!P) return;
    free(P->obs_cam); free(P->obs_pt); free(P->uv); free(P->cam_row);
    free(P->pt_ptr); free(P->pt_obs); free(P->row_ptr); free(P->col_idx);
    free(P->e); free(P->Jc); free(P->Jp); free(P->blk); free(P->rhs);
    free(P->Vinv); free(P->lp);
    free(P);
}

/* Builds the point -> observation lists and the BSMC pattern: block (r, s),
 * r <= s, is present iff r == s or cameras of rows r and s share a point
 * (Sec. 4: a block is non-zero iff the two cameras have common points; only
 * the upper triangle is kept).  Returns NULL on invalid input. */
orc_problem* orc_create(int32_t n_cams, int32_t n_pts, int64_t n_obs,
                        const int32_t* obs_cam, const int32_t* obs_pt,
                        const double* uv, const uint8_t* cam_fixed, int32_t n_threads) {
    if (n_cams <= 0 || n_pts <= 0 || n_obs <= 0) return NULL;
    orc_problem* P = (orc_problem*)calloc(1, sizeof(orc_problem));
    P->n_cams = n_cams; P->n_pts = n_pts; P->n_obs = n_obs;
    P->n_threads = n_threads > 0 ? n_threads : 1;
    P->obs_cam = (int32_t*)malloc(sizeof(int32_t) * n_obs);
    P->obs_pt = (int32_t*)malloc(sizeof(int32_t) * n_obs);
    P->uv = (double*)malloc(sizeof(double) * 2 * n_obs);
    memcpy(P->obs_cam, obs_cam, sizeof(int32_t) * n_obs);
    memcpy(P->obs_pt, obs_pt, sizeof(int32_t) * n_obs);
    memcpy(P->uv, uv, sizeof(double) * 2 * n_obs);
    for (int64_t k = 0; k < n_obs; ++k)
        if (obs_cam[k] < 0 || obs_cam[k] >= n_cams || obs_pt[k] < 0 || obs_pt[k] >= n_pts) {
            orc_destroy(P); return NULL;
        }
    P->cam_row = (int32_t*)malloc(sizeof(int32_t) * n_cams);
    P->n_rows = 0;
    for (int32_t c = 0; c < n_cams; ++c)
        P->cam_row[c] = (cam_fixed && cam_fixed[c]) ? -1 : P->n_rows++;
    /* observations of each point, ordered by camera */
    P->pt_ptr = (int64_t*)calloc((size_t)n_pts + 1, sizeof(int64_t));
    for (int64_t k = 0; k < n_obs; ++k) P->pt_ptr[obs_pt[k] + 1]++;
    for (int32_t p = 0; p < n_pts; ++p) P->pt_ptr[p + 1] += P->pt_ptr[p];
    P->pt_obs = (int64_t*)malloc(sizeof(int64_t) * n_obs);
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * n_pts);
    for (int32_t p = 0; p < n_pts; ++p) fill[p] = P->pt_ptr[p];
    for (int64_t k = 0; k < n_obs; ++k) P->pt_obs[fill[obs_pt[k]]++] = k;
    free(fill);
    for (int32_t p = 0; p < n_pts; ++p) {   /* insertion sort by camera */
        int64_t b = P->pt_ptr[p], e = P->pt_ptr[p + 1];
        for (int64_t i = b + 1; i < e; ++i) {
            int64_t v = P->pt_obs[i]; int64_t j = i - 1;
            while (j >= b && obs_cam[P->pt_obs[j]] > obs_cam[v]) { P->pt_obs[j + 1] = P->pt_obs[j]; --j; }
            P->pt_obs[j + 1] = v;
        }
        for (int64_t i = b + 1; i < e; ++i)
            if (obs_cam[P->pt_obs[i]] == obs_cam[P->pt_obs[i - 1]]) { orc_destroy(P); return NULL; }
        if (e - b < 2) { orc_destroy(P); return NULL; }
    }
    /* pattern: all (r, s) keys, r <= s */
    int64_t n_keys = P->n_rows;
    for (int32_t p = 0; p < n_pts; ++p) {
        int64_t t = P->pt_ptr[p + 1] - P->pt_ptr[p];
        n_keys += t * (t - 1) / 2;
    }
    int64_t* keys = (int64_t*)malloc(sizeof(int64_t) * (n_keys > 0 ? n_keys : 1));
    int64_t nk = 0;
    for (int32_t r = 0; r < P->n_rows; ++r) keys[nk++] = (int64_t)r * P->n_rows + r;
    for (int32_t p = 0; p < n_pts; ++p)
        for (int64_t a = P->pt_ptr[p]; a < P->pt_ptr[p + 1]; ++a)
            for (int64_t b = a + 1; b < P->pt_ptr[p + 1]; ++b) {
                int32_t ra = P->cam_row[obs_cam[P->pt_obs[a]]], rb = P->cam_row[obs_cam[P->pt_obs[b]]];
                if (ra < 0 || rb < 0) continue;
                int32_t r = ra < rb ? ra : rb, s = ra < rb ? rb : ra;
                keys[nk++] = (int64_t)r * P->n_rows + s;
            }
    qsort(keys, (size_t)nk, sizeof(int64_t), cmp_i64);
    int64_t nu = 0;
    for (int64_t i = 0; i < nk; ++i)
        if (nu == 0 || keys[i] != keys[nu - 1]) keys[nu++] = keys[i];
    P->n_blk = nu;
    P->row_ptr = (int64_t*)calloc((size_t)P->n_rows + 1, sizeof(int64_t));
    P->col_idx = (int32_t*)malloc(sizeof(int32_t) * (nu > 0 ? nu : 1));
    for (int64_t i = 0; i < nu; ++i) {
        int32_t r = (int32_t)(keys[i] / P->n_rows);
        P->col_idx[i] = (int32_t)(keys[i] % P->n_rows);
        P->row_ptr[r + 1]++;
    }
    for (int32_t r = 0; r < P->n_rows; ++r) P->row_ptr[r + 1] += P->row_ptr[r];
    free(keys);
    P->e = (double*)malloc(sizeof(double) * 2 * n_obs);
    P->Jc = (double*)malloc(sizeof(double) * 18 * n_obs);
    P->Jp = (double*)malloc(sizeof(double) * 6 * n_obs);
    P->blk = (double*)malloc(sizeof(double) * 81 * (nu > 0 ? nu : 1));
    P->rhs = (double*)malloc(sizeof(double) * 9 * (P->n_rows > 0 ? P->n_rows : 1));
    P->Vinv = (double*)malloc(sizeof(double) * 9 * n_pts);
    P->lp = (double*)malloc(sizeof(double) * 3 * n_pts);
    return P;
}

int32_t orc_n_rows(const orc_problem* P) { return P->n_rows; }
int64_t orc_n_blk(const orc_problem* P) { return P->n_blk; }

void orc_get_pattern(const orc_problem* P, int64_t* row_ptr, int32_t* col_idx) {
    if (row_ptr) memcpy(row_ptr, P->row_ptr, sizeof(int64_t) * (P->n_rows + 1));
    if (col_idx) memcpy(col_idx, P->col_idx, sizeof(int32_t) * P->n_blk);
}

void orc_get_cam_row(const orc_problem* P, int32_t* cam_row) {
    memcpy(cam_row, P->cam_row, sizeof(int32_t) * P->n_cams);
}

/* BSMC block lookup (the second operation of Table 1): the block of (r, s) by binary search of
 * s inside row r; -1 if absent. */
static int64_t find_block(const orc_problem* P, int32_t r, int32_t s) {
    int64_t lo = P->row_ptr[r], hi = P->row_ptr[r + 1] - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) / 2;
        if (P->col_idx[mid] == s) return mid;
        if (P->col_idx[mid] < s) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

double orc_prob_linearize(orc_problem* P, const double* cams, const double* pts) {
    P->cost = orc_linearize(P->n_obs, cams, pts, P->obs_cam, P->obs_pt, P->uv, P->e, P->Jc, P->Jp);
    P->have_lin = 1;
    P->have_rcs = 0;
    return P->cost;
}

void orc_get_linearization(const orc_problem* P, double* e, double* Jc, double* Jp) {
    if (e) memcpy(e, P->e, sizeof(double) * 2 * P->n_obs);
    if (Jc) memcpy(Jc, P->Jc, sizeof(double) * 18 * P->n_obs);
    if (Jp) memcpy(Jp, P->Jp, sizeof(double) * 6 * P->n_obs);
}

/* inverse of a symmetric 3x3 by cofactors; returns 0 unless positive definite
 * (all leading principal minors > 0, Sylvester's criterion). */
static int inv3_spd(const double A[9], double Ai[9]) {
    double m1 = A[0];
    double m2 = A[0] * A[4] - A[1] * A[3];
    double c00 = A[4] * A[8] - A[5] * A[7];
    double c01 = A[5] * A[6] - A[3] * A[8];
    double c02 = A[3] * A[7] - A[4] * A[6];
    double det = A[0] * c00 + A[1] * c01 + A[2] * c02;
    if (!(m1 > 0.0) || !(m2 > 0.0) || !(det > 0.0)) return 0;
    Ai[0] = c00 / det;
    Ai[1] = (A[2] * A[7] - A[1] * A[8]) / det;
    Ai[2] = (A[1] * A[5] - A[2] * A[4]) / det;
    Ai[3] = c01 / det;
    Ai[4] = (A[0] * A[8] - A[2] * A[6]) / det;
    Ai[5] = (A[2] * A[3] - A[0] * A[5]) / det;
    Ai[6] = c02 / det;
    Ai[7] = (A[1] * A[6] - A[0] * A[7]) / det;
    Ai[8] = (A[0] * A[4] - A[1] * A[3]) / det;
    return 1;
}

/* Adds the sub-RCS of point p (Sec. 5 step (1)) into the group's arrays:
 *   V   = sum_a Jp_a^T Jp_a,   l_p = -sum_a Jp_a^T e_a,
 *   V*  = V + lambda diag(V)             (Marquardt damping, Eq. (1)),
 *   W_a = Jc_a^T Jp_a  (9x3),  Y_a = W_a (V*)^-1,
 *   U_i += Jc_a^T Jc_a,  b_i += -Jc_a^T e_a - Y_a l_p,
 *   S_ij -= Y_a W_b^T for every ordered pair of the track with row(a) <= row(b).
 * U is kept apart and damped once the sum over all points is complete. */
static int add_point(const orc_problem* P, int32_t p, double lambda,
                     double* blk, double* U, double* rhs) {
    int64_t b0 = P->pt_ptr[p], b1 = P->pt_ptr[p + 1];
    int64_t t = b1 - b0;
    double V[9] = {0}, lp[3] = {0}, Vs[9], Vi[9];
    for (int64_t q = b0; q < b1; ++q) {
        int64_t k = P->pt_obs[q];
        const double* Jp = P->Jp + k * 6;
        const double* e = P->e + 2 * k;
        for (int i = 0; i < 3; ++i) {
            for (int j = 0; j < 3; ++j) V[i * 3 + j] += Jp[i] * Jp[j] + Jp[3 + i] * Jp[3 + j];
            lp[i] -= Jp[i] * e[0] + Jp[3 + i] * e[1];
        }
    }
    memcpy(Vs, V, sizeof V);
    for (int i = 0; i < 3; ++i) Vs[i * 4] += lambda * V[i * 4];
    if (!inv3_spd(Vs, Vi)) return 0;
    memcpy(P->Vinv + (int64_t)p * 9, Vi, sizeof Vi);
    memcpy(P->lp + (int64_t)p * 3, lp, sizeof lp);
    double* W = (double*)malloc(sizeof(double) * 27 * t);
    double* Y = (double*)malloc(sizeof(double) * 27 * t);
    for (int64_t q = 0; q < t; ++q) {
        int64_t k = P->pt_obs[b0 + q];
        const double* Jc = P->Jc + k * 18;
        const double* Jp = P->Jp + k * 6;
        double* Wq = W + q * 27;
        double* Yq = Y + q * 27;
        for (int i = 0; i < 9; ++i)
            for (int j = 0; j < 3; ++j) Wq[i * 3 + j] = Jc[i] * Jp[j] + Jc[9 + i] * Jp[3 + j];
        for (int i = 0; i < 9; ++i)
            for (int j = 0; j < 3; ++j)
                Yq[i * 3 + j] = Wq[i * 3 + 0] * Vi[0 * 3 + j] + Wq[i * 3 + 1] * Vi[1 * 3 + j] + Wq[i * 3 + 2] * Vi[2 * 3 + j];
    }
    for (int64_t qa = 0; qa < t; ++qa) {
        int64_t ka = P->pt_obs[b0 + qa];
        int32_t ra = P->cam_row[P->obs_cam[ka]];
        if (ra < 0) continue;
        const double* Jc = P->Jc + ka * 18;
        const double* e = P->e + 2 * ka;
        const double* Ya = Y + qa * 27;
        double* Ui = U + (int64_t)ra * 81;
        double* bi = rhs + (int64_t)ra * 9;
        for (int i = 0; i < 9; ++i) {
            for (int j = 0; j < 9; ++j) Ui[i * 9 + j] += Jc[i] * Jc[j] + Jc[9 + i] * Jc[9 + j];
            bi[i] += -(Jc[i] * e[0] + Jc[9 + i] * e[1])
                     - (Ya[i * 3 + 0] * lp[0] + Ya[i * 3 + 1] * lp[1] + Ya[i * 3 + 2] * lp[2]);
        }
        for (int64_t qb = 0; qb < t; ++qb) {
            int64_t kb = P->pt_obs[b0 + qb];
            int32_t rb = P->cam_row[P->obs_cam[kb]];
            if (rb < ra) continue;   /* rb < 0 (fixed) included */
            int64_t blk_id = find_block(P, ra, rb);
            double* S = blk + blk_id * 81;
            const double* Wb = W + qb * 27;
            for (int i = 0; i < 9; ++i)
                for (int j = 0; j < 9; ++j)
                    S[i * 9 + j] -= Ya[i * 3 + 0] * Wb[j * 3 + 0] + Ya[i * 3 + 1] * Wb[j * 3 + 1] + Ya[i * 3 + 2] * Wb[j * 3 + 2];
        }
    }
    free(W); free(Y);
    return 1;
}

/* RCS formation (Sec. 5 and 6.1): the points are divided into n_groups groups
 * of equal point count; each group forms its sub-RCS point by point; the
 * global RCS is the sum of the sub-RCSs (in group order).  Finally
 * S_ii += U_i + lambda diag(U_i).  n_groups <= 0 means one group per thread.
 * Returns 0 on success, 3 if some damped V_p is not positive definite. */
int orc_form_rcs(orc_problem* P, double lambda, int32_t n_groups) {
    if (!P->have_lin) return 2;
    int G = n_groups > 0 ? n_groups : P->n_threads;
    int64_t nb = P->n_blk, nr = P->n_rows;
    size_t per = (size_t)(nb * 81 + nr * 81 + nr * 9);
    double* sub = (double*)calloc((size_t)G * per, sizeof(double));
    int bad = 0;
#ifdef _OPENMP
    omp_set_num_threads(P->n_threads);
#endif
    #pragma omp parallel for schedule(dynamic, 1) reduction(|:bad)
    for (int g = 0; g < G; ++g) {
        double* blk = sub + (size_t)g * per;
        double* U = blk + nb * 81;
        double* rhs = U + nr * 81;
        int32_t p0 = (int32_t)((int64_t)P->n_pts * g / G), p1 = (int32_t)((int64_t)P->n_pts * (g + 1) / G);
        for (int32_t p = p0; p < p1; ++p)
            if (!add_point(P, p, lambda, blk, U, rhs)) bad = 1;
    }
    if (bad) { free(sub); return 3; }
    /* aggregation of the sub-RCSs */
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < (int64_t)per; ++i) {
        double s = 0.0;
        for (int g = 0; g < G; ++g) s += sub[(size_t)g * per + i];
        sub[i] = s;
    }
    memcpy(P->blk, sub, sizeof(double) * nb * 81);
    const double* U = sub + nb * 81;
    memcpy(P->rhs, U + nr * 81, sizeof(double) * nr * 9);
    for (int32_t r = 0; r < nr; ++r) {
        double* S = P->blk + P->row_ptr[r] * 81;    /* diagonal is first in its row */
        const double* Ur = U + (int64_t)r * 81;
        for (int i = 0; i < 81; ++i) S[i] += Ur[i];
        for (int i = 0; i < 9; ++i) S[i * 10] += lambda * Ur[i * 10];
    }
    free(sub);
    P->have_rcs = 1;
    P->lambda = lambda;
    return 0;
}

void orc_get_rcs(const orc_problem* P, double* blk, double* rhs) {
    if (blk) memcpy(blk, P->blk, sizeof(double) * 81 * P->n_blk);
    if (rhs) memcpy(rhs, P->rhs, sizeof(double) * 9 * P->n_rows);
}

void orc_set_rcs(orc_problem* P, const double* blk, const double* rhs) {
    if (blk) memcpy(P->blk, blk, sizeof(double) * 81 * P->n_blk);
    if (rhs) memcpy(P->rhs, rhs, sizeof(double) * 9 * P->n_rows);
    P->have_rcs = 1;
}

void orc_get_point_terms(const orc_problem* P, double* Vinv, double* lp) {
    if (Vinv) memcpy(Vinv, P->Vinv, sizeof(double) * 9 * P->n_pts);
    if (lp) memcpy(lp, P->lp, sizeof(double) * 3 * P->n_pts);
}

/* ------------------------------------------------------------------------ */
/* PCG on the RCS (Sec. 3.2 and 6.2)                                         */
/* ------------------------------------------------------------------------ */

/* y = S x for the symmetric S stored as its upper blocks: each block (r, s)
 * contributes S_rs x_s to y_r and, off the diagonal, S_rs^T x_r to y_s.  The
 * blocks are split into n_thr groups, each producing a partial result vector;
 * the partial vectors are then summed (Sec. 6.2). */
static void spmv(const orc_problem* P, const double* x, double* y, double* part, int n_thr) {
    int64_t n = (int64_t)P->n_rows * 9;
    #pragma omp parallel for schedule(static, 1)
    for (int g = 0; g < n_thr; ++g) {
        double* yg = part + (int64_t)g * n;
        memset(yg, 0, sizeof(double) * n);
        int32_t r0 = (int32_t)((int64_t)P->n_rows * g / n_thr), r1 = (int32_t)((int64_t)P->n_rows * (g + 1) / n_thr);
        for (int32_t r = r0; r < r1; ++r)
            for (int64_t k = P->row_ptr[r]; k < P->row_ptr[r + 1]; ++k) {
                int32_t s = P->col_idx[k];
                const double* S = P->blk + k * 81;
                for (int i = 0; i < 9; ++i) {
                    double acc = 0.0;
                    for (int j = 0; j < 9; ++j) acc += S[i * 9 + j] * x[s * 9 + j];
                    yg[r * 9 + i] += acc;
                }
                if (s != r)
                    for (int j = 0; j < 9; ++j) {
                        double acc = 0.0;
                        for (int i = 0; i < 9; ++i) acc += S[i * 9 + j] * x[r * 9 + i];
                        yg[s * 9 + j] += acc;
                    }
            }
    }
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int g = 0; g < n_thr; ++g) s += part[(int64_t)g * n + i];
        y[i] = s;
    }
}

static double dot(const double* a, const double* b, int64_t n) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* Cholesky factor (lower, row-major) of a 9x9 SPD matrix; 0 if not SPD. */
static int chol9(const double* A, double* L) {
    memset(L, 0, sizeof(double) * 81);
    for (int j = 0; j < 9; ++j) {
        double s = A[j * 9 + j];
        for (int k = 0; k < j; ++k) s -= L[j * 9 + k] * L[j * 9 + k];
        if (!(s > 0.0)) return 0;
        L[j * 9 + j] = sqrt(s);
        for (int i = j + 1; i < 9; ++i) {
            double t = A[i * 9 + j];
            for (int k = 0; k < j; ++k) t -= L[i * 9 + k] * L[j * 9 + k];
            L[i * 9 + j] = t / L[j * 9 + j];
        }
    }
    return 1;
}

static void chol9_solve(const double* L, const double* b, double* x) {
    double y[9];
    for (int i = 0; i < 9; ++i) {
        double s = b[i];
        for (int k = 0; k < i; ++k) s -= L[i * 9 + k] * y[k];
        y[i] = s / L[i * 9 + i];
    }
    for (int i = 8; i >= 0; --i) {
        double s = y[i];
        for (int k = i + 1; k < 9; ++k) s -= L[k * 9 + i] * x[k];
        x[i] = s / L[i * 9 + i];
    }
}

/* Preconditioned CG on S y = b (Eq. (6)-(7)) with M = blockdiag(S_ii) (the
 * block-diagonal preconditioner; by default built from the RCS diagonal
 * blocks, or from Mblk [n_rows][81] if not NULL, each of which must be SPD).
 * Recurrence of Sec. 3.2: y0 = x0 (or 0), r0 = b - S y0, d0 = M^-1 r0;
 * alpha = r^T M^-1 r / d^T S d; y += alpha d; r -= alpha S d; stop when
 * |r_k| / |r_0| <= tol (the printed ratio |r_0|/|r_k| > T is read inverted);
 * beta = r_new^T M^-1 r_new / r^T M^-1 r; d = M^-1 r_new + beta d.
 * Returns 0 converged, 4 not converged after max_iter, 3 not SPD. */
int orc_pcg(orc_problem* P, double tol, int32_t max_iter, const double* x0,
            const double* Mblk, double* x, int32_t* iters, double* relres) {
    int64_t nr = P->n_rows, n = nr * 9;
    int nt = P->n_threads;
    double* L = (double*)malloc(sizeof(double) * 81 * (nr > 0 ? nr : 1));
    double *r = (double*)malloc(sizeof(double) * n), *z = (double*)malloc(sizeof(double) * n);
    double *d = (double*)malloc(sizeof(double) * n), *q = (double*)malloc(sizeof(double) * n);
    double* part = (double*)malloc(sizeof(double) * n * nt);
    int status = 0;
    *iters = 0; *relres = 0.0;
    for (int64_t i = 0; i < nr; ++i) {
        const double* M = Mblk ? Mblk + i * 81 : P->blk + P->row_ptr[i] * 81;
        if (!chol9(M, L + i * 81)) { status = 3; goto done; }
    }
    if (x0) {
        memcpy(x, x0, sizeof(double) * n);
        spmv(P, x, q, part, nt);
        for (int64_t i = 0; i < n; ++i) r[i] = P->rhs[i] - q[i];
    } else {
        memset(x, 0, sizeof(double) * n);
        memcpy(r, P->rhs, sizeof(double) * n);
    }
    double r0 = sqrt(dot(r, r, n));
    if (r0 == 0.0) goto done;
    for (int64_t i = 0; i < nr; ++i) chol9_solve(L + i * 81, r + i * 9, z + i * 9);
    memcpy(d, z, sizeof(double) * n);
    double rz = dot(r, z, n);
    int k = 0;
    for (;;) {
        spmv(P, d, q, part, nt);
        double dq = dot(d, q, n);
        if (!(dq > 0.0)) { status = 3; break; }
        double alpha = rz / dq;
        for (int64_t i = 0; i < n; ++i) { x[i] += alpha * d[i]; r[i] -= alpha * q[i]; }
        ++k;
        double rn = sqrt(dot(r, r, n));
        *relres = rn / r0;
        if (*relres <= tol) break;
        if (k >= max_iter) { status = 4; break; }
        for (int64_t i = 0; i < nr; ++i) chol9_solve(L + i * 81, r + i * 9, z + i * 9);
        double rz_new = dot(r, z, n);
        double beta = rz_new / rz;
        for (int64_t i = 0; i < n; ++i) d[i] = z[i] + beta * d[i];
        rz = rz_new;
    }
    *iters = k;
done:
    free(L); free(r); free(z); free(d); free(q); free(part);
    return status;
}

/* y = S x (exposed for tests) */
void orc_spmv(orc_problem* P, const double* x, double* y) {
    double* part = (double*)malloc(sizeof(double) * (int64_t)P->n_rows * 9 * P->n_threads);
    spmv(P, x, y, part, P->n_threads);
    free(part);
}

/* Eq. (5): dx_p = (V*)^-1 (l_p - sum_a W_a^T dx_c(row of a)), with W_a from
 * the stored Jacobians and fixed cameras contributing nothing. */
void orc_back_substitute(const orc_problem* P, const double* dxc, double* dxp) {
    #pragma omp parallel for schedule(static)
    for (int32_t p = 0; p < P->n_pts; ++p) {
        double g[3];
        for (int i = 0; i < 3; ++i) g[i] = P->lp[(int64_t)p * 3 + i];
        for (int64_t q = P->pt_ptr[p]; q < P->pt_ptr[p + 1]; ++q) {
            int64_t k = P->pt_obs[q];
            int32_t r = P->cam_row[P->obs_cam[k]];
            if (r < 0) continue;
            const double* Jc = P->Jc + k * 18;
            const double* Jp = P->Jp + k * 6;
            for (int j = 0; j < 3; ++j) {
                double s = 0.0;
                for (int i = 0; i < 9; ++i) {
                    double Wij = Jc[i] * Jp[j] + Jc[9 + i] * Jp[3 + j];
                    s += Wij * dxc[(int64_t)r * 9 + i];
                }
                g[j] -= s;
            }
        }
        const double* Vi = P->Vinv + (int64_t)p * 9;
        for (int i = 0; i < 3; ++i)
            dxp[(int64_t)p * 3 + i] = Vi[i * 3 + 0] * g[0] + Vi[i * 3 + 1] * g[1] + Vi[i * 3 + 2] * g[2];
    }
}

/* cost F = 1/2 sum |e|^2 at the given parameters */
double orc_cost(const orc_problem* P, const double* cams, const double* pts) {
    return orc_linearize(P->n_obs, cams, pts, P->obs_cam, P->obs_pt, P->uv, NULL, NULL, NULL);
}

/* From the stored linearization: |J dx|^2 and dx^T l with l = -J^T e, where
 * J dx per observation is Jc dx_c(row) + Jp dx_p(point). */
void orc_model_terms(const orc_problem* P, const double* dxc, const double* dxp,
                     double* jdx2, double* dxl) {
    double s2 = 0.0, sl = 0.0;
    #pragma omp parallel for schedule(static) reduction(+:s2, sl)
    for (int64_t k = 0; k < P->n_obs; ++k) {
        int32_t r = P->cam_row[P->obs_cam[k]];
        int32_t p = P->obs_pt[k];
        for (int row = 0; row < 2; ++row) {
            double g = 0.0;
            if (r >= 0)
                for (int i = 0; i < 9; ++i) g += P->Jc[k * 18 + row * 9 + i] * dxc[(int64_t)r * 9 + i];
            for (int i = 0; i < 3; ++i) g += P->Jp[k * 6 + row * 3 + i] * dxp[(int64_t)p * 3 + i];
            s2 += g * g;
            sl -= g * P->e[2 * k + row];
        }
    }
    *jdx2 = s2; *dxl = sl;
}

/* ------------------------------------------------------------------------ */
/* one LM iteration (Eq. (1) solved through Eq. (4), (6)-(7), (5))           */
/* ------------------------------------------------------------------------ */
typedef struct { double lambda, nu; int32_t iter, pad; } orc_lm_state;
typedef struct {
    double cost, cost_new, rho, model_decrease, pcg_relres;
    int32_t accepted, pcg_iters, pcg_status, stop;
} orc_lm_info;

/* Readings (the paper gives no schedule): gain ratio
 * rho = (F - F') / (dx^T l - 1/2 |J dx|^2); a step is accepted iff the
 * predicted decrease is positive and F' < F; Nielsen's update: accept ->
 * lambda *= max(1/3, 1 - (2 rho - 1)^3), nu = 2; reject -> lambda *= nu,
 * nu *= 2.  Every attempt counts as an iteration.  stop = 1 when an accepted
 * step lowers the cost by less than 1e-12 relative. */
int orc_lm_step(orc_problem* P, double* cams, double* pts, orc_lm_state* st,
                orc_lm_info* info, double pcg_tol, int32_t pcg_max_iter) {
    int64_t nr = P->n_rows;
    memset(info, 0, sizeof *info);
    double F = orc_prob_linearize(P, cams, pts);
    info->cost = F;
    int rc = orc_form_rcs(P, st->lambda, 0);
    double* dxc = (double*)calloc((size_t)nr * 9 + 1, sizeof(double));
    double* dxp = (double*)calloc((size_t)P->n_pts * 3, sizeof(double));
    double* c2 = (double*)malloc(sizeof(double) * 9 * P->n_cams);
    double* p2 = (double*)malloc(sizeof(double) * 3 * P->n_pts);
    int ok = 0;
    if (rc == 0) {
        int32_t it; double rr;
        int ps = orc_pcg(P, pcg_tol, pcg_max_iter, NULL, NULL, dxc, &it, &rr);
        info->pcg_iters = it; info->pcg_relres = rr; info->pcg_status = ps;
        if (ps == 0 || ps == 4) {
            orc_back_substitute(P, dxc, dxp);
            for (int32_t c = 0; c < P->n_cams; ++c)
                for (int i = 0; i < 9; ++i)
                    c2[c * 9 + i] = cams[c * 9 + i] + (P->cam_row[c] >= 0 ? dxc[(int64_t)P->cam_row[c] * 9 + i] : 0.0);
            for (int64_t i = 0; i < (int64_t)P->n_pts * 3; ++i) p2[i] = pts[i] + dxp[i];
            double Fn = orc_cost(P, c2, p2);
            double jdx2, dxl;
            orc_model_terms(P, dxc, dxp, &jdx2, &dxl);
            double L = dxl - 0.5 * jdx2;
            info->cost_new = Fn;
            info->model_decrease = L;
            info->rho = (F - Fn) / L;
            ok = (L > 0.0) && (Fn < F) && isfinite(Fn);
        }
    } else {
        info->pcg_status = rc;
    }
    if (ok) {
        memcpy(cams, c2, sizeof(double) * 9 * P->n_cams);
        memcpy(pts, p2, sizeof(double) * 3 * P->n_pts);
        double tt = 2.0 * info->rho - 1.0;
        double f = 1.0 - tt * tt * tt;
        st->lambda *= (f > 1.0 / 3.0 ? f : 1.0 / 3.0);
        st->nu = 2.0;
        info->accepted = 1;
        if ((F - info->cost_new) < 1e-12 * F) info->stop = 1;
    } else {
        st->lambda *= st->nu;
        st->nu *= 2.0;
    }
    st->iter += 1;
    free(dxc); free(dxp); free(c2); free(p2);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* re-triangulation of points with the cameras held fixed                     */
/* ------------------------------------------------------------------------ */
/* The paper's alternative to Eq. (5): after the camera step the points are
 * re-estimated from the updated camera poses (Sec. 3.1, after Eq. (5); Sec. 6 names it
 * among the costly steps).  For each point, with every camera fixed:
 *   - linear start (init = 1): each observed pixel is undistorted (the
 *     radius r of the normalised image point solves r (1 + k1 r^2 + k2 r^4)
 *     = |pixel| / f, by Newton's method from r = |pixel| / f), giving (x, y)
 *     with R X + t parallel to (x, y, 1); the two linear equations
 *       (x R_3 - R_1) X = t_1 - x t_3,   (y R_3 - R_2) X = t_2 - y t_3
 *     of every observation are solved in the least-squares sense (normal
 *     equations, 3x3);
 *   - otherwise the start is the given point;
 *   - then n_gn Gauss-Newton steps on the point's reprojection error,
 *     X += (Jp^T Jp)^-1 (-Jp^T e), with Jp and e from the dual-number
 *     projection.
 * A point whose 3x3 normal matrix is not positive definite keeps its start
 * (or its last iterate) and is counted.  which (or NULL: every point) lists
 * the points to triangulate; pts_out receives them (others untouched).
 * Returns the number of points that failed. */
static double undistort_radius(double rho, double k1, double k2) {
    double r = rho;
    for (int it = 0; it < 60; ++it) {
        double r2 = r * r;
        double g = r * (1.0 + k1 * r2 + k2 * r2 * r2) - rho;
        double dg = 1.0 + 3.0 * k1 * r2 + 5.0 * k2 * r2 * r2;
        double step = g / dg;
        r -= step;
        if (fabs(step) <= 1e-17 * (1.0 + r)) break;
    }
    return r;
}

static void rotation_matrix(const double* w, double R[9]) {
    /* columns R e_j from the same Rodrigues map as the projection */
    dual wd[3], e[3], out[3];
    for (int i = 0; i < 3; ++i) wd[i] = dconst(w[i]);
    for (int j = 0; j < 3; ++j) {
        for (int i = 0; i < 3; ++i) e[i] = dconst(i == j ? 1.0 : 0.0);
        rotate(wd, e, out);
        for (int i = 0; i < 3; ++i) R[i * 3 + j] = out[i].v;
    }
}

/* 3x3 SPD solve A x = b through the cofactor inverse; 0 if not PD */
static int solve3_spd(const double A[9], const double b[3], double x[3]) {
    double Ai[9];
    if (!inv3_spd(A, Ai)) return 0;
    for (int i = 0; i < 3; ++i) x[i] = Ai[i * 3 + 0] * b[0] + Ai[i * 3 + 1] * b[1] + Ai[i * 3 + 2] * b[2];
    return 1;
}

int64_t orc_triangulate(const orc_problem* P, const double* cams, const double* pts_start, double* pts_out,
                        const int32_t* which, int64_t n_which, int32_t init, int32_t n_gn) {
    const int64_t n = which ? n_which : P->n_pts;
    int64_t failed = 0;
    #pragma omp parallel for schedule(dynamic, 256) reduction(+:failed)
    for (int64_t ii = 0; ii < n; ++ii) {
        const int32_t p = which ? which[ii] : (int32_t)ii;
        double X[3] = {pts_start[(int64_t)p * 3], pts_start[(int64_t)p * 3 + 1], pts_start[(int64_t)p * 3 + 2]};
        int ok = 1;
        if (init) {
            double A[9] = {0}, b[3] = {0};
            for (int64_t q = P->pt_ptr[p]; q < P->pt_ptr[p + 1]; ++q) {
                const int64_t k = P->pt_obs[q];
                const double* c = cams + (int64_t)P->obs_cam[k] * NCP;
                const double u = P->uv[k], v = P->uv[P->n_obs + k];
                const double rho = sqrt(u * u + v * v) / c[6];
                double x = 0.0, y = 0.0;
                if (rho > 0.0) {
                    const double r = undistort_radius(rho, c[7], c[8]);
                    x = u / c[6] * (r / rho);
                    y = v / c[6] * (r / rho);
                }
                double R[9];
                rotation_matrix(c, R);
                const double a1[3] = {x * R[6] - R[0], x * R[7] - R[1], x * R[8] - R[2]};
                const double a2[3] = {y * R[6] - R[3], y * R[7] - R[4], y * R[8] - R[5]};
                const double b1 = c[3] - x * c[5], b2 = c[4] - y * c[5];
                for (int i = 0; i < 3; ++i) {
                    for (int j = 0; j < 3; ++j) A[i * 3 + j] += a1[i] * a1[j] + a2[i] * a2[j];
                    b[i] += a1[i] * b1 + a2[i] * b2;
                }
            }
            double X0[3];
            if (solve3_spd(A, b, X0)) { X[0] = X0[0]; X[1] = X0[1]; X[2] = X0[2]; }
            else ok = 0;
        }
        for (int it = 0; ok && it < n_gn; ++it) {
            double V[9] = {0}, g[3] = {0};
            for (int64_t q = P->pt_ptr[p]; q < P->pt_ptr[p + 1]; ++q) {
                const int64_t k = P->pt_obs[q];
                dual pr[2];
                project_dual(cams + (int64_t)P->obs_cam[k] * NCP, X, pr);
                const double e0 = pr[0].v - P->uv[k], e1 = pr[1].v - P->uv[P->n_obs + k];
                for (int i = 0; i < 3; ++i) {
                    for (int j = 0; j < 3; ++j) V[i * 3 + j] += pr[0].d[9 + i] * pr[0].d[9 + j] + pr[1].d[9 + i] * pr[1].d[9 + j];
                    g[i] -= pr[0].d[9 + i] * e0 + pr[1].d[9 + i] * e1;
                }
            }
            double dX[3];
            if (!solve3_spd(V, g, dX)) { ok = 0; break; }
            for (int i = 0; i < 3; ++i) X[i] += dX[i];
        }
        if (!ok) failed += 1;
        for (int i = 0; i < 3; ++i) pts_out[(int64_t)p * 3 + i] = X[i];
    }
    return failed;
}

/* BSMC memory in bytes from the stored pattern (Eq. (9) counted on the
 * actual blocks: c*c doubles and 3 ints per stored block, plus one int per
 * row). */
int64_t orc_bsmc_bytes(const orc_problem* P, int32_t c) {
    return P->n_blk * (int64_t)c * c * 8 + P->n_blk * 3 * 4 + (int64_t)P->n_rows * 4;
}
