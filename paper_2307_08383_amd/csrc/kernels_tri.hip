// Re-triangulation of points with the cameras held fixed: the alternative to
// the back-substitution of Eq. (5) that Sec. 3.1 names (points re-estimated
// from the camera poses), and the third costly step Sec. 6 lists.
//
// Per point, over its track:
//   - optional linear start: each observed pixel is undistorted (the radius
//     r of the normalised image point solves r (1 + k1 r^2 + k2 r^4) =
//     |pixel| / f, Newton from r = |pixel| / f) to (x, y) with R X + t
//     parallel to (x, y, 1); the equations (x R_3 - R_1) X = t_1 - x t_3,
//     (y R_3 - R_2) X = t_2 - y t_3 of all observations are solved in the
//     least-squares sense through their 3x3 normal matrix;
//   - n_gn Gauss-Newton steps on the point's reprojection error:
//     X += (sum J_p^T J_p)^-1 (-sum J_p^T e).
// One wave per chunk of whole tracks, one lane per observation (the layout
// of the point stage): lanes form their terms, the track's first lane sums
// them from LDS, solves the 3x3 system and hands X back through LDS.
#include "ba_common.hpp"

namespace ba {

namespace {

constexpr int BS = 256;
constexpr int WPB = BS / kWave;

// s = (A00 A01 A02 A11 A12 A22, b0 b1 b2): x = A^-1 b by Cholesky; false
// unless A is positive definite
__device__ __forceinline__ bool solve3(const double* s, double* x) {
    const double L00 = sqrt(s[0]);
    const double L10 = s[1] / L00, L20 = s[2] / L00;
    const double d1 = s[3] - L10 * L10;
    const double L11 = sqrt(d1);
    const double L21 = (s[4] - L20 * L10) / L11;
    const double d2 = s[5] - L20 * L20 - L21 * L21;
    const double L22 = sqrt(d2);
    const double y0 = s[6] / L00;
    const double y1 = (s[7] - L10 * y0) / L11;
    const double y2 = (s[8] - L20 * y0 - L21 * y1) / L22;
    x[2] = y2 / L22;
    x[1] = (y1 - L21 * x[2]) / L11;
    x[0] = (y0 - L10 * x[1] - L20 * x[2]) / L00;
    return s[0] > 0.0 && d1 > 0.0 && d2 > 0.0 && isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2]);
}

// radius of the normalised image point whose distorted radius is rho
__device__ __forceinline__ double undistort_radius(double rho, double k1, double k2) {
    double r = rho;
    for (int it = 0; it < 60; ++it) {
        const double r2 = r * r;
        const double g = r * (1.0 + k1 * r2 + k2 * r2 * r2) - rho;
        const double dg = 1.0 + 3.0 * k1 * r2 + 5.0 * k2 * r2 * r2;
        const double step = g / dg;
        r -= step;
        if (fabs(step) <= 1e-17 * (1.0 + r)) break;
    }
    return r;
}

// The terms of observation (camera c, pixel ou, ov) in the normal equations
// of the linear multi-view solve: A^T A (6 unique) and A^T b of its two rows
// (x R_3 - R_1) X = t_1 - x t_3, (y R_3 - R_2) X = t_2 - y t_3.
__device__ __forceinline__ void tri_linear_terms(const double* c, double ou, double ov, double* m) {
    const double rho = sqrt(ou * ou + ov * ov) / c[6];
    double x = 0.0, y = 0.0;
    if (rho > 0.0) {
        const double r = undistort_radius(rho, c[7], c[8]);
        x = ou / c[6] * (r / rho);
        y = ov / c[6] * (r / rho);
    }
    const double w0 = c[0], w1 = c[1], w2 = c[2];
    const double s = w0 * w0 + w1 * w1 + w2 * w2;
    double a, b, as, bs;
    rot_coeffs(s, a, b, as, bs);
    const double R[9] = {1.0 + b * (w0 * w0 - s), -a * w2 + b * w0 * w1, a * w1 + b * w0 * w2,
                         a * w2 + b * w1 * w0, 1.0 + b * (w1 * w1 - s), -a * w0 + b * w1 * w2,
                         -a * w1 + b * w2 * w0, a * w0 + b * w2 * w1, 1.0 + b * (w2 * w2 - s)};
    const double a1[3] = {x * R[6] - R[0], x * R[7] - R[1], x * R[8] - R[2]};
    const double a2[3] = {y * R[6] - R[3], y * R[7] - R[4], y * R[8] - R[5]};
    const double b1 = c[3] - x * c[5], b2 = c[4] - y * c[5];
    m[0] = a1[0] * a1[0] + a2[0] * a2[0];
    m[1] = a1[0] * a1[1] + a2[0] * a2[1];
    m[2] = a1[0] * a1[2] + a2[0] * a2[2];
    m[3] = a1[1] * a1[1] + a2[1] * a2[1];
    m[4] = a1[1] * a1[2] + a2[1] * a2[2];
    m[5] = a1[2] * a1[2] + a2[2] * a2[2];
    m[6] = a1[0] * b1 + a2[0] * b2;
    m[7] = a1[1] * b1 + a2[1] * b2;
    m[8] = a1[2] * b1 + a2[2] * b2;
}

// The terms of the Gauss-Newton step on the point's reprojection error at X:
// J_p^T J_p (6 unique) and -J_p^T e.
__device__ __forceinline__ void tri_gn_terms(const double* c, const double* X, double ou, double ov, double* m) {
    double pu, pv, jp[6];
    project_point<true, false>(c, X[0], X[1], X[2], pu, pv, nullptr, jp);
    const double eu = pu - ou, ev = pv - ov;
    m[0] = jp[0] * jp[0] + jp[3] * jp[3];
    m[1] = jp[0] * jp[1] + jp[3] * jp[4];
    m[2] = jp[0] * jp[2] + jp[3] * jp[5];
    m[3] = jp[1] * jp[1] + jp[4] * jp[4];
    m[4] = jp[1] * jp[2] + jp[4] * jp[5];
    m[5] = jp[2] * jp[2] + jp[5] * jp[5];
    m[6] = -(jp[0] * eu + jp[3] * ev);
    m[7] = -(jp[1] * eu + jp[4] * ev);
    m[8] = -(jp[2] * eu + jp[5] * ev);
}

template <bool LINEAR>
__global__ __launch_bounds__(BS) void k_triangulate(int n_chunk, const int32_t* __restrict__ chunk_ptr, int n,
                                                    const int32_t* __restrict__ obs_cam,
                                                    const int32_t* __restrict__ obs_pt,
                                                    const int32_t* __restrict__ obs_row,
                                                    const double* __restrict__ uv, const double* __restrict__ cams,
                                                    const double* __restrict__ dxc, const double* __restrict__ pts,
                                                    double* __restrict__ out, int delta, int n_gn,
                                                    int* __restrict__ n_failed) {
    __shared__ double sA[WPB][kWave][9];   // per-lane terms
    __shared__ double sX[WPB][kWave][3];   // the track's current point, at its first lane
    const int wv = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int chunk = blockIdx.x * WPB + wv;
    int k0 = 0, k1 = 0;
    if (chunk < n_chunk) { k0 = chunk_ptr[chunk]; k1 = chunk_ptr[chunk + 1]; }
    const int k = k0 + lane;
    const bool act = k < k1;
    const int p = act ? obs_pt[k] : -1;
    const Track tk = chunk_track(act, p, lane, k1 - k0);
    const int head = tk.head, tl = tk.len;
    double c[9];
    double ou = 0.0, ov = 0.0;
    bool ok = true;                        // meaningful at the head lane
    if (act) {
        const double* c0 = cams + (int64_t)obs_cam[k] * 9;
        const int row = obs_row[k];
#pragma unroll
        for (int i = 0; i < 9; ++i) c[i] = c0[i] + ((dxc && row >= 0) ? dxc[(int64_t)row * 9 + i] : 0.0);
        ou = uv[k];
        ov = uv[n + k];
        if (head == lane) {
            // start: the point as given (read in place: only this lane reads
            // or writes point p)
#pragma unroll
            for (int i = 0; i < 3; ++i) sX[wv][lane][i] = pts[(int64_t)p * 3 + i] + (delta ? out[(int64_t)p * 3 + i] : 0.0);
        }
    }
    if (LINEAR) {
        if (act) {
            tri_linear_terms(c, ou, ov, sA[wv][lane]);
        }
        __syncthreads();
        if (act && head == lane) {
            double sum[9];
#pragma unroll
            for (int m = 0; m < 9; ++m) sum[m] = 0.0;
            for (int q = 0; q < tl; ++q)
#pragma unroll
                for (int m = 0; m < 9; ++m) sum[m] += sA[wv][lane + q][m];
            double X[3];
            ok = solve3(sum, X);
            if (ok)
#pragma unroll
                for (int i = 0; i < 3; ++i) sX[wv][lane][i] = X[i];
        }
    }
    __syncthreads();
    for (int it = 0; it < n_gn; ++it) {
        if (act) {
            const double X[3] = {sX[wv][head][0], sX[wv][head][1], sX[wv][head][2]};
            tri_gn_terms(c, X, ou, ov, sA[wv][lane]);
        }
        __syncthreads();
        if (act && head == lane && ok) {
            double sum[9];
#pragma unroll
            for (int m = 0; m < 9; ++m) sum[m] = 0.0;
            for (int q = 0; q < tl; ++q)
#pragma unroll
                for (int m = 0; m < 9; ++m) sum[m] += sA[wv][lane + q][m];
            double dX[3];
            ok = solve3(sum, dX);
            if (ok)
#pragma unroll
                for (int i = 0; i < 3; ++i) sX[wv][lane][i] += dX[i];
        }
        __syncthreads();
    }
    if (act && head == lane) {
        if (!ok) atomicAdd(n_failed, 1);
#pragma unroll
        for (int i = 0; i < 3; ++i)
            out[(int64_t)p * 3 + i] = sX[wv][lane][i] - (delta ? pts[(int64_t)p * 3 + i] : 0.0);
    }
}

// The same for a track longer than a wave: one workgroup per point, its
// threads striding over the track, sums reduced in a fixed order (strided
// thread sums, the wave's shuffle tree, then the waves in order).
template <bool LINEAR>
__global__ __launch_bounds__(BS) void k_triangulate_long(const int32_t* __restrict__ long_ptr, int n,
                                                         const int32_t* __restrict__ obs_cam,
                                                         const int32_t* __restrict__ obs_pt,
                                                         const int32_t* __restrict__ obs_row,
                                                         const double* __restrict__ uv, const double* __restrict__ cams,
                                                         const double* __restrict__ dxc, const double* __restrict__ pts,
                                                         double* __restrict__ out, int delta, int n_gn,
                                                         int* __restrict__ n_failed) {
    __shared__ double sh[9][WPB];
    __shared__ double sX[3];
    __shared__ int sok;
    const int k0 = long_ptr[blockIdx.x], k1 = long_ptr[blockIdx.x + 1];
    const int p = obs_pt[k0];
    const int wv = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    if (threadIdx.x == 0) {
        for (int i = 0; i < 3; ++i) sX[i] = pts[(int64_t)p * 3 + i] + (delta ? out[(int64_t)p * 3 + i] : 0.0);
        sok = 1;
    }
    __syncthreads();
    auto camera = [&](int k, double* c) {
        const double* c0 = cams + (int64_t)obs_cam[k] * 9;
        const int row = obs_row[k];
#pragma unroll
        for (int i = 0; i < 9; ++i) c[i] = c0[i] + ((dxc && row >= 0) ? dxc[(int64_t)row * 9 + i] : 0.0);
    };
    // sums of the track's terms into sh[m][0] (all threads then read them)
    auto reduce9 = [&](double* v) {
#pragma unroll
        for (int m = 0; m < 9; ++m) {
            const double w = wave_sum(v[m]);
            if (lane == 0) sh[m][wv] = w;
        }
        __syncthreads();
        if (threadIdx.x == 0)
#pragma unroll
            for (int m = 0; m < 9; ++m) {
                double t = 0.0;
#pragma unroll
                for (int w = 0; w < WPB; ++w) t += sh[m][w];
                v[m] = t;
            }
    };
    for (int it = LINEAR ? -1 : 0; it < n_gn; ++it) {
        double v[9];
#pragma unroll
        for (int m = 0; m < 9; ++m) v[m] = 0.0;
        const double X[3] = {sX[0], sX[1], sX[2]};
        for (int k = k0 + threadIdx.x; k < k1; k += BS) {
            double c[9], t[9];
            camera(k, c);
            if (it < 0) tri_linear_terms(c, uv[k], uv[n + k], t);
            else tri_gn_terms(c, X, uv[k], uv[n + k], t);
#pragma unroll
            for (int m = 0; m < 9; ++m) v[m] += t[m];
        }
        reduce9(v);
        if (threadIdx.x == 0 && sok) {
            double d[3];
            sok = solve3(v, d);
            if (sok)
                for (int i = 0; i < 3; ++i) sX[i] = it < 0 ? d[i] : sX[i] + d[i];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (!sok) atomicAdd(n_failed, 1);
        for (int i = 0; i < 3; ++i) out[(int64_t)p * 3 + i] = sX[i] - (delta ? pts[(int64_t)p * 3 + i] : 0.0);
    }
}

}  // namespace

void launch_triangulate(ba_ctx* c, const double* cams, const double* dxc, const double* pts, double* out, int delta,
                        int linear, int n_gn, int* n_failed) {
    const int nb = (c->n_chunk + WPB - 1) / WPB;
    const int n = (int)c->n_obs;
    if (nb > 0) {
        if (linear)
            k_triangulate<true><<<nb, BS, 0, c->stream>>>(c->n_chunk, c->chunk_ptr, n, c->obs_cam, c->obs_pt,
                                                          c->obs_row, c->obs_uv, cams, dxc, pts, out, delta, n_gn,
                                                          n_failed);
        else
            k_triangulate<false><<<nb, BS, 0, c->stream>>>(c->n_chunk, c->chunk_ptr, n, c->obs_cam, c->obs_pt,
                                                           c->obs_row, c->obs_uv, cams, dxc, pts, out, delta, n_gn,
                                                           n_failed);
    }
    if (c->n_long > 0) {
        if (linear)
            k_triangulate_long<true><<<c->n_long, BS, 0, c->stream>>>(c->long_ptr, n, c->obs_cam, c->obs_pt,
                                                                      c->obs_row, c->obs_uv, cams, dxc, pts, out,
                                                                      delta, n_gn, n_failed);
        else
            k_triangulate_long<false><<<c->n_long, BS, 0, c->stream>>>(c->long_ptr, n, c->obs_cam, c->obs_pt,
                                                                       c->obs_row, c->obs_uv, cams, dxc, pts, out,
                                                                       delta, n_gn, n_failed);
    }
}

}  // namespace ba
