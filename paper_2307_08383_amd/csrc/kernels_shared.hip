// Shared intrinsics: images share the interior parameters of their physical
// camera (the paper's 6 exterior + 5 interior unknowns, Sec. 4.1; fewer
// cameras than images, Table 2).  FP64.
//
// Camera-side unknowns become RCS rows of two kinds: the exterior block
// [w, t] of every free image and the interior block [f, cx, cy, k1, k2] of
// every physical camera, each padded to 9 slots (the padding has an identity
// diagonal and a zero right-hand side, so its solution is exactly zero and
// the 9x9 block machinery of the product and PCG is unchanged).  Every
// observation gives two records of the usual layout (2x9 Jacobian rows, then
// K = J_p L^-T): its exterior part at the image's row and its interior part
// at the camera's row.  With D_ab = 1 for two records of one observation and
// 0 otherwise, every RCS block is
//   S_uv = sum over record couples (a at row u, b at row v, same point)
//          J_a^T (D_ab I - K_a K_b^T) J_b   (+ lambda diag(U_uu) on u = v),
// which is Eq. (3)-(4) with U's image-camera coupling (D_ab = 1 across the
// two records of one observation) and the same-camera terms on the interior
// diagonal block.  The pair stage forms all of them (same-row couples
// included); this file holds the per-observation kernels and the diagonal
// stage that adds damping and padding and factors the diagonal blocks.
#include <algorithm>

#include "ba_common.hpp"

namespace ba {

namespace {

constexpr int BS = 256;
constexpr int WPB = BS / kWave;
constexpr int kPT = 12;

// the 9-parameter camera of the projection code: exterior of the image,
// focal length and distortion of its physical camera (the principal point
// is added to the pixel)
__device__ __forceinline__ void compose(const double* __restrict__ ext, const double* __restrict__ intr, double* c9) {
#pragma unroll
    for (int i = 0; i < 6; ++i) c9[i] = ext[i];
    c9[6] = intr[0];
    c9[7] = intr[3];
    c9[8] = intr[4];
}

__device__ __forceinline__ bool point_terms_s(const double* s, double lambda, double* r) {
    const double V00 = s[0] * (1.0 + lambda), V11 = s[3] * (1.0 + lambda), V22 = s[5] * (1.0 + lambda);
    const double L00 = sqrt(V00), i00 = 1.0 / L00;
    const double L10 = s[1] * i00, L20 = s[2] * i00;
    const double d1 = V11 - L10 * L10;
    const double L11 = sqrt(d1), i11 = 1.0 / L11;
    const double L21 = (s[4] - L20 * L10) * i11;
    const double d2 = V22 - L20 * L20 - L21 * L21;
    const double L22 = sqrt(d2), i22 = 1.0 / L22;
    const double y0 = s[6] * i00;
    const double y1 = (s[7] - L10 * y0) * i11;
    const double y2 = (s[8] - L20 * y0 - L21 * y1) * i22;
    r[0] = L00; r[1] = L10; r[2] = L11; r[3] = L20; r[4] = L21; r[5] = L22;
    r[6] = y0; r[7] = y1; r[8] = y2; r[9] = i00; r[10] = i11; r[11] = i22;
    return V00 > 0.0 && d1 > 0.0 && d2 > 0.0;
}

// one wave per chunk of whole tracks, one lane per observation (the layout
// of the 9-parameter point stage); both records of an observation are
// written by its lane
__global__ __launch_bounds__(BS) void k_linpoint_s(int n_chunk, const int32_t* __restrict__ chunk_ptr, int n,
                                                   const int32_t* __restrict__ obs_img,
                                                   const int32_t* __restrict__ obs_pt,
                                                   const int32_t* __restrict__ chunk_q,
                                                   const int32_t* __restrict__ img_cam, int n_img,
                                                   const double* __restrict__ uv, const double* __restrict__ params,
                                                   const double* __restrict__ pts, double lambda,
                                                   double* __restrict__ R, double* __restrict__ Jp_out,
                                                   double* __restrict__ e, double* __restrict__ ptL,
                                                   double* __restrict__ ebar, double* __restrict__ part,
                                                   int* __restrict__ flags) {
    __shared__ double sP[WPB][kWave][kPT];
    __shared__ double sh[WPB];
    const int wv = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int chunk = blockIdx.x * WPB + wv;
    int k0 = 0, k1 = 0;
    if (chunk < n_chunk) { k0 = chunk_ptr[chunk]; k1 = chunk_ptr[chunk + 1]; }
    const int k = k0 + lane;
    const bool act = k < k1;
    double jc[18], jp[6];
    double cost = 0.0, eu = 0.0, ev = 0.0;
    const int p = act ? obs_pt[k] : -1;
    const Track tk = chunk_track(act, p, lane, k1 - k0);
    const int head = tk.head, tl = tk.len;
    const int64_t q = chunk < n_chunk ? (int64_t)chunk_q[chunk] + tk.idx : 0;
    if (act) {
        const int img = obs_img[k];
        const double* intr = params + 6 * (int64_t)n_img + 5 * (int64_t)img_cam[img];
        double c9[9];
        compose(params + 6 * (int64_t)img, intr, c9);
        const double* X = pts + (int64_t)p * 3;
        double pu, pv;
        project_point<true>(c9, X[0], X[1], X[2], pu, pv, jc, jp);
        eu = pu + intr[1] - uv[k];
        ev = pv + intr[2] - uv[n + k];
        if (!records_in_range<double>(jc, jp, eu, ev)) flags[2] = 1;
        reinterpret_cast<double2*>(Jp_out)[3 * (int64_t)k] = make_double2(jp[0], jp[1]);
        reinterpret_cast<double2*>(Jp_out)[3 * (int64_t)k + 1] = make_double2(jp[2], jp[3]);
        reinterpret_cast<double2*>(Jp_out)[3 * (int64_t)k + 2] = make_double2(jp[4], jp[5]);
        reinterpret_cast<double2*>(e)[k] = make_double2(eu, ev);
        cost = 0.5 * (eu * eu + ev * ev);
        sP[wv][lane][0] = jp[0] * jp[0] + jp[3] * jp[3];
        sP[wv][lane][1] = jp[0] * jp[1] + jp[3] * jp[4];
        sP[wv][lane][2] = jp[0] * jp[2] + jp[3] * jp[5];
        sP[wv][lane][3] = jp[1] * jp[1] + jp[4] * jp[4];
        sP[wv][lane][4] = jp[1] * jp[2] + jp[4] * jp[5];
        sP[wv][lane][5] = jp[2] * jp[2] + jp[5] * jp[5];
        sP[wv][lane][6] = -(jp[0] * eu + jp[3] * ev);
        sP[wv][lane][7] = -(jp[1] * eu + jp[4] * ev);
        sP[wv][lane][8] = -(jp[2] * eu + jp[5] * ev);
    }
    const double csum = block_sum<BS>(cost, sh);   // contains the barrier for sP
    if (threadIdx.x == 0) part[blockIdx.x] = csum;
    if (act && head == lane) {
        double s[9];
#pragma unroll
        for (int m = 0; m < 9; ++m) s[m] = 0.0;
        for (int t = 0; t < tl; ++t)
#pragma unroll
            for (int m = 0; m < 9; ++m) s[m] += sP[wv][lane + t][m];
        double r[kPT];
        if (!point_terms_s(s, lambda, r)) flags[0] = 1;
#pragma unroll
        for (int m = 0; m < kPT; ++m) sP[wv][lane][m] = r[m];
#pragma unroll
        for (int m = 0; m < 9; ++m) ptL[q * 9 + m] = r[m];
    }
    __syncthreads();
    if (act) {
        const double* r = sP[wv][head];
        double K[6];
#pragma unroll
        for (int rr = 0; rr < 2; ++rr) {
            const double y0 = jp[3 * rr] * r[9];
            const double y1 = (jp[3 * rr + 1] - r[1] * y0) * r[10];
            const double y2 = (jp[3 * rr + 2] - r[3] * y0 - r[4] * y1) * r[11];
            K[3 * rr] = y0; K[3 * rr + 1] = y1; K[3 * rr + 2] = y2;
        }
        // exterior record: J_c columns 0..5 of both rows; interior record:
        // d/df (column 6), d/dcx = (1, 0), d/dcy = (0, 1), d/dk1, d/dk2
        double re[24], ri[24];
#pragma unroll
        for (int m = 0; m < 24; ++m) { re[m] = 0.0; ri[m] = 0.0; }
#pragma unroll
        for (int j = 0; j < 6; ++j) { re[j] = jc[j]; re[9 + j] = jc[9 + j]; }
        ri[0] = jc[6]; ri[1] = 1.0; ri[2] = 0.0; ri[3] = jc[7]; ri[4] = jc[8];
        ri[9] = jc[15]; ri[10] = 0.0; ri[11] = 1.0; ri[12] = jc[16]; ri[13] = jc[17];
#pragma unroll
        for (int m = 0; m < 6; ++m) { re[18 + m] = K[m]; ri[18 + m] = K[m]; }
        double2* de = reinterpret_cast<double2*>(R + (int64_t)(2 * k) * kRec);
        double2* di = reinterpret_cast<double2*>(R + (int64_t)(2 * k + 1) * kRec);
#pragma unroll
        for (int m = 0; m < 12; ++m) {
            de[m] = make_double2(re[2 * m], re[2 * m + 1]);
            di[m] = make_double2(ri[2 * m], ri[2 * m + 1]);
        }
        const double v0 = eu + K[0] * r[6] + K[1] * r[7] + K[2] * r[8];
        const double v1 = ev + K[3] * r[6] + K[4] * r[7] + K[5] * r[8];
        reinterpret_cast<double2*>(ebar)[k] = make_double2(v0, v1);
    }
}

// Tracks longer than a wave: one workgroup per point (q0 + blockIdx.x), its
// threads striding over the track, the point's sums reduced in a fixed order
// (each thread's strided sum, the wave's shuffle tree, the waves in order).
// The first pass writes J_p, e and the Jacobian parts of both records; the
// second, with the point terms, K and e + K lhat.  A thread reads back in the
// second pass only what it wrote in the first.  part[blockIdx.x] = the
// track's cost.
__global__ __launch_bounds__(BS) void k_linpoint_s_long(int q0, const int32_t* __restrict__ long_ptr, int n,
                                                        const int32_t* __restrict__ obs_img,
                                                        const int32_t* __restrict__ obs_pt,
                                                        const int32_t* __restrict__ img_cam, int n_img,
                                                        const double* __restrict__ uv,
                                                        const double* __restrict__ params,
                                                        const double* __restrict__ pts, double lambda,
                                                        double* __restrict__ R, double* __restrict__ Jp_out,
                                                        double* __restrict__ e, double* __restrict__ ptL,
                                                        double* __restrict__ ebar, double* __restrict__ part,
                                                        int* __restrict__ flags) {
    __shared__ double sh[10][WPB];
    __shared__ double sr[kPT];
    const int k0 = long_ptr[blockIdx.x], k1 = long_ptr[blockIdx.x + 1];
    const int64_t q = (int64_t)q0 + blockIdx.x;
    const int p = obs_pt[k0];
    const double X0 = pts[(int64_t)p * 3], X1 = pts[(int64_t)p * 3 + 1], X2 = pts[(int64_t)p * 3 + 2];
    double v[10];
#pragma unroll
    for (int m = 0; m < 10; ++m) v[m] = 0.0;
    for (int k = k0 + threadIdx.x; k < k1; k += BS) {
        const int img = obs_img[k];
        const double* intr = params + 6 * (int64_t)n_img + 5 * (int64_t)img_cam[img];
        double c9[9], jc[18], jp[6], pu, pv;
        compose(params + 6 * (int64_t)img, intr, c9);
        project_point<true>(c9, X0, X1, X2, pu, pv, jc, jp);
        const double eu = pu + intr[1] - uv[k], ev = pv + intr[2] - uv[n + k];
        if (!records_in_range<double>(jc, jp, eu, ev)) flags[2] = 1;
#pragma unroll
        for (int m = 0; m < 6; ++m) Jp_out[(int64_t)k * 6 + m] = jp[m];
        reinterpret_cast<double2*>(e)[k] = make_double2(eu, ev);
        // Jacobian parts of the exterior and interior records (layout of
        // k_linpoint_s)
        double re[18], ri[18];
#pragma unroll
        for (int m = 0; m < 18; ++m) { re[m] = 0.0; ri[m] = 0.0; }
#pragma unroll
        for (int j = 0; j < 6; ++j) { re[j] = jc[j]; re[9 + j] = jc[9 + j]; }
        ri[0] = jc[6]; ri[1] = 1.0; ri[3] = jc[7]; ri[4] = jc[8];
        ri[9] = jc[15]; ri[11] = 1.0; ri[12] = jc[16]; ri[13] = jc[17];
        store_jc(R + (int64_t)(2 * k) * kRec, re);
        store_jc(R + (int64_t)(2 * k + 1) * kRec, ri);
        v[0] += jp[0] * jp[0] + jp[3] * jp[3];
        v[1] += jp[0] * jp[1] + jp[3] * jp[4];
        v[2] += jp[0] * jp[2] + jp[3] * jp[5];
        v[3] += jp[1] * jp[1] + jp[4] * jp[4];
        v[4] += jp[1] * jp[2] + jp[4] * jp[5];
        v[5] += jp[2] * jp[2] + jp[5] * jp[5];
        v[6] -= jp[0] * eu + jp[3] * ev;
        v[7] -= jp[1] * eu + jp[4] * ev;
        v[8] -= jp[2] * eu + jp[5] * ev;
        v[9] += 0.5 * (eu * eu + ev * ev);
    }
    block_reduce<10>(v, sh);
    if (threadIdx.x == 0) {
        double r[kPT];
        if (!point_terms_s(v, lambda, r)) flags[0] = 1;
#pragma unroll
        for (int m = 0; m < kPT; ++m) sr[m] = r[m];
#pragma unroll
        for (int m = 0; m < 9; ++m) ptL[q * 9 + m] = r[m];
        part[blockIdx.x] = v[9];
    }
    __syncthreads();
    for (int k = k0 + threadIdx.x; k < k1; k += BS) {
        double jp[6], K[6];
#pragma unroll
        for (int m = 0; m < 6; ++m) jp[m] = Jp_out[(int64_t)k * 6 + m];
#pragma unroll
        for (int rr = 0; rr < 2; ++rr) {
            const double y0 = jp[3 * rr] * sr[9];
            const double y1 = (jp[3 * rr + 1] - sr[1] * y0) * sr[10];
            const double y2 = (jp[3 * rr + 2] - sr[3] * y0 - sr[4] * y1) * sr[11];
            K[3 * rr] = y0; K[3 * rr + 1] = y1; K[3 * rr + 2] = y2;
        }
        store6(R + (int64_t)(2 * k) * kRec + 18, K);
        store6(R + (int64_t)(2 * k + 1) * kRec + 18, K);
        const double2 ek = reinterpret_cast<const double2*>(e)[k];
        const double v0 = ek.x + K[0] * sr[6] + K[1] * sr[7] + K[2] * sr[8];
        const double v1 = ek.y + K[3] * sr[6] + K[4] * sr[7] + K[5] * sr[8];
        reinterpret_cast<double2*>(ebar)[k] = make_double2(v0, v1);
    }
}

// Diagonal stage: one wave per RCS row over its records (the row's list):
// diag(U) and b_u = -sum J^T (e + K lhat); then the diagonal block that the
// pair stage formed gets lambda diag(U) and the identity on its padding,
// and is factored (Cholesky, L^-1, block-Jacobi inverse).
__global__ __launch_bounds__(BS) void k_node_diag(int n_rows, int n_free, const int32_t* __restrict__ rowobs_ptr,
                                                  const int32_t* __restrict__ rowobs,
                                                  const int32_t* __restrict__ row_ptr, const double* __restrict__ R,
                                                  const double* __restrict__ ebar, double lambda,
                                                  double* __restrict__ blk, double* __restrict__ rhs,
                                                  double* __restrict__ Minv, double* __restrict__ Linv,
                                                  int* __restrict__ flags) {
    __shared__ double sred[WPB][18];
    __shared__ double sS[WPB][81];
    __shared__ double sL[WPB][81];
    const int wv = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int row = blockIdx.x * WPB + wv;
    const bool live = row < n_rows;
    double du[9], bb[9];
#pragma unroll
    for (int m = 0; m < 9; ++m) { du[m] = 0.0; bb[m] = 0.0; }
    const int i0 = live ? rowobs_ptr[row] : 0, i1 = live ? rowobs_ptr[row + 1] : 0;
    for (int idx = i0 + lane; idx < i1; idx += kWave) {
        const int a = rowobs[idx];
        double jc[18];
        load_jc(R + (int64_t)a * kRec, jc);
        const double2 v = reinterpret_cast<const double2*>(ebar)[a >> 1];
#pragma unroll
        for (int c = 0; c < 9; ++c) {
            du[c] += jc[c] * jc[c] + jc[9 + c] * jc[9 + c];
            bb[c] -= jc[c] * v.x + jc[9 + c] * v.y;
        }
    }
#pragma unroll
    for (int m = 0; m < 9; ++m) {
        const double t = wave_sum(du[m]), w = wave_sum(bb[m]);
        if (lane == 0) { sred[wv][m] = t; sred[wv][9 + m] = w; }
    }
    __syncthreads();
    double* S = sS[wv];
    double* L = sL[wv];
    const int nreal = row < n_free ? 6 : 5;
    if (live) {
        // the pair stage summed the (a, b) and (b, a) terms of this block in
        // separate lanes: the mean with the transpose makes it exactly symmetric
        const double* B = blk + (int64_t)row_ptr[row] * 81;
        for (int e = lane; e < 81; e += kWave) {
            const int i = e / 9, j = e % 9;
            double v = 0.5 * (B[e] + B[j * 9 + i]);
            if (i == j) v = i < nreal ? B[e] + lambda * sred[wv][i] : 1.0;
            S[e] = v;
        }
        if (lane < 9) rhs[(int64_t)row * 9 + lane] = sred[wv][9 + lane];
    }
    __syncthreads();
    if (live)
        for (int e = lane; e < 81; e += kWave) blk[(int64_t)row_ptr[row] * 81 + e] = S[e];
    if (live && lane == 0) {
        bool ok = true;
        for (int j = 0; j < 9; ++j) {
            double sj = S[j * 9 + j];
            for (int q = 0; q < j; ++q) sj -= L[j * 9 + q] * L[j * 9 + q];
            if (!(sj > 0.0)) { ok = false; sj = 1.0; }
            const double ljj = sqrt(sj);
            L[j * 9 + j] = ljj;
            for (int i = j + 1; i < 9; ++i) {
                double t = S[i * 9 + j];
                for (int q = 0; q < j; ++q) t -= L[i * 9 + q] * L[j * 9 + q];
                L[i * 9 + j] = t / ljj;
            }
            for (int i = 0; i < j; ++i) L[i * 9 + j] = 0.0;
        }
        if (!ok) flags[1] = 1;
        for (int j = 0; j < 9; ++j) {
            L[j * 9 + j] = 1.0 / L[j * 9 + j];
            for (int i = j + 1; i < 9; ++i) {
                double t = 0.0;
                for (int q = j; q < i; ++q) t -= L[i * 9 + q] * L[q * 9 + j];
                L[i * 9 + j] = t / L[i * 9 + i];
            }
        }
    }
    __syncthreads();
    if (live) {
        for (int e = lane; e < 81; e += kWave) {
            const int i = e / 9, j = e % 9;
            double t = 0.0;
            for (int q = (i > j ? i : j); q < 9; ++q) t += L[q * 9 + i] * L[q * 9 + j];
            Minv[(int64_t)row * 81 + e] = t;
            Linv[(int64_t)row * 81 + e] = L[e];
        }
    }
}

// J_a dx of an observation's two records: exterior part with the image's
// row of dx (none for a fixed image), interior part with the camera's row
__device__ __forceinline__ void jdx(const double* __restrict__ R, int k, int img_row, int cam_node,
                                    const double* __restrict__ dxc, double& g0, double& g1) {
    double je[18], jq[18];
    load_jc(R + (int64_t)(2 * k) * kRec, je);
    load_jc(R + (int64_t)(2 * k + 1) * kRec, jq);
    g0 = 0.0; g1 = 0.0;
    if (img_row >= 0) {
        const double* d = dxc + (int64_t)img_row * 9;
#pragma unroll
        for (int i = 0; i < 6; ++i) { g0 += je[i] * d[i]; g1 += je[9 + i] * d[i]; }
    }
    const double* d = dxc + (int64_t)cam_node * 9;
#pragma unroll
    for (int i = 0; i < 5; ++i) { g0 += jq[i] * d[i]; g1 += jq[9 + i] * d[i]; }
}

// dx_p = L^-T (lhat - sum_a K_a^T J_a dx), Eq. (5)
__global__ __launch_bounds__(BS) void k_backsub_s(int n_chunk, const int32_t* __restrict__ chunk_ptr,
                                                  const int32_t* __restrict__ obs_img,
                                                  const int32_t* __restrict__ obs_pt,
                                                  const int32_t* __restrict__ obs_row,
                                                  const int32_t* __restrict__ chunk_q,
                                                  const int32_t* __restrict__ img_cam, int n_free,
                                                  const double* __restrict__ R, const double* __restrict__ ptL,
                                                  const double* __restrict__ dxc, double* __restrict__ dxp) {
    __shared__ double sP[WPB][kWave][3];
    const int wv = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int chunk = blockIdx.x * WPB + wv;
    int k0 = 0, k1 = 0;
    if (chunk < n_chunk) { k0 = chunk_ptr[chunk]; k1 = chunk_ptr[chunk + 1]; }
    const int k = k0 + lane;
    const bool act = k < k1;
    const int p = act ? obs_pt[k] : -1;
    const Track tk = chunk_track(act, p, lane, k1 - k0);
    const int head = tk.head, tl = tk.len;
    const int64_t q = chunk < n_chunk ? (int64_t)chunk_q[chunk] + tk.idx : 0;
    if (act) {
        double g0, g1;
        jdx(R, k, obs_row[k], n_free + img_cam[obs_img[k]], dxc, g0, g1);
        double K[6];
        load6(R + (int64_t)(2 * k) * kRec + 18, K);
        sP[wv][lane][0] = K[0] * g0 + K[3] * g1;
        sP[wv][lane][1] = K[1] * g0 + K[4] * g1;
        sP[wv][lane][2] = K[2] * g0 + K[5] * g1;
    }
    __syncthreads();
    if (act && head == lane) {
        double u0 = 0.0, u1 = 0.0, u2 = 0.0;
        for (int t = 0; t < tl; ++t) { u0 += sP[wv][lane + t][0]; u1 += sP[wv][lane + t][1]; u2 += sP[wv][lane + t][2]; }
        const double* L = ptL + q * 9;
        u0 = L[6] - u0; u1 = L[7] - u1; u2 = L[8] - u2;
        const double x2 = u2 / L[5];
        const double x1 = (u1 - L[4] * x2) / L[2];
        const double x0 = (u0 - L[1] * x1 - L[3] * x2) / L[0];
        dxp[(int64_t)p * 3 + 0] = x0;
        dxp[(int64_t)p * 3 + 1] = x1;
        dxp[(int64_t)p * 3 + 2] = x2;
    }
}

// dx_p of a track longer than a wave (point q0 + blockIdx.x), as k_backsub_s
// with the sums reduced over the workgroup in a fixed order
__global__ __launch_bounds__(BS) void k_backsub_s_long(int q0, const int32_t* __restrict__ long_ptr,
                                                       const int32_t* __restrict__ obs_img,
                                                       const int32_t* __restrict__ obs_pt,
                                                       const int32_t* __restrict__ obs_row,
                                                       const int32_t* __restrict__ img_cam, int n_free,
                                                       const double* __restrict__ R, const double* __restrict__ ptL,
                                                       const double* __restrict__ dxc, double* __restrict__ dxp) {
    __shared__ double sh[3][WPB];
    const int k0 = long_ptr[blockIdx.x], k1 = long_ptr[blockIdx.x + 1];
    const int64_t q = (int64_t)q0 + blockIdx.x;
    const int p = obs_pt[k0];
    double v[3] = {0.0, 0.0, 0.0};
    for (int k = k0 + threadIdx.x; k < k1; k += BS) {
        double g0, g1, K[6];
        jdx(R, k, obs_row[k], n_free + img_cam[obs_img[k]], dxc, g0, g1);
        load6(R + (int64_t)(2 * k) * kRec + 18, K);
        v[0] += K[0] * g0 + K[3] * g1;
        v[1] += K[1] * g0 + K[4] * g1;
        v[2] += K[2] * g0 + K[5] * g1;
    }
    block_reduce<3>(v, sh);
    if (threadIdx.x == 0) {
        const double* L = ptL + q * 9;
        const double u0 = L[6] - v[0], u1 = L[7] - v[1], u2 = L[8] - v[2];
        const double x2 = u2 / L[5];
        const double x1 = (u1 - L[4] * x2) / L[2];
        const double x0 = (u0 - L[1] * x1 - L[3] * x2) / L[0];
        dxp[(int64_t)p * 3 + 0] = x0;
        dxp[(int64_t)p * 3 + 1] = x1;
        dxp[(int64_t)p * 3 + 2] = x2;
    }
}

// F' at the candidate parameters and, from the stored linearization,
// |J dx|^2 and dx^T l (l = -J^T e)
__global__ __launch_bounds__(BS) void k_evaluate_s(int n, const int32_t* __restrict__ obs_img,
                                                   const int32_t* __restrict__ obs_pt,
                                                   const int32_t* __restrict__ obs_row,
                                                   const int32_t* __restrict__ img_cam, int n_img, int n_free,
                                                   const double* __restrict__ uv, const double* __restrict__ params,
                                                   const double* __restrict__ pts, const double* __restrict__ dxc,
                                                   const double* __restrict__ dxp, const double* __restrict__ R,
                                                   const double* __restrict__ Jp, const double* __restrict__ e,
                                                   double* __restrict__ part, int nb) {
    __shared__ double sh[BS / kWave];
    const int k = blockIdx.x * BS + threadIdx.x;
    double cost = 0.0, jdx2 = 0.0, dxl = 0.0;
    if (k < n) {
        const int img = obs_img[k], cam = img_cam[img], row = obs_row[k], node = n_free + cam;
        const int p = obs_pt[k];
        double ext[6], intr[5];
#pragma unroll
        for (int i = 0; i < 6; ++i) ext[i] = params[6 * (int64_t)img + i] + (row >= 0 ? dxc[(int64_t)row * 9 + i] : 0.0);
#pragma unroll
        for (int i = 0; i < 5; ++i) intr[i] = params[6 * (int64_t)n_img + 5 * (int64_t)cam + i] + dxc[(int64_t)node * 9 + i];
        double c9[9];
        compose(ext, intr, c9);
        const double* X = pts + (int64_t)p * 3;
        const double* dX = dxp + (int64_t)p * 3;
        double pu, pv;
        project_point<false>(c9, X[0] + dX[0], X[1] + dX[1], X[2] + dX[2], pu, pv, nullptr, nullptr);
        const double eu = pu + intr[1] - uv[k], ev = pv + intr[2] - uv[n + k];
        cost = 0.5 * (eu * eu + ev * ev);
        double g0, g1;
        jdx(R, k, row, node, dxc, g0, g1);
        double jp[6];
        load6(Jp + (int64_t)k * 6, jp);
#pragma unroll
        for (int i = 0; i < 3; ++i) { g0 += jp[i] * dX[i]; g1 += jp[3 + i] * dX[i]; }
        const double2 ek = reinterpret_cast<const double2*>(e)[k];
        jdx2 = g0 * g0 + g1 * g1;
        dxl = -(g0 * ek.x + g1 * ek.y);
    }
    const double s0 = block_sum<BS>(cost, sh);
    const double s1 = block_sum<BS>(jdx2, sh);
    const double s2 = block_sum<BS>(dxl, sh);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = s0;
        part[nb + blockIdx.x] = s1;
        part[2 * nb + blockIdx.x] = s2;
    }
}

__global__ __launch_bounds__(BS) void k_update_s(int n_img, int n_phys, int n_pts, int n_free,
                                                 const int32_t* __restrict__ cam_row, double* __restrict__ params,
                                                 double* __restrict__ pts, const double* __restrict__ dxc,
                                                 const double* __restrict__ dxp) {
    const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
    const int64_t ne = 6 * (int64_t)n_img, nq = 5 * (int64_t)n_phys;
    if (i < ne) {
        const int img = (int)(i / 6), j = (int)(i % 6);
        const int r = cam_row[img];
        if (r >= 0) params[i] += dxc[(int64_t)r * 9 + j];
    } else if (i < ne + nq) {
        const int cam = (int)((i - ne) / 5), j = (int)((i - ne) % 5);
        params[i] += dxc[(int64_t)(n_free + cam) * 9 + j];
    }
    if (i < (int64_t)n_pts * 3) pts[i] += dxp[i];
}

inline int nblk(int64_t n) { return (int)((n + BS - 1) / BS); }

}  // namespace

void launch_linpoint_shared(ba_ctx* c, const double* params, const double* pts, double lambda) {
    const int nb = (c->n_chunk + WPB - 1) / WPB;
    if (nb + c->n_long == 0) return;
    if (nb + (int64_t)c->n_long > c->n_part)
        throw ba_hip_error(hipErrorInvalidValue, "cost partials exceed their buffer", __FILE__, __LINE__);
    if (nb > 0)
        k_linpoint_s<<<nb, BS, 0, c->stream>>>(c->n_chunk, c->chunk_ptr, (int)c->n_obs, c->obs_cam, c->obs_pt,
                                               c->chunk_q, c->img_cam, c->n_cams, c->obs_uv, params, pts, lambda,
                                               (double*)c->R, (double*)c->Jp, c->e, c->ptL, c->ebar, c->part,
                                               c->flags);
    if (c->n_long > 0)
        k_linpoint_s_long<<<c->n_long, BS, 0, c->stream>>>(c->q_long0, c->long_ptr, (int)c->n_obs, c->obs_cam,
                                                           c->obs_pt, c->img_cam, c->n_cams, c->obs_uv, params, pts,
                                                           lambda, (double*)c->R, (double*)c->Jp, c->e, c->ptL,
                                                           c->ebar, c->part + nb, c->flags);
    launch_reduce(c, c->part, nb + c->n_long, 1, c->scal + 0);
}

void launch_node_diag(ba_ctx* c, double lambda) {
    if (c->n_rows == 0) return;
    k_node_diag<<<(c->n_rows + WPB - 1) / WPB, BS, 0, c->stream>>>(c->n_rows, c->n_free, c->rowobs_ptr, c->rowobs,
                                                                   c->row_ptr, (const double*)c->R, c->ebar, lambda,
                                                                   c->blk, c->rhs, c->Minv, c->Linv, c->flags);
}

void launch_back_substitute_shared(ba_ctx* c, const double* dxc, double* dxp) {
    const int nb = (c->n_chunk + WPB - 1) / WPB;
    if (nb > 0)
        k_backsub_s<<<nb, BS, 0, c->stream>>>(c->n_chunk, c->chunk_ptr, c->obs_cam, c->obs_pt, c->obs_row,
                                              c->chunk_q, c->img_cam, c->n_free, (const double*)c->R, c->ptL, dxc,
                                              dxp);
    if (c->n_long > 0)
        k_backsub_s_long<<<c->n_long, BS, 0, c->stream>>>(c->q_long0, c->long_ptr, c->obs_cam, c->obs_pt,
                                                          c->obs_row, c->img_cam, c->n_free, (const double*)c->R,
                                                          c->ptL, dxc, dxp);
}

void launch_evaluate_shared(ba_ctx* c, const double* params, const double* pts, const double* dxc, const double* dxp) {
    const int n = (int)c->n_obs, nb = nblk(n);
    k_evaluate_s<<<nb, BS, 0, c->stream>>>(n, c->obs_cam, c->obs_pt, c->obs_row, c->img_cam, c->n_cams, c->n_free,
                                           c->obs_uv, params, pts, dxc, dxp, (const double*)c->R, (const double*)c->Jp,
                                           c->e, c->part, nb);
    launch_reduce(c, c->part, nb, 3, c->scal + 1);
}

void launch_update_shared(ba_ctx* c, double* params, double* pts, const double* dxc, const double* dxp) {
    const int64_t n = std::max<int64_t>(6 * (int64_t)c->n_cams + 5 * (int64_t)c->n_phys, 3 * (int64_t)c->n_pts);
    k_update_s<<<nblk(n), BS, 0, c->stream>>>(c->n_cams, c->n_phys, c->n_pts, c->n_free, c->cam_row, params, pts,
                                              dxc, dxp);
}

}  // namespace ba
