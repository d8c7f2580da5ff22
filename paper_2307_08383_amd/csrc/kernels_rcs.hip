// Reduced-camera-system formation (Eq. (3)-(4), Sec. 5) and point
// back-substitution (Eq. (5)).
//
// With V*_p = L_p L_p^T (3x3 Cholesky) every Schur term factors as
//   W_ip V*_p^-1 W_jp^T = What_ip What_jp^T,   What_ip = W_ip L_p^-T  (9x3),
//   W_ip V*_p^-1 l_p    = What_ip lhat_p,      lhat_p = L_p^-1 l_p,
// so the point stage stores one 9x3 record per observation and the camera
// pairs only need products of those records:
//   S_ij = delta_ij U*_i - sum_p What_ip What_jp^T,
//   b_i  = sum_p (-J_ci^T e_ip - What_ip lhat_p).
// The off-diagonal blocks are segmented reductions over the observation
// pairs of each camera pair (sorted once by pair, no atomics); the diagonal
// blocks are reductions over each camera's observations.
#include "ba_common.hpp"

namespace ba {

namespace {

constexpr int BS = 256;
constexpr int WPB = BS / kWave;   // waves per block

template <typename T, int N>
__device__ __forceinline__ void load_vals(const T* __restrict__ src, double* v);

template <>
__device__ __forceinline__ void load_vals<double, 24>(const double* __restrict__ src, double* v) {
    const double2* s2 = reinterpret_cast<const double2*>(src);
#pragma unroll
    for (int i = 0; i < 12; ++i) { double2 t = s2[i]; v[2 * i] = t.x; v[2 * i + 1] = t.y; }
}
template <>
__device__ __forceinline__ void load_vals<float, 24>(const float* __restrict__ src, double* v) {
    const float4* s4 = reinterpret_cast<const float4*>(src);
#pragma unroll
    for (int i = 0; i < 6; ++i) { float4 t = s4[i]; v[4 * i] = t.x; v[4 * i + 1] = t.y; v[4 * i + 2] = t.z; v[4 * i + 3] = t.w; }
}
template <>
__device__ __forceinline__ void load_vals<double, 18>(const double* __restrict__ src, double* v) {
    const double2* s2 = reinterpret_cast<const double2*>(src);
#pragma unroll
    for (int i = 0; i < 9; ++i) { double2 t = s2[i]; v[2 * i] = t.x; v[2 * i + 1] = t.y; }
}
template <>
__device__ __forceinline__ void load_vals<float, 18>(const float* __restrict__ src, double* v) {
    const float2* s2 = reinterpret_cast<const float2*>(src);
#pragma unroll
    for (int i = 0; i < 9; ++i) { float2 t = s2[i]; v[2 * i] = t.x; v[2 * i + 1] = t.y; }
}
// W-hat record: 27 values (padded stride 32)
template <>
__device__ __forceinline__ void load_vals<double, 27>(const double* __restrict__ src, double* v) {
    const double2* s2 = reinterpret_cast<const double2*>(src);
#pragma unroll
    for (int i = 0; i < 13; ++i) { double2 t = s2[i]; v[2 * i] = t.x; v[2 * i + 1] = t.y; }
    v[26] = src[26];
}
template <>
__device__ __forceinline__ void load_vals<float, 27>(const float* __restrict__ src, double* v) {
    const float4* s4 = reinterpret_cast<const float4*>(src);
#pragma unroll
    for (int i = 0; i < 6; ++i) { float4 t = s4[i]; v[4 * i] = t.x; v[4 * i + 1] = t.y; v[4 * i + 2] = t.z; v[4 * i + 3] = t.w; }
    v[24] = src[24]; v[25] = src[25]; v[26] = src[26];
}

template <typename T>
__device__ __forceinline__ void store_what(T* dst, const double* v);
template <>
__device__ __forceinline__ void store_what<double>(double* dst, const double* v) {
    double2* d2 = reinterpret_cast<double2*>(dst);
#pragma unroll
    for (int i = 0; i < 13; ++i) d2[i] = make_double2(v[2 * i], v[2 * i + 1]);
    dst[26] = v[26];
}
template <>
__device__ __forceinline__ void store_what<float>(float* dst, const double* v) {
    float4* d4 = reinterpret_cast<float4*>(dst);
#pragma unroll
    for (int i = 0; i < 6; ++i) d4[i] = make_float4((float)v[4 * i], (float)v[4 * i + 1], (float)v[4 * i + 2], (float)v[4 * i + 3]);
    dst[24] = (float)v[24]; dst[25] = (float)v[25]; dst[26] = (float)v[26];
}

// ---------------------------------------------------------------------------
// point stage: one wave per chunk of whole tracks (<= 64 observations), one
// lane per observation.  Track sums V_p, l_p are reduced through LDS by the
// lane holding the first observation of the track.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(BS) void k_point(int n_chunk, const int32_t* __restrict__ chunk_ptr,
                                              const int32_t* __restrict__ obs_pt, const int32_t* __restrict__ obs_row,
                                              const int32_t* __restrict__ pt_ptr, const T* __restrict__ J,
                                              const double* __restrict__ e, double lambda, T* __restrict__ What,
                                              double* __restrict__ g, double* __restrict__ ptL, int* __restrict__ flags) {
    __shared__ double sP[WPB][kWave][9];
    __shared__ double sR[WPB][kWave][9];
    const int wv = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int chunk = blockIdx.x * WPB + wv;
    int k0 = 0, k1 = 0;
    if (chunk < n_chunk) { k0 = chunk_ptr[chunk]; k1 = chunk_ptr[chunk + 1]; }
    const int k = k0 + lane;
    const bool act = k < k1;
    double v[24];
    double e0 = 0.0, e1 = 0.0;
    int p = 0, head = 0, tl = 0;
    if (act) {
        load_vals<T, 24>(J + (int64_t)k * kJStride, v);
        const double2 ek = reinterpret_cast<const double2*>(e)[k];
        e0 = ek.x; e1 = ek.y;
        p = obs_pt[k];
        const int b = pt_ptr[p];
        head = b - k0;
        tl = pt_ptr[p + 1] - b;
        const double* Jp = v + 18;
        sP[wv][lane][0] = Jp[0] * Jp[0] + Jp[3] * Jp[3];
        sP[wv][lane][1] = Jp[0] * Jp[1] + Jp[3] * Jp[4];
        sP[wv][lane][2] = Jp[0] * Jp[2] + Jp[3] * Jp[5];
        sP[wv][lane][3] = Jp[1] * Jp[1] + Jp[4] * Jp[4];
        sP[wv][lane][4] = Jp[1] * Jp[2] + Jp[4] * Jp[5];
        sP[wv][lane][5] = Jp[2] * Jp[2] + Jp[5] * Jp[5];
        sP[wv][lane][6] = -(Jp[0] * e0 + Jp[3] * e1);
        sP[wv][lane][7] = -(Jp[1] * e0 + Jp[4] * e1);
        sP[wv][lane][8] = -(Jp[2] * e0 + Jp[5] * e1);
    }
    __syncthreads();
    if (act && head == lane) {
        double s[9];
#pragma unroll
        for (int m = 0; m < 9; ++m) s[m] = 0.0;
        for (int q = 0; q < tl; ++q)
#pragma unroll
            for (int m = 0; m < 9; ++m) s[m] += sP[wv][lane + q][m];
        // V* = V + lambda diag(V), then V* = L L^T
        const double V00 = s[0] * (1.0 + lambda), V11 = s[3] * (1.0 + lambda), V22 = s[5] * (1.0 + lambda);
        const double L00 = sqrt(V00);
        const double L10 = s[1] / L00, L20 = s[2] / L00;
        const double d1 = V11 - L10 * L10;
        const double L11 = sqrt(d1);
        const double L21 = (s[4] - L20 * L10) / L11;
        const double d2 = V22 - L20 * L20 - L21 * L21;
        const double L22 = sqrt(d2);
        if (!(V00 > 0.0) || !(d1 > 0.0) || !(d2 > 0.0)) flags[0] = 1;
        const double y0 = s[6] / L00;
        const double y1 = (s[7] - L10 * y0) / L11;
        const double y2 = (s[8] - L20 * y0 - L21 * y1) / L22;
        const double r[9] = {L00, L10, L11, L20, L21, L22, y0, y1, y2};
#pragma unroll
        for (int m = 0; m < 9; ++m) { sR[wv][lane][m] = r[m]; ptL[(int64_t)p * 9 + m] = r[m]; }
    }
    __syncthreads();
    if (act) {
        const double L00 = sR[wv][head][0], L10 = sR[wv][head][1], L11 = sR[wv][head][2];
        const double L20 = sR[wv][head][3], L21 = sR[wv][head][4], L22 = sR[wv][head][5];
        const double h0 = sR[wv][head][6], h1 = sR[wv][head][7], h2 = sR[wv][head][8];
        const double i00 = 1.0 / L00, i11 = 1.0 / L11, i22 = 1.0 / L22;
        const double* Jc = v;
        const double* Jp = v + 18;
        double wh[27];
        const int row = obs_row[k];
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            // row i of W = J_c^T J_p, then solve L y = w_i^T
            const double w0 = Jc[i] * Jp[0] + Jc[9 + i] * Jp[3];
            const double w1 = Jc[i] * Jp[1] + Jc[9 + i] * Jp[4];
            const double w2 = Jc[i] * Jp[2] + Jc[9 + i] * Jp[5];
            const double y0 = w0 * i00;
            const double y1 = (w1 - L10 * y0) * i11;
            const double y2 = (w2 - L20 * y0 - L21 * y1) * i22;
            wh[3 * i] = y0; wh[3 * i + 1] = y1; wh[3 * i + 2] = y2;
        }
        store_what<T>(What + (int64_t)k * kWhatStride, wh);
        if (row >= 0) {
            double* gk = g + (int64_t)k * 9;
#pragma unroll
            for (int i = 0; i < 9; ++i)
                gk[i] = -(Jc[i] * e0 + Jc[9 + i] * e1) - (wh[3 * i] * h0 + wh[3 * i + 1] * h1 + wh[3 * i + 2] * h2);
        }
    }
}

// ---------------------------------------------------------------------------
// off-diagonal pair stage: G lanes per camera pair (BS/G pairs per block),
// each lane accumulating the full 9x9 product over a strided subset of the
// pair's observation couples, then a shuffle reduction inside the group.
// ---------------------------------------------------------------------------
template <typename T, int G>
__global__ __launch_bounds__(BS) void k_offdiag(int n_seg, const int32_t* __restrict__ off_blk,
                                                const int32_t* __restrict__ pair_ptr, const int32_t* __restrict__ trip,
                                                const T* __restrict__ What, double* __restrict__ blk) {
    const int gl = threadIdx.x % G;
    const int seg = blockIdx.x * (BS / G) + threadIdx.x / G;
    double acc[81];
#pragma unroll
    for (int m = 0; m < 81; ++m) acc[m] = 0.0;
    int t0 = 0, t1 = 0;
    if (seg < n_seg) { t0 = pair_ptr[seg]; t1 = pair_ptr[seg + 1]; }
    for (int t = t0 + gl; t < t1; t += G) {
        const int2 ab = reinterpret_cast<const int2*>(trip)[t];
        double wb[27];
        load_vals<T, 27>(What + (int64_t)ab.y * kWhatStride, wb);
        const T* wa_p = What + (int64_t)ab.x * kWhatStride;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const double a0 = (double)wa_p[3 * i], a1 = (double)wa_p[3 * i + 1], a2 = (double)wa_p[3 * i + 2];
#pragma unroll
            for (int j = 0; j < 9; ++j) acc[i * 9 + j] += a0 * wb[3 * j] + a1 * wb[3 * j + 1] + a2 * wb[3 * j + 2];
        }
    }
#pragma unroll
    for (int m = 0; m < 81; ++m)
#pragma unroll
        for (int o = G / 2; o > 0; o >>= 1) acc[m] += __shfl_xor(acc[m], o, kWave);
    if (seg < n_seg) {
        double* out = blk + (int64_t)off_blk[seg] * 81;
#pragma unroll
        for (int m = 0; m < 81; ++m)
            if ((m % G) == gl) out[m] = -acc[m];
    }
}

// ---------------------------------------------------------------------------
// diagonal stage: one wave per RCS row over the camera's observations;
// S_ii = sum (J_c^T J_c - What What^T) + lambda diag(U), b_i = sum g, then
// the block-Jacobi inverse S_ii^-1 (Cholesky, triangular inverse).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(BS) void k_diag(int n_rows, const int32_t* __restrict__ rowobs_ptr,
                                             const int32_t* __restrict__ rowobs, const int32_t* __restrict__ row_ptr,
                                             const T* __restrict__ J, const T* __restrict__ What,
                                             const double* __restrict__ g, double lambda, double* __restrict__ blk,
                                             double* __restrict__ rhs, double* __restrict__ Minv, int* __restrict__ flags) {
    __shared__ double sS[WPB][81];
    __shared__ double sL[WPB][81];
    __shared__ double sb[WPB][9];
    const int wv = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int row = blockIdx.x * WPB + wv;
    double A[45], du[9], bb[9];
#pragma unroll
    for (int m = 0; m < 45; ++m) A[m] = 0.0;
#pragma unroll
    for (int m = 0; m < 9; ++m) { du[m] = 0.0; bb[m] = 0.0; }
    int i0 = 0, i1 = 0;
    if (row < n_rows) { i0 = rowobs_ptr[row]; i1 = rowobs_ptr[row + 1]; }
    for (int idx = i0 + lane; idx < i1; idx += kWave) {
        const int k = rowobs[idx];
        double jc[18], wh[27];
        load_vals<T, 18>(J + (int64_t)k * kJStride, jc);
        load_vals<T, 27>(What + (int64_t)k * kWhatStride, wh);
        const double* gk = g + (int64_t)k * 9;
        int m = 0;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            du[i] += jc[i] * jc[i] + jc[9 + i] * jc[9 + i];
            bb[i] += gk[i];
#pragma unroll
            for (int j = i; j < 9; ++j, ++m)
                A[m] += jc[i] * jc[j] + jc[9 + i] * jc[9 + j]
                        - (wh[3 * i] * wh[3 * j] + wh[3 * i + 1] * wh[3 * j + 1] + wh[3 * i + 2] * wh[3 * j + 2]);
        }
    }
#pragma unroll
    for (int m = 0; m < 45; ++m) A[m] = wave_sum(A[m]);
#pragma unroll
    for (int m = 0; m < 9; ++m) { du[m] = wave_sum(du[m]); bb[m] = wave_sum(bb[m]); }
    if (lane == 0) {
        int m = 0;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            sb[wv][i] = bb[i];
#pragma unroll
            for (int j = i; j < 9; ++j, ++m) {
                const double v = A[m] + (i == j ? lambda * du[i] : 0.0);
                sS[wv][i * 9 + j] = v;
                sS[wv][j * 9 + i] = v;
            }
        }
    }
    __syncthreads();
    if (row < n_rows) {
        double* out = blk + (int64_t)row_ptr[row] * 81;
        out[lane] = sS[wv][lane];
        if (lane < 17) out[64 + lane] = sS[wv][64 + lane];
        if (lane < 9) rhs[(int64_t)row * 9 + lane] = sb[wv][lane];
        if (lane == 0) {
            // Cholesky S = L L^T in sL, then L^-1 in place (lower triangle)
            double* L = sL[wv];
            const double* S = sS[wv];
            bool ok = true;
            for (int j = 0; j < 9; ++j) {
                double s = S[j * 9 + j];
                for (int q = 0; q < j; ++q) s -= L[j * 9 + q] * L[j * 9 + q];
                if (!(s > 0.0)) { ok = false; s = 1.0; }
                const double ljj = sqrt(s);
                L[j * 9 + j] = ljj;
                for (int i = j + 1; i < 9; ++i) {
                    double t = S[i * 9 + j];
                    for (int q = 0; q < j; ++q) t -= L[i * 9 + q] * L[j * 9 + q];
                    L[i * 9 + j] = t / ljj;
                }
                for (int i = 0; i < j; ++i) L[i * 9 + j] = 0.0;
            }
            if (!ok) flags[1] = 1;
            // in-place inverse of the lower-triangular L
            for (int j = 0; j < 9; ++j) {
                L[j * 9 + j] = 1.0 / L[j * 9 + j];
                for (int i = j + 1; i < 9; ++i) {
                    double t = 0.0;
                    for (int q = j; q < i; ++q) t -= L[i * 9 + q] * L[q * 9 + j];
                    L[i * 9 + j] = t / L[i * 9 + i];
                }
            }
        }
    }
    __syncthreads();
    if (row < n_rows) {
        // S^-1 = L^-T L^-1: entry (i, j) = sum_{q >= max(i,j)} Li[q][i] Li[q][j]
        const double* Li = sL[wv];
        double* M = Minv + (int64_t)row * 81;
        for (int m = lane; m < 81; m += kWave) {
            const int i = m / 9, j = m % 9;
            double t = 0.0;
            for (int q = (i > j ? i : j); q < 9; ++q) t += Li[q * 9 + i] * Li[q * 9 + j];
            M[m] = t;
        }
    }
}

// ---------------------------------------------------------------------------
// back-substitution (Eq. (5)): dx_p = L^-T (lhat - sum_a What_a^T dxc_a)
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(BS) void k_backsub(int n_chunk, const int32_t* __restrict__ chunk_ptr,
                                                const int32_t* __restrict__ obs_pt, const int32_t* __restrict__ obs_row,
                                                const int32_t* __restrict__ pt_ptr, const T* __restrict__ What,
                                                const double* __restrict__ ptL, const double* __restrict__ dxc,
                                                double* __restrict__ dxp) {
    __shared__ double sP[WPB][kWave][3];
    const int wv = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int chunk = blockIdx.x * WPB + wv;
    int k0 = 0, k1 = 0;
    if (chunk < n_chunk) { k0 = chunk_ptr[chunk]; k1 = chunk_ptr[chunk + 1]; }
    const int k = k0 + lane;
    const bool act = k < k1;
    int p = 0, head = -1, tl = 0;
    if (act) {
        p = obs_pt[k];
        const int b = pt_ptr[p];
        head = b - k0;
        tl = pt_ptr[p + 1] - b;
        const int row = obs_row[k];
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        if (row >= 0) {
            double wh[27];
            load_vals<T, 27>(What + (int64_t)k * kWhatStride, wh);
            const double* dc = dxc + (int64_t)row * 9;
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                const double c = dc[i];
                s0 += wh[3 * i] * c; s1 += wh[3 * i + 1] * c; s2 += wh[3 * i + 2] * c;
            }
        }
        sP[wv][lane][0] = s0; sP[wv][lane][1] = s1; sP[wv][lane][2] = s2;
    }
    __syncthreads();
    if (act && head == lane) {
        double u0 = 0.0, u1 = 0.0, u2 = 0.0;
        for (int q = 0; q < tl; ++q) { u0 += sP[wv][lane + q][0]; u1 += sP[wv][lane + q][1]; u2 += sP[wv][lane + q][2]; }
        const double* L = ptL + (int64_t)p * 9;
        u0 = L[6] - u0; u1 = L[7] - u1; u2 = L[8] - u2;
        // L^T x = u with L = [[L00,0,0],[L10,L11,0],[L20,L21,L22]]
        const double x2 = u2 / L[5];
        const double x1 = (u1 - L[4] * x2) / L[2];
        const double x0 = (u0 - L[1] * x1 - L[3] * x2) / L[0];
        dxp[(int64_t)p * 3 + 0] = x0;
        dxp[(int64_t)p * 3 + 1] = x1;
        dxp[(int64_t)p * 3 + 2] = x2;
    }
}

constexpr int kPairLanes = 16;

}  // namespace

void launch_point(ba_ctx* c, double lambda) {
    const int nb = (c->n_chunk + WPB - 1) / WPB;
    if (nb == 0) return;
    if (c->precision == BA_MIXED)
        k_point<float><<<nb, BS, 0, c->stream>>>(c->n_chunk, c->chunk_ptr, c->obs_pt, c->obs_row, c->pt_ptr,
                                                 (const float*)c->J, c->e, lambda, (float*)c->What, c->g, c->ptL, c->flags);
    else
        k_point<double><<<nb, BS, 0, c->stream>>>(c->n_chunk, c->chunk_ptr, c->obs_pt, c->obs_row, c->pt_ptr,
                                                  (const double*)c->J, c->e, lambda, (double*)c->What, c->g, c->ptL, c->flags);
}

void launch_offdiag(ba_ctx* c) {
    constexpr int G = kPairLanes;
    const int nb = (c->n_offseg + (BS / G) - 1) / (BS / G);
    if (nb == 0) return;
    if (c->precision == BA_MIXED)
        k_offdiag<float, G><<<nb, BS, 0, c->stream>>>(c->n_offseg, c->off_blk, c->pair_ptr, c->trip,
                                                      (const float*)c->What, c->blk);
    else
        k_offdiag<double, G><<<nb, BS, 0, c->stream>>>(c->n_offseg, c->off_blk, c->pair_ptr, c->trip,
                                                       (const double*)c->What, c->blk);
}

void launch_diag(ba_ctx* c, double lambda) {
    const int nb = (c->n_rows + WPB - 1) / WPB;
    if (nb == 0) return;
    if (c->precision == BA_MIXED)
        k_diag<float><<<nb, BS, 0, c->stream>>>(c->n_rows, c->rowobs_ptr, c->rowobs, c->row_ptr, (const float*)c->J,
                                                (const float*)c->What, c->g, lambda, c->blk, c->rhs, c->Minv, c->flags);
    else
        k_diag<double><<<nb, BS, 0, c->stream>>>(c->n_rows, c->rowobs_ptr, c->rowobs, c->row_ptr, (const double*)c->J,
                                                 (const double*)c->What, c->g, lambda, c->blk, c->rhs, c->Minv, c->flags);
}

void launch_back_substitute(ba_ctx* c, const double* dxc, double* dxp) {
    const int nb = (c->n_chunk + WPB - 1) / WPB;
    if (nb == 0) return;
    if (c->precision == BA_MIXED)
        k_backsub<float><<<nb, BS, 0, c->stream>>>(c->n_chunk, c->chunk_ptr, c->obs_pt, c->obs_row, c->pt_ptr,
                                                   (const float*)c->What, c->ptL, dxc, dxp);
    else
        k_backsub<double><<<nb, BS, 0, c->stream>>>(c->n_chunk, c->chunk_ptr, c->obs_pt, c->obs_row, c->pt_ptr,
                                                    (const double*)c->What, c->ptL, dxc, dxp);
}

}  // namespace ba
