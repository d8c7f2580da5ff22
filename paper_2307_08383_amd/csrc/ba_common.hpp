// Internal declarations of the MI355X bundle-adjustment library: context
// layout, device math shared by the kernels, and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "../../include/ba.h"

namespace ba {

constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kMaxTrack = 64;      // observations per point handled by one wave (longer tracks: one workgroup)
constexpr int kPcgBatch = 16;      // PCG iterations per enqueued batch (one graph)
constexpr int kRec = 24;           // per-observation record: J_c (18), then K = J_p L^-T (6)

// Durations of the phases of a host build (ba_create, the FSAI index
// structure) on stderr when BA_TIMING is set in the environment.
struct Phases {
    const char* label;
    bool on = std::getenv("BA_TIMING") != nullptr;
    std::chrono::steady_clock::time_point t = std::chrono::steady_clock::now();
    explicit Phases(const char* l) : label(l) {}
    void mark(const char* what) {
        if (!on) return;
        const auto now = std::chrono::steady_clock::now();
        std::fprintf(stderr, "%s %-14s %9.1f ms\n", label, what,
                     std::chrono::duration<double, std::milli>(now - t).count());
        t = now;
    }
};

// ---------------------------------------------------------------------------
// device math
// ---------------------------------------------------------------------------

// Coefficients of R(w) X = X + a (w x X) + b w x (w x X), with s = |w|^2,
// a = sin(th)/th, b = (1 - cos th)/th^2 and their s-derivatives as = da/ds,
// bs = db/ds.  Below th = 0.5 the Taylor series in s (truncated after the
// s^7 term, error < 1e-17) avoids the cancellation of the closed forms.
__device__ __forceinline__ void rot_coeffs(double s, double& a, double& b, double& as, double& bs) {
    if (s < 0.25) {
        a = 1.0 + s * (-1.0 / 6 + s * (1.0 / 120 + s * (-1.0 / 5040 + s * (1.0 / 362880 + s * (-1.0 / 39916800 + s * (1.0 / 6227020800.0 + s * (-1.0 / 1307674368000.0)))))));
        b = 0.5 + s * (-1.0 / 24 + s * (1.0 / 720 + s * (-1.0 / 40320 + s * (1.0 / 3628800 + s * (-1.0 / 479001600 + s * (1.0 / 87178291200.0 + s * (-1.0 / 20922789888000.0)))))));
        as = -1.0 / 6 + s * (2.0 / 120 + s * (-3.0 / 5040 + s * (4.0 / 362880 + s * (-5.0 / 39916800 + s * (6.0 / 6227020800.0 + s * (-7.0 / 1307674368000.0))))));
        bs = -1.0 / 24 + s * (2.0 / 720 + s * (-3.0 / 40320 + s * (4.0 / 3628800 + s * (-5.0 / 479001600 + s * (6.0 / 87178291200.0 + s * (-7.0 / 20922789888000.0))))));
    } else {
        const double th = sqrt(s), it = 1.0 / th, is = it * it;   // one division
        double sn, cs;
        sincos(th, &sn, &cs);
        const double sh = sin(0.5 * th);
        const double omc = 2.0 * sh * sh;   // 1 - cos th without cancellation
        a = sn * it;
        b = omc * is;
        as = (th * cs - sn) * (0.5 * is * it);
        bs = (th * sn - 2.0 * omc) * (0.5 * is * is);
    }
}

// Predicted pixel of point X in camera c (9 params) and, if JAC, the
// hand-derived Jacobian rows: Jc[r*9 + j] = d pix_r / d c_j,
// Jp[r*3 + j] = d pix_r / d X_j.
//   dP/dw = 2 as (w x X) w^T - a [X]x + 2 bs (w x (w x X)) w^T
//           + b ((w.X) I + w X^T - 2 X w^T)
//   dP/dX = R = I + a [w]x + b (w w^T - s I)
template <bool JAC, bool JC = true>
__device__ __forceinline__ void project_point(const double* __restrict__ c, double X0, double X1, double X2,
                                              double& pu, double& pv, double* Jc, double* Jp) {
    const double w0 = c[0], w1 = c[1], w2 = c[2];
    const double s = w0 * w0 + w1 * w1 + w2 * w2;
    double a, b, as, bs;
    rot_coeffs(s, a, b, as, bs);
    const double cx0 = w1 * X2 - w2 * X1, cx1 = w2 * X0 - w0 * X2, cx2 = w0 * X1 - w1 * X0;
    const double cc0 = w1 * cx2 - w2 * cx1, cc1 = w2 * cx0 - w0 * cx2, cc2 = w0 * cx1 - w1 * cx0;
    const double P0 = X0 + a * cx0 + b * cc0 + c[3];
    const double P1 = X1 + a * cx1 + b * cc1 + c[4];
    const double P2 = X2 + a * cx2 + b * cc2 + c[5];
    const double iz = 1.0 / P2;
    const double x = P0 * iz, y = P1 * iz;
    const double r2 = x * x + y * y;
    const double f = c[6], k1 = c[7], k2 = c[8];
    const double d = 1.0 + r2 * (k1 + k2 * r2);
    pu = f * d * x;
    pv = f * d * y;
    if (!JAC) return;
    const double dd = k1 + 2.0 * k2 * r2;
    const double A00 = f * (d + 2.0 * x * x * dd), A01 = f * (2.0 * x * y * dd), A11 = f * (d + 2.0 * y * y * dd);
    const double E00 = A00 * iz, E01 = A01 * iz, E02 = -(A00 * x + A01 * y) * iz;
    const double E10 = A01 * iz, E11 = A11 * iz, E12 = -(A01 * x + A11 * y) * iz;
    if (JC) {
    const double wX = w0 * X0 + w1 * X1 + w2 * X2;
    const double g0 = 2.0 * (as * cx0 + bs * cc0), g1 = 2.0 * (as * cx1 + bs * cc1), g2 = 2.0 * (as * cx2 + bs * cc2);
    const double M00 = g0 * w0 + b * (wX + w0 * X0 - 2.0 * X0 * w0);
    const double M01 = g0 * w1 + a * X2 + b * (w0 * X1 - 2.0 * X0 * w1);
    const double M02 = g0 * w2 - a * X1 + b * (w0 * X2 - 2.0 * X0 * w2);
    const double M10 = g1 * w0 - a * X2 + b * (w1 * X0 - 2.0 * X1 * w0);
    const double M11 = g1 * w1 + b * (wX + w1 * X1 - 2.0 * X1 * w1);
    const double M12 = g1 * w2 + a * X0 + b * (w1 * X2 - 2.0 * X1 * w2);
    const double M20 = g2 * w0 + a * X1 + b * (w2 * X0 - 2.0 * X2 * w0);
    const double M21 = g2 * w1 - a * X0 + b * (w2 * X1 - 2.0 * X2 * w1);
    const double M22 = g2 * w2 + b * (wX + w2 * X2 - 2.0 * X2 * w2);
    Jc[0] = E00 * M00 + E01 * M10 + E02 * M20;
    Jc[1] = E00 * M01 + E01 * M11 + E02 * M21;
    Jc[2] = E00 * M02 + E01 * M12 + E02 * M22;
    Jc[3] = E00; Jc[4] = E01; Jc[5] = E02;
    Jc[6] = d * x; Jc[7] = f * x * r2; Jc[8] = f * x * r2 * r2;
    Jc[9] = E10 * M00 + E11 * M10 + E12 * M20;
    Jc[10] = E10 * M01 + E11 * M11 + E12 * M21;
    Jc[11] = E10 * M02 + E11 * M12 + E12 * M22;
    Jc[12] = E10; Jc[13] = E11; Jc[14] = E12;
    Jc[15] = d * y; Jc[16] = f * y * r2; Jc[17] = f * y * r2 * r2;
    }
    const double R00 = 1.0 + b * (w0 * w0 - s), R01 = -a * w2 + b * w0 * w1, R02 = a * w1 + b * w0 * w2;
    const double R10 = a * w2 + b * w1 * w0, R11 = 1.0 + b * (w1 * w1 - s), R12 = -a * w0 + b * w1 * w2;
    const double R20 = -a * w1 + b * w2 * w0, R21 = a * w0 + b * w2 * w1, R22 = 1.0 + b * (w2 * w2 - s);
    Jp[0] = E00 * R00 + E01 * R10 + E02 * R20;
    Jp[1] = E00 * R01 + E01 * R11 + E02 * R21;
    Jp[2] = E00 * R02 + E01 * R12 + E02 * R22;
    Jp[3] = E10 * R00 + E11 * R10 + E12 * R20;
    Jp[4] = E10 * R01 + E11 * R11 + E12 * R21;
    Jp[5] = E10 * R02 + E11 * R12 + E12 * R22;
}

// The Jacobian blocks of an observation fit the record type T (FP32 records
// overflow above 3.4e38) and the residual is finite.  NaN compares false.
template <typename T>
__device__ __forceinline__ bool records_in_range(const double* Jc, const double* Jp, double eu, double ev) {
    constexpr double kMax = sizeof(T) == 4 ? 3.4028234663852886e38 : 1.7976931348623157e308;
    bool ok = fabs(eu) <= 1.7976931348623157e308 && fabs(ev) <= 1.7976931348623157e308;
#pragma unroll
    for (int m = 0; m < 18; ++m) ok = ok && fabs(Jc[m]) <= kMax;
#pragma unroll
    for (int m = 0; m < 6; ++m) ok = ok && fabs(Jp[m]) <= kMax;
    return ok;
}

// Typed record access (T = double, or float for the mixed-precision path).
// Records start on 16-byte boundaries (24 values of 8 or 4 bytes); the K part
// and the separate J_p rows are 8-byte aligned.
__device__ __forceinline__ void load_jc(const double* __restrict__ r, double* v) {
    const double2* p = reinterpret_cast<const double2*>(r);
#pragma unroll
    for (int i = 0; i < 9; ++i) { const double2 t = p[i]; v[2 * i] = t.x; v[2 * i + 1] = t.y; }
}
__device__ __forceinline__ void load_jc(const float* __restrict__ r, double* v) {
    const float4* p = reinterpret_cast<const float4*>(r);
#pragma unroll
    for (int i = 0; i < 4; ++i) { const float4 t = p[i]; v[4 * i] = t.x; v[4 * i + 1] = t.y; v[4 * i + 2] = t.z; v[4 * i + 3] = t.w; }
    const float2 t = reinterpret_cast<const float2*>(r)[8];
    v[16] = t.x; v[17] = t.y;
}
__device__ __forceinline__ void store_jc(double* __restrict__ r, const double* v) {
    double2* p = reinterpret_cast<double2*>(r);
#pragma unroll
    for (int i = 0; i < 9; ++i) p[i] = make_double2(v[2 * i], v[2 * i + 1]);
}
__device__ __forceinline__ void store_jc(float* __restrict__ r, const double* v) {
    float4* p = reinterpret_cast<float4*>(r);
#pragma unroll
    for (int i = 0; i < 4; ++i) p[i] = make_float4((float)v[4 * i], (float)v[4 * i + 1], (float)v[4 * i + 2], (float)v[4 * i + 3]);
    reinterpret_cast<float2*>(r)[8] = make_float2((float)v[16], (float)v[17]);
}
// six values at an 8-byte aligned address (the K part of a record, J_p rows)
__device__ __forceinline__ void load6(const double* __restrict__ r, double* v) {
    const double2* p = reinterpret_cast<const double2*>(r);
#pragma unroll
    for (int i = 0; i < 3; ++i) { const double2 t = p[i]; v[2 * i] = t.x; v[2 * i + 1] = t.y; }
}
__device__ __forceinline__ void load6(const float* __restrict__ r, double* v) {
    const float2* p = reinterpret_cast<const float2*>(r);
#pragma unroll
    for (int i = 0; i < 3; ++i) { const float2 t = p[i]; v[2 * i] = t.x; v[2 * i + 1] = t.y; }
}
__device__ __forceinline__ void store6(double* __restrict__ r, const double* v) {
    double2* p = reinterpret_cast<double2*>(r);
#pragma unroll
    for (int i = 0; i < 3; ++i) p[i] = make_double2(v[2 * i], v[2 * i + 1]);
}
__device__ __forceinline__ void store6(float* __restrict__ r, const double* v) {
    float2* p = reinterpret_cast<float2*>(r);
#pragma unroll
    for (int i = 0; i < 3; ++i) p[i] = make_float2((float)v[2 * i], (float)v[2 * i + 1]);
}

// J_p = K L^T (K = J_p L^-T, the record's last 6 values; L the point's
// Cholesky factor packed as L00, L10, L11, L20, L21, L22)
__device__ __forceinline__ void jp_from_K(const double* K, const double* L, double* jp) {
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const double a = K[3 * r], b = K[3 * r + 1], c = K[3 * r + 2];
        jp[3 * r] = a * L[0];
        jp[3 * r + 1] = a * L[1] + b * L[2];
        jp[3 * r + 2] = a * L[3] + b * L[4] + c * L[5];
    }
}

// v from another lane by a DPP lane pattern (CTRL), both halves of the double
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
// v from lane ^ 16 (swizzle, bit mode, inside each 32 lanes)
__device__ __forceinline__ double swz_xor16(double v) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_ds_swizzle((int)(unsigned)b, 0x401F);
    const int hi = __builtin_amdgcn_ds_swizzle((int)(unsigned)(b >> 32), 0x401F);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
// Sum over the wave, the same value in every lane: each step adds the value
// of a partner lane (the pairing is symmetric, so both partners form the same
// sum): lane ^ 1 and lane ^ 2 (quad permutes), the mirrored lane within 8 and
// within 16 (DPP), lane ^ 16 (swizzle), lane ^ 32.
__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_mov<0xB1>(v);
    v += dpp_mov<0x4E>(v);
    v += dpp_mov<0x141>(v);
    v += dpp_mov<0x140>(v);
    v += swz_xor16(v);
    v += __shfl_xor(v, 32, kWave);
    return v;
}

// Track of a lane of a wave that holds a chunk of whole tracks (lane i holds
// the chunk's observation i, i < len; a track's observations are adjacent):
// the lane of the track's first observation, the track length and the
// track's index among the chunk's tracks.  Called by every lane of the wave.
struct Track { int head, len, idx; };
__device__ __forceinline__ Track chunk_track(bool act, int p, int lane, int len) {
    const int prev = __shfl_up(p, 1, kWave);
    const bool first = act && (lane == 0 || prev != p);
    const unsigned long long heads = __ballot(first);
    const unsigned long long upto = heads & (~0ull >> (63 - lane));   // heads at lanes <= lane
    const unsigned long long after = heads & ~upto;                   // heads at lanes > lane
    Track t;
    t.head = upto ? 63 - __clzll(upto) : 0;
    t.len = (after ? __ffsll((long long)after) - 1 : len) - t.head;
    t.idx = __popcll(upto) - 1;
    return t;
}

// Block index in XCD-contiguous order: the blocks that run on one XCD
// (hardware block id mod 8) take one contiguous range of indices, so the
// lines that neighbouring blocks share stay in that XCD's L2.
__device__ __forceinline__ int xcd_block() {
    const int nb = gridDim.x, x = blockIdx.x % 8, per = nb / 8, extra = nb % 8;
    return x * per + min(x, extra) + blockIdx.x / 8;
}

// Deterministic block sum (fixed shuffle tree, then fixed LDS order); the
// result is valid in thread 0.
template <int BS>
__device__ __forceinline__ double block_sum(double v, double* sh) {
    v = wave_sum(v);
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < BS / kWave; ++i) t += sh[i];
    __syncthreads();
    return t;
}

// Deterministic sums of NV values over a workgroup of NW waves: each
// thread's value, the wave's shuffle tree, then the waves in order.  Every
// thread receives the totals in v.  Called by every thread of the workgroup.
template <int NV, int NW>
__device__ __forceinline__ void block_reduce(double* v, double (*sh)[NW]) {
    const int wv = threadIdx.x / kWave, lane = threadIdx.x % kWave;
#pragma unroll
    for (int m = 0; m < NV; ++m) {
        const double w = wave_sum(v[m]);
        if (lane == 0) sh[m][wv] = w;
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < NV; ++m) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) t += sh[m][w];
        v[m] = t;
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
struct Pcg {
    double *x = nullptr, *r[2] = {nullptr, nullptr}, *z = nullptr, *q = nullptr, *d = nullptr, *t = nullptr;
    double* pA = nullptr;      // per-block partials of d^T q
    double* pR = nullptr;      // per-block partials of r^T z, r^T r, (S W)^T z, two step parities
    double *W = nullptr, *SW = nullptr;   // gauge vectors and S W, [n_rows][7][9]
    double *Einv = nullptr, *pW = nullptr, *pE = nullptr;
    int* state = nullptr;      // [0] done, [1] step, [2] status, [3] completed steps
    double* scal = nullptr;    // [0] r0^2, [1] final relres
    // UPPER product: u [n_rows][9] = the upper blocks' part of S z,
    // tb [n_blk][9] = S_rs^T z_r of each stored block
    double *u = nullptr, *tb = nullptr;
    double* bm = nullptr;      // [8] beta and mu of the step, from the first UPPER kernel to the
                               // second; [8..57) the sums of E = W^T S W (deflation set-up)
};

// Factorised sparse approximate inverse G (M^-1 = G^T G) on the lower RCS
// pattern.  Row i's set J_i: at most kFsaiM - 1 lower neighbours (the ones
// with the most common points) and i itself, ascending.
constexpr int kFsaiM = 28;
constexpr int kFsaiTiles = kFsaiM * (kFsaiM + 1) / 2;
struct Fsai {
    bool built = false, ready = false;
    int32_t *ptr = nullptr;           // [n_rows+1] into J / slot
    int32_t *J = nullptr;             // members of each set
    int32_t *slot = nullptr;          // block slot of G_{i, J_b}: upper block (J_b, i), or i's diagonal
    int64_t *tptr = nullptr;          // [n_rows+1] into tile
    int32_t *tile = nullptr;          // per set, lower tiles (a, b), a >= b, packed a(a+1)/2 + b:
                                      // upper block (J_b, J_a), -2 on the diagonal, -1 if absent
    int32_t *brow = nullptr;          // [n_blk] block row of every RCS block
    int32_t *gu_ptr = nullptr, *gu_col = nullptr;   // rows of G^T: [n_rows+1], column (row i of G)
    int32_t *gu_pos = nullptr;        // per set member (like J): its position in the rows of G^T
    int32_t max_m = 0;
    int64_t n_mem = 0;                // members of all sets (entries of Gl)
    float *Gl = nullptr, *Gu = nullptr;   // G by rows (like J) and G^T by rows (like gu_col), 9x9 each
    float* An = nullptr;              // [n_blk][81] L_r^-1 S_rc L_c^-T of off-diagonal blocks
    float* G = nullptr;               // [n_blk][81] G in the upper slots
    int32_t* gu_src = nullptr;        // entry of Gl for each entry of Gu (inverse of gu_pos)
    // Gu holds G^T by rows of G^T (entry gu_pos[e] for Gl entry e; FULL
    // products), or, with gu_upper, each Gl block transposed at its own
    // entry (gl_self = identity; the UPPER apply reads columns of G as rows)
    int32_t* gl_self = nullptr;
    int gu_upper = 0;
    double* tg = nullptr;             // [entries][9] G_ij^T t_i per entry of Gl (UPPER apply of G^T)
    // half-precision copy for the UPPER apply: member e (G_e = G_{i,j},
    // j = J[e]) as Gh_e = G_e D_j^-1 / hs[e] in FP16, D_j = diag(S_jj)^-1/2
    // (Dn [n_rows][9]), hs[e] = max |G_e D_j^-1|; rows 0..7 of column c of
    // G_e as eight halves in one 16-byte group (Gh[e * 36 + 4 c ..], 144
    // bytes per member), row 8 in Gh8[e * 9 + c] (the array after the groups
    // of all members)
    uint32_t* Gh = nullptr;
    uint16_t* Gh8 = nullptr;
    float* hs = nullptr;
    double* Dn = nullptr;
    int half = 0;                     // the layouts hold a packed copy of the current factor
};

// Scalar CSR copy of both triangles of the RCS (the layout BSMC is compared
// with): block slots of each block row in ascending column order, the
// scalar row pointer, columns and values.
struct Csr {
    bool built = false, ready = false;
    int64_t n_slot = 0, nnz = 0;
    int32_t *bptr = nullptr;       // [n_rows+1] first slot of each block row
    int32_t *slot_src = nullptr;   // [n_slot] source block << 1 | transposed
    int32_t *slot_col = nullptr;   // [n_slot] block column
    int32_t *slot_row = nullptr;   // [n_slot] block row
    int32_t *rowptr = nullptr;     // [9 n_rows + 1]
    int32_t *col = nullptr;        // [nnz]
    double* val = nullptr;         // [nnz]
};

}  // namespace ba

struct ba_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int32_t n_cams = 0, n_pts = 0, n_rows = 0, precision = BA_FP64;
    int64_t n_obs = 0, n_blk = 0, n_pairs = 0;
    int32_t n_chunk = 0, n_offseg = 0;
    size_t bytes = 0, cap = 0;
    std::string err;
    // host copies
    std::vector<int64_t> h_row_ptr;
    std::vector<int32_t> h_col_idx;
    std::vector<int64_t> h_perm;       // internal observation -> caller index
    // device: observations in internal order (whole tracks, points by their
    // lowest camera, each track by camera)
    int32_t *obs_cam = nullptr, *obs_pt = nullptr, *obs_row = nullptr;
    double* obs_uv = nullptr;          // [2][n_obs]
    int32_t* chunk_q = nullptr;        // [n_chunk] internal index of each chunk's first point
    int32_t* chunk_ptr = nullptr;      // [n_chunk+1] point-aligned chunks of <= 64 observations
    // points with more than 64 observations (longer than a wave) come last
    // in the internal order, after every chunk: n_long of them, internal
    // indices q_long0 .. q_long0 + n_long - 1, their tracks long_ptr[j] ..
    // long_ptr[j + 1]; one workgroup works through each
    int32_t n_long = 0, q_long0 = 0;
    int32_t* long_ptr = nullptr;       // [n_long+1]
    int32_t* cam_row = nullptr;        // [n_cams] RCS row or -1
    // pattern
    int32_t *row_ptr = nullptr, *col_idx = nullptr;
    int32_t *off_blk = nullptr, *pair_ptr = nullptr, *trip = nullptr;
    int32_t *rowobs_ptr = nullptr, *rowobs = nullptr;
    // both triangles of the RCS by rows (upper blocks of the row, then the
    // transposed blocks of its column): pointer, column, source block << 1 |
    // transposed, and the FP64 copy made for PCG after each formation
    int32_t *sf_ptr = nullptr, *sf_col = nullptr, *sf_src = nullptr;
    int64_t n_sf = 0;
    double* Sf = nullptr;
    bool sf_ready = false;
    float* Sf32 = nullptr;             // FP32 copy of Sf for solver_fp32 (allocated on first use)
    bool sf32_ready = false;
    float* Su32 = nullptr;             // [n_blk][81] upper blocks in FP32, each transposed (UPPER product)
    bool su32_ready = false;
    // blocks (r, s), r < s, of each column s, ascending r (UPPER product)
    int32_t *lo_ptr = nullptr, *lo_blk = nullptr;
    int s32 = 0;                       // the current solve uses Sf32
    int upper = 0;                     // the current solve reads each upper block once (UPPER)
    int defl_s32 = 0;                  // precision of S in the deflation set-up (S W, E)
    // linearization / formation
    void* R = nullptr;                 // [n_obs][24] T: J_c (18) from linearize, K (6) from the point stage
    void* Jp = nullptr;                // [n_obs][6] T: J_p
    double* e = nullptr;               // [n_obs][2]
    int32_t* obs_rpos = nullptr;       // [n_obs] position in rowobs (-1: fixed camera)
    double* ebar = nullptr;            // [n_rowobs][2] e + K lhat in rowobs order (point stage -> diagonal)
    // pair-stage work units: couple ranges unit_rng[u] = [t0, t1) and
    // destinations (block index, or -(partial block + 1) for a chunk of a
    // split segment); split segment l sums partial blocks
    // [lseg_ptr[l], lseg_ptr[l+1]) into block lseg_blk[l].  Waves (4 units
    // each) [xcd_wv[x], xcd_wv[x+1]) run on XCD x.
    int32_t n_unit = 0, n_lseg = 0, n_pblk = 0;
    int32_t xcd_wv[9] = {0};
    int32_t *unit_rng = nullptr, *unit_dst = nullptr, *lseg_blk = nullptr, *lseg_ptr = nullptr;
    double* pblk = nullptr;            // [n_pblk][81]
    double* ptL = nullptr;             // [n_pts][9] by internal point index: Cholesky of V* (6), L^-1 l_p (3)
    double *blk = nullptr, *rhs = nullptr, *Minv = nullptr, *Mlearn = nullptr;
    double* Linv = nullptr;            // [n_rows][81] L_i^-1 (lower) of S_ii = L_i L_i^T
    double* lin_cams = nullptr;        // [n_cams][9] camera parameters of the last linearization
    bool defl_ready = false;
    std::vector<int32_t> h_blk_pairs;  // common points of every block (diagonal: 0)
    // LM
    double *dxc = nullptr, *dxp = nullptr, *part = nullptr, *scal = nullptr;
    double* part2 = nullptr;           // [3][kReduceParts] first-pass sums of launch_reduce
    int* flags = nullptr;
    int* tri_failed = nullptr;         // [1] points whose re-triangulation failed
    double* h_scal = nullptr;          // pinned
    int* h_flags = nullptr;            // pinned
    int32_t n_part = 0;
    ba::Pcg pcg;
    ba::Fsai fs;
    ba::Csr csr;
    hipEvent_t ev[16] = {};
    hipStream_t capture_stream = nullptr;
    bool use_graphs = true;
    struct PcgGraph {
        const double* M;
        int mode;
        int defl;
        int s32;
        int upper;
        int half;
        double tol;
        int max_iter;
        hipGraphExec_t exec;
    };
    std::vector<PcgGraph> pcg_graphs;
    // shared intrinsics: images (the n_cams "cameras" above) take the
    // interior parameters of physical camera img_cam[i]; RCS rows are the
    // n_free free images (exterior, 6 of 9 slots) then the n_phys cameras
    // (interior, 5 of 9 slots); parameters [n_cams][6] then [n_phys][5]
    bool shared = false;
    int32_t n_phys = 0, n_free = 0;
    std::vector<int32_t> h_img_cam;
    int32_t* img_cam = nullptr;
    double *lin_params = nullptr, *lin_pts = nullptr;   // parameters of the last linearization
    bool have_lin = false, have_rcs = false, learned_ready = false;
    // Jp holds J_p of the current linearization (k_linearize writes it; the
    // fused linearize + point stage does not, and J_p = K L^T is formed from
    // the records and the point terms where it is needed)
    bool jp_valid = false;
    ba_gnn* net = nullptr;             // learned preconditioner (not owned)
    void* lgraph = nullptr;            // its graph of this context's pattern (owned)
    double lambda = 0.0;
    double stage_ms[4] = {0, 0, 0, 0};
};

namespace ba {

// launchers (stream-ordered, no synchronisation)
void launch_project(const double* cams, const double* pts, const int32_t* obs_cam, const int32_t* obs_pt,
                    int64_t n_obs, const double* noise, double* uv, hipStream_t st);
void launch_linearize(ba_ctx* c, const double* cams, const double* pts);      // -> J, e, scal[0] = F
void launch_point(ba_ctx* c, double lambda);
// linearize + point stage in one pass (J, e, scal[0] = F, K, point terms)
void launch_linearize_point(ba_ctx* c, const double* cams, const double* pts, double lambda);
constexpr int kReduceParts = 1024;   // pieces of the first pass of launch_reduce
// out[j] = sum of part[j*n .. j*n + n) for j < count (<= 3), fixed order
void launch_reduce(ba_ctx* c, const double* part, int n, int count, double* out);
void launch_offdiag(ba_ctx* c);
void launch_diag(ba_ctx* c, double lambda);
void launch_back_substitute(ba_ctx* c, const double* dxc, double* dxp);
// J_p of the current linearization into Jp if the fused stage left it out
void ensure_jp(ba_ctx* c);
void launch_gather_obs(ba_ctx* c, const int32_t* perm, const int32_t* pt_in, const double* uv_in,
                       unsigned long long* bad);
// |J dx|^2 and dx^T l into scal[2], scal[3] for a dx_p replaced after
// back-substitution (which forms them for its own dx_p)
void launch_model_terms(ba_ctx* c, const double* dxc, const double* dxp);
void launch_evaluate(ba_ctx* c, const double* cams, const double* pts, const double* dxc, const double* dxp);
void launch_update(ba_ctx* c, double* cams, double* pts, const double* dxc, const double* dxp);
// PCG: returns status; fills iters/relres (synchronises).  mode 0: block
// diagonal M^-1 (Mblocks [n_rows][81]); mode 1: M^-1 = G^T G from c->fs.
// defl: deflate the similarity gauge (prepare_deflation first).
ba_status run_pcg(ba_ctx* c, int mode, const double* Mblocks, int defl, double tol, int max_iter,
                  const double* x0, double* out, int* iters, double* relres);
// gauge vectors of the last linearization's cameras, S W and (W^T S W)^-1
void prepare_deflation(ba_ctx* c);
// FSAI: index structure (host, once per context) and the factor of the
// current RCS (stream-ordered)
void build_fsai(ba_ctx* c);
void launch_fsai(ba_ctx* c);
// the UPPER apply's FP16 copy of the factor (Fsai::Gh): the Jacobi scaling
// Dn of the current RCS, and the copy made from Gu
void launch_dscale(ba_ctx* c);
void launch_pack_half(ba_ctx* c);
// CSR copy: index structure (host, once per context), values of the current
// RCS, and y = S x on it
void build_csr(ba_ctx* c);
void launch_csr_fill(ba_ctx* c);
void launch_csr_spmv(ba_ctx* c, const double* x, double* y);
// shared intrinsics (FP64): fused linearize + point stage over the
// parameters [n_cams][6] + [n_phys][5] (two records per observation), the
// diagonal stage (damping, padding, rhs, block-Jacobi factors; the blocks
// come from the pair stage), back-substitution, evaluation and update
void launch_linpoint_shared(ba_ctx* c, const double* params, const double* pts, double lambda);
void launch_node_diag(ba_ctx* c, double lambda);
void launch_back_substitute_shared(ba_ctx* c, const double* dxc, double* dxp);
void launch_evaluate_shared(ba_ctx* c, const double* params, const double* pts, const double* dxc, const double* dxp);
void launch_update_shared(ba_ctx* c, double* params, double* pts, const double* dxc, const double* dxp);
// re-triangulation of every point with cameras cams (+ dxc by RCS row when
// not null): start pts (+ out when delta), linear start if `linear`, n_gn
// Gauss-Newton steps; out = X, or X - pts when delta; failures counted
void launch_triangulate(ba_ctx* c, const double* cams, const double* dxc, const double* pts, double* out, int delta,
                        int linear, int n_gn, int* n_failed);

}  // namespace ba

#define BA_HIP_CHECK(call)                                                     \
    do {                                                                       \
        hipError_t _e = (call);                                                \
        if (_e != hipSuccess) throw ba_hip_error(_e, #call, __FILE__, __LINE__); \
    } while (0)

struct ba_hip_error {
    hipError_t code;
    std::string what;
    ba_hip_error(hipError_t c, const char* call, const char* file, int line)
        : code(c), what(std::string(call) + " failed: " + hipGetErrorString(c) + " at " + file + ":" + std::to_string(line)) {}
};
