// Preconditioned CG on the RCS (Sec. 3.2, Eq. (6)-(7)) with the symmetric
// block product of Sec. 6.2 on upper-triangle storage.
//
// Recurrence (Sec. 3.2): y0 = 0, r0 = b, z0 = M^-1 r0, d0 = z0; per step
//   alpha = r^T z / d^T S d;  y += alpha d;  r -= alpha S d;
//   stop when |r| / |r0| <= tol;  z = M^-1 r;  beta = r^T z / (r^T z)_old;
//   d = z + beta d.
// S d is formed as q_k = S z_k + beta q_{k-1} (the same vector, since
// d_k = z_k + beta d_{k-1}), so the block product only reads z.
//
// Two preconditioners:
//   block-diagonal M^-1 (block-Jacobi inverses, or the learned blocks):
//     A: s = S z (one wave per block row), q = s + beta q, d = z + beta d,
//        d^T q; also the stop test and the iteration cap.
//     B: alpha = rz / d^T q; y += alpha d; r -= alpha q; z = M^-1 r;
//        r^T z and r^T r; the iteration counter.
//   factorised M^-1 = G^T G (G block-lower-triangular, FP32 blocks):
//     A as above;
//     Bf: alpha; y += alpha d; r' = r - alpha q into the other r buffer;
//         t = G r' gathered over the row's lower blocks (r' of a neighbour
//         is formed from its r and q, which are complete); r'^T r'.
//     Cf: z = G^T t gathered over the row's upper blocks; r'^T z; counter.
//
// Optional deflation of the similarity gauge (Saad, Yeung, Erhel and
// Guyomarc'h's deflated CG): with W the seven gauge vectors of the cameras
// (camera parts of the null space of J, Eq. (1)), E = W^T S W,
//   x0 = x_s + W E^-1 W^T r_s, r0 = r_s - (S W) E^-1 W^T r_s,
//   p = z + beta p - W mu, q = S z + beta q - (S W) mu, mu = E^-1 (S W)^T z,
// so that W^T r stays zero; (S W)^T z rides along with r^T z.
//
// The product S z takes one of two layouts: FULL gathers every block row of
// both triangles (a copy made after each formation: each stored block is
// read twice); UPPER reads each stored upper block once (kernel A1 forms
// S_rs z_s for row r and writes S_rs^T z_r per block, kernel A2 sums those
// per row s in a fixed order and finishes A).
//
// All kernels run the same fixed number of blocks (grid-stride over rows)
// and leave one partial per block for each scalar product; every block of
// the next kernel re-sums those partials in the same order, so all blocks
// take the same decisions and the sums are deterministic.  The iteration
// number lives in device memory, so a batch of iterations is one fixed HIP
// graph.
#include <algorithm>

#include "ba_common.hpp"

namespace ba {

namespace {

constexpr int BS = 256;
constexpr int WPB = BS / kWave;    // 4 waves per block: one row each in the gathers
constexpr int GRPW = kWave / 9;    // 7 lane groups of 9 per wave
constexpr int RPB = BS / 9;        // 28 rows per block pass in kernels init and B
constexpr int kMaxGrid = 1024;   // the partial buffers hold this many blocks

// state: [0] done, [1] step index as published by kernel A (read by B, Bf,
//        Cf), [2] status, [3] completed steps as published by B or Cf
//        (read by the next A).  No kernel writes a word that its own blocks
//        read.
// scal:  [0] |r0|^2, [1] final relative residual
// partials: pA[g] (d^T q of block g), pR[p][g][0..8] (r^T z, r^T r and
//        (S W)^T z of the step with parity p)
constexpr int NP = 9;
constexpr int kW = 7;      // gauge vectors

// Fixed-order sum of NV interleaved partial streams of n blocks
// (src[i * stride + j]); every thread gets the totals.
template <int NV>
__device__ __forceinline__ void sum_partials(const double* __restrict__ src, int n, int stride, double* out,
                                             double* sh) {
    double s[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) s[j] = 0.0;
    for (int i = threadIdx.x; i < n; i += BS)
#pragma unroll
        for (int j = 0; j < NV; ++j) s[j] += src[(int64_t)i * stride + j];
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        const double v = wave_sum(s[j]);
        if (threadIdx.x % kWave == 0) sh[j * WPB + threadIdx.x / kWave] = v;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < WPB; ++w) t += sh[j * WPB + w];
        out[j] = t;
    }
    __syncthreads();
}

// Block totals of NV per-thread values (fixed shuffle tree, then fixed wave
// order); valid in thread 0.
template <int NV>
__device__ __forceinline__ void block_totals(const double* v, double* out, double* sh) {
#pragma unroll
    for (int j = 0; j < NV; ++j) {
        const double w = wave_sum(v[j]);
        if (threadIdx.x % kWave == 0) sh[j * WPB + threadIdx.x / kWave] = w;
    }
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int j = 0; j < NV; ++j) {
            double t = 0.0;
#pragma unroll
            for (int w = 0; w < WPB; ++w) t += sh[j * WPB + w];
            out[j] = t;
        }
    __syncthreads();
}

// Block total of per-wave values held in lane 0 of each wave (fixed order);
// valid in thread 0.
__device__ __forceinline__ double block_total(double wave_value, double* sh) {
    if (threadIdx.x % kWave == 0) sh[threadIdx.x / kWave] = wave_value;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
#pragma unroll
        for (int w = 0; w < WPB; ++w) t += sh[w];
    __syncthreads();
    return t;
}

// Nine consecutive values (one block row) with wide loads: rows start on
// 4-byte (FP32) or 8-byte (FP64) boundaries, which 16-byte global loads
// accept, so a row takes 3 (FP32) or 5 (FP64) loads instead of 9.
struct __attribute__((packed, aligned(4))) Row3f { float a, b, c; };
typedef double Row2d __attribute__((ext_vector_type(2), aligned(8)));
__device__ __forceinline__ void load_row9(const float* __restrict__ p, float* v) {
    const Row3f* r = reinterpret_cast<const Row3f*>(p);
    const Row3f x = r[0], y = r[1], z = r[2];
    v[0] = x.a; v[1] = x.b; v[2] = x.c; v[3] = y.a; v[4] = y.b; v[5] = y.c; v[6] = z.a; v[7] = z.b; v[8] = z.c;
}
__device__ __forceinline__ void load_row9(const double* __restrict__ p, double* v) {
    const Row2d* r = reinterpret_cast<const Row2d*>(p);
    const Row2d a = r[0], b = r[1], c = r[2], d = r[3];
    v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y; v[4] = c.x; v[5] = c.y; v[6] = d.x; v[7] = d.y; v[8] = p[8];
}

// Column c of a 9x9 block: stored row-major (TR false: nine loads one
// block row apart, the lanes of a group contiguous) or stored transposed (TR true: one
// row of the stored block, with wide loads).
template <bool TR, typename TS>
__device__ __forceinline__ void load_col9(const TS* __restrict__ b, int c, TS* v) {
    if (TR) {
        load_row9(b + c * 9, v);
    } else {
#pragma unroll
        for (int i = 0; i < 9; ++i) v[i] = b[i * 9 + c];
    }
}

// Half-precision factor blocks (see Fsai::Gh): rows 0..7 of column c of
// member e are the 16 bytes at word e * 36 + 4 c (two halves per word), row 8
// is Gh8[e * 9 + c]; all scaled back by hs[e].
constexpr int kHW = 36;
__device__ __forceinline__ float half_lo(uint32_t w) { return (float)__builtin_bit_cast(_Float16, (uint16_t)(w & 0xffffu)); }
__device__ __forceinline__ float half_hi(uint32_t w) { return (float)__builtin_bit_cast(_Float16, (uint16_t)(w >> 16)); }
__device__ __forceinline__ void load_colh(const uint32_t* __restrict__ Gh, const uint16_t* __restrict__ Gh8,
                                          const float* __restrict__ hs, int64_t e, int c, float* v) {
    const uint4 a = *reinterpret_cast<const uint4*>(Gh + e * kHW + c * 4);
    const uint16_t r8 = Gh8[e * 9 + c];
    const float s = hs[e];
    const uint32_t w[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        v[2 * k] = s * half_lo(w[k]);
        v[2 * k + 1] = s * half_hi(w[k]);
    }
    v[8] = s * (float)__builtin_bit_cast(_Float16, r8);
}

// Row gather by one wave over a block-CSR row (entries start..start+n-1,
// blocks stored row-major in the orientation they are applied in): y[c] =
// sum_e B_e v_e, returned in lanes 0..8 (component c = lane).  v_e is
// v0[col_e] (VM == 0) or v0[col_e] - alpha v1[col_e] (VM == 1), vector rows
// vs apart.  Lane group g (lanes 9g..9g+8) takes entries g, g + 7, ...;
// four entries per round: their block rows and columns are requested
// together; lane c of a group loads component c of each entry's vector row
// and the group shares the nine values through its LDS slot (one global
// load per entry instead of nine copies of the row).
template <typename TB, int VM>
__device__ __forceinline__ double row_gather(int start, int n, const int32_t* __restrict__ col,
                                             const TB* __restrict__ blk, const double* __restrict__ v0,
                                             const double* __restrict__ v1, double alpha, int vs = 9) {
    constexpr int U = 4;
    __shared__ double sx[WPB][GRPW * U][9];
    const int lane = threadIdx.x % kWave;
    const int grp = lane / 9, comp = lane % 9;
    double (*xs)[9] = sx[threadIdx.x / kWave] + grp * U;
    double acc = 0.0;
    if (grp < GRPW) {
        for (int e0 = grp; e0 < n; e0 += GRPW * U) {
            int ci[U];
            TB bv[U][9];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = e0 + u * GRPW;
                const int ee = start + (e < n ? e : e0);
                ci[u] = col[ee];
                load_row9(blk + (int64_t)ee * 81 + comp * 9, bv[u]);
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                double x = v0[(int64_t)ci[u] * vs + comp];
                if (VM == 1) x -= alpha * v1[(int64_t)ci[u] * vs + comp];
                xs[u][comp] = x;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (e0 + u * GRPW >= n) break;
#pragma unroll
                for (int c = 0; c < 9; ++c) acc += (double)bv[u][c] * xs[u][c];
            }
        }
    }
    // lanes 0..8: sum over the 7 groups in group order
    double tot = acc;
#pragma unroll
    for (int g = 1; g < GRPW; ++g) {
        const double o = __shfl(acc, lane + 9 * g < kWave ? lane + 9 * g : lane, kWave);
        tot += o;
    }
    return tot;
}

// S W for the kW gauge vectors of one block row (W rows kW * 9 apart): the
// row's blocks are read once for all of them; results in lanes 0..8 of
// out[v].  Same entry order and group sums as row_gather.
template <typename TB>
__device__ __forceinline__ void row_gather_w(int start, int n, const int32_t* __restrict__ col,
                                             const TB* __restrict__ blk, const double* __restrict__ W, double* out) {
    constexpr int U = 4;
    __shared__ double sxw[WPB][GRPW * U][9];
    const int lane = threadIdx.x % kWave;
    const int grp = lane / 9, comp = lane % 9;
    double (*xs)[9] = sxw[threadIdx.x / kWave] + grp * U;
    double acc[kW];
#pragma unroll
    for (int v = 0; v < kW; ++v) acc[v] = 0.0;
    if (grp < GRPW) {
        for (int e0 = grp; e0 < n; e0 += GRPW * U) {
            int ci[U];
            TB bv[U][9];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = e0 + u * GRPW;
                const int ee = start + (e < n ? e : e0);
                ci[u] = col[ee];
                load_row9(blk + (int64_t)ee * 81 + comp * 9, bv[u]);
            }
#pragma unroll
            for (int v = 0; v < kW; ++v) {
#pragma unroll
                for (int u = 0; u < U; ++u) xs[u][comp] = W[(int64_t)ci[u] * kW * 9 + v * 9 + comp];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    if (e0 + u * GRPW >= n) break;
#pragma unroll
                    for (int c = 0; c < 9; ++c) acc[v] += (double)bv[u][c] * xs[u][c];
                }
            }
        }
    }
#pragma unroll
    for (int v = 0; v < kW; ++v) {
        double tot = acc[v];
#pragma unroll
        for (int g = 1; g < GRPW; ++g) tot += __shfl(acc[v], lane + 9 * g < kWave ? lane + 9 * g : lane, kWave);
        out[v] = tot;
    }
}

// Sf: both triangles of the RCS by rows (FP64, or rounded to FP32), from the
// upper blocks
template <typename TS>
__global__ __launch_bounds__(BS) void k_build_sf(int64_t n_sf, const int32_t* __restrict__ sf_src,
                                                 const double* __restrict__ blk, TS* __restrict__ Sf) {
    const int64_t n = n_sf * 81;
    for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS) {
        const int64_t e = i / 81;
        const int pq = (int)(i % 81), p = pq / 9, q = pq % 9;
        const int src = sf_src[e];
        const double* B = blk + (int64_t)(src >> 1) * 81;
        Sf[i] = (TS)((src & 1) ? B[q * 9 + p] : B[pq]);
    }
}

// Su32: the upper blocks rounded to FP32, each stored transposed (so that a
// column of S_rs is a contiguous row for the UPPER product)
__global__ __launch_bounds__(BS) void k_build_su32(int64_t n_blk, const double* __restrict__ blk,
                                                   float* __restrict__ Su) {
    const int64_t n = n_blk * 81;
    for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < n; i += (int64_t)gridDim.x * BS) {
        const int64_t e = i / 81;
        const int pq = (int)(i % 81), p = pq / 9, q = pq % 9;
        Su[i] = (float)blk[e * 81 + q * 9 + p];
    }
}

// ---------------------------------------------------------------------------
// gauge deflation set-up
// ---------------------------------------------------------------------------

// W [n_rows][7][9]: rotation generators (dw = -J_r(w)^-1 e_k), translation
// generators (dt = -R e_k), scale (dt = t) of every free camera, from the
// parameters of the last linearization.  J_r^-1 = I + K/2 + c K^2,
// K = [w]x, c = 1/th^2 - (1 + cos th) / (2 th sin th), with its series
// near th = 0 and its limit near th = pi.
__global__ void k_gauge_W(int n_cams, const int32_t* __restrict__ cam_row, const double* __restrict__ cams,
                          double* __restrict__ W) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_cams) return;
    const int row = cam_row[c];
    if (row < 0) return;
    const double* p = cams + (int64_t)c * 9;
    const double w0 = p[0], w1 = p[1], w2 = p[2];
    const double th2 = w0 * w0 + w1 * w1 + w2 * w2, th = sqrt(th2);
    double a, b, cc;   // R = I + a K + b K^2; J_r^-1 = I + K/2 + cc K^2
    if (th < 1e-4) {
        a = 1.0 - th2 / 6.0;
        b = 0.5 - th2 / 24.0;
        cc = 1.0 / 12.0 + th2 / 720.0;
    } else {
        const double s = sin(th), co = cos(th);
        a = s / th;
        b = (1.0 - co) / th2;
        const double dl = 3.14159265358979323846 - th;
        cc = (fabs(dl) < 1e-4) ? 1.0 / th2 - dl / (4.0 * th) : 1.0 / th2 - (1.0 + co) / (2.0 * th * s);
    }
    const double K[9] = {0.0, -w2, w1, w2, 0.0, -w0, -w1, w0, 0.0};
    double K2[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double t = 0.0;
            for (int k = 0; k < 3; ++k) t += K[i * 3 + k] * K[k * 3 + j];
            K2[i * 3 + j] = t;
        }
    double* Wr = W + (int64_t)row * kW * 9;
    for (int i = 0; i < kW * 9; ++i) Wr[i] = 0.0;
    for (int k = 0; k < 3; ++k)
        for (int i = 0; i < 3; ++i) {
            const double id = i == k ? 1.0 : 0.0;
            Wr[k * 9 + i] = -(id + 0.5 * K[i * 3 + k] + cc * K2[i * 3 + k]);   // -J_r^-1 e_k
            Wr[(3 + k) * 9 + 3 + i] = -(id + a * K[i * 3 + k] + b * K2[i * 3 + k]);   // -R e_k
        }
    for (int i = 0; i < 3; ++i) Wr[6 * 9 + 3 + i] = p[3 + i];
}

// SW = S W, one wave per block row, the seven columns in turn
template <typename TS>
__global__ __launch_bounds__(BS) void k_spmm_W(int n_rows, const int32_t* __restrict__ sf_ptr,
                                               const int32_t* __restrict__ sf_col, const TS* __restrict__ Sf,
                                               const double* __restrict__ W, double* __restrict__ SW) {
    const int lane = threadIdx.x % kWave;
    for (int row = blockIdx.x * WPB + threadIdx.x / kWave; row < n_rows; row += gridDim.x * WPB) {
        const int a = sf_ptr[row];
        double y[kW];
        row_gather_w<TS>(a, sf_ptr[row + 1] - a, sf_col, Sf, W, y);
        if (lane < 9)
#pragma unroll
            for (int v = 0; v < kW; ++v) SW[(int64_t)row * kW * 9 + v * 9 + lane] = y[v];
    }
}

// partials of E = W^T S W (49 per block)
__global__ __launch_bounds__(BS) void k_defl_E_part(int n_rows, const double* __restrict__ W,
                                                    const double* __restrict__ SW, double* __restrict__ pE) {
    __shared__ double sh[kW * kW * WPB];
    double e[kW * kW];
#pragma unroll
    for (int j = 0; j < kW * kW; ++j) e[j] = 0.0;
    const int64_t n = (int64_t)n_rows * 9;
    for (int64_t idx = (int64_t)blockIdx.x * BS + threadIdx.x; idx < n; idx += (int64_t)gridDim.x * BS) {
        const int64_t row = idx / 9, c = idx % 9;
        double wv[kW], sv[kW];
#pragma unroll
        for (int v = 0; v < kW; ++v) {
            wv[v] = W[row * kW * 9 + v * 9 + c];
            sv[v] = SW[row * kW * 9 + v * 9 + c];
        }
#pragma unroll
        for (int u = 0; u < kW; ++u)
#pragma unroll
            for (int v = 0; v < kW; ++v) e[u * kW + v] += wv[u] * sv[v];
    }
    double t[kW * kW];
    block_totals<kW * kW>(e, t, sh);
    if (threadIdx.x == 0)
        for (int j = 0; j < kW * kW; ++j) pE[(int64_t)blockIdx.x * kW * kW + j] = t[j];
}

// E[j] = sum of the partials of entry j over the blocks (one block per
// entry, fixed order)
__global__ __launch_bounds__(BS) void k_defl_E_sum(int n_part, const double* __restrict__ pE,
                                                   double* __restrict__ E) {
    __shared__ double sh[WPB];
    const int j = blockIdx.x;
    double t = 0.0;
    for (int b = threadIdx.x; b < n_part; b += BS) t += pE[(int64_t)b * kW * kW + j];
    t = block_sum<BS>(t, sh);
    if (threadIdx.x == 0) E[j] = t;
}

// E symmetrised, then E^-1 by Cholesky (one thread).  A non-positive pivot
// leaves E^-1 = 0: no deflation.
__global__ void k_defl_E_fin(const double* __restrict__ Esum, double* __restrict__ Einv, int* __restrict__ flags) {
    __shared__ double E[kW * kW];
    const int j = threadIdx.x;
    if (j < kW * kW) E[j] = Esum[j];
    __syncthreads();
    if (threadIdx.x != 0) return;
    double L[kW * kW], X[kW * kW];
    bool ok = true;
    for (int a = 0; a < kW; ++a)
        for (int b = 0; b <= a; ++b) {
            double s = 0.5 * (E[a * kW + b] + E[b * kW + a]);
            for (int k = 0; k < b; ++k) s -= L[a * kW + k] * L[b * kW + k];
            if (a == b) {
                if (!(s > 0.0)) { ok = false; s = 1.0; }
                L[a * kW + a] = sqrt(s);
            } else {
                L[a * kW + b] = s / L[b * kW + b];
            }
        }
    // E^-1 = L^-T L^-1, column by column
    for (int col = 0; col < kW; ++col) {
        double y[kW];
        for (int a = 0; a < kW; ++a) {
            double s = a == col ? 1.0 : 0.0;
            for (int k = 0; k < a; ++k) s -= L[a * kW + k] * y[k];
            y[a] = s / L[a * kW + a];
        }
        for (int a = kW - 1; a >= 0; --a) {
            double s = y[a];
            for (int k = a + 1; k < kW; ++k) s -= L[k * kW + a] * X[k * kW + col];
            X[a * kW + col] = s / L[a * kW + a];
        }
    }
    for (int i = 0; i < kW * kW; ++i) Einv[i] = ok ? X[i] : 0.0;
    if (!ok) flags[3] = 1;
}

// partials of W^T r_s, r_s = rhs - q0 (7 per block)
__global__ __launch_bounds__(BS) void k_defl_Wr(int n_rows, const double* __restrict__ rhs,
                                                const double* __restrict__ q0, const double* __restrict__ W,
                                                double* __restrict__ pW) {
    __shared__ double sh[kW * WPB];
    double a[kW];
#pragma unroll
    for (int v = 0; v < kW; ++v) a[v] = 0.0;
    const int64_t n = (int64_t)n_rows * 9;
    for (int64_t idx = (int64_t)blockIdx.x * BS + threadIdx.x; idx < n; idx += (int64_t)gridDim.x * BS) {
        const int64_t row = idx / 9, c = idx % 9;
        const double rs = rhs[idx] - (q0 ? q0[idx] : 0.0);
#pragma unroll
        for (int v = 0; v < kW; ++v) a[v] += W[row * kW * 9 + v * 9 + c] * rs;
    }
    double t[kW];
    block_totals<kW>(a, t, sh);
    if (threadIdx.x == 0)
        for (int v = 0; v < kW; ++v) pW[(int64_t)blockIdx.x * kW + v] = t[v];
}

// mu = E^-1 a (7x7), every thread
__device__ __forceinline__ void einv_apply(const double* __restrict__ Einv, const double* a, double* mu) {
#pragma unroll
    for (int u = 0; u < kW; ++u) {
        double t = 0.0;
#pragma unroll
        for (int v = 0; v < kW; ++v) t += Einv[u * kW + v] * a[v];
        mu[u] = t;
    }
}

// D = diag(S_jj)^-1/2 of every row (the Jacobi scaling of the half copy)
__global__ __launch_bounds__(BS) void k_dscale(int n_rows, const int32_t* __restrict__ row_ptr,
                                               const double* __restrict__ blk, double* __restrict__ Dn) {
    const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
    if (i >= (int64_t)n_rows * 9) return;
    const int j = (int)(i / 9), b = (int)(i % 9);
    Dn[i] = 1.0 / sqrt(blk[(int64_t)row_ptr[j] * 81 + b * 10]);
}

// Half-precision copy of the transposed factor blocks GuT (member e: column
// block J[e]): row b of the transposed block (column b of G_e) divided by
// Dn[J[e]][b], the block by its largest magnitude; three members per
// workgroup
__global__ __launch_bounds__(BS) void k_pack_half(int64_t n_mem, const int32_t* __restrict__ J,
                                                  const float* __restrict__ GuT, const double* __restrict__ Dn,
                                                  uint32_t* __restrict__ Gh, uint16_t* __restrict__ Gh8,
                                                  float* __restrict__ hs) {
    __shared__ float sv[3][81];
    __shared__ float smax[3];
    const int t = threadIdx.x, m = t / 81, v = t % 81;
    const int64_t e = (int64_t)blockIdx.x * 3 + m;
    const bool act = t < 243 && e < n_mem;
    if (act) sv[m][v] = (float)((double)GuT[e * 81 + v] / Dn[(int64_t)J[e] * 9 + v / 9]);
    __syncthreads();
    if (act && v == 0) {
        float mx = 0.f;
        for (int k = 0; k < 81; ++k) mx = fmaxf(mx, fabsf(sv[m][k]));
        smax[m] = mx > 0.f && mx <= 3.0e38f ? mx : 1.f;
    }
    __syncthreads();
    if (act) {
        const float s = smax[m];
        const int b = v / 9, a = v % 9;
        if (a < 8 && a % 2 == 0) {
            const _Float16 lo = (_Float16)(sv[m][v] / s);
            const _Float16 hi = (_Float16)(sv[m][v + 1] / s);
            Gh[e * kHW + b * 4 + a / 2] = (uint32_t)__builtin_bit_cast(uint16_t, lo) |
                                          ((uint32_t)__builtin_bit_cast(uint16_t, hi) << 16);
        }
        if (a == 8) Gh8[e * 9 + b] = __builtin_bit_cast(uint16_t, (_Float16)(sv[m][v] / s));
        if (v == 0) hs[e] = s;
    }
}

// ---------------------------------------------------------------------------
// PCG kernels
// ---------------------------------------------------------------------------

// x = x_s (x0 or 0), r = rhs - q0 (q0 = S x0, or 0); deflated: x += W y,
// r -= SW y with y = E^-1 W^T r_s.  With a block-diagonal preconditioner
// also z = M^-1 r; partials of r^T z, r^T r, (SW)^T z (parity 0); the state.
__global__ __launch_bounds__(BS) void k_pcg_init(int n_rows, const double* __restrict__ rhs,
                                                 const double* __restrict__ q0, const double* __restrict__ x0,
                                                 const double* __restrict__ M, double* __restrict__ x,
                                                 double* __restrict__ r, double* __restrict__ z,
                                                 double* __restrict__ pR, int* __restrict__ state,
                                                 double* __restrict__ scal, int defl, const double* __restrict__ W,
                                                 const double* __restrict__ SW, const double* __restrict__ Einv,
                                                 const double* __restrict__ pW, int n_part) {
    __shared__ double sr[RPB][9];
    __shared__ double sh[NP * WPB];
    double y[kW];
#pragma unroll
    for (int v = 0; v < kW; ++v) y[v] = 0.0;
    if (defl) {
        double a[kW];
        sum_partials<kW>(pW, n_part, kW, a, sh);
        einv_apply(Einv, a, y);
    }
    const int lr = threadIdx.x / 9, i = threadIdx.x % 9;
    double acc[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) acc[j] = 0.0;
    for (int base = blockIdx.x * RPB; base < n_rows; base += gridDim.x * RPB) {
        const int row = base + lr;
        const bool act = threadIdx.x < RPB * 9 && row < n_rows;
        const int64_t o = (int64_t)row * 9 + i;
        double rv = 0.0;
        if (act) {
            double xv = x0 ? x0[o] : 0.0;
            rv = rhs[o] - (q0 ? q0[o] : 0.0);
            if (defl) {
                const double* Wr = W + (int64_t)row * kW * 9 + i;
                const double* Sr = SW + (int64_t)row * kW * 9 + i;
#pragma unroll
                for (int v = 0; v < kW; ++v) {
                    xv += Wr[v * 9] * y[v];
                    rv -= Sr[v * 9] * y[v];
                }
            }
            x[o] = xv;
            r[o] = rv;
            sr[lr][i] = rv;
        }
        __syncthreads();
        if (act && M) {
            const double* Mr = M + (int64_t)row * 81 + i * 9;
            double zv = 0.0;
#pragma unroll
            for (int c = 0; c < 9; ++c) zv += Mr[c] * sr[lr][c];
            z[o] = zv;
            acc[0] += rv * zv;
            if (defl) {
                const double* Sr = SW + (int64_t)row * kW * 9 + i;
#pragma unroll
                for (int v = 0; v < kW; ++v) acc[2 + v] += Sr[v * 9] * zv;
            }
        }
        acc[1] += rv * rv;
        __syncthreads();
    }
    double t[NP];
    block_totals<NP>(acc, t, sh);
    if (threadIdx.x == 0)
        for (int j = 0; j < NP; ++j) pR[(int64_t)NP * blockIdx.x + j] = t[j];
    if (blockIdx.x == 0 && threadIdx.x == 0) { state[0] = 0; state[1] = 0; state[2] = BA_OK; state[3] = 0; scal[1] = -1.0; }
}

// plain y = S x
template <typename TS>
__global__ __launch_bounds__(BS) void k_spmv(int n_rows, const int32_t* __restrict__ sf_ptr,
                                             const int32_t* __restrict__ sf_col, const TS* __restrict__ Sf,
                                             const double* __restrict__ x, double* __restrict__ y) {
    const int lane = threadIdx.x % kWave;
    for (int row = blockIdx.x * WPB + threadIdx.x / kWave; row < n_rows; row += gridDim.x * WPB) {
        const int a = sf_ptr[row];
        const double v = row_gather<TS, 0>(a, sf_ptr[row + 1] - a, sf_col, Sf, x, nullptr, 0.0);
        if (lane < 9) y[(int64_t)row * 9 + lane] = v;
    }
}

// One-read apply of a factor and its transpose over one block row (FP32
// blocks B_e with columns col_e, each stored transposed so that a column is
// one wide load): lane c of a group of nine holds column c of its blocks, so
//   t_row[i] = sum_e sum_c B_e[i][c] v_e[c]   accumulates in the lane (its
//              own component of each v_e) and is summed over the wave once;
//   (B_e^T t_row)[c] = sum_i B_e[i][c] t_row[i]   needs only that lane: written
//              to tg per entry.
// v_e = v0[col_e] (VM 0) or v0[col_e] - alpha v1[col_e] (VM 1).  Rows of up
// to 28 entries keep their blocks in registers between the two products;
// longer rows load them again.  Returns t_row in lanes 0..8.
// H: blocks from the half-precision copy (Gh, hs) in the Jacobi-scaled
// space, v_e scaled by Dn[col_e] (the products written to tg then lack the
// factor Dn of their column, which the column sums apply).
template <int VM, bool H = false>
__device__ __forceinline__ double row_factor_t(int start, int n, const int32_t* __restrict__ col,
                                               const float* __restrict__ blkT, const double* __restrict__ v0,
                                               const double* __restrict__ v1, double alpha,
                                               double* __restrict__ tg, const uint32_t* __restrict__ Gh = nullptr,
                                               const uint16_t* __restrict__ Gh8 = nullptr,
                                               const float* __restrict__ hs = nullptr,
                                               const double* __restrict__ Dn = nullptr) {
    constexpr int U = 4;
    const int lane = threadIdx.x % kWave;
    const int grp = lane / 9, comp = lane % 9;
    double acc[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) acc[i] = 0.0;
    float bv[U][9];
    const bool one_round = n <= GRPW * U;   // wave-uniform
    if (grp < GRPW) {
        for (int e0 = grp; e0 < n; e0 += GRPW * U) {
            double x[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = e0 + u * GRPW;
                const int ee = start + (e < n ? e : e0);
                const int cj = col[ee];
                if (H) load_colh(Gh, Gh8, hs, ee, comp, bv[u]);
                else load_col9<true>(blkT + (int64_t)ee * 81, comp, bv[u]);
                x[u] = v0[(int64_t)cj * 9 + comp];
                if (VM == 1) x[u] -= alpha * v1[(int64_t)cj * 9 + comp];
                if (H) x[u] *= Dn[(int64_t)cj * 9 + comp];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (e0 + u * GRPW >= n) break;
#pragma unroll
                for (int i = 0; i < 9; ++i) acc[i] += (double)bv[u][i] * x[u];
            }
        }
    }
    double t[9], out = 0.0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        t[i] = wave_sum(acc[i]);
        if (lane == i) out = t[i];
    }
    if (grp < GRPW) {
        for (int e0 = grp; e0 < n; e0 += GRPW * U) {
            if (!one_round) {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int e = e0 + u * GRPW;
                    const int64_t ee = start + (e < n ? e : e0);
                    if (H) load_colh(Gh, Gh8, hs, ee, comp, bv[u]);
                    else load_col9<true>(blkT + ee * 81, comp, bv[u]);
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = e0 + u * GRPW;
                if (e >= n) break;
                double y = 0.0;
#pragma unroll
                for (int i = 0; i < 9; ++i) y += (double)bv[u][i] * t[i];
                tg[(int64_t)(start + e) * 9 + comp] = y;
            }
        }
    }
    return out;
}

// init + sum of v[src[a0 + e]][c] for e = 0..n-1 in ascending e (one lane
// per component; each round requests up to 16 indices, then their values)
__device__ __forceinline__ double index_sum(int a0, int n, const int32_t* __restrict__ src,
                                            const double* __restrict__ v, int c, double init) {
    constexpr int U = 16;
    double acc = init;
    for (int e0 = 0; e0 < n; e0 += U) {
        int bi[U];
#pragma unroll
        for (int k = 0; k < U; ++k) bi[k] = e0 + k < n ? src[a0 + e0 + k] : -1;
        double w[U];
#pragma unroll
        for (int k = 0; k < U; ++k) w[k] = bi[k] >= 0 ? v[(int64_t)bi[k] * 9 + c] : 0.0;
#pragma unroll
        for (int k = 0; k < U; ++k) acc += w[k];
    }
    return acc;
}

// t = G r (initial step of the factorised preconditioner); UP: from the
// transposed blocks GlT, with the transposed products G_row,j^T t_row per
// entry (tg)
template <bool UP, bool H = false>
__global__ __launch_bounds__(BS) void k_gather_lower(int n_rows, const int32_t* __restrict__ gl_ptr,
                                                     const int32_t* __restrict__ gl_col, const float* __restrict__ Gl,
                                                     const float* __restrict__ GlT, const double* __restrict__ r,
                                                     double* __restrict__ t, double* __restrict__ tg,
                                                     const uint32_t* __restrict__ Gh, const uint16_t* __restrict__ Gh8,
                                                     const float* __restrict__ hs,
                                                     const double* __restrict__ Dn) {
    const int lane = threadIdx.x % kWave;
    for (int row = blockIdx.x * WPB + threadIdx.x / kWave; row < n_rows; row += gridDim.x * WPB) {
        const int a = gl_ptr[row], n = gl_ptr[row + 1] - a;
        const double v = UP ? row_factor_t<0, H>(a, n, gl_col, GlT, r, nullptr, 0.0, tg, Gh, Gh8, hs, Dn)
                            : row_gather<float, 0>(a, n, gl_col, Gl, r, nullptr, 0.0);
        if (lane < 9) t[(int64_t)row * 9 + lane] = v;
    }
}

// Decisions of kernel A from the partials of the previous step: false if
// the solve is over (stop test or iteration cap, recorded by block 0),
// else beta and, when deflating, mu = E^-1 (S W)^T z.
template <bool FIRST>
__device__ __forceinline__ bool a_step(const double* __restrict__ pR, int n_part, int* __restrict__ state,
                                       double* __restrict__ scal, double tol, int max_iter, int defl,
                                       const double* __restrict__ Einv, double* sh, double& beta, double* mu) {
    const int done = state[0];
    const int k = state[3];
    // rz_k, rr_k, (SW)^T z_k (parity k) and rz_{k-1} (other parity)
    double s[NP + 1];
#pragma unroll
    for (int j = 0; j < NP + 1; ++j) s[j] = 0.0;
    const double* pk = pR + (int64_t)NP * n_part * (k & 1);
    if (defl)
        sum_partials<NP>(pk, n_part, NP, s, sh);
    else
        sum_partials<2>(pk, n_part, NP, s, sh);
    if (!FIRST) sum_partials<1>(pR + (int64_t)NP * n_part * ((k + 1) & 1), n_part, NP, s + NP, sh);
    if (done) return false;
    const double rz = s[0], rr = s[1], rz_old = FIRST ? 1.0 : s[NP];
    const double r0sq = FIRST ? rr : scal[0];
    if (FIRST && blockIdx.x == 0 && threadIdx.x == 0) scal[0] = rr;
    const bool conv = (rr == 0.0) || (sqrt(rr) <= tol * sqrt(r0sq));
    if (conv || k >= max_iter) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            state[0] = 1;
            state[2] = conv ? BA_OK : BA_ERR_NOT_CONVERGED;
            scal[1] = r0sq > 0.0 ? sqrt(rr / r0sq) : 0.0;
        }
        return false;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) state[1] = k;
    beta = FIRST ? 0.0 : rz / rz_old;
#pragma unroll
    for (int v = 0; v < kW; ++v) mu[v] = 0.0;
    if (defl) einv_apply(Einv, s + 2, mu);
    return true;
}

// The end of kernel A for component c of block row `row`, given
// sv = (S z)_row[c]: q = sv + beta q - (S W) mu, d = z + beta d - W mu;
// returns the component's share of d^T q.
template <bool FIRST>
__device__ __forceinline__ double a_finish(int row, int c, double sv, const double* __restrict__ z,
                                           double* __restrict__ d, double* __restrict__ q, double beta, int defl,
                                           const double* __restrict__ W, const double* __restrict__ SW,
                                           const double* mu) {
    const int64_t o = (int64_t)row * 9 + c;
    double wm = 0.0, swm = 0.0;
    if (defl) {
        const double* Wr = W + (int64_t)row * kW * 9 + c;
        const double* Sr = SW + (int64_t)row * kW * 9 + c;
#pragma unroll
        for (int v = 0; v < kW; ++v) {
            wm += Wr[v * 9] * mu[v];
            swm += Sr[v * 9] * mu[v];
        }
    }
    const double zv = z[o];
    const double qv = (FIRST ? sv : sv + beta * q[o]) - swm;
    const double dv = (FIRST ? zv : zv + beta * d[o]) - wm;
    q[o] = qv;
    d[o] = dv;
    return dv * qv;
}

// kernel A (FULL product); FIRST: the iteration k = 0 (records |r0|^2).
template <bool FIRST, typename TS>
__global__ __launch_bounds__(BS) void k_pcg_A(int n_rows, const int32_t* __restrict__ sf_ptr,
                                              const int32_t* __restrict__ sf_col, const TS* __restrict__ Sf,
                                              const double* __restrict__ z,
                                              double* __restrict__ d, double* __restrict__ q,
                                              double* __restrict__ pA, const double* __restrict__ pR, int n_part,
                                              int* __restrict__ state, double* __restrict__ scal, double tol,
                                              int max_iter, int defl, const double* __restrict__ W,
                                              const double* __restrict__ SW, const double* __restrict__ Einv) {
    __shared__ double sh[NP * WPB];
    double beta, mu[kW];
    if (!a_step<FIRST>(pR, n_part, state, scal, tol, max_iter, defl, Einv, sh, beta, mu)) return;
    const int lane = threadIdx.x % kWave;
    double dq = 0.0;
    for (int row = blockIdx.x * WPB + threadIdx.x / kWave; row < n_rows; row += gridDim.x * WPB) {
        const int a0 = sf_ptr[row];
        const double sv = row_gather<TS, 0>(a0, sf_ptr[row + 1] - a0, sf_col, Sf, z, nullptr, 0.0);
        if (lane < 9) dq += a_finish<FIRST>(row, lane, sv, z, d, q, beta, defl, W, SW, mu);
    }
    const double t = block_total(wave_sum(dq), sh);
    if (threadIdx.x == 0) pA[blockIdx.x] = t;
}


// UPPER product, first kernel: the wave of block row r walks the row's
// stored blocks B_e = S_{r,s_e} (the diagonal block first, then s_e > r);
// lane c of a group of nine holds column c of its block, so
//   (B_e^T z_r)_c = sum_i B_e[i][c] z_r[i]      needs only that lane: written
//                                               to tb[e] for s_e != r;
//   (S z)_r[i] += B_e[i][c] z_{s_e}[c]           is summed over the lanes once
//                                               per row (wave sums, fixed).
// Every stored block is read once.  Returns (S z)_r restricted to the upper
// blocks in lanes 0..8.
template <bool TR, typename TS>
__device__ __forceinline__ double row_upper(int row, int start, int n, const int32_t* __restrict__ col,
                                            const TS* __restrict__ blk, const double* __restrict__ z,
                                            double* __restrict__ tb) {
    constexpr int U = sizeof(TS) == 8 ? 1 : 4;   // blocks in flight per group (72 or 144 bytes per lane)
    const int lane = threadIdx.x % kWave;
    const int grp = lane / 9, comp = lane % 9;
    double zr[9], acc[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) { zr[i] = z[(int64_t)row * 9 + i]; acc[i] = 0.0; }
    if (grp < GRPW) {
        for (int e0 = grp; e0 < n; e0 += GRPW * U) {
            int ci[U];
            TS bv[U][9];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = e0 + u * GRPW;
                const int ee = start + (e < n ? e : e0);
                ci[u] = col[ee];
                load_col9<TR>(blk + (int64_t)ee * 81, comp, bv[u]);
            }
            double zs[U];
#pragma unroll
            for (int u = 0; u < U; ++u) zs[u] = z[(int64_t)ci[u] * 9 + comp];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int e = e0 + u * GRPW;
                if (e >= n) break;
                double t = 0.0;
#pragma unroll
                for (int i = 0; i < 9; ++i) {
                    const double b = (double)bv[u][i];
                    acc[i] += b * zs[u];
                    t += b * zr[i];
                }
                if (e > 0) tb[(int64_t)(start + e) * 9 + comp] = t;
            }
        }
    }
    double out = 0.0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const double v = wave_sum(acc[i]);
        if (lane == i) out = v;
    }
    return out;
}

template <bool FIRST, bool TR, typename TS>
__global__ __launch_bounds__(BS) void k_pcg_A1(int n_rows, const int32_t* __restrict__ row_ptr,
                                               const int32_t* __restrict__ col_idx, const TS* __restrict__ blk,
                                               const double* __restrict__ z, double* __restrict__ u,
                                               double* __restrict__ tb, const double* __restrict__ pR, int n_part,
                                               int* __restrict__ state, double* __restrict__ scal, double tol,
                                               int max_iter, int defl, const double* __restrict__ Einv,
                                               double* __restrict__ bm) {
    __shared__ double sh[NP * WPB];
    double beta, mu[kW];
    if (!a_step<FIRST>(pR, n_part, state, scal, tol, max_iter, defl, Einv, sh, beta, mu)) return;
    // the step's beta and mu for the second kernel (every block has the same)
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        bm[0] = beta;
#pragma unroll
        for (int v = 0; v < kW; ++v) bm[1 + v] = mu[v];
    }
    const int lane = threadIdx.x % kWave;
    for (int row = blockIdx.x * WPB + threadIdx.x / kWave; row < n_rows; row += gridDim.x * WPB) {
        const int a0 = row_ptr[row];
        const double v = row_upper<TR, TS>(row, a0, row_ptr[row + 1] - a0, col_idx, blk, z, tb);
        if (lane < 9) u[(int64_t)row * 9 + lane] = v;
    }
}

// (S z)_s[c] from the UPPER product's two parts: u_s plus the transposed
// products tb of the blocks (r, s), r < s, of column s, summed in ascending
// r by the lane group that owns row s (lane c of the group: component c).
// A wave owns seven rows at a time, so their dependent index and value
// loads overlap.
__device__ __forceinline__ double column_sum(int row, int c, const int32_t* __restrict__ lo_ptr,
                                             const int32_t* __restrict__ lo_blk, const double* __restrict__ u,
                                             const double* __restrict__ tb) {
    const int a0 = lo_ptr[row];
    return index_sum(a0, lo_ptr[row + 1] - a0, lo_blk, tb, c, u[(int64_t)row * 9 + c]);
}

// UPPER product, second kernel: (S z)_s (column_sum), then the end of
// kernel A with the beta and mu that the first kernel published; lane group
// g of wave w takes rows (block * WPB + w) * 7 + g, ...
template <bool FIRST>
__global__ __launch_bounds__(BS) void k_pcg_A2(int n_rows, const int32_t* __restrict__ lo_ptr,
                                               const int32_t* __restrict__ lo_blk, const double* __restrict__ u,
                                               const double* __restrict__ tb, const double* __restrict__ z,
                                               double* __restrict__ d, double* __restrict__ q,
                                               double* __restrict__ pA, const int* __restrict__ state, int defl,
                                               const double* __restrict__ W, const double* __restrict__ SW,
                                               const double* __restrict__ bm) {
    __shared__ double sh[WPB];
    if (state[0]) return;   // the first kernel stopped the solve
    const double beta = bm[0];
    double mu[kW];
#pragma unroll
    for (int v = 0; v < kW; ++v) mu[v] = bm[1 + v];
    const int lane = threadIdx.x % kWave;
    const int grp = lane / 9, comp = lane % 9;
    double dq = 0.0;
    if (grp < GRPW) {
        for (int r0 = (blockIdx.x * WPB + threadIdx.x / kWave) * GRPW; r0 < n_rows; r0 += gridDim.x * WPB * GRPW) {
            const int row = r0 + grp;
            if (row >= n_rows) break;
            const double sv = column_sum(row, comp, lo_ptr, lo_blk, u, tb);
            dq += a_finish<FIRST>(row, comp, sv, z, d, q, beta, defl, W, SW, mu);
        }
    }
    const double t = block_total(wave_sum(dq), sh);
    if (threadIdx.x == 0) pA[blockIdx.x] = t;
}

// plain y = S x with the UPPER product (two kernels)
template <bool TR, typename TS>
__global__ __launch_bounds__(BS) void k_upper_part(int n_rows, const int32_t* __restrict__ row_ptr,
                                                   const int32_t* __restrict__ col_idx, const TS* __restrict__ blk,
                                                   const double* __restrict__ x, double* __restrict__ u,
                                                   double* __restrict__ tb) {
    const int lane = threadIdx.x % kWave;
    for (int row = blockIdx.x * WPB + threadIdx.x / kWave; row < n_rows; row += gridDim.x * WPB) {
        const int a0 = row_ptr[row];
        const double v = row_upper<TR, TS>(row, a0, row_ptr[row + 1] - a0, col_idx, blk, x, tb);
        if (lane < 9) u[(int64_t)row * 9 + lane] = v;
    }
}
__global__ __launch_bounds__(BS) void k_upper_sum(int n_rows, const int32_t* __restrict__ lo_ptr,
                                                  const int32_t* __restrict__ lo_blk, const double* __restrict__ u,
                                                  const double* __restrict__ tb, double* __restrict__ y) {
    const int lane = threadIdx.x % kWave;
    const int grp = lane / 9, comp = lane % 9;
    if (grp >= GRPW) return;
    for (int r0 = (blockIdx.x * WPB + threadIdx.x / kWave) * GRPW; r0 < n_rows; r0 += gridDim.x * WPB * GRPW) {
        const int row = r0 + grp;
        if (row >= n_rows) break;
        y[(int64_t)row * 9 + comp] = column_sum(row, comp, lo_ptr, lo_blk, u, tb);
    }
}

__global__ __launch_bounds__(BS) void k_pcg_B(int n_rows, const double* __restrict__ M, const double* __restrict__ d,
                                              const double* __restrict__ q, double* __restrict__ x,
                                              double* __restrict__ r, double* __restrict__ z,
                                              const double* __restrict__ pA, double* __restrict__ pR, int n_part,
                                              int* __restrict__ state, int defl, const double* __restrict__ SW) {
    __shared__ double sh[NP * WPB];
    __shared__ double sr[RPB][9];
    const int lr = threadIdx.x / 9, i = threadIdx.x % 9;
    // row i of the thread's block of M, requested a pass ahead (the first
    // one before the partial sums): M does not depend on the step
    double mr[9];
    auto load_m = [&](int base) {
        const int row = base + lr;
        if (threadIdx.x < RPB * 9 && row < n_rows) {
            const double* Mr = M + (int64_t)row * 81 + i * 9;
#pragma unroll
            for (int c = 0; c < 9; ++c) mr[c] = Mr[c];
        }
    };
    load_m(blockIdx.x * RPB);
    const int done = state[0];
    const int k = state[1];
    double s[2];
    sum_partials<1>(pA, n_part, 1, s, sh);
    sum_partials<1>(pR + (int64_t)NP * n_part * (k & 1), n_part, NP, s + 1, sh);
    if (done) return;
    const double dq = s[0], rz = s[1];
    if (!(dq > 0.0)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) { state[0] = 1; state[2] = BA_ERR_NOT_SPD; }
        return;
    }
    const double alpha = rz / dq;
    double acc[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) acc[j] = 0.0;
    for (int base = blockIdx.x * RPB; base < n_rows; base += gridDim.x * RPB) {
        const int row = base + lr;
        const bool act = threadIdx.x < RPB * 9 && row < n_rows;
        const int64_t o = (int64_t)row * 9 + i;
        double rv = 0.0;
        if (act) {
            x[o] += alpha * d[o];
            rv = r[o] - alpha * q[o];
            r[o] = rv;
            sr[lr][i] = rv;
        }
        __syncthreads();
        if (act) {
            double zv = 0.0;
#pragma unroll
            for (int c = 0; c < 9; ++c) zv += mr[c] * sr[lr][c];
            z[o] = zv;
            acc[0] += rv * zv;
            acc[1] += rv * rv;
            if (defl) {
                const double* Sr = SW + (int64_t)row * kW * 9 + i;
#pragma unroll
                for (int v = 0; v < kW; ++v) acc[2 + v] += Sr[v * 9] * zv;
            }
        }
        load_m(base + gridDim.x * RPB);
        __syncthreads();
    }
    double t[NP];
    block_totals<NP>(acc, t, sh);
    double* out = pR + (int64_t)NP * n_part * ((k + 1) & 1) + (int64_t)NP * blockIdx.x;
    if (threadIdx.x == 0)
        for (int j = 0; j < NP; ++j) out[j] = t[j];
    if (blockIdx.x == 0 && threadIdx.x == 0) state[3] = k + 1;
}

// factorised preconditioner, first half: update and t = G r'; UP: from the
// transposed blocks GlT, with the transposed products G_row,j^T t_row per
// entry (tg) for the one-read apply of G^T
template <bool UP, bool H = false>
__global__ __launch_bounds__(BS) void k_pcg_Bf(int n_rows, const int32_t* __restrict__ gl_ptr,
                                               const int32_t* __restrict__ gl_col, const float* __restrict__ Gl,
                                               const float* __restrict__ GlT,
                                               const double* __restrict__ d,
                                               const double* __restrict__ q, double* __restrict__ x,
                                               double* __restrict__ r0buf, double* __restrict__ r1buf,
                                               double* __restrict__ t, double* __restrict__ tg,
                                               const double* __restrict__ pA,
                                               double* __restrict__ pR, int n_part, int* __restrict__ state,
                                               const uint32_t* __restrict__ Gh, const uint16_t* __restrict__ Gh8,
                                               const float* __restrict__ hs,
                                               const double* __restrict__ Dn) {
    __shared__ double sh[2 * WPB];
    const int done = state[0];
    const int k = state[1];
    double s[2];
    sum_partials<1>(pA, n_part, 1, s, sh);
    sum_partials<1>(pR + (int64_t)NP * n_part * (k & 1), n_part, NP, s + 1, sh);
    if (done) return;
    const double dq = s[0], rz = s[1];
    if (!(dq > 0.0)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) { state[0] = 1; state[2] = BA_ERR_NOT_SPD; }
        return;
    }
    const double alpha = rz / dq;
    const double* rin = (k & 1) ? r1buf : r0buf;
    double* rout = (k & 1) ? r0buf : r1buf;
    const int lane = threadIdx.x % kWave;
    double rr = 0.0;
    for (int row = blockIdx.x * WPB + threadIdx.x / kWave; row < n_rows; row += gridDim.x * WPB) {
        const int a0 = gl_ptr[row], n = gl_ptr[row + 1] - a0;
        const double tv = UP ? row_factor_t<1, H>(a0, n, gl_col, GlT, rin, q, alpha, tg, Gh, Gh8, hs, Dn)
                             : row_gather<float, 1>(a0, n, gl_col, Gl, rin, q, alpha);
        if (lane < 9) {
            const int64_t o = (int64_t)row * 9 + lane;
            x[o] += alpha * d[o];
            const double rv = rin[o] - alpha * q[o];
            rout[o] = rv;
            if (!UP) t[o] = tv;
            rr += rv * rv;
        }
    }
    const double tot = block_total(wave_sum(rr), sh);
    if (threadIdx.x == 0) pR[(int64_t)NP * n_part * ((k + 1) & 1) + (int64_t)NP * blockIdx.x + 1] = tot;
}

// factorised preconditioner, second half: z = G^T t, r'^T z, (SW)^T z.
// INIT: the initial z0 (r in buffer 0, parity 0, no counter update).
// UP: z_j = sum of the transposed products tg of the entries (i, j) of
// column j of G (ascending i, one lane group per row) instead of a gather
// over a transposed copy of G.
template <bool INIT, bool UP, bool H = false>
__global__ __launch_bounds__(BS) void k_pcg_Cf(int n_rows, const int32_t* __restrict__ gu_ptr,
                                               const int32_t* __restrict__ gu_col, const float* __restrict__ Gu,
                                               const double* __restrict__ t, const int32_t* __restrict__ gu_src,
                                               const double* __restrict__ tg,
                                               const double* __restrict__ r0buf, const double* __restrict__ r1buf,
                                               double* __restrict__ z, double* __restrict__ pR, int n_part,
                                               int* __restrict__ state, int defl, const double* __restrict__ SW,
                                               const double* __restrict__ Dn) {
    __shared__ double sh[NP * WPB];
    int k = -1;
    if (!INIT) {
        if (state[0]) return;
        k = state[1];
    }
    const double* r = ((k + 1) & 1) ? r1buf : r0buf;
    const int lane = threadIdx.x % kWave;
    double acc[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) acc[j] = 0.0;
    auto finish = [&](int row, int c, double zv) {
        const int64_t o = (int64_t)row * 9 + c;
        z[o] = zv;
        acc[0] += r[o] * zv;
        if (defl) {
            const double* Sr = SW + (int64_t)row * kW * 9 + c;
#pragma unroll
            for (int v = 0; v < kW; ++v) acc[2 + v] += Sr[v * 9] * zv;
        }
    };
    if (UP) {
        const int grp = lane / 9, comp = lane % 9;
        if (grp < GRPW)
            for (int r0 = (blockIdx.x * WPB + threadIdx.x / kWave) * GRPW; r0 < n_rows;
                 r0 += gridDim.x * WPB * GRPW) {
                const int row = r0 + grp;
                if (row >= n_rows) break;
                const int a0 = gu_ptr[row];
                double zv = index_sum(a0, gu_ptr[row + 1] - a0, gu_src, tg, comp, 0.0);
                if (H) zv *= Dn[(int64_t)row * 9 + comp];
                finish(row, comp, zv);
            }
    } else {
        for (int row = blockIdx.x * WPB + threadIdx.x / kWave; row < n_rows; row += gridDim.x * WPB) {
            const int a0 = gu_ptr[row];
            const double zv = row_gather<float, 0>(a0, gu_ptr[row + 1] - a0, gu_col, Gu, t, nullptr, 0.0);
            if (lane < 9) finish(row, lane, zv);
        }
    }
    double tot[NP];
    block_totals<NP>(acc, tot, sh);
    double* out = pR + (int64_t)NP * n_part * ((k + 1) & 1) + (int64_t)NP * blockIdx.x;
    if (threadIdx.x == 0) {
        out[0] = tot[0];
        for (int j = 2; j < NP; ++j) out[j] = tot[j];
    }
    if (!INIT && blockIdx.x == 0 && threadIdx.x == 0) state[3] = k + 1;
}

int grid_of(int n_rows) { return std::max(1, std::min((n_rows + WPB - 1) / WPB, kMaxGrid)); }

// S products of the current solve: FULL (FP64 Sf or FP32 Sf32) or UPPER
// (the FP64 upper blocks, or their transposed FP32 copy Su32)
template <bool FIRST>
void launch_A(ba_ctx* c, int g, double tol, int max_iter, int defl, hipStream_t st) {
    Pcg& P = c->pcg;
    const int nr = c->n_rows;
    if (c->upper) {
        if (c->s32)
            k_pcg_A1<FIRST, true, float><<<g, BS, 0, st>>>(nr, c->row_ptr, c->col_idx, c->Su32, P.z, P.u, P.tb, P.pR,
                                                          g, P.state, P.scal, tol, max_iter, defl, P.Einv, P.bm);
        else
            k_pcg_A1<FIRST, false, double><<<g, BS, 0, st>>>(nr, c->row_ptr, c->col_idx, c->blk, P.z, P.u, P.tb,
                                                            P.pR, g, P.state, P.scal, tol, max_iter, defl, P.Einv, P.bm);
        k_pcg_A2<FIRST><<<g, BS, 0, st>>>(nr, c->lo_ptr, c->lo_blk, P.u, P.tb, P.z, P.d, P.q, P.pA, P.state, defl,
                                          P.W, P.SW, P.bm);
        return;
    }
    if (c->s32)
        k_pcg_A<FIRST, float><<<g, BS, 0, st>>>(nr, c->sf_ptr, c->sf_col, c->Sf32, P.z, P.d, P.q, P.pA, P.pR, g,
                                                P.state, P.scal, tol, max_iter, defl, P.W, P.SW, P.Einv);
    else
        k_pcg_A<FIRST, double><<<g, BS, 0, st>>>(nr, c->sf_ptr, c->sf_col, c->Sf, P.z, P.d, P.q, P.pA, P.pR, g,
                                                 P.state, P.scal, tol, max_iter, defl, P.W, P.SW, P.Einv);
}

// Kernels Bf and Cf of an iteration with the factorised preconditioner
// (UPPER: G^T applied from the transposed products of Bf)
void launch_factor_step(ba_ctx* c, int g, int defl, hipStream_t st) {
    Pcg& P = c->pcg;
    Fsai& F = c->fs;
    const int nr = c->n_rows;
    if (F.gu_upper != c->upper) throw ba_hip_error(hipErrorInvalidValue, "factor apply (layout of the transposed blocks)", __FILE__, __LINE__);
    if (c->upper && F.half) {
        k_pcg_Bf<true, true><<<g, BS, 0, st>>>(nr, F.ptr, F.J, F.Gl, F.Gu, P.d, P.q, P.x, P.r[0], P.r[1], P.t, F.tg,
                                               P.pA, P.pR, g, P.state, F.Gh, F.Gh8, F.hs, F.Dn);
        k_pcg_Cf<false, true, true><<<g, BS, 0, st>>>(nr, F.gu_ptr, F.gu_col, F.Gu, P.t, F.gu_src, F.tg, P.r[0],
                                                      P.r[1], P.z, P.pR, g, P.state, defl, P.SW, F.Dn);
    } else if (c->upper) {
        k_pcg_Bf<true><<<g, BS, 0, st>>>(nr, F.ptr, F.J, F.Gl, F.Gu, P.d, P.q, P.x, P.r[0], P.r[1], P.t, F.tg, P.pA,
                                         P.pR, g, P.state, nullptr, nullptr, nullptr, nullptr);
        k_pcg_Cf<false, true><<<g, BS, 0, st>>>(nr, F.gu_ptr, F.gu_col, F.Gu, P.t, F.gu_src, F.tg, P.r[0], P.r[1],
                                                P.z, P.pR, g, P.state, defl, P.SW, nullptr);
    } else {
        k_pcg_Bf<false><<<g, BS, 0, st>>>(nr, F.ptr, F.J, F.Gl, F.Gu, P.d, P.q, P.x, P.r[0], P.r[1], P.t, F.tg, P.pA,
                                          P.pR, g, P.state, nullptr, nullptr, nullptr, nullptr);
        k_pcg_Cf<false, false><<<g, BS, 0, st>>>(nr, F.gu_ptr, F.gu_col, F.Gu, P.t, F.gu_src, F.tg, P.r[0],
                                                 P.r[1], P.z, P.pR, g, P.state, defl, P.SW, nullptr);
    }
}

// z0 = G^T G r0 (the initial preconditioner application)
void launch_factor_init(ba_ctx* c, int g, int defl, hipStream_t st) {
    Pcg& P = c->pcg;
    Fsai& F = c->fs;
    const int nr = c->n_rows;
    if (F.gu_upper != c->upper) throw ba_hip_error(hipErrorInvalidValue, "factor apply (layout of the transposed blocks)", __FILE__, __LINE__);
    if (c->upper && F.half) {
        k_gather_lower<true, true><<<g, BS, 0, st>>>(nr, F.ptr, F.J, F.Gl, F.Gu, P.r[0], P.t, F.tg, F.Gh, F.Gh8, F.hs, F.Dn);
        k_pcg_Cf<true, true, true><<<g, BS, 0, st>>>(nr, F.gu_ptr, F.gu_col, F.Gu, P.t, F.gu_src, F.tg, P.r[0],
                                                     P.r[1], P.z, P.pR, g, P.state, defl, P.SW, F.Dn);
    } else if (c->upper) {
        k_gather_lower<true><<<g, BS, 0, st>>>(nr, F.ptr, F.J, F.Gl, F.Gu, P.r[0], P.t, F.tg, nullptr, nullptr, nullptr,
                                               nullptr);
        k_pcg_Cf<true, true><<<g, BS, 0, st>>>(nr, F.gu_ptr, F.gu_col, F.Gu, P.t, F.gu_src, F.tg, P.r[0], P.r[1],
                                               P.z, P.pR, g, P.state, defl, P.SW, nullptr);
    } else {
        k_gather_lower<false><<<g, BS, 0, st>>>(nr, F.ptr, F.J, F.Gl, F.Gu, P.r[0], P.t, F.tg, nullptr, nullptr, nullptr,
                                                nullptr);
        k_pcg_Cf<true, false><<<g, BS, 0, st>>>(nr, F.gu_ptr, F.gu_col, F.Gu, P.t, F.gu_src, F.tg, P.r[0],
                                                P.r[1], P.z, P.pR, g, P.state, defl, P.SW, nullptr);
    }
}

// y = S x with the copies of the current solve (FULL: Sf or Sf32; UPPER:
// the upper blocks or Su32, through the u / tb buffers)
void product_cur(ba_ctx* c, const double* x, double* y, hipStream_t st) {
    const int nr = c->n_rows, g = grid_of(nr);
    if (c->upper) {
        Pcg& P = c->pcg;
        if (c->s32)
            k_upper_part<true, float><<<g, BS, 0, st>>>(nr, c->row_ptr, c->col_idx, c->Su32, x, P.u, P.tb);
        else
            k_upper_part<false, double><<<g, BS, 0, st>>>(nr, c->row_ptr, c->col_idx, c->blk, x, P.u, P.tb);
        k_upper_sum<<<g, BS, 0, st>>>(nr, c->lo_ptr, c->lo_blk, P.u, P.tb, y);
    } else if (c->s32) {
        k_spmv<float><<<g, BS, 0, st>>>(nr, c->sf_ptr, c->sf_col, c->Sf32, x, y);
    } else {
        k_spmv<double><<<g, BS, 0, st>>>(nr, c->sf_ptr, c->sf_col, c->Sf, x, y);
    }
}

void enqueue_iterations(ba_ctx* c, int mode, const double* M, int defl, double tol, int max_iter, int count,
                        hipStream_t st) {
    Pcg& P = c->pcg;
    const int nr = c->n_rows, g = grid_of(nr);
    for (int i = 0; i < count; ++i) {
        launch_A<false>(c, g, tol, max_iter, defl, st);
        if (mode == 0) {
            k_pcg_B<<<g, BS, 0, st>>>(nr, M, P.d, P.q, P.x, P.r[0], P.z, P.pA, P.pR, g, P.state, defl, P.SW);
        } else {
            launch_factor_step(c, g, defl, st);
        }
    }
}

}  // namespace

// The copies of the current RCS that the next products read: the
// row-major copy of both triangles (FULL products, and with `full` always)
// and its FP32 rounding for an FP32 solve; for an FP32 UPPER solve the
// transposed FP32 upper blocks.
void ensure_sf(ba_ctx* c, bool full) {
    if (c->n_sf == 0) return;
    const int64_t n = c->n_sf * 81;
    const unsigned g = (unsigned)std::min<int64_t>((n + BS - 1) / BS, 8192);
    if (full || !c->upper) {
        if (!c->sf_ready) {
            k_build_sf<double><<<g, BS, 0, c->stream>>>(c->n_sf, c->sf_src, c->blk, c->Sf);
            c->sf_ready = true;
        }
        if (c->s32 && !c->sf32_ready) {
            k_build_sf<float><<<g, BS, 0, c->stream>>>(c->n_sf, c->sf_src, c->blk, c->Sf32);
            c->sf32_ready = true;
        }
    }
    if (c->s32 && c->upper && !c->su32_ready && c->n_blk > 0) {
        const unsigned gu = (unsigned)std::min<int64_t>((c->n_blk * 81 + BS - 1) / BS, 8192);
        k_build_su32<<<gu, BS, 0, c->stream>>>(c->n_blk, c->blk, c->Su32);
        c->su32_ready = true;
    }
}

// Gauge vectors of the last linearization, S W and E^-1 of the current RCS
void prepare_deflation(ba_ctx* c) {
    Pcg& P = c->pcg;
    const int nr = c->n_rows, g = grid_of(nr);
    hipStream_t st = c->stream;
    k_gauge_W<<<(c->n_cams + 255) / 256, 256, 0, st>>>(c->n_cams, c->cam_row, c->lin_cams, P.W);
    ensure_sf(c, true);
    if (c->s32)
        k_spmm_W<float><<<g, BS, 0, st>>>(nr, c->sf_ptr, c->sf_col, c->Sf32, P.W, P.SW);
    else
        k_spmm_W<double><<<g, BS, 0, st>>>(nr, c->sf_ptr, c->sf_col, c->Sf, P.W, P.SW);
    c->defl_s32 = c->s32;
    k_defl_E_part<<<g, BS, 0, st>>>(nr, P.W, P.SW, P.pE);
    k_defl_E_sum<<<kW * kW, BS, 0, st>>>(g, P.pE, P.bm + 8);
    k_defl_E_fin<<<1, 64, 0, st>>>(P.bm + 8, P.Einv, c->flags);
}

ba_status run_pcg(ba_ctx* c, int mode, const double* M, int defl, double tol, int max_iter, const double* x0,
                  double* out, int* iters, double* relres) {
    Pcg& P = c->pcg;
    const int nr = c->n_rows, g = grid_of(nr);
    hipStream_t st = c->stream;
    ensure_sf(c, false);
    const double* q0 = nullptr;
    if (x0) {
        product_cur(c, x0, P.q, st);
        q0 = P.q;
    }
    if (defl) k_defl_Wr<<<g, BS, 0, st>>>(nr, c->rhs, q0, P.W, P.pW);
    k_pcg_init<<<g, BS, 0, st>>>(nr, c->rhs, q0, x0, mode == 0 ? M : nullptr, P.x, P.r[0], P.z, P.pR, P.state, P.scal,
                                 defl, P.W, P.SW, P.Einv, P.pW, g);
    if (mode != 0) {
        launch_factor_init(c, g, defl, st);
    }
    launch_A<true>(c, g, tol, max_iter, defl, st);
    if (max_iter > 0) {
        if (mode == 0) {
            k_pcg_B<<<g, BS, 0, st>>>(nr, M, P.d, P.q, P.x, P.r[0], P.z, P.pA, P.pR, g, P.state, defl, P.SW);
        } else {
            launch_factor_step(c, g, defl, st);
        }
    }
    // remaining iterations in fixed batches (a captured graph when possible);
    // the stop flag of a batch is read back while the next batch runs, and
    // kernels after the stop return at once
    const int batch = kPcgBatch;
    const int n_batches = max_iter > 0 ? (max_iter + batch - 1) / batch : 0;
    hipGraphExec_t exec = nullptr;
    if (c->use_graphs && n_batches > 0) {
        for (auto& gr : c->pcg_graphs)
            if (gr.M == M && gr.mode == mode && gr.defl == defl && gr.s32 == c->s32 && gr.upper == c->upper &&
                gr.half == c->fs.half && gr.tol == tol && gr.max_iter == max_iter)
                exec = gr.exec;
        if (!exec) {
            hipStream_t cs = c->capture_stream;
            hipGraph_t graph = nullptr;
            BA_HIP_CHECK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
            enqueue_iterations(c, mode, M, defl, tol, max_iter, batch, cs);
            BA_HIP_CHECK(hipStreamEndCapture(cs, &graph));
            BA_HIP_CHECK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
            BA_HIP_CHECK(hipGraphDestroy(graph));
            c->pcg_graphs.push_back({M, mode, defl, c->s32, c->upper, c->fs.half, tol, max_iter, exec});
        }
    }
    hipEvent_t evb[2] = {c->ev[12], c->ev[13]};
    int* hflag[2] = {c->h_flags + 8, c->h_flags + 12};
    int slot = 0, pending = 0, launched = 0;
    bool done = max_iter == 0;
    while (!done) {
        if (launched < n_batches) {
            if (exec)
                BA_HIP_CHECK(hipGraphLaunch(exec, st));
            else
                enqueue_iterations(c, mode, M, defl, tol, max_iter, batch, st);
            ++launched;
            BA_HIP_CHECK(hipMemcpyAsync(hflag[slot], P.state, 3 * sizeof(int), hipMemcpyDeviceToHost, st));
            BA_HIP_CHECK(hipEventRecord(evb[slot], st));
            slot ^= 1;
            ++pending;
            if (pending < 2 && launched < n_batches) continue;   // keep one batch in flight
        }
        if (pending == 0) break;
        const int s_old = slot ^ (pending == 2 ? 0 : 1);
        BA_HIP_CHECK(hipEventSynchronize(evb[s_old]));
        --pending;
        if (hflag[s_old][0]) done = true;
        if (launched >= n_batches && pending == 0) break;
    }
    BA_HIP_CHECK(hipMemcpyAsync(c->h_flags + 4, P.state, 4 * sizeof(int), hipMemcpyDeviceToHost, st));
    BA_HIP_CHECK(hipMemcpyAsync(c->h_scal + 8, P.scal, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    BA_HIP_CHECK(hipMemcpyAsync(out, P.x, (size_t)nr * 9 * sizeof(double), hipMemcpyDeviceToDevice, st));
    BA_HIP_CHECK(hipStreamSynchronize(st));
    *iters = c->h_flags[7];
    *relres = c->h_scal[9];
    return (ba_status)c->h_flags[6];
}

// y = S x in the layout selected for the next solve (c->upper, c->s32)
void launch_product(ba_ctx* c, const double* x, double* y) {
    if (c->n_rows == 0) return;
    ensure_sf(c, false);
    product_cur(c, x, y, c->stream);
}

void launch_dscale(ba_ctx* c) {
    const int nr = c->n_rows;
    if (nr > 0)
        k_dscale<<<(unsigned)(((int64_t)nr * 9 + BS - 1) / BS), BS, 0, c->stream>>>(nr, c->row_ptr, c->blk, c->fs.Dn);
}

void launch_pack_half(ba_ctx* c) {
    Fsai& F = c->fs;
    if (F.n_mem > 0)
        k_pack_half<<<(unsigned)((F.n_mem + 2) / 3), BS, 0, c->stream>>>(F.n_mem, F.J, F.Gu, F.Dn, F.Gh, F.Gh8, F.hs);
}

}  // namespace ba
