// Block-diagonal preconditioned CG on the RCS (Sec. 3.2, Eq. (6)-(7)) with
// the symmetric block product of Sec. 6.2 on upper-triangle storage.
//
// One iteration is two kernels and no host round trip:
//   A_k: beta = rz_k / rz_{k-1};  d_k = z_k + beta d_{k-1} (recomputed on the
//        fly for every neighbour it reads);  q = S d_k;  partial d_k^T q.
//        Also the stop test |r_k| / |r_0| <= tol and the iteration cap.
//   B_k: alpha = rz_k / d_k^T q;  y += alpha d_k;  r -= alpha q;
//        z = M^-1 r;  partial r^T z and r^T r.
// Every block re-sums the partials of the previous kernel in the same fixed
// order, so all blocks take the same decisions; block 0 records them.
#include "ba_common.hpp"

namespace ba {

namespace {

constexpr int BS = 256;
constexpr int RPA = BS / kWave;   // rows per block in kernel A (one wave per row)
constexpr int RPB = BS / 9;       // rows per block in kernel B (9 threads per row)

// deterministic sum of n values, result valid in every lane of wave 0 (and
// broadcast through LDS to the block)
__device__ __forceinline__ double block_sum_of(const double* __restrict__ v, int n, int stride, double* sh) {
    if (threadIdx.x < kWave) {
        double s = 0.0;
        for (int i = threadIdx.x; i < n; i += kWave) s += v[(int64_t)i * stride];
        s = wave_sum(s);
        if (threadIdx.x == 0) sh[0] = s;
    }
    __syncthreads();
    const double r = sh[0];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(BS) void k_pcg_init(int n_rows, const double* __restrict__ rhs, const double* __restrict__ q,
                                                 const double* __restrict__ x0, const double* __restrict__ M,
                                                 double* __restrict__ x, double* __restrict__ r, double* __restrict__ z,
                                                 double* __restrict__ pB, int* __restrict__ state,
                                                 double* __restrict__ scal) {
    __shared__ double sr[RPB][9];
    __shared__ double sh[BS / kWave];
    const int lr = threadIdx.x / 9, i = threadIdx.x % 9;
    const int row = blockIdx.x * RPB + lr;
    const bool act = threadIdx.x < RPB * 9 && row < n_rows;
    double rv = 0.0;
    if (act) {
        const int64_t o = (int64_t)row * 9 + i;
        rv = rhs[o] - (q ? q[o] : 0.0);
        x[o] = x0 ? x0[o] : 0.0;
        r[o] = rv;
        sr[lr][i] = rv;
    }
    __syncthreads();
    double zv = 0.0;
    if (act) {
        const double* Mr = M + (int64_t)row * 81 + i * 9;
#pragma unroll
        for (int c = 0; c < 9; ++c) zv += Mr[c] * sr[lr][c];
        z[(int64_t)row * 9 + i] = zv;
    }
    const double rz = block_sum<BS>(rv * zv, sh);
    const double rr = block_sum<BS>(rv * rv, sh);
    if (threadIdx.x == 0) {
        pB[2 * blockIdx.x] = rz;
        pB[2 * blockIdx.x + 1] = rr;
        if (blockIdx.x == 0) { state[0] = 0; state[1] = 0; state[2] = BA_OK; scal[1] = -1.0; }
    }
}

// Symmetric block product row by row: one wave per block row, lanes as 7
// groups of 9 (block, output component); upper blocks S_rs contribute
// S_rs x_s, transposed blocks (s, r), s < r, contribute S_sr^T x_s.
// mode 0: plain q = S x (x = z argument, no PCG logic).
// mode 1: PCG kernel A.
template <int MODE>
__global__ __launch_bounds__(BS) void k_pcg_A(int k, int n_rows, const int32_t* __restrict__ row_ptr,
                                              const int32_t* __restrict__ col_idx, const int32_t* __restrict__ tr_ptr,
                                              const int32_t* __restrict__ tr, const double* __restrict__ blk,
                                              const double* __restrict__ z, const double* __restrict__ dprev,
                                              double* __restrict__ dcur, double* __restrict__ q,
                                              double* __restrict__ pA, const double* __restrict__ pBk,
                                              const double* __restrict__ pBkm1, int nB, int* __restrict__ state,
                                              double* __restrict__ scal, double tol, int max_iter) {
    __shared__ double sh[4];
    __shared__ double sacc[RPA][kWave];
    __shared__ double sdq[RPA];
    double beta = 0.0;
    if (MODE == 1) {
        if (state[0]) return;
        const double rz = block_sum_of(pBk, nB, 2, sh);
        const double rr = block_sum_of(pBk + 1, nB, 2, sh);
        double r0sq;
        if (k == 0) {
            r0sq = rr;
            if (blockIdx.x == 0 && threadIdx.x == 0) scal[0] = rr;
        } else {
            r0sq = scal[0];
        }
        const bool conv = (rr == 0.0) || (sqrt(rr) <= tol * sqrt(r0sq));
        if (conv || k >= max_iter) {
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                state[0] = 1;
                state[1] = k;
                state[2] = conv ? BA_OK : BA_ERR_NOT_CONVERGED;
                scal[1] = r0sq > 0.0 ? sqrt(rr / r0sq) : 0.0;
            }
            return;
        }
        if (k > 0) beta = rz / block_sum_of(pBkm1, nB, 2, sh);
    }
    const int wv = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int row = blockIdx.x * RPA + wv;
    const int grp = lane / 9, comp = lane % 9;
    double acc = 0.0;
    if (row < n_rows && grp < 7) {
        for (int kk = row_ptr[row] + grp; kk < row_ptr[row + 1]; kk += 7) {
            const int s = col_idx[kk];
            const double* S = blk + (int64_t)kk * 81 + comp * 9;
            const double* zs = z + (int64_t)s * 9;
            if (MODE == 1 && k > 0) {
                const double* ds = dprev + (int64_t)s * 9;
#pragma unroll
                for (int c = 0; c < 9; ++c) acc += S[c] * (zs[c] + beta * ds[c]);
            } else {
#pragma unroll
                for (int c = 0; c < 9; ++c) acc += S[c] * zs[c];
            }
        }
        for (int t = tr_ptr[row] + grp; t < tr_ptr[row + 1]; t += 7) {
            const int kb = tr[2 * t], s = tr[2 * t + 1];
            const double* S = blk + (int64_t)kb * 81 + comp;
            const double* zs = z + (int64_t)s * 9;
            if (MODE == 1 && k > 0) {
                const double* ds = dprev + (int64_t)s * 9;
#pragma unroll
                for (int c = 0; c < 9; ++c) acc += S[c * 9] * (zs[c] + beta * ds[c]);
            } else {
#pragma unroll
                for (int c = 0; c < 9; ++c) acc += S[c * 9] * zs[c];
            }
        }
    }
    sacc[wv][lane] = acc;
    __syncthreads();
    double dq = 0.0;
    if (row < n_rows && lane < 9) {
        double qv = 0.0;
#pragma unroll
        for (int gq = 0; gq < 7; ++gq) qv += sacc[wv][gq * 9 + lane];
        const int64_t o = (int64_t)row * 9 + lane;
        q[o] = qv;
        if (MODE == 1) {
            const double dv = (k > 0) ? z[o] + beta * dprev[o] : z[o];
            dcur[o] = dv;
            dq = dv * qv;
        }
    }
    if (MODE == 1) {
        dq = wave_sum(dq);
        if (lane == 0) sdq[wv] = dq;
        __syncthreads();
        if (threadIdx.x == 0) {
            double s = 0.0;
            for (int w = 0; w < RPA; ++w) s += sdq[w];
            pA[blockIdx.x] = s;
        }
    }
}

__global__ __launch_bounds__(BS) void k_pcg_B(int k, int n_rows, const double* __restrict__ M,
                                              const double* __restrict__ dcur, const double* __restrict__ q,
                                              double* __restrict__ x, double* __restrict__ r, double* __restrict__ z,
                                              const double* __restrict__ pA, int nA, const double* __restrict__ pBk,
                                              double* __restrict__ pBk1, int nB, int* __restrict__ state) {
    __shared__ double sh[BS / kWave];
    __shared__ double sr[RPB][9];
    if (state[0]) return;
    const double dq = block_sum_of(pA, nA, 1, sh);
    const double rz = block_sum_of(pBk, nB, 2, sh);
    if (!(dq > 0.0)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) { state[0] = 1; state[1] = k; state[2] = BA_ERR_NOT_SPD; }
        return;
    }
    const double alpha = rz / dq;
    const int lr = threadIdx.x / 9, i = threadIdx.x % 9;
    const int row = blockIdx.x * RPB + lr;
    const bool act = threadIdx.x < RPB * 9 && row < n_rows;
    double rv = 0.0;
    if (act) {
        const int64_t o = (int64_t)row * 9 + i;
        x[o] += alpha * dcur[o];
        rv = r[o] - alpha * q[o];
        r[o] = rv;
        sr[lr][i] = rv;
    }
    __syncthreads();
    double zv = 0.0;
    if (act) {
        const double* Mr = M + (int64_t)row * 81 + i * 9;
#pragma unroll
        for (int c = 0; c < 9; ++c) zv += Mr[c] * sr[lr][c];
        z[(int64_t)row * 9 + i] = zv;
    }
    const double rzn = block_sum<BS>(rv * zv, sh);
    const double rr = block_sum<BS>(rv * rv, sh);
    if (threadIdx.x == 0) {
        pBk1[2 * blockIdx.x] = rzn;
        pBk1[2 * blockIdx.x + 1] = rr;
    }
}

}  // namespace

ba_status run_pcg(ba_ctx* c, const double* M, double tol, int max_iter, const double* x0, double* out, int* iters,
                  double* relres) {
    Pcg& P = c->pcg;
    const int nr = c->n_rows;
    const int nA = (nr + RPA - 1) / RPA, nB = (nr + RPB - 1) / RPB;
    const double* q0 = nullptr;
    if (x0) {
        k_pcg_A<0><<<nA, BS, 0, c->stream>>>(0, nr, c->row_ptr, c->col_idx, c->tr_ptr, c->tr_blk, c->blk, x0, nullptr,
                                             nullptr, P.q, nullptr, nullptr, nullptr, 0, nullptr, nullptr, 0.0, 0);
        q0 = P.q;
    }
    k_pcg_init<<<nB, BS, 0, c->stream>>>(nr, c->rhs, q0, x0, M, P.x, P.r, P.z, P.pB[0], P.state, P.scal);
    const int batch = 16;
    for (int k0 = 0; k0 <= max_iter; k0 += batch) {
        const int k1 = std::min(max_iter, k0 + batch - 1);
        for (int k = k0; k <= k1; ++k) {
            k_pcg_A<1><<<nA, BS, 0, c->stream>>>(k, nr, c->row_ptr, c->col_idx, c->tr_ptr, c->tr_blk, c->blk, P.z,
                                                 P.d[(k + 1) & 1], P.d[k & 1], P.q, P.pA, P.pB[k & 1],
                                                 P.pB[(k + 1) & 1], nB, P.state, P.scal, tol, max_iter);
            if (k < max_iter)
                k_pcg_B<<<nB, BS, 0, c->stream>>>(k, nr, M, P.d[k & 1], P.q, P.x, P.r, P.z, P.pA, nA, P.pB[k & 1],
                                                  P.pB[(k + 1) & 1], nB, P.state);
        }
        BA_HIP_CHECK(hipMemcpyAsync(c->h_flags + 4, P.state, 3 * sizeof(int), hipMemcpyDeviceToHost, c->stream));
        BA_HIP_CHECK(hipStreamSynchronize(c->stream));
        if (c->h_flags[4]) break;
    }
    BA_HIP_CHECK(hipMemcpyAsync(c->h_scal + 8, P.scal, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    BA_HIP_CHECK(hipMemcpyAsync(out, P.x, (size_t)nr * 9 * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    BA_HIP_CHECK(hipStreamSynchronize(c->stream));
    *iters = c->h_flags[5];
    *relres = c->h_scal[9];
    return (ba_status)c->h_flags[6];
}

void launch_spmv(ba_ctx* c, const double* x, double* y) {
    const int nr = c->n_rows;
    const int nA = (nr + RPA - 1) / RPA;
    k_pcg_A<0><<<nA, BS, 0, c->stream>>>(0, nr, c->row_ptr, c->col_idx, c->tr_ptr, c->tr_blk, c->blk, x, nullptr,
                                         nullptr, y, nullptr, nullptr, nullptr, 0, nullptr, nullptr, 0.0, 0);
}

}  // namespace ba
