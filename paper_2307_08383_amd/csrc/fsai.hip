// Factorised sparse approximate inverse of the RCS (Kolotilina-Yeremin FSAI
// on the lower pattern of Eq. (4)'s camera blocks): M^-1 = G^T G with G
// block-lower-triangular, row i non-zero in the columns J_i (camera i and
// up to kFsaiM - 1 lower neighbours).  Row i is the last block row of the
// inverse Cholesky factor of the local matrix S[J_i, J_i]:
//   S[J_i, J_i] = L L^T  =>  G_i = E_i^T L^-1,
// which satisfies (G_i S)_j = 0 for j in J_i, j != i and G_i S G_i^T = I,
// with G_ii lower triangular with positive diagonal.
//
// The local matrix is factored in FP32 in LDS after block-Jacobi
// normalisation (its diagonal blocks become I):
//   Ahat_jk = L_j^-1 S_jk L_k^-T,  S_jj = L_j L_j^T,
// and the result is mapped back: G_ij = Ghat_ij L_j^-1.  G is written in
// three layouts: the RCS block slots (for copies out), by rows of G and by
// rows of G^T (the two products of the PCG).
#include "ba_common.hpp"

namespace ba {

namespace {

constexpr int BS = 256;

__device__ __forceinline__ int tix(int a, int b) { return a * (a + 1) / 2 + b; }

// An[kb] = L_r^-1 S_rc L_c^-T for the off-diagonal blocks, three blocks per
// workgroup (81 threads each); FP64 arithmetic, FP32 result.
__global__ __launch_bounds__(BS) void k_fsai_norm(int64_t n_blk, const int32_t* __restrict__ brow,
                                                  const int32_t* __restrict__ col_idx, const double* __restrict__ blk,
                                                  const double* __restrict__ Linv, float* __restrict__ An) {
    __shared__ double sS[3][81], sLr[3][81], sLc[3][81], sW[3][81];
    const int lb = threadIdx.x / 81, pq = threadIdx.x % 81;
    const int64_t kb = (int64_t)blockIdx.x * 3 + lb;
    const bool act = lb < 3 && kb < n_blk;
    int r = 0, c = 0;
    if (act) {
        r = brow[kb];
        c = col_idx[kb];
        sS[lb][pq] = blk[kb * 81 + pq];
        sLr[lb][pq] = Linv[(int64_t)r * 81 + pq];
        sLc[lb][pq] = Linv[(int64_t)c * 81 + pq];
    }
    __syncthreads();
    const int p = pq / 9, q = pq % 9;
    if (act && r != c) {
        double w = 0.0;   // W = L_r^-1 S: W[p][q] = sum_{u <= p} Lr[p][u] S[u][q]
        for (int u = 0; u <= p; ++u) w += sLr[lb][p * 9 + u] * sS[lb][u * 9 + q];
        sW[lb][pq] = w;
    }
    __syncthreads();
    if (act && r != c) {
        double a = 0.0;   // W L_c^-T: sum_{v <= q} W[p][v] Lc[q][v]
        for (int v = 0; v <= q; ++v) a += sW[lb][p * 9 + v] * sLc[lb][q * 9 + v];
        An[kb * 81 + pq] = (float)a;
    }
}

// Cholesky of a 9x9 SPD tile by the 64 lanes of one wave (lane l < 45 holds
// lower element (r, c), l = r(r+1)/2 + c); writes L (lower, zero upper) over
// T; returns false if a pivot was not positive (the wave's lanes agree).
__device__ __forceinline__ bool chol9_wave(float* T) {
    const int l = threadIdx.x % kWave;
    const bool act = l < 45;
    int rr = 0;
    while (act && (rr + 1) * (rr + 2) / 2 <= l) ++rr;
    const int cc = act ? l - rr * (rr + 1) / 2 : 0;
    float v = act ? T[rr * 9 + cc] : 0.f;
    bool ok = true;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const float dkk = __shfl(v, k * (k + 1) / 2 + k, kWave);
        ok = ok && dkk > 0.f;
        const float s = dkk > 0.f ? sqrtf(dkk) : 1.f;
        if (act && cc == k) v = (rr == k) ? s : v / s;
        const bool upd = act && cc > k;
        const int la = upd ? rr * (rr + 1) / 2 + k : 0;
        const int lc = upd ? cc * (cc + 1) / 2 + k : 0;
        const float x = __shfl(v, la, kWave);
        const float y = __shfl(v, lc, kWave);
        if (upd) v -= x * y;
    }
    if (act) {
        T[rr * 9 + cc] = v;
        if (rr != cc) T[cc * 9 + rr] = 0.f;
    }
    return ok;
}

// One workgroup per RCS row.
__global__ __launch_bounds__(BS) void k_fsai(const int32_t* __restrict__ fs_ptr, const int32_t* __restrict__ fs_J,
                                             const int32_t* __restrict__ fs_slot, const int64_t* __restrict__ fs_tptr,
                                             const int32_t* __restrict__ fs_tile, const float* __restrict__ An,
                                             const double* __restrict__ Linv, const int32_t* __restrict__ gu_pos,
                                             float* __restrict__ G, float* __restrict__ Gl, float* __restrict__ Gu,
                                             int* __restrict__ flags) {
    __shared__ float T[kFsaiTiles][81];
    __shared__ float sP[3][81];
    __shared__ float sC[81];
    __shared__ int s_bad;
    const int row = blockIdx.x;
    const int j0 = fs_ptr[row], m = fs_ptr[row + 1] - j0;
    const int32_t* tiles = fs_tile + fs_tptr[row];
    const int nt = m * (m + 1) / 2;
    // tiles (a, b), a >= b: Ahat(J_a, J_b) = An[(J_b, J_a)]^T
    for (int e = threadIdx.x; e < nt * 81; e += BS) {
        const int ti = e / 81, pq = e % 81;
        const int kb = tiles[ti];
        float v;
        if (kb == -2)
            v = (pq / 9 == pq % 9) ? 1.f : 0.f;
        else if (kb < 0)
            v = 0.f;
        else
            v = An[(int64_t)kb * 81 + (pq % 9) * 9 + pq / 9];
        T[ti][pq] = v;
    }
    if (threadIdx.x == 0) s_bad = 0;
    __syncthreads();
    for (int b = 0; b < m; ++b) {
        if (threadIdx.x < kWave) {
            const bool ok = chol9_wave(T[tix(b, b)]);
            if (!ok && threadIdx.x == 0) s_bad = 1;
        }
        __syncthreads();
        // panel: L_ab L_bb^T = T_ab, row p of L_ab by forward substitution
        // (one thread per (a, p))
        const float* Lbb = T[tix(b, b)];
        const int np = (m - 1 - b) * 9;
        for (int task = threadIdx.x; task < np; task += BS) {
            const int a = b + 1 + task / 9, p = task % 9;
            float* Tr = &T[tix(a, b)][p * 9];
            float x[9];
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                float s = Tr[q];
#pragma unroll
                for (int c = 0; c < q; ++c) s -= x[c] * Lbb[q * 9 + c];
                x[q] = s / Lbb[q * 9 + q];
            }
#pragma unroll
            for (int q = 0; q < 9; ++q) Tr[q] = x[q];
        }
        __syncthreads();
        // trailing update: T_ac -= L_ab L_cb^T for b < c <= a, one thread
        // per (tile, three rows)
        const int nrem = m - 1 - b;
        const int ntask = nrem * (nrem + 1) / 2 * 3;
        for (int task = threadIdx.x; task < ntask; task += BS) {
            const int tt = task / 3, p0 = (task % 3) * 3;
            int a2 = 0;
            while ((a2 + 1) * (a2 + 2) / 2 <= tt) ++a2;
            const int c2 = tt - a2 * (a2 + 1) / 2;
            const int a = b + 1 + a2, c = b + 1 + c2;
            const float* La = T[tix(a, b)];
            const float* Lc = T[tix(c, b)];
            float* Out = T[tix(a, c)];
            float lr[3][9];
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int u = 0; u < 9; ++u) lr[r][u] = La[(p0 + r) * 9 + u];
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                float lc[9];
#pragma unroll
                for (int u = 0; u < 9; ++u) lc[u] = Lc[q * 9 + u];
#pragma unroll
                for (int r = 0; r < 3; ++r) {
                    float s = 0.f;
#pragma unroll
                    for (int u = 0; u < 9; ++u) s += lr[r][u] * lc[u];
                    Out[(p0 + r) * 9 + q] -= s;
                }
            }
        }
        __syncthreads();
    }
    // last block row of L^-1: R_{m-1} = L_{m-1,m-1}^-1; for b < m-1
    // R_b L_bb = -(sum_{a > b} R_a L_ab).  R_a is kept in tile (m-1, a)
    // (tile (m-1, b) still holds L_{m-1,b} when R_b is formed).
    const int last = m - 1;
    if (threadIdx.x < 9) {
        // column c of L^-1 by forward substitution
        const int c = threadIdx.x;
        const float* L = T[tix(last, last)];
        float x[9];
#pragma unroll
        for (int r = 0; r < 9; ++r) {
            float s = (r == c) ? 1.f : 0.f;
#pragma unroll
            for (int q = 0; q < r; ++q) s -= L[r * 9 + q] * x[q];
            x[r] = r < c ? 0.f : s / L[r * 9 + r];
        }
#pragma unroll
        for (int r = 0; r < 9; ++r) sC[r * 9 + c] = x[r];
    }
    __syncthreads();
    if (threadIdx.x < 81) T[tix(last, last)][threadIdx.x] = sC[threadIdx.x];
    __syncthreads();
    for (int b = last - 1; b >= 0; --b) {
        if (threadIdx.x < 243) {
            const int part = threadIdx.x / 81, pq = threadIdx.x % 81, p = pq / 9, q = pq % 9;
            float s = 0.f;
            for (int a = b + 1 + part; a <= last; a += 3) {
                const float* Ra = T[tix(last, a)];
                const float* Lab = T[tix(a, b)];
#pragma unroll
                for (int u = 0; u < 9; ++u) s += Ra[p * 9 + u] * Lab[u * 9 + q];
            }
            sP[part][pq] = s;
        }
        __syncthreads();
        if (threadIdx.x < 9) {
            // row p of R_b: R_b L_bb = -C, backward over q
            const int p = threadIdx.x;
            const float* Lbb = T[tix(b, b)];
            float r[9];
#pragma unroll
            for (int q = 8; q >= 0; --q) {
                float s = -(sP[0][p * 9 + q] + sP[1][p * 9 + q] + sP[2][p * 9 + q]);
#pragma unroll
                for (int u = q + 1; u < 9; ++u) s -= r[u] * Lbb[u * 9 + q];
                r[q] = s / Lbb[q * 9 + q];
            }
#pragma unroll
            for (int q = 0; q < 9; ++q) sC[p * 9 + q] = r[q];
        }
        __syncthreads();
        if (threadIdx.x < 81) T[tix(last, b)][threadIdx.x] = sC[threadIdx.x];
        __syncthreads();
    }
    // G_{i, J_b} = R_b L_{J_b}^-1 (FP64 accumulation); block-Jacobi row if
    // the local factorisation failed
    const bool bad = s_bad != 0;
    for (int e = threadIdx.x; e < m * 81; e += BS) {
        const int b = e / 81, pq = e % 81, p = pq / 9, q = pq % 9;
        const int j = fs_J[j0 + b];
        const double* Lj = Linv + (int64_t)j * 81;
        double s = 0.0;
        if (!bad) {
            const float* Rb = T[tix(last, b)];
            for (int u = q; u < 9; ++u) s += (double)Rb[p * 9 + u] * Lj[u * 9 + q];
        } else if (b == last) {
            s = Lj[pq];
        }
        const float g = (float)s;
        G[(int64_t)fs_slot[j0 + b] * 81 + pq] = g;
        Gl[(int64_t)(j0 + b) * 81 + pq] = g;
        Gu[(int64_t)gu_pos[j0 + b] * 81 + q * 9 + p] = g;
    }
    if (bad && threadIdx.x == 0) atomicAdd(flags + 2, 1);
}

}  // namespace

void launch_fsai(ba_ctx* c) {
    const int64_t nb = c->n_blk;
    if (nb > 0)
        k_fsai_norm<<<(unsigned)((nb + 2) / 3), BS, 0, c->stream>>>(nb, c->fs.brow, c->col_idx, c->blk, c->Linv,
                                                                    c->fs.An);
    if (c->n_rows > 0)
        k_fsai<<<c->n_rows, BS, 0, c->stream>>>(c->fs.ptr, c->fs.J, c->fs.slot, c->fs.tptr, c->fs.tile, c->fs.An,
                                                c->Linv, c->upper ? c->fs.gl_self : c->fs.gu_pos, c->fs.G, c->fs.Gl,
                                                c->fs.Gu, c->flags);
    c->fs.gu_upper = c->upper;
}

}  // namespace ba
