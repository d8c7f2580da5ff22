// Block-diagonal preconditioned CG on the RCS (Sec. 3.2, Eq. (6)-(7)) with
// the symmetric block product of Sec. 6.2 on upper-triangle storage.
//
// Recurrence (Sec. 3.2): y0 = 0, r0 = b, z0 = M^-1 r0, d0 = z0; per step
//   alpha = r^T z / d^T S d;  y += alpha d;  r -= alpha S d;
//   stop when |r| / |r0| <= tol;  z = M^-1 r;  beta = r^T z / (r^T z)_old;
//   d = z + beta d.
// S d is formed as q_k = S z_k + beta q_{k-1} (the same vector, since
// d_k = z_k + beta d_{k-1}), so the block product only reads z.
//
// One iteration is two kernels and no host round trip:
//   A: s = S z (one 256-thread block per block row), q = s + beta q,
//      d = z + beta d, partial d^T q; also the stop test and iteration cap.
//   B: alpha = rz / d^T q; y += alpha d; r -= alpha q; z = M^-1 r;
//      partial r^T z and r^T r; the iteration counter.
// The iteration number lives in device memory, so a batch of iterations is
// one fixed HIP graph.  Every block re-sums the partials of the previous
// kernel in the same order, so all blocks take the same decisions.
#include "ba_common.hpp"

namespace ba {

namespace {

constexpr int BS = 256;
constexpr int GRP = BS / 9;       // 28 lane groups per row in kernel A
constexpr int RPB = BS / 9;       // rows per block in kernel B (9 threads per row)

// state: [0] done, [1] step index as published by kernel A (read by B),
//        [2] status, [3] completed steps as published by kernel B (read by
//        the next A).  No kernel writes a word that its own blocks read.
// scal:  [0] |r0|^2, [1] final relative residual

template <int N>
__device__ __forceinline__ void sum_partials(const double* __restrict__ const* src, const int* n, const int* stride,
                                             double* out, double* sh) {
    double s[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
        s[j] = 0.0;
        for (int i = threadIdx.x; i < n[j]; i += BS) s[j] += src[j][(int64_t)i * stride[j]];
    }
#pragma unroll
    for (int j = 0; j < N; ++j) {
        const double v = wave_sum(s[j]);
        if ((threadIdx.x % kWave) == 0) sh[j * (BS / kWave) + threadIdx.x / kWave] = v;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < N; ++j) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < BS / kWave; ++w) t += sh[j * (BS / kWave) + w];
        out[j] = t;
    }
    __syncthreads();
}

// s_row = sum over the row's entries, result in sacc[BS..BS+8] (after sync).
// Entries are taken two per lane group per round; both entries of a round,
// then both blocks and vector rows, are requested before any is used.
__device__ __forceinline__ void row_product(int row, int ent_stride, const int2* __restrict__ ent,
                                            const double* __restrict__ blk, const double* __restrict__ x, double* sacc) {
    const int grp = threadIdx.x / 9, comp = threadIdx.x % 9;
    double acc = 0.0;
    if (grp < GRP) {
        const int2* er = ent + (int64_t)row * ent_stride;
        for (int e = grp; e < ent_stride; e += 2 * GRP) {
            const int2 na = er[e];
            const int2 nb = (e + GRP < ent_stride) ? er[e + GRP] : make_int2(-1, 0);
            if (na.x < 0) break;   // padding: the rest of the row is empty
            const bool hb = nb.x >= 0;
            const double* Sa = blk + (int64_t)na.x * 81;
            const double* Sb = blk + (int64_t)(hb ? nb.x : na.x) * 81;
            const double* xa = x + (int64_t)(na.y >> 1) * 9;
            const double* xb = x + (int64_t)((hb ? nb.y : na.y) >> 1) * 9;
            const int sa_row = (na.y & 1) ? 1 : 9, sa_col = (na.y & 1) ? 9 : 1;
            const int sb_row = (nb.y & 1) ? 1 : 9, sb_col = (nb.y & 1) ? 9 : 1;
            double va[9], vb[9], ya[9], yb[9];
#pragma unroll
            for (int c = 0; c < 9; ++c) {
                va[c] = Sa[comp * sa_row + c * sa_col];
                vb[c] = Sb[comp * sb_row + c * sb_col];
                ya[c] = xa[c];
                yb[c] = xb[c];
            }
#pragma unroll
            for (int c = 0; c < 9; ++c) acc += va[c] * ya[c];
            if (hb) {
#pragma unroll
                for (int c = 0; c < 9; ++c) acc += vb[c] * yb[c];
            }
        }
    }
    sacc[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x < 9) {
        double v = 0.0;
        for (int g = 0; g < GRP; ++g) v += sacc[g * 9 + threadIdx.x];
        sacc[BS + threadIdx.x] = v;
    }
    __syncthreads();
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
    double rz = rv * zv, rr = rv * rv;
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        rz += __shfl_xor(rz, off, kWave);
        rr += __shfl_xor(rr, off, kWave);
    }
    if ((threadIdx.x % kWave) == 0) {
        const int w = blockIdx.x * (BS / kWave) + threadIdx.x / kWave;
        pB[2 * w] = rz;
        pB[2 * w + 1] = rr;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) { state[0] = 0; state[1] = 0; state[2] = BA_OK; state[3] = 0; scal[1] = -1.0; }
}

// plain y = S x
__global__ __launch_bounds__(BS) void k_spmv(int ent_stride, const int2* __restrict__ ent, const double* __restrict__ blk,
                                             const double* __restrict__ x, double* __restrict__ y) {
    __shared__ double sacc[BS + 16];
    row_product(blockIdx.x, ent_stride, ent, blk, x, sacc);
    if (threadIdx.x < 9) y[(int64_t)blockIdx.x * 9 + threadIdx.x] = sacc[BS + threadIdx.x];
}

// kernel A; FIRST: the iteration k = 0 (records |r0|^2, d = z, q = S z).
// The block product, the partials of both parities and the state are all
// loaded before any decision, so the kernel is two dependent memory round
// trips (entries, then blocks and z).
template <bool FIRST>
__global__ __launch_bounds__(BS) void k_pcg_A(int ent_stride, const int2* __restrict__ ent,
                                              const double* __restrict__ blk, const double* __restrict__ z,
                                              double* __restrict__ d, double* __restrict__ q, double* __restrict__ pA,
                                              const double* __restrict__ pB0, const double* __restrict__ pB1, int nB,
                                              int* __restrict__ state, double* __restrict__ scal, double tol,
                                              int max_iter) {
    __shared__ double sh[4 * (BS / kWave)];
    __shared__ double sacc[BS + 16];
    const int row = blockIdx.x;
    const int done = state[0];
    const int k = state[3];
    double zv = 0.0, qo = 0.0, dold = 0.0;
    const int64_t o = (int64_t)row * 9 + (threadIdx.x < 9 ? threadIdx.x : 0);
    if (threadIdx.x < 9) {
        zv = z[o];
        if (!FIRST) { qo = q[o]; dold = d[o]; }
    }
    // rz, rr of both parities (pB0: even steps, pB1: odd steps), requested
    // before the product so that they arrive with its first round trip
    double ps[4] = {0.0, 0.0, 0.0, 0.0};
    for (int i = threadIdx.x; i < nB; i += BS) {
        const double2 a = reinterpret_cast<const double2*>(pB0)[i];
        ps[0] += a.x; ps[1] += a.y;
        if (!FIRST) {
            const double2 b = reinterpret_cast<const double2*>(pB1)[i];
            ps[2] += b.x; ps[3] += b.y;
        }
    }
    row_product(row, ent_stride, ent, blk, z, sacc);
    double s[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const double v = wave_sum(ps[j]);
        if ((threadIdx.x % kWave) == 0) sh[j * (BS / kWave) + threadIdx.x / kWave] = v;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < BS / kWave; ++w) t += sh[j * (BS / kWave) + w];
        s[j] = t;
    }
    if (done) return;
    const double rz = (k & 1) ? s[2] : s[0];
    const double rr = (k & 1) ? s[3] : s[1];
    const double rz_old = (k & 1) ? s[0] : s[2];
    const double r0sq = FIRST ? rr : scal[0];
    if (FIRST && row == 0 && threadIdx.x == 0) scal[0] = rr;
    const bool conv = (rr == 0.0) || (sqrt(rr) <= tol * sqrt(r0sq));
    if (conv || k >= max_iter) {
        if (row == 0 && threadIdx.x == 0) {
            state[0] = 1;
            state[2] = conv ? BA_OK : BA_ERR_NOT_CONVERGED;
            scal[1] = r0sq > 0.0 ? sqrt(rr / r0sq) : 0.0;
        }
        return;
    }
    const double beta = FIRST ? 0.0 : rz / rz_old;
    if (row == 0 && threadIdx.x == 0) state[1] = k;
    if (threadIdx.x < 9) {
        const double sv = sacc[BS + threadIdx.x];
        const double qv = FIRST ? sv : sv + beta * qo;
        const double dv = FIRST ? zv : zv + beta * dold;
        q[o] = qv;
        d[o] = dv;
        double dq = dv * qv;
        // sum of the 9 components held by lanes 0..8
#pragma unroll
        for (int off = 8; off > 0; off >>= 1) {
            const double o2 = __shfl_down(dq, off, 16);
            if (threadIdx.x + off < 9) dq += o2;
        }
        if (threadIdx.x == 0) pA[row] = dq;
    }
}

__global__ __launch_bounds__(BS) void k_pcg_B(int n_rows, const double* __restrict__ M, const double* __restrict__ d,
                                              const double* __restrict__ q, double* __restrict__ x,
                                              double* __restrict__ r, double* __restrict__ z,
                                              const double* __restrict__ pA, int nA, double* __restrict__ pB0,
                                              double* __restrict__ pB1, int nB, int* __restrict__ state) {
    __shared__ double sh[3 * (BS / kWave)];
    __shared__ double sr[RPB][9];
    const int done = state[0];
    const int k = state[1];
    const int lr = threadIdx.x / 9, i = threadIdx.x % 9;
    const int row = blockIdx.x * RPB + lr;
    const bool act = threadIdx.x < RPB * 9 && row < n_rows;
    double Mr[9], dv = 0.0, qv = 0.0, xv = 0.0, rv0 = 0.0;
    const int64_t o = (int64_t)row * 9 + i;
    if (act) {
        const double* Mp = M + (int64_t)row * 81 + i * 9;
#pragma unroll
        for (int c = 0; c < 9; ++c) Mr[c] = Mp[c];
        dv = d[o]; qv = q[o]; xv = x[o]; rv0 = r[o];
    }
    const double* src[3] = {pA, pB0, pB1};
    const int n[3] = {nA, nB, nB};
    const int stride[3] = {1, 2, 2};
    double s[3];
    sum_partials<3>(src, n, stride, s, sh);
    if (done) return;
    const double dq = s[0], rz = (k & 1) ? s[2] : s[1];
    double* pk1 = (k & 1) ? pB0 : pB1;
    if (!(dq > 0.0)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) { state[0] = 1; state[2] = BA_ERR_NOT_SPD; }
        return;
    }
    const double alpha = rz / dq;
    double rv = 0.0;
    if (act) {
        x[o] = xv + alpha * dv;
        rv = rv0 - alpha * qv;
        r[o] = rv;
        sr[lr][i] = rv;
    }
    __syncthreads();
    double zv = 0.0;
    if (act) {
#pragma unroll
        for (int c = 0; c < 9; ++c) zv += Mr[c] * sr[lr][c];
        z[o] = zv;
    }
    // per-wave partials of r^T z and r^T r (4 per block)
    double rzn = rv * zv, rr = rv * rv;
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        rzn += __shfl_xor(rzn, off, kWave);
        rr += __shfl_xor(rr, off, kWave);
    }
    if ((threadIdx.x % kWave) == 0) {
        const int w = blockIdx.x * (BS / kWave) + threadIdx.x / kWave;
        pk1[2 * w] = rzn;
        pk1[2 * w + 1] = rr;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) state[3] = k + 1;
}

void enqueue_iterations(ba_ctx* c, const double* M, double tol, int max_iter, int count, hipStream_t st) {
    Pcg& P = c->pcg;
    const int nr = c->n_rows, nB = (nr + RPB - 1) / RPB, nPB = nB * (BS / kWave);
    for (int i = 0; i < count; ++i) {
        k_pcg_A<false><<<nr, BS, 0, st>>>(c->ent_stride, (const int2*)c->sp_ent, c->blk, P.z, P.d[0], P.q, P.pA,
                                          P.pB[0], P.pB[1], nPB, P.state, P.scal, tol, max_iter);
        k_pcg_B<<<nB, BS, 0, st>>>(nr, M, P.d[0], P.q, P.x, P.r, P.z, P.pA, nr, P.pB[0], P.pB[1], nPB, P.state);
    }
}

}  // namespace

ba_status run_pcg(ba_ctx* c, const double* M, double tol, int max_iter, const double* x0, double* out, int* iters,
                  double* relres) {
    Pcg& P = c->pcg;
    const int nr = c->n_rows;
    const int nB = (nr + RPB - 1) / RPB, nPB = nB * (BS / kWave);
    hipStream_t st = c->stream;
    const double* q0 = nullptr;
    if (x0) {
        k_spmv<<<nr, BS, 0, st>>>(c->ent_stride, (const int2*)c->sp_ent, c->blk, x0, P.q);
        q0 = P.q;
    }
    k_pcg_init<<<nB, BS, 0, st>>>(nr, c->rhs, q0, x0, M, P.x, P.r, P.z, P.pB[0], P.state, P.scal);
    k_pcg_A<true><<<nr, BS, 0, st>>>(c->ent_stride, (const int2*)c->sp_ent, c->blk, P.z, P.d[0], P.q, P.pA, P.pB[0],
                                     P.pB[1], nPB, P.state, P.scal, tol, max_iter);
    if (max_iter > 0)
        k_pcg_B<<<nB, BS, 0, st>>>(nr, M, P.d[0], P.q, P.x, P.r, P.z, P.pA, nr, P.pB[0], P.pB[1], nPB, P.state);
    // remaining iterations in fixed batches (a captured graph when possible);
    // the stop flag of a batch is read back while the next batch runs, and
    // kernels after the stop return at once
    const int batch = kPcgBatch;
    const int n_batches = max_iter > 0 ? (max_iter + batch - 1) / batch : 0;
    hipGraphExec_t exec = nullptr;
    if (c->use_graphs && n_batches > 0) {
        for (auto& g : c->pcg_graphs)
            if (g.M == M && g.tol == tol && g.max_iter == max_iter) exec = g.exec;
        if (!exec) {
            hipStream_t cs = c->capture_stream;
            hipGraph_t graph = nullptr;
            BA_HIP_CHECK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
            enqueue_iterations(c, M, tol, max_iter, batch, cs);
            BA_HIP_CHECK(hipStreamEndCapture(cs, &graph));
            BA_HIP_CHECK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
            BA_HIP_CHECK(hipGraphDestroy(graph));
            c->pcg_graphs.push_back({M, tol, max_iter, exec});
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
                enqueue_iterations(c, M, tol, max_iter, batch, st);
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

void launch_spmv(ba_ctx* c, const double* x, double* y) {
    if (c->n_rows == 0) return;
    k_spmv<<<c->n_rows, BS, 0, c->stream>>>(c->ent_stride, (const int2*)c->sp_ent, c->blk, x, y);
}

}  // namespace ba
