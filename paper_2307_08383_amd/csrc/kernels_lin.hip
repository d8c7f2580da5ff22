// Per-observation kernels: projection, linearization (residual + Jacobian
// blocks, Sec. 3.1), candidate-cost / model evaluation and the parameter
// update of an accepted LM step.  One lane per observation, observations in
// the context's (point, camera) order so that point reads stream.
#include <algorithm>

#include "ba_common.hpp"

namespace ba {

namespace {

constexpr int BS = 256;

__global__ __launch_bounds__(BS) void k_project(int64_t n, const double* __restrict__ cams, const double* __restrict__ pts,
                                                const int32_t* __restrict__ obs_cam, const int32_t* __restrict__ obs_pt,
                                                const double* __restrict__ noise, double* __restrict__ uv) {
    const int64_t k = (int64_t)blockIdx.x * BS + threadIdx.x;
    if (k >= n) return;
    const double* X = pts + (int64_t)obs_pt[k] * 3;
    double pu, pv;
    project_point<false>(cams + (int64_t)obs_cam[k] * 9, X[0], X[1], X[2], pu, pv, nullptr, nullptr);
    if (noise) { pu += noise[k]; pv += noise[n + k]; }
    uv[k] = pu;
    uv[n + k] = pv;
}

template <typename T>
__global__ __launch_bounds__(BS) void k_linearize(int n, const int32_t* __restrict__ obs_cam, const int32_t* __restrict__ obs_pt,
                                                  const double* __restrict__ uv, const double* __restrict__ cams,
                                                  const double* __restrict__ pts, T* __restrict__ R, T* __restrict__ Jp_out,
                                                  double* __restrict__ e, double* __restrict__ part,
                                                  int* __restrict__ flags) {
    __shared__ double sh[BS / kWave];
    const int k = blockIdx.x * BS + threadIdx.x;
    double cost = 0.0;
    if (k < n) {
        const double* X = pts + (int64_t)obs_pt[k] * 3;
        double pu, pv, Jc[18], Jp[6];
        project_point<true>(cams + (int64_t)obs_cam[k] * 9, X[0], X[1], X[2], pu, pv, Jc, Jp);
        const double eu = pu - uv[k], ev = pv - uv[n + k];
        if (!records_in_range<T>(Jc, Jp, eu, ev)) flags[2] = 1;
        store_jc(R + (int64_t)k * kRec, Jc);
        store6(Jp_out + (int64_t)k * 6, Jp);
        reinterpret_cast<double2*>(e)[k] = make_double2(eu, ev);
        cost = 0.5 * (eu * eu + ev * ev);
    }
    const double s = block_sum<BS>(cost, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// F' at x + dx (the model terms of the gain ratio come with
// back-substitution)
__global__ __launch_bounds__(BS) void k_evaluate(int n, const int32_t* __restrict__ obs_cam, const int32_t* __restrict__ obs_pt,
                                                 const int32_t* __restrict__ obs_row, const double* __restrict__ uv,
                                                 const double* __restrict__ cams, const double* __restrict__ pts,
                                                 const double* __restrict__ dxc, const double* __restrict__ dxp,
                                                 double* __restrict__ part) {
    __shared__ double sh[BS / kWave];
    const int k = xcd_block() * BS + threadIdx.x;
    double cost = 0.0;
    if (k < n) {
        const int row = obs_row[k];
        const int p = obs_pt[k];
        const double* c0 = cams + (int64_t)obs_cam[k] * 9;
        double c[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) c[i] = c0[i] + (row >= 0 ? dxc[(int64_t)row * 9 + i] : 0.0);
        const double* X = pts + (int64_t)p * 3;
        const double* dX = dxp + (int64_t)p * 3;
        double pu, pv;
        project_point<false>(c, X[0] + dX[0], X[1] + dX[1], X[2] + dX[2], pu, pv, nullptr, nullptr);
        const double eu = pu - uv[k], ev = pv - uv[n + k];
        cost = 0.5 * (eu * eu + ev * ev);
    }
    const double s0 = block_sum<BS>(cost, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s0;
}

// J_p = K L^T of every observation into Jp (for the getter, after the fused
// linearize + point stage): one wave per chunk of whole tracks
template <typename T>
__global__ __launch_bounds__(BS) void k_jp_from_K(int n_chunk, const int32_t* __restrict__ chunk_ptr,
                                                  const int32_t* __restrict__ chunk_q, const int32_t* __restrict__ obs_pt,
                                                  const T* __restrict__ R, const double* __restrict__ ptL,
                                                  T* __restrict__ Jp) {
    const int wv = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int chunk = blockIdx.x * (BS / kWave) + wv;
    int k0 = 0, k1 = 0;
    if (chunk < n_chunk) { k0 = chunk_ptr[chunk]; k1 = chunk_ptr[chunk + 1]; }
    const int k = k0 + lane;
    const bool act = k < k1;
    const int p = act ? obs_pt[k] : -1;
    const Track tk = chunk_track(act, p, lane, k1 - k0);
    const int64_t q = chunk < n_chunk ? (int64_t)chunk_q[chunk] + tk.idx : 0;
    if (act) {
        double K[6], jp[6];
        load6(R + (int64_t)k * kRec + 18, K);
        jp_from_K(K, ptL + q * 9, jp);
        store6(Jp + (int64_t)k * 6, jp);
    }
}

// point ids and pixels of the caller's observations in the internal order
// (perm: internal position -> caller's index); *bad = the lowest caller's
// index whose pixel is not finite (unchanged if none)
__global__ __launch_bounds__(BS) void k_gather_obs(int64_t n, const int32_t* __restrict__ perm,
                                                   const int32_t* __restrict__ pt_in,
                                                   const double* __restrict__ uv_in, int32_t* __restrict__ pt,
                                                   double* __restrict__ uv, unsigned long long* __restrict__ bad) {
    const int64_t k = (int64_t)blockIdx.x * BS + threadIdx.x;
    if (k >= n) return;
    const int64_t s = perm[k];
    const double u = uv_in[s], v = uv_in[n + s];
    pt[k] = pt_in[s];
    uv[k] = u;
    uv[n + k] = v;
    if (!isfinite(u) || !isfinite(v)) atomicMin(bad, (unsigned long long)s);
}

// the same for the tracks longer than a wave: one workgroup per point
template <typename T>
__global__ __launch_bounds__(BS) void k_jp_from_K_long(int q0, const int32_t* __restrict__ long_ptr,
                                                       const T* __restrict__ R, const double* __restrict__ ptL,
                                                       T* __restrict__ Jp) {
    const int k0 = long_ptr[blockIdx.x], k1 = long_ptr[blockIdx.x + 1];
    const double* L = ptL + ((int64_t)q0 + blockIdx.x) * 9;
    for (int k = k0 + threadIdx.x; k < k1; k += BS) {
        double K[6], jp[6];
        load6(R + (int64_t)k * kRec + 18, K);
        jp_from_K(K, L, jp);
        store6(Jp + (int64_t)k * 6, jp);
    }
}

// out[j * ostride + b] = sum of part[j*n + b*chunk .. j*n + min(n, (b+1)*chunk))
// in a fixed order (block (b, j); b = 0 with chunk >= n sums the whole
// vector)
__global__ __launch_bounds__(BS) void k_reduce(const double* __restrict__ part, int n, int chunk,
                                               double* __restrict__ out, int ostride) {
    __shared__ double sh[BS / kWave];
    const int j = blockIdx.y, b = blockIdx.x;
    const double* p = part + (int64_t)j * n;
    const int lo = b * chunk, hi = min(n, lo + chunk);
    double s = 0.0;
    for (int i = lo + threadIdx.x; i < hi; i += BS) s += p[i];
    s = block_sum<BS>(s, sh);
    if (threadIdx.x == 0) out[(int64_t)j * ostride + b] = s;
}

__global__ __launch_bounds__(BS) void k_update(int n_cams, int n_pts, const int32_t* __restrict__ cam_row,
                                               double* __restrict__ cams, double* __restrict__ pts,
                                               const double* __restrict__ dxc, const double* __restrict__ dxp) {
    const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
    if (i < (int64_t)n_cams * 9) {
        const int c = (int)(i / 9), j = (int)(i % 9);
        const int r = cam_row[c];
        if (r >= 0) cams[i] += dxc[(int64_t)r * 9 + j];
    }
    if (i < (int64_t)n_pts * 3) pts[i] += dxp[i];
}

inline int nblk(int64_t n) { return (int)((n + BS - 1) / BS); }

}  // namespace

void launch_project(const double* cams, const double* pts, const int32_t* obs_cam, const int32_t* obs_pt,
                    int64_t n_obs, const double* noise, double* uv, hipStream_t st) {
    if (n_obs <= 0) return;
    k_project<<<nblk(n_obs), BS, 0, st>>>(n_obs, cams, pts, obs_cam, obs_pt, noise, uv);
}

void launch_linearize(ba_ctx* c, const double* cams, const double* pts) {
    const int n = (int)c->n_obs, nb = nblk(n);
    if (c->precision == BA_MIXED)
        k_linearize<float><<<nb, BS, 0, c->stream>>>(n, c->obs_cam, c->obs_pt, c->obs_uv, cams, pts,
                                                     (float*)c->R, (float*)c->Jp, c->e, c->part, c->flags);
    else
        k_linearize<double><<<nb, BS, 0, c->stream>>>(n, c->obs_cam, c->obs_pt, c->obs_uv, cams, pts,
                                                      (double*)c->R, (double*)c->Jp, c->e, c->part, c->flags);
    launch_reduce(c, c->part, nb, 1, c->scal + 0);
    c->jp_valid = true;
}

// out[j] = sum of part[j*n .. j*n + n), j < count (count <= 3), in a fixed
// order: long vectors in two passes (up to kReduceParts contiguous pieces
// summed by separate blocks into c->part2, then the pieces in order), so
// that the sum is not left to a single block
void launch_reduce(ba_ctx* c, const double* part, int n, int count, double* out) {
    constexpr int kPiece = 2048;
    if (n <= 2 * kPiece) {
        k_reduce<<<dim3(1, count), BS, 0, c->stream>>>(part, n, n, out, 1);
        return;
    }
    const int pieces = std::min(kReduceParts, (n + kPiece - 1) / kPiece);
    const int chunk = (n + pieces - 1) / pieces;
    k_reduce<<<dim3(pieces, count), BS, 0, c->stream>>>(part, n, chunk, c->part2, kReduceParts);
    k_reduce<<<dim3(1, count), BS, 0, c->stream>>>(c->part2, kReduceParts, pieces, out, 1);
}

void launch_evaluate(ba_ctx* c, const double* cams, const double* pts, const double* dxc, const double* dxp) {
    const int n = (int)c->n_obs, nb = nblk(n);
    k_evaluate<<<nb, BS, 0, c->stream>>>(n, c->obs_cam, c->obs_pt, c->obs_row, c->obs_uv, cams, pts, dxc, dxp,
                                         c->part);
    launch_reduce(c, c->part, nb, 1, c->scal + 1);   // scal[1] F'
}

void launch_gather_obs(ba_ctx* c, const int32_t* perm, const int32_t* pt_in, const double* uv_in,
                       unsigned long long* bad) {
    const int64_t n = c->n_obs;
    k_gather_obs<<<(unsigned)((n + BS - 1) / BS), BS, 0, c->stream>>>(n, perm, pt_in, uv_in, c->obs_pt, c->obs_uv, bad);
    BA_HIP_CHECK(hipGetLastError());
}

void ensure_jp(ba_ctx* c) {
    if (c->jp_valid) return;
    const int nb = (c->n_chunk + BS / kWave - 1) / (BS / kWave);
    if (nb > 0) {
        if (c->precision == BA_MIXED)
            k_jp_from_K<float><<<nb, BS, 0, c->stream>>>(c->n_chunk, c->chunk_ptr, c->chunk_q, c->obs_pt,
                                                         (const float*)c->R, c->ptL, (float*)c->Jp);
        else
            k_jp_from_K<double><<<nb, BS, 0, c->stream>>>(c->n_chunk, c->chunk_ptr, c->chunk_q, c->obs_pt,
                                                          (const double*)c->R, c->ptL, (double*)c->Jp);
    }
    if (c->n_long > 0) {
        if (c->precision == BA_MIXED)
            k_jp_from_K_long<float><<<c->n_long, BS, 0, c->stream>>>(c->q_long0, c->long_ptr, (const float*)c->R,
                                                                     c->ptL, (float*)c->Jp);
        else
            k_jp_from_K_long<double><<<c->n_long, BS, 0, c->stream>>>(c->q_long0, c->long_ptr, (const double*)c->R,
                                                                      c->ptL, (double*)c->Jp);
    }
    c->jp_valid = true;
}

void launch_update(ba_ctx* c, double* cams, double* pts, const double* dxc, const double* dxp) {
    const int64_t n = std::max<int64_t>((int64_t)c->n_cams * 9, (int64_t)c->n_pts * 3);
    k_update<<<nblk(n), BS, 0, c->stream>>>(c->n_cams, c->n_pts, c->cam_row, cams, pts, dxc, dxp);
}

}  // namespace ba
