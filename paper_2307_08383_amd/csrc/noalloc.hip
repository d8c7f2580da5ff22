// The cost of Sec. 3.1 Eq. (1), F = 1/2 sum |e|^2, for callers that cannot
// allocate device memory (code under HIP graph capture, serving loops): the
// value ba_linearize returns, without a context.  The per-block partial
// sums live in a file-scope device buffer that every call on a GPU shares
// (each GPU holds its own copy until the process ends).
#include <mutex>

#include "ba_common.hpp"

namespace {

constexpr int BS = 256;
constexpr int kObsPerBlock = 1024;                       // observations summed by one block
constexpr int kMaxBlocks = 131072;                       // partial sums held: 1 MiB
constexpr int64_t kMaxObs = (int64_t)kObsPerBlock * kMaxBlocks;

static __device__ __align__(256) double scratch[kMaxBlocks];

// per-device address of `scratch` (the host-side name is not a device address)
std::mutex g_mu;
double* g_scratch[64] = {};

double* scratch_ptr(int dev) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
        g_scratch[dev] = static_cast<double*>(p);
    }
    return g_scratch[dev];
}

// block b sums the costs of observations [b * 1024, (b + 1) * 1024) in a
// fixed order (four per thread, then the block's shuffle tree)
__global__ __launch_bounds__(BS) void k_cost_part(int64_t n, const double* __restrict__ cams,
                                                  const double* __restrict__ pts, const int32_t* __restrict__ obs_cam,
                                                  const int32_t* __restrict__ obs_pt, const double* __restrict__ uv,
                                                  double* __restrict__ part) {
    __shared__ double sh[BS / ba::kWave];
    double s = 0.0;
    const int64_t k0 = (int64_t)blockIdx.x * kObsPerBlock;
    for (int j = 0; j < kObsPerBlock / BS; ++j) {
        const int64_t k = k0 + j * BS + threadIdx.x;
        if (k < n) {
            const double* X = pts + (int64_t)obs_pt[k] * 3;
            double pu, pv;
            ba::project_point<false>(cams + (int64_t)obs_cam[k] * 9, X[0], X[1], X[2], pu, pv, nullptr, nullptr);
            const double eu = pu - uv[k], ev = pv - uv[n + k];
            s += 0.5 * (eu * eu + ev * ev);
        }
    }
    s = ba::block_sum<BS>(s, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// out = sum of part[0 .. nb) in a fixed order (one block)
__global__ __launch_bounds__(1024) void k_cost_total(int nb, const double* __restrict__ part, double* __restrict__ out) {
    __shared__ double sh[1024 / ba::kWave];
    double s = 0.0;
    for (int i = threadIdx.x; i < nb; i += 1024) s += part[i];
    s = ba::block_sum<1024>(s, sh);
    if (threadIdx.x == 0) *out = s;
}

}  // namespace

extern "C" ba_status ba_cost_noalloc(const double* cams, const double* pts, const int32_t* obs_cam,
                                     const int32_t* obs_pt, const double* uv, int64_t n_obs, double* cost,
                                     void* stream) {
    if (n_obs < 0 || n_obs > kMaxObs || !cost) return BA_ERR_INVALID_ARG;
    if (n_obs > 0 && (!cams || !pts || !obs_cam || !obs_pt || !uv)) return BA_ERR_INVALID_ARG;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return BA_ERR_DEVICE;
    double* part = scratch_ptr(dev);
    if (!part) return BA_ERR_DEVICE;
    const hipStream_t st = (hipStream_t)stream;
    const int nb = (int)((n_obs + kObsPerBlock - 1) / kObsPerBlock);
    if (nb > 0)
        k_cost_part<<<nb, BS, 0, st>>>(n_obs, cams, pts, obs_cam, obs_pt, uv, part);
    k_cost_total<<<1, 1024, 0, st>>>(nb, part, cost);
    return hipGetLastError() == hipSuccess ? BA_OK : BA_ERR_DEVICE;
}
