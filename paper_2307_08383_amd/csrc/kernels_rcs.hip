// Reduced-camera-system formation (Eq. (3)-(4), Sec. 5) and point
// back-substitution (Eq. (5)).
//
// With V*_p = L_p L_p^T (3x3 Cholesky) and K_a = J_pa L_p^-T (2x3) for an
// observation a of point p by camera i:
//   W_ip V*_p^-1 W_jp^T = J_ca^T (K_a K_b^T) J_cb          (camera pair i, j)
//   U_i - sum_p W_ip V*_p^-1 W_ip^T = sum_a J_ca^T (I - K_a K_a^T) J_ca
//   b_i = l_c - W V*^-1 l_p = -sum_a J_ca^T (e_a + K_a lhat_p),  lhat_p = L_p^-1 l_p
//   dx_p = L_p^-T (lhat_p - sum_a K_a^T J_ca dx_c)          (Eq. (5))
// so the point stage only adds K (6 values) to each observation's J_c record
// and every later stage reads one 24-value record per observation.  The
// off-diagonal blocks are segmented reductions over the observation couples
// of each camera pair (sorted once, no atomics); the diagonal blocks are
// reductions over each camera's observations.
#include <type_traits>

#include "ba_common.hpp"

namespace ba {

namespace {

constexpr int BS = 256;
constexpr int WPB = BS / kWave;   // waves per block

// Point terms from the track sums s = (V: 00 01 02 11 12 22, l_p): the
// Cholesky factor of V* = V + lambda diag(V), lhat = L^-1 l_p and the
// reciprocals of L's diagonal, r = (L00, L10, L11, L20, L21, L22, lhat,
// 1/L00, 1/L11, 1/L22).  Returns false if V* is not positive definite.
constexpr int kPT = 12;   // point terms shared with a track's lanes
__device__ __forceinline__ bool point_terms(const double* s, double lambda, double* r) {
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

// K = J_p L^-T from the point terms r: row r of K solves L y = J_p[r]^T.
__device__ __forceinline__ void point_K(const double* r, const double* jp, double* K) {
    const double L10 = r[1], L20 = r[3], L21 = r[4], i00 = r[9], i11 = r[10], i22 = r[11];
#pragma unroll
    for (int rr = 0; rr < 2; ++rr) {
        const double y0 = jp[3 * rr] * i00;
        const double y1 = (jp[3 * rr + 1] - L10 * y0) * i11;
        const double y2 = (jp[3 * rr + 2] - L20 * y0 - L21 * y1) * i22;
        K[3 * rr] = y0; K[3 * rr + 1] = y1; K[3 * rr + 2] = y2;
    }
}

// ebar = e + K lhat, with K as stored (T), at the observation's position in
// its camera's list (rpos < 0: fixed camera, no RCS row).  The diagonal
// stage reads it in that order instead of gathering e and lhat.
template <typename T>
__device__ __forceinline__ void store_ebar(const double* r, const double* K, double eu, double ev, int rpos,
                                           double* __restrict__ ebar) {
    if (rpos < 0) return;
    double Kt[6];
#pragma unroll
    for (int m = 0; m < 6; ++m) Kt[m] = (double)(T)K[m];
    const double v0 = eu + Kt[0] * r[6] + Kt[1] * r[7] + Kt[2] * r[8];
    const double v1 = ev + Kt[3] * r[6] + Kt[4] * r[7] + Kt[5] * r[8];
    reinterpret_cast<double2*>(ebar)[rpos] = make_double2(v0, v1);
}

// ---------------------------------------------------------------------------
// point stage: one wave per chunk of whole tracks (<= 64 observations), one
// lane per observation.  Track sums V_p, l_p are reduced through LDS by the
// lane holding the first observation of the track.
// ---------------------------------------------------------------------------
// FROM_K: J_p is not stored; it is formed as K L^T from the record and the
// point terms of the previous formation (read before they are replaced),
// rounded to T and stored in Jp, so that later formations of the same
// linearization read it instead of forming it again.
template <typename T, bool FROM_K = false>
__global__ __launch_bounds__(BS) void k_point(int n_chunk, const int32_t* __restrict__ chunk_ptr,
                                              const int32_t* __restrict__ obs_pt, const int32_t* __restrict__ chunk_q,
                                              T* __restrict__ R, T* __restrict__ Jp, const double* __restrict__ e,
                                              double lambda, double* __restrict__ ptL, const int32_t* __restrict__ obs_rpos,
                                              double* __restrict__ ebar, int* __restrict__ flags) {
    __shared__ double sP[WPB][kWave][kPT];   // track sums, then the head's point terms
    const int wv = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int chunk = blockIdx.x * WPB + wv;
    int k0 = 0, k1 = 0;
    if (chunk < n_chunk) { k0 = chunk_ptr[chunk]; k1 = chunk_ptr[chunk + 1]; }
    const int k = k0 + lane;
    const bool act = k < k1;
    double jp[6];
    double2 ek = make_double2(0.0, 0.0);
    const int p = act ? obs_pt[k] : -1;
    const Track tk = chunk_track(act, p, lane, k1 - k0);
    const int head = tk.head, tl = tk.len;
    const int64_t q = chunk < n_chunk ? (int64_t)chunk_q[chunk] + tk.idx : 0;   // internal point index
    if (act) {
        if (FROM_K) {
            double K[6];
            load6(R + (int64_t)k * kRec + 18, K);
            jp_from_K(K, ptL + q * 9, jp);
#pragma unroll
            for (int m = 0; m < 6; ++m) jp[m] = (double)(T)jp[m];
            store6(Jp + (int64_t)k * 6, jp);
        } else {
            load6(Jp + (int64_t)k * 6, jp);
        }
        ek = reinterpret_cast<const double2*>(e)[k];
        sP[wv][lane][0] = jp[0] * jp[0] + jp[3] * jp[3];
        sP[wv][lane][1] = jp[0] * jp[1] + jp[3] * jp[4];
        sP[wv][lane][2] = jp[0] * jp[2] + jp[3] * jp[5];
        sP[wv][lane][3] = jp[1] * jp[1] + jp[4] * jp[4];
        sP[wv][lane][4] = jp[1] * jp[2] + jp[4] * jp[5];
        sP[wv][lane][5] = jp[2] * jp[2] + jp[5] * jp[5];
        sP[wv][lane][6] = -(jp[0] * ek.x + jp[3] * ek.y);
        sP[wv][lane][7] = -(jp[1] * ek.x + jp[4] * ek.y);
        sP[wv][lane][8] = -(jp[2] * ek.x + jp[5] * ek.y);
    }
    __syncthreads();
    if (act && head == lane) {
        double s[9];
#pragma unroll
        for (int m = 0; m < 9; ++m) s[m] = 0.0;
        for (int q = 0; q < tl; ++q)
#pragma unroll
            for (int m = 0; m < 9; ++m) s[m] += sP[wv][lane + q][m];
        double r[kPT];
        if (!point_terms(s, lambda, r)) flags[0] = 1;
        // the head's own row is read by no other lane: it holds the track's terms now
#pragma unroll
        for (int m = 0; m < kPT; ++m) sP[wv][lane][m] = r[m];
#pragma unroll
        for (int m = 0; m < 9; ++m) ptL[q * 9 + m] = r[m];
    }
    __syncthreads();
    if (act) {
        double K[6];
        point_K(sP[wv][head], jp, K);
        store6(R + (int64_t)k * kRec + 18, K);
        store_ebar<T>(sP[wv][head], K, ek.x, ek.y, obs_rpos[k], ebar);
    }
}

// n_bytes (a multiple of CH) from LDS to global memory, contiguous CH-byte
// chunks spread over the wave's lanes (one fully used cache line per few
// lanes per instruction)
template <int CH>
__device__ __forceinline__ void wave_copy_out(char* __restrict__ dst, const char* src, int n_bytes, int lane) {
    using V = typename std::conditional<CH == 16, uint4, uint2>::type;
    for (int o = lane * CH; o < n_bytes; o += kWave * CH)
        *reinterpret_cast<V*>(dst + o) = *reinterpret_cast<const V*>(src + o);
}

// ---------------------------------------------------------------------------
// linearization fused with the point stage (the LM step after an accepted
// step): one wave per chunk of whole tracks, one lane per observation.  Each
// lane forms its residual and Jacobian blocks (Eq. (1)); J_c and J_p are
// rounded to T first, so the records, point terms and e + K lhat equal
// those of k_linearize followed by k_point.  J_p itself is not stored: it
// is K L^T wherever it is needed.  The track sums go through LDS as in
// k_point, and the records are written whole through LDS (below).
// ---------------------------------------------------------------------------
// Waves per workgroup of the fused stage: one, so that its barriers hold a
// single wave (on the 60,000-camera partition, FP64, measured against four
// waves on the same GPU: 7.01 against 7.29 ms, and 7.82 against 7.97 ms on
// another; two waves 7.09 ms).  Its chunks go to the XCDs in contiguous
// ranges (7.56 against 7.80 ms): a chunk boundary splits lines of the
// observation arrays, which the neighbouring chunk then finds in L2.
constexpr int kLinNW = 1;

template <typename T, int NW>
__device__ __forceinline__ void linpoint(int n_chunk, const int32_t* __restrict__ chunk_ptr, int n,
                                                 const int32_t* __restrict__ obs_cam,
                                                 const int32_t* __restrict__ obs_pt,
                                                 const int32_t* __restrict__ chunk_q, const double* __restrict__ uv,
                                                 const double* __restrict__ cams, const double* __restrict__ pts,
                                                 double lambda, T* __restrict__ R,
                                                 double* __restrict__ e, double* __restrict__ ptL,
                                                 const int32_t* __restrict__ obs_rpos, double* __restrict__ ebar,
                                                 double* __restrict__ part, int* __restrict__ flags) {
    __shared__ __align__(16) double sP[NW][kWave][kPT];   // track sums, the head's point terms, then staging
    __shared__ double sh[NW];
    const int wv = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int chunk = xcd_block() * NW + wv;   // neighbouring chunks on one XCD
    int k0 = 0, k1 = 0;
    if (chunk < n_chunk) { k0 = chunk_ptr[chunk]; k1 = chunk_ptr[chunk + 1]; }
    const int k = k0 + lane;
    const bool act = k < k1;
    double jc[18], jp[6];
    double cost = 0.0, eu = 0.0, ev = 0.0;
    const int p = act ? obs_pt[k] : -1;
    const Track tk = chunk_track(act, p, lane, k1 - k0);
    const int head = tk.head, tl = tk.len;
    const int64_t q = chunk < n_chunk ? (int64_t)chunk_q[chunk] + tk.idx : 0;   // internal point index
    if (act) {
        const double* X = pts + (int64_t)p * 3;
        double pu, pv;
        project_point<true>(cams + (int64_t)obs_cam[k] * 9, X[0], X[1], X[2], pu, pv, jc, jp);
        eu = pu - uv[k];
        ev = pv - uv[n + k];
        if (!records_in_range<T>(jc, jp, eu, ev)) flags[2] = 1;
#pragma unroll
        for (int m = 0; m < 18; ++m) jc[m] = (double)(T)jc[m];
#pragma unroll
        for (int m = 0; m < 6; ++m) jp[m] = (double)(T)jp[m];
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
    const double csum = block_sum<NW * kWave>(cost, sh);   // contains the barrier for sP
    if (threadIdx.x == 0) part[blockIdx.x] = csum;
    if (act && head == lane) {
        double s[9];
#pragma unroll
        for (int m = 0; m < 9; ++m) s[m] = 0.0;
        for (int q = 0; q < tl; ++q)
#pragma unroll
            for (int m = 0; m < 9; ++m) s[m] += sP[wv][lane + q][m];
        double r[kPT];
        if (!point_terms(s, lambda, r)) flags[0] = 1;
        // the head's own row is read by no other lane: it holds the track's terms now
#pragma unroll
        for (int m = 0; m < kPT; ++m) sP[wv][lane][m] = r[m];
#pragma unroll
        for (int m = 0; m < 9; ++m) ptL[q * 9 + m] = r[m];
    }
    __syncthreads();
    double K[6];
    if (act) {
        point_K(sP[wv][head], jp, K);
        store_ebar<T>(sP[wv][head], K, eu, ev, obs_rpos[k], ebar);
    }
    __syncthreads();   // every lane has its point terms: sP is free for staging
    // The wave's records (J_c, K) are contiguous in memory; they are staged
    // through the wave's 6 KB of sP and written with contiguous 16-byte
    // chunks spread over the lanes, instead of each lane writing its own
    // record at a 192-byte (96-byte) stride.
    char* stage = reinterpret_cast<char*>(&sP[wv][0][0]);
    constexpr int kStageB = kWave * kPT * (int)sizeof(double);
    constexpr int kRecB = kRec * (int)sizeof(T);
    constexpr int kPer = kStageB / kRecB;      // records per round: 32 (FP64), 64 (FP32)
    const int nrec = k1 - k0;
#pragma unroll
    for (int r0 = 0; r0 < kWave; r0 += kPer) {
        if (act && lane >= r0 && lane < r0 + kPer) {
            T* d = reinterpret_cast<T*>(stage + (lane - r0) * kRecB);
            store_jc(d, jc);
            store6(d + 18, K);
        }
        __syncthreads();
        wave_copy_out<16>(reinterpret_cast<char*>(R + (int64_t)(k0 + r0) * kRec), stage,
                          max(0, min(nrec - r0, kPer)) * kRecB, lane);
        __syncthreads();
    }
}

// FP32 records: 96 registers allow five waves per SIMD without spilling;
// the FP64 build keeps the default (it would spill).
__global__ __launch_bounds__(kLinNW * kWave) __attribute__((amdgpu_waves_per_eu(5))) void k_linpoint_f(int n_chunk, const int32_t* __restrict__ chunk_ptr, int n,
                                                 const int32_t* __restrict__ obs_cam,
                                                 const int32_t* __restrict__ obs_pt,
                                                 const int32_t* __restrict__ chunk_q, const double* __restrict__ uv,
                                                 const double* __restrict__ cams, const double* __restrict__ pts,
                                                 double lambda, float* __restrict__ R,
                                                 double* __restrict__ e, double* __restrict__ ptL,
                                                 const int32_t* __restrict__ obs_rpos, double* __restrict__ ebar,
                                                 double* __restrict__ part, int* __restrict__ flags) {
    linpoint<float, kLinNW>(n_chunk, chunk_ptr, n, obs_cam, obs_pt, chunk_q, uv, cams, pts, lambda, R, e, ptL, obs_rpos, ebar, part, flags);
}
__global__ __launch_bounds__(kLinNW * kWave) void k_linpoint_d(int n_chunk, const int32_t* __restrict__ chunk_ptr, int n,
                                                 const int32_t* __restrict__ obs_cam,
                                                 const int32_t* __restrict__ obs_pt,
                                                 const int32_t* __restrict__ chunk_q, const double* __restrict__ uv,
                                                 const double* __restrict__ cams, const double* __restrict__ pts,
                                                 double lambda, double* __restrict__ R,
                                                 double* __restrict__ e, double* __restrict__ ptL,
                                                 const int32_t* __restrict__ obs_rpos, double* __restrict__ ebar,
                                                 double* __restrict__ part, int* __restrict__ flags) {
    linpoint<double, kLinNW>(n_chunk, chunk_ptr, n, obs_cam, obs_pt, chunk_q, uv, cams, pts, lambda, R, e, ptL, obs_rpos, ebar, part, flags);
}

// ---------------------------------------------------------------------------
// off-diagonal pair stage.  One wave per workgroup, 16 lanes per camera pair
// = 4 couple slots x 4 column quarters ({0,1,2}, {3,4}, {5,6}, {7,8}); each
// lane accumulates the 9 rows of its columns of
//   S_ij -= J_ca^T (K_a K_b^T) J_cb
// over the couples of its slot, then the 4 slots are reduced by shuffles.
// A lane group works on one unit: a whole segment, or a chunk of a long one
// whose partial block is summed by k_pair_sum.  A step covers the wave's 16
// couples; their two records are copied from global memory straight into LDS
// (16-byte lane copies that bypass the registers, spread over the whole wave,
// so every record is fetched once per step instead of once per lane of its
// couple).  The copies of step s + 1 are issued before step s is computed
// from the other of two LDS buffers.  A buffer is chunk-major: 16-byte chunk
// h of couple i sits at slot h * 16 + i, so the 16 couples' copies of one
// value lie in consecutive banks.  Units are stored in windows of rows
// (longest first inside a window); workgroup b runs on XCD b mod 8, which
// takes the waves of its own contiguous range of rows (ranges of equal work),
// keeping the records of neighbouring cameras in its L2.
// ---------------------------------------------------------------------------
constexpr int kPairWave = 4;   // units (camera pairs or chunks) per wave

struct XcdRanges { int wv[9]; };

// Three waves per SIMD: the FP64 instance's two 6 KB LDS buffers allow no
// more (12 per CU), and asking for four made the compiler spill to fit 128
// registers (12.26 against 12.14 ms on the 60,000-camera partition).
template <typename T, bool SUB = false>
__global__ __launch_bounds__(kWave) __attribute__((amdgpu_waves_per_eu(3))) void k_offdiag(
    int n_unit, XcdRanges xr, const int32_t* __restrict__ unit_rng, const int32_t* __restrict__ unit_dst,
    const int32_t* __restrict__ trip, const T* __restrict__ R, double* __restrict__ blk, double* __restrict__ pblk) {
    constexpr int kVal = 16 / sizeof(T);                             // values per 16-byte chunk
    constexpr int kCh = kRec / kVal;                                 // chunks per record (12 or 6)
    constexpr int kCpl = 4 * kPairWave;                              // couples per step
    constexpr int kLoads = kCpl * 2 * kCh / kWave;                   // chunk copies per lane per step
    constexpr int kRow = kCpl * kVal;                                // values per chunk slot row
    static_assert(kCpl == 16 && kLoads * kWave == kCpl * 2 * kCh, "staging must tile the wave");
    __shared__ __align__(16) T sC[2][2 * kCh * kRow];
    __shared__ int2 sT[2][kCpl];
    const int xcd = blockIdx.x % 8;
    const int wv = xr.wv[xcd] + (int)(blockIdx.x / 8);
    if (wv >= xr.wv[xcd + 1]) return;   // whole workgroup (one wave) leaves
    const int lane = threadIdx.x;
    const int grp = lane / 16, gl = lane % 16;
    const int slot = gl / 4, quarter = gl % 4;
    const int unit = wv * kPairWave + grp;
    const int cpl = grp * 4 + slot;                      // this lane's couple in a step
    const int c0 = quarter == 0 ? 0 : 2 * quarter + 1;   // 0, 3, 5, 7
    const int nc = quarter == 0 ? 3 : 2;
    const bool live = unit < n_unit;
    int t0 = 0, t1 = 0;
    if (live) { const int2 r = reinterpret_cast<const int2*>(unit_rng)[unit]; t0 = r.x; t1 = r.y; }
    int steps = (t1 - t0 + 3) / 4;
    steps = max(steps, __shfl_xor(steps, 16, kWave));
    steps = max(steps, __shfl_xor(steps, 32, kWave));
    // couple (a, b) of step st for this lane's slot; (-1, -1) past the unit's end
    auto couple = [&](int st) {
        const int t = t0 + 4 * st + slot;
        return (st < steps && t < t1) ? reinterpret_cast<const int2*>(trip)[t] : make_int2(-1, -1);
    };
    // copy k of the wave fills slots k * 64 .. k * 64 + 63: lane L moves
    // chunk 4 k + L / 16 of couple L % 16 (chunks past kCh: the b record's)
    auto issue = [&](int b) {
        const int2 ab = sT[b][lane % kCpl];
#pragma unroll
        for (int k = 0; k < kLoads; ++k) {
            const int h = 4 * k + lane / kCpl;
            const int o = h < kCh ? ab.x : ab.y;
            const T* src = o >= 0 ? R + (int64_t)o * kRec + (h % kCh) * kVal : R;   // unused couple: any valid chunk
            __builtin_amdgcn_global_load_lds((const void*)src,
                                             (__attribute__((address_space(3))) void*)(sC[b] + k * kWave * kVal), 16,
                                             0, 0);
        }
    };
    double acc[27];
#pragma unroll
    for (int m = 0; m < 27; ++m) acc[m] = 0.0;
    if (quarter == 0) { sT[0][cpl] = couple(0); sT[1][cpl] = couple(1); }
    __syncthreads();
    if (steps > 0) issue(0);
    for (int st = 0; st < steps; ++st) {
        const int b = st & 1;
        const int2 nxt = quarter == 0 ? couple(st + 2) : make_int2(-1, -1);
        __builtin_amdgcn_s_waitcnt(0);   // step st's records have landed in sC[b]
        __syncthreads();
        if (st + 1 < steps) issue(b ^ 1);
        // value v of this lane's couple (v < kRec: record a, else record b)
        const T* me = sC[b] + cpl * kVal;
        auto at = [&](int v) { return (double)me[(v / kVal) * kRow + v % kVal]; };
        const int t = t0 + 4 * st + slot;
        if (t < t1) {
            double ka[6], kb[6], jb0[3], jb1[3];
#pragma unroll
            for (int m = 0; m < 6; ++m) { ka[m] = at(18 + m); kb[m] = at(kRec + 18 + m); }
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                const int c = c0 + (q < nc ? q : 0);
                jb0[q] = at(kRec + c);
                jb1[q] = at(kRec + 9 + c);
            }
            double m00 = ka[0] * kb[0] + ka[1] * kb[1] + ka[2] * kb[2];
            const double m01 = ka[0] * kb[3] + ka[1] * kb[4] + ka[2] * kb[5];
            const double m10 = ka[3] * kb[0] + ka[4] * kb[1] + ka[5] * kb[2];
            double m11 = ka[3] * kb[3] + ka[4] * kb[4] + ka[5] * kb[5];
            if (SUB) {
                const int2 ab = sT[b][cpl];
                if ((ab.x >> 1) == (ab.y >> 1)) { m00 -= 1.0; m11 -= 1.0; }
            }
            double p0[3], p1[3];
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                p0[q] = m00 * jb0[q] + m01 * jb1[q];
                p1[q] = m10 * jb0[q] + m11 * jb1[q];
            }
#pragma unroll
            for (int r = 0; r < 9; ++r) {
                const double a0 = at(r), a1 = at(9 + r);
#pragma unroll
                for (int q = 0; q < 3; ++q) acc[r * 3 + q] += a0 * p0[q] + a1 * p1[q];
            }
        }
        __syncthreads();   // every lane is done with sT[b] and sC[b]
        if (quarter == 0) sT[b][cpl] = nxt;
    }
#pragma unroll
    for (int m = 0; m < 27; ++m) {
        acc[m] += __shfl_xor(acc[m], 4, kWave);
        acc[m] += __shfl_xor(acc[m], 8, kWave);
    }
    if (live && slot == 0) {
        const int dst = unit_dst[unit];
        double* out = dst >= 0 ? blk + (int64_t)dst * 81 : pblk + (int64_t)(-dst - 1) * 81;
#pragma unroll
        for (int r = 0; r < 9; ++r)
#pragma unroll
            for (int q = 0; q < 3; ++q)
                if (q < nc) out[r * 9 + c0 + q] = -acc[r * 3 + q];
    }
}

// Blocks of split segments: the sum of their chunks' partial blocks, in
// chunk order (one thread per block entry).
__global__ __launch_bounds__(BS) void k_pair_sum(int n_lseg, const int32_t* __restrict__ lseg_blk,
                                                 const int32_t* __restrict__ lseg_ptr,
                                                 const double* __restrict__ pblk, double* __restrict__ blk) {
    const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
    if (i >= (int64_t)n_lseg * 81) return;
    const int l = (int)(i / 81), e = (int)(i % 81);
    double v = 0.0;
    for (int p = lseg_ptr[l]; p < lseg_ptr[l + 1]; ++p) v += pblk[(int64_t)p * 81 + e];
    blk[(int64_t)lseg_blk[l] * 81 + e] = v;
}

// ---------------------------------------------------------------------------
// diagonal stage: one wave per RCS row over the camera's observations
// (four rows per workgroup); S_ii = sum J_c^T (I - K K^T) J_c +
// lambda diag(U), U = sum J_c^T J_c, b_i = -sum J_c^T (e + K lhat), then the
// block-Jacobi inverse S_ii^-1 (Cholesky and triangular inverse).  A lane
// holds 63 FP64 sums, which allows two waves per SIMD: with a wave per row a
// CU works on eight rows at once, and while one lane of a wave factors its
// row's block the other waves keep loading.
// ---------------------------------------------------------------------------
// one wave per workgroup, so that the three barriers hold a single wave
// (on the 60,000-camera partition, FP64: 4.37 against 4.51 ms with four)
constexpr int kDiagNW = 1;

template <typename T>
__global__ __launch_bounds__(kDiagNW * kWave) void k_diag(int n_rows, const int32_t* __restrict__ rowobs_ptr,
                                             const int32_t* __restrict__ rowobs, const int32_t* __restrict__ row_ptr,
                                             const T* __restrict__ R, const double* __restrict__ ebar, double lambda, double* __restrict__ blk, double* __restrict__ rhs,
                                             double* __restrict__ Minv, double* __restrict__ Linv,
                                             int* __restrict__ flags) {
    __shared__ double sred[kDiagNW][64];
    __shared__ double sS[kDiagNW][81];
    __shared__ double sL[kDiagNW][81];
    const int wv = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int row = blockIdx.x * kDiagNW + wv;
    const bool live = row < n_rows;   // wave-uniform; every wave takes part in the barriers
    double A[45], du[9], bb[9];
#pragma unroll
    for (int m = 0; m < 45; ++m) A[m] = 0.0;
#pragma unroll
    for (int m = 0; m < 9; ++m) { du[m] = 0.0; bb[m] = 0.0; }
    const int i0 = live ? rowobs_ptr[row] : 0, i1 = live ? rowobs_ptr[row + 1] : 0;
    for (int idx = i0 + lane; idx < i1; idx += kWave) {
        const int k = rowobs[idx];
        double jc[18], K[6];
        const T* rk = R + (int64_t)k * kRec;
        load_jc(rk, jc);
        load6(rk + 18, K);
        const double2 v = reinterpret_cast<const double2*>(ebar)[idx];   // e + K lhat
        const double n00 = 1.0 - (K[0] * K[0] + K[1] * K[1] + K[2] * K[2]);
        const double n01 = -(K[0] * K[3] + K[1] * K[4] + K[2] * K[5]);
        const double n11 = 1.0 - (K[3] * K[3] + K[4] * K[4] + K[5] * K[5]);
        const double v0 = v.x, v1 = v.y;
        double q0[9], q1[9];
#pragma unroll
        for (int c = 0; c < 9; ++c) {
            q0[c] = n00 * jc[c] + n01 * jc[9 + c];
            q1[c] = n01 * jc[c] + n11 * jc[9 + c];
        }
        int m = 0;
#pragma unroll
        for (int r = 0; r < 9; ++r) {
            du[r] += jc[r] * jc[r] + jc[9 + r] * jc[9 + r];
            bb[r] -= jc[r] * v0 + jc[9 + r] * v1;
#pragma unroll
            for (int c = r; c < 9; ++c, ++m) A[m] += jc[r] * q0[c] + jc[9 + r] * q1[c];
        }
    }
    // the wave's 63 sums (fixed shuffle tree), each stored as soon as it is
    // formed so that the totals do not occupy registers
#pragma unroll
    for (int m = 0; m < 45; ++m) {
        const double t = wave_sum(A[m]);
        if (lane == 0) sred[wv][m] = t;
    }
#pragma unroll
    for (int m = 0; m < 9; ++m) {
        const double t = wave_sum(du[m]), w = wave_sum(bb[m]);
        if (lane == 0) { sred[wv][45 + m] = t; sred[wv][54 + m] = w; }
    }
    __syncthreads();
    double* S = sS[wv];
    double* L = sL[wv];
    if (live) {
        for (int e = lane; e < 81; e += kWave) {
            const int i = e / 9, j = e % 9;
            const int a = i < j ? i : j, b = i < j ? j : i;
            const int m = a * 9 - a * (a - 1) / 2 + (b - a);   // packed upper-triangle index
            double v = sred[wv][m];
            if (i == j) v += lambda * sred[wv][45 + i];
            S[e] = v;
            blk[(int64_t)row_ptr[row] * 81 + e] = v;
        }
        if (lane < 9) rhs[(int64_t)row * 9 + lane] = sred[wv][54 + lane];
    }
    __syncthreads();
    if (live && lane == 0) {
        // Cholesky S = L L^T, then L^-1 in place (lower triangle)
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
        // S^-1 = L^-T L^-1: entry (i, j) = sum_{q >= max(i,j)} Li[q][i] Li[q][j]
        for (int e = lane; e < 81; e += kWave) {
            const int i = e / 9, j = e % 9;
            double t = 0.0;
            for (int q = (i > j ? i : j); q < 9; ++q) t += L[q * 9 + i] * L[q * 9 + j];
            Minv[(int64_t)row * 81 + e] = t;
            Linv[(int64_t)row * 81 + e] = L[e];
        }
    }
}

// ---------------------------------------------------------------------------
// back-substitution (Eq. (5)): dx_p = L^-T (lhat - sum_a K_a^T J_ca dxc_a),
// and with it the model terms of the gain ratio, |J dx|^2 and dx^T l with
// l = -J^T e: the solve's right-hand side is w = L^T dx_p, so an
// observation's J dx = J_c dxc + K w with no J_p (J_p = K L^T).  One wave per
// chunk of whole tracks, one lane per observation; per-block partials of the
// two model terms.
// ---------------------------------------------------------------------------
// four waves per workgroup (on the 60,000-camera partition, FP64: 6.40 ms
// against 6.46 with two and 6.50 with one), blocks in XCD-contiguous order
// (6.31 against 6.39 ms)
constexpr int kBackNW = 4;

template <typename T>
__global__ __launch_bounds__(kBackNW * kWave) void k_backsub(int n_chunk, const int32_t* __restrict__ chunk_ptr,
                                                const int32_t* __restrict__ obs_pt, const int32_t* __restrict__ obs_row,
                                                const int32_t* __restrict__ chunk_q, const T* __restrict__ R,
                                                const double* __restrict__ ptL, const double* __restrict__ dxc,
                                                const double* __restrict__ e, double* __restrict__ dxp,
                                                double* __restrict__ part, int nb) {
    __shared__ double sP[kBackNW][kWave][3];
    __shared__ double sh[kBackNW];
    const int wv = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int chunk = xcd_block() * kBackNW + wv;
    int k0 = 0, k1 = 0;
    if (chunk < n_chunk) { k0 = chunk_ptr[chunk]; k1 = chunk_ptr[chunk + 1]; }
    const int k = k0 + lane;
    const bool act = k < k1;
    const int p = act ? obs_pt[k] : -1;
    const Track tk = chunk_track(act, p, lane, k1 - k0);
    const int head = tk.head, tl = tk.len;
    const int64_t q = chunk < n_chunk ? (int64_t)chunk_q[chunk] + tk.idx : 0;   // internal point index
    double K[6], g0 = 0.0, g1 = 0.0;
    if (act) {
        const int row = obs_row[k];
        const T* rk = R + (int64_t)k * kRec;
        load6(rk + 18, K);
        if (row >= 0) {
            double jc[18];
            load_jc(rk, jc);
            const double* dc = dxc + (int64_t)row * 9;
#pragma unroll
            for (int i = 0; i < 9; ++i) {
                const double c = dc[i];
                g0 += jc[i] * c;
                g1 += jc[9 + i] * c;
            }
        }
        sP[wv][lane][0] = K[0] * g0 + K[3] * g1;
        sP[wv][lane][1] = K[1] * g0 + K[4] * g1;
        sP[wv][lane][2] = K[2] * g0 + K[5] * g1;
    }
    __syncthreads();
    if (act && head == lane) {
        double u0 = 0.0, u1 = 0.0, u2 = 0.0;
        for (int q = 0; q < tl; ++q) { u0 += sP[wv][lane + q][0]; u1 += sP[wv][lane + q][1]; u2 += sP[wv][lane + q][2]; }
        const double* L = ptL + q * 9;
        u0 = L[6] - u0; u1 = L[7] - u1; u2 = L[8] - u2;
        // L^T x = u with L = [[L00,0,0],[L10,L11,0],[L20,L21,L22]]
        const double x2 = u2 / L[5];
        const double x1 = (u1 - L[4] * x2) / L[2];
        const double x0 = (u0 - L[1] * x1 - L[3] * x2) / L[0];
        dxp[(int64_t)p * 3 + 0] = x0;
        dxp[(int64_t)p * 3 + 1] = x1;
        dxp[(int64_t)p * 3 + 2] = x2;
        // the head's own row is read by no other lane now: w for the track
        sP[wv][lane][0] = u0; sP[wv][lane][1] = u1; sP[wv][lane][2] = u2;
    }
    __syncthreads();
    double jdx2 = 0.0, dxl = 0.0;
    if (act) {
        const double* w = sP[wv][head];
        const double a0 = g0 + K[0] * w[0] + K[1] * w[1] + K[2] * w[2];
        const double a1 = g1 + K[3] * w[0] + K[4] * w[1] + K[5] * w[2];
        const double2 ek = reinterpret_cast<const double2*>(e)[k];
        jdx2 = a0 * a0 + a1 * a1;
        dxl = -(a0 * ek.x + a1 * ek.y);
    }
    const double s0 = block_sum<kBackNW * kWave>(jdx2, sh);
    const double s1 = block_sum<kBackNW * kWave>(dxl, sh);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = s0;
        part[nb + blockIdx.x] = s1;
    }
}

// The model terms |J dx|^2 and dx^T l for a dx_p given from outside (after
// re-triangulation): J_p dx_p = K (L^T dx_p) with L from the point terms;
// same layout and partials as k_backsub
template <typename T>
__global__ __launch_bounds__(BS) void k_model_terms(int n_chunk, const int32_t* __restrict__ chunk_ptr,
                                                    const int32_t* __restrict__ obs_pt,
                                                    const int32_t* __restrict__ obs_row,
                                                    const int32_t* __restrict__ chunk_q, const T* __restrict__ R,
                                                    const double* __restrict__ ptL, const double* __restrict__ dxc,
                                                    const double* __restrict__ dxp, const double* __restrict__ e,
                                                    double* __restrict__ part, int nb) {
    __shared__ double sh[WPB];
    const int wv = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int chunk = blockIdx.x * WPB + wv;
    int k0 = 0, k1 = 0;
    if (chunk < n_chunk) { k0 = chunk_ptr[chunk]; k1 = chunk_ptr[chunk + 1]; }
    const int k = k0 + lane;
    const bool act = k < k1;
    const int p = act ? obs_pt[k] : -1;
    const Track tk = chunk_track(act, p, lane, k1 - k0);
    const int64_t q = chunk < n_chunk ? (int64_t)chunk_q[chunk] + tk.idx : 0;
    double jdx2 = 0.0, dxl = 0.0;
    if (act) {
        const int row = obs_row[k];
        const T* rk = R + (int64_t)k * kRec;
        double K[6], g0 = 0.0, g1 = 0.0;
        load6(rk + 18, K);
        if (row >= 0) {
            double jc[18];
            load_jc(rk, jc);
            const double* dc = dxc + (int64_t)row * 9;
#pragma unroll
            for (int i = 0; i < 9; ++i) { g0 += jc[i] * dc[i]; g1 += jc[9 + i] * dc[i]; }
        }
        const double* L = ptL + q * 9;   // L00, L10, L11, L20, L21, L22
        const double* d = dxp + (int64_t)p * 3;
        const double w0 = L[0] * d[0] + L[1] * d[1] + L[3] * d[2];
        const double w1 = L[2] * d[1] + L[4] * d[2];
        const double w2 = L[5] * d[2];
        const double a0 = g0 + K[0] * w0 + K[1] * w1 + K[2] * w2;
        const double a1 = g1 + K[3] * w0 + K[4] * w1 + K[5] * w2;
        const double2 ek = reinterpret_cast<const double2*>(e)[k];
        jdx2 = a0 * a0 + a1 * a1;
        dxl = -(a0 * ek.x + a1 * ek.y);
    }
    const double s0 = block_sum<BS>(jdx2, sh);
    const double s1 = block_sum<BS>(dxl, sh);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = s0;
        part[nb + blockIdx.x] = s1;
    }
}

// ---------------------------------------------------------------------------
// Tracks longer than a wave (more than 64 observations): one workgroup per
// point, its threads striding over the track; the track sums are reduced in
// a fixed order (each thread's strided sum, the wave's shuffle tree, then the
// four waves in order).  The arithmetic per observation is that of the wave
// kernels above.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void add_point_sums(const double* jp, double eu, double ev, double* v) {
    v[0] += jp[0] * jp[0] + jp[3] * jp[3];
    v[1] += jp[0] * jp[1] + jp[3] * jp[4];
    v[2] += jp[0] * jp[2] + jp[3] * jp[5];
    v[3] += jp[1] * jp[1] + jp[4] * jp[4];
    v[4] += jp[1] * jp[2] + jp[4] * jp[5];
    v[5] += jp[2] * jp[2] + jp[5] * jp[5];
    v[6] -= jp[0] * eu + jp[3] * ev;
    v[7] -= jp[1] * eu + jp[4] * ev;
    v[8] -= jp[2] * eu + jp[5] * ev;
}

// linearization fused with the point stage for point q0 + blockIdx.x (as
// linpoint: J_p is not stored, the second pass projects again for it);
// part[blockIdx.x] = the track's cost
template <typename T>
__global__ __launch_bounds__(BS) void k_linpoint_long(int q0, const int32_t* __restrict__ long_ptr, int n,
                                                      const int32_t* __restrict__ obs_cam,
                                                      const int32_t* __restrict__ obs_pt, const double* __restrict__ uv,
                                                      const double* __restrict__ cams, const double* __restrict__ pts,
                                                      double lambda, T* __restrict__ R, double* __restrict__ e,
                                                      double* __restrict__ ptL, const int32_t* __restrict__ obs_rpos,
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
        double jc[18], jp[6], pu, pv;
        project_point<true>(cams + (int64_t)obs_cam[k] * 9, X0, X1, X2, pu, pv, jc, jp);
        const double eu = pu - uv[k], ev = pv - uv[n + k];
        if (!records_in_range<T>(jc, jp, eu, ev)) flags[2] = 1;
#pragma unroll
        for (int m = 0; m < 18; ++m) jc[m] = (double)(T)jc[m];
#pragma unroll
        for (int m = 0; m < 6; ++m) jp[m] = (double)(T)jp[m];
        reinterpret_cast<double2*>(e)[k] = make_double2(eu, ev);
        store_jc(R + (int64_t)k * kRec, jc);
        add_point_sums(jp, eu, ev, v);
        v[9] += 0.5 * (eu * eu + ev * ev);
    }
    block_reduce<10>(v, sh);
    if (threadIdx.x == 0) {
        double r[kPT];
        if (!point_terms(v, lambda, r)) flags[0] = 1;
#pragma unroll
        for (int m = 0; m < kPT; ++m) sr[m] = r[m];
#pragma unroll
        for (int m = 0; m < 9; ++m) ptL[q * 9 + m] = r[m];
        part[blockIdx.x] = v[9];
    }
    __syncthreads();
    for (int k = k0 + threadIdx.x; k < k1; k += BS) {
        double jp[6], pu, pv, K[6];
        project_point<true, false>(cams + (int64_t)obs_cam[k] * 9, X0, X1, X2, pu, pv, nullptr, jp);
#pragma unroll
        for (int m = 0; m < 6; ++m) jp[m] = (double)(T)jp[m];
        point_K(sr, jp, K);
        store6(R + (int64_t)k * kRec + 18, K);
        store_ebar<T>(sr, K, pu - uv[k], pv - uv[n + k], obs_rpos[k], ebar);
    }
}

// point stage (a new damping) for point q0 + blockIdx.x, as k_point
template <typename T, bool FROM_K>
__global__ __launch_bounds__(BS) void k_point_long(int q0, const int32_t* __restrict__ long_ptr, T* __restrict__ R,
                                                   T* __restrict__ Jp, const double* __restrict__ e, double lambda,
                                                   double* __restrict__ ptL, const int32_t* __restrict__ obs_rpos,
                                                   double* __restrict__ ebar, int* __restrict__ flags) {
    __shared__ double sh[9][WPB];
    __shared__ double sr[kPT];
    __shared__ double sL[6];   // the previous formation's factor (FROM_K)
    const int k0 = long_ptr[blockIdx.x], k1 = long_ptr[blockIdx.x + 1];
    const int64_t q = (int64_t)q0 + blockIdx.x;
    if (FROM_K && threadIdx.x < 6) sL[threadIdx.x] = ptL[q * 9 + threadIdx.x];
    __syncthreads();
    auto jp_of = [&](int k, double* jp) {
        if (FROM_K) {
            double K[6];
            load6(R + (int64_t)k * kRec + 18, K);
            jp_from_K(K, sL, jp);
#pragma unroll
            for (int m = 0; m < 6; ++m) jp[m] = (double)(T)jp[m];
        } else {
            load6(Jp + (int64_t)k * 6, jp);
        }
    };
    double v[9];
#pragma unroll
    for (int m = 0; m < 9; ++m) v[m] = 0.0;
    for (int k = k0 + threadIdx.x; k < k1; k += BS) {
        double jp[6];
        jp_of(k, jp);
        if (FROM_K) store6(Jp + (int64_t)k * 6, jp);
        const double2 ek = reinterpret_cast<const double2*>(e)[k];
        add_point_sums(jp, ek.x, ek.y, v);
    }
    block_reduce<9>(v, sh);
    if (threadIdx.x == 0) {
        double r[kPT];
        if (!point_terms(v, lambda, r)) flags[0] = 1;
#pragma unroll
        for (int m = 0; m < kPT; ++m) sr[m] = r[m];
#pragma unroll
        for (int m = 0; m < 9; ++m) ptL[q * 9 + m] = r[m];
    }
    __syncthreads();
    for (int k = k0 + threadIdx.x; k < k1; k += BS) {
        double jp[6], K[6];
        jp_of(k, jp);   // FROM_K: from the previous K, which this thread replaces only now
        const double2 ek = reinterpret_cast<const double2*>(e)[k];
        point_K(sr, jp, K);
        store6(R + (int64_t)k * kRec + 18, K);
        store_ebar<T>(sr, K, ek.x, ek.y, obs_rpos[k], ebar);
    }
}

// J_c dxc of observation k (0 for a fixed camera)
template <typename T>
__device__ __forceinline__ void jc_dxc(const T* __restrict__ rk, int row, const double* __restrict__ dxc, double& g0,
                                       double& g1) {
    g0 = 0.0; g1 = 0.0;
    if (row < 0) return;
    double jc[18];
    load_jc(rk, jc);
    const double* dc = dxc + (int64_t)row * 9;
#pragma unroll
    for (int i = 0; i < 9; ++i) { g0 += jc[i] * dc[i]; g1 += jc[9 + i] * dc[i]; }
}

// back-substitution and the model terms for point q0 + blockIdx.x, as
// k_backsub; part[blockIdx.x], part[stride + blockIdx.x]
template <typename T>
__global__ __launch_bounds__(BS) void k_backsub_long(int q0, const int32_t* __restrict__ long_ptr,
                                                     const int32_t* __restrict__ obs_pt,
                                                     const int32_t* __restrict__ obs_row, const T* __restrict__ R,
                                                     const double* __restrict__ ptL, const double* __restrict__ dxc,
                                                     const double* __restrict__ e, double* __restrict__ dxp,
                                                     double* __restrict__ part, int stride) {
    __shared__ double sh[3][WPB];
    __shared__ double su[3];
    const int k0 = long_ptr[blockIdx.x], k1 = long_ptr[blockIdx.x + 1];
    const int64_t q = (int64_t)q0 + blockIdx.x;
    const int p = obs_pt[k0];
    double v[3] = {0.0, 0.0, 0.0};
    for (int k = k0 + threadIdx.x; k < k1; k += BS) {
        const T* rk = R + (int64_t)k * kRec;
        double K[6], g0, g1;
        load6(rk + 18, K);
        jc_dxc(rk, obs_row[k], dxc, g0, g1);
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
        su[0] = u0; su[1] = u1; su[2] = u2;
    }
    __syncthreads();
    double t[2] = {0.0, 0.0};
    for (int k = k0 + threadIdx.x; k < k1; k += BS) {
        const T* rk = R + (int64_t)k * kRec;
        double K[6], g0, g1;
        load6(rk + 18, K);
        jc_dxc(rk, obs_row[k], dxc, g0, g1);
        const double a0 = g0 + K[0] * su[0] + K[1] * su[1] + K[2] * su[2];
        const double a1 = g1 + K[3] * su[0] + K[4] * su[1] + K[5] * su[2];
        const double2 ek = reinterpret_cast<const double2*>(e)[k];
        t[0] += a0 * a0 + a1 * a1;
        t[1] -= a0 * ek.x + a1 * ek.y;
    }
    block_reduce<2>(t, sh);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = t[0];
        part[stride + blockIdx.x] = t[1];
    }
}

// the model terms for a given dx_p (after re-triangulation), as k_model_terms
template <typename T>
__global__ __launch_bounds__(BS) void k_model_terms_long(int q0, const int32_t* __restrict__ long_ptr,
                                                         const int32_t* __restrict__ obs_pt,
                                                         const int32_t* __restrict__ obs_row, const T* __restrict__ R,
                                                         const double* __restrict__ ptL, const double* __restrict__ dxc,
                                                         const double* __restrict__ dxp, const double* __restrict__ e,
                                                         double* __restrict__ part, int stride) {
    __shared__ double sh[2][WPB];
    const int k0 = long_ptr[blockIdx.x], k1 = long_ptr[blockIdx.x + 1];
    const int64_t q = (int64_t)q0 + blockIdx.x;
    const int p = obs_pt[k0];
    const double* L = ptL + q * 9;   // L00, L10, L11, L20, L21, L22
    const double* d = dxp + (int64_t)p * 3;
    const double w0 = L[0] * d[0] + L[1] * d[1] + L[3] * d[2];
    const double w1 = L[2] * d[1] + L[4] * d[2];
    const double w2 = L[5] * d[2];
    double t[2] = {0.0, 0.0};
    for (int k = k0 + threadIdx.x; k < k1; k += BS) {
        const T* rk = R + (int64_t)k * kRec;
        double K[6], g0, g1;
        load6(rk + 18, K);
        jc_dxc(rk, obs_row[k], dxc, g0, g1);
        const double a0 = g0 + K[0] * w0 + K[1] * w1 + K[2] * w2;
        const double a1 = g1 + K[3] * w0 + K[4] * w1 + K[5] * w2;
        const double2 ek = reinterpret_cast<const double2*>(e)[k];
        t[0] += a0 * a0 + a1 * a1;
        t[1] -= a0 * ek.x + a1 * ek.y;
    }
    block_reduce<2>(t, sh);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = t[0];
        part[stride + blockIdx.x] = t[1];
    }
}

}  // namespace

template <typename T>
void launch_point_t(ba_ctx* c, double lambda) {
    const int nb = (c->n_chunk + WPB - 1) / WPB;
    T* R = (T*)c->R;
    T* Jp = (T*)c->Jp;
    if (nb > 0) {
        if (c->jp_valid)
            k_point<T><<<nb, BS, 0, c->stream>>>(c->n_chunk, c->chunk_ptr, c->obs_pt, c->chunk_q, R, Jp, c->e, lambda,
                                                 c->ptL, c->obs_rpos, c->ebar, c->flags);
        else
            k_point<T, true><<<nb, BS, 0, c->stream>>>(c->n_chunk, c->chunk_ptr, c->obs_pt, c->chunk_q, R, Jp, c->e,
                                                       lambda, c->ptL, c->obs_rpos, c->ebar, c->flags);
    }
    if (c->n_long > 0) {
        if (c->jp_valid)
            k_point_long<T, false><<<c->n_long, BS, 0, c->stream>>>(c->q_long0, c->long_ptr, R, Jp, c->e, lambda,
                                                                    c->ptL, c->obs_rpos, c->ebar, c->flags);
        else
            k_point_long<T, true><<<c->n_long, BS, 0, c->stream>>>(c->q_long0, c->long_ptr, R, Jp, c->e, lambda,
                                                                   c->ptL, c->obs_rpos, c->ebar, c->flags);
    }
}

void launch_point(ba_ctx* c, double lambda) {
    if (c->precision == BA_MIXED)
        launch_point_t<float>(c, lambda);
    else
        launch_point_t<double>(c, lambda);
    c->jp_valid = true;
}

void launch_linearize_point(ba_ctx* c, const double* cams, const double* pts, double lambda) {
    const int nb = (c->n_chunk + kLinNW - 1) / kLinNW;
    const int n = (int)c->n_obs;
    if (nb + (int64_t)c->n_long > c->n_part)
        throw ba_hip_error(hipErrorInvalidValue, "cost partials exceed their buffer", __FILE__, __LINE__);
    if (nb > 0) {
        if (c->precision == BA_MIXED)
            k_linpoint_f<<<nb, kLinNW * kWave, 0, c->stream>>>(c->n_chunk, c->chunk_ptr, n, c->obs_cam, c->obs_pt, c->chunk_q,
                                                   c->obs_uv, cams, pts, lambda, (float*)c->R, c->e, c->ptL,
                                                   c->obs_rpos, c->ebar, c->part, c->flags);
        else
            k_linpoint_d<<<nb, kLinNW * kWave, 0, c->stream>>>(c->n_chunk, c->chunk_ptr, n, c->obs_cam, c->obs_pt, c->chunk_q,
                                                   c->obs_uv, cams, pts, lambda, (double*)c->R, c->e, c->ptL,
                                                   c->obs_rpos, c->ebar, c->part, c->flags);
    }
    if (c->n_long > 0) {
        if (c->precision == BA_MIXED)
            k_linpoint_long<float><<<c->n_long, BS, 0, c->stream>>>(c->q_long0, c->long_ptr, n, c->obs_cam,
                                                                    c->obs_pt, c->obs_uv, cams, pts, lambda,
                                                                    (float*)c->R, c->e, c->ptL, c->obs_rpos,
                                                                    c->ebar, c->part + nb, c->flags);
        else
            k_linpoint_long<double><<<c->n_long, BS, 0, c->stream>>>(c->q_long0, c->long_ptr, n, c->obs_cam,
                                                                     c->obs_pt, c->obs_uv, cams, pts, lambda,
                                                                     (double*)c->R, c->e, c->ptL, c->obs_rpos,
                                                                     c->ebar, c->part + nb, c->flags);
    }
    launch_reduce(c, c->part, nb + c->n_long, 1, c->scal + 0);
    c->jp_valid = false;   // J_p = K L^T where it is needed
}

void launch_offdiag(ba_ctx* c) {
    if (c->n_unit == 0) return;
    XcdRanges xr;
    int most = 0;
    for (int x = 0; x < 9; ++x) xr.wv[x] = c->xcd_wv[x];
    for (int x = 0; x < 8; ++x) most = std::max(most, xr.wv[x + 1] - xr.wv[x]);
    const int grid = 8 * most;
    if (c->shared)
        k_offdiag<double, true><<<grid, kWave, 0, c->stream>>>(c->n_unit, xr, c->unit_rng, c->unit_dst, c->trip,
                                                               (const double*)c->R, c->blk, c->pblk);
    else if (c->precision == BA_MIXED)
        k_offdiag<float><<<grid, kWave, 0, c->stream>>>(c->n_unit, xr, c->unit_rng, c->unit_dst, c->trip,
                                                        (const float*)c->R, c->blk, c->pblk);
    else
        k_offdiag<double><<<grid, kWave, 0, c->stream>>>(c->n_unit, xr, c->unit_rng, c->unit_dst, c->trip,
                                                         (const double*)c->R, c->blk, c->pblk);
    if (c->n_lseg > 0) {
        const int64_t n = (int64_t)c->n_lseg * 81;
        k_pair_sum<<<(unsigned)((n + BS - 1) / BS), BS, 0, c->stream>>>(c->n_lseg, c->lseg_blk, c->lseg_ptr,
                                                                        c->pblk, c->blk);
    }
}

void launch_diag(ba_ctx* c, double lambda) {
    if (c->n_rows == 0) return;
    if (c->precision == BA_MIXED)
        k_diag<float><<<(c->n_rows + kDiagNW - 1) / kDiagNW, kDiagNW * kWave, 0, c->stream>>>(c->n_rows, c->rowobs_ptr, c->rowobs, c->row_ptr,
                                                       (const float*)c->R, c->ebar, lambda, c->blk, c->rhs,
                                                       c->Minv, c->Linv, c->flags);
    else
        k_diag<double><<<(c->n_rows + kDiagNW - 1) / kDiagNW, kDiagNW * kWave, 0, c->stream>>>(c->n_rows, c->rowobs_ptr, c->rowobs, c->row_ptr,
                                                        (const double*)c->R, c->ebar, lambda, c->blk, c->rhs,
                                                        c->Minv, c->Linv, c->flags);
}

// back-substitution; the model terms go to scal[2] (|J dx|^2) and scal[3]
// (dx^T l): per-block partials of the chunks, then one per long track
template <typename T>
void launch_back_substitute_t(ba_ctx* c, const double* dxc, double* dxp, int nb, int stride) {
    const T* R = (const T*)c->R;
    if (nb > 0)
        k_backsub<T><<<nb, kBackNW * kWave, 0, c->stream>>>(c->n_chunk, c->chunk_ptr, c->obs_pt, c->obs_row, c->chunk_q, R, c->ptL,
                                               dxc, c->e, dxp, c->part, stride);
    if (c->n_long > 0)
        k_backsub_long<T><<<c->n_long, BS, 0, c->stream>>>(c->q_long0, c->long_ptr, c->obs_pt, c->obs_row, R, c->ptL,
                                                           dxc, c->e, dxp, c->part + nb, stride);
}

void launch_back_substitute(ba_ctx* c, const double* dxc, double* dxp) {
    const int nb = (c->n_chunk + kBackNW - 1) / kBackNW;
    const int stride = nb + c->n_long;
    if (stride == 0) return;
    if (2 * (int64_t)stride > c->n_part)
        throw ba_hip_error(hipErrorInvalidValue, "model-term partials exceed their buffer", __FILE__, __LINE__);
    if (c->precision == BA_MIXED)
        launch_back_substitute_t<float>(c, dxc, dxp, nb, stride);
    else
        launch_back_substitute_t<double>(c, dxc, dxp, nb, stride);
    launch_reduce(c, c->part, stride, 2, c->scal + 2);
}

// the model terms for dx_p replaced after back-substitution
template <typename T>
void launch_model_terms_t(ba_ctx* c, const double* dxc, const double* dxp, int nb, int stride) {
    const T* R = (const T*)c->R;
    if (nb > 0)
        k_model_terms<T><<<nb, BS, 0, c->stream>>>(c->n_chunk, c->chunk_ptr, c->obs_pt, c->obs_row, c->chunk_q, R,
                                                   c->ptL, dxc, dxp, c->e, c->part, stride);
    if (c->n_long > 0)
        k_model_terms_long<T><<<c->n_long, BS, 0, c->stream>>>(c->q_long0, c->long_ptr, c->obs_pt, c->obs_row, R,
                                                               c->ptL, dxc, dxp, c->e, c->part + nb, stride);
}

void launch_model_terms(ba_ctx* c, const double* dxc, const double* dxp) {
    const int nb = (c->n_chunk + WPB - 1) / WPB;
    const int stride = nb + c->n_long;
    if (stride == 0) return;
    if (2 * (int64_t)stride > c->n_part)
        throw ba_hip_error(hipErrorInvalidValue, "model-term partials exceed their buffer", __FILE__, __LINE__);
    if (c->precision == BA_MIXED)
        launch_model_terms_t<float>(c, dxc, dxp, nb, stride);
    else
        launch_model_terms_t<double>(c, dxc, dxp, nb, stride);
    launch_reduce(c, c->part, stride, 2, c->scal + 2);
}

}  // namespace ba
