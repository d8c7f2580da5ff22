// C ABI of the bundle-adjustment library: context creation (validation and
// the co-visibility pattern, built once), the per-stage entry points and one
// LM iteration.  All device work goes to the context's stream.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <numeric>
#include <cstdlib>

#include "ba_common.hpp"
#include "host_par.hpp"
#include "gnn.hpp"

namespace ba {
void launch_product(ba_ctx* c, const double* x, double* y);
}

namespace {

using ba::kMaxTrack;
using ba::counting_sort;
using ba::host_threads;
using ba::parallel_for;
using ba::kRec;
using ba::Pcg;

thread_local std::string g_create_error;

const char* const kRangeMsg =
    "a Jacobian entry exceeds the range of the record type (FP32 in mixed precision) or a residual is not finite";

struct ba_oom {
    std::string what;
};
struct ba_invalid {
    std::string what;
};

template <typename T>
void dalloc(ba_ctx* c, T** p, size_t n) {
    const size_t bytes = std::max<size_t>(n, 1) * sizeof(T);
    if (c->cap && c->bytes + bytes > c->cap)
        throw ba_oom{"device workspace cap of " + std::to_string(c->cap) + " bytes exceeded"};
    hipError_t e = hipMalloc((void**)p, bytes);
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        throw ba_oom{"hipMalloc of " + std::to_string(bytes) + " bytes failed"};
    }
    if (e != hipSuccess) throw ba_hip_error(e, "hipMalloc", __FILE__, __LINE__);
    c->bytes += bytes;
}

template <typename T>
void upload(ba_ctx* c, T** p, const std::vector<T>& h) {
    dalloc(c, p, h.size());
    if (!h.empty())
        BA_HIP_CHECK(hipMemcpyAsync(*p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, c->stream));
}

void free_ctx(ba_ctx* c) {
    if (!c) return;
    void* ptrs[] = {c->obs_cam, c->obs_pt, c->obs_row, c->obs_uv, c->chunk_q, c->chunk_ptr, c->long_ptr, c->cam_row,
                    c->row_ptr, c->col_idx, c->off_blk, c->pair_ptr, c->trip, c->rowobs_ptr, c->rowobs,
                    c->sf_ptr, c->sf_col, c->sf_src, c->Sf, c->Sf32, c->Su32, c->lo_ptr, c->lo_blk, c->unit_rng, c->unit_dst, c->lseg_blk, c->lseg_ptr, c->pblk, c->R, c->Jp, c->e, c->obs_rpos, c->ebar, c->ptL, c->blk, c->rhs, c->Minv,
                    c->Linv, c->Mlearn, c->dxc, c->dxp, c->part, c->part2, c->scal, c->flags, c->pcg.x, c->pcg.r[0],
                    c->pcg.r[1], c->pcg.z, c->pcg.q, c->pcg.d, c->pcg.t, c->pcg.u, c->pcg.tb, c->pcg.pA, c->pcg.pR, c->pcg.W, c->pcg.SW, c->pcg.Einv,
                    c->pcg.pW, c->pcg.pE, c->lin_cams, c->pcg.state,
                    c->pcg.scal, c->fs.ptr, c->fs.J, c->fs.slot, c->fs.tptr, c->fs.tile, c->fs.brow,
                    c->fs.gu_ptr, c->fs.gu_col, c->fs.gu_pos, c->fs.gu_src, c->fs.gl_self, c->fs.tg, c->pcg.bm, c->fs.Gl, c->fs.Gu, c->fs.An, c->fs.G,
                    c->fs.Gh, c->fs.hs, c->fs.Dn, c->tri_failed, c->img_cam, c->lin_params, c->lin_pts, c->csr.bptr, c->csr.slot_src, c->csr.slot_col, c->csr.slot_row, c->csr.rowptr, c->csr.col, c->csr.val};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    if (c->h_scal) (void)hipHostFree(c->h_scal);
    if (c->h_flags) (void)hipHostFree(c->h_flags);
    for (auto& e : c->ev)
        if (e) (void)hipEventDestroy(e);
    for (auto& g : c->pcg_graphs) (void)hipGraphExecDestroy(g.exec);
    if (c->lgraph) {
        ba::gnn::free_graph(*(ba::gnn::Graph*)c->lgraph);
        delete (ba::gnn::Graph*)c->lgraph;
    }
    if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
    delete c;
}

// The first index in [0, n) where bad(k) holds, or n (threads in parallel).
template <typename F>
int64_t first_where(int64_t n, F&& bad) {
    std::atomic<int64_t> first{n};
    parallel_for(n, 1 << 18, [&](int64_t k0, int64_t k1, int) {
        for (int64_t k = k0; k < k1 && k < first.load(std::memory_order_relaxed); ++k)
            if (bad(k)) {
                int64_t cur = first.load();
                while (k < cur && !first.compare_exchange_weak(cur, k)) {}
                break;
            }
    });
    return first.load();
}

// Builds the internal observation order, the pattern and every index
// structure on the host, then uploads them; the caller's point ids and
// pixels (device arrays d_pt, d_uv) are put in the internal order on the
// device, where the pixels are also checked.
void build(ba_ctx* c, const std::vector<int32_t>& cam, const std::vector<int32_t>& pt, const int32_t* d_pt,
           const double* d_uv, const std::vector<uint8_t>& fixed) {
    ba::Phases ph("ba_create");
    const int64_t n = c->n_obs;
    const int32_t nc = c->n_cams, np = c->n_pts;
    {
        const int64_t k = first_where(n, [&](int64_t i) { return cam[i] < 0 || cam[i] >= nc || pt[i] < 0 || pt[i] >= np; });
        if (k < n) {
            if (cam[k] < 0 || cam[k] >= nc) throw ba_invalid{"obs_cam[" + std::to_string(k) + "] out of range"};
            throw ba_invalid{"obs_pt[" + std::to_string(k) + "] out of range"};
        }
    }
    ph.mark("validate");
    // internal order: whole tracks, points by the lowest camera that sees
    // them (ties by point), observations of a track by camera.  Points seen by
    // one neighbourhood of cameras end up close together, so the records that
    // a camera pair (or a camera) reads lie in a narrow window of memory.
    // track lengths and lowest cameras (order-free sums and minima, all
    // threads at once)
    std::vector<int32_t> cnt(np), key(np);
    {
        std::unique_ptr<std::atomic<int32_t>[]> acnt(new std::atomic<int32_t>[np]), akey(new std::atomic<int32_t>[np]);
        parallel_for(np, 1 << 16, [&](int64_t p0, int64_t p1, int) {
            for (int64_t p = p0; p < p1; ++p) {
                acnt[p].store(0, std::memory_order_relaxed);
                akey[p].store(nc, std::memory_order_relaxed);
            }
        });
        parallel_for(n, 1 << 18, [&](int64_t k0, int64_t k1, int) {
            for (int64_t k = k0; k < k1; ++k) {
                const int32_t p = pt[k], cm = cam[k];
                acnt[p].fetch_add(1, std::memory_order_relaxed);
                int32_t cur = akey[p].load(std::memory_order_relaxed);
                while (cm < cur && !akey[p].compare_exchange_weak(cur, cm, std::memory_order_relaxed)) {}
            }
        });
        parallel_for(np, 1 << 16, [&](int64_t p0, int64_t p1, int) {
            for (int64_t p = p0; p < p1; ++p) {
                cnt[p] = acnt[p].load(std::memory_order_relaxed);
                key[p] = akey[p].load(std::memory_order_relaxed);
            }
        });
    }
    {
        const int64_t p = first_where(np, [&](int64_t i) { return cnt[i] < 2; });
        if (p < np)
            throw ba_invalid{"point " + std::to_string(p) + " has " + std::to_string(cnt[p]) +
                             " observations (need >= 2)"};
    }
    const int32_t n_long = (int32_t)std::count_if(cnt.begin(), cnt.end(), [](int32_t t) { return t > kMaxTrack; });
    ph.mark("track counts");
    // internal position -> point: counting sort by key (stable), the points
    // of tracks longer than a wave after all others
    std::vector<int32_t> ord;
    {
        std::vector<int64_t> kc;
        counting_sort(np, 2 * nc, [&](int64_t p) { return (cnt[p] > kMaxTrack ? nc : 0) + key[p]; }, kc, ord);
    }
    c->n_long = n_long;
    c->q_long0 = np - n_long;
    std::vector<int32_t>().swap(key);
    std::vector<int32_t> ptr(np + 1, 0);   // track start by internal position
    std::vector<int32_t> trk(2 * (size_t)np);   // (track start, length) by point, for the permutation
    parallel_for(np, 1 << 16, [&](int64_t q0, int64_t q1, int) {
        for (int64_t q = q0; q < q1; ++q) ptr[q + 1] = cnt[ord[q]];
    });
    for (int32_t q = 0; q < np; ++q) ptr[q + 1] += ptr[q];
    parallel_for(np, 1 << 16, [&](int64_t q0, int64_t q1, int) {
        for (int64_t q = q0; q < q1; ++q) {
            const int32_t p = ord[q];
            trk[2 * (size_t)p] = ptr[q];
            trk[2 * (size_t)p + 1] = cnt[p];
        }
    });
    ph.mark("point order");
    // observations of each track, then sorted by camera: placed by all
    // threads at once (the order inside a track is set by its sort), each
    // track sorted on its own; a camera repeated in a track is an error,
    // reported for the first such track in internal order
    std::vector<int64_t> perm(n);
    {
        std::unique_ptr<std::atomic<int32_t>[]> fill(new std::atomic<int32_t>[np]);
        parallel_for(np, 1 << 16, [&](int64_t p0, int64_t p1, int) {
            for (int64_t p = p0; p < p1; ++p) fill[p].store(trk[2 * (size_t)p], std::memory_order_relaxed);
        });
        parallel_for(n, 1 << 18, [&](int64_t k0, int64_t k1, int) {
            for (int64_t k = k0; k < k1; ++k) perm[fill[pt[k]].fetch_add(1, std::memory_order_relaxed)] = k;
        });
    }
    {
        std::atomic<int32_t> bad{np};   // internal index of the first track with a repeated camera
        parallel_for(np, 1 << 14, [&](int64_t q0, int64_t q1, int) {
            auto less = [&](int64_t x, int64_t y) { return cam[x] < cam[y]; };
            for (int64_t q = q0; q < q1; ++q) {
                int64_t* b = perm.data() + ptr[q];
                int64_t* e = perm.data() + ptr[q + 1];
                if (e - b > 32) {
                    std::sort(b, e, less);
                } else {
                    for (int64_t* i = b + 1; i < e; ++i)
                        for (int64_t* j = i; j > b && less(*j, *(j - 1)); --j) std::swap(*j, *(j - 1));
                }
                for (int64_t* i = b + 1; i < e; ++i)
                    if (cam[*i] == cam[*(i - 1)]) {
                        int32_t cur = bad.load();
                        while ((int32_t)q < cur && !bad.compare_exchange_weak(cur, (int32_t)q)) {}
                        break;
                    }
            }
        });
        const int32_t q = bad.load();
        if (q < np)
            for (int32_t i = ptr[q] + 1; i < ptr[q + 1]; ++i)
                if (cam[perm[i]] == cam[perm[i - 1]])
                    throw ba_invalid{"duplicate observation of point " + std::to_string(ord[q]) + " by camera " +
                                     std::to_string(cam[perm[i]])};
    }
    ph.mark("track sort");
    std::vector<int32_t>().swap(ord);
    std::vector<int32_t>().swap(cnt);
    std::vector<int32_t>().swap(trk);
    std::vector<int32_t> cam_row(nc);
    int32_t nr = 0;
    for (int32_t i = 0; i < nc; ++i) cam_row[i] = (!fixed.empty() && fixed[i]) ? -1 : nr++;
    // shared intrinsics: the physical cameras' interior blocks are rows after
    // the free images' exterior blocks
    const bool shared = c->shared;
    c->n_free = nr;
    if (shared) nr += c->n_phys;
    c->n_rows = nr;
    std::vector<int32_t> ocam(n), orow(n);
    parallel_for(n, 1 << 18, [&](int64_t k0, int64_t k1, int) {
        for (int64_t k = k0; k < k1; ++k) {
            const int32_t cs = cam[perm[k]];
            ocam[k] = cs;
            orow[k] = cam_row[cs];
        }
    });
    ph.mark("permute");
    // point-aligned chunks of at most 64 observations, and the internal index
    // of each chunk's first point
    std::vector<int32_t> chunk{0}, chunk_q{0};
    const int32_t q_long0 = np - n_long;
    for (int32_t q = 0; q < q_long0; ++q)
        if (ptr[q + 1] - chunk.back() > kMaxTrack) {
            chunk.push_back(ptr[q]);
            chunk_q.push_back(q);
        }
    chunk.push_back(ptr[q_long0]);
    c->n_chunk = q_long0 > 0 ? (int32_t)chunk.size() - 1 : 0;
    std::vector<int32_t> long_ptr(ptr.begin() + q_long0, ptr.end());   // [n_long + 1]
    // records: one per observation (J_c, K), or with shared intrinsics two
    // (exterior part at the image's row, interior part at its camera's row);
    // rrow is the RCS row of each record (-1: fixed), rptr the tracks
    const int64_t n_rec = shared ? 2 * n : n;
    std::vector<int32_t> rrow(n_rec), rptr(np + 1);
    parallel_for(n, 1 << 18, [&](int64_t k0, int64_t k1, int) {
        for (int64_t k = k0; k < k1; ++k) {
            if (shared) {
                rrow[2 * k] = orow[k];
                rrow[2 * k + 1] = c->n_free + c->h_img_cam[ocam[k]];
            } else {
                rrow[k] = orow[k];
            }
        }
    });
    for (int32_t q = 0; q <= np; ++q) rptr[q] = shared ? 2 * ptr[q] : ptr[q];
    ph.mark("records");
    // records of each RCS row, in record order, and each record's position
    // in its row's list
    std::vector<int32_t> rowobs_ptr(nr + 1, 0), rowobs;
    std::vector<int32_t> obs_rpos(n_rec, -1);
    {
        std::vector<int64_t> rp64;
        counting_sort(n_rec, nr, [&](int64_t k) { return rrow[k]; }, rp64, rowobs);
        for (int32_t r = 0; r <= nr; ++r) rowobs_ptr[r] = (int32_t)rp64[r];
        parallel_for(nr, 64, [&](int64_t r0, int64_t r1, int) {
            for (int64_t r = r0; r < r1; ++r)
                for (int32_t d = rowobs_ptr[r]; d < rowobs_ptr[r + 1]; ++d) obs_rpos[rowobs[d]] = d;
        });
    }
    ph.mark("row lists");
    // couples of records of a track whose rows differ (each unordered pair
    // once, oriented from the lower row); with shared intrinsics also every
    // ordered pair of records on the same row, itself included: those sum
    // into the diagonal block (a camera's images seeing one point)
    // Built row by row (rows in parallel): the couples (a, b) with a on row
    // r, in record order of a, then b; grouped by the row s of b into
    // segments, one per block (r, s) (s = r: the diagonal block); inside the
    // row the segments are ordered longest first (ties by column), so that
    // lanes sharing a wavefront get similar amounts of work.  Blocks of a
    // row: the diagonal, then the columns s > r in ascending order.
    std::vector<int32_t> rq(n_rec);   // internal point of each record
    parallel_for(np, 1 << 14, [&](int64_t q0, int64_t q1, int) {
        for (int64_t q = q0; q < q1; ++q)
            for (int32_t a = rptr[q]; a < rptr[q + 1]; ++a) rq[a] = (int32_t)q;
    });
    auto scan_row = [&](int32_t r, auto&& visit) {
        for (int32_t i = rowobs_ptr[r]; i < rowobs_ptr[r + 1]; ++i) {
            const int32_t a = rowobs[i], q = rq[a];
            for (int32_t b = shared ? rptr[q] : a + 1; b < rptr[q + 1]; ++b) {
                const int32_t rb = rrow[b];
                if (rb < 0 || (shared && rb < r)) continue;
                visit(a, b, rb);
            }
        }
    };
    const int nth = host_threads();
    std::vector<std::vector<int32_t>> t_cnt(nth, std::vector<int32_t>(nr, 0)), t_blk(nth, std::vector<int32_t>(nr));
    std::vector<std::vector<int64_t>> t_pos(nth, std::vector<int64_t>(nr));
    std::vector<std::vector<int32_t>> t_touch(nth);
    // the row's columns with their couple counts (t_cnt, t_touch)
    auto count_row = [&](int32_t r, int t) {
        std::vector<int32_t>& cnt_s = t_cnt[t];
        std::vector<int32_t>& touch = t_touch[t];
        int64_t m = 0;
        scan_row(r, [&](int32_t, int32_t, int32_t s) {
            if (cnt_s[s]++ == 0) touch.push_back(s);
            ++m;
        });
        return m;
    };
    std::vector<int64_t> ctr(nr + 1, 0), row_ptr(nr + 1, 0);
    std::vector<int32_t> sptr(nr + 1, 0);
    parallel_for(nr, 16, [&](int64_t r0, int64_t r1, int t) {
        for (int64_t r = r0; r < r1; ++r) {
            ctr[r + 1] = count_row((int32_t)r, t);
            int32_t nb = 1;
            for (int32_t s2 : t_touch[t]) {
                if (s2 != r) ++nb;
                t_cnt[t][s2] = 0;
            }
            sptr[r + 1] = (int32_t)t_touch[t].size();
            row_ptr[r + 1] = nb;
            t_touch[t].clear();
        }
    });
    for (int32_t r = 0; r < nr; ++r) {
        ctr[r + 1] += ctr[r];
        sptr[r + 1] += sptr[r];
        row_ptr[r + 1] += row_ptr[r];
    }
    const int64_t ntr = ctr[nr];
    if (ntr > INT32_MAX) throw ba_invalid{"too many camera-pair couples for 32-bit indices"};
    if (row_ptr[nr] > INT32_MAX) throw ba_invalid{"too many RCS blocks for 32-bit indices"};
    const int32_t nseg = sptr[nr];
    std::vector<int32_t> trip(2 * (size_t)ntr), col_idx(row_ptr[nr]);
    std::vector<int32_t> off_blk(nseg), pair_ptr(nseg + 1), seg_row(nseg);
    parallel_for(nr, 16, [&](int64_t r0, int64_t r1, int t) {
        std::vector<int32_t>& cnt_s = t_cnt[t];
        std::vector<int32_t>& blk_s = t_blk[t];
        std::vector<int64_t>& pos_s = t_pos[t];
        std::vector<int32_t>& touch = t_touch[t];
        for (int64_t r = r0; r < r1; ++r) {
            count_row((int32_t)r, t);
            std::sort(touch.begin(), touch.end());
            int64_t kb = row_ptr[r];
            col_idx[kb++] = (int32_t)r;
            for (int32_t s2 : touch) {
                if (s2 == r) {
                    blk_s[s2] = (int32_t)row_ptr[r];
                } else {
                    blk_s[s2] = (int32_t)kb;
                    col_idx[kb++] = s2;
                }
            }
            std::stable_sort(touch.begin(), touch.end(), [&](int32_t x, int32_t y) { return cnt_s[x] > cnt_s[y]; });
            int64_t m = ctr[r];
            int32_t sg = sptr[r];
            for (int32_t s2 : touch) {
                off_blk[sg] = blk_s[s2];
                seg_row[sg] = (int32_t)r;
                pair_ptr[sg] = (int32_t)m;
                pos_s[s2] = m;
                m += cnt_s[s2];
                ++sg;
            }
            scan_row((int32_t)r, [&](int32_t a, int32_t b, int32_t s2) {
                const int64_t d = pos_s[s2]++;
                trip[2 * d] = a;
                trip[2 * d + 1] = b;
            });
            for (int32_t s2 : touch) cnt_s[s2] = 0;
            touch.clear();
        }
    });
    pair_ptr[nseg] = (int32_t)ntr;
    std::vector<int32_t>().swap(rq);
    c->n_blk = row_ptr[nr];
    c->n_offseg = nseg;
    c->n_pairs = ntr;
    ph.mark("couples");
    // pair-stage work units.  One lane group works through a unit's couples
    // one after another, so a long segment would set the stage's duration on
    // small problems: segments longer than the cap are cut into chunks that
    // write partial blocks, summed afterwards in chunk order.  The cap is a
    // quarter of the average work of one of the lane groups the chip holds at
    // once (256 CUs x 16 waves x 4 groups), at least 8 steps of 4 couples.
    // A wave runs until the longest of its four units ends, so inside each
    // camera cluster (below) the units are ordered longest first (neighbouring
    // units have similar lengths); the waves are then cut into 8 contiguous
    // ranges of equal work, one per XCD.
    // The order of the units follows camera clusters: breadth-first growth
    // over the co-visibility graph from the lowest unassigned row, up to
    // about 4 MB of records per cluster (an XCD's L2; 1, 2, 16 and 64 MB
    // measured slower).  A point's track is read by the rows
    // of each of its cameras; inside a compact cluster those rows run close
    // together on one XCD, so the track's records come from L2 / MALL instead
    // of HBM after the first of them.
    std::vector<int32_t> clus(nr, -1);
    {
        std::vector<int32_t> adj_ptr(nr + 1, 0), adj;
        for (int32_t r = 0; r < nr; ++r)
            for (int64_t kb = row_ptr[r] + 1; kb < row_ptr[r + 1]; ++kb) {
                adj_ptr[r + 1]++;
                adj_ptr[col_idx[kb] + 1]++;
            }
        for (int32_t r = 0; r < nr; ++r) adj_ptr[r + 1] += adj_ptr[r];
        adj.resize(adj_ptr[nr]);
        {
            std::vector<int32_t> fill(adj_ptr.begin(), adj_ptr.end() - 1);
            for (int32_t r = 0; r < nr; ++r)
                for (int64_t kb = row_ptr[r] + 1; kb < row_ptr[r + 1]; ++kb) {
                    adj[fill[r]++] = col_idx[kb];
                    adj[fill[col_idx[kb]]++] = r;
                }
        }
        std::vector<int64_t> row_obs(nr, 0);
        for (int64_t k = 0; k < n_rec; ++k)
            if (rrow[k] >= 0) row_obs[rrow[k]]++;
        const double rec = (double)kRec * (c->precision == BA_MIXED ? sizeof(float) : sizeof(double));
        // one XCD's L2 (budgets of 1 to 16 MiB time alike on the 60,000-image
        // partition workload)
        const double budget = 4.0 * (1 << 20);
        std::vector<int32_t> queue;
        int32_t n_cl = 0;
        for (int32_t s0 = 0; s0 < nr; ++s0) {
            if (clus[s0] >= 0) continue;
            queue.assign(1, s0);
            clus[s0] = n_cl;
            double bytes = 0.0;
            for (size_t h = 0; h < queue.size() && bytes < budget; ++h) {
                const int32_t r = queue[h];
                bytes += (double)row_obs[r] * rec;
                for (int32_t e = adj_ptr[r]; e < adj_ptr[r + 1] && bytes < budget; ++e)
                    if (clus[adj[e]] < 0) {
                        clus[adj[e]] = n_cl;
                        queue.push_back(adj[e]);
                    }
            }
            ++n_cl;
        }
    }
    ph.mark("clusters");
    std::vector<int32_t> unit_rng, unit_dst, lseg_blk, lseg_ptr{0};
    {
        struct Unit { int32_t win, t0, t1, dst; };
        std::vector<Unit> units;
        int64_t steps = 0;
        for (int32_t sg = 0; sg < c->n_offseg; ++sg) steps += (pair_ptr[sg + 1] - pair_ptr[sg] + 3) / 4;
        const int64_t groups = 256 * 16 * 4;
        const int64_t cap = 4 * std::max<int64_t>(8, steps / (4 * groups));
        int32_t n_p = 0;
        for (int32_t sg = 0; sg < c->n_offseg; ++sg) {
            const int32_t a = pair_ptr[sg], b = pair_ptr[sg + 1], w = clus[seg_row[sg]];
            if (b - a <= cap) {
                units.push_back({w, a, b, off_blk[sg]});
                continue;
            }
            for (int64_t t = a; t < b; t += cap) {
                units.push_back({w, (int32_t)t, (int32_t)std::min<int64_t>(t + cap, b), -(n_p + 1)});
                ++n_p;
            }
            lseg_blk.push_back(off_blk[sg]);
            lseg_ptr.push_back(n_p);
        }
        std::stable_sort(units.begin(), units.end(), [](const Unit& x, const Unit& y) {
            return x.win != y.win ? x.win < y.win : x.t1 - x.t0 > y.t1 - y.t0;
        });
        const int32_t nu = (int32_t)units.size();
        for (const Unit& u : units) {
            unit_rng.push_back(u.t0);
            unit_rng.push_back(u.t1);
            unit_dst.push_back(u.dst);
        }
        // XCD ranges of equal work: a wave costs its longest unit's steps plus one
        const int32_t nw = (nu + 3) / 4;
        std::vector<int64_t> cum(nw + 1, 0);
        for (int32_t w = 0; w < nw; ++w) {
            int32_t st = 0;
            for (int32_t u = 4 * w; u < std::min(nu, 4 * w + 4); ++u) st = std::max(st, (units[u].t1 - units[u].t0 + 3) / 4);
            cum[w + 1] = cum[w] + st + 1;
        }
        c->xcd_wv[0] = 0;
        for (int x = 1; x < 8; ++x) {
            const int64_t target = cum[nw] * x / 8;
            c->xcd_wv[x] = (int32_t)(std::lower_bound(cum.begin(), cum.end(), target) - cum.begin());
            c->xcd_wv[x] = std::max(c->xcd_wv[x], c->xcd_wv[x - 1]);
        }
        c->xcd_wv[8] = nw;
        c->n_unit = nu;
        c->n_lseg = (int32_t)lseg_blk.size();
        c->n_pblk = n_p;
    }
    ph.mark("units");
    c->h_blk_pairs.assign(c->n_blk, 0);
    for (int32_t sg = 0; sg < c->n_offseg; ++sg)
        if (off_blk[sg] != row_ptr[seg_row[sg]]) c->h_blk_pairs[off_blk[sg]] = pair_ptr[sg + 1] - pair_ptr[sg];
    // both triangles by rows: the row's upper blocks S_rs (column s), then the
    // blocks (s, r), s < r, of its column, transposed (column s)
    std::vector<int32_t> sf_ptr(nr + 1, 0), sf_col, sf_src;
    std::vector<int32_t> lo_ptr, lo_blk;   // upper blocks (s, r), s < r, of each column r
    {
        std::vector<int32_t> trn(nr, 0);
        for (int32_t r = 0; r < nr; ++r)
            for (int64_t kb = row_ptr[r] + 1; kb < row_ptr[r + 1]; ++kb) trn[col_idx[kb]]++;
        for (int32_t r = 0; r < nr; ++r) sf_ptr[r + 1] = sf_ptr[r] + (int32_t)(row_ptr[r + 1] - row_ptr[r]) + trn[r];
        std::vector<int32_t> tr_ptr(nr + 1, 0);
        for (int32_t r = 0; r < nr; ++r) tr_ptr[r + 1] = tr_ptr[r] + trn[r];
        std::vector<int32_t> tr_blk(tr_ptr[nr]), tr_row(tr_ptr[nr]);
        std::vector<int32_t> fill(tr_ptr.begin(), tr_ptr.end() - 1);
        for (int32_t r = 0; r < nr; ++r)   // in row order
            for (int64_t kb = row_ptr[r] + 1; kb < row_ptr[r + 1]; ++kb) {
                const int32_t d = fill[col_idx[kb]]++;
                tr_blk[d] = (int32_t)kb;
                tr_row[d] = r;
            }
        sf_col.resize(sf_ptr[nr]);
        sf_src.resize(sf_ptr[nr]);
        for (int32_t r = 0; r < nr; ++r) {
            int64_t d = sf_ptr[r];
            for (int64_t kb = row_ptr[r]; kb < row_ptr[r + 1]; ++kb, ++d) {
                sf_col[d] = col_idx[kb];
                sf_src[d] = (int32_t)kb << 1;
            }
            for (int32_t t = tr_ptr[r]; t < tr_ptr[r + 1]; ++t, ++d) {
                sf_col[d] = tr_row[t];
                sf_src[d] = (tr_blk[t] << 1) | 1;
            }
        }
        c->n_sf = sf_ptr[nr];
        lo_ptr = std::move(tr_ptr);
        lo_blk = std::move(tr_blk);
    }
    ph.mark("sf/lo lists");
    std::vector<int32_t> row_ptr32(row_ptr.begin(), row_ptr.end());
    // device copies
    upload(c, &c->obs_cam, ocam);
    upload(c, &c->obs_row, orow);
    upload(c, &c->chunk_q, chunk_q);
    upload(c, &c->chunk_ptr, chunk);
    upload(c, &c->long_ptr, long_ptr);
    upload(c, &c->cam_row, cam_row);
    upload(c, &c->row_ptr, row_ptr32);
    upload(c, &c->col_idx, col_idx);
    upload(c, &c->off_blk, off_blk);
    upload(c, &c->pair_ptr, pair_ptr);
    upload(c, &c->trip, trip);
    upload(c, &c->unit_rng, unit_rng);
    upload(c, &c->unit_dst, unit_dst);
    upload(c, &c->lseg_blk, lseg_blk);
    upload(c, &c->lseg_ptr, lseg_ptr);
    upload(c, &c->rowobs_ptr, rowobs_ptr);
    upload(c, &c->rowobs, rowobs);
    upload(c, &c->obs_rpos, obs_rpos);
    upload(c, &c->sf_ptr, sf_ptr);
    upload(c, &c->sf_col, sf_col);
    upload(c, &c->sf_src, sf_src);
    upload(c, &c->lo_ptr, lo_ptr);
    upload(c, &c->lo_blk, lo_blk);
    if (shared) upload(c, &c->img_cam, c->h_img_cam);
    BA_HIP_CHECK(hipStreamSynchronize(c->stream));
    ph.mark("uploads");
    c->h_row_ptr = std::move(row_ptr);
    c->h_col_idx = std::move(col_idx);
    c->h_perm = std::move(perm);
    // workspace
    const size_t es = c->precision == BA_MIXED ? sizeof(float) : sizeof(double);
    dalloc(c, (char**)&c->R, (size_t)n_rec * kRec * es);
    dalloc(c, (char**)&c->Jp, (size_t)n * 6 * es);
    dalloc(c, &c->e, (size_t)n * 2);
    dalloc(c, &c->ptL, (size_t)np * 9);
    // e + K lhat: in row-list order, or (shared intrinsics) by observation
    dalloc(c, &c->ebar, (size_t)(shared ? n : rowobs_ptr[nr]) * 2);
    dalloc(c, &c->pblk, (size_t)c->n_pblk * 81);
    dalloc(c, &c->blk, (size_t)c->n_blk * 81);
    dalloc(c, &c->Sf, (size_t)c->n_sf * 81);
    dalloc(c, &c->rhs, (size_t)nr * 9);
    dalloc(c, &c->Minv, (size_t)nr * 81);
    dalloc(c, &c->Linv, (size_t)nr * 81);
    dalloc(c, &c->dxc, (size_t)nr * 9);
    dalloc(c, &c->dxp, (size_t)np * 3);
    // per-block partials of up to three sums: grids of one block per 256
    // observations, or per chunk at most (chunk-based kernels), plus one per
    // long track
    c->n_part = (int32_t)(3 * std::max<int64_t>((n + 255) / 256, (int64_t)c->n_chunk + c->n_long) + 8);
    dalloc(c, &c->part, (size_t)c->n_part);
    dalloc(c, &c->part2, (size_t)3 * ba::kReduceParts);
    dalloc(c, &c->scal, 16);
    dalloc(c, &c->flags, 8);
    dalloc(c, &c->tri_failed, 1);
    Pcg& P = c->pcg;
    dalloc(c, &P.x, (size_t)nr * 9);
    dalloc(c, &P.r[0], (size_t)nr * 9);
    dalloc(c, &P.r[1], (size_t)nr * 9);
    dalloc(c, &P.z, (size_t)nr * 9);
    dalloc(c, &P.q, (size_t)nr * 9);
    dalloc(c, &P.d, (size_t)nr * 9);
    dalloc(c, &P.t, (size_t)nr * 9);
    dalloc(c, &P.u, (size_t)nr * 9);
    dalloc(c, &P.tb, (size_t)c->n_blk * 9);
    dalloc(c, &P.bm, 8 + 49);
    dalloc(c, &P.pA, 1024);
    dalloc(c, &P.pR, 2 * 9 * 1024);
    dalloc(c, &P.W, (size_t)nr * 63);
    dalloc(c, &P.SW, (size_t)nr * 63);
    dalloc(c, &P.Einv, 49);
    dalloc(c, &P.pW, 7 * 1024);
    dalloc(c, &P.pE, 49 * 1024);
    dalloc(c, &c->lin_cams, (size_t)c->n_cams * 9);
    dalloc(c, &P.state, 8);
    dalloc(c, &P.scal, 8);
    BA_HIP_CHECK(hipHostMalloc((void**)&c->h_scal, 32 * sizeof(double), hipHostMallocDefault));
    BA_HIP_CHECK(hipHostMalloc((void**)&c->h_flags, 16 * sizeof(int), hipHostMallocDefault));
    for (auto& e : c->ev) BA_HIP_CHECK(hipEventCreate(&e));
    BA_HIP_CHECK(hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking));
    if (const char* g = std::getenv("BA_PCG_GRAPHS")) c->use_graphs = std::atoi(g) != 0;
    ph.mark("workspace");
    // point ids and pixels in the internal order, gathered on the device
    // (the permutation travels in the record buffer, written only later)
    {
        dalloc(c, &c->obs_pt, (size_t)n);
        dalloc(c, &c->obs_uv, (size_t)n * 2);
        std::vector<int32_t> perm32(n);
        parallel_for(n, 1 << 18, [&](int64_t k0, int64_t k1, int) {
            for (int64_t k = k0; k < k1; ++k) perm32[k] = (int32_t)c->h_perm[k];
        });
        int32_t* d_perm = (int32_t*)c->R;
        BA_HIP_CHECK(hipMemcpyAsync(d_perm, perm32.data(), (size_t)n * sizeof(int32_t), hipMemcpyHostToDevice,
                                    c->stream));
        unsigned long long* d_bad = reinterpret_cast<unsigned long long*>(c->part);
        BA_HIP_CHECK(hipMemsetAsync(d_bad, 0xff, sizeof(unsigned long long), c->stream));
        ba::launch_gather_obs(c, d_perm, d_pt, d_uv, d_bad);
        unsigned long long bad = 0;
        BA_HIP_CHECK(hipMemcpyAsync(&bad, d_bad, sizeof(bad), hipMemcpyDeviceToHost, c->stream));
        BA_HIP_CHECK(hipStreamSynchronize(c->stream));
        if (bad < (unsigned long long)n)
            throw ba_invalid{"obs_uv of observation " + std::to_string(bad) + " is not finite"};
    }
    ph.mark("gather");
}

template <typename F>
ba_status guarded(ba_ctx* c, F&& f) {
    try {
        return f();
    } catch (const ba_oom& e) {
        if (c) c->err = e.what;
        return BA_ERR_OUT_OF_MEMORY;
    } catch (const ba_invalid& e) {
        if (c) c->err = e.what;
        return BA_ERR_INVALID_ARG;
    } catch (const ba_hip_error& e) {
        if (c) c->err = e.what;
        return BA_ERR_DEVICE;
    } catch (const std::bad_alloc&) {
        if (c) c->err = "host allocation failed";
        return BA_ERR_OUT_OF_MEMORY;
    } catch (...) {
        if (c) c->err = "unexpected exception";
        return BA_ERR_DEVICE;
    }
}

float elapsed(hipEvent_t a, hipEvent_t b) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, a, b) != hipSuccess) return 0.f;
    return ms;
}

// point_done: the point stage already ran, fused with the linearization
ba_status form_rcs_async(ba_ctx* c, double lambda, bool point_done = false) {
    if (!point_done) {
        // flags[2] (records out of range) belongs to the linearization and stays
        BA_HIP_CHECK(hipMemsetAsync(c->flags, 0, 2 * sizeof(int), c->stream));
        BA_HIP_CHECK(hipMemsetAsync(c->flags + 3, 0, 5 * sizeof(int), c->stream));
    }
    BA_HIP_CHECK(hipEventRecord(c->ev[1], c->stream));
    if (!point_done) {
        if (c->shared)   // the point terms need the Jacobians again: one fused pass
            ba::launch_linpoint_shared(c, c->lin_params, c->lin_pts, lambda);
        else
            ba::launch_point(c, lambda);
    }
    BA_HIP_CHECK(hipEventRecord(c->ev[2], c->stream));
    ba::launch_offdiag(c);
    BA_HIP_CHECK(hipEventRecord(c->ev[3], c->stream));
    if (c->shared)
        ba::launch_node_diag(c, lambda);
    else
        ba::launch_diag(c, lambda);
    BA_HIP_CHECK(hipEventRecord(c->ev[4], c->stream));
    BA_HIP_CHECK(hipGetLastError());
    c->have_rcs = true;
    c->sf_ready = false;
    c->sf32_ready = false;
    c->su32_ready = false;
    c->fs.ready = false;
    c->defl_ready = false;
    c->csr.ready = false;
    c->lambda = lambda;
    return BA_OK;
}

// parameters of a shared-intrinsics context: [n_cams][6] then [n_phys][5]
size_t n_params(const ba_ctx* c) { return 6 * (size_t)c->n_cams + 5 * (size_t)c->n_phys; }

// selects the S copy and the product layout of the next solve (allocating
// the FP32 copies on first use)
void select_solver_matrix(ba_ctx* c, int fp32, int product) {
    c->s32 = fp32 ? 1 : 0;
    const double full_bytes = (double)c->n_sf * 81 * (c->s32 ? sizeof(float) : sizeof(double));
    c->upper = (product == BA_PRODUCT_UPPER || (product == BA_PRODUCT_AUTO && full_bytes > 256.0 * (1 << 20))) ? 1 : 0;
    if (c->s32 && !c->Sf32) dalloc(c, &c->Sf32, (size_t)std::max<int64_t>(c->n_sf, 1) * 81);
    if (c->upper && c->s32 && !c->Su32) dalloc(c, &c->Su32, (size_t)c->n_blk * 81);
}

void prepare_defl(ba_ctx* c) {
    if (c->defl_ready && c->defl_s32 != c->s32) c->defl_ready = false;
    if (!c->defl_ready) {
        ba::prepare_deflation(c);
        BA_HIP_CHECK(hipGetLastError());
        c->defl_ready = true;
    }
}

// the network's factor of the current RCS into the FSAI layouts
void prepare_learned_fsai(ba_ctx* c) {
    if (!c->fs.built) ba::build_fsai(c);
    auto* g = (ba::gnn::Graph*)c->lgraph;
    ba::gnn::compute_features(*g, c->blk, c->stream);
    // the UPPER apply reads the FP16 copy only; FULL reads Gl and Gu
    c->fs.half = c->upper;
    if (c->fs.half) ba::launch_dscale(c);
    ba::gnn::infer_factor(c->net, *g, c->upper ? c->fs.gl_self : c->fs.gu_pos, c->upper ? nullptr : c->fs.Gl,
                          c->upper ? nullptr : c->fs.Gu, c->fs.G, c->stream, c->fs.half ? c->fs.Dn : nullptr,
                          c->fs.half ? c->fs.Gh : nullptr, c->fs.half ? c->fs.Gh8 : nullptr, c->fs.hs);
    c->fs.gu_upper = c->upper;
    c->fs.ready = false;   // the layouts now hold the network's factor
}

// the FSAI factor of the current RCS (index structure on first use)
void prepare_fsai(ba_ctx* c) {
    if (!c->fs.built) ba::build_fsai(c);
    if (c->fs.ready && c->fs.gu_upper != c->upper) c->fs.ready = false;
    if (!c->fs.ready) {
        ba::launch_fsai(c);
        c->fs.half = c->upper;
        if (c->fs.half) {
            ba::launch_dscale(c);
            ba::launch_pack_half(c);
        }
        BA_HIP_CHECK(hipGetLastError());
        c->fs.ready = true;
    }
}

// a learned preconditioner gave a solve that cannot be used: d^T S d was
// not positive (non-finite or indefinite preconditioner) or the residual is
// not finite; block-Jacobi then solves the system instead
bool learned_failed(int pre, ba_status s, double relres) {
    return (pre == BA_PRECOND_LEARNED || pre == BA_PRECOND_LEARNED_FSAI) &&
           (s == BA_ERR_NOT_SPD || !std::isfinite(relres));
}

// the CSR copy of the current RCS (index structure on first use)
void prepare_csr(ba_ctx* c) {
    if (!c->csr.built) ba::build_csr(c);
    if (!c->csr.ready) {
        ba::launch_csr_fill(c);
        BA_HIP_CHECK(hipGetLastError());
        c->csr.ready = true;
    }
}

// network inference on the current RCS -> Mlearn (context stream)
void prepare_learned(ba_ctx* c) {
    auto* g = (ba::gnn::Graph*)c->lgraph;
    ba::gnn::compute_features(*g, c->blk, c->stream);
    ba::gnn::infer_preconditioner(c->net, *g, c->Minv, c->Mlearn, c->stream);
}

}  // namespace

namespace ba {

// Index structure of the FSAI factor (host, once per context): the sets J_i
// (lower neighbours with the most common points, ties to the lower index,
// then ascending, then i), the G slot of each member, the local tiles and
// the gather lists of G (lower, per row) and G^T (upper, per row).
void build_fsai(ba_ctx* c) {
    Phases ph("build_fsai");
    const int32_t nr = c->n_rows;
    const std::vector<int64_t>& rp = c->h_row_ptr;
    const std::vector<int32_t>& ci = c->h_col_idx;
    const std::vector<int32_t>& cnt = c->h_blk_pairs;
    std::vector<int32_t> brow(c->n_blk);
    for (int32_t r = 0; r < nr; ++r)
        for (int64_t kb = rp[r]; kb < rp[r + 1]; ++kb) brow[kb] = r;
    std::vector<int32_t> ptr, J, slot, tile;
    ph.mark("rows");
    ba::gnn::fsai_sets(nr, rp.data(), ci.data(), cnt.data(), ptr, J, slot);
    ph.mark("sets");
    // local tiles of each set (rows in parallel): for members a >= b of
    // J_i the block (J_b, J_a) (-2 on the diagonal, -1 if not stored)
    std::vector<int64_t> tptr(nr + 1, 0);
    int32_t max_m = 1;
    for (int32_t i = 0; i < nr; ++i) {
        const int32_t m = ptr[i + 1] - ptr[i];
        max_m = std::max(max_m, m);
        tptr[i + 1] = tptr[i] + (int64_t)m * (m + 1) / 2;
    }
    tile.resize(tptr[nr]);
    ba::parallel_for(nr, 256, [&](int64_t i0, int64_t i1, int) {
        for (int64_t i = i0; i < i1; ++i) {
            const int32_t m = ptr[i + 1] - ptr[i];
            const int32_t* Jm = J.data() + ptr[i];
            int64_t d = tptr[i];
            for (int32_t a = 0; a < m; ++a)
                for (int32_t b = 0; b <= a; ++b, ++d) {
                    if (a == b) {
                        tile[d] = -2;
                        continue;
                    }
                    const int32_t jb = Jm[b], ja = Jm[a];   // jb < ja: upper block (jb, ja)
                    auto first = ci.begin() + rp[jb] + 1, last = ci.begin() + rp[jb + 1];
                    auto it = std::lower_bound(first, last, ja);
                    tile[d] = it != last && *it == ja ? (int32_t)(it - ci.begin()) : -1;
                }
        }
    });
    ph.mark("tiles");
    // rows of G^T: row j lists (i, member) for every set J_i containing j, in
    // i order (a stable counting sort of the members by J)
    std::vector<int32_t> mem_row(J.size());
    for (int32_t i = 0; i < nr; ++i)
        for (int32_t e = ptr[i]; e < ptr[i + 1]; ++e) mem_row[e] = i;
    std::vector<int64_t> gp64;
    std::vector<int32_t> gu_list;
    ba::counting_sort((int64_t)J.size(), nr, [&](int64_t e) { return J[e]; }, gp64, gu_list);
    std::vector<int32_t> gu_ptr(nr + 1, 0), gu_col(gu_list.size()), gu_pos(J.size());
    for (int32_t j = 0; j <= nr; ++j) gu_ptr[j] = (int32_t)gp64[j];
    for (size_t d = 0; d < gu_list.size(); ++d) {
        gu_col[d] = mem_row[gu_list[d]];
        gu_pos[gu_list[d]] = (int32_t)d;
    }
    ph.mark("transpose");
    Fsai& F = c->fs;
    upload(c, &F.ptr, ptr);
    upload(c, &F.J, J);
    upload(c, &F.slot, slot);
    upload(c, &F.tptr, tptr);
    upload(c, &F.tile, tile);
    upload(c, &F.brow, brow);
    upload(c, &F.gu_ptr, gu_ptr);
    upload(c, &F.gu_col, gu_col);
    upload(c, &F.gu_pos, gu_pos);
    std::vector<int32_t> gu_src(gu_pos.size());
    for (size_t p = 0; p < gu_pos.size(); ++p) gu_src[gu_pos[p]] = (int32_t)p;
    upload(c, &F.gu_src, gu_src);
    std::vector<int32_t> gl_self(gu_pos.size());
    for (size_t p = 0; p < gl_self.size(); ++p) gl_self[p] = (int32_t)p;
    upload(c, &F.gl_self, gl_self);
    F.max_m = max_m;
    F.n_mem = (int64_t)J.size();
    dalloc(c, &F.Gl, J.size() * 81);
    dalloc(c, &F.Gu, J.size() * 81);
    dalloc(c, &F.tg, J.size() * 9);
    // 36 words of groups per member, then the row-8 halves (9 per member)
    dalloc(c, &F.Gh, J.size() * 36 + (J.size() * 9 + 1) / 2);
    F.Gh8 = reinterpret_cast<uint16_t*>(F.Gh + J.size() * 36);
    dalloc(c, &F.hs, J.size());
    dalloc(c, &F.Dn, (size_t)nr * 9);
    dalloc(c, &F.An, (size_t)c->n_blk * 81);
    dalloc(c, &F.G, (size_t)c->n_blk * 81);
    BA_HIP_CHECK(hipMemsetAsync(F.G, 0, (size_t)c->n_blk * 81 * sizeof(float), c->stream));
    ph.mark("upload+alloc");
    F.built = true;
}

// Index structure of the CSR copy (host, once per context): per block row
// its slots in ascending column order (the transposed blocks (s, r), s < r,
// of column r, then the row's own upper blocks, diagonal first), each
// slot's source block (<< 1 | transposed), block column and row, and the
// scalar row pointer (row 9 r + a starts at 81 P_r + 9 m_r a for the P_r
// slots before row r and the m_r slots of row r).
void build_csr(ba_ctx* c) {
    const int32_t nr = c->n_rows;
    const std::vector<int64_t>& rp = c->h_row_ptr;
    const std::vector<int32_t>& ci = c->h_col_idx;
    std::vector<std::vector<int32_t>> lower(nr);
    std::vector<int32_t> brow(c->n_blk);
    for (int32_t r = 0; r < nr; ++r)
        for (int64_t kb = rp[r]; kb < rp[r + 1]; ++kb) {
            brow[kb] = r;
            if (kb > rp[r]) lower[ci[kb]].push_back((int32_t)kb);
        }
    std::vector<int32_t> bptr(nr + 1, 0), src, col, row;
    for (int32_t r = 0; r < nr; ++r) {
        for (int32_t kb : lower[r]) {
            src.push_back(kb << 1 | 1);
            col.push_back(brow[kb]);
            row.push_back(r);
        }
        for (int64_t kb = rp[r]; kb < rp[r + 1]; ++kb) {
            src.push_back((int32_t)kb << 1);
            col.push_back(ci[kb]);
            row.push_back(r);
        }
        bptr[r + 1] = (int32_t)src.size();
    }
    const int64_t nnz = 81 * (int64_t)src.size();
    if (nnz >= INT32_MAX) throw ba_invalid{"the CSR copy would need 2^31 or more non-zeros"};
    std::vector<int32_t> rowptr(9 * (size_t)nr + 1);
    for (int32_t r = 0; r < nr; ++r) {
        const int64_t m = bptr[r + 1] - bptr[r];
        for (int a = 0; a < 9; ++a) rowptr[9 * (size_t)r + a] = (int32_t)(81 * (int64_t)bptr[r] + 9 * m * a);
    }
    rowptr[9 * (size_t)nr] = (int32_t)nnz;
    Csr& C = c->csr;
    upload(c, &C.bptr, bptr);
    upload(c, &C.slot_src, src);
    upload(c, &C.slot_col, col);
    upload(c, &C.slot_row, row);
    upload(c, &C.rowptr, rowptr);
    dalloc(c, &C.col, (size_t)nnz);
    dalloc(c, &C.val, (size_t)nnz);
    C.n_slot = (int64_t)src.size();
    C.nnz = nnz;
    C.built = true;
}

}  // namespace ba

extern "C" {

ba_status ba_set_preconditioner_net(ba_ctx* c, ba_gnn* net) {
    if (!c) return BA_ERR_INVALID_ARG;
    if (c->shared && net) { c->err = "the network is trained on 9-parameter camera blocks"; return BA_ERR_INVALID_ARG; }
    return guarded(c, [&]() {
        c->net = net;
        c->learned_ready = net != nullptr;
        if (net && !c->Mlearn) dalloc(c, &c->Mlearn, (size_t)c->n_rows * 81);
        if (net && !c->lgraph && c->n_rows > 0) {
            auto* g = new ba::gnn::Graph();
            ba::gnn::build_graph(*g, c->n_rows, c->h_row_ptr.data(), c->h_col_idx.data(), c->h_blk_pairs.data(),
                                 c->stream);
            c->lgraph = g;
        }
        return BA_OK;
    });
}

ba_status ba_gnn_graph_from_ctx(ba_ctx* c, ba_gnn_graph** out) {
    if (!c || !out) return BA_ERR_INVALID_ARG;
    *out = nullptr;
    if (!c->have_rcs) { c->err = "no RCS formed"; return BA_ERR_STATE; }
    if (c->n_rows == 0) { c->err = "no free cameras"; return BA_ERR_INVALID_ARG; }
    ba_gnn_graph* G = new ba_gnn_graph();
    ba_status s = guarded(c, [&]() {
        ba::gnn::build_graph(G->g, c->n_rows, c->h_row_ptr.data(), c->h_col_idx.data(), c->h_blk_pairs.data(),
                             c->stream);
        ba::gnn::compute_features(G->g, c->blk, c->stream);
        BA_HIP_CHECK(hipStreamSynchronize(c->stream));
        return BA_OK;
    });
    if (s != BA_OK) {
        ba::gnn::free_graph(G->g);
        delete G;
        return s;
    }
    *out = G;
    return BA_OK;
}

const char* ba_status_str(ba_status s) {
    switch (s) {
        case BA_OK: return "ok";
        case BA_ERR_INVALID_ARG: return "invalid argument";
        case BA_ERR_STATE: return "call out of order";
        case BA_ERR_NOT_SPD: return "matrix not positive definite";
        case BA_ERR_NOT_CONVERGED: return "PCG did not converge";
        case BA_ERR_OUT_OF_MEMORY: return "out of memory";
        case BA_ERR_DEVICE: return "HIP runtime error";
        case BA_ERR_RANGE: return "value outside the range of the record type";
    }
    return "unknown status";
}

const char* ba_last_error(const ba_ctx* ctx) { return ctx ? ctx->err.c_str() : g_create_error.c_str(); }

ba_status ba_create(const ba_problem_desc* d, ba_ctx** out) {
    if (out) *out = nullptr;
    g_create_error.clear();
    if (!d || !out) { g_create_error = "null descriptor or output"; return BA_ERR_INVALID_ARG; }
    if (d->n_cams <= 0 || d->n_pts <= 0 || d->n_obs <= 0 || d->n_obs >= INT32_MAX) {
        g_create_error = "sizes must satisfy n_cams > 0, n_pts > 0, 0 < n_obs < 2^31";
        return BA_ERR_INVALID_ARG;
    }
    if (!d->obs_cam || !d->obs_pt || !d->obs_uv) { g_create_error = "null observation arrays"; return BA_ERR_INVALID_ARG; }
    if (d->precision != BA_FP64 && d->precision != BA_MIXED) { g_create_error = "unknown precision"; return BA_ERR_INVALID_ARG; }
    ba_ctx* c = new ba_ctx();
    c->n_cams = d->n_cams;
    c->n_pts = d->n_pts;
    c->n_obs = d->n_obs;
    c->precision = d->precision;
    c->stream = (hipStream_t)d->stream;
    c->cap = d->workspace_cap;
    ba_status st = guarded(c, [&]() {
        BA_HIP_CHECK(hipGetDevice(&c->device));
        const int64_t n = c->n_obs;
        std::vector<int32_t> cam(n), pt(n);
        std::vector<uint8_t> fixed;
        BA_HIP_CHECK(hipMemcpyAsync(cam.data(), d->obs_cam, n * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
        BA_HIP_CHECK(hipMemcpyAsync(pt.data(), d->obs_pt, n * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
        if (d->cam_fixed) {
            fixed.resize(c->n_cams);
            BA_HIP_CHECK(hipMemcpyAsync(fixed.data(), d->cam_fixed, c->n_cams, hipMemcpyDeviceToHost, c->stream));
        }
        BA_HIP_CHECK(hipStreamSynchronize(c->stream));
        build(c, cam, pt, d->obs_pt, d->obs_uv, fixed);
        return BA_OK;
    });
    if (st != BA_OK) {
        g_create_error = c->err;
        free_ctx(c);
        return st;
    }
    *out = c;
    return BA_OK;
}

ba_status ba_create_shared(const ba_shared_desc* d, ba_ctx** out) {
    if (out) *out = nullptr;
    g_create_error.clear();
    if (!d || !out) { g_create_error = "null descriptor or output"; return BA_ERR_INVALID_ARG; }
    if (d->n_imgs <= 0 || d->n_phys <= 0 || d->n_pts <= 0 || d->n_obs <= 0 || d->n_obs >= INT32_MAX / 2) {
        g_create_error = "sizes must satisfy n_imgs, n_phys, n_pts > 0 and 0 < n_obs < 2^30";
        return BA_ERR_INVALID_ARG;
    }
    if (!d->obs_img || !d->obs_pt || !d->obs_uv || !d->img_cam) {
        g_create_error = "null observation or camera arrays";
        return BA_ERR_INVALID_ARG;
    }
    ba_ctx* c = new ba_ctx();
    c->n_cams = d->n_imgs;
    c->n_pts = d->n_pts;
    c->n_obs = d->n_obs;
    c->precision = BA_FP64;
    c->stream = (hipStream_t)d->stream;
    c->cap = d->workspace_cap;
    c->shared = true;
    c->n_phys = d->n_phys;
    ba_status st = guarded(c, [&]() {
        BA_HIP_CHECK(hipGetDevice(&c->device));
        const int64_t n = c->n_obs;
        std::vector<int32_t> cam(n), pt(n);
        std::vector<uint8_t> fixed;
        c->h_img_cam.resize(c->n_cams);
        BA_HIP_CHECK(hipMemcpyAsync(cam.data(), d->obs_img, n * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
        BA_HIP_CHECK(hipMemcpyAsync(pt.data(), d->obs_pt, n * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
        BA_HIP_CHECK(hipMemcpyAsync(c->h_img_cam.data(), d->img_cam, c->n_cams * sizeof(int32_t),
                                    hipMemcpyDeviceToHost, c->stream));
        if (d->img_fixed) {
            fixed.resize(c->n_cams);
            BA_HIP_CHECK(hipMemcpyAsync(fixed.data(), d->img_fixed, c->n_cams, hipMemcpyDeviceToHost, c->stream));
        }
        BA_HIP_CHECK(hipStreamSynchronize(c->stream));
        for (int32_t i = 0; i < c->n_cams; ++i)
            if (c->h_img_cam[i] < 0 || c->h_img_cam[i] >= c->n_phys)
                throw ba_invalid{"img_cam[" + std::to_string(i) + "] out of range"};
        build(c, cam, pt, d->obs_pt, d->obs_uv, fixed);
        dalloc(c, &c->lin_params, n_params(c));
        dalloc(c, &c->lin_pts, (size_t)c->n_pts * 3);
        return BA_OK;
    });
    if (st != BA_OK) {
        g_create_error = c->err;
        free_ctx(c);
        return st;
    }
    *out = c;
    return BA_OK;
}

void ba_destroy(ba_ctx* ctx) {
    if (!ctx) return;
    (void)hipStreamSynchronize(ctx->stream);
    free_ctx(ctx);
}

ba_status ba_get_sizes(const ba_ctx* c, ba_sizes* o) {
    if (!c || !o) return BA_ERR_INVALID_ARG;
    o->n_cams = c->n_cams; o->n_pts = c->n_pts; o->n_rows = c->n_rows; o->precision = c->precision;
    o->n_obs = c->n_obs; o->n_blk = c->n_blk; o->n_pairs = c->n_pairs; o->device_bytes = (int64_t)c->bytes;
    return BA_OK;
}

ba_status ba_project(const double* cams, const double* pts, const int32_t* obs_cam, const int32_t* obs_pt, int64_t n_obs,
                     const double* noise, double* uv, void* stream) {
    if (n_obs < 0 || (n_obs > 0 && (!cams || !pts || !obs_cam || !obs_pt || !uv))) return BA_ERR_INVALID_ARG;
    ba::launch_project(cams, pts, obs_cam, obs_pt, n_obs, noise, uv, (hipStream_t)stream);
    return hipGetLastError() == hipSuccess ? BA_OK : BA_ERR_DEVICE;
}

ba_status ba_triangulate(ba_ctx* c, const double* cams, double* pts, int32_t linear_init, int32_t n_gn,
                         int64_t* n_failed) {
    if (!c) return BA_ERR_INVALID_ARG;
    if (c->shared) { c->err = "ba_triangulate takes 9-parameter cameras"; return BA_ERR_INVALID_ARG; }
    if (!cams || !pts) { c->err = "null parameter arrays"; return BA_ERR_INVALID_ARG; }
    if (n_gn < 0 || n_gn > 100) { c->err = "n_gn must be 0..100"; return BA_ERR_INVALID_ARG; }
    return guarded(c, [&]() {
        BA_HIP_CHECK(hipMemsetAsync(c->tri_failed, 0, sizeof(int), c->stream));
        ba::launch_triangulate(c, cams, nullptr, pts, pts, 0, linear_init ? 1 : 0, n_gn, c->tri_failed);
        BA_HIP_CHECK(hipGetLastError());
        BA_HIP_CHECK(hipMemcpyAsync(c->h_flags + 3, c->tri_failed, sizeof(int), hipMemcpyDeviceToHost, c->stream));
        BA_HIP_CHECK(hipStreamSynchronize(c->stream));
        if (n_failed) *n_failed = c->h_flags[3];
        return BA_OK;
    });
}

ba_status ba_linearize(ba_ctx* c, const double* cams, const double* pts, double* cost_host) {
    if (!c) return BA_ERR_INVALID_ARG;
    if (!cams || !pts) { c->err = "null parameter arrays"; return BA_ERR_INVALID_ARG; }
    return guarded(c, [&]() {
        BA_HIP_CHECK(hipEventRecord(c->ev[0], c->stream));
        BA_HIP_CHECK(hipMemsetAsync(c->flags + 2, 0, sizeof(int), c->stream));
        if (c->shared) {
            // the Jacobians are formed again with the damping by ba_form_rcs
            // (one fused pass); the parameters are kept for it
            BA_HIP_CHECK(hipMemcpyAsync(c->lin_params, cams, n_params(c) * sizeof(double), hipMemcpyDeviceToDevice,
                                        c->stream));
            BA_HIP_CHECK(hipMemcpyAsync(c->lin_pts, pts, (size_t)c->n_pts * 3 * sizeof(double),
                                        hipMemcpyDeviceToDevice, c->stream));
            ba::launch_linpoint_shared(c, c->lin_params, c->lin_pts, 0.0);
        } else {
            ba::launch_linearize(c, cams, pts);
            BA_HIP_CHECK(hipMemcpyAsync(c->lin_cams, cams, (size_t)c->n_cams * 9 * sizeof(double),
                                        hipMemcpyDeviceToDevice, c->stream));
        }
        c->defl_ready = false;
        BA_HIP_CHECK(hipEventRecord(c->ev[5], c->stream));
        BA_HIP_CHECK(hipGetLastError());
        c->have_lin = true;
        c->have_rcs = false;
        if (cost_host) {
            BA_HIP_CHECK(hipMemcpyAsync(c->h_scal, c->scal, sizeof(double), hipMemcpyDeviceToHost, c->stream));
            BA_HIP_CHECK(hipMemcpyAsync(c->h_flags + 2, c->flags + 2, sizeof(int), hipMemcpyDeviceToHost, c->stream));
            BA_HIP_CHECK(hipStreamSynchronize(c->stream));
            *cost_host = c->h_scal[0];
            if (c->h_flags[2]) { c->err = kRangeMsg; return BA_ERR_RANGE; }
        }
        return BA_OK;
    });
}

ba_status ba_form_rcs(ba_ctx* c, double lambda) {
    if (!c) return BA_ERR_INVALID_ARG;
    if (!c->have_lin) { c->err = "ba_form_rcs needs a prior ba_linearize"; return BA_ERR_STATE; }
    if (!(lambda >= 0.0) || !std::isfinite(lambda)) { c->err = "lambda must be finite and >= 0"; return BA_ERR_INVALID_ARG; }
    return guarded(c, [&]() {
        form_rcs_async(c, lambda);
        BA_HIP_CHECK(hipMemcpyAsync(c->h_flags, c->flags, 3 * sizeof(int), hipMemcpyDeviceToHost, c->stream));
        BA_HIP_CHECK(hipStreamSynchronize(c->stream));
        if (c->h_flags[2]) { c->err = kRangeMsg; return BA_ERR_RANGE; }
        if (c->h_flags[0]) { c->err = "a damped point block V* is not positive definite"; return BA_ERR_NOT_SPD; }
        if (c->h_flags[1]) { c->err = "an RCS diagonal block is not positive definite"; return BA_ERR_NOT_SPD; }
        return BA_OK;
    });
}

ba_status ba_get_stage_ms(ba_ctx* c, double* ms) {
    if (!c || !ms) return BA_ERR_INVALID_ARG;
    return guarded(c, [&]() {
        BA_HIP_CHECK(hipStreamSynchronize(c->stream));
        ms[0] = elapsed(c->ev[0], c->ev[5]);
        ms[1] = elapsed(c->ev[1], c->ev[2]);
        ms[2] = elapsed(c->ev[2], c->ev[3]);
        ms[3] = elapsed(c->ev[3], c->ev[4]);
        return BA_OK;
    });
}

ba_status ba_pcg_solve(ba_ctx* c, const ba_pcg_opts* o, double* dxc, ba_pcg_info* info) {
    if (!c) return BA_ERR_INVALID_ARG;
    if (!c->have_rcs) { c->err = "ba_pcg_solve needs a formed RCS"; return BA_ERR_STATE; }
    if (!dxc) { c->err = "null dxc"; return BA_ERR_INVALID_ARG; }
    const double tol = o ? o->tol : 1e-6;
    const int max_iter = o ? o->max_iter : 1000;
    const int pre = o ? o->precond : BA_PRECOND_BLOCK_JACOBI;
    if (!(tol >= 0.0) || max_iter < 0) { c->err = "tol must be >= 0 and max_iter >= 0"; return BA_ERR_INVALID_ARG; }
    if (o && (o->product < BA_PRODUCT_AUTO || o->product > BA_PRODUCT_UPPER)) {
        c->err = "unknown product layout";
        return BA_ERR_INVALID_ARG;
    }
    if ((pre == BA_PRECOND_LEARNED || pre == BA_PRECOND_LEARNED_FSAI) && !c->learned_ready) {
        c->err = "no learned preconditioner set";
        return BA_ERR_STATE;
    }
    if (pre != BA_PRECOND_LEARNED && pre != BA_PRECOND_BLOCK_JACOBI && pre != BA_PRECOND_FSAI &&
        pre != BA_PRECOND_LEARNED_FSAI) {
        c->err = "unknown preconditioner";
        return BA_ERR_INVALID_ARG;
    }
    if (c->shared && ((o && o->deflate) || pre == BA_PRECOND_LEARNED || pre == BA_PRECOND_LEARNED_FSAI)) {
        c->err = "shared-intrinsics contexts take block-Jacobi or FSAI, without deflation";
        return BA_ERR_INVALID_ARG;
    }
    return guarded(c, [&]() {
        int it = 0;
        double rr = 0.0;
        select_solver_matrix(c, o ? o->solver_fp32 : 0, o ? o->product : BA_PRODUCT_AUTO);
        if (pre == BA_PRECOND_LEARNED && c->n_rows > 0) prepare_learned(c);
        if (pre == BA_PRECOND_FSAI && c->n_rows > 0) prepare_fsai(c);
        if (pre == BA_PRECOND_LEARNED_FSAI && c->n_rows > 0) prepare_learned_fsai(c);
        const int defl = (o && o->deflate && c->n_rows > 0) ? 1 : 0;
        if (defl) prepare_defl(c);
        BA_HIP_CHECK(hipEventRecord(c->ev[6], c->stream));
        ba_status s = BA_OK;
        int fell_back = 0;
        if (c->n_rows > 0) {
            s = ba::run_pcg(c, (pre == BA_PRECOND_FSAI || pre == BA_PRECOND_LEARNED_FSAI) ? 1 : 0, pre == BA_PRECOND_LEARNED ? c->Mlearn : c->Minv, defl,
                            tol, max_iter, o ? o->x0 : nullptr, dxc, &it, &rr);
            if (learned_failed(pre, s, rr)) {
                fell_back = 1;
                s = ba::run_pcg(c, 0, c->Minv, defl, tol, max_iter, o ? o->x0 : nullptr, dxc, &it, &rr);
            }
        }
        BA_HIP_CHECK(hipEventRecord(c->ev[7], c->stream));
        BA_HIP_CHECK(hipEventSynchronize(c->ev[7]));
        if (info) {
            info->iters = it;
            info->status = s;
            info->relres = rr;
            info->ms = elapsed(c->ev[6], c->ev[7]);
            info->precond_fallback = fell_back;
            info->reserved = 0;
        }
        if (s == BA_ERR_NOT_SPD) c->err = "d^T S d <= 0 in PCG";
        if (s == BA_ERR_NOT_CONVERGED) c->err = "PCG reached max_iter";
        return s;
    });
}

ba_status ba_rcs_product(ba_ctx* c, const double* x, double* y, int32_t product, int32_t solver_fp32) {
    if (!c) return BA_ERR_INVALID_ARG;
    if (!c->have_rcs) { c->err = "ba_rcs_product needs a formed RCS"; return BA_ERR_STATE; }
    if (!x || !y || x == y) { c->err = "x and y must be distinct device arrays"; return BA_ERR_INVALID_ARG; }
    if (product < BA_PRODUCT_AUTO || product > BA_PRODUCT_CSR) { c->err = "unknown product layout"; return BA_ERR_INVALID_ARG; }
    if (product == BA_PRODUCT_CSR && solver_fp32) { c->err = "the CSR copy is FP64 only"; return BA_ERR_INVALID_ARG; }
    return guarded(c, [&]() {
        if (product == BA_PRODUCT_CSR) {
            prepare_csr(c);
            ba::launch_csr_spmv(c, x, y);
            BA_HIP_CHECK(hipGetLastError());
            BA_HIP_CHECK(hipStreamSynchronize(c->stream));
            return BA_OK;
        }
        select_solver_matrix(c, solver_fp32, product);
        ba::launch_product(c, x, y);
        BA_HIP_CHECK(hipGetLastError());
        BA_HIP_CHECK(hipStreamSynchronize(c->stream));
        return BA_OK;
    });
}

ba_status ba_back_substitute(ba_ctx* c, const double* dxc, double* dxp) {
    if (!c) return BA_ERR_INVALID_ARG;
    if (!c->have_rcs) { c->err = "ba_back_substitute needs a formed RCS"; return BA_ERR_STATE; }
    if (!dxc || !dxp) { c->err = "null dxc or dxp"; return BA_ERR_INVALID_ARG; }
    return guarded(c, [&]() {
        if (c->shared)
            ba::launch_back_substitute_shared(c, dxc, dxp);
        else
            ba::launch_back_substitute(c, dxc, dxp);
        BA_HIP_CHECK(hipGetLastError());
        return BA_OK;
    });
}

ba_status ba_lm_step(ba_ctx* c, double* cams, double* pts, ba_lm_state* st, const ba_lm_opts* o, ba_lm_info* info) {
    if (!c) return BA_ERR_INVALID_ARG;
    if (!cams || !pts || !st) { c->err = "null parameters or state"; return BA_ERR_INVALID_ARG; }
    if (!(st->lambda >= 0.0) || !std::isfinite(st->lambda) || !(st->nu >= 1.0)) {
        c->err = "state needs lambda >= 0 and nu >= 1";
        return BA_ERR_INVALID_ARG;
    }
    const double tol = o ? o->pcg_tol : 1e-6;
    const int max_iter = o ? o->pcg_max_iter : 1000;
    const int pre = o ? o->precond : BA_PRECOND_BLOCK_JACOBI;
    if ((pre == BA_PRECOND_LEARNED || pre == BA_PRECOND_LEARNED_FSAI) && !c->learned_ready) {
        c->err = "no learned preconditioner set";
        return BA_ERR_STATE;
    }
    if (pre != BA_PRECOND_LEARNED && pre != BA_PRECOND_BLOCK_JACOBI && pre != BA_PRECOND_FSAI &&
        pre != BA_PRECOND_LEARNED_FSAI) {
        c->err = "unknown preconditioner";
        return BA_ERR_INVALID_ARG;
    }
    if (o && (o->product < BA_PRODUCT_AUTO || o->product > BA_PRODUCT_UPPER)) {
        c->err = "unknown product layout";
        return BA_ERR_INVALID_ARG;
    }
    if (o && (o->retriangulate < 0 || o->retriangulate > 100)) {
        c->err = "retriangulate must be 0..100 Gauss-Newton steps";
        return BA_ERR_INVALID_ARG;
    }
    if (c->shared && ((o && (o->deflate || o->retriangulate)) || pre == BA_PRECOND_LEARNED ||
                      pre == BA_PRECOND_LEARNED_FSAI)) {
        c->err = "shared-intrinsics contexts take block-Jacobi or FSAI, without deflation or re-triangulation";
        return BA_ERR_INVALID_ARG;
    }
    return guarded(c, [&]() {
        ba_lm_info I;
        std::memset(&I, 0, sizeof I);
        hipEvent_t* ev = c->ev;
        BA_HIP_CHECK(hipEventRecord(ev[8], c->stream));
        const bool relin = !(st->flags & 1) || !c->have_lin;
        BA_HIP_CHECK(hipEventRecord(ev[0], c->stream));
        if (relin) {
            // linearization and point stage in one pass (the records are written whole)
            BA_HIP_CHECK(hipMemsetAsync(c->flags, 0, 8 * sizeof(int), c->stream));
            if (c->shared) {
                BA_HIP_CHECK(hipMemcpyAsync(c->lin_params, cams, n_params(c) * sizeof(double),
                                            hipMemcpyDeviceToDevice, c->stream));
                BA_HIP_CHECK(hipMemcpyAsync(c->lin_pts, pts, (size_t)c->n_pts * 3 * sizeof(double),
                                            hipMemcpyDeviceToDevice, c->stream));
                ba::launch_linpoint_shared(c, c->lin_params, c->lin_pts, st->lambda);
            } else {
                ba::launch_linearize_point(c, cams, pts, st->lambda);
                BA_HIP_CHECK(hipMemcpyAsync(c->lin_cams, cams, (size_t)c->n_cams * 9 * sizeof(double),
                                            hipMemcpyDeviceToDevice, c->stream));
            }
            c->defl_ready = false;
        }
        BA_HIP_CHECK(hipEventRecord(ev[5], c->stream));
        c->have_lin = true;
        form_rcs_async(c, st->lambda, relin);
        int it = 0;
        double rr = 0.0;
        ba_status ps = BA_OK;
        BA_HIP_CHECK(hipEventRecord(ev[14], c->stream));
        select_solver_matrix(c, o ? o->solver_fp32 : 0, o ? o->product : BA_PRODUCT_AUTO);
        if (pre == BA_PRECOND_LEARNED && c->n_rows > 0) prepare_learned(c);
        if (pre == BA_PRECOND_FSAI && c->n_rows > 0) prepare_fsai(c);
        if (pre == BA_PRECOND_LEARNED_FSAI && c->n_rows > 0) prepare_learned_fsai(c);
        const int defl = (o && o->deflate && c->n_rows > 0) ? 1 : 0;
        if (defl) prepare_defl(c);
        BA_HIP_CHECK(hipEventRecord(ev[6], c->stream));
        if (c->n_rows > 0) {
            ps = ba::run_pcg(c, (pre == BA_PRECOND_FSAI || pre == BA_PRECOND_LEARNED_FSAI) ? 1 : 0, pre == BA_PRECOND_LEARNED ? c->Mlearn : c->Minv, defl,
                             tol, max_iter, nullptr, c->dxc, &it, &rr);
            if (learned_failed(pre, ps, rr)) {
                // the network's preconditioner is not usable on this RCS (not
                // SPD, or non-finite): solve again with block-Jacobi
                I.precond_fallback = 1;
                ps = ba::run_pcg(c, 0, c->Minv, defl, tol, max_iter, nullptr, c->dxc, &it, &rr);
            }
        } else
            BA_HIP_CHECK(hipMemsetAsync(c->dxc, 0, sizeof(double), c->stream));
        BA_HIP_CHECK(hipEventRecord(ev[7], c->stream));
        if (c->shared)
            ba::launch_back_substitute_shared(c, c->dxc, c->dxp);
        else
            ba::launch_back_substitute(c, c->dxc, c->dxp);
        const int n_tri = o ? o->retriangulate : 0;
        if (n_tri > 0) {
            // the points re-triangulated with the candidate cameras, starting
            // from the back-substituted ones; dxp becomes their displacement
            BA_HIP_CHECK(hipMemsetAsync(c->tri_failed, 0, sizeof(int), c->stream));
            ba::launch_triangulate(c, cams, c->dxc, pts, c->dxp, 1, 0, n_tri, c->tri_failed);
            ba::launch_model_terms(c, c->dxc, c->dxp);
            BA_HIP_CHECK(hipMemcpyAsync(c->h_flags + 3, c->tri_failed, sizeof(int), hipMemcpyDeviceToHost, c->stream));
        } else {
            c->h_flags[3] = 0;
        }
        BA_HIP_CHECK(hipEventRecord(ev[9], c->stream));
        if (c->shared)
            ba::launch_evaluate_shared(c, cams, pts, c->dxc, c->dxp);
        else
            ba::launch_evaluate(c, cams, pts, c->dxc, c->dxp);
        BA_HIP_CHECK(hipEventRecord(ev[10], c->stream));
        BA_HIP_CHECK(hipMemcpyAsync(c->h_scal, c->scal, 4 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        BA_HIP_CHECK(hipMemcpyAsync(c->h_flags, c->flags, 3 * sizeof(int), hipMemcpyDeviceToHost, c->stream));
        BA_HIP_CHECK(hipStreamSynchronize(c->stream));
        BA_HIP_CHECK(hipGetLastError());
        const double F = c->h_scal[0], Fn = c->h_scal[1], jdx2 = c->h_scal[2], dxl = c->h_scal[3];
        const double L = dxl - 0.5 * jdx2;
        I.cost = F;
        I.cost_new = Fn;
        I.model_decrease = L;
        I.rho = (F - Fn) / L;
        I.pcg_iters = it;
        I.pcg_status = ps;
        I.pcg_relres = rr;
        I.tri_failed = c->h_flags[3];
        if (c->h_flags[2]) {
            // the linearization does not fit the records: no step is taken and
            // the state is left as it was
            BA_HIP_CHECK(hipEventRecord(ev[11], c->stream));
            BA_HIP_CHECK(hipEventSynchronize(ev[11]));
            if (info) *info = I;
            c->err = kRangeMsg;
            return BA_ERR_RANGE;
        }
        const bool formed = !c->h_flags[0] && !c->h_flags[1];
        if (!formed) I.pcg_status = BA_ERR_NOT_SPD;
        const bool ok = formed && (ps == BA_OK || ps == BA_ERR_NOT_CONVERGED) && L > 0.0 && std::isfinite(Fn) && Fn < F;
        if (ok) {
            if (c->shared)
                ba::launch_update_shared(c, cams, pts, c->dxc, c->dxp);
            else
                ba::launch_update(c, cams, pts, c->dxc, c->dxp);
            const double t = 2.0 * I.rho - 1.0;
            st->lambda *= std::max(1.0 / 3.0, 1.0 - t * t * t);
            st->nu = 2.0;
            st->flags &= ~1;
            I.accepted = 1;
            if (F - Fn < 1e-12 * F) I.stop = 1;
        } else {
            st->lambda *= st->nu;
            st->nu *= 2.0;
            st->flags |= 1;
        }
        st->iter += 1;
        BA_HIP_CHECK(hipEventRecord(ev[11], c->stream));
        BA_HIP_CHECK(hipEventSynchronize(ev[11]));
        I.ms_linearize = elapsed(ev[0], ev[5]);
        I.ms_form_rcs = elapsed(ev[1], ev[4]);
        I.ms_pcg = elapsed(ev[6], ev[7]);
        I.ms_back_substitute = elapsed(ev[7], ev[9]);
        I.ms_evaluate = elapsed(ev[9], ev[10]);
        I.ms_total = elapsed(ev[8], ev[11]);
        I.ms_precond = (pre != BA_PRECOND_BLOCK_JACOBI || (o && o->deflate)) ? elapsed(ev[14], ev[6]) : 0.0;
        if (info) *info = I;
        return BA_OK;
    });
}

ba_status ba_get_pattern(ba_ctx* c, int64_t* row_ptr, int32_t* col_idx) {
    if (!c) return BA_ERR_INVALID_ARG;
    if (row_ptr) std::memcpy(row_ptr, c->h_row_ptr.data(), c->h_row_ptr.size() * sizeof(int64_t));
    if (col_idx) std::memcpy(col_idx, c->h_col_idx.data(), c->h_col_idx.size() * sizeof(int32_t));
    return BA_OK;
}

ba_status ba_get_rcs(ba_ctx* c, double* blk, double* rhs) {
    if (!c) return BA_ERR_INVALID_ARG;
    if (!c->have_rcs) { c->err = "no RCS formed"; return BA_ERR_STATE; }
    return guarded(c, [&]() {
        if (blk) BA_HIP_CHECK(hipMemcpyAsync(blk, c->blk, c->n_blk * 81 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        if (rhs) BA_HIP_CHECK(hipMemcpyAsync(rhs, c->rhs, (size_t)c->n_rows * 9 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        BA_HIP_CHECK(hipStreamSynchronize(c->stream));
        return BA_OK;
    });
}

ba_status ba_get_gauge(ba_ctx* c, double* W) {
    if (!c || !W) return BA_ERR_INVALID_ARG;
    if (c->shared) { c->err = "no gauge vectors for shared-intrinsics contexts"; return BA_ERR_INVALID_ARG; }
    if (!c->have_rcs) { c->err = "no RCS formed"; return BA_ERR_STATE; }
    return guarded(c, [&]() {
        if (c->n_rows > 0) prepare_defl(c);
        BA_HIP_CHECK(hipMemcpyAsync(W, c->pcg.W, (size_t)c->n_rows * 63 * sizeof(double), hipMemcpyDeviceToHost,
                                    c->stream));
        BA_HIP_CHECK(hipStreamSynchronize(c->stream));
        return BA_OK;
    });
}

ba_status ba_get_fsai(ba_ctx* c, float* G) {
    if (!c || !G) return BA_ERR_INVALID_ARG;
    if (!c->fs.built || !c->have_rcs) { c->err = "no FSAI factor of the current RCS"; return BA_ERR_STATE; }
    return guarded(c, [&]() {
        BA_HIP_CHECK(hipMemcpyAsync(G, c->fs.G, (size_t)c->n_blk * 81 * sizeof(float), hipMemcpyDeviceToHost, c->stream));
        BA_HIP_CHECK(hipStreamSynchronize(c->stream));
        return BA_OK;
    });
}

ba_status ba_get_csr(ba_ctx* c, int32_t* row_ptr, int32_t* col, double* val, int64_t* nnz) {
    if (!c) return BA_ERR_INVALID_ARG;
    if (!c->have_rcs) { c->err = "no RCS formed"; return BA_ERR_STATE; }
    return guarded(c, [&]() {
        prepare_csr(c);
        const ba::Csr& C = c->csr;
        if (nnz) *nnz = C.nnz;
        if (row_ptr)
            BA_HIP_CHECK(hipMemcpyAsync(row_ptr, C.rowptr, (9 * (size_t)c->n_rows + 1) * sizeof(int32_t),
                                        hipMemcpyDeviceToHost, c->stream));
        if (col) BA_HIP_CHECK(hipMemcpyAsync(col, C.col, C.nnz * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
        if (val) BA_HIP_CHECK(hipMemcpyAsync(val, C.val, C.nnz * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        BA_HIP_CHECK(hipStreamSynchronize(c->stream));
        return BA_OK;
    });
}

ba_status ba_get_store_sizes(const ba_ctx* c, ba_store_sizes* o) {
    if (!c || !o) return BA_ERR_INVALID_ARG;
    const int64_t nb = c->n_blk, nr = c->n_rows, both = 2 * nb - nr;
    o->bsmc_bytes = nb * 81 * 8 + nb * 4 + (nr + 1) * 4;
    o->full_bytes = c->n_sf * 81 * 8 + c->n_sf * 4 * 2 + (nr + 1) * 4;
    o->csr_nnz = 81 * both;
    o->csr_bytes = 81 * both * (8 + 4) + (9 * nr + 1) * 4;
    return BA_OK;
}

ba_status ba_get_jacobians(ba_ctx* c, double* J, double* e) {
    if (!c) return BA_ERR_INVALID_ARG;
    if (c->shared) { c->err = "ba_get_jacobians takes 9-parameter contexts"; return BA_ERR_INVALID_ARG; }
    if (!c->have_lin) { c->err = "no linearization"; return BA_ERR_STATE; }
    return guarded(c, [&]() {
        const int64_t n = c->n_obs;
        if (J) {
            ba::ensure_jp(c);
            const size_t es = c->precision == BA_MIXED ? sizeof(float) : sizeof(double);
            std::vector<char> hr((size_t)n * kRec * es), hp((size_t)n * 6 * es);
            BA_HIP_CHECK(hipMemcpyAsync(hr.data(), c->R, hr.size(), hipMemcpyDeviceToHost, c->stream));
            BA_HIP_CHECK(hipMemcpyAsync(hp.data(), c->Jp, hp.size(), hipMemcpyDeviceToHost, c->stream));
            BA_HIP_CHECK(hipStreamSynchronize(c->stream));
            for (int64_t k = 0; k < n; ++k) {
                double* out = J + c->h_perm[k] * 24;
                for (int i = 0; i < 18; ++i)
                    out[i] = es == 4 ? ((const float*)hr.data())[k * kRec + i] : ((const double*)hr.data())[k * kRec + i];
                for (int i = 0; i < 6; ++i)
                    out[18 + i] = es == 4 ? ((const float*)hp.data())[k * 6 + i] : ((const double*)hp.data())[k * 6 + i];
            }
        }
        if (e) {
            std::vector<double> h((size_t)n * 2);
            BA_HIP_CHECK(hipMemcpyAsync(h.data(), c->e, h.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
            BA_HIP_CHECK(hipStreamSynchronize(c->stream));
            for (int64_t k = 0; k < n; ++k) {
                e[2 * c->h_perm[k]] = h[2 * k];
                e[2 * c->h_perm[k] + 1] = h[2 * k + 1];
            }
        }
        return BA_OK;
    });
}

}  // extern "C"
