// Learned correction to block-Jacobi: objects shared by the network kernels
// and the context API.
#pragma once

#include "ba_common.hpp"

namespace ba {
namespace gnn {

constexpr int H = 64;                  // hidden width
constexpr int F_NODE = 64;             // node input (45 used)
constexpr int F_EDGE = 96;             // edge input (81 used)
constexpr int F_OUT = 48;              // decoder output (45 used)
constexpr int N_LAYERS = 3;
constexpr int64_t LAYER = 3 * H * H + H + 2 * H * H + H;
constexpr int64_t OFF_WN = 0, OFF_BN = OFF_WN + F_NODE * H, OFF_WE = OFF_BN + H, OFF_BE = OFF_WE + F_EDGE * H;
constexpr int64_t OFF_L0 = OFF_BE + H;
constexpr int64_t OFF_WD = OFF_L0 + N_LAYERS * LAYER, OFF_BD = OFF_WD + H * F_OUT;
constexpr int64_t N_PARAMS = OFF_BD + F_OUT;
inline int64_t off_M(int l) { return OFF_L0 + l * LAYER; }
inline int64_t off_c(int l) { return off_M(l) + 3 * H * H; }
inline int64_t off_U(int l) { return off_c(l) + H; }
inline int64_t off_u(int l) { return off_U(l) + 2 * H * H; }

// Directed camera-pair graph of an RCS pattern plus the network inputs of
// one RCS instance.
struct Graph {
    int n = 0, E = 0;
    int32_t *eptr = nullptr, *esrc = nullptr, *edst = nullptr, *etwin = nullptr, *eblk = nullptr, *etr = nullptr;
    int32_t* diag_blk = nullptr;       // block index of each node's diagonal block
    __bf16 *xn = nullptr, *xe = nullptr;
    float* A = nullptr;                // [E][81] normalised blocks L_i^-1 S_ij L_j^-T
    double* Linv = nullptr;            // [n][81] L_i^-1 (lower)
    int* flags = nullptr;              // [0] a diagonal block was not SPD
    size_t bytes = 0;
};

// Activations and gradients of one forward/backward pass, grown on demand.
struct Work {
    int cap_n = 0, cap_E = 0, cap_p = 0;
    float *H0 = nullptr, *Hf = nullptr, *G = nullptr, *O = nullptr, *Z = nullptr, *Y = nullptr;
    __bf16 *Hb = nullptr, *Gb = nullptr;               // Hb: 4 x [n][64]
    __bf16 *Xm = nullptr, *Xu = nullptr;               // per layer
    float *Mm = nullptr, *T = nullptr;                 // per layer
    float *dO = nullptr, *dH = nullptr, *dT = nullptr, *dXu = nullptr, *dMm = nullptr, *dXm = nullptr, *dG = nullptr;
    __bf16 *dOb = nullptr, *dTb = nullptr, *dMmb = nullptr, *dPb = nullptr;
    float *dP = nullptr, *split = nullptr, *colpart = nullptr, *loss_part = nullptr;
    double* loss = nullptr;
};

}  // namespace gnn
}  // namespace ba

struct ba_gnn {
    hipStream_t stream = nullptr;
    float *w = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr, *gsum = nullptr;
    __bf16* wb = nullptr;
    int64_t step = 0;
    ba::gnn::Work work;
    std::string err;
};

struct ba_gnn_graph {
    ba::gnn::Graph g;
};

namespace ba {
namespace gnn {
// graph structure from a host pattern (row_ptr int64 [n+1], col_idx [n_blk])
void build_graph(Graph& g, int n, const int64_t* row_ptr, const int32_t* col_idx, hipStream_t st);
void free_graph(Graph& g);
// features of the RCS in blk (device, FP64 blocks indexed like the pattern)
void compute_features(Graph& g, const double* blk, hipStream_t st);
// inference: P_i = L_i^-T Lt_i Lt_i^T L_i^-1 into P [n][81] (FP64), as
// Minv_i + L_i^-T (Lt_i Lt_i^T - I) L_i^-1 when the block-Jacobi inverses
// Minv are given
void infer_preconditioner(ba_gnn* net, Graph& g, const double* Minv, double* P, hipStream_t st);
void free_work(Work& w);
}  // namespace gnn
}  // namespace ba
