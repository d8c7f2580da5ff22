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
// factorised head: off-diagonal blocks of G from [h_i, h_j, g_ij] through
// one hidden layer of HO units
constexpr int F_OFF = 96;              // head output (81 used)
constexpr int HO = 128;                // head hidden width
constexpr int64_t OFF_WO1 = OFF_BD + F_OUT, OFF_BO1 = OFF_WO1 + 3 * H * HO, OFF_WO2 = OFF_BO1 + HO;
constexpr int64_t OFF_BO2 = OFF_WO2 + HO * F_OFF, OFF_AO = OFF_BO2 + F_OFF;
constexpr int64_t OFF_HEAD = OFF_WO1;
constexpr int64_t N_PARAMS = OFF_AO + F_OFF;
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
    // FSAI sets of the factorised head (same sets as the library's FSAI):
    // per row its members J (ascending, the row last); per member the
    // directed edge row -> member (-1 for the row) and the RCS block slot;
    // per row the packed lower tiles (a, b), a >= b: directed edge
    // J_a -> J_b, -2 on the diagonal, -1 if the cameras share no point;
    // the FSAI edges (row, member) in row order and, for the backward
    // scatter, the FSAI edges by member.
    bool has_fsai = false;
    int n_blk = 0, fm = 0, fE = 0, max_m = 0;
    int32_t *fptr = nullptr, *fJ = nullptr, *fedge = nullptr, *fslot = nullptr, *ftile = nullptr;
    int64_t* ftptr = nullptr;
    int32_t *fsrc = nullptr, *fdst = nullptr, *fe = nullptr, *fd_ptr = nullptr, *fd_list = nullptr;
    int32_t* e2f = nullptr;            // FSAI edge of each directed edge, or -1
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
    // factorised head
    int cap_f = 0, cap_fn = 0;
    __bf16 *Xf = nullptr, *dOEb = nullptr, *Z1b = nullptr, *dZ1b = nullptr;
    float *OE = nullptr, *dOE = nullptr, *dXf = nullptr, *aE = nullptr, *Z1 = nullptr, *dZ1 = nullptr, *dZ1p = nullptr;
    double* kpart = nullptr;
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
// graph structure from a host pattern (row_ptr int64 [n+1], col_idx [n_blk]);
// with blk_pairs (common points per block) also the FSAI sets
void build_graph(Graph& g, int n, const int64_t* row_ptr, const int32_t* col_idx, const int32_t* blk_pairs,
                 hipStream_t st);
void free_graph(Graph& g);
// features of the RCS in blk (device, FP64 blocks indexed like the pattern)
void compute_features(Graph& g, const double* blk, hipStream_t st);
// inference: P_i = L_i^-T Lt_i Lt_i^T L_i^-1 into P [n][81] (FP64), as
// Minv_i + L_i^-T (Lt_i Lt_i^T - I) L_i^-1 when the block-Jacobi inverses
// Minv are given
void infer_preconditioner(ba_gnn* net, Graph& g, const double* Minv, double* P, hipStream_t st);
// factorised head: G of the graph's FSAI sets into the layouts of the
// library's FSAI (Gl by member, Gu at gu_pos, G at the block slots; any may
// be null)
// with Gh (and Gh8, hs, Dn): the FP16 copy of the UPPER apply instead of Gu
void infer_factor(ba_gnn* net, Graph& g, const int32_t* gu_pos, float* Gl, float* Gu, float* Gslots, hipStream_t st,
                  const double* Dn = nullptr, uint32_t* Gh = nullptr, uint16_t* Gh8 = nullptr,
                  float* hs = nullptr);
// the FSAI sets of a pattern (shared with the library's FSAI): per row, its
// lower neighbours with the most common points (at most kFsaiM - 1, ties to
// the lower index), ascending, then the row
void fsai_sets(int n, const int64_t* row_ptr, const int32_t* col_idx, const int32_t* blk_pairs,
               std::vector<int32_t>& ptr, std::vector<int32_t>& J, std::vector<int32_t>& slot);
void free_work(Work& w);
}  // namespace gnn
}  // namespace ba
