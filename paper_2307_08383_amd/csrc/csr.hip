// Scalar CSR copy of the RCS and its product, the storage the paper
// compares BSMC with (Sec. 4.1, Eq. (8)-(10); Sec. 4.2, Table 1).
//
// CSR keeps every non-zero of both triangles as a (column, value) pair:
// 81 (2 n_blk - n_rows) non-zeros, 12 bytes each, plus a row pointer per
// scalar row (Eq. (8) with c = 9).  The BSMC store keeps the upper blocks
// only, one column index per 9x9 block (Eq. (9)).  The copy is built from
// the blocks after a formation, on first use, and serves the comparison of
// the two layouts (bytes held and product time); PCG itself runs on the
// block layouts.
#include "ba_common.hpp"

namespace ba {

namespace {

constexpr int BS = 256;

// One thread per (block slot, row a of the block): the 9 values of scalar
// row 9 r + a that the slot contributes, and their columns.  Slots of a
// block row are in ascending column order (the transposed blocks of the
// lower triangle first, then the diagonal and the upper blocks), so each
// scalar row is sorted by column.
__global__ __launch_bounds__(BS) void k_csr_fill(int64_t n_slot, const int32_t* __restrict__ slot_row,
                                                 const int32_t* __restrict__ slot_src,
                                                 const int32_t* __restrict__ slot_col,
                                                 const int32_t* __restrict__ bptr, const double* __restrict__ blk,
                                                 int32_t* __restrict__ col, double* __restrict__ val) {
    const int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x;
    if (i >= n_slot * 9) return;
    const int64_t slot = i / 9;
    const int a = (int)(i % 9);
    const int r = slot_row[slot];
    const int64_t p = bptr[r], m = bptr[r + 1] - p;
    const int64_t base = 81 * p + 9 * m * a + 9 * (slot - p);
    const int src = slot_src[slot];
    const double* B = blk + (int64_t)(src >> 1) * 81;
    const bool tr = src & 1;
    const int c0 = 9 * slot_col[slot];
#pragma unroll
    for (int b = 0; b < 9; ++b) {
        val[base + b] = tr ? B[b * 9 + a] : B[a * 9 + b];
        col[base + b] = c0 + b;
    }
}

// y = S x with one wave per scalar row: the lanes stride over the row's
// non-zeros (coalesced value and column loads, gathered x), then a fixed
// shuffle tree sums the lanes.
__global__ __launch_bounds__(BS) void k_csr_spmv(int n_srows, const int32_t* __restrict__ rowptr,
                                                 const int32_t* __restrict__ col, const double* __restrict__ val,
                                                 const double* __restrict__ x, double* __restrict__ y) {
    const int row = blockIdx.x * (BS / kWave) + threadIdx.x / kWave;
    const int lane = threadIdx.x % kWave;
    if (row >= n_srows) return;   // whole wave
    double s = 0.0;
    for (int k = rowptr[row] + lane; k < rowptr[row + 1]; k += kWave) s += val[k] * x[col[k]];
    s = wave_sum(s);
    if (lane == 0) y[row] = s;
}

}  // namespace

void launch_csr_fill(ba_ctx* c) {
    Csr& C = c->csr;
    if (C.n_slot == 0) return;
    const int64_t n = C.n_slot * 9;
    k_csr_fill<<<(unsigned)((n + BS - 1) / BS), BS, 0, c->stream>>>(C.n_slot, C.slot_row, C.slot_src, C.slot_col,
                                                                    C.bptr, c->blk, C.col, C.val);
}

void launch_csr_spmv(ba_ctx* c, const double* x, double* y) {
    const int n = 9 * c->n_rows;
    if (n == 0) return;
    const int wpb = BS / kWave;
    k_csr_spmv<<<(n + wpb - 1) / wpb, BS, 0, c->stream>>>(n, c->csr.rowptr, c->csr.col, c->csr.val, x, y);
}

}  // namespace ba
