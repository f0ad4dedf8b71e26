// Streaming kernels over cells: rate constants, and f / sparse J evaluation.
//
// Layout: every per-cell array is [entity][ld] with the cell index fastest, so
// a wavefront of 64 consecutive cells reads and writes 512 contiguous bytes
// per row.  The mechanism structure is identical for every cell, so each
// lane (cell) walks the same term list in lockstep; the list is read through
// the scalar unit (one load per wavefront, no divergence), in place of the
// paper's thread-per-reaction kernel with atomic adds (Section 3): every
// output value is produced by exactly one lane, with no atomics.
#include <algorithm>

#include "mcc_internal.hpp"

namespace mcc {

// k[j][c] = A_j exp(-theta_j / T_c) (thermal, Arrhenius) or A_j s_c (photolysis).
__global__ __launch_bounds__(256) void rates_kernel(RatesParams p)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (c >= p.n_cells) return;
    const double Tc = p.T[c];
    const double sc = p.jscale ? p.jscale[c] : 1.0;
    const double kj = p.rxn_type[j] == MCC_RXN_PHOTOLYSIS ? p.A[j] * sc : p.A[j] * exp(-p.theta[j] / Tc);
    p.k[(int64_t)j * p.ld + c] = kj;
}

hipError_t launch_rates(const RatesParams &p, hipStream_t s)
{
    if (p.n_cells == 0 || p.R == 0) return hipSuccess;
    dim3 grid((unsigned)((p.n_cells + 255) / 256), (unsigned)p.R);
    hipLaunchKernelGGL(rates_kernel, grid, dim3(256), 0, s, p);
    return hipGetLastError();
}

// f and J.  Every cell is a lane: a block is one wavefront of 64 consecutive
// cells and one work item (a run of chunks).  The mechanism structure, the
// same for every cell, comes from tables read through the scalar unit
// (uniform across the wavefront).  Per chunk the wavefront computes its
// monomials k_j * y_a * y_b * y_c -- the reaction rates of a few f rows, or
// the rate partials of a few Jacobian columns -- eight at a time so that
// their loads are in flight together, into a per-lane LDS scratchpad; then
// its output records four at a time: a record adds up to three terms
// coef * monomial to a running sum and may write it.  Every output row has
// one owner: no atomics.  The cost that bounds this kernel is instruction
// issue, so addressing is kept off the vector ALU: a row's base address is
// uniform (scalar registers) and each lane adds one 32-bit byte offset, the
// global_load "saddr" form; a missing factor points at a row of ones.  The
// work items of one cell tile are mapped to one XCD (workgroups go to the 8
// XCDs round-robin), so that XCD's L2 serves the tile's repeated y and k
// reads.  Restrict-qualified arguments: no output aliases a table or input.
__device__ __forceinline__ double at(const double *row, uint32_t boff)
{
    return *(const double *)((const char *)row + boff);
}

__global__ __launch_bounds__(64) void fj_kernel(const FjMono *__restrict__ monos,
                                                const FjRec *__restrict__ recs,
                                                const FjChunk *__restrict__ chunks,
                                                const int32_t *__restrict__ items,
                                                const double *__restrict__ y,
                                                const double *__restrict__ k,
                                                const double *__restrict__ ones,
                                                double *__restrict__ f, double *__restrict__ jac,
                                                int64_t n_cells, int64_t ld, int32_t N,
                                                int32_t item_begin, int32_t n_items, int32_t n_tiles)
{
    __shared__ double scratch[(kFjQmax + 1) * 64];
    const int bid = blockIdx.x;
    const int xcd = bid & 7;
    const int q = bid >> 3;
    const int item = q % n_items;
    const int tile = (q / n_items) * 8 + xcd;
    if (tile >= n_tiles) return;
    const int lane = threadIdx.x;
    const int64_t c = (int64_t)tile * 64 + lane;
    const bool live = c < n_cells;
    const uint32_t boff = (uint32_t)((live ? c : 0) * (int64_t)sizeof(double));  // this lane's cell in a row
    double *mine = scratch + lane;
    mine[kFjQmax * 64] = 0.0;  // the zero slot of padding terms
    const int it = item_begin + item;
    for (int ci = items[it]; ci < items[it + 1]; ++ci) {
        const FjChunk ch = chunks[ci];
        const FjMono *mo = monos + ch.mono_begin;
        for (int q0 = 0; q0 < ch.n_mono; q0 += kFjGroup) {
            double v[kFjGroup];
            FjMono mg[kFjGroup];  // the group's table entries first: their scalar loads overlap
#pragma unroll
            for (int i = 0; i < kFjGroup; ++i) mg[i] = mo[q0 + i];
#pragma unroll
            for (int i = 0; i < kFjGroup; ++i) {
                const FjMono m = mg[i];
                const double *pk = m.j >= 0 ? k + (int64_t)m.j * ld : ones;
                const double *pa = m.a >= 0 ? y + (int64_t)m.a * ld : ones;
                const double *pb = m.b >= 0 ? y + (int64_t)m.b * ld : ones;
                const double *pc = m.c >= 0 ? y + (int64_t)m.c * ld : ones;
                v[i] = at(pk, boff) * at(pa, boff) * at(pb, boff) * at(pc, boff);
            }
#pragma unroll
            for (int i = 0; i < kFjGroup; ++i) mine[(q0 + i) * 64] = v[i];
        }
        const FjRec *rc = recs + ch.rec_begin;
        double acc = 0.0;
        for (int r0 = 0; r0 < ch.n_rec; r0 += kFjRecGroup) {
            FjRec rec[kFjRecGroup];
            double sum[kFjRecGroup];
#pragma unroll
            for (int i = 0; i < kFjRecGroup; ++i) rec[i] = rc[r0 + i];
            // sums first, branch-free, so that all scratchpad reads are in flight together
#pragma unroll
            for (int i = 0; i < kFjRecGroup; ++i) {
                const uint32_t sl = rec[i].slots;
                const double s = rec[i].coef[0] * mine[(sl & 0xff) * 64] +
                                 rec[i].coef[1] * mine[((sl >> 8) & 0xff) * 64] +
                                 rec[i].coef[2] * mine[((sl >> 16) & 0xff) * 64];
                acc = ((rec[i].meta >> 24) & kFjKeep) ? acc + s : s;
                sum[i] = acc;
            }
#pragma unroll
            for (int i = 0; i < kFjRecGroup; ++i) {
                const uint32_t flags = rec[i].meta >> 24;
                if ((flags & kFjStore) && live) {
                    const uint32_t row = rec[i].meta & kFjRowMask;
                    double *dst = row < (uint32_t)N ? f + (int64_t)row * ld : jac + (int64_t)(row - N) * ld;
                    double *d = (double *)((char *)dst + boff);
                    *d = (flags & kFjAdd) ? *d + sum[i] : sum[i];
                }
            }
        }
    }
}

hipError_t launch_fj(const FJParams &p, hipStream_t s)
{
    if (p.n_cells == 0 || p.n_items == 0) return hipSuccess;
    const int64_t groups = (p.n_tiles + 7) / 8;
    const int64_t blocks = groups * 8 * p.n_items;
    if (blocks > 0x7fffffff || p.n_cells * (int64_t)sizeof(double) > 0xffffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(fj_kernel, dim3((unsigned)blocks), dim3(64), 0, s, p.monos, p.recs, p.chunks, p.items, p.y,
                       p.k, p.ones, p.f, p.jac, p.n_cells, p.ld, p.N, p.item_begin, p.n_items, p.n_tiles);
    return hipGetLastError();
}

}  // namespace mcc
