// Streaming kernels over cells: rate constants, and f / sparse J evaluation.
//
// Layout: every per-cell array is [entity][ld] with the cell index fastest, so
// a wavefront of 64 consecutive cells reads and writes 512 contiguous bytes
// per row.  The mechanism structure is identical for every cell, so each
// lane (cell) walks the same term list in lockstep; the list is read through
// the scalar unit (one load per wavefront, no divergence), in place of the
// paper's thread-per-reaction kernel with atomic adds (Section 3): every
// output value is produced by exactly one lane, with no atomics.
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

// f and J by chunks.  A block is one wavefront of 64 consecutive cells (lane =
// cell) and one work item (a run of chunks).  For each chunk the wavefront
// first computes the chunk's monomials k_j * y_a * y_b * y_c -- the reaction
// rates of a few f rows, or the rate partials of one Jacobian column --
// eight at a time so that their loads are in flight together (a missing
// factor reads a row of ones), into a per-lane LDS scratchpad; then every
// output row of the chunk is sum coef * monomial, read back from the
// scratchpad, and written once (no atomics: each output has one owner).
// Table entries come through the scalar unit.  The work items of one cell
// tile are mapped to one XCD (workgroups go to the 8 XCDs round-robin), so
// that XCD's L2 serves the tile's repeated y and k reads.
__global__ __launch_bounds__(64) void fj_kernel(FJParams p)
{
    __shared__ double scratch[kFjQmax * 64];
    const int bid = blockIdx.x;
    const int xcd = bid & 7;
    const int q = bid >> 3;
    const int item = q % p.n_items;
    const int tile = (q / p.n_items) * 8 + xcd;
    if (tile >= p.n_tiles) return;
    const int lane = threadIdx.x;
    const int64_t c = (int64_t)tile * 64 + lane;
    const bool live = c < p.n_cells;
    const int64_t cc = live ? c : 0;
    const double *ones = p.ones + cc;
    double *mine = scratch + lane;
    const int it = p.item_begin + item;
    for (int ci = p.items[it]; ci < p.items[it + 1]; ++ci) {
        const FjChunk ch = p.chunks[ci];
        const FjMono *mo = p.monos + ch.mono_begin;
        for (int q0 = 0; q0 < ch.n_mono; q0 += kFjGroup) {
            double v[kFjGroup];
#pragma unroll
            for (int i = 0; i < kFjGroup; ++i) {
                const FjMono m = mo[min(q0 + i, ch.n_mono - 1)];
                const double *ya = m.a >= 0 ? p.y + (int64_t)m.a * p.ld + cc : ones;
                const double *yb = m.b >= 0 ? p.y + (int64_t)m.b * p.ld + cc : ones;
                const double *yc = m.c >= 0 ? p.y + (int64_t)m.c * p.ld + cc : ones;
                v[i] = p.k[(int64_t)m.j * p.ld + cc] * *ya * *yb * *yc;
            }
#pragma unroll
            for (int i = 0; i < kFjGroup; ++i)
                if (q0 + i < ch.n_mono) mine[(q0 + i) * 64] = v[i];
        }
        const FjOut *ou = p.outs + ch.out_begin;
        for (int o = 0; o < ch.n_out; ++o) {
            const FjOut out = ou[o];
            double acc = 0.0;
            for (int t = out.t_begin; t < out.t_begin + out.t_count; ++t) {
                const FjTerm tm = p.terms[t];
                acc += tm.coef * mine[tm.slot * 64];
            }
            if (live) {
                double *dst = out.row < p.N ? p.f + (int64_t)out.row * p.ld + c
                                            : p.jac + (int64_t)(out.row - p.N) * p.ld + c;
                *dst = out.accum ? *dst + acc : acc;
            }
        }
    }
}

hipError_t launch_fj(const FJParams &p, hipStream_t s)
{
    if (p.n_cells == 0 || p.n_items == 0) return hipSuccess;
    const int groups = (p.n_tiles + 7) / 8;
    const int64_t blocks = (int64_t)groups * 8 * p.n_items;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(fj_kernel, dim3((unsigned)blocks), dim3(64), 0, s, p);
    return hipGetLastError();
}

}  // namespace mcc
