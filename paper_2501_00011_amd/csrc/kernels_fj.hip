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

// Sum-of-monomials evaluation.  A block of 256 lanes covers 256 consecutive
// cells and one chunk of whole output rows; rows 0..N-1 go to f, the rest to
// the Jacobian.  The chunk's terms are taken 8 at a time: their indices come
// through the scalar unit and all their k and y loads (a missing factor reads
// a row of ones) are issued before any is consumed, so a wavefront keeps up
// to 32 loads in flight instead of walking a dependent chain per term.
// Blocks of one cell tile are spread over chunks such that all the chunks of
// a tile land on the same XCD (workgroups are dispatched to the 8 XCDs
// round-robin), so y and k of a tile are fetched from HBM once into that
// XCD's L2 and re-read from there.
__global__ __launch_bounds__(256) void fj_kernel(FJParams p)
{
    const int bid = blockIdx.x;
    const int xcd = bid & 7;
    const int q = bid >> 3;
    const int chunk = q % p.n_chunks;
    const int tile = (q / p.n_chunks) * 8 + xcd;
    if (tile >= p.n_tiles) return;
    const int64_t c = (int64_t)tile * 256 + threadIdx.x;
    const bool live = c < p.n_cells;
    const int64_t cc = live ? c : 0;
    const FjChunk ch = p.chunks[p.chunk_begin + chunk];
    const FjTerm *tm = p.terms + ch.term_begin;
    const double *ones = p.ones + cc;
    int row = ch.row_begin;
    double acc = 0.0;
    for (int g = 0; g < ch.term_count; g += kFjGroup) {
        double v[kFjGroup];
#pragma unroll
        for (int i = 0; i < kFjGroup; ++i) {
            const FjTerm t = tm[g + i];
            const double *ya = t.a >= 0 ? p.y + (int64_t)t.a * p.ld + cc : ones;
            const double *yb = t.b >= 0 ? p.y + (int64_t)t.b * p.ld + cc : ones;
            const double *yc = t.c >= 0 ? p.y + (int64_t)t.c * p.ld + cc : ones;
            v[i] = t.coef * p.k[(int64_t)t.j * p.ld + cc] * *ya * *yb * *yc;
        }
#pragma unroll
        for (int i = 0; i < kFjGroup; ++i) {
            acc += v[i];
            if (tm[g + i].end) {
                if (live) {
                    if (row < p.N)
                        p.f[(int64_t)row * p.ld + c] = acc;
                    else
                        p.jac[(int64_t)(row - p.N) * p.ld + c] = acc;
                }
                acc = 0.0;
                row++;
            }
        }
    }
}

hipError_t launch_fj(const FJParams &p, hipStream_t s)
{
    if (p.n_cells == 0 || p.n_chunks == 0) return hipSuccess;
    const int groups = (p.n_tiles + 7) / 8;
    const int64_t blocks = (int64_t)groups * 8 * p.n_chunks;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(fj_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p);
    return hipGetLastError();
}

}  // namespace mcc
