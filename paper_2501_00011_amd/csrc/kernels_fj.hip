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
// cells and one chunk of output rows; rows 0..N-1 go to f, the rest to the
// Jacobian.  Blocks of one cell tile are spread over chunks such that all the
// chunks of a tile land on the same XCD (workgroups are dispatched to the 8
// XCDs round-robin), so y and k of a tile are fetched from HBM once into that
// XCD's L2 and re-read from there.
__global__ __launch_bounds__(256) void fj_kernel(FJParams p)
{
    const int b = blockIdx.x;
    const int xcd = b & 7;
    const int q = b >> 3;
    const int chunk = q % p.n_chunks;
    const int tile = (q / p.n_chunks) * 8 + xcd;
    if (tile >= p.n_tiles) return;
    const int64_t c = (int64_t)tile * 256 + threadIdx.x;
    const bool live = c < p.n_cells;
    const int64_t cc = live ? c : 0;
    const int N = p.N;
    const int ch = p.chunk_begin + chunk;
    const int r0 = p.chunks[ch], r1 = p.chunks[ch + 1];
    for (int r = r0; r < r1; ++r) {
        double acc = 0.0;
        const int t1 = p.out_ptr[r + 1];
        for (int t = p.out_ptr[r]; t < t1; ++t) {
            const int j = p.term_idx[4 * t + 0];
            const int a = p.term_idx[4 * t + 1];
            const int bb = p.term_idx[4 * t + 2];
            const int e = p.term_idx[4 * t + 3];
            double v = p.term_coef[t] * p.k[(int64_t)j * p.ld + cc];
            if (a < N) v *= p.y[(int64_t)a * p.ld + cc];
            if (bb < N) v *= p.y[(int64_t)bb * p.ld + cc];
            if (e < N) v *= p.y[(int64_t)e * p.ld + cc];
            acc += v;
        }
        if (live) {
            if (r < N)
                p.f[(int64_t)r * p.ld + c] = acc;
            else
                p.jac[(int64_t)(r - N) * p.ld + c] = acc;
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
