// Ablation: the paper's GPU Derivative kernel (Section 3), rebuilt on this
// GPU so that its design can be timed beside the library's f kernel.  As in
// the paper: one thread per (cell, reaction) -- consecutive threads take
// consecutive reactions of one cell -- 1024 threads per block, the cells'
// data concatenated cell after cell (species i of cell c at c * N + i, rate
// constant j at c * R + j), and every contribution to f added with an
// atomic add.  The reaction data come in the two layouts the paper compares:
// one record per reaction ([reaction][parameter]) or the "inverted" layout,
// one array per parameter ([parameter][reaction]), which makes the reads of
// consecutive threads consecutive.  Test and measurement code, not used by
// the library's own entry points.
#include "mcc_internal.hpp"

namespace mcc {

namespace {

__global__ __launch_bounds__(1024) void zero_kernel(double *p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

// record layout: kPaperRec ints per reaction, then kPaperProd yields per reaction
__global__ __launch_bounds__(1024) void paper_deriv_records(const int32_t *__restrict__ rec,
                                                            const double *__restrict__ yld,
                                                            const double *__restrict__ y, const double *__restrict__ k,
                                                            double *f, int32_t N, int32_t R, int64_t n_cells)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_cells * R) return;
    const int64_t c = t / R;
    const int j = (int)(t - c * R);
    const int32_t *q = rec + (int64_t)j * kPaperRec;
    const double *yc = y + c * N;
    double *fc = f + c * N;
    const int nr = q[0], np = q[4];
    double r = k[c * R + j];
    for (int a = 0; a < nr; ++a) r *= yc[q[1 + a]];
    for (int a = 0; a < nr; ++a) atomicAdd(&fc[q[1 + a]], -r);
    for (int a = 0; a < np; ++a) atomicAdd(&fc[q[5 + a]], yld[(int64_t)j * kPaperProd + a] * r);
}

// inverted layout: parameter p of reaction j at p * R + j
__global__ __launch_bounds__(1024) void paper_deriv_inverted(const int32_t *__restrict__ rec,
                                                             const double *__restrict__ yld,
                                                             const double *__restrict__ y, const double *__restrict__ k,
                                                             double *f, int32_t N, int32_t R, int64_t n_cells)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_cells * R) return;
    const int64_t c = t / R;
    const int j = (int)(t - c * R);
    const double *yc = y + c * N;
    double *fc = f + c * N;
    const int nr = rec[j], np = rec[4 * R + j];
    double r = k[c * R + j];
    for (int a = 0; a < nr; ++a) r *= yc[rec[(1 + a) * R + j]];
    for (int a = 0; a < nr; ++a) atomicAdd(&fc[rec[(1 + a) * R + j]], -r);
    for (int a = 0; a < np; ++a) atomicAdd(&fc[rec[(5 + a) * R + j]], yld[(int64_t)a * R + j] * r);
}

}  // namespace

hipError_t launch_paper_deriv(const int32_t *rec, const double *yld, bool inverted, const double *y,
                              const double *k, double *f, int N, int R, int64_t n_cells, hipStream_t s)
{
    if (n_cells == 0 || R == 0) return hipSuccess;
    const int64_t nf = n_cells * N, nt = n_cells * R;
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)((nf + 1023) / 1024)), dim3(1024), 0, s, f, nf);
    const dim3 grid((unsigned)((nt + 1023) / 1024)), block(1024);
    if (inverted)
        hipLaunchKernelGGL(paper_deriv_inverted, grid, block, 0, s, rec, yld, y, k, f, N, R, n_cells);
    else
        hipLaunchKernelGGL(paper_deriv_records, grid, block, 0, s, rec, yld, y, k, f, N, R, n_cells);
    return hipGetLastError();
}

}  // namespace mcc
