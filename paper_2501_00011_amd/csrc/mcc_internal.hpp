// Internal declarations of libmcchem: compiled mechanism tables, kernel
// parameter blocks and launchers.  Not part of the public ABI (include/mcc.h).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/mcc.h"

namespace mcc {

constexpr int kWave = 64;     // CDNA wavefront width
constexpr int kMaxOrder = 5;  // BDF orders 1..5
constexpr int kMaxSlots = 4;  // species slots per lane in the solver: N <= 256

// ---------------------------------------------------------------------------
// Host-side compiled mechanism (built once by compile_mechanism).
// ---------------------------------------------------------------------------
struct HostTables {
    int N = 0, R = 0, nnz = 0, lu_nnz = 0, NS = 0, n_partials = 0;

    // Jacobian pattern, species order, CSR with sorted columns, diagonal present.
    std::vector<int32_t> row_ptr, col_idx;

    // Rate constants.
    std::vector<int32_t> rxn_type;
    std::vector<double> A, theta;

    // Streaming f/J evaluation, species order.  Output rows 0..N-1 are f_i,
    // rows N..N+nnz-1 the Jacobian nonzeros in CSR order.  Each output is a
    // sum of monomials coef * k_j * y_a * y_b * y_c (index N = the constant 1).
    std::vector<int32_t> out_ptr;     // [N + nnz + 1]
    std::vector<int32_t> term_idx;    // [4 * n_terms]: j, a, b, c
    std::vector<double> term_coef;    // [n_terms]
    std::vector<int32_t> fj_chunks;   // row boundaries of the work chunks
    int n_fchunks = 0, n_jchunks = 0; // f chunks first, then J chunks

    // Solver, in the fill-reducing (permuted) order p = 0..N-1.
    std::vector<int32_t> perm;        // perm[p] = species at position p
    std::vector<int32_t> iperm;       // iperm[species] = p
    std::vector<int32_t> rx_reac;     // [4 * R]: permuted reactant ids (N = one), pad
    std::vector<int32_t> part;        // [4 * P]: j, o1, o2, pad (other slots, N = one)
    // f gather, ELL per slot: width fg_w[s]; entries [s][t][lane].
    std::vector<int32_t> fg_w, fg_off, fg_idx;
    std::vector<double> fg_coef;
    // Newton-matrix gather over LU entries, ELL per pass of 64 entries.
    std::vector<int32_t> jg_dest;     // [n_pass * 64]: LU offset | diag flag
    std::vector<int32_t> jg_w, jg_off, jg_idx;
    std::vector<double> jg_coef;
    // LU: per pivot k, the diagonal offset, the L column (below diagonal) and
    // the update triples (dst, l, u) packed 16/16/16 bits.
    std::vector<int32_t> lu_diag, lcol_ptr, lcol_off, upd_ptr;
    std::vector<uint64_t> upd;
    // Triangular solves: [k][slot][lane] LU offset of L(p,k) (p > k) or
    // U(p,k) (p < k), else the zero cell.
    std::vector<uint16_t> fwd_map, bwd_map;
    int64_t lu_updates = 0;           // multiply-adds per factorisation
    mcc_op_counts counts{};           // algorithmic work per cell
};

// Validates desc and fills t.  Returns MCC_OK or MCC_ERR_MECH with *err set.
mcc_status compile_mechanism(const mcc_mech_desc *desc, HostTables *t, std::string *err);

// ---------------------------------------------------------------------------
// Device parameter blocks (passed by value as kernel arguments).
// ---------------------------------------------------------------------------
struct RatesParams {
    const int32_t *rxn_type;
    const double *A, *theta;
    const double *T, *jscale;  // jscale may be null (= 1)
    double *k;
    int64_t n_cells, ld;
    int32_t R;
};

struct FJParams {
    const int32_t *out_ptr, *term_idx, *chunks;
    const double *term_coef;
    const double *y, *k;
    double *f, *jac;
    int64_t n_cells, ld;
    int32_t N, chunk_begin, n_chunks, n_tiles;
};

struct SolveParams {
    // mechanism tables (device)
    const int32_t *perm, *rx_reac, *part;
    const int32_t *fg_w, *fg_off, *fg_idx;
    const double *fg_coef;
    const int32_t *jg_dest, *jg_w, *jg_off, *jg_idx;
    const double *jg_coef;
    const int32_t *lu_diag, *lcol_ptr, *lcol_off, *upd_ptr;
    const uint64_t *upd;
    const uint16_t *fwd_map, *bwd_map;
    int32_t N, R, P, lu_nnz, n_jpass;
    // LDS layout (offsets in doubles)
    int32_t off_y, off_k, off_r, off_p, off_lu, off_invd, lds_doubles;
    // batch
    const double *k;
    double *y;
    int32_t *status;
    mcc_cell_stats *stats;
    int64_t n_cells, ld;
    double dt;
    mcc_solver_opts opts;
};

// Launchers (enqueue only; return the launch error).
hipError_t launch_rates(const RatesParams &p, hipStream_t s);
hipError_t launch_fj(const FJParams &p, hipStream_t s);
hipError_t launch_solve(const SolveParams &p, int NS, hipStream_t s);
// Raise the dynamic-LDS limit of the solver kernels (once per device).
hipError_t prepare_solve_kernels(int max_lds_bytes);

}  // namespace mcc
