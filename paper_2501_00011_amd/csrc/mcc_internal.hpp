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
constexpr int kBlk = 4;       // ops per lane per prefetched block of an op stream
// The dense tail block (M x M, M a multiple of 16) is stored column-major
// with the rows of column j permuted by row ^ 4 (j & m), m + 1 = (the largest
// power of two dividing M) / 4: consecutive rows of a column stay contiguous,
// while the 16 x 16 matrix-core tiles (16 columns of 4 rows per access) and
// the k-step operand blocks spread over all LDS banks.
__host__ __device__ constexpr int tail_swizzle_mask(int M) { return ((M & -M) >> 2) - 1; }
__host__ __device__ constexpr int tail_at(int M, int row, int col)
{
    return col * M + (row ^ (4 * (col & tail_swizzle_mask(M))));
}
constexpr int kOffBits = 14;  // bits of an LDS offset inside an op
constexpr uint32_t kOffMask = (1u << kOffBits) - 1;
// flags of a Newton-matrix op (Op16::flags)
constexpr uint32_t kFirst = 1, kLast = 2, kDiag = 4;
// An LU op (64 bits) is four 16-bit fields -- destination, l, u and the
// stored 1/U_kk, each a 14-bit LDS index from bit 0 of its field, so that a
// field is taken out with one mask or bit-field extract -- with the flags in
// the top bits of the destination and l fields.  The u and 1/U_kk fields
// carry nothing else (each is read with one multiply-add of the 16-bit
// field); where a level ends is kept on the host (HostTables::lu_barrier).
constexpr uint64_t kLuFirst = 1ull << 14, kLuLast = 1ull << 15, kLuScale = 1ull << 30, kLuRecip = 1ull << 31;

// Streaming f/J kernel tables.  A work item is a run of chunks processed by
// one wavefront in order.  A chunk computes its monomials -- the product of
// a rate-constant row and up to three y rows (index -1: the constant 1);
// padded to a multiple of kFjGroup with monomials equal to 1 -- into a
// per-lane LDS scratchpad, then runs its output records.  A record adds up
// to three terms coef * monomial[slot] (unused terms: coefficient 0 on the
// zero slot kFjQmax) to a running sum that it starts or continues, and may
// write the sum to its output row, or add it to what an earlier chunk of the
// same work item wrote there.  A chunk's records are padded to a multiple of
// kFjRecGroup with records that do nothing.
struct FjMono {
    int32_t j, a, b, c;  // k row j, y rows a, b, c (-1: the constant 1)
};
struct alignas(32) FjRec {
    double coef[3];
    uint32_t slots;  // three 8-bit scratchpad slots
    uint32_t meta;   // output row (row < N: f row, else J nonzero row - N) | flags << 24
};
constexpr uint32_t kFjKeep = 1;   // continue the running sum of the previous record
constexpr uint32_t kFjStore = 2;  // write the sum to the output row
constexpr uint32_t kFjAdd = 4;    // ... adding it to the value already there
constexpr uint32_t kFjRowMask = (1u << 24) - 1;
struct FjChunk {
    int32_t mono_begin, n_mono, rec_begin, n_rec;  // counts include padding
};
#ifndef MCC_FJ_QMAX
#define MCC_FJ_QMAX 16
#endif
constexpr int kFjQmax = MCC_FJ_QMAX;  // monomials per chunk (a multiple of kFjGroup)
constexpr int kFjGroup = 8;           // monomials whose loads are issued together
constexpr int kFjRecGroup = 4;        // records whose table loads are issued together
static_assert(kFjQmax % kFjGroup == 0 && kFjQmax < 256, "chunk size");

// A 16-byte op of the gather streams: coefficient, packed indices, flags.
// f gather: meta = the rate's index.  Newton matrix: meta = source index |
// destination << 16 (two bare 16-bit fields), flags = kFirst | kLast | kDiag.
struct alignas(16) Op16 {
    double coef;
    uint32_t meta;
    uint32_t flags;
};

// A work item of the generated VJP kernel (reverse mode of f).  With
// w_j = sum_i nu_ij v_i, gy = J^T v is gy_s = sum_j w_j d r_j / d y_s over
// the reactions with s among their reactants, and d(v.f)/d ln k_j = r_j w_j.
// An item forms gy_s for its species columns `cols` from the reactions in
// `rounds` (every reaction with a reactant in cols; each round's k, y and v
// rows are loaded together, at most kVjpRoundLoads of them unless a single
// reaction needs more) and writes d/d ln k_j for the reactions in `glnk`
// (each reaction in exactly one item: the item of its first reactant).
struct VjpItem {
    std::vector<int32_t> cols;
    std::vector<std::vector<int32_t>> rounds;
    std::vector<int32_t> glnk;
};
constexpr int kVjpRoundLoads = 64;  // measured: 48-96 beat 16-32 at 200k cells, equal at 10k

// ---------------------------------------------------------------------------
// Host-side compiled mechanism (built once by compile_mechanism).
// ---------------------------------------------------------------------------
struct HostTables {
    int N = 0, R = 0, nnz = 0, lu_nnz = 0, NS = 0, n_partials = 0;
    bool transposed = false;  // solver tables for I - c J^T

    // Jacobian pattern, species order, CSR with sorted columns, diagonal present.
    std::vector<int32_t> row_ptr, col_idx;

    // Rate constants.
    std::vector<int32_t> rxn_type;
    std::vector<double> A, theta;

    // Streaming f/J evaluation, species order.  Output rows 0..N-1 are f_i,
    // rows N..N+nnz-1 the Jacobian nonzeros in CSR order.
    std::vector<int32_t> out_ptr;     // [N + nnz + 1] algorithmic term counts
    std::vector<FjMono> fj_monos;
    std::vector<FjRec> fj_recs;
    std::vector<FjChunk> fj_chunks;
    std::vector<int32_t> fj_items;    // first chunk of every work item + end
    int n_fitems = 0, n_jitems = 0;   // f items first, then J items
    // reactions as written: reactant species per slot (-1: none) and the net
    // stoichiometry nu_ij (CSR over reactions), for the generated VJP kernel
    std::vector<int32_t> rx_sp;       // [3 * R]
    std::vector<int32_t> nu_ptr, nu_sp;
    std::vector<double> nu_coef;
    std::vector<int32_t> nu_vid;      // nu_sp as indices of the solver's compact LDS state vector
    std::vector<VjpItem> vjp_items;   // work items of the generated VJP kernel (plan_vjp)
    // the paper's Derivative kernel data (ablation): records and inverted
    std::vector<int32_t> paper_rec, paper_rec_inv;
    std::vector<double> paper_yld, paper_yld_inv;
    bool paper_ok = false;  // at most kPaperProd products per reaction

    // Solver.  Positions p = 0..N-1 are the elimination (fill-reducing)
    // order; every position lives at a virtual index v = slot * 64 + lane of
    // the per-lane register vectors and of the LDS state vector.
    std::vector<int32_t> perm;        // perm[p] = species at position p
    std::vector<int32_t> iperm;       // iperm[species] = p
    std::vector<int32_t> vspecies;    // [NV]: species at virtual index v, or -1
    std::vector<int32_t> vpos;        // [N]: virtual index of position p
    int NV = 0;                       // NS * 64
    int M = 0, F = 0;                 // dense tail size and front size (F = N - M)
    int tail_base = 0;                // LU offset of the tail block (entry (i, j) at tail_base + tail_at(M, i, j))
    std::vector<int32_t> slot_cols;   // [NS]: columns (lanes) in use per slot
    // The solver's LDS copy of the state is compact: virtual index (slot s,
    // lane l) at ybase[s] + l, with ybase[s] the lanes in use of the slots
    // before s (slot_cols); index N holds the constant 1.
    std::vector<int32_t> rx_reac;     // [4 * R]: compact reactant ids (N = one), pad
    std::vector<int32_t> part;        // [4 * P]: j, o1, o2 (other slots, compact ids, N = one), own species (virtual)
    // Op streams, laid out [block][lane][kBlk] so that a lane prefetches one
    // block (kBlk consecutive ops) with wide loads.
    // f gather: one stream per species slot (fg_blocks[s] blocks from block fg_base[s]).
    std::vector<Op16> fg_ops;
    std::vector<int32_t> fg_blocks, fg_base;
    // Newton matrix: chains of terms per LU entry.
    std::vector<Op16> nm_ops;
    int nm_blocks = 0;
    // LU: level-scheduled update / reciprocal / scale ops (kLu* layout:
    // dst | l | u | d in 16-bit fields, the flags in the top bits of dst
    // and l); lu_barrier marks the blocks that end a level.
    std::vector<uint64_t> lu_ops;
    int lu_blocks = 0, lu_steps = 0;
    std::vector<uint8_t> lu_barrier;  // per LU block: 1 if a level ends with it (host checks only)
    // Schur complement of the front pivots onto the dense tail, as FP64
    // matrix-core products (16 x 16 x 4 blocks): the tail block T (M x M)
    // receives T -= L_TF U_FT, where L_TF holds the final L entries of the tail
    // rows in the front columns and U_FT the final U entries of the front rows
    // in the tail columns.  schur_tab[(ks * 2 * nt + q) * 64 + lane] (nt =
    // M / 16) is the LU offset of the operand a lane contributes to k-step ks:
    // q < nt, the A block of tile row q (row F + 16 q + lane % 16, column
    // 4 ks + lane / 16 of L); q >= nt, the B block of tile column q - nt (row
    // 4 ks + lane / 16, column F + 16 (q - nt) + lane % 16 of U); the zero cell
    // where the entry is structurally zero or beyond the front.  Stored as
    // 16-bit offsets grouped for 16-byte loads: the entries of one lane in
    // (ks, q) order, cut into vectors of 8; vector v of lane l at
    // schur_tab[(v * 64 + l) * 8 ...].  A group of schur_sk k-steps fills
    // whole vectors; the last group is padded with the zero cell.
    std::vector<uint16_t> schur_tab;
    int schur_sk = 0;                 // k-steps per group of vectors
    int schur_ks = 0;                 // k-steps: ceil(F / 4)
    // Triangular solves: [slot][lane][NV] LU offsets per virtual column.
    std::vector<uint16_t> fwd_map, bwd_map;
    int64_t lu_lower = 0, lu_upper = 0;  // strictly lower / upper nonzeros of the sparse factors
    int64_t lu_updates = 0;           // multiply-adds per factorisation
    mcc_op_counts counts{};           // algorithmic work per cell
};

// Validates desc and fills t.  Returns MCC_OK or MCC_ERR_MECH with *err set.
// transpose: the solver tables are built for I - c J^T (reverse mode).
mcc_status compile_mechanism(const mcc_mech_desc *desc, int dense_tail, HostTables *t, std::string *err,
                             bool transpose = false);

// Host emulation of the solver's table-driven phases (testing aid).
int emulate_cell(const HostTables &t, const double *k, const double *y_species, double c,
                 const double *b_species, double *f_species, double *x_species);
// Host emulation of the streaming f/J tables for one cell (testing aid).
int emulate_fj(const HostTables &t, const double *k, const double *y_species, double *f, double *jac);
// Host emulation of the generated VJP kernel's work items for one cell
// (same plan, same arithmetic in the same order).  Returns the number of
// plan violations: a column formed twice or never, a reaction whose
// d/d ln k is written twice or never, a reaction missing from the item of
// one of its reactants, a round over the load budget with more than one
// reaction, an index out of range.
int emulate_vjp(const HostTables &t, const double *k, const double *y_species, const double *v, double *gy,
                double *glnk);
// Groups the species columns into VJP work items (see VjpItem).
std::vector<VjpItem> plan_vjp(const HostTables &t, int round_loads);

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
    const FjMono *monos;
    const FjRec *recs;
    const FjChunk *chunks;
    const int32_t *items;
    const double *y, *k, *ones;
    double *f, *jac;
    int64_t n_cells, ld;
    int32_t N, item_begin, n_items, n_tiles;
};

struct SolveParams {
    // mechanism tables (device)
    const int32_t *vspecies, *rx_reac, *part;
    const Op16 *fg_ops, *nm_ops;
    const uint64_t *lu_ops;
    const uint16_t *fwd_map, *bwd_map;
    const uint16_t *schur_tab;  // Schur complement operands (HostTables::schur_tab)
    int32_t schur_ks;
    int32_t fg_blocks[kMaxSlots], fg_base[kMaxSlots], slot_cols[kMaxSlots];
    int32_t ybase[kMaxSlots];  // compact LDS state vector: slot s at ybase[s] + lane
    int32_t nm_blocks, lu_blocks, NV, tail_base;
    int32_t N, R, P, lu_nnz;
    // LDS layout (offsets in doubles)
    int32_t off_y, off_k, off_r, off_p, off_lu, off_tm, lds_doubles;
    // batch
    const int32_t *order;  // workgroup -> cell (a permutation of the cells), or null: the identity
    const double *k;
    double *y;
    int32_t *status;
    mcc_cell_stats *stats;
    int64_t n_cells, ld;
    double dt;
    mcc_solver_opts opts;
    // per-launch form (opts.steps_per_launch > 0): solver state per cell kept
    // in HBM between launches, [n_cells][state_stride] doubles: the backward
    // differences [kMaxOrder + 3][NV], then the scalars of kStateScalars
    double *state;
    int32_t *pending;  // cells this launch left unfinished (one atomic add per cell)
    int64_t state_stride;
    int32_t call_id;   // the outer step this launch belongs to
    // Multi-cells (one system over all cells): [2][n_cells] reduction slots
    double *mc_slots;
    // step tape for reverse mode (null: none): [n_cells][tape_stride]
    // doubles in the entry format of AdjointParams, doubles used per cell in
    // tape_len (-1: the tape did not fit)
    double *tape;
    int64_t *tape_len;
    int64_t tape_stride;
};
constexpr int kStateScalars = 16;

// Step tapes: per cell, entries in time order, each [type, state (n_species
// doubles, accepted steps only), order, value, type]; types 0 start (value:
// first h), 1 re-sampling (value: factor), 2 accepted step (value:
// h / gamma_order).  kTapeScalars: the doubles of an entry besides the state.
constexpr int kTapeScalars = 4;

// Reverse mode of one outer step (adjoint_kernel), with a SolveParams built
// from the transposed solver tables.
struct AdjointParams {
    const double *tape;    // [n_cells][stride] entries, walked backwards
    const int64_t *len;    // [n_cells] doubles of the tape in use
    int64_t stride;
    const double *y0;      // [N][ld] state at the start of the outer step
    double *lam;           // [N][ld] in: dL/dy(end), out: dL/dy0
    double *glnk;          // [R][ld] dL/d ln k (overwritten, or added to)
    int32_t *status;       // [n_cells] or null
    const int32_t *nu_ptr, *nu_vid;  // net stoichiometry per reaction, virtual indices
    const double *nu_coef;
    int32_t off_w;         // LDS offset (doubles) of R + 1 scratch values (used after the last factorisation)
    int32_t accumulate;    // glnk += instead of =
};
constexpr int kAdjMaxR = 512;  // reactions per mechanism the reverse-mode kernel handles

// Replay of a tape's frozen step sequence (replay_kernel), forward solver tables.
struct ReplayParams {
    const double *tape;
    const int64_t *len;
    int64_t stride;
    const double *y0;  // [N][ld]
    double *y;         // [N][ld] out
    int32_t *status;   // [n_cells] or null
    int32_t max_newton;
    double tol;        // largest Newton correction relative to its component
};

// Launchers (enqueue only; return the launch error).
hipError_t launch_rates(const RatesParams &p, hipStream_t s);
hipError_t launch_fj(const FJParams &p, hipStream_t s);
// Mechanism-specialised f/J and VJP kernels (same work items, compiled with
// hipRTC), each in a one-cell and a two-cell (16-byte access) variant.
std::string generate_fj_source(const HostTables &t, bool pair);
std::string generate_vjp_source(const HostTables &t, bool pair);
std::string generate_module_source(const HostTables &t);  // preamble + all four
// Ablation of the paper's Derivative kernel: reaction data as records
// [reaction][kPaperRec] (n_reac, 3 reactants, n_prod, kPaperProd products)
// with yields [reaction][kPaperProd], or inverted [parameter][reaction].
constexpr int kPaperProd = 4;
constexpr int kPaperRec = 5 + kPaperProd;
hipError_t launch_paper_deriv(const int32_t *rec, const double *yld, bool inverted, const double *y,
                              const double *k, double *f, int N, int R, int64_t n_cells, hipStream_t s);  // appended to the f/J source: one module
bool compile_fj_source(const std::string &src, const std::string &arch, std::vector<char> *code, std::string *log);
// waves: wavefronts per SIMD of the build to launch (solve_waves_available).
hipError_t launch_solve(const SolveParams &p, int NS, int M, int waves, hipStream_t s);
int solve_default_waves(int NS, int M);
bool solve_waves_available(int NS, int M, int waves);
// Raise the dynamic-LDS limit of the solver kernels (once per device).
hipError_t prepare_solve_kernels(int max_lds_bytes);
// Reverse-mode kernels: shapes available, LDS limit, launch.
bool adjoint_shape_supported(int NS, int M);
hipError_t prepare_adjoint_kernels(int max_lds_bytes);
hipError_t launch_adjoint(const SolveParams &p, const AdjointParams &a, int NS, int M, hipStream_t s);
hipError_t launch_replay(const SolveParams &p, const ReplayParams &r, int NS, int M, hipStream_t s);
hipError_t launch_fill_i32(int32_t *p, int32_t v, hipStream_t s);  // *p = v by a kernel (graph-safe)
// Multi-cells solver: largest co-resident batch (0: no kernel for this shape), cooperative launch.
hipError_t multicell_capacity(int NS, int M, size_t lds_bytes, int device, int64_t *max_cells);
hipError_t launch_solve_multicell(const SolveParams &p, int NS, int M, hipStream_t s);
// Statically allocated Multi-cells reduction slots ([2][kMcScratchCells]
// doubles per device): the device address of the current device's copy,
// looked up once per device (that device must be current).
constexpr int64_t kMcScratchCells = 16384;
hipError_t multicell_scratch(int device, double **ptr);

}  // namespace mcc
