/*
 * mcc.h -- C ABI of libmcchem: many independent grid cells, each integrating
 * the same stiff mass-action chemical mechanism, on one AMD Instinct MI355X
 * (gfx950) GPU in double precision.
 *
 * Paper: "Adapting atmospheric chemistry components for efficient GPU
 * accelerators" (arXiv 2501.00011).
 *   Section 2 (Background): the state array y holds species concentrations
 *     and the deriv array f their time derivatives; an ODE solver integrates
 *     y' = f(t, y) with a sparse Jacobian supplied by the chemistry; a cell
 *     is an independent volume of atmosphere with its own state.
 *   Section 2, reaction equations: c_1 y_1 + ... + c_m y_m -> ... + c_n y_n;
 *     (dy_i/dt)_j = -c_i r_j for reactants and +c_i r_j for products;
 *     f_i = sum_j (dy_i/dt)_j.
 *   Section 3 (Implementations): Multi-cells groups the data of all cells in
 *     one structure, f_ik = sum_j (dy_ik/dt)_j for species i of cell k; the
 *     reaction data lives in GPU memory from initialisation on; the device
 *     limits are checked at run time.
 *   Section 6 (Conclusions): move the Jacobian and the solver onto the GPU and
 *     move data only at the start and end of the solve -- which is what this
 *     library does: state stays in device memory across f, J and solver calls.
 *
 * Conventions
 *   Layout.   Per-cell arrays are [entity][ld] in row-major order with the
 *             cell index fastest (element (e, c) at e*ld + c), ld >= n_cells.
 *             Species arrays have n_species rows, rate constants n_reactions
 *             rows, Jacobians nnz rows in the CSR order of mcc_mech_jac_pattern.
 *   Memory.   Pointers documented as "device" are caller-owned device memory
 *             (for instance from a PyTorch CUDA/HIP tensor) on the handle's
 *             device; the library never frees them and keeps no pointer past
 *             the call.  "host" pointers are ordinary host memory.
 *   Streams.  `stream` is a hipStream_t passed as void* (NULL = the default
 *             stream).  Calls that take a stream only enqueue work and return
 *             (except the per-launch solver form, which waits for each of its
 *             launches); errors inside kernels surface at mcc_sync() or at
 *             the next synchronising call.  *_create, *_destroy and the
 *             schedule calls synchronise.
 *   Errors.   Every call returns an mcc_status; on anything but MCC_OK a
 *             message is available from mcc_last_error() (thread-local).
 *             Invalid arguments are rejected before any work is enqueued.
 *   Threads.  A handle must not be used from two threads at once; distinct
 *             handles are independent.
 */
#ifndef MCC_H
#define MCC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MCC_OK = 0,
    MCC_ERR_INVALID_ARG = 1, /* null pointer, size out of range, bad option */
    MCC_ERR_MECH = 2,        /* mechanism fails validation or exceeds device limits */
    MCC_ERR_OOM = 3,         /* device allocation failed */
    MCC_ERR_DEVICE = 4,      /* HIP runtime error (text in mcc_last_error) */
    MCC_ERR_STATE = 5,       /* call out of order (e.g. solve before bind) */
    MCC_ERR_SOLVE = 6        /* reserved: per-cell failures are reported per cell */
} mcc_status;

/* Per-cell outcome of mcc_solve_step. */
typedef enum {
    MCC_CELL_OK = 0,
    MCC_CELL_TOO_MUCH_WORK = 1, /* max_steps step attempts without reaching dt */
    MCC_CELL_CONV_FAIL = 2,     /* Newton failures drove h below its minimum */
    MCC_CELL_ERR_FAIL = 3,      /* error-test failures drove h below its minimum */
    MCC_CELL_NONFINITE = 4,     /* non-finite state or derivative */
    MCC_CELL_SINGULAR = 5,      /* zero/non-finite pivot drove h below its minimum
                                   (mcc_adjoint_step, mcc_replay_step: a singular
                                   Newton matrix) */
    MCC_CELL_BAD_TAPE = 6       /* mcc_adjoint_step, mcc_replay_step: the cell's
                                   tape is malformed or did not fit */
} mcc_cell_status;

/* Reaction types. */
enum { MCC_RXN_THERMAL = 0, MCC_RXN_PHOTOLYSIS = 1 };

/* Mechanism description (host memory, read only during mcc_mech_create).
 * Reaction j: reactant slots reac_idx[reac_ptr[j] .. reac_ptr[j+1]) (1 to 3
 * slots; a repeated species index is a stoichiometric multiplicity) and
 * products prod_idx[prod_ptr[j] .. prod_ptr[j+1]) with floating-point yields
 * (0 to 8 products).  Rate r_j = k_j * prod over slots of y_s (mass action),
 * with k_j = A_j exp(-theta_j / T) for thermal reactions (theta = Ea/R in K)
 * and k_j = A_j * s for photolysis (A_j is the J-rate, s a per-cell scale). */
typedef struct {
    int32_t n_species;          /* 1 .. MCC_MAX_SPECIES */
    int32_t n_reactions;        /* 0 .. 65535 */
    const int32_t *rxn_type;    /* [n_reactions] MCC_RXN_* */
    const int32_t *reac_ptr;    /* [n_reactions + 1], reac_ptr[0] = 0, non-decreasing */
    const int32_t *reac_idx;    /* [reac_ptr[n_reactions]] species indices */
    const int32_t *prod_ptr;    /* [n_reactions + 1] */
    const int32_t *prod_idx;    /* [prod_ptr[n_reactions]] species indices */
    const double *prod_yield;   /* [prod_ptr[n_reactions]] finite yields */
    const double *A;            /* [n_reactions] finite, >= 0 */
    const double *theta;        /* [n_reactions] finite (ignored for photolysis) */
} mcc_mech_desc;

#define MCC_MAX_SPECIES 256

/* Constants of the BDF outer step (all read by every cell):
 *   weights w_i = 1/(rtol |y_i| + atol) from the last accepted state;
 *   Newton converged when rho/(1-rho)*|dy| < eta_newton (WRMS norm);
 *   accepted-step factor = min(fac_max, safety * best order factor);
 *   rejected-step factor = max(fac_min, safety * err^(-1/(k+1)));
 *   Newton-failure factor = fac_newton_fail;
 *   failure once h < h_min_rel * dt (or h vanishes against t);
 *   max_order 1..5, max_newton 1..16, max_steps >= 1 step attempts.
 * steps_per_launch selects how the outer step is launched (the results are
 * identical bit for bit): 0 = the whole outer step of every cell in one
 * launch (the default); K > 0 = the per-launch form, in which a launch takes
 * every unfinished cell at most K accepted steps further, the cell's solver
 * state (backward differences, t, h, order, counters) kept in HBM between
 * launches, and the host relaunches until no cell is left (it waits for
 * each launch, so this form cannot be captured into a graph).
 * warm_start (0 or 1): 0 = every outer step starts afresh at order 1 with the
 * Hairer-Norsett-Wanner starting step (the per-call re-initialisation of the
 * solver that Section 3 describes for the per-cell calls); 1 = each cell
 * starts at order 1 with the step size its previous outer step would have
 * taken next, read from its stats record (stats->h_next, so stats must be
 * given and hold that step's counters; a non-positive or non-finite h_next
 * falls back to the starting-step algorithm), skipping the ramp up from a
 * tiny first step.  The Multi-cells solver requires 0. */
typedef struct {
    double rtol, atol, eta_newton, safety, fac_min, fac_max, fac_newton_fail, h_min_rel;
    int32_t max_order, max_newton, max_steps, steps_per_launch, warm_start;
} mcc_solver_opts;

/* Per-cell counters of one mcc_solve_step.  h_last: the last step size
 * taken (the landing step that ends on dt, usually shortened); h_next: the
 * step size the controller had chosen before that shortening (the step the
 * cell would take next; read back by warm_start). */
typedef struct {
    int32_t steps, rejects, newton_fails, newton_iters, f_evals, jac_evals, lu_count, order;
    double h_last, y_min, h_next;
} mcc_cell_stats;

typedef struct mcc_mech mcc_mech;
typedef struct mcc_cells mcc_cells;

/* Text of the last error on this thread ("" if none).  Never NULL. */
const char *mcc_last_error(void);

/* Library version string. */
const char *mcc_version(void);

/* Fill *opts with the defaults: rtol 1e-8, atol 1.0, eta_newton 0.03,
 * safety 0.9, fac_min 0.2, fac_max 10, fac_newton_fail 0.5, h_min_rel 1e-30,
 * max_order 5, max_newton 4, max_steps 100000, steps_per_launch 0,
 * warm_start 0. */
mcc_status mcc_solver_opts_default(mcc_solver_opts *opts);

/* Validate a mechanism, compile its tables (Jacobian pattern, gather lists,
 * fill-reducing ordering, symbolic LU and the operation schedules of the
 * solver) and upload them to `device` (Section 3: reaction data on the GPU
 * from initialisation; device limits checked at run time).  Synchronous.
 * device = -1 validates and compiles on the host only (no GPU needed): such a
 * handle answers mcc_mech_info and mcc_mech_jac_pattern, and
 * mcc_cells_create refuses it with MCC_ERR_STATE.
 * Errors: MCC_ERR_INVALID_ARG (null desc/out, bad device), MCC_ERR_MECH
 * (validation, or the per-cell solver state does not fit the device's local
 * data share), MCC_ERR_OOM, MCC_ERR_DEVICE.  On success *out owns the tables. */
mcc_status mcc_mech_create(const mcc_mech_desc *desc, int device, mcc_mech **out);

/* Choices the mechanism compiler otherwise makes itself.  dense_tail: the
 * number of trailing pivots of the solver's LU factorised as a dense block,
 * one of 0, 32, 48, 64 (at most n_species), or -1 for the compiler's cost
 * model.  Results are the same mathematics either way; the rounding order of
 * the LU differs.  waves_per_simd: the register budget of the solver build
 * launched by mcc_solve_step -- 0 the library's choice (two wavefronts per
 * SIMD for one or two species slots with a tail of at most 48, else one), 1
 * one wavefront (more registers, fewer cells per compute unit; built for
 * every shape), 2 two wavefronts (only where that is the library's choice;
 * MCC_ERR_INVALID_ARG otherwise).  Results are identical bit for bit.
 * reserved: zero. */
typedef struct {
    int32_t dense_tail;
    int32_t waves_per_simd;
    int32_t reserved[6];
} mcc_mech_config;

/* Fill *cfg with the defaults (dense_tail -1, waves_per_simd 0). */
mcc_status mcc_mech_config_default(mcc_mech_config *cfg);

/* mcc_mech_create with a configuration (NULL = defaults); an invalid choice
 * gives MCC_ERR_INVALID_ARG.  Used by the solver autotuner, which times the
 * dense-tail sizes on a sample of cells. */
mcc_status mcc_mech_create_ex(const mcc_mech_desc *desc, int device, const mcc_mech_config *cfg, mcc_mech **out);

/* Sizes of a compiled mechanism (any output pointer may be NULL):
 * species, reactions, Jacobian nonzeros (diagonal included), LU nonzeros
 * after fill, and the dynamic local-data-share bytes one cell of the solver
 * uses. */
mcc_status mcc_mech_info(const mcc_mech *mech, int32_t *n_species, int32_t *n_reactions,
                         int32_t *nnz, int32_t *lu_nnz, int32_t *solver_lds_bytes);

/* Algorithmic work of one cell for a compiled mechanism: the arithmetic the
 * method needs (sparse, no padding), not what a kernel happens to execute.
 * Flops count a multiply-add as 2. */
typedef struct {
    int64_t deriv_flops;          /* one f: sum_j arity_j products + 2 per (reaction, species) term */
    int64_t newton_matrix_flops;  /* one M = I - c J: rate partials + 2 per J term + scaling */
    int64_t lu_flops;             /* one sparse LU of M: 2 per update + pivot reciprocals + L scaling */
    int64_t solve_flops;          /* one forward + backward substitution */
    int64_t fj_bytes;             /* HBM bytes of one fused f+J: read y, k; write f, J */
    int64_t f_bytes;              /* HBM bytes of one f: read y, k; write f */
    int64_t j_bytes;              /* HBM bytes of one J: read y, k; write J */
    int64_t reserved;
} mcc_op_counts;

mcc_status mcc_mech_op_counts(const mcc_mech *mech, mcc_op_counts *counts);

/* Copy the Jacobian sparsity pattern (species order, CSR with sorted columns
 * and the diagonal always present) into caller host arrays row_ptr
 * [n_species + 1] and col_idx [nnz].  Row = tendency index i, column =
 * concentration index s (J_is = d f_i / d y_s). */
mcc_status mcc_mech_jac_pattern(const mcc_mech *mech, int32_t *row_ptr, int32_t *col_idx);

/* Testing aid (host only, works on a device -1 handle): runs the solver's
 * table-driven phases for one cell on the host exactly as the kernel
 * sequences them -- f at y, the Newton matrix M = I - c J(y), its sparse LU
 * and x = M^-1 b -- and counts table violations (offsets out of range,
 * reads or writes of an entry written by another op of the same LU level).
 * k [n_reactions], y, b, f, x [n_species] host arrays in species order.
 * *violations receives the count (0 for a sound schedule). */
mcc_status mcc_debug_emulate_cell(const mcc_mech *mech, const double *k, const double *y, double c,
                                  const double *b, double *f, double *x, int32_t *violations);

/* Testing aid (host only): as mcc_debug_emulate_cell with the solver tables
 * of the transposed system, x = (I - c J(y))^-T b (the reverse-mode step). */
mcc_status mcc_debug_emulate_cell_adjoint(const mcc_mech *mech, const double *k, const double *y, double c,
                                          const double *b, double *f, double *x, int32_t *violations);

/* Testing aid (host only): f and the sparse J of one cell from the tables of
 * the streaming f/J kernel, run on the host in the kernel's order; k
 * [n_reactions], y [n_species] in, f [n_species], jac [nnz] out (host
 * arrays); *violations counts table errors (0 for sound tables). */
mcc_status mcc_debug_emulate_fj(const mcc_mech *mech, const double *k, const double *y, double *f, double *jac,
                                int32_t *violations);

/* Testing aid (host only): the generated VJP kernel's work items for one
 * cell, run on the host in the kernel's order: gy = J^T v [n_species] and
 * glnk = d(v.f)/d ln k [n_reactions] at y with rate constants k (host
 * arrays); *violations counts plan errors (0 for a sound plan: every
 * species column formed once, every reaction's d/d ln k written once, every
 * reaction in the item of each of its reactants). */
mcc_status mcc_debug_emulate_vjp(const mcc_mech *mech, const double *k, const double *y, const double *v,
                                 double *gy, double *glnk, int32_t *violations);

/* Which f/J kernel mcc_calc_deriv / mcc_calc_jac / mcc_calc_deriv_jac of
 * this mechanism launch.  MCC_FJ_GENERATED (the default): straight-line HIP
 * written for this mechanism from its f/J tables and compiled with hipRTC
 * for the handle's device on the first such call (which then blocks for the
 * compile, a few seconds); MCC_FJ_TABLES: one generic kernel that reads the
 * same work from the tables at run time.  Both evaluate the same terms in
 * the same order (Section 2 definitions of f and J).  MCC_ERR_INVALID_ARG for
 * another kind. */
typedef enum { MCC_FJ_GENERATED = 0, MCC_FJ_TABLES = 1 } mcc_fj_kernel;
mcc_status mcc_mech_set_fj_kernel(mcc_mech *mech, int32_t kind);

/* Testing aid (host only): the generated f/J source of this mechanism.
 * Copies min(cap, len + 1) bytes, NUL-terminated when cap > len, into buf
 * (buf may be null with cap 0) and the source length to *len. */
mcc_status mcc_debug_fj_source(const mcc_mech *mech, char *buf, int64_t cap, int64_t *len);

/* Testing aid (host only, needs no GPU): compiles the generated f/J source
 * with hipRTC for the named architecture (e.g. "gfx950") without loading
 * it; *code_bytes receives the code object size.  MCC_ERR_DEVICE with the
 * compiler log in mcc_last_error() on failure. */
mcc_status mcc_debug_compile_fj(const mcc_mech *mech, const char *arch, int64_t *code_bytes);

/* Testing aid: sizes of the solver schedule, written to out[0..8]: LU
 * blocks, LU levels, Newton-matrix blocks, f-gather blocks of slots 0..3,
 * the size of the dense tail, and the wavefronts per SIMD of the solver
 * build mcc_solve_step launches. */
mcc_status mcc_debug_schedule_info(const mcc_mech *mech, int64_t *out);

/* Release a mechanism.  MCC_ERR_STATE if cell batches created from it are
 * still alive (nothing is released then). */
mcc_status mcc_mech_destroy(mcc_mech *mech);

/* A batch of n_cells cells (0 allowed: every call is then a no-op) with
 * leading dimension ld >= n_cells for every per-cell array (Section 3,
 * Multi-cells: many grid cells of one mechanism solved together, their
 * data laid out so that consecutive cells are consecutive in memory for
 * every species and reaction).  Allocates the device array of rate
 * constants [n_reactions][ld].  MCC_ERR_INVALID_ARG for n_cells < 0 or
 * ld < n_cells or n_cells > 2^31 - 1; MCC_ERR_STATE for a host-only
 * mechanism.  Synchronous. */
mcc_status mcc_cells_create(const mcc_mech *mech, int64_t n_cells, int64_t ld, mcc_cells **out);

/* Per-cell environment (device arrays [n_cells]): temperature T in K
 * (finite, > 0), pressure P in hPa (reserved: the current reaction types do
 * not use it, may be NULL), photolysis scale jscale (may be NULL = 1).
 * Computes the rate constants k [n_reactions][ld] on `stream` and keeps
 * them with the batch for every later call (Section 2: rate constants are
 * evaluated from the environment once and stored with the reaction
 * parameters; Section 4: thermal reactions follow the Arrhenius form
 * A exp(-theta / T), photolysis reactions A times the cell's scale). */
mcc_status mcc_cells_bind(mcc_cells *cells, const double *T, const double *P,
                          const double *jscale, void *stream);

/* Device pointer to the batch's rate constants [n_reactions][ld] (owned by
 * the batch, valid until mcc_cells_destroy; filled by mcc_cells_bind). */
mcc_status mcc_cells_rate_constants(const mcc_cells *cells, const double **k);

/* f = dy/dt for every cell (Section 2, derivative; Section 3, Multi-cells):
 * y, f device [n_species][ld].  MCC_ERR_STATE before mcc_cells_bind. */
mcc_status mcc_calc_deriv(const mcc_cells *cells, const double *y, double *f, void *stream);

/* Sparse Jacobian J_is = d f_i / d y_s for every cell (Section 2: sparse
 * Jacobian handed to the solver): y device [n_species][ld], jac device
 * [nnz][ld] in the CSR order of mcc_mech_jac_pattern. */
mcc_status mcc_calc_jac(const mcc_cells *cells, const double *y, double *jac, void *stream);

/* f and J in one pass over y and k (same outputs as the two calls above). */
mcc_status mcc_calc_deriv_jac(const mcc_cells *cells, const double *y, double *f, double *jac,
                              void *stream);

/* Vector-Jacobian products of f at y for every cell, for reverse-mode
 * differentiation (Section 2 definitions of f and J):
 *   gy_s   = sum_i v_i d f_i / d y_s            (gy = J^T v),
 *   glnk_j = sum_i v_i d f_i / d ln k_j = r_j sum_i nu_ij v_i
 * (f is linear in each k_j).  y, v, gy device [n_species][ld]; glnk device
 * [n_reactions][ld]; one of gy and glnk may be NULL.  Uses the generated
 * kernel of the mechanism (compiled on the first call, as for f/J). */
mcc_status mcc_calc_vjp(const mcc_cells *cells, const double *y, const double *v, double *gy, double *glnk,
                        void *stream);

/* Ablation (measurement aid, not the library's path): the paper's GPU
 * Derivative kernel (Section 3) -- one thread per (cell, reaction), 1024
 * threads per block, f accumulated with atomic adds -- on the paper's
 * concatenated layout: y, f device [n_cells][n_species] (species i of cell c
 * at c * n_species + i), k device [n_cells][n_reactions].  inverted = 0
 * reads the reaction data as one record per reaction, 1 as one array per
 * parameter (the paper's inversion).  f is zeroed by the call.  MCC_ERR_MECH
 * if a reaction has more than 4 products. */
mcc_status mcc_ablation_paper_deriv(const mcc_mech *mech, int64_t n_cells, const double *y, const double *k,
                                    double *f, int32_t inverted, void *stream);

/* Replace the batch's rate constants by caller values (device [n_reactions]
 * [ld], copied on `stream`), e.g. k = exp(ln k) of a parameter being
 * differentiated; the batch then counts as bound. */
mcc_status mcc_cells_set_rate_constants(mcc_cells *cells, const double *k, void *stream);

/* One outer step of length dt > 0 for every cell: each cell integrates
 * y' = f(y) from 0 to dt on its own with the variable-order BDF method and a
 * Newton iteration on a sparse LU of I - (h/gamma_k) J (Section 2: solver
 * with a sparse Jacobian; Section 6: the whole solve on the GPU).
 * y: device [n_species][ld], overwritten with y(dt).  cell_status: device
 * int32 [n_cells] (mcc_cell_status).  stats: device mcc_cell_stats
 * [n_cells] or NULL (required with opts->warm_start, which reads each
 * record's h_next before overwriting the record).  opts: host, NULL =
 * defaults.  A cell that fails keeps its last accepted state; other cells are
 * unaffected. */
mcc_status mcc_solve_step(mcc_cells *cells, double *y, double dt, const mcc_solver_opts *opts,
                          int32_t *cell_status, mcc_cell_stats *stats, void *stream);

/* The step sequence of each cell's tape (format of mcc_adjoint_step) run
 * again from y0 with the batch's current rate constants: the map whose
 * derivative mcc_adjoint_step computes, for checking it by finite
 * differences (Section 2 solver with its steps frozen).  The start and the
 * re-samplings are applied as taped; each accepted step solves its implicit
 * equation by Newton with a fresh Newton matrix at every iterate, starting
 * from the taped state, until the largest correction relative to its
 * component is at most tol, or for max_newton iterations.  y0, y device
 * [n_species][ld] (y receives the end state; NaN for a failed cell).
 * cell_status as mcc_adjoint_step (MCC_CELL_SINGULAR: a Newton matrix was
 * singular).  An empty tape maps y0 to itself.  Mechanism shapes as
 * mcc_adjoint_step. */
mcc_status mcc_replay_step(const mcc_cells *cells, const double *y0, const double *tape, const int64_t *tape_len,
                           int64_t tape_stride, double *y, int32_t max_newton, double tol, int32_t *cell_status,
                           void *stream);

/* mcc_solve_step recording every cell's step tape for mcc_adjoint_step
 * (the entry format described there): tape device doubles [n_cells]
 * [tape_stride >= 4], tape_len device int64 [n_cells] receives the doubles
 * written per cell, or -1 when the cell's tape did not fit in tape_stride
 * (its solve is unaffected; mcc_adjoint_step then reports MCC_CELL_BAD_TAPE).
 * A cell takes at most 4 + 8 * attempts + n_species * steps doubles (steps
 * as in mcc_cell_stats; attempts = steps + rejects + newton_fails).
 * The tape starts from the y passed in: keep a copy of it for the reverse
 * pass.  Also in the per-launch form. */
mcc_status mcc_solve_step_taped(mcc_cells *cells, double *y, double dt, const mcc_solver_opts *opts,
                                int32_t *cell_status, mcc_cell_stats *stats, double *tape, int64_t *tape_len,
                                int64_t tape_stride, void *stream);

/* The paper's Multi-cells mode (Section 3: the data of every cell grouped
 * into one structure and solved as one system; Section 5: the solver then
 * needs about as many iterations for all cells as for one): one outer step
 * of length dt in which all cells form one ODE system of n_species x n_cells
 * unknowns with one shared step size and order, every WRMS norm taken over
 * all cells, and one Newton iteration for the whole system (the Jacobian is
 * block-diagonal, factorised cell by cell).  Arguments as mcc_solve_step;
 * every cell gets the system's status, and the system's counters in its
 * stats (y_min is the cell's own).  All cells are resident at once (a
 * cooperative launch), so n_cells is limited by the device
 * (MCC_ERR_INVALID_ARG beyond, with the limit in mcc_last_error());
 * opts->steps_per_launch must be 0.  Implemented for mechanisms whose
 * solver uses one slot, or two slots with no or a 48-row dense tail (up to
 * about 110 species). */
mcc_status mcc_solve_step_multicell(mcc_cells *cells, double *y, double dt, const mcc_solver_opts *opts,
                                    int32_t *cell_status, mcc_cell_stats *stats, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * mcc_solve_step_multicell with the grid-wide reduction slots in a
 * statically allocated device array of the library (256 KiB per device,
 * held until the process ends) instead of memory the batch allocates on
 * first use.  Arguments, results and errors as mcc_solve_step_multicell;
 * MCC_ERR_INVALID_ARG for more than 16,384 cells.  The call itself
 * allocates nothing (no hipMalloc or hipFree; the caller passes y, the
 * statuses and the counters).  Every call on one device shares that
 * device's slots: calls that overlap on one device (other streams, other
 * threads) race and give wrong results; calls in sequence are independent
 * (each writes every slot it reads). */
mcc_status mcc_solve_step_multicell_noalloc(mcc_cells *cells, double *y, double dt, const mcc_solver_opts *opts,
                                            int32_t *cell_status, mcc_cell_stats *stats, void *stream);

/* Reverse mode of one outer step (the discrete adjoint of the BDF step
 * sequence of mcc_solve_step, Section 2 solver, with that sequence frozen):
 * given lam = dL/dy(dt), overwrite lam with dL/dy0 and write (accumulate != 0:
 * add) dL/d ln k_j to glnk, for every cell.  The step sequence of each cell
 * is its tape: device doubles [n_cells][tape_stride], cell c using the first
 * tape_len[c] (device int64 [n_cells]).  Entries are written in time order,
 * each as [type, payload, order, value, type] (the type at both ends, so a
 * tape can be walked either way):
 *   type 0, start: value = the first step size h (D_0 = y0, D_1 = h f(y0));
 *   type 1, re-sampling of the differences D_0..D_order to spacing value * h;
 *   type 2, accepted step of order k with value c = h / gamma_k; payload:
 *        the step's converged state z (n_species values, species order).
 * Other entries have no payload.  Every tape starts with one type-0 entry.  For a step the transpose of
 * I - c J(z) is factorised with the mechanism's transposed solver tables.
 * y0 device [n_species][ld] (the state the tape starts from), lam device
 * [n_species][ld] in/out, glnk device [n_reactions][ld], cell_status device
 * int32 [n_cells] or NULL: MCC_CELL_OK, MCC_CELL_SINGULAR, or
 * MCC_CELL_BAD_TAPE (that cell's outputs are NaN).  MCC_ERR_MECH when the
 * mechanism has no reverse-mode kernel (the reason in mcc_last_error()):
 * it is built for one or two species slots with no, a 32-, 48- or 64-row
 * dense tail, three slots with a 64-row tail (up to about 190 species), and
 * at most 512 reactions. */
mcc_status mcc_adjoint_step(const mcc_cells *cells, const double *y0, const double *tape, const int64_t *tape_len,
                            int64_t tape_stride, double *lam, double *glnk, int32_t accumulate,
                            int32_t *cell_status, void *stream);

/* Cell schedule of the per-cell solver kernels (mcc_solve_step and its
 * per-launch and taped forms, mcc_adjoint_step, mcc_replay_step): workgroup i
 * integrates cell order[i], so cells listed first start first.  Cells whose
 * integrations take many steps listed first shorten the tail of a launch
 * (longest-processing-time-first); the per-cell counters of the previous
 * outer step (mcc_cell_stats) predict them.  order: host int32 [n_cells], a
 * permutation of 0..n_cells-1 (MCC_ERR_INVALID_ARG otherwise), copied by the
 * call; NULL restores the identity.  Results do not depend on the schedule
 * (every cell's integration is independent of the others).  Synchronises
 * the device.  The Multi-cells solver ignores it. */
mcc_status mcc_cells_set_schedule(mcc_cells *cells, const int32_t *order);

/* mcc_cells_set_schedule with the cells ordered longest first by the step
 * attempts (steps + rejects + newton_fails) of a previous outer step:
 * stats device mcc_cell_stats [n_cells] as mcc_solve_step wrote them
 * (copied to the host; synchronous).  Equal counts keep their cell order.
 * order_out: host int32 [n_cells] receiving the schedule, or NULL. */
mcc_status mcc_cells_schedule_from_stats(mcc_cells *cells, const mcc_cell_stats *stats, int32_t *order_out);

/* mcc_cells_schedule_from_stats with a choice of order (the solver
 * autotuner times them): MCC_SCHEDULE_LONGEST_FIRST as above, or
 * MCC_SCHEDULE_ZIGZAG, the longest-first list taken alternately from its two
 * ends (longest, shortest, second longest, ...).  MCC_ERR_INVALID_ARG for
 * another kind. */
enum { MCC_SCHEDULE_LONGEST_FIRST = 0, MCC_SCHEDULE_ZIGZAG = 1 };
mcc_status mcc_cells_schedule_from_stats_ex(mcc_cells *cells, const mcc_cell_stats *stats, int32_t kind,
                                            int32_t *order_out);

/* Wait for all work of this batch's device and report any asynchronous error. */
mcc_status mcc_sync(mcc_cells *cells);

/* Release a batch.  Synchronous. */
mcc_status mcc_cells_destroy(mcc_cells *cells);

#ifdef __cplusplus
}
#endif

#endif /* MCC_H */
