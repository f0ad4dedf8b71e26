// One BDF outer step per cell: a whole wavefront (64 lanes) integrates one
// cell from t = 0 to t = dt, so every control decision (Newton convergence,
// error test, step size and order) is uniform across the wavefront and cells
// of different stiffness never make lanes diverge; the hardware dispatcher
// hands a finished wavefront's compute unit the next cell.
//
// Method (variable-order BDF in backward-difference form, orders 1..5, with a
// simplified Newton iteration on a freshly evaluated Jacobian at every step
// attempt; Shampine & Reichelt 1997, kappa = 0; Hairer-Norsett-Wanner starting
// step).  It is the per-cell solve of Section 2 (an implicit solver with a
// sparse Jacobian) moved entirely onto the GPU as Section 6 proposes: the
// state never leaves the device between f, J and linear-solver calls.
//
// Per-cell storage
//   registers : every per-species vector at virtual index v = s*64 + lane,
//               s = 0..NS-1 (the mechanism compiler maps species to v): the
//               backward differences D[0..7], the Newton correction, ...;
//               during the factorisation also the dense tail of the LU
//               (lane = row).
//   LDS       : the evaluation point y, compact (slot s, lane l at the
//               lanes in use of the earlier slots + l; then the constant 1),
//               the cell's rate constants, one scratch region for the
//               reaction rates, the rate partials or the 6 x 6 transform of a
//               step-size change (never live together), and the LU factors
//               (1/U_kk in place of U_kk; the tail block column-major; + a
//               zero cell and a write-only cell).
//   HBM       : y in/out, k in, status and stats out; in the per-launch form
//               the solver state between launches; when taping, the step
//               tape.
#include <hip/hip_cooperative_groups.h>

#include <map>
#include <mutex>

#include "mcc_internal.hpp"

namespace mcc {
namespace {

// Every workgroup of the kernels below is one wavefront (64 lanes, one cell),
// and a wavefront's local-memory instructions are performed in the order it
// issues them.  A hand-over of local memory between its lanes therefore needs
// only that the compiler keep the accesses in program order on either side:
// a fence at wavefront scope, which emits no instruction and no wait (a
// workgroup barrier would also wait for every outstanding local-memory access
// to complete).
__device__ __forceinline__ void lds_handover() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); }

__device__ __forceinline__ double lane_bcast(double v, int src_lane)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), src_lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src_lane);
    return __hiloint2double(hi, lo);
}

// The value of another lane of the same row of 16, by a DPP lane pattern
// (no local-memory round trip).
template <int CTRL>
__device__ __forceinline__ double row_move(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

// Reduction over the 64 lanes (all active): within each row of 16 lanes by
// exchanges with lane ^ 1, lane ^ 2 (quad patterns), then the mirror lane of
// the half row and of the row, so that every lane of a row holds the row's
// result (each exchange combines two equal partial results, so the lanes of a
// row agree bit for bit); then the four row results combined in one fixed
// order on every lane.
template <class Op>
__device__ __forceinline__ double wave_reduce(double v, Op op)
{
    v = op(v, row_move<0xb1>(v));   // quad_perm [1, 0, 3, 2]
    v = op(v, row_move<0x4e>(v));   // quad_perm [2, 3, 0, 1]
    v = op(v, row_move<0x141>(v));  // row_half_mirror
    v = op(v, row_move<0x140>(v));  // row_mirror
    return op(op(lane_bcast(v, 0), lane_bcast(v, 16)), op(lane_bcast(v, 32), lane_bcast(v, 48)));
}

__device__ __forceinline__ double wave_sum(double v)
{
    return wave_reduce(v, [](double a, double b) { return a + b; });
}

__device__ __forceinline__ double wave_min(double v)
{
    return wave_reduce(v, [](double a, double b) { return fmin(a, b); });
}

// This lane's index, taken afresh where a phase begins.  The empty asm makes
// it a new value on every call, so the lane predicates of the phase (64-bit
// masks in scalar registers) are formed where they are used: the compiler
// would otherwise move them out of the solver loop, keep dozens of them live
// across it and spill them to vector-register lanes, each use then costing
// two readlane instructions instead of one compare.
__device__ __forceinline__ int lane_here()
{
    int l = (int)threadIdx.x;
    asm volatile("" : "+v"(l));
    return l;
}

// 1/x of a pivot (finite and not tiny: checked before use): the hardware's
// reciprocal estimate refined by two Newton steps r <- r + r (1 - x r),
// within about an ulp, in five dependent instructions where an IEEE-rounded
// division takes about twice as many; it sits in the dense tail's chain of
// pivots, and in the front factorisation's level steps.
__device__ __forceinline__ double pivot_rcp(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    r = fma(r, fma(-x, r, 1.0), r);
    return fma(r, fma(-x, r, 1.0), r);
}

// A value the same on every lane, marked so for the compiler (readfirstlane
// of both halves): decisions taken on it are then scalar branches, not
// per-lane masks.
__device__ __forceinline__ double uniform(double x)
{
    return __hiloint2double(__builtin_amdgcn_readfirstlane(__double2hiint(x)),
                            __builtin_amdgcn_readfirstlane(__double2loint(x)));
}

// The step-size factors need x^y a few times per step; one out-of-line copy
// of the FP64 power function keeps its temporaries out of the solver loop.
// Its arguments are uniform, but its result comes back in a vector register,
// which the compiler would take as varying across lanes (and with it the
// step size, the order and every decision on them).
__device__ __noinline__ double step_pow_call(double x, double y) { return pow(x, y); }
__device__ __forceinline__ double step_pow(double x, double y) { return uniform(step_pow_call(x, y)); }

// gamma_j = sum_{i=1..j} 1/i, summed in that order; the reciprocals are
// compile-time constants, so a run-time j costs no division.
__device__ __forceinline__ double bdf_gamma(int j)
{
    double g = 0.0;
#pragma unroll
    for (int i = 1; i <= kMaxOrder; ++i) g = i <= j ? g + 1.0 / i : g;
    return g;
}

// Reads one lane's op stream, laid out [block][lane][kBlk] in global memory,
// one block ahead of its use: the next block's loads are in flight while the
// current block's LDS work runs, so table latency stays off the critical path.
template <class T>
struct Prefetcher {
    const T *base;
    int lane, nblk, blk;
    T nxt[kBlk];

    __device__ __forceinline__ void start(const T *b, int ln, int nb)
    {
        base = b;
        lane = ln;
        nblk = nb;
        blk = 0;
        if (nb > 0) fetch(0);
    }
    __device__ __forceinline__ void fetch(int bi)
    {
        const T *q = base + ((size_t)bi * kWave + lane) * kBlk;
#pragma unroll
        for (int i = 0; i < kBlk; ++i) nxt[i] = q[i];
    }
    __device__ __forceinline__ void take(T (&cur)[kBlk])
    {
#pragma unroll
        for (int i = 0; i < kBlk; ++i) cur[i] = nxt[i];
        ++blk;
        if (blk < nblk) fetch(blk);
    }
};

// Entry e of a table of 16-bit LDS indices packed two to a 32-bit word,
// read from the double array whose LDS byte address is base: index * 8 +
// base is one v_mad_u32_u16 (its op_sel picks the word's high half), where
// an extract and a shift-add take two vector instructions.  A generic
// pointer into LDS carries the LDS byte address in its low 32 bits.
__device__ __forceinline__ uint32_t lds_base(const double *p) { return (uint32_t)(uintptr_t)p; }

// (e is a compile-time constant wherever this is inlined: the loops around
// every use are unrolled)
__device__ __forceinline__ uint32_t lds_addr(const uint32_t *w, int e, uint32_t base)
{
    uint32_t a;
    if (e & 1)
        asm("v_mad_u32_u16 %0, %1, 8, %2 op_sel:[1,0,0,0]" : "=v"(a) : "v"(w[e >> 1]), "s"(base));
    else
        asm("v_mad_u32_u16 %0, %1, 8, %2" : "=v"(a) : "v"(w[e >> 1]), "s"(base));
    return a;
}

__device__ __forceinline__ __attribute__((address_space(3))) double &lds_ref(uint32_t a)
{
    return *reinterpret_cast<__attribute__((address_space(3))) double *>(static_cast<uintptr_t>(a));
}

__device__ __forceinline__ double lds_field(const uint32_t *w, int e, uint32_t base) { return lds_ref(lds_addr(w, e, base)); }

// the eight entries of a 16-byte group
__device__ __forceinline__ void lds_fields8(const uint32_t (&w)[4], uint32_t base, double (&v)[8])
{
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = lds_field(w, e, base);
}


typedef double v4d __attribute__((ext_vector_type(4)));

template <int NS, int M>
struct Cell {
    const SolveParams &p;
    double *yv, *kv, *rv, *pv, *lu, *tm;
    int lane;
    int N;
    bool vld[NS];

    __device__ Cell(const SolveParams &pp, double *smem)
        : p(pp), yv(smem + pp.off_y), kv(smem + pp.off_k), rv(smem + pp.off_r), pv(smem + pp.off_p),
          lu(smem + pp.off_lu), tm(smem + pp.off_tm), lane((int)threadIdx.x), N(pp.N)
    {
#pragma unroll
        for (int s = 0; s < NS; ++s) vld[s] = pp.vspecies[s * kWave + lane] >= 0;
    }

    __device__ __forceinline__ bool valid(int s) const { return vld[s]; }

    // The launch parameters, read afresh where a phase begins (the empty asm
    // makes the pointer a new value on every call): the compiler would
    // otherwise load every field the loop uses once, keep them all in scalar
    // registers across the loop and spill them to vector-register lanes; a
    // scalar load per phase is cheaper than two readlanes per use.  Every
    // kernel that builds a Cell takes its SolveParams, unchanged, as its first
    // argument, at offset 0 of the kernel-argument segment.
    typedef const __attribute__((address_space(4))) SolveParams KParams;
    __device__ __forceinline__ KParams &params_here() const
    {
        KParams *q = (KParams *)__builtin_amdgcn_kernarg_segment_ptr();
        asm volatile("" : "+s"(q));
        return *q;
    }

    // offset of entry (row, col) in the tail block (column-major, the rows
    // of a column permuted against LDS bank conflicts: tail_at)
    static __device__ __forceinline__ int tat(int row, int col) { return tail_at(M, row, col); }

    // order of slot s in the elimination order: the front slots 1.. come
    // before the dense tail in slot 0
    static constexpr int ord(int s) { return M > 0 ? (s == 0 ? NS - 1 : s - 1) : s; }

    __device__ __forceinline__ void put_y(const double (&v)[NS])
    {
        lds_handover();
#pragma unroll
        for (int s = 0; s < NS; ++s)
            if (lane < p.slot_cols[s]) yv[p.ybase[s] + lane] = v[s];
        lds_handover();
    }

    // f at v: reaction rates r_j = k_j y_a y_b y_c (lane per reaction), then
    // f_v = sum nu r gathered per virtual index (lane per index).
    __device__ __forceinline__ void deriv(const double (&v)[NS], double (&f)[NS])
    {
        rates(v);
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            Prefetcher<Op16> st;
            st.start(p.fg_ops + (size_t)p.fg_base[s] * kWave * kBlk, lane, p.fg_blocks[s]);
            double acc = 0.0;
            for (int b = 0; b < p.fg_blocks[s]; ++b) {
                Op16 op[kBlk];
                st.take(op);
                double r[kBlk];
#pragma unroll
                for (int i = 0; i < kBlk; ++i) r[i] = rv[op[i].meta];
#pragma unroll
                for (int i = 0; i < kBlk; ++i) acc += op[i].coef * r[i];
            }
            f[s] = acc;
        }
    }

    // Reaction rates at v into rv (lane per reaction); rv[R] = 0.
    __device__ __forceinline__ void rates(const double (&v)[NS])
    {
        // the first round's reactant ids are requested before y is stored,
        // so that their global-memory latency overlaps that store
        const int4 *rx = reinterpret_cast<const int4 *>(p.rx_reac);
        int4 a[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int j = u * kWave + lane;
            a[u] = j < p.R ? rx[j] : make_int4(p.NV, p.NV, p.NV, 0);
        }
        put_y(v);
        for (int j0 = 0; j0 < p.R; j0 += 4 * kWave) {
            if (j0 > 0)
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int j = j0 + u * kWave + lane;
                    a[u] = j < p.R ? rx[j] : make_int4(p.NV, p.NV, p.NV, 0);
                }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int j = j0 + u * kWave + lane;
                if (j < p.R) {
                    double r = kv[j] * yv[a[u].x];
                    r *= yv[a[u].y];
                    r *= yv[a[u].z];
                    rv[j] = r;
                }
            }
        }
        if (lane == 0) rv[p.R] = 0.0;  // the zero rate idle gather lanes read
        lds_handover();
    }

    // Newton matrix M = I - c J(v) written over the LU storage (fill = 0).
    __device__ __forceinline__ void newton_matrix(const double (&v)[NS], double c)
    {
        KParams &p = params_here();
        partials(v);
        Prefetcher<Op16> st;
        st.start(p.nm_ops, lane, p.nm_blocks);
        const uint32_t pvb = lds_base(pv), lub = lds_base(lu);
        double acc = 0.0;
        for (int b = 0; b < p.nm_blocks; ++b) {
            Op16 op[kBlk];
            st.take(op);
            double x[kBlk];
#pragma unroll
            for (int i = 0; i < kBlk; ++i) x[i] = lds_field(&op[i].meta, 0, pvb);
#pragma unroll
            for (int i = 0; i < kBlk; ++i) {
                const uint32_t fl = op[i].flags;
                acc = (fl & kFirst) ? op[i].coef * x[i] : acc + op[i].coef * x[i];
                if (fl & kLast) {
                    const double m = -c * acc;
                    lds_ref(lds_addr(&op[i].meta, 1, lub)) = (fl & kDiag) ? 1.0 + m : m;
                }
            }
        }
        lds_handover();
    }

    // Rate partials d r_j / d y_s at v into pv (lane per partial); pv[P] = 0.
    __device__ __forceinline__ void partials(const double (&v)[NS])
    {
        KParams &p = params_here();
        const int4 *pt = reinterpret_cast<const int4 *>(p.part);
        int4 a[4];  // requested before y is stored, as in rates()
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int q = u * kWave + lane;
            a[u] = q < p.P ? pt[q] : make_int4(0, p.NV, p.NV, 0);
        }
        put_y(v);
        for (int q0 = 0; q0 < p.P; q0 += 4 * kWave) {
            if (q0 > 0)
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int q = q0 + u * kWave + lane;
                    a[u] = q < p.P ? pt[q] : make_int4(0, p.NV, p.NV, 0);
                }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int q = q0 + u * kWave + lane;
                if (q < p.P) {
                    double d = kv[a[u].x] * yv[a[u].y];
                    d *= yv[a[u].z];
                    pv[q] = d;
                }
            }
        }
        if (lane == 0) pv[p.P] = 0.0;  // the zero partial of fill entries and idle lanes
        lds_handover();
    }

    // Front pivots: level-scheduled right-looking sparse LU with the static
    // diagonal pivot order.  Each op: acc = a[dst] (first of a chain);
    // acc -= a[l] * a[d] * a[u] (a[d] holds 1/U_kk) or acc *= a[d] (column
    // scaling); a[dst] = acc, or 1/acc when it completes a pivot (last of a
    // chain).  All operands of a block are read before any of its writes:
    // inside one level no op reads what another op of that level writes.
    // Then the dense tail.  Returns true if a pivot is zero, tiny or not
    // finite (uniform across the wavefront).
    __device__ __forceinline__ bool factor()
    {
        KParams &p = params_here();
        Prefetcher<uint64_t> st;
        st.start(p.lu_ops, lane, p.lu_blocks);
        const uint32_t lub = lds_base(lu);
        double acc = 0.0;
        int bad = 0;
        for (int b = 0; b < p.lu_blocks; ++b) {
            uint64_t op[kBlk];
            st.take(op);
            double ad[kBlk], al[kBlk], au[kBlk], ag[kBlk];
#pragma unroll
            for (int i = 0; i < kBlk; ++i) {
                const uint32_t w[2] = {(uint32_t)op[i], (uint32_t)(op[i] >> 32)};
                ad[i] = lu[w[0] & kOffMask];
                al[i] = lu[(w[0] >> 16) & kOffMask];
                au[i] = lds_field(w, 2, lub);  // bare 16-bit fields
                ag[i] = lds_field(w, 3, lub);
            }
            bool any_recip = false;
            double res[kBlk];
            int dst[kBlk];
            bool store[kBlk], recip[kBlk];
#pragma unroll
            for (int i = 0; i < kBlk; ++i) {
                const double a0 = (op[i] & kLuFirst) ? ad[i] : acc;
                // a scaling op reads the zero cell for l and u, so one form
                // serves both kinds: (a0 or a0 / U_kk) - l / U_kk * u.  Every
                // operand is then used on every lane, and no branch per op
                // re-reads l and u inside it.
                acc = ((op[i] & kLuScale) ? a0 * ag[i] : a0) - (al[i] * ag[i]) * au[i];
                res[i] = acc;
                dst[i] = (int)(op[i] & kOffMask);
                store[i] = op[i] & kLuLast;
                recip[i] = op[i] & kLuRecip;
                any_recip |= recip[i];
            }
            if (__any(any_recip)) {
#pragma unroll
                for (int i = 0; i < kBlk; ++i)
                    if (recip[i]) {
                        bad |= !(fabs(res[i]) >= 1e-300) || !isfinite(res[i]);
                        res[i] = pivot_rcp(res[i]);
                    }
            }
#pragma unroll
            for (int i = 0; i < kBlk; ++i)
                if (store[i]) lu[dst[i]] = res[i];
            // the next level reads what this one wrote: keep the order
            lds_handover();
        }
        const bool front_bad = __any(bad);
        schur();
        const bool tail_bad = dense_tail();
        return front_bad || tail_bad;
    }

    // Schur complement of the front onto the dense tail: T -= L_TF U_FT with
    // the FP64 16 x 16 x 4 matrix-core product (the tail block is dense after
    // the fill-reducing order, so this is a dense contraction).  A k-step
    // brings one 16 x 4 block of L per tile row and one 4 x 16 block of U per
    // tile column (a lane holds entry (lane % 16, lane / 16) of an A block and
    // (lane / 16, lane % 16) of a B block; structurally zero entries read the
    // zero cell).  An accumulator tile holds, in lane l and register r, the
    // entry (4 r + l / 16, l % 16); tiles start from and go back to the
    // column-major tail block.  The operand offsets of SK k-steps arrive with
    // one group of 16-byte loads per lane (the table is laid out [vector]
    // [lane][8 offsets]); tile rows are taken TI at a time.
    static constexpr int NT = M / 16;
    static constexpr int SK = NT == 3 ? 4 : (NT > 0 ? 16 / NT : 1);  // k-steps per table group (2 NT SK % 8 == 0)
    static constexpr int SV = (2 * NT * SK) / 8;                      // 16-byte vectors per group

    __device__ __forceinline__ void schur()
    {
        KParams &p = params_here();
        if constexpr (M > 0) {
            constexpr int TI = NT <= 2 ? NT : 1;
            const int KS = p.schur_ks;
            if (KS == 0) return;
            const int g = lane >> 4, c16 = lane & 15;
            double *tb = lu + p.tail_base;
            const uint4 *tab = reinterpret_cast<const uint4 *>(p.schur_tab) + lane;
            const uint32_t lub = lds_base(lu);
#pragma unroll
            for (int i0 = 0; i0 < NT; i0 += TI) {
                v4d acc[TI][NT];
#pragma unroll
                for (int i = 0; i < TI; ++i)
#pragma unroll
                    for (int j = 0; j < NT; ++j)
#pragma unroll
                        for (int r = 0; r < 4; ++r) acc[i][j][r] = tb[tat(16 * (i0 + i) + 4 * r + g, 16 * j + c16)];
                for (int k0 = 0; k0 < KS; k0 += SK) {
                    uint32_t w[4 * SV];
#pragma unroll
                    for (int v = 0; v < SV; ++v) {
                        const uint4 o = tab[(size_t)((k0 / SK) * SV + v) * kWave];
                        w[4 * v] = o.x;
                        w[4 * v + 1] = o.y;
                        w[4 * v + 2] = o.z;
                        w[4 * v + 3] = o.w;
                    }
#pragma unroll
                    for (int kk = 0; kk < SK; ++kk) {
                        if (k0 + kk >= KS) break;
                        double a[TI], b[NT];
#pragma unroll
                        for (int i = 0; i < TI; ++i) a[i] = -lds_field(w, kk * 2 * NT + i0 + i, lub);
#pragma unroll
                        for (int j = 0; j < NT; ++j) b[j] = lds_field(w, kk * 2 * NT + NT + j, lub);
#pragma unroll
                        for (int i = 0; i < TI; ++i)
#pragma unroll
                            for (int j = 0; j < NT; ++j)
                                acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
                    }
                }
#pragma unroll
                for (int i = 0; i < TI; ++i)
#pragma unroll
                    for (int j = 0; j < NT; ++j)
#pragma unroll
                        for (int r = 0; r < 4; ++r) tb[tat(16 * (i0 + i) + 4 * r + g, 16 * j + c16)] = acc[i][j][r];
            }
            lds_handover();
        }
    }

    // Dense tail (the Schur complement left by the front pivots), M x M in
    // LDS (entry (i, j) at tat(i, j)), factorised in place by blocked
    // right-looking LU with panels of four columns:
    //   1. the panel (its four columns, all rows): lane = row, the pivot row's
    //      values broadcast with readlane; 1/U_kk replaces U_kk;
    //   2. the panel's four rows right of it: U12 = L11^-1 A12, lane = column;
    //   3. the trailing matrix: A22 -= L21 U12 with the FP64 16 x 16 x 4
    //      matrix-core product on the 16 x 16 tiles that meet A22 (the
    //      operands' entries outside A22 read as zero, so the rest of such a
    //      tile is unchanged).
    // Returns true if a pivot is zero, tiny or not finite (uniform).
    __device__ __forceinline__ bool dense_tail()
    {
        KParams &p = params_here();
        if constexpr (M == 0) {
            return false;
        } else {
            double *T = lu + p.tail_base;
            const int lane = lane_here();
            const bool in = lane < M;
            const int row = in ? lane : 0;  // this lane's row (panel phase) or column (row phase)
            const int g = lane >> 4, c16 = lane & 15;
            bool bad = false;
#pragma unroll 1
            for (int k0 = 0; k0 < M; k0 += 4) {
                // 1. panel
                double a[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) a[c] = T[tat(row, k0 + c)];
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    const int k = k0 + kk;
                    const double ukk = lane_bcast(a[kk], k);
                    bad |= !(fabs(ukk) >= 1e-300) || !isfinite(ukk);
                    const double inv = pivot_rcp(ukk);
                    if (lane > k && in) {
                        const double l = a[kk] * inv;
                        a[kk] = l;
#pragma unroll
                        for (int c = kk + 1; c < 4; ++c) a[c] -= l * lane_bcast(a[c], k);
                    }
                    if (lane == k) a[kk] = inv;
                }
                if (in && lane >= k0)
#pragma unroll
                    for (int c = 0; c < 4; ++c) T[tat(row, k0 + c)] = a[c];
                lds_handover();
                const int kt = k0 + 4;
                if (kt >= M) break;
                // 2. the panel's rows right of it (unit lower L11 from the panel)
                if (lane >= kt && in) {
                    const double l10 = T[tat(k0 + 1, k0)], l20 = T[tat(k0 + 2, k0)], l30 = T[tat(k0 + 3, k0)];
                    const double l21 = T[tat(k0 + 2, k0 + 1)], l31 = T[tat(k0 + 3, k0 + 1)];
                    const double l32 = T[tat(k0 + 3, k0 + 2)];
                    const double u0 = T[tat(k0, row)];
                    double u1 = T[tat(k0 + 1, row)], u2 = T[tat(k0 + 2, row)], u3 = T[tat(k0 + 3, row)];
                    u1 -= l10 * u0;
                    u2 -= l20 * u0;
                    u2 -= l21 * u1;
                    u3 -= l30 * u0;
                    u3 -= l31 * u1;
                    u3 -= l32 * u2;
                    T[tat(k0 + 1, row)] = u1;
                    T[tat(k0 + 2, row)] = u2;
                    T[tat(k0 + 3, row)] = u3;
                }
                lds_handover();
                // 3. trailing update on the tiles that meet rows and columns >= kt
                const int t0 = kt / 16;
                double af[NT], bf[NT];
#pragma unroll
                for (int q = 0; q < NT; ++q)
                    if (q >= t0) {
                        const int rc = 16 * q + c16;
                        af[q] = rc >= kt ? -T[tat(rc, k0 + g)] : 0.0;  // A(rc, g) = L(rc, k0 + g)
                        bf[q] = rc >= kt ? T[tat(k0 + g, rc)] : 0.0;   // B(g, rc) = U(k0 + g, rc)
                    }
#pragma unroll
                for (int i = 0; i < NT; ++i)
#pragma unroll
                    for (int j = 0; j < NT; ++j) {
                        if (i < t0 || j < t0) continue;
                        v4d acc;
#pragma unroll
                        for (int r = 0; r < 4; ++r) acc[r] = T[tat(16 * i + 4 * r + g, 16 * j + c16)];
                        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc, 0, 0, 0);
#pragma unroll
                        for (int r = 0; r < 4; ++r) T[tat(16 * i + 4 * r + g, 16 * j + c16)] = acc[r];
                    }
                lds_handover();
            }
            return __any(bad);
        }
    }

    // b <- (LU)^-1 b with b held in registers by virtual index.  Columns are
    // swept in elimination order (front slots, then the tail in slot 0);
    // each column's value is broadcast from its lane with readlane.  For the
    // front columns, the LU offsets of 8 columns come with one 16-byte load
    // per slot, one block ahead; the dense tail block is addressed directly
    // (column-major, lane = row).  Every block loop is unrolled (a slot has
    // at most eight blocks of eight columns), so each column's lane is a
    // compile-time constant: the broadcasts read a fixed lane, the lane
    // predicates compare with constants and the tail addresses are fixed
    // offsets.
    __device__ __forceinline__ void solve(double (&b)[NS])
    {
        KParams &p = params_here();
        const int NVB = p.NV / 8;
        const uint4 *fw = reinterpret_cast<const uint4 *>(p.fwd_map);
        const uint4 *bw = reinterpret_cast<const uint4 *>(p.bwd_map);
        const double *T = lu + p.tail_base;
        const uint32_t lub = lds_base(lu);
        const int lane = lane_here();
        const int trow = M > 0 && lane < M ? lane : 0;  // this lane's tail row
#pragma unroll
        for (int t = 0; t < NS; ++t) {
            const int ks = M > 0 ? (t + 1) % NS : t;
            if (M > 0 && ks == 0) {
                // tail columns: only tail rows (slot 0) lie below them.  A
                // block's eight entries are loaded together ahead of the
                // dependent chain of broadcasts (the scheduling barrier keeps
                // the compiler from sinking each load to its use, which put a
                // local-memory round trip into every column).
#pragma unroll
                for (int k8 = 0; k8 < M; k8 += 8) {
                    double tv[8];
#pragma unroll
                    for (int i = 0; i < 8; ++i) tv[i] = T[tat(trow, k8 + i)];
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int i = 0; i < 8; ++i) {
                        const int k = k8 + i;
                        const double xk = lane_bcast(b[0], k);
                        if (lane > k && lane < M) b[0] -= tv[i] * xk;
                    }
                }
                continue;
            }
            const int ncol = p.slot_cols[ks];
            const int b0 = ks * 8, b1 = ks * 8 + (ncol + 7) / 8;
            if (b0 >= b1) continue;
            uint4 nxt[NS];
#pragma unroll
            for (int s = 0; s < NS; ++s)
                if (ord(s) >= ord(ks)) nxt[s] = fw[(size_t)(s * kWave + lane) * NVB + b0];
#pragma unroll
            for (int bb = 0; bb < 8; ++bb) {
                const int blk = b0 + bb;
                if (blk >= b1) break;
                double v[NS][8];
#pragma unroll
                for (int s = 0; s < NS; ++s)
                    if (ord(s) >= ord(ks)) {
                        const uint4 o = nxt[s];
                        const uint32_t w[4] = {o.x, o.y, o.z, o.w};
                        lds_fields8(w, lub, v[s]);
                    }
                if (blk + 1 < b1)
#pragma unroll
                    for (int s = 0; s < NS; ++s)
                        if (ord(s) >= ord(ks)) nxt[s] = fw[(size_t)(s * kWave + lane) * NVB + blk + 1];
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int kl = (blk - b0) * 8 + i;
                    if (kl >= ncol) break;
                    const double xk = lane_bcast(b[ks], kl);
#pragma unroll
                    for (int s = 0; s < NS; ++s)
                        if (ord(s) >= ord(ks)) b[s] -= v[s][i] * xk;
                }
            }
        }
#pragma unroll
        for (int t = NS - 1; t >= 0; --t) {
            const int ks = M > 0 ? (t + 1) % NS : t;
            if (M > 0 && ks == 0) {
                // tail columns (slot 0, blocks 0 .. M/8 - 1): the tail rows
                // above (dense, addressed directly) and the front rows (slots
                // 1.., their U entries from the map)
                uint4 nxt[NS];
#pragma unroll
                for (int s = 1; s < NS; ++s) nxt[s] = bw[(size_t)(s * kWave + lane) * NVB + M / 8 - 1];
#pragma unroll
                for (int blk = M / 8 - 1; blk >= 0; --blk) {
                    double v[NS][8];
#pragma unroll
                    for (int s = 1; s < NS; ++s) {
                        const uint4 o = nxt[s];
                        const uint32_t w[4] = {o.x, o.y, o.z, o.w};
                        lds_fields8(w, lub, v[s]);
                    }
                    if (blk > 0)
#pragma unroll
                        for (int s = 1; s < NS; ++s) nxt[s] = bw[(size_t)(s * kWave + lane) * NVB + blk - 1];
                    double tv[8];  // 1/U_kk on the diagonal, U above it; loaded ahead as above
#pragma unroll
                    for (int i = 0; i < 8; ++i) tv[i] = T[tat(trow, blk * 8 + i)];
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int i = 7; i >= 0; --i) {
                        const int kl = blk * 8 + i;
                        const double xk = lane_bcast(b[0] * tv[i], kl);
                        b[0] = lane == kl ? xk : (lane < kl ? b[0] - tv[i] * xk : b[0]);
#pragma unroll
                        for (int s = 1; s < NS; ++s) b[s] -= v[s][i] * xk;
                    }
                }
                continue;
            }
            const int ncol = p.slot_cols[ks];
            const int b0 = ks * 8, b1 = ks * 8 + (ncol + 7) / 8;
            if (b0 >= b1) continue;
            uint4 nxt[NS];
#pragma unroll
            for (int s = 0; s < NS; ++s)
                if (ord(s) <= ord(ks)) nxt[s] = bw[(size_t)(s * kWave + lane) * NVB + b1 - 1];
#pragma unroll
            for (int bb = 7; bb >= 0; --bb) {
                const int blk = b0 + bb;
                if (blk >= b1) continue;
                double v[NS][8];
#pragma unroll
                for (int s = 0; s < NS; ++s)
                    if (ord(s) <= ord(ks)) {
                        const uint4 o = nxt[s];
                        const uint32_t w[4] = {o.x, o.y, o.z, o.w};
                        lds_fields8(w, lub, v[s]);
                    }
                if (blk - 1 >= b0)
#pragma unroll
                    for (int s = 0; s < NS; ++s)
                        if (ord(s) <= ord(ks)) nxt[s] = bw[(size_t)(s * kWave + lane) * NVB + blk - 1];
#pragma unroll
                for (int i = 7; i >= 0; --i) {
                    const int kl = (blk - b0) * 8 + i;
                    if (kl >= ncol) continue;
                    // lane kl holds 1/U_kk in v[ks][i]
                    const double xk = lane_bcast(b[ks] * v[ks][i], kl);
#pragma unroll
                    for (int s = 0; s < NS; ++s)
                        if (ord(s) <= ord(ks)) {
                            const double nb = b[s] - v[s][i] * xk;
                            b[s] = (s == ks && lane == kl) ? xk : nb;
                        }
                }
            }
        }
    }

    // sum over this cell of (v_i w_i)^2, the same on every lane
    __device__ __forceinline__ double ssq(const double (&v)[NS], const double (&w)[NS]) const
    {
        double acc = 0.0;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const double t = v[s] * w[s];
            acc += t * t;
        }
        return wave_sum(acc);
    }

    __device__ __forceinline__ double wrms(const double (&v)[NS], const double (&w)[NS]) const
    {
        return sqrt(ssq(v, w) / N);
    }

    __device__ __forceinline__ bool any_nonfinite(const double (&v)[NS]) const
    {
        int bad = 0;
#pragma unroll
        for (int s = 0; s < NS; ++s) bad |= valid(s) && !isfinite(v[s]);
        return __any(bad);
    }
};

// Re-sample the backward differences D[0..order] from spacing h to rho*h:
//   D'_i = sum_j T_ij D_j,  T_ij = sum_l R_jl U_li,
//   R_jl = prod_{m=1..j} (m - 1 - rho l) / m,  U_li = prod_{m=1..l} (m - 1 - i) / m
// (the interpolating polynomial's values at the new spacing, R, turned back
// into differences by U = R(1), an involution).  Lane (i, j) of the first 36
// lanes computes T_ij into LDS; every lane then applies T to its entries
// with broadcast reads.
//
// T_ij without a division per factor: U_li = (-1)^l C(i, l) (the product
// has the factor 0 once l > i), and R_jl = P_jl / j! with P_jl the product
// of the j numerators, so T_ij = (sum_{l <= order} P_jl (-1)^l C(i, l)) / j!.
__device__ __forceinline__ double rescale_entry(int i, int j, int order, double rho)
{
    double acc = 0.0, u = 1.0;  // u = (-1)^l C(i, l)
    for (int l = 0; l <= order; ++l) {
        // (-1)^l C(i, l) = (-1)^(l-1) C(i, l - 1) (l - 1 - i) / l, an integer of
        // magnitude at most 10: the rounded product with the reciprocal
        // estimate of l is exact
        if (l > 0) u = rint(u * (l - 1 - i) * __builtin_amdgcn_rcp((double)l));
        const double x = rho * l;
        double num = 1.0;
#pragma unroll
        for (int m = 1; m <= kMaxOrder; ++m) num = m <= j ? num * ((m - 1) - x) : num;
        acc = fma(num, u, acc);
    }
    int fact = 1;
#pragma unroll
    for (int m = 2; m <= kMaxOrder; ++m) fact = m <= j ? fact * m : fact;
    return acc / fact;
}

template <int NS>
__device__ __forceinline__ void rescale(double (&D)[kMaxOrder + 3][NS], int order, double rho, double *tm)
{
    constexpr int M6 = kMaxOrder + 1;
    const int lane = (int)threadIdx.x;
    lds_handover();
    if (lane < M6 * M6) tm[lane] = rescale_entry(lane / M6, lane % M6, order, rho);
    lds_handover();
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        double out[M6];
#pragma unroll
        for (int i = 0; i < M6; ++i) {
            double acc = 0.0;
#pragma unroll
            for (int j = 0; j < M6; ++j)
                if (j <= order) acc += tm[i * M6 + j] * D[j][s];
            out[i] = acc;
        }
#pragma unroll
        for (int i = 0; i < M6; ++i)
            D[i][s] = i <= order ? out[i] : D[i][s];
    }
}

// The transpose of rescale (reverse mode): L_j = sum_{i <= order} T_ij L'_i.
template <int NS>
__device__ __forceinline__ void rescale_transposed(double (&L)[kMaxOrder + 3][NS], int order, double rho, double *tm)
{
    constexpr int M6 = kMaxOrder + 1;
    const int lane = (int)threadIdx.x;
    lds_handover();
    if (lane < M6 * M6) tm[lane] = rescale_entry(lane / M6, lane % M6, order, rho);
    lds_handover();
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        double out[M6];
#pragma unroll
        for (int j = 0; j < M6; ++j) {
            double acc = 0.0;
#pragma unroll
            for (int i = 0; i < M6; ++i)
                if (i <= order) acc += tm[i * M6 + j] * L[i][s];
            out[j] = acc;
        }
#pragma unroll
        for (int j = 0; j < M6; ++j)
            L[j][s] = j <= order ? out[j] : L[j][s];
    }
}

// Multi-cells: sums over all cells of the launch (one workgroup per cell,
// all co-resident: a cooperative launch).  Every wavefront publishes its
// value in a slot of its own, waits at the grid barrier, then adds all slots
// in one fixed order, so every wavefront obtains the same bits and takes the
// same decisions.  Two slot arrays alternate: the barrier of reduction r + 1
// separates reading r from writing r + 2.  Slots are read and written with
// device-scope atomics, coherent across the XCDs' separate L2 caches.
struct GridSum {
    double *slots;  // [2][n]
    int n, r;

    __device__ __forceinline__ double sum(double v)  // v: the same on every lane
    {
        double *b = slots + (size_t)(r & 1) * n;
        if (threadIdx.x == 0) __hip_atomic_store(&b[blockIdx.x], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        cooperative_groups::this_grid().sync();
        double acc = 0.0;
        for (int i = (int)threadIdx.x; i < n; i += kWave) acc += __hip_atomic_load(&b[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ++r;
        return wave_sum(acc);
    }
};

// Wavefronts per SIMD the solver, reverse-mode and replay kernels are
// compiled for: two for one or two register slots (up to 128 species) with a
// dense tail of at most 48 rows, where the second wavefront hides more
// latency than the few registers it spills cost (measured: 387 -> 295 ms for
// 10,000 cells of 72 species); one for the larger shapes, whose registers
// would spill heavily.
template <int NS, int M>
constexpr int kSolveWaves = (NS <= 2 && M <= 48) ? 2 : 1;

// The reverse-mode kernel holds the multipliers of the backward differences
// and the per-reaction gradient in registers besides the solver's own state.
// For one or two slots and a tail of at most 48 rows it fits two wavefronts
// per SIMD without spilling (232 vector registers for 72 species), and is
// compiled so; one wavefront for the larger shapes.  An earlier build that
// spilled at two wavefronts returned wrong d L / d ln k with the 32-row tail
// (the multipliers stayed right; cause not identified), so setting up the
// kernels refuses a two-wavefront build that uses scratch memory.
template <int NS, int M>
constexpr int kAdjointWaves = (NS <= 2 && M <= 48) ? 2 : 1;

// MC: Multi-cells (one system over all cells); TAPE: record the step tape;
// W: wavefronts per SIMD the registers are budgeted for.
template <int NS, int M, bool MC, bool TAPE = false, int W = kSolveWaves<NS, M>>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(W))) void bdf_kernel(SolveParams p)
{
    extern __shared__ double smem[];
    if ((int64_t)blockIdx.x >= p.n_cells) return;
    const int64_t cell = p.order ? p.order[blockIdx.x] : blockIdx.x;  // the batch's cell schedule
    // per-launch form: where this cell's state lives between launches
    const int K = p.opts.steps_per_launch;
    double *st_d = K > 0 ? p.state + cell * p.state_stride : nullptr;
    double *st_s = K > 0 ? st_d + (kMaxOrder + 3) * NS * kWave : nullptr;
    bool resumed = false;
    if (K > 0 && st_s[0] == (double)p.call_id) {
        if (st_s[1] == 2.0) return;  // finished in an earlier launch of this outer step
        resumed = true;
    }
    Cell<NS, M> C(p, smem);
    const int lane = C.lane, N = p.N;
    // norms and failure flags: of this cell, or (Multi-cells) of the whole system
    GridSum grid{p.mc_slots, (int)p.n_cells, 0};
    const double n_all = MC ? (double)N * (double)p.n_cells : (double)N;
    auto norm = [&](const double (&v)[NS], const double (&w)[NS]) -> double {
        const double q = C.ssq(v, w);
        return sqrt((MC ? grid.sum(q) : q) / n_all);
    };
    auto any_cell = [&](bool b) -> bool { return MC ? grid.sum(b ? 1.0 : 0.0) > 0.0 : b; };
    const mcc_solver_opts &o = p.opts;
    const double dt = p.dt;
    const int maxord = o.max_order < 1 ? 1 : (o.max_order > kMaxOrder ? kMaxOrder : o.max_order);

    for (int j = lane; j < p.R; j += kWave) C.kv[j] = p.k[(int64_t)j * p.ld + cell];
    if (lane == 0) C.yv[p.N] = 1.0;
    if (lane == 0) {
        C.lu[p.lu_nnz] = 0.0;
        C.lu[p.lu_nnz + 1] = 0.0;
    }
    int sp[NS];
    double D[kMaxOrder + 3][NS], f[NS], w[NS], ypred[NS], psi[NS], d[NS], tmp[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        sp[s] = C.valid(s) ? p.vspecies[s * kWave + lane] : 0;
        const double y0 = C.valid(s) && !resumed ? p.y[(int64_t)sp[s] * p.ld + cell] : 0.0;
#pragma unroll
        for (int j = 0; j < kMaxOrder + 3; ++j) D[j][s] = resumed ? st_d[(j * NS + s) * kWave + lane] : 0.0;
        if (!resumed) D[0][s] = y0;
    }
    // counters (uniform)
    int steps = 0, rejects = 0, newton_fails = 0, newton_iters = 0, f_evals = 0, jac_evals = 0, lu_count = 0;
    int status = MCC_CELL_OK;
    double h = 0.0, t = 0.0;
    double h_uncut = 0.0, h_next = 0.0;  // the step size before the landing cut, and the one to take next
    int order = 1, n_equal = 0, attempts = 0;
    bool bad = false;
    // step tape (reverse mode): start, re-samplings and accepted steps with
    // their states, in time order; tpos = doubles written, -1 once one did not fit
    double *tp = TAPE && !MC ? p.tape + cell * p.tape_stride : nullptr;
    int64_t tpos = TAPE && resumed ? (int64_t)st_s[15] : 0;
    auto record = [&](int type, int ord, double x, bool with_state) {
        if (!TAPE || tpos < 0) return;
        if (tpos + kTapeScalars + (with_state ? N : 0) > p.tape_stride) {
            tpos = -1;
            return;
        }
        if (lane == 0) tp[tpos] = type;
        tpos += 1;
        if (with_state) {
#pragma unroll
            for (int s = 0; s < NS; ++s)
                if (C.valid(s)) tp[tpos + sp[s]] = D[0][s];
            tpos += N;
        }
        if (lane == 0) {
            tp[tpos] = ord;
            tp[tpos + 1] = x;
            tp[tpos + 2] = type;
        }
        tpos += 3;
    };
    if (resumed) {
        t = st_s[2];
        h = st_s[3];
        order = (int)st_s[4];
        n_equal = (int)st_s[5];
        attempts = (int)st_s[6];
        steps = (int)st_s[7];
        rejects = (int)st_s[8];
        newton_fails = (int)st_s[9];
        newton_iters = (int)st_s[10];
        f_evals = (int)st_s[11];
        jac_evals = (int)st_s[12];
        lu_count = (int)st_s[13];
        status = (int)st_s[14];
    } else {
        // ---- starting step size -------------------------------------------------
        // warm start: the step size the cell's previous outer step would have taken next
        const double h_warm = !MC && o.warm_start ? p.stats[cell].h_next : 0.0;
        C.deriv(D[0], f);
        f_evals++;
        bad = any_cell(C.any_nonfinite(D[0]) || C.any_nonfinite(f));
        if (bad) {
            status = MCC_CELL_NONFINITE;
            order = 0;
        } else if (h_warm > 0.0 && isfinite(h_warm)) {
            h = fmin(h_warm, dt);
        } else {
#pragma unroll
            for (int s = 0; s < NS; ++s) w[s] = C.valid(s) ? 1.0 / (o.rtol * fabs(D[0][s]) + o.atol) : 0.0;
            const double d0 = norm(D[0], w), d1 = norm(f, w);
            const double h0 = (d0 < 1e-5 || d1 < 1e-5) ? 1e-6 * dt : 0.01 * d0 / d1;
#pragma unroll
            for (int s = 0; s < NS; ++s) ypred[s] = D[0][s] + h0 * f[s];
            C.deriv(ypred, tmp);
            f_evals++;
#pragma unroll
            for (int s = 0; s < NS; ++s) tmp[s] -= f[s];
            const double d2 = norm(tmp, w) / h0;
            const double dm = d1 > d2 ? d1 : d2;
            const double h1 = dm <= 1e-15 ? fmax(1e-6, 1e-3 * h0) : sqrt(0.01 / dm);
            h = fmin(100.0 * h0, fmin(h1, dt));
            if (!(h > 0.0) || !isfinite(h)) {
                status = MCC_CELL_NONFINITE;
                order = 0;
                h = 0.0;
                bad = true;
            }
        }

        if (!bad) {
#pragma unroll
            for (int s = 0; s < NS; ++s) D[1][s] = h * f[s];
            record(0, 0, h, false);
        }
    }

    bool suspended = false;
    if (!bad) {
        int steps_here = 0;
        bool done = false;
        while (!done && t < dt) {
            if (K > 0 && steps_here >= K) {  // per-launch form: the rest in a later launch
                suspended = true;
                break;
            }
            bool accepted = false, landing = false;
            double err_norm = 0.0;
            while (!accepted) {
                if (attempts >= o.max_steps) {
                    status = MCC_CELL_TOO_MUCH_WORK;
                    done = true;
                    break;
                }
                attempts++;
                landing = false;
                if (h >= dt - t) {
                    h_uncut = h;
                    const double hn = dt - t, rho = hn / h;
                    rescale<NS>(D, order, rho, C.tm);
                    record(1, order, rho, false);
                    h = hn;
                    n_equal = 0;
                    landing = true;
                }
                const double gk = bdf_gamma(order);
                const double c = h / gk;
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    double yp = 0.0, ps = 0.0;
#pragma unroll
                    for (int j = 0; j <= kMaxOrder; ++j)
                        yp += j <= order ? D[j][s] : 0.0;
#pragma unroll
                    for (int j = 1; j <= kMaxOrder; ++j)
                        ps += j <= order ? bdf_gamma(j) * D[j][s] : 0.0;
                    ypred[s] = yp;
                    psi[s] = ps / gk;
                    w[s] = C.valid(s) ? 1.0 / (o.rtol * fabs(D[0][s]) + o.atol) : 0.0;
                    d[s] = 0.0;
                }
                C.newton_matrix(ypred, c);
                jac_evals++;
                lu_count++;
                const bool singular = any_cell(C.factor());
                bool converged = false;
                if (!singular) {
                    double nrm_old = 0.0;
                    for (int it = 0; it < o.max_newton; ++it) {
#pragma unroll
                        for (int s = 0; s < NS; ++s) tmp[s] = ypred[s] + d[s];
                        C.deriv(tmp, f);
                        f_evals++;
                        if (any_cell(C.any_nonfinite(f))) break;
#pragma unroll
                        for (int s = 0; s < NS; ++s) tmp[s] = c * f[s] - psi[s] - d[s];
                        C.solve(tmp);
                        newton_iters++;
                        const double nrm = norm(tmp, w);
                        if (!isfinite(nrm)) break;
                        double rho = 0.0;
                        if (it >= 1) {
                            rho = nrm / nrm_old;
                            if (rho >= 1.0) break;
                        }
#pragma unroll
                        for (int s = 0; s < NS; ++s) d[s] += tmp[s];
                        if (nrm == 0.0 || (it >= 1 && rho / (1.0 - rho) * nrm < o.eta_newton)) {
                            converged = true;
                            break;
                        }
                        nrm_old = nrm;
                    }
                }
                if (!converged) {
                    newton_fails++;
                    rescale<NS>(D, order, o.fac_newton_fail, C.tm);
                    record(1, order, o.fac_newton_fail, false);
                    h *= o.fac_newton_fail;
                    n_equal = 0;
                    if (h < o.h_min_rel * dt || t + h == t) {
                        status = singular ? MCC_CELL_SINGULAR : MCC_CELL_CONV_FAIL;
                        done = true;
                        break;
                    }
                    continue;
                }
                err_norm = norm(d, w) / (order + 1);
                if (err_norm > 1.0) {
                    rejects++;
                    double fac = o.safety * step_pow(err_norm, -1.0 / (order + 1));
                    if (fac < o.fac_min) fac = o.fac_min;
                    rescale<NS>(D, order, fac, C.tm);
                    record(1, order, fac, false);
                    h *= fac;
                    n_equal = 0;
                    if (h < o.h_min_rel * dt || t + h == t) {
                        status = MCC_CELL_ERR_FAIL;
                        done = true;
                        break;
                    }
                    continue;
                }
                accepted = true;
            }
            if (done) break;
            t = landing ? dt : t + h;
            if (t >= dt) h_next = landing ? h_uncut : h;
            steps++;
            steps_here++;
#pragma unroll
            for (int s = 0; s < NS; ++s) {
#pragma unroll
                for (int j = 3; j < kMaxOrder + 3; ++j)
                    D[j][s] = j == order + 2 ? d[s] - D[j - 1][s] : D[j][s];
#pragma unroll
                for (int j = 2; j < kMaxOrder + 2; ++j)
                    D[j][s] = j == order + 1 ? d[s] : D[j][s];
#pragma unroll
                for (int j = kMaxOrder; j >= 0; --j)
                    D[j][s] = j <= order ? D[j][s] + D[j + 1][s] : D[j][s];
            }
            record(2, order, h / bdf_gamma(order), true);  // the step's state z = the new D_0
            n_equal++;
            if (t >= dt) break;
            if (n_equal < order + 1) continue;
            const double e_cur = err_norm;
            double e_low = INFINITY, e_high = INFINITY;
            if (order > 1) {
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    double v = 0.0;
#pragma unroll
                    for (int j = 1; j <= kMaxOrder; ++j)
                        v += j == order ? D[j][s] : 0.0;
                    tmp[s] = v;
                }
                e_low = norm(tmp, w) / order;
            }
            if (order < maxord) {
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    double v = 0.0;
#pragma unroll
                    for (int j = 3; j < kMaxOrder + 3; ++j)
                        v += j == order + 2 ? D[j][s] : 0.0;
                    tmp[s] = v;
                }
                e_high = norm(tmp, w) / (order + 2);
            }
            const double r_cur = step_pow(e_cur, -1.0 / (order + 1));
            const double r_low = order > 1 ? step_pow(e_low, -1.0 / order) : 0.0;
            const double r_high = order < maxord ? step_pow(e_high, -1.0 / (order + 2)) : 0.0;
            int new_order = order;
            double best = r_cur;
            if (r_low > best) { best = r_low; new_order = order - 1; }
            if (r_high > best) { best = r_high; new_order = order + 1; }
            double fac = o.safety * best;
            if (fac > o.fac_max) fac = o.fac_max;
            order = new_order;
            rescale<NS>(D, order, fac, C.tm);
            record(1, order, fac, false);
            h *= fac;
            n_equal = 0;
        }
    }

    if (suspended) {
#pragma unroll
        for (int j = 0; j < kMaxOrder + 3; ++j)
#pragma unroll
            for (int s = 0; s < NS; ++s) st_d[(j * NS + s) * kWave + lane] = D[j][s];
        if (lane == 0) {
            st_s[0] = (double)p.call_id;
            st_s[1] = 1.0;
            st_s[2] = t;
            st_s[3] = h;
            st_s[4] = order;
            st_s[5] = n_equal;
            st_s[6] = attempts;
            st_s[7] = steps;
            st_s[8] = rejects;
            st_s[9] = newton_fails;
            st_s[10] = newton_iters;
            st_s[11] = f_evals;
            st_s[12] = jac_evals;
            st_s[13] = lu_count;
            st_s[14] = status;
            if (TAPE) st_s[15] = (double)tpos;
            atomicAdd(p.pending, 1);
        }
        return;
    }

    double ymin = 0.0;
    if (status != MCC_CELL_NONFINITE) {
        double lm = INFINITY;
#pragma unroll
        for (int s = 0; s < NS; ++s)
            if (C.valid(s)) {
                p.y[(int64_t)sp[s] * p.ld + cell] = D[0][s];
                lm = fmin(lm, D[0][s]);
            }
        if (status == MCC_CELL_OK) {
            ymin = wave_min(lm);
            bool fin = !any_cell(C.any_nonfinite(D[0]));
            if (!fin) status = MCC_CELL_NONFINITE;
        }
    }
    if (lane == 0) {
        p.status[cell] = status;
        if (TAPE) p.tape_len[cell] = tpos;
        if (p.stats) {
            mcc_cell_stats st;
            st.steps = steps;
            st.rejects = rejects;
            st.newton_fails = newton_fails;
            st.newton_iters = newton_iters;
            st.f_evals = f_evals;
            st.jac_evals = jac_evals;
            st.lu_count = lu_count;
            st.order = order;
            st.h_last = h;
            st.y_min = ymin;
            st.h_next = status == MCC_CELL_OK ? h_next : h;
            p.stats[cell] = st;
        }
        if (K > 0) {  // finished: later launches of this outer step skip the cell
            st_s[0] = (double)p.call_id;
            st_s[1] = 2.0;
        }
    }
}

__global__ void fill_i32_kernel(int32_t *q, int32_t v)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) q[0] = v;
}

// Reverse mode of one outer step (the discrete adjoint of its frozen step
// sequence), one wavefront per cell, with the solver tables of the
// transposed system I - c J^T.  The tape holds, per cell, entries [type,
// z (n_species, species order; accepted steps only), order, value, type];
// it is walked backwards.  For an accepted step of order k with
// c = h / gamma_k at its converged state z: the difference update is
// reversed, lam_d = lam_{k+1} + lam_{k+2}, mu = (I - c J(z))^-T lam_d (the
// transposed matrix assembled, factorised and solved by the forward code),
// then lam_ypred = c J^T mu = mu - lam_d and lam_psi = -mu go back onto the
// differences, and d L / d ln k_j gains c r_j(z) sum_i nu_ij mu_i.  A
// re-sampling of the differences is reversed with its transpose.  The start
// D_0 = y0, D_1 = h f(y0) gives dL/dy0 = lam_0 + h J(y0)^T lam_1 and
// d L / d ln k_j += h r_j(y0) sum_i nu_ij lam_1,i.
constexpr int kAdjMaxRPass = kAdjMaxR / kWave;  // reactions per lane

template <int NS, int M>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(kAdjointWaves<NS, M>))) void adjoint_kernel(
    SolveParams p, AdjointParams a)
{
    extern __shared__ double smem[];
    if ((int64_t)blockIdx.x >= p.n_cells) return;
    const int64_t cell = p.order ? p.order[blockIdx.x] : blockIdx.x;  // the batch's cell schedule
    Cell<NS, M> C(p, smem);
    double *wv = smem + a.off_w;
    const int lane = C.lane, N = p.N;
    for (int j = lane; j < p.R; j += kWave) C.kv[j] = p.k[(int64_t)j * p.ld + cell];
    if (lane == 0) C.yv[p.N] = 1.0;
    if (lane == 0) {
        C.lu[p.lu_nnz] = 0.0;
        C.lu[p.lu_nnz + 1] = 0.0;
    }
    int sp[NS];
    double L[kMaxOrder + 3][NS], z[NS], mu[NS], ld_[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        sp[s] = C.valid(s) ? p.vspecies[s * kWave + lane] : 0;
#pragma unroll
        for (int j = 0; j < kMaxOrder + 3; ++j) L[j][s] = 0.0;
        L[0][s] = C.valid(s) ? a.lam[(int64_t)sp[s] * p.ld + cell] : 0.0;
    }
    double g[kAdjMaxRPass];
#pragma unroll
    for (int u = 0; u < kAdjMaxRPass; ++u) g[u] = 0.0;
    const int32_t *nu_ptr = a.nu_ptr, *nu_vid = a.nu_vid;
    const double *nu_coef = a.nu_coef;
    // d L / d ln k_j += cc * r_j * sum_i nu_ij yv_i (rv = the rates, yv = the multiplier)
    auto add_lnk = [&](double cc) {
#pragma unroll
        for (int u = 0; u < kAdjMaxRPass; ++u) {
            const int j = u * kWave + lane;
            if (j < p.R) {
                double w = 0.0;
                for (int e = nu_ptr[j]; e < nu_ptr[j + 1]; ++e) w += nu_coef[e] * C.yv[nu_vid[e]];
                g[u] += cc * C.rv[j] * w;
            }
        }
    };
    const double *tp = a.tape + cell * a.stride;
    int64_t pos = a.len[cell];
    int status = (pos >= 0 && pos <= a.stride) ? 0 : 1;
    const bool empty = pos == 0;
    bool started = false;
    while (status == 0 && pos >= kTapeScalars) {
        const int type = (int)tp[pos - 1];
        const double x = tp[pos - 2];
        const int order = (int)tp[pos - 3];
        const int64_t n_state = type == 2 ? N : 0;
        pos -= 3;
        // the entry's leading copy of its type
        if (pos < n_state + 1 || (type != 0 && (order < 1 || order > kMaxOrder)) ||
            tp[pos - n_state - 1] != (double)type) {
            status = 1;
            break;
        }
        const double *pl = tp + pos - n_state;  // the step's state
        pos -= n_state + 1;
        if (type == 1) {  // re-sampling of the differences
            rescale_transposed<NS>(L, order, x, C.tm);
        } else if (type == 2) {  // accepted step
            const int k = order;
            const double c = x;
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                z[s] = C.valid(s) ? pl[sp[s]] : 0.0;
                // D_j += D_{j+1} (j = k..0), reversed: lam_{j+1} += lam_j (j = 0..k)
#pragma unroll
                for (int j = 0; j <= kMaxOrder; ++j)
                    if (j <= k) L[j + 1][s] += L[j][s];
                double l1 = 0.0, l2 = 0.0;
#pragma unroll
                for (int j = 0; j < kMaxOrder + 3; ++j) {
                    l1 = j == k + 1 ? L[j][s] : l1;
                    l2 = j == k + 2 ? L[j][s] : l2;
                }
                ld_[s] = l1 + l2;  // lam_d
                mu[s] = ld_[s];
#pragma unroll
                for (int j = 0; j < kMaxOrder + 3; ++j) {
                    L[j][s] = j == k + 1 ? -l2 : L[j][s];
                    L[j][s] = j == k + 2 ? 0.0 : L[j][s];
                }
            }
            C.newton_matrix(z, c);  // assembles I - c J(z)^T (transposed tables)
            if (C.factor()) {
                status = 2;
                break;
            }
            C.solve(mu);
            const double gk = bdf_gamma(k);
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const double lp = mu[s] - ld_[s];  // lam_ypred = c J^T mu
#pragma unroll
                for (int j = 0; j <= kMaxOrder; ++j) {
                    if (j <= k) L[j][s] += lp;
                    if (j >= 1 && j <= k) L[j][s] -= bdf_gamma(j) / gk * mu[s];
                }
            }
            C.rates(z);
            C.put_y(mu);
            add_lnk(c);
        } else if (type == 0) {  // start: D_0 = y0, D_1 = h f(y0)
            const double h = x;
#pragma unroll
            for (int s = 0; s < NS; ++s) z[s] = C.valid(s) ? a.y0[(int64_t)sp[s] * p.ld + cell] : 0.0;
            C.rates(z);
            C.put_y(L[1]);
            // w_j = sum_i nu_ij lam_1,i (kept in wv), d L / d ln k_j += h r_j w_j, then
            // (J^T lam_1)_s = sum over the partials taken with respect to s of partial * w_j
#pragma unroll
            for (int u = 0; u < kAdjMaxRPass; ++u) {
                const int j = u * kWave + lane;
                if (j < p.R) {
                    double w = 0.0;
                    for (int e = nu_ptr[j]; e < nu_ptr[j + 1]; ++e) w += nu_coef[e] * C.yv[nu_vid[e]];
                    g[u] += h * C.rv[j] * w;
                    wv[j] = w;
                }
            }
            C.partials(z);
            const int4 *pt = reinterpret_cast<const int4 *>(p.part);
            double jt[NS];
#pragma unroll
            for (int s = 0; s < NS; ++s) jt[s] = 0.0;
            for (int q = 0; q < p.P; ++q) {
                const int4 e = pt[q];
                const double v = C.pv[q] * wv[e.x];
#pragma unroll
                for (int s = 0; s < NS; ++s) jt[s] += e.w == s * kWave + lane ? v : 0.0;
            }
#pragma unroll
            for (int s = 0; s < NS; ++s) L[0][s] += h * jt[s];
            if (pos != 0) status = 1;  // the start must be the first entry
            started = true;
            break;
        } else {
            status = 1;
        }
    }
    if (status == 0 && !empty && !started) status = 1;  // no start entry, or a remainder shorter than an entry
#pragma unroll
    for (int s = 0; s < NS; ++s)
        if (C.valid(s)) a.lam[(int64_t)sp[s] * p.ld + cell] = status == 0 ? L[0][s] : NAN;
#pragma unroll
    for (int u = 0; u < kAdjMaxRPass; ++u) {
        const int j = u * kWave + lane;
        if (j < p.R) {
            double *o = a.glnk + (int64_t)j * p.ld + cell;
            *o = status != 0 ? NAN : (a.accumulate ? *o + g[u] : g[u]);
        }
    }
    if (lane == 0 && a.status) a.status[cell] = status == 0 ? MCC_CELL_OK : (status == 2 ? MCC_CELL_SINGULAR : MCC_CELL_BAD_TAPE);
}

// The step sequence of a tape run again from y0 with the batch's rate
// constants (the frozen-sequence map that the reverse pass differentiates):
// the start and every re-sampling as taped; every accepted step of order k
// and c = h / gamma_k solves d - c f(ypred + d) + psi = 0 by Newton with a
// fresh Newton matrix at every iterate, from the taped state, until the
// largest correction relative to its component is at most tol (or
// max_newton iterations), then updates the differences as the solver does.
template <int NS, int M>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(kSolveWaves<NS, M>))) void replay_kernel(
    SolveParams p, ReplayParams r)
{
    extern __shared__ double smem[];
    if ((int64_t)blockIdx.x >= p.n_cells) return;
    const int64_t cell = p.order ? p.order[blockIdx.x] : blockIdx.x;  // the batch's cell schedule
    Cell<NS, M> C(p, smem);
    const int lane = C.lane, N = p.N;
    for (int j = lane; j < p.R; j += kWave) C.kv[j] = p.k[(int64_t)j * p.ld + cell];
    if (lane == 0) C.yv[p.N] = 1.0;
    if (lane == 0) {
        C.lu[p.lu_nnz] = 0.0;
        C.lu[p.lu_nnz + 1] = 0.0;
    }
    int sp[NS];
    double D[kMaxOrder + 3][NS], f[NS], ypred[NS], psi[NS], d[NS], tmp[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        sp[s] = C.valid(s) ? p.vspecies[s * kWave + lane] : 0;
#pragma unroll
        for (int j = 0; j < kMaxOrder + 3; ++j) D[j][s] = 0.0;
        D[0][s] = C.valid(s) ? r.y0[(int64_t)sp[s] * p.ld + cell] : 0.0;
    }
    const double *tp = r.tape + cell * r.stride;
    const int64_t len = r.len[cell];
    int status = (len >= 0 && len <= r.stride) ? 0 : 1;  // 1: malformed tape, 2: singular matrix
    bool started = false;
    int64_t pos = 0;
    while (status == 0 && pos < len) {
        if (len - pos < kTapeScalars) {
            status = 1;
            break;
        }
        const int type = (int)tp[pos];
        const int64_t n_state = type == 2 ? N : 0;
        if (len - pos < kTapeScalars + n_state) {
            status = 1;
            break;
        }
        const double *pl = tp + pos + 1;
        const int order = (int)tp[pos + 1 + n_state];
        const double x = tp[pos + 2 + n_state];
        // the trailing copy of the type matches; the start comes first and once
        if (tp[pos + 3 + n_state] != (double)type || (type != 0 && (order < 1 || order > kMaxOrder)) ||
            (type == 0) == started || type < 0 || type > 2) {
            status = 1;
            break;
        }
        pos += kTapeScalars + n_state;
        if (type == 0) {  // D_0 = y0, D_1 = h f(y0)
            started = true;
            C.deriv(D[0], f);
#pragma unroll
            for (int s = 0; s < NS; ++s) D[1][s] = x * f[s];
        } else if (type == 1) {
            rescale<NS>(D, order, x, C.tm);
        } else {
            const int k = order;
            const double c = x, gk = bdf_gamma(k);
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                double yp = 0.0, ps = 0.0;
#pragma unroll
                for (int j = 0; j <= kMaxOrder; ++j) yp += j <= k ? D[j][s] : 0.0;
#pragma unroll
                for (int j = 1; j <= kMaxOrder; ++j) ps += j <= k ? bdf_gamma(j) * D[j][s] : 0.0;
                ypred[s] = yp;
                psi[s] = ps / gk;
                d[s] = C.valid(s) ? pl[sp[s]] - yp : 0.0;  // from the taped state
            }
            for (int it = 0; it < r.max_newton; ++it) {
#pragma unroll
                for (int s = 0; s < NS; ++s) tmp[s] = ypred[s] + d[s];
                C.deriv(tmp, f);
                C.newton_matrix(tmp, c);
                if (C.factor()) {
                    status = 2;
                    break;
                }
#pragma unroll
                for (int s = 0; s < NS; ++s) tmp[s] = c * f[s] - psi[s] - d[s];
                C.solve(tmp);
                double nr = 0.0;
#pragma unroll
                for (int s = 0; s < NS; ++s)
                    if (C.valid(s)) {
                        d[s] += tmp[s];
                        nr = fmax(nr, fabs(tmp[s]) / (fabs(ypred[s] + d[s]) + 1e-300));
                    }
                if (-wave_min(-nr) <= r.tol) break;
            }
            if (status != 0) break;
#pragma unroll
            for (int s = 0; s < NS; ++s) {
#pragma unroll
                for (int j = 3; j < kMaxOrder + 3; ++j)
                    D[j][s] = j == k + 2 ? d[s] - D[j - 1][s] : D[j][s];
#pragma unroll
                for (int j = 2; j < kMaxOrder + 2; ++j)
                    D[j][s] = j == k + 1 ? d[s] : D[j][s];
#pragma unroll
                for (int j = kMaxOrder; j >= 0; --j)
                    D[j][s] = j <= k ? D[j][s] + D[j + 1][s] : D[j][s];
            }
        }
    }
    if (status == 0 && len > 0 && !started) status = 1;
#pragma unroll
    for (int s = 0; s < NS; ++s)
        if (C.valid(s)) r.y[(int64_t)sp[s] * p.ld + cell] = status == 0 ? D[0][s] : NAN;
    if (lane == 0 && r.status)
        r.status[cell] = status == 0 ? MCC_CELL_OK : (status == 2 ? MCC_CELL_SINGULAR : MCC_CELL_BAD_TAPE);
}

}  // namespace

#define MCC_SOLVE_VARIANTS(X) \
    X(1, 0) X(2, 0) X(3, 0) X(4, 0) X(1, 32) X(2, 32) X(3, 32) X(4, 32) \
    X(1, 48) X(2, 48) X(3, 48) X(4, 48) X(1, 64) X(2, 64) X(3, 64) X(4, 64)

// The shapes built for two wavefronts per SIMD also come built for one (the
// solver autotuner times both).
#define MCC_SOLVE_ONEWAVE_VARIANTS(X) X(1, 0) X(2, 0) X(1, 32) X(2, 32) X(1, 48) X(2, 48)

// Multi-cells instantiations (small and 72-species class mechanisms).
#define MCC_MULTICELL_VARIANTS(X) X(1, 0) X(2, 0) X(2, 48)

// Reverse mode (the taping forward solver, the adjoint and the replay
// kernels), for the shapes of small, 72- and 150-species class mechanisms.
#define MCC_ADJOINT_VARIANTS(X) X(1, 0) X(2, 0) X(1, 32) X(2, 32) X(1, 48) X(2, 48) X(1, 64) X(2, 64) X(3, 64)

hipError_t prepare_solve_kernels(int max_lds_bytes)
{
    hipError_t e = hipSuccess;
#define MCC_SET_LDS(ns, m)                                                                                    \
    if (e == hipSuccess)                                                                                     \
        e = hipFuncSetAttribute((const void *)bdf_kernel<ns, m, false>, hipFuncAttributeMaxDynamicSharedMemorySize, \
                                max_lds_bytes);
    MCC_SOLVE_VARIANTS(MCC_SET_LDS)
#undef MCC_SET_LDS
#define MCC_SET_LDS_1W(ns, m)                                                                                \
    if (e == hipSuccess)                                                                                    \
        e = hipFuncSetAttribute((const void *)bdf_kernel<ns, m, false, false, 1>,                            \
                                hipFuncAttributeMaxDynamicSharedMemorySize, max_lds_bytes);
    MCC_SOLVE_ONEWAVE_VARIANTS(MCC_SET_LDS_1W)
#undef MCC_SET_LDS_1W
#define MCC_SET_LDS_MC(ns, m)                                                                                \
    if (e == hipSuccess)                                                                                    \
        e = hipFuncSetAttribute((const void *)bdf_kernel<ns, m, true>, hipFuncAttributeMaxDynamicSharedMemorySize, \
                                max_lds_bytes);
    MCC_MULTICELL_VARIANTS(MCC_SET_LDS_MC)
#undef MCC_SET_LDS_MC
#define MCC_SET_LDS_TAPE(ns, m)                                                                                     \
    if (e == hipSuccess)                                                                                           \
        e = hipFuncSetAttribute((const void *)bdf_kernel<ns, m, false, true>, hipFuncAttributeMaxDynamicSharedMemorySize, \
                                max_lds_bytes);
    MCC_ADJOINT_VARIANTS(MCC_SET_LDS_TAPE)
#undef MCC_SET_LDS_TAPE
    return e;
}

hipError_t launch_fill_i32(int32_t *q, int32_t v, hipStream_t s)
{
    hipLaunchKernelGGL(fill_i32_kernel, dim3(1), dim3(64), 0, s, q, v);
    return hipGetLastError();
}

int solve_default_waves(int NS, int M) { return (NS <= 2 && M <= 48) ? 2 : 1; }

bool solve_waves_available(int NS, int M, int waves)
{
    if (waves == solve_default_waves(NS, M)) return true;
#define MCC_1W_OK(ns, m) \
    if (waves == 1 && NS == ns && M == m) return true;
    MCC_SOLVE_ONEWAVE_VARIANTS(MCC_1W_OK)
#undef MCC_1W_OK
    return false;
}

hipError_t launch_solve(const SolveParams &p, int NS, int M, int waves, hipStream_t s)
{
    if (p.n_cells == 0) return hipSuccess;
    if (p.n_cells > 0x7fffffff) return hipErrorInvalidValue;
    const dim3 grid((unsigned)p.n_cells), block(kWave);
    const size_t lds = (size_t)p.lds_doubles * sizeof(double);
    if (p.tape) {
#define MCC_LAUNCH_TAPE(ns, m)                                                          \
    if (NS == ns && M == m) {                                                           \
        hipLaunchKernelGGL((bdf_kernel<ns, m, false, true>), grid, block, lds, s, p); \
        return hipGetLastError();                                                       \
    }
        MCC_ADJOINT_VARIANTS(MCC_LAUNCH_TAPE)
#undef MCC_LAUNCH_TAPE
        return hipErrorInvalidValue;
    }
    if (waves != solve_default_waves(NS, M)) {
#define MCC_LAUNCH_1W(ns, m)                                                                \
    if (waves == 1 && NS == ns && M == m) {                                                 \
        hipLaunchKernelGGL((bdf_kernel<ns, m, false, false, 1>), grid, block, lds, s, p); \
        return hipGetLastError();                                                           \
    }
        MCC_SOLVE_ONEWAVE_VARIANTS(MCC_LAUNCH_1W)
#undef MCC_LAUNCH_1W
        return hipErrorInvalidValue;
    }
#define MCC_LAUNCH(ns, m)                                                         \
    if (NS == ns && M == m) {                                                     \
        hipLaunchKernelGGL((bdf_kernel<ns, m, false>), grid, block, lds, s, p); \
        return hipGetLastError();                                                 \
    }
    MCC_SOLVE_VARIANTS(MCC_LAUNCH)
#undef MCC_LAUNCH
    return hipErrorInvalidValue;
}

hipError_t prepare_adjoint_kernels(int max_lds_bytes)
{
    hipError_t e = hipSuccess;
#define MCC_SET_LDS_ADJ(ns, m)                                                                           \
    if (e == hipSuccess)                                                                                \
        e = hipFuncSetAttribute((const void *)adjoint_kernel<ns, m>, hipFuncAttributeMaxDynamicSharedMemorySize, \
                                max_lds_bytes);                                                          \
    if (e == hipSuccess && kAdjointWaves<ns, m> == 2) {                                                 \
        hipFuncAttributes fa;                                                                           \
        e = hipFuncGetAttributes(&fa, (const void *)adjoint_kernel<ns, m>);                             \
        if (e == hipSuccess && fa.localSizeBytes > 0) e = hipErrorInvalidDeviceFunction;                \
    }
    MCC_ADJOINT_VARIANTS(MCC_SET_LDS_ADJ)
#undef MCC_SET_LDS_ADJ
#define MCC_SET_LDS_REPLAY(ns, m)                                                                       \
    if (e == hipSuccess)                                                                               \
        e = hipFuncSetAttribute((const void *)replay_kernel<ns, m>, hipFuncAttributeMaxDynamicSharedMemorySize, \
                                max_lds_bytes);
    MCC_ADJOINT_VARIANTS(MCC_SET_LDS_REPLAY)
#undef MCC_SET_LDS_REPLAY
    return e;
}

hipError_t launch_replay(const SolveParams &p, const ReplayParams &r, int NS, int M, hipStream_t s)
{
    if (p.n_cells == 0) return hipSuccess;
    if (p.n_cells > 0x7fffffff) return hipErrorInvalidValue;
    const dim3 grid((unsigned)p.n_cells), block(kWave);
    const size_t lds = (size_t)p.lds_doubles * sizeof(double);
#define MCC_LAUNCH_REPLAY(ns, m)                                              \
    if (NS == ns && M == m) {                                                 \
        hipLaunchKernelGGL((replay_kernel<ns, m>), grid, block, lds, s, p, r); \
        return hipGetLastError();                                             \
    }
    MCC_ADJOINT_VARIANTS(MCC_LAUNCH_REPLAY)
#undef MCC_LAUNCH_REPLAY
    return hipErrorInvalidValue;
}

bool adjoint_shape_supported(int NS, int M)
{
#define MCC_ADJ_OK(ns, m) \
    if (NS == ns && M == m) return true;
    MCC_ADJOINT_VARIANTS(MCC_ADJ_OK)
#undef MCC_ADJ_OK
    return false;
}

hipError_t launch_adjoint(const SolveParams &p, const AdjointParams &a, int NS, int M, hipStream_t s)
{
    if (p.n_cells == 0) return hipSuccess;
    if (p.n_cells > 0x7fffffff) return hipErrorInvalidValue;
    const dim3 grid((unsigned)p.n_cells), block(kWave);
    const size_t lds = (size_t)p.lds_doubles * sizeof(double);
#define MCC_LAUNCH_ADJ(ns, m)                                                 \
    if (NS == ns && M == m) {                                                 \
        hipLaunchKernelGGL((adjoint_kernel<ns, m>), grid, block, lds, s, p, a); \
        return hipGetLastError();                                             \
    }
    MCC_ADJOINT_VARIANTS(MCC_LAUNCH_ADJ)
#undef MCC_LAUNCH_ADJ
    return hipErrorInvalidValue;
}

hipError_t multicell_capacity(int NS, int M, size_t lds_bytes, int device, int64_t *max_cells)
{
    *max_cells = 0;
    const void *fn = nullptr;
#define MCC_FN(ns, m) \
    if (NS == ns && M == m) fn = (const void *)bdf_kernel<ns, m, true>;
    MCC_MULTICELL_VARIANTS(MCC_FN)
#undef MCC_FN
    if (!fn) return hipSuccess;  // no Multi-cells kernel for this solver shape
    int per_cu = 0, n_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kWave, lds_bytes);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device);
    if (e == hipSuccess) *max_cells = (int64_t)per_cu * n_cu;
    return e;
}

// Multi-cells reduction slots, [2][kMcScratchCells] doubles, for the entry
// point that allocates nothing (mcc_solve_step_multicell_noalloc).  Every
// device the library runs on holds its own copy (256 KiB) until the process
// ends.  Host code never passes the array's name to a kernel (on the host it
// is only a stand-in for the symbol); it passes the device address that
// hipGetSymbolAddress returned for the current device.
static __device__ __align__(256) double scratch[2 * kMcScratchCells];

hipError_t multicell_scratch(int device, double **ptr)
{
    static std::mutex mu;
    static std::map<int, double *> addr;  // device -> address of that device's copy
    std::lock_guard<std::mutex> lock(mu);
    auto it = addr.find(device);
    if (it != addr.end()) {
        *ptr = it->second;
        return hipSuccess;
    }
    void *q = nullptr;
    const hipError_t e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));  // the caller made `device` current
    if (e != hipSuccess) return e;
    addr[device] = static_cast<double *>(q);
    *ptr = static_cast<double *>(q);
    return hipSuccess;
}

hipError_t launch_solve_multicell(const SolveParams &p, int NS, int M, hipStream_t s)
{
    if (p.n_cells == 0) return hipSuccess;
    const dim3 grid((unsigned)p.n_cells), block(kWave);
    const size_t lds = (size_t)p.lds_doubles * sizeof(double);
    SolveParams q = p;
    void *args[] = {(void *)&q};
#define MCC_LAUNCH_MC(ns, m)                                                                               \
    if (NS == ns && M == m)                                                                                \
        return hipLaunchCooperativeKernel((const void *)bdf_kernel<ns, m, true>, grid, block, args, lds, s);
    MCC_MULTICELL_VARIANTS(MCC_LAUNCH_MC)
#undef MCC_LAUNCH_MC
    return hipErrorInvalidValue;
}

}  // namespace mcc
