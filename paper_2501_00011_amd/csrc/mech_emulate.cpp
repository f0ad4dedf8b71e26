// Host emulation of the solver kernel's table-driven phases, for testing the
// mechanism compiler without a GPU.  It runs the same op streams with the same
// semantics as the kernel (one array per LDS region, 64 lanes, blocks of kBlk
// ops whose operands are all read before any of their writes, a barrier at
// the end of each LU level) and checks on the way that every offset is in
// range and that no op reads or writes what another op of the same LU level
// writes.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <set>
#include <string>
#include <vector>

#include "mcc_internal.hpp"

namespace mcc {

// Returns the number of violations found (bounds or same-level hazards).
int emulate_cell(const HostTables &t, const double *k, const double *y_species, double c,
                 const double *b_species, double *f_species, double *x_species)
{
    const int N = t.N, R = t.R, P = t.n_partials, NS = t.NS, NV = t.NV, M = t.M;
    const int ZERO = t.lu_nnz, TRASH = t.lu_nnz + 1;
    int bad = 0;
    std::vector<double> yv(N + 1, 0.0), rv(R + 1, 0.0), pv(P + 1, 0.0), lu(t.lu_nnz + 2, 0.0);
    auto chk = [&](long v, long n) {
        if (v < 0 || v >= n) bad++;
        return v < 0 || v >= n ? 0 : v;
    };
    {  // the compact state vector: slot s, lane l at (lanes in use of earlier slots) + l
        int base = 0;
        for (int s = 0; s < NS; ++s) {
            for (int l = 0; l < t.slot_cols[s]; ++l)
                if (t.vspecies[s * 64 + l] >= 0) yv[chk(base + l, N)] = y_species[t.vspecies[s * 64 + l]];
            base += t.slot_cols[s];
        }
    }
    yv[N] = 1.0;

    // deriv: rates then the per-slot gathers
    for (int j = 0; j < R; ++j) {
        double r = k[j] * yv[chk(t.rx_reac[4 * j], N + 1)];
        r *= yv[chk(t.rx_reac[4 * j + 1], N + 1)];
        r *= yv[chk(t.rx_reac[4 * j + 2], N + 1)];
        rv[j] = r;
    }
    for (int s = 0; s < NS; ++s)
        for (int lane = 0; lane < kWave; ++lane) {
            double acc = 0.0;
            for (int bk = 0; bk < t.fg_blocks[s]; ++bk)
                for (int i = 0; i < kBlk; ++i) {
                    const Op16 &o = t.fg_ops[(((size_t)(t.fg_base[s] + bk)) * kWave + lane) * kBlk + i];
                    acc += o.coef * rv[chk(o.meta, R + 1)];
                }
            const int v = s * kWave + lane;
            if (t.vspecies[v] >= 0) f_species[t.vspecies[v]] = acc;
        }

    // Newton matrix
    for (int q = 0; q < P; ++q) {
        double d = k[chk(t.part[4 * q], R)] * yv[chk(t.part[4 * q + 1], N + 1)];
        d *= yv[chk(t.part[4 * q + 2], N + 1)];
        pv[q] = d;
    }
    std::vector<int> written(t.lu_nnz + 2, 0);
    for (int lane = 0; lane < kWave; ++lane) {
        double acc = 0.0;
        for (int bk = 0; bk < t.nm_blocks; ++bk)
            for (int i = 0; i < kBlk; ++i) {
                const Op16 &o = t.nm_ops[((size_t)bk * kWave + lane) * kBlk + i];
                const uint32_t fl = o.flags;
                if (fl & ~(kFirst | kLast | kDiag)) bad++;
                const double x = pv[chk(o.meta & 0xffff, P + 1)];
                acc = (fl & kFirst) ? o.coef * x : acc + o.coef * x;
                if (fl & kLast) {
                    const int dst = chk(o.meta >> 16, t.lu_nnz + 2);
                    if (dst == ZERO) bad++;
                    if (dst < t.lu_nnz) written[dst]++;
                    const double m = -c * acc;
                    lu[dst] = (fl & kDiag) ? 1.0 + m : m;
                }
            }
    }
    for (int e = 0; e < t.lu_nnz; ++e)
        if (written[e] != 1) bad++;  // every LU entry is set exactly once
    lu[ZERO] = 0.0;

    // LU: blocks of all lanes, reads before writes, barrier per level
    std::vector<double> acc(kWave, 0.0);
    std::set<int> operand_reads, step_writes;  // per LU level
    for (int bk = 0; bk < t.lu_blocks; ++bk) {
        std::vector<double> res(kWave * kBlk);
        std::vector<int> dsts(kWave * kBlk), store(kWave * kBlk);
        for (int lane = 0; lane < kWave; ++lane)
            for (int i = 0; i < kBlk; ++i) {
                const uint64_t w = t.lu_ops[((size_t)bk * kWave + lane) * kBlk + i];
                const int dst = chk(w & kOffMask, t.lu_nnz + 2), l = chk((w >> 16) & kOffMask, t.lu_nnz + 2);
                const int u = chk((w >> 32) & kOffMask, t.lu_nnz + 2), g = chk((w >> 48) & kOffMask, t.lu_nnz + 2);
                if ((w >> 46) & 3 || (w >> 62) & 3) bad++;  // the u and 1/U_kk fields are bare indices
                const double a0 = (w & kLuFirst) ? lu[dst] : acc[lane];
                if (w & kLuScale) {
                    acc[lane] = a0 * lu[g];
                    operand_reads.insert(g);
                } else {
                    acc[lane] = a0 - (lu[l] * lu[g]) * lu[u];
                    operand_reads.insert(l);
                    operand_reads.insert(u);
                    operand_reads.insert(g);
                }
                double r = acc[lane];
                if ((w & kLuLast) && (w & kLuRecip)) r = 1.0 / r;
                res[lane * kBlk + i] = r;
                dsts[lane * kBlk + i] = dst;
                store[lane * kBlk + i] = (w & kLuLast) != 0;
            }
        for (int q = 0; q < kWave * kBlk; ++q)
            if (store[q]) {
                const int dst = dsts[q];
                if (dst != TRASH) {
                    if (dst == ZERO || step_writes.count(dst)) bad++;  // zero cell or written twice
                    step_writes.insert(dst);
                }
                lu[dst] = res[q];
            }
        if ((size_t)bk >= t.lu_barrier.size()) {
            bad++;
            break;
        }
        if (t.lu_barrier[bk]) {
            // an operand (l, u or 1/U_kk) written in the same level is a hazard
            for (int rd : operand_reads)
                if (rd != TRASH && rd != ZERO && step_writes.count(rd)) bad++;
            operand_reads.clear();
            step_writes.clear();
        }
    }
    if (!step_writes.empty()) bad++;  // the last level must end with a barrier

    // Schur complement onto the tail in 16 x 16 x 4 blocks, as the matrix
    // cores take them: for tile (I, J) and k-step ks, lane i + 16 kk holds
    // A(i, kk) and lane j + 16 kk holds B(kk, j); T(16 I + i, 16 J + j) -=
    // sum_kk A(i, kk) B(kk, j).  Operands must lie outside the tail block.
    if (M > 0 && t.schur_ks > 0) {
        const int nt = M / 16, KS = t.schur_ks, SK = t.schur_sk;
        if (SK < 1 || (2 * nt * SK) % 8 || t.schur_tab.size() != (size_t)((KS + SK - 1) / SK) * SK * 2 * nt * kWave)
            bad++;
        auto opnd = [&](int ks, int q, int lane) {
            const int e = ks * 2 * nt + q;
            const size_t at = ((size_t)(e / 8) * kWave + lane) * 8 + e % 8;
            const int o = at < t.schur_tab.size() ? (int)chk(t.schur_tab[at], t.lu_nnz + 1) : ZERO;
            if (o >= t.tail_base && o < t.lu_nnz) bad++;  // an operand inside the tail block
            return lu[o];
        };
        for (int I = 0; I < nt; ++I)
            for (int J = 0; J < nt; ++J)
                for (int i = 0; i < 16; ++i)
                    for (int j = 0; j < 16; ++j) {
                        double &dst = lu[t.tail_base + tail_at(M, 16 * I + i, 16 * J + j)];
                        double acc = dst;
                        for (int ks = 0; ks < KS; ++ks)
                            for (int kk = 0; kk < 4; ++kk)
                                acc -= opnd(ks, I, i + 16 * kk) * opnd(ks, nt + J, j + 16 * kk);
                        dst = acc;
                    }
    }

    // dense tail: row r of the Schur complement, pivot rows broadcast
    if (M > 0) {
        std::vector<std::vector<double>> a(M, std::vector<double>(M));
        for (int r = 0; r < M; ++r)
            for (int c = 0; c < M; ++c) a[r][c] = lu[t.tail_base + tail_at(M, r, c)];
        for (int kk = 0; kk < M; ++kk) {
            const double inv = 1.0 / a[kk][kk];
            for (int r = kk + 1; r < M; ++r) {
                const double l = a[r][kk] * inv;
                a[r][kk] = l;
                for (int c = kk + 1; c < M; ++c) a[r][c] -= l * a[kk][c];
            }
            a[kk][kk] = inv;
        }
        for (int r = 0; r < M; ++r)
            for (int c = 0; c < M; ++c) lu[t.tail_base + tail_at(M, r, c)] = a[r][c];
    }

    // triangular sweeps in elimination order over virtual columns; a column
    // of slot ks updates only the slots the kernel updates (ord >= / <=)
    auto ord = [&](int s) { return M > 0 ? (s == 0 ? NS - 1 : s - 1) : s; };
    std::vector<double> bv(NV, 0.0);
    for (int v = 0; v < NV; ++v)
        if (t.vspecies[v] >= 0) bv[v] = b_species[t.vspecies[v]];
    auto map_at = [&](const std::vector<uint16_t> &m, int u, int v) {
        return (int)chk(m[(size_t)u * NV + v], t.lu_nnz + 2);
    };
    for (int pk = 0; pk < N; ++pk) {
        const int v = t.vpos[pk], ks = v / kWave;
        const double xk = bv[v];
        for (int u = 0; u < NV; ++u) {
            const int o = map_at(t.fwd_map, u, v);
            if (ord(u / kWave) >= ord(ks))
                bv[u] -= lu[o] * xk;
            else if (o != ZERO)
                bad++;  // an entry the kernel would skip
        }
    }
    for (int pk = N - 1; pk >= 0; --pk) {
        const int v = t.vpos[pk], ks = v / kWave;
        const double xk = bv[v] * lu[map_at(t.bwd_map, v, v)];
        for (int u = 0; u < NV; ++u) {
            const int o = map_at(t.bwd_map, u, v);
            if (u == v)
                bv[u] = xk;
            else if (ord(u / kWave) <= ord(ks))
                bv[u] -= lu[o] * xk;
            else if (o != ZERO)
                bad++;
        }
    }
    for (int v = 0; v < NV; ++v)
        if (t.vspecies[v] >= 0) x_species[t.vspecies[v]] = bv[v];
    return bad;
}

// Host emulation of the streaming f/J tables for one cell: every work item in
// order, chunk by chunk, monomials into a scratchpad of kFjQmax entries (plus
// the zero slot), then the output records.  Counts violations: indices or
// slots out of range, unpadded chunks, an output row written twice, added to
// before it was written, or never written, a running sum continued across
// chunks or left unwritten.
int emulate_fj(const HostTables &t, const double *k, const double *y_species, double *f, double *jac)
{
    const int N = t.N, R = t.R;
    int bad = 0;
    std::vector<int> written(N + t.nnz, 0);
    std::vector<double> out(N + t.nnz, 0.0);
    if (t.fj_items.empty() || (int)t.fj_items.size() != t.n_fitems + t.n_jitems + 1) return 1;
    for (int it = 0; it + 1 < (int)t.fj_items.size(); ++it) {
        for (int ci = t.fj_items[it]; ci < t.fj_items[it + 1]; ++ci) {
            const FjChunk &ch = t.fj_chunks[ci];
            if (ch.n_mono > kFjQmax || ch.n_mono % kFjGroup || ch.n_rec % kFjRecGroup) bad++;
            double scratch[kFjQmax + 1] = {0};
            for (int q = 0; q < ch.n_mono && q < kFjQmax; ++q) {
                const FjMono &m = t.fj_monos[ch.mono_begin + q];
                if (m.j >= R || m.j < -1) { bad++; continue; }
                double v = m.j >= 0 ? k[m.j] : 1.0;
                for (int f3 : {m.a, m.b, m.c}) {
                    if (f3 >= N || f3 < -1) { bad++; continue; }
                    if (f3 >= 0) v *= y_species[f3];
                }
                scratch[q] = v;
            }
            double acc = 0.0;
            bool open = false;
            for (int o = 0; o < ch.n_rec; ++o) {
                const FjRec &r = t.fj_recs[ch.rec_begin + o];
                const uint32_t flags = r.meta >> 24, row = r.meta & kFjRowMask;
                double s = 0.0;
                for (int q = 0; q < 3; ++q) {
                    const int slot = (r.slots >> (8 * q)) & 0xff;
                    if (slot > kFjQmax || (slot >= ch.n_mono && slot != kFjQmax)) { bad++; continue; }
                    s += r.coef[q] * scratch[slot];
                }
                if ((flags & kFjKeep) && !open) bad++;
                acc = (flags & kFjKeep) ? acc + s : s;
                open = !(flags & kFjStore);
                if (!(flags & kFjStore)) continue;
                if (row >= (uint32_t)(N + t.nnz)) { bad++; continue; }
                if (flags & kFjAdd) {
                    if (written[row] != 1) bad++;
                    out[row] += acc;
                } else {
                    if (written[row]) bad++;
                    written[row] = 1;
                    out[row] = acc;
                }
            }
            if (open && acc != 0.0) bad++;
        }
        if (it + 1 == t.n_fitems) {  // f items cover exactly the f rows
            for (int r = 0; r < N; ++r)
                if (!written[r]) bad++;
        }
    }
    for (int r = 0; r < N + t.nnz; ++r)
        if (!written[r]) bad++;
    for (int r = 0; r < N; ++r) f[r] = out[r];
    for (int e = 0; e < t.nnz; ++e) jac[e] = out[N + e];
    return bad;
}

// The generated VJP kernel's arithmetic for one cell, item by item and round
// by round as in the generated source (plan_vjp): w_j = sum_i nu_ij v_i in
// the stored order, then gy_s += w_j * (multiplicity * k_j * the other
// reactants) for the item's columns among j's reactants, and
// glnk_j = (k_j * reactants) * w_j in the item that owns j.
int emulate_vjp(const HostTables &t, const double *k, const double *y_species, const double *v, double *gy,
                double *glnk)
{
    const int N = t.N, R = t.R;
    int bad = 0;
    std::vector<int> col_seen(N, 0), rx_seen(R, 0);
    for (const VjpItem &it : t.vjp_items) {
        std::vector<double> g(it.cols.size(), 0.0);
        std::vector<int> col_slot(N, -1);
        for (size_t q = 0; q < it.cols.size(); ++q) {
            const int s = it.cols[q];
            if (s < 0 || s >= N) { bad++; continue; }
            col_seen[s]++;
            col_slot[s] = (int)q;
        }
        std::vector<char> in_item(R, 0), owned(R, 0);
        for (int j : it.glnk) {
            if (j < 0 || j >= R) { bad++; continue; }
            owned[j] = 1;
            rx_seen[j]++;
        }
        for (const std::vector<int32_t> &round : it.rounds) {
            std::vector<int> rows;
            for (int j : round) {
                if (j < 0 || j >= R) { bad++; continue; }
                rows.push_back(j);
                for (int q = 0; q < 3; ++q)
                    if (t.rx_sp[3 * j + q] >= 0) rows.push_back(R + t.rx_sp[3 * j + q]);
                for (int e = t.nu_ptr[j]; e < t.nu_ptr[j + 1]; ++e) rows.push_back(R + N + t.nu_sp[e]);
            }
            std::sort(rows.begin(), rows.end());
            const int n_rows = (int)(std::unique(rows.begin(), rows.end()) - rows.begin());
            if (n_rows > kVjpRoundLoads && round.size() > 1) bad++;
            for (int j : round) {
                if (j < 0 || j >= R) continue;
                in_item[j] = 1;
                double w = 0.0;
                for (int e = t.nu_ptr[j]; e < t.nu_ptr[j + 1]; ++e) w += t.nu_coef[e] * v[t.nu_sp[e]];
                const int *a = &t.rx_sp[3 * j];
                for (int q = 0; q < 3; ++q) {
                    const int s = a[q];
                    if (s < 0 || col_slot[s] < 0) continue;
                    bool first = true;  // each distinct reactant once
                    for (int p = 0; p < q; ++p) first = first && a[p] != s;
                    if (!first) continue;
                    int mult = 0;
                    double d = k[j];
                    bool skipped = false;
                    for (int p = 0; p < 3; ++p) {
                        if (a[p] < 0) continue;
                        if (a[p] == s) {
                            mult++;
                            if (!skipped) { skipped = true; continue; }
                        }
                        d *= y_species[a[p]];
                    }
                    g[col_slot[s]] += w * (mult > 1 ? mult * d : d);
                }
                if (owned[j]) {
                    double r = k[j];
                    for (int p = 0; p < 3; ++p)
                        if (a[p] >= 0) r *= y_species[a[p]];
                    glnk[j] = r * w;
                }
            }
        }
        // every reaction with a reactant among the columns is in the item; owned ones too
        for (int s : it.cols)
            for (int j = 0; j < R && s >= 0 && s < N; ++j)
                for (int q = 0; q < 3; ++q)
                    if (t.rx_sp[3 * j + q] == s && !in_item[j]) bad++;
        for (int j : it.glnk)
            if (j >= 0 && j < R && !in_item[j]) bad++;
        for (size_t q = 0; q < it.cols.size(); ++q)
            if (it.cols[q] >= 0 && it.cols[q] < N) gy[it.cols[q]] = g[q];
    }
    for (int s = 0; s < N; ++s)
        if (col_seen[s] != 1) bad++;
    for (int j = 0; j < R; ++j)
        if (rx_seen[j] != 1) bad++;
    return bad;
}

}  // namespace mcc
