// Mechanism compiler: validates a mass-action mechanism and builds every table
// the kernels need.  Runs once per mechanism on the host (Section 3 of the
// paper keeps reaction data in GPU memory from initialisation on; here it is
// also pre-arranged so that the kernels never search or branch on structure).
//
// Definitions (Section 2, reaction and tendency equations):
//   r_j    = k_j * prod over reactant slots l of y_{a_jl}          (mass action)
//   nu_ij  = (yield of i as product of j) - (count of i as reactant of j)
//   f_i    = sum_j nu_ij r_j
//   J_is   = sum_j nu_ij d r_j / d y_s,
//   d r_j / d y_s = sum over slots l with a_jl = s of k_j prod_{l' != l} y_{a_jl'}
// Every f value and every J entry is thus a sum of monomials
//   coef * k_j * y_a * y_b * y_c  (missing factors are the constant 1),
// which is the single form the streaming kernel evaluates.
#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <cstdlib>
#include <numeric>
#include <sstream>

#include "mcc_internal.hpp"

namespace mcc {
namespace {

constexpr int kMaxProducts = 8;

bool fail(std::string *err, const std::string &msg)
{
    *err = msg;
    return false;
}

bool validate(const mcc_mech_desc *d, std::string *err)
{
    const int N = d->n_species, R = d->n_reactions;
    if (N < 1 || N > MCC_MAX_SPECIES)
        return fail(err, "n_species must be in 1.." + std::to_string(MCC_MAX_SPECIES));
    if (R < 0 || R > 65535)
        return fail(err, "n_reactions must be in 0..65535");
    if (R > 0 && (!d->rxn_type || !d->reac_ptr || !d->reac_idx || !d->prod_ptr || !d->A || !d->theta))
        return fail(err, "null mechanism array");
    if (R > 0 && d->prod_ptr[R] > 0 && (!d->prod_idx || !d->prod_yield))
        return fail(err, "null product array");
    if (R > 0 && (d->reac_ptr[0] != 0 || d->prod_ptr[0] != 0))
        return fail(err, "reac_ptr[0] and prod_ptr[0] must be 0");
    for (int j = 0; j < R; ++j) {
        const int na = d->reac_ptr[j + 1] - d->reac_ptr[j];
        const int np = d->prod_ptr[j + 1] - d->prod_ptr[j];
        std::ostringstream at;
        at << "reaction " << j << ": ";
        if (na < 1 || na > 3) return fail(err, at.str() + "needs 1 to 3 reactant slots");
        if (np < 0 || np > kMaxProducts) return fail(err, at.str() + "needs 0 to 8 products");
        if (d->rxn_type[j] != MCC_RXN_THERMAL && d->rxn_type[j] != MCC_RXN_PHOTOLYSIS)
            return fail(err, at.str() + "unknown reaction type");
        if (!std::isfinite(d->A[j]) || d->A[j] < 0.0) return fail(err, at.str() + "A must be finite and >= 0");
        if (!std::isfinite(d->theta[j])) return fail(err, at.str() + "theta must be finite");
        for (int q = d->reac_ptr[j]; q < d->reac_ptr[j + 1]; ++q)
            if (d->reac_idx[q] < 0 || d->reac_idx[q] >= N) return fail(err, at.str() + "reactant index out of range");
        for (int q = d->prod_ptr[j]; q < d->prod_ptr[j + 1]; ++q) {
            if (d->prod_idx[q] < 0 || d->prod_idx[q] >= N) return fail(err, at.str() + "product index out of range");
            if (!std::isfinite(d->prod_yield[q])) return fail(err, at.str() + "yield must be finite");
        }
    }
    return true;
}

// Net stoichiometry of reaction j: species -> nu (products minus reactant counts).
std::map<int, double> net_stoich(const mcc_mech_desc *d, int j)
{
    std::map<int, double> nu;
    for (int q = d->reac_ptr[j]; q < d->reac_ptr[j + 1]; ++q) nu[d->reac_idx[q]] -= 1.0;
    for (int q = d->prod_ptr[j]; q < d->prod_ptr[j + 1]; ++q) nu[d->prod_idx[q]] += d->prod_yield[q];
    return nu;
}

// Greedy Markowitz ordering with diagonal pivots: at every step eliminate the
// node whose (row count - 1) * (column count - 1) in the active submatrix is
// smallest (ties: smaller row + column count, then lower index).
std::vector<int32_t> markowitz_order(const std::vector<std::vector<char>> &pat)
{
    const int N = (int)pat.size();
    std::vector<std::vector<char>> a = pat;
    std::vector<char> alive(N, 1);
    std::vector<int32_t> order;
    for (int step = 0; step < N; ++step) {
        long best_score = -1, best_sum = 0;
        int best = -1;
        for (int i = 0; i < N; ++i) {
            if (!alive[i]) continue;
            long r = 0, c = 0;
            for (int j = 0; j < N; ++j)
                if (alive[j]) {
                    r += a[i][j];
                    c += a[j][i];
                }
            const long score = (r - 1) * (c - 1), sum = r + c;
            if (best < 0 || score < best_score || (score == best_score && sum < best_sum)) {
                best = i;
                best_score = score;
                best_sum = sum;
            }
        }
        order.push_back(best);
        alive[best] = 0;
        for (int i = 0; i < N; ++i) {
            if (!alive[i] || !a[i][best]) continue;
            for (int j = 0; j < N; ++j)
                if (alive[j] && a[best][j]) a[i][j] = 1;
        }
    }
    return order;
}

Op16 make_op16(double coef, uint32_t meta, uint32_t flags = 0)
{
    Op16 o;
    o.coef = coef;
    o.meta = meta;
    o.flags = flags;
    return o;
}

uint64_t lu_op(int dst, int l, int u, int dg, uint64_t flags)
{
    return (uint64_t)dst | ((uint64_t)l << 16) | ((uint64_t)u << 32) | ((uint64_t)dg << 48) | flags;
}

// Longest-first greedy assignment of op chains to the 64 lanes of a wave.
template <class T>
std::vector<std::vector<T>> pack_chains(std::vector<std::vector<T>> &chains)
{
    std::vector<int> order(chains.size());
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return chains[a].size() > chains[b].size(); });
    std::vector<std::vector<T>> lanes(kWave);
    for (int c : order) {
        int best = 0;
        for (int l = 1; l < kWave; ++l)
            if (lanes[l].size() < lanes[best].size()) best = l;
        lanes[best].insert(lanes[best].end(), chains[c].begin(), chains[c].end());
    }
    return lanes;
}

// Pads per-lane op lists to a common multiple of kBlk and appends them in the
// [block][lane][kBlk] layout the kernels prefetch.  Returns the block count.
template <class T>
int emit_blocks(std::vector<std::vector<T>> &lanes, const T &pad, std::vector<T> *out)
{
    size_t len = 0;
    for (auto &l : lanes) len = std::max(len, l.size());
    len = (len + kBlk - 1) / kBlk * kBlk;
    for (auto &l : lanes) l.resize(len, pad);
    const int nb = (int)(len / kBlk);
    for (int b = 0; b < nb; ++b)
        for (int lane = 0; lane < kWave; ++lane)
            for (int i = 0; i < kBlk; ++i) out->push_back(lanes[lane][(size_t)b * kBlk + i]);
    return nb;
}

}  // namespace

mcc_status compile_mechanism(const mcc_mech_desc *d, int dense_tail, HostTables *t, std::string *err, bool transpose)
{
    if (!validate(d, err)) return MCC_ERR_MECH;
    const int N = d->n_species, R = d->n_reactions;
    t->N = N;
    t->R = R;
    t->NS = (N + kWave - 1) / kWave;
    t->rxn_type.assign(d->rxn_type, d->rxn_type + R);
    t->A.assign(d->A, d->A + R);
    t->theta.assign(d->theta, d->theta + R);

    // ---- Jacobian pattern (species order) --------------------------------
    std::vector<std::vector<char>> pat(N, std::vector<char>(N, 0));
    for (int i = 0; i < N; ++i) pat[i][i] = 1;
    for (int j = 0; j < R; ++j) {
        const auto nu = net_stoich(d, j);
        for (int q = d->reac_ptr[j]; q < d->reac_ptr[j + 1]; ++q)
            for (const auto &kv : nu) pat[kv.first][d->reac_idx[q]] = 1;
    }
    t->row_ptr.assign(N + 1, 0);
    t->col_idx.clear();
    std::vector<std::vector<int>> jpos(N, std::vector<int>(N, -1));
    for (int i = 0; i < N; ++i) {
        for (int s = 0; s < N; ++s)
            if (pat[i][s]) {
                jpos[i][s] = (int)t->col_idx.size();
                t->col_idx.push_back(s);
            }
        t->row_ptr[i + 1] = (int32_t)t->col_idx.size();
    }
    t->nnz = (int)t->col_idx.size();

    // ---- partials: one per (reaction, reactant slot) -----------------------
    struct Partial { int j, slot, s, o1, o2; };  // o1, o2: other slots' species or N
    std::vector<Partial> parts;
    for (int j = 0; j < R; ++j) {
        const int b = d->reac_ptr[j], e = d->reac_ptr[j + 1];
        for (int l = b; l < e; ++l) {
            int others[2] = {N, N}, n = 0;
            for (int q = b; q < e; ++q)
                if (q != l) others[n++] = d->reac_idx[q];
            parts.push_back({j, l - b, d->reac_idx[l], others[0], others[1]});
        }
    }
    t->n_partials = (int)parts.size();

    // ---- reactions as written (for the VJP kernel) -------------------------
    t->rx_sp.assign(3 * (size_t)R, -1);
    t->nu_ptr.assign(1, 0);
    t->nu_sp.clear();
    t->nu_coef.clear();
    for (int j = 0; j < R; ++j) {
        for (int q = d->reac_ptr[j]; q < d->reac_ptr[j + 1]; ++q) t->rx_sp[3 * j + (q - d->reac_ptr[j])] = d->reac_idx[q];
        for (const auto &kv : net_stoich(d, j))
            if (kv.second != 0.0) {
                t->nu_sp.push_back(kv.first);
                t->nu_coef.push_back(kv.second);
            }
        t->nu_ptr.push_back((int32_t)t->nu_sp.size());
    }
    t->vjp_items = plan_vjp(*t, kVjpRoundLoads);

    // ---- the paper's Derivative kernel data (ablation only) ---------------
    t->paper_ok = true;
    t->paper_rec.assign((size_t)R * kPaperRec, 0);
    t->paper_yld.assign((size_t)R * kPaperProd, 0.0);
    for (int j = 0; j < R; ++j) {
        const int nr = d->reac_ptr[j + 1] - d->reac_ptr[j], np = d->prod_ptr[j + 1] - d->prod_ptr[j];
        if (np > kPaperProd) {
            t->paper_ok = false;
            continue;
        }
        int32_t *q = &t->paper_rec[(size_t)j * kPaperRec];
        q[0] = nr;
        for (int a = 0; a < nr; ++a) q[1 + a] = d->reac_idx[d->reac_ptr[j] + a];
        q[4] = np;
        for (int a = 0; a < np; ++a) {
            q[5 + a] = d->prod_idx[d->prod_ptr[j] + a];
            t->paper_yld[(size_t)j * kPaperProd + a] = d->prod_yield[d->prod_ptr[j] + a];
        }
    }
    t->paper_rec_inv.assign((size_t)R * kPaperRec, 0);
    t->paper_yld_inv.assign((size_t)R * kPaperProd, 0.0);
    for (int j = 0; j < R; ++j) {
        for (int p = 0; p < kPaperRec; ++p) t->paper_rec_inv[(size_t)p * R + j] = t->paper_rec[(size_t)j * kPaperRec + p];
        for (int p = 0; p < kPaperProd; ++p) t->paper_yld_inv[(size_t)p * R + j] = t->paper_yld[(size_t)j * kPaperProd + p];
    }

    // ---- streaming f/J tables (species order) ------------------------------
    // Units: an f row i (monomials = the rates of the reactions that change
    // i) and a J column s (monomials = the partials d r_j / d y_s through each
    // reactant slot holding s; outputs = every J entry of column s).  Units
    // are packed into chunks of at most kFjQmax monomials; a unit with more
    // is split, its later parts accumulating into the same outputs.
    struct Unit {
        std::vector<std::array<int32_t, 4>> monos;            // j, a, b, c (-1 = one)
        std::vector<std::pair<int, std::vector<std::pair<int, double>>>> outs;  // row, (slot, coef)
    };
    std::vector<Unit> units;
    t->out_ptr.assign(1, 0);
    std::vector<std::vector<std::pair<int, double>>> frow(N);  // species -> (reaction, nu)
    for (int j = 0; j < R; ++j)
        for (const auto &kv : net_stoich(d, j))
            if (kv.second != 0.0) frow[kv.first].push_back({j, kv.second});
    auto rate_mono = [&](int j) {
        std::array<int32_t, 4> m = {j, -1, -1, -1};
        for (int q = d->reac_ptr[j]; q < d->reac_ptr[j + 1]; ++q) m[1 + (q - d->reac_ptr[j])] = d->reac_idx[q];
        return m;
    };
    for (int i = 0; i < N; ++i) {
        Unit u;
        std::vector<std::pair<int, double>> terms;
        for (const auto &rc : frow[i]) {
            terms.push_back({(int)u.monos.size(), rc.second});
            u.monos.push_back(rate_mono(rc.first));
        }
        u.outs.push_back({i, terms});
        units.push_back(u);
        t->out_ptr.push_back(t->out_ptr.back() + (int32_t)frow[i].size());
    }
    const int n_funits = (int)units.size();
    std::vector<int32_t> jterms_of_row(t->nnz, 0);
    for (int s = 0; s < N; ++s) {
        Unit u;
        std::map<int, std::vector<std::pair<int, double>>> by_row;  // J row index -> terms
        for (int i = 0; i < N; ++i)
            if (jpos[i][s] >= 0) by_row[jpos[i][s]];
        for (const Partial &pt : parts) {
            if (pt.s != s) continue;
            const int slot = (int)u.monos.size();
            u.monos.push_back({pt.j, pt.o1 < N ? pt.o1 : -1, pt.o2 < N ? pt.o2 : -1, -1});
            for (const auto &kv : net_stoich(d, pt.j))
                if (kv.second != 0.0) {
                    by_row[jpos[kv.first][s]].push_back({slot, kv.second});
                    jterms_of_row[jpos[kv.first][s]]++;
                }
        }
        for (auto &kv : by_row) u.outs.push_back({N + kv.first, kv.second});
        units.push_back(u);
    }
    for (int e = 0; e < t->nnz; ++e) t->out_ptr.push_back(t->out_ptr.back() + jterms_of_row[e]);

    t->fj_monos.clear();
    t->fj_recs.clear();
    t->fj_chunks.clear();
    t->fj_items.clear();
    FjChunk cur{0, 0, 0, 0};
    bool cur_cont = false;  // the open chunk continues the previous work item
    auto close_chunk = [&]() {
        if (cur.n_mono > 0 || cur.n_rec > 0) {
            while (cur.n_mono % kFjGroup) {  // padding monomials: the constant 1
                t->fj_monos.push_back(FjMono{-1, -1, -1, -1});
                cur.n_mono++;
            }
            while (cur.n_rec % kFjRecGroup) {  // padding records: no effect
                FjRec r{};
                r.slots = (uint32_t)kFjQmax * 0x10101u;
                t->fj_recs.push_back(r);
                cur.n_rec++;
            }
            if (!cur_cont) t->fj_items.push_back((int32_t)t->fj_chunks.size());
            t->fj_chunks.push_back(cur);
        }
        cur = FjChunk{(int32_t)t->fj_monos.size(), 0, (int32_t)t->fj_recs.size(), 0};
        cur_cont = false;
    };
    auto add_part = [&](const Unit &u, int m0, int m1, bool accum) {
        // monomials [m0, m1) of unit u, with the terms that use them
        if (cur.n_mono + (m1 - m0) > kFjQmax) close_chunk();
        const int base = cur.n_mono;
        for (int q = m0; q < m1; ++q) {
            FjMono mo{u.monos[q][0], u.monos[q][1], u.monos[q][2], u.monos[q][3]};
            t->fj_monos.push_back(mo);
        }
        cur.n_mono += m1 - m0;
        for (const auto &o : u.outs) {
            std::vector<std::pair<int, double>> terms;
            for (const auto &tm : o.second)
                if (tm.first >= m0 && tm.first < m1) terms.push_back({base + (tm.first - m0), tm.second});
            if (accum && terms.empty()) continue;  // nothing to add
            if (terms.empty()) terms.push_back({kFjQmax, 0.0});
            for (size_t q0 = 0; q0 < terms.size(); q0 += 3) {
                FjRec r{};
                r.slots = (uint32_t)kFjQmax * 0x10101u;
                for (size_t q = q0; q < std::min(terms.size(), q0 + 3); ++q) {
                    r.coef[q - q0] = terms[q].second;
                    r.slots = (r.slots & ~(0xffu << (8 * (q - q0)))) | ((uint32_t)terms[q].first << (8 * (q - q0)));
                }
                uint32_t flags = 0;
                if (q0 > 0) flags |= kFjKeep;
                if (q0 + 3 >= terms.size()) flags |= kFjStore | (accum ? kFjAdd : 0);
                r.meta = (uint32_t)o.first | flags << 24;
                t->fj_recs.push_back(r);
                cur.n_rec++;
            }
        }
    };
    auto add_unit = [&](const Unit &u) {
        const int n = (int)u.monos.size();
        if (n == 0) {
            add_part(u, 0, 0, false);
            return;
        }
        for (int m0 = 0; m0 < n; m0 += kFjQmax) {
            const int m1 = std::min(n, m0 + kFjQmax);
            if (m0 > 0) {  // later parts: a fresh chunk of the same work item
                close_chunk();
                cur_cont = true;
            }
            add_part(u, m0, m1, m0 > 0);
        }
    };
    for (int q = 0; q < n_funits; ++q) add_unit(units[q]);
    close_chunk();
    t->n_fitems = (int)t->fj_items.size();
    for (size_t q = n_funits; q < units.size(); ++q) add_unit(units[q]);
    close_chunk();
    t->n_jitems = (int)t->fj_items.size() - t->n_fitems;
    t->fj_items.push_back((int32_t)t->fj_chunks.size());
    // one spare entry at each table's end: a lane's table read stays in
    // bounds even for a chunk without monomials at the end
    t->fj_monos.push_back(FjMono{-1, -1, -1, -1});
    {
        FjRec r{};
        r.slots = (uint32_t)kFjQmax * 0x10101u;
        t->fj_recs.push_back(r);
    }

    // ---- fill-reducing order and symbolic LU (elimination positions) -------
    // The solver's system: M = I - c J, or with transpose its transpose
    // I - c J^T (the reverse-mode step), whose pattern is the transposed one.
    std::vector<std::vector<char>> spat = pat;
    if (transpose)
        for (int i = 0; i < N; ++i)
            for (int s = 0; s < N; ++s) spat[i][s] = pat[s][i];
    t->transposed = transpose;
    t->perm = markowitz_order(spat);
    t->iperm.assign(N, 0);
    for (int p = 0; p < N; ++p) t->iperm[t->perm[p]] = p;
    std::vector<std::vector<char>> lp(N, std::vector<char>(N, 0));
    for (int i = 0; i < N; ++i)
        for (int s = 0; s < N; ++s)
            if (spat[i][s]) lp[t->iperm[i]][t->iperm[s]] = 1;
    for (int k = 0; k < N; ++k)
        for (int i = k + 1; i < N; ++i)
            if (lp[i][k])
                for (int j = k + 1; j < N; ++j)
                    if (lp[k][j]) lp[i][j] = 1;
    // algorithmic LU work, from the sparse symbolic factorisation
    t->lu_updates = 0;
    t->lu_lower = 0;
    t->lu_upper = 0;
    for (int k = 0; k < N; ++k) {
        int64_t r = 0, c = 0;
        for (int i = k + 1; i < N; ++i) r += lp[i][k];
        for (int j = k + 1; j < N; ++j) c += lp[k][j];
        t->lu_updates += r * c;
        t->lu_lower += r;
        t->lu_upper += c;
    }

    // ---- dense tail --------------------------------------------------------
    // After the ordering the trailing block of the factors is nearly dense.
    // Its last M pivots are factorised in registers (lane = row) and the
    // first F = N - M pivots by the level-scheduled sparse op streams.  M is
    // chosen from {0, 32, 48, 64} by a cost model (cycles of one wavefront:
    // ~1000 per sparse block, ~8 per dense (pivot, column) pair) with the LDS
    // the tail adds priced in; a caller's configuration overrides the choice.
    auto tail_density = [&](int m) {
        double nzc = 0;
        for (int i = N - m; i < N; ++i)
            for (int j = N - m; j < N; ++j) nzc += lp[i][j];
        return m > 0 ? nzc / ((double)m * m) : 1.0;
    };
    auto front_cost = [&](int F) {
        std::vector<int> lev(F, 1);
        int maxl = 0;
        int64_t ops = 0;
        for (int k = 0; k < F; ++k) {
            for (int q = 0; q < k; ++q)
                if (lp[k][q] || lp[q][k]) lev[k] = std::max(lev[k], lev[q] + 1);
            maxl = std::max(maxl, lev[k]);
            int64_t r = 0, c = 0;
            for (int i = k + 1; i < N; ++i) r += lp[i][k];
            for (int j = k + 1; j < N; ++j) c += lp[k][j];
            ops += r * c + r + 1;
        }
        return 1000.0 * std::max<double>(maxl + (F > 0 ? 2 : 0), (double)ops / (kWave * kBlk) * 1.5);
    };
    int M = 0;
    {
        double best = front_cost(N);
        for (int m : {32, 48, 64}) {
            if (m > N) continue;
            const double extra_lds = (1.0 - tail_density(m)) * m * m * 8.0;  // bytes
            const double cost = front_cost(N - m) + 8.0 * m * (m - 1) / 2 + 4.0 * extra_lds;
            if (cost < best) {
                best = cost;
                M = m;
            }
        }
        if (dense_tail >= 0) {  // the caller's choice (e.g. an autotuner's)
            if (!(dense_tail == 0 || dense_tail == 32 || dense_tail == 48 || dense_tail == 64) || dense_tail > N) {
                *err = "dense_tail must be -1, 0, 32, 48 or 64, and at most the number of species";
                return MCC_ERR_INVALID_ARG;
            }
            M = dense_tail;
        }
    }
    const int F = N - M;
    t->M = M;
    t->F = F;
    for (int i = F; i < N; ++i)
        for (int j = F; j < N; ++j) lp[i][j] = 1;  // the tail is stored dense

    // ---- virtual (slot, lane) index of every position ----------------------
    // With a dense tail, slot 0 lane r holds tail row r and the front
    // positions fill slots 1..; otherwise position p is slot p/64, lane p%64.
    t->NS = M > 0 ? 1 + (F + kWave - 1) / kWave : (N + kWave - 1) / kWave;
    if (t->NS > kMaxSlots) {
        *err = "too many species for the solver's register slots";
        return MCC_ERR_MECH;
    }
    t->NV = t->NS * kWave;
    std::vector<int> vpos(N);  // position -> virtual index
    for (int p = 0; p < N; ++p) vpos[p] = M > 0 ? (p >= F ? p - F : kWave + p) : p;
    t->vspecies.assign(t->NV, -1);
    for (int p = 0; p < N; ++p) t->vspecies[vpos[p]] = t->perm[p];
    t->vpos.assign(vpos.begin(), vpos.end());
    auto vid = [&](int species) { return vpos[t->iperm[species]]; };
    // The LDS copy of the state is compact: slot s keeps lanes 0..cols_s-1
    // (the lanes in use are contiguous) at ybase[s] + lane, so the N values
    // take N places and yv[N] holds the constant 1.
    std::vector<int> cols(t->NS, 0), ybase(t->NS, 0);
    for (int p = 0; p < N; ++p) cols[vpos[p] / kWave] = std::max(cols[vpos[p] / kWave], vpos[p] % kWave + 1);
    for (int s = 1; s < t->NS; ++s) ybase[s] = ybase[s - 1] + cols[s - 1];
    if (ybase[t->NS - 1] + cols[t->NS - 1] != N) {
        *err = "internal: the solver's lanes in use are not contiguous";
        return MCC_ERR_MECH;
    }
    auto yid = [&](int species) {
        const int v = vid(species);
        return ybase[v / kWave] + v % kWave;
    };
    const int ONE = N;

    // ---- LU storage: front entries row by row, then the tail column-major --
    std::vector<std::vector<int>> lpos(N, std::vector<int>(N, -1));
    int nlu = 0;
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j)
            if (lp[i][j] && !(i >= F && j >= F)) lpos[i][j] = nlu++;
    t->tail_base = nlu;
    for (int j = F; j < N; ++j)
        for (int i = F; i < N; ++i) lpos[i][j] = t->tail_base + tail_at(M, i - F, j - F);
    nlu = t->tail_base + M * M;
    t->lu_nnz = nlu;
    if (nlu + 2 >= (1 << kOffBits)) {
        *err = "LU fill exceeds the 14-bit offset range of the solver tables";
        return MCC_ERR_MECH;
    }
    const int ZERO = nlu;       // LDS cell holding 0.0
    const int TRASH = nlu + 1;  // LDS cell written by idle lanes

    // ---- solver: reactions and partials in virtual ids --------------------
    t->rx_reac.assign(4 * (size_t)R, ONE);
    for (int j = 0; j < R; ++j) {
        const int b = d->reac_ptr[j], e = d->reac_ptr[j + 1];
        for (int q = b; q < e; ++q) t->rx_reac[4 * j + (q - b)] = yid(d->reac_idx[q]);
        t->rx_reac[4 * j + 3] = 0;
    }
    t->part.assign(4 * parts.size(), 0);
    for (size_t q = 0; q < parts.size(); ++q) {
        t->part[4 * q + 0] = parts[q].j;
        t->part[4 * q + 1] = parts[q].o1 < N ? yid(parts[q].o1) : ONE;
        t->part[4 * q + 2] = parts[q].o2 < N ? yid(parts[q].o2) : ONE;
        t->part[4 * q + 3] = vid(parts[q].s);  // the species the partial is taken with respect to (virtual index)
    }
    t->nu_vid.resize(t->nu_sp.size());
    for (size_t e = 0; e < t->nu_sp.size(); ++e) t->nu_vid[e] = yid(t->nu_sp[e]);
    const int P = (int)parts.size();
    if (P + 1 >= (1 << kOffBits)) {
        *err = "too many rate partials for the 14-bit offsets of the solver tables";
        return MCC_ERR_MECH;
    }

    // ---- solver: f gather, one chain per (slot, lane) ----------------------
    std::vector<std::vector<std::pair<int, double>>> fcon(t->NV);
    for (int j = 0; j < R; ++j)
        for (const auto &kv : net_stoich(d, j))
            if (kv.second != 0.0) fcon[vid(kv.first)].push_back({j, kv.second});
    t->fg_ops.clear();
    t->fg_blocks.assign(t->NS, 0);
    t->fg_base.assign(t->NS, 0);
    for (int s = 0; s < t->NS; ++s) {
        std::vector<std::vector<Op16>> lanes(kWave);
        for (int lane = 0; lane < kWave; ++lane)
            for (const auto &c : fcon[s * kWave + lane]) lanes[lane].push_back(make_op16(c.second, (uint32_t)c.first));
        t->fg_base[s] = (int32_t)(t->fg_ops.size() / (kWave * kBlk));
        t->fg_blocks[s] = emit_blocks(lanes, make_op16(0.0, (uint32_t)R), &t->fg_ops);
    }

    // ---- solver: Newton-matrix gather over all LU entries -----------------
    // Chain per LU entry: acc = sum coef * partial; entry = [diag] 1 - c acc.
    // Fill entries are chains of one zero term (they are reset every time).
    {
        std::vector<std::vector<std::pair<int, double>>> eterms(nlu);
        std::vector<char> ediag(nlu, 0);
        for (int p = 0; p < N; ++p) ediag[lpos[p][p]] = 1;
        for (int qi = 0; qi < P; ++qi)
            for (const auto &kv : net_stoich(d, parts[qi].j))
                if (kv.second != 0.0)
                {
                    // J entry (i = species changed, s = the partial's species); transposed: entry (s, i)
                    const int ri = t->iperm[kv.first], cs = t->iperm[parts[qi].s];
                    eterms[transpose ? lpos[cs][ri] : lpos[ri][cs]].push_back({qi, kv.second});
                }
        std::vector<std::vector<Op16>> chains(nlu);
        for (int e = 0; e < nlu; ++e) {
            auto &tl = eterms[e];
            if (tl.empty()) tl.push_back({P, 0.0});
            for (size_t q = 0; q < tl.size(); ++q) {
                uint32_t fl = 0;
                if (q == 0) fl |= kFirst;
                if (q + 1 == tl.size()) fl |= kLast | (ediag[e] ? kDiag : 0u);
                chains[e].push_back(make_op16(tl[q].second, (uint32_t)tl[q].first | ((uint32_t)e << 16), fl));
            }
        }
        auto lanes = pack_chains(chains);
        t->nm_ops.clear();
        t->nm_blocks = emit_blocks(lanes, make_op16(0.0, (uint32_t)P | ((uint32_t)TRASH << 16)), &t->nm_ops);
    }

    // ---- solver: level-scheduled right-looking LU of the front pivots ------
    // Pivot k depends on every earlier pivot that updates its row or column
    // (L(k,k') or U(k',k) structurally nonzero).  Pivots of one level only
    // write entries no other pivot of that level reads, so a level is one
    // step between barriers.  Entries written by several pivots of a level
    // are summed by one lane (a chain).  1/U_kk replaces U_kk in storage as
    // soon as U_kk is final (flag on its last update, or in step 0 if nothing
    // updates it); column k is scaled by it one level after pivot k.  Updates
    // into the tail block form its Schur complement.
    std::vector<int> level(F, 1);
    int maxlev = 0;
    for (int k = 0; k < F; ++k) {
        for (int q = 0; q < k; ++q)
            if (lp[k][q] || lp[q][k]) level[k] = std::max(level[k], level[q] + 1);
        maxlev = std::max(maxlev, level[k]);
    }
    std::vector<int> diag_last(F, 0);  // level of the last update of (k,k)
    for (int q = 0; q < F; ++q)
        for (int k = q + 1; k < F; ++k)
            if (lp[k][q] && lp[q][k]) diag_last[k] = std::max(diag_last[k], level[q]);
    t->lu_ops.clear();
    t->lu_barrier.clear();
    t->lu_steps = 0;
    const uint64_t NOP = lu_op(TRASH, ZERO, ZERO, ZERO, kLuFirst | kLuLast);
    auto emit_step = [&](std::vector<std::vector<uint64_t>> &chains) {
        if (chains.empty()) return;
        auto lanes = pack_chains(chains);
        size_t len = 0;
        for (auto &l : lanes) len = std::max(len, l.size());
        len = (len + kBlk - 1) / kBlk * kBlk;
        for (auto &l : lanes)
            while (l.size() < len) l.push_back(NOP);
        const int nb = emit_blocks(lanes, NOP, &t->lu_ops);
        for (int b = 0; b < nb; ++b) t->lu_barrier.push_back(b + 1 == nb ? 1 : 0);
        t->lu_steps++;
    };
    if (F > 0) {
        std::vector<std::vector<uint64_t>> chains;
        for (int k = 0; k < F; ++k)
            if (diag_last[k] == 0) chains.push_back({lu_op(lpos[k][k], ZERO, ZERO, ZERO, kLuFirst | kLuLast | kLuRecip)});
        emit_step(chains);
    }
    for (int L = 1; L <= maxlev + 1 && F > 0; ++L) {
        std::map<int, std::vector<uint64_t>> by_dst;
        std::vector<std::vector<uint64_t>> chains;
        for (int k = 0; k < F; ++k) {
            if (level[k] == L - 1)  // scale column k of a pivot finished one level ago
                for (int i = k + 1; i < N; ++i)
                    if (lp[i][k]) chains.push_back({lu_op(lpos[i][k], ZERO, ZERO, lpos[k][k], kLuFirst | kLuLast | kLuScale)});
            if (level[k] != L) continue;
            for (int i = k + 1; i < N; ++i) {
                if (!lp[i][k]) continue;
                for (int j = k + 1; j < N; ++j) {
                    if (!lp[k][j]) continue;
                    if (i >= F && j >= F) continue;  // into the tail block: the Schur product below
                    by_dst[lpos[i][j]].push_back(lu_op(lpos[i][j], lpos[i][k], lpos[k][j], lpos[k][k], 0));
                }
            }
        }
        for (auto &kv : by_dst) {
            auto &c = kv.second;
            c.front() |= kLuFirst;
            c.back() |= kLuLast;
            const int dst = kv.first;
            // front diagonal entry whose last update happens at this level
            for (int k = 0; k < F; ++k)
                if (lpos[k][k] == dst && diag_last[k] == L) c.back() |= kLuRecip;
            chains.push_back(c);
        }
        emit_step(chains);
    }
    t->lu_blocks = (int)(t->lu_ops.size() / (kWave * kBlk));

    // ---- solver: Schur complement of the front onto the tail ----------------
    // Every update of a tail entry by a front pivot, a_ij -= l_ik u_kj with
    // i, j >= F and k < F, together: T -= L_TF U_FT once the front is done
    // (its L columns scaled), in 16 x 16 x 4 matrix-core blocks.
    t->schur_ks = 0;
    t->schur_sk = 0;
    t->schur_tab.clear();
    if (M > 0 && F > 0) {
        const int nt = M / 16, KS = (F + 3) / 4;
        const int SK = nt == 3 ? 4 : 16 / nt;  // 2 nt SK offsets fill whole vectors of 8
        const int groups = (KS + SK - 1) / SK, per_lane = groups * SK * 2 * nt;
        t->schur_ks = KS;
        t->schur_sk = SK;
        t->schur_tab.assign((size_t)per_lane * kWave, (uint16_t)ZERO);
        for (int ks = 0; ks < KS; ++ks)
            for (int lane = 0; lane < kWave; ++lane) {
                const int kc = 4 * ks + lane / 16;
                if (kc >= F) continue;
                for (int q = 0; q < 2 * nt; ++q) {
                    const int e = ks * 2 * nt + q;  // this lane's e-th offset: vector e / 8, place e % 8
                    const size_t at = ((size_t)(e / 8) * kWave + lane) * 8 + e % 8;
                    if (q < nt) {
                        const int row = F + 16 * q + lane % 16;
                        if (lp[row][kc]) t->schur_tab[at] = (uint16_t)lpos[row][kc];
                    } else {
                        const int col = F + 16 * (q - nt) + lane % 16;
                        if (lp[kc][col]) t->schur_tab[at] = (uint16_t)lpos[kc][col];
                    }
                }
            }
    }

    // ---- solver: column maps for the triangular solves ---------------------
    // [slot][lane][v]: for the column at virtual index v, the offset of L(p,k)
    // (p after k) for the forward sweep, of U(p,k) (p before k) or of the
    // stored 1/U_kk (p == k) for the backward sweep; else the zero cell.
    const size_t map_n = (size_t)t->NS * kWave * t->NV;
    t->fwd_map.assign(map_n, (uint16_t)ZERO);
    t->bwd_map.assign(map_n, (uint16_t)ZERO);
    for (int pr = 0; pr < N; ++pr)
        for (int k = 0; k < N; ++k) {
            const size_t at = (size_t)vpos[pr] * t->NV + vpos[k];
            if (pr > k && lp[pr][k]) t->fwd_map[at] = (uint16_t)lpos[pr][k];
            if (pr <= k && lp[pr][k]) t->bwd_map[at] = (uint16_t)lpos[pr][k];
        }
    // per-slot column counts (virtual columns in use)
    t->slot_cols.assign(t->NS, 0);
    for (int p = 0; p < N; ++p) t->slot_cols[vpos[p] / kWave] = std::max(t->slot_cols[vpos[p] / kWave], vpos[p] % kWave + 1);

    // ---- algorithmic work per cell -----------------------------------------
    {
        int64_t prod_mults = 0, part_mults = 0, n_fterms = 0, n_jterms = 0, n_lower = 0, n_upper = 0;
        (void)TRASH;
        for (int j = 0; j < R; ++j) {
            const int a = d->reac_ptr[j + 1] - d->reac_ptr[j];
            prod_mults += a;
            part_mults += (int64_t)a * (a - 1);
        }
        for (int r = 0; r < N; ++r) n_fterms += t->out_ptr[r + 1] - t->out_ptr[r];
        n_jterms = (int64_t)t->out_ptr[N + t->nnz] - t->out_ptr[N];
        n_lower = t->lu_lower;
        n_upper = t->lu_upper;
        mcc_op_counts &oc = t->counts;
        oc.deriv_flops = prod_mults + 2 * n_fterms;
        oc.newton_matrix_flops = part_mults + 2 * n_jterms + t->nnz + N;
        oc.lu_flops = 2 * t->lu_updates + N + n_lower;
        oc.solve_flops = 2 * (n_lower + n_upper) + N;
        oc.f_bytes = 8 * (int64_t)(2 * N + R);
        oc.j_bytes = 8 * (int64_t)(N + R + t->nnz);
        oc.fj_bytes = 8 * (int64_t)(2 * N + R + t->nnz);
        oc.reserved = 0;
    }

    return MCC_OK;
}

// VJP work items.  Rows are numbered k_j -> j, y_s -> R + s, v_s -> R + N + s.
// Columns are taken largest first (most rows to load); each item then grows
// by the column that shares reactions with it and adds the fewest new rows,
// while its rows stay within the budget (a column over the budget on its own
// is an item of its own, loaded in several rounds).  Columns of species that
// are no reactant (gy_s = 0) are dealt out over the items at the end.
std::vector<VjpItem> plan_vjp(const HostTables &t, int round_loads)
{
    const int N = t.N, R = t.R, n_rows = R + 2 * N;
    std::vector<std::vector<int32_t>> rx_rows(R), col_rx(N);
    for (int j = 0; j < R; ++j) {
        std::vector<int32_t> &r = rx_rows[j];
        r.push_back(j);
        for (int q = 0; q < 3; ++q) {
            const int s = t.rx_sp[3 * j + q];
            if (s < 0) continue;
            r.push_back(R + s);
            if (col_rx[s].empty() || col_rx[s].back() != j) col_rx[s].push_back(j);
        }
        for (int e = t.nu_ptr[j]; e < t.nu_ptr[j + 1]; ++e) r.push_back(R + N + t.nu_sp[e]);
        std::sort(r.begin(), r.end());
        r.erase(std::unique(r.begin(), r.end()), r.end());
    }
    std::vector<std::vector<int32_t>> col_rows(N);
    for (int s = 0; s < N; ++s) {
        for (int j : col_rx[s]) col_rows[s].insert(col_rows[s].end(), rx_rows[j].begin(), rx_rows[j].end());
        std::sort(col_rows[s].begin(), col_rows[s].end());
        col_rows[s].erase(std::unique(col_rows[s].begin(), col_rows[s].end()), col_rows[s].end());
    }
    std::vector<int> order(N);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return col_rows[a].size() > col_rows[b].size(); });
    std::vector<char> done(N, 0), in_item(n_rows, 0);
    std::vector<VjpItem> items;
    std::vector<int> zero_cols;
    for (int s0 : order) {
        if (done[s0]) continue;
        if (col_rx[s0].empty()) {
            zero_cols.push_back(s0);
            done[s0] = 1;
            continue;
        }
        VjpItem it;
        std::vector<int32_t> rows = col_rows[s0];
        for (int r : rows) in_item[r] = 1;
        it.cols.push_back(s0);
        done[s0] = 1;
        while (true) {
            int best = -1, best_n = 0;
            for (int c0 : it.cols)
                for (int j : col_rx[c0])
                    for (int q = 0; q < 3; ++q) {
                        const int s = t.rx_sp[3 * j + q];
                        if (s < 0 || done[s]) continue;
                        int n = 0;
                        for (int r : col_rows[s]) n += !in_item[r];
                        if ((int)rows.size() + n > round_loads) continue;
                        if (best < 0 || n < best_n || (n == best_n && s < best)) best = s, best_n = n;
                    }
            if (best < 0) break;
            for (int r : col_rows[best])
                if (!in_item[r]) in_item[r] = 1, rows.push_back(r);
            it.cols.push_back(best);
            done[best] = 1;
        }
        for (int r : rows) in_item[r] = 0;
        items.push_back(it);
    }
    if (items.empty()) items.push_back(VjpItem{});  // no reaction has a reactant
    for (size_t q = 0; q < zero_cols.size(); ++q) items[q % items.size()].cols.push_back(zero_cols[q]);
    // reactions of each item, d/d ln k ownership, then the load rounds
    std::vector<int> owner(R, -1), col_item(N, -1);
    for (size_t i = 0; i < items.size(); ++i)
        for (int s : items[i].cols) col_item[s] = (int)i;
    std::vector<std::vector<int32_t>> item_rx(items.size());
    for (int j = 0; j < R; ++j) {
        const int s = t.rx_sp[3 * j];
        owner[j] = s >= 0 ? col_item[s] : (int)items.size() - 1;  // no reactant: the last item
        if (s < 0) item_rx[owner[j]].push_back(j);
    }
    for (size_t i = 0; i < items.size(); ++i) {
        for (int s : items[i].cols) item_rx[i].insert(item_rx[i].end(), col_rx[s].begin(), col_rx[s].end());
        std::vector<int32_t> &rx = item_rx[i];
        std::sort(rx.begin(), rx.end());
        rx.erase(std::unique(rx.begin(), rx.end()), rx.end());
        std::vector<int32_t> cur;
        std::vector<int32_t> round_rows;
        for (int j : rx) {
            int n = 0;
            for (int r : rx_rows[j]) n += !in_item[r];
            if (!cur.empty() && (int)round_rows.size() + n > round_loads) {
                items[i].rounds.push_back(cur);
                for (int r : round_rows) in_item[r] = 0;
                cur.clear();
                round_rows.clear();
            }
            cur.push_back(j);
            for (int r : rx_rows[j])
                if (!in_item[r]) in_item[r] = 1, round_rows.push_back(r);
            if (owner[j] == (int)i) items[i].glnk.push_back(j);
        }
        if (!cur.empty()) items[i].rounds.push_back(cur);
        for (int r : round_rows) in_item[r] = 0;
    }
    return items;
}

}  // namespace mcc
