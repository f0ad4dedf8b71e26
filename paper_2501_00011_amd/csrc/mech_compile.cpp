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

}  // namespace

mcc_status compile_mechanism(const mcc_mech_desc *d, HostTables *t, std::string *err)
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

    // ---- streaming terms (species order) ----------------------------------
    // f_i: one term per (reaction, participant i) with the full rate monomial.
    // J_is: one term per (partial of slot l with species s, participant i).
    std::vector<std::vector<std::pair<std::array<int32_t, 4>, double>>> out_terms(N + t->nnz);
    for (int j = 0; j < R; ++j) {
        const auto nu = net_stoich(d, j);
        const int b = d->reac_ptr[j], e = d->reac_ptr[j + 1];
        std::array<int32_t, 4> mono = {j, N, N, N};
        for (int q = b; q < e; ++q) mono[1 + (q - b)] = d->reac_idx[q];
        for (const auto &kv : nu)
            if (kv.second != 0.0) out_terms[kv.first].push_back({mono, kv.second});
    }
    for (const Partial &p : parts) {
        const auto nu = net_stoich(d, p.j);
        std::array<int32_t, 4> mono = {p.j, p.o1, p.o2, N};
        for (const auto &kv : nu)
            if (kv.second != 0.0) out_terms[N + jpos[kv.first][p.s]].push_back({mono, kv.second});
    }
    t->out_ptr.assign(1, 0);
    t->term_idx.clear();
    t->term_coef.clear();
    for (const auto &ot : out_terms) {
        for (const auto &tm : ot) {
            t->term_idx.insert(t->term_idx.end(), tm.first.begin(), tm.first.end());
            t->term_coef.push_back(tm.second);
        }
        t->out_ptr.push_back((int32_t)t->term_coef.size());
    }
    // Chunks of consecutive output rows with about `target` terms each (every
    // row is at least one unit of work: it is written even with no terms).
    auto make_chunks = [&](int r0, int r1, int target) {
        int count = 0;
        int begin = r0;
        t->fj_chunks.push_back(r0);
        for (int r = r0; r < r1; ++r) {
            count += std::max(1, t->out_ptr[r + 1] - t->out_ptr[r]);
            if (count >= target && r + 1 < r1) {
                t->fj_chunks.push_back(r + 1);
                count = 0;
                begin = r + 1;
            }
        }
        (void)begin;
        return 0;
    };
    t->fj_chunks.clear();
    const int target = 64;
    make_chunks(0, N, target);
    t->n_fchunks = (int)t->fj_chunks.size();
    make_chunks(N, N + t->nnz, target);
    t->n_jchunks = (int)t->fj_chunks.size() - t->n_fchunks;
    t->fj_chunks.push_back(N + t->nnz);

    // ---- fill-reducing order and symbolic LU (permuted order) -------------
    t->perm = markowitz_order(pat);
    t->iperm.assign(N, 0);
    for (int p = 0; p < N; ++p) t->iperm[t->perm[p]] = p;
    std::vector<std::vector<char>> lp(N, std::vector<char>(N, 0));
    for (int i = 0; i < N; ++i)
        for (int s = 0; s < N; ++s)
            if (pat[i][s]) lp[t->iperm[i]][t->iperm[s]] = 1;
    for (int k = 0; k < N; ++k)
        for (int i = k + 1; i < N; ++i)
            if (lp[i][k])
                for (int j = k + 1; j < N; ++j)
                    if (lp[k][j]) lp[i][j] = 1;
    std::vector<std::vector<int>> lpos(N, std::vector<int>(N, -1));
    int nlu = 0;
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j)
            if (lp[i][j]) lpos[i][j] = nlu++;
    t->lu_nnz = nlu;
    if (nlu + 2 > 65535) {
        *err = "LU fill exceeds the 16-bit offset range of the solver tables";
        return MCC_ERR_MECH;
    }
    const int ZERO = nlu;       // LDS cell holding 0.0
    const int TRASH = nlu + 1;  // LDS cell written by idle lanes

    // ---- solver: reactions and partials in permuted ids -------------------
    t->rx_reac.assign(4 * (size_t)R, N);
    for (int j = 0; j < R; ++j) {
        const int b = d->reac_ptr[j], e = d->reac_ptr[j + 1];
        for (int q = b; q < e; ++q) t->rx_reac[4 * j + (q - b)] = t->iperm[d->reac_idx[q]];
        t->rx_reac[4 * j + 3] = 0;
    }
    t->part.assign(4 * parts.size(), 0);
    for (size_t q = 0; q < parts.size(); ++q) {
        t->part[4 * q + 0] = parts[q].j;
        t->part[4 * q + 1] = parts[q].o1 < N ? t->iperm[parts[q].o1] : N;
        t->part[4 * q + 2] = parts[q].o2 < N ? t->iperm[parts[q].o2] : N;
    }

    // ---- solver: f gather per slot (rv[R] is a zero rate) -----------------
    std::vector<std::vector<std::pair<int, double>>> fcon(N);
    for (int j = 0; j < R; ++j)
        for (const auto &kv : net_stoich(d, j))
            if (kv.second != 0.0) fcon[t->iperm[kv.first]].push_back({j, kv.second});
    t->fg_w.assign(t->NS, 0);
    t->fg_off.assign(t->NS, 0);
    t->fg_idx.clear();
    t->fg_coef.clear();
    for (int s = 0; s < t->NS; ++s) {
        int w = 0;
        for (int lane = 0; lane < kWave; ++lane) {
            const int p = s * kWave + lane;
            if (p < N) w = std::max(w, (int)fcon[p].size());
        }
        t->fg_w[s] = w;
        t->fg_off[s] = (int32_t)t->fg_idx.size();
        for (int q = 0; q < w; ++q)
            for (int lane = 0; lane < kWave; ++lane) {
                const int p = s * kWave + lane;
                const bool have = p < N && q < (int)fcon[p].size();
                t->fg_idx.push_back(have ? fcon[p][q].first : R);
                t->fg_coef.push_back(have ? fcon[p][q].second : 0.0);
            }
    }

    // ---- solver: Newton-matrix gather over all LU entries -----------------
    // LU entry (p, q) <- J entry (perm[p], perm[q]) if present; fill entries get 0.
    struct Entry { int dest; bool diag; std::vector<std::pair<int, double>> terms; };
    std::vector<Entry> entries(nlu);
    for (int p = 0; p < N; ++p)
        for (int q = 0; q < N; ++q)
            if (lpos[p][q] >= 0) entries[lpos[p][q]] = {lpos[p][q], p == q, {}};
    for (size_t qi = 0; qi < parts.size(); ++qi) {
        const auto nu = net_stoich(d, parts[qi].j);
        for (const auto &kv : nu)
            if (kv.second != 0.0) {
                const int e = lpos[t->iperm[kv.first]][t->iperm[parts[qi].s]];
                entries[e].terms.push_back({(int)qi, kv.second});
            }
    }
    std::vector<int> eorder(nlu);
    std::iota(eorder.begin(), eorder.end(), 0);
    std::stable_sort(eorder.begin(), eorder.end(), [&](int a, int b) {
        return entries[a].terms.size() > entries[b].terms.size();
    });
    const int n_pass = (nlu + kWave - 1) / kWave;
    t->jg_dest.assign((size_t)n_pass * kWave, TRASH);
    t->jg_w.assign(n_pass, 0);
    t->jg_off.assign(n_pass, 0);
    t->jg_idx.clear();
    t->jg_coef.clear();
    const int P = (int)parts.size();
    for (int ps = 0; ps < n_pass; ++ps) {
        int w = 0;
        for (int lane = 0; lane < kWave; ++lane) {
            const int x = ps * kWave + lane;
            if (x < nlu) {
                const Entry &en = entries[eorder[x]];
                t->jg_dest[(size_t)ps * kWave + lane] = en.dest | (en.diag ? (1 << 30) : 0);
                w = std::max(w, (int)en.terms.size());
            }
        }
        t->jg_w[ps] = w;
        t->jg_off[ps] = (int32_t)t->jg_idx.size();
        for (int q = 0; q < w; ++q)
            for (int lane = 0; lane < kWave; ++lane) {
                const int x = ps * kWave + lane;
                const bool have = x < nlu && q < (int)entries[eorder[x]].terms.size();
                t->jg_idx.push_back(have ? entries[eorder[x]].terms[q].first : P);
                t->jg_coef.push_back(have ? entries[eorder[x]].terms[q].second : 0.0);
            }
    }

    // ---- solver: right-looking LU schedule -------------------------------
    t->lu_diag.assign(N, 0);
    t->lcol_ptr.assign(1, 0);
    t->upd_ptr.assign(1, 0);
    t->lcol_off.clear();
    t->upd.clear();
    t->lu_updates = 0;
    for (int k = 0; k < N; ++k) {
        t->lu_diag[k] = lpos[k][k];
        std::vector<int> rows, cols;
        for (int i = k + 1; i < N; ++i)
            if (lp[i][k]) rows.push_back(i);
        for (int j = k + 1; j < N; ++j)
            if (lp[k][j]) cols.push_back(j);
        for (int i : rows) t->lcol_off.push_back(lpos[i][k]);
        for (int i : rows)
            for (int j : cols) {
                const uint64_t dst = (uint64_t)lpos[i][j], l = (uint64_t)lpos[i][k], u = (uint64_t)lpos[k][j];
                t->upd.push_back(dst | (l << 16) | (u << 32));
            }
        t->lu_updates += (int64_t)rows.size() * (int64_t)cols.size();
        t->lcol_ptr.push_back((int32_t)t->lcol_off.size());
        t->upd_ptr.push_back((int32_t)t->upd.size());
    }

    // ---- algorithmic work per cell -----------------------------------------
    {
        int64_t prod_mults = 0, part_mults = 0, n_fterms = 0, n_jterms = 0, n_lower = 0, n_upper = 0;
        for (int j = 0; j < R; ++j) {
            const int a = d->reac_ptr[j + 1] - d->reac_ptr[j];
            prod_mults += a;
            part_mults += (int64_t)a * (a - 1);
        }
        for (int r = 0; r < N; ++r) n_fterms += t->out_ptr[r + 1] - t->out_ptr[r];
        n_jterms = (int64_t)t->out_ptr[N + t->nnz] - t->out_ptr[N];
        for (int p = 0; p < N; ++p)
            for (int q = 0; q < N; ++q)
                if (lp[p][q]) {
                    if (p > q) n_lower++;
                    if (p < q) n_upper++;
                }
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

    // ---- solver: dense column maps for the triangular solves ---------------
    const size_t map_n = (size_t)N * t->NS * kWave;
    t->fwd_map.assign(map_n, (uint16_t)ZERO);
    t->bwd_map.assign(map_n, (uint16_t)ZERO);
    for (int k = 0; k < N; ++k)
        for (int s = 0; s < t->NS; ++s)
            for (int lane = 0; lane < kWave; ++lane) {
                const int p = s * kWave + lane;
                if (p >= N) continue;
                const size_t at = ((size_t)k * t->NS + s) * kWave + lane;
                if (p > k && lp[p][k]) t->fwd_map[at] = (uint16_t)lpos[p][k];
                if (p < k && lp[p][k]) t->bwd_map[at] = (uint16_t)lpos[p][k];
            }
    return MCC_OK;
}

}  // namespace mcc
