// Mechanism-specialised f/J kernel: the streaming f/J tables (work items ->
// chunks -> monomials and output records) written out as straight-line HIP,
// one switch case per work item, and compiled at mechanism creation with
// hipRTC.  Row indices become constants (the row address is a scalar
// multiply of the leading dimension), coefficients become literals, each y
// or k row an item uses is loaded once into a register, and no table is
// read at run time: what is left is the loads, the products and sums of the
// rate expressions, and the stores.  The arithmetic is the one the tables
// describe (Section 2: mass-action rates and their partials, f = sum nu r,
// J = sum nu dr/dy), term by term in the same order.
#include <hip/hiprtc.h>

#include <algorithm>
#include <cstdio>
#include <set>
#include <sstream>
#include <string>
#include <vector>

#include "mcc_internal.hpp"

namespace mcc {

namespace {

std::string lit(double v)
{
    char b[64];
    std::snprintf(b, sizeof b, "%a", v);  // exact: hexadecimal floating literal
    return b;
}

}  // namespace

// Token placeholders of the generated bodies, filled per variant: @V@ the
// per-cell value type (double, or the two-cell pair d2), @L@ the row stride
// in values (ld, or ld / 2), @Z@ a zero value.
namespace {

std::string fill(std::string s, bool pair)
{
    const std::pair<const char *, const char *> rep[] = {
        {"@V@", pair ? "d2" : "double"}, {"@L@", pair ? "ldv" : "ld"}, {"@Z@", pair ? "d2{0.0, 0.0}" : "0.0"}};
    for (const auto &r : rep)
        for (size_t at = s.find(r.first); at != std::string::npos; at = s.find(r.first, at)) s.replace(at, 3, r.second);
    return s;
}

// Kernel head: block -> (64-lane tile, work item).  Blocks come in groups
// of 8 * grp_tiles tiles times n_items; within a group the order is item
// major: block q of XCD xcd (bid = 8 q + xcd) runs item r / grp_tiles on tile
// (group * grp_tiles + r % grp_tiles) * 8 + xcd, r = q mod (n_items *
// grp_tiles).  grp_tiles = 1 runs all items of a tile on one XCD, one tile
// after the other (the inputs of a tile are fetched once and then served by
// that XCD's L2); a larger grp_tiles runs each item over 8 * grp_tiles
// consecutive tiles at about the same time, so that the first reads of every
// row are long runs of consecutive cells.  One-cell variant: lane = cell
// c_begin + tile * 64 + lane.  Pair variant: lane = cells 2c and 2c + 1 with
// c = tile * 64 + lane, 16-byte accesses (the caller guarantees an even ld,
// 16-byte aligned arrays and whole pairs: n_cells even).
std::string head(const char *name, const char *args, const char *ptrs, bool pair)
{
    std::ostringstream o;
    o << "extern \"C\" __global__ __launch_bounds__(64) void " << name << (pair ? "2" : "") << "(\n" << args
      << ", long long n_cells, long long ld, long long c_begin, int item_begin, int n_items, int n_tiles,\n"
      << "    int grp_tiles)\n"
      << "{\n"
      << "    const int bid = blockIdx.x, xcd = bid & 7, q = bid >> 3;\n"
      << "    const int grp = q / (n_items * grp_tiles), r = q - grp * (n_items * grp_tiles);\n"
      << "    const int item = item_begin + r / grp_tiles, tile = (grp * grp_tiles + r % grp_tiles) * 8 + xcd;\n"
      << "    if (tile >= n_tiles) return;\n";
    if (pair)
        o << "    const long long c = (long long)tile * 64 + threadIdx.x;  // pair index\n"
          << "    if (2 * c + 1 >= n_cells) return;\n"
          << "    const long long ldv = ld >> 1;\n"
          << "    (void)c_begin;\n";
    else
        o << "    const long long c = c_begin + (long long)tile * 64 + threadIdx.x;\n"
          << "    if (c >= n_cells) return;\n";
    o << ptrs;
    return o.str();
}

}  // namespace

std::string generate_preamble()
{
    return "// generated per mechanism; d2 = the values of two adjacent cells\n"
           "struct __attribute__((aligned(16))) d2 { double x, y; };\n"
           "__device__ __forceinline__ d2 operator+(d2 a, d2 b) { return d2{a.x + b.x, a.y + b.y}; }\n"
           "__device__ __forceinline__ d2 operator*(d2 a, d2 b) { return d2{a.x * b.x, a.y * b.y}; }\n"
           "__device__ __forceinline__ d2 operator*(double s, d2 b) { return d2{s * b.x, s * b.y}; }\n"
           "__device__ __forceinline__ d2 &operator+=(d2 &a, d2 b) { a.x += b.x; a.y += b.y; return a; }\n"
           "// outputs are stored non-temporally: no kernel reads them back soon\n"
           "__device__ __forceinline__ void st_out(double *p, double x) { __builtin_nontemporal_store(x, p); }\n"
           "typedef double d2v __attribute__((ext_vector_type(2)));\n"
           "__device__ __forceinline__ void st_out(d2 *p, d2 x) { __builtin_nontemporal_store(d2v{x.x, x.y}, (d2v *)p); }\n";
}

std::string generate_fj_source(const HostTables &t, bool pair)
{
    const int N = t.N;
    std::ostringstream o;
    o << "// f/J kernel: " << N << " species, " << t.R << " reactions, " << t.nnz << " Jacobian nonzeros\n"
      << head("mcc_fj_generated",
              "    const double *__restrict__ y, const double *__restrict__ k, double *__restrict__ f,\n"
              "    double *__restrict__ jac",
              "    const @V@ *__restrict__ Y = (const @V@ *)y + c;\n"
              "    const @V@ *__restrict__ K = (const @V@ *)k + c;\n"
              "    @V@ *__restrict__ F = (@V@ *)f + c;\n"
              "    @V@ *__restrict__ G = (@V@ *)jac + c;\n",
              pair)
      << "    switch (item) {\n";

    const int n_items = t.n_fitems + t.n_jitems;
    for (int it = 0; it < n_items; ++it) {
        o << "    case " << it << ": {\n";
        // every row the item uses, loaded once, at the top (all in flight together)
        std::set<int> ys, ks;
        for (int ci = t.fj_items[it]; ci < t.fj_items[it + 1]; ++ci) {
            const FjChunk &ch = t.fj_chunks[ci];
            for (int qm = 0; qm < ch.n_mono; ++qm) {
                const FjMono &m = t.fj_monos[ch.mono_begin + qm];
                if (m.j >= 0) ks.insert(m.j);
                for (int f3 : {m.a, m.b, m.c})
                    if (f3 >= 0) ys.insert(f3);
            }
        }
        for (int j : ks) o << "        const @V@ k" << j << " = K[" << j << " * @L@];\n";
        for (int r : ys) o << "        const @V@ y" << r << " = Y[" << r << " * @L@];\n";
        for (int ci = t.fj_items[it]; ci < t.fj_items[it + 1]; ++ci) {
            const FjChunk &ch = t.fj_chunks[ci];
            o << "        {\n";
            std::vector<std::string> mono(kFjQmax);
            for (int qm = 0; qm < ch.n_mono; ++qm) {
                const FjMono &m = t.fj_monos[ch.mono_begin + qm];
                if (m.j < 0 && m.a < 0 && m.b < 0 && m.c < 0) continue;  // padding
                std::string e;
                if (m.j >= 0) e = "k" + std::to_string(m.j);
                for (int f3 : {m.a, m.b, m.c})
                    if (f3 >= 0) e += (e.empty() ? "" : " * ") + ("y" + std::to_string(f3));
                mono[qm] = "m" + std::to_string(qm);
                o << "            const @V@ " << mono[qm] << " = " << e << ";\n";
            }
            o << "            @V@ acc = @Z@;\n";
            for (int r = 0; r < ch.n_rec; ++r) {
                const FjRec &rec = t.fj_recs[ch.rec_begin + r];
                const uint32_t flags = rec.meta >> 24, row = rec.meta & kFjRowMask;
                std::string sum;
                for (int qq = 0; qq < 3; ++qq) {
                    const int slot = (rec.slots >> (8 * qq)) & 0xff;
                    if (slot >= kFjQmax || rec.coef[qq] == 0.0 || mono[slot].empty()) continue;
                    sum += (sum.empty() ? "" : " + ") + lit(rec.coef[qq]) + " * " + mono[slot];
                }
                if (sum.empty()) sum = "@Z@";
                if (!(flags & (kFjKeep | kFjStore))) {
                    if (sum == "@Z@") continue;  // padding record
                }
                o << "            acc " << ((flags & kFjKeep) ? "+=" : "=") << " " << sum << ";\n";
                if (flags & kFjStore) {
                    const std::string dst = row < (uint32_t)N ? "F[" + std::to_string(row) + " * @L@]"
                                                              : "G[" + std::to_string(row - N) + " * @L@]";
                    if (flags & kFjAdd)
                        o << "            " << dst << " += acc;\n";  // a later part of a split sum
                    else
                        o << "            st_out(&" << dst << ", acc);\n";
                }
            }
            o << "            (void)acc;\n        }\n";
        }
        o << "    } break;\n";
    }
    o << "    default: break;\n    }\n}\n";
    return fill(o.str(), pair);
}

}  // namespace mcc

namespace mcc {

// Vector-Jacobian products (reverse mode of f), one switch case per work
// item of the plan (plan_vjp): per load round, the round's k, y and v rows
// are loaded together; then per reaction w_j = sum_i nu_ij v_i, the item's
// columns among j's reactants gain w_j * d r_j / d y_s, and the item that
// owns j writes d(v.f)/d ln k_j = r_j * w_j.  gy_s is written when the item
// ends.  A null gy or glnk skips its stores (the same arithmetic runs).
std::string generate_vjp_source(const HostTables &t, bool pair)
{
    std::ostringstream o;
    o << head("mcc_vjp_generated",
              "    const double *__restrict__ y, const double *__restrict__ k, const double *__restrict__ v,\n"
              "    double *__restrict__ gy, double *__restrict__ glnk",
              "    const bool want_gy = gy != nullptr, want_glnk = glnk != nullptr;\n"
              "    const @V@ *__restrict__ Y = (const @V@ *)y + c;\n"
              "    const @V@ *__restrict__ K = (const @V@ *)k + c;\n"
              "    const @V@ *__restrict__ V = (const @V@ *)v + c;\n"
              "    @V@ *__restrict__ GY = (@V@ *)gy + c;\n"
              "    @V@ *__restrict__ GK = (@V@ *)glnk + c;\n",
              pair)
      << "    switch (item) {\n";
    for (size_t it = 0; it < t.vjp_items.size(); ++it) {
        const VjpItem &item = t.vjp_items[it];
        std::set<int> cols(item.cols.begin(), item.cols.end()), owned(item.glnk.begin(), item.glnk.end());
        o << "    case " << it << ": {\n";
        for (int s : item.cols) o << "        @V@ g" << s << " = @Z@;\n";
        for (const std::vector<int32_t> &round : item.rounds) {
            o << "        {\n";
            std::set<int> ks, ys, vs;
            for (int j : round) {
                ks.insert(j);
                for (int q = 0; q < 3; ++q)
                    if (t.rx_sp[3 * j + q] >= 0) ys.insert(t.rx_sp[3 * j + q]);
                for (int e = t.nu_ptr[j]; e < t.nu_ptr[j + 1]; ++e) vs.insert(t.nu_sp[e]);
            }
            for (int j : ks) o << "            const @V@ k" << j << " = K[" << j << " * @L@];\n";
            for (int r : ys) o << "            const @V@ y" << r << " = Y[" << r << " * @L@];\n";
            for (int r : vs) o << "            const @V@ v" << r << " = V[" << r << " * @L@];\n";
            for (int j : round) {
                std::string w;
                for (int e = t.nu_ptr[j]; e < t.nu_ptr[j + 1]; ++e)
                    w += (w.empty() ? "" : " + ") + lit(t.nu_coef[e]) + " * v" + std::to_string(t.nu_sp[e]);
                o << "            const @V@ w" << j << " = " << (w.empty() ? "@Z@" : w) << ";\n";
                const int32_t *a = &t.rx_sp[3 * j];
                for (int q = 0; q < 3; ++q) {
                    const int s = a[q];
                    if (s < 0 || !cols.count(s)) continue;
                    bool first = true;  // each distinct reactant once
                    for (int p = 0; p < q; ++p) first = first && a[p] != s;
                    if (!first) continue;
                    int mult = 0;
                    bool skipped = false;
                    std::string d = "k" + std::to_string(j);
                    for (int p = 0; p < 3; ++p) {
                        if (a[p] < 0) continue;
                        if (a[p] == s) {
                            mult++;
                            if (!skipped) {
                                skipped = true;
                                continue;
                            }
                        }
                        d += " * y" + std::to_string(a[p]);
                    }
                    o << "            g" << s << " += w" << j << " * ("
                      << (mult > 1 ? lit((double)mult) + " * (" + d + ")" : d) << ");\n";
                }
                if (owned.count(j)) {
                    std::string r = "k" + std::to_string(j);
                    for (int p = 0; p < 3; ++p)
                        if (a[p] >= 0) r += " * y" + std::to_string(a[p]);
                    o << "            if (want_glnk) st_out(&GK[" << j << " * @L@], (" << r << ") * w" << j << ");\n";
                }
            }
            o << "        }\n";
        }
        if (!item.cols.empty()) {
            o << "        if (want_gy) {\n";
            for (int s : item.cols) o << "            st_out(&GY[" << s << " * @L@], g" << s << ");\n";
            o << "        }\n";
        }
        o << "    } break;\n";
    }
    o << "    default: break;\n    }\n}\n";
    return fill(o.str(), pair);
}

std::string generate_module_source(const HostTables &t)
{
    return generate_preamble() + generate_fj_source(t, false) + generate_fj_source(t, true) +
           generate_vjp_source(t, false) + generate_vjp_source(t, true);
}

bool compile_fj_source(const std::string &src, const std::string &arch, std::vector<char> *code, std::string *log)
{
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, src.c_str(), "mcc_fj_generated.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS) {
        *log = "hiprtcCreateProgram failed";
        return false;
    }
    const std::string arch_opt = "--offload-arch=" + arch;
    const char *opts[] = {arch_opt.c_str(), "-O3", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
    const hiprtcResult r = hiprtcCompileProgram(prog, (int)(sizeof opts / sizeof opts[0]), opts);
    size_t n = 0;
    if (hiprtcGetProgramLogSize(prog, &n) == HIPRTC_SUCCESS && n > 1) {
        std::string l(n, '\0');
        if (hiprtcGetProgramLog(prog, &l[0]) == HIPRTC_SUCCESS) *log = l.c_str();
    }
    bool ok = r == HIPRTC_SUCCESS;
    if (!ok && log->empty()) *log = hiprtcGetErrorString(r);
    if (ok) {
        size_t cs = 0;
        ok = hiprtcGetCodeSize(prog, &cs) == HIPRTC_SUCCESS && cs > 0;
        if (ok) {
            code->resize(cs);
            ok = hiprtcGetCode(prog, code->data()) == HIPRTC_SUCCESS;
        }
        if (!ok) *log = "hiprtcGetCode failed";
    }
    hiprtcDestroyProgram(&prog);
    return ok;
}

}  // namespace mcc
