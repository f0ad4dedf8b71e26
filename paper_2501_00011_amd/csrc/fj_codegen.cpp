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

// Kernel head: block -> (64-lane tile, work item), the tiles of one XCD
// together.  One-cell variant: lane = cell c_begin + tile * 64 + lane.  Pair
// variant: lane = cells 2c and 2c + 1 with c = tile * 64 + lane, 16-byte
// accesses (the caller guarantees an even ld, 16-byte aligned arrays and
// whole pairs: n_cells even).
std::string head(const char *name, const char *args, const char *ptrs, bool pair)
{
    std::ostringstream o;
    o << "extern \"C\" __global__ __launch_bounds__(64) void " << name << (pair ? "2" : "") << "(\n" << args
      << ", long long n_cells, long long ld, long long c_begin, int item_begin, int n_items, int n_tiles)\n"
      << "{\n"
      << "    const int bid = blockIdx.x, xcd = bid & 7, q = bid >> 3;\n"
      << "    const int item = item_begin + q % n_items, tile = (q / n_items) * 8 + xcd;\n"
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
           "__device__ __forceinline__ d2 &operator+=(d2 &a, d2 b) { a.x += b.x; a.y += b.y; return a; }\n";
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
                    o << "            " << dst << ((flags & kFjAdd) ? " += acc;\n" : " = acc;\n");
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

// Vector-Jacobian products, generated from the same tables.  Work items
// 0 .. n_jitems-1 are the Jacobian-column items of the f/J kernel: each J
// entry (i, s) they form is contracted at once with v_i into a register
// accumulator gy_s (gy = J^T v), stored when the item ends (a column never
// spans two items).  Items n_jitems .. are groups of kVjpRxnGroup reactions:
// glnk_j = r_j * sum_i nu_ij v_i, the derivative of v.f with respect to
// ln k_j (f is linear in each k_j).
std::string generate_vjp_source(const HostTables &t, bool pair)
{
    const int N = t.N, R = t.R;
    std::vector<int> entry_row(t.nnz), entry_col(t.nnz);
    for (int i = 0; i < N; ++i)
        for (int e = t.row_ptr[i]; e < t.row_ptr[i + 1]; ++e) {
            entry_row[e] = i;
            entry_col[e] = t.col_idx[e];
        }
    std::ostringstream o;
    o << head("mcc_vjp_generated",
              "    const double *__restrict__ y, const double *__restrict__ k, const double *__restrict__ v,\n"
              "    double *__restrict__ gy, double *__restrict__ glnk",
              "    const @V@ *__restrict__ Y = (const @V@ *)y + c;\n"
              "    const @V@ *__restrict__ K = (const @V@ *)k + c;\n"
              "    const @V@ *__restrict__ V = (const @V@ *)v + c;\n"
              "    @V@ *__restrict__ GY = (@V@ *)gy + c;\n"
              "    @V@ *__restrict__ GK = (@V@ *)glnk + c;\n",
              pair)
      << "    switch (item) {\n";

    int case_no = 0;
    for (int it = t.n_fitems; it < t.n_fitems + t.n_jitems; ++it, ++case_no) {
        o << "    case " << case_no << ": {\n";
        std::set<int> ys, ks, vs, cols;
        for (int ci = t.fj_items[it]; ci < t.fj_items[it + 1]; ++ci) {
            const FjChunk &ch = t.fj_chunks[ci];
            for (int qm = 0; qm < ch.n_mono; ++qm) {
                const FjMono &m = t.fj_monos[ch.mono_begin + qm];
                if (m.j >= 0) ks.insert(m.j);
                for (int f3 : {m.a, m.b, m.c})
                    if (f3 >= 0) ys.insert(f3);
            }
            for (int r = 0; r < ch.n_rec; ++r) {
                const FjRec &rec = t.fj_recs[ch.rec_begin + r];
                const uint32_t flags = rec.meta >> 24, row = rec.meta & kFjRowMask;
                if ((flags & kFjStore) && row >= (uint32_t)N) {
                    vs.insert(entry_row[row - N]);
                    cols.insert(entry_col[row - N]);
                }
            }
        }
        for (int j : ks) o << "        const @V@ k" << j << " = K[" << j << " * @L@];\n";
        for (int r : ys) o << "        const @V@ y" << r << " = Y[" << r << " * @L@];\n";
        for (int r : vs) o << "        const @V@ v" << r << " = V[" << r << " * @L@];\n";
        for (int sc : cols) o << "        @V@ g" << sc << " = @Z@;\n";
        for (int ci = t.fj_items[it]; ci < t.fj_items[it + 1]; ++ci) {
            const FjChunk &ch = t.fj_chunks[ci];
            o << "        {\n";
            std::vector<std::string> mono(kFjQmax);
            for (int qm = 0; qm < ch.n_mono; ++qm) {
                const FjMono &m = t.fj_monos[ch.mono_begin + qm];
                if (m.j < 0 && m.a < 0 && m.b < 0 && m.c < 0) continue;
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
                if (!(flags & (kFjKeep | kFjStore)) && sum == "@Z@") continue;
                o << "            acc " << ((flags & kFjKeep) ? "+=" : "=") << " " << sum << ";\n";
                if ((flags & kFjStore) && row >= (uint32_t)N) {
                    const int e = (int)row - N;
                    o << "            g" << entry_col[e] << " += v" << entry_row[e] << " * acc;\n";
                }
            }
            o << "            (void)acc;\n        }\n";
        }
        for (int sc : cols) o << "        GY[" << sc << " * @L@] = g" << sc << ";\n";
        o << "    } break;\n";
    }
    for (int j0 = 0; j0 < R; j0 += kVjpRxnGroup, ++case_no) {
        const int j1 = std::min(R, j0 + kVjpRxnGroup);
        o << "    case " << case_no << ": {\n";
        std::set<int> ys, vs;
        for (int j = j0; j < j1; ++j) {
            for (int q = 0; q < 3; ++q)
                if (t.rx_sp[3 * j + q] >= 0) ys.insert(t.rx_sp[3 * j + q]);
            for (int e = t.nu_ptr[j]; e < t.nu_ptr[j + 1]; ++e) vs.insert(t.nu_sp[e]);
        }
        for (int r : ys) o << "        const @V@ y" << r << " = Y[" << r << " * @L@];\n";
        for (int r : vs) o << "        const @V@ v" << r << " = V[" << r << " * @L@];\n";
        for (int j = j0; j < j1; ++j) {
            std::string rate = "K[" + std::to_string(j) + " * @L@]";
            for (int q = 0; q < 3; ++q)
                if (t.rx_sp[3 * j + q] >= 0) rate += " * y" + std::to_string(t.rx_sp[3 * j + q]);
            std::string w;
            for (int e = t.nu_ptr[j]; e < t.nu_ptr[j + 1]; ++e)
                w += (w.empty() ? "" : " + ") + lit(t.nu_coef[e]) + " * v" + std::to_string(t.nu_sp[e]);
            if (w.empty()) w = "@Z@";
            o << "        GK[" << j << " * @L@] = (" << rate << ") * (" << w << ");\n";
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
