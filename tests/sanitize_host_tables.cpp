// Host-side checks of the mechanism compiler, run under AddressSanitizer
// and UndefinedBehaviorSanitizer by tests/test_sanitizers.py: for every
// dense-tail size a mechanism admits (and for the transposed system of the
// reverse mode), compile the tables, run the host emulation of the solver,
// of the f/J kernel and of the VJP kernel's work items on a seeded state,
// and generate the per-mechanism kernel source.  Exit status 0 when every
// emulation reports no table violation (a sanitizer finding aborts the
// process on its own).
//
// Input: a mechanism file written by the test (int32 N, R, reactant and
// product counts, then the arrays of mcc_mech_desc in order).
#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include <vector>

#include "../paper_2501_00011_amd/csrc/mcc_internal.hpp"

using namespace mcc;

template <class T>
static bool read_n(FILE *f, std::vector<T> &v, size_t n)
{
    v.resize(n);
    return fread(v.data(), sizeof(T), n, f) == n;
}

int main(int argc, char **argv)
{
    if (argc < 2) return 2;
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 2;
    int32_t h[4];
    if (fread(h, sizeof(int32_t), 4, f) != 4) return 2;
    const int N = h[0], R = h[1];
    std::vector<int32_t> rt, rp, ri, pp, pi;
    std::vector<double> py, A, th;
    bool ok = read_n(f, rt, R) && read_n(f, rp, R + 1) && read_n(f, ri, h[2]) && read_n(f, pp, R + 1) &&
              read_n(f, pi, h[3]) && read_n(f, py, h[3]) && read_n(f, A, R) && read_n(f, th, R);
    fclose(f);
    if (!ok) return 2;
    const mcc_mech_desc d{N, R, rt.data(), rp.data(), ri.data(), pp.data(), pi.data(), py.data(), A.data(), th.data()};
    std::mt19937_64 rng(12345);
    std::uniform_real_distribution<double> u(0.5, 2.0);
    std::vector<double> k(R), y(N), b(N), fv(N), x(N);
    for (auto &v : k) v = 1e-3 * u(rng);
    for (auto &v : y) v = u(rng);
    for (auto &v : b) v = u(rng) - 1.25;
    int total = 0;
    for (int tail : {-1, 0, 32, 48, 64}) {
        if (tail > N) continue;
        for (bool transpose : {false, true}) {
            HostTables t;
            std::string err;
            if (compile_mechanism(&d, tail, &t, &err, transpose) != MCC_OK) {
                if (err.find("slots") != std::string::npos) continue;  // does not fit the register slots
                fprintf(stderr, "tail %d: %s\n", tail, err.c_str());
                return 1;
            }
            const int v = emulate_cell(t, k.data(), y.data(), 0.37, b.data(), fv.data(), x.data());
            std::vector<double> ff(N), jac(t.nnz > 0 ? t.nnz : 1);
            const int vf = transpose ? 0 : emulate_fj(t, k.data(), y.data(), ff.data(), jac.data());
            std::vector<double> gy(N), gk(R > 0 ? R : 1);
            const int vv = transpose ? 0 : emulate_vjp(t, k.data(), y.data(), b.data(), gy.data(), gk.data());
            const std::string src = transpose ? std::string() : generate_module_source(t);
            printf("tail %d (built %d)%s: %d solver-table, %d f/J-table and %d VJP-plan violations, source %zu bytes\n",
                   tail, t.M, transpose ? " transposed" : "", v, vf, vv, src.size());
            total += v + vf + vv;
        }
    }
    return total == 0 ? 0 : 1;
}
