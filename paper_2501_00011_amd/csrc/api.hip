// C ABI of libmcchem (declared in include/mcc.h): handles, argument checks,
// table upload and kernel launches.  All arithmetic happens in the kernels.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>

#include "mcc_internal.hpp"

using namespace mcc;

struct mcc_mech {
    HostTables t;
    HostTables ta;  // solver tables of the transposed system I - c J^T (reverse mode)
    int device = 0;
    void *dev_buf = nullptr;  // every device table, sub-allocated
    // device views
    const int32_t *rxn_type = nullptr;
    const FjMono *fj_monos = nullptr;
    const FjRec *fj_recs = nullptr;
    const FjChunk *fj_chunks = nullptr;
    const int32_t *fj_items = nullptr;
    const int32_t *paper_rec = nullptr, *paper_rec_inv = nullptr;
    const double *paper_yld = nullptr, *paper_yld_inv = nullptr;
    const double *A = nullptr, *theta = nullptr;
    const int32_t *vspecies = nullptr, *rx_reac = nullptr, *part = nullptr;
    const Op16 *fg_ops = nullptr, *nm_ops = nullptr;
    const uint64_t *lu_ops = nullptr;
    const uint16_t *fwd_map = nullptr, *bwd_map = nullptr;
    const uint16_t *schur_tab = nullptr;
    int32_t off_y = 0, off_k = 0, off_r = 0, off_p = 0, off_lu = 0, off_tm = 0, lds_doubles = 0;
    int live_batches = 0;
    int solve_waves = 0;  // wavefronts per SIMD of the solver build launched
    // mechanism-specialised f/J kernel, compiled on first use
    int fj_kind = MCC_FJ_GENERATED;
    std::string arch;
    hipModule_t fj_mod = nullptr;
    hipFunction_t fj_fn = nullptr, fj2_fn = nullptr, vjp_fn = nullptr, vjp2_fn = nullptr;
    // reverse mode: the transposed solver tables on the device and their LDS layout
    struct {
        const int32_t *vspecies = nullptr, *rx_reac = nullptr, *part = nullptr;
        const int32_t *nu_ptr = nullptr, *nu_vid = nullptr;
        const double *nu_coef = nullptr;
        const Op16 *fg_ops = nullptr, *nm_ops = nullptr;
        const uint64_t *lu_ops = nullptr;
        const uint16_t *fwd_map = nullptr, *bwd_map = nullptr;
        const uint16_t *schur_tab = nullptr;
        int32_t off_y = 0, off_k = 0, off_r = 0, off_lu = 0, off_tm = 0, off_w = 0, lds_doubles = 0;
        std::string unavailable;  // empty: the reverse-mode kernel runs for this mechanism
    } adj;
};

struct mcc_cells {
    mcc_mech *mech = nullptr;
    int64_t n_cells = 0, ld = 0;
    double *k = nullptr;
    double *ones = nullptr;  // [ld] of 1.0: the factor of a missing reactant
    bool bound = false;
    // per-launch solver form: state between launches, count of unfinished cells
    double *state = nullptr;
    int64_t state_doubles = 0;
    int32_t *pending = nullptr;
    int32_t *pending_host = nullptr;  // pinned
    int32_t call_id = 0;
    double *mc_slots = nullptr;  // Multi-cells reduction slots [2][mc_cells]
    int64_t mc_cells = 0;
    int32_t *order = nullptr;    // the solver's cell schedule (device [n_cells]), or null
};

namespace {

thread_local std::string g_last_error;

mcc_status set_error(mcc_status s, const std::string &msg)
{
    g_last_error = msg;
    return s;
}

mcc_status ok()
{
    g_last_error.clear();
    return MCC_OK;
}

mcc_status hip_error(hipError_t e, const char *what)
{
    return set_error(e == hipErrorOutOfMemory ? MCC_ERR_OOM : MCC_ERR_DEVICE,
                     std::string(what) + ": " + hipGetErrorString(e));
}

// Appends host vectors to one device buffer at 256-byte aligned offsets.
struct Packer {
    std::vector<char> bytes;
    template <class T>
    size_t add(const std::vector<T> &v)
    {
        size_t off = (bytes.size() + 255) & ~size_t(255);
        bytes.resize(off + std::max<size_t>(v.size() * sizeof(T), 8), 0);
        if (!v.empty()) std::memcpy(bytes.data() + off, v.data(), v.size() * sizeof(T));
        return off;
    }
};

class DeviceGuard {
  public:
    explicit DeviceGuard(int dev) : ok_(hipGetDevice(&prev_) == hipSuccess)
    {
        if (ok_ && prev_ != dev) ok_ = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (hipGetDevice(&cur) == hipSuccess && cur != prev_) (void)hipSetDevice(prev_);
    }
    bool ok() const { return ok_; }

  private:
    int prev_ = 0;
    bool ok_;
};

}  // namespace

extern "C" {

const char *mcc_last_error(void) { return g_last_error.c_str(); }

const char *mcc_version(void) { return "mcchem 0.1 (gfx950, fp64)"; }

mcc_status mcc_solver_opts_default(mcc_solver_opts *o)
{
    if (!o) return set_error(MCC_ERR_INVALID_ARG, "opts is null");
    o->rtol = 1e-8;
    o->atol = 1.0;
    o->eta_newton = 0.03;
    o->safety = 0.9;
    o->fac_min = 0.2;
    o->fac_max = 10.0;
    o->fac_newton_fail = 0.5;
    o->h_min_rel = 1e-30;
    o->max_order = 5;
    o->max_newton = 4;
    o->max_steps = 100000;
    o->steps_per_launch = 0;
    o->warm_start = 0;
    return ok();
}

mcc_status mcc_mech_config_default(mcc_mech_config *cfg)
{
    if (!cfg) return set_error(MCC_ERR_INVALID_ARG, "cfg is null");
    std::memset(cfg, 0, sizeof(*cfg));
    cfg->dense_tail = -1;
    return ok();
}

mcc_status mcc_mech_create(const mcc_mech_desc *desc, int device, mcc_mech **out)
{
    return mcc_mech_create_ex(desc, device, nullptr, out);
}

mcc_status mcc_mech_create_ex(const mcc_mech_desc *desc, int device, const mcc_mech_config *cfg, mcc_mech **out)
{
    if (!desc || !out) return set_error(MCC_ERR_INVALID_ARG, "desc and out must not be null");
    *out = nullptr;
    if (device < -1) return set_error(MCC_ERR_INVALID_ARG, "device index out of range");
    mcc_mech_config c;
    if (cfg)
        c = *cfg;
    else
        mcc_mech_config_default(&c);

    mcc_mech *m = new (std::nothrow) mcc_mech;
    if (!m) return set_error(MCC_ERR_OOM, "host allocation failed");
    std::string err;
    if (c.waves_per_simd < 0 || c.waves_per_simd > 2) {
        delete m;
        return set_error(MCC_ERR_INVALID_ARG, "waves_per_simd must be 0, 1 or 2");
    }
    mcc_status st = compile_mechanism(desc, c.dense_tail, &m->t, &err);
    if (st == MCC_OK) st = compile_mechanism(desc, c.dense_tail, &m->ta, &err, true);
    if (st != MCC_OK) {
        delete m;
        return set_error(st, err);
    }
    HostTables &t = m->t;
    m->device = device;
    m->solve_waves = c.waves_per_simd ? c.waves_per_simd : solve_default_waves(t.NS, t.M);
    if (!solve_waves_available(t.NS, t.M, m->solve_waves)) {
        const std::string why = "no solver build for " + std::to_string(m->solve_waves) + " wavefronts per SIMD with " +
                                std::to_string(t.NS) + " species slots and a dense tail of " + std::to_string(t.M);
        delete m;
        return set_error(MCC_ERR_INVALID_ARG, why);
    }

    // LDS layout of one solver cell (doubles): the compact state (N + 1),
    // k, one scratch region for the rates (f), the rate partials (Newton
    // matrix) and the re-sampling matrix -- never live together -- and the LU.
    constexpr int kTm = (kMaxOrder + 1) * (kMaxOrder + 1);
    m->off_y = 0;
    m->off_k = t.N + 1;
    m->off_r = m->off_k + t.R;
    m->off_p = m->off_r;
    m->off_tm = m->off_r;
    m->off_lu = m->off_r + std::max({t.R + 1, t.n_partials + 1, kTm});
    m->lds_doubles = m->off_lu + t.lu_nnz + 2;
    {
        // reverse mode: the same regions for the transposed tables, then R + 1 scratch values
        const HostTables &a = m->ta;
        auto &d = m->adj;
        d.off_y = 0;
        d.off_k = a.N + 1;
        d.off_r = d.off_k + a.R;
        d.off_tm = d.off_r;
        d.off_lu = d.off_r + std::max({a.R + 1, a.n_partials + 1, kTm});
        // the R + 1 scratch values of the start entry, the last one reversed:
        // no factorisation follows, so they may take the LU storage
        d.off_w = a.lu_nnz + 2 >= a.R + 1 ? d.off_lu : d.off_lu + a.lu_nnz + 2;
        d.lds_doubles = std::max(d.off_lu + a.lu_nnz + 2, d.off_w + a.R + 1);
        if (!adjoint_shape_supported(a.NS, a.M))
            d.unavailable = "no reverse-mode kernel for " + std::to_string(a.NS) + " species slots with a dense tail of " +
                            std::to_string(a.M);
        else if (a.R > kAdjMaxR)
            d.unavailable = "the reverse-mode kernel handles at most " + std::to_string(kAdjMaxR) + " reactions";
    }
    if (device == -1) {  // host-only: validated and compiled, nothing uploaded
        *out = m;
        return ok();
    }

    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess) {
        delete m;
        return hip_error(e, "hipGetDeviceCount");
    }
    if (device >= ndev) {
        delete m;
        return set_error(MCC_ERR_INVALID_ARG, "device index out of range");
    }
    DeviceGuard g(device);
    if (!g.ok()) {
        delete m;
        return set_error(MCC_ERR_DEVICE, "cannot select device");
    }
    {
        hipDeviceProp_t prop;
        e = hipGetDeviceProperties(&prop, device);
        if (e != hipSuccess) {
            delete m;
            return hip_error(e, "hipGetDeviceProperties");
        }
        m->arch = prop.gcnArchName;
    }
    // Device limits (Section 3: checked at run time rather than assumed).
    int max_lds = 0;
    e = hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device);
    if (e != hipSuccess) {
        delete m;
        return hip_error(e, "hipDeviceGetAttribute");
    }
    const size_t lds_bytes = (size_t)m->lds_doubles * sizeof(double);
    if (lds_bytes > (size_t)max_lds) {
        delete m;
        return set_error(MCC_ERR_MECH, "solver state of one cell needs " + std::to_string(lds_bytes) +
                                           " bytes of LDS; the device allows " + std::to_string(max_lds));
    }
    if ((e = prepare_solve_kernels(max_lds)) != hipSuccess) {
        delete m;
        return hip_error(e, "hipFuncSetAttribute");
    }
    if (m->adj.unavailable.empty() && (size_t)m->adj.lds_doubles * sizeof(double) > (size_t)max_lds)
        m->adj.unavailable = "the reverse-mode state of one cell needs " +
                             std::to_string((size_t)m->adj.lds_doubles * sizeof(double)) + " bytes of LDS";
    if (m->adj.unavailable.empty() && (e = prepare_adjoint_kernels(max_lds)) != hipSuccess) {
        if (e == hipErrorInvalidDeviceFunction) {
            // a two-wavefront reverse-mode build that spills is not trusted
            m->adj.unavailable = "the reverse-mode kernel was built with spilled registers";
        } else {
            delete m;
            return hip_error(e, "hipFuncSetAttribute");
        }
    }

    Packer pk;
    const size_t o_rxn = pk.add(t.rxn_type), o_A = pk.add(t.A), o_th = pk.add(t.theta);
    const size_t o_monos = pk.add(t.fj_monos), o_recs = pk.add(t.fj_recs);
    const size_t o_chunks = pk.add(t.fj_chunks), o_items = pk.add(t.fj_items);
    const size_t o_prec = pk.add(t.paper_rec), o_pyld = pk.add(t.paper_yld);
    const size_t o_preci = pk.add(t.paper_rec_inv), o_pyldi = pk.add(t.paper_yld_inv);
    const size_t o_perm = pk.add(t.vspecies), o_rxr = pk.add(t.rx_reac), o_part = pk.add(t.part);
    const size_t o_fg = pk.add(t.fg_ops), o_nm = pk.add(t.nm_ops), o_lu = pk.add(t.lu_ops);
    const size_t o_fwd = pk.add(t.fwd_map), o_bwd = pk.add(t.bwd_map), o_sch = pk.add(t.schur_tab);
    const HostTables &ta = m->ta;
    const size_t oa_perm = pk.add(ta.vspecies), oa_rxr = pk.add(ta.rx_reac), oa_part = pk.add(ta.part);
    const size_t oa_fg = pk.add(ta.fg_ops), oa_nm = pk.add(ta.nm_ops), oa_lu = pk.add(ta.lu_ops);
    const size_t oa_fwd = pk.add(ta.fwd_map), oa_bwd = pk.add(ta.bwd_map), oa_sch = pk.add(ta.schur_tab);
    const size_t oa_nup = pk.add(ta.nu_ptr), oa_nuv = pk.add(ta.nu_vid), oa_nuc = pk.add(ta.nu_coef);
    if ((e = hipMalloc(&m->dev_buf, pk.bytes.size())) != hipSuccess) {
        delete m;
        return hip_error(e, "hipMalloc (mechanism tables)");
    }
    if ((e = hipMemcpy(m->dev_buf, pk.bytes.data(), pk.bytes.size(), hipMemcpyHostToDevice)) != hipSuccess) {
        (void)hipFree(m->dev_buf);
        delete m;
        return hip_error(e, "hipMemcpy (mechanism tables)");
    }
    char *b = static_cast<char *>(m->dev_buf);
    m->rxn_type = (const int32_t *)(b + o_rxn);
    m->A = (const double *)(b + o_A);
    m->theta = (const double *)(b + o_th);
    m->fj_monos = (const FjMono *)(b + o_monos);
    m->fj_recs = (const FjRec *)(b + o_recs);
    m->fj_chunks = (const FjChunk *)(b + o_chunks);
    m->fj_items = (const int32_t *)(b + o_items);
    m->paper_rec = (const int32_t *)(b + o_prec);
    m->paper_yld = (const double *)(b + o_pyld);
    m->paper_rec_inv = (const int32_t *)(b + o_preci);
    m->paper_yld_inv = (const double *)(b + o_pyldi);

    m->vspecies = (const int32_t *)(b + o_perm);
    m->rx_reac = (const int32_t *)(b + o_rxr);
    m->part = (const int32_t *)(b + o_part);
    m->fg_ops = (const Op16 *)(b + o_fg);
    m->nm_ops = (const Op16 *)(b + o_nm);
    m->lu_ops = (const uint64_t *)(b + o_lu);
    m->fwd_map = (const uint16_t *)(b + o_fwd);
    m->bwd_map = (const uint16_t *)(b + o_bwd);
    m->schur_tab = (const uint16_t *)(b + o_sch);
    m->adj.vspecies = (const int32_t *)(b + oa_perm);
    m->adj.rx_reac = (const int32_t *)(b + oa_rxr);
    m->adj.part = (const int32_t *)(b + oa_part);
    m->adj.fg_ops = (const Op16 *)(b + oa_fg);
    m->adj.nm_ops = (const Op16 *)(b + oa_nm);
    m->adj.lu_ops = (const uint64_t *)(b + oa_lu);
    m->adj.fwd_map = (const uint16_t *)(b + oa_fwd);
    m->adj.bwd_map = (const uint16_t *)(b + oa_bwd);
    m->adj.schur_tab = (const uint16_t *)(b + oa_sch);
    m->adj.nu_ptr = (const int32_t *)(b + oa_nup);
    m->adj.nu_vid = (const int32_t *)(b + oa_nuv);
    m->adj.nu_coef = (const double *)(b + oa_nuc);
    *out = m;
    return ok();
}

mcc_status mcc_mech_info(const mcc_mech *m, int32_t *n_species, int32_t *n_reactions, int32_t *nnz,
                         int32_t *lu_nnz, int32_t *solver_lds_bytes)
{
    if (!m) return set_error(MCC_ERR_INVALID_ARG, "mech is null");
    if (n_species) *n_species = m->t.N;
    if (n_reactions) *n_reactions = m->t.R;
    if (nnz) *nnz = m->t.nnz;
    if (lu_nnz) *lu_nnz = m->t.lu_nnz;
    if (solver_lds_bytes) *solver_lds_bytes = m->lds_doubles * (int32_t)sizeof(double);
    return ok();
}

mcc_status mcc_mech_op_counts(const mcc_mech *m, mcc_op_counts *counts)
{
    if (!m || !counts) return set_error(MCC_ERR_INVALID_ARG, "null argument");
    *counts = m->t.counts;
    return ok();
}

mcc_status mcc_debug_emulate_cell(const mcc_mech *m, const double *k, const double *y, double c, const double *b,
                                  double *f, double *x, int32_t *violations)
{
    if (!m || (!k && m->t.R > 0) || !y || !b || !f || !x || !violations)
        return set_error(MCC_ERR_INVALID_ARG, "null argument");
    *violations = emulate_cell(m->t, k, y, c, b, f, x);
    return ok();
}

mcc_status mcc_debug_emulate_cell_adjoint(const mcc_mech *m, const double *k, const double *y, double c,
                                          const double *b, double *f, double *x, int32_t *violations)
{
    if (!m || (!k && m->ta.R > 0) || !y || !b || !f || !x || !violations)
        return set_error(MCC_ERR_INVALID_ARG, "null argument");
    *violations = emulate_cell(m->ta, k, y, c, b, f, x);
    return ok();
}

mcc_status mcc_debug_emulate_fj(const mcc_mech *m, const double *k, const double *y, double *f, double *jac,
                                int32_t *violations)
{
    if (!m || (!k && m->t.R > 0) || !y || !f || !jac || !violations)
        return set_error(MCC_ERR_INVALID_ARG, "null argument");
    *violations = emulate_fj(m->t, k, y, f, jac);
    return ok();
}

mcc_status mcc_debug_emulate_vjp(const mcc_mech *m, const double *k, const double *y, const double *v, double *gy,
                                 double *glnk, int32_t *violations)
{
    if (!m || (!k && m->t.R > 0) || !y || !v || !gy || (!glnk && m->t.R > 0) || !violations)
        return set_error(MCC_ERR_INVALID_ARG, "null argument");
    *violations = emulate_vjp(m->t, k, y, v, gy, glnk);
    return ok();
}

mcc_status mcc_debug_schedule_info(const mcc_mech *m, int64_t *out)
{
    if (!m || !out) return set_error(MCC_ERR_INVALID_ARG, "null argument");
    out[0] = m->t.lu_blocks;
    out[1] = m->t.lu_steps;
    out[2] = m->t.nm_blocks;
    for (int q = 0; q < 4; ++q) out[3 + q] = q < m->t.NS ? m->t.fg_blocks[q] : 0;
    out[7] = m->t.M;
    out[8] = m->solve_waves;
    return ok();
}

mcc_status mcc_mech_jac_pattern(const mcc_mech *m, int32_t *row_ptr, int32_t *col_idx)
{
    if (!m || !row_ptr || !col_idx) return set_error(MCC_ERR_INVALID_ARG, "null argument");
    std::memcpy(row_ptr, m->t.row_ptr.data(), m->t.row_ptr.size() * sizeof(int32_t));
    std::memcpy(col_idx, m->t.col_idx.data(), m->t.col_idx.size() * sizeof(int32_t));
    return ok();
}

mcc_status mcc_mech_destroy(mcc_mech *m)
{
    if (!m) return ok();
    if (m->live_batches > 0) return set_error(MCC_ERR_STATE, "cell batches created from this mechanism are alive");
    if (m->device < 0) {
        delete m;
        return ok();
    }
    DeviceGuard g(m->device);
    if (m->fj_mod) {
        hipError_t e = hipModuleUnload(m->fj_mod);
        if (e != hipSuccess) return hip_error(e, "hipModuleUnload");
        m->fj_mod = nullptr;
        m->fj_fn = m->fj2_fn = m->vjp_fn = m->vjp2_fn = nullptr;
    }
    if (m->dev_buf) {
        hipError_t e = hipFree(m->dev_buf);
        if (e != hipSuccess) return hip_error(e, "hipFree");
    }
    delete m;
    return ok();
}

mcc_status mcc_mech_set_fj_kernel(mcc_mech *m, int32_t kind)
{
    if (!m) return set_error(MCC_ERR_INVALID_ARG, "mech is null");
    if (kind != MCC_FJ_GENERATED && kind != MCC_FJ_TABLES) return set_error(MCC_ERR_INVALID_ARG, "unknown f/J kernel kind");
    m->fj_kind = kind;
    return ok();
}

mcc_status mcc_debug_fj_source(const mcc_mech *m, char *buf, int64_t cap, int64_t *len)
{
    if (!m || !len || (cap > 0 && !buf) || cap < 0) return set_error(MCC_ERR_INVALID_ARG, "bad argument");
    const std::string src = generate_module_source(m->t);
    *len = (int64_t)src.size();
    if (cap > 0) {
        const size_t n = std::min((size_t)cap, src.size() + 1);
        std::memcpy(buf, src.c_str(), n);
    }
    return ok();
}

mcc_status mcc_debug_compile_fj(const mcc_mech *m, const char *arch, int64_t *code_bytes)
{
    if (!m || !arch || !code_bytes) return set_error(MCC_ERR_INVALID_ARG, "null argument");
    std::vector<char> code;
    std::string log;
    if (!compile_fj_source(generate_module_source(m->t), arch, &code, &log))
        return set_error(MCC_ERR_DEVICE, "generated f/J kernel does not compile: " + log);
    *code_bytes = (int64_t)code.size();
    return ok();
}

mcc_status mcc_cells_create(const mcc_mech *mech, int64_t n_cells, int64_t ld, mcc_cells **out)
{
    if (!mech || !out) return set_error(MCC_ERR_INVALID_ARG, "mech and out must not be null");
    *out = nullptr;
    if (n_cells < 0 || ld < n_cells) return set_error(MCC_ERR_INVALID_ARG, "need 0 <= n_cells <= ld");
    if (n_cells > 0x7fffffff) return set_error(MCC_ERR_INVALID_ARG, "n_cells exceeds 2^31-1");
    if (mech->device < 0) return set_error(MCC_ERR_STATE, "mechanism was compiled host-only (device -1)");
    mcc_cells *c = new (std::nothrow) mcc_cells;
    if (!c) return set_error(MCC_ERR_OOM, "host allocation failed");
    c->mech = const_cast<mcc_mech *>(mech);
    c->n_cells = n_cells;
    c->ld = ld;
    DeviceGuard g(mech->device);
    const size_t kbytes = (size_t)mech->t.R * (size_t)ld * sizeof(double);
    if (kbytes > 0) {
        hipError_t e = hipMalloc(&c->k, kbytes);
        if (e != hipSuccess) {
            delete c;
            return hip_error(e, "hipMalloc (rate constants)");
        }
    }
    if (ld > 0) {
        hipError_t e = hipMalloc(&c->ones, (size_t)ld * sizeof(double));
        if (e == hipSuccess) {
            std::vector<double> h((size_t)ld, 1.0);
            e = hipMemcpy(c->ones, h.data(), (size_t)ld * sizeof(double), hipMemcpyHostToDevice);
        }
        if (e != hipSuccess) {
            if (c->k) (void)hipFree(c->k);
            if (c->ones) (void)hipFree(c->ones);
            delete c;
            return hip_error(e, "ones row");
        }
    }
    c->mech->live_batches++;
    *out = c;
    return ok();
}

mcc_status mcc_cells_bind(mcc_cells *c, const double *T, const double *P, const double *jscale, void *stream)
{
    (void)P;  // reserved: no current reaction type depends on pressure
    if (!c) return set_error(MCC_ERR_INVALID_ARG, "cells is null");
    if (c->n_cells > 0 && !T) return set_error(MCC_ERR_INVALID_ARG, "T is null");
    DeviceGuard g(c->mech->device);
    RatesParams p{};
    p.rxn_type = c->mech->rxn_type;
    p.A = c->mech->A;
    p.theta = c->mech->theta;
    p.T = T;
    p.jscale = jscale;
    p.k = c->k;
    p.n_cells = c->n_cells;
    p.ld = c->ld;
    p.R = c->mech->t.R;
    hipError_t e = launch_rates(p, (hipStream_t)stream);
    if (e != hipSuccess) return hip_error(e, "rates kernel launch");
    c->bound = true;
    return ok();
}

mcc_status mcc_cells_rate_constants(const mcc_cells *c, const double **k)
{
    if (!c || !k) return set_error(MCC_ERR_INVALID_ARG, "null argument");
    *k = c->k;
    return ok();
}

static bool aligned16(const void *p) { return p == nullptr || ((uintptr_t)p & 15) == 0; }

// Memory-side cache of the MI355X (Infinity Cache), bytes.
constexpr int64_t kMallBytes = (int64_t)256 << 20;

// Launches a generated kernel over cells [0, n_cells): the two-cell variant
// (fn2) over whole pairs when ld is even and every array is 16-byte aligned,
// the one-cell variant (fn) over the rest.  arrays: the kernel's pointer
// arguments in order (null allowed for an unused output).  in_rows: input
// rows the kernel reads per cell; stream_grp: grp_tiles (see the generated
// kernel head) once the inputs exceed the memory-side cache.  While the
// inputs fit in that cache the items of a tile run together (grp_tiles 1:
// one fetch per tile, later items hit the XCD's L2).  Beyond it the f/J
// kernel, whose reads are a fifth of its traffic, runs each item over 128
// consecutive tiles at once (16) so that the first reads of every row are
// long runs: 55% of HBM peak instead of 44% at 200,000 cells of 72 species;
// the VJP kernel, mostly reads, keeps 1 (its items then reuse the XCD's L2;
// 16 measured slower).
static mcc_status launch_generated(hipFunction_t fn, hipFunction_t fn2, std::vector<const void *> arrays,
                                   int64_t n_cells, int64_t ld, int item_begin, int n_items, int in_rows,
                                   int stream_grp, void *stream)
{
    if (n_items == 0 || n_cells == 0) return ok();
    bool pair = ld % 2 == 0;
    for (const void *a : arrays) pair = pair && aligned16(a);
    const int64_t n_pair_cells = pair ? n_cells / 2 * 2 : 0;
    const bool streaming = 8 * (int64_t)in_rows * n_cells > kMallBytes;
    auto go = [&](hipFunction_t f, int64_t lanes, int64_t c_begin, int64_t n_end) -> mcc_status {
        if (lanes <= 0) return ok();
        const int64_t n_tiles = (lanes + 63) / 64;
        const int grp = streaming ? (int)std::max<int64_t>(1, std::min<int64_t>(stream_grp, (n_tiles + 7) / 8)) : 1;
        const int64_t blocks = (n_tiles + 8 * grp - 1) / (8 * grp) * 8 * grp * n_items;
        if (blocks > 0x7fffffff) return set_error(MCC_ERR_INVALID_ARG, "too many cells for one launch");
        std::vector<void *> args;
        for (const void *&a : arrays) args.push_back((void *)&a);
        long long nc = n_end, ldl = ld, cb = c_begin;
        int ib = item_begin, ni = n_items, nt = (int)n_tiles, gt = grp;
        for (void *a : {(void *)&nc, (void *)&ldl, (void *)&cb, (void *)&ib, (void *)&ni, (void *)&nt, (void *)&gt})
            args.push_back(a);
        hipError_t e = hipModuleLaunchKernel(f, (unsigned)blocks, 1, 1, 64, 1, 1, 0, (hipStream_t)stream, args.data(),
                                             nullptr);
        if (e != hipSuccess) return hip_error(e, "generated kernel launch");
        return ok();
    };
    mcc_status st = go(fn2, n_pair_cells / 2, 0, n_pair_cells);
    if (st != MCC_OK) return st;
    return go(fn, n_cells - n_pair_cells, n_pair_cells, n_cells);
}

// Code objects of generated kernels, compiled once per process for each
// (architecture, source): mechanisms created again reuse them (a compile
// takes seconds; loading a module, microseconds).
static bool cached_code(const std::string &src, const std::string &arch, const std::vector<char> **code,
                        std::string *log)
{
    static std::mutex mu;
    static std::map<std::string, std::vector<char>> cache;
    const std::string key = arch + '\n' + src;
    {
        std::lock_guard<std::mutex> g(mu);
        auto it = cache.find(key);
        if (it != cache.end()) {
            *code = &it->second;
            return true;
        }
    }
    std::vector<char> obj;
    if (!compile_fj_source(src, arch, &obj, log)) return false;
    std::lock_guard<std::mutex> g(mu);
    auto ins = cache.emplace(key, std::move(obj));  // map nodes never move: the pointer stays valid
    *code = &ins.first->second;
    return true;
}

// Generates, compiles (hipRTC) and loads the mechanism's f/J kernel once.
static mcc_status ensure_fj_module(mcc_mech *m)
{
    if (m->fj_fn) return ok();
    const std::vector<char> *code = nullptr;
    std::string log;
    if (!cached_code(generate_module_source(m->t), m->arch, &code, &log))
        return set_error(MCC_ERR_DEVICE, "generated f/J kernel does not compile: " + log);
    hipError_t e = hipModuleLoadData(&m->fj_mod, code->data());
    if (e != hipSuccess) {
        m->fj_mod = nullptr;
        return hip_error(e, "hipModuleLoadData (generated f/J kernel)");
    }
    e = hipModuleGetFunction(&m->fj_fn, m->fj_mod, "mcc_fj_generated");
    if (e == hipSuccess) e = hipModuleGetFunction(&m->fj2_fn, m->fj_mod, "mcc_fj_generated2");
    if (e == hipSuccess) e = hipModuleGetFunction(&m->vjp_fn, m->fj_mod, "mcc_vjp_generated");
    if (e == hipSuccess) e = hipModuleGetFunction(&m->vjp2_fn, m->fj_mod, "mcc_vjp_generated2");
    if (e != hipSuccess) {
        (void)hipModuleUnload(m->fj_mod);
        m->fj_mod = nullptr;
        m->fj_fn = m->fj2_fn = m->vjp_fn = m->vjp2_fn = nullptr;
        return hip_error(e, "hipModuleGetFunction (generated f/J kernel)");
    }
    return ok();
}

static mcc_status run_fj(const mcc_cells *c, const double *y, double *f, double *jac, void *stream)
{
    if (!c) return set_error(MCC_ERR_INVALID_ARG, "cells is null");
    if (!c->bound) return set_error(MCC_ERR_STATE, "mcc_cells_bind has not been called");
    if (c->n_cells == 0) return ok();
    if (!y) return set_error(MCC_ERR_INVALID_ARG, "y is null");
    const HostTables &t = c->mech->t;
    DeviceGuard g(c->mech->device);
    FJParams p{};
    p.monos = c->mech->fj_monos;
    p.recs = c->mech->fj_recs;
    p.chunks = c->mech->fj_chunks;
    p.items = c->mech->fj_items;
    p.y = y;
    p.k = c->k;
    p.ones = c->ones;
    p.f = f;
    p.jac = jac;
    p.n_cells = c->n_cells;
    p.ld = c->ld;
    p.N = t.N;
    p.n_tiles = (int)((c->n_cells + 63) / 64);
    if (f && jac) {
        p.item_begin = 0;
        p.n_items = t.n_fitems + t.n_jitems;
    } else if (f) {
        p.item_begin = 0;
        p.n_items = t.n_fitems;
    } else {
        p.item_begin = t.n_fitems;
        p.n_items = t.n_jitems;
    }
    if (c->mech->fj_kind == MCC_FJ_TABLES) {
        hipError_t e = launch_fj(p, (hipStream_t)stream);
        if (e != hipSuccess) return hip_error(e, "f/J kernel launch");
        return ok();
    }
    mcc_status st = ensure_fj_module(c->mech);
    if (st != MCC_OK) return st;
    return launch_generated(c->mech->fj_fn, c->mech->fj2_fn, {p.y, p.k, p.f, p.jac}, p.n_cells, p.ld, p.item_begin,
                            p.n_items, t.N + t.R, 16, stream);
}

mcc_status mcc_calc_vjp(const mcc_cells *c, const double *y, const double *v, double *gy, double *glnk,
                        void *stream)
{
    if (!c) return set_error(MCC_ERR_INVALID_ARG, "cells is null");
    if (!c->bound) return set_error(MCC_ERR_STATE, "the batch has no rate constants yet");
    if (c->n_cells == 0) return ok();
    if (!y || !v) return set_error(MCC_ERR_INVALID_ARG, "y and v must not be null");
    if (!gy && !glnk) return set_error(MCC_ERR_INVALID_ARG, "gy and glnk are both null");
    const HostTables &t = c->mech->t;
    DeviceGuard g(c->mech->device);
    mcc_status st = ensure_fj_module(c->mech);
    if (st != MCC_OK) return st;
    return launch_generated(c->mech->vjp_fn, c->mech->vjp2_fn, {y, c->k, v, gy, glnk}, c->n_cells, c->ld, 0,
                            (int)t.vjp_items.size(), 2 * t.N + t.R, 1, stream);
}

mcc_status mcc_ablation_paper_deriv(const mcc_mech *m, int64_t n_cells, const double *y, const double *k,
                                    double *f, int32_t inverted, void *stream)
{
    if (!m) return set_error(MCC_ERR_INVALID_ARG, "mech is null");
    if (m->device < 0) return set_error(MCC_ERR_STATE, "mechanism was compiled host-only (device -1)");
    if (n_cells < 0) return set_error(MCC_ERR_INVALID_ARG, "n_cells < 0");
    if (!m->t.paper_ok) return set_error(MCC_ERR_MECH, "a reaction has more products than the paper-layout records hold");
    if (n_cells == 0) return ok();
    if (!y || !k || !f) return set_error(MCC_ERR_INVALID_ARG, "null array");
    if (n_cells * (int64_t)m->t.R > ((int64_t)1 << 40)) return set_error(MCC_ERR_INVALID_ARG, "too many cells");
    DeviceGuard g(m->device);
    hipError_t e = launch_paper_deriv(inverted ? m->paper_rec_inv : m->paper_rec, inverted ? m->paper_yld_inv : m->paper_yld,
                                      inverted != 0, y, k, f, m->t.N, m->t.R, n_cells, (hipStream_t)stream);
    if (e != hipSuccess) return hip_error(e, "paper Derivative kernel launch");
    return ok();
}

mcc_status mcc_cells_set_rate_constants(mcc_cells *c, const double *k, void *stream)
{
    if (!c) return set_error(MCC_ERR_INVALID_ARG, "cells is null");
    if (c->n_cells > 0 && !k) return set_error(MCC_ERR_INVALID_ARG, "k is null");
    DeviceGuard g(c->mech->device);
    const size_t bytes = (size_t)c->mech->t.R * (size_t)c->ld * sizeof(double);
    if (bytes > 0) {
        hipError_t e = hipMemcpyAsync(c->k, k, bytes, hipMemcpyDeviceToDevice, (hipStream_t)stream);
        if (e != hipSuccess) return hip_error(e, "hipMemcpyAsync (rate constants)");
    }
    c->bound = true;
    return ok();
}

mcc_status mcc_calc_deriv(const mcc_cells *c, const double *y, double *f, void *stream)
{
    if (c && c->n_cells > 0 && !f) return set_error(MCC_ERR_INVALID_ARG, "f is null");
    return run_fj(c, y, f, nullptr, stream);
}

mcc_status mcc_calc_jac(const mcc_cells *c, const double *y, double *jac, void *stream)
{
    if (c && c->n_cells > 0 && !jac) return set_error(MCC_ERR_INVALID_ARG, "jac is null");
    return run_fj(c, y, nullptr, jac, stream);
}

mcc_status mcc_calc_deriv_jac(const mcc_cells *c, const double *y, double *f, double *jac, void *stream)
{
    if (c && c->n_cells > 0 && (!f || !jac)) return set_error(MCC_ERR_INVALID_ARG, "f and jac must not be null");
    return run_fj(c, y, f, jac, stream);
}

static bool opts_valid(const mcc_solver_opts &o, std::string *why)
{
    if (!(o.rtol >= 0.0) || !(o.atol > 0.0) || !std::isfinite(o.rtol) || !std::isfinite(o.atol)) {
        *why = "need rtol >= 0 and atol > 0, both finite";
        return false;
    }
    if (!(o.eta_newton > 0.0) || !(o.safety > 0.0) || !(o.fac_min > 0.0) || !(o.fac_max >= 1.0) ||
        !(o.fac_newton_fail > 0.0 && o.fac_newton_fail < 1.0) || !(o.h_min_rel >= 0.0)) {
        *why = "need eta_newton, safety, fac_min > 0, fac_max >= 1, 0 < fac_newton_fail < 1, h_min_rel >= 0";
        return false;
    }
    if (o.max_order < 1 || o.max_order > kMaxOrder || o.max_newton < 1 || o.max_newton > 16 || o.max_steps < 1) {
        *why = "need max_order in 1..5, max_newton in 1..16, max_steps >= 1";
        return false;
    }
    if (o.steps_per_launch < 0) {
        *why = "need steps_per_launch >= 0";
        return false;
    }
    if (o.warm_start != 0 && o.warm_start != 1) {
        *why = "warm_start must be 0 or 1";
        return false;
    }
    return true;
}

static SolveParams solve_params(mcc_cells *c, double *y, double dt, const mcc_solver_opts &o, int32_t *cell_status,
                                mcc_cell_stats *stats)
{
    const mcc_mech *m = c->mech;
    SolveParams p{};
    p.vspecies = m->vspecies;
    p.rx_reac = m->rx_reac;
    p.part = m->part;
    p.fg_ops = m->fg_ops;
    p.nm_ops = m->nm_ops;
    p.lu_ops = m->lu_ops;
    p.fwd_map = m->fwd_map;
    p.bwd_map = m->bwd_map;
    p.schur_tab = m->schur_tab;
    p.schur_ks = m->t.schur_ks;
    for (int q = 0, base = 0; q < kMaxSlots; ++q) {
        p.fg_blocks[q] = q < m->t.NS ? m->t.fg_blocks[q] : 0;
        p.fg_base[q] = q < m->t.NS ? m->t.fg_base[q] : 0;
        p.slot_cols[q] = q < m->t.NS ? m->t.slot_cols[q] : 0;
        p.ybase[q] = base;
        base += p.slot_cols[q];
    }
    p.nm_blocks = m->t.nm_blocks;
    p.lu_blocks = m->t.lu_blocks;
    p.NV = m->t.NV;
    p.tail_base = m->t.tail_base;
    p.N = m->t.N;
    p.R = m->t.R;
    p.P = m->t.n_partials;
    p.lu_nnz = m->t.lu_nnz;
    p.off_y = m->off_y;
    p.off_k = m->off_k;
    p.off_r = m->off_r;
    p.off_p = m->off_p;
    p.off_lu = m->off_lu;
    p.off_tm = m->off_tm;
    p.lds_doubles = m->lds_doubles;
    p.order = c->order;
    p.k = c->k;
    p.y = y;
    p.status = cell_status;
    p.stats = stats;
    p.n_cells = c->n_cells;
    p.ld = c->ld;
    p.dt = dt;
    p.opts = o;
    return p;
}

mcc_status mcc_adjoint_step(const mcc_cells *c, const double *y0, const double *tape, const int64_t *tape_len,
                            int64_t tape_stride, double *lam, double *glnk, int32_t accumulate, int32_t *cell_status,
                            void *stream)
{
    if (!c) return set_error(MCC_ERR_INVALID_ARG, "cells is null");
    if (!c->bound) return set_error(MCC_ERR_STATE, "the batch has no rate constants yet");
    const mcc_mech *m = c->mech;
    if (!m->adj.unavailable.empty()) return set_error(MCC_ERR_MECH, m->adj.unavailable);
    if (tape_stride < 0) return set_error(MCC_ERR_INVALID_ARG, "tape_stride < 0");
    if (c->n_cells == 0) return ok();
    if (!y0 || !tape_len || !lam || !glnk || (!tape && tape_stride > 0))
        return set_error(MCC_ERR_INVALID_ARG, "y0, tape, tape_len, lam and glnk must not be null");
    if (c->n_cells > 0x7fffffff) return set_error(MCC_ERR_INVALID_ARG, "too many cells");
    const HostTables &t = m->ta;
    SolveParams p{};
    p.vspecies = m->adj.vspecies;
    p.rx_reac = m->adj.rx_reac;
    p.part = m->adj.part;
    p.fg_ops = m->adj.fg_ops;
    p.nm_ops = m->adj.nm_ops;
    p.lu_ops = m->adj.lu_ops;
    p.fwd_map = m->adj.fwd_map;
    p.bwd_map = m->adj.bwd_map;
    p.schur_tab = m->adj.schur_tab;
    p.schur_ks = t.schur_ks;
    for (int q = 0, base = 0; q < kMaxSlots; ++q) {
        p.fg_blocks[q] = q < t.NS ? t.fg_blocks[q] : 0;
        p.fg_base[q] = q < t.NS ? t.fg_base[q] : 0;
        p.slot_cols[q] = q < t.NS ? t.slot_cols[q] : 0;
        p.ybase[q] = base;
        base += p.slot_cols[q];
    }
    p.nm_blocks = t.nm_blocks;
    p.lu_blocks = t.lu_blocks;
    p.NV = t.NV;
    p.tail_base = t.tail_base;
    p.N = t.N;
    p.R = t.R;
    p.P = t.n_partials;
    p.lu_nnz = t.lu_nnz;
    p.off_y = m->adj.off_y;
    p.off_k = m->adj.off_k;
    p.off_r = m->adj.off_r;
    p.off_p = m->adj.off_r;
    p.off_lu = m->adj.off_lu;
    p.off_tm = m->adj.off_tm;
    p.lds_doubles = m->adj.lds_doubles;
    p.order = c->order;
    p.k = c->k;
    p.n_cells = c->n_cells;
    p.ld = c->ld;
    AdjointParams a{};
    a.tape = tape;
    a.len = tape_len;
    a.stride = tape_stride;
    a.y0 = y0;
    a.lam = lam;
    a.glnk = glnk;
    a.status = cell_status;
    a.nu_ptr = m->adj.nu_ptr;
    a.nu_vid = m->adj.nu_vid;
    a.nu_coef = m->adj.nu_coef;
    a.off_w = m->adj.off_w;
    a.accumulate = accumulate != 0;
    DeviceGuard g(m->device);
    hipError_t e = launch_adjoint(p, a, t.NS, t.M, (hipStream_t)stream);
    if (e != hipSuccess) return hip_error(e, "reverse-mode kernel launch");
    return ok();
}

static mcc_status solve_step(mcc_cells *c, double *y, double dt, const mcc_solver_opts *opts, int32_t *cell_status,
                             mcc_cell_stats *stats, double *tape, int64_t *tape_len, int64_t tape_stride, void *stream);

mcc_status mcc_solve_step(mcc_cells *c, double *y, double dt, const mcc_solver_opts *opts, int32_t *cell_status,
                          mcc_cell_stats *stats, void *stream)
{
    return solve_step(c, y, dt, opts, cell_status, stats, nullptr, nullptr, 0, stream);
}

mcc_status mcc_solve_step_taped(mcc_cells *c, double *y, double dt, const mcc_solver_opts *opts, int32_t *cell_status,
                                mcc_cell_stats *stats, double *tape, int64_t *tape_len, int64_t tape_stride,
                                void *stream)
{
    if (!c) return set_error(MCC_ERR_INVALID_ARG, "cells is null");
    if (tape_stride < kTapeScalars)
        return set_error(MCC_ERR_INVALID_ARG, "tape_stride must hold at least the start entry (4 doubles)");
    if (c->n_cells > 0 && (!tape || !tape_len)) return set_error(MCC_ERR_INVALID_ARG, "tape and tape_len must not be null");
    const mcc_mech *m = c->mech;
    if (!m->adj.unavailable.empty()) return set_error(MCC_ERR_MECH, m->adj.unavailable);
    if (!adjoint_shape_supported(m->t.NS, m->t.M)) return set_error(MCC_ERR_MECH, "no taping solver for this mechanism's shape");
    return solve_step(c, y, dt, opts, cell_status, stats, tape, tape_len, tape_stride, stream);
}

mcc_status mcc_replay_step(const mcc_cells *c, const double *y0, const double *tape, const int64_t *tape_len,
                           int64_t tape_stride, double *y, int32_t max_newton, double tol, int32_t *cell_status,
                           void *stream)
{
    if (!c) return set_error(MCC_ERR_INVALID_ARG, "cells is null");
    if (!c->bound) return set_error(MCC_ERR_STATE, "the batch has no rate constants yet");
    const mcc_mech *m = c->mech;
    if (!adjoint_shape_supported(m->t.NS, m->t.M)) return set_error(MCC_ERR_MECH, "no replay kernel for this mechanism's shape");
    if (tape_stride < 0) return set_error(MCC_ERR_INVALID_ARG, "tape_stride < 0");
    if (max_newton < 1 || !(tol >= 0.0)) return set_error(MCC_ERR_INVALID_ARG, "need max_newton >= 1 and tol >= 0");
    if (c->n_cells == 0) return ok();
    if (!y0 || !y || !tape_len || (!tape && tape_stride > 0))
        return set_error(MCC_ERR_INVALID_ARG, "y0, tape, tape_len and y must not be null");
    DeviceGuard g(m->device);
    mcc_solver_opts o;
    mcc_solver_opts_default(&o);
    SolveParams p = solve_params(const_cast<mcc_cells *>(c), y, 1.0, o, cell_status, nullptr);
    ReplayParams r{};
    r.tape = tape;
    r.len = tape_len;
    r.stride = tape_stride;
    r.y0 = y0;
    r.y = y;
    r.status = cell_status;
    r.max_newton = max_newton;
    r.tol = tol;
    hipError_t e = launch_replay(p, r, m->t.NS, m->t.M, (hipStream_t)stream);
    if (e != hipSuccess) return hip_error(e, "replay kernel launch");
    return ok();
}

static mcc_status solve_step(mcc_cells *c, double *y, double dt, const mcc_solver_opts *opts, int32_t *cell_status,
                             mcc_cell_stats *stats, double *tape, int64_t *tape_len, int64_t tape_stride, void *stream)
{
    if (!c) return set_error(MCC_ERR_INVALID_ARG, "cells is null");
    if (!c->bound) return set_error(MCC_ERR_STATE, "mcc_cells_bind has not been called");
    if (!(dt > 0.0) || !std::isfinite(dt)) return set_error(MCC_ERR_INVALID_ARG, "dt must be finite and > 0");
    mcc_solver_opts o;
    if (opts)
        o = *opts;
    else
        mcc_solver_opts_default(&o);
    std::string why;
    if (!opts_valid(o, &why)) return set_error(MCC_ERR_INVALID_ARG, why);
    if (c->n_cells == 0) return ok();
    if (!y || !cell_status) return set_error(MCC_ERR_INVALID_ARG, "y and cell_status must not be null");
    if (o.warm_start && !stats)
        return set_error(MCC_ERR_INVALID_ARG, "warm_start reads each cell's previous stats: stats must not be null");
    const mcc_mech *m = c->mech;
    DeviceGuard g(m->device);
    SolveParams p = solve_params(c, y, dt, o, cell_status, stats);
    p.tape = tape;
    p.tape_len = tape_len;
    p.tape_stride = tape_stride;
    if (o.steps_per_launch <= 0) {  // the whole outer step in one launch
        hipError_t e = launch_solve(p, m->t.NS, m->t.M, p.tape ? 0 : m->solve_waves, (hipStream_t)stream);
        if (e != hipSuccess) return hip_error(e, "solver kernel launch");
        return ok();
    }
    // Per-launch form: state in HBM between launches; relaunch until every
    // cell has finished.  Every launch takes each unfinished cell at least one
    // accepted step (or to its end), so max_steps / K + 1 launches suffice.
    p.state_stride = (int64_t)(kMaxOrder + 3) * m->t.NV + kStateScalars;
    const int64_t need = p.state_stride * c->n_cells;
    hipStream_t s = (hipStream_t)stream;
    if (c->state_doubles < need) {
        if (c->state) (void)hipFree(c->state);
        c->state = nullptr;
        c->state_doubles = 0;
        hipError_t e = hipMalloc(&c->state, (size_t)need * sizeof(double));
        if (e != hipSuccess) return hip_error(e, "hipMalloc (solver state)");
        e = hipMemset(c->state, 0, (size_t)need * sizeof(double));  // no call id matches 0
        if (e != hipSuccess) return hip_error(e, "hipMemset (solver state)");
        c->state_doubles = need;
    }
    if (!c->pending) {
        hipError_t e = hipMalloc(&c->pending, sizeof(int32_t));
        if (e == hipSuccess) e = hipHostMalloc((void **)&c->pending_host, sizeof(int32_t), hipHostMallocDefault);
        if (e != hipSuccess) return hip_error(e, "allocating the pending-cell counter");
    }
    c->call_id = c->call_id >= 0x3fffffff ? 1 : c->call_id + 1;
    p.state = c->state;
    p.pending = c->pending;
    p.call_id = c->call_id;
    const int64_t max_launches = (int64_t)o.max_steps / o.steps_per_launch + 2;
    for (int64_t launch = 0;; ++launch) {
        if (launch >= max_launches) return set_error(MCC_ERR_DEVICE, "per-launch solver did not finish");
        hipError_t e = launch_fill_i32(c->pending, 0, s);
        if (e == hipSuccess) e = launch_solve(p, m->t.NS, m->t.M, p.tape ? 0 : m->solve_waves, s);
        if (e == hipSuccess) e = hipMemcpyAsync(c->pending_host, c->pending, sizeof(int32_t), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_error(e, "per-launch solver");
        if (*c->pending_host == 0) break;
    }
    return ok();
}

// The Multi-cells outer step; slots: caller-provided reduction slots
// [2][n_cells] (the allocation-free entry point), or null for the batch's own.
static mcc_status solve_step_multicell(mcc_cells *c, double *y, double dt, const mcc_solver_opts *opts,
                                       int32_t *cell_status, mcc_cell_stats *stats, double *slots, void *stream);

mcc_status mcc_solve_step_multicell(mcc_cells *c, double *y, double dt, const mcc_solver_opts *opts,
                                    int32_t *cell_status, mcc_cell_stats *stats, void *stream)
{
    return solve_step_multicell(c, y, dt, opts, cell_status, stats, nullptr, stream);
}

mcc_status mcc_solve_step_multicell_noalloc(mcc_cells *c, double *y, double dt, const mcc_solver_opts *opts,
                                            int32_t *cell_status, mcc_cell_stats *stats, void *stream)
{
    if (!c) return set_error(MCC_ERR_INVALID_ARG, "cells is null");
    if (c->n_cells > kMcScratchCells)
        return set_error(MCC_ERR_INVALID_ARG, "mcc_solve_step_multicell_noalloc handles at most " +
                                                  std::to_string(kMcScratchCells) + " cells (its static reduction "
                                                  "slots); this batch has " + std::to_string(c->n_cells));
    DeviceGuard g(c->mech->device);
    if (!g.ok()) return set_error(MCC_ERR_DEVICE, "cannot select the batch's device");
    double *slots = nullptr;
    const hipError_t e = multicell_scratch(c->mech->device, &slots);
    if (e != hipSuccess) return hip_error(e, "hipGetSymbolAddress (static Multi-cells slots)");
    return solve_step_multicell(c, y, dt, opts, cell_status, stats, slots, stream);
}

static mcc_status solve_step_multicell(mcc_cells *c, double *y, double dt, const mcc_solver_opts *opts,
                                       int32_t *cell_status, mcc_cell_stats *stats, double *slots, void *stream)
{
    if (!c) return set_error(MCC_ERR_INVALID_ARG, "cells is null");
    if (!c->bound) return set_error(MCC_ERR_STATE, "mcc_cells_bind has not been called");
    if (!(dt > 0.0) || !std::isfinite(dt)) return set_error(MCC_ERR_INVALID_ARG, "dt must be finite and > 0");
    mcc_solver_opts o;
    if (opts)
        o = *opts;
    else
        mcc_solver_opts_default(&o);
    std::string why;
    if (!opts_valid(o, &why)) return set_error(MCC_ERR_INVALID_ARG, why);
    if (o.steps_per_launch != 0) return set_error(MCC_ERR_INVALID_ARG, "Multi-cells runs in one launch: steps_per_launch must be 0");
    if (o.warm_start != 0) return set_error(MCC_ERR_INVALID_ARG, "Multi-cells starts every step afresh: warm_start must be 0");
    if (c->n_cells == 0) return ok();
    if (!y || !cell_status) return set_error(MCC_ERR_INVALID_ARG, "y and cell_status must not be null");
    const mcc_mech *m = c->mech;
    DeviceGuard g(m->device);
    int64_t cap = 0;
    hipError_t e = multicell_capacity(m->t.NS, m->t.M, (size_t)m->lds_doubles * sizeof(double), m->device, &cap);
    if (e != hipSuccess) return hip_error(e, "Multi-cells occupancy");
    if (cap == 0) return set_error(MCC_ERR_INVALID_ARG, "no Multi-cells solver for this mechanism's size");
    if (c->n_cells > cap)
        return set_error(MCC_ERR_INVALID_ARG, "Multi-cells needs every cell resident at once: at most " +
                                                  std::to_string(cap) + " cells of this mechanism on this device");
    if (!slots && c->mc_cells < c->n_cells) {
        if (c->mc_slots) (void)hipFree(c->mc_slots);
        c->mc_slots = nullptr;
        c->mc_cells = 0;
        e = hipMalloc(&c->mc_slots, 2 * (size_t)c->n_cells * sizeof(double));
        if (e != hipSuccess) return hip_error(e, "hipMalloc (Multi-cells reduction slots)");
        c->mc_cells = c->n_cells;
    }
    SolveParams p = solve_params(c, y, dt, o, cell_status, stats);
    p.order = nullptr;  // the grid-wide sums are taken in workgroup order: keep it the cell order
    p.mc_slots = slots ? slots : c->mc_slots;
    e = launch_solve_multicell(p, m->t.NS, m->t.M, (hipStream_t)stream);
    if (e != hipSuccess) return hip_error(e, "Multi-cells solver launch");
    return ok();
}

mcc_status mcc_cells_set_schedule(mcc_cells *c, const int32_t *order)
{
    if (!c) return set_error(MCC_ERR_INVALID_ARG, "cells is null");
    DeviceGuard g(c->mech->device);
    if (!order) {
        if (c->order) {
            hipError_t e = hipDeviceSynchronize();  // no launch may still read it
            if (e == hipSuccess) e = hipFree(c->order);
            c->order = nullptr;
            if (e != hipSuccess) return hip_error(e, "releasing the cell schedule");
        }
        return ok();
    }
    const int64_t n = c->n_cells;
    std::vector<char> seen((size_t)n, 0);
    for (int64_t i = 0; i < n; ++i) {
        const int32_t v = order[i];
        if (v < 0 || v >= n || seen[(size_t)v])
            return set_error(MCC_ERR_INVALID_ARG, "order is not a permutation of the cells (entry " +
                                                      std::to_string(i) + ")");
        seen[(size_t)v] = 1;
    }
    if (n == 0) return ok();
    hipError_t e = hipSuccess;
    if (!c->order) e = hipMalloc(&c->order, (size_t)n * sizeof(int32_t));
    else e = hipDeviceSynchronize();  // earlier launches may still read the old schedule
    if (e == hipSuccess) e = hipMemcpy(c->order, order, (size_t)n * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_error(e, "uploading the cell schedule");
    return ok();
}

mcc_status mcc_cells_schedule_from_stats(mcc_cells *c, const mcc_cell_stats *stats, int32_t *order_out)
{
    return mcc_cells_schedule_from_stats_ex(c, stats, MCC_SCHEDULE_LONGEST_FIRST, order_out);
}

mcc_status mcc_cells_schedule_from_stats_ex(mcc_cells *c, const mcc_cell_stats *stats, int32_t kind,
                                            int32_t *order_out)
{
    if (kind != MCC_SCHEDULE_LONGEST_FIRST && kind != MCC_SCHEDULE_ZIGZAG)
        return set_error(MCC_ERR_INVALID_ARG, "unknown schedule kind");
    if (!c) return set_error(MCC_ERR_INVALID_ARG, "cells is null");
    const int64_t n = c->n_cells;
    if (n == 0) return ok();
    if (!stats) return set_error(MCC_ERR_INVALID_ARG, "stats is null");
    DeviceGuard g(c->mech->device);
    std::vector<mcc_cell_stats> st((size_t)n);
    // the counters may come from work on any stream (e.g. a non-blocking one)
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(st.data(), stats, (size_t)n * sizeof(mcc_cell_stats), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_error(e, "copying the counters to the host");
    // longest first: attempts = accepted steps + rejections + Newton failures
    std::vector<int32_t> order((size_t)n);
    for (int64_t i = 0; i < n; ++i) order[(size_t)i] = (int32_t)i;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        const int64_t wa = (int64_t)st[a].steps + st[a].rejects + st[a].newton_fails;
        const int64_t wb = (int64_t)st[b].steps + st[b].rejects + st[b].newton_fails;
        return wa > wb;
    });
    if (kind == MCC_SCHEDULE_ZIGZAG) {  // longest, shortest, second longest, second shortest, ...
        std::vector<int32_t> z;
        z.reserve((size_t)n);
        for (int64_t lo = 0, hi = n - 1; lo <= hi; ++lo, --hi) {
            z.push_back(order[(size_t)lo]);
            if (hi != lo) z.push_back(order[(size_t)hi]);
        }
        order.swap(z);
    }
    const mcc_status r = mcc_cells_set_schedule(c, order.data());
    if (r == MCC_OK && order_out) std::memcpy(order_out, order.data(), (size_t)n * sizeof(int32_t));
    return r;
}

mcc_status mcc_sync(mcc_cells *c)
{
    if (!c) return set_error(MCC_ERR_INVALID_ARG, "cells is null");
    DeviceGuard g(c->mech->device);
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_error(e, "hipDeviceSynchronize");
    return ok();
}

mcc_status mcc_cells_destroy(mcc_cells *c)
{
    if (!c) return ok();
    DeviceGuard g(c->mech->device);
    hipError_t e = hipDeviceSynchronize();
    for (void *buf : {(void *)c->k, (void *)c->ones, (void *)c->state, (void *)c->pending, (void *)c->mc_slots,
                      (void *)c->order})
        if (buf) {
            hipError_t e2 = hipFree(buf);
            if (e == hipSuccess) e = e2;
        }
    if (c->pending_host) {
        hipError_t e2 = hipHostFree(c->pending_host);
        if (e == hipSuccess) e = e2;
    }
    c->mech->live_batches--;
    delete c;
    if (e != hipSuccess) return hip_error(e, "mcc_cells_destroy");
    return ok();
}

}  // extern "C"
