// C ABI entry points: argument validation, context lifecycle, the grid build
// sequence and the wave plan. All numerical work runs in the HIP kernels of
// grid.hip, batching.hip and integrate.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "xc_internal.hpp"

namespace xc {

static thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    const int code = (e == hipErrorOutOfMemory) ? XC_ERR_NOMEM : XC_ERR_DEVICE;
    return fail(code, std::string(what) + ": " + hipGetErrorString(e));
}

int dev_reserve(DevBuf& b, size_t bytes) {
    if (bytes == 0) bytes = 8;
    if (b.p && b.cap >= bytes) return XC_OK;
    if (b.al) {
        if (b.p) b.al->free(b.p, b.al->user);
        b.p = b.al->alloc(bytes, b.al->user);
        if (!b.p) {
            b.cap = 0;
            return fail(XC_ERR_NOMEM, "device allocator returned NULL for " +
                                          std::to_string(bytes) + " bytes");
        }
        b.cap = bytes;
        return XC_OK;
    }
    if (b.p) {
        hipError_t e = hipFree(b.p);
        b.p = nullptr;
        b.cap = 0;
        if (e != hipSuccess) return hip_fail(e, "hipFree");
    }
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e != hipSuccess) {
        b.p = nullptr;
        (void)hipGetLastError();
        return hip_fail(e, "hipMalloc");
    }
    b.cap = bytes;
    return XC_OK;
}

void dev_release(DevBuf& b) {
    if (b.p) {
        if (b.al) b.al->free(b.p, b.al->user);
        else (void)hipFree(b.p);
    }
    b.p = nullptr;
    b.cap = 0;
}

int upload(DevBuf& b, const void* src, size_t bytes, hipStream_t s) {
    XC_TRY(dev_reserve(b, bytes));
    // an empty host vector has no storage: only reserve
    if (bytes && src) XC_HIP(hipMemcpyAsync(b.p, src, bytes, hipMemcpyHostToDevice, s));
    return XC_OK;
}

static hipEvent_t take_event(PhaseTimer& t) {
    if (!t.pool.empty()) {
        hipEvent_t e = t.pool.back();
        t.pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}

PhaseScope::PhaseScope(xc_context* c, int phase) : PhaseScope(&c->timer, c->stream, phase) {}

PhaseScope::PhaseScope(PhaseTimer* t, hipStream_t s, int phase) : t_(t), s_(s), phase_(phase) {
    if (!t_ || !t_->enabled) return;
    e0_ = take_event(*t_);
    if (e0_) (void)hipEventRecord(e0_, s_);
}

PhaseScope::~PhaseScope() {
    if (!e0_) return;
    hipEvent_t e1 = take_event(*t_);
    if (!e1) return;
    (void)hipEventRecord(e1, s_);
    t_->pending[phase_].emplace_back(e0_, e1);
}

static int fold_timer(xc_context* c) {
    PhaseTimer& t = c->timer;
    XC_HIP(hipStreamSynchronize(c->stream));
    for (int p = 0; p < XC_NUM_PHASES; ++p) {
        for (auto& pr : t.pending[p]) {
            float ms = 0.0f;
            XC_HIP(hipEventElapsedTime(&ms, pr.first, pr.second));
            t.ms[p] += ms;
            t.launches[p] += 1;
            t.pool.push_back(pr.first);
            t.pool.push_back(pr.second);
        }
        t.pending[p].clear();
    }
    return XC_OK;
}

void release_build_temporaries(xc_context* c) {
    DevBuf* bufs[] = {&c->raw_x, &c->raw_y, &c->raw_z, &c->raw_w, &c->tx, &c->ty, &c->tz,
                      &c->tw, &c->tidx, &c->blk_count, &c->blk_off, &c->atom_count,
                      &c->cells_a, &c->cells_b, &c->child_count, &c->child_begin,
                      &c->counters, &c->scr_nsh, &c->scr_nfn, &c->scr_shoff, &c->scr_fnoff};
    for (DevBuf* b : bufs) dev_release(*b);
}

size_t device_bytes(const xc_context* c) {
    const DevBuf* bufs[] = {&c->d_atoms, &c->d_invR, &c->d_nnhalf, &c->d_shells, &c->d_palpha,
                            &c->d_pcoef, &c->d_ang, &c->d_gatoms, &c->d_fshell, &c->d_nbr_idx, &c->d_nbr_R, &c->d_becke_a,
                            &c->raw_x, &c->raw_y,
                            &c->raw_z, &c->raw_w, &c->px, &c->py, &c->pz, &c->pw, &c->pidx,
                            &c->tx, &c->ty, &c->tz, &c->tw, &c->tidx, &c->blk_count,
                            &c->blk_off, &c->atom_count, &c->cells_a, &c->cells_b,
                            &c->child_count, &c->child_begin, &c->batches, &c->counters,
                            &c->scr_nsh, &c->scr_nfn, &c->scr_shoff, &c->scr_fnoff,
                            &c->shell_list, &c->shell_loff, &c->func_list, &c->d_wb,
                            &c->d_gemm_pre, &c->d_syr_pre, &c->d_wide_pre, &c->d_tmap, &c->scratch,
                            &c->epart, &c->npart, &c->d_req, &c->pdig, &c->pscale, &c->d_wb_beta,
                            &c->d_wb_meta};
    size_t n = 0;
    for (const DevBuf* b : bufs) n += b->cap;
    return n;
}

static void destroy_timer(PhaseTimer& t) {
    for (int p = 0; p < XC_NUM_PHASES; ++p) {
        for (auto& pr : t.pending[p]) {
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
        t.pending[p].clear();
    }
    for (hipEvent_t e : t.pool) (void)hipEventDestroy(e);
    t.pool.clear();
}

// Functions of shell s of a basis: spherical shells only from L = 2 on.
static int nfunc(const xc_basis* b, int s) {
    const int L = b->shell_L[s];
    return shell_nfunc(L, (b->shell_pure && b->shell_pure[s] && L >= 2) ? 1 : 0);
}

static bool finite(double v) { return std::isfinite(v); }

static int validate_inputs(const xc_molecule* mol, const xc_basis* basis,
                           const xc_grid_spec* g) {
    if (!mol || !basis || !g) return fail(XC_ERR_INVALID_ARG, "null molecule, basis or grid");
    if (mol->natoms < 1 || !mol->xyz || !mol->mk_alpha)
        return fail(XC_ERR_INVALID_ARG, "molecule needs natoms >= 1 and coordinate/alpha arrays");
    for (int a = 0; a < mol->natoms; ++a) {
        for (int q = 0; q < 3; ++q)
            if (!finite(mol->xyz[3 * a + q])) return fail(XC_ERR_INVALID_ARG, "non-finite atom coordinate");
        if (!(mol->mk_alpha[a] > 0.0) || !finite(mol->mk_alpha[a]))
            return fail(XC_ERR_INVALID_ARG, "Mura-Knowles alpha must be positive");
    }
    for (int a = 0; a < mol->natoms; ++a)
        for (int b = 0; b < a; ++b) {
            const double dx = mol->xyz[3 * a] - mol->xyz[3 * b];
            const double dy = mol->xyz[3 * a + 1] - mol->xyz[3 * b + 1];
            const double dz = mol->xyz[3 * a + 2] - mol->xyz[3 * b + 2];
            if (dx * dx + dy * dy + dz * dz < 1e-16)
                return fail(XC_ERR_INVALID_ARG, "two atoms at the same position");
        }
    if (basis->nshells < 1 || !basis->shell_atom || !basis->shell_L || !basis->shell_nprim ||
        !basis->prim_alpha || !basis->prim_coef)
        return fail(XC_ERR_INVALID_ARG, "basis needs nshells >= 1 and all arrays");
    long long np = 0;
    for (int s = 0; s < basis->nshells; ++s) {
        if (basis->shell_atom[s] < 0 || basis->shell_atom[s] >= mol->natoms)
            return fail(XC_ERR_INVALID_ARG, "shell_atom out of range");
        if (basis->shell_L[s] < 0) return fail(XC_ERR_INVALID_ARG, "negative angular momentum");
        if (basis->shell_L[s] > kMaxL) return fail(XC_ERR_UNSUPPORTED, "angular momentum above 3");
        if (basis->shell_nprim[s] < 1) return fail(XC_ERR_INVALID_ARG, "shell without primitives");
        if (basis->shell_nprim[s] > kMaxPrim) return fail(XC_ERR_UNSUPPORTED, "more than 16 primitives");
        if (basis->shell_pure && basis->shell_pure[s] != 0 && basis->shell_pure[s] != 1)
            return fail(XC_ERR_INVALID_ARG, "shell_pure flags must be 0 or 1");
        np += basis->shell_nprim[s];
    }
    for (long long p = 0; p < np; ++p) {
        if (!(basis->prim_alpha[p] > 0.0) || !finite(basis->prim_alpha[p]))
            return fail(XC_ERR_INVALID_ARG, "exponents must be positive and finite");
        if (!finite(basis->prim_coef[p])) return fail(XC_ERR_INVALID_ARG, "non-finite coefficient");
    }
    if (g->n_rad < 1 || g->n_ang < 1 || !g->ang_xyzw)
        return fail(XC_ERR_INVALID_ARG, "grid needs n_rad, n_ang >= 1 and an angular table");
    if ((long long)g->n_rad * g->n_ang > (1LL << 30))
        return fail(XC_ERR_INVALID_ARG, "too many points per atom");
    for (long long k = 0; k < 4LL * g->n_ang; ++k)
        if (!finite(g->ang_xyzw[k])) return fail(XC_ERR_INVALID_ARG, "non-finite angular table");
    if (g->partition != XC_PARTITION_SSF && g->partition != XC_PARTITION_BECKE)
        return fail(XC_ERR_INVALID_ARG, "unknown partition");
    if (g->partition == XC_PARTITION_SSF && !(g->ssf_a > 0.0 && g->ssf_a < 1.0))
        return fail(XC_ERR_INVALID_ARG, "ssf_a must lie in (0, 1)");
    if (g->partition == XC_PARTITION_BECKE) {
        if (mol->natoms > kSsfWaveMaxAtoms)
            return fail(XC_ERR_UNSUPPORTED, "Becke's partition is limited to 1024 atoms");
        if (g->becke_radius)
            for (int a = 0; a < mol->natoms; ++a)
                if (!(g->becke_radius[a] > 0.0) || !finite(g->becke_radius[a]))
                    return fail(XC_ERR_INVALID_ARG, "becke_radius must be positive");
    }
    if (!(g->screen_eta >= 0.0) || !finite(g->screen_eta))
        return fail(XC_ERR_INVALID_ARG, "screen_eta must be >= 0");
    if (g->batch_max < 16 || g->batch_max > kMaxBatch)
        return fail(XC_ERR_INVALID_ARG, "batch_max must lie in [16, 1024]");
    if (!(g->rho_thresh > 0.0) || !finite(g->rho_thresh))
        return fail(XC_ERR_INVALID_ARG, "rho_thresh must be positive");
    return XC_OK;
}

static int check_func_prec(int functional, int precision) {
    if (functional != XC_LDA_SVWN5 && functional != XC_GGA_PBE && functional != XC_MGGA_TPSS)
        return fail(XC_ERR_UNSUPPORTED, "unknown functional");
    if (functional == XC_MGGA_TPSS && precision != XC_FP64)
        return fail(XC_ERR_UNSUPPORTED, "meta-GGA integrations run in FP64 only");
    if (precision != XC_FP64 && precision != XC_MIXED_FP32 && precision != XC_MIXED_FP32_V &&
        precision != XC_MIXED_BF16)
        return fail(XC_ERR_UNSUPPORTED, "precision not available");
    return XC_OK;
}

// Every device buffer of a context.
static std::vector<DevBuf*> all_buffers(xc_context* c) {
    return {&c->d_atoms, &c->d_invR, &c->d_nnhalf, &c->d_shells, &c->d_palpha,
                      &c->d_pcoef, &c->d_ang, &c->d_gatoms, &c->d_fshell, &c->d_nbr_idx, &c->d_nbr_R, &c->d_becke_a,
                      &c->raw_x, &c->raw_y,
                      &c->raw_z, &c->raw_w, &c->px, &c->py, &c->pz, &c->pw, &c->pidx,
                      &c->tx, &c->ty, &c->tz, &c->tw, &c->tidx, &c->blk_count,
                      &c->blk_off, &c->atom_count, &c->cells_a, &c->cells_b,
                      &c->child_count, &c->child_begin, &c->batches, &c->counters,
                      &c->scr_nsh, &c->scr_nfn, &c->scr_shoff, &c->scr_fnoff,
                      &c->shell_list, &c->shell_loff, &c->func_list, &c->d_wb,
                      &c->d_gemm_pre, &c->d_syr_pre, &c->d_wide_pre, &c->d_tmap, &c->scratch, &c->epart,
                      &c->npart, &c->d_req, &c->pdig, &c->pscale, &c->d_wb_beta, &c->d_wb_meta};
}

static void release_all(xc_context* c) {
    for (DevBuf* b : all_buffers(c)) dev_release(*b);
}

// Split the batches into consecutive waves whose scratch (Phi and its
// gradient, or Z, plus density partials) fits the budget (Alg. 2: subsets
// that saturate device memory), and build each wave's tile tables.
static int plan_waves(xc_context* c) {
    c->phi_cached_kind = 0;
    c->waves.clear();
    c->h_wb.clear();
    std::vector<int> gpre, spre, wpre;
    c->max_nb = c->max_ng = 0;
    c->sum_nb_ng = c->sum_nb2_ng = c->flops_contract = 0.0;
    size_t budget = c->wave_budget;
    if (budget == 0) {
        size_t fr = 0, tot = 0;
        XC_HIP(hipMemGetInfo(&fr, &tot));
        budget = std::min<size_t>(fr / 2, (size_t)48 << 30);
    }
    Wave cur{};
    cur.wb_off = 0;
    cur.pre_off = 0;
    size_t used = 0;
    gpre.push_back(0);
    spre.push_back(0);
    wpre.push_back(0);
    double s2 = 0.0, s1 = 0.0;   // the open wave's sum n_b^2 n_g and sum n_b n_g
    auto close_wave = [&]() {
        if (cur.count == 0) return;
        cur.wide = s2 >= kWideNb * s1;
        s2 = s1 = 0.0;
        c->waves.push_back(cur);
        c->max_wave_bytes = std::max(c->max_wave_bytes, used);
        Wave nx{};
        nx.first = cur.first + cur.count;
        nx.wb_off = (long long)c->h_wb.size();
        nx.pre_off = (long long)gpre.size();
        cur = nx;
        used = 0;
        gpre.push_back(0);
        spre.push_back(0);
        wpre.push_back(0);
    };
    c->max_wave_bytes = 0;
    for (long long j = 0; j < c->n_batches; ++j) {
        const Cell& b = c->h_batches[j];
        const int nb = c->h_nfn[j], ng = b.count;
        const int nbp = (nb + kRowPad - 1) / kRowPad * kRowPad;
        const int ngp = (ng + kColPad - 1) / kColPad * kColPad;
        const int nmt = (nb + kTile - 1) / kTile;
        const size_t slab = (size_t)nbp * ngp;
        WaveBatch w{};
        w.nbp = nbp;
        w.ngp = ngp;
        w.nmt = nmt;
        // the spin and the meta-GGA extras share the room after the partials
        const size_t bytes =
            batch_scratch_bytes(w) + std::max(c->spin_plan ? batch_spin_bytes(w) : 0,
                                              c->meta_plan ? batch_meta_bytes(w) : 0);
        if (cur.count > 0 && used + bytes > budget) close_wave();
        w.phi_off = (long long)(used / 8);
        w.z_off = w.phi_off + (long long)(batch_phi_bytes(w) / 8);
        w.part_off = w.z_off + (long long)slab;
        w.pt_off = b.begin;
        w.shell_off = c->h_shoff[j];
        w.func_off = c->h_fnoff[j];
        w.nb = nb;
        w.ng = ng;
        w.nshell = c->h_nsh[j];
        w.batch = (int)j;
        w.req = 0;
        c->h_wb.push_back(w);
        used += bytes;
        const int gt = nmt * (ngp / kTile);
        const int st = nmt * (nmt + 1) / 2;
        const int pt = batch_wide_tiles(w);
        gpre.push_back(gpre.back() + gt);
        spre.push_back(spre.back() + st);
        wpre.push_back(wpre.back() + pt);
        cur.gemm_tiles += gt;
        cur.syr_tiles += st;
        cur.wide_tiles += pt;
        cur.count += 1;
        cur.scratch_bytes = used;
        c->max_nb = std::max(c->max_nb, nb);
        c->max_ng = std::max(c->max_ng, ng);
        c->sum_nb_ng += (double)nb * ng;
        c->sum_nb2_ng += (double)nb * nb * ng;
        s1 += (double)nb * ng;
        s2 += (double)nb * nb * ng;
        c->flops_contract += 2.0 * nb * nb * ng + 2.0 * nb * (nb + 1.0) * ng;
    }
    close_wave();
    XC_TRY(upload(c->d_wb, c->h_wb.data(), sizeof(WaveBatch) * std::max<size_t>(1, c->h_wb.size()),
                  c->stream));
    if (c->spin_plan) {
        // the same batches with the beta partials (after the alpha ones) and
        // the second request descriptor (P^b, V^b)
        c->h_wb_beta = c->h_wb;
        for (WaveBatch& w : c->h_wb_beta) {
            w.part_off += (long long)(batch_spin_bytes(w) / 8);
            w.req = 1;
        }
        XC_TRY(upload(c->d_wb_beta, c->h_wb_beta.data(),
                      sizeof(WaveBatch) * std::max<size_t>(1, c->h_wb_beta.size()), c->stream));
    }
    if (c->meta_plan) {
        // three copies of the batches: gradient slab d in place of Phi,
        // partial set d in place of the density partials
        const size_t n = c->h_wb.size();
        c->h_wb_meta.resize(3 * n);
        for (int d = 0; d < 3; ++d)
            for (size_t j = 0; j < n; ++j) {
                WaveBatch w = c->h_wb[j];
                w.phi_off = meta_grad_off(c->h_wb[j], d);
                w.part_off = meta_part_off(c->h_wb[j], d);
                c->h_wb_meta[d * n + j] = w;
            }
        XC_TRY(upload(c->d_wb_meta, c->h_wb_meta.data(),
                      sizeof(WaveBatch) * std::max<size_t>(1, c->h_wb_meta.size()), c->stream));
    }
    XC_TRY(upload(c->d_gemm_pre, gpre.data(), sizeof(int) * gpre.size(), c->stream));
    XC_TRY(upload(c->d_syr_pre, spre.data(), sizeof(int) * spre.size(), c->stream));
    XC_TRY(upload(c->d_wide_pre, wpre.data(), sizeof(int) * wpre.size(), c->stream));
    int max_tiles = 1;
    for (const Wave& w : c->waves) max_tiles = std::max({max_tiles, w.gemm_tiles, w.syr_tiles});
    c->max_tiles = max_tiles;
    XC_TRY(dev_reserve(c->d_tmap, 2 * sizeof(int) * (size_t)max_tiles));
    XC_TRY(dev_reserve(c->d_req, (c->spin_plan ? 2 : 1) * sizeof(ReqDev)));
    if (!c->external_scratch)
        XC_TRY(dev_reserve(c->scratch, std::max<size_t>(c->max_wave_bytes, 8)));
    XC_TRY(dev_reserve(c->epart, 8 * (size_t)std::max<long long>(1, c->n_batches)));
    XC_TRY(dev_reserve(c->npart, 8 * (size_t)std::max<long long>(1, c->n_batches)));
    XC_HIP(hipStreamSynchronize(c->stream));
    return XC_OK;
}

size_t estimate_build_bytes(const xc_context* c) {
    // points, weights and build temporaries scale with the nominal grid;
    // screening lists with points x basis size
    const double npts = (double)c->n_rad * c->n_ang * (double)c->gatoms.size();
    const double build = npts * (32.0 + 80.0 + 8.0);
    const double lists = npts / 64.0 * (8.0 + 8.0 * std::min(c->nbf, 4096));
    const double fixed = 8.0 * c->natoms * (double)c->natoms + 4096.0 * 1024.0;
    return (size_t)(build + lists + fixed);
}

int build_grid(xc_context* c) {
    c->built = false;
    c->phi_cached_kind = 0;
    const long long npa = (long long)c->n_rad * c->n_ang;
    c->n_nominal = npa * (long long)c->gatoms.size();
    if (c->n_nominal == 0) {
        c->n_points = 0;
        c->n_batches = 0;
        c->h_batches.clear();
        XC_TRY(run_screening(c));
        XC_TRY(plan_waves(c));
        c->built = true;
        return XC_OK;
    }
    const size_t bytes = 8 * (size_t)c->n_nominal;
    XC_TRY(dev_reserve(c->raw_x, bytes));
    XC_TRY(dev_reserve(c->raw_y, bytes));
    XC_TRY(dev_reserve(c->raw_z, bytes));
    XC_TRY(dev_reserve(c->raw_w, bytes));
    XC_TRY(launch_grid_points(c));
    XC_TRY(launch_ssf(c));
    std::vector<long long> kept;
    XC_TRY(launch_compact(c, kept));
    XC_TRY(run_batching(c, kept));
    XC_TRY(run_screening(c));
    XC_TRY(plan_waves(c));
    c->built = true;
    return XC_OK;
}

}  // namespace xc

using namespace xc;

extern "C" {

const char* xc_strerror(int code) {
    switch (code) {
        case XC_OK: return "ok";
        case XC_ERR_INVALID_ARG: return "invalid argument";
        case XC_ERR_UNSUPPORTED: return "unsupported input";
        case XC_ERR_NOMEM: return "out of device memory";
        case XC_ERR_DEVICE: return "device error";
        case XC_ERR_STATE: return "invalid state";
        case XC_ERR_BUSY: return "busy";
        default: return "unknown error";
    }
}

const char* xc_last_error(void) { return g_last_error.c_str(); }

int xc_abi_version(void) { return XC_ABI_VERSION; }

int xc_context_create(const xc_molecule* mol, const xc_basis* basis,
                      const xc_grid_spec* g, const xc_device_opts* opts,
                      xc_context** out) {
    g_last_error.clear();
    if (!out) return fail(XC_ERR_INVALID_ARG, "null output pointer");
    *out = nullptr;
    XC_TRY(validate_inputs(mol, basis, g));
    xc_context* c = new (std::nothrow) xc_context();
    if (!c) return fail(XC_ERR_NOMEM, "host allocation failed");
    c->stream = opts ? (hipStream_t)opts->stream : nullptr;
    c->wave_budget = opts ? opts->wave_bytes : 0;
    if (opts && (opts->alloc || opts->free)) {
        if (!opts->alloc || !opts->free) {
            delete c;
            return fail(XC_ERR_INVALID_ARG, "set both alloc and free, or neither");
        }
        c->alloc = {opts->alloc, opts->free, opts->alloc_user};
        for (DevBuf* b : all_buffers(c)) b->al = &c->alloc;
    }
    c->natoms = mol->natoms;
    c->atoms4.resize(4 * (size_t)c->natoms);
    for (int a = 0; a < c->natoms; ++a) {
        for (int q = 0; q < 3; ++q) c->atoms4[4 * a + q] = mol->xyz[3 * a + q];
        c->atoms4[4 * a + 3] = mol->mk_alpha[a];
    }
    c->nshells = basis->nshells;
    int po = 0, ff = 0;
    std::vector<ShellDev> sh(c->nshells);
    for (int s = 0; s < c->nshells; ++s) {
        const int a = basis->shell_atom[s];
        c->shell_atom.push_back(a);
        c->shell_L.push_back(basis->shell_L[s]);
        c->shell_nprim.push_back(basis->shell_nprim[s]);
        const int pure = (basis->shell_pure && basis->shell_pure[s] && basis->shell_L[s] >= 2)
                             ? 1 : 0;
        c->shell_pure.push_back(pure);
        c->any_pure = c->any_pure || pure;
        c->prim_off.push_back(po);
        c->first_func.push_back(ff);
        sh[s].x = c->atoms4[4 * a];
        sh[s].y = c->atoms4[4 * a + 1];
        sh[s].z = c->atoms4[4 * a + 2];
        sh[s].rcut2 = 0.0;
        sh[s].L = basis->shell_L[s];
        sh[s].nprim = basis->shell_nprim[s];
        sh[s].prim_off = po;
        sh[s].first_func = ff;
        sh[s].pure = pure;
        sh[s].pad_ = 0;
        po += basis->shell_nprim[s];
        ff += nfunc(basis, s);
    }
    c->nbf = ff;
    std::vector<int> fshell;
    for (int s2 = 0; s2 < c->nshells; ++s2)
        for (int k = 0; k < nfunc(basis, s2); ++k) fshell.push_back(s2);
    c->prim_alpha.assign(basis->prim_alpha, basis->prim_alpha + po);
    c->prim_coef.assign(basis->prim_coef, basis->prim_coef + po);
    c->n_rad = g->n_rad;
    c->n_ang = g->n_ang;
    c->ang.assign(g->ang_xyzw, g->ang_xyzw + 4 * (size_t)g->n_ang);
    c->ssf_a = g->partition == XC_PARTITION_SSF ? g->ssf_a : 0.64;
    c->partition = g->partition;
    if (g->partition == XC_PARTITION_BECKE && g->becke_radius)
        c->becke_radius.assign(g->becke_radius, g->becke_radius + c->natoms);
    c->screen_eta = g->screen_eta;
    c->rho_thresh = g->rho_thresh;
    c->batch_max = g->batch_max;
    c->batch_merge = g->batch_merge ? 1 : 0;
    for (int a = 0; a < c->natoms; ++a)
        if (!g->atom_mask || g->atom_mask[a]) c->gatoms.push_back(a);
    hipError_t e = hipGetDevice(&c->device);
    int rc = XC_OK;
    if (e != hipSuccess) rc = hip_fail(e, "hipGetDevice");
    if (rc == XC_OK) rc = upload(c->d_atoms, c->atoms4.data(), 8 * c->atoms4.size(), c->stream);
    if (rc == XC_OK) rc = dev_reserve(c->d_invR, 8 * (size_t)c->natoms * c->natoms);
    if (rc == XC_OK) rc = dev_reserve(c->d_nnhalf, 8 * (size_t)c->natoms);
    if (rc == XC_OK && c->partition == XC_PARTITION_BECKE)
        rc = dev_reserve(c->d_becke_a, 8 * (size_t)c->natoms * c->natoms);
    if (rc == XC_OK && c->natoms > kSsfWaveMaxAtoms && c->natoms <= kNbrMaxAtoms) {
        rc = dev_reserve(c->d_nbr_idx, sizeof(int) * (size_t)c->natoms * c->natoms);
        if (rc == XC_OK) rc = dev_reserve(c->d_nbr_R, 8 * (size_t)c->natoms * c->natoms);
    }
    if (rc == XC_OK) rc = upload(c->d_shells, sh.data(), sizeof(ShellDev) * sh.size(), c->stream);
    if (rc == XC_OK) rc = upload(c->d_palpha, c->prim_alpha.data(), 8 * (size_t)po, c->stream);
    if (rc == XC_OK) rc = upload(c->d_fshell, fshell.data(), sizeof(int) * fshell.size(), c->stream);
    if (rc == XC_OK) rc = upload(c->d_pcoef, c->prim_coef.data(), 8 * (size_t)po, c->stream);
    if (rc == XC_OK) rc = upload(c->d_ang, c->ang.data(), 8 * c->ang.size(), c->stream);
    if (rc == XC_OK) {
        if (c->gatoms.empty()) rc = dev_reserve(c->d_gatoms, sizeof(int));
        else rc = upload(c->d_gatoms, c->gatoms.data(), sizeof(int) * c->gatoms.size(), c->stream);
    }
    if (rc == XC_OK) rc = launch_shell_setup(c);
    if (rc == XC_OK) {
        e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) rc = hip_fail(e, "hipStreamSynchronize");
    }
    if (rc != XC_OK) {
        release_all(c);
        delete c;
        return rc;
    }
    *out = c;
    return XC_OK;
}

int xc_context_build_grid(xc_context* c) {
    g_last_error.clear();
    if (!c) return fail(XC_ERR_INVALID_ARG, "null context");
    return build_grid(c);
}

int xc_context_integrate(xc_context* c, int functional, int precision, const double* dP,
                         double* dV, double* dEN) {
    g_last_error.clear();
    if (!c) return fail(XC_ERR_INVALID_ARG, "null context");
    if (!dP || !dV || !dEN) return fail(XC_ERR_INVALID_ARG, "null device buffer");
    XC_TRY(check_func_prec(functional, precision));
    if (!c->built) XC_TRY(build_grid(c));
    if (functional == XC_MGGA_TPSS) {
        if (!c->meta_plan) {
            c->meta_plan = true;
            XC_TRY(plan_waves(c));
        }
        return run_integrate_meta(c, dP, dV, dEN);
    }
    return run_integrate(c, functional, precision, dP, dV, dEN);
}

int xc_context_integrate_uks(xc_context* c, int functional, int precision, const double* dPa,
                             const double* dPb, double* dVa, double* dVb, double* dEN) {
    g_last_error.clear();
    if (!c) return fail(XC_ERR_INVALID_ARG, "null context");
    if (!dPa || !dPb || !dVa || !dVb || !dEN) return fail(XC_ERR_INVALID_ARG, "null device buffer");
    XC_TRY(check_func_prec(functional, precision));
    if (precision != XC_FP64)
        return fail(XC_ERR_UNSUPPORTED, "spin-unrestricted integrations run in FP64 only");
    if (functional == XC_MGGA_TPSS)
        return fail(XC_ERR_UNSUPPORTED, "meta-GGA integrations are spin-restricted only");
    if (!c->built) XC_TRY(build_grid(c));
    if (!c->spin_plan) {
        c->spin_plan = true;
        XC_TRY(plan_waves(c));
    }
    return run_integrate_uks(c, functional, dPa, dPb, dVa, dVb, dEN);
}

int xc_context_integrate_noalloc(xc_context* c, int functional, int precision,
                                 const double* dP, double* dV, double* dEN) {
    g_last_error.clear();
    if (!c) return fail(XC_ERR_INVALID_ARG, "null context");
    if (!dP || !dV || !dEN) return fail(XC_ERR_INVALID_ARG, "null device buffer");
    XC_TRY(check_func_prec(functional, precision));
    if (functional == XC_MGGA_TPSS)
        return fail(XC_ERR_UNSUPPORTED, "meta-GGA integrations need the allocating entry point");
    if (!c->built) return fail(XC_ERR_STATE, "grid not built (building allocates device memory)");
    return run_integrate_noalloc(c, functional, precision, dP, dV, dEN);
}

int xc_context_stats(xc_context* c, xc_stats* s) {
    g_last_error.clear();
    if (!c || !s) return fail(XC_ERR_INVALID_ARG, "null context or stats");
    std::memset(s, 0, sizeof(*s));
    s->built = c->built ? 1 : 0;
    s->n_points_nominal = (long long)c->n_rad * c->n_ang * (long long)c->gatoms.size();
    if (!c->built) return XC_OK;
    s->n_points = c->n_points;
    s->n_batches = c->n_batches;
    s->n_shell_entries = c->n_shell_entries;
    s->n_func_entries = c->n_func_entries;
    s->max_nb = c->max_nb;
    s->max_ng = c->max_ng;
    s->sum_nb_ng = c->sum_nb_ng;
    s->sum_nb2_ng = c->sum_nb2_ng;
    s->flops_contract = c->flops_contract;
    s->n_waves = (int)c->waves.size();
    s->n_wide_waves = 0;
    for (const Wave& w : c->waves) s->n_wide_waves += w.wide ? 1 : 0;
    size_t pers = 0;
    const DevBuf* bufs[] = {&c->d_atoms, &c->d_invR, &c->d_nnhalf, &c->d_shells,
                            &c->d_palpha, &c->d_pcoef, &c->d_ang, &c->d_gatoms,
                            &c->d_fshell, &c->d_nbr_idx, &c->d_nbr_R, &c->d_becke_a, &c->px, &c->py, &c->pz, &c->pw, &c->pidx, &c->batches,
                            &c->shell_list, &c->shell_loff, &c->func_list, &c->d_wb,
                            &c->d_gemm_pre, &c->d_syr_pre, &c->d_wide_pre, &c->d_tmap, &c->epart,
                            &c->npart, &c->d_req};
    for (const DevBuf* b : bufs) pers += b->cap;
    s->persistent_bytes = pers;
    s->wave_bytes = c->max_wave_bytes;
    return XC_OK;
}

int xc_context_footprint(xc_context* c, size_t* min_bytes, size_t* cached_bytes) {
    g_last_error.clear();
    if (!c) return fail(XC_ERR_INVALID_ARG, "null context");
    size_t mn = 0, all = 0;
    if (c->built) {
        // persistent buffers except those that follow the wave plan (tile
        // map, per-wave tile-count prefixes)
        const DevBuf* bufs[] = {&c->d_atoms, &c->d_invR, &c->d_nnhalf, &c->d_shells,
                                &c->d_palpha, &c->d_pcoef, &c->d_ang, &c->d_gatoms,
                                &c->d_fshell, &c->d_nbr_idx, &c->d_nbr_R, &c->d_becke_a, &c->px, &c->py,
                                &c->pz, &c->pw, &c->pidx, &c->batches, &c->shell_list,
                                &c->shell_loff, &c->func_list, &c->d_wb, &c->epart,
                                &c->npart, &c->d_req};
        size_t core = 0;
        for (const DevBuf* b : bufs) core += b->cap;
        size_t big = 0, sum = 0;
        long long tiles_big = 1, gt_all = 0, st_all = 0;
        for (const WaveBatch& w : c->h_wb) {
            big = std::max(big, batch_scratch_bytes(w));
            sum += batch_scratch_bytes(w);
            tiles_big = std::max<long long>(tiles_big, batch_tiles(w));
            gt_all += (long long)w.nmt * (w.ngp / kTile);
            st_all += (long long)w.nmt * (w.nmt + 1) / 2;
        }
        const size_t nbat = c->h_wb.size();
        // three prefix arrays (64 x 64 and 64 x 128 GEMM tiles, SYR2K tiles) of
        // 1 + batches + waves ints each
        const size_t pre_each = 3 * sizeof(int) * (1 + 2 * nbat);
        const size_t pre_one = 3 * sizeof(int) * (nbat ? nbat + 2 : 1);
        mn = core + pre_each + big + 8 * (size_t)tiles_big;
        all = core + pre_one + sum + 8 * (size_t)std::max<long long>(1, std::max(gt_all, st_all));
    } else {
        // before screening n_b is unknown: bound one batch by the whole basis
        const size_t nbp = (size_t)(c->nbf + kRowPad - 1) / kRowPad * kRowPad;
        const size_t ngp = (size_t)(c->batch_max + kColPad - 1) / kColPad * kColPad;
        const size_t nmt = (size_t)(c->nbf + kTile - 1) / kTile;
        mn = estimate_build_bytes(c) + 8 * (kSlabs * nbp * ngp + nmt * 4 * ngp) +
             8 * nmt * std::max(ngp / kTile, (nmt + 1) / 2);
        all = 0;
    }
    if (min_bytes) *min_bytes = mn;
    if (cached_bytes) *cached_bytes = all;
    return XC_OK;
}

int xc_context_export_grid(xc_context* c, double* xyzw, long long* index) {
    g_last_error.clear();
    if (!c) return fail(XC_ERR_INVALID_ARG, "null context");
    if (!c->built) return fail(XC_ERR_STATE, "grid not built");
    const size_t n = (size_t)c->n_points;
    if (n == 0) return XC_OK;
    std::vector<double> t(n);
    if (xyzw) {
        const DevBuf* comp[4] = {&c->px, &c->py, &c->pz, &c->pw};
        for (int q = 0; q < 4; ++q) {
            XC_HIP(hipMemcpyAsync(t.data(), comp[q]->p, 8 * n, hipMemcpyDeviceToHost, c->stream));
            XC_HIP(hipStreamSynchronize(c->stream));
            for (size_t i = 0; i < n; ++i) xyzw[4 * i + q] = t[i];
        }
    }
    if (index) {
        XC_HIP(hipMemcpyAsync(index, c->pidx.p, 8 * n, hipMemcpyDeviceToHost, c->stream));
        XC_HIP(hipStreamSynchronize(c->stream));
    }
    return XC_OK;
}

int xc_context_export_batches(xc_context* c, long long* point_ptr, double* bbox,
                              long long* shell_ptr, int* shells) {
    g_last_error.clear();
    if (!c) return fail(XC_ERR_INVALID_ARG, "null context");
    if (!c->built) return fail(XC_ERR_STATE, "grid not built");
    const long long nb = c->n_batches;
    for (long long j = 0; j < nb; ++j) {
        const Cell& b = c->h_batches[j];
        if (point_ptr) point_ptr[j] = b.begin;
        if (bbox)
            for (int q = 0; q < 3; ++q) {
                bbox[6 * j + q] = b.lo[q];
                bbox[6 * j + 3 + q] = b.hi[q];
            }
        if (shell_ptr) shell_ptr[j] = c->h_shoff[j];
    }
    if (point_ptr) point_ptr[nb] = c->n_points;
    if (shell_ptr) shell_ptr[nb] = c->n_shell_entries;
    if (shells && c->n_shell_entries > 0) {
        XC_HIP(hipMemcpyAsync(shells, c->shell_list.p, sizeof(int) * c->n_shell_entries,
                              hipMemcpyDeviceToHost, c->stream));
        XC_HIP(hipStreamSynchronize(c->stream));
    }
    return XC_OK;
}

int xc_context_set_timing(xc_context* c, int enable) {
    g_last_error.clear();
    if (!c) return fail(XC_ERR_INVALID_ARG, "null context");
    XC_TRY(fold_timer(c));
    c->timer.enabled = enable != 0;
    for (int p = 0; p < XC_NUM_PHASES; ++p) {
        c->timer.ms[p] = 0.0;
        c->timer.launches[p] = 0;
    }
    return XC_OK;
}

int xc_context_set_phi_cache(xc_context* c, int enable) {
    g_last_error.clear();
    if (!c) return fail(XC_ERR_INVALID_ARG, "null context");
    c->phi_cache = enable != 0;
    if (!c->phi_cache) c->phi_cached_kind = 0;
    return XC_OK;
}

int xc_context_timing(xc_context* c, xc_timing* out) {
    g_last_error.clear();
    if (!c || !out) return fail(XC_ERR_INVALID_ARG, "null context or timing");
    XC_TRY(fold_timer(c));
    for (int p = 0; p < XC_NUM_PHASES; ++p) {
        out->ms[p] = c->timer.ms[p];
        out->launches[p] = c->timer.launches[p];
    }
    return XC_OK;
}

int xc_context_destroy(xc_context* c) {
    if (!c) return XC_OK;
    (void)hipStreamSynchronize(c->stream);
    destroy_timer(c->timer);
    release_all(c);
    delete c;
    return XC_OK;
}

int xc_integrate(const xc_molecule* mol, const xc_basis* basis, const xc_grid_spec* g,
                 int functional, int precision, const double* P, int nbf, double* E_xc,
                 double* N_e, double* V) {
    g_last_error.clear();
    XC_TRY(validate_inputs(mol, basis, g));
    XC_TRY(check_func_prec(functional, precision));
    if (!P || !V || !E_xc || !N_e) return fail(XC_ERR_INVALID_ARG, "null P, V, E_xc or N_e");
    int want = 0;
    for (int s = 0; s < basis->nshells; ++s) want += nfunc(basis, s);
    if (nbf != want) return fail(XC_ERR_INVALID_ARG, "nbf does not match the basis");
    xc_context* c = nullptr;
    XC_TRY(xc_context_create(mol, basis, g, nullptr, &c));
    const size_t mb = 8 * (size_t)nbf * nbf;
    DevBuf dP, dV, dEN;
    c->meta_plan = functional == XC_MGGA_TPSS;   // planned with the meta-GGA extras
    int rc = build_grid(c);
    if (rc == XC_OK) rc = upload(dP, P, mb, c->stream);
    if (rc == XC_OK) rc = dev_reserve(dV, mb);
    if (rc == XC_OK) rc = dev_reserve(dEN, 16);
    if (rc == XC_OK)
        rc = functional == XC_MGGA_TPSS
                 ? run_integrate_meta(c, (const double*)dP.p, (double*)dV.p, (double*)dEN.p)
                 : run_integrate(c, functional, precision, (const double*)dP.p, (double*)dV.p,
                                 (double*)dEN.p);
    double en[2] = {0.0, 0.0};
    std::vector<double> hv;
    if (rc == XC_OK) {
        hv.resize((size_t)nbf * nbf);
        hipError_t e = hipMemcpyAsync(hv.data(), dV.p, mb, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipMemcpyAsync(en, dEN.p, 16, hipMemcpyDeviceToHost, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) rc = hip_fail(e, "copy of V, E, N to host");
    }
    dev_release(dP);
    dev_release(dV);
    dev_release(dEN);
    xc_context_destroy(c);
    if (rc != XC_OK) return rc;
    std::memcpy(V, hv.data(), mb);
    *E_xc = en[0];
    *N_e = en[1];
    return XC_OK;
}

}  // extern "C"
