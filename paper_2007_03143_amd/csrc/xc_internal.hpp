// Internal declarations shared by the HIP sources of the XC library.
// Device structures, the context, and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "xc.h"

namespace xc {

// ---------------------------------------------------------------- errors --
// Set the calling thread's error message and return code.
int fail(int code, const std::string& msg);
// Map a HIP status to XC_ERR_DEVICE with a message naming the call site.
int hip_fail(hipError_t e, const char* what);

#define XC_HIP(call)                                           \
    do {                                                       \
        hipError_t e_ = (call);                                \
        if (e_ != hipSuccess) return ::xc::hip_fail(e_, #call); \
    } while (0)

#define XC_TRY(call)                \
    do {                            \
        int r_ = (call);            \
        if (r_ != XC_OK) return r_; \
    } while (0)

// ------------------------------------------------------ device structures --
constexpr int kMaxL = 3;
constexpr int kMaxPrim = 16;
constexpr int kMaxBatch = 1024;     // largest batch_max accepted
constexpr int kTile = 64;           // contraction tile edge (rows and columns)
constexpr int kRowPad = 16;         // n_b is stored padded to a multiple of this
constexpr int kColPad = 64;         // n_g is stored padded to a multiple of this
constexpr int kSsfWaveMaxAtoms = 1024;  // partition with one wave per point up to this many atoms
constexpr int kNbrMaxAtoms = 4096;  // beyond that, distance-ordered neighbour lists up to this many

// One basis shell as the kernels read it.
struct ShellDev {
    double x, y, z;     // centre
    double rcut2;       // squared cutoff radius (eq. rcut); +inf: no truncation
    int L;
    int nprim;
    int prim_off;       // first primitive in the packed exponent/coefficient arrays
    int first_func;     // global index of the shell's first function
    int pure;           // 1: 2L+1 real solid harmonics (only for L >= 2); 0: Cartesian
    int pad_;
};

// Functions of a shell: 2L+1 spherical or (L+1)(L+2)/2 Cartesian.
__host__ __device__ inline int shell_nfunc(int L, int pure) {
    return pure ? 2 * L + 1 : (L + 1) * (L + 2) / 2;
}

// A cuboid cell of points during batching, and a finished batch.
struct Cell {
    long long begin;    // first point (into the compacted point arrays)
    int count;
    int atom;           // parent atom
    double lo[3];
    double hi[3];
};

// Per-batch wave scratch: the Phi slab (n_bp x n_gp, FP64 size whatever the
// storage type) and one row of per-point digit scales (split-BF16 mode), the
// Z slab (n_bp x n_gp), then the rho / grad rho partials. Phi and its scale
// row may instead live in a request's own Phi store (ReqDev::phi_base).
constexpr int kSlabs = 2;

// One batch as the integration kernels of a wave read it.
struct WaveBatch {
    long long phi_off;  // offset (doubles) of its Phi slab, from the request's Phi
                        // store if it has one, else from the wave scratch
    long long z_off;    // offset (doubles) of its Z slab in the wave scratch
    long long part_off; // offset (doubles) of its density partials in the wave scratch
    long long pt_off;   // first point
    long long shell_off;// first entry in the shell list
    long long func_off; // first entry in the function list
    int nb;             // screened function count n_b
    int nbp;            // n_b padded to kRowPad
    int ng;             // point count n_g
    int ngp;            // n_g padded to kColPad
    int nmt;            // row tiles: ceil(n_b / kTile)
    int nshell;
    int batch;          // batch index within its request
    int req;            // index of the request descriptor (ReqDev) of the launch
    int flags;          // kSkipColloc: Phi of this batch is already in place
    int pad_;
};
constexpr int kSkipColloc = 1;

// Bytes of a batch's Phi slab and scale row.
inline size_t batch_phi_bytes(const WaveBatch& w) {
    return 8 * ((size_t)w.nbp * w.ngp + w.ngp);
}
// Bytes of a batch's Z slab and density partials (four per row tile and
// padded point).
inline size_t batch_zpart_bytes(const WaveBatch& w) {
    return 8 * ((size_t)w.nbp * w.ngp + (size_t)w.nmt * 4 * w.ngp);
}
// Wave-scratch bytes of one batch whose Phi lives in the scratch too.
inline size_t batch_scratch_bytes(const WaveBatch& w) {
    return batch_phi_bytes(w) + batch_zpart_bytes(w);
}

// Extra wave-scratch bytes of one batch for spin-unrestricted integrations:
// a second set of density partials (the beta spin's), after the first.
inline size_t batch_spin_bytes(const WaveBatch& w) {
    return 8 * (size_t)w.nmt * 4 * w.ngp;
}

// Extra wave-scratch bytes of one batch for meta-GGA integrations, after
// its Phi, Z and partials: the three gradient slabs d phi/dx, /dy, /dz, then
// three sets of partials for the kinetic energy density (set d from the
// contraction of P with the d-th gradient slab).
inline size_t batch_meta_bytes(const WaveBatch& w) {
    return 8 * 3 * ((size_t)w.nbp * w.ngp + (size_t)w.nmt * 4 * w.ngp);
}
// Offsets (doubles, in the wave scratch) of gradient slab d and of partial
// set d of a batch in a meta-GGA plan.
__host__ __device__ inline long long meta_base_off(const WaveBatch& w) {
    return w.part_off + (long long)w.nmt * 4 * w.ngp;
}
__host__ __device__ inline long long meta_grad_off(const WaveBatch& w, int d) {
    return meta_base_off(w) + (long long)d * w.nbp * w.ngp;
}
__host__ __device__ inline long long meta_part_off(const WaveBatch& w, int d) {
    return meta_base_off(w) + 3LL * w.nbp * w.ngp + (long long)d * w.nmt * 4 * w.ngp;
}

// Offset (doubles, from the batch's Phi slab) of its per-point digit scales.
__host__ __device__ inline long long scale_row_off(const WaveBatch& w) {
    return (long long)w.nbp * w.ngp;
}

// A launch of FP64 density tiles uses 64 x 128 tiles when the work-weighted
// mean n_b of its batches, sum n_b^2 n_g / sum n_b n_g, is at least this.
constexpr double kWideNb = 512.0;

// Density tiles of a batch for the FP64 kernel: 64 rows x 128 points.
inline int batch_wide_tiles(const WaveBatch& w) {
    return w.nmt * ((w.ngp + 127) / 128);
}

// Larger of the batch's density-GEMM and potential-SYR2K tile counts.
inline int batch_tiles(const WaveBatch& w) {
    const int gt = w.nmt * (w.ngp / kTile), st = w.nmt * (w.nmt + 1) / 2;
    return gt > st ? gt : st;
}

// Everything a launch needs about the request (context + one integration)
// a batch belongs to; a launch may mix batches of many requests.
struct ReqDev {
    const ShellDev* shells;
    const double* palpha;
    const double* pcoef;
    const int* shell_list;
    const int* shell_loff;
    const int* func_list;
    const int* func_shell;   // global shell of every global function
    const double* px;
    const double* py;
    const double* pz;
    const double* pw;
    const double* P;
    double* V;
    double* epart;
    double* npart;
    const unsigned long long* Pdig;  // split-BF16 mode: four BF16 digits per entry of P
    const double* Pscale;            // and the power-of-two scale of each row of P
    char* phi_base;                  // the request's Phi store, or null (Phi in the scratch)
    double rho_thresh;
    int nbf;
    int pad_;
};

struct Wave {
    int first;          // first batch (global index)
    int count;          // number of batches
    int gemm_tiles;     // 64 x 64 density tiles (FP32 and split-BF16 kernels)
    int syr_tiles;
    int wide_tiles;     // 64 x 128 density tiles (FP64 kernel)
    bool wide;          // FP64 density tiles of 64 x 128 (else 64 x 64)
    long long wb_off;   // offset into the WaveBatch array
    long long pre_off;  // offset into the tile-prefix arrays (count + 1 entries)
    size_t scratch_bytes;
};

// ------------------------------------------------------------- context ----
// A caller-supplied device allocator (both callbacks set).
struct DevAlloc {
    xc_alloc_fn alloc = nullptr;
    xc_free_fn free = nullptr;
    void* user = nullptr;
};

// A device buffer; memory from `al` when set, else from hipMalloc.
struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
    const DevAlloc* al = nullptr;
};

// HIP-event phase timer: pairs of events recorded around launches, folded
// into milliseconds when the caller asks for the totals.
struct PhaseTimer {
    bool enabled = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending[XC_NUM_PHASES];
    std::vector<hipEvent_t> pool;
    double ms[XC_NUM_PHASES] = {};
    long long launches[XC_NUM_PHASES] = {};
};

}  // namespace xc

struct xc_context {
    hipStream_t stream = nullptr;
    int device = 0;
    xc::DevAlloc alloc;          // the caller's allocator (alloc == nullptr: hipMalloc)

    // inputs (host copies)
    int natoms = 0;
    std::vector<double> atoms4;       // x, y, z, mk_alpha per atom
    int nshells = 0;
    std::vector<int> shell_atom, shell_L, shell_nprim, shell_pure, prim_off, first_func;
    std::vector<double> prim_alpha, prim_coef;
    int nbf = 0;
    bool any_pure = false;            // some shell is spherical
    int n_rad = 0, n_ang = 0;
    std::vector<double> ang;          // n_ang x 4
    double ssf_a = 0.64, screen_eta = 1e-10, rho_thresh = 1e-15;
    int partition = XC_PARTITION_SSF;
    std::vector<double> becke_radius;  // empty: no size adjustment
    int batch_max = 512;
    int batch_merge = 1;
    std::vector<int> gatoms;          // parent atoms whose grids are built
    size_t wave_budget = 0;

    // device inputs
    xc::DevBuf d_atoms, d_invR, d_nnhalf, d_shells, d_palpha, d_pcoef, d_ang, d_gatoms;
    xc::DevBuf d_fshell;
    xc::DevBuf d_nbr_idx, d_nbr_R;  // per atom: all atoms by distance
    xc::DevBuf d_becke_a;           // Becke size adjustments a_AB (natoms x natoms)

    // grid and batches
    bool built = false;
    long long n_nominal = 0, n_points = 0;
    xc::DevBuf raw_x, raw_y, raw_z, raw_w;                 // unpruned grid
    xc::DevBuf px, py, pz, pw, pidx, tx, ty, tz, tw, tidx;  // compacted (batch order) + temp
    xc::DevBuf blk_count, blk_off, atom_count;
    xc::DevBuf cells_a, cells_b, child_count, child_begin, batches, counters;
    std::vector<xc::Cell> h_batches;
    long long n_batches = 0;
    xc::DevBuf scr_nsh, scr_nfn, scr_shoff, scr_fnoff;
    xc::DevBuf shell_list, shell_loff, func_list;
    long long n_shell_entries = 0, n_func_entries = 0;
    std::vector<int> h_nsh, h_nfn;
    std::vector<long long> h_shoff, h_fnoff;

    // wave plan
    std::vector<xc::Wave> waves;
    std::vector<xc::WaveBatch> h_wb;
    xc::DevBuf d_wb, d_gemm_pre, d_syr_pre, d_wide_pre;
    xc::DevBuf d_tmap;           // tile -> (batch, tile in batch) of one launch
    xc::DevBuf scratch;
    size_t max_wave_bytes = 0;
    int max_tiles = 1;           // most tiles of one contraction launch in any wave
    bool spin_plan = false;      // batches carry a second (beta) set of partials
    std::vector<xc::WaveBatch> h_wb_beta;
    xc::DevBuf d_wb_beta;        // the batches with the beta partials and request 1
    bool meta_plan = false;      // batches carry gradient slabs and kinetic-energy partials
    std::vector<xc::WaveBatch> h_wb_meta;
    xc::DevBuf d_wb_meta;        // three copies of the batches (d = x, y, z): Phi slab ->
                                 // gradient slab d, partials -> partial set d
    xc::DevBuf epart, npart;
    xc::DevBuf d_req;            // one ReqDev for the context's own integrations
    xc::DevBuf pdig, pscale;     // digits and row scales of P (split-BF16 mode)
    bool external_scratch = false;  // wave scratch supplied by an engine
    bool phi_cache = false;         // keep Phi in the scratch between integrations
    int phi_cached_kind = 0;        // phi_kind() of the Phi the scratch holds; 0: none

    xc::PhaseTimer timer;

    // statistics
    int max_nb = 0, max_ng = 0;
    double sum_nb_ng = 0, sum_nb2_ng = 0, flops_contract = 0;
};

namespace xc {

// Brackets the launches issued during its lifetime with timer events when
// the context's timer is on.
class PhaseScope {
  public:
    PhaseScope(xc_context* c, int phase);
    PhaseScope(PhaseTimer* t, hipStream_t s, int phase);
    ~PhaseScope();

  private:
    PhaseTimer* t_;
    hipStream_t s_;
    int phase_;
    hipEvent_t e0_ = nullptr;
};

// device memory helpers (context stream ordered where relevant)
int dev_reserve(DevBuf& b, size_t bytes);
void dev_release(DevBuf& b);
int upload(DevBuf& b, const void* src, size_t bytes, hipStream_t s);

// abi.cpp
int build_grid(xc_context* c);
void release_build_temporaries(xc_context* c);
size_t device_bytes(const xc_context* c);
// Device bytes an unbuilt context is expected to need for its build and its
// persistent data (no wave scratch): an estimate from the nominal grid size
// and the basis size.
size_t estimate_build_bytes(const xc_context* c);

// grid.hip
int launch_shell_setup(xc_context* c);
int launch_grid_points(xc_context* c);
int launch_ssf(xc_context* c);
int launch_compact(xc_context* c, std::vector<long long>& atom_kept);

// batching.hip
int run_batching(xc_context* c, const std::vector<long long>& atom_kept);
int run_screening(xc_context* c);

// integrate.hip
int run_integrate(xc_context* c, int functional, int precision, const double* dP,
                  double* dV, double* dEN);
// Request descriptor of an integration of context c with the given buffers.
ReqDev make_req(const xc_context* c, const double* dP, double* dV);
// Write one request descriptor to device memory with a one-thread kernel (the
// descriptor travels as a kernel argument: no host staging buffer).
int launch_put_req(hipStream_t s, ReqDev* dst, const ReqDev& v);
// The per-wave launches (collocation, density, functional, Z,
// potential) over count batches whose descriptors are already on the device.
// d_tmap: room for 2 * max(gemm_tiles, syr_tiles) ints (tile -> batch map).
// colloc = false skips the collocation kernel: the scratch already holds Phi
// of these batches in the storage type of this precision. sph: some batch of
// the launch has spherical shells (selects the Z kernel that forms them).
// wide: FP64 density tiles of 64 x 128 (d_wpre, wide_tiles), else 64 x 64
// (d_gpre, gemm_tiles); the FP32 and split-BF16 density kernels use 64 x 64.
int launch_wave(PhaseTimer* timer, hipStream_t s, bool gga, int precision,
                const WaveBatch* d_wb, const int* d_gpre, const int* d_spre,
                const int* d_wpre, int count, int gemm_tiles, int syr_tiles,
                int wide_tiles, bool wide, const ReqDev* d_reqs,
                char* scratch, int* d_tmap, bool colloc, bool sph);
// Meta-GGA (TPSS) integration of a context planned with meta_plan: FP64,
// P in, V and (E_xc, N_e) out.
int run_integrate_meta(xc_context* c, const double* dP, double* dV, double* dEN);
// Spin-unrestricted integration (FP64) of a context planned with
// spin_plan: P^a, P^b in, V^a, V^b and (E_xc, N_e) out.
int run_integrate_uks(xc_context* c, int functional, const double* dPa, const double* dPb,
                      double* dVa, double* dVb, double* dEN);
// noalloc.hip: the integration with its wave scratch, tile map and request
// descriptor in the library's static device array (no allocation).
int run_integrate_noalloc(xc_context* c, int functional, int precision, const double* dP,
                          double* dV, double* dEN);
// What the collocation kernel stores under a precision code: 1 Phi in FP64,
// 2 Phi in FP32, 3 Phi in FP64 with per-point digit scales (split BF16).
int phi_kind(int precision);
// Split-BF16 digits and row scales of the nbf x nbf density matrix P.
int launch_p_digits(hipStream_t s, const double* P, int nbf, unsigned long long* dig,
                    double* scale);
// Fill n doubles with v (a kernel, so it can be captured in a graph).
int launch_fill(hipStream_t s, double* p, long long n, double v);
// V mirror and the fixed-order E_xc / N_e sums of one finished integration.
int launch_finish(PhaseTimer* timer, hipStream_t s, double* dV, int nbf,
                  const double* epart, const double* npart, long long nbatch,
                  double* dEN);

}  // namespace xc
