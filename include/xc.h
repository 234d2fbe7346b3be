/*
 * xc.h - C ABI of the MI355X (gfx950) library for the numerical integration
 * of the Kohn-Sham exchange-correlation energy E_xc and potential matrix V_xc
 * over an atom-centred molecular grid in a Cartesian Gaussian basis
 * (arXiv 2007.03143, Sec. 2.1-2.3).
 *
 * What one integration computes (Sec. 2.1 eq. vxc_exact, eq. zvec_r;
 * Sec. 2.2 eq. exc_batch, eq. vxc_inc, eq. vxc_batch, eq. z_mat):
 *
 *   rho_i   = sum_{mu nu} P_{mu nu} phi~_mu(r_i) phi~_nu(r_i)
 *   grad_i  = 2 sum_{mu nu} P_{mu nu} grad phi~_mu(r_i) phi~_nu(r_i)
 *   sigma_i = |grad_i|^2
 *   E_xc    = sum_i w_i e(rho_i, sigma_i)        (points with rho_i >= rho_thresh)
 *   N_e     = sum_i w_i rho_i                     (all points)
 *   V_{mu nu} = sum_i w_i [ v_rho phi~_mu phi~_nu
 *                 + 2 v_sigma grad_i . (phi~_mu grad phi~_nu + grad phi~_mu phi~_nu) ]
 *
 * with e = rho * eps the energy per unit volume, v_rho = de/drho,
 * v_sigma = de/dsigma, phi~ the basis function truncated at its shell's
 * cutoff radius (Sec. 2.2 eq. rcut) and w_i the Stratmann-Scuseria-Frisch
 * scaled weights of the Mura-Knowles x Lebedev product grid
 * (Sec. 2.2 eq. atomic_partition, eq. num_int).
 *
 * Units: bohr and hartree. Matrices are row-major nbf x nbf FP64.
 *
 * Errors: every function returns XC_OK (0) or a negative code; on error no
 * output is written and xc_last_error() returns a message for the calling
 * thread. No C++ exception crosses this boundary.
 *
 * Threading: one context must not be used from two threads at once;
 * distinct contexts are independent.
 */
#ifndef XC_MI355X_H
#define XC_MI355X_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define XC_ABI_VERSION 3

/* return codes */
#define XC_OK               0
#define XC_ERR_INVALID_ARG (-1)  /* a pointer, size or value is out of range */
#define XC_ERR_UNSUPPORTED (-2)  /* L > 3, nprim > 16, unknown functional or precision */
#define XC_ERR_NOMEM       (-3)  /* device memory exhausted or budget too small */
#define XC_ERR_DEVICE      (-4)  /* a HIP runtime call or kernel launch failed */
#define XC_ERR_STATE       (-5)  /* call not valid in the context's current state */
#define XC_ERR_BUSY        (-6)  /* the object still has work in flight (retry later) */

/* exchange-correlation functionals (spin-unpolarised) */
#define XC_LDA_SVWN5 1   /* Slater exchange + VWN5 correlation */
#define XC_GGA_PBE   2   /* PBE exchange + PBE correlation (PW92 base) */
#define XC_MGGA_TPSS 3   /* TPSS meta-GGA (Tao, Perdew, Staroverov, Scuseria 2003):
                            e(rho, sigma, tau) with the kinetic energy density
                            tau = 1/2 sum P_mn grad phi_m . grad phi_n, the extension
                            Sec. 2.1 notes needs only a few more intermediates; V adds
                            sum_i w_i v_tau grad phi_m . grad phi_n / 2. XC_FP64 only,
                            spin-restricted only; z = tau_W/tau is held at 1 where
                            tau < tau_W. The first such call on a context re-plans its
                            waves with room for three gradient slabs and three more
                            sets of partials per batch (allocates); not available
                            through xc_context_integrate_noalloc or the engine. */

/* arithmetic of the collocation and the two batched contractions */
#define XC_FP64          0   /* everything FP64 */
#define XC_MIXED_FP32    1   /* Phi and Z formed in FP64 and stored in FP32; both
                                contractions on FP32 MFMA with FP32 accumulation;
                                FP64 functional, Z formation, E_xc/N_e sums and V
                                accumulation */
#define XC_MIXED_BF16    2   /* split BF16 on BF16 MFMA (v_mfma_f32_16x16x32_bf16) with
                                FP32 accumulation in both contractions. Density
                                contraction X = P^j Phi^j (eq. x_mat): every row of P
                                and every point's column of Phi is scaled by a power
                                of two and cut into four signed 8-bit digits (the
                                first 7 bits), so digit products are exact and their
                                FP32 sums stay exact up to 128 terms, after which
                                they are added into FP64: X carries about 31 bits
                                relative to the largest entry of its row of P and
                                point's column of Phi (10 digit products per FP64
                                product). Potential contraction: Phi (FP64) and Z
                                (FP32) split as hi + lo BF16, products
                                hi hi + hi lo + lo hi (about 16 bits). Collocation
                                and Phi in FP64; FP64 functional, Z formation,
                                E_xc/N_e sums and V accumulation */
#define XC_MIXED_FP32_V  3   /* FP64 collocation and density contraction, so E_xc, N_e
                                and the functional inputs are as in XC_FP64; Z and the
                                V^j contraction in FP32 (FP32 MFMA, FP32 accumulate),
                                V accumulated in FP64 */

/*
 * Atoms (Sec. 2.2, eq. atomic_partition): centres R_A in bohr (natoms x 3,
 * row-major) and the Mura-Knowles radial scale alpha_A of each atom's grid.
 * Borrowed for the duration of the call only.
 */
typedef struct xc_molecule {
    int natoms;
    const double* xyz;        /* natoms x 3 */
    const double* mk_alpha;   /* natoms, > 0 */
} xc_molecule;

/*
 * Contracted Gaussian shells (Sec. 2.1, eq. gau_cart). Shell s sits on atom
 * shell_atom[s], has angular momentum shell_L[s] (0..3) and shell_nprim[s]
 * (1..16) primitives; exponents and coefficients are packed in shell order
 * and the coefficients are used as given (no normalisation is applied).
 * A Cartesian shell holds (L+1)(L+2)/2 functions ordered xx, xy, xz, yy, yz,
 * zz (for L = 2; lexicographic in general). A spherical shell (shell_pure[s]
 * = 1 and L >= 2; Sec. 2.1's spherical-harmonic combinations, as in the
 * cc-pVDZ basis sets of Table 1) holds the 2L+1 real solid harmonics
 * S_{L,m}(r - R) times the same radial factor, m = -L..L, Racah-normalised
 * (the integral of S_{L,m}^2 over the unit sphere is 4 pi / (2L+1), that of
 * x^L): for L = 2, sqrt3 xy, sqrt3 yz, z^2 - (x^2+y^2)/2, sqrt3 xz,
 * sqrt3/2 (x^2-y^2). Shells with L <= 1 are Cartesian whatever their flag.
 * shell_pure may be NULL (every shell Cartesian). The global function order
 * is shell order. Borrowed for the duration of the call only.
 */
typedef struct xc_basis {
    int nshells;
    const int* shell_atom;
    const int* shell_L;
    const int* shell_nprim;
    const double* prim_alpha;   /* sum(nprim), > 0 */
    const double* prim_coef;    /* sum(nprim) */
    const int* shell_pure;      /* nshells flags 0/1, or NULL */
} xc_basis;

/*
 * Grid specification (Sec. 2.2; Table 2 shapes; eq. rcut; batch threshold).
 *  n_rad       radial points per atom, Mura-Knowles r = -alpha ln(1 - x^3)
 *              on midpoint nodes x_k = (k - 1/2)/n_rad
 *  n_ang       angular points per atom
 *  ang_xyzw    n_ang x 4: unit vector and weight (weights sum to 4 pi)
 *  ssf_a       Stratmann-Scuseria-Frisch cell parameter, 0 < a < 1 (0.64)
 *  screen_eta  eq. rcut tolerance eta; 0 disables truncation and screening
 *  batch_max   largest number of points in one batch, 16..1024 (512)
 *  rho_thresh  points with rho below it add nothing to E_xc and V_xc
 *  atom_mask   NULL, or natoms flags: only the grids of flagged parent atoms
 *              are integrated (the partition still uses every atom)
 *  batch_merge 0: every non-empty cuboid of the recursive split is a batch;
 *              1: consecutive small sibling cuboids are joined while the
 *              joined count stays <= batch_max (fewer, fuller batches; the
 *              result is the same either way)
 *  partition   XC_PARTITION_SSF: Stratmann-Scuseria-Frisch (the paper's
 *              choice, Sec. 2.2); XC_PARTITION_BECKE: Becke's partition (one
 *              of the choices Sec. 2.2 lists; J. Chem. Phys. 88, 2547 (1988)):
 *              s(nu) = (1 - p(p(p(nu))))/2 with p(x) = 3x/2 - x^3/2 and
 *              nu_AB = mu_AB + a_AB (1 - mu_AB^2), P_A = prod_{B != A} s(nu_AB),
 *              p_A = P_A / sum_B P_B. Becke needs natoms <= 1024
 *              (XC_ERR_UNSUPPORTED otherwise); ssf_a is then ignored.
 *  becke_radius NULL (a_AB = 0), or natoms atomic radii for Becke's size
 *              adjustment: chi = R_A / R_B, u = (chi - 1)/(chi + 1),
 *              a_AB = u / (u^2 - 1) clipped to [-1/2, 1/2] (only ratios
 *              matter; > 0). Ignored for SSF.
 */
#define XC_PARTITION_SSF   0
#define XC_PARTITION_BECKE 1
typedef struct xc_grid_spec {
    int n_rad;
    int n_ang;
    const double* ang_xyzw;
    double ssf_a;
    double screen_eta;
    int batch_max;
    double rho_thresh;
    const unsigned char* atom_mask;
    int batch_merge;
    int partition;
    const double* becke_radius;
} xc_grid_spec;

/*
 * Device options for a context.
 *  stream      hipStream_t every launch and copy of the context is ordered
 *              on (NULL: the null stream). The library never changes stream
 *              priorities.
 *  wave_bytes  budget of device scratch for one wave of batches (the
 *              subsets of batches that fill the device memory, Alg. 2); 0:
 *              min(half the free device memory, 48 GiB).
 *  alloc, free caller-supplied device allocator (a framework's caching
 *              allocator, an arena of its own), both set or both NULL
 *              (NULL: hipMalloc and hipFree). Every device buffer the
 *              context holds is obtained with alloc(bytes, alloc_user),
 *              which returns a device pointer to at least `bytes` bytes or
 *              NULL on failure, and is given back with free(ptr,
 *              alloc_user) when it grows, on xc_context_release and on
 *              xc_context_destroy (after the context's stream has been
 *              synchronised there). The library uses the memory on the
 *              context's stream only; an allocator that hands out
 *              stream-ordered memory must tie it to that stream. A NULL
 *              from alloc makes the call that needed the memory return
 *              XC_ERR_NOMEM; the context stays valid and can be released or
 *              destroyed. The callbacks run on the calling thread, inside
 *              the library's entry points; they must not call back into
 *              the same context.
 */
typedef void* (*xc_alloc_fn)(size_t bytes, void* user);
typedef void (*xc_free_fn)(void* ptr, void* user);

typedef struct xc_device_opts {
    void* stream;
    size_t wave_bytes;
    xc_alloc_fn alloc;
    xc_free_fn free;
    void* alloc_user;
} xc_device_opts;

/* Sizes of a built grid; all counts refer to the points actually integrated. */
typedef struct xc_stats {
    long long n_points_nominal;  /* masked atoms x n_rad x n_ang */
    long long n_points;          /* points with non-zero weight */
    long long n_batches;
    long long n_shell_entries;   /* sum over batches of the screened shell count */
    long long n_func_entries;    /* sum over batches of n_b */
    int max_nb;
    int max_ng;
    double sum_nb_ng;            /* sum_j n_b^j n_g^j */
    double sum_nb2_ng;           /* sum_j (n_b^j)^2 n_g^j */
    double flops_contract;       /* algorithmic FP64 flops of the two contractions
                                    per integration: sum_j 2 n_b^2 n_g + 2 n_b (n_b+1) n_g */
    int n_waves;
    int built;                   /* 1 once xc_context_build_grid has run */
    size_t persistent_bytes;     /* device bytes held between integrations */
    size_t wave_bytes;           /* device scratch bytes of the largest wave */
    int n_wide_waves;            /* waves whose FP64 density tiles are 64 x 128 (their
                                    work-weighted mean n_b, sum n_b^2 n_g / sum n_b n_g,
                                    is at least 512); the others use 64 x 64 */
} xc_stats;

/*
 * Per-phase device time, measured with HIP events recorded on the
 * context's stream around each phase's launches (the component split of the
 * paper's profile: weights, collocation, the two contractions, the
 * functional, the rest). Phases:
 */
#define XC_PHASE_GRID       0   /* grid points */
#define XC_PHASE_WEIGHTS    1   /* SSF partition weights */
#define XC_PHASE_COMPACT    2   /* removal of zero-weight points */
#define XC_PHASE_BATCH      3   /* cuboid batching */
#define XC_PHASE_SCREEN     4   /* shell screening (Alg. 1) */
#define XC_PHASE_COLLOC     5   /* collocation Phi (grad Phi is re-evaluated where used) */
#define XC_PHASE_DENSITY    6   /* X = P Phi on MFMA with rho, grad rho epilogue */
#define XC_PHASE_FUNCTIONAL 7   /* functional, E_xc/N_e partials, Z */
#define XC_PHASE_POTENTIAL  8   /* V = Z Phi^T + Phi Z^T on MFMA with scatter-add */
#define XC_PHASE_OTHER      9   /* zero fill, mirror, final sums */
#define XC_NUM_PHASES      10

typedef struct xc_timing {
    double ms[XC_NUM_PHASES];          /* accumulated device milliseconds */
    long long launches[XC_NUM_PHASES]; /* timed intervals (one per launch or phase) */
} xc_timing;

typedef struct xc_context xc_context;

/* Static message for a return code. */
const char* xc_strerror(int code);
/* Message describing the calling thread's most recent error ("" if none). */
const char* xc_last_error(void);
/* XC_ABI_VERSION of the loaded library. */
int xc_abi_version(void);

/*
 * One-shot integration with host buffers: builds the grid, integrates and
 * releases every device resource before returning. P (nbf x nbf, symmetric)
 * is read; V (nbf x nbf) is written in full and exactly symmetric; *E_xc and
 * *N_e are written. nbf must equal the basis function count. Synchronous.
 */
int xc_integrate(const xc_molecule* mol, const xc_basis* basis,
                 const xc_grid_spec* grid, int functional, int precision,
                 const double* P, int nbf,
                 double* E_xc, double* N_e, double* V);

/*
 * Create a context that keeps atoms, shells and (after build) the grid,
 * weights, batches and screening lists on the device across integrations
 * (grid reuse across Fock builds, Sec. 2.3.1). Inputs are copied; the caller
 * keeps ownership of everything it passed. *out receives the new context.
 */
int xc_context_create(const xc_molecule* mol, const xc_basis* basis,
                      const xc_grid_spec* grid, const xc_device_opts* opts,
                      xc_context** out);

/*
 * Build or rebuild the grid on the device (grid points, SSF weights, removal
 * of zero-weight points, cuboid batching, shell screening by Alg. 1, wave
 * plan). Synchronises the context's stream to learn sizes. A rebuild of an
 * unchanged context reuses its allocations and gives the same batches.
 */
int xc_context_build_grid(xc_context* ctx);

/*
 * Integrate with device buffers, ordered on the context's stream and
 * asynchronous with respect to the host (no synchronisation inside once the
 * grid is built; builds it first otherwise).
 *  d_P   nbf x nbf FP64 density matrix in device memory (read)
 *  d_V   nbf x nbf FP64 in device memory (overwritten with V_xc)
 *  d_EN  2 FP64 in device memory (overwritten with E_xc, N_e)
 */
int xc_context_integrate(xc_context* ctx, int functional, int precision,
                         const double* d_P, double* d_V, double* d_EN);

/*
 * Spin-unrestricted integration (the extension Sec. 2.1 notes needs only a
 * few more intermediates): two density matrices P^a, P^b (nbf x nbf FP64,
 * device) give rho_a, rho_b, sigma_aa, sigma_ab, sigma_bb and
 *   E_xc = sum_i w_i e(rho_a, rho_b, sigma_aa, sigma_ab, sigma_bb)
 *   V^a = sum_i w_i [ v_rho_a phi phi^T + (2 v_sigma_aa grad rho_a
 *         + v_sigma_ab grad rho_b) . (phi grad phi^T + grad phi phi^T) ]
 * and V^b likewise (both written in full, exactly symmetric); d_EN receives
 * E_xc and N_e (both spins). Functionals: Slater exchange by spin scaling +
 * VWN5 with its spin interpolation (XC_LDA_SVWN5); PBE by spin scaling +
 * PBE correlation on the spin-interpolated PW92 (XC_GGA_PBE). A point adds
 * nothing when rho_a + rho_b < rho_thresh, a spin's exchange nothing when
 * its density is below rho_thresh, and zeta = (rho_a - rho_b)/rho is held
 * within [-1 + 1e-10, 1 - 1e-10]. Precision: XC_FP64 only
 * (XC_ERR_UNSUPPORTED otherwise). The first such call re-plans the waves of
 * the context with room for a second set of density partials (allocates);
 * later calls, and XC_FP64 restricted integrations, use that plan.
 * Stream-ordered like xc_context_integrate.
 */
int xc_context_integrate_uks(xc_context* ctx, int functional, int precision,
                             const double* d_Pa, const double* d_Pb, double* d_Va,
                             double* d_Vb, double* d_EN);

/*
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc. The same
 * integration as xc_context_integrate (same kernels, same arguments and
 * results), with its per-integration scratch (the Phi and Z slabs and density
 * partials of a wave, the tile map, the request descriptor) placed in a
 * static device array of XC_STATIC_SCRATCH_BYTES instead of the context's
 * own scratch. It calls no hipMalloc, hipFree or other allocating routine.
 *  - The context must be built (xc_context_build_grid) and its device must be
 *    the current device: XC_ERR_STATE otherwise.
 *  - The context's largest wave, plus 256 bytes, its tile map and (for
 *    XC_MIXED_BF16) 8 nbf (nbf + 1) bytes of digits of P, must fit in the
 *    array: XC_ERR_NOMEM otherwise (nothing is launched, no output is
 *    written). A context created with wave_bytes <= XC_STATIC_SCRATCH_BYTES / 2
 *    fits whenever one batch does (a 512-point batch with n_b screened
 *    functions needs about 8.2 n_b KiB).
 *  - The library holds one such array on every GPU it runs on, until the
 *    process ends; the first call on a device looks up its address. Every
 *    call on one GPU shares that GPU's array, which keeps the last call's
 *    contents; nothing in it has to start at zero (each call writes every
 *    byte it later reads). Calls that overlap on one GPU (from other streams,
 *    contexts or threads) race on the array: the caller must order them.
 *  - The context's Phi cache (xc_context_set_phi_cache) is neither used nor
 *    disturbed, and per-phase timing is not recorded.
 */
#define XC_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
int xc_context_integrate_noalloc(xc_context* ctx, int functional, int precision,
                                 const double* d_P, double* d_V, double* d_EN);

/*
 * Device memory of this context's integrations, for admission decisions
 * (the batch-subset waves of Alg. 2 are planned against a memory budget).
 *  min_bytes     persistent data (grid, batches, screened lists,
 *                descriptors, partial sums) plus the wave scratch of the
 *                largest single batch: the least with which the context can
 *                integrate (one batch per wave at worst)
 *  cached_bytes  persistent data plus the scratch of all batches at once:
 *                a one-wave plan, which also lets xc_context_set_phi_cache
 *                keep Phi
 * Exact once the grid is built, for restricted LDA/GGA integrations: the
 * spin-unrestricted and meta-GGA entry points re-plan the waves with more
 * scratch per batch (a second set of partials; three gradient slabs and
 * three sets of partials) and are not covered. Before the build only
 * min_bytes is given, as an estimate from the nominal grid size (build
 * temporaries included) with one batch bounded by the whole basis;
 * cached_bytes is then 0 (it depends on the screening). Either pointer may
 * be NULL. No device work.
 */
int xc_context_footprint(xc_context* ctx, size_t* min_bytes, size_t* cached_bytes);

/* Sizes of the built grid (host struct, filled synchronously). */
int xc_context_stats(xc_context* ctx, xc_stats* out);

/*
 * Copy the built grid to host arrays in batch order: xyzw (n_points x 4:
 * point and SSF-scaled weight), index (n_points: position of the point in
 * the unpruned masked-atom grid, atom-major, radial outer, angular inner).
 * Synchronous. Either pointer may be NULL.
 */
int xc_context_export_grid(xc_context* ctx, double* xyzw, long long* index);

/*
 * Copy the batches to host arrays. point_ptr (n_batches + 1): first point of
 * each batch in export_grid order; bbox (n_batches x 6: min xyz, max xyz);
 * shell_ptr (n_batches + 1) and shells (n_shell_entries): the screened shell
 * list of each batch, ascending. Synchronous. Any pointer may be NULL.
 */
int xc_context_export_batches(xc_context* ctx, long long* point_ptr,
                              double* bbox, long long* shell_ptr, int* shells);

/*
 * Keep the collocation matrices between integrations (enable != 0), for
 * SCF iterations that integrate many density matrices on one grid: the
 * matrices Phi^j of the batch-local quantities (Sec. 2.2, Alg. 4) depend on
 * the grid and the basis only, not on P. When the wave plan has a single
 * wave, the wave scratch still holds Phi after an integration, and the next
 * integration that stores Phi in the same type (FP64 for XC_FP64 and
 * XC_MIXED_FP32_V, FP32 for XC_MIXED_FP32, FP64 with per-point digit scales
 * for XC_MIXED_BF16) skips the
 * collocation kernel; the results are bitwise the same. Costs no device
 * memory. A grid rebuild, a change of the Phi type or enable = 0 drops the
 * cached matrices; a plan with several waves never caches. Default off.
 */
int xc_context_set_phi_cache(xc_context* ctx, int enable);

/*
 * Turn per-phase timing on (enable != 0) or off; either way the accumulated
 * times are reset. While on, every launch is bracketed by two events on the
 * context's stream.
 */
int xc_context_set_timing(xc_context* ctx, int enable);

/* Accumulated per-phase times since the last reset (synchronises the stream). */
int xc_context_timing(xc_context* ctx, xc_timing* out);

/* Release every device resource of the context (synchronises its stream). */
int xc_context_destroy(xc_context* ctx);

/*
 * Continuous-batching engine. Many integrations (typically the successive
 * SCF iterations of many molecules) share one device and one stream:
 *  - a request is a molecule + basis + grid + functional + precision; it is
 *    admitted when its expected device footprint fits the engine's budget
 *    next to the already admitted requests; admission builds its grid, which
 *    then stays on the device until the request is released (grid reuse
 *    across Fock builds, Sec. 2.3.1);
 *  - an integration (one P -> V, E_xc, N_e) is submitted against a request;
 *    a request runs its integrations one at a time, in submission order;
 *  - every step co-batches the pending grid batches of all in-flight
 *    integrations (round-robin, one batch of each in turn, until the wave
 *    scratch is full) into the same launches, so integrations that arrive
 *    while others run join the next step;
 *  - grids are built by a thread of the engine on a stream of its own
 *    (default priority), so building a new request's grid never holds up
 *    the steps of the requests already running; a request takes part in
 *    steps once its grid is built;
 *  - with cache_phi, an admitted request also keeps its collocation
 *    matrices Phi^j (Sec. 2.2, Alg. 4; they depend on the grid and the basis
 *    only) on the device when its footprint with them still fits the
 *    budget: its first integration writes them, later ones skip the
 *    collocation (the results are the same bit for bit).
 * Device buffers passed to xc_engine_submit must stay valid until the
 * ticket polls done. Calls on one engine must not overlap.
 */
typedef struct xc_engine xc_engine;

typedef struct xc_engine_opts {
    void* stream;        /* hipStream_t for all engine work (NULL: null stream) */
    size_t hbm_budget;   /* device bytes admitted requests may hold; 0: half the free memory */
    size_t wave_bytes;   /* scratch of one co-batched step; 0: min(free/8, 8 GiB) */
    int cache_phi;       /* 1: keep admitted requests' Phi on the device across their
                            integrations when the budget allows; 0: recompute it */
} xc_engine_opts;

typedef struct xc_engine_info {
    int waiting;                /* requests not yet admitted */
    int admitted;
    int in_flight;              /* requests with an integration in progress */
    size_t bytes_used;          /* device bytes held by admitted requests */
    size_t budget;
    size_t wave_bytes;
    long long steps;
    long long batches_launched;
    long long completed;        /* integrations polled done */
    long long colloc_batches;   /* batches whose collocation ran */
    int phi_cached;             /* admitted requests keeping their Phi */
} xc_engine_info;

/* Create an engine; allocates its wave scratch. */
int xc_engine_create(const xc_engine_opts* opts, xc_engine** out);

/* Add a request (inputs are copied). XC_ERR_NOMEM if it can never fit. */
int xc_engine_add_request(xc_engine* eng, const xc_molecule* mol,
                          const xc_basis* basis, const xc_grid_spec* grid,
                          int functional, int precision, long long* req_id);

/*
 * Queue one integration of a request. d_P (read), d_V (written, nbf x nbf)
 * and d_EN (written, 2 doubles) are device buffers owned by the caller.
 */
int xc_engine_submit(xc_engine* eng, long long req_id, const double* d_P,
                     double* d_V, double* d_EN, long long* ticket);

/*
 * Hand waiting requests that fit to the grid builder, finish the admission
 * of those whose grids are built, then launch one co-batched step.
 * *n_batches (may be NULL) receives the number of batches launched. A
 * request whose grid cannot be built (or has a batch larger than the wave
 * scratch) leaves the queue: the call returns that error, and polls of its
 * tickets return it too.
 */
int xc_engine_step(xc_engine* eng, int* n_batches);

/* *done = 1 once the ticket's V, E_xc and N_e are final (non-blocking). A
 * ticket reported done is retired and cannot be polled again. */
int xc_engine_poll(xc_engine* eng, long long ticket, int* done);

/* Drop a request with no integration in flight; frees its device memory.
 * XC_ERR_BUSY while one of its integrations is queued or running. */
int xc_engine_release(xc_engine* eng, long long req_id);

int xc_engine_stats(xc_engine* eng, xc_engine_info* out);

/* Synchronise and free everything the engine holds. */
int xc_engine_destroy(xc_engine* eng);

#ifdef __cplusplus
}
#endif

#endif /* XC_MI355X_H */
