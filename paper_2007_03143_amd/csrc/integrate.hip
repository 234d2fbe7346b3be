// Per-wave integration kernels (Sec. 2.2 eq. eval_local_den, eq.
// eval_local_den_grad, eq. x_mat, eq. exc_batch, eq. vxc_inc, eq. vxc_batch,
// eq. z_mat; Sec. 2.3.2 Alg. 4).
//
// For every batch j of a wave, in four steps, each one or two launches over
// all its batches:
//  1. collocation Phi^j (n_b x n_g), written in compressed form over the
//     screened functions (only Phi is stored; gradients are re-evaluated
//     from the shell data wherever they are needed, which costs far less
//     than moving three more n_b x n_g slabs through HBM);
//  2. X = P^j Phi^j on MFMA with P^j gathered straight from the full P
//     (never packed), and rho, grad rho reduced from X in the epilogue
//     (X is never stored);
//  3. the functional per point, the batch's E_xc and N_e partials (one
//     kernel), then Z^j = (1/2) w v_rho Phi + 2 w v_sigma grad rho . grad Phi
//     (another);
//  4. V^j = Z Phi^T + Phi Z^T on MFMA over lower-triangle tiles only,
//     added into the lower triangle of the full V with FP64 atomics.
// Then V is mirrored and E_xc, N_e are summed in a fixed order.
#include <cmath>
#include <type_traits>

#include "device_util.hpp"
#include "functional.hpp"
#include "functional_mgga.hpp"
#include "xc_internal.hpp"


namespace xc {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// 16x16x4 MFMA of the storage type: FP64 (v_mfma_f64_16x16x4f64) or FP32
// (v_mfma_f32_16x16x4f32). Operand lane l holds A[l % 16][l / 16] and
// B[l / 16][l % 16]; accumulator register r of lane l holds C[row][l % 16]
// with row = acc_row(r, l): 4 r + l / 16 for FP64 but 4 (l / 16) + r for
// FP32 (both checked on gfx950).
template <typename T> struct Mfma;
template <> struct Mfma<double> {
    using acc = v4d;
    __device__ static inline acc zero() { return acc{0.0, 0.0, 0.0, 0.0}; }
    __device__ static inline acc mma(double a, double b, acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static inline int acc_row(int r, int lane) { return 4 * r + (lane >> 4); }
};
template <> struct Mfma<float> {
    using acc = v4f;
    __device__ static inline acc zero() { return acc{0.f, 0.f, 0.f, 0.f}; }
    __device__ static inline acc mma(float a, float b, acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static inline int acc_row(int r, int lane) { return 4 * (lane >> 4) + r; }
};

// The request descriptor with every array typed as global memory.
struct ReqG {
    gptr<const ShellDev> shells;
    gptr<const double> palpha, pcoef;
    gptr<const int> shell_list, shell_loff, func_list, func_shell;
    gptr<const double> px, py, pz, pw, P;
    gptr<double> V, epart, npart;
    gptr<const unsigned long long> Pdig;
    gptr<const double> Pscale;
    char* phi_base;
    double rho_thresh;
    int nbf;
};

// Start of a batch's Phi slab: the request's Phi store, or the wave scratch
// (both global memory; typed so, the slab's loads and stores do not become
// flat instructions, which would also hold up every wait for LDS data).
__device__ inline gptr<char> phi_slab(const WaveBatch& B, const ReqG& R, char* scratch) {
    return to_global(R.phi_base ? R.phi_base : scratch) + 8 * B.phi_off;
}

__device__ inline ReqG global_view(const ReqDev& r) {
    ReqG g;
    g.shells = to_global(r.shells);
    g.palpha = to_global(r.palpha);
    g.pcoef = to_global(r.pcoef);
    g.shell_list = to_global(r.shell_list);
    g.shell_loff = to_global(r.shell_loff);
    g.func_list = to_global(r.func_list);
    g.func_shell = to_global(r.func_shell);
    g.px = to_global(r.px);
    g.py = to_global(r.py);
    g.pz = to_global(r.pz);
    g.pw = to_global(r.pw);
    g.P = to_global(r.P);
    g.V = to_global(r.V);
    g.epart = to_global(r.epart);
    g.npart = to_global(r.npart);
    g.Pdig = to_global(r.Pdig);
    g.Pscale = to_global(r.Pscale);
    g.phi_base = r.phi_base;
    g.rho_thresh = r.rho_thresh;
    g.nbf = r.nbf;
    return g;
}

__device__ inline ShellDev load_shell(gptr<const ShellDev> p) {
    ShellDev s;
    s.x = p->x;
    s.y = p->y;
    s.z = p->z;
    s.rcut2 = p->rcut2;
    s.L = p->L;
    s.nprim = p->nprim;
    s.prim_off = p->prim_off;
    s.first_func = p->first_func;
    s.pure = p->pure;
    return s;
}

// Digits of a value y with |y| <= 1 for the split-BF16 density contraction:
// d0 = rint(128 y), then d_u = rint(256 r) with r the remainder scaled by
// the previous step; every digit is an integer of magnitude <= 128 (exact in
// BF16), every subtraction is exact (its operands lie within a factor of
// two, or the digit is zero), and y = sum_u d_u 2^{-7-8u} up to a remainder
// below 2^{-32}. Packed as four BF16 bit patterns, digit u in bits
// 16 u .. 16 u + 15.
__device__ inline unsigned long long digits_packed(double y) {
    double a = y * 128.0;
    double q = rint(a);
    unsigned long long w = __builtin_bit_cast(unsigned short, (__bf16)(float)q);
#pragma unroll
    for (int u = 1; u < 4; ++u) {
        a = (a - q) * 256.0;
        q = rint(a);
        w |= (unsigned long long)__builtin_bit_cast(unsigned short, (__bf16)(float)q)
             << (16 * u);
    }
    return w;
}

// Real solid harmonics of a spherical shell (Racah normalisation, m = -L..L)
// as combinations of its Cartesian components in lexicographic order:
// S_m = sum_c sph<L>(m, c) x^l y^m z^n.
//  L = 2 (xx xy xz yy yz zz): sqrt3 xy, sqrt3 yz, z^2 - (x^2 + y^2)/2,
//        sqrt3 xz, sqrt3/2 (x^2 - y^2)
//  L = 3 (xxx xxy xxz xyy xyz xzz yyy yyz yzz zzz):
//        sqrt10/4 (3 x^2 y - y^3), sqrt15 xyz, sqrt6/4 y (4 z^2 - x^2 - y^2),
//        z (2 z^2 - 3 x^2 - 3 y^2)/2, sqrt6/4 x (4 z^2 - x^2 - y^2),
//        sqrt15/2 z (x^2 - y^2), sqrt10/4 (x^3 - 3 x y^2)
constexpr double kSqrt3 = 1.7320508075688772;
constexpr double kSqrt15 = 3.8729833462074170;
constexpr double kSqrt6q = 0.61237243569579452;   // sqrt6 / 4
constexpr double kSqrt10q = 0.79056941504209483;  // sqrt10 / 4
constexpr double kSph2[5][6] = {{0, kSqrt3, 0, 0, 0, 0},
                                {0, 0, 0, 0, kSqrt3, 0},
                                {-0.5, 0, 0, -0.5, 0, 1.0},
                                {0, 0, kSqrt3, 0, 0, 0},
                                {0.5 * kSqrt3, 0, 0, -0.5 * kSqrt3, 0, 0}};
constexpr double kSph3[7][10] = {
    {0, 3 * kSqrt10q, 0, 0, 0, 0, -kSqrt10q, 0, 0, 0},
    {0, 0, 0, 0, kSqrt15, 0, 0, 0, 0, 0},
    {0, -kSqrt6q, 0, 0, 0, 0, -kSqrt6q, 0, 4 * kSqrt6q, 0},
    {0, 0, -1.5, 0, 0, 0, 0, -1.5, 0, 1.0},
    {-kSqrt6q, 0, 0, -kSqrt6q, 0, 4 * kSqrt6q, 0, 0, 0, 0},
    {0, 0, 0.5 * kSqrt15, 0, 0, 0, 0, -0.5 * kSqrt15, 0, 0},
    {kSqrt10q, 0, 0, -3 * kSqrt10q, 0, 0, 0, 0, 0, 0}};
template <int L>
__device__ constexpr double sph(int m, int c) {
    if constexpr (L == 2) return kSph2[m][c];
    else return kSph3[m][c];
}

// ------------------------------------------------------------ collocation --
// e^{-x} for x >= 0, table-driven (Tang's method, ACM TOMS 15, 1989, with 64
// table entries): x = (64 m + j) ln2 / 64 + r with |r| <= ln2 / 128, so
// e^{-x} = 2^{-m} 2^{-j/64} e^{-r}. The reduction subtracts n ln2 / 64 in two
// parts (ln2 split into its nearest double and the remainder) with fused
// multiply-adds; e^{-r} is its Taylor polynomial of degree 6 (truncation
// below r^7 / 7! < 3e-20 relative); 2^{-j/64} comes from a table in LDS that
// each workgroup fills with the library exp2 (exp_table_init, before its
// first barrier). About half the FP64 operations of the library exp; within
// 2 ulp where the result is a normal number (an exact replay of these steps
// over 5,000 arguments finds at most 1.74 ulp). The argument is first clamped
// to 746, where e^{-x} already rounds to zero, so the integer conversion below
// stays in range for any input (a huge alpha r^2, +inf or NaN all give 0).
__shared__ double g_exp_tab[64];
__device__ inline void exp_table_init() {
    if (threadIdx.x < 64) g_exp_tab[threadIdx.x] = exp2(-(double)threadIdx.x / 64.0);
}
__device__ inline double exp_neg(double x) {
    x = fmin(x, 746.0);
    const double nd = rint(x * 92.33248261689366);       // 64 / ln 2
    const int n = (int)nd;
    double r = fma(-nd, 0.010830424696249145, x);         // ln2 (nearest double) / 64
    r = fma(-nd, 3.623510646634843e-19, r);               // (ln2 - that double) / 64
    double p = fma(r, 1.0 / 720.0, -1.0 / 120.0);
    p = fma(r, p, 1.0 / 24.0);
    p = fma(r, p, -1.0 / 6.0);
    p = fma(r, p, 0.5);
    p = fma(r, p, -1.0);
    p = fma(r, p, 1.0);
    return ldexp(g_exp_tab[n & 63] * p, -(n >> 6));
}

// Radial part of a shell at squared distance r2: rad = sum_xi d e^{-alpha r2}
// and drad = -2 sum_xi alpha d e^{-alpha r2} (d rad / d r2 times 2), zero
// outside the cutoff sphere.
__device__ inline void shell_radial(const ShellDev& sh, gptr<const double> palpha,
                                    gptr<const double> pcoef, double r2, double& rad,
                                    double& drad) {
    rad = 0.0;
    drad = 0.0;
    if (!(r2 <= sh.rcut2)) return;
    for (int p = 0; p < sh.nprim; ++p) {
        const double a = palpha[sh.prim_off + p];
        const double de = pcoef[sh.prim_off + p] * exp_neg(a * r2);
        rad += de;
        drad -= 2.0 * a * de;
    }
}

// alpha r2 at and beyond which e^{-alpha r2} is exactly zero in FP64.
constexpr double kExpZero = 746.0;

// Squared distance with the same rounding in every kernel (no contraction),
// so the cutoff test gives the same answer wherever it is evaluated.
__device__ inline double dist2_nc(double x, double y, double z, const ShellDev& sh,
                                  double& dx, double& dy, double& dz) {
#pragma clang fp contract(off)
    dx = x - sh.x;
    dy = y - sh.y;
    dz = z - sh.z;
    return dx * dx + dy * dy + dz * dz;
}

// Z entries of the (L+1)(L+2)/2 functions of one shell at one point:
// z = a phi + b . grad phi, written down the rows starting at out. With
// phi = A(d) rad and grad phi = grad A rad + A drad d (eq. gau_cart: A the
// Cartesian monomial, d the displacement from the centre),
// z = A (a rad + drad b.d) + rad b.grad A, so the shell-wide factors are
// formed once and each component costs a few products with its exponents
// known at compile time.
// PURE: the Cartesian z values are formed in registers and combined into
// the shell's 2L+1 spherical rows.
template <int L, typename T, bool PURE = false>
__device__ inline void z_shell(double dx, double dy, double dz, double rad, double drad,
                               double a, double bx, double by, double bz, T* out,
                               int ngp) {
    double xp[L + 1], yp[L + 1], zp[L + 1];
    xp[0] = yp[0] = zp[0] = 1.0;
#pragma unroll
    for (int k = 1; k <= L; ++k) {
        xp[k] = xp[k - 1] * dx;
        yp[k] = yp[k - 1] * dy;
        zp[k] = zp[k - 1] * dz;
    }
    const double t0 = a * rad + (bx * dx + by * dy + bz * dz) * drad;
    const double rbx = rad * bx, rby = rad * by, rbz = rad * bz;
    double zc[PURE ? (L + 1) * (L + 2) / 2 : 1];
    int c = 0;
#pragma unroll
    for (int l = L; l >= 0; --l) {
#pragma unroll
        for (int m = L - l; m >= 0; --m) {
            const int n = L - l - m;
            const double yz = yp[m] * zp[n];
            double z = xp[l] * yz * t0;
            if (l > 0) z += rbx * (l * xp[l - 1] * yz);
            if (m > 0) z += rby * (m * xp[l] * yp[m - 1] * zp[n]);
            if (n > 0) z += rbz * (n * xp[l] * yp[m] * zp[n - 1]);
            if constexpr (PURE) zc[c] = z;
            else out[(size_t)c * ngp] = T(z);
            ++c;
        }
    }
    if constexpr (PURE) {
#pragma unroll
        for (int m = 0; m < 2 * L + 1; ++m) {
            double v = 0.0;
#pragma unroll
            for (int k = 0; k < (L + 1) * (L + 2) / 2; ++k)
                if (sph<L>(m, k) != 0.0) v = fma(sph<L>(m, k), zc[k], v);
            out[(size_t)m * ngp] = T(v);
        }
    }
}

// One workgroup per batch; wave w evaluates shells w, w+4, ... of the
// batch's screened list, one lane per point, so a wave never diverges on
// the contraction length. Points of the batch are staged in LDS. Values are
// formed in FP64 in every mode and rounded once on store. SCALE (split-BF16
// mode): a first pass over the shells keeps only the largest magnitude
// max_mu |phi_mu(r_i)| of every point as a running maximum in LDS (the bit
// patterns of non-negative doubles order like unsigned integers); the digit
// scale of a point is the least power of two not below it (1 where all are
// zero) and goes to the batch's scale row; a second pass forms the values
// again, bit for bit the same, and cuts each into its four digits
// (digits_packed) straight into the Phi slab.
// phi of one shell at one point in one of three modes: MODE 0 stores the
// values (type T), MODE 1 only returns their largest magnitude, MODE 2
// stores the digits of value * inv (T = unsigned long long).
template <int L, int MODE, typename T>
__device__ inline double phi_shell_mode(const ShellDev& sh, double dx, double dy, double dz,
                                        double rad, gptr<T> out, int ngp, double inv) {
    constexpr int NC = (L + 1) * (L + 2) / 2;
    double xp[L + 1], yp[L + 1], zp[L + 1];
    xp[0] = yp[0] = zp[0] = 1.0;
#pragma unroll
    for (int k = 1; k <= L; ++k) {
        xp[k] = xp[k - 1] * dx;
        yp[k] = yp[k - 1] * dy;
        zp[k] = zp[k - 1] * dz;
    }
    double mx = 0.0;
    auto put = [&](int r, double v) {
        mx = fmax(mx, fabs(v));
        if constexpr (MODE == 0) out[(size_t)r * ngp] = T(v);
        if constexpr (MODE == 2) out[(size_t)r * ngp] = digits_packed(v * inv);
    };
    if (L >= 2 && sh.pure) {
        double v[NC];
        int c = 0;
#pragma unroll
        for (int l = L; l >= 0; --l)
#pragma unroll
            for (int m = L - l; m >= 0; --m) v[c++] = xp[l] * yp[m] * zp[L - l - m];
#pragma unroll
        for (int m = 0; m < 2 * L + 1; ++m) {
            double a = 0.0;
#pragma unroll
            for (int k = 0; k < NC; ++k)
                if (sph<L>(m, k) != 0.0) a = fma(sph<L>(m, k), v[k], a);
            put(m, a * rad);
        }
    } else {
        int c = 0;
#pragma unroll
        for (int l = L; l >= 0; --l)
#pragma unroll
            for (int m = L - l; m >= 0; --m) {
                put(c, xp[l] * yp[m] * zp[L - l - m] * rad);
                ++c;
            }
    }
    return mx;
}

// One collocation pass over the batch's shells (wave-strided) and points
// (lane-strided) in the given mode; MODE 1 folds each point's largest
// magnitude into smax, MODE 2 reads each point's inverse scale from it.
template <int MODE, typename T>
__device__ inline void colloc_pass(const WaveBatch& B, const ReqG& R, const double* sx,
                                   const double* sy, const double* sz,
                                   unsigned long long* smax, gptr<T> Phi) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
    for (int sl = wave; sl < B.nshell; sl += 4) {
        const int s = R.shell_list[B.shell_off + sl];
        const int loff = R.shell_loff[B.shell_off + sl];
        const ShellDev sh = load_shell(R.shells + s);
        for (int i = lane; i < B.ngp; i += 64) {
            double dx, dy, dz, rad, drad;
            const double r2 = dist2_nc(sx[i], sy[i], sz[i], sh, dx, dy, dz);
            if (i < B.ng) shell_radial(sh, R.palpha, R.pcoef, r2, rad, drad);
            else rad = drad = 0.0;
            const gptr<T> out = Phi + (size_t)loff * B.ngp + i;
            const double inv = MODE == 2 ? __longlong_as_double((long long)smax[i]) : 0.0;
            double mx;
            switch (sh.L) {
                case 0: mx = phi_shell_mode<0, MODE, T>(sh, dx, dy, dz, rad, out, B.ngp, inv); break;
                case 1: mx = phi_shell_mode<1, MODE, T>(sh, dx, dy, dz, rad, out, B.ngp, inv); break;
                case 2: mx = phi_shell_mode<2, MODE, T>(sh, dx, dy, dz, rad, out, B.ngp, inv); break;
                default: mx = phi_shell_mode<3, MODE, T>(sh, dx, dy, dz, rad, out, B.ngp, inv); break;
            }
            if (MODE == 1 && mx > 0.0)
                atomicMax(&smax[i], (unsigned long long)__double_as_longlong(mx));
        }
    }
}

template <typename T, bool SCALE>
__global__ __launch_bounds__(256) void k_colloc(const WaveBatch* __restrict__ wb,
                                                const ReqDev* __restrict__ reqs,
                                                char* __restrict__ scratch) {
    const WaveBatch B = wb[blockIdx.x];
    if (B.flags & kSkipColloc) return;   // Phi already in the request's store
    exp_table_init();
    const ReqG R = global_view(reqs[B.req]);
    __shared__ double sx[kMaxBatch], sy[kMaxBatch], sz[kMaxBatch];
    __shared__ unsigned long long smax[SCALE ? kMaxBatch : 1];
    for (int i = threadIdx.x; i < B.ngp; i += blockDim.x) {
        const bool v = i < B.ng;
        sx[i] = v ? R.px[B.pt_off + i] : 0.0;
        sy[i] = v ? R.py[B.pt_off + i] : 0.0;
        sz[i] = v ? R.pz[B.pt_off + i] : 0.0;
        if (SCALE) smax[i] = 0ull;
    }
    __syncthreads();
    const gptr<char> phi = phi_slab(B, R, scratch);
    // zero the padding rows n_b .. n_bp - 1 (a zero value has zero digits)
    const long long npad = (long long)(B.nbp - B.nb) * B.ngp;
    if constexpr (SCALE) {
        const gptr<unsigned long long> dig = (gptr<unsigned long long>)phi;
        for (long long k = threadIdx.x; k < npad; k += blockDim.x) dig[(size_t)B.nb * B.ngp + k] = 0ull;
        colloc_pass<1, unsigned long long>(B, R, sx, sy, sz, smax, dig);
        __syncthreads();
        const gptr<double> sc = (gptr<double>)phi + scale_row_off(B);
        for (int i = threadIdx.x; i < B.ngp; i += blockDim.x) {
            const double m = __longlong_as_double((long long)smax[i]);
            int e = 0;
            (void)frexp(m, &e);  // m = f 2^e with f in [0.5, 1), so m <= 2^e
            e = max(e, -1000);   // 1 / scale stays finite
            sc[i] = m > 0.0 ? ldexp(1.0, e) : 1.0;
            // the exact inverse, for the cut (kept in smax from here on)
            smax[i] = (unsigned long long)__double_as_longlong(m > 0.0 ? ldexp(1.0, -e) : 1.0);
        }
        __syncthreads();
        colloc_pass<2, unsigned long long>(B, R, sx, sy, sz, smax, dig);
    } else {
        const gptr<T> Phi = (gptr<T>)phi;
        for (long long k = threadIdx.x; k < npad; k += blockDim.x) Phi[(size_t)B.nb * B.ngp + k] = T(0);
        colloc_pass<0, T>(B, R, sx, sy, sz, smax, Phi);
    }
}

// Radial part of a shell that is the same on every lane of the wave. A
// primitive is skipped when alpha r2 >= kExpZero on every lane: its
// exponential is then zero everywhere, so the sums are the same bit for bit
// (tight primitives far from their centre, the common case here), and the
// wave-wide test keeps the lanes together. `in` is false on lanes without a
// point.
__device__ inline void shell_radial_wave(const ShellDev& sh, gptr<const double> palpha,
                                         gptr<const double> pcoef, double r2, bool in,
                                         double& rad, double& drad) {
    rad = 0.0;
    drad = 0.0;
    in = in && r2 <= sh.rcut2;
    for (int p = 0; p < sh.nprim; ++p) {
        const double a = palpha[sh.prim_off + p];
        const double x = a * r2;
        if (__any(in && x < kExpZero)) {
            const double de = in ? pcoef[sh.prim_off + p] * exp_neg(x) : 0.0;
            rad += de;
            drad -= 2.0 * a * de;
        }
    }
}

// Contributions of the components k0 .. k0 + cnt - 1 of one shell (tile
// rows rl .. rl + cnt - 1; all wave-uniform) at one point: phi*X and, for
// GGA, grad phi*X. With phi = A(d) rad and grad phi = grad A rad + A drad d,
// the sums over the components need only S = sum X A and the three sums
// X dA/dx, X dA/dy, X dA/dz, formed with the exponents known at compile
// time. The X values are read first, all at once. PURE: the shell's rows
// are its 2L+1 spherical functions, whose X values are first folded into
// weights of the Cartesian components (sum_m X_m S_m = sum_c w_c A_c).
template <int L, bool GGA, bool PURE>
__device__ inline void rho_shell(int k0, int cnt, double dx, double dy, double dz, double rad,
                                 double drad, const double (*Xs)[kTile + 1], int rl, int c,
                                 double (&q)[4]) {
    constexpr int NC = (L + 1) * (L + 2) / 2;
    constexpr int NF = PURE ? 2 * L + 1 : NC;
    double xv[NF];
#pragma unroll
    for (int k = 0; k < NF; ++k) {
        const double v = Xs[min(max(rl + k - k0, 0), kTile - 1)][c];
        xv[k] = (k >= k0 && k < k0 + cnt) ? v : 0.0;
    }
    double wv[NC];
    if constexpr (PURE) {
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            double a = 0.0;
#pragma unroll
            for (int m = 0; m < NF; ++m)
                if (sph<L>(m, k) != 0.0) a = fma(sph<L>(m, k), xv[m], a);
            wv[k] = a;
        }
    } else {
#pragma unroll
        for (int k = 0; k < NC; ++k) wv[k] = xv[k];
    }
    double xp[L + 1], yp[L + 1], zp[L + 1];
    xp[0] = yp[0] = zp[0] = 1.0;
#pragma unroll
    for (int k = 1; k <= L; ++k) {
        xp[k] = xp[k - 1] * dx;
        yp[k] = yp[k - 1] * dy;
        zp[k] = zp[k - 1] * dz;
    }
    double s0 = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
    int comp = 0;
#pragma unroll
    for (int l = L; l >= 0; --l) {
#pragma unroll
        for (int m = L - l; m >= 0; --m) {
            const int n = L - l - m;
            if (PURE || (comp >= k0 && comp < k0 + cnt)) {
                const double yz = yp[m] * zp[n];
                s0 += wv[comp] * (xp[l] * yz);
                if (GGA) {
                    if (l > 0) sx += wv[comp] * (l * xp[l - 1] * yz);
                    if (m > 0) sy += wv[comp] * (m * xp[l] * yp[m - 1] * zp[n]);
                    if (n > 0) sz += wv[comp] * (n * xp[l] * yp[m] * zp[n - 1]);
                }
            }
            ++comp;
        }
    }
    q[0] += rad * s0;
    if (GGA) {
        const double ds = drad * s0;
        q[1] += ds * dx + rad * sx;
        q[2] += ds * dy + rad * sy;
        q[3] += ds * dz + rad * sz;
    }
}

// Epilogue of the density contraction: the X tile (64 functions x 64
// points, FP64) is in LDS. Each thread takes one point and the 16
// consecutive functions of its wave, walks them shell by shell (the rows of
// a shell are consecutive components of it), re-evaluates the radial part
// once per shell and phi (and grad phi) per component in FP64, and reduces
// phi*X (grad phi * X) into the per-row-tile partials part[mt][q][point],
// q = rho, dx, dy, dz. All lanes take part; a lane past n_g has no point
// (has = false: zero radial part, and its X column is zero padding). The
// point's coordinates x, y, z are loaded by the caller before its main loop,
// so their latency is hidden.
template <bool GGA>
__device__ inline void rho_epilogue(const WaveBatch& B, const ReqG& R, int m0, int n0, int mt,
                                    double (*Xs)[kTile + 1], const int* fsh, const int* frow,
                                    double x, double y, double z, bool has, char* scratch) {
    const int c = threadIdx.x & 63;
    const int g = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    double q[4] = {0.0, 0.0, 0.0, 0.0};
    const int rend = min(g * 16 + 16, B.nb - m0);
    for (int rl = g * 16; rl < rend;) {
        const int sidx = __builtin_amdgcn_readfirstlane(fsh[rl]);
        const ShellDev sh = load_shell(R.shells + sidx);
        const int nc = shell_nfunc(sh.L, sh.pure);
        const int k0 = min(max(__builtin_amdgcn_readfirstlane(frow[rl]) - sh.first_func, 0),
                           nc - 1);
        const int cnt = min(nc - k0, rend - rl);
        double dx, dy, dz, rad, drad;
        const double r2 = dist2_nc(x, y, z, sh, dx, dy, dz);
        shell_radial_wave(sh, R.palpha, R.pcoef, r2, has, rad, drad);
        if (sh.pure) {
            if (sh.L == 2) rho_shell<2, GGA, true>(k0, cnt, dx, dy, dz, rad, drad, Xs, rl, c, q);
            else rho_shell<3, GGA, true>(k0, cnt, dx, dy, dz, rad, drad, Xs, rl, c, q);
        } else {
            switch (sh.L) {
                case 0: rho_shell<0, GGA, false>(k0, cnt, dx, dy, dz, rad, drad, Xs, rl, c, q); break;
                case 1: rho_shell<1, GGA, false>(k0, cnt, dx, dy, dz, rad, drad, Xs, rl, c, q); break;
                case 2: rho_shell<2, GGA, false>(k0, cnt, dx, dy, dz, rad, drad, Xs, rl, c, q); break;
                default: rho_shell<3, GGA, false>(k0, cnt, dx, dy, dz, rad, drad, Xs, rl, c, q); break;
            }
        }
        rl += cnt;
    }
    __syncthreads();
    double* red = &Xs[0][0];
#pragma unroll
    for (int qq = 0; qq < 4; ++qq) red[(g * 4 + qq) * kTile + c] = q[qq];
    __syncthreads();
    if (g == 0) {
        double* part = (double*)(scratch + 8 * B.part_off);
        constexpr int NQ = GGA ? 4 : 1;
#pragma unroll
        for (int qq = 0; qq < NQ; ++qq) {
            const double v = red[(0 * 4 + qq) * kTile + c] + red[(1 * 4 + qq) * kTile + c] +
                             red[(2 * 4 + qq) * kTile + c] + red[(3 * 4 + qq) * kTile + c];
            part[(size_t)(mt * 4 + qq) * B.ngp + n0 + c] = v;
        }
    }
}

// ------------------------------------------------------- density (GEMM) ----
// Tile of 64 functions x 64 NW points of X = P^j Phi^j; 4 waves, each a
// 32 x 32 NW block of 2 x 2 NW MFMA 16x16x4 tiles (NW = 2 for FP64: twice
// the MFMAs per barrier and per A fragment read, and the A operand, a
// gather from P, loaded once per 128 points). A operand rows are gathered from the
// full P through the batch's function list. The epilogue (rho_epilogue)
// spills X to LDS and reduces phi*X (grad phi * X) into per-row-tile
// partials part[mt][q][point], q = rho, dx, dy, dz.
template <bool GGA, typename T, int NW>
__device__ __forceinline__ void gemm_rho_tile(
    const WaveBatch* __restrict__ wb, const int2* __restrict__ tmap, int ntiles,
    const ReqDev* __restrict__ reqs, char* __restrict__ scratch) {
    using M = Mfma<T>;
    const int t = xcd_remap(blockIdx.x, ntiles);
    const int2 tb = tmap[t];
    const int bi = tb.x;
    const WaveBatch B = wb[bi];
    const ReqG R = global_view(reqs[B.req]);
    const gptr<const double> P = R.P;
    const int nbf = R.nbf;
    const gptr<const int> func_list = R.func_list;
    const int lt = tb.y;
    constexpr int NC = kTile * NW;   // points per tile
    const int ntn = NW == 1 ? B.ngp / kTile : (B.ngp + NC - 1) / NC;
    const int mt = lt / ntn, nt = lt - mt * ntn;
    const int m0 = mt * kTile, n0 = nt * NC;
    const int ncol = min(NC, B.ngp - n0);   // a multiple of 64
    exp_table_init();
    const gptr<const T> Phi = (gptr<const T>)phi_slab(B, R, scratch);
    const gptr<const int> fl = func_list + B.func_off;
    // the first epilogue point (one per lane), loaded now so that its latency hides
    bool has = n0 + (int)(threadIdx.x & 63) < B.ng;
    double ex = 0.0, ey = 0.0, ez = 0.0;
    if (has) {
        const long long pi = B.pt_off + n0 + (threadIdx.x & 63);
        ex = R.px[pi];
        ey = R.py[pi];
        ez = R.pz[pi];
    }

    // operand tiles during the main loop, the X tile in the epilogue
    constexpr int kABytes = 2 * kTile * 17 * (int)sizeof(T);
    constexpr int kBBytes = 2 * 16 * (NC + 1) * (int)sizeof(T);
    constexpr int kXBytes = kTile * (kTile + 1) * 8;
    constexpr int kLds = (kABytes + kBBytes > kXBytes) ? kABytes + kBBytes : kXBytes;
    __shared__ __attribute__((aligned(16))) char lds[kLds];
    T (*As)[kTile][17] = reinterpret_cast<T (*)[kTile][17]>(lds);
    T (*Bs)[16][NC + 1] = reinterpret_cast<T (*)[16][NC + 1]>(lds + kABytes);
    double (*Xs)[kTile + 1] = reinterpret_cast<double (*)[kTile + 1]>(lds);
    __shared__ int frow[kTile], fsh[kTile];
    // function indices (columns of P) of four consecutive K steps
    __shared__ __attribute__((aligned(16))) int sfl[4][16];

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform
    const int wm = wave >> 1, wn = wave & 1;
    const int nk = B.nbp / 16;
    // The 16 column indices of a K step are passed on through a ring of
    // four LDS slots (slot = step mod 4), written by threads 0-15; a padding
    // column (k >= n_b) holds the last function's index and is zeroed at
    // the LDS store by its position. Every thread loads, so that each step
    // issues the same number of loads on every path, and the loaded index is
    // not touched before its ring store a step later: the waits for older
    // loads can then leave the newer ones in flight.
    int fnext = 0;
    auto fetch = [&](int ks) { fnext = fl[min(ks * 16 + (tid & 15), B.nb - 1)]; };
    auto fput = [&](int ks) {
        if (tid < 16) sfl[ks & 3][tid] = fnext;
    };
    for (int s0 = 0; s0 < 3; ++s0) {
        fetch(s0);
        fput(s0);
    }
    if (tid < kTile) {
        const int f = (m0 + tid < B.nb) ? fl[m0 + tid] : -1;
        frow[tid] = f;
        fsh[tid] = f >= 0 ? R.func_shell[f] : 0;
    }
    __syncthreads();

    const int ar = tid >> 2, ac = (tid & 3) * 4;
    const int br = tid >> 4, bc = (tid & 15) * 4;   // B columns bc + 64 w, w < NW
    const int fr = frow[ar];
    const gptr<const double> Prow = P + (size_t)(fr >= 0 ? fr : 0) * nbf;

    // Two register sets: the operands of step ks + 2 are loaded while step
    // ks is computed and those of step ks + 1 wait in the other set. The P^j
    // columns of a step are gathered through the function list. The P
    // values stay FP64 until the LDS store, where they are rounded (FP32) and
    // the padding is selected away.
    struct Regs {
        T ra[4], rb[4 * NW];
        double pv[4];
        int fc[4];
    };
    Regs RA, RB;
    auto fread = [&](Regs& r, int ks) {
        const int4 v = *reinterpret_cast<const int4*>(&sfl[ks & 3][ac]);
        r.fc[0] = v.x;
        r.fc[1] = v.y;
        r.fc[2] = v.z;
        r.fc[3] = v.w;
    };
    // All loads go to valid (clamped) addresses and none is skipped: a
    // padding entry of P^j is selected away at the LDS store, a K step past
    // the last reloads the last one's Phi rows, and a 64-point half past the
    // slab's end reloads the first half (its blocks are not computed).
    auto gload = [&](Regs& r, int ks) {
#pragma unroll
        for (int q = 0; q < 4; ++q) r.pv[q] = Prow[r.fc[q]];
        const gptr<const T> src =
            Phi + (size_t)(min(ks, nk - 1) * 16 + br) * B.ngp + n0 + bc;
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            const int off = (w == 0 || w * kTile < ncol) ? kTile * w : 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) r.rb[4 * w + q] = src[off + q];
        }
    };
    auto sstore = [&](Regs& r, int ks) {
        const int buf = ks & 1;
#pragma unroll
        for (int q = 0; q < 4; ++q)
            r.ra[q] = (fr >= 0 && ks * 16 + ac + q < B.nb) ? T(r.pv[q]) : T(0);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            As[buf][ar][ac + q] = r.ra[q];
            Bs[buf][br][bc + q] = r.rb[q];
        }
#pragma unroll
        for (int w = 1; w < NW; ++w)
#pragma unroll
            for (int q = 0; q < 4; ++q) Bs[buf][br][kTile * w + bc + q] = r.rb[4 * w + q];
    };

    // the wave's output blocks: rows wm * 32 + 16 mb, columns
    // 64 w + wn * 32 + 16 nb of the tile (block index 2 w + nb)
    constexpr int NB = 2 * NW;
    typename M::acc acc[2][NB];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) acc[i][j] = M::zero();
    auto bcol = [&](int nb) { return kTile * (nb >> 1) + wn * 32 + (nb & 1) * 16; };

    // 16 x 16 output blocks made only of padding rows or columns are skipped
    // (wave-uniform)
    bool live[2][NB];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb)
            live[mb][nb] = (m0 + wm * 32 + mb * 16 < B.nb) && (n0 + bcol(nb) < B.ng);

    fread(RA, 0);
    gload(RA, 0);
    sstore(RA, 0);
    fread(RB, 1);
    gload(RB, 1);
    fetch(3);
    __syncthreads();
    // step ks: load step ks + 2 into rl, compute from LDS buffer ks & 1,
    // store step ks + 1 from rs into the other buffer; then refill the ring
    // slot of step ks + 3 (last read three steps ago) and fetch step ks + 4.
    // Steps past the last load and store clamped, valid indices, so every
    // slot a step reads holds one.
    auto step = [&](int ks, Regs& rl, Regs& rs) {
        const int cur = ks & 1;
        fread(rl, ks + 2);
        gload(rl, ks + 2);
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
            T a[2], b[NB];
#pragma unroll
            for (int mb = 0; mb < 2; ++mb)
                a[mb] = As[cur][wm * 32 + mb * 16 + (lane & 15)][kk * 4 + (lane >> 4)];
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
                b[nb] = Bs[cur][kk * 4 + (lane >> 4)][bcol(nb) + (lane & 15)];
#pragma unroll
            for (int mb = 0; mb < 2; ++mb)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
                    if (live[mb][nb]) acc[mb][nb] = M::mma(a[mb], b[nb], acc[mb][nb]);
        }
        if (ks + 1 < nk) sstore(rs, ks + 1);
        fput(ks + 3);
        fetch(ks + 4);
        __syncthreads();
    };
    for (int ks = 0; ks < nk; ks += 2) {
        step(ks, RA, RB);
        if (ks + 1 < nk) step(ks + 1, RB, RA);
    }

    // X by 64-point halves: spill, then the epilogue (the loop ended on a
    // barrier, so the operand tiles are free)
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        if (w > 0 && w * kTile >= ncol) break;
        if (w > 0) {
            has = n0 + kTile * w + (int)(threadIdx.x & 63) < B.ng;
            if (has) {
                const long long pi = B.pt_off + n0 + kTile * w + (threadIdx.x & 63);
                ex = R.px[pi];
                ey = R.py[pi];
                ez = R.pz[pi];
            }
            __syncthreads();   // the previous half's epilogue is done with Xs
        }
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
            for (int nb = 2 * w; nb < 2 * w + 2; ++nb)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    Xs[wm * 32 + mb * 16 + M::acc_row(r, lane)][wn * 32 + (nb & 1) * 16 + (lane & 15)] =
                        double(acc[mb][nb][r]);
        __syncthreads();
        rho_epilogue<GGA>(B, R, m0, n0 + kTile * w, mt, Xs, fsh, frow, ex, ey, ez, has, scratch);
    }
}

// 64 x 64 tiles (FP64 and FP32), four workgroups per CU.
template <bool GGA, typename T>
__global__ __launch_bounds__(256) void k_gemm_rho(
    const WaveBatch* __restrict__ wb, const int2* __restrict__ tmap, int ntiles,
    const ReqDev* __restrict__ reqs, char* __restrict__ scratch) {
    gemm_rho_tile<GGA, T, 1>(wb, tmap, ntiles, reqs, scratch);
}

// 64 x 128 tiles (FP64), three workgroups per CU.
template <bool GGA>
__global__ __launch_bounds__(256, 3) void k_gemm_rho_wide(
    const WaveBatch* __restrict__ wb, const int2* __restrict__ tmap, int ntiles,
    const ReqDev* __restrict__ reqs, char* __restrict__ scratch) {
    gemm_rho_tile<GGA, double, 2>(wb, tmap, ntiles, reqs, scratch);
}

// ------------------------------------------------- functional + Z matrix --
// Functional: one workgroup per batch, one thread per point: rho, grad rho
// from the partials, the functional, the batch's E_xc and N_e partials, and
// the point's Z factors a = w v_rho / 2 and b = 2 w v_sigma grad rho, written
// over the first row tile's partials (each thread reads all of its point's
// partials before it writes there, and no other thread touches that point).
template <bool GGA>
__global__ __launch_bounds__(256) void k_func(const WaveBatch* __restrict__ wb,
                                              const ReqDev* __restrict__ reqs,
                                              char* __restrict__ scratch) {
    const WaveBatch B = wb[blockIdx.x];
    const ReqG R = global_view(reqs[B.req]);
    const gptr<const double> W = R.pw;
    const double rho_thresh = R.rho_thresh;
    __shared__ double red[256];
    double* part = (double*)(scratch + 8 * B.part_off);
    double eacc = 0.0, nacc = 0.0;
    for (int i = threadIdx.x; i < B.ngp; i += blockDim.x) {
        double a = 0.0, bx = 0.0, by = 0.0, bz = 0.0;
        if (i < B.ng) {
            double rho = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
            for (int mt = 0; mt < B.nmt; ++mt) {
                const double* pp = part + (size_t)mt * 4 * B.ngp + i;
                rho += pp[0];
                if (GGA) {
                    gx += pp[B.ngp];
                    gy += pp[2 * B.ngp];
                    gz += pp[3 * B.ngp];
                }
            }
            const double w = W[B.pt_off + i];
            nacc += w * rho;
            if (rho >= rho_thresh) {
                if (GGA) {
                    gx *= 2.0;
                    gy *= 2.0;
                    gz *= 2.0;
                    const double sigma = gx * gx + gy * gy + gz * gz;
                    double e, vr, vs;
                    fn::gga_pbe(rho, sigma, e, vr, vs);
                    eacc += w * e;
                    a = 0.5 * w * vr;
                    const double f = 2.0 * w * vs;
                    bx = f * gx;
                    by = f * gy;
                    bz = f * gz;
                } else {
                    double e, vr;
                    fn::lda_svwn5(rho, e, vr);
                    eacc += w * e;
                    a = 0.5 * w * vr;
                }
            }
        }
        part[i] = a;
        part[(size_t)B.ngp + i] = bx;
        part[2 * (size_t)B.ngp + i] = by;
        part[3 * (size_t)B.ngp + i] = bz;
    }
    const double es = block_sum_256(eacc, red);
    const double ns = block_sum_256(nacc, red);
    if (threadIdx.x == 0) {
        R.epart[B.batch] = es;
        R.npart[B.batch] = ns;
    }
}

// Spin-unrestricted functional: one workgroup per batch, one thread per
// point. rho_s and grad rho_s from the alpha and the beta partials, the
// spin-polarised functional, the batch's E_xc and N_e partials, and each
// spin's Z factors a_s = w v_rho_s / 2 and
// b_a = w (2 v_sigma_aa grad rho_a + v_sigma_ab grad rho_b) (b_b likewise),
// written over the first row tile of that spin's partials.
template <bool GGA>
__global__ __launch_bounds__(256) void k_func_spin(const WaveBatch* __restrict__ wb,
                                                   const ReqDev* __restrict__ reqs,
                                                   char* __restrict__ scratch) {
    const WaveBatch B = wb[blockIdx.x];
    const ReqG R = global_view(reqs[B.req]);
    const gptr<const double> W = R.pw;
    const double thr = R.rho_thresh;
    __shared__ double red[256];
    double* pa = (double*)(scratch + 8 * B.part_off);
    double* pb = pa + (size_t)B.nmt * 4 * B.ngp;
    double eacc = 0.0, nacc = 0.0;
    for (int i = threadIdx.x; i < B.ngp; i += blockDim.x) {
        double fa[4] = {0.0, 0.0, 0.0, 0.0}, fb[4] = {0.0, 0.0, 0.0, 0.0};
        if (i < B.ng) {
            double ra = 0.0, rb = 0.0, ga[3] = {0.0, 0.0, 0.0}, gb[3] = {0.0, 0.0, 0.0};
            for (int mt = 0; mt < B.nmt; ++mt) {
                const size_t o = (size_t)mt * 4 * B.ngp + i;
                ra += pa[o];
                rb += pb[o];
                if (GGA) {
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        ga[d] += pa[o + (size_t)(d + 1) * B.ngp];
                        gb[d] += pb[o + (size_t)(d + 1) * B.ngp];
                    }
                }
            }
            const double w = W[B.pt_off + i];
            nacc += w * (ra + rb);
            if (ra + rb >= thr) {
                double e, va, vb;
                if (GGA) {
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        ga[d] *= 2.0;
                        gb[d] *= 2.0;
                    }
                    const double saa = ga[0] * ga[0] + ga[1] * ga[1] + ga[2] * ga[2];
                    const double sab = ga[0] * gb[0] + ga[1] * gb[1] + ga[2] * gb[2];
                    const double sbb = gb[0] * gb[0] + gb[1] * gb[1] + gb[2] * gb[2];
                    double vsaa, vsab, vsbb;
                    fn::gga_pbe_spin(ra, rb, saa, sab, sbb, thr, e, va, vb, vsaa, vsab, vsbb);
#pragma unroll
                    for (int d = 0; d < 3; ++d) {
                        fa[d + 1] = w * (2.0 * vsaa * ga[d] + vsab * gb[d]);
                        fb[d + 1] = w * (2.0 * vsbb * gb[d] + vsab * ga[d]);
                    }
                } else {
                    fn::lda_svwn5_spin(ra, rb, thr, e, va, vb);
                }
                eacc += w * e;
                fa[0] = 0.5 * w * va;
                fb[0] = 0.5 * w * vb;
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            pa[(size_t)q * B.ngp + i] = fa[q];
            pb[(size_t)q * B.ngp + i] = fb[q];
        }
    }
    const double es = block_sum_256(eacc, red);
    const double ns = block_sum_256(nacc, red);
    if (threadIdx.x == 0) {
        R.epart[B.batch] = es;
        R.npart[B.batch] = ns;
    }
}

// Z^j (eq. z_mat), stored in slab 1: z = a phi + b . grad phi with phi and
// grad phi re-evaluated from the shell data. One workgroup per batch; each
// lane takes a point (its coordinates and Z factors read once), the wave
// takes shells wave, wave + 4, ... of the batch's list. No LDS and few
// registers, so many workgroups share a CU.
template <typename T, bool SPH>
__global__ __launch_bounds__(256) void k_z(const WaveBatch* __restrict__ wb,
                                           const ReqDev* __restrict__ reqs,
                                           char* __restrict__ scratch) {
    exp_table_init();
    const WaveBatch B = wb[blockIdx.x];
    const ReqG R = global_view(reqs[B.req]);
    const double* fac = (const double*)(scratch + 8 * B.part_off);
    T* Zm = (T*)(scratch + 8 * B.z_off);
    const long long npad = (long long)(B.nbp - B.nb) * B.ngp;
    for (long long k = threadIdx.x; k < npad; k += blockDim.x) Zm[(size_t)B.nb * B.ngp + k] = T(0);
    __syncthreads();  // the exponential table
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
    for (int i = lane; i < B.ngp; i += 64) {
        const bool hasp = i < B.ng;
        double px = 0.0, py = 0.0, pz = 0.0;
        if (hasp) {
            px = R.px[B.pt_off + i];
            py = R.py[B.pt_off + i];
            pz = R.pz[B.pt_off + i];
        }
        const double a = fac[i], bx = fac[(size_t)B.ngp + i], by = fac[2 * (size_t)B.ngp + i],
                     bz = fac[3 * (size_t)B.ngp + i];
        for (int sl = wave; sl < B.nshell; sl += 4) {
            const int sidx = R.shell_list[B.shell_off + sl];
            const int loff = R.shell_loff[B.shell_off + sl];
            const ShellDev sh = load_shell(R.shells + sidx);
            double dx = 0.0, dy = 0.0, dz = 0.0, rad = 0.0, drad = 0.0;
            if (hasp) {
                const double r2 = dist2_nc(px, py, pz, sh, dx, dy, dz);
                shell_radial(sh, R.palpha, R.pcoef, r2, rad, drad);
            }
            T* out = Zm + (size_t)loff * B.ngp + i;
            if (SPH && sh.pure) {
                if (sh.L == 2) z_shell<2, T, SPH>(dx, dy, dz, rad, drad, a, bx, by, bz, out, B.ngp);
                else z_shell<3, T, SPH>(dx, dy, dz, rad, drad, a, bx, by, bz, out, B.ngp);
            } else {
                switch (sh.L) {
                    case 0: z_shell<0, T>(dx, dy, dz, rad, drad, a, bx, by, bz, out, B.ngp); break;
                    case 1: z_shell<1, T>(dx, dy, dz, rad, drad, a, bx, by, bz, out, B.ngp); break;
                    case 2: z_shell<2, T>(dx, dy, dz, rad, drad, a, bx, by, bz, out, B.ngp); break;
                    default: z_shell<3, T>(dx, dy, dz, rad, drad, a, bx, by, bz, out, B.ngp); break;
                }
            }
        }
    }
}

// Gradient slabs of a meta-GGA batch: d phi/dx, d phi/dy, d phi/dz of its
// screened functions at its points (rows and padding as in Phi), in the
// three slabs after its partials. The walk of the Z kernel, with the Z
// factors a = 0 and b = the unit vector of each direction.
template <int L, bool PURE>
__device__ inline void grad_shell3(double dx, double dy, double dz, double rad, double drad,
                                   double* out, size_t slab, int ngp) {
    z_shell<L, double, PURE>(dx, dy, dz, rad, drad, 0.0, 1.0, 0.0, 0.0, out, ngp);
    z_shell<L, double, PURE>(dx, dy, dz, rad, drad, 0.0, 0.0, 1.0, 0.0, out + slab, ngp);
    z_shell<L, double, PURE>(dx, dy, dz, rad, drad, 0.0, 0.0, 0.0, 1.0, out + 2 * slab, ngp);
}

template <bool SPH>
__global__ __launch_bounds__(256) void k_grad(const WaveBatch* __restrict__ wb,
                                              const ReqDev* __restrict__ reqs,
                                              char* __restrict__ scratch) {
    exp_table_init();
    const WaveBatch B = wb[blockIdx.x];
    const ReqG R = global_view(reqs[B.req]);
    double* G = (double*)(scratch + 8 * meta_grad_off(B, 0));
    const size_t slab = (size_t)B.nbp * B.ngp;
    const long long npad = (long long)(B.nbp - B.nb) * B.ngp;
    for (int d = 0; d < 3; ++d)
        for (long long k = threadIdx.x; k < npad; k += blockDim.x)
            G[d * slab + (size_t)B.nb * B.ngp + k] = 0.0;
    __syncthreads();  // the exponential table
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
    for (int i = lane; i < B.ngp; i += 64) {
        const bool hasp = i < B.ng;
        double px = 0.0, py = 0.0, pz = 0.0;
        if (hasp) {
            px = R.px[B.pt_off + i];
            py = R.py[B.pt_off + i];
            pz = R.pz[B.pt_off + i];
        }
        for (int sl = wave; sl < B.nshell; sl += 4) {
            const int sidx = R.shell_list[B.shell_off + sl];
            const int loff = R.shell_loff[B.shell_off + sl];
            const ShellDev sh = load_shell(R.shells + sidx);
            double dx = 0.0, dy = 0.0, dz = 0.0, rad = 0.0, drad = 0.0;
            if (hasp) {
                const double r2 = dist2_nc(px, py, pz, sh, dx, dy, dz);
                shell_radial(sh, R.palpha, R.pcoef, r2, rad, drad);
            }
            double* out = G + (size_t)loff * B.ngp + i;
            if (SPH && sh.pure) {
                if (sh.L == 2) grad_shell3<2, SPH>(dx, dy, dz, rad, drad, out, slab, B.ngp);
                else grad_shell3<3, SPH>(dx, dy, dz, rad, drad, out, slab, B.ngp);
            } else {
                switch (sh.L) {
                    case 0: grad_shell3<0, false>(dx, dy, dz, rad, drad, out, slab, B.ngp); break;
                    case 1: grad_shell3<1, false>(dx, dy, dz, rad, drad, out, slab, B.ngp); break;
                    case 2: grad_shell3<2, false>(dx, dy, dz, rad, drad, out, slab, B.ngp); break;
                    default: grad_shell3<3, false>(dx, dy, dz, rad, drad, out, slab, B.ngp); break;
                }
            }
        }
    }
}

// Meta-GGA functional (TPSS): one workgroup per batch, one thread per point.
// rho and grad rho from the density partials; tau = 1/2 sum_d of row 1 + d
// of partial set d (the contraction of P with d phi/dd, dotted with d phi/dd
// in the density epilogue); E_xc and N_e partials. Writes the Z factors
// a = w v_rho / 2, b = 2 w v_sigma grad rho over the first row tile of the
// density partials and, over the first row tile of set d, the factors
// (0, c e_d) with c = w v_tau / 4, so that the Z kernel run on set d forms
// Z_d = c d phi/dd and the potential contraction with the d-th gradient
// slab adds 2 c d phi/dd d phi/dd^T = w v_tau / 2 d phi/dd d phi/dd^T.
__global__ __launch_bounds__(256) void k_func_meta(const WaveBatch* __restrict__ wb,
                                                   const ReqDev* __restrict__ reqs,
                                                   char* __restrict__ scratch) {
    const WaveBatch B = wb[blockIdx.x];
    const ReqG R = global_view(reqs[B.req]);
    const gptr<const double> W = R.pw;
    const double thr = R.rho_thresh;
    __shared__ double red[256];
    double* part = (double*)(scratch + 8 * B.part_off);
    double* tp[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) tp[d] = (double*)(scratch + 8 * meta_part_off(B, d));
    double eacc = 0.0, nacc = 0.0;
    for (int i = threadIdx.x; i < B.ngp; i += blockDim.x) {
        double f[4] = {0.0, 0.0, 0.0, 0.0}, cf = 0.0;
        if (i < B.ng) {
            double rho = 0.0, g[3] = {0.0, 0.0, 0.0}, tau = 0.0;
            for (int mt = 0; mt < B.nmt; ++mt) {
                const size_t o = (size_t)mt * 4 * B.ngp + i;
                rho += part[o];
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    g[d] += part[o + (size_t)(d + 1) * B.ngp];
                    tau += tp[d][o + (size_t)(d + 1) * B.ngp];
                }
            }
            tau *= 0.5;
            const double w = W[B.pt_off + i];
            nacc += w * rho;
            if (rho >= thr) {
#pragma unroll
                for (int d = 0; d < 3; ++d) g[d] *= 2.0;
                const double sigma = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
                double e, vr, vs, vt;
                mgga::tpss(rho, sigma, tau, e, vr, vs, vt);
                eacc += w * e;
                f[0] = 0.5 * w * vr;
#pragma unroll
                for (int d = 0; d < 3; ++d) f[d + 1] = 2.0 * w * vs * g[d];
                cf = 0.25 * w * vt;
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) part[(size_t)q * B.ngp + i] = f[q];
#pragma unroll
        for (int d = 0; d < 3; ++d)
#pragma unroll
            for (int q = 0; q < 4; ++q) tp[d][(size_t)q * B.ngp + i] = (q == d + 1) ? cf : 0.0;
    }
    const double es = block_sum_256(eacc, red);
    const double ns = block_sum_256(nacc, red);
    if (threadIdx.x == 0) {
        R.epart[B.batch] = es;
        R.npart[B.batch] = ns;
    }
}

// ------------------------------------------------------ potential (SYR2K) --
// Lower-triangle tile (I >= J) of V^j = Z Phi^T + Phi Z^T, 64 x 64, over all
// points of the batch, added into V[f(row)][f(col)] (f ascending, so the
// global entry is in the lower triangle too). A diagonal tile (I = J) loads
// its row operands only and reads them again as its column operands. T is
// the arithmetic (and the storage of Z), TP the storage of Phi.
template <typename T, typename TP>
__global__ __launch_bounds__(256) void k_syr2k(
    const WaveBatch* __restrict__ wb, const int2* __restrict__ tmap, int ntiles,
    const ReqDev* __restrict__ reqs, const char* __restrict__ scratch) {
    using M = Mfma<T>;
    const int t = xcd_remap(blockIdx.x, ntiles);
    const int2 tb = tmap[t];
    const int bi = tb.x;
    const WaveBatch B = wb[bi];
    const ReqG R = global_view(reqs[B.req]);
    const gptr<const int> func_list = R.func_list;
    const gptr<double> V = R.V;
    const int nbf = R.nbf;
    const int lt = tb.y;
    int I = (int)((sqrt(8.0 * lt + 1.0) - 1.0) * 0.5);
    while ((I + 1) * (I + 2) / 2 <= lt) ++I;
    while (I * (I + 1) / 2 > lt) --I;
    const int J = lt - I * (I + 1) / 2;
    const gptr<const TP> Phi = (gptr<const TP>)phi_slab(B, R, (char*)scratch);
    const gptr<const T> Zm = (gptr<const T>)to_global(scratch + 8 * B.z_off);
    const gptr<const int> fl = func_list + B.func_off;

    // K steps of 8. FP64: one LDS buffer, 19 KB, and two register sets (the
    // operands of the next two steps), so the register count (four
    // workgroups per CU) sets the occupancy, not LDS; one register set fits
    // five workgroups per CU but waits for each step's loads within the
    // step (1.4 % slower on the chain), and so does forcing five with two
    // sets (registers spilled). FP32 arithmetic: two LDS buffers (measured
    // faster there).
    constexpr int KS = 8;
    // row pitch: 9 doubles, or 12 floats (the 4-byte operand reads of a wave
    // then fall in distinct banks)
    constexpr int KP = sizeof(T) == 8 ? KS + 1 : KS + 4;
    constexpr int NBUF = sizeof(T) == 8 ? 1 : 2;
    __shared__ T sZI[NBUF][kTile][KP], sPI[NBUF][kTile][KP];
    __shared__ T sPJ[NBUF][kTile][KP], sZJ[NBUF][kTile][KP];
    // global function indices of the tile's rows and columns (-1: padding)
    __shared__ int sfI[kTile], sfJ[kTile];

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform
    if (tid < kTile) {
        const int r = I * kTile + tid;
        sfI[tid] = r < B.nb ? fl[r] : -1;
    } else if (tid < 2 * kTile) {
        const int r = J * kTile + tid - kTile;
        sfJ[tid - kTile] = r < B.nb ? fl[r] : -1;
    }
    const int wm = wave >> 1, wn = wave & 1;
    const int lr = tid >> 2, lc = (tid & 3) * 2;
    const int rI = I * kTile + lr, rJ = J * kTile + lr;
    // a diagonal tile's column operands are its row operands
    const bool diag = I == J;
    T (*tPJ)[kTile][KP] = diag ? sPI : sPJ;
    T (*tZJ)[kTile][KP] = diag ? sZI : sZJ;
    const bool vI = rI < B.nbp, vJ = rJ < B.nbp;
    const gptr<const T> zI = Zm + (size_t)(vI ? rI : 0) * B.ngp;
    const gptr<const TP> pI = Phi + (size_t)(vI ? rI : 0) * B.ngp;
    const gptr<const T> zJ = Zm + (size_t)(vJ ? rJ : 0) * B.ngp;
    const gptr<const TP> pJ = Phi + (size_t)(vJ ? rJ : 0) * B.ngp;

    // FP32 (one register set, two LDS buffers): loads from the clamped
    // (always valid) rows, padding rows zeroed after the load, so no branch
    // separates the loads (with a branch around each, the 4-byte loads were
    // issued and waited for one at a time).
    T g[4][2];
    auto gload = [&](int ks) {
        const int k0 = ks * KS + lc;
        if constexpr (sizeof(T) == 4) {
            TP ph[2][2];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                g[0][q] = zI[k0 + q];
                ph[0][q] = pI[k0 + q];
            }
            if (!diag) {
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    ph[1][q] = pJ[k0 + q];
                    g[3][q] = zJ[k0 + q];
                }
            }
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                g[0][q] = vI ? g[0][q] : T(0);
                g[1][q] = vI ? T(ph[0][q]) : T(0);
            }
            if (!diag) {
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    g[2][q] = vJ ? T(ph[1][q]) : T(0);
                    g[3][q] = vJ ? g[3][q] : T(0);
                }
            }
        }
    };
    auto sstore = [&](int buf) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            sZI[buf][lr][lc + q] = g[0][q];
            sPI[buf][lr][lc + q] = g[1][q];
        }
        if (!diag) {
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                sPJ[buf][lr][lc + q] = g[2][q];
                sZJ[buf][lr][lc + q] = g[3][q];
            }
        }
    };
    typename M::acc acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = M::zero();

    // the points beyond n_g are zero padding: K runs to n_g rounded up to KS
    const int nk = (B.ng + KS - 1) / KS;
    // skip 16 x 16 blocks that are padding or lie above the diagonal
    bool live[2][2];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
            const int r0 = I * kTile + wm * 32 + mb * 16;
            const int c0 = J * kTile + wn * 32 + nb * 16;
            live[mb][nb] = (r0 < B.nb) && (c0 < B.nb) && (c0 <= r0 + 15);
        }
    // one K step of 8 from LDS buffer cur
    auto compute = [&](int cur) {
#pragma unroll
        for (int kk = 0; kk < KS / 4; ++kk) {
            const int kc = kk * 4 + (lane >> 4);
            T az[2], ap[2], bp[2], bz[2];
#pragma unroll
            for (int mb = 0; mb < 2; ++mb) {
                const int r = wm * 32 + mb * 16 + (lane & 15);
                az[mb] = sZI[cur][r][kc];
                ap[mb] = sPI[cur][r][kc];
            }
#pragma unroll
            for (int nb = 0; nb < 2; ++nb) {
                const int r = wn * 32 + nb * 16 + (lane & 15);
                bp[nb] = tPJ[cur][r][kc];
                bz[nb] = tZJ[cur][r][kc];
            }
#pragma unroll
            for (int mb = 0; mb < 2; ++mb)
#pragma unroll
                for (int nb = 0; nb < 2; ++nb) {
                    if (!live[mb][nb]) continue;
                    acc[mb][nb] = M::mma(az[mb], bp[nb], acc[mb][nb]);
                    acc[mb][nb] = M::mma(ap[mb], bz[nb], acc[mb][nb]);
                }
        }
    };
    if constexpr (NBUF == 1) {
        // FP64: two register sets, the operands of step ks + 2 loading while
        // step ks is computed and those of step ks + 1 waiting to be stored.
        // Every step issues the same loads (clamped rows and steps; padding
        // rows zeroed at the store; a diagonal tile's loop is compiled
        // apart, without its column operands), so the wait before a store
        // leaves the newer step's loads in flight.
        T ga[4][2], gb[4][2];
        auto run = [&](auto dtag) {
            constexpr bool D = decltype(dtag)::value;
            auto load2 = [&](int ks, T (&gg)[4][2]) {
                const int k0 = min(ks, nk - 1) * KS + lc;
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    gg[0][q] = zI[k0 + q];
                    gg[1][q] = pI[k0 + q];
                }
                if constexpr (!D) {
#pragma unroll
                    for (int q = 0; q < 2; ++q) {
                        gg[2][q] = pJ[k0 + q];
                        gg[3][q] = zJ[k0 + q];
                    }
                }
            };
            auto store2 = [&](const T (&gg)[4][2]) {
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    sZI[0][lr][lc + q] = vI ? gg[0][q] : T(0);
                    sPI[0][lr][lc + q] = vI ? gg[1][q] : T(0);
                }
                if constexpr (!D) {
#pragma unroll
                    for (int q = 0; q < 2; ++q) {
                        sPJ[0][lr][lc + q] = vJ ? gg[2][q] : T(0);
                        sZJ[0][lr][lc + q] = vJ ? gg[3][q] : T(0);
                    }
                }
            };
            load2(0, ga);
            store2(ga);
            load2(1, gb);
            __syncthreads();
            auto step = [&](int ks, T (&gl)[4][2], T (&gs)[4][2]) {
                load2(ks + 2, gl);
                compute(0);
                __syncthreads();
                if (ks + 1 < nk) {
                    store2(gs);
                    __syncthreads();
                }
            };
            for (int ks = 0; ks < nk; ks += 2) {
                step(ks, ga, gb);
                if (ks + 1 < nk) step(ks + 1, gb, ga);
            }
        };
        if (diag) run(std::true_type{});
        else run(std::false_type{});
    } else {
        gload(0);
        sstore(0);
        __syncthreads();
        for (int ks = 0; ks < nk; ++ks) {
            const int cur = ks & 1;
            if (ks + 1 < nk) gload(ks + 1);
            compute(cur);
            if (ks + 1 < nk) sstore(cur ^ 1);
            __syncthreads();
        }
    }
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int tr = wm * 32 + mb * 16 + M::acc_row(r, lane);
            const int row = I * kTile + tr;
            if (row >= B.nb) continue;
            const gptr<double> vrow = V + (size_t)sfI[tr] * nbf;
#pragma unroll
            for (int nb = 0; nb < 2; ++nb) {
                const int tc = wn * 32 + nb * 16 + (lane & 15);
                const int col = J * kTile + tc;
                if (col < B.nb && col <= row)
                    __hip_atomic_fetch_add(vrow + sfJ[tc], double(acc[mb][nb][r]),
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
}

// ----------------------------------------------- split-BF16 contractions --
// Both contractions run on v_mfma_f32_16x16x32_bf16 (FP32 accumulation).
// Operand lane l of the MFMA holds A[l % 16][8 (l / 16) + t] and
// B[8 (l / 16) + t][l % 16], t = 0..7; the accumulator layout is FP32's (row
// 4 (l / 16) + r). Tiles are 64 x 64 with K steps of 32, stored k-contiguous
// in LDS with a row pitch of 40 bf16, so that the 16-byte fragment reads of
// 16 lanes fall in distinct banks.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));
typedef unsigned long long v2u64 __attribute__((ext_vector_type(2)));
constexpr int kKB = 32;        // K step of the split-BF16 kernels
constexpr int kBP = kKB + 8;   // LDS row pitch in bf16

// Potential contraction: x = hi + lo with hi = bf16(x), lo = bf16(x - hi),
// and a b ~ hi hi + hi lo + lo hi (the lo lo term and what lies below the
// two parts are dropped: about 16 significant bits per product).
__device__ inline void split_bf16(double x, __bf16& h, __bf16& l) {
    h = (__bf16)(float)x;
    l = (__bf16)(float)(x - (double)(float)h);
}

__device__ inline v4f mfma_bf16x3(const bf16x8& ah, const bf16x8& al, const bf16x8& bh,
                                  const bf16x8& bl, v4f c) {
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, c, 0, 0, 0);
    return c;
}

// Density contraction: exact digit products. The entries of P over their
// row's scale and of Phi over their point's scale (both powers of two) are
// cut into four digits each (digits_packed). A product of two digits is an
// integer below 2^14 in magnitude and a sum of 2^10 of them stays below
// 2^24, so FP32 accumulation of digit products is exact however the
// hardware orders it. The products of digit orders u + v = g (g <= 3, ten
// products per pair of entries) share one accumulator of weight
// 2^{-14-8g}; every eight K steps (256 terms: at most 4 x 256 products of
// 2^14, i.e. 2^24) the accumulators are added into FP64 and cleared.
__device__ inline __bf16 bits_bf16(unsigned short v) {
    return __builtin_bit_cast(__bf16, v);
}

// Digits of P, one workgroup per row mu: the row scale s_mu is the least
// power of two not below max_nu |P_mu nu| (1 for a zero row), and entry
// (mu, nu) is stored as its four digits of P_mu nu / s_mu packed in 64 bits
// (digit u in bits 16 u .. 16 u + 15).
__global__ __launch_bounds__(256) void k_p_digits(const double* __restrict__ P, int nbf,
                                                  unsigned long long* __restrict__ dig,
                                                  double* __restrict__ scale) {
    const int mu = blockIdx.x;
    const double* row = P + (size_t)mu * nbf;
    __shared__ double red[256];
    double m = 0.0;
    for (int nu = threadIdx.x; nu < nbf; nu += blockDim.x) m = fmax(m, fabs(row[nu]));
    red[threadIdx.x] = m;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + st]);
        __syncthreads();
    }
    const double mx = red[0];
    int e = 0;
    (void)frexp(mx, &e);
    e = max(e, -1000);  // 1 / scale stays finite
    const double sc = mx > 0.0 ? ldexp(1.0, e) : 1.0;
    const double inv = mx > 0.0 ? ldexp(1.0, -e) : 1.0;
    if (threadIdx.x == 0) scale[mu] = sc;
    unsigned long long* drow = dig + (size_t)mu * nbf;
    for (int nu = threadIdx.x; nu < nbf; nu += blockDim.x) drow[nu] = digits_packed(row[nu] * inv);
}

// X = P^j Phi^j from digits: X[mu][i] = s_mu s_i 2^{-14}
// sum_{u+v<=3} 2^{-8(u+v)} sum_nu dP_u[mu][nu] dPhi_v[nu][i], with the digits
// of P gathered from the precomputed array through the batch's function list
// and those of Phi read from the digit slab the collocation kernel wrote.
// Same tiles and epilogue as k_gemm_rho; one LDS buffer (eight digit planes,
// 40 KB) with the next step's loads in registers.
template <bool GGA>
__global__ __launch_bounds__(256, 3) void k_gemm_rho_bf16(
    const WaveBatch* __restrict__ wb, const int2* __restrict__ tmap, int ntiles,
    const ReqDev* __restrict__ reqs, char* __restrict__ scratch) {
    const int t = xcd_remap(blockIdx.x, ntiles);
    const int2 tb = tmap[t];
    const WaveBatch B = wb[tb.x];
    const ReqG R = global_view(reqs[B.req]);
    const int nbf = R.nbf;
    const int lt = tb.y;
    const int ntn = B.ngp / kTile;
    const int mt = lt / ntn, nt = lt - mt * ntn;
    const int m0 = mt * kTile, n0 = nt * kTile;
    exp_table_init();
    const gptr<const char> phi = phi_slab(B, R, scratch);
    const gptr<const unsigned long long> Phid = (gptr<const unsigned long long>)phi;
    const gptr<const double> pscale = (gptr<const double>)phi + scale_row_off(B);
    const gptr<const int> fl = R.func_list + B.func_off;
    // the epilogue's point (one per lane), loaded now so that its latency hides
    const bool has = n0 + (int)(threadIdx.x & 63) < B.ng;
    double ex = 0.0, ey = 0.0, ez = 0.0;
    if (has) {
        const long long pi = B.pt_off + n0 + (threadIdx.x & 63);
        ex = R.px[pi];
        ey = R.py[pi];
        ez = R.pz[pi];
    }

    // digit planes 0-3 of the A tile (rows of P^j), 4-7 of the B tile (points)
    constexpr int kPlaneBytes = kTile * kBP * 2;
    constexpr int kOpBytes = 8 * kPlaneBytes;
    constexpr int kXBytes = kTile * (kTile + 1) * 8;
    __shared__ __attribute__((aligned(16))) char lds[kOpBytes > kXBytes ? kOpBytes : kXBytes];
    auto plane = [&](int p) { return reinterpret_cast<__bf16 (*)[kBP]>(lds + p * kPlaneBytes); };
    double (*Xs)[kTile + 1] = reinterpret_cast<double (*)[kTile + 1]>(lds);
    __shared__ int frow[kTile], fsh[kTile];
    __shared__ __attribute__((aligned(16))) int sfl[2][kKB];

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform
    const int wm = wave >> 1, wn = wave & 1;
    const int nk = (B.nbp + kKB - 1) / kKB;
    int fnext = -1;
    auto fetch = [&](int ks) {
        if (tid < kKB) {
            const int k = ks * kKB + tid;
            fnext = k < B.nb ? fl[k] : -1;
        }
    };
    auto fput = [&](int slot) {
        if (tid < kKB) sfl[slot][tid] = fnext;
    };
    fetch(0);
    fput(0);
    if (nk > 1) {
        fetch(1);
        fput(1);
    }
    if (tid < kTile) {
        const int f = (m0 + tid < B.nb) ? fl[m0 + tid] : -1;
        frow[tid] = f;
        fsh[tid] = f >= 0 ? R.func_shell[f] : 0;
    }
    __syncthreads();

    // A: row tid / 4 and K offset 8 (tid % 4); B: point tid % 64 and K offset
    // 8 (tid / 64), so that a wave's Phi loads are 64 consecutive points
    const int ar = tid >> 2, ak = (tid & 3) * 8;
    const int bn = tid & 63, bk = (tid >> 6) * 8;
    const int fr = frow[ar];
    const gptr<const unsigned long long> Prow = R.Pdig + (size_t)(fr >= 0 ? fr : 0) * nbf;
    int fc[8];
    unsigned long long pa[8], pb[8];
    auto gload = [&](int ks) {
        const int4 u = *reinterpret_cast<const int4*>(&sfl[ks & 1][ak]);
        const int4 v = *reinterpret_cast<const int4*>(&sfl[ks & 1][ak + 4]);
        fc[0] = u.x; fc[1] = u.y; fc[2] = u.z; fc[3] = u.w;
        fc[4] = v.x; fc[5] = v.y; fc[6] = v.z; fc[7] = v.w;
        // loads go to valid (clamped) addresses; padding is zeroed at the store
#pragma unroll
        for (int q = 0; q < 8; ++q) pa[q] = Prow[fc[q] >= 0 ? fc[q] : 0];
        const int kb = ks * kKB + bk;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int k = kb + q;
            pb[q] = Phid[(size_t)(k < B.nbp ? k : 0) * B.ngp + n0 + bn];
        }
    };
    auto sstore = [&](int ks) {
        bf16x8 d[4];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const unsigned long long w = (fr >= 0 && fc[q] >= 0) ? pa[q] : 0ull;
#pragma unroll
            for (int u = 0; u < 4; ++u) d[u][q] = bits_bf16((unsigned short)(w >> (16 * u)));
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) *reinterpret_cast<bf16x8*>(&plane(u)[ar][ak]) = d[u];
        const int kb = ks * kKB + bk;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const unsigned long long w = kb + q < B.nbp ? pb[q] : 0ull;
#pragma unroll
            for (int u = 0; u < 4; ++u) d[u][q] = bits_bf16((unsigned short)(w >> (16 * u)));
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) *reinterpret_cast<bf16x8*>(&plane(4 + u)[bn][bk]) = d[u];
    };

    // each wave: one 32 x 32 block (v_mfma_f32_32x32x16_bf16; operand lane l
    // holds A[l % 32][8 (l / 32) + t] and B[8 (l / 32) + t][l % 32], and
    // accumulator register r of lane l holds C[8 (r / 4) + 4 (l / 32) + r % 4][l % 32])
    v16f acc[4];
    double acc64[16];
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[g][r] = 0.f;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc64[r] = 0.0;
    const bool live = (m0 + wm * 32 < B.nb) && (n0 + wn * 32 < B.ng);
    auto flush = [&]() {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            double v = (double)acc[3][r];
            v = fma(v, 0x1p-8, (double)acc[2][r]);
            v = fma(v, 0x1p-8, (double)acc[1][r]);
            v = fma(v, 0x1p-8, (double)acc[0][r]);
            acc64[r] += v;
#pragma unroll
            for (int g = 0; g < 4; ++g) acc[g][r] = 0.f;
        }
    };

    // per step: load, stage into LDS, compute (no operands carried across the
    // MFMAs in registers: three workgroups per CU hide each other's loads)
    if (nk > 2) fetch(2);
    const int ar32 = lane & 31, fk = 8 * (lane >> 5);
    for (int ks = 0; ks < nk; ++ks) {
        gload(ks);
        sstore(ks);
        __syncthreads();
        // every thread has read this step's index slot: refill it with step ks + 2
        if (ks + 2 < nk) {
            fput(ks & 1);
            if (ks + 3 < nk) fetch(ks + 3);
        }
        if (live) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                bf16x8 a[4], b[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    a[u] = *reinterpret_cast<const bf16x8*>(
                        &plane(u)[wm * 32 + ar32][h * 16 + fk]);
                    b[u] = *reinterpret_cast<const bf16x8*>(
                        &plane(4 + u)[wn * 32 + ar32][h * 16 + fk]);
                }
#pragma unroll
                for (int g = 0; g < 4; ++g)
#pragma unroll
                    for (int u = 0; u <= g; ++u)
                        acc[g] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[u], b[g - u], acc[g],
                                                                         0, 0, 0);
            }
        }
        if ((ks & 7) == 7) flush();
        __syncthreads();
    }
    flush();

    // X = acc64 2^{-14} s_mu s_i (the loop ended on a barrier, so the operand
    // planes are free for the X tile)
    {
        const int tc = wn * 32 + ar32;
        const double sn = pscale[n0 + tc] * 0x1p-14;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int tr = wm * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
            const int f = frow[tr];
            const double sm = f >= 0 ? R.Pscale[f] : 0.0;
            Xs[tr][tc] = acc64[r] * sm * sn;
        }
    }
    __syncthreads();
    rho_epilogue<GGA>(B, R, m0, n0, mt, Xs, fsh, frow, ex, ey, ez, has, scratch);
}

// Potential contraction V^j = Z Phi^T + Phi Z^T in split BF16, lower-
// triangle tiles as in k_syr2k (diagonal tiles reuse their row operands),
// one LDS buffer with the next step's loads in registers. Z (FP32) is split
// as hi + lo; Phi comes from the digit slab: hi = s_i 2^-7 d0 and
// lo = s_i 2^-15 d1 (exact in BF16), about 15 bits relative to the point's
// largest function value.
__global__ __launch_bounds__(256) void k_syr2k_bf16(
    const WaveBatch* __restrict__ wb, const int2* __restrict__ tmap, int ntiles,
    const ReqDev* __restrict__ reqs, const char* __restrict__ scratch) {
    const int t = xcd_remap(blockIdx.x, ntiles);
    const int2 tb = tmap[t];
    const WaveBatch B = wb[tb.x];
    const ReqG R = global_view(reqs[B.req]);
    const gptr<const int> func_list = R.func_list;
    const gptr<double> V = R.V;
    const int nbf = R.nbf;
    const int lt = tb.y;
    int I = (int)((sqrt(8.0 * lt + 1.0) - 1.0) * 0.5);
    while ((I + 1) * (I + 2) / 2 <= lt) ++I;
    while (I * (I + 1) / 2 > lt) --I;
    const int J = lt - I * (I + 1) / 2;
    const gptr<const char> phi = phi_slab(B, R, (char*)scratch);
    const gptr<const unsigned long long> Phid = (gptr<const unsigned long long>)phi;
    const gptr<const float> Zm = (gptr<const float>)to_global(scratch + 8 * B.z_off);
    const gptr<const double> pscale = (gptr<const double>)phi + scale_row_off(B);
    const gptr<const int> fl = func_list + B.func_off;

    // ZI, PI, PJ, ZJ, each (hi, lo): one buffer
    constexpr int kOpBytes = kTile * kBP * 2;
    __shared__ __attribute__((aligned(16))) char lds[8 * kOpBytes];
    auto tile = [&](int which) {
        return reinterpret_cast<__bf16 (*)[kBP]>(lds + which * kOpBytes);
    };
    __shared__ int sfI[kTile], sfJ[kTile];

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform
    if (tid < kTile) {
        const int r = I * kTile + tid;
        sfI[tid] = r < B.nb ? fl[r] : -1;
    } else if (tid < 2 * kTile) {
        const int r = J * kTile + tid - kTile;
        sfJ[tid - kTile] = r < B.nb ? fl[r] : -1;
    }
    const int wm = wave >> 1, wn = wave & 1;
    const int lr = tid >> 2, lk = (tid & 3) * 8;
    const int rI = I * kTile + lr, rJ = J * kTile + lr;
    const bool vI = rI < B.nbp, vJ = rJ < B.nbp;
    // operand a: 0 = Z_I, 1 = Phi_I, 2 = Phi_J, 3 = Z_J
    const gptr<const float> zsrc[2] = {Zm + (size_t)(vI ? rI : 0) * B.ngp,
                                       Zm + (size_t)(vJ ? rJ : 0) * B.ngp};
    const gptr<const unsigned long long> psrc[2] = {Phid + (size_t)(vI ? rI : 0) * B.ngp,
                                         Phid + (size_t)(vJ ? rJ : 0) * B.ngp};
    // a diagonal tile's column operands are its row operands
    const bool diag = I == J;
    v4f gz[2][2];
    v2u64 gp[2][4];
    float sc[8];     // s_i 2^-7 of the step's eight points
    auto gload = [&](int ks) {
        const int k0 = ks * kKB + lk;
#pragma unroll
        for (int q = 0; q < 8; ++q) sc[q] = (float)(pscale[k0 + q] * 0x1p-7);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (h == 1 && diag) continue;
            gz[h][0] = *reinterpret_cast<gptr<const v4f>>(zsrc[h] + k0);
            gz[h][1] = *reinterpret_cast<gptr<const v4f>>(zsrc[h] + k0 + 4);
#pragma unroll
            for (int q = 0; q < 4; ++q)
                gp[h][q] = *reinterpret_cast<gptr<const v2u64>>(psrc[h] + k0 + 2 * q);
        }
    };
    auto put_z = [&](int which, const v4f (&g)[2], bool valid) {
        const float x[8] = {g[0].x, g[0].y, g[0].z, g[0].w, g[1].x, g[1].y, g[1].z, g[1].w};
        bf16x8 hv, lv;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            __bf16 hq, lq;
            split_bf16(valid ? (double)x[q] : 0.0, hq, lq);
            hv[q] = hq;
            lv[q] = lq;
        }
        *reinterpret_cast<bf16x8*>(&tile(which)[lr][lk]) = hv;
        *reinterpret_cast<bf16x8*>(&tile(which + 1)[lr][lk]) = lv;
    };
    auto put_phi = [&](int which, const v2u64 (&g)[4], bool valid) {
        const unsigned long long w[8] = {g[0].x, g[0].y, g[1].x, g[1].y,
                                         g[2].x, g[2].y, g[3].x, g[3].y};
        bf16x8 hv, lv;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const float d0 = (float)bits_bf16((unsigned short)w[q]);
            const float d1 = (float)bits_bf16((unsigned short)(w[q] >> 16));
            hv[q] = (__bf16)(valid ? d0 * sc[q] : 0.f);
            lv[q] = (__bf16)(valid ? d1 * (sc[q] * 0x1p-8f) : 0.f);
        }
        *reinterpret_cast<bf16x8*>(&tile(which)[lr][lk]) = hv;
        *reinterpret_cast<bf16x8*>(&tile(which + 1)[lr][lk]) = lv;
    };
    auto sstore = [&]() {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (h == 1 && diag) continue;
            const bool valid = h == 0 ? vI : vJ;
            put_z(h == 0 ? 0 : 6, gz[h], valid);
            put_phi(h == 0 ? 2 : 4, gp[h], valid);
        }
    };

    v4f acc[2][2];
    bool live[2][2];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
            acc[mb][nb] = v4f{0.f, 0.f, 0.f, 0.f};
            const int r0 = I * kTile + wm * 32 + mb * 16;
            const int c0 = J * kTile + wn * 32 + nb * 16;
            live[mb][nb] = (r0 < B.nb) && (c0 < B.nb) && (c0 <= r0 + 15);
        }
    // the points beyond n_g are zero padding, and n_gp is a multiple of 64:
    // K steps of 32 up to n_g stay inside the slab rows
    const int nk = (B.ng + kKB - 1) / kKB;
    gload(0);
    sstore();
    __syncthreads();
    const int fk = 8 * (lane >> 4);
    for (int ks = 0; ks < nk; ++ks) {
        if (ks + 1 < nk) gload(ks + 1);
        bf16x8 zih[2], zil[2], pih[2], pil[2], pjh[2], pjl[2], zjh[2], zjl[2];
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) {
            const int r = wm * 32 + mb * 16 + (lane & 15);
            zih[mb] = *reinterpret_cast<const bf16x8*>(&tile(0)[r][fk]);
            zil[mb] = *reinterpret_cast<const bf16x8*>(&tile(1)[r][fk]);
            pih[mb] = *reinterpret_cast<const bf16x8*>(&tile(2)[r][fk]);
            pil[mb] = *reinterpret_cast<const bf16x8*>(&tile(3)[r][fk]);
        }
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) {
            const int r = wn * 32 + nb * 16 + (lane & 15);
            pjh[nb] = *reinterpret_cast<const bf16x8*>(&tile(diag ? 2 : 4)[r][fk]);
            pjl[nb] = *reinterpret_cast<const bf16x8*>(&tile(diag ? 3 : 5)[r][fk]);
            zjh[nb] = *reinterpret_cast<const bf16x8*>(&tile(diag ? 0 : 6)[r][fk]);
            zjl[nb] = *reinterpret_cast<const bf16x8*>(&tile(diag ? 1 : 7)[r][fk]);
        }
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
            for (int nb = 0; nb < 2; ++nb) {
                if (!live[mb][nb]) continue;
                acc[mb][nb] = mfma_bf16x3(zih[mb], zil[mb], pjh[nb], pjl[nb], acc[mb][nb]);
                acc[mb][nb] = mfma_bf16x3(pih[mb], pil[mb], zjh[nb], zjl[nb], acc[mb][nb]);
            }
        __syncthreads();
        if (ks + 1 < nk) {
            sstore();
            __syncthreads();
        }
    }
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int tr = wm * 32 + mb * 16 + 4 * (lane >> 4) + r;
            const int row = I * kTile + tr;
            if (row >= B.nb) continue;
            const gptr<double> vrow = V + (size_t)sfI[tr] * nbf;
#pragma unroll
            for (int nb = 0; nb < 2; ++nb) {
                const int tc = wn * 32 + nb * 16 + (lane & 15);
                const int col = J * kTile + tc;
                if (col < B.nb && col <= row)
                    __hip_atomic_fetch_add(vrow + sfJ[tc], double(acc[mb][nb][r]),
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
}

// ---------------------------------------------------------------- misc ----
// Tile -> (batch, tile within the batch) for one launch over nwb batches whose
// tile counts have the exclusive prefix `prefix`: one thread per batch.
__global__ void k_tile_map(const int* __restrict__ prefix, int nwb, int2* __restrict__ map) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nwb) return;
    const int t0 = prefix[b], t1 = prefix[b + 1];
    for (int t = t0; t < t1; ++t) map[t] = make_int2(b, t - t0);
}

__global__ void k_put_req(ReqDev* dst, ReqDev v) { *dst = v; }

__global__ void k_fill(double* p, long long n, double v) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// upper triangle <- lower triangle
__global__ void k_mirror(double* V, int n) {
    const int c = blockIdx.x * 16 + (threadIdx.x & 15);
    const int r = blockIdx.y * 16 + (threadIdx.x >> 4);
    if (r < n && c < n && c > r) V[(size_t)r * n + c] = V[(size_t)c * n + r];
}

// E_xc and N_e from the per-batch partials: Neumaier-compensated sums in a
// fixed order (one workgroup), so the result does not depend on timing.
__device__ inline void two_sum_add(double& s, double& c, double x) {
    const double t = s + x;
    if (fabs(s) >= fabs(x)) c += (s - t) + x;
    else c += (x - t) + s;
    s = t;
}

__global__ void k_reduce_en(const double* epart, const double* npart, long long n,
                            double* out) {
    __shared__ double ss[2][256], cc[2][256];
    double se = 0.0, ce = 0.0, sn = 0.0, cn = 0.0;
    for (long long j = threadIdx.x; j < n; j += blockDim.x) {
        two_sum_add(se, ce, epart[j]);
        two_sum_add(sn, cn, npart[j]);
    }
    ss[0][threadIdx.x] = se;
    cc[0][threadIdx.x] = ce;
    ss[1][threadIdx.x] = sn;
    cc[1][threadIdx.x] = cn;
    __syncthreads();
    if (threadIdx.x < 2) {
        const int k = threadIdx.x;
        double s = 0.0, c = 0.0;
        for (int i = 0; i < 256; ++i) {
            two_sum_add(s, c, ss[k][i]);
            c += cc[k][i];
        }
        out[k] = s + c;
    }
}

// ------------------------------------------------------------- driver -----
// FP64 density contraction of one wave's batches: 64 x 128 tiles when the
// wave's work-weighted mean n_b is large (wide; the long K loops amortise
// the lower occupancy), else 64 x 64 tiles.
template <bool GGA>
static int launch_density_fp64(hipStream_t s, const WaveBatch* b, const int* gpre,
                               const int* wpre, int count, int gemm_tiles, int wide_tiles,
                               bool wide, const ReqDev* reqs, char* scr, int2* tmap) {
    const int n = wide ? wide_tiles : gemm_tiles;
    if (n <= 0) return XC_OK;
    hipLaunchKernelGGL(k_tile_map, dim3(grid_1d(count, 256)), dim3(256), 0, s, wide ? wpre : gpre,
                       count, tmap);
    XC_HIP(hipGetLastError());
    if (wide)
        hipLaunchKernelGGL((k_gemm_rho_wide<GGA>), dim3(n), dim3(256), 0, s, b,
                           (const int2*)tmap, n, reqs, scr);
    else
        hipLaunchKernelGGL((k_gemm_rho<GGA, double>), dim3(n), dim3(256), 0, s, b,
                           (const int2*)tmap, n, reqs, scr);
    XC_HIP(hipGetLastError());
    return XC_OK;
}

// T: storage of Phi and arithmetic of the density contraction; TZ: storage
// of Z and arithmetic of the potential contraction.
template <bool GGA, typename T, typename TZ>
static int launch_wave_t(PhaseTimer* timer, hipStream_t s, const WaveBatch* b,
                         const int* gpre, const int* spre, const int* wpre, int count,
                         int gemm_tiles, int syr_tiles, int wide_tiles, bool wide,
                         const ReqDev* reqs, char* scr, int2* tmap, bool colloc, bool sph) {
    if (colloc) {
        PhaseScope ps(timer, s, XC_PHASE_COLLOC);
        hipLaunchKernelGGL((k_colloc<T, false>), dim3(count), dim3(256), 0, s, b, reqs, scr);
        XC_HIP(hipGetLastError());
    }
    if constexpr (sizeof(T) == 8) {
        PhaseScope ps(timer, s, XC_PHASE_DENSITY);
        XC_TRY(launch_density_fp64<GGA>(s, b, gpre, wpre, count, gemm_tiles, wide_tiles, wide,
                                        reqs, scr, tmap));
    } else if (gemm_tiles > 0) {
        PhaseScope ps(timer, s, XC_PHASE_DENSITY);
        hipLaunchKernelGGL(k_tile_map, dim3(grid_1d(count, 256)), dim3(256), 0, s, gpre, count,
                           tmap);
        XC_HIP(hipGetLastError());
        hipLaunchKernelGGL((k_gemm_rho<GGA, T>), dim3(gemm_tiles), dim3(256), 0, s, b,
                           (const int2*)tmap, gemm_tiles, reqs, scr);
        XC_HIP(hipGetLastError());
    }
    {
        PhaseScope ps(timer, s, XC_PHASE_FUNCTIONAL);
        hipLaunchKernelGGL((k_func<GGA>), dim3(count), dim3(256), 0, s, b, reqs, scr);
        XC_HIP(hipGetLastError());
        if (sph) hipLaunchKernelGGL((k_z<TZ, true>), dim3(count), dim3(256), 0, s, b, reqs, scr);
        else hipLaunchKernelGGL((k_z<TZ, false>), dim3(count), dim3(256), 0, s, b, reqs, scr);
        XC_HIP(hipGetLastError());
    }
    if (syr_tiles > 0) {
        PhaseScope ps(timer, s, XC_PHASE_POTENTIAL);
        hipLaunchKernelGGL(k_tile_map, dim3(grid_1d(count, 256)), dim3(256), 0, s, spre, count,
                           tmap);
        XC_HIP(hipGetLastError());
        hipLaunchKernelGGL((k_syr2k<TZ, T>), dim3(syr_tiles), dim3(256), 0, s, b,
                           (const int2*)tmap, syr_tiles, reqs, (const char*)scr);
        XC_HIP(hipGetLastError());
    }
    return XC_OK;
}

// Split-BF16 mode: Phi stored in FP64 with per-point digit scales, Z in
// FP32, both contractions on BF16 MFMA.
template <bool GGA>
static int launch_wave_bf16(PhaseTimer* timer, hipStream_t s, const WaveBatch* b,
                            const int* gpre, const int* spre, const int* /*wpre*/, int count,
                            int gemm_tiles, int syr_tiles, int /*wide_tiles*/, bool /*wide*/,
                            const ReqDev* reqs, char* scr, int2* tmap, bool colloc, bool sph) {
    if (colloc) {
        PhaseScope ps(timer, s, XC_PHASE_COLLOC);
        hipLaunchKernelGGL((k_colloc<double, true>), dim3(count), dim3(256), 0, s, b, reqs, scr);
        XC_HIP(hipGetLastError());
    }
    if (gemm_tiles > 0) {
        PhaseScope ps(timer, s, XC_PHASE_DENSITY);
        hipLaunchKernelGGL(k_tile_map, dim3(grid_1d(count, 256)), dim3(256), 0, s, gpre, count,
                           tmap);
        XC_HIP(hipGetLastError());
        hipLaunchKernelGGL((k_gemm_rho_bf16<GGA>), dim3(gemm_tiles), dim3(256), 0, s, b,
                           (const int2*)tmap, gemm_tiles, reqs, scr);
        XC_HIP(hipGetLastError());
    }
    {
        PhaseScope ps(timer, s, XC_PHASE_FUNCTIONAL);
        hipLaunchKernelGGL((k_func<GGA>), dim3(count), dim3(256), 0, s, b, reqs, scr);
        XC_HIP(hipGetLastError());
        if (sph) hipLaunchKernelGGL((k_z<float, true>), dim3(count), dim3(256), 0, s, b, reqs, scr);
        else hipLaunchKernelGGL((k_z<float, false>), dim3(count), dim3(256), 0, s, b, reqs, scr);
        XC_HIP(hipGetLastError());
    }
    if (syr_tiles > 0) {
        PhaseScope ps(timer, s, XC_PHASE_POTENTIAL);
        hipLaunchKernelGGL(k_tile_map, dim3(grid_1d(count, 256)), dim3(256), 0, s, spre, count,
                           tmap);
        XC_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_syr2k_bf16, dim3(syr_tiles), dim3(256), 0, s, b,
                           (const int2*)tmap, syr_tiles, reqs, (const char*)scr);
        XC_HIP(hipGetLastError());
    }
    return XC_OK;
}

int launch_wave(PhaseTimer* timer, hipStream_t s, bool gga, int precision,
                const WaveBatch* d_wb, const int* d_gpre, const int* d_spre, const int* d_wpre,
                int count, int gemm_tiles, int syr_tiles, int wide_tiles, bool wide,
                const ReqDev* d_reqs, char* scratch, int* d_tmap_i, bool colloc, bool sph) {
    if (count == 0) return XC_OK;
    int2* t = (int2*)d_tmap_i;
#define XC_WAVE_ARGS timer, s, d_wb, d_gpre, d_spre, d_wpre, count, gemm_tiles, syr_tiles, \
                     wide_tiles, wide, d_reqs, scratch, t, colloc, sph
    if (precision == XC_MIXED_FP32)
        return gga ? launch_wave_t<true, float, float>(XC_WAVE_ARGS)
                   : launch_wave_t<false, float, float>(XC_WAVE_ARGS);
    if (precision == XC_MIXED_BF16)
        return gga ? launch_wave_bf16<true>(XC_WAVE_ARGS) : launch_wave_bf16<false>(XC_WAVE_ARGS);
    if (precision == XC_MIXED_FP32_V)
        return gga ? launch_wave_t<true, double, float>(XC_WAVE_ARGS)
                   : launch_wave_t<false, double, float>(XC_WAVE_ARGS);
    return gga ? launch_wave_t<true, double, double>(XC_WAVE_ARGS)
               : launch_wave_t<false, double, double>(XC_WAVE_ARGS);
#undef XC_WAVE_ARGS
}

// Spin-unrestricted wave (FP64): collocation once, the density contraction
// for each spin (d_wa: alpha batches with request 0, d_wb_b: the same
// batches with the beta partials and request 1), the spin functional, then Z
// and the potential contraction for each spin in turn (the Z slab is reused).
template <bool GGA>
static int launch_wave_uks_t(hipStream_t s, const WaveBatch* wa, const WaveBatch* wbb,
                             const Wave& wv, const int* gpre, const int* wpre, const int* spre,
                             const ReqDev* reqs, char* scr, int2* tmap, bool sph) {
    const int count = wv.count, syr_tiles = wv.syr_tiles;
    hipLaunchKernelGGL((k_colloc<double, false>), dim3(count), dim3(256), 0, s, wa, reqs, scr);
    XC_HIP(hipGetLastError());
    for (const WaveBatch* w : {wa, wbb})
        XC_TRY(launch_density_fp64<GGA>(s, w, gpre, wpre, count, wv.gemm_tiles, wv.wide_tiles,
                                        wv.wide, reqs, scr, tmap));
    hipLaunchKernelGGL((k_func_spin<GGA>), dim3(count), dim3(256), 0, s, wa, reqs, scr);
    XC_HIP(hipGetLastError());
    if (syr_tiles > 0) {
        hipLaunchKernelGGL(k_tile_map, dim3(grid_1d(count, 256)), dim3(256), 0, s, spre, count,
                           tmap);
        XC_HIP(hipGetLastError());
    }
    for (const WaveBatch* w : {wa, wbb}) {
        if (sph) hipLaunchKernelGGL((k_z<double, true>), dim3(count), dim3(256), 0, s, w, reqs, scr);
        else hipLaunchKernelGGL((k_z<double, false>), dim3(count), dim3(256), 0, s, w, reqs, scr);
        XC_HIP(hipGetLastError());
        if (syr_tiles > 0) {
            hipLaunchKernelGGL((k_syr2k<double, double>), dim3(syr_tiles), dim3(256), 0, s, w,
                               (const int2*)tmap, syr_tiles, reqs, (const char*)scr);
            XC_HIP(hipGetLastError());
        }
    }
    return XC_OK;
}

int run_integrate_uks(xc_context* c, int functional, const double* dPa, const double* dPb,
                      double* dVa, double* dVb, double* dEN) {
    const bool gga = functional == XC_GGA_PBE;
    const long long nn = (long long)c->nbf * c->nbf;
    XC_TRY(launch_fill(c->stream, dVa, nn, 0.0));
    XC_TRY(launch_fill(c->stream, dVb, nn, 0.0));
    XC_TRY(dev_reserve(c->d_req, 2 * sizeof(ReqDev)));
    ReqDev* d_req = (ReqDev*)c->d_req.p;
    XC_TRY(launch_put_req(c->stream, d_req, make_req(c, dPa, dVa)));
    XC_TRY(launch_put_req(c->stream, d_req + 1, make_req(c, dPb, dVb)));
    c->phi_cached_kind = 0;
    const WaveBatch* wa = (const WaveBatch*)c->d_wb.p;
    const WaveBatch* wbb = (const WaveBatch*)c->d_wb_beta.p;
    const int* gpre = (const int*)c->d_gemm_pre.p;
    const int* wpre = (const int*)c->d_wide_pre.p;
    const int* spre = (const int*)c->d_syr_pre.p;
    for (const Wave& w : c->waves) {
        if (w.count == 0) continue;
        XC_TRY((gga ? launch_wave_uks_t<true> : launch_wave_uks_t<false>)(
            c->stream, wa + w.wb_off, wbb + w.wb_off, w, gpre + w.pre_off, wpre + w.pre_off,
            spre + w.pre_off, d_req, (char*)c->scratch.p, (int2*)c->d_tmap.p, c->any_pure));
    }
    XC_TRY(launch_finish(nullptr, c->stream, dVb, c->nbf, (const double*)c->epart.p,
                         (const double*)c->npart.p, c->n_batches, dEN));
    return launch_finish(nullptr, c->stream, dVa, c->nbf, (const double*)c->epart.p,
                         (const double*)c->npart.p, c->n_batches, dEN);
}

// Meta-GGA wave (FP64). wb: the batches; wm: three copies of them (d = x,
// y, z), each with gradient slab d in place of Phi and partial set d in
// place of the density partials, n_all batches apart. Collocation and the
// gradient slabs; the density contraction with Phi (rho, grad rho) and with
// each gradient slab (tau); the functional; then Z and the potential
// contraction with Phi, and Z_d = c d phi/dd with the potential contraction
// against gradient slab d, for d = x, y, z (the Z slab is reused).
static int launch_wave_meta(hipStream_t s, const WaveBatch* wb, const WaveBatch* wm,
                            long long n_all, const Wave& wv, const int* gpre, const int* wpre,
                            const int* spre, const ReqDev* reqs, char* scr, int2* tmap,
                            bool sph) {
    const int count = wv.count, syr_tiles = wv.syr_tiles;
    hipLaunchKernelGGL((k_colloc<double, false>), dim3(count), dim3(256), 0, s, wb, reqs, scr);
    XC_HIP(hipGetLastError());
    if (sph) hipLaunchKernelGGL(k_grad<true>, dim3(count), dim3(256), 0, s, wb, reqs, scr);
    else hipLaunchKernelGGL(k_grad<false>, dim3(count), dim3(256), 0, s, wb, reqs, scr);
    XC_HIP(hipGetLastError());
    const WaveBatch* sets[4] = {wb, wm, wm + n_all, wm + 2 * n_all};
    for (const WaveBatch* w : sets)
        XC_TRY(launch_density_fp64<true>(s, w, gpre, wpre, count, wv.gemm_tiles, wv.wide_tiles,
                                         wv.wide, reqs, scr, tmap));
    hipLaunchKernelGGL(k_func_meta, dim3(count), dim3(256), 0, s, wb, reqs, scr);
    XC_HIP(hipGetLastError());
    if (syr_tiles > 0) {
        hipLaunchKernelGGL(k_tile_map, dim3(grid_1d(count, 256)), dim3(256), 0, s, spre, count,
                           tmap);
        XC_HIP(hipGetLastError());
    }
    for (const WaveBatch* w : sets) {
        if (sph) hipLaunchKernelGGL((k_z<double, true>), dim3(count), dim3(256), 0, s, w, reqs, scr);
        else hipLaunchKernelGGL((k_z<double, false>), dim3(count), dim3(256), 0, s, w, reqs, scr);
        XC_HIP(hipGetLastError());
        if (syr_tiles > 0) {
            hipLaunchKernelGGL((k_syr2k<double, double>), dim3(syr_tiles), dim3(256), 0, s, w,
                               (const int2*)tmap, syr_tiles, reqs, (const char*)scr);
            XC_HIP(hipGetLastError());
        }
    }
    return XC_OK;
}

int run_integrate_meta(xc_context* c, const double* dP, double* dV, double* dEN) {
    const long long nn = (long long)c->nbf * c->nbf;
    XC_TRY(launch_fill(c->stream, dV, nn, 0.0));
    XC_TRY(dev_reserve(c->d_req, sizeof(ReqDev)));
    XC_TRY(launch_put_req(c->stream, (ReqDev*)c->d_req.p, make_req(c, dP, dV)));
    c->phi_cached_kind = 0;
    const WaveBatch* wb = (const WaveBatch*)c->d_wb.p;
    const WaveBatch* wm = (const WaveBatch*)c->d_wb_meta.p;
    const long long n_all = (long long)c->h_wb.size();
    const int* gpre = (const int*)c->d_gemm_pre.p;
    const int* wpre = (const int*)c->d_wide_pre.p;
    const int* spre = (const int*)c->d_syr_pre.p;
    for (const Wave& w : c->waves) {
        if (w.count == 0) continue;
        XC_TRY(launch_wave_meta(c->stream, wb + w.wb_off, wm + w.wb_off, n_all, w,
                                gpre + w.pre_off, wpre + w.pre_off, spre + w.pre_off,
                                (const ReqDev*)c->d_req.p, (char*)c->scratch.p,
                                (int2*)c->d_tmap.p, c->any_pure));
    }
    return launch_finish(nullptr, c->stream, dV, c->nbf, (const double*)c->epart.p,
                         (const double*)c->npart.p, c->n_batches, dEN);
}

int phi_kind(int precision) {
    if (precision == XC_MIXED_FP32) return 2;
    if (precision == XC_MIXED_BF16) return 3;
    return 1;
}

int launch_p_digits(hipStream_t s, const double* P, int nbf, unsigned long long* dig,
                    double* scale) {
    if (nbf <= 0) return XC_OK;
    hipLaunchKernelGGL(k_p_digits, dim3(nbf), dim3(256), 0, s, P, nbf, dig, scale);
    XC_HIP(hipGetLastError());
    return XC_OK;
}

int launch_finish(PhaseTimer* timer, hipStream_t s, double* dV, int nbf,
                  const double* epart, const double* npart, long long nbatch,
                  double* dEN) {
    PhaseScope ps(timer, s, XC_PHASE_OTHER);
    const unsigned nt = (unsigned)((nbf + 15) / 16);
    hipLaunchKernelGGL(k_mirror, dim3(nt, nt), dim3(256), 0, s, dV, nbf);
    XC_HIP(hipGetLastError());
    if (nbatch > 0)
        hipLaunchKernelGGL(k_reduce_en, dim3(1), dim3(256), 0, s, epart, npart, nbatch, dEN);
    else
        hipLaunchKernelGGL(k_fill, dim3(1), dim3(64), 0, s, dEN, 2LL, 0.0);
    XC_HIP(hipGetLastError());
    return XC_OK;
}

int launch_put_req(hipStream_t s, ReqDev* dst, const ReqDev& v) {
    hipLaunchKernelGGL(k_put_req, dim3(1), dim3(1), 0, s, dst, v);
    XC_HIP(hipGetLastError());
    return XC_OK;
}

int launch_fill(hipStream_t s, double* p, long long n, double v) {
    if (n <= 0) return XC_OK;
    hipLaunchKernelGGL(k_fill, dim3(grid_1d(n, 256)), dim3(256), 0, s, p, n, v);
    XC_HIP(hipGetLastError());
    return XC_OK;
}

ReqDev make_req(const xc_context* c, const double* dP, double* dV) {
    ReqDev r{};
    r.shells = (const ShellDev*)c->d_shells.p;
    r.palpha = (const double*)c->d_palpha.p;
    r.pcoef = (const double*)c->d_pcoef.p;
    r.shell_list = (const int*)c->shell_list.p;
    r.shell_loff = (const int*)c->shell_loff.p;
    r.func_list = (const int*)c->func_list.p;
    r.px = (const double*)c->px.p;
    r.py = (const double*)c->py.p;
    r.pz = (const double*)c->pz.p;
    r.pw = (const double*)c->pw.p;
    r.P = dP;
    r.V = dV;
    r.epart = (double*)c->epart.p;
    r.npart = (double*)c->npart.p;
    r.func_shell = (const int*)c->d_fshell.p;
    r.Pdig = (const unsigned long long*)c->pdig.p;
    r.Pscale = (const double*)c->pscale.p;
    r.phi_base = nullptr;
    r.rho_thresh = c->rho_thresh;
    r.nbf = c->nbf;
    return r;
}

int run_integrate(xc_context* c, int functional, int precision, const double* dP,
                  double* dV, double* dEN) {
    const bool gga = functional == XC_GGA_PBE;
    const long long nn = (long long)c->nbf * c->nbf;
    {
        PhaseScope ps(c, XC_PHASE_OTHER);
        hipLaunchKernelGGL(k_fill, dim3(grid_1d(nn, 256)), dim3(256), 0, c->stream, dV, nn, 0.0);
        XC_HIP(hipGetLastError());
    }
    if (precision == XC_MIXED_BF16) {
        XC_TRY(dev_reserve(c->pdig, 8 * (size_t)c->nbf * c->nbf));
        XC_TRY(dev_reserve(c->pscale, 8 * (size_t)c->nbf));
        XC_TRY(launch_p_digits(c->stream, dP, c->nbf, (unsigned long long*)c->pdig.p,
                               (double*)c->pscale.p));
    }
    XC_TRY(dev_reserve(c->d_req, sizeof(ReqDev)));
    XC_TRY(launch_put_req(c->stream, (ReqDev*)c->d_req.p, make_req(c, dP, dV)));
    const WaveBatch* wb = (const WaveBatch*)c->d_wb.p;
    const int* gpre = (const int*)c->d_gemm_pre.p;
    const int* spre = (const int*)c->d_syr_pre.p;
    const int* wpre = (const int*)c->d_wide_pre.p;
    // With one wave the scratch still holds the previous integration's Phi
    // (no later kernel writes its slab), so a cached Phi of the same storage
    // type is used as it stands.
    const int kind = phi_kind(precision);
    const bool cacheable = c->phi_cache && !c->external_scratch && c->waves.size() == 1;
    const bool colloc = !(cacheable && c->phi_cached_kind == kind);
    c->phi_cached_kind = 0;
    for (const Wave& w : c->waves)
        XC_TRY(launch_wave(&c->timer, c->stream, gga, precision, wb + w.wb_off,
                           gpre + w.pre_off, spre + w.pre_off, wpre + w.pre_off, w.count,
                           w.gemm_tiles, w.syr_tiles, w.wide_tiles, w.wide,
                           (const ReqDev*)c->d_req.p, (char*)c->scratch.p, (int*)c->d_tmap.p,
                           colloc, c->any_pure));
    if (cacheable) c->phi_cached_kind = kind;
    return launch_finish(&c->timer, c->stream, dV, c->nbf, (const double*)c->epart.p,
                         (const double*)c->npart.p, c->n_batches, dEN);
}

}  // namespace xc
