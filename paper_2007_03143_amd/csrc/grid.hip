// Grid construction on the device: shell cutoff radii (eq. rcut), the
// Mura-Knowles x Lebedev product grid of every parent atom (Sec. 2.2,
// eq. num_int), Stratmann-Scuseria-Frisch partition weights (eq.
// atomic_partition), and stable removal of zero-weight points.
#include <cmath>

#include "device_util.hpp"
#include "xc_internal.hpp"

namespace xc {

// ---------------------------------------------------------------- rcut ----
// r_cut = max over primitives of sqrt((ln(alpha)/2 - ln(eta)) / alpha);
// eta <= 0 disables truncation (rcut2 = +inf).
__global__ void k_shell_rcut(ShellDev* sh, int nshells, const double* alpha,
                             double eta) {
    int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nshells) return;
    ShellDev d = sh[s];
    if (!(eta > 0.0)) {
        sh[s].rcut2 = INFINITY;
        return;
    }
    const double leta = log(eta);
    double rc = 0.0;
    for (int p = 0; p < d.nprim; ++p) {
        const double a = alpha[d.prim_off + p];
        double arg = (0.5 * log(a) - leta) / a;
        rc = fmax(rc, sqrt(fmax(arg, 0.0)));
    }
    sh[s].rcut2 = rc * rc;
}

// inverse inter-atomic distances and the nearest-neighbour shortcut radius
// (1 - a)/2 * min_B R_AB of every atom
__global__ void k_atom_pairs(const double4* atoms, int natoms, double a,
                             double* invR, double* nnhalf) {
    int A = blockIdx.x * blockDim.x + threadIdx.x;
    if (A >= natoms) return;
    const double4 ra = atoms[A];
    double rmin = INFINITY;
    for (int B = 0; B < natoms; ++B) {
        if (B == A) {
            invR[(size_t)A * natoms + B] = 0.0;
            continue;
        }
        const double4 rb = atoms[B];
        const double dx = ra.x - rb.x, dy = ra.y - rb.y, dz = ra.z - rb.z;
        const double R = sqrt(dx * dx + dy * dy + dz * dz);
        invR[(size_t)A * natoms + B] = 1.0 / R;
        rmin = fmin(rmin, R);
    }
    nnhalf[A] = 0.5 * (1.0 - a) * rmin;
}

// For every atom C, all atoms ordered by distance R_CB (C itself first, with
// R = 0): a rank sort, one workgroup per atom.
__global__ void k_atom_neighbours(const double4* atoms, int natoms, int* nbr_idx,
                                  double* nbr_R) {
    extern __shared__ double row[];
    const int C = blockIdx.x;
    const double4 rc = atoms[C];
    for (int j = threadIdx.x; j < natoms; j += blockDim.x) {
        const double4 rb = atoms[j];
        const double dx = rc.x - rb.x, dy = rc.y - rb.y, dz = rc.z - rb.z;
        row[j] = (j == C) ? 0.0 : sqrt(dx * dx + dy * dy + dz * dz);
    }
    __syncthreads();
    for (int j = threadIdx.x; j < natoms; j += blockDim.x) {
        const double r = row[j];
        int rank = 0;
        for (int k = 0; k < natoms; ++k) {
            const double q = row[k];
            rank += (q < r) || (q == r && k < j);
        }
        nbr_idx[(size_t)C * natoms + rank] = j;
        nbr_R[(size_t)C * natoms + rank] = r;
    }
}

// Becke's size adjustment a_AB from the atomic radii (one thread per pair):
// chi = R_A / R_B, u = (chi - 1)/(chi + 1), a = u / (u^2 - 1), clipped to
// [-1/2, 1/2]; zero on the diagonal and without radii.
__global__ void k_becke_adjust(const double* radius, int natoms, double* adj) {
    const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (long long)natoms * natoms) return;
    const int A = (int)(k / natoms), B = (int)(k - (long long)A * natoms);
    double a = 0.0;
    if (radius && A != B) {
        const double chi = radius[A] / radius[B];
        const double u = (chi - 1.0) / (chi + 1.0);
        a = fmin(fmax(u / (u * u - 1.0), -0.5), 0.5);
    }
    adj[k] = a;
}

int launch_shell_setup(xc_context* c) {
    hipLaunchKernelGGL(k_shell_rcut, dim3(grid_1d(c->nshells, 128)), dim3(128), 0,
                       c->stream, (ShellDev*)c->d_shells.p, c->nshells,
                       (const double*)c->d_palpha.p, c->screen_eta);
    XC_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_atom_pairs, dim3(grid_1d(c->natoms, 128)), dim3(128), 0,
                       c->stream, (const double4*)c->d_atoms.p, c->natoms, c->ssf_a,
                       (double*)c->d_invR.p, (double*)c->d_nnhalf.p);
    XC_HIP(hipGetLastError());
    if (c->partition == XC_PARTITION_BECKE) {
        const double* rad = nullptr;
        DevBuf tmp;
        if (!c->becke_radius.empty()) {
            XC_TRY(upload(tmp, c->becke_radius.data(), 8 * c->becke_radius.size(), c->stream));
            rad = (const double*)tmp.p;
        }
        const long long np = (long long)c->natoms * c->natoms;
        hipLaunchKernelGGL(k_becke_adjust, dim3(grid_1d(np, 256)), dim3(256), 0, c->stream,
                           rad, c->natoms, (double*)c->d_becke_a.p);
        XC_HIP(hipGetLastError());
        if (tmp.p) {
            XC_HIP(hipStreamSynchronize(c->stream));
            dev_release(tmp);
        }
    }
    if (c->natoms > kSsfWaveMaxAtoms && c->natoms <= kNbrMaxAtoms) {
        hipLaunchKernelGGL(k_atom_neighbours, dim3(c->natoms), dim3(256),
                           sizeof(double) * (size_t)c->natoms, c->stream,
                           (const double4*)c->d_atoms.p, c->natoms, (int*)c->d_nbr_idx.p,
                           (double*)c->d_nbr_R.p);
        XC_HIP(hipGetLastError());
    }
    return XC_OK;
}

// ---------------------------------------------------------- grid points ---
// Point i of masked atom g: radial index k (outer), angular index l (inner).
// r_k = -alpha ln(1 - x_k^3), x_k = (k + 1/2)/n_rad, weight
// (3 alpha x_k^2 / (1 - x_k^3)) / n_rad * r_k^2 * w_l.
__global__ void k_grid_points(long long n, int npa, int n_rad, int n_ang,
                              const int* gatoms, const double4* atoms,
                              const double4* ang, double* X, double* Y,
                              double* Z, double* W) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int g = (int)(i / npa);
    const int rem = (int)(i - (long long)g * npa);
    const int k = rem / n_ang, l = rem - k * n_ang;
    const double4 at = atoms[gatoms[g]];
    const double alpha = at.w;
    const double xk = (k + 0.5) / n_rad;
    const double om = 1.0 - xk * xk * xk;
    const double r = -alpha * log(om);
    const double wr = (3.0 * alpha * xk * xk / om) / n_rad * r * r;
    const double4 s = ang[l];
    X[i] = at.x + r * s.x;
    Y[i] = at.y + r * s.y;
    Z[i] = at.z + r * s.z;
    W[i] = wr * s.w;
}

int launch_grid_points(xc_context* c) {
    PhaseScope ps(c, XC_PHASE_GRID);
    const int npa = c->n_rad * c->n_ang;
    hipLaunchKernelGGL(k_grid_points, dim3(grid_1d(c->n_nominal, 256)), dim3(256), 0,
                       c->stream, c->n_nominal, npa, c->n_rad, c->n_ang,
                       (const int*)c->d_gatoms.p, (const double4*)c->d_atoms.p,
                       (const double4*)c->d_ang.p, (double*)c->raw_x.p,
                       (double*)c->raw_y.p, (double*)c->raw_z.p, (double*)c->raw_w.p);
    XC_HIP(hipGetLastError());
    return XC_OK;
}

// ------------------------------------------------------------------ SSF ---
// s(mu) = (1 - g(mu))/2 with g the SSF polynomial on |mu| < a, +-1 outside.
__device__ inline double ssf_s(double mu, double a) {
    if (mu <= -a) return 1.0;
    if (mu >= a) return 0.0;
    const double z = mu / a, z2 = z * z;
    const double g = z * (35.0 + z2 * (-35.0 + z2 * (21.0 - 5.0 * z2))) * 0.0625;
    return 0.5 * (1.0 - g);
}

__device__ inline double dist2_to(const double4& at, double x, double y, double z) {
    const double dx = x - at.x, dy = y - at.y, dz = z - at.z;
    return dx * dx + dy * dy + dz * dz;
}

// Unnormalised cell product P_C(r) = prod_{B != C} s(mu_CB); stops at zero.
// Only atoms with R_CB < 2 d_C / (1 - a) can give a factor other than 1
// (otherwise d_B >= R_CB - d_C gives mu_CB <= -a, s = 1 exactly), so the
// loop runs over C's neighbours in order of distance and stops there.
__device__ inline double ssf_product_nbr(int C, double dC, const double4* atoms,
                                         const int* nbr_idx, const double* nbr_R,
                                         int natoms, double x, double y, double z,
                                         double a, double reach) {
    double p = 1.0;
    const int* ni = nbr_idx + (size_t)C * natoms;
    const double* nr = nbr_R + (size_t)C * natoms;
    const double lim = dC * reach;
    for (int t = 1; t < natoms; ++t) {
        const double R = nr[t];
        if (R >= lim) break;
        const int B = ni[t];
        // s(mu_CB) = 1 unless d_B < d_C + a R_CB: test on the squared distance
        const double d2 = dist2_to(atoms[B], x, y, z);
        const double edge = dC + a * R * (1.0 + 1e-12);
        if (d2 >= edge * edge) continue;
        p *= ssf_s((dC - sqrt(d2)) / R, a);
        if (p == 0.0) break;
    }
    return p;
}

// Same product without neighbour lists (very large molecules): atoms B with
// d_B >= d_C (1 + a)/(1 - a) have mu_CB <= -a and are skipped on their
// squared distance.
__device__ inline double ssf_product_all(int C, double dC, const double4* atoms,
                                         const double* invR, int natoms, double x,
                                         double y, double z, double a, double far2) {
    double p = 1.0;
    const double* ir = invR + (size_t)C * natoms;
    const double lim2 = dC * dC * far2;
    for (int B = 0; B < natoms; ++B) {
        if (B == C) continue;
        const double d2 = dist2_to(atoms[B], x, y, z);
        if (d2 >= lim2) continue;
        p *= ssf_s((dC - sqrt(d2)) * ir[B], a);
        if (p == 0.0) break;
    }
    return p;
}

// w_i <- w_i * P_parent / sum_C P_C. Exact reductions of the work:
//  * |r - R_A| < (1-a)/2 min_B R_AB: the parent owns the point (p = 1);
//  * an atom C with (d_C - d_min) / R_{C,nearest} >= a has s(mu_{C,nearest}) = 0,
//    hence P_C = 0, and is skipped;
//  * inside a product only nearby atoms can differ from 1 (see above).
// One lane per point; used for molecules with more atoms than the
// one-wave-per-point kernel below takes, so the atom centres are read from
// global memory.
__global__ __launch_bounds__(256) void k_ssf(long long n, int npa, const int* gatoms,
                                             const double4* atoms_g, const double* invR,
                                             const int* nbr_idx, const double* nbr_R,
                                             const double* nnhalf, int natoms, double a,
                                             const double* X, const double* Y,
                                             const double* Z, double* W) {
    const double4* atoms = atoms_g;
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double w = W[i];
    if (w == 0.0 || natoms == 1) return;
    const int A = gatoms[(int)(i / npa)];
    const double x = X[i], y = Y[i], z = Z[i];
    const double dA = sqrt(dist2_to(atoms[A], x, y, z));
    if (dA < nnhalf[A]) return;
    const double reach = 2.0 / (1.0 - a) * (1.0 + 1e-12);
    const double far = (1.0 + a) / (1.0 - a) * (1.0 + 1e-12);
    const bool use_nbr = nbr_idx != nullptr;
    // the four nearest atoms (squared distances, ascending)
    constexpr int kNear = 4;
    double nd2[kNear];
    int nb[kNear];
#pragma unroll
    for (int k = 0; k < kNear; ++k) {
        nd2[k] = INFINITY;
        nb[k] = -1;
    }
    for (int B = 0; B < natoms; ++B) {
        double d2 = dist2_to(atoms[B], x, y, z);
        int b = B;
#pragma unroll
        for (int k = 0; k < kNear; ++k) {
            if (d2 < nd2[k]) {
                const double td = nd2[k];
                const int tb = nb[k];
                nd2[k] = d2;
                nb[k] = b;
                d2 = td;
                b = tb;
            }
        }
    }
    const int bmin = nb[0];
    const double dmin = sqrt(nd2[0]);
    double nd[kNear];
#pragma unroll
    for (int k = 0; k < kNear; ++k) nd[k] = sqrt(nd2[k]);
    const double PA = use_nbr
        ? ssf_product_nbr(A, dA, atoms, nbr_idx, nbr_R, natoms, x, y, z, a, reach)
        : ssf_product_all(A, dA, atoms, invR, natoms, x, y, z, a, far * far);
    if (PA == 0.0) {
        W[i] = 0.0;
        return;
    }
    // candidates C need d_C < d_min + a R_{C,nearest} <= d_min + a (d_C + d_min)
    const double cand = dmin * far;
    const double cand2 = cand * cand;
    double sum = 0.0;
    for (int C = 0; C < natoms; ++C) {
        if (C == A) {
            sum += PA;
            continue;
        }
        const double dC2 = dist2_to(atoms[C], x, y, z);
        if (C != bmin && dC2 >= cand2) continue;
        const double dC = sqrt(dC2);
        // P_C = 0 if s(mu_CB) = 0 for one of the nearest atoms B
        bool zero = false;
#pragma unroll
        for (int k = 0; k < kNear; ++k)
            if (nb[k] >= 0 && nb[k] != C &&
                (dC - nd[k]) * invR[(size_t)C * natoms + nb[k]] >= a)
                zero = true;
        if (zero) continue;
        sum += use_nbr
            ? ssf_product_nbr(C, dC, atoms, nbr_idx, nbr_R, natoms, x, y, z, a, reach)
            : ssf_product_all(C, dC, atoms, invR, natoms, x, y, z, a, far * far);
    }
    W[i] = w * (PA / sum);
}

// ------------------------------------------- partition, one wave a point --
// For molecules up to kSsfWaveMaxAtoms atoms. The lanes of a wave first test
// one point each (zero weight, shortcut). The wave then takes the remaining
// points one at a time and spreads each cell product over the atoms, lane l
// holding atoms l, l + 64, ...: every lane does the same work whatever the
// point, the rows of 1/R_CB are read coalesced, and the product is finished
// by a butterfly over the wave. The atoms C that can share a point are those
// with d_C < d_min (1 + a)/(1 - a) whose factor against the nearest atom is
// not zero; every other P_C is exactly zero.

// Wave reductions without the LDS unit: DPP moves inside each 16-lane row
// (swap neighbours, swap pairs, mirror the half-rows, mirror the rows), then
// the four row results are read into scalar registers. Every lane ends with
// the same value.
template <int CTRL>
__device__ __forceinline__ int dpp_i32(int v) {
    return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, true);
}
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = dpp_i32<CTRL>((int)b);
    const int hi = dpp_i32<CTRL>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
constexpr int kDppXor1 = 0xB1;        // quad_perm [1, 0, 3, 2]
constexpr int kDppXor2 = 0x4E;        // quad_perm [2, 3, 0, 1]
constexpr int kDppHalfMirror = 0x141; // row_half_mirror
constexpr int kDppMirror = 0x140;     // row_mirror

// s(mu) with z = mu (1/a): a multiplication in place of the division
__device__ inline double ssf_s_inv(double mu, double a, double inv_a) {
    if (mu <= -a) return 1.0;
    if (mu >= a) return 0.0;
    const double z = mu * inv_a, z2 = z * z;
    const double g = z * (35.0 + z2 * (-35.0 + z2 * (21.0 - 5.0 * z2))) * 0.0625;
    return 0.5 * (1.0 - g);
}

__device__ inline double wave_product(double v) {
    v *= dpp_f64<kDppXor1>(v);
    v *= dpp_f64<kDppXor2>(v);
    v *= dpp_f64<kDppHalfMirror>(v);
    v *= dpp_f64<kDppMirror>(v);
    return (readlane_f64(v, 0) * readlane_f64(v, 16)) *
           (readlane_f64(v, 32) * readlane_f64(v, 48));
}

__device__ inline void argmin_take(double& d, int& b, double od, int ob) {
    if (od < d || (od == d && ob < b)) {
        d = od;
        b = ob;
    }
}

// smallest d over the wave, ties to the smaller index b
__device__ inline void wave_argmin(double& d, int& b) {
    argmin_take(d, b, dpp_f64<kDppXor1>(d), dpp_i32<kDppXor1>(b));
    argmin_take(d, b, dpp_f64<kDppXor2>(d), dpp_i32<kDppXor2>(b));
    argmin_take(d, b, dpp_f64<kDppHalfMirror>(d), dpp_i32<kDppHalfMirror>(b));
    argmin_take(d, b, dpp_f64<kDppMirror>(d), dpp_i32<kDppMirror>(b));
    double rd = readlane_f64(d, 0);
    int rb = __builtin_amdgcn_readlane(b, 0);
#pragma unroll
    for (int r = 16; r < 64; r += 16)
        argmin_take(rd, rb, readlane_f64(d, r), __builtin_amdgcn_readlane(b, r));
    d = rd;
    b = rb;
}

template <int NPER>
__global__ __launch_bounds__(256) void k_ssf_wave(long long n, int npa, const int* gatoms,
                                                  const double4* atoms_g, const double* invR,
                                                  const double* nnhalf, int natoms, double a,
                                                  const double* X, const double* Y,
                                                  const double* Z, double* W) {
    extern __shared__ double4 sat[];
    for (int k = threadIdx.x; k < natoms; k += blockDim.x) sat[k] = atoms_g[k];
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    double x = 0.0, y = 0.0, z = 0.0, w = 0.0;
    int A = 0;
    bool need = false;
    if (i < n && natoms > 1) {
        w = W[i];
        if (w != 0.0) {
            A = gatoms[(int)(i / npa)];
            x = X[i];
            y = Y[i];
            z = Z[i];
            need = !(sqrt(dist2_to(sat[A], x, y, z)) < nnhalf[A]);
        }
    }
    const double far = (1.0 + a) / (1.0 - a) * (1.0 + 1e-12);
    const double inv_a = 1.0 / a;
    unsigned long long todo = __ballot(need);
    while (todo) {
        const int l = __ffsll((unsigned long long)todo) - 1;
        todo &= todo - 1;
        const double px = readlane_f64(x, l), py = readlane_f64(y, l), pz = readlane_f64(z, l);
        const int pA = __builtin_amdgcn_readlane(A, l);
        // this lane's atoms: distances, and the nearest atom over the wave
        double d[NPER];
        double dmin = INFINITY;
        int bmin = natoms;
#pragma unroll
        for (int j = 0; j < NPER; ++j) {
            const int B = lane + 64 * j;
            d[j] = B < natoms ? sqrt(dist2_to(sat[B], px, py, pz)) : INFINITY;
            if (d[j] < dmin) {
                dmin = d[j];
                bmin = B;
            }
        }
        wave_argmin(dmin, bmin);
        // P_C = prod_{B != C} s(mu_CB), spread over the lanes. If any
        // mu_CB >= a the product is exactly zero: a wave vote skips the
        // polynomials and the reduction (about half the candidates).
        auto cell = [&](int C) {
            const double dC = sqrt(dist2_to(sat[C], px, py, pz));
            const double* ir = invR + (size_t)C * natoms;
            double mu[NPER];
            bool zero = false;
#pragma unroll
            for (int j = 0; j < NPER; ++j) {
                const int B = lane + 64 * j;
                const bool use = B < natoms && B != C;
                // s(-a) = 1 exactly stands in for the absent factors
                mu[j] = use ? (dC - d[j]) * ir[use ? B : 0] : -a;
                zero = zero || mu[j] >= a;
            }
            if (__any(zero)) return 0.0;
            double p = 1.0;
#pragma unroll
            for (int j = 0; j < NPER; ++j) p *= ssf_s_inv(mu[j], a, inv_a);
            return wave_product(p);
        };
        const double PA = cell(pA);
        double frac = 0.0;
        if (PA != 0.0) {
            double sum = PA;
            const double cand = dmin * far;
#pragma unroll
            for (int j = 0; j < NPER; ++j) {
                const int C = lane + 64 * j;
                bool c = C < natoms && C != pA && (C == bmin || d[j] < cand);
                if (c && C != bmin && bmin < natoms)
                    c = (d[j] - dmin) * invR[(size_t)C * natoms + bmin] < a;
                unsigned long long cm = __ballot(c);
                while (cm) {
                    const int lc = __ffsll((unsigned long long)cm) - 1;
                    cm &= cm - 1;
                    sum += cell(lc + 64 * j);
                }
            }
            frac = PA / sum;
        }
        if (lane == l) W[i] = w * frac;
    }
}

// ------------------------------------------ Becke partition, one wave a point --
// Becke's cell function is s(nu) = (1 - p(p(p(nu))))/2, p(x) = 3x/2 - x^3/2;
// p is odd, so s(-nu) = 1 - s(nu) = (1 + p(p(p(nu))))/2.
__device__ inline double wave_sum(double v) {
    v += dpp_f64<kDppXor1>(v);
    v += dpp_f64<kDppXor2>(v);
    v += dpp_f64<kDppHalfMirror>(v);
    v += dpp_f64<kDppMirror>(v);
    return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}

// Weights with Becke's partition (molecules up to kSsfWaveMaxAtoms atoms).
// No factor is exactly 0 or 1 away from the nuclei, so every point needs
// every atom's cell product. The wave takes the points of its lanes PTS at
// a time (4 up to 256 atoms, 2 up to 512, then 1: the registers they take); lane l holds atoms B = l, l + 64, ... with their distances to each
// of those points and accumulates their own products P_B = prod_{C != B}
// s(nu_BC) while the wave steps through C, using s(nu_BC) = s(-nu_CB) =
// (1 + p(p(p(nu_CB))))/2 (mu and the size adjustment are antisymmetric), so
// that every lane reads row C of the pair tables at its own column B
// (consecutive across the lanes), once for the PTS points, and no
// cross-lane product is needed; the wave sums the P_B of each point at the
// end. d_C of a point is read from the lane that holds atom C. Points of
// zero weight are skipped.
template <int NPER>
__global__ __launch_bounds__(256) void k_becke_wave(long long n, int npa, const int* gatoms,
                                                    const double4* atoms_g,
                                                    const double* invR, const double* adj,
                                                    int natoms, const double* X,
                                                    const double* Y, const double* Z,
                                                    double* W) {
    constexpr int PTS = NPER <= 4 ? 4 : NPER <= 8 ? 2 : 1;
    extern __shared__ double4 sat[];
    for (int k = threadIdx.x; k < natoms; k += blockDim.x) sat[k] = atoms_g[k];
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    double x = 0.0, y = 0.0, z = 0.0, w = 0.0;
    int A = 0;
    bool need = false;
    if (i < n && natoms > 1) {
        w = W[i];
        if (w != 0.0) {
            A = gatoms[(int)(i / npa)];
            x = X[i];
            y = Y[i];
            z = Z[i];
            need = true;
        }
    }
    unsigned long long todo = __ballot(need);
    while (todo) {
        // up to PTS points of the wave's lanes (slots past the last repeat it)
        int ln[PTS];
#pragma unroll
        for (int p = 0; p < PTS; ++p) {
            ln[p] = __ffsll((unsigned long long)todo) - 1;
            if (todo & (todo - 1)) todo &= todo - 1;
            else if (p + 1 < PTS) {
#pragma unroll
                for (int r = p + 1; r < PTS; ++r) ln[r] = ln[p];
                todo = 0;
                break;
            } else {
                todo = 0;
            }
        }
        double d[PTS][NPER], q[PTS][NPER];
#pragma unroll
        for (int p = 0; p < PTS; ++p) {
            const double px = readlane_f64(x, ln[p]), py = readlane_f64(y, ln[p]),
                         pz = readlane_f64(z, ln[p]);
#pragma unroll
            for (int j = 0; j < NPER; ++j) {
                const int B = lane + 64 * j;
                d[p][j] = B < natoms ? sqrt(dist2_to(sat[B], px, py, pz)) : 0.0;
                q[p][j] = 1.0;
            }
        }
        for (int C = 0; C < natoms; ++C) {
            const int jc = C >> 6, lc = C & 63;
            double dC[PTS];
#pragma unroll
            for (int p = 0; p < PTS; ++p) {
                double v = 0.0;
#pragma unroll
                for (int j = 0; j < NPER; ++j)
                    if (j == jc) v = d[p][j];
                dC[p] = readlane_f64(v, lc);
            }
            const double* ir = invR + (size_t)C * natoms;
            const double* ar = adj + (size_t)C * natoms;
#pragma unroll
            for (int j = 0; j < NPER; ++j) {
                const int B = lane + 64 * j;
                if (B < natoms && B != C) {
                    const double irb = ir[B], arb = ar[B];
#pragma unroll
                    for (int p = 0; p < PTS; ++p) {
                        const double mu = (dC[p] - d[p][j]) * irb;
                        double f = mu + arb * (1.0 - mu * mu);
#pragma unroll
                        for (int k = 0; k < 3; ++k) f = f * (1.5 - 0.5 * f * f);
                        q[p][j] *= 0.5 * (1.0 + f);
                    }
                }
            }
        }
#pragma unroll
        for (int p = 0; p < PTS; ++p) {
            const int pA = __builtin_amdgcn_readlane(A, ln[p]);
            double qs = 0.0, qa = 0.0;
#pragma unroll
            for (int j = 0; j < NPER; ++j) {
                if (lane + 64 * j < natoms) qs += q[p][j];
                if (j == (pA >> 6)) qa = q[p][j];
            }
            const double sum = wave_sum(qs);
            const double PA = readlane_f64(qa, pA & 63);
            if (lane == ln[p]) W[i] = w * (PA / sum);
        }
    }
}

int launch_ssf(xc_context* c) {
    PhaseScope ps(c, XC_PHASE_WEIGHTS);
    const int npa = c->n_rad * c->n_ang;
    if (c->partition == XC_PARTITION_BECKE) {
        const int nper = (c->natoms + 63) / 64;
        auto k = nper <= 1 ? k_becke_wave<1> : nper <= 2 ? k_becke_wave<2>
               : nper <= 4 ? k_becke_wave<4> : nper <= 8 ? k_becke_wave<8> : k_becke_wave<16>;
        hipLaunchKernelGGL(k, dim3(grid_1d(c->n_nominal, 256)), dim3(256),
                           sizeof(double4) * (size_t)c->natoms, c->stream, c->n_nominal, npa,
                           (const int*)c->d_gatoms.p, (const double4*)c->d_atoms.p,
                           (const double*)c->d_invR.p, (const double*)c->d_becke_a.p,
                           c->natoms, (const double*)c->raw_x.p, (const double*)c->raw_y.p,
                           (const double*)c->raw_z.p, (double*)c->raw_w.p);
        XC_HIP(hipGetLastError());
        return XC_OK;
    }
    if (c->natoms <= kSsfWaveMaxAtoms) {
        const int nper = (c->natoms + 63) / 64;
        // atom slots per lane: the fewest instantiated that cover the atoms
        // (a slot past the last atom still costs its share of the work)
        auto k = nper <= 1 ? k_ssf_wave<1> : nper <= 2 ? k_ssf_wave<2>
               : nper <= 4 ? k_ssf_wave<4> : nper <= 6 ? k_ssf_wave<6>
               : nper <= 8 ? k_ssf_wave<8> : nper <= 10 ? k_ssf_wave<10>
               : nper <= 12 ? k_ssf_wave<12> : k_ssf_wave<16>;
        hipLaunchKernelGGL(k, dim3(grid_1d(c->n_nominal, 256)), dim3(256),
                           sizeof(double4) * (size_t)c->natoms, c->stream, c->n_nominal, npa,
                           (const int*)c->d_gatoms.p, (const double4*)c->d_atoms.p,
                           (const double*)c->d_invR.p, (const double*)c->d_nnhalf.p,
                           c->natoms, c->ssf_a, (const double*)c->raw_x.p,
                           (const double*)c->raw_y.p, (const double*)c->raw_z.p,
                           (double*)c->raw_w.p);
        XC_HIP(hipGetLastError());
        return XC_OK;
    }
    hipLaunchKernelGGL(k_ssf, dim3(grid_1d(c->n_nominal, 256)), dim3(256), 0, c->stream,
                       c->n_nominal, npa, (const int*)c->d_gatoms.p,
                       (const double4*)c->d_atoms.p, (const double*)c->d_invR.p,
                       c->natoms <= kNbrMaxAtoms ? (const int*)c->d_nbr_idx.p : nullptr,
                       (const double*)c->d_nbr_R.p, (const double*)c->d_nnhalf.p,
                       c->natoms, c->ssf_a,
                       (const double*)c->raw_x.p, (const double*)c->raw_y.p,
                       (const double*)c->raw_z.p, (double*)c->raw_w.p);
    XC_HIP(hipGetLastError());
    return XC_OK;
}

// ------------------------------------------------------------ compaction --
// Blocks of kCompactSpan points, aligned to each atom's segment, count their
// non-zero weights; a second pass writes the kept points in order.
constexpr int kCompactSpan = 1024;

__global__ void k_compact_count(const double* W, int npa, int nblk_atom, int* count) {
    const int g = blockIdx.x / nblk_atom, kb = blockIdx.x - g * nblk_atom;
    const long long base = (long long)g * npa + (long long)kb * kCompactSpan;
    const int len = min(kCompactSpan, npa - kb * kCompactSpan);
    int c = 0;
    for (int j = threadIdx.x; j < len; j += blockDim.x) c += (W[base + j] != 0.0);
    __shared__ int red[256];
    red[threadIdx.x] = c;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) count[blockIdx.x] = red[0];
}

__global__ void k_compact_write(const double* X, const double* Y, const double* Z,
                                const double* W, int npa, int nblk_atom,
                                const long long* off, double* ox, double* oy,
                                double* oz, double* ow, long long* oidx) {
    const int g = blockIdx.x / nblk_atom, kb = blockIdx.x - g * nblk_atom;
    const long long base = (long long)g * npa + (long long)kb * kCompactSpan;
    const int len = min(kCompactSpan, npa - kb * kCompactSpan);
    // 256 threads x 4 consecutive points each
    const int j0 = threadIdx.x * 4;
    int keep[4];
    int c = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int j = j0 + q;
        keep[q] = (j < len) && (W[base + j] != 0.0);
        c += keep[q];
    }
    __shared__ int smem[17];
    int total;
    int pos = block_exclusive_scan(c, smem, total);
    long long dst = off[blockIdx.x] + pos;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (!keep[q]) continue;
        const long long s = base + j0 + q;
        ox[dst] = X[s];
        oy[dst] = Y[s];
        oz[dst] = Z[s];
        ow[dst] = W[s];
        oidx[dst] = s;
        ++dst;
    }
}

int launch_compact(xc_context* c, std::vector<long long>& atom_kept) {
    PhaseScope ps(c, XC_PHASE_COMPACT);
    const int npa = c->n_rad * c->n_ang;
    const int nblk_atom = (npa + kCompactSpan - 1) / kCompactSpan;
    const int nga = (int)c->gatoms.size();
    const int nblk = nga * nblk_atom;
    XC_TRY(dev_reserve(c->blk_count, sizeof(int) * (size_t)nblk));
    XC_TRY(dev_reserve(c->blk_off, sizeof(long long) * (size_t)nblk));
    hipLaunchKernelGGL(k_compact_count, dim3(nblk), dim3(256), 0, c->stream,
                       (const double*)c->raw_w.p, npa, nblk_atom, (int*)c->blk_count.p);
    XC_HIP(hipGetLastError());
    std::vector<int> cnt(nblk);
    XC_HIP(hipMemcpyAsync(cnt.data(), c->blk_count.p, sizeof(int) * (size_t)nblk,
                          hipMemcpyDeviceToHost, c->stream));
    XC_HIP(hipStreamSynchronize(c->stream));
    std::vector<long long> off(nblk);
    atom_kept.assign(nga, 0);
    long long run = 0;
    for (int b = 0; b < nblk; ++b) {
        off[b] = run;
        run += cnt[b];
        atom_kept[b / nblk_atom] += cnt[b];
    }
    c->n_points = run;
    XC_TRY(upload(c->blk_off, off.data(), sizeof(long long) * (size_t)nblk, c->stream));
    const size_t np = (size_t)(run > 0 ? run : 1);
    XC_TRY(dev_reserve(c->px, 8 * np));
    XC_TRY(dev_reserve(c->py, 8 * np));
    XC_TRY(dev_reserve(c->pz, 8 * np));
    XC_TRY(dev_reserve(c->pw, 8 * np));
    XC_TRY(dev_reserve(c->pidx, 8 * np));
    XC_TRY(dev_reserve(c->tx, 8 * np));
    XC_TRY(dev_reserve(c->ty, 8 * np));
    XC_TRY(dev_reserve(c->tz, 8 * np));
    XC_TRY(dev_reserve(c->tw, 8 * np));
    XC_TRY(dev_reserve(c->tidx, 8 * np));
    hipLaunchKernelGGL(k_compact_write, dim3(nblk), dim3(256), 0, c->stream,
                       (const double*)c->raw_x.p, (const double*)c->raw_y.p,
                       (const double*)c->raw_z.p, (const double*)c->raw_w.p, npa,
                       nblk_atom, (const long long*)c->blk_off.p, (double*)c->px.p,
                       (double*)c->py.p, (double*)c->pz.p, (double*)c->pw.p,
                       (long long*)c->pidx.p);
    XC_HIP(hipGetLastError());
    return XC_OK;
}

}  // namespace xc
