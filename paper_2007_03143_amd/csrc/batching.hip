// Spatial batching of the grid and per-batch shell screening, on the device.
//
// Batching (Sec. 2.2, Fig. 1 of the paper): each atom's points form a cuboid
// (their bounding box) that is split recursively until no cell holds more
// than batch_max points; a cell whose closed bounding box contains an atomic
// centre is split into 27 equal cuboids, any other cell into 8 octants.
// Points of a cell stay contiguous; one workgroup reorders one cell with a
// stable counting sort, so the batches are the same on every run.
//
// Screening (Sec. 2.2 Alg. 1, Alg. 3): a shell is kept for a batch when its
// cutoff sphere meets the batch's bounding box (closed-ball test d >= 0).
#include <algorithm>
#include <cmath>

#include "device_util.hpp"
#include "xc_internal.hpp"

namespace xc {

constexpr int kMaxChild = 27;

// tight bounding box of every cell's points
__global__ void k_cell_bbox(Cell* cells, const double* X, const double* Y,
                            const double* Z) {
    Cell c = cells[blockIdx.x];
    double lo[3] = {INFINITY, INFINITY, INFINITY};
    double hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int j = threadIdx.x; j < c.count; j += blockDim.x) {
        const long long p = c.begin + j;
        const double v[3] = {X[p], Y[p], Z[p]};
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            lo[q] = fmin(lo[q], v[q]);
            hi[q] = fmax(hi[q], v[q]);
        }
    }
    __shared__ double red[6][256];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        red[q][threadIdx.x] = lo[q];
        red[3 + q][threadIdx.x] = hi[q];
    }
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                red[q][threadIdx.x] = fmin(red[q][threadIdx.x], red[q][threadIdx.x + s]);
                red[3 + q][threadIdx.x] =
                    fmax(red[3 + q][threadIdx.x], red[3 + q][threadIdx.x + s]);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            cells[blockIdx.x].lo[q] = red[q][0];
            cells[blockIdx.x].hi[q] = red[3 + q][0];
        }
    }
}

__device__ inline int cell_coord(double v, double lo, double ext, int ns) {
    if (!(ext > 0.0)) return 0;
    int t = (int)((v - lo) * ns / ext);
    return t < 0 ? 0 : (t >= ns ? ns - 1 : t);
}

// One workgroup (kSplitThreads threads) splits one cell into its 27 or 8
// children, stably (points keep their order within each child). The cell's
// points are taken in rounds of kSplitThreads consecutive points, one per
// thread, so every load is coalesced. A first pass counts the children with
// LDS atomics; the second gives each point its rank among the round's points
// of the same child (ballots within the wave, a prefix over the waves) and
// writes it to its child's range of the scratch arrays, which are then
// copied back.
constexpr int kSplitThreads = 1024;
constexpr int kSplitWaves = kSplitThreads / 64;

__global__ __launch_bounds__(kSplitThreads) void k_split(
    const Cell* cells, const double4* atoms, int natoms, double* X, double* Y,
    double* Z, double* W, long long* I, double* TX, double* TY, double* TZ,
    double* TW, long long* TI, int* child_count, long long* child_begin) {
    const Cell c = cells[blockIdx.x];
    __shared__ int wcnt[kSplitWaves][kMaxChild];
    __shared__ int tot[kMaxChild], base[kMaxChild], run[kMaxChild];
    __shared__ int has_centre;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    if (tid == 0) has_centre = 0;
    if (tid < kMaxChild) {
        tot[tid] = 0;
        run[tid] = 0;
    }
    __syncthreads();
    for (int a = tid; a < natoms; a += blockDim.x) {
        const double4 r = atoms[a];
        if (r.x >= c.lo[0] && r.x <= c.hi[0] && r.y >= c.lo[1] && r.y <= c.hi[1] &&
            r.z >= c.lo[2] && r.z <= c.hi[2])
            has_centre = 1;
    }
    __syncthreads();
    const int ns = has_centre ? 3 : 2;
    const int nchild = ns * ns * ns;
    const double ex = c.hi[0] - c.lo[0], ey = c.hi[1] - c.lo[1], ez = c.hi[2] - c.lo[2];
    const int n = c.count;
    auto child = [&](double x, double y, double z) {
        return (cell_coord(x, c.lo[0], ex, ns) * ns + cell_coord(y, c.lo[1], ey, ns)) * ns +
               cell_coord(z, c.lo[2], ez, ns);
    };
    for (int j = tid; j < n; j += kSplitThreads) {
        const long long p = c.begin + j;
        atomicAdd(&tot[child(X[p], Y[p], Z[p])], 1);
    }
    __syncthreads();
    if (tid == 0) {
        int b = 0;
        for (int k = 0; k < nchild; ++k) {
            base[k] = b;
            b += tot[k];
        }
    }
    __syncthreads();
    const unsigned long long below = (1ull << lane) - 1ull;
    for (int r0 = 0; r0 < n; r0 += kSplitThreads) {
        const int j = r0 + tid;
        const bool v = j < n;
        const long long p = c.begin + j;
        double x = 0.0, y = 0.0, z = 0.0;
        int k = -1;
        if (v) {
            x = X[p];
            y = Y[p];
            z = Z[p];
            k = child(x, y, z);
        }
        int rank = 0;
        for (int kk = 0; kk < nchild; ++kk) {
            const unsigned long long m = __ballot(k == kk);
            if (k == kk) rank = __popcll(m & below);
            if (lane == 0) wcnt[wv][kk] = __popcll(m);
        }
        __syncthreads();
        if (tid < nchild) {
            int s = run[tid];
            for (int w = 0; w < kSplitWaves; ++w) {
                const int t = wcnt[w][tid];
                wcnt[w][tid] = s;
                s += t;
            }
            run[tid] = s;
        }
        __syncthreads();
        if (v) {
            const long long d = c.begin + base[k] + wcnt[wv][k] + rank;
            TX[d] = x;
            TY[d] = y;
            TZ[d] = z;
            TW[d] = W[p];
            TI[d] = I[p];
        }
        __syncthreads();
    }
    for (int j = tid; j < n; j += blockDim.x) {
        const long long p = c.begin + j;
        X[p] = TX[p];
        Y[p] = TY[p];
        Z[p] = TZ[p];
        W[p] = TW[p];
        I[p] = TI[p];
    }
    if (tid < kMaxChild) {
        child_count[(size_t)blockIdx.x * kMaxChild + tid] = (tid < nchild) ? tot[tid] : 0;
        child_begin[(size_t)blockIdx.x * kMaxChild + tid] =
            c.begin + ((tid < nchild) ? base[tid] : 0);
    }
}

// Single workgroup: walk every parent's children in order and append the
// non-empty ones either to the finished batches (count <= batch_max) or to
// the next level. With merge on, runs of consecutive small children of one
// parent (their points are contiguous) are joined while the joined count
// stays <= batch_max. counters[0] = batches written, counters[1] = next-level
// cells written.
__device__ inline int classify_parent(const int* cnt, const long long* beg,
                                      int batch_max, int merge, int atom,
                                      Cell* ob, Cell* on, bool write) {
    int nb = 0, nn = 0;
    long long gb = 0;
    int gc = 0;
    auto emit = [&](Cell* dst, int idx, long long b, int n) {
        if (!write) return;
        Cell o;
        o.begin = b;
        o.count = n;
        o.atom = atom;
        for (int q = 0; q < 3; ++q) {
            o.lo[q] = 0.0;
            o.hi[q] = 0.0;
        }
        dst[idx] = o;
    };
    for (int k = 0; k < kMaxChild; ++k) {
        const int n = cnt[k];
        if (n == 0) continue;
        if (n > batch_max) {
            if (gc > 0) emit(ob, nb++, gb, gc);
            gc = 0;
            emit(on, nn++, beg[k], n);
        } else if (!merge) {
            emit(ob, nb++, beg[k], n);
        } else {
            if (gc > 0 && gc + n > batch_max) {
                emit(ob, nb++, gb, gc);
                gc = 0;
            }
            if (gc == 0) gb = beg[k];
            gc += n;
        }
    }
    if (gc > 0) emit(ob, nb++, gb, gc);
    return (nb << 16) | nn;
}

__global__ __launch_bounds__(1024) void k_classify(
    const int* child_count, const long long* child_begin, const Cell* parents,
    int nparents, int batch_max, int merge, Cell* out_batches, Cell* out_next,
    int* counters) {
    __shared__ int smem[17];
    int nb = 0, nn = 0;
    for (int p0 = 0; p0 < nparents; p0 += blockDim.x) {
        const int p = p0 + threadIdx.x;
        int cb = 0, cn = 0;
        const int* cnt = child_count + (size_t)p * kMaxChild;
        const long long* beg = child_begin + (size_t)p * kMaxChild;
        const int atom = (p < nparents) ? parents[p].atom : 0;
        if (p < nparents) {
            const int r = classify_parent(cnt, beg, batch_max, merge, atom, nullptr,
                                          nullptr, false);
            cb = r >> 16;
            cn = r & 0xffff;
        }
        int tb, tn;
        const int pb = block_exclusive_scan(cb, smem, tb);
        const int pn = block_exclusive_scan(cn, smem, tn);
        if (p < nparents)
            classify_parent(cnt, beg, batch_max, merge, atom, out_batches + nb + pb,
                            out_next + nn + pn, true);
        nb += tb;
        nn += tn;
    }
    if (threadIdx.x == 0) {
        counters[0] = nb;
        counters[1] = nn;
    }
}

int run_batching(xc_context* c, const std::vector<long long>& atom_kept) {
    PhaseScope ps(c, XC_PHASE_BATCH);
    std::vector<Cell> cells, batches;
    long long off = 0;
    for (size_t g = 0; g < c->gatoms.size(); ++g) {
        const long long cnt = atom_kept[g];
        if (cnt > 0) {
            Cell x{};
            x.begin = off;
            x.count = (int)cnt;
            x.atom = c->gatoms[g];
            if (cnt <= c->batch_max) batches.push_back(x);
            else cells.push_back(x);
        }
        off += cnt;
    }
    XC_TRY(dev_reserve(c->counters, 4 * sizeof(int)));
    int ncur = (int)cells.size();
    if (ncur > 0) {
        XC_TRY(dev_reserve(c->cells_a, sizeof(Cell) * (size_t)ncur));
        XC_TRY(upload(c->cells_a, cells.data(), sizeof(Cell) * (size_t)ncur, c->stream));
        hipLaunchKernelGGL(k_cell_bbox, dim3(ncur), dim3(256), 0, c->stream,
                           (Cell*)c->cells_a.p, (const double*)c->px.p,
                           (const double*)c->py.p, (const double*)c->pz.p);
        XC_HIP(hipGetLastError());
    }
    int level = 0;
    while (ncur > 0) {
        if (++level > 48)
            return fail(XC_ERR_INVALID_ARG,
                        "batching did not converge (coincident grid points?)");
        const size_t nch = (size_t)ncur * kMaxChild;
        XC_TRY(dev_reserve(c->child_count, sizeof(int) * nch));
        XC_TRY(dev_reserve(c->child_begin, sizeof(long long) * nch));
        XC_TRY(dev_reserve(c->cells_b, sizeof(Cell) * nch));
        XC_TRY(dev_reserve(c->batches, sizeof(Cell) * nch));
        hipLaunchKernelGGL(k_split, dim3(ncur), dim3(kSplitThreads), 0, c->stream,
                           (const Cell*)c->cells_a.p, (const double4*)c->d_atoms.p,
                           c->natoms, (double*)c->px.p, (double*)c->py.p,
                           (double*)c->pz.p, (double*)c->pw.p, (long long*)c->pidx.p,
                           (double*)c->tx.p, (double*)c->ty.p, (double*)c->tz.p,
                           (double*)c->tw.p, (long long*)c->tidx.p,
                           (int*)c->child_count.p, (long long*)c->child_begin.p);
        XC_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_classify, dim3(1), dim3(1024), 0, c->stream,
                           (const int*)c->child_count.p,
                           (const long long*)c->child_begin.p,
                           (const Cell*)c->cells_a.p, ncur, c->batch_max, c->batch_merge,
                           (Cell*)c->batches.p, (Cell*)c->cells_b.p, (int*)c->counters.p);
        XC_HIP(hipGetLastError());
        int cnt[2];
        XC_HIP(hipMemcpyAsync(cnt, c->counters.p, 2 * sizeof(int), hipMemcpyDeviceToHost,
                              c->stream));
        XC_HIP(hipStreamSynchronize(c->stream));
        if (cnt[0] > 0) {
            const size_t old = batches.size();
            batches.resize(old + cnt[0]);
            XC_HIP(hipMemcpyAsync(batches.data() + old, c->batches.p,
                                  sizeof(Cell) * (size_t)cnt[0], hipMemcpyDeviceToHost,
                                  c->stream));
        }
        ncur = cnt[1];
        if (ncur > 0) {
            hipLaunchKernelGGL(k_cell_bbox, dim3(ncur), dim3(256), 0, c->stream,
                               (Cell*)c->cells_b.p, (const double*)c->px.p,
                               (const double*)c->py.p, (const double*)c->pz.p);
            XC_HIP(hipGetLastError());
        }
        std::swap(c->cells_a, c->cells_b);
        XC_HIP(hipStreamSynchronize(c->stream));
    }
    std::sort(batches.begin(), batches.end(),
              [](const Cell& a, const Cell& b) { return a.begin < b.begin; });
    c->n_batches = (long long)batches.size();
    if (c->n_batches > 0) {
        XC_TRY(dev_reserve(c->batches, sizeof(Cell) * batches.size()));
        XC_TRY(upload(c->batches, batches.data(), sizeof(Cell) * batches.size(), c->stream));
        hipLaunchKernelGGL(k_cell_bbox, dim3((unsigned)batches.size()), dim3(256), 0,
                           c->stream, (Cell*)c->batches.p, (const double*)c->px.p,
                           (const double*)c->py.p, (const double*)c->pz.p);
        XC_HIP(hipGetLastError());
        XC_HIP(hipMemcpyAsync(batches.data(), c->batches.p, sizeof(Cell) * batches.size(),
                              hipMemcpyDeviceToHost, c->stream));
        XC_HIP(hipStreamSynchronize(c->stream));
    }
    c->h_batches.swap(batches);
    return XC_OK;
}

// ------------------------------------------------------------ screening ---
// Alg. 1 with the closed-ball reading: the sphere (R, r_cut) meets the box
// [lo, hi] when r_cut^2 minus the squared distance from R to the box is >= 0.
__device__ inline bool shell_meets_box(const ShellDev& s, const Cell& b) {
#pragma clang fp contract(off)
    double d = s.rcut2;
    if (isinf(d)) return true;
    const double r[3] = {s.x, s.y, s.z};
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        if (r[p] < b.lo[p]) {
            const double t = r[p] - b.lo[p];
            d -= t * t;
        } else if (r[p] > b.hi[p]) {
            const double t = r[p] - b.hi[p];
            d -= t * t;
        }
    }
    return d >= 0.0;
}

__global__ void k_screen_count(const Cell* batches, const ShellDev* shells,
                               int nshells, int* nsh, int* nfn) {
    const Cell b = batches[blockIdx.x];
    int cs = 0, cf = 0;
    for (int s = threadIdx.x; s < nshells; s += blockDim.x) {
        const ShellDev sh = shells[s];
        if (shell_meets_box(sh, b)) {
            cs += 1;
            cf += shell_nfunc(sh.L, sh.pure);
        }
    }
    __shared__ int r1[256], r2[256];
    r1[threadIdx.x] = cs;
    r2[threadIdx.x] = cf;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            r1[threadIdx.x] += r1[threadIdx.x + s];
            r2[threadIdx.x] += r2[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        nsh[blockIdx.x] = r1[0];
        nfn[blockIdx.x] = r2[0];
    }
}

// Ordered write of the kept shells, their first local function, and the
// global index of every local function (ascending).
__global__ void k_screen_fill(const Cell* batches, const ShellDev* shells, int nshells,
                              const long long* shoff, const long long* fnoff,
                              int* shell_list, int* shell_loff, int* func_list) {
    const Cell b = batches[blockIdx.x];
    __shared__ int smem[17];
    long long so = shoff[blockIdx.x], fo = fnoff[blockIdx.x];
    int lf = 0;
    for (int s0 = 0; s0 < nshells; s0 += blockDim.x) {
        const int s = s0 + threadIdx.x;
        int keep = 0, nf = 0;
        ShellDev sh{};
        if (s < nshells) {
            sh = shells[s];
            keep = shell_meets_box(sh, b);
            nf = keep ? shell_nfunc(sh.L, sh.pure) : 0;
        }
        int ts, tf;
        const int ps = block_exclusive_scan(keep, smem, ts);
        const int pf = block_exclusive_scan(nf, smem, tf);
        if (keep) {
            shell_list[so + ps] = s;
            shell_loff[so + ps] = lf + pf;
            for (int f = 0; f < nf; ++f) func_list[fo + lf + pf + f] = sh.first_func + f;
        }
        so += ts;
        lf += tf;
    }
}

int run_screening(xc_context* c) {
    PhaseScope ps(c, XC_PHASE_SCREEN);
    const long long nb = c->n_batches;
    c->h_nsh.assign(nb, 0);
    c->h_nfn.assign(nb, 0);
    c->h_shoff.assign(nb + 1, 0);
    c->h_fnoff.assign(nb + 1, 0);
    c->n_shell_entries = c->n_func_entries = 0;
    if (nb == 0) return XC_OK;
    XC_TRY(dev_reserve(c->scr_nsh, sizeof(int) * nb));
    XC_TRY(dev_reserve(c->scr_nfn, sizeof(int) * nb));
    XC_TRY(dev_reserve(c->scr_shoff, sizeof(long long) * (nb + 1)));
    XC_TRY(dev_reserve(c->scr_fnoff, sizeof(long long) * (nb + 1)));
    hipLaunchKernelGGL(k_screen_count, dim3((unsigned)nb), dim3(256), 0, c->stream,
                       (const Cell*)c->batches.p, (const ShellDev*)c->d_shells.p,
                       c->nshells, (int*)c->scr_nsh.p, (int*)c->scr_nfn.p);
    XC_HIP(hipGetLastError());
    XC_HIP(hipMemcpyAsync(c->h_nsh.data(), c->scr_nsh.p, sizeof(int) * nb,
                          hipMemcpyDeviceToHost, c->stream));
    XC_HIP(hipMemcpyAsync(c->h_nfn.data(), c->scr_nfn.p, sizeof(int) * nb,
                          hipMemcpyDeviceToHost, c->stream));
    XC_HIP(hipStreamSynchronize(c->stream));
    for (long long j = 0; j < nb; ++j) {
        c->h_shoff[j + 1] = c->h_shoff[j] + c->h_nsh[j];
        c->h_fnoff[j + 1] = c->h_fnoff[j] + c->h_nfn[j];
    }
    c->n_shell_entries = c->h_shoff[nb];
    c->n_func_entries = c->h_fnoff[nb];
    XC_TRY(upload(c->scr_shoff, c->h_shoff.data(), sizeof(long long) * (nb + 1), c->stream));
    XC_TRY(upload(c->scr_fnoff, c->h_fnoff.data(), sizeof(long long) * (nb + 1), c->stream));
    XC_TRY(dev_reserve(c->shell_list, sizeof(int) * (size_t)std::max(1LL, c->n_shell_entries)));
    XC_TRY(dev_reserve(c->shell_loff, sizeof(int) * (size_t)std::max(1LL, c->n_shell_entries)));
    XC_TRY(dev_reserve(c->func_list, sizeof(int) * (size_t)std::max(1LL, c->n_func_entries)));
    hipLaunchKernelGGL(k_screen_fill, dim3((unsigned)nb), dim3(256), 0, c->stream,
                       (const Cell*)c->batches.p, (const ShellDev*)c->d_shells.p,
                       c->nshells, (const long long*)c->scr_shoff.p,
                       (const long long*)c->scr_fnoff.p, (int*)c->shell_list.p,
                       (int*)c->shell_loff.p, (int*)c->func_list.p);
    XC_HIP(hipGetLastError());
    return XC_OK;
}

}  // namespace xc
