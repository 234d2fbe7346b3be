// Small device helpers: block scans and reductions, launch geometry.
#pragma once

#include <hip/hip_runtime.h>

namespace xc {

// Exclusive scan of one int per thread across the block (blockDim.x a
// multiple of 64, at most 1024). smem needs 17 ints. Every thread receives
// the block total.
__device__ inline int block_exclusive_scan(int v, int* smem, int& total) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) smem[wid] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        int run = 0;
        for (int w = 0; w < nw; ++w) {
            int t = smem[w];
            smem[w] = run;
            run += t;
        }
        smem[nw] = run;
    }
    __syncthreads();
    int excl = smem[wid] + x - v;
    total = smem[nw];
    __syncthreads();
    return excl;
}

// Sum of one double per thread across a 256-thread block in a fixed order
// (the same tree every run). smem needs 256 doubles. Result valid in thread 0.
__device__ inline double block_sum_256(double v, double* smem) {
    smem[threadIdx.x] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) smem[threadIdx.x] += smem[threadIdx.x + s];
        __syncthreads();
    }
    double r = smem[0];
    __syncthreads();
    return r;
}

// Workgroups are dispatched round-robin over the 8 XCDs; this maps the
// hardware block id to a logical id so that consecutive logical ids run on
// the same XCD and share its L2.
// Value of v on lane l of the wave (l wave-uniform). The register is read
// even where lane l is inactive, so v must have been written there.
__device__ __forceinline__ double readlane_f64(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Cartesian functions of a shell of angular momentum L.
__device__ inline int ncart(int L) { return (L + 1) * (L + 2) / 2; }

__device__ inline int xcd_remap(int bid, int nblk) {
    const int xcd = bid & 7, idx = bid >> 3;
    const int base = nblk >> 3, rem = nblk & 7;
    return (xcd < rem) ? xcd * (base + 1) + idx
                       : rem * (base + 1) + (xcd - rem) * base + idx;
}

// Pointers that kernels read out of device-side descriptors are generic to
// the compiler, so their loads and atomics become flat instructions. Flat
// operations also count against the LDS wait counter: a wait for LDS data
// then also waits for every global load in flight, which defeats
// prefetching. Typed global pointers keep these accesses on the global path.
template <typename T> using gptr = __attribute__((address_space(1))) T*;
template <typename T> __device__ __forceinline__ gptr<T> to_global(T* p) {
    return (gptr<T>)p;
}

inline unsigned grid_1d(long long n, int block) {
    return (unsigned)((n + block - 1) / block);
}

}  // namespace xc
