// Device helpers shared by the kernel translation units.
#pragma once
#include "hh_common.h"
#include "hh_kernels.h"

namespace hh {

__device__ __forceinline__ bool gate_ok(const RhsState* st, int r, int gate) {
    if (st == nullptr || gate == GATE_ALL) return true;
    int s = st[r].status;
    if (gate == GATE_FINISHED) return s != ST_RUN && s != ST_IDLE && s != ST_HALF;
    return s == gate;
}

template <typename R>
__device__ __forceinline__ cx<R> czero() { return cx<R>{R(0), R(0)}; }

// Streaming access: loads and stores with the non-temporal hint, for data a
// kernel touches once (the Krylov vectors in the update kernels of
// Bi-CGSTAB, IDR(s) and GMRES).  Measured on the 513^3 cube: the x / r update
// 2.87 -> 2.57 ms, the p update 1.96 -> 1.84 ms, the s update 1.44 -> 1.38 ms
// against plain loads and stores; on the wedge IDR(4) 35.7 -> 34.4 ms and
// GMRES 252 -> 238 ms per solve.  The stencil kernels, whose halos are
// re-read through the caches, are slower with them.
typedef double hh_d2 __attribute__((ext_vector_type(2)));
typedef float hh_f2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ c128 ld_stream(const c128* p) {
    const hh_d2 v = __builtin_nontemporal_load(reinterpret_cast<const hh_d2*>(p));
    return {v.x, v.y};
}
__device__ __forceinline__ c64 ld_stream(const c64* p) {
    const hh_f2 v = __builtin_nontemporal_load(reinterpret_cast<const hh_f2*>(p));
    return {v.x, v.y};
}
__device__ __forceinline__ void st_stream(c128* p, const c128& a) {
    const hh_d2 v = {a.re, a.im};
    __builtin_nontemporal_store(v, reinterpret_cast<hh_d2*>(p));
}
__device__ __forceinline__ void st_stream(c64* p, const c64& a) {
    const hh_f2 v = {a.re, a.im};
    __builtin_nontemporal_store(v, reinterpret_cast<hh_f2*>(p));
}

// Deterministic block reduction of NT doubles: butterfly within each 64-lane
// wavefront, then wavefront partials summed by thread 0 in wave order.  The
// result goes to out[t * stride] for t < NT.
template <int NT>
__device__ __forceinline__ void block_sum_store(double (&v)[NT], double* out, long long stride) {
    __shared__ double sm[NT][16];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
        for (int t = 0; t < NT; ++t) v[t] += __shfl_xor(v[t], off, 64);
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int t = 0; t < NT; ++t) sm[t][wid] = v[t];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            double s = 0.0;
            for (int w = 0; w < nw; ++w) s += sm[t][w];
            out[t * stride] = s;
        }
    }
}

// Sum of the per-workgroup partials of NT consecutive rows (row t at
// part[t * nblk_max]) in a fixed order, for the one-workgroup finalize kernels.
// Every thread receives the sums.
template <int NT>
__device__ inline void block_fixed_sum(const double* __restrict__ part, long long nblk, long long nblk_max,
                                double (&out)[NT]) {
    __shared__ double sm[NT][16];
    double v[NT];
    // lane t adds partials t, t + blockDim, t + 2 blockDim, ... in that order; the
    // loads of U consecutive terms of that sequence are issued before their adds
    // (out-of-range slots read a valid partial and add exactly zero).  U only
    // sets how many loads are in flight (fewer for many rows, to stay in
    // registers); the order of the adds, and so the sum, does not depend on it.
    constexpr int U = NT <= 4 ? 8 : (NT <= 8 ? 4 : 2);
#pragma unroll
    for (int t = 0; t < NT; ++t) v[t] = 0.0;
    for (long long b0 = threadIdx.x; b0 < nblk; b0 += (long long)U * blockDim.x) {
        double ld[NT][U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long long b = b0 + (long long)u * blockDim.x;
            const long long bc = b < nblk ? b : nblk - 1;
#pragma unroll
            for (int t = 0; t < NT; ++t) ld[t][u] = part[t * nblk_max + bc];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool in = b0 + (long long)u * blockDim.x < nblk;
#pragma unroll
            for (int t = 0; t < NT; ++t) v[t] += in ? ld[t][u] : 0.0;
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
        for (int t = 0; t < NT; ++t) v[t] += __shfl_xor(v[t], off, 64);
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int t = 0; t < NT; ++t) sm[t][wid] = v[t];
    }
    __syncthreads();
    const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += sm[t][w];
        out[t] = s;
    }
}

__device__ __forceinline__ long long part_index(int r, int slot, int term, long long nblk_max) {
    return ((long long)(r * NSLOT + slot) * MAX_TERMS + term) * nblk_max;
}


// Workgroup -> tile map that keeps neighbouring tiles on one XCD.  The
// dispatcher hands workgroup i to XCD i % 8 (round robin over the 8 XCDs of
// the MI355X); this permutation gives XCD x a contiguous range of tiles, so
// the halo rows two neighbouring tiles share stay in that XCD's L2.  It is a
// bijection of [0, N) whatever the dispatch order.
__device__ __forceinline__ int xcd_tile_id(int id, int N) {
    constexpr int NX = 8;
    const int per = N / NX, rem = N % NX;
    const int x = id % NX, k = id / NX;
    return x < rem ? x * (per + 1) + k : rem * (per + 1) + (x - rem) * per + k;
}

// Index of a fine-grid node reached through the boundary: a position outside
// [0, n) is replaced by its mirror image (the eliminated ghost point of a
// Sommerfeld boundary, or the even extension of the full-weighting stencil),
// then clamped so that lanes past the end of a tile stay in bounds.
__device__ __forceinline__ int mirror_clamp(int g, int n) {
    if (g < 0) g = -g;
    if (g > n - 1) g = 2 * (n - 1) - g;
    return g < 0 ? 0 : (g > n - 1 ? n - 1 : g);
}

}  // namespace hh
