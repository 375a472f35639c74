// Large coarsest grids on gfx950: the dense inverse of the coarsest
// rediscretised M by Gauss-Jordan elimination with partial pivoting on the
// device (set-up, once per model), and the exact coarsest solve e = M_c^-1 b as
// a multi-workgroup product with that inverse.
//
// The multigrid cycle ends in an exact solve on the coarsest level (paper
// section 3.4, Algorithm 1; the paper's own runs use GMRES to a 1e-11 residual
// there, which is the exact solve up to that tolerance).  Small coarsest grids
// are solved inside the single-workgroup tail kernel, with an inverse formed
// on the host up to 256 unknowns and here above.  A grid such as the 17^3
// coarsest level of the paper's closed-off experiments (Table 1) has
// thousands of unknowns, too many for one workgroup's LDS and for a host
// elimination at set-up: its inverse is formed here and the solve is the
// multi-workgroup product below.
#include "hh_coarse.h"
#include "hh_device.h"

namespace hh {

namespace {
constexpr int GJ_PIVOT_LANES = 1024;
constexpr int GJ_LANES = 256;
}  // namespace

// Pivot row of column col: largest |a_rc|^2 over rows col .. n - 1, the first
// one on ties; its value goes to pval (read by the next kernels before the
// pivot row is overwritten).
__global__ __launch_bounds__(GJ_PIVOT_LANES) void k_gj_pivot(int n, const c128* __restrict__ a, int col,
                                                             int* piv, c128* pval, int* bad) {
    __shared__ double sv[GJ_PIVOT_LANES];
    __shared__ int si[GJ_PIVOT_LANES];
    const int t = threadIdx.x;
    double best = -1.0;
    int bi = col;
    for (int r = col + t; r < n; r += GJ_PIVOT_LANES) {
        const double m = abs2(a[(long long)r * n + col]);
        if (m > best) {
            best = m;
            bi = r;
        }
    }
    sv[t] = best;
    si[t] = bi;
    __syncthreads();
    for (int w = GJ_PIVOT_LANES / 2; w > 0; w >>= 1) {
        if (t < w) {
            const double o = sv[t + w];
            const int oi = si[t + w];
            if (o > sv[t] || (o == sv[t] && oi < si[t])) {
                sv[t] = o;
                si[t] = oi;
            }
        }
        __syncthreads();
    }
    if (t == 0) {
        *piv = si[0];
        *pval = a[(long long)si[0] * n + col];
        if (!(sv[0] > 0.0) || !isfinite(sv[0])) *bad = 1;
    }
}

// Swap rows col and piv of [a | inv] and scale row col by 1 / pval: one lane
// per column of the augmented matrix.
__global__ __launch_bounds__(GJ_LANES) void k_gj_swap_scale(int n, c128* __restrict__ a,
                                                            c128* __restrict__ inv, int col,
                                                            const int* piv, const c128* pval) {
    const int j = blockIdx.x * GJ_LANES + threadIdx.x;
    if (j >= 2 * n) return;
    c128* m = j < n ? a : inv;
    const int jj = j < n ? j : j - n;
    const int p = *piv;
    const c128 dinv = cdiv(mk(1.0, 0.0), *pval);
    c128 v = m[(long long)col * n + jj];
    if (p != col) {
        const c128 vp = m[(long long)p * n + jj];
        m[(long long)p * n + jj] = v;
        v = vp;
    }
    m[(long long)col * n + jj] = v * dinv;
}

// Elimination factors f_r = a_r,col, taken before the elimination changes
// them; the pivot row gets 0.
__global__ __launch_bounds__(GJ_LANES) void k_gj_factors(int n, const c128* __restrict__ a, int col,
                                                         c128* __restrict__ f) {
    const int r = blockIdx.x * GJ_LANES + threadIdx.x;
    if (r >= n) return;
    f[r] = r == col ? mk(0.0, 0.0) : a[(long long)r * n + col];
}

// row_r -= f_r row_col for every row r != col.  Columns of a left of col are
// already unit vectors and unchanged, so the a part covers columns col .. n - 1;
// the inv part covers all n columns.  gridDim = (column blocks, n rows).
__global__ __launch_bounds__(GJ_LANES) void k_gj_eliminate(int n, c128* __restrict__ a,
                                                           c128* __restrict__ inv, int col,
                                                           const c128* __restrict__ f) {
    const int r = blockIdx.y;
    if (r == col) return;
    const c128 fr = f[r];
    if (fr.re == 0.0 && fr.im == 0.0) return;
    const int na = n - col;
    const int j = blockIdx.x * GJ_LANES + threadIdx.x;
    if (j >= na + n) return;
    c128* m;
    int jj;
    if (j < na) {
        m = a;
        jj = col + j;
    } else {
        m = inv;
        jj = j - na;
    }
    const long long o = (long long)r * n + jj;
    m[o] = m[o] - fr * m[(long long)col * n + jj];
}

// inv = I
__global__ __launch_bounds__(GJ_LANES) void k_gj_identity(int n, c128* __restrict__ inv) {
    const long long i = (long long)blockIdx.x * GJ_LANES + threadIdx.x;
    if (i >= (long long)n * n) return;
    const int r = (int)(i / n), j = (int)(i - (long long)r * n);
    inv[i] = mk(r == j ? 1.0 : 0.0, 0.0);
}

template <typename T>
__global__ __launch_bounds__(GJ_LANES) void k_gj_store(int n, const c128* __restrict__ inv,
                                                       cx<T>* __restrict__ minv) {
    const long long i = (long long)blockIdx.x * GJ_LANES + threadIdx.x;
    if (i >= (long long)n * n) return;
    const int j = (int)(i / n), r = (int)(i - (long long)j * n);
    minv[i] = cvt<T>(inv[(long long)r * n + j]);
}

// e = M_c^-1 b with the inverse and the sums in complex128 for either
// multigrid precision (a large coarsest grid's solve adds thousands of terms
// per row; complex64 sums perturb the preconditioner enough to cost Krylov
// steps).  Two passes so that the product fills the chip:
//   k_coarse_gemv: workgroup (row block, column chunk) of 256 lanes = 64 rows x
//     4 waves; the chunk's CG_COLS gathered right-hand-side entries are staged
//     in LDS, wave w sums its quarter of the chunk for the 64 rows (the lanes of
//     a wave read one column's 64 consecutive rows: coalesced), and the four
//     wave sums are added in wave order into part[rhs][chunk][row];
//   k_coarse_sum: e at every node of the level: the chunk sums of its unknown
//     in chunk order, or 0 at a node that is not an unknown.
// gridDim = (row blocks, chunks, right-hand sides) and (node blocks, 1, rhs).
constexpr int CG_ROWS = 64, CG_LANES = 256, CG_WAVES = CG_LANES / CG_ROWS, CG_COLS = 128;
static_assert(CG_COLS <= CG_LANES, "one staging load per lane");

template <typename R>
__global__ __launch_bounds__(CG_LANES) void k_coarse_gemv(int nnode, int n, const int* __restrict__ cidx,
                                                          const c128* __restrict__ minv,
                                                          const cx<R>* __restrict__ b, c128* __restrict__ part,
                                                          const RhsState* st, int gate) {
    __shared__ c128 bg[CG_COLS];
    __shared__ c128 ps[CG_WAVES][CG_ROWS];
    const int r = blockIdx.z;
    if (!gate_ok(st, r, gate)) return;
    const int t = threadIdx.x;
    const int chunk = blockIdx.y, nch = gridDim.y;
    const int c0 = chunk * CG_COLS, c1 = min(n, c0 + CG_COLS);
    const cx<R>* br = b + (long long)r * nnode;
    if (t < c1 - c0) bg[t] = cvt<double>(br[cidx[c0 + t]]);
    __syncthreads();
    const int lane = t & (CG_ROWS - 1), w = t / CG_ROWS;
    const int row = blockIdx.x * CG_ROWS + lane;
    const int rr = row < n ? row : n - 1;  // lanes past the last row read a valid row and store nothing
    constexpr int PER = CG_COLS / CG_WAVES;
    const int a0 = c0 + w * PER, a1 = min(c1, a0 + PER);
    c128 acc = czero<double>();
#pragma unroll 8
    for (int c = a0; c < a1; ++c) acc = acc + minv[(long long)c * n + rr] * bg[c - c0];
    ps[w][lane] = acc;
    __syncthreads();
    if (w == 0 && row < n) {
        c128 sum = ps[0][lane];
#pragma unroll
        for (int q = 1; q < CG_WAVES; ++q) sum = sum + ps[q][lane];
        part[((long long)r * nch + chunk) * n + row] = sum;
    }
}

template <typename R>
__global__ __launch_bounds__(CG_LANES) void k_coarse_sum(int nnode, int n, int nch, const int* __restrict__ unk_of,
                                                         const c128* __restrict__ part, cx<R>* __restrict__ e,
                                                         const RhsState* st, int gate) {
    const int r = blockIdx.z;
    if (!gate_ok(st, r, gate)) return;
    const int i = blockIdx.x * CG_LANES + threadIdx.x;
    if (i >= nnode) return;
    const int u = unk_of[i];
    c128 sum = czero<double>();
    if (u >= 0)
        for (int ch = 0; ch < nch; ++ch) sum = sum + part[((long long)r * nch + ch) * n + u];
    e[(long long)r * nnode + i] = cvt<R>(sum);
}

// ---------------------------------------------------------------------------
// Host-side launchers
// ---------------------------------------------------------------------------
void launch_gj_step(hipStream_t s, int n, c128* a, c128* inv, int col, int* piv, c128* pval, c128* f,
                    int* bad) {
    hipLaunchKernelGGL(k_gj_pivot, dim3(1), dim3(GJ_PIVOT_LANES), 0, s, n, a, col, piv, pval, bad);
    hipLaunchKernelGGL(k_gj_swap_scale, dim3((2 * n + GJ_LANES - 1) / GJ_LANES), dim3(GJ_LANES), 0, s, n, a,
                       inv, col, piv, pval);
    hipLaunchKernelGGL(k_gj_factors, dim3((n + GJ_LANES - 1) / GJ_LANES), dim3(GJ_LANES), 0, s, n, a, col, f);
    const int cols = (n - col) + n;
    hipLaunchKernelGGL(k_gj_eliminate, dim3((cols + GJ_LANES - 1) / GJ_LANES, n), dim3(GJ_LANES), 0, s, n, a,
                       inv, col, f);
}

void launch_gj_identity(hipStream_t s, int n, c128* inv) {
    const long long nn = (long long)n * n;
    hipLaunchKernelGGL(k_gj_identity, dim3((unsigned)((nn + GJ_LANES - 1) / GJ_LANES)), dim3(GJ_LANES), 0, s, n,
                       inv);
}

void launch_gj_store(hipStream_t s, int n, const c128* inv, void* minv, bool low) {
    const long long nn = (long long)n * n;
    const dim3 grid((unsigned)((nn + GJ_LANES - 1) / GJ_LANES));
    if (low) hipLaunchKernelGGL(k_gj_store<float>, grid, dim3(GJ_LANES), 0, s, n, inv, (c64*)minv);
    else hipLaunchKernelGGL(k_gj_store<double>, grid, dim3(GJ_LANES), 0, s, n, inv, (c128*)minv);
}

int coarse_gemv_chunks(int n_unk) { return (n_unk + CG_COLS - 1) / CG_COLS; }

template <typename R>
void launch_coarse_gemv(hipStream_t s, int nnode, int n_unk, const int* unk_of, const int* cidx,
                        const c128* minv, const cx<R>* b, cx<R>* e, c128* part, int nrhs, const RhsState* st,
                        int gate) {
    const int nch = coarse_gemv_chunks(n_unk);
    hipLaunchKernelGGL((k_coarse_gemv<R>), dim3((unsigned)((n_unk + CG_ROWS - 1) / CG_ROWS), (unsigned)nch,
                                                (unsigned)nrhs),
                       dim3(CG_LANES), 0, s, nnode, n_unk, cidx, minv, b, part, st, gate);
    hipLaunchKernelGGL((k_coarse_sum<R>), dim3((unsigned)((nnode + CG_LANES - 1) / CG_LANES), 1, (unsigned)nrhs),
                       dim3(CG_LANES), 0, s, nnode, n_unk, nch, unk_of, part, e, st, gate);
}
template void launch_coarse_gemv<double>(hipStream_t, int, int, const int*, const int*, const c128*, const c128*,
                                         c128*, c128*, int, const RhsState*, int);
template void launch_coarse_gemv<float>(hipStream_t, int, int, const int*, const int*, const c128*, const c64*,
                                        c64*, c128*, int, const RhsState*, int);

}  // namespace hh
