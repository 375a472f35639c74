// Full GMRES on the left-preconditioned system K A x = K b (paper sections
// 3.1, 3.2; K = one multigrid cycle on M), stopped when the preconditioned
// residual ||K b - K A x|| / ||K b|| reaches the tolerance (the paper's GMRES
// criterion, section 5).  Arnoldi step j:
//
//   z = A v_j;  w = K z                                    k_apply, cycle
//   h  = V^H w;        w1 = w - V h                        k_gm_dots, k_gm_axpy
//   if ||w1|| < ||w|| / sqrt(2):                           (device flag)
//       h' = V^H w1;   w1 -= V h';  h += h'                (the same again)
//   h_{j+1,j} = ||w1||;  v_{j+1} = w1 / h_{j+1,j}          k_gm_scale
//   Givens rotations on column j; |g_{j+1}| is the residual norm   k_gm_finalize
//
// Classical Gram-Schmidt with the second sweep taken when the first one
// cancelled more than half the norm (the criterion of Daniel, Gragg,
// Kaufman and Stewart 1976, after Kahan) orthogonalises as well as the
// modified Gram-Schmidt of the published algorithm and needs two passes over
// the basis per sweep instead of j + 1 dependent ones.  The passes of a
// skipped second sweep are still launched and return at once.
// The inner products are exact sums in a fixed order: per-workgroup partials,
// then one workgroup per group of rows adds them (k_gm_rowsum).
//
// Basis vector (i, r) at V + (i * nrhs_max + r) * n.  The per-RHS state
// (Hessenberg matrix, rotations, right-hand side g, coefficients) is a
// GmHead followed by its arrays, GmLayout::words doubles per right-hand side.
#include "hh_common.h"
#include "hh_device.h"
#include "hh_kernels.h"
#include "hh_krylov.h"

namespace hh {

// Layout of one right-hand side's state, in doubles from its start (every
// array starts 16-byte aligned).  Partial-sum rows per right-hand side: the
// inner products of up to M + 1 basis vectors (rounded up to whole groups of
// GM_GROUP) and, after them, one block of 8 rows whose first is ||w||^2
// (a second one, ||K b||^2, at the start of a solve).
constexpr int GM_GROUP = 8;  // basis vectors per workgroup of the inner-product pass
__host__ __device__ inline GmLayout gm_layout(int M) {
    GmLayout L;
    L.norm_row = 2 * ((M + 1 + GM_GROUP - 1) / GM_GROUP) * GM_GROUP;
    L.rows = L.norm_row + 8;
    long long o = sizeof(GmHead) / sizeof(double);
    L.H = o;  o += 2LL * (M + 1) * M;     // H[i][j] at (i * M + j), complex
    L.cs = o; o += 2LL * M;
    L.sn = o; o += 2LL * M;
    L.g = o;  o += 2LL * (M + 1);
    L.y = o;  o += 2LL * M;
    L.h1 = o; o += 2LL * (M + 1);
    L.dots = o; o += L.rows;              // row sums of the last reduction
    L.words = o;
    return L;
}
GmLayout gm_host_layout(int M) { return gm_layout(M); }

namespace {

__device__ __forceinline__ c128* cpt(double* base, long long off) { return reinterpret_cast<c128*>(base + off); }

}  // namespace

// Partial inner products <v_i, w>, i = GM_GROUP * blockIdx.y + 0..GM_GROUP-1 (<= j),
// rows 2i, 2i + 1 of part (row stride nblk); vectors past j give zero rows.
// With wrow >= 0 the workgroups of group 0 also write the partial ||w||^2 to
// row wrow; with gated, only right-hand sides whose reorthogonalisation flag
// is set run.
__global__ __launch_bounds__(256) void k_gm_dots(long long n, int j, const c128* __restrict__ w,
                                                 const c128* __restrict__ V, long long rsv,
                                                 double* __restrict__ part, long long rows_per_rhs, int wrow,
                                                 const double* gst, long long gst_words, int gated,
                                                 const RhsState* st) {
    const int r = blockIdx.z;
    if (st[r].status != ST_RUN) return;
    if (gated && !reinterpret_cast<const GmHead*>(gst + r * gst_words)->reorth) return;
    const int i0 = blockIdx.y * GM_GROUP;
    const bool wn = wrow >= 0 && blockIdx.y == 0;
    const long long off = (long long)r * n;
    double acc[2 * GM_GROUP], an[1] = {0.0};
#pragma unroll
    for (int q = 0; q < 2 * GM_GROUP; ++q) acc[q] = 0.0;
    for (long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x; x < n;
         x += (long long)gridDim.x * blockDim.x) {
        const c128 wv = w[off + x];
        if (wn) an[0] += abs2(wv);
#pragma unroll
        for (int q = 0; q < GM_GROUP; ++q)
            if (i0 + q <= j) {
                const c128 d = cdot(ld_stream(&V[(i0 + q) * rsv + off + x]), wv);
                acc[2 * q] += d.re;
                acc[2 * q + 1] += d.im;
            }
    }
    const long long nblk = gridDim.x;
    double* dst = part + ((long long)r * rows_per_rhs + 2LL * i0) * nblk + blockIdx.x;
    block_sum_store<2 * GM_GROUP>(acc, dst, nblk);
    if (wn) block_sum_store<1>(an, part + ((long long)r * rows_per_rhs + wrow) * nblk + blockIdx.x, nblk);
}

// w_out = w_in - sum_{i<=j} c_i v_i with c from the state's h1 (first sweep) or
// dots (second sweep); with NORM also the partial ||w_out||^2 (row norm_row).
template <bool NORM>
__global__ __launch_bounds__(256) void k_gm_axpy(long long n, int j, const c128* __restrict__ w_in,
                                                 c128* __restrict__ w_out, const c128* __restrict__ V,
                                                 long long rsv, const double* __restrict__ gst,
                                                 long long gst_words, long long coef_off,
                                                 double* __restrict__ part, long long rows_per_rhs,
                                                 int norm_row, int gated, const RhsState* st) {
    const int r = blockIdx.z;
    if (st[r].status != ST_RUN) return;
    if (gated && !reinterpret_cast<const GmHead*>(gst + r * gst_words)->reorth) return;
    const c128* coef = reinterpret_cast<const c128*>(gst + r * gst_words + coef_off);
    const long long off = (long long)r * n;
    double acc[1] = {0.0};
    for (long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x; x < n;
         x += (long long)gridDim.x * blockDim.x) {
        c128 a = ld_stream(&w_in[off + x]);
        for (int i = 0; i <= j; ++i) a = a - coef[i] * ld_stream(&V[i * rsv + off + x]);
        st_stream(&w_out[off + x], a);
        if (NORM) acc[0] += abs2(a);
    }
    if (NORM) {
        const long long nblk = gridDim.x;
        block_sum_store<1>(acc, part + ((long long)r * rows_per_rhs + norm_row) * nblk + blockIdx.x, nblk);
    }
}

// Row sums of the partials: rows row_begin + [8 blockIdx.x, 8 blockIdx.x + 8)
// (those below row_begin + nrows) of right-hand side blockIdx.y, each over
// nblk partials in a fixed order, into the same rows of the state's dots array.
__global__ __launch_bounds__(256) void k_gm_rowsum(int row_begin, int nrows, const double* __restrict__ part,
                                                   long long nblk, long long rows_per_rhs, double* __restrict__ gst,
                                                   long long gst_words, long long dots_off, int gated,
                                                   const RhsState* st) {
    const int r = blockIdx.y;
    if (st[r].status != ST_RUN) return;
    if (gated && !reinterpret_cast<const GmHead*>(gst + r * gst_words)->reorth) return;
    const int row0 = row_begin + blockIdx.x * 8;
    double o[8];
    block_fixed_sum<8>(part + ((long long)r * rows_per_rhs + row0) * nblk, nblk, nblk, o);
    if (threadIdx.x == 0)
        for (int q = 0; q < 8 && row0 + q < row_begin + nrows; ++q) gst[r * gst_words + dots_off + row0 + q] = o[q];
}

// Partial ||a||^2 into row `row` (start of a cycle: ||K r0||^2 and ||K b||^2)
__global__ __launch_bounds__(256) void k_gm_norm2(long long n, const c128* __restrict__ a, double* __restrict__ part,
                                                  long long rows_per_rhs, int row, const RhsState* st) {
    const int r = blockIdx.z;
    if (st[r].status != ST_RUN) return;
    const long long off = (long long)r * n;
    double acc[1] = {0.0};
    for (long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x; x < n;
         x += (long long)gridDim.x * blockDim.x)
        acc[0] += abs2(a[off + x]);
    const long long nblk = gridDim.x;
    block_sum_store<1>(acc, part + ((long long)r * rows_per_rhs + row) * nblk + blockIdx.x, nblk);
}

// clear the update flags after the solution update
__global__ void k_gm_clear(int nrhs, double* gst, long long gst_words) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < nrhs) reinterpret_cast<GmHead*>(gst + r * gst_words)->update = 0;
}

// dst = src * state.scale (the new basis vector, or the first one); src2
// replaces src when the reorthogonalisation flag is set
__global__ __launch_bounds__(256) void k_gm_scale(long long n, const c128* __restrict__ src1,
                                                  const c128* __restrict__ src2, c128* __restrict__ dst,
                                                  const double* __restrict__ gst, long long gst_words,
                                                  const RhsState* st) {
    const int r = blockIdx.z;
    if (st[r].status != ST_RUN) return;
    const GmHead* hd = reinterpret_cast<const GmHead*>(gst + r * gst_words);
    const double sc = hd->scale;
    const c128* __restrict__ src = hd->reorth ? src2 : src1;
    const long long off = (long long)r * n;
    for (long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x; x < n;
         x += (long long)gridDim.x * blockDim.x)
        dst[off + x] = sc * src[off + x];
}

// x += sum_{i<m} y_i v_i for right-hand sides whose cycle ended (status CONV,
// or the restart flag of a full basis)
__global__ __launch_bounds__(256) void k_gm_xupdate(long long n, c128* __restrict__ xk, const c128* __restrict__ V,
                                                    long long rsv, const double* __restrict__ gst,
                                                    long long gst_words, long long y_off) {
    const int r = blockIdx.z;
    const GmHead* hd = reinterpret_cast<const GmHead*>(gst + r * gst_words);
    if (!hd->update) return;
    const int m = hd->m;
    const c128* y = reinterpret_cast<const c128*>(gst + r * gst_words + y_off);
    const long long off = (long long)r * n;
    for (long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x; x < n;
         x += (long long)gridDim.x * blockDim.x) {
        c128 a = ld_stream(&xk[off + x]);
        for (int i = 0; i < m; ++i) a = a + y[i] * ld_stream(&V[i * rsv + off + x]);
        st_stream(&xk[off + x], a);
    }
}

// Scalar part, one thread per right-hand side.
//   GM_FIN_START: beta = ||K r0|| (row norm_row); ||K b|| from row norm_row + 1
//     (kb = 1), equal to beta (kb = 0: x0 = 0), or kept (kb = 2: a restart, whose
//     new residual cost one product); g = beta e_1; scale = 1 / beta; stop if
//     beta / ||K b|| <= tol.
//   GM_FIN_DOTS1: h1 = first-sweep inner products (rows 0 .. 2j+1).
//   GM_FIN_DOTS2: column j of H = h1 + second-sweep products; h_{j+1,j} =
//     ||w|| (row norm_row); rotations; |g_{j+1}| test; scale = 1 / h_{j+1,j};
//     at the tolerance or at the last column: y = H^-1 g and the update flag.
__global__ void k_gm_finalize(int mode, int j, int M, int kb, double tol, RhsState* st, double* gst,
                              long long gst_words) {
    const int r = blockIdx.x;
    if (threadIdx.x != 0) return;
    RhsState& R = st[r];
    if (R.status != ST_RUN) return;
    const GmLayout L = gm_layout(M);
    const int norm_row = L.norm_row;
    double* base = gst + r * gst_words;
    GmHead& hd = *reinterpret_cast<GmHead*>(base);
    const double* dots = base + L.dots;
    c128* H = cpt(base, L.H);
    c128* cs = cpt(base, L.cs);
    c128* sn = cpt(base, L.sn);
    c128* g = cpt(base, L.g);
    c128* y = cpt(base, L.y);
    c128* h1 = cpt(base, L.h1);
    auto solve_y = [&](int m) {
        for (int i = m - 1; i >= 0; --i) {
            c128 a = g[i];
            for (int k = i + 1; k < m; ++k) a = a - H[i * M + k] * y[k];
            y[i] = cdiv(a, H[i * M + i]);
        }
        hd.m = m;
        hd.update = 1;
    };
    // the relative preconditioned residual is reported through rnorm2 / bnorm2
    auto set_res = [&](double rel) { R.rnorm2 = rel * rel * R.bnorm2; };
    if (mode == GM_FIN_START) {
        const double b2 = dots[norm_row];
        if (!isfinite(b2)) { R.status = ST_NUMERIC; return; }
        hd.beta = sqrt(b2);
        if (kb == 1) {
            if (!isfinite(dots[norm_row + 1])) { R.status = ST_NUMERIC; return; }
            hd.kbn = sqrt(dots[norm_row + 1]);
        } else if (kb == 0) {
            hd.kbn = hd.beta;
            R.matvecs = 0;  // r0 = b: no product with A yet
        } else {
            R.matvecs += 1;  // restart of a full basis: its residual b - A x
            R.restarts += 1;
        }
        hd.m = 0;
        hd.update = 0;
        g[0] = mk(hd.beta, 0.0);
        set_res(hd.kbn > 0.0 ? hd.beta / hd.kbn : 0.0);
        if (hd.kbn == 0.0 || hd.beta <= tol * hd.kbn) { R.status = ST_CONV; return; }
        hd.scale = 1.0 / hd.beta;
        return;
    }
    if (mode == GM_FIN_DOTS1) {
        for (int i = 0; i <= j; ++i) h1[i] = mk(dots[2 * i], dots[2 * i + 1]);
        hd.reorth = 0;
        return;
    }
    if (mode == GM_FIN_REORTH) {
        // second sweep when the first one removed more than half of ||w||^2
        const double w2 = dots[norm_row + 2], w12 = dots[norm_row];
        if (!isfinite(w2) || !isfinite(w12)) { R.status = ST_NUMERIC; return; }
        hd.reorth = w12 < 0.5 * w2;
        return;
    }
    // GM_FIN_DOTS2
    R.matvecs += 1;
    R.iters2 += 2;
    for (int i = 0; i <= j; ++i) {
        const c128 hij = hd.reorth ? h1[i] + mk(dots[2 * i], dots[2 * i + 1]) : h1[i];
        if (!isfinite(hij.re) || !isfinite(hij.im)) { R.status = ST_NUMERIC; return; }
        H[i * M + j] = hij;
    }
    const double hn = sqrt(dots[norm_row]);
    if (!isfinite(hn)) { R.status = ST_NUMERIC; return; }
    // earlier rotations on column j
    for (int i = 0; i < j; ++i) {
        const c128 a = H[i * M + j], b = H[(i + 1) * M + j];
        H[i * M + j] = cs[i] * a + sn[i] * b;
        H[(i + 1) * M + j] = conj(cs[i]) * b - conj(sn[i]) * a;
    }
    // the rotation that zeroes h_{j+1,j}: [c s; -conj(s) c] with c real
    const c128 a = H[j * M + j];
    const double aa = sqrt(abs2(a));
    const double den = sqrt(abs2(a) + hn * hn);
    if (den == 0.0) { R.status = ST_BREAK; return; }
    const c128 c = mk(aa / den, 0.0);
    const c128 s = aa > 0.0 ? (1.0 / (aa * den)) * mk(a.re * hn, a.im * hn) : mk(1.0, 0.0);
    cs[j] = c;
    sn[j] = s;
    H[j * M + j] = c * a + mk(s.re * hn, s.im * hn);
    g[j + 1] = mk(0.0, 0.0) - conj(s) * g[j];
    g[j] = c * g[j];
    const double res = sqrt(abs2(g[j + 1]));
    set_res(res / hd.kbn);
    if (res <= tol * hd.kbn || hn == 0.0) {
        solve_y(j + 1);
        R.status = ST_CONV;
        return;
    }
    if (j + 1 == M || R.iters2 >= R.maxit2) {
        // basis full (the host restarts from the updated x) or iteration limit
        solve_y(j + 1);
        if (R.iters2 >= R.maxit2) R.status = ST_MAXIT;
        return;
    }
    hd.scale = 1.0 / hn;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
void launch_gm_dots(hipStream_t s, long long n, int nrhs, int j, const c128* w, const c128* V, long long rsv,
                    double* part, long long rows_per_rhs, int wrow, const double* gst, long long gst_words,
                    bool gated, const RhsState* st) {
    const dim3 grid(GM_NBLK, (j + GM_GROUP) / GM_GROUP, nrhs);
    hipLaunchKernelGGL(k_gm_dots, grid, dim3(256), 0, s, n, j, w, V, rsv, part, rows_per_rhs, wrow, gst, gst_words,
                       (int)gated, st);
}
void launch_gm_axpy(hipStream_t s, long long n, int nrhs, int j, const c128* w_in, c128* w_out, const c128* V,
                    long long rsv, const double* gst, long long gst_words, long long coef_off, bool norm,
                    double* part, long long rows_per_rhs, int norm_row, bool gated, const RhsState* st) {
    const dim3 grid(GM_NBLK, 1, nrhs);
    if (norm)
        hipLaunchKernelGGL(k_gm_axpy<true>, grid, dim3(256), 0, s, n, j, w_in, w_out, V, rsv, gst, gst_words,
                           coef_off, part, rows_per_rhs, norm_row, (int)gated, st);
    else
        hipLaunchKernelGGL(k_gm_axpy<false>, grid, dim3(256), 0, s, n, j, w_in, w_out, V, rsv, gst, gst_words,
                           coef_off, part, rows_per_rhs, norm_row, (int)gated, st);
}
void launch_gm_rowsum(hipStream_t s, int nrhs, int row_begin, int nrows, const double* part, long long rows_per_rhs,
                      double* gst, long long gst_words, long long dots_off, bool gated, const RhsState* st) {
    hipLaunchKernelGGL(k_gm_rowsum, dim3((nrows + 7) / 8, nrhs), dim3(256), 0, s, row_begin, nrows, part,
                       (long long)GM_NBLK, rows_per_rhs, gst, gst_words, dots_off, (int)gated, st);
}
void launch_gm_norm2(hipStream_t s, long long n, int nrhs, const c128* a, double* part, long long rows_per_rhs,
                     int row, const RhsState* st) {
    hipLaunchKernelGGL(k_gm_norm2, dim3(GM_NBLK, 1, nrhs), dim3(256), 0, s, n, a, part, rows_per_rhs, row, st);
}
void launch_gm_clear(hipStream_t s, int nrhs, double* gst, long long gst_words) {
    hipLaunchKernelGGL(k_gm_clear, dim3(1), dim3(64), 0, s, nrhs, gst, gst_words);
}
void launch_gm_scale(hipStream_t s, long long n, int nrhs, const c128* src1, const c128* src2, c128* dst,
                     const double* gst, long long gst_words, const RhsState* st) {
    hipLaunchKernelGGL(k_gm_scale, dim3(GM_NBLK, 1, nrhs), dim3(256), 0, s, n, src1, src2, dst, gst, gst_words, st);
}
void launch_gm_xupdate(hipStream_t s, long long n, int nrhs, c128* xk, const c128* V, long long rsv,
                       const double* gst, long long gst_words, long long y_off) {
    hipLaunchKernelGGL(k_gm_xupdate, dim3(GM_NBLK, 1, nrhs), dim3(256), 0, s, n, xk, V, rsv, gst, gst_words, y_off);
}
void launch_gm_finalize(hipStream_t s, int mode, int j, int M, int kb, double tol, int nrhs, RhsState* st,
                        double* gst, long long gst_words) {
    hipLaunchKernelGGL(k_gm_finalize, dim3(nrhs), dim3(64), 0, s, mode, j, M, kb, tol, st, gst, gst_words);
}

}  // namespace hh
