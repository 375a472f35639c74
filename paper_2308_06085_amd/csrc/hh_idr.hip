// IDR(s) on the device (paper section 3.1: the IDR(4) solver of the paper's
// framework, after Sonneveld and van Gijzen), biorthogonal variant with the
// preconditioner on the right, so r stays the residual b - A x that the
// stopping rule of section 5 tests.  One cycle is s inner steps and one
// dimension-reduction step:
//
//   inner step k (0 <= k < s), with c = M[k:s, k:s]^-1 f[k:s] (lower triangular):
//     v   = K (r - sum_{j>=k} c_j g_j)                   k_idr_v / k_idr_update, cycle
//     u_k = om v + sum_{j>=k} c_j u_j                    k_idr_u
//     g_k = A u_k,  d_i = <p_i, g_k>                      k_apply<OP_P>
//     a_i = (d_i - sum_{j<i} a_j M[i][j]) / M[i][i], i < k      (finalize)
//     M[i][k] = d_i - sum_{j<k} a_j M[i][j], i >= k;  beta = f_k / M[k][k]
//     g_k -= sum_{j<k} a_j g_j;  u_k -= sum_{j<k} a_j u_j;
//     r -= beta g_k;  x += beta u_k;  f[k+1:] -= beta M[k+1:, k]   k_idr_update
//   reduction: v = K r; t = A v; om = <t, r> / <t, t> (enlarged to kappa when
//     |<t, r>| / (|t| |r|) < kappa); x += om v; r -= om t; f = <p_i, r>   k_idr_xr
//
// The a_i are the modified Gram-Schmidt coefficients of the published
// algorithm written as the forward substitution they amount to: with
// M[i][j] = <p_i, g_j> (j < i) already known, the inner products d_i of the
// new g_k with every p_i are all the algorithm needs, and they come fused into
// the operator apply instead of k - 1 more passes over g_k.
//
// The s x s algebra runs in one thread per right-hand side (k_idr_finalize).
// G and U hold s vectors per right-hand side, vector (j, r) at
// (j * rstride_j + r * n); the shadow vectors p_i are complex64, shared by all
// right-hand sides.  In the first cycle after a (re)start the g_j and u_j of
// the sums over j >= k are still zero and are not read.
#include "hh_common.h"
#include "hh_device.h"
#include "hh_kernels.h"
#include "hh_krylov.h"

namespace hh {

namespace {

__device__ __forceinline__ long long idr_row(int r, int row, long long nblk_max) {
    return part_index(r, 0, row, nblk_max);
}

// lower-triangular solve L y = b over rows/columns k .. s-1 of M (forward substitution)
__device__ void tri_solve(const IdrState& S, int k, const c128* b, c128* y) {
    for (int i = k; i < S.s; ++i) {
        c128 acc = b[i - k];
        for (int j = k; j < i; ++j) acc = acc - S.M[i][j] * y[j - k];
        y[i - k] = cdiv(acc, S.M[i][i]);
    }
}

__device__ __forceinline__ bool finite_c(c128 a) { return isfinite(a.re) && isfinite(a.im); }

}  // namespace

// v = r - sum_{j >= k} c_j g_j (start of a cycle: k = 0)
template <bool LOW>
__global__ __launch_bounds__(512) void k_idr_v(long long n, int k, const c128* __restrict__ G,
                                               long long rsj, const c128* __restrict__ rr,
                                               c128* __restrict__ v, c64* __restrict__ v_low,
                                               const IdrState* is, const RhsState* st) {
    const int r = blockIdx.z;
    if (st[r].status != ST_RUN) return;
    const IdrState& S = is[r];
    const int s = S.first ? 0 : S.s;  // first cycle: the g_j are zero
    // coefficient of g_j at index j (registers: every index below is a constant)
    c128 cj[IDR_SMAX];
#pragma unroll
    for (int j = 0; j < IDR_SMAX; ++j) cj[j] = j >= k && j < s ? S.c[j - k] : czero<double>();
    const long long off = (long long)r * n;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        c128 a = ld_stream(&rr[off + i]);
#pragma unroll
        for (int j = 0; j < IDR_SMAX; ++j)
            if (j >= k && j < s) a = a - cj[j] * ld_stream(&G[j * rsj + off + i]);
        if (LOW) st_stream(&v_low[off + i], cvt<float>(a));
        else st_stream(&v[off + i], a);
    }
}

// u_k = om v_hat + sum_{j >= k} c_j u_j  (in place: the j = k term reads u_k first)
template <typename TH>
__global__ __launch_bounds__(512) void k_idr_u(long long n, int k, c128* __restrict__ U, long long rsj,
                                               const cx<TH>* __restrict__ vh, const IdrState* is,
                                               const RhsState* st) {
    const int r = blockIdx.z;
    if (st[r].status != ST_RUN) return;
    const IdrState& S = is[r];
    const int s = S.first ? 0 : S.s;  // first cycle: the u_j are zero
    const c128 om = S.om;
    c128 cj[IDR_SMAX];
#pragma unroll
    for (int j = 0; j < IDR_SMAX; ++j) cj[j] = j >= k && j < s ? S.c[j - k] : czero<double>();
    const long long off = (long long)r * n;
    c128* uk = U + k * rsj + off;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        c128 a = om * cvt<double>(ld_stream(&vh[off + i]));
#pragma unroll
        for (int j = 0; j < IDR_SMAX; ++j)
            if (j >= k && j < s) a = a + cj[j] * ld_stream(&U[j * rsj + off + i]);
        st_stream(&uk[i], a);
    }
}

// Inner step k after g_k = A u_k and the finalize:
//   g_k -= sum_{j<k} a_j g_j;  u_k -= sum_{j<k} a_j u_j;  r -= beta g_k;  x += beta u_k;
//   partial ||r||^2 (row IDR_ROW_RN); the next preconditioner input
//   v = r - sum_{j>k} c_j g_j (next step's c), or v = r after the last step.
template <bool LOW>
__global__ __launch_bounds__(512) void k_idr_update(long long n, int k, c128* __restrict__ G,
                                                    c128* __restrict__ U, long long rsj,
                                                    c128* __restrict__ rr, c128* __restrict__ x,
                                                    c128* __restrict__ v, c64* __restrict__ v_low,
                                                    const IdrState* is, const RhsState* st,
                                                    double* __restrict__ part, long long nblk_max) {
    const int r = blockIdx.z;
    if (st[r].status != ST_RUN) return;
    const IdrState& S = is[r];
    const int sn = S.first ? 0 : S.s;  // first cycle: the g_j, j > k, are zero
    const c128 beta = S.beta;
    c128 a[IDR_SMAX], cn[IDR_SMAX];
#pragma unroll
    for (int j = 0; j < IDR_SMAX; ++j) {
        a[j] = j < k ? S.a[j] : czero<double>();
        cn[j] = j > k && j < sn ? S.c[j - k - 1] : czero<double>();  // next step's coefficient of g_j
    }
    const long long off = (long long)r * n;
    c128* gk = G + k * rsj + off;
    c128* uk = U + k * rsj + off;
    double acc[1] = {0.0};
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        c128 g = ld_stream(&gk[i]), u = ld_stream(&uk[i]);
#pragma unroll
        for (int j = 0; j < IDR_SMAX; ++j)
            if (j < k) {
                g = g - a[j] * ld_stream(&G[j * rsj + off + i]);
                u = u - a[j] * ld_stream(&U[j * rsj + off + i]);
            }
        st_stream(&gk[i], g);
        st_stream(&uk[i], u);
        const c128 rv = ld_stream(&rr[off + i]) - beta * g;
        st_stream(&rr[off + i], rv);
        st_stream(&x[off + i], ld_stream(&x[off + i]) + beta * u);
        acc[0] += abs2(rv);
        c128 nv = rv;
#pragma unroll
        for (int j = 0; j < IDR_SMAX; ++j)
            if (j > k && j < sn) nv = nv - cn[j] * ld_stream(&G[j * rsj + off + i]);
        if (LOW) st_stream(&v_low[off + i], cvt<float>(nv));
        else st_stream(&v[off + i], nv);
    }
    block_sum_store<1>(acc, part + idr_row(r, IDR_ROW_RN, nblk_max) + blockIdx.x, nblk_max);
}

// Reduction step after t = A v_hat and the finalize: x += om v_hat; r -= om t;
// partials <p_i, r> (rows 0 .. 2s - 1) and ||r||^2 (row IDR_ROW_RN).
template <typename TH, int NS>
__global__ __launch_bounds__(512) void k_idr_xr(long long n, c128* __restrict__ x, c128* __restrict__ rr,
                                                const cx<TH>* __restrict__ vh, const c128* __restrict__ t,
                                                const c64* __restrict__ P, const IdrState* is,
                                                const RhsState* st, double* __restrict__ part,
                                                long long nblk_max) {
    const int r = blockIdx.z;
    if (st[r].status != ST_RUN) return;
    const c128 om = is[r].om;
    const long long off = (long long)r * n;
    double acc[2 * NS], rn[1] = {0.0};
#pragma unroll
    for (int q = 0; q < 2 * NS; ++q) acc[q] = 0.0;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        st_stream(&x[off + i], ld_stream(&x[off + i]) + om * cvt<double>(ld_stream(&vh[off + i])));
        const c128 rv = ld_stream(&rr[off + i]) - om * ld_stream(&t[off + i]);
        st_stream(&rr[off + i], rv);
#pragma unroll
        for (int q = 0; q < NS; ++q) {
            const c128 d = cdot(cvt<double>(ld_stream(&P[q * n + i])), rv);
            acc[2 * q] += d.re;
            acc[2 * q + 1] += d.im;
        }
        rn[0] += abs2(rv);
    }
    block_sum_store<2 * NS>(acc, part + idr_row(r, 0, nblk_max) + blockIdx.x, nblk_max);
    block_sum_store<1>(rn, part + idr_row(r, IDR_ROW_RN, nblk_max) + blockIdx.x, nblk_max);
}

// <p_i, r> and ||r||^2 of the current residual (start and restarts)
template <int NS>
__global__ __launch_bounds__(512) void k_idr_pr(long long n, const c128* __restrict__ rr,
                                                const c64* __restrict__ P, const RhsState* st,
                                                double* __restrict__ part, long long nblk_max) {
    const int r = blockIdx.z;
    if (st[r].status != ST_RUN) return;
    const long long off = (long long)r * n;
    double acc[2 * NS], rn[1] = {0.0};
#pragma unroll
    for (int q = 0; q < 2 * NS; ++q) acc[q] = 0.0;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const c128 rv = rr[off + i];
#pragma unroll
        for (int q = 0; q < NS; ++q) {
            const c128 d = cdot(cvt<double>(P[q * n + i]), rv);
            acc[2 * q] += d.re;
            acc[2 * q + 1] += d.im;
        }
        rn[0] += abs2(rv);
    }
    block_sum_store<2 * NS>(acc, part + idr_row(r, 0, nblk_max) + blockIdx.x, nblk_max);
    block_sum_store<1>(rn, part + idr_row(r, IDR_ROW_RN, nblk_max) + blockIdx.x, nblk_max);
}

// Shadow vectors from a counter-based generator: entry (i, node) takes the
// real and imaginary parts from SplitMix64 (Steele, Lea and Flood, OOPSLA 2014)
// of the counters seed * 2^40 + 2 (i n + node) and the next one, mapped to
// [-1, 1) through the top 53 bits.
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
__global__ void k_idr_gen_p(long long n, int s, unsigned long long seed, c64* __restrict__ P) {
    const long long total = (long long)s * n;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const unsigned long long ctr = (seed << 40) + 2ull * (unsigned long long)e;
        const double re = (double)(splitmix64(ctr) >> 11) * 0x1.0p-52 - 1.0;
        const double im = (double)(splitmix64(ctr + 1) >> 11) * 0x1.0p-52 - 1.0;
        P[e] = c64{(float)re, (float)im};
    }
}

// caller's shadow vectors (complex128) rounded to complex64
__global__ void k_idr_set_p(long long total, const c128* __restrict__ src, c64* __restrict__ P) {
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x)
        P[e] = cvt<float>(src[e]);
}

// Scalar part of the IDR cycle, one workgroup per right-hand side (sums in a
// fixed order, one thread does the algebra).
//   IDR_FIN_START (reset: M = I, om = 1, first cycle): f = <p_i, r>, stop test
//       on ||r||, c = M^-1 f for inner step 0.
//   IDR_FIN_STEP k: stop test on the ||r|| of step k - 1 (k > 0); then a_i,
//       column k of M, beta, f update and the next step's c.
//   IDR_FIN_OMEGA: stop test on the ||r|| of step s - 1; om from t^H r, t^H t.
template <int NT>
__device__ __forceinline__ void sum_rows(const double* part, long long nblk, long long nblk_max, double* out) {
    double o[NT];
    block_fixed_sum<NT>(part, nblk, nblk_max, o);
#pragma unroll
    for (int t = 0; t < NT; ++t) out[t] = o[t];
}

__device__ void sum_dots(int s, const double* part, long long nblk, long long nblk_max, double* out) {
    switch (s) {
        case 1: sum_rows<2>(part, nblk, nblk_max, out); break;
        case 2: sum_rows<4>(part, nblk, nblk_max, out); break;
        case 3: sum_rows<6>(part, nblk, nblk_max, out); break;
        case 4: sum_rows<8>(part, nblk, nblk_max, out); break;
        case 5: sum_rows<10>(part, nblk, nblk_max, out); break;
        case 6: sum_rows<12>(part, nblk, nblk_max, out); break;
        case 7: sum_rows<14>(part, nblk, nblk_max, out); break;
        default: sum_rows<16>(part, nblk, nblk_max, out); break;
    }
}

// The state is staged in LDS for the one-thread algebra (a chain of dependent
// global loads and stores would cost far more than the arithmetic) and
// written back by all lanes.
constexpr int IDR_STATE_WORDS = sizeof(IdrState) / sizeof(double);
static_assert(sizeof(IdrState) % sizeof(double) == 0, "IdrState is copied as doubles");

__device__ void idr_fin_algebra(int mode, int k, int reset, int s, double kappa, RhsState& R, IdrState& S,
                                const double* d, double rn2, const double* tsum);

__global__ __launch_bounds__(1024) void k_idr_finalize(int mode, int k, int reset, int s, double kappa,
                                                       RhsState* st, IdrState* is, const double* part,
                                                       long long nblk, long long nblk_max) {
    const int r = blockIdx.x;
    if (st[r].status != ST_RUN) return;
    __shared__ IdrState sS;
    __shared__ RhsState sR;
    {
        const double* src = reinterpret_cast<const double*>(&is[r]);
        double* dst = reinterpret_cast<double*>(&sS);
        for (int w = threadIdx.x; w < IDR_STATE_WORDS; w += blockDim.x) dst[w] = src[w];
        if (threadIdx.x == 0) sR = st[r];
    }
    double d[2 * IDR_SMAX] = {};
    double rn2 = 0.0, tsum[3] = {0.0, 0.0, 0.0};
    if (mode != IDR_FIN_OMEGA) sum_dots(s, part + idr_row(r, 0, nblk_max), nblk, nblk_max, d);
    else sum_rows<3>(part + part_index(r, SLOT_T, 0, nblk_max), nblk, nblk_max, tsum);
    __syncthreads();
    {
        double o[1];
        block_fixed_sum<1>(part + idr_row(r, IDR_ROW_RN, nblk_max), nblk, nblk_max, o);
        rn2 = o[0];
    }
    __syncthreads();
    if (threadIdx.x == 0) idr_fin_algebra(mode, k, reset, s, kappa, sR, sS, d, rn2, tsum);
    __syncthreads();
    {
        const double* src = reinterpret_cast<const double*>(&sS);
        double* dst = reinterpret_cast<double*>(&is[r]);
        for (int w = threadIdx.x; w < IDR_STATE_WORDS; w += blockDim.x) dst[w] = src[w];
        if (threadIdx.x == 0) st[r] = sR;
    }
}

__device__ void idr_fin_algebra(int mode, int k, int reset, int s, double kappa, RhsState& R, IdrState& S,
                                const double* d, double rn2, const double* tsum) {
    const double tiny = 1e-300;
    // stop test on the residual of the previous update (none before step 0)
    if (mode != IDR_FIN_STEP || k > 0) {
        if (!isfinite(rn2)) { R.status = ST_NUMERIC; return; }
        R.rnorm2 = rn2;
        if (rn2 <= R.tol2) { R.status = ST_CONV; return; }
        if (R.iters2 >= R.maxit2) { R.status = ST_MAXIT; return; }
    }
    if (mode == IDR_FIN_START) {
        if (reset) {
            for (int i = 0; i < IDR_SMAX; ++i)
                for (int j = 0; j < IDR_SMAX; ++j) S.M[i][j] = mk(i == j ? 1.0 : 0.0, 0.0);
            S.om = mk(1.0, 0.0);
            S.first = 1;
            S.s = s;
            S.kappa = kappa;
        }
        for (int i = 0; i < s; ++i) {
            S.f[i] = mk(d[2 * i], d[2 * i + 1]);
            if (!finite_c(S.f[i])) { R.status = ST_NUMERIC; return; }
        }
        tri_solve(S, 0, S.f, S.c);
        return;
    }
    if (mode == IDR_FIN_STEP) {
        R.matvecs += 1;
        R.iters2 += 2;
        c128 dk[IDR_SMAX];
        for (int i = 0; i < s; ++i) {
            dk[i] = mk(d[2 * i], d[2 * i + 1]);
            if (!finite_c(dk[i])) { R.status = ST_NUMERIC; return; }
        }
        for (int i = 0; i < k; ++i) {
            c128 acc = dk[i];
            for (int j = 0; j < i; ++j) acc = acc - S.a[j] * S.M[i][j];
            S.a[i] = cdiv(acc, S.M[i][i]);
        }
        for (int i = k; i < s; ++i) {
            c128 acc = dk[i];
            for (int j = 0; j < k; ++j) acc = acc - S.a[j] * S.M[i][j];
            S.M[i][k] = acc;
        }
        if (abs2(S.M[k][k]) <= tiny * tiny) { R.status = ST_BREAK; return; }
        S.beta = cdiv(S.f[k], S.M[k][k]);
        for (int i = k + 1; i < s; ++i) S.f[i] = S.f[i] - S.beta * S.M[i][k];
        if (k + 1 < s) tri_solve(S, k + 1, S.f + (k + 1), S.c);
        return;
    }
    // IDR_FIN_OMEGA
    R.matvecs += 1;
    R.iters2 += 2;
    const c128 tr = mk(tsum[0], tsum[1]);
    const double tt = tsum[2];
    if (!finite_c(tr) || !isfinite(tt)) { R.status = ST_NUMERIC; return; }
    if (tt == 0.0) { R.status = ST_BREAK; return; }
    c128 om = mk(tr.re / tt, tr.im / tt);
    const double rho = sqrt(abs2(tr)) / (sqrt(tt) * sqrt(rn2));
    if (rho < S.kappa) om = (S.kappa / rho) * om;
    if (abs2(om) <= tiny * tiny) { R.status = ST_BREAK; return; }
    S.om = om;
    S.first = 0;
}

// ---------------------------------------------------------------------------
// launchers (flat kernels: exactly L.flat_cap workgroups per right-hand side)
// ---------------------------------------------------------------------------
void launch_idr_v(hipStream_t s, long long n, int nrhs, int k, const c128* G, long long rsj, const c128* r,
                  c128* v, c64* v_low, const IdrState* is, const RhsState* st, const Launch& L) {
    const dim3 grid(L.flat_cap, 1, nrhs);
    if (v_low) hipLaunchKernelGGL(k_idr_v<true>, grid, dim3(L.block), 0, s, n, k, G, rsj, r, v, v_low, is, st);
    else hipLaunchKernelGGL(k_idr_v<false>, grid, dim3(L.block), 0, s, n, k, G, rsj, r, v, v_low, is, st);
}

template <typename TH>
void launch_idr_u(hipStream_t s, long long n, int nrhs, int k, c128* U, long long rsj, const cx<TH>* vh,
                  const IdrState* is, const RhsState* st, const Launch& L) {
    hipLaunchKernelGGL(k_idr_u<TH>, dim3(L.flat_cap, 1, nrhs), dim3(L.block), 0, s, n, k, U, rsj, vh, is, st);
}
template void launch_idr_u<double>(hipStream_t, long long, int, int, c128*, long long, const c128*,
                                   const IdrState*, const RhsState*, const Launch&);
template void launch_idr_u<float>(hipStream_t, long long, int, int, c128*, long long, const c64*,
                                  const IdrState*, const RhsState*, const Launch&);

void launch_idr_update(hipStream_t s, long long n, int nrhs, int k, c128* G, c128* U, long long rsj, c128* r,
                       c128* x, c128* v, c64* v_low, const IdrState* is, const RhsState* st, double* part,
                       long long nblk_max, const Launch& L) {
    const dim3 grid(L.flat_cap, 1, nrhs);
    if (v_low)
        hipLaunchKernelGGL(k_idr_update<true>, grid, dim3(L.block), 0, s, n, k, G, U, rsj, r, x, v, v_low, is,
                           st, part, nblk_max);
    else
        hipLaunchKernelGGL(k_idr_update<false>, grid, dim3(L.block), 0, s, n, k, G, U, rsj, r, x, v, v_low,
                           is, st, part, nblk_max);
}

#define HH_IDR_NS_SWITCH(ns, MACRO) \
    switch (ns) {                   \
        case 1: MACRO(1); break;    \
        case 2: MACRO(2); break;    \
        case 3: MACRO(3); break;    \
        case 4: MACRO(4); break;    \
        case 5: MACRO(5); break;    \
        case 6: MACRO(6); break;    \
        case 7: MACRO(7); break;    \
        default: MACRO(8); break;   \
    }

template <typename TH>
void launch_idr_xr(hipStream_t s, long long n, int nrhs, int ns, c128* x, c128* r, const cx<TH>* vh,
                   const c128* t, const c64* P, const IdrState* is, const RhsState* st, double* part,
                   long long nblk_max, const Launch& L) {
    const dim3 grid(L.flat_cap, 1, nrhs);
#define HH_XR(NSV)                                                                                        \
    hipLaunchKernelGGL((k_idr_xr<TH, NSV>), grid, dim3(L.block), 0, s, n, x, r, vh, t, P, is, st, part, \
                       nblk_max)
    HH_IDR_NS_SWITCH(ns, HH_XR)
#undef HH_XR
}
template void launch_idr_xr<double>(hipStream_t, long long, int, int, c128*, c128*, const c128*, const c128*,
                                    const c64*, const IdrState*, const RhsState*, double*, long long,
                                    const Launch&);
template void launch_idr_xr<float>(hipStream_t, long long, int, int, c128*, c128*, const c64*, const c128*,
                                   const c64*, const IdrState*, const RhsState*, double*, long long,
                                   const Launch&);

void launch_idr_pr(hipStream_t s, long long n, int nrhs, int ns, const c128* r, const c64* P,
                   const RhsState* st, double* part, long long nblk_max, const Launch& L) {
    const dim3 grid(L.flat_cap, 1, nrhs);
#define HH_PR(NSV) hipLaunchKernelGGL((k_idr_pr<NSV>), grid, dim3(L.block), 0, s, n, r, P, st, part, nblk_max)
    HH_IDR_NS_SWITCH(ns, HH_PR)
#undef HH_PR
}
#undef HH_IDR_NS_SWITCH

void launch_idr_finalize(hipStream_t s, int mode, int k, int reset, int nrhs, int ns, double kappa,
                         RhsState* st, IdrState* is, const double* part, long long nblk, long long nblk_max) {
    hipLaunchKernelGGL(k_idr_finalize, dim3(nrhs), dim3(1024), 0, s, mode, k, reset, ns, kappa, st, is, part,
                       nblk, nblk_max);
}

void launch_idr_gen_p(hipStream_t s, long long n, int ns, unsigned long long seed, c64* P) {
    hipLaunchKernelGGL(k_idr_gen_p, dim3(2048), dim3(256), 0, s, n, ns, seed, P);
}
void launch_idr_set_p(hipStream_t s, long long total, const c128* src, c64* P) {
    hipLaunchKernelGGL(k_idr_set_p, dim3(2048), dim3(256), 0, s, total, src, P);
}

}  // namespace hh
