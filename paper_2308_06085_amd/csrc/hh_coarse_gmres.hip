// The paper's coarsest-grid solve: full GMRES on the rediscretised coarsest
// CSLP operator M_c, without preconditioner, from a zero initial guess, until
// the relative residual ||b - M_c e|| / ||b|| reaches 1e-11 (paper, end of
// section 3.4.5 and section 4.2: the coarsest problem is solved iteratively by
// GMRES; section 5: tolerance 1e-11 for the coarse solve).
//
// One workgroup of 1024 lanes per right-hand side runs the whole solve in one
// launch, so the V-cycle stays one captured graph.  Each lane owns the nodes
// t, t + 1024, ... of the coarse grid (up to 8192 nodes).  The basis V (up to
// m complex128 vectors), the vector w being orthogonalised and the iterate x
// lie in device memory, which the workgroup reads through the caches; the
// rotated Hessenberg matrix, the Givens rotations and g are in LDS.
// Arnoldi step j:
//   w = M_c v_j                       (7-point stencil, mirrored neighbours at
//                                      Sommerfeld faces, zero Dirichlet nodes)
//   classical Gram-Schmidt, two sweeps: h = V^H w (wavefront butterfly
//   partials, summed in wavefront order), w -= V h
//   h_{j+1,j} = ||w||, v_{j+1} = w / h_{j+1,j}
//   earlier rotations on the column, a new one zeroing h_{j+1,j}, g updated
//   stop when |g_{j+1}| / ||b|| <= tol
// then y = R^-1 g (back substitution by one wavefront) and x += V y.  If the m
// steps of a cycle end without meeting tol, GMRES restarts from x (at most
// `cycles` cycles).  Every sum has a fixed order, so results are bitwise
// repeatable and independent of the number of right-hand sides.
#include "hh_coarse.h"
#include "hh_device.h"

namespace hh {

namespace {

constexpr int CG_LANES = 1024;
constexpr int CG_WAVES = CG_LANES / 64;

__device__ __forceinline__ c128 wave_sum(c128 v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        v.re += __shfl_xor(v.re, off, 64);
        v.im += __shfl_xor(v.im, off, 64);
    }
    return v;
}

// y = M_c x at node i (x: a full coarse vector in device memory)
template <int BC>
__device__ __forceinline__ c128 coarse_apply(const CoarseGmres& D, const c128* __restrict__ x, int i) {
    const Geo& g = D.g;
    const int z = i / g.plane, rem = i - z * g.plane;
    const int y = rem / g.nx, xx = rem - y * g.nx;
    const int nf = (xx == 0) + (xx == g.nx - 1) + (y == 0) + (y == g.ny - 1) + (z == 0) + (z == g.nz - 1);
    if (BC == BC_DIRICHLET && nf) return czero<double>();
    const c128 u = x[i];
    const int xm = mirror_clamp(xx - 1, g.nx), xp = mirror_clamp(xx + 1, g.nx);
    const int ym = mirror_clamp(y - 1, g.ny), yp = mirror_clamp(y + 1, g.ny);
    const int zm = mirror_clamp(z - 1, g.nz), zp = mirror_clamp(z + 1, g.nz);
    const int row = z * g.plane + y * g.nx;
    c128 lap = (u - x[row + xm]) + (u - x[row + xp]);
    lap = lap + (u - x[z * g.plane + ym * g.nx + xx]);
    lap = lap + (u - x[z * g.plane + yp * g.nx + xx]);
    lap = lap + (u - x[zm * g.plane + y * g.nx + xx]);
    lap = lap + (u - x[zp * g.plane + y * g.nx + xx]);
    const double kk = D.k[i];
    c128 c = {D.sr * kk * kk, D.si * kk * kk};
    if (BC == BC_SOMMERFELD) c.im += (double)nf * D.two_over_h * kk;
    return D.ih2 * lap - c * u;
}

template <int BC, typename TB>
__global__ __launch_bounds__(CG_LANES) void k_coarse_gmres(CoarseGmres D, const cx<TB>* __restrict__ b,
                                                           cx<TB>* __restrict__ e, const RhsState* st,
                                                           int gate) {
    extern __shared__ c128 lds[];
    __shared__ double s_part[CG_WAVES];
    __shared__ int s_flag;
    const int r = blockIdx.x;
    if (!gate_ok(st, r, gate)) return;
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    const int n = (int)D.g.n, m = D.m;
    c128* red = lds;                      // (m + 1) x CG_WAVES partial inner products
    c128* hs = red + (m + 1) * CG_WAVES;  // m + 1: one sweep's coefficients
    c128* hc = hs + (m + 1);              // m + 2: the current column
    c128* Rm = hc + (m + 2);              // rotated columns, column j at j (j + 1) / 2
    c128* gv = Rm + m * (m + 1) / 2;      // m + 1
    c128* cs = gv + (m + 1);              // m (real cosines, stored complex)
    c128* sn = cs + m;                    // m
    c128* yv = sn + m;                    // m
    // slots 0 .. m - 1: basis vectors; slot j + 1 holds w during step j;
    // slot m + 1: the iterate x.  Each lane reads and writes its own nodes of
    // w and x; the stencil reads neighbours of v_j, complete at a barrier.
    c128* V = D.V + (long long)r * (m + 2) * n;
    c128* X = V + (long long)(m + 1) * n;
    const cx<TB>* br = b + (long long)r * n;
    cx<TB>* er = e + (long long)r * n;

    auto boundary = [&](int i) {
        const int z = i / D.g.plane, rem = i - z * D.g.plane;
        const int y = rem / D.g.nx, xx = rem - y * D.g.nx;
        return xx == 0 || xx == D.g.nx - 1 || y == 0 || y == D.g.ny - 1 || z == 0 || z == D.g.nz - 1;
    };
    // sum over the workgroup of one double per lane, in a fixed order
    auto block_sum = [&](double v) -> double {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) s_part[wid] = v;
        __syncthreads();
        double s = 0.0;
        for (int w = 0; w < CG_WAVES; ++w) s += s_part[w];
        __syncthreads();  // s_part is reused by the next call
        return s;
    };
    // one classical Gram-Schmidt sweep of w against v_0 .. v_j:
    // hs = V^H w (four basis vectors per pass over w; every inner product is
    // summed over a lane's nodes in order, then by wavefront butterfly, then
    // over the wavefronts in order), then w -= V hs
    auto sweep = [&](c128* w, int j) {
        constexpr int CH = 4;
        for (int i0 = 0; i0 <= j; i0 += CH) {
            c128 acc[CH];
#pragma unroll
            for (int c = 0; c < CH; ++c) acc[c] = czero<double>();
            for (int nd = t; nd < n; nd += CG_LANES) {
                const c128 wn = w[nd];
#pragma unroll
                for (int c = 0; c < CH; ++c)
                    if (i0 + c <= j) acc[c] = acc[c] + cdot(V[(long long)(i0 + c) * n + nd], wn);
            }
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                if (i0 + c > j) break;
                const c128 p = wave_sum(acc[c]);
                if (lane == 0) red[(i0 + c) * CG_WAVES + wid] = p;
            }
        }
        __syncthreads();
        for (int i = t; i <= j; i += CG_LANES) {
            c128 sum = czero<double>();
            for (int w2 = 0; w2 < CG_WAVES; ++w2) sum = sum + red[i * CG_WAVES + w2];
            hs[i] = sum;
        }
        __syncthreads();
        for (int nd = t; nd < n; nd += CG_LANES) {
            c128 wn = w[nd];
            for (int i = 0; i <= j; ++i) wn = wn - hs[i] * V[(long long)i * n + nd];
            w[nd] = wn;
        }
    };

    // start: x = 0, v_0 = b (Dirichlet boundary nodes 0), scaled below
    double nb = 0.0;
    for (int nd = t; nd < n; nd += CG_LANES) {
        X[nd] = czero<double>();
        const c128 v = (BC == BC_DIRICHLET && boundary(nd)) ? czero<double>() : cvt<double>(br[nd]);
        V[nd] = v;
        nb += abs2(v);
    }
    const double bnorm = sqrt(block_sum(nb));
    int steps = 0;
    if (bnorm > 0.0) {
        double beta = bnorm;  // residual norm at the start of the cycle
        for (int cycle = 0; cycle < D.cycles; ++cycle) {
            // v_0 = r / beta (r in slot 0), g = beta e_1
            const double ib = 1.0 / beta;
            for (int nd = t; nd < n; nd += CG_LANES) V[nd] = ib * V[nd];
            if (t == 0) gv[0] = mk(beta, 0.0);
            __syncthreads();
            int used = 0;
            bool done = false;
            for (int j = 0; j < m; ++j) {
                const c128* vj = V + (long long)j * n;
                c128* w = V + (long long)(j + 1) * n;
                for (int nd = t; nd < n; nd += CG_LANES) w[nd] = coarse_apply<BC>(D, vj, nd);
                sweep(w, j);
                for (int i = t; i <= j; i += CG_LANES) hc[i] = hs[i];
                __syncthreads();
                sweep(w, j);
                double nw = 0.0;
                for (int nd = t; nd < n; nd += CG_LANES) nw += abs2(w[nd]);
                for (int i = t; i <= j; i += CG_LANES) hc[i] = hc[i] + hs[i];
                const double hn = sqrt(block_sum(nw));
                if (t == 0) {
                    // the earlier rotations on column j, then the one zeroing h_{j+1,j}
                    for (int i = 0; i < j; ++i) {
                        const c128 a0 = hc[i], a1 = hc[i + 1];
                        hc[i] = cs[i] * a0 + sn[i] * a1;
                        hc[i + 1] = cs[i] * a1 - conj(sn[i]) * a0;  // cs real: conj(cs) = cs
                    }
                    const c128 a = hc[j];
                    const double aa = sqrt(abs2(a));
                    const double den = sqrt(aa * aa + hn * hn);
                    int flag = 0;
                    if (den == 0.0 || !isfinite(den)) {
                        flag = 2;  // breakdown: keep the steps before this one
                    } else {
                        const double c0 = aa / den;
                        const c128 s0 = aa != 0.0 ? (1.0 / (aa * den)) * (a * mk(hn, 0.0)) : mk(1.0, 0.0);
                        cs[j] = mk(c0, 0.0);
                        sn[j] = s0;
                        hc[j] = c0 * a + s0 * mk(hn, 0.0);
                        const c128 gj = gv[j];
                        gv[j + 1] = mk(-1.0, 0.0) * (conj(s0) * gj);
                        gv[j] = c0 * gj;
                        for (int i = 0; i <= j; ++i) Rm[j * (j + 1) / 2 + i] = hc[i];
                        if (sqrt(abs2(gv[j + 1])) <= D.tol * bnorm || hn == 0.0) flag = 1;
                    }
                    s_flag = flag;
                }
                __syncthreads();
                const int flag = s_flag;
                if (flag == 2) {
                    done = true;
                    break;
                }
                used = j + 1;
                ++steps;
                if (flag == 1) {
                    done = true;
                    break;
                }
                if (j + 1 < m) {
                    // v_{j+1} = w / h_{j+1,j}, in place
                    const double inv = 1.0 / hn;
                    for (int nd = t; nd < n; nd += CG_LANES) w[nd] = inv * w[nd];
                    __syncthreads();
                }
            }
            // y = R^-1 g by wavefront 0 (lane l holds g_l and g_{l+64}), then x += V y
            if (wid == 0) {
                c128 g0 = lane < used ? gv[lane] : czero<double>();
                c128 g1 = lane + 64 < used ? gv[lane + 64] : czero<double>();
                for (int k = used - 1; k >= 0; --k) {
                    const c128 gk = k < 64 ? mk(__shfl(g0.re, k, 64), __shfl(g0.im, k, 64))
                                           : mk(__shfl(g1.re, k - 64, 64), __shfl(g1.im, k - 64, 64));
                    const c128 yk = cdiv(gk, Rm[k * (k + 1) / 2 + k]);
                    if (lane == 0) yv[k] = yk;
                    if (lane < k) g0 = g0 - Rm[k * (k + 1) / 2 + lane] * yk;
                    if (lane + 64 < k) g1 = g1 - Rm[k * (k + 1) / 2 + lane + 64] * yk;
                }
            }
            __syncthreads();
            for (int nd = t; nd < n; nd += CG_LANES) {
                c128 xv = X[nd];
                for (int i = 0; i < used; ++i) xv = xv + yv[i] * V[(long long)i * n + nd];
                X[nd] = xv;
            }
            if (done || cycle + 1 == D.cycles) break;
            // restart from x: slot 0 = b - M_c x
            __syncthreads();
            double nr = 0.0;
            for (int nd = t; nd < n; nd += CG_LANES) {
                c128 v = czero<double>();
                if (!(BC == BC_DIRICHLET && boundary(nd))) v = cvt<double>(br[nd]) - coarse_apply<BC>(D, X, nd);
                V[nd] = v;
                nr += abs2(v);
            }
            beta = sqrt(block_sum(nr));
            if (!(beta > D.tol * bnorm)) break;
        }
    }
    for (int nd = t; nd < n; nd += CG_LANES) er[nd] = cvt<TB>(X[nd]);
    if (t == 0 && D.steps) D.steps[r] = steps;
}

}  // namespace

size_t coarse_gmres_lds_bytes(int m) {
    const size_t words = (size_t)(m + 1) * CG_WAVES + (m + 1) + (m + 2) + (size_t)m * (m + 1) / 2 + (m + 1) +
                         3 * (size_t)m;
    return words * sizeof(c128);
}

bool coarse_gmres_allow_lds(size_t bytes) {
    const int v = (int)bytes;
    return hipFuncSetAttribute((const void*)k_coarse_gmres<BC_SOMMERFELD, double>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, v) == hipSuccess &&
           hipFuncSetAttribute((const void*)k_coarse_gmres<BC_DIRICHLET, double>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, v) == hipSuccess &&
           hipFuncSetAttribute((const void*)k_coarse_gmres<BC_SOMMERFELD, float>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, v) == hipSuccess &&
           hipFuncSetAttribute((const void*)k_coarse_gmres<BC_DIRICHLET, float>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, v) == hipSuccess;
}

template <typename R>
void launch_coarse_gmres(hipStream_t s, int bc, const CoarseGmres& D, const cx<R>* b, cx<R>* e, int nrhs,
                         const RhsState* st, int gate) {
    const size_t lds = coarse_gmres_lds_bytes(D.m);
    if (bc == BC_SOMMERFELD)
        hipLaunchKernelGGL((k_coarse_gmres<BC_SOMMERFELD, R>), dim3(nrhs), dim3(CG_LANES), lds, s, D, b, e, st,
                           gate);
    else
        hipLaunchKernelGGL((k_coarse_gmres<BC_DIRICHLET, R>), dim3(nrhs), dim3(CG_LANES), lds, s, D, b, e, st,
                           gate);
}
template void launch_coarse_gmres<double>(hipStream_t, int, const CoarseGmres&, const c128*, c128*, int,
                                          const RhsState*, int);
template void launch_coarse_gmres<float>(hipStream_t, int, const CoarseGmres&, const c64*, c64*, int,
                                         const RhsState*, int);

}  // namespace hh
