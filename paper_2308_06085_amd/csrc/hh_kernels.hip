// gfx950 kernels of the matrix-free CSLP / multigrid / Bi-CGSTAB Helmholtz solver.
//
// Launch shape of the fine-grid operator kernels (apply, start residual): a
// workgroup owns an x-y tile of at most AP_LANES nodes, one per lane, and
// marches along z over `zb` planes; the apply stages the tile and its
// one-node halo in LDS (a ring of three planes).  gridDim = (tiles, z chunks,
// right-hand sides).  The Krylov vector kernels are flat grid-stride loops
// with the same workgroup count.
//
// The operator (paper section 2.4, eq. Helmstencil; Algorithm 2):
//   (A x)_j = D_j x_j - (1/h^2) sum'_nb x_nb,
//   D_j = 6/h^2 - sigma k_j^2 - n_j 2 i k_j / h,
// where sum' replaces a neighbour outside the domain by its mirror image
// (Sommerfeld ghost elimination, eq. elimination, applied independently per
// axis) or by 0 (Dirichlet), n_j is the number of faces node j lies on
// (Sommerfeld only) and sigma = 1 for A, beta1 - beta2 i for the CSLP M
// (section 3.3).
//
// The multigrid passes are in hh_mg_fused.hip; this file holds the operator
// apply, the coarsest-grid solve, the Krylov vector updates, the reductions and
// the set-up kernels.
#include "hh_common.h"
#include "hh_device.h"
#include "hh_kernels.h"

namespace hh {

// Workgroup and lane position in the operator kernels' tiling
// (ap_tile_shape(); gridDim = (tiles, z chunks, right-hand sides)).  The
// XCD-aware map keeps neighbouring tiles, which share halo nodes, on one XCD
// and so in one L2.
struct ApPos {
    int X0, Y0;   // origin of the workgroup's tile
    int z0, z1;   // its z-planes [z0, z1)
    int ox, oy;   // this lane's node in the tile
    int i, j;     // its x, y; column (0, 0) for a lane without a node
    bool own;     // the lane owns a node of the grid
};
__device__ __forceinline__ ApPos ap_pos(const Geo& g, const TileShape& T, int zb) {
    ApPos q;
    const int id = xcd_tile_id(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
    const int bz = id / (int)gridDim.x, tile = id - bz * (int)gridDim.x;
    const int tyi = tile / T.ntx, txi = tile - tyi * T.ntx;
    q.X0 = txi * T.tw;
    q.Y0 = tyi * T.th;
    q.z0 = bz * zb;
    q.z1 = min(g.nz, q.z0 + zb);
    q.oy = (int)threadIdx.x / T.tw;
    q.ox = (int)threadIdx.x - q.oy * T.tw;
    const int gx = q.X0 + q.ox, gy = q.Y0 + q.oy;
    q.own = q.oy < T.th && gx < g.nx && gy < g.ny;
    q.i = q.own ? gx : 0;
    q.j = q.own ? gy : 0;
    return q;
}

// Neighbour sum with the boundary rule of the level.  `ld(i, j)` returns the
// value at in-plane position (i, j) of the current plane; zm / zp are the
// column's values on the planes below / above (already mirrored or zeroed).
template <int BC, typename R, typename LD>
__device__ __forceinline__ cx<R> inplane_sum(const LD& ld, int i, int j, int nx, int ny) {
    cx<R> s;
    if (BC == BC_SOMMERFELD) {
        int im = i > 0 ? i - 1 : 1;
        int ip = i < nx - 1 ? i + 1 : nx - 2;
        int jm = j > 0 ? j - 1 : 1;
        int jp = j < ny - 1 ? j + 1 : ny - 2;
        s = ld(im, j) + ld(ip, j);
        s = s + ld(i, jm);
        s = s + ld(i, jp);
    } else {
        s = czero<R>();
        if (i > 1) s = s + ld(i - 1, j);
        if (i < nx - 2) s = s + ld(i + 1, j);
        if (j > 1) s = s + ld(i, j - 1);
        if (j < ny - 2) s = s + ld(i, j + 1);
    }
    return s;
}

__device__ __forceinline__ int faces(int i, int j, int z, int nx, int ny, int nz) {
    return (i == 0) + (i == nx - 1) + (j == 0) + (j == ny - 1) + (z == 0) + (z == nz - 1);
}

__device__ __forceinline__ bool on_boundary(int i, int j, int z, int nx, int ny, int nz) {
    return i == 0 || j == 0 || z == 0 || i == nx - 1 || j == ny - 1 || z == nz - 1;
}

// ---------------------------------------------------------------------------
// Reductions and the Bi-CGSTAB scalar recurrences.
//
// Every reduction-producing kernel writes one partial sum per workgroup.  The
// partials of a slot are added in a fixed order (lane t takes partials t,
// t + blockDim, ...; then a fixed butterfly) by the one-workgroup-per-RHS
// kernel k_finalize, which then does the scalar update, so a solve is bitwise
// repeatable.  (Finishing the sum in the last workgroup of the producing kernel
// would need a device-scope fence per workgroup, which on a multi-XCD device
// writes back the XCD's L2 and costs more than the extra launch.)
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool finite2(c128 a) { return isfinite(a.re) && isfinite(a.im); }

// Scalar update of one right-hand side from the slot sums (one thread).
__device__ void fin_update(int mode, RhsState& S, const double* s, double tol) {
    const double tiny = 1e-300;
    const int status = S.status;
    switch (mode) {
        case FIN_INIT:
        case FIN_INIT_DECADE:
            S.bnorm2 = s[3];
            S.rnorm2 = s[0];
            S.rhat_norm2 = s[0];
            S.tol2 = tol * tol * s[3];
            S.rho = mk(1.0, 0.0);
            S.alpha = mk(1.0, 0.0);
            S.omega = mk(1.0, 0.0);
            S.beta = mk(0.0, 0.0);
            S.iters2 = 0;
            S.matvecs = 1;
            S.restarts = 0;
            S.true_rnorm2 = 0.0;
            S.pend = 0;
            S.decades = 0;
            // the first restart when ||r|| / ||b|| < 0.1, then below 0.01, ...
            S.next2 = 0.0;
            if (mode == FIN_INIT_DECADE) {
                S.next2 = 0.01 * s[3];
                while (S.next2 > 0.0 && S.next2 >= s[0]) S.next2 *= 0.01;
            }
            if (!isfinite(s[0]) || !isfinite(s[3])) S.status = ST_NUMERIC;
            else if (s[3] == 0.0 || s[0] <= S.tol2) S.status = ST_CONV;
            return;
        case FIN_RESTART:
            // a right-hand side stopped at a power of ten: s[0] is its true
            // ||b - A x||^2 from the start kernel, which has also set r_hat = r
            // and p = v = 0; the next step's rho finalize takes rho from there
            S.true_rnorm2 = s[0];
            S.pend = 0;  // applied by the flush before the start kernel
            if (!isfinite(s[0])) {
                S.status = ST_NUMERIC;
                return;
            }
            S.rnorm2 = s[0];
            if (s[0] <= S.tol2) {
                S.status = ST_CONV;
                return;
            }
            S.status = ST_RUN;
            S.rhat_norm2 = s[0];
            S.rho = mk(1.0, 0.0);
            S.alpha = mk(1.0, 0.0);
            S.omega = mk(1.0, 0.0);
            S.beta = mk(0.0, 0.0);
            S.matvecs += 1;
            S.decades += 1;
            return;
        case FIN_TRUE_RECORD:
            S.true_rnorm2 = s[0];
            if (!isfinite(s[0])) S.status = ST_NUMERIC;
            return;
        case FIN_TRUE:
            S.true_rnorm2 = s[0];
            S.pend = 0;  // applied by the flush before the true residual
            if (!isfinite(s[0])) {
                S.status = ST_NUMERIC;
            } else if (status == ST_CONV && S.bnorm2 > 0.0 && s[0] > S.tol2 && S.iters2 < S.maxit2 &&
                       S.restarts < 5) {
                // the recursive residual drifted from the true one: restart from x
                S.status = ST_RUN;
                S.rnorm2 = s[0];
                S.rhat_norm2 = s[0];
                S.rho = mk(1.0, 0.0);
                S.alpha = mk(1.0, 0.0);
                S.omega = mk(1.0, 0.0);
                S.matvecs += 1;
                S.restarts += 1;
            }
            return;
        case FIN_RHO_DEFER:
        case FIN_RHO: {
            if (mode == FIN_RHO_DEFER && status == ST_RUN) {
                // the even step just finished left x += alpha p_hat + omega s_hat
                // to the odd step (or to the flush, if this right-hand side stops here)
                S.alpha_d = S.alpha;
                S.omega_d = S.omega;
                S.pend = 1;
            } else {
                S.pend = 0;  // consumed by the odd step's x / r update
            }
            if (status == ST_HALF) {
                // the half step has added alpha p_hat to x: this right-hand side is done
                S.status = ST_CONV;
                S.iters2 += 1;
                S.rnorm2 = S.snorm2;
                return;
            }
            const double rn2 = s[0];
            const c128 rho_new = mk(s[1], s[2]);
            if (!isfinite(rn2) || !finite2(rho_new)) { S.status = ST_NUMERIC; return; }
            S.rnorm2 = rn2;
            if (rn2 <= S.tol2) { S.status = ST_CONV; return; }
            if (abs2(S.omega) <= tiny * tiny) { S.status = ST_BREAK; return; }
            if (S.iters2 >= S.maxit2) { S.status = ST_MAXIT; return; }
            if (rn2 <= S.next2) {
                // restart from x, due at the next power of ten below this residual
                S.status = ST_RESTART;
                do S.next2 *= 0.01;
                while (S.next2 >= rn2);
                return;
            }
            if (sqrt(abs2(rho_new)) <= tiny * sqrt(S.rhat_norm2) * sqrt(rn2)) { S.status = ST_BREAK; return; }
            S.beta = cdiv(rho_new, S.rho) * cdiv(S.alpha, S.omega);
            S.rho = rho_new;
            return;
        }
        case FIN_ALPHA: {
            const c128 rv = mk(s[0], s[1]);
            S.matvecs += 1;
            if (!finite2(rv)) { S.status = ST_NUMERIC; return; }
            if (abs2(rv) == 0.0) { S.status = ST_BREAK; return; }
            S.alpha = cdiv(S.rho, rv);
            return;
        }
        case FIN_OMEGA: {
            // half step first: ||s|| small means x += alpha p_hat ends this
            // right-hand side, and t = A s_hat (already formed) is not used
            if (!isfinite(s[3])) { S.status = ST_NUMERIC; return; }
            S.snorm2 = s[3];
            if (s[3] <= S.tol2) { S.status = ST_HALF; return; }
            S.matvecs += 1;
            const c128 ts = mk(s[0], s[1]);
            const double tt = s[2];
            if (!finite2(ts) || !isfinite(tt)) { S.status = ST_NUMERIC; return; }
            if (tt == 0.0) { S.status = ST_BREAK; return; }
            S.omega = mk(ts.re / tt, ts.im / tt);
            S.iters2 += 2;
            return;
        }
        default:
            return;
    }
}

__device__ __forceinline__ int fin_slot(int mode) {
    switch (mode) {
        case FIN_ALPHA: return SLOT_V;
        case FIN_OMEGA: return SLOT_T;
        default: return SLOT_R;  // FIN_INIT, FIN_RHO, FIN_RHO_DEFER, FIN_TRUE*
    }
}
__device__ __forceinline__ int fin_terms(int mode) {
    switch (mode) {
        case FIN_ALPHA: return 2;
        case FIN_OMEGA: return 4;
        case FIN_RHO:
        case FIN_RHO_DEFER: return 3;
        case FIN_TRUE:
        case FIN_TRUE_RECORD:
        case FIN_RESTART: return 1;
        default: return 4;
    }
}

// the first NT terms of a slot into sums[0 .. NT)
template <int NT>
__device__ __forceinline__ void fixed_sum_into(const double* __restrict__ part, long long nblk,
                                               long long nblk_max, double* sums) {
    double o[NT];
    block_fixed_sum<NT>(part, nblk, nblk_max, o);
#pragma unroll
    for (int t = 0; t < NT; ++t) sums[t] = o[t];
}

__global__ __launch_bounds__(1024) void k_finalize(int mode, RhsState* st, const double* part,
                                                   long long nblk, long long nblk_max, double tol) {
    const int r = blockIdx.x;
    RhsState& S = st[r];
    const int status = S.status;
    bool act;
    switch (mode) {
        case FIN_TRUE:
        case FIN_TRUE_RECORD: act = status != ST_RUN && status != ST_IDLE && status != ST_HALF; break;
        case FIN_RHO:
        case FIN_RHO_DEFER: act = status == ST_RUN || status == ST_HALF; break;
        case FIN_RESTART: act = status == ST_RESTART; break;
        default: act = status == ST_RUN; break;
    }
    if (!act) return;
    double sums[4] = {0.0, 0.0, 0.0, 0.0};
    if (status != ST_HALF) {
        // only the terms the mode reads are loaded
        const double* base = part + part_index(r, fin_slot(mode), 0, nblk_max);
        switch (fin_terms(mode)) {
            case 1: fixed_sum_into<1>(base, nblk, nblk_max, sums); break;
            case 2: fixed_sum_into<2>(base, nblk, nblk_max, sums); break;
            case 3: fixed_sum_into<3>(base, nblk, nblk_max, sums); break;
            default: fixed_sum_into<4>(base, nblk, nblk_max, sums); break;
        }
    }
    if (threadIdx.x == 0) fin_update(mode, S, sums, tol);
}

// ---------------------------------------------------------------------------
// Operator apply in complex128 arithmetic; the input x is complex128 or, for
// the single-precision preconditioner's outputs, complex64 (converted exactly
// on load).  MODE selects the fused epilogue:
//   OP_PLAIN : y = Op x
//   OP_V     : y = A x, partials Re/Im sum conj(rhat) y          (slot V);
//              rhat (aux) is stored in the input's precision
//   OP_T     : y = A x, partials Re/Im sum conj(y) s, sum |y|^2   (slot T)
//   OP_P     : y = A x, partials Re/Im sum conj(p_i) y for the NS complex64
//              shadow vectors p_i of IDR(s) (rows 0 .. 2 NS - 1; aux points
//              to them, NS vectors of n nodes, shared by all right-hand sides)
// ---------------------------------------------------------------------------
template <int BC, int MODE, typename TX, int NS = 0>
__global__ __launch_bounds__(AP_LANES) void k_apply(Geo g, int zb, const cx<TX>* __restrict__ x,
                                                    c128* __restrict__ y, const double* __restrict__ k2,
                                                    const double* __restrict__ kb, double sr, double si,
                                                    const c128* __restrict__ aux, double* __restrict__ part,
                                                    long long nblk_max, const RhsState* st, int gate) {
    constexpr int NSL = AP_REGION / AP_LANES;  // region slots per lane
    // ring of three planes of the tile and its halo: z - 1 is kept in a
    // register, planes z and z + 1 are read from here
    __shared__ cx<TX> xs[3][AP_REGION];
    const int r = blockIdx.z;
    if (!gate_ok(st, r, gate)) return;
    const TileShape T = ap_tile_shape(g.nx, g.ny);
    const ApPos q = ap_pos(g, T, zb);
    const int t = threadIdx.x;
    const int RW = T.tw + 2, RN = RW * (T.th + 2);
    const double ih2 = 1.0 / (g.h * g.h);
    const double two_over_h = 2.0 / g.h;
    const long long roff = (long long)r * g.n;
    const cx<TX>* xr = x + roff;
    c128* yr = y + roff;
    const int i = q.i, j = q.j;
    // Halo nodes outside the domain hold their mirror image: for a Sommerfeld
    // boundary that is the eliminated ghost point; a Dirichlet neighbour on the
    // boundary (not an unknown) is selected away below.
    const bool use_im = BC == BC_SOMMERFELD || i > 1, use_ip = BC == BC_SOMMERFELD || i < g.nx - 2;
    const bool use_jm = BC == BC_SOMMERFELD || j > 1, use_jp = BC == BC_SOMMERFELD || j < g.ny - 2;
    const int col = j * g.nx + i;
    const int nf_col = (i == 0) + (i == g.nx - 1) + (j == 0) + (j == g.ny - 1);
    // the lane's LDS slot (a lane without a node reads the tile's first one)
    const int ls = q.own ? (q.oy + 1) * RW + q.ox + 1 : RW + 1;
    // in-plane offsets of this lane's region slots t, t + AP_LANES, ...
    int off[NSL];
    bool has[NSL];
#pragma unroll
    for (int m = 0; m < NSL; ++m) {
        const int sl = t + m * AP_LANES;
        has[m] = sl < RN;
        const int ly = sl / RW, lx = sl - ly * RW;
        off[m] = has[m] ? mirror_clamp(q.Y0 - 1 + ly, g.ny) * g.nx + mirror_clamp(q.X0 - 1 + lx, g.nx) : 0;
    }
    auto plane = [&](int z) {
        const int zz = z < 0 ? 1 : (z > g.nz - 1 ? g.nz - 2 : z);
        return xr + (long long)zz * g.plane;
    };
    constexpr int NACC = MODE == OP_P ? 2 * NS : 3;
    double acc[NACC];
#pragma unroll
    for (int a = 0; a < NACC; ++a) acc[a] = 0.0;
    const c64* pshadow = reinterpret_cast<const c64*>(aux);
    // prologue: plane z0 into LDS, plane z0 + 1 into registers, the lane's node below z0
    cx<TX> nxt[NSL];
    {
        const cx<TX>* p0 = plane(q.z0);
        const cx<TX>* p1 = plane(q.z0 + 1);
#pragma unroll
        for (int m = 0; m < NSL; ++m) {
            if (has[m]) xs[q.z0 % 3][t + m * AP_LANES] = p0[off[m]];
            nxt[m] = has[m] ? p1[off[m]] : cx<TX>{};
        }
    }
    c128 xm = cvt<double>(plane(q.z0 - 1)[col]);
    for (int z = q.z0; z < q.z1; ++z) {
        const int cur = z % 3, up = (z + 1) % 3;
#pragma unroll
        for (int m = 0; m < NSL; ++m)
            if (has[m]) xs[up][t + m * AP_LANES] = nxt[m];
        // the global loads of plane z + 2 stay in flight while plane z is computed
        if (z + 1 < q.z1) {
            const cx<TX>* p2 = plane(z + 2);
#pragma unroll
            for (int m = 0; m < NSL; ++m)
                if (has[m]) nxt[m] = p2[off[m]];
        }
        const long long idx = (long long)z * g.plane + col;
        const double kk = k2[idx];
        const int nf = nf_col + (z == 0) + (z == g.nz - 1);
        // interior nodes all read kb[0] (one cache line): no branch around the load
        const double kbv = kb[nf ? idx : 0];
        c128 aux_v = czero<double>();
        c64 pv[MODE == OP_P ? NS : 1];
        if (MODE == OP_V) aux_v = cvt<double>(reinterpret_cast<const cx<TX>*>(aux)[roff + idx]);
        if (MODE == OP_T) aux_v = aux[roff + idx];
        if constexpr (MODE == OP_P) {
#pragma unroll
            for (int a = 0; a < NS; ++a) pv[a] = pshadow[(long long)a * g.n + idx];
        }
        __syncthreads();
        const cx<TX>* b = xs[cur];
        const c128 xc = cvt<double>(b[ls]);
        c128 s = (use_im ? cvt<double>(b[ls - 1]) : czero<double>()) +
                 (use_ip ? cvt<double>(b[ls + 1]) : czero<double>());
        s = s + (use_jm ? cvt<double>(b[ls - RW]) : czero<double>());
        s = s + (use_jp ? cvt<double>(b[ls + RW]) : czero<double>());
        c128 zm = xm, zpv = cvt<double>(xs[up][ls]);
        if (BC == BC_DIRICHLET) {
            if (z - 1 < 1) zm = czero<double>();
            if (z + 1 > g.nz - 2) zpv = czero<double>();
        }
        s = s + zm;
        s = s + zpv;
        c128 d = mk(6.0 * ih2 - sr * kk, -si * kk);
        if (BC == BC_SOMMERFELD && nf) d.im -= nf * two_over_h * kbv;
        c128 out = d * xc - ih2 * s;
        if (BC == BC_DIRICHLET && (nf_col || z == 0 || z == g.nz - 1)) out = czero<double>();
        if (q.own) {
            yr[idx] = out;
            if (MODE == OP_V) {
                const c128 w = cdot(aux_v, out);
                acc[0] += w.re;
                acc[1] += w.im;
            } else if (MODE == OP_T) {
                const c128 w = cdot(out, aux_v);
                acc[0] += w.re;
                acc[1] += w.im;
                acc[2] += abs2(out);
            } else if constexpr (MODE == OP_P) {
#pragma unroll
                for (int a = 0; a < NS; ++a) {
                    const c128 w = cdot(cvt<double>(pv[a]), out);
                    acc[2 * a] += w.re;
                    acc[2 * a + 1] += w.im;
                }
            }
        }
        xm = xc;
    }
    const long long blk = (long long)blockIdx.y * gridDim.x + blockIdx.x;
    if constexpr (MODE == OP_P) {
        block_sum_store<NACC>(acc, part + part_index(r, 0, 0, nblk_max) + blk, nblk_max);
    }
    if constexpr (MODE == OP_V) {
        double v[2] = {acc[0], acc[1]};
        block_sum_store<2>(v, part + part_index(r, SLOT_V, 0, nblk_max) + blk, nblk_max);
    }
    if constexpr (MODE == OP_T) {
        block_sum_store<3>(acc, part + part_index(r, SLOT_T, 0, nblk_max) + blk, nblk_max);
    }
}

// ---------------------------------------------------------------------------
// Start of a (re)start: r = b - A x (use_x0) or r = b (x := 0); r_hat = r
// stored in precision TS (complex64 in the mixed solve: the shadow vector is
// then r rounded to complex64); p = v = 0; partials ||r||^2,
// Re/Im r_hat^H r (= ||r||^2, 0 when TS is double), ||b||^2 (slot R).
// ---------------------------------------------------------------------------
template <int BC, typename TS>
__global__ __launch_bounds__(AP_LANES) void k_init(Geo g, int zb, const c128* __restrict__ b,
                                              c128* __restrict__ x, c128* __restrict__ rr,
                                              cx<TS>* __restrict__ rhat, c128* __restrict__ p,
                                              c128* __restrict__ v, const double* __restrict__ k2,
                                              const double* __restrict__ kb, int use_x0,
                                              double* __restrict__ part, long long nblk_max,
                                              const RhsState* st, int gate) {
    const int r = blockIdx.z;
    if (!gate_ok(st, r, gate)) return;
    const ApPos q = ap_pos(g, ap_tile_shape(g.nx, g.ny), zb);
    const int z0 = q.z0, z1 = q.z1;
    const double ih2 = 1.0 / (g.h * g.h);
    const double two_over_h = 2.0 / g.h;
    const long long roff = (long long)r * g.n;
    const long long col = (long long)q.j * g.nx + q.i;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (q.own) {
        const c128* xr = x + roff;
        auto ldz = [&](int z) -> c128 {
            if (BC == BC_DIRICHLET && (z < 1 || z > g.nz - 2)) return czero<double>();
            return xr[(long long)z * g.plane + col];
        };
        const bool bnd_col = BC == BC_DIRICHLET &&
                             (q.i == 0 || q.j == 0 || q.i == g.nx - 1 || q.j == g.ny - 1);
        c128 xm = czero<double>(), xc = czero<double>();
        if (use_x0) {
            xm = z0 > 0 ? ldz(z0 - 1) : czero<double>();
            xc = ldz(z0);
        }
        for (int z = z0; z < z1; ++z) {
            const long long idx = (long long)z * g.plane + col;
            const bool bnd = BC == BC_DIRICHLET && (bnd_col || z == 0 || z == g.nz - 1);
            c128 bv = bnd ? czero<double>() : b[roff + idx];
            c128 res = bv;
            c128 xp = czero<double>();
            if (use_x0) {
                xp = z + 1 < g.nz ? ldz(z + 1) : czero<double>();
                if (!bnd) {
                    const c128* pl = xr + (long long)z * g.plane;
                    auto ld = [&](int ii, int jj) -> c128 { return pl[(long long)jj * g.nx + ii]; };
                    c128 s = inplane_sum<BC, double>(ld, q.i, q.j, g.nx, g.ny);
                    c128 zm = xm, zpv = xp;
                    if (BC == BC_SOMMERFELD) {
                        if (z == 0) zm = xp;
                        if (z == g.nz - 1) zpv = xm;
                    }
                    s = s + zm;
                    s = s + zpv;
                    const double kk = k2[idx];
                    c128 d = mk(6.0 * ih2 - kk, 0.0);
                    if (BC == BC_SOMMERFELD) {
                        const int nf = faces(q.i, q.j, z, g.nx, g.ny, g.nz);
                        if (nf) d.im -= nf * two_over_h * kb[idx];
                    }
                    res = bv - (d * xc - ih2 * s);
                }
            } else {
                x[roff + idx] = czero<double>();
            }
            rr[roff + idx] = res;
            const cx<TS> rh = cvt<TS>(res);
            rhat[roff + idx] = rh;
            p[roff + idx] = czero<double>();
            v[roff + idx] = czero<double>();
            const double n2 = abs2(res);
            acc[0] += n2;
            if constexpr (sizeof(TS) == sizeof(double)) {
                acc[1] += n2;
            } else {
                const c128 d = cdot(cvt<double>(rh), res);
                acc[1] += d.re;
                acc[2] += d.im;
            }
            acc[3] += abs2(bv);
            xm = xc;
            xc = xp;
        }
    }
    const long long blk = (long long)blockIdx.y * gridDim.x + blockIdx.x;
    block_sum_store<4>(acc, part + part_index(r, SLOT_R, 0, nblk_max) + blk, nblk_max);
}

// ---------------------------------------------------------------------------
// Krylov vector updates (complex128), grid-stride over nodes with exactly the
// fine-grid kernels' workgroup count per right-hand side: gridDim = (nblk, 1, nrhs).
// Every vector is read and written once per launch, with streaming loads and stores.
// ---------------------------------------------------------------------------
template <bool LOW>
__global__ __launch_bounds__(512) void k_p_update(long long n, c128* __restrict__ p,
                                                  const c128* __restrict__ rr,
                                                  const c128* __restrict__ v, c64* __restrict__ p_low,
                                                  const RhsState* st) {
    const int r = blockIdx.z;
    if (st[r].status != ST_RUN) return;
    const c128 beta = st[r].beta, om = st[r].omega;
    const long long off = (long long)r * n;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const c128 pv =
            ld_stream(&rr[off + i]) + beta * (ld_stream(&p[off + i]) - om * ld_stream(&v[off + i]));
        st_stream(&p[off + i], pv);
        if (LOW) st_stream(&p_low[off + i], cvt<float>(pv));
    }
}

// s = r - alpha v and the partial sums of ||s||^2 (slot T, term 3) for the
// half-step test.
template <bool LOW>
__global__ __launch_bounds__(512) void k_s_update(long long n, c128* __restrict__ s,
                                                  const c128* __restrict__ rr,
                                                  const c128* __restrict__ v, c64* __restrict__ s_low,
                                                  const RhsState* st, double* __restrict__ part,
                                                  long long nblk_max) {
    const int r = blockIdx.z;
    if (st[r].status != ST_RUN) return;
    const c128 al = st[r].alpha;
    const long long off = (long long)r * n;
    double acc[1] = {0.0};
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        c128 sv = ld_stream(&rr[off + i]) - al * ld_stream(&v[off + i]);
        st_stream(&s[off + i], sv);
        if (LOW) st_stream(&s_low[off + i], cvt<float>(sv));
        acc[0] += abs2(sv);
    }
    block_sum_store<1>(acc, part + part_index(r, SLOT_T, 3, nblk_max) + blockIdx.x, nblk_max);
}

// Iterating right-hand sides: r = s - omega t and the partials ||r||^2,
// r_hat^H r (p_hat, s_hat and r_hat in precision TH).  The solution is
// updated every second step: an even step (ODD false) leaves its
// x += alpha p_hat + omega s_hat outstanding (the next FIN_RHO_DEFER records
// it), and the odd step adds both steps' terms, reading p_hat' and s_hat' of
// the even step from their own buffers (php, shp), so x is read and written
// once per two steps.  Right-hand sides that stopped at the half step add
// alpha p_hat (and an outstanding update) to x; the next FIN_RHO marks them
// converged.
template <typename TH, bool ODD>
__global__ __launch_bounds__(512) void k_update_xr(long long n, c128* __restrict__ x,
                                                   c128* __restrict__ rr,
                                                   const cx<TH>* __restrict__ ph,
                                                   const cx<TH>* __restrict__ sh,
                                                   const cx<TH>* __restrict__ php,
                                                   const cx<TH>* __restrict__ shp,
                                                   const c128* __restrict__ s,
                                                   const c128* __restrict__ t,
                                                   const cx<TH>* __restrict__ rhat, const RhsState* st,
                                                   double* __restrict__ part, long long nblk_max) {
    const int r = blockIdx.z;
    const int status = st[r].status;
    if (status != ST_RUN && status != ST_HALF) return;
    const c128 al = st[r].alpha, om = st[r].omega;
    const bool pend = ODD && st[r].pend;
    const c128 ald = st[r].alpha_d, omd = st[r].omega_d;
    const long long off = (long long)r * n;
    // x plus the outstanding update of the even step, if any
    auto x_pend = [&](long long k) -> c128 {
        c128 xv = ld_stream(&x[k]);
        if (pend) xv = xv + ald * cvt<double>(ld_stream(&php[k])) + omd * cvt<double>(ld_stream(&shp[k]));
        return xv;
    };
    if (status == ST_HALF) {
        for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
             i += (long long)gridDim.x * blockDim.x)
            st_stream(&x[off + i], x_pend(off + i) + al * cvt<double>(ld_stream(&ph[off + i])));
        return;
    }
    double acc[3] = {0.0, 0.0, 0.0};
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        if (ODD)
            st_stream(&x[off + i], x_pend(off + i) + al * cvt<double>(ld_stream(&ph[off + i])) +
                                       om * cvt<double>(ld_stream(&sh[off + i])));
        c128 rv = ld_stream(&s[off + i]) - om * ld_stream(&t[off + i]);
        st_stream(&rr[off + i], rv);
        acc[0] += abs2(rv);
        c128 d = cdot(cvt<double>(ld_stream(&rhat[off + i])), rv);
        acc[1] += d.re;
        acc[2] += d.im;
    }
    block_sum_store<3>(acc, part + part_index(r, SLOT_R, 0, nblk_max) + blockIdx.x, nblk_max);
}

// The outstanding even-step update of right-hand sides that stopped after an
// even step (pend set, status neither iterating nor at the half step):
// x += alpha_d p_hat' + omega_d s_hat'.  FIN_TRUE, which follows the true
// residual, clears pend.
template <typename TH>
__global__ __launch_bounds__(512) void k_flush_x(long long n, c128* __restrict__ x,
                                                 const cx<TH>* __restrict__ php,
                                                 const cx<TH>* __restrict__ shp, const RhsState* st,
                                                 int only) {
    const int r = blockIdx.z;
    const int status = st[r].status;
    if (!st[r].pend || status == ST_RUN || status == ST_HALF || status == ST_IDLE) return;
    if (only >= 0 && status != only) return;
    const c128 ald = st[r].alpha_d, omd = st[r].omega_d;
    const long long off = (long long)r * n;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        st_stream(&x[off + i], ld_stream(&x[off + i]) + ald * cvt<double>(ld_stream(&php[off + i])) +
                                   omd * cvt<double>(ld_stream(&shp[off + i])));
}

// ---------------------------------------------------------------------------
// Set-up and auxiliary kernels
// ---------------------------------------------------------------------------
__global__ void k_model_check(long long n, const double* __restrict__ k, double* __restrict__ k2,
                              double* __restrict__ kb, int* __restrict__ bad) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const double v = k[i];
        if (!isfinite(v) || v < 0.0) atomicAdd(bad, 1);
        k2[i] = v * v;
        kb[i] = v;
    }
}

// k = omega sqrt(s) from the squared slowness s = 1/c^2 (k = 2 pi f / c);
// NaN/Inf or negative s, or a non-finite product, counts as bad
__global__ void k_model_from_slowness2(long long n, const double* __restrict__ s2, double omega,
                                       double* __restrict__ k, int* __restrict__ bad) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const double v = s2[i];
        const bool ok = isfinite(v) && v >= 0.0;
        const double kv = ok ? omega * sqrt(v) : 0.0;
        if (!ok || !isfinite(kv)) atomicAdd(bad, 1);
        k[i] = kv;
    }
}

// k_{l+1}(I) = k_l(2I)  (injection)
__global__ void k_inject(Geo gf, Geo gc, const double* __restrict__ kf, double* __restrict__ kc) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < gc.n;
         i += (long long)gridDim.x * blockDim.x) {
        const int z = (int)(i / gc.plane);
        const int rem = (int)(i - (long long)z * gc.plane);
        const int y = rem / gc.nx, x = rem - y * gc.nx;
        kc[i] = kf[(long long)(2 * z) * gf.plane + (long long)(2 * y) * gf.nx + 2 * x];
    }
}

// k^2 of a level in the multigrid precision.
template <typename R>
__global__ void k_level_k2(long long n, const double* __restrict__ k, R* __restrict__ k2) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const double v = k[i];
        k2[i] = R(v * v);
    }
}

__global__ void k_copy_rhs(Geo g, int bc, int nrhs, const c128* __restrict__ src,
                           c128* __restrict__ dst) {
    const long long tot = (long long)nrhs * g.n;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < tot;
         i += (long long)gridDim.x * blockDim.x) {
        const long long node = i % g.n;
        const int z = (int)(node / g.plane);
        const int rem = (int)(node - (long long)z * g.plane);
        const int y = rem / g.nx, x = rem - y * g.nx;
        c128 v = src[i];
        if (bc == BC_DIRICHLET && on_boundary(x, y, z, g.nx, g.ny, g.nz)) v = mk(0.0, 0.0);
        dst[i] = v;
    }
}

// rhs = D^-1 conj(g), D_j = 2^(-n_j)  (Sommerfeld); Dirichlet: conj(g) inside, 0 on the boundary
__global__ void k_adjoint_rhs(Geo g, int bc, int nrhs, const c128* __restrict__ gin,
                              c128* __restrict__ out) {
    const long long tot = (long long)nrhs * g.n;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < tot;
         i += (long long)gridDim.x * blockDim.x) {
        const long long node = i % g.n;
        const int z = (int)(node / g.plane);
        const int rem = (int)(node - (long long)z * g.plane);
        const int y = rem / g.nx, x = rem - y * g.nx;
        c128 v = conj(gin[i]);
        if (bc == BC_SOMMERFELD) {
            v = double(1 << faces(x, y, z, g.nx, g.ny, g.nz)) * v;
        } else if (on_boundary(x, y, z, g.nx, g.ny, g.nz)) {
            v = mk(0.0, 0.0);
        }
        out[i] = v;
    }
}

// grad_j = -sum_r Re(D_j w_rj a'_j u_rj), a'_j = -omega^2 - i n_j omega / (h sqrt(s_j))
__global__ void k_grad_s(Geo g, int bc, int nrhs, const c128* __restrict__ u,
                         const c128* __restrict__ w, const double* __restrict__ s, double omega,
                         double* __restrict__ grad) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < g.n;
         i += (long long)gridDim.x * blockDim.x) {
        const int z = (int)(i / g.plane);
        const int rem = (int)(i - (long long)z * g.plane);
        const int y = rem / g.nx, x = rem - y * g.nx;
        int nf = 0;
        double d = 1.0;
        if (bc == BC_SOMMERFELD) {
            nf = faces(x, y, z, g.nx, g.ny, g.nz);
            d = 1.0 / double(1 << nf);
        } else if (on_boundary(x, y, z, g.nx, g.ny, g.nz)) {
            grad[i] = 0.0;
            continue;
        }
        const c128 ap = mk(-omega * omega, -nf * omega / (g.h * sqrt(s[i])));
        double acc = 0.0;
        for (int r = 0; r < nrhs; ++r) {
            const c128 t = (w[(long long)r * g.n + i] * ap) * u[(long long)r * g.n + i];
            acc += t.re;
        }
        grad[i] = -d * acc;
    }
}

__global__ void k_set_point(long long off, double val, c128* __restrict__ b) {
    if (threadIdx.x == 0 && blockIdx.x == 0) b[off] = mk(val, 0.0);
}

__global__ void k_fill_status(int n, RhsState* st, int status, int maxit2, double tol2) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n) {
        st[r].status = status;
        st[r].maxit2 = maxit2;
        st[r].pend = 0;
        if (tol2 < 0.0) st[r].tol2 = tol2;
    }
}

// ---------------------------------------------------------------------------
// Host-side launchers
// ---------------------------------------------------------------------------
static inline dim3 grid_fine(const Geo& g, const Launch& L, int nrhs) {
    const TileShape T = ap_tile_shape(g.nx, g.ny);
    return dim3((unsigned)(T.ntx * T.nty), (unsigned)((g.nz + L.zb - 1) / L.zb), (unsigned)nrhs);
}

long long nblk_of(const Geo& g, const Launch& L) {
    const TileShape T = ap_tile_shape(g.nx, g.ny);
    return (long long)T.ntx * T.nty * ((g.nz + L.zb - 1) / L.zb);
}

static inline unsigned flat_blocks(long long n, int block, int cap) {
    long long b = (n + block - 1) / block;
    if (b > cap) b = cap;
    if (b < 1) b = 1;
    return (unsigned)b;
}

template <typename TX>
void launch_apply(hipStream_t s, int bc, int mode, const Geo& g, const Launch& L, int nrhs,
                  const cx<TX>* x, c128* y, const double* k2, const double* kb, double sr, double si,
                  const c128* aux, double* part, long long nblk_max, const RhsState* st, int gate) {
    dim3 grid = grid_fine(g, L, nrhs);
#define HH_APPLY(BCV, MV)                                                                             \
    hipLaunchKernelGGL((k_apply<BCV, MV, TX>), grid, dim3(AP_LANES), 0, s, g, L.zb, x, y, k2, kb, sr, si, \
                       aux, part, nblk_max, st, gate)
    if (bc == BC_SOMMERFELD) {
        if (mode == OP_PLAIN) HH_APPLY(BC_SOMMERFELD, OP_PLAIN);
        else if (mode == OP_V) HH_APPLY(BC_SOMMERFELD, OP_V);
        else HH_APPLY(BC_SOMMERFELD, OP_T);
    } else {
        if (mode == OP_PLAIN) HH_APPLY(BC_DIRICHLET, OP_PLAIN);
        else if (mode == OP_V) HH_APPLY(BC_DIRICHLET, OP_V);
        else HH_APPLY(BC_DIRICHLET, OP_T);
    }
#undef HH_APPLY
}
// y = A x with the fused IDR shadow products <p_i, y>, i < ns (rows 0 .. 2 ns - 1)
void launch_apply_p(hipStream_t s, int bc, const Geo& g, const Launch& L, int nrhs, int ns, const c128* x,
                    c128* y, const double* k2, const double* kb, const c64* P, double* part,
                    long long nblk_max, const RhsState* st, int gate) {
    dim3 grid = grid_fine(g, L, nrhs);
    const c128* aux = reinterpret_cast<const c128*>(P);
#define HH_APPLY_P(BCV, NSV)                                                                             \
    hipLaunchKernelGGL((k_apply<BCV, OP_P, double, NSV>), grid, dim3(AP_LANES), 0, s, g, L.zb, x, y, k2, kb, \
                       1.0, 0.0, aux, part, nblk_max, st, gate)
#define HH_APPLY_P_NS(BCV)                \
    switch (ns) {                         \
        case 1: HH_APPLY_P(BCV, 1); break; \
        case 2: HH_APPLY_P(BCV, 2); break; \
        case 3: HH_APPLY_P(BCV, 3); break; \
        case 4: HH_APPLY_P(BCV, 4); break; \
        case 5: HH_APPLY_P(BCV, 5); break; \
        case 6: HH_APPLY_P(BCV, 6); break; \
        case 7: HH_APPLY_P(BCV, 7); break; \
        default: HH_APPLY_P(BCV, 8); break; \
    }
    if (bc == BC_SOMMERFELD) {
        HH_APPLY_P_NS(BC_SOMMERFELD)
    } else {
        HH_APPLY_P_NS(BC_DIRICHLET)
    }
#undef HH_APPLY_P_NS
#undef HH_APPLY_P
}

template void launch_apply<double>(hipStream_t, int, int, const Geo&, const Launch&, int, const c128*,
                                   c128*, const double*, const double*, double, double, const c128*,
                                   double*, long long, const RhsState*, int);
template void launch_apply<float>(hipStream_t, int, int, const Geo&, const Launch&, int, const c64*,
                                  c128*, const double*, const double*, double, double, const c128*,
                                  double*, long long, const RhsState*, int);

void launch_init(hipStream_t s, int bc, const Geo& g, const Launch& L, int nrhs, const c128* b,
                 c128* x, c128* r, void* rhat, bool rhat_low, c128* p, c128* v, const double* k2,
                 const double* kb, int use_x0, double* part, long long nblk_max, const RhsState* st, int gate) {
    dim3 grid = grid_fine(g, L, nrhs);
#define HH_INIT(BCV, TSV)                                                                                     \
    hipLaunchKernelGGL((k_init<BCV, TSV>), grid, dim3(AP_LANES), 0, s, g, L.zb, b, x, r,                     \
                       reinterpret_cast<cx<TSV>*>(rhat), p, v, k2, kb, use_x0, part, nblk_max, st, gate)
    if (bc == BC_SOMMERFELD) {
        if (rhat_low) HH_INIT(BC_SOMMERFELD, float);
        else HH_INIT(BC_SOMMERFELD, double);
    } else {
        if (rhat_low) HH_INIT(BC_DIRICHLET, float);
        else HH_INIT(BC_DIRICHLET, double);
    }
#undef HH_INIT
}

void launch_p_update(hipStream_t s, long long n, int nrhs, c128* p, const c128* r, const c128* v,
                     c64* p_low, const RhsState* st, const Launch& L) {
    const dim3 grid(L.flat_cap, 1, nrhs);
    if (p_low) hipLaunchKernelGGL(k_p_update<true>, grid, dim3(L.block), 0, s, n, p, r, v, p_low, st);
    else hipLaunchKernelGGL(k_p_update<false>, grid, dim3(L.block), 0, s, n, p, r, v, p_low, st);
}
void launch_s_update(hipStream_t s, long long n, int nrhs, c128* sv, const c128* r, const c128* v,
                     c64* s_low, const RhsState* st, double* part, long long nblk_max, const Launch& L) {
    const dim3 grid(L.flat_cap, 1, nrhs);
    if (s_low)
        hipLaunchKernelGGL(k_s_update<true>, grid, dim3(L.block), 0, s, n, sv, r, v, s_low, st, part, nblk_max);
    else
        hipLaunchKernelGGL(k_s_update<false>, grid, dim3(L.block), 0, s, n, sv, r, v, s_low, st, part,
                           nblk_max);
}
template <typename TH>
void launch_update_xr(hipStream_t s, bool odd, long long n, int nrhs, c128* x, c128* r, const cx<TH>* ph,
                      const cx<TH>* sh, const cx<TH>* php, const cx<TH>* shp, const c128* sv, const c128* t,
                      const cx<TH>* rhat, const RhsState* st, double* part, long long nblk_max,
                      const Launch& L) {
    const dim3 grid(L.flat_cap, 1, nrhs);
    if (odd)
        hipLaunchKernelGGL((k_update_xr<TH, true>), grid, dim3(L.block), 0, s, n, x, r, ph, sh, php, shp, sv, t,
                           rhat, st, part, nblk_max);
    else
        hipLaunchKernelGGL((k_update_xr<TH, false>), grid, dim3(L.block), 0, s, n, x, r, ph, sh, php, shp, sv,
                           t, rhat, st, part, nblk_max);
}
template <typename TH>
void launch_flush_x(hipStream_t s, long long n, int nrhs, c128* x, const cx<TH>* php, const cx<TH>* shp,
                    const RhsState* st, const Launch& L, int only) {
    hipLaunchKernelGGL(k_flush_x<TH>, dim3(L.flat_cap, 1, nrhs), dim3(L.block), 0, s, n, x, php, shp, st,
                       only);
}
template void launch_update_xr<double>(hipStream_t, bool, long long, int, c128*, c128*, const c128*,
                                       const c128*, const c128*, const c128*, const c128*, const c128*,
                                       const c128*, const RhsState*, double*, long long, const Launch&);
template void launch_update_xr<float>(hipStream_t, bool, long long, int, c128*, c128*, const c64*, const c64*,
                                      const c64*, const c64*, const c128*, const c128*, const c64*,
                                      const RhsState*, double*, long long, const Launch&);
template void launch_flush_x<double>(hipStream_t, long long, int, c128*, const c128*, const c128*,
                                     const RhsState*, const Launch&, int);
template void launch_flush_x<float>(hipStream_t, long long, int, c128*, const c64*, const c64*,
                                    const RhsState*, const Launch&, int);
void launch_finalize(hipStream_t s, int mode, int nrhs, RhsState* st, const double* part,
                     long long nblk, long long nblk_max, double tol) {
    hipLaunchKernelGGL(k_finalize, dim3(nrhs), dim3(1024), 0, s, mode, st, part, nblk, nblk_max, tol);
}

void launch_model_check(hipStream_t s, long long n, const double* k, double* k2, double* kb, int* bad) {
    hipLaunchKernelGGL(k_model_check, dim3(flat_blocks(n, 256, 8192)), dim3(256), 0, s, n, k, k2, kb,
                       bad);
}
void launch_model_from_slowness2(hipStream_t s, long long n, const double* s2, double omega, double* k, int* bad) {
    hipLaunchKernelGGL(k_model_from_slowness2, dim3(flat_blocks(n, 256, 8192)), dim3(256), 0, s, n, s2, omega,
                       k, bad);
}
void launch_inject(hipStream_t s, const Geo& gf, const Geo& gc, const double* kf, double* kc) {
    hipLaunchKernelGGL(k_inject, dim3(flat_blocks(gc.n, 256, 8192)), dim3(256), 0, s, gf, gc, kf, kc);
}
template <typename R>
void launch_level_k2(hipStream_t s, long long n, const double* k, R* k2) {
    hipLaunchKernelGGL((k_level_k2<R>), dim3(flat_blocks(n, 256, 8192)), dim3(256), 0, s, n, k, k2);
}
template void launch_level_k2<double>(hipStream_t, long long, const double*, double*);
template void launch_level_k2<float>(hipStream_t, long long, const double*, float*);
template <typename R>
__global__ void k_level_k(long long n, const double* __restrict__ k, R* __restrict__ kl) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        kl[i] = R(k[i]);
}
template <typename R>
void launch_level_k(hipStream_t s, long long n, const double* k, R* kl) {
    hipLaunchKernelGGL((k_level_k<R>), dim3(flat_blocks(n, 256, 8192)), dim3(256), 0, s, n, k, kl);
}
template void launch_level_k<double>(hipStream_t, long long, const double*, double*);
template void launch_level_k<float>(hipStream_t, long long, const double*, float*);
void launch_copy_rhs(hipStream_t s, const Geo& g, int bc, int nrhs, const c128* src, c128* dst) {
    hipLaunchKernelGGL(k_copy_rhs, dim3(flat_blocks((long long)nrhs * g.n, 256, 8192)), dim3(256), 0,
                       s, g, bc, nrhs, src, dst);
}
void launch_adjoint_rhs(hipStream_t s, const Geo& g, int bc, int nrhs, const c128* gin, c128* out) {
    hipLaunchKernelGGL(k_adjoint_rhs, dim3(flat_blocks((long long)nrhs * g.n, 256, 8192)), dim3(256),
                       0, s, g, bc, nrhs, gin, out);
}
void launch_grad_s(hipStream_t s, const Geo& g, int bc, int nrhs, const c128* u, const c128* w,
                   const double* sl, double omega, double* grad) {
    hipLaunchKernelGGL(k_grad_s, dim3(flat_blocks(g.n, 256, 8192)), dim3(256), 0, s, g, bc, nrhs, u, w,
                       sl, omega, grad);
}
void launch_set_point(hipStream_t s, long long off, double val, c128* b) {
    hipLaunchKernelGGL(k_set_point, dim3(1), dim3(64), 0, s, off, val, b);
}
void launch_fill_status(hipStream_t s, int n, RhsState* st, int status, int maxit2, double tol2) {
    hipLaunchKernelGGL(k_fill_status, dim3(1), dim3(64), 0, s, n, st, status, maxit2, tol2);
}

}  // namespace hh
