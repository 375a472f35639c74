// Multigrid kernels for gfx950: one fused pass down and one fused pass up per level.
//
// With M u = (1/h^2) lap(u) - c u,  lap(u)_j = sum_nb (u_j - u_nb),
//      c_j = (beta1 - beta2 i) k_j^2 + n_j 2 i k_j / h,   D_j = 6/h^2 - c_j,
// (paper section 3.3 and Algorithm 2: the 7-point stencil with its Sommerfeld
// ghost points eliminated; n_j = faces node j lies on) and W = omega D^-1:
//
// Down (Algorithm 1 steps 1-3: zero initial guess, one damped-Jacobi sweep,
// residual, full-weighting restriction of section 3.4.2):
//   u1 = W b,   r = b - (1/h^2) lap(u1) + c u1,   b_H = R r.
// Since D u1 = omega b, the residual is r = (1 - omega) b + (1/h^2) sum_nb u1_nb:
// the node's own u1 and c drop out, and every term has the size of b (no
// cancellation to guard against, unlike the up pass's residual of u2).
// Up (Algorithm 1 steps 5-7: trilinear prolongation of section 3.4.3,
// correction, one damped-Jacobi sweep):
//   u2 = W b + P e_H,   u3 = u2 + W (b - (1/h^2) lap(u2) + c u2).
//
// The Laplacian is summed as differences u_j - u_nb: for the smooth part of u
// each difference is exact in floating point, so the correction keeps its
// relative accuracy in single precision instead of losing a factor of about
// 6 / (k h)^2 to cancellation in 6 u_j - sum u_nb.
//
// Only the level's k is stored; c, D and W are recomputed per node.  Both
// kernels stage x-y planes of a tile and its halo in LDS and march along z with
// a ring of three planes; the global loads of the next two planes are issued
// into registers before the current plane is computed.  Halo positions outside the
// domain are read from their mirror image: for Sommerfeld levels that is the
// eliminated ghost point (its 2hik part is in c) and the even extension of the
// full-weighting stencil; for Dirichlet levels the boundary values are zero and
// boundary outputs are forced to zero.
#include <type_traits>

#include "hh_common.h"
#include "hh_device.h"
#include "hh_kernels.h"

namespace hh {

__device__ __forceinline__ int ring3(int f) { return ((f % 3) + 3) % 3; }

constexpr int DN_LANES = 256, DN_MAXH = 16;
// Fine region nodes staged by a down-pass workgroup: DN_REGION on the large
// levels; the one-plane pass of the small levels may take a smaller region
// (more workgroups, fewer region nodes per lane), see dn_region().
constexpr int DN_REGION = 1280;
__host__ __device__ constexpr int dn_maxw(int reg) { return reg >= 1280 ? 32 : reg >= 512 ? 16 : 8; }
// Tile of the down pass on the coarse grid: tile_shape() with the height
// bounded so that the fine region, (2 tw + 3)(2 th + 3) nodes, fits reg
// (tw <= dn_maxw(reg) leaves th >= 1).
__host__ __device__ inline TileShape dn_tile_shape(int nx, int ny, int reg) {
    TileShape T = tile_shape(nx, ny, dn_maxw(reg), DN_LANES, DN_MAXH);
    const int hmax = (reg / (2 * T.tw + 3) - 3) / 2;
    if (T.th > hmax) {
        T.th = hmax;
        T.nty = (ny + T.th - 1) / T.th;
    }
    return T;
}
// Up pass: 512 lanes, each owning two x-adjacent nodes (an x-pair) of the
// tile-plus-halo region, so a region row holds up to 64 nodes.
constexpr int UP_LANES = 512, UP_MAXW = 62;
// Tile of the up pass: an even width tw <= UP_MAXW (the region, tw + 2 nodes
// wide from X0 - 1, is then a whole number of x-pairs), the plane split into
// nearly equal tiles, and as many rows th as leave the region's rows of pairs
// within the lanes: (th + 2) (tw + 2) / 2 <= UP_LANES.
__host__ __device__ inline TileShape up_tile_shape(int nx, int ny) {
    TileShape T;
    T.ntx = (nx + UP_MAXW - 1) / UP_MAXW;
    T.tw = (nx + T.ntx - 1) / T.ntx;
    T.tw += T.tw & 1;
    T.th = UP_LANES / ((T.tw + 2) / 2) - 2;
    if (T.th > ny) T.th = ny;
    T.nty = (ny + T.th - 1) / T.th;
    return T;
}

// Tile of the one-node-per-lane up pass (double precision): the tile plus a
// one-node halo must fit the lanes, (tw + 2)(th + 2) <= UP_LANES.
constexpr int UP1_MAXW = 32;
__host__ __device__ inline TileShape up1_tile_shape(int nx, int ny) {
    TileShape T;
    T.ntx = (nx + UP1_MAXW - 1) / UP1_MAXW;
    T.tw = (nx + T.ntx - 1) / T.ntx;
    T.th = UP_LANES / (T.tw + 2) - 2;
    if (T.th > ny) T.th = ny;
    T.nty = (ny + T.th - 1) / T.th;
    return T;
}
__device__ __forceinline__ int ring4i(int f) { return f & 3; }  // also for f = -1

// Coarse nodes an x-pair up-pass tile interpolates from: a window of cw x ch nodes of
// one coarse plane starting at (cx0, cy0).  A region node at fine (x, y) of the
// tile (or the mirror image of a halo position) reads coarse columns x >> 1 and
// x >> 1 + 1 (clamped), so the window spans (X0 - 1) >> 1 .. (X0 + tw) >> 1 + 1
// and likewise in y.  Region positions past the grid's far end that are
// neither output nor halo of an output may fall outside; their coarse indices
// are clamped into the window (their results are never used).  The window is
// staged in LDS one node per lane, so cw ch <= UP_LANES is required (checked
// on the host for every level by mg_up_windows_fit).
struct CoarseWin {
    int cx0, cy0, cw, ch;
};
__host__ __device__ inline CoarseWin up_coarse_window(int X0, int Y0, int tw, int th, int gcnx, int gcny) {
    CoarseWin W;
    W.cx0 = X0 >= 1 ? (X0 - 1) >> 1 : 0;
    W.cy0 = Y0 >= 1 ? (Y0 - 1) >> 1 : 0;
    const int xe = ((X0 + tw) >> 1) + 1, ye = ((Y0 + th) >> 1) + 1;
    W.cw = (xe < gcnx - 1 ? xe : gcnx - 1) - W.cx0 + 1;
    W.ch = (ye < gcny - 1 ? ye : gcny - 1) - W.cy0 + 1;
    return W;
}

// Level constants of the CSLP operator in the compute precision.
template <typename R>
struct LevelCoef {
    R ih2, six_ih2, two_over_h, sr, si, omega;
};
template <typename R>
__device__ __forceinline__ LevelCoef<R> level_coef(const Geo& g, double beta1, double beta2,
                                                   double omega) {
    LevelCoef<R> L;
    L.ih2 = R(1.0 / (g.h * g.h));
    L.six_ih2 = R(6.0 / (g.h * g.h));
    L.two_over_h = R(2.0 / g.h);
    L.sr = R(beta1);
    L.si = R(-beta2);
    L.omega = R(omega);
    return L;
}

// Fused multiply-adds are written out: this file is compiled without implicit
// contraction (-ffp-contract=off), so every rounding is fixed by the source
// and is the same in every inlined copy of a loop body -- the passes' results
// do not depend on their z-blocks or regions.
__device__ __forceinline__ float fmar(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmar(double a, double b, double c) { return __builtin_fma(a, b, c); }
// a b + c (complex)
template <typename R>
__device__ __forceinline__ cx<R> cfma(const cx<R>& a, const cx<R>& b, const cx<R>& c) {
    return {fmar(a.re, b.re, fmar(-a.im, b.im, c.re)), fmar(a.re, b.im, fmar(a.im, b.re, c.im))};
}
// a b (complex)
template <typename R>
__device__ __forceinline__ cx<R> cmul(const cx<R>& a, const cx<R>& b) {
    return {fmar(a.re, b.re, -(a.im * b.im)), fmar(a.re, b.im, a.im * b.re)};
}
// s a + c (s real)
template <typename R>
__device__ __forceinline__ cx<R> sfma(R s, const cx<R>& a, const cx<R>& c) {
    return {fmar(s, a.re, c.re), fmar(s, a.im, c.im)};
}
// s a + t b (s, t real)
template <typename R>
__device__ __forceinline__ cx<R> lerp2(R s, const cx<R>& a, R t, const cx<R>& b) {
    return sfma(s, a, t * b);
}
// the residual of M at a node, b - (1/h^2) lap + c u
template <typename R>
__device__ __forceinline__ cx<R> mresid(const cx<R>& b, R ih2, const cx<R>& lap, const cx<R>& c, const cx<R>& u) {
    return cfma(c, u, sfma(-ih2, lap, b));
}

// Reciprocal of |D|^2, a positive normal number far from both ends of the
// range: in single precision the hardware v_rcp_f32 (about 1 ulp), far inside
// the accuracy a complex64 V-cycle is held to; in double precision v_rcp_f64
// refined by two Newton steps y += y (1 - x y), about 1 ulp as well, instead
// of the correctly rounded division's scaling and fix-up sequence.
__device__ __forceinline__ double mg_rcp(double x) {
    double y = __builtin_amdgcn_rcp(x);
    y = fmar(y, fmar(-x, y, 1.0), y);
    return fmar(y, fmar(-x, y, 1.0), y);
}
__device__ __forceinline__ float mg_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// c_j = (beta1 - beta2 i) k^2 + n_j 2 i k / h from the level's k (k^2 formed
// in the compute precision)
template <typename R>
__device__ __forceinline__ cx<R> shift_c(const LevelCoef<R>& L, R k, int nf) {
    const R k2 = k * k;
    cx<R> c = {L.sr * k2, L.si * k2};
    if (nf) c.im = fmar(R(nf) * L.two_over_h, k, c.im);
    return c;
}
// W = omega / (6/h^2 - c)
template <typename R>
__device__ __forceinline__ cx<R> jacobi_w(const LevelCoef<R>& L, cx<R> c) {
    const R dr = L.six_ih2 - c.re, di = -c.im;
    const R s = L.omega * mg_rcp(fmar(dr, dr, di * di));
    return {dr * s, -di * s};
}

__device__ __forceinline__ int faces_of(int x, int y, int z, const Geo& g) {
    return (x == 0) + (x == g.nx - 1) + (y == 0) + (y == g.ny - 1) + (z == 0) + (z == g.nz - 1);
}

// ---------------------------------------------------------------------------
// Down: b_H = R (b - M W b).  The workgroup owns a tw x th tile of coarse
// columns and marches over `zbc` coarse planes (2 zbc + 1 fine residual
// planes).  Each lane owns NU nodes of the fine region (tile plus a two-node
// halo): it loads their b and k, writes u1 = W b to the LDS ring, and keeps
// (1 - omega) b in registers for the residual of the same nodes one plane
// later, so every input is read once per plane.  Two planes of loads are in
// flight.
// ---------------------------------------------------------------------------
template <typename TB, typename R, int NU>
struct DownRaw {
    cx<TB> b[NU];
    R k[NU];
};
template <typename R, int NU>
struct DownKeep {
    cx<R> b[NU];  // (1 - omega) b
};

template <int BC, typename TB, typename R, bool ONE, int REG>
__global__ __launch_bounds__(DN_LANES) void k_mg_down(Geo gf, Geo gc, int zbc,
                                                      const cx<TB>* __restrict__ b,
                                                      long long b_rstride,
                                                      const R* __restrict__ kl, double beta1,
                                                      double beta2, double omega,
                                                      cx<R>* __restrict__ bc_out,
                                                      const RhsState* st, int gate) {
    static_assert(REG % DN_LANES == 0, "every lane's region slots must lie inside the LDS arrays");
    constexpr int NU = REG / DN_LANES;
    __shared__ cx<R> u1s[3][REG];
    __shared__ cx<R> rs[REG];

    const int r = blockIdx.z;
    if (!gate_ok(st, r, gate)) return;
    const int t = threadIdx.x;
    const TileShape T = dn_tile_shape(gc.nx, gc.ny, REG);
    const int RW = 2 * T.tw + 3, RH = 2 * T.th + 3;
    const int id = xcd_tile_id(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
    const int tz = id / gridDim.x;
    const int txy = id - tz * gridDim.x;
    const int tyi = txy / T.ntx, txi = txy - tyi * T.ntx;
    const int X0 = txi * T.tw, Y0 = tyi * T.th;
    const int Z0 = tz * zbc, Z1 = min(gc.nz, Z0 + zbc);
    const int gx0 = 2 * X0 - 2, gy0 = 2 * Y0 - 2;
    const cx<TB>* br = b + (long long)r * b_rstride;
    const LevelCoef<R> L = level_coef<R>(gf, beta1, beta2, omega);

    // region nodes of this lane: in-plane offset, face count within the x-y
    // plane, and whether the residual is needed there (region minus its rim)
    int uoff[NU], unf[NU];
    bool ubnd[NU], uin[NU];
#pragma unroll
    for (int k = 0; k < NU; ++k) {
        const int idx = t + k * DN_LANES;
        const int ly = idx / RW, lx = idx - ly * RW;
        const int gx = mirror_clamp(gx0 + lx, gf.nx), gy = mirror_clamp(gy0 + ly, gf.ny);
        uoff[k] = gy * gf.nx + gx;
        unf[k] = (gx == 0) + (gx == gf.nx - 1) + (gy == 0) + (gy == gf.ny - 1);
        ubnd[k] = unf[k] != 0;
        uin[k] = idx < RW * RH && lx >= 1 && lx <= RW - 2 && ly >= 1 && ly <= RH - 2;
    }

    // Loads are issued unconditionally (every offset is a valid node) so the
    // compiler can count them and keep later planes in flight.  Planes past
    // the chunk's last one re-read that plane instead (an L2 hit).
    const int flast = 2 * Z1;
    auto fetch = [&](int f, DownRaw<TB, R, NU>& w) {
        const long long base = (long long)mirror_clamp(min(f, flast), gf.nz) * gf.plane;
#pragma unroll
        for (int k = 0; k < NU; ++k) {
            w.b[k] = br[base + uoff[k]];
            w.k[k] = kl[base + uoff[k]];
        }
        // keep the scheduler from moving these loads past later ones: loads
        // complete in issue order, so a plane must be issued as one group
        __builtin_amdgcn_sched_barrier(0);
    };
    // u1 = W b to the ring; (1 - omega) b kept for this plane's residual
    const R omc = R(1.0 - omega);
    auto commit = [&](int f, const DownRaw<TB, R, NU>& w, DownKeep<R, NU>& kp) {
        const int fz = mirror_clamp(f, gf.nz);
        const int zf = (fz == 0) + (fz == gf.nz - 1);
        cx<R>* dst = u1s[ring3(f)];
#pragma unroll
        for (int k = 0; k < NU; ++k) {
            const int idx = t + k * DN_LANES;
            const int nf = BC == BC_SOMMERFELD ? unf[k] + zf : 0;
            const cx<R> c = shift_c(L, w.k[k], nf);
            const cx<R> bb = cvt<R>(w.b[k]);
            cx<R> v = cmul(jacobi_w(L, c), bb);
            if (BC == BC_DIRICHLET && (ubnd[k] || zf)) v = czero<R>();
            // unguarded: idx < NU * DN_LANES = REG, and slots past the
            // region are never read (a guard would sink the loads into it)
            dst[idx] = v;
            kp.b[k] = {omc * bb.re, omc * bb.im};
        }
    };
    // r = (1 - omega) b + (1/h^2) sum_nb u1_nb on the region's inner nodes (on
    // a Dirichlet boundary node, where u1 is held at zero, this is not its
    // residual; such nodes feed only coarse boundary nodes, whose output is zero)
    auto residual = [&](int f, const DownKeep<R, NU>& kp) {
        const cx<R>* um = u1s[ring3(f - 1)];
        const cx<R>* uc = u1s[ring3(f)];
        const cx<R>* up = u1s[ring3(f + 1)];
#pragma unroll
        for (int k = 0; k < NU; ++k) {
            if (uin[k]) {
                const int c = t + k * DN_LANES;
                cx<R> nb = uc[c - 1] + uc[c + 1];
                nb = nb + uc[c - RW];
                nb = nb + uc[c + RW];
                nb = nb + um[c];
                nb = nb + up[c];
                rs[c] = sfma(L.ih2, nb, kp.b[k]);
            }
        }
    };

    const int cxl = t % T.tw, cyl = t / T.tw;
    const int X = X0 + cxl, Y = Y0 + cyl;
    const bool mine = cyl < T.th && X < gc.nx && Y < gc.ny;
    const int ic = mine ? (2 * cyl + 2) * RW + 2 * cxl + 2 : RW + 1;
    cx<R> acc = czero<R>();
    // one step: u1 of plane f + 1, residual of plane f, its 2D full weighting
    // accumulated with z weights 1, 2, 1 over fine planes 2Z - 1, 2Z, 2Z + 1
    auto step = [&](int f, DownRaw<TB, R, NU>& w, DownKeep<R, NU>& cur, DownKeep<R, NU>& nxt,
                    bool refill) {
        commit(f + 1, w, nxt);
        if (refill) fetch(f + 3, w);
        __syncthreads();
        residual(f, cur);
        __syncthreads();
        cx<R> q = R(4) * rs[ic];
        cx<R> e = rs[ic - 1] + rs[ic + 1];
        e = e + rs[ic - RW];
        e = e + rs[ic + RW];
        cx<R> c4 = rs[ic - RW - 1] + rs[ic - RW + 1];
        c4 = c4 + rs[ic + RW - 1];
        c4 = c4 + rs[ic + RW + 1];
        q = q + R(2) * e;
        q = q + c4;
        if (f == 2 * Z0 - 1) {
            acc = q;
        } else if ((f & 1) == 0) {
            acc = acc + R(2) * q;
        } else {
            const int Z = (f - 1) >> 1;
            if (mine) {
                cx<R> v = R(1.0 / 64.0) * (acc + q);
                if (BC == BC_DIRICHLET &&
                    (X == 0 || Y == 0 || Z == 0 || X == gc.nx - 1 || Y == gc.ny - 1 || Z == gc.nz - 1))
                    v = czero<R>();
                bc_out[(long long)r * gc.n + (long long)Z * gc.plane + (long long)Y * gc.nx + X] = v;
            }
            acc = q;
        }
    };

    // u1 planes 2 Z0 - 2 .. 2 Z1, residual planes 2 Z0 - 1 .. 2 Z1 - 1.
    const int F0 = 2 * Z0 - 2;
    if constexpr (ONE) {
        // one coarse plane per workgroup (the small levels, where latency
        // rules): all five fine planes are loaded in one round
        DownRaw<TB, R, NU> S0, S1, S2, S3, S4;
        DownKeep<R, NU> K0, K1;
        fetch(F0, S0);
        fetch(F0 + 1, S1);
        fetch(F0 + 2, S2);
        fetch(F0 + 3, S3);
        fetch(F0 + 4, S4);
        commit(F0, S0, K1);  // plane F0 only feeds the residual stencil; K1 is overwritten below
        commit(F0 + 1, S1, K0);
        step(F0 + 1, S2, K0, K1, false);
        step(F0 + 2, S3, K1, K0, false);
        step(F0 + 3, S4, K0, K1, false);
    } else {
        // set A holds the planes F0 + even, set B the odd ones
        DownRaw<TB, R, NU> A, B;
        DownKeep<R, NU> K0, K1;
        fetch(F0, A);
        fetch(F0 + 1, B);
        commit(F0, A, K1);  // plane F0 only feeds the residual stencil; K1 is overwritten below
        fetch(F0 + 2, A);
        commit(F0 + 1, B, K0);
        fetch(F0 + 3, B);
        for (int f = F0 + 1; f <= 2 * Z1 - 1; f += 2) {
            step(f, A, K0, K1, true);
            if (f + 1 > 2 * Z1 - 1) break;
            step(f + 1, B, K1, K0, true);
        }
    }
}

// ---------------------------------------------------------------------------
// Up: u3 = u2 + W (b - (1/h^2) lap(u2) + c u2), u2 = W b + P e_H.  Each lane
// owns one node of the tile-plus-halo region; the lanes inside the halo
// compute the output.  The workgroup marches over `zb` planes (double
// precision; single precision takes the x-pair kernel k_mg_up below, which
// needs fewer instructions per node but more registers per lane than double
// precision leaves).  Every node's arithmetic is the same for every tile and
// z-block.  With ACC the pass adds u3 to the output instead of storing it
// (the F-cycle's second coarse-grid cycle).
// ---------------------------------------------------------------------------
// Compiled for two 512-lane workgroups per CU (<= 128 VGPRs).
template <int BC, typename TB, typename R, typename TO, bool ACC>
__global__ __launch_bounds__(UP_LANES, 4) void k_mg_up1(Geo g, Geo gc, int zb,
                                                    const cx<TB>* __restrict__ b, long long b_rstride,
                                                    const R* __restrict__ kl, double beta1,
                                                    double beta2, double omega,
                                                    const cx<R>* __restrict__ ec,
                                                    cx<TO>* __restrict__ out, long long o_rstride,
                                                    const RhsState* st, int gate) {
    // a ring of four u2 planes: the stencil of plane z reads z - 1 .. z + 1
    // while plane z + 2 is written, so one barrier per plane suffices
    __shared__ cx<R> us[4][UP_LANES];

    const int r = blockIdx.z;
    if (!gate_ok(st, r, gate)) return;
    const int t = threadIdx.x;
    const TileShape T = up1_tile_shape(g.nx, g.ny);
    const int RW = T.tw + 2, RH = T.th + 2;
    const int id = xcd_tile_id(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
    const int tz = id / gridDim.x;
    const int txy = id - tz * gridDim.x;
    const int tyi = txy / T.ntx, txi = txy - tyi * T.ntx;
    const int X0 = txi * T.tw, Y0 = tyi * T.th;
    const int z0 = tz * zb, z1 = min(g.nz, z0 + zb);
    const cx<TB>* br = b + (long long)r * b_rstride;
    const cx<R>* er = ec + (long long)r * gc.n;
    const LevelCoef<R> L = level_coef<R>(g, beta1, beta2, omega);

    // this lane's region node: fine in-plane offset (mirrored into the grid),
    // face count in the plane, the coarse corners and weights of its interpolation
    const bool in_region = t < RW * RH;
    const int ly = t / RW, lx = t - ly * RW;
    const int gxr = X0 - 1 + lx, gyr = Y0 - 1 + ly;
    const int gx = mirror_clamp(gxr, g.nx), gy = mirror_clamp(gyr, g.ny);
    const int uoff = gy * g.nx + gx;
    const int unf = (gx == 0) + (gx == g.nx - 1) + (gy == 0) + (gy == g.ny - 1);
    const int cx0 = gx >> 1, cx1 = min((gx >> 1) + (gx & 1), gc.nx - 1);
    const int cy0 = (gy >> 1) * gc.nx, cy1 = min((gy >> 1) + (gy & 1), gc.ny - 1) * gc.nx;
    const R ax = (gx & 1) ? R(0.5) : R(1), ay = (gy & 1) ? R(0.5) : R(1);
    const R bx = R(1) - ax, by = R(1) - ay;
    // output lanes: inside the halo and on the grid
    const bool own = in_region && lx >= 1 && lx <= T.tw && ly >= 1 && ly <= T.th && gxr < g.nx &&
                     gyr < g.ny;

    // shift c of a node, made with its u2 and kept for its output step; in
    // double precision also its Jacobi weight W = omega / (6/h^2 - c) (in
    // single precision recomputing W is cheaper than the registers that
    // would push the pass past its occupancy bound)
    constexpr bool KEEP_W = sizeof(R) == sizeof(double);
    struct CW {
        cx<R> c, w;
    };
    cx<TO>* orr = out + (long long)r * o_rstride;
    const long long ooff = own ? (long long)gyr * g.nx + gxr : 0;
    // u3 of plane z at the output lanes, from the u2 ring and this lane's u2, b, c.
    // Past the bottom / top plane the stencil reads the mirror image, plane 1 /
    // nz - 2 (the eliminated ghost point), whose u2 is already in the ring.
    auto emit = [&](int z, const cx<R>& u, const CW& k, const cx<TB>& bz) {
        if (own) {
            const cx<R>* um = us[ring4i(z == 0 ? 1 : z - 1)];
            const cx<R>* uc = us[ring4i(z)];
            const cx<R>* up = us[ring4i(z == g.nz - 1 ? g.nz - 2 : z + 1)];
            cx<R> lap = (u - uc[t - 1]) + (u - uc[t + 1]);
            lap = lap + (u - uc[t - RW]);
            lap = lap + (u - uc[t + RW]);
            lap = lap + (u - um[t]);
            lap = lap + (u - up[t]);
            const cx<R> wj = KEEP_W ? k.w : jacobi_w(L, k.c);
            cx<R> v = cfma(wj, mresid(cvt<R>(bz), L.ih2, lap, k.c, u), u);
            if (BC == BC_DIRICHLET && (unf || z == 0 || z == g.nz - 1)) v = czero<R>();
            cx<TO>* o = orr + (long long)z * g.plane + ooff;
            if constexpr (ACC) v = cvt<R>(*o) + v;  // out already holds an earlier cycle's result
            *o = cvt<TO>(v);
        }
    };
    // per plane this lane keeps its own u2, b, c for the output step
    cx<R> u_cur;
    CW c_cur, c_nxt, c_unused;
    cx<TB> b_cur, b_nxt;
    {
        // March over the u2 planes z0 - 1 .. z1 clamped into the grid (the
        // output step reads a mirrored plane's image instead), two planes of
        // loads in flight.  Plane f interpolates between coarse planes
        // c0 = f >> 1 and c1 = c0 + (f & 1).  The in-plane interpolation on
        // c0 is the previous plane's, and for even f c1 = c0: only odd planes
        // load coarse values (a branch on the plane, the same for every lane).
        const int plo = max(z0 - 1, 0), phi = min(z1, g.nz - 1);
        auto clampz = [&](int f) { return min(max(f, plo), phi); };
        struct RawC {
            cx<TB> b;
            R k;
            cx<R> e[4];  // the four corners on c1, odd planes only
        };
        auto fetch_c = [&](int f, RawC& v) {
            const int fc = clampz(f);
            const long long base = (long long)fc * g.plane;
            v.b = br[base + uoff];
            v.k = kl[base + uoff];
            if (fc & 1) {
                const cx<R>* e1 = er + (long long)((fc >> 1) + 1) * gc.plane;
                v.e[0] = e1[cy0 + cx0];
                v.e[1] = e1[cy0 + cx1];
                v.e[2] = e1[cy1 + cx0];
                v.e[3] = e1[cy1 + cx1];
            }
        };
        auto interp = [&](const cx<R>& e00, const cx<R>& e01, const cx<R>& e10, const cx<R>& e11) -> cx<R> {
            const cx<R> p0 = lerp2(ax, e00, bx, e01);
            const cx<R> p1 = lerp2(ax, e10, bx, e11);
            return lerp2(ay, p0, by, p1);
        };
        cx<R> carry;  // in-plane interpolation on the previous plane's c1
        auto make_c = [&](int f, const RawC& v, CW& k_out) -> cx<R> {
            const int fc = clampz(f);
            const int zf = (fc == 0) + (fc == g.nz - 1);
            const R wz = (fc & 1) ? R(0.5) : R(1), bz = R(1) - wz;
            const cx<R> pn = (fc & 1) ? interp(v.e[0], v.e[1], v.e[2], v.e[3]) : carry;
            const cx<R> pe = lerp2(wz, (fc & 1) ? carry : pn, bz, pn);
            carry = pn;
            const int nf = BC == BC_SOMMERFELD ? unf + zf : 0;
            k_out.c = shift_c(L, v.k, nf);
            const cx<R> wj = jacobi_w(L, k_out.c);
            if constexpr (KEEP_W) k_out.w = wj;
            cx<R> u = cfma(wj, cvt<R>(v.b), pe);
            if (BC == BC_DIRICHLET && (unf || zf)) u = czero<R>();
            us[ring4i(f)][t] = u;  // unguarded: lanes past the region write slots never read
            return u;
        };
        auto step = [&](int z, RawC& v) {
            b_nxt = v.b;
            const cx<R> u_nxt = make_c(z + 1, v, c_nxt);
            fetch_c(z + 3, v);
            __syncthreads();
            emit(z, u_cur, c_cur, b_cur);
            u_cur = u_nxt;
            c_cur = c_nxt;
            b_cur = b_nxt;
        };
        // set A holds the planes z0 - 1 + even, set B the odd ones
        RawC A, B;
        fetch_c(z0 - 1, A);
        fetch_c(z0, B);
        {
            // the in-plane interpolation on coarse plane c0 of the first plane
            const cx<R>* e0 = er + (long long)(plo >> 1) * gc.plane;
            carry = interp(e0[cy0 + cx0], e0[cy0 + cx1], e0[cy1 + cx0], e0[cy1 + cx1]);
        }
        (void)make_c(z0 - 1, A, c_unused);
        fetch_c(z0 + 1, A);
        b_cur = B.b;
        u_cur = make_c(z0, B, c_cur);
        fetch_c(z0 + 2, B);
        for (int z = z0; z < z1; z += 2) {
            step(z, A);
            if (z + 1 >= z1) break;
            step(z + 1, B);
        }
    }
}

// ---------------------------------------------------------------------------
// Up: u3 = u2 + W (b - (1/h^2) lap(u2) + c u2), u2 = W b + P e_H.  Each lane
// owns an x-pair of the tile-plus-halo region: nodes x_a = X0 - 1 + 2 p and
// x_b = x_a + 1 of region row ly.  The two nodes' trilinear interpolations
// draw on the same two coarse columns (two columns on the two coarse rows of
// its fine row), so a lane interpolates each column in y and z once.  The
// coarse values come from LDS: every second fine plane starts a new coarse
// plane, whose window for the tile is loaded one node per lane a plane ahead
// and staged before the barrier that precedes its use.  The workgroup marches
// over `zb` planes; the u2 planes go to a ring of four LDS planes, one barrier
// per plane.  Every node's arithmetic is the same for every tile and z-block,
// so the result does not depend on them.  With ACC the pass adds u3 to the
// output instead of storing it (the F-cycle's second coarse-grid cycle).
// ---------------------------------------------------------------------------
template <typename R>
constexpr int UP_WAVES_PER_SIMD = 4;  // two 512-lane workgroups per CU

template <int BC, typename TB, typename R, typename TO, bool ACC>
__global__ __launch_bounds__(UP_LANES, UP_WAVES_PER_SIMD<R>) void k_mg_up(Geo g, Geo gc, int zb,
                                                    const cx<TB>* __restrict__ b, long long b_rstride,
                                                    const R* __restrict__ kl, double beta1,
                                                    double beta2, double omega,
                                                    const cx<R>* __restrict__ ec,
                                                    cx<TO>* __restrict__ out, long long o_rstride,
                                                    const RhsState* st, int gate) {
    // a ring of four u2 planes: the output step of plane z reads planes z - 1
    // and z while plane z + 1 is written, so one barrier per plane suffices.
    // Each plane holds the region's a nodes (even region columns) in its
    // first half and the b nodes (odd columns) in its second: consecutive
    // lanes touch consecutive slots.
    __shared__ cx<R> us[4][2 * UP_LANES];
    // the tile's coarse window of one coarse plane (see up_coarse_window)
    __shared__ cx<R> cs[UP_LANES];

    const int r = blockIdx.z;
    if (!gate_ok(st, r, gate)) return;
    const int t = threadIdx.x;
    const TileShape T = up_tile_shape(g.nx, g.ny);
    const int P = (T.tw + 2) / 2;  // x-pairs per region row
    const int id = xcd_tile_id(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
    const int tz = id / gridDim.x;
    const int txy = id - tz * gridDim.x;
    const int tyi = txy / T.ntx, txi = txy - tyi * T.ntx;
    const int X0 = txi * T.tw, Y0 = tyi * T.th;
    const int z0 = tz * zb, z1 = min(g.nz, z0 + zb);
    const cx<TB>* br = b + (long long)r * b_rstride;
    const cx<R>* er = ec + (long long)r * gc.n;
    const LevelCoef<R> L = level_coef<R>(g, beta1, beta2, omega);

    // this lane's pair: region row ly, nodes at region columns 2 px, 2 px + 1
    const int ly = t / P, px = t - ly * P;
    const int xa = X0 - 1 + 2 * px, xb = xa + 1, yr = Y0 - 1 + ly;
    const int gxa = mirror_clamp(xa, g.nx), gxb = mirror_clamp(xb, g.nx), gy = mirror_clamp(yr, g.ny);
    const int offa = gy * g.nx + gxa, offb = gy * g.nx + gxb;
    const int nfxy = (gy == 0) + (gy == g.ny - 1);
    const int nfa = nfxy + (gxa == 0) + (gxa == g.nx - 1), nfb = nfxy + (gxb == 0) + (gxb == g.nx - 1);
    // coarse columns cb, cb + 1 and rows cy0, cy1 of the pair's interpolation
    const int cb = min(gxa >> 1, gxb >> 1), cb1 = min(cb + 1, gc.nx - 1);
    const int cy0 = gy >> 1, cy1 = min(cy0 + (gy & 1), gc.ny - 1);
    const int e00 = cy0 * gc.nx + cb, e01 = cy0 * gc.nx + cb1, e10 = cy1 * gc.nx + cb, e11 = cy1 * gc.nx + cb1;
    // linear interpolation weights on the two points of an axis: an odd fine
    // index takes 1/2 of each, an even one all of its own coarse point
    const R ay = (gy & 1) ? R(0.5) : R(1), by = R(1) - ay;
    const R wa0 = (gxa & 1) ? R(0.5) : ((gxa >> 1) == cb ? R(1) : R(0)), wa1 = R(1) - wa0;
    const R wb0 = (gxb & 1) ? R(0.5) : ((gxb >> 1) == cb ? R(1) : R(0)), wb1 = R(1) - wb0;
    // output nodes: inside the halo and on the grid
    const bool rows_own = ly >= 1 && ly <= T.th && yr < g.ny;
    const bool own_a = rows_own && 2 * px >= 1 && 2 * px <= T.tw && xa < g.nx;
    const bool own_b = rows_own && 2 * px + 1 <= T.tw && xb < g.nx;
    // LDS slots: node a at t (first half), node b at UP_LANES + t; the row
    // neighbours of a slot are P slots away
    const int sa = t, sb = UP_LANES + t;
    // the coarse window: lane t stages window node t; the pair's four corners
    // as window slots (clamped: lanes whose nodes lie outside are never used)
    const CoarseWin win = up_coarse_window(X0, Y0, T.tw, T.th, gc.nx, gc.ny);
    const bool stager = t < win.cw * win.ch;
    const int soff = (win.cy0 + min(t / win.cw, win.ch - 1)) * gc.nx + win.cx0 + t % win.cw;
    auto wslot = [&](int cyy, int cxx) {
        return min(max(cyy - win.cy0, 0), win.ch - 1) * win.cw + min(max(cxx - win.cx0, 0), win.cw - 1);
    };
    const int s00 = wslot(cy0, cb), s01 = wslot(cy0, cb1), s10 = wslot(cy1, cb), s11 = wslot(cy1, cb1);

    // raw loads of one plane: b and k of both nodes and, when plane f + 1 is
    // odd, this lane's window node of its coarse plane c1 = (f + 1) / 2 + 1
    // (plane f interpolates between coarse planes c0 = f >> 1 and
    // c1 = c0 + (f & 1); even planes reuse the previous plane's in-plane
    // interpolation).  Issued unconditionally within the plane (every offset
    // is a valid node); planes are clamped into plo .. phi.
    const int plo = max(z0 - 1, 0), phi = min(z1, g.nz - 1);
    auto clampz = [&](int f) { return min(max(f, plo), phi); };
    struct Raw {
        cx<TB> ba, bb;
        R ka, kb;
        cx<R> ce;
    };
    auto fetch = [&](int f, Raw& v) {
        const int fc = clampz(f), fn = clampz(f + 1);
        const long long base = (long long)fc * g.plane;
        v.ba = br[base + offa];
        v.bb = br[base + offb];
        v.ka = kl[base + offa];
        v.kb = kl[base + offb];
        if (fn & 1) v.ce = er[(long long)((fn >> 1) + 1) * gc.plane + soff];
        __builtin_amdgcn_sched_barrier(0);
    };
    // stage the window of plane f's c1 (from the set fetched for f - 1) when
    // f is odd and not a clamped repeat of f - 1
    auto stage_at = [&](int f) { return (clampz(f) & 1) && clampz(f) != clampz(f - 1); };
    auto stage = [&](const Raw& v) {
        if (stager) cs[t] = v.ce;
    };
    static_assert(sizeof(R) == sizeof(float), "the x-pair up pass runs in single precision");
    // per node and plane: u2 and the b, c and W its output step needs
    struct Node {
        cx<R> u, b, c, w;
    };
    struct Pair {
        Node a, b;
    };
    cx<R> carry0, carry1;  // y-interpolated coarse columns of the previous plane's c1
    // u2 of plane f for both nodes, staged in the ring
    auto make = [&](int f, const Raw& v, Pair& o) {
        const int fc = clampz(f);
        const int zf = (fc == 0) + (fc == g.nz - 1);
        // y on the new coarse plane c1 (for even f the previous plane's), then
        // z with the previous plane's c1 (= this plane's c0 for odd f), then x
        const R wz = (fc & 1) ? R(0.5) : R(1), bz = R(1) - wz;
        const cx<R> p0 = (fc & 1) ? lerp2(ay, cs[s00], by, cs[s10]) : carry0;
        const cx<R> p1 = (fc & 1) ? lerp2(ay, cs[s01], by, cs[s11]) : carry1;
        const cx<R> q0 = lerp2(wz, (fc & 1) ? carry0 : p0, bz, p0);
        const cx<R> q1 = lerp2(wz, (fc & 1) ? carry1 : p1, bz, p1);
        carry0 = p0;
        carry1 = p1;
        const cx<R> pea = lerp2(wa0, q0, wa1, q1);
        const cx<R> peb = lerp2(wb0, q0, wb1, q1);
        o.a.b = cvt<R>(v.ba);
        o.b.b = cvt<R>(v.bb);
        o.a.c = shift_c(L, v.ka, BC == BC_SOMMERFELD ? nfa + zf : 0);
        o.b.c = shift_c(L, v.kb, BC == BC_SOMMERFELD ? nfb + zf : 0);
        o.a.w = jacobi_w(L, o.a.c);
        o.b.w = jacobi_w(L, o.b.c);
        o.a.u = cfma(o.a.w, o.a.b, pea);
        o.b.u = cfma(o.b.w, o.b.b, peb);
        if (BC == BC_DIRICHLET && (nfa || zf)) o.a.u = czero<R>();
        if (BC == BC_DIRICHLET && (nfb || zf)) o.b.u = czero<R>();
        cx<R>* dst = us[f & 3];  // f >= -1: f & 3 is the ring slot (also for -1)
        dst[sa] = o.a.u;
        dst[sb] = o.b.u;
    };

    cx<TO>* orr = out + (long long)r * o_rstride;
    const long long oa = (long long)gy * g.nx + gxa, ob = (long long)gy * g.nx + gxb;
    // u3 of plane z at the pair's output nodes (past the bottom / top plane
    // the z neighbour is the mirror image: plane 1 / nz - 2)
    auto emit = [&](int z, const Pair& c, const Pair& n) {
        const cx<R>* uc = us[z & 3];
        const cx<R>* um = us[(z - 1) & 3];
        const bool bot = z == 0, top = z == g.nz - 1;
        auto out1 = [&](const Node& nd, const cx<R>& xm, const cx<R>& xp, const cx<R>& ym, const cx<R>& yp,
                        const cx<R>& zm, const cx<R>& zp, int nf, long long off) {
            const cx<R> u = nd.u;
            cx<R> lap = (u - xm) + (u - xp);
            lap = lap + (u - ym);
            lap = lap + (u - yp);
            lap = lap + (u - (bot ? zp : zm));
            lap = lap + (u - (top ? zm : zp));
            cx<R> v = cfma(nd.w, mresid(nd.b, L.ih2, lap, nd.c, u), u);
            if (BC == BC_DIRICHLET && (nf || bot || top)) v = czero<R>();
            cx<TO>* o = orr + (long long)z * g.plane + off;
            if constexpr (ACC) v = cvt<R>(*o) + v;  // out already holds an earlier cycle's result
            *o = cvt<TO>(v);
        };
        if (own_a)  // x - 1: the b node of the pair to the left; x + 1: this pair's b node
            out1(c.a, uc[sb - 1], c.b.u, uc[sa - P], uc[sa + P], um[sa], n.a.u, nfa, oa);
        if (own_b)  // x - 1: this pair's a node; x + 1: the a node of the pair to the right
            out1(c.b, c.a.u, uc[sa + 1], uc[sb - P], uc[sb + P], um[sb], n.b.u, nfb, ob);
    };

    // carry for the first plane: the y-interpolated columns of coarse plane plo >> 1
    {
        const cx<R>* e0 = er + (long long)(plo >> 1) * gc.plane;
        carry0 = lerp2(ay, e0[e00], by, e0[e10]);
        carry1 = lerp2(ay, e0[e01], by, e0[e11]);
    }
    // u2 on planes z0 - 1 .. z1 (clamped into the grid; a clamped duplicate is
    // never read).  Two pair sets X, Y alternate as the current and the next
    // plane, and two planes of loads are in flight (set A holds the planes
    // z0 - 1 + even, set B the odd ones).
    Pair X, Y;
    auto step = [&](int z, Pair& cur, Pair& nxt, Raw& v, int ahead) {
        make(z + 1, v, nxt);
        if (stage_at(z + 2)) stage(v);
        fetch(z + 1 + ahead, v);
        __syncthreads();
        emit(z, cur, nxt);
    };
    Raw A, B;
    fetch(z0 - 1, A);
    fetch(z0, B);
    if ((plo & 1) && stager) cs[t] = er[(long long)((plo >> 1) + 1) * gc.plane + soff];
    // the window is read only by odd planes and written only for an odd plane
    // when the plane before it (even) is made: a barrier between each write
    // and its reads, and between the reads and the next write
    __syncthreads();
    make(z0 - 1, A, Y);
    if (stage_at(z0)) stage(A);
    __syncthreads();
    fetch(z0 + 1, A);
    make(z0, B, X);
    if (stage_at(z0 + 1)) stage(B);
    __syncthreads();
    fetch(z0 + 2, B);
    for (int z = z0; z < z1; z += 2) {
        step(z, X, Y, A, 2);
        if (z + 1 >= z1) break;
        step(z + 1, Y, X, B, 2);
    }
}

// ---------------------------------------------------------------------------
// Residual in place: b = b - M e = b - (1/h^2) lap(e) + c e on a level below
// the finest (the F-cycle's second coarse-grid cycle starts from it).  One
// lane per in-plane node marching over `zb` planes; the neighbours are read
// straight from global memory (the x and y ones from lines the workgroup
// loads anyway, the z ones from the previous planes, in L2).
// ---------------------------------------------------------------------------
constexpr int RS_LANES = 256;

template <int BC, typename R>
__global__ __launch_bounds__(RS_LANES) void k_mg_resid(Geo g, int zb, cx<R>* __restrict__ b,
                                                       const cx<R>* __restrict__ e,
                                                       const R* __restrict__ kl, double beta1,
                                                       double beta2, double omega, const RhsState* st,
                                                       int gate) {
    const int r = blockIdx.z;
    if (!gate_ok(st, r, gate)) return;
    const int i = blockIdx.x * RS_LANES + threadIdx.x;
    if (i >= g.plane) return;
    const int y = i / g.nx, x = i - y * g.nx;
    const int z0 = blockIdx.y * zb, z1 = min(g.nz, z0 + zb);
    const LevelCoef<R> L = level_coef<R>(g, beta1, beta2, omega);
    // neighbour offsets, a missing neighbour replaced by its mirror image
    const int dxm = x > 0 ? -1 : 1, dxp = x < g.nx - 1 ? 1 : -1;
    const int dym = y > 0 ? -g.nx : g.nx, dyp = y < g.ny - 1 ? g.nx : -g.nx;
    const int nfxy = (x == 0) + (x == g.nx - 1) + (y == 0) + (y == g.ny - 1);
    cx<R>* br = b + (long long)r * g.n;
    const cx<R>* er = e + (long long)r * g.n;
    for (int z = z0; z < z1; ++z) {
        const long long j = (long long)z * g.plane + i;
        const long long dzm = z > 0 ? -(long long)g.plane : g.plane;
        const long long dzp = z < g.nz - 1 ? g.plane : -(long long)g.plane;
        const cx<R> u = er[j];
        cx<R> lap = (u - er[j + dxm]) + (u - er[j + dxp]);
        lap = lap + (u - er[j + dym]);
        lap = lap + (u - er[j + dyp]);
        lap = lap + (u - er[j + dzm]);
        lap = lap + (u - er[j + dzp]);
        const int nf = nfxy + (z == 0) + (z == g.nz - 1);
        const cx<R> c = shift_c(L, kl[j], BC == BC_SOMMERFELD ? nf : 0);
        cx<R> v = mresid(br[j], L.ih2, lap, c, u);
        if (BC == BC_DIRICHLET && nf) v = czero<R>();
        br[j] = v;
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
int mg_down_blocks(const Geo& gc, int zbc) {
    const TileShape T = dn_tile_shape(gc.nx, gc.ny, DN_REGION);
    return T.ntx * T.nty * ((gc.nz + zbc - 1) / zbc);
}
int mg_up_blocks(const Geo& g, int zb, bool single) {
    const TileShape T = single ? up_tile_shape(g.nx, g.ny) : up1_tile_shape(g.nx, g.ny);
    return T.ntx * T.nty * ((g.nz + zb - 1) / zb);
}
bool mg_up_windows_fit(const Geo& g, const Geo& gc) {
    const TileShape T = up_tile_shape(g.nx, g.ny);
    for (int ty = 0; ty < T.nty; ++ty)
        for (int tx = 0; tx < T.ntx; ++tx) {
            const CoarseWin W = up_coarse_window(tx * T.tw, ty * T.th, T.tw, T.th, gc.nx, gc.ny);
            if (W.cw < 1 || W.ch < 1 || W.cw * W.ch > UP_LANES) return false;
        }
    return true;
}

// Region of the down pass.  The z-marching pass (zbc > 1, the large levels)
// keeps DN_REGION.  The one-plane pass runs on the small levels, where the
// chain of region nodes a lane works through (REG / DN_LANES per plane) sets
// the duration: a smaller region is taken when region nodes per lane times
// waves per SIMD (rounded up; 256 CUs of 4 SIMDs) drops by at least 10 %.
// Every node's arithmetic is the same for every region, so the output is too.
int dn_region(const Geo& gc, int zbc, int nrhs) {
    if (zbc != 1) return DN_REGION;
    auto cost = [&](int reg) {
        const TileShape T = dn_tile_shape(gc.nx, gc.ny, reg);
        const long long waves = (long long)T.ntx * T.nty * gc.nz * nrhs * (DN_LANES / 64);
        return (double)(reg / DN_LANES) * (double)((waves + 1023) / 1024);
    };
    int best = DN_REGION;
    double cbest = cost(DN_REGION);
    for (int reg : {512, 256}) {
        const double cr = cost(reg);
        if (cr < 0.9 * cbest) {
            best = reg;
            cbest = cr;
        }
    }
    return best;
}

int mg_down_region(const Geo& gc, int zbc, int nrhs, int want) {
    if (zbc != 1) return DN_REGION;
    if (want == 256 || want == 512 || want == DN_REGION) return want;
    return dn_region(gc, zbc, nrhs);
}

template <typename TB, typename R>
void launch_mg_down(hipStream_t s, int bc, const Geo& gf, const Geo& gc, int zbc, int nrhs,
                    const cx<TB>* b, long long b_rstride, const R* kl, const MgParams& P,
                    cx<R>* bc_out, const RhsState* st, int gate, int reg_want) {
    const int reg = mg_down_region(gc, zbc, nrhs, reg_want);
    const TileShape T = dn_tile_shape(gc.nx, gc.ny, reg);
    dim3 grid(T.ntx * T.nty, (gc.nz + zbc - 1) / zbc, nrhs);
#define HH_DOWN(BCV, ONEV, REGV)                                                                                \
    hipLaunchKernelGGL((k_mg_down<BCV, TB, R, ONEV, REGV>), grid, dim3(DN_LANES), 0, s, gf, gc, zbc, b, b_rstride, \
                       kl, P.beta1, P.beta2, P.omega, bc_out, st, gate)
#define HH_DOWN_BC(BCV)                                   \
    if (zbc != 1) HH_DOWN(BCV, false, DN_REGION);         \
    else if (reg == 256) HH_DOWN(BCV, true, 256);         \
    else if (reg == 512) HH_DOWN(BCV, true, 512);         \
    else HH_DOWN(BCV, true, DN_REGION);
    if (bc == BC_SOMMERFELD) {
        HH_DOWN_BC(BC_SOMMERFELD)
    } else {
        HH_DOWN_BC(BC_DIRICHLET)
    }
#undef HH_DOWN_BC
#undef HH_DOWN
}

template <typename TB, typename R, typename TO>
void launch_mg_up(hipStream_t s, int bc, const Geo& g, const Geo& gc, int zb, int nrhs,
                  const cx<TB>* b, long long b_rstride, const R* kl, const MgParams& P,
                  const cx<R>* ec, cx<TO>* out, long long o_rstride, const RhsState* st, int gate,
                  bool acc) {
    constexpr bool PAIRS = sizeof(R) == sizeof(float);  // x-pair kernel in single precision
    const TileShape T = PAIRS ? up_tile_shape(g.nx, g.ny) : up1_tile_shape(g.nx, g.ny);
    dim3 grid(T.ntx * T.nty, (g.nz + zb - 1) / zb, nrhs);
#define HH_UP(BCV, ACCV)                                                                                 \
    if constexpr (PAIRS)                                                                                \
        hipLaunchKernelGGL((k_mg_up<BCV, TB, R, TO, ACCV>), grid, dim3(UP_LANES), 0, s, g, gc, zb, b,     \
                           b_rstride, kl, P.beta1, P.beta2, P.omega, ec, out, o_rstride, st, gate);      \
    else                                                                                                \
        hipLaunchKernelGGL((k_mg_up1<BCV, TB, R, TO, ACCV>), grid, dim3(UP_LANES), 0, s, g, gc, zb, b,    \
                           b_rstride, kl, P.beta1, P.beta2, P.omega, ec, out, o_rstride, st, gate)
#define HH_UP_BC(ACCV)                     \
    if (bc == BC_SOMMERFELD) {             \
        HH_UP(BC_SOMMERFELD, ACCV);        \
    } else {                               \
        HH_UP(BC_DIRICHLET, ACCV);         \
    }
    // accumulation only on the levels below the finest, where input, compute
    // and output precision are one
    if constexpr (std::is_same<TB, R>::value && std::is_same<TO, R>::value) {
        if (acc) {
            HH_UP_BC(true)
            return;
        }
    }
    HH_UP_BC(false)
#undef HH_UP_BC
#undef HH_UP
}

template <typename R>
void launch_mg_resid(hipStream_t s, int bc, const Geo& g, int nrhs, cx<R>* b, const cx<R>* e, const R* kl,
                     const MgParams& P, const RhsState* st, int gate) {
    // about four planes per lane, enough workgroups to spread over the chip
    const int bx = (g.plane + RS_LANES - 1) / RS_LANES;
    int zb = 4;
    while (zb > 1 && (long long)bx * ((g.nz + zb - 1) / zb) * nrhs < 1024) zb >>= 1;
    dim3 grid(bx, (g.nz + zb - 1) / zb, nrhs);
    if (bc == BC_SOMMERFELD)
        hipLaunchKernelGGL((k_mg_resid<BC_SOMMERFELD, R>), grid, dim3(RS_LANES), 0, s, g, zb, b, e, kl,
                           P.beta1, P.beta2, P.omega, st, gate);
    else
        hipLaunchKernelGGL((k_mg_resid<BC_DIRICHLET, R>), grid, dim3(RS_LANES), 0, s, g, zb, b, e, kl,
                           P.beta1, P.beta2, P.omega, st, gate);
}
template void launch_mg_resid<double>(hipStream_t, int, const Geo&, int, c128*, const c128*, const double*,
                                      const MgParams&, const RhsState*, int);
template void launch_mg_resid<float>(hipStream_t, int, const Geo&, int, c64*, const c64*, const float*,
                                     const MgParams&, const RhsState*, int);

#define HH_INST_F(TB, R, TO)                                                                           \
    template void launch_mg_down<TB, R>(hipStream_t, int, const Geo&, const Geo&, int, int, const cx<TB>*, \
                                        long long, const R*, const MgParams&, cx<R>*, const RhsState*,   \
                                        int, int);                                                        \
    template void launch_mg_up<TB, R, TO>(hipStream_t, int, const Geo&, const Geo&, int, int,              \
                                          const cx<TB>*, long long, const R*, const MgParams&,            \
                                          const cx<R>*, cx<TO>*, long long, const RhsState*, int, bool);
HH_INST_F(double, double, double)
HH_INST_F(double, float, double)
HH_INST_F(float, float, float)
#undef HH_INST_F

}  // namespace hh
