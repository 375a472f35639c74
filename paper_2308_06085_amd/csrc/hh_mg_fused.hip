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
// Up (Algorithm 1 steps 5-7: trilinear prolongation of section 3.4.3,
// correction, one damped-Jacobi sweep):
//   u2 = W b + P e_H,   u3 = u2 + W (b - (1/h^2) lap(u2) + c u2).
//
// The Laplacian is summed as differences u_j - u_nb: for the smooth part of u
// each difference is exact in floating point, so the correction keeps its
// relative accuracy in single precision instead of losing a factor of about
// 6 / (k h)^2 to cancellation in 6 u_j - sum u_nb.
//
// Only the level's k^2 is stored; c, D and W are recomputed per node.  Both
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
__device__ __forceinline__ int ring4(int f) { return f & 3; }  // also for f = -1

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
constexpr int UP_LANES = 512, UP_MAXW = 32;  // up pass: one lane per region node
// Tile of the up pass: the tile plus a one-node halo must fit the lanes,
// (tw + 2)(th + 2) <= lanes.
__host__ __device__ inline TileShape up_tile_shape(int nx, int ny) {
    TileShape T;
    T.ntx = (nx + UP_MAXW - 1) / UP_MAXW;
    T.tw = (nx + T.ntx - 1) / T.ntx;
    T.th = UP_LANES / (T.tw + 2) - 2;
    if (T.th > ny) T.th = ny;
    T.nty = (ny + T.th - 1) / T.th;
    return T;
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

// Square root and reciprocal: correctly rounded in double; in single precision
// the hardware v_sqrt_f32 / v_rcp_f32 (about 1 ulp), far inside the accuracy a
// complex64 V-cycle is held to.
__device__ __forceinline__ double mg_sqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float mg_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double mg_rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float mg_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// c_j = (beta1 - beta2 i) k^2 + n_j 2 i k / h
template <typename R>
__device__ __forceinline__ cx<R> shift_c(const LevelCoef<R>& L, R k2, int nf) {
    cx<R> c = {L.sr * k2, L.si * k2};
    if (nf) c.im += R(nf) * L.two_over_h * mg_sqrt(k2);
    return c;
}
// W = omega / (6/h^2 - c)
template <typename R>
__device__ __forceinline__ cx<R> jacobi_w(const LevelCoef<R>& L, cx<R> c) {
    const R dr = L.six_ih2 - c.re, di = -c.im;
    const R s = L.omega * mg_rcp(dr * dr + di * di);
    return {dr * s, -di * s};
}

__device__ __forceinline__ int faces_of(int x, int y, int z, const Geo& g) {
    return (x == 0) + (x == g.nx - 1) + (y == 0) + (y == g.ny - 1) + (z == 0) + (z == g.nz - 1);
}

// ---------------------------------------------------------------------------
// Down: b_H = R (b - M W b).  The workgroup owns a tw x th tile of coarse
// columns and marches over `zbc` coarse planes (2 zbc + 1 fine residual
// planes).  Each lane owns NU nodes of the fine region (tile plus a two-node
// halo): it loads their b and k^2, writes u1 = W b to the LDS ring, and keeps
// b and c in registers for the residual of the same nodes one plane later, so
// every input is read once per plane.  Two planes of loads are in flight.
// ---------------------------------------------------------------------------
template <typename TB, typename R, int NU>
struct DownRaw {
    cx<TB> b[NU];
    R k[NU];
};
template <typename R, int NU>
struct DownKeep {
    cx<R> b[NU];
    cx<R> c[NU];
};

template <int BC, typename TB, typename R, bool ONE, int REG>
__global__ __launch_bounds__(DN_LANES) void k_mg_down(Geo gf, Geo gc, int zbc,
                                                      const cx<TB>* __restrict__ b,
                                                      long long b_rstride,
                                                      const R* __restrict__ k2l, double beta1,
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
            w.k[k] = k2l[base + uoff[k]];
        }
        // keep the scheduler from moving these loads past later ones: loads
        // complete in issue order, so a plane must be issued as one group
        __builtin_amdgcn_sched_barrier(0);
    };
    // u1 = W b to the ring; b and c kept for this plane's residual
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
            cx<R> v = jacobi_w(L, c) * bb;
            if (BC == BC_DIRICHLET && (ubnd[k] || zf)) v = czero<R>();
            // unguarded: idx < NU * DN_LANES = REG, and slots past the
            // region are never read (a guard would sink the loads into it)
            dst[idx] = v;
            kp.b[k] = bb;
            kp.c[k] = c;
        }
    };
    // r = b - (1/h^2) lap(u1) + c u1 on the region's inner nodes
    auto residual = [&](int f, const DownKeep<R, NU>& kp) {
        const cx<R>* um = u1s[ring3(f - 1)];
        const cx<R>* uc = u1s[ring3(f)];
        const cx<R>* up = u1s[ring3(f + 1)];
#pragma unroll
        for (int k = 0; k < NU; ++k) {
            if (uin[k]) {
                const int c = t + k * DN_LANES;
                const cx<R> u = uc[c];
                cx<R> lap = (u - uc[c - 1]) + (u - uc[c + 1]);
                lap = lap + (u - uc[c - RW]);
                lap = lap + (u - uc[c + RW]);
                lap = lap + (u - um[c]);
                lap = lap + (u - up[c]);
                rs[c] = (kp.b[k] - L.ih2 * lap) + kp.c[k] * u;
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
// compute the output.  The workgroup marches over `zb` planes.  With ACC the
// pass adds u3 to the output instead of storing it (the F-cycle's second
// coarse-grid cycle).
// ---------------------------------------------------------------------------
// Waves per SIMD the up pass is compiled for: three 512-lane workgroups per CU
// in single precision (<= 80 VGPRs), two in double (<= 128 VGPRs).
template <typename R>
constexpr int UP_WAVES_PER_SIMD = sizeof(R) == sizeof(float) ? 6 : 4;

template <int BC, typename TB, typename R, typename TO, bool ONE, bool ACC>
__global__ __launch_bounds__(UP_LANES, UP_WAVES_PER_SIMD<R>) void k_mg_up(Geo g, Geo gc, int zb,
                                                    const cx<TB>* __restrict__ b, long long b_rstride,
                                                    const R* __restrict__ k2l, double beta1,
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
    const TileShape T = up_tile_shape(g.nx, g.ny);
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

    // raw loads of one plane: b, k^2 and the eight coarse corners.  Loads are
    // issued unconditionally (every offset is a valid node); a plane past the
    // chunk's last one re-reads that plane instead (an L2 hit).
    struct Raw {
        cx<TB> b;
        R k;
        cx<R> e[8];
    };
    // shift c of a node, made with its u2 and kept for its output step; in
    // double precision also its Jacobi weight W = omega / (6/h^2 - c) (in
    // single precision recomputing W is cheaper than the registers that
    // would push the pass past its occupancy bound)
    constexpr bool KEEP_W = sizeof(R) == sizeof(double);
    struct CW {
        cx<R> c, w;
    };
    auto fetch = [&](int f, Raw& w) {
        const int fz = mirror_clamp(min(f, z1), g.nz);
        const long long base = (long long)fz * g.plane;
        const cx<R>* e0 = er + (long long)(fz >> 1) * gc.plane;
        const cx<R>* e1 = er + (long long)min((fz >> 1) + (fz & 1), gc.nz - 1) * gc.plane;
        w.b = br[base + uoff];
        w.k = k2l[base + uoff];
        w.e[0] = e0[cy0 + cx0];
        w.e[1] = e0[cy0 + cx1];
        w.e[2] = e0[cy1 + cx0];
        w.e[3] = e0[cy1 + cx1];
        w.e[4] = e1[cy0 + cx0];
        w.e[5] = e1[cy0 + cx1];
        w.e[6] = e1[cy1 + cx0];
        w.e[7] = e1[cy1 + cx1];
    };
    // u2 at this lane's node of plane f, also written to the ring for the
    // stencil of the output lanes; c is returned for the output step
    auto make_u2 = [&](int f, const Raw& w, CW& k_out) -> cx<R> {
        const int fz = mirror_clamp(f, g.nz);
        const int zf = (fz == 0) + (fz == g.nz - 1);
        const R wz = (fz & 1) ? R(0.5) : R(1), bz = R(1) - wz;
        // trilinear interpolation; an even index takes its own coarse node only
        const cx<R> p0 = ax * w.e[0] + bx * w.e[1];
        const cx<R> p1 = ax * w.e[2] + bx * w.e[3];
        const cx<R> p2 = ax * w.e[4] + bx * w.e[5];
        const cx<R> p3 = ax * w.e[6] + bx * w.e[7];
        const cx<R> pe = wz * (ay * p0 + by * p1) + bz * (ay * p2 + by * p3);
        const int nf = BC == BC_SOMMERFELD ? unf + zf : 0;
        k_out.c = shift_c(L, w.k, nf);
        const cx<R> wj = jacobi_w(L, k_out.c);
        if constexpr (KEEP_W) k_out.w = wj;
        cx<R> v = wj * cvt<R>(w.b) + pe;
        if (BC == BC_DIRICHLET && (unf || zf)) v = czero<R>();
        us[ring4(f)][t] = v;  // unguarded: lanes past the region write slots never read
        return v;
    };

    cx<TO>* orr = out + (long long)r * o_rstride;
    const long long ooff = own ? (long long)gyr * g.nx + gxr : 0;
    // u3 of plane z at the output lanes, from the u2 ring and this lane's u2, b, c.
    // Past the bottom / top plane the stencil reads the mirror image, plane 1 /
    // nz - 2 (the eliminated ghost point), whose u2 is already in the ring.
    auto emit = [&](int z, const cx<R>& u, const CW& k, const cx<TB>& bz) {
        if (own) {
            const cx<R>* um = us[ring4(z == 0 ? 1 : z - 1)];
            const cx<R>* uc = us[ring4(z)];
            const cx<R>* up = us[ring4(z == g.nz - 1 ? g.nz - 2 : z + 1)];
            cx<R> lap = (u - uc[t - 1]) + (u - uc[t + 1]);
            lap = lap + (u - uc[t - RW]);
            lap = lap + (u - uc[t + RW]);
            lap = lap + (u - um[t]);
            lap = lap + (u - up[t]);
            const cx<R> wj = KEEP_W ? k.w : jacobi_w(L, k.c);
            cx<R> v = u + wj * ((cvt<R>(bz) - L.ih2 * lap) + k.c * u);
            if (BC == BC_DIRICHLET && (unf || z == 0 || z == g.nz - 1)) v = czero<R>();
            cx<TO>* o = orr + (long long)z * g.plane + ooff;
            if constexpr (ACC) v = cvt<R>(*o) + v;  // out already holds an earlier cycle's result
            *o = cvt<TO>(v);
        }
    };
    // per plane this lane keeps its own u2, b, c for the output step
    Raw w, w2;
    cx<R> u_cur;
    CW c_cur, c_nxt, c_unused;
    cx<TB> b_cur, b_nxt;
    if constexpr (ONE) {
        // one plane per workgroup (the small levels, where latency rules):
        // its three planes are loaded in one round
        Raw w3;
        fetch(z0 - 1, w);
        fetch(z0, w2);
        fetch(z0 + 1, w3);
        (void)make_u2(z0 - 1, w, c_unused);
        u_cur = make_u2(z0, w2, c_cur);
        (void)make_u2(z0 + 1, w3, c_unused);
        __syncthreads();
        emit(z0, u_cur, c_cur, w2.b);
    } else {
        // March over the u2 planes z0 - 1 .. z1 clamped into the grid (the
        // output step reads a mirrored plane's image instead), two planes of
        // loads in flight.  Plane f interpolates between coarse planes
        // c0 = f >> 1 and c1 = c0 + (f & 1): only c1 is loaded, the in-plane
        // interpolation on c0 is the previous plane's (the same plane for even f).
        const int plo = max(z0 - 1, 0), phi = min(z1, g.nz - 1);
        struct RawC {
            cx<TB> b;
            R k;
            cx<R> e[4];
        };
        auto fetch_c = [&](int f, RawC& v) {
            const int fc = min(max(f, plo), phi);
            const long long base = (long long)fc * g.plane;
            const cx<R>* e1 = er + (long long)((fc >> 1) + (fc & 1)) * gc.plane;
            v.b = br[base + uoff];
            v.k = k2l[base + uoff];
            v.e[0] = e1[cy0 + cx0];
            v.e[1] = e1[cy0 + cx1];
            v.e[2] = e1[cy1 + cx0];
            v.e[3] = e1[cy1 + cx1];
        };
        auto interp = [&](const cx<R>(&e)[4]) -> cx<R> {
            const cx<R> p0 = ax * e[0] + bx * e[1];
            const cx<R> p1 = ax * e[2] + bx * e[3];
            return ay * p0 + by * p1;
        };
        cx<R> carry;  // in-plane interpolation on the previous plane's c1
        auto make_c = [&](int f, const RawC& v, CW& k_out) -> cx<R> {
            const int fc = min(max(f, plo), phi);
            const int zf = (fc == 0) + (fc == g.nz - 1);
            const R wz = (fc & 1) ? R(0.5) : R(1), bz = R(1) - wz;
            const cx<R> pn = interp(v.e);
            const cx<R> pe = wz * ((fc & 1) ? carry : pn) + bz * pn;
            carry = pn;
            const int nf = BC == BC_SOMMERFELD ? unf + zf : 0;
            k_out.c = shift_c(L, v.k, nf);
            const cx<R> wj = jacobi_w(L, k_out.c);
            if constexpr (KEEP_W) k_out.w = wj;
            cx<R> u = wj * cvt<R>(v.b) + pe;
            if (BC == BC_DIRICHLET && (unf || zf)) u = czero<R>();
            us[ring4(f)][t] = u;  // unguarded: lanes past the region write slots never read
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
        cx<R> e_first[4];  // coarse plane c0 of the first plane
        {
            const cx<R>* e0 = er + (long long)(plo >> 1) * gc.plane;
            e_first[0] = e0[cy0 + cx0];
            e_first[1] = e0[cy0 + cx1];
            e_first[2] = e0[cy1 + cx0];
            e_first[3] = e0[cy1 + cx1];
        }
        fetch_c(z0 - 1, A);
        fetch_c(z0, B);
        carry = interp(e_first);
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
                                                       const R* __restrict__ k2l, double beta1,
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
        const cx<R> c = shift_c(L, k2l[j], BC == BC_SOMMERFELD ? nf : 0);
        cx<R> v = (br[j] - L.ih2 * lap) + c * u;
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
int mg_up_blocks(const Geo& g, int zb) {
    const TileShape T = up_tile_shape(g.nx, g.ny);
    return T.ntx * T.nty * ((g.nz + zb - 1) / zb);
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
                    const cx<TB>* b, long long b_rstride, const R* k2l, const MgParams& P,
                    cx<R>* bc_out, const RhsState* st, int gate, int reg_want) {
    const int reg = mg_down_region(gc, zbc, nrhs, reg_want);
    const TileShape T = dn_tile_shape(gc.nx, gc.ny, reg);
    dim3 grid(T.ntx * T.nty, (gc.nz + zbc - 1) / zbc, nrhs);
#define HH_DOWN(BCV, ONEV, REGV)                                                                                \
    hipLaunchKernelGGL((k_mg_down<BCV, TB, R, ONEV, REGV>), grid, dim3(DN_LANES), 0, s, gf, gc, zbc, b, b_rstride, \
                       k2l, P.beta1, P.beta2, P.omega, bc_out, st, gate)
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
                  const cx<TB>* b, long long b_rstride, const R* k2l, const MgParams& P,
                  const cx<R>* ec, cx<TO>* out, long long o_rstride, const RhsState* st, int gate,
                  bool acc) {
    const TileShape T = up_tile_shape(g.nx, g.ny);
    dim3 grid(T.ntx * T.nty, (g.nz + zb - 1) / zb, nrhs);
#define HH_UP(BCV, ONEV, ACCV)                                                                          \
    hipLaunchKernelGGL((k_mg_up<BCV, TB, R, TO, ONEV, ACCV>), grid, dim3(UP_LANES), 0, s, g, gc, zb, b,    \
                       b_rstride, k2l, P.beta1, P.beta2, P.omega, ec, out, o_rstride, st, gate)
#define HH_UP_BC(ACCV)                                     \
    if (bc == BC_SOMMERFELD) {                             \
        if (zb == 1) HH_UP(BC_SOMMERFELD, true, ACCV);     \
        else HH_UP(BC_SOMMERFELD, false, ACCV);            \
    } else {                                               \
        if (zb == 1) HH_UP(BC_DIRICHLET, true, ACCV);      \
        else HH_UP(BC_DIRICHLET, false, ACCV);             \
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
void launch_mg_resid(hipStream_t s, int bc, const Geo& g, int nrhs, cx<R>* b, const cx<R>* e, const R* k2l,
                     const MgParams& P, const RhsState* st, int gate) {
    // about four planes per lane, enough workgroups to spread over the chip
    const int bx = (g.plane + RS_LANES - 1) / RS_LANES;
    int zb = 4;
    while (zb > 1 && (long long)bx * ((g.nz + zb - 1) / zb) * nrhs < 1024) zb >>= 1;
    dim3 grid(bx, (g.nz + zb - 1) / zb, nrhs);
    if (bc == BC_SOMMERFELD)
        hipLaunchKernelGGL((k_mg_resid<BC_SOMMERFELD, R>), grid, dim3(RS_LANES), 0, s, g, zb, b, e, k2l,
                           P.beta1, P.beta2, P.omega, st, gate);
    else
        hipLaunchKernelGGL((k_mg_resid<BC_DIRICHLET, R>), grid, dim3(RS_LANES), 0, s, g, zb, b, e, k2l,
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
