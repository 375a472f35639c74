// The smallest multigrid levels in one workgroup, with every array in LDS.
//
// Below a few thousand nodes a level's passes are pure latency: a separate
// kernel per pass costs a launch and a memory round trip for microseconds of
// work.  This kernel runs the rest of the cycle from level `first` down to the
// coarsest level and back up (Algorithm 1 applied recursively: damped-Jacobi
// pre-smoothing from zero, residual, full weighting, exact coarsest solve with
// the dense inverse, trilinear prolongation, correction, damped-Jacobi
// post-smoothing) with one workgroup per right-hand side; the passes are
// separated by workgroup barriers instead of kernel boundaries.  The order of
// the passes is a small program built on the host: the V-cycle, or the F-cycle's
// coarse-grid solve, which adds residual passes and a second cycle.
// Operators and boundary rules are those of the fused passes:
//   M u = (1/h^2) lap(u) - c u,  lap(u)_j = sum_nb (u_j - u_nb) with the
//   Sommerfeld ghost point replaced by its mirror image (its 2hik part is in c),
//   W = omega / (6/h^2 - c).
#include "hh_common.h"
#include "hh_device.h"
#include "hh_kernels.h"

namespace hh {

namespace {

// |D|^2 is positive and normal: the hardware reciprocal (about 1 ulp in single
// precision; in double refined by two Newton steps) needs no range scaling
__device__ __forceinline__ double t_rcp(double x) {
    double y = __builtin_amdgcn_rcp(x);
    y = __builtin_fma(y, __builtin_fma(-x, y, 1.0), y);
    return __builtin_fma(y, __builtin_fma(-x, y, 1.0), y);
}
__device__ __forceinline__ float t_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

template <typename R>
struct TailCoef {
    R ih2, six_ih2, two_over_h, sr, si, omega;
};

// node index -> (x, y, z).  The quotients are multiply-highs by ceil(2^32 / d),
// exact for index and divisor below 2^16 (the tail levels are far smaller).
__device__ __forceinline__ void unflat(int i, const TailLevel& L, int& x, int& y, int& z) {
    const int plane = L.nx * L.ny;
    z = (int)__umulhi((unsigned)i, L.rcp_plane);
    const int rem = i - z * plane;
    y = (int)__umulhi((unsigned)rem, L.rcp_nx);
    x = rem - y * L.nx;
}

__device__ __forceinline__ int mirror_in(int g, int n) { return g < 0 ? -g : (g > n - 1 ? 2 * (n - 1) - g : g); }

// c_j = (beta1 - beta2 i) k^2 + n_j 2 i k / h from the level's k (k^2 formed
// in the compute precision)
template <int BC, typename R>
__device__ __forceinline__ cx<R> shift_c_t(const TailCoef<R>& C, R k, int nf) {
    const R k2 = k * k;
    cx<R> c = {C.sr * k2, C.si * k2};
    if (BC == BC_SOMMERFELD && nf) c.im += R(nf) * C.two_over_h * k;
    return c;
}
template <typename R>
__device__ __forceinline__ cx<R> jacobi_w_t(const TailCoef<R>& C, cx<R> c) {
    const R dr = C.six_ih2 - c.re, di = -c.im;
    const R s = C.omega * t_rcp(dr * dr + di * di);
    return {dr * s, -di * s};
}

// lap(u) at (x, y, z) of level L from the LDS array u
template <typename R>
__device__ __forceinline__ cx<R> lap_at(const cx<R>* u, const TailLevel& L, int x, int y, int z) {
    const int plane = L.nx * L.ny;
    const int i = (z * L.ny + y) * L.nx + x;
    const cx<R> c = u[i];
    const int xm = mirror_in(x - 1, L.nx), xp = mirror_in(x + 1, L.nx);
    const int ym = mirror_in(y - 1, L.ny), yp = mirror_in(y + 1, L.ny);
    const int zm = mirror_in(z - 1, L.nz), zp = mirror_in(z + 1, L.nz);
    cx<R> s = (c - u[i - x + xm]) + (c - u[i - x + xp]);
    s = s + (c - u[i + (ym - y) * L.nx]);
    s = s + (c - u[i + (yp - y) * L.nx]);
    s = s + (c - u[i + (zm - z) * plane]);
    s = s + (c - u[i + (zp - z) * plane]);
    return s;
}

}  // namespace

template <int BC, typename R>
__global__ __launch_bounds__(1024) void k_mg_tail(TailDesc D, TailProg prog,
                                                  const cx<R>* __restrict__ b_first,
                                                  cx<R>* __restrict__ e_first,
                                                  const RhsState* st, int gate) {
    extern __shared__ unsigned char tail_smem[];
    const int r = blockIdx.x;
    if (!gate_ok(st, r, gate)) return;
    const int t = threadIdx.x, nt = blockDim.x;
    // LDS layout: per level b, u (the level's cycle result) and w (scratch),
    // then every level's s (an earlier result kept while another cycle runs),
    // then every level's k
    cx<R>* base = reinterpret_cast<cx<R>*>(tail_smem);
    auto B = [&](int l) { return base + 3 * D.lv[l].off; };
    auto U = [&](int l) { return base + 3 * D.lv[l].off + D.lv[l].n; };
    auto T = [&](int l) { return base + 3 * D.lv[l].off + 2 * D.lv[l].n; };
    auto S = [&](int l) { return base + 3 * D.total + D.lv[l].off; };
    R* kbase = reinterpret_cast<R*>(base + 4 * D.total);
    auto K = [&](int l) { return kbase + D.lv[l].off; };
    auto coef = [&](int l) {
        TailCoef<R> C;
        const double h = D.lv[l].h;
        C.ih2 = R(1.0 / (h * h));
        C.six_ih2 = R(6.0 / (h * h));
        C.two_over_h = R(2.0 / h);
        C.sr = R(D.beta1);
        C.si = R(-D.beta2);
        C.omega = R(D.omega);
        return C;
    };
    auto faces = [&](const TailLevel& L, int x, int y, int z) {
        return (x == 0) + (x == L.nx - 1) + (y == 0) + (y == L.ny - 1) + (z == 0) + (z == L.nz - 1);
    };
    const int nl = D.nlev;
    // Coarsest solve layout: G lanes per row (a power of two <= 64, so a group
    // stays inside one wavefront); lane j of a group sums the columns
    // c = j, j + G, ..., then the group adds its partial sums with a fixed
    // butterfly.  When every row fits one pass and a lane has at most
    // MAX_PRE columns, the lane's inverse entries and node indices are loaded
    // here, with the staging loads, instead of after the down passes.
    constexpr int MAX_PRE = 8;
    int G = 1;
    while (G < 64 && 2 * G * D.n_unk <= nt) G *= 2;
    const int sub = t & (G - 1);
    const bool pre = D.n_unk <= nt / G && D.n_unk <= MAX_PRE * G;
    const cx<R>* minv = reinterpret_cast<const cx<R>*>(D.minv);
    cx<R> mv[MAX_PRE];
    int ci[MAX_PRE];
    int crow = 0;  // node of this lane's row
    if (pre) {
        const int row = min(t / G, D.n_unk - 1);
        crow = D.cidx[row];
#pragma unroll
        for (int k = 0; k < MAX_PRE; ++k) {
            const int cc = min(sub + k * G, D.n_unk - 1);
            mv[k] = minv[(long long)cc * D.n_unk + row];
            ci[k] = D.cidx[cc];
        }
    }
    // stage the right-hand side of the first level and every level's k
    const cx<R>* bsrc = b_first + (long long)r * D.lv[0].n;
    for (int i = t; i < D.lv[0].n; i += nt) B(0)[i] = bsrc[i];
    for (int l = 0; l < nl; ++l) {
        const R* kg = reinterpret_cast<const R*>(D.lv[l].k);
        for (int i = t; i < D.lv[l].n; i += nt) K(l)[i] = kg[i];
    }
    __syncthreads();

    // pre-smoothing from zero, residual and full weighting: b_{l+1} = R (b - M W b)
    auto down = [&](int l) {
        const TailLevel& L = D.lv[l];
        const TailLevel& Lc = D.lv[l + 1];
        const TailCoef<R> C = coef(l);
        cx<R>* b = B(l);
        cx<R>* u = U(l);
        cx<R>* w = T(l);
        const R* kk = K(l);
        // u1 = W b
        for (int i = t; i < L.n; i += nt) {
            int x, y, z;
            unflat(i, L, x, y, z);
            const int nf = faces(L, x, y, z);
            cx<R> v = jacobi_w_t(C, shift_c_t<BC>(C, kk[i], nf)) * b[i];
            if (BC == BC_DIRICHLET && nf) v = czero<R>();
            u[i] = v;
        }
        __syncthreads();
        // r = b - (1/h^2) lap(u1) + c u1
        for (int i = t; i < L.n; i += nt) {
            int x, y, z;
            unflat(i, L, x, y, z);
            const int nf = faces(L, x, y, z);
            cx<R> v = (b[i] - C.ih2 * lap_at(u, L, x, y, z)) + shift_c_t<BC>(C, kk[i], nf) * u[i];
            if (BC == BC_DIRICHLET && nf) v = czero<R>();
            w[i] = v;
        }
        __syncthreads();
        // full weighting onto the next level (mirror extension at the boundary)
        cx<R>* bc = B(l + 1);
        for (int i = t; i < Lc.n; i += nt) {
            int X, Y, Z;
            unflat(i, Lc, X, Y, Z);
            cx<R> acc = czero<R>();
            if (!(BC == BC_DIRICHLET && faces(Lc, X, Y, Z))) {
                for (int dz = -1; dz <= 1; ++dz) {
                    const int fz = mirror_in(2 * Z + dz, L.nz);
                    for (int dy = -1; dy <= 1; ++dy) {
                        const int fy = mirror_in(2 * Y + dy, L.ny);
                        const cx<R>* row = w + (fz * L.ny + fy) * L.nx;
                        const int fx0 = mirror_in(2 * X - 1, L.nx), fx2 = mirror_in(2 * X + 1, L.nx);
                        cx<R> rs = row[fx0] + row[fx2];
                        rs = rs + R(2) * row[2 * X];
                        const R wyz = (dy == 0 ? R(2) : R(1)) * (dz == 0 ? R(2) : R(1));
                        acc = acc + wyz * rs;
                    }
                }
                acc = R(1.0 / 64.0) * acc;
            }
            bc[i] = acc;
        }
        __syncthreads();
    };
    // coarsest: e = M_c^-1 b over the unknown nodes (inverse stored column-major)
    auto coarse = [&]() {
        const TailLevel& L = D.lv[nl - 1];
        cx<R>* b = B(nl - 1);
        cx<R>* u = U(nl - 1);
        for (int i = t; i < L.n; i += nt) u[i] = czero<R>();
        __syncthreads();
        if (pre) {
            const int row = t / G;
            cx<R> s = czero<R>();
#pragma unroll
            for (int k = 0; k < MAX_PRE; ++k)
                if (sub + k * G < D.n_unk) s = s + mv[k] * b[ci[k]];
            for (int off = G >> 1; off > 0; off >>= 1) {
                s.re += __shfl_xor(s.re, off, 64);
                s.im += __shfl_xor(s.im, off, 64);
            }
            if (row < D.n_unk && sub == 0) u[crow] = s;
        }
        for (int row0 = 0; !pre && row0 < D.n_unk; row0 += nt / G) {
            const int row = row0 + t / G;
            cx<R> s = czero<R>();
            if (row < D.n_unk)
                for (int c = sub; c < D.n_unk; c += G)
                    s = s + minv[(long long)c * D.n_unk + row] * b[D.cidx[c]];
            for (int off = G >> 1; off > 0; off >>= 1) {
                s.re += __shfl_xor(s.re, off, 64);
                s.im += __shfl_xor(s.im, off, 64);
            }
            if (row < D.n_unk && sub == 0) u[D.cidx[row]] = s;
        }
        __syncthreads();
    };
    // trilinear prolongation, correction and post-smoothing:
    // u2 = W b + P e_{l+1},  u3 = u2 + W (b - (1/h^2) lap(u2) + c u2)
    auto up = [&](int l) {
        const TailLevel& L = D.lv[l];
        const TailLevel& Lc = D.lv[l + 1];
        const TailCoef<R> C = coef(l);
        cx<R>* b = B(l);
        cx<R>* u = U(l);
        cx<R>* w = T(l);
        const cx<R>* ec = U(l + 1);
        const R* kk = K(l);
        for (int i = t; i < L.n; i += nt) {
            int x, y, z;
            unflat(i, L, x, y, z);
            const int nf = faces(L, x, y, z);
            const int cxi = x >> 1, cyi = y >> 1, czi = z >> 1;
            const int ox = x & 1, oy = y & 1, oz = z & 1;
            cx<R> pe = czero<R>();
            for (int a = 0; a <= oz; ++a)
                for (int bb = 0; bb <= oy; ++bb)
                    for (int c = 0; c <= ox; ++c)
                        pe = pe + ec[((czi + a) * Lc.ny + cyi + bb) * Lc.nx + cxi + c];
            const R wt = R(1) / R(1 << (ox + oy + oz));
            cx<R> v = jacobi_w_t(C, shift_c_t<BC>(C, kk[i], nf)) * b[i] + wt * pe;
            if (BC == BC_DIRICHLET && nf) v = czero<R>();
            w[i] = v;
        }
        __syncthreads();
        for (int i = t; i < L.n; i += nt) {
            int x, y, z;
            unflat(i, L, x, y, z);
            const int nf = faces(L, x, y, z);
            const cx<R> cc = shift_c_t<BC>(C, kk[i], nf);
            const cx<R> u2 = w[i];
            cx<R> v = u2 + jacobi_w_t(C, cc) * ((b[i] - C.ih2 * lap_at(w, L, x, y, z)) + cc * u2);
            if (BC == BC_DIRICHLET && nf) v = czero<R>();
            u[i] = v;
        }
        __syncthreads();
    };
    // keep the level's result and replace its right-hand side by the residual:
    // s = u, b = b - (1/h^2) lap(u) + c u  (b and s written only at the node itself)
    auto resid = [&](int l) {
        const TailLevel& L = D.lv[l];
        const TailCoef<R> C = coef(l);
        cx<R>* b = B(l);
        const cx<R>* u = U(l);
        cx<R>* sv = S(l);
        const R* kk = K(l);
        for (int i = t; i < L.n; i += nt) {
            int x, y, z;
            unflat(i, L, x, y, z);
            const int nf = faces(L, x, y, z);
            const cx<R> ui = u[i];
            cx<R> v = (b[i] - C.ih2 * lap_at(u, L, x, y, z)) + shift_c_t<BC>(C, kk[i], nf) * ui;
            if (BC == BC_DIRICHLET && nf) v = czero<R>();
            sv[i] = ui;
            b[i] = v;
        }
        __syncthreads();
    };
    // u = s + u: the kept result plus the correction computed from its residual
    auto accumulate = [&](int l) {
        const TailLevel& L = D.lv[l];
        cx<R>* u = U(l);
        const cx<R>* sv = S(l);
        for (int i = t; i < L.n; i += nt) u[i] = sv[i] + u[i];
        __syncthreads();
    };

    for (int p = 0; p < prog.n; ++p) {
        const int op = prog.op[p] >> 4, l = prog.op[p] & 15;
        switch (op) {
            case TAIL_DOWN: down(l); break;
            case TAIL_COARSE: coarse(); break;
            case TAIL_UP: up(l); break;
            case TAIL_RESID: resid(l); break;
            default: accumulate(l); break;
        }
    }
    cx<R>* edst = e_first + (long long)r * D.lv[0].n;
    for (int i = t; i < D.lv[0].n; i += nt) edst[i] = U(0)[i];
}

size_t mg_tail_lds_bytes(const TailDesc& D, bool single) {
    const size_t cs = single ? sizeof(c64) : sizeof(c128);
    const size_t rs = single ? sizeof(float) : sizeof(double);
    return (size_t)D.total * (4 * cs + rs);
}

bool mg_tail_allow_lds(size_t bytes) {
    const int v = (int)bytes;
    return hipFuncSetAttribute((const void*)k_mg_tail<BC_SOMMERFELD, double>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, v) == hipSuccess &&
           hipFuncSetAttribute((const void*)k_mg_tail<BC_DIRICHLET, double>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, v) == hipSuccess &&
           hipFuncSetAttribute((const void*)k_mg_tail<BC_SOMMERFELD, float>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, v) == hipSuccess &&
           hipFuncSetAttribute((const void*)k_mg_tail<BC_DIRICHLET, float>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, v) == hipSuccess;
}

template <typename R>
void launch_mg_tail(hipStream_t s, int bc, const TailDesc& D, const TailProg& P, int nrhs,
                    const cx<R>* b_first, cx<R>* e_first, const RhsState* st, int gate) {
    const size_t lds = mg_tail_lds_bytes(D, sizeof(R) == sizeof(float));
    if (bc == BC_SOMMERFELD)
        hipLaunchKernelGGL((k_mg_tail<BC_SOMMERFELD, R>), dim3(nrhs), dim3(1024), lds, s, D, P, b_first,
                           e_first, st, gate);
    else
        hipLaunchKernelGGL((k_mg_tail<BC_DIRICHLET, R>), dim3(nrhs), dim3(1024), lds, s, D, P, b_first,
                           e_first, st, gate);
}
template void launch_mg_tail<double>(hipStream_t, int, const TailDesc&, const TailProg&, int, const c128*,
                                     c128*, const RhsState*, int);
template void launch_mg_tail<float>(hipStream_t, int, const TailDesc&, const TailProg&, int, const c64*,
                                    c64*, const RhsState*, int);

namespace {
// Builds a tail program: F(l) = down l, coarse-grid solve C(l + 1), up l, where
// C(l) is the F-cycle on level l followed, unless l is the coarsest level, by
// one V-cycle on the residual that F-cycle leaves, added to its result
// (section 3.4.5); F on the coarsest level is the exact solve.
struct ProgBuilder {
    TailProg P{};
    int nlev;
    void put(int op, int l) { P.op[P.n++] = (unsigned char)(op << 4 | l); }
    void v(int l) {
        for (int m = l; m < nlev - 1; ++m) put(TAIL_DOWN, m);
        put(TAIL_COARSE, 0);
        for (int m = nlev - 2; m >= l; --m) put(TAIL_UP, m);
    }
    void f(int l) {
        if (l == nlev - 1) {
            put(TAIL_COARSE, 0);
            return;
        }
        put(TAIL_DOWN, l);
        c(l + 1);
        put(TAIL_UP, l);
    }
    void c(int l) {
        f(l);
        if (l < nlev - 1) {
            put(TAIL_RESID, l);
            v(l);
            put(TAIL_ACC, l);
        }
    }
};
}  // namespace

// The V-cycle from the tail's first level: down all levels, coarsest solve, up.
TailProg tail_prog_v(int nlev) {
    ProgBuilder b{TailProg{}, nlev};
    b.v(0);
    return b.P;
}

// The coarse-grid solver of an F-cycle one level above the tail's first level.
TailProg tail_prog_f(int nlev) {
    ProgBuilder b{TailProg{}, nlev};
    b.c(0);
    return b.P;
}

}  // namespace hh
