// Host-callable launchers of the gfx950 kernels (internal to the library).
#pragma once
#include "hh_common.h"

namespace hh {

// Launch shape of the fine-grid kernels: `zb` z-planes per workgroup of the
// operator kernels (tiles of ap_tile_shape()), `block` lanes per workgroup of
// the flat (grid-stride) Krylov vector kernels, which launch exactly
// `flat_cap` workgroups, set to the operator kernels' workgroup count so every
// reduction slot holds the same number of partial sums.
struct Launch {
    int block = 256;
    int zb = 8;
    int flat_cap = 2048;
};

// Runtime tile shape of a level: width = ceil(n / ceil(n / maxw)) so a row of
// 2^k + 1 nodes splits into nearly equal tiles, height = as many rows as the
// workgroup's lanes allow (at most maxh).
struct TileShape {
    int tw, th, ntx, nty;
};
__host__ __device__ inline TileShape tile_shape(int nx, int ny, int maxw, int lanes, int maxh) {
    TileShape T;
    T.ntx = (nx + maxw - 1) / maxw;
    T.tw = (nx + T.ntx - 1) / T.ntx;
    T.th = lanes / T.tw;
    if (T.th > maxh) T.th = maxh;
    if (T.th > ny) T.th = ny;
    T.nty = (ny + T.th - 1) / T.th;
    return T;
}

// Tiling of the fine-grid operator kernels (operator apply, start residual):
// a workgroup of AP_LANES lanes owns a tw x th tile of an x-y plane, one node
// per lane, and marches along z; the apply stages the tile and its one-node
// halo, (tw + 2)(th + 2) <= AP_REGION nodes, in LDS (AP_REGION / AP_LANES
// region nodes per lane).  Every axis has >= 3 nodes, so tw >= 3 and the
// region bound holds without shrinking th (the loop is a guard).
constexpr int AP_LANES = 256, AP_MAXW = 64, AP_REGION = 512;
static_assert(AP_REGION % AP_LANES == 0, "every lane's region slots must lie inside the LDS arrays");
__host__ __device__ inline TileShape ap_tile_shape(int nx, int ny) {
    TileShape T = tile_shape(nx, ny, AP_MAXW, AP_LANES, AP_LANES);
    while (T.th > 1 && (T.tw + 2) * (T.th + 2) > AP_REGION) --T.th;
    T.nty = (ny + T.th - 1) / T.th;
    return T;
}

enum OpMode : int { OP_PLAIN = 0, OP_V = 1, OP_T = 2, OP_P = 3 };
// FIN_OMEGA also takes the half-step test on ||s||: the s update writes its
// partial sums beside those of t = A s_hat, so one finalize serves both.
// FIN_TRUE_RECORD: the true residual only, no restart (GMRES stops on the
// preconditioned residual)
// FIN_RHO_DEFER: FIN_RHO at the start of an odd step, which also records the
// even step's solution update as outstanding (alpha_d, omega_d, pend)
enum FinMode : int {
    FIN_INIT = 0,
    FIN_RHO = 1,
    FIN_ALPHA = 2,
    FIN_OMEGA = 4,
    FIN_TRUE = 5,
    FIN_TRUE_RECORD = 6,
    FIN_RHO_DEFER = 7,
    FIN_INIT_DECADE = 8,  // FIN_INIT with restarts from x at every power of ten of the residual
    FIN_RESTART = 9       // restart from x the right-hand sides stopped for it (true residual in slot R)
};
constexpr int GATE_ALL = -1;       // act on every right-hand side
constexpr int GATE_FINISHED = -2;  // act on right-hand sides that stopped iterating

long long nblk_of(const Geo& g, const Launch& L);

// x: complex128, or complex64 (double / float); y and the arithmetic are complex128
template <typename TX>
void launch_apply(hipStream_t s, int bc, int mode, const Geo& g, const Launch& L, int nrhs,
                  const cx<TX>* x, c128* y, const double* k2, const double* kb, double sr, double si,
                  const c128* aux, double* part, long long nblk_max, const RhsState* st, int gate);
// y = A x and the IDR(s) shadow products <p_i, y>, i < ns <= IDR_SMAX, into
// partial-sum rows 0 .. 2 ns - 1 (P: ns complex64 vectors of g.n nodes)
void launch_apply_p(hipStream_t s, int bc, const Geo& g, const Launch& L, int nrhs, int ns, const c128* x,
                    c128* y, const double* k2, const double* kb, const c64* P, double* part,
                    long long nblk_max, const RhsState* st, int gate);
// rhat: the shadow residual, complex64 when rhat_low (the mixed solve), else complex128
void launch_init(hipStream_t s, int bc, const Geo& g, const Launch& L, int nrhs, const c128* b,
                 c128* x, c128* r, void* rhat, bool rhat_low, c128* p, c128* v, const double* k2,
                 const double* kb, int use_x0, double* part, long long nblk_max, const RhsState* st, int gate);

// CSLP parameters of the multigrid kernels: M = -Laplace - (beta1 - beta2 i) k^2,
// damped-Jacobi weight omega.
struct MgParams {
    double beta1, beta2, omega;
};
// reg: fine region nodes a workgroup of a one-plane pass (zbc = 1) stages,
// 256, 512 or 1280; 0 = chosen by dn_region().  Ignored when zbc > 1.
template <typename TB, typename R>
void launch_mg_down(hipStream_t s, int bc, const Geo& gf, const Geo& gc, int zbc, int nrhs,
                    const cx<TB>* b, long long b_rstride, const R* kl, const MgParams& P,
                    cx<R>* bc_out, const RhsState* st, int gate, int reg = 0);
template <typename TB, typename R, typename TO>
void launch_mg_up(hipStream_t s, int bc, const Geo& g, const Geo& gc, int zb, int nrhs,
                  const cx<TB>* b, long long b_rstride, const R* kl, const MgParams& P,
                  const cx<R>* ec, cx<TO>* out, long long o_rstride, const RhsState* st, int gate,
                  bool acc = false);
// b = b - M e in place on a level below the finest (one precision throughout)
template <typename R>
void launch_mg_resid(hipStream_t s, int bc, const Geo& g, int nrhs, cx<R>* b, const cx<R>* e, const R* kl,
                     const MgParams& P, const RhsState* st, int gate);
int mg_down_blocks(const Geo& gc, int zbc);
// region of the down pass into a coarse grid gc: the automatic choice for
// (zbc, nrhs), or `want` (256, 512, 1280) where it applies (zbc = 1)
int mg_down_region(const Geo& gc, int zbc, int nrhs, int want);
// workgroups of the up pass on level g in the compute precision (single: the x-pair kernel)
int mg_up_blocks(const Geo& g, int zb, bool single);
// whether every tile of the single-precision (x-pair) up pass on level g
// (coarse grid gc) reads a coarse window of at most one node per lane
bool mg_up_windows_fit(const Geo& g, const Geo& gc);

// The trailing (smallest) levels of the hierarchy, run by one workgroup per
// right-hand side with every array in LDS.  off = offset of the level's nodes
// in the LDS arrays, total = sum of the levels' node counts.
constexpr int MAX_TAIL = 8;
struct TailLevel {
    int nx, ny, nz, n, off;
    unsigned rcp_nx, rcp_plane;  // ceil(2^32 / nx), ceil(2^32 / (nx ny)): index division by multiply-high
    double h;
    const void* k;   // level wavenumber in the multigrid precision (device)
};
struct TailDesc {
    int nlev, total, n_unk;
    double beta1, beta2, omega;
    const int* cidx;   // coarsest unknown -> node
    const void* minv;  // dense inverse of the coarsest M, column-major
    TailLevel lv[MAX_TAIL];
};
// A tail program: the passes to run, in order, each one byte (op << 4 | level).
enum TailOp { TAIL_DOWN = 0, TAIL_COARSE = 1, TAIL_UP = 2, TAIL_RESID = 3, TAIL_ACC = 4 };
constexpr int MAX_TAIL_OPS = 96;  // the F program on MAX_TAIL levels has 92 passes
struct TailProg {
    int n;
    unsigned char op[MAX_TAIL_OPS];
};
TailProg tail_prog_v(int nlev);
TailProg tail_prog_f(int nlev);
size_t mg_tail_lds_bytes(const TailDesc& D, bool single);
// Raise the kernel's dynamic-LDS limit to `bytes`; returns false if refused.
bool mg_tail_allow_lds(size_t bytes);
template <typename R>
void launch_mg_tail(hipStream_t s, int bc, const TailDesc& D, const TailProg& P, int nrhs,
                    const cx<R>* b_first, cx<R>* e_first, const RhsState* st, int gate);
// p_low / s_low (may be null): a complex64 copy of the new p / s for a
// single-precision preconditioner
void launch_p_update(hipStream_t s, long long n, int nrhs, c128* p, const c128* r, const c128* v,
                     c64* p_low, const RhsState* st, const Launch& L);
void launch_s_update(hipStream_t s, long long n, int nrhs, c128* sv, const c128* r, const c128* v,
                     c64* s_low, const RhsState* st, double* part, long long nblk_max, const Launch& L);
// p_hat, s_hat: complex128, or complex64 from a single-precision preconditioner
template <typename TH>
void launch_update_xr(hipStream_t s, bool odd, long long n, int nrhs, c128* x, c128* r, const cx<TH>* ph,
                      const cx<TH>* sh, const cx<TH>* php, const cx<TH>* shp, const c128* sv, const c128* t,
                      const cx<TH>* rhat, const RhsState* st, double* part, long long nblk_max,
                      const Launch& L);
// x += alpha_d p_hat' + omega_d s_hat' for the stopped right-hand sides with an
// outstanding even-step update (before the true residual of a solve or of a
// restart); only >= 0 restricts it to the right-hand sides with that status
template <typename TH>
void launch_flush_x(hipStream_t s, long long n, int nrhs, c128* x, const cx<TH>* php, const cx<TH>* shp,
                    const RhsState* st, const Launch& L, int only = -1);
void launch_finalize(hipStream_t s, int mode, int nrhs, RhsState* st, const double* part,
                     long long nblk, long long nblk_max, double tol);

void launch_model_check(hipStream_t s, long long n, const double* k, double* k2, double* kb, int* bad);
// k = omega sqrt(s) (s = squared slowness); bad counts invalid entries
void launch_model_from_slowness2(hipStream_t s, long long n, const double* s2, double omega, double* k, int* bad);
void launch_inject(hipStream_t s, const Geo& gf, const Geo& gc, const double* kf, double* kc);
template <typename R>
void launch_level_k2(hipStream_t s, long long n, const double* k, R* k2);
// k of a level rounded to the multigrid precision (the multigrid passes form k^2 from it)
template <typename R>
void launch_level_k(hipStream_t s, long long n, const double* k, R* kl);
void launch_copy_rhs(hipStream_t s, const Geo& g, int bc, int nrhs, const c128* src, c128* dst);
void launch_adjoint_rhs(hipStream_t s, const Geo& g, int bc, int nrhs, const c128* gin, c128* out);
void launch_grad_s(hipStream_t s, const Geo& g, int bc, int nrhs, const c128* u, const c128* w,
                   const double* sl, double omega, double* grad);
void launch_set_point(hipStream_t s, long long off, double val, c128* b);
// status and iteration limit of the first n right-hand sides; tol2 < 0 also
// replaces the squared stopping threshold (no reduction then meets it)
void launch_fill_status(hipStream_t s, int n, RhsState* st, int status, int maxit2, double tol2 = 0.0);

}  // namespace hh
