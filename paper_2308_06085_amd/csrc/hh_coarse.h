// Host-callable launchers of the large-coarsest-grid kernels (internal to the
// library): the device Gauss-Jordan inverse of the coarsest rediscretised M and
// the multi-workgroup dense solve that replaces the single-workgroup tail when
// the coarsest level does not fit one workgroup's LDS.
#pragma once
#include "hh_common.h"

namespace hh {

// inv = I (n x n, complex128)
void launch_gj_identity(hipStream_t s, int n, c128* inv);
// One Gauss-Jordan step on the n x n row-major matrices a and inv (complex128):
// partial pivoting over rows col .. n - 1 of column col (the row of largest
// modulus, the first one on ties), row swap, scaling of the pivot row, and
// elimination of column col from every other row.  piv, pval, f (n entries)
// and bad are device scratch; bad is set when the pivot is zero or not finite.
void launch_gj_step(hipStream_t s, int n, c128* a, c128* inv, int col, int* piv, c128* pval, c128* f,
                    int* bad);
// minv[j * n + r] = inv[r * n + j] (column-major, the layout of the coarsest
// solve), rounded to complex64 when low is set (the tail kernel's inverse in
// the mixed form).
void launch_gj_store(hipStream_t s, int n, const c128* inv, void* minv, bool low);

// e = M_c^-1 b on the coarsest level for every right-hand side the gate
// admits: unknown u of node cidx[u] gets sum_c minv[c * n_unk + u] b[cidx[c]]
// (complex128 inverse and sums, fixed summation order), nodes with
// unk_of[i] < 0 (Dirichlet boundary) get 0.  b and e hold nrhs slices of
// nnode nodes in the multigrid precision; part is device scratch of
// nrhs x coarse_gemv_chunks(n_unk) x n_unk complex128 values.
int coarse_gemv_chunks(int n_unk);
template <typename R>
void launch_coarse_gemv(hipStream_t s, int nnode, int n_unk, const int* unk_of, const int* cidx,
                        const c128* minv, const cx<R>* b, cx<R>* e, c128* part, int nrhs, const RhsState* st,
                        int gate);

// The paper's iterative coarsest solve (option "coarse_solver" = 1): full
// GMRES on M_c, no preconditioner, x0 = 0, to ||b - M_c e|| <= tol ||b||, one
// 1024-lane workgroup per right-hand side (see hh_coarse_gmres.hip).
constexpr int COARSE_GMRES_MAX_NODES = 8192;  // coarsest-grid nodes
constexpr int COARSE_GMRES_MAX_M = 100;       // Arnoldi steps per cycle
struct CoarseGmres {
    Geo g;                // the coarsest level
    double sr, si;        // shift: M_c = -Laplace - (sr + i si) k^2, sr = beta1, si = -beta2
    double ih2, two_over_h;
    const double* k;      // wavenumber at the coarsest nodes (device)
    int m;                // Arnoldi steps per cycle, 1 .. COARSE_GMRES_MAX_M
    int cycles;           // cycles (restarts + 1) at most
    double tol;           // relative residual
    c128* V;              // device, (m + 2) g.n complex128 per right-hand side (basis, x)
    int* steps;           // device, nrhs entries: Arnoldi steps of the last solve (may be null)
};
// LDS bytes of the kernel for m steps, and the attribute call that allows them
size_t coarse_gmres_lds_bytes(int m);
bool coarse_gmres_allow_lds(size_t bytes);
// e = M_c^-1 b (to the tolerance) on the coarsest level for every right-hand
// side the gate admits; b and e hold nrhs slices of g.n nodes in the
// multigrid precision, the solve itself runs in complex128.
template <typename R>
void launch_coarse_gmres(hipStream_t s, int bc, const CoarseGmres& D, const cx<R>* b, cx<R>* e, int nrhs,
                         const RhsState* st, int gate);

}  // namespace hh
