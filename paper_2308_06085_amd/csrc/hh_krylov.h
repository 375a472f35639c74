// Declarations of the IDR(s) and full-GMRES kernels (hh_idr.hip,
// hh_gmres.hip) and their device state, used by those files and the solver.
#pragma once
#include "hh_common.h"
#include "hh_kernels.h"

namespace hh {

// IDR(s) (s <= IDR_SMAX): per right-hand side small state kept on the device.
// Partial-sum rows of the IDR kernels, counting the NSLOT * MAX_TERMS rows of
// a right-hand side flat: rows 2i, 2i + 1 = Re/Im <p_i, y>; row IDR_ROW_RN =
// ||r||^2; the t-step uses the rows of slot T as Bi-CGSTAB does.
constexpr int IDR_SMAX = 8;
constexpr int IDR_ROW_RN = NSLOT * MAX_TERMS - 1;
static_assert(2 * IDR_SMAX <= IDR_ROW_RN, "IDR rows overlap");
struct IdrState {
    c128 M[IDR_SMAX][IDR_SMAX];  // M[i][k] = <p_i, g_k>, lower triangular
    c128 f[IDR_SMAX];            // <p_i, r>, updated within a cycle
    c128 c[IDR_SMAX];            // coefficients of the current inner step, c[j - k]
    c128 a[IDR_SMAX];            // biorthogonalisation coefficients of the current step
    c128 beta, om;
    double kappa;
    int s, first, pad_;
};

// IDR(s) kernels (hh_idr.hip).  G and U: s vectors per right-hand side,
// vector (j, r) at j * rsj + r * n; P: ns complex64 shadow vectors of n nodes.
enum IdrFin : int { IDR_FIN_START = 0, IDR_FIN_STEP = 1, IDR_FIN_OMEGA = 2 };
void launch_idr_v(hipStream_t s, long long n, int nrhs, int k, const c128* G, long long rsj, const c128* r,
                  c128* v, c64* v_low, const IdrState* is, const RhsState* st, const Launch& L);
template <typename TH>
void launch_idr_u(hipStream_t s, long long n, int nrhs, int k, c128* U, long long rsj, const cx<TH>* vh,
                  const IdrState* is, const RhsState* st, const Launch& L);
void launch_idr_update(hipStream_t s, long long n, int nrhs, int k, c128* G, c128* U, long long rsj, c128* r,
                       c128* x, c128* v, c64* v_low, const IdrState* is, const RhsState* st, double* part,
                       long long nblk_max, const Launch& L);
template <typename TH>
void launch_idr_xr(hipStream_t s, long long n, int nrhs, int ns, c128* x, c128* r, const cx<TH>* vh,
                   const c128* t, const c64* P, const IdrState* is, const RhsState* st, double* part,
                   long long nblk_max, const Launch& L);
void launch_idr_pr(hipStream_t s, long long n, int nrhs, int ns, const c128* r, const c64* P,
                   const RhsState* st, double* part, long long nblk_max, const Launch& L);
void launch_idr_finalize(hipStream_t s, int mode, int k, int reset, int nrhs, int ns, double kappa,
                         RhsState* st, IdrState* is, const double* part, long long nblk, long long nblk_max);
void launch_idr_gen_p(hipStream_t s, long long n, int ns, unsigned long long seed, c64* P);
void launch_idr_set_p(hipStream_t s, long long total, const c128* src, c64* P);

// Full GMRES kernels (hh_gmres.hip).  Basis vector (i, r) at V + i * rsv + r * n;
// per right-hand side a GmHead and its arrays (GmLayout, in doubles); partial
// sums of GM_NBLK workgroups per row, `rows` rows per right-hand side.
constexpr int GM_NBLK = 1024;
struct alignas(16) GmHead {
    double beta, kbn, scale, pad0;
    int m, update, reorth, pad1;
};
static_assert(sizeof(GmHead) % 16 == 0, "GmHead keeps the arrays after it 16-byte aligned");
struct GmLayout {
    long long H, cs, sn, g, y, h1, dots, words;
    int norm_row, rows;
};
GmLayout gm_host_layout(int M);
enum GmFin : int { GM_FIN_START = 0, GM_FIN_DOTS1 = 1, GM_FIN_DOTS2 = 2, GM_FIN_REORTH = 3 };
// gated: only right-hand sides whose reorthogonalisation flag is set
void launch_gm_dots(hipStream_t s, long long n, int nrhs, int j, const c128* w, const c128* V, long long rsv,
                    double* part, long long rows_per_rhs, int wrow, const double* gst, long long gst_words,
                    bool gated, const RhsState* st);
void launch_gm_axpy(hipStream_t s, long long n, int nrhs, int j, const c128* w_in, c128* w_out, const c128* V,
                    long long rsv, const double* gst, long long gst_words, long long coef_off, bool norm,
                    double* part, long long rows_per_rhs, int norm_row, bool gated, const RhsState* st);
void launch_gm_rowsum(hipStream_t s, int nrhs, int row_begin, int nrows, const double* part, long long rows_per_rhs,
                      double* gst, long long gst_words, long long dots_off, bool gated, const RhsState* st);
void launch_gm_norm2(hipStream_t s, long long n, int nrhs, const c128* a, double* part, long long rows_per_rhs,
                     int row, const RhsState* st);
void launch_gm_scale(hipStream_t s, long long n, int nrhs, const c128* src1, const c128* src2, c128* dst,
                     const double* gst, long long gst_words, const RhsState* st);
void launch_gm_xupdate(hipStream_t s, long long n, int nrhs, c128* xk, const c128* V, long long rsv,
                       const double* gst, long long gst_words, long long y_off);
void launch_gm_clear(hipStream_t s, int nrhs, double* gst, long long gst_words);
void launch_gm_finalize(hipStream_t s, int mode, int j, int M, int kb, double tol, int nrhs, RhsState* st,
                        double* gst, long long gst_words);

}  // namespace hh
