// Shared device/host definitions of the gfx950 Helmholtz library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hh {

// ---------------------------------------------------------------------------
// Complex numbers: interleaved {re, im}; 16 B (complex128) or 8 B (complex64)
// so that a wavefront moves 1 KB / 512 B per load instruction.
// ---------------------------------------------------------------------------
template <typename R>
struct alignas(2 * sizeof(R)) cx {
    R re, im;
};
using c128 = cx<double>;
using c64 = cx<float>;

template <typename R>
__host__ __device__ __forceinline__ cx<R> mk(R a, R b) { return cx<R>{a, b}; }
template <typename R>
__host__ __device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) { return {a.re + b.re, a.im + b.im}; }
template <typename R>
__host__ __device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) { return {a.re - b.re, a.im - b.im}; }
template <typename R>
__host__ __device__ __forceinline__ cx<R> operator*(cx<R> a, cx<R> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R>
__host__ __device__ __forceinline__ cx<R> operator*(R s, cx<R> a) { return {s * a.re, s * a.im}; }
template <typename R>
__host__ __device__ __forceinline__ cx<R> conj(cx<R> a) { return {a.re, -a.im}; }
// conj(a) * b
template <typename R>
__host__ __device__ __forceinline__ cx<R> cdot(cx<R> a, cx<R> b) {
    return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
template <typename R>
__host__ __device__ __forceinline__ R abs2(cx<R> a) { return a.re * a.re + a.im * a.im; }
template <typename R>
__host__ __device__ __forceinline__ cx<R> cdiv(cx<R> a, cx<R> b) {
    R d = R(1) / abs2(b);
    return {(a.re * b.re + a.im * b.im) * d, (a.im * b.re - a.re * b.im) * d};
}

template <typename To, typename From>
__host__ __device__ __forceinline__ cx<To> cvt(cx<From> a) { return {To(a.re), To(a.im)}; }

// ---------------------------------------------------------------------------
// Grid geometry of one level.  Arrays are (nrhs, nz, ny, nx), x fastest.
// ---------------------------------------------------------------------------
struct Geo {
    int nx, ny, nz;
    int plane;      // nx * ny
    long long n;    // nx * ny * nz
    double h;
};

enum Bc : int { BC_DIRICHLET = 0, BC_SOMMERFELD = 1 };

// Per right-hand-side Bi-CGSTAB state kept on the device so that a whole
// iteration runs without host involvement.
enum RhsStatus : int {
    ST_RUN = 0,      // iterating
    ST_CONV = 1,     // converged (recursive residual)
    ST_HALF = 2,     // converged at the half step, x += alpha p_hat pending
    ST_BREAK = 3,    // breakdown
    ST_MAXIT = 4,    // iteration limit
    ST_NUMERIC = 5,  // NaN / Inf
    ST_IDLE = 6,     // slot not in use
    ST_RESTART = 7   // stopped for a restart from x: the residual fell below the next power of ten
};

struct RhsState {
    c128 rho, alpha, omega, beta;
    // the solution update of an even step, x += alpha_d p_hat + omega_d s_hat,
    // waits for the odd step that follows (pend = 1 while it is outstanding)
    c128 alpha_d, omega_d;
    double bnorm2, rnorm2, snorm2, rhat_norm2, tol2, true_rnorm2;
    // ||r||^2 at which the next restart from x is due (restarts at every power
    // of ten of ||r|| / ||b||; 0 = none)
    double next2;
    // restarts: after a true-residual check missed rtol (at most 5);
    // decades: at a power of ten of the residual
    int status, iters2, maxit2, matvecs, restarts, pend, decades;
};

// Reduction slots (each holds `nterm` doubles per block per right-hand side).
enum Slot : int {
    SLOT_R = 0,   // ||r||^2, Re/Im r_hat^H r, ||b||^2
    SLOT_V = 1,   // Re/Im r_hat^H v
    SLOT_T = 2,   // Re/Im t^H s, ||t||^2 (from t = A s_hat), ||s||^2 (from the s update)
    NSLOT = 3
};
constexpr int MAX_TERMS = 6;

}  // namespace hh
