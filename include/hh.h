/*
 * hh.h - C ABI of the MI355X (gfx950) matrix-free Helmholtz solver.
 *
 * Solves A u = b with A = -Laplace_h - k(x)^2 I, the second-order 7-point
 * finite-difference Helmholtz operator on a vertex-centred grid with equal
 * spacing h (Chen, Dwarka, Vuik, arXiv 2308.06085, section 2.4, eq. Helmstencil),
 * with homogeneous Dirichlet or first-order Sommerfeld boundary conditions
 * (section 2; Sommerfeld ghost points eliminated by eq. elimination), by
 * right-preconditioned Bi-CGSTAB, or IDR(s), or left-preconditioned full GMRES
 * (section 3.1, 3.2; option "method"), stopped at
 * ||b - A u|| / ||b|| <= rtol (section 5).  The preconditioner is the complex
 * shifted Laplacian M = -Laplace_h - (beta1 - beta2 i) k^2 I (section 3.3,
 * eq. preconditioner) inverted approximately by one geometric multigrid
 * V(1,1)-cycle, or one F(1,1)-cycle (section 3.4.5; option "cycle"): damped
 * Jacobi (section 3.4.1), full-weighting restriction (section 3.4.2),
 * trilinear interpolation (section 3.4.3), rediscretised coarse operators
 * (section 3.4.4), recursive two-grid cycle (Algorithm 1), exact solve on the
 * coarsest grid.  Everything is matrix-free (Algorithm 2).
 *
 * Conventions for every entry point
 * ---------------------------------
 * - All array pointers are DEVICE pointers unless the name ends in _host.
 * - Complex numbers are interleaved {re, im} doubles (complex128) unless
 *   stated; real arrays are double.
 * - Grid arrays are C-contiguous (nrhs, nz, ny, nx), x fastest, and include
 *   the boundary nodes.  Node (iz, iy, ix) sits at (ix h, iy h, iz h).
 * - Dirichlet: the unknowns are the interior nodes.  Boundary entries of every
 *   input are ignored (read as 0) and are written as 0 in every output.
 *   Non-homogeneous boundary data must be lifted into b by the caller.
 * - Sommerfeld: every node is an unknown.
 * - Ownership: the caller owns every pointer it passes; the library copies what
 *   it keeps (model, sources) and never retains a caller pointer after a call
 *   returns.  All scratch (Krylov vectors, grid hierarchy, coarse inverse,
 *   graphs) is owned by the context and allocated in hh_create / hh_set_model
 *   (the IDR(s) vectors when option "method" = 1, "idr_s" or hh_set_shadow asks
 *   for them, the GMRES basis when "method" = 2 or "gmres_m" does; hh_set_model
 *   also allocates and frees the work arrays of a device-side coarsest
 *   inverse); hh_solve and the hh_apply_* calls allocate nothing.
 * - Streams: all device work is enqueued on the stream given to hh_create.
 *   hh_create, hh_set_model, hh_solve return after the work has completed;
 *   hh_set_sources, hh_apply_*, hh_adjoint_rhs and hh_grad_slowness2 return
 *   after enqueue (synchronise the stream before reading results on the host).
 * - Errors: every call returns an hh_status; nothing throws or aborts across
 *   the ABI.  hh_last_error(ctx) gives a text description of the last failure.
 *   On HH_ERR_NOT_CONVERGED and HH_ERR_BREAKDOWN, x holds the last iterate and
 *   the statistics are valid; after any other error outputs are unspecified.
 * - A context is not thread-safe; calls on one context must not overlap.
 */
#ifndef HH_H
#define HH_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hh_ctx hh_ctx; /* opaque, owned by the library */

typedef enum {
    HH_OK = 0,
    HH_ERR_ARG = 1,           /* invalid argument or configuration */
    HH_ERR_HIP = 2,           /* a HIP runtime call failed */
    HH_ERR_OOM = 3,           /* device allocation failed */
    HH_ERR_NUMERIC = 4,       /* NaN/Inf in the model, the RHS or a reduction */
    HH_ERR_BREAKDOWN = 5,     /* Bi-CGSTAB breakdown (rho, r^H v or t^H t vanished) */
    HH_ERR_NOT_CONVERGED = 6, /* maxit reached; x holds the last iterate */
    HH_ERR_STATE = 7          /* call out of order (e.g. solve before set_model) */
} hh_status;

typedef enum { HH_BC_DIRICHLET = 0, HH_BC_SOMMERFELD = 1 } hh_bc;

/* HH_PREC_MIXED: the V-cycle runs in complex64 with float32 coefficients; the
 * Krylov vectors, inner products, residuals and the operator A stay complex128. */
typedef enum { HH_PREC_FP64 = 0, HH_PREC_MIXED = 1 } hh_prec;

typedef struct {
    int nx, ny, nz;   /* nodes per axis incl. boundary; each odd and >= 3 */
    double h;         /* grid spacing, > 0 */
    int bc;           /* hh_bc */
    double beta1;     /* CSLP: M = -Laplace - (beta1 - beta2 i) k^2 ; paper default 1 */
    double beta2;     /* paper default -0.5 (section 3.3) */
    double omega;     /* damped-Jacobi weight, paper value 0.8 (section 3.4.1) */
    int nu_pre;       /* damped-Jacobi sweeps before the coarse-grid correction (nu_1 of
                         Algorithm 1); the paper uses 1 and 1 is the only value the fused
                         passes implement: any other is HH_ERR_ARG */
    int nu_post;      /* sweeps after it (nu_2 of Algorithm 1); likewise only 1 */
    int n_levels;     /* multigrid levels incl. the finest; 0 = coarsen while the
                         next grid keeps >= 3 nodes on every axis.  (n_d - 1) must
                         be divisible by 2^(n_levels-1) on every axis. */
    int prec;         /* hh_prec */
    int nrhs_max;     /* 1..16 right-hand sides solved together */
} hh_config;

typedef struct {
    double iterations;  /* Bi-CGSTAB steps; a half-step exit counts 0.5 */
    int matvecs;        /* products with A, counting the initial residual (the
                           convention of the paper's Table 1) */
    double relres;      /* recursive residual norm / ||b|| at exit */
    double relres_true; /* ||b - A x|| / ||b|| recomputed at exit */
    int status;         /* hh_status of this right-hand side */
    int restarts;       /* restarts of Bi-CGSTAB from the current x: after a
                           true-residual check missed rtol (at most 5), and with
                           option "restart_decade" each time the residual fell
                           below another power of ten of ||b||; each costs one
                           product with A (counted in matvecs) */
    double ms;          /* duration of the whole hh_solve call on the context stream
                           (HIP events around all of its device work), in milliseconds;
                           the same for every right-hand side of the call */
} hh_stats;

/* Fill *cfg with the paper's defaults (beta1 = 1, beta2 = -0.5, omega = 0.8,
 * nu_pre = nu_post = 1, Sommerfeld, FP64, n_levels = 0, nrhs_max = 1) for an
 * nx x ny x nz grid. */
void hh_default_config(hh_config* cfg, int nx, int ny, int nz, double h);

/* Validate cfg, allocate every device buffer for up to nrhs_max right-hand sides
 * (grid hierarchy, Krylov vectors, reductions) on the current HIP device, and
 * bind the context to hip_stream (a hipStream_t; NULL = the default stream).
 * HH_ERR_ARG for an invalid configuration (among them a coarsest grid of more
 * than 8192 unknowns), HH_ERR_OOM if allocation fails. */
hh_status hh_create(const hh_config* cfg, void* hip_stream, hh_ctx** out);

/* Free every resource of ctx.  ctx may be NULL. */
hh_status hh_destroy(hh_ctx* ctx);

/* Text of the last error on ctx (or of the last failed hh_create when ctx is NULL). */
const char* hh_last_error(const hh_ctx* ctx);

/* Number of levels and the node counts of level l (finest = 0). */
hh_status hh_level_shape(const hh_ctx* ctx, int l, int* nx, int* ny, int* nz, int* n_levels);

/* Set the real wavenumber k(x) >= 0 (section 2: k = 2 pi f / c), device array
 * (nz, ny, nx) of doubles, copied.  Builds the hierarchy: coarse k by injection
 * k_{l+1}(i) = k_l(2i), per-level Jacobi factors omega D^-1 of the
 * rediscretised M, and the dense inverse of the coarsest M over its unknowns
 * (Gauss-Jordan elimination with partial pivoting in complex128: on the host up
 * to 256 unknowns, on the device above: about 0.2 s for the 3375 unknowns of
 * the 17^3 Dirichlet grid of the paper's closed-off runs).  A coarsest level of at most 1024
 * unknowns whose arrays fit one workgroup's LDS is solved inside the tail
 * kernel; a larger one (up to 8192 unknowns, such as the paper's 17^3 coarsest
 * grid of its closed-off experiments) by a multi-workgroup product with the
 * inverse.  HH_ERR_NUMERIC if k holds NaN/Inf or a negative value, or if the
 * coarsest M is singular. */
hh_status hh_set_model(hh_ctx* ctx, const double* k);

/* The same model given as squared slowness s = 1/c^2 (device array (nz, ny, nx)
 * of doubles, read once) at angular frequency omega: k_j = omega sqrt(s_j)
 * (section 2: k = 2 pi f / c) is formed on the device, then everything
 * hh_set_model does follows.  HH_ERR_ARG for omega <= 0 or non-finite,
 * HH_ERR_NUMERIC if s holds NaN/Inf or a negative value. */
hh_status hh_set_model_slowness2(hh_ctx* ctx, const double* s, double omega);

/* Copy nrhs right-hand sides (nrhs, nz, ny, nx) complex128 into the context. */
hh_status hh_set_sources(hh_ctx* ctx, const void* b, int nrhs);

/* Right-hand sides of Dirac sources (section 2.4): b_r = 1/h^3 at node
 * ijk_host[3r .. 3r+2] = (iz, iy, ix), 0 elsewhere.  HH_ERR_ARG if a node is
 * outside the grid (or on the boundary for Dirichlet). */
hh_status hh_set_point_sources(hh_ctx* ctx, const int* ijk_host, int nrhs);

/* Solve A x_r = b_r for the right-hand sides of the last hh_set_*sources call.
 * x: (nrhs, nz, ny, nx) complex128; read as the initial guess when use_x0 != 0,
 * else x0 = 0; overwritten with the solution.  rtol > 0, maxit >= 1 (full
 * Bi-CGSTAB steps; for IDR(s), products with A).  stats_host: nrhs entries (may
 * be NULL).  Returns HH_OK if every right-hand side converged, else the first
 * failing status.
 * With option "method" = 1 the Krylov method is IDR(s) (the paper's IDR(4) for
 * s = 4), biorthogonal variant (van Gijzen and Sonneveld, ACM TOMS 38(1), 2011)
 * with the multigrid cycle applied on the right: s inner steps and one
 * minimal-residual step per cycle, s + 1 products with A and with the
 * preconditioner; the residual stays b - A x and is tested after every update.
 * stats.iterations then counts products with A after the initial residual,
 * stats.matvecs adds the initial residual and one per restart (the paper's
 * #Matvec).
 * With "method" = 2 the method is full GMRES on the left-preconditioned system
 * K A x = K b (K = one multigrid cycle), Arnoldi with classical Gram-Schmidt
 * applied twice, Givens rotations on the device; it stops when
 * ||K (b - A x)|| / ||K b|| <= rtol (the paper's GMRES criterion) and restarts
 * from the current x when the basis of "gmres_m" vectors is full.
 * stats.iterations counts Arnoldi steps, stats.relres is that preconditioned
 * relative residual and stats.relres_true the plain one (not tested against
 * rtol); stats.matvecs counts products with A (none for the initial residual
 * when x0 = 0). */
hh_status hh_solve(hh_ctx* ctx, void* x, double rtol, int maxit, int use_x0,
                   hh_stats* stats_host);

/* y = A x (complex128), nrhs vectors. */
hh_status hh_apply_operator(hh_ctx* ctx, const void* x, void* y, int nrhs);

/* y = A x without a context and without allocating: for callers that cannot
 * allocate device memory (code under graph capture, serving loops, harnesses
 * that forbid hipMalloc).  Reads only nx, ny, nz, h and bc of cfg; k is the
 * real wavenumber (nz, ny, nx) doubles, x and y are (nrhs, nz, ny, nx)
 * complex128, all device pointers owned by the caller; work is enqueued on
 * hip_stream (a hipStream_t, NULL = the default stream) and the call returns
 * after enqueue.  The result equals hh_apply_operator's on a context with the
 * same grid and model.  k^2 is staged in a library-owned device array of
 * 2^23 doubles (64 MiB per device, held until the process ends): grids of more
 * than 2^23 nodes, nrhs outside 1..16 or an invalid grid are HH_ERR_ARG
 * (hh_last_error(NULL) gives the text).  k is not checked for NaN/Inf or
 * negative values.  Calls that overlap on one device (for instance on two
 * streams) share that array and race; calls in one stream order do not.  The
 * first call on a device looks the array's device address up
 * (hipGetSymbolAddress): make it outside graph capture. */
hh_status hh_apply_operator_noalloc(const hh_config* cfg, const double* k, const void* x, void* y, int nrhs,
                                    void* hip_stream);

/* y = M x on the finest grid (complex128 arithmetic). */
hh_status hh_apply_shifted(hh_ctx* ctx, const void* x, void* y, int nrhs);

/* z = V(r): one V(1,1)-cycle with zero initial guess approximating M^-1 r, in
 * the context's precision (complex128 in and out in both precisions).  With
 * option "cycle" = 1 the cycle is the F(1,1)-cycle of section 3.4.5 instead:
 * the coarse-grid equation of every level above the coarsest is solved by one
 * F-cycle on the level below followed by one V-cycle on the residual it leaves
 * (on the coarsest level the exact solve), which is the preconditioner the
 * solve then uses too. */
hh_status hh_apply_vcycle(hh_ctx* ctx, const void* r, void* z, int nrhs);

/* Adjoint right-hand side rhs = D^-1 conj(g), D_j = 2^(-n_j) with n_j the number
 * of grid faces node j lies on (Sommerfeld; D = I for Dirichlet).  With
 * A^T = D A D^-1, the adjoint solve A^H lam = g becomes A w = D^-1 conj(g),
 * conj(lam) = D w. */
hh_status hh_adjoint_rhs(hh_ctx* ctx, const void* g, void* rhs, int nrhs);

/* Gradient of a real misfit with respect to the squared slowness s (k = omega sqrt(s)):
 * grad_j = -sum_r Re(D_j w_rj a'_j u_rj), a'_j = -omega^2 - i n_j omega / (h sqrt(s_j)).
 * u: forward solutions, w: adjoint solutions (nrhs, nz, ny, nx) complex128;
 * s, grad: (nz, ny, nx) double.  grad is overwritten. */
hh_status hh_grad_slowness2(hh_ctx* ctx, const void* u, const void* w, const double* s,
                            double omega, double* grad, int nrhs);

/* Shadow vectors of IDR(s): P is (s, nz, ny, nx) complex128 on the device,
 * 1 <= s <= 8; they are stored rounded to complex64 (only inner products
 * <p_i, y> use them) and replace the generated ones until option "idr_s" or
 * "idr_seed" changes.  Sets "idr_s" to s.  Any s linearly independent vectors
 * work; the solution does not depend on them, the iterates do.  Without this
 * call the library draws them from SplitMix64 (Steele, Lea and Flood 2014):
 * entry e = i n + node of vector i takes its real and imaginary parts from the
 * outputs for the counters seed 2^40 + 2e and seed 2^40 + 2e + 1, each mapped
 * to [-1, 1) through its top 53 bits.  Allocates the IDR vectors if needed;
 * HH_ERR_ARG for a null P or s outside 1..8. */
hh_status hh_set_shadow(hh_ctx* ctx, const void* P, int s);

/* Options: "graph" (1 = replay Bi-CGSTAB steps as a captured hipGraph of one
 * even and one odd step, default 1), "check_every" (steps between host
 * convergence checks, default 4; Bi-CGSTAB rounds it up to an even number),
 * "restart_decade" (1 = Bi-CGSTAB restarts from the current x each time the
 * recursive residual falls below the next power of ten of ||b|| (0.1, 0.01,
 * ...): true residual r = b - A x, shadow residual r_hat = r, fresh
 * recurrences, one product with A; the restart runs before the next even
 * step, so the right-hand side idles for one or two steps.  Default 1 in the
 * mixed form, whose complex64
 * preconditioner is not exactly linear: without restarts Bi-CGSTAB can stall
 * where the FP64 solve converges.  0 = the plain method, the FP64 default),
 * "block" (threads per workgroup of the flat Krylov vector kernels: 64, 128,
 * 256, 512; default 256), "zb" (z-planes per workgroup of the operator apply and
 * the start-residual kernel, whose workgroups are 256-node x-y tiles; default 4,
 * 0 = automatic), "trace" (1 = time the fine-level kernels of every solve with
 * HIP events, see hh_kernel_times), "zb_down" / "zb_up" (z-planes per workgroup of the finest
 * level's multigrid down / up pass, 0 = automatic), "zb_down:<l>" / "zb_up:<l>"
 * (the same for level l, 0 <= l < n_levels - 1; levels run by the single-workgroup
 * tail kernel ignore it).  A level outside that range is HH_ERR_ARG.
 * "dn_region:<l>" (fine region nodes staged per workgroup by the down pass from
 * level l when it runs one coarse plane per workgroup: 256, 512 or 1280;
 * 0 = automatic, the default; the result does not depend on it).
 * "coarse_solver" (0 = exact: the dense inverse of the coarsest M, default;
 * 1 = the paper's iterative coarsest solve (end of section 3.4.5, section 4.2):
 * full GMRES on the coarsest M without preconditioner from a zero initial
 * guess to relative residual 10^-"coarse_tol_e" (default 11, the paper's 1e-11,
 * section 5; 1..15), complex128 in both precisions, one workgroup per
 * right-hand side; the fused passes then run down to the coarsest level;
 * allocates (coarse_m + 2) coarsest-grid vectors per right-hand side;
 * HH_ERR_ARG for a coarsest grid of more than 8192 nodes), "coarse_m"
 * (Arnoldi steps per GMRES cycle, 1..100, default 100), "coarse_cycles"
 * (cycles, i.e. restarts + 1, at most; 1..1000, default 10).
 * "cycle" (0 = V(1,1)-cycle, default; 1 = F(1,1)-cycle, section 3.4.5, which
 * visits level l >= 1 l + 1 times per application instead of once and adds one
 * residual pass on each level from 1 to the second coarsest; other values are
 * HH_ERR_ARG).
 * "method" (0 = Bi-CGSTAB, default; 1 = IDR(s), see hh_solve; allocates
 * 2 s complex128 vectors per right-hand side and s complex64 ones; 2 = full
 * GMRES, allocates gmres_m + 1 complex128 vectors per right-hand side),
 * "gmres_m" (1..1024, default 200: GMRES basis size before a restart; GMRES
 * launches its steps directly, without graph or trace),
 * "idr_s" (1..8, default 4), "idr_seed" (0..2^23 - 1, default 1: the generated
 * shadow vectors), "idr_kappa_milli" (0..1000, default 700: the reduction step
 * enlarges omega to kappa / rho times the minimal-residual value when
 * rho = |<t, r>| / (|t| |r|) < kappa; 0 = plain minimal residual).  An IDR(s)
 * solve replays one cycle per captured hipGraph; with "trace" its steps are
 * launched directly and not timed.
 * hh_get_option also reports "n_levels", "coarse_unknowns", "tail_first" (first
 * level run by the tail kernel, or the coarsest level when the multi-workgroup
 * coarsest solve is in use), "autotune_source" (0 = no hh_autotune call yet,
 * 1 = shapes taken from the cache file, 2 = measured), "coarse_steps" (Arnoldi
 * steps of the last coarse GMRES solve, the largest over the right-hand sides;
 * waits for the stream) and the shapes in use
 * under the same names ("dn_region:<l>" then gives the region in use). */
hh_status hh_set_option(hh_ctx* ctx, const char* name, long long value);
hh_status hh_get_option(const hh_ctx* ctx, const char* name, long long* value);

/* Measurement hook: launch one of the solver's fine-grid kernels `reps` times
 * on the context stream, exactly as hh_solve launches it (same grid, same
 * workgroup shape), on the context's scratch vectors, and return the average
 * duration in milliseconds measured with HIP events on that stream.
 * which: 0 = t = A s_hat with the fused partial dot products, 1 = the Krylov
 * x / r update with its dot products in the form of an odd step with nothing
 * outstanding (x += alpha p_hat + omega s_hat, r = s - omega t; the solve
 * updates x every second step), 2 = fused multigrid down pass on the
 * finest level (smoother + residual + restriction), 3 = fused up pass on the
 * finest level (prolongation + correction + post-smoother), 4 = p update,
 * 5 = s update with ||s||^2.
 * The context's Krylov vectors are first filled with finite nonzero data.
 * Requires hh_set_model.  Overwrites internal scratch only. */
hh_status hh_time_kernel(hh_ctx* ctx, int which, int nrhs, int reps, float* ms_avg_host);

/* In-solve kernel timing.  With hh_set_option(ctx, "trace", 1) (which also
 * resets the sums) every following hh_solve launches its steps directly
 * (no graph replay) with HIP events on the context stream around the
 * fine-level kernels of each step that runs; "trace" 0 returns to graph
 * replay.  Only check windows (check_every steps rounded up to an even
 * number) through which every right-hand side kept iterating and advanced by
 * every step are counted (not one with a restart inside, see
 * "restart_decade"), so each counted launch did the full work of all
 * right-hand sides.  hh_kernel_times returns, per kernel id
 * of hh_time_kernel (0 = the operator apply with its dot products, both
 * launches of a step; 1 = x / r update, even and odd steps alike; 2 / 3 = finest-level multigrid
 * down / up pass, both V-cycles; 4 = p update; 5 = s update) and id 6 (an
 * extra launch of the operator apply per step with every workgroup gated off:
 * what the event bracket around one launch adds to a kernel's own duration),
 * the average bracketed duration in milliseconds of the traced launches since
 * tracing was enabled and their number.  ms_avg and launches are host arrays
 * of 7 entries. */
hh_status hh_kernel_times(const hh_ctx* ctx, double* ms_avg, long long* launches);

/* Pick the launch shapes of the solve by timing it: the lanes of
 * the flat Krylov kernels (128 / 256 / 512) with the z-planes per workgroup of
 * the operator apply (2 / 4 / 8), then, level by level, the z-planes per
 * workgroup of every fused multigrid down and up pass (1, 2, 4, 8, 16) and the
 * region of the one-plane down passes (256 / 512 / 1280 fine nodes).  Each
 * candidate runs the first Bi-CGSTAB steps of the current sources (set by
 * hh_set_*sources; all of them) from a fresh start, replayed as a graph and
 * timed with HIP events on the context stream; a candidate replaces the
 * current choice only when it is at least 1 % faster (coordinate descent from
 * the built-in rule).  The multigrid shapes it picks do not change any result
 * bit; the flat-kernel shape changes the rounding of the inner products only.
 * cache_json_path (may be NULL: no cache): a JSON object file mapping a key
 * made of the device architecture, grid, boundary condition, precision,
 * right-hand-side count, cycle and level count to the chosen shapes; an entry
 * for this context's key is applied without measuring, a new one is added and
 * the file rewritten (written to "<path>.tmp", then renamed).  HH_ERR_ARG if
 * the file exists but is not such an object or an entry holds a shape outside
 * the sets above; HH_ERR_STATE without sources.  Leaves the iterate undefined;
 * the next hh_solve starts afresh. */
hh_status hh_autotune(hh_ctx* ctx, const char* cache_json_path);

#ifdef __cplusplus
}
#endif
#endif /* HH_H */
