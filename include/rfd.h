/*
 * rfd.h -- C ABI of the RF-DDES interface-filter library for AMD MI355X (gfx950).
 *
 * RF-DDES (Kalantzis, Xi, Saad, "Beyond AMLS: domain decomposition with
 * rational filtering", arXiv 1711.09487) computes the eigenpairs of a sparse
 * symmetric pencil A x = lambda M x (M SPD) with lambda in [alpha, beta]:
 *
 *   rfd_create_pencil           the pencil (A, M)                       Sec. 1
 *   rfd_set_partition           interior-first reordering               Sec. 2.3, eq. (2.5)
 *   rfd_set_interval_and_poles  rational filter poles / weights         Sec. 2.1, eqs. (2.1)-(2.3)
 *   rfd_set_precision           FP64, or FP32 factors + FP64 refinement
 *   rfd_set_interface_groups    two-level (nested-dissection) S(zeta)   Sec. 2.3 applied to S, Sec. 7
 *   rfd_filter_interface        Q = orth of 2 Re sum_l w_l S(z_l)^{-1} applied
 *                               to a block (block Krylov)               Sec. 3.1 eq. (3.5), Alg. 3.1
 *   rfd_filter_lanczos          Q by Alg. 3.1 with its stopping test    Sec. 3.2, Alg. 3.1, Sec. 6
 *   rfd_prepare_interior        V_j and B_sigma factors, concurrently   Sec. 4, Alg. 5.1 step 3
 *   rfd_solve_interior          V_j, Sigma_j, Gamma_j and Z             Sec. 4, Sec. 5.1 eqs. (5.2)-(5.5)
 *   rfd_rayleigh_ritz           Ritz pairs in [alpha, beta]             Alg. 5.1 steps 6-8
 *   rfd_inertia_count           eigenvalue count in [alpha, beta]      Sylvester / Haynsworth inertia
 *   rfd_solve_slices            spectrum slicing of [alpha, beta]       Sec. 7
 *   rfd_batch_run               many independent solves at once (whole Alg. 5.1 each)
 *   rfd_server_*                continuous serving of solve requests
 *
 * Conventions (all entry points):
 *  - Every call returns an rfd_status; RFD_OK is 0.  No exception crosses the
 *    ABI.  On error rfd_last_error() returns a message (thread-local, valid
 *    until the next call on the same thread).
 *  - Matrices are column-major, FP64 unless stated.  Index arrays are int32
 *    except CSR row pointers (int64).
 *  - "host" pointers are read (or written) before the call returns; "device"
 *    pointers are HBM addresses on the current HIP device, owned by the
 *    caller, and are read/written by work enqueued on `stream` (0 = the null
 *    stream); the call returns after that work has been enqueued and, where a
 *    host scalar output is produced (mu, k, nfound), after the stream has
 *    reached that point.
 *  - A pencil handle is not thread-safe: use one handle per host thread.
 *  - The library owns its device workspaces; rfd_destroy_pencil frees them.
 */
#ifndef RFD_H_
#define RFD_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rfd_pencil_s* rfd_pencil_t;
typedef void* rfd_stream_t; /* a hipStream_t */

typedef enum {
  RFD_OK = 0,
  RFD_EINVAL = 1,      /* invalid argument or inconsistent input            */
  RFD_ENOMEM = 2,      /* device or host allocation failed                  */
  RFD_EBREAKDOWN = 3,  /* a pivot below the breakdown threshold (singular)  */
  RFD_ENOCONV = 4,     /* iterative refinement did not reach its tolerance  */
  RFD_EDEVICE = 5,     /* a HIP runtime error                               */
  RFD_ESTATE = 6,      /* call out of order (e.g. filter before partition)  */
  RFD_EPENDING = 7     /* a served request has not finished yet             */
} rfd_status;

enum { RFD_RULE_GAUSS = 0, RFD_RULE_MIDPOINT = 1, RFD_RULE_EXPLICIT = 2 };
enum { RFD_FP64 = 0, RFD_FP32_REFINE = 1, RFD_FP32_AUTO = 2 };
enum { RFD_INTERIOR_LU = 0, RFD_INTERIOR_SPECTRAL = 1 };

/*
 * rfd_create_pencil -- the pencil (A, M) of Sec. 1: A symmetric, M symmetric
 * positive definite, both n x n in CSR with FULL symmetric storage (host
 * arrays A_ptr[n+1], A_idx[nnz], A_val[nnz], same for M).  Column indices
 * need not be sorted; duplicates are summed.  The arrays are copied; the
 * caller keeps ownership.  Errors: RFD_EINVAL if n < 1, an index is out of
 * range, A or M is not symmetric (|a_ij - a_ji| > 1e-12 max|a|), or some
 * M_ii <= 0.  Allocates nothing on the device yet.
 */
rfd_status rfd_create_pencil(int64_t n, const int64_t* A_ptr, const int32_t* A_idx,
                             const double* A_val, const int64_t* M_ptr,
                             const int32_t* M_idx, const double* M_val, rfd_pencil_t* out);

/*
 * rfd_set_partition -- the interior-first reordering of eq. (2.5).
 * part[i] in {0..p-1} puts node i in the interior of subdomain part[i];
 * part[i] = -1 makes it an interface node (host array of length n).  Interior
 * nodes of each subdomain and the interface keep ascending global order; the
 * interface block of every interface-sized array in this API uses that order.
 * Errors: RFD_EINVAL if p < 1, a subdomain is empty, a value is out of range,
 * or two different subdomains are coupled directly (in |A| + |M|) rather than
 * through the interface.  Uploads the pencil and index maps to the device
 * (RFD_ENOMEM / RFD_EDEVICE).  Drops every factor and cache of the pencil.
 */
rfd_status rfd_set_partition(rfd_pencil_t pencil, int32_t p, const int32_t* part);

/*
 * rfd_set_interval_and_poles -- the filter of Sec. 2.1 on the circle with
 * centre (alpha+beta)/2 and radius (beta-alpha)/2.  rule = RFD_RULE_GAUSS:
 * n_c Gauss-Legendre nodes on the upper half circle; RFD_RULE_MIDPOINT: the
 * n_c upper-half nodes of the 2 n_c-point midpoint rule (the paper's choice,
 * Sec. 6); RFD_RULE_EXPLICIT: zeta[2 n_c] and omega[2 n_c] (host, interleaved
 * re, im) give the n_c upper-half-plane poles and weights, and the filter is
 * rho(x) = 2 Re sum_l omega_l / (x - zeta_l), eq. (2.3).  For the built-in
 * rules zeta/omega may be NULL.  Errors: RFD_EINVAL if alpha >= beta,
 * n_c < 1 or n_c > 64, or an explicit pole has Im <= 0.  Invalidates the
 * per-pole factors; keeps the per-pencil caches.
 */
rfd_status rfd_set_interval_and_poles(rfd_pencil_t pencil, double alpha, double beta,
                                      int32_t n_c, int32_t rule, const double* zeta,
                                      const double* omega);

/*
 * rfd_set_precision -- RFD_FP64 (default): every factorization and solve in
 * FP64.  RFD_FP32_REFINE: the shifted interior blocks B_j - zeta M_Bj and the
 * Schur complements S(zeta) are factored in FP32 on the matrix cores and
 * every shifted solve is refined in FP64 (FP64 residuals against the FP64
 * operators) until ||r||_F <= refine_tol ||b||_F, at most max_sweeps
 * corrections (refine_tol <= 0 or max_sweeps <= 0 select 1e-13 and 8).
 * RFD_FP32_AUTO: FP32 factors with FP64 refinement where the refinement
 * costs less than the FP32 factorization saves, FP64 factors elsewhere.  The
 * interior blocks (padded to D rows; TS = the trailing rows that hold every
 * row coupled to the interface, those rows being numbered last; SJ = the
 * largest number of interface nodes coupled to one subdomain) are FP64 when
 * D^3 / 6 < SJ (D^2 - TS^2): FP64 factors then need Schur solves on the
 * trailing TS x TS blocks only, while refining FP32 factors needs the full
 * solves (Sec. 3.1 uses only the rows of the solution that E_i touches).
 * Otherwise they are FP32 with a sparse-product refinement residual.
 * S(zeta) is FP32 when sum N^3 > 12 c sum N^2 over its factored
 * blocks (N: their sizes; c: the columns the filter will carry, m * steps
 * for rfd_filter_interface, m * max_steps for rfd_filter_lanczos, m for
 * rfd_filter_apply): each filtered column then costs about 16 N^2 FP64
 * flops more (two residuals and two FP32 solves against one FP64 solve) and
 * the FP32 LU saves about (4/3) N^3.
 * Orthonormalisation, the interior levels' residuals and Rayleigh-Ritz stay
 * FP64.  Errors: RFD_EINVAL for an unknown mode.  Invalidates the factors.
 */
rfd_status rfd_set_precision(rfd_pencil_t pencil, int32_t mode, double refine_tol,
                             int32_t max_sweeps);

/*
 * rfd_filter_interface -- the interface subspace (Sec. 3.1-3.2).
 * Factors B_j - zeta_l M_Bj and S(zeta_l), l = 1..n_c, on the first call
 * after a change of poles/precision/partition, then keeps them.
 * F = 2 Re sum_l omega_l S(zeta_l)^{-1} (eq. (3.5)); with W_1 = F Y0,
 * Q_1 = orth(W_1), Q_t = orth(F Q_{t-1}) against [Q_1..Q_{t-1}] (twice),
 * t = 2..steps, Q = [Q_1 .. Q_steps] (a block form of Alg. 3.1 with full
 * reorthogonalisation).  orth() drops directions whose residual norm is
 * <= 1e-13 times the largest column norm of the unprojected block.
 *   m       block width, 1 <= m <= s
 *   Y0      device, s x m, leading dimension s (FP64)
 *   steps   >= 1
 *   Q       device, s x ldq_cols with leading dimension s, caller-owned;
 *           ldq_cols >= min(s, steps * m); receives mu orthonormal columns
 *   mu      host out: number of columns written
 * Errors: RFD_ESTATE before set_partition / set_interval_and_poles,
 * RFD_EINVAL for bad sizes, RFD_EBREAKDOWN on a pivot below 1e-300 (FP64) or
 * 1e-30 (FP32) in magnitude, RFD_ENOCONV if refinement stalls, RFD_ENOMEM.
 */
rfd_status rfd_filter_interface(rfd_pencil_t pencil, int32_t m, const double* Y0,
                                int32_t steps, double* Q, int64_t ldq_cols, int32_t* mu,
                                rfd_stream_t stream);

/*
 * rfd_filter_apply -- one application of the interface filter, the left side
 * of eq. (3.5): W = 2 Re sum_l omega_l S(zeta_l)^{-1} Y (the factor 2 of
 * eq. (3.5); Alg. 3.1 line 2 omits it, which does not change the range).
 * Uses (and on first use builds) the same factors as rfd_filter_interface.
 *   m   number of columns, m >= 1
 *   Y   device, s x m, leading dimension s (FP64)
 *   W   device, s x m, leading dimension s (FP64), caller-owned; may not alias Y
 * Errors as rfd_filter_interface.
 */
rfd_status rfd_filter_apply(rfd_pencil_t pencil, int32_t m, const double* Y, double* W,
                            rfd_stream_t stream);

/*
 * rfd_filter_lanczos -- the interface subspace by the paper's own driver,
 * Alg. 3.1 (Sec. 3.2), taken on a block of m vectors: Lanczos on
 * F = 2 Re sum_l omega_l S(zeta_l)^{-1} with full reorthogonalisation and the
 * stopping test of line 13.
 *   Q_1 = orth(Y0); for t = 1, 2, ...: W = F Q_t, A_t = Q_t^T W; the sum of
 *   the eigenvalues of the block tridiagonal T_t is its trace
 *   tr(T_t) = sum_i tr(A_i); every test_every vectors (<= 0: 10, as in
 *   Sec. 6) the process stops when tr(T_t) changed by at most tol * |tr(T_t)|
 *   since the previous test (Sec. 6 uses tol = 1e-6); otherwise
 *   Q_{t+1} = orth(W) against Q_1..Q_t (twice; directions below 1e-13 of the
 *   block's largest column norm are dropped, lines 8-9).
 * Q = [Q_1 .. Q_t] at the stop (line 15), or after max_steps blocks, or when
 * the interface is exhausted or no direction survives.  Factors as
 * rfd_filter_interface (shared with it).  rfd_solve_interior uses this Q.
 *   m          block width, 1 <= m <= s
 *   Y0         device, s x m, leading dimension s (FP64)
 *   Q          device, s x ldq_cols (ld s), caller-owned; receives mu columns
 *   mu, steps  host out: columns of Q, block steps taken
 *   traces     host, max_steps doubles (tr(T_t) after block t), or NULL
 *   converged  host out: 1 when the stopping test fired
 * Errors: as rfd_filter_interface; RFD_EINVAL for max_steps < 1, tol < 0 or
 * ldq_cols < min(s, m).
 */
rfd_status rfd_filter_lanczos(rfd_pencil_t pencil, int32_t m, const double* Y0, double tol,
                              int32_t max_steps, int32_t test_every, double* Q, int64_t ldq_cols,
                              int32_t* mu, int32_t* steps, double* traces, int32_t* converged,
                              rfd_stream_t stream);

/*
 * rfd_prepare_interior -- starts the parts of the interior step that do not
 * depend on Q (Sec. 4: the deflation basis V_j for (sigma, nev_b), Alg. 5.1
 * step 3, and the factors of B_j - sigma M_Bj) on a thread and stream of the
 * library's own, and returns at once, so that they run on the device while
 * rfd_filter_interface / rfd_filter_apply work on the caller's stream.
 * rfd_solve_interior with the same sigma and nev_b then reuses them.  Every
 * other call on the pencil first waits for the preparation to finish.
 * Errors: RFD_EINVAL for nev_b < 0 or a non-finite sigma (at this call);
 * errors of the preparation itself (RFD_EBREAKDOWN for a singular B_sigma,
 * RFD_ENOMEM) are returned by the next call on the pencil that waits for it.
 */
rfd_status rfd_prepare_interior(rfd_pencil_t pencil, double sigma, int32_t nev_b);

/*
 * rfd_solve_interior -- the interior part (Sec. 4 and 5.1) for the Q of the
 * last rfd_filter_interface call.
 * V_j: eigenvectors of (B_j, M_Bj) for the nev_b eigenvalues closest to
 * sigma (a cluster at the cut is kept whole), M_Bj-orthonormal (Alg. 5.1
 * step 3; cached per pencil and sigma); for a non-diagonal M they come from
 * the standard form G^{-1} B_j G^{-T} with M_Bj = G G^T.  Sigma_j^(psi),
 * Gamma_j^(psi) as in eqs. (5.2)-(5.4) with B_sigma = B_j - sigma M_Bj (the
 * Gamma_j blocks exist when M couples interiors to the interface, M_E != 0,
 * and give Z psi * mu more columns); every level is made M_Bj-orthogonal to
 * V_j before the next one is formed (this leaves range(Z) unchanged because
 * V_j is part of Z).  Z of eq. (5.5) stays on the device.
 * For a large basis (A Z of 2^24 entries or more) the projected matrix
 * Z^T A Z of rfd_rayleigh_ritz is assembled block by block on a library
 * stream while Z is built, and may still be in progress when this call
 * returns; rfd_rayleigh_ritz waits for it on its own stream, and any later
 * call that reuses the pencil's buffers waits for it first.
 *   k_out   host out: number of columns of Z
 * Errors: RFD_ESTATE without a Q, RFD_EINVAL for nev_b < 0 or psi < 1,
 * RFD_EBREAKDOWN if B_sigma is singular to working precision or a block M_Bj
 * is not positive definite.
 */
rfd_status rfd_solve_interior(rfd_pencil_t pencil, double sigma, int32_t nev_b, int32_t psi,
                              int64_t* k_out, rfd_stream_t stream);

/*
 * rfd_rayleigh_ritz -- Alg. 5.1 steps 6-8: Z^T A Z G = Z^T M Z G Theta on an
 * M-orthonormal basis of range(Z) (directions below 1e-12 relative dropped),
 * Ritz values theta in [alpha, beta] ascending, Ritz vectors x = Z g
 * permuted back to the original numbering, residuals
 * ||A x - theta M x||_2 / (||A|| ||x||_2) with ||A|| the largest absolute row
 * sum of A.
 *   max_out  capacity of the outputs
 *   evals    device, max_out           (FP64)
 *   evecs    device, n x max_out, ld n (FP64), or NULL
 *   resid    device, max_out, or NULL (then not computed)
 *   nfound   host out: number of Ritz values in [alpha, beta]; set also when
 *            it exceeds max_out, in which case RFD_EINVAL is returned and only
 *            the first max_out are written.
 */
rfd_status rfd_rayleigh_ritz(rfd_pencil_t pencil, int32_t max_out, double* evals, double* evecs,
                             double* resid, int32_t* nfound, rfd_stream_t stream);

/*
 * rfd_inertia_count -- the number of eigenvalues of (A, M) in [alpha, beta]
 * by Sylvester's law of inertia: nu(A - beta M) - nu(A - alpha M), nu = the
 * number of negative eigenvalues.  With the partition, Haynsworth's
 * additivity gives nu(A - tau M) = sum_j nu(B_j - tau M_Bj) + nu(S(tau)) at a
 * real tau (Sec. 2.3, 3.1), each counted from the pivots of an FP64 LU without
 * pivoting (with the two-level grouping: of S_gg and of the top complement).
 * alpha and beta should lie in gaps of the spectrum; a pivot that is exactly
 * zero returns RFD_EBREAKDOWN.  Uses the pencil's factor buffers (the next
 * filter call factors again).
 *   count   host out
 * Errors: RFD_ESTATE before set_partition, RFD_EINVAL unless alpha < beta.
 */
rfd_status rfd_inertia_count(rfd_pencil_t pencil, double alpha, double beta, int64_t* count,
                             rfd_stream_t stream);

/*
 * rfd_solve_slices -- spectrum slicing (Sec. 7) on one device: the interval
 * [cuts[0], cuts[nslices]] is split at the host array cuts (nslices + 1
 * strictly increasing values, best placed in spectral gaps), and every slice
 * [cuts[i], cuts[i+1]] runs a whole solve (its own n_c poles of the given
 * rule, rfd_filter_interface with m and steps on the start block Y0 (device,
 * s x m), rfd_solve_interior with sigma and nev_b, psi, rfd_rayleigh_ritz).
 * The slices share the pencil's maps, reordered matrices and workspaces; with
 * a finite sigma they also share the interior basis V_j and the B_sigma
 * factors (computed once); sigma = NaN uses each slice's centre.
 * Outputs are appended slice after slice: evals (device, max_out), evecs
 * (device, n x max_out, or NULL), resid (device, max_out, or NULL); nfound
 * (host) the total; counts (host, nslices, or NULL) per slice; inertia (host,
 * or NULL) the number of eigenvalues in [cuts[0], cuts[nslices]] from
 * rfd_inertia_count, to check the merged result against.  Leaves the pencil's
 * poles at the last slice.
 * Errors: RFD_EINVAL for bad cuts or sizes, or when more Ritz values than
 * max_out are found (nfound and counts are still set); as the calls above.
 */
rfd_status rfd_solve_slices(rfd_pencil_t pencil, int32_t nslices, const double* cuts, int32_t n_c,
                            int32_t rule, int32_t m, const double* Y0, int32_t steps, double sigma,
                            int32_t nev_b, int32_t psi, int32_t max_out, double* evals,
                            double* evecs, double* resid, int32_t* nfound, int32_t* counts,
                            int64_t* inertia, rfd_stream_t stream);

/*
 * rfd_reset_caches -- invalidates every factorization and per-pencil cache
 * (the B_j(zeta), S(zeta) and B_sigma factors, V_j, Z) while keeping the
 * pencil, partition, poles and precision; the next calls recompute them.
 * release = 0 keeps the device buffers for reuse (no allocation on the next
 * solve of the same shape); release = 1 frees them.
 */
rfd_status rfd_reset_caches(rfd_pencil_t pencil, int32_t release);

/* Frees the handle and every device buffer it owns.  NULL is accepted. */
rfd_status rfd_destroy_pencil(rfd_pencil_t pencil);

/* Thread-local message of the last failed call on this thread ("" if none). */
const char* rfd_last_error(void);

/*
 * rfd_pencil_info -- sizes of a partitioned pencil (host outputs, any may be
 * NULL): n, p, s, max interior size, and the device bytes currently held.
 */
rfd_status rfd_pencil_info(rfd_pencil_t pencil, int64_t* n, int32_t* p, int64_t* s,
                           int64_t* d_max, int64_t* device_bytes);

/*
 * rfd_phase_times -- milliseconds spent in each phase of the last calls,
 * measured with HIP events on the work stream (host array of 16 doubles):
 * [0] factor B_j(zeta), [1] Schur solves + refinement, [2] Schur assembly,
 * [3] factor S(zeta), [4] filter solves + refinement, [5] orthonormalisation,
 * [6] interior basis V_j, [7] factor B_sigma, [8] resolvent levels,
 * [9] Rayleigh-Ritz projection, [10] small eigensolve, [11] Ritz vectors and
 * residuals, [12] refinement sweeps (max, Schur solves), [13] refinement
 * sweeps (max, filter solves), [14], [15] reserved.  Timing is enabled by
 * rfd_set_timing(pencil, 1); it adds event records but no synchronisation
 * until this call.
 */
rfd_status rfd_set_timing(rfd_pencil_t pencil, int32_t on);
rfd_status rfd_phase_times(rfd_pencil_t pencil, double* ms16);

/*
 * rfd_set_pole_window -- the filter (eq. (3.5)) sums over the poles; by
 * default the factors of B_j - zeta_l M_Bj's Schur complements S(zeta_l) for
 * all poles are kept on the device together when they fit in the free device
 * memory, and are otherwise computed and applied a window of poles at a time
 * (each window's factors replace the previous ones, so every application of
 * the filter factors again).  max_poles >= 1 caps the window at that many
 * poles; 0 restores the default.  Results do not depend on the window beyond
 * the order of the final sum.  Errors: RFD_EINVAL for max_poles < 0.
 */
rfd_status rfd_set_pole_window(rfd_pencil_t pencil, int32_t max_poles);

/*
 * rfd_set_interior_solver -- how the shifted interior blocks are inverted.
 * RFD_INTERIOR_LU (default): every B_j - zeta_l M_Bj is factored for each
 * pole (Sec. 3.1) and B_j - sigma M_Bj once per sigma (Sec. 4).
 * RFD_INTERIOR_SPECTRAL: the eigendecomposition B_j V_j = M_Bj V_j Lambda_j,
 * V_j^T M_Bj V_j = I, of every subdomain block is computed once per pencil
 * (the expansion (B_j - z M_Bj)^{-1} = V_j (Lambda_j - z I)^{-1} V_j^T of
 * Sec. 4.1, used in the proof of Thm. 4.2) and serves every pole, sigma and
 * interval afterwards: the Schur contributions become X_j = V_j (Lambda_j -
 * zeta I)^{-1} V_j^T Ehat_j (real products, FP64 in either precision mode,
 * no refinement), the resolvent levels V_j (Lambda_j - sigma I)^{-1} V_j^T
 * M_B X, and the deflation vectors V_j of Alg. 5.1 step 3 a column window of
 * the stored eigenvectors.  The decomposition is kept until the pencil is
 * destroyed, re-partitioned or rfd_reset_caches(pencil, 1) releases the
 * buffers; it holds p D^2 + p D SJ doubles (D, SJ: interior and adjacency
 * sizes padded to 64), and for a non-diagonal M another p D^2 (the factors
 * of M_Bj for the standard form) and, when M couples the interiors to the
 * interface, p D SJ (V^T Mhat_E).  Results equal the LU path's up to
 * rounding.  Errors: RFD_EINVAL for another kind; RFD_ESTATE before
 * rfd_set_partition; RFD_EBREAKDOWN (at the next solve) when a block M_Bj is
 * not positive definite.  The next solve rebuilds what depends on the
 * choice.
 */
rfd_status rfd_set_interior_solver(rfd_pencil_t pencil, int32_t kind);

/*
 * rfd_set_interface_groups -- factor S(zeta) in two levels (a nested
 * dissection of the interface: the paper's interior-first reordering of
 * Sec. 2.3, eq. (2.5), applied once more to S itself, as in the recursive
 * form of RF-DDES proposed in Sec. 7).  group[a] (host array over the s
 * interface nodes, in the interface order of rfd_set_partition) is in
 * {0..ngroups-1} for a node of group g and -1 for a node of the top set T.
 * S(zeta) must not couple two different groups: no C or M_C entry may join
 * them and no subdomain may be adjacent to nodes of two groups.  Then, with
 * the groups ordered first, S = [S_GG S_GT; S_GT^T S_TT] with S_GG block
 * diagonal (S is complex symmetric), and the filter solves use its block LU:
 * the group blocks S_gg, X_g = S_gg^{-1} S_gT, the top complement
 * S_TT - sum_g S_gT^T X_g and its LU, all without pivoting (every shifted
 * block has a field of values off the real axis, Sec. 3.1), in the current
 * precision mode (FP32 mode refines against the FP64 blocks).  The result
 * equals the dense S(zeta)^{-1} up to rounding; the work and memory fall from
 * s^2 per pole to sum_g (|g|^2 + |g| |T_g|) + |T|^2, T_g being the top
 * nodes coupled to g.  ngroups = 0 returns to the dense S.  Invalidates the
 * per-pole factors; rfd_set_partition drops the grouping.
 * Errors: RFD_ESTATE before rfd_set_partition; RFD_EINVAL for a value out of
 * range, an empty group, an empty top set, or a coupling between groups.
 */
rfd_status rfd_set_interface_groups(rfd_pencil_t pencil, int32_t ngroups, const int32_t* group);

/*
 * rfd_set_gemm_tuning -- process-wide tile choices of the matrix-core GEMM
 * behind every dense step (LU updates, triangular solves, refinement
 * residuals, basis products; Secs. 3-5), as measured by an autotuner
 * (python -m paper_1711_09487_amd.tune writes them per GPU architecture;
 * the Python binding loads the file of the device's architecture).
 *   entries  host, count x 9 int32: {fp64 (0 FP32, 1 FP64), complex, transA,
 *            transB, floor(log2 M), floor(log2 N), floor(log2 K),
 *            floor(log2 batch), variant} with variant 1: 64 x 64 tile, 2:
 *            128 x 128 tile (real FP32 only), 3: the large-tile FP64 kernel
 *            (FP64 only); log2 values in 0..62
 *   count    number of entries; 0 clears the table (built-in rules only)
 * Products whose class has no entry keep the built-in rules, and so do
 * products an entry's variant cannot run.  Results differ only by rounding.
 * Errors: RFD_EINVAL for a malformed entry (the table is then unchanged).
 */
rfd_status rfd_set_gemm_tuning(const int32_t* entries, int32_t count);

/*
 * rfd_device_arch -- the current HIP device's architecture name (for example
 * "gfx950", without feature suffixes) into buf (host, len bytes, NUL-terminated).
 * Errors: RFD_EINVAL for a null buf or len < 2; RFD_EDEVICE without a device.
 */
rfd_status rfd_device_arch(char* buf, int32_t len);

/*
 * rfd_kernel_accounting / rfd_kernel_stats -- process-wide, sampled timing of
 * selected kernels: the batched GEMM (the matrix-core kernel behind the LU
 * updates, the triangular solves, the refinement residuals and the
 * Rayleigh-Ritz products, Secs. 3-5) and the symmetric mat-vec of the dense
 * eigensolver's tridiagonalization.  With every = k >= 1, one launch in k of
 * each kernel (picked by a fixed hash of the launch count, so that a periodic
 * launch sequence is not sampled at a few phases only; the same launches in
 * every run), and every launch of 1e11 flops or more, gets a pair of HIP
 * events on its own stream, stamped at the
 * kernel's start and end by the launch itself, and its algorithmic flop and
 * byte counts are recorded
 * (GEMM: 2MNK real or 8MNK complex flops; bytes of A and B read once and of
 * C written, plus read when beta != 0; mat-vec: the lower triangle of the
 * trailing block and its vectors).  every = 0 turns it off.
 * rfd_kernel_stats synchronises the events and returns, for 32 keys (host
 * arrays of 32 doubles each), the number of launches, the number timed, and
 * the estimated milliseconds, flops and bytes of all launches (the launches
 * timed for their size summed, the hashed sample of the others scaled by
 * their count over the sample), then clears the record.  Keys 0..15:
 * the hand-written GEMM with key = 8*fp64 + 4*complex + 2*transA + transB;
 * key 16: the tridiagonalization mat-vec; keys 17..24: the large-tile FP64
 * GEMM that takes the large FP64 products, key = 17 + 4*complex + 2*transA +
 * transB; the other keys are unused.
 */
rfd_status rfd_kernel_accounting(int32_t every);
rfd_status rfd_kernel_stats(double* launches, double* sampled, double* ms, double* flops,
                            double* bytes);

/*
 * ---------------------------------------------------------------------------
 * Batching and serving.  A job is one complete solve (Alg. 5.1: poles and
 * weights of Sec. 2.1, the interface filter of Sec. 3 with `steps` block-
 * Krylov steps, the interior part of Sec. 4 and the Rayleigh-Ritz step) on a
 * pencil whose partition is set.  Jobs run on a pool of worker threads, each
 * with its own HIP stream, so the kernels of independent jobs overlap on the
 * device.  A job is admitted when its estimated device footprint fits the
 * memory budget next to the jobs already running and the caches that idle
 * pencils hold (idle pencils' caches are released, least recently used
 * first, to make room); a job larger than the whole budget runs alone.
 * Jobs on one pencil run one at a time, in submission order; the pencil's
 * interval, poles and precision are set from the job, and its per-pencil
 * state (maps, reordered matrices, and the interior basis and B_sigma
 * factors while sigma and nev_b repeat) stays on the device between jobs.
 * While a job on a pencil is queued or running, the caller must not use
 * that pencil handle directly.
 * ---------------------------------------------------------------------------
 */
typedef struct rfd_job {
  double alpha, beta;   /* interval, alpha < beta                                  */
  int32_t n_c;          /* poles in the upper half plane                           */
  int32_t rule;         /* RFD_RULE_GAUSS or RFD_RULE_MIDPOINT                     */
  int32_t mode;         /* RFD_FP64, RFD_FP32_REFINE or RFD_FP32_AUTO              */
  int32_t max_sweeps;   /* refinement sweeps (<= 0: default)                       */
  double refine_tol;    /* refinement tolerance (<= 0: default)                    */
  int32_t m, steps;     /* interface block width and block-Krylov steps            */
  const double* Y0;     /* device, s x m column-major starting block               */
  double sigma;         /* interior shift (Sec. 4)                                 */
  int32_t nev_b, psi;   /* interior eigenvectors per subdomain, resolvent levels   */
  int32_t max_out;      /* capacity of the outputs                                 */
  double* evals;        /* device, max_out: Ritz values in [alpha, beta], ascending */
  double* evecs;        /* device, n x max_out (original numbering) or NULL        */
  double* resid;        /* device, max_out relative residuals or NULL              */
} rfd_job;

typedef struct rfd_result {
  int32_t status;       /* rfd_status of the job                                   */
  int32_t nfound;       /* Ritz values found in [alpha, beta]                      */
  int32_t mu;           /* columns of the interface basis                          */
  int32_t worker;       /* worker (stream) that ran the job                        */
  int64_t k;            /* dimension of the projection subspace                    */
  int64_t bytes;        /* device footprint admitted for the job                   */
  double queued_s;      /* seconds from submission to admission                    */
  double run_s;         /* seconds from admission to completion                    */
  char message[160];    /* error message when status != RFD_OK                     */
} rfd_result;

/*
 * rfd_batch_run -- runs the nb jobs (jobs[i] on pencils[i]; a pencil may
 * appear several times) on `workers` worker streams (<= 0: 4) within a
 * device memory budget of hbm_budget bytes (<= 0: 90% of the free device
 * memory) and returns when all have finished; results[i] (host) receives
 * each job's outcome.  Returns RFD_OK when every job succeeded, otherwise
 * the status of the first failed job (the others still ran).  Errors:
 * RFD_EINVAL for nb < 1 or null arrays.
 */
rfd_status rfd_batch_run(int32_t nb, const rfd_pencil_t* pencils, const rfd_job* jobs,
                         rfd_result* results, int32_t workers, int64_t hbm_budget);

typedef struct rfd_server_s* rfd_server_t;

/*
 * rfd_server_create -- a serving loop with `workers` worker streams (<= 0: 4)
 * and a device memory budget (<= 0: 90% of the free device memory).
 * rfd_server_submit queues a job (copied; Y0 and the outputs must stay valid
 * until the job finishes) and returns its id in *request_id; requests are
 * admitted as workers and memory free up, in submission order except that a
 * request that fits may pass one that does not.  rfd_server_poll returns
 * RFD_EPENDING while the request is queued or running (wait = 0), or blocks
 * until it has finished (wait != 0); on completion *out receives the result
 * and the id is retired (a second poll returns RFD_EINVAL).
 * rfd_server_destroy finishes every submitted request, then stops the workers.
 */
rfd_status rfd_server_create(int32_t workers, int64_t hbm_budget, rfd_server_t* out);
rfd_status rfd_server_submit(rfd_server_t server, rfd_pencil_t pencil, const rfd_job* job,
                             int64_t* request_id);
rfd_status rfd_server_poll(rfd_server_t server, int64_t request_id, int32_t wait,
                           rfd_result* out);
rfd_status rfd_server_destroy(rfd_server_t server);

/*
 * rfd_server_stats -- host snapshot: queued and running requests, bytes
 * admitted to running requests, bytes held by idle pencils' caches, and the
 * number of cache releases made for admission.
 */
rfd_status rfd_server_stats(rfd_server_t server, int32_t* queued, int32_t* running,
                            int64_t* bytes_running, int64_t* bytes_cached, int64_t* evictions);

/*
 * rfd_server_cache_stats -- host snapshot of the per-pencil cache reuse:
 * admitted requests whose pencil still held its device caches from an earlier
 * request (hits: maps, reordered matrices, workspaces, and the interior basis
 * and B_sigma factors while sigma and nev_b repeat), and those whose pencil
 * held none (misses: first use, or caches released to admit other work).
 */
rfd_status rfd_server_cache_stats(rfd_server_t server, int64_t* hits, int64_t* misses);

#ifdef __cplusplus
}
#endif

#endif /* RFD_H_ */
