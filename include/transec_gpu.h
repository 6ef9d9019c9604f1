/* libtransec_gpu: partitioned shift-without-invert eigensolution of the
 * complex-symmetric real-space operator A = H - i(Gamma_L + Gamma_R) and the
 * transmission T(E), on one AMD Instinct MI355X (gfx950).
 *
 * Method: B. Feldman and Y. Zhou, "A partitioned shift-without-invert
 * algorithm to improve parallel eigensolution efficiency in real-space
 * electronic transport", arXiv:1606.01139.
 *
 * Conventions for every entry point:
 *   - Every function returns a tsg_status and never aborts or throws.  On any
 *     status other than TSG_OK, tsg_last_error() describes the failure.
 *   - The caller owns every input array; the library copies what it needs
 *     during the call and keeps no pointer to caller memory.
 *   - Outputs go to caller-allocated arrays with an explicit capacity;
 *     TSG_ECAPACITY reports that the capacity was too small and sets the
 *     count output to the size needed.
 *   - "host" arrays are in CPU memory; "device" arrays are in the GPU memory
 *     of the device that is current when the context is built.
 *   - Grid vectors are indexed n = x + nx (y + ny z) (x fastest); a block of
 *     B vectors stores each vector contiguously: element (n, c) at
 *     ptr[c * ld + n] with ld >= N.
 *   - Complex numbers are pairs (re, im) of the stated real type.
 *   - Units are Hartree and bohr.
 *   - A context is used by one host thread at a time; distinct contexts are
 *     independent.  GPU work of a context runs on its stream, except that a
 *     solve drains that stream, runs on internal streams (one per window
 *     group) and has finished when it returns.
 */
#ifndef TRANSEC_GPU_H
#define TRANSEC_GPU_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TSG_OK = 0,
  TSG_EINVAL = 1,      /* invalid argument (null pointer, size, non-finite value) */
  TSG_ENOMEM = 2,      /* device or host allocation failed */
  TSG_ENOCONV = 3,     /* a window did not converge within max_restarts; the converged subset is kept */
  TSG_EBREAKDOWN = 4,  /* block orthogonalisation lost rank and could not recover */
  TSG_EDEVICE = 5,     /* HIP runtime error, or no usable gfx950 device */
  TSG_ESTATE = 6,      /* call out of order (e.g. transmission before a solve) */
  TSG_ECAPACITY = 7    /* output capacity too small; count output holds the size needed */
} tsg_status;

enum { TSG_FP64 = 0, TSG_FP32_BULK = 1 };                 /* tsg_opts.precision */
enum { TSG_PLAN_ALG1 = 0, TSG_PLAN_EQUAL = 1, TSG_PLAN_SAMPLED = 2, TSG_PLAN_SEMICLASSICAL = 3 }; /* tsg_plan_windows mode */
enum { TSG_SELECT_NEAREST = 0, TSG_SELECT_SMALLEST_REAL = 1, TSG_SELECT_LARGEST_REAL = 2 };
enum { TSG_C128 = 0, TSG_C64 = 1 };                       /* element types of device blocks */
enum { TSG_EXTRACT_RITZ = 0, TSG_EXTRACT_HARMONIC = 1 };   /* tsg_opts.extraction */

typedef struct tsg_ctx tsg_ctx;

/* Uniform real-space grid (Section 1: N ~ V / h^3 points, spacing h).
 * fd_radius R in 1..6 selects the central difference of order 2R for the
 * Laplacian (default 6). */
typedef struct {
  int32_t nx, ny, nz;
  double h;
  int32_t fd_radius;
} tsg_grid;

/* Gaussian absorbers (Section 1; Section 3 gives amplitude and standard
 * deviation): Gamma_X(z) = amp_X exp(-(z - z_X)^2 / (2 width_X^2)). */
typedef struct {
  double amp_L, width_L, z_L;
  double amp_R, width_R, z_R;
} tsg_absorber;

/* One spectral partition (Eq. (3)): shift E_{S,j} and count n_{r,j}.  The
 * shift is real (shift_im = 0) on the paper's one-dimensional partitioning;
 * a nonzero shift_im places the window in the complex plane (the
 * two-dimensional partitioning Section 2 proposes for strongly
 * non-Hermitian operators, whose eigenvalues spread down to -max Gamma,
 * Eq. (5)). */
typedef struct {
  double shift;
  int32_t nev;
  double shift_im;
} tsg_window;

/* Solver options.  tsg_default_opts() fills every field. */
typedef struct {
  int32_t precision;    /* TSG_FP64, or TSG_FP32_BULK: complex64 block work then an FP64 polish */
  double tol;           /* backward error ||A u - theta u|| / (||A||_G ||u||) to reach (default 1e-8) */
  int32_t block;        /* vectors per block step b (default 2) */
  int32_t basis;        /* basis size m per window (0: automatic, about 9 n_{r,j} and at least 40) */
  int32_t keep;         /* vectors kept at a restart k (0: automatic, about m/2) */
  int32_t max_restarts; /* per window (default 2000) */
  uint64_t seed;        /* start-vector seed */
  int32_t keep_lowest;  /* combine keeps only the n lowest by real part (0: keep all) */
  int32_t select;       /* TSG_SELECT_NEAREST ('SM' on the shifted operator), or an exterior selection */
  double bulk_tol;      /* TSG_FP32_BULK: backward error the complex64 phase stops at (default 1e-5) */
  int32_t graphs;       /* 1 (default): each restart cycle after the first is captured once as a
                           hipGraph and replayed; 0: every kernel is launched directly */
  int32_t groups;       /* windows are dealt round-robin into this many groups, each a batched
                           iteration on its own internal stream and host thread, so that the groups'
                           small eigensolves and expansion steps can overlap (default 1: one batch,
                           the faster choice measured on MI355X) */
  int32_t imag_bands;   /* tsg_plan_windows, TSG_PLAN_SEMICLASSICAL: q >= 1 (default 1).  With q > 1
                           the p windows are p/q real placements of n_r/(p/q) pairs, each split into
                           q windows at imaginary shifts -max(Gamma) (i + 1/2)/q, i < q, of equal
                           counts (two-dimensional partitioning); p must be a multiple of q */
  int32_t extraction;   /* TSG_EXTRACT_RITZ (default): Ritz pairs of V^H A V nearest the shift;
                           TSG_EXTRACT_HARMONIC: harmonic Ritz pairs for the shift (the pairs
                           (sigma + nu, V y) with ((A - sigma) V)^H ((A - sigma) V y - nu V y) = 0, the
                           cheap variant of the mixed inversion Section 2 proposes for interior
                           windows), ordered by |nu| and estimated by their Rayleigh quotients */
} tsg_opts;

/* Per-window solver statistics of the last solve. */
typedef struct {
  double shift;             /* real part of the window's shift */
  int32_t nev;
  int32_t n_conv;
  int32_t restarts;
  int64_t matvecs;          /* single-vector operator applications */
  double max_backward_error;
  int32_t restarts_bulk;    /* FP32-bulk: restarts spent in the complex64 phase */
  int32_t breakdowns;       /* block steps whose new block A P lay in the span of the basis (to within
                               1e-12 ||A||_G in FP64, 1e-6 in complex64) and was replaced by a fresh
                               random block orthonormal to the basis */
  int32_t cnorm_failures;   /* converged pairs dropped because u^T u vanished (|u^T u| < 1e-10 ||u||^2):
                               such a vector cannot be c-normalised (bi-orthogonality of Section 1 fails) */
  double shift_im;          /* imaginary part of the window's shift */
} tsg_window_stats;

/* Fills *opts with the defaults listed in tsg_opts. */
void tsg_default_opts(tsg_opts* opts);

/* Builds the operator of Eq. (1) on the current device and returns a new
 * context in *out.
 *   grid:       grid sizes (each >= 1), spacing h > 0, fd_radius 1..6;
 *   V:          host, N = nx ny nz finite doubles, the local potential V(r);
 *   ab:         absorber parameters (amplitudes >= 0, widths > 0, finite);
 *   hip_stream: hipStream_t the context uses (NULL: the null stream).
 * Errors: TSG_EINVAL, TSG_ENOMEM, TSG_EDEVICE.  On error *out is NULL. */
tsg_status tsg_build_operator(const tsg_grid* grid, const double* V, const tsg_absorber* ab,
                              void* hip_stream, tsg_ctx** out);

/* Algorithm 1, first part (Section 2.2).  E_min is the real part of the
 * eigenvalue of smallest real part (an exterior solve); E_max is the exact
 * upper bound max V + 3 max|symbol|/(2h^2) on the real parts.  Modes:
 *   TSG_PLAN_ALG1:    n_{r,j} from the load-balancing formula and
 *                     E_{S,j} = E_{S,j-1} + ((E_max - E_min)/N)(n_{r,j} + n_{r,j-1})/2,
 *                     with E_{S,0} = E_min and n_{r,0} = 0;
 *   TSG_PLAN_EQUAL:   the same shifts with n_{r,j} = n_r/p;
 *   TSG_PLAN_SAMPLED: n_{r,j} = n_r/p; the local eigenvalue density is
 *                     sampled by solving 8 eigenpairs at each of max(2p, 8)
 *                     shifts (Section 2.2's density estimate) and the shifts
 *                     are the midpoints of consecutive intervals of n_{r,j}
 *                     eigenvalues of the integrated density;
 *   TSG_PLAN_SEMICLASSICAL: n_{r,j} = n_r/p; the shifts are the midpoints
 *                     of consecutive intervals of n_{r,j} eigenvalues of the
 *                     semiclassical counting function (phase-space volume of
 *                     p^2/2 + V over the box with Weyl's Dirichlet surface
 *                     term), a density estimate that needs no eigensolve
 *                     beyond E_min.
 *   out:     host, capacity p windows;
 *   e_range: host, 2 doubles {E_min, E_max}, or NULL.
 * Errors: TSG_EINVAL (n_r < 1, p < 1, mode), TSG_ESTATE (no convergence),
 * TSG_EDEVICE.  Stored partitions are left unchanged; a combined set is
 * discarded. */
tsg_status tsg_plan_windows(tsg_ctx* ctx, int32_t n_r, int32_t p, int32_t mode, const tsg_opts* opts,
                            tsg_window* out, double* e_range);

/* Solves one partition of Eq. (3): the win.nev eigenpairs of A closest to
 * win.shift (Section 2.1, 'SM' on the shifted operator, no inversion), and
 * appends it to the context's list of partitions (a continuation run in the
 * sense of Section 2).  *n_conv gets the number converged: a partition keeps
 * only the pairs whose backward error is at most opts->tol.
 * Errors: TSG_EINVAL, TSG_ENOCONV (converged subset kept), TSG_EBREAKDOWN (a
 * converged pair had u^T u = 0 and was dropped, see tsg_window_stats; takes
 * precedence over TSG_ENOCONV), TSG_EDEVICE. */
tsg_status tsg_solve_partition(tsg_ctx* ctx, tsg_window win, const tsg_opts* opts, int32_t* n_conv);

/* Clears the partition list, solves all p windows together (one batched
 * iteration on the device), then combines them (tsg_combine).
 *   windows:    host, p entries;
 *   n_unique:   host, count after redundancy removal;
 *   hole_flags: host, p-1 bytes (1 = no redundancy found between partitions
 *               j and j+1, i.e. a suspected hole), or NULL.
 * Errors: as tsg_solve_partition. */
tsg_status tsg_solve_all_partitions(tsg_ctx* ctx, const tsg_window* windows, int32_t p, const tsg_opts* opts,
                                    int32_t* n_unique, uint8_t* hole_flags);

/* Algorithm 1's repeat loop (Section 2.2) on the stored partitions after a
 * solve.  The partitions are reordered by shift (stable), so that interface
 * j lies between partitions j and j+1, and combined as by tsg_combine.
 * While a gap is left and fewer than max_rounds rounds have run, every gap
 * gets a new partition.  A gap is a flagged interface, between the largest
 * real part among the lower partition's eigenvalues and the smallest among
 * the upper one's, or the stretch from E_min (itself an eigenvalue) up to the
 * lowest computed real part when that lies more than Algorithm 2's tau
 * (1e-6 ||A||_G) above E_min.  The new partition sits at the middle of the
 * gap and holds ceil(3/2 gap / Delta) eigenpairs with
 * Delta = (E_max - E_min)/N, clamped to [1, n_cap] (a gap <= 0 gives 1); a
 * round's new partitions are solved together (one batched iteration), then
 * all partitions are reordered and combined again.  Partition indices of
 * tsg_get_partition and tsg_get_stats follow the new order.
 *   e_min:      E_min of the plan (e_range[0] of tsg_plan_windows); E_max is
 *               the bound tsg_plan_windows uses;
 *   n_cap:      largest count of an inserted partition (>= 1), for example
 *               the largest planned n_{r,j}: Delta is the mean spacing over
 *               the whole spectrum, and where eigenvalues are sparser than
 *               that the formula asks for more than one window should hold;
 *   max_rounds: >= 0;
 *   n_added, rounds, n_unique, holes_left: host outputs or NULL (partitions
 *               inserted, rounds run, combined count, gaps left after the
 *               last combine).
 * Errors: TSG_EINVAL, TSG_ESTATE (no partitions), TSG_ENOCONV (an inserted
 * partition did not converge; its converged subset is kept), TSG_EDEVICE. */
tsg_status tsg_fill_holes(tsg_ctx* ctx, double e_min, int32_t n_cap, int32_t max_rounds, const tsg_opts* opts,
                          int32_t* n_added, int32_t* rounds, int32_t* n_unique, int32_t* holes_left);

/* The windows of n_sys independent systems (one context each, same device
 * and fd_radius) in one batched iteration: every kernel launch covers all
 * windows of all systems, each window on its own grid (the partitions of
 * Section 2 are independent, so windows of different systems share the
 * device like windows of one system).  System s's partitions replace those
 * of ctx[s], which is then combined as by tsg_combine.
 *   ctx:      host, n_sys context pointers;
 *   windows:  host, n_sys pointers, windows[s] has p[s] entries;
 *   p:        host, n_sys counts (>= 1);
 *   n_unique: host, n_sys outputs (count after combine), or NULL.
 * The work runs on ctx[0]'s device; every context's stream is drained first.
 * Errors: TSG_EINVAL, TSG_ENOCONV (some window of some system did not
 * converge; converged subsets kept), TSG_ENOMEM, TSG_EDEVICE. */
tsg_status tsg_solve_batch(tsg_ctx* const* ctx, int32_t n_sys, const tsg_window* const* windows, const int32_t* p,
                           const tsg_opts* opts, int32_t* n_unique);

/* Algorithm 2 (Section 2.2) over the stored partitions in order: pairs
 * whose eigenvalues agree within 1e-6 ||A||_G are Gram-Schmidt
 * bi-orthogonalised under the unconjugated product; a pair whose vector
 * norm falls below 1e-3 of its value is removed and clears the hole flags of
 * the interfaces between the two partitions that hold it (windows sharing an
 * eigenvalue overlap, so no interface between them hides a gap).  The result is sorted by real
 * part and c-normalised (u^T u = 1); keep_lowest > 0 truncates it.
 *   hole_flags: host, (number of partitions - 1) bytes, or NULL.
 * Errors: TSG_ESTATE (no partitions), TSG_EDEVICE. */
tsg_status tsg_combine(tsg_ctx* ctx, int32_t keep_lowest, int32_t* n_unique, uint8_t* hole_flags);

/* Combined eigenvalues, ascending real part.
 *   re_im: host, capacity cap pairs (2*cap doubles).  *n gets the count.
 * Errors: TSG_ESTATE (no combined set), TSG_ECAPACITY. */
tsg_status tsg_get_eigenvalues(tsg_ctx* ctx, double* re_im, int32_t cap, int32_t* n);

/* Combined eigenvectors: borrowed device view, complex128, N x n with each
 * vector contiguous (element (n, c) at ptr[c * ld + n], *ld = N); valid
 * until the next solve, combine or tsg_destroy.  Each column satisfies
 * u^T u = 1.
 * Errors: TSG_ESTATE. */
tsg_status tsg_get_eigenvectors(tsg_ctx* ctx, void** dev_ptr, int64_t* ld, int32_t* n);

/* Eigenpairs of stored partition j (0-based), ascending real part; vectors
 * as in tsg_get_eigenvectors (borrowed, complex128, c-normalised).
 *   re_im: host, capacity cap pairs; dev_ptr, ld: may be NULL.
 * Errors: TSG_EINVAL (j out of range), TSG_ECAPACITY. */
tsg_status tsg_get_partition(tsg_ctx* ctx, int32_t j, double* re_im, int32_t cap, int32_t* n, void** dev_ptr,
                             int64_t* ld);

/* Statistics of stored partition j.  Errors: TSG_EINVAL. */
tsg_status tsg_get_stats(tsg_ctx* ctx, int32_t j, tsg_window_stats* stats);

/* Transmission (Section 1) T(E) = Tr{G Gamma_R G^dagger Gamma_L} with G
 * built from the combined eigenpairs, G(E) = sum_k u_k u_k^T / (E - eps_k):
 *   T(E) = sum_kl g_k conj(g_l) (U^T Gamma_R conj U)_kl (U^T Gamma_L conj U)_kl.
 *   E: host, nE energies; T: host, nE outputs.
 * Errors: TSG_EINVAL (nE < 1, null), TSG_ESTATE (no combined set). */
tsg_status tsg_transmission(tsg_ctx* ctx, const double* E, int32_t nE, double* T);

/* Vector-Jacobian product of the transmission: the gradient of
 * L = sum_e dL_dT[e] T(E[e]) (energies held fixed, T as in
 * tsg_transmission over the combined eigenpairs) with respect to the
 * potential V(r) and the absorber parameters.  The paper does not
 * differentiate T; this is the derivative of what the pipeline computes.
 * First-order perturbation of the c-normalised pairs (d eps_k = u_k^T dA u_k
 * with dA = diag(dV) - i diag(dGamma)) gives the part inside the computed
 * set from n x n products; the part outside it comes from the projected
 * solves (eps_k - A) x_k = (I - U U^T) z_k, all k at once by COCR on
 * P (eps_k - A) P with P = I - U U^T (complex symmetric since P^T = P).
 *   E, dL_dT: host, nE values;
 *   dL_dV:    host, N outputs (grid order as V);
 *   dL_dabs:  host, 4 outputs: d/d amp_L, width_L, amp_R, width_R
 *             (z_L, z_R held fixed).
 * Errors: TSG_EINVAL, TSG_ESTATE (no combined set), TSG_ENOCONV (the
 * projected solves missed their 1e-11 relative residual; outputs still
 * written), TSG_EDEVICE. */
tsg_status tsg_transmission_vjp(tsg_ctx* ctx, const double* E, int32_t nE, const double* dL_dT, double* dL_dV,
                                double* dL_dabs);

/* Y = A X for a block of ncols vectors (the stencil matrix-vector product of
 * Section 1, used by every iteration).  X, Y: device, ncols vectors of N
 * elements, vector c at ptr + c * ld (ld >= N), element type dtype
 * (TSG_C128 or TSG_C64); X and Y must not overlap.  Runs on the context
 * stream; returns without synchronising.  Errors: TSG_EINVAL. */
tsg_status tsg_apply_operator(tsg_ctx* ctx, const void* X, void* Y, int32_t ncols, int64_t ld, int32_t dtype);

/* Dense eigen-decomposition of `batch` general complex m x m matrices (the
 * small Rayleigh-Ritz problem inside each window iteration).  H: device,
 * batch row-major m x m complex128 matrices, 1 <= m <= 896, overwritten;
 * theta: device, batch*m complex128 eigenvalues; Y: device, batch row-major
 * m x m, unit 2-norm eigenvector columns; info: device, batch int32
 * (0 = converged).
 * hip_stream as in tsg_build_operator.  Errors: TSG_EINVAL (null pointer,
 * m or batch out of range; nothing launched), TSG_ENOMEM, TSG_EDEVICE. */
tsg_status tsg_dense_eig(void* H, int32_t m, int32_t batch, void* theta, void* Y, int32_t* info, void* hip_stream);

/* Autotuner of the stencil launch geometry (the matrix-vector product
 * formula of Section 1, applied to many vectors at once).  Every candidate
 * (256 or 512 threads per workgroup, tile width 16/32/64, one or two
 * points per thread in y, z chunk of 16..192 planes, workgroups in launch
 * order or grouped so that each of the eight XCDs runs a contiguous range of
 * neighbouring tiles, one or (complex64 only) two columns per thread) is timed on ctx's grid for a launch of ncols vectors of
 * element type dtype (reps launches each, HIP events on ctx's stream); the
 * fastest is recorded in the process-wide table that every later stencil
 * launch with the same grid shape, column count, element size and radius
 * uses.  Solver launches cover (windows x columns) vectors, which is the
 * count to tune for.
 *   path:     if not NULL, the whole table is written there as JSON
 *             ({"stencil": [{nx, ny, nz, cols, elem, radius, tx, yb, zchunk, xcd, nt, cb, us}, ...]};
 *             elem is the complex element size, 16 or 8 bytes; an entry
 *             without "xcd" reads as launch order, without "nt" as 512,
 *             without "cb" as one column per thread);
 *   geometry: host, 7 outputs or NULL: tx, yb, zchunk, xcd (0 or 1), nt,
 *             cb, candidates timed;
 *   best_us:  host, or NULL: the best time per launch in microseconds.
 * Allocates two N x ncols blocks while it runs and synchronises ctx's stream.
 * Errors: TSG_EINVAL (ncols, reps < 1, dtype, unwritable path), TSG_ENOMEM,
 * TSG_EDEVICE. */
tsg_status tsg_tune_stencil(tsg_ctx* ctx, int32_t ncols, int32_t dtype, int32_t reps, const char* path,
                            int32_t* geometry, double* best_us);

/* The stencil launch geometry the library uses for a launch of ncols vectors
 * (windows x columns for the solver) of element type dtype on an nx x ny x nz
 * grid with the given radius (1..6): the tuned entry when the process-wide
 * table holds one for exactly this key, else the built-in rule.  Host only:
 * needs no device and launches nothing.
 *   geometry: host, 7 outputs: tx, yb, zchunk, xcd, nt, cb, 1 if tuned else 0.
 * Errors: TSG_EINVAL (NULL geometry, sizes out of range, dtype). */
tsg_status tsg_stencil_geometry(int32_t nx, int32_t ny, int32_t nz, int32_t radius, int32_t ncols, int32_t dtype,
                                int32_t* geometry);

/* Loads a tuning file written by tsg_tune_stencil into the process-wide
 * table (entries with the same key are replaced).  *n_entries (or NULL) gets
 * the number read.  Errors: TSG_EINVAL (unreadable or malformed file). */
tsg_status tsg_load_tuning(const char* path, int32_t* n_entries);

/* tsg_dense_eig for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same arguments, kernels and results, but the workspace lives in a
 * fixed 64 MiB device array that each GPU holds from its first call until
 * the process ends, so the call allocates nothing.  It returns as soon as the
 * work is enqueued on hip_stream (no synchronisation); the outputs are
 * complete when that stream reaches this point.  Every call on one GPU shares
 * the array: calls that overlap on one GPU (other streams or threads) race.
 * Limit: batch * (2 m^2 + rotation log(m)) complex128 values must fit in the
 * 64 MiB (m = 450: 2 matrices; m = 300: 3; m = 128: 8; m = 64: 12).
 * Errors: TSG_EINVAL (null pointer, m out of range, or more than fits in the
 * scratch; nothing launched), TSG_EDEVICE. */
tsg_status tsg_dense_eig_noalloc(void* H, int32_t m, int32_t batch, void* theta, void* Y, int32_t* info,
                                 void* hip_stream);

/* Message for the last failed call on ctx (or for the last failed call
 * without a context when ctx is NULL).  Never NULL. */
const char* tsg_last_error(const tsg_ctx* ctx);

/* Releases the context and all its device memory.  NULL is ignored. */
void tsg_destroy(tsg_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* TRANSEC_GPU_H */
