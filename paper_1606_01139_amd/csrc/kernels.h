// Internal kernel launchers of libtransec_gpu.  Not part of the C-ABI.
#pragma once
#include <mutex>
#include <vector>

#include "tsg_common.h"

namespace tsg {

// Row count of each window's vectors: `per` (indexed by window) when the
// windows of one launch belong to systems of different size, else N.
struct Rows {
  int64_t N = 0;             // largest row count (sizes the launch)
  const int* per = nullptr;  // device, per window, or null
  __host__ __device__ int64_t of(int w) const { return per ? int64_t(per[w]) : N; }
};

// ---------------------------------------------------------------- K1
// One grid system: dimensions, its potential V (N values) and absorber
// profile Gamma_L + Gamma_R (nz values, one per z plane) in both
// precisions, and its finite-difference weights: diag0 = -3 c_0 / (2 h^2)
// and coef[m] = -c_m / (2 h^2).
struct SysDesc {
  int32_t nx, ny, nz, pad;
  const double* Vd;
  const float* Vf;
  const double* Gd;
  const float* Gf;
  double diag0;
  double coef[7];
};

template <typename T> struct StencilArgs {
  const cplx<T>* X; int64_t ldx, wsx;      // input: column j of window w at X + w*wsx + j*ldx
  cplx<T>* Y; int64_t ldy, wsy;            // output, same form
  int ncols;                               // columns per window
  int radius;
  const SysDesc* sys;                      // device table
  const int* wsys;                         // window -> system index, or null (system 0)
  const int* wmap;                         // launch slot -> window index (< 0: idle), or null
  int tx, ty, zchunk, tiles;               // launch geometry (tiles = largest tile count)
  int nt;                                  // threads per workgroup (256 or 512)
  int cb;                                  // columns per thread (1, or 2 for complex64)
  int yb;                                  // points per thread stacked in y (1 or 2)
  int xcd;                                 // 1: XCD-aware block order (one-dimensional, padded grid)
  int nzc;                                 // z chunks of the largest system (set at launch)
  int64_t nblocks;                         // logical blocks (set at launch)
};
template <typename T> void launch_stencil(StencilArgs<T> a, int nwin, int max_nz, hipStream_t s);
// Tile geometry for the largest system of a launch: the tuned one for this
// shape, launch width and element size when the table has it, else the
// default rule.
template <typename T> void stencil_geometry(StencilArgs<T>& a, int nx, int ny, int nz, int nwin);

// A stencil launch geometry: tile width tx (nt / tx thread rows, nt = 256 or
// 512 threads per workgroup), yb points per thread in y, zchunk planes per
// workgroup, xcd = 1 for the XCD-grouped block order, cb columns per thread.
struct StencilGeom {
  int tx = 64, yb = 1, zchunk = 32, xcd = 0, nt = 512, cb = 1;
};
// Whether the kernel supports g at this radius and complex element size
// (tile, block size, columns per thread and a halo that fits the per-thread
// slots).
bool stencil_geometry_valid(const StencilGeom& g, int radius, int elem);
StencilGeom stencil_default_geometry(int nx, int ny, int nz, int64_t launch_cols, int radius);
// The geometry a launch uses: the tuned entry for (shape, launch columns,
// complex element size in bytes, radius) if the table has one (*tuned set
// to true), else the default rule.
StencilGeom stencil_lookup(int nx, int ny, int nz, int64_t launch_cols, int elem, int radius, bool* tuned);
template <typename T>
void stencil_apply_geometry(StencilArgs<T>& a, int nx, int ny, int nz, const StencilGeom& gm);
// Tuned geometries (filled by the autotuner or read from a tuning file).
struct StencilTuneEntry {
  int nx, ny, nz, cols, elem, radius;
  StencilGeom g;
  double us;  // measured time per launch
};
// Process-wide; every member locks, so launches may read it while another
// thread loads or tunes.
struct StencilTuneTable {
  bool find(int nx, int ny, int nz, int64_t cols, int elem, int radius, StencilGeom& out) const {
    std::lock_guard<std::mutex> lock(mu);
    for (const auto& x : e)
      if (x.nx == nx && x.ny == ny && x.nz == nz && x.cols == cols && x.elem == elem && x.radius == radius) {
        out = x.g;
        return true;
      }
    return false;
  }
  void put(const StencilTuneEntry& v) {
    std::lock_guard<std::mutex> lock(mu);
    for (auto& x : e)
      if (x.nx == v.nx && x.ny == v.ny && x.nz == v.nz && x.cols == v.cols && x.elem == v.elem &&
          x.radius == v.radius) {
        x = v;
        return;
      }
    e.push_back(v);
  }
  std::vector<StencilTuneEntry> entries() const {
    std::lock_guard<std::mutex> lock(mu);
    return e;
  }

 private:
  mutable std::mutex mu;
  std::vector<StencilTuneEntry> e;
};
StencilTuneTable& stencil_tune_table();

// ---------------------------------------------------------------- dense
// Batched tall-skinny products over the grid index n < rows.of(w).  Grid
// vectors are contiguous: column j of window w's block is X + w*wsx + j*ldx.
// All small matrices are FP64 complex, row-major.

// C[w] (r x s, ldc) = X[w]^H Y[w], reduced deterministically.
// `partials` holds `cap` c128 entries (at least nwin * r * s); the number of
// row chunks is capped to fit.  gram_workspace() is a good size.
template <typename TX, typename TY>
void gram(const cplx<TX>* X, int64_t ldx, int64_t wsx, const cplx<TY>* Y, int64_t ldy, int64_t wsy, Rows rows,
          int r, int s, c128* C, int64_t ldc, int64_t wsc, int nwin, c128* partials, int64_t cap, hipStream_t st,
          const int* wmap = nullptr);
int64_t gram_workspace(int64_t N, int r, int s, int nwin);

// Y[w] (N x s) = beta * Y[w] + alpha * X[w] (N x r) * B[w] (r x s, ldb).  Y must not alias X.
template <typename T>
void gemm_cols(const cplx<T>* X, int64_t ldx, int64_t wsx, const c128* B, int64_t ldb, int64_t wsb, cplx<T>* Y,
               int64_t ldy, int64_t wsy, Rows rows, int r, int s, double beta, int nwin, hipStream_t st,
               const int* wmap = nullptr, double alpha = 1.0);

// Per-column sums over rows of |AU - theta U|^2 and |U|^2 (FP64 partials,
// reduced); out[w*s + j] = {res2, unorm2}.
template <typename T>
void residual_norms(const cplx<T>* U, int64_t ldu, int64_t wsu, const cplx<T>* AU, int64_t lda, int64_t wsa,
                    const c128* theta, int64_t wst, Rows rows, int s, int nwin, double* out, double* partials,
                    int64_t cap, hipStream_t st, const int* wmap = nullptr);
int64_t residual_workspace(int64_t N, int s, int nwin);

// F[:, q] = AU[:, sel[w*b+q]] - theta * U[:, sel[w*b+q]] (columns with a
// negative selection are left unchanged).
template <typename T>
void residual_block(const cplx<T>* U, const cplx<T>* AU, int64_t ld, int64_t ws, const c128* theta, int64_t wst,
                    const int* sel, int b, cplx<T>* F, int64_t ldf, int64_t wsf, Rows rows, int nwin, hipStream_t st,
                    const int* wmap = nullptr);

// c-products u^T A u and u^T u of each column (unconjugated), FP64.
template <typename T>
void cdots(const cplx<T>* U, int64_t ldu, int64_t wsu, const cplx<T>* AU, int64_t lda, int64_t wsa, Rows rows, int s,
           int nwin, c128* out, double* partials, int64_t cap, hipStream_t st, const int* wmap = nullptr);

// Counter-based start vectors: real values uniform in [-1, 1) from a
// 64-bit mix of (seed, window, row, column).
template <typename T>
void random_block(cplx<T>* X, int64_t ldx, int64_t wsx, Rows rows, int s, int nwin, uint64_t seed, hipStream_t st,
                  const int* wmap = nullptr);

// Y = X (columns), with precision conversion.
template <typename TX, typename TY>
void copy_block(const cplx<TX>* X, int64_t ldx, int64_t wsx, cplx<TY>* Y, int64_t ldy, int64_t wsy, Rows rows, int s,
                int nwin, hipStream_t st, const int* wmap = nullptr);

// Column scaling Y[:, j] *= scale[w*s + j] (complex FP64 factors).
template <typename T>
void scale_cols(cplx<T>* Y, int64_t ldy, int64_t wsy, const c128* scale, Rows rows, int s, int nwin, hipStream_t st,
                const int* wmap = nullptr);

// Squared 2-norms of the s columns of each window: out[w*s + j].
template <typename T>
void col_sqnorms(const cplx<T>* X, int64_t ldx, int64_t wsx, Rows rows, int s, int nwin, double* out, double* partials,
                 int64_t cap, hipStream_t st, const int* wmap = nullptr);
// wmap2[slot] = wmap[slot] where some column kept less than half its squared
// norm through a Gram-Schmidt pass (after < before / 2), else -1.
void dgks_select(const double* before, const double* after, int s, int nslot, const int* wmap, int* wmap2,
                 hipStream_t st);

// Lagged second Gram-Schmidt pass of a block step: from the (j + b) x 2b
// product G = [V_j P]^H [P W] (ld 2b, window stride wsg) forms the 2b x 2b
// matrix M with [P' W'] M = [final P, W' orthogonal to it] (see dense.hip);
// flags[w] = 1 on a Cholesky breakdown.  b <= kLagMax.
constexpr int kLagMax = 4;
void lagfix(const c128* G, int64_t wsg, int j, int b, c128* M, int64_t wsm, int* flags, int nwin, hipStream_t st,
            const int* wmap = nullptr);
// Y[w] (N x s contiguous columns) <- Y[w] M[w] (s x s, row-major), in place; s <= 2 kLagMax.
template <typename T>
void rowmix(cplx<T>* Y, int64_t ldy, int64_t wsy, const c128* M, int64_t wsm, Rows rows, int s, int nwin,
            hipStream_t st, const int* wmap = nullptr);

// Small per-window kernels on b x b Gram matrices (one workgroup per window):
// G = R^H R (Cholesky), writes Rinv (upper triangular) and flags[w] = 1 when
// a pivot falls below 1e-26 trace(G) or below abs_floor[w] (when given),
// else 0.
void cholesky_inv(const c128* G, int64_t wsg, int b, c128* Rinv, int64_t wsr, int* flags, int nwin, hipStream_t st,
                  const int* wmap = nullptr, const double* abs_floor = nullptr);
// For windows with flags[w] set: W (b contiguous columns) is replaced by a
// random block orthonormal to V[:, 0:J) and within itself, Rinv[w] is set to
// the identity and count[w] is incremented (breakdown of the block step).
template <typename T>
void reseed_block(const cplx<T>* V, int64_t ldv, int64_t wsv, int J, cplx<T>* W, int64_t ldw, int64_t wsw, int b,
                  Rows rows, const int* flags, int* count, c128* Rinv, int64_t wsr, uint64_t seed, int nwin,
                  hipStream_t st, const int* wmap = nullptr);

// ---------------------------------------------------------------- K4
// Eigen-decomposition of general complex m x m matrices, one workgroup per
// window for the sequential parts.  H (row-major, ld m) is overwritten; theta
// gets the eigenvalues and Y (row-major m x m) the unit-2-norm right
// eigenvectors (columns).  work must hold smalleig_workspace(m) c128 per
// window.  m is at most kMaxDenseBasis (a Hessenberg row must fit the
// registers of one wavefront, 14 values per lane).
constexpr int kMaxDenseBasis = 14 * 64;
void smalleig(c128* H, int64_t wsh, int m, c128* theta, int64_t wst, c128* Y, int64_t wsy, c128* work,
              int64_t wsw, int* info, int nwin, hipStream_t st, const int* wmap = nullptr);
int64_t smalleig_workspace(int m);
// Schur form of upper Hessenberg H (in place) with Schur vectors accumulated
// into Z (which holds the Hessenberg reduction's unitary on entry); log is
// scratch of schur_log_size(m) c128 per window (stride wsl).
void launch_schur(c128* H, int64_t wsh, int m, c128* Z, int64_t wsz, c128* log, int64_t wsl, c128* theta,
                  int64_t wst, int* info, int nwin, hipStream_t st, const int* wmap);
int64_t schur_log_size(int m);

// Selection by |theta - sigma| (sigma complex; ties: Re, then Im) and restart basis:
// out (m x (k + nev), row-major, ld = k + nev):
//   columns [0, k): orthonormal basis of the k selected eigenvectors,
//   columns [k, k + nev): the nev nearest eigenvectors (unit 2-norm).
// theta_sel[w*(nev)] gets their eigenvalues (nearest first).
void select_restart(const c128* theta, int64_t wst, const c128* Y, int64_t wsy, int m, const c128* sigma,
                    int mode, int k, int nev, c128* out, int64_t wso, c128* theta_sel, int64_t wss,
                    int nwin, hipStream_t st, const int* wmap = nullptr);

// Harmonic Ritz extraction (harmonic.hip): H[w] (m x m) += X G E^T with
// X = (H - sigma)^{-H} E, E the last b columns of the identity, G = F^H F
// (b x b, upper Cholesky factor inverse Rinv, same stride wsg); XG (m x b)
// gets X G Rinv, the basis combination to subtract from the pending block at
// the restart.  L (m x m) and X (m x b) per window are scratch.
void harmonic_update(c128* H, int64_t wsh, int m, int b, const c128* sigma, const c128* G, const c128* Rinv,
                     int64_t wsg, c128* L, int64_t wsl, c128* X, int64_t wsx, c128* XG, int nwin, hipStream_t st,
                     const int* wmap = nullptr);
// theta[w*wst + i] = y^H H y / y^H y for y = column off + i of Y (row-major
// m x ld), i < nev.
void rayleigh_quotients(const c128* H, int64_t wsh, int m, const c128* Y, int64_t wsy, int ld, int off, int nev,
                        c128* theta, int64_t wst, int nwin, hipStream_t st, const int* wmap = nullptr);

// ---------------------------------------------------------------- K7/K8
// Transmission: T[e] = Re sum_kl g_k conj(g_l) W_kl, g_k = 1/(E_e - eps_k).
void transmission_sweep(const c128* W, int n, const c128* eps, const double* E, int nE, double* T,
                        hipStream_t st);
// M^X = U^T diag(gamma_X) conj(U) for X = L, R and W = M^R o M^L (Hadamard).
// U is N x n with contiguous columns (ld >= N).
template <typename T>
void gamma_grams(const cplx<T>* U, int64_t ldu, int64_t N, int n, const double* gL, const double* gR,
                 int plane, c128* MR, c128* ML, c128* W, c128* partials, hipStream_t st);
int64_t gamma_gram_workspace(int64_t N, int n);

// Combine (Algorithm 2): v -= U[:, m] (U[:, m]^T v) for each partner m in
// order; out = {||v|| before, ||v|| after, Re v^T v, Im v^T v}.
void project_out(c128* v, const c128* U, int64_t ldu, const int* partners, int np, int64_t N, double* out,
                 hipStream_t st);
// dst[:, j] = scale[j] * (contiguous vector srcs[j]); dst column j at dst + j*ldd.
void gather_columns(c128* dst, int64_t ldd, const c128* const* srcs, const c128* scale, int n, int64_t N,
                    hipStream_t st);

// ---------------------------------------------------------------- adjoint
// Building blocks of the transmission adjoint (adjoint.hip).  U, Y, Z are
// N x n with contiguous columns (ld N); n x n matrices are row-major.
void adj_gmat(const c128* eps, int n, const double* E, int nE, c128* G, hipStream_t st);
void adj_kmats(const c128* G, int n, int nE, const double* w, const c128* MR, const c128* ML, c128* KRt, c128* KLt,
               hipStream_t st);
// In-set part of the adjoint: B = (P + P^T)/2 with
// P_jk = sum_e w_e g_j g_k sum_l conj(g_l) MR_jl ML_kl (P is scratch, n x n).
void adj_inset(const c128* G, int n, int nE, const double* w, const c128* MR, const c128* ML, c128* P, c128* B,
               hipStream_t st);
void adj_conj(const c128* X, c128* Y, int64_t total, hipStream_t st);
void adj_zcombine(const c128* YR, const c128* YL, const double* gR, const double* gL, int64_t N, int n,
                  int64_t plane, c128* Z, hipStream_t st);
void adj_rowdot(const c128* U, const c128* Y, int64_t N, int n, double scale, bool use_im, double* out,
                hipStream_t st);
int64_t adj_cocr_workspace(int64_t N, int n);
void adj_cocr_sums(const c128* R, const c128* S, const c128* P, int64_t N, int n, double* part, double* out,
                   hipStream_t st);
void adj_shift(const c128* R, c128* AR, const c128* eps, int64_t N, int n, hipStream_t st);
void adj_scalars(const double* sums, int n, int mode, c128* rho, c128* alpha, c128* beta, int* done,
                 hipStream_t st);
void adj_xr(c128* X, c128* R, const c128* P, const c128* MP, const c128* alpha, int64_t N, int n, hipStream_t st);
void adj_p(c128* P, c128* MP, const c128* R, const c128* MR, const c128* beta, int64_t N, int n, hipStream_t st);
void adj_add(c128* Y, const c128* X, int64_t total, hipStream_t st);
void adj_absorber(const double* dGL, const double* dGR, const double* prof, int64_t N, int nz, int64_t plane,
                  double* out, hipStream_t st);

}  // namespace tsg
