// Host engine: operator set-up, the batched per-window shift-without-invert
// iteration, the FP64 finish of each eigenpair, Algorithm 2 and T(E).
//
// The window iteration (Section 2.1 of Feldman & Zhou): for each partition j
// a restarted Krylov method is applied to A - E_{S,j} without inversion and
// the Ritz values of smallest magnitude of the shifted operator (nearest the
// shift) are kept ('SM').  Here every window of a solve advances together:
//   expansion    Y = A X on the newest block of every window (K1), then the
//                block is orthogonalised against its window's basis (two
//                passes of classical Gram-Schmidt, Cholesky-QR inside);
//   projection   H = V^H (A V)  (FP64 accumulation);
//   small eig    eigenpairs of H (K4), ordered by |theta - E_{S,j}|;
//   restart      keep the k nearest Ritz vectors (thick restart, the
//                Krylov-Schur form of ARPACK's implicit restart) and continue
//                from the component of A X_last orthogonal to the basis;
//   convergence  backward error of the n_{r,j} nearest Ritz pairs.
// In TSG_FP32_BULK mode the blocks are complex64 until the backward error
// reaches bulk_tol, then the kept basis is promoted to complex128 and the
// iteration continues in FP64 to tol.  Every converged pair is finished in
// FP64: a fresh matrix-vector product, the c-Rayleigh quotient u^T A u/u^T u
// and c-normalisation u^T u = 1 (the bi-orthogonality of Section 1).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <numeric>
#include <thread>

#include "engine.h"

namespace tsg {

namespace {

double fd_coef(int R, int m) {
  // c_m = 2 (-1)^(m+1) (R!)^2 / (m^2 (R-m)! (R+m)!)
  auto fact = [](int n) { double f = 1.0; for (int i = 2; i <= n; ++i) f *= i; return f; };
  const double fr = fact(R);
  const double v = 2.0 * fr * fr / (double(m) * m * fact(R - m) * fact(R + m));
  return (m % 2 == 1) ? v : -v;
}

void check(hipError_t e, const char* what) {
  if (e != hipSuccess) throw DeviceError(std::string(what) + ": " + hipGetErrorString(e));
}

int round_up(int x, int b) { return ((x + b - 1) / b) * b; }
int64_t round_up64(int64_t x, int64_t b) { return ((x + b - 1) / b) * b; }

// TSG_TRACE=1 in the environment prints one line per restart and window.
bool trace_on() {
  static const bool on = [] { const char* v = std::getenv("TSG_TRACE"); return v && v[0] == '1'; }();
  return on;
}
// TSG_PROGRESS=1 prints one summary line per restart cycle.
bool progress_on() {
  static const bool on = [] { const char* v = std::getenv("TSG_PROGRESS"); return v && v[0] == '1'; }();
  return on;
}
// Restart cycles are replayed from a captured hipGraph unless the options or
// TSG_NO_GRAPH=1 (or the K4 phase profiler) turn it off.
bool graphs_allowed() {
  static const bool ok = [] {
    const char* a = std::getenv("TSG_NO_GRAPH");
    const char* b = std::getenv("TSG_K4PROF");
    return !(a && a[0] == '1') && !(b && b[0] == '1');
  }();
  return ok;
}

// ------------------------------------------------------------------ systems
// The grid systems of one batched solve and the window -> system map.  A
// single system needs no device tables beyond its own descriptor.
struct Systems {
  std::vector<tsg_ctx*> ctx;
  std::vector<int> wsys_h;                 // per window
  DevArr<SysDesc> table_own;
  DevArr<int> wsys_own, rows_own;
  const SysDesc* table = nullptr;
  const int* wsys = nullptr;               // null: every window on system 0
  const int* rows = nullptr;               // null: every window has Nmax rows
  int64_t Nmax = 0, Nmin = 0, ldN = 0;
  int nx = 0, ny = 0, nz = 0, R = 6;
  hipStream_t st = nullptr;
  Rows rows_arg() const { return Rows{Nmax, rows}; }
  tsg_ctx* of(int w) const { return ctx[wsys_h.empty() ? 0 : wsys_h[w]]; }
};

void one_system(Systems& S, tsg_ctx* c, hipStream_t st) {
  S.ctx = {c};
  S.table = c->sysd.p;
  S.Nmax = S.Nmin = c->N;
  S.ldN = round_up64(c->N, 64);
  S.nx = c->nx; S.ny = c->ny; S.nz = c->nz; S.R = c->R;
  S.st = st;
}

void many_systems(Systems& S, const std::vector<tsg_ctx*>& ctx, const std::vector<int>& wsys, hipStream_t st) {
  S.ctx = ctx;
  S.wsys_h = wsys;
  S.st = st;
  std::vector<SysDesc> tab(ctx.size());
  S.Nmax = 0;
  S.Nmin = ctx[0]->N;
  S.R = ctx[0]->R;
  for (size_t s = 0; s < ctx.size(); ++s) {
    tab[s] = ctx[s]->sys;
    S.Nmax = std::max(S.Nmax, ctx[s]->N);
    S.Nmin = std::min(S.Nmin, ctx[s]->N);
    S.nx = std::max(S.nx, ctx[s]->nx); S.ny = std::max(S.ny, ctx[s]->ny); S.nz = std::max(S.nz, ctx[s]->nz);
    if (ctx[s]->R != S.R) throw InvalidArg("all systems of a batch must use the same fd_radius");
  }
  S.ldN = round_up64(S.Nmax, 64);
  std::vector<int> rows(wsys.size());
  for (size_t w = 0; w < wsys.size(); ++w) rows[w] = int(ctx[wsys[w]]->N);
  S.table_own.alloc(tab.size());
  S.wsys_own.alloc(wsys.size());
  S.rows_own.alloc(rows.size());
  check(hipMemcpyAsync(S.table_own.p, tab.data(), sizeof(SysDesc) * tab.size(), hipMemcpyHostToDevice, st), "sys");
  check(hipMemcpyAsync(S.wsys_own.p, wsys.data(), sizeof(int) * wsys.size(), hipMemcpyHostToDevice, st), "wsys");
  check(hipMemcpyAsync(S.rows_own.p, rows.data(), sizeof(int) * rows.size(), hipMemcpyHostToDevice, st), "rows");
  check(hipStreamSynchronize(st), "sync");
  S.table = S.table_own.p;
  S.wsys = S.wsys_own.p;
  S.rows = S.rows_own.p;
}

template <typename T>
void stencil(const Systems& S, const cplx<T>* X, int64_t ldx, int64_t wsx, cplx<T>* Y, int64_t ldy, int64_t wsy,
             int ncols, int nwin, const int* wmap) {
  StencilArgs<T> a;
  a.X = X; a.ldx = ldx; a.wsx = wsx;
  a.Y = Y; a.ldy = ldy; a.wsy = wsy;
  a.ncols = ncols;
  a.radius = S.R;
  a.sys = S.table;
  a.wsys = S.wsys;
  a.wmap = wmap;
  stencil_geometry<T>(a, S.nx, S.ny, S.nz, nwin);
  launch_stencil<T>(a, nwin, S.nz, S.st);
}

// Private non-blocking stream of one solve (graph capture needs a stream
// other than the null stream); the caller's stream is drained first.
struct SolveStream {
  hipStream_t s = nullptr;
  explicit SolveStream(hipStream_t user) {
    check(hipStreamSynchronize(user), "sync");
    check(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "hipStreamCreate");
  }
  ~SolveStream() {
    if (s) { (void)hipStreamSynchronize(s); (void)hipStreamDestroy(s); }
  }
};

// ------------------------------------------------------------------ batch
// Device state of one batched solve in storage precision T.  Window w's
// basis V (ldN x (m + b), contiguous columns) starts at V + w * ws(): the m
// basis columns, then the next block (the continuation of the cycle);
// likewise the rotation target Vr.  AV (ldN x m, window stride ldN m) holds
// A V for the Rayleigh-Ritz projection; AR (ldN x nev, window stride ws())
// holds A times the wanted Ritz vectors.  Ft is a b-column temporary.
template <typename T> struct Batch {
  int nw = 0, m = 0, k = 0, b = 0, nv = 0;
  int bw = 0;  // widest block orthonormalize handles (b, or the residual block of the FP64 polish)
  uint64_t seed = 0;
  bool harmonic = false;
  DevArr<c128> Hs, Lh, Xh, XG;  // harmonic extraction: saved H, LU and solution scratch, restart update
  int64_t ldN = 0;
  Rows rows;
  DevArr<cplx<T>> V, AV, Vr, AR, Ft;
  DevArr<c128> H, Ys, work, theta, Ysel, thsel, C, G, Rinv, Mx, part;
  DevArr<double> res, nb, na, bfloor;
  DevArr<c128> sig;
  DevArr<int> flags, info, wmap, wmap2, sel, nbreak;

  void alloc(int nw_, const Systems& S, int m_, int k_, int b_, int nv_, int bw_ = 0) {
    nw = nw_; ldN = S.ldN; rows = S.rows_arg(); m = m_; k = k_; b = b_; nv = nv_;
    bw = std::max(b, bw_);
    const int64_t N = S.Nmax;
    V.alloc(size_t(ws()) * nw); Vr.alloc(size_t(ws()) * nw);
    AV.alloc(size_t(ldN) * m * nw); AR.alloc(size_t(ws()) * nw);
    Ft.alloc(size_t(ldN) * bw * nw);
    H.alloc(size_t(m) * m * nw); Ys.alloc(size_t(m) * m * nw);
    work.alloc(size_t(smalleig_workspace(m)) * nw);
    theta.alloc(size_t(m) * nw);
    Ysel.alloc(size_t(m) * (k + nv) * nw);
    thsel.alloc(size_t(nv) * nw);
    C.alloc(size_t(wsc()) * nw);
    G.alloc(size_t(bw) * bw * nw);
    Rinv.alloc(size_t(bw) * bw * nw);
    Mx.alloc(size_t(4) * b * b * nw);
    int64_t pw = gram_workspace(N, m, m, nw);
    pw = std::max(pw, gram_workspace(N, m + b, 2 * b, nw));
    pw = std::max(pw, gram_workspace(N, bw, bw, nw));
    pw = std::max(pw, gram_workspace(N, m, bw, nw));
    pw = std::max(pw, residual_workspace(N, nv, nw));
    part.alloc(size_t(pw));
    res.alloc(size_t(2) * nv * nw);
    sig.alloc(size_t(nw));
    flags.alloc(size_t(nw)); info.alloc(size_t(nw)); wmap.alloc(size_t(nw)); sel.alloc(size_t(nw) * bw);
    wmap2.alloc(size_t(nw)); nb.alloc(size_t(nw) * bw); na.alloc(size_t(nw) * bw);
    bfloor.alloc(size_t(nw)); nbreak.alloc(size_t(nw));
  }
  void alloc_harmonic() {
    harmonic = true;
    Hs.alloc(size_t(m) * m * nw); Lh.alloc(size_t(m) * m * nw); Xh.alloc(size_t(m) * b * nw);
    XG.alloc(size_t(m) * b * nw);
  }
  int64_t ws() const { return ldN * (m + b); }
  int64_t wsc() const { return int64_t(m + b) * std::max(2 * b, bw); }
};

// dest (ldN x b per window, column stride ldd, window stride wsd) is made
// orthonormal against the first J basis columns (CGS2) and within itself
// (Cholesky-QR, twice).
template <typename T>
void orthonormalize(const Systems& S, Batch<T>& B, cplx<T>* dest, int64_t ldd, int64_t wsd, int J, int width = 0) {
  const int b = width > 0 ? width : B.b, nw = B.nw;
  if (b > B.bw) throw DeviceError("orthonormalize: block wider than the batch's buffers");
  const int* wm = B.wmap.p;
  hipStream_t st = S.st;
  const int64_t ldN = B.ldN;
  // classical Gram-Schmidt; the second pass runs only for windows whose
  // block lost more than half of a column's squared norm in the first
  if (J > 0) {
    double* cpart = reinterpret_cast<double*>(B.part.p);
    const int64_t ccap = 2 * int64_t(B.part.n);
    col_sqnorms<T>(dest, ldd, wsd, B.rows, b, nw, B.nb.p, cpart, ccap, st, wm);
    for (int pass = 0; pass < 2; ++pass) {
      const int* wp = pass == 0 ? wm : B.wmap2.p;
      gram<T, T>(B.V.p, ldN, B.ws(), dest, ldd, wsd, B.rows, J, b, B.C.p, b, B.wsc(), nw, B.part.p,
                 int64_t(B.part.n), st, wp);
      gemm_cols<T>(B.V.p, ldN, B.ws(), B.C.p, b, B.wsc(), dest, ldd, wsd, B.rows, J, b, 1.0, nw, st, wp, -1.0);
      if (pass == 0) {
        col_sqnorms<T>(dest, ldd, wsd, B.rows, b, nw, B.na.p, cpart, ccap, st, wm);
        dgks_select(B.nb.p, B.na.p, b, nw, wm, B.wmap2.p, st);
      }
    }
  }
  for (int pass = 0; pass < 2; ++pass) {
    cplx<T>* src = pass == 0 ? dest : B.Ft.p;
    int64_t lds = pass == 0 ? ldd : ldN, wss = pass == 0 ? wsd : ldN * b;
    cplx<T>* dst = pass == 0 ? B.Ft.p : dest;
    int64_t ldo = pass == 0 ? ldN : ldd, wso = pass == 0 ? ldN * b : wsd;
    gram<T, T>(src, lds, wss, src, lds, wss, B.rows, b, b, B.G.p, b, int64_t(b) * b, nw, B.part.p,
               int64_t(B.part.n), st, wm);
    cholesky_inv(B.G.p, int64_t(b) * b, b, B.Rinv.p, int64_t(b) * b, B.flags.p, nw, st, wm);
    gemm_cols<T>(src, lds, wss, B.Rinv.p, b, int64_t(b) * b, dst, ldo, wso, B.rows, b, b, 0.0, nw, st, wm, 1.0);
  }
}

// One block step of the expansion with the second Gram-Schmidt pass lagged
// by one step (two sweeps over the basis instead of four).  On entry the
// columns [0, j) of V are final and P = V[:, j:j+b] is pending: orthogonal to
// them after one pass and orthonormal within itself.  The step computes
// W = A P into V[:, j+b:j+2b]; one Gram pass gives [V_j P]^H [P W]; one update
// pass applies P' = P - V_j S (the second pass for P) and W' = W - V_j C; a
// b-column mix makes P' orthonormal (final) and W' orthogonal to it; W' is
// then normalised (Cholesky-QR) and becomes the pending block.  W is taken
// from the pending P: the terms A V_j S it carries lie in the span of the
// basis and are projected out with the rest.
template <typename T>
void expand_step(const Systems& S, Batch<T>& B, int j) {
  const int b = B.b, nw = B.nw;
  const int* wm = B.wmap.p;
  hipStream_t st = S.st;
  const int64_t ldN = B.ldN, wsV = B.ws();
  cplx<T>* P = B.V.p + j * ldN;
  cplx<T>* W = B.V.p + (j + b) * ldN;
  stencil<T>(S, P, ldN, wsV, W, ldN, wsV, b, nw, wm);
  gram<T, T>(B.V.p, ldN, wsV, P, ldN, wsV, B.rows, j + b, 2 * b, B.C.p, 2 * b, B.wsc(), nw, B.part.p,
             int64_t(B.part.n), st, wm);
  lagfix(B.C.p, B.wsc(), j, b, B.Mx.p, int64_t(4) * b * b, B.flags.p, nw, st, wm);
  if (j > 0)
    gemm_cols<T>(B.V.p, ldN, wsV, B.C.p, 2 * b, B.wsc(), P, ldN, wsV, B.rows, j, 2 * b, 1.0, nw, st, wm, -1.0);
  rowmix<T>(P, ldN, wsV, B.Mx.p, int64_t(4) * b * b, B.rows, 2 * b, nw, st, wm);
  gram<T, T>(W, ldN, wsV, W, ldN, wsV, B.rows, b, b, B.G.p, b, int64_t(b) * b, nw, B.part.p, int64_t(B.part.n), st,
             wm);
  // a pivot below the floor (a fixed fraction of ||A||) means A P lies in
  // the span of the basis: that window's block is replaced by a fresh random
  // block orthonormal to the basis (breakdown of the Krylov sequence)
  cholesky_inv(B.G.p, int64_t(b) * b, b, B.Rinv.p, int64_t(b) * b, B.flags.p, nw, st, wm, B.bfloor.p);
  reseed_block<T>(B.V.p, ldN, wsV, j + b, W, ldN, wsV, b, B.rows, B.flags.p, B.nbreak.p, B.Rinv.p, int64_t(b) * b,
                  B.seed ^ 0x6A09E667F3BCC908ull, nw, st, wm);
  rowmix<T>(W, ldN, wsV, B.Rinv.p, int64_t(b) * b, B.rows, b, nw, st, wm);
}

struct WinOut {
  bool done = false;
  bool converged = false;
  int restarts = 0;
  int breakdowns = 0;       // block steps whose new block lost rank and was replaced
  int64_t matvecs = 0;
  std::vector<c128> theta;   // selection order
  std::vector<double> rho;
};

// A captured restart cycle, one per assignment of the two basis buffers.
struct CycleGraphs {
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  ~CycleGraphs() {
    for (auto& e : exec)
      if (e) (void)hipGraphExecDestroy(e);
  }
};

// Runs the batched iteration on windows of one precision.  Every launch
// covers all nw window slots; slots of finished windows hold -1 in wmap and
// their workgroups exit at once, so one captured cycle stays valid as
// windows converge.  init_from: nullptr = random start; otherwise
// per-window [V_k | F] blocks (ldN x (k+b), complex64) from a complex64
// phase.  On convergence of window w, `save` receives the current device
// state.
template <typename T, typename Save>
void iterate(const Systems& S, Batch<T>& B, const std::vector<WindowSpec>& wins, const std::vector<double>& normA,
             int mode, double tol, int max_restarts, uint64_t seed, const cplx<float>* init_from,
             std::vector<WinOut>& out, Save&& save, bool use_graphs, double stall_floor = 0.0,
             bool davidson = false) {
  const int nw = B.nw, m = B.m, k = B.k, b = B.b, nv = B.nv;
  const int64_t ldN = B.ldN, wsV = B.ws();
  hipStream_t st = S.st;
  std::vector<int> active(nw);
  std::iota(active.begin(), active.end(), 0);
  std::vector<int> slots(nw);
  auto upload_slots = [&]() {
    for (int q = 0; q < nw; ++q) slots[q] = q < int(active.size()) ? active[q] : -1;
    check(hipMemcpyAsync(B.wmap.p, slots.data(), sizeof(int) * nw, hipMemcpyHostToDevice, st), "wmap");
  };
  upload_slots();
  std::vector<c128> shifts(nw);
  for (int w = 0; w < nw; ++w) shifts[w] = c128{wins[w].shift, wins[w].shift_im};
  check(hipMemcpyAsync(B.sig.p, shifts.data(), sizeof(c128) * nw, hipMemcpyHostToDevice, st), "shifts");
  // breakdown floor on the squared norm of a new block column after
  // orthogonalisation: (eta ||A||)^2, eta well above the rounding level of
  // the storage precision
  const double eta = sizeof(T) == 4 ? 1e-6 : 1e-12;
  std::vector<double> floors(nw);
  for (int w = 0; w < nw; ++w) floors[w] = (eta * normA[w]) * (eta * normA[w]);
  check(hipMemcpyAsync(B.bfloor.p, floors.data(), sizeof(double) * nw, hipMemcpyHostToDevice, st), "floors");
  check(hipMemsetAsync(B.nbreak.p, 0, sizeof(int) * nw, st), "nbreak");
  B.seed = seed;
  std::vector<int> hbreak(nw, 0);
  out.assign(nw, WinOut{});
  const int* wm = B.wmap.p;
  const Rows rows = B.rows;
  int j0 = 0;
  if (!init_from) {
    random_block<T>(B.V.p, ldN, wsV, rows, b, nw, seed, st, wm);
    orthonormalize<T>(S, B, B.V.p, ldN, wsV, 0);
  } else {
    // promote the complex64 kept basis and continuation block and
    // re-orthonormalise them block by block in this precision
    copy_block<float, T>(init_from, ldN, ldN * (k + b), B.V.p, ldN, wsV, rows, k + b, nw, st, wm);
    for (int j = 0; j <= k; j += b) orthonormalize<T>(S, B, B.V.p + j * ldN, ldN, wsV, j);
    j0 = k;
  }
  // expansion from column j0, projection, small eigenproblem, selection,
  // rotation and residual norms; with `cont`, first the continuation block
  // left pending after the previous cycle's last step (in Davidson mode the
  // residual block of the wanted Ritz pairs instead, orthonormalised)
  // residual block width of the FP64 polish: the b worst pairs (measured on
  // c2: feeding all nev residuals each cycle stalls near 1e-6, as the
  // residual directions crowd out the Krylov steps)
  const int dw = b;
  if (dw > B.bw) throw DeviceError("iterate: residual block wider than the batch's buffers");
  auto body = [&](int jstart, bool cont) {
    if (cont) {
      if (davidson) {
        // the residuals of dw wanted pairs (all of them when they fit),
        // orthonormalised, continue the basis; the Krylov steps then extend
        // it from the last b of them
        residual_block<T>(B.V.p + k * ldN, B.AR.p, ldN, wsV, B.thsel.p, nv, B.sel.p, dw, B.Ft.p, ldN, ldN * dw, rows,
                          nw, st, wm);
        copy_block<T, T>(B.Ft.p, ldN, ldN * dw, B.V.p + k * ldN, ldN, wsV, rows, dw, nw, st, wm);
        orthonormalize<T>(S, B, B.V.p + k * ldN, ldN, wsV, k, dw);
      } else {
        copy_block<T, T>(B.Vr.p + m * ldN, ldN, wsV, B.V.p + k * ldN, ldN, wsV, rows, b, nw, st, wm);
        if (B.harmonic) {
          // harmonic vectors have their residuals along F - V X G: continue
          // from that block (the old basis is still intact in Vr)
          gemm_cols<T>(B.Vr.p, ldN, wsV, B.XG.p, b, int64_t(m) * b, B.V.p + k * ldN, ldN, wsV, rows, m, b, 1.0, nw,
                       st, wm, -1.0);
          orthonormalize<T>(S, B, B.V.p + k * ldN, ldN, wsV, k);
        }
      }
    }
    // in Davidson mode the first dw - b columns after the kept ones are final
    const int jfirst = (cont && davidson) ? jstart + dw - b : jstart;
    for (int j = jfirst; j < m; j += b) expand_step<T>(S, B, j);
    // Rayleigh-Ritz on the final basis: A V afresh, then H = V^H A V
    stencil<T>(S, B.V.p, ldN, wsV, B.AV.p, ldN, ldN * m, m, nw, wm);
    gram<T, T>(B.V.p, ldN, wsV, B.AV.p, ldN, ldN * m, rows, m, m, B.H.p, m, int64_t(m) * m, nw, B.part.p,
               int64_t(B.part.n), st, wm);
    if (B.harmonic) {
      // harmonic Ritz pairs: eigenpairs of H + (H - sigma)^{-H} E (F^H F) E^T,
      // F^H F being the Gram of the block the last step left pending
      check(hipMemcpyAsync(B.Hs.p, B.H.p, sizeof(c128) * size_t(m) * m * nw, hipMemcpyDeviceToDevice, st), "Hs");
      harmonic_update(B.H.p, int64_t(m) * m, m, b, B.sig.p, B.G.p, B.Rinv.p, int64_t(b) * b, B.Lh.p, int64_t(m) * m,
                      B.Xh.p, int64_t(m) * b, B.XG.p, nw, st, wm);
    }
    smalleig(B.H.p, int64_t(m) * m, m, B.theta.p, m, B.Ys.p, int64_t(m) * m, B.work.p, smalleig_workspace(m),
             B.info.p, nw, st, wm);
    select_restart(B.theta.p, m, B.Ys.p, int64_t(m) * m, m, B.sig.p, mode, k, nv, B.Ysel.p, int64_t(m) * (k + nv),
                   B.thsel.p, nv, nw, st, wm);
    if (B.harmonic)  // eigenvalue estimates of the wanted harmonic vectors
      rayleigh_quotients(B.Hs.p, int64_t(m) * m, m, B.Ysel.p, int64_t(m) * (k + nv), k + nv, k, nv, B.thsel.p, nv, nw,
                         st, wm);
    // rotation [V Q_k | V Y_nev], then A times the wanted Ritz vectors
    gemm_cols<T>(B.V.p, ldN, wsV, B.Ysel.p, k + nv, int64_t(m) * (k + nv), B.Vr.p, ldN, wsV, rows, m, k + nv, 0.0,
                 nw, st, wm);
    stencil<T>(S, B.Vr.p + k * ldN, ldN, wsV, B.AR.p, ldN, wsV, nv, nw, wm);
    residual_norms<T>(B.Vr.p + k * ldN, ldN, wsV, B.AR.p, ldN, wsV, B.thsel.p, nv, rows, nv, nw, B.res.p,
                      reinterpret_cast<double*>(B.part.p), 2 * int64_t(B.part.n), st, wm);
  };
  CycleGraphs graphs;
  cplx<T>* const buf0 = B.V.p;
  // complex64 phase: a window whose worst wanted backward error stops
  // improving (no 5% gain in 8 restarts) below stall_floor is handed on, as
  // complex64 storage bounds the attainable residual
  std::vector<double> best(nw, 1e300);
  std::vector<int> since(nw, 0);
  std::vector<double> hres(size_t(2) * nv * nw);
  std::vector<c128> hth(size_t(nv) * nw);
  std::vector<int> hinfo(nw);
  for (int cyc = 0; cyc < max_restarts && !active.empty(); ++cyc) {
    const bool steady = cyc > 0;
    if (steady && use_graphs) {
      const int par = B.V.p == buf0 ? 0 : 1;
      if (!graphs.exec[par]) {
        hipGraph_t g = nullptr;
        check(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal), "capture");
        body(k, true);
        check(hipStreamEndCapture(st, &g), "capture");
        const hipError_t e = hipGraphInstantiate(&graphs.exec[par], g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        check(e, "hipGraphInstantiate");
      }
      check(hipGraphLaunch(graphs.exec[par], st), "hipGraphLaunch");
    } else {
      body(steady ? k : j0, steady);
    }
    for (int w : active) out[w].matvecs += (m - (steady ? k : j0)) + m + nv;
    check(hipMemcpyAsync(hres.data(), B.res.p, sizeof(double) * 2 * nv * nw, hipMemcpyDeviceToHost, st), "res");
    check(hipMemcpyAsync(hth.data(), B.thsel.p, sizeof(c128) * nv * nw, hipMemcpyDeviceToHost, st), "theta");
    check(hipMemcpyAsync(hinfo.data(), B.info.p, sizeof(int) * nw, hipMemcpyDeviceToHost, st), "info");
    check(hipMemcpyAsync(hbreak.data(), B.nbreak.p, sizeof(int) * nw, hipMemcpyDeviceToHost, st), "nbreak");
    check(hipStreamSynchronize(st), "sync");
    std::swap(B.V, B.Vr);
    std::vector<int> still;
    for (int w : active) {
      WinOut& o = out[w];
      o.restarts = cyc + 1;
      if (hbreak[w] > o.breakdowns && trace_on())
        std::fprintf(stderr, "[tsg] cycle %d window %d: %d block breakdown(s), fresh random block(s)\n", cyc, w,
                     hbreak[w] - o.breakdowns);
      o.breakdowns = hbreak[w];
      const int nev = wins[w].nev;
      o.theta.assign(hth.begin() + size_t(w) * nv, hth.begin() + size_t(w) * nv + nev);
      o.rho.resize(nev);
      int nconv = 0;
      for (int i = 0; i < nev; ++i) {
        const double r2 = hres[(size_t(w) * nv + i) * 2], u2 = hres[(size_t(w) * nv + i) * 2 + 1];
        const double rho = std::sqrt(std::max(r2, 0.0)) / (normA[w] * std::sqrt(std::max(u2, 1e-300)));
        o.rho[i] = std::isfinite(rho) ? rho : 1e300;
        nconv += (o.rho[i] <= tol) ? 1 : 0;
      }
      const double worst = *std::max_element(o.rho.begin(), o.rho.end());
      if (trace_on())
        std::fprintf(stderr, "[tsg] %s cycle %d window %d nconv %d/%d worst %.3e info %d\n",
                     sizeof(T) == 4 ? "c64" : "c128", cyc, w, nconv, nev, worst, hinfo[w]);
      if (worst < 0.95 * best[w]) { best[w] = worst; since[w] = 0; } else { ++since[w]; }
      const bool stalled = stall_floor > 0.0 && since[w] >= 8 && worst <= stall_floor;
      if (nconv == nev || stalled) {
        o.done = true;
        o.converged = true;
        save(w);
      } else if (cyc + 1 == max_restarts) {
        o.done = true;
        o.converged = false;
        save(w);
      } else {
        still.push_back(w);
      }
    }
    if (progress_on()) {
      double worst_all = 0.0;
      for (int w : active) worst_all = std::max(worst_all, out[w].rho.empty() ? 0.0 : *std::max_element(
                                                                out[w].rho.begin(), out[w].rho.end()));
      std::fprintf(stderr, "[tsg] %s cycle %d active %zu of %d, worst backward error %.2e\n",
                   sizeof(T) == 4 ? "c64" : "c128", cyc, still.size(), nw, worst_all);
    }
    if (still.size() != active.size()) {
      active = still;
      upload_slots();
    }
    if (active.empty()) break;
    if (davidson) {
      // after a precision change the kept basis has a residual of full rank,
      // so the next block is built from the explicit residuals of the b
      // wanted Ritz pairs with the largest backward error
      // the dw pairs with the largest backward errors, ordered so that the
      // worst come last: the Krylov steps continue from the last b columns
      std::vector<int> hsel(size_t(nw) * dw, -1);
      for (int w : active) {
        std::vector<int> ord(wins[w].nev);
        std::iota(ord.begin(), ord.end(), 0);
        std::sort(ord.begin(), ord.end(), [&](int a, int c2) { return out[w].rho[a] > out[w].rho[c2]; });
        const int nsel = std::min(dw, int(ord.size()));
        for (int q = 0; q < nsel; ++q) hsel[size_t(w) * dw + (dw - 1 - q)] = ord[q];
      }
      check(hipMemcpyAsync(B.sel.p, hsel.data(), sizeof(int) * hsel.size(), hipMemcpyHostToDevice, st), "sel");
      check(hipStreamSynchronize(st), "sync");  // hsel is a host temporary
    }
  }
}

void choose_sizes(int64_t N, int nvmax, const tsg_opts& o, int& m, int& k, int& b) {
  b = o.block > 0 ? o.block : 2;
  // automatic: about 9 nev (fewer, costlier restarts pay off: on c2,
  // 8 x 50 pairs, 38.8 s at m = 420..500 against 42.7 s at m = 300 and
  // 46.7 s at m = 600), and at least 40 so that a window of few pairs (hole
  // filling inserts such) still has room for the Ritz values crowding its
  // shift
  m = o.basis > 0 ? round_up(o.basis, b) : round_up(std::max({9 * nvmax, nvmax + 4 * b, 40}), b);
  const int mcap = int(std::min<int64_t>(N / b, 4096) * b) - b;
  if (m > mcap) m = std::max(mcap, 2 * b);
  k = o.keep > 0 ? (o.keep / b) * b : ((m / 2) / b) * b;
  if (k < round_up(nvmax, b)) k = round_up(nvmax, b);
  if (k + b > m) throw InvalidArg("basis too small for the requested eigenpairs (need keep + block <= basis)");
  if (k + nvmax > m) throw InvalidArg("basis too small: keep + nev must not exceed basis");
  // the restart basis is orthonormalised in LDS: (k + m) * 8 complex values
  if (int64_t(k + m) * 8 * 16 + int64_t(m) * 4 > 150 * 1024)
    throw InvalidArg("basis too large: keep + basis must stay below about 1200");
}

// FP64 finish of one window's nev vectors (device c128, N x nev, ld N):
// fresh A u, c-Rayleigh quotient, backward error, c-normalisation, sort by
// real part.  Returns the partition, which keeps only the pairs whose
// backward error is at most tol (all of them when the iteration converged).
Partition finish_window(tsg_ctx* c, hipStream_t st, const WindowSpec& ws, DevArr<c128>&& U, int nev,
                        const WinOut& o, int restarts_bulk, int breakdowns_bulk, double tol) {
  const int64_t N = c->N;
  Systems S;
  one_system(S, c, st);
  DevArr<c128> AU, dots, part;
  DevArr<double> res;
  AU.alloc(size_t(N) * nev);
  stencil<double>(S, U.p, N, 0, AU.p, N, 0, nev, 1, nullptr);
  dots.alloc(size_t(nev) * 2);
  part.alloc(size_t(std::max(residual_workspace(N, nev, 1), int64_t(1))) * 2);
  const Rows rows{N, nullptr};
  cdots<double>(U.p, N, 0, AU.p, N, 0, rows, nev, 1, dots.p, reinterpret_cast<double*>(part.p), 2 * int64_t(part.n),
                st);
  std::vector<c128> hd(size_t(nev) * 2);
  check(hipMemcpyAsync(hd.data(), dots.p, sizeof(c128) * 2 * nev, hipMemcpyDeviceToHost, st), "dots");
  check(hipStreamSynchronize(st), "sync");
  std::vector<c128> thc(nev), sc(nev);
  for (int i = 0; i < nev; ++i) {
    const c128 uAu = hd[2 * i], uu = hd[2 * i + 1];
    thc[i] = cdiv(uAu, uu);
    const c128 r = csqrt(uu);
    sc[i] = cdiv(c128{1.0, 0.0}, r);
  }
  DevArr<c128> thd;
  thd.alloc(nev);
  check(hipMemcpyAsync(thd.p, thc.data(), sizeof(c128) * nev, hipMemcpyHostToDevice, st), "thc");
  res.alloc(size_t(2) * nev);
  residual_norms<double>(U.p, N, 0, AU.p, N, 0, thd.p, 0, rows, nev, 1, res.p, reinterpret_cast<double*>(part.p),
                         2 * int64_t(part.n), st);
  std::vector<double> hr(size_t(2) * nev);
  check(hipMemcpyAsync(hr.data(), res.p, sizeof(double) * 2 * nev, hipMemcpyDeviceToHost, st), "res");
  check(hipStreamSynchronize(st), "sync");
  // sort by real part (then imaginary part)
  std::vector<int> ord(nev);
  std::iota(ord.begin(), ord.end(), 0);
  std::sort(ord.begin(), ord.end(), [&](int a, int b) {
    if (thc[a].re != thc[b].re) return thc[a].re < thc[b].re;
    return thc[a].im < thc[b].im;
  });
  Partition P;
  P.shift = ws.shift;
  P.shift_im = ws.shift_im;
  P.nev = ws.nev;
  double maxrho = 0.0;
  std::vector<double> rho(nev);
  for (int i = 0; i < nev; ++i) {
    const double r = std::sqrt(std::max(hr[2 * i], 0.0)) / (c->normA * std::sqrt(std::max(hr[2 * i + 1], 1e-300)));
    rho[i] = std::isfinite(r) ? r : 1e300;
    maxrho = std::max(maxrho, rho[i]);
  }
  // gather the kept pairs as sorted, c-normalised columns; a converged
  // vector whose u^T u vanishes cannot be c-normalised and is dropped
  std::vector<const c128*> srcs;
  std::vector<c128> scs;
  int cfail = 0;
  for (int i = 0; i < nev; ++i) {
    if (!(rho[ord[i]] <= tol)) continue;
    const c128 uu = hd[2 * ord[i] + 1];
    if (!(cabs(uu) >= 1e-10 * hr[2 * ord[i] + 1])) { ++cfail; continue; }
    srcs.push_back(U.p + int64_t(ord[i]) * N);
    scs.push_back(sc[ord[i]]);
    P.eps.push_back(thc[ord[i]]);
  }
  const int nk = int(srcs.size());
  P.U.alloc(size_t(N) * std::max(nk, 1));
  if (nk > 0) {
    DevArr<const c128*> dsrc;
    DevArr<c128> dsc;
    dsrc.alloc(nk); dsc.alloc(nk);
    check(hipMemcpyAsync(dsrc.p, srcs.data(), sizeof(void*) * nk, hipMemcpyHostToDevice, st), "srcs");
    check(hipMemcpyAsync(dsc.p, scs.data(), sizeof(c128) * nk, hipMemcpyHostToDevice, st), "sc");
    gather_columns(P.U.p, N, dsrc.p, dsc.p, nk, N, st);
    check(hipStreamSynchronize(st), "sync");
  }
  P.stats.shift = ws.shift;
  P.stats.shift_im = ws.shift_im;
  P.stats.nev = ws.nev;
  P.stats.n_conv = nk;
  P.stats.restarts = o.restarts;
  P.stats.matvecs = o.matvecs + nev;
  P.stats.max_backward_error = maxrho;
  P.stats.restarts_bulk = restarts_bulk;
  P.stats.breakdowns = o.breakdowns + breakdowns_bulk;
  P.stats.cnorm_failures = cfail;
  return P;
}

// Solves the windows (window w on system S.of(w)); returns the partitions in
// window order and per-window convergence.
void solve_group(Systems& S, const std::vector<WindowSpec>& wins, const tsg_opts& o, std::vector<Partition>& parts,
                 std::vector<bool>& conv) {
  const int nw = int(wins.size());
  if (nw < 1) throw InvalidArg("need at least one window");
  int nvmax = 0;
  for (const auto& w : wins) {
    if (w.nev < 1) throw InvalidArg("nev must be >= 1");
    if (!std::isfinite(w.shift) || !std::isfinite(w.shift_im)) throw InvalidArg("shift must be finite");
    nvmax = std::max(nvmax, w.nev);
  }
  if (!(o.tol > 0.0) || !std::isfinite(o.tol)) throw InvalidArg("tol must be positive");
  if (o.max_restarts < 1) throw InvalidArg("max_restarts must be >= 1");
  if (o.precision != TSG_FP64 && o.precision != TSG_FP32_BULK) throw InvalidArg("unknown precision");
  if (o.select < 0 || o.select > 2) throw InvalidArg("unknown selection");
  if (o.extraction != TSG_EXTRACT_RITZ && o.extraction != TSG_EXTRACT_HARMONIC)
    throw InvalidArg("unknown extraction");
  if (o.extraction == TSG_EXTRACT_HARMONIC && o.select != TSG_SELECT_NEAREST)
    throw InvalidArg("harmonic extraction targets the shift: it needs TSG_SELECT_NEAREST");
  const bool harmonic = o.extraction == TSG_EXTRACT_HARMONIC;
  int m, k, b;
  choose_sizes(S.Nmin, nvmax, o, m, k, b);
  if (int64_t(m) >= S.Nmin) throw InvalidArg("grid too small for the basis size");
  const int64_t ldN = S.ldN;
  hipStream_t st = S.st;
  const bool use_graphs = o.graphs != 0 && graphs_allowed();
  // the iteration aims a little below tol: the FP64 finish (fresh matvec,
  // c-Rayleigh quotient) must still report every pair at or below tol
  const double itol = 0.7 * o.tol;
  std::vector<double> normA(nw);
  for (int w = 0; w < nw; ++w) normA[w] = S.of(w)->normA;
  std::vector<DevArr<c128>> results(nw);
  std::vector<WinOut> outs;
  std::vector<int> bulk_restarts(nw, 0), bulk_breaks(nw, 0);
  std::vector<int64_t> bulk_mv(nw, 0);
  auto save_fp64 = [&](Batch<double>& Bd) {
    return [&](int w) {
      const int64_t Nw = S.of(w)->N;
      results[w].alloc(size_t(Nw) * wins[w].nev);
      check(hipMemcpy2DAsync(results[w].p, sizeof(c128) * Nw, Bd.V.p + size_t(w) * Bd.ws() + size_t(k) * ldN,
                             sizeof(c128) * ldN, sizeof(c128) * Nw, wins[w].nev, hipMemcpyDeviceToDevice, st),
            "save");
    };
  };
  if (o.precision == TSG_FP32_BULK) {
    // complex64 phase to bulk_tol; keep [V_k | F] of each window for the FP64 phase
    DevArr<c64> hand;
    hand.alloc(size_t(ldN) * (k + b) * nw);
    {
      Batch<float> Bf;
      Bf.alloc(nw, S, m, k, b, nvmax);
      if (harmonic) Bf.alloc_harmonic();
      std::vector<WinOut> fo;
      const double btol = std::max(o.bulk_tol > 0 ? o.bulk_tol : 1e-5, o.tol);
      iterate<float>(S, Bf, wins, normA, o.select, btol, o.max_restarts, o.seed, nullptr, fo, [&](int w) {
        // V (already swapped) holds the kept basis in columns [0, k); the
        // other buffer the cycle's pending continuation block in [m, m + b)
        check(hipMemcpyAsync(hand.p + size_t(w) * ldN * (k + b), Bf.V.p + size_t(w) * Bf.ws(),
                             sizeof(c64) * ldN * k, hipMemcpyDeviceToDevice, st), "handoff");
        check(hipMemcpyAsync(hand.p + size_t(w) * ldN * (k + b) + size_t(k) * ldN,
                             Bf.Vr.p + size_t(w) * Bf.ws() + size_t(m) * ldN, sizeof(c64) * ldN * b,
                             hipMemcpyDeviceToDevice, st), "handoff");
      }, use_graphs, 100.0 * btol);
      for (int w = 0; w < nw; ++w) {
        bulk_restarts[w] = fo[w].restarts;
        bulk_mv[w] = fo[w].matvecs;
        bulk_breaks[w] = fo[w].breakdowns;
      }
    }
    Batch<double> Bd;
    Bd.alloc(nw, S, m, k, b, nvmax);
    if (harmonic) Bd.alloc_harmonic();
    iterate<double>(S, Bd, wins, normA, o.select, itol, o.max_restarts, o.seed + 1, hand.p, outs, save_fp64(Bd),
                    use_graphs, 0.0, true);
  } else {
    Batch<double> Bd;
    Bd.alloc(nw, S, m, k, b, nvmax);
    if (harmonic) Bd.alloc_harmonic();
    iterate<double>(S, Bd, wins, normA, o.select, itol, o.max_restarts, o.seed, nullptr, outs, save_fp64(Bd),
                    use_graphs);
  }
  check(hipStreamSynchronize(st), "sync");
  parts.clear();
  conv.assign(nw, true);
  for (int w = 0; w < nw; ++w) {
    outs[w].matvecs += bulk_mv[w];
    Partition P = finish_window(S.of(w), st, wins[w], std::move(results[w]), wins[w].nev, outs[w], bulk_restarts[w],
                                bulk_breaks[w], o.tol);
    conv[w] = outs[w].converged && P.stats.n_conv == wins[w].nev;
    parts.push_back(std::move(P));
  }
}

// Solves windows of the systems ctx (window w on ctx[wsys[w]]; wsys empty:
// all on ctx[0]).  The windows are dealt round-robin into o.groups groups;
// each group is one batched iteration on its own stream and host thread, so
// one group's small eigensolves (a few compute units) overlap the other
// groups' bandwidth-bound expansion steps.  Results come back in window
// order.
// Device bytes one window of a batched solve holds (FP64 storage; the
// complex64 phase of FP32-bulk needs less): the basis and its rotation
// target, A V, A times the wanted vectors, the small matrices of the
// eigensolve, and the FP32-bulk hand-over block.
int64_t window_bytes(int64_t ldN, int m, int k, int b, int nv, bool bulk, bool harmonic) {
  const int64_t grid = ldN * int64_t(4 * m + 4 * b + (bulk ? (k + b) / 2 : 0)) * 16;
  const int64_t small = (int64_t(5) * m * m + smalleig_workspace(m) + int64_t(m) * (k + nv)) * 16 +
                        (harmonic ? int64_t(3) * m * m * 16 : 0);
  return grid + small;
}

void solve_core(const std::vector<tsg_ctx*>& ctx, const std::vector<int>& wsys, const std::vector<WindowSpec>& wins,
                const tsg_opts& o, hipStream_t user, std::vector<Partition>& parts, std::vector<bool>& conv) {
  const int nw = int(wins.size());
  if (nw < 1) throw InvalidArg("need at least one window");
  if (o.groups < 0) throw InvalidArg("groups must be >= 0");
  {
    // memory: when the batch does not fit in the free device memory, the
    // windows run in consecutive batches that do (each a batched iteration)
    int nvmax = 1;
    int64_t Nmax = 1, Nmin = ctx[0]->N;
    for (const auto& w : wins) nvmax = std::max(nvmax, w.nev);
    for (tsg_ctx* c : ctx) { Nmax = std::max(Nmax, c->N); Nmin = std::min(Nmin, c->N); }
    int m = 0, k = 0, b = 0;
    choose_sizes(Nmin, nvmax, o, m, k, b);
    const int64_t per = window_bytes(round_up64(Nmax, 64), m, k, b, nvmax, o.precision == TSG_FP32_BULK,
                                     o.extraction == TSG_EXTRACT_HARMONIC);
    size_t free_b = 0, total_b = 0;
    check(hipMemGetInfo(&free_b, &total_b), "hipMemGetInfo");
    // TSG_MEMORY_LIMIT_MB lowers the budget (to exercise the split on a test system)
    if (const char* lim = std::getenv("TSG_MEMORY_LIMIT_MB")) {
      const long long mb = std::atoll(lim);
      if (mb > 0) free_b = std::min<size_t>(free_b, size_t(mb) << 20);
    }
    const int64_t budget = int64_t(0.9 * double(free_b));
    const int64_t fit = per > 0 ? budget / per : nw;
    if (fit < 1)
      throw OutOfMemory("one window needs about " + std::to_string(per >> 20) + " MiB of device memory (basis " +
                        std::to_string(m) + " x N = " + std::to_string(Nmax) + " complex128), but " +
                        std::to_string(free_b >> 20) + " MiB are free: use a smaller basis (tsg_opts.basis)");
    if (fit < nw) {
      parts.clear();
      conv.clear();
      for (int w0 = 0; w0 < nw; w0 += int(fit)) {
        const int w1 = std::min(nw, w0 + int(fit));
        std::vector<WindowSpec> sub(wins.begin() + w0, wins.begin() + w1);
        std::vector<int> ssys;
        if (!wsys.empty()) ssys.assign(wsys.begin() + w0, wsys.begin() + w1);
        std::vector<Partition> sp;
        std::vector<bool> sc;
        solve_core(ctx, ssys, sub, o, user, sp, sc);
        for (auto& P : sp) parts.push_back(std::move(P));
        for (bool c2 : sc) conv.push_back(c2);
      }
      return;
    }
  }
  const int G = std::max(1, std::min(nw, o.groups > 0 ? o.groups : 1));
  check(hipStreamSynchronize(user), "sync");
  for (size_t s = 1; s < ctx.size(); ++s) check(hipStreamSynchronize(ctx[s]->st), "sync");
  std::vector<std::vector<int>> idx(G);
  for (int w = 0; w < nw; ++w) idx[w % G].push_back(w);
  std::vector<std::vector<Partition>> gparts(G);
  std::vector<std::vector<bool>> gconv(G);
  std::vector<std::exception_ptr> errs(G);
  int dev = 0;
  check(hipGetDevice(&dev), "hipGetDevice");
  auto run = [&](int g) {
    try {
      check(hipSetDevice(dev), "hipSetDevice");
      SolveStream ss(user);
      Systems S;
      std::vector<WindowSpec> wg;
      std::vector<int> sg;
      for (int w : idx[g]) {
        wg.push_back(wins[w]);
        sg.push_back(wsys.empty() ? 0 : wsys[w]);
      }
      if (ctx.size() == 1) one_system(S, ctx[0], ss.s);
      else many_systems(S, ctx, sg, ss.s);
      solve_group(S, wg, o, gparts[g], gconv[g]);
    } catch (...) {
      errs[g] = std::current_exception();
    }
  };
  if (G == 1) {
    run(0);
  } else {
    std::vector<std::thread> th;
    for (int g = 0; g < G; ++g) th.emplace_back(run, g);
    for (auto& t : th) t.join();
  }
  for (auto& e : errs)
    if (e) std::rethrow_exception(e);
  parts.clear();
  parts.resize(nw);
  conv.assign(nw, true);
  for (int g = 0; g < G; ++g)
    for (size_t q = 0; q < idx[g].size(); ++q) {
      parts[idx[g][q]] = std::move(gparts[g][q]);
      conv[idx[g][q]] = gconv[g][q];
    }
}

}  // namespace

// ------------------------------------------------------------------ public
void validate_build(const tsg_grid* g, const double* V, const tsg_absorber* ab) {
  if (!g || !V || !ab) throw InvalidArg("null argument");
  if (g->nx < 1 || g->ny < 1 || g->nz < 1) throw InvalidArg("grid sizes must be >= 1");
  if (!(g->h > 0.0) || !std::isfinite(g->h)) throw InvalidArg("h must be positive and finite");
  const int R = g->fd_radius == 0 ? 6 : g->fd_radius;
  if (R < 1 || R > 6) throw InvalidArg("fd_radius must be in 1..6");
  const double vals[6] = {ab->amp_L, ab->width_L, ab->z_L, ab->amp_R, ab->width_R, ab->z_R};
  for (double v : vals)
    if (!std::isfinite(v)) throw InvalidArg("absorber parameters must be finite");
  if (ab->amp_L < 0 || ab->amp_R < 0) throw InvalidArg("absorber amplitudes must be >= 0");
  if (!(ab->width_L > 0) || !(ab->width_R > 0)) throw InvalidArg("absorber widths must be > 0");
  const int64_t N = int64_t(g->nx) * g->ny * g->nz;
  if (N > (int64_t(1) << 31)) throw InvalidArg("grid too large");
  for (int64_t n = 0; n < N; ++n)
    if (!std::isfinite(V[n])) throw InvalidArg("V contains a non-finite value at index " + std::to_string(n));
}

void build_context(tsg_ctx* c, const tsg_grid* g, const double* V, const tsg_absorber* ab, void* stream) {
  validate_build(g, V, ab);
  const int R = g->fd_radius == 0 ? 6 : g->fd_radius;
  const int64_t N = int64_t(g->nx) * g->ny * g->nz;
  double vmin = V[0], vmax = V[0], vabs = 0.0;
  for (int64_t n = 0; n < N; ++n) {
    vmin = std::min(vmin, V[n]);
    vmax = std::max(vmax, V[n]);
    vabs = std::max(vabs, std::fabs(V[n]));
  }
  int dev = 0;
  check(hipGetDevice(&dev), "hipGetDevice");
  c->nx = g->nx; c->ny = g->ny; c->nz = g->nz; c->R = R; c->h = g->h; c->N = N;
  c->ab = *ab;
  c->st = static_cast<hipStream_t>(stream);
  const double s = -1.0 / (2.0 * g->h * g->h);
  double c0 = 0.0, sabs = 0.0;
  for (int m = 1; m <= R; ++m) {
    const double cm = fd_coef(R, m);
    c->coef[m] = s * cm;
    c0 -= 2.0 * cm;
    sabs += std::fabs(cm);
  }
  c->coef[0] = s * c0;
  c->diag0 = 3.0 * s * c0;
  std::vector<double> gL(g->nz), gR(g->nz), gam(g->nz);
  double gmax = 0.0;
  for (int k = 0; k < g->nz; ++k) {
    const double z = k * g->h;
    gL[k] = ab->amp_L * std::exp(-(z - ab->z_L) * (z - ab->z_L) / (2.0 * ab->width_L * ab->width_L));
    gR[k] = ab->amp_R * std::exp(-(z - ab->z_R) * (z - ab->z_R) / (2.0 * ab->width_R * ab->width_R));
    gam[k] = gL[k] + gR[k];
    gmax = std::max(gmax, gam[k]);
  }
  c->normA = 3.0 * (std::fabs(c0) + 2.0 * sabs) / (2.0 * g->h * g->h) + vabs + gmax;
  c->vmin = vmin; c->vmax = vmax; c->gmax = gmax;
  c->Vh.assign(V, V + N);
  c->V.alloc(N); c->Vf.alloc(N);
  c->gam.alloc(g->nz); c->gamf.alloc(g->nz); c->gL.alloc(g->nz); c->gR.alloc(g->nz);
  std::vector<float> Vf(V, V + N), gamf(gam.begin(), gam.end());
  check(hipMemcpy(c->V.p, V, sizeof(double) * N, hipMemcpyHostToDevice), "upload V");
  check(hipMemcpy(c->Vf.p, Vf.data(), sizeof(float) * N, hipMemcpyHostToDevice), "upload V");
  check(hipMemcpy(c->gam.p, gam.data(), sizeof(double) * g->nz, hipMemcpyHostToDevice), "upload gamma");
  check(hipMemcpy(c->gamf.p, gamf.data(), sizeof(float) * g->nz, hipMemcpyHostToDevice), "upload gamma");
  check(hipMemcpy(c->gL.p, gL.data(), sizeof(double) * g->nz, hipMemcpyHostToDevice), "upload gamma");
  check(hipMemcpy(c->gR.p, gR.data(), sizeof(double) * g->nz, hipMemcpyHostToDevice), "upload gamma");
  SysDesc& d = c->sys;
  d.nx = g->nx; d.ny = g->ny; d.nz = g->nz; d.pad = 0;
  d.Vd = c->V.p; d.Vf = c->Vf.p; d.Gd = c->gam.p; d.Gf = c->gamf.p;
  d.diag0 = c->diag0;
  for (int m = 0; m < 7; ++m) d.coef[m] = c->coef[m];
  c->sysd.alloc(1);
  check(hipMemcpy(c->sysd.p, &d, sizeof(SysDesc), hipMemcpyHostToDevice), "upload system");
}

void apply_operator(tsg_ctx* c, const void* X, void* Y, int ncols, int64_t ld, int dtype) {
  if (!X || !Y) throw InvalidArg("null device pointer");
  if (ncols < 1 || ld < c->N) throw InvalidArg("need ncols >= 1 and ld >= N");
  Systems S;
  one_system(S, c, c->st);
  if (dtype == TSG_C128) {
    stencil<double>(S, static_cast<const c128*>(X), ld, 0, static_cast<c128*>(Y), ld, 0, ncols, 1, nullptr);
  } else if (dtype == TSG_C64) {
    stencil<float>(S, static_cast<const c64*>(X), ld, 0, static_cast<c64*>(Y), ld, 0, ncols, 1, nullptr);
  } else {
    throw InvalidArg("dtype must be TSG_C128 or TSG_C64");
  }
  check(hipGetLastError(), "stencil launch");
}

bool solve_windows(tsg_ctx* c, const std::vector<WindowSpec>& wins, const tsg_opts& o) {
  c->have_combined = false;
  c->have_grams = false;
  std::vector<Partition> parts;
  std::vector<bool> conv;
  solve_core({c}, {}, wins, o, c->st, parts, conv);
  bool all = true;
  for (size_t w = 0; w < parts.size(); ++w) {
    all = all && conv[w];
    c->parts.push_back(std::move(parts[w]));
  }
  return all;
}

void solve_batch(const std::vector<tsg_ctx*>& ctx, const std::vector<std::vector<WindowSpec>>& wins,
                 const tsg_opts& o, std::vector<bool>& ok) {
  const int ns = int(ctx.size());
  if (ns < 1) throw InvalidArg("need at least one system");
  std::vector<WindowSpec> all;
  std::vector<int> wsys;
  for (int s = 0; s < ns; ++s) {
    if (!ctx[s]) throw InvalidArg("null context in batch");
    if (wins[s].empty()) throw InvalidArg("every system needs at least one window");
    for (const auto& w : wins[s]) { all.push_back(w); wsys.push_back(s); }
  }
  std::vector<Partition> parts;
  std::vector<bool> conv;
  solve_core(ctx, wsys, all, o, ctx[0]->st, parts, conv);
  ok.assign(ns, true);
  for (int s = 0; s < ns; ++s) {
    ctx[s]->parts.clear();
    ctx[s]->have_combined = false;
    ctx[s]->have_grams = false;
  }
  for (size_t w = 0; w < parts.size(); ++w) {
    const int s = wsys[w];
    ok[s] = ok[s] && conv[w];
    ctx[s]->parts.push_back(std::move(parts[w]));
  }
  for (int s = 0; s < ns; ++s) combine(ctx[s], o.keep_lowest);
}

void combine(tsg_ctx* c, int keep_lowest) {
  const int p = int(c->parts.size());
  if (p == 0) throw StateError("no partitions to combine");
  const int64_t N = c->N;
  hipStream_t st = c->st;
  int total = 0;
  for (auto& P : c->parts) total += int(P.eps.size());
  const double tau = 1e-6 * c->normA;
  DevArr<c128> Ucomb, v;
  DevArr<double> out;
  DevArr<int> partners;
  Ucomb.alloc(size_t(N) * std::max(total, 1));
  v.alloc(size_t(N));
  out.alloc(4);
  partners.alloc(size_t(std::max(total, 1)));
  std::vector<c128> keps;
  std::vector<int> kown;
  std::vector<uint8_t> holes(std::max(p - 1, 0), 1);
  // pending plain copies into Ucomb
  std::vector<const c128*> psrc;
  std::vector<c128> psc;
  int pend_start = 0;
  DevArr<const c128*> dsrc;
  DevArr<c128> dsc;
  dsrc.alloc(size_t(std::max(total, 1))); dsc.alloc(size_t(std::max(total, 1)));
  auto flush = [&]() {
    const int n = int(psrc.size());
    if (n == 0) return;
    check(hipMemcpyAsync(dsrc.p, psrc.data(), sizeof(void*) * n, hipMemcpyHostToDevice, st), "srcs");
    check(hipMemcpyAsync(dsc.p, psc.data(), sizeof(c128) * n, hipMemcpyHostToDevice, st), "sc");
    gather_columns(Ucomb.p + int64_t(pend_start) * N, N, dsrc.p, dsc.p, n, N, st);
    check(hipStreamSynchronize(st), "sync");
    pend_start += n;
    psrc.clear(); psc.clear();
  };
  for (int j = 0; j < p; ++j) {
    Partition& P = c->parts[j];
    const int n = int(P.eps.size());
    for (int i = 0; i < n; ++i) {
      const c128 lam = P.eps[i];
      std::vector<int> pt;
      for (int q = 0; q < int(keps.size()); ++q)
        if (cabs(keps[q] - lam) <= tau) pt.push_back(q);
      if (pt.empty()) {
        psrc.push_back(P.U.p + int64_t(i) * N);
        psc.push_back(c128{1.0, 0.0});
        keps.push_back(lam);
        kown.push_back(j);
        continue;
      }
      flush();
      check(hipMemcpyAsync(v.p, P.U.p + int64_t(i) * N, sizeof(c128) * N, hipMemcpyDeviceToDevice, st), "copy v");
      check(hipMemcpyAsync(partners.p, pt.data(), sizeof(int) * pt.size(), hipMemcpyHostToDevice, st), "partners");
      project_out(v.p, Ucomb.p, N, partners.p, int(pt.size()), N, out.p, st);
      double h[4];
      check(hipMemcpyAsync(h, out.p, sizeof(h), hipMemcpyDeviceToHost, st), "norms");
      check(hipStreamSynchronize(st), "sync");
      if (h[1] < 1e-3 * h[0]) {
        // partitions o and j share this eigenvalue, so their windows overlap
        // and no interface between them hides a gap
        for (int q : pt) {
          const int o = kown[q];
          for (int t = std::min(o, j); t < std::max(o, j); ++t) holes[t] = 0;
        }
        continue;
      }
      const c128 sc = cdiv(c128{1.0, 0.0}, csqrt(c128{h[2], h[3]}));
      psrc.push_back(v.p);
      psc.push_back(sc);
      keps.push_back(lam);
      kown.push_back(j);
      flush();  // v is reused: materialise now
    }
  }
  flush();
  const int nk = int(keps.size());
  std::vector<int> ord(nk);
  std::iota(ord.begin(), ord.end(), 0);
  std::sort(ord.begin(), ord.end(), [&](int a, int b) {
    if (keps[a].re != keps[b].re) return keps[a].re < keps[b].re;
    return keps[a].im < keps[b].im;
  });
  int nout = nk;
  if (keep_lowest > 0 && keep_lowest < nk) nout = keep_lowest;
  c->Uc.alloc(size_t(N) * std::max(nout, 1));
  std::vector<const c128*> srcs(nout);
  std::vector<c128> scs(nout, c128{1.0, 0.0});
  c->epsc.resize(nout);
  c->ownerc.resize(nout);
  for (int i = 0; i < nout; ++i) {
    srcs[i] = Ucomb.p + int64_t(ord[i]) * N;
    c->epsc[i] = keps[ord[i]];
    c->ownerc[i] = kown[ord[i]];
  }
  if (nout > 0) {
    check(hipMemcpyAsync(dsrc.p, srcs.data(), sizeof(void*) * nout, hipMemcpyHostToDevice, st), "srcs");
    check(hipMemcpyAsync(dsc.p, scs.data(), sizeof(c128) * nout, hipMemcpyHostToDevice, st), "sc");
    gather_columns(c->Uc.p, N, dsrc.p, dsc.p, nout, N, st);
  }
  check(hipStreamSynchronize(st), "sync");
  c->nc = nout;
  c->holes = holes;
  c->have_combined = true;
  c->have_grams = false;
}

// Algorithm 1's repeat loop (Section 2.2): partitions ordered by shift, so
// interface j lies between partitions j and j+1; each flagged interface (and
// the stretch above E_min when no computed pair reaches down to it) gets a
// partition centred in the gap between the two partitions' eigenvalues with
// 3/2 gap / Delta eigenpairs, clamped to [1, n_cap] (Delta is the spectrum's
// mean spacing, which overstates the count where eigenvalues are sparse, so
// the cap keeps one window's basis bounded and the loop repeats instead).
FillResult fill_holes(tsg_ctx* c, double e_min, int n_cap, int max_rounds, const tsg_opts& o) {
  if (c->parts.empty()) throw StateError("no partitions: run a solve first");
  for (const Partition& P : c->parts)
    if (P.shift_im != 0.0)
      throw InvalidArg("hole filling orders partitions along the real axis: every shift must be real");
  if (n_cap < 1 || max_rounds < 0) throw InvalidArg("need n_cap >= 1 and max_rounds >= 0");
  const double e_max = upper_bound_real(c);
  if (!std::isfinite(e_min) || !(e_min < e_max)) throw InvalidArg("e_min must be finite and below E_max");
  const double delta = (e_max - e_min) / double(c->N);
  const double tau = 1e-6 * c->normA;
  auto window = [&](double lo, double hi) {
    const double gap = hi - lo;
    double cnt = gap > 0 ? std::ceil(1.5 * gap / delta) : 1.0;
    cnt = std::min(std::max(cnt, 1.0), double(n_cap));
    return WindowSpec{0.5 * (lo + hi), int(cnt)};
  };
  // the interval starts at E_min, itself an eigenvalue: a lowest computed
  // real part more than tau above it leaves a gap at the bottom
  auto lowest = [&]() {
    double low = HUGE_VAL;
    for (const Partition& P : c->parts)
      for (const c128& e : P.eps) low = std::min(low, e.re);
    return low;
  };
  auto reorder = [&]() {
    std::stable_sort(c->parts.begin(), c->parts.end(),
                     [](const Partition& a, const Partition& b) { return a.shift < b.shift; });
  };
  FillResult r;
  reorder();
  combine(c, o.keep_lowest);
  while (r.rounds < max_rounds) {
    std::vector<WindowSpec> add;
    const double low = lowest();
    if (std::isfinite(low) && low > e_min + tau) add.push_back(window(e_min, low));
    for (size_t j = 0; j + 1 < c->parts.size(); ++j) {
      if (!c->holes[j]) continue;
      const auto& lo = c->parts[j].eps;
      const auto& hi = c->parts[j + 1].eps;
      if (lo.empty() || hi.empty()) continue;
      double a = lo[0].re, b = hi[0].re;
      for (const c128& e : lo) a = std::max(a, e.re);
      for (const c128& e : hi) b = std::min(b, e.re);
      add.push_back(window(a, b));
    }
    if (add.empty()) break;
    ++r.rounds;
    r.added += int(add.size());
    r.converged = solve_windows(c, add, o) && r.converged;
    reorder();
    combine(c, o.keep_lowest);
  }
  for (uint8_t h : c->holes) r.holes_left += h ? 1 : 0;
  const double low = lowest();
  if (std::isfinite(low) && low > e_min + tau) r.holes_left += 1;
  return r;
}

namespace {

std::vector<int> window_counts(int n_r, int p, int mode) {
  std::vector<int> counts(p);
  if (mode != TSG_PLAN_ALG1) {
    const int base = n_r / p;
    for (int j = 0; j < p; ++j) counts[j] = base + (j < n_r - base * p ? 1 : 0);
    return counts;
  }
  // Algorithm 1: n_{r,j} = round(2/(1.5 + (j-1)/p) n_r/p) for j <= p/2,
  // ceil(2 n_r/p) - n_{r,p-j+1} otherwise (middle of odd p: half of it).
  const long top = (2L * n_r + p - 1) / p;
  for (int j = 1; j <= p; ++j)
    if (2 * j <= p) counts[j - 1] = int(std::floor(2.0 / (1.5 + double(j - 1) / p) * double(n_r) / p + 0.5));
  for (int j = 1; j <= p; ++j)
    if (2 * j > p) {
      const int mirror = p - j + 1;
      counts[j - 1] = (mirror == j) ? int((top + 1) / 2) : int(top - counts[mirror - 1]);
    }
  return counts;
}

double smallest_real_part(tsg_ctx* c, const tsg_opts& o) {
  // the exterior eigenvalue of smallest real part (Section 2.2), as a
  // temporary one-eigenpair partition
  const size_t keep_parts = c->parts.size();
  tsg_opts oe = o;
  oe.precision = TSG_FP64;
  oe.basis = 0;
  oe.keep = 0;
  oe.select = TSG_SELECT_SMALLEST_REAL;
  oe.extraction = TSG_EXTRACT_RITZ;  // an exterior end: ordinary Ritz pairs
  oe.max_restarts = std::max(o.max_restarts, 2000);
  const bool ok = solve_windows(c, {WindowSpec{0.0, 1}}, oe);
  const bool found = ok && !c->parts.back().eps.empty();
  const double e = found ? c->parts.back().eps[0].re : 0.0;
  c->parts.resize(keep_parts);
  if (!found) throw StateError("exterior eigenvalue did not converge");
  return e;
}

}  // namespace

double upper_bound_real(const tsg_ctx* c) {
  // Re eps = u^H (K + V) u / u^H u <= max V + 3 max_theta s(theta) / (2 h^2); the
  // radius-R symbol s(theta) = -(c_0 + 2 sum c_m cos m theta) peaks at theta = pi
  // for these weights, where it equals |c_0| + 2 sum |c_m|.
  double smax = std::fabs(c->coef[0]);
  for (int m = 1; m <= c->R; ++m) smax += 2.0 * std::fabs(c->coef[m]);
  return c->vmax + 3.0 * smax;
}

void plan_windows(tsg_ctx* c, int n_r, int p, int mode, const tsg_opts& o, std::vector<WindowSpec>& out,
                  double* e_range) {
  if (n_r < 1 || p < 1) throw InvalidArg("need n_r >= 1 and p >= 1");
  if (mode != TSG_PLAN_ALG1 && mode != TSG_PLAN_EQUAL && mode != TSG_PLAN_SAMPLED && mode != TSG_PLAN_SEMICLASSICAL)
    throw InvalidArg("unknown planning mode");
  const int q = o.imag_bands > 0 ? o.imag_bands : 1;
  if (q > 1 && (mode != TSG_PLAN_SEMICLASSICAL || p % q != 0))
    throw InvalidArg("imaginary bands need TSG_PLAN_SEMICLASSICAL and p a multiple of imag_bands");
  if (q > 1) {
    // two-dimensional partitioning: p/q real placements, each split into q
    // windows spread over the imaginary range [-max Gamma, 0] of Eq. (5)
    tsg_opts o1 = o;
    o1.imag_bands = 1;
    std::vector<WindowSpec> re;
    plan_windows(c, n_r, p / q, mode, o1, re, e_range);
    out.clear();
    for (const WindowSpec& r : re)
      for (int i = 0; i < q; ++i) {
        const int base = r.nev / q, extra = (i < r.nev - base * q) ? 1 : 0;
        out.push_back(WindowSpec{r.shift, std::max(base + extra, 1), -c->gmax * (i + 0.5) / q});
      }
    return;
  }
  const double e_min = smallest_real_part(c, o);
  const double e_max = upper_bound_real(c);
  const std::vector<int> counts = window_counts(n_r, p, mode == TSG_PLAN_ALG1 ? TSG_PLAN_ALG1 : TSG_PLAN_EQUAL);
  out.resize(p);
  if (mode == TSG_PLAN_SEMICLASSICAL) {
    // Counting function from the phase-space volume of p^2/2 + V over the
    // box, N(E) = w sum_r k_r^3 / (6 pi^2) - S <k_r^2> / (16 pi) with
    // k_r^2 = 2 max(E - V_r, 0) (Weyl's law with its Dirichlet surface
    // term); windows at the midpoints of consecutive intervals of n_{r,j}
    // eigenvalues (the placement of Section 3).
    const double lx = (c->nx + 1) * c->h, ly = (c->ny + 1) * c->h, lz = (c->nz + 1) * c->h;
    const double vol = lx * ly * lz, surf = 2.0 * (lx * ly + ly * lz + lx * lz);
    std::vector<double> vs(c->Vh);
    std::sort(vs.begin(), vs.end());
    auto count = [&](double E) {
      double s3 = 0.0, s2 = 0.0;
      for (double v : vs) {
        if (v >= E) break;
        const double k2 = 2.0 * (E - v);
        s3 += k2 * std::sqrt(k2);
        s2 += k2;
      }
      const double n = double(vs.size());
      return (vol / n) * s3 / (6.0 * M_PI * M_PI) - surf * (s2 / n) / (16.0 * M_PI);
    };
    auto inverse = [&](double target) {
      if (target <= 0) return e_min;
      double lo = e_min, width = 1.0;
      while (count(lo + width) < target) width *= 2.0;
      double hi = lo + width;
      for (int it = 0; it < 100; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (count(mid) < target) lo = mid; else hi = mid;
      }
      return 0.5 * (lo + hi);
    };
    int acc = 0;
    for (int j = 0; j < p; ++j) {
      out[j] = WindowSpec{0.5 * (inverse(acc) + inverse(acc + counts[j])), counts[j]};
      acc += counts[j];
    }
  } else if (mode != TSG_PLAN_SAMPLED) {
    // E_{S,j} = E_{S,j-1} + ((E_max - E_min)/N)(n_{r,j} + n_{r,j-1})/2
    const double delta = (e_max - e_min) / double(c->N);
    double prev_s = e_min;
    int prev_n = 0;
    for (int j = 0; j < p; ++j) {
      const double s = prev_s + delta * (counts[j] + prev_n) / 2.0;
      out[j] = WindowSpec{s, counts[j]};
      prev_s = s;
      prev_n = counts[j];
    }
  } else {
    // Density sampling (Section 2.2): a few eigenpairs at sample shifts over
    // the region of interest give the local eigenvalue density; its integral
    // estimates the counting function, and the windows sit at the midpoints
    // of consecutive intervals holding n_{r,j} eigenvalues (the placement of
    // Section 3).  The region's top is first guessed from the free-particle
    // counting function of the box.
    const double lx = (c->nx + 1) * c->h, ly = (c->ny + 1) * c->h, lz = (c->nz + 1) * c->h;
    const double kf = std::pow(6.0 * M_PI * M_PI * double(n_r) / (lx * ly * lz), 1.0 / 3.0);
    double top = std::max(0.5 * kf * kf, 0.0);
    top = std::max(top, e_min + 0.25) * 1.25 + 0.25 * std::fabs(e_min);
    const int S = std::max(2 * p, 8), ns = 8;
    std::vector<WindowSpec> probes(S);
    for (int i = 0; i < S; ++i) probes[i] = WindowSpec{e_min + (top - e_min) * (i + 0.5) / S, ns};
    const size_t keep_parts = c->parts.size();
    tsg_opts op = o;
    op.precision = TSG_FP64;
    op.tol = std::max(o.tol, 1e-6);
    op.basis = 0;
    op.keep = 0;
    op.select = TSG_SELECT_NEAREST;
    op.max_restarts = std::max(o.max_restarts, 2000);
    (void)solve_windows(c, probes, op);
    std::vector<double> pc(1, e_min), rho(1, 0.0);
    for (int i = 0; i < S; ++i) {
      const Partition& P = c->parts[keep_parts + i];
      if (P.eps.size() < 2) continue;  // a probe left with fewer than two pairs gives no density
      double lo = P.eps[0].re, hi = P.eps[0].re, sum = 0.0;
      for (const auto& e : P.eps) { lo = std::min(lo, e.re); hi = std::max(hi, e.re); sum += e.re; }
      pc.push_back(sum / P.eps.size());
      rho.push_back(double(P.eps.size() - 1) / std::max(hi - lo, 1e-12));
    }
    c->parts.resize(keep_parts);
    const int nsv = int(pc.size()) - 1;
    if (nsv < 1) throw StateError("density sampling: no probe converged");
    rho[0] = rho[1];
    // order the sample points, then integrate the piecewise-linear density
    std::vector<int> ord(nsv + 1);
    std::iota(ord.begin(), ord.end(), 0);
    std::sort(ord.begin(), ord.end(), [&](int a, int b2) { return pc[a] < pc[b2]; });
    std::vector<double> xs, cum;
    xs.push_back(pc[ord[0]]);
    cum.push_back(0.0);
    for (int q = 1; q <= nsv; ++q) {
      const double x0 = pc[ord[q - 1]], x1 = pc[ord[q]];
      xs.push_back(x1);
      cum.push_back(cum.back() + 0.5 * (rho[ord[q - 1]] + rho[ord[q]]) * (x1 - x0));
    }
    auto inverse = [&](double target) {
      for (size_t q = 1; q < xs.size(); ++q)
        if (cum[q] >= target) {
          const double f = (target - cum[q - 1]) / std::max(cum[q] - cum[q - 1], 1e-300);
          return xs[q - 1] + f * (xs[q] - xs[q - 1]);
        }
      const double last_rho = rho[ord[nsv]];
      return xs.back() + (target - cum.back()) / std::max(last_rho, 1e-12);
    };
    double acc = 0.0;
    for (int j = 0; j < p; ++j) {
      const double a = inverse(acc), b2 = inverse(acc + counts[j]);
      out[j] = WindowSpec{0.5 * (a + b2), counts[j]};
      acc += counts[j];
    }
  }
  if (e_range) { e_range[0] = e_min; e_range[1] = e_max; }
}

namespace {

// M^R, M^L, W = M^R o M^L of the combined set (cached until the next solve).
void ensure_grams(tsg_ctx* c) {
  if (c->have_grams) return;
  const int n = c->nc;
  hipStream_t st = c->st;
  const size_t nn = size_t(n) * n;
  c->MR.alloc(nn); c->ML.alloc(nn); c->Wt.alloc(nn); c->epsd.alloc(n);
  DevArr<c128> part;
  part.alloc(size_t(gamma_gram_workspace(c->N, n)));
  gamma_grams<double>(c->Uc.p, c->N, c->N, n, c->gL.p, c->gR.p, c->nx * c->ny, c->MR.p, c->ML.p, c->Wt.p, part.p, st);
  check(hipMemcpyAsync(c->epsd.p, c->epsc.data(), sizeof(c128) * n, hipMemcpyHostToDevice, st), "eps");
  check(hipStreamSynchronize(st), "sync");
  c->have_grams = true;
}

}  // namespace

void transmission(tsg_ctx* c, const double* E, int nE, double* T) {
  if (!E || !T || nE < 1) throw InvalidArg("need energies and outputs, nE >= 1");
  if (!c->have_combined) throw StateError("no combined eigenpairs: run a solve first");
  for (int e = 0; e < nE; ++e)
    if (!std::isfinite(E[e])) throw InvalidArg("energies must be finite");
  const int n = c->nc;
  hipStream_t st = c->st;
  if (n == 0) {
    for (int e = 0; e < nE; ++e) T[e] = 0.0;
    return;
  }
  ensure_grams(c);
  DevArr<double> dE, dT;
  dE.alloc(nE); dT.alloc(nE);
  check(hipMemcpyAsync(dE.p, E, sizeof(double) * nE, hipMemcpyHostToDevice, st), "E");
  transmission_sweep(c->Wt.p, n, c->epsd.p, dE.p, nE, dT.p, st);
  check(hipMemcpyAsync(T, dT.p, sizeof(double) * nE, hipMemcpyDeviceToHost, st), "T");
  check(hipStreamSynchronize(st), "sync");
}

int transmission_vjp(tsg_ctx* c, const double* E, int nE, const double* w, double* dV, double* dabs) {
  if (!E || !w || !dV || !dabs || nE < 1) throw InvalidArg("need energies, weights and outputs, nE >= 1");
  if (!c->have_combined) throw StateError("no combined eigenpairs: run a solve first");
  for (int e = 0; e < nE; ++e)
    if (!std::isfinite(E[e]) || !std::isfinite(w[e])) throw InvalidArg("energies and weights must be finite");
  const int n = c->nc;
  const int64_t N = c->N, plane = int64_t(c->nx) * c->ny;
  hipStream_t st = c->st;
  if (n == 0) {
    std::fill(dV, dV + N, 0.0);
    std::fill(dabs, dabs + 4, 0.0);
    return 0;
  }
  ensure_grams(c);
  const size_t nn = size_t(n) * n, Nn = size_t(N) * n;
  const Rows rows{N, nullptr};
  DevArr<double> dE, dw, dVd, dGL, dGR, prof, dab, sums, cpart;
  DevArr<c128> G, KRt, KLt, Ub, YR, YL, Z, C, B, MU, X, R, MRv, P, MP, Ct, rho, alpha, beta, gpart;
  DevArr<int> done;
  dE.alloc(nE); dw.alloc(nE);
  check(hipMemcpyAsync(dE.p, E, sizeof(double) * nE, hipMemcpyHostToDevice, st), "E");
  check(hipMemcpyAsync(dw.p, w, sizeof(double) * nE, hipMemcpyHostToDevice, st), "w");
  G.alloc(size_t(n) * nE); KRt.alloc(nn); KLt.alloc(nn);
  adj_gmat(c->epsd.p, n, dE.p, nE, G.p, st);
  adj_kmats(G.p, n, nE, dw.p, c->MR.p, c->ML.p, KRt.p, KLt.p, st);
  // Y^X = conj(U) (K^X)^T; explicit Gamma terms D_X = Re rowsum(U o Y^X)
  Ub.alloc(Nn); YR.alloc(Nn); YL.alloc(Nn); Z.alloc(Nn);
  adj_conj(c->Uc.p, Ub.p, int64_t(Nn), st);
  gemm_cols<double>(Ub.p, N, 0, KRt.p, n, 0, YR.p, N, 0, rows, n, n, 0.0, 1, st);
  gemm_cols<double>(Ub.p, N, 0, KLt.p, n, 0, YL.p, N, 0, rows, n, n, 0.0, 1, st);
  dVd.alloc(N); dGL.alloc(N); dGR.alloc(N);
  check(hipMemsetAsync(dVd.p, 0, sizeof(double) * N, st), "zero");
  check(hipMemsetAsync(dGL.p, 0, sizeof(double) * N, st), "zero");
  check(hipMemsetAsync(dGR.p, 0, sizeof(double) * N, st), "zero");
  adj_rowdot(c->Uc.p, YR.p, N, n, 1.0, false, dGR.p, st);
  adj_rowdot(c->Uc.p, YL.p, N, n, 1.0, false, dGL.p, st);
  adj_zcombine(YR.p, YL.p, c->gR.p, c->gL.p, N, n, plane, Z.p, st);
  // in-set part: mu = U B with B = (P + P^T)/2 (no eigenvalue differences)
  int64_t pw = std::max<int64_t>(gram_workspace(N, n, n, 1), 1);
  gpart.alloc(size_t(pw));
  C.alloc(nn); B.alloc(nn); MU.alloc(Nn); Ct.alloc(nn);
  adj_inset(G.p, n, nE, dw.p, c->MR.p, c->ML.p, Ct.p, B.p, st);
  gemm_cols<double>(c->Uc.p, N, 0, B.p, n, 0, MU.p, N, 0, rows, n, n, 0.0, 1, st);
  // C = U^T Z for the right-hand sides of the out-of-set solves
  gram<double, double>(Ub.p, N, 0, Z.p, N, 0, rows, n, n, C.p, n, 0, 1, gpart.p, pw, st);
  // out-of-set part: (eps_k - A) x_k = P z_k with P = I - U U^T, solved by
  // COCR on the projected operator P (eps_k - A) P (complex symmetric, as
  // P^T = P), all k together
  X.alloc(Nn); R.alloc(Nn); MRv.alloc(Nn); P.alloc(Nn); MP.alloc(Nn);
  rho.alloc(n); alpha.alloc(n); beta.alloc(n); done.alloc(n);
  sums.alloc(size_t(n) * 5);
  cpart.alloc(size_t(adj_cocr_workspace(N, n)));
  check(hipMemsetAsync(X.p, 0, sizeof(c128) * Nn, st), "zero");
  check(hipMemsetAsync(done.p, 0, sizeof(int) * n, st), "zero");
  check(hipMemcpyAsync(R.p, Z.p, sizeof(c128) * Nn, hipMemcpyDeviceToDevice, st), "rhs");
  gemm_cols<double>(c->Uc.p, N, 0, C.p, n, 0, R.p, N, 0, rows, n, n, 1.0, 1, st, nullptr, -1.0);
  Systems S;
  one_system(S, c, st);
  auto project = [&](c128* V) {  // V -= U (U^T V)
    gram<double, double>(Ub.p, N, 0, V, N, 0, rows, n, n, Ct.p, n, 0, 1, gpart.p, pw, st);
    gemm_cols<double>(c->Uc.p, N, 0, Ct.p, n, 0, V, N, 0, rows, n, n, 1.0, 1, st, nullptr, -1.0);
  };
  auto apply_M = [&](const c128* V, c128* MV) {  // MV = P (eps_k V - A V)
    stencil<double>(S, V, N, 0, MV, N, 0, n, 1, nullptr);
    adj_shift(V, MV, c->epsd.p, N, n, st);
    project(MV);
  };
  project(R.p);
  apply_M(R.p, MRv.p);
  check(hipMemcpyAsync(P.p, R.p, sizeof(c128) * Nn, hipMemcpyDeviceToDevice, st), "p");
  check(hipMemcpyAsync(MP.p, MRv.p, sizeof(c128) * Nn, hipMemcpyDeviceToDevice, st), "mp");
  adj_cocr_sums(R.p, MRv.p, MP.p, N, n, cpart.p, sums.p, st);
  adj_scalars(sums.p, n, 0, rho.p, alpha.p, beta.p, done.p, st);
  std::vector<double> hs(size_t(n) * 5), bnorm(n);
  check(hipMemcpyAsync(hs.data(), sums.p, sizeof(double) * 5 * n, hipMemcpyDeviceToHost, st), "sums");
  check(hipStreamSynchronize(st), "sync");
  for (int k = 0; k < n; ++k) bnorm[k] = std::sqrt(hs[size_t(k) * 5 + 4]);
  const double tol = 1e-11;
  const int maxit = 20000;
  std::vector<int> hdone(n, 0);
  int it = 0;
  bool conv = false;
  for (auto& x : hdone) x = 0;
  for (it = 1; it <= maxit; ++it) {
    adj_scalars(sums.p, n, 1, rho.p, alpha.p, beta.p, done.p, st);
    adj_xr(X.p, R.p, P.p, MP.p, alpha.p, N, n, st);
    apply_M(R.p, MRv.p);
    adj_cocr_sums(R.p, MRv.p, MP.p, N, n, cpart.p, sums.p, st);
    adj_scalars(sums.p, n, 2, rho.p, alpha.p, beta.p, done.p, st);
    adj_p(P.p, MP.p, R.p, MRv.p, beta.p, N, n, st);
    // (Mp)^T (Mp) for the next alpha
    adj_cocr_sums(R.p, MRv.p, MP.p, N, n, cpart.p, sums.p, st);
    if (it % 10 == 0 || it == maxit) {
      check(hipMemcpyAsync(hs.data(), sums.p, sizeof(double) * 5 * n, hipMemcpyDeviceToHost, st), "sums");
      check(hipStreamSynchronize(st), "sync");
      bool all = true;
      for (int k = 0; k < n; ++k) {
        if (!hdone[k] && std::sqrt(hs[size_t(k) * 5 + 4]) <= tol * std::max(bnorm[k], 1e-300)) hdone[k] = 1;
        all = all && hdone[k];
      }
      check(hipMemcpyAsync(done.p, hdone.data(), sizeof(int) * n, hipMemcpyHostToDevice, st), "done");
      if (progress_on() && it % 100 == 0) {
        int nd = 0;
        for (int k = 0; k < n; ++k) nd += hdone[k];
        std::fprintf(stderr, "[tsg] adjoint COCR iteration %d: %d of %d solves converged\n", it, nd, n);
      }
      if (all) { conv = true; break; }
    }
  }
  project(X.p);
  adj_add(MU.p, X.p, int64_t(Nn), st);
  // dL/dV = 2 Re sum_k mu_k u_k; through A, dL/dGamma_X gains 2 Im sum_k mu_k u_k
  adj_rowdot(c->Uc.p, MU.p, N, n, 2.0, false, dVd.p, st);
  adj_rowdot(c->Uc.p, MU.p, N, n, 2.0, true, dGL.p, st);
  adj_rowdot(c->Uc.p, MU.p, N, n, 2.0, true, dGR.p, st);
  // absorber parameters: dGamma_X/da_X = e_X(z), dGamma_X/dw_X = a_X e_X(z) (z - z_X)^2 / w_X^3
  std::vector<double> hp(size_t(4) * c->nz);
  const tsg_absorber& ab = c->ab;
  for (int k = 0; k < c->nz; ++k) {
    const double z = k * c->h;
    const double eL = std::exp(-(z - ab.z_L) * (z - ab.z_L) / (2.0 * ab.width_L * ab.width_L));
    const double eR = std::exp(-(z - ab.z_R) * (z - ab.z_R) / (2.0 * ab.width_R * ab.width_R));
    hp[k] = eL;
    hp[size_t(c->nz) + k] = ab.amp_L * eL * (z - ab.z_L) * (z - ab.z_L) / std::pow(ab.width_L, 3);
    hp[size_t(2) * c->nz + k] = eR;
    hp[size_t(3) * c->nz + k] = ab.amp_R * eR * (z - ab.z_R) * (z - ab.z_R) / std::pow(ab.width_R, 3);
  }
  prof.alloc(hp.size()); dab.alloc(4);
  check(hipMemcpyAsync(prof.p, hp.data(), sizeof(double) * hp.size(), hipMemcpyHostToDevice, st), "prof");
  adj_absorber(dGL.p, dGR.p, prof.p, N, c->nz, plane, dab.p, st);
  check(hipMemcpyAsync(dV, dVd.p, sizeof(double) * N, hipMemcpyDeviceToHost, st), "dV");
  check(hipMemcpyAsync(dabs, dab.p, sizeof(double) * 4, hipMemcpyDeviceToHost, st), "dabs");
  check(hipStreamSynchronize(st), "sync");
  if (!conv) throw NotConverged("projected COCR did not reach its tolerance in " + std::to_string(maxit) + " steps");
  return it;
}

void dense_eig(void* H, int m, int batch, void* theta, void* Y, int* info, hipStream_t st) {
  if (!H || !theta || !Y || !info) throw InvalidArg("null device pointer");
  if (m < 1 || batch < 1) throw InvalidArg("need m >= 1 and batch >= 1");
  if (m > kMaxDenseBasis) throw InvalidArg("m exceeds the largest supported matrix (896)");
  DevArr<c128> work;
  work.alloc(size_t(smalleig_workspace(m)) * batch);
  smalleig(static_cast<c128*>(H), int64_t(m) * m, m, static_cast<c128*>(theta), m, static_cast<c128*>(Y),
           int64_t(m) * m, work.p, smalleig_workspace(m), info, batch, st);
  check(hipStreamSynchronize(st), "sync");
}

}  // namespace tsg
