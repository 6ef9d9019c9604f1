// K4, QR phase: Schur form of an upper Hessenberg matrix (complex FP64),
// one workgroup per window, accumulating the Schur vectors Z.
//
// The QR iteration (Golub & Van Loan, Matrix Computations, Sec. 7.5) is a
// chain of dependent Givens rotations, so its speed on a GPU is set by the
// latency of one rotation step.  Two paths:
//   * block of at most kFin rows: the whole active block and its accumulated
//     unitary live in LDS; single-shift (Wilkinson) sweeps with one barrier
//     per rotation; then the unitary is applied to Z and to the parts of H
//     outside the block as small matrix products;
//   * larger blocks: multishift sweeps with a chain of bulges, three
//     positions apart, chased together through global memory (Braman, Byers
//     & Mathias, SIAM J. Matrix Anal. Appl. 23 (2002) 929), the shifts being
//     the eigenvalues of the trailing block; rotations of different bulges
//     touch disjoint row pairs (left) and column pairs (right), and left and
//     right rotations commute, so each step applies all left rotations, then
//     all right rotations.
// The chase updates H only.  Every step's rotations (and every unitary of a
// block finished in LDS) go to a per-window log, and a second kernel replays
// the log onto the rows of Z, many workgroups per window: a row of Z is
// transformed by right rotations independently of every other row, so the
// replay is parallel over rows and off the chase's critical path.
// Likewise the left transformations of the columns to the right of the
// active block [lo, ihi]: nothing in the iteration reads those columns again
// (ihi only decreases), so the chase leaves them and a third kernel replays
// the log onto them, many workgroups per window over bands of columns.  Each
// record carries the ihi of its step; column j takes the records whose ihi is
// below j, a suffix of the log.
// Within a sweep the same holds for most of the active block: no later step
// of the sweep reads the rows above the bulge train, and none reads a column
// well to the right of it before the train arrives.  Those updates go to
// helper workgroups of the same launch on other CUs (see chase_helper), so
// that the chase itself only touches the rows and columns around the train;
// the helpers also take the sweep's share of the two replays above.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <string>

#include "kernels.h"

namespace tsg {
namespace {

#ifndef TSG_SCHUR_THREADS
#define TSG_SCHUR_THREADS 1024
#endif
constexpr int kQT = TSG_SCHUR_THREADS;  // threads per workgroup
// largest block finished in LDS (measured at 8 x 450: 32 is 1-2% faster than
// 64, the multishift sweeps being quicker than the one-wavefront QR from there)
constexpr int kFin = 32;
constexpr int kMaxShift = 64;
// Shifts per multishift sweep.  Measured on gfx950 (m = 304, 8 matrices):
// 12-16 shifts are fastest (about 0.7x the time of 48), since the shift
// computation (an eigenvalue QR of the trailing block in one wavefront)
// grows with the cube of the count.
#ifndef TSG_SCHUR_SHIFTS
#define TSG_SCHUR_SHIFTS 16
#endif
constexpr int kShifts = TSG_SCHUR_SHIFTS;
constexpr int kQAcc = (kFin + kShifts - 1) / kShifts;  // outputs per lane of a Q-block row
// Rotation items a thread loads before it stores any (memory-level
// parallelism of the chase phases).
#ifndef TSG_SCHUR_BATCH
#define TSG_SCHUR_BATCH 2
#endif
constexpr int kBatch = TSG_SCHUR_BATCH;

// One logged rotation: Z(:, [p, p+1]) <- Z(:, [p, p+1]) [c -s; conj(s) c].
// A step holds kShifts records (p = -1: inactive slot).  A step whose first
// record has p = -2 stands for the unitary of a block finished in LDS:
// Z(:, lo:lo+n) <- Z(:, lo:lo+n) Q, with lo = c, n = s.re and Q the block
// (n x n, row-major) at offset s.im of the Q store (blocks packed).
struct RotRec {
  double c;
  int p;
  int pad;
  c128 s;
};
static_assert(sizeof(RotRec) == 32, "RotRec layout");
// Set in record 1's ihi field of every step of a sweep whose far updates went
// to helper workgroups: they have applied its left rotations to the columns
// beyond ihi and its right rotations to Z, so the replays skip the step.
constexpr int kDeferredStep = 1 << 30;

// Per-window log, in c128 units: a 2-entry header (steps, Q blocks), the
// step records, the Q store.  The capacity covers 80 multishift sweeps; a
// chase that needs more flushes the log onto Z itself and starts over.
__host__ __device__ inline int64_t log_steps_cap(int m) { return int64_t(80) * (m + 3 * kShifts); }
__host__ __device__ inline int64_t log_qstore_offset(int m) { return 2 + log_steps_cap(m) * kShifts * 2; }
constexpr int kQCap = 32 * kFin * kFin;  // Q store entries before the chase flushes the log
__host__ __device__ inline int64_t log_sync_offset(int m) { return log_qstore_offset(m) + kQCap; }

__device__ inline double cabs1(c128 z) { return fabs(z.re) + fabs(z.im); }

// 1/sqrt(v): hardware estimate refined by two Newton steps (full FP64
// accuracy, so that each rotation is unitary to rounding).
__device__ inline double rsqrt_nr(double v) {
  double r = __builtin_amdgcn_rsq(v);
  r = r * (1.5 - 0.5 * v * r * r);
  return r * (1.5 - 0.5 * v * r * r);
}

__device__ inline void givens(c128 x, c128 y, double& c, c128& s) {
  // [c s; -conj(s) c] [x; y] = [r; 0], c real >= 0, without divisions:
  // c = |x| / r, s = (x / |x|) conj(y) / r, r = sqrt(|x|^2 + |y|^2)
  const double nx2 = norm2(x), ny2 = norm2(y);
  if (ny2 == 0.0) { c = 1.0; s = c128{0.0, 0.0}; return; }
  if (nx2 == 0.0) { c = 0.0; s = rsqrt_nr(ny2) * conj(y); return; }
  const double ir = rsqrt_nr(nx2 + ny2), ix = rsqrt_nr(nx2);
  c = nx2 * ix * ir;
  s = (ix * ir) * (x * conj(y));
}

// Synchronisation for the single-wavefront LDS sweeps: a wavefront runs in
// lockstep and its LDS operations complete in order, so a fence plus a
// wave barrier orders the lanes' LDS traffic.
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline c128 wilkinson(c128 a, c128 b, c128 c2, c128 d) {
  // eigenvalue of [[a b][c2 d]] closer to d
  const c128 hd = 0.5 * (a - d);
  const c128 disc = csqrt(hd * hd + b * c2);
  const c128 mid = 0.5 * (a + d);
  const c128 l1 = mid + disc, l2 = mid - disc;
  return (cabs(l1 - d) <= cabs(l2 - d)) ? l1 : l2;
}

// Optional phase timers (wall clock, 100 MHz), summed over windows; read
// and printed by the host when TSG_K4PROF=1.
__device__ unsigned long long g_k4prof[8];

struct QRShared {
  int lo, flag, iter;
  double rc[2];
  c128 rs[2];
  c128 mu;
  double red[kQT];
  int ired[kQT];
  c128 shift[kMaxShift];
  double bc[kMaxShift];
  c128 bs[kMaxShift];
  int bp[kMaxShift];
  // column p of rows p+1 and p+2 after bulge j's right rotation at p: the
  // two values its next rotation is built from
  c128 fx[kMaxShift], fy[kMaxShift];
  int hflag;               // helper protocol: result of thread 0's wait
  unsigned long long hp;   // helper protocol: the published word thread 0 read
};

// Single-shift QR on the n x n block B (LDS, row-major) until all its
// eigenvalues are deflated, full Schur form of the block.  If Q is not null
// the rotations are accumulated, Q <- Q G^H.  Returns false when the sweep
// limit is hit.  Run by the first wavefront only (threads 0..63).
__device__ bool lds_qr(c128* B, c128* Q, int n, QRShared& S) {
  constexpr int NT = 64;
  const int t = threadIdx.x;
  // a block whose eigenvalues only serve as shifts (no Q) is deflated at a
  // relative 1e-7: the sweeps converge as fast with shifts that close, and
  // the shift QR takes fewer iterations (measured at 8 x 450: 1e-10 112 ms,
  // 1e-7 108 ms, 1e-5 110 ms per call, the last from slower sweeps)
  const double ulp = Q ? 2.220446049250313e-16 : 1e-7;
  int ihi = n - 1;
  int total = 0;
  const int maxsweeps = 40 * n + 40;
  if (t == 0) S.iter = 0;
  wave_sync();
  while (ihi > 0) {
    if (t == 0) {
      int l = ihi;
      while (l > 0) {
        double tst = cabs1(B[(l - 1) * n + l - 1]) + cabs1(B[l * n + l]);
        if (tst == 0.0) tst = 1.0;
        if (cabs1(B[l * n + l - 1]) <= ulp * tst) break;
        --l;
      }
      if (l > 0) B[l * n + l - 1] = c128{0.0, 0.0};
      S.lo = l;
      if (l < ihi) {
        S.iter += 1;
        c128 mu;
        if (S.iter % 11 == 10) {
          mu = B[ihi * n + ihi] + c128{0.75 * cabs1(B[ihi * n + ihi - 1]), 0.0};
        } else {
          mu = wilkinson(B[(ihi - 1) * n + ihi - 1], B[(ihi - 1) * n + ihi], B[ihi * n + ihi - 1], B[ihi * n + ihi]);
        }
        double c; c128 s;
        givens(B[l * n + l] - mu, B[(l + 1) * n + l], c, s);
        S.rc[0] = c;
        S.rs[0] = s;
      } else {
        S.iter = 0;
      }
    }
    wave_sync();
    const int l = S.lo;
    if (l == ihi) { --ihi; continue; }
    if (++total > maxsweeps) return false;
    c128 bx{0.0, 0.0}, by{0.0, 0.0};  // thread 0: values the current rotation came from
    for (int k = l; k < ihi; ++k) {
      const int slot = (k - l) & 1;
      const double c = S.rc[slot];
      const c128 s = S.rs[slot];
      const int imax = min(k + 2, ihi);
      if (t == 0) {
        // column k-1 (rows k, k+1): becomes (r, 0)
        if (k > l) {
          B[k * n + k - 1] = c * bx + s * by;
          B[(k + 1) * n + k - 1] = c128{0.0, 0.0};
        }
        // 2 x 2 block rows k..k+1, cols k..k+1: left then right
        c128 a = B[k * n + k], b = B[k * n + k + 1], cc = B[(k + 1) * n + k], d = B[(k + 1) * n + k + 1];
        c128 a1 = c * a + s * cc, b1 = c * b + s * d;
        c128 c1 = c * cc - conj(s) * a, d1 = c * d - conj(s) * b;
        B[k * n + k] = c * a1 + conj(s) * b1;
        B[k * n + k + 1] = c * b1 - s * a1;
        const c128 nx = c * c1 + conj(s) * d1;
        B[(k + 1) * n + k] = nx;
        B[(k + 1) * n + k + 1] = c * d1 - s * c1;
        // row k+2 (right rotation only): creates the bulge
        if (k + 2 <= imax) {
          const c128 e = B[(k + 2) * n + k], f = B[(k + 2) * n + k + 1];
          const c128 ny = c * e + conj(s) * f;
          B[(k + 2) * n + k] = ny;
          B[(k + 2) * n + k + 1] = c * f - s * e;
          if (k + 1 < ihi) {
            double c2; c128 s2;
            givens(nx, ny, c2, s2);
            S.rc[slot ^ 1] = c2;
            S.rs[slot ^ 1] = s2;
            bx = nx;
            by = ny;
          }
        }
      } else {
        // left: rows k, k+1, columns k+2 .. n-1; right: rows 0 .. k-1 (rows
        // k..k+2 are thread 0's).  Without Q only eigenvalues are wanted, so
        // the rotations stay inside the active block [l, ihi].
        const int cend = Q ? n : ihi + 1;
        const int rbeg = Q ? 0 : l;
        const int nl = max(0, cend - (k + 2));
        const int nr = k - rbeg;
        const int nq = Q ? n : 0;
        for (int it = t - 1; it < nl + nr + nq; it += NT - 1) {
          if (it < nl) {
            const int j = k + 2 + it;
            const c128 u = B[k * n + j], v = B[(k + 1) * n + j];
            B[k * n + j] = c * u + s * v;
            B[(k + 1) * n + j] = c * v - conj(s) * u;
          } else if (it < nl + nr) {
            const int i = rbeg + it - nl;
            const c128 u = B[i * n + k], v = B[i * n + k + 1];
            B[i * n + k] = c * u + conj(s) * v;
            B[i * n + k + 1] = c * v - s * u;
          } else {
            const int i = it - nl - nr;
            const c128 u = Q[i * n + k], v = Q[i * n + k + 1];
            Q[i * n + k] = c * u + conj(s) * v;
            Q[i * n + k + 1] = c * v - s * u;
          }
        }
      }
      wave_sync();
    }
  }
  return true;
}

// Y[rows, blk] = Y[rows, blk] Q for rows r0 <= r < r1 of a row-major matrix
// with leading dimension ld; blk = [c0, c0+n).  Q in LDS (n x n).
__device__ void apply_right(c128* Y, int64_t ld, int r0, int r1, int c0, const c128* Q, int n) {
  const int t = threadIdx.x;
  const int per = max(1, kQT / n);  // rows per pass
  for (int rb = r0; rb < r1; rb += per) {
    const int r = rb + t / n, j = t % n;
    c128 acc{0.0, 0.0};
    const bool ok = (t < per * n) && r < r1;
    if (ok) {
      const c128* row = Y + int64_t(r) * ld + c0;
      for (int p = 0; p < n; ++p) fma_acc(acc, row[p], Q[p * n + j]);
    }
    __syncthreads();
    if (ok) Y[int64_t(r) * ld + c0 + j] = acc;
    __syncthreads();
  }
}

// Y[blk, cols] = Q^H Y[blk, cols] for columns c0 <= col < c1; blk = [r0, r0+n).
__device__ void apply_left(c128* Y, int64_t ld, int r0, int c0, int c1, const c128* Q, int n) {
  const int t = threadIdx.x;
  const int per = max(1, kQT / n);
  for (int cb = c0; cb < c1; cb += per) {
    const int col = cb + t / n, i = t % n;
    c128 acc{0.0, 0.0};
    const bool ok = (t < per * n) && col < c1;
    if (ok) {
      for (int p = 0; p < n; ++p) fma_cacc(acc, Q[p * n + i], Y[int64_t(r0 + p) * ld + col]);
    }
    __syncthreads();
    if (ok) Y[int64_t(r0 + i) * ld + col] = acc;
    __syncthreads();
  }
}

// Applies one logged rotation to a row of Z (length m).
__device__ inline void replay_rot(c128* row, const RotRec& R) {
  const int p = R.p;
  const c128 u = row[p], v = row[p + 1];
  row[p] = R.c * u + conj(R.s) * v;
  row[p + 1] = R.c * v - R.s * u;
}

// Outputs j, j + kShifts, ... of row[lo : lo+n] Q for a logged Q block
// (the caller stores them with qstore_row after a barrier).
__device__ inline void qblock_row(const c128* row, const RotRec& R0, const c128* qs, int j,
                                  c128 (&acc)[kQAcc]) {
  const int lo = int(R0.c), n = int(R0.s.re);
  const c128* Q = qs + int64_t(R0.s.im);
#pragma unroll
  for (int q = 0; q < kQAcc; ++q) {
    const int jj = j + q * kShifts;
    c128 a{0.0, 0.0};
    if (jj < n)
      for (int pp = 0; pp < n; ++pp) fma_acc(a, row[lo + pp], Q[pp * n + jj]);
    acc[q] = a;
  }
}

__device__ inline void qstore_row(c128* row, const RotRec& R0, int j, const c128 (&acc)[kQAcc]) {
  const int lo = int(R0.c), n = int(R0.s.re);
#pragma unroll
  for (int q = 0; q < kQAcc; ++q) {
    const int jj = j + q * kShifts;
    if (jj < n) row[lo + jj] = acc[q];
  }
}

// The chase's own replay of its log onto every row of Z (global memory),
// used only when the log is full; kQT / kShifts rows at a time, lane j of a
// row applying record j of each step.
__device__ __attribute__((noinline)) void flush_log(c128* Z, int m, const RotRec* rec, int nstep, const c128* qs) {
  const int t = threadIdx.x, j = t % kShifts;
  constexpr int kRows = kQT / kShifts;  // rows per pass; threads beyond kRows * kShifts idle
  for (int r0 = 0; r0 < m; r0 += kRows) {
    const int r = t < kRows * kShifts ? r0 + t / kShifts : m;
    c128* row = Z + int64_t(min(r, m - 1)) * m;
    for (int st = 0; st < nstep; ++st) {
      const RotRec* R = rec + int64_t(st) * kShifts;
      if (R[1].pad & kDeferredStep) continue;  // uniform: the helpers did it
      if (R[0].p <= -2) {
        c128 acc[kQAcc];
        if (r < m) qblock_row(row, R[0], qs, j, acc);
        __syncthreads();
        if (r < m) qstore_row(row, R[0], j, acc);
      } else {
        const RotRec Rj = R[j];
        if (r < m && Rj.p >= 0) replay_rot(row, Rj);
      }
      __syncthreads();
    }
  }
}

// Applies one logged left rotation to a column of H (held with stride cs).
__device__ inline void replay_rot_col(c128* col, int cs, const RotRec& R) {
  const int p = R.p;
  const c128 u = col[int64_t(p) * cs], v = col[int64_t(p + 1) * cs];
  col[int64_t(p) * cs] = R.c * u + R.s * v;
  col[int64_t(p + 1) * cs] = R.c * v - conj(R.s) * u;
}

// Outputs i = j, j + kShifts, ... of Q^H col[lo : lo+n] for a logged Q block
// (stored by qstore_col after a barrier).
__device__ inline void qblock_col(const c128* col, int cs, const RotRec& R0, const c128* qs, int j,
                                  c128 (&acc)[kQAcc]) {
  const int lo = int(R0.c), n = int(R0.s.re);
  const c128* Q = qs + int64_t(R0.s.im);
#pragma unroll
  for (int q = 0; q < kQAcc; ++q) {
    const int ii = j + q * kShifts;
    c128 a{0.0, 0.0};
    if (ii < n)
      for (int pp = 0; pp < n; ++pp) fma_cacc(a, Q[pp * n + ii], col[int64_t(lo + pp) * cs]);
    acc[q] = a;
  }
}

__device__ inline void qstore_col(c128* col, int cs, const RotRec& R0, int j, const c128 (&acc)[kQAcc]) {
  const int lo = int(R0.c), n = int(R0.s.re);
#pragma unroll
  for (int q = 0; q < kQAcc; ++q) {
    const int ii = j + q * kShifts;
    if (ii < n) col[int64_t(lo + ii) * cs] = acc[q];
  }
}

// The chase's own replay of the deferred left transformations onto the
// columns of H (global memory), used only when the log is full: column c
// takes the records whose ihi is below c.
__device__ __attribute__((noinline)) void flush_log_cols(c128* H, int m, const RotRec* rec, int nstep, const c128* qs) {
  const int t = threadIdx.x, j = t % kShifts;
  constexpr int kCols = kQT / kShifts;
  for (int c0 = 0; c0 < m; c0 += kCols) {
    const int c = t < kCols * kShifts ? c0 + t / kShifts : m;
    const bool mine = c < m;
    c128* col = H + min(c, m - 1);
    for (int st = 0; st < nstep; ++st) {
      const RotRec* R = rec + int64_t(st) * kShifts;
      if (R[1].pad & kDeferredStep) continue;  // uniform: the helpers did it
      const bool take = mine && R[0].pad < c;
      if (R[0].p <= -2) {
        c128 acc[kQAcc];
        if (take) qblock_col(col, m, R[0], qs, j, acc);
        __syncthreads();
        if (take) qstore_col(col, m, R[0], j, acc);
      } else {
        const RotRec Rj = R[j];
        if (take && Rj.p >= 0) replay_rot_col(col, m, Rj);
      }
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------- helpers
// Each helper owns a band of kHelpBand rows and the band of columns with the
// same indices.  In a sweep that uses them (a deferred sweep):
//   * row r is the helper's from step srow(r) on: all later right rotations
//     of the sweep act on it only above the train;
//   * column c is the helper's before step scol(c): until then the left
//     rotations reach it only to the right of the train.  The chase owns the
//     columns up to e(s) = lo + kTake (s / kTake + 2) at step s, so it takes
//     them back kTake at a time, each block before the train gets near it.
//   * columns beyond ihi and the band's rows of Z take every rotation of the
//     sweep from the helper (left ones, right ones), so the column and Z
//     replays skip the sweep's steps (flagged kDeferredStep).
// The helper replays the logged rotations of each chunk of published steps
// onto the parts of its rows and columns that chunk touches, staged in LDS
// (lane j of a row or column applies record j of each step), and reports the
// steps done.  The chase publishes its records every kPub steps, waits for
// the helpers owning a block of columns before it takes it, and for all of
// them at the end of the sweep.  A helper announces itself when it starts; a sweep is deferred
// only if every helper of the window has, so the chase never waits on a
// workgroup that is not running, and helpers wait only on the chase.  Every
// wait gives up after kSpinTicks (the window then fails with info > 0).
constexpr int kHelpBand = 32;     // rows and columns per helper
constexpr int kMaxHelpers = 64;
constexpr int kHelpChunk = 32;    // steps a helper replays per LDS pass
constexpr int kTake = 32;         // columns the chase takes back at a time
constexpr int kHelpSpan = 3 * (kShifts - 1) + kHelpChunk + 2;  // rows (columns) one pass touches
constexpr int kDeferMin = 128;    // smallest active block whose sweeps are deferred
constexpr int kPub = 8;           // the chase publishes its records every kPub steps
constexpr unsigned long long kSpinTicks = 1000000000ull;  // 10 s of the 100 MHz wall clock
static_assert(2 * kHelpBand * kShifts == kQT, "helper lanes: one band of rows, one of columns");
static_assert(kHelpChunk <= kTake, "a helper's row pass stays left of its deferred columns");
static_assert(kTake % kPub == 0, "the step before each take is published");
// dynamic LDS of the chase kernel: the LDS finish (block and unitary) or a
// helper's staging (records, rows, columns), whichever is larger
constexpr size_t kSchurLds =
    std::max(2 * size_t(kFin) * kFin * sizeof(c128),
             size_t(kHelpChunk) * kShifts * sizeof(RotRec) + 2 * size_t(kHelpBand) * kHelpSpan * sizeof(c128));
static_assert(kSchurLds <= size_t(150) * 1024, "chase LDS");

// Per-window state shared by the chase and its helpers (after the log).
struct ChaseSync {
  unsigned long long pub;                // (sweep << 32) | steps whose records are out
  unsigned long long prog[kMaxHelpers];  // per helper: (sweep << 32) | steps replayed
  int present;                           // helpers running
  int state;                             // 0 chasing, 1 finished, 2 failed
  int lo, ihi, ns, nsteps, s0, pad;      // the current deferred sweep (s0: log index of its step 0)
};
constexpr int64_t kSyncC128 = int64_t((sizeof(ChaseSync) + sizeof(c128) - 1) / sizeof(c128));

__device__ inline unsigned long long ld_agent(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline int ld_agent(const int* p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
__device__ inline void st_agent(unsigned long long* p, unsigned long long v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_agent(int* p, int v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

// Shared data on the helpers' side goes through 64-bit device-coherent
// accesses, so that a helper never has to invalidate its L2 (which is also
// the chase's when both run on one XCD) to see what the chase wrote.
__device__ inline c128 ld_shared(const c128* p) {
  const unsigned long long* q = reinterpret_cast<const unsigned long long*>(p);
  return c128{__longlong_as_double((long long)ld_agent(q)), __longlong_as_double((long long)ld_agent(q + 1))};
}
__device__ inline void st_shared(c128* p, c128 v) {
  unsigned long long* q = reinterpret_cast<unsigned long long*>(p);
  st_agent(q, (unsigned long long)__double_as_longlong(v.re));
  st_agent(q + 1, (unsigned long long)__double_as_longlong(v.im));
}
__device__ inline RotRec ld_shared(const RotRec* p) {
  const unsigned long long* q = reinterpret_cast<const unsigned long long*>(p);
  const unsigned long long a = ld_agent(q), b = ld_agent(q + 1), c = ld_agent(q + 2), d = ld_agent(q + 3);
  RotRec R;
  R.c = __longlong_as_double((long long)a);
  R.p = int(b & 0xffffffffull);
  R.pad = int(b >> 32);
  R.s = c128{__longlong_as_double((long long)c), __longlong_as_double((long long)d)};
  return R;
}

// Every thread's earlier stores have completed (reached the L2), then thread
// 0 writes the L2 back (agent-scope release) and stores v to *p.  Called by
// the whole workgroup.
__device__ inline void publish(unsigned long long* p, unsigned long long v) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this wave's loads and stores are done
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    st_agent(p, v);
  }
}

// Thread 0: polls until done() holds (false after kSpinTicks); with acquire,
// then an agent-scope acquire fence (the chase, before it reads what helpers
// wrote), so that the workgroup sees it once it has passed a barrier.
template <typename F>
__device__ inline bool spin_wait(F done, bool acquire) {
  const unsigned long long start = wall_clock64();
  while (!done()) {
    if (wall_clock64() - start > kSpinTicks) return false;
    __builtin_amdgcn_s_sleep(2);
  }
  if (acquire) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return true;
}

// First step of a deferred sweep from which row r is the helper's.
__device__ inline int helper_srow(int r, int lo, int ns) { return r < lo ? 0 : r - lo + 3 * (ns - 1) + 1; }
// Step at which the chase takes column c back (0: the chase's all sweep).
// A column beyond ihi is never read again, so it takes the whole sweep's
// left rotations from its helper (the column replay skips deferred steps).
__device__ inline int helper_scol(int c, int lo, int ihi) {
  if (c < lo) return 0;
  if (c > ihi) return 0x7fffffff;
  return kTake * max(0, (c - lo + kTake - 1) / kTake - 2);
}

// One pass of helper h over steps [sa, sb) of the deferred sweep: the steps'
// right rotations on its rows and left rotations on its columns, the parts
// they touch ([base, top], by the bulge positions lo + s - 3 j) held in LDS.
__device__ void helper_pass(c128* H, c128* Z, int m, const RotRec* rec, int s0, int lo, int ihi, int ns, int b0,
                            int sa, int sb, c128* lds) {
  const int t = threadIdx.x;
  RotRec* rl = reinterpret_cast<RotRec*>(lds);
  c128* rows = lds + int64_t(kHelpChunk) * kShifts * (sizeof(RotRec) / sizeof(c128));
  c128* cols = rows + kHelpBand * kHelpSpan;
  const int base = max(lo, lo + sa - 3 * (ns - 1));
  const int top = min(ihi, lo + sb);
  const int W = top - base + 1;
  for (int e = t; e < (sb - sa) * kShifts; e += kQT) rl[e] = ld_shared(rec + int64_t(s0 + sa) * kShifts + e);
  for (int e = t; e < 2 * kHelpBand * W; e += kQT) {
    const int side = e / (kHelpBand * W), i = (e / W) % kHelpBand, q = e % W, x = b0 + i;
    if (side == 0) {
      if (x < m && helper_srow(x, lo, ns) < sb) rows[i * kHelpSpan + q] = ld_shared(H + int64_t(x) * m + base + q);
    } else {
      if (x < m && helper_scol(x, lo, ihi) > sa) cols[i * kHelpSpan + q] = ld_shared(H + int64_t(base + q) * m + x);
    }
  }
  __syncthreads();
  {
    const int j = t % kShifts, side = t / (kHelpBand * kShifts), i = (t / kShifts) % kHelpBand, x = b0 + i;
    c128* seg = (side == 0 ? rows : cols) + i * kHelpSpan;
    int s_from = sb, s_to = sb;  // steps this lane's row or column takes
    if (side == 0) {
      if (x < m && helper_srow(x, lo, ns) < sb) s_from = max(sa, helper_srow(x, lo, ns));
    } else if (x < m && helper_scol(x, lo, ihi) > sa) {
      s_from = sa;
      s_to = min(sb, helper_scol(x, lo, ihi));
    }
    for (int s = sa; s < sb; ++s) {
      if (s >= s_from && s < s_to) {
        const RotRec R = rl[(s - sa) * kShifts + j];
        if (R.p >= 0) {
          c128* a = seg + (R.p - base);
          const c128 u = a[0], v = a[1];
          if (side == 0) {  // right rotation, as the chase applies it to rows
            a[0] = R.c * u + conj(R.s) * v;
            a[1] = R.c * v - R.s * u;
          } else {          // left rotation, as the chase applies it to columns
            a[0] = R.c * u + R.s * v;
            a[1] = R.c * v - conj(R.s) * u;
          }
        }
      }
      wave_sync();
    }
  }
  __syncthreads();
  for (int e = t; e < 2 * kHelpBand * W; e += kQT) {
    const int side = e / (kHelpBand * W), i = (e / W) % kHelpBand, q = e % W, x = b0 + i;
    if (side == 0) {
      if (x < m && helper_srow(x, lo, ns) < sb) st_shared(H + int64_t(x) * m + base + q, rows[i * kHelpSpan + q]);
    } else {
      if (x < m && helper_scol(x, lo, ihi) > sa) st_shared(H + int64_t(base + q) * m + x, cols[i * kHelpSpan + q]);
    }
  }
  __syncthreads();
  // the band's rows of Z take every right rotation of the steps (the Z
  // replay skips deferred steps), in the rows' staging
  for (int e = t; e < kHelpBand * W; e += kQT) {
    const int i = e / W, q = e % W, x = b0 + i;
    if (x < m) rows[i * kHelpSpan + q] = ld_shared(Z + int64_t(x) * m + base + q);
  }
  __syncthreads();
  if (t < kHelpBand * kShifts) {
    const int j = t % kShifts, i = t / kShifts;
    c128* seg = rows + i * kHelpSpan;
    const bool on = b0 + i < m;
    for (int s = sa; s < sb; ++s) {
      if (on) {
        const RotRec R = rl[(s - sa) * kShifts + j];
        if (R.p >= 0) {
          c128* a = seg + (R.p - base);
          const c128 u = a[0], v = a[1];
          a[0] = R.c * u + conj(R.s) * v;
          a[1] = R.c * v - R.s * u;
        }
      }
      wave_sync();
    }
  }
  __syncthreads();
  for (int e = t; e < kHelpBand * W; e += kQT) {
    const int i = e / W, q = e % W, x = b0 + i;
    if (x < m) st_shared(Z + int64_t(x) * m + base + q, rows[i * kHelpSpan + q]);
  }
  __syncthreads();
}

// Helper h of a window: announces itself, then serves every deferred sweep
// the chase publishes until the chase has finished (or a wait gives up).
__device__ void chase_helper(c128* H, c128* Z, int m, const RotRec* rec, ChaseSync* sy, int h, QRShared& S,
                             c128* lds) {
  const int t = threadIdx.x;
  if (t == 0) __hip_atomic_fetch_add(&sy->present, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  unsigned long long seen = 0;  // last sweep served
  for (;;) {
    if (t == 0) {
      unsigned long long p = 0;
      int st = 0;
      const bool ok = spin_wait([&] {
        p = ld_agent(&sy->pub);
        st = ld_agent(&sy->state);
        return (p >> 32) > seen || st != 0;
      }, false);
      if (!ok) st_agent(&sy->state, 2);
      S.hp = p;
      S.hflag = (ok && (p >> 32) > seen) ? 0 : 1;
    }
    __syncthreads();
    const int stop = S.hflag;
    const unsigned long long p0 = S.hp;
    __syncthreads();
    if (stop) return;
    seen = p0 >> 32;
    const int lo = ld_agent(&sy->lo), ihi = ld_agent(&sy->ihi), ns = ld_agent(&sy->ns);
    const int nsteps = ld_agent(&sy->nsteps), s0 = ld_agent(&sy->s0);
    int done = 0, avail = int(p0 & 0xffffffffull);
    while (done < nsteps) {
      if (avail <= done) {
        if (t == 0) {
          unsigned long long p = 0;
          int st = 0;
          const bool ok = spin_wait([&] {
            p = ld_agent(&sy->pub);
            st = ld_agent(&sy->state);
            return (p >> 32) != seen || int(p & 0xffffffffull) > done || st != 0;
          }, false);
          if (!ok) st_agent(&sy->state, 2);
          S.hp = p;
          S.hflag = (ok && (p >> 32) == seen && int(p & 0xffffffffull) > done) ? 0 : 1;
        }
        __syncthreads();
        const int bad = S.hflag;
        avail = int(S.hp & 0xffffffffull);
        __syncthreads();
        if (bad) return;
      }
      for (int sa = done; sa < avail; sa += kHelpChunk)
        helper_pass(H, Z, m, rec, s0, lo, ihi, ns, h * kHelpBand, sa, min(avail, sa + kHelpChunk), lds);
      done = avail;
      publish(&sy->prog[h], (seen << 32) | (unsigned long long)(unsigned)done);
    }
  }
}

// Clears each window's ChaseSync before the chase (a kernel, not a memset, so
// that the sequence can be captured in a graph).
__global__ void chase_sync_init_kernel(c128* logall, int64_t wsl, int m, const int* __restrict__ wmap) {
  const int w = wmap ? wmap[blockIdx.x] : blockIdx.x;
  if (w < 0) return;
  c128* z = logall + int64_t(w) * wsl + log_sync_offset(m);
  for (int64_t e = threadIdx.x; e < kSyncC128; e += blockDim.x) z[e] = c128{0.0, 0.0};
}

__global__ __launch_bounds__(kQT) void schur_kernel(c128* Hall, int64_t wsh, int m, c128* Zall, int64_t wsz,
                                                    c128* logall, int64_t wsl, int64_t cap, c128* theta, int64_t wst,
                                                    int* info, const int* __restrict__ wmap, int prof,
                                                    int nshift_max, int nh) {
  extern __shared__ c128 lds[];  // B (kFin^2) and Q (kFin^2), or a helper's staging
  __shared__ QRShared S;
  // role-major: the chases of all window slots, then helper 0 of each, ...
  // (consecutive workgroups go to consecutive XCDs, so with 8 slots a chase
  // and its helpers share one XCD and each chase has an L2 of its own)
  const int nslot = int(gridDim.x) / (1 + nh);
  const int slot = int(blockIdx.x) % nslot, role = int(blockIdx.x) / nslot;
  const int w = wmap ? wmap[slot] : slot;
  if (w < 0) return;  // idle slot (whole workgroup)
  c128* H = Hall + int64_t(w) * wsh;
  c128* Z = Zall + int64_t(w) * wsz;
  c128* th = theta + int64_t(w) * wst;
  c128* lg = logall + int64_t(w) * wsl;
  RotRec* rec = reinterpret_cast<RotRec*>(lg + 2);
  c128* qs = lg + log_qstore_offset(m);
  ChaseSync* sy = reinterpret_cast<ChaseSync*>(lg + log_sync_offset(m));
  if (role > 0) {
    chase_helper(H, Z, m, rec, sy, role - 1, S, lds);
    return;
  }
  // the Hessenberg step leaves its reflectors below the subdiagonal
  for (int64_t e = threadIdx.x; e < int64_t(m) * m; e += kQT)
    if (e / m > e % m + 1) H[e] = c128{0.0, 0.0};
  __syncthreads();
  int nstep = 0, nq = 0;  // steps logged, Q store entries used: the same in every thread
  bool nd_log = false;    // the log holds steps of a sweep without helpers on a block of >= kDeferMin rows
  auto make_room = [&](int qneed) {
    if (nstep < cap && nq + qneed <= kQCap) return;
    __syncthreads();
    flush_log(Z, m, rec, nstep, qs);
    flush_log_cols(H, m, rec, nstep, qs);
    nstep = 0;
    nq = 0;
    nd_log = false;
  };
  const int t = threadIdx.x;
  const double ulp = 2.220446049250313e-16;
  int ihi = m - 1;
  int sweeps = 0;
  unsigned long long dsweep = 0;  // deferred sweeps published
  const int maxsweeps = 20 * m + 20;
  bool failed = false;
  unsigned long long tp = wall_clock64();
  auto tick = [&](int slot) {
    if (prof && t == 0) {
      const unsigned long long now = wall_clock64();
      atomicAdd(&g_k4prof[slot], now - tp);
      tp = now;
    }
  };
  while (ihi >= 0) {
    // deflation scan: largest l in (0, ihi] with a negligible subdiagonal
    int best = 0;
    for (int l = 1 + t; l <= ihi; l += kQT) {
      double tst = cabs1(H[int64_t(l - 1) * m + l - 1]) + cabs1(H[int64_t(l) * m + l]);
      if (tst == 0.0) tst = 1.0;
      if (cabs1(H[int64_t(l) * m + l - 1]) <= ulp * tst) best = max(best, l);
    }
    S.ired[t] = best;
    __syncthreads();
    for (int o = kQT / 2; o > 0; o >>= 1) {
      if (t < o) S.ired[t] = max(S.ired[t], S.ired[t + o]);
      __syncthreads();
    }
    const int lo = S.ired[0];
    __syncthreads();
    tick(0);
    if (lo > 0 && t == 0) H[int64_t(lo) * m + lo - 1] = c128{0.0, 0.0};
    const int n = ihi - lo + 1;
    if (n == 1) {
      if (t == 0) th[ihi] = H[int64_t(ihi) * m + ihi];
      ihi -= 1;
      __syncthreads();
      continue;
    }
    if (n <= kFin) {
      // finish the block in LDS
      c128* B = lds;
      c128* Q = lds + kFin * kFin;
      for (int e = t; e < n * n; e += kQT) {
        const int i = e / n, j = e % n;
        B[e] = H[int64_t(lo + i) * m + lo + j];
        Q[e] = c128{i == j ? 1.0 : 0.0, 0.0};
      }
      __syncthreads();
      if (t < 64) {
        const bool ok = lds_qr(B, Q, n, S);
        if (t == 0) S.flag = ok ? 0 : 1;
      }
      __syncthreads();
      tick(5);
      if (S.flag) failed = true;
      for (int e = t; e < n * n; e += kQT) {
        const int i = e / n, j = e % n;
        H[int64_t(lo + i) * m + lo + j] = B[e];
      }
      for (int i = t; i < n; i += kQT) th[lo + i] = B[i * n + i];
      make_room(n * n);
      {
        c128* Qd = qs + nq;
        for (int e = t; e < n * n; e += kQT) Qd[e] = Q[e];
        if (t < kShifts) {
          RotRec R;
          R.c = t == 0 ? double(lo) : 0.0;
          R.p = t == 0 ? -2 : -1;
          R.pad = ihi;
          R.s = c128{t == 0 ? double(n) : 0.0, t == 0 ? double(nq) : 0.0};
          rec[int64_t(nstep) * kShifts + t] = R;
        }
        ++nstep;
        nq += n * n;
      }
      __syncthreads();
      apply_right(H, m, 0, lo, lo, Q, n);
      // columns beyond the block take Q^H in the column replay
      tick(6);
      ihi = lo - 1;
      __syncthreads();
      continue;
    }
    if (++sweeps > maxsweeps) { failed = true; break; }
    // shifts: eigenvalues of the trailing ns x ns block (in LDS)
    const int ns = min(nshift_max, max(2, n / 3));
    {
      c128* B = lds;
      const int b0 = ihi - ns + 1;
      for (int e = t; e < ns * ns; e += kQT) {
        const int i = e / ns, j = e % ns;
        B[e] = H[int64_t(b0 + i) * m + b0 + j];
      }
      __syncthreads();
      if (t < 64) {
        const bool ok = lds_qr(B, nullptr, ns, S);
        if (t == 0) S.flag = ok ? 0 : 1;
      }
      __syncthreads();
      const bool ok = S.flag == 0;
      if (t < ns) S.shift[t] = ok ? B[t * ns + t] : H[int64_t(b0 + t) * m + b0 + t];
      if (t == 0 && sweeps % 6 == 5) {
        // occasional exceptional shift against stagnation
        S.shift[0] = H[int64_t(ihi) * m + ihi] + c128{0.75 * cabs1(H[int64_t(ihi) * m + ihi - 1]), 0.0};
      }
      __syncthreads();
      tick(1);
    }
    // pipelined chase: bulge j sits at position lo + step - 3 j
    const int nsteps = (ihi - lo) + 3 * (ns - 1);
    // defer the sweep's far updates to the helpers if all of them are
    // running and the log holds the whole sweep (they address it by index)
    bool defer = false, aborted = false;
    if (nh > 0 && n >= kDeferMin && cap >= nsteps) {
      // the log must hold the whole sweep; and steps of sweeps without
      // helpers still pending for the column replay are applied first, so
      // that every column beyond ihi takes its rotations in log order
      if (nstep + nsteps > cap || nq > kQCap || nd_log) {
        __syncthreads();
        flush_log(Z, m, rec, nstep, qs);
        flush_log_cols(H, m, rec, nstep, qs);
        nstep = 0;
        nq = 0;
        nd_log = false;
      }
      if (t == 0) S.hflag = ld_agent(&sy->present) == nh ? 1 : 0;
      __syncthreads();
      defer = S.hflag != 0;
      __syncthreads();
    }
    if (defer) {
      ++dsweep;
      if (t == 0) {
        st_agent(&sy->lo, lo);
        st_agent(&sy->ihi, ihi);
        st_agent(&sy->ns, ns);
        st_agent(&sy->nsteps, nsteps);
        st_agent(&sy->s0, nstep);
      }
      publish(&sy->pub, dsweep << 32);
    }
    for (int step = 0; step < nsteps; ++step) {
      if (!defer) make_room(0);
      if (t < ns) {
        const int p = lo + step - 3 * t;
        if (p >= lo && p < ihi) {
          c128 x, y;
          if (p == lo) {
            x = H[int64_t(lo) * m + lo] - S.shift[t];
            y = H[int64_t(lo + 1) * m + lo];
          } else {
            // H[p][p-1] and H[p+1][p-1], forwarded by the previous step's
            // right phase (the same values it stored to H)
            x = S.fx[t];
            y = S.fy[t];
          }
          double c; c128 s;
          givens(x, y, c, s);
          S.bc[t] = c;
          S.bs[t] = s;
          S.bp[t] = p;
        } else {
          S.bp[t] = -1;
        }
      }
      __syncthreads();
      if (t < kShifts) {
        RotRec R;
        R.c = t < ns ? S.bc[t] : 1.0;
        R.p = t < ns ? S.bp[t] : -1;
        R.pad = (defer && t == 1) ? (ihi | kDeferredStep) : ihi;
        R.s = t < ns ? S.bs[t] : c128{0.0, 0.0};
        rec[int64_t(nstep) * kShifts + t] = R;
      }
      ++nstep;
      // a sweep without helpers on a block the helpers could have taken: a
      // later deferred sweep of the same block overlaps it (blocks below
      // 128 rows never are: lo only grows within a block, and later blocks
      // lie above it, so their rotations act on other rows and columns)
      if (!defer && n >= kDeferMin) nd_log = true;
      // columns up to ecol are the chase's at this step; in a deferred sweep
      // it takes the next kTake of them from the helpers every kTake steps
      int ecol = ihi;
      if (defer) {
        if ((step + 1) % kPub == 0 || step + 1 == nsteps)
          publish(&sy->pub, (dsweep << 32) | (unsigned long long)(unsigned)(step + 1));
        ecol = min(ihi, lo + kTake * (step / kTake + 2));
        const int cfirst = lo + kTake * (step / kTake + 1) + 1;
        if (step > 0 && step % kTake == 0 && cfirst <= ecol) {
          if (t == 0) {
            const unsigned long long need = (dsweep << 32) | (unsigned long long)(unsigned)step;
            const bool ok = spin_wait([&] {
              for (int hh = cfirst / kHelpBand; hh <= ecol / kHelpBand; ++hh)
                if (ld_agent(&sy->prog[hh]) < need) return false;
              return true;
            }, true);
            S.hflag = ok ? 0 : 1;
          }
          __syncthreads();
          aborted = S.hflag != 0;
          __syncthreads();
          if (aborted) break;
        }
      }
      tick(2);
      // active bulges form the contiguous range [ja, jb]
      // bulge j is at p = lo + step - 3 j, active while lo <= p <= ihi - 1
      const int dd = step - (ihi - 1 - lo);
      const int ja = dd > 0 ? (dd + 2) / 3 : 0;
      const int jb = min(ns - 1, step / 3);
      const int nact = jb >= ja ? jb - ja + 1 : 0;
      // all left rotations: rows p, p+1, columns from max(p-1, lo) to m-1.
      // Items (bulge, column), column fastest, over the columns from the
      // last active bulge's first one (no bulge starts further left); each
      // thread loads a batch of independent items before storing any.
      {
        const int cstart = nact > 0 ? max(lo + step - 3 * jb - 1, lo) : lo;
        // columns beyond ihi are left to the column replay, those beyond
        // ecol to the helpers
        const int W = max(0, ecol + 1 - cstart);
        const int total = nact * W;
        for (int base = t; base < total; base += kQT * kBatch) {
          // every item loads (a skipped one from H's first elements) so that
          // the batch's loads are all in flight before the first is used
          c128 av[kBatch], bv[kBatch];
          int pr[kBatch], cl[kBatch], pp[kBatch];
#pragma unroll
          for (int q = 0; q < kBatch; ++q) {
            const int idx = base + q * kQT;
            const bool in = idx < total;
            const int j = in ? ja + idx / W : ja;
            const int col = in ? cstart + idx % W : lo;
            const int p = in ? S.bp[j] : -1;
            const int c0 = (p > lo) ? p - 1 : lo;
            const bool ok = p >= 0 && col >= c0;
            pr[q] = ok ? j : -1;
            pp[q] = ok ? p : 0;
            cl[q] = ok ? col : 0;
            av[q] = H[int64_t(pp[q]) * m + cl[q]];
            bv[q] = H[int64_t(pp[q] + 1) * m + cl[q]];
          }
#pragma unroll
          for (int q = 0; q < kBatch; ++q) {
            if (pr[q] < 0) continue;
            const int j = pr[q], p = pp[q], col = cl[q];
            const double c = S.bc[j];
            const c128 sj = S.bs[j];
            H[int64_t(p) * m + col] = c * av[q] + sj * bv[q];
            H[int64_t(p + 1) * m + col] = (col == p - 1) ? c128{0.0, 0.0} : c * bv[q] - conj(sj) * av[q];
          }
        }
      }
      __syncthreads();
      tick(3);
      // all right rotations: columns p, p+1 of H for rows 0..min(p+2, ihi)
      // (Z gets them from the log).  Items (row, bulge), bulge fastest:
      // neighbouring lanes touch nearby column pairs of one row.
      {
        // rows below the deepest active bulge's last one are untouched
        const int Rh = nact > 0 ? min(lo + step - 3 * ja + 2, ihi) + 1 : 0;
        // in a deferred sweep the rows above the topmost bulge are the helpers'
        const int rlo = defer ? max(lo, lo + step - 3 * (ns - 1)) : 0;
        const int total = max(0, Rh - rlo) * nact;
        for (int base = t; base < total; base += kQT * kBatch) {
          // every item loads (a skipped one from H's first elements) so that
          // the batch's loads are all in flight before the first is used
          c128 av[kBatch], bv[kBatch];
          c128* ap[kBatch];
          int pr[kBatch];  // bulge + kMaxShift * (r - p if 1 or 2, else 0); -1: skipped
#pragma unroll
          for (int q = 0; q < kBatch; ++q) {
            const int idx = base + q * kQT;
            const bool in = idx < total;
            const int r = in ? rlo + idx / nact : 0;
            const int j = in ? ja + idx % nact : ja;
            const int p = in ? S.bp[j] : -1;
            const bool ok = p >= 0 && r <= min(p + 2, ihi);
            const int fwd = (r - p == 1 || r - p == 2) ? r - p : 0;
            pr[q] = ok ? j + kMaxShift * fwd : -1;
            ap[q] = ok ? H + int64_t(r) * m + p : H;
            av[q] = ap[q][0];
            bv[q] = ap[q][1];
          }
#pragma unroll
          for (int q = 0; q < kBatch; ++q) {
            if (pr[q] < 0) continue;
            const int j = pr[q] % kMaxShift, fwd = pr[q] / kMaxShift;
            const double c = S.bc[j];
            const c128 sj = S.bs[j];
            const c128 n0 = c * av[q] + conj(sj) * bv[q];
            ap[q][0] = n0;
            ap[q][1] = c * bv[q] - sj * av[q];
            if (fwd == 1) S.fx[j] = n0;
            else if (fwd == 2) S.fy[j] = n0;
          }
        }
      }
      __syncthreads();
      tick(4);
      if (prof && t == 0) atomicAdd(&g_k4prof[7], 1ull);
    }
    if (defer && !aborted) {
      // the helpers' rows and columns are needed from here on
      if (t == 0) {
        const unsigned long long need = (dsweep << 32) | (unsigned long long)(unsigned)nsteps;
        const bool ok = spin_wait([&] {
          for (int hh = 0; hh < nh; ++hh)
            if (ld_agent(&sy->prog[hh]) < need) return false;
          return true;
        }, true);
        S.hflag = ok ? 0 : 1;
      }
      __syncthreads();
      aborted = S.hflag != 0;
      __syncthreads();
    }
    if (aborted) { failed = true; break; }
  }
  if (t == 0) {
    info[w] = failed ? max(ihi + 1, 1) : 0;
    int* hdr = reinterpret_cast<int*>(lg);
    hdr[0] = nstep;
    hdr[1] = nq;
    st_agent(&sy->state, failed ? 2 : 1);  // releases the helpers
  }
  if (failed) {
    for (int i = t; i <= ihi; i += kQT) th[i] = H[int64_t(i) * m + i];
  }
}

// Replays a window's log onto rows [r0, r0 + rows) of Z, held in LDS; the
// step records are staged through LDS in chunks of kChunk steps.  Lane j of
// a row applies record j of each step.
constexpr int kChunk = 32;

__global__ __launch_bounds__(256) void zreplay_kernel(c128* Zall, int64_t wsz, int m, const c128* __restrict__ logall,
                                                     int64_t wsl, int rows, const int* __restrict__ wmap) {
  extern __shared__ c128 zl[];  // rows x m, then kChunk x kShifts records
  const int w = wmap ? wmap[blockIdx.y] : blockIdx.y;
  if (w < 0) return;
  const int r0 = int(blockIdx.x) * rows;
  if (r0 >= m) return;
  const int nr = min(rows, m - r0);
  c128* Z = Zall + int64_t(w) * wsz;
  const c128* lg = logall + int64_t(w) * wsl;
  const int nstep = reinterpret_cast<const int*>(lg)[0];
  const RotRec* rec = reinterpret_cast<const RotRec*>(lg + 2);
  const c128* qs = lg + log_qstore_offset(m);
  RotRec* chunk = reinterpret_cast<RotRec*>(zl + int64_t(rows) * m);
  const int t = threadIdx.x, nt = blockDim.x, j = t % kShifts, r = t / kShifts;
  for (int e = t; e < nr * m; e += nt) zl[e] = Z[int64_t(r0) * m + e];
  c128* row = zl + int64_t(min(r, nr - 1)) * m;
  const bool mine = r < nr;
  for (int c0 = 0; c0 < nstep; c0 += kChunk) {
    const int nc = min(kChunk, nstep - c0);
    __syncthreads();
    for (int e = t; e < nc * kShifts; e += nt) chunk[e] = rec[int64_t(c0) * kShifts + e];
    __syncthreads();
    for (int st = 0; st < nc; ++st) {
      const RotRec* R = chunk + st * kShifts;
      if (R[1].pad & kDeferredStep) continue;  // uniform: the helpers did it
      if (R[0].p <= -2) {
        c128 acc[kQAcc];
        if (mine) qblock_row(row, R[0], qs, j, acc);
        __syncthreads();
        if (mine) qstore_row(row, R[0], j, acc);
      } else {
        const RotRec Rj = R[j];
        if (mine && Rj.p >= 0) replay_rot(row, Rj);
      }
      __syncthreads();
    }
  }
  __syncthreads();
  for (int e = t; e < nr * m; e += nt) Z[int64_t(r0) * m + e] = zl[e];
}

// Replays a window's deferred left transformations onto columns
// [c0, c0 + cols) of H, held in LDS (m x cols, row-major); column c takes
// the records whose ihi is below c.  Lane j of a column applies record j of
// each step; steps before the first one that concerns the band are skipped
// (ihi never increases along the log).
__global__ __launch_bounds__(256) void hreplay_kernel(c128* Hall, int64_t wsh, int m, const c128* __restrict__ logall,
                                                     int64_t wsl, int cols, const int* __restrict__ wmap) {
  extern __shared__ c128 hl[];  // m x cols, then kChunk x kShifts records
  const int w = wmap ? wmap[blockIdx.y] : blockIdx.y;
  if (w < 0) return;
  const int c0 = int(blockIdx.x) * cols;
  if (c0 >= m) return;
  const int nc = min(cols, m - c0);
  c128* H = Hall + int64_t(w) * wsh;
  const c128* lg = logall + int64_t(w) * wsl;
  const int nstep = reinterpret_cast<const int*>(lg)[0];
  const RotRec* rec = reinterpret_cast<const RotRec*>(lg + 2);
  const c128* qs = lg + log_qstore_offset(m);
  RotRec* chunk = reinterpret_cast<RotRec*>(hl + int64_t(m) * cols);
  const int t = threadIdx.x, nt = blockDim.x, j = t % kShifts, cc = t / kShifts;
  // first step whose ihi is below the band's last column
  int s0 = nstep;
  {
    int lo = 0, hi = nstep;
    const int cmax = c0 + nc - 1;
    while (lo < hi) {
      const int mid = (lo + hi) / 2;
      if (rec[int64_t(mid) * kShifts].pad < cmax) hi = mid; else lo = mid + 1;
    }
    s0 = lo;
  }
  if (s0 >= nstep) return;
  for (int e = t; e < m * nc; e += nt) {
    const int i = e / nc, q = e % nc;
    hl[int64_t(i) * cols + q] = H[int64_t(i) * m + c0 + q];
  }
  const int c = c0 + min(cc, nc - 1);
  c128* col = hl + min(cc, nc - 1);
  const bool mine = cc < nc;
  for (int b0 = s0; b0 < nstep; b0 += kChunk) {
    const int n = min(kChunk, nstep - b0);
    __syncthreads();
    for (int e = t; e < n * kShifts; e += nt) chunk[e] = rec[int64_t(b0) * kShifts + e];
    __syncthreads();
    for (int st = 0; st < n; ++st) {
      const RotRec* R = chunk + st * kShifts;
      if (R[1].pad & kDeferredStep) continue;  // uniform: the helpers did it
      const bool take = mine && R[0].pad < c;
      if (R[0].p <= -2) {
        c128 acc[kQAcc];
        if (take) qblock_col(col, cols, R[0], qs, j, acc);
        __syncthreads();
        if (take) qstore_col(col, cols, R[0], j, acc);
      } else {
        const RotRec Rj = R[j];
        if (take && Rj.p >= 0) replay_rot_col(col, cols, Rj);
      }
      __syncthreads();
    }
  }
  __syncthreads();
  for (int e = t; e < m * nc; e += nt) {
    const int i = e / nc, q = e % nc;
    H[int64_t(i) * m + c0 + q] = hl[int64_t(i) * cols + q];
  }
}

}  // namespace

size_t schur_lds_bytes() { return kSchurLds; }

int64_t schur_log_size(int m) { return log_sync_offset(m) + kSyncC128; }

void launch_schur(c128* H, int64_t wsh, int m, c128* Z, int64_t wsz, c128* log, int64_t wsl, c128* theta,
                  int64_t wst, int* info, int nwin, hipStream_t st, const int* wmap) {
  static const int prof = [] { const char* v = std::getenv("TSG_K4PROF"); return (v && v[0] == '1') ? 1 : 0; }();
  if (prof) {
    unsigned long long z[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    (void)hipMemcpyToSymbolAsync(HIP_SYMBOL(g_k4prof), z, sizeof(z), 0, hipMemcpyHostToDevice, st);
  }
  static bool attr_set = false;
  if (!attr_set) {
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(schur_kernel),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, int(schur_lds_bytes()));
    if (e != hipSuccess) throw DeviceError(std::string("schur: LDS attribute: ") + hipGetErrorString(e));
    attr_set = true;
  }
  // steps a log holds before the chase applies it to Z itself; the
  // TSG_SCHUR_LOG_STEPS environment variable may lower it (for testing that path)
  int64_t cap = log_steps_cap(m);
  if (const char* e = std::getenv("TSG_SCHUR_LOG_STEPS")) {
    const long v = std::atol(e);
    if (v >= 1 && v < cap) cap = v;
  }
  // helpers per window: one per kHelpBand rows and columns, when every
  // window's chase and helpers fit on the device at once (otherwise the CUs
  // serve more windows' chases instead); the TSG_SCHUR_HELPERS environment
  // variable set to 0 turns them off (for testing that path)
  static const int n_cu = [] {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      n = 0;
    return n;
  }();
  int nh = (m + kHelpBand - 1) / kHelpBand;
  if (m < kDeferMin || nh > kMaxHelpers || int64_t(nwin) * (1 + nh) > n_cu) nh = 0;
  if (const char* e = std::getenv("TSG_SCHUR_HELPERS"))
    if (std::atoi(e) == 0) nh = 0;
  if (nh > 0) hipLaunchKernelGGL(chase_sync_init_kernel, dim3(nwin), dim3(64), 0, st, log, wsl, m, wmap);
  hipLaunchKernelGGL(schur_kernel, dim3(nwin * (1 + nh)), dim3(kQT), schur_lds_bytes(), st, H, wsh, m, Z, wsz, log,
                     wsl, cap, theta, wst, info, wmap, prof, kShifts, nh);
  // rows of Z per replay workgroup: as many as 150 KiB of LDS hold next to
  // the staged records, at most 256 / kShifts
  const size_t rec_bytes = size_t(kChunk) * kShifts * sizeof(RotRec);
  const int rows = int(std::max<size_t>(1, std::min<size_t>(256 / kShifts,
                                                          (size_t(150) * 1024 - rec_bytes) / (size_t(m) * sizeof(c128)))));
  const size_t lds = size_t(rows) * m * sizeof(c128) + rec_bytes;
  if (lds > size_t(150) * 1024) throw DeviceError("schur: basis too large for the Z replay");
  if (lds > size_t(64) * 1024) {
    static size_t granted = 0;
    if (lds > granted) {
      const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(zreplay_kernel),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
      if (e != hipSuccess) throw DeviceError(std::string("zreplay: LDS attribute: ") + hipGetErrorString(e));
      granted = lds;
    }
  }
  hipLaunchKernelGGL(zreplay_kernel, dim3((m + rows - 1) / rows, nwin), dim3(rows * kShifts), lds, st, Z, wsz, m,
                     log, wsl, rows, wmap);
  // the deferred left transformations of the columns beyond each block
  const int hcols = int(std::max<size_t>(1, std::min<size_t>(256 / kShifts,
                                                           (size_t(150) * 1024 - rec_bytes) / (size_t(m) * sizeof(c128)))));
  const size_t hlds = size_t(hcols) * m * sizeof(c128) + rec_bytes;
  if (hlds > size_t(150) * 1024) throw DeviceError("schur: basis too large for the column replay");
  if (hlds > size_t(64) * 1024) {
    static size_t hgranted = 0;
    if (hlds > hgranted) {
      const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(hreplay_kernel),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, int(hlds));
      if (e != hipSuccess) throw DeviceError(std::string("hreplay: LDS attribute: ") + hipGetErrorString(e));
      hgranted = hlds;
    }
  }
  hipLaunchKernelGGL(hreplay_kernel, dim3((m + hcols - 1) / hcols, nwin), dim3(hcols * kShifts), hlds, st, H, wsh, m,
                     log, wsl, hcols, wmap);
  if (prof) {
    unsigned long long z[8];
    (void)hipMemcpyFromSymbolAsync(z, HIP_SYMBOL(g_k4prof), sizeof(z), 0, hipMemcpyDeviceToHost, st);
    (void)hipStreamSynchronize(st);
    std::fprintf(stderr, "[k4] m=%d nwin=%d us: scan %.0f shifts %.0f chaseA %.0f chaseB %.0f chaseC %.0f fin %.0f apply %.0f"
                 " chase steps %llu\n",
                 m, nwin, z[0] / 100.0, z[1] / 100.0, z[2] / 100.0, z[3] / 100.0, z[4] / 100.0, z[5] / 100.0,
                 z[6] / 100.0, z[7]);
  }
}

}  // namespace tsg
